// Host side of the hgs_nn_* entry points (learned warm start) of include/hgs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "../../include/hgs.h"
#include "k_nn.hpp"

static_assert(hgs::nn::MAXABS_CHUNKS == HGS_NN_MAXABS_CHUNKS, "scratch size of hgs_nn_maxabs");

// Partials of hgs_nn_maxabs_noalloc (see scratch_on_current_device below).
constexpr int MAXABS_NOALLOC_MAX_B = HGS_NN_MAXABS_NOALLOC_MAX_B;
static __device__ __align__(256) float scratch[MAXABS_NOALLOC_MAX_B * hgs::nn::MAXABS_CHUNKS];  // 1 MiB per device

using namespace hgs::nn;

namespace {

thread_local std::string g_nn_err;

hgs_status nfail(hgs_status s, const std::string& m) {
    g_nn_err = m;
    return s;
}

hgs_status nlaunched(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return nfail(HGS_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return HGS_OK;
}

bool dims_ok(int32_t B, int32_t Z, int32_t Y, int32_t X) {
    return B >= 1 && Z >= 1 && Y >= 1 && X >= 16 && X % 16 == 0 && (int64_t)B * Z * Y * X <= ((int64_t)1 << 31);
}

int wgrad_blocks(int32_t B, int32_t Z, int32_t Y) {
    const int64_t rows = (int64_t)B * Z * Y;
    return (int)std::max<int64_t>(1, std::min<int64_t>(512, (rows + 3) / 4));
}

int grid_of(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(65536, (n + 255) / 256)); }

// Partials of hgs_nn_maxabs_noalloc: a file-scope device array, so that the
// call allocates nothing.  Each device holds its own copy at its own address;
// host code reaches it only through the address hipGetSymbolAddress returns
// for the current device (the array's name in host code is a host-side
// stand-in, not a device address).  The kernels write every partial they read,
// so nothing has to be cleared between calls.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the current device's scratch array, looked up once per
// device on its first use; nullptr (with the reason in g_nn_err) on failure.
float* scratch_on_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        nfail(HGS_ERR_DEVICE, "hgs_nn_maxabs_noalloc: no current HIP device");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            nfail(HGS_ERR_DEVICE, std::string("hgs_nn_maxabs_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

const char* hgs_nn_last_error(void) { return g_nn_err.c_str(); }

hgs_status hgs_nn_conv3d(const uint16_t* in, const uint16_t* w, const float* bias, int32_t B, int32_t Z, int32_t Y,
                         int32_t X, int32_t mode, const uint16_t* aux, void* out, void* stream) {
    if (!in || !w || !out) return nfail(HGS_ERR_ARG, "in, w and out must be non-NULL");
    if (!dims_ok(B, Z, Y, X)) return nfail(HGS_ERR_ARG, "need B, Z, Y >= 1 and X a positive multiple of 16");
    if (mode < 0 || mode > 3) return nfail(HGS_ERR_ARG, "mode must be 0..3");
    if (mode == HGS_NN_DTANH_BF16 && !aux) return nfail(HGS_ERR_ARG, "DTANH needs aux");
    if (reinterpret_cast<uintptr_t>(in) % 16 || reinterpret_cast<uintptr_t>(out) % 16 ||
        reinterpret_cast<uintptr_t>(w) % 16)
        return nfail(HGS_ERR_ARG, "in, w and out must be 16-byte aligned");
    (void)hipGetLastError();
    if (X <= CONV_LDS_MAXX) {
        // input rows staged in LDS, four output rows per workgroup
        const int64_t blocks = (int64_t)B * Z * ((Y + 3) / 4);
        if (blocks > 0x7fffffff) return nfail(HGS_ERR_ARG, "tensor too large");
        const dim3 grid((unsigned)blocks), blk(256);
        hipStream_t st = static_cast<hipStream_t>(stream);
        switch (X / 16) {
            case 1: hipLaunchKernelGGL(k_conv3d_lds<1>, grid, blk, 0, st, in, w, bias, B, Z, Y, mode, aux, out); break;
            case 2: hipLaunchKernelGGL(k_conv3d_lds<2>, grid, blk, 0, st, in, w, bias, B, Z, Y, mode, aux, out); break;
            case 3: hipLaunchKernelGGL(k_conv3d_lds<3>, grid, blk, 0, st, in, w, bias, B, Z, Y, mode, aux, out); break;
            default: hipLaunchKernelGGL(k_conv3d_lds<4>, grid, blk, 0, st, in, w, bias, B, Z, Y, mode, aux, out); break;
        }
    } else {
        const int64_t waves = (int64_t)B * Z * Y * (X / 16);
        const int64_t blocks = (waves + 3) / 4;
        if (blocks > 0x7fffffff) return nfail(HGS_ERR_ARG, "tensor too large");
        hipLaunchKernelGGL(k_conv3d, dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(stream), in, w,
                           bias, B, Z, Y, X, mode, aux, out);
    }
    return nlaunched("hgs_nn_conv3d");
}

hgs_status hgs_nn_flip_weights(const uint16_t* w, uint16_t* wt, void* stream) {
    if (!w || !wt) return nfail(HGS_ERR_ARG, "w and wt must be non-NULL");
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_flip_weights, dim3((27 * NC * NC + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), w, wt);
    return nlaunched("hgs_nn_flip_weights");
}

hgs_status hgs_nn_wgrad_workspace_bytes(int32_t B, int32_t Z, int32_t Y, int32_t X, size_t* bytes) {
    if (!bytes) return nfail(HGS_ERR_ARG, "bytes is NULL");
    if (!dims_ok(B, Z, Y, X) || X > WG_MAXX) return nfail(HGS_ERR_ARG, "need X a multiple of 16 and at most 128");
    *bytes = (size_t)wgrad_blocks(B, Z, Y) * 4 * (27 * NC * NC + NC) * sizeof(float);
    return HGS_OK;
}

hgs_status hgs_nn_wgrad(const uint16_t* a, const uint16_t* g, int32_t B, int32_t Z, int32_t Y, int32_t X, float* dw,
                        float* db, void* workspace, size_t bytes, void* stream) {
    size_t need = 0;
    hgs_status s = hgs_nn_wgrad_workspace_bytes(B, Z, Y, X, &need);
    if (s != HGS_OK) return s;
    if (!a || !g || !dw || !db) return nfail(HGS_ERR_ARG, "a, g, dw and db must be non-NULL");
    if (!workspace || bytes < need) return nfail(HGS_ERR_WORKSPACE, "workspace smaller than hgs_nn_wgrad_workspace_bytes()");
    (void)hipGetLastError();
    const int nb = wgrad_blocks(B, Z, Y);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_wgrad_partial, dim3(nb), dim3(256), 0, st, a, g, B, Z, Y, X, static_cast<float*>(workspace));
    hipLaunchKernelGGL(k_wgrad_final, dim3((27 * NC * NC + NC + 15) / 16), dim3(256), 0, st,
                       static_cast<const float*>(workspace), nb * 4, dw, db);
    return nlaunched("hgs_nn_wgrad");
}

hgs_status hgs_nn_pack(const float* fields, int32_t B, int32_t C, int64_t nvox, uint16_t* out, void* stream) {
    if (!fields || !out) return nfail(HGS_ERR_ARG, "fields and out must be non-NULL");
    if (B < 1 || C < 1 || C > NC || nvox < 1) return nfail(HGS_ERR_ARG, "need B >= 1, 1 <= C <= 16, nvox >= 1");
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_pack, dim3(grid_of((int64_t)B * nvox)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       fields, B, C, nvox, out);
    return nlaunched("hgs_nn_pack");
}

hgs_status hgs_nn_unpack(const float* in, int32_t B, int32_t C, int64_t nvox, float* fields, void* stream) {
    if (!fields || !in) return nfail(HGS_ERR_ARG, "in and fields must be non-NULL");
    if (B < 1 || C < 1 || C > NC || nvox < 1) return nfail(HGS_ERR_ARG, "need B >= 1, 1 <= C <= 16, nvox >= 1");
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_unpack, dim3(grid_of((int64_t)B * nvox)), dim3(256), 0, static_cast<hipStream_t>(stream), in,
                       B, C, nvox, fields);
    return nlaunched("hgs_nn_unpack");
}

hgs_status hgs_nn_mse(const float* out, const float* target, int32_t B, int32_t C, int64_t nvox, uint16_t* grad,
                      double* loss_dev, double* partials, void* stream) {
    if (!out || !target || !grad || !loss_dev || !partials) return nfail(HGS_ERR_ARG, "NULL argument");
    if (B < 1 || C < 1 || C > NC || nvox < 1) return nfail(HGS_ERR_ARG, "need B >= 1, 1 <= C <= 16, nvox >= 1");
    (void)hipGetLastError();
    const int nb = std::min(HGS_NN_MSE_PARTIALS, grid_of((int64_t)B * nvox));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const float inv = (float)(1.0 / ((double)B * C * nvox));
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, st, out, target, B, C, nvox, inv, grad, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, partials, nb, loss_dev);
    return nlaunched("hgs_nn_mse");
}

hgs_status hgs_nn_lapmse(const float* out, const float* target, int32_t B, int32_t C, int32_t nz, int32_t ny,
                         int32_t nx, int32_t ch, float w, float* scratch, uint16_t* grad, double* loss_dev,
                         double* partials, void* stream) {
    if (!out || !target || !scratch || !grad || !loss_dev || !partials) return nfail(HGS_ERR_ARG, "NULL argument");
    if (B < 1 || C < 1 || C > NC || nz < 1 || ny < 1 || nx < 1 || ch < 0 || ch >= C)
        return nfail(HGS_ERR_ARG, "need B, nz, ny, nx >= 1, 1 <= C <= 16, 0 <= ch < C");
    if (!(w >= 0.f) || !std::isfinite(w)) return nfail(HGS_ERR_ARG, "w must be >= 0 and finite");
    (void)hipGetLastError();
    const int64_t nvox = (int64_t)nz * ny * nx;
    const int nb = std::min(HGS_NN_MSE_PARTIALS, grid_of((int64_t)B * nvox));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const float inv = (float)(1.0 / ((double)B * C * nvox));
    hipLaunchKernelGGL(k_lapres, dim3(grid_of((int64_t)B * nvox)), dim3(256), 0, st, out, target, B, C, ch, nz, ny, nx,
                       scratch);
    hipLaunchKernelGGL(k_lapmse, dim3(nb), dim3(256), 0, st, out, target, scratch, B, C, ch, nz, ny, nx, w, inv, grad,
                       partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, partials, nb, loss_dev);
    return nlaunched("hgs_nn_lapmse");
}

hgs_status hgs_nn_maxabs(const float* x, int32_t B, int64_t nvox, float* out, float* scratch, void* stream) {
    if (!x || !out || !scratch) return nfail(HGS_ERR_ARG, "x, out and scratch must be non-NULL");
    if (B < 1 || B > 65535 || nvox < 1) return nfail(HGS_ERR_ARG, "need 1 <= B <= 65535 and nvox >= 1");
    (void)hipGetLastError();
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_maxabs_partial, dim3(MAXABS_CHUNKS, B), dim3(256), 0, st, x, nvox, scratch);
    hipLaunchKernelGGL(k_maxabs_final, dim3((B + 255) / 256), dim3(256), 0, st, scratch, B, out);
    return nlaunched("hgs_nn_maxabs");
}

hgs_status hgs_nn_maxabs_noalloc(const float* x, int32_t B, int64_t nvox, float* out, void* stream) {
    if (!x || !out) return nfail(HGS_ERR_ARG, "x and out must be non-NULL");
    if (B < 1 || B > MAXABS_NOALLOC_MAX_B || nvox < 1)
        return nfail(HGS_ERR_ARG, "hgs_nn_maxabs_noalloc: need 1 <= B <= " + std::to_string(MAXABS_NOALLOC_MAX_B) +
                                      " (the static scratch size) and nvox >= 1");
    float* part = scratch_on_current_device();
    if (!part) return HGS_ERR_DEVICE;
    (void)hipGetLastError();
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_maxabs_partial, dim3(MAXABS_CHUNKS, B), dim3(256), 0, st, x, nvox, part);
    hipLaunchKernelGGL(k_maxabs_final, dim3((B + 255) / 256), dim3(256), 0, st, part, B, out);
    return nlaunched("hgs_nn_maxabs_noalloc");
}

hgs_status hgs_nn_features(const float* rho, const float* phi, const float* scale, int32_t B, int32_t nz, int32_t ny,
                           int32_t nx, double c, float* out, void* stream) {
    if (!rho || !phi || !scale || !out) return nfail(HGS_ERR_ARG, "NULL argument");
    if (B < 1 || nz < 1 || ny < 1 || nx < 1) return nfail(HGS_ERR_ARG, "need B, nz, ny, nx >= 1");
    if (!(c > 0.0) || !std::isfinite(c)) return nfail(HGS_ERR_ARG, "c must be positive and finite");
    (void)hipGetLastError();
    const int64_t n = (int64_t)B * nz * ny * nx;
    hipLaunchKernelGGL(k_features, dim3(grid_of(n)), dim3(256), 0, static_cast<hipStream_t>(stream), rho, phi, scale, B,
                       nz, ny, nx, c, out);
    return nlaunched("hgs_nn_features");
}

hgs_status hgs_nn_compose(const float* phi_c, const float* y, const float* scale, int32_t B, int64_t nvox,
                          double inv_out_scale, float* phi, float* phidot, void* stream) {
    if (!phi_c || !y || !scale || !phi) return nfail(HGS_ERR_ARG, "phi_c, y, scale and phi must be non-NULL");
    if (B < 1 || nvox < 1) return nfail(HGS_ERR_ARG, "need B >= 1 and nvox >= 1");
    if (!std::isfinite(inv_out_scale)) return nfail(HGS_ERR_ARG, "inv_out_scale must be finite");
    (void)hipGetLastError();
    const int64_t n = (int64_t)B * nvox;
    hipLaunchKernelGGL(k_compose, dim3(grid_of(n)), dim3(256), 0, static_cast<hipStream_t>(stream), phi_c, y, scale, B,
                       nvox, inv_out_scale, phi, phidot);
    return nlaunched("hgs_nn_compose");
}

hgs_status hgs_nn_adam(float* p, float* m, float* v, const float* g, uint16_t* p16, int32_t n, float lr, float b1,
                       float b2, float eps, int32_t t, void* stream) {
    if (!p || !m || !v || !g) return nfail(HGS_ERR_ARG, "p, m, v and g must be non-NULL");
    if (n < 1 || t < 1 || !(lr > 0.f) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f))
        return nfail(HGS_ERR_ARG, "need n >= 1, t >= 1, lr > 0, 0 <= b1, b2 < 1, eps > 0");
    (void)hipGetLastError();
    const float c1 = (float)(1.0 - std::pow((double)b1, t)), c2 = (float)(1.0 - std::pow((double)b2, t));
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream), p, m, v, g, p16, n,
                       lr, b1, b2, eps, c1, c2);
    return nlaunched("hgs_nn_adam");
}

hgs_status hgs_nn_restrict2(const void* fine, void* coarse, int32_t B, int32_t cz, int32_t cy, int32_t cx,
                            int32_t dtype, void* stream) {
    if (!fine || !coarse) return nfail(HGS_ERR_ARG, "fine and coarse must be non-NULL");
    if (B < 1 || cz < 1 || cy < 1 || cx < 1 || (dtype != HGS_F32 && dtype != HGS_F64))
        return nfail(HGS_ERR_ARG, "bad sizes or dtype");
    (void)hipGetLastError();
    const int64_t n = (int64_t)B * cz * cy * cx;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (dtype == HGS_F32)
        hipLaunchKernelGGL(k_restrict2<float>, dim3(grid_of(n)), dim3(256), 0, st, static_cast<const float*>(fine), B,
                           cz, cy, cx, static_cast<float*>(coarse));
    else
        hipLaunchKernelGGL(k_restrict2<double>, dim3(grid_of(n)), dim3(256), 0, st, static_cast<const double*>(fine),
                           B, cz, cy, cx, static_cast<double*>(coarse));
    return nlaunched("hgs_nn_restrict2");
}

hgs_status hgs_nn_prolong2(const void* coarse, void* fine, int32_t B, int32_t cz, int32_t cy, int32_t cx,
                           int32_t dtype, void* stream) {
    if (!fine || !coarse) return nfail(HGS_ERR_ARG, "fine and coarse must be non-NULL");
    if (B < 1 || cz < 1 || cy < 1 || cx < 1 || (dtype != HGS_F32 && dtype != HGS_F64))
        return nfail(HGS_ERR_ARG, "bad sizes or dtype");
    (void)hipGetLastError();
    const int64_t n = (int64_t)B * 8 * cz * cy * cx;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (dtype == HGS_F32)
        hipLaunchKernelGGL(k_prolong2<float>, dim3(grid_of(n)), dim3(256), 0, st, static_cast<const float*>(coarse), B,
                           cz, cy, cx, static_cast<float*>(fine));
    else
        hipLaunchKernelGGL(k_prolong2<double>, dim3(grid_of(n)), dim3(256), 0, st, static_cast<const double*>(coarse),
                           B, cz, cy, cx, static_cast<double*>(fine));
    return nlaunched("hgs_nn_prolong2");
}

}  // extern "C"
