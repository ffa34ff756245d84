// Kernels of the learned warm start: a 3x3x3 convolution network with
// bfloat16 weights and activations and FP32 accumulation on CDNA MFMA.
//
// Tensors are channels-last with 16 channels: (B, Z, Y, X, 16), bfloat16 bits
// in uint16.  A convolution is an implicit GEMM: for one tap t,
//   out^T[co][v] += W_t[co][ci] * in_t[ci][v]     (16 x 16 x 16 per MFMA),
// with v sixteen consecutive x positions of one row.  In the MFMA
// v_mfma_f32_16x16x16_bf16 lane l holds A[l%16][4(l/16)..+3],
// B[4(l/16)..+3][l%16] and C[4(l/16)..+3][l%16]; with A = W_t (rows co, k ci),
// B = the input (k ci, columns v) and C = out^T, lane l reads 4 contiguous
// channels of voxel v = l%16 and ends up holding 4 contiguous output channels
// of that voxel, so every load and store is one 8- or 16-byte access.
#pragma once

#include "common.hpp"

namespace hgs {
namespace nn {

constexpr int NC = 16;  // channels per tensor

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
    // round to nearest even (values here are finite)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

enum ConvMode {
    CONV_F32 = 0,         // out (FP32) = conv + bias
    CONV_TANH_BF16 = 1,   // out (bf16) = tanh(conv + bias)
    CONV_DTANH_BF16 = 2,  // out (bf16) = conv * (1 - aux^2)   (backward through aux = tanh output)
    CONV_BF16 = 3,        // out (bf16) = conv + bias
};

// One wave per 16 consecutive x positions of a row; 4 waves per workgroup.
__global__ __launch_bounds__(256) void k_conv3d(const uint16_t* __restrict__ in, const uint16_t* __restrict__ w,
                                                const float* __restrict__ bias, int B, int Z, int Y, int X, int mode,
                                                const uint16_t* __restrict__ aux, void* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int segs = X / 16;
    const int nw = B * Z * Y * segs;
    if (wave >= nw) return;  // whole waves only: the MFMA needs all 64 lanes
    const int seg = wave % segs;
    int r = wave / segs;
    const int y = r % Y;
    r /= Y;
    const int z = r % Z;
    const int b = r / Z;
    const int col = lane & 15;   // voxel within the segment / row of A
    const int kq = lane >> 4;    // which group of 4 along k
    const int x = seg * 16 + col;
    f32x4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 3
    for (int t = 0; t < 27; ++t) {
        const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
        const bf16x4 a = *reinterpret_cast<const bf16x4*>(w + (t * NC + col) * NC + 4 * kq);
        const int zz = z + dz, yy = y + dy, xx = x + dx;
        bf16x4 bv = {0, 0, 0, 0};
        if (zz >= 0 && zz < Z && yy >= 0 && yy < Y && xx >= 0 && xx < X)
            bv = *reinterpret_cast<const bf16x4*>(in + ((((int64_t)b * Z + zz) * Y + yy) * X + xx) * NC + 4 * kq);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc, 0, 0, 0);
    }
    const int64_t o = ((((int64_t)b * Z + z) * Y + y) * X + x) * NC + 4 * kq;
    if (mode == CONV_F32) {
        f32x4v v;
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = acc[i] + (bias ? bias[4 * kq + i] : 0.f);
        *reinterpret_cast<f32x4v*>(static_cast<float*>(out) + o) = v;
    } else {
        bf16x4 v;
        bf16x4 ax = {0, 0, 0, 0};
        if (mode == CONV_DTANH_BF16) ax = *reinterpret_cast<const bf16x4*>(aux + o);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float s = acc[i];
            if (mode == CONV_TANH_BF16) {
                s = tanhf(s + (bias ? bias[4 * kq + i] : 0.f));
            } else if (mode == CONV_DTANH_BF16) {
                const float yv = bf2f((uint16_t)ax[i]);
                s = s * (1.f - yv * yv);
            } else {
                s = s + (bias ? bias[4 * kq + i] : 0.f);
            }
            v[i] = (short)f2bf(s);
        }
        *reinterpret_cast<bf16x4*>(static_cast<uint16_t*>(out) + o) = v;
    }
}

// wt[26 - t][ci][co] = w[t][co][ci]: the weights of the input-gradient convolution.
__global__ void k_flip_weights(const uint16_t* __restrict__ w, uint16_t* __restrict__ wt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 27 * NC * NC) return;
    const int t = i / (NC * NC), co = (i / NC) % NC, ci = i % NC;
    wt[((26 - t) * NC + ci) * NC + co] = w[i];
}

// Weight and bias gradients: dW[t][co][ci] = sum_v g[v][co] a[v + tap][ci],
// db[co] = sum_v g[v][co].  Each wave takes whole x rows (X = 16 * segs <= 128)
// in turn and keeps the 27 16x16 accumulators in registers; rows are staged
// transposed in LDS so that voxels become the MFMA k dimension.  Per-workgroup
// partials are summed by k_wgrad_final in a fixed order.
constexpr int WG_MAXX = 128;
__global__ __launch_bounds__(256) void k_wgrad_partial(const uint16_t* __restrict__ a, const uint16_t* __restrict__ g,
                                                       int B, int Z, int Y, int X, float* __restrict__ partial) {
    __shared__ uint16_t gT[4][NC][WG_MAXX];        // [wave][co][v]
    __shared__ uint16_t aT[4][NC][WG_MAXX + 2];    // [wave][ci][v + 1] (x halo at both ends)
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int rows = B * Z * Y;
    f32x4v acc[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) acc[t] = (f32x4v){0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;  // lane < 16: bias gradient of channel lane
    for (int row = blockIdx.x * 4 + wv; row < rows; row += gridDim.x * 4) {
        const int y = row % Y;
        const int z = (row / Y) % Z;
        const int b = row / (Y * Z);
        // g row, transposed
        for (int v = lane; v < X; v += 64) {
            const uint16_t* src = g + ((((int64_t)b * Z + z) * Y + y) * X + v) * NC;
#pragma unroll
            for (int c = 0; c < NC; ++c) gT[wv][c][v] = src[c];
        }
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        if (lane < NC) {
            for (int v = 0; v < X; ++v) bsum += bf2f(gT[wv][lane][v]);
        }
        for (int dzy = 0; dzy < 9; ++dzy) {
            const int dz = dzy / 3 - 1, dy = dzy % 3 - 1;
            const int zz = z + dz, yy = y + dy;
            const bool ok = zz >= 0 && zz < Z && yy >= 0 && yy < Y;
            __builtin_amdgcn_wave_barrier();
            for (int v = lane; v < X + 2; v += 64) {
                const int xx = v - 1;
                const bool in = ok && xx >= 0 && xx < X;
                const uint16_t* src = a + ((((int64_t)b * Z + (in ? zz : 0)) * Y + (in ? yy : 0)) * X + (in ? xx : 0)) * NC;
#pragma unroll
                for (int c = 0; c < NC; ++c) aT[wv][c][v] = in ? src[c] : (uint16_t)0;
            }
            __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_wave_barrier();
            if (!ok) continue;
#pragma unroll
            for (int dxi = 0; dxi < 3; ++dxi) {
                const int t = dzy * 3 + dxi;
                for (int kc = 0; kc < X / 16; ++kc) {
                    const int v0 = kc * 16 + 4 * kq;
                    bf16x4 A, Bv;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        A[i] = (short)gT[wv][col][v0 + i];
                        Bv[i] = (short)aT[wv][col][v0 + i + dxi];  // a[v + dx] at LDS column v + 1 + dx
                    }
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, Bv, acc[t], 0, 0, 0);
                }
            }
        }
    }
    // partial[block][t][co][ci] (+ bias in the last 16 slots): lane holds
    // C[co = 4 kq + i][ci = col]
    float* p = partial + (size_t)blockIdx.x * (27 * NC * NC + NC) * 4 + (size_t)wv * (27 * NC * NC + NC);
#pragma unroll
    for (int t = 0; t < 27; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) p[(t * NC + 4 * kq + i) * NC + col] = acc[t][i];
    if (lane < NC) p[27 * NC * NC + lane] = bsum;
}

// dw[t][co][ci] and db[co]: fixed-order sums of the per-wave partials.
__global__ void k_wgrad_final(const float* __restrict__ partial, int nparts, float* __restrict__ dw,
                              float* __restrict__ db) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int per = 27 * NC * NC + NC;
    if (i >= per) return;
    float s = 0.f;
    for (int k = 0; k < nparts; ++k) s += partial[(size_t)k * per + i];
    if (i < 27 * NC * NC)
        dw[i] = s;
    else
        db[i - 27 * NC * NC] = s;
}

// Planar FP32 fields [B][C][vox] -> channels-last bf16 [B][vox][16] (zero beyond C).
__global__ void k_pack(const float* __restrict__ f, int B, int C, int64_t nvox, uint16_t* __restrict__ out) {
    const int64_t total = (int64_t)B * nvox;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = t / nvox, v = t % nvox;
        uint16_t h[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) h[c] = c < C ? f2bf(f[(b * C + c) * nvox + v]) : (uint16_t)0;
        uint16_t* o = out + t * NC;
#pragma unroll
        for (int c = 0; c < NC; ++c) o[c] = h[c];
    }
}

// channels-last FP32 [B][vox][16] -> planar [B][C][vox]
__global__ void k_unpack(const float* __restrict__ in, int B, int C, int64_t nvox, float* __restrict__ f) {
    const int64_t total = (int64_t)B * nvox;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = t / nvox, v = t % nvox;
        for (int c = 0; c < C; ++c) f[(b * C + c) * nvox + v] = in[t * NC + c];
    }
}

// Mean-squared error over the first C channels against planar targets
// [B][C][vox]: grad (bf16, channels-last, zero beyond C) = 2 (out - target) / count
// and per-workgroup partial sums of (out - target)^2 for the loss.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ out, const float* __restrict__ target, int B,
                                             int C, int64_t nvox, float inv_count, uint16_t* __restrict__ grad,
                                             double* __restrict__ partial) {
    __shared__ double red[4];
    double acc = 0.0;
    const int64_t total = (int64_t)B * nvox;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = t / nvox, v = t % nvox;
        uint16_t h[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            float d = 0.f;
            if (c < C) {
                d = out[t * NC + c] - target[(b * C + c) * nvox + v];
                acc += (double)d * d;
            }
            h[c] = f2bf(2.f * d * inv_count);
        }
        uint16_t* o = grad + t * NC;
#pragma unroll
        for (int c = 0; c < NC; ++c) o[c] = h[c];
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Laplacian-weighted loss.  With e = out[..., ch] - target[b][ch] and L the
// 7-point Laplacian in index units with zero outside the box,
//   loss = sum_c sum_v e_c^2 + w sum_v (L e_ch)^2,
//   d loss / d out_c = 2 e_c + [c == ch] 2 w L(L e_ch)     (L is symmetric).
// First pass: r = L e_ch into an FP32 planar scratch [B][nvox].
__device__ __forceinline__ double lap_err(const float* __restrict__ out, const float* __restrict__ target, int C,
                                          int ch, int nz, int ny, int nx, int64_t b, int i, int j, int k) {
    if (i < 0 || i >= nx || j < 0 || j >= ny || k < 0 || k >= nz) return 0.0;
    const int64_t nvox = (int64_t)nz * ny * nx;
    const int64_t v = ((int64_t)k * ny + j) * nx + i;
    return (double)out[(b * nvox + v) * NC + ch] - (double)target[(b * C + ch) * nvox + v];
}

__global__ __launch_bounds__(256) void k_lapres(const float* __restrict__ out, const float* __restrict__ target, int B,
                                                int C, int ch, int nz, int ny, int nx, float* __restrict__ r) {
    const int64_t nvox = (int64_t)nz * ny * nx, total = (int64_t)B * nvox;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = t / nvox, v = t % nvox;
        const int i = (int)(v % nx), j = (int)((v / nx) % ny), k = (int)(v / ((int64_t)nx * ny));
        const double nb = ((lap_err(out, target, C, ch, nz, ny, nx, b, i - 1, j, k) +
                            lap_err(out, target, C, ch, nz, ny, nx, b, i + 1, j, k)) +
                           (lap_err(out, target, C, ch, nz, ny, nx, b, i, j - 1, k) +
                            lap_err(out, target, C, ch, nz, ny, nx, b, i, j + 1, k))) +
                          (lap_err(out, target, C, ch, nz, ny, nx, b, i, j, k - 1) +
                           lap_err(out, target, C, ch, nz, ny, nx, b, i, j, k + 1));
        r[t] = (float)(nb - 6.0 * lap_err(out, target, C, ch, nz, ny, nx, b, i, j, k));
    }
}

__device__ __forceinline__ double lap_at(const float* __restrict__ r, int nz, int ny, int nx, int64_t b, int i, int j,
                                         int k) {
    if (i < 0 || i >= nx || j < 0 || j >= ny || k < 0 || k >= nz) return 0.0;
    return (double)r[(b * nz + k) * (int64_t)ny * nx + (int64_t)j * nx + i];
}

// Second pass: gradient (bf16 channels-last, scaled by inv_count) and block
// partial sums of the loss.
__global__ __launch_bounds__(256) void k_lapmse(const float* __restrict__ out, const float* __restrict__ target,
                                                const float* __restrict__ r, int B, int C, int ch, int nz, int ny,
                                                int nx, float w, float inv_count, uint16_t* __restrict__ grad,
                                                double* __restrict__ partial) {
    __shared__ double red[4];
    double acc = 0.0;
    const int64_t nvox = (int64_t)nz * ny * nx, total = (int64_t)B * nvox;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = t / nvox, v = t % nvox;
        const int i = (int)(v % nx), j = (int)((v / nx) % ny), k = (int)(v / ((int64_t)nx * ny));
        const double rc = (double)r[t];
        const double lr = (((lap_at(r, nz, ny, nx, b, i - 1, j, k) + lap_at(r, nz, ny, nx, b, i + 1, j, k)) +
                            (lap_at(r, nz, ny, nx, b, i, j - 1, k) + lap_at(r, nz, ny, nx, b, i, j + 1, k))) +
                           (lap_at(r, nz, ny, nx, b, i, j, k - 1) + lap_at(r, nz, ny, nx, b, i, j, k + 1))) -
                          6.0 * rc;
        acc += (double)w * rc * rc;
        uint16_t h[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double g = 0.0;
            if (c < C) {
                const double d = (double)out[t * NC + c] - (double)target[(b * C + c) * nvox + v];
                acc += d * d;
                g = 2.0 * d;
                if (c == ch) g += 2.0 * (double)w * lr;
            }
            h[c] = f2bf((float)(g * (double)inv_count));
        }
        uint16_t* o = grad + t * NC;
#pragma unroll
        for (int c = 0; c < NC; ++c) o[c] = h[c];
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Per-sample peak |x| over nvox values: one workgroup per sample.
__global__ __launch_bounds__(256) void k_maxabs(const float* __restrict__ x, int64_t nvox, float* __restrict__ out) {
    __shared__ float red[4];
    const float* p = x + (int64_t)blockIdx.x * nvox;
    float m = 0.f;
    for (int64_t t = threadIdx.x; t < nvox; t += blockDim.x) m = fmaxf(m, fabsf(p[t]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// second difference along one axis, 0 at the first and last cell
__device__ __forceinline__ double d2_ext(const float* __restrict__ f, int i, int n, int64_t stride) {
    if (i <= 0 || i >= n - 1) return 0.0;
    return ((double)f[-stride] + (double)f[stride]) - 2.0 * (double)f[0];
}

// Network inputs, planar [B][3][Z][Y][X] FP32:
//   rho / s, phi / s, (L_ext phi - c rho) / (c s),  c = 4 pi G h^2, s = scale[b],
// L_ext the 7-point Laplacian in index units with the second difference along
// an axis taken as 0 at the first and last cell.
__global__ __launch_bounds__(256) void k_features(const float* __restrict__ rho, const float* __restrict__ phi,
                                                  const float* __restrict__ scale, int B, int nz, int ny, int nx,
                                                  double c, float* __restrict__ out) {
    const int64_t nvox = (int64_t)nz * ny * nx, total = (int64_t)B * nvox;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = t / nvox, v = t % nvox;
        const int i = (int)(v % nx), j = (int)((v / nx) % ny), k = (int)(v / ((int64_t)nx * ny));
        const float* pf = phi + t;
        const double lap = (d2_ext(pf, i, nx, 1) + d2_ext(pf, j, ny, nx)) + d2_ext(pf, k, nz, (int64_t)nx * ny);
        const double s = (double)scale[b];
        const double r = (double)rho[t];
        float* o = out + b * 3 * nvox + v;
        o[0] = (float)(r / s);
        o[nvox] = (float)((double)pf[0] / s);
        o[2 * nvox] = (float)((lap - c * r) / (c * s));
    }
}

// (phi, dphi/dt) = (phi_c + y0 s f, y1 s f) from the last layer's FP32
// channels-last output y, f = 1 / out_scale.
__global__ __launch_bounds__(256) void k_compose(const float* __restrict__ phi_c, const float* __restrict__ y,
                                                 const float* __restrict__ scale, int B, int64_t nvox, double inv_out,
                                                 float* __restrict__ phi, float* __restrict__ phidot) {
    const int64_t total = (int64_t)B * nvox;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const double f = (double)scale[t / nvox] * inv_out;
        phi[t] = (float)((double)phi_c[t] + (double)y[t * NC] * f);
        if (phidot) phidot[t] = (float)((double)y[t * NC + 1] * f);
    }
}

__global__ void k_sum_partials(const double* __restrict__ partial, int n, double* __restrict__ out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += partial[i];
        *out = s;
    }
}

// Adam with bias correction; FP32 master parameters, optional bf16 copy.
__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ g,
                       uint16_t* __restrict__ p16, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    if (p16) p16[i] = f2bf(pi);
}

// Restriction (2x2x2 mean) and cell-centred trilinear prolongation of
// [B][nz][ny][nx] fields; coarse dims (cz, cy, cx), fine = twice that.
template <typename T>
__global__ void k_restrict2(const T* __restrict__ f, int B, int cz, int cy, int cx, T* __restrict__ c) {
    const int64_t total = (int64_t)B * cz * cy * cx;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % cx);
        const int j = (int)((t / cx) % cy);
        const int k = (int)((t / ((int64_t)cx * cy)) % cz);
        const int64_t b = t / ((int64_t)cx * cy * cz);
        const int fx = 2 * cx, fy = 2 * cy, fz = 2 * cz;
        double s = 0.0;
        for (int dk = 0; dk < 2; ++dk)
            for (int dj = 0; dj < 2; ++dj)
                for (int di = 0; di < 2; ++di)
                    s += (double)f[((b * fz + 2 * k + dk) * fy + 2 * j + dj) * (int64_t)fx + 2 * i + di];
        c[t] = (T)(s * 0.125);
    }
}

// weights of fine cell f along one axis of length n (coarse): (index, weight) pairs
__device__ __forceinline__ void prolong_w(int f, int n, int& i0, double& w0, int& i1, double& w1) {
    const int c = f >> 1;
    const bool hi = f & 1;
    int nb = hi ? c + 1 : c - 1;
    if (n == 1) {
        i0 = c; w0 = 1.0; i1 = c; w1 = 0.0;
        return;
    }
    if (nb < 0 || nb >= n) {  // linear extrapolation: 3/4 c + 1/4 (2 c - c_inner)
        const int inner = hi ? c - 1 : c + 1;
        i0 = c; w0 = 1.25; i1 = inner; w1 = -0.25;
        return;
    }
    i0 = c; w0 = 0.75; i1 = nb; w1 = 0.25;
}

template <typename T>
__global__ void k_prolong2(const T* __restrict__ c, int B, int cz, int cy, int cx, T* __restrict__ f) {
    const int fx = 2 * cx, fy = 2 * cy, fz = 2 * cz;
    const int64_t total = (int64_t)B * fz * fy * fx;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % fx);
        const int j = (int)((t / fx) % fy);
        const int k = (int)((t / ((int64_t)fx * fy)) % fz);
        const int64_t b = t / ((int64_t)fx * fy * fz);
        int xi[2], yi[2], zi[2];
        double xw[2], yw[2], zw[2];
        prolong_w(i, cx, xi[0], xw[0], xi[1], xw[1]);
        prolong_w(j, cy, yi[0], yw[0], yi[1], yw[1]);
        prolong_w(k, cz, zi[0], zw[0], zi[1], zw[1]);
        double s = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int q = 0; q < 2; ++q)
                for (int r = 0; r < 2; ++r)
                    s += zw[a] * yw[q] * xw[r] * (double)c[((b * cz + zi[a]) * cy + yi[q]) * (int64_t)cx + xi[r]];
        f[t] = (T)s;
    }
}

}  // namespace nn
}  // namespace hgs
