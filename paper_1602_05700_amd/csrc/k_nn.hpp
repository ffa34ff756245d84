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

// tanh for bf16 outputs: (1 - e) / (1 + e) with e = exp(-2|x|), sign restored,
// the quotient by the hardware reciprocal; the error (a few 1e-7 absolute) is
// far below one bf16 rounding step
__device__ __forceinline__ float tanh_bf(float x) {
    const float e = __expf(-2.f * fabsf(x));
    return copysignf((1.f - e) * __builtin_amdgcn_rcpf(1.f + e), x);
}

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
                s = tanh_bf(s + (bias ? bias[4 * kq + i] : 0.f));
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

// The same convolution with the input and the weights staged in LDS.  A
// workgroup of four waves computes four consecutive output rows (y0..y0+3) of
// one z plane over the whole x extent X = 16 SEGS.  It first copies the 27
// weight matrices and the 3 x 6 x (X+2) input voxels those rows read (z-1..z+1,
// y0-1..y0+4, x -1..X; zero outside the grid) into LDS with 16-byte loads,
// then each wave runs its row's 27 taps x SEGS MFMAs with both fragments read
// from LDS (8 bytes per lane; a wave's B reads are 512 contiguous bytes).
// SEGS is a template parameter so that the tap loop has no branches: with a
// run-time segment count every guarded MFMA made the compiler shuffle all
// accumulators through copies.  X <= CONV_LDS_MAXX keeps tile and weights
// within 64 KB.
//
// LDS swizzle: a voxel (or a weight row) is 32 bytes, two 16-byte halves of
// 8 channels.  Where bit 3 of the voxel's x index (of the weight row's index)
// is set the halves are stored swapped, so the 8-byte reads of 32 lanes, which
// cover 16 consecutive voxels, fall on 64 distinct banks instead of two lanes
// per bank.
constexpr int CONV_LDS_MAXX = 64;
template <int SEGS>
__global__ __launch_bounds__(256) void k_conv3d_lds(const uint16_t* __restrict__ in, const uint16_t* __restrict__ w,
                                                    const float* __restrict__ bias, int B, int Z, int Y, int mode,
                                                    const uint16_t* __restrict__ aux, void* __restrict__ out) {
    constexpr int X = 16 * SEGS;
    constexpr int XE = X + 2;
    __shared__ __align__(16) uint16_t tile[3][6][XE][NC];
    __shared__ __align__(16) uint16_t wsh[27][NC][NC];
    const int ybl = (Y + 3) / 4;
    const int yb = blockIdx.x % ybl;
    const int z = (blockIdx.x / ybl) % Z;
    const int b = blockIdx.x / (ybl * Z);
    if (b >= B) return;  // whole workgroup, before the barrier (the grid is B Z ceil(Y/4))
    const int y0 = yb * 4;
    // stage: 2 halves of 8 channels (16 bytes) per voxel, then the weights.
    // Every load of a thread is issued before its first LDS store, so the
    // global latencies overlap instead of adding up.
    constexpr int NHALF = 3 * 6 * XE * 2;
    constexpr int NSTAGE = (NHALF + 255) / 256;
    uint4 buf[NSTAGE];
#pragma unroll
    for (int i = 0; i < NSTAGE; ++i) {
        const int h = threadIdx.x + i * 256;
        buf[i] = make_uint4(0u, 0u, 0u, 0u);
        if (h < NHALF) {
            const int v = h >> 1;
            const int xe = v % XE;
            const int xx = xe - 1, yy = y0 + (v / XE) % 6 - 1, zz = z + v / (XE * 6) - 1;
            const int half = (h ^ (xe >> 3)) & 1;  // the swizzled half this slot holds
            if (xx >= 0 && xx < X && yy >= 0 && yy < Y && zz >= 0 && zz < Z)
                buf[i] = *reinterpret_cast<const uint4*>(in + ((((int64_t)b * Z + zz) * Y + yy) * X + xx) * NC +
                                                         8 * half);
        }
    }
    // the 27 x 16 x 16 weights: 864 16-byte pieces, at most four per thread
    const uint4* wsrc = reinterpret_cast<const uint4*>(w);
    constexpr int NWP = 27 * NC * NC / 8;
    static_assert(NWP > 768 && NWP <= 1024, "weight staging expects four pieces per thread");
    const int t0 = threadIdx.x;
    // piece P = 2 (32 t + row) + half; slot P holds piece P ^ bit 3 of row
    const int wsw = t0 ^ ((t0 >> 4) & 1);  // the same for t0 + 256 k
    const uint4 wb0 = wsrc[wsw], wb1 = wsrc[wsw + 256], wb2 = wsrc[wsw + 512];
    const uint4 wb3 = t0 + 768 < NWP ? wsrc[wsw + 768] : make_uint4(0u, 0u, 0u, 0u);
    // the staged halves are consecutive 16-byte slots of tile in this order
    uint4* tdst = reinterpret_cast<uint4*>(&tile[0][0][0][0]);
#pragma unroll
    for (int i = 0; i < NSTAGE; ++i) {
        const int h = threadIdx.x + i * 256;
        if (h < NHALF) tdst[h] = buf[i];
    }
    uint4* wdst = reinterpret_cast<uint4*>(&wsh[0][0][0]);
    wdst[t0] = wb0;
    wdst[t0 + 256] = wb1;
    wdst[t0 + 512] = wb2;
    if (t0 + 768 < NWP) wdst[t0 + 768] = wb3;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int y = y0 + wv;
    if (y >= Y) return;  // after the only barrier; whole waves
    const int col = lane & 15, kq = lane >> 4;
    f32x4v acc[SEGS];
#pragma unroll
    for (int s = 0; s < SEGS; ++s) acc[s] = (f32x4v){0.f, 0.f, 0.f, 0.f};
    // 4-channel group kq sits at group kq ^ 2 where the halves are swapped
    const uint16_t* wbase = &wsh[0][col][4 * (kq ^ (2 * ((col >> 3) & 1)))];
    const uint16_t* tb[3];  // per dx: x index col + dx (+ 16 s, which keeps bit 3)
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
        tb[dx] = &tile[0][wv][col + dx][4 * (kq ^ (2 * (((col + dx) >> 3) & 1)))];
#pragma unroll
    for (int t = 0; t < 27; ++t) {
        const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;  // offsets into the tile (0..2)
        const bf16x4 a = *reinterpret_cast<const bf16x4*>(wbase + t * NC * NC);
        bf16x4 bv[SEGS];
#pragma unroll
        for (int s = 0; s < SEGS; ++s)
            bv[s] = *reinterpret_cast<const bf16x4*>(tb[dx] + ((dz * 6 + dy) * XE + s * 16) * NC);
#pragma unroll
        for (int s = 0; s < SEGS; ++s) acc[s] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv[s], acc[s], 0, 0, 0);
    }
    float bz[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) bz[i] = bias ? bias[4 * kq + i] : 0.f;
#pragma unroll
    for (int s = 0; s < SEGS; ++s) {
        const int x = s * 16 + col;
        const int64_t o = ((((int64_t)b * Z + z) * Y + y) * X + x) * NC + 4 * kq;
        if (mode == CONV_F32) {
            f32x4v v;
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = acc[s][i] + bz[i];
            *reinterpret_cast<f32x4v*>(static_cast<float*>(out) + o) = v;
        } else {
            bf16x4 v;
            bf16x4 ax = {0, 0, 0, 0};
            if (mode == CONV_DTANH_BF16) ax = *reinterpret_cast<const bf16x4*>(aux + o);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float sv = acc[s][i];
                if (mode == CONV_TANH_BF16) {
                    sv = tanh_bf(sv + bz[i]);
                } else if (mode == CONV_DTANH_BF16) {
                    const float yv = bf2f((uint16_t)ax[i]);
                    sv = sv * (1.f - yv * yv);
                } else {
                    sv = sv + bz[i];
                }
                v[i] = (short)f2bf(sv);
            }
            *reinterpret_cast<bf16x4*>(static_cast<uint16_t*>(out) + o) = v;
        }
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
constexpr int WG_VPL = (WG_MAXX + 2 + 63) / 64;  // voxels per lane in a staged row
// LDS row pitch of the transposed rows: 136 elements (68 banks of 4 bytes)
// spreads the 16 rows a wave reads at once over distinct banks, and keeps
// 4-element groups 8-byte aligned
constexpr int WG_PITCH = WG_MAXX + 8;

// One row of 16-channel voxels into registers (two 16-byte loads per voxel);
// voxel slot j of this lane is x = lane + 64 j - off, zero outside [0, X) or
// when the row is outside the grid.
__device__ __forceinline__ void wg_load_row(const uint16_t* __restrict__ src, bool ok, int n, int off, int X,
                                            int lane, uint4 (&r)[WG_VPL][2]) {
#pragma unroll
    for (int j = 0; j < WG_VPL; ++j) {
        const int v = lane + 64 * j;
        const int xx = v - off;
        r[j][0] = r[j][1] = make_uint4(0u, 0u, 0u, 0u);
        if (ok && v < n && xx >= 0 && xx < X) {
            const uint4* p = reinterpret_cast<const uint4*>(src + (int64_t)xx * NC);
            r[j][0] = p[0];
            r[j][1] = p[1];
        }
    }
}

// Registers of wg_load_row into LDS transposed: dst[c * pitch + v] = channel c.
__device__ __forceinline__ void wg_store_T(uint16_t* __restrict__ dst, int pitch, int n, int lane,
                                           const uint4 (&r)[WG_VPL][2]) {
#pragma unroll
    for (int j = 0; j < WG_VPL; ++j) {
        const int v = lane + 64 * j;
        if (v < n) {
            const uint32_t wds[8] = {r[j][0].x, r[j][0].y, r[j][0].z, r[j][0].w,
                                     r[j][1].x, r[j][1].y, r[j][1].z, r[j][1].w};
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                dst[(2 * q) * pitch + v] = (uint16_t)(wds[q] & 0xffffu);
                dst[(2 * q + 1) * pitch + v] = (uint16_t)(wds[q] >> 16);
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_wgrad_partial(const uint16_t* __restrict__ a, const uint16_t* __restrict__ g,
                                                       int B, int Z, int Y, int X, float* __restrict__ partial) {
    __shared__ __align__(16) uint16_t gT[4][NC][WG_PITCH];  // [wave][co][v]
    __shared__ __align__(16) uint16_t aT[4][NC][WG_PITCH];  // [wave][ci][v + 1] (x halo at both ends)
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int rows = B * Z * Y;
    f32x4v acc[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) acc[t] = (f32x4v){0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;  // lane < 16: bias gradient of channel lane
    uint4 nx[WG_VPL][2];
    for (int row = blockIdx.x * 4 + wv; row < rows; row += gridDim.x * 4) {
        const int y = row % Y;
        const int z = (row / Y) % Z;
        const int b = row / (Y * Z);
        // g row, transposed
        wg_load_row(g + (((int64_t)b * Z + z) * Y + y) * X * NC, true, X, 0, X, lane, nx);
        // LDS regions are per wave and a wave's LDS operations execute in
        // order; the wavefront-scope fences only keep the compiler from moving
        // LDS accesses across them (they wait for nothing, so the prefetched
        // global loads stay in flight)
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        wg_store_T(&gT[wv][0][0], WG_PITCH, X, lane, nx);
        // first neighbour row (dz, dy) = (-1, -1)
        {
            const int zz = z - 1, yy = y - 1;
            const bool ok = zz >= 0 && yy >= 0;
            wg_load_row(a + (((int64_t)b * Z + (ok ? zz : 0)) * Y + (ok ? yy : 0)) * X * NC, ok, X + 2, 1, X, lane,
                        nx);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (lane < NC) {
            for (int v = 0; v < X; ++v) bsum += bf2f(gT[wv][lane][v]);
        }
        // unrolled: the 27 accumulators are then indexed by constants and stay
        // in registers
#pragma unroll
        for (int dzy = 0; dzy < 9; ++dzy) {
            const int dz = dzy / 3 - 1, dy = dzy % 3 - 1;
            const bool ok = z + dz >= 0 && z + dz < Z && y + dy >= 0 && y + dy < Y;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // after the previous row's LDS reads
            wg_store_T(&aT[wv][0][0], WG_PITCH, X + 2, lane, nx);
            if (dzy < 8) {  // next row's loads fly during this row's MFMAs
                const int zz = z + (dzy + 1) / 3 - 1, yy = y + (dzy + 1) % 3 - 1;
                const bool nok = zz >= 0 && zz < Z && yy >= 0 && yy < Y;
                wg_load_row(a + (((int64_t)b * Z + (nok ? zz : 0)) * Y + (nok ? yy : 0)) * X * NC, nok, X + 2, 1, X,
                            lane, nx);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // before this row's LDS reads
            if (!ok) continue;
#pragma unroll
            for (int dxi = 0; dxi < 3; ++dxi) {
                const int t = dzy * 3 + dxi;
                for (int kc = 0; kc < X / 16; ++kc) {
                    const int v0 = kc * 16 + 4 * kq;
                    const bf16x4 A = *reinterpret_cast<const bf16x4*>(&gT[wv][col][v0]);
                    bf16x4 Bv;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        Bv[i] = (short)aT[wv][col][v0 + i + dxi];  // a[v + dx] at LDS column v + 1 + dx
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
// Sum of the per-workgroup partials: a workgroup takes 16 outputs and splits
// the partials into 16 interleaved slices (fixed order in each), then adds
// the 16 slice sums in order.
__global__ __launch_bounds__(256) void k_wgrad_final(const float* __restrict__ partial, int nparts,
                                                     float* __restrict__ dw, float* __restrict__ db) {
    __shared__ float red[16][17];
    const int per = 27 * NC * NC + NC;
    const int o = threadIdx.x & 15, sl = threadIdx.x >> 4;
    const int i = blockIdx.x * 16 + o;
    float s = 0.f;
    if (i < per)
        for (int k = sl; k < nparts; k += 16) s += partial[(size_t)k * per + i];
    red[sl][o] = s;
    __syncthreads();
    if (threadIdx.x < 16 && i < per) {
        float t = 0.f;
        for (int q = 0; q < 16; ++q) t += red[q][threadIdx.x];
        if (i < 27 * NC * NC)
            dw[i] = t;
        else
            db[i - 27 * NC * NC] = t;
    }
}

// Planar FP32 fields [B][C][vox] -> channels-last bf16 [B][vox][16] (zero beyond C).
__global__ void k_pack(const float* __restrict__ f, int B, int C, int64_t nvox, uint16_t* __restrict__ out) {
    const int64_t total = (int64_t)B * nvox;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        int64_t v;
        const int64_t b = divmod(t, nvox, v);
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

// Per-sample peak |x| over nvox values: workgroup (c, b) takes chunk c of
// sample b and writes its maximum to partial[b * chunks + c]; k_maxabs_final
// takes the maximum over the chunks (max is exact, so the result does not
// depend on the split).
constexpr int MAXABS_CHUNKS = 64;
__global__ __launch_bounds__(256) void k_maxabs_partial(const float* __restrict__ x, int64_t nvox,
                                                        float* __restrict__ partial) {
    __shared__ float red[4];
    const int b = blockIdx.y;
    // chunks of a multiple of 4 values, so that aligned samples are read as
    // 16-byte vectors with several loads in flight per lane
    const int64_t per = ((nvox + MAXABS_CHUNKS - 1) / MAXABS_CHUNKS + 3) / 4 * 4;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < nvox ? lo + per : nvox;
    const float* p = x + (int64_t)b * nvox;
    float m = 0.f;
    if (lo < hi && nvox % 4 == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0) {
        const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll 4
        for (int64_t t = lo / 4 + threadIdx.x; t < hi / 4; t += blockDim.x) {
            const float4 v = q[t];
            m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        }
    } else {
        for (int64_t t = lo + threadIdx.x; t < hi; t += blockDim.x) m = fmaxf(m, fabsf(p[t]));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        partial[(int64_t)b * MAXABS_CHUNKS + blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

__global__ void k_maxabs_final(const float* __restrict__ partial, int B, float* __restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float m = 0.f;
    for (int c = 0; c < MAXABS_CHUNKS; ++c) m = fmaxf(m, partial[(int64_t)b * MAXABS_CHUNKS + c]);
    out[b] = m;
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
        int i, j, k;
        const int64_t b = split3(t, nx, ny, nz, i, j, k);
        const int64_t v = t - b * nvox;
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
        int64_t v;
        const double f = (double)scale[divmod(t, nvox, v)] * inv_out;
        phi[t] = (float)((double)phi_c[t] + (double)y[t * NC] * f);
        if (phidot) phidot[t] = (float)((double)y[t * NC + 1] * f);
    }
}

// out = the sum of n partials in a fixed order: thread t adds partials t,
// t + 256, ..., then the wave butterflies and the four waves pairwise.  One
// workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partial, int n,
                                                      double* __restrict__ out) {
    __shared__ double red[4];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) v += partial[i];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
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
        int i, j, k;
        const int64_t b = split3(t, cx, cy, cz, i, j, k);
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
        int i, j, k;
        const int64_t b = split3(t, fx, fy, fz, i, j, k);
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
