// Temporally blocked leapfrog: T substeps of Eq. (2) in one launch.
//
// Valid because rho and the Dirichlet ghosts are frozen over the substeps of
// one hydrodynamical step (Sec. 2: the wave equation is sub-cycled with the
// density held fixed).  Out of place: (phi^n, phi^{n-1}) -> (phi^{n+T},
// phi^{n+T-1}) in two other buffers, so no tile ever overwrites a value a
// neighbouring tile still has to read.
//
// Shape of the computation.  A workgroup owns an (x, y) tile of
// (64 - 2T) x (W*R - 2T) columns, extended by T on every side, and marches up
// a chunk of z planes as a pipeline: when input plane p arrives, level t
// (substep n+t) is computed at plane p - t, for t = 1..T.  Lane l of wave w holds
// column x = x_tile - T + l and the R rows y = y_tile - T + w*R + r in
// registers, with a three-plane window (z-1, z, z+1) per level, stored in the
// storage type (every level is rounded to it anyway) and updated in it (the
// FP32 increment form for FP32 storage).  Neighbours:
//   z: the thread's own window;
//   y: the thread's own rows, except across strip edges, which go through a
//      double-buffered LDS slot per level (one barrier per plane);
//   x: the neighbouring lanes of the same wave (DPP wave shift for FP32).
// The valid region shrinks by one column per level, so the extended ring of
// width T makes level T exact on the tile; rings of garbage outside it are
// never written.  Cells outside the grid interior (ghosts) keep their input
// value at every level.  Every level is rounded to the storage type exactly as
// a streaming launch stores it, so any T gives bit-identical results.
//
// The plane loop is unrolled by U = lcm(3, 2, T) so that the three-plane
// windows, the LDS slot parity and the ring of rho planes rotate by
// compile-time index instead of register moves.  Tiles whose extended region
// lies inside the grid take a path without per-cell boundary selects.
#pragma once

#include "common.hpp"

namespace hgs {

// value held by lane l-1 (xm) / lane l+1 (xp) of the wave
// (DPP wave_shr:1 / wave_shl:1; the lane without a source reads 0 and is
// always outside the valid region)
__device__ __forceinline__ float lane_prev(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_next(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_prev(double v) { return __shfl_up(v, 1, 64); }
__device__ __forceinline__ double lane_next(double v) { return __shfl_down(v, 1, 64); }

template <int T>
struct Unroll {
    static constexpr int U = (T == 4) ? 12 : 6;  // lcm(3, 2, T, prefetch depth 3)
};
// Input planes loaded ahead: one plane step keeps a SIMD busy for about a
// microsecond, so three planes in flight cover the HBM latency under load
// (measured at 512^3: 4% faster than two).
constexpr int PF = 3;

template <typename S, int T, int R, int W>
struct TBShared {
    S edge[T][2][W][2][64];  // [level][slot][wave][0 first row, 1 last row][lane]
};

template <typename S, int T, int R, int W, bool EDGE>
struct TBTile {
    static constexpr int IX = 64 - 2 * T;
    static constexpr int IY = W * R - 2 * T;
    static constexpr int U = Unroll<T>::U;

    // per-thread constants
    const S* in_n;
    const S* in_nm1;
    const S* rho;
    S* out_n;
    S* out_nm1;
    const Layout& L;
    const StepCoef& c;
    TBShared<S, T, R, W>& sh;
    int lane, w, x, y0, k0, k1, wm, wp;
    int off_p[R];  // lane offsets within a padded plane (clamped to the ghost box)
    int off_c[R];  // lane offsets within a compact rho plane (clamped to the interior)
    bool x_in, y_in[R], in_ok[R], out_ok[R];

    // pipeline state
    S win[T][3][R];  // [level][ring slot][row]
    S rq[T][R];      // ring of rho planes
    S pn[PF][R], po[PF][R], pr[PF][R];  // prefetch ring

    __device__ TBTile(const S* a, const S* b, const S* rh, S* o0, S* o1, const Layout& Ly, const StepCoef& cc,
                      TBShared<S, T, R, W>& s, int tx, int ty, int kk0, int kk1)
        : in_n(a), in_nm1(b), rho(rh), out_n(o0), out_nm1(o1), L(Ly), c(cc), sh(s) {
        lane = threadIdx.x & 63;
        w = threadIdx.x >> 6;
        x = tx * IX - T + lane;
        y0 = ty * IY - T + w * R;
        k0 = kk0;
        k1 = kk1;
        wm = w > 0 ? w - 1 : 0;
        wp = w < W - 1 ? w + 1 : W - 1;
        x_in = x >= 0 && x < L.nx;
        const bool x_out = x_in && lane >= T && lane < T + IX;
        const int xc = min(max(x, -1), L.nx);
        const int xr = min(max(x, 0), L.nx - 1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = y0 + r;
            const int er = w * R + r;
            y_in[r] = y >= 0 && y < L.ny;
            in_ok[r] = x_in && y_in[r];
            out_ok[r] = x_out && y_in[r] && er >= T && er < T + IY;
            const int yc = min(max(y, -1), L.ny);
            const int yr = min(max(y, 0), L.ny - 1);
            off_p[r] = (yc + HALO) * L.pitch + (xc + L.xoff);
            off_c[r] = yr * L.nx + xr;
        }
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                win[t][0][r] = win[t][1][r] = win[t][2][r] = (S)0;
                rq[t][r] = (S)0;
            }
    }

    // inputs of plane p: phi^n(p), phi^{n-1}(p-1), rho(p-1), into ring slot B.
    // Loads are never predicated: plane and lane offsets are clamped into the
    // ghost box (the interior for rho), and every value read that way lands in
    // a cell outside the interior, which keeps its input value and feeds no
    // valid cell.
    template <int B>
    __device__ __forceinline__ void load(int p) {
        const int pc = min(max(p, -1), L.nz);
        const int qc = min(max(p - 1, 0), L.nz - 1);
        const S* bn = in_n + (int64_t)(pc + HALO) * L.plane;
        const S* bo = in_nm1 + (int64_t)(qc + HALO) * L.plane;
        const S* br = rho + (int64_t)qc * L.nx * L.ny;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            pn[B][r] = bn[off_p[r]];
            po[B][r] = bo[off_p[r]];
            pr[B][r] = br[off_c[r]];
        }
    }

    // one pipeline step at phase PH (= iteration index mod U), input plane p
    template <int PH>
    __device__ __forceinline__ void step(int p, int pend) {
        constexpr int NEW = PH % 3, MID = (PH + 2) % 3, OLD = (PH + 1) % 3;
        constexpr int SLOT = PH & 1, PREV = SLOT ^ 1;
        constexpr int B = PH % PF;
        S old1[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            win[0][NEW][r] = pn[B][r];
            old1[r] = po[B][r];
            rq[PH % T][r] = pr[B][r];
        }
        if (p + PF < pend) load<B>(p + PF);
        __syncthreads();  // LDS writes of plane p-1 are visible; its reads are done
        sh.edge[0][SLOT][w][0][lane] = win[0][NEW][0];
        sh.edge[0][SLOT][w][1][lane] = win[0][NEW][R - 1];
#pragma unroll
        for (int t = 1; t <= T; ++t) {
            const int q = p - t;
            const bool z_in = q >= 0 && q < L.nz;
            // level t-1 holds plane q in MID, q+1 in NEW, q-1 in OLD; level t-2
            // holds plane q in OLD (its NEW is q+2)
            S nv[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const S ce = win[t - 1][MID][r];
                const S zm = win[t - 1][OLD][r];
                const S zp = win[t - 1][NEW][r];
                const S ym = (r > 0) ? win[t - 1][MID][r - 1] : sh.edge[t - 1][PREV][wm][1][lane];
                const S yp = (r < R - 1) ? win[t - 1][MID][r + 1] : sh.edge[t - 1][PREV][wp][0][lane];
                const S xm = (S)lane_prev(ce);
                const S xp = (S)lane_next(ce);
                const S ol = (t == 1) ? old1[r] : win[t >= 2 ? t - 2 : 0][OLD][r];
                const int RS = ((PH - t + 1) % T + T) % T;  // ring slot of rho(p - t)
                const S v = (S)update(c, ce, xm, xp, ym, yp, zm, zp, ol, rq[RS][r]);
                if (EDGE)
                    nv[r] = (in_ok[r] && z_in) ? v : ce;
                else
                    nv[r] = z_in ? v : ce;
            }
            if (t < T) {
#pragma unroll
                for (int r = 0; r < R; ++r) win[t][NEW][r] = nv[r];
                sh.edge[t][SLOT][w][0][lane] = nv[0];
                sh.edge[t][SLOT][w][1][lane] = nv[R - 1];
            } else if (q >= k0 && q < k1) {
                S* on = out_n + (int64_t)(q + HALO) * L.plane;
                S* oo = out_nm1 + (int64_t)(q + HALO) * L.plane;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (out_ok[r]) {
                        on[off_p[r]] = nv[r];
                        oo[off_p[r]] = win[T - 1][MID][r];
                    }
                }
            }
        }
    }

    template <int PH>
    __device__ __forceinline__ bool run_from(int p, int pend) {
        if constexpr (PH < U) {
            if (p + PH >= pend) return false;
            step<PH>(p + PH, pend);
            return run_from<PH + 1>(p, pend);
        }
        return true;
    }

    __device__ void run() {
        const int pend = k1 + T;
        load<0>(k0 - T);
        load<1>(k0 - T + 1);
        load<2>(k0 - T + 2);
        for (int p = k0 - T; p < pend; p += U)
            if (!run_from<0>(p, pend)) break;
    }
};

template <typename S, int T, int R, int W>
__global__ __launch_bounds__(64 * W) void k_leapfrog_tblock(const S* __restrict__ in_n, const S* __restrict__ in_nm1,
                                                            const S* __restrict__ rho, S* __restrict__ out_n,
                                                            S* __restrict__ out_nm1, Layout L, StepCoef c, int zc,
                                                            int tiles_x, int tiles_y) {
    constexpr int IX = 64 - 2 * T;
    constexpr int IY = W * R - 2 * T;
    static_assert(IX > 0 && IY > 0, "tile too small for the temporal depth");
    __shared__ TBShared<S, T, R, W> sh;
    // tiles vary fastest and z chunks slowest, so the workgroups resident at
    // one time are neighbours at the same heights and share halo lines in L2
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = bid % tiles_x;
    const int ty = (bid / tiles_x) % tiles_y;
    const int tz = bid / (tiles_x * tiles_y);
    const int k0 = tz * zc;
    const int k1 = min(k0 + zc, L.nz);
    // the extended tile lies strictly inside the grid: no per-cell boundary work
    const int xlo = tx * IX - T, ylo = ty * IY - T;
    const bool inner = xlo >= 0 && xlo + 64 <= L.nx && ylo >= 0 && ylo + W * R <= L.ny;
    if (inner) {
        TBTile<S, T, R, W, false> t(in_n, in_nm1, rho, out_n, out_nm1, L, c, sh, tx, ty, k0, k1);
        t.run();
    } else {
        TBTile<S, T, R, W, true> t(in_n, in_nm1, rho, out_n, out_nm1, L, c, sh, tx, ty, k0, k1);
        t.run();
    }
}

// Launch geometry of the fused kernel for a grid.
struct TBlockDims {
    int tiles_x, tiles_y, zc, nblocks;
};

// Number of z chunks: each workgroup occupies one CU slot for (chunk planes +
// 2T) pipeline steps and the launch runs in ceil(blocks / slots) rounds, so
// pick the chunk count that minimises rounds x steps.
template <int T, int R, int W>
inline TBlockDims tblock_dims(const Layout& L, int slots) {
    constexpr int IX = 64 - 2 * T;
    constexpr int IY = W * R - 2 * T;
    TBlockDims d;
    d.tiles_x = (L.nx + IX - 1) / IX;
    d.tiles_y = (L.ny + IY - 1) / IY;
    const int64_t cols = (int64_t)d.tiles_x * d.tiles_y;
    int best = 1;
    int64_t best_cost = -1;
    const int maxz = std::max(1, std::min(64, L.nz / (2 * T)));
    for (int nzc = 1; nzc <= maxz; ++nzc) {
        const int zc = (L.nz + nzc - 1) / nzc;
        const int64_t nb = cols * ((L.nz + zc - 1) / zc);
        const int64_t cost = ((nb + slots - 1) / slots) * (int64_t)(zc + 2 * T);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = nzc;
        }
    }
    d.zc = (L.nz + best - 1) / best;
    d.nblocks = (int)(cols * ((L.nz + d.zc - 1) / d.zc));
    return d;
}

// Tile shape (R rows per thread, W waves per workgroup) per storage type and
// depth, chosen by measurement on MI355X at 512^3 and bounded by registers:
// every level keeps three planes per cell in registers.  FP32: 16 waves of
// 2 rows (extended tile 64 x 32; 112 VGPRs at T = 4, so the 16 waves fit one
// CU): as fast as 8 waves of 4 rows at T = 4 and 6-11% faster at T = 2, 3.
// FP64: 8 waves of 2 rows.
template <typename S, int T>
struct TBConfig {
    static constexpr int R = 2;
    static constexpr int W = sizeof(S) == 4 ? 16 : 8;
};

template <typename S, int T>
void launch_tblock_t(const S* in_n, const S* in_nm1, const S* rho, S* out_n, S* out_nm1, const Layout& L,
                     const StepCoef& c, int ncu, hipStream_t st) {
    constexpr int R = TBConfig<S, T>::R;
    constexpr int W = TBConfig<S, T>::W;
    const TBlockDims d = tblock_dims<T, R, W>(L, ncu);
    hipLaunchKernelGGL((k_leapfrog_tblock<S, T, R, W>), dim3(d.nblocks), dim3(64 * W), 0, st, in_n, in_nm1, rho, out_n,
                       out_nm1, L, c, d.zc, d.tiles_x, d.tiles_y);
}

// ncu: compute units of the device (one resident workgroup of this kernel each)
template <typename S>
void launch_tblock(const S* in_n, const S* in_nm1, const S* rho, S* out_n, S* out_nm1, const Layout& L,
                   const StepCoef& c, int T, int ncu, hipStream_t st) {
    switch (T) {
        case 2: launch_tblock_t<S, 2>(in_n, in_nm1, rho, out_n, out_nm1, L, c, ncu, st); break;
        case 3: launch_tblock_t<S, 3>(in_n, in_nm1, rho, out_n, out_nm1, L, c, ncu, st); break;
        case 4: launch_tblock_t<S, 4>(in_n, in_nm1, rho, out_n, out_nm1, L, c, ncu, st); break;
        default: break;
    }
}

}  // namespace hgs
