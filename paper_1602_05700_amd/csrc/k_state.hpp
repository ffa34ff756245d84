// State bookkeeping kernels (fill, set_state, dt rescale, readback, raw copies,
// ghost faces) and the FP64 residual norms of the steady state L_h phi = 4 pi G rho.
#pragma once

#include "common.hpp"

namespace hgs {

// Interior cells are addressed through a flat index t in [0, nx*ny*nz):
// i = t % nx, j = (t / nx) % ny, k = t / (nx*ny), i.e. the caller's compact layout.
struct Flat {
    int i, j, k;
};
__device__ __forceinline__ Flat unflat(int64_t t, const Layout& L) {
    Flat f;
    f.i = (int)(t % L.nx);
    int64_t r = t / L.nx;
    f.j = (int)(r % L.ny);
    f.k = (int)(r / L.ny);
    return f;
}

#define HGS_GRID_STRIDE(t, n) \
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (n); t += (int64_t)gridDim.x * blockDim.x)

// Whole padded buffer: NaN everywhere, then 0 on the interior and the six ghost
// faces (edges and corners of the ghost box and all other padding stay NaN).
template <typename S>
__global__ void k_init_buffer(S* b, Layout L) {
    HGS_GRID_STRIDE(t, L.total) {
        int64_t kz = t / L.plane;
        int64_t rem = t % L.plane;
        int jy = (int)(rem / L.pitch);
        int ix = (int)(rem % L.pitch);
        int i = ix - L.xoff, j = jy - HALO, k = (int)kz - HALO;
        int outside = (i < 0 || i >= L.nx) + (j < 0 || j >= L.ny) + (k < 0 || k >= L.nz);
        bool in_box = i >= -1 && i <= L.nx && j >= -1 && j <= L.ny && k >= -1 && k <= L.nz;
        b[t] = (in_box && outside <= 1) ? (S)0 : (S)__builtin_nan("");
    }
}

template <typename S>
__global__ void k_set_state(S* cur, S* old, const S* __restrict__ phi, const S* __restrict__ phidot, double dt,
                            Layout L) {
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    HGS_GRID_STRIDE(t, n) {
        Flat f = unflat(t, L);
        int64_t o = L.idx(f.i, f.j, f.k);
        double p = (double)phi[t];
        double pd = phidot ? (double)phidot[t] : 0.0;
        cur[o] = (S)p;
        old[o] = (S)(p - dt * pd);
    }
}

// phi^{n-1} <- phi^n - ratio (phi^n - phi^{n-1}), ratio = dt_new / dt_old.
template <typename S>
__global__ void k_rescale(const S* __restrict__ cur, S* old, double ratio, Layout L) {
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    HGS_GRID_STRIDE(t, n) {
        Flat f = unflat(t, L);
        int64_t o = L.idx(f.i, f.j, f.k);
        double c = (double)cur[o];
        double d = c - (double)old[o];
        double u = ratio * d;
        old[o] = (S)(c - u);
    }
}

template <typename S>
__global__ void k_potential(const S* __restrict__ cur, const S* __restrict__ old, double inv_dt, Layout L,
                            S* __restrict__ phi, S* __restrict__ phidot) {
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    HGS_GRID_STRIDE(t, n) {
        Flat f = unflat(t, L);
        int64_t o = L.idx(f.i, f.j, f.k);
        double c = (double)cur[o];
        if (phi) phi[t] = (S)c;
        if (phidot) phidot[t] = (inv_dt > 0.0) ? (S)((c - (double)old[o]) * inv_dt) : (S)0;
    }
}

// Raw interior copy, padded <-> compact, bit-exact.
template <typename S>
__global__ void k_interior_out(const S* __restrict__ src, Layout L, S* __restrict__ dst) {
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    HGS_GRID_STRIDE(t, n) {
        Flat f = unflat(t, L);
        dst[t] = src[L.idx(f.i, f.j, f.k)];
    }
}
template <typename S>
__global__ void k_interior_in(const S* __restrict__ src, Layout L, S* __restrict__ dst) {
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    HGS_GRID_STRIDE(t, n) {
        Flat f = unflat(t, L);
        dst[L.idx(f.i, f.j, f.k)] = src[t];
    }
}

// Face cell t (face order x-, x+, y-, y+, z-, z+) -> padded coordinates.
__device__ __forceinline__ Flat face_cell(int64_t u, const Layout& L) {
    const int64_t nxf = (int64_t)L.nz * L.ny, nyf = (int64_t)L.nz * L.nx, nzf = (int64_t)L.ny * L.nx;
    Flat f;
    if (u < 2 * nxf) {
        int side = (int)(u / nxf);
        int64_t v = u % nxf;
        f.k = (int)(v / L.ny);
        f.j = (int)(v % L.ny);
        f.i = side ? L.nx : -1;
    } else if ((u -= 2 * nxf) < 2 * nyf) {
        int side = (int)(u / nyf);
        int64_t v = u % nyf;
        f.k = (int)(v / L.nx);
        f.i = (int)(v % L.nx);
        f.j = side ? L.ny : -1;
    } else {
        u -= 2 * nyf;
        int side = (int)(u / nzf);
        int64_t v = u % nzf;
        f.j = (int)(v / L.nx);
        f.i = (int)(v % L.nx);
        f.k = side ? L.nz : -1;
    }
    return f;
}

template <typename S>
__global__ void k_faces_out(const S* __restrict__ src, Layout L, S* __restrict__ dst) {
    const int64_t n = 2 * ((int64_t)L.nz * L.ny + (int64_t)L.nz * L.nx + (int64_t)L.ny * L.nx);
    HGS_GRID_STRIDE(t, n) {
        Flat f = face_cell(t, L);
        dst[t] = src[L.idx(f.i, f.j, f.k)];
    }
}
template <typename S>
__global__ void k_faces_in(const S* __restrict__ src, Layout L, S* b0, S* b1, S* b2, S* b3) {
    const int64_t n = 2 * ((int64_t)L.nz * L.ny + (int64_t)L.nz * L.nx + (int64_t)L.ny * L.nx);
    HGS_GRID_STRIDE(t, n) {
        Flat f = face_cell(t, L);
        const int64_t o = L.idx(f.i, f.j, f.k);
        const S v = src[t];
        b0[o] = v;
        b1[o] = v;
        b2[o] = v;
        b3[o] = v;
    }
}

// Residual partial sums per workgroup: [rr, bb, ss, pp, bad].
//   r = L_h phi - s,  s = 4 pi G (rho - rbar)  (rbar nullable: 0),
//   b = s - (adjacent ghosts)/dx^2 for a fixed boundary (ghosts_in_b), else
//   b = s: a local boundary's ghosts are images of interior unknowns.
constexpr int NRED = 5;
// One workgroup per (64 x 4 column tile, z chunk); each thread marches its
// column.  Fixed-order reductions: wave butterfly, then the four waves.
template <typename S>
__global__ __launch_bounds__(256) void k_residual_partial(const S* __restrict__ phi, const S* __restrict__ rho,
                                                          Layout L, double idx2, double four_pi_g, int zc,
                                                          int tiles_x, int tiles_y, const double* __restrict__ rbar,
                                                          int ghosts_in_b, double* __restrict__ partial) {
    __shared__ double red[4][NRED];
    double acc[NRED] = {0, 0, 0, 0, 0};
    const int bid = blockIdx.x;
    const int tx = bid % tiles_x;
    const int ty = (bid / tiles_x) % tiles_y;
    const int tz = bid / (tiles_x * tiles_y);
    const int i = tx * 64 + threadIdx.x;
    const int j = ty * 4 + threadIdx.y;
    if (i < L.nx && j < L.ny) {
        const int k0 = tz * zc;
        const int k1 = min(k0 + zc, L.nz);
        const int64_t sxy = (int64_t)L.nx * L.ny;
        const S* pc = phi + L.idx(i, j, k0);
        const S* pr = rho + (int64_t)k0 * sxy + (int64_t)j * L.nx + i;
        const double rb = rbar ? *rbar : 0.0;
        for (int k = k0; k < k1; ++k) {
            const double c = (double)pc[0];
            const double xm = (double)pc[-1], xp = (double)pc[1];
            const double ym = (double)pc[-L.pitch], yp = (double)pc[L.pitch];
            const double zm = (double)pc[-L.plane], zp = (double)pc[L.plane];
            double gb = 0.0;
            if (i == 0) gb += xm;
            if (i == L.nx - 1) gb += xp;
            if (j == 0) gb += ym;
            if (j == L.ny - 1) gb += yp;
            if (k == 0) gb += zm;
            if (k == L.nz - 1) gb += zp;
            const double rv = (double)pr[0];
            const double s = four_pi_g * (rv - rb);
            const double nb = ((xm + xp) + (ym + yp)) + (zm + zp);
            const double r = (nb - 6.0 * c) * idx2 - s;
            const double b = ghosts_in_b ? s - gb * idx2 : s;
            acc[0] += r * r;
            acc[1] += b * b;
            acc[2] += s * s;
            acc[3] += c * c;
            if (!isfinite(c) || !isfinite(rv)) acc[4] = 1.0;
            pc += L.plane;
            pr += sxy;
        }
    }
    const int lane = threadIdx.x, wave = threadIdx.y;
#pragma unroll
    for (int q = 0; q < NRED; ++q) {
        double v = acc[q];
        if (q == 4) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
        } else {
            v = wave_sum(v);
        }
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    const int t = threadIdx.y * 64 + threadIdx.x;
    if (t < NRED) {
        double v = (t == 4) ? fmax(fmax(red[0][t], red[1][t]), fmax(red[2][t], red[3][t]))
                            : ((red[0][t] + red[1][t]) + (red[2][t] + red[3][t]));
        partial[(size_t)blockIdx.x * NRED + t] = v;
    }
}

__global__ __launch_bounds__(256) void k_residual_final(const double* __restrict__ partial, int nblocks,
                                                        double* __restrict__ out) {
    __shared__ double red[4][NRED];
    double acc[NRED] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += 256) {
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += partial[(size_t)b * NRED + q];
        acc[4] = fmax(acc[4], partial[(size_t)b * NRED + 4]);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NRED; ++q) {
        double v = acc[q];
        if (q == 4) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
        } else {
            v = wave_sum(v);
        }
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < NRED) {
        const int q = threadIdx.x;
        out[q] = (q == 4) ? fmax(fmax(red[0][q], red[1][q]), fmax(red[2][q], red[3][q]))
                          : ((red[0][q] + red[1][q]) + (red[2][q] + red[3][q]));
    }
}

// The fallback rule of a predicted start, decided on the device from the
// residual sums of the state (k_residual_final's out: [sum r^2, sum b^2, ...,
// non-finite count]): the start is kept when it is finite and its R_b is below
// the zero start's R_b = 1, i.e. sum r^2 < sum b^2; otherwise the interiors of
// phi^n and phi^{n-1} are set to zero.  The decision is uniform, so a kept
// start costs each workgroup one read of two values.
template <typename S>
__global__ __launch_bounds__(256) void k_keep_or_zero(const double* __restrict__ red, Layout L, S* __restrict__ p0,
                                                      S* __restrict__ p1, int32_t* __restrict__ kept) {
    const bool keep = red[4] == 0.0 && red[0] < red[1];
    if (kept && blockIdx.x == 0 && threadIdx.x == 0) *kept = keep ? 1 : 0;
    if (keep) return;
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        split3(c, L.nx, L.ny, L.nz, i, j, k);
        const int64_t o = L.idx(i, j, k);
        p0[o] = (S)0;
        p1[o] = (S)0;
    }
}

}  // namespace hgs
