// Local outer boundaries: the ghost layer follows the interior after every
// substep, instead of being frozen over a hydrodynamical step.
//
//   Robin    -- the paper's default outer boundary, a Robin condition that
//               is equivalent to a monopole far field (Sec. 2, Sec. 4), read
//               as the monopole fall-off d(r phi)/dr = 0 between a ghost and
//               its interior neighbour: r_g phi_g = r_i phi_i (r from the
//               expansion centre).  Exact for -G M / r.
//   outgoing -- its radiative form d(r phi)/dt + c d(r phi)/dr = 0 (an
//               outgoing spherical wave), so that errors leave through the
//               boundary (Sec. 4).  With u = r phi and d/dr = d/dn / cos(theta)
//               at the midpoint x_f of ghost and neighbour, the box scheme
//               centred on x_f and t^{n+1/2} gives, alpha = c dt / (dx cos(theta)),
//                 u_g^{n+1} = [(1 - alpha) u_g^n + (1 + alpha) u_i^n
//                              - (1 - alpha) u_i^{n+1}] / (1 + alpha).
//   periodic -- ghost = the interior cell at the opposite face; the source
//               subtracts the domain-mean density (Sec. 4).
#pragma once

#include "common.hpp"

namespace hgs {

struct LocalGeom {
    double x0, y0, z0, dx, ox, oy, oz;
};

// One thread per face ghost; grid (ceil(max(nx, ny) / 256), max(ny, nz), 6),
// face f = blockIdx.z in the order x-, x+, y-, y+, z-, z+.  In-face index
// (a, b): x faces (j, k), y faces (i, k), z faces (i, j).  nxt holds the new
// level's interior; cur (the previous level with its ghosts) is read by the
// outgoing rule only, and cur == nullptr applies each rule's steady form.
template <typename S>
__global__ __launch_bounds__(256) void k_local_ghosts(Layout L, LocalGeom g, int bc, S* __restrict__ nxt,
                                                      const S* __restrict__ cur, double c_dt) {
    const int f = blockIdx.z, axis = f >> 1, hi = f & 1;
    const int a = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
    const int na = axis == 0 ? L.ny : L.nx, nb = axis == 2 ? L.ny : L.nz;
    if (a >= na || b >= nb) return;
    const int n[3] = {L.nx, L.ny, L.nz};
    int gh[3], in[3], op[3];
    gh[0] = axis == 0 ? 0 : a;
    gh[1] = axis == 0 ? a : (axis == 1 ? 0 : b);
    gh[2] = axis == 2 ? 0 : b;
    for (int d = 0; d < 3; ++d) in[d] = op[d] = gh[d];
    gh[axis] = hi ? n[axis] : -1;
    in[axis] = hi ? n[axis] - 1 : 0;
    op[axis] = hi ? 0 : n[axis] - 1;
    const int64_t pg = L.idx(gh[0], gh[1], gh[2]);
    const int64_t pi = L.idx(in[0], in[1], in[2]);
    if (bc == HGS_BC_PERIODIC) {
        nxt[pg] = nxt[L.idx(op[0], op[1], op[2])];
        return;
    }
    const double lo[3] = {g.x0 - g.ox, g.y0 - g.oy, g.z0 - g.oz};
    double xg[3], xi[3];
    for (int d = 0; d < 3; ++d) {
        xg[d] = lo[d] + (gh[d] + 0.5) * g.dx;
        xi[d] = lo[d] + (in[d] + 0.5) * g.dx;
    }
    const double rg = sqrt(xg[0] * xg[0] + xg[1] * xg[1] + xg[2] * xg[2]);
    const double ri = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
    double v;
    if (bc == HGS_BC_ROBIN || cur == nullptr) {
        v = ri * (double)nxt[pi] / rg;
    } else {
        const double xf[3] = {0.5 * (xg[0] + xi[0]), 0.5 * (xg[1] + xi[1]), 0.5 * (xg[2] + xi[2])};
        const double rf = sqrt(xf[0] * xf[0] + xf[1] * xf[1] + xf[2] * xf[2]);
        const double cth = (hi ? xf[axis] : -xf[axis]) / rf;
        const double al = c_dt / (g.dx * cth);
        const double ug0 = rg * (double)cur[pg], ui0 = ri * (double)cur[pi], ui1 = ri * (double)nxt[pi];
        const double ug1 = ((1.0 - al) * ug0 + (1.0 + al) * ui0 - (1.0 - al) * ui1) / (1.0 + al);
        v = ug1 / rg;
    }
    nxt[pg] = (S)v;
}

// Sum of a compact field in FP64: per-workgroup partials (grid-stride, fixed
// order), then one thread adds them in order and scales.
template <typename S>
__global__ __launch_bounds__(256) void k_sum_partial(const S* __restrict__ f, int64_t n, double* __restrict__ partial) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        acc += (double)f[t];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_sum_final(const double* __restrict__ partial, int nb, double scale, double* __restrict__ out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < nb; ++i) s += partial[i];
        *out = s * scale;
    }
}

}  // namespace hgs

namespace hgs {

// Largest signal speed c_s + |v| over the cells (FP64) and a non-finite flag,
// per workgroup: partial[2 b] = max, partial[2 b + 1] = 1 if any value was not
// finite.  vx, vy, vz nullable (0).
template <typename S>
__global__ __launch_bounds__(256) void k_speed_partial(const S* __restrict__ cs, const S* __restrict__ vx,
                                                       const S* __restrict__ vy, const S* __restrict__ vz, int64_t n,
                                                       double* __restrict__ partial) {
    __shared__ double red[4][2];
    double m = 0.0, bad = 0.0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const double a = vx ? (double)vx[t] : 0.0, b = vy ? (double)vy[t] : 0.0, c = vz ? (double)vz[t] : 0.0;
        const double v = (double)cs[t] + sqrt(a * a + b * b + c * c);
        if (!isfinite(v)) bad = 1.0;
        else m = fmax(m, v);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        m = fmax(m, __shfl_xor(m, o, 64));
        bad = fmax(bad, __shfl_xor(bad, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6][0] = m;
        red[threadIdx.x >> 6][1] = bad;
    }
    __syncthreads();
    if (threadIdx.x < 2)
        partial[2 * blockIdx.x + threadIdx.x] =
            fmax(fmax(red[0][threadIdx.x], red[1][threadIdx.x]), fmax(red[2][threadIdx.x], red[3][threadIdx.x]));
}

__global__ void k_speed_final(const double* __restrict__ partial, int nb, double* __restrict__ out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double m = 0.0, bad = 0.0;
        for (int i = 0; i < nb; ++i) {
            m = fmax(m, partial[2 * i]);
            bad = fmax(bad, partial[2 * i + 1]);
        }
        out[0] = m;
        out[1] = bad;
    }
}

// sum over interior cells of rho * phi (phi in the padded layout), FP64
// partials per workgroup; the caller scales by dx^3 / 2 for W.
template <typename S>
__global__ __launch_bounds__(256) void k_dot_partial(const S* __restrict__ rho, const S* __restrict__ phi, Layout L,
                                                     double* __restrict__ partial) {
    __shared__ double red[4];
    double acc = 0.0;
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % L.nx);
        const int j = (int)((t / L.nx) % L.ny);
        const int k = (int)(t / ((int64_t)L.nx * L.ny));
        acc += (double)rho[t] * (double)phi[L.idx(i, j, k)];
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

}  // namespace hgs

namespace hgs {

// Extended gravity-only grid (Sec. 4: solve the wave equation on a grid wider
// than the hydrodynamics region, the extension taken as vacuum).  Compact
// fields: inner (nz, ny, nx) <-> outer (nz + 2e, ny + 2e, nx + 2e).
// k_embed writes every outer cell (inner values in the centre, 0 around).
template <typename S>
__global__ __launch_bounds__(256) void k_embed(const S* __restrict__ inner, int nx, int ny, int nz, int e,
                                               S* __restrict__ outer) {
    const int ox = nx + 2 * e, oy = ny + 2 * e, oz = nz + 2 * e;
    const int64_t total = (int64_t)ox * oy * oz;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % ox) - e;
        const int j = (int)((t / ox) % oy) - e;
        const int k = (int)(t / ((int64_t)ox * oy)) - e;
        const bool in = i >= 0 && i < nx && j >= 0 && j < ny && k >= 0 && k < nz;
        outer[t] = in ? inner[((int64_t)k * ny + j) * nx + i] : (S)0;
    }
}

template <typename S>
__global__ __launch_bounds__(256) void k_extract(const S* __restrict__ outer, int nx, int ny, int nz, int e,
                                                 S* __restrict__ inner) {
    const int ox = nx + 2 * e, oy = ny + 2 * e;
    const int64_t total = (int64_t)nx * ny * nz;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % nx);
        const int j = (int)((t / nx) % ny);
        const int k = (int)(t / ((int64_t)nx * ny));
        inner[t] = outer[((int64_t)(k + e) * oy + (j + e)) * ox + (i + e)];
    }
}

}  // namespace hgs
