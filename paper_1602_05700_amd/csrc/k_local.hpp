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

// One thread per face ghost; grid (ceil(max(nx, ny) / 256), max(ny, nz), 6),
// face f = blockIdx.z in the order x-, x+, y-, y+, z-, z+.  In-face index
// (a, b): x faces (j, k), y faces (i, k), z faces (i, j).  The ghosts of nxt
// from its interior: the periodic copy, else Robin's relation (the Robin rule,
// and the steady form of the outgoing one, which the state set-up uses).  The
// substeps themselves evaluate (Robin) or advance (outgoing) the ghosts they
// need: outgoing_ghost and robin_ghost, with these operands, in the stencil
// kernels.
template <typename S>
__global__ __launch_bounds__(256) void k_local_ghosts(Layout L, LocalGeom g, int bc, S* __restrict__ nxt) {
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
    const S ci[3] = {local_coord<S>(g.x0, g.ox, g.dx, in[0]), local_coord<S>(g.y0, g.oy, g.dx, in[1]),
                     local_coord<S>(g.z0, g.oz, g.dx, in[2])};
    S cg[3] = {ci[0], ci[1], ci[2]};
    cg[axis] = axis == 0   ? local_coord<S>(g.x0, g.ox, g.dx, gh[0])
               : axis == 1 ? local_coord<S>(g.y0, g.oy, g.dx, gh[1])
                           : local_coord<S>(g.z0, g.oz, g.dx, gh[2]);
    nxt[pg] = robin_ghost(local_r2(ci[0], ci[1], ci[2]), local_r2(cg[0], cg[1], cg[2]), nxt[pi]);
}

// Block-wide FP64 sum over 256 threads in a fixed order (wave butterflies,
// then the four waves pairwise); every thread returns the same sum.
__device__ __forceinline__ double block_sum_256(double v, double* red4) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red4[0] + red4[1]) + (red4[2] + red4[3]);
}

// Sum of a compact field in FP64: per-workgroup partials, then one workgroup
// adds them.  Threads take 16-byte vectors of the field (when it is 16-byte
// aligned) in a grid-stride loop with four independent loads in flight, and
// the scalar tail; the order of every addition is fixed, so the result is the
// same from run to run.
template <typename S>
__global__ __launch_bounds__(256) void k_sum_partial(const S* __restrict__ f, int64_t n, double* __restrict__ partial) {
    constexpr int N = 16 / sizeof(S);
    typedef S VT __attribute__((ext_vector_type(N)));
    __shared__ double red[4];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t done = 0;
    if ((reinterpret_cast<uintptr_t>(f) & 15) == 0) {
        const VT* fv = reinterpret_cast<const VT*>(f);
        const int64_t nv = n / N;
        int64_t t = t0;
        for (; t + 3 * stride < nv; t += 4 * stride) {
            VT v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = fv[t + u * stride];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int e = 0; e < N; ++e) a[u] += (double)v[u][e];
        }
        for (; t < nv; t += stride) {
            const VT v = fv[t];
#pragma unroll
            for (int e = 0; e < N; ++e) a[0] += (double)v[e];
        }
        done = nv * N;
    }
    for (int64_t t = done + t0; t < n; t += stride) a[1] += (double)f[t];
    const double s = block_sum_256((a[0] + a[1]) + (a[2] + a[3]), red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out = scale * (sum of the nb partials): thread t adds partials t, t + 256,
// ... in order, then the fixed block tree.  Launched as one workgroup of 256.
__global__ __launch_bounds__(256) void k_sum_final(const double* __restrict__ partial, int nb, double scale,
                                                   double* __restrict__ out) {
    __shared__ double red[4];
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) v += partial[i];
    const double s = block_sum_256(v, red);
    if (threadIdx.x == 0) *out = s * scale;
}

}  // namespace hgs

namespace hgs {

// Largest signal speed c_s + |v| over the cells (FP64) and a non-finite flag,
// per workgroup: partial[2 b] = max, partial[2 b + 1] = 1 if any value was not
// finite.  vx, vy, vz nullable (0).  16-byte vectors of all four fields when
// they are all 16-byte aligned (two vectors per field in flight per thread),
// then the scalar tail; max is exact, so the split does not change the result.
__device__ __forceinline__ void speed_acc(double s, double a, double b, double c, double& m, double& bad) {
    const double v = s + sqrt(a * a + b * b + c * c);
    if (!isfinite(v)) bad = 1.0;
    else m = fmax(m, v);
}

template <typename S>
__global__ __launch_bounds__(256) void k_speed_partial(const S* __restrict__ cs, const S* __restrict__ vx,
                                                       const S* __restrict__ vy, const S* __restrict__ vz, int64_t n,
                                                       double* __restrict__ partial) {
    constexpr int N = 16 / sizeof(S);
    typedef S VT __attribute__((ext_vector_type(N)));
    __shared__ double red[4][2];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double m = 0.0, bad = 0.0;
    const uintptr_t mis = (reinterpret_cast<uintptr_t>(cs) | reinterpret_cast<uintptr_t>(vx) |
                           reinterpret_cast<uintptr_t>(vy) | reinterpret_cast<uintptr_t>(vz)) & 15;
    int64_t done = 0;
    if (mis == 0) {
        const int64_t nv = n / N;
        const VT zero = (VT)(S)0;
        const VT* pc = reinterpret_cast<const VT*>(cs);
        const VT* px = reinterpret_cast<const VT*>(vx);
        const VT* py = reinterpret_cast<const VT*>(vy);
        const VT* pz = reinterpret_cast<const VT*>(vz);
        for (int64_t t = t0; t < nv; t += 2 * stride) {
            // the second vector repeats the first past the end: max and the
            // flag are idempotent, and the loads stay unconditional
            const bool two = t + stride < nv;
            VT c[2], x[2], y[2], z[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int64_t q = (u == 0 || two) ? t + u * stride : t;
                c[u] = pc[q];
                x[u] = px ? px[q] : zero;
                y[u] = py ? py[q] : zero;
                z[u] = pz ? pz[q] : zero;
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int e = 0; e < N; ++e)
                    speed_acc((double)c[u][e], (double)x[u][e], (double)y[u][e], (double)z[u][e], m, bad);
        }
        done = nv * N;
    }
    for (int64_t t = done + t0; t < n; t += stride)
        speed_acc((double)cs[t], vx ? (double)vx[t] : 0.0, vy ? (double)vy[t] : 0.0, vz ? (double)vz[t] : 0.0,
                     m, bad);
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

// out[0] = max of the partial maxima, out[1] = the non-finite flag.  One
// workgroup of 256: thread t takes partials t, t + 256, ..., then the block.
__global__ __launch_bounds__(256) void k_speed_final(const double* __restrict__ partial, int nb,
                                                     double* __restrict__ out) {
    __shared__ double red[4][2];
    double m = 0.0, bad = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        m = fmax(m, partial[2 * i]);
        bad = fmax(bad, partial[2 * i + 1]);
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
    if (threadIdx.x < 2) out[threadIdx.x] = fmax(fmax(red[0][threadIdx.x], red[1][threadIdx.x]),
                                                 fmax(red[2][threadIdx.x], red[3][threadIdx.x]));
}

// sum over interior cells of rho * phi (phi in the padded layout), FP64
// partials per workgroup; the caller scales by dx^3 / 2 for W.  Each wave
// walks whole rows (rows w, w + 4 G, ... of workgroup b with G workgroups).
template <typename S>
__global__ __launch_bounds__(256) void k_dot_partial(const S* __restrict__ rho, const S* __restrict__ phi, Layout L,
                                                     double* __restrict__ partial) {
    __shared__ double red[4];
    double acc = 0.0;
    const int64_t rows = (int64_t)L.ny * L.nz;
    const int lane = threadIdx.x & 63;
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < rows; r += (int64_t)gridDim.x * 4) {
        const int j = (int)(r % L.ny), k = (int)(r / L.ny);
        const S* pr = rho + r * L.nx;
        const S* pp = phi + L.idx(0, j, k);
        for (int i = lane; i < L.nx; i += 64) acc += (double)pr[i] * (double)pp[i];
    }
    const double s = block_sum_256(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

}  // namespace hgs

namespace hgs {

// Extended gravity-only grid (Sec. 4: solve the wave equation on a grid wider
// than the hydrodynamics region, the extension taken as vacuum).  Compact
// fields: inner (nz, ny, nx) <-> outer (nz + 2e, ny + 2e, nx + 2e).
// k_embed writes every outer cell (inner values in the centre, 0 around).
// Both kernels give each wave one row (workgroups of 64 x 4 rows, grid
// (rows / 4, planes)), so no per-element index division is needed.
template <typename S>
__global__ __launch_bounds__(256) void k_embed(const S* __restrict__ inner, int nx, int ny, int nz, int e,
                                               S* __restrict__ outer) {
    const int ox = nx + 2 * e, oy = ny + 2 * e;
    const int j = blockIdx.x * 4 + threadIdx.y;
    const int k = blockIdx.y;
    if (j >= oy) return;
    S* dst = outer + ((int64_t)k * oy + j) * ox;
    const int jj = j - e, kk = k - e;
    if (jj < 0 || jj >= ny || kk < 0 || kk >= nz) {
        for (int i = threadIdx.x; i < ox; i += 64) dst[i] = (S)0;
        return;
    }
    const S* src = inner + ((int64_t)kk * ny + jj) * nx;
    for (int i = threadIdx.x; i < ox; i += 64) dst[i] = (i >= e && i < e + nx) ? src[i - e] : (S)0;
}

template <typename S>
__global__ __launch_bounds__(256) void k_extract(const S* __restrict__ outer, int nx, int ny, int nz, int e,
                                                 S* __restrict__ inner) {
    const int ox = nx + 2 * e, oy = ny + 2 * e;
    const int j = blockIdx.x * 4 + threadIdx.y;
    const int k = blockIdx.y;
    if (j >= ny) return;
    const S* src = outer + ((int64_t)(k + e) * oy + (j + e)) * ox + e;
    S* dst = inner + ((int64_t)k * ny + j) * nx;
    for (int i = threadIdx.x; i < nx; i += 64) dst[i] = src[i];
}

}  // namespace hgs
