// Direct solve of the discrete Dirichlet Poisson problem, the steady state of
// every damped run of the wave equation (Eq. 1 with the 7-point Laplacian;
// the runs of the paper start from a Poisson solution, Sec. 2).
//
// With the ghosts moved to the right-hand side the interior system is
//   (D_x + D_y + D_z) phi / dx^2 = b,   b = 4 pi G rho - (adjacent ghosts) / dx^2,
// each D the 1D second difference with zero Dirichlet ends.  D has the
// eigenvectors sin(pi k (i+1) / (n+1)) and eigenvalues
// -4 sin^2(pi k / (2 (n+1))), k = 1..n, so the type-I sine transform along
// each axis diagonalises the system: transform b along x, y, z, divide by the
// summed eigenvalues, transform back (the transform is its own inverse up to
// the factor 2 / (n+1)).  FP64 throughout; each transform is a dense product
// along one axis (n multiply-adds per output), which suits the small grids
// the warm start needs.
#pragma once

#include "common.hpp"

namespace hgs {

// b over the interior (compact (nz, ny, nx), FP64) from rho and the ghosts held
// in the padded state buffer P
template <typename S>
__global__ __launch_bounds__(256) void k_dst_rhs(const S* __restrict__ rho, const S* __restrict__ P, Layout L,
                                                 double fourpiG, double inv_dx2, double* __restrict__ b) {
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        split3(c, L.nx, L.ny, L.nz, i, j, k);
        double gs = 0.0;
        if (i == 0) gs += (double)P[L.idx(-1, j, k)];
        if (i == L.nx - 1) gs += (double)P[L.idx(L.nx, j, k)];
        if (j == 0) gs += (double)P[L.idx(i, -1, k)];
        if (j == L.ny - 1) gs += (double)P[L.idx(i, L.ny, k)];
        if (k == 0) gs += (double)P[L.idx(i, j, -1)];
        if (k == L.nz - 1) gs += (double)P[L.idx(i, j, L.nz)];
        b[c] = fourpiG * (double)rho[c] - gs * inv_dx2;
    }
}

// out = S in along one axis (0 = x, 1 = y, 2 = z) of a compact (nz, ny, nx)
// FP64 array: out[.., m, ..] = sum_j sin(pi (j+1)(m+1) / (n+1)) in[.., j, ..].
// The sine of an integer multiple q of pi / (n+1) depends on q mod 2(n+1)
// only, so one table of 2(n+1) values in LDS serves every product.
constexpr int DST_MAXN = 1024;
__global__ __launch_bounds__(256) void k_dst_axis(const double* __restrict__ in, double* __restrict__ out, int nx,
                                                  int ny, int nz, int axis) {
    __shared__ double tab[2 * (DST_MAXN + 1)];
    const int n = axis == 0 ? nx : (axis == 1 ? ny : nz);
    const int per = 2 * (n + 1);
    for (int q = threadIdx.x; q < per; q += blockDim.x) tab[q] = sinpi((double)q / (double)(n + 1));
    __syncthreads();
    const int64_t stride = axis == 0 ? 1 : (axis == 1 ? (int64_t)nx : (int64_t)nx * ny);
    const int64_t total = (int64_t)nx * ny * nz;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < total; c += (int64_t)gridDim.x * blockDim.x) {
        int64_t line;  // coordinate m of c along the axis
        divmod(divmod(c, stride, line), n, line);
        const int m1 = (int)line + 1;
        const double* src = in + (c - line * stride);  // the line's first element
        double acc = 0.0;
        int q = 0;  // (j + 1) (m + 1) mod 2(n + 1), advanced by m + 1 per j
        for (int j = 0; j < n; ++j) {
            q += m1;
            if (q >= per) q -= per;
            acc = fma(tab[q], src[j * stride], acc);
        }
        out[c] = acc;
    }
}

// divide by the summed eigenvalues and apply the inverse normalisation
__global__ __launch_bounds__(256) void k_dst_scale(double* __restrict__ a, int nx, int ny, int nz, double inv_dx2,
                                                   double norm) {
    const int64_t total = (int64_t)nx * ny * nz;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < total; c += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        split3(c, nx, ny, nz, i, j, k);
        const double sx = sinpi((double)(i + 1) / (2.0 * (nx + 1)));
        const double sy = sinpi((double)(j + 1) / (2.0 * (ny + 1)));
        const double sz = sinpi((double)(k + 1) / (2.0 * (nz + 1)));
        const double lam = -4.0 * inv_dx2 * ((sx * sx + sy * sy) + sz * sz);
        a[c] = a[c] / lam * norm;
    }
}

// phi^n = phi^{n-1} = the solution (interior of two padded state buffers)
template <typename S>
__global__ __launch_bounds__(256) void k_dst_store(const double* __restrict__ a, Layout L, S* __restrict__ p0,
                                                   S* __restrict__ p1) {
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        split3(c, L.nx, L.ny, L.nz, i, j, k);
        const S v = (S)a[c];
        const int64_t o = L.idx(i, j, k);
        p0[o] = v;
        p1[o] = v;
    }
}

}  // namespace hgs
