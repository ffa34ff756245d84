// Nested coarse outer level.  Sec. 4 names nested grids as a way to put the
// outer boundary far from the matter at little cost; the scheme is this
// library's reading: a coarse grid of cell size 2 dx covers the fine grid and
// ext coarse cells more on every side, with a local boundary at its own faces.
// Per hydrodynamical step its source is the density averaged over 2 x 2 x 2
// fine cells (zero in the extension), and after its substeps the fine grid's
// Dirichlet ghosts are its potential interpolated trilinearly at the fine
// ghost centres, frozen over the fine substeps.
#pragma once

#include "common.hpp"

namespace hgs {

// Coarse source: out (nz/2 + 2e, ny/2 + 2e, nx/2 + 2e) = the 2 x 2 x 2 means of
// rho (nz, ny, nx) in the centre, 0 around; every coarse cell is written.
// One wave per coarse row: workgroups of 64 x 4 rows, grid (rows / 4, planes).
template <typename S>
__global__ __launch_bounds__(256) void k_nest_source(const S* __restrict__ rho, int nx, int ny, int nz, int e,
                                                     S* __restrict__ out) {
    const int hx = nx / 2, hy = ny / 2, hz = nz / 2;
    const int mx = hx + 2 * e, my = hy + 2 * e;
    const int j = blockIdx.x * 4 + threadIdx.y, k = blockIdx.y;
    if (j >= my) return;
    S* dst = out + ((int64_t)k * my + j) * mx;
    const int jj = j - e, kk = k - e;
    const bool row_in = jj >= 0 && jj < hy && kk >= 0 && kk < hz;
    for (int i = threadIdx.x; i < mx; i += 64) {
        const int ii = i - e;
        double s = 0.0;
        if (row_in && ii >= 0 && ii < hx) {
            for (int dz = 0; dz < 2; ++dz)
                for (int dy = 0; dy < 2; ++dy) {
                    const S* p = rho + ((int64_t)(2 * kk + dz) * ny + (2 * jj + dy)) * nx + 2 * ii;
                    s += (double)p[0];
                    s += (double)p[1];
                }
        }
        dst[i] = (S)(0.125 * s);
    }
}

struct NestGeom {
    int mx, my, mz;          // coarse interior cells
    double cx0, cy0, cz0;    // coarse lower corner
    double cdx;              // coarse cell size
    int nx, ny, nz;          // fine interior cells
    double fx0, fy0, fz0;    // fine lower corner
    double fdx;              // fine cell size
};

// Position along one axis -> lower coarse centre index and weight of the upper
// one (u = (p - lo) / dx - 1/2, i = floor(u) kept in [0, n - 2], w = u - i).
__device__ __forceinline__ void nest_axis(double p, double lo, double dx, int n, int& i, double& w) {
    const double u = (p - lo) / dx - 0.5;
    i = min(max((int)floor(u), 0), n - 2);
    w = u - (double)i;
}

// Fine ghost faces in the layout of hgs_set_boundary (x-, x+, y-, y+, z-, z+;
// x faces (nz, ny), y faces (nz, nx), z faces (ny, nx), each in C order) from
// the coarse compact potential, by trilinear interpolation at the ghost
// centres (FP64).  One thread per ghost; grid
// (ceil(max(nx, ny) / 256), max(ny, nz), 6); the host checks that every
// ghost centre lies within the span of the coarse centres.
template <typename S>
__global__ __launch_bounds__(256) void k_nest_ghosts(const S* __restrict__ phi, NestGeom g, S* __restrict__ faces) {
    const int f = blockIdx.z, axis = f >> 1, hi = f & 1;
    const int a = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
    const int na = axis == 0 ? g.ny : g.nx, nb = axis == 2 ? g.ny : g.nz;
    if (a >= na || b >= nb) return;
    const int64_t sx = (int64_t)g.nz * g.ny, sy = (int64_t)g.nz * g.nx;
    const int64_t base = axis == 0 ? hi * sx : axis == 1 ? 2 * sx + hi * sy : 2 * sx + 2 * sy + hi * ((int64_t)g.ny * g.nx);
    const int gi = axis == 0 ? (hi ? g.nx : -1) : a;
    const int gj = axis == 0 ? a : axis == 1 ? (hi ? g.ny : -1) : b;
    const int gk = axis == 2 ? (hi ? g.nz : -1) : b;
    int ix, iy, iz;
    double wx, wy, wz;
    nest_axis(g.fx0 + (gi + 0.5) * g.fdx, g.cx0, g.cdx, g.mx, ix, wx);
    nest_axis(g.fy0 + (gj + 0.5) * g.fdx, g.cy0, g.cdx, g.my, iy, wy);
    nest_axis(g.fz0 + (gk + 0.5) * g.fdx, g.cz0, g.cdx, g.mz, iz, wz);
    double v = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const double w = (dz ? wz : 1.0 - wz) * (dy ? wy : 1.0 - wy) * (dx ? wx : 1.0 - wx);
                v += w * (double)phi[((int64_t)(iz + dz) * g.my + (iy + dy)) * g.mx + (ix + dx)];
            }
    faces[base + (int64_t)b * na + a] = (S)v;
}

}  // namespace hgs
