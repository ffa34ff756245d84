// Leapfrog substep of Eq. (2) (streaming form, one substep per launch) and the
// central-difference gradient g = -grad phi.
//
// Streaming kernel: a workgroup owns a BX x BY tile of (x, y) columns and
// marches up a chunk of ZC planes.  Each thread keeps phi at z-1, z, z+1 of its
// column in registers, so per cell it issues one new load of phi (z+1), the
// four in-plane neighbours (L1/L2 hits: they are its neighbours' centres), one
// load of phi^{n-1} and of rho, and one store.  The update is in place: the new
// level overwrites phi^{n-1} at the same cell, which no other thread reads.
#pragma once

#include "common.hpp"

namespace hgs {

template <typename S, int BX, int BY>
__global__ __launch_bounds__(BX* BY) void k_leapfrog_stream(const S* __restrict__ cur, S* __restrict__ old_new,
                                                            const S* __restrict__ rho, Layout L, StepCoef c,
                                                            int zc, int tiles_x, int tiles_y) {
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = bid % tiles_x;
    const int ty = (bid / tiles_x) % tiles_y;
    const int tz = bid / (tiles_x * tiles_y);
    const int i = tx * BX + threadIdx.x;
    const int j = ty * BY + threadIdx.y;
    if (i >= L.nx || j >= L.ny) return;  // no barriers below
    const int k0 = tz * zc;
    const int k1 = min(k0 + zc, L.nz);
    const int64_t plane = L.plane;
    const int pitch = L.pitch;
    const int64_t o0 = L.idx(i, j, k0);
    const S* pc = cur + o0;
    S* po = old_new + o0;
    const int64_t sxy = (int64_t)L.nx * L.ny;
    const S* pr = rho + (int64_t)k0 * sxy + (int64_t)j * L.nx + i;
    double zm = ld(pc - plane);
    double z0 = ld(pc);
    for (int k = k0; k < k1; ++k) {
        const double zp = ld(pc + plane);
        const double xm = ld(pc - 1), xp = ld(pc + 1);
        const double ym = ld(pc - pitch), yp = ld(pc + pitch);
        const double o = ld(po);
        const double r = ld(pr);
        *po = (S)leapfrog_update(c, z0, xm, xp, ym, yp, zm, zp, o, r);
        zm = z0;
        z0 = zp;
        pc += plane;
        po += plane;
        pr += sxy;
    }
}

// g = -grad phi, second-order central differences, ghosts at the faces.
template <typename S, int BX, int BY>
__global__ __launch_bounds__(BX* BY) void k_gradient(const S* __restrict__ phi, Layout L, double half_inv_dx, int zc,
                                                     int tiles_x, int tiles_y, S* __restrict__ gx,
                                                     S* __restrict__ gy, S* __restrict__ gz) {
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = bid % tiles_x;
    const int ty = (bid / tiles_x) % tiles_y;
    const int tz = bid / (tiles_x * tiles_y);
    const int i = tx * BX + threadIdx.x;
    const int j = ty * BY + threadIdx.y;
    if (i >= L.nx || j >= L.ny) return;
    const int k0 = tz * zc;
    const int k1 = min(k0 + zc, L.nz);
    const int64_t plane = L.plane;
    const int pitch = L.pitch;
    const S* pc = phi + L.idx(i, j, k0);
    const int64_t sxy = (int64_t)L.nx * L.ny;
    const int64_t c0 = (int64_t)k0 * sxy + (int64_t)j * L.nx + i;
    S* ox = gx + c0;
    S* oy = gy + c0;
    S* oz = gz + c0;
    double zm = ld(pc - plane);
    double z0 = ld(pc);
    for (int k = k0; k < k1; ++k) {
        const double zp = ld(pc + plane);
        const double xm = ld(pc - 1), xp = ld(pc + 1);
        const double ym = ld(pc - pitch), yp = ld(pc + pitch);
        *ox = (S)(-(xp - xm) * half_inv_dx);
        *oy = (S)(-(yp - ym) * half_inv_dx);
        *oz = (S)(-(zp - zm) * half_inv_dx);
        zm = z0;
        z0 = zp;
        pc += plane;
        ox += sxy;
        oy += sxy;
        oz += sxy;
    }
}

}  // namespace hgs
