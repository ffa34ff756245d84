// Shared device-side definitions of the hyperbolic self-gravity library.
//
// Padded field layout in HBM (one per state buffer):
//   x: interior cell i at element xoff + i of a row; xoff is 128 bytes worth of
//      elements so every interior row starts on a 128-byte line; the row pitch
//      is a multiple of 128 bytes with room for a 16-byte vector at x = nx;
//   y: one row below and above the interior;  z: one plane below and above.
// Ghost cells (the Dirichlet boundary) are that layer adjacent to each face;
// edges, corners and the rest of each row are padding that no update reads.
// Padding is filled with NaN at init so that an erroneous read poisons the
// result instead of passing silently.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hgs.h"

namespace hgs {

constexpr int HALO = 1;  // ghost rows/planes around the interior
constexpr int NQ = (HGS_LMAX + 1) * (HGS_LMAX + 1);  // 25 multipole coefficients

struct Layout {
    int nx, ny, nz;
    int xoff;       // element index of interior x = 0 within a row
    int pitch;      // elements per row
    int rows;       // ny + 2*HALO
    int64_t plane;  // pitch * rows
    int64_t total;  // plane * (nz + 2*HALO)

    __host__ __device__ int64_t idx(int i, int j, int k) const {
        return ((int64_t)(k + HALO) * rows + (j + HALO)) * pitch + (i + xoff);
    }
};

inline Layout make_layout(int nx, int ny, int nz, int elem_bytes) {
    Layout L;
    L.nx = nx;
    L.ny = ny;
    L.nz = nz;
    const int line = 128 / elem_bytes;
    L.xoff = line;
    // the ghost cell plus room for one 16-byte vector starting at x = nx
    int need = L.xoff + nx + 4;
    L.pitch = (need + line - 1) / line * line;
    L.rows = ny + 2 * HALO;
    L.plane = (int64_t)L.pitch * L.rows;
    L.total = L.plane * (nz + 2 * HALO);
    return L;
}

// Coefficients of one leapfrog substep, all FP64:
//   phi^{n+1} = c0 phi + c1 (sum of the six neighbours) + cm phi^{n-1} + cs rho
// with kk = c^2 dt^2 / dx^2, a = eta dt / 2:
//   c0 = (2 - 6 kk) / (1 + a), c1 = kk / (1 + a), cm = -(1 - a) / (1 + a),
//   cs = -c^2 dt^2 4 pi G / (1 + a).
//
// For FP32 storage the same update is evaluated in FP32 in increment form,
//   phi^{n+1} = phi + [(1 - a)(phi - phi^{n-1}) + kk sum_6 (nb - phi)
//                      - c^2 dt^2 4 pi G rho] / (1 + a),
// with fo = (1 - a)/(1 + a), fl = kk/(1 + a), fs = cs rounded to FP32.  The
// differences nb - phi and phi - phi^{n-1} of nearby FP32 values are exact
// (Sterbenz), so rounding acts on the small increment only and the stored
// state stays as close to the FP64 solution as with FP64 arithmetic (checked
// against FP64 runs at converged 64^3 and 128^3 states); evaluating
// c0 phi + c1 sum nb directly in FP32 instead cancels and biases the fixed
// point by a term growing as 1/dx^2.  The FP32 form needs no conversions and
// half the registers, which the fused kernel turns into deeper prefetch and
// taller tiles.
struct StepCoef {
    double c0, c1, cm, cs;
    float fo, fl, fs;
};

// The one place the update is written.  The summation order and the explicit
// fused multiply-adds are fixed so that every kernel variant (streaming,
// temporally blocked, batched) produces bit-identical results.
__device__ __forceinline__ double leapfrog_update(const StepCoef& c, double p, double xm, double xp, double ym,
                                                  double yp, double zm, double zp, double old, double rho) {
    double nb = ((xm + xp) + (ym + yp)) + (zm + zp);
    return fma(c.cs, rho, fma(c.cm, old, fma(c.c1, nb, c.c0 * p)));
}

// The update in the storage type: FP64 storage takes the FP64 form above,
// FP32 storage the FP32 increment form.  Every kernel variant calls these, so
// streaming, fused and batched launches stay bit-identical.
__device__ __forceinline__ double update(const StepCoef& c, double p, double xm, double xp, double ym, double yp,
                                         double zm, double zp, double old, double rho) {
    return leapfrog_update(c, p, xm, xp, ym, yp, zm, zp, old, rho);
}
__device__ __forceinline__ float update(const StepCoef& c, float p, float xm, float xp, float ym, float yp, float zm,
                                        float zp, float old, float rho) {
    const float d = (((xm - p) + (xp - p)) + ((ym - p) + (yp - p))) + ((zm - p) + (zp - p));
    const float inc = fmaf(c.fs, rho, fmaf(c.fl, d, c.fo * (p - old)));
    return p + inc;
}

// rho minus a subtracted mean (periodic boundary) in the storage type; rb = 0
// leaves rho unchanged
__device__ __forceinline__ double source(double r, double rb) { return r - rb; }
__device__ __forceinline__ float source(float r, double rb) { return r - (float)rb; }

template <typename S>
__device__ __forceinline__ double ld(const S* p) {
    return (double)(*p);
}

// Cell-centre positions relative to the expansion centre, for the outer
// boundaries whose ghosts follow the interior (Robin, outgoing).
struct LocalGeom {
    double x0, y0, z0, dx, ox, oy, oz;
};

// Coordinate of cell index i along one axis (lo = that axis's grid corner,
// o = the centre's coordinate), rounded to the storage type.
template <typename S>
__device__ __forceinline__ S local_coord(double lo, double o, double dx, int i) {
    return (S)(lo + ((double)i + 0.5) * dx - o);
}

// |x|^2 in the storage type, in one fixed order of operations.
template <typename S>
__device__ __forceinline__ S local_r2(S x, S y, S z) {
    return fma(x, x, fma(y, y, z * z));
}

// Robin ghost (Sec. 2, Sec. 4: a monopole far field, r phi equal at the ghost
// and its interior neighbour) from the neighbour's value v:
// v |x_i| / |x_g| in the storage type: FP64 as v sqrt(|x_i|^2 / |x_g|^2) with
// the correctly rounded divide and square root; FP32 as
// v |x_i|^2 / sqrt(|x_i|^2 |x_g|^2) with the hardware reciprocal square root
// (a few ulp, far below the FP32 storage rounding of the state, and one
// transcendental where the fused launch evaluates it per face cell and level).  Every kernel that sets
// or reads a Robin ghost calls this with the same operands, so streamed and
// fused substeps agree bit for bit.
__device__ __forceinline__ double robin_ratio(double ri2, double rg2) { return sqrt(ri2 / rg2); }
__device__ __forceinline__ float robin_ratio(float ri2, float rg2) {
    // |x_i| / |x_g| = |x_i|^2 / sqrt(|x_i|^2 |x_g|^2): one transcendental
    return ri2 * __builtin_amdgcn_rsqf(ri2 * rg2);
}
template <typename S>
__device__ __forceinline__ S robin_ghost(S ri2, S rg2, S v) {
    return v * robin_ratio(ri2, rg2);
}

// Coordinate of a face plane (cell index i, the plane at the cell's lower
// side) along one axis, rounded to the storage type.
template <typename S>
__device__ __forceinline__ S local_face(double lo, double o, double dx, int i) {
    return (S)(lo + (double)i * dx - o);
}

// Outgoing ghost (Sec. 4: the radiative form of the Robin condition,
// d(r phi)/dt + c d(r phi)/dr = 0 with d/dr = d/dn / cos(theta) at the
// midpoint x_f of ghost and neighbour, box scheme at t^{n+1/2}):
//   g1 = a (g0 - b i1) + b i0,  a = (1 - al) / (1 + al),  b = r_i / r_g,
//   al = (c dt / dx) |x_f| / s,  s = the face-normal component of x_f,
// from the ghost's previous value g0 and the interior neighbour's previous
// and new values i0, i1 (the form u_g' = [(1 - al) u_g + (1 + al) u_i -
// (1 - al) u_i'] / (1 + al) with u = r phi, divided by r_g).  In the storage
// type: FP64 with correctly rounded divides and square roots, FP32 with the
// hardware reciprocal and reciprocal square root.  One function for the
// streaming and the fused substeps, so both give the same bits.
__device__ __forceinline__ double outgoing_ghost(double ri2, double rg2, double rf2, double s, double kk,
                                                 double g0, double i0, double i1) {
    const double b = sqrt(ri2 / rg2);
    const double al = kk * sqrt(rf2) / s;
    const double a = (1.0 - al) / (1.0 + al);
    return fma(a, fma(-b, i1, g0), b * i0);
}
__device__ __forceinline__ float outgoing_ghost(float ri2, float rg2, float rf2, float s, float kk, float g0,
                                                float i0, float i1) {
    const float b = ri2 * __builtin_amdgcn_rsqf(ri2 * rg2);
    const float al = kk * (rf2 * __builtin_amdgcn_rsqf(rf2)) * __builtin_amdgcn_rcpf(s);
    const float a = (1.0f - al) * __builtin_amdgcn_rcpf(1.0f + al);
    return fmaf(a, fmaf(-b, i1, g0), b * i0);
}

// Workgroups of one launch are handed to the 8 XCDs round-robin.  Renumber
// them so that XCD x runs a contiguous range of tiles: neighbouring tiles then
// share that XCD's L2 for their halos.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
    const int nx = 8;
    int q = nblocks / nx, r = nblocks % nx;
    int xcd = bid % nx, local = bid / nx;
    return (xcd < r) ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// q = a / d, r = a - q d for a >= 0, d > 0: 32-bit unsigned arithmetic while
// both fit (every index of the grids and tensors here; a 64-bit division is a
// long instruction sequence), the 64-bit division otherwise.
__device__ __forceinline__ int64_t divmod(int64_t a, int64_t d, int64_t& r) {
    if (a <= 0xffffffffll && d <= 0xffffffffll) {
        const unsigned q = (unsigned)a / (unsigned)d;
        r = (int64_t)((unsigned)a - q * (unsigned)d);
        return q;
    }
    const int64_t q = a / d;
    r = a - q * d;
    return q;
}

// (i, j, k) of index c of a compact (nz, ny, nx) array, and the sample b when
// c runs over several of them
__device__ __forceinline__ int64_t split3(int64_t c, int nx, int ny, int nz, int& i, int& j, int& k) {
    int64_t r;
    int64_t q = divmod(c, nx, r);
    i = (int)r;
    q = divmod(q, ny, r);
    j = (int)r;
    q = divmod(q, nz, r);
    k = (int)r;
    return q;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace hgs
