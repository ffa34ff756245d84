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

// Outer-boundary forms of the streaming substep:
//   ST_PLAIN     ghosts read from the ghost layer (frozen ghosts, or ghosts a
//                launch after the substep sets);
//   ST_ROBIN     face cells evaluate their Robin ghosts where they read them
//                (robin_beside), so no ghost launch is needed between substeps;
//   ST_OUTGOING  face cells read the old ghost from the ghost layer and store
//                the new level's ghost beside their own new value (the
//                outgoing rule needs nothing else: its old ghost, the cell's
//                old and new values), so no ghost launch follows the substep;
//   ST_PERIODIC  face cells store their new value also into the ghost across
//                the opposite face, whose periodic image they are, so no
//                ghost launch follows the substep.
constexpr int ST_PLAIN = 0, ST_ROBIN = 1, ST_OUTGOING = 2, ST_PERIODIC = 3;

// The new level's outgoing ghost beside a face cell: g0 the old ghost, i0 and
// i1 the cell's old and new values; (x, y, z) the cell, (gx, gy, gz) the
// ghost and (fx, fy, fz) the face point between them, s the face's signed
// normal coordinate: the operands the fused launch uses, the same bits.
template <typename S>
__device__ __forceinline__ S outgoing_beside(S x, S y, S z, S gx, S gy, S gz, S fx, S fy, S fz, S s, S kk, S g0,
                                             S i0, S i1) {
    return outgoing_ghost(local_r2(x, y, z), local_r2(gx, gy, gz), local_r2(fx, fy, fz), s, kk, g0, i0, i1);
}

// The Robin ghost beside a face cell, evaluated where it is read: the rule's
// value from the cell's own value v, with the ghost at the cell's position
// moved past the face, (gx, gy, gz).  These are the operands the ghost launch
// uses, so the result equals the stored ghost bit for bit, and a substep that
// evaluates its Robin ghosts this way needs no ghost launch before it.
template <typename S>
__device__ __forceinline__ S robin_beside(S x, S y, S z, S gx, S gy, S gz, S v) {
    return robin_ghost(local_r2(x, y, z), local_r2(gx, gy, gz), v);
}

// rbar (nullable, device): density subtracted from rho in the source, the
// domain mean on a periodic grid; rho - 0 = rho exactly, so results without it
// are bit-identical to the fused kernels.  BND: ST_PLAIN, ST_ROBIN or
// ST_OUTGOING (above; lg: cell positions, c_dt = c_g dt).
template <typename S, int BX, int BY, int BND = ST_PLAIN>
__global__ __launch_bounds__(BX* BY) void k_leapfrog_stream(const S* __restrict__ cur, S* __restrict__ old_new,
                                                            const S* __restrict__ rho, Layout L, StepCoef c,
                                                            int zc, int tiles_x, int tiles_y,
                                                            const double* __restrict__ rbar, LocalGeom lg,
                                                            double c_dt) {
    constexpr bool ROBIN = BND == ST_ROBIN;
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
    const double rb = rbar ? *rbar : 0.0;
    S zm = pc[-plane];
    S z0 = pc[0];
    for (int k = k0; k < k1; ++k) {
        const S zp = pc[plane];
        S xm = pc[-1], xp = pc[1];
        S ym = pc[-pitch], yp = pc[pitch];
        S zmu = zm, zpu = zp;
        if (ROBIN && (i == 0 || i == L.nx - 1 || j == 0 || j == L.ny - 1 || k == 0 || k == L.nz - 1)) {
            const S cx = local_coord<S>(lg.x0, lg.ox, lg.dx, i), cy = local_coord<S>(lg.y0, lg.oy, lg.dx, j),
                    cz = local_coord<S>(lg.z0, lg.oz, lg.dx, k);
            if (i == 0) xm = robin_beside(cx, cy, cz, local_coord<S>(lg.x0, lg.ox, lg.dx, -1), cy, cz, z0);
            if (i == L.nx - 1) xp = robin_beside(cx, cy, cz, local_coord<S>(lg.x0, lg.ox, lg.dx, L.nx), cy, cz, z0);
            if (j == 0) ym = robin_beside(cx, cy, cz, cx, local_coord<S>(lg.y0, lg.oy, lg.dx, -1), cz, z0);
            if (j == L.ny - 1) yp = robin_beside(cx, cy, cz, cx, local_coord<S>(lg.y0, lg.oy, lg.dx, L.ny), cz, z0);
            if (k == 0) zmu = robin_beside(cx, cy, cz, cx, cy, local_coord<S>(lg.z0, lg.oz, lg.dx, -1), z0);
            if (k == L.nz - 1) zpu = robin_beside(cx, cy, cz, cx, cy, local_coord<S>(lg.z0, lg.oz, lg.dx, L.nz), z0);
        }
        const S o = *po;
        const S r = source(*pr, rb);
        const S nv = (S)update(c, z0, xm, xp, ym, yp, zmu, zpu, o, r);
        *po = nv;
        if (BND == ST_PERIODIC) {
            if (i == 0) po[L.nx] = nv;  // the ghost x = nx
            if (i == L.nx - 1) po[-L.nx] = nv;  // the ghost x = -1
            if (j == 0) po[(int64_t)L.ny * pitch] = nv;
            if (j == L.ny - 1) po[-(int64_t)L.ny * pitch] = nv;
            if (k == 0) po[(int64_t)L.nz * plane] = nv;
            if (k == L.nz - 1) po[-(int64_t)L.nz * plane] = nv;
        }
        if (BND == ST_OUTGOING && (i == 0 || i == L.nx - 1 || j == 0 || j == L.ny - 1 || k == 0 || k == L.nz - 1)) {
            const S kk = (S)(c_dt / lg.dx);
            const S cx = local_coord<S>(lg.x0, lg.ox, lg.dx, i), cy = local_coord<S>(lg.y0, lg.oy, lg.dx, j),
                    cz = local_coord<S>(lg.z0, lg.oz, lg.dx, k);
            if (i == 0) {
                const S f = local_face<S>(lg.x0, lg.ox, lg.dx, 0);
                po[-1] = outgoing_beside(cx, cy, cz, local_coord<S>(lg.x0, lg.ox, lg.dx, -1), cy, cz, f, cy, cz, -f, kk,
                                         xm, z0, nv);
            }
            if (i == L.nx - 1) {
                const S f = local_face<S>(lg.x0, lg.ox, lg.dx, L.nx);
                po[1] = outgoing_beside(cx, cy, cz, local_coord<S>(lg.x0, lg.ox, lg.dx, L.nx), cy, cz, f, cy, cz, f, kk,
                                        xp, z0, nv);
            }
            if (j == 0) {
                const S f = local_face<S>(lg.y0, lg.oy, lg.dx, 0);
                po[-pitch] = outgoing_beside(cx, cy, cz, cx, local_coord<S>(lg.y0, lg.oy, lg.dx, -1), cz, cx, f, cz, -f,
                                             kk, ym, z0, nv);
            }
            if (j == L.ny - 1) {
                const S f = local_face<S>(lg.y0, lg.oy, lg.dx, L.ny);
                po[pitch] = outgoing_beside(cx, cy, cz, cx, local_coord<S>(lg.y0, lg.oy, lg.dx, L.ny), cz, cx, f, cz, f,
                                            kk, yp, z0, nv);
            }
            if (k == 0) {
                const S f = local_face<S>(lg.z0, lg.oz, lg.dx, 0);
                po[-plane] = outgoing_beside(cx, cy, cz, cx, cy, local_coord<S>(lg.z0, lg.oz, lg.dx, -1), cx, cy, f, -f,
                                             kk, zm, z0, nv);
            }
            if (k == L.nz - 1) {
                const S f = local_face<S>(lg.z0, lg.oz, lg.dx, L.nz);
                po[plane] = outgoing_beside(cx, cy, cz, cx, cy, local_coord<S>(lg.z0, lg.oz, lg.dx, L.nz), cx, cy, f, f,
                                            kk, zp, z0, nv);
            }
        }
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

// ---------------------------------------------------------------------------
// Vectorised forms (16 bytes per lane: 4 FP32 or 2 FP64 cells along x), used
// when nx is a multiple of the vector width.  A wave covers 64*N consecutive x
// cells of one row; x neighbours across lanes come from a DPP wave shift, and
// only the first and last lane of a wave read their outer neighbour from
// memory.  The arithmetic and its order are those of the scalar kernels, so
// results are bit-identical.
namespace hgs {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename S>
struct Vec16;
template <>
struct Vec16<float> {
    using T = f32x4;
    static constexpr int N = 4;
    __device__ static float get(const T& v, int i) { return v[i]; }
    __device__ static void set(T& v, int i, float s) { v[i] = s; }
};
template <>
struct Vec16<double> {
    using T = f64x2;
    static constexpr int N = 2;
    __device__ static double get(const T& v, int i) { return v[i]; }
    __device__ static void set(T& v, int i, double s) { v[i] = s; }
};

// value of lane l-1 (from_prev) or l+1 (from_next); edge lanes get 0
__device__ __forceinline__ float from_prev(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_next(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double from_prev(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_next(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

// Per-lane geometry of a vectorised sweep: lanes past the interior load a
// clamped (valid) vector and store nothing.
struct VLane {
    int i0;      // first x cell of the lane
    int j;       // row
    int xl, jl;  // clamped load coordinates (padded layout)
    int xr, jr;  // clamped coordinates in a compact array
    bool active;
};

template <int N>
__device__ __forceinline__ VLane vlane(const Layout& L, int tx, int ty, int BY) {
    VLane v;
    const int lane = threadIdx.x;
    v.i0 = (tx * 64 + lane) * N;
    v.j = ty * BY + (int)threadIdx.y;
    v.active = v.i0 < L.nx && v.j < L.ny;
    v.xl = min(v.i0, L.nx);  // [nx, nx+N) lies inside the row padding
    v.jl = min(v.j, L.ny);
    v.xr = min(v.i0, L.nx - N);
    v.jr = min(v.j, L.ny - 1);
    return v;
}

// ST_OUTGOING ghosts of a vectorised lane at the faces it touches: the x
// ghost beside its first / last cell (old ghost: the lane's left / right
// neighbour, loaded from the ghost layer), the y ghost row beside a face row
// and the z ghost plane beside a face plane (old ghosts: the loaded ym, yp,
// zm, zp vectors); new values stored into the new level's ghost layer.
template <typename S>
__device__ __forceinline__ void stream_v_outgoing(const Layout& L, const LocalGeom& lg, double c_dt, const VLane& g,
                                               int k, S* po, int pitch, int64_t plane, const typename Vec16<S>::T& z0,
                                               const typename Vec16<S>::T& out, S left, S right,
                                               const typename Vec16<S>::T& ym, const typename Vec16<S>::T& yp,
                                               const typename Vec16<S>::T& zm, const typename Vec16<S>::T& zp) {
    using V = Vec16<S>;
    using VT = typename V::T;
    constexpr int N = V::N;
    const S kk = (S)(c_dt / lg.dx);
    const S cy = local_coord<S>(lg.y0, lg.oy, lg.dx, g.j), cz = local_coord<S>(lg.z0, lg.oz, lg.dx, k);
    if (g.i0 == 0) {
        const S cx = local_coord<S>(lg.x0, lg.ox, lg.dx, 0), f = local_face<S>(lg.x0, lg.ox, lg.dx, 0);
        po[-1] = outgoing_beside(cx, cy, cz, local_coord<S>(lg.x0, lg.ox, lg.dx, -1), cy, cz, f, cy, cz, -f, kk, left,
                                 (S)V::get(z0, 0), (S)V::get(out, 0));
    }
    if (g.i0 + N == L.nx) {
        const S cx = local_coord<S>(lg.x0, lg.ox, lg.dx, L.nx - 1), f = local_face<S>(lg.x0, lg.ox, lg.dx, L.nx);
        po[N] = outgoing_beside(cx, cy, cz, local_coord<S>(lg.x0, lg.ox, lg.dx, L.nx), cy, cz, f, cy, cz, f, kk, right,
                                (S)V::get(z0, N - 1), (S)V::get(out, N - 1));
    }
    // y and z ghost rows / planes: one vector per face
    for (int face = 0; face < 4; ++face) {
        const bool on = face == 0 ? g.j == 0 : face == 1 ? g.j == L.ny - 1 : face == 2 ? k == 0 : k == L.nz - 1;
        if (!on) continue;
        const bool hi = face & 1;
        const VT& gold = face == 0 ? ym : face == 1 ? yp : face == 2 ? zm : zp;
        S gc, fc;  // ghost and face coordinate along the normal
        if (face < 2) {
            gc = local_coord<S>(lg.y0, lg.oy, lg.dx, hi ? L.ny : -1);
            fc = local_face<S>(lg.y0, lg.oy, lg.dx, hi ? L.ny : 0);
        } else {
            gc = local_coord<S>(lg.z0, lg.oz, lg.dx, hi ? L.nz : -1);
            fc = local_face<S>(lg.z0, lg.oz, lg.dx, hi ? L.nz : 0);
        }
        VT gnew;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const S cx = local_coord<S>(lg.x0, lg.ox, lg.dx, g.i0 + n);
            const S v = face < 2 ? outgoing_beside(cx, cy, cz, cx, gc, cz, cx, fc, cz, hi ? fc : -fc, kk,
                                                   (S)V::get(gold, n), (S)V::get(z0, n), (S)V::get(out, n))
                                 : outgoing_beside(cx, cy, cz, cx, cy, gc, cx, cy, fc, hi ? fc : -fc, kk,
                                                   (S)V::get(gold, n), (S)V::get(z0, n), (S)V::get(out, n));
            V::set(gnew, n, v);
        }
        const int64_t off = face == 0 ? -(int64_t)pitch : face == 1 ? (int64_t)pitch : face == 2 ? -plane : plane;
        *reinterpret_cast<VT*>(po + off) = gnew;
    }
}

// One (64N x BY) column tile, planes [k0, k1): the body shared by the
// single-grid and the batched launches.  BND as in k_leapfrog_stream.
template <typename S, int BY, int BND = ST_PLAIN>
__device__ __forceinline__ void stream_v_tile(const S* __restrict__ cur, S* __restrict__ old_new,
                                              const S* __restrict__ rho, const Layout& L, const StepCoef& c, int tx,
                                              int ty, int k0, int k1, double rb, const LocalGeom& lg = LocalGeom{},
                                              double c_dt = 0.0) {
    constexpr bool ROBIN = BND == ST_ROBIN;
    using V = Vec16<S>;
    using VT = typename V::T;
    constexpr int N = V::N;
    const VLane g = vlane<N>(L, tx, ty, BY);
    const int lane = threadIdx.x;
    const int64_t plane = L.plane;
    const int pitch = L.pitch;
    const int64_t o0 = L.idx(g.xl, g.jl, k0);
    const S* pc = cur + o0;
    S* po = old_new + o0;
    const int64_t sxy = (int64_t)L.nx * L.ny;
    const S* pr = rho + (int64_t)k0 * sxy + (int64_t)g.jr * L.nx + g.xr;
    VT zm = *reinterpret_cast<const VT*>(pc - plane);
    VT z0 = *reinterpret_cast<const VT*>(pc);
    for (int k = k0; k < k1; ++k) {
        const VT zp = *reinterpret_cast<const VT*>(pc + plane);
        const VT ym = *reinterpret_cast<const VT*>(pc - pitch);
        const VT yp = *reinterpret_cast<const VT*>(pc + pitch);
        const VT o = *reinterpret_cast<const VT*>(po);
        const VT r = *reinterpret_cast<const VT*>(pr);
        S left = from_prev(V::get(z0, N - 1));
        S right = from_next(V::get(z0, 0));
        if (lane == 0) left = pc[-1];
        if (lane == 63) right = pc[N];
        // ROBIN: the row (y) and the plane (z) are the same for the whole wave
        const bool yzface = ROBIN && (g.j == 0 || g.j == L.ny - 1 || k == 0 || k == L.nz - 1);
        S cy = (S)0, cz = (S)0;
        if (ROBIN) {
            cy = local_coord<S>(lg.y0, lg.oy, lg.dx, g.j);
            cz = local_coord<S>(lg.z0, lg.oz, lg.dx, k);
            if (g.i0 == 0)
                left = robin_beside(local_coord<S>(lg.x0, lg.ox, lg.dx, 0), cy, cz,
                                    local_coord<S>(lg.x0, lg.ox, lg.dx, -1), cy, cz, (S)V::get(z0, 0));
            if (g.i0 + N == L.nx)
                right = robin_beside(local_coord<S>(lg.x0, lg.ox, lg.dx, L.nx - 1), cy, cz,
                                     local_coord<S>(lg.x0, lg.ox, lg.dx, L.nx), cy, cz, (S)V::get(z0, N - 1));
        }
        VT out;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const S xm = n > 0 ? (S)V::get(z0, n - 1) : left;
            const S xp = n < N - 1 ? (S)V::get(z0, n + 1) : right;
            S ymn = (S)V::get(ym, n), ypn = (S)V::get(yp, n), zmn = (S)V::get(zm, n), zpn = (S)V::get(zp, n);
            if (yzface) {
                const S cx = local_coord<S>(lg.x0, lg.ox, lg.dx, g.i0 + n), ce = (S)V::get(z0, n);
                if (g.j == 0) ymn = robin_beside(cx, cy, cz, cx, local_coord<S>(lg.y0, lg.oy, lg.dx, -1), cz, ce);
                if (g.j == L.ny - 1)
                    ypn = robin_beside(cx, cy, cz, cx, local_coord<S>(lg.y0, lg.oy, lg.dx, L.ny), cz, ce);
                if (k == 0) zmn = robin_beside(cx, cy, cz, cx, cy, local_coord<S>(lg.z0, lg.oz, lg.dx, -1), ce);
                if (k == L.nz - 1)
                    zpn = robin_beside(cx, cy, cz, cx, cy, local_coord<S>(lg.z0, lg.oz, lg.dx, L.nz), ce);
            }
            const S v = (S)update(c, (S)V::get(z0, n), xm, xp, ymn, ypn, zmn, zpn, (S)V::get(o, n),
                                  source((S)V::get(r, n), rb));
            V::set(out, n, v);
        }
        if (g.active) *reinterpret_cast<VT*>(po) = out;
        if (BND == ST_PERIODIC && g.active) {
            // the periodic images: x ghosts from the first / last cell of the
            // row, y ghost rows and z ghost planes from whole vectors
            if (g.i0 == 0) po[L.nx] = (S)V::get(out, 0);
            if (g.i0 + N == L.nx) po[N - 1 - L.nx] = (S)V::get(out, N - 1);
            if (g.j == 0) *reinterpret_cast<VT*>(po + (int64_t)L.ny * pitch) = out;
            if (g.j == L.ny - 1) *reinterpret_cast<VT*>(po - (int64_t)L.ny * pitch) = out;
            if (k == 0) *reinterpret_cast<VT*>(po + (int64_t)L.nz * plane) = out;
            if (k == L.nz - 1) *reinterpret_cast<VT*>(po - (int64_t)L.nz * plane) = out;
        }
        if (BND == ST_OUTGOING && g.active &&
            (g.i0 == 0 || g.i0 + N == L.nx || g.j == 0 || g.j == L.ny - 1 || k == 0 || k == L.nz - 1))
            stream_v_outgoing<S>(L, lg, c_dt, g, k, po, pitch, plane, z0, out, left, right, ym, yp, zm, zp);
        zm = z0;
        z0 = zp;
        pc += plane;
        po += plane;
        pr += sxy;
    }
}

template <typename S, int BY, int BND = ST_PLAIN>
__global__ __launch_bounds__(64 * BY) void k_leapfrog_stream_v(const S* __restrict__ cur, S* __restrict__ old_new,
                                                               const S* __restrict__ rho, Layout L, StepCoef c, int zc,
                                                               int tiles_x, int tiles_y,
                                                               const double* __restrict__ rbar, LocalGeom lg,
                                                               double c_dt) {
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = bid % tiles_x;
    const int ty = (bid / tiles_x) % tiles_y;
    const int tz = bid / (tiles_x * tiles_y);
    const int k0 = tz * zc;
    stream_v_tile<S, BY, BND>(cur, old_new, rho, L, c, tx, ty, k0, min(k0 + zc, L.nz), rbar ? *rbar : 0.0, lg,
                              c_dt);
}

// Central-difference gradient, 16 bytes per lane along x, R rows per thread:
// each thread marches up its z chunk with a three-plane window of its R rows
// in registers, so a row is loaded once per plane (plus the two rows that
// border the thread's rows in y) instead of once for itself and once for
// each y neighbour.  g = -(phi(+1) - phi(-1)) / (2 dx) per axis in FP64,
// rounded to the storage type; outputs are compact, written with streaming
// stores.
template <typename S, int R, int BY>
__global__ __launch_bounds__(64 * BY) void k_gradient_v(const S* __restrict__ phi, Layout L, double half_inv_dx,
                                                        int zc, int tiles_x, int tiles_y, S* __restrict__ gx,
                                                        S* __restrict__ gy, S* __restrict__ gz) {
    using V = Vec16<S>;
    using VT = typename V::T;
    constexpr int N = V::N;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = bid % tiles_x;
    const int ty = (bid / tiles_x) % tiles_y;
    const int tz = bid / (tiles_x * tiles_y);
    const int lane = threadIdx.x;
    const int i0 = (tx * 64 + lane) * N;
    const bool x_act = i0 < L.nx;
    const int xl = min(i0, L.nx);      // [nx, nx+N) lies inside the row padding
    const int xr = min(i0, L.nx - N);  // an in-bounds output column for idle lanes
    const int jb = ty * (BY * R) + (int)threadIdx.y * R;
    const int k0 = tz * zc;
    const int k1 = min(k0 + zc, L.nz);
    const int64_t plane = L.plane;
    const int64_t sxy = (int64_t)L.nx * L.ny;
    // padded offsets of the thread's rows (clamped into the ghost box) and of
    // the rows below and above them; compact output offsets
    int64_t ro[R], co[R];
    bool act[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = jb + r;
        act[r] = x_act && j < L.ny;
        ro[r] = L.idx(xl, min(j, L.ny), k0);
        co[r] = (int64_t)k0 * sxy + (int64_t)min(j, L.ny - 1) * L.nx + xr;
    }
    const int64_t rm = L.idx(xl, min(jb - 1, L.ny), k0);
    const int64_t rp = L.idx(xl, min(jb + R, L.ny), k0);
    VT zm[R], z0[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        zm[r] = *reinterpret_cast<const VT*>(phi + ro[r] - plane);
        z0[r] = *reinterpret_cast<const VT*>(phi + ro[r]);
    }
    int64_t pin = 0, pout = 0;
    for (int k = k0; k < k1; ++k) {
        VT zp[R];
#pragma unroll
        for (int r = 0; r < R; ++r) zp[r] = *reinterpret_cast<const VT*>(phi + ro[r] + pin + plane);
        const VT below = *reinterpret_cast<const VT*>(phi + rm + pin);
        const VT above = *reinterpret_cast<const VT*>(phi + rp + pin);
        S left[R], right[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            left[r] = from_prev(V::get(z0[r], N - 1));
            right[r] = from_next(V::get(z0[r], 0));
            if (lane == 0) left[r] = phi[ro[r] + pin - 1];
            if (lane == 63) right[r] = phi[ro[r] + pin + N];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const VT& ym = r > 0 ? z0[r - 1] : below;
            const VT& yp = r < R - 1 ? z0[r + 1] : above;
            VT ax, ay, az;
#pragma unroll
            for (int n = 0; n < N; ++n) {
                const double xm = n > 0 ? (double)V::get(z0[r], n - 1) : (double)left[r];
                const double xp = n < N - 1 ? (double)V::get(z0[r], n + 1) : (double)right[r];
                V::set(ax, n, (S)(-(xp - xm) * half_inv_dx));
                V::set(ay, n, (S)(-((double)V::get(yp, n) - (double)V::get(ym, n)) * half_inv_dx));
                V::set(az, n, (S)(-((double)V::get(zp[r], n) - (double)V::get(zm[r], n)) * half_inv_dx));
            }
            if (act[r]) {
                __builtin_nontemporal_store(ax, reinterpret_cast<VT*>(gx + co[r] + pout));
                __builtin_nontemporal_store(ay, reinterpret_cast<VT*>(gy + co[r] + pout));
                __builtin_nontemporal_store(az, reinterpret_cast<VT*>(gz + co[r] + pout));
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            zm[r] = z0[r];
            z0[r] = zp[r];
        }
        pin += plane;
        pout += sxy;
    }
}

}  // namespace hgs
