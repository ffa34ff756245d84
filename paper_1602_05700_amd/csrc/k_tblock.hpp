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
// Outer boundaries.  Frozen ghosts (multipole, user) keep their input value
// at every level.  Robin ghosts follow the interior at every level: an
// interior cell beside a face reads its ghost neighbour as the Robin value of
// its own level (the ghost is a multiple of that cell alone), so no ghost
// needs a value of its own inside the launch; the launch's host then sets the
// ghosts of both output levels by the same rule.  Periodic: there are no
// ghosts, the tile's cells wrap around the grid (every cell is an interior
// one), and the source is rho minus the domain mean.  Outgoing ghosts depend
// on their own previous level, so they are advanced inside the launch, level
// by level, next to the interior (TBTile below), and the launch stores them.
// Each gives the streaming substeps' results bit for bit.
//
// The plane loop is unrolled by U = lcm(3, 2, T, PF) so that the three-plane
// windows, the LDS slot parity, the ring of rho planes and the prefetch ring
// rotate by compile-time index instead of register moves.  Tiles whose
// extended region lies inside the grid take a path without per-cell x/y
// boundary selects.  The tile shape (rows per thread, waves, planes in
// flight) is a template parameter; several shapes are compiled and the
// autotuner picks one.
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

// Plane-loop unroll: lcm(3, 2, T, PF), so that the three-plane windows, the
// LDS slot parity, the ring of rho planes and the prefetch ring all rotate by
// compile-time index.
constexpr int tb_gcd(int a, int b) { return b == 0 ? a : tb_gcd(b, a % b); }
constexpr int tb_lcm(int a, int b) { return a / tb_gcd(a, b) * b; }
template <int T, int PF>
struct Unroll {
    static constexpr int U = tb_lcm(tb_lcm(6, T), PF);
};

constexpr int TB_FROZEN = 0, TB_ROBIN = 1, TB_PERIODIC = 2, TB_OUTGOING = 3;

__device__ __forceinline__ int wrap(int i, int n) {
    const int m = i % n;
    return m < 0 ? m + n : m;
}
// the same for -n <= i < 2n, without a division
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename S, int T, int W>
struct TBShared {
    S edge[T][2][W][2][64];  // [level][slot][wave][0 first row, 1 last row][lane]
};

// PF: input planes loaded ahead (the prefetch ring, in registers).
// SB: addresses as a uniform plane base plus a 32-bit byte offset kept in the
//     block of each access (no per-access 64-bit address arithmetic), else a
//     64-bit address per access.
// UPF: prefetch loads issued unconditionally (past the chunk's end the
//     clamped loads read planes that are never used: no branch and no ring
//     copies), else only while planes remain.
// Which is faster depends on the shape and depth (measured; see TileSet).
// BND: TB_FROZEN, TB_ROBIN, TB_PERIODIC or TB_OUTGOING (above)
template <typename S, int T, int R, int W, int PF, bool SB, bool UPF, bool EDGE, int BND = TB_FROZEN>
struct TBTile {
    static constexpr int IX = 64 - 2 * T;
    static constexpr int IY = W * R - 2 * T;
    static constexpr int U = Unroll<T, PF>::U;

    // uniform values (scalar registers)
    const S* in_n;
    const S* in_nm1;
    const S* rho;
    S* out_n;
    S* out_nm1;
    const StepCoef& c;
    TBShared<S, T, W>& sh;
    int64_t plane, cplane;  // elements per padded / compact plane
    int nx, ny, nz, k0, k1;
    uint32_t prow;  // bytes per padded row
    bool down;  // march the chunk from its top plane downwards
    double rb;  // TB_PERIODIC: domain-mean density subtracted from rho
    // TB_ROBIN: which faces this thread's cells touch, the coordinates
    // (storage type) of its cells, and the ghost layers' coordinates
    // (x = -1 and nx, and so on; the same for every thread)
    LocalGeom lg;
    bool fxl, fxh, fyl[R], fyh[R];
    S cxi, cyi[R];
    S gx0, gx1, gy0, gy1, gz0, gz1;
    // TB_OUTGOING: each face ghost follows its own rule inside the launch,
    // g^{t} = outgoing_ghost(g^{t-1}, i^{t-1}, i^{t}) from its interior
    // neighbour i along the normal.
    //   x ghosts are lanes: updated in place, the neighbour's two levels by
    //     lane shifts.
    //   y ghosts: the thread holding the row y = 0 (ny - 1) keeps the ghost
    //     row's levels beside it in registers (one per level) and reads its y
    //     neighbour from there, so no level of a ghost row crosses a wave; the
    //     ghost rows themselves are never read otherwise.
    //   z ghosts: the launch has an even number of z chunks, at least T planes
    //     deep, so the bottom chunk marches up and the top one down, a grid's
    //     ghost plane is always the plane before its chunk in marching order,
    //     and no chunk's halo reaches the other one.  Its level t is
    //     set one step late, when plane k0's level t exists and before any
    //     cell reads it (pipeline iteration T + t, a compile-time phase).
    // The launch stores the face ghosts of both new levels (edges and corners
    // are never read).
    S okk;                  // c dt / dx
    bool oxg[R], oxs[R];    // x-face ghost (y inside the grid); stored by this tile
    bool oxw;               // the tile reaches an x face (the same in the whole workgroup)
    bool oxlo;              // the lane is at x = -1 (else x = nx)
    S ocx;                  // x of the cell
    S ocy[R];               // y of the cells
    int oyl, oyh;           // row of this thread at y = 0 / y = ny - 1, or -1
    bool osl, osh;          // ... whose ghost this tile stores
    S gyl[T], gyh[T];       // level t of the y ghosts beside those rows (1 <= t < T)
    bool ozb;               // the plane before the chunk is a ghost
    // per-thread constants.  Addresses are a uniform plane base plus a 32-bit
    // byte offset, so loads and stores take the scalar-base form and need no
    // per-access 64-bit address arithmetic.
    int lane, w, wm, wp;
    uint32_t bp[R];  // byte offsets within a padded plane (clamped to the ghost box)
    uint32_t bc[R];  // byte offsets within a compact rho plane (clamped to the interior)
    bool in_ok[R], out_ok[R];

    // pipeline state
    S win[T][3][R];  // [level][ring slot][row]
    S rq[T][R];      // ring of rho planes
    S pn[PF][R], po[PF][R], pr[PF][R];  // prefetch ring

    // always inlined: a constructor left behind a call takes the address of
    // the whole tile, whose pipeline state then lives in scratch memory
    __device__ __forceinline__ TBTile(const S* a, const S* b, const S* rh, S* o0, S* o1, const Layout& L, const StepCoef& cc,
                      TBShared<S, T, W>& s, int tx, int ty, int kk0, int kk1,
                      const LocalGeom& geo = LocalGeom{}, double rbar = 0.0, bool march_down = false,
                      double c_dt = 0.0)
        : in_n(a), in_nm1(b), rho(rh), out_n(o0), out_nm1(o1), c(cc), sh(s), down(march_down), rb(rbar), lg(geo) {
        plane = L.plane;
        cplane = (int64_t)L.nx * L.ny;
        nx = L.nx;
        ny = L.ny;
        nz = L.nz;
        prow = (uint32_t)(L.pitch * (int)sizeof(S));
        lane = threadIdx.x & 63;
        w = threadIdx.x >> 6;
        const int x = tx * IX - T + lane;
        const int y0 = ty * IY - T + w * R;
        k0 = kk0;
        k1 = kk1;
        wm = w > 0 ? w - 1 : 0;
        wp = w < W - 1 ? w + 1 : W - 1;
        const bool x_in = x >= 0 && x < L.nx;
        const bool x_out = x_in && lane >= T && lane < T + IX;
        // periodic: every cell of the tile is the interior cell it wraps onto
        const int xc = BND == TB_PERIODIC ? wrap(x, L.nx) : min(max(x, -1), L.nx);
        const int xr = BND == TB_PERIODIC ? xc : min(max(x, 0), L.nx - 1);
        if (BND == TB_ROBIN) {
            fxl = x == 0;
            fxh = x == L.nx - 1;
            cxi = local_coord<S>(lg.x0, lg.ox, lg.dx, x);
            gx0 = local_coord<S>(lg.x0, lg.ox, lg.dx, -1);
            gx1 = local_coord<S>(lg.x0, lg.ox, lg.dx, L.nx);
            gy0 = local_coord<S>(lg.y0, lg.oy, lg.dx, -1);
            gy1 = local_coord<S>(lg.y0, lg.oy, lg.dx, L.ny);
            gz0 = local_coord<S>(lg.z0, lg.oz, lg.dx, -1);
            gz1 = local_coord<S>(lg.z0, lg.oz, lg.dx, L.nz);
        }
        if (BND == TB_OUTGOING) {
            okk = (S)(c_dt / lg.dx);
            const int xlo = tx * IX - T;
            oxw = xlo < 0 || xlo + 64 > L.nx;
            oxlo = x == -1;
            ocx = local_coord<S>(lg.x0, lg.ox, lg.dx, x);
            oyl = oyh = -1;
            osl = osh = false;
            ozb = down ? k1 == L.nz : k0 == 0;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = y0 + r;
            const int er = w * R + r;
            const bool y_in = y >= 0 && y < L.ny;
            in_ok[r] = BND == TB_PERIODIC || (x_in && y_in);
            out_ok[r] = x_out && y_in && er >= T && er < T + IY;
            const int yc = BND == TB_PERIODIC ? wrap(y, L.ny) : min(max(y, -1), L.ny);
            const int yr = BND == TB_PERIODIC ? yc : min(max(y, 0), L.ny - 1);
            bp[r] = (uint32_t)(((yc + HALO) * L.pitch + (xc + L.xoff)) * (int)sizeof(S));
            bc[r] = (uint32_t)((yr * L.nx + xr) * (int)sizeof(S));
            if (BND == TB_ROBIN) {
                fyl[r] = y == 0;
                fyh[r] = y == L.ny - 1;
                cyi[r] = local_coord<S>(lg.y0, lg.oy, lg.dx, y);
            }
            if (BND == TB_OUTGOING) {
                const int ln = x == -1 ? lane + 1 : lane - 1;  // the x ghost's neighbour lane
                oxg[r] = (x == -1 || x == L.nx) && y_in;
                oxs[r] = oxg[r] && ln >= T && ln < T + IX && er >= T && er < T + IY;
                ocy[r] = local_coord<S>(lg.y0, lg.oy, lg.dx, y);
                if (y == 0) {
                    oyl = r;
                    osl = out_ok[r];
                }
                if (y == L.ny - 1) {
                    oyh = r;
                    osh = out_ok[r];
                }
            }
        }
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                win[t][0][r] = win[t][1][r] = win[t][2][r] = (S)0;
                rq[t][r] = (S)0;
            }
        if (BND == TB_OUTGOING)
#pragma unroll
            for (int t = 0; t < T; ++t) gyl[t] = gyh[t] = (S)0;
    }

    // Plane of pipeline position p.  The pipeline runs p = k0 - T, ...,
    // k1 + T - 1 either way; marching down reflects it onto the chunk.  The
    // update is symmetric in its two z neighbours (their sum, or the sum of
    // their differences, commutes exactly), so either direction gives the
    // same bits.
    __device__ __forceinline__ int zr(int p) const { return down ? k0 + k1 - 1 - p : p; }

    __device__ __forceinline__ static S at(const S* base, uint32_t off) {
        return *reinterpret_cast<const S*>(reinterpret_cast<const char*>(base) + off);
    }
    __device__ __forceinline__ static void put(S* base, uint32_t off, S v) {
        *reinterpret_cast<S*>(reinterpret_cast<char*>(base) + off) = v;
    }

    // inputs of plane p: phi^n(p), phi^{n-1}(p-1), rho(p-1), into ring slot B.
    // Loads are never predicated: plane and lane offsets are clamped into the
    // ghost box (the interior for rho), and every value read that way lands in
    // a cell outside the interior, which keeps its input value and feeds no
    // valid cell.
    template <int B>
    __device__ __forceinline__ void load(int p) {
        // periodic: planes in [k0 - T, k1 + T) wrap once when nz > T
        const int zp = zr(p), zq = zr(p - 1);
        const int pc = BND == TB_PERIODIC ? (nz > T ? wrap1(zp, nz) : wrap(zp, nz)) : min(max(zp, -1), nz);
        const int qc = BND == TB_PERIODIC ? (nz > T ? wrap1(zq, nz) : wrap(zq, nz)) : min(max(zq, 0), nz - 1);
        const S* bn = in_n + (int64_t)(pc + HALO) * plane;
        const S* bo = in_nm1 + (int64_t)(qc + HALO) * plane;
        const S* br = rho + (int64_t)qc * cplane;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            // SB: keep the 32-bit offsets in this block so the loads take the
            // scalar-base form (no 64-bit address per access)
            uint32_t op = bp[r], oc = bc[r];
            if (SB) asm("" : "+v"(op), "+v"(oc));
            pn[B][r] = at(bn, op);
            po[B][r] = at(bo, op);
            pr[B][r] = BND == TB_PERIODIC ? source(at(br, oc), rb) : at(br, oc);
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
        if (UPF || p + PF < pend) load<B>(p + PF);
        __syncthreads();  // LDS writes of plane p-1 are visible; its reads are done
        sh.edge[0][SLOT][w][0][lane] = win[0][NEW][0];
        sh.edge[0][SLOT][w][1][lane] = win[0][NEW][R - 1];
        S cl = (S)0, ch = (S)0;  // TB_OUTGOING: level t-1 of the y ghosts at plane q (t >= 2)
#pragma unroll
        for (int t = 1; t <= T; ++t) {
            const int q = p - t;
            const int qz = zr(q);
            // level t-1 holds pipeline position q in MID, q+1 in NEW, q-1 in
            // OLD; level t-2 holds q in OLD (its NEW is q+2).  Planes outside
            // the grid (the ghost plane and the clamped ring below and above
            // it) keep their input value (a select on a uniform condition).
            const bool z_in = BND == TB_PERIODIC || (qz >= 0 && qz < nz);
            S zz = (S)0;
            if (BND == TB_ROBIN) {
                const S cz = local_coord<S>(lg.z0, lg.oz, lg.dx, qz);
                zz = cz * cz;
            }
            S nv[R];
            // TB_OUTGOING: the y ghosts' level t-1 at plane q (the input at
            // t = 1, then the registers kept beside rows oyl / oyh), and the
            // levels t-1 and t of those rows
            S gl = (S)0, gh = (S)0, il = (S)0, ih = (S)0, nl = (S)0, nh = (S)0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const S ce = win[t - 1][MID][r];
                    S zm = win[t - 1][OLD][r];
                    S zp = win[t - 1][NEW][r];
                    S ym = (r > 0) ? win[t - 1][MID][r - 1] : sh.edge[t - 1][PREV][wm][1][lane];
                    S yp = (r < R - 1) ? win[t - 1][MID][r + 1] : sh.edge[t - 1][PREV][wp][0][lane];
                    S xm = (S)lane_prev(ce);
                    S xp = (S)lane_next(ce);
                    // Robin: a ghost neighbour is the Robin value of this cell's
                    // own level (robin_ghost on the operands the ghost launch
                    // uses); x and y faces only in tiles that reach them, z faces
                    // in any tile at the first and last plane
                    if (BND == TB_ROBIN && EDGE) {
                        if (fxl || fxh) {
                            const S yz = fma(cyi[r], cyi[r], zz);
                            const S cg = fxl ? gx0 : gx1;
                            const S g = robin_ghost(fma(cxi, cxi, yz), fma(cg, cg, yz), ce);
                            if (fxl)
                                xm = g;
                            else
                                xp = g;
                        }
                        if (fyl[r] || fyh[r]) {
                            const S cg = fyl[r] ? gy0 : gy1;
                            const S g = robin_ghost(fma(cxi, cxi, fma(cyi[r], cyi[r], zz)),
                                                    fma(cxi, cxi, fma(cg, cg, zz)), ce);
                            if (fyl[r])
                                ym = g;
                            else
                                yp = g;
                        }
                    }
                    if (BND == TB_ROBIN) {
                        if (qz == 0 || qz == nz - 1) {
                            const S cg = qz == 0 ? gz0 : gz1;
                            const S g = robin_ghost(fma(cxi, cxi, fma(cyi[r], cyi[r], zz)),
                                                    fma(cxi, cxi, fma(cyi[r], cyi[r], cg * cg)), ce);
                            // the ghost is the neighbour below plane 0 and above
                            // plane nz - 1: OLD going up, NEW going down
                            if ((qz == 0) != down)
                                zm = g;
                            else
                                zp = g;
                        }
                    }
                    if (BND == TB_OUTGOING) {
                        if (r == oyl) {
                            if (t >= 2) ym = cl;
                            gl = ym;
                            il = ce;
                        }
                        if (r == oyh) {
                            if (t >= 2) yp = ch;
                            gh = yp;
                            ih = ce;
                        }
                    }
                    const S ol = (t == 1) ? old1[r] : win[t >= 2 ? t - 2 : 0][OLD][r];
                    const int RS = ((PH - t + 1) % T + T) % T;  // ring slot of rho(p - t)
                    const S v = (S)update(c, ce, xm, xp, ym, yp, zm, zp, ol, rq[RS][r]);
                    nv[r] = (EDGE ? (in_ok[r] && z_in) : z_in) ? v : ce;
                    if (BND == TB_OUTGOING && oxw) {
                        // x ghosts in place: the neighbour lane's levels t-1
                        // (xp / xm) and t (shifted here by every lane)
                        const S nn = (S)lane_next(nv[r]), np = (S)lane_prev(nv[r]);
                        if (oxg[r] && z_in) {
                            const S cz = local_coord<S>(lg.z0, lg.oz, lg.dx, qz);
                            const S yz = fma(ocy[r], ocy[r], cz * cz);
                            const S xn = local_coord<S>(lg.x0, lg.ox, lg.dx, oxlo ? 0 : nx - 1);
                            const S xf = local_face<S>(lg.x0, lg.ox, lg.dx, oxlo ? 0 : nx);
                            nv[r] = outgoing_ghost(fma(xn, xn, yz), fma(ocx, ocx, yz), fma(xf, xf, yz),
                                                   oxlo ? -xf : xf, okk, ce, oxlo ? xp : xm, oxlo ? nn : np);
                        }
                    }
                    if (BND == TB_OUTGOING) {
                        if (r == oyl) nl = nv[r];
                        if (r == oyh) nh = nv[r];
                    }
                }
            // TB_OUTGOING: y ghosts beside rows oyl / oyh, and the z ghost planes
            S Gl = (S)0, Gh = (S)0;
            if (BND == TB_OUTGOING) {
                if (oyl >= 0 || oyh >= 0) {
                    const S cz = local_coord<S>(lg.z0, lg.oz, lg.dx, qz);
                    if (oyl >= 0) {
                        const S yf = local_face<S>(lg.y0, lg.oy, lg.dx, 0);
                        Gl = outgoing_ghost(local_r2(ocx, local_coord<S>(lg.y0, lg.oy, lg.dx, 0), cz),
                                            local_r2(ocx, local_coord<S>(lg.y0, lg.oy, lg.dx, -1), cz),
                                            local_r2(ocx, yf, cz), -yf, okk, gl, il, nl);
                    }
                    if (oyh >= 0) {
                        const S yf = local_face<S>(lg.y0, lg.oy, lg.dx, ny);
                        Gh = outgoing_ghost(local_r2(ocx, local_coord<S>(lg.y0, lg.oy, lg.dx, ny - 1), cz),
                                            local_r2(ocx, local_coord<S>(lg.y0, lg.oy, lg.dx, ny), cz),
                                            local_r2(ocx, yf, cz), yf, okk, gh, ih, nh);
                    }
                    if (t < T) {
                        // level t+1 (plane q - 1) reads level t of plane q - 1
                        cl = gyl[t];
                        ch = gyh[t];
                        gyl[t] = Gl;
                        gyh[t] = Gh;
                    }
                }
                // the plane before the chunk: level t from plane k0's levels
                // t-1 and t (its own level t-1 is level t-1's OLD plane);
                // level t reaches plane k0 at iteration T + t
                if ((T + t) % U == PH && ozb && q == k0) {
                    const int zg = zr(k0 - 1), zi = zr(k0);
                    const bool hi = zg >= 0;
                    const S czi = local_coord<S>(lg.z0, lg.oz, lg.dx, zi), czg = local_coord<S>(lg.z0, lg.oz, lg.dx, zg),
                            czf = local_face<S>(lg.z0, lg.oz, lg.dx, hi ? nz : 0);
                    S g[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        g[r] = outgoing_ghost(local_r2(ocx, ocy[r], czi), local_r2(ocx, ocy[r], czg),
                                              local_r2(ocx, ocy[r], czf), hi ? czf : -czf, okk,
                                              win[t - 1][OLD][r], win[t - 1][MID][r], nv[r]);
                    }
                    if (t < T) {
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            if (in_ok[r]) win[t][MID][r] = g[r];
                    } else {
                        S* on = out_n + (int64_t)(zg + HALO) * plane;
                        S* oo = out_nm1 + (int64_t)(zg + HALO) * plane;
#pragma unroll
                        for (int r = 0; r < R; ++r)
                            if (out_ok[r]) {
                                uint32_t o = bp[r];
                                if (SB) asm("" : "+v"(o));
                                put(on, o, g[r]);
                                put(oo, o, win[T - 1][OLD][r]);
                            }
                    }
                }
            }
            if (t < T) {
#pragma unroll
                for (int r = 0; r < R; ++r) win[t][NEW][r] = nv[r];
                sh.edge[t][SLOT][w][0][lane] = nv[0];
                sh.edge[t][SLOT][w][1][lane] = nv[R - 1];
            } else if (q >= k0 && q < k1) {  // the reflection keeps [k0, k1)
                S* on = out_n + (int64_t)(qz + HALO) * plane;
                S* oo = out_nm1 + (int64_t)(qz + HALO) * plane;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    // TB_OUTGOING: x ghost lanes store their own levels too
                    if (out_ok[r] || (BND == TB_OUTGOING && oxs[r])) {
                        uint32_t o = bp[r];
                        // SB: keep the 32-bit offset in this block so the
                        // stores take the scalar-base form like the loads
                        if (SB) asm("" : "+v"(o));
                        put(on, o, nv[r]);
                        put(oo, o, win[T - 1][MID][r]);
                    }
                }
                if (BND == TB_OUTGOING) {
                    // the y ghosts beside rows oyl / oyh (level T-1 is the
                    // value their rows read at level T)
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        if (r == oyl && osl) {
                            put(on, bp[r] - prow, Gl);
                            put(oo, bp[r] - prow, gl);
                        }
                        if (r == oyh && osh) {
                            put(on, bp[r] + prow, Gh);
                            put(oo, bp[r] + prow, gh);
                        }
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

    // the first PF input planes, from p0 on
    template <int B>
    __device__ __forceinline__ void prime(int p0) {
        if constexpr (B < PF) {
            load<B>(p0 + B);
            prime<B + 1>(p0);
        }
    }

    __device__ void run() {
        const int pend = k1 + T;
        prime<0>(k0 - T);
        for (int p = k0 - T; p < pend; p += U)
            if (!run_from<0>(p, pend)) break;
    }
    // the same, always inlined (for bodies the inliner would leave behind a
    // call, whose pipeline state would then live in scratch memory)
    __device__ __forceinline__ void run_inline() {
        const int pend = k1 + T;
        prime<0>(k0 - T);
        for (int p = k0 - T; p < pend; p += U)
            if (!run_from<0>(p, pend)) break;
    }
};

// BND: TB_FROZEN, TB_ROBIN (lg: cell positions), TB_PERIODIC (rbar: device
// pointer to the domain-mean density) or TB_OUTGOING (lg, and c_dt = c_g dt)
template <typename S, int T, int R, int W, int PF, bool SB, bool UPF, int BND>
__global__ __launch_bounds__(64 * W) void k_leapfrog_tblock(const S* __restrict__ in_n, const S* __restrict__ in_nm1,
                                                            const S* __restrict__ rho, S* __restrict__ out_n,
                                                            S* __restrict__ out_nm1, Layout L, StepCoef c, int zc,
                                                            int tiles_x, int tiles_y, LocalGeom lg,
                                                            const double* __restrict__ rbar, double c_dt) {
    constexpr int IX = 64 - 2 * T;
    constexpr int IY = W * R - 2 * T;
    static_assert(IX > 0 && IY > 0, "tile too small for the temporal depth");
    __shared__ TBShared<S, T, W> sh;
    // tiles vary fastest and z chunks slowest, so the workgroups resident at
    // one time are neighbours at the same heights and share halo lines in L2
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = bid % tiles_x;
    const int ty = (bid / tiles_x) % tiles_y;
    const int tz = bid / (tiles_x * tiles_y);
    const int k0 = tz * zc;
    const int k1 = min(k0 + zc, L.nz);
    // the extended tile lies strictly inside the grid: no per-cell boundary
    // work across x and y
    const int xlo = tx * IX - T, ylo = ty * IY - T;
    const bool inner = xlo >= 0 && xlo + 64 <= L.nx && ylo >= 0 && ylo + W * R <= L.ny;
    const double rb = BND == TB_PERIODIC ? *rbar : 0.0;
    // odd chunks march downwards, so two neighbouring chunks reach the planes
    // they both read (T each side of their common face) at the same time, and
    // the second read can find them in the last-level cache
    const bool down = (tz & 1) != 0;
    // Local-boundary launches compile the edge body only: two bodies of
    // the larger shapes with the boundary terms exceed the inliner's budget,
    // and a pipeline left behind a call reaches its state through scratch
    // memory (measured: 15 times slower)
    if (BND == TB_FROZEN && inner) {
        TBTile<S, T, R, W, PF, SB, UPF, false, BND> t(in_n, in_nm1, rho, out_n, out_nm1, L, c, sh, tx, ty, k0, k1, lg,
                                                      rb, down, c_dt);
        t.run();
    } else {
        TBTile<S, T, R, W, PF, SB, UPF, true, BND> t(in_n, in_nm1, rho, out_n, out_nm1, L, c, sh, tx, ty, k0, k1, lg,
                                                     rb, down, c_dt);
        if (BND == TB_OUTGOING)
            t.run_inline();
        else
            t.run();
    }
}

// Launch geometry of the fused kernel for a grid.
struct TBlockDims {
    int tiles_x, tiles_y, zc, nblocks;
};

// Number of z chunks: each workgroup occupies one CU slot for (chunk planes +
// 2T) pipeline steps and the launch runs in ceil(blocks / slots) rounds, so
// pick the chunk count that minimises rounds x steps.  even: only even counts
// of chunks at least T planes deep (needs nz >= 2T), so that the bottom chunk
// marches up and the top one down, and no chunk's T-plane halo reaches a
// ghost plane other than the one before it (the outgoing form's ghost planes).
template <int T, int R, int W>
inline TBlockDims tblock_dims(const Layout& L, int slots, bool even = false) {
    constexpr int IX = 64 - 2 * T;
    constexpr int IY = W * R - 2 * T;
    TBlockDims d;
    d.tiles_x = (L.nx + IX - 1) / IX;
    d.tiles_y = (L.ny + IY - 1) / IY;
    const int64_t cols = (int64_t)d.tiles_x * d.tiles_y;
    int best = 1;
    int64_t best_cost = -1;
    const int maxz = std::max(even ? 2 : 1, std::min(64, L.nz / (2 * T)));
    for (int nzc = 1; nzc <= maxz; ++nzc) {
        const int zc = (L.nz + nzc - 1) / nzc;
        const int nch = (L.nz + zc - 1) / zc;
        if (even && (nch % 2 != 0 || zc < T || L.nz - (nch - 1) * zc < T)) continue;
        const int64_t nb = cols * nch;
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

// Tile shapes: R rows per thread, W waves per workgroup, PF input planes in
// flight, and the addressing / prefetch forms (SB, UPF above).  Registers
// bound them: every level keeps three planes per cell, so a taller tile (less
// halo per cell) leaves room for fewer planes in flight.  Index 0 is each
// depth's default, the fastest measured on MI355X for 512^3 FP32 and 256^3
// FP64 (us per fused launch inside hydro steps, i.e. after the moment and
// ghost launches):
//   FP32 T=4: R2 W16 PF3 64-bit 751-782, R2 W16 PF2 SB 804-824,
//             R2 W16 PF2 64-bit (standalone 830 against 813 for the first);
//             taller tiles spill or lack planes in flight (R3 W16 PF1 SB 883,
//             spilling 13 registers once the chunk direction became a
//             run-time value, so it was replaced by the third shape);
//   FP32 T=3 and T=2: R2 W16 PF3 64-bit 729 and 735 (SB forms 762 and 873
//             in standalone timing against 735 and 738);
//   FP64 T=4: R3 W8 PF1 SB 196, R2 W8 PF2 SB 257, R2 W8 PF3 64-bit 289
//             (a 64 x 24 tile has a 56 x 16 core, against 56 x 8 for 64 x 16);
//   FP64 T=3 and T=2: R3 W8 PF1 SB 180, R4 W8 PF1 SB 158 (standalone: 200
//             and 162 against 241 and 174 for R2 W8 PF3 64-bit).
// The autotuner times every shape of every depth.
struct TileShape {
    int R, W, PF;
    bool SB, UPF;
};
template <typename S, int T>
struct TileSet {
    static constexpr int N = 2;
    static constexpr TileShape at(int i) {
        // the second shape of depths 2 and 3 is the other family: the taller
        // tile for FP32, the shorter one for FP64 (more tiles for small grids)
        return sizeof(S) == 4 ? (i == 1 ? (T == 2 ? TileShape{4, 16, 2, true, true} : TileShape{3, 16, 2, true, true})
                                        : TileShape{2, 16, 3, false, false})
                              : (i == 1 ? TileShape{2, 8, 3, false, false}
                                        : (T == 2 ? TileShape{4, 8, 1, true, true} : TileShape{3, 8, 1, true, true}));
    }
};
template <typename S>
struct TileSet<S, 4> {
    static constexpr int N = 3;
    static constexpr TileShape at(int i) {
        return sizeof(S) == 4 ? (i == 1   ? TileShape{2, 16, 2, true, true}
                                 : i == 2 ? TileShape{2, 16, 2, false, false}
                                          : TileShape{2, 16, 3, false, false})
                              : (i == 1   ? TileShape{2, 8, 3, false, false}
                                 : i == 2 ? TileShape{2, 8, 2, true, true}
                                          : TileShape{3, 8, 1, true, true});
    }
};

inline int tile_count(int T) { return T == 4 ? 3 : (T >= 2 ? 2 : 1); }

// Outer boundary of a fused launch: mode (TB_*), cell positions (Robin,
// outgoing), the device mean density (periodic) and c_g dt (outgoing)
struct TBBound {
    int mode;
    LocalGeom lg;
    const double* rbar;
    double c_dt;
};

template <typename S, int T, int I, int BND>
void launch_tblock_shape(const S* in_n, const S* in_nm1, const S* rho, S* out_n, S* out_nm1, const Layout& L,
                         const StepCoef& c, int ncu, hipStream_t st, const TBBound& b) {
    constexpr TileShape sh = TileSet<S, T>::at(I);
    const TBlockDims d = tblock_dims<T, sh.R, sh.W>(L, ncu, BND == TB_OUTGOING);
    hipLaunchKernelGGL((k_leapfrog_tblock<S, T, sh.R, sh.W, sh.PF, sh.SB, sh.UPF, BND>), dim3(d.nblocks),
                       dim3(64 * sh.W), 0, st, in_n, in_nm1, rho, out_n, out_nm1, L, c, d.zc, d.tiles_x, d.tiles_y,
                       b.lg, b.rbar, b.c_dt);
}

template <typename S, int T, int I>
void launch_tblock_bnd(const S* in_n, const S* in_nm1, const S* rho, S* out_n, S* out_nm1, const Layout& L,
                       const StepCoef& c, int ncu, hipStream_t st, const TBBound& b) {
    switch (b.mode) {
        case TB_ROBIN: {
            // Shapes whose Robin form does not compile clean run another shape
            // (shapes give identical results): FP32 depth 4 shape 0 spills past
            // the 128 registers of a 16-wave workgroup and shape 2 is not
            // inlined (its pipeline would sit behind a call, in scratch), so
            // both run shape 1; FP32 depth 2 shape 1 spills and runs shape 0;
            // FP64 depth 4 shape 0 is not inlined and runs shape 2.
            constexpr int IR = sizeof(S) == 4 ? (T == 4 ? 1 : (T == 2 ? 0 : I)) : (T == 4 && I == 0 ? 2 : I);
            launch_tblock_shape<S, T, IR, TB_ROBIN>(in_n, in_nm1, rho, out_n, out_nm1, L, c, ncu, st, b);
            break;
        }
        case TB_PERIODIC:
            launch_tblock_shape<S, T, I, TB_PERIODIC>(in_n, in_nm1, rho, out_n, out_nm1, L, c, ncu, st, b);
            break;
        case TB_OUTGOING: {
            // The same for the outgoing form: FP32 depth 4 runs shape 1 (the
            // others spill), FP32 depths 2 and 3 shape 0 (shape 1 spills),
            // FP64 depth 4 shape 2 (the others spill).
            constexpr int IO = sizeof(S) == 4 ? (T == 4 ? 1 : 0) : (T == 4 ? 2 : I);
            launch_tblock_shape<S, T, IO, TB_OUTGOING>(in_n, in_nm1, rho, out_n, out_nm1, L, c, ncu, st, b);
            break;
        }
        default: launch_tblock_shape<S, T, I, TB_FROZEN>(in_n, in_nm1, rho, out_n, out_nm1, L, c, ncu, st, b);
    }
}

template <typename S, int T>
void launch_tblock_t(const S* in_n, const S* in_nm1, const S* rho, S* out_n, S* out_nm1, const Layout& L,
                     const StepCoef& c, int tile, int ncu, hipStream_t st, const TBBound& b) {
    if constexpr (TileSet<S, T>::N > 2) {
        if (tile == 2) return launch_tblock_bnd<S, T, 2>(in_n, in_nm1, rho, out_n, out_nm1, L, c, ncu, st, b);
    }
    if constexpr (TileSet<S, T>::N > 1) {
        if (tile == 1) return launch_tblock_bnd<S, T, 1>(in_n, in_nm1, rho, out_n, out_nm1, L, c, ncu, st, b);
    }
    launch_tblock_bnd<S, T, 0>(in_n, in_nm1, rho, out_n, out_nm1, L, c, ncu, st, b);
}

// ncu: compute units of the device (one resident workgroup of this kernel
// each); tile: index into TileSet<S, T> (a depth with fewer shapes takes 0);
// b: the outer boundary (frozen ghosts by default)
template <typename S>
void launch_tblock(const S* in_n, const S* in_nm1, const S* rho, S* out_n, S* out_nm1, const Layout& L,
                   const StepCoef& c, int T, int tile, int ncu, hipStream_t st,
                   const TBBound& b = TBBound{TB_FROZEN, LocalGeom{}, nullptr, 0.0}) {
    switch (T) {
        case 2: launch_tblock_t<S, 2>(in_n, in_nm1, rho, out_n, out_nm1, L, c, tile, ncu, st, b); break;
        case 3: launch_tblock_t<S, 3>(in_n, in_nm1, rho, out_n, out_nm1, L, c, tile, ncu, st, b); break;
        case 4: launch_tblock_t<S, 4>(in_n, in_nm1, rho, out_n, out_nm1, L, c, tile, ncu, st, b); break;
        default: break;
    }
}

}  // namespace hgs
