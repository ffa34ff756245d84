// Host side of the C ABI declared in include/hgs.h.
//
// The library never allocates device memory: hgs_init carves the caller's
// workspace into four padded state buffers (two levels in use, two more for
// the out-of-place temporally blocked launches), the moment partials and the
// reduction scratch.  Every entry point validates on the host first and only
// then enqueues work on the context's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hgs.h"
#include "common.hpp"
#include "k_multipole.hpp"
#include "k_state.hpp"
#include "k_stencil.hpp"
#include "k_tblock.hpp"
#include "k_batch.hpp"
#include "k_local.hpp"
#include "k_nest.hpp"
#include "k_poisson.hpp"
#include <algorithm>
#include <cstdlib>
#include <fstream>
#include <map>
#include <sstream>
#include <tuple>

using namespace hgs;

struct hgs_ctx {
    hgs_config cfg;
    Layout L;
    hipStream_t stream;
    int esize;
    void* buf[4];
    int cur, old;  // buffers holding phi^n and phi^{n-1}
    double* mom_partial;
    double* mom;
    int mom_blocks, mom_zc, mom_tx, mom_ty;
    bool mom_vec;  // 16-byte loads along x (nx a multiple of the vector width)
    double* red_partial;
    double* red_out;
    double* mean;  // domain-mean density (periodic boundary), device
    int red_blocks;
    double dt_prev;
    bool have_moments;
    int tblock;
    int tile;  // tile shape of the fused launches (index into TileSet)
    int ncu;  // compute units of the device
    std::string err;
    // launch timing (hgs_timing_*)
    bool timing;
    struct Rec {
        int kind;
        hipEvent_t a, b;
        double bytes, updates;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    size_t pool_used;
};

namespace {

thread_local std::string g_err;

constexpr int kMaxN = 8192;
constexpr size_t kAlign = 256;
constexpr int kRedBlocks = 1024;
constexpr int kMomMinZ = 32;  // fewest z planes per moment chunk (when nz allows)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

hgs_status fail(hgs_ctx* c, hgs_status s, const std::string& msg) {
    if (c)
        c->err = msg;
    else
        g_err = msg;
    return s;
}

struct Plan {
    size_t buf_bytes;  // one padded state buffer
    size_t mom_partial_off, mom_off, red_partial_off, red_out_off, mean_off, total;
    int mom_blocks, mom_zc, mom_tx, mom_ty;
    bool mom_vec;
};

hgs_status check_config(const hgs_config* cfg, std::string& why) {
    if (!cfg) {
        why = "cfg is NULL";
        return HGS_ERR_ARG;
    }
    if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1 || cfg->nx > kMaxN || cfg->ny > kMaxN || cfg->nz > kMaxN) {
        why = "grid sizes must be in 1..8192";
        return HGS_ERR_ARG;
    }
    if (!(cfg->dx > 0.0) || !std::isfinite(cfg->dx)) {
        why = "dx must be positive and finite";
        return HGS_ERR_ARG;
    }
    if (!std::isfinite(cfg->x0) || !std::isfinite(cfg->y0) || !std::isfinite(cfg->z0) || !std::isfinite(cfg->G) ||
        !std::isfinite(cfg->origin[0]) || !std::isfinite(cfg->origin[1]) || !std::isfinite(cfg->origin[2])) {
        why = "x0, y0, z0, G and origin must be finite";
        return HGS_ERR_ARG;
    }
    if (cfg->lmax < 0 || cfg->lmax > HGS_LMAX) {
        why = "lmax must be in 0..4";
        return HGS_ERR_ARG;
    }
    if (cfg->bc < HGS_BC_MULTIPOLE || cfg->bc > HGS_BC_PERIODIC) {
        why = "bc must be one of HGS_BC_MULTIPOLE, USER, ROBIN, OUTGOING, PERIODIC";
        return HGS_ERR_ARG;
    }
    if (cfg->storage != HGS_F64 && cfg->storage != HGS_F32) {
        why = "storage must be HGS_F64 or HGS_F32";
        return HGS_ERR_ARG;
    }
    if (cfg->tblock < 0 || cfg->tblock > HGS_TMAX) {
        why = "tblock must be in 0..4";
        return HGS_ERR_ARG;
    }
    if (!(cfg->eta >= 0.0) || !std::isfinite(cfg->eta)) {
        why = "eta must be >= 0 and finite";
        return HGS_ERR_ARG;
    }
    if (cfg->bc == HGS_BC_MULTIPOLE || cfg->bc == HGS_BC_ROBIN || cfg->bc == HGS_BC_OUTGOING) {
        // the exterior expansion and the r-weighted local rules are evaluated
        // at the ghost centres; with the centre strictly inside the grid they
        // all lie at r >= dx/2 > 0 and every face is seen at cos(theta) > 0
        const double lo[3] = {cfg->x0, cfg->y0, cfg->z0};
        const int n[3] = {cfg->nx, cfg->ny, cfg->nz};
        for (int d = 0; d < 3; ++d)
            if (!(cfg->origin[d] > lo[d] && cfg->origin[d] < lo[d] + n[d] * cfg->dx)) {
                why = "the multipole expansion centre must lie strictly inside the grid";
                return HGS_ERR_ARG;
            }
    }
    int es = cfg->storage == HGS_F64 ? 8 : 4;
    Layout L = make_layout(cfg->nx, cfg->ny, cfg->nz, es);
    if (L.total >= ((int64_t)1 << 31)) {
        why = "grid too large for one buffer (padded elements must stay below 2^31)";
        return HGS_ERR_ARG;
    }
    return HGS_OK;
}

Plan make_plan(const hgs_config* cfg) {
    Plan p;
    int es = cfg->storage == HGS_F64 ? 8 : 4;
    Layout L = make_layout(cfg->nx, cfg->ny, cfg->nz, es);
    p.buf_bytes = align_up((size_t)L.total * es, kAlign);
    // moments: 64 x 4 lanes over (x, y) columns (N columns per lane when
    // vectorised); split z towards >= 2048 workgroups, but keep at least
    // kMomMinZ planes per chunk: every lane ends its chunk with the harmonics
    // of its columns (about 150 FP64 operations each) and a 25-value block
    // reduction, which short chunks do not amortise (256^3 FP32 with 8-plane
    // chunks read rho at 1.7 TB/s)
    const int vec = 16 / es;
    p.mom_vec = cfg->nx % vec == 0;
    const int colw = p.mom_vec ? 64 * vec : 64;
    p.mom_tx = (cfg->nx + colw - 1) / colw;
    p.mom_ty = (cfg->ny + 3) / 4;
    int cols = p.mom_tx * p.mom_ty;
    // small grids would get too few workgroups from kMomMinZ-plane chunks
    // (32^3: 8 workgroups, 24 us for 128 KB of rho); there chunks go down to 4
    // planes, since the harmonics per column then cost little in absolute terms
    const int zmin = (int64_t)cols * (cfg->nz / kMomMinZ) < 512 ? 4 : kMomMinZ;
    int zsplit = std::max(1, std::min(cfg->nz / zmin, (2048 + cols - 1) / cols));
    p.mom_zc = (cfg->nz + zsplit - 1) / zsplit;
    p.mom_blocks = cols * ((cfg->nz + p.mom_zc - 1) / p.mom_zc);
    size_t off = 4 * p.buf_bytes;
    p.mom_partial_off = off;
    off = align_up(off + (size_t)p.mom_blocks * NQ * sizeof(double), kAlign);
    p.mom_off = off;
    off = align_up(off + NQ * sizeof(double), kAlign);
    p.red_partial_off = off;
    off = align_up(off + (size_t)kRedBlocks * NRED * sizeof(double), kAlign);
    p.red_out_off = off;
    off = align_up(off + NRED * sizeof(double), kAlign);
    p.mean_off = off;
    off = align_up(off + sizeof(double), kAlign);
    p.total = off;
    return p;
}

template <typename S>
S* B(hgs_ctx* c, int k) {
    return static_cast<S*>(c->buf[k]);
}

hgs_status launch_check(hgs_ctx* c, const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, HGS_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return HGS_OK;
}

int grid_for(int64_t n, int block = 256, int cap = 65536) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

MomGeom geom(const hgs_ctx* c) {
    MomGeom g;
    g.nx = c->cfg.nx;
    g.ny = c->cfg.ny;
    g.nz = c->cfg.nz;
    g.x0 = c->cfg.x0;
    g.y0 = c->cfg.y0;
    g.z0 = c->cfg.z0;
    g.dx = c->cfg.dx;
    g.ox = c->cfg.origin[0];
    g.oy = c->cfg.origin[1];
    g.oz = c->cfg.origin[2];
    return g;
}

StepCoef step_coef(const hgs_ctx* c, double cg, double dt) {
    const double c2dt2 = cg * cg * dt * dt;
    const double kk = c2dt2 / (c->cfg.dx * c->cfg.dx);
    const double a = 0.5 * c->cfg.eta * dt;
    const double inv = 1.0 / (1.0 + a);
    StepCoef s;
    s.c0 = (2.0 - 6.0 * kk) * inv;
    s.c1 = kk * inv;
    s.cm = -(1.0 - a) * inv;
    s.cs = -c2dt2 * 4.0 * M_PI * c->cfg.G * inv;
    s.fo = (float)((1.0 - a) * inv);
    s.fl = (float)s.c1;
    s.fs = (float)s.cs;
    return s;
}

// ---- launch timing ----------------------------------------------------------

hipEvent_t pool_event(hgs_ctx* c) {
    if (c->pool_used == c->pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->pool.push_back(e);
    }
    return c->pool[c->pool_used++];
}

// Brackets one launch: call begin() before it and end() after it.
struct Timed {
    hgs_ctx* c;
    hipEvent_t a = nullptr;
    int kind;
    Timed(hgs_ctx* ctx, int k) : c(ctx), kind(k) {
        if (c->timing) {
            a = pool_event(c);
            if (a && hipEventRecord(a, c->stream) != hipSuccess) a = nullptr;
        }
    }
    void end(double bytes, double updates) {
        if (!a) return;
        hipEvent_t b = pool_event(c);
        if (!b) return;
        if (hipEventRecord(b, c->stream) != hipSuccess) return;
        c->recs.push_back({kind, a, b, bytes, updates});
    }
};

// ---- launches, templated on the storage type ---------------------------------

constexpr int SBX = 64, SBY = 4;  // streaming tile (scalar kernels)
// Gradient tile: GR rows per thread, GBY waves.  Measured at 512^3 FP32 (us
// per launch, z chunks of 16 planes unless noted): 4 x 2 428, 8 x 1 429,
// 4 x 4 430, 4 x 8 430, 2 x 4 446; 4 x 2 with 32 and 64 planes 462 and 450;
// one row per thread in 8 waves (each row loaded again by the threads above
// and below it) 475.  Bound by its three output streams (12 of its ~16.5
// bytes per cell in FP32).
constexpr int GR = 4, GBY = 2;

// Tiles of bx x by columns marching up z chunks of >= 16 planes, with enough
// workgroups to fill every CU several times over.
inline void stream_dims(const Layout& L, int bx, int& zc, int& tiles_x, int& tiles_y, int& nblocks, int by = SBY) {
    tiles_x = (L.nx + bx - 1) / bx;
    tiles_y = (L.ny + by - 1) / by;
    int cols = tiles_x * tiles_y;
    int zsplit = std::max(1, std::min((L.nz + 15) / 16, (4096 + cols - 1) / cols));
    zc = (L.nz + zsplit - 1) / zsplit;
    nblocks = cols * ((L.nz + zc - 1) / zc);
}

// the 16-byte-per-lane kernels need whole vectors along x
template <typename S>
bool use_vec(const Layout& L) {
    return L.nx % Vec16<S>::N == 0;
}

// Boundaries whose ghosts follow the interior every substep, as opposed to
// ghosts frozen over a hydrodynamical step (multipole, user).
bool local_bc(int bc) { return bc == HGS_BC_ROBIN || bc == HGS_BC_OUTGOING || bc == HGS_BC_PERIODIC; }

// Substeps per launch: the fused depth, except for grids with a local
// boundary thinner than two cells (a cell there borders both faces of an
// axis), and at most nz / 2 for the outgoing rule (its fused launch splits z
// into two or more chunks at least that deep).
int fused_depth(const hgs_ctx* c) {
    if (local_bc(c->cfg.bc) && std::min(c->cfg.nx, std::min(c->cfg.ny, c->cfg.nz)) < 2) return 1;
    if (c->cfg.bc == HGS_BC_OUTGOING) {
        const int t = std::min(c->tblock, c->cfg.nz / 2);
        return t >= 2 ? t : 1;
    }
    return c->tblock;
}

// Buffers that hold phi^n at some point of the coming nsub substeps, the
// last state included: a fused launch reads (cur, old) and makes the other
// two buffers (phi^{n+T}, phi^{n+T-1}); a streaming substep writes the new
// level over old, which becomes cur.  Only these read their ghosts (the
// update reads phi^{n-1} at the cell alone), so only they need this
// hydrodynamical step's ghosts.  Bit k of the result = buffer k.
int ghost_buffers(const hgs_ctx* c, int nsub) {
    const int T = fused_depth(c);
    int cur = c->cur, old = c->old;
    int mask = 1 << cur;
    while (nsub > 0) {
        if (T > 1 && nsub >= T) {
            int o0 = -1, o1 = -1;
            for (int k = 0; k < 4; ++k)
                if (k != cur && k != old) (o0 < 0 ? o0 : o1) = k;
            cur = o0;
            old = o1;
            nsub -= T;
        } else {
            std::swap(cur, old);
            nsub -= 1;
        }
        mask |= 1 << cur;
    }
    return mask;
}

// mask: the buffers that receive the ghosts (bit k = buffer k)
template <typename S>
void run_moments_and_ghosts(hgs_ctx* c, const void* rho, int mask) {
    const MomGeom g = geom(c);
    Timed tm(c, HGS_KERNEL_MULTIPOLE);
    dim3 blk(64, 4);
    if (c->mom_vec)
        hipLaunchKernelGGL(k_moments_partial_v<S>, dim3(c->mom_blocks), blk, 0, c->stream,
                           static_cast<const S*>(rho), g, c->mom_zc, c->mom_tx, c->mom_ty, c->mom_partial);
    else
        hipLaunchKernelGGL(k_moments_partial<S>, dim3(c->mom_blocks), blk, 0, c->stream, static_cast<const S*>(rho),
                           g, c->mom_zc, c->mom_tx, c->mom_ty, c->mom_partial);
    hipLaunchKernelGGL(k_moments_final, dim3(NQ), dim3(256), 0, c->stream, c->mom_partial, c->mom_blocks,
                       c->cfg.dx * c->cfg.dx * c->cfg.dx, c->mom);
    const int64_t nf = 2 * ((int64_t)c->L.nz * c->L.ny + (int64_t)c->L.nz * c->L.nx + (int64_t)c->L.ny * c->L.nx);
    const int maxfast = std::max(c->L.nx, c->L.ny), maxslow = std::max(c->L.ny, c->L.nz);
    S* b[4];
    int nb = 0;
    for (int k = 0; k < 4; ++k) b[k] = (mask >> k & 1) ? B<S>(c, k) : nullptr, nb += (mask >> k) & 1;
    hipLaunchKernelGGL(k_ghosts<S>, dim3((maxfast + 255) / 256, maxslow, 6), dim3(256), 0, c->stream, c->L, g,
                       c->cfg.lmax, c->cfg.G, c->mom, b[0], b[1], b[2], b[3]);
    tm.end((double)sizeof(S) * (double)c->L.nx * c->L.ny * c->L.nz + (double)nb * sizeof(S) * (double)nf, 0.0);
}


// Direct Poisson solve into the state: ghosts of buffer cur (MULTIPOLE: from
// the moments of rho, written into cur and old; USER: already there), the
// right-hand side, three sine transforms, the eigenvalue division, three
// inverse transforms, then phi^n = phi^{n-1} = the solution.
template <typename S>
void run_poisson_direct(hgs_ctx* c, const void* rho, double* scratch) {
    const Layout& L = c->L;
    if (c->cfg.bc == HGS_BC_MULTIPOLE) run_moments_and_ghosts<S>(c, rho, (1 << c->cur) | (1 << c->old));
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(65536, (n + 255) / 256));
    double* a = scratch;
    double* b = scratch + n;
    const double inv_dx2 = 1.0 / (c->cfg.dx * c->cfg.dx);
    hipLaunchKernelGGL(k_dst_rhs<S>, dim3(nb), dim3(256), 0, c->stream, static_cast<const S*>(rho), B<S>(c, c->cur),
                       L, 4.0 * M_PI * c->cfg.G, inv_dx2, a);
    hipLaunchKernelGGL(k_dst_axis, dim3(nb), dim3(256), 0, c->stream, a, b, L.nx, L.ny, L.nz, 0);
    hipLaunchKernelGGL(k_dst_axis, dim3(nb), dim3(256), 0, c->stream, b, a, L.nx, L.ny, L.nz, 1);
    hipLaunchKernelGGL(k_dst_axis, dim3(nb), dim3(256), 0, c->stream, a, b, L.nx, L.ny, L.nz, 2);
    const double norm = (2.0 / (L.nx + 1)) * (2.0 / (L.ny + 1)) * (2.0 / (L.nz + 1));
    hipLaunchKernelGGL(k_dst_scale, dim3(nb), dim3(256), 0, c->stream, b, L.nx, L.ny, L.nz, inv_dx2, norm);
    hipLaunchKernelGGL(k_dst_axis, dim3(nb), dim3(256), 0, c->stream, b, a, L.nx, L.ny, L.nz, 0);
    hipLaunchKernelGGL(k_dst_axis, dim3(nb), dim3(256), 0, c->stream, a, b, L.nx, L.ny, L.nz, 1);
    hipLaunchKernelGGL(k_dst_axis, dim3(nb), dim3(256), 0, c->stream, b, a, L.nx, L.ny, L.nz, 2);
    hipLaunchKernelGGL(k_dst_store<S>, dim3(nb), dim3(256), 0, c->stream, a, L, B<S>(c, c->cur), B<S>(c, c->old));
}

LocalGeom local_geom(const hgs_ctx* c) {
    return LocalGeom{c->cfg.x0, c->cfg.y0, c->cfg.z0, c->cfg.dx, c->cfg.origin[0], c->cfg.origin[1], c->cfg.origin[2]};
}

// Ghosts of buffer nxt from its interior: the periodic copy, else Robin's
// relation (the outgoing rule's steady form).
template <typename S>
void run_local_ghosts(hgs_ctx* c, int nxt) {
    const int maxfast = std::max(c->L.nx, c->L.ny), maxslow = std::max(c->L.ny, c->L.nz);
    hipLaunchKernelGGL(k_local_ghosts<S>, dim3((maxfast + 255) / 256, maxslow, 6), dim3(256), 0, c->stream, c->L,
                       local_geom(c), c->cfg.bc, B<S>(c, nxt));
}

// Domain-mean density into c->mean (FP64; fixed-order partial sums).
template <typename S>
void run_mean(hgs_ctx* c, const void* rho) {
    const int64_t n = (int64_t)c->cfg.nx * c->cfg.ny * c->cfg.nz;
    const int nb = grid_for(n, 256, kRedBlocks);
    hipLaunchKernelGGL(k_sum_partial<S>, dim3(nb), dim3(256), 0, c->stream, static_cast<const S*>(rho), n,
                       c->red_partial);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, c->stream, c->red_partial, nb, 1.0 / (double)n, c->mean);
}

template <typename S>
void run_substeps(hgs_ctx* c, const void* rho, const StepCoef& sc, int nsub, double c_dt) {
    const S* r = static_cast<const S*>(rho);
    const double* rbar = c->cfg.bc == HGS_BC_PERIODIC ? c->mean : nullptr;
    const int T = fused_depth(c);
    const int mode = c->cfg.bc == HGS_BC_ROBIN      ? TB_ROBIN
                     : c->cfg.bc == HGS_BC_PERIODIC ? TB_PERIODIC
                     : c->cfg.bc == HGS_BC_OUTGOING ? TB_OUTGOING
                                                    : TB_FROZEN;
    const TBBound bnd{mode, local_geom(c), c->mean, c_dt};
    while (nsub > 0) {
        if (T > 1 && nsub >= T) {
            // out of place: (cur, old) -> (the other two buffers)
            int o0 = -1, o1 = -1;
            for (int k = 0; k < 4; ++k)
                if (k != c->cur && k != c->old) {
                    if (o0 < 0)
                        o0 = k;
                    else
                        o1 = k;
                }
            Timed tm(c, HGS_KERNEL_STENCIL);
            launch_tblock<S>(B<S>(c, c->cur), B<S>(c, c->old), r, B<S>(c, o0), B<S>(c, o1), c->L, sc, T, c->tile, c->ncu,
                             c->stream, bnd);
            const double cells = (double)c->L.nx * c->L.ny * c->L.nz;
            tm.end(5.0 * sizeof(S) * cells, cells * T);
            // periodic ghosts of the new phi^n (a streaming substep after it
            // reads them; phi^{n-1}'s ghosts are never read: the next substep
            // writes its new level over them and sets them again); Robin
            // ghosts are set once at the end; the fused outgoing launch stores
            // its ghosts itself
            if (mode == TB_PERIODIC) run_local_ghosts<S>(c, o0);
            c->cur = o0;
            c->old = o1;
            nsub -= T;
        } else {
            int zc, tx, ty, nb;
            Timed tm(c, HGS_KERNEL_STENCIL);
            const LocalGeom lg = local_geom(c);
            const S* a = B<S>(c, c->cur);
            S* o = B<S>(c, c->old);
            if (use_vec<S>(c->L)) {
                stream_dims(c->L, 64 * Vec16<S>::N, zc, tx, ty, nb);
                if (mode == TB_ROBIN)
                    hipLaunchKernelGGL((k_leapfrog_stream_v<S, SBY, ST_ROBIN>), dim3(nb), dim3(64, SBY), 0, c->stream,
                                       a, o, r, c->L, sc, zc, tx, ty, rbar, lg, c_dt);
                else if (mode == TB_OUTGOING)
                    hipLaunchKernelGGL((k_leapfrog_stream_v<S, SBY, ST_OUTGOING>), dim3(nb), dim3(64, SBY), 0,
                                       c->stream, a, o, r, c->L, sc, zc, tx, ty, rbar, lg, c_dt);
                else if (mode == TB_PERIODIC)
                    hipLaunchKernelGGL((k_leapfrog_stream_v<S, SBY, ST_PERIODIC>), dim3(nb), dim3(64, SBY), 0,
                                       c->stream, a, o, r, c->L, sc, zc, tx, ty, rbar, lg, c_dt);
                else
                    hipLaunchKernelGGL((k_leapfrog_stream_v<S, SBY>), dim3(nb), dim3(64, SBY), 0, c->stream, a, o, r,
                                       c->L, sc, zc, tx, ty, rbar, lg, c_dt);
            } else {
                stream_dims(c->L, SBX, zc, tx, ty, nb);
                if (mode == TB_ROBIN)
                    hipLaunchKernelGGL((k_leapfrog_stream<S, SBX, SBY, ST_ROBIN>), dim3(nb), dim3(SBX, SBY), 0,
                                       c->stream, a, o, r, c->L, sc, zc, tx, ty, rbar, lg, c_dt);
                else if (mode == TB_OUTGOING)
                    hipLaunchKernelGGL((k_leapfrog_stream<S, SBX, SBY, ST_OUTGOING>), dim3(nb), dim3(SBX, SBY), 0,
                                       c->stream, a, o, r, c->L, sc, zc, tx, ty, rbar, lg, c_dt);
                else if (mode == TB_PERIODIC)
                    hipLaunchKernelGGL((k_leapfrog_stream<S, SBX, SBY, ST_PERIODIC>), dim3(nb), dim3(SBX, SBY), 0,
                                       c->stream, a, o, r, c->L, sc, zc, tx, ty, rbar, lg, c_dt);
                else
                    hipLaunchKernelGGL((k_leapfrog_stream<S, SBX, SBY>), dim3(nb), dim3(SBX, SBY), 0, c->stream, a, o,
                                       r, c->L, sc, zc, tx, ty, rbar, lg, c_dt);
            }
            const double cells = (double)c->L.nx * c->L.ny * c->L.nz;
            tm.end(4.0 * sizeof(S) * cells, cells);
            // no ghost launch: Robin substeps evaluate their ghosts where they
            // read them (set at the end), outgoing and periodic substeps store
            // the new level's ghosts themselves
            std::swap(c->cur, c->old);
            nsub -= 1;
        }
    }
    // Robin: the substeps evaluate their ghosts where they read them; phi^n's
    // ghost layer is set once, for the gradient, the residual and the faces
    if (mode == TB_ROBIN) run_local_ghosts<S>(c, c->cur);
}

// Gradient over the cells of layout W read from phi (W may be a box inside
// the grid: the same pitch and plane with a shifted base), compact outputs.
template <typename S>
void launch_gradient(hgs_ctx* c, const S* phi, const Layout& W, void* gx, void* gy, void* gz, bool vec) {
    int zc, tx, ty, nb;
    Timed tm(c, HGS_KERNEL_GRADIENT);
    if (vec) {
        stream_dims(W, 64 * Vec16<S>::N, zc, tx, ty, nb, GR * GBY);
        hipLaunchKernelGGL((k_gradient_v<S, GR, GBY>), dim3(nb), dim3(64, GBY), 0, c->stream, phi, W, 0.5 / c->cfg.dx, zc,
                           tx, ty, static_cast<S*>(gx), static_cast<S*>(gy), static_cast<S*>(gz));
    } else {
        stream_dims(W, SBX, zc, tx, ty, nb);
        hipLaunchKernelGGL((k_gradient<S, SBX, SBY>), dim3(nb), dim3(SBX, SBY), 0, c->stream, phi, W,
                           0.5 / c->cfg.dx, zc, tx, ty, static_cast<S*>(gx), static_cast<S*>(gy), static_cast<S*>(gz));
    }
    tm.end(4.0 * sizeof(S) * (double)W.nx * W.ny * W.nz, 0.0);
}

template <typename S>
void run_accel(hgs_ctx* c, void* gx, void* gy, void* gz) {
    launch_gradient<S>(c, B<S>(c, c->cur), c->L, gx, gy, gz, use_vec<S>(c->L));
}

// The box [i0, i0 + bx) x [j0, j0 + by) x [k0, k0 + bz) of the interior as a
// layout of its own: its cells are those of the grid, so the stencil reads
// the grid's neighbours (ghosts where the box touches a face).  16-byte lanes
// need the box to start and end on whole vectors along x.
template <typename S>
void run_accel_box(hgs_ctx* c, const int* box, void* gx, void* gy, void* gz) {
    Layout W = c->L;
    W.nx = box[3];
    W.ny = box[4];
    W.nz = box[5];
    const S* phi = B<S>(c, c->cur) + ((int64_t)box[2] * W.plane + (int64_t)box[1] * W.pitch + box[0]);
    const bool vec = box[0] % Vec16<S>::N == 0 && use_vec<S>(W);
    launch_gradient<S>(c, phi, W, gx, gy, gz, vec);
}

template <typename S>
void run_init(hgs_ctx* c) {
    for (int k = 0; k < 4; ++k)
        hipLaunchKernelGGL(k_init_buffer<S>, dim3(grid_for(c->L.total)), dim3(256), 0, c->stream, B<S>(c, k), c->L);
}

int64_t ncell(const hgs_ctx* c) { return (int64_t)c->cfg.nx * c->cfg.ny * c->cfg.nz; }
int64_t nface(const hgs_ctx* c) {
    return 2 * ((int64_t)c->L.nz * c->L.ny + (int64_t)c->L.nz * c->L.nx + (int64_t)c->L.ny * c->L.nx);
}

#define DISPATCH(c, fn, ...)                   \
    do {                                       \
        if ((c)->cfg.storage == HGS_F64)       \
            fn<double>(__VA_ARGS__);           \
        else                                   \
            fn<float>(__VA_ARGS__);            \
    } while (0)

template <typename S>
void run_potential(hgs_ctx* c, void* phi, void* phidot) {
    double inv = c->dt_prev > 0.0 ? 1.0 / c->dt_prev : 0.0;
    hipLaunchKernelGGL(k_potential<S>, dim3(grid_for(ncell(c))), dim3(256), 0, c->stream, B<S>(c, c->cur),
                       B<S>(c, c->old), inv, c->L, static_cast<S*>(phi), static_cast<S*>(phidot));
}

template <typename S>
void run_set_state(hgs_ctx* c, const void* phi, const void* phidot, double dt) {
    hipLaunchKernelGGL(k_set_state<S>, dim3(grid_for(ncell(c))), dim3(256), 0, c->stream, B<S>(c, c->cur),
                       B<S>(c, c->old), static_cast<const S*>(phi), static_cast<const S*>(phidot), dt, c->L);
    if (local_bc(c->cfg.bc)) {
        run_local_ghosts<S>(c, c->cur);
        run_local_ghosts<S>(c, c->old);
    }
}

template <typename S>
void run_rescale(hgs_ctx* c, double ratio) {
    hipLaunchKernelGGL(k_rescale<S>, dim3(grid_for(ncell(c))), dim3(256), 0, c->stream, B<S>(c, c->cur),
                       B<S>(c, c->old), ratio, c->L);
}

template <typename S>
void run_faces_in(hgs_ctx* c, const void* src) {
    hipLaunchKernelGGL(k_faces_in<S>, dim3(grid_for(nface(c))), dim3(256), 0, c->stream, static_cast<const S*>(src),
                       c->L, B<S>(c, 0), B<S>(c, 1), B<S>(c, 2), B<S>(c, 3));
}

template <typename S>
void run_faces_out(hgs_ctx* c, void* dst) {
    hipLaunchKernelGGL(k_faces_out<S>, dim3(grid_for(nface(c))), dim3(256), 0, c->stream, B<S>(c, c->cur), c->L,
                       static_cast<S*>(dst));
}

template <typename S>
void run_residual(hgs_ctx* c, const void* rho) {
    const double idx2 = 1.0 / (c->cfg.dx * c->cfg.dx);
    // 64 x 4 column tiles, z split so that the partials fit kRedBlocks slots
    const int tx = (c->L.nx + 63) / 64, ty = (c->L.ny + 3) / 4;
    const int cols = tx * ty;
    int zsplit = std::max(1, std::min(c->L.nz, kRedBlocks / std::max(1, cols)));
    int zc = (c->L.nz + zsplit - 1) / zsplit;
    int nb = cols * ((c->L.nz + zc - 1) / zc);
    if (nb > kRedBlocks) {  // very wide grids: one chunk per column tile is still too many
        zc = c->L.nz;
        nb = cols;
    }
    const double* rbar = nullptr;
    if (c->cfg.bc == HGS_BC_PERIODIC) {
        run_mean<S>(c, rho);
        rbar = c->mean;
    }
    hipLaunchKernelGGL(k_residual_partial<S>, dim3(nb), dim3(64, 4), 0, c->stream, B<S>(c, c->cur),
                       static_cast<const S*>(rho), c->L, idx2, 4.0 * M_PI * c->cfg.G, zc, tx, ty, rbar,
                       local_bc(c->cfg.bc) ? 0 : 1, c->red_partial);
    hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(256), 0, c->stream, c->red_partial, nb, c->red_out);
}

template <typename S>
void run_keep_or_zero(hgs_ctx* c, int32_t* kept) {
    hipLaunchKernelGGL(k_keep_or_zero<S>, dim3(grid_for(ncell(c))), dim3(256), 0, c->stream, c->red_out, c->L,
                       B<S>(c, c->cur), B<S>(c, c->old), kept);
}

template <typename S>
void run_raw_out(hgs_ctx* c, void* a, void* b) {
    hipLaunchKernelGGL(k_interior_out<S>, dim3(grid_for(ncell(c))), dim3(256), 0, c->stream, B<S>(c, c->cur), c->L,
                       static_cast<S*>(a));
    hipLaunchKernelGGL(k_interior_out<S>, dim3(grid_for(ncell(c))), dim3(256), 0, c->stream, B<S>(c, c->old), c->L,
                       static_cast<S*>(b));
}

template <typename S>
void run_raw_in(hgs_ctx* c, const void* a, const void* b) {
    hipLaunchKernelGGL(k_interior_in<S>, dim3(grid_for(ncell(c))), dim3(256), 0, c->stream,
                       static_cast<const S*>(a), c->L, B<S>(c, c->cur));
    hipLaunchKernelGGL(k_interior_in<S>, dim3(grid_for(ncell(c))), dim3(256), 0, c->stream,
                       static_cast<const S*>(b), c->L, B<S>(c, c->old));
    if (local_bc(c->cfg.bc)) {
        run_local_ghosts<S>(c, c->cur);
        run_local_ghosts<S>(c, c->old);
    }
}

// max over cells of c_s + |v| and a non-finite flag into red_out[0..1]
template <typename S>
void run_speed(hgs_ctx* c, const void* cs, const void* vx, const void* vy, const void* vz) {
    const int64_t n = ncell(c);
    const int nb = grid_for(n, 256, kRedBlocks);
    hipLaunchKernelGGL(k_speed_partial<S>, dim3(nb), dim3(256), 0, c->stream, static_cast<const S*>(cs),
                       static_cast<const S*>(vx), static_cast<const S*>(vy), static_cast<const S*>(vz), n,
                       c->red_partial);
    hipLaunchKernelGGL(k_speed_final, dim3(1), dim3(256), 0, c->stream, c->red_partial, nb, c->red_out);
}

// W = 1/2 sum rho phi dx^3 into red_out[0]
template <typename S>
void run_energy(hgs_ctx* c, const void* rho) {
    const int nb = grid_for(ncell(c), 256, kRedBlocks);
    hipLaunchKernelGGL(k_dot_partial<S>, dim3(nb), dim3(256), 0, c->stream, static_cast<const S*>(rho),
                       B<S>(c, c->cur), c->L, c->red_partial);
    const double dv = c->cfg.dx * c->cfg.dx * c->cfg.dx;
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, c->stream, c->red_partial, nb, 0.5 * dv, c->red_out);
}

hgs_status read_out(hgs_ctx* c, double* dst, int n, const char* what) {
    hipError_t e = hipMemcpyAsync(dst, c->red_out, n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(c, HGS_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return HGS_OK;
}

// Default fused depth: four substeps per launch (the usual substeps per hydro
// step); cfg->tblock or hgs_set_tblock override it.
int default_tblock(const hgs_config* cfg) { return cfg->tblock > 0 ? cfg->tblock : 4; }

}  // namespace

extern "C" {

int32_t hgs_abi_version(void) { return 2; }

const char* hgs_status_str(hgs_status s) {
    switch (s) {
        case HGS_OK: return "HGS_OK";
        case HGS_ERR_ARG: return "HGS_ERR_ARG";
        case HGS_ERR_CFL: return "HGS_ERR_CFL";
        case HGS_ERR_WORKSPACE: return "HGS_ERR_WORKSPACE";
        case HGS_ERR_DEVICE: return "HGS_ERR_DEVICE";
        case HGS_ERR_NONFINITE: return "HGS_ERR_NONFINITE";
        case HGS_ERR_STATE: return "HGS_ERR_STATE";
    }
    return "HGS_ERR_UNKNOWN";
}

const char* hgs_last_error(const hgs_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

hgs_status hgs_config_cube(hgs_config* cfg, int32_t n, double lo, double hi) {
    if (!cfg) return fail(nullptr, HGS_ERR_ARG, "cfg is NULL");
    if (n < 1 || n > kMaxN || !(hi > lo)) return fail(nullptr, HGS_ERR_ARG, "need 1 <= n <= 8192 and hi > lo");
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->nx = cfg->ny = cfg->nz = n;
    cfg->x0 = cfg->y0 = cfg->z0 = lo;
    cfg->dx = (hi - lo) / n;
    cfg->G = 1.0;
    cfg->lmax = HGS_LMAX;
    cfg->bc = HGS_BC_MULTIPOLE;
    cfg->storage = HGS_F32;
    cfg->tblock = 0;
    cfg->eta = 0.0;
    cfg->stream = nullptr;
    return HGS_OK;
}

hgs_status hgs_workspace_bytes(const hgs_config* cfg, size_t* bytes) {
    std::string why;
    hgs_status s = check_config(cfg, why);
    if (s != HGS_OK) return fail(nullptr, s, why);
    if (!bytes) return fail(nullptr, HGS_ERR_ARG, "bytes is NULL");
    *bytes = make_plan(cfg).total;
    return HGS_OK;
}

hgs_status hgs_init(const hgs_config* cfg, void* workspace, size_t bytes, hgs_ctx** out) {
    std::string why;
    hgs_status s = check_config(cfg, why);
    if (s != HGS_OK) return fail(nullptr, s, why);
    if (!out) return fail(nullptr, HGS_ERR_ARG, "out is NULL");
    Plan p = make_plan(cfg);
    if (!workspace) return fail(nullptr, HGS_ERR_WORKSPACE, "workspace is NULL");
    if (bytes < p.total) return fail(nullptr, HGS_ERR_WORKSPACE, "workspace smaller than hgs_workspace_bytes()");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(nullptr, HGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    hgs_ctx* c = new (std::nothrow) hgs_ctx();
    if (!c) return fail(nullptr, HGS_ERR_ARG, "out of host memory");
    c->cfg = *cfg;
    c->esize = cfg->storage == HGS_F64 ? 8 : 4;
    c->L = make_layout(cfg->nx, cfg->ny, cfg->nz, c->esize);
    c->stream = static_cast<hipStream_t>(cfg->stream);
    char* w = static_cast<char*>(workspace);
    for (int k = 0; k < 4; ++k) c->buf[k] = w + k * p.buf_bytes;
    c->cur = 0;
    c->old = 1;
    c->mom_partial = reinterpret_cast<double*>(w + p.mom_partial_off);
    c->mom = reinterpret_cast<double*>(w + p.mom_off);
    c->mom_blocks = p.mom_blocks;
    c->mom_zc = p.mom_zc;
    c->mom_tx = p.mom_tx;
    c->mom_ty = p.mom_ty;
    c->mom_vec = p.mom_vec;
    c->red_partial = reinterpret_cast<double*>(w + p.red_partial_off);
    c->red_out = reinterpret_cast<double*>(w + p.red_out_off);
    c->mean = reinterpret_cast<double*>(w + p.mean_off);
    c->red_blocks = kRedBlocks;
    c->dt_prev = 0.0;
    c->have_moments = false;
    c->tblock = default_tblock(cfg);
    c->tile = 0;
    c->timing = false;
    c->pool_used = 0;
    {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            c->ncu = n;
        else
            c->ncu = 256;
    }
    (void)hipGetLastError();
    DISPATCH(c, run_init, c);
    s = launch_check(c, "hgs_init");
    if (s != HGS_OK) {
        g_err = c->err;
        delete c;
        return s;
    }
    *out = c;
    return HGS_OK;
}

hgs_status hgs_destroy(hgs_ctx* ctx) {
    if (ctx) {
        if (!ctx->pool.empty()) (void)hipStreamSynchronize(ctx->stream);
        for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    }
    delete ctx;
    return HGS_OK;
}

hgs_status hgs_timing_enable(hgs_ctx* ctx, int32_t enable) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (enable) {
        // events in the pool may still be pending on the stream
        if (!ctx->pool.empty() && hipStreamSynchronize(ctx->stream) != hipSuccess)
            return fail(ctx, HGS_ERR_DEVICE, "hgs_timing_enable: stream synchronisation failed");
        ctx->recs.clear();
        ctx->pool_used = 0;
    }
    ctx->timing = enable != 0;
    return HGS_OK;
}

hgs_status hgs_timing_read(hgs_ctx* ctx, int32_t kind, double out[4]) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (!out || kind < 0 || kind > 2) return fail(ctx, HGS_ERR_ARG, "out must be non-NULL and kind in 0..2");
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(ctx, HGS_ERR_DEVICE, std::string("hgs_timing_read: ") + hipGetErrorString(e));
    double n = 0, ms = 0, bytes = 0, upd = 0;
    for (const auto& r : ctx->recs) {
        if (r.kind != kind) continue;
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return fail(ctx, HGS_ERR_DEVICE, "event timing failed");
        n += 1;
        ms += t;
        bytes += r.bytes;
        upd += r.updates;
    }
    out[0] = n;
    out[1] = ms;
    out[2] = bytes;
    out[3] = upd;
    return HGS_OK;
}

hgs_status hgs_set_tblock(hgs_ctx* ctx, int32_t tblock) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (tblock < 0 || tblock > HGS_TMAX) return fail(ctx, HGS_ERR_ARG, "tblock must be in 0..4");
    ctx->tblock = tblock == 0 ? 4 : tblock;
    return HGS_OK;
}

int32_t hgs_get_tblock(const hgs_ctx* ctx) { return ctx ? ctx->tblock : 0; }

int32_t hgs_tile_count(int32_t tblock) { return tblock >= 2 && tblock <= HGS_TMAX ? tile_count(tblock) : 0; }

hgs_status hgs_tile_shape(int32_t storage, int32_t tblock, int32_t tile, int32_t shape[3]) {
    if (!shape) return fail(nullptr, HGS_ERR_ARG, "shape is NULL");
    if (storage != HGS_F32 && storage != HGS_F64) return fail(nullptr, HGS_ERR_ARG, "storage must be HGS_F32 or HGS_F64");
    if (tblock < 2 || tblock > HGS_TMAX) return fail(nullptr, HGS_ERR_ARG, "tblock must be in 2..4");
    if (tile < 0 || tile >= tile_count(tblock)) return fail(nullptr, HGS_ERR_ARG, "no such tile for this depth");
    TileShape t{0, 0, 0};
    const bool f32 = storage == HGS_F32;
    switch (tblock) {
        case 2: t = f32 ? TileSet<float, 2>::at(tile) : TileSet<double, 2>::at(tile); break;
        case 3: t = f32 ? TileSet<float, 3>::at(tile) : TileSet<double, 3>::at(tile); break;
        default: t = f32 ? TileSet<float, 4>::at(tile) : TileSet<double, 4>::at(tile); break;
    }
    shape[0] = t.R;
    shape[1] = t.W;
    shape[2] = t.PF;
    return HGS_OK;
}

hgs_status hgs_set_tile(hgs_ctx* ctx, int32_t tile) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (tile < 0 || tile >= tile_count(HGS_TMAX)) return fail(ctx, HGS_ERR_ARG, "tile out of range");
    ctx->tile = tile;
    return HGS_OK;
}

int32_t hgs_get_tile(const hgs_ctx* ctx) { return ctx ? ctx->tile : 0; }

static hgs_status validate_step(hgs_ctx* ctx, const hgs_config* cfg, const void* rho, double c_g, double dt,
                                int32_t nsub) {
    if (!rho) return fail(ctx, HGS_ERR_ARG, "rho is NULL");
    if (nsub < 1) return fail(ctx, HGS_ERR_ARG, "nsub must be >= 1");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, HGS_ERR_ARG, "dt must be positive and finite");
    if (!(c_g > 0.0) || !std::isfinite(c_g)) return fail(ctx, HGS_ERR_ARG, "c_g must be positive and finite");
    const double courant = c_g * dt / cfg->dx;
    if (courant > 1.0 / std::sqrt(3.0)) {
        char m[160];
        std::snprintf(m, sizeof m, "c_g dt / dx = %.6g exceeds the 3D leapfrog limit 1/sqrt(3)", courant);
        return fail(ctx, HGS_ERR_CFL, m);
    }
    return HGS_OK;
}

hgs_status hgs_validate_step(const hgs_config* cfg, const void* rho, double c_g, double dt, int32_t nsub) {
    std::string why;
    hgs_status s = check_config(cfg, why);
    if (s != HGS_OK) return fail(nullptr, s, why);
    return validate_step(nullptr, cfg, rho, c_g, dt, nsub);
}

hgs_status hgs_step(hgs_ctx* ctx, const void* rho, double c_g, double dt, int32_t nsub) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    hgs_status vs = validate_step(ctx, &ctx->cfg, rho, c_g, dt, nsub);
    if (vs != HGS_OK) return vs;
    (void)hipGetLastError();
    if (ctx->cfg.bc == HGS_BC_MULTIPOLE) {
        DISPATCH(ctx, run_moments_and_ghosts, ctx, rho, ghost_buffers(ctx, nsub));
        ctx->have_moments = true;
    }
    if (ctx->cfg.bc == HGS_BC_PERIODIC) DISPATCH(ctx, run_mean, ctx, rho);
    if (ctx->dt_prev > 0.0 && dt != ctx->dt_prev) DISPATCH(ctx, run_rescale, ctx, dt / ctx->dt_prev);
    DISPATCH(ctx, run_substeps, ctx, rho, step_coef(ctx, c_g, dt), nsub, c_g * dt);
    ctx->dt_prev = dt;
    return launch_check(ctx, "hgs_step");
}

hgs_status hgs_multipole_boundary(hgs_ctx* ctx, const void* rho) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (!rho) return fail(ctx, HGS_ERR_ARG, "rho is NULL");
    if (ctx->cfg.bc != HGS_BC_MULTIPOLE)
        return fail(ctx, HGS_ERR_STATE, "hgs_multipole_boundary needs bc = HGS_BC_MULTIPOLE");
    (void)hipGetLastError();
    DISPATCH(ctx, run_moments_and_ghosts, ctx, rho, (1 << ctx->cur) | (1 << ctx->old));
    ctx->have_moments = true;
    return launch_check(ctx, "hgs_multipole_boundary");
}

hgs_status hgs_keep_start_if_better(hgs_ctx* ctx, const void* rho, int32_t* kept) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (!rho) return fail(ctx, HGS_ERR_ARG, "rho is NULL");
    if (local_bc(ctx->cfg.bc))
        return fail(ctx, HGS_ERR_STATE, "hgs_keep_start_if_better needs a Dirichlet boundary (MULTIPOLE or USER)");
    (void)hipGetLastError();
    if (ctx->cfg.bc == HGS_BC_MULTIPOLE) {
        DISPATCH(ctx, run_moments_and_ghosts, ctx, rho, (1 << ctx->cur) | (1 << ctx->old));
        ctx->have_moments = true;
    }
    DISPATCH(ctx, run_residual, ctx, rho);
    DISPATCH(ctx, run_keep_or_zero, ctx, kept);
    return launch_check(ctx, "hgs_keep_start_if_better");
}

hgs_status hgs_poisson_direct(hgs_ctx* ctx, const void* rho, void* scratch, size_t bytes) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (!rho) return fail(ctx, HGS_ERR_ARG, "rho is NULL");
    if (ctx->cfg.bc != HGS_BC_MULTIPOLE && ctx->cfg.bc != HGS_BC_USER)
        return fail(ctx, HGS_ERR_STATE, "hgs_poisson_direct needs a Dirichlet boundary (MULTIPOLE or USER)");
    const Layout& L = ctx->L;
    if (L.nx > DST_MAXN || L.ny > DST_MAXN || L.nz > DST_MAXN)
        return fail(ctx, HGS_ERR_ARG, "hgs_poisson_direct: at most 1024 cells per axis");
    const size_t need = 2 * sizeof(double) * (size_t)L.nx * L.ny * L.nz;
    if (!scratch || bytes < need || reinterpret_cast<uintptr_t>(scratch) % kAlign)
        return fail(ctx, HGS_ERR_WORKSPACE, "scratch must hold 2 nx ny nz doubles, 256-byte aligned");
    (void)hipGetLastError();
    DISPATCH(ctx, run_poisson_direct, ctx, rho, static_cast<double*>(scratch));
    if (ctx->cfg.bc == HGS_BC_MULTIPOLE) ctx->have_moments = true;
    return launch_check(ctx, "hgs_poisson_direct");
}

hgs_status hgs_potential(hgs_ctx* ctx, void* phi, void* phidot) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (!phi) return fail(ctx, HGS_ERR_ARG, "phi is NULL");
    (void)hipGetLastError();
    DISPATCH(ctx, run_potential, ctx, phi, phidot);
    return launch_check(ctx, "hgs_potential");
}

hgs_status hgs_accel(hgs_ctx* ctx, void* gx, void* gy, void* gz) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (!gx || !gy || !gz) return fail(ctx, HGS_ERR_ARG, "gx, gy and gz must be non-NULL");
    (void)hipGetLastError();
    DISPATCH(ctx, run_accel, ctx, gx, gy, gz);
    return launch_check(ctx, "hgs_accel");
}

hgs_status hgs_accel_box(hgs_ctx* ctx, int32_t i0, int32_t j0, int32_t k0, int32_t bx, int32_t by, int32_t bz,
                         void* gx, void* gy, void* gz) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (!gx || !gy || !gz) return fail(ctx, HGS_ERR_ARG, "gx, gy and gz must be non-NULL");
    const Layout& L = ctx->L;
    if (i0 < 0 || j0 < 0 || k0 < 0 || bx < 1 || by < 1 || bz < 1 || (int64_t)i0 + bx > L.nx ||
        (int64_t)j0 + by > L.ny || (int64_t)k0 + bz > L.nz)
        return fail(ctx, HGS_ERR_ARG, "the box must be non-empty and inside the interior");
    (void)hipGetLastError();
    const int box[6] = {i0, j0, k0, bx, by, bz};
    DISPATCH(ctx, run_accel_box, ctx, box, gx, gy, gz);
    return launch_check(ctx, "hgs_accel_box");
}

hgs_status hgs_set_state(hgs_ctx* ctx, const void* phi, const void* phidot, double dt) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (!phi) return fail(ctx, HGS_ERR_ARG, "phi is NULL");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, HGS_ERR_ARG, "dt must be positive and finite");
    (void)hipGetLastError();
    DISPATCH(ctx, run_set_state, ctx, phi, phidot, dt);
    ctx->dt_prev = dt;
    return launch_check(ctx, "hgs_set_state");
}

hgs_status hgs_set_boundary(hgs_ctx* ctx, const void* ghosts) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (ctx->cfg.bc != HGS_BC_USER && ctx->cfg.bc != HGS_BC_OUTGOING)
        return fail(ctx, HGS_ERR_STATE, "hgs_set_boundary needs bc = HGS_BC_USER or HGS_BC_OUTGOING");
    if (!ghosts) return fail(ctx, HGS_ERR_ARG, "ghosts is NULL");
    (void)hipGetLastError();
    DISPATCH(ctx, run_faces_in, ctx, ghosts);
    return launch_check(ctx, "hgs_set_boundary");
}

hgs_status hgs_get_boundary(hgs_ctx* ctx, void* ghosts) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (!ghosts) return fail(ctx, HGS_ERR_ARG, "ghosts is NULL");
    (void)hipGetLastError();
    DISPATCH(ctx, run_faces_out, ctx, ghosts);
    return launch_check(ctx, "hgs_get_boundary");
}

hgs_status hgs_moments(hgs_ctx* ctx, double* q_host) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (!q_host) return fail(ctx, HGS_ERR_ARG, "q_host is NULL");
    if (!ctx->have_moments) return fail(ctx, HGS_ERR_STATE, "no moments before the first multipole step");
    double ab[NQ];
    hipError_t e = hipMemcpyAsync(ab, ctx->mom, sizeof ab, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(ctx, HGS_ERR_DEVICE, std::string("hgs_moments: ") + hipGetErrorString(e));
    // A_lm + i B_lm = sum m r^l P_l^m e^{i m phi} (no Condon-Shortley phase).  With
    // Y_lm = N_lm (-1)^m P_l^m e^{i m phi}:  Q_lm = N_lm (-1)^m (A_lm - i B_lm), m >= 0,
    // and Q_{l,-m} = (-1)^m conj(Q_lm).
    const int lmax = ctx->cfg.lmax;
    for (int l = 0; l <= lmax; ++l) {
        for (int m = 0; m <= l; ++m) {
            double ratio = 1.0;
            for (int f = l - m + 1; f <= l + m; ++f) ratio /= (double)f;
            const double N = std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * ratio);
            const double sg = (m % 2) ? -1.0 : 1.0;
            const double A = ab[l * l + l + m];
            const double Bv = m > 0 ? ab[l * l + l - m] : 0.0;
            const double re = N * sg * A, im = -N * sg * Bv;
            q_host[2 * (l * l + l + m)] = re;
            q_host[2 * (l * l + l + m) + 1] = im;
            if (m > 0) {
                q_host[2 * (l * l + l - m)] = sg * re;
                q_host[2 * (l * l + l - m) + 1] = -sg * im;
            }
        }
    }
    return HGS_OK;
}

hgs_status hgs_residual(hgs_ctx* ctx, const void* rho, double out[4]) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (!rho || !out) return fail(ctx, HGS_ERR_ARG, "rho and out must be non-NULL");
    (void)hipGetLastError();
    DISPATCH(ctx, run_residual, ctx, rho);
    hgs_status s = launch_check(ctx, "hgs_residual");
    if (s != HGS_OK) return s;
    double r[NRED];
    hipError_t e = hipMemcpyAsync(r, ctx->red_out, sizeof r, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(ctx, HGS_ERR_DEVICE, std::string("hgs_residual: ") + hipGetErrorString(e));
    const double rn = std::sqrt(r[0]);
    out[0] = r[1] > 0.0 ? rn / std::sqrt(r[1]) : (rn == 0.0 ? 0.0 : INFINITY);
    out[1] = r[2] > 0.0 ? rn / std::sqrt(r[2]) : (rn == 0.0 ? 0.0 : INFINITY);
    out[2] = std::sqrt(r[3]);
    out[3] = r[4] > 0.0 ? 1.0 : 0.0;
    if (out[3] != 0.0) return fail(ctx, HGS_ERR_NONFINITE, "phi or rho holds a non-finite value");
    return HGS_OK;
}

hgs_status hgs_max_signal_speed(hgs_ctx* ctx, const void* cs, const void* vx, const void* vy, const void* vz,
                                double* vmax) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (!cs || !vmax) return fail(ctx, HGS_ERR_ARG, "cs and vmax must be non-NULL");
    (void)hipGetLastError();
    DISPATCH(ctx, run_speed, ctx, cs, vx, vy, vz);
    hgs_status s = launch_check(ctx, "hgs_max_signal_speed");
    if (s != HGS_OK) return s;
    double r[2];
    s = read_out(ctx, r, 2, "hgs_max_signal_speed");
    if (s != HGS_OK) return s;
    *vmax = r[0];
    if (r[1] != 0.0) return fail(ctx, HGS_ERR_NONFINITE, "c_s or v holds a non-finite value");
    return HGS_OK;
}

hgs_status hgs_hydro_step(hgs_ctx* ctx, const void* rho, const void* cs, const void* vx, const void* vy,
                          const void* vz, double k_g, double courant_hydro, double courant_grav, double* dt_hydro,
                          int32_t* nsub, double* c_g) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (!rho || !cs || !dt_hydro || !nsub || !c_g)
        return fail(ctx, HGS_ERR_ARG, "rho, cs, dt_hydro, nsub and c_g must be non-NULL");
    if (!(k_g >= 1.0) || !std::isfinite(k_g)) return fail(ctx, HGS_ERR_ARG, "k_g must be >= 1 and finite");
    if (!(courant_hydro > 0.0) || !std::isfinite(courant_hydro))
        return fail(ctx, HGS_ERR_ARG, "courant_hydro must be positive and finite");
    if (!(courant_grav > 0.0) || courant_grav > 1.0 / std::sqrt(3.0))
        return fail(ctx, HGS_ERR_ARG, "courant_grav must be in (0, 1/sqrt(3)]");
    double vmax = 0.0;
    hgs_status s = hgs_max_signal_speed(ctx, cs, vx, vy, vz, &vmax);
    if (s != HGS_OK) return s;
    if (!(vmax > 0.0)) return fail(ctx, HGS_ERR_ARG, "the largest signal speed c_s + |v| is zero");
    const double dth = courant_hydro * ctx->cfg.dx / vmax;
    const double cg = k_g * vmax;
    // the wave step must satisfy c_g dt / dx <= courant_grav
    const double need = k_g * courant_hydro / courant_grav;
    if (need > 1.0e6) return fail(ctx, HGS_ERR_ARG, "more than 1e6 substeps per hydrodynamical step");
    int n = (int)std::ceil(need * (1.0 - 1e-12));
    if (n < 1) n = 1;
    s = hgs_step(ctx, rho, cg, dth / n, n);
    if (s != HGS_OK) return s;
    *dt_hydro = dth;
    *nsub = n;
    *c_g = cg;
    return HGS_OK;
}

hgs_status hgs_energy(hgs_ctx* ctx, const void* rho, double* w) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (!rho || !w) return fail(ctx, HGS_ERR_ARG, "rho and w must be non-NULL");
    (void)hipGetLastError();
    DISPATCH(ctx, run_energy, ctx, rho);
    hgs_status s = launch_check(ctx, "hgs_energy");
    if (s != HGS_OK) return s;
    return read_out(ctx, w, 1, "hgs_energy");
}

static hgs_status ext_check(const void* a, const void* b, int32_t nx, int32_t ny, int32_t nz, int32_t ext,
                            int32_t dtype) {
    if (!a || !b) return fail(nullptr, HGS_ERR_ARG, "field pointers must be non-NULL");
    if (nx < 1 || ny < 1 || nz < 1 || ext < 0 || nx > kMaxN || ny > kMaxN || nz > kMaxN || ext > kMaxN)
        return fail(nullptr, HGS_ERR_ARG, "need 1 <= nx, ny, nz <= 8192 and 0 <= ext <= 8192");
    if ((int64_t)nx + 2 * (int64_t)ext > kMaxN || (int64_t)ny + 2 * (int64_t)ext > kMaxN ||
        (int64_t)nz + 2 * (int64_t)ext > kMaxN)
        return fail(nullptr, HGS_ERR_ARG, "extended grid larger than 8192 cells along an axis");
    if (dtype != HGS_F32 && dtype != HGS_F64) return fail(nullptr, HGS_ERR_ARG, "dtype must be HGS_F32 or HGS_F64");
    return HGS_OK;
}

hgs_status hgs_embed(const void* inner, int32_t nx, int32_t ny, int32_t nz, int32_t ext, void* outer, int32_t dtype,
                     void* stream) {
    hgs_status s = ext_check(inner, outer, nx, ny, nz, ext, dtype);
    if (s != HGS_OK) return s;
    (void)hipGetLastError();
    // one wave per outer row, four rows per workgroup
    const dim3 grid((ny + 2 * ext + 3) / 4, nz + 2 * ext);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (dtype == HGS_F32)
        hipLaunchKernelGGL(k_embed<float>, grid, dim3(64, 4), 0, st, static_cast<const float*>(inner), nx, ny, nz,
                           ext, static_cast<float*>(outer));
    else
        hipLaunchKernelGGL(k_embed<double>, grid, dim3(64, 4), 0, st, static_cast<const double*>(inner), nx, ny, nz,
                           ext, static_cast<double*>(outer));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? HGS_OK : fail(nullptr, HGS_ERR_DEVICE, std::string("hgs_embed: ") + hipGetErrorString(e));
}

hgs_status hgs_extract(const void* outer, int32_t nx, int32_t ny, int32_t nz, int32_t ext, void* inner, int32_t dtype,
                       void* stream) {
    hgs_status s = ext_check(outer, inner, nx, ny, nz, ext, dtype);
    if (s != HGS_OK) return s;
    (void)hipGetLastError();
    // one wave per inner row, four rows per workgroup
    const dim3 grid((ny + 3) / 4, nz);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (dtype == HGS_F32)
        hipLaunchKernelGGL(k_extract<float>, grid, dim3(64, 4), 0, st, static_cast<const float*>(outer), nx, ny, nz,
                           ext, static_cast<float*>(inner));
    else
        hipLaunchKernelGGL(k_extract<double>, grid, dim3(64, 4), 0, st, static_cast<const double*>(outer), nx, ny,
                           nz, ext, static_cast<double*>(inner));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? HGS_OK
                           : fail(nullptr, HGS_ERR_DEVICE, std::string("hgs_extract: ") + hipGetErrorString(e));
}

hgs_status hgs_nest_source(const void* rho, int32_t nx, int32_t ny, int32_t nz, int32_t ext, void* coarse,
                           int32_t dtype, void* stream) {
    if (!rho || !coarse) return fail(nullptr, HGS_ERR_ARG, "rho and coarse must be non-NULL");
    if (nx < 2 || ny < 2 || nz < 2 || nx % 2 || ny % 2 || nz % 2 || nx > kMaxN || ny > kMaxN || nz > kMaxN)
        return fail(nullptr, HGS_ERR_ARG, "need even nx, ny, nz in 2..8192");
    if (ext < 0 || ext > kMaxN || nx / 2 + 2 * (int64_t)ext > kMaxN || ny / 2 + 2 * (int64_t)ext > kMaxN ||
        nz / 2 + 2 * (int64_t)ext > kMaxN)
        return fail(nullptr, HGS_ERR_ARG, "need ext >= 0 and a coarse grid of at most 8192 cells along an axis");
    if (dtype != HGS_F32 && dtype != HGS_F64) return fail(nullptr, HGS_ERR_ARG, "dtype must be HGS_F32 or HGS_F64");
    (void)hipGetLastError();
    // one wave per coarse row, four rows per workgroup
    const dim3 grid((ny / 2 + 2 * ext + 3) / 4, nz / 2 + 2 * ext);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (dtype == HGS_F32)
        hipLaunchKernelGGL(k_nest_source<float>, grid, dim3(64, 4), 0, st, static_cast<const float*>(rho), nx, ny, nz,
                           ext, static_cast<float*>(coarse));
    else
        hipLaunchKernelGGL(k_nest_source<double>, grid, dim3(64, 4), 0, st, static_cast<const double*>(rho), nx, ny,
                           nz, ext, static_cast<double*>(coarse));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? HGS_OK
                           : fail(nullptr, HGS_ERR_DEVICE, std::string("hgs_nest_source: ") + hipGetErrorString(e));
}

hgs_status hgs_nest_ghosts(const void* coarse_phi, int32_t mx, int32_t my, int32_t mz, const double* coarse_x0,
                           double coarse_dx, int32_t nx, int32_t ny, int32_t nz, const double* fine_x0,
                           double fine_dx, void* faces, int32_t dtype, void* stream) {
    if (!coarse_phi || !coarse_x0 || !fine_x0 || !faces)
        return fail(nullptr, HGS_ERR_ARG, "coarse_phi, coarse_x0, fine_x0 and faces must be non-NULL");
    if (mx < 2 || my < 2 || mz < 2 || mx > kMaxN || my > kMaxN || mz > kMaxN || nx < 1 || ny < 1 || nz < 1 ||
        nx > kMaxN || ny > kMaxN || nz > kMaxN)
        return fail(nullptr, HGS_ERR_ARG, "need coarse sizes in 2..8192 and fine sizes in 1..8192");
    if (!(coarse_dx > 0.0) || !std::isfinite(coarse_dx) || !(fine_dx > 0.0) || !std::isfinite(fine_dx))
        return fail(nullptr, HGS_ERR_ARG, "cell sizes must be positive and finite");
    if (dtype != HGS_F32 && dtype != HGS_F64) return fail(nullptr, HGS_ERR_ARG, "dtype must be HGS_F32 or HGS_F64");
    const int m[3] = {mx, my, mz}, n[3] = {nx, ny, nz};
    for (int d = 0; d < 3; ++d) {
        if (!std::isfinite(coarse_x0[d]) || !std::isfinite(fine_x0[d]))
            return fail(nullptr, HGS_ERR_ARG, "corners must be finite");
        // the outermost ghost centres against the outermost coarse centres
        const double lo = fine_x0[d] - 0.5 * fine_dx, hi = fine_x0[d] + (n[d] + 0.5) * fine_dx;
        const double clo = coarse_x0[d] + 0.5 * coarse_dx, chi = coarse_x0[d] + (m[d] - 0.5) * coarse_dx;
        const double tol = 1e-9 * coarse_dx;
        if (lo < clo - tol || hi > chi + tol)
            return fail(nullptr, HGS_ERR_ARG, "the fine ghost centres must lie within the span of the coarse centres");
    }
    (void)hipGetLastError();
    const NestGeom g{mx, my, mz, coarse_x0[0], coarse_x0[1], coarse_x0[2], coarse_dx,
                     nx, ny, nz, fine_x0[0],   fine_x0[1],   fine_x0[2],   fine_dx};
    const dim3 grid((std::max(nx, ny) + 255) / 256, std::max(ny, nz), 6);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (dtype == HGS_F32)
        hipLaunchKernelGGL(k_nest_ghosts<float>, grid, dim3(256), 0, st, static_cast<const float*>(coarse_phi), g,
                           static_cast<float*>(faces));
    else
        hipLaunchKernelGGL(k_nest_ghosts<double>, grid, dim3(256), 0, st, static_cast<const double*>(coarse_phi), g,
                           static_cast<double*>(faces));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? HGS_OK
                           : fail(nullptr, HGS_ERR_DEVICE, std::string("hgs_nest_ghosts: ") + hipGetErrorString(e));
}

hgs_status hgs_save_raw(hgs_ctx* ctx, void* phi_n, void* phi_nm1, double* dt_prev) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (!phi_n || !phi_nm1 || !dt_prev) return fail(ctx, HGS_ERR_ARG, "phi_n, phi_nm1 and dt_prev must be non-NULL");
    (void)hipGetLastError();
    DISPATCH(ctx, run_raw_out, ctx, phi_n, phi_nm1);
    *dt_prev = ctx->dt_prev;
    return launch_check(ctx, "hgs_save_raw");
}

hgs_status hgs_load_raw(hgs_ctx* ctx, const void* phi_n, const void* phi_nm1, double dt_prev) {
    if (!ctx) return fail(nullptr, HGS_ERR_ARG, "ctx is NULL");
    if (!phi_n || !phi_nm1) return fail(ctx, HGS_ERR_ARG, "phi_n and phi_nm1 must be non-NULL");
    if (!(dt_prev >= 0.0) || !std::isfinite(dt_prev)) return fail(ctx, HGS_ERR_ARG, "dt_prev must be >= 0");
    (void)hipGetLastError();
    DISPATCH(ctx, run_raw_in, ctx, phi_n, phi_nm1);
    ctx->dt_prev = dt_prev;
    return launch_check(ctx, "hgs_load_raw");
}

}  // extern "C"

// ============================================================================
// Batched form
// ============================================================================

struct hgs_batch {
    int n;
    hgs_dtype storage;
    int tblock;
    hipStream_t stream;
    std::vector<hgs_ctx*> grids;
    void* desc_dev;     // GridDesc<S>[n]
    WorkItem* tb_items;   // fused items in cost order (persistent launch)
    int n_tb_items;
    WorkItem* tbg_items;  // fused items in grid order (one workgroup per item)
    int n_tbg_items;
    int launch;           // hgs_batch_launch
    WorkItem* st_items;
    int n_st_items;
    // host staging of the descriptors, double-buffered: buffer k is refilled
    // only after the event recorded behind its previous upload has passed
    std::vector<unsigned char> desc_host[2];
    hipEvent_t desc_done[2];
    bool desc_pending[2];
    int desc_k;
    hipStream_t capture;  // stream used only to record graphs
    std::map<std::tuple<int, int, int, int, int>, hipGraphExec_t> graphs;  // (nsub, T, cur, old, launch)
    bool graph_ok;
    bool used_graph;
    std::string err;
};

namespace {

thread_local std::string g_batch_err;

hgs_status bfail(hgs_batch* b, hgs_status s, const std::string& m) {
    if (b)
        b->err = m;
    else
        g_err = m;
    return s;
}

struct BatchPlan {
    std::vector<size_t> grid_off, grid_bytes;
    size_t desc_off, tb_off, tbg_off, st_off, total;
    std::vector<WorkItem> tb_items, tbg_items, st_items;
};

// Fused items of every grid in grid order -- per grid z chunks, then tile
// rows, then tiles (x fastest), the order of a single-grid launch -- for the
// launch with one workgroup per item.
template <typename S>
void batch_grid_items(const std::vector<Layout>& Ls, int T, int zchunk, std::vector<WorkItem>& tb) {
    tb.clear();
    if (T < 2) return;
    for (int g = 0; g < (int)Ls.size(); ++g) {
        const Layout& L = Ls[g];
        int IY = 0;
        switch (T) {
            case 2: IY = BatchTile<S, 2>::W * BatchTile<S, 2>::R - 4; break;
            case 3: IY = BatchTile<S, 3>::W * BatchTile<S, 3>::R - 6; break;
            default: IY = BatchTile<S, 4>::W * BatchTile<S, 4>::R - 8; break;
        }
        const int IX = 64 - 2 * T;
        const int tx = (L.nx + IX - 1) / IX, ty = (L.ny + IY - 1) / IY;
        const int zc = std::min(L.nz, zchunk);
        for (int z = 0; z < L.nz; z += zc)
            for (int y = 0; y < ty; ++y)
                for (int x = 0; x < tx; ++x) tb.push_back(WorkItem{g, x, y, z, std::min(L.nz, z + zc)});
    }
}

// z-chunk of the grid-ordered items: the hardware hands items to free CUs, so
// the launch takes about (total pipeline steps) / slots plus the longest item;
// pick the chunk that minimises that.
template <typename S>
int batch_grid_zchunk(const std::vector<Layout>& Ls, int T, int slots) {
    static const int cand[] = {128, 96, 64, 48, 32, 24, 16, 12, 8};
    int best = 64;
    double best_cost = -1.0;
    std::vector<WorkItem> tb;
    for (int zc : cand) {
        if (zc < 2 * T) continue;
        batch_grid_items<S>(Ls, T, zc, tb);
        int64_t total = 0, longest = 0;
        for (const WorkItem& w : tb) {
            total += w.k1 - w.k0 + 2 * T;
            longest = std::max<int64_t>(longest, w.k1 - w.k0 + 2 * T);
        }
        const double cost = (double)total / slots + (double)longest;
        if (best_cost < 0.0 || cost < best_cost) {
            best_cost = cost;
            best = zc;
        }
    }
    return best;
}

template <typename S>
void batch_items(const std::vector<Layout>& Ls, int T, int zchunk, std::vector<WorkItem>& tb,
                 std::vector<WorkItem>& st) {
    tb.clear();
    st.clear();
    std::vector<std::pair<int64_t, WorkItem>> a, b;
    for (int g = 0; g < (int)Ls.size(); ++g) {
        const Layout& L = Ls[g];
        if (T > 1) {
            int IX = 64 - 2 * T, IY = 0;
            switch (T) {
                case 2: IY = BatchTile<S, 2>::W * BatchTile<S, 2>::R - 4; break;
                case 3: IY = BatchTile<S, 3>::W * BatchTile<S, 3>::R - 6; break;
                default: IY = BatchTile<S, 4>::W * BatchTile<S, 4>::R - 8; break;
            }
            const int tx = (L.nx + IX - 1) / IX, ty = (L.ny + IY - 1) / IY;
            const int zc = std::min(L.nz, zchunk);
            for (int z = 0; z < L.nz; z += zc)
                for (int y = 0; y < ty; ++y)
                    for (int x = 0; x < tx; ++x) {
                        WorkItem w{g, x, y, z, std::min(L.nz, z + zc)};
                        a.push_back({(int64_t)(w.k1 - w.k0 + 2 * T), w});
                    }
        }
        const int N = 16 / (int)sizeof(S);
        const int tx = (L.nx + 64 * N - 1) / (64 * N), ty = (L.ny + 3) / 4;
        const int zc = std::min(L.nz, 32);
        for (int z = 0; z < L.nz; z += zc)
            for (int y = 0; y < ty; ++y)
                for (int x = 0; x < tx; ++x) {
                    WorkItem w{g, x, y, z, std::min(L.nz, z + zc)};
                    const int wx = std::min(64 * N, L.nx - x * 64 * N);
                    b.push_back({(int64_t)wx * (w.k1 - w.k0), w});
                }
    }
    auto by_cost = [](const std::pair<int64_t, WorkItem>& p, const std::pair<int64_t, WorkItem>& q) {
        return p.first > q.first;
    };
    std::stable_sort(a.begin(), a.end(), by_cost);
    std::stable_sort(b.begin(), b.end(), by_cost);
    for (auto& p : a) tb.push_back(p.second);
    for (auto& p : b) st.push_back(p.second);
}

// z-chunk of the fused work items: each item costs (chunk + 2T) pipeline
// steps; the launch's min(items, slots) workgroups take items in cost order,
// strided.  Pick the chunk whose busiest workgroup has the fewest steps (ties
// to the longer chunk, which recomputes fewer halo planes).  Small batches
// then split z finely instead of leaving most CUs idle.
template <typename S>
int batch_zchunk(const std::vector<Layout>& Ls, int T, int slots) {
    static const int cand[] = {64, 48, 32, 24, 16, 12, 8, 6, 4};
    int best = 64;
    int64_t best_span = -1;
    std::vector<WorkItem> tb, st;
    for (int zc : cand) {
        if (zc < 2 * T) continue;  // as the single-grid launcher: at least 2T planes per chunk
        batch_items<S>(Ls, T, zc, tb, st);
        const int nb = std::max(1, std::min((int)tb.size(), slots));
        std::vector<int64_t> load(nb, 0);
        for (size_t j = 0; j < tb.size(); ++j) load[j % nb] += tb[j].k1 - tb[j].k0 + 2 * T;
        const int64_t span = *std::max_element(load.begin(), load.end());
        if (best_span < 0 || span < best_span) {
            best_span = span;
            best = zc;
        }
    }
    return best;
}

// workgroup slots the batch planner assumes (one fused workgroup per CU of
// an MI355X); planning runs on the host, also without a device
constexpr int kPlanSlots = 256;

hgs_status batch_plan(const hgs_config* cfgs, int32_t n, BatchPlan& p, std::string& why) {
    if (!cfgs || n < 1 || n > 4096) {
        why = "need 1 <= n <= 4096 configurations";
        return HGS_ERR_ARG;
    }
    std::vector<Layout> Ls;
    for (int i = 0; i < n; ++i) {
        hgs_status s = check_config(&cfgs[i], why);
        if (s != HGS_OK) {
            why = "grid " + std::to_string(i) + ": " + why;
            return s;
        }
        if (local_bc(cfgs[i].bc)) {
            why = "grid " + std::to_string(i) + ": batched grids need a boundary frozen over the step (multipole or user)";
            return HGS_ERR_ARG;
        }
        if (cfgs[i].storage != cfgs[0].storage || cfgs[i].stream != cfgs[0].stream ||
            cfgs[i].tblock != cfgs[0].tblock) {
            why = "all grids of a batch share storage, stream and tblock";
            return HGS_ERR_ARG;
        }
        const int vec = cfgs[i].storage == HGS_F64 ? 2 : 4;
        if (cfgs[i].nx % vec) {
            why = "grid " + std::to_string(i) + ": nx must be a multiple of " + std::to_string(vec) + " in a batch";
            return HGS_ERR_ARG;
        }
        Ls.push_back(make_layout(cfgs[i].nx, cfgs[i].ny, cfgs[i].nz, cfgs[i].storage == HGS_F64 ? 8 : 4));
    }
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        size_t b = make_plan(&cfgs[i]).total;
        p.grid_off.push_back(off);
        p.grid_bytes.push_back(b);
        off = align_up(off + b, kAlign);
    }
    const int T = default_tblock(&cfgs[0]);
    if (cfgs[0].storage == HGS_F64) {
        batch_items<double>(Ls, T, batch_zchunk<double>(Ls, T, kPlanSlots), p.tb_items, p.st_items);
        batch_grid_items<double>(Ls, T, batch_grid_zchunk<double>(Ls, T, kPlanSlots), p.tbg_items);
    } else {
        batch_items<float>(Ls, T, batch_zchunk<float>(Ls, T, kPlanSlots), p.tb_items, p.st_items);
        batch_grid_items<float>(Ls, T, batch_grid_zchunk<float>(Ls, T, kPlanSlots), p.tbg_items);
    }
    const size_t dsz = cfgs[0].storage == HGS_F64 ? sizeof(GridDesc<double>) : sizeof(GridDesc<float>);
    p.desc_off = off;
    off = align_up(off + dsz * n, kAlign);
    p.tb_off = off;
    off = align_up(off + sizeof(WorkItem) * std::max<size_t>(1, p.tb_items.size()), kAlign);
    p.tbg_off = off;
    off = align_up(off + sizeof(WorkItem) * std::max<size_t>(1, p.tbg_items.size()), kAlign);
    p.st_off = off;
    off = align_up(off + sizeof(WorkItem) * std::max<size_t>(1, p.st_items.size()), kAlign);
    p.total = off;
    return HGS_OK;
}

template <typename S>
void batch_fill_desc(hgs_batch* b, std::vector<unsigned char>& host, const void* const* rho, const double* c_g,
                     const double* dt) {
    host.resize(sizeof(GridDesc<S>) * b->n);
    GridDesc<S>* d = reinterpret_cast<GridDesc<S>*>(host.data());
    for (int i = 0; i < b->n; ++i) {
        hgs_ctx* c = b->grids[i];
        d[i].L = c->L;
        d[i].c = step_coef(c, c_g[i], dt[i]);
        for (int k = 0; k < 4; ++k) d[i].buf[k] = static_cast<S*>(c->buf[k]);
        d[i].rho = static_cast<const S*>(rho[i]);
    }
}

// The launches of nsub substeps for all grids, starting from buffers (cur, old).
template <typename S>
void batch_launches(hgs_batch* b, int nsub, int cur, int old, hipStream_t st) {
    const GridDesc<S>* d = static_cast<const GridDesc<S>*>(b->desc_dev);
    const int ncu = b->grids[0]->ncu;
    const int T = b->tblock;
    while (nsub > 0) {
        if (T > 1 && nsub >= T) {
            int o0 = -1, o1 = -1;
            for (int k = 0; k < 4; ++k)
                if (k != cur && k != old) {
                    if (o0 < 0)
                        o0 = k;
                    else
                        o1 = k;
                }
            const int nb = std::min(b->n_tb_items, ncu);
            if (b->launch == HGS_BATCH_PER_ITEM) {
                const dim3 g((unsigned)b->n_tbg_items);
                switch (T) {
                    case 2:
                        hipLaunchKernelGGL((k_tblock_batch_items<S, 2, BatchTile<S, 2>::R, BatchTile<S, 2>::W,
                                                                 BatchTile<S, 2>::PF, BatchTile<S, 2>::SB,
                                                                 BatchTile<S, 2>::UPF>),
                                           g, dim3(64 * BatchTile<S, 2>::W), 0, st, d, b->tbg_items, cur, old, o0, o1);
                        break;
                    case 3:
                        hipLaunchKernelGGL((k_tblock_batch_items<S, 3, BatchTile<S, 3>::R, BatchTile<S, 3>::W,
                                                                 BatchTile<S, 3>::PF, BatchTile<S, 3>::SB,
                                                                 BatchTile<S, 3>::UPF>),
                                           g, dim3(64 * BatchTile<S, 3>::W), 0, st, d, b->tbg_items, cur, old, o0, o1);
                        break;
                    default:
                        hipLaunchKernelGGL((k_tblock_batch_items<S, 4, BatchTile<S, 4>::R, BatchTile<S, 4>::W,
                                                                 BatchTile<S, 4>::PF, BatchTile<S, 4>::SB,
                                                                 BatchTile<S, 4>::UPF>),
                                           g, dim3(64 * BatchTile<S, 4>::W), 0, st, d, b->tbg_items, cur, old, o0, o1);
                        break;
                }
                cur = o0;
                old = o1;
                nsub -= T;
                continue;
            }
            switch (T) {
                case 2:
                    hipLaunchKernelGGL((k_tblock_batch<S, 2, BatchTile<S, 2>::R, BatchTile<S, 2>::W, BatchTile<S, 2>::PF,
                                                        BatchTile<S, 2>::SB, BatchTile<S, 2>::UPF>),
                                       dim3(nb), dim3(64 * BatchTile<S, 2>::W), 0, st, d, b->tb_items, b->n_tb_items, cur, old,
                                       o0, o1);
                    break;
                case 3:
                    hipLaunchKernelGGL((k_tblock_batch<S, 3, BatchTile<S, 3>::R, BatchTile<S, 3>::W, BatchTile<S, 3>::PF,
                                                        BatchTile<S, 3>::SB, BatchTile<S, 3>::UPF>),
                                       dim3(nb), dim3(64 * BatchTile<S, 3>::W), 0, st, d, b->tb_items, b->n_tb_items, cur, old,
                                       o0, o1);
                    break;
                default:
                    hipLaunchKernelGGL((k_tblock_batch<S, 4, BatchTile<S, 4>::R, BatchTile<S, 4>::W, BatchTile<S, 4>::PF,
                                                        BatchTile<S, 4>::SB, BatchTile<S, 4>::UPF>),
                                       dim3(nb), dim3(64 * BatchTile<S, 4>::W), 0, st, d, b->tb_items, b->n_tb_items, cur, old,
                                       o0, o1);
                    break;
            }
            cur = o0;
            old = o1;
            nsub -= T;
        } else {
            const int nb = std::min(b->n_st_items, ncu * 8);
            hipLaunchKernelGGL((k_stream_batch<S, SBY>), dim3(nb), dim3(64, SBY), 0, st, d, b->st_items,
                               b->n_st_items, cur, old);
            std::swap(cur, old);
            nsub -= 1;
        }
    }
}

// buffer roles after nsub substeps from (cur, old)
void batch_roles(int T, int nsub, int& cur, int& old) {
    while (nsub > 0) {
        if (T > 1 && nsub >= T) {
            int o0 = -1, o1 = -1;
            for (int k = 0; k < 4; ++k)
                if (k != cur && k != old) {
                    if (o0 < 0)
                        o0 = k;
                    else
                        o1 = k;
                }
            cur = o0;
            old = o1;
            nsub -= T;
        } else {
            std::swap(cur, old);
            nsub -= 1;
        }
    }
}

template <typename S>
hgs_status batch_run(hgs_batch* b, int nsub) {
    const int cur = b->grids[0]->cur, old = b->grids[0]->old;
    b->used_graph = false;
    if (b->graph_ok) {
        auto key = std::make_tuple(nsub, b->tblock, cur, old, b->launch);
        auto it = b->graphs.find(key);
        hipGraphExec_t exec = nullptr;
        if (it != b->graphs.end()) {
            exec = it->second;
        } else {
            hipGraph_t graph = nullptr;
            bool ok = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                batch_launches<S>(b, nsub, cur, old, b->capture);
                ok = hipStreamEndCapture(b->capture, &graph) == hipSuccess && graph;
            }
            if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
            if (ok) {
                b->graphs[key] = exec;
            } else {
                exec = nullptr;
                b->graph_ok = false;  // capture unsupported here: launch directly from now on
            }
        }
        if (exec) {
            if (hipGraphLaunch(exec, b->stream) != hipSuccess) return bfail(b, HGS_ERR_DEVICE, "hipGraphLaunch failed");
            b->used_graph = true;
        }
    }
    if (!b->used_graph) batch_launches<S>(b, nsub, cur, old, b->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(b, HGS_ERR_DEVICE, std::string("hgs_step_batch: ") + hipGetErrorString(e));
    int c2 = cur, o2 = old;
    batch_roles(b->tblock, nsub, c2, o2);
    for (hgs_ctx* c : b->grids) {
        c->cur = c2;
        c->old = o2;
    }
    return HGS_OK;
}

}  // namespace

extern "C" {

hgs_status hgs_workspace_bytes_batch(const hgs_config* cfgs, int32_t n, size_t* bytes) {
    if (!bytes) return fail(nullptr, HGS_ERR_ARG, "bytes is NULL");
    BatchPlan p;
    std::string why;
    hgs_status s = batch_plan(cfgs, n, p, why);
    if (s != HGS_OK) return fail(nullptr, s, why);
    *bytes = p.total;
    return HGS_OK;
}

hgs_status hgs_init_batch(const hgs_config* cfgs, int32_t n, void* workspace, size_t bytes, hgs_batch** out) {
    if (!out) return fail(nullptr, HGS_ERR_ARG, "out is NULL");
    BatchPlan p;
    std::string why;
    hgs_status s = batch_plan(cfgs, n, p, why);
    if (s != HGS_OK) return fail(nullptr, s, why);
    if (!workspace) return fail(nullptr, HGS_ERR_WORKSPACE, "workspace is NULL");
    if (bytes < p.total) return fail(nullptr, HGS_ERR_WORKSPACE, "workspace smaller than hgs_workspace_bytes_batch()");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(nullptr, HGS_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    hgs_batch* b = new (std::nothrow) hgs_batch();
    if (!b) return fail(nullptr, HGS_ERR_ARG, "out of host memory");
    char* w = static_cast<char*>(workspace);
    b->n = n;
    b->storage = (hgs_dtype)cfgs[0].storage;
    b->tblock = default_tblock(&cfgs[0]);
    b->stream = static_cast<hipStream_t>(cfgs[0].stream);
    b->graph_ok = true;
    b->used_graph = false;
    b->capture = nullptr;
    b->desc_k = 0;
    b->desc_pending[0] = b->desc_pending[1] = false;
    b->desc_done[0] = b->desc_done[1] = nullptr;
    for (int i = 0; i < n; ++i) {
        hgs_ctx* c = nullptr;
        s = hgs_init(&cfgs[i], w + p.grid_off[i], p.grid_bytes[i], &c);
        if (s != HGS_OK) {
            for (hgs_ctx* q : b->grids) hgs_destroy(q);
            delete b;
            return s;
        }
        b->grids.push_back(c);
    }
    b->desc_dev = w + p.desc_off;
    b->tb_items = reinterpret_cast<WorkItem*>(w + p.tb_off);
    b->tbg_items = reinterpret_cast<WorkItem*>(w + p.tbg_off);
    b->st_items = reinterpret_cast<WorkItem*>(w + p.st_off);
    b->n_tb_items = (int)p.tb_items.size();
    b->n_tbg_items = (int)p.tbg_items.size();
    b->n_st_items = (int)p.st_items.size();
    b->launch = HGS_BATCH_PER_ITEM;
    hipError_t e = hipSuccess;
    if (!p.tb_items.empty())
        e = hipMemcpyAsync(b->tb_items, p.tb_items.data(), sizeof(WorkItem) * p.tb_items.size(),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && !p.tbg_items.empty())
        e = hipMemcpyAsync(b->tbg_items, p.tbg_items.data(), sizeof(WorkItem) * p.tbg_items.size(),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->st_items, p.st_items.data(), sizeof(WorkItem) * p.st_items.size(),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->desc_done[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->desc_done[1], hipEventDisableTiming);
    if (e == hipSuccess && hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess) {
        b->capture = nullptr;
        b->graph_ok = false;
    }
    if (e != hipSuccess) {
        for (hgs_ctx* q : b->grids) hgs_destroy(q);
        delete b;
        return fail(nullptr, HGS_ERR_DEVICE, std::string("hgs_init_batch: ") + hipGetErrorString(e));
    }
    *out = b;
    return HGS_OK;
}

hgs_status hgs_batch_grid(hgs_batch* b, int32_t i, hgs_ctx** ctx) {
    if (!b || !ctx) return fail(nullptr, HGS_ERR_ARG, "batch and ctx must be non-NULL");
    if (i < 0 || i >= b->n) return bfail(b, HGS_ERR_ARG, "grid index out of range");
    *ctx = b->grids[i];
    return HGS_OK;
}

int32_t hgs_batch_used_graph(const hgs_batch* b) { return b && b->used_graph ? 1 : 0; }

hgs_status hgs_batch_set_launch(hgs_batch* b, int32_t launch) {
    if (!b) return fail(nullptr, HGS_ERR_ARG, "batch is NULL");
    if (launch != HGS_BATCH_PER_ITEM && launch != HGS_BATCH_PERSISTENT)
        return bfail(b, HGS_ERR_ARG, "launch must be HGS_BATCH_PER_ITEM or HGS_BATCH_PERSISTENT");
    b->launch = launch;
    return HGS_OK;
}

int32_t hgs_batch_get_launch(const hgs_batch* b) { return b ? b->launch : -1; }

const char* hgs_batch_last_error(const hgs_batch* b) { return b ? b->err.c_str() : g_err.c_str(); }

hgs_status hgs_step_batch(hgs_batch* b, const void* const* rho, const double* c_g, const double* dt, int32_t nsub) {
    if (!b) return fail(nullptr, HGS_ERR_ARG, "batch is NULL");
    if (!rho || !c_g || !dt) return bfail(b, HGS_ERR_ARG, "rho, c_g and dt must be non-NULL");
    for (int i = 0; i < b->n; ++i) {
        hgs_status s = validate_step(b->grids[i], &b->grids[i]->cfg, rho[i], c_g[i], dt[i], nsub);
        if (s != HGS_OK) return bfail(b, s, "grid " + std::to_string(i) + ": " + b->grids[i]->err);
    }
    (void)hipGetLastError();
    for (int i = 0; i < b->n; ++i) {
        hgs_ctx* c = b->grids[i];
        if (c->cfg.bc == HGS_BC_MULTIPOLE) {
            DISPATCH(c, run_moments_and_ghosts, c, rho[i], 0xF);
            c->have_moments = true;
        }
        if (c->dt_prev > 0.0 && dt[i] != c->dt_prev) DISPATCH(c, run_rescale, c, dt[i] / c->dt_prev);
    }
    const int k = b->desc_k;
    b->desc_k ^= 1;
    hipError_t e = hipSuccess;
    if (b->desc_pending[k]) e = hipEventSynchronize(b->desc_done[k]);
    if (e != hipSuccess) return bfail(b, HGS_ERR_DEVICE, std::string("descriptor staging: ") + hipGetErrorString(e));
    if (b->storage == HGS_F64)
        batch_fill_desc<double>(b, b->desc_host[k], rho, c_g, dt);
    else
        batch_fill_desc<float>(b, b->desc_host[k], rho, c_g, dt);
    e = hipMemcpyAsync(b->desc_dev, b->desc_host[k].data(), b->desc_host[k].size(), hipMemcpyHostToDevice,
                       b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->desc_done[k], b->stream);
    if (e != hipSuccess) return bfail(b, HGS_ERR_DEVICE, std::string("descriptor upload: ") + hipGetErrorString(e));
    b->desc_pending[k] = true;
    hgs_status s = b->storage == HGS_F64 ? batch_run<double>(b, nsub) : batch_run<float>(b, nsub);
    if (s != HGS_OK) return s;
    for (int i = 0; i < b->n; ++i) b->grids[i]->dt_prev = dt[i];
    return HGS_OK;
}

hgs_status hgs_destroy_batch(hgs_batch* b) {
    if (!b) return HGS_OK;
    (void)hipStreamSynchronize(b->stream);
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    for (int k = 0; k < 2; ++k)
        if (b->desc_done[k]) (void)hipEventDestroy(b->desc_done[k]);
    for (hgs_ctx* c : b->grids) hgs_destroy(c);
    delete b;
    return HGS_OK;
}

}  // extern "C"

// ============================================================================
// Autotuner
// ============================================================================

namespace {

const char* bc_name(int bc) {
    switch (bc) {
        case HGS_BC_USER: return "user";
        case HGS_BC_ROBIN: return "robin";
        case HGS_BC_OUTGOING: return "outgoing";
        case HGS_BC_PERIODIC: return "periodic";
        default: return "multipole";
    }
}

std::string tune_key(const hgs_config* cfg, int nsub) {
    hipDeviceProp_t p;
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) {
        arch = p.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
    }
    std::ostringstream k;
    k << arch << ' ' << cfg->nx << ' ' << cfg->ny << ' ' << cfg->nz << ' ' << (cfg->storage == HGS_F64 ? "f64" : "f32")
      << ' ' << nsub << ' ' << bc_name(cfg->bc);
    return k.str();
}

// cache file: one "<key> <tblock> <tile>" entry per line (an entry without a
// tile means tile 0)
bool tune_cache_lookup(const std::string& path, const std::string& key, int& t_out, int& tile_out) {
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        if (line.size() > key.size() && line.compare(0, key.size(), key) == 0 && line[key.size()] == ' ') {
            std::istringstream v(line.substr(key.size() + 1));
            int t = 0, tile = 0;
            v >> t;
            if (!(v >> tile)) tile = 0;
            if (t >= 1 && t <= HGS_TMAX && tile >= 0 && tile < (t >= 2 ? tile_count(t) : 1)) {  // last entry wins
                t_out = t;
                tile_out = tile;
                found = true;
            }
        }
    }
    return found;
}

void tune_cache_store(const std::string& path, const std::string& key, int t, int tile) {
    std::ofstream f(path, std::ios::app);
    if (f) f << key << ' ' << t << ' ' << tile << '\n';
}

}  // namespace

extern "C" hgs_status hgs_autotune(const hgs_config* cfg, const void* rho, double c_g, double dt, int32_t nsub,
                                   void* workspace, size_t bytes, int32_t* best_tblock, int32_t* best_tile,
                                   double* ms_per_substep) {
    std::string why;
    hgs_status s = check_config(cfg, why);
    if (s != HGS_OK) return fail(nullptr, s, why);
    if (!best_tblock) return fail(nullptr, HGS_ERR_ARG, "best_tblock is NULL");
    s = validate_step(nullptr, cfg, rho, c_g, dt, nsub);
    if (s != HGS_OK) return s;
    if (best_tile) *best_tile = 0;
    const char* cache = std::getenv("HGS_TUNE_CACHE");
    const std::string key = tune_key(cfg, nsub);
    if (cache && *cache) {
        int t = 0, tile = 0;
        if (tune_cache_lookup(cache, key, t, tile)) {
            *best_tblock = t;
            if (best_tile) *best_tile = tile;
            if (ms_per_substep)
                for (int i = 0; i < HGS_TMAX; ++i) ms_per_substep[i] = -1.0;
            return HGS_OK;
        }
    }
    hgs_ctx* c = nullptr;
    s = hgs_init(cfg, workspace, bytes, &c);
    if (s != HGS_OK) return s;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        hgs_destroy(c);
        return fail(nullptr, HGS_ERR_DEVICE, "hgs_autotune: event creation failed");
    }
    const int reps = 3;
    // every depth 1..HGS_TMAX, and every tile shape compiled for a depth; a
    // depth whose fused launch nsub never reaches (T > nsub) is timed as well,
    // it then runs streaming substeps only.  Two passes, the second in reverse
    // order, each candidate keeping its faster one: launches right after an
    // idle gap run slower for a while, which would otherwise count against
    // whichever candidate comes first.
    std::vector<std::pair<int, int>> cand;
    for (int t = 1; t <= HGS_TMAX; ++t)
        for (int tile = 0; tile < (t >= 2 ? tile_count(t) : 1); ++tile) cand.emplace_back(t, tile);
    std::vector<double> per_cand(cand.size(), -1.0);
    hgs_status st = HGS_OK;
    for (int pass = 0; pass < 2 && st == HGS_OK; ++pass) {
        for (size_t q = 0; q < cand.size() && st == HGS_OK; ++q) {
            const size_t i = pass == 0 ? q : cand.size() - 1 - q;
            c->tblock = cand[i].first;
            c->tile = cand[i].second;
            st = hgs_step(c, rho, c_g, dt, nsub);  // warm-up
            if (st != HGS_OK) break;
            (void)hipEventRecord(e0, c->stream);
            for (int r = 0; r < reps && st == HGS_OK; ++r) st = hgs_step(c, rho, c_g, dt, nsub);
            (void)hipEventRecord(e1, c->stream);
            if (hipEventSynchronize(e1) != hipSuccess) {
                st = fail(nullptr, HGS_ERR_DEVICE, "hgs_autotune: timing failed");
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const double per = (double)ms / (reps * nsub);
            if (per_cand[i] < 0.0 || per < per_cand[i]) per_cand[i] = per;
        }
    }
    double best_ms = -1.0;
    int best = 1, best_t = 0;
    if (ms_per_substep)
        for (int i = 0; i < HGS_TMAX; ++i) ms_per_substep[i] = -1.0;
    for (size_t i = 0; i < cand.size() && st == HGS_OK; ++i) {
        const int t = cand[i].first;
        if (ms_per_substep && (ms_per_substep[t - 1] < 0.0 || per_cand[i] < ms_per_substep[t - 1]))
            ms_per_substep[t - 1] = per_cand[i];
        if (best_ms < 0.0 || per_cand[i] < best_ms) {
            best_ms = per_cand[i];
            best = t;
            best_t = cand[i].second;
        }
    }
    if (st != HGS_OK && c) g_err = c->err;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    hgs_destroy(c);
    if (st != HGS_OK) return st;
    *best_tblock = best;
    if (best_tile) *best_tile = best_t;
    if (cache && *cache) tune_cache_store(cache, key, best, best_t);
    return HGS_OK;
}
