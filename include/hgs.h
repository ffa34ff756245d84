/*
 * hgs.h -- C ABI of the MI355X (gfx950) hyperbolic self-gravity library.
 *
 * The method (Hirai, Nagakura, Okawa & Fujisawa, arXiv:1602.05700): instead of
 * solving the Poisson equation  Laplacian(phi) = 4 pi G rho  (Eq. 1), the
 * potential is advanced in time by the inhomogeneous wave equation
 *     (-c_g^-2 d^2/dt^2 + Laplacian) phi = 4 pi G rho                (Eq. 2)
 * by explicit time stepping on the hydrodynamic grid.  Per hydrodynamical step
 * the density is frozen and the wave equation is sub-cycled with a smaller step
 * (Sec. 2, separate timelines for gravity and hydrodynamics).  The outer
 * boundary is a Dirichlet condition from a multipole expansion of rho (Sec. 2
 * and Sec. 4, Table I model aD05), a caller-supplied Dirichlet one, or a local
 * one that follows the interior every substep (Robin -- the paper's default --,
 * its outgoing-wave form, periodic; Sec. 2 and Sec. 4).  Calls near the end
 * move a local boundary away from the matter (Sec. 4): an extended
 * gravity-only grid and a nested coarse outer level.  The gravitational
 * acceleration is g = -grad phi.
 *
 * Discretisation (Sec. 2 leaves it unspecified):
 *   cell-centred uniform grid of nx*ny*nz cubic cells of size dx; cell (i,j,k)
 *   centre = (x0 + (i+1/2) dx, y0 + (j+1/2) dx, z0 + (k+1/2) dx);
 *   7-point Laplacian L_h with one layer of ghost cells outside each face;
 *   3-level leapfrog in time with an optional damping term eta (eta = 0 is
 *   Eq. 2 exactly; eta > 0 adds eta dphi/dt, which leaves the steady state --
 *   the discrete Poisson solution -- unchanged and lets a zero start relax):
 *     phi^{n+1} = [2 phi^n - (1 - a) phi^{n-1} + c^2 dt^2 (L_h phi^n - 4 pi G rho)] / (1 + a),
 *     a = eta dt / 2.
 *   FP64 storage: FP64 arithmetic.  FP32 storage: the substep is evaluated in
 *   FP32 in increment form, phi^{n+1} = phi^n + [(1-a)(phi^n - phi^{n-1}) +
 *   kk sum(nb - phi^n) - c^2 dt^2 4 pi G rho]/(1+a), whose differences of
 *   nearby FP32 values are exact, so the stored state keeps the accuracy of
 *   FP64 arithmetic; moments, boundary values, gradient and norms are FP64.
 *
 * Conventions for every call below.
 *   - 3D field buffers passed by the caller (rho, phi, phidot, gx, gy, gz, the
 *     raw state) are DEVICE pointers to contiguous arrays of shape (nz, ny, nx),
 *     x fastest, element type = cfg.storage.  The caller owns them.
 *   - Ghost-face buffers hold the six faces back to back in the order
 *     x-, x+, y-, y+, z-, z+; x faces are (nz, ny) arrays, y faces (nz, nx),
 *     z faces (ny, nx); ghost centres lie dx/2 outside the face.
 *     Element type = cfg.storage, device memory.
 *   - All work is enqueued on cfg.stream (a hipStream_t, NULL = the null
 *     stream) and is asynchronous, except the calls marked "synchronises".
 *     Input buffers must stay valid until the stream has passed the call.
 *   - Every call validates its arguments on the host before enqueueing anything;
 *     on any non-OK status no state has changed.  No call prints, aborts or
 *     throws.  hgs_last_error() gives a readable reason for the last failure.
 *   - A context is used by one host thread at a time.
 */
#ifndef HGS_H
#define HGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hgs_ctx hgs_ctx; /* opaque; host memory owned by the library */

typedef enum {
    HGS_OK = 0,
    HGS_ERR_ARG = 1,       /* invalid argument (null pointer, bad size, dt <= 0, ...) */
    HGS_ERR_CFL = 2,       /* c_g dt / dx above 1/sqrt(3), the 3D leapfrog stability limit */
    HGS_ERR_WORKSPACE = 3, /* workspace missing, too small or misaligned */
    HGS_ERR_DEVICE = 4,    /* a HIP call failed */
    HGS_ERR_NONFINITE = 5, /* a synchronising call found NaN/Inf in phi or rho */
    HGS_ERR_STATE = 6      /* call not valid in the context's current state */
} hgs_status;

typedef enum { HGS_F64 = 0, HGS_F32 = 1 } hgs_dtype;

typedef enum {
    HGS_BC_MULTIPOLE = 0, /* Dirichlet ghosts from multipole moments of rho (Sec. 2, Sec. 4) */
    HGS_BC_USER = 1,      /* Dirichlet ghosts set by hgs_set_boundary and kept */
    /* Local boundaries: after every substep each face ghost g is set from the
     * interior cell i next to it (r measured from cfg.origin, which must lie
     * strictly inside the grid).  All three fuse tblock substeps per launch
     * like the frozen boundaries, with the same results bit for bit as one
     * substep per launch: Robin ghosts are taken inside the launch as the
     * rule's value of the neighbour's level, periodic tiles wrap around the
     * grid, and outgoing ghosts are advanced level by level inside the launch
     * (which then splits z into an even number of chunks at least tblock
     * planes deep, so its depth is at most nz / 2).  A grid with an axis of
     * one cell runs one substep per launch.  Robin ghosts are evaluated in the
     * storage type:
     * FP64 as phi_i sqrt(r_i^2 / r_g^2), FP32 as phi_i r_i^2 / sqrt(r_i^2 r_g^2)
     * with the hardware reciprocal square root.  Substeps evaluate or advance
     * the ghosts they need themselves; the ghost layer of phi^n is the rule's
     * after every hgs_step (hgs_get_boundary, the gradient, the residual).
     * Not available in batches. */
    HGS_BC_ROBIN = 2,     /* the paper's default outer boundary, a Robin condition amounting to
                             monopole gravity (Sec. 2, Sec. 4): r_g phi_g = r_i phi_i, i.e.
                             d(r phi)/dr = 0; exact for -G M / r */
    HGS_BC_OUTGOING = 3,  /* its radiative form d(r phi)/dt + c_g d(r phi)/dr = 0, so that errors
                             leave through the boundary (Sec. 4); box scheme on u = r phi at the
                             ghost/neighbour midpoint x_f, d/dr = d/dn / cos(theta),
                             alpha = c_g dt / (dx cos(theta)):
                               u_g' = [(1-alpha) u_g + (1+alpha) u_i - (1-alpha) u_i'] / (1+alpha)
                             (primes: the new level).  Steady state = Robin's.  Lets a zero
                             start relax with eta = 0. */
    HGS_BC_PERIODIC = 4   /* ghost = interior cell at the opposite face; the source is
                             4 pi G (rho - mean rho) (Sec. 4), the mean taken in FP64 each
                             hgs_step; a zero start keeps mean(phi) = 0 */
} hgs_bc;

/* Largest temporal-blocking depth (substeps fused per launch). */
#define HGS_TMAX 4
/* Largest multipole degree. */
#define HGS_LMAX 4

typedef struct {
    int32_t nx, ny, nz; /* interior cells, each 1..8192 */
    double x0, y0, z0;  /* lower corner of the interior */
    double dx;          /* cubic cell size, > 0 */
    double G;           /* gravitational constant, finite */
    double origin[3];   /* multipole expansion centre; strictly inside the grid when bc = MULTIPOLE */
    int32_t lmax;       /* multipole degree 0..HGS_LMAX; 0 gives phi_b = -G M / r */
    int32_t bc;         /* hgs_bc */
    int32_t storage;    /* hgs_dtype of every stored field and I/O buffer */
    int32_t tblock;     /* substeps fused per stencil launch: 1..HGS_TMAX, 0 = library default */
    double eta;         /* damping rate >= 0; 0 = the paper's Eq. (2) */
    void* stream;       /* hipStream_t for all work, NULL = null stream */
} hgs_config;

/* Fill *cfg for an n^3 grid on [lo, hi]^3 with G = 1, origin 0, lmax 4,
 * multipole boundary, FP32 storage, eta 0, default blocking, null stream. */
hgs_status hgs_config_cube(hgs_config* cfg, int32_t n, double lo, double hi);

/* Device workspace the context needs, in bytes (the library never allocates
 * device memory; the caller provides it to hgs_init). */
hgs_status hgs_workspace_bytes(const hgs_config* cfg, size_t* bytes);

/* Create a context over a caller-owned device workspace of at least
 * hgs_workspace_bytes(cfg) bytes, 256-byte aligned, that outlives the context.
 * The state starts at phi = phi_prev = 0 with zero ghosts.  Enqueues fill
 * kernels on cfg->stream. */
hgs_status hgs_init(const hgs_config* cfg, void* workspace, size_t bytes, hgs_ctx** out);

/* One hydrodynamical step (Sec. 2): with rho frozen,
 *   1. (bc = MULTIPOLE) moments Q_lm of rho and the Dirichlet ghosts
 *      phi_b(x) = -G sum_{l<=lmax} sum_m 4 pi/(2l+1) Q_lm Y_lm(x^) / |x|^{l+1},
 *      Q_lm = sum_cells rho dx^3 |x|^l conj(Y_lm(x^)), positions relative to
 *      cfg.origin;
 *   2. nsub leapfrog substeps of size dt with propagation speed c_g.
 * If dt differs from the previous step's, phi_prev is first rescaled so that
 * (phi - phi_prev)/dt is kept.  Errors: HGS_ERR_ARG (null rho, nsub < 1,
 * dt or c_g not positive and finite), HGS_ERR_CFL (c_g dt / dx > 1/sqrt(3)). */
hgs_status hgs_step(hgs_ctx* ctx, const void* rho, double c_g, double dt, int32_t nsub);

/* The host-side validation hgs_step applies, without a context or a GPU:
 * HGS_ERR_ARG for a bad cfg, NULL rho, nsub < 1, dt or c_g not positive and
 * finite; HGS_ERR_CFL when c_g dt / dx > 1/sqrt(3); else HGS_OK. */
hgs_status hgs_validate_step(const hgs_config* cfg, const void* rho, double c_g, double dt, int32_t nsub);

/* bc = MULTIPOLE: the first stage of hgs_step alone -- the moments of rho and
 * the Dirichlet ghost shell they give (Sec. 2, Sec. 4), written into the
 * current state (phi^n and phi^{n-1}), with no substep.  For a residual of a
 * state set by hgs_set_state against the boundary of a density (the warm
 * start's check against the zero start).  HGS_ERR_STATE for another bc,
 * HGS_ERR_ARG for a NULL ctx or rho. */
hgs_status hgs_multipole_boundary(hgs_ctx* ctx, const void* rho);

/* The zero start as the fallback of a predicted start, decided on the device
 * in stream order (no synchronisation): after hgs_set_state has set a start,
 * its residual R_b for rho is computed (bc = MULTIPOLE: with the ghost shell
 * of rho computed first, as hgs_step does) and, unless the state is finite
 * and R_b is below the zero start's R_b = 1, the state is reset to
 * phi^n = phi^{n-1} = 0.  kept (nullable): device int32 set to 1 when the
 * start was kept, 0 when it was reset.  Errors: HGS_ERR_ARG (NULL ctx or
 * rho), HGS_ERR_STATE (a local boundary, whose ghosts follow the state). */
hgs_status hgs_keep_start_if_better(hgs_ctx* ctx, const void* rho, int32_t* kept);

/* The steady state directly: the discrete Dirichlet Poisson problem
 * L_h phi = 4 pi G rho (Eq. 1, the 7-point Laplacian, the ghosts as boundary
 * values) -- the fixed point of every damped run, and the Poisson solution the
 * paper's runs start from (Sec. 2) -- solved by type-I sine transforms along
 * each axis (the eigenvectors of the 1D second difference with Dirichlet
 * ends) in FP64; the state becomes phi^n = phi^{n-1} = phi (phidot = 0).
 * bc = MULTIPOLE: the ghosts are first computed from the moments of rho, as
 * hgs_step does; bc = USER: the ghosts set by hgs_set_boundary.  rho: device
 * (nz, ny, nx), storage dtype.  scratch: device memory of at least
 * 2 nx ny nz doubles, 256-byte aligned, used during the call only.  The cost
 * is nx ny nz (nx + ny + nz) multiply-adds (dense transforms): meant for
 * grids up to ~128 per axis.  Errors: HGS_ERR_ARG (NULL ctx or rho, an axis
 * above 1024 cells), HGS_ERR_STATE (a local boundary), HGS_ERR_WORKSPACE
 * (scratch missing, too small or misaligned). */
hgs_status hgs_poisson_direct(hgs_ctx* ctx, const void* rho, void* scratch, size_t bytes);

/* Copy the current potential out; phidot (nullable) receives the backward
 * difference (phi^n - phi^{n-1}) / dt of the last step (zero before any step). */
hgs_status hgs_potential(hgs_ctx* ctx, void* phi, void* phidot);

/* g = -grad phi of the current potential by second-order central
 * differences, ghosts at the faces; three separate (nz,ny,nx) arrays. */
hgs_status hgs_accel(hgs_ctx* ctx, void* gx, void* gy, void* gz);

/* Set the state from a potential and its time derivative: phi^n = phi,
 * phi^{n-1} = phi - dt * phidot (phidot NULL means 0).  dt > 0 becomes the
 * "previous step" for the dt-rescaling rule of hgs_step.  With a local
 * boundary the ghosts of both levels are then set from their interiors by the
 * steady rule (Robin's relation for ROBIN and OUTGOING, the wrap for PERIODIC). */
hgs_status hgs_set_state(hgs_ctx* ctx, const void* phi, const void* phidot, double dt);

/* bc = USER (else HGS_ERR_STATE, except OUTGOING): set the ghost faces
 * (device, storage dtype, face layout above); they stay until the next call.
 * bc = OUTGOING: the ghosts carry state (u_g of the box scheme); this call
 * restores them, e.g. after hgs_load_raw, which otherwise rebuilds every local
 * boundary's ghosts from the interior by the steady rule. */
hgs_status hgs_set_boundary(hgs_ctx* ctx, const void* ghosts);

/* Copy the current ghost faces into a device buffer (face layout above). */
hgs_status hgs_get_boundary(hgs_ctx* ctx, void* ghosts);

/* Synchronises.  The moments of the last hgs_step (bc = MULTIPOLE) as
 * 2*(lmax+1)^2 doubles on the host: (Re, Im) of Q_lm for l = 0..lmax,
 * m = -l..l, index l*l + l + m, with orthonormal complex Y_lm including the
 * Condon-Shortley phase.  HGS_ERR_STATE before the first step. */
hgs_status hgs_moments(hgs_ctx* ctx, double* q_host);

/* Synchronises.  Residual of the steady state L_h phi = 4 pi G rho (Eq. 1)
 * for the current phi and the given rho (device, (nz,ny,nx)), on the host:
 *   out[0] = R_b = ||L_h phi - s|| / ||b||, b = s - (adjacent ghosts)/dx^2
 *            (the textbook relative residual of the interior linear system;
 *            1 at phi = 0),
 *            With a local boundary the ghosts are images of interior unknowns,
 *            so b = s and R_b = R_f,
 *   out[1] = R_f = ||L_h phi - s|| / ||s||,  s = 4 pi G rho (PERIODIC:
 *            4 pi G (rho - mean rho)),
 *   out[2] = ||phi|| over the interior,
 *   out[3] = 1 if phi or rho holds a NaN/Inf (status HGS_ERR_NONFINITE), else 0.
 * 2-norms over interior cells, FP64.  A zero denominator gives 0 for a zero
 * numerator and +inf otherwise. */
hgs_status hgs_residual(hgs_ctx* ctx, const void* rho, double out[4]);

/* ---- Coupling to a hydrodynamics code ---------------------------------------
 * The paper sets the propagation speed from the flow, c_g = k_g (c_s + |v|)
 * (Eq. 3, k_g > 1), and advances gravity on its own timeline: k_g wave
 * substeps per hydrodynamical step with the same Courant number (Sec. 2).
 * Read here with c_s + |v| maximised over the grid, since c_g is one speed. */

/* Synchronises.  *vmax = max over cells of c_s + |v| (FP64); cs: device
 * (nz,ny,nx) in the storage dtype; vx, vy, vz likewise, each nullable (0).
 * HGS_ERR_NONFINITE if any value is NaN/Inf. */
hgs_status hgs_max_signal_speed(hgs_ctx* ctx, const void* cs, const void* vx, const void* vy, const void* vz,
                                double* vmax);

/* Synchronises (reads the signal speed back).  One hydrodynamical step of the
 * coupled scheme: vmax = max(c_s + |v|), dt_hydro = courant_hydro dx / vmax,
 * c_g = k_g vmax, nsub = ceil(k_g courant_hydro / courant_grav) (the smallest
 * count with c_g (dt_hydro / nsub) / dx <= courant_grav; = ceil(k_g) for equal
 * Courant numbers), then hgs_step(rho, c_g, dt_hydro / nsub, nsub).  Outputs
 * dt_hydro, nsub and c_g.  Errors: HGS_ERR_ARG for k_g < 1, courant_hydro <= 0,
 * courant_grav outside (0, 1/sqrt(3)], a zero signal speed or more than 1e6
 * substeps; those of hgs_max_signal_speed and hgs_step. */
hgs_status hgs_hydro_step(hgs_ctx* ctx, const void* rho, const void* cs, const void* vx, const void* vy,
                          const void* vz, double k_g, double courant_hydro, double courant_grav, double* dt_hydro,
                          int32_t* nsub, double* c_g);

/* Synchronises.  Gravitational energy W = 1/2 sum_cells rho phi dx^3 of the
 * current potential (FP64), rho device (nz,ny,nx) in the storage dtype. */
hgs_status hgs_energy(hgs_ctx* ctx, const void* rho, double* w);

/* ---- Extended gravity-only grid --------------------------------------------
 * Sec. 4 proposes solving the wave equation on a grid wider than the region of
 * the hydrodynamics, the extension close to vacuum, so that a local (Robin)
 * boundary sits far from the matter at little cost.  A context built for the
 * wider grid ((nx + 2 ext) x (ny + 2 ext) x (nz + 2 ext) cells, x0 moved out
 * by ext dx) does this; these two calls move compact fields between the
 * hydrodynamics region (nz, ny, nx) and the wider grid, both device arrays of
 * the given dtype, enqueued on stream.
 * hgs_embed: outer = inner in the centre, 0 in the extension (every outer
 *   cell written).  hgs_extract: inner = the centre of outer.
 * HGS_ERR_ARG for NULL pointers, sizes outside 1..8192 (or a wider grid beyond
 * 8192 cells along an axis), ext < 0 or a bad dtype. */
hgs_status hgs_embed(const void* inner, int32_t nx, int32_t ny, int32_t nz, int32_t ext, void* outer, int32_t dtype,
                     void* stream);
hgs_status hgs_extract(const void* outer, int32_t nx, int32_t ny, int32_t nz, int32_t ext, void* inner, int32_t dtype,
                       void* stream);

/* g = -grad phi on the box [i0, i0 + bx) x [j0, j0 + by) x [k0, k0 + bz) of
 * the interior only, written as three compact (bz, by, bx) device arrays of the
 * storage dtype, enqueued on the context's stream.  Every value equals
 * hgs_accel's at the same cell (same arithmetic; the box's neighbours are the
 * grid's cells, ghosts where the box touches a face).  On an extended grid the
 * hydrodynamics region is the box (ext, ext, ext, nx, ny, nz), which spares the
 * gradient of the extension and the three extractions.  HGS_ERR_ARG for a NULL
 * ctx or output, or a box that is empty or not inside the interior. */
hgs_status hgs_accel_box(hgs_ctx* ctx, int32_t i0, int32_t j0, int32_t k0, int32_t bx, int32_t by, int32_t bz,
                         void* gx, void* gy, void* gz);

/* ---- Nested coarse outer level ----------------------------------------------
 * Sec. 4 names nested grids as a way to put the outer boundary far from the
 * matter at little cost; it gives no scheme, and the one here is this
 * library's reading.  A coarse context of cell size 2 dx covers the fine grid
 * and ext coarse cells more on every side (corner moved out by 2 ext dx),
 * with a local boundary (ROBIN or OUTGOING) at its faces; the fine context has
 * bc = USER.  Per hydrodynamical step: hgs_nest_source gives the coarse
 * density, the coarse context takes ceil(nsub / 2) substeps spanning
 * nsub * dt, hgs_nest_ghosts turns its potential (hgs_potential) into the
 * fine ghosts for hgs_set_boundary, and the fine context takes its nsub
 * substeps with those ghosts frozen.  More levels repeat this outwards (each
 * inner one bc = USER, only the outermost local), advanced from the outermost
 * inwards.  Device buffers of the given dtype, enqueued on stream, no
 * synchronisation.
 * hgs_nest_source: coarse (nz/2 + 2 ext, ny/2 + 2 ext, nx/2 + 2 ext) = the
 *   means of rho (nz, ny, nx) over 2 x 2 x 2 blocks in the centre, 0 in the
 *   extension (every coarse cell written).  HGS_ERR_ARG for NULL pointers,
 *   odd or out-of-range sizes, ext < 0 or a bad dtype.
 * hgs_nest_ghosts: faces (the layout of hgs_set_boundary for an (nz, ny, nx)
 *   grid with lower corner fine_x0[3] (host) and cell fine_dx) = the coarse
 *   compact potential (mz, my, mx; corner coarse_x0[3], cell coarse_dx)
 *   interpolated trilinearly between the nearest coarse cell centres at every
 *   ghost centre, in FP64.  HGS_ERR_ARG for NULL pointers, sizes out of range
 *   (coarse at least 2 per axis), cell sizes not positive and finite, or a
 *   ghost centre outside the span of the coarse cell centres. */
hgs_status hgs_nest_source(const void* rho, int32_t nx, int32_t ny, int32_t nz, int32_t ext, void* coarse,
                           int32_t dtype, void* stream);
hgs_status hgs_nest_ghosts(const void* coarse_phi, int32_t mx, int32_t my, int32_t mz, const double* coarse_x0,
                           double coarse_dx, int32_t nx, int32_t ny, int32_t nz, const double* fine_x0,
                           double fine_dx, void* faces, int32_t dtype, void* stream);

/* Bitwise copy of the raw two-level state (phi^n, phi^{n-1} interiors, device
 * (nz,ny,nx) buffers) and the previous step size, for checkpoint/resume. */
hgs_status hgs_save_raw(hgs_ctx* ctx, void* phi_n, void* phi_nm1, double* dt_prev);
hgs_status hgs_load_raw(hgs_ctx* ctx, const void* phi_n, const void* phi_nm1, double dt_prev);

/* Substeps fused per stencil launch for later steps (1..HGS_TMAX, 0 = default). */
hgs_status hgs_set_tblock(hgs_ctx* ctx, int32_t tblock);
int32_t hgs_get_tblock(const hgs_ctx* ctx);

/* Tile shape of the fused launches.  A fused launch of depth T gives each
 * workgroup an (x, y) tile that it marches up a chunk of z planes; several
 * shapes are compiled per storage type and depth, trading the tile's height
 * (less halo recomputed and re-read per cell) against the input planes kept
 * in flight (both live in registers).  Results are bit-identical for every
 * shape.  hgs_tile_count(T): shapes compiled for depth T (0 for T outside
 * 2..HGS_TMAX).  hgs_tile_shape: shape[0] rows per thread, shape[1] waves per
 * workgroup (the tile is 64 x rows*waves cells, T of them halo on each side),
 * shape[2] input planes in flight; HGS_ERR_ARG for an unknown storage, depth
 * or index.  hgs_set_tile selects index tile (0 = default) for later steps;
 * a depth with fewer shapes uses its shape 0.  HGS_ERR_ARG if tile is outside
 * 0..hgs_tile_count(HGS_TMAX)-1. */
int32_t hgs_tile_count(int32_t tblock);
hgs_status hgs_tile_shape(int32_t storage, int32_t tblock, int32_t tile, int32_t shape[3]);
hgs_status hgs_set_tile(hgs_ctx* ctx, int32_t tile);
int32_t hgs_get_tile(const hgs_ctx* ctx);

/* Per-launch timing with HIP events recorded on the context's stream around
 * each kernel launch of the given kind, for roofline measurements:
 *   HGS_KERNEL_STENCIL  the substep launches of hgs_step (streaming or fused),
 *   HGS_KERNEL_MULTIPOLE the moment and ghost-shell launches of hgs_step,
 *   HGS_KERNEL_GRADIENT the launches of hgs_accel and hgs_accel_box.
 * hgs_timing_enable(ctx, 1) clears earlier records and starts recording;
 * 0 stops.  hgs_timing_read synchronises and returns, for one kind,
 *   out[0] launches, out[1] summed launch time in ms, out[2] algorithmic HBM
 *   bytes of those launches (each array element read or written once:
 *   streaming substep 4 elements per cell, fused launch of T substeps 5,
 *   moments 1, gradient 4), out[3] cell updates (cells x substeps). */
typedef enum { HGS_KERNEL_STENCIL = 0, HGS_KERNEL_MULTIPOLE = 1, HGS_KERNEL_GRADIENT = 2 } hgs_kernel_kind;
hgs_status hgs_timing_enable(hgs_ctx* ctx, int32_t enable);
hgs_status hgs_timing_read(hgs_ctx* ctx, int32_t kind, double out[4]);

/* ---- Batched form: many independent grids stepped together ------------------
 * A batch is n ordinary contexts carved from one workspace; hgs_batch_grid
 * gives grid i's context for every single-grid call (potential, accel,
 * residual, set_state, ...).  hgs_step_batch performs one hydrodynamical step
 * on all grids: per grid the multipole moments and ghosts, then nsub substeps
 * for every grid in launches that each cover all grids (work items of tiles
 * and z chunks, see hgs_batch_set_launch), replayed from a captured hipGraph
 * of the substep sequence.  Results are bit-identical to stepping each grid alone with the
 * same tblock.  Requirements: all grids share storage, stream and tblock (taken
 * from cfgs[0]); every nx is a multiple of the 16-byte vector width (4 for
 * FP32, 2 for FP64). */
typedef struct hgs_batch hgs_batch;
hgs_status hgs_workspace_bytes_batch(const hgs_config* cfgs, int32_t n, size_t* bytes);
hgs_status hgs_init_batch(const hgs_config* cfgs, int32_t n, void* workspace, size_t bytes, hgs_batch** out);
/* Grid i's context, owned by the batch (do not destroy it). */
hgs_status hgs_batch_grid(hgs_batch* b, int32_t i, hgs_ctx** ctx);
/* rho: host array of n device pointers; c_g, dt: host arrays of n values.
 * Validates every grid (as hgs_step) before enqueueing anything. */
hgs_status hgs_step_batch(hgs_batch* b, const void* const* rho, const double* c_g, const double* dt, int32_t nsub);
/* Whether the last hgs_step_batch replayed a captured graph (1) or fell back
 * to direct launches (0). */
int32_t hgs_batch_used_graph(const hgs_batch* b);
/* How the fused substeps of a batch are launched (results are bit-identical):
 *   HGS_BATCH_PER_ITEM (default): one workgroup per work item, items in grid
 *     order (z chunks, tile rows, tiles) with a contiguous range per XCD, so
 *     neighbouring tiles of one grid run together and share halo lines in L2;
 *     the hardware hands items to CUs as they free up;
 *   HGS_BATCH_PERSISTENT: one workgroup per CU walking the items in
 *     decreasing cost, strided (a static longest-first assignment).
 * HGS_ERR_ARG for another value. */
typedef enum { HGS_BATCH_PER_ITEM = 0, HGS_BATCH_PERSISTENT = 1 } hgs_batch_launch;
hgs_status hgs_batch_set_launch(hgs_batch* b, int32_t launch);
int32_t hgs_batch_get_launch(const hgs_batch* b);
/* Reason for the batch's last non-OK status ("" if none). */
const char* hgs_batch_last_error(const hgs_batch* b);
hgs_status hgs_destroy_batch(hgs_batch* b);

/* ---- Learned warm start: network kernels ---------------------------------
 * An extension of the method (the paper starts its runs from a Poisson
 * solution, Sec. 2): a 3x3x3 convolution network predicts the potential from
 * the density and a coarse solve, and the solver continues from it.  Tensors
 * are channels-last with 16 channels, (B, Z, Y, X, 16), bfloat16 bit patterns
 * in uint16 unless stated; weights are (27 taps, 16 out, 16 in) bfloat16 with
 * tap t = (dz+1)*9 + (dy+1)*3 + (dx+1); the convolution is a correlation with
 * zero padding ("same" size): out[v][co] = sum_t,ci w[t][co][ci] in[v+tap][ci].
 * All pointers are device pointers owned by the caller; all calls are
 * asynchronous on `stream` (NULL = null stream) and validate on the host
 * before launching: a NULL required pointer, a size out of range or a
 * misaligned tensor returns HGS_ERR_ARG and launches nothing, a failed launch
 * HGS_ERR_DEVICE; the reason is in hgs_nn_last_error(). */
#define HGS_NN_CHANNELS 16
typedef enum {
    HGS_NN_F32 = 0,        /* out (FP32) = conv + bias */
    HGS_NN_TANH_BF16 = 1,  /* out (bf16) = tanh(conv + bias) */
    HGS_NN_DTANH_BF16 = 2, /* out (bf16) = conv * (1 - aux^2), aux a tanh output (backward) */
    HGS_NN_BF16 = 3        /* out (bf16) = conv + bias */
} hgs_nn_mode;
/* X must be a multiple of 16; in, w and out 16-byte aligned; bias may be NULL
 * (zero); aux only for DTANH. */
hgs_status hgs_nn_conv3d(const uint16_t* in, const uint16_t* w, const float* bias, int32_t B, int32_t Z, int32_t Y,
                         int32_t X, int32_t mode, const uint16_t* aux, void* out, void* stream);
/* wt[26 - t][ci][co] = w[t][co][ci]: the weights of the input-gradient convolution. */
hgs_status hgs_nn_flip_weights(const uint16_t* w, uint16_t* wt, void* stream);
/* Weight and bias gradients dw[t][co][ci] = sum_v g[v][co] a[v+tap][ci] (FP32),
 * db[co] = sum_v g[v][co]; X a multiple of 16 and at most 128.  Needs a device
 * workspace of hgs_nn_wgrad_workspace_bytes(). Fixed-order reductions. */
hgs_status hgs_nn_wgrad_workspace_bytes(int32_t B, int32_t Z, int32_t Y, int32_t X, size_t* bytes);
hgs_status hgs_nn_wgrad(const uint16_t* a, const uint16_t* g, int32_t B, int32_t Z, int32_t Y, int32_t X, float* dw,
                        float* db, void* workspace, size_t bytes, void* stream);
/* Planar FP32 fields [B][C][nvox] <-> channels-last (bf16 out / FP32 in), C <= 16. */
hgs_status hgs_nn_pack(const float* fields, int32_t B, int32_t C, int64_t nvox, uint16_t* out, void* stream);
hgs_status hgs_nn_unpack(const float* in, int32_t B, int32_t C, int64_t nvox, float* fields, void* stream);
/* Mean-squared error of the first C channels of out (FP32 channels-last)
 * against planar targets [B][C][nvox]: grad (bf16 channels-last, zero beyond
 * C) = 2 (out - target) / (B C nvox); *loss_dev (device double) = sum of
 * squares.  Needs a device workspace of HGS_NN_MSE_PARTIALS doubles. */
#define HGS_NN_MSE_PARTIALS 1024
hgs_status hgs_nn_mse(const float* out, const float* target, int32_t B, int32_t C, int64_t nvox, uint16_t* grad,
                      double* loss_dev, double* partials, void* stream);
/* The same with a Laplacian term on channel ch: with e = out - target and L
 * the 7-point Laplacian in index units (zero outside the (nz, ny, nx) box),
 *   loss = sum_c,v e_c^2 + w sum_v (L e_ch)^2      (*loss_dev, device double)
 *   grad = (2 e + [c == ch] 2 w L(L e_ch)) / (B C nvox)   (bf16 channels-last).
 * The residual of a predicted potential, which sets the solver's steps from a
 * warm start, weighs fine-scale error with the Laplacian.  scratch: device
 * FP32, B*nz*ny*nx elements; partials: HGS_NN_MSE_PARTIALS doubles. */
hgs_status hgs_nn_lapmse(const float* out, const float* target, int32_t B, int32_t C, int32_t nz, int32_t ny,
                         int32_t nx, int32_t ch, float w, float* scratch, uint16_t* grad, double* loss_dev,
                         double* partials, void* stream);
/* Warm-start inputs and outputs (FP32, device).
 * hgs_nn_maxabs: out[b] = max |x[b][v]| over nvox values (one per sample);
 *   scratch: B * HGS_NN_MAXABS_CHUNKS floats of device memory.
 * hgs_nn_features: planar inputs out[B][3][nz][ny][nx] from rho and a coarse
 *   potential phi ([B][nz][ny][nx]) on a grid of spacing h, c = 4 pi G h^2:
 *   rho / s, phi / s and the potential's residual of the discrete Poisson
 *   equation (Eq. 1), (L phi - c rho) / (c s), with L the 7-point Laplacian in
 *   index units whose second difference along an axis is 0 at the first and
 *   last cell; s = scale[b].
 * hgs_nn_compose: phi = phi_c + y[..., 0] s / out_scale and (phidot nullable)
 *   phidot = y[..., 1] s / out_scale from the last layer's channels-last FP32
 *   output y ([B][nvox][16]); inv_out_scale = 1 / out_scale. */
#define HGS_NN_MAXABS_CHUNKS 64
hgs_status hgs_nn_maxabs(const float* x, int32_t B, int64_t nvox, float* out, float* scratch, void* stream);
/* hgs_nn_maxabs for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and result, with the per-chunk partials in a static device
 * array of the library (B * HGS_NN_MAXABS_CHUNKS floats, at most
 * HGS_NN_MAXABS_NOALLOC_MAX_B samples: 1 MiB per device, held until the
 * process ends) instead of a caller's scratch buffer.  Allocates nothing.
 * The stream must belong to the current device.  Every call on one device
 * shares that device's array: calls that overlap on one device (different
 * streams or host threads without ordering) race and give undefined results.
 * Errors: HGS_ERR_ARG for NULL pointers, nvox < 1 or B outside
 * 1..HGS_NN_MAXABS_NOALLOC_MAX_B; HGS_ERR_DEVICE when the array's address
 * cannot be obtained or a launch fails. */
#define HGS_NN_MAXABS_NOALLOC_MAX_B 4096
hgs_status hgs_nn_maxabs_noalloc(const float* x, int32_t B, int64_t nvox, float* out, void* stream);
hgs_status hgs_nn_features(const float* rho, const float* phi, const float* scale, int32_t B, int32_t nz, int32_t ny,
                           int32_t nx, double c, float* out, void* stream);
hgs_status hgs_nn_compose(const float* phi_c, const float* y, const float* scale, int32_t B, int64_t nvox,
                          double inv_out_scale, float* phi, float* phidot, void* stream);
/* Adam with bias correction (step t >= 1) on FP32 master parameters; p16
 * (nullable) receives their bfloat16 copy. */
hgs_status hgs_nn_adam(float* p, float* m, float* v, const float* g, uint16_t* p16, int32_t n, float lr, float b1,
                       float b2, float eps, int32_t t, void* stream);
/* [B][2cz][2cy][2cx] <-> [B][cz][cy][cx]: 2x2x2 mean restriction, and
 * cell-centred trilinear prolongation (weights 3/4, 1/4 per axis; linear
 * extrapolation, 5/4 and -1/4, at the faces).  dtype: hgs_dtype. */
hgs_status hgs_nn_restrict2(const void* fine, void* coarse, int32_t B, int32_t cz, int32_t cy, int32_t cx,
                            int32_t dtype, void* stream);
hgs_status hgs_nn_prolong2(const void* coarse, void* fine, int32_t B, int32_t cz, int32_t cy, int32_t cx,
                           int32_t dtype, void* stream);
/* Reason for the last non-OK status of an hgs_nn_* call on this thread. */
const char* hgs_nn_last_error(void);

/* ---- Autotuner -------------------------------------------------------------
 * Picks the fused depth (substeps per stencil launch) and the tile shape for a
 * configuration by timing whole hydrodynamical steps, hgs_step(rho, c_g, dt,
 * nsub), with HIP events for every depth 1..HGS_TMAX and every tile shape
 * compiled for it (two passes, the second in reverse order, each candidate
 * keeping its faster time), on a temporary context built over the caller's workspace
 * (hgs_workspace_bytes(cfg) bytes; its contents are overwritten).
 * Synchronises.
 * *best_tblock receives the fastest depth, *best_tile
 * (nullable) its tile index (for hgs_set_tile); ms_per_substep (nullable,
 * HGS_TMAX entries) the best measured time per substep for each depth
 * 1..HGS_TMAX.  If the environment variable HGS_TUNE_CACHE names a file,
 * results are cached there per (device architecture, nx, ny, nz, storage,
 * nsub, bc) as (depth, tile) and a cached entry is returned without timing
 * (times set to -1). */
hgs_status hgs_autotune(const hgs_config* cfg, const void* rho, double c_g, double dt, int32_t nsub,
                        void* workspace, size_t bytes, int32_t* best_tblock, int32_t* best_tile,
                        double* ms_per_substep);

/* Release the host context (the workspace stays the caller's).  NULL is a no-op. */
hgs_status hgs_destroy(hgs_ctx* ctx);

const char* hgs_status_str(hgs_status s);
/* Reason for the last non-OK status of this context ("" if none; for a NULL
 * context, the last failure of hgs_init/hgs_workspace_bytes on this thread). */
const char* hgs_last_error(const hgs_ctx* ctx);

/* ABI version, bumped on incompatible changes. */
int32_t hgs_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HGS_H */
