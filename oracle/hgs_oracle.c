/*
 * Oracle core -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, slow, obviously correct FP64 CPU implementation of what the
 * hyperbolic self-gravity hot path computes (Hirai, Nagakura, Okawa &
 * Fujisawa, "Hyperbolic Self-Gravity Solver for Large Scale Hydrodynamical
 * Simulations", arXiv:1602.05700).  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code with
 * the HIP library: no header, no table, no helper.
 *
 * Grid convention (the paper fixes none; the readings are listed in the design
 * notes): cell-centred uniform grid, interior cell (i,j,k) sits at
 * x0+(i+1/2)dx, y0+(j+1/2)dx, z0+(k+1/2)dx.  One ghost layer lies one cell
 * outside each face.  The oracle keeps every 3D field in its own padded
 * array of shape (nz+2, ny+2, nx+2), x fastest; interior cell (i,j,k) lives
 * at padded index ((k+1)*(ny+2)+(j+1))*(nx+2)+(i+1).  Edge and corner cells
 * of the padding are never read.
 *
 * Functions:
 *   orc_moments    multipole moments of rho (Sec. 2 / Sec. 4: Dirichlet
 *                  boundary from a multipole expansion), complex orthonormal
 *                  Y_lm written out from the textbook definition.
 *   orc_boundary   ghost values phi_b = -G sum_lm 4pi/(2l+1) Q_lm Y_lm / r^(l+1).
 *   orc_substeps   explicit leapfrog time stepping of Eq. (2), optionally with a
 *                  damping term eta*dphi/dt (an extension; eta = 0 is Eq. (2)).
 *   orc_laplacian  the 7-point Laplacian with ghosts, L_h phi.
 *   orc_gradient   g = -grad phi by central differences.
 *   orc_residual   residual norms of L_h phi = 4 pi G rho.
 *   orc_substeps_local, orc_local_ghosts, orc_residual_local
 *                  the same with a local outer boundary (Robin, outgoing,
 *                  periodic) whose ghosts follow the interior every substep.
 *
 * Parity status of every function is listed in oracle/__init__.py.
 */
#include <math.h>
#include <omp.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

static inline size_t pidx(int nx, int ny, int i, int j, int k) {
    /* padded index of cell (i,j,k); i,j,k may be -1 or n (ghosts) */
    return ((size_t)(k + 1) * (size_t)(ny + 2) + (size_t)(j + 1)) * (size_t)(nx + 2) + (size_t)(i + 1);
}

/* ---------------------------------------------------------------------------
 * Spherical harmonics, textbook definition (Condon-Shortley phase):
 *   Y_lm(theta,phi) = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) P_l^m(cos theta) e^{i m phi},  m >= 0
 *   Y_l,-m = (-1)^m conj(Y_lm)
 * P_l^m from P_m^m = (-1)^m (2m-1)!! (1-x^2)^{m/2},  P_{m+1}^m = x (2m+1) P_m^m,
 * (l-m) P_l^m = x (2l-1) P_{l-1}^m - (l+m-1) P_{l-2}^m.
 * Output index: l*l + (m+l), m = -l..l.
 * ------------------------------------------------------------------------- */
static double factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return f;
}

static double assoc_legendre(int l, int m, double x) {
    /* m >= 0, l >= m */
    double pmm = 1.0;
    double s = sqrt(fmax(0.0, 1.0 - x * x));
    for (int i = 1; i <= m; ++i) pmm *= -(2.0 * i - 1.0) * s;
    if (l == m) return pmm;
    double pm1 = x * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return pm1;
    double pl = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pl = (x * (2.0 * ll - 1.0) * pm1 - (ll + m - 1.0) * pmm) / (double)(ll - m);
        pmm = pm1;
        pm1 = pl;
    }
    return pl;
}

/* all Y_lm for l <= lmax at direction (cos theta, phi) */
static void ylm_all(int lmax, double ct, double ph, double* re, double* im) {
    for (int l = 0; l <= lmax; ++l) {
        for (int m = 0; m <= l; ++m) {
            double norm = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - m) / factorial(l + m));
            double p = assoc_legendre(l, m, ct);
            double yr = norm * p * cos(m * ph);
            double yi = norm * p * sin(m * ph);
            re[l * l + l + m] = yr;
            im[l * l + l + m] = yi;
            if (m > 0) {
                double sg = (m % 2) ? -1.0 : 1.0;
                re[l * l + l - m] = sg * yr;
                im[l * l + l - m] = -sg * yi;
            }
        }
    }
}

/* Spherical coordinates of x about the origin.  At r = 0 the direction is
 * taken as the +z axis (only r^0 Y_00 survives there). */
static void to_spherical(double x, double y, double z, double* r, double* ct, double* ph) {
    *r = sqrt(x * x + y * y + z * z);
    if (*r > 0.0) {
        *ct = z / *r;
        *ph = atan2(y, x);
    } else {
        *ct = 1.0;
        *ph = 0.0;
    }
}

/* Q_lm = sum over interior cells of rho dx^3 r^l conj(Y_lm(theta, phi)),
 * positions relative to origin[3].  rho is COMPACT (nz, ny, nx), x fastest. */
void orc_moments(int nx, int ny, int nz, double x0, double y0, double z0, double dx,
                 const double* origin, int lmax, const double* rho,
                 double* q_re, double* q_im) {
    int nq = (lmax + 1) * (lmax + 1);
    double dv = dx * dx * dx;
    /* one partial sum per z-plane, added up in plane order afterwards */
    double* part = (double*)calloc((size_t)nz * 2 * nq, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k) {
        double zr[25], zi[25];
        double* acc_re = part + (size_t)k * 2 * nq;
        double* acc_im = acc_re + nq;
        for (int j = 0; j < ny; ++j) {
            for (int i = 0; i < nx; ++i) {
                double m = rho[((size_t)k * ny + j) * nx + i] * dv;
                if (m == 0.0) continue;
                double x = x0 + (i + 0.5) * dx - origin[0];
                double y = y0 + (j + 0.5) * dx - origin[1];
                double z = z0 + (k + 0.5) * dx - origin[2];
                double r, ct, ph;
                to_spherical(x, y, z, &r, &ct, &ph);
                ylm_all(lmax, ct, ph, zr, zi);
                double rl = 1.0;
                for (int l = 0; l <= lmax; ++l) {
                    for (int mm = -l; mm <= l; ++mm) {
                        int q = l * l + l + mm;
                        acc_re[q] += m * rl * zr[q];
                        acc_im[q] -= m * rl * zi[q]; /* conjugate */
                    }
                    rl *= r;
                }
            }
        }
    }
    for (int q = 0; q < nq; ++q) { q_re[q] = 0.0; q_im[q] = 0.0; }
    for (int k = 0; k < nz; ++k)
        for (int q = 0; q < nq; ++q) {
            q_re[q] += part[(size_t)k * 2 * nq + q];
            q_im[q] += part[(size_t)k * 2 * nq + nq + q];
        }
    free(part);
}

/* Multipole potential at one point outside the mass. */
static double multipole_phi(int lmax, double G, const double* q_re, const double* q_im,
                            double x, double y, double z) {
    double r, ct, ph;
    double yr[25], yi[25];
    to_spherical(x, y, z, &r, &ct, &ph);
    ylm_all(lmax, ct, ph, yr, yi);
    double sum = 0.0;
    double rinv = 1.0 / r;
    double rpow = rinv; /* 1/r^(l+1) */
    for (int l = 0; l <= lmax; ++l) {
        double pref = 4.0 * M_PI / (2.0 * l + 1.0);
        for (int mm = -l; mm <= l; ++mm) {
            int q = l * l + l + mm;
            /* real part of Q_lm * Y_lm */
            sum += pref * (q_re[q] * yr[q] - q_im[q] * yi[q]) * rpow;
        }
        rpow *= rinv;
    }
    return -G * sum;
}

/* Fill the six ghost faces of the padded array phi with the multipole
 * potential (one layer outside each face, at ghost-cell centres). */
void orc_boundary(int nx, int ny, int nz, double x0, double y0, double z0, double dx,
                  const double* origin, int lmax, double G,
                  const double* q_re, const double* q_im, double* phi) {
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) {
            double y = y0 + (j + 0.5) * dx - origin[1];
            double z = z0 + (k + 0.5) * dx - origin[2];
            phi[pidx(nx, ny, -1, j, k)] = multipole_phi(lmax, G, q_re, q_im, x0 - 0.5 * dx - origin[0], y, z);
            phi[pidx(nx, ny, nx, j, k)] = multipole_phi(lmax, G, q_re, q_im, x0 + (nx + 0.5) * dx - origin[0], y, z);
        }
    for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nx; ++i) {
            double x = x0 + (i + 0.5) * dx - origin[0];
            double z = z0 + (k + 0.5) * dx - origin[2];
            phi[pidx(nx, ny, i, -1, k)] = multipole_phi(lmax, G, q_re, q_im, x, y0 - 0.5 * dx - origin[1], z);
            phi[pidx(nx, ny, i, ny, k)] = multipole_phi(lmax, G, q_re, q_im, x, y0 + (ny + 0.5) * dx - origin[1], z);
        }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double x = x0 + (i + 0.5) * dx - origin[0];
            double y = y0 + (j + 0.5) * dx - origin[1];
            phi[pidx(nx, ny, i, j, -1)] = multipole_phi(lmax, G, q_re, q_im, x, y, z0 - 0.5 * dx - origin[2]);
            phi[pidx(nx, ny, i, j, nz)] = multipole_phi(lmax, G, q_re, q_im, x, y, z0 + (nz + 0.5) * dx - origin[2]);
        }
}

/* L_h phi at interior cells: (sum of the six neighbours - 6 phi) / dx^2,
 * neighbours outside the interior being ghosts.  out is COMPACT. */
void orc_laplacian(int nx, int ny, int nz, double dx, const double* phi, double* out) {
    double idx2 = 1.0 / (dx * dx);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double c = phi[pidx(nx, ny, i, j, k)];
                double nb = phi[pidx(nx, ny, i - 1, j, k)] + phi[pidx(nx, ny, i + 1, j, k)]
                          + phi[pidx(nx, ny, i, j - 1, k)] + phi[pidx(nx, ny, i, j + 1, k)]
                          + phi[pidx(nx, ny, i, j, k - 1)] + phi[pidx(nx, ny, i, j, k + 1)];
                out[((size_t)k * ny + j) * nx + i] = (nb - 6.0 * c) * idx2;
            }
}

/* copy the six ghost faces of src into dst (padded layout) */
static void copy_ghosts(int nx, int ny, int nz, const double* src, double* dst) {
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) {
            dst[pidx(nx, ny, -1, j, k)] = src[pidx(nx, ny, -1, j, k)];
            dst[pidx(nx, ny, nx, j, k)] = src[pidx(nx, ny, nx, j, k)];
        }
    for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nx; ++i) {
            dst[pidx(nx, ny, i, -1, k)] = src[pidx(nx, ny, i, -1, k)];
            dst[pidx(nx, ny, i, ny, k)] = src[pidx(nx, ny, i, ny, k)];
        }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            dst[pidx(nx, ny, i, j, -1)] = src[pidx(nx, ny, i, j, -1)];
            dst[pidx(nx, ny, i, j, nz)] = src[pidx(nx, ny, i, j, nz)];
        }
}

static inline double round_storage(double v, int f32) {
    return f32 ? (double)(float)v : v;
}

/* One substep of Eq. (2) at every interior cell, reading cur (with ghosts)
 * and old, writing nxt:
 *   (phi^{n+1} - 2 phi^n + phi^{n-1}) / dt^2 + eta (phi^{n+1} - phi^{n-1}) / (2 dt)
 *       = c^2 (L_h phi^n - 4 pi G (rho - rbar))
 * solved for phi^{n+1}.  eta = 0 is the paper's equation; rbar is the mean
 * density subtracted from the source on a periodic domain (Sec. 4), else 0. */
static void leapfrog_interior(int nx, int ny, int nz, double dx, const double* cur, const double* old,
                              double* nxt, const double* rho, double rbar, double c, double dt, double eta,
                              double G, int f32) {
    double a = 0.5 * eta * dt;
    double c2dt2 = c * c * dt * dt;
    double idx2 = 1.0 / (dx * dx);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t p = pidx(nx, ny, i, j, k);
                double ph = cur[p];
                double lap = (cur[pidx(nx, ny, i - 1, j, k)] + cur[pidx(nx, ny, i + 1, j, k)]
                            + cur[pidx(nx, ny, i, j - 1, k)] + cur[pidx(nx, ny, i, j + 1, k)]
                            + cur[pidx(nx, ny, i, j, k - 1)] + cur[pidx(nx, ny, i, j, k + 1)]
                            - 6.0 * ph) * idx2;
                double s = 4.0 * M_PI * G * (rho[((size_t)k * ny + j) * nx + i] - rbar);
                double v = (2.0 * ph - (1.0 - a) * old[p] + c2dt2 * (lap - s)) / (1.0 + a);
                nxt[p] = round_storage(v, f32);
            }
}

/* after a run of substeps the newest level is in cur and the previous in old,
 * both among {phi_n, phi_nm1, spare}: copy them into the caller's arrays */
static void copy_home(size_t np, double* cur, double* old, double* phi_n, double* phi_nm1) {
    if (cur != phi_n) {
        double* tmp_cur = (double*)malloc(np * sizeof(double));
        double* tmp_old = (double*)malloc(np * sizeof(double));
        memcpy(tmp_cur, cur, np * sizeof(double));
        memcpy(tmp_old, old, np * sizeof(double));
        memcpy(phi_n, tmp_cur, np * sizeof(double));
        memcpy(phi_nm1, tmp_old, np * sizeof(double));
        free(tmp_cur);
        free(tmp_old);
    } else if (old != phi_nm1) {
        memcpy(phi_nm1, old, np * sizeof(double));
    }
}

/* nsub explicit substeps of Eq. (2), rho frozen (Sec. 2: the wave equation is
 * sub-cycled within one hydrodynamical step), with a fixed (Dirichlet) ghost
 * layer.  phi_n / phi_nm1: padded arrays, in/out; their ghost values are the
 * frozen boundary: the ghosts of phi_n are used and copied into phi_nm1.
 * rho: COMPACT.  If f32 != 0 every new level is rounded to binary32 (emulates
 * FP32 storage; arithmetic stays FP64). */
void orc_substeps(int nx, int ny, int nz, double dx, double* phi_n, double* phi_nm1,
                  const double* rho, double c, double dt, double eta, double G, int nsub, int f32) {
    size_t np = (size_t)(nx + 2) * (ny + 2) * (nz + 2);
    double* cur = phi_n;
    double* old = phi_nm1;
    double* nxt = (double*)malloc(np * sizeof(double));
    double* spare = nxt;
    copy_ghosts(nx, ny, nz, phi_n, phi_nm1);
    memcpy(nxt, phi_n, np * sizeof(double)); /* carries the ghosts */
    for (int n = 0; n < nsub; ++n) {
        leapfrog_interior(nx, ny, nz, dx, cur, old, nxt, rho, 0.0, c, dt, eta, G, f32);
        /* rotate: old <- cur, cur <- nxt, nxt <- old's storage */
        double* t = old;
        old = cur;
        cur = nxt;
        nxt = t;
    }
    copy_home(np, cur, old, phi_n, phi_nm1);
    free(spare);
}

/* ---------------------------------------------------------------------------
 * Local outer boundaries (the ghost layer follows the interior every substep).
 *
 * 2 = Robin: the paper's default outer boundary, a Robin condition that
 *     is equivalent to a monopole far field (Sec. 2, Sec. 4).  Read as the
 *     monopole fall-off d(r phi)/dr = 0 between a ghost and the interior cell
 *     next to it:  r_g phi_g = r_i phi_i,  r measured from the expansion
 *     centre.  Exact for any potential -G M / r about that centre.
 * 3 = outgoing: the radiative form of the same condition, an outgoing
 *     spherical wave  d(r phi)/dt + c d(r phi)/dr = 0, which lets errors
 *     leave the domain through the boundary (Sec. 4).  With u = r phi and the
 *     radial derivative taken along the face normal, d/dr = d/dn / cos(theta),
 *     cos(theta) = n . x_f / |x_f| at the midpoint x_f of ghost and neighbour,
 *     the condition is discretised by the box scheme centred on that midpoint
 *     and on t^{n+1/2}:
 *       (u_g^{n+1} + u_i^{n+1} - u_g^n - u_i^n) / (2 dt)
 *         + c (u_g^{n+1} - u_i^{n+1} + u_g^n - u_i^n) / (2 dx cos(theta)) = 0.
 *     Its steady state is the Robin relation above.
 * 4 = periodic: ghost = the interior cell on the opposite face; the source
 *     uses rho minus its mean over the domain (Sec. 4).
 * ------------------------------------------------------------------------- */
#define ORC_BC_ROBIN 2
#define ORC_BC_OUTGOING 3
#define ORC_BC_PERIODIC 4

typedef struct {
    int nx, ny, nz;
    double x0, y0, z0, dx, ox, oy, oz;
} orc_geom;

static void centre(const orc_geom* g, const int c[3], double x[3]) {
    x[0] = g->x0 + (c[0] + 0.5) * g->dx - g->ox;
    x[1] = g->y0 + (c[1] + 0.5) * g->dx - g->oy;
    x[2] = g->z0 + (c[2] + 0.5) * g->dx - g->oz;
}

/* face f (0..5 = x-, x+, y-, y+, z-, z+), in-face cell (a, b) in the face
 * layout (x faces: a = j, b = k; y faces: a = i, b = k; z faces: a = i, b = j):
 * the ghost cell, its interior neighbour, the interior cell on the opposite
 * face, and the outward normal */
static void face_cells(const orc_geom* g, int f, int a, int b, int gh[3], int in[3], int opp[3], int nrm[3]) {
    int axis = f / 2, hi = f % 2;
    int n[3] = {g->nx, g->ny, g->nz};
    int c[3] = {0, 0, 0};
    if (axis == 0) { c[1] = a; c[2] = b; }
    else if (axis == 1) { c[0] = a; c[2] = b; }
    else { c[0] = a; c[1] = b; }
    for (int d = 0; d < 3; ++d) {
        gh[d] = in[d] = opp[d] = c[d];
        nrm[d] = 0;
    }
    gh[axis] = hi ? n[axis] : -1;
    in[axis] = hi ? n[axis] - 1 : 0;
    opp[axis] = hi ? 0 : n[axis] - 1;
    nrm[axis] = hi ? 1 : -1;
}

static void face_extent(const orc_geom* g, int f, int* na, int* nb) {
    int axis = f / 2;
    *na = axis == 0 ? g->ny : g->nx;
    *nb = axis == 2 ? g->ny : g->nz;
}

/* Write the ghost layer of nxt from its interior.  cur (the previous level,
 * with its ghosts) is read by the outgoing rule only; cur == NULL applies the
 * rule's steady form (Robin for bc 2 and 3). */
static void local_ghosts(const orc_geom* g, int bc, double* nxt, const double* cur, double c, double dt, int f32) {
    for (int f = 0; f < 6; ++f) {
        int na, nb;
        face_extent(g, f, &na, &nb);
        for (int b = 0; b < nb; ++b)
            for (int a = 0; a < na; ++a) {
                int gh[3], in[3], opp[3], nrm[3];
                face_cells(g, f, a, b, gh, in, opp, nrm);
                size_t pg = pidx(g->nx, g->ny, gh[0], gh[1], gh[2]);
                size_t pi = pidx(g->nx, g->ny, in[0], in[1], in[2]);
                if (bc == ORC_BC_PERIODIC) {
                    nxt[pg] = nxt[pidx(g->nx, g->ny, opp[0], opp[1], opp[2])];
                    continue;
                }
                double xg[3], xi[3];
                centre(g, gh, xg);
                centre(g, in, xi);
                double rg = sqrt(xg[0] * xg[0] + xg[1] * xg[1] + xg[2] * xg[2]);
                double ri = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
                double v;
                if (bc == ORC_BC_ROBIN || cur == NULL) {
                    v = ri * nxt[pi] / rg;
                } else {
                    double xf[3] = {0.5 * (xg[0] + xi[0]), 0.5 * (xg[1] + xi[1]), 0.5 * (xg[2] + xi[2])};
                    double rf = sqrt(xf[0] * xf[0] + xf[1] * xf[1] + xf[2] * xf[2]);
                    double cth = (nrm[0] * xf[0] + nrm[1] * xf[1] + nrm[2] * xf[2]) / rf;
                    double al = c * dt / (g->dx * cth);
                    double ug0 = rg * cur[pg], ui0 = ri * cur[pi], ui1 = ri * nxt[pi];
                    double ug1 = ((1.0 - al) * ug0 + (1.0 + al) * ui0 - (1.0 - al) * ui1) / (1.0 + al);
                    v = ug1 / rg;
                }
                nxt[pg] = round_storage(v, f32);
            }
    }
}

/* The steady form of a local rule (Robin for bc 2 and 3, the wrap for 4)
 * applied to the ghost layer of a padded array, in place. */
void orc_local_ghosts(int nx, int ny, int nz, double x0, double y0, double z0, double dx, const double* origin,
                      int bc, double* phi, int f32) {
    orc_geom g = {nx, ny, nz, x0, y0, z0, dx, origin[0], origin[1], origin[2]};
    local_ghosts(&g, bc, phi, NULL, 0.0, 0.0, f32);
}

/* nsub substeps of Eq. (2) with a local outer boundary bc (2, 3 or 4): after
 * each interior update the new level's ghosts follow the rule above.  rbar is
 * subtracted from rho in the source (the caller passes the domain mean for
 * bc = 4, else 0).  Arguments as for orc_substeps; the ghosts of phi_n must
 * hold the current level's boundary values. */
void orc_substeps_local(int nx, int ny, int nz, double x0, double y0, double z0, double dx, const double* origin,
                        int bc, double* phi_n, double* phi_nm1, const double* rho, double rbar, double c, double dt,
                        double eta, double G, int nsub, int f32) {
    orc_geom g = {nx, ny, nz, x0, y0, z0, dx, origin[0], origin[1], origin[2]};
    size_t np = (size_t)(nx + 2) * (ny + 2) * (nz + 2);
    double* cur = phi_n;
    double* old = phi_nm1;
    double* nxt = (double*)calloc(np, sizeof(double));
    double* spare = nxt;
    for (int n = 0; n < nsub; ++n) {
        leapfrog_interior(nx, ny, nz, dx, cur, old, nxt, rho, rbar, c, dt, eta, G, f32);
        local_ghosts(&g, bc, nxt, cur, c, dt, f32);
        double* t = old;
        old = cur;
        cur = nxt;
        nxt = t;
    }
    copy_home(np, cur, old, phi_n, phi_nm1);
    free(spare);
}

/* g = -grad phi, central differences with ghosts at the faces; outputs COMPACT. */
void orc_gradient(int nx, int ny, int nz, double dx, const double* phi,
                  double* gx, double* gy, double* gz) {
    double h = 1.0 / (2.0 * dx);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t o = ((size_t)k * ny + j) * nx + i;
                gx[o] = -(phi[pidx(nx, ny, i + 1, j, k)] - phi[pidx(nx, ny, i - 1, j, k)]) * h;
                gy[o] = -(phi[pidx(nx, ny, i, j + 1, k)] - phi[pidx(nx, ny, i, j - 1, k)]) * h;
                gz[o] = -(phi[pidx(nx, ny, i, j, k + 1)] - phi[pidx(nx, ny, i, j, k - 1)]) * h;
            }
}

/* Residual of the discrete Poisson problem L_h phi = s, s = 4 pi G rho.
 * The linear system for the interior unknowns is A phi = b with the ghost
 * values moved to the right-hand side: b = s - (sum of adjacent ghosts)/dx^2.
 * out[0] = ||L_h phi - s|| / ||b||   (1 at phi = 0)
 * out[1] = ||L_h phi - s|| / ||s||
 * out[2] = ||phi||  (interior, 2-norm)
 * out[3] = 1 if any interior value of phi or rho is not finite, else 0
 * A zero denominator gives 0 when the numerator is 0 and +inf otherwise. */
static void residual_core(int nx, int ny, int nz, double dx, const double* phi, const double* rho, double G,
                          double rbar, int ghosts_in_b, double* out) {
    double rr = 0.0, bb = 0.0, ss = 0.0, pp = 0.0;
    int bad = 0;
    double idx2 = 1.0 / (dx * dx);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double c = phi[pidx(nx, ny, i, j, k)];
                double nb = 0.0, gb = 0.0;
                int ii[6] = {i - 1, i + 1, i, i, i, i};
                int jj[6] = {j, j, j - 1, j + 1, j, j};
                int kk[6] = {k, k, k, k, k - 1, k + 1};
                for (int q = 0; q < 6; ++q) {
                    double v = phi[pidx(nx, ny, ii[q], jj[q], kk[q])];
                    nb += v;
                    int ghost = ii[q] < 0 || ii[q] >= nx || jj[q] < 0 || jj[q] >= ny || kk[q] < 0 || kk[q] >= nz;
                    if (ghost) gb += v;
                }
                double rhov = rho[((size_t)k * ny + j) * nx + i];
                double s = 4.0 * M_PI * G * (rhov - rbar);
                double r = (nb - 6.0 * c) * idx2 - s;
                double b = ghosts_in_b ? s - gb * idx2 : s;
                rr += r * r;
                bb += b * b;
                ss += s * s;
                pp += c * c;
                if (!isfinite(c) || !isfinite(rhov)) bad = 1;
            }
    double rn = sqrt(rr);
    out[0] = bb > 0.0 ? rn / sqrt(bb) : (rn == 0.0 ? 0.0 : INFINITY);
    out[1] = ss > 0.0 ? rn / sqrt(ss) : (rn == 0.0 ? 0.0 : INFINITY);
    out[2] = sqrt(pp);
    out[3] = bad ? 1.0 : 0.0;
}

void orc_residual(int nx, int ny, int nz, double dx, const double* phi, const double* rho,
                  double G, double* out) {
    residual_core(nx, ny, nz, dx, phi, rho, G, 0.0, 1, out);
}

/* The same norms for a local outer boundary: the ghosts are images of interior
 * unknowns, so the right-hand side is b = s alone (R_b = R_f), and the source
 * is s = 4 pi G (rho - rbar). */
void orc_residual_local(int nx, int ny, int nz, double dx, const double* phi, const double* rho,
                        double G, double rbar, double* out) {
    residual_core(nx, ny, nz, dx, phi, rho, G, rbar, 0, out);
}

int orc_abi_version(void) { return 1; }

int orc_max_threads(void) { return omp_get_max_threads(); }
/* threads for the following parallel loops of the calling thread (n >= 1) */
void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
