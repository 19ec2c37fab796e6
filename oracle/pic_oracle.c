/*
 * FP64 CPU oracle for the relativistic 3D3V particle-in-cell cycle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source with the HIP library.
 *
 * The paper names the methods of its benchmark run (section "Evaluation",
 * the Kelvin-Helmholtz setup): Boris pusher, Esirkepov current solver, Yee
 * field solver, separable ("trilinear") interpolation in field gathering,
 * 3D3V, and quadratic-spline (TSC) particle shape.  It prints no formula, so
 * every routine below is the textbook definition of the named method:
 *   - CIC / TSC assignment functions (Hockney & Eastwood, cited there), and
 *     the cubic B-spline (PCS) of the same family as a further shape,
 *   - relativistic Boris rotation (Boris 1970; Birdsall & Langdon),
 *   - Esirkepov charge-conserving current (Comput. Phys. Commun. 135, 2001),
 *   - Yee staggered-grid FDTD (IEEE Trans. Antennas Propag. 14, 1966),
 *   - Philox4x64-10 counter-based generator (Salmon et al., SC'11).
 * It is deliberately plain: global FP64 arrays, global positions in cell
 * units, periodic index wrapping, no tiling, no supercells, no fusion.
 *
 * Units: c = eps0 = 1, e = m_e = 1, n0 = 1 (so omega_p = 1).  Positions are
 * in cell units along each axis; momenta are u = gamma*v/c.
 *
 * Field layout: comp * N + idx, idx = i + nx*(j + ny*k), N = nx*ny*nz.
 * Yee locations: Ex (i+1/2,j,k), Ey (i,j+1/2,k), Ez (i,j,k+1/2),
 *                Bx (i,j+1/2,k+1/2), By (i+1/2,j,k+1/2), Bz (i+1/2,j+1/2,k).
 * J shares the locations of E; rho lives on nodes (i,j,k).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nx, ny, nz, order; /* order 1 = CIC, 2 = TSC, 3 = PCS */
    double dx, dy, dz, dt;
    double b0[3];   /* uniform background B, added at gather time only */
    double rho_bg;  /* immobile neutralising background charge density */
    int32_t gather; /* 0: every axis with the shape's order; 1: Galerkin, one
                       order lower along each of a component's staggered axes */
    int32_t pad;
} orc_grid;

typedef struct {
    int64_t n;
    double *x, *y, *z, *ux, *uy, *uz, *w;
    int64_t *id;
    int32_t *zstate; /* charge state per particle, or NULL */
    double q;        /* charge in e; multiplied by zstate when present */
    double m;        /* mass in m_e */
    int32_t mobile;
} orc_particles;

/* ------------------------------------------------------------------------ */
/* Philox4x64-10, as defined by Salmon, Moraes, Dror & Shaw (SC'11):
 * ten rounds of two 64x64->128 multiplies with a Weyl-sequence key bump. */

static const uint64_t PHX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHX_W0 = 0x9E3779B97F4A7C15ULL;
static const uint64_t PHX_W1 = 0xBB67AE8584CAA73BULL;

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += PHX_W0; k1 += PHX_W1; }
        __uint128_t p0 = (__uint128_t)PHX_M0 * c0;
        __uint128_t p1 = (__uint128_t)PHX_M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in the open interval (0,1) from the top 53 bits of a word. */
double orc_u01(uint64_t word)
{
    return ((double)(word >> 11) + 0.5) * 0x1.0p-53;
}

/* Counter layout: (particle id, species, purpose, step); key = (seed, 0).
 * Purposes: 0 position, 1 momentum, 2 ionisation draw. */
static void draw4(uint64_t seed, uint64_t id, uint64_t species, uint64_t purpose,
                  uint64_t step, double u[4])
{
    uint64_t ctr[4] = {id, species, purpose, step}, key[2] = {seed, 0}, o[4];
    orc_philox4x64_10(ctr, key, o);
    for (int i = 0; i < 4; ++i) u[i] = orc_u01(o[i]);
}

/* ------------------------------------------------------------------------ */
/* Assignment functions (Hockney & Eastwood), delta in cell units. */

double orc_shape(int order, double d)
{
    double a = fabs(d);
    if (order == 0) return (d >= -0.5 && d < 0.5) ? 1.0 : 0.0; /* NGP; a tie goes to the upper node */
    if (order == 1) return a < 1.0 ? 1.0 - a : 0.0;
    if (order == 3) {  /* cubic B-spline (PCS) */
        if (a < 1.0) return (4.0 - 6.0 * a * a + 3.0 * a * a * a) / 6.0;
        if (a < 2.0) { double t = 2.0 - a; return t * t * t / 6.0; }
        return 0.0;
    }
    if (a <= 0.5) return 0.75 - a * a;
    if (a < 1.5) { double t = 1.5 - a; return 0.5 * t * t; }
    return 0.0;
}

static inline int64_t wrapi(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

static inline int64_t gidx(const orc_grid* g, int64_t i, int64_t j, int64_t k)
{
    return wrapi(i, g->nx) + (int64_t)g->nx * (wrapi(j, g->ny) + (int64_t)g->ny * wrapi(k, g->nz));
}

static inline int64_t ncell(const orc_grid* g)
{
    return (int64_t)g->nx * g->ny * g->nz;
}

/* Field interpolation at one point: sum over all nodes in reach of the
 * shape, weight Sx*Sy*Sz, with the component's own half-cell offsets.  In
 * the Galerkin gather an axis along which the component is staggered uses
 * the shape one order lower. */
static double interp(const orc_grid* g, const double* f, double x, double y, double z,
                     double ox, double oy, double oz)
{
    double px = x - ox, py = y - oy, pz = z - oz;
    int64_t bx = (int64_t)floor(px), by = (int64_t)floor(py), bz = (int64_t)floor(pz);
    const int qx = (g->gather && ox != 0.0) ? g->order - 1 : g->order;
    const int qy = (g->gather && oy != 0.0) ? g->order - 1 : g->order;
    const int qz = (g->gather && oz != 0.0) ? g->order - 1 : g->order;
    double acc = 0.0;
    for (int64_t k = bz - 2; k <= bz + 3; ++k) {
        double sz = orc_shape(qz, pz - (double)k);
        if (sz == 0.0) continue;
        for (int64_t j = by - 2; j <= by + 3; ++j) {
            double sy = orc_shape(qy, py - (double)j);
            if (sy == 0.0) continue;
            for (int64_t i = bx - 2; i <= bx + 3; ++i) {
                double sx = orc_shape(qx, px - (double)i);
                if (sx == 0.0) continue;
                acc += sx * sy * sz * f[gidx(g, i, j, k)];
            }
        }
    }
    return acc;
}

/* Gather E and B (B includes the uniform b0) at n points.  Out: 3 per point. */
void orc_gather(const orc_grid* g, const double* E, const double* B, int64_t n,
                const double* x, const double* y, const double* z, double* Ep, double* Bp)
{
    const int64_t N = ncell(g);
    for (int64_t p = 0; p < n; ++p) {
        Ep[3 * p + 0] = interp(g, E + 0 * N, x[p], y[p], z[p], 0.5, 0.0, 0.0);
        Ep[3 * p + 1] = interp(g, E + 1 * N, x[p], y[p], z[p], 0.0, 0.5, 0.0);
        Ep[3 * p + 2] = interp(g, E + 2 * N, x[p], y[p], z[p], 0.0, 0.0, 0.5);
        Bp[3 * p + 0] = interp(g, B + 0 * N, x[p], y[p], z[p], 0.0, 0.5, 0.5) + g->b0[0];
        Bp[3 * p + 1] = interp(g, B + 1 * N, x[p], y[p], z[p], 0.5, 0.0, 0.5) + g->b0[1];
        Bp[3 * p + 2] = interp(g, B + 2 * N, x[p], y[p], z[p], 0.5, 0.5, 0.0) + g->b0[2];
    }
}

/* ------------------------------------------------------------------------ */
/* Relativistic Boris push for one particle: half electric kick, magnetic
 * rotation through t = (q dt / 2 m gamma-) B and s = 2t/(1+t^2), second half
 * kick.  qm = q/m, u = gamma v. */
static void boris1(double qm, double dt, const double* E, const double* B, double u[3])
{
    double h = 0.5 * qm * dt;
    double um[3] = {u[0] + h * E[0], u[1] + h * E[1], u[2] + h * E[2]};
    double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    double t[3] = {h * B[0] / gm, h * B[1] / gm, h * B[2] / gm};
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    double s[3] = {2.0 * t[0] / (1.0 + t2), 2.0 * t[1] / (1.0 + t2), 2.0 * t[2] / (1.0 + t2)};
    double up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]),
                    um[1] + (um[2] * t[0] - um[0] * t[2]),
                    um[2] + (um[0] * t[1] - um[1] * t[0])};
    double uplus[3] = {um[0] + (up[1] * s[2] - up[2] * s[1]),
                       um[1] + (up[2] * s[0] - up[0] * s[2]),
                       um[2] + (up[0] * s[1] - up[1] * s[0])};
    u[0] = uplus[0] + h * E[0];
    u[1] = uplus[1] + h * E[1];
    u[2] = uplus[2] + h * E[2];
}

void orc_boris(int64_t n, const double* qm, double dt, const double* Ep, const double* Bp,
               double* ux, double* uy, double* uz)
{
    for (int64_t p = 0; p < n; ++p) {
        double u[3] = {ux[p], uy[p], uz[p]};
        boris1(qm[p], dt, Ep + 3 * p, Bp + 3 * p, u);
        ux[p] = u[0]; uy[p] = u[1]; uz[p] = u[2];
    }
}

/* ------------------------------------------------------------------------ */
/* Esirkepov current of one particle moving x0 -> x1 (unwrapped positions,
 * cell units, |x1-x0| < 1 per axis).  Adds into J (layout of E).
 * qw = charge * weight of the macro-particle. */
static int first_node(int order, double x)
{
    if (order == 1) return (int)floor(x);
    if (order == 3) return (int)floor(x) - 1;
    return (int)floor(x + 0.5) - 1;
}

static void esirkepov1(const orc_grid* g, double qw, const double x0[3], const double x1[3], double* J)
{
    const int W = g->order + 2;
    const double dl[3] = {g->dx, g->dy, g->dz};
    const double dV = g->dx * g->dy * g->dz;
    const int64_t N = ncell(g);
    int m[3];
    double S0[3][5], DS[3][5];
    for (int d = 0; d < 3; ++d) {
        int f0 = first_node(g->order, x0[d]), f1 = first_node(g->order, x1[d]);
        m[d] = f0 < f1 ? f0 : f1;
        for (int a = 0; a < W; ++a) {
            double node = (double)(m[d] + a);
            S0[d][a] = orc_shape(g->order, x0[d] - node);
            DS[d][a] = orc_shape(g->order, x1[d] - node) - S0[d][a];
        }
    }
    /* W_d for each window node, then the running sum along axis d. */
    for (int d = 0; d < 3; ++d) {
        const int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
        const double coef = -qw * dl[d] / (dV * g->dt);
        for (int b = 0; b < W; ++b)
            for (int c = 0; c < W; ++c) {
                double acc = 0.0;
                for (int a = 0; a < W - 1; ++a) {
                    double wgt = DS[d][a] * (S0[e1][b] * S0[e2][c] + 0.5 * DS[e1][b] * S0[e2][c] +
                                             0.5 * S0[e1][b] * DS[e2][c] +
                                             (1.0 / 3.0) * DS[e1][b] * DS[e2][c]);
                    acc += wgt;
                    int64_t idx3[3];
                    idx3[d] = m[d] + a;
                    idx3[e1] = m[e1] + b;
                    idx3[e2] = m[e2] + c;
                    J[(int64_t)d * N + gidx(g, idx3[0], idx3[1], idx3[2])] += coef * acc;
                }
            }
    }
}

void orc_esirkepov(const orc_grid* g, int64_t n, const double* qw,
                   const double* x0, const double* y0, const double* z0,
                   const double* x1, const double* y1, const double* z1, double* J)
{
    for (int64_t p = 0; p < n; ++p) {
        double a[3] = {x0[p], y0[p], z0[p]}, b[3] = {x1[p], y1[p], z1[p]};
        esirkepov1(g, qw[p], a, b, J);
    }
}

/* Node charge density of n particles with the grid's shape (adds into rho). */
void orc_deposit_rho(const orc_grid* g, int64_t n, const double* qw,
                     const double* x, const double* y, const double* z, double* rho)
{
    const double dV = g->dx * g->dy * g->dz;
    for (int64_t p = 0; p < n; ++p) {
        int64_t bx = (int64_t)floor(x[p]), by = (int64_t)floor(y[p]), bz = (int64_t)floor(z[p]);
        for (int64_t k = bz - 2; k <= bz + 3; ++k) {
            double sz = orc_shape(g->order, z[p] - (double)k);
            if (sz == 0.0) continue;
            for (int64_t j = by - 2; j <= by + 3; ++j) {
                double sy = orc_shape(g->order, y[p] - (double)j);
                if (sy == 0.0) continue;
                for (int64_t i = bx - 2; i <= bx + 3; ++i) {
                    double sx = orc_shape(g->order, x[p] - (double)i);
                    if (sx == 0.0) continue;
                    rho[gidx(g, i, j, k)] += qw[p] * sx * sy * sz / dV;
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Yee updates.  B -= coef * curl E (forward differences of E);
 * E += coef * (curl B - J) (backward differences of B).  Periodic. */

void orc_update_b(const orc_grid* g, double coef, const double* E, double* B)
{
    const int64_t N = ncell(g);
    const double* Ex = E; const double* Ey = E + N; const double* Ez = E + 2 * N;
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                int64_t c = gidx(g, i, j, k);
                double cx = (Ez[gidx(g, i, j + 1, k)] - Ez[c]) / g->dy - (Ey[gidx(g, i, j, k + 1)] - Ey[c]) / g->dz;
                double cy = (Ex[gidx(g, i, j, k + 1)] - Ex[c]) / g->dz - (Ez[gidx(g, i + 1, j, k)] - Ez[c]) / g->dx;
                double cz = (Ey[gidx(g, i + 1, j, k)] - Ey[c]) / g->dx - (Ex[gidx(g, i, j + 1, k)] - Ex[c]) / g->dy;
                B[c] -= coef * cx;
                B[N + c] -= coef * cy;
                B[2 * N + c] -= coef * cz;
            }
}

void orc_update_e(const orc_grid* g, double coef, const double* B, const double* J, double* E)
{
    const int64_t N = ncell(g);
    const double* Bx = B; const double* By = B + N; const double* Bz = B + 2 * N;
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                int64_t c = gidx(g, i, j, k);
                double cx = (Bz[c] - Bz[gidx(g, i, j - 1, k)]) / g->dy - (By[c] - By[gidx(g, i, j, k - 1)]) / g->dz;
                double cy = (Bx[c] - Bx[gidx(g, i, j, k - 1)]) / g->dz - (Bz[c] - Bz[gidx(g, i - 1, j, k)]) / g->dx;
                double cz = (By[c] - By[gidx(g, i - 1, j, k)]) / g->dx - (Bx[c] - Bx[gidx(g, i, j - 1, k)]) / g->dy;
                E[c] += coef * (cx - (J ? J[c] : 0.0));
                E[N + c] += coef * (cy - (J ? J[N + c] : 0.0));
                E[2 * N + c] += coef * (cz - (J ? J[2 * N + c] : 0.0));
            }
}

/* Divergence of an E-located field at nodes (backward differences). */
void orc_div_nodes(const orc_grid* g, const double* F, double* out)
{
    const int64_t N = ncell(g);
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                int64_t c = gidx(g, i, j, k);
                out[c] = (F[c] - F[gidx(g, i - 1, j, k)]) / g->dx +
                         (F[N + c] - F[N + gidx(g, i, j - 1, k)]) / g->dy +
                         (F[2 * N + c] - F[2 * N + gidx(g, i, j, k - 1)]) / g->dz;
            }
}

/* Divergence of a B-located field at cell centres (forward differences). */
void orc_div_cells(const orc_grid* g, const double* F, double* out)
{
    const int64_t N = ncell(g);
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                int64_t c = gidx(g, i, j, k);
                out[c] = (F[gidx(g, i + 1, j, k)] - F[c]) / g->dx +
                         (F[N + gidx(g, i, j + 1, k)] - F[N + c]) / g->dy +
                         (F[2 * N + gidx(g, i, j, k + 1)] - F[2 * N + c]) / g->dz;
            }
}

/* ------------------------------------------------------------------------ */
/* Diagnostics. */

void orc_field_energy(const orc_grid* g, const double* E, const double* B, double out[2])
{
    const int64_t N3 = 3 * ncell(g);
    const double dV = g->dx * g->dy * g->dz;
    double we = 0.0, wb = 0.0;
    for (int64_t c = 0; c < N3; ++c) {
        we += E[c] * E[c];
        wb += B[c] * B[c];
    }
    out[0] = 0.5 * we * dV;
    out[1] = 0.5 * wb * dV;
}

double orc_kinetic(const orc_particles* s)
{
    double k = 0.0;
    for (int64_t p = 0; p < s->n; ++p) {
        double u2 = s->ux[p] * s->ux[p] + s->uy[p] * s->uy[p] + s->uz[p] * s->uz[p];
        double gm = sqrt(1.0 + u2);
        k += s->w[p] * s->m * (gm - 1.0);
    }
    return k;
}

static inline double charge_of(const orc_particles* s, int64_t p)
{
    return s->zstate ? s->q * (double)s->zstate[p] : s->q;
}

/* Node charge density of all species plus the neutralising background. */
void orc_rho(const orc_grid* g, int nsp, const orc_particles* sp, double* rho)
{
    const int64_t N = ncell(g);
    for (int64_t c = 0; c < N; ++c) rho[c] = g->rho_bg;
    for (int s = 0; s < nsp; ++s) {
        const orc_particles* S = &sp[s];
        double* qw = (double*)malloc(sizeof(double) * (S->n > 0 ? S->n : 1));
        for (int64_t p = 0; p < S->n; ++p) qw[p] = charge_of(S, p) * S->w[p];
        orc_deposit_rho(g, S->n, qw, S->x, S->y, S->z, rho);
        free(qw);
    }
}

/* ------------------------------------------------------------------------ */
/* One PIC cycle per step, in this order:
 *   gather(E^n, B^n + b0) -> Boris -> move -> zero J, Esirkepov J^{n+1/2}
 *   -> B half step -> E full step with -J -> B half step.
 * Immobile species are skipped.  Positions are wrapped into [0, n_d).
 * trace (optional) receives per step: W_E^n, W_B^n, K^{n-1/2}, K^{n+1/2}. */
/* Particle p of species S: gather, Boris, move, Esirkepov into J, wrap. */
static void push_one(const orc_grid* g, orc_particles* S, int64_t p, const double* E, const double* B, double* J)
{
    const double len[3] = {(double)g->nx, (double)g->ny, (double)g->nz};
    const double dl[3] = {g->dx, g->dy, g->dz};
    double Ep[3], Bp[3];
    orc_gather(g, E, B, 1, &S->x[p], &S->y[p], &S->z[p], Ep, Bp);
    double q = charge_of(S, p);
    double u[3] = {S->ux[p], S->uy[p], S->uz[p]};
    boris1(q / S->m, g->dt, Ep, Bp, u);
    S->ux[p] = u[0]; S->uy[p] = u[1]; S->uz[p] = u[2];
    double gm = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double x0[3] = {S->x[p], S->y[p], S->z[p]}, x1[3];
    for (int d = 0; d < 3; ++d) x1[d] = x0[d] + g->dt * u[d] / (gm * dl[d]);
    esirkepov1(g, q * S->w[p], x0, x1, J);
    for (int d = 0; d < 3; ++d) {
        double v = fmod(x1[d], len[d]);
        if (v < 0.0) v += len[d];
        if (v >= len[d]) v -= len[d];
        x1[d] = v;
    }
    S->x[p] = x1[0]; S->y[p] = x1[1]; S->z[p] = x1[2];
}

int orc_step(const orc_grid* g, int nsp, orc_particles* sp, double* E, double* B, double* J,
             int nsteps, double* trace)
{
    const int64_t N = ncell(g);
    for (int st = 0; st < nsteps; ++st) {
        if (trace) {
            double wf[2];
            orc_field_energy(g, E, B, wf);
            double km = 0.0;
            for (int s = 0; s < nsp; ++s) km += orc_kinetic(&sp[s]);
            trace[4 * st + 0] = wf[0];
            trace[4 * st + 1] = wf[1];
            trace[4 * st + 2] = km;
        }
        memset(J, 0, sizeof(double) * 3 * N);
        for (int s = 0; s < nsp; ++s) {
            orc_particles* S = &sp[s];
            if (!S->mobile) continue;
            for (int64_t p = 0; p < S->n; ++p) push_one(g, S, p, E, B, J);
        }
        orc_update_b(g, 0.5 * g->dt, E, B);
        orc_update_e(g, g->dt, B, J, E);
        orc_update_b(g, 0.5 * g->dt, E, B);
        if (trace) {
            double kp = 0.0;
            for (int s = 0; s < nsp; ++s) kp += orc_kinetic(&sp[s]);
            trace[4 * st + 3] = kp;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Initial particles of one species (see the header for the draw layout).
 *   id = (cell_linear * ppc + slot) + id_offset, cell_linear = i + nx(j + ny k)
 *   position: cell corner + three Philox uniforms (purpose 0); a species
 *     placed "coincident" with another takes that species' draw for the same
 *     cell and slot, so the two start at identical positions;
 *   momentum: drift + u_th * N(0,1) per component from two Box-Muller pairs
 *     (purpose 1).  layout 0 uniform drift, 1 shear layer (+drift for
 *     j in [ny/4, 3ny/4), -drift elsewhere), 2 interpenetrating beams
 *     (+drift for even slots, -drift for odd slots).
 * drift_u is the drift momentum u_d = gamma*beta (already converted). */
typedef struct {
    int32_t index;     /* species index in the Philox counter */
    int32_t ppc;
    int64_t id_offset;
    double u_th;
    double drift_u[3];
    int32_t layout;
    int32_t pos_index; /* species index whose position draws are used */
    int32_t pos_ppc;
    int64_t pos_id_offset;
    double w;
} orc_init_spec;

void orc_init_species(const orc_grid* g, uint64_t seed, const orc_init_spec* sp,
                      double* x, double* y, double* z, double* ux, double* uy, double* uz,
                      double* w, int64_t* id)
{
    const double two_pi = 6.283185307179586476925286766559;
    int64_t p = 0;
    for (int64_t k = 0; k < g->nz; ++k)
        for (int64_t j = 0; j < g->ny; ++j)
            for (int64_t i = 0; i < g->nx; ++i) {
                int64_t cell = i + (int64_t)g->nx * (j + (int64_t)g->ny * k);
                for (int64_t s = 0; s < sp->ppc; ++s, ++p) {
                    int64_t myid = cell * sp->ppc + s + sp->id_offset;
                    int64_t pid = cell * sp->pos_ppc + s + sp->pos_id_offset;
                    double a[4], b[4];
                    draw4(seed, (uint64_t)pid, (uint64_t)sp->pos_index, 0, 0, a);
                    draw4(seed, (uint64_t)myid, (uint64_t)sp->index, 1, 0, b);
                    x[p] = (double)i + a[0];
                    y[p] = (double)j + a[1];
                    z[p] = (double)k + a[2];
                    double r0 = sqrt(-2.0 * log(b[0])), r1 = sqrt(-2.0 * log(b[2]));
                    double n0 = r0 * cos(two_pi * b[1]);
                    double n1 = r0 * sin(two_pi * b[1]);
                    double n2 = r1 * cos(two_pi * b[3]);
                    double sign = 1.0;
                    if (sp->layout == 1) sign = (4 * j >= g->ny && 4 * j < 3 * (int64_t)g->ny) ? 1.0 : -1.0;
                    if (sp->layout == 2) sign = (s % 2 == 0) ? 1.0 : -1.0;
                    ux[p] = sign * sp->drift_u[0] + sp->u_th * n0;
                    uy[p] = sign * sp->drift_u[1] + sp->u_th * n1;
                    uz[p] = sign * sp->drift_u[2] + sp->u_th * n2;
                    w[p] = sp->w;
                    id[p] = myid;
                }
            }
}

/* ------------------------------------------------------------------------ */
/* The cycle of orc_step (no trace) with each species' particle loop split
 * over nthreads threads (contiguous ranges), each depositing into a private
 * current array; the private arrays are added into J in thread order after
 * the loop.  For timing the CPU on all host cores only; orc_step is the
 * reference.  Returns the number of threads that ran, or -1 if the private
 * arrays cannot be allocated. */
int orc_step_threads(const orc_grid* g, int nsp, orc_particles* sp, double* E, double* B, double* J,
                     int nsteps, int nthreads)
{
    const int64_t N3 = 3 * ncell(g);
    if (nthreads < 1) nthreads = 1;
#ifndef _OPENMP
    nthreads = 1;
#endif
    double* priv = (double*)malloc(sizeof(double) * (size_t)N3 * (size_t)nthreads);
    if (!priv) return -1;
    int used = 1;
    for (int st = 0; st < nsteps; ++st) {
        memset(priv, 0, sizeof(double) * (size_t)N3 * (size_t)nthreads);
        for (int s = 0; s < nsp; ++s) {
            orc_particles* S = &sp[s];
            if (!S->mobile) continue;
#ifdef _OPENMP
#pragma omp parallel num_threads(nthreads)
#endif
            {
                int t = 0, nt = 1;
#ifdef _OPENMP
                t = omp_get_thread_num();
                nt = omp_get_num_threads();
#endif
                if (t == 0) used = nt;
                const int64_t lo = S->n * t / nt, hi = S->n * (t + 1) / nt;
                for (int64_t p = lo; p < hi; ++p) push_one(g, S, p, E, B, priv + (size_t)t * N3);
            }
        }
        memset(J, 0, sizeof(double) * N3);
        for (int t = 0; t < used; ++t)
            for (int64_t i = 0; i < N3; ++i) J[i] += priv[(size_t)t * N3 + i];
        orc_update_b(g, 0.5 * g->dt, E, B);
        orc_update_e(g, g->dt, B, J, E);
        orc_update_b(g, 0.5 * g->dt, E, B);
    }
    free(priv);
    return used;
}
