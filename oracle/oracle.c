/*
 * FP64 CPU oracle of the electromagnetic particle-in-cell (PIC) time step.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this library.  It shares no code, header, table
 * or helper with the HIP library; the two are separate implementations of the
 * same discrete scheme.
 *
 * Source: "Porting WarpX to GPU-accelerated platforms" (arXiv 2101.12149).
 * The paper names the methods but prints no equation of the scheme:
 *   - Sec. 1: the EM-PIC method for relativistic charged particles;
 *   - Sec. 2.4 (SyncNodal item): Yee discretisation, B on cell faces,
 *     E and J on cell edges;
 *   - Sec. 4.1.1: standard Yee FDTD solver, Esirkepov current deposition,
 *     third-order shape functions;
 *   - Sec. 4.2: energy-conserving field gathering;
 *   - Sec. 3.1: the gather is fused with the push, no stored per-particle
 *     fields.
 * Every formula below is written from those method names and textbook
 * mathematics (Yee 1966; Esirkepov 2001; Boris 1970).  It is deliberately
 * plain: shapes are evaluated from the B-spline's definition as a function
 * of distance, sums run over fixed generous node windows, positions are an
 * integer cell plus an FP64 offset (so the oracle's own rounding does not
 * grow with the box size), and nothing is tiled, sorted or fused.
 *
 * Conventions (all arrays x fastest, index i + n0*(j + n1*k), periodic):
 *   E_x(i+1/2,j,k)  E_y(i,j+1/2,k)  E_z(i,j,k+1/2)      J like E
 *   B_x(i,j+1/2,k+1/2)  B_y(i+1/2,j,k+1/2)  B_z(i+1/2,j+1/2,k)
 *   particle position in cell units: xi_d = cell_d + off_d, off in [0,1)
 *   u = gamma*v, gamma = sqrt(1+|u|^2/c^2)
 * State at step n is (x^n, u^{n-1/2}, E^n, B^n); J holds the last current.
 *
 * Parity-pinned functions: every exported function is pinned by the CPU
 * tests (closed forms, invariants, brute force, dot-product transposes,
 * central finite differences of the adjoint).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t n[3];
    double d[3];
    double dt, c, eps0;
    int32_t order;
    int32_t pusher; /* 0: Boris, 1: Vay */
    int32_t solver; /* 0: Yee, 1: Cole-Karkkainen-Cowan */
    const double *gather_filter; /* NULL, or double[6][4]: z taps per component */
} or_grid;

typedef struct {
    int64_t n;
    int32_t *cell[3];
    double *off[3];
    double *u[3];
    const double *w; /* NULL -> every particle has weight w0 */
    double w0, q, m;
} or_species;

typedef struct {
    double *E[3], *B[3], *J[3];
} or_fields;

typedef struct {
    int32_t k_plane; /* < 0: no source */
    const double *amp; /* n0*n1 map, x fastest */
    const double *g;   /* g[step] */
    int64_t n_g;
} or_source;

typedef struct {
    double *lx[3], *lu[3], *lE[3], *lB[3];
} or_adjoint;

/* Threads the oracle's parallel loops use. */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the thread count of later parallel loops (n >= 1).  Only the order in
   which the per-thread current buffers are summed depends on it. */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* indexing                                                            */

static inline int64_t wrapi(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

static inline int64_t idx3(const or_grid *g, int64_t i, int64_t j, int64_t k)
{
    return wrapi(i, g->n[0]) + (int64_t)g->n[0] * (wrapi(j, g->n[1]) + (int64_t)g->n[1] * wrapi(k, g->n[2]));
}

static inline double weight_of(const or_species *s, int64_t p)
{
    return s->w ? s->w[p] : s->w0;
}

/* Staggering (in cells) of each component, Sec. 2.4 (Yee: E, J on edges,
 * B on faces). */
static const double STAG_E[3][3] = {{0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 0.5}};
static const double STAG_B[3][3] = {{0, 0.5, 0.5}, {0.5, 0, 0.5}, {0.5, 0.5, 0}};

/* ------------------------------------------------------------------ */
/* Shape functions: centred cardinal B-splines (Sec. 4.1.1 "third order
 * shape functions"; order 1 is the cloud-in-cell hat).                */

double or_shape(int order, double r)
{
    double a = fabs(r);
    if (order == 1)
        return a < 1.0 ? 1.0 - a : 0.0;
    if (order == 3) {
        if (a < 1.0)
            return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
        if (a < 2.0) {
            double t = 2.0 - a;
            return t * t * t / 6.0;
        }
        return 0.0;
    }
    return NAN;
}

/* d S(r) / d r */
double or_dshape(int order, double r)
{
    double a = fabs(r);
    double sg = r > 0 ? 1.0 : (r < 0 ? -1.0 : 0.0);
    if (order == 1)
        return a < 1.0 ? -sg : 0.0;
    if (order == 3) {
        if (a < 1.0)
            return -2.0 * r + 1.5 * r * a;
        if (a < 2.0) {
            double t = 2.0 - a;
            return -sg * 0.5 * t * t;
        }
        return 0.0;
    }
    return NAN;
}

/* ------------------------------------------------------------------ */
/* Field gather (Sec. 4.2, energy-conserving variant: every component is
 * interpolated from its own staggered location with the same order in
 * all three directions).  Nodes -2..3 around the particle's cell cover
 * the support of order <= 3.                                          */

#define GW0 (-2)
#define GW1 3

static double gather_one(const or_grid *g, const double *F, const double st[3], const int32_t cell[3],
                         const double off[3], double grad[3])
{
    double wx[GW1 - GW0 + 1][2], wy[GW1 - GW0 + 1][2], wz[GW1 - GW0 + 1][2];
    for (int a = GW0; a <= GW1; ++a) {
        wx[a - GW0][0] = or_shape(g->order, off[0] - a - st[0]);
        wx[a - GW0][1] = or_dshape(g->order, off[0] - a - st[0]);
        wy[a - GW0][0] = or_shape(g->order, off[1] - a - st[1]);
        wy[a - GW0][1] = or_dshape(g->order, off[1] - a - st[1]);
        wz[a - GW0][0] = or_shape(g->order, off[2] - a - st[2]);
        wz[a - GW0][1] = or_dshape(g->order, off[2] - a - st[2]);
    }
    double v = 0, gx = 0, gy = 0, gz = 0;
    for (int c = GW0; c <= GW1; ++c)
        for (int b = GW0; b <= GW1; ++b)
            for (int a = GW0; a <= GW1; ++a) {
                double f = F[idx3(g, (int64_t)cell[0] + a, (int64_t)cell[1] + b, (int64_t)cell[2] + c)];
                const double *X = wx[a - GW0], *Y = wy[b - GW0], *Z = wz[c - GW0];
                v += X[0] * Y[0] * Z[0] * f;
                gx += X[1] * Y[0] * Z[0] * f;
                gy += X[0] * Y[1] * Z[0] * f;
                gz += X[0] * Y[0] * Z[1] * f;
            }
    if (grad) {
        grad[0] = gx;
        grad[1] = gy;
        grad[2] = gz;
    }
    return v;
}

static void particle_pos(const or_species *s, int64_t p, int32_t cell[3], double off[3])
{
    for (int d = 0; d < 3; ++d) {
        cell[d] = s->cell[d][p];
        off[d] = s->off[d][p];
    }
}

/* Digital filter of the fields before the gather (the paper applies the
 * Godfrey filter there, Sec. 4.2, against the numerical Cherenkov
 * instability): a symmetric stencil along z per component m (E_x..E_z,
 * B_x..B_z),
 *   F~(i,j,k) = w[m][0] F(i,j,k) + sum_{s=1..3} w[m][s] (F(i,j,k+s) + F(i,j,k-s)),
 * periodic.  It is its own transpose.  The taps are the caller's.        */
static void filter_z(const or_grid *g, const double w[4], const double *F, double *out)
{
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                double v = w[0] * F[idx3(g, i, j, k)];
                for (int sft = 1; sft <= 3; ++sft)
                    v += w[sft] * (F[idx3(g, i, j, k + sft)] + F[idx3(g, i, j, k - sft)]);
                out[idx3(g, i, j, k)] = v;
            }
}

/* The six field components the gather reads: the fields themselves, or
 * filtered copies in buf (freed by the caller) when the grid has a filter. */
static double *gather_fields(const or_grid *g, const or_fields *f, const double *F[6])
{
    for (int m = 0; m < 3; ++m) {
        F[m] = f->E[m];
        F[3 + m] = f->B[m];
    }
    if (!g->gather_filter)
        return NULL;
    int64_t nc = (int64_t)g->n[0] * g->n[1] * g->n[2];
    double *buf = (double *)malloc(sizeof(double) * 6 * (size_t)nc);
    for (int m = 0; m < 6; ++m) {
        filter_z(g, g->gather_filter + 4 * m, F[m], buf + m * nc);
        F[m] = buf + m * nc;
    }
    return buf;
}

void or_gather(const or_grid *g, const or_species *s, const or_fields *f, double *Ep[3], double *Bp[3])
{
    const double *F[6];
    double *fbuf = gather_fields(g, f, F);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < s->n; ++p) {
        int32_t cell[3];
        double off[3];
        particle_pos(s, p, cell, off);
        for (int m = 0; m < 3; ++m) {
            Ep[m][p] = gather_one(g, F[m], STAG_E[m], cell, off, NULL);
            Bp[m][p] = gather_one(g, F[3 + m], STAG_B[m], cell, off, NULL);
        }
    }
    free(fbuf);
}

/* ------------------------------------------------------------------ */
/* Relativistic Boris rotation (Boris 1970): half electric kick, magnetic
 * rotation through the tangent-half-angle vector t and s = 2t/(1+t^2),
 * second half kick.  h = q dt / (2 m).                                  */

typedef struct {
    double a[3], gbar, t[3], s[3], up[3], tt;
} boris_tape;

static void cross(const double a[3], const double b[3], double r[3])
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

static void boris(double h, double c, const double u0[3], const double E[3], const double B[3], double u1[3],
                  boris_tape *tp)
{
    boris_tape T;
    for (int d = 0; d < 3; ++d)
        T.a[d] = u0[d] + h * E[d];
    T.gbar = sqrt(1.0 + (T.a[0] * T.a[0] + T.a[1] * T.a[1] + T.a[2] * T.a[2]) / (c * c));
    for (int d = 0; d < 3; ++d)
        T.t[d] = h * B[d] / T.gbar;
    T.tt = T.t[0] * T.t[0] + T.t[1] * T.t[1] + T.t[2] * T.t[2];
    for (int d = 0; d < 3; ++d)
        T.s[d] = 2.0 * T.t[d] / (1.0 + T.tt);
    double axt[3];
    cross(T.a, T.t, axt);
    for (int d = 0; d < 3; ++d)
        T.up[d] = T.a[d] + axt[d];
    double upxs[3];
    cross(T.up, T.s, upxs);
    for (int d = 0; d < 3; ++d)
        u1[d] = T.a[d] + upxs[d] + h * E[d];
    if (tp)
        *tp = T;
}

static double gamma_of(const double u[3], double c)
{
    return sqrt(1.0 + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / (c * c));
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Vay's relativistic push (J.-L. Vay, Phys. Plasmas 15, 056701, 2008), the
 * pusher the paper runs for relativistic beams (Sec. 4.2).  The magnetic
 * force takes the mean of the old and the new velocity,
 *     u1 - u0 = 2h E + h (u0/gamma0 + u1/gamma1) x B,      h = q dt / (2 m),
 * which is implicit in u1.  Collecting the known terms in
 *     w = u0 + 2h E + h (u0/gamma0) x B
 * and writing tau = h B, t = tau / gamma1, it reads u1 - u1 x t = w, a
 * linear system once gamma1 is known, solved by
 *     u1 = (w + (w.t) t + w x t) / (1 + |t|^2).
 * Its norm, |u1|^2 = (gamma1^2 |w|^2 + (w.tau)^2) / (gamma1^2 + |tau|^2),
 * inserted in gamma1^2 = 1 + |u1|^2/c^2 gives a quadratic in G = gamma1^2,
 *     G^2 - sigma G - X = 0,  sigma = 1 + |w|^2/c^2 - |tau|^2,
 *                              X = |tau|^2 + (w.tau)^2/c^2,
 * of which the positive root is the physical one (taken in the form that
 * does not cancel when sigma < 0).                                       */
static double vay_gamma2(double sigma, double X, double *D)
{
    *D = sqrt(sigma * sigma + 4.0 * X);
    return sigma >= 0.0 ? 0.5 * (sigma + *D) : 2.0 * X / (*D - sigma);
}

static void vay(double h, double c, const double u0[3], const double E[3], const double B[3], double u1[3])
{
    double c2 = c * c, g0 = gamma_of(u0, c);
    double v0[3], v0xB[3], w[3], tau[3];
    for (int d = 0; d < 3; ++d)
        v0[d] = u0[d] / g0;
    cross(v0, B, v0xB);
    for (int d = 0; d < 3; ++d) {
        w[d] = u0[d] + 2.0 * h * E[d] + h * v0xB[d];
        tau[d] = h * B[d];
    }
    double tau2 = dot3(tau, tau), wt = dot3(w, tau);
    double D, G = vay_gamma2(1.0 + dot3(w, w) / c2 - tau2, tau2 + wt * wt / c2, &D);
    double g1 = sqrt(G);
    double t[3], wxt[3];
    for (int d = 0; d < 3; ++d)
        t[d] = tau[d] / g1;
    cross(w, t, wxt);
    double a = dot3(w, t), den = 1.0 + dot3(t, t);
    for (int d = 0; d < 3; ++d)
        u1[d] = (w[d] + a * t[d] + wxt[d]) / den;
}

/* Transpose of vay(): given ub = dL/du1, return dL/du0, dL/dE, dL/dB.  The
 * forward quantities are evaluated again and the chain rule is applied to
 * them in reverse order; the root G(sigma, X) has dG/dsigma = G/D and
 * dG/dX = 1/D with D = sqrt(sigma^2 + 4 X). */
static void vay_adjoint(double h, double c, const double u0[3], const double E[3], const double B[3],
                        const double ub[3], double u0b[3], double Eb[3], double Bb[3])
{
    double c2 = c * c, g0 = gamma_of(u0, c);
    double v0[3], v0xB[3], w[3], tau[3];
    for (int d = 0; d < 3; ++d)
        v0[d] = u0[d] / g0;
    cross(v0, B, v0xB);
    for (int d = 0; d < 3; ++d) {
        w[d] = u0[d] + 2.0 * h * E[d] + h * v0xB[d];
        tau[d] = h * B[d];
    }
    double tau2 = dot3(tau, tau), wt = dot3(w, tau);
    double sigma = 1.0 + dot3(w, w) / c2 - tau2;
    double D, G = vay_gamma2(sigma, tau2 + wt * wt / c2, &D);
    double g1 = sqrt(G);
    double t[3], wxt[3], q[3];
    for (int d = 0; d < 3; ++d)
        t[d] = tau[d] / g1;
    cross(w, t, wxt);
    double a = dot3(w, t), den = 1.0 + dot3(t, t), s = 1.0 / den;
    for (int d = 0; d < 3; ++d)
        q[d] = w[d] + a * t[d] + wxt[d];
    /* u1 = s q */
    double sb = dot3(ub, q), qb[3];
    for (int d = 0; d < 3; ++d)
        qb[d] = s * ub[d];
    /* q = w + a t + w x t */
    double wb[3], tb[3], tmp[3];
    cross(t, qb, tmp); /* d((w x t).qb)/dw = t x qb */
    for (int d = 0; d < 3; ++d)
        wb[d] = qb[d] + tmp[d];
    double ab = dot3(qb, t);
    cross(qb, w, tmp); /* d((w x t).qb)/dt = qb x w */
    for (int d = 0; d < 3; ++d)
        tb[d] = a * qb[d] + tmp[d];
    /* a = w.t */
    for (int d = 0; d < 3; ++d) {
        wb[d] += ab * t[d];
        tb[d] += ab * w[d];
    }
    /* s = 1 / (1 + |t|^2) */
    for (int d = 0; d < 3; ++d)
        tb[d] += -2.0 * s * s * sb * t[d];
    /* t = tau / g1 */
    double taub[3], g1b = 0.0;
    for (int d = 0; d < 3; ++d) {
        taub[d] = tb[d] / g1;
        g1b -= tb[d] * tau[d] / (g1 * g1);
    }
    /* g1 = sqrt(G), G = G(sigma, X) */
    double Gb = g1b / (2.0 * g1);
    double sigb = Gb * G / D, Xb = Gb / D;
    /* X = |tau|^2 + (w.tau)^2 / c^2 */
    double wtb = 2.0 * Xb * wt / c2;
    for (int d = 0; d < 3; ++d)
        taub[d] += 2.0 * Xb * tau[d];
    /* sigma = 1 + |w|^2 / c^2 - |tau|^2 */
    for (int d = 0; d < 3; ++d) {
        wb[d] += 2.0 * sigb * w[d] / c2;
        taub[d] -= 2.0 * sigb * tau[d];
    }
    /* w.tau */
    for (int d = 0; d < 3; ++d) {
        wb[d] += wtb * tau[d];
        taub[d] += wtb * w[d];
    }
    /* tau = h B;  w = u0 + 2h E + h v0 x B */
    double v0b[3], wxv[3];
    cross(B, wb, v0b); /* d((v0 x B).wb)/dv0 = B x wb */
    cross(wb, v0, wxv); /* d((v0 x B).wb)/dB = wb x v0 */
    for (int d = 0; d < 3; ++d) {
        Bb[d] = h * taub[d] + h * wxv[d];
        Eb[d] = 2.0 * h * wb[d];
        u0b[d] = wb[d];
        v0b[d] *= h;
    }
    /* v0 = u0 / g0,  g0 = sqrt(1 + |u0|^2 / c^2) */
    double g0b = -dot3(v0b, v0) / g0;
    for (int d = 0; d < 3; ++d)
        u0b[d] += v0b[d] / g0 + g0b * v0[d] / c2;
    (void)E;
}

/* The momentum update the grid selects. */
static void push_momentum(const or_grid *g, double h, const double u0[3], const double E[3], const double B[3],
                          double u1[3])
{
    if (g->pusher == 1)
        vay(h, g->c, u0, E, B, u1);
    else
        boris(h, g->c, u0, E, B, u1, NULL);
}

/* Displacement of one step in cell units: dt u / (gamma dx_d). */
static void displacement(const or_grid *g, const double u[3], double disp[3])
{
    double gm = gamma_of(u, g->c);
    for (int d = 0; d < 3; ++d)
        disp[d] = g->dt * u[d] / (gm * g->d[d]);
}

/* Move one coordinate by disp cells and wrap periodically; if rounding
 * leaves the offset at exactly 1, it belongs to the next cell. */
static void move_coord(int32_t *cell, double *off, double disp, int32_t n)
{
    double xi = *off + disp;
    double k = floor(xi);
    double f = xi - k;
    int64_t c = (int64_t)*cell + (int64_t)k;
    if (f >= 1.0) {
        f -= 1.0;
        c += 1;
    }
    *cell = (int32_t)wrapi(c, n);
    *off = f;
}

/* Momentum update (Boris or Vay) followed by the position update. */
void or_push(const or_grid *g, or_species *s, double *const Ep[3], double *const Bp[3])
{
    double h = s->q * g->dt / (2.0 * s->m);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < s->n; ++p) {
        double u0[3], E[3], B[3], u1[3], disp[3];
        for (int d = 0; d < 3; ++d) {
            u0[d] = s->u[d][p];
            E[d] = Ep[d][p];
            B[d] = Bp[d][p];
        }
        push_momentum(g, h, u0, E, B, u1);
        displacement(g, u1, disp);
        for (int d = 0; d < 3; ++d) {
            s->u[d][p] = u1[d];
            move_coord(&s->cell[d][p], &s->off[d][p], disp[d], g->n[d]);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Esirkepov charge-conserving deposition (Esirkepov 2001; Sec. 3.4.1 and
 * 4.1.1).  With S0, S1 the 1D shapes at the old and new position and
 * DS = S1 - S0,
 *   W_x(i,j,k) = DS_x(i) [ (S0y S0z + S1y S1z)/3 + (S1y S0z + S0y S1z)/6 ]
 * (and cyclically), and J_x(i+1/2,j,k) is the running sum along x of
 * -(q w / (dt dy dz)) W_x, starting from zero below the stencil.  Nodes
 * -2..3 around the old cell cover both supports for |disp| < 1 cell.
 * J_x at the top node of the window is the full sum of W_x, which is zero
 * because the shapes sum to one, so it is not stored.                    */

#define DW0 (-2)
#define DW1 3
#define DWN (DW1 - DW0 + 1)

typedef struct {
    double S0[3][DWN], S1[3][DWN], D0[3][DWN], D1[3][DWN];
} esk_shapes;

static void esk_fill(const or_grid *g, const double off0[3], const double disp[3], esk_shapes *E)
{
    for (int d = 0; d < 3; ++d)
        for (int a = DW0; a <= DW1; ++a) {
            double r0 = off0[d] - a, r1 = off0[d] + disp[d] - a;
            E->S0[d][a - DW0] = or_shape(g->order, r0);
            E->S1[d][a - DW0] = or_shape(g->order, r1);
            E->D0[d][a - DW0] = or_dshape(g->order, r0);
            E->D1[d][a - DW0] = or_dshape(g->order, r1);
        }
}

/* W for component m at window node (a,b,c) in the (m, m+1, m+2) frame. */
static double esk_w(const esk_shapes *E, int m, int a, int b, int c)
{
    int p = (m + 1) % 3, q = (m + 2) % 3;
    double ds = E->S1[m][a] - E->S0[m][a];
    return ds * ((E->S0[p][b] * E->S0[q][c] + E->S1[p][b] * E->S1[q][c]) / 3.0 +
                 (E->S1[p][b] * E->S0[q][c] + E->S0[p][b] * E->S1[q][c]) / 6.0);
}

/* global index of window node (a along m, b along m+1, c along m+2) */
static int64_t esk_index(const or_grid *g, const int32_t cell[3], int m, int a, int b, int c)
{
    int64_t v[3];
    v[m] = (int64_t)cell[m] + a + DW0;
    v[(m + 1) % 3] = (int64_t)cell[(m + 1) % 3] + b + DW0;
    v[(m + 2) % 3] = (int64_t)cell[(m + 2) % 3] + c + DW0;
    return idx3(g, v[0], v[1], v[2]);
}

static double esk_coef(const or_grid *g, int m, double qw)
{
    return -qw / (g->dt * g->d[(m + 1) % 3] * g->d[(m + 2) % 3]);
}

static void deposit_one(const or_grid *g, const int32_t cell[3], const double off0[3], const double disp[3],
                        double qw, double *J[3])
{
    esk_shapes E;
    esk_fill(g, off0, disp, &E);
    for (int m = 0; m < 3; ++m) {
        double K = esk_coef(g, m, qw);
        for (int c = 0; c < DWN; ++c)
            for (int b = 0; b < DWN; ++b) {
                double run = 0.0;
                for (int a = 0; a < DWN - 1; ++a) {
                    run += esk_w(&E, m, a, b, c);
                    J[m][esk_index(g, cell, m, a, b, c)] += K * run;
                }
            }
    }
}

/* Minimal-image displacement (cells) between two periodic positions. */
static double periodic_disp(int32_t c0, double f0, int32_t c1, double f1, int32_t n)
{
    double d = (double)(c1 - c0) + (f1 - f0);
    if (d >= 0.5 * n)
        d -= n;
    if (d < -0.5 * n)
        d += n;
    return d;
}

/* Deposit particles with private per-thread current buffers that are summed
 * afterwards: the "data duplication" scheme of Sec. 3.4.1 for CPU threads. */
static void deposit_all(const or_grid *g, const or_species *s, const double *const disp[3], double *J[3])
{
    int64_t nc = (int64_t)g->n[0] * g->n[1] * g->n[2];
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double *priv = (double *)calloc((size_t)nt * 3 * (size_t)nc, sizeof(double));
#pragma omp parallel num_threads(nt)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        double *Jt[3] = {priv + ((size_t)t * 3 + 0) * nc, priv + ((size_t)t * 3 + 1) * nc,
                         priv + ((size_t)t * 3 + 2) * nc};
#pragma omp for schedule(static)
        for (int64_t p = 0; p < s->n; ++p) {
            int32_t cell[3];
            double off[3], dp[3];
            particle_pos(s, p, cell, off);
            for (int d = 0; d < 3; ++d)
                dp[d] = disp[d][p];
            deposit_one(g, cell, off, dp, s->q * weight_of(s, p), Jt);
        }
    }
    for (int t = 0; t < nt; ++t)
        for (int m = 0; m < 3; ++m) {
            const double *src = priv + ((size_t)t * 3 + m) * nc;
            for (int64_t i = 0; i < nc; ++i)
                J[m][i] += src[i];
        }
    free(priv);
}

/* J += current of particles moving from `before` to `after`. */
void or_deposit(const or_grid *g, const or_species *before, const or_species *after, or_fields *f)
{
    int64_t n = before->n;
    double *disp[3];
    for (int d = 0; d < 3; ++d)
        disp[d] = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t p = 0; p < n; ++p)
        for (int d = 0; d < 3; ++d)
            disp[d][p] = periodic_disp(before->cell[d][p], before->off[d][p], after->cell[d][p],
                                       after->off[d][p], g->n[d]);
    deposit_all(g, before, (const double *const *)disp, f->J);
    for (int d = 0; d < 3; ++d)
        free(disp[d]);
}

/* Nodal charge density rho(i,j,k) = sum_p q w S S S / dV (diagnostic). */
void or_rho(const or_grid *g, const or_species *s, double *rho)
{
    double dV = g->d[0] * g->d[1] * g->d[2];
    for (int64_t p = 0; p < s->n; ++p) {
        int32_t cell[3];
        double off[3];
        particle_pos(s, p, cell, off);
        double qw = s->q * weight_of(s, p) / dV;
        for (int c = GW0; c <= GW1; ++c)
            for (int b = GW0; b <= GW1; ++b)
                for (int a = GW0; a <= GW1; ++a) {
                    double S = or_shape(g->order, off[0] - a) * or_shape(g->order, off[1] - b) *
                               or_shape(g->order, off[2] - c);
                    rho[idx3(g, (int64_t)cell[0] + a, (int64_t)cell[1] + b, (int64_t)cell[2] + c)] += qw * S;
                }
    }
}

/* ------------------------------------------------------------------ */
/* Yee FDTD (Sec. 2.4 and 4.1.1).  Forward differences take edge fields to
 * faces, backward differences take face fields to edges:
 *   curlE_x = D+y Ez - D+z Ey  (on faces)
 *   curlB_x = D-y Bz - D-z By  (on edges), cyclically.
 * One step: B -= dt/2 curlE; E += dt (c^2 curlB - J/eps0); source;
 *           B -= dt/2 curlE.                                           */

/* Cole-Karkkainen-Cowan field solver (the paper's solver for the
 * accelerator stage, Sec. 4.2; Cole 1997/2002, Karkkainen et al. 2006): the
 * E update keeps Yee's differences, and in the B update every difference
 * along axis a is averaged over its transverse neighbours p, q:
 *   D_a -> alpha_a D_a + beta_ap (D_a[p+1] + D_a[p-1]) + beta_aq (D_a[q+1] + D_a[q-1])
 *          + gamma_a (D_a[p+1,q+1] + D_a[p+1,q-1] + D_a[p-1,q+1] + D_a[p-1,q-1]).
 * With delta = min cell size, r_a = (delta/d_a)^2, S = r_x r_y + r_y r_z + r_z r_x:
 *   beta = (1 - r_x r_y r_z / S) / 8,  beta_ap = r_p beta,  beta_aq = r_q beta,
 *   gamma_a = r_p r_q (1/16 - r_p r_q / (8 S)),
 *   alpha_a = 1 - 2 beta_ap - 2 beta_aq - 4 gamma_a,
 * for cubic cells 7/12, 1/12, 1/48; the step is stable up to c dt = delta
 * and has no dispersion along an axis with d_a = delta at that step.      */
static void ckc_coeffs(const or_grid *g, double co[3][4])
{
    double dl = g->d[0];
    for (int a = 1; a < 3; ++a)
        if (g->d[a] < dl)
            dl = g->d[a];
    double r[3];
    for (int a = 0; a < 3; ++a)
        r[a] = (dl / g->d[a]) * (dl / g->d[a]);
    double S = r[0] * r[1] + r[1] * r[2] + r[2] * r[0];
    double beta = (1.0 - r[0] * r[1] * r[2] / S) / 8.0;
    for (int a = 0; a < 3; ++a) {
        int p = (a + 1) % 3, q = (a + 2) % 3;
        double bp = r[p] * beta, bq = r[q] * beta;
        double gm = r[p] * r[q] * (1.0 / 16.0 - r[p] * r[q] / (8.0 * S));
        co[a][0] = 1.0 - 2.0 * bp - 2.0 * bq - 4.0 * gm;
        co[a][1] = bp;
        co[a][2] = bq;
        co[a][3] = gm;
    }
}

/* The coefficients above, co[a][0..3] = (alpha_a, beta_ap, beta_aq,
 * gamma_a) for a = x, y, z (exported so that the tests can check them). */
void or_ckc_coeffs(const or_grid *g, double co[12])
{
    double c3[3][4];
    ckc_coeffs(g, c3);
    for (int a = 0; a < 3; ++a)
        for (int s = 0; s < 4; ++s)
            co[4 * a + s] = c3[a][s];
}

/* Difference of component F along axis a at cell (i,j,k): forward
 * (F[+a] - F) or backward (F - F[-a]), divided by d_a; with co != NULL
 * averaged over the transverse neighbours as above. */
static double diff_axis(const or_grid *g, const double *F, int a, int fwd, int64_t i, int64_t j, int64_t k,
                        const double co[3][4])
{
    int64_t c0[3] = {i, j, k};
    int p = (a + 1) % 3, q = (a + 2) % 3;
    double sum = 0.0;
    for (int sp = -1; sp <= 1; ++sp)
        for (int sq = -1; sq <= 1; ++sq) {
            double w;
            if (!co)
                w = (sp == 0 && sq == 0) ? 1.0 : 0.0;
            else if (sp == 0 && sq == 0)
                w = co[a][0];
            else if (sq == 0)
                w = co[a][1];
            else if (sp == 0)
                w = co[a][2];
            else
                w = co[a][3];
            if (w == 0.0)
                continue;
            int64_t c[3] = {c0[0], c0[1], c0[2]};
            c[p] += sp;
            c[q] += sq;
            int64_t o = idx3(g, c[0], c[1], c[2]);
            int64_t cn[3] = {c[0], c[1], c[2]};
            cn[a] += fwd ? 1 : -1;
            int64_t on = idx3(g, cn[0], cn[1], cn[2]);
            sum += w * (fwd ? F[on] - F[o] : F[o] - F[on]);
        }
    return sum / g->d[a];
}

/* out = curl F with forward differences (edges -> faces) or backward
 * differences (faces -> edges), Yee's or the CKC-averaged ones. */
static void curl_any(const or_grid *g, double *const F[3], double *out[3], int fwd, int ckc)
{
    double co[3][4];
    ckc_coeffs(g, co);
    const double(*cp)[4] = ckc ? (const double(*)[4])co : NULL;
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t o = idx3(g, i, j, k);
                out[0][o] = diff_axis(g, F[2], 1, fwd, i, j, k, cp) - diff_axis(g, F[1], 2, fwd, i, j, k, cp);
                out[1][o] = diff_axis(g, F[0], 2, fwd, i, j, k, cp) - diff_axis(g, F[2], 0, fwd, i, j, k, cp);
                out[2][o] = diff_axis(g, F[1], 0, fwd, i, j, k, cp) - diff_axis(g, F[0], 1, fwd, i, j, k, cp);
            }
}

/* The curl of E in the B update (the solver's) and of B in the E update. */
static void curl_fwd(const or_grid *g, double *const F[3], double *out[3])
{
    curl_any(g, F, out, 1, g->solver == 1);
}

static void curl_bwd(const or_grid *g, double *const F[3], double *out[3])
{
    curl_any(g, F, out, 0, 0);
}

/* Transposes: the transpose of the periodic forward difference is minus
 * the backward one (and the curl flips the sign back), and the CKC
 * averaging is symmetric and commutes with the differences, so
 * curl_fwd^T = curl_bwd with the same averaging and curl_bwd^T = Yee's
 * curl_fwd. */
static void curl_fwd_T(const or_grid *g, double *const F[3], double *out[3])
{
    curl_any(g, F, out, 0, g->solver == 1);
}

static void curl_bwd_T(const or_grid *g, double *const F[3], double *out[3])
{
    curl_any(g, F, out, 1, 0);
}

static int64_t ncells(const or_grid *g)
{
    return (int64_t)g->n[0] * g->n[1] * g->n[2];
}

static double src_g(const or_source *src, int64_t step)
{
    if (!src || src->k_plane < 0 || !src->g || step < 0 || step >= src->n_g)
        return 0.0;
    return src->g[step];
}

void or_yee(const or_grid *g, or_fields *f, const or_source *src, int64_t step)
{
    int64_t nc = ncells(g);
    double *tmp = (double *)malloc(sizeof(double) * 3 * (size_t)nc);
    double *C[3] = {tmp, tmp + nc, tmp + 2 * nc};
    double mu0 = 1.0 / (g->eps0 * g->c * g->c);
    (void)mu0;
    curl_fwd(g, f->E, C);
    for (int m = 0; m < 3; ++m)
        for (int64_t i = 0; i < nc; ++i)
            f->B[m][i] -= 0.5 * g->dt * C[m][i];
    curl_bwd(g, f->B, C);
    for (int m = 0; m < 3; ++m)
        for (int64_t i = 0; i < nc; ++i)
            f->E[m][i] += g->dt * (g->c * g->c * C[m][i] - f->J[m][i] / g->eps0);
    double gs = src_g(src, step);
    if (src && src->k_plane >= 0 && src->amp) {
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i)
                f->E[0][idx3(g, i, j, src->k_plane)] += src->amp[i + (int64_t)g->n[0] * j] * gs;
    }
    curl_fwd(g, f->E, C);
    for (int m = 0; m < 3; ++m)
        for (int64_t i = 0; i < nc; ++i)
            f->B[m][i] -= 0.5 * g->dt * C[m][i];
    free(tmp);
}

/* ------------------------------------------------------------------ */
/* Diagnostics, FP64 (Sec. 2.6 reductions):
 *   out[0] U_E = dV/2 sum eps0 |E|^2      out[1] U_B = dV/2 sum |B|^2/mu0
 *   out[2] K   = sum w m c^2 (gamma-1)    out[3] Q   = sum q w
 *   out[4] P_z = sum w m u_z                                            */

void or_reduce(const or_grid *g, const or_species *s, const or_fields *f, double out[5])
{
    double dV = g->d[0] * g->d[1] * g->d[2];
    double mu0 = 1.0 / (g->eps0 * g->c * g->c);
    int64_t nc = ncells(g);
    double se = 0, sb = 0;
    for (int m = 0; m < 3; ++m)
        for (int64_t i = 0; i < nc; ++i) {
            se += f->E[m][i] * f->E[m][i];
            sb += f->B[m][i] * f->B[m][i];
        }
    out[0] = 0.5 * dV * g->eps0 * se;
    out[1] = 0.5 * dV * sb / mu0;
    double K = 0, Q = 0, P = 0;
    if (s) {
        for (int64_t p = 0; p < s->n; ++p) {
            double u[3] = {s->u[0][p], s->u[1][p], s->u[2][p]};
            double w = weight_of(s, p);
            double gm = gamma_of(u, g->c);
            /* gamma - 1 = (|u|/c)^2 / (gamma + 1), free of cancellation */
            double uu = (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / (g->c * g->c);
            K += w * s->m * g->c * g->c * uu / (gm + 1.0);
            Q += s->q * w;
            P += w * s->m * u[2];
        }
    }
    out[2] = K;
    out[3] = Q;
    out[4] = P;
}

/* Gauss-law residual (diagnostic of charge conservation).  Charge density
 * at the nodes from or_rho plus a uniform background equal to minus its
 * mean (the immobile neutralising ions); divergence of the edge field E at
 * the nodes by backward differences, div E(i,j,k) = sum_d (E_d(node) -
 * E_d(node - e_d)) / d_d.  res (may be NULL) receives div E - rho/eps0 per
 * node; out[0] = its 2-norm over the nodes, out[1] = the 2-norm of rho/eps0,
 * out[2] = sum of the species' rho times dV.                            */
void or_gauss(const or_grid *g, const or_species *s, const or_fields *f, double *res, double out[3])
{
    int64_t nc = ncells(g);
    double dV = g->d[0] * g->d[1] * g->d[2];
    double *rho = (double *)calloc((size_t)nc, sizeof(double));
    or_rho(g, s, rho);
    double mean = 0;
    for (int64_t i = 0; i < nc; ++i)
        mean += rho[i];
    out[2] = mean * dV;
    mean /= (double)nc;
    double sr = 0, sq = 0;
    for (int64_t k = 0; k < g->n[2]; ++k)
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i) {
                int64_t o = idx3(g, i, j, k);
                double div = (f->E[0][o] - f->E[0][idx3(g, i - 1, j, k)]) / g->d[0] +
                             (f->E[1][o] - f->E[1][idx3(g, i, j - 1, k)]) / g->d[1] +
                             (f->E[2][o] - f->E[2][idx3(g, i, j, k - 1)]) / g->d[2];
                double rt = (rho[o] - mean) / g->eps0;
                double r = div - rt;
                if (res)
                    res[o] = r;
                sr += r * r;
                sq += rt * rt;
            }
    out[0] = sqrt(sr);
    out[1] = sqrt(sq);
    free(rho);
}

/* ------------------------------------------------------------------ */
/* One full PIC step, in the order gather -> push -> deposit -> field
 * solve (Sec. 3.1 fuses gather and push; the step order is the standard
 * leapfrog one, fields at integer and momenta at half-integer times).
 * J is zeroed before each step's deposit.  diag (optional) receives the
 * five reductions after every step.                                   */

void or_step(const or_grid *g, or_species *s, or_fields *f, const or_source *src, int64_t step0, int32_t nsteps,
             double *diag)
{
    int64_t n = s->n, nc = ncells(g);
    double h = s->q * g->dt / (2.0 * s->m);
    double *disp[3];
    for (int d = 0; d < 3; ++d)
        disp[d] = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int32_t it = 0; it < nsteps; ++it) {
        int64_t step = step0 + it;
        const double *F[6];
        double *fbuf = gather_fields(g, f, F);
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < n; ++p) {
            int32_t cell[3];
            double off[3], E[3], B[3], u0[3], u1[3], dp[3];
            particle_pos(s, p, cell, off);
            for (int m = 0; m < 3; ++m) {
                E[m] = gather_one(g, F[m], STAG_E[m], cell, off, NULL);
                B[m] = gather_one(g, F[3 + m], STAG_B[m], cell, off, NULL);
                u0[m] = s->u[m][p];
            }
            push_momentum(g, h, u0, E, B, u1);
            displacement(g, u1, dp);
            for (int d = 0; d < 3; ++d) {
                s->u[d][p] = u1[d];
                disp[d][p] = dp[d];
            }
        }
        free(fbuf);
        for (int m = 0; m < 3; ++m)
            memset(f->J[m], 0, sizeof(double) * (size_t)nc);
        deposit_all(g, s, (const double *const *)disp, f->J);
        for (int64_t p = 0; p < n; ++p)
            for (int d = 0; d < 3; ++d)
                move_coord(&s->cell[d][p], &s->off[d][p], disp[d][p], g->n[d]);
        or_yee(g, f, src, step);
        if (diag)
            or_reduce(g, s, f, diag + 5 * (int64_t)it);
    }
    for (int d = 0; d < 3; ++d)
        free(disp[d]);
}

/* ------------------------------------------------------------------ */
/* Loss and its terminal adjoint: L = U_E + U_B of the given fields;
 * lam_E = eps0 dV E, lam_B = dV B / mu0, lam_x = lam_u = 0.           */

double or_loss(const or_grid *g, const or_fields *f, or_adjoint *lam, int64_t np)
{
    double out[5];
    or_reduce(g, NULL, f, out);
    if (lam) {
        double dV = g->d[0] * g->d[1] * g->d[2];
        double mu0 = 1.0 / (g->eps0 * g->c * g->c);
        int64_t nc = ncells(g);
        for (int m = 0; m < 3; ++m) {
            for (int64_t i = 0; i < nc; ++i) {
                lam->lE[m][i] = g->eps0 * dV * f->E[m][i];
                lam->lB[m][i] = dV * f->B[m][i] / mu0;
            }
            for (int64_t p = 0; p < np; ++p) {
                lam->lx[m][p] = 0.0;
                lam->lu[m][p] = 0.0;
            }
        }
    }
    return out[0] + out[1];
}

/* ------------------------------------------------------------------ */
/* Hand-written adjoint of one step (reverse mode).  On entry lam holds
 * dL/d(state n+1) = (x^{n+1}, u^{n+1/2}, E^{n+1}, B^{n+1}); on exit
 * dL/d(state n).  dA (n0*n1) accumulates dL/d(source amplitude map).
 * lam_x is with respect to the position in cell units.
 *
 * Field solve transpose (the periodic forward difference is minus the
 * transpose of the backward one, so curl_fwd^T = curl_bwd):
 * (with the CKC solver the curls below that transpose the B update's carry
 * its transverse averaging)
 *   lhatE = lE - dt/2 curl_bwd(lB);  dA += g(n) lhatE_x[:,:,k_s]
 *   lJ    = -dt/eps0 lhatE
 *   lB'   = lB + dt c^2 curl_fwd(lhatE)
 *   lE^n  = lhatE - dt/2 curl_bwd(lB');   lB^n = lB'
 * Particle part, per particle, in reverse order of the forward step:
 * deposit transpose (a gather of lJ, differentiated in both positions),
 * position transpose, Boris transpose, gather transpose (a scatter of the
 * field adjoints plus the gradient of the shapes).                      */

static void boris_adjoint(double h, double c, const double E[3], const double B[3], const boris_tape *T,
                          const double ub[3], double u0b[3], double Eb[3], double Bb[3])
{
    double ab[3], upb[3], sb[3], tb[3], tmp[3];
    for (int d = 0; d < 3; ++d) {
        Eb[d] = h * ub[d];
        ab[d] = ub[d];
    }
    /* u+ = a + u' x s */
    cross(T->s, ub, upb);    /* upb = s x ub */
    cross(ub, T->up, sb);    /* sb  = ub x u' */
    /* u' = a + a x t */
    cross(T->t, upb, tmp);   /* t x upb */
    for (int d = 0; d < 3; ++d)
        ab[d] += upb[d] + tmp[d];
    cross(upb, T->a, tb);    /* tb = upb x a */
    /* s = 2 t / (1 + |t|^2) */
    double den = 1.0 + T->tt;
    double tsb = T->t[0] * sb[0] + T->t[1] * sb[1] + T->t[2] * sb[2];
    for (int d = 0; d < 3; ++d)
        tb[d] += 2.0 * sb[d] / den - 4.0 * tsb * T->t[d] / (den * den);
    /* t = h B / gbar */
    double Btb = 0;
    for (int d = 0; d < 3; ++d) {
        Bb[d] = h * tb[d] / T->gbar;
        Btb += B[d] * tb[d];
    }
    double gb = -h * Btb / (T->gbar * T->gbar);
    /* gbar = sqrt(1 + |a|^2/c^2) */
    for (int d = 0; d < 3; ++d)
        ab[d] += gb * T->a[d] / (c * c * T->gbar);
    /* a = u0 + h E */
    for (int d = 0; d < 3; ++d) {
        u0b[d] = ab[d];
        Eb[d] += h * ab[d];
    }
    (void)E;
}

/* Deposit transpose: for phi = <lJ, J_p(x0, x1)> return d phi/d off0 and
 * d phi/d off1 (cell units). */
static void deposit_adjoint_one(const or_grid *g, const int32_t cell[3], const double off0[3], const double disp[3],
                                double qw, double *const lJ[3], double g0[3], double g1[3])
{
    esk_shapes E;
    esk_fill(g, off0, disp, &E);
    for (int d = 0; d < 3; ++d)
        g0[d] = g1[d] = 0.0;
    for (int m = 0; m < 3; ++m) {
        int p = (m + 1) % 3, q = (m + 2) % 3;
        double K = esk_coef(g, m, qw);
        for (int c = 0; c < DWN; ++c)
            for (int b = 0; b < DWN; ++b) {
                /* suffix sums of lJ along m over the window nodes that
                 * carry current (the top node carries none) */
                double Lam[DWN];
                double run = 0.0;
                Lam[DWN - 1] = 0.0;
                for (int a = DWN - 2; a >= 0; --a) {
                    run += lJ[m][esk_index(g, cell, m, a, b, c)];
                    Lam[a] = run;
                }
                double S0p = E.S0[p][b], S1p = E.S1[p][b], S0q = E.S0[q][c], S1q = E.S1[q][c];
                double D0p = E.D0[p][b], D1p = E.D1[p][b], D0q = E.D0[q][c], D1q = E.D1[q][c];
                double Y = (S0p * S0q + S1p * S1q) / 3.0 + (S1p * S0q + S0p * S1q) / 6.0;
                double Y0p = D0p * S0q / 3.0 + D0p * S1q / 6.0;
                double Y1p = D1p * S1q / 3.0 + D1p * S0q / 6.0;
                double Y0q = S0p * D0q / 3.0 + S1p * D0q / 6.0;
                double Y1q = S1p * D1q / 3.0 + S0p * D1q / 6.0;
                for (int a = 0; a < DWN; ++a) {
                    double L = K * Lam[a];
                    if (L == 0.0)
                        continue;
                    double ds = E.S1[m][a] - E.S0[m][a];
                    g0[m] += L * (-E.D0[m][a]) * Y;
                    g1[m] += L * E.D1[m][a] * Y;
                    g0[p] += L * ds * Y0p;
                    g1[p] += L * ds * Y1p;
                    g0[q] += L * ds * Y0q;
                    g1[q] += L * ds * Y1q;
                }
            }
    }
}

/* Gather transpose for one component: F_adj += S * vb, and the gradient
 * of the gathered value with respect to the offset times vb. */
static void gather_adjoint_one(const or_grid *g, const double *F, double *Fadj, const double st[3],
                               const int32_t cell[3], const double off[3], double vb, double gpos[3])
{
    double gr[3];
    gather_one(g, F, st, cell, off, gr);
    for (int d = 0; d < 3; ++d)
        gpos[d] += vb * gr[d];
    for (int c = GW0; c <= GW1; ++c)
        for (int b = GW0; b <= GW1; ++b)
            for (int a = GW0; a <= GW1; ++a) {
                double S = or_shape(g->order, off[0] - a - st[0]) * or_shape(g->order, off[1] - b - st[1]) *
                           or_shape(g->order, off[2] - c - st[2]);
                if (S != 0.0)
                    Fadj[idx3(g, (int64_t)cell[0] + a, (int64_t)cell[1] + b, (int64_t)cell[2] + c)] += S * vb;
            }
}

void or_step_adjoint(const or_grid *g, const or_species *s, const or_fields *f, const or_source *src, int64_t step,
                     or_adjoint *lam, double *dA)
{
    int64_t nc = ncells(g), n = s->n;
    double *buf = (double *)malloc(sizeof(double) * 9 * (size_t)nc);
    double *hatE[3] = {buf, buf + nc, buf + 2 * nc};
    double *C[3] = {buf + 3 * nc, buf + 4 * nc, buf + 5 * nc};
    double *lJ[3] = {buf + 6 * nc, buf + 7 * nc, buf + 8 * nc};
    /* field solve transpose */
    curl_fwd_T(g, lam->lB, C);
    for (int m = 0; m < 3; ++m)
        for (int64_t i = 0; i < nc; ++i)
            hatE[m][i] = lam->lE[m][i] - 0.5 * g->dt * C[m][i];
    if (src && src->k_plane >= 0 && dA) {
        double gs = src_g(src, step);
        for (int64_t j = 0; j < g->n[1]; ++j)
            for (int64_t i = 0; i < g->n[0]; ++i)
                dA[i + (int64_t)g->n[0] * j] += gs * hatE[0][idx3(g, i, j, src->k_plane)];
    }
    for (int m = 0; m < 3; ++m)
        for (int64_t i = 0; i < nc; ++i)
            lJ[m][i] = -g->dt / g->eps0 * hatE[m][i];
    curl_bwd_T(g, hatE, C);
    for (int m = 0; m < 3; ++m)
        for (int64_t i = 0; i < nc; ++i)
            lam->lB[m][i] += g->dt * g->c * g->c * C[m][i];
    curl_fwd_T(g, lam->lB, C);
    for (int m = 0; m < 3; ++m)
        for (int64_t i = 0; i < nc; ++i)
            lam->lE[m][i] = hatE[m][i] - 0.5 * g->dt * C[m][i];

    /* particle part: the gather transpose scatters into lE, lB (or, with a
     * filter, into the adjoints of the filtered fields, which the filter's
     * transpose (itself) adds to lE, lB at the end); particles are split
     * over threads, each scattering into private buffers that are added to
     * the targets afterwards in thread order (as the forward's current) */
    const double *F[6];
    double *fbuf = gather_fields(g, f, F);
    double *lF[6], *lfbuf = NULL;
    for (int m = 0; m < 3; ++m) {
        lF[m] = lam->lE[m];
        lF[3 + m] = lam->lB[m];
    }
    if (fbuf) {
        lfbuf = (double *)calloc(6 * (size_t)nc, sizeof(double));
        for (int m = 0; m < 6; ++m)
            lF[m] = lfbuf + m * nc;
    }
    double h = s->q * g->dt / (2.0 * s->m);
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double *priv = (double *)calloc((size_t)nt * 6 * (size_t)nc, sizeof(double));
#pragma omp parallel num_threads(nt)
    {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    double *lFt[6];
    for (int m = 0; m < 6; ++m)
        lFt[m] = priv + ((size_t)t * 6 + m) * nc;
#pragma omp for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        int32_t cell[3];
        double off[3], E[3], B[3], u0[3], u1[3], dp[3];
        boris_tape T;
        particle_pos(s, p, cell, off);
        for (int m = 0; m < 3; ++m) {
            E[m] = gather_one(g, F[m], STAG_E[m], cell, off, NULL);
            B[m] = gather_one(g, F[3 + m], STAG_B[m], cell, off, NULL);
            u0[m] = s->u[m][p];
        }
        if (g->pusher == 1)
            vay(h, g->c, u0, E, B, u1);
        else
            boris(h, g->c, u0, E, B, u1, &T);
        displacement(g, u1, dp);
        /* deposit transpose */
        double g0[3], g1[3];
        deposit_adjoint_one(g, cell, off, dp, s->q * weight_of(s, p), lJ, g0, g1);
        double lx1[3], lx0[3];
        for (int d = 0; d < 3; ++d) {
            lx1[d] = lam->lx[d][p] + g1[d];
            lx0[d] = g0[d];
        }
        /* position transpose: off1 = off0 + dt u1 / (gamma1 dx) */
        double gm = gamma_of(u1, g->c);
        double v[3], uv = 0;
        for (int d = 0; d < 3; ++d) {
            v[d] = g->dt * lx1[d] / g->d[d];
            uv += u1[d] * v[d];
            lx0[d] += lx1[d];
        }
        double ub[3];
        for (int d = 0; d < 3; ++d)
            ub[d] = lam->lu[d][p] + v[d] / gm - u1[d] * uv / (gm * gm * gm * g->c * g->c);
        /* momentum-update transpose */
        double u0b[3], Eb[3], Bb[3];
        if (g->pusher == 1)
            vay_adjoint(h, g->c, u0, E, B, ub, u0b, Eb, Bb);
        else
            boris_adjoint(h, g->c, E, B, &T, ub, u0b, Eb, Bb);
        /* gather transpose */
        for (int m = 0; m < 3; ++m) {
            gather_adjoint_one(g, F[m], lFt[m], STAG_E[m], cell, off, Eb[m], lx0);
            gather_adjoint_one(g, F[3 + m], lFt[3 + m], STAG_B[m], cell, off, Bb[m], lx0);
        }
        for (int d = 0; d < 3; ++d) {
            lam->lx[d][p] = lx0[d];
            lam->lu[d][p] = u0b[d];
        }
    }
    }
    for (int t = 0; t < nt; ++t)
        for (int m = 0; m < 6; ++m) {
            const double *src = priv + ((size_t)t * 6 + m) * nc;
            for (int64_t i = 0; i < nc; ++i)
                lF[m][i] += src[i];
        }
    free(priv);
    if (lfbuf) {
        for (int m = 0; m < 6; ++m) {
            double *dst = m < 3 ? lam->lE[m] : lam->lB[m - 3];
            filter_z(g, g->gather_filter + 4 * m, lF[m], C[0]);
            for (int64_t i = 0; i < nc; ++i)
                dst[i] += C[0][i];
        }
    }
    free(lfbuf);
    free(fbuf);
    free(buf);
}
