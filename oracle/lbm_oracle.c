/*
 * Plain FP64 CPU oracle for the volumetric curvilinear lattice Boltzmann step
 * (Chekhlov, Staroselsky, Zhang, Chen, arXiv:2301.01868).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call this
 * file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or helper with the HIP
 * library: the lattice tables below are typed in from the paper's appendices,
 * and every formula is written in the paper's own f-units with literal index
 * sums, in the order the paper states them.  Compiled with -O2
 * -ffp-contract=off and no fast-math.
 *
 * Conventions (the paper's, Sec. 2 and App. B):
 *   - computational lattice q = (q1, q2) with unit spacing; q1 is the
 *     wall-normal ("radial"/"horizontal") index, q2 the periodic
 *     ("azimuthal"/"vertical") index;
 *   - interior cells i = 0..n1-1 (q1), j = 0..n2-1 (q2), stored row-major with
 *     j fastest; populations are stored cell-major, P[cell*Q + alpha];
 *   - the mapping x(q) is given on the halo-extended index range
 *     (n1+2h) x (n2+2h), halo h >= c_max + 1, ghost rows beyond a wall holding
 *     the symmetrically continued geometry.
 *
 * Readings of places where the paper is silent or garbled (each is listed in
 * the design notes):
 *   - D2Q21 weights are the unique solution of the isotropy conditions
 *     (App. A): the printed 7/432 and 7/1620 do not sum to one; 1/432, 1/1620;
 *   - velocity numbering is inferred from the App. B index tables;
 *   - wall sources: the source node x - c_alpha beyond a wall is replaced by
 *     its mirror image across the wall plane (App. B.2 continues the source
 *     through the wall by symmetry without giving the rule); no-slip takes the bounce-back direction
 *     alpha*, a moving wall the specular direction alpha-hat plus
 *     2 w_alpha m(z) c^2_alpha (U0^2 - Utilde^2(z)) / T0 with m(z) the
 *     number of particles in the image cell z from its last collision, only
 *     the tangential (q2) component kept (App. B.3);
 *   - the external body force enters as F_total = F_inertial + rho a_ext
 *     (contravariant, not lagged);
 *   - the lagged force term uses the own cell's previous post-collision value
 *     N'(q, t-1), which is the stored state before streaming (Sec. 2, the
 *     explicit split of the implicit relation); the initial state serves as
 *     N'(q, -1).
 *
 * Parity unpinned (no value in the paper to check against, only agreement
 * with the GPU path): the first-step lag N'(q, -1) beyond the rest state
 * staying at rest on uniform metrics, and D2Q21 accuracy next to walls.  (The
 * steady-state residual, a definition chosen by this project since the paper
 * gives none, is formed by the tests from this oracle's moments.)  Every other
 * part is checked by the CPU tests against closed forms, invariants or
 * textbook special cases.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_QMAX 21

enum { ORC_PERIODIC = 0, ORC_NOSLIP = 1, ORC_MOVING = 2 };

/* ---------------------------------------------------------------------------
 * Lattices (App. A and App. B).
 * Velocity vectors: 0 rest; 1..4 (1,0),(0,1),(-1,0),(0,-1); 5..8 (1,1),
 * (-1,1),(-1,-1),(1,-1); 9..12 twice 1..4; 13..16 twice 5..8; 17..20 three
 * times 1..4.  The App. B tables (bounce-back, specular) fix this numbering up
 * to the choice of which axis is "1".
 * ------------------------------------------------------------------------- */
static const int C21x[21] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0, 2, -2, -2, 2, 3, 0, -3, 0};
static const int C21y[21] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2, 2, 2, -2, -2, 0, 3, 0, -3};

/* App. A, Table "D2Q9 lattice weights". */
static const double W9[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* App. A, Table "D2Q21 lattice weights", with the last two classes read as
 * 1/432 and 1/1620 (the isotropy conditions of App. A fix them uniquely). */
static const double W21[21] = {
    91.0 / 324.0,
    1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0,
    2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0,
    7.0 / 360.0, 7.0 / 360.0, 7.0 / 360.0, 7.0 / 360.0,
    1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0,
    1.0 / 1620.0, 1.0 / 1620.0, 1.0 / 1620.0, 1.0 / 1620.0};

/* App. B, Table "Bounce-back" (alpha -> alpha*) and Table "Specular
 * Reflection" (alpha -> alpha-hat), typed in as printed.  Directions with
 * c^1 = 0 never cross a q1 wall and are not listed there (-1 here). */
static const int BB21[21] = {-1, 3, -1, 1, -1, 7, 8, 5, 6, 11, -1, 9, -1, 15, 16, 13, 14, 19, -1, 17, -1};
static const int SP21[21] = {-1, 3, -1, 1, -1, 6, 5, 8, 7, 11, -1, 9, -1, 14, 13, 16, 15, 19, -1, 17, -1};

void orc_lattice(int q, int *cx, int *cy, double *w, double *T0, int *bb, int *sp)
{
    for (int a = 0; a < q; ++a) {
        cx[a] = C21x[a];
        cy[a] = C21y[a];
        w[a] = (q == 9) ? W9[a] : W21[a];
        bb[a] = BB21[a];
        sp[a] = SP21[a];
    }
    *T0 = (q == 9) ? 1.0 / 3.0 : 2.0 / 3.0;
}

/* ---------------------------------------------------------------------------
 * Grid state.
 * ------------------------------------------------------------------------- */
typedef struct {
    int q, n1, n2, h, H1, H2;
    int periodic1;
    int bc[2];         /* q1 low side (i = 1/2), q1 high side (i = n1 + 1/2) */
    double ut[2];      /* contravariant tangential (q2) wall velocity U0^2 */
    double tau, a_ext[2], T0;
    int cx[ORC_QMAX], cy[ORC_QMAX], bb[ORC_QMAX], sp[ORC_QMAX];
    double w[ORC_QMAX];
    double *X, *Y;                 /* mapping on the halo range */
    double *g1x, *g1y, *g2x, *g2y; /* tangent basis on the halo range */
    double *Jgeo;                  /* geometric volume (interior) */
    double *Jused;                 /* J, or J' after the no-flow adjustment */
    double *P, *Pn;                /* post-collision populations [cell][alpha] */
    double *side_m, *side_u1, *side_u2, *side_mn, *side_u1n, *side_u2n;
    long step;
    int iters;         /* 0: lagged N'(q, t-1) in the force; k > 0: k fixed-point
                          re-evaluations with the current N'(q, t) */
} orc_grid;

static inline int hidx(const orc_grid *g, int a, int b) { return a * g->H2 + b; }

/* Eq. (tangent): g_i(q) = [D_i(q) - D_{-i}(q)] / (2 dx), D from Eq. (distance);
 * coordinates are in lattice units (dx = 1). */
static void orc_geometry_init(orc_grid *g)
{
    int H1 = g->H1, H2 = g->H2;
    for (int a = 0; a < H1; ++a)
        for (int b = 0; b < H2; ++b) {
            int k = hidx(g, a, b);
            if (a == 0 || b == 0 || a == H1 - 1 || b == H2 - 1) {
                g->g1x[k] = g->g1y[k] = g->g2x[k] = g->g2y[k] = NAN;
                continue;
            }
            double D1x = g->X[hidx(g, a + 1, b)] - g->X[k], D1y = g->Y[hidx(g, a + 1, b)] - g->Y[k];
            double Dm1x = g->X[hidx(g, a - 1, b)] - g->X[k], Dm1y = g->Y[hidx(g, a - 1, b)] - g->Y[k];
            double D2x = g->X[hidx(g, a, b + 1)] - g->X[k], D2y = g->Y[hidx(g, a, b + 1)] - g->Y[k];
            double Dm2x = g->X[hidx(g, a, b - 1)] - g->X[k], Dm2y = g->Y[hidx(g, a, b - 1)] - g->Y[k];
            g->g1x[k] = (D1x - Dm1x) / 2.0;
            g->g1y[k] = (D1y - Dm1y) / 2.0;
            g->g2x[k] = (D2x - Dm2x) / 2.0;
            g->g2y[k] = (D2y - Dm2y) / 2.0;
        }
    for (int i = 0; i < g->n1; ++i)
        for (int j = 0; j < g->n2; ++j) {
            int k = hidx(g, i + g->h, j + g->h);
            /* Eq. (metric) with g_3 = z-hat: J = (g_1 x g_2) . z-hat */
            g->Jgeo[i * g->n2 + j] = g->g1x[k] * g->g2y[k] - g->g1y[k] * g->g2x[k];
        }
}

/* Tangent vector g_m (m = 0 for g_1, 1 for g_2) at halo position (a, b). */
static inline void tangent(const orc_grid *g, int m, int a, int b, double v[2])
{
    int k = hidx(g, a, b);
    if (m == 0) { v[0] = g->g1x[k]; v[1] = g->g1y[k]; }
    else        { v[0] = g->g2x[k]; v[1] = g->g2y[k]; }
}

/* Eq. (covectors): co-tangent basis g^i with g_i . g^j = delta_i^j.  In 2D,
 * with g_3 = z-hat, g^1 = (g_2 x z)/J and g^2 = (z x g_1)/J; J is the
 * geometric volume of Eq. (metric). */
static inline void cotangent(const orc_grid *g, int m, int a, int b, double v[2])
{
    int k = hidx(g, a, b);
    double J = g->g1x[k] * g->g2y[k] - g->g1y[k] * g->g2x[k];
    if (m == 0) { v[0] = g->g2y[k] / J; v[1] = -g->g2x[k] / J; }
    else        { v[0] = -g->g1y[k] / J; v[1] = g->g1x[k] / J; }
}

/* Inverse metric g^{ij} = g^i . g^j (Eq. covectors). */
static inline void inv_metric(const orc_grid *g, int a, int b, double G[2][2])
{
    double c0[2], c1[2];
    cotangent(g, 0, a, b, c0);
    cotangent(g, 1, a, b, c1);
    G[0][0] = c0[0] * c0[0] + c0[1] * c0[1];
    G[0][1] = c0[0] * c1[0] + c0[1] * c1[1];
    G[1][0] = G[0][1];
    G[1][1] = c1[0] * c1[0] + c1[1] * c1[1];
}

/* Eq. (gamma): Theta^i_j(p, q) = [g_j(p) - g_j(q)] . g^i(q). */
static inline double Theta(const orc_grid *g, int i, int j, int pa, int pb, int qa, int qb)
{
    double gp[2], gq[2], co[2];
    tangent(g, j, pa, pb, gp);
    tangent(g, j, qa, qb, gq);
    cotangent(g, i, qa, qb, co);
    return (gp[0] - gq[0]) * co[0] + (gp[1] - gq[1]) * co[1];
}

/* Eq. (equilibrium), the literal index sums over i, j, k in {1, 2}. */
static void feq_literal(const orc_grid *g, double rho, const double U[2], const double Ut[2],
                        double G[2][2], double *feq)
{
    const double T0 = g->T0;
    for (int al = 0; al < g->q; ++al) {
        double c[2] = {(double)g->cx[al], (double)g->cy[al]};
        double s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int i = 0; i < 2; ++i)
            s1 += c[i] * U[i] / T0;
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                double dij = (i == j) ? 1.0 : 0.0;
                s2 += (c[i] * c[j] / T0 - dij) * ((G[i][j] - dij) * T0 + Ut[i] * Ut[j]);
            }
        s2 /= 2.0 * T0;
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                for (int k = 0; k < 2; ++k) {
                    double dij = (i == j) ? 1.0 : 0.0;
                    double djk = (j == k) ? 1.0 : 0.0;
                    double dki = (k == i) ? 1.0 : 0.0;
                    double H3 = c[i] * c[j] * c[k] - T0 * (c[i] * djk + c[j] * dki + c[k] * dij);
                    double B3 = T0 * ((G[i][j] * Ut[k] - dij * U[k]) + (G[j][k] * Ut[i] - djk * U[i]) +
                                      (G[k][i] * Ut[j] - dki * U[j])) +
                                Ut[i] * Ut[j] * Ut[k];
                    s3 += H3 * B3;
                }
        s3 /= 6.0 * T0 * T0 * T0;
        feq[al] = rho * g->w[al] * (1.0 + s1 + s2 + s3);
    }
}

void orc_feq(int q, double rho, const double *U, const double *Ut, const double *G3, double *out)
{
    orc_grid g;
    memset(&g, 0, sizeof g);
    g.q = q;
    double T0;
    orc_lattice(q, g.cx, g.cy, g.w, &T0, g.bb, g.sp);
    g.T0 = T0;
    double G[2][2] = {{G3[0], G3[1]}, {G3[1], G3[2]}};
    feq_literal(&g, rho, U, Ut, G, out);
}

/* ---------------------------------------------------------------------------
 * Streaming source (Eq. adv and App. B).  For target (i, j) and direction
 * alpha, returns the source interior cell, the source direction, and which
 * wall (0 none, 1 low, 2 high) the hop crossed.
 * ------------------------------------------------------------------------- */
static void stream_source(const orc_grid *g, int i, int j, int al, int *si, int *sj, int *beta, int *wall)
{
    int ti = i - g->cx[al];
    int tj = j - g->cy[al];
    /* App. B.1: the q2 direction is periodic. */
    tj = ((tj % g->n2) + g->n2) % g->n2;
    *sj = tj;
    *beta = al;
    *wall = 0;
    if (ti >= 0 && ti < g->n1) {
        *si = ti;
        return;
    }
    if (g->periodic1) {
        *si = ((ti % g->n1) + g->n1) % g->n1;
        return;
    }
    int side = (ti < 0) ? 0 : 1;
    /* mirror image across the wall plane at i = 1/2 or i = n1 + 1/2
     * (1-based), i.e. row -1 - ti or 2 n1 - 1 - ti (0-based) */
    *si = (side == 0) ? (-1 - ti) : (2 * g->n1 - 1 - ti);
    /* App. B.2 / B.3: bounce-back for no-slip, specular reflection for a
     * moving wall. */
    *beta = (g->bc[side] == ORC_NOSLIP) ? g->bb[al] : g->sp[al];
    *wall = side + 1;
}

/* Pulled value N_alpha(q, t+1) from the current post-collision field. */
static double pulled(const orc_grid *g, const double *P, const double *sm, const double *su2, int i, int j, int al)
{
    int si, sj, beta, wall;
    stream_source(g, i, j, al, &si, &sj, &beta, &wall);
    int s = si * g->n2 + sj;
    double v = P[(size_t)s * g->q + beta];
    if (wall && g->bc[wall - 1] == ORC_MOVING) {
        /* App. B.3 moving-wall correction, tangential component only */
        double Uw = g->ut[wall - 1];
        v += 2.0 * g->w[al] * sm[s] * (double)g->cy[al] * (Uw - su2[s]) / g->T0;
    }
    return v;
}

/* Full per-cell update for interior cell (i, j) from field P (and side state).
 * Writes N' into out[Q]; optional diagnostics into diag (see below). */
typedef struct {
    double N[ORC_QMAX], m, rho, U[2], F[2], Ut[2], feq[ORC_QMAX], dPi[2][2], dN[ORC_QMAX], Np[ORC_QMAX];
} orc_cell_diag;

static void cell_update(const orc_grid *g, const double *P, const double *sm, const double *su2, int i, int j,
                        double *out, orc_cell_diag *dg, int moments_only)
{
    const int Q = g->q;
    const double T0 = g->T0;
    const int qa = i + g->h, qb = j + g->h;
    const int cell = i * g->n2 + j;
    const double J = g->Jused[cell];
    double N[ORC_QMAX], f[ORC_QMAX], feq[ORC_QMAX];
    const double *Pown = P + (size_t)cell * Q;

    for (int al = 0; al < Q; ++al)
        N[al] = pulled(g, P, sm, su2, i, j, al);
    /* Eq. (dist) and Eqs. (moments), (vcomp) */
    double rho = 0.0, rU[2] = {0.0, 0.0};
    for (int al = 0; al < Q; ++al) {
        f[al] = N[al] / J;
        rho += f[al];
        rU[0] += g->cx[al] * f[al];
        rU[1] += g->cy[al] * f[al];
    }
    double U[2] = {rU[0] / rho, rU[1] / rho};
    double Nown[ORC_QMAX];
    for (int al = 0; al < Q; ++al)
        Nown[al] = Pown[al];
    double F[2], Ut[2], G[2][2], dPi[2][2];
    for (int it = 0; it <= (moments_only ? 0 : g->iters); ++it) {
        /* Eq. (compo-constr) with N'(q, t-1) in place of N'(q, t) (first
         * pass) plus the external body force rho a_ext */
        for (int ii = 0; ii < 2; ++ii) {
            double s = 0.0;
            for (int al = 0; al < Q; ++al) {
                int c[2] = {g->cx[al], g->cy[al]};
                for (int jj = 0; jj < 2; ++jj) {
                    if (c[jj] == 0)
                        continue;
                    double thp = Theta(g, ii, jj, qa + c[0], qb + c[1], qa, qb);
                    double thm = Theta(g, ii, jj, qa - c[0], qb - c[1], qa, qb);
                    s += c[jj] * (thp * Nown[al] - thm * N[al]);
                }
            }
            F[ii] = -s / (2.0 * J) + rho * g->a_ext[ii];
        }
        /* physical velocity: Utilde = U + a/2, a = F / rho */
        Ut[0] = U[0] + 0.5 * F[0] / rho;
        Ut[1] = U[1] + 0.5 * F[1] / rho;
        inv_metric(g, qa, qb, G);
        feq_literal(g, rho, U, Ut, G, feq);
        if (dg) {
            for (int al = 0; al < Q; ++al) { dg->N[al] = N[al]; dg->feq[al] = feq[al]; }
            dg->m = rho * J; dg->rho = rho;
            dg->U[0] = U[0]; dg->U[1] = U[1]; dg->F[0] = F[0]; dg->F[1] = F[1];
            dg->Ut[0] = Ut[0]; dg->Ut[1] = Ut[1];
        }
        if (moments_only)
            return;
        /* Eq. (delta-flux) */
        const double pre = -0.5 * (1.0 - 1.0 / (2.0 * g->tau));
        for (int ii = 0; ii < 2; ++ii)
            for (int jj = 0; jj < 2; ++jj) {
                double s = 0.0;
                for (int al = 0; al < Q; ++al) {
                    int c[2] = {g->cx[al], g->cy[al]};
                    for (int kk = 0; kk < 2; ++kk) {
                        double ck = c[ii] * c[kk];
                        if (ck == 0.0)
                            continue;
                        double thp = Theta(g, jj, kk, qa + c[0], qb + c[1], qa, qb);
                        double thm = Theta(g, jj, kk, qa - c[0], qb - c[1], qa, qb);
                        s += ck * (thp - thm) * feq[al];
                    }
                }
                dPi[ii][jj] = pre * s;
            }
        /* Eq. (deltaN), Eq. (collide), Eq. (lbe) */
        for (int al = 0; al < Q; ++al) {
            double c[2] = {(double)g->cx[al], (double)g->cy[al]};
            double t1 = 0.0, t2 = 0.0;
            for (int jj = 0; jj < 2; ++jj)
                t1 += c[jj] * F[jj] / T0;
            for (int jj = 0; jj < 2; ++jj)
                for (int kk = 0; kk < 2; ++kk)
                    t2 += (c[jj] * c[kk] / T0 - (jj == kk ? 1.0 : 0.0)) * dPi[jj][kk] / T0;
            double dN = g->w[al] * J * (t1 + t2);
            double Om = -J * (f[al] - feq[al]) / g->tau;
            out[al] = N[al] + Om + dN;
            if (dg) dg->dN[al] = dN, dg->Np[al] = out[al];
        }
        /* optional fixed-point re-evaluation of the implicit force relation
         * (Sec. 2 names iteration as the alternative to the one-step lag) */
        for (int al = 0; al < Q; ++al)
            Nown[al] = out[al];
    }
    if (dg) {
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                dg->dPi[a][b] = dPi[a][b];
    }
}

/* ---------------------------------------------------------------------------
 * Public API (ctypes).
 * ------------------------------------------------------------------------- */
orc_grid *orc_create(int q, int n1, int n2, int h, const double *X, const double *Y, int periodic1, int bc_lo,
                     int bc_hi, double ut_lo, double ut_hi, double tau, double ax, double ay)
{
    if (q != 9 && q != 21)
        return NULL;
    int cmax = (q == 9) ? 1 : 3;
    if (h < cmax + 1 || n1 < 1 || n2 < 1 || !(tau > 0.5))
        return NULL;
    if (!periodic1 && n1 < cmax)
        return NULL;
    orc_grid *g = (orc_grid *)calloc(1, sizeof(orc_grid));
    g->q = q; g->n1 = n1; g->n2 = n2; g->h = h;
    g->H1 = n1 + 2 * h; g->H2 = n2 + 2 * h;
    g->periodic1 = periodic1;
    g->bc[0] = periodic1 ? ORC_PERIODIC : bc_lo;
    g->bc[1] = periodic1 ? ORC_PERIODIC : bc_hi;
    g->ut[0] = ut_lo; g->ut[1] = ut_hi;
    g->tau = tau; g->a_ext[0] = ax; g->a_ext[1] = ay;
    orc_lattice(q, g->cx, g->cy, g->w, &g->T0, g->bb, g->sp);
    size_t nh = (size_t)g->H1 * g->H2, nc = (size_t)n1 * n2;
    g->X = (double *)malloc(nh * sizeof(double));
    g->Y = (double *)malloc(nh * sizeof(double));
    memcpy(g->X, X, nh * sizeof(double));
    memcpy(g->Y, Y, nh * sizeof(double));
    g->g1x = (double *)malloc(nh * sizeof(double));
    g->g1y = (double *)malloc(nh * sizeof(double));
    g->g2x = (double *)malloc(nh * sizeof(double));
    g->g2y = (double *)malloc(nh * sizeof(double));
    g->Jgeo = (double *)malloc(nc * sizeof(double));
    g->Jused = (double *)malloc(nc * sizeof(double));
    g->P = (double *)calloc(nc * q, sizeof(double));
    g->Pn = (double *)calloc(nc * q, sizeof(double));
    g->side_m = (double *)calloc(nc, sizeof(double));
    g->side_u1 = (double *)calloc(nc, sizeof(double));
    g->side_u2 = (double *)calloc(nc, sizeof(double));
    g->side_mn = (double *)calloc(nc, sizeof(double));
    g->side_u1n = (double *)calloc(nc, sizeof(double));
    g->side_u2n = (double *)calloc(nc, sizeof(double));
    orc_geometry_init(g);
    memcpy(g->Jused, g->Jgeo, nc * sizeof(double));
    return g;
}

void orc_destroy(orc_grid *g)
{
    if (!g) return;
    free(g->X); free(g->Y); free(g->g1x); free(g->g1y); free(g->g2x); free(g->g2y);
    free(g->Jgeo); free(g->Jused); free(g->P); free(g->Pn);
    free(g->side_m); free(g->side_u1); free(g->side_u2);
    free(g->side_mn); free(g->side_u1n); free(g->side_u2n);
    free(g);
}

/* Volume used in Eq. (dist): NULL restores the geometric J; otherwise the
 * "no flow" adjusted J' (Sec. 3.1). */
void orc_set_volume(orc_grid *g, const double *J)
{
    size_t nc = (size_t)g->n1 * g->n2;
    if (J) memcpy(g->Jused, J, nc * sizeof(double));
    else memcpy(g->Jused, g->Jgeo, nc * sizeof(double));
}

/* Initial state: N = J f^eq(rho0, U = Utilde = u0; g^ij), which also serves as
 * the lagged N'(q, -1).  u0: contravariant [cell][2] or NULL (rest). */
void orc_init(orc_grid *g, double rho0, const double *u0)
{
    for (int i = 0; i < g->n1; ++i)
        for (int j = 0; j < g->n2; ++j) {
            int cell = i * g->n2 + j;
            double U[2] = {0.0, 0.0};
            if (u0) { U[0] = u0[2 * cell]; U[1] = u0[2 * cell + 1]; }
            double G[2][2], feq[ORC_QMAX];
            inv_metric(g, i + g->h, j + g->h, G);
            feq_literal(g, rho0, U, U, G, feq);
            double m = 0.0;
            for (int al = 0; al < g->q; ++al) {
                g->P[(size_t)cell * g->q + al] = g->Jused[cell] * feq[al];
                m += g->P[(size_t)cell * g->q + al];
            }
            g->side_m[cell] = m;
            g->side_u1[cell] = U[0];
            g->side_u2[cell] = U[1];
        }
    g->step = 0;
}

void orc_step(orc_grid *g, long nsteps, int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    (void)nthreads;
#endif
    for (long s = 0; s < nsteps; ++s) {
#pragma omp parallel for schedule(static) num_threads(nthreads)
        for (int i = 0; i < g->n1; ++i) {
            orc_cell_diag dg;
            for (int j = 0; j < g->n2; ++j) {
                int cell = i * g->n2 + j;
                cell_update(g, g->P, g->side_m, g->side_u2, i, j, g->Pn + (size_t)cell * g->q, &dg, 0);
                g->side_mn[cell] = dg.m;
                g->side_u1n[cell] = dg.Ut[0];
                g->side_u2n[cell] = dg.Ut[1];
            }
        }
        double *t;
        t = g->P; g->P = g->Pn; g->Pn = t;
        t = g->side_m; g->side_m = g->side_mn; g->side_mn = t;
        t = g->side_u1; g->side_u1 = g->side_u1n; g->side_u1n = t;
        t = g->side_u2; g->side_u2 = g->side_u2n; g->side_u2n = t;
        g->step++;
    }
}

long orc_get_step(const orc_grid *g) { return g->step; }
void orc_set_iterations(orc_grid *g, int k) { g->iters = k; }

void orc_get_state(const orc_grid *g, double *P) { memcpy(P, g->P, (size_t)g->n1 * g->n2 * g->q * sizeof(double)); }
void orc_set_state(orc_grid *g, const double *P) { memcpy(g->P, P, (size_t)g->n1 * g->n2 * g->q * sizeof(double)); }

/* Side state: number of particles m and physical velocity Utilde (both
 * components) of every interior cell from its last collision. */
void orc_get_side(const orc_grid *g, double *m, double *u1, double *u2)
{
    size_t nc = (size_t)g->n1 * g->n2;
    memcpy(m, g->side_m, nc * sizeof(double));
    if (u1) memcpy(u1, g->side_u1, nc * sizeof(double));
    memcpy(u2, g->side_u2, nc * sizeof(double));
}
void orc_set_side(orc_grid *g, const double *m, const double *u2)
{
    size_t nc = (size_t)g->n1 * g->n2;
    memcpy(g->side_m, m, nc * sizeof(double));
    memcpy(g->side_u2, u2, nc * sizeof(double));
}

/* Moments of the next pre-collision state (pull + moments + force):
 * m = sum N, U^i, Utilde^i (contravariant), per interior cell. */
void orc_moments(const orc_grid *g, double *m, double *U, double *Ut, int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    (void)nthreads;
#endif
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int i = 0; i < g->n1; ++i) {
        orc_cell_diag dg;
        double dummy[ORC_QMAX];
        for (int j = 0; j < g->n2; ++j) {
            int cell = i * g->n2 + j;
            cell_update(g, g->P, g->side_m, g->side_u2, i, j, dummy, &dg, 1);
            m[cell] = dg.m;
            U[2 * cell] = dg.U[0]; U[2 * cell + 1] = dg.U[1];
            Ut[2 * cell] = dg.Ut[0]; Ut[2 * cell + 1] = dg.Ut[1];
        }
    }
}

/* One step for selected cells from the current state, without committing. */
void orc_step_cells(const orc_grid *g, int ncells, const int *cells, double *out)
{
    for (int k = 0; k < ncells; ++k) {
        int cell = cells[k];
        cell_update(g, g->P, g->side_m, g->side_u2, cell / g->n2, cell % g->n2, out + (size_t)k * g->q, NULL, 0);
    }
}

/* Diagnostics of one cell's update (for the per-cell identity tests).
 * out layout: N[Q], m, rho, U[2], F[2], Ut[2], feq[Q], dPi[4], dN[Q], Np[Q]. */
void orc_cell_detail(const orc_grid *g, int cell, double *out)
{
    orc_cell_diag dg;
    double tmp[ORC_QMAX];
    cell_update(g, g->P, g->side_m, g->side_u2, cell / g->n2, cell % g->n2, tmp, &dg, 0);
    int Q = g->q, o = 0;
    for (int a = 0; a < Q; ++a) out[o++] = dg.N[a];
    out[o++] = dg.m; out[o++] = dg.rho;
    out[o++] = dg.U[0]; out[o++] = dg.U[1];
    out[o++] = dg.F[0]; out[o++] = dg.F[1];
    out[o++] = dg.Ut[0]; out[o++] = dg.Ut[1];
    for (int a = 0; a < Q; ++a) out[o++] = dg.feq[a];
    out[o++] = dg.dPi[0][0]; out[o++] = dg.dPi[0][1]; out[o++] = dg.dPi[1][0]; out[o++] = dg.dPi[1][1];
    for (int a = 0; a < Q; ++a) out[o++] = dg.dN[a];
    for (int a = 0; a < Q; ++a) out[o++] = dg.Np[a];
}

/* Geometry export: per interior cell J (geometric), g^11, g^12, g^22, the
 * tangent basis, and for every alpha the sums
 *   Aplus^i_alpha  = sum_j c^j_alpha Theta^i_j(q + c_alpha, q)
 *   Aminus^i_alpha = sum_j c^j_alpha Theta^i_j(q - c_alpha, q)
 * (layout per cell: J, G11, G12, G22, g1x, g1y, g2x, g2y, Aplus[Q][2],
 * Aminus[Q][2]). */
void orc_geometry(const orc_grid *g, double *out)
{
    int Q = g->q, W = 8 + 4 * Q;
    for (int i = 0; i < g->n1; ++i)
        for (int j = 0; j < g->n2; ++j) {
            int cell = i * g->n2 + j, qa = i + g->h, qb = j + g->h, k = hidx(g, qa, qb);
            double *o = out + (size_t)cell * W;
            double G[2][2];
            inv_metric(g, qa, qb, G);
            o[0] = g->Jgeo[cell]; o[1] = G[0][0]; o[2] = G[0][1]; o[3] = G[1][1];
            o[4] = g->g1x[k]; o[5] = g->g1y[k]; o[6] = g->g2x[k]; o[7] = g->g2y[k];
            for (int al = 0; al < Q; ++al) {
                int c[2] = {g->cx[al], g->cy[al]};
                for (int ii = 0; ii < 2; ++ii) {
                    double sp = 0.0, sm = 0.0;
                    for (int jj = 0; jj < 2; ++jj) {
                        if (c[jj] == 0) continue;
                        sp += c[jj] * Theta(g, ii, jj, qa + c[0], qb + c[1], qa, qb);
                        sm += c[jj] * Theta(g, ii, jj, qa - c[0], qb - c[1], qa, qb);
                    }
                    o[8 + 2 * al + ii] = sp;
                    o[8 + 2 * Q + 2 * al + ii] = sm;
                }
            }
        }
}

/* Streaming map: for every (cell, alpha) the source cell, source direction
 * and crossed wall (0 none, 1 low, 2 high). */
void orc_stream_map(const orc_grid *g, int32_t *src_cell, int32_t *src_dir, int32_t *wall)
{
    for (int i = 0; i < g->n1; ++i)
        for (int j = 0; j < g->n2; ++j)
            for (int al = 0; al < g->q; ++al) {
                int si, sj, beta, w;
                stream_source(g, i, j, al, &si, &sj, &beta, &w);
                size_t k = ((size_t)(i * g->n2 + j)) * g->q + al;
                src_cell[k] = si * g->n2 + sj;
                src_dir[k] = beta;
                wall[k] = w;
            }
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
