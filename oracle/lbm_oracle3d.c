/*
 * Plain FP64 CPU oracle for the three-dimensional form of the volumetric
 * curvilinear lattice Boltzmann step (Chekhlov, Staroselsky, Zhang, Chen,
 * arXiv:2301.01868, Sec. 2, which states the method for i = 1, 2, 3).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call this
 * file; only the tests (and the checks that call the tests' helpers) do.  It
 * shares no code, header, table or helper with the HIP library.  Every formula
 * is written in the paper's f-units with literal index sums over {1, 2, 3}, in
 * the order Sec. 2 states them.  Compiled with -O2 -ffp-contract=off and no
 * fast-math.
 *
 * Lattice: 39 velocities with 6th-order moment isotropy, T0 = 2/3, derived
 * from the isotropy and normalisation conditions of App. A written for three
 * dimensions (tests/golden/derive_lattice3d.py solves them in exact rationals;
 * the table below is typed from its output).  Numbering: rest, then shell by
 * shell each vector followed by its opposite.
 *
 * Conventions:
 *   - computational lattice q = (q1, q2, q3), unit spacing; q1 wall-normal (or
 *     periodic), q2 and q3 periodic; interior cells (i, j, k), cell index
 *     (i n2 + j) n3 + k (q3 fastest); populations cell-major P[cell*Q + a];
 *   - the mapping x(q) is given on the halo-extended range (n1+2h)(n2+2h)(n3+2h),
 *     h >= c_max + 1, ghost rows beyond a wall holding the symmetrically
 *     continued geometry.
 *
 * Readings (the same as the 2D oracle's, carried to 3D):
 *   - co-tangents g^1 = (g_2 x g_3)/J, g^2 = (g_3 x g_1)/J, g^3 = (g_1 x g_2)/J
 *     (Eq. covectors, whose double sum over j, k counts each product twice;
 *     g_i . g^j = delta fixes the factor);
 *   - walls on q1: the source beyond a wall is the mirror image of q - c across
 *     the wall plane (same q2, q3); no-slip takes the reversed direction, a
 *     moving wall the direction with c^1 flipped, plus the App. B.3 correction
 *     for both tangential components, 2 w_a m(z) sum_{t=2,3} c^t_a
 *     (U0^t - Ut^t(z)) / T0, with m(z) and Ut(z) of the image cell from its
 *     last collision;
 *   - the external force enters as F_total = F_inertial + rho a_ext;
 *   - the lagged force uses the own cell's previous post-collision value
 *     N'(q, t-1) (the state before streaming); the initial state serves as
 *     N'(q, -1).
 *
 * Pins (tests/test_oracle3d.py): exact isotropy of the lattice and its
 * uniqueness for its shells; the moments of the equilibrium; the reduction to
 * a textbook BGK step on cubic cells; mass conservation and the rest state;
 * the per-cell identities of the correction; the exact planar Couette and
 * Poiseuille profiles and the circular Couette and Poiseuille profiles under
 * refinement.  Parity unpinned (no value in the paper to check against): the
 * first-step lag N'(q, -1) beyond the rest state staying at rest on uniform
 * metrics, and the 3D form of the moving-wall correction beyond the
 * convergence of the Couette flows it drives.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define O3_Q 39

enum { O3_PERIODIC = 0, O3_NOSLIP = 1, O3_MOVING = 2 };

/* the derived lattice: velocity vectors and weights (T0 = 2/3) */
static const int C3[O3_Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, -1}, {1, -1, -1}, {-1, 1, 1},
    {2, 0, 0}, {-2, 0, 0}, {0, 2, 0}, {0, -2, 0}, {0, 0, 2}, {0, 0, -2},
    {2, 2, 0}, {-2, -2, 0}, {2, 0, 2}, {-2, 0, -2}, {2, 0, -2}, {-2, 0, 2}, {2, -2, 0}, {-2, 2, 0},
    {0, 2, 2}, {0, -2, -2}, {0, 2, -2}, {0, -2, 2},
    {3, 0, 0}, {-3, 0, 0}, {0, 3, 0}, {0, -3, 0}, {0, 0, 3}, {0, 0, -3}};
static const double W3[O3_Q] = {
    1.0 / 12.0,
    1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0,
    1.0 / 27.0, 1.0 / 27.0, 1.0 / 27.0, 1.0 / 27.0, 1.0 / 27.0, 1.0 / 27.0, 1.0 / 27.0, 1.0 / 27.0,
    2.0 / 135.0, 2.0 / 135.0, 2.0 / 135.0, 2.0 / 135.0, 2.0 / 135.0, 2.0 / 135.0,
    1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0,
    1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0, 1.0 / 432.0,
    1.0 / 1620.0, 1.0 / 1620.0, 1.0 / 1620.0, 1.0 / 1620.0, 1.0 / 1620.0, 1.0 / 1620.0};
static const double T0_3 = 2.0 / 3.0;

/* direction with the opposite vector, and with the q1 component flipped */
static int find_dir(int x, int y, int z)
{
    for (int a = 0; a < O3_Q; ++a)
        if (C3[a][0] == x && C3[a][1] == y && C3[a][2] == z) return a;
    return -1;
}
static int bounce3(int a) { return find_dir(-C3[a][0], -C3[a][1], -C3[a][2]); }
static int specular3(int a) { return find_dir(-C3[a][0], C3[a][1], C3[a][2]); }

void o3_lattice(int *c, double *w, double *T0)
{
    for (int a = 0; a < O3_Q; ++a) {
        for (int d = 0; d < 3; ++d) c[3 * a + d] = C3[a][d];
        w[a] = W3[a];
    }
    *T0 = T0_3;
}

typedef struct {
    int n1, n2, n3, h, H1, H2, H3;
    int periodic1, bc[2];
    double ut[2][2];      /* [wall][t = q2, q3]: contravariant wall velocity */
    double tau, a_ext[3];
    double *X, *Y, *Z;    /* mapping on the halo range */
    double *gt;           /* tangents g_1, g_2, g_3 on the halo range: [pos][3 vectors][3] */
    double *J;            /* geometric volume of the interior cells */
    double *P, *Pn;       /* post-collision populations [cell][a] */
    double *sm, *su, *smn, *sun;   /* side state: m and Ut (3) of every cell from its last collision */
    long step;
    int iters;
} o3_grid;

static inline long hpos(const o3_grid *g, int a, int b, int c) { return ((long)a * g->H2 + b) * g->H3 + c; }
static inline long cidx(const o3_grid *g, int i, int j, int k) { return ((long)i * g->n2 + j) * g->n3 + k; }

/* Eqs. (distance), (tangent): g_i = [x(q + e_i) - x(q - e_i)] / 2 in lattice units */
static void geometry_init(o3_grid *g)
{
    for (int a = 0; a < g->H1; ++a)
        for (int b = 0; b < g->H2; ++b)
            for (int c = 0; c < g->H3; ++c) {
                double *t = g->gt + hpos(g, a, b, c) * 9;
                if (a == 0 || b == 0 || c == 0 || a == g->H1 - 1 || b == g->H2 - 1 || c == g->H3 - 1) {
                    for (int k = 0; k < 9; ++k) t[k] = NAN;
                    continue;
                }
                const long p[3][2] = {{hpos(g, a + 1, b, c), hpos(g, a - 1, b, c)},
                                      {hpos(g, a, b + 1, c), hpos(g, a, b - 1, c)},
                                      {hpos(g, a, b, c + 1), hpos(g, a, b, c - 1)}};
                const long o = hpos(g, a, b, c);
                for (int i = 0; i < 3; ++i) {
                    double Dp[3] = {g->X[p[i][0]] - g->X[o], g->Y[p[i][0]] - g->Y[o], g->Z[p[i][0]] - g->Z[o]};
                    double Dm[3] = {g->X[p[i][1]] - g->X[o], g->Y[p[i][1]] - g->Y[o], g->Z[p[i][1]] - g->Z[o]};
                    for (int d = 0; d < 3; ++d) t[3 * i + d] = (Dp[d] - Dm[d]) / 2.0;
                }
            }
}

static inline void cross(const double u[3], const double v[3], double w[3])
{
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
}
static inline double dot(const double u[3], const double v[3]) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; }

/* tangent g_m (m = 0, 1, 2) at halo position (a, b, c) */
static inline const double *tangent3(const o3_grid *g, int m, int a, int b, int c)
{
    return g->gt + hpos(g, a, b, c) * 9 + 3 * m;
}

/* Eq. (metric): J = (g_1 x g_2) . g_3 */
static inline double volume3(const o3_grid *g, int a, int b, int c)
{
    double x[3];
    cross(tangent3(g, 0, a, b, c), tangent3(g, 1, a, b, c), x);
    return dot(x, tangent3(g, 2, a, b, c));
}

/* Eq. (covectors): g^m = (g_{m+1} x g_{m+2}) / J, indices cyclic */
static inline void cotangent3(const o3_grid *g, int m, int a, int b, int c, double v[3])
{
    cross(tangent3(g, (m + 1) % 3, a, b, c), tangent3(g, (m + 2) % 3, a, b, c), v);
    double J = volume3(g, a, b, c);
    for (int d = 0; d < 3; ++d) v[d] /= J;
}

/* g^{ij} = g^i . g^j */
static inline void inv_metric3(const o3_grid *g, int a, int b, int c, double G[3][3])
{
    double co[3][3];
    for (int m = 0; m < 3; ++m) cotangent3(g, m, a, b, c, co[m]);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) G[i][j] = dot(co[i], co[j]);
}

/* Eq. (gamma): Theta^i_j(p, q) = [g_j(p) - g_j(q)] . g^i(q) */
static inline double Theta3(const o3_grid *g, int i, int j, const int p[3], const int q[3])
{
    const double *gp = tangent3(g, j, p[0], p[1], p[2]);
    const double *gq = tangent3(g, j, q[0], q[1], q[2]);
    double co[3], d[3];
    cotangent3(g, i, q[0], q[1], q[2], co);
    for (int k = 0; k < 3; ++k) d[k] = gp[k] - gq[k];
    return dot(d, co);
}

/* Eq. (equilibrium), literal index sums over i, j, k in {1, 2, 3} */
static void feq3(double rho, const double U[3], const double Ut[3], double G[3][3], double *feq)
{
    const double T0 = T0_3;
    for (int a = 0; a < O3_Q; ++a) {
        double c[3] = {(double)C3[a][0], (double)C3[a][1], (double)C3[a][2]};
        double s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int i = 0; i < 3; ++i) s1 += c[i] * U[i] / T0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double dij = (i == j) ? 1.0 : 0.0;
                s2 += (c[i] * c[j] / T0 - dij) * ((G[i][j] - dij) * T0 + Ut[i] * Ut[j]);
            }
        s2 /= 2.0 * T0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < 3; ++k) {
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
        feq[a] = rho * W3[a] * (1.0 + s1 + s2 + s3);
    }
}

void o3_feq(double rho, const double *U, const double *Ut, const double *G6, double *out)
{
    double G[3][3] = {{G6[0], G6[1], G6[2]}, {G6[1], G6[3], G6[4]}, {G6[2], G6[4], G6[5]}};
    feq3(rho, U, Ut, G, out);
}

/* Streaming source (Eq. adv, App. B): source cell, source direction, wall
 * crossed (0 none, 1 low, 2 high) for target (i, j, k) and direction a. */
static void source3(const o3_grid *g, int i, int j, int k, int a, int *si, int *sj, int *sk, int *beta, int *wall)
{
    int ti = i - C3[a][0], tj = j - C3[a][1], tk = k - C3[a][2];
    *sj = ((tj % g->n2) + g->n2) % g->n2;
    *sk = ((tk % g->n3) + g->n3) % g->n3;
    *beta = a;
    *wall = 0;
    if (ti >= 0 && ti < g->n1) { *si = ti; return; }
    if (g->periodic1) { *si = ((ti % g->n1) + g->n1) % g->n1; return; }
    int side = ti < 0 ? 0 : 1;
    *si = side == 0 ? -1 - ti : 2 * g->n1 - 1 - ti;
    *beta = g->bc[side] == O3_NOSLIP ? bounce3(a) : specular3(a);
    *wall = side + 1;
}

static double pulled3(const o3_grid *g, const double *P, const double *sm, const double *su, int i, int j, int k, int a)
{
    int si, sj, sk, beta, wall;
    source3(g, i, j, k, a, &si, &sj, &sk, &beta, &wall);
    long s = cidx(g, si, sj, sk);
    double v = P[s * O3_Q + beta];
    if (wall && g->bc[wall - 1] == O3_MOVING) {
        /* App. B.3 correction, both tangential components (q2, q3) */
        for (int t = 1; t < 3; ++t)
            v += 2.0 * W3[a] * sm[s] * (double)C3[a][t] * (g->ut[wall - 1][t - 1] - su[s * 3 + t]) / T0_3;
    }
    return v;
}

typedef struct {
    double N[O3_Q], m, rho, U[3], F[3], Ut[3];
} o3_diag;

/* Per-cell update of interior cell (i, j, k): N' into out[Q]. */
static void cell3(const o3_grid *g, const double *P, const double *sm, const double *su, int i, int j, int k,
                  double *out, o3_diag *dg, int moments_only)
{
    const double T0 = T0_3;
    const int q[3] = {i + g->h, j + g->h, k + g->h};
    const long cell = cidx(g, i, j, k);
    const double J = g->J[cell];
    double N[O3_Q], f[O3_Q], feq[O3_Q], Nown[O3_Q];
    for (int a = 0; a < O3_Q; ++a) N[a] = pulled3(g, P, sm, su, i, j, k, a);
    /* Eqs. (dist), (moments), (vcomp) */
    double rho = 0.0, rU[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < O3_Q; ++a) {
        f[a] = N[a] / J;
        rho += f[a];
        for (int d = 0; d < 3; ++d) rU[d] += C3[a][d] * f[a];
    }
    double U[3] = {rU[0] / rho, rU[1] / rho, rU[2] / rho};
    for (int a = 0; a < O3_Q; ++a) Nown[a] = P[cell * O3_Q + a];
    double F[3], Ut[3], G[3][3], dPi[3][3];
    inv_metric3(g, q[0], q[1], q[2], G);
    for (int it = 0; it <= (moments_only ? 0 : g->iters); ++it) {
        /* Eq. (compo-constr), the lagged N'(q, t-1) in the first pass */
        for (int ii = 0; ii < 3; ++ii) {
            double s = 0.0;
            for (int a = 0; a < O3_Q; ++a) {
                const int pp[3] = {q[0] + C3[a][0], q[1] + C3[a][1], q[2] + C3[a][2]};
                const int pm[3] = {q[0] - C3[a][0], q[1] - C3[a][1], q[2] - C3[a][2]};
                for (int jj = 0; jj < 3; ++jj) {
                    if (C3[a][jj] == 0) continue;
                    s += C3[a][jj] * (Theta3(g, ii, jj, pp, q) * Nown[a] - Theta3(g, ii, jj, pm, q) * N[a]);
                }
            }
            F[ii] = -s / (2.0 * J) + rho * g->a_ext[ii];
        }
        for (int d = 0; d < 3; ++d) Ut[d] = U[d] + 0.5 * F[d] / rho;
        feq3(rho, U, Ut, G, feq);
        if (dg) {
            for (int a = 0; a < O3_Q; ++a) dg->N[a] = N[a];
            dg->m = rho * J;
            dg->rho = rho;
            for (int d = 0; d < 3; ++d) { dg->U[d] = U[d]; dg->F[d] = F[d]; dg->Ut[d] = Ut[d]; }
        }
        if (moments_only) return;
        /* Eq. (delta-flux) */
        const double pre = -0.5 * (1.0 - 1.0 / (2.0 * g->tau));
        for (int ii = 0; ii < 3; ++ii)
            for (int jj = 0; jj < 3; ++jj) {
                double s = 0.0;
                for (int a = 0; a < O3_Q; ++a) {
                    const int pp[3] = {q[0] + C3[a][0], q[1] + C3[a][1], q[2] + C3[a][2]};
                    const int pm[3] = {q[0] - C3[a][0], q[1] - C3[a][1], q[2] - C3[a][2]};
                    for (int kk = 0; kk < 3; ++kk) {
                        double ck = (double)(C3[a][ii] * C3[a][kk]);
                        if (ck == 0.0) continue;
                        s += ck * (Theta3(g, jj, kk, pp, q) - Theta3(g, jj, kk, pm, q)) * feq[a];
                    }
                }
                dPi[ii][jj] = pre * s;
            }
        /* Eqs. (deltaN), (collide), (lbe) */
        for (int a = 0; a < O3_Q; ++a) {
            double c[3] = {(double)C3[a][0], (double)C3[a][1], (double)C3[a][2]};
            double t1 = 0.0, t2 = 0.0;
            for (int jj = 0; jj < 3; ++jj) t1 += c[jj] * F[jj] / T0;
            for (int jj = 0; jj < 3; ++jj)
                for (int kk = 0; kk < 3; ++kk) t2 += (c[jj] * c[kk] / T0 - (jj == kk ? 1.0 : 0.0)) * dPi[jj][kk] / T0;
            double dN = W3[a] * J * (t1 + t2);
            double Om = -J * (f[a] - feq[a]) / g->tau;
            out[a] = N[a] + Om + dN;
        }
        /* optional fixed-point passes of the implicit force relation */
        for (int a = 0; a < O3_Q; ++a) Nown[a] = out[a];
    }
}

o3_grid *o3_create(int n1, int n2, int n3, int h, const double *X, const double *Y, const double *Z, int periodic1,
                   int bc_lo, int bc_hi, const double *ut_lo, const double *ut_hi, double tau, const double *a)
{
    if (h < 4 || n1 < 1 || n2 < 1 || n3 < 1 || !(tau > 0.5)) return NULL;
    if (!periodic1 && n1 < 3) return NULL;
    o3_grid *g = (o3_grid *)calloc(1, sizeof(o3_grid));
    g->n1 = n1; g->n2 = n2; g->n3 = n3; g->h = h;
    g->H1 = n1 + 2 * h; g->H2 = n2 + 2 * h; g->H3 = n3 + 2 * h;
    g->periodic1 = periodic1;
    g->bc[0] = periodic1 ? O3_PERIODIC : bc_lo;
    g->bc[1] = periodic1 ? O3_PERIODIC : bc_hi;
    for (int t = 0; t < 2; ++t) { g->ut[0][t] = ut_lo[t]; g->ut[1][t] = ut_hi[t]; }
    g->tau = tau;
    for (int d = 0; d < 3; ++d) g->a_ext[d] = a[d];
    size_t nh = (size_t)g->H1 * g->H2 * g->H3, nc = (size_t)n1 * n2 * n3;
    g->X = (double *)malloc(nh * sizeof(double));
    g->Y = (double *)malloc(nh * sizeof(double));
    g->Z = (double *)malloc(nh * sizeof(double));
    memcpy(g->X, X, nh * sizeof(double));
    memcpy(g->Y, Y, nh * sizeof(double));
    memcpy(g->Z, Z, nh * sizeof(double));
    g->gt = (double *)malloc(nh * 9 * sizeof(double));
    g->J = (double *)malloc(nc * sizeof(double));
    g->P = (double *)calloc(nc * O3_Q, sizeof(double));
    g->Pn = (double *)calloc(nc * O3_Q, sizeof(double));
    g->sm = (double *)calloc(nc, sizeof(double));
    g->smn = (double *)calloc(nc, sizeof(double));
    g->su = (double *)calloc(nc * 3, sizeof(double));
    g->sun = (double *)calloc(nc * 3, sizeof(double));
    geometry_init(g);
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j)
            for (int k = 0; k < n3; ++k) g->J[cidx(g, i, j, k)] = volume3(g, i + h, j + h, k + h);
    return g;
}

void o3_destroy(o3_grid *g)
{
    if (!g) return;
    free(g->X); free(g->Y); free(g->Z); free(g->gt); free(g->J);
    free(g->P); free(g->Pn); free(g->sm); free(g->smn); free(g->su); free(g->sun);
    free(g);
}

void o3_set_iterations(o3_grid *g, int k) { g->iters = k; }

/* initial state N = J f^eq(rho0, U = Ut = u0; g^ij); side state m = J rho0, Ut = u0 */
void o3_init(o3_grid *g, double rho0, const double *u0)
{
    for (int i = 0; i < g->n1; ++i)
        for (int j = 0; j < g->n2; ++j)
            for (int k = 0; k < g->n3; ++k) {
                long c = cidx(g, i, j, k);
                double U[3] = {0.0, 0.0, 0.0};
                if (u0) for (int d = 0; d < 3; ++d) U[d] = u0[c * 3 + d];
                double G[3][3], feq[O3_Q];
                inv_metric3(g, i + g->h, j + g->h, k + g->h, G);
                feq3(rho0, U, U, G, feq);
                for (int a = 0; a < O3_Q; ++a) g->P[c * O3_Q + a] = g->J[c] * feq[a];
                g->sm[c] = g->J[c] * rho0;
                for (int d = 0; d < 3; ++d) g->su[c * 3 + d] = U[d];
            }
    g->step = 0;
}

void o3_step(o3_grid *g, long n, int threads)
{
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    for (long s = 0; s < n; ++s) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i < g->n1; ++i)
            for (int j = 0; j < g->n2; ++j)
                for (int k = 0; k < g->n3; ++k) {
                    long c = cidx(g, i, j, k);
                    o3_diag dg;
                    cell3(g, g->P, g->sm, g->su, i, j, k, g->Pn + c * O3_Q, &dg, 0);
                    g->smn[c] = dg.m;
                    for (int d = 0; d < 3; ++d) g->sun[c * 3 + d] = dg.Ut[d];
                }
        double *t = g->P; g->P = g->Pn; g->Pn = t;
        t = g->sm; g->sm = g->smn; g->smn = t;
        t = g->su; g->su = g->sun; g->sun = t;
        g->step++;
    }
}

long o3_get_step(const o3_grid *g) { return g->step; }

void o3_get_state(const o3_grid *g, double *P)
{
    memcpy(P, g->P, (size_t)g->n1 * g->n2 * g->n3 * O3_Q * sizeof(double));
}
void o3_set_state(o3_grid *g, const double *P)
{
    memcpy(g->P, P, (size_t)g->n1 * g->n2 * g->n3 * O3_Q * sizeof(double));
}
void o3_get_side(const o3_grid *g, double *m, double *u)
{
    size_t nc = (size_t)g->n1 * g->n2 * g->n3;
    memcpy(m, g->sm, nc * sizeof(double));
    memcpy(u, g->su, nc * 3 * sizeof(double));
}
void o3_set_side(o3_grid *g, const double *m, const double *u)
{
    size_t nc = (size_t)g->n1 * g->n2 * g->n3;
    memcpy(g->sm, m, nc * sizeof(double));
    memcpy(g->su, u, nc * 3 * sizeof(double));
}

/* moments the next step would see: m, U (3), Ut (3) per cell */
void o3_moments(const o3_grid *g, double *m, double *U, double *Ut)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < g->n1; ++i)
        for (int j = 0; j < g->n2; ++j)
            for (int k = 0; k < g->n3; ++k) {
                long c = cidx(g, i, j, k);
                o3_diag dg;
                double out[O3_Q];
                cell3(g, g->P, g->sm, g->su, i, j, k, out, &dg, 1);
                m[c] = dg.m;
                for (int d = 0; d < 3; ++d) { U[c * 3 + d] = dg.U[d]; Ut[c * 3 + d] = dg.Ut[d]; }
            }
}

/* one step of the listed cells from the current state (no state change) */
void o3_step_cells(const o3_grid *g, int n, const int *cells, double *out)
{
#pragma omp parallel for schedule(static)
    for (int t = 0; t < n; ++t) {
        long c = cells[t];
        int k = (int)(c % g->n3), j = (int)((c / g->n3) % g->n2), i = (int)(c / ((long)g->n2 * g->n3));
        cell3(g, g->P, g->sm, g->su, i, j, k, out + (size_t)t * O3_Q, NULL, 0);
    }
}

/* per cell: J, g^ij (6: 11 12 13 22 23 33), tangents (9), A+^i_a (3 Q) with
 * A+^i_a = sum_j c^j_a Theta^i_j(q + c_a, q) */
void o3_geometry(const o3_grid *g, double *out)
{
    const int W = 1 + 6 + 9 + 3 * O3_Q;
    for (int i = 0; i < g->n1; ++i)
        for (int j = 0; j < g->n2; ++j)
            for (int k = 0; k < g->n3; ++k) {
                long c = cidx(g, i, j, k);
                const int q[3] = {i + g->h, j + g->h, k + g->h};
                double *o = out + c * W;
                double G[3][3];
                inv_metric3(g, q[0], q[1], q[2], G);
                o[0] = g->J[c];
                o[1] = G[0][0]; o[2] = G[0][1]; o[3] = G[0][2]; o[4] = G[1][1]; o[5] = G[1][2]; o[6] = G[2][2];
                for (int m = 0; m < 3; ++m)
                    for (int d = 0; d < 3; ++d) o[7 + 3 * m + d] = tangent3(g, m, q[0], q[1], q[2])[d];
                for (int a = 0; a < O3_Q; ++a) {
                    const int pp[3] = {q[0] + C3[a][0], q[1] + C3[a][1], q[2] + C3[a][2]};
                    for (int ii = 0; ii < 3; ++ii) {
                        double s = 0.0;
                        for (int jj = 0; jj < 3; ++jj)
                            if (C3[a][jj]) s += C3[a][jj] * Theta3(g, ii, jj, pp, q);
                        o[16 + 3 * a + ii] = s;
                    }
                }
            }
}

void o3_stream_map(const o3_grid *g, int *src_cell, int *src_dir, int *wall)
{
    for (int i = 0; i < g->n1; ++i)
        for (int j = 0; j < g->n2; ++j)
            for (int k = 0; k < g->n3; ++k)
                for (int a = 0; a < O3_Q; ++a) {
                    int si, sj, sk, b, w;
                    source3(g, i, j, k, a, &si, &sj, &sk, &b, &w);
                    long t = cidx(g, i, j, k) * O3_Q + a;
                    src_cell[t] = (int)cidx(g, si, sj, sk);
                    src_dir[t] = b;
                    wall[t] = w;
                }
}
