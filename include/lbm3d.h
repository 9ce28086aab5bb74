/*
 * lbm3d.h -- C ABI of the three-dimensional curvilinear lattice Boltzmann
 * step (same library as lbm.h).
 *
 * Chekhlov, Staroselsky, Zhang and Chen (arXiv:2301.01868) state the method
 * of Sec. 2 for a 3D mapping x(q): tangents g_i by central differences (Eqs.
 * distance, tangent), the volume J = (g_1 x g_2) . g_3 and the co-tangents
 * g^i (Eqs. metric, covectors), the Christoffel sums of Eq. (gamma), the
 * equilibrium of Eq. (equilibrium) and the corrections of Eqs.
 * (compo-constr), (delta-flux) and (deltaN), summed over i, j, k = 1, 2, 3.
 * This interface runs that step on a 39-velocity lattice with 6th-order
 * isotropy (T0 = 2/3), the solution of the isotropy conditions of App. A
 * written for three dimensions, with the boundaries of App. B on the two q1
 * sides (q2 and q3 periodic).  Populations are FP64 particle numbers
 * N = J f; the force takes the own cell's previous post-collision populations
 * (the paper's one-step lag).
 *
 * Conventions:
 *   - cells (i, j, k), i = 0..n1-1 along q1 (wall-normal, or periodic),
 *     j along q2 and k along q3 (both periodic); host per-cell arrays are
 *     ordered with k fastest, then j, then i (cell = (i n2 + j) n3 + k);
 *     population arrays are direction-major [39][cell];
 *   - the mapping is given on the halo-extended range
 *     (n1 + 2 halo)(n2 + 2 halo)(n3 + 2 halo), k fastest, halo >= 4, ghost
 *     rows beyond a wall holding the symmetrically continued geometry;
 *   - the metric terms must depend on q1 only (planar slabs stretched across
 *     the walls, cylinders around the q3 axis, boxes with uniform cells); other
 *     mappings are rejected with LBM_EINVAL;
 *   - velocities are contravariant (U^1, U^2, U^3);
 *   - return codes and error text as in lbm.h (lbm3d_last_error); host
 *     arrays are caller-owned; calls that return data synchronise the grid's
 *     stream; one grid is not thread safe.
 */
#ifndef LBM3D_H
#define LBM3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm3d_grid lbm3d_grid;

typedef struct {
    int32_t n1, n2, n3;      /* interior cells along q1, q2, q3 */
    int32_t halo;            /* layers of the mapping beyond the interior, >= 4 */
    const double *x, *y, *z; /* host: cell centres on the halo-extended range, k fastest */
    int32_t bc_lo, bc_hi;    /* q1 sides: LBM_NOSLIP (1), LBM_MOVING (2), or LBM_PERIODIC (0) for both */
    double ut_lo[2], ut_hi[2]; /* moving walls: contravariant tangential velocity (U0^2, U0^3) (App. B.3) */
    double tau;              /* BGK relaxation time, > 1/2 */
    double accel[3];         /* constant external acceleration, contravariant */
    double rho0;             /* reference density of the initial state */
    void *stream;            /* hipStream_t for all work on this grid; NULL: the library makes one */
} lbm3d_grid_desc;

/* The lattice (host only): c[39][3] velocity components, w[39], T0. */
int lbm3d_lattice(int32_t *c, double *w, double *T0);

/* Create a grid: FP64 geometry on the GPU (Sec. 2, Eqs. distance..gamma),
 * per-row tables, double-buffered populations.  Errors: LBM_EINVAL (sizes,
 * n1 < 3 with walls, halo < 4, tau <= 1/2, unpaired periodic side, unknown
 * boundary kind, J <= 0 or non-finite geometry, metric terms that depend on
 * q2 or q3, populations beyond 2^31 elements per buffer, or 7 rows i of
 * populations (n2 x 39 x n3 rounded up to 64, FP64) of 4 GiB or more),
 * LBM_ENOMEM, LBM_EDEVICE. */
int lbm3d_grid_create(const lbm3d_grid_desc *desc, lbm3d_grid **out);
void lbm3d_grid_destroy(lbm3d_grid *g);
const char *lbm3d_last_error(const lbm3d_grid *g);

/* Initial state of Sec. 3.1 continued to 3D: N = J f^eq(rho0, U = Ut = u0;
 * g^ij) (Eq. equilibrium), which also serves as the lagged N'(q, -1);
 * u0[cell][3] contravariant, or NULL for rest.  Errors: LBM_EINVAL,
 * LBM_ENOMEM, LBM_EDEVICE. */
int lbm3d_init(lbm3d_grid *g, const double *u0);

/* Advance n steps of Eq. (lbe) (asynchronous on the grid's stream): pull
 * streaming (Eq. adv) with the periodic, bounce-back and moving-wall sources
 * of App. B; moments (Eqs. moments, vcomp); the lagged inertial force of Eq.
 * (compo-constr); Ut = U + J F / (2 m); BGK toward Eq. (equilibrium) (Eq.
 * collide); the corrections of Eqs. (delta-flux) and (deltaN).  Errors:
 * LBM_EINVAL (n < 0), LBM_ESTATE (before lbm3d_init), LBM_EDEVICE. */
int lbm3d_step(lbm3d_grid *g, int64_t n);

/* Moments of the current state as the next step sees them: m[cell]
 * (= J rho, Eq. moments), U[cell][3] (Eq. vcomp), Ut[cell][3] (the physical
 * velocity of Sec. 2); any pointer may be NULL.  Synchronises. */
int lbm3d_moments(lbm3d_grid *g, double *m, double *U, double *Ut);

/* Full FP64 state: P[39][cell] post-collision populations, and the
 * moving-wall side state side[2 walls][3 fields m, Ut^2, Ut^3][3 rows from the
 * wall][n2][n3].  Either pointer may be NULL.  Synchronises. */
int lbm3d_get_state(lbm3d_grid *g, double *P, double *side);
int lbm3d_set_state(lbm3d_grid *g, const double *P, const double *side);

/* Streaming map of the step: source cell, source direction, wall crossed
 * (0 none, 1 low, 2 high) for every cell and direction, [cell][39].
 * Synchronises. */
int lbm3d_stream_map(lbm3d_grid *g, int32_t *src_cell, int32_t *src_dir, int32_t *wall);

/* FP64 geometry per cell: out[cell][1 + 6 + 3*39] = J, g^11, g^12, g^13,
 * g^22, g^23, g^33, then A+^i_a = sum_j c^j_a Theta^i_j(q + c_a, q) for
 * every direction a (Eq. gamma).  Synchronises. */
int lbm3d_geometry(lbm3d_grid *g, double *out);

int lbm3d_synchronize(lbm3d_grid *g);

#ifdef __cplusplus
}
#endif

#endif /* LBM3D_H */
