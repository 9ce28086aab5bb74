/*
 * lbm.h -- C ABI of the MI355X volumetric curvilinear lattice Boltzmann library.
 *
 * The library advances the lattice Boltzmann equation of Chekhlov,
 * Staroselsky, Zhang and Chen (arXiv:2301.01868, Sec. 2) on a body-fitted 2D
 * grid: pull streaming in computational coordinates (Eq. adv), BGK collision
 * toward the metric-dependent equilibrium (Eqs. collide, equilibrium), the
 * inertial force from the discrete Christoffel symbols (Eqs. gamma,
 * compo-constr), the momentum-flux correction (Eq. delta-flux) and the
 * curvilinear correction (Eq. deltaN), with the periodic, no-slip and
 * moving-wall boundaries of App. B and the "no flow" volume adjustment of
 * Sec. 3.1.  D2Q9 and D2Q21 lattices (App. A).
 *
 * Conventions used by every entry point:
 *   - q1 is the wall-normal computational index (rows i = 0..n1-1, walls at
 *     i = -1/2 and n1 - 1/2), q2 the periodic index (columns j = 0..n2-1);
 *   - all host arrays are row-major with q2 fastest; per-cell vectors are
 *     cell-major ([cell][2]); population arrays are direction-major
 *     ([alpha][i][j]); lengths are in lattice units (mean wall-normal step 1,
 *     time step 1);
 *   - velocities are contravariant components U^i in the tangent basis g_i;
 *   - every call returns LBM_OK (0) or a negative LBM_E* code; the text of the
 *     last error is lbm_last_error(grid) (or lbm_last_error(NULL) for errors
 *     raised before a grid exists);
 *   - host arrays passed in are owned by the caller and copied; output arrays
 *     are allocated by the caller with the stated sizes;
 *   - each grid is bound to one HIP stream; calls on one grid are not thread
 *     safe; calls that return data to the host synchronise that stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* bad argument: shape, tau <= 1/2, J <= 0, halo too small, ... */
    LBM_ENOMEM = -2,     /* device or host allocation failed */
    LBM_EDEVICE = -3,    /* a HIP runtime call failed */
    LBM_EUNSTABLE = -4,  /* a reduction found non-finite values or m <= 0 */
    LBM_ESTATE = -5      /* call out of order (e.g. step before init) */
};

/* boundary kinds of the two q1 sides (App. B); q2 is always periodic */
enum { LBM_PERIODIC = 0, LBM_NOSLIP = 1, LBM_MOVING = 2 };

/* population storage / arithmetic */
enum {
    LBM_FP64 = 0,   /* FP64 populations, FP64 arithmetic */
    LBM_FP32 = 1,   /* FP32 populations stored as offsets from a per-cell base, FP32 arithmetic */
    LBM_FP16 = 2    /* FP16 offsets divided by the direction's lattice weight (per-plane scaling),
                       FP32 arithmetic; the error against FP64 is the caller's to measure */
};

/* offset base for LBM_FP32 storage: the stored value is N_alpha - B_alpha */
enum {
    LBM_BASE_LOCAL_REST = 0, /* B = J rho0 f^eq_alpha(rho0, U = 0; g^ij) / rho0 (default) */
    LBM_BASE_W_RHO0 = 1,     /* B = J w_alpha rho0 */
    LBM_BASE_NONE = 2        /* B = 0 (always used for LBM_FP64) */
};

/* geometry table mode (Sec. 2: the metric terms of the step, Eqs. metric,
 * covectors and gamma, per row of the grid or per cell) */
enum {
    LBM_GEOM_AUTO = 0,       /* per-row tables when the metric terms do not depend on q2,
                                else as LBM_GEOM_CELL */
    LBM_GEOM_CELL = 1,       /* per cell, rebuilt in the step from the geometry of the cell and
                                its neighbours (staged in LDS: FP64 values for LBM_FP64, FP32
                                deviations from a reference cell of the tile for offset storage;
                                32 or 64 B per cell in HBM); offset storage with a base other
                                than LBM_BASE_LOCAL_REST reads the stored table instead
                                (table_kind 1) */
    LBM_GEOM_CELL_TABLE = 2  /* per cell, read from a stored table of every term (4Q + 3 values
                                and more per cell) */
};

typedef struct lbm_grid lbm_grid;
typedef struct lbm_batch lbm_batch;

/* Device memory provider (e.g. PyTorch's caching allocator); NULL = hipMalloc. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} lbm_allocator;

typedef struct {
    int32_t q;              /* 9 or 21 */
    int32_t n1, n2;         /* interior cells along q1 and q2 */
    int32_t halo;           /* layers of the mapping given beyond the interior, >= c_max + 1 (2 or 4) */
    const double *x, *y;    /* host: cell-centre coordinates on the halo-extended range,
                               (n1 + 2 halo) x (n2 + 2 halo), q2 fastest; ghost rows beyond a wall
                               hold the symmetrically continued geometry (Sec. 3.1) */
    int32_t bc_lo, bc_hi;   /* q1 low / high side: LBM_NOSLIP, LBM_MOVING, or LBM_PERIODIC for both */
    double ut_lo, ut_hi;    /* moving walls: contravariant tangential velocity U0^2 (App. B.3) */
    double tau;             /* BGK relaxation time, > 1/2 */
    double accel[2];        /* constant external acceleration, contravariant components */
    double rho0;            /* reference density (initial state and offset base) */
    int32_t precision;      /* LBM_FP64 | LBM_FP32 | LBM_FP16 */
    int32_t offset_base;    /* LBM_BASE_* (ignored for LBM_FP64) */
    int32_t iterations;     /* 0: force with the lagged N'(q, t-1) (Sec. 2); k > 0: k extra
                               fixed-point passes of the implicit force relation */
    int32_t geometry;       /* LBM_GEOM_AUTO | LBM_GEOM_CELL | LBM_GEOM_CELL_TABLE */
    const lbm_allocator *alloc; /* NULL: hipMalloc/hipFree */
    void *stream;           /* hipStream_t for all work on this grid; NULL: the library makes one */
} lbm_grid_desc;

/* Residual and global diagnostics (all FP64, interior cells).  residual is
 * |m Ut(t) - m Ut(t-K)|_2 / (K |m Ut(t)|_2) with K the steps since the last
 * call (infinite on the first call); mass = sum m; kinetic_energy =
 * sum m g_ij Ut^i Ut^j / 2; angular_momentum = sum m (x u_y - y u_x) with
 * u = Ut^i g_i; bad_cells counts cells with non-finite values or m <= 0. */
typedef struct {
    int64_t step;
    double residual;
    double mass;
    double mass_rel_drift;  /* relative to the mass at lbm_init */
    double kinetic_energy;
    double angular_momentum;
    int64_t bad_cells;
} lbm_resid;

typedef struct {
    int32_t q, n1, n2, pitch;
    int32_t precision, row_tables; /* row_tables = 1 when per-row geometry tables are used */
    int64_t step;
    double bytes_per_update;       /* algorithmic HBM bytes per lattice update: 2 Q sizeof(population) */
    size_t device_bytes;           /* device memory held by the grid */
    int32_t waves_per_block;       /* step launch: waves (rows of 64 cells) per workgroup */
    int32_t waves_per_cu_cap;      /* step launch: resident waves per CU cap, 0 = none */
    int32_t table_kind;            /* 0 per-row tables, 1 per-cell tables, 2 per-cell terms
                                      rebuilt from the geometry in the step */
    int32_t reserved;
} lbm_grid_info;

/* Lattice tables of App. A / App. B (host only): velocities cx[q], cy[q],
 * weights w[q], T0.  Returns LBM_EINVAL for q other than 9 or 21. */
int lbm_lattice(int32_t q, int32_t *cx, int32_t *cy, double *w, double *T0);

/* Mapping helpers (host only): the halo-extended cell centres x, y
 * [(n1 + 2 halo)(n2 + 2 halo)], q2 fastest, that lbm_grid_create takes, for
 * the paper's two grid families.  Rows run along q1 (wall-normal), defined by
 * the n1 + 1 strictly increasing face positions faces[0..n1] (lattice units:
 * uniform, the linear contraction of App. C, geometric stretching ...); cell
 * centres are the face midpoints.  The halo rows beyond each wall hold the
 * symmetrically continued geometry of Sec. 3.1: row 1 - k is the mirror image
 * of row k across the low wall (faces[0]) and row n1 + k that of row
 * n1 + 1 - k across the high wall (faces[n1]), repeated when halo > n1.  The
 * periodic q2 direction continues the mapping.  halo: 1..64.  Errors:
 * LBM_EINVAL (null pointer, sizes, faces not finite or not increasing, and the
 * family's own conditions below), with the text in lbm_last_error(NULL).
 *
 * lbm_map_planar: planar channel (Sec. 3.1, App. C); x = the wall-normal
 * position, y = (j + 1/2) d_per for columns j = -halo .. n2 + halo - 1;
 * d_per > 0.
 *
 * lbm_map_polar: annulus on the half-spaced polar lattice of App. D; faces
 * are radii, theta_j = (j + 1/2) 2 pi / ntheta, x = r cos theta,
 * y = r sin theta.  n2 <= ntheta columns are kept (n2 < ntheta: a theta
 * reduction, exact for theta-invariant states); every ring, ghosts included,
 * must have r > 0. */
int lbm_map_planar(int32_t n1, int32_t n2, int32_t halo, const double *faces, double d_per, double *x, double *y);
int lbm_map_polar(int32_t n1, int32_t n2, int32_t halo, const double *r_faces, int32_t ntheta, double *x, double *y);

/* Create a grid from a coordinate mapping (Sec. 2, Eqs. distance..gamma).
 * Computes the geometry (tangent basis by central differences, metric,
 * volume J, co-tangents, discrete Christoffel sums) in FP64 on the GPU, builds
 * the step tables and allocates the double-buffered populations.  Errors:
 * LBM_EINVAL (q, sizes: n1 n2 > 2^30 cells, n1 + 2 halo > 65535 or rows
 * so long that 2 c_max + 1 rows of populations reach 4 GiB; halo < c_max + 1,
 * n1 < c_max with
 * walls, tau <= 1/2, J <= 0 anywhere, unpaired periodic side, unknown
 * precision, offset base, geometry mode or boundary kind), LBM_ENOMEM,
 * LBM_EDEVICE.
 *
 * Walls sit on the two q1 sides only, as in App. B (whose reflection rules
 * are stated for walls normal to q1 with q2 periodic); a problem with walls
 * across q2 is posed by naming its wall-normal axis q1 in the mapping. */
int lbm_grid_create(const lbm_grid_desc *desc, lbm_grid **out);
void lbm_grid_destroy(lbm_grid *g);
const char *lbm_last_error(const lbm_grid *g);
int lbm_grid_info_get(const lbm_grid *g, lbm_grid_info *out);

/* Volume used for the initial state and the reported density: NULL restores
 * the geometric J; otherwise J[n1*n2] > 0 (the "no flow" adjusted J', Sec. 3.1).
 * The step itself does not depend on J (everything is in particle numbers). */
int lbm_set_volume(lbm_grid *g, const double *J);

/* Volume currently used for initial state and density output, J[n1*n2]. */
int lbm_get_volume(lbm_grid *g, double *J);

/* Initial state of Sec. 3.1 (uniform density rho0, fluid at rest or at u0):
 * N = J f^eq(rho0, U = Ut = u0; g^ij) with the equilibrium of Eq.
 * (equilibrium), J the grid's current volume (geometric, or J' after the
 * no-flow adjustment).  The same state serves as the lagged N'(q, -1) that
 * the force of the first step reads (Eq. compo-constr takes the own cell's
 * previous post-collision populations; before the first step there are none,
 * and the initial state is used: a reading, since the paper does not say).
 * u0[n1*n2][2] contravariant, or NULL for rest.  Resets the step counter and
 * the residual reference.  Errors: LBM_EINVAL (null grid), LBM_ENOMEM,
 * LBM_EDEVICE. */
int lbm_init(lbm_grid *g, const double *u0);

/* Advance n time steps (asynchronous on the grid's stream).  One step is
 * the lattice Boltzmann equation of Eq. (lbe): pull streaming in
 * computational coordinates (Eq. adv) with the periodic, bounce-back and
 * moving-wall sources of App. B.1-B.3; moments (Eqs. moments, vcomp); the
 * inertial force of Eq. (compo-constr) from the Christoffel sums of Eq.
 * (gamma), with the own cell's previous post-collision populations (the
 * one-step lag the paper adopts) or `iterations` fixed-point passes of the
 * implicit relation; the physical velocity Ut = U + J F / (2 m); BGK
 * relaxation toward the equilibrium of Eq. (equilibrium) (Eq. collide); the
 * momentum-flux correction of Eq. (delta-flux) and the correction term of
 * Eq. (deltaN).  Errors: LBM_EINVAL (null grid, n < 0), LBM_ESTATE (before
 * lbm_init), LBM_EDEVICE (launch or graph failure). */
int lbm_step(lbm_grid *g, int64_t n);

/* Moments of the current state, computed as the next step would see them
 * (pull, moments, force): m[n1*n2] = sum_alpha N_alpha (= J rho, Eq.
 * moments), U[n1*n2][2] = sum_alpha c_alpha N_alpha / m (Eqs. velocity,
 * vcomp) and the physical velocity Ut = U + J F / (2 m) of Sec. 2, both as
 * contravariant components (Eq. result maps them to Cartesian ones with the
 * tangents g_i; lbm_physical_velocity does that).  Any pointer may be NULL.
 * Synchronises.  Errors: LBM_EINVAL, LBM_ESTATE (before lbm_init),
 * LBM_EDEVICE. */
int lbm_moments(lbm_grid *g, double *m, double *U, double *Ut);

/* FP64 residual and diagnostics (see lbm_resid).  Sec. 3.1 runs every flow
 * to steady state and judges it by the kinetic energy and the conservation
 * of mass and angular momentum; the paper defines no residual, so
 * lbm_resid.residual is this library's reading: the relative change of the
 * momentum m Ut per step since the previous call.  Synchronises.  Returns
 * LBM_EUNSTABLE (after filling *out) when bad_cells > 0; LBM_EINVAL,
 * LBM_ESTATE (before lbm_init), LBM_EDEVICE. */
int lbm_residual(lbm_grid *g, lbm_resid *out);

/* The "no flow" adjustment of Sec. 3.1: from rest, with the grid's boundary
 * kinds but zero wall velocities and zero external force, run to
 * residual < tol (checked every check_every steps, at most max_steps), then
 * set J' = m / rho0 per cell as the grid's volume.  Leaves the grid needing
 * lbm_init.  *steps_out (may be NULL) receives the steps taken. */
int lbm_noflow_adjust(lbm_grid *g, double tol, int64_t max_steps, int32_t check_every, int64_t *steps_out);

/* Full state as FP64 particle numbers: P[q][n1][n2] (absolute N'_alpha, base
 * added back) and the moving-wall side state side[2][2][c_max][n2]
 * (wall low/high, field m / Ut^2, distance from the wall, column).  Either
 * pointer may be NULL.  Synchronises. */
int lbm_get_state(lbm_grid *g, double *P, double *side);
int lbm_set_state(lbm_grid *g, const double *P, const double *side);

/* lbm_get_state without allocating: for callers that cannot allocate device
 * memory (serving loops that checkpoint resident solves, harnesses that
 * forbid allocation after set-up).  Same outputs as lbm_get_state, bitwise.
 * The FP64 state is staged through a fixed device array of
 * LBM_NOALLOC_STAGING_BYTES that each GPU the library runs on holds until the
 * process ends, in chunks of whole rows, and copied to the caller's host
 * arrays; no device or host memory is allocated by the library.  Errors:
 * LBM_EINVAL (null grid; one row of the state, q * n2 * 8 bytes, or the side
 * state, 4 * c_max * n2 * 8 bytes, larger than the staging array),
 * LBM_EDEVICE.  The staging array is shared by every call on a GPU: the
 * library serialises calls made from the threads of one process; it keeps
 * the last call's contents, which no call reads before writing them.
 * Synchronises the grid's stream. */
#define LBM_NOALLOC_STAGING_BYTES ((size_t)8 << 20)
int lbm_get_state_noalloc(lbm_grid *g, double *P, double *side);

/* Checkpoint blob (host memory, owned by the caller): a header (lattice,
 * shape, storage precision of the writer, step count) followed by the FP64
 * state of lbm_get_state.  lbm_save with buf = NULL stores the required size
 * in *len; otherwise *len must be at least that size (LBM_EINVAL) and
 * receives the bytes written.  lbm_load restores the state into a grid of the
 * same lattice and shape (LBM_EINVAL otherwise), in any storage precision,
 * and resets the step count; the grid must have been created (not
 * necessarily initialised).  Both synchronise. */
int lbm_save(lbm_grid *g, void *buf, size_t *len);
int lbm_load(lbm_grid *g, const void *buf, size_t len);

/* Physical velocity Ut^i g_i per cell (Sec. 2; the velocity the paper's
 * profiles show): u[n1*n2][2] = (x, y) components, FP64, from the same
 * moments as lbm_moments.  Synchronises. */
int lbm_physical_velocity(lbm_grid *g, double *u);

/* Streaming map actually used by the step kernel: for every cell and
 * direction, the source cell (i*n2 + j), source direction and crossed wall
 * (0 none, 1 low, 2 high).  Arrays [n1*n2][q].  Synchronises. */
int lbm_stream_map(lbm_grid *g, int32_t *src_cell, int32_t *src_dir, int32_t *wall);

/* FP64 geometry precompute per cell: out[n1*n2][4 + 2q] = J, g^11, g^12,
 * g^22, then for every alpha (A+^1, A+^2) with
 * A+^i_alpha = sum_j c^j_alpha Theta^i_j(q + c_alpha, q).  Synchronises. */
int lbm_geometry(lbm_grid *g, double *out);

int lbm_synchronize(lbm_grid *g);
void *lbm_stream(lbm_grid *g);

/* Move all later work of grid g to `stream` (a hipStream_t of the grid's
 * device; NULL: a stream the library makes and owns).  Work already queued on
 * the old stream stays ordered before it (an event wait; a stream the library
 * owned is then destroyed, which waits for that work).  Lets a caller create
 * and initialise a grid on a setup stream while other work runs, then hand it
 * to the stream its batch runs on.  LBM_ESTATE while a batch holds the grid. */
int lbm_grid_set_stream(lbm_grid *g, void *stream);

/* Many grids advanced together: one launch per group of grids sharing lattice,
 * precision, table kind and force mode (lagged, or fixed-point passes) per step
 * over a flattened table of row tiles; steps of a batch are captured in HIP
 * graphs and run on the stream of grids[0] (grids on other streams are joined
 * with events before and after).  Every grid must be initialised
 * (LBM_ESTATE otherwise) and appear once (LBM_EINVAL otherwise); n > 0.
 * The batch does not own the grids: destroy the batch before its grids.  A
 * grid destroyed while a batch still holds it leaves that batch broken: the
 * batch drops its references to the grid and its stream, lbm_batch_step,
 * lbm_batch_step_group, lbm_batch_residuals and lbm_batch_autotune return
 * LBM_ESTATE, and lbm_batch_destroy only releases it.
 * While it is in a batch a grid must only be stepped through the batch. */
int lbm_batch_create(lbm_grid *const *grids, int32_t n, lbm_batch **out);

/* lbm_batch_create with options.  LBM_BATCH_FUSE_LATTICES puts D2Q9 and D2Q21
 * grids of one precision, table kind and force mode into a single launch per
 * step (each workgroup runs its tile's lattice): half the kernel launches of a
 * mixed batch, which shortens the steps of small, launch-bound batches (the
 * serving loop), at some cost in throughput on large ones, since both
 * lattices then run with the larger kernel's register allocation.  Other
 * flag bits: LBM_EINVAL. */
enum { LBM_BATCH_FUSE_LATTICES = 1 };
int lbm_batch_create_ex(lbm_grid *const *grids, int32_t n, uint32_t flags, lbm_batch **out);
int lbm_batch_step(lbm_batch *b, int64_t n);
void lbm_batch_destroy(lbm_batch *b);

/* Continuous batching: make grids[0..n-1] the batch's members (n >= 0; the
 * same rules as lbm_batch_create for each grid; grids may join at any step
 * count, each keeps its own buffer parity).  Waits for the batch's queued
 * steps, then rewrites the groups' instance and tile tables in place (a table
 * grows, to twice its size or more, only when the new one does not fit) and,
 * when every group keeps its step kernel, updates the kernel nodes of the
 * batch's instantiated step graph in place (new tile counts and tables)
 * instead of building a new graph.  Grids that leave may then be stepped
 * alone or destroyed.  The batch keeps its stream, unless that stream is
 * owned by a grid that leaves: then the batch moves, in stream order, to the
 * first remaining grid's stream (or to one of its own).  With n = 0 the
 * batch is empty and lbm_batch_step only counts steps.  Errors in the grids
 * leave the batch as it was; an allocation or device error leaves it broken
 * (LBM_ESTATE from then on). */
int lbm_batch_update(lbm_batch *b, lbm_grid *const *grids, int32_t n);

/* Residuals of every grid of the batch (out[n], batch order) with one
 * synchronisation; same definitions as lbm_residual.  Returns LBM_EUNSTABLE
 * (after filling every record) if any grid has bad cells. */
int lbm_batch_residuals(lbm_batch *b, lbm_resid *out);

/* Group g of a batch (one lattice/precision/table kind/force mode, one kernel launch per
 * step): returns the number of groups (>= 0) or an error; fills the lattice
 * (0 for a fused group holding both lattices), precision and total cells of
 * group g.  With every output pointer NULL, any g returns the count (an
 * empty batch has none); otherwise g out of range is LBM_EINVAL. */
int lbm_batch_info(const lbm_batch *b, int32_t group, int32_t *q, int32_t *precision, int64_t *cells);

/* Measurement hook: launch only group g's step kernel n times (n even, so
 * buffer parities are unchanged); the other groups do not advance, so the
 * batch's states are no longer one consistent time level afterwards. */
int lbm_batch_step_group(lbm_batch *b, int32_t group, int64_t n);

/* Autotuner for a batch: for each group, times `steps` launches (rounded up
 * to even, after 2 untimed ones) of the group's own step kernel over all of
 * its tiles for each tile shape (1, 2 or 4 rows per workgroup) and each
 * occupancy cap (none, 24, 20 or 16 waves per CU), in two sweeps over these
 * 12 configurations, and keeps the pair with the fastest of its two times
 * for that group (until then a group launches with the choice of its first
 * grid).  The trials step the batch's own state: every grid advances by the
 * same even number of steps, 24 (steps + 2), exactly as lbm_batch_step would
 * have advanced it, since no result depends on the launch shape.  Step
 * counters advance accordingly.  Synchronises; LBM_EINVAL for a null batch,
 * LBM_ENOMEM / LBM_EDEVICE if a trial's tile table or launch fails (the
 * grids' states are then not at one time level: initialise them again). */
int lbm_batch_autotune(lbm_batch *b, int32_t steps);

/* Launch shape of batch group g: waves (rows) per workgroup and the resident
 * waves per CU cap (0 = none).  LBM_EINVAL when g is out of range. */
int lbm_batch_group_launch(const lbm_batch *b, int32_t group, int32_t *waves_per_block, int32_t *waves_per_cu_cap);

/* Launch configuration of the step kernels for a grid (and the batches made
 * from it later): waves per workgroup (1, 2 or 4; each wave covers 64
 * columns of one row; 0 = default 4). */
int lbm_set_launch(lbm_grid *g, int32_t waves_per_block);

/* Cap on the resident waves per CU of a grid's step launches (and of the
 * batches made from it later): 0 = no cap, else 4..64 (LBM_EINVAL
 * otherwise).  The cap is enforced by reserving unused LDS per workgroup; it
 * trades memory-level parallelism against the number of DRAM pages open at
 * once and changes no result. */
int lbm_set_occupancy(lbm_grid *g, int32_t waves_per_cu);

/* Autotuner: times `steps` step launches for each tile shape (1, 2 or 4
 * waves, i.e. rows, per workgroup) and each occupancy cap (none, 24, 20 or
 * 16 waves per CU), in two sweeps, keeps the pair with the fastest of its two
 * times and caches it for the process per
 * (q, precision, table kind, n1, n2).  The timing steps run on the grid's own
 * buffers, so call it between create and init (the grid needs lbm_init
 * afterwards).  Returns the chosen waves per workgroup (> 0; the cap is in
 * lbm_grid_info) or an error code. */
int lbm_autotune(lbm_grid *g, int32_t steps);

/* Plain device copy kernel (for calibrating memory-traffic counters): copies
 * `bytes` (a multiple of 16) from src to dst on `stream`, one 16-byte element
 * per lane. */
int lbm_copy_probe(void *dst, const void *src, size_t bytes, void *stream);

/* Bandwidth probes with non-temporal 16-byte accesses, one element per lane
 * over a full grid: kind 0 copies src to dst, kind 1 reads src (dst is a
 * 16-byte sink written only if src holds a fixed 128-bit pattern), kind 2
 * fills dst.  bytes: a multiple of 16.  Returns LBM_EINVAL on bad arguments,
 * LBM_EDEVICE if the launch fails; asynchronous on `stream`. */
int lbm_bandwidth_probe(void *dst, const void *src, size_t bytes, int32_t kind, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
