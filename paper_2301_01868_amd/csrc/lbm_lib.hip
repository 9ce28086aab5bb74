// Host side of the C ABI declared in include/lbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_maps.hpp"
#include "lbm_setup.hpp"

using namespace lbm;

namespace {

thread_local std::string g_last_error;

struct GraphCache {
    hipGraphExec_t exec = nullptr;
    int steps = 0;
};

} // namespace

struct lbm_grid {
    lbm_grid_desc desc{};
    int q = 0, n1 = 0, n2 = 0, h = 0, pitch = 0, hw = 0, ncell = 0;
    int row = 1, nent = 0;
    int ct = 0;                   // step tables: 0 per row, 1 per cell, 2 per cell rebuilt from the geometry
    int wide = 0;                 // a population buffer of 2 GiB or more: the step's row-based addressing
    double *ge = nullptr;         // staged geometry of ct = 2 (GE_* fields)
    int precision = LBM_FP64;
    int device = 0;               // device current at create (the grid's buffers live there)
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool has_alloc = false;
    lbm_allocator alloc{};
    std::vector<void *> allocs;
    std::vector<size_t> alloc_bytes;   // size of each entry of allocs
    size_t bytes = 0;                  // device bytes currently held
    // device buffers
    void *P[2] = {nullptr, nullptr};
    void *side[2] = {nullptr, nullptr};
    void *lag[2] = {nullptr, nullptr};
    void *tab = nullptr;
    double *base = nullptr, *mB64 = nullptr;
    double *X = nullptr, *Y = nullptr;
    double *Jgeo = nullptr, *Jused = nullptr, *G3 = nullptr, *g4 = nullptr, *xc = nullptr, *yc = nullptr;
    double *mom = nullptr, *snap = nullptr, *partial = nullptr, *redout = nullptr;
    InstDesc *d_inst = nullptr;
    int4 *d_tiles = nullptr;
    int ntiles = 0, wpb = 4;
    int cap = 0;                  // resident waves per CU (0: no cap), see occupancy_lds
    InstDesc h_inst{};
    int64_t step = 0;
    int par = 0;
    bool inited = false;
    double mass0 = 0.0;
    bool snap_valid = false;
    int64_t snap_step = 0;
    GraphCache graph[2];
    std::vector<lbm_batch *> batches;   // batches that hold this grid
    std::string err;
};

struct lbm_batch {
    std::vector<lbm_grid *> grids;
    hipStream_t stream = nullptr;
    std::vector<hipStream_t> others;   // distinct grid streams other than `stream`
    hipEvent_t ev = nullptr;
    uint32_t flags = 0;
    bool own_stream = false;           // the stream was made for the batch (its members left)
    double *d_res = nullptr;           // [res_cap][RED_NF] reduction results
    size_t res_cap = 0;
    struct Group {
        int q = 0, precision = 0, cell = 0, iter = 0, wide = 0;
        InstDesc *d_inst = nullptr;
        int4 *d_tiles = nullptr;
        int ntiles = 0, wpb = 4, cap = 0;
        int inst_cap = 0, tile_cap = 0; // capacity of d_inst and d_tiles (entries)
        std::vector<int> members;      // indices into grids
    };
    std::vector<Group> groups;
    std::vector<void *> allocs;
    // the step graph: GS steps, one kernel node per group and step, built node
    // by node so that membership changes can update the nodes in place
    hipGraph_t gtmpl = nullptr;
    hipGraphExec_t gexec = nullptr;
    struct Node {
        hipGraphNode_t node;
        int group, par;
    };
    std::vector<Node> nodes;
    int64_t step = 0;
    bool broken = false;               // a member grid was destroyed first: only destroy is allowed
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
static int fail(lbm_grid *g, int code, const std::string &msg)
{
    if (g) g->err = msg;
    g_last_error = msg;
    return code;
}

#define HIPCHK(g, call)                                                                              \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return fail((g), LBM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));        \
    } while (0)

static void *dalloc(lbm_grid *g, size_t bytes)
{
    bytes = (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    if (g->has_alloc) {
        p = g->alloc.alloc(bytes, g->alloc.ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) {
        g->allocs.push_back(p);
        g->alloc_bytes.push_back(bytes);
        g->bytes += bytes;
    }
    return p;
}

static void dfree(lbm_grid *g, void *p)
{
    if (!p) return;
    auto it = std::find(g->allocs.begin(), g->allocs.end(), p);
    if (it != g->allocs.end()) {
        const size_t k = (size_t)(it - g->allocs.begin());
        g->bytes -= g->alloc_bytes[k];
        g->alloc_bytes.erase(g->alloc_bytes.begin() + k);
        g->allocs.erase(it);
    }
    if (g->has_alloc) g->alloc.free(p, g->alloc.ctx);
    else (void)hipFree(p);
}

static size_t store_size(int precision)
{
    return precision == LBM_FP64 ? sizeof(double) : (precision == LBM_FP16 ? 2 : sizeof(float));
}
static size_t comp_size(int precision) { return precision == LBM_FP64 ? sizeof(double) : sizeof(float); }

static dim3 cell_grid(int n1, int n2) { return dim3((n2 + 127) / 128, n1); }

// Dynamic LDS reserved per workgroup of a step launch to cap the resident
// waves per CU at `cap` (0: no reservation).  Beyond the staged geometry of
// per-cell steps and the exchange tile of D2Q9 steps the step kernels use no
// LDS; the reservation only limits how many workgroups share a CU's 160 KiB.  At
// most 64 KiB is reserved per workgroup, so caps below three workgroups per
// CU are not enforced exactly.
static unsigned occupancy_lds(int cap, int wpb)
{
    if (cap <= 0) return 0u;
    const unsigned lds_per_cu = 160u * 1024u;
    const unsigned wg = (unsigned)(cap / wpb > 1 ? cap / wpb : 1);
    const unsigned b = (lds_per_cu / wg + 255u) & ~255u;
    return b > 65536u ? 65536u : b;
}

// kernel dispatch tables -------------------------------------------------------
typedef void (*StepFn)(const InstDesc *, const int4 *, int);

template <int Q, int CT, bool MOM, bool ITER, bool WIDE>
static StepFn step_fn4(int precision)
{
    if (precision == LBM_FP64) return k_step<Q, double, double, CT, MOM, ITER, WIDE>;
    if (precision == LBM_FP16) return k_step<Q, float, _Float16, CT, MOM, ITER, WIDE>;
    return k_step<Q, float, float, CT, MOM, ITER, WIDE>;
}
template <int Q, int CT, bool MOM, bool ITER>
static StepFn step_fn3(int precision, int wide)
{
    return wide ? step_fn4<Q, CT, MOM, ITER, true>(precision) : step_fn4<Q, CT, MOM, ITER, false>(precision);
}

// the moments pass reads the stored tables (per-cell tables exist for every
// per-cell grid)
template <int Q>
static StepFn step_fn(int precision, int ct, int mom, int iter, int wide)
{
    if (mom) return ct ? step_fn3<Q, 1, true, false>(precision, wide) : step_fn3<Q, 0, true, false>(precision, wide);
    if (iter)
        return ct == 2 ? step_fn3<Q, 2, false, true>(precision, wide)
                       : (ct ? step_fn3<Q, 1, false, true>(precision, wide) : step_fn3<Q, 0, false, true>(precision, wide));
    return ct == 2 ? step_fn3<Q, 2, false, false>(precision, wide)
                   : (ct ? step_fn3<Q, 1, false, false>(precision, wide) : step_fn3<Q, 0, false, false>(precision, wide));
}

// kernel for a grid or batch group: lattice, storage precision, table kind,
// moments pass, fixed-point force passes (iterations > 0)
template <int CT, bool ITER>
static StepFn mixed_fn(int precision)
{
    if (precision == LBM_FP64) return k_step_mixed<double, double, CT, false, ITER>;
    if (precision == LBM_FP16) return k_step_mixed<float, _Float16, CT, false, ITER>;
    return k_step_mixed<float, float, CT, false, ITER>;
}

// q = 0: a batch group holding both lattices (one fused launch, no moments
// pass; its grids are never wide)
static StepFn pick_step(int q, int precision, int ct, int mom, int iter, int wide)
{
    if (q == 0) {
        if (iter) return ct == 2 ? mixed_fn<2, true>(precision) : (ct ? mixed_fn<1, true>(precision) : mixed_fn<0, true>(precision));
        return ct == 2 ? mixed_fn<2, false>(precision) : (ct ? mixed_fn<1, false>(precision) : mixed_fn<0, false>(precision));
    }
    return q == 9 ? step_fn<9>(precision, ct, mom, iter, wide) : step_fn<21>(precision, ct, mom, iter, wide);
}

// dynamic LDS of a step launch: the occupancy reservation, or the staged
// geometry of ct = 2 if larger (q = 0, both lattices: the D2Q21 tile)
static unsigned step_lds(int ct, int q, int precision, int cap, int wpb)
{
    unsigned b = occupancy_lds(cap, wpb);
    if (ct == 2) {
        const unsigned sg = q == 9 ? (precision == LBM_FP64 ? geo_stage_bytes<9, double>() : geo_stage_bytes<9, float>())
                                   : (precision == LBM_FP64 ? geo_stage_bytes<21, double>() : geo_stage_bytes<21, float>());
        if (sg > b) b = sg;
    }
    if (ct == 0 && (q == 9 || q == 0) && precision != LBM_FP16) {
        // the D2Q9 exchange tile (q = 0: the group's D2Q9 tiles) of FP32 and FP64 storage
        static_assert(xch_step<9, float, 0, false>() && xch_step<9, double, 0, false>() &&
                          !xch_step<9, _Float16, 0, false>() && !xch_step<21, float, 0, false>(),
                      "exchange tiles of D2Q9 FP32 and FP64 steps only");
        const unsigned xb = precision == LBM_FP64 ? xch_bytes<9, double>(wpb) : xch_bytes<9, float>(wpb);
        if (xb > b) b = xb;
    }
    return b;
}

// tiles of one grid in row-major order: (instance, first row, first column, lattice)
static std::vector<int4> make_tiles(int inst, int n1, int n2, int wpb, int q)
{
    std::vector<int4> nat;
    const int ncs = (n2 + 63) / 64;
    for (int r0 = 0; r0 < n1; r0 += wpb)
        for (int cs = 0; cs < ncs; ++cs) nat.push_back(make_int4(inst, r0, cs * 64, q));
    return nat;
}

// Workgroups are dealt round-robin to the 8 XCDs.  Order the tile table so
// that each XCD takes runs of XCD_RUN consecutive tiles while the 8 XCDs stay
// side by side: at any moment the whole chip streams one narrow band of rows.
// Measured on the step kernel, this beats both the natural order (neighbouring
// tiles on different XCDs) and one contiguous slab per XCD (8 distant bands
// at once, which spreads the Q concurrent row streams over many more DRAM
// pages); runs of 16 to 64 tiles perform alike.
static constexpr size_t XCD_RUN = 32;
static std::vector<int4> xcd_order(const std::vector<int4> &nat, int dummy_row)
{
    const size_t nt = nat.size();
    const size_t nt8 = (nt + 8 * XCD_RUN - 1) / (8 * XCD_RUN) * (8 * XCD_RUN);
    std::vector<int4> out(nt8);
    for (size_t b = 0; b < nt8; ++b) {
        const size_t x = b % 8, y = b / 8;
        const size_t t = ((y / XCD_RUN) * 8 + x) * XCD_RUN + y % XCD_RUN;
        out[b] = t < nt ? nat[t] : make_int4(nat.empty() ? 0 : nat[0].x, dummy_row, 0, 0);
    }
    return out;
}

static int upload_inst(lbm_grid *g)
{
    HIPCHK(g, hipMemcpyAsync(g->d_inst, &g->h_inst, sizeof(InstDesc), hipMemcpyHostToDevice, g->stream));
    HIPCHK(g, hipStreamSynchronize(g->stream));
    return LBM_OK;
}

static void drop_graphs(lbm_grid *g)
{
    for (auto &gc : g->graph) {
        if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
        gc.exec = nullptr;
        gc.steps = 0;
    }
}

static int build_tiles(lbm_grid *g)
{
    auto nat = make_tiles(0, g->n1, g->n2, g->wpb, g->q);
    auto ord = xcd_order(nat, g->n1);
    if (g->d_tiles) dfree(g, g->d_tiles);
    g->d_tiles = (int4 *)dalloc(g, ord.size() * sizeof(int4));
    if (!g->d_tiles) return fail(g, LBM_ENOMEM, "tile table allocation failed");
    g->ntiles = (int)ord.size();
    HIPCHK(g, hipMemcpyAsync(g->d_tiles, ord.data(), ord.size() * sizeof(int4), hipMemcpyHostToDevice, g->stream));
    HIPCHK(g, hipStreamSynchronize(g->stream));
    drop_graphs(g);
    return LBM_OK;
}

static int launch_step(lbm_grid *g, int par, int mom)
{
    StepFn fn = pick_step(g->q, g->precision, g->ct, mom, g->h_inst.iters > 0, g->wide);
    hipLaunchKernelGGL(fn, dim3(g->ntiles), dim3(64 * g->wpb), step_lds(g->ct, g->q, g->precision, g->cap, g->wpb), g->stream, (const InstDesc *)g->d_inst,
                       (const int4 *)g->d_tiles, par);
    HIPCHK(g, hipGetLastError());
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// API
// ---------------------------------------------------------------------------
extern "C" {

int lbm_lattice(int32_t q, int32_t *cxo, int32_t *cyo, double *w, double *T0)
{
    if (q != 9 && q != 21) return fail(nullptr, LBM_EINVAL, "q must be 9 or 21");
    for (int a = 0; a < q; ++a) {
        if (cxo) cxo[a] = cx(a);
        if (cyo) cyo[a] = cy(a);
        if (w) w[a] = q == 9 ? weight<9>(a) : weight<21>(a);
    }
    if (T0) *T0 = q == 9 ? lattice_T0<9>() : lattice_T0<21>();
    return LBM_OK;
}

int lbm_map_planar(int32_t n1, int32_t n2, int32_t halo, const double *faces, double d_per, double *x, double *y)
{
    std::string e = lbm_maps::map_planar(n1, n2, halo, faces, d_per, x, y);
    return e.empty() ? LBM_OK : fail(nullptr, LBM_EINVAL, "lbm_map_planar: " + e);
}

int lbm_map_polar(int32_t n1, int32_t n2, int32_t halo, const double *r_faces, int32_t ntheta, double *x, double *y)
{
    std::string e = lbm_maps::map_polar(n1, n2, halo, r_faces, ntheta, x, y);
    return e.empty() ? LBM_OK : fail(nullptr, LBM_EINVAL, "lbm_map_polar: " + e);
}

const char *lbm_last_error(const lbm_grid *g)
{
    if (g && !g->err.empty()) return g->err.c_str();
    return g_last_error.c_str();
}

// A grid destroyed while a batch still holds it: the batch no longer
// references the grid or its stream (which may be destroyed below), and every
// call on it other than lbm_batch_destroy returns LBM_ESTATE.
static void detach_from_batches(lbm_grid *g)
{
    for (lbm_batch *b : g->batches) {
        b->broken = true;
        if (b->stream == g->stream) b->stream = nullptr;
        b->others.erase(std::remove(b->others.begin(), b->others.end(), g->stream), b->others.end());
        for (auto &m : b->grids)
            if (m == g) m = nullptr;
    }
    g->batches.clear();
}

void lbm_grid_destroy(lbm_grid *g)
{
    if (!g) return;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    detach_from_batches(g);
    drop_graphs(g);
    auto all = g->allocs;
    for (void *p : all) dfree(g, p);
    if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
}

int lbm_grid_create(const lbm_grid_desc *desc, lbm_grid **out)
{
    if (!desc || !out) return fail(nullptr, LBM_EINVAL, "null argument");
    *out = nullptr;
    const lbm_grid_desc &D = *desc;
    if (D.q != 9 && D.q != 21) return fail(nullptr, LBM_EINVAL, "q must be 9 or 21");
    const int cm = D.q == 9 ? 1 : 3;
    if (D.n1 < 1 || D.n2 < 1) return fail(nullptr, LBM_EINVAL, "n1 and n2 must be positive");
    if (D.halo < cm + 1) return fail(nullptr, LBM_EINVAL, "halo must be at least c_max + 1");
    if (!D.x || !D.y) return fail(nullptr, LBM_EINVAL, "mapping coordinates missing");
    if (!(D.tau > 0.5)) return fail(nullptr, LBM_EINVAL, "tau must exceed 1/2");
    const bool per1 = D.bc_lo == LBM_PERIODIC || D.bc_hi == LBM_PERIODIC;
    if (per1 && D.bc_lo != D.bc_hi) return fail(nullptr, LBM_EINVAL, "a periodic q1 side must be paired");
    for (int b : {D.bc_lo, D.bc_hi})
        if (b != LBM_PERIODIC && b != LBM_NOSLIP && b != LBM_MOVING) return fail(nullptr, LBM_EINVAL, "unknown boundary kind");
    if (D.n1 < cm) return fail(nullptr, LBM_EINVAL, "n1 must be at least c_max");
    if (D.precision != LBM_FP64 && D.precision != LBM_FP32 && D.precision != LBM_FP16)
        return fail(nullptr, LBM_EINVAL, "unknown precision");
    if (D.offset_base != LBM_BASE_LOCAL_REST && D.offset_base != LBM_BASE_W_RHO0 && D.offset_base != LBM_BASE_NONE)
        return fail(nullptr, LBM_EINVAL, "unknown offset base");
    if (D.iterations < 0 || D.iterations > 16) return fail(nullptr, LBM_EINVAL, "iterations must be in 0..16");
    if (D.geometry != LBM_GEOM_AUTO && D.geometry != LBM_GEOM_CELL && D.geometry != LBM_GEOM_CELL_TABLE)
        return fail(nullptr, LBM_EINVAL, "unknown geometry mode");
    if ((int64_t)D.n1 * D.n2 > (int64_t)1 << 30) return fail(nullptr, LBM_EINVAL, "grid too large");
    // the set-up kernels launch one grid row of threads per mapping row
    if ((int64_t)D.n1 + 2 * (int64_t)D.halo > 65535)
        return fail(nullptr, LBM_EINVAL, "n1 + 2 halo must not exceed 65535");
    {   // the step addresses populations through resources based at a row: the
        // 2 c_max + 1 rows of a stencil must stay below 4 GiB (32-bit offsets)
        const int64_t pitch = D.n2 >= 64 ? (D.n2 + 63) / 64 * 64 : D.n2;
        const int64_t row_bytes = (int64_t)D.q * pitch * (D.precision == LBM_FP64 ? 8 : (D.precision == LBM_FP16 ? 2 : 4));
        if ((2 * cm + 1) * row_bytes >= ((int64_t)1 << 32))
            return fail(nullptr, LBM_EINVAL, "rows too long: 2 c_max + 1 rows of populations must stay below 4 GiB");
    }

    lbm_grid *g = new lbm_grid();
    if (hipGetDevice(&g->device) != hipSuccess) {
        delete g;
        return fail(nullptr, LBM_EDEVICE, "hipGetDevice failed");
    }
    g->desc = D;
    g->desc.x = g->desc.y = nullptr;
    g->q = D.q;
    g->n1 = D.n1;
    g->n2 = D.n2;
    g->h = D.halo;
    g->hw = cm;
    g->ncell = D.n1 * D.n2;
    g->pitch = D.n2 >= 64 ? (D.n2 + 63) / 64 * 64 : D.n2;
    g->precision = D.precision;
    if (D.alloc) {
        g->has_alloc = true;
        g->alloc = *D.alloc;
    }
    if (D.stream) {
        g->stream = (hipStream_t)D.stream;
    } else {
        if (hipStreamCreate(&g->stream) != hipSuccess) {
            delete g;
            return fail(nullptr, LBM_EDEVICE, "hipStreamCreate failed");
        }
        g->own_stream = true;
    }
    auto bail = [&](int code, const std::string &m) {
        g_last_error = m;
        lbm_grid_destroy(g);
        return code;
    };

    const int q = g->q, n1 = g->n1, n2 = g->n2, h = g->h, nc = g->ncell;
    const int H1 = n1 + 2 * h, H2 = n2 + 2 * h;
    const size_t nh = (size_t)H1 * H2;
    const int nf = geo_fields(q);

    // FP64 per-cell arrays kept for the grid's lifetime
    g->X = (double *)dalloc(g, nh * 8);
    g->Y = (double *)dalloc(g, nh * 8);
    g->Jgeo = (double *)dalloc(g, (size_t)nc * 8);
    g->Jused = (double *)dalloc(g, (size_t)nc * 8);
    g->G3 = (double *)dalloc(g, (size_t)nc * 3 * 8);
    g->g4 = (double *)dalloc(g, (size_t)nc * 4 * 8);
    g->xc = (double *)dalloc(g, (size_t)nc * 8);
    g->yc = (double *)dalloc(g, (size_t)nc * 8);
    g->mom = (double *)dalloc(g, (size_t)nc * 5 * 8);
    g->snap = (double *)dalloc(g, (size_t)nc * 2 * 8);
    g->partial = (double *)dalloc(g, (size_t)RED_BLOCKS * RED_NF * 8);
    g->redout = (double *)dalloc(g, 8 * 8);
    g->d_inst = (InstDesc *)dalloc(g, sizeof(InstDesc));
    double *tg = (double *)dalloc(g, nh * 4 * 8);
    double *geo = (double *)dalloc(g, (size_t)nc * nf * 8);
    int *flag = (int *)dalloc(g, 2 * sizeof(int));
    if (!g->X || !g->Y || !g->Jgeo || !g->Jused || !g->G3 || !g->g4 || !g->xc || !g->yc || !g->mom || !g->snap ||
        !g->partial || !g->redout || !g->d_inst || !tg || !geo || !flag)
        return bail(LBM_ENOMEM, "device allocation failed (geometry)");

    hipStream_t st = g->stream;
#define HIPB(call)                                                                                       \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess) return bail(LBM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)
    HIPB(hipMemcpyAsync(g->X, D.x, nh * 8, hipMemcpyHostToDevice, st));
    HIPB(hipMemcpyAsync(g->Y, D.y, nh * 8, hipMemcpyHostToDevice, st));
    // cell centres
    for (int i = 0; i < n1; ++i) {
        HIPB(hipMemcpy2DAsync(g->xc + (size_t)i * n2, n2 * 8, D.x + (size_t)(i + h) * H2 + h, H2 * 8, n2 * 8, 1,
                              hipMemcpyHostToDevice, st));
        HIPB(hipMemcpy2DAsync(g->yc + (size_t)i * n2, n2 * 8, D.y + (size_t)(i + h) * H2 + h, H2 * 8, n2 * 8, 1,
                              hipMemcpyHostToDevice, st));
    }
    // geometry precompute (FP64)
    hipLaunchKernelGGL(k_tangent, dim3((H2 + 127) / 128, H1), dim3(128), 0, st, g->X, g->Y, H1, H2, tg);
    if (q == 9)
        hipLaunchKernelGGL(k_geom_cell<9>, cell_grid(n1, n2), dim3(128), 0, st, tg, n1, n2, h, geo, g->Jgeo, g->g4);
    else
        hipLaunchKernelGGL(k_geom_cell<21>, cell_grid(n1, n2), dim3(128), 0, st, tg, n1, n2, h, geo, g->Jgeo, g->g4);
    HIPB(hipGetLastError());
    HIPB(hipMemcpyAsync(g->G3, geo + (size_t)GEO_G11 * nc, (size_t)nc * 3 * 8, hipMemcpyDeviceToDevice, st));
    HIPB(hipMemcpyAsync(g->Jused, g->Jgeo, (size_t)nc * 8, hipMemcpyDeviceToDevice, st));
    int hflag[2] = {0, 0};
    HIPB(hipMemcpyAsync(flag, hflag, sizeof hflag, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_rowcheck, cell_grid(n1, n2), dim3(128), 0, st, geo, n1, n2, nf, 1e-11, flag);
    HIPB(hipGetLastError());
    HIPB(hipMemcpyAsync(hflag, flag, sizeof hflag, hipMemcpyDeviceToHost, st));
    HIPB(hipStreamSynchronize(st));
    if (hflag[1]) return bail(LBM_EINVAL, "the mapping has J <= 0 (or non-finite geometry) in some cell");
    g->row = (D.geometry != LBM_GEOM_AUTO) ? 0 : (hflag[0] ? 0 : 1);
    g->ct = g->row ? 0 : (D.geometry == LBM_GEOM_CELL_TABLE ? 1 : 2);
    // offset storage with a base other than the local rest state shifts every
    // pulled value by base differences the rebuilt FP32 terms carry only to a
    // few 1e-6: such grids read the stored table instead
    if (g->ct == 2 && g->precision != LBM_FP64 && D.offset_base != LBM_BASE_LOCAL_REST) g->ct = 1;
    g->nent = g->row ? n1 : nc;
    const int nfe = g->precision == LBM_FP64 ? (int)GE_J : (int)GE_NF;
    const size_t gfs = (size_t)(n1 + 2 * cm) * (n2 + 2 * cm);
    if (g->ct == 2) {
        // geometry the step stages (the tangents are freed below)
        g->ge = (double *)dalloc(g, gfs * nfe * 8);
        if (!g->ge) return bail(LBM_ENOMEM, "device allocation failed (geometry)");
        hipLaunchKernelGGL(k_geo_ext, dim3((n2 + 2 * cm + 127) / 128, n1 + 2 * cm), dim3(128), 0, st, tg, n1, n2, h, cm, nfe,
                           g->ge);
        HIPB(hipGetLastError());
    }
    if (g->row) {
        hipLaunchKernelGGL(k_canon_rows, cell_grid(n1, n2), dim3(128), 0, st, n1, n2, g->Jgeo, g->G3);
        HIPB(hipGetLastError());
        HIPB(hipMemcpyAsync(g->Jused, g->Jgeo, (size_t)nc * 8, hipMemcpyDeviceToDevice, st));
    }

    // tables
    TableArgs ta{};
    ta.geo = geo;
    ta.n1 = n1;
    ta.n2 = n2;
    ta.ncell = nc;
    ta.cellmode = !g->row;
    ta.nent = g->nent;
    ta.periodic1 = per1;
    ta.bc_lo = D.bc_lo;
    ta.bc_hi = D.bc_hi;
    // FP64 stores and computes with the particle numbers themselves; FP32 and
    // FP16 store offsets from the requested base and compute relative to the
    // local rest state, whose offsets are the smallest numbers
    ta.base_kind = (D.precision == LBM_FP64) ? 2 : D.offset_base;
    ta.cbase_kind = (D.precision == LBM_FP64) ? 2 : 0;
    ta.rho0 = D.rho0;
    ta.kpi = -(1.0 - 1.0 / (2.0 * D.tau));
    g->base = (double *)dalloc(g, (size_t)g->nent * q * 8);
    double *cbase = (double *)dalloc(g, (size_t)g->nent * q * 8);
    g->mB64 = (double *)dalloc(g, (size_t)g->nent * 8);
    const int tabw = q == 9 ? Tab<9>::STRIDE : Tab<21>::STRIDE;
    g->tab = dalloc(g, (size_t)g->nent * tabw * comp_size(g->precision));
    if (!g->base || !cbase || !g->mB64 || !g->tab) return bail(LBM_ENOMEM, "device allocation failed (tables)");
    const dim3 eb((g->nent + 127) / 128);
    if (q == 9) {
        hipLaunchKernelGGL(k_base<9>, eb, dim3(128), 0, st, ta, g->base, cbase, g->mB64);
        if (g->precision == LBM_FP64)
            hipLaunchKernelGGL((k_table<9, double>), eb, dim3(128), 0, st, ta, g->base, cbase, g->mB64, (double *)g->tab);
        else
            hipLaunchKernelGGL((k_table<9, float>), eb, dim3(128), 0, st, ta, g->base, cbase, g->mB64, (float *)g->tab);
    } else {
        hipLaunchKernelGGL(k_base<21>, eb, dim3(128), 0, st, ta, g->base, cbase, g->mB64);
        if (g->precision == LBM_FP64)
            hipLaunchKernelGGL((k_table<21, double>), eb, dim3(128), 0, st, ta, g->base, cbase, g->mB64, (double *)g->tab);
        else
            hipLaunchKernelGGL((k_table<21, float>), eb, dim3(128), 0, st, ta, g->base, cbase, g->mB64, (float *)g->tab);
    }
    HIPB(hipGetLastError());

    // populations and side state
    const size_t plane = (size_t)n1 * g->pitch;
    g->wide = plane * q * store_size(g->precision) >= ((size_t)1 << 31) ? 1 : 0;
    for (int b = 0; b < 2; ++b) {
        g->P[b] = dalloc(g, plane * q * store_size(g->precision));
        g->side[b] = dalloc(g, (size_t)4 * g->hw * g->pitch * comp_size(g->precision));
        g->lag[b] = dalloc(g, 2 * plane * comp_size(g->precision));
        if (!g->P[b] || !g->side[b] || !g->lag[b]) return bail(LBM_ENOMEM, "device allocation failed (populations)");
        HIPB(hipMemsetAsync(g->lag[b], 0, 2 * plane * comp_size(g->precision), st));
        HIPB(hipMemsetAsync(g->P[b], 0, plane * q * store_size(g->precision), st));
        HIPB(hipMemsetAsync(g->side[b], 0, (size_t)4 * g->hw * g->pitch * comp_size(g->precision), st));
    }
    HIPB(hipStreamSynchronize(st));
    dfree(g, tg);
    dfree(g, geo);
    dfree(g, flag);
    dfree(g, cbase);

    InstDesc &I = g->h_inst;
    I.P[0] = g->P[0];
    I.P[1] = g->P[1];
    I.side[0] = g->side[0];
    I.side[1] = g->side[1];
    I.lag[0] = g->lag[0];
    I.lag[1] = g->lag[1];
    I.tab = g->tab;
    I.mom = g->mom;
    I.mB64 = g->mB64;
    I.plane = (long long)plane;
    // populations [row][column block][direction][block width] (pidx): FP32
    // and FP64 rows in blocks of 64 columns, FP16 rows (and rows narrower
    // than 64) as one block, the faster layout measured for each storage
    // type; the two force sums [row][2][column]
    {
        const bool blocks = g->precision != LBM_FP16 && g->pitch >= 64;
        const int bw = blocks ? 64 : g->pitch;
        I.bs = blocks ? 6 : 30;
        I.bm = (1 << I.bs) - 1;
        I.sa = bw;
        I.sr = (long long)q * g->pitch;
        I.sb = (long long)q * bw;
    }
    I.lsa = g->pitch;
    I.lsr = 2LL * g->pitch;
    I.n1 = n1;
    I.n2 = n2;
    I.pitch = g->pitch;
    I.hw = g->hw;
    I.periodic1 = per1;
    I.bc_lo = per1 ? BC_PERIODIC : D.bc_lo;
    I.bc_hi = per1 ? BC_PERIODIC : D.bc_hi;
    I.cell = !g->row;
    I.iters = D.iterations;
    I.ncell = nc;
    I.par0 = 0;
    I.sbase = ta.base_kind;
    I.rho0 = D.rho0;
    I.geo = g->ge;
    I.gfs = (long long)gfs;
    I.gw = n2 + 2 * cm;
    I.ut_lo = D.ut_lo;
    I.ut_hi = D.ut_hi;
    I.a1 = D.accel[0];
    I.a2 = D.accel[1];
    I.omega = 1.0 / D.tau;
    I.kpi = -(1.0 - 1.0 / (2.0 * D.tau));
    if (upload_inst(g) != LBM_OK) return bail(LBM_EDEVICE, g->err);
    g->wpb = 4;
    if (build_tiles(g) != LBM_OK) return bail(LBM_EDEVICE, g->err);
    HIPB(hipStreamSynchronize(st));
#undef HIPB
    *out = g;
    return LBM_OK;
}

int lbm_grid_info_get(const lbm_grid *g, lbm_grid_info *out)
{
    if (!g || !out) return fail(nullptr, LBM_EINVAL, "null argument");
    out->q = g->q;
    out->n1 = g->n1;
    out->n2 = g->n2;
    out->pitch = g->pitch;
    out->precision = g->precision;
    out->row_tables = g->row;
    out->table_kind = g->ct;
    out->step = g->step;
    out->bytes_per_update = 2.0 * g->q * (double)store_size(g->precision);
    out->device_bytes = g->bytes;
    out->waves_per_block = g->wpb;
    out->waves_per_cu_cap = g->cap;
    return LBM_OK;
}

int lbm_set_launch(lbm_grid *g, int32_t wpb)
{
    if (!g) return fail(nullptr, LBM_EINVAL, "null grid");
    if (wpb == 0) wpb = 4;
    if (wpb != 1 && wpb != 2 && wpb != 4) return fail(g, LBM_EINVAL, "waves per block must be 1, 2 or 4");
    g->wpb = wpb;
    return build_tiles(g);
}

int lbm_set_occupancy(lbm_grid *g, int32_t waves_per_cu)
{
    if (!g) return fail(nullptr, LBM_EINVAL, "null grid");
    if (waves_per_cu != 0 && (waves_per_cu < 4 || waves_per_cu > 64))
        return fail(g, LBM_EINVAL, "waves per CU cap must be 0 or 4..64");
    g->cap = waves_per_cu;
    drop_graphs(g);
    return LBM_OK;
}

namespace {
// process-wide autotuner cache: (q, precision, table kind, n1, n2) ->
// (waves per block, waves per CU cap)
// (shared by every grid of the process, so guarded)
std::map<std::tuple<int, int, int, int, int>, std::pair<int, int>> g_tuned;
std::mutex g_tuned_mu;
} // namespace

int lbm_autotune(lbm_grid *g, int32_t steps)
{
    if (!g) return fail(nullptr, LBM_EINVAL, "null grid");
    if (steps < 2) steps = 2;
    const auto key = std::make_tuple(g->q, g->precision, g->ct, g->n1, g->n2);
    {
        std::pair<int, int> hit{0, 0};
        {
            std::lock_guard<std::mutex> lk(g_tuned_mu);
            auto it = g_tuned.find(key);
            if (it != g_tuned.end()) hit = it->second;
        }
        if (hit.first) {
            int rc = lbm_set_launch(g, hit.first);
            if (rc == LBM_OK) rc = lbm_set_occupancy(g, hit.second);
            return rc != LBM_OK ? rc : hit.first;
        }
    }
    struct Events {   // destroyed on every return path
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Events()
        {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } ev;
    HIPCHK(g, hipEventCreate(&ev.e0));
    HIPCHK(g, hipEventCreate(&ev.e1));
    // two sweeps, each configuration keeping its faster time (the first
    // launches after the host has been busy run at lower clocks)
    const int shapes[3] = {4, 2, 1}, caps[4] = {0, 24, 20, 16};
    float t_ms[3][4];
    for (int sweep = 0; sweep < 2; ++sweep)
        for (int wi = 0; wi < 3; ++wi)
            for (int ci = 0; ci < 4; ++ci) {
                int rc = lbm_set_launch(g, shapes[wi]);
                if (rc == LBM_OK) rc = lbm_set_occupancy(g, caps[ci]);
                for (int s = 0; rc == LBM_OK && s < 2; ++s) rc = launch_step(g, s & 1, 0);
                if (rc != LBM_OK) return rc;
                HIPCHK(g, hipEventRecord(ev.e0, g->stream));
                for (int s = 0; rc == LBM_OK && s < steps; ++s) rc = launch_step(g, s & 1, 0);
                if (rc != LBM_OK) return rc;
                HIPCHK(g, hipEventRecord(ev.e1, g->stream));
                HIPCHK(g, hipEventSynchronize(ev.e1));
                float ms = 0.f;
                HIPCHK(g, hipEventElapsedTime(&ms, ev.e0, ev.e1));
                t_ms[wi][ci] = sweep == 0 ? ms : std::min(t_ms[wi][ci], ms);
            }
    int best_w = 4, best_c = 0;
    float best_ms = 1e30f;
    for (int wi = 0; wi < 3; ++wi)
        for (int ci = 0; ci < 4; ++ci)
            if (t_ms[wi][ci] < best_ms) {
                best_ms = t_ms[wi][ci];
                best_w = shapes[wi];
                best_c = caps[ci];
            }
    {
        std::lock_guard<std::mutex> lk(g_tuned_mu);
        g_tuned[key] = std::make_pair(best_w, best_c);
    }
    g->inited = false;   // the timing steps ran on whatever state the grid held
    int rc = lbm_set_launch(g, best_w);
    if (rc == LBM_OK) rc = lbm_set_occupancy(g, best_c);
    return rc != LBM_OK ? rc : best_w;
}

int lbm_set_volume(lbm_grid *g, const double *J)
{
    if (!g) return fail(nullptr, LBM_EINVAL, "null grid");
    if (J) {
        for (int c = 0; c < g->ncell; ++c)
            if (!(J[c] > 0.0)) return fail(g, LBM_EINVAL, "volume must be positive");
        HIPCHK(g, hipMemcpyAsync(g->Jused, J, (size_t)g->ncell * 8, hipMemcpyHostToDevice, g->stream));
    } else {
        HIPCHK(g, hipMemcpyAsync(g->Jused, g->Jgeo, (size_t)g->ncell * 8, hipMemcpyDeviceToDevice, g->stream));
    }
    HIPCHK(g, hipStreamSynchronize(g->stream));
    return LBM_OK;
}

static int reduce(lbm_grid *g, int update_snap, double out[RED_NF]);

static int form_lag(lbm_grid *g, int pin)
{
    const dim3 gr = cell_grid(g->n1, g->n2);
    if (g->q == 9) {
        if (g->precision == LBM_FP64) hipLaunchKernelGGL((k_lag<9, double, double>), gr, dim3(128), 0, g->stream, g->d_inst, pin);
        else if (g->precision == LBM_FP16) hipLaunchKernelGGL((k_lag<9, float, _Float16>), gr, dim3(128), 0, g->stream, g->d_inst, pin);
        else hipLaunchKernelGGL((k_lag<9, float, float>), gr, dim3(128), 0, g->stream, g->d_inst, pin);
    } else {
        if (g->precision == LBM_FP64) hipLaunchKernelGGL((k_lag<21, double, double>), gr, dim3(128), 0, g->stream, g->d_inst, pin);
        else if (g->precision == LBM_FP16) hipLaunchKernelGGL((k_lag<21, float, _Float16>), gr, dim3(128), 0, g->stream, g->d_inst, pin);
        else hipLaunchKernelGGL((k_lag<21, float, float>), gr, dim3(128), 0, g->stream, g->d_inst, pin);
    }
    HIPCHK(g, hipGetLastError());
    return LBM_OK;
}

int lbm_init(lbm_grid *g, const double *u0)
{
    if (!g) return fail(nullptr, LBM_EINVAL, "null grid");
    double *du = nullptr;
    if (u0) {
        du = (double *)dalloc(g, (size_t)g->ncell * 2 * 8);
        if (!du) return fail(g, LBM_ENOMEM, "allocation failed");
        HIPCHK(g, hipMemcpyAsync(du, u0, (size_t)g->ncell * 2 * 8, hipMemcpyHostToDevice, g->stream));
    }
    g->par = 0;
    g->step = 0;
    InitArgs ia{g->G3, g->Jused, du, g->base, g->desc.rho0, !g->row, 0};
    const dim3 gr = cell_grid(g->n1, g->n2);
    if (g->q == 9) {
        if (g->precision == LBM_FP64) hipLaunchKernelGGL((k_init<9, double, double>), gr, dim3(128), 0, g->stream, g->d_inst, ia);
        else if (g->precision == LBM_FP16) hipLaunchKernelGGL((k_init<9, float, _Float16>), gr, dim3(128), 0, g->stream, g->d_inst, ia);
        else hipLaunchKernelGGL((k_init<9, float, float>), gr, dim3(128), 0, g->stream, g->d_inst, ia);
    } else {
        if (g->precision == LBM_FP64) hipLaunchKernelGGL((k_init<21, double, double>), gr, dim3(128), 0, g->stream, g->d_inst, ia);
        else if (g->precision == LBM_FP16) hipLaunchKernelGGL((k_init<21, float, _Float16>), gr, dim3(128), 0, g->stream, g->d_inst, ia);
        else hipLaunchKernelGGL((k_init<21, float, float>), gr, dim3(128), 0, g->stream, g->d_inst, ia);
    }
    HIPCHK(g, hipGetLastError());
    {
        const int rc = form_lag(g, 0);
        if (rc != LBM_OK) return rc;
    }
    HIPCHK(g, hipStreamSynchronize(g->stream));
    if (du) dfree(g, du);
    g->inited = true;
    g->snap_valid = false;
    double r[RED_NF];
    int rc = reduce(g, 1, r);
    if (rc != LBM_OK) return rc;
    g->mass0 = r[0];
    g->snap_valid = true;
    g->snap_step = 0;
    return LBM_OK;
}

static int capture_graph(lbm_grid *g, int start_par, int steps)
{
    GraphCache &gc = g->graph[start_par];
    if (gc.exec && gc.steps == steps) return LBM_OK;
    if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
    gc.exec = nullptr;
    hipGraph_t graph = nullptr;
    HIPCHK(g, hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
    int par = start_par;
    for (int s = 0; s < steps; ++s) {
        StepFn fn = pick_step(g->q, g->precision, g->ct, 0, g->h_inst.iters > 0, g->wide);
        hipLaunchKernelGGL(fn, dim3(g->ntiles), dim3(64 * g->wpb), step_lds(g->ct, g->q, g->precision, g->cap, g->wpb), g->stream, (const InstDesc *)g->d_inst,
                           (const int4 *)g->d_tiles, par);
        par ^= 1;
    }
    HIPCHK(g, hipStreamEndCapture(g->stream, &graph));
    HIPCHK(g, hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0));
    (void)hipGraphDestroy(graph);
    gc.steps = steps;
    return LBM_OK;
}

int lbm_step(lbm_grid *g, int64_t n)
{
    if (!g) return fail(nullptr, LBM_EINVAL, "null grid");
    if (!g->inited) return fail(g, LBM_ESTATE, "lbm_init must be called before lbm_step");
    if (n < 0) return fail(g, LBM_EINVAL, "negative step count");
    const int GS = 32;   // steps per captured graph (even: the buffer parity returns)
    if (n >= GS) {
        int rc = capture_graph(g, g->par, GS);
        if (rc != LBM_OK) return rc;
        const int64_t reps = n / GS;
        for (int64_t k = 0; k < reps; ++k) HIPCHK(g, hipGraphLaunch(g->graph[g->par].exec, g->stream));
        g->step += reps * GS;
        n -= reps * GS;
    }
    for (int64_t k = 0; k < n; ++k) {
        int rc = launch_step(g, g->par, 0);
        if (rc != LBM_OK) return rc;
        g->par ^= 1;
        g->step += 1;
    }
    return LBM_OK;
}

static int run_moments(lbm_grid *g) { return launch_step(g, g->par, 1); }

static int launch_reduce(lbm_grid *g, int update_snap, double *dst)
{
    int rc = run_moments(g);
    if (rc != LBM_OK) return rc;
    ReduceArgs ra{g->mom, g->snap, g->g4, g->xc, g->yc, g->ncell, update_snap, g->partial};
    hipLaunchKernelGGL(k_reduce, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, g->stream, ra);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64), 0, g->stream, (const double *)g->partial, dst);
    HIPCHK(g, hipGetLastError());
    return LBM_OK;
}

static int reduce(lbm_grid *g, int update_snap, double out[RED_NF])
{
    int rc = launch_reduce(g, update_snap, g->redout);
    if (rc != LBM_OK) return rc;
    HIPCHK(g, hipMemcpyAsync(out, g->redout, RED_NF * 8, hipMemcpyDeviceToHost, g->stream));
    HIPCHK(g, hipStreamSynchronize(g->stream));
    return LBM_OK;
}

// residual record from the reduced sums; advances the residual reference
static int fill_resid(lbm_grid *g, const double r[RED_NF], lbm_resid *out)
{
    const int64_t K = g->step - g->snap_step;
    out->step = g->step;
    out->mass = r[0];
    out->mass_rel_drift = g->mass0 != 0.0 ? (r[0] - g->mass0) / g->mass0 : 0.0;
    out->residual = (g->snap_valid && K > 0 && r[2] > 0.0) ? std::sqrt(r[1]) / ((double)K * std::sqrt(r[2]))
                                                            : INFINITY;
    out->kinetic_energy = r[3];
    out->angular_momentum = r[4];
    out->bad_cells = (int64_t)r[5];
    g->snap_valid = true;
    g->snap_step = g->step;
    if (out->bad_cells > 0) return fail(g, LBM_EUNSTABLE, "non-finite values or m <= 0 in some cells");
    return LBM_OK;
}

int lbm_residual(lbm_grid *g, lbm_resid *out)
{
    if (!g || !out) return fail(g, LBM_EINVAL, "null argument");
    if (!g->inited) return fail(g, LBM_ESTATE, "lbm_init must be called first");
    double r[RED_NF];
    int rc = reduce(g, 1, r);
    if (rc != LBM_OK) return rc;
    return fill_resid(g, r, out);
}

int lbm_moments(lbm_grid *g, double *m, double *U, double *Ut)
{
    if (!g) return fail(nullptr, LBM_EINVAL, "null grid");
    if (!g->inited) return fail(g, LBM_ESTATE, "lbm_init must be called first");
    int rc = run_moments(g);
    if (rc != LBM_OK) return rc;
    const size_t nc = g->ncell;
    std::vector<double> h(nc * 5);
    HIPCHK(g, hipMemcpyAsync(h.data(), g->mom, nc * 5 * 8, hipMemcpyDeviceToHost, g->stream));
    HIPCHK(g, hipStreamSynchronize(g->stream));
    for (size_t c = 0; c < nc; ++c) {
        if (m) m[c] = h[c];
        if (U) {
            U[2 * c] = h[nc + c];
            U[2 * c + 1] = h[2 * nc + c];
        }
        if (Ut) {
            Ut[2 * c] = h[3 * nc + c];
            Ut[2 * c + 1] = h[4 * nc + c];
        }
    }
    return LBM_OK;
}

int lbm_physical_velocity(lbm_grid *g, double *u)
{
    if (!g || !u) return fail(g, LBM_EINVAL, "null argument");
    if (!g->inited) return fail(g, LBM_ESTATE, "lbm_init must be called first");
    int rc = run_moments(g);
    if (rc != LBM_OK) return rc;
    const size_t nc = g->ncell;
    double *d = (double *)dalloc(g, nc * 2 * 8);
    if (!d) return fail(g, LBM_ENOMEM, "allocation failed");
    hipLaunchKernelGGL(k_physical_velocity, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, g->stream, g->mom, g->g4,
                       (int)nc, d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(u, d, nc * 2 * 8, hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    dfree(g, d);
    if (e != hipSuccess) return fail(g, LBM_EDEVICE, std::string("physical velocity: ") + hipGetErrorString(e));
    return LBM_OK;
}

namespace {
// checkpoint blob: header, then P[q][n1][n2] and side[2][2][c_max][n2] (FP64)
struct CkptHeader {
    char magic[8];
    int32_t q, n1, n2, precision;
    int64_t step;
    double mass0;        // mass at lbm_init (drift reference)
    int64_t nP, nside;
};
const char CKPT_MAGIC[8] = {'L', 'B', 'M', 'C', 'K', 'P', 'T', '1'};
} // namespace

static size_t ckpt_counts(const lbm_grid *g, int64_t *nP, int64_t *nside)
{
    *nP = (int64_t)g->q * g->ncell;
    *nside = (int64_t)4 * g->hw * g->n2;
    return sizeof(CkptHeader) + (size_t)(*nP + *nside) * sizeof(double);
}

int lbm_save(lbm_grid *g, void *buf, size_t *len)
{
    if (!g || !len) return fail(g, LBM_EINVAL, "null argument");
    int64_t nP, ns;
    const size_t need = ckpt_counts(g, &nP, &ns);
    if (!buf) {
        *len = need;
        return LBM_OK;
    }
    if (*len < need) return fail(g, LBM_EINVAL, "checkpoint buffer too small");
    if (!g->inited) return fail(g, LBM_ESTATE, "lbm_init must be called first");
    CkptHeader h{};
    std::memcpy(h.magic, CKPT_MAGIC, 8);
    h.q = g->q;
    h.n1 = g->n1;
    h.n2 = g->n2;
    h.precision = g->precision;
    h.step = g->step;
    h.mass0 = g->mass0;
    h.nP = nP;
    h.nside = ns;
    std::memcpy(buf, &h, sizeof h);
    double *P = (double *)((char *)buf + sizeof h);
    const int rc = lbm_get_state(g, P, P + nP);
    if (rc != LBM_OK) return rc;
    *len = need;
    return LBM_OK;
}

int lbm_load(lbm_grid *g, const void *buf, size_t len)
{
    if (!g || !buf) return fail(g, LBM_EINVAL, "null argument");
    int64_t nP, ns;
    const size_t need = ckpt_counts(g, &nP, &ns);
    CkptHeader h{};
    if (len < sizeof h) return fail(g, LBM_EINVAL, "checkpoint too short");
    std::memcpy(&h, buf, sizeof h);
    if (std::memcmp(h.magic, CKPT_MAGIC, 8) != 0) return fail(g, LBM_EINVAL, "not a checkpoint of this library");
    if (h.q != g->q || h.n1 != g->n1 || h.n2 != g->n2 || h.nP != nP || h.nside != ns)
        return fail(g, LBM_EINVAL, "checkpoint lattice or grid shape differs from the grid's");
    if (len < need) return fail(g, LBM_EINVAL, "checkpoint truncated");
    const double *P = (const double *)((const char *)buf + sizeof h);
    int rc = lbm_set_state(g, P, P + nP);
    if (rc != LBM_OK) return rc;
    g->step = h.step;
    // residual snapshot at the restored step; drift keeps the writer's reference
    double r[RED_NF];
    rc = reduce(g, 1, r);
    if (rc != LBM_OK) return rc;
    g->mass0 = h.mass0 > 0.0 ? h.mass0 : r[0];
    g->snap_valid = true;
    g->snap_step = g->step;
    return LBM_OK;
}

int lbm_noflow_adjust(lbm_grid *g, double tol, int64_t max_steps, int32_t check_every, int64_t *steps_out)
{
    if (!g) return fail(nullptr, LBM_EINVAL, "null grid");
    if (check_every <= 0 || max_steps <= 0 || !(tol > 0)) return fail(g, LBM_EINVAL, "bad no-flow parameters");
    const InstDesc saved = g->h_inst;
    g->h_inst.ut_lo = g->h_inst.ut_hi = 0.0;
    g->h_inst.a1 = g->h_inst.a2 = 0.0;
    int rc = upload_inst(g);
    if (rc == LBM_OK) rc = lbm_set_volume(g, nullptr);
    if (rc == LBM_OK) rc = lbm_init(g, nullptr);
    int64_t done = 0;
    lbm_resid res{};
    while (rc == LBM_OK && done < max_steps) {
        rc = lbm_step(g, check_every);
        done += check_every;
        if (rc == LBM_OK) rc = lbm_residual(g, &res);
        if (rc == LBM_OK && res.residual < tol) break;
    }
    if (rc == LBM_OK) {
        rc = run_moments(g);
        if (rc == LBM_OK) {
            hipLaunchKernelGGL(k_volume_from_mass, dim3((g->ncell + 255) / 256), dim3(256), 0, g->stream,
                               (const double *)g->mom, g->desc.rho0, g->ncell, g->Jused);
            if (hipGetLastError() != hipSuccess) rc = fail(g, LBM_EDEVICE, "volume kernel failed");
        }
    }
    g->h_inst = saved;
    const int rc2 = upload_inst(g);
    if (hipStreamSynchronize(g->stream) != hipSuccess && rc == LBM_OK) rc = fail(g, LBM_EDEVICE, "sync failed");
    g->inited = false;
    if (steps_out) *steps_out = done;
    return rc != LBM_OK ? rc : rc2;
}

// rows row0 .. row0 + rows - 1 of the FP64 state into dst [Q][rows][n2] (device)
static int launch_state_out(lbm_grid *g, int row0, int rows, double *dst)
{
    const dim3 gr((g->n2 + 127) / 128, rows);
    if (g->q == 9) {
        if (g->precision == LBM_FP64) hipLaunchKernelGGL((k_state_out<9, double>), gr, dim3(128), 0, g->stream, g->d_inst, g->base, !g->row, g->par, row0, dst);
        else if (g->precision == LBM_FP16) hipLaunchKernelGGL((k_state_out<9, _Float16>), gr, dim3(128), 0, g->stream, g->d_inst, g->base, !g->row, g->par, row0, dst);
        else hipLaunchKernelGGL((k_state_out<9, float>), gr, dim3(128), 0, g->stream, g->d_inst, g->base, !g->row, g->par, row0, dst);
    } else {
        if (g->precision == LBM_FP64) hipLaunchKernelGGL((k_state_out<21, double>), gr, dim3(128), 0, g->stream, g->d_inst, g->base, !g->row, g->par, row0, dst);
        else if (g->precision == LBM_FP16) hipLaunchKernelGGL((k_state_out<21, _Float16>), gr, dim3(128), 0, g->stream, g->d_inst, g->base, !g->row, g->par, row0, dst);
        else hipLaunchKernelGGL((k_state_out<21, float>), gr, dim3(128), 0, g->stream, g->d_inst, g->base, !g->row, g->par, row0, dst);
    }
    HIPCHK(g, hipGetLastError());
    return LBM_OK;
}

// the moving-wall side state into dst [2][2][hw][n2] (device)
static int launch_side_out(lbm_grid *g, double *dst)
{
    const dim3 sg((g->n2 + 127) / 128, 4 * g->hw);
    if (g->precision == LBM_FP64) hipLaunchKernelGGL(k_side_io<double>, sg, dim3(128), 0, g->stream, g->d_inst, g->par, dst, 0);
    else hipLaunchKernelGGL(k_side_io<float>, sg, dim3(128), 0, g->stream, g->d_inst, g->par, dst, 0);
    HIPCHK(g, hipGetLastError());
    return LBM_OK;
}

int lbm_get_state(lbm_grid *g, double *P, double *side)
{
    if (!g) return fail(nullptr, LBM_EINVAL, "null grid");
    if (P) {
        double *tmp = (double *)dalloc(g, (size_t)g->ncell * g->q * 8);
        if (!tmp) return fail(g, LBM_ENOMEM, "allocation failed");
        int rc = launch_state_out(g, 0, g->n1, tmp);
        if (rc != LBM_OK) return rc;
        HIPCHK(g, hipMemcpyAsync(P, tmp, (size_t)g->ncell * g->q * 8, hipMemcpyDeviceToHost, g->stream));
        HIPCHK(g, hipStreamSynchronize(g->stream));
        dfree(g, tmp);
    }
    if (side) {
        const size_t ns = (size_t)4 * g->hw * g->n2;
        double *tmp = (double *)dalloc(g, ns * 8);
        if (!tmp) return fail(g, LBM_ENOMEM, "allocation failed");
        int rc = launch_side_out(g, tmp);
        if (rc != LBM_OK) return rc;
        HIPCHK(g, hipMemcpyAsync(side, tmp, ns * 8, hipMemcpyDeviceToHost, g->stream));
        HIPCHK(g, hipStreamSynchronize(g->stream));
        dfree(g, tmp);
    }
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free state export.  The FP64 state is staged through `scratch`,
// a fixed device array of LBM_NOALLOC_STAGING_BYTES that every GPU the library
// runs on holds until the process ends, in chunks of whole rows.  In host
// code `scratch` names a host-side stand-in, never the device array: its
// device address comes from hipGetSymbolAddress, taken once per device with
// that device current and kept in g_scratch_dev.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[LBM_NOALLOC_STAGING_BYTES / sizeof(double)];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;              // guards g_scratch_dev and serialises the staging
double *g_scratch_dev[MAX_DEVICES] = {};
} // namespace

// device address of `scratch` on device `dev` (with `dev` current)
static int scratch_address(lbm_grid *g, int dev, double **out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return fail(g, LBM_EDEVICE, "device index out of range");
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HIPCHK(g, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(g, LBM_EDEVICE, "hipGetSymbolAddress returned no address for the staging array");
        g_scratch_dev[dev] = (double *)p;
    }
    *out = g_scratch_dev[dev];
    return LBM_OK;
}

int lbm_get_state_noalloc(lbm_grid *g, double *P, double *side)
{
    if (!g) return fail(nullptr, LBM_EINVAL, "null grid");
    const size_t row_bytes = (size_t)g->q * g->n2 * sizeof(double);
    const size_t side_bytes = (size_t)4 * g->hw * g->n2 * sizeof(double);
    if (P && row_bytes > LBM_NOALLOC_STAGING_BYTES)
        return fail(g, LBM_EINVAL, "lbm_get_state_noalloc: one row of the state (" + std::to_string(row_bytes) +
                                       " bytes) exceeds the staging buffer (" +
                                       std::to_string((size_t)LBM_NOALLOC_STAGING_BYTES) + " bytes)");
    if (side && side_bytes > LBM_NOALLOC_STAGING_BYTES)
        return fail(g, LBM_EINVAL, "lbm_get_state_noalloc: the side state (" + std::to_string(side_bytes) +
                                       " bytes) exceeds the staging buffer");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    int cur = -1;
    HIPCHK(g, hipGetDevice(&cur));
    if (cur != g->device) HIPCHK(g, hipSetDevice(g->device));
    struct Restore {   // the caller's current device, on every return path
        int dev, was;
        ~Restore()
        {
            if (dev != was) (void)hipSetDevice(was);
        }
    } restore{g->device, cur};
    double *buf = nullptr;
    int rc = scratch_address(g, g->device, &buf);
    if (rc != LBM_OK) return rc;
    if (P) {
        // whole rows per chunk; each chunk's copy is ordered on the stream
        // before the next chunk's kernel overwrites the staging array
        const int rows = (int)std::min<size_t>((size_t)g->n1, LBM_NOALLOC_STAGING_BYTES / row_bytes);
        for (int r0 = 0; r0 < g->n1; r0 += rows) {
            const int nr = std::min(rows, g->n1 - r0);
            rc = launch_state_out(g, r0, nr, buf);
            if (rc != LBM_OK) return rc;
            const size_t w = (size_t)nr * g->n2 * sizeof(double);
            HIPCHK(g, hipMemcpy2DAsync(P + (size_t)r0 * g->n2, (size_t)g->ncell * sizeof(double), buf, w, w, g->q,
                                       hipMemcpyDeviceToHost, g->stream));
        }
    }
    if (side) {
        rc = launch_side_out(g, buf);
        if (rc != LBM_OK) return rc;
        HIPCHK(g, hipMemcpyAsync(side, buf, side_bytes, hipMemcpyDeviceToHost, g->stream));
    }
    HIPCHK(g, hipStreamSynchronize(g->stream));
    return LBM_OK;
}

int lbm_set_state(lbm_grid *g, const double *P, const double *side)
{
    if (!g) return fail(nullptr, LBM_EINVAL, "null grid");
    const dim3 gr = cell_grid(g->n1, g->n2);
    if (P) {
        double *tmp = (double *)dalloc(g, (size_t)g->ncell * g->q * 8);
        if (!tmp) return fail(g, LBM_ENOMEM, "allocation failed");
        HIPCHK(g, hipMemcpyAsync(tmp, P, (size_t)g->ncell * g->q * 8, hipMemcpyHostToDevice, g->stream));
        if (g->q == 9) {
            if (g->precision == LBM_FP64) hipLaunchKernelGGL((k_state_in<9, double>), gr, dim3(128), 0, g->stream, g->d_inst, g->base, !g->row, g->par, tmp);
            else if (g->precision == LBM_FP16) hipLaunchKernelGGL((k_state_in<9, _Float16>), gr, dim3(128), 0, g->stream, g->d_inst, g->base, !g->row, g->par, tmp);
            else hipLaunchKernelGGL((k_state_in<9, float>), gr, dim3(128), 0, g->stream, g->d_inst, g->base, !g->row, g->par, tmp);
        } else {
            if (g->precision == LBM_FP64) hipLaunchKernelGGL((k_state_in<21, double>), gr, dim3(128), 0, g->stream, g->d_inst, g->base, !g->row, g->par, tmp);
            else if (g->precision == LBM_FP16) hipLaunchKernelGGL((k_state_in<21, _Float16>), gr, dim3(128), 0, g->stream, g->d_inst, g->base, !g->row, g->par, tmp);
            else hipLaunchKernelGGL((k_state_in<21, float>), gr, dim3(128), 0, g->stream, g->d_inst, g->base, !g->row, g->par, tmp);
        }
        HIPCHK(g, hipGetLastError());
        const int rc = form_lag(g, g->par);
        if (rc != LBM_OK) return rc;
        HIPCHK(g, hipStreamSynchronize(g->stream));
        dfree(g, tmp);
    }
    if (side) {
        const size_t ns = (size_t)4 * g->hw * g->n2;
        double *tmp = (double *)dalloc(g, ns * 8);
        if (!tmp) return fail(g, LBM_ENOMEM, "allocation failed");
        HIPCHK(g, hipMemcpyAsync(tmp, side, ns * 8, hipMemcpyHostToDevice, g->stream));
        const dim3 sg((g->n2 + 127) / 128, 4 * g->hw);
        if (g->precision == LBM_FP64) hipLaunchKernelGGL(k_side_io<double>, sg, dim3(128), 0, g->stream, g->d_inst, g->par, tmp, 1);
        else hipLaunchKernelGGL(k_side_io<float>, sg, dim3(128), 0, g->stream, g->d_inst, g->par, tmp, 1);
        HIPCHK(g, hipGetLastError());
        HIPCHK(g, hipStreamSynchronize(g->stream));
        dfree(g, tmp);
    }
    g->inited = true;
    return LBM_OK;
}

int lbm_stream_map(lbm_grid *g, int32_t *src_cell, int32_t *src_dir, int32_t *wall)
{
    if (!g || !src_cell || !src_dir || !wall) return fail(g, LBM_EINVAL, "null argument");
    const size_t n = (size_t)g->ncell * g->q;
    int *t = (int *)dalloc(g, n * 3 * sizeof(int));
    if (!t) return fail(g, LBM_ENOMEM, "allocation failed");
    const dim3 gr = cell_grid(g->n1, g->n2);
    if (g->q == 9) hipLaunchKernelGGL(k_stream_map<9>, gr, dim3(128), 0, g->stream, g->d_inst, t, t + n, t + 2 * n);
    else hipLaunchKernelGGL(k_stream_map<21>, gr, dim3(128), 0, g->stream, g->d_inst, t, t + n, t + 2 * n);
    HIPCHK(g, hipGetLastError());
    HIPCHK(g, hipMemcpyAsync(src_cell, t, n * 4, hipMemcpyDeviceToHost, g->stream));
    HIPCHK(g, hipMemcpyAsync(src_dir, t + n, n * 4, hipMemcpyDeviceToHost, g->stream));
    HIPCHK(g, hipMemcpyAsync(wall, t + 2 * n, n * 4, hipMemcpyDeviceToHost, g->stream));
    HIPCHK(g, hipStreamSynchronize(g->stream));
    dfree(g, t);
    return LBM_OK;
}

int lbm_geometry(lbm_grid *g, double *out)
{
    if (!g || !out) return fail(g, LBM_EINVAL, "null argument");
    const int q = g->q, n1 = g->n1, n2 = g->n2, h = g->h, nc = g->ncell;
    const int H1 = n1 + 2 * h, H2 = n2 + 2 * h;
    const size_t nh = (size_t)H1 * H2;
    const int nf = geo_fields(q);
    double *tg = (double *)dalloc(g, nh * 4 * 8);
    double *geo = (double *)dalloc(g, (size_t)nc * nf * 8);
    double *jt = (double *)dalloc(g, (size_t)nc * 8);
    double *g4t = (double *)dalloc(g, (size_t)nc * 4 * 8);
    if (!tg || !geo || !jt || !g4t) return fail(g, LBM_ENOMEM, "allocation failed");
    hipLaunchKernelGGL(k_tangent, dim3((H2 + 127) / 128, H1), dim3(128), 0, g->stream, g->X, g->Y, H1, H2, tg);
    if (q == 9) hipLaunchKernelGGL(k_geom_cell<9>, cell_grid(n1, n2), dim3(128), 0, g->stream, tg, n1, n2, h, geo, jt, g4t);
    else hipLaunchKernelGGL(k_geom_cell<21>, cell_grid(n1, n2), dim3(128), 0, g->stream, tg, n1, n2, h, geo, jt, g4t);
    HIPCHK(g, hipGetLastError());
    std::vector<double> hg((size_t)nc * nf);
    HIPCHK(g, hipMemcpyAsync(hg.data(), geo, hg.size() * 8, hipMemcpyDeviceToHost, g->stream));
    HIPCHK(g, hipStreamSynchronize(g->stream));
    dfree(g, tg);
    dfree(g, geo);
    dfree(g, jt);
    dfree(g, g4t);
    const int W = 4 + 2 * q;
    for (int c = 0; c < nc; ++c) {
        out[(size_t)c * W + 0] = hg[(size_t)GEO_J * nc + c];
        out[(size_t)c * W + 1] = hg[(size_t)GEO_G11 * nc + c];
        out[(size_t)c * W + 2] = hg[(size_t)GEO_G12 * nc + c];
        out[(size_t)c * W + 3] = hg[(size_t)GEO_G22 * nc + c];
        for (int k = 0; k < 2 * q; ++k) out[(size_t)c * W + 4 + k] = hg[(size_t)(GEO_A0 + k) * nc + c];
    }
    return LBM_OK;
}

int lbm_get_volume(lbm_grid *g, double *J)
{
    if (!g || !J) return fail(g, LBM_EINVAL, "null argument");
    HIPCHK(g, hipMemcpyAsync(J, g->Jused, (size_t)g->ncell * 8, hipMemcpyDeviceToHost, g->stream));
    HIPCHK(g, hipStreamSynchronize(g->stream));
    return LBM_OK;
}

int lbm_synchronize(lbm_grid *g)
{
    if (!g) return fail(nullptr, LBM_EINVAL, "null grid");
    HIPCHK(g, hipStreamSynchronize(g->stream));
    return LBM_OK;
}

void *lbm_stream(lbm_grid *g) { return g ? (void *)g->stream : nullptr; }

int lbm_grid_set_stream(lbm_grid *g, void *stream)
{
    if (!g) return fail(nullptr, LBM_EINVAL, "null grid");
    if (!g->batches.empty()) return fail(g, LBM_ESTATE, "a grid held by a batch keeps its stream");
    hipStream_t s = (hipStream_t)stream;
    if (s && s == g->stream) return LBM_OK;
    bool own = false;
    if (!s) {
        if (hipStreamCreate(&s) != hipSuccess) return fail(g, LBM_EDEVICE, "hipStreamCreate failed");
        own = true;
    }
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess || hipEventRecord(ev, g->stream) != hipSuccess ||
        hipStreamWaitEvent(s, ev, 0) != hipSuccess) {
        if (ev) (void)hipEventDestroy(ev);
        if (own) (void)hipStreamDestroy(s);
        return fail(g, LBM_EDEVICE, "stream handover failed");
    }
    (void)hipEventDestroy(ev);
    if (g->own_stream) (void)hipStreamDestroy(g->stream);
    g->stream = s;
    g->own_stream = own;
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
static void batch_drop_graph(lbm_batch *b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->gtmpl) (void)hipGraphDestroy(b->gtmpl);
    b->gexec = nullptr;
    b->gtmpl = nullptr;
    b->nodes.clear();
}

void lbm_batch_destroy(lbm_batch *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (hipStream_t s : b->others) (void)hipStreamSynchronize(s);
    batch_drop_graph(b);
    for (void *p : b->allocs) (void)hipFree(p);
    if (b->ev) (void)hipEventDestroy(b->ev);
    for (lbm_grid *g : b->grids)
        if (g) g->batches.erase(std::remove(g->batches.begin(), g->batches.end(), b), g->batches.end());
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

static int batch_usable(const lbm_batch *b)
{
    if (!b) return fail(nullptr, LBM_EINVAL, "null batch");
    if (b->broken) return fail(nullptr, LBM_ESTATE, "a grid of this batch was destroyed before the batch");
    return LBM_OK;
}

static void batch_free(lbm_batch *b, void *p)
{
    auto it = std::find(b->allocs.begin(), b->allocs.end(), p);
    if (it != b->allocs.end()) b->allocs.erase(it);
    (void)hipFree(p);
}

// Copy `count` entries of `each` bytes into the device array *d holding *cap
// entries; a larger count replaces the array by one of at least twice the
// capacity (so a changing membership reallocates rarely).
static int upload_grow(lbm_batch *b, void **d, int *cap, const void *src, size_t count, size_t each)
{
    if (!*d || count > (size_t)*cap) {
        const size_t nc = std::max<size_t>(std::max<size_t>(count, 1), 2 * (size_t)*cap);
        void *p = nullptr;
        if (hipMalloc(&p, nc * each) != hipSuccess) return fail(nullptr, LBM_ENOMEM, "batch allocation failed");
        b->allocs.push_back(p);
        if (*d) batch_free(b, *d);
        *d = p;
        *cap = (int)nc;
    }
    if (count && hipMemcpy(*d, src, count * each, hipMemcpyHostToDevice) != hipSuccess)
        return fail(nullptr, LBM_EDEVICE, "batch upload failed");
    return LBM_OK;
}

// Tile list of a batch group for `wpb` rows per workgroup: the members' tiles
// (instance = position in the group) in the XCD-run order.  Instances stay
// contiguous, so each XCD works on few grids.
static std::vector<int4> group_tile_list(const lbm_batch *b, const std::vector<int> &members, int wpb)
{
    std::vector<int4> nat;
    int inst = 0;
    for (int k : members) {
        const lbm_grid *g = b->grids[k];
        auto t = make_tiles(inst++, g->n1, g->n2, wpb, g->q);
        nat.insert(nat.end(), t.begin(), t.end());
    }
    return xcd_order(nat, 1 << 30);
}

// the same, uploaded to a new device allocation the batch owns
static int group_tiles(lbm_batch *b, const std::vector<int> &members, int wpb, int4 **d_out, int *nt_out, int *cap_out)
{
    const auto ord = group_tile_list(b, members, wpb);
    void *dt = nullptr;
    int cap = 0;
    const int rc = upload_grow(b, &dt, &cap, ord.data(), ord.size(), sizeof(int4));
    if (rc != LBM_OK) return rc;
    *d_out = (int4 *)dt;
    *nt_out = (int)ord.size();
    *cap_out = cap;
    return LBM_OK;
}

static bool same_kernel(const lbm_batch::Group &a, const lbm_batch::Group &c)
{
    return a.q == c.q && a.precision == c.precision && a.cell == c.cell && a.iter == c.iter && a.wide == c.wide;
}

// Group the batch's grids by step kernel (lattice, or 0 for a fused group
// holding both; storage precision; table kind; fixed-point force passes; wide
// addressing) and upload each group's instance descriptors and tile table.
// A group whose kernel was there before keeps its device arrays (rewritten in
// place, grown when too small) and its tuned launch shape.
static int batch_regroup(lbm_batch *b)
{
    const bool fuse = (b->flags & LBM_BATCH_FUSE_LATTICES) != 0;
    std::map<std::tuple<int, int, int, int, int>, std::vector<int>> keyed;
    for (int k = 0; k < (int)b->grids.size(); ++k) {
        const lbm_grid *g = b->grids[k];
        // wide grids keep their lattice's kernel (the fused one addresses whole buffers)
        keyed[std::make_tuple(fuse && !g->wide ? 0 : g->q, g->precision, g->ct, g->h_inst.iters > 0 ? 1 : 0, g->wide)]
            .push_back(k);
    }
    std::vector<lbm_batch::Group> old;
    old.swap(b->groups);
    std::vector<bool> kept(old.size(), false);
    int rc = LBM_OK;
    for (auto &kv : keyed) {
        lbm_batch::Group G;
        // a fused group with a single lattice keeps that lattice's kernel
        G.q = b->grids[kv.second[0]]->q;
        for (int k : kv.second)
            if (b->grids[k]->q != G.q) G.q = 0;
        G.precision = std::get<1>(kv.first);
        G.cell = std::get<2>(kv.first);
        G.iter = std::get<3>(kv.first);
        G.wide = std::get<4>(kv.first);
        G.wpb = b->grids[kv.second[0]]->wpb;
        G.cap = b->grids[kv.second[0]]->cap;
        for (size_t o = 0; o < old.size(); ++o)
            if (!kept[o] && same_kernel(old[o], G)) {
                kept[o] = true;
                G.d_inst = old[o].d_inst;
                G.inst_cap = old[o].inst_cap;
                G.d_tiles = old[o].d_tiles;
                G.tile_cap = old[o].tile_cap;
                G.wpb = old[o].wpb;
                G.cap = old[o].cap;
                break;
            }
        G.members = kv.second;
        std::vector<InstDesc> descs;
        for (int k : G.members) {
            const lbm_grid *g = b->grids[k];
            InstDesc I = g->h_inst;
            // step s of the batch runs with par = s & 1; the grid's current buffer is g->par
            I.par0 = g->par ^ (int)(b->step & 1);
            descs.push_back(I);
        }
        const auto tiles = group_tile_list(b, G.members, G.wpb);
        G.ntiles = (int)tiles.size();
        b->groups.push_back(G);
        lbm_batch::Group &H = b->groups.back();
        if ((rc = upload_grow(b, (void **)&H.d_inst, &H.inst_cap, descs.data(), descs.size(), sizeof(InstDesc))) != LBM_OK ||
            (rc = upload_grow(b, (void **)&H.d_tiles, &H.tile_cap, tiles.data(), tiles.size(), sizeof(int4))) != LBM_OK)
            break;
    }
    for (size_t o = 0; o < old.size(); ++o)
        if (!kept[o]) {
            if (old[o].d_inst) batch_free(b, old[o].d_inst);
            if (old[o].d_tiles) batch_free(b, old[o].d_tiles);
        }
    return rc;
}

// kernel node of group gi at batch parity par
static void batch_node_params(const lbm_batch *b, int gi, hipKernelNodeParams &p, void **args)
{
    const auto &G = b->groups[gi];
    p = hipKernelNodeParams{};
    p.func = (void *)pick_step(G.q, G.precision, G.cell, 0, G.iter, G.wide);
    p.gridDim = dim3(G.ntiles);
    p.blockDim = dim3(64 * G.wpb);
    p.sharedMemBytes = step_lds(G.cell, G.q, G.precision, G.cap, G.wpb);
    p.kernelParams = args;
    p.extra = nullptr;
}

static const int BATCH_GS = 16;   // steps per graph launch

// The step graph: BATCH_GS steps, each one kernel node per group, chained.
static int batch_build_graph(lbm_batch *b)
{
    batch_drop_graph(b);
    if (hipGraphCreate(&b->gtmpl, 0) != hipSuccess) return fail(nullptr, LBM_EDEVICE, "graph creation failed");
    hipGraphNode_t prev = nullptr;
    for (int s = 0; s < BATCH_GS; ++s)
        for (int gi = 0; gi < (int)b->groups.size(); ++gi) {
            const InstDesc *a0 = b->groups[gi].d_inst;
            const int4 *a1 = b->groups[gi].d_tiles;
            int a2 = s & 1;
            void *args[3] = {(void *)&a0, (void *)&a1, (void *)&a2};
            hipKernelNodeParams p;
            batch_node_params(b, gi, p, args);
            hipGraphNode_t node = nullptr;
            if (hipGraphAddKernelNode(&node, b->gtmpl, prev ? &prev : nullptr, prev ? 1 : 0, &p) != hipSuccess) {
                batch_drop_graph(b);
                return fail(nullptr, LBM_EDEVICE, "graph node creation failed");
            }
            b->nodes.push_back({node, gi, s & 1});
            prev = node;
        }
    if (hipGraphInstantiate(&b->gexec, b->gtmpl, nullptr, nullptr, 0) != hipSuccess) {
        batch_drop_graph(b);
        return fail(nullptr, LBM_EDEVICE, "graph instantiation failed");
    }
    return LBM_OK;
}

// After a membership change that kept every group's kernel: the nodes of the
// instantiated graph take the new grid sizes and tables in place.  Any
// failure drops the graph (the next step builds a new one).
static void batch_update_graph(lbm_batch *b)
{
    for (const auto &nd : b->nodes) {
        const InstDesc *a0 = b->groups[nd.group].d_inst;
        const int4 *a1 = b->groups[nd.group].d_tiles;
        int a2 = nd.par;
        void *args[3] = {(void *)&a0, (void *)&a1, (void *)&a2};
        hipKernelNodeParams p;
        batch_node_params(b, nd.group, p, args);
        if (hipGraphExecKernelNodeSetParams(b->gexec, nd.node, &p) != hipSuccess) {
            (void)hipGetLastError();
            batch_drop_graph(b);
            return;
        }
    }
}

// Make `grids` the batch's members.  The batch keeps its stream unless that
// stream is owned by a grid that leaves (then it moves, in stream order, to
// the first remaining grid's stream, or to a stream of its own).
static int batch_set_members(lbm_batch *b, lbm_grid *const *grids, int32_t n)
{
    std::vector<lbm_grid *> list;
    for (int k = 0; k < n; ++k) {
        lbm_grid *g = grids[k];
        if (!g || !g->inited) return fail(nullptr, LBM_ESTATE, "every grid of a batch must be initialised");
        if (std::find(list.begin(), list.end(), g) != list.end()) return fail(nullptr, LBM_EINVAL, "a grid appears twice in the batch");
        list.push_back(g);
    }
    bool stream_leaves = false;
    for (lbm_grid *g : b->grids)
        if (g && std::find(list.begin(), list.end(), g) == list.end()) {
            g->batches.erase(std::remove(g->batches.begin(), g->batches.end(), b), g->batches.end());
            if (g->own_stream && g->stream == b->stream) stream_leaves = true;
        }
    if (stream_leaves) {
        hipStream_t ns = nullptr;
        if (!list.empty()) {
            ns = list[0]->stream;
        } else if (hipStreamCreate(&ns) != hipSuccess) {
            b->broken = true;
            return fail(nullptr, LBM_EDEVICE, "hipStreamCreate failed");
        }
        if (hipEventRecord(b->ev, b->stream) != hipSuccess || hipStreamWaitEvent(ns, b->ev, 0) != hipSuccess) {
            b->broken = true;
            return fail(nullptr, LBM_EDEVICE, "stream handover failed");
        }
        if (b->own_stream) (void)hipStreamDestroy(b->stream);
        b->own_stream = list.empty();
        b->stream = ns;
    }
    for (lbm_grid *g : list)
        if (std::find(g->batches.begin(), g->batches.end(), b) == g->batches.end()) g->batches.push_back(b);
    b->grids = list;
    b->others.clear();
    for (lbm_grid *g : list)
        if (g->stream != b->stream && std::find(b->others.begin(), b->others.end(), g->stream) == b->others.end())
            b->others.push_back(g->stream);
    std::vector<lbm_batch::Group> before = b->groups;
    const int rc = batch_regroup(b);
    if (rc != LBM_OK) {
        b->broken = true;
        batch_drop_graph(b);
        return rc;
    }
    bool same = before.size() == b->groups.size();
    for (size_t k = 0; same && k < before.size(); ++k) same = same_kernel(before[k], b->groups[k]);
    if (b->gexec) {
        if (same) batch_update_graph(b);
        else batch_drop_graph(b);
    }
    return LBM_OK;
}

int lbm_batch_create(lbm_grid *const *grids, int32_t n, lbm_batch **out)
{
    return lbm_batch_create_ex(grids, n, 0u, out);
}

int lbm_batch_create_ex(lbm_grid *const *grids, int32_t n, uint32_t flags, lbm_batch **out)
{
    if (!grids || n <= 0 || !out || (flags & ~(uint32_t)LBM_BATCH_FUSE_LATTICES))
        return fail(nullptr, LBM_EINVAL, "bad batch arguments");
    *out = nullptr;
    if (!grids[0]) return fail(nullptr, LBM_ESTATE, "every grid of a batch must be initialised");
    lbm_batch *b = new lbm_batch();
    b->stream = grids[0]->stream;
    b->flags = flags;
    if (hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) != hipSuccess) {
        delete b;
        return fail(nullptr, LBM_EDEVICE, "event creation failed");
    }
    const int rc = batch_set_members(b, grids, n);
    if (rc != LBM_OK) {
        const std::string msg = g_last_error;
        lbm_batch_destroy(b);
        g_last_error = msg;
        return rc;
    }
    *out = b;
    return LBM_OK;
}

int lbm_batch_update(lbm_batch *b, lbm_grid *const *grids, int32_t n)
{
    if (!b || n < 0 || (n > 0 && !grids)) return fail(nullptr, LBM_EINVAL, "bad batch update arguments");
    if (const int u = batch_usable(b)) return u;
    // the tables are rewritten: the steps already queued must be done with them
    if (hipStreamSynchronize(b->stream) != hipSuccess) return fail(nullptr, LBM_EDEVICE, "sync failed");
    for (hipStream_t s : b->others)
        if (hipStreamSynchronize(s) != hipSuccess) return fail(nullptr, LBM_EDEVICE, "sync failed");
    return batch_set_members(b, grids, n);
}

// grids on other streams: the batch stream waits for their pending work before
// stepping, and they wait for the batch's steps afterwards
static int batch_join_in(lbm_batch *b)
{
    for (hipStream_t s : b->others) {
        if (hipEventRecord(b->ev, s) != hipSuccess || hipStreamWaitEvent(b->stream, b->ev, 0) != hipSuccess)
            return fail(nullptr, LBM_EDEVICE, "stream join failed");
    }
    return LBM_OK;
}

static int batch_join_out(lbm_batch *b)
{
    if (b->others.empty()) return LBM_OK;
    if (hipEventRecord(b->ev, b->stream) != hipSuccess) return fail(nullptr, LBM_EDEVICE, "event record failed");
    for (hipStream_t s : b->others)
        if (hipStreamWaitEvent(s, b->ev, 0) != hipSuccess) return fail(nullptr, LBM_EDEVICE, "stream join failed");
    return LBM_OK;
}

static int batch_launch(lbm_batch *b, int par)
{
    for (auto &G : b->groups) {
        StepFn fn = pick_step(G.q, G.precision, G.cell, 0, G.iter, G.wide);
        hipLaunchKernelGGL(fn, dim3(G.ntiles), dim3(64 * G.wpb), step_lds(G.cell, G.q, G.precision, G.cap, G.wpb), b->stream, (const InstDesc *)G.d_inst,
                           (const int4 *)G.d_tiles, par);
    }
    if (hipGetLastError() != hipSuccess) return fail(nullptr, LBM_EDEVICE, "batch step launch failed");
    return LBM_OK;
}

int lbm_batch_step(lbm_batch *b, int64_t n)
{
    if (!b || n < 0) return fail(nullptr, LBM_EINVAL, "bad batch step arguments");
    if (const int u = batch_usable(b)) return u;
    if (b->groups.empty()) {            // no members: time passes, nothing to step
        b->step += n;
        return LBM_OK;
    }
    const int GS = BATCH_GS;
    int64_t left = n;
    {
        const int rc = batch_join_in(b);
        if (rc != LBM_OK) return rc;
    }
    // the batch's own parity: step s of the batch uses par = s & 1
    if (left >= GS && (b->step & 1) == 0) {
        if (!b->gexec) {
            const int rc = batch_build_graph(b);
            if (rc != LBM_OK) return rc;
        }
        while (left >= GS) {
            if (hipGraphLaunch(b->gexec, b->stream) != hipSuccess) return fail(nullptr, LBM_EDEVICE, "graph launch failed");
            left -= GS;
            b->step += GS;
        }
    }
    for (; left > 0; --left) {
        int rc = batch_launch(b, (int)(b->step & 1));
        if (rc != LBM_OK) return rc;
        b->step += 1;
    }
    for (lbm_grid *g : b->grids) {
        g->par ^= (int)(n & 1);
        g->step += n;
    }
    return batch_join_out(b);
}

int lbm_batch_residuals(lbm_batch *b, lbm_resid *out)
{
    if (!b || !out) return fail(nullptr, LBM_EINVAL, "null argument");
    if (const int u = batch_usable(b)) return u;
    const size_t n = b->grids.size();
    if (n == 0) return LBM_OK;
    if (!b->d_res || n > b->res_cap) {
        double *p = nullptr;
        const size_t cap = std::max(n, 2 * b->res_cap);
        if (hipMalloc((void **)&p, cap * RED_NF * 8) != hipSuccess) return fail(nullptr, LBM_ENOMEM, "allocation failed");
        b->allocs.push_back(p);
        if (b->d_res) batch_free(b, b->d_res);
        b->d_res = p;
        b->res_cap = cap;
    }
    for (size_t k = 0; k < n; ++k) {
        const int rc = launch_reduce(b->grids[k], 1, b->d_res + k * RED_NF);
        if (rc != LBM_OK) return rc;
    }
    if (hipStreamSynchronize(b->stream) != hipSuccess) return fail(nullptr, LBM_EDEVICE, "sync failed");
    for (hipStream_t s : b->others)
        if (hipStreamSynchronize(s) != hipSuccess) return fail(nullptr, LBM_EDEVICE, "sync failed");
    std::vector<double> h(n * RED_NF);
    if (hipMemcpy(h.data(), b->d_res, n * RED_NF * 8, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(nullptr, LBM_EDEVICE, "copy failed");
    int first = LBM_OK;
    for (size_t k = 0; k < n; ++k) {
        const int rc = fill_resid(b->grids[k], h.data() + k * RED_NF, out + k);
        if (rc != LBM_OK && first == LBM_OK) first = rc;
    }
    return first;
}

int lbm_batch_info(const lbm_batch *b, int32_t group, int32_t *q, int32_t *precision, int64_t *cells)
{
    if (!b) return fail(nullptr, LBM_EINVAL, "null batch");
    if (group < 0 || group >= (int32_t)b->groups.size()) {
        if (q || precision || cells) return fail(nullptr, LBM_EINVAL, "no such group");
        return (int)b->groups.size();   // the count alone (also for an empty batch)
    }
    const auto &G = b->groups[group];
    if (q) *q = G.q;
    if (precision) *precision = G.precision;
    if (cells) {
        int64_t c = 0;
        for (int k : G.members) c += b->grids[k]->ncell;
        *cells = c;
    }
    return (int)b->groups.size();
}

int lbm_batch_step_group(lbm_batch *b, int32_t group, int64_t n)
{
    if (!b || group < 0 || group >= (int32_t)b->groups.size() || n < 0 || (n & 1))
        return fail(nullptr, LBM_EINVAL, "bad group step arguments (n must be even)");
    if (const int u = batch_usable(b)) return u;
    const auto &G = b->groups[group];
    StepFn fn = pick_step(G.q, G.precision, G.cell, 0, G.iter, G.wide);
    for (int64_t k = 0; k < n; ++k)
        hipLaunchKernelGGL(fn, dim3(G.ntiles), dim3(64 * G.wpb), step_lds(G.cell, G.q, G.precision, G.cap, G.wpb), b->stream, (const InstDesc *)G.d_inst,
                           (const int4 *)G.d_tiles, (int)((b->step + k) & 1));
    if (hipGetLastError() != hipSuccess) return fail(nullptr, LBM_EDEVICE, "group step launch failed");
    return LBM_OK;
}

int lbm_batch_autotune(lbm_batch *b, int32_t steps)
{
    if (const int u = batch_usable(b)) return u;
    if (steps < 2) steps = 2;
    steps += steps & 1;                 // even, so every trial keeps the buffer parity
    const int64_t per_trial = 2 + (int64_t)steps;
    int rc = batch_join_in(b);
    if (rc != LBM_OK) return rc;
    struct Events {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Events()
        {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } ev;
    if (hipEventCreate(&ev.e0) != hipSuccess || hipEventCreate(&ev.e1) != hipSuccess)
        return fail(nullptr, LBM_EDEVICE, "event creation failed");
    const int shapes[3] = {4, 2, 1}, caps[4] = {0, 24, 20, 16};
    int64_t advanced = 0;
    for (auto &G : b->groups) {
        int4 *tiles[3] = {nullptr, nullptr, nullptr};
        int nts[3] = {0, 0, 0}, tcaps[3] = {0, 0, 0};
        for (int s = 0; s < 3; ++s) {
            if (shapes[s] == G.wpb) {
                tiles[s] = G.d_tiles;
                nts[s] = G.ntiles;
                tcaps[s] = G.tile_cap;
            } else if ((rc = group_tiles(b, G.members, shapes[s], &tiles[s], &nts[s], &tcaps[s])) != LBM_OK) {
                return rc;
            }
        }
        StepFn fn = pick_step(G.q, G.precision, G.cell, 0, G.iter, G.wide);
        // two sweeps over the 12 configurations, each keeping its faster
        // time: the first launches after the host has been busy run at lower
        // clocks, which alone made the first configuration lose
        float t_ms[3][4];
        int64_t k = b->step;            // this group's grids are at the batch's time level
        for (int sweep = 0; sweep < 2; ++sweep)
            for (int s = 0; s < 3; ++s)
                for (int ci = 0; ci < 4; ++ci) {
                    const unsigned lds = step_lds(G.cell, G.q, G.precision, caps[ci], shapes[s]);
                    for (int64_t t = 0; t < per_trial; ++t, ++k) {
                        if (t == 2 && hipEventRecord(ev.e0, b->stream) != hipSuccess)
                            return fail(nullptr, LBM_EDEVICE, "event record failed");
                        hipLaunchKernelGGL(fn, dim3(nts[s]), dim3(64 * shapes[s]), lds, b->stream,
                                           (const InstDesc *)G.d_inst, (const int4 *)tiles[s], (int)(k & 1));
                    }
                    if (hipGetLastError() != hipSuccess) return fail(nullptr, LBM_EDEVICE, "trial launch failed");
                    float ms = 0.f;
                    if (hipEventRecord(ev.e1, b->stream) != hipSuccess || hipEventSynchronize(ev.e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, ev.e0, ev.e1) != hipSuccess)
                        return fail(nullptr, LBM_EDEVICE, "trial timing failed");
                    t_ms[s][ci] = sweep == 0 ? ms : std::min(t_ms[s][ci], ms);
                }
        int best_s = 0, best_c = 0;
        float best_ms = 1e30f;
        for (int s = 0; s < 3; ++s)
            for (int ci = 0; ci < 4; ++ci)
                if (t_ms[s][ci] < best_ms) {
                    best_ms = t_ms[s][ci];
                    best_s = s;
                    best_c = caps[ci];
                }
        advanced = k - b->step;         // the same for every group
        for (int s = 0; s < 3; ++s)
            if (s != best_s) batch_free(b, tiles[s]);
        G.wpb = shapes[best_s];
        G.cap = best_c;
        G.d_tiles = tiles[best_s];
        G.ntiles = nts[best_s];
        G.tile_cap = tcaps[best_s];
    }
    // every grid advanced by the same even number of steps, as lbm_batch_step would have moved it
    b->step += advanced;
    for (lbm_grid *g : b->grids) g->step += advanced;
    batch_drop_graph(b);
    return batch_join_out(b);
}

int lbm_batch_group_launch(const lbm_batch *b, int32_t group, int32_t *waves_per_block, int32_t *waves_per_cu_cap)
{
    if (!b || group < 0 || group >= (int32_t)b->groups.size()) return fail(nullptr, LBM_EINVAL, "no such group");
    if (waves_per_block) *waves_per_block = b->groups[group].wpb;
    if (waves_per_cu_cap) *waves_per_cu_cap = b->groups[group].cap;
    return LBM_OK;
}

int lbm_bandwidth_probe(void *dst, const void *src, size_t bytes, int32_t kind, void *stream)
{
    if (!dst || (bytes & 15) || (kind != 2 && !src)) return fail(nullptr, LBM_EINVAL, "bad probe arguments");
    const size_t n16 = bytes / 16, blocks = (n16 + 255) / 256;
    if (blocks == 0 || blocks > 0x7fffffff) return fail(nullptr, LBM_EINVAL, "probe size out of range");
    const dim3 gr((unsigned)blocks), bl(256);
    const hipStream_t st = (hipStream_t)stream;
    if (kind == 0) hipLaunchKernelGGL(k_copy_nt, gr, bl, 0, st, (const u32x4 *)src, (u32x4 *)dst, n16);
    else if (kind == 1) hipLaunchKernelGGL(k_read_nt, gr, bl, 0, st, (const u32x4 *)src, (u32x4 *)dst, n16);
    else if (kind == 2) hipLaunchKernelGGL(k_write_nt, gr, bl, 0, st, (u32x4 *)dst, n16);
    else return fail(nullptr, LBM_EINVAL, "probe kind must be 0, 1 or 2");
    if (hipGetLastError() != hipSuccess) return fail(nullptr, LBM_EDEVICE, "probe launch failed");
    return LBM_OK;
}

int lbm_copy_probe(void *dst, const void *src, size_t bytes, void *stream)
{
    if (!dst || !src || (bytes & 15)) return fail(nullptr, LBM_EINVAL, "copy probe needs 16-byte multiples");
    const size_t n16 = bytes / 16, blocks = (n16 + 255) / 256;
    if (blocks == 0 || blocks > 0x7fffffff) return fail(nullptr, LBM_EINVAL, "probe size out of range");
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, (const uint4 *)src,
                       (uint4 *)dst, n16);
    if (hipGetLastError() != hipSuccess) return fail(nullptr, LBM_EDEVICE, "copy probe launch failed");
    return LBM_OK;
}

} // extern "C"
