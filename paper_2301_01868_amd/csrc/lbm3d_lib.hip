// Host side of the 3D C ABI declared in include/lbm3d.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm3d.h"
#include "lbm3d_kernels.hpp"

using namespace lbm3;

namespace {
thread_local std::string g3_last_error;
}

struct lbm3d_grid {
    int n1 = 0, n2 = 0, n3 = 0, h = 0, pitch = 0;
    long long ncell = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<void *> allocs;
    double *P[2] = {nullptr, nullptr}, *side[2] = {nullptr, nullptr}, *lag[2] = {nullptr, nullptr};
    double *tab = nullptr, *Jrow = nullptr, *geo = nullptr, *mom = nullptr;
    Desc3 h_desc{};
    Desc3 *d_desc = nullptr;
    double rho0 = 1.0;
    int par = 0;
    int64_t step = 0;
    bool inited = false;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    std::string err;
};

static int fail3(lbm3d_grid *g, int code, const std::string &msg)
{
    if (g) g->err = msg;
    g3_last_error = msg;
    return code;
}

#define HIP3(g, call)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return fail3((g), LBM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

static void *dalloc3(lbm3d_grid *g, size_t bytes)
{
    void *p = nullptr;
    if (hipMalloc(&p, (bytes + 255) & ~(size_t)255) != hipSuccess) return nullptr;
    g->allocs.push_back(p);
    return p;
}

static unsigned ntiles3(const lbm3d_grid *g) { return (unsigned)((long long)g->n1 * g->n2 * ((g->n3 + 63) / 64)); }

extern "C" {

int lbm3d_lattice(int32_t *c, double *w, double *T0o)
{
    for (int a = 0; a < Q; ++a) {
        if (c)
            for (int d = 0; d < 3; ++d) c[3 * a + d] = cvec(a, d);
        if (w) w[a] = weight(a);
    }
    if (T0o) *T0o = T0;
    return LBM_OK;
}

const char *lbm3d_last_error(const lbm3d_grid *g)
{
    if (g && !g->err.empty()) return g->err.c_str();
    return g3_last_error.c_str();
}

void lbm3d_grid_destroy(lbm3d_grid *g)
{
    if (!g) return;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    for (auto &e : g->graph)
        if (e) (void)hipGraphExecDestroy(e);
    for (void *p : g->allocs) (void)hipFree(p);
    if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
}

int lbm3d_grid_create(const lbm3d_grid_desc *desc, lbm3d_grid **out)
{
    if (!desc || !out) return fail3(nullptr, LBM_EINVAL, "null argument");
    *out = nullptr;
    const lbm3d_grid_desc &D = *desc;
    if (D.n1 < 1 || D.n2 < 1 || D.n3 < 1) return fail3(nullptr, LBM_EINVAL, "n1, n2 and n3 must be positive");
    if (D.halo < CMAX + 1) return fail3(nullptr, LBM_EINVAL, "halo must be at least 4");
    if (!D.x || !D.y || !D.z) return fail3(nullptr, LBM_EINVAL, "mapping coordinates missing");
    if (!(D.tau > 0.5)) return fail3(nullptr, LBM_EINVAL, "tau must exceed 1/2");
    const bool per1 = D.bc_lo == LBM_PERIODIC || D.bc_hi == LBM_PERIODIC;
    if (per1 && D.bc_lo != D.bc_hi) return fail3(nullptr, LBM_EINVAL, "a periodic q1 side must be paired");
    for (int b : {D.bc_lo, D.bc_hi})
        if (b != LBM_PERIODIC && b != LBM_NOSLIP && b != LBM_MOVING) return fail3(nullptr, LBM_EINVAL, "unknown boundary kind");
    if (!per1 && D.n1 < CMAX) return fail3(nullptr, LBM_EINVAL, "n1 must be at least 3 with walls");
    const long long pitch = D.n3 >= 64 ? (D.n3 + 63) / 64 * 64 : D.n3;
    if ((long long)D.n1 * D.n2 * Q * pitch >= (1LL << 31) || (long long)D.n1 * D.n2 * ((D.n3 + 63) / 64) >= (1LL << 31))
        return fail3(nullptr, LBM_EINVAL, "grid too large");
    // the step addresses 2 c_max + 1 rows i of populations through one buffer resource (32-bit offsets)
    if ((2LL * CMAX + 1) * D.n2 * Q * pitch * 8 >= (1LL << 32))
        return fail3(nullptr, LBM_EINVAL, "rows too large: 7 rows of populations must stay below 4 GiB");

    lbm3d_grid *g = new lbm3d_grid();
    g->n1 = D.n1;
    g->n2 = D.n2;
    g->n3 = D.n3;
    g->h = D.halo;
    g->pitch = (int)pitch;
    g->rho0 = D.rho0;
    g->ncell = (long long)D.n1 * D.n2 * D.n3;
    if (D.stream) {
        g->stream = (hipStream_t)D.stream;
    } else {
        if (hipStreamCreate(&g->stream) != hipSuccess) {
            delete g;
            return fail3(nullptr, LBM_EDEVICE, "hipStreamCreate failed");
        }
        g->own_stream = true;
    }
    auto bail = [&](int code, const std::string &m) {
        g3_last_error = m;
        lbm3d_grid_destroy(g);
        return code;
    };
    const int h = g->h, H1 = g->n1 + 2 * h, H2 = g->n2 + 2 * h, H3 = g->n3 + 2 * h;
    const size_t nh = (size_t)H1 * H2 * H3, nc = (size_t)g->ncell;
    double *X = (double *)dalloc3(g, nh * 8), *Y = (double *)dalloc3(g, nh * 8), *Z = (double *)dalloc3(g, nh * 8);
    double *tg = (double *)dalloc3(g, nh * 9 * 8);
    g->geo = (double *)dalloc3(g, nc * GW * 8);
    g->tab = (double *)dalloc3(g, (size_t)g->n1 * TW * 8);
    g->Jrow = (double *)dalloc3(g, (size_t)g->n1 * 8);
    g->mom = (double *)dalloc3(g, nc * 7 * 8);
    int *flag = (int *)dalloc3(g, 2 * sizeof(int));
    g->d_desc = (Desc3 *)dalloc3(g, sizeof(Desc3));
    const size_t pe = (size_t)g->n1 * g->n2 * Q * g->pitch, se = (size_t)2 * 3 * CMAX * g->n2 * g->pitch;
    const size_t le = (size_t)3 * g->n1 * g->n2 * g->pitch;
    for (int b = 0; b < 2; ++b) {
        g->P[b] = (double *)dalloc3(g, pe * 8);
        g->side[b] = (double *)dalloc3(g, se * 8);
        g->lag[b] = (double *)dalloc3(g, le * 8);
    }
    if (!X || !Y || !Z || !tg || !g->geo || !g->tab || !g->Jrow || !g->mom || !flag || !g->d_desc || !g->P[0] ||
        !g->P[1] || !g->side[0] || !g->side[1] || !g->lag[0] || !g->lag[1])
        return bail(LBM_ENOMEM, "device allocation failed");
    hipStream_t st = g->stream;
#define HIPB3(call)                                                                                       \
    do {                                                                                                  \
        hipError_t e_ = (call);                                                                           \
        if (e_ != hipSuccess) return bail(LBM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)
    HIPB3(hipMemcpyAsync(X, D.x, nh * 8, hipMemcpyHostToDevice, st));
    HIPB3(hipMemcpyAsync(Y, D.y, nh * 8, hipMemcpyHostToDevice, st));
    HIPB3(hipMemcpyAsync(Z, D.z, nh * 8, hipMemcpyHostToDevice, st));
    int hflag[2] = {0, 0};
    HIPB3(hipMemcpyAsync(flag, hflag, sizeof hflag, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_tangent3, dim3((unsigned)((nh + 255) / 256)), dim3(256), 0, st, X, Y, Z, H1, H2, H3, tg);
    hipLaunchKernelGGL(k_geom3, dim3((unsigned)((nc + 127) / 128)), dim3(128), 0, st, tg, g->n1, g->n2, g->n3, h, g->geo);
    hipLaunchKernelGGL(k_rowcheck3, dim3((unsigned)((nc + 127) / 128)), dim3(128), 0, st, g->geo, g->n1, g->n2, g->n3,
                       1e-11, flag);
    hipLaunchKernelGGL(k_rowtab3, dim3(g->n1), dim3(128), 0, st, g->geo, g->n1, g->n2, g->n3, g->tab, g->Jrow);
    HIPB3(hipGetLastError());
    HIPB3(hipMemcpyAsync(hflag, flag, sizeof hflag, hipMemcpyDeviceToHost, st));
    HIPB3(hipMemsetAsync(g->side[0], 0, se * 8, st));
    HIPB3(hipMemsetAsync(g->side[1], 0, se * 8, st));
    HIPB3(hipStreamSynchronize(st));
    if (hflag[1]) return bail(LBM_EINVAL, "the mapping has J <= 0 (or non-finite geometry) in some cell");
    if (hflag[0]) return bail(LBM_EINVAL, "the metric terms depend on q2 or q3 (only q1-dependent mappings are served)");
    Desc3 &I = g->h_desc;
    I.P[0] = g->P[0];
    I.P[1] = g->P[1];
    I.side[0] = g->side[0];
    I.side[1] = g->side[1];
    I.lag[0] = g->lag[0];
    I.lag[1] = g->lag[1];
    I.tab = g->tab;
    I.Jrow = g->Jrow;
    I.mom = g->mom;
    I.n1 = g->n1;
    I.n2 = g->n2;
    I.n3 = g->n3;
    I.pitch = g->pitch;
    I.ncell = g->ncell;
    I.periodic1 = per1;
    I.bc_lo = per1 ? BC_PERIODIC : D.bc_lo;
    I.bc_hi = per1 ? BC_PERIODIC : D.bc_hi;
    for (int t = 0; t < 2; ++t) {
        I.ut_lo[t] = D.ut_lo[t];
        I.ut_hi[t] = D.ut_hi[t];
    }
    for (int e = 0; e < 3; ++e) I.a[e] = D.accel[e];
    I.omega = 1.0 / D.tau;
    I.kpi = -0.5 * (1.0 - 1.0 / (2.0 * D.tau));
    HIPB3(hipMemcpyAsync(g->d_desc, &I, sizeof(Desc3), hipMemcpyHostToDevice, st));
    HIPB3(hipStreamSynchronize(st));
#undef HIPB3
    (void)hipFree(X);
    (void)hipFree(Y);
    (void)hipFree(Z);
    (void)hipFree(tg);
    (void)hipFree(flag);
    for (void *p : {(void *)X, (void *)Y, (void *)Z, (void *)tg, (void *)flag})
        for (size_t k = 0; k < g->allocs.size(); ++k)
            if (g->allocs[k] == p) {
                g->allocs.erase(g->allocs.begin() + k);
                break;
            }
    g3_last_error.clear();
    *out = g;
    return LBM_OK;
}

int lbm3d_init(lbm3d_grid *g, const double *u0)
{
    if (!g) return fail3(nullptr, LBM_EINVAL, "null grid");
    double *du = nullptr;
    if (u0) {
        if (hipMalloc(&du, (size_t)g->ncell * 3 * 8) != hipSuccess) return fail3(g, LBM_ENOMEM, "allocation failed");
        HIP3(g, hipMemcpyAsync(du, u0, (size_t)g->ncell * 3 * 8, hipMemcpyHostToDevice, g->stream));
    }
    g->par = 0;
    g->step = 0;
    hipLaunchKernelGGL(k_init3, dim3(ntiles3(g)), dim3(64), 0, g->stream, (const Desc3 *)g->d_desc, (const double *)du,
                       g->rho0);
    // the initial state also serves as N'(q, -1): its lagged force sums
    hipLaunchKernelGGL(k_lag3, dim3(ntiles3(g)), dim3(64), 0, g->stream, (const Desc3 *)g->d_desc, 0);
    HIP3(g, hipGetLastError());
    HIP3(g, hipStreamSynchronize(g->stream));
    if (du) (void)hipFree(du);
    g->inited = true;
    return LBM_OK;
}

static int capture3(lbm3d_grid *g, int start, int steps)
{
    if (g->graph[start]) return LBM_OK;
    hipGraph_t graph = nullptr;
    HIP3(g, hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
    for (int s = 0; s < steps; ++s)
        hipLaunchKernelGGL(k_step3<false>, dim3(ntiles3(g)), dim3(64), 0, g->stream, (const Desc3 *)g->d_desc,
                           (start + s) & 1);
    HIP3(g, hipStreamEndCapture(g->stream, &graph));
    HIP3(g, hipGraphInstantiate(&g->graph[start], graph, nullptr, nullptr, 0));
    (void)hipGraphDestroy(graph);
    return LBM_OK;
}

int lbm3d_step(lbm3d_grid *g, int64_t n)
{
    if (!g) return fail3(nullptr, LBM_EINVAL, "null grid");
    if (!g->inited) return fail3(g, LBM_ESTATE, "lbm3d_init must be called before lbm3d_step");
    if (n < 0) return fail3(g, LBM_EINVAL, "negative step count");
    const int GS = 32;   // steps per captured graph (even: the buffer parity returns)
    if (n >= GS) {
        const int rc = capture3(g, g->par, GS);
        if (rc != LBM_OK) return rc;
        for (int64_t r = 0; r < n / GS; ++r) HIP3(g, hipGraphLaunch(g->graph[g->par], g->stream));
        g->step += n / GS * GS;
        n %= GS;
    }
    for (int64_t s = 0; s < n; ++s) {
        hipLaunchKernelGGL(k_step3<false>, dim3(ntiles3(g)), dim3(64), 0, g->stream, (const Desc3 *)g->d_desc, g->par);
        HIP3(g, hipGetLastError());
        g->par ^= 1;
        g->step += 1;
    }
    return LBM_OK;
}

int lbm3d_moments(lbm3d_grid *g, double *m, double *U, double *Ut)
{
    if (!g) return fail3(nullptr, LBM_EINVAL, "null grid");
    if (!g->inited) return fail3(g, LBM_ESTATE, "lbm3d_init must be called first");
    hipLaunchKernelGGL(k_step3<true>, dim3(ntiles3(g)), dim3(64), 0, g->stream, (const Desc3 *)g->d_desc, g->par);
    HIP3(g, hipGetLastError());
    const size_t nc = (size_t)g->ncell;
    std::vector<double> hm(nc * 7);
    HIP3(g, hipMemcpyAsync(hm.data(), g->mom, nc * 7 * 8, hipMemcpyDeviceToHost, g->stream));
    HIP3(g, hipStreamSynchronize(g->stream));
    for (size_t c = 0; c < nc; ++c) {
        if (m) m[c] = hm[c];
        for (int e = 0; e < 3; ++e) {
            if (U) U[3 * c + e] = hm[(1 + e) * nc + c];
            if (Ut) Ut[3 * c + e] = hm[(4 + e) * nc + c];
        }
    }
    return LBM_OK;
}

static int state_io(lbm3d_grid *g, double *P, double *side, int to_device)
{
    const size_t nP = (size_t)g->ncell * Q, ns = (size_t)2 * 3 * CMAX * g->n2 * g->n3;
    double *tmp = nullptr;
    if (hipMalloc(&tmp, std::max(nP, ns) * 8) != hipSuccess) return fail3(g, LBM_ENOMEM, "allocation failed");
    struct Free {
        double *p;
        ~Free() { (void)hipFree(p); }
    } fr{tmp};
    if (P) {
        if (to_device) HIP3(g, hipMemcpyAsync(tmp, P, nP * 8, hipMemcpyHostToDevice, g->stream));
        hipLaunchKernelGGL(k_state3, dim3(ntiles3(g)), dim3(64), 0, g->stream, (const Desc3 *)g->d_desc, g->par, tmp, to_device);
        if (to_device)
            hipLaunchKernelGGL(k_lag3, dim3(ntiles3(g)), dim3(64), 0, g->stream, (const Desc3 *)g->d_desc, g->par);
        HIP3(g, hipGetLastError());
        if (!to_device) HIP3(g, hipMemcpyAsync(P, tmp, nP * 8, hipMemcpyDeviceToHost, g->stream));
        HIP3(g, hipStreamSynchronize(g->stream));
    }
    if (side) {
        if (to_device) HIP3(g, hipMemcpyAsync(tmp, side, ns * 8, hipMemcpyHostToDevice, g->stream));
        hipLaunchKernelGGL(k_side3, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, g->stream, (const Desc3 *)g->d_desc,
                           g->par, tmp, to_device);
        HIP3(g, hipGetLastError());
        if (!to_device) HIP3(g, hipMemcpyAsync(side, tmp, ns * 8, hipMemcpyDeviceToHost, g->stream));
        HIP3(g, hipStreamSynchronize(g->stream));
    }
    return LBM_OK;
}

int lbm3d_get_state(lbm3d_grid *g, double *P, double *side)
{
    if (!g) return fail3(nullptr, LBM_EINVAL, "null grid");
    return state_io(g, P, side, 0);
}

int lbm3d_set_state(lbm3d_grid *g, const double *P, const double *side)
{
    if (!g) return fail3(nullptr, LBM_EINVAL, "null grid");
    const int rc = state_io(g, const_cast<double *>(P), const_cast<double *>(side), 1);
    if (rc == LBM_OK) g->inited = true;
    return rc;
}

int lbm3d_stream_map(lbm3d_grid *g, int32_t *src_cell, int32_t *src_dir, int32_t *wall)
{
    if (!g || !src_cell || !src_dir || !wall) return fail3(g, LBM_EINVAL, "null argument");
    const size_t n = (size_t)g->ncell * Q;
    int *t = nullptr;
    if (hipMalloc(&t, n * 3 * sizeof(int)) != hipSuccess) return fail3(g, LBM_ENOMEM, "allocation failed");
    struct Free {
        int *p;
        ~Free() { (void)hipFree(p); }
    } fr{t};
    hipLaunchKernelGGL(k_stream_map3, dim3(ntiles3(g)), dim3(64), 0, g->stream, (const Desc3 *)g->d_desc, t, t + n, t + 2 * n);
    HIP3(g, hipGetLastError());
    HIP3(g, hipMemcpyAsync(src_cell, t, n * 4, hipMemcpyDeviceToHost, g->stream));
    HIP3(g, hipMemcpyAsync(src_dir, t + n, n * 4, hipMemcpyDeviceToHost, g->stream));
    HIP3(g, hipMemcpyAsync(wall, t + 2 * n, n * 4, hipMemcpyDeviceToHost, g->stream));
    HIP3(g, hipStreamSynchronize(g->stream));
    return LBM_OK;
}

int lbm3d_geometry(lbm3d_grid *g, double *out)
{
    if (!g || !out) return fail3(g, LBM_EINVAL, "null argument");
    HIP3(g, hipMemcpyAsync(out, g->geo, (size_t)g->ncell * GW * 8, hipMemcpyDeviceToHost, g->stream));
    HIP3(g, hipStreamSynchronize(g->stream));
    return LBM_OK;
}

int lbm3d_synchronize(lbm3d_grid *g)
{
    if (!g) return fail3(nullptr, LBM_EINVAL, "null grid");
    HIP3(g, hipStreamSynchronize(g->stream));
    return LBM_OK;
}

} // extern "C"
