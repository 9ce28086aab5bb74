// Device code of the curvilinear lattice Boltzmann library (gfx950).
//
// Method: Chekhlov, Staroselsky, Zhang, Chen, arXiv:2301.01868, Sec. 2 and
// App. A-B.  The step works entirely in particle numbers N = J f, in which the
// volume J cancels from the update:
//   m = sum N,  m U^i = sum c^i N                          (Eqs. moments, vcomp)
//   J F^i = -1/2 sum_a [A+^i_a N'_a(q, t-1) - A-^i_a N_a]  (Eq. compo-constr)
//            + m a_ext^i,  with A-^i_a = -A+^i_{-a}
//   Ut = U + J F / (2 m)
//   J f^eq_a = m phi_a(U, Ut; g^ij)                         (Eq. equilibrium)
//   J dPi^ij = -1/2 (1 - 1/(2 tau)) sum_a c^i_a (A+^j_a - A-^j_a) m phi_a   (Eq. delta-flux)
//   dN_a = w_a [c.JF / T0 + (c^j c^k / T0 - delta^jk) J dPi^jk / T0]        (Eq. deltaN)
//   N'_a = N_a - (N_a - m phi_a) / tau + dN_a                (Eqs. collide, lbe)
// with A+^i_a(q) = sum_j c^j_a Theta^i_j(q + c_a, q) (Eq. gamma) precomputed.
//
// The equilibrium is evaluated in closed form, split into the part even and
// the part odd in c for each +-c pair: with G = g^ij,
//   phi_a = R_a + w_a [((c.Ut)^2 / T0 - |Ut|^2) / (2 T0)]                      (even)
//         + w_a [(c.U)(1/T0 + (4 T0 - |c|^2)/(2 T0^2)) - c.G.Ut / T0
//                + ((c.Ut)^2 - 3 T0 |Ut|^2)(c.Ut) / (6 T0^3)] + K_a (c.Ut)    (odd)
//   R_a = w_a [1 + (c.G.c - |c|^2 - T0 (tr G - 2)) / (2 T0)],
//   K_a = w_a (c.G.c - T0 tr G) / (2 T0^2),
// which is the index sum of Eq. (equilibrium) contracted with the isotropic
// Hermite tensors of a two-dimensional lattice.  Only the odd part enters the
// momentum-flux correction (the c^i factor makes even parts cancel in pairs).
//
// Populations may be stored as offsets s_a = N_a - B_a(q) from a per-cell base
// B (FP32 storage); the base terms are folded into per-row (or per-cell)
// constants so that every sum runs over small numbers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lbm_lattice.hpp"

namespace lbm {

enum { BC_PERIODIC = 0, BC_NOSLIP = 1, BC_MOVING = 2 };

// ---------------------------------------------------------------------------
// step table layout (compute type T), one entry per row (row-invariant
// geometry) or per cell
// ---------------------------------------------------------------------------
template <int Q>
struct Tab {
    static constexpr int G11 = 0, G12 = 1, G22 = 2, MB = 3, C1 = 4, C2 = 5, D0 = 6, PHIB0 = 7;
    static constexpr int NP = npair<Q>();
    // per direction a = 1..Q-1: A+^1_a, A+^2_a, base difference of the pulled source
    __host__ __device__ static constexpr int A1(int a) { return 8 + 3 * (a - 1); }
    __host__ __device__ static constexpr int A2(int a) { return 8 + 3 * (a - 1) + 1; }
    __host__ __device__ static constexpr int DB(int a) { return 8 + 3 * (a - 1) + 2; }
    // per +-c pair p: K (odd equilibrium coefficient), D (even rest part minus
    // the base's share), PHIB (the base's share), and the momentum-flux weights
    // X11 = k c1 S1, X12 = k (c1 S2 + c2 S1), X22 = k c2 S2 with
    // S^j = A+^j_a + A+^j_{-a} and k = -(1 - 1/(2 tau))
    __host__ __device__ static constexpr int PB(int p) { return 8 + 3 * (Q - 1) + 6 * p; }
    __host__ __device__ static constexpr int K(int p) { return PB(p); }
    __host__ __device__ static constexpr int D(int p) { return PB(p) + 1; }
    __host__ __device__ static constexpr int PHIB(int p) { return PB(p) + 2; }
    __host__ __device__ static constexpr int X11(int p) { return PB(p) + 3; }
    __host__ __device__ static constexpr int X12(int p) { return PB(p) + 4; }
    __host__ __device__ static constexpr int X22(int p) { return PB(p) + 5; }
    // per direction a = 0..Q-1: compute base minus storage base (added to a
    // computed offset to store it)
    __host__ __device__ static constexpr int SB(int a) { return 8 + 3 * (Q - 1) + 6 * NP + a; }
    static constexpr int W = 8 + 3 * (Q - 1) + 6 * NP + Q;
    static constexpr int STRIDE = (W + 3) & ~3;   // row stride, 16-byte multiple for FP32
};

// Per-instance launch descriptor (device memory, read with scalar loads).
struct InstDesc {
    void *P[2];          // population storage buffers, [n1][blocks][Q][block width] (see pidx)
    void *side[2];       // moving-wall side state, [2 walls][2 fields][hw][pitch]
    void *lag[2];        // lagged own-cell force sums sum_a A+^i_a s_a, [n1][2][pitch] (compute type)
    const void *tab;     // step table
    double *mom;         // moments output [5][ncell] (m, U1, U2, Ut1, Ut2)
    const double *mB64;  // FP64 base mass per table entry
    long long plane;     // n1 * pitch: a population buffer holds Q * plane elements, a lag buffer 2 * plane
    long long sa, sr;    // element strides between directions and between rows of a population buffer
    long long sb;        // element stride between column blocks of a row (see pidx)
    int bs, bm;          // column block: j >> bs is the block, j & bm the position (bm = 2^bs - 1)
    long long lsa, lsr;  // the same for the two force-sum fields of a lag buffer
    int n1, n2, pitch, hw;
    int periodic1, bc_lo, bc_hi, cell;
    int iters, ncell, par0;
    int sbase;           // storage base kind of the population offsets (0 local rest, 1 J w rho0, 2 none)
    double ut_lo, ut_hi, a1, a2, omega, kpi, rho0;
    // per-cell geometry for steps that rebuild their table fields (GE_* fields,
    // FP64, [field][n1 + 2 c_max][n2 + 2 c_max]: the cells and c_max layers of
    // the mapping's continuation around them)
    const double *geo;
    long long gfs;       // element stride between fields
    int gw, gpad;        // row width n2 + 2 c_max
};

// Element index of population a of cell (i, j) in a population buffer.  Each
// row holds column blocks, each block its Q direction segments.  FP32 and FP64
// storage use blocks of 64 columns (bs = 6: a wave's pulls and stores touch a
// few contiguous blocks); FP16 storage, and rows narrower than 64, use one
// block per row (bs = 30: [row][direction][column]).  Each choice was the
// faster one measured for its storage type.
__host__ __device__ inline size_t pidx(const InstDesc *d, int a, int i, int j)
{
    return (size_t)i * d->sr + (size_t)(j >> d->bs) * d->sb + (size_t)a * d->sa + (size_t)(j & d->bm);
}

// Source of the pulled population N_a(i, .) (Eq. adv, App. B): row r and
// direction beta of the post-collision field, and the crossed wall (0 none,
// 1 low side, 2 high side).  Beyond a wall the source node is replaced by its
// mirror image across the wall plane; no-slip takes the bounce-back direction,
// a moving wall the specular one.  Requires n1 >= c_max.
__host__ __device__ inline void pull_source(int i, int a, int n1, int periodic1, int bc_lo, int bc_hi, int &r,
                                            int &beta, int &wall)
{
    const int ti = i - cx(a);
    r = ti;
    beta = a;
    wall = 0;
    if (ti < 0) {
        if (periodic1) {
            r = ti + n1;
        } else {
            r = -1 - ti;
            wall = 1;
            beta = (bc_lo == BC_NOSLIP) ? bounce(a) : specular(a);
        }
    } else if (ti >= n1) {
        if (periodic1) {
            r = ti - n1;
        } else {
            r = 2 * n1 - 1 - ti;
            wall = 2;
            beta = (bc_hi == BC_NOSLIP) ? bounce(a) : specular(a);
        }
    }
}

__device__ inline int wrap_col(int c, int n2)
{
    if (c < 0) c += n2;
    if (c >= n2) c -= n2;
    return c;
}

// Raw buffer access (MUBUF): the 128-bit resource holds the buffer base and
// its size, so an access outside the buffer returns zero / is dropped instead
// of faulting; the per-direction row offset goes in the scalar offset, the
// column in the per-lane offset.
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
// Resource over rows r0 .. r0 + nrows - 1 of a buffer whose rows are
// row_bytes apart: offsets inside it stay small (32-bit) however large the
// buffer (the base address carries the row, in 64-bit arithmetic).  The step
// kernels' WIDE instances address buffers of 2 GiB and more this way; the
// others keep one resource over the whole buffer (fewer live scalar
// registers).  r0 may lie outside the buffer (a window that starts above its
// first row or a periodic wrap shifted by n1 rows): only the accessed rows
// must exist.
__device__ inline __amdgpu_buffer_rsrc_t row_rsrc(const void *base, size_t row_bytes, int r0, int nrows)
{
    return make_rsrc((const char *)base + (long long)r0 * (long long)row_bytes, (uint32_t)(row_bytes * (size_t)nrows));
}

// Cache policy of the population and force-sum accesses.  Stores are
// non-temporal (nt): each value is written once per step; so are the loads
// of the force sums (read once).  Population loads take the
// policy measured fastest for the lattice and storage type on gfx950 (the
// same kernels built both ways, alternating on one GPU): the pulled rows are
// read again by the neighbouring rows' tiles, and with FP32 storage, and for
// D2Q9 with FP64, the default policy keeps more of those re-reads in the
// cache (D2Q21 FP32 group 300-302 against 309-312 us, one 4096 x 16384 FP32
// grid 2049 against 2213 us, D2Q9 FP64 group about 310 against 349 us), while
// D2Q21 with FP64 or FP16 storage, and the FP64 per-cell step, run faster with
// nt loads (FP16 D2Q21 group 191-193 against 226-229 us).
#ifndef LBM_ST_AUX
#define LBM_ST_AUX 2
#endif
template <int Q, typename S>
__host__ __device__ constexpr int ld_aux()
{
    if constexpr (sizeof(S) == 4) return 0;              // FP32: default
    else if constexpr (sizeof(S) == 8) return Q == 9 ? 0 : 2;  // FP64: default for D2Q9, nt for D2Q21
    else return 2;                                       // FP16: nt
}
template <typename S, typename T, int AUX>
__device__ inline T bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    if constexpr (sizeof(S) == 8) {
        return (T)__builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
    } else {
        return (T)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
    }
}
template <typename S, typename T>
__device__ inline void bstore(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, T v)
{
    if constexpr (sizeof(S) == 8) {
        using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, (double)v), r, voff, soff, LBM_ST_AUX);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, (float)v), r, voff, soff, LBM_ST_AUX);
    }
}

// Population storage encoding.  FP64 and FP32 store the (offset) value as is;
// FP16 stores it divided by the direction's lattice weight, which brings the
// offsets of every direction to the same magnitude (per-plane scaling; the
// bounce-back and specular partners share the weight).
template <int Q, typename S>
__host__ __device__ constexpr double plane_scale(int a)
{
    if constexpr (sizeof(S) == 2) return weight<Q>(a);
    else return 1.0;
}
// The FP16 plane scales held in vector registers.  A decode (T)h * w + b is
// one v_fma_mix_f32, and an instruction of that encoding reads at most one
// scalar register; with both w (a constant) and b (a per-row base term) scalar,
// every decode needed a v_mov first.  A function that decodes many values
// makes one of these at its start (identical moves merge, one register per
// distinct weight).  For FP32 and FP64 storage, and where the base terms are
// per-lane values already (VREG = false: per-cell tables, stored or rebuilt),
// it holds nothing and the weights stay constants.
template <int Q, typename S, typename T, bool VREG = true>
struct PScale {
    static constexpr bool V = VREG && sizeof(S) == 2;
    T w[V ? Q : 1];
    __device__ __forceinline__ PScale()
    {
        if constexpr (V) {
#pragma unroll
            for (int a = 0; a < Q; ++a) __asm__("v_mov_b32 %0, %1" : "=v"(w[a]) : "s"((T)plane_scale<Q, S>(a)));
        }
    }
    __device__ __forceinline__ T operator()(int a) const
    {
        if constexpr (V) return w[a];
        else return (T)plane_scale<Q, S>(a);
    }
};

template <int Q, typename S, typename T, bool VREG>
__device__ inline T pload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, int a,
                          const PScale<Q, S, T, VREG> &ps)
{
    if constexpr (sizeof(S) == 2) {
        const _Float16 h =
            __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, ld_aux<Q, S>()));
        return (T)h * ps(a);
    } else {
        return bload<S, T, ld_aux<Q, S>()>(r, voff, soff);
    }
}
template <int Q, typename S, typename T, bool VREG>
__device__ inline T pdec(S v, int a, const PScale<Q, S, T, VREG> &ps)
{
    if constexpr (sizeof(S) == 2) return (T)v * ps(a);
    else return (T)v;
}
template <int Q, typename S, typename T>
__device__ inline T pload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, int a)
{
    if constexpr (sizeof(S) == 2) {
        const _Float16 h =
            __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, ld_aux<Q, S>()));
        return (T)h * (T)plane_scale<Q, S>(a);
    } else {
        return bload<S, T, ld_aux<Q, S>()>(r, voff, soff);
    }
}
template <int Q, typename S, typename T>
__device__ inline S penc(T v, int a)
{
    if constexpr (sizeof(S) == 2) return (S)(v * (T)(1.0 / plane_scale<Q, S>(a)));
    else return (S)v;
}
template <int Q, typename S, typename T>
__device__ inline T pdec(S v, int a)
{
    if constexpr (sizeof(S) == 2) return (T)v * (T)plane_scale<Q, S>(a);
    else return (T)v;
}
template <int Q, typename S, typename T>
__device__ inline void pstore(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, int a, T v)
{
    if constexpr (sizeof(S) == 2) {
        using U16 = decltype(__builtin_amdgcn_raw_buffer_load_b16(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(U16, penc<Q, S, T>(v, a)), r, voff, soff, LBM_ST_AUX);
    } else {
        bstore<S, T>(r, voff, soff, v);
    }
}

// uniform (scalar-cache) view of a row table
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

template <typename T, bool CELL>
struct TabView {
    const T *p;
    int s;
    __device__ inline T operator()(int f) const
    {
        if constexpr (CELL) {
            return p[(size_t)f * s];
        } else {
            return ((cptr<T>)p)[f];
        }
    }
};

// ---------------------------------------------------------------------------
// Per-cell table fields rebuilt from the geometry (general mappings).  A grid
// whose metric terms depend on q2 can step without streaming a stored table
// of every term: the workgroup stages the FP64 tangents g_1, g_2 of its cells
// and of c_max layers around them (and, for offset storage, J and H = J g^ij)
// into LDS, and the fields of Tab<Q> are evaluated where the step uses them,
// from the cell's own geometry and that of q + c_a, q - c_a or the pulled
// source (only the base's share of the force sum, two values per cell, is
// read from the grid's per-cell table):
//   A+^i_a(q) = g^i(q) . [e_a(q + c_a) - e_a(q)],  e_a = c^1_a g_1 + c^2_a g_2   (Eq. gamma)
//   S^i_a = A+^i_a + A+^i_{-a} = g^i(q) . [e_a(q + c_a) - e_a(q - c_a)]
// The differences of neighbouring tangents are taken in FP64, so the
// Christoffel sums keep the relative accuracy of the compute type where the
// mapping varies slowly.  The base terms of offset storage come from the local
// rest state, linear in (J, H):
//   J phi_rest,a = w_a [(2 - |c_a|^2 / (2 T0)) J + (c_a.H.c_a - T0 tr H) / (2 T0)]
// FP64 compute (GeoTab) stages the FP64 geometry and takes the differences in
// FP64.  FP32 compute (GeoTabF) stages FP32 deviations of every field from
// its value at a reference cell of the tile's 4-row band (the band's first
// row, the tile's first column; the same for every launch shape), rounded
// once from FP64, and takes every difference and term in FP32: a difference
// over one cell then carries the rounding of deviations of at most about 35
// cells' variation, a few 1e-6 of itself, and the step needs no FP64
// arithmetic per direction (FP64 values take two registers and two LDS words
// each, which held FP32 compute to fewer waves).
// ---------------------------------------------------------------------------
enum { GE_G1X = 0, GE_G1Y, GE_G2X, GE_G2Y, GE_J, GE_H11, GE_H12, GE_H22, GE_NF };

// geometry fields a step of compute type T stages: the tangents, plus J and H
// where populations are offsets from the local rest state (FP32 compute)
template <typename T>
__host__ __device__ constexpr int geo_stage_fields()
{
    return sizeof(T) == 4 ? GE_NF : GE_J;
}
// Staged tile of a workgroup of up to 4 rows of 64 cells: [field][4 + 2 c_max]
// [64 + 2 c_max] whatever the workgroup's row count, so that every offset in
// it is a compile-time constant
template <int Q>
__host__ __device__ constexpr int geo_tile_cols()
{
    return 64 + 2 * cmax<Q>();
}
template <int Q>
__host__ __device__ constexpr int geo_tile_field()
{
    return (4 + 2 * cmax<Q>()) * geo_tile_cols<Q>();
}
// LDS bytes of one workgroup's staged geometry (FP64 values for FP64
// compute, FP32 deviations for FP32 compute)
template <int Q, typename T>
__host__ __device__ constexpr unsigned geo_stage_bytes()
{
    return (unsigned)(geo_stage_fields<T>() * geo_tile_field<Q>() * sizeof(T));
}

// Own-cell values by exchange.  The lagged force of Eq. (compo-constr) needs
// the own cell's N'_a(q, t-1), which in this step is the value the neighbour
// q + c_a pulls.  Steps of D2Q9 grids with per-row tables and FP32 or FP64
// storage take it from there (FP16 keeps the stored sums: its step is bound
// by the vector ALU, which the tile's work would add to).  Every lane writes
// its pulled values, as loaded, to an LDS tile [wave][a - 1][lane] of the
// workgroup's rows, and after a barrier each cell reads those of its
// partners inside the tile; the rest (partners in another workgroup's rows or
// columns, or outside the grid) are loaded from the own cell in HBM.  Either
// way the value is the stored one, bit for bit, and the sum is formed in the
// same order as the stored force sums of the other kernels, so the results
// are the same bits.  (With c_max = 1 a 4-row tile finds 6.4 of the 8
// partners inside; the 20 D2Q21 partners reach 3 rows out and keep the stored
// sums.)
template <int Q, typename S, int CT, bool MOM>
__host__ __device__ constexpr bool xch_step()
{
    return CT == 0 && !MOM && Q == 9 && sizeof(S) >= 4;
}
// LDS bytes of the exchange tile of a workgroup of wpb waves
template <int Q, typename T>
__host__ __device__ constexpr unsigned xch_bytes(int wpb)
{
    return (unsigned)(wpb * (Q - 1) * 64 * (int)sizeof(T));
}

// Start copying the geometry of the workgroup's rows tl.y .. tl.y + wpb - 1
// and columns tl.z .. tl.z + 63, with c_max layers around them, into the LDS
// tile.  The loads go straight to LDS (no registers): each instruction moves
// 64 consecutive dwords of a field's tile rows, which lie contiguously both
// in LDS and, row by row, in the geometry array.  Rows and columns past the
// stored range are clamped to it; those entries are never read by a cell
// inside the grid.  The caller waits for the loads (s_waitcnt) and then for
// the other waves (barrier) before reading the tile, and may issue other
// loads in between.
template <int Q, typename T>
__device__ __forceinline__ const double *stage_geometry(const InstDesc *__restrict__ d, const int4 tl, int wave)
{
    extern __shared__ double geo_lds[];
    constexpr int CM = cmax<Q>(), TC = geo_tile_cols<Q>(), FS = geo_tile_field<Q>();
    constexpr int NF = geo_stage_fields<T>();
    const int nw = (int)(blockDim.x >> 6), TR = nw + 2 * CM;
    const int lane = (int)(threadIdx.x & 63);
    const int ger = d->n1 + 2 * CM, gw = d->gw;
    const double *__restrict__ ge = d->geo;
    const int nd = 2 * TR * TC;   // dwords of one field's tile rows
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const double *gf = ge + (size_t)f * d->gfs;
        for (int k0 = wave * 64; k0 < nd; k0 += nw * 64) {
            const int k = k0 + lane;
            if (k < nd) {
                const int e = k >> 1, rr = e / TC, cc = e - rr * TC;
                const int er = min(tl.y + rr, ger - 1), ec = min(tl.z + cc, gw - 1);
                const char *src = (const char *)(gf + (size_t)er * gw + ec) + (k & 1) * 4;
                __builtin_amdgcn_global_load_lds(
                    src, (__attribute__((address_space(3))) void *)((char *)(geo_lds + f * FS) + 4 * k0), 4, 0, 0);
            }
        }
    }
    return geo_lds;
}

// FP32 compute: stage, per field, the FP32 deviation of every tile entry
// from the field's value at the reference cell (band row tl.y & ~3, column
// tl.z), into the LDS tile; ref[f] receives those reference values.  All
// loads of a pass are issued before its stores.  Returns the tile; the
// caller waits for the other waves (barrier) before reading it.
// J and H are read only at the pulled sources (the base differences).
// Beyond a wall the pulled source is the mirror cell (App. B), so the tile
// rows past a wall hold the mirror row's J and H there, with H12 negated at a
// moving wall (the specular direction flips c^1, hence the sign of the c^1 c^2
// H12 term of the source's rest state): every base difference then reads the
// row of q - c_a, whatever the row of q.  The tangents keep the ghost rows of
// the extended geometry (the rebuilt Christoffel sums difference them).
template <int Q>
__device__ __forceinline__ const float *stage_geometry_f(const InstDesc *__restrict__ d, const int4 tl, int wave,
                                                         double (&ref)[GE_NF])
{
    extern __shared__ float geo_ldsf[];
    constexpr int CM = cmax<Q>(), TC = geo_tile_cols<Q>(), FS = geo_tile_field<Q>();
    const int nw = (int)(blockDim.x >> 6), TR = nw + 2 * CM;
    const int lane = (int)(threadIdx.x & 63);
    const int ger = d->n1 + 2 * CM, gw = d->gw;
    const double *__restrict__ ge = d->geo;
    const size_t gfs = (size_t)d->gfs;
    // reference cell (extended indices: cell row r is geometry row r + c_max)
    const size_t rc = (size_t)((tl.y & ~3) + CM) * gw + (size_t)(tl.z + CM);
#pragma unroll
    for (int f = 0; f < GE_NF; ++f) ref[f] = ge[f * gfs + rc];
    // each wave takes whole tile rows (one field, one row of 64 + 2 c_max
    // entries: lanes 0-63 and, for the last 2 c_max, lanes 0 .. 2 c_max - 1
    // again), U rows per pass with every load issued before the stores
    constexpr int U = 4;
    const int nrows = GE_NF * TR;
    const int n1 = d->n1;
    const bool walls = !d->periodic1;
    const bool flip_lo = d->bc_lo != BC_NOSLIP, flip_hi = d->bc_hi != BC_NOSLIP;
    // extended geometry row of tile row rr of field f, and whether its value is negated
    auto src_row = [&](int f, int rr, bool &neg) {
        int er = min(tl.y + rr, ger - 1);
        neg = false;
        if (walls && f >= GE_J) {
            const int ti = er - CM;   // cell row
            if (ti < 0) {
                er = -1 - ti + CM;
                neg = f == GE_H12 && flip_lo;
            } else if (ti >= n1) {
                er = 2 * n1 - 1 - ti + CM;
                neg = f == GE_H12 && flip_hi;
            }
            er = min(max(er, 0), ger - 1);   // rows no cell reads (narrow grids) stay in range
        }
        return er;
    };
    for (int t0 = wave; t0 < nrows; t0 += U * nw) {
        double v[U][2];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * nw;
            const int f = t / TR, rr = t - f * TR;
            bool neg;
            const int er = src_row(f, rr, neg);
            const double *src = ge + f * gfs + (size_t)er * gw;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int cc = lane + 64 * h;
                v[u][h] = (t < nrows && cc < TC) ? src[min(tl.z + cc, gw - 1)] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u * nw;
            if (t < nrows) {
                const int f = t / TR, rr = t - f * TR;
                bool neg;
                (void)src_row(f, rr, neg);
                double r = ref[0];
#pragma unroll
                for (int g = 1; g < GE_NF; ++g)
                    if (f == g) r = ref[g];
                // +-v - r in one rounding (the sign is exact), the same bits as v - r
                const double sg = neg ? -1.0 : 1.0;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int cc = lane + 64 * h;
                    if (cc < TC) geo_ldsf[f * FS + rr * TC + cc] = (float)__builtin_fma(sg, v[u][h], -r);
                }
            }
        }
    }
    return geo_ldsf;
}

// Rebuilt table fields for FP32 compute, from the staged FP32 deviations.
template <int Q>
struct GeoTabF {
    using T = float;
    using TB = Tab<Q>;
    static constexpr int CM = cmax<Q>();
    static constexpr double T0 = lattice_T0<Q>();
    static constexpr int TC = geo_tile_cols<Q>(), FS = geo_tile_field<Q>();
    const float *L;    // staged deviations
    int o;             // own cell in a staged field
    float eJ, e11, e12, e22, e1x, e1y, e2x, e2y;   // own deviations
    float rho0f;
    T u1x, u1y, u2x, u2y, G11, G12, G22, mb, c1s, c2s, kpi;

    __device__ __forceinline__ float ld(int f, int dr, int dc) const { return L[o + (f * FS + dr * TC + dc)]; }

    // e_a(q + c_a) - e_a(q)
    __device__ __forceinline__ void dA(int a, T &dx, T &dy) const
    {
        const int c1 = cx(a), c2 = cy(a);
        dx = 0.f;
        dy = 0.f;
        if (c1 != 0) {
            dx += (T)c1 * (ld(GE_G1X, c1, c2) - e1x);
            dy += (T)c1 * (ld(GE_G1Y, c1, c2) - e1y);
        }
        if (c2 != 0) {
            dx += (T)c2 * (ld(GE_G2X, c1, c2) - e2x);
            dy += (T)c2 * (ld(GE_G2Y, c1, c2) - e2y);
        }
    }
    // e_a(q + c_a) - e_a(q - c_a)
    __device__ __forceinline__ void dS(int a, T &dx, T &dy) const
    {
        const int c1 = cx(a), c2 = cy(a);
        dx = 0.f;
        dy = 0.f;
        if (c1 != 0) {
            dx += (T)c1 * (ld(GE_G1X, c1, c2) - ld(GE_G1X, -c1, -c2));
            dy += (T)c1 * (ld(GE_G1Y, c1, c2) - ld(GE_G1Y, -c1, -c2));
        }
        if (c2 != 0) {
            dx += (T)c2 * (ld(GE_G2X, c1, c2) - ld(GE_G2X, -c1, -c2));
            dy += (T)c2 * (ld(GE_G2Y, c1, c2) - ld(GE_G2Y, -c1, -c2));
        }
    }

    __device__ __forceinline__ void setup(const InstDesc *__restrict__ d, const float *lds, const double (&ref)[GE_NF],
                                          int wave, int lane, int row, int col)
    {
        L = lds;
        o = (wave + CM) * TC + lane + CM;
        const double rho0 = d->rho0;
        rho0f = (float)rho0;
        kpi = (T)d->kpi;
        e1x = ld(GE_G1X, 0, 0);
        e1y = ld(GE_G1Y, 0, 0);
        e2x = ld(GE_G2X, 0, 0);
        e2y = ld(GE_G2Y, 0, 0);
        eJ = ld(GE_J, 0, 0);
        e11 = ld(GE_H11, 0, 0);
        e12 = ld(GE_H12, 0, 0);
        e22 = ld(GE_H22, 0, 0);
        // the cell's own values, once per cell in FP64
        const double g1x = ref[GE_G1X] + e1x, g1y = ref[GE_G1Y] + e1y;
        const double g2x = ref[GE_G2X] + e2x, g2y = ref[GE_G2Y] + e2y;
        const double J = ref[GE_J] + eJ, H11 = ref[GE_H11] + e11, H12 = ref[GE_H12] + e12, H22 = ref[GE_H22] + e22;
        const double iJ = 1.0 / J;
        G11 = (T)(H11 * iJ);
        G12 = (T)(H12 * iJ);
        G22 = (T)(H22 * iJ);
        // co-tangents g^1 = (g_2 x z) / J, g^2 = (z x g_1) / J
        u1x = (T)(g2y * iJ);
        u1y = (T)(-g2x * iJ);
        u2x = (T)(-g1y * iJ);
        u2y = (T)(g1x * iJ);
        mb = (T)(rho0 * J);
        // the base's share of the force sum, sum_a (A+_a + A+_-a) B_a, sums
        // products of population-size bases: formed in FP64 when the grid is
        // created, read from the grid's per-cell table
        const T *tab = (const T *)d->tab + (size_t)row * d->n2 + col;
        c1s = tab[(size_t)TB::C1 * d->ncell];
        c2s = tab[(size_t)TB::C2 * d->ncell];
    }

    // rest equilibrium phi_rest,a(g^ij)
    __device__ __forceinline__ T rest(int a) const
    {
        const T c1 = (T)cx(a), c2 = (T)cy(a);
        const T cGc = c1 * c1 * G11 + (T)2 * c1 * c2 * G12 + c2 * c2 * G22;
        return (T)weight<Q>(a) *
               ((T)1 + (cGc - (c1 * c1 + c2 * c2) - (T)T0 * (G11 + G22 - (T)2)) * (T)(1.0 / (2.0 * T0)));
    }
    // odd equilibrium coefficient K_a = w_a (c.G.c - T0 tr G) / (2 T0^2)
    __device__ __forceinline__ T kodd(int a) const
    {
        const T c1 = (T)cx(a), c2 = (T)cy(a);
        const T cGc = c1 * c1 * G11 + (T)2 * c1 * c2 * G12 + c2 * c2 * G22;
        return (T)(weight<Q>(a) / (2.0 * T0 * T0)) * (cGc - (T)T0 * (G11 + G22));
    }
    // storage base of the pulled source (its local rest state), moved to
    // this cell's compute base: rho0 (J phi_rest,a at the source - at this
    // cell), linear in the differences of J and H (the q1 component of c_a
    // flipped at a moving wall flips the sign of the source's c1 c2 H12 term)
    __device__ __forceinline__ T dbase(int a) const
    {
        // the source q - c_a: past a wall, the staged tile holds the mirror
        // cell's J and H there (with H12 negated at a moving wall)
        const int dr = -cx(a), dc = -cy(a);
        const T c1 = (T)cx(a), c2 = (T)cy(a);
        const T dJ = ld(GE_J, dr, dc) - eJ;
        const T d11 = ld(GE_H11, dr, dc) - e11;
        const T d22 = ld(GE_H22, dr, dc) - e22;
        const T d12 = ld(GE_H12, dr, dc) - e12;
        return rho0f * (T)weight<Q>(a) *
               ((T)(2.0 - (cx(a) * cx(a) + cy(a) * cy(a)) / (2.0 * T0)) * dJ +
                (c1 * c1 * d11 + (T)2 * c1 * c2 * d12 + c2 * c2 * d22 - (T)T0 * (d11 + d22)) * (T)(1.0 / (2.0 * T0)));
    }
    // compute base minus storage base: both the local rest state
    __device__ __forceinline__ T sbdiff(int) const { return (T)0; }

    // Sums over directions of the rebuilt terms, formed on the vectors and
    // projected once: every A+^i_a is g^i . D_a with D_a = e_a(q + c_a) - e_a(q),
    // so sum_a A+^i_a x_a = g^i . sum_a D_a x_a; accA adds D_a x_a to V, proj
    // adds g^i . V to L^i
    __device__ __forceinline__ void accA(int a, T x, T &V1, T &V2) const
    {
        T dx, dy;
        dA(a, dx, dy);
        V1 += dx * x;
        V2 += dy * x;
    }
    __device__ __forceinline__ void proj(T V1, T V2, T &L1, T &L2) const
    {
        L1 += V1 * u1x + V2 * u1y;
        L2 += V1 * u2x + V2 * u2y;
    }
    // the momentum-flux sums P^ij = sum_p X^ij_p x_p likewise: with S_p =
    // e_a(q + c_a) - e_a(q - c_a), accS adds c^1_a x S_p to (W[0], W[1]) and
    // c^2_a x S_p to (W[2], W[3]); flux projects them onto g^1 and g^2
    __device__ __forceinline__ void accS(int a, T x, T (&W)[4]) const
    {
        const int c1 = cx(a), c2 = cy(a);
        T sx, sy;
        dS(a, sx, sy);
        const T xs = sx * x, ys = sy * x;
        if (c1 != 0) {
            W[0] += (T)c1 * xs;
            W[1] += (T)c1 * ys;
        }
        if (c2 != 0) {
            W[2] += (T)c2 * xs;
            W[3] += (T)c2 * ys;
        }
    }
    __device__ __forceinline__ void flux(const T (&W)[4], T &P11, T &P12, T &P22) const
    {
        P11 = kpi * (W[0] * u1x + W[1] * u1y);
        P22 = kpi * (W[2] * u2x + W[3] * u2y);
        P12 = kpi * ((W[0] * u2x + W[1] * u2y) + (W[2] * u1x + W[3] * u1y));
    }

    __device__ __forceinline__ T operator()(int f) const
    {
        if (f == TB::G11) return G11;
        if (f == TB::G12) return G12;
        if (f == TB::G22) return G22;
        if (f == TB::MB) return mb;
        if (f == TB::C1) return c1s;
        if (f == TB::C2) return c2s;
        if (f == TB::D0) return (T)0;
        if (f == TB::PHIB0) return rest(0);
        if (f < TB::PB(0)) {
            const int a = (f - 8) / 3 + 1, k = (f - 8) % 3;
            if (k == 2) return dbase(a);
            T dx, dy;
            dA(a, dx, dy);
            return k == 0 ? dx * u1x + dy * u1y : dx * u2x + dy * u2y;
        }
        if (f < TB::SB(0)) {
            const int p = (f - TB::PB(0)) / 6, k = (f - TB::PB(0)) % 6;
            const int a = pair_rep(p);
            if (k == 0) return kodd(a);
            if (k == 1) return (T)0;
            if (k == 2) return rest(a);
            T sx, sy;
            dS(a, sx, sy);
            const T S1 = sx * u1x + sy * u1y, S2 = sx * u2x + sy * u2y;
            const T c1 = (T)cx(a), c2 = (T)cy(a);
            if (k == 3) return kpi * c1 * S1;
            if (k == 4) return kpi * (c1 * S2 + c2 * S1);
            return kpi * c2 * S2;
        }
        return sbdiff(f - TB::SB(0));
    }
};

// Rebuilt table fields for FP64 compute (the particle numbers themselves,
// no offset base), from the staged FP64 tangents.
template <int Q, typename T>
struct GeoTab {
    static_assert(sizeof(T) == 8, "FP32 compute uses GeoTabF");
    using TB = Tab<Q>;
    static constexpr int CM = cmax<Q>();
    static constexpr double T0 = lattice_T0<Q>();
    static constexpr int TC = geo_tile_cols<Q>(), FS = geo_tile_field<Q>();
    const double *L;   // staged geometry
    int o;             // own cell in a staged field
    double g1x, g1y, g2x, g2y;
    T u1x, u1y, u2x, u2y, G11, G12, G22, kpi;

    __device__ __forceinline__ double ld(int f, int dr, int dc) const { return L[o + (f * FS + dr * TC + dc)]; }

    // e_a(q + c_a) - e_a(q)
    __device__ __forceinline__ void dA(int a, double &dx, double &dy) const
    {
        const int c1 = cx(a), c2 = cy(a);
        dx = 0.0;
        dy = 0.0;
        if (c1 != 0) {
            dx += c1 * (ld(GE_G1X, c1, c2) - g1x);
            dy += c1 * (ld(GE_G1Y, c1, c2) - g1y);
        }
        if (c2 != 0) {
            dx += c2 * (ld(GE_G2X, c1, c2) - g2x);
            dy += c2 * (ld(GE_G2Y, c1, c2) - g2y);
        }
    }
    // e_a(q + c_a) - e_a(q - c_a)
    __device__ __forceinline__ void dS(int a, double &dx, double &dy) const
    {
        const int c1 = cx(a), c2 = cy(a);
        dx = 0.0;
        dy = 0.0;
        if (c1 != 0) {
            dx += c1 * (ld(GE_G1X, c1, c2) - ld(GE_G1X, -c1, -c2));
            dy += c1 * (ld(GE_G1Y, c1, c2) - ld(GE_G1Y, -c1, -c2));
        }
        if (c2 != 0) {
            dx += c2 * (ld(GE_G2X, c1, c2) - ld(GE_G2X, -c1, -c2));
            dy += c2 * (ld(GE_G2Y, c1, c2) - ld(GE_G2Y, -c1, -c2));
        }
    }

    __device__ __forceinline__ void setup(const InstDesc *__restrict__ d, const double *lds, int wave, int lane, int,
                                          int)
    {
        L = lds;
        o = (wave + CM) * TC + lane + CM;
        kpi = (T)d->kpi;
        g1x = ld(GE_G1X, 0, 0);
        g1y = ld(GE_G1Y, 0, 0);
        g2x = ld(GE_G2X, 0, 0);
        g2y = ld(GE_G2Y, 0, 0);
        const double J = g1x * g2y - g1y * g2x;
        const double iJ = 1.0 / J, iJ2 = iJ * iJ;
        G11 = (T)((g2x * g2x + g2y * g2y) * iJ2);
        G12 = (T)(-(g1x * g2x + g1y * g2y) * iJ2);
        G22 = (T)((g1x * g1x + g1y * g1y) * iJ2);
        // co-tangents g^1 = (g_2 x z) / J, g^2 = (z x g_1) / J
        u1x = (T)(g2y * iJ);
        u1y = (T)(-g2x * iJ);
        u2x = (T)(-g1y * iJ);
        u2y = (T)(g1x * iJ);
    }

    // rest equilibrium phi_rest,a(g^ij)
    __device__ __forceinline__ T rest(int a) const
    {
        const T c1 = (T)cx(a), c2 = (T)cy(a);
        const T cGc = c1 * c1 * G11 + (T)2 * c1 * c2 * G12 + c2 * c2 * G22;
        return (T)weight<Q>(a) *
               ((T)1 + (cGc - (c1 * c1 + c2 * c2) - (T)T0 * (G11 + G22 - (T)2)) * (T)(1.0 / (2.0 * T0)));
    }
    // odd equilibrium coefficient K_a = w_a (c.G.c - T0 tr G) / (2 T0^2)
    __device__ __forceinline__ T kodd(int a) const
    {
        const T c1 = (T)cx(a), c2 = (T)cy(a);
        const T cGc = c1 * c1 * G11 + (T)2 * c1 * c2 * G12 + c2 * c2 * G22;
        return (T)(weight<Q>(a) / (2.0 * T0 * T0)) * (cGc - (T)T0 * (G11 + G22));
    }

    // direction sums formed on the vectors and projected once (as GeoTabF)
    __device__ __forceinline__ void accA(int a, T x, T &V1, T &V2) const
    {
        double dx, dy;
        dA(a, dx, dy);
        V1 += (T)dx * x;
        V2 += (T)dy * x;
    }
    __device__ __forceinline__ void proj(T V1, T V2, T &L1, T &L2) const
    {
        L1 += V1 * u1x + V2 * u1y;
        L2 += V1 * u2x + V2 * u2y;
    }
    __device__ __forceinline__ void accS(int a, T x, T (&W)[4]) const
    {
        const int c1 = cx(a), c2 = cy(a);
        double sx, sy;
        dS(a, sx, sy);
        const T xs = (T)sx * x, ys = (T)sy * x;
        if (c1 != 0) {
            W[0] += (T)c1 * xs;
            W[1] += (T)c1 * ys;
        }
        if (c2 != 0) {
            W[2] += (T)c2 * xs;
            W[3] += (T)c2 * ys;
        }
    }
    __device__ __forceinline__ void flux(const T (&W)[4], T &P11, T &P12, T &P22) const
    {
        P11 = kpi * (W[0] * u1x + W[1] * u1y);
        P22 = kpi * (W[2] * u2x + W[3] * u2y);
        P12 = kpi * ((W[0] * u2x + W[1] * u2y) + (W[2] * u1x + W[3] * u1y));
    }

    __device__ __forceinline__ T operator()(int f) const
    {
        if (f == TB::G11) return G11;
        if (f == TB::G12) return G12;
        if (f == TB::G22) return G22;
        if (f == TB::MB || f == TB::C1 || f == TB::C2 || f == TB::PHIB0) return (T)0;
        if (f == TB::D0) return rest(0);
        if (f < TB::PB(0)) {
            const int a = (f - 8) / 3 + 1, k = (f - 8) % 3;
            if (k == 2) return (T)0;   // no offset base
            double dx, dy;
            dA(a, dx, dy);
            return k == 0 ? (T)dx * u1x + (T)dy * u1y : (T)dx * u2x + (T)dy * u2y;
        }
        if (f < TB::SB(0)) {
            const int p = (f - TB::PB(0)) / 6, k = (f - TB::PB(0)) % 6;
            const int a = pair_rep(p);
            if (k == 0) return kodd(a);
            if (k == 1) return rest(a);
            if (k == 2) return (T)0;
            double sx, sy;
            dS(a, sx, sy);
            const T S1 = (T)sx * u1x + (T)sy * u1y, S2 = (T)sx * u2x + (T)sy * u2y;
            const T c1 = (T)cx(a), c2 = (T)cy(a);
            if (k == 3) return kpi * c1 * S1;
            if (k == 4) return kpi * (c1 * S2 + c2 * S1);
            return kpi * c2 * S2;
        }
        return (T)0;   // storage base differences: none
    }
};

// Per-lane table fields (stored per-cell tables, or fields rebuilt from the
// staged geometry) are cheap to read again but costly to keep: without a
// fence between the phases of the step the compiler holds every field it has
// read until its last use, over a hundred extra VGPRs for D2Q21.  The fence
// (a compiler barrier on memory, no instruction) makes it read them again.
template <int CT>
__device__ __forceinline__ void phase_fence()
{
    if constexpr (CT != 0) __asm__ volatile("" ::: "memory");
}

// Scheduling boundary between the directions of a loop over per-lane table
// fields: the scheduler would otherwise start every field's loads at once.
template <int CT>
__device__ __forceinline__ void sgroup()
{
    if constexpr (CT != 0) __builtin_amdgcn_sched_barrier(0);
}

template <int Q, typename T, int CT>
struct TabSel {
    using type = TabView<T, CT == 1>;
};
template <int Q, typename T>
struct TabSel<Q, T, 2> {
    using type = typename std::conditional<sizeof(T) == 4, GeoTabF<Q>, GeoTab<Q, T>>::type;
};

// ---------------------------------------------------------------------------
// Pieces of the fused step (pull + moments + force + equilibrium + flux
// correction + curvilinear correction + BGK + store), one cell per lane.
// CT: 0 per-row tables, 1 per-cell tables, 2 per-cell fields rebuilt from
// the staged geometry.
// ---------------------------------------------------------------------------

// Per-lane base terms of the pulled populations (per-cell tables or rebuilt
// fields): the source's storage base moved to this cell's compute base, added
// once every pull is in flight.
template <int Q, typename T, int CT, typename TBT>
__device__ __forceinline__ void add_bases(const TBT &tb, T (&n)[Q])
{
    using TB = Tab<Q>;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        n[a] += (a > 0) ? tb(TB::DB(a)) : -tb(TB::SB(0));
        sgroup<CT>();
    }
    phase_fence<CT>();
}

// Pulled populations N_a(i, j) of Eq. (adv) with the boundary sources of
// App. B, read from the post-collision field in HBM and moved to the cell's
// compute base.  j0 is the first column of the wave's 64.  XW: each value as
// loaded (before any base or wall term) also goes to xw[(a - 1) * 64], a = 1..Q-1,
// the lane's slots of the exchange tile.
template <int Q, typename T, typename S, int CT, bool WIDE, bool BASES = true, bool XW = false, typename TBT>
__device__ __forceinline__ void pull_cell(const InstDesc *__restrict__ d, const TBT &tb, int i, int j, int j0, int pin,
                                          T (&n)[Q], T *xw = nullptr)
{
    constexpr int CM = cmax<Q>();
    constexpr double T0d = lattice_T0<Q>();
    using TB = Tab<Q>;
    const int n1 = d->n1, n2 = d->n2;
    const int pitch = d->pitch, hw = d->hw;
    const long long plane = d->plane;
    const int bclo = d->bc_lo, bchi = d->bc_hi, per1 = d->periodic1;
    constexpr uint32_t ES = sizeof(S);
    const uint32_t sa_b = (uint32_t)d->sa * ES, sb_b = (uint32_t)d->sb * ES;
    const size_t row_b = (size_t)d->sr * ES;
    const uint32_t sr_b = (uint32_t)row_b;
    const int bs = d->bs, bm = d->bm;
    const int lane = j - j0;
    // byte offset of the wave's own cells inside a row
    const uint32_t jb = (uint32_t)(j >> bs) * sb_b + (uint32_t)(j & bm) * ES;

    const PScale<Q, S, T, CT == 0> ps;
    const bool interior = (i >= CM && i < n1 - CM);
    const bool nowrap = (j0 >= CM) && (j0 + 63 + CM < n2);
    if (interior && nowrap) {
        // one resource over the whole buffer, or (WIDE) over the stencil's
        // rows i - c_max .. i + c_max; r0 is row i inside it
        const __amdgpu_buffer_rsrc_t rin = WIDE ? row_rsrc(d->P[pin], row_b, i - CM, 2 * CM + 1)
                                                : make_rsrc(d->P[pin], (uint32_t)(plane * Q) * ES);
        const int r0 = WIDE ? CM : i;
        // the whole stencil of the wave stays inside: source (i - c1, j - c2),
        // same direction
        if constexpr (sizeof(S) >= 4) {
            // 64-column blocks (the fast path needs n2 > 64, so bs = 6):
            // column j - c2 lies in block j0/64 - 1, j0/64 or j0/64 + 1
            // (j0 >= 64 here); one per-lane offset per shift c2, counted from
            // the start of block j0/64 - 1, which rides in the scalar offset
            // with the direction and the source row
            uint32_t vsh[2 * CM + 1];
#pragma unroll
            for (int k = -CM; k <= CM; ++k) {
                const int p = 64 + lane - k;
                vsh[k + CM] = (uint32_t)(p >> 6) * sb_b + (uint32_t)(p & 63) * ES;
            }
            const uint32_t blk = (uint32_t)((j0 >> 6) - 1) * sb_b;
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                const uint32_t soff = (uint32_t)a * sa_b + (uint32_t)(r0 - cx(a)) * sr_b + blk;
                n[a] = pload<Q, S, T>(rin, vsh[cy(a) + CM], soff, a, ps);
                if constexpr (XW) if (a > 0) xw[(a - 1) * 64] = n[a];
                // to this cell's compute base (the rest direction pulls from the cell itself)
                if constexpr (CT == 0) n[a] += (a > 0) ? tb(TB::DB(a)) : -tb(TB::SB(0));
            }
        } else {
            // one block per row (FP16): the column shift rides in the scalar offset
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                const uint32_t soff = (uint32_t)((int)(a * sa_b + (r0 - cx(a)) * sr_b) - cy(a) * (int)ES);
                n[a] = pload<Q, S, T>(rin, jb, soff, a, ps);
                if constexpr (XW) if (a > 0) xw[(a - 1) * 64] = n[a];
                // to this cell's compute base (the rest direction pulls from the cell itself)
                if constexpr (CT == 0) n[a] += (a > 0) ? tb(TB::DB(a)) : -tb(TB::SB(0));
            }
        }
    } else {
        // wrapped columns j - c2, c2 = -CM..CM (q2 is periodic), and their
        // byte offsets inside a row
        int colv[2 * CM + 1];
        uint32_t colb[2 * CM + 1];
#pragma unroll
        for (int k = -CM; k <= CM; ++k) {
            const int c = n2 >= CM ? wrap_col(j - k, n2) : ((j - k) % n2 + n2) % n2;
            colv[k + CM] = c;
            colb[k + CM] = (uint32_t)(c >> bs) * sb_b + (uint32_t)(c & bm) * ES;
        }
        const T *side_in = (const T *)d->side[pin];
        // WIDE: every source row lies in the window i - c_max .. i + c_max
        // (mirror rows at a wall included) or, for a periodic q1, in that
        // window shifted by +-n1 rows: three resources over 2 c_max + 1 rows
        // each (rows of a window outside the buffer are never accessed).
        // Otherwise one resource over the whole buffer.
        const __amdgpu_buffer_rsrc_t rw = WIDE ? row_rsrc(d->P[pin], row_b, i - CM, 2 * CM + 1)
                                               : make_rsrc(d->P[pin], (uint32_t)(plane * Q) * ES);
        const __amdgpu_buffer_rsrc_t rwlo = WIDE ? row_rsrc(d->P[pin], row_b, i - CM + n1, 2 * CM + 1) : rw;
        const __amdgpu_buffer_rsrc_t rwhi = WIDE ? row_rsrc(d->P[pin], row_b, i - CM - n1, 2 * CM + 1) : rw;
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            const int c2 = cy(a);
            int r, beta, wall;
            pull_source(i, a, n1, per1, bclo, bchi, r, beta, wall);
            const uint32_t cb = colb[c2 + CM];
            const int ti = i - cx(a);
            const bool wlo = WIDE && per1 && ti < 0, whi = WIDE && per1 && ti >= n1;
            // row inside its resource (a wrapped row sits in its window where
            // the unwrapped one would)
            const uint32_t rrel = WIDE ? (uint32_t)((wlo || whi ? ti : r) - (i - CM)) : (uint32_t)r;
            T v = pload<Q, S, T>(wlo ? rwlo : (whi ? rwhi : rw), cb, (uint32_t)beta * sa_b + rrel * sr_b, a, ps);
            if constexpr (XW) if (a > 0) xw[(a - 1) * 64] = v;
            if constexpr (CT == 0) v += (a > 0) ? tb(TB::DB(a)) : -tb(TB::SB(0));
            if (c2 != 0 && wall != 0) {
                const int sd = wall - 1;
                if ((sd ? bchi : bclo) == BC_MOVING) {
                    // App. B.3 moving-wall correction (tangential component)
                    const int k = sd ? (n1 - 1 - r) : r;
                    const T *sp = side_in + ((size_t)(sd * 2) * hw + k) * pitch + colv[c2 + CM];
                    const T mz = sp[0];
                    const T uz = sp[(size_t)hw * pitch];
                    const T U0 = (T)(sd ? d->ut_hi : d->ut_lo);
                    v += (T)(2.0 * weight<Q>(a) * c2 / T0d) * mz * (U0 - uz);
                }
            }
            n[a] = v;
        }
    }
    if constexpr (CT != 0 && BASES) add_bases<Q, T, CT>(tb, n);
    if constexpr (CT == 0 || BASES) phase_fence<CT>();
}

// what the store and the moments pass need besides the post-collision values
template <typename T>
struct CellOut {
    T m, dm, U1, U2, Ut1, Ut2, JF1, JF2;
};

// Moments, lagged (or iterated) force, physical velocity, equilibrium,
// momentum-flux correction, curvilinear correction and BGK relaxation of one
// cell: n are the pulled populations, Lo the lagged own-cell force sums
// sum_a A+^i_a s_a(q, t - 1) (Eq. compo-constr), s the post-collision values,
// all relative to the cell's compute base.  MOM stops after the force.
template <int Q, typename T, int CT, bool MOM, bool ITER, typename TBT>
__device__ __forceinline__ void collide_cell(const InstDesc *__restrict__ d, const TBT &tb, const T (&n)[Q], T Lo1,
                                             T Lo2, T (&s)[Q], CellOut<T> &o)
{
    constexpr int NP = npair<Q>();
    constexpr double T0d = lattice_T0<Q>();
    using TB = Tab<Q>;

    // ---- moments (in +-c pairs) ----
    T dm = n[0], mU1 = 0, mU2 = 0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int a = pair_rep(p), b = opp(a);
        const T sp = n[a] + n[b], dp = n[a] - n[b];
        dm += sp;
        if (cx(a) != 0) mU1 += (T)cx(a) * dp;
        if (cy(a) != 0) mU2 += (T)cy(a) * dp;
    }
    const T m = tb(TB::MB) + dm;
    T im;
    if constexpr (sizeof(T) == 4) im = __builtin_amdgcn_rcpf(m);   // 1-ulp hardware reciprocal
    else im = 1.0 / m;
    const T U1 = mU1 * im, U2 = mU2 * im;
    const T ma1 = m * (T)d->a1, ma2 = m * (T)d->a2;
    const T G11 = tb(TB::G11), G12 = tb(TB::G12), G22 = tb(TB::G22);
    const T omega = (T)d->omega, omw = (T)1 - (T)d->omega;
    // fixed-point passes of the force relation: only the ITER instances read
    // the count; the others do the single lagged pass, so the pulled
    // populations need not stay live past the collision
    const int iters = (MOM || !ITER) ? 0 : d->iters;

    T JF1, JF2, Ut1, Ut2;
    // pulled part of the force sum: sum_a A+_a n_{-a} (pass independent)
    T Ln1 = tb(TB::C1), Ln2 = tb(TB::C2);
    if constexpr (CT == 2) {
        T V1 = 0, V2 = 0;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int a = pair_rep(p), b = opp(a);
            tb.accA(a, n[b], V1, V2);
            tb.accA(b, n[a], V1, V2);
            sgroup<CT>();
        }
        tb.proj(V1, V2, Ln1, Ln2);
    } else {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int a = pair_rep(p), b = opp(a);
            Ln1 += tb(TB::A1(a)) * n[b] + tb(TB::A1(b)) * n[a];
            Ln2 += tb(TB::A2(a)) * n[b] + tb(TB::A2(b)) * n[a];
            sgroup<CT>();
        }
    }
    phase_fence<CT>();
    for (int it = 0;; ++it) {
        // ---- force: J F = -1/2 [C + sum_a A+_a (s_a + n_{-a})] + m a_ext ----
        T L1 = Ln1, L2 = Ln2;
        if (it == 0) {
            L1 += Lo1;
            L2 += Lo2;
        } else if constexpr (CT == 2) {
            T V1 = 0, V2 = 0;
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                tb.accA(a, s[a], V1, V2);
                sgroup<CT>();
            }
            tb.proj(V1, V2, L1, L2);
        } else {
#pragma unroll
            for (int a = 1; a < Q; ++a) {
                L1 += tb(TB::A1(a)) * s[a];
                L2 += tb(TB::A2(a)) * s[a];
                sgroup<CT>();
            }
        }
        JF1 = (T)-0.5 * L1 + ma1;
        JF2 = (T)-0.5 * L2 + ma2;
        Ut1 = U1 + (T)0.5 * JF1 * im;
        Ut2 = U2 + (T)0.5 * JF2 * im;
        if constexpr (MOM) break;

        // ---- odd part of the equilibrium and the momentum-flux correction ----
        const T GU1 = G11 * Ut1 + G12 * Ut2;
        const T GU2 = G12 * Ut1 + G22 * Ut2;
        const T uu = Ut1 * Ut1 + Ut2 * Ut2;
        const T uu3 = (T)(3.0 * T0d) * uu;
        const T uuT = (T)T0d * uu;
        T mO[NP], cUt[NP];
        T P11 = 0, P12 = 0, P22 = 0;
        T W[4] = {0, 0, 0, 0};   // rebuilt fields: the flux sums' vectors
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int a = pair_rep(p);
            const int c1 = cx(a), c2 = cy(a);
            const double w = weight<Q>(a);
            const double cc = (double)(c1 * c1 + c2 * c2);
            const T cU = (T)c1 * U1 + (T)c2 * U2;
            const T cut = (T)c1 * Ut1 + (T)c2 * Ut2;
            const T cGU = (T)c1 * GU1 + (T)c2 * GU2;
            const T q3 = (cut * cut - uu3) * cut;
            const T O = (T)(w * (1.0 / T0d + (4.0 * T0d - cc) / (2.0 * T0d * T0d))) * cU - (T)(w / T0d) * cGU +
                        (T)(w / (6.0 * T0d * T0d * T0d)) * q3 + tb(TB::K(p)) * cut;
            const T mo = m * O;
            mO[p] = mo;
            cUt[p] = cut;
            if constexpr (CT == 2) {
                tb.accS(a, mo, W);
            } else {
                if (c1 != 0) P11 += tb(TB::X11(p)) * mo;
                if (c2 != 0) P22 += tb(TB::X22(p)) * mo;
                P12 += tb(TB::X12(p)) * mo;
            }
            sgroup<CT>();
        }
        if constexpr (CT == 2) tb.flux(W, P11, P12, P22);
        const T trP = P11 + P22;
        phase_fence<CT>();

        // ---- even part, curvilinear correction and BGK (offset form) ----
        {
            constexpr double w0 = weight<Q>(0);
            const T feq0 = m * (tb(TB::D0) - (T)(w0 / (2.0 * T0d)) * uu) + dm * tb(TB::PHIB0);
            s[0] = omw * n[0] + omega * feq0 - (T)(w0 / T0d) * trP;
        }
        if constexpr (sizeof(T) == 4) {
            // omega feq_a + dN_a for a pair: the even part's quadratic forms in c
            // (omega m (c.Ut)^2 / (2 T0^2) from the equilibrium, c.P.c / T0^2 from
            // the correction) combine into one, c.M.c with M = P + (omega m / 2) Ut Ut,
            // and its constants into w C0 (FP32 compute: about 5% fewer vector
            // instructions; FP64 keeps the term-by-term form and its bits)
            const T om = omega * m, odm = omega * dm, hm = (T)0.5 * om;
            const T M11 = P11 + hm * (Ut1 * Ut1), M22 = P22 + hm * (Ut2 * Ut2), M12 = P12 + om * (Ut1 * Ut2);
            const T C0 = -(T)(1.0 / T0d) * trP - (T)(1.0 / (T0d * T0d)) * (hm * uuT);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int a = pair_rep(p), b = opp(a);
                const int c1 = cx(a), c2 = cy(a);
                const double w = weight<Q>(a);
                T ev = om * tb(TB::D(p)) + odm * tb(TB::PHIB(p)) + (T)w * C0;
                if (c1 != 0) ev += (T)(w * c1 * c1 / (T0d * T0d)) * M11;
                if (c1 != 0 && c2 != 0) ev += (T)(w * c1 * c2 / (T0d * T0d)) * M12;
                if (c2 != 0) ev += (T)(w * c2 * c2 / (T0d * T0d)) * M22;
                T od = omega * mO[p];
                if (c1 != 0) od += (T)(w * c1 / T0d) * JF1;
                if (c2 != 0) od += (T)(w * c2 / T0d) * JF2;
                s[a] = omw * n[a] + (ev + od);
                s[b] = omw * n[b] + (ev - od);
                sgroup<CT>();
            }
        } else {
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int a = pair_rep(p), b = opp(a);
                const int c1 = cx(a), c2 = cy(a);
                const double w = weight<Q>(a);
                const T mo = mO[p], cut = cUt[p];
                const T E = tb(TB::D(p)) + (T)(w / (2.0 * T0d * T0d)) * (cut * cut - uuT);
                const T base = m * E + dm * tb(TB::PHIB(p));
                const T feqA = base + mo;
                const T feqB = base - mo;
                const T even = (T)(w * c1 * c1 / (T0d * T0d)) * P11 + (T)(w * c1 * c2 / (T0d * T0d)) * P12 +
                               (T)(w * c2 * c2 / (T0d * T0d)) * P22 - (T)(w / T0d) * trP;
                const T odd = (T)(w * c1 / T0d) * JF1 + (T)(w * c2 / T0d) * JF2;
                s[a] = omw * n[a] + (omega * feqA + (even + odd));
                s[b] = omw * n[b] + (omega * feqB + (even - odd));
                sgroup<CT>();
            }
        }
        phase_fence<CT>();
        if (it >= iters) break;
    }
    o.m = m;
    o.dm = dm;
    o.U1 = U1;
    o.U2 = U2;
    o.Ut1 = Ut1;
    o.Ut2 = Ut2;
    o.JF1 = JF1;
    o.JF2 = JF2;
}

// FP32 storage: the update's mass and momentum projected onto their values in
// exact arithmetic.  In exact arithmetic the update keeps sum_a N_a and
// changes sum_a c_a N_a by exactly J F (with fourth-order isotropy the
// equilibrium carries momentum m U, the correction dN carries J F).
// Single-precision products of population size miss these moments by ~1e-7 of
// the local momentum, the same miss every step once the flow is steady, which
// acts as a spurious body force integrated over the slowest viscous time.  The
// miss is measured on the small differences N' - N and removed along
// w_a (1, c_a / T0), which changes no other moment of the update.  (FP16
// storage rounds far above this level.)
template <int Q, typename T, typename S>
__device__ __forceinline__ void project_update(const T (&n)[Q], T (&s)[Q], T JF1, T JF2)
{
    if constexpr (sizeof(T) == 4 && sizeof(S) == 4) {
        constexpr double T0d = lattice_T0<Q>();
        T r0 = 0, r1 = -JF1, r2 = -JF2;
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            const T dd = s[a] - n[a];
            r0 += dd;
            if (cx(a) != 0) r1 += (T)cx(a) * dd;
            if (cy(a) != 0) r2 += (T)cy(a) * dd;
        }
        const T e1 = r1 * (T)(1.0 / T0d), e2 = r2 * (T)(1.0 / T0d);
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            T corr = r0;
            if (cx(a) != 0) corr += (T)cx(a) * e1;
            if (cy(a) != 0) corr += (T)cy(a) * e2;
            s[a] -= (T)weight<Q>(a) * corr;
        }
    }
}

// Store the post-collision values of cell (i, j) (moved to the storage base
// and encoded), with LAGW the lagged force sums the next step of the
// lag-buffer kernels reads, and the moving walls' side state: m and Ut^2 of
// the rows a wall pulls from (App. B.3).
template <int Q, typename T, typename S, int CT, bool LAGW, bool WIDE, typename TBT>
__device__ __forceinline__ void store_cell(const InstDesc *__restrict__ d, const TBT &tb, int i, int j, int pin,
                                           const T (&s)[Q], const CellOut<T> &o)
{
    using TB = Tab<Q>;
    constexpr uint32_t ES = sizeof(S);
    const uint32_t sa_b = (uint32_t)d->sa * ES, sb_b = (uint32_t)d->sb * ES;
    const uint32_t jb = (uint32_t)(j >> d->bs) * sb_b + (uint32_t)(j & d->bm) * ES;
    const __amdgpu_buffer_rsrc_t rout = WIDE ? row_rsrc(d->P[pin ^ 1], (size_t)d->sr * ES, i, 1)
                                             : make_rsrc(d->P[pin ^ 1], (uint32_t)(d->plane * Q) * ES);
    const uint32_t rowb = WIDE ? 0u : (uint32_t)i * (uint32_t)d->sr * ES;
    const PScale<Q, S, T, CT == 0> ps;
    T Lx1 = 0, Lx2 = 0;
    if constexpr (CT == 2) {
        // rebuilt fields: the storage base is the compute base (the local
        // rest state, or none in FP64), so the store needs no per-direction
        // base terms; the force sums are formed on the vectors
        T V1 = 0, V2 = 0;
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            pstore<Q, S, T>(rout, jb, (uint32_t)a * sa_b + rowb, a, s[a]);
            if constexpr (LAGW) {
                const T v = pdec<Q, S, T>(penc<Q, S, T>(s[a], a), a, ps);   // as stored
                if (a > 0) tb.accA(a, v, V1, V2);
            }
            sgroup<CT>();
        }
        if constexpr (LAGW) tb.proj(V1, V2, Lx1, Lx2);
    } else {
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            const T st = s[a] + tb(TB::SB(a));                                  // storage base
            pstore<Q, S, T>(rout, jb, (uint32_t)a * sa_b + rowb, a, st);
            if constexpr (LAGW) {
                const T v = pdec<Q, S, T>(penc<Q, S, T>(st, a), a, ps) - tb(TB::SB(a));  // as stored, compute base
                if (a > 0) {
                    Lx1 += tb(TB::A1(a)) * v;
                    Lx2 += tb(TB::A2(a)) * v;
                }
            }
            sgroup<CT>();
        }
    }
    if constexpr (LAGW) {
        constexpr uint32_t ET = sizeof(T);
        const uint32_t lsa_b = (uint32_t)d->lsa * ET;
        const uint32_t jt = (uint32_t)j * ET;
        const __amdgpu_buffer_rsrc_t rlago = WIDE ? row_rsrc(d->lag[pin ^ 1], (size_t)d->lsr * ET, i, 1)
                                                  : make_rsrc(d->lag[pin ^ 1], 2 * (uint32_t)d->plane * ET);
        const uint32_t rowt = WIDE ? 0u : (uint32_t)i * (uint32_t)d->lsr * ET;
        bstore<T, T>(rlago, jt, rowt, Lx1);
        bstore<T, T>(rlago, jt, lsa_b + rowt, Lx2);
    }
    const int n1 = d->n1, hw = d->hw, pitch = d->pitch;
    T *side_out = (T *)d->side[pin ^ 1];
    if (d->bc_lo == BC_MOVING && i < hw) {
        side_out[((size_t)0 * hw + i) * pitch + j] = o.m;
        side_out[((size_t)1 * hw + i) * pitch + j] = o.Ut2;
    }
    if (d->bc_hi == BC_MOVING && i >= n1 - hw) {
        const int k = n1 - 1 - i;
        side_out[((size_t)2 * hw + k) * pitch + j] = o.m;
        side_out[((size_t)3 * hw + k) * pitch + j] = o.Ut2;
    }
}

// Lagged own-cell force sums sum_a A+^i_a s_a(q, t - 1) from the own cell's
// stored post-collision values (the sums the lag-buffer kernels store, formed
// in the same order, so bitwise the same)
template <int Q, typename T, typename S, bool WIDE, typename TBT>
__device__ __forceinline__ void own_lag_global(const InstDesc *__restrict__ d, const TBT &tb, int i, int j, int pin,
                                               T &Lo1, T &Lo2)
{
    using TB = Tab<Q>;
    constexpr uint32_t ES = sizeof(S);
    const uint32_t sa_b = (uint32_t)d->sa * ES, sb_b = (uint32_t)d->sb * ES;
    const uint32_t jb = (uint32_t)(j >> d->bs) * sb_b + (uint32_t)(j & d->bm) * ES;
    const __amdgpu_buffer_rsrc_t rin = WIDE ? row_rsrc(d->P[pin], (size_t)d->sr * ES, i, 1)
                                            : make_rsrc(d->P[pin], (uint32_t)(d->plane * Q) * ES);
    const uint32_t rowb = WIDE ? 0u : (uint32_t)i * (uint32_t)d->sr * ES;
    const PScale<Q, S, T> ps;
    Lo1 = 0;
    Lo2 = 0;
#pragma unroll
    for (int a = 1; a < Q; ++a) {
        const T v = pload<Q, S, T>(rin, jb, (uint32_t)a * sa_b + rowb, a, ps) - tb(TB::SB(a));
        Lo1 += tb(TB::A1(a)) * v;
        Lo2 += tb(TB::A2(a)) * v;
    }
}

// ---------------------------------------------------------------------------
// The step of the lag-buffer kernels: one row segment of 64 columns per wave;
// the lagged force sums of the own cell are read from, and the next ones
// written to, a per-cell buffer.  MOM = true computes and writes the moments
// instead of colliding (for per-row tables it forms the lagged sums from the
// own cell's stored values, which serves grids stepped by either kernel).
// ---------------------------------------------------------------------------
template <int Q, typename T, typename S, int CT, bool MOM, bool ITER, bool WIDE>
__device__ __forceinline__ void step_tile(const InstDesc *__restrict__ insts, const int4 tl, int par)
{
    using TB = Tab<Q>;

    const InstDesc *__restrict__ d = insts + tl.x;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int i = tl.y + wave;
    const int n1 = d->n1, n2 = d->n2;
    const int j0 = tl.z;
    const int j = j0 + (int)(threadIdx.x & 63);
    const int pin = (par ^ d->par0) & 1;

    // lagged own-cell force sums, formed when the previous step produced
    // N'(q, t-1); each is read once, so non-temporal whatever the policy of
    // the population loads (measured: the D2Q21 FP32 group 298-299 against
    // 300 us, one 4096 x 16384 FP32 grid 2002 against 2019 us)
    auto load_lag = [&](T &L1, T &L2) {
        constexpr uint32_t ET = sizeof(T);
        const uint32_t lsa_b = (uint32_t)d->lsa * ET;
        const __amdgpu_buffer_rsrc_t rlag = WIDE ? row_rsrc(d->lag[pin], (size_t)d->lsr * ET, i, 1)
                                                 : make_rsrc(d->lag[pin], 2 * (uint32_t)d->plane * ET);
        const uint32_t jt = (uint32_t)j * ET, rowt = WIDE ? 0u : (uint32_t)i * (uint32_t)d->lsr * ET;
        L1 = bload<T, T, 2>(rlag, jt, rowt);
        L2 = bload<T, T, 2>(rlag, jt, lsa_b + rowt);
    };

    typename TabSel<Q, T, CT>::type tb;
    T n[Q], s[Q];
    T Lo1, Lo2;
    if constexpr (CT == 2) {
        if (tl.y >= n1) return;   // padding tile (the whole workgroup)
        const bool act = i < n1 && j < n2;
        if constexpr (sizeof(T) == 8) {
            // the geometry goes to LDS while the pulls and force sums, which
            // need none of it, are loaded; every wave reaches the barrier
            const double *geo_lds = stage_geometry<Q, T>(d, tl, wave);
            if (act) {
                pull_cell<Q, T, S, CT, WIDE, false>(d, tb, i, j, j0, pin, n);
                load_lag(Lo1, Lo2);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (!act) return;
            tb.setup(d, geo_lds, wave, j - j0, i, j);
        } else {
            double ref[GE_NF];
            const float *geo_lds = stage_geometry_f<Q>(d, tl, wave, ref);
            if (act) {
                pull_cell<Q, T, S, CT, WIDE, false>(d, tb, i, j, j0, pin, n);
                load_lag(Lo1, Lo2);
            }
            __syncthreads();
            if (!act) return;
            tb.setup(d, geo_lds, ref, wave, j - j0, i, j);
        }
        add_bases<Q, T, CT>(tb, n);
    } else if constexpr (xch_step<Q, S, CT, MOM>()) {
        extern __shared__ float xch_lds[];
        T *xt = (T *)xch_lds;
        if (tl.y >= n1) return;   // padding tile (the whole workgroup)
        const int nw = (int)(blockDim.x >> 6), lane = (int)(threadIdx.x & 63);
        const bool act = i < n1 && j < n2;
        tb.p = (const T *)d->tab + (size_t)i * TB::STRIDE;
        tb.s = 1;
        // partner q + c_a of direction a inside the tile (an active cell of
        // the workgroup's rows and of this wave's 64 columns)
        auto inside = [&](int a) {
            const int pr = wave + cx(a), pl = lane + cy(a);
            return pr >= 0 && pr < nw && i + cx(a) < n1 && pl >= 0 && pl < 64 && j + cy(a) < n2;
        };
        T own[Q];
        if (act) {
            // the own cell's stored values that no partner in the tile pulls,
            // loaded first so that they are in flight with the pulls.  Every
            // lane issues the load, without a branch, so that the loads
            // overlap; a lane whose value comes from the tile loads from
            // offset 2^31, past the end of the resource (2 GiB at most), which
            // returns zero without touching memory
            constexpr uint32_t ES = sizeof(S);
            const uint32_t sa_b = (uint32_t)d->sa * ES, sb_b = (uint32_t)d->sb * ES;
            const uint32_t jb = (uint32_t)(j >> d->bs) * sb_b + (uint32_t)(j & d->bm) * ES;
            const __amdgpu_buffer_rsrc_t rown = WIDE ? row_rsrc(d->P[pin], (size_t)d->sr * ES, i, 1)
                                                     : make_rsrc(d->P[pin], (uint32_t)(d->plane * Q) * ES);
            const uint32_t rowb = WIDE ? 0u : (uint32_t)i * (uint32_t)d->sr * ES;
            const PScale<Q, S, T> ps;
#pragma unroll
            for (int a = 1; a < Q; ++a)
                own[a] = pload<Q, S, T>(rown, inside(a) ? 0x80000000u : jb + (uint32_t)a * sa_b + rowb, 0u, a, ps);
            pull_cell<Q, T, S, CT, WIDE, true, true>(d, tb, i, j, j0, pin, n, xt + wave * (Q - 1) * 64 + lane);
        }
        __syncthreads();
        if (!act) return;
        // lagged own-cell force sums sum_a A+^i_a N'_a(q, t - 1), in the
        // stored sums' order; the tile index is clamped into the tile, so
        // the read stays inside it whichever way the select goes
        Lo1 = 0;
        Lo2 = 0;
#pragma unroll
        for (int a = 1; a < Q; ++a) {
            const int pr = min(max(wave + cx(a), 0), nw - 1), pl = min(max(lane + cy(a), 0), 63);
            const T x = xt[(pr * (Q - 1) + a - 1) * 64 + pl];
            const T v = (inside(a) ? x : own[a]) - tb(TB::SB(a));
            Lo1 += tb(TB::A1(a)) * v;
            Lo2 += tb(TB::A2(a)) * v;
        }
    } else {
        if (i >= n1 || j >= n2) return;
        if constexpr (CT == 1) {
            tb.p = (const T *)d->tab + (size_t)i * n2 + j;
            tb.s = d->ncell;
        } else {
            tb.p = (const T *)d->tab + (size_t)i * TB::STRIDE;
            tb.s = 1;
        }
        pull_cell<Q, T, S, CT, WIDE>(d, tb, i, j, j0, pin, n);
        if constexpr (MOM && CT == 0)
            own_lag_global<Q, T, S, WIDE>(d, tb, i, j, pin, Lo1, Lo2);
        else
            load_lag(Lo1, Lo2);
    }

    CellOut<T> o;
    collide_cell<Q, T, CT, MOM, ITER>(d, tb, n, Lo1, Lo2, s, o);

    if constexpr (!MOM) project_update<Q, T, S>(n, s, o.JF1, o.JF2);

    phase_fence<CT>();
    if constexpr (MOM) {
        const int c = i * n2 + j;
        const int e = CT ? c : i;
        double *mo = d->mom;
        const size_t nc = (size_t)d->ncell;
        mo[c] = d->mB64[e] + (double)o.dm;
        mo[nc + c] = (double)o.U1;
        mo[2 * nc + c] = (double)o.U2;
        mo[3 * nc + c] = (double)o.Ut1;
        mo[4 * nc + c] = (double)o.Ut2;
    } else {
        store_cell<Q, T, S, CT, !xch_step<Q, S, CT, MOM>(), WIDE>(d, tb, i, j, pin, s, o);
    }
}

// One tile (row segment of 64 columns per wave) per workgroup.  The tile
// table holds (instance, first row, first column, lattice).  WIDE instances
// serve population buffers of 2 GiB and more.
template <int Q, typename T, typename S, int CT, bool MOM, bool ITER, bool WIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CT == 2 && sizeof(T) == 4 && Q == 21 ? (ITER ? 4 : 5) : 1)))
void k_step(const InstDesc *__restrict__ insts, const int4 *__restrict__ tiles, int par)
{
    step_tile<Q, T, S, CT, MOM, ITER, WIDE>(insts, tiles[blockIdx.x], par);
}

// D2Q9 and D2Q21 tiles in one launch: the lattice is the tile's fourth field
// (wave-uniform, so each workgroup runs one of the two bodies).
template <typename T, typename S, int CT, bool MOM, bool ITER>
__global__ __launch_bounds__(256) void k_step_mixed(const InstDesc *__restrict__ insts,
                                                    const int4 *__restrict__ tiles, int par)
{
    const int4 tl = tiles[blockIdx.x];
    if (tl.w == 9)
        step_tile<9, T, S, CT, MOM, ITER, false>(insts, tl, par);
    else
        step_tile<21, T, S, CT, MOM, ITER, false>(insts, tl, par);
}

} // namespace lbm
