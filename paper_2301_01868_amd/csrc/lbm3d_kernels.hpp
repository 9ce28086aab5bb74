// Device code of the three-dimensional step (arXiv:2301.01868, Sec. 2 for
// i = 1, 2, 3; boundaries of App. B on the q1 sides, q2 and q3 periodic).
//
// FP64 populations in particle numbers N = J f, in which J cancels from the
// update:
//   m = sum N,  m U^i = sum c^i N                                   (Eqs. moments, vcomp)
//   J F^i = -1/2 sum_a A+^i_a [N'_a(q, t-1) + N_{-a}(q, t)] + m a^i  (Eq. compo-constr,
//            with A-^i_a = -A+^i_{-a} and the paper's one-step lag)
//   Ut = U + J F / (2 m)
//   J f^eq_a = m phi_a                                              (Eq. equilibrium)
//   J dPi^ij = -1/2 (1 - 1/(2 tau)) sum_a c^i_a (A+^j_a + A+^j_{-a}) m phi_a   (Eq. delta-flux)
//   dN_a = w_a [c.JF / T0 + (c^j c^k / T0 - delta^jk) J dPi^jk / T0]          (Eq. deltaN)
//   N'_a = N_a - (N_a - m phi_a) / tau + dN_a                        (Eqs. collide, lbe)
// with A+^i_a(q) = sum_j c^j_a Theta^i_j(q + c_a, q) (Eq. gamma) from per-row
// tables (grids whose metric terms depend on q1 only).  The lagged sum
// sum_a A+^i_a N'_a(q, t-1) is formed by the step that produces N'(q, t-1)
// and kept as three values per cell.
//
// The equilibrium is the index sum of Eq. (equilibrium) contracted once per
// cell into the symmetric tensors
//   A2^ij = (g^ij - delta^ij) T0 + Ut^i Ut^j,
//   B3^ijk = T0 [(g^ij Ut^k - delta^ij U^k) + (cyclic)] + Ut^i Ut^j Ut^k,
//   V^i = sum_j B3^ijj,
// so that per direction
//   phi_a = w_a [1 + c.U / T0 + (c.A2.c / T0 - tr A2) / (2 T0)
//               + (B3(c, c, c) - 3 T0 c.V) / (6 T0^3)],
// the Hermite polynomials (c^i c^j / T0 - delta^ij) and
// (c^i c^j c^k - T0 (c^i delta^jk + c^j delta^ki + c^k delta^ij)) contracted
// with the symmetric tensors of the equilibrium.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lbm3d_lattice.hpp"

namespace lbm3 {

enum { BC_PERIODIC = 0, BC_NOSLIP = 1, BC_MOVING = 2 };

// compile-time loop: f(std::integral_constant<int, I>) for I = B .. E - 1, so
// every lattice constant indexed by I folds at compile time
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

// The equilibrium as a polynomial in c: phi_a = w_a sum_k K_k P_k(c_a) over
// the 20 monomials P_k of degree <= 3 (1; c_x; c_x c_y for x <= y; c_x c_y c_z
// for x <= y <= z), with per-cell coefficients K from U, Ut and g^ij.  The
// momentum-flux correction is then a per-row moment table contracted with K:
//   J dPi^ij = kpi m sum_k K_k T^ij_k,  T^ij_k = sum_a w_a c^i_a S^j_a P_k(c_a),
// S^j_a = A+^j_a + A+^j_{-a}, the same sum over directions in another order.
// The correction dN_a of Eq. (deltaN) contracts dPi with the symmetric c_a c_a,
// so only the symmetric parts are needed: for x <= y the table holds
// U^xy_k = T^xy_k + T^yx_k (x < y) or T^xx_k, and
//   sum_ij c^i c^j J dPi^ij = kpi m sum_{x <= y} c^x c^y sum_k K_k U^xy_k.
constexpr int NK = 20;
// per-row table: g^11, g^12, g^13, g^22, g^23, g^33; A+^i_a at 6 + 3 a + i;
// U^xy_k at TT + sym2(x, y) NK + k
constexpr int TG = 6 + 3 * Q;
constexpr int TT = TG;
constexpr int TW = TG + 6 * NK;
// per-cell geometry output: J, the six g^ij, A+ (3 Q)
constexpr int GW = 1 + TG;

// uniform (scalar-cache) view of constant data: the descriptor and the per-row tables
template <typename T>
using cptr3 = const __attribute__((address_space(4))) T *;

struct Desc3 {
    double *P[2];        // populations, element ((i n2 + j) Q + a) pitch + k
    double *side[2];     // moving-wall side state [2 walls][3 fields: m, Ut^2, Ut^3][CMAX rows][n2][pitch]
    double *lag[2];      // lagged own-cell force sums sum_a A+^i_a N'_a, [3][n1 n2][pitch]
    const double *tab;   // per-row tables [n1][TW]
    const double *Jrow;  // per-row volume [n1]
    double *mom;         // moments output [7][ncell]: m, U^1..3, Ut^1..3
    int n1, n2, n3, pitch;
    long long ncell;
    int periodic1, bc_lo, bc_hi;
    double ut_lo[2], ut_hi[2];
    double a[3], omega, kpi;
};

__host__ __device__ inline size_t pidx3(int n2, int pitch, int i, int j, int a, int k)
{
    return ((size_t)(i * n2 + j) * Q + a) * pitch + k;
}
__host__ __device__ inline size_t sidx3(int n2, int pitch, int wall, int field, int row, int j, int k)
{
    return (((size_t)(wall * 3 + field) * CMAX + row) * n2 + j) * pitch + k;
}
__device__ inline int wrap3(int x, int n)
{
    if (n >= CMAX) return x < 0 ? x + n : (x >= n ? x - n : x);
    return ((x % n) + n) % n;
}

// Source of N_a(i, .): row r and direction beta of the post-collision field,
// and the wall crossed (0 none, 1 low, 2 high); beyond a wall the mirror image
// of the source row, with the reversed (no-slip) or specular (moving wall)
// direction (App. B).
__host__ __device__ inline void source_row(int i, int a, int n1, int per1, int bclo, int bchi, int &r, int &beta,
                                           int &wall)
{
    const int ti = i - cvec(a, 0);
    r = ti;
    beta = a;
    wall = 0;
    if (ti < 0) {
        if (per1) {
            r = ti + n1;
        } else {
            r = -1 - ti;
            wall = 1;
            beta = bclo == BC_NOSLIP ? opp(a) : specular(a);
        }
    } else if (ti >= n1) {
        if (per1) {
            r = ti - n1;
        } else {
            r = 2 * n1 - 1 - ti;
            wall = 2;
            beta = bchi == BC_NOSLIP ? opp(a) : specular(a);
        }
    }
}

// the wave's cell: tile t = ((i n2 + j) nkb + kb), lanes along q3
struct Cell3 {
    int i, j, k;
};
__device__ inline bool cell_of(int n1, int n2, int n3, Cell3 &c)
{
    const int nkb = (n3 + 63) >> 6;
    const int t = (int)blockIdx.x;
    const int kb = t % nkb, ij = t / nkb;
    c.i = ij / n2;
    c.j = ij - c.i * n2;
    c.k = kb * 64 + (int)(threadIdx.x & 63);
    return c.i < n1 && c.k < n3;
}
__device__ inline bool cell_of(const Desc3 &d, Cell3 &c) { return cell_of(d.n1, d.n2, d.n3, c); }

__host__ __device__ constexpr int sym2(int x, int y)
{
    return x <= y ? (x == 0 ? y : (x == 1 ? 2 + y : 5)) : sym2(y, x);
}
__host__ __device__ constexpr int sym3(int x, int y, int z)
{
    // sort (x, y, z), then index the 10 non-decreasing triples
    return x > y ? sym3(y, x, z) : (y > z ? sym3(x, z, y) : (x == 0 ? (y == 0 ? z : (y == 1 ? 2 + z : 5)) : (x == 1 ? (y == 1 ? 5 + z : 8) : 9)));
}
// monomial k of c (k = 0: 1; 1..3: c_x; 4..9: c_x c_y, x <= y; 10..19:
// c_x c_y c_z, x <= y <= z, in the sym2 / sym3 orders) and its multiplicity
// in a symmetric contraction
__host__ __device__ constexpr int mono(int k, int c0, int c1, int c2)
{
    const int c[3] = {c0, c1, c2};
    if (k == 0) return 1;
    if (k < 4) return c[k - 1];
    if (k < 10) {
        constexpr int px[6] = {0, 0, 0, 1, 1, 2}, py[6] = {0, 1, 2, 1, 2, 2};
        return c[px[k - 4]] * c[py[k - 4]];
    }
    constexpr int tx[10] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 2}, ty[10] = {0, 0, 0, 1, 1, 2, 1, 1, 2, 2},
                  tz[10] = {0, 1, 2, 1, 2, 2, 1, 2, 2, 2};
    return c[tx[k - 10]] * c[ty[k - 10]] * c[tz[k - 10]];
}
__host__ __device__ constexpr int mult(int k)
{
    constexpr int m2[6] = {1, 2, 2, 1, 2, 1};
    constexpr int m3[10] = {1, 3, 3, 3, 6, 3, 1, 3, 3, 1};
    return k < 4 ? 1 : (k < 10 ? m2[k - 4] : m3[k - 10]);
}

// Coefficients K of phi_a = w_a sum_k K_k P_k(c_a) (see NK): the index sum of
// Eq. (equilibrium) contracted into the symmetric tensors
//   A2^xy = (g^xy - delta^xy) T0 + Ut^x Ut^y,
//   B3^xyz = T0 [(g^xy Ut^z - delta^xy U^z) + (cyclic)] + Ut^x Ut^y Ut^z,
//   V^x = sum_y B3^xyy,
// through the Hermite polynomials: K_0 = 1 - tr A2 / (2 T0),
// K_x = U^x / T0 - V^x / (2 T0^2), K_xy = mult A2^xy / (2 T0^2),
// K_xyz = mult B3^xyz / (6 T0^3).  G holds g^11 g^12 g^13 g^22 g^23 g^33.
__device__ __forceinline__ void eq_coeffs(const double G[6], const double U[3], const double Ut[3], double K[NK])
{
    double trA2 = 0.0, V[3] = {0.0, 0.0, 0.0};
    sfor<0, 3>([&](auto X) {
        constexpr int x = decltype(X)::value;
        sfor<x, 3>([&](auto Y) {
            constexpr int y = decltype(Y)::value;
            const double a2 = (G[sym2(x, y)] - (x == y ? 1.0 : 0.0)) * T0 + Ut[x] * Ut[y];
            if constexpr (x == y) trA2 += a2;
            K[4 + sym2(x, y)] = a2 * (mult(4 + sym2(x, y)) / (2.0 * T0 * T0));
            sfor<y, 3>([&](auto Z) {
                constexpr int z = decltype(Z)::value;
                const double b3 = T0 * ((G[sym2(x, y)] * Ut[z] - (x == y ? U[z] : 0.0)) +
                                        (G[sym2(y, z)] * Ut[x] - (y == z ? U[x] : 0.0)) +
                                        (G[sym2(z, x)] * Ut[y] - (z == x ? U[y] : 0.0))) +
                                  Ut[x] * Ut[y] * Ut[z];
                K[10 + sym3(x, y, z)] = b3 * (mult(10 + sym3(x, y, z)) / (6.0 * T0 * T0 * T0));
                // V^w = sum_v B3^wvv: this (x, y, z) contributes where two indices agree
                if constexpr (x == y && y == z) V[x] += b3;
                else if constexpr (x == y) V[z] += b3;
                else if constexpr (y == z) V[x] += b3;
            });
        });
    });
    K[0] = 1.0 - trA2 * (1.0 / (2.0 * T0));
    sfor<0, 3>([&](auto X) {
        constexpr int x = decltype(X)::value;
        K[1 + x] = U[x] * (1.0 / T0) - V[x] * (1.0 / (2.0 * T0 * T0));
    });
}
// the even (degree 0 and 2) and odd (degree 1 and 3) parts of sum_k K_k P_k(c_A):
// phi_A = w_A (E + O) and phi_-A = w_A (E - O)
template <int A>
__device__ __forceinline__ void phi_parts(const double K[NK], double &E, double &O)
{
    E = 0.0;
    O = 0.0;
    sfor<0, NK>([&](auto Kc) {
        constexpr int k = decltype(Kc)::value;
        constexpr int p = mono(k, cvec(A, 0), cvec(A, 1), cvec(A, 2));
        constexpr bool odd = (k >= 1 && k < 4) || k >= 10;
        if constexpr (p != 0) {
            if constexpr (odd) O += (double)p * K[k];
            else E += (double)p * K[k];
        }
    });
}
template <int A>
__device__ __forceinline__ double phi_poly(const double K[NK])
{
    double s = 0.0;
    sfor<0, NK>([&](auto Kc) {
        constexpr int k = decltype(Kc)::value;
        constexpr int p = mono(k, cvec(A, 0), cvec(A, 1), cvec(A, 2));
        if constexpr (p != 0) s += (double)p * K[k];
    });
    return weight(A) * s;
}

// MOM = true writes the moments the next step would see instead of colliding
template <bool MOM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MOM ? 1 : 3)))
void k_step3(const Desc3 *__restrict__ dp, int par)
{
    const cptr3<Desc3> d = (cptr3<Desc3>)dp;
    Cell3 c;
    if (!cell_of(d->n1, d->n2, d->n3, c)) return;
    const int pin = par & 1;
    const double *__restrict__ P = d->P[pin];
    const cptr3<double> tb = (cptr3<double>)(d->tab + (size_t)c.i * TW);
    const double *__restrict__ side_in = d->side[pin];

    // ---- pull (Eq. adv, App. B) ----
    double n[Q];
    if (c.i >= CMAX && c.i < d->n1 - CMAX) {
        // rows i - c_max .. i + c_max, all inside the grid: one buffer
        // resource based at row i - c_max; the wave's 64 cells share (i, j),
        // so a direction's source offset is a scalar part (row, wrapped j,
        // direction) plus one of 2 c_max + 1 per-lane k offsets (wrapped
        // along the periodic q3)
        const int n2 = d->n2, pitch = d->pitch;
        const size_t plane_b = (size_t)n2 * Q * pitch * sizeof(double);   // one row i
        const __amdgpu_buffer_rsrc_t rin = __builtin_amdgcn_make_buffer_rsrc(
            (void *)((const char *)P + (size_t)(c.i - CMAX) * plane_b), (short)0, (int)(uint32_t)((2 * CMAX + 1) * plane_b),
            0x00020000);
        uint32_t vk[2 * CMAX + 1];
#pragma unroll
        for (int s = -CMAX; s <= CMAX; ++s) vk[s + CMAX] = (uint32_t)wrap3(c.k - s, d->n3) * (uint32_t)sizeof(double);
        sfor<0, Q>([&](auto Aic) {
            constexpr int a = decltype(Aic)::value;
            const int jj = wrap3(c.j - cvec(a, 1), n2);
            const uint32_t soff =
                (uint32_t)((((CMAX - cvec(a, 0)) * n2 + jj) * Q + a) * pitch) * (uint32_t)sizeof(double);
            n[a] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rin, vk[cvec(a, 2) + CMAX], soff, 2));
        });
    } else {
        // rows at a wall (mirror sources, App. B) or at a periodic q1 wrap
        sfor<0, Q>([&](auto Aic) {
            constexpr int a = decltype(Aic)::value;
            int r, beta, wall;
            source_row(c.i, a, d->n1, d->periodic1, d->bc_lo, d->bc_hi, r, beta, wall);
            const int jj = wrap3(c.j - cvec(a, 1), d->n2), kk = wrap3(c.k - cvec(a, 2), d->n3);
            double v = P[pidx3(d->n2, d->pitch, r, jj, beta, kk)];
            if constexpr (cvec(a, 1) != 0 || cvec(a, 2) != 0) {
                if (wall != 0) {
                    const int sd = wall - 1;
                    if ((sd ? d->bc_hi : d->bc_lo) == BC_MOVING) {
                        // App. B.3 correction, both tangential components
                        const int row = sd ? d->n1 - 1 - r : r;
                        const double mz = side_in[sidx3(d->n2, d->pitch, sd, 0, row, jj, kk)];
                        const double U02 = sd ? d->ut_hi[0] : d->ut_lo[0], U03 = sd ? d->ut_hi[1] : d->ut_lo[1];
                        double corr = 0.0;
                        if constexpr (cvec(a, 1) != 0)
                            corr += cvec(a, 1) * (U02 - side_in[sidx3(d->n2, d->pitch, sd, 1, row, jj, kk)]);
                        if constexpr (cvec(a, 2) != 0)
                            corr += cvec(a, 2) * (U03 - side_in[sidx3(d->n2, d->pitch, sd, 2, row, jj, kk)]);
                        v += 2.0 * weight(a) / T0 * mz * corr;
                    }
                }
            }
            n[a] = v;
        });
    }

    // ---- moments ----
    double m = 0.0, mU[3] = {0.0, 0.0, 0.0};
    sfor<0, Q>([&](auto Aic) {
        constexpr int a = decltype(Aic)::value;
        m += n[a];
        if constexpr (cvec(a, 0) != 0) mU[0] += cvec(a, 0) * n[a];
        if constexpr (cvec(a, 1) != 0) mU[1] += cvec(a, 1) * n[a];
        if constexpr (cvec(a, 2) != 0) mU[2] += cvec(a, 2) * n[a];
    });
    const double im = 1.0 / m;
    const double U[3] = {mU[0] * im, mU[1] * im, mU[2] * im};

    // ---- force: the lagged own-cell sums sum_a A+_a N'_a(q, t-1), formed when
    // the previous step produced N'(q, t-1), plus sum_a A+_a N_{-a}(q, t) ----
    const size_t lrow = ((size_t)c.i * d->n2 + c.j) * d->pitch + c.k, lpl = (size_t)d->n1 * d->n2 * d->pitch;
    double L[3] = {d->lag[pin][lrow], d->lag[pin][lpl + lrow], d->lag[pin][2 * lpl + lrow]};
    sfor<1, Q>([&](auto Aic) {
        constexpr int a = decltype(Aic)::value;
        L[0] += tb[6 + 3 * a + 0] * n[opp(a)];
        L[1] += tb[6 + 3 * a + 1] * n[opp(a)];
        L[2] += tb[6 + 3 * a + 2] * n[opp(a)];
        __builtin_amdgcn_sched_barrier(0);
    });
    double JF[3], Ut[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        JF[e] = -0.5 * L[e] + m * d->a[e];
        Ut[e] = U[e] + 0.5 * JF[e] * im;
    }
    if constexpr (MOM) {
        const size_t cell = ((size_t)c.i * d->n2 + c.j) * d->n3 + c.k, nc = (size_t)d->ncell;
        d->mom[cell] = m;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            d->mom[(1 + e) * nc + cell] = U[e];
            d->mom[(4 + e) * nc + cell] = Ut[e];
        }
        return;
    } else {
        // side state of the moving walls: m, Ut^2, Ut^3 of the rows a wall
        // pulls from (for the next step; written here so that none of it
        // stays live through the store)
        double *__restrict__ so = d->side[pin ^ 1];
        if (d->bc_lo == BC_MOVING && c.i < CMAX) {
            so[sidx3(d->n2, d->pitch, 0, 0, c.i, c.j, c.k)] = m;
            so[sidx3(d->n2, d->pitch, 0, 1, c.i, c.j, c.k)] = Ut[1];
            so[sidx3(d->n2, d->pitch, 0, 2, c.i, c.j, c.k)] = Ut[2];
        }
        if (d->bc_hi == BC_MOVING && c.i >= d->n1 - CMAX) {
            const int row = d->n1 - 1 - c.i;
            so[sidx3(d->n2, d->pitch, 1, 0, row, c.j, c.k)] = m;
            so[sidx3(d->n2, d->pitch, 1, 1, row, c.j, c.k)] = Ut[1];
            so[sidx3(d->n2, d->pitch, 1, 2, row, c.j, c.k)] = Ut[2];
        }
        // ---- equilibrium coefficients of the cell ----
        const double G[6] = {tb[0], tb[1], tb[2], tb[3], tb[4], tb[5]};   // 11 12 13 22 23 33
        double K[NK];
        eq_coeffs(G, U, Ut, K);
        // ---- the momentum-flux correction through the per-row moment table
        // (its symmetric parts: Q^xy = J dPi^xy + J dPi^yx for x < y, J dPi^xx) ----
        double Qs[6];
        sfor<0, 6>([&](auto XY) {
            constexpr int xy = decltype(XY)::value;
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < NK; ++k) s += tb[TT + xy * NK + k] * K[k];
            Qs[xy] = d->kpi * m * s;
            __builtin_amdgcn_sched_barrier(0);
        });
        const double trPi = Qs[sym2(0, 0)] + Qs[sym2(1, 1)] + Qs[sym2(2, 2)];

        // ---- correction, BGK, store; the next step's lagged force sums ----
        // N'_a = (1 - omega) N_a + omega m phi_a + dN_a.  Both omega m phi_a
        // and dN_a are polynomials in c_a: dN's constant part (-tr dPi / T0),
        // linear part (c.JF / T0) and quadratic part (c c : dPi / T0^2) fold
        // into the equilibrium's coefficients, K' = omega m K + those, so that
        //   N'_a = (1 - omega) N_a + w_a sum_k P_k(c_a) K'_k
        // (this frees the correction's registers before the store: the kernel
        // fits three waves per SIMD)
        {
            const double om = d->omega * m;
#pragma unroll
            for (int k = 0; k < NK; ++k) K[k] *= om;
            K[0] -= trPi * (1.0 / T0);
#pragma unroll
            for (int x = 0; x < 3; ++x) K[1 + x] += JF[x] * (1.0 / T0);
#pragma unroll
            for (int xy = 0; xy < 6; ++xy) K[4 + xy] += Qs[xy] * (1.0 / (T0 * T0));
        }
        const double omw = 1.0 - d->omega;
        double *__restrict__ Pout = d->P[pin ^ 1];
        double Ln[3] = {0.0, 0.0, 0.0};
        // the Christoffel sums are read again from the scalar cache here: an
        // opaque copy of the row pointer keeps the compiler from holding the
        // 117 values loaded for the force in scalar registers across the step
        cptr3<double> tbs = tb;
        __asm__ volatile("" : "+s"(tbs));
        auto store = [&](auto Aic, double wphi) {
            constexpr int a = decltype(Aic)::value;
            const double np = omw * n[a] + wphi;
            Pout[pidx3(d->n2, d->pitch, c.i, c.j, a, c.k)] = np;
            if constexpr (a > 0) {
                Ln[0] += tbs[6 + 3 * a + 0] * np;
                Ln[1] += tbs[6 + 3 * a + 1] * np;
                Ln[2] += tbs[6 + 3 * a + 2] * np;
            }
        };
        // the rest direction, then the pairs (a, -a) = (2p - 1, 2p): the even
        // and odd parts of the polynomial are formed once per pair (the odd
        // one flips sign for -a)
        store(std::integral_constant<int, 0>{}, phi_poly<0>(K));
        __builtin_amdgcn_sched_barrier(0);
        sfor<1, (Q + 1) / 2>([&](auto Pc) {
            constexpr int a = 2 * decltype(Pc)::value - 1, b = a + 1;
            static_assert(opp(a) == b, "pairs (2p - 1, 2p)");
            double E, O;
            phi_parts<a>(K, E, O);
            store(std::integral_constant<int, a>{}, weight(a) * (E + O));
            store(std::integral_constant<int, b>{}, weight(a) * (E - O));
            // one pair at a time: without this boundary the scheduler starts
            // every direction's arithmetic at once and runs out of registers
            __builtin_amdgcn_sched_barrier(0);
        });
        d->lag[pin ^ 1][lrow] = Ln[0];
        d->lag[pin ^ 1][lpl + lrow] = Ln[1];
        d->lag[pin ^ 1][2 * lpl + lrow] = Ln[2];
    }
}

// ---------------------------------------------------------------------------
// set-up (FP64): tangents, metric, volume, co-tangents, Christoffel sums
// ---------------------------------------------------------------------------
// g_i = [x(q + e_i) - x(q - e_i)] / 2 on the halo range (Eqs. distance,
// tangent); out[pos][9] = g_1, g_2, g_3; the outermost layer is left NaN
__global__ void k_tangent3(const double *X, const double *Y, const double *Z, int H1, int H2, int H3, double *tg)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)H1 * H2 * H3;
    if (p >= n) return;
    const int c3 = (int)(p % H3), c2 = (int)((p / H3) % H2), c1 = (int)(p / ((long long)H2 * H3));
    double *t = tg + p * 9;
    if (c1 == 0 || c2 == 0 || c3 == 0 || c1 == H1 - 1 || c2 == H2 - 1 || c3 == H3 - 1) {
        for (int e = 0; e < 9; ++e) t[e] = __builtin_nan("");
        return;
    }
    const long long st[3] = {(long long)H2 * H3, H3, 1};
    for (int i = 0; i < 3; ++i) {
        const long long pp = p + st[i], pm = p - st[i];
        t[3 * i + 0] = 0.5 * ((X[pp] - X[p]) - (X[pm] - X[p]));
        t[3 * i + 1] = 0.5 * ((Y[pp] - Y[p]) - (Y[pm] - Y[p]));
        t[3 * i + 2] = 0.5 * ((Z[pp] - Z[p]) - (Z[pm] - Z[p]));
    }
}

__device__ inline void cross3(const double *u, const double *v, double *w)
{
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
}

// per interior cell: out[cell][GW] = J, g^ij (6), A+^i_a (3 Q), with
// J = (g_1 x g_2) . g_3 (Eq. metric), g^1 = (g_2 x g_3) / J and cyclic (Eq.
// covectors), A+^i_a = g^i(q) . sum_j c^j_a [g_j(q + c_a) - g_j(q)] (Eq. gamma)
__global__ void k_geom3(const double *tg, int n1, int n2, int n3, int h, double *out)
{
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nc = (long long)n1 * n2 * n3;
    if (cell >= nc) return;
    const int k = (int)(cell % n3), j = (int)((cell / n3) % n2), i = (int)(cell / ((long long)n2 * n3));
    const int H2 = n2 + 2 * h, H3 = n3 + 2 * h;
    auto pos = [&](int a, int b, int cc) { return ((long long)a * H2 + b) * H3 + cc; };
    const long long q = pos(i + h, j + h, k + h);
    const double *g = tg + q * 9;
    double x12[3], co[3][3];
    cross3(g + 0, g + 3, x12);
    const double J = x12[0] * g[6] + x12[1] * g[7] + x12[2] * g[8];
    for (int m = 0; m < 3; ++m) {
        cross3(g + 3 * ((m + 1) % 3), g + 3 * ((m + 2) % 3), co[m]);
        for (int e = 0; e < 3; ++e) co[m][e] /= J;
    }
    double *o = out + cell * GW;
    o[0] = J;
    int f = 1;
    for (int x = 0; x < 3; ++x)
        for (int y = x; y < 3; ++y) o[f++] = co[x][0] * co[y][0] + co[x][1] * co[y][1] + co[x][2] * co[y][2];
    for (int a = 0; a < Q; ++a) {
        double dvec[3] = {0.0, 0.0, 0.0};
        if (a > 0) {
            const double *gp = tg + pos(i + h + cvec(a, 0), j + h + cvec(a, 1), k + h + cvec(a, 2)) * 9;
            for (int jj = 0; jj < 3; ++jj) {
                const int cj = cvec(a, jj);
                if (cj == 0) continue;
                for (int e = 0; e < 3; ++e) dvec[e] += cj * (gp[3 * jj + e] - g[3 * jj + e]);
            }
        }
        for (int x = 0; x < 3; ++x) o[7 + 3 * a + x] = co[x][0] * dvec[0] + co[x][1] * dvec[1] + co[x][2] * dvec[2];
    }
}

// flag[0] = 1 if some cell's g^ij or A+ differ from its row's first cell by
// more than tol relative (the metric terms depend on more than q1); flag[1] =
// 1 if J <= 0 or a value is not finite
__global__ void k_rowcheck3(const double *geo, int n1, int n2, int n3, double tol, int *flag)
{
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nc = (long long)n1 * n2 * n3;
    if (cell >= nc) return;
    const int i = (int)(cell / ((long long)n2 * n3));
    const double *o = geo + cell * GW;
    const double *r = geo + (long long)i * n2 * n3 * GW;
    if (!(o[0] > 0.0)) atomicOr(flag + 1, 1);
    double scale = 0.0;
    for (int f = 1; f < GW; ++f) scale = fmax(scale, fabs(r[f]));
    for (int f = 0; f < GW; ++f) {
        if (!isfinite(o[f])) atomicOr(flag + 1, 1);
        const double s = f == 0 ? fabs(r[0]) : scale;
        if (fabs(o[f] - r[f]) > tol * s) atomicOr(flag, 1);
    }
}

// per-row tables and volume from the first cell of each row, and the moment
// table T^ij_k = sum_a w_a c^i_a (A+^j_a + A+^j_{-a}) P_k(c_a)
__global__ void k_rowtab3(const double *geo, int n1, int n2, int n3, double *tab, double *Jrow)
{
    const int i = (int)blockIdx.x;
    if (i >= n1) return;
    const double *r = geo + (long long)i * n2 * n3 * GW;
    for (int f = (int)threadIdx.x; f < TG; f += (int)blockDim.x) tab[(size_t)i * TW + f] = r[1 + f];
    if (threadIdx.x == 0) Jrow[i] = r[0];
    for (int e = (int)threadIdx.x; e < 6 * NK; e += (int)blockDim.x) {
        const int xy = e / NK, k = e % NK;
        constexpr int px[6] = {0, 0, 0, 1, 1, 2}, py[6] = {0, 1, 2, 1, 2, 2};   // the sym2 order
        const int x = px[xy], y = py[xy];
        double s = 0.0;
        for (int a = 1; a < Q; ++a) {
            const int p = mono(k, cvec(a, 0), cvec(a, 1), cvec(a, 2));
            if (p == 0) continue;
            const double Sx = r[1 + 6 + 3 * a + x] + r[1 + 6 + 3 * opp(a) + x];
            const double Sy = r[1 + 6 + 3 * a + y] + r[1 + 6 + 3 * opp(a) + y];
            // w_a c^x S^y P_k (+ w_a c^y S^x P_k off the diagonal)
            double t = cvec(a, x) * Sy;
            if (x != y) t += cvec(a, y) * Sx;
            s += weight(a) * t * p;
        }
        tab[(size_t)i * TW + TT + e] = s;
    }
}

// lagged force sums of the stored state: lag[pin] = sum_a A+^i_a N_a(q)
__global__ __launch_bounds__(64) void k_lag3(const Desc3 *__restrict__ dp, int pin)
{
    const Desc3 &d = *dp;
    Cell3 c;
    if (!cell_of(d, c)) return;
    const double *tb = d.tab + (size_t)c.i * TW;
    double L[3] = {0.0, 0.0, 0.0};
    sfor<1, Q>([&](auto Aic) {
        constexpr int a = decltype(Aic)::value;
        const double v = d.P[pin][pidx3(d.n2, d.pitch, c.i, c.j, a, c.k)];
        L[0] += tb[6 + 3 * a + 0] * v;
        L[1] += tb[6 + 3 * a + 1] * v;
        L[2] += tb[6 + 3 * a + 2] * v;
    });
    const size_t lrow = ((size_t)c.i * d.n2 + c.j) * d.pitch + c.k, lpl = (size_t)d.n1 * d.n2 * d.pitch;
    for (int e = 0; e < 3; ++e) d.lag[pin][e * lpl + lrow] = L[e];
}

// initial state N = J f^eq(rho0, U = Ut = u0; g^ij) (u0 may be null: rest);
// side state m = J rho0, Ut = u0
__global__ __launch_bounds__(64) void k_init3(const Desc3 *__restrict__ dp, const double *u0, double rho0)
{
    const Desc3 &d = *dp;
    Cell3 c;
    if (!cell_of(d, c)) return;
    const size_t cell = ((size_t)c.i * d.n2 + c.j) * d.n3 + c.k;
    const double *tb = d.tab + (size_t)c.i * TW;
    double U[3] = {0.0, 0.0, 0.0};
    if (u0)
        for (int e = 0; e < 3; ++e) U[e] = u0[cell * 3 + e];
    const double G[6] = {tb[0], tb[1], tb[2], tb[3], tb[4], tb[5]};
    double K[NK];
    eq_coeffs(G, U, U, K);
    const double m = d.Jrow[c.i] * rho0;
    sfor<0, Q>([&](auto Aic) {
        constexpr int a = decltype(Aic)::value;
        d.P[0][pidx3(d.n2, d.pitch, c.i, c.j, a, c.k)] = m * phi_poly<a>(K);
    });
    if (c.i < CMAX) {
        d.side[0][sidx3(d.n2, d.pitch, 0, 0, c.i, c.j, c.k)] = m;
        d.side[0][sidx3(d.n2, d.pitch, 0, 1, c.i, c.j, c.k)] = U[1];
        d.side[0][sidx3(d.n2, d.pitch, 0, 2, c.i, c.j, c.k)] = U[2];
    }
    if (c.i >= d.n1 - CMAX) {
        const int row = d.n1 - 1 - c.i;
        d.side[0][sidx3(d.n2, d.pitch, 1, 0, row, c.j, c.k)] = m;
        d.side[0][sidx3(d.n2, d.pitch, 1, 1, row, c.j, c.k)] = U[1];
        d.side[0][sidx3(d.n2, d.pitch, 1, 2, row, c.j, c.k)] = U[2];
    }
}

// state <-> host layout [Q][ncell] (to_device = 0: out; 1: in)
__global__ __launch_bounds__(64) void k_state3(const Desc3 *__restrict__ dp, int pin, double *host, int to_device)
{
    const Desc3 &d = *dp;
    Cell3 c;
    if (!cell_of(d, c)) return;
    const size_t cell = ((size_t)c.i * d.n2 + c.j) * d.n3 + c.k;
    for (int a = 0; a < Q; ++a) {
        double &v = d.P[pin][pidx3(d.n2, d.pitch, c.i, c.j, a, c.k)];
        if (to_device) v = host[(size_t)a * d.ncell + cell];
        else host[(size_t)a * d.ncell + cell] = v;
    }
}

// side state <-> host layout [2 walls][3 fields][CMAX rows][n2][n3]
__global__ void k_side3(const Desc3 *__restrict__ dp, int pin, double *host, int to_device)
{
    const Desc3 &d = *dp;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = 2LL * 3 * CMAX * d.n2 * d.n3;
    if (t >= n) return;
    const int k = (int)(t % d.n3);
    const long long rest = t / d.n3;
    const int j = (int)(rest % d.n2);
    const long long wfr = rest / d.n2;   // ((wall * 3 + field) * CMAX + row)
    double &v = d.side[pin][(size_t)(wfr * d.n2 + j) * d.pitch + k];
    if (to_device) v = host[t];
    else host[t] = v;
}

// the streaming map the step uses: source cell, source direction, wall
__global__ __launch_bounds__(64) void k_stream_map3(const Desc3 *__restrict__ dp, int *sc, int *sd, int *wl)
{
    const Desc3 &d = *dp;
    Cell3 c;
    if (!cell_of(d, c)) return;
    const size_t cell = ((size_t)c.i * d.n2 + c.j) * d.n3 + c.k;
    for (int a = 0; a < Q; ++a) {
        int r, beta, wall;
        source_row(c.i, a, d.n1, d.periodic1, d.bc_lo, d.bc_hi, r, beta, wall);
        const int jj = wrap3(c.j - cvec(a, 1), d.n2), kk = wrap3(c.k - cvec(a, 2), d.n3);
        sc[cell * Q + a] = (int)(((size_t)r * d.n2 + jj) * d.n3 + kk);
        sd[cell * Q + a] = beta;
        wl[cell * Q + a] = wall;
    }
}

} // namespace lbm3
