// The 39-velocity lattice of the three-dimensional step: 6th-order moment
// isotropy with T0 = 2/3, the solution of the isotropy and normalisation
// conditions of App. A (arXiv:2301.01868) written for three dimensions, for
// the shells of (0,0,0), (1,0,0), (1,1,1), (2,0,0), (2,2,0) and (3,0,0)
// (weights 1/12, 1/12, 1/27, 2/135, 1/432, 1/1620 per vector).
//
// Numbering: rest; then shell by shell, each vector followed by its opposite
// (so opp(a) = a + 1 for odd a, a - 1 for even a > 0):
//   1..6    the unit axis vectors     +e1, -e1, +e2, -e2, +e3, -e3
//   7..14   the cube diagonals        (1, s2, s3) and its opposite, for
//                                     (s2, s3) = (+,+), (+,-), (-,+), (-,-)
//   15..20  the axis vectors doubled
//   21..32  the face diagonals doubled: (2,2,0), (2,0,2), (2,0,-2), (2,-2,0),
//                                     (0,2,2), (0,2,-2), each with its opposite
//   33..38  the axis vectors tripled
#pragma once

namespace lbm3 {

constexpr int Q = 39;
constexpr int CMAX = 3;
constexpr double T0 = 2.0 / 3.0;

// component d (0, 1, 2) of velocity a, built from the shell structure above
__host__ __device__ constexpr int shell_component(int a, int d)
{
    if (a == 0) return 0;
    const int sgn = (a & 1) ? 1 : -1;   // the first of each pair, then its opposite
    if (a <= 6 || (a >= 15 && a <= 20) || a >= 33) {
        const int base = a <= 6 ? 1 : (a <= 20 ? 15 : 33);
        const int len = a <= 6 ? 1 : (a <= 20 ? 2 : 3);
        const int axis = (a - base) / 2;
        return d == axis ? sgn * len : 0;
    }
    if (a <= 14) {
        const int p = (a - 7) / 2;      // (s2, s3) = (+,+), (+,-), (-,+), (-,-)
        const int v = d == 0 ? 1 : (d == 1 ? ((p & 2) ? -1 : 1) : ((p & 1) ? -1 : 1));
        return sgn * v;
    }
    const int p = (a - 21) / 2;         // face diagonals
    constexpr int fd[6][3] = {{2, 2, 0}, {2, 0, 2}, {2, 0, -2}, {2, -2, 0}, {0, 2, 2}, {0, 2, -2}};
    return sgn * fd[p][d];
}
struct VecTable {
    int c[Q][3];
};
__host__ __device__ constexpr VecTable make_vectors()
{
    VecTable t{};
    for (int a = 0; a < Q; ++a)
        for (int d = 0; d < 3; ++d) t.c[a][d] = shell_component(a, d);
    return t;
}
// tabulated once at compile time, so that a constant index folds to a constant
__host__ __device__ constexpr int cvec(int a, int d)
{
    constexpr VecTable T = make_vectors();
    return T.c[a][d];
}

__host__ __device__ constexpr int opp(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }

__host__ __device__ constexpr double weight(int a)
{
    return a == 0 ? 1.0 / 12.0 : (a <= 6 ? 1.0 / 12.0 : (a <= 14 ? 1.0 / 27.0 : (a <= 20 ? 2.0 / 135.0 : (a <= 32 ? 1.0 / 432.0 : 1.0 / 1620.0))));
}

// the direction with the q1 component of c_a flipped (specular source at a q1
// wall): the opposite vector for the axis vectors along q1, the same vector
// for c^1 = 0, and for the diagonals the pair partner's neighbour with the
// same (c^2, c^3)
__host__ __device__ constexpr int specular_search(int a)
{
    for (int b = 0; b < Q; ++b)
        if (shell_component(b, 0) == -shell_component(a, 0) && shell_component(b, 1) == shell_component(a, 1) &&
            shell_component(b, 2) == shell_component(a, 2))
            return b;
    return -1;
}
struct SpecTable {
    int t[Q];
};
__host__ __device__ constexpr SpecTable make_spec()
{
    SpecTable s{};
    for (int a = 0; a < Q; ++a) s.t[a] = specular_search(a);
    return s;
}
__host__ __device__ constexpr int specular(int a)
{
    constexpr SpecTable S = make_spec();
    return S.t[a];
}

} // namespace lbm3
