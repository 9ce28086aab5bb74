// Lattice constants of the two lattices used by the method (App. A, App. B of
// arXiv:2301.01868), as compile-time tables for host and device code.
//
// Velocity numbering: 0 rest; 1..4 the unit vectors (+1,0), (0,+1), (-1,0),
// (0,-1); 5..8 the diagonals (+1,+1), (-1,+1), (-1,-1), (+1,-1); 9..12 and
// 13..16 the same two sets doubled; 17..20 the unit set tripled.  This is the
// numbering the App. B index tables imply (bounce-back reverses a vector,
// specular reflection flips its first component).  D2Q9 is the first nine.
//
// D2Q21 weights: the unique solution of the 6th-order isotropy conditions of
// App. A for T0 = 2/3 (the printed 7/432 and 7/1620 are read as 1/432 and
// 1/1620, the values for which the weights sum to one).
#pragma once

namespace lbm {

struct Lat21 {
    static constexpr int Q = 21;
    static constexpr int CMAX = 3;
    static constexpr int NPAIR = 10;
};
struct Lat9 {
    static constexpr int Q = 9;
    static constexpr int CMAX = 1;
    static constexpr int NPAIR = 4;
};

// components of the velocity vectors (shared prefix for both lattices)
__host__ __device__ constexpr int cx(int a)
{
    constexpr int t[21] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0, 2, -2, -2, 2, 3, 0, -3, 0};
    return t[a];
}
__host__ __device__ constexpr int cy(int a)
{
    constexpr int t[21] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2, 2, 2, -2, -2, 0, 3, 0, -3};
    return t[a];
}
// opposite vector: -c
__host__ __device__ constexpr int opp(int a)
{
    constexpr int t[21] = {0, 3, 4, 1, 2, 7, 8, 5, 6, 11, 12, 9, 10, 15, 16, 13, 14, 19, 20, 17, 18};
    return t[a];
}
// bounce-back alpha* (reverse) and specular alpha-hat (flip the q1 component)
__host__ __device__ constexpr int bounce(int a) { return opp(a); }
__host__ __device__ constexpr int specular(int a)
{
    constexpr int t[21] = {0, 3, 2, 1, 4, 6, 5, 8, 7, 11, 10, 9, 12, 14, 13, 16, 15, 19, 18, 17, 20};
    return t[a];
}
// representative of each +-c pair: the direction listed first in the numbering
__host__ __device__ constexpr int pair_rep(int p)
{
    constexpr int t[10] = {1, 2, 5, 6, 9, 10, 13, 14, 17, 18};
    return t[p];
}

template <int Q>
__host__ __device__ constexpr double weight(int a)
{
    if constexpr (Q == 9) {
        return a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    } else {
        return a == 0    ? 91.0 / 324.0
               : a < 5   ? 1.0 / 12.0
               : a < 9   ? 2.0 / 27.0
               : a < 13  ? 7.0 / 360.0
               : a < 17  ? 1.0 / 432.0
                         : 1.0 / 1620.0;
    }
}
template <int Q>
__host__ __device__ constexpr double lattice_T0()
{
    return Q == 9 ? 1.0 / 3.0 : 2.0 / 3.0;
}
template <int Q>
__host__ __device__ constexpr int cmax()
{
    return Q == 9 ? 1 : 3;
}
template <int Q>
__host__ __device__ constexpr int npair()
{
    return (Q - 1) / 2;
}

} // namespace lbm
