"""Derive a three-dimensional lattice with 6th-order moment isotropy from the
isotropy and normalisation conditions of App. A, in exact rational arithmetic,
and write it as a fixture (tests/golden/lattice_d3q39.txt).

The conditions of App. A, written for i, j, ... in {1, 2, 3}, say that the
weighted moments of the velocity set up to 6th order equal T0^n times the
isotropic tensors Delta^(2n).  For a set made of whole orbits ("shells") of
integer vectors under the symmetry group of the cube, each tensor condition
collapses to scalar conditions on a few components (the others vanish or
follow by symmetry):

    order 0:  sum w                      = 1
    order 2:  sum w cx^2                 = T0
    order 4:  sum w cx^4 = 3 T0^2,        sum w cx^2 cy^2 = T0^2
    order 6:  sum w cx^6 = 15 T0^3,       sum w cx^4 cy^2 = 3 T0^3,
              sum w cx^2 cy^2 cz^2 = T0^3

Seven conditions; with one weight per shell they fix six shell weights and
T0.  The script tries every set of six shells (the rest shell included) drawn
from the orbits of vectors with components up to 3, solves the conditions for
T0 (a cubic once the weights are eliminated) and the weights, and keeps the
solutions with rational T0 > 0 and all weights positive.  The fewest
velocities such a set can have is 39, reached by two shell sets: T0 = 2/3 with
the shells of (0,0,0), (1,0,0), (1,1,1), (2,0,0), (2,2,0), (3,0,0), and
T0 = 4/9 with (0,0,0), (1,0,0), (1,1,0), (2,0,0), (2,2,2), (3,0,0).  The
fixture takes the first: its T0 is that of the paper's 6th-order 2D lattice
(D2Q21, App. A).  Run the script to regenerate the fixture; it imports
nothing from the library or the oracle.
"""
from __future__ import annotations

import itertools
import os
from fractions import Fraction as Fr


def shells(cmax=3):
    reps = [(a, b, c) for a in range(cmax + 1) for b in range(a + 1) for c in range(b + 1)]
    out = []
    for r in reps:
        vs = set()
        for p in itertools.permutations(r):
            for s in itertools.product((1, -1), repeat=3):
                vs.add(tuple(x * y for x, y in zip(p, s)))
        out.append((r, sorted(vs)))
    return out


def moments(vs):
    """Shell sums of cx^2, cx^4, cx^2 cy^2, cx^6, cx^4 cy^2, cx^2 cy^2 cz^2."""
    return [len(vs), sum(v[0] ** 2 for v in vs), sum(v[0] ** 4 for v in vs),
            sum(v[0] ** 2 * v[1] ** 2 for v in vs), sum(v[0] ** 6 for v in vs),
            sum(v[0] ** 4 * v[1] ** 2 for v in vs), sum(v[0] ** 2 * v[1] ** 2 * v[2] ** 2 for v in vs)]


def rhs(T):
    return [Fr(1), T, 3 * T ** 2, T ** 2, 15 * T ** 3, 3 * T ** 3, T ** 3]


def det(M):
    """Exact determinant (Fractions) by elimination."""
    M = [row[:] for row in M]
    n = len(M)
    d = Fr(1)
    for c in range(n):
        p = next((r for r in range(c, n) if M[r][c] != 0), None)
        if p is None:
            return Fr(0)
        if p != c:
            M[c], M[p] = M[p], M[c]
            d = -d
        d *= M[c][c]
        for r in range(c + 1, n):
            f = M[r][c] / M[c][c]
            for k in range(c, n):
                M[r][k] -= f * M[c][k]
    return d


def solve(A, b):
    """Exact solution of the square system A x = b, or None if singular."""
    n = len(A)
    M = [A[r][:] + [b[r]] for r in range(n)]
    for c in range(n):
        p = next((r for r in range(c, n) if M[r][c] != 0), None)
        if p is None:
            return None
        M[c], M[p] = M[p], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                for k in range(c, n + 1):
                    M[r][k] -= f * M[c][k]
    return [M[r][n] / M[r][r] for r in range(n)]


def derive(cmax=3, nshell=6, max_velocities=45):
    import numpy as np
    sh = shells(cmax)
    rest, others = sh[0], sh[1:]
    best = None
    for combo in itertools.combinations(others, nshell - 1):
        S = [rest] + list(combo)
        if sum(len(vs) for (_, vs) in S) > max_velocities:
            continue
        Am = np.array([[moments(vs)[e] for (_, vs) in S] for e in range(7)], dtype=float)
        # det [A | rhs(T)] is a cubic in T: its values at T = 0..3 fix it
        vals = [np.linalg.det(np.column_stack([Am, [float(x) for x in rhs(Fr(t))]])) for t in range(4)]
        coef = np.polyfit(np.arange(4.0), vals, 3)
        if not np.isfinite(coef).all() or np.abs(coef).max() == 0:
            continue
        for root in np.roots(coef):
            if abs(root.imag) > 1e-9 or root.real <= 0:
                continue
            # candidate T0 as a small-denominator rational, then checked exactly
            T = Fr(float(root.real)).limit_denominator(1000)
            A = [[Fr(moments(vs)[e]) for (_, vs) in S] for e in range(7)]
            w = None
            for drop in range(7):
                rows = [e for e in range(7) if e != drop]
                w = solve([A[e] for e in rows], [rhs(T)[e] for e in rows])
                if w is not None:
                    break
            if w is None or any(x <= 0 for x in w):
                continue
            if any(sum(A[e][k] * w[k] for k in range(6)) != rhs(T)[e] for e in range(7)):
                continue
            nvel = sum(len(vs) for (_, vs) in S)
            # fewest velocities, then the T0 of D2Q21 (2/3) before any other
            key = (nvel, T != Fr(2, 3), T)
            if best is None or key < best[0]:
                best = (key, T, [(r, vs, x) for (r, vs), x in zip(S, w)])
    return best


def numbering(sol):
    """Velocity numbering: shells in the order found (rest first), and within
    a shell the vectors sorted by (-c1, -c2, -c3) reversed into pairs: each
    vector is followed by its opposite, the one with the larger first nonzero
    component first."""
    vel, wts = [], []
    for r, vs, w in sol:
        seen = set()
        for v in sorted(vs, reverse=True):
            if v in seen:
                continue
            o = tuple(-x for x in v)
            for u in ((v, o) if v != o else (v,)):
                seen.add(u)
                vel.append(u)
                wts.append(w)
    return vel, wts


def main():
    key, T, sol = derive()
    vel, wts = numbering(sol)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lattice_d3q39.txt")
    with open(path, "w") as fh:
        fh.write("# 3D lattice with 6th-order isotropy, derived from the isotropy conditions of App. A\n")
        fh.write("# (tests/golden/derive_lattice3d.py): T0, then one line per velocity: c1 c2 c3 weight\n")
        fh.write("T0 %s\n" % T)
        for v, w in zip(vel, wts):
            fh.write("%d %d %d %s\n" % (v[0], v[1], v[2], w))
    print("Q = %d, T0 = %s, shells %s" % (len(vel), T, [(r, str(w)) for r, _, w in sol]))


if __name__ == "__main__":
    main()
