"""Oracle lattice tables pinned to the paper's App. A / App. B (CPU only)."""
import itertools
from fractions import Fraction

import numpy as np
import sympy as sp

import oracle
from conftest import golden_path


def _printed_weights():
    out = {9: {}, 21: {}}
    for line in open(golden_path("lattice_weights.txt")):
        if line.startswith("#") or not line.strip():
            continue
        q, a, n, d = map(int, line.split())
        out[q][a] = Fraction(n, d)
    return out


def _pairings(idx):
    """All perfect matchings of an index tuple (the 1, 3, 15 terms of the
    isotropic tensors Delta^(2), Delta^(4), Delta^(6))."""
    if not idx:
        yield []
        return
    a = idx[0]
    for k in range(1, len(idx)):
        rest = idx[1:k] + idx[k + 1:]
        for m in _pairings(rest):
            yield [(a, idx[k])] + m


def _delta_tensor(idx):
    return sum(all(i == j for i, j in m) for m in _pairings(tuple(idx)))


def _moment(c, w, idx):
    return sum(wa * np.prod([ca[i] for i in idx]) for ca, wa in zip(c, w))


def test_velocity_set_and_shells():
    for q in (9, 21):
        c, w, T0, bb, sp_ = oracle.lattice(q)
        assert len({tuple(v) for v in c}) == q
        assert tuple(c[0]) == (0, 0)
        # odd moments vanish: every velocity has its opposite
        assert all(any((c[b] == -c[a]).all() for b in range(q)) for a in range(q))


def test_q21_weights_are_the_unique_isotropic_solution():
    """App. A isotropy conditions up to 6th order with T0 = 2/3 determine the six
    shell weights; the printed 7/432 and 7/1620 violate them, 1/432 and 1/1620
    satisfy them (reading of the garbled table)."""
    c, w, T0, *_ = oracle.lattice(21)
    shells = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 2), (3, 0)]
    W = sp.symbols("w0:6")
    T = sp.Rational(2, 3)

    def shell_of(v):
        a, b = sorted((abs(v[0]), abs(v[1])), reverse=True)
        return shells.index((a, b))

    def mom(idx):
        return sum(W[shell_of(v)] * sp.Mul(*[v[i] for i in idx]) for v in c)

    eqs = [sp.Eq(mom(()), 1)]
    for order in (2, 4, 6):
        for idx in set(itertools.combinations_with_replacement((0, 1), order)):
            eqs.append(sp.Eq(mom(idx), T ** (order // 2) * _delta_tensor(idx)))
    sol = sp.solve(eqs, W, dict=True)
    assert len(sol) == 1
    expect = [sp.Rational(91, 324), sp.Rational(1, 12), sp.Rational(2, 27), sp.Rational(7, 360),
              sp.Rational(1, 432), sp.Rational(1, 1620)]
    assert [sol[0][x] for x in W] == expect
    for a in range(21):
        assert w[a] == float(expect[shell_of(c[a])])
    printed = _printed_weights()[21]
    assert sum(printed.values()) == Fraction(289, 270)


def test_isotropy_orders():
    """Q21 isotropic to 6th order, Q9 to 4th order only (App. A, Discussion)."""
    for q, T0e in ((9, 1 / 3), (21, 2 / 3)):
        c, w, T0, *_ = oracle.lattice(q)
        assert T0 == T0e
        assert abs(sum(w) - 1) < 1e-15
        printed = _printed_weights()[q]
        if q == 9:
            assert all(w[a] == float(printed[a]) for a in range(9))
        for order in (1, 3, 5):
            for idx in itertools.product((0, 1), repeat=order):
                assert abs(_moment(c, w, idx)) < 1e-15
        for order in (2, 4, 6):
            for idx in itertools.product((0, 1), repeat=order):
                m, e = _moment(c, w, idx), T0 ** (order // 2) * _delta_tensor(idx)
                if q == 9 and order == 6:
                    continue
                assert abs(m - e) < 1e-14, (q, idx, m, e)
    c, w, T0, *_ = oracle.lattice(9)
    # D2Q9 misses the 6th order: sum w cx^6 = 1/3 while 15 T0^3 = 5/9
    assert abs(_moment(c, w, (0,) * 6) - 1 / 3) < 1e-15
    assert abs(15 * T0 ** 3 - 5 / 9) < 1e-15


def test_app_b_index_maps():
    rows = [list(map(int, ln.split())) for ln in open(golden_path("app_b_index_maps.txt"))
            if ln.strip() and not ln.startswith("#")]
    c, w, T0, bb, spec = oracle.lattice(21)
    for a, astar, ahat in rows:
        assert bb[a] == astar and spec[a] == ahat
        assert (c[astar] == -c[a]).all()                      # full reversal
        assert c[ahat][0] == -c[a][0] and c[ahat][1] == c[a][1]  # wall-normal flip
    listed = {r[0] for r in rows}
    c1_zero = {a for a in range(21) if c[a][0] == 0}
    assert c1_zero == {0, 2, 4, 10, 12, 18, 20}
    assert listed == set(range(21)) - c1_zero
    # the periodicity list "1, 8, 9, 11, 17, 19": the c^2 = 0 set is 1, 3, 9, 11, 17, 19
    c2_zero = {a for a in range(1, 21) if c[a][1] == 0}
    assert c2_zero == {1, 3, 9, 11, 17, 19}
    assert len(c2_zero ^ {1, 8, 9, 11, 17, 19}) == 2
