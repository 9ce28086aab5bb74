"""Streaming/boundary index maps of the oracle (Eq. adv, App. B) (CPU only)."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2301_01868_amd import grids as G

KINDS = ["noslip", "moving"]


def _case(q, n1, n2, lo, hi):
    return G.planar_channel(q, G.faces_uniform(n1), n2, bc_lo=lo, bc_hi=hi, ut_lo=0.01, ut_hi=-0.02)


@pytest.mark.parametrize("q", [9, 21])
def test_stream_map_is_a_permutation(q):
    """Every (cell, direction) of the post-collision field is pulled exactly
    once (mirror-image wall sources), for every wall combination and width."""
    cmax = 1 if q == 9 else 3
    for n1 in range(cmax, cmax + 6):
        for n2 in (1, 2, 5, 9):
            for lo, hi in itertools.product(KINDS, KINDS):
                o = oracle.OracleGrid(_case(q, n1, n2, lo, hi))
                sc, sd, wl = o.stream_map()
                key = sc.astype(np.int64) * q + sd
                assert np.unique(key).size == key.size == n1 * n2 * q
    o = oracle.OracleGrid(G.periodic_box(q, 4, 5))
    sc, sd, wl = o.stream_map()
    assert np.unique(sc.astype(np.int64) * q + sd).size == 4 * 5 * q
    assert (wl == 0).all()


def test_stream_map_interior_and_walls():
    q = 21
    n1, n2 = 9, 7
    o = oracle.OracleGrid(_case(q, n1, n2, "noslip", "moving"))
    sc, sd, wl = o.stream_map()
    cl, w, T0, bb, sp = oracle.lattice(q)
    for i in range(n1):
        for j in range(n2):
            for a in range(q):
                si, sj = i - cl[a][0], (j - cl[a][1]) % n2
                k = i * n2 + j
                if 0 <= si < n1:
                    assert sc[k, a] == si * n2 + sj and sd[k, a] == a and wl[k, a] == 0
                elif si < 0:
                    assert sc[k, a] == (-1 - si) * n2 + sj and sd[k, a] == bb[a] and wl[k, a] == 1
                else:
                    assert sc[k, a] == (2 * n1 - 1 - si) * n2 + sj and sd[k, a] == sp[a] and wl[k, a] == 2
