"""D2Q9 steps with FP32 or FP64 storage take the own cell's lagged N'_a(q, t-1)
(Eq. compo-constr with the one-step lag of Sec. 2) from the values the
workgroup's lanes pull (an LDS tile) and, for partners outside the tile, from
the own cell in HBM.  Which partners are inside depends on the launch shape
(rows per workgroup); the states must not: they must be the same bits for
every shape.  The FP16 D2Q9 step keeps the stored sums and is checked the same
way.  FP64 parity of the D2Q9 step with the oracle is in test_gpu_parity.py."""
import numpy as np
import pytest

from gpu_util import initial_velocity, say
from paper_2301_01868_amd import grids as G
from paper_2301_01868_amd import lbm

pytestmark = pytest.mark.gpu


def _cases():
    # fewer rows than a 4-row tile and 5 of a wave's 64 lanes
    yield "couette_3x5", G.planar_couette(9, G.faces_uniform(3), n2=5, u_wall=0.04, tau=0.8)
    # a stretched channel moving at q1 = 0, a ragged second column tile, 6 rows (one full tile and half of one)
    yield "couette_6x70_lo", G.planar_couette(9, G.faces_geometric(6, 1.1), n2=70, moving="lo", tau=0.7)
    # periodic q1 over 5 rows (partners across the periodic seam) and 3 column tiles
    yield "box_5x130", G.periodic_box(9, 5, 130, dx=1.0, dy=1.2, tau=0.9)
    # a polar grid with moving walls, 13 rows
    yield "annulus_13x140", G.circular_couette(9, 13, 140, 12.0, u_inner=0.05, u_outer=-0.02, tau=0.7)


CASES = list(_cases())
PRECS = [(lbm.LBM_FP64, "fp64"), (lbm.LBM_FP32, "fp32"), (lbm.LBM_FP16, "fp16")]


def _run(case, prec, wpb=4, cap=0, steps=37, **kw):
    g = lbm.Grid(case, precision=prec, **kw)
    g.set_launch(wpb)
    g.set_occupancy(cap)
    g.init(initial_velocity(case))
    g.step(steps)
    return g


@pytest.mark.parametrize("prec,pname", PRECS, ids=[p[1] for p in PRECS])
@pytest.mark.parametrize("name,case", CASES, ids=[c[0] for c in CASES])
def test_d2q9_states_independent_of_tile(name, case, prec, pname):
    ref = _run(case, prec, 1)
    assert ref.info.table_kind == 0
    P0 = ref.get_state()[0]
    assert np.isfinite(P0).all()
    for wpb, cap in ((2, 0), (4, 0), (4, 24), (2, 16)):
        P = _run(case, prec, wpb, cap).get_state()[0]
        say(name, pname, "wpb", wpb, "cap", cap, "max diff", float(np.abs(P - P0).max()))
        assert np.array_equal(P, P0)


@pytest.mark.parametrize("fuse", [0, lbm.LBM_BATCH_FUSE_LATTICES], ids=["groups", "fused"])
def test_d2q9_exchange_in_batches(fuse):
    """In a batch group (or the fused launch with D2Q21 tiles) every grid ends
    as it does alone, whatever the group's tile shape."""
    cases = [c for _, c in CASES] + [G.circular_couette(21, 12, 100, 10.0, u_inner=0.05, tau=0.8)]
    for prec in (lbm.LBM_FP64, lbm.LBM_FP32):
        batched = [lbm.Grid(c, precision=prec) for c in cases]
        for g, c in zip(batched, cases):
            g.init(initial_velocity(c))
        b = lbm.lbm_batch_create_ex([g.h for g in batched], fuse)
        # the autotuner's trials step the batch with every tile shape and cap
        lbm.lbm_batch_autotune(b, 3)
        say("groups", lbm.lbm_batch_groups(b))
        lbm.lbm_batch_step(b, 29)
        lbm.lbm_batch_destroy(b)
        steps = batched[0].info.step
        assert steps > 29 and all(g.info.step == steps for g in batched)
        for gb, c in zip(batched, cases):
            ga = _run(c, prec, 4, steps=steps)
            assert np.array_equal(ga.get_state()[0], gb.get_state()[0])


@pytest.mark.parametrize("prec,pname", PRECS[:2], ids=[p[1] for p in PRECS[:2]])
def test_d2q9_iterated_force_independent_of_tile(prec, pname):
    """Fixed-point force passes (iterations > 0) start from the same exchanged
    own-cell values: the states are the same bits for every tile shape."""
    name, case = CASES[3]
    states = []
    for wpb in (1, 2, 4):
        g = _run(case, prec, wpb, iterations=2)
        states.append(g.get_state()[0])
    say(name, pname, "iterations 2, max diff", float(np.abs(states[2] - states[0]).max()))
    assert np.array_equal(states[0], states[1]) and np.array_equal(states[0], states[2])
