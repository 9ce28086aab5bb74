"""Batched stepping (one launch per lattice/precision group over a shared tile
table, HIP-graph captured) gives every grid exactly the result it gets alone
(needs an MI355X)."""
import numpy as np
import pytest

from gpu_util import say
from paper_2301_01868_amd import grids as G
from paper_2301_01868_amd import lbm

pytestmark = pytest.mark.gpu


def _cases():
    return [G.circular_couette(21, 12, 100, 10.0, u_inner=0.05, tau=0.8),
            G.circular_poiseuille(9, 10, 70, 12.0, g2=1e-4, tau=0.7),
            G.planar_couette(21, G.faces_linear(16, 0.3), n2=70, u_wall=0.04, tau=0.9),
            G.workload_planar_couette_q9(),
            G.circular_couette(21, 20, 130, 12.0, u_inner=-0.03, tau=0.65)]


@pytest.mark.parametrize("prec", [lbm.LBM_FP64, lbm.LBM_FP32, lbm.LBM_FP16], ids=["fp64", "fp32", "fp16"])
def test_batch_equals_alone(prec):
    cases = _cases()
    alone = [lbm.Grid(c, precision=prec) for c in cases]
    mixed = [lbm.Grid(c, precision=prec) for c in cases]
    for g in alone + mixed:
        g.init()
    # stagger one grid's parity before batching
    mixed[1].step(3)
    alone[1].step(3)
    steps = 101   # graph replays plus an odd tail
    for g in alone:
        g.step(steps)
    b = lbm.lbm_batch_create([g.h for g in mixed])
    groups = lbm.lbm_batch_groups(b)
    say("groups", groups)
    assert len(groups) == 2
    lbm.lbm_batch_step(b, steps)
    lbm.lbm_batch_destroy(b)
    for ga, gm, c in zip(alone, mixed, cases):
        Pa, sa = ga.get_state()
        Pm, sm = gm.get_state()
        assert ga.info.step == gm.info.step
        assert np.array_equal(Pa, Pm), c.meta
        assert np.array_equal(sa, sm)


@pytest.mark.parametrize("fuse", [0, lbm.LBM_BATCH_FUSE_LATTICES], ids=["per_lattice", "fused"])
def test_batch_autotune_advances_like_steps(fuse):
    """The batch autotuner's trial launches advance every grid by the same even
    number of steps; afterwards the batch ends exactly where plain steps end."""
    cases = _cases()
    tuned = [lbm.Grid(c, precision=lbm.LBM_FP32) for c in cases]
    plain = [lbm.Grid(c, precision=lbm.LBM_FP32) for c in cases]
    for g in tuned + plain:
        g.set_launch(1)         # the group starts from a shape the tuner may replace
        g.init()
    tuned[1].step(3)            # one grid on the other buffer parity
    plain[1].step(3)
    bt = lbm.lbm_batch_create_ex([g.h for g in tuned], fuse)
    s0 = [g.info.step for g in tuned]
    lbm.lbm_batch_autotune(bt, 3)                     # rounded up to 4: 2 sweeps x 12 x 6 = 144 steps
    adv = [g.info.step - s for g, s in zip(tuned, s0)]
    say("autotune advanced", adv, "shapes", [lbm.lbm_batch_group_launch(bt, k) for k in range(len(lbm.lbm_batch_groups(bt)))])
    assert adv == [144] * len(cases)
    for k in range(len(lbm.lbm_batch_groups(bt))):
        w, c = lbm.lbm_batch_group_launch(bt, k)
        assert w in (1, 2, 4) and c in (0, 16, 20, 24)
    lbm.lbm_batch_step(bt, 41)
    bp = lbm.lbm_batch_create_ex([g.h for g in plain], fuse)
    lbm.lbm_batch_step(bp, 144 + 41)
    lbm.lbm_batch_destroy(bt)
    lbm.lbm_batch_destroy(bp)
    for gt, gp, c in zip(tuned, plain, cases):
        assert gt.info.step == gp.info.step
        Pt, st = gt.get_state()
        Pp, sp = gp.get_state()
        assert np.array_equal(Pt, Pp), c.meta
        assert np.array_equal(st, sp)


def test_batch_autotune_per_cell_and_iterated_groups():
    """Autotuning groups of per-cell geometry (LDS-staged) and fixed-point force
    grids also leaves the batch where plain steps leave it."""
    specs = [(G.periodic_box(21, 9, 70, dx=1.0, dy=1.1, skew=0.1, wobble=0.25, tau=0.9), 0),
             (G.periodic_box(21, 12, 130, dx=1.0, dy=1.1, skew=0.1, wobble=0.2, tau=0.8), 0),
             (G.circular_couette(21, 12, 100, 10.0, u_inner=0.05, tau=0.8), 1),
             (G.circular_poiseuille(9, 10, 70, 12.0, g2=1e-4, tau=0.7), 0)]

    def make():
        gs = [lbm.Grid(c, precision=lbm.LBM_FP32, iterations=k) for c, k in specs]
        for g in gs:
            g.init()
        return gs

    tuned, plain = make(), make()
    assert tuned[0].info.table_kind == 2
    bt = lbm.lbm_batch_create([g.h for g in tuned])
    ngroups = len(lbm.lbm_batch_groups(bt))
    assert ngroups == 3
    lbm.lbm_batch_autotune(bt, 2)                     # 2 sweeps x 12 x 4 = 96 steps
    say("per-cell / iterated autotune shapes", [lbm.lbm_batch_group_launch(bt, k) for k in range(ngroups)])
    lbm.lbm_batch_step(bt, 21)
    bp = lbm.lbm_batch_create([g.h for g in plain])
    lbm.lbm_batch_step(bp, 96 + 21)
    lbm.lbm_batch_destroy(bt)
    lbm.lbm_batch_destroy(bp)
    for gt, gp in zip(tuned, plain):
        assert gt.info.step == gp.info.step == 117
        Pt, st = gt.get_state()
        Pp, sp = gp.get_state()
        assert np.array_equal(Pt, Pp)
        assert np.array_equal(st, sp)


@pytest.mark.parametrize("prec", [lbm.LBM_FP64, lbm.LBM_FP32, lbm.LBM_FP16], ids=["fp64", "fp32", "fp16"])
def test_fused_lattice_batch_equals_alone(prec):
    """D2Q9 and D2Q21 grids in one fused launch per step end exactly as alone."""
    cases = _cases()
    alone = [lbm.Grid(c, precision=prec) for c in cases]
    fused = [lbm.Grid(c, precision=prec) for c in cases]
    for g in alone + fused:
        g.init()
    steps = 37
    for g in alone:
        g.step(steps)
    b = lbm.lbm_batch_create_ex([g.h for g in fused], lbm.LBM_BATCH_FUSE_LATTICES)
    groups = lbm.lbm_batch_groups(b)
    say("fused groups", groups)
    assert len(groups) == 1 and groups[0][0] == 0 and groups[0][2] == sum(c.ncell for c in cases)
    lbm.lbm_batch_step(b, steps)
    lbm.lbm_batch_destroy(b)
    for ga, gf, c in zip(alone, fused, cases):
        assert np.array_equal(ga.get_state()[0], gf.get_state()[0]), c.meta
        assert np.array_equal(ga.get_state()[1], gf.get_state()[1])


def test_launch_shape_does_not_change_results():
    """Tile shape (waves per workgroup), the occupancy cap and the autotuner's
    choice leave every cell's arithmetic unchanged: bitwise identical states."""
    case = G.circular_couette(21, 13, 140, 12.0, u_inner=0.05, tau=0.7)
    states = []
    for w, cap in ((1, 0), (2, 0), (4, 0), (1, 20), (2, 16), (4, 24)):
        g = lbm.Grid(case, precision=lbm.LBM_FP32)
        g.set_launch(w)
        g.set_occupancy(cap)
        assert (g.info.waves_per_block, g.info.waves_per_cu_cap) == (w, cap)
        g.init()
        g.step(77)
        states.append(g.get_state()[0])
    g = lbm.Grid(case, precision=lbm.LBM_FP32)
    chosen = g.autotune(6)
    assert chosen in (1, 2, 4)
    assert g.info.waves_per_block == chosen and g.info.waves_per_cu_cap in (0, 24, 20, 16)
    g.init()
    g.step(77)
    states.append(g.get_state()[0])
    for s in states[1:]:
        assert np.array_equal(s, states[0])


def test_checkpoint_resume():
    """lbm_get_state / lbm_set_state round trip: a run saved at step t and
    resumed in a fresh grid continues like the uninterrupted run."""
    case = G.circular_couette(21, 12, 100, 10.0, u_inner=0.05, tau=0.8)
    for prec, tol in ((lbm.LBM_FP64, 0.0), (lbm.LBM_FP32, 0.0)):
        a = lbm.Grid(case, precision=prec)
        a.init()
        a.step(40)
        P, side = a.get_state()
        a.step(60)
        b = lbm.Grid(case, precision=prec)
        b.set_state(P, side)
        b.step(60)
        Pa, _ = a.get_state()
        Pb, _ = b.get_state()
        err = np.abs(Pa - Pb).max() / np.abs(Pa).max()
        say("resume", prec, err)
        assert err <= max(tol, 1e-15 if prec == lbm.LBM_FP64 else 1e-7)


def test_batch_rejects_repeated_or_uninitialised_grids():
    case = G.planar_couette(21, G.faces_uniform(8), n2=70, u_wall=0.04, tau=0.8)
    a = lbm.Grid(case, precision=lbm.LBM_FP32)
    b = lbm.Grid(case, precision=lbm.LBM_FP32)
    a.init()
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_batch_create([a.h, a.h])
    assert e.value.code == lbm.LBM_EINVAL
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_batch_create([a.h, b.h])
    assert e.value.code == lbm.LBM_ESTATE
    b.init()
    bt = lbm.lbm_batch_create([a.h, b.h])
    lbm.lbm_batch_step(bt, 4)
    # an update naming a grid twice or an uninitialised one leaves the batch as it was
    c = lbm.Grid(case, precision=lbm.LBM_FP32)
    for bad, code in (([a.h, a.h], lbm.LBM_EINVAL), ([a.h, c.h], lbm.LBM_ESTATE)):
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_batch_update(bt, bad)
        assert e.value.code == code
    lbm.lbm_batch_step(bt, 4)
    assert [g[2] for g in lbm.lbm_batch_groups(bt)] == [2 * case.ncell]
    lbm.lbm_batch_destroy(bt)
    Pa, _ = a.get_state()
    Pb, _ = b.get_state()
    assert np.array_equal(Pa, Pb)
    assert a.info.step == 8


def test_batch_with_fixed_point_force_grids():
    """Grids with fixed-point force passes (iterations > 0) form their own
    launch group; each grid still ends exactly as it does alone."""
    cases = [(G.planar_couette(9, G.faces_linear(12, 0.4), n2=70, u_wall=0.05, tau=0.8), 2),
             (G.planar_couette(9, G.faces_linear(12, 0.4), n2=70, u_wall=0.05, tau=0.8), 0),
             (G.circular_couette(21, 12, 100, 10.0, u_inner=0.05, tau=0.8), 1)]
    alone = [lbm.Grid(c, precision=lbm.LBM_FP64, iterations=k) for c, k in cases]
    mixed = [lbm.Grid(c, precision=lbm.LBM_FP64, iterations=k) for c, k in cases]
    for g in alone + mixed:
        g.init()
    for g in alone:
        g.step(40)
    b = lbm.lbm_batch_create([g.h for g in mixed])
    groups = lbm.lbm_batch_groups(b)
    say("groups", groups)
    assert len(groups) == 3
    lbm.lbm_batch_step(b, 40)
    lbm.lbm_batch_destroy(b)
    for ga, gm in zip(alone, mixed):
        assert np.array_equal(ga.get_state()[0], gm.get_state()[0])
    # the fixed-point passes change the result
    assert not np.array_equal(mixed[0].get_state()[0], mixed[1].get_state()[0])


@pytest.mark.parametrize("prec", [lbm.LBM_FP64, lbm.LBM_FP32], ids=["fp64", "fp32"])
def test_checkpoint_blob_resume(prec):
    """lbm_save / lbm_load: a grid restored from the blob into a fresh grid
    continues exactly as the original does; metadata is checked."""
    case = G.circular_couette(21, 12, 100, 10.0, u_inner=0.05, u_outer=-0.02, tau=0.8)
    a = lbm.Grid(case, precision=prec)
    a.init()
    a.step(57)
    blob = a.save()
    b = lbm.Grid(case, precision=prec)
    b.load(blob)
    assert b.info.step == a.info.step == 57
    a.step(40)
    b.step(40)
    assert np.array_equal(a.get_state()[0], b.get_state()[0])
    assert np.array_equal(a.get_state()[1], b.get_state()[1])
    ra, rb = a.residual(), b.residual()
    assert ra.mass_rel_drift == rb.mass_rel_drift
    # a blob loads into any storage precision of the same lattice and shape
    c = lbm.Grid(case, precision=lbm.LBM_FP64 if prec == lbm.LBM_FP32 else lbm.LBM_FP32)
    c.load(blob)
    # and is refused by a grid of another shape
    other = lbm.Grid(G.circular_couette(21, 12, 96, 10.0, u_inner=0.05, tau=0.8), precision=prec)
    with pytest.raises(lbm.LbmError) as e:
        other.load(blob)
    assert e.value.code == lbm.LBM_EINVAL
    with pytest.raises(lbm.LbmError):
        b.load(b"not a checkpoint" * 4)


def test_grid_destroyed_before_its_batch():
    """A grid destroyed while a batch still holds it (its own stream goes with
    it) leaves the batch broken: stepping or reducing it returns LBM_ESTATE,
    destroying it is safe, and the other grid keeps working alone."""
    cases = [G.circular_couette(21, 12, 100, 10.0, u_inner=0.05, tau=0.8),
             G.planar_couette(9, G.faces_uniform(8), n2=70, u_wall=0.05, tau=0.8)]
    grids = [lbm.Grid(c, precision=lbm.LBM_FP32) for c in cases]
    for g in grids:
        g.init()
    b = lbm.lbm_batch_create([g.h for g in grids])
    lbm.lbm_batch_step(b, 20)
    grids[0].close()          # the batch runs on this grid's stream
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_batch_step(b, 2)
    assert e.value.code == lbm.LBM_ESTATE
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_batch_residuals(b, 2)
    assert e.value.code == lbm.LBM_ESTATE
    lbm.lbm_batch_destroy(b)
    grids[1].step(10)
    assert grids[1].residual().bad_cells == 0
    assert grids[1].info.step == 30


@pytest.mark.parametrize("fuse", [0, lbm.LBM_BATCH_FUSE_LATTICES], ids=["per_lattice", "fused"])
def test_batch_update_in_place_equals_alone(fuse):
    """Continuous batching: members leave and join a running batch (at an odd
    batch step, with grids of either buffer parity, and through a change of
    group structure) and every grid ends bitwise as the same steps taken
    alone.  Steps of 48 run as graph replays whose kernel nodes the updates
    rewrite in place; odd counts add single launches."""
    cases = _cases()
    alone = [lbm.Grid(c, precision=lbm.LBM_FP32) for c in cases]
    mixed = [lbm.Grid(c, precision=lbm.LBM_FP32) for c in cases]
    for g in alone + mixed:
        g.init()
    # grid 3 joins with the other buffer parity
    for g in (alone[3], mixed[3]):
        g.step(5)
    plan = [([0, 1], 48), ([0, 1, 2], 33), ([1, 2, 3], 48), ([1, 2, 3, 4], 64), ([4], 16), ([], 10),
            ([0, 2, 4], 48)]
    b = lbm.lbm_batch_create_ex([mixed[k].h for k in plan[0][0]], fuse)
    for members, n in plan:
        lbm.lbm_batch_update(b, [mixed[k].h for k in members])
        say("members", members, "groups", lbm.lbm_batch_groups(b))
        lbm.lbm_batch_step(b, n)
        for k in members:
            alone[k].step(n)
    # grids outside the batch step alone too
    mixed[3].step(7)
    alone[3].step(7)
    lbm.lbm_batch_destroy(b)
    for ga, gm, c in zip(alone, mixed, cases):
        assert ga.info.step == gm.info.step
        Pa, sa = ga.get_state()
        Pm, sm = gm.get_state()
        assert np.array_equal(Pa, Pm), c.meta
        assert np.array_equal(sa, sm)


def test_batch_update_moves_off_a_leaving_grids_stream():
    """The batch runs on its first grid's library-owned stream; when that grid
    leaves and is destroyed, the batch has moved to a remaining grid's stream
    and keeps stepping correctly."""
    cases = [G.circular_couette(21, 12, 100, 10.0, u_inner=0.05, tau=0.8),
             G.planar_couette(9, G.faces_uniform(8), n2=70, u_wall=0.05, tau=0.8)]
    grids = [lbm.Grid(c, precision=lbm.LBM_FP32) for c in cases]
    ref = lbm.Grid(cases[1], precision=lbm.LBM_FP32)
    for g in grids + [ref]:
        g.init()
    b = lbm.lbm_batch_create([g.h for g in grids])
    lbm.lbm_batch_step(b, 20)
    lbm.lbm_batch_update(b, [grids[1].h])
    grids[0].close()
    lbm.lbm_batch_step(b, 20)
    lbm.lbm_batch_residuals(b, 1)
    lbm.lbm_batch_destroy(b)
    ref.step(40)
    assert np.array_equal(ref.get_state()[0], grids[1].get_state()[0])


def test_grid_created_on_a_setup_stream_then_moved():
    """A grid created and initialised on one stream and handed to another
    (lbm_grid_set_stream) steps exactly like one made on the second stream."""
    import torch
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    c = _cases()[0]
    a = lbm.Grid(c, precision=lbm.LBM_FP32, stream=s2.cuda_stream)
    g = lbm.Grid(c, precision=lbm.LBM_FP32, stream=s1.cuda_stream)
    a.init()
    g.init()
    g.set_stream(s2.cuda_stream)
    assert g.stream == s2.cuda_stream
    a.step(50)
    g.step(50)
    assert np.array_equal(a.get_state()[0], g.get_state()[0])
    # a grid held by a batch keeps its stream
    b = lbm.lbm_batch_create([g.h])
    with pytest.raises(lbm.LbmError) as e:
        g.set_stream(s1.cuda_stream)
    assert e.value.code == lbm.LBM_ESTATE
    lbm.lbm_batch_destroy(b)
    g.set_stream(None)          # to a library-owned stream
    g.step(2)
    a.step(2)
    assert np.array_equal(a.get_state()[0], g.get_state()[0])
