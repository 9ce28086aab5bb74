"""Host-side checks of bench.py: the one-GPU contract and the traffic record it quotes."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_workloads_have_the_stated_sizes():
    w = bench.workloads()
    ens = w["ensemble_64_annuli"]()
    assert len(ens) == 64
    assert {c.q for c in ens} == {9, 21}
    assert sum(c.ncell for c in ens if c.q == 21) == 9_665_148
    assert sum(c.ncell for c in ens) == 22_108_104
    (a,) = w["annulus_couette_256x1024"]()
    assert (a.q, a.n1, a.n2) == (21, 256, 1024)
    (p,) = w["planar_couette_q9_32x16"]()
    assert (p.q, p.ncell) == (9, 512)


def test_traffic_record_is_used_only_for_its_sources(monkeypatch):
    path = os.path.join(ROOT, "profiles", "k_step_ensemble_64_annuli_traffic.json")
    with open(path) as fh:
        rec = json.load(fh)
    f32 = rec["launches"]["f32"]
    # the record describes the D2Q21 group of the 64-annulus workload
    assert f32["cells"] == 9_665_148
    # HBM bytes at least the algorithmic 2 Q s per cell update
    assert f32["hbm_bytes_per_launch"] >= 2 * 21 * 4 * f32["cells"]
    monkeypatch.setattr(bench, "step_source_hash", lambda sources=None: rec["source_sha256"])
    assert bench.recorded_traffic("ensemble_64_annuli", "f32", f32["cells"]) == int(f32["hbm_bytes_per_launch"])
    # another launch size, an unknown workload or changed sources: no figure
    assert bench.recorded_traffic("ensemble_64_annuli", "f32", f32["cells"] + 1) is None
    assert bench.recorded_traffic("wobbled_box_q21_1024x1024", "f32", f32["cells"]) is None
    monkeypatch.setattr(bench, "step_source_hash", lambda sources=None: "0" * 64)
    assert bench.recorded_traffic("ensemble_64_annuli", "f32", f32["cells"]) is None


def test_traffic_records_of_the_large_grid_and_3d_step():
    """The single 4096 x 16384 grid and the 3D step have records of their own,
    keyed to their own kernel sources."""
    for name, prec, cells, q, s, srcs in (("k_step_annulus_couette_4096x16384", "f32", 4096 * 16384, 21, 4,
                                           bench.STEP_SOURCES),
                                          ("k_step3_cylinder_couette_128x512x64", "f64", 128 * 512 * 64, 39, 8,
                                           bench.STEP3_SOURCES)):
        with open(os.path.join(ROOT, "profiles", name + "_traffic.json")) as fh:
            rec = json.load(fh)
        e = rec["launches"][prec]
        assert e["cells"] == cells and e["hbm_bytes_per_launch"] >= 2 * q * s * cells
        assert rec["sources"] == srcs
