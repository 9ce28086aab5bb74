"""Pins of the 3D oracle (CPU only) against what the paper and the
mathematics fix: the isotropy conditions of App. A written for three
dimensions, the moments of Eq. (equilibrium), the Cartesian reduction to a
textbook BGK step written here independently, conservation, the rest state,
the per-cell identities of the correction terms, and the exact profiles of
the paper's flows in their 3D continuations (slab channel, cylinder)."""
import itertools
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle.oracle3d import Oracle3D, feq3, lattice3
from oracle import exact as ex
from paper_2301_01868_amd import grids3d as G3

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "lattice_d3q39.txt")


def _fixture():
    T0, vel, w = None, [], []
    for line in open(GOLDEN):
        if line.startswith("#"):
            continue
        t = line.split()
        if t[0] == "T0":
            T0 = Fr(t[1])
        else:
            vel.append(tuple(int(x) for x in t[:3]))
            w.append(Fr(t[3]))
    return T0, vel, w


def _delta(i, j):
    return 1 if i == j else 0


def _iso(idx):
    """Isotropic tensor Delta^(n) of App. A: the sum over all pairings of the indices."""
    if not idx:
        return 1
    first, rest = idx[0], idx[1:]
    return sum(_delta(first, rest[k]) * _iso(rest[:k] + rest[k + 1:]) for k in range(len(rest)))


def test_lattice3_satisfies_the_isotropy_conditions_exactly():
    T0, vel, w = _fixture()
    assert len(vel) == 39 and sum(w) == 1
    for n in range(1, 7):
        for idx in itertools.product(range(3), repeat=n):
            m = sum(wa * np.prod([c[i] for i in idx]) for c, wa in zip(vel, w))
            want = 0 if n % 2 else T0 ** (n // 2) * _iso(list(idx))
            assert m == want, (idx, m, want)
    # the 8th-order condition fails (the lattice is 6th order, not more)
    idx = (0,) * 8
    m8 = sum(wa * c[0] ** 8 for c, wa in zip(vel, w))
    assert m8 != T0 ** 4 * _iso(list(idx))


def test_lattice3_is_the_unique_solution_for_its_shells():
    """For the six shells of the lattice the seven scalar conditions fix T0
    and the weights: the elimination cubic has T0 = 2/3 as its only positive
    root with positive weights, and the weight system is nonsingular."""
    import sys
    sys.path.insert(0, os.path.dirname(GOLDEN))
    import derive_lattice3d as D
    T0, vel, w = _fixture()
    reps = sorted({tuple(sorted((abs(x) for x in v), reverse=True)) for v in vel})
    shells = [s for s in D.shells(3) if s[0] in reps]
    assert len(shells) == 6
    A = [[Fr(D.moments(vs)[e]) for (_, vs) in shells] for e in range(7)]
    # the 7 x 7 determinant of [A | rhs(T)] is a cubic in T; sample it exactly
    vals = [D.det([A[e] + [D.rhs(Fr(t))[e]] for e in range(7)]) for t in range(4)]
    c3 = (vals[3] - 3 * vals[2] + 3 * vals[1] - vals[0]) / 6
    assert c3 != 0
    roots = np.roots([float(c3), float((vals[2] - 2 * vals[1] + vals[0]) / 2 - 3 * c3),
                      float(vals[1] - vals[0] - (vals[2] - 2 * vals[1] + vals[0]) / 2 + 2 * c3), float(vals[0])])
    pos = []
    for r in roots:
        if abs(r.imag) < 1e-12 and r.real > 1e-12:
            Tr = Fr(float(r.real)).limit_denominator(10 ** 6)
            ww = D.solve([A[e] for e in range(6)], [D.rhs(Tr)[e] for e in range(6)])
            if ww is not None and all(x > 0 for x in ww) and \
                    all(sum(A[e][k] * ww[k] for k in range(6)) == D.rhs(Tr)[e] for e in range(7)):
                pos.append((Tr, ww))
    assert len(pos) == 1 and pos[0][0] == T0 == Fr(2, 3)
    shell_w = {s[0]: x for s, x in zip(shells, pos[0][1])}
    for v, wa in zip(vel, w):
        assert shell_w[tuple(sorted((abs(x) for x in v), reverse=True))] == wa


def test_oracle_lattice_table_is_the_derived_one():
    T0, vel, w = _fixture()
    c, wo, T0o = lattice3()
    assert [tuple(x) for x in c] == vel
    assert np.array_equal(wo, np.array([float(x) for x in w]))
    assert T0o == float(T0)


def _rand_sym(rng):
    A = rng.standard_normal((3, 3))
    G = A @ A.T * 0.2 + np.eye(3)
    return G


def test_equilibrium3_moments():
    """Moments of Eq. (equilibrium) with 6th-order isotropy: sum f = rho,
    sum c f = rho U, sum c c f = rho (T0 G + Ut Ut), and
    sum c c c f = rho [T0 (G_ij Ut_k + G_jk Ut_i + G_ki Ut_j) + Ut_i Ut_j Ut_k]."""
    c, w, T0 = lattice3()
    rng = np.random.default_rng(3)
    for _ in range(5):
        G = _rand_sym(rng)
        U = 0.05 * rng.standard_normal(3)
        Ut = U + 0.01 * rng.standard_normal(3)
        rho = 1.0 + 0.1 * rng.random()
        f = feq3(rho, U, Ut, [G[0, 0], G[0, 1], G[0, 2], G[1, 1], G[1, 2], G[2, 2]])
        cf = c.astype(float)
        assert abs(f.sum() - rho) < 1e-14
        assert np.abs(cf.T @ f - rho * U).max() < 1e-15
        M2 = np.einsum("a,ai,aj->ij", f, cf, cf)
        assert np.abs(M2 - rho * (T0 * G + np.outer(Ut, Ut))).max() < 1e-14
        M3 = np.einsum("a,ai,aj,ak->ijk", f, cf, cf, cf)
        want = rho * (T0 * (np.einsum("ij,k->ijk", G, Ut) + np.einsum("jk,i->ijk", G, Ut) +
                            np.einsum("ki,j->ijk", G, Ut)) + np.einsum("i,j,k->ijk", Ut, Ut, Ut))
        assert np.abs(M3 - want).max() < 1e-14


def _textbook_bgk3(f, cvec, w, T0, tau):
    """Standard BGK on a unit cubic periodic lattice (written independently):
    third-order Hermite equilibrium, pull streaming by array shifts."""
    rho = f.sum(-1)
    U = np.einsum("...a,ad->...d", f, cvec) / rho[..., None]
    cu = np.einsum("ad,...d->...a", cvec, U)
    uu = (U * U).sum(-1)[..., None]
    cc = (cvec * cvec).sum(-1)
    # H3 : UUU = (c.U)^3 - 3 T0 |U|^2 (c.U)
    feq = rho[..., None] * w * (1 + cu / T0 + (cu ** 2 - T0 * uu) / (2 * T0 ** 2)
                                + (cu ** 3 - 3 * T0 * uu * cu) / (6 * T0 ** 3))
    del cc
    post = f - (f - feq) / tau
    out = np.empty_like(post)
    for a, cv in enumerate(cvec):
        out[..., a] = np.roll(post[..., a], shift=tuple(int(x) for x in cv), axis=(0, 1, 2))
    return out


def test_cartesian_box_reduces_to_textbook_bgk():
    """On cubic unit cells the metric terms vanish (Theta = 0 exactly, F = dPi
    = 0) and the oracle's step is the standard BGK step."""
    n1, n2, n3 = 7, 6, 9
    case = G3.box3(n1, n2, n3, d=(1.0, 1.0, 1.0), tau=0.8)
    o = Oracle3D(case)
    c, w, T0 = lattice3()
    rng = np.random.default_rng(5)
    u0 = 0.03 * rng.standard_normal((o.ncell, 3))
    o.init(1.0, u0)
    P0 = o.get_state()
    # one oracle step = collide the state then stream (the state is post-collision N');
    # the textbook step below streams first, so compare after streaming both ways:
    o.step(1)
    P1 = o.get_state().reshape(n1, n2, n3, 39)
    # oracle: P1(q) = collide(pull(P0))(q); textbook: pull then collide
    f = P0.reshape(n1, n2, n3, 39)
    pulled = np.empty_like(f)
    for a, cv in enumerate(c):
        pulled[..., a] = np.roll(f[..., a], shift=tuple(int(x) for x in cv), axis=(0, 1, 2))
    rho = pulled.sum(-1)
    U = np.einsum("...a,ad->...d", pulled, c.astype(float)) / rho[..., None]
    cu = np.einsum("ad,...d->...a", c.astype(float), U)
    uu = (U * U).sum(-1)[..., None]
    feq = rho[..., None] * w * (1 + cu / T0 + (cu ** 2 - T0 * uu) / (2 * T0 ** 2)
                                + (cu ** 3 - 3 * T0 * uu * cu) / (6 * T0 ** 3))
    want = pulled - (pulled - feq) / 0.8
    assert np.abs(P1 - want).max() < 1e-15 * 10
    # and the independent stepper agrees over a few steps (stream-collide order)
    o2 = Oracle3D(case)
    o2.init(1.0, u0)
    o2.step(3)
    g = P0.reshape(n1, n2, n3, 39)
    # the textbook stepper collides then streams; the oracle streams then
    # collides: three oracle steps = stream, (collide, stream) x 2, collide
    s = pulled
    for _ in range(2):
        s = _textbook_bgk3(s, c.astype(float), w, T0, 0.8)
    rho = s.sum(-1)
    U = np.einsum("...a,ad->...d", s, c.astype(float)) / rho[..., None]
    cu = np.einsum("ad,...d->...a", c.astype(float), U)
    uu = (U * U).sum(-1)[..., None]
    feq = rho[..., None] * w * (1 + cu / T0 + (cu ** 2 - T0 * uu) / (2 * T0 ** 2)
                                + (cu ** 3 - 3 * T0 * uu * cu) / (6 * T0 ** 3))
    s = s - (s - feq) / 0.8
    assert np.abs(o2.get_state().reshape(n1, n2, n3, 39) - s).max() < 1e-14
    del g


def test_mass_conserved_and_rest_kept():
    rng = np.random.default_rng(7)
    # a non-cubic, sheared periodic box: uniform metric (Theta = 0), rest stays rest
    box = G3.box3(5, 6, 7, d=(1.0, 1.1, 0.9), skew=0.1, tau=0.9)
    o = Oracle3D(box)
    o.init(1.0)
    o.step(50)
    m, U, Ut = o.moments()
    assert np.abs(Ut).max() < 1e-14
    # a wobbled box (metric terms vary with q3) from a random start: mass conserved
    wob = G3.box3(5, 6, 8, d=(1.0, 1.1, 0.9), wobble=0.2, tau=0.9)
    o = Oracle3D(wob)
    o.init(1.0, 0.02 * rng.standard_normal((wob.ncell, 3)))
    M0 = o.get_state().sum()
    o.step(30)
    assert abs(o.get_state().sum() - M0) < 1e-13 * M0
    # a channel with a moving wall (specular source plus correction) and a resting one
    ch = G3.couette3(G3.faces_linear(8, 0.3), n2=4, n3=5, d2=1.2, d3=0.8, u_wall=(0.05, 0.02), tau=0.8)
    o = Oracle3D(ch)
    o.init(1.0)
    M0 = o.get_state().sum()
    o.step(40)
    assert abs(o.get_state().sum() - M0) < 1e-13 * M0
    # a uniform channel with walls at rest keeps the rest state
    rest = G3.channel3(G3.faces_uniform(8), 3, 4, d2=1.1, d3=0.9, tau=0.8)
    o = Oracle3D(rest)
    o.init(1.0)
    o.step(40)
    assert np.abs(o.moments()[2]).max() < 1e-14


def test_per_cell_identities():
    """Collision keeps each cell's mass; the momentum of N' equals
    m (U + a) with a = F / rho = 2 (Ut - U), i.e. the correction carries J F
    (Eqs. collide, deltaN with 4th-order isotropy)."""
    rng = np.random.default_rng(11)
    cyl = G3.circular_couette3(6, 24, 8.0, n3=4, dz=0.9, u_inner=0.05, tau=0.8)
    o = Oracle3D(cyl)
    o.init(1.0, 0.01 * rng.standard_normal((cyl.ncell, 3)))
    o.step(3)
    m, U, Ut = o.moments()
    cells = np.arange(o.ncell, dtype=np.int32)
    Np = o.step_cells(cells)
    c, w, T0 = lattice3()
    assert np.abs(Np.sum(1) - m).max() < 1e-13 * m.max()
    mom = Np @ c.astype(float)
    want = m[:, None] * (2 * Ut - U)
    assert np.abs(mom - want).max() < 1e-13 * m.max()


def _couette_profile(N, axis, tau=0.8):
    u_wall = (0.05, 0.0) if axis == 1 else (0.0, 0.05)
    case = G3.couette3(G3.faces_uniform(N), d2=1.1, d3=0.9, u_wall=u_wall, tau=tau)
    o = Oracle3D(case)
    o.init(1.0)
    o.step(int(6 * N * N / G3.viscosity3(tau)) + 200)
    u = o.physical_velocity()
    x = case.meta["centres"]
    other = 2 if axis == 1 else 1
    assert np.abs(u[:, other]).max() < 1e-14       # no flow across the sliding direction
    return np.abs(u[:, axis] - ex.planar_couette(x, case.meta["l"], 0.0, 0.05)).max() / 0.05


@pytest.mark.parametrize("axis", [1, 2], ids=["slide_y", "slide_z"])
def test_planar_couette3_profile(axis):
    """The slab channel with a wall sliding along y (q2) or along z (q3),
    cells of 1 x 1.1 x 0.9: the moving-wall correction acts on either
    tangential component, and the flow reaches the linear profile of Sec. 3.1
    to an error that shrinks under refinement."""
    e8, e16 = _couette_profile(8, axis), _couette_profile(16, axis)
    assert e8 < 5e-2 and e16 < e8


def test_planar_poiseuille3_parabola():
    """The slab channel driven along z between walls at rest: the parabola of
    Sec. 3.2 to second order in the wall-normal step."""
    errs = []
    for N in (8, 16):
        nu = G3.viscosity3(1.0)
        g = 8 * nu * 0.02 / N ** 2
        case = G3.poiseuille3(G3.faces_uniform(N), g=(0.0, g), tau=1.0)
        o = Oracle3D(case)
        o.init(1.0)
        o.step(int(6 * N * N / nu) + 200)
        u = o.physical_velocity()[:, 2]
        sol = ex.planar_poiseuille(case.meta["centres"], case.meta["l"], g, nu)
        errs.append(np.abs(u - sol).max() / sol.max())
    assert errs[1] < errs[0] < 2e-2 and errs[0] / errs[1] > 3.0, errs


def test_stream_map_is_a_permutation():
    """Every (cell, direction) of the post-collision field is pulled exactly
    once (periodic seams, mirror sources at both walls), so streaming keeps
    the mass exactly."""
    for case in (G3.couette3(G3.faces_uniform(5), n2=4, n3=3, u_wall=(0.05, 0.01)),
                 G3.box3(4, 3, 5),
                 G3.circular_couette3(4, 8, 6.0, n3=2)):
        o = Oracle3D(case)
        sc, sd, wl = o.stream_map()
        pairs = sc.astype(np.int64) * 39 + sd
        assert np.array_equal(np.sort(pairs.ravel()), np.arange(case.ncell * 39))


def _circular(N, problem):
    from paper_2301_01868_amd import grids as G2
    M = float(N)         # R2 / R1 = 2
    nu = G3.viscosity3(1.0)
    if problem == "couette":
        case = G3.circular_couette3(N, 4 * N, M, n2=1, u_inner=0.05, tau=1.0)
        sol = lambda r: ex.circular_couette(r, M, M + N, 0.05 / M, 0.0)
    else:
        # the same polar geometry as the 2D flows: g2 for a peak speed of 0.05
        g2 = G2.poiseuille_g2_for_peak(N, 4 * N, M, nu, 0.05)
        case = G3.circular_poiseuille3(N, 4 * N, M, n2=1, g2=g2, tau=1.0)
        K = g2 * np.sin(case.meta["dtheta"])
        sol = lambda r: ex.circular_poiseuille(r, M, M + N, K, nu)
    o = Oracle3D(case)
    o.init(1.0)
    o.step(int(5 * N * N / nu) + 500)
    m, U, Ut = o.moments()
    r = case.meta["centres"]
    uth = Ut[:, 1] * r * np.sin(case.meta["dtheta"])     # App. D: u_theta = U^2 sin(dtheta) r
    return np.abs(uth - sol(r)).max() / 0.05


@pytest.mark.parametrize("problem", ["couette", "poiseuille"])
def test_circular_flows3_converge(problem):
    """Circular Couette and circular Poiseuille flow in a cylinder, on the
    exact theta and z reduction (one column continued with the true angular
    step and one layer): the error against the exact profile shrinks as the
    radial resolution doubles."""
    errs = [_circular(N, problem) for N in (8, 16, 32)]
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 0.02, errs
