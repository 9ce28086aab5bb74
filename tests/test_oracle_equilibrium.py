"""Equilibrium moment identities of Eq. (equilibrium) (CPU only).

The expected moments follow from the equilibrium's Hermite structure and the
isotropy of App. A; the third moment is exact only for the 6th-order
isotropic D2Q21, which is the concrete form of the paper's isotropy argument
for curvilinear grids (Sec. 3.3)."""
import numpy as np
import pytest

import oracle


def _rand_inputs(rng):
    A = rng.normal(size=(2, 2))
    G = A @ A.T + 0.3 * np.eye(2)
    U = rng.normal(scale=0.1, size=2)
    Ut = rng.normal(scale=0.1, size=2)
    rho = rng.uniform(0.5, 1.5)
    return rho, U, Ut, G


@pytest.mark.parametrize("q", [9, 21])
def test_moments_0_to_2(q):
    c, w, T0, *_ = oracle.lattice(q)
    rng = np.random.default_rng(7)
    for _ in range(20):
        rho, U, Ut, G = _rand_inputs(rng)
        f = oracle.feq(q, rho, U, Ut, [G[0, 0], G[0, 1], G[1, 1]])
        assert abs(f.sum() - rho) < 1e-14
        assert np.allclose(c.T @ f, rho * U, atol=1e-14, rtol=0)
        P2 = np.einsum("a,ai,aj->ij", f, c, c)
        assert np.allclose(P2, rho * (T0 * G + np.outer(Ut, Ut)), atol=1e-13, rtol=0)


def _third_expected(rho, Ut, G, T0):
    E = np.zeros((2, 2, 2))
    for i in range(2):
        for j in range(2):
            for k in range(2):
                E[i, j, k] = rho * (T0 * (G[i, j] * Ut[k] + G[j, k] * Ut[i] + G[k, i] * Ut[j]) + Ut[i] * Ut[j] * Ut[k])
    return E


def test_third_moment_exact_for_q21_only():
    rng = np.random.default_rng(11)
    for q in (21, 9):
        c, w, T0, *_ = oracle.lattice(q)
        for _ in range(20):
            rho, U, Ut, G = _rand_inputs(rng)
            f = oracle.feq(q, rho, U, Ut, [G[0, 0], G[0, 1], G[1, 1]])
            P3 = np.einsum("a,ai,aj,ak->ijk", f, c, c, c)
            E = _third_expected(rho, Ut, G, T0)
            if q == 21:
                assert np.allclose(P3, E, atol=1e-13, rtol=0)
            else:
                # D2Q9: c^3 = c on the lattice, so the xxx component equals the
                # first moment rho U^1 instead of rho (3 T0 g^11 Ut^1 + Ut^1^3).
                d = P3 - E
                assert abs(d[0, 0, 0] - rho * (U[0] - G[0, 0] * Ut[0] - Ut[0] ** 3)) < 1e-13
                assert abs(d[1, 1, 1] - rho * (U[1] - G[1, 1] * Ut[1] - Ut[1] ** 3)) < 1e-13
                assert np.allclose(d[0, 0, 1], 0, atol=1e-13) and np.allclose(d[0, 1, 1], 0, atol=1e-13)


@pytest.mark.parametrize("q", [9, 21])
def test_cartesian_reduces_to_textbook_hermite(q):
    """With g^ij = delta^ij and Ut = U the equilibrium is the standard
    third-order Hermite form rho w [1 + cu/T + ((cu)^2 - T u^2)/(2T^2) +
    cu ((cu)^2 - 3 T u^2)/(6 T^3)]."""
    c, w, T0, *_ = oracle.lattice(q)
    rng = np.random.default_rng(3)
    for _ in range(10):
        u = rng.normal(scale=0.1, size=2)
        rho = rng.uniform(0.8, 1.2)
        f = oracle.feq(q, rho, u, u, [1.0, 0.0, 1.0])
        cu = c @ u
        uu = u @ u
        ref = rho * w * (1 + cu / T0 + (cu ** 2 - T0 * uu) / (2 * T0 ** 2) + cu * (cu ** 2 - 3 * T0 * uu) / (6 * T0 ** 3))
        assert np.allclose(f, ref, atol=1e-15, rtol=1e-14)


def test_rest_equilibrium_closed_form_q21():
    """Rest state on a curved cell: rho w (1 + [(c.G.c - |c|^2)/T0 - (tr G - 2)]/2);
    for c = (0, 3) this is rho w (25 g22/4 - g11/2 - 19/4)."""
    c, w, T0, *_ = oracle.lattice(21)
    G = np.array([[1.0, 0.0], [0.0, 0.1]])
    f = oracle.feq(21, 1.0, [0, 0], [0, 0], [1.0, 0.0, 0.1])
    a = 18  # (0, 3)
    assert abs(f[a] - w[a] * (25 * G[1, 1] / 4 - G[0, 0] / 2 - 19 / 4)) < 1e-15
    cGc = np.einsum("ai,ij,aj->a", c, G, c)
    ref = w * (1 + 0.5 * ((cGc - (c * c).sum(1)) / T0 - (np.trace(G) - 2)))
    assert np.allclose(f, ref, atol=1e-15)
