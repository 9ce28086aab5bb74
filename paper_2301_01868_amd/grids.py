"""Seeded synthetic inputs: body-fitted grids (the mapping x(q)) and cases.

This module only generates inputs.  It holds none of the method's
arithmetic (no geometry derivatives, no lattice tables, no update): it
produces cell-centre coordinates on the halo-extended computational range,
the boundary description and the run parameters, which both the HIP library
and the CPU oracle consume.

Conventions shared with the library's C ABI:
  * q1 is the wall-normal index (i = 1..n1, walls at i = 1/2 and n1 + 1/2,
    the half-spaced lattice of App. B), q2 the periodic index (j = 1..n2);
  * coordinates are in lattice units: the mean wall-normal step is 1, the
    time step is 1;
  * ``X``, ``Y`` have shape (n1 + 2h, n2 + 2h), q2 fastest; ghost rows beyond a
    wall hold the mirror image of the interior rows across the wall (the
    "symmetrically continued geometry" of Sec. 3.1); the periodic direction
    simply continues the mapping.

Grid families (the paper's):
  * planar channels with uniform, linearly contracting (App. C) or
    geometrically stretched wall-normal faces;
  * polar annuli on the half-spaced (r, theta) lattice (App. D), optionally
    reduced to fewer theta columns than the true N_theta: the periodic q2
    direction is then continued with the true angular step, which is exact for
    theta-invariant states.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

CMAX = {9: 1, 21: 3}
T0 = {9: 1.0 / 3.0, 21: 2.0 / 3.0}   # lattice temperature of App. A (input parameter)


@dataclass
class Case:
    q: int
    n1: int
    n2: int
    halo: int
    X: np.ndarray
    Y: np.ndarray
    periodic1: bool = False
    bc_lo: str = "noslip"          # "noslip" | "moving" | "periodic"
    bc_hi: str = "noslip"
    ut_lo: float = 0.0             # contravariant tangential wall velocity U0^2
    ut_hi: float = 0.0
    tau: float = 1.0
    accel: tuple = (0.0, 0.0)      # contravariant external acceleration a^i
    rho0: float = 1.0
    meta: dict = field(default_factory=dict)

    @property
    def ncell(self):
        return self.n1 * self.n2

    def replace(self, **kw):
        d = dict(self.__dict__)
        d.update(kw)
        return Case(**d)

    def no_flow(self):
        """Same geometry and boundary kinds, wall speeds and force zeroed."""
        return self.replace(ut_lo=0.0, ut_hi=0.0, accel=(0.0, 0.0), meta=dict(self.meta, no_flow=True))


def viscosity(q, tau):
    """Lattice kinematic viscosity nu = T0 (tau - 1/2) (Tables of Sec. 3)."""
    return T0[q] * (tau - 0.5)


# ---------------------------------------------------------------------------
# wall-normal face positions (0 = x'_0 < ... < x'_N = N, mean step 1)
# ---------------------------------------------------------------------------
def faces_uniform(N):
    return np.arange(N + 1, dtype=np.float64)


def faces_linear(N, CR):
    """App. C linearly contracting lattice, contraction ratio CR = (1 - D'_1)."""
    assert N % 2 == 0 and N >= 4
    a = 2.0 * CR / (N / 2 - 1)
    i = np.arange(N + 1, dtype=np.float64)
    left = i * (1.0 + 0.5 * a * (i - N / 2))
    right = N / 2 + (i - N / 2) * (1.0 + 0.5 * a * (N - i))
    return np.where(i <= N / 2, left, right)


def faces_geometric(N, ratio):
    """Symmetric faces whose cell size grows by ``ratio`` per cell from each wall."""
    assert N % 2 == 0
    K = N // 2
    h0 = K * (ratio - 1.0) / (ratio ** K - 1.0) if ratio != 1.0 else 1.0
    sizes = h0 * ratio ** np.arange(K)
    sizes = np.concatenate([sizes, sizes[::-1]])
    f = np.concatenate([[0.0], np.cumsum(sizes)])
    f[-1] = float(N)
    return f


def _reflect_rows(c, n1, h, lo, hi):
    """Extend interior centres c[0:n1] by h mirror rows at both walls (repeated
    reflection when the channel is narrower than the halo)."""
    def pos(k):   # 1-based row index
        if k < 1:
            return 2.0 * lo - pos(1 - k)
        if k > n1:
            return 2.0 * hi - pos(2 * n1 + 1 - k)
        return c[k - 1]
    return np.array([pos(k) for k in range(1 - h, n1 + h + 1)], dtype=np.float64)


# ---------------------------------------------------------------------------
# planar channel: X wall-normal (q1), Y periodic (q2)
# ---------------------------------------------------------------------------
def planar_channel(q, faces, n2, d_per=1.0, halo=None, **kw):
    n1 = len(faces) - 1
    h = halo if halo is not None else CMAX[q] + 1
    cen = 0.5 * (faces[1:] + faces[:-1])
    Xr = _reflect_rows(cen, n1, h, faces[0], faces[-1])
    jj = np.arange(-h, n2 + h, dtype=np.float64)      # 0-based j = -h .. n2+h-1
    Yc = (jj + 0.5) * d_per
    X = np.repeat(Xr[:, None], n2 + 2 * h, axis=1)
    Y = np.repeat(Yc[None, :], n1 + 2 * h, axis=0)
    meta = dict(family="planar", faces=np.asarray(faces), centres=cen, d_per=d_per, l=float(faces[-1] - faces[0]))
    meta.update(kw.pop("meta", {}))
    return Case(q=q, n1=n1, n2=n2, halo=h, X=np.ascontiguousarray(X), Y=np.ascontiguousarray(Y), meta=meta, **kw)


def planar_couette(q, faces, n2=1, d_per=1.0, u_wall=0.05, tau=1.0, moving="hi", **kw):
    """Planar Couette: one wall at rest, the other sliding at physical speed u_wall."""
    ut = u_wall / d_per          # contravariant component along g_2 = d_per * y-hat
    lo, hi = ("moving", "noslip") if moving == "lo" else ("noslip", "moving")
    c = planar_channel(q, faces, n2, d_per=d_per, bc_lo=lo, bc_hi=hi,
                       ut_lo=ut if moving == "lo" else 0.0, ut_hi=ut if moving == "hi" else 0.0, tau=tau, **kw)
    c.meta.update(problem="planar_couette", u_wall=u_wall, moving=moving)
    return c


def planar_poiseuille(q, faces, n2=1, d_per=1.0, g=1e-6, tau=1.0, **kw):
    """Planar Poiseuille driven by a uniform physical acceleration g along q2."""
    c = planar_channel(q, faces, n2, d_per=d_per, bc_lo="noslip", bc_hi="noslip", tau=tau,
                       accel=(0.0, g / d_per), **kw)
    c.meta.update(problem="planar_poiseuille", g=g)
    return c


def periodic_box(q, n1, n2, dx=1.0, dy=1.0, skew=0.0, wobble=0.0, halo=None, **kw):
    """Doubly periodic Cartesian (optionally sheared / smoothly wobbled) grid."""
    h = halo if halo is not None else CMAX[q] + 1
    ii = np.arange(-h, n1 + h, dtype=np.float64)[:, None] + 0.5
    jj = np.arange(-h, n2 + h, dtype=np.float64)[None, :] + 0.5
    X = dx * ii + skew * jj + wobble * np.sin(2 * np.pi * jj / n2)
    Y = dy * jj + wobble * np.sin(2 * np.pi * ii / n1)
    c = Case(q=q, n1=n1, n2=n2, halo=h, X=np.ascontiguousarray(X), Y=np.ascontiguousarray(Y), periodic1=True,
             bc_lo="periodic", bc_hi="periodic", **kw)
    c.meta.update(family="box", dx=dx, dy=dy, skew=skew, wobble=wobble)
    return c


# ---------------------------------------------------------------------------
# polar annulus: r wall-normal (q1), theta periodic (q2)
# ---------------------------------------------------------------------------
def polar_annulus(q, Nr, Ntheta, M, n2=None, halo=None, r_faces=None, **kw):
    """Half-spaced polar lattice (App. D) in units of the mean radial step.

    R1 = M, R2 = M + Nr; r_i = M + (i - 1/2) for uniform radial faces;
    theta_j = (j - 1/2) * 2 pi / Ntheta.  ``n2`` < Ntheta keeps only n2 columns
    but continues them with the true angular step (theta-invariant states)."""
    h = halo if halo is not None else CMAX[q] + 1
    n2 = Ntheta if n2 is None else n2
    faces = (M + np.arange(Nr + 1, dtype=np.float64)) if r_faces is None else np.asarray(r_faces, dtype=np.float64)
    cen = 0.5 * (faces[1:] + faces[:-1])
    R1, R2 = float(faces[0]), float(faces[-1])
    r = _reflect_rows(cen, Nr, h, R1, R2)
    if r.min() <= 0:
        raise ValueError("inner radius too small for the ghost layers")
    dth = 2.0 * np.pi / Ntheta
    th = (np.arange(-h, n2 + h, dtype=np.float64) + 0.5) * dth
    X = r[:, None] * np.cos(th)[None, :]
    Y = r[:, None] * np.sin(th)[None, :]
    meta = dict(family="polar", Nr=Nr, Ntheta=Ntheta, M=M, R1=R1, R2=R2, dtheta=dth, centres=cen, faces=faces)
    meta.update(kw.pop("meta", {}))
    return Case(q=q, n1=Nr, n2=n2, halo=h, X=np.ascontiguousarray(X), Y=np.ascontiguousarray(Y), meta=meta, **kw)


def wall_ut_polar(R_wall, dtheta, u_wall):
    """Contravariant U0^2 of a wall sliding at physical speed u_wall (App. D:
    |g_2| = r sin(dtheta) on the wall, in units of the mean radial step)."""
    return u_wall / (R_wall * math.sin(dtheta))


def circular_couette(q, Nr, Ntheta, M, u_inner=0.05, u_outer=0.0, tau=1.0, n2=None, **kw):
    """Inner cylinder sliding at u_inner, outer at u_outer (rest: no-slip)."""
    dth = 2.0 * np.pi / Ntheta
    R1, R2 = float(M), float(M + Nr)
    lo = "moving" if u_inner != 0.0 else "noslip"
    hi = "moving" if u_outer != 0.0 else "noslip"
    c = polar_annulus(q, Nr, Ntheta, M, n2=n2, bc_lo=lo, bc_hi=hi, ut_lo=wall_ut_polar(R1, dth, u_inner),
                      ut_hi=wall_ut_polar(R2, dth, u_outer), tau=tau, **kw)
    c.meta.update(problem="circular_couette", u_inner=u_inner, u_outer=u_outer)
    return c


def circular_poiseuille(q, Nr, Ntheta, M, g2=1e-6, tau=1.0, n2=None, **kw):
    """Annulus with no-slip walls driven by a constant contravariant force g^2
    (Sec. 3.4: physical azimuthal acceleration K r with K = g^2 sin(dtheta))."""
    c = polar_annulus(q, Nr, Ntheta, M, n2=n2, bc_lo="noslip", bc_hi="noslip", tau=tau, accel=(0.0, g2), **kw)
    c.meta.update(problem="circular_poiseuille", g2=g2, K=g2 * math.sin(2 * np.pi / Ntheta))
    return c


def poiseuille_g2_for_peak(Nr, Ntheta, M, nu, u_peak):
    """Force g^2 whose annular profile K (r^2-R1^2)(R2^2-r^2)/(8 nu r) peaks at u_peak."""
    R1, R2 = float(M), float(M + Nr)
    r = np.linspace(R1, R2, 20001)
    shape = (r ** 2 - R1 ** 2) * (R2 ** 2 - r ** 2) / (8.0 * nu * r)
    K = u_peak / shape.max()
    return K / math.sin(2 * np.pi / Ntheta)


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------
def eccentric_annulus(q, Nr, Ntheta, M, ecc, u_inner=0.05, tau=1.0, n2=None, halo=None, **kw):
    """Journal bearing: the gap between an inner circle of radius R1 = M centred
    at (ecc, 0), sliding at u_inner, and an outer circle of radius R2 = M + Nr
    centred at the origin, at rest.  Each theta line blends the two walls,
    x(s, theta) = (1 - s) (c + R1 e(theta)) + s R2 e(theta) with
    e = (cos theta, sin theta), c = (ecc, 0) and s = (i - 1/2) / Nr, so the
    mean wall-normal step is 1.  For ecc != 0 the grid is not orthogonal
    (g_1 . g_2 = -ecc sin(theta) |g_2| / Nr) and its metric terms depend on q2.
    The ghost rows continue the blend beyond s = 0 and 1, which places them at
    the mirror image of the interior rows through the wall point of the same
    theta index."""
    h = halo if halo is not None else CMAX[q] + 1
    n2 = Ntheta if n2 is None else n2
    R1, R2 = float(M), float(M + Nr)
    if not 0.0 <= ecc < 0.5 * Nr:
        raise ValueError("eccentricity must leave the gap at least half its mean width")
    sc = (np.arange(Nr, dtype=np.float64) + 0.5) / Nr
    s = _reflect_rows(sc, Nr, h, 0.0, 1.0)
    dth = 2.0 * np.pi / Ntheta
    th = (np.arange(-h, n2 + h, dtype=np.float64) + 0.5) * dth
    cs, sn = np.cos(th)[None, :], np.sin(th)[None, :]
    S = s[:, None]
    X = (1.0 - S) * (ecc + R1 * cs) + S * R2 * cs
    Y = (1.0 - S) * R1 * sn + S * R2 * sn
    c = Case(q=q, n1=Nr, n2=n2, halo=h, X=np.ascontiguousarray(X), Y=np.ascontiguousarray(Y),
             bc_lo="moving" if u_inner != 0.0 else "noslip", bc_hi="noslip", ut_lo=wall_ut_polar(R1, dth, u_inner),
             tau=tau, **kw)
    c.meta.update(family="eccentric", problem="journal_bearing", Nr=Nr, Ntheta=Ntheta, M=M, R1=R1, R2=R2, ecc=ecc,
                  dtheta=dth, u_inner=u_inner)
    return c


def workload_planar_couette_q9():
    """Planar Couette, D2Q9, 16 wall-normal x 32 periodic cells with the
    periodic step twice the wall-normal step (dx = 2 dy), one wall at rest,
    the other sliding at 0.05, tau = 1.  The channel is drawn with its walls
    normal to X (the paper's orientation)."""
    return planar_couette(9, faces_uniform(16), n2=32, d_per=2.0, u_wall=0.05, tau=1.0, moving="hi",
                          meta=dict(workload="planar_couette_q9_32x16"))


def workload_planar_poiseuille(Ny, tau, q=21, ratio=1.02, n_per=16, g=1e-6):
    """Planar Poiseuille on a geometrically stretched channel (ratio per cell
    from both walls), Ny wall-normal x n_per periodic cells."""
    return planar_poiseuille(q, faces_geometric(Ny, ratio), n2=n_per, d_per=1.0, g=g, tau=tau,
                             meta=dict(workload="planar_poiseuille_%dx%d" % (n_per, Ny), ratio=ratio))


def workload_annulus_couette(Nr=256, Ntheta=1024, R1=1.0, R2=2.0, tau=0.8, q=21, u_inner=0.05, n2=None):
    """Circular Couette in the annulus R1..R2 on a uniform polar grid."""
    M = R1 / ((R2 - R1) / Nr)
    c = circular_couette(q, Nr, Ntheta, M, u_inner=u_inner, tau=tau, n2=n2)
    c.meta.update(workload="annulus_couette_%dx%d" % (Nr, Ntheta))
    return c


def workload_ensemble(seed=2301_01868, n=64):
    """Seed-fixed ensemble of annuli: half circular Couette, half circular
    Poiseuille; Nr ~ U{32..512}, Ntheta = 4 Nr, R2/R1 ~ U(1.5, 4) with
    R2 - R1 = Nr, tau ~ U(0.55, 1.0), Q ~ {9, 21} with equal odds."""
    rng = np.random.default_rng(seed)
    cases = []
    for k in range(n):
        Nr = int(rng.integers(32, 513))
        ratio = float(rng.uniform(1.5, 4.0))
        tau = float(rng.uniform(0.55, 1.0))
        q = 21 if rng.random() < 0.5 else 9
        M = Nr / (ratio - 1.0)
        Nt = 4 * Nr
        if k < n // 2:
            c = circular_couette(q, Nr, Nt, M, u_inner=0.05, tau=tau)
        else:
            g2 = poiseuille_g2_for_peak(Nr, Nt, M, viscosity(q, tau), 0.05)
            c = circular_poiseuille(q, Nr, Nt, M, g2=g2, tau=tau)
        c.meta.update(instance=k, ratio=ratio)
        cases.append(c)
    return cases
