"""Seeded synthetic inputs for the three-dimensional form of the method: the
mapping x(q) of body-fitted 3D grids and the cases built on them.

Like ``grids``, this module only generates inputs and holds none of the
method's arithmetic: cell-centre coordinates on the halo-extended
computational range, the boundary description and the run parameters, which
the HIP library and the CPU oracle both consume.

Conventions (shared with ``include/lbm3d.h``):
  * q1 is the wall-normal index (walls at i = 1/2 and n1 + 1/2, or periodic),
    q2 and q3 are periodic;
  * ``X``, ``Y``, ``Z`` have shape (n1 + 2h, n2 + 2h, n3 + 2h), q3 fastest;
    ghost rows beyond a wall hold the mirror image of the interior rows across
    the wall at the same (q2, q3) (the symmetrically continued geometry of
    Sec. 3.1); the periodic directions continue the mapping;
  * lengths in lattice units (mean wall-normal step 1, time step 1).

Families: the paper's planar channel and annulus, continued along a third,
periodic axis (a slab channel and a cylinder), and doubly or triply periodic
boxes whose cells are not cubes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .grids import _reflect_rows, faces_uniform, faces_linear  # noqa: F401  (face generators)

Q3 = 39            # velocities of the 3D lattice (derived in tests/golden/derive_lattice3d.py)
CMAX3 = 3
T0_3 = 2.0 / 3.0   # its lattice temperature (input parameter)


def viscosity3(tau):
    """Lattice kinematic viscosity nu = T0 (tau - 1/2)."""
    return T0_3 * (tau - 0.5)


@dataclass
class Case3:
    n1: int
    n2: int
    n3: int
    halo: int
    X: np.ndarray
    Y: np.ndarray
    Z: np.ndarray
    periodic1: bool = False
    bc_lo: str = "noslip"            # "noslip" | "moving" | "periodic"
    bc_hi: str = "noslip"
    ut_lo: tuple = (0.0, 0.0)        # contravariant tangential wall velocity (U0^2, U0^3)
    ut_hi: tuple = (0.0, 0.0)
    tau: float = 1.0
    accel: tuple = (0.0, 0.0, 0.0)   # contravariant external acceleration a^i
    rho0: float = 1.0
    meta: dict = field(default_factory=dict)
    q: int = Q3

    @property
    def ncell(self):
        return self.n1 * self.n2 * self.n3

    def replace(self, **kw):
        d = dict(self.__dict__)
        d.update(kw)
        return Case3(**d)


def _axis(n, h, d, off=0.0):
    return (np.arange(-h, n + h, dtype=np.float64) + 0.5) * d + off


def box3(n1, n2, n3, d=(1.0, 1.0, 1.0), skew=0.0, wobble=0.0, tau=1.0, halo=CMAX3 + 1, **kw):
    """Triply periodic box of cells d1 x d2 x d3; skew shears x by skew * y;
    wobble adds a smooth periodic displacement of x along q3 (so the metric
    terms depend on the position)."""
    h = halo
    a1, a2, a3 = _axis(n1, h, d[0]), _axis(n2, h, d[1]), _axis(n3, h, d[2])
    A1, A2, A3 = np.meshgrid(a1, a2, a3, indexing="ij")
    k = (np.arange(-h, n3 + h) + 0.5)[None, None, :] * np.ones_like(A1)
    X = A1 + skew * A2 + wobble * np.sin(2.0 * np.pi * k / n3)
    meta = dict(family="box3", d=tuple(d), skew=skew, wobble=wobble)
    meta.update(kw.pop("meta", {}))
    return Case3(n1=n1, n2=n2, n3=n3, halo=h, X=np.ascontiguousarray(X), Y=np.ascontiguousarray(A2),
                 Z=np.ascontiguousarray(A3), periodic1=True, bc_lo="periodic", bc_hi="periodic", tau=tau, meta=meta,
                 **kw)


def channel3(faces, n2, n3, d2=1.0, d3=1.0, halo=CMAX3 + 1, **kw):
    """Slab channel: q1 wall-normal along x with the given faces, q2 along y
    (step d2) and q3 along z (step d3) periodic."""
    n1 = len(faces) - 1
    h = halo
    cen = 0.5 * (faces[1:] + faces[:-1])
    xr = _reflect_rows(cen, n1, h, faces[0], faces[-1])
    X = np.broadcast_to(xr[:, None, None], (n1 + 2 * h, n2 + 2 * h, n3 + 2 * h))
    Y = np.broadcast_to(_axis(n2, h, d2)[None, :, None], X.shape)
    Z = np.broadcast_to(_axis(n3, h, d3)[None, None, :], X.shape)
    meta = dict(family="channel3", faces=np.asarray(faces), centres=cen, d2=d2, d3=d3,
                l=float(faces[-1] - faces[0]))
    meta.update(kw.pop("meta", {}))
    return Case3(n1=n1, n2=n2, n3=n3, halo=h, X=np.ascontiguousarray(X), Y=np.ascontiguousarray(Y),
                 Z=np.ascontiguousarray(Z), meta=meta, **kw)


def couette3(faces, n2=1, n3=1, d2=1.0, d3=1.0, u_wall=(0.05, 0.0), tau=1.0, **kw):
    """Planar Couette flow in the slab channel: the low wall at rest, the high
    wall sliding at the physical velocity u_wall = (along y, along z)."""
    ut = (u_wall[0] / d2, u_wall[1] / d3)
    c = channel3(faces, n2, n3, d2=d2, d3=d3, bc_lo="noslip", bc_hi="moving", ut_hi=ut, tau=tau, **kw)
    c.meta.update(problem="planar_couette", u_wall=tuple(u_wall))
    return c


def poiseuille3(faces, n2=1, n3=1, d2=1.0, d3=1.0, g=(1e-5, 0.0), tau=1.0, **kw):
    """Planar Poiseuille flow in the slab channel driven by the physical
    acceleration g = (along y, along z); both walls at rest."""
    c = channel3(faces, n2, n3, d2=d2, d3=d3, bc_lo="noslip", bc_hi="noslip",
                 accel=(0.0, g[0] / d2, g[1] / d3), tau=tau, **kw)
    c.meta.update(problem="planar_poiseuille", g=tuple(g))
    return c


def cylinder3(Nr, Ntheta, M, n3=1, dz=1.0, n2=None, halo=CMAX3 + 1, **kw):
    """Annulus of the half-spaced polar lattice (App. D) continued along z:
    radii M .. M + Nr in lattice units (uniform radial step 1), Ntheta
    columns around, n3 layers of height dz.  n2 < Ntheta keeps only n2 theta
    columns, continued with the true angular step (a theta reduction, exact
    for theta-invariant states)."""
    n2 = Ntheta if n2 is None else n2
    h = halo
    faces = M + np.arange(Nr + 1, dtype=np.float64)
    cen = 0.5 * (faces[1:] + faces[:-1])
    r = _reflect_rows(cen, Nr, h, faces[0], faces[-1])
    dth = 2.0 * np.pi / Ntheta
    th = (np.arange(-h, n2 + h, dtype=np.float64) + 0.5) * dth
    z = _axis(n3, h, dz)
    R, TH, ZZ = np.meshgrid(r, th, z, indexing="ij")
    meta = dict(family="cylinder3", M=M, Nr=Nr, Ntheta=Ntheta, dtheta=dth, dz=dz, centres=cen, faces=faces)
    meta.update(kw.pop("meta", {}))
    return Case3(n1=Nr, n2=n2, n3=n3, halo=h, X=np.ascontiguousarray(R * np.cos(TH)),
                 Y=np.ascontiguousarray(R * np.sin(TH)), Z=np.ascontiguousarray(ZZ), meta=meta, **kw)


def wall_ut_cylinder(u, R_wall, dtheta, cells_r, ghost_r):
    """Contravariant azimuthal wall velocity U0^2 for a physical wall speed u:
    the azimuthal tangent |g_2| = r sin(dtheta) averaged between the first
    cell and its ghost image (App. D)."""
    return u / (0.5 * (cells_r + ghost_r) * np.sin(dtheta))


def circular_couette3(Nr, Ntheta, M, n3=1, u_inner=0.05, tau=0.8, n2=None, **kw):
    """Circular Couette flow in the cylinder: inner wall rotating at the
    physical speed u_inner, outer wall at rest."""
    c = cylinder3(Nr, Ntheta, M, n3=n3, n2=n2, tau=tau, **kw)
    r0 = c.meta["centres"][0]
    rg = 2.0 * M - r0
    ut = wall_ut_cylinder(u_inner, M, c.meta["dtheta"], r0, rg)
    c = c.replace(bc_lo="moving", bc_hi="noslip", ut_lo=(ut, 0.0))
    c.meta.update(problem="circular_couette", u_inner=u_inner)
    return c


def circular_poiseuille3(Nr, Ntheta, M, n3=1, g2=1e-5, tau=0.8, n2=None, **kw):
    """Circular flow driven by a constant contravariant azimuthal force g2
    (Sec. 3.4), both walls at rest."""
    c = cylinder3(Nr, Ntheta, M, n3=n3, n2=n2, tau=tau, accel=(0.0, g2, 0.0), **kw)
    c.meta.update(problem="circular_poiseuille", g2=g2)
    return c
