"""Closed-form exact solutions of Sec. 3 (test infrastructure only).

All lengths in lattice units (mean wall-normal step = 1), so the paper's
lattice-unit forms follow from the continuous ones with R1 = M, R2 = M + N_r
and l = N_x.  Each function cites the equation it writes out.
"""
from __future__ import annotations

import math

import numpy as np


def planar_couette(X, l, u_lo=0.0, u_hi=0.0):
    """Sec. 3.1, Eq. (PlaneCouetteExactSolution): linear profile between a wall
    at X = 0 moving with u_lo and one at X = l moving with u_hi.  The paper's
    case is u_lo = -U0, u_hi = 0: u_y = U0 (X/l - 1)."""
    X = np.asarray(X, dtype=np.float64)
    return u_lo + (u_hi - u_lo) * X / l


def planar_poiseuille(X, l, g, nu):
    """Sec. 3.2, Eq. (PlanePoiseuilleSolution2) with G = g/nu for an
    acceleration -g: u_y = (G/2) X (X - l).  Written here for an acceleration
    +g along the channel: u = g X (l - X) / (2 nu)."""
    X = np.asarray(X, dtype=np.float64)
    G = -g / nu
    return 0.5 * G * X * (X - l)


def circular_couette_ab(R1, R2, Om1, Om2):
    """Eq. (CircularCouetteSolution2)."""
    a = (Om2 * R2 ** 2 - Om1 * R1 ** 2) / (R2 ** 2 - R1 ** 2)
    b = R1 ** 2 * R2 ** 2 * (Om1 - Om2) / (R2 ** 2 - R1 ** 2)
    return a, b


def circular_couette(r, R1, R2, Om1, Om2=0.0):
    """Eq. (CircularCouetteSolution1): u_theta = a r + b / r."""
    a, b = circular_couette_ab(R1, R2, Om1, Om2)
    r = np.asarray(r, dtype=np.float64)
    return a * r + b / r


def circular_couette_density(r, R1, R2, Om1, Om2, T0, rho0=1.0):
    """Eqs. (CircularCouetteSolution3, 4): leading order in Ma,
    rho = rho0 {1 + [h(r) - 2 H / (R2^2 - R1^2)] / T0} with
    h = -b^2/(2 r^2) + 2 a b log(r/R1) + a^2 r^2 / 2."""
    a, b = circular_couette_ab(R1, R2, Om1, Om2)
    r = np.asarray(r, dtype=np.float64)
    h = -b ** 2 / (2 * r ** 2) + 2 * a * b * np.log(r / R1) + a ** 2 * r ** 2 / 2
    L = math.log(R2 / R1)
    H = -b ** 2 / 2 * L + a * b * (R2 ** 2 * L - (R2 ** 2 - R1 ** 2) / 2) + a ** 2 / 8 * (R2 ** 4 - R1 ** 4)
    return rho0 * (1.0 + (h - 2 * H / (R2 ** 2 - R1 ** 2)) / T0)


def circular_poiseuille_coeffs(R1, R2, A):
    """Sec. 3.4: a = -(A/8)(R1^2 + R2^2), b = (A/8) R1^2 R2^2."""
    return -A / 8 * (R1 ** 2 + R2 ** 2), A / 8 * R1 ** 2 * R2 ** 2


def circular_poiseuille(r, R1, R2, K, nu):
    """Eq. (CircularPoiseuilleSolution1): u_theta = a r + b / r + (A/8) r^3.

    The paper's driving acceleration is -alpha r g (clockwise for alpha g > 0)
    with A = alpha g / nu; here the acceleration is written +K r
    (counter-clockwise for K > 0), i.e. A = -K / nu."""
    A = -K / nu
    a, b = circular_poiseuille_coeffs(R1, R2, A)
    r = np.asarray(r, dtype=np.float64)
    return a * r + b / r + A / 8 * r ** 3


def circular_poiseuille_mean(R1, R2, K, nu):
    """Sec. 3.4: mean velocity over [R1, R2]."""
    A = -K / nu
    a, b = circular_poiseuille_coeffs(R1, R2, A)
    return a / 2 * (R2 + R1) + b * math.log(R2 / R1) / (R2 - R1) + A / 32 * (R2 + R1) * (R2 ** 2 + R1 ** 2)


def circular_poiseuille_density(r, R1, R2, K, nu, T0, rho0=1.0):
    """Sec. 3.4 leading-order density with h(r), H(R1, R2) of the force-driven case."""
    A = -K / nu
    a, b = circular_poiseuille_coeffs(R1, R2, A)
    r = np.asarray(r, dtype=np.float64)
    h = (-b ** 2 / (2 * r ** 2) + 2 * a * b * np.log(r / R1) + 0.5 * (a ** 2 + b * A / 4) * r ** 2
         + a * A * r ** 4 / 16 + A ** 2 * r ** 6 / 384)
    L = math.log(R2 / R1)
    H = (-b ** 2 / 2 * L + a * b * (R2 ** 2 * L - (R2 ** 2 - R1 ** 2) / 2)
         + (a ** 2 + b * A / 4) / 8 * (R2 ** 4 - R1 ** 4) + a * A / 96 * (R2 ** 6 - R1 ** 6)
         + A ** 2 / 3072 * (R2 ** 8 - R1 ** 8))
    return rho0 * (1.0 + (h - 2 * H / (R2 ** 2 - R1 ** 2)) / T0)


# ---------------------------------------------------------------------------
# the paper's parameter relations (Tables of Sec. 3)
# ---------------------------------------------------------------------------
def nu_lat(T0, tau):
    return T0 * (tau - 0.5)


def mach(U, T0):
    return U / math.sqrt(T0)


def reynolds(U, N, nu):
    return U * N / nu


def planar_poiseuille_g(U, N, nu):
    """Acceleration whose parabola has mean velocity U... the tables quote
    g = 12 nu U / N^2 (mean of a X(l-X)/(2 nu) over [0, l] equals g l^2/(12 nu))."""
    return 12.0 * nu * U / N ** 2
