"""The paper's closed form for the cosmological I-front (Sec. 4.6) and the
ionized-volume radius it is compared with.

For a uniform medium whose proper density falls as a^-3 and a source of
constant photon rate, the comoving ionized volume V obeys the photon balance
dV/dt = (Ndot - alpha_B n_H^2 V_prop) / n_H (every photon ionizes one atom,
recombinations inside the ionized region use up the rest).  In units of the
initial Stromgren volume and with a = 1 at z_i its solution is the printed
r_I(t) = r_S,i (lambda e^-tau(a) int_1^a e^tau(b) [1 - 2 q0 + 2 q0 (1+z_i)/b]^-1/2 db)^1/3
with lambda = alpha_B n_H,i / H0 / (1 + z_i), tau from the printed F(a).  This
module evaluates that formula by quadrature (test infrastructure: the
numbers are the paper's formula, the integral is scipy's).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import quad


def stromgren_radius(Ndot, alpha_B, n_H):
    """r_S = (3 Ndot / (4 pi alpha_B n_H^2))^(1/3) (proper cm)."""
    return (3.0 * Ndot / (4.0 * math.pi * alpha_B * n_H ** 2)) ** (1.0 / 3.0)


def front_radius(a_rel, lam, q0, z_i):
    """r_I / r_S,i at a_rel = a / a_i >= 1 (the printed solution)."""
    def F(a):
        return (2.0 - 4.0 * q0 - 2.0 * q0 * (1.0 + z_i) / a) * math.sqrt(
            1.0 - 2.0 * q0 + 2.0 * q0 * (1.0 + z_i) / a)

    def tau(a):
        return lam / (6.0 * q0 ** 2 * (1.0 + z_i) ** 2) * (F(a) - F(1.0))

    if a_rel <= 1.0:
        return 0.0
    v, _ = quad(lambda b: math.exp(tau(b)) * (1.0 - 2.0 * q0 + 2.0 * q0 * (1.0 + z_i) / b) ** -0.5,
                1.0, a_rel, limit=200, epsabs=0.0, epsrel=1e-12)
    return (lam * math.exp(-tau(a_rel)) * v) ** (1.0 / 3.0)


def ionized_radius(x_HI, dx, a_i):
    """Radius of the sphere holding the ionized comoving volume sum(1 - x) dx^3,
    expressed in comoving units that equal proper ones at a_i."""
    V = float(np.sum(1.0 - x_HI)) * dx ** 3
    return (3.0 * V / (4.0 * math.pi)) ** (1.0 / 3.0) * a_i
