"""Shared construction helpers for the oracle pin tests and parity tests.

These build oracle models and seeded inputs for the special cases used to
pin the oracle (constant-coefficient diffusion, isothermal hydrogen, ...).
"""
from __future__ import annotations

import dataclasses

import numpy as np

import synth
from oracle import model as om


def heat_model(n, L=1.0, D0=1.0, theta=1.0, a=1.0, **kw):
    """Pure constant-coefficient diffusion: no opacity, no chemistry coupling."""
    m = om.Model(nspecies=1, n=(n, n, n), dx=L / n, theta=theta, u_e=1.0,
                 u_E=1.0, m=0, y_he=0.0, isothermal=1, T_iso=1e4,
                 K_gamma=np.zeros(3), K_kappa=np.zeros(3), K_heat=np.zeros(3),
                 hnu_mean=om.HNU_HI, limiter_mode=1, D0=D0, newton_tol=1e-12,
                 pcg_rtol=1e-14, pcg_maxit=400, mg_levels=3)
    return dataclasses.replace(m, **kw) if kw else m


def gaussian_state(n, L=1.0, s0=0.1, Eb=1.0, A=1.0):
    x = (np.arange(n) + 0.5) * L / n - 0.5 * L
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    E = Eb + A * np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / (2 * s0 ** 2))
    U = np.zeros((3, n, n, n))
    U[1] = 1.0
    U[2] = E
    return U


def hii_workload(n, box_kpc=13.2, **kw):
    return synth.CFG_SMALL.replace(n=n, dx=box_kpc * synth.KPC_CM / n, **kw)
