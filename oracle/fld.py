"""Flux-limited diffusion: limiter (Sec. 2.2, Eq. 12) and D_E (Eq. 25).

Face discretization (a reading: the paper does not print one).  For the face
between cell P and Q = P + e_d (periodic):
  E_f     = (E_P + E_Q) / 2
  kappa_f = max((kappa_P + kappa_Q) / 2, 1e-6 / (a dx))      (proper 1/cm)
  R_f     = |E_Q - E_P| / (a dx * max(E_f, tiny))            (Eq. 12's R_i)
  D_f     = c (2 kappa_f + R_f) / (6 kappa_f^2 + 3 kappa_f R_f + R_f^2)
and, in comoving form, (D_E)_P = -(1/(a^2 dx^2)) sum_d [D_{P+}(E_{P+d} - E_P)
- D_{P-}(E_P - E_{P-d})].  kappa_T = kappa (no scattering, Sec. 2.2).
"""
from __future__ import annotations

import numpy as np

from .model import C_LIGHT, E_FLOOR, KAPPA_FLOOR_CELLS


def limiter(kappa, R):
    """Diffusion coefficient D(kappa_T, R) of Eq. 12."""
    return C_LIGHT * (2.0 * kappa + R) / (6.0 * kappa * kappa + 3.0 * kappa * R + R * R)


def face_coefficients(E, kappa, a, model):
    """D on the +x, +y, +z faces of every cell (list of 3 arrays)."""
    out = []
    for d in range(3):
        if model.limiter_mode == 1:
            out.append(np.full(E.shape, model.D0))
            continue
        Eq = np.roll(E, -1, axis=d)
        kq = np.roll(kappa, -1, axis=d)
        Ef = 0.5 * (E + Eq)
        kf = np.maximum(0.5 * (kappa + kq), KAPPA_FLOOR_CELLS / (a * model.dx))
        R = np.abs(Eq - E) / (a * model.dx * np.maximum(Ef, E_FLOOR))
        out.append(limiter(kf, R))
    if model.boundary in (1, 2):
        # non-periodic: the face after the last cell of each row joins the
        # domain's two ends and carries no flux; with the x-left Dirichlet
        # face (boundary 2) that x slot holds the face between the ghost cell
        # (E_dirichlet, the first cell's opacity) and the first cell
        for d in range(3):
            idx = [slice(None)] * 3
            idx[d] = -1
            out[d] = out[d].copy()
            out[d][tuple(idx)] = 0.0
        if model.boundary == 2:
            E0, k0 = E[0], kappa[0]
            if model.limiter_mode == 1:
                out[0][-1] = model.D0
            else:
                Ef = 0.5 * (model.E_dirichlet + E0)
                kf = np.maximum(k0, KAPPA_FLOOR_CELLS / (a * model.dx))
                R = np.abs(E0 - model.E_dirichlet) / (a * model.dx * np.maximum(Ef, E_FLOOR))
                out[0][-1] = limiter(kf, R)
    return out


def diffusion_operator(E, Dfaces, a, dx, E_dirichlet=None):
    """D_E = -div(D grad E) in comoving form with the face coefficients Dfaces.
    E_dirichlet (x-left Dirichlet face): the x slot after the last cell then
    holds the ghost face of the first cell, whose neighbour value is fixed."""
    acc = np.zeros_like(E)
    for d in range(3):
        Dd = Dfaces[d]
        if d == 0 and E_dirichlet is not None:
            Dd = Dd.copy()
            Db = Dd[-1].copy()
            Dd[-1] = 0.0
            acc[0] += Db * (E_dirichlet - E[0])
        flux_plus = Dd * (np.roll(E, -1, axis=d) - E)          # on the + face
        flux_minus = np.roll(flux_plus, 1, axis=d)             # the - face
        acc += flux_plus - flux_minus
    return -acc / (a * a * dx * dx)
