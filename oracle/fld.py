"""Flux-limited diffusion: limiter (Sec. 2.2, Eq. 12) and D_E (Eq. 25).

Face discretization (a reading: the paper does not print one).  For the face
between cell P and Q = P + e_d (periodic):
  E_f     = (E_P + E_Q) / 2
  kappa_f = max((kappa_P + kappa_Q) / 2, 1e-3 / (a dx))      (proper 1/cm)
  R_f     = |E_Q - E_P| / (a dx * max(E_f, tiny))            (Eq. 12's R_i)
  D_f     = c (2 kappa_f + R_f) / (6 kappa_f^2 + 3 kappa_f R_f + R_f^2)
and, in comoving form, (D_E)_P = -(1/(a^2 dx^2)) sum_d [D_{P+}(E_{P+d} - E_P)
- D_{P-}(E_P - E_{P-d})].  kappa_T = kappa (no scattering, Sec. 2.2).

The face "flux" below is F = D_f (E_Q - E_P) (the a^2 dx^2 of the comoving
operator is applied by the caller).  D_f depends on the unknowns through E_P,
E_Q (R_f and E_f) and through the species fractions of both cells (kappa_f);
the Newton matrix of Sec. 3.2 needs its derivatives with respect to both,
which face_derivatives returns in closed form:
  T       = R dD/dR = -c R^2 (4 kappa + R) / P^2,  P = 6 kappa^2 + 3 kappa R + R^2
  dF/dE_Q =  D + T - (E_Q - E_P) T / (2 E_f)
  dF/dE_P = -D - T - (E_Q - E_P) T / (2 E_f)
  dF/dkappa_f = (E_Q - E_P) dD/dkappa,  dD/dkappa = -c (12 kappa^2 + 12 kappa R + R^2) / P^2
(kappa_f is the mean of the two cells' opacities, so each gets half; where
the floor binds the opacity derivative is zero).
"""
from __future__ import annotations

import numpy as np

from .model import C_LIGHT, E_FLOOR, KAPPA_FLOOR_CELLS


def limiter(kappa, R):
    """Diffusion coefficient D(kappa_T, R) of Eq. 12."""
    return C_LIGHT * (2.0 * kappa + R) / (6.0 * kappa * kappa + 3.0 * kappa * R + R * R)


def _face(EP, EQ, kP, kQ, adx, mean_kappa=True):
    """(D, D + T, dF/dE_P, dF/dE_Q, dF/dkappa_P, dF/dkappa_Q) of one face
    family; D + T = dF/d(E_Q - E_P) at fixed E_f and kappa_f."""
    Ef = 0.5 * (EP + EQ)
    dE = EQ - EP
    km = 0.5 * (kP + kQ) if mean_kappa else kQ
    kfl = KAPPA_FLOOR_CELLS / adx
    kf = np.maximum(km, kfl)
    Efl = np.maximum(Ef, E_FLOOR)
    R = np.abs(dE) / (adx * Efl)
    Pd = 6.0 * kf * kf + 3.0 * kf * R + R * R
    D = C_LIGHT * (2.0 * kf + R) / Pd
    T = -C_LIGHT * R * R * (4.0 * kf + R) / (Pd * Pd)
    tail = np.where(Ef > E_FLOOR, dE * T / (2.0 * Efl), 0.0)
    dQ = D + T - tail
    dP = -D - T - tail
    dDdk = -C_LIGHT * (12.0 * kf * kf + 12.0 * kf * R + R * R) / (Pd * Pd)
    dk = np.where(km > kfl, dE * dDdk, 0.0)
    if mean_kappa:
        return D, D + T, dP, dQ, 0.5 * dk, 0.5 * dk
    return D, D + T, dP, dQ, 0.0 * dk, dk


def face_derivatives(E, kappa, a, model):
    """Per +x, +y, +z face of every cell: dict with arrays D, DT (= D + T),
    dEP, dEQ, dkP, dkQ (dF/d of F = D (E_Q - E_P)).  Non-periodic grids: the slot after the
    last cell of each row carries nothing (zero), except, with the x-left
    Dirichlet face (boundary 2), the x slot after the last cell holds the
    ghost face (P the ghost with its fixed value and the first cell's
    opacity, Q the first cell), whose P derivatives are zero."""
    adx = a * model.dx
    out = []
    for d in range(3):
        if model.limiter_mode == 1:
            z = np.zeros(E.shape)
            out.append(dict(D=np.full(E.shape, model.D0), DT=np.full(E.shape, model.D0),
                            dEP=-np.full(E.shape, model.D0),
                            dEQ=np.full(E.shape, model.D0), dkP=z, dkQ=z.copy()))
            continue
        Eq = np.roll(E, -1, axis=d)
        kq = np.roll(kappa, -1, axis=d)
        D, DT, dP, dQ, kP, kQ = _face(E, Eq, kappa, kq, adx)
        out.append(dict(D=D, DT=DT, dEP=dP, dEQ=dQ, dkP=kP, dkQ=kQ))
    if model.boundary in (1, 2):
        for d in range(3):
            idx = [slice(None)] * 3
            idx[d] = -1
            for key in out[d]:
                out[d][key] = out[d][key].copy()
                out[d][key][tuple(idx)] = 0.0
        if model.boundary == 2:
            E0, k0 = E[0], kappa[0]
            if model.limiter_mode == 1:
                out[0]["D"][-1] = model.D0
                out[0]["DT"][-1] = model.D0
                out[0]["dEQ"][-1] = model.D0
            else:
                Eb = np.full(E0.shape, model.E_dirichlet)
                D, DT, dP, dQ, kP, kQ = _face(Eb, E0, k0, k0, adx, mean_kappa=False)
                out[0]["D"][-1] = D
                out[0]["DT"][-1] = DT
                out[0]["dEQ"][-1] = dQ
                out[0]["dkQ"][-1] = kQ
    return out


def face_coefficients(E, kappa, a, model):
    """D on the +x, +y, +z faces of every cell (list of 3 arrays); the same
    slot conventions as face_derivatives."""
    return [fd["D"] for fd in face_derivatives(E, kappa, a, model)]


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
