"""Theta-scheme time level and nonlinear residual (Sec. 3.2, Eqs. 22-30).

  f(U) = U + dt theta [L_e; L_n; D_E + L_E](U) - g^n                (Eq. 29)
  g^n  = U^n + dt (theta - 1) [L_e; L_n; D_E + L_E](U^n)            (Eqs. 22-24)

D_E(U) is the flux-limited diffusion of Eq. 25 with the limiter of Eq. 12
evaluated at the state it acts on: the face coefficients of f(U) come from
E and the opacity (species fractions) of U itself, those of the explicit
part of g^n from U^n.  (Only the Newton matrix approximates anything; the
residual is the paper's.)  A second reading, model.limiter_lag = 1, holds
the face coefficients at their U^n values for the whole step (the diffusion
term is then linear in E within the step); it is not Eq. 29 as printed and
serves where Newton on the printed residual does not converge.

The point-source emissivity 4 pi eta = Q <h nu> / dx^3 in the source cell
(comoving) does not depend on U, so both theta-weighted copies of it are
folded into g^n: g^n_E gains dt * 4 pi eta.  e_c^n = 0 (Sec. 3.1): the caller
passes U^n with a zero energy correction.

The residual is returned in scaled variables f_v / u_v (Sec. 3.2.2, Eqs.
36-40) and its RMS norm is Eq. 30.
"""
from __future__ import annotations

import numpy as np

from . import fld
from .physics import local_operators, opacity


def tendency(U, nH, eh, a, H, Dfaces, model):
    """[L_e; L_n; D_E + L_E_local](U) with diffusion coefficients Dfaces."""
    L = local_operators(U, nH, eh, a, H, model)
    L[-1] = L[-1] + fld.diffusion_operator(
        U[-1], Dfaces, a, model.dx, model.E_dirichlet if model.boundary == 2 else None)
    return L


def limiter_at(U, nH, a, model):
    """Face coefficients D_f of Eq. 12 evaluated at the state U."""
    return fld.face_coefficients(U[-1], opacity(U, nH, a, model), a, model)


def source_field(shape, src_cells, src_Q, model):
    """4 pi eta per cell (erg cm^-3 s^-1, comoving)."""
    eta = np.zeros(int(np.prod(shape)))
    np.add.at(eta, np.asarray(src_cells, dtype=np.int64),
              np.asarray(src_Q) * model.hnu_mean / model.dx ** 3)
    return eta.reshape(shape)


def time_level(Un, nH, eh, src_cells, src_Q, dt, cosmo, model):
    """Time-level data of a step: dict(g=g^n incl. sources), and with
    model.limiter_lag the face coefficients at U^n for the whole step (D).

    cosmo = (a_old, H_old, a_new, H_new): the explicit part uses t^n values.
    """
    a_old, H_old = cosmo[0], cosmo[1]
    g = Un.copy()
    D = None
    if model.theta != 1.0 or model.limiter_lag:
        D = limiter_at(Un, nH, a_old, model)
    if model.theta != 1.0:
        g = g + dt * (model.theta - 1.0) * tendency(Un, nH, eh, a_old, H_old, D, model)
    g[-1] = g[-1] + dt * source_field(Un.shape[1:], src_cells, src_Q, model)
    return dict(g=g, D=D) if model.limiter_lag else dict(g=g)


def residual(U, tl, nH, eh, dt, a, H, model, D=None):
    """Scaled residual f~ (same shape as U); tl from time_level().  D: face
    coefficients to hold fixed instead of the limiter at U (a test device:
    with them the diffusion term is linear in E)."""
    if D is None:
        D = tl["D"] if "D" in tl else limiter_at(U, nH, a, model)
    f = U + dt * model.theta * tendency(U, nH, eh, a, H, D, model) - tl["g"]
    return f / model.scales.reshape((-1, 1, 1, 1))


def rms(v):
    """RMS norm of Eq. 30: sqrt(||v||_2^2 / (N (N_s + 2)))."""
    return float(np.sqrt(np.sum(v * v) / v.size))
