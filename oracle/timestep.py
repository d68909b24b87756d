"""Adaptive time-step selection and the explicit predictor (Sec. 3.2.3,
Eqs. 41-43; Sec. 3.2.4, Eq. 44).  Test infrastructure: plain NumPy FP64.

Predictor (Eq. 44): the explicit Euler update of the coupled system from
U^n, with the sign of the tendency read so that it is the forward Euler step
of dU/dt = -[L_e; L_n; D_E + L_E](U) + [0; 0; 4 pi eta] (the paper's printed
"+ dt L" would step backwards in time), the expansion factors and the
limiter at t^n as in the explicit part of the time level.  It is then projected onto the physical
bounds like a line-search trial point, and where the predicted gas energy
e_h + e_c would not be positive e_c keeps its value at t^n (a reading).

Error estimate (Eqs. 41-42), in the normalized unknowns U_v / u_v:
  w = sqrt(|U^{n+1} U^pred|) + 1,  q = (U^{n+1} - U^pred) / w,
  eps = max |q|                              (p = inf)
  eps = (sum |q|^p / (N (N_s + 2)))^(1/p)    (finite p).
Step selection (Eq. 43): dt^{n+1} = tau dt^n / eps, here capped at dt_max
(the paper gives no cap; eps -> 0 would otherwise give an unbounded step).
"""
from __future__ import annotations

import numpy as np

from . import newton, residual


def predictor(Un, nH, eh, src_cells, src_Q, dt, cosmo, model):
    """U^pred of Eq. 44 (projected); cosmo = (a_old, H_old, a_new, H_new)."""
    a_old, H_old = cosmo[0], cosmo[1]
    D = residual.limiter_at(Un, nH, a_old, model)
    U = Un - dt * residual.tendency(Un, nH, eh, a_old, H_old, D, model)
    U[-1] = U[-1] + dt * residual.source_field(Un.shape[1:], src_cells, src_Q, model)
    U = newton.project(U, eh, model)
    U[0] = np.where(eh + U[0] > 0.0, U[0], Un[0])
    return U


def time_error(Unew, Upred, model, p=np.inf):
    """eps_loc of Eq. 42 (p = inf: the max norm, no division by the size)."""
    sc = model.scales.reshape((-1, 1, 1, 1))
    a, b = Unew / sc, Upred / sc
    q = np.abs(a - b) / (np.sqrt(np.abs(a * b)) + 1.0)
    if np.isinf(p):
        return float(np.max(q))
    return float((np.sum(q ** p) / q.size) ** (1.0 / p))


def next_dt(dt, eps, tau, dt_max):
    """Eq. 43 with the cap dt_max."""
    if not eps > 0.0:
        return dt_max
    return min(tau * dt / eps, dt_max)


def adaptive_step(Un, nH, eh, src_cells, src_Q, dt, cosmo, model, p=np.inf):
    """One step with the predictor offered as the Newton guess: the guess is
    whichever of U^n and U^pred has the smaller initial residual norm.
    Returns (U^{n+1}, stats, U^pred, eps)."""
    tl = residual.time_level(Un, nH, eh, src_cells, src_Q, dt, cosmo, model)
    Up = predictor(Un, nH, eh, src_cells, src_Q, dt, cosmo, model)
    a, H = cosmo[2], cosmo[3]
    f0 = residual.rms(residual.residual(Un, tl, nH, eh, dt, a, H, model))
    fp = residual.rms(residual.residual(Up, tl, nH, eh, dt, a, H, model))
    # the predictor is projected like a trial point: only e_h + e_c > 0 is
    # tested (the projection enforces the other bounds)
    use_pred = bool(np.isfinite(fp) and newton.energy_ok(Up, eh) and fp < f0)
    U, st = newton.newton_step(Un, Up if use_pred else Un, nH, eh, src_cells, src_Q, dt, cosmo,
                               model, tl=tl)
    st["used_predictor"] = int(use_pred)
    return U, st, Up, time_error(U, Up, model, p)
