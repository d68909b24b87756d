"""Globalised inexact Newton step for f(U) = 0 (Sec. 3.2).

Given an initial guess U_0, iterate while ||f(U_k)|| >= eps (RMS norm, Eq. 30)
and k < maxit:
  1. solve J(U_k) S_k = -f(U_k) through the Schur complement (Sec. 3.2.1),
     the scalar system by MG-preconditioned CG to ||r|| <= rtol ||b||;
  2. U_{k+1} = U_k + lambda_k S_k with lambda_k in (lambda_min, 1].
The convergence test runs before every iteration, so an initial guess that
already satisfies the tolerance takes zero iterations (Sec. 3.2.4).

Line-search rule (a reading; the paper states only the interval): start at
lambda = 1 and halve while the trial point leaves the physical bounds
(E < 0, any fraction outside [0, 1], x_HeI + x_HeII > 1, e_h + e_c <= 0) or
fails the sufficient-decrease test ||f(U_t)|| <= (1 - 1e-4 lambda) ||f(U_k)||;
below lambda_min = 2^-10 the step fails.

Two linear-solve modes: 'mgpcg' (the algorithm) and 'direct' (a sparse
direct solve of the Schur system: the definition of the Newton correction).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import jacobian, mg, residual

OK, ENOCONV, ELINESEARCH, ENONFINITE = 0, -3, -4, -5
LAMBDA_MIN = 2.0 ** -10
ARMIJO = 1.0e-4
PROJECT = True


def project(U, eh, model):
    """Clip a trial point onto the physical bounds (fractions in [0, 1], E >= 0)."""
    ns = model.nspecies
    V = U.copy()
    V[1:1 + ns] = np.clip(V[1:1 + ns], 0.0, 1.0)
    if ns == 3:
        # keep x_HeI + x_HeII <= 1 by scaling both down
        tot = V[2] + V[3]
        over = tot > 1.0
        V[2] = np.where(over, V[2] / np.where(over, tot, 1.0), V[2])
        V[3] = np.where(over, V[3] / np.where(over, tot, 1.0), V[3])
    V[-1] = np.maximum(V[-1], 0.0)
    return V


def bounds_ok(U, eh, model):
    ns = model.nspecies
    xs = U[1:1 + ns]
    ok = bool(np.all(U[-1] >= 0.0) and np.all(xs >= 0.0) and np.all(xs <= 1.0)
              and np.all(eh + U[0] > 0.0))
    if ns == 3:
        ok = ok and bool(np.all(U[2] + U[3] <= 1.0))
    return ok


def schur_matrix(op):
    """Sparse matrix of the 7-point periodic Schur operator."""
    diag, cx, cy, cz = op
    shape = diag.shape
    N = diag.size
    cell = np.arange(N).reshape(shape)
    rows, cols, vals = [cell.ravel()], [cell.ravel()], [diag.ravel()]
    for d, c in enumerate((cx, cy, cz)):
        nbr = np.roll(cell, -1, axis=d).ravel()
        rows += [cell.ravel(), nbr]
        cols += [nbr, cell.ravel()]
        vals += [-c.ravel(), -c.ravel()]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


def direct_solve(op, b):
    A = schur_matrix(op).tocsc()
    return spla.spsolve(A, b.ravel()).reshape(b.shape)


def newton_step(Un, U0, nH, eh, src_cells, src_Q, dt, cosmo, model,
                linear="mgpcg", tol=None, tl=None):
    """One implicit time step.  Returns (U^{n+1}, stats dict)."""
    tol = model.newton_tol if tol is None else tol
    a, H = cosmo[2], cosmo[3]
    if tl is None:
        tl = residual.time_level(Un, nH, eh, src_cells, src_Q, dt, cosmo, model)
    scales = model.scales.reshape((-1, 1, 1, 1))
    U = U0.copy()
    f = residual.residual(U, tl, nH, eh, dt, a, H, model)
    fn = residual.rms(f)
    st = dict(status=OK, newton_its=0, cg_its=[], lambdas=[], fnorms=[fn])
    if not np.isfinite(fn):
        st["status"] = ENONFINITE
        return U, st
    k = 0
    while fn >= tol and k < model.newton_maxit:
        sch = jacobian.schur_form(U, f, tl["D"], nH, eh, dt, a, H, model)
        op = (sch["diag"], sch["cx"], sch["cy"], sch["cz"])
        if linear == "direct":
            sE, its = direct_solve(op, sch["b"]), 0
        else:
            # inexact Newton (Sec. 3.2.1): with a forcing factor the linear
            # solve may also stop at ||J S + f|| <= forcing ||f(U_k)||; the
            # local rows are solved exactly, so ||J S + f||_2 is the Schur
            # residual norm, and ||f||_2 = sqrt(size) times the RMS norm
            atol = model.pcg_forcing * fn * np.sqrt(f.size)
            centres = [np.unravel_index(int(c), U.shape[1:]) for c in src_cells]
            sE, its, _ = mg.pcg(op, sch["b"], model, atol=atol, centres=centres)
        step = jacobian.recover(sE, sch) * scales
        st["cg_its"].append(its)
        lam = 1.0
        while True:
            Ut = U + lam * step
            if PROJECT:
                Ut = project(Ut, eh, model)
            if bounds_ok(Ut, eh, model):
                ft = residual.residual(Ut, tl, nH, eh, dt, a, H, model)
                ftn = residual.rms(ft)
                if ftn <= (1.0 - ARMIJO * lam) * fn:
                    break
            lam *= 0.5
            if lam < LAMBDA_MIN:
                st["status"] = ELINESEARCH
                st["newton_its"] = k
                return U, st
        U, f, fn = Ut, ft, ftn
        st["lambdas"].append(lam)
        st["fnorms"].append(fn)
        k += 1
    st["newton_its"] = k
    if not np.isfinite(fn):
        st["status"] = ENONFINITE
    elif fn >= tol:
        st["status"] = ENOCONV
    return U, st
