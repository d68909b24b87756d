"""Globalised inexact Newton step for f(U) = 0 (Sec. 3.2).

Given an initial guess U_0, iterate while ||f(U_k)|| >= eps (RMS norm, Eq. 30)
and k < maxit:
  1. solve J(U_k) S_k = -f(U_k) through the Schur complement (Sec. 3.2.1),
     the scalar system by MG-preconditioned CG to ||r|| <= rtol ||b||;
  2. U_{k+1} = U_k + lambda_k S_k with lambda_k in (lambda_min, 1].
The convergence test runs before every iteration, so an initial guess that
already satisfies the tolerance takes zero iterations (Sec. 3.2.4).

Line-search rule (a reading; the paper states only the interval): start at
lambda = 1; the trial point is projected onto the physical bounds (fractions
into [0, 1], the helium pair rescaled to a sum <= 1, E >= 0) and accepted
when e_h + e_c > 0 (the one bound the projection does not enforce) and the
sufficient-decrease test ||f(U_t)|| <= (1 - 1e-4 lambda) ||f(U_k)|| holds,
else lambda is halved; below lambda_min = 2^-10 the step fails.  (The
rescaled helium pair sums to 1 only to within a rounding, so the projected
bounds are not re-tested.)

Two linear-solve modes: 'mgpcg' (the algorithm: MG-preconditioned FGMRES on
the Schur system, or flexible PCG for a symmetric one) and 'direct' (a sparse
direct solve of the Schur system: the definition of the Newton correction).

Replay mode (replay=dict(its=[...], lambdas=[...])) executes a recorded
schedule instead of taking the decisions: Newton iteration k runs exactly
its[k] Krylov iterations and steps with lambda = lambdas[k], and the step
takes len(its) Newton iterations.  A run of another implementation, whose
stop tests may fall within rounding of their thresholds, can so be compared
iterate for iterate.
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


def energy_ok(U, eh):
    """The bound a projected state is tested on: e_h + e_c > 0 everywhere."""
    return bool(np.all(eh + U[0] > 0.0))


def bounds_ok(U, eh, model):
    ns = model.nspecies
    xs = U[1:1 + ns]
    ok = bool(np.all(U[-1] >= 0.0) and np.all(xs >= 0.0) and np.all(xs <= 1.0)
              and np.all(eh + U[0] > 0.0))
    if ns == 3:
        ok = ok and bool(np.all(U[2] + U[3] <= 1.0))
    return ok


def schur_matrix(op):
    """Sparse matrix of the 7-point periodic operator (diag, fx, fy, fz
    [, bx, by, bz]): row P couples to P + e_d with -f_d[P] and row P + e_d to
    P with -b_d[P] (b omitted: b = f, symmetric)."""
    diag, fs = op[0], op[1:4]
    bs = op[4:7] if len(op) == 7 else fs
    shape = diag.shape
    N = diag.size
    cell = np.arange(N).reshape(shape)
    rows, cols, vals = [cell.ravel()], [cell.ravel()], [diag.ravel()]
    for d, (fw, bw) in enumerate(zip(fs, bs)):
        nbr = np.roll(cell, -1, axis=d).ravel()
        rows += [cell.ravel(), nbr]
        cols += [nbr, cell.ravel()]
        vals += [-fw.ravel(), -bw.ravel()]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


def direct_solve(op, b):
    A = schur_matrix(op).tocsc()
    return spla.spsolve(A, b.ravel()).reshape(b.shape)


def newton_step(Un, U0, nH, eh, src_cells, src_Q, dt, cosmo, model,
                linear="mgpcg", tol=None, tl=None, replay=None, D=None):
    """One implicit time step.  Returns (U^{n+1}, stats dict).  D: face
    coefficients held fixed (a test device, see residual.residual)."""
    tol = model.newton_tol if tol is None else tol
    a, H = cosmo[2], cosmo[3]
    if tl is None:
        tl = residual.time_level(Un, nH, eh, src_cells, src_Q, dt, cosmo, model)
    if D is None and "D" in tl:
        D = tl["D"]          # the lagged-limiter reading
    scales = model.scales.reshape((-1, 1, 1, 1))
    U = U0.copy()
    f = residual.residual(U, tl, nH, eh, dt, a, H, model, D)
    fn = residual.rms(f)
    st = dict(status=OK, newton_its=0, cg_its=[], lambdas=[], fnorms=[fn])
    if not np.isfinite(fn):
        st["status"] = ENONFINITE
        return U, st
    k = 0
    nits = model.newton_maxit if replay is None else len(replay["its"])
    while (fn >= tol or replay is not None) and k < nits:
        sch = jacobian.schur_form(U, f, nH, eh, dt, a, H, model, D)
        op = jacobian.operator(sch)
        pop = jacobian.preconditioner_operator(sch)
        centres = [np.unravel_index(int(c), U.shape[1:]) for c in src_cells]
        if linear == "direct":
            sE, its = direct_solve(op, sch["b"]), 0
        elif replay is not None:
            sE, its, _ = mg.krylov(op, pop, sch["b"], model, rtol=0.0,
                                   maxit=int(replay["its"][k]), centres=centres)
        else:
            # inexact Newton (Sec. 3.2.1): with a forcing factor the linear
            # solve may also stop at ||J S + f|| <= forcing ||f(U_k)||; the
            # local rows are solved exactly, so ||J S + f||_2 is the Schur
            # residual norm, and ||f||_2 = sqrt(size) times the RMS norm
            atol = model.pcg_forcing * fn * np.sqrt(f.size)
            sE, its, _ = mg.krylov(op, pop, sch["b"], model, atol=atol, centres=centres)
        step = jacobian.recover(sE, sch) * scales
        st["cg_its"].append(its)
        if replay is not None:
            lam = float(replay["lambdas"][k])
            Ut = U + lam * step
            if PROJECT:
                Ut = project(Ut, eh, model)
            ft = residual.residual(Ut, tl, nH, eh, dt, a, H, model, D)
            U, f, fn = Ut, ft, residual.rms(ft)
            st["lambdas"].append(lam)
            st["fnorms"].append(fn)
            k += 1
            continue
        lam = 1.0
        while True:
            Ut = U + lam * step
            if PROJECT:
                Ut = project(Ut, eh, model)
            if energy_ok(Ut, eh) if PROJECT else bounds_ok(Ut, eh, model):
                ft = residual.residual(Ut, tl, nH, eh, dt, a, H, model, D)
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
