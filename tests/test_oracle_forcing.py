"""The inexact-Newton forcing term (Sec. 3.2.1): the linear solve of Newton
iteration k may stop once ||J(U_k) S_k + f(U_k)|| <= delta_k with
delta_k = forcing * ||f(U_k)||.

The oracle tests this on the Schur residual.  That rests on an identity: the
local rows are solved exactly in step (iii), so the full linear residual
J S + f is zero there and equals minus the Schur residual in the E rows.  It
is pinned here with the dense Newton matrix on 4^3 grids; then a full step
with the paper's delta_k = 1e-6 ||f|| still meets the Newton tolerance.
"""
import numpy as np
import pytest

import synth
import oracle
from oracle import jacobian, mg, newton, residual

from tests.test_oracle_dense_lu import CASES, case


@pytest.mark.parametrize("ns,theta,a,seed", CASES[:2] + CASES[3:])
def test_full_linear_residual_is_the_schur_residual(ns, theta, a, seed):
    m, U, nH, eh, tl, dt, a, H = case(ns, theta, a, seed)
    f = residual.residual(U, tl, nH, eh, dt, a, H, m)
    J = jacobian.dense_jacobian(U, nH, eh, dt, a, H, m)
    sch = jacobian.schur_form(U, f, nH, eh, dt, a, H, m)
    op = jacobian.operator(sch)
    fnorm2 = np.linalg.norm(f)
    for forcing in (1e-2, 1e-4):
        sE, its, _ = mg.fgmres(op, jacobian.preconditioner_operator(sch), sch["b"], m,
                               rtol=0.0, maxit=200, atol=forcing * fnorm2)
        S = jacobian.recover(sE, sch)
        full = J @ S.reshape(-1) + f.reshape(-1)
        schur_r = sch["b"] - jacobian.apply_schur(sE, *op)
        # zero in the local rows, minus the Schur residual in the E rows
        nloc = m.nb * U[0].size
        assert np.max(np.abs(full[:nloc])) <= 1e-9 * fnorm2
        assert np.allclose(full[nloc:], -schur_r.reshape(-1), rtol=1e-8, atol=1e-10 * fnorm2)
        assert np.linalg.norm(full) <= forcing * fnorm2 * (1 + 1e-9)


def test_forcing_step_meets_tolerance_with_fewer_cg_iterations():
    # first step of the 256^3-spacing centred-source problem on a 32^3 box
    w = synth.CFG_256.replace(n=32, mg_levels=3)
    s = synth.initial_state(w)
    args = (s["U"], s["U"], s["nH"], s["eh"], s["src_cells"], s["src_Q"], w.dt, w.cosmology(0))
    U0, st0 = newton.newton_step(*args, oracle.model_from_workload(w))
    U1, st1 = newton.newton_step(*args, oracle.model_from_workload(w.replace(pcg_forcing=1e-6)))
    assert st0["status"] == 0 and st1["status"] == 0
    assert st1["fnorms"][-1] < w.newton_tol
    assert sum(st1["cg_its"]) < sum(st0["cg_its"])
    # both are converged solutions of the same step: they agree to the level
    # the Newton tolerance leaves
    for v in range(U0.shape[0]):
        err = np.linalg.norm(U1[v] - U0[v]) / np.linalg.norm(U0[v])
        assert err < 1e-5, (v, err)
