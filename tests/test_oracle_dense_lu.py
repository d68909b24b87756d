"""Pin 4: dense-LU brute force of the full Newton matrix on 4^3 grids.

On random physical states (Sec. 3.2.1, Eqs. 31-35):
  (i)   the assembled Newton matrix equals central finite differences of the
        residual of Eq. 29, whose flux limiter (Eq. 12) is evaluated at the
        perturbed state itself: every column, including the E-E couplings
        through R_f and E_f and the E-row couplings to the neighbours'
        species fractions through the face opacity;
  (ii)  the dense solve of J S = -f equals the oracle's Schur + MG-FGMRES
        result;
  (iii) the dense Schur complement D - L M^-1 U equals the 7-point arrays;
  (iv)  the diffusion part is conservative: every column of S sums to the
        cell's local part 1 + dt theta dL_E/dE - L M^-1 U, which is at least
        1 for monochromatic hydrogen; the preconditioner's operator is that
        local part plus a symmetric diffusion with non-negative face
        couplings, its diagonal raised to S's own where that is larger: a
        symmetric positive definite, diagonally dominant M-matrix.
The lagged reading (face coefficients held at U^n) is checked the same way
with those coefficients fixed in the differences.
"""
import numpy as np
import pytest

import synth
import oracle
from oracle import jacobian, mg, newton, residual


def case(nspecies, theta, a, seed, lag=0):
    n = 4
    if nspecies == 1:
        w = synth.CFG_SMALL.replace(n=n, theta=theta, mg_levels=2, limiter_lag=lag)
    else:
        w = synth.CFG_HHE.replace(n=n, theta=theta, mg_levels=2, limiter_lag=lag)
    m = oracle.model_from_workload(w, pcg_rtol=1e-14, pcg_maxit=500)
    rng = np.random.default_rng(seed)
    U, nH, eh = synth.random_physical_state(n, nspecies, rng, nH_mean=1e-3 * a ** 3)
    U[-1] *= a ** 3
    Un, _, _ = synth.random_physical_state(n, nspecies, rng, nH_mean=1e-3 * a ** 3)
    Un[-1] *= a ** 3
    Un[0] = 0.0
    m.u_E = 1e-20 * a ** 3
    H = 0.0 if a == 1.0 else synth.eds_hubble(a)
    cosmo = (a, H, a, H)
    cells = rng.choice(n ** 3, 3, replace=False)
    Q = 10 ** rng.uniform(47, 49, 3)
    dt = 1e11 if a == 1.0 else 5e12
    tl = residual.time_level(Un, nH, eh, cells, Q, dt, cosmo, m)
    return m, U, nH, eh, tl, dt, a, H


CASES = [(1, 1.0, 1.0, 1), (1, 0.51, 1.0, 2), (1, 1.0, 0.1, 3), (3, 1.0, 1.0, 4),
         (3, 0.51, 0.1, 5)]


@pytest.mark.parametrize("ns,theta,a,seed,lag", [c + (0,) for c in CASES] + [CASES[3] + (1,)])
def test_dense_brute_force(ns, theta, a, seed, lag):
    """lag = 1: the lagged reading (face coefficients at U^n), whose Newton
    matrix is the derivative with those coefficients fixed."""
    m, U, nH, eh, tl, dt, a, H = case(ns, theta, a, seed, lag)
    u = m.scales.reshape(-1, 1, 1, 1)
    f = residual.residual(U, tl, nH, eh, dt, a, H, m)
    J = jacobian.dense_jacobian(U, nH, eh, dt, a, H, m, tl.get("D"))
    nv, N = m.nv, U[0].size

    # (i) Richardson-extrapolated central differences, column by column
    def cd(v, c, h):
        Up, Um = Us.copy(), Us.copy()
        Up[v].flat[c] += h
        Um[v].flat[c] -= h
        fp = residual.residual(Up * u, tl, nH, eh, dt, a, H, m)
        fm = residual.residual(Um * u, tl, nH, eh, dt, a, H, m)
        return ((fp - fm) / (2 * h)).ravel()

    Jfd = np.zeros_like(J)
    Us = U / u
    for v in range(nv):
        for c in range(N):
            # relative steps: the fractions enter the face opacities, whose
            # floor must not be crossed by the perturbation
            h = 1e-2 * max(abs(Us[v].flat[c]), 1e-8)
            Jfd[:, v * N + c] = (4.0 * cd(v, c, 0.5 * h) - cd(v, c, h)) / 3.0
    assert np.linalg.norm(Jfd - J) <= 1e-9 * np.linalg.norm(J)
    # block by block (row variable, column variable; entries of the cell
    # itself and of its neighbours apart), so that a small block such as the
    # E rows' coupling to the neighbours' fractions is checked on its own
    # scale: extrapolated central differences leave ~1e-6 of roundoff
    eye = np.eye(N, dtype=bool)
    for r in range(nv):
        for c in range(nv):
            for mask in (eye, ~eye):
                Bj = J[r * N:(r + 1) * N, c * N:(c + 1) * N][mask]
                Bf = Jfd[r * N:(r + 1) * N, c * N:(c + 1) * N][mask]
                ref = np.linalg.norm(Bj)
                if ref == 0.0:
                    ref = np.linalg.norm(J[r * N:(r + 1) * N])
                assert np.linalg.norm(Bf - Bj) <= 2e-5 * ref, (r, c)

    # (ii) dense solve vs Schur + MG-FGMRES
    S_dense = np.linalg.solve(J, -f.ravel()).reshape(U.shape)
    sch = jacobian.schur_form(U, f, nH, eh, dt, a, H, m, tl.get("D"))
    op = jacobian.operator(sch)
    sE = newton.direct_solve(op, sch["b"])
    S_schur = jacobian.recover(sE, sch)
    # the Schur route (7-point system solved directly) solves the full system
    # (residual at rounding level) ...
    assert np.linalg.norm(J @ S_schur.ravel() + f.ravel()) <= 1e-12 * np.linalg.norm(f)
    # ... and agrees with the dense LU solution up to its conditioning
    for v in range(nv):
        ref = np.max(np.abs(S_dense[v]))
        assert np.max(np.abs(S_schur[v] - S_dense[v])) <= 1e-9 * ref, v
    # MG-preconditioned FGMRES reaches the direct Schur solution.  Not
    # asserted for the a = 0.1 hydrogen case: its random E (seven decades
    # from cell to cell) at dt = 5e12 s puts hundreds of light-crossings per
    # cell into the limiter's E_f derivative and the opacity terms, which
    # leave S far from any symmetric preconditioner (diagonal entries down to
    # -5e4); a physical state is smooth
    if a == 1.0 or ns == 3:
        sK, its, rr = mg.fgmres(op, jacobian.preconditioner_operator(sch), sch["b"], m,
                                rtol=1e-12)
        assert rr <= 1e-12 and its < 60
        assert np.linalg.norm(sK - sE) <= 1e-8 * np.linalg.norm(sE)

    # (iii) dense Schur complement vs the 7-point arrays
    nb = m.nb
    Mb, Ub = J[:nb * N, :nb * N], J[:nb * N, nb * N:]
    Lb, Db = J[nb * N:, :nb * N], J[nb * N:, nb * N:]
    S = Db - Lb @ np.linalg.solve(Mb, Ub)
    A = newton.schur_matrix(op).toarray()
    assert np.max(np.abs(S - A)) <= 1e-13 * np.max(np.abs(S))

    # (iv) column sums = local part; the preconditioner's operator is the
    # local part plus a symmetric diffusion, its diagonal raised to S's where
    # that is larger: an SPD M-matrix, diagonally dominant
    M_, Ucol, Lrow, dloc = jacobian.local_blocks(U, nH, eh, dt, a, H, m)
    local = dloc - np.sum(Lrow * sch["W"], axis=0)
    assert np.max(np.abs(A.sum(axis=0) - local.ravel())) <= 1e-12 * np.max(np.abs(A))
    if ns == 1:
        assert np.min(local) >= 1.0 - 1e-12
    Pm = newton.schur_matrix(jacobian.preconditioner_operator(sch)).toarray()
    assert np.array_equal(Pm, Pm.T)
    off = Pm - np.diag(np.diag(Pm))
    assert np.all(off <= 0.0)
    sums = Pm.sum(axis=0)
    tol = 1e-12 * np.max(np.abs(Pm))
    assert np.all(sums >= local.ravel() - tol)
    raised = np.diag(Pm) - (local.ravel() - off.sum(axis=0))
    assert np.all(raised >= -tol)
    # where the diagonal is raised it is S's own
    up = raised > tol
    assert np.allclose(np.diag(Pm)[up], np.diag(A)[up], rtol=0, atol=tol)
    assert np.min(np.linalg.eigvalsh(Pm)) > 0
