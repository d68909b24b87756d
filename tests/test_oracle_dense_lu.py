"""Pin 4: dense-LU brute force of the full Newton matrix on 4^3 grids.

On random physical states (Sec. 3.2.1, Eqs. 31-35):
  (i)   the assembled Newton matrix equals central finite differences of the
        residual (limiter coefficients held at their time-level values);
  (ii)  the dense solve of J S = -f equals the oracle's Schur + MG-PCG result;
  (iii) the dense Schur complement D - L M^-1 U equals the 7-point arrays;
  (iv)  the Schur matrix is symmetric positive definite;
  (v)   for monochromatic hydrogen the local part of every Schur diagonal is
        at least 1 (S is an M-matrix).
"""
import numpy as np
import pytest

import synth
import oracle
from oracle import jacobian, mg, newton, residual


def case(nspecies, theta, a, seed):
    n = 4
    if nspecies == 1:
        w = synth.CFG_SMALL.replace(n=n, theta=theta, mg_levels=2)
    else:
        w = synth.CFG_HHE.replace(n=n, theta=theta, mg_levels=2)
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


@pytest.mark.parametrize("ns,theta,a,seed", CASES)
def test_dense_brute_force(ns, theta, a, seed):
    m, U, nH, eh, tl, dt, a, H = case(ns, theta, a, seed)
    u = m.scales.reshape(-1, 1, 1, 1)
    f = residual.residual(U, tl, nH, eh, dt, a, H, m)
    J = jacobian.dense_jacobian(U, tl["D"], nH, eh, dt, a, H, m)
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
            h = 1e-2 * max(abs(Us[v].flat[c]), 1.0)
            Jfd[:, v * N + c] = (4.0 * cd(v, c, 0.5 * h) - cd(v, c, h)) / 3.0
    colscale = np.maximum(np.max(np.abs(J), axis=0), 1e-300)
    # central differences: O(h^2) truncation plus roundoff of large residuals
    assert np.max(np.abs(Jfd - J) / colscale) <= 2e-6
    assert np.linalg.norm(Jfd - J) <= 1e-6 * np.linalg.norm(J)

    # (ii) dense solve vs Schur + MG-PCG
    S_dense = np.linalg.solve(J, -f.ravel()).reshape(U.shape)
    sch = jacobian.schur_form(U, f, tl["D"], nH, eh, dt, a, H, m)
    op = (sch["diag"], sch["cx"], sch["cy"], sch["cz"])
    sE, its, rr = mg.pcg(op, sch["b"], m, rtol=1e-14)
    S_schur = jacobian.recover(sE, sch)
    # the Schur route solves the full system (residual at rounding level) ...
    assert np.linalg.norm(J @ S_schur.ravel() + f.ravel()) <= 1e-12 * np.linalg.norm(f)
    # ... and agrees with the dense LU solution up to its conditioning
    for v in range(nv):
        ref = np.max(np.abs(S_dense[v]))
        assert np.max(np.abs(S_schur[v] - S_dense[v])) <= 1e-9 * ref, v

    # (iii) dense Schur complement vs the 7-point arrays
    nb = m.nb
    Mb, Ub = J[:nb * N, :nb * N], J[:nb * N, nb * N:]
    Lb, Db = J[nb * N:, :nb * N], J[nb * N:, nb * N:]
    S = Db - Lb @ np.linalg.solve(Mb, Ub)
    A = newton.schur_matrix(op).toarray()
    assert np.max(np.abs(S - A)) <= 1e-13 * np.max(np.abs(S))

    # (iv) SPD
    assert np.array_equal(A, A.T)
    assert np.min(np.linalg.eigvalsh(A)) > 0

    # (v) monochromatic hydrogen: local part of the diagonal >= 1
    if ns == 1:
        csum = sum(c + np.roll(c, 1, axis=d) for d, c in enumerate(op[1:]))
        assert np.min(op[0] - csum) >= 1.0 - 1e-12
