"""Pin 3: single-cell ionization equilibrium.

A uniform medium in which every cell emits the same photon rate has no
gradients, so the diffusion term vanishes and every cell follows the same
local system (Sec. 3.2, Eqs. 22-24 with Eqs. 26-28).
  (a) Steady state, closed form (isothermal, monochromatic, a = 1):
      recombinations = emissions gives 1 - x = sqrt(q / (alpha n^2)), and
      absorption = emission gives E = 4 pi eta / (c sigma n x).
  (b) One backward-Euler step: eliminating E(x) = (E^n + dt 4 pi eta) /
      (1 + dt c sigma n x) leaves one scalar equation in x whose left side is
      strictly increasing, so its root is unique and found by bisection.
  (c) Non-isothermal hydrogen and H+He: a multi-start brute-force root of the
      same single-cell system (scipy.optimize.fsolve) agrees with the oracle.
"""
import math

import numpy as np
import pytest
from scipy import optimize

import synth
import oracle
from oracle import newton
from oracle.model import ALPHA_B_1E4, C_LIGHT, HNU_HI, SIGMA_HI
from oracle.physics import local_operators


def uniform_case(n=4, q=1e-13, nH=1e-3, **kw):
    """Workload with a source in every cell emitting q photons/cm^3/s."""
    w = synth.CFG_SMALL.replace(n=n, mg_levels=1, **kw)
    m = oracle.model_from_workload(w)
    s = synth.initial_state(w)
    s["nH"][:] = nH
    cells = np.arange(n ** 3, dtype=np.int64)
    Q = np.full(n ** 3, q * w.dx ** 3)
    return w, m, s, cells, Q


def test_closed_form_equilibrium():
    # q < alpha n^2 so a partially ionized equilibrium exists
    q, n_H = 1e-20, 1e-3
    w, m, s, cells, Q = uniform_case(q=q, nH=n_H, isothermal=1, newton_tol=1e-1,
                                      pcg_rtol=1e-14, newton_maxit=60)
    ion = math.sqrt(q / (ALPHA_B_1E4 * n_H ** 2))
    x = 1.0 - ion
    E = q * HNU_HI / (C_LIGHT * SIGMA_HI * n_H * x)
    # a step much longer than every rate time scale, from a start within a
    # factor of two of the equilibrium (the tolerance sits at the roundoff
    # floor of terms scaled by dt)
    U0 = s["U"].copy()
    U0[1] = 1.0 - 0.5 * ion
    U0[2] = 2.0 * E
    U, st = newton.newton_step(U0, U0, s["nH"], s["eh"], cells, Q, 1e24,
                               (1.0, 0.0, 1.0, 0.0), m)
    assert st["status"] == 0, st
    assert np.allclose(1.0 - U[1], ion, rtol=1e-6, atol=0)
    assert np.allclose(U[2], E, rtol=1e-6, atol=0)


@pytest.mark.parametrize("dt", [1e11, 1e12, 1e13])
def test_backward_euler_bisection(dt):
    q, n_H = 1e-13, 1e-3
    w, m, s, cells, Q = uniform_case(q=q, nH=n_H, isothermal=1, newton_tol=1e-13,
                                      pcg_rtol=1e-14, newton_maxit=60)
    xn, En = 0.9999, w.E0
    eta4pi = q * HNU_HI
    K = dt * C_LIGHT * SIGMA_HI * n_H

    def F(x):
        E = (En + dt * eta4pi) / (1.0 + K * x)
        return x - xn + dt * (x * C_LIGHT * SIGMA_HI * E / HNU_HI
                              - ALPHA_B_1E4 * n_H * (1.0 - x) ** 2)

    lo, hi = 0.0, 1.0
    assert F(lo) < 0 < F(hi)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if F(mid) > 0:
            hi = mid
        else:
            lo = mid
    x_ref = 0.5 * (lo + hi)
    E_ref = (En + dt * eta4pi) / (1.0 + K * x_ref)
    U, st = newton.newton_step(s["U"], s["U"], s["nH"], s["eh"], cells, Q, dt,
                               (1.0, 0.0, 1.0, 0.0), m)
    assert st["status"] == 0, st
    assert np.max(np.abs(U[1] / x_ref - 1)) <= 1e-12
    assert np.max(np.abs(U[2] / E_ref - 1)) <= 1e-12


@pytest.mark.parametrize("nspecies", [1, 3])
def test_nonisothermal_brute_force(nspecies):
    """Newton on the grid equals a brute-force root of the one-cell system."""
    if nspecies == 1:
        w0 = synth.CFG_SMALL
    else:
        w0 = synth.CFG_HHE.replace(a_start=1.0, a_end=None, nH_mean=1e-3, E0=1e-20,
                                   u_E=1e-20, sigma_ln=0.0, centred=True, dt=1e11)
    q, n_H, dt = 1e-16, 1e-3, 3e12
    w = w0.replace(n=4, mg_levels=1, newton_tol=1e-12, pcg_rtol=1e-14, newton_maxit=60,
                   nsources=1, centred=True)
    m = oracle.model_from_workload(w)
    s = synth.initial_state(w)
    s["nH"][:] = n_H
    n = w.n
    cells = np.arange(n ** 3, dtype=np.int64)
    Q = np.full(n ** 3, q * w.dx ** 3)
    U, st = newton.newton_step(s["U"], s["U"], s["nH"], s["eh"], cells, Q, dt,
                               (1.0, 0.0, 1.0, 0.0), m)
    assert st["status"] == 0, st
    u = m.scales
    Un = s["U"][:, 0, 0, 0]
    g = Un.copy()
    g[-1] += dt * q * m.hnu_mean
    nH1 = np.array([n_H])
    eh1 = np.array([w.eh0])

    def F(v):
        Uc = (v * u)[:, None]
        L = local_operators(Uc, nH1, eh1, 1.0, 0.0, m)[:, 0]
        return (Uc[:, 0] + dt * L - g) / u

    # brute force: random starts over the physical box, keep the roots
    roots = []
    rng = np.random.default_rng(0)
    for _ in range(60):
        start = np.empty(m.nv)
        start[0] = rng.uniform(-0.1, 0.1)
        fr = rng.uniform(0, 1, nspecies)
        if nspecies == 3:
            fr[2] = (1 - fr[1]) * fr[2]
        start[1:1 + nspecies] = fr
        start[-1] = 10 ** rng.uniform(0, 8)
        with np.errstate(all="ignore"):
            sol = optimize.root(F, start, method="hybr", tol=1e-15).x
            res = np.max(np.abs(F(sol)))
        xs = sol[1:1 + nspecies]
        if res < 1e-9 and np.all(xs >= 0) and np.all(xs <= 1) and sol[-1] >= 0:
            roots.append(sol)
    assert len(roots) >= 3
    best = roots[0]
    for r in roots[1:]:
        assert np.allclose(r, best, rtol=1e-9, atol=1e-12)   # one physical root
    got = U[:, 0, 0, 0] / u
    for v in range(m.nv):
        assert abs(got[v] - best[v]) <= 1e-10 * max(abs(best[v]), 1e-3 if v == 0 else 1.0)
    # all cells identical
    assert np.max(np.abs(U - U[:, :1, :1, :1])) <= 1e-12 * np.max(np.abs(U), axis=(1, 2, 3)).max()
