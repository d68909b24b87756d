"""Pin of the reflecting walls (boundary = 1: no diffusive flux through the
six domain faces).

Mirror equivalence: an n^3 box with reflecting walls, a source in the corner
cell (0, 0, 0) and a medium rho(i, j, k) equals the restriction to [0, n)^3
of the periodic (2n)^3 box holding the medium mirrored across the planes
i = n - 1/2 (and j, k) and the 8 mirror images of the source, cells
{0, 2n - 1}^3: that problem is symmetric under i -> 2n - 1 - i, so no flux
crosses the mirror planes, which are exactly the walls.  Two implicit steps
agree to the solver tolerances.  A closed reflecting box also conserves
photons plus ions up to emission and recombination, like the periodic one.
"""
import dataclasses

import numpy as np
import pytest

import synth
import oracle
from oracle import newton as onewt


def mirrored(a):
    b = np.concatenate([a, a[::-1]], axis=0)
    b = np.concatenate([b, b[:, ::-1]], axis=1)
    return np.concatenate([b, b[:, :, ::-1]], axis=2)


def run(w, state, steps, **over):
    m = dataclasses.replace(oracle.model_from_workload(w), newton_tol=1e-11, pcg_rtol=1e-13,
                            **over)
    U, eh = state["U"].copy(), state["eh"].copy()
    for k in range(steps):
        U1, st = onewt.newton_step(U, U, state["nH"], eh, state["src_cells"], state["src_Q"],
                                   w.dt, w.cosmology(k), m)
        assert st["status"] == 0, st
        eh = eh + U1[0]
        U1[0] = 0.0
        U = U1
    return U, eh


@pytest.mark.parametrize("sigma", [0.0, 0.5])
def test_mirror_equivalence(sigma):
    n = 8
    base = synth.CFG_SMALL.replace(n=n, dx=synth.CFG_SMALL.dx * 4, mg_levels=2, sigma_ln=sigma,
                                   seed=7)
    wr = base.replace(boundary=1, corner_source=True)
    sr = synth.initial_state(wr)
    wp = base.replace(n=2 * n, mg_levels=3)
    sp = synth.initial_state(wp)
    sp["nH"] = mirrored(sr["nH"])
    sp["eh"] = mirrored(sr["eh"])
    sp["U"] = np.stack([mirrored(v) for v in sr["U"]])
    m2 = 2 * n
    cells = [((i * m2) + j) * m2 + k for i in (0, m2 - 1) for j in (0, m2 - 1) for k in (0, m2 - 1)]
    sp["src_cells"] = np.array(cells, dtype=np.int64)
    sp["src_Q"] = np.full(8, wr.Q)
    Ur, _ = run(wr, sr, 2)
    Up, _ = run(wp, sp, 2)
    Up = Up[:, :n, :n, :n]
    for v in range(Ur.shape[0]):
        s = max(float(np.max(np.abs(Up[v]))), 1e-300)
        assert np.max(np.abs(Ur[v] - Up[v])) / s <= 1e-8, v
    # and the walls matter: in the periodic n^3 box the cell across the wall
    # from the source is its neighbour and holds far more radiation
    Uq, _ = run(wr, sr, 2, boundary=0)
    assert Uq[-1][n - 1, 0, 0] > 10.0 * Ur[-1][n - 1, 0, 0]


def test_closed_box_photon_balance():
    from oracle import residual as ores
    from oracle.model import HNU_HI
    from oracle.physics import recombination_coefficients, temperature
    w = synth.CFG_SMALL.replace(n=8, dx=synth.CFG_SMALL.dx * 4, mg_levels=2, boundary=1,
                                corner_source=True)
    s = synth.initial_state(w)
    m = dataclasses.replace(oracle.model_from_workload(w), newton_tol=1e-11, pcg_rtol=1e-13)
    Un, eh, nH = s["U"], s["eh"], s["nH"]
    U, st = onewt.newton_step(Un, Un, nH, eh, s["src_cells"], s["src_Q"], w.dt, w.cosmology(0), m)
    assert st["status"] == 0
    h3 = w.dx ** 3

    def count(V):
        return (np.sum(V[2]) / HNU_HI + np.sum(nH * (1 - V[1]))) * h3

    T = temperature(eh + U[0], U[1], 0.0, 0.0, m)
    recomb = np.sum(recombination_coefficients(T)[0] * (nH * (1 - U[1])) ** 2) * h3
    lhs = count(U) - count(Un)
    rhs = w.dt * (w.Q - recomb)
    assert abs(lhs - rhs) <= 1e-8 * w.dt * w.Q
