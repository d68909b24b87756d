"""Pins of the explicit predictor and the time-error estimate (Sec. 3.2.3,
Eqs. 41-43; Sec. 3.2.4, Eq. 44).

- On the constant-coefficient heat problem the predictor's E is the forward
  Euler step of the discrete diffusion equation, computed independently by
  FFT diagonalisation of the periodic 7-point Laplacian (amplitude
  1 - dt D lambda_k / a^2), at a = 1 and a = 0.5.
- On an HII-region state the predictor and the implicit step agree to first
  order, so their difference, measured by the error estimate, falls as dt^2
  (ratio -> 4 when dt halves): a wrong sign, a dropped term or a wrong time
  level in the predictor breaks this.
- The estimate itself: zero for equal states; for one perturbed value the
  max norm is |delta| / w and the p-norms are that over size^(1/p).
"""
import dataclasses
import math

import numpy as np
import pytest

import synth
import oracle
from oracle import newton, timestep
from tests.oracle_cases import gaussian_state, heat_model
from tests.test_oracle_heat_kernel import fft_step


@pytest.mark.parametrize("a", [1.0, 0.5])
def test_predictor_heat_kernel(a):
    n = 16
    model = heat_model(n)
    U = gaussian_state(n)
    h = 1.0 / n
    dt = 0.1 * h * h
    nH = np.ones((n, n, n))
    eh = np.ones((n, n, n))
    Up = timestep.predictor(U, nH, eh, [], [], dt, (a, 0.0, a, 0.0), model)
    ref = fft_step(U[2], dt, 1.0, h, 0.0, a=a)
    assert np.max(np.abs(Up[2] - ref)) / np.max(np.abs(ref)) <= 1e-13
    assert np.array_equal(Up[:2], U[:2])


def hii_state(steps=3):
    w = synth.CFG_SMALL.replace(n=16, dx=synth.CFG_SMALL.dx * 2, mg_levels=3)
    m = dataclasses.replace(oracle.model_from_workload(w), newton_tol=1e-11, pcg_rtol=1e-13)
    s = synth.initial_state(w)
    U, eh = s["U"].copy(), s["eh"].copy()
    cos = (1.0, 0.0, 1.0, 0.0)
    for _ in range(steps):
        U1, st = newton.newton_step(U, U, s["nH"], eh, s["src_cells"], s["src_Q"], w.dt, cos, m)
        assert st["status"] == 0
        eh = eh + U1[0]
        U1[0] = 0.0
        U = U1
    return w, m, s, U, eh


def test_predictor_is_first_order():
    w, m, s, U, eh = hii_state()
    cos = (1.0, 0.0, 1.0, 0.0)
    d = []
    for dt in (2e8, 1e8, 5e7):
        Up = timestep.predictor(U, s["nH"], eh, s["src_cells"], s["src_Q"], dt, cos, m)
        Ui, st = newton.newton_step(U, U, s["nH"], eh, s["src_cells"], s["src_Q"], dt, cos, m)
        assert st["status"] == 0
        d.append(timestep.time_error(Ui, Up, m, 2))
    for r in (d[0] / d[1], d[1] / d[2]):
        assert 3.7 < r < 4.2, d


def test_time_error_norms():
    m = heat_model(4, u_e=2.0, u_E=3.0)
    rng = np.random.default_rng(3)
    U = rng.uniform(0.5, 2.0, size=(3, 4, 4, 4))
    assert timestep.time_error(U, U, m) == 0.0
    assert timestep.time_error(U, U, m, 2) == 0.0
    V = U.copy()
    V[2, 1, 2, 3] += 0.3
    a, b = U[2, 1, 2, 3] / 3.0, V[2, 1, 2, 3] / 3.0
    e_inf = abs(a - b) / (math.sqrt(a * b) + 1.0)
    assert timestep.time_error(V, U, m) == pytest.approx(e_inf, rel=1e-15)
    for p in (1, 2, 3):
        assert timestep.time_error(V, U, m, p) == pytest.approx(e_inf / U.size ** (1.0 / p), rel=1e-14)
    # symmetric in its two arguments
    assert timestep.time_error(U, V, m, 2) == timestep.time_error(V, U, m, 2)


def test_next_dt():
    assert timestep.next_dt(1e10, 0.02, 1e-2, 1e12) == pytest.approx(5e9)
    assert timestep.next_dt(1e10, 0.0, 1e-2, 1e12) == 1e12
    assert timestep.next_dt(1e10, 1e-6, 1e-2, 1e12) == 1e12
