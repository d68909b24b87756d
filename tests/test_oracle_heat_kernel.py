"""Pin 1: constant-coefficient Gaussian-pulse heat kernel.

With the limiter replaced by a constant D0 and no opacity, the E equation of
Eq. 21 reduces to dE/dt = (D0/a^2) lap E.  (i) One theta-step of the oracle's
full Newton / Schur / MG-PCG chain must equal the exact solution of the
discrete system, computed independently by FFT diagonalisation of the
periodic 7-point Laplacian.  (ii) Repeated steps converge to the continuum
Gaussian heat kernel at second order.
"""
import numpy as np
import pytest

from oracle import newton
from tests.oracle_cases import gaussian_state, heat_model


def fft_step(E, dt, D0, h, theta, a=1.0):
    n = E.shape[0]
    m = np.arange(n)
    s2 = np.sin(np.pi * m / n) ** 2
    lam = 4.0 / (h * h * a * a) * (s2[:, None, None] + s2[None, :, None] + s2[None, None, :])
    amp = (1.0 - (1.0 - theta) * dt * D0 * lam) / (1.0 + theta * dt * D0 * lam)
    return np.real(np.fft.ifftn(np.fft.fftn(E) * amp))


def step(U, model, dt, a=1.0):
    n = U.shape[1]
    nH = np.ones((n, n, n))
    eh = np.ones((n, n, n))
    cosmo = (a, 0.0, a, 0.0)
    U1, st = newton.newton_step(U, U, nH, eh, [], [], dt, cosmo, model)
    assert st["status"] == 0, st
    return U1, st


@pytest.mark.parametrize("theta", [1.0, 0.5, 0.51])
@pytest.mark.parametrize("n", [16, 32])
def test_exact_discrete_step(n, theta):
    model = heat_model(n, theta=theta)
    U = gaussian_state(n)
    h = 1.0 / n
    dt = 2.0 * h * h
    U1, st = step(U, model, dt)
    ref = fft_step(U[2], dt, 1.0, h, theta)
    err = np.max(np.abs(U1[2] - ref)) / np.max(np.abs(ref))
    assert err <= 1e-12, err
    # the limiter-free test problem is linear: one Newton iteration
    assert st["newton_its"] == 1


def test_exact_discrete_step_expanding():
    """The comoving diffusion carries 1/a^2 (checked at a = 0.5)."""
    n = 16
    model = heat_model(n)
    U = gaussian_state(n)
    h = 1.0 / n
    dt = 0.5 * h * h
    U1, _ = step(U, model, dt, a=0.5)
    ref = fft_step(U[2], dt, 1.0, h, 1.0, a=0.5)
    assert np.max(np.abs(U1[2] - ref)) / np.max(np.abs(ref)) <= 1e-12


def continuum(n, t, s0=0.1, Eb=1.0, A=1.0, D0=1.0):
    x = (np.arange(n) + 0.5) / n - 0.5
    s2 = s0 ** 2 + 2 * D0 * t
    out = np.zeros((n, n, n))
    for ix in range(-2, 3):
        for iy in range(-2, 3):
            for iz in range(-2, 3):
                X, Y, Z = np.meshgrid(x + ix, x + iy, x + iz, indexing="ij")
                out += np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / (2 * s2))
    return Eb + A * (s0 ** 2 / s2) ** 1.5 * out


def test_continuum_second_order():
    """Crank-Nicolson (theta = 1/2) with dt ~ h converges at order 2."""
    t_end = 0.005
    errs = []
    for n in (16, 32, 64):
        model = heat_model(n, theta=0.5, mg_levels=3)
        U = gaussian_state(n)
        nsteps = n // 4
        dt = t_end / nsteps
        for _ in range(nsteps):
            U, _ = step(U, model, dt)
        errs.append(np.max(np.abs(U[2] - continuum(n, t_end))))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert abs(orders[-1] - 2.0) <= 0.1, (errs, orders)
    assert orders[0] > 1.8, (errs, orders)
