"""Pins of the FP64 reference network (learned initial guess).

- convolution: a single-offset kernel is a periodic shift (closed form), and
  the 27-offset convolution equals a direct triple loop on a tiny grid;
- dgrad is the adjoint of conv: <conv(x), g> = <x, dgrad(g)> (bias-free);
- the full backward pass equals central finite differences of the loss;
- decode(transformed(U)) is the identity (zero change -> level-n state).
"""
import numpy as np
import pytest

from oracle import conv as C


def test_shift_kernel_is_periodic_translation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 4, 5, 6))
    for o, off in enumerate(C.OFFSETS):
        W = np.zeros((27, 2, 2))
        W[o] = np.eye(2)
        y = C.conv(x, W, np.zeros(2))
        for i in range(4):
            for j in range(5):
                for k in range(6):
                    assert np.allclose(y[:, i, j, k],
                                       x[:, (i + off[0]) % 4, (j + off[1]) % 5, (k + off[2]) % 6])


def test_conv_matches_triple_loop():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 3, 4, 3))
    W = rng.standard_normal((27, 2, 3))
    b = rng.standard_normal(2)
    y = C.conv(x, W, b)
    ref = np.zeros_like(y)
    for co in range(2):
        for i in range(3):
            for j in range(4):
                for k in range(3):
                    s = b[co]
                    for o, (a, bb, c) in enumerate(C.OFFSETS):
                        for ci in range(3):
                            s += W[o, co, ci] * x[ci, (i + a) % 3, (j + bb) % 4, (k + c) % 3]
                    ref[co, i, j, k] = s
    assert np.allclose(y, ref, rtol=1e-13, atol=1e-13)


def test_dgrad_is_adjoint():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((5, 4, 4, 4))
    g = rng.standard_normal((3, 4, 4, 4))
    W = rng.standard_normal((27, 3, 5))
    lhs = np.sum(C.conv(x, W, np.zeros(3)) * g)
    rhs = np.sum(x * C.conv_dgrad(g, W))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("nin,nout", [(7, 3), (11, 5)])
def test_backward_matches_finite_differences(nin, nout):
    rng = np.random.default_rng(3)
    n = 4
    feat = rng.standard_normal((nin, n, n, n))
    target = rng.standard_normal((nout, n, n, n)) * 0.1
    theta = C.init_params(nin, nout, seed=4, last_scale=0.5)
    wt = rng.uniform(0.1, 3.0, target.shape)
    loss, grad = C.loss_and_grad(theta, feat, target, nin, nout, wt)
    idx = rng.choice(theta.size, 60, replace=False)
    for p in idx:
        h = 1e-6 * max(1.0, abs(theta[p]))
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        lp = C.loss_and_grad(tp, feat, target, nin, nout, wt)[0]
        lm = C.loss_and_grad(tm, feat, target, nin, nout, wt)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[p]) <= 1e-6 * max(abs(fd), 1e-3 * np.max(np.abs(grad))), p


def test_parameter_count():
    assert C.n_params(7, 3) == 18195
    assert C.n_params(11, 5) == 27 * (11 * 16 + 16 * 16 * 2 + 16 * 5) + 16 * 3 + 5


@pytest.mark.parametrize("ns", [1, 3])
def test_decode_of_zero_correction_is_extrapolation(ns):
    rng = np.random.default_rng(5)
    n = 4
    Un = np.empty((ns + 2, n, n, n))
    Un[-1] = 10 ** rng.uniform(-22, -14, (n, n, n))
    Un[1] = rng.uniform(1e-6, 1 - 1e-6, (n, n, n))
    if ns == 3:
        Un[2] = rng.uniform(0, 0.5, (n, n, n))
        Un[3] = rng.uniform(0, 0.5, (n, n, n))
    eh = rng.uniform(1e12, 2e12, (n, n, n))
    Un[0] = 0.0
    out = np.zeros((ns + 2, n, n, n))
    # two equal levels: the extrapolation is the level itself
    U = C.decode(out, Un, Un, eh, eh, eh, 1.2e12, 1e-20, ns)
    assert np.allclose(U[1:], Un[1:], rtol=1e-12, atol=1e-15)
    assert np.allclose(U[0], 0.0, atol=1e-3)
    # geometric decay of E continues geometrically
    Unm1 = Un.copy()
    Unm1[-1] = Un[-1] * 20.0
    U = C.decode(out, Un, Unm1, eh, eh, eh, 1.2e12, 1e-20, ns)
    keep = Un[-1] / 20.0 >= 1e-30
    assert np.allclose(U[-1][keep], Un[-1][keep] / 20.0, rtol=1e-12)
