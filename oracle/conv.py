"""FP64 reference of the learned Newton initial guess (test infrastructure).

Not part of the paper: a small 3-D convolutional network proposes the Newton
initial iterate from the two previous time levels; the unchanged Newton
tolerance judges it and the previous state is the fallback.  Definitions
(a stated reading):

Features per cell, channels (H):  for level t in (n, n-1):
    log10(E_t / u_E), e_t / u_e, logit(x_t) / 10          -> 6 channels
  plus log10(n_H / mean n_H)                              -> 7 channels
  (x clipped to [1e-12, 1 - 1e-12]; E floored at 1e-10 u_E, below which a
  cell's radiation is invisible in the scaled residual).  With helium the
  fractions x_HeI, x_HeII add logit channels: 11 channels.
Network: four 3x3x3 periodic convolutions, channels nin -> 16 -> 16 -> 16 ->
  nout, bias, LeakyReLU(0.01) after the first three.
Output: per cell a correction Delta to the linear extrapolation
  2 t^n - t^(n-1) of the transformed unknowns t = (log10 E/u_E, e/u_e,
  logit x / 10); the guess is the inverse transform of that sum, with
  e_c = e_guess - e_h.  The last layer starts at zero, so an untrained
  network proposes the extrapolation.
Loss: weighted mean squared error of Delta against t^(n+1) - (2 t^n -
  t^(n-1)); the radiation channel of each cell is weighted by E^n / u_E
  divided by its box mean, capped at 100 (the scaled Newton residual grows
  with E, so the guess must be most accurate where the radiation is
  strongest), the other channels by 1.

Everything here is plain loops over the 27 kernel offsets with NumPy, FP64.
"""
from __future__ import annotations

import numpy as np

LEAK = 0.01
HIDDEN = 16
OFFSETS = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
X_CLIP = 1e-12
LOGIT_SCALE = 10.0
E_FLOOR_REL = 1e-10
W_CAP = 100.0


def layer_shapes(nin, nout):
    return [(nin, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, nout)]


def n_params(nin, nout):
    return sum(27 * ci * co + co for ci, co in layer_shapes(nin, nout))


def unpack(theta, nin, nout):
    """Flat parameter vector -> [(W (27, co, ci), b (co,))] per layer.

    Flat order per layer: W in (offset, co, ci) order, then b.  Offset o is
    (dx, dy, dz) = OFFSETS[o] and the layer computes
    out[co, P] = b[co] + sum_o sum_ci W[o, co, ci] * in[ci, P + offset_o].
    """
    out, p = [], 0
    for ci, co in layer_shapes(nin, nout):
        W = theta[p:p + 27 * co * ci].reshape(27, co, ci)
        p += 27 * co * ci
        b = theta[p:p + co]
        p += co
        out.append((W, b))
    return out


def shift(a, off):
    """a[..., P + off] with periodic wrap (channels first, grid last 3 axes)."""
    return np.roll(a, shift=(-off[0], -off[1], -off[2]), axis=(-3, -2, -1))


def conv(x, W, b):
    co = W.shape[1]
    y = np.zeros((co,) + x.shape[1:])
    for o, off in enumerate(OFFSETS):
        y += np.einsum("kc,c...->k...", W[o], shift(x, off))
    return y + b.reshape((-1, 1, 1, 1))


def conv_dgrad(g, W):
    """Gradient of conv with respect to its input, given dL/dy = g."""
    ci = W.shape[2]
    dx = np.zeros((ci,) + g.shape[1:])
    for o, off in enumerate(OFFSETS):
        # y[P] uses x[P + off]  =>  dx[Q] += W^T g[Q - off]
        dx += np.einsum("kc,k...->c...", W[o], shift(g, tuple(-v for v in off)))
    return dx


def conv_wgrad(g, x):
    """dL/dW (27, co, ci) and dL/db (co,)."""
    dW = np.stack([np.einsum("kijl,cijl->kc", g, shift(x, off)) for off in OFFSETS])
    return dW, g.sum(axis=(1, 2, 3))


def leaky(z):
    return np.where(z > 0, z, LEAK * z)


def leaky_grad(z):
    return np.where(z > 0, 1.0, LEAK)


def forward(theta, feat, nin, nout):
    """Returns (output, cache of pre-activations and layer inputs)."""
    layers = unpack(theta, nin, nout)
    h = feat
    cache = []
    for li, (W, b) in enumerate(layers):
        z = conv(h, W, b)
        cache.append((h, z))
        h = leaky(z) if li < 3 else z
    return h, cache


def loss_weights(Un, u_E, nout):
    """Per-value loss weights: E^n/u_E over its mean for channel 0, else 1."""
    w = np.ones((nout,) + Un.shape[1:])
    e = np.maximum(Un[-1], E_FLOOR_REL * u_E) / u_E
    w[0] = np.minimum(e / e.mean(), W_CAP)
    return w


def loss_and_grad(theta, feat, target, nin, nout, weight=None):
    """(Weighted) mean squared error over all output values and its gradient."""
    out, cache = forward(theta, feat, nin, nout)
    diff = out - target
    wt = np.ones_like(diff) if weight is None else weight
    loss = float(np.mean(wt * diff * diff))
    g = 2.0 * wt * diff / diff.size
    layers = unpack(theta, nin, nout)
    grads = [None] * 4
    for li in range(3, -1, -1):
        h, z = cache[li]
        if li < 3:
            g = g * leaky_grad(z)
        dW, db = conv_wgrad(g, h)
        grads[li] = (dW, db)
        if li > 0:
            g = conv_dgrad(g, layers[li][0])
    flat = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return loss, flat


# ---- feature transforms -----------------------------------------------------
def _logit(x):
    x = np.clip(x, X_CLIP, 1.0 - X_CLIP)
    return np.log(x / (1.0 - x)) / LOGIT_SCALE


def _sigmoid(t):
    return 1.0 / (1.0 + np.exp(-t * LOGIT_SCALE))


def features(Un, Unm1, e_n, e_nm1, nH, u_e, u_E, nspecies):
    """Network input channels (nin, *grid) from two time levels."""
    ch = []
    for U, e in ((Un, e_n), (Unm1, e_nm1)):
        ch.append(np.log10(np.maximum(U[-1], E_FLOOR_REL * u_E) / u_E))
        ch.append(e / u_e)
        for s in range(nspecies):
            ch.append(_logit(U[1 + s]))
    ch.append(np.log10(nH / nH.mean()))
    return np.stack(ch)


def transformed(U, e, u_e, u_E, nspecies):
    """Output-space coordinates (log10 E/u_E, e/u_e, logit x / 10 ...)."""
    ch = [np.log10(np.maximum(U[-1], E_FLOOR_REL * u_E) / u_E), e / u_e]
    ch += [_logit(U[1 + s]) for s in range(nspecies)]
    return np.stack(ch)


def extrapolation(Un, Unm1, e_n, e_nm1, u_e, u_E, nspecies):
    """2 t^n - t^(n-1) in transformed coordinates."""
    return (2.0 * transformed(Un, e_n, u_e, u_E, nspecies)
            - transformed(Unm1, e_nm1, u_e, u_E, nspecies))


def target(Unp1, e_np1, Un, Unm1, e_n, e_nm1, u_e, u_E, nspecies):
    return (transformed(Unp1, e_np1, u_e, u_E, nspecies)
            - extrapolation(Un, Unm1, e_n, e_nm1, u_e, u_E, nspecies))


def decode(out, Un, Unm1, e_n, e_nm1, eh, u_e, u_E, nspecies):
    """Guess U from the network output (correction to the extrapolation)."""
    t = extrapolation(Un, Unm1, e_n, e_nm1, u_e, u_E, nspecies) + out
    U = np.empty_like(Un)
    U[-1] = u_E * 10.0 ** t[0]
    U[0] = u_e * t[1] - eh
    for s in range(nspecies):
        U[1 + s] = _sigmoid(t[2 + s])
    if nspecies == 3:
        tot = U[2] + U[3]
        over = tot > 1.0
        U[2] = np.where(over, U[2] / np.where(over, tot, 1), U[2])
        U[3] = np.where(over, U[3] / np.where(over, tot, 1), U[3])
    return U


def init_params(nin, nout, seed=0, last_scale=0.0):
    """He-normal weights (fan-in 27 * ci), zero biases; the last layer is
    scaled by last_scale (0: the untrained network outputs zero)."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (ci, co) in enumerate(layer_shapes(nin, nout)):
        std = np.sqrt(2.0 / (27 * ci)) * (last_scale if li == 3 else 1.0)
        parts.append(rng.standard_normal(27 * co * ci) * std)
        parts.append(np.zeros(co))
    return np.concatenate(parts)
