"""Newton matrix pieces and the Schur complement (Sec. 3.2.1, Eqs. 31-35).

J(U) = I + dt theta [[J_ee, J_en, J_eE], [J_ne, J_nn, J_nE], [J_Ee, J_En, J_EE]]
(Eq. 31).  All blocks but J_EE are cell-local (Eq. 32); J_EE adds the
diffusion operator, whose face coefficients are the time-lagged D_f of the
step (see residual.py), so the E-E block is exact and symmetric.

The local derivatives are taken by complex-step differentiation of
`physics.local_operators`: d L / d U_j = Im L(U + i h e_j) / h, which is exact
to rounding for these analytic expressions.  Everything is in the scaled
variables of Sec. 3.2.2.

Schur steps (Sec. 3.2.1): with [[M, U], [L, D]] (Eq. 33-34)
  (i)   f~_M = M^-1 f_M, W = M^-1 U                 (Eq. 35, dense per cell)
  (ii)  S = D - L W,  b = L f~_M - f_E,  solve S s_E = b
  (iii) s_M = -f~_M - W s_E
"""
from __future__ import annotations

import numpy as np

from .physics import local_operators


def local_derivatives(U, nH, eh, a, H, model):
    """dL_i / dU~_j (unscaled rows, scaled columns): array (nv, nv, *grid)."""
    nv = model.nv
    u = model.scales
    out = np.empty((nv, nv) + U.shape[1:])
    for j in range(nv):
        h = 1e-30 * (np.abs(U[j]) / u[j] + 1.0)
        Uc = U.astype(complex)
        Uc[j] = Uc[j] + 1j * h * u[j]
        Lc = local_operators(Uc, nH, eh, a, H, model)
        out[:, j] = Lc.imag / h
    return out


def local_blocks(U, nH, eh, dt, a, H, model):
    """Scaled local blocks per cell.

    Returns (M (nb, nb, *g), Ucol (nb, *g), Lrow (nb, *g), dloc (*g)) where
    M = I + dt theta J_MM, Ucol = dt theta J_ME, Lrow = dt theta J_EM and
    dloc = 1 + dt theta dL_E,loc/dE, all in scaled variables.
    """
    nb = model.nb
    u = model.scales
    dtt = dt * model.theta
    dL = local_derivatives(U, nH, eh, a, H, model)
    J = dtt * dL / u.reshape((-1, 1) + (1,) * (U.ndim - 1))
    M = J[:nb, :nb].copy()
    for i in range(nb):
        M[i, i] += 1.0
    return M, J[:nb, nb].copy(), J[nb, :nb].copy(), 1.0 + J[nb, nb]


def face_couplings(Dfaces, dt, a, model):
    """c_f = dt theta D_f / (a^2 dx^2) on the +x, +y, +z faces."""
    s = dt * model.theta / (a * a * model.dx * model.dx)
    return [s * D for D in Dfaces]


def schur_form(U, f, Dfaces, nH, eh, dt, a, H, model):
    """Steps (i)-(ii) setup: returns dict(ftM, W, diag, cx, cy, cz, b)."""
    nb = model.nb
    M, Ucol, Lrow, dloc = local_blocks(U, nH, eh, dt, a, H, model)
    shape = U.shape[1:]
    Mc = np.moveaxis(M.reshape(nb, nb, -1), -1, 0)                      # (N, nb, nb)
    rhs = np.stack([f[:nb].reshape(nb, -1), Ucol.reshape(nb, -1)], axis=-1)  # (nb, N, 2)
    rhs = np.moveaxis(rhs, 1, 0)                                         # (N, nb, 2)
    sol = np.linalg.solve(Mc, rhs)                                       # GEPP per cell
    ftM = np.moveaxis(sol[:, :, 0], 0, 1).reshape((nb,) + shape)
    W = np.moveaxis(sol[:, :, 1], 0, 1).reshape((nb,) + shape)
    c = face_couplings(Dfaces, dt, a, model)
    cb = None
    if model.boundary == 2:
        # the x-left Dirichlet face couples the first cell to a fixed value:
        # it enters that cell's diagonal and no coupling
        c[0] = c[0].copy()
        cb = c[0][-1].copy()
        c[0][-1] = 0.0
    csum = sum(cd + np.roll(cd, 1, axis=d) for d, cd in enumerate(c))
    if cb is not None:
        csum[0] = csum[0] + cb
    diag = dloc + csum - np.sum(Lrow * W, axis=0)
    b = np.sum(Lrow * ftM, axis=0) - f[-1]
    return dict(ftM=ftM, W=W, diag=diag, cx=c[0], cy=c[1], cz=c[2], b=b)


def recover(sE, sch):
    """Step (iii): full scaled Newton correction [s_M; s_E]."""
    sM = -sch["ftM"] - sch["W"] * sE[None]
    return np.concatenate([sM, sE[None]], axis=0)


def apply_schur(x, diag, cx, cy, cz):
    """7-point Schur operator: (S x)_P = diag_P x_P - sum_faces c_f x_nbr."""
    y = diag * x
    for d, c in enumerate((cx, cy, cz)):
        y = y - c * np.roll(x, -1, axis=d) - np.roll(c * x, 1, axis=d)
    return y


def dense_jacobian(U, Dfaces, nH, eh, dt, a, H, model):
    """Full scaled Newton matrix (nv*N, nv*N) for brute force on tiny grids.

    Unknown ordering: variable-major, (v, i, j, k) flattened.
    """
    nv = model.nv
    shape = U.shape[1:]
    N = int(np.prod(shape))
    M, Ucol, Lrow, dloc = local_blocks(U, nH, eh, dt, a, H, model)
    nb = model.nb
    J = np.zeros((nv * N, nv * N))
    idx = np.arange(N)
    for i in range(nb):
        for j in range(nb):
            J[i * N + idx, j * N + idx] = M[i, j].ravel()
        J[i * N + idx, nb * N + idx] = Ucol[i].ravel()
        J[nb * N + idx, i * N + idx] = Lrow[i].ravel()
    # E-E block: dloc on the diagonal plus frozen diffusion
    c = face_couplings(Dfaces, dt, a, model)
    cell = idx.reshape(shape)
    base = nb * N
    J[base + idx, base + idx] += dloc.ravel()
    for d in range(3):
        nbr = np.roll(cell, -1, axis=d).ravel()
        cd = c[d].ravel()
        np.add.at(J, (base + idx, base + idx), cd)
        np.add.at(J, (base + nbr, base + nbr), cd)
        np.add.at(J, (base + idx, base + nbr), -cd)
        np.add.at(J, (base + nbr, base + idx), -cd)
    return J
