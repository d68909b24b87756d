"""Newton matrix pieces and the Schur complement (Sec. 3.2.1, Eqs. 31-35).

J(U) = I + dt theta [[J_ee, J_en, J_eE], [J_ne, J_nn, J_nE], [J_Ee, J_En, J_EE]]
(Eq. 31), the derivative of the residual f(U) of Eq. 29.  The cell-local
blocks (Eq. 32) are taken by complex-step differentiation of
`physics.local_operators`: d L / d U_j = Im L(U + i h e_j) / h, exact to
rounding for these analytic expressions.

The diffusion term D_E(U) of the E rows depends on E (through the face
gradients and the limiter's R_f and E_f) and on the species fractions of
both cells of every face (through the face opacity).  The E-E part is the
7-point matrix of the face-flux derivatives (fld.face_derivatives); it is not
symmetric, because the limiter depends on E.  The species part couples the E
row of a cell to the fractions of itself and its six neighbours.  Sec. 3.2.1
lags that species dependence to the previous iterate to keep the Newton
matrix's off-diagonal blocks cell-local; here it is kept exact instead: the
species unknowns are still eliminated cell by cell (step (i) solves M per
cell), so their neighbour couplings fold into the 7-point Schur matrix and
its right side,
  with  omega_P = sum_s dkappa/dx_s W_s,   phi_P = sum_s dkappa/dx_s f~_s,
  and for a face (P, Q) with k = dt theta / (a^2 dx^2) dF/dkappa / u_E:
    S_PQ += k omega_Q,  S_PP += k omega_P,  S_QP -= k omega_P,  S_QQ -= k omega_Q,
    b_P  -= k (phi_P + phi_Q),  b_Q += k (phi_P + phi_Q).
So the Newton matrix here is the exact derivative of f, and the Schur
complement S = D - L M^-1 U (with these terms) is the exact reduction of
J S = -f.  Everything is in the scaled variables of Sec. 3.2.2.

Schur steps (Sec. 3.2.1): with [[M, U], [L, D]] (Eq. 33-34)
  (i)   f~_M = M^-1 f_M, W = M^-1 U                 (Eq. 35, dense per cell)
  (ii)  S s_E = b,  b = L f~_M - f_E (+ the species-opacity terms)
  (iii) s_M = -f~_M - W s_E
The 7-point S is stored as its diagonal and, per +x/+y/+z face, its two
off-diagonal couplings fw = -S_{P,P+d} and bw = -S_{P+d,P}:
  (S x)_P = diag_P x_P - sum_d [fw_d[P] x_{P+d} + bw_d[P-d] x_{P-d}].
The Krylov solve is preconditioned by a multigrid V-cycle of the symmetric
M-matrix P = [the cell-local part of S] + [the diffusion of the face-flux
derivative with respect to E_Q - E_P at fixed E_f and opacity, k (D + T) on
every face], whose diagonal is raised to S's own where that is larger:
pdiag = max(diag, local + sum of the six face couplings c), with
local = 1 + dt theta dL_E/dE - L W (>= 1 for monochromatic hydrogen) and
c = k (D + T) >= 0.  Raising the diagonal keeps P diagonally dominant; it
carries the part of the limiter's E_f derivative and of the opacity terms
that adds to S's diagonal (the Krylov iterations of the 256^3-cell-size HII
region drop by a third).  (The symmetric part (S + S^T)/2 is not used: those
terms add to its diagonal with either sign and can make it indefinite.)
"""
from __future__ import annotations

import numpy as np

from . import fld
from .physics import local_operators, opacity, opacity_derivatives


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


def diffusion_derivatives(U, nH, dt, a, model, D=None):
    """Scaled face derivatives of dt theta D_E: per +face d a dict with
    eP, eQ (d/dE_P, d/dE_Q of dt theta F / (a^2 dx^2)), c (the same factor
    times D + T) and kP, kQ (the kappa derivatives, divided by u_E); plus the
    list dkappa/dx_s.  With D (face
    coefficients held fixed) the flux is linear in E: dF/dE_Q = -dF/dE_P = D
    and nothing depends on kappa."""
    s = dt * model.theta / (a * a * model.dx * model.dx)
    if D is not None:
        out = []
        for Dd in D:
            z = np.zeros(Dd.shape)
            out.append(dict(eP=-s * Dd, eQ=s * Dd, c=s * Dd, kP=z, kQ=z))
        return out, opacity_derivatives(U, nH, a, model)
    fd = fld.face_derivatives(U[-1], opacity(U, nH, a, model), a, model)
    out = [dict(eP=s * f["dEP"], eQ=s * f["dEQ"], c=s * f["DT"], kP=s * f["dkP"] / model.u_E,
                kQ=s * f["dkQ"] / model.u_E) for f in fd]
    return out, opacity_derivatives(U, nH, a, model)


def schur_form(U, f, nH, eh, dt, a, H, model, D=None):
    """Steps (i)-(ii) setup: returns dict(ftM, W, diag, fx, fy, fz, bx, by, bz,
    b) for S and its right side, and dict entries pdiag, cx, cy, cz for the
    preconditioner's operator.  D: face coefficients held fixed (the
    residual's D argument)."""
    nb = model.nb
    ns = model.nspecies
    M, Ucol, Lrow, dloc = local_blocks(U, nH, eh, dt, a, H, model)
    shape = U.shape[1:]
    Mc = np.moveaxis(M.reshape(nb, nb, -1), -1, 0)                      # (N, nb, nb)
    rhs = np.stack([f[:nb].reshape(nb, -1), Ucol.reshape(nb, -1)], axis=-1)  # (nb, N, 2)
    rhs = np.moveaxis(rhs, 1, 0)                                         # (N, nb, 2)
    sol = np.linalg.solve(Mc, rhs)                                       # GEPP per cell
    ftM = np.moveaxis(sol[:, :, 0], 0, 1).reshape((nb,) + shape)
    W = np.moveaxis(sol[:, :, 1], 0, 1).reshape((nb,) + shape)
    dd, dkdx = diffusion_derivatives(U, nH, dt, a, model, D)
    omega = sum(dkdx[s] * W[1 + s] for s in range(ns)) if ns else np.zeros(shape)
    phi = sum(dkdx[s] * ftM[1 + s] for s in range(ns)) if ns else np.zeros(shape)
    local = dloc - np.sum(Lrow * W, axis=0)
    diag = local.copy()
    pdiag = local.copy()
    b = np.sum(Lrow * ftM, axis=0) - f[-1]
    fws, bws, cs = [], [], []
    for d in range(3):
        c = dd[d]["c"].copy()                            # k (D + T)
        fw = dd[d]["eQ"] - dd[d]["kQ"] * np.roll(omega, -1, axis=d)
        bw = -dd[d]["eP"] + dd[d]["kP"] * omega
        flow = dd[d]["kP"] * phi + dd[d]["kQ"] * np.roll(phi, -1, axis=d)
        if model.boundary == 2 and d == 0:
            # the ghost face (x slot after the last cell): Q is the first cell,
            # P a fixed value; it adds to the first cell's diagonal and right
            # side only
            g_fw, g_flow = fw[-1].copy(), dd[0]["kQ"][-1] * phi[0]
            g_c = c[-1].copy()                           # k (D + T), ghost face
            fw[-1] = 0.0
            bw[-1] = 0.0
            c[-1] = 0.0
            flow[-1] = 0.0
            diag[0] += g_fw
            pdiag[0] += g_c
            b[0] += g_flow
        diag = diag + bw + np.roll(fw, 1, axis=d)
        pdiag = pdiag + c + np.roll(c, 1, axis=d)
        b = b - flow + np.roll(flow, 1, axis=d)
        fws.append(fw)
        bws.append(bw)
        cs.append(c)
    pdiag = np.where(diag > pdiag, diag, pdiag)
    return dict(ftM=ftM, W=W, diag=diag, fx=fws[0], fy=fws[1], fz=fws[2],
                bx=bws[0], by=bws[1], bz=bws[2], b=b,
                pdiag=pdiag, cx=cs[0], cy=cs[1], cz=cs[2])


def operator(sch):
    """The full 7-point Schur operator (diag, fx, fy, fz, bx, by, bz)."""
    return tuple(sch[k] for k in ("diag", "fx", "fy", "fz", "bx", "by", "bz"))


def preconditioner_operator(sch):
    """The symmetric operator (pdiag, cx, cy, cz) the V-cycle is built on."""
    return tuple(sch[k] for k in ("pdiag", "cx", "cy", "cz"))


def recover(sE, sch):
    """Step (iii): full scaled Newton correction [s_M; s_E]."""
    sM = -sch["ftM"] - sch["W"] * sE[None]
    return np.concatenate([sM, sE[None]], axis=0)


def apply_schur(x, diag, cx, cy, cz, bx=None, by=None, bz=None):
    """7-point operator: (S x)_P = diag_P x_P - sum_d [fw_d[P] x_{P+d}
    + bw_d[P-d] x_{P-d}] with fw = (cx, cy, cz) and bw = (bx, by, bz); bw
    omitted: the symmetric operator with bw = fw."""
    y = diag * x
    for d, (fw, bw) in enumerate(zip((cx, cy, cz), (bx, by, bz))):
        bw = fw if bw is None else bw
        y = y - fw * np.roll(x, -1, axis=d) - np.roll(bw * x, 1, axis=d)
    return y


def dense_jacobian(U, nH, eh, dt, a, H, model, D=None):
    """Full scaled Newton matrix (nv*N, nv*N) for brute force on tiny grids:
    the local blocks, the E-E face-flux derivatives and the E-row couplings
    to the species fractions through the face opacities.

    Unknown ordering: variable-major, (v, i, j, k) flattened.  D: face
    coefficients held fixed (the lagged reading), as in schur_form.
    """
    nv = model.nv
    ns = model.nspecies
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
    dd, dkdx = diffusion_derivatives(U, nH, dt, a, model, D)
    cell = idx.reshape(shape)
    base = nb * N
    J[base + idx, base + idx] += dloc.ravel()
    # dt theta (D_E)_P = -k (F_{P+} - F_{P-}): row P takes -dF_{P+}, row Q
    # (its - face) takes +dF
    for d in range(3):
        nbr = np.roll(cell, -1, axis=d).ravel()
        P, Q = idx, nbr
        eP, eQ = dd[d]["eP"].ravel(), dd[d]["eQ"].ravel()
        kP, kQ = dd[d]["kP"].ravel(), dd[d]["kQ"].ravel()
        ghost = np.zeros(shape, dtype=bool)
        if model.boundary == 2 and d == 0:
            ghost[-1] = True          # the x slot after the last cell
        ghost = ghost.ravel()
        reg = ~ghost
        np.add.at(J, (base + P[reg], base + P[reg]), -eP[reg])
        np.add.at(J, (base + P[reg], base + Q[reg]), -eQ[reg])
        np.add.at(J, (base + Q[reg], base + P[reg]), eP[reg])
        np.add.at(J, (base + Q[reg], base + Q[reg]), eQ[reg])
        for s in range(ns):
            kap = dkdx[s].ravel()
            col = (1 + s) * N
            np.add.at(J, (base + P[reg], col + P[reg]), -kP[reg] * kap[P[reg]])
            np.add.at(J, (base + P[reg], col + Q[reg]), -kQ[reg] * kap[Q[reg]])
            np.add.at(J, (base + Q[reg], col + P[reg]), kP[reg] * kap[P[reg]])
            np.add.at(J, (base + Q[reg], col + Q[reg]), kQ[reg] * kap[Q[reg]])
        if ghost.any():
            # the ghost face of the x-left Dirichlet boundary enters the first
            # cell's row as +dF (its - face) with only Q derivatives
            Qg = Q[ghost]
            np.add.at(J, (base + Qg, base + Qg), eQ[ghost])
            for s in range(ns):
                kap = dkdx[s].ravel()
                np.add.at(J, (base + Qg, (1 + s) * N + Qg), kQ[ghost] * kap[Qg])
    return J
