"""Geometric multigrid V-cycle and preconditioned CG for the Schur system.

The paper solves the scalar Schur system with a multigrid-preconditioned
conjugate gradient method (Sec. 3.2.1) but gives the multigrid only by
reference to a library, so its definition here is a stated reading:

Hierarchy (periodic, n_{l+1} = n_l / 2), built once per Schur matrix:
  local_l   = diag_l - sum over the 6 faces of c_l
  local_l+1 = mean of local_l over the 8 children
  c^d_l+1   = (1/4) * mean over the 4 fine columns crossing the coarse face
              (I, I + e_d) of the series (weighted harmonic) coupling of the
              three fine faces 2I, 2I+1, 2I+2 along d, weights 1/4, 1/2, 1/4:
              the path between the two coarse centres crosses half of the
              first segment, the whole middle one and half of the last;
              equal fine couplings c give c/4 (rediscretization at 2h)
  diag_l+1  = local_l+1 + sum over the 6 faces of c_l+1
Smoother: red-black Gauss-Seidel, colour (i + j + k) mod 2 (red = 0),
  x_P <- (b_P + sum_faces c_f x_nbr) / diag_P.
Transfers: cell-centred trilinear prolongation P (weights 3/4, 1/4 per axis)
  and restriction R = P^T / 8.
V(l): x = 0; nu1 x (red, black); r = b - A x; V(l+1) on R r; x += P e;
  nu2 x (black, red).  Coarsest: k x (red, black) then k x (black, red).
PCG: flexible (Polak-Ribiere) beta, x0 = 0, stop when ||r||_2 <= rtol ||b||_2
  or, in a Newton step with a forcing factor, ||r||_2 <= forcing ||f(U_k)||_2.
  Optional source-subdomain correction added to the V-cycle (see pcg).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .jacobian import apply_schur


def colour_mask(shape, colour):
    i, j, k = np.indices(shape)
    return ((i + j + k) % 2) == colour


def _pair_mean(a, axis):
    """Mean of consecutive pairs (2I, 2I+1) along `axis`."""
    ev = np.take(a, np.arange(0, a.shape[axis], 2), axis=axis)
    od = np.take(a, np.arange(1, a.shape[axis], 2), axis=axis)
    return 0.5 * (ev + od)


def coarsen(op):
    """Coarse operator (diag, cx, cy, cz) from a fine one (periodic)."""
    diag, cs = op[0], op[1:]
    csum = sum(c + np.roll(c, 1, axis=d) for d, c in enumerate(cs))
    local_c = diag - csum
    for ax in range(3):
        local_c = _pair_mean(local_c, ax)            # mean over the 8 children
    cc = []
    for d, c in enumerate(cs):
        n = c.shape[d]
        ca = np.take(c, np.arange(0, n, 2), axis=d)              # face 2I
        cb = np.take(c, np.arange(1, n, 2), axis=d)              # face 2I+1
        cc_ = np.take(c, (np.arange(0, n, 2) + 2) % n, axis=d)   # face 2I+2
        with np.errstate(divide="ignore"):
            inv = 0.25 / ca + 0.5 / cb + 0.25 / cc_
        series = np.where(np.isfinite(inv) & (inv > 0), 1.0 / np.where(inv > 0, inv, 1.0), 0.0)
        for ax in range(3):
            if ax != d:
                series = _pair_mean(series, ax)      # parallel: mean over the 4 columns
        cc.append(0.25 * series)
    csum_c = sum(c + np.roll(c, 1, axis=d) for d, c in enumerate(cc))
    return (local_c + csum_c, cc[0], cc[1], cc[2])


def hierarchy(op, levels):
    ops = [tuple(op)]
    for _ in range(levels - 1):
        ops.append(coarsen(ops[-1]))
    return ops


def rbgs_colour(x, b, op, colour):
    """One red-black Gauss-Seidel half sweep on cells of `colour` (in place)."""
    diag, cx, cy, cz = op
    s = b.copy()
    for d, c in enumerate((cx, cy, cz)):
        s = s + c * np.roll(x, -1, axis=d) + np.roll(c * x, 1, axis=d)
    m = colour_mask(x.shape, colour)
    x[m] = s[m] / diag[m]


def _prolong_axis(c, axis):
    n = c.shape[axis]
    f = np.repeat(c, 2, axis=axis) * 0.75
    left = np.repeat(np.roll(c, 1, axis=axis), 2, axis=axis)    # I-1 for even children
    right = np.repeat(np.roll(c, -1, axis=axis), 2, axis=axis)  # I+1 for odd children
    idx = np.arange(2 * n)
    shape = [1, 1, 1]
    shape[axis] = 2 * n
    even = (idx % 2 == 0).reshape(shape)
    return f + 0.25 * np.where(even, left, right)


def prolong(xc):
    """Cell-centred trilinear interpolation to the fine grid."""
    f = xc
    for ax in range(3):
        f = _prolong_axis(f, ax)
    return f


def _restrict_axis(f, axis):
    a0 = np.take(f, np.arange(0, f.shape[axis], 2), axis=axis)     # 2I
    a1 = np.take(f, np.arange(1, f.shape[axis], 2), axis=axis)     # 2I+1
    am = np.roll(a1, 1, axis=axis)                                  # 2I-1
    ap = np.roll(a0, -1, axis=axis)                                 # 2I+2
    return 0.375 * (a0 + a1) + 0.125 * (am + ap)


def restrict(r):
    """R = P^T / 8."""
    c = r
    for ax in range(3):
        c = _restrict_axis(c, ax)
    return c


def vcycle(b, ops, model, level=0, dtype=np.float64):
    """Apply the V-cycle preconditioner on level `level` to right side b."""
    op = tuple(o.astype(dtype) for o in ops[level])
    b = b.astype(dtype)
    x = np.zeros_like(b)
    if level == len(ops) - 1:
        for _ in range(model.mg_coarse_sweeps):
            rbgs_colour(x, b, op, 0)
            rbgs_colour(x, b, op, 1)
        for _ in range(model.mg_coarse_sweeps):
            rbgs_colour(x, b, op, 1)
            rbgs_colour(x, b, op, 0)
        return x
    for _ in range(model.mg_pre):
        rbgs_colour(x, b, op, 0)
        rbgs_colour(x, b, op, 1)
    r = b - apply_schur(x, *op)
    e = vcycle(restrict(r), ops, model, level + 1, dtype)
    x = x + prolong(e)
    for _ in range(model.mg_post):
        rbgs_colour(x, b, op, 1)
        rbgs_colour(x, b, op, 0)
    return x


def box_cells(centre, B, shape):
    """Index arrays of the B^3 box centred on `centre` (periodic wrap)."""
    return [(np.arange(B) - B // 2 + c) % n for c, n in zip(centre, shape)]


def box_operator(op, centres, B):
    """The operator restricted to boxes around `centres`, stacked along x:
    diagonal unchanged, couplings inside a box kept, couplings out of a box
    (its last layer in each direction) zero."""
    shape = op[0].shape
    parts = [[], [], [], []]
    for c in centres:
        sel = np.ix_(*box_cells(c, B, shape))
        parts[0].append(op[0][sel])
        for d in range(3):
            cd = op[1 + d][sel].copy()
            last = [slice(None)] * 3
            last[d] = B - 1
            cd[tuple(last)] = 0.0
            parts[1 + d].append(cd)
    return tuple(np.concatenate(q, axis=0) for q in parts)


def pcg_fixed(op, b, ops, model, k, dtype=np.float64):
    """k iterations of flexible PCG from zero with the V-cycle on `ops`."""
    def V(r):
        return vcycle(r, ops, model, 0, dtype).astype(np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    z = V(r)
    p = z.copy()
    rho = np.sum(r * z)
    for it in range(1, k + 1):
        q = apply_schur(p, *op)
        # the count is fixed: once the residual has vanished (p = 0, rho = 0)
        # the iterate stays where it is
        pq = np.sum(p * q)
        alpha = rho / pq if pq > 0.0 else 0.0
        x = x + alpha * p
        r_old = r
        r = r - alpha * q
        if it == k:
            break
        z = V(r)
        rho_new = np.sum(z * r)
        beta = (rho_new - np.sum(z * r_old)) / rho if rho != 0.0 else 0.0
        rho = rho_new
        p = z + beta * p
    return x


def box_smooth(z, r, sop, centres, B, sweeps):
    """Red-black Gauss-Seidel on S z = r over the cells of each source's box
    (the box_cells of box_operator), box by box in source order, `sweeps`
    (red, black) pairs per box, with the full (non-symmetric) 7-point
    operator sop = (diag, fx, fy, fz, bx, by, bz); cells outside the boxes
    are read, not changed.  Each half-sweep works on the box plus a one-cell
    halo (periodic), so the update of a box cell sees its six neighbours."""
    diag, fx, fy, fz, bx, by, bz = sop
    shape = z.shape
    inner = (slice(1, B + 1),) * 3
    for c in centres:
        idx = [(np.arange(-1, B + 1) - B // 2 + ci) % n for ci, n in zip(c, shape)]
        sel = np.ix_(*idx)
        box = np.ix_(*[i[1:-1] for i in idx])
        parity = (idx[0][:, None, None] + idx[1][None, :, None] + idx[2][None, None, :]) % 2
        d_box = diag[box]
        fb = [a[sel] for a in (fx, fy, fz)]
        bb = [a[sel] for a in (bx, by, bz)]
        r_box = r[box]
        for _ in range(sweeps):
            for colour in (0, 1):
                zh = z[sel]
                t = r_box.copy()
                for d in range(3):
                    t = t + fb[d][inner] * np.roll(zh, -1, axis=d)[inner] \
                        + np.roll(bb[d] * zh, 1, axis=d)[inner]
                z[box] = np.where(parity[inner] == colour, t / d_box, zh[inner])
    return z


def preconditioner(op, model, centres=None, precond=True, sop=None):
    """z = P r for the symmetric 7-point operator op = (diag, cx, cy, cz):
    the V-cycle on its hierarchy, followed (model.box_size > 0 with source
    `centres`, (i, j, k) cells) by the source-subdomain correction: on a
    box_size^3 box around every source, model.box_inner iterations of
    flexible PCG from zero for the operator restricted to the boxes, with its
    own box_levels-level V-cycle, applied to the residual the V-cycle left;
    the boxes' parts are added box by box.  With model.box_s_sweeps > 0 and
    the full operator sop, box_smooth then runs that many (red, black) pairs
    on S z = r over each box: the part of S that the symmetric operator
    leaves out matters most around the sources."""
    op = tuple(op[:4])
    if not precond:
        return lambda r: r.copy()
    ops = hierarchy(op, model.mg_levels)
    dt = np.float32 if model.mg_fp32 else np.float64
    boxes = model.box_size > 0 and centres is not None and len(centres) > 0
    if boxes:
        B = model.box_size
        bop = box_operator(op, centres, B)
        bops = hierarchy(bop, model.box_levels)
        bmodel = dataclasses.replace(
            model, mg_coarse_sweeps=model.box_coarse_sweeps or model.mg_coarse_sweeps)
        sels = [np.ix_(*box_cells(c, B, op[0].shape)) for c in centres]

    def V(r):
        z = vcycle(r, ops, model, 0, dt).astype(np.float64)
        if boxes:
            res = r - apply_schur(z, *op)
            rb = np.concatenate([res[sel] for sel in sels], axis=0)
            y = pcg_fixed(bop, rb, bops, bmodel, model.box_inner, dt)
            for s_, sel in enumerate(sels):
                z[sel] += y[s_ * B:(s_ + 1) * B]
            if model.box_s_sweeps > 0 and sop is not None:
                z = box_smooth(z, r, sop, centres, B, model.box_s_sweeps)
        return z
    return V


def pcg(op, b, model, rtol=None, maxit=None, precond=True, atol=0.0, centres=None):
    """Flexible PCG on S s = b for a symmetric operator op = (diag, cx, cy,
    cz); stops at ||r||_2 <= max(rtol ||b||_2, atol).  The preconditioner is
    preconditioner(op, ...).  Returns (s, iterations, ||r||/||b||)."""
    rtol = model.pcg_rtol if rtol is None else rtol
    maxit = model.pcg_maxit if maxit is None else maxit
    V = preconditioner(op, model, centres, precond)
    x = np.zeros_like(b)
    bn = np.sqrt(np.sum(b * b))
    if bn == 0.0:
        return x, 0, 0.0
    r = b.copy()
    z = V(r)
    p = z.copy()
    rho = np.sum(r * z)
    rn = bn
    for k in range(1, maxit + 1):
        q = apply_schur(p, *op)
        alpha = rho / np.sum(p * q)
        x = x + alpha * p
        r_old = r
        r = r - alpha * q
        rn = np.sqrt(np.sum(r * r))
        if rn <= max(rtol * bn, atol):
            return x, k, rn / bn
        z = V(r)
        rho_new = np.sum(z * r)
        beta = (rho_new - np.sum(z * r_old)) / rho
        rho = rho_new
        p = z + beta * p
    return x, maxit, rn / bn


# second Gram-Schmidt pass when the projection leaves less than this
# fraction of the product's norm: a loss of two digits or more
REORTH = 0.01


def fgmres(op, pop, b, model, rtol=None, maxit=None, precond=True, atol=0.0, centres=None,
           restart=None):
    """Flexible GMRES (right preconditioning, restarted every `restart`
    iterations) on S s = b for the 7-point operator op = (diag, fx, fy, fz,
    bx, by, bz), which need not be symmetric; the preconditioner is
    preconditioner(pop, ...) for a symmetric operator pop = (diag, cx, cy,
    cz) (the V-cycle, plus the subdomain correction).  Stops once the least-squares
    residual ||b - S s||_2 <= max(rtol ||b||_2, atol), or after maxit
    iterations (rtol = atol = 0: exactly maxit).

    Arnoldi with classical Gram-Schmidt and one conditional second pass:
    v_0 = r / ||r||, z_j = P v_j, w = S z_j, h_ij = w . v_i (i <= j),
    w' = w - sum_i h_ij v_i; if ||w'|| < REORTH ||w|| (cancellation of two
    digits or more: the test of Daniel, Gragg, Kaufman and Stewart with a
    smaller threshold than their 1/sqrt(2); the orthogonality lost by one
    pass is then at most ~1e-14) the projection is repeated on w' and its
    coefficients added to h; h_{j+1,j} = ||w'||,
    v_{j+1} = w' / h_{j+1,j}.  The Hessenberg columns are reduced by Givens
    rotations, whose last sine gives the residual norm, and the update is
    s += sum_j y_j z_j.  Returns (s, iterations, estimate / ||b||)."""
    rtol = model.pcg_rtol if rtol is None else rtol
    maxit = model.pcg_maxit if maxit is None else maxit
    m = model.krylov_restart if restart is None else restart
    P = preconditioner(pop, model, centres, precond, sop=op)
    x = np.zeros_like(b)
    bn = np.sqrt(np.sum(b * b))
    if bn == 0.0:
        return x, 0, 0.0
    tol = max(rtol * bn, atol)
    its = 0
    r = b.copy()
    est = bn
    while True:
        beta = np.sqrt(np.sum(r * r))
        if beta == 0.0:
            return x, its, 0.0
        V = [r / beta]
        Z = []
        Hc = []                       # rotated Hessenberg columns
        cs, sn = [], []
        g = [beta]
        done = False
        for j in range(m):
            Z.append(P(V[j]))
            w = apply_schur(Z[j], *op)
            wn = np.sqrt(np.sum(w * w))
            h = [float(np.sum(w * V[i])) for i in range(j + 1)]
            for i in range(j + 1):
                w = w - h[i] * V[i]
            hn = np.sqrt(np.sum(w * w))
            if hn < REORTH * wn:
                h2 = [float(np.sum(w * V[i])) for i in range(j + 1)]
                for i in range(j + 1):
                    w = w - h2[i] * V[i]
                    h[i] += h2[i]
                hn = np.sqrt(np.sum(w * w))
            h.append(hn)
            V.append(w / hn if hn > 0.0 else w)
            for i in range(j):
                t = cs[i] * h[i] + sn[i] * h[i + 1]
                h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1]
                h[i] = t
            den = np.sqrt(h[j] * h[j] + h[j + 1] * h[j + 1])
            c_, s_ = (h[j] / den, h[j + 1] / den) if den > 0.0 else (1.0, 0.0)
            cs.append(c_)
            sn.append(s_)
            h[j] = den
            g.append(-s_ * g[j])
            g[j] = c_ * g[j]
            Hc.append(h[:j + 1])
            its += 1
            est = abs(g[j + 1])
            if est <= tol or its >= maxit or hn == 0.0:
                done = True
                break
        k = len(Hc)
        y = [0.0] * k
        for i in range(k - 1, -1, -1):
            t = g[i]
            for l in range(i + 1, k):
                t -= Hc[l][i] * y[l]
            y[i] = t / Hc[i][i] if Hc[i][i] != 0.0 else 0.0
        for i in range(k):
            x = x + y[i] * Z[i]
        if done:
            return x, its, est / bn
        r = b - apply_schur(x, *op)


def krylov(op, pop, b, model, **kw):
    """The Schur solve of a Newton iteration: FGMRES (model.krylov_restart
    > 0) on the operator op preconditioned through pop, or flexible PCG (0)
    on pop itself, which is the whole operator only when the limiter does not
    depend on E (constant D) and there are no species-opacity terms."""
    if model.krylov_restart > 0:
        return fgmres(op, pop, b, model, **kw)
    return pcg(pop, b, model, **kw)
