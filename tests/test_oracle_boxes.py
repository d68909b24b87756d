"""The source-subdomain correction of the preconditioner.

The stacked box operator must be the Schur operator restricted to each box's
cells (diagonal kept, couplings out of the box dropped), and block-diagonal
across boxes: checked against the dense matrix of the 7-point operator on an
8^3 grid, with two boxes that overlap.  A preconditioner change must not
change the solution: PCG with the correction converges to the dense solve.
"""
import dataclasses

import numpy as np

import synth
import oracle
from oracle import mg
from oracle.jacobian import apply_schur


def random_op(n, seed):
    rng = np.random.default_rng(seed)
    cs = [rng.uniform(0.1, 10.0, (n,) * 3) for _ in range(3)]
    csum = sum(c + np.roll(c, 1, axis=d) for d, c in enumerate(cs))
    return (1.0 + rng.uniform(0.0, 5.0, (n,) * 3) + csum, cs[0], cs[1], cs[2])


def dense(opr, shape):
    N = int(np.prod(shape))
    M = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1.0
        M[:, j] = apply_schur(e.reshape(shape), *opr).ravel()
    return M


def test_box_operator_is_the_restriction():
    n, B = 8, 4
    op = random_op(n, 1)
    centres = [(1, 2, 3), (2, 3, 3)]          # overlapping boxes
    bop = mg.box_operator(op, centres, B)
    Mb = dense(bop, (len(centres) * B, B, B))
    Mf = dense(op, (n, n, n))
    nb = B ** 3
    for s, c in enumerate(centres):
        idx = np.ravel_multi_index(np.meshgrid(*mg.box_cells(c, B, (n, n, n)), indexing="ij"),
                                   (n, n, n)).ravel()
        blk = Mb[s * nb:(s + 1) * nb, s * nb:(s + 1) * nb]
        assert np.allclose(blk, Mf[np.ix_(idx, idx)], rtol=0, atol=1e-13)
        for t in range(len(centres)):
            if t != s:
                assert not np.any(Mb[s * nb:(s + 1) * nb, t * nb:(t + 1) * nb])


def test_pcg_with_boxes_reaches_the_dense_solution():
    n = 16
    op = random_op(n, 2)
    rng = np.random.default_rng(3)
    b = rng.standard_normal((n,) * 3)
    w = synth.CFG_SMALL.replace(n=n, mg_levels=3)
    m = oracle.model_from_workload(w, pcg_rtol=1e-12, pcg_maxit=100)
    mb = dataclasses.replace(m, box_size=8, box_levels=2, box_inner=3)
    x_ref = np.linalg.solve(dense(op, (n,) * 3), b.ravel()).reshape((n,) * 3)
    x0, it0, _ = mg.pcg(op, b, m)
    x1, it1, _ = mg.pcg(op, b, mb, centres=[(8, 8, 8), (1, 14, 5)])
    for x in (x0, x1):
        assert np.max(np.abs(x - x_ref)) <= 1e-9 * np.max(np.abs(x_ref))
    assert it1 <= it0


def test_fixed_count_pcg_stops_moving_once_converged():
    """The inner PCG of the correction runs a fixed number of iterations: a
    zero right side stays zero (no 0/0), and on a box small enough for the
    V-cycle to be an exact solve, iterations beyond convergence leave the
    solution of the dense system unchanged."""
    n = 8
    op = random_op(n, 5)
    w = synth.CFG_SMALL.replace(n=n, mg_levels=1)
    m = oracle.model_from_workload(w)
    m = dataclasses.replace(m, mg_coarse_sweeps=200)
    ops = mg.hierarchy(op, 1)
    x = mg.pcg_fixed(op, np.zeros((n,) * 3), ops, m, 6)
    assert np.all(x == 0.0)
    b = np.random.default_rng(6).standard_normal((n,) * 3)
    x_ref = np.linalg.solve(dense(op, (n,) * 3), b.ravel()).reshape((n,) * 3)
    for k in (2, 8):
        x = mg.pcg_fixed(op, b, ops, m, k)
        assert np.all(np.isfinite(x))
        assert np.max(np.abs(x - x_ref)) <= 1e-10 * np.max(np.abs(x_ref)), k


def test_box_smoothing_on_the_full_operator():
    """box_smooth: Gauss-Seidel on S z = r over a box.  With the box covering
    the whole grid, repeated sweeps on a diagonally dominant non-symmetric
    7-point operator converge to the direct solution; with a smaller box only
    its cells change, and one sweep there equals the red then black updates
    written out cell by cell."""
    import scipy.sparse.linalg as spla
    from oracle import mg, newton
    rng = np.random.default_rng(5)
    n = 8
    shape = (n, n, n)
    fs = [rng.uniform(0.0, 1.0, shape) for _ in range(3)]
    bs = [rng.uniform(0.0, 1.0, shape) for _ in range(3)]
    diag = 7.0 + rng.uniform(0.0, 1.0, shape)
    sop = (diag, fs[0], fs[1], fs[2], bs[0], bs[1], bs[2])
    r = rng.standard_normal(shape)
    A = newton.schur_matrix(sop).tocsc()
    exact = spla.spsolve(A, r.ravel()).reshape(shape)
    z = mg.box_smooth(np.zeros(shape), r, sop, [(4, 4, 4)], n, 60)
    assert np.max(np.abs(z - exact)) <= 1e-10 * np.max(np.abs(exact))
    # a 4^3 box: cells outside keep their values
    z0 = rng.standard_normal(shape)
    z1 = mg.box_smooth(z0.copy(), r, sop, [(2, 3, 4)], 4, 1)
    inside = np.zeros(shape, dtype=bool)
    inside[np.ix_(*mg.box_cells((2, 3, 4), 4, shape))] = True
    assert np.array_equal(z1[~inside], z0[~inside])
    # the same sweep written cell by cell (red cells first, then black)
    z2 = z0.copy()
    for colour in (0, 1):
        for i, j, k in zip(*np.nonzero(inside)):
            if (i + j + k) % 2 != colour:
                continue
            t = r[i, j, k]
            for d, (f, b) in enumerate(zip(fs, bs)):
                p = [i, j, k]
                q = list(p)
                p[d] = (p[d] + 1) % n
                q[d] = (q[d] - 1) % n
                t += f[i, j, k] * z2[tuple(p)] + b[tuple(q)] * z2[tuple(q)]
            z2[i, j, k] = t / diag[i, j, k]
    assert np.allclose(z1, z2, rtol=1e-14, atol=0.0)
