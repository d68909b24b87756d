"""Writes hii256_first_step.npz: the oracle's first implicit step of the
256^3 isothermal-HII-region workload (Sec. 4.5 set-up at 256^3: centred
5e48 photons/s source, 13.2 kpc box, dt = 1e11 s, theta = 1, Newton tol 1e-6)
in the configuration the benchmark times (FP64, MG-preconditioned FGMRES with
the inexact-Newton forcing 1e-6 and the 16^3 source-subdomain correction
with 48 red-black sweeps on the Schur matrix over the box).

The full fields (3 x 256^3 doubles) are too large to keep, so the file holds
the step's schedule (Newton count, Krylov counts, line-search factors,
residual norms), per-variable sums, sums of squares, minima and maxima over
all cells, and the new state at sampled cells: the 16^3 block around the
source, the x, y and z lines through it, and 4096 cells drawn at random
(seed 2024).  Only the oracle and the seeded input generators run here.

Run from the repository root:  python tests/golden/make_hii256_first_step.py
(about 20 minutes on one core).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
import oracle  # noqa: E402
from oracle import newton  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hii256_first_step.npz")
# the benchmark's preconditioner and forcing
CONFIG = dict(box_size=16, box_levels=2, box_inner=4, box_coarse_sweeps=4, box_s_sweeps=48,
              pcg_forcing=1e-6,
              mg_fp32=0)


def workload():
    return synth.WORKLOADS["hii_256"].replace(**CONFIG)


def sample_cells(n, src_cell):
    """Flat indices of the sampled cells (sorted, unique)."""
    i, j, k = np.unravel_index(int(src_cell), (n, n, n))
    r = np.arange(-8, 8)
    bi, bj, bk = np.meshgrid((i + r) % n, (j + r) % n, (k + r) % n, indexing="ij")
    block = np.ravel_multi_index((bi.ravel(), bj.ravel(), bk.ravel()), (n, n, n))
    line = np.arange(n)
    lines = np.concatenate([
        np.ravel_multi_index((line, np.full(n, j), np.full(n, k)), (n, n, n)),
        np.ravel_multi_index((np.full(n, i), line, np.full(n, k)), (n, n, n)),
        np.ravel_multi_index((np.full(n, i), np.full(n, j), line), (n, n, n))])
    rnd = np.random.default_rng(2024).choice(n ** 3, 4096, replace=False)
    return np.unique(np.concatenate([block, lines, rnd])).astype(np.int64)


def main():
    w = workload()
    m = oracle.model_from_workload(w)
    s = synth.initial_state(w)
    t0 = time.perf_counter()
    U, st = newton.newton_step(s["U"], s["U"], s["nH"], s["eh"], s["src_cells"], s["src_Q"],
                               w.dt, w.cosmology(0), m)
    secs = time.perf_counter() - t0
    print("status %d, Newton %d, Krylov %s, lambdas %s, %.0f s"
          % (st["status"], st["newton_its"], st["cg_its"], st["lambdas"], secs), flush=True)
    n = w.n
    cells = sample_cells(n, s["src_cells"][0])
    flat = U.reshape(U.shape[0], -1)
    np.savez_compressed(
        OUT, n=n, status=st["status"], newton_its=st["newton_its"],
        krylov_its=np.asarray(st["cg_its"], dtype=np.int64),
        lambdas=np.asarray(st["lambdas"]), fnorms=np.asarray(st["fnorms"]),
        cells=cells, U_cells=flat[:, cells],
        sums=flat.sum(axis=1), sumsq=(flat * flat).sum(axis=1),
        mins=flat.min(axis=1), maxs=flat.max(axis=1), oracle_seconds=secs)


if __name__ == "__main__":
    main()
