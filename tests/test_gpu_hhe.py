"""Hydrogen + helium (4x4 local blocks, grey T_B = 1e5 K blackbody) in the
512^3 configuration: lognormal medium with sigma_ln = 1.5, 64 sources, an
expanding box from a = 0.1, FP32 V-cycle and the learned-guess network, whose
untrained form (zero last layer) proposes the linear extrapolation of the two
previous levels.

At 512^3 the oracle checks sampled outputs: the residual and the time level
are cell-local given a one-cell neighbourhood, so a block cut around sampled
cells and evaluated by the oracle is exact in its interior.  The 64^3-aligned
block of the 512^3 initial state that holds the most sources is cut out and
rerun as a periodic 64^3 problem with those sources on both sides: the FP64
library step for step against the oracle (counts, fields to 1e-10), and the
FP32 V-cycle with the learned guess against the FP64 oracle, per field.  The
same generator at 64^3 (the same cell size, a medium of its own) is rerun the
same way.
"""
import numpy as np
import pytest
import torch

import synth
import oracle
from oracle import newton as onewt
from oracle import residual as ores
from paper_0901_1110_amd.binding import RtNet
from paper_0901_1110_amd.driver import LearnedSimulation, init_net_params
from tests.gpu_cases import host, newton_parity, rel

pytestmark = pytest.mark.gpu

W = synth.CFG_HHE
STEPS = 3
CUT, HALO = 16, 4


def block(a, c0, n):
    idx = [(np.arange(-HALO, CUT + HALO) + c) % n for c in c0]
    return a[..., idx[0][:, None, None], idx[1][None, :, None], idx[2][None, None, :]]


def inner(a):
    return a[..., HALO:HALO + CUT, HALO:HALO + CUT, HALO:HALO + CUT]


def learned_sim(w, s):
    net = RtNet(3, (w.n,) * 3)
    net.set_params(init_net_params(11, 5))
    return LearnedSimulation(w, net, state=s)


@pytest.fixture(scope="module")
def hhe512():
    s = synth.initial_state(W)
    sim = learned_sim(W, s)
    stats = []
    for k in range(STEPS):
        st = sim.step()
        stats.append(st)
        print("512^3 H+He step %d: status %d, Newton %d, CG %s, |f| %.2e -> %.2e, alt guess %d"
              % (k, st["status"], st["newton_its"], st["cg_its"], st["fnorms"][0],
                 st["fnorm_final"], st["used_alt_guess"]), flush=True)
        if k + 1 < STEPS:
            sim.advance()
    return s, sim, stats


def test_hhe512_steps_converge(hhe512):
    _, _, stats = hhe512
    for st in stats:
        assert st["status"] == 0, st
        assert st["fnorm_final"] < W.newton_tol


@pytest.mark.parametrize("c0", [None, (0, 0, 0), (300, 77, 491)])
def test_hhe512_sampled_blocks(hhe512, c0):
    """Time level and residual of the converged last step on sampled blocks;
    c0 = None puts the block around the first source."""
    s, sim, _ = hhe512
    n = W.n
    cells = s["src_cells"]
    ijk = np.stack(np.unravel_index(cells, (n, n, n)), axis=1)
    if c0 is None:
        c0 = tuple(int(v) - CUT // 2 for v in ijk[0])
    cos = W.cosmology(STEPS - 1)
    gn = sim.grid.rt_time_level(sim.Un, W.dt, cos)
    f, _ = sim.grid.rt_eval_residual(sim.U, gn, W.dt, cos)
    # blocks are cut on the device: the full 512^3 H+He fields stay there
    idx = [torch.from_numpy((np.arange(-HALO, CUT + HALO) + c) % n).cuda() for c in c0]

    def hb(t):
        return host(t[..., idx[0][:, None, None], idx[1][None, :, None], idx[2][None, None, :]])
    Un_b, U_b, eh_b, f_b, gn_b = hb(sim.Un), hb(sim.U), hb(sim.eh), hb(f), hb(gn)
    nH_b = block(s["nH"], c0, n)
    loc = (ijk - (np.array(c0) - HALO)) % n
    keep = np.all(loc < CUT + 2 * HALO, axis=1)
    nb = CUT + 2 * HALO
    bcells = np.ravel_multi_index(loc[keep].T, (nb, nb, nb)) if keep.any() else np.zeros(0, int)
    mb = oracle.model_from_workload(W.replace(n=nb))
    tl = ores.time_level(Un_b, nH_b, eh_b, bcells, s["src_Q"][keep], W.dt, cos, mb)
    f_o = ores.residual(U_b, tl, nH_b, eh_b, W.dt, cos[2], cos[3], mb)
    u = mb.scales
    for v in range(mb.nv):
        g_sc = max(np.max(np.abs(inner(tl["g"][v]))), 1e-300)
        assert rel(inner(gn_b[v]), inner(tl["g"][v]), g_sc) <= 1e-12, ("g", v)
        # the converged residual f = (U + dt theta L - g) / u is a small
        # difference of large terms: scale by the largest of them (g carries
        # the source injection, larger than E in the source cell)
        f_sc = max(np.max(np.abs(inner(U_b[v]))), np.max(np.abs(inner(tl["g"][v])))) / u[v]
        f_sc = max(f_sc, 1e-300)
        assert rel(inner(f_b[v]), inner(f_o[v]), f_sc) <= 1e-12, ("f", v)


def test_hhe64_rerun_against_fp64_oracle():
    """The 512^3 H+He recipe at 64^3: every GPU step (FP32 V-cycle, learned guess)
    meets the FP64 tolerance and stays within 1e-5 of the FP64 oracle."""
    w = W.replace(n=64, mg_levels=4)
    s = synth.initial_state(w)
    m = oracle.model_from_workload(w)
    sim = learned_sim(w, {k: (v.copy() if hasattr(v, "copy") else v) for k, v in s.items()})
    Un, eh = s["U"].copy(), s["eh"].copy()
    names = ["e_c", "x_HI", "x_HeI", "x_HeII", "E"]
    for k in range(STEPS):
        st = sim.step()
        assert st["status"] == 0 and st["fnorm_final"] < w.newton_tol, st
        U_o, st_o = onewt.newton_step(Un, Un, s["nH"], eh, s["src_cells"], s["src_Q"], w.dt,
                                      w.cosmology(k), m)
        assert st_o["status"] == 0
        U = host(sim.U)
        errs = [np.linalg.norm(U[v] - U_o[v]) / max(np.linalg.norm(U_o[v]), 1e-300)
                for v in range(5)]
        print("64^3 H+He step %d: " % k + ", ".join("%s %.2e" % (a, b) for a, b in zip(names, errs)),
              flush=True)
        for v in range(1, 5):
            assert errs[v] < 1e-5, (k, names[v], errs[v])
        # e_c is a correction around zero: compare against the total energy
        etot = np.linalg.norm(eh + U_o[0])
        assert np.linalg.norm(U[0] - U_o[0]) / etot < 1e-8
        sim.advance()
        eh = eh + U_o[0]
        U_o[0] = 0.0
        Un = U_o


def densest_block(s, n, b=64):
    """The b^3-aligned block of an n^3 state holding the most sources (the
    first such block in (i, j, k) order on a tie), as a state of its own with
    those sources; returns (state, block index, source count)."""
    ijk = np.stack(np.unravel_index(s["src_cells"], (n, n, n)), axis=1)
    blk = ijk // b
    keys, counts = np.unique(blk, axis=0, return_counts=True)
    best = keys[int(np.argmax(counts))]
    inside = np.all(blk == best, axis=1)
    sl = tuple(slice(int(c) * b, (int(c) + 1) * b) for c in best)
    loc = ijk[inside] - best * b
    sub = dict(U=np.ascontiguousarray(s["U"][(slice(None),) + sl]),
               nH=np.ascontiguousarray(s["nH"][sl]), eh=np.ascontiguousarray(s["eh"][sl]),
               src_cells=np.ravel_multi_index(loc.T, (b, b, b)).astype(np.int64),
               src_Q=s["src_Q"][inside].copy())
    return sub, tuple(int(c) for c in best), int(inside.sum())


SUB_STEPS = 50


def test_hhe512_densest_subvolume_rerun(hhe512):
    """The 512^3 H+He workload against the oracle on a 64^3 subvolume: the
    block of the initial state with the most sources, made periodic with
    them, for the workload's 50 steps.  FP64 library against the oracle:
    equal Newton and Krylov counts and line-search factors (a Krylov count
    within rounding of its stop test may differ by one, then the oracle
    replays the library's schedule), fields to 1e-10 (per element 1e-8).
    FP32 V-cycle with the learned guess (untrained network: the
    extrapolation base): every step meets the FP64 tolerance and its fields
    lie within 1e-5 (L2, relative) of the FP64 oracle's."""
    s, _, _ = hhe512
    sub, best, nsrc = densest_block(s, W.n)
    assert nsrc >= 2, (best, nsrc)
    w = W.replace(n=64, mg_levels=4, nsources=nsrc)
    ref = newton_parity(w.replace(mg_fp32=0), sub, steps=SUB_STEPS, keep=True)
    sim = learned_sim(w, {k: (v.copy() if hasattr(v, "copy") else v) for k, v in sub.items()})
    eh = sub["eh"].copy()
    names = ["e_c", "x_HI", "x_HeI", "x_HeII", "E"]
    worst = np.zeros(5)
    used = 0
    for k in range(SUB_STEPS):
        st = sim.step()
        assert st["status"] == 0 and st["fnorm_final"] < w.newton_tol, (k, st)
        used += st["used_alt_guess"]
        U_o = ref[k][2]
        U = host(sim.U)
        errs = [np.linalg.norm(U[v] - U_o[v]) / max(np.linalg.norm(U_o[v]), 1e-300)
                for v in range(5)]
        errs[0] = np.linalg.norm(U[0] - U_o[0]) / np.linalg.norm(eh + U_o[0])
        worst = np.maximum(worst, errs)
        for v in range(1, 5):
            assert errs[v] < 1e-5, (k, names[v], errs[v])
        # e_c is a correction around zero: compared against the total energy
        assert errs[0] < 1e-8, (k, errs[0])
        sim.advance()
        eh = eh + U_o[0]
    print("512^3 block %s (%d sources), %d steps: FP64 Newton its %d; mixed+learned worst "
          "per-field L2 %s, proposal taken in %d steps"
          % (best, nsrc, SUB_STEPS, sum(r[0]["newton_its"] for r in ref),
             ", ".join("%s %.1e" % (a, b) for a, b in zip(names, worst)), used), flush=True)
