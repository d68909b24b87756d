"""The expanding lognormal medium at full size: 128^3 periodic hydrogen,
lognormal n_H (sigma_ln = 1, P(k) ~ k^-2), 16 sources with log-uniform Q,
a = 0.1 with the Hubble terms, 20 steps of the plain FP64 method.

The first step is compared with the FP64 oracle's own Newton step at full
size, field by field.  Every step must converge, and the last one is checked
through the oracle's residual of the GPU result, which holds at any size.
"""
import numpy as np
import pytest

import synth
import oracle
from oracle import newton as onewt
from oracle import residual as ores
from paper_0901_1110_amd.driver import Simulation
from tests.gpu_cases import host, rel

pytestmark = pytest.mark.gpu

W = synth.CFG_COSMO


@pytest.fixture(scope="module")
def run():
    s = synth.initial_state(W)
    sim = Simulation(W, state={k: (v.copy() if hasattr(v, "copy") else v) for k, v in s.items()})
    stats, first = [], None
    for k in range(W.steps):
        st = sim.step()
        stats.append(st)
        if k == 0:
            first = host(sim.U)
        if k + 1 < W.steps:
            sim.advance()
    return s, sim, stats, first


def test_every_step_converges(run):
    _, _, stats, _ = run
    for k, st in enumerate(stats):
        assert st["status"] == 0 and st["fnorm_final"] < W.newton_tol, (k, st)


def test_first_step_equals_oracle(run):
    s, _, stats, first = run
    m = oracle.model_from_workload(W)
    U_o, st_o = onewt.newton_step(s["U"], s["U"], s["nH"], s["eh"], s["src_cells"], s["src_Q"],
                                  W.dt, W.cosmology(0), m)
    assert st_o["status"] == 0
    assert stats[0]["newton_its"] == st_o["newton_its"]
    for v in range(m.nv):
        assert rel(first[v], U_o[v]) <= 1e-10, v


def test_last_step_oracle_residual(run):
    s, sim, stats, _ = run
    m = oracle.model_from_workload(W)
    k = W.steps - 1
    cos = W.cosmology(k)
    Un, eh, U = host(sim.Un), host(sim.eh), host(sim.U)
    tl = ores.time_level(Un, s["nH"], eh, s["src_cells"], s["src_Q"], W.dt, cos, m)
    f = ores.residual(U, tl, s["nH"], eh, W.dt, cos[2], cos[3], m)
    fn = ores.rms(f)
    assert fn < W.newton_tol
    assert abs(fn - stats[-1]["fnorm_final"]) <= 1e-3 * stats[-1]["fnorm_final"] + 1e-9
