"""The x-left Dirichlet face (boundary = 2) through the C ABI: per-call parity
on random states, the first free-streaming steps (Sec. 4.1) against the
oracle, and the 128^3 front, which follows c t with a lag that shrinks with
the step."""
import time

import numpy as np
import pytest
import torch

import synth
import oracle
from oracle import jacobian as ojac
from oracle import residual as ores
from oracle.model import C_LIGHT
from paper_0901_1110_amd.driver import Simulation
from tests.gpu_cases import dev, host, pair, random_case, rel
from tests.gpu_cases import newton_parity

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ns,seed", [(1, 41), (3, 42)])
def test_calls_dirichlet(ns, seed):
    w, c = random_case(ns, 16, 1.0, 1.0, seed, boundary=2, E_dirichlet=3e-16)
    m, g = pair(w, c)
    cos = c["cosmo"]
    tl = ores.time_level(c["Un"], c["nH"], c["eh"], c["cells"], c["Q"], c["dt"], cos, m)
    f_o = ores.residual(c["U"], tl, c["nH"], c["eh"], c["dt"], cos[2], cos[3], m)
    gn = g.rt_time_level(dev(c["Un"]), c["dt"], cos)
    f, rms = g.rt_eval_residual(dev(c["U"]), gn, c["dt"], cos)
    f = host(f)
    for v in range(m.nv):
        s = max(float(np.max(np.abs(f_o[v]))), float(np.max(np.abs(c["U"][v] / m.scales[v]))),
                float(np.max(np.abs(tl["g"][v] / m.scales[v]))))
        assert rel(f[v], f_o[v], s) <= 1e-12, v
    sch = ojac.schur_form(c["U"], f_o, c["nH"], c["eh"], c["dt"], cos[2], cos[3], m)
    b = host(g.rt_schur_form(dev(c["U"]), dev(f_o), c["dt"], cos))
    got = {k: host(v) for k, v in g.rt_schur_get().items()}
    got.update({k: host(v) for k, v in g.rt_schur_get_full().items()})
    scale = max(float(np.max(np.abs(sch["diag"]))), float(np.max(np.abs(sch["pdiag"]))))
    for k in ("diag", "cx", "cy", "cz", "pdiag"):
        assert rel(got[k], sch[k], scale) <= 1e-12, k
    for d, ax in enumerate("xyz"):
        assert rel(got["fw"][d], sch["f" + ax], scale) <= 1e-12, ax
        assert rel(got["bw"][d], sch["b" + ax], scale) <= 1e-12, ax
    assert rel(b, sch["b"]) <= 1e-12


def test_free_stream_steps_parity():
    w = synth.CFG_FS.replace(n=16, dx=1.0 / 16, mg_levels=3, steps=50, dt=8.3391e-12 / 50)
    newton_parity(w, synth.initial_state(w), steps=3)


def front(E):
    prof = E.mean(axis=(1, 2))
    n = E.shape[0]
    x = (np.arange(n) + 0.5) / n
    i = int(np.argmax(prof < 0.5))
    return x[i - 1] + (0.5 - prof[i - 1]) * (x[i] - x[i - 1]) / (prof[i] - prof[i - 1]), prof


def test_front_128():
    fronts = {}
    for steps in (100, 400):
        w = synth.CFG_FS.replace(steps=steps, dt=8.3391e-12 / steps)
        sim = Simulation(w)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            st = sim.step()
            assert st["status"] == 0, st
            sim.advance()
        torch.cuda.synchronize()
        E = host(sim.Un[1])
        xf, prof = front(E)
        fronts[steps] = xf
        print("128^3, %d steps: front %.4f cm (c t = 0.25), %.1f ms/step"
              % (steps, xf, 1e3 * (time.perf_counter() - t0) / steps))
        assert E.max() <= 1.0 + 1e-12
        assert np.ptp(E, axis=(1, 2)).max() <= 1e-9
    ct = C_LIGHT * 8.3391e-12
    assert 0.2 < fronts[100] < ct + 0.005
    assert fronts[100] - 1e-3 <= fronts[400] < ct + 0.005
