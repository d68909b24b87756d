"""The expanding-universe I-front (Sec. 4.6, q0 = 0.5, z_i = 4) on the GPU.

Parity: the first steps at 16^3 equal the oracle's (counts, line-search
factors, fields to 1e-10).  Accuracy: at 64^3 the library's front follows
the paper's closed form r_I(t) within 1.5 % over 50 steps (z = 4 -> 1.08),
in FP64 and with the FP32 V-cycle.
"""
import time

import numpy as np
import pytest
import torch

import synth
from paper_0901_1110_amd.driver import Simulation
from tests.gpu_cases import host
from tests.sg_closed_form import front_radius, ionized_radius
from tests.gpu_cases import newton_parity
from tests.test_oracle_shapiro_giroux import SG, sg_constants

pytestmark = pytest.mark.gpu


def test_sg_steps_parity():
    w = synth.CFG_SG.replace(n=16, dx=synth.CFG_SG.dx * 8, mg_levels=3)
    newton_parity(w, synth.initial_state(w), steps=3)


@pytest.mark.parametrize("mg_fp32", [0, 1])
def test_sg_front_64(mg_fp32):
    w = synth.CFG_SG.replace(n=64, dx=synth.CFG_SG.dx * 2, mg_levels=4)
    _, _, rS, lam = sg_constants(w)
    sim = Simulation(w, mg_fp32=mg_fp32)
    worst = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(w.steps):
        st = sim.step()
        assert st["status"] == 0, (k, st)
        sim.advance()
        a_rel = w.cosmology(k)[2] / w.a_start
        r = ionized_radius(host(sim.Un[1]), w.dx, w.a_start)
        worst = max(worst, abs(r / rS / front_radius(a_rel, lam, SG["q0"], SG["z_i"]) - 1.0))
    dt = time.perf_counter() - t0
    print("64^3 mg_fp32=%d: %d steps in %.2f s (with read-back), worst front error %.4f"
          % (mg_fp32, w.steps, dt, worst))
    assert worst < 0.015, worst
