"""Full-size (256^3) checks in the configuration the benchmark times.

At 256^3 the oracle checks sampled outputs: every residual / Schur value is
cell-local given its 1-cell neighbourhood (and the time-level coefficients
given theirs), so a 24^3 block cut around sampled cells, evaluated by the
oracle with any wrap, is exact on its 16^3 interior.  The converged Newton
step is checked through properties that hold at any size: the oracle's own
residual of the GPU result is below the Newton tolerance, and photons plus
ions are conserved up to emission, recombination and that residual.
"""
import numpy as np
import pytest
import torch

import synth
import oracle
from oracle import jacobian as ojac
from oracle import residual as ores
from oracle.model import HNU_HI
from oracle.physics import recombination_coefficients, temperature
from paper_0901_1110_amd.driver import Simulation
from tests.gpu_cases import host, rel

pytestmark = pytest.mark.gpu

W = synth.CFG_256
CUT, HALO = 16, 4


def block(a, c0):
    """Block of size CUT + 2*HALO starting at corner c0 - HALO (periodic)."""
    n = a.shape[-1]
    idx = [(np.arange(-HALO, CUT + HALO) + c) % n for c in c0]
    return a[..., idx[0][:, None, None], idx[1][None, :, None], idx[2][None, None, :]]


def inner(a):
    return a[..., HALO:HALO + CUT, HALO:HALO + CUT, HALO:HALO + CUT]


@pytest.fixture(scope="module")
def full():
    s = synth.initial_state(W)
    sim = Simulation(W, state={k: (v.copy() if hasattr(v, "copy") else v) for k, v in s.items()})
    st0 = sim.step()          # first step: a non-trivial state to start from
    assert st0["status"] == 0
    sim.advance()
    return s, sim


CORNERS = [(120, 120, 120), (0, 0, 0), (240, 17, 129)]


@pytest.mark.parametrize("c0", CORNERS)
def test_residual_and_schur_sampled_blocks(full, c0):
    s, sim = full
    m = oracle.model_from_workload(W)
    Un = host(sim.Un)
    eh = host(sim.eh)
    nH = s["nH"]
    cos = W.cosmology(1)
    # a perturbed iterate: U^n with E raised by 30 % and fractions nudged
    U = Un.copy()
    U[2] *= 1.3
    U[1] = np.clip(U[1] * 0.99, 0, 1)
    Ud = torch.from_numpy(U).cuda()
    gn = sim.grid.rt_time_level(sim.Un, W.dt, cos)
    f, _ = sim.grid.rt_eval_residual(Ud, gn, W.dt, cos)
    b = sim.grid.rt_schur_form(Ud, f, W.dt, cos)
    sch = {k: host(v) for k, v in sim.grid.rt_schur_get().items()}
    full = {k: host(v) for k, v in sim.grid.rt_schur_get_full().items()}
    sch["pdiag"] = full["pdiag"]
    for d, ax in enumerate("xyz"):
        sch["f" + ax], sch["b" + ax] = full["fw"][d], full["bw"][d]
    f, gn, b = host(f), host(gn), host(b)
    # oracle on the block; sources inside the block keep their offsets
    n = W.n
    cells = s["src_cells"]
    ijk = np.stack(np.unravel_index(cells, (n, n, n)), axis=1)
    loc = (ijk - (np.array(c0) - HALO)) % n
    keep = np.all(loc < CUT + 2 * HALO, axis=1)
    nb = CUT + 2 * HALO
    bcells = np.ravel_multi_index(loc[keep].T, (nb, nb, nb)) if keep.any() else np.zeros(0, int)
    mb = oracle.model_from_workload(W.replace(n=nb))
    tl = ores.time_level(block(Un, c0), block(nH, c0), block(eh, c0), bcells, s["src_Q"][keep],
                         W.dt, cos, mb)
    f_o = ores.residual(block(U, c0), tl, block(nH, c0), block(eh, c0), W.dt, cos[2], cos[3], mb)
    # the Schur set-up is compared on the same residual input (the GPU's)
    so = ojac.schur_form(block(U, c0), block(f, c0), block(nH, c0), block(eh, c0), W.dt,
                         cos[2], cos[3], mb)
    u = m.scales
    for v in range(3):
        sc = max(np.max(np.abs(inner(f_o[v]))), np.max(np.abs(inner(block(U, c0)[v]))) / u[v], 1e-300)
        assert rel(inner(block(f, c0)[v]), inner(f_o[v]), sc) <= 1e-12, v
        assert rel(inner(block(gn, c0)[v]), inner(tl["g"][v]),
                   max(np.max(np.abs(inner(tl["g"][v]))), 1e-300)) <= 1e-13
    scale = max(np.max(np.abs(inner(so["diag"]))), np.max(np.abs(inner(so["pdiag"]))))
    for k in ("diag", "cx", "cy", "cz", "pdiag", "fx", "fy", "fz", "bx", "by", "bz"):
        assert rel(inner(block(sch[k], c0)), inner(so[k]), scale) <= 1e-12, k
    for r in range(2):
        assert rel(inner(block(sch["ftM"][r], c0)), inner(so["ftM"][r])) <= 1e-12
        assert rel(inner(block(sch["W"][r], c0)), inner(so["W"][r])) <= 1e-12
    assert rel(inner(block(b, c0)), inner(so["b"])) <= 1e-12


# the benchmark's default preconditioner: the 32^3 subdomain correction with
# a two-level box V-cycle (4 coarsest sweeps) and 20 inner iterations, and
# the inexact-Newton forcing 1e-6
BENCH = dict(box_size=32, box_levels=2, box_inner=20, box_coarse_sweeps=4, pcg_forcing=1e-6)


# far more inner iterations than the FP32 box solve can use: its residual
# vanishes and the fixed-count iteration must stand still, not divide 0 by 0
MANY_INNER = dict(BENCH, box_inner=40)


@pytest.mark.parametrize("mg_fp32,over", [(0, {}), (1, {}), (0, BENCH), (1, BENCH), (1, MANY_INNER)])
def test_full_step_properties(full, mg_fp32, over):
    s, sim0 = full
    # start from the state after one step (shared fixture), run one more step
    st_in = dict(U=host(sim0.Un), nH=s["nH"], eh=host(sim0.eh), src_cells=s["src_cells"],
                 src_Q=s["src_Q"])
    sim = Simulation(W.replace(**over),
                     state={k: (v.copy() if hasattr(v, "copy") else v) for k, v in st_in.items()},
                     mg_fp32=mg_fp32)
    sim.step_index = 1
    st = sim.step()
    assert st["status"] == 0 and st["fnorm_final"] < W.newton_tol
    m = oracle.model_from_workload(W)
    U = host(sim.U)
    Un, eh, nH = st_in["U"], st_in["eh"], s["nH"]
    tl = ores.time_level(Un, nH, eh, s["src_cells"], s["src_Q"], W.dt, W.cosmology(1), m)
    f = ores.residual(U, tl, nH, eh, W.dt, 1.0, 0.0, m)
    fn = ores.rms(f)
    assert fn < W.newton_tol
    # the residual is a difference of terms up to ~1e5 (scaled), so both
    # norms carry rounding noise of ~1e-10; above that floor they agree
    assert abs(fn - st["fnorm_final"]) <= 1e-3 * st["fnorm_final"] + 1e-9
    # photon-number balance over the step (theta = 1, a = 1)
    h3 = W.dx ** 3

    def recomb(V):
        T = temperature(eh + V[0], V[1], 0.0, 0.0, m)
        return np.sum(recombination_coefficients(T)[0] * (nH * (1 - V[1])) ** 2) * h3

    def count(V):
        return (np.sum(V[2]) / HNU_HI + np.sum(nH * (1 - V[1]))) * h3

    Q = float(np.sum(s["src_Q"]))
    lhs = count(U) - count(Un)
    rhs = W.dt * (Q - recomb(U))
    bound = np.sum(m.u_E * np.abs(f[2]) / HNU_HI + nH * np.abs(f[1])) * h3
    slack = 1e-15 * np.sum(nH) * h3 + 1e-13 * W.dt * Q
    assert abs(lhs - rhs) <= bound + slack
