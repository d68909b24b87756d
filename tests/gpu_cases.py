"""Helpers for the GPU parity tests: the same seeded inputs go to the oracle and
to the HIP library, and results are compared array by array."""
from __future__ import annotations

import numpy as np
import torch

import synth
import oracle
from paper_0901_1110_amd.binding import RtGrid, params_from_workload


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b, scale=None):
    """max |a - b| / scale (scale defaults to max |b|)."""
    s = np.max(np.abs(b)) if scale is None else scale
    return float(np.max(np.abs(a - b)) / (s if s > 0 else 1.0))


def rel_elem(a, b, floor):
    """Per element: max over cells of |a - b| / max(|b|, floor).  Unlike rel()
    this checks every cell on its own scale down to `floor` (a radiation
    background decades below the source cell, a nearly ionized fraction)."""
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), floor)))


# per-variable floors of rel_elem for a state (e_c, x_1..x_Ns, E): e_c is a
# correction that may vanish (floor 1e-6 of its unit), fractions are checked
# relative down to 1e-12, radiation relative down to 1e-10 of its unit
def state_floors(m):
    return [1e-6 * m.u_e] + [1e-12] * m.nspecies + [1e-10 * m.u_E]


def workload(ns, n, theta=1.0, a=1.0, levels=2, **kw):
    """Random-state cases: the limiter at the iterate unless kw asks for the
    lagged reading."""
    base = synth.CFG_SMALL if ns == 1 else synth.CFG_HHE
    kw.setdefault("limiter_lag", 0)
    w = base.replace(n=n, theta=theta, mg_levels=levels, a_start=a, a_end=None,
                     u_E=1e-20 * a ** 3, E0=1e-20 * a ** 3, nH_mean=1e-3 * a ** 3, **kw)
    return w


def random_case(ns, n, theta, a, seed, levels=2, **kw):
    """Random physical state, an independent random U^n, a few sources."""
    w = workload(ns, n, theta, a, levels, **kw)
    rng = np.random.default_rng(seed)
    U, nH, eh = synth.random_physical_state(n, ns, rng, nH_mean=1e-3 * a ** 3)
    U[-1] *= a ** 3
    Un, _, _ = synth.random_physical_state(n, ns, rng, nH_mean=1e-3 * a ** 3)
    Un[-1] *= a ** 3
    Un[0] = 0.0
    cells = rng.choice(n ** 3, 3, replace=False).astype(np.int64)
    Q = 10 ** rng.uniform(47, 49, 3)
    H = 0.0 if a == 1.0 else synth.eds_hubble(a)
    cosmo = (a, H, a, H)
    dt = 1e11 if a == 1.0 else 5e12
    return w, dict(U=U, Un=Un, nH=nH, eh=eh, cells=cells, Q=Q, cosmo=cosmo, dt=dt)


def newton_parity(w, state, steps=1, tol_fields=1e-10, tol_elem=1e-8, keep=False):
    """Run `steps` implicit steps on both sides from the same state and
    compare each.  The oracle runs with its own decisions: Newton count and
    line search factors must equal the library's, and so must the Krylov
    counts, except where a Krylov stop test falls within rounding of its
    threshold: then a count may differ by one (at most two such flips per
    step), and the library's step is compared with the oracle replaying the
    library's schedule (replay mode: its Krylov counts and lambdas), so that
    the comparison stays iterate for iterate.  Fields: normwise to
    tol_fields and per element (state_floors) to tol_elem.  keep: the
    entries also carry the oracle's new state of the step."""
    from oracle import newton as onewt
    from paper_0901_1110_amd.driver import Simulation
    m = oracle.model_from_workload(w)
    sim = Simulation(w, state={k: v.copy() if hasattr(v, "copy") else v
                               for k, v in state.items()})
    Un, eh = state["U"].copy(), state["eh"].copy()
    floors = state_floors(m)
    out = []
    for n in range(steps):
        cos = w.cosmology(n)
        U_o, st_o = onewt.newton_step(Un, Un, state["nH"], eh, state["src_cells"],
                                      state["src_Q"], w.dt, cos, m)
        st = sim.step()
        assert st["status"] == 0 and st_o["status"] == 0, (st, st_o)
        assert st["newton_its"] == st_o["newton_its"], (st, st_o)
        assert st["lambdas"] == st_o["lambdas"], (st, st_o)
        if st["cg_its"] != st_o["cg_its"]:
            flips = [abs(x - y) for x, y in zip(st["cg_its"], st_o["cg_its"])]
            assert max(flips) <= 1 and sum(flips) <= 2, (st, st_o)
            U_o, st_r = onewt.newton_step(Un, Un, state["nH"], eh, state["src_cells"],
                                          state["src_Q"], w.dt, cos, m,
                                          replay=dict(its=st["cg_its"], lambdas=st["lambdas"]))
            assert st_r["fnorms"][-1] < w.newton_tol, st_r
        U = host(sim.U)
        for v in range(m.nv):
            assert rel(U[v], U_o[v]) <= tol_fields, (n, v, rel(U[v], U_o[v]))
            e = rel_elem(U[v], U_o[v], floors[v])
            assert e <= tol_elem, (n, v, e)
        out.append((st, st_o, U_o.copy()) if keep else (st, st_o))
        sim.advance()
        eh = eh + U_o[0]
        U_o[0] = 0.0
        Un = U_o
    return out


def replay_parity(w, state, steps=1, tol_fields=1e-10, tol_elem=1e-8):
    """As newton_parity, with the oracle in replay mode (the library's Krylov
    counts and lambdas): the comparison is iterate for iterate even where a
    stop test lies within rounding of its threshold.  Returns the list of
    (library stats, oracle's own stats) and the per-field errors."""
    from oracle import newton as onewt
    from paper_0901_1110_amd.driver import Simulation
    m = oracle.model_from_workload(w)
    sim = Simulation(w, state={k: v.copy() if hasattr(v, "copy") else v
                               for k, v in state.items()})
    Un, eh = state["U"].copy(), state["eh"].copy()
    floors = state_floors(m)
    out = []
    for n in range(steps):
        cos = w.cosmology(n)
        st = sim.step()
        assert st["status"] == 0, st
        U_r, st_r = onewt.newton_step(Un, Un, state["nH"], eh, state["src_cells"],
                                      state["src_Q"], w.dt, cos, m,
                                      replay=dict(its=st["cg_its"], lambdas=st["lambdas"]))
        assert st_r["fnorms"][-1] < w.newton_tol, st_r
        U = host(sim.U)
        errs = []
        for v in range(m.nv):
            errs.append((rel(U[v], U_r[v]), rel_elem(U[v], U_r[v], floors[v])))
            assert errs[-1][0] <= tol_fields and errs[-1][1] <= tol_elem, (n, v, errs[-1])
        out.append((st, st_r, errs))
        sim.advance()
        eh = eh + U_r[0]
        U_r[0] = 0.0
        Un = U_r
    return out


def pair(w, case, **over):
    """(oracle model, GPU grid with medium and sources set)."""
    m = oracle.model_from_workload(w, **{k: v for k, v in over.items() if k != "mg_fp32"})
    if "mg_fp32" in over:
        m.mg_fp32 = over["mg_fp32"]
    g = RtGrid(params_from_workload(w, **over))
    d = dict(nH=dev(case["nH"]), eh=dev(case["eh"]))
    g.rt_set_medium(d["nH"], d["eh"])
    g.rt_set_sources(case["cells"], case["Q"])
    g._cells = case["cells"]
    g._dev = d
    return m, g
