"""Pins of the LTE coupling (Sec. 2.1, Eq. 9) on the matter-radiation
equilibration test of Sec. 4.2 (fixture tests/golden/turner_stone.json).

- The printed derived values follow from the printed inputs and the
  constants used (radiation constant, T_r, the two gas temperatures, the
  heat capacities).
- On the uniform 4^3 medium diffusion vanishes and a backward Euler step
  reduces to one scalar equation: total energy rho e + E is unchanged, so
  E_1 = E_0 - rho (e_1 - e_0) and rho (e_1 - e_0) = dt c kappa (E_1 - a_r T(e_1)^4)
  (kappa_P = kappa).  Its root, by bracketing, equals the oracle's full
  Newton / Schur / MG-PCG step for the first steps of both starts.
- Over the 250 steps to t = 2.5e-7 s total energy is conserved to 1e-12
  (the paper's Table 1 reports 3e-13 .. 4e-11 for its tolerances), both
  starts reach e_eq of Eq. 48 evaluated at the final E to 1e-6, monotonically,
  and the printed constant-E estimate of e_eq to 0.5 %.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq

import synth
import oracle
from oracle import newton as onewt
from oracle.model import A_RAD, C_LIGHT, GAMMA, K_B, M_H

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "turner_stone.json")))
RHO, KAP, MU = GOLD["rho_g_cm3"], GOLD["kappa_per_cm"], GOLD["mu_in_m_H"]


def temperature(e_spec):
    return (GAMMA - 1.0) * MU * M_H * e_spec / K_B


def e_eq(E):
    """Eq. 48 (volumetric gas energy at the radiation temperature of E)."""
    return 1.5 * (RHO * K_B / (MU * M_H)) * (E / A_RAD) ** 0.25


def test_printed_derived_values():
    E = GOLD["E_erg_cm3"]
    assert A_RAD == pytest.approx(GOLD["a_r_printed"], rel=1e-3)
    Tr = (E / A_RAD) ** 0.25
    assert Tr == pytest.approx(GOLD["T_r_K_about"], rel=0.01)
    assert temperature(GOLD["e_hot_erg_cm3"] / RHO) == pytest.approx(GOLD["T_hot_K_roughly"], rel=0.02)
    assert temperature(GOLD["e_cold_erg_cm3"] / RHO) == pytest.approx(GOLD["T_cold_K_roughly"], rel=0.02)
    assert A_RAD * Tr ** 3 == pytest.approx(GOLD["radiation_heat_capacity_erg_K_roughly"], rel=0.02)
    cv = K_B / ((GAMMA - 1.0) * MU * M_H)
    assert cv == pytest.approx(GOLD["gas_specific_heat_erg_g_K_roughly"], rel=0.05)
    assert RHO * cv == pytest.approx(GOLD["gas_heat_capacity_erg_K"], rel=0.05)


def test_workloads_match_printed_case():
    for w, e in ((synth.CFG_TS_HOT, GOLD["e_hot_erg_cm3"]), (synth.CFG_TS_COLD, GOLD["e_cold_erg_cm3"])):
        assert w.lte == 1 and w.nspecies == 0 and w.n == GOLD["zones"]
        assert w.kappa_lte == KAP and w.kappaP_lte == KAP and w.mu_lte == MU
        assert w.nH_mean * M_H == pytest.approx(RHO, rel=1e-15)
        assert w.E0 == GOLD["E_erg_cm3"] and w.eh0 * RHO == pytest.approx(e, rel=1e-15)
        assert w.dt * w.steps == pytest.approx(GOLD["t_final_s"], rel=1e-12)


def scalar_step(e0, E0, dt):
    """Backward Euler of the uniform closed system (see module docstring)."""
    def F(e1):
        E1 = E0 - RHO * (e1 - e0)
        return RHO * (e1 - e0) - dt * C_LIGHT * KAP * (E1 - A_RAD * temperature(e1) ** 4)
    hi = e0 + E0 / RHO
    e1 = brentq(F, 1e-30, hi, xtol=1e-300, rtol=1e-15, maxiter=500)
    return e1, E0 - RHO * (e1 - e0)


def run(w, steps):
    m = oracle.model_from_workload(w)
    s = synth.initial_state(w)
    U, eh = s["U"].copy(), s["eh"].copy()
    out = []
    for k in range(steps):
        U1, st = onewt.newton_step(U, U, s["nH"], eh, s["src_cells"], s["src_Q"], w.dt,
                                   w.cosmology(k), m)
        assert st["status"] == 0, (k, st)
        eh = eh + U1[0]
        U1[0] = 0.0
        U = U1
        out.append((float(np.mean(eh)), float(np.mean(U[-1])), float(np.ptp(eh)), float(np.ptp(U[-1]))))
    return s, out


@pytest.mark.parametrize("w", [synth.CFG_TS_HOT, synth.CFG_TS_COLD], ids=["hot", "cold"])
def test_steps_equal_scalar_root(w):
    _, out = run(w, 3)
    e, E = w.eh0, w.E0
    for k in range(3):
        e, E = scalar_step(e, E, w.dt)
        assert out[k][2] == 0.0 and out[k][3] == 0.0      # stays uniform
        assert out[k][0] == pytest.approx(e, rel=1e-9), k
        assert out[k][1] == pytest.approx(E, rel=1e-12), k


@pytest.mark.parametrize("w", [synth.CFG_TS_HOT, synth.CFG_TS_COLD], ids=["hot", "cold"])
def test_equilibrium_and_conservation(w):
    s, out = run(w, w.steps)
    tot0 = RHO * w.eh0 + w.E0
    e_end, E_end = out[-1][0] * RHO, out[-1][1]
    assert abs(e_end + E_end - tot0) / tot0 <= 1e-12
    assert e_end == pytest.approx(e_eq(E_end), rel=1e-6)
    assert e_end == pytest.approx(e_eq(GOLD["E_erg_cm3"]), rel=5e-3)
    es = [o[0] for o in out]
    d = np.diff(es)
    assert np.all(d <= 1e-12 * es[0]) if w.eh0 * RHO > e_end else np.all(d >= -1e-12 * es[-1])
