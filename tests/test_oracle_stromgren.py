"""Pin 2: Stromgren sphere of the isothermal HII-region test (Sec. 4.5).

At fixed T = 1e4 K the steady state of a point source in uniform hydrogen is
a sphere of radius r_S = (3 Q / (4 pi alpha_B n_H^2))^(1/3) (Sec. 4.5,
Eq. 63); the paper prints r_S = 5.4 kpc and t_rec = 1/(alpha_B n_H) =
3.86e15 s.  The oracle is driven to (near) steady state by one backward-Euler
step of length 1e21 s >> t_rec from the analytic sphere, then
  (a) the ionized volume's equivalent radius is within one cell of r_S,
  (b) every emitted photon is balanced by a recombination, up to the storage
      term of the finite step (exact discrete photon conservation).
"""
import json
import math
import os

import numpy as np
import pytest

import synth
import oracle
from oracle import newton, residual
from oracle.model import ALPHA_B_1E4, HNU_HI
from tests.oracle_cases import hii_workload

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "iliev_test1.json")))


def test_printed_constants():
    """The printed r_S and t_rec follow from the printed inputs."""
    Q, n, a = GOLD["N_gamma_photons_per_s"], GOLD["n_H_cm3"], GOLD["alpha_B_cm3_per_s"]
    rS = (3 * Q / (4 * math.pi * a * n * n)) ** (1 / 3) / synth.KPC_CM
    assert abs(rS - GOLD["r_S_kpc_printed"]) < 0.05
    t_rec = 1.0 / (a * n)
    assert abs(t_rec / GOLD["t_rec_s_printed"] - 1) < 2e-3
    assert abs(t_rec / 3.15576e13 - GOLD["t_rec_Myr_printed"]) < 0.1
    assert ALPHA_B_1E4 == a
    assert abs(HNU_HI / 1.602176634e-12 - GOLD["h_nu_eV"]) < 1e-12


@pytest.mark.parametrize("n", [16, 32])
def test_stromgren_steady_state(n):
    Q, nH0, aB = GOLD["N_gamma_photons_per_s"], GOLD["n_H_cm3"], GOLD["alpha_B_cm3_per_s"]
    rS = (3 * Q / (4 * math.pi * aB * nH0 * nH0)) ** (1 / 3)
    w = hii_workload(n, isothermal=1, newton_tol=1e-2, pcg_rtol=1e-12, newton_maxit=40)
    m = oracle.model_from_workload(w)
    s = synth.initial_state(w)
    x = (np.arange(n) + 0.5 - n / 2) * w.dx
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    U0 = s["U"].copy()
    U0[1] = np.where(np.sqrt(X ** 2 + Y ** 2 + Z ** 2) < rS, 1e-3, 0.9999)
    dt = 1e21
    # The radius and the photon balance of the steady state do not depend on
    # the diffusion coefficients (periodic diffusion telescopes out of the
    # photon count; the front is optically thick), so the steady state is
    # computed with the face coefficients held at their values for the
    # guess: one step of 1e21 s (~3e5 recombination times) with the limiter
    # of the iterate would ask Newton for a jump of 1e10 light-crossings of
    # a cell, which the method's own runs take in adaptive steps
    D0 = residual.limiter_at(U0, s["nH"], 1.0, m)
    U, st = newton.newton_step(U0, U0, s["nH"], s["eh"], s["src_cells"], s["src_Q"], dt,
                               (1.0, 0.0, 1.0, 0.0), m, D=D0)
    assert st["status"] == 0, st
    xh = 1.0 - U[1]
    h3 = w.dx ** 3
    V = np.count_nonzero(xh >= 0.5) * h3
    r_ion = (3 * V / (4 * math.pi)) ** (1 / 3)
    assert abs(r_ion - rS) <= w.dx, (r_ion / synth.KPC_CM, rS / synth.KPC_CM)
    nH = s["nH"]
    recomb = np.sum(aB * (nH * xh) ** 2) * h3
    # storage: change of photons + ions over the step, per unit time
    store = (np.sum(U[2] - U0[2]) / HNU_HI + np.sum(nH * (U0[1] - U[1]))) * h3 / dt
    assert abs(recomb / Q - 1) < 1e-5
    # exact discrete identity: the violation is bounded by the final residual
    tl = residual.time_level(U0, nH, s["eh"], s["src_cells"], s["src_Q"], dt,
                             (1.0, 0.0, 1.0, 0.0), m)
    f = residual.residual(U, tl, nH, s["eh"], dt, 1.0, 0.0, m, D=D0)
    bound = np.sum(m.u_E * np.abs(f[2]) / HNU_HI + nH * np.abs(f[1])) * h3 / dt
    assert abs(recomb + store - Q) <= bound + 1e-12 * Q, (recomb + store - Q, bound)
    assert bound < 1e-6 * Q
