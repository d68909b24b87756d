"""Multi-step driver: runs consecutive implicit steps of a workload on one GPU.

Between steps the energy correction is folded into the hydrodynamic energy
(Sec. 3.1: e^{n+1} = e_h + e_c, and e_c = 0 at the start of every step), the
expansion factor advances, and U^{n+1} becomes U^n.  All arithmetic runs in
the HIP library; this module only moves tensors and calls the C ABI.
"""
from __future__ import annotations

import numpy as np
import torch

import synth
from .binding import RtGrid, params_from_workload


class Simulation:
    def __init__(self, w: "synth.Workload", device="cuda", state=None, **overrides):
        self.w = w
        s = synth.initial_state(w) if state is None else state
        self.device = torch.device(device)
        self.grid = RtGrid(params_from_workload(w, **overrides), device=self.device)
        self.nH = torch.from_numpy(np.ascontiguousarray(s["nH"])).to(self.device)
        self.eh = torch.from_numpy(np.ascontiguousarray(s["eh"])).to(self.device)
        self.Un = torch.from_numpy(np.ascontiguousarray(s["U"])).to(self.device)
        self.U = self.Un.clone()
        self.grid.rt_set_medium(self.nH, self.eh)
        self.grid.rt_set_sources(s["src_cells"], s["src_Q"])
        self.step_index = 0

    def step(self, Ualt=None):
        """One implicit step from Un (guess: Un, or the better of Un and Ualt)."""
        c = self.w.cosmology(self.step_index)
        self.U.copy_(self.Un)
        st = self.grid.rt_newton_step(self.Un, self.U, self.w.dt, c, Ualt=Ualt)
        return st

    def advance(self):
        """Accept U as the new time level."""
        self.grid.rt_fold_energy(self.U, self.eh)
        self.Un, self.U = self.U, self.Un
        self.step_index += 1
