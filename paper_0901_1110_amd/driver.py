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
        self.nH_mean = float(np.mean(s["nH"]))
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


class AdaptiveSimulation(Simulation):
    """Steps of adaptive length (Sec. 3.2.3): the explicit predictor is
    offered as the Newton guess, the time-error estimate between the new
    state and the predictor sets the next step, dt <- min(tau dt / eps,
    dt_max); a step whose Newton iteration fails is retried at half length."""

    def __init__(self, w, tau, p=0.0, dt_max=None, device="cuda", state=None, **overrides):
        super().__init__(w, device=device, state=state, **overrides)
        self.tau, self.p = float(tau), float(p)
        self.dt = float(w.dt)
        self.dt_max = float(dt_max) if dt_max is not None else 1.0e3 * self.dt
        self.t = 0.0
        self.Up = self.grid.new_state()
        self.eps = None

    def step(self, Ualt=None, max_halvings=10):
        for _ in range(max_halvings + 1):
            c = self.w.cosmology_at(self.t, self.dt)
            self.grid.rt_predict(self.Un, self.dt, c, self.Up)
            self.U.copy_(self.Un)
            st = self.grid.rt_newton_step(self.Un, self.U, self.dt, c, Ualt=self.Up)
            st["dt"] = self.dt
            if st["status"] == 0:
                self.eps = self.grid.rt_time_error(self.U, self.Up, self.p)
                st["eps"] = self.eps
                return st
            self.dt *= 0.5
        return st

    def advance(self):
        self.grid.rt_fold_energy(self.U, self.eh)
        self.Un, self.U = self.U, self.Un
        self.step_index += 1
        self.t += self.dt
        eps = self.eps
        self.dt = self.dt_max if not eps > 0.0 else min(self.tau * self.dt / eps, self.dt_max)


class LearnedSimulation(Simulation):
    """Simulation whose Newton guess is the better (by initial residual) of
    U^n and the network's proposal from levels n and n-1."""

    def __init__(self, w, net, device="cuda", state=None, **overrides):
        super().__init__(w, device=device, state=state, **overrides)
        self.net = net
        self.Unm1 = None
        self.ehm1 = None
        self.Uguess = torch.empty_like(self.Un)

    def step(self):
        c = self.w.cosmology(self.step_index)
        self.U.copy_(self.Un)
        Ualt = None
        if self.Unm1 is not None:
            self.net.forward(self.Un, self.Unm1, self.eh, self.ehm1, self.nH, self.nH_mean,
                             self.w.u_e, self.w.u_E, self.eh, self.Uguess)
            Ualt = self.Uguess
        return self.grid.rt_newton_step(self.Un, self.U, self.w.dt, c, Ualt=Ualt)

    def advance(self):
        if self.Unm1 is None:
            self.Unm1 = torch.empty_like(self.Un)
            self.ehm1 = torch.empty_like(self.eh)
        # level n becomes level n - 1 by rotating the three state buffers (U
        # is overwritten by the next step's guess anyway); e_h is updated in
        # place, so its old value is copied
        self.ehm1.copy_(self.eh)
        self.grid.rt_fold_energy(self.U, self.eh)
        self.Unm1, self.Un, self.U = self.Un, self.U, self.Unm1
        self.step_index += 1


def generate_trajectory(w, steps, device="cuda", state=None, **overrides):
    """Run the plain method for `steps` steps; keep every level on the device.

    Returns dict(U=[U^0..U^T], e=[e^0..e^T], nH, nH_mean, stats) where e^n is
    the total specific gas energy of level n.
    """
    sim = Simulation(w, device=device, state=state, **overrides)
    Us, es, stats = [sim.Un.clone()], [sim.eh.clone()], []
    for _ in range(steps):
        st = sim.step()
        if st["status"] != 0:
            raise RuntimeError("trajectory step %d failed: %s" % (sim.step_index, st))
        stats.append(st)
        sim.advance()
        Us.append(sim.Un.clone())
        es.append(sim.eh.clone())
    return dict(U=Us, e=es, nH=sim.nH, nH_mean=sim.nH_mean, stats=stats, u_e=w.u_e, u_E=w.u_E,
                grid=sim.grid, dt=w.dt, cosmology=w.cosmology)


def guess_score(net, trajectories, grids, every=1, first=2):
    """Mean log10 of ||f(network guess)|| / ||f(U^n)|| over every `every`-th
    sample from level `first` on (the first levels follow the start-up
    transient of a cold box, where no extrapolation holds): the Newton
    initial residual the guess would save (negative is better than the
    previous-state guess)."""
    tot, cnt = 0.0, 0
    for T, g in zip(trajectories, grids):
        Ug = torch.empty_like(T["U"][0])
        for n in range(max(1, first), len(T["U"]) - 1, every):
            g.rt_set_medium(T["nH"], T["e"][n])
            c = T["cosmology"](n)
            gn = g.rt_time_level(T["U"][n], T["dt"], c)
            net.forward(T["U"][n], T["U"][n - 1], T["e"][n], T["e"][n - 1], T["nH"], T["nH_mean"],
                        T["u_e"], T["u_E"], T["e"][n], Ug)
            _, fg = g.rt_eval_residual(Ug, gn, T["dt"], c)
            _, fp = g.rt_eval_residual(T["U"][n], gn, T["dt"], c)
            tot += float(np.log10(max(fg, 1e-300) / max(fp, 1e-300)))
            cnt += 1
    return tot / max(cnt, 1)


def train_net(net, trajectories, epochs, lr=3e-4, seed=0, log=None, select=True):
    """Adam on every (n-1, n -> n+1) sample of the trajectories, shuffled per
    epoch.  With select=True the parameters kept are those (including the
    starting ones) with the best guess_score on the trajectories."""
    samples = [(t, n) for t in range(len(trajectories))
               for n in range(1, len(trajectories[t]["U"]) - 1)]
    rng = np.random.default_rng(seed)
    history = []
    grids = [T["grid"] for T in trajectories] if select else None
    best = (guess_score(net, trajectories, grids), net.get_params()) if select else None
    if log and select:
        log("start: guess score %.4f" % best[0])
    for ep in range(epochs):
        order = rng.permutation(len(samples))
        tot = 0.0
        for idx in order:
            t, n = samples[idx]
            T = trajectories[t]
            loss = net.train_step(T["U"][n], T["U"][n - 1], T["e"][n], T["e"][n - 1], T["nH"],
                                  T["nH_mean"], T["u_e"], T["u_E"], T["U"][n + 1], T["e"][n + 1], lr)
            tot += loss
        history.append(tot / max(1, len(samples)))
        msg = "epoch %d: mean loss %.4e" % (ep, history[-1])
        if select:
            sc = guess_score(net, trajectories, grids)
            msg += ", guess score %.4f" % sc
            if sc < best[0]:
                best = (sc, net.get_params())
        if log:
            log(msg)
    if select:
        net.set_params(best[1])
        net.best_score = best[0]
    return history


def init_net_params(nin, nout, hidden=16, seed=0):
    """Initial FP32 parameters in the flat order of rt_net_set_params: per
    layer the (offset, co, ci) weights, He-normal with fan-in 27 ci, then zero
    biases; the last layer is zero so the untrained network proposes the
    linear extrapolation."""
    rng = np.random.default_rng(seed)
    shapes = [(nin, hidden), (hidden, hidden), (hidden, hidden), (hidden, nout)]
    parts = []
    for li, (ci, co) in enumerate(shapes):
        std = np.sqrt(2.0 / (27 * ci)) if li < 3 else 0.0
        parts.append(rng.standard_normal(27 * co * ci) * std)
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)
