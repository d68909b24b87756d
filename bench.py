#!/usr/bin/env python
"""Benchmark: implicit Newton-step cell-updates/s at 256^3 on one MI355X.

A step is one full implicit time step of the 256^3 periodic hydrogen problem
(centred 5e48 photons/s source in a 13.2 kpc box, dt = 1e11 s, theta = 1):
time-level set-up, Newton iterations with Schur elimination, MG-preconditioned
FGMRES and line search until the RMS residual is below 1e-6, then the energy
fold.  Inputs
stay resident in HBM; W warm-up steps run first (default 5), then K steps
are timed (default 10), each from the state the previous one produced.

Modes: plain (FP64 V-cycle, previous-state guess), mixed (FP32 V-cycle
inside FP64 Newton/Krylov), learned and mixed+learned (the better, by initial
residual, of the previous state and the convolutional network's guess; the
network is trained first, untimed, on a plain-method trajectory at 128^3
with the same cell size and time step).  The JSON line reports the headline
mode (mixed+learned) in `value` and every mode in `modes`.

`roofline` covers the kernel class with the largest share of the timed
region (HIP events on the library's stream around that class's launches);
its algorithmic bytes are the library's own per-launch count (every field a
launch must read or write, once).  `step_hbm` divides the algorithmic bytes
of every launch of the timed steps by the timed region, `box_correction`
those of the source-subdomain graphs by their replay time.  `cpu_baseline`
times the CPU FP64 oracle on a bounded sample of the same problem, on all
host cores and on one.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Newton-step cell-updates/s at 256^3, mixed+learned vs plain FP64, Newton tol 1e-6"
METRIC_SG = "Newton-step cell-updates/s, expanding-universe I-front (Sec. 4.6), Newton tol 1e-6"
WORKLOAD_HII = ("hii_256: %d^3 periodic hydrogen, centred 5e48 photons/s source, 13.2 kpc box, "
                "dt=1e11 s, theta=1, Newton tol 1e-6, FGMRES(30) rtol 1e-8%s, 5-level V-cycle RB-GS %d+%d%s")
METRIC_HHE = ("Newton-step cell-updates/s at 512^3 H+He (lognormal, 64 sources), mixed+learned vs "
              "plain FP64, Newton tol 1e-6")
WORKLOAD_HHE = ("hhe_lognormal_512: %d^3 periodic hydrogen+helium, lognormal sigma_ln=1.5, 64 sources "
                "log-uniform in [1e47, 1e49] photons/s, grey T_B=1e5 K, a=0.1 -> 0.125 over 50 steps, "
                "limiter held at time level n, Newton tol 1e-6, FGMRES(30) rtol 1e-8%s, 6-level "
                "V-cycle RB-GS %d+%d%s")
WORKLOAD_SG = ("sg_q05_z4: %d^3 periodic uniform hydrogen, 0.625 kpc proper cells at z=4, "
               "centred 5e48 photons/s source, isothermal 1e4 K, Einstein-de Sitter from z=4, "
               "dt=2e15 s, theta=1, limiter held at time level n, Newton tol 1e-6, FGMRES(30) rtol "
               "1e-8%s, 4-level V-cycle RB-GS %d+%d%s")
HBM_PEAK_GBS = 8000.0

# HBM traffic of a kernel class, keyed (class, mode, grid), from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) scaled
# by what the counters read for a plain 2 GiB device copy (FETCH_SIZE x 2.0,
# WRITE_SIZE x 1.0), as the ratio of the summed traffic to the summed
# algorithmic bytes over the class's dispatches of a one-step run; a run's
# traffic per launch is that ratio times its own algorithmic bytes per
# launch (the vector count, hence the bytes, differs from launch to launch).
# A figure belongs to the kernel source it was measured on and is reported
# as null for any other.
PMC_TRAFFIC = {
    ("cg_vector", "mixed", 256): {"ratio": 1.000, "kernels_sha256":
        "0f5ef77ae2f9c6e4290132ac295879fbbe56a2f6f0e8c311c39c85680033313a"},
    ("cg_vector", "mixed+learned", 256): {"ratio": 1.000, "kernels_sha256":
        "0f5ef77ae2f9c6e4290132ac295879fbbe56a2f6f0e8c311c39c85680033313a"},
    ("spmv", "mixed", 256): {"ratio": 1.029, "kernels_sha256":
        "0f5ef77ae2f9c6e4290132ac295879fbbe56a2f6f0e8c311c39c85680033313a"},
    ("spmv", "mixed+learned", 256): {"ratio": 1.029, "kernels_sha256":
        "0f5ef77ae2f9c6e4290132ac295879fbbe56a2f6f0e8c311c39c85680033313a"},
    ("rbgs_fine", "mixed", 256): {"ratio": 1.134, "kernels_sha256":
        "0f5ef77ae2f9c6e4290132ac295879fbbe56a2f6f0e8c311c39c85680033313a"},
    ("rbgs_fine", "mixed+learned", 256): {"ratio": 1.134, "kernels_sha256":
        "0f5ef77ae2f9c6e4290132ac295879fbbe56a2f6f0e8c311c39c85680033313a"},
}


def kernels_sha256():
    import hashlib
    with open(os.path.join(ROOT, "paper_0901_1110_amd", "csrc", "kernels.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def train_guess(n_train=128, steps=100, epochs=8, lr=3e-4, log=None, box=(0, 3, 6, 0),
                trajectories=1, workload="hii_256"):
    """Train the learned-guess network on plain-method trajectories of the
    workload's generator at n_train^3 (same cell size and time step; the
    source count scaled with the volume, at least one)."""
    import numpy as np
    import synth
    from paper_0901_1110_amd.binding import RtNet
    from paper_0901_1110_amd.driver import generate_trajectory, init_net_params, train_net

    t0 = time.perf_counter()
    W = synth.WORKLOADS[workload]
    base = W.replace(n=n_train, mg_levels=4, box_size=box[0], box_levels=box[1],
                     box_inner=box[2], box_coarse_sweeps=box[3],
                     box_s_sweeps=box[4] if len(box) > 4 and box[0] > 0 else 0, mg_fp32=0,
                     nsources=max(1, (W.nsources * n_train ** 3) // W.n ** 3))
    media = [base, base.replace(nsources=2, centred=False, seed=100,
                                logQ_range=(48.0, 48.7))][:trajectories]
    trajs = []
    for w in media:
        ts = time.perf_counter()
        trajs.append(generate_trajectory(w, steps))
        st = trajs[-1]["stats"]
        if log:
            log("trajectory %s: %d steps in %.1f s, Newton its %d, CG its %d, max CG/Newton %.1f"
                % (w.name + ("" if w.sigma_ln == 0 else "_lognormal"), steps,
                   time.perf_counter() - ts, sum(s["newton_its"] for s in st),
                   sum(s["cg_its_total"] for s in st),
                   max(s["cg_its_total"] / max(1, s["newton_its"]) for s in st)))
    t1 = time.perf_counter()
    net = RtNet(W.nspecies, (n_train,) * 3)
    net.set_params(init_net_params(net.nin, net.nout, seed=0))
    hist = train_net(net, trajs, epochs=epochs, lr=lr, seed=0, log=log)
    t2 = time.perf_counter()
    theta = net.get_params()
    info_score = getattr(net, "best_score", None)
    del trajs
    info = dict(train_grid=n_train, trajectory_steps=steps, trajectories=len(media),
                epochs=epochs, lr=lr, loss_first=hist[0] if hist else None,
                loss_last=hist[-1] if hist else None,
                selected_guess_score=info_score,
                trajectory_s=round(t1 - t0, 2), train_s=round(t2 - t1, 2))
    out = os.path.join(ROOT, "gpurun_out")
    if os.path.isdir(out):
        np.save(os.path.join(out, "net_params.npy"), theta)
    return theta, info


def run_mode(mode, steps, warmup, n=256, theta=None, forcing=0.0, box=(0, 3, 6, 0, 0),
             workload="hii_256", adaptive=0.0, smoothing=(2, 2)):
    import torch
    import synth
    from paper_0901_1110_amd.binding import RtNet
    from paper_0901_1110_amd.driver import AdaptiveSimulation, LearnedSimulation, Simulation

    w = synth.WORKLOADS[workload].replace(
        n=n, mg_fp32=1 if mode.startswith("mixed") else 0, pcg_forcing=forcing,
        box_size=box[0], box_levels=box[1], box_inner=box[2], box_coarse_sweeps=box[3],
        box_s_sweeps=box[4] if box[0] > 0 else 0, mg_pre=smoothing[0], mg_post=smoothing[1])
    if mode.endswith("learned"):
        net = RtNet(w.nspecies, (n, n, n))
        net.set_params(theta)
        sim = LearnedSimulation(w, net)
        warmup = max(warmup, 2)
    elif adaptive > 0.0:
        # adaptive steps (max-norm estimate), at most ten times the fixed step
        sim = AdaptiveSimulation(w, adaptive, p=0.0, dt_max=10.0 * w.dt)
    else:
        sim = Simulation(w)
    # the warm-up times every kernel class to find the dominant one; the timed
    # steps record events around that class's launches only (and count the
    # bytes of all)
    sim.grid.rt_timing(True)
    for _ in range(warmup):
        st = sim.step()
        if st["status"] != 0:
            raise RuntimeError("warm-up step failed: %s" % st)
        sim.advance()
    kt_warm = sim.grid.rt_timing(False)
    # the subdomain correction is one graph of a few hundred small kernels,
    # timed per replay: it is reported beside the roofline, not as a kernel
    dom = max((k for k in kt_warm if k != "box" and kt_warm[k][2] > 0),
              key=lambda k: kt_warm[k][1])
    stats = []
    torch.cuda.synchronize()
    sim.grid.rt_timing_classes([dom, "box"])
    sim.grid.rt_timing(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(sim.grid.stream)
    t0 = time.perf_counter()
    for _ in range(steps):
        st = sim.step()
        if st["status"] != 0:
            raise RuntimeError("timed step failed: %s" % st)
        stats.append(st)
        sim.advance()
    ev1.record(sim.grid.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = sim.grid.rt_timing(False)
    sim.grid.rt_timing_classes(None)
    gpu_ms = ev0.elapsed_time(ev1)
    N = n ** 3
    newton = sum(s["newton_its"] for s in stats)
    cg = sum(s["cg_its_total"] for s in stats)
    vc = sum(s["vcycles"] for s in stats)
    net_ms = None
    if mode.endswith("learned"):
        # the network's cost per step: its forward pass timed alone
        reps = 5
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sim.net.stream)
        for _ in range(reps):
            sim.net.forward(sim.Un, sim.Unm1, sim.eh, sim.ehm1, sim.nH, sim.nH_mean, w.u_e,
                            w.u_E, sim.eh, sim.Uguess)
        e1.record(sim.net.stream)
        torch.cuda.synchronize()
        net_ms = e0.elapsed_time(e1) / reps
    res = dict(mode=mode, cells=N, steps=steps, wall_s=wall, event_ms=gpu_ms,
               value=N * steps / wall, ms_per_step=1e3 * wall / steps,
               newton_its=newton, cg_its=cg, vcycles=vc,
               model_seconds_per_s=sum(st_.get("dt", w.dt) for st_ in stats) / wall,
               cell_newton_its_per_s=N * newton / wall, kernels_warmup=kt_warm,
               network_guess_used=sum(s["used_alt_guess"] for s in stats),
               network_ms_per_step=None if net_ms is None else round(net_ms, 3),
               fnorm0_mean=sum(min(s["fnorm_guess"], s["fnorm_alt"]) if s["fnorm_alt"] >= 0
                               else s["fnorm_guess"] for s in stats) / len(stats))
    # roofline of the dominant kernel class, on the library's byte count
    cnt, ms, nbytes = kt[dom]
    if cnt > 0 and ms > 0:
        achieved = nbytes / (ms * 1e-3) / 1e9
        tr = PMC_TRAFFIC.get((dom, mode, n))
        traffic = None
        if tr and kernels_sha256() == tr["kernels_sha256"]:
            traffic = round(tr["ratio"] * nbytes / cnt)
        res["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                           "algorithmic_bytes_per_launch": round(nbytes / cnt),
                           "launches": cnt, "avg_launch_us": round(1e3 * ms / cnt, 2),
                           "share_of_timed": round(ms / gpu_ms, 3)}
    # the whole step: every launch's algorithmic bytes over the timed region
    tot_bytes = sum(v[2] for v in kt.values())
    res["step_hbm"] = {"algorithmic_GB_per_step": round(tot_bytes / steps / 1e9, 3),
                       "achieved": round(tot_bytes / (gpu_ms * 1e-3) / 1e9, 1),
                       "frac": round(tot_bytes / (gpu_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "bytes_share": {k: round(v[2] / tot_bytes, 3) for k, v in kt.items()
                                       if v[2] > 0}}
    if kt["box"][0] > 0:
        res["box_correction"] = {"replays": kt["box"][0],
                                 "avg_replay_us": round(1e3 * kt["box"][1] / kt["box"][0], 1),
                                 "share_of_timed": round(kt["box"][1] / gpu_ms, 3),
                                 "hbm_frac": round(kt["box"][2] / (kt["box"][1] * 1e-3) / 1e9
                                                   / HBM_PEAK_GBS, 4)}
    del sim
    torch.cuda.empty_cache()
    return res


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def host_cores():
    """Cores this process may run on (the affinity mask; a container's CPU
    share can be smaller than what the machine reports)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(n=64, box=(0, 3, 6, 0), workload="hii_256"):
    """The oracle on a bounded sample: the first implicit step of the same
    problem (same cell size) on an n^3 periodic box around the source, on
    all host cores (NumPy/BLAS threads) and on one."""
    from threadpoolctl import threadpool_limits

    import synth
    import oracle
    from oracle import newton

    w = synth.WORKLOADS[workload].replace(n=n, mg_levels=min(4, synth.WORKLOADS[workload].mg_levels),
                                          box_size=box[0], box_levels=box[1],
                                          box_inner=box[2], box_coarse_sweeps=box[3],
                                          box_s_sweeps=box[4] if len(box) > 4 and box[0] > 0
                                          else 0)
    m = oracle.model_from_workload(w)
    s = synth.initial_state(w)
    out = {}
    for cores in (host_cores(), 1):
        with threadpool_limits(limits=cores):
            t0 = time.perf_counter()
            U, st = newton.newton_step(s["U"], s["U"], s["nH"], s["eh"], s["src_cells"],
                                       s["src_Q"], w.dt, w.cosmology(0), m)
            dt = time.perf_counter() - t0
        out[cores] = (n ** 3 / dt, dt, st)
        if cores == 1:
            break
    allc = max(out)
    v, dt, st = out[allc]
    res = {"value": v, "unit": "cell-updates/s", "cores": allc, "kind": "oracle",
           "cpu": cpu_model(),
           "sample": "first implicit step (status %d, %d Newton its, %d Krylov its) of the "
                     "%s problem (same cell size) on a %d^3 periodic box around the source, "
                     "same solver and preconditioner, NumPy FP64, %.1f s on %d threads"
                     % (st["status"], st["newton_its"], sum(st["cg_its"]), workload, n, dt,
                        allc)}
    if 1 in out and allc != 1:
        res["one_core"] = {"value": out[1][0], "seconds": round(out[1][1], 2)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--modes", default=None,
                    help="default plain,mixed,learned,mixed+learned (plain,mixed for sg_q05_z4)")
    ap.add_argument("--train-epochs", type=int, default=8)
    ap.add_argument("--train-steps", type=int, default=100)
    ap.add_argument("--train-trajectories", type=int, default=1)
    ap.add_argument("--workload", default="hii_256",
                    choices=["hii_256", "sg_q05_z4", "hhe_lognormal_512"],
                    help="hii_256: the timed 256^3 HII region; sg_q05_z4: the expanding-universe "
                         "I-front of Sec. 4.6 at 128^3; hhe_lognormal_512: the 512^3 "
                         "hydrogen+helium medium with 64 sources (cell size fixed, --n sets the "
                         "box)")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--pcg-forcing", type=float, default=1e-6,
                    help="inexact-Newton forcing factor delta_k / ||f(U_k)|| (Sec. 3.2.1; "
                         "0: the fixed relative CG tolerance alone)")
    ap.add_argument("--box-size", type=int, default=None,
                    help="source-subdomain correction: box edge in cells (0: V-cycle alone; "
                         "default 16 for hii_256, 0 for the others)")
    ap.add_argument("--box-levels", type=int, default=2)
    ap.add_argument("--box-inner", type=int, default=4)
    ap.add_argument("--box-coarse-sweeps", type=int, default=4,
                    help="sweeps of the coarsest box level (0: those of the main hierarchy)")
    ap.add_argument("--box-s-sweeps", type=int, default=48,
                    help="red-black sweeps on the Schur matrix itself over each box after the "
                         "correction")
    ap.add_argument("--mg-pre", type=int, default=2, help="V-cycle pre-smoothing (red, black) pairs")
    ap.add_argument("--mg-post", type=int, default=2, help="V-cycle post-smoothing pairs")
    ap.add_argument("--adaptive", type=float, default=0.0,
                    help="tau_tol > 0: adaptive steps with the explicit predictor as the guess "
                         "(plain and mixed modes; 0: the fixed step)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 2 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print("# copy calibration: 3 x %d bytes read + written" % (8 << 28), file=sys.stderr,
              flush=True)
        del a, b
    if args.n is None:
        args.n = {"hii_256": 256, "sg_q05_z4": 128, "hhe_lognormal_512": 512}[args.workload]
    if args.box_size is None:
        args.box_size = 16 if args.workload == "hii_256" else 0
    if args.modes is None:
        args.modes = "plain,mixed" if args.workload == "sg_q05_z4" \
            else "plain,mixed,learned,mixed+learned"
    modes = [m for m in args.modes.split(",") if m]
    if args.adaptive > 0.0 and any(m.endswith("learned") for m in modes):
        print("--adaptive offers the predictor as the guess: plain and mixed modes only",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "sg_q05_z4" and any(m.endswith("learned") for m in modes):
        print("no learned guess for the expanding-universe front", file=sys.stderr)
        sys.exit(2)
    box = (args.box_size, args.box_levels, args.box_inner, args.box_coarse_sweeps,
           args.box_s_sweeps)
    results = {}
    theta, train_info = None, None
    if any(m.endswith("learned") for m in modes):
        print("# training the learned guess (untimed)", file=sys.stderr, flush=True)
        theta, train_info = train_guess(steps=args.train_steps, epochs=args.train_epochs,
                                        log=lambda s: print("#   " + s, file=sys.stderr, flush=True),
                                        box=box, trajectories=args.train_trajectories,
                                        workload=args.workload)
        print("# trained: %s" % train_info, file=sys.stderr, flush=True)
    for mode in modes:
        print("# mode %s: %d warm-up + %d timed steps at %d^3" % (mode, args.warmup, args.steps, args.n),
              file=sys.stderr, flush=True)
        results[mode] = run_mode(mode, args.steps, args.warmup, args.n, theta, args.pcg_forcing,
                                 box, args.workload, args.adaptive, (args.mg_pre, args.mg_post))
        print("# %s: %.3e cell-updates/s, %.1f ms/step" % (mode, results[mode]["value"],
                                                          results[mode]["ms_per_step"]),
              file=sys.stderr, flush=True)
    head = next((m for m in ("mixed+learned", "mixed", "learned") if m in results), modes[0])
    H = results[head]
    line = {
        "metric": {"hii_256": METRIC, "sg_q05_z4": METRIC_SG,
                   "hhe_lognormal_512": METRIC_HHE}[args.workload],
        "value": H["value"], "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": H["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32" if head.startswith("mixed") else "f64",
        "data": "synthetic",
        "config": {"workload": {"hii_256": WORKLOAD_HII, "sg_q05_z4": WORKLOAD_SG,
                                "hhe_lognormal_512": WORKLOAD_HHE}[args.workload] % (
                                   args.n, " or ||r|| <= %g ||f(U_k)|| (inexact-Newton forcing)"
                                   % args.pcg_forcing if args.pcg_forcing > 0 else "",
                                   args.mg_pre, args.mg_post,
                                   ", then a %d^3 source-subdomain correction (%d inner PCG its, "
                                   "%d-level box V-cycle, %d red-black sweeps on S)"
                                   % (args.box_size, args.box_inner, args.box_levels,
                                      args.box_s_sweeps)
                                   if args.box_size > 0 else ""),
                   "mode": head, "grid": args.n, "parallelism": "single GPU"},
        "roofline": H.get("roofline"),
        "step_hbm": H.get("step_hbm"),
        "modes": {k: {kk: v[kk] for kk in ("value", "ms_per_step", "newton_its", "cg_its",
                                           "vcycles", "cell_newton_its_per_s", "model_seconds_per_s",
                                           "network_guess_used", "network_ms_per_step",
                                           "fnorm0_mean", "roofline", "step_hbm",
                                           "box_correction")
                      if v.get(kk) is not None}
                  for k, v in results.items()},
    }
    if train_info:
        line["learned_training"] = train_info
    if "plain" in results and head != "plain":
        line["speedup_vs_plain"] = H["value"] / results["plain"]["value"]
    if head.endswith("learned"):
        # what the learned guess did in the timed steps: the proposals the
        # initial-residual test accepted, the network's cost, and the gain
        # over the same mode without the network
        taken = H["network_guess_used"]
        base = results.get(head.replace("+learned", "") if "+" in head else "plain")
        line["learned_guess"] = {
            "proposals_taken": taken, "timed_steps": args.steps,
            "network_ms_per_step": H["network_ms_per_step"],
            "speedup_vs_same_mode_without_network":
                None if base is None else H["value"] / base["value"],
            "outcome": ("no proposal passed the initial-residual test: the learned mode ran "
                        "the previous-state guess plus the network's cost") if taken == 0 else
                       ("the proposal was taken in %d of %d timed steps" % (taken, args.steps))}
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        # about 10-30 s of oracle work in all: 96^3 for the HII region, 64^3 otherwise
        line["cpu_baseline"] = cpu_baseline(96 if args.workload == "hii_256" else 64, box,
                                            args.workload)
    print(json.dumps(line), flush=True)
    with open(os.path.join(ROOT, "gpurun_out", "bench_kernels.json") if os.path.isdir(
            os.path.join(ROOT, "gpurun_out")) else os.devnull, "w") as fh:
        json.dump({k: v["kernels_warmup"] for k, v in results.items()}, fh, indent=1)


if __name__ == "__main__":
    main()
