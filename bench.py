#!/usr/bin/env python
"""Benchmark: implicit Newton-step cell-updates/s at 256^3 on one MI355X.

A step is one full implicit time step of the 256^3 periodic hydrogen problem
(centred 5e48 photons/s source in a 13.2 kpc box, dt = 1e11 s, theta = 1):
time-level set-up, Newton iterations with Schur elimination, MG-PCG and line
search until the RMS residual is below 1e-6, then the energy fold.  Inputs
stay resident in HBM; W warm-up steps run first (default 20: past the
start-up transient of the 200-step trajectory), then K steps are timed, each
from the state the previous one produced.

Modes: plain (FP64 V-cycle, previous-state guess), mixed (FP32 V-cycle
inside FP64 Newton/CG), learned and mixed+learned (the better, by initial
residual, of the previous state and the convolutional network's guess; the
network is trained first, untimed, on 200-step plain-method trajectories at
128^3 with the same cell size and time step).  The JSON line reports the
headline mode (mixed+learned) in `value` and every mode in `modes`;
`roofline` covers the kernel class with the largest share of the timed region, timed with HIP events on the library's stream; `cpu_baseline`
times the CPU FP64 oracle on a bounded sample of the same problem.
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
                "dt=1e11 s, theta=1, Newton tol 1e-6, PCG rtol 1e-8%s, 5-level V-cycle RB-GS 2+2%s")
WORKLOAD_SG = ("sg_q05_z4: %d^3 periodic uniform hydrogen, 0.625 kpc proper cells at z=4, "
               "centred 5e48 photons/s source, isothermal 1e4 K, Einstein-de Sitter from z=4, "
               "dt=2e15 s, theta=1, Newton tol 1e-6, PCG rtol 1e-8%s, 4-level V-cycle RB-GS 2+2%s")
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per cell and launch of each kernel class (H-only, FP64
# fields = 8 B; FP32 V-cycle fields = 4 B).  Neighbour values read through the
# cache are not counted: a stencil needs each field once.
#   residual : read U(3) g(3) n_H e_h D(3), write f(3)                  = 14 x 8
#   schur    : read U(3) f(3) n_H e_h D(3), write f~_M(2) W(2) S(4) b   = 20 x 8
#   trial    : read U(3) f~_M(2) W(2) s_E, write U_t(3)                 = 11 x 8
#   spmv     : read diag cx cy cz p, write q                            = 6 x 8
#   rbgs     : one half-sweep: all 3 couplings, diag and b of the colour,
#              the other colour's x, write the colour's x              = (3 + 1) w + 1 w = 5 w
#              first (red, black) pair from x = 0, one launch: diag, b,
#              the 3 couplings, write x                                = 6 w
#              FP32 cycle's last half-sweep: 4 w, write z (FP64, both
#              colours), read r and q (FP64) for the CG dots           = 4 w + 24 B
#              (the subdomain correction, when on, adds its own part of
#              the dots over the box cells)
# (w = 4 B for the FP32 V-cycle, 8 B for FP64)
BYTES_PER_CELL = {"residual": 112.0, "schur": 160.0, "trial": 88.0, "spmv": 48.0}
# with the FP32 cycle the Schur assembly also writes the four FP32 operator
# arrays of the finest level
SCHUR_FP32_EXTRA = 16.0


def class_bytes_per_cell(dom, wbytes):
    """Algorithmic bytes per cell of one launch of a modelled Newton-level class."""
    b = BYTES_PER_CELL[dom]
    return b + (SCHUR_FP32_EXTRA if dom == "schur" and wbytes == 4.0 else 0.0)


# HBM traffic per launch of the finest-level FP32 smoother class at 256^3 with
# V(2,2), from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) scaled by
# what the counters read for a plain 2 GiB device copy (FETCH_SIZE x 2.0,
# WRITE_SIZE x 1.0), averaged over one V-cycle's 7 launches, with the subdomain
# correction on.  It belongs to the
# kernel source it was measured on and is reported as null for any other.
PMC_TRAFFIC = {"rbgs_fine": {"w": 4, "n": 256, "pre_post": (2, 2), "dots": True,
                             "bytes_per_launch": 4.198e8,
                             "kernels_sha256": "30d3d56a17f7a2c42448280a75d4a956f54a4660e32b1f764829694b9c264f47"}}


def kernels_sha256():
    import hashlib
    with open(os.path.join(ROOT, "paper_0901_1110_amd", "csrc", "kernels.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def rbgs_fine_per_vcycle(pre, post, w, dots=True):
    """(launches, algorithmic bytes per cell) of the fine-level smoothing in one
    V-cycle of the CG loop; in the FP32 cycle the last half-sweep writes the
    FP64 result and forms the CG dots (pre, post > 0 there)."""
    if pre > 0:
        launches = 1 + 2 * (pre - 1) + 2 * post
        b = 6.0 * w + (2 * (pre - 1) + 2 * post) * 5.0 * w
        if w == 4.0 and post > 0:
            b += (4.0 * w + (24.0 if dots else 8.0)) - 5.0 * w
        return launches, b
    return 2 * post, 2 * post * 5.0 * w


def train_guess(n_train=128, steps=200, epochs=8, lr=3e-4, log=None, box=(0, 3, 6, 0)):
    """Train the learned-guess network on plain-method trajectories."""
    import numpy as np
    import synth
    from paper_0901_1110_amd.binding import RtNet
    from paper_0901_1110_amd.driver import generate_trajectory, init_net_params, train_net

    t0 = time.perf_counter()
    base = synth.CFG_256.replace(n=n_train, mg_levels=4, box_size=box[0], box_levels=box[1],
                                 box_inner=box[2], box_coarse_sweeps=box[3])
    media = [base, base.replace(sigma_ln=1.0, nsources=4, centred=False, seed=100,
                                logQ_range=(48.0, 48.7))]
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
    net = RtNet(1, (n_train,) * 3)
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


def run_mode(mode, steps, warmup, n=256, theta=None, forcing=0.0, box=(0, 3, 6, 0),
             workload="hii_256", adaptive=0.0):
    import torch
    import synth
    from paper_0901_1110_amd.binding import RtNet
    from paper_0901_1110_amd.driver import AdaptiveSimulation, LearnedSimulation, Simulation

    w = synth.WORKLOADS[workload].replace(
        n=n, mg_fp32=1 if mode.startswith("mixed") else 0, pcg_forcing=forcing,
        box_size=box[0], box_levels=box[1], box_inner=box[2], box_coarse_sweeps=box[3])
    if mode.endswith("learned"):
        net = RtNet(1, (n, n, n))
        net.set_params(theta)
        sim = LearnedSimulation(w, net)
        warmup = max(warmup, 2)
    elif adaptive > 0.0:
        # adaptive steps (max-norm estimate), at most ten times the fixed step
        sim = AdaptiveSimulation(w, adaptive, p=0.0, dt_max=10.0 * w.dt)
    else:
        sim = Simulation(w)
    # the warm-up times every kernel class to find the dominant one; the timed
    # steps record events around that class's launches only
    sim.grid.rt_timing(True)
    for _ in range(warmup):
        st = sim.step()
        if st["status"] != 0:
            raise RuntimeError("warm-up step failed: %s" % st)
        sim.advance()
    kt_warm = sim.grid.rt_timing(False)
    # the subdomain correction is one graph of a few hundred small kernels,
    # timed per replay: it is reported beside the roofline, not as a kernel.
    # The roofline covers the largest class with a byte model.
    modelled = ["rbgs_fine"] + list(BYTES_PER_CELL)
    dom_all = max((k for k in kt_warm if k != "box"), key=lambda k: kt_warm[k][1])
    dom = max(modelled, key=lambda k: kt_warm[k][1])
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
    res = dict(mode=mode, cells=N, steps=steps, wall_s=wall, event_ms=gpu_ms,
               value=N * steps / wall, ms_per_step=1e3 * wall / steps,
               newton_its=newton, cg_its=cg, vcycles=vc,
               model_seconds_per_s=sum(st_.get("dt", w.dt) for st_ in stats) / wall,
               cell_newton_its_per_s=N * newton / wall, kernels_warmup=kt_warm,
               network_guess_used=sum(s["used_alt_guess"] for s in stats),
               fnorm0_mean=sum(min(s["fnorm_guess"], s["fnorm_alt"]) if s["fnorm_alt"] >= 0
                               else s["fnorm_guess"] for s in stats) / len(stats))
    # roofline of the dominant kernel class
    wbytes = 4.0 if mode.startswith("mixed") else 8.0
    p = sim.grid.params
    launches_vc, bytes_vc = rbgs_fine_per_vcycle(p.mg_pre, p.mg_post, wbytes)
    cnt, ms = kt[dom]
    if dom == "rbgs_fine":
        total_bytes = cnt / float(launches_vc) * bytes_vc * N
    elif dom in BYTES_PER_CELL:
        total_bytes = cnt * class_bytes_per_cell(dom, wbytes) * N
    else:
        total_bytes = None
    if total_bytes is not None and ms > 0:
        achieved = total_bytes / (ms * 1e-3) / 1e9
        tr = PMC_TRAFFIC.get(dom)
        traffic = None
        if (tr and tr["w"] == wbytes and tr["n"] == n and tr["pre_post"] == (p.mg_pre, p.mg_post)
                and tr["dots"] and kernels_sha256() == tr["kernels_sha256"]):
            traffic = tr["bytes_per_launch"]
        res["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                           "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                           "algorithmic_bytes_per_launch": round(total_bytes / cnt),
                           "launches": cnt, "avg_launch_us": round(1e3 * ms / cnt, 2),
                           "largest_class_in_warmup": dom_all,
                           "share_of_timed": round(ms / gpu_ms, 3)}
    if kt["box"][0] > 0:
        res["box_correction"] = {"replays": kt["box"][0],
                                 "avg_replay_us": round(1e3 * kt["box"][1] / kt["box"][0], 1),
                                 "share_of_timed": round(kt["box"][1] / gpu_ms, 3)}
    del sim
    torch.cuda.empty_cache()
    return res


def cpu_baseline(n=128, box=(0, 3, 6, 0), workload="hii_256"):
    """The oracle on a bounded sample: the first implicit step of the same
    problem (same cell size) on an n^3 periodic box around the source."""
    from threadpoolctl import threadpool_limits

    import synth
    import oracle
    from oracle import newton

    w = synth.WORKLOADS[workload].replace(n=n, mg_levels=4, box_size=box[0], box_levels=box[1],
                                          box_inner=box[2], box_coarse_sweeps=box[3])
    m = oracle.model_from_workload(w)
    s = synth.initial_state(w)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        U, st = newton.newton_step(s["U"], s["U"], s["nH"], s["eh"], s["src_cells"], s["src_Q"],
                                   w.dt, w.cosmology(0), m)
        dt = time.perf_counter() - t0
    return {"value": n ** 3 / dt, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": "first implicit step (status %d, %d Newton its, %d CG its) of the "
                      "%s problem (same cell size) on a %d^3 periodic box around the source, "
                      "same preconditioner, NumPy FP64, 1 thread, %.1f s"
                      % (st["status"], st["newton_its"], sum(st["cg_its"]), workload, n, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--modes", default=None,
                    help="default plain,mixed,learned,mixed+learned (plain,mixed for sg_q05_z4)")
    ap.add_argument("--train-epochs", type=int, default=8)
    ap.add_argument("--train-steps", type=int, default=200)
    ap.add_argument("--workload", default="hii_256", choices=["hii_256", "sg_q05_z4"],
                    help="hii_256: the timed 256^3 HII region; sg_q05_z4: the expanding-universe "
                         "I-front of Sec. 4.6 at 128^3 (cell size fixed, --n sets the box)")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--pcg-forcing", type=float, default=1e-6,
                    help="inexact-Newton forcing factor delta_k / ||f(U_k)|| (Sec. 3.2.1; "
                         "0: the fixed relative CG tolerance alone)")
    ap.add_argument("--box-size", type=int, default=None,
                    help="source-subdomain correction: box edge in cells (0: V-cycle alone; "
                         "default 32 for hii_256, 0 for sg_q05_z4)")
    ap.add_argument("--box-levels", type=int, default=2)
    ap.add_argument("--box-inner", type=int, default=20)
    ap.add_argument("--box-coarse-sweeps", type=int, default=4,
                    help="sweeps of the coarsest box level (0: those of the main hierarchy)")
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
        args.n = 256 if args.workload == "hii_256" else 128
    if args.box_size is None:
        args.box_size = 32 if args.workload == "hii_256" else 0
    if args.modes is None:
        args.modes = "plain,mixed,learned,mixed+learned" if args.workload == "hii_256" \
            else "plain,mixed"
    modes = [m for m in args.modes.split(",") if m]
    if args.adaptive > 0.0 and any(m.endswith("learned") for m in modes):
        print("--adaptive offers the predictor as the guess: plain and mixed modes only",
              file=sys.stderr)
        sys.exit(2)
    if args.workload != "hii_256" and any(m.endswith("learned") for m in modes):
        print("the learned guess is trained for the HII-region workload only", file=sys.stderr)
        sys.exit(2)
    box = (args.box_size, args.box_levels, args.box_inner, args.box_coarse_sweeps)
    results = {}
    theta, train_info = None, None
    if any(m.endswith("learned") for m in modes):
        print("# training the learned guess (untimed)", file=sys.stderr, flush=True)
        theta, train_info = train_guess(steps=args.train_steps, epochs=args.train_epochs,
                                        log=lambda s: print("#   " + s, file=sys.stderr, flush=True),
                                        box=box)
        print("# trained: %s" % train_info, file=sys.stderr, flush=True)
    for mode in modes:
        print("# mode %s: %d warm-up + %d timed steps at %d^3" % (mode, args.warmup, args.steps, args.n),
              file=sys.stderr, flush=True)
        results[mode] = run_mode(mode, args.steps, args.warmup, args.n, theta, args.pcg_forcing,
                                 box, args.workload, args.adaptive)
        print("# %s: %.3e cell-updates/s, %.1f ms/step" % (mode, results[mode]["value"],
                                                          results[mode]["ms_per_step"]),
              file=sys.stderr, flush=True)
    head = next((m for m in ("mixed+learned", "mixed", "learned") if m in results), modes[0])
    H = results[head]
    line = {
        "metric": METRIC if args.workload == "hii_256" else METRIC_SG,
        "value": H["value"], "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": H["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32" if head.startswith("mixed") else "f64",
        "data": "synthetic",
        "config": {"workload": (WORKLOAD_HII if args.workload == "hii_256" else WORKLOAD_SG) % (
                                   args.n, " or ||r|| <= %g ||f(U_k)|| (inexact-Newton forcing)"
                                   % args.pcg_forcing if args.pcg_forcing > 0 else "",
                                   ", then a %d^3 source-subdomain correction (%d inner PCG its, "
                                   "%d-level box V-cycle)" % (args.box_size, args.box_inner,
                                                              args.box_levels)
                                   if args.box_size > 0 else ""),
                   "mode": head, "grid": args.n, "parallelism": "single GPU"},
        "roofline": H.get("roofline"),
        "modes": {k: {kk: v[kk] for kk in ("value", "ms_per_step", "newton_its", "cg_its",
                                           "vcycles", "cell_newton_its_per_s", "model_seconds_per_s",
                                           "network_guess_used", "fnorm0_mean")
                      if kk in v} | ({"box_correction": v["box_correction"]}
                                     if "box_correction" in v else {})
                  for k, v in results.items()},
    }
    if train_info:
        line["learned_training"] = train_info
    if "plain" in results and head != "plain":
        line["speedup_vs_plain"] = H["value"] / results["plain"]["value"]
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = (cpu_baseline(box=box) if args.workload == "hii_256"
                                else cpu_baseline(64, box, args.workload))
    print(json.dumps(line), flush=True)
    with open(os.path.join(ROOT, "gpurun_out", "bench_kernels.json") if os.path.isdir(
            os.path.join(ROOT, "gpurun_out")) else os.devnull, "w") as fh:
        json.dump({k: v["kernels_warmup"] for k, v in results.items()}, fh, indent=1)


if __name__ == "__main__":
    main()
