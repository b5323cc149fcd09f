#!/usr/bin/env python3
"""Throughput of the explicit well-balanced Osher-Romberg step on one MI355X.

One step = one pass of the whole scheme over the grid: free-surface detection, reconstruction with
predictor, every x- and y-edge fluctuation, cell update, CFL reduction.  Default workload: the
2048 x 1024 dam break with an obstacle (seed 0), 2000 timed steps at CFL 0.9, state resident in HBM.
Prints one JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VECTOR = 78.6e12     # MI355X FP64 vector peak, FLOP/s
PEAK_HBM = 8.0e12              # MI355X HBM3E peak, B/s
STATE_BYTES_PER_CELL = 64      # read 4 FP64 + write 4 FP64 per cell update
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_dam_break_2048x1024_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1806_04960_amd", "csrc", f)
                  for f in ("bn2d_step.hip", "bn2d_physics.h")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on the
    current kernel source; otherwise None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    fields = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def build_workload(name):
    from paper_1806_04960_amd import scenarios as sc
    if name == "dam_break":
        return sc.dam_break(0)
    if name == "elliptic_drop":
        return sc.elliptic_drop(0)
    if name == "dam_break_small":
        return sc.dam_break_small()
    raise ValueError(name)


def attainable_peaks():
    """Measured on this GPU: FP64 FMA rate (FLOP/s) and triad HBM bandwidth (B/s), from the probe
    library, or None where it is not built."""
    import ctypes
    path = os.path.join(ROOT, "paper_1806_04960_amd", "libbn2d_probe.so")
    if not os.path.exists(path):
        return None
    L = ctypes.CDLL(path)
    L.bn_probe_fma.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    L.bn_probe_triad.argtypes = [ctypes.c_longlong, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    f, b = ctypes.c_double(), ctypes.c_double()
    out = {}
    if L.bn_probe_fma(256 * 4 * 8, 200, 5, ctypes.byref(f)) == 0:
        out["fp64_fma_tflops"] = f.value / 1e12
    if L.bn_probe_triad(1 << 27, 5, ctypes.byref(b)) == 0:
        out["triad_tb_per_s"] = b.value / 1e12
    return out


def cpu_baseline(s, steps):
    """The CPU oracle, single thread, on `steps` full steps of the same workload from its initial
    state (a bounded sample of the timed run)."""
    from oracle import bnref
    q = s.q.copy()
    t0 = time.perf_counter()
    for _ in range(steps):
        lam, dt = bnref.cfl(s, q)
        q = bnref.step(s, q, dt)
    el = time.perf_counter() - t0
    return {"value": s.nx * s.ny * steps / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} full oracle steps of the {s.nx}x{s.ny} {s.name} from its initial state "
                      f"({el:.1f} s, 1 thread)"}


def copy_probe(nbytes):
    """A plain copy of known size, 5 times: FETCH_SIZE and WRITE_SIZE read for it give the scale
    of those counters (bytes counted per byte moved) used for the step kernel's HBM traffic."""
    import torch
    n = nbytes // 8
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 8, "launches": 5}), flush=True)


def ensemble_main(args):
    """A batch of uneven dam breaks (sizes 256x128 .. 1024x512, seed 0) advanced together, one
    launch per step, each member with its own CFL step; against the same members run one after
    another as single grids for the same number of steps."""
    import numpy as np
    import torch

    from paper_1806_04960_amd import bn2d, flops
    from paper_1806_04960_amd import scenarios as sc

    members = sc.ensemble(0, args.members)
    cells = sum(s.nx * s.ny for s in members)
    print(f"# ensemble of {len(members)} members, {cells} cells, warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    with bn2d.Batch(members, rows_per_block=args.rows, wavefronts=args.wavefronts) as b:
        for k, s in enumerate(members):
            b.set_state(k, torch.from_numpy(s.q).cuda())
        rows, waves = b.launch()
        start_info = [(b.y0(k), b.time(k)[1]) for k in range(len(members))]
        b.run(args.warmup)
        b.status()
        start, end = ev(), ev()
        torch.cuda.synchronize()
        start.record()
        b.run(args.steps)
        end.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(end)
        b.status()
        end_info = [(b.get_state(k).cpu().numpy(), b.y0(k), b.time(k)[1]) for k in range(len(members))]
    print(f"# batch: {ms / args.steps:.4f} ms per step", file=sys.stderr, flush=True)

    # the same members one after another, each as a single grid, the same number of steps
    seq_ms = 0.0
    for s in members:
        with bn2d.Simulation(s, rows_per_block=args.rows, wavefronts=args.wavefronts) as sim:
            sim.set_state(torch.from_numpy(s.q).cuda())
            sim.run(args.warmup)
            start, end = ev(), ev()
            torch.cuda.synchronize()
            start.record()
            sim.run(args.steps)
            end.record()
            torch.cuda.synchronize()
            seq_ms += start.elapsed_time(end)
            sim.status()
    print(f"# sequential: {seq_ms / args.steps:.4f} ms per step of all members", file=sys.stderr, flush=True)

    launch_ms = ms / args.steps
    f = 0.0
    for s, (y0a, dta), (qe, y0e, dte) in zip(members, start_info, end_info):
        f += 0.5 * (flops.count(s, s.q, y0a, dta)["total"] + flops.count(s, qe, y0e, dte)["total"])
    achieved = f / (launch_ms / 1e3)
    line = {
        "metric": "FP64 cell updates/sec",
        "value": cells * args.steps / (ms / 1e3),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": launch_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"ensemble of {len(members)} uneven dam breaks (256x128..1024x512, seed 0), "
                               f"one launch per step", "members": len(members), "cells": cells,
                   "rows_per_block": rows, "wavefronts": waves},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VECTOR / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR, "traffic": None,
                     "flops_per_cell_update": f / cells, "kernel_ms": launch_ms},
        "sequential": {"value": cells * args.steps / (seq_ms / 1e3), "ms_per_step": seq_ms / args.steps,
                       "speedup_of_batch": seq_ms / ms},
    }
    if not args.no_cpu_baseline and args.cpu_baseline_steps > 0:
        line["cpu_baseline"] = cpu_baseline(members[0], args.cpu_baseline_steps)
    print(json.dumps(line), flush=True)


def adjoint_main(args):
    """Gradient of a wall-load functional through a trajectory of the 512 x 256 wall-impact
    workload (seed 0): N steps of fixed dt (the CFL step of the initial state), loss
    J = sum_n dt sum_j dy (alpha p)(Q^n) over the column in front of the wall, checkpoints every 20
    steps, each segment recomputed and reversed with bn_adjoint_step.  Reports the cost of the whole
    gradient (forward with checkpoints + recomputation + reverse) over a plain forward run, the
    adjoint step's own throughput, and a check of the gradient along seeded directions of the
    initial state against central differences of J."""
    import numpy as np
    import torch

    from paper_1806_04960_amd import bn2d
    from paper_1806_04960_amd import scenarios as sc

    N, seg = args.steps, 20
    s = sc.wall_impact(0)
    iw = s.meta["wall_column"] - 1
    n = s.nx * s.ny
    print(f"# adjoint workload {s.nx}x{s.ny}, {N} steps, checkpoints every {seg}", file=sys.stderr, flush=True)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    sim = bn2d.Simulation(s)
    q0 = torch.from_numpy(s.q).cuda()
    sim.set_state(q0)
    dt = sim.compute_dt()
    w = torch.zeros((4, s.ny, s.nx), dtype=torch.float64, device="cuda")
    fl = torch.from_numpy(s.fluid()).cuda()
    w[0, :, iw] = dt * s.dy * s.k0 / s.rho0   # d(alpha p)/d(alpha rho) = k0/rho0
    w[3, :, iw] = -dt * s.dy * s.k0           # d(alpha p)/d(alpha) = -k0
    w *= fl

    def loss(q_init):
        sim.set_state(q_init)
        J = torch.zeros((), dtype=torch.float64, device="cuda")
        for _ in range(N):
            sim.step(dt)
            J += (w * sim.get_state()).sum()
        return float(J)

    def forward_plain():
        sim.set_state(q0)
        for _ in range(N):
            sim.step(dt)

    def gradient(q_init=None):
        return bn2d.trajectory_gradient(sim, q0 if q_init is None else q_init, dt, N, w, seg)

    forward_plain()
    gradient()
    torch.cuda.synchronize()
    reps = 3
    a, b = ev(), ev()
    a.record()
    for _ in range(reps):
        forward_plain()
    b.record()
    torch.cuda.synchronize()
    fwd_ms = a.elapsed_time(b) / reps
    a.record()
    for _ in range(reps):
        g = gradient()
    b.record()
    torch.cuda.synchronize()
    grad_ms = a.elapsed_time(b) / reps
    # the same gradient keeping all N states in HBM (no recomputation)
    bn2d.trajectory_gradient(sim, q0, dt, N, w, store_all=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        g_all = bn2d.trajectory_gradient(sim, q0, dt, N, w, store_all=True)
    b.record()
    torch.cuda.synchronize()
    grad_all_ms = a.elapsed_time(b) / reps
    assert torch.equal(g_all, g)
    del g_all
    # the adjoint step alone
    lam = torch.randn((4, s.ny, s.nx), dtype=torch.float64, device="cuda")
    out = torch.empty_like(lam)
    a.record()
    for _ in range(100):
        sim.adjoint_step(q0, lam, dt, out=out)
    b.record()
    torch.cuda.synchronize()
    adj_ms = a.elapsed_time(b) / 100
    a.record()
    sim.set_state(q0)
    for _ in range(100):
        sim.step(dt)
    b.record()
    torch.cuda.synchronize()
    step_ms = a.elapsed_time(b) / 100
    print(f"# forward {fwd_ms:.2f} ms, gradient {grad_ms:.2f} ms (x{grad_ms / fwd_ms:.2f}), all states kept "
          f"{grad_all_ms:.2f} ms (x{grad_all_ms / fwd_ms:.2f}); step {step_ms*1e3:.1f} us, "
          f"adjoint step {adj_ms*1e3:.1f} us", file=sys.stderr, flush=True)

    # gradient checks: dJ/dq0 along seeded patch directions of the initial state, and dJ/dtheta
    # (the 64 profile values, chained through the state's construction) along seeded directions;
    # difference quotients at h and h/2, whose disagreement estimates the quotient's own error
    # (large where the trajectory crosses one of the scheme's kinks: the liquid at rest sits on the
    # limiter's min/max ties).  Each kind alternately from the workload's initial state and from a
    # smooth departure from it (see scenarios.smooth_state).
    rng = np.random.default_rng(0)
    checks = []
    scale = np.stack([np.abs(s.q[0])] * 3 + [np.abs(s.q[3])]) * s.fluid()
    q_smooth = torch.from_numpy(sc.smooth_state(s).q).cuda()
    g_of = {"initial": g.cpu().numpy(), "smooth": gradient(q_smooth).cpu().numpy()}
    q_of = {"initial": q0, "smooth": q_smooth}
    theta0 = np.asarray(s.meta["theta"])
    gth_of = {"initial": sc.wall_impact_theta_vjp(s, g_of["initial"]),
              "smooth": sc.wall_impact_theta_vjp(s, sc.smooth_state_vjp(s, g_of["smooth"]))}

    def q_theta(theta, kind):
        st = sc.wall_impact(0, theta=theta)
        return torch.from_numpy((sc.smooth_state(st) if kind == "smooth" else st).q).cuda()

    def record(entry, ad, fd1, fd2):
        spread = abs(fd1 - fd2) / abs(fd2) if fd2 else None
        # a quotient that moves by more than 1e-4 between h and h/2 straddles a kink: reported,
        # not a check of the gradient
        entry.update({"adjoint": ad, "fd": fd2, "rel": abs(ad - fd2) / abs(fd2) if fd2 else None,
                      "fd_h_vs_h2": spread, "kink": spread is None or spread > 1e-4})
        checks.append(entry)
        print(f"# check {len(checks) - 1}: {entry}", file=sys.stderr, flush=True)

    for m in range(2 * args.fd_directions):
        kind = "smooth" if m % 2 else "initial"
        # a patch in the reservoir (rows below 0.75 m, left of the wall)
        j0, i0 = int(rng.integers(0, 96 - 24)), int(rng.integers(0, iw - 24))
        d = np.zeros_like(s.q)
        d[:, j0:j0 + 24, i0:i0 + 24] = rng.normal(size=(4, 24, 24))
        d *= scale
        dd = torch.from_numpy(d).cuda()
        qa, h = q_of[kind], 1e-7
        fd1 = (loss(qa + h * dd) - loss(qa - h * dd)) / (2 * h)
        fd2 = (loss(qa + h / 2 * dd) - loss(qa - h / 2 * dd)) / h
        record({"wrt": "q0", "state": kind, "patch": [j0, i0]}, float(np.sum(g_of[kind] * d)), fd1, fd2)
    for m in range(2 * args.fd_directions):
        kind = "smooth" if m % 2 else "initial"
        dth = rng.normal(size=theta0.size)
        h = 1e-6
        fd1 = (loss(q_theta(theta0 + h * dth, kind)) - loss(q_theta(theta0 - h * dth, kind))) / (2 * h)
        fd2 = (loss(q_theta(theta0 + h / 2 * dth, kind)) - loss(q_theta(theta0 - h / 2 * dth, kind))) / h
        record({"wrt": "theta", "state": kind}, float(gth_of[kind] @ dth), fd1, fd2)
    # the same theta directions over a horizon on which J is smooth in theta (40 steps)
    N_short = 40
    short = []
    rng = np.random.default_rng(1)
    for m in range(2 * args.fd_directions):
        kind = "smooth" if m % 2 else "initial"
        gq = bn2d.trajectory_gradient(sim, q_of[kind], dt, N_short, w, seg).cpu().numpy()
        gth = sc.wall_impact_theta_vjp(s, sc.smooth_state_vjp(s, gq) if kind == "smooth" else gq)
        dth = rng.normal(size=theta0.size)
        h = 1e-7

        def loss_short(theta):
            sim.set_state(q_theta(theta, kind))
            J = torch.zeros((), dtype=torch.float64, device="cuda")
            for _ in range(N_short):
                sim.step(dt)
                J += (w * sim.get_state()).sum()
            return float(J)

        fd1 = (loss_short(theta0 + h * dth) - loss_short(theta0 - h * dth)) / (2 * h)
        fd2 = (loss_short(theta0 + h / 2 * dth) - loss_short(theta0 - h / 2 * dth)) / h
        entry = {"wrt": "theta", "state": kind, "steps": N_short}
        n_before = len(checks)
        record(entry, float(gth @ dth), fd1, fd2)
        short.append(checks.pop(n_before))
    sim.close()
    line = {
        "metric": "FP64 cell updates/sec",
        "value": n / (adj_ms / 1e3),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": N,
        "warmup": 1,
        "ms_per_step": adj_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"discrete adjoint, wall impact {s.nx}x{s.ny} seed 0, {N} steps of fixed dt, "
                               f"checkpoints every {seg}", "nx": s.nx, "ny": s.ny},
        "adjoint": {"forward_ms": fwd_ms, "gradient_ms": grad_ms, "cost_ratio": grad_ms / fwd_ms,
                    "gradient_all_states_ms": grad_all_ms, "cost_ratio_all_states": grad_all_ms / fwd_ms,
                    "step_us": step_ms * 1e3, "adjoint_step_us": adj_ms * 1e3,
                    "grad_theta_norm": float(np.linalg.norm(gth_of["initial"])), "fd_checks": checks,
                    "fd_checks_theta_40_steps": short},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="dam_break",
                    choices=["dam_break", "elliptic_drop", "dam_break_small", "ensemble", "adjoint"])
    ap.add_argument("--members", type=int, default=64, help="ensemble size (workload ensemble)")
    ap.add_argument("--fd-directions", type=int, default=4, help="gradient checks (workload adjoint)")
    ap.add_argument("--rows", type=int, default=None, help="rows per claimed block of the step kernel")
    ap.add_argument("--wavefronts", type=int, default=None, help="wavefronts of the persistent step kernel")
    ap.add_argument("--cpu-baseline-steps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run device-to-device copies of BYTES bytes (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (each GPU would own a strip "
              "of columns; see the design notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1806_04960_amd import bn2d, flops

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.workload == "ensemble":
        ensemble_main(args)
        return
    if args.workload == "adjoint":
        adjoint_main(args)
        return
    s = build_workload(args.workload)
    print(f"# workload {s.name} {s.nx}x{s.ny}, warmup {args.warmup}, steps {args.steps}", file=sys.stderr,
          flush=True)

    q0 = torch.from_numpy(s.q).cuda()
    with bn2d.Simulation(s, rows_per_block=args.rows, wavefronts=args.wavefronts) as sim:
        sim.set_state(q0)
        rows, waves = sim.launch()
        y0_start = sim.y0()
        dt_start = sim.compute_dt()
        sim.run(args.warmup)
        sim.status()
        # timed region: K steps, one kernel launch each, back to back on the stream the kernel
        # runs on (the context uses torch's current stream); the average launch duration is the
        # region's duration over K
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        sim.run(args.steps)
        end.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(end)
        launch_ms = ms / args.steps
        sim.status()
        q_end = sim.get_state().cpu().numpy()
        y0_end = sim.y0()
        t_end, dt_end = sim.time()

    cells = s.nx * s.ny
    ms_per_step = ms / args.steps
    value = cells * args.steps / (ms / 1e3)

    # algorithmic FLOPs per launch: mean of the counts on the first and last state of the run
    f0 = flops.count(s, s.q, y0_start, dt_start)
    f1 = flops.count(s, q_end, y0_end, dt_end)
    flops_per_launch = 0.5 * (f0["total"] + f1["total"])
    achieved = flops_per_launch / (launch_ms / 1e3)
    # (the committed counter summary is of the dam break workload)
    traffic = measured_traffic() if args.workload == "dam_break" else None
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VECTOR / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR, "traffic": traffic,
                "flops_per_cell_update": flops_per_launch / cells, "kernel_ms": launch_ms,
                "hbm_frac_at_algorithmic_bytes": cells * STATE_BYTES_PER_CELL / (launch_ms / 1e3) / PEAK_HBM}

    peaks = attainable_peaks()
    if peaks:
        roofline["attainable"] = peaks
        if "fp64_fma_tflops" in peaks:
            roofline["frac_of_attainable"] = achieved / 1e12 / peaks["fp64_fma_tflops"]

    line = {
        "metric": "FP64 cell updates/sec",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{s.name} {s.nx}x{s.ny} seed 0, CFL {s.cfl}", "nx": s.nx, "ny": s.ny,
                   "cells": cells, "simulated_time_s": t_end,
                   "rows_per_block": rows, "wavefronts": waves},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline and args.cpu_baseline_steps > 0:
        line["cpu_baseline"] = cpu_baseline(s, args.cpu_baseline_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
