#!/usr/bin/env python3
"""Throughput of the explicit well-balanced Osher-Romberg step on one MI355X.

One step = one pass of the whole scheme over the grid: free-surface detection, reconstruction with
predictor, every x- and y-edge fluctuation, cell update, CFL reduction.  Headline workload: the
2048 x 1024 dam break with an obstacle (seed 0), K timed steps at CFL 0.9 after W warm-up steps,
state resident in HBM; the K steps are timed as one region split into 5 consecutive parts, whose
median is reported beside the whole-region rate.  The default run adds, in the same JSON line:
the 4096 x 4096 elliptical drop (K steps, at most 980 after at most 20 warm-up steps: its stated
1000; its own roofline), the 64-member ensemble (K steps, at most 480 after at most 20: its stated 500;
the batch against the same members run one after another), the checkpointed gradient of the 512 x 256
wall-impact workload over its 400 steps against the plain forward run, and the CPU oracle on a
bounded sample of the headline workload (one thread and all host threads).
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


def host_info():
    import platform
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "sched_cpus": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_baseline(s, steps, steps_single):
    """The CPU oracle as it stands on a bounded sample of the same workload from its initial state:
    `steps` full steps with its row sweeps on all host threads (OpenMP, deterministic: the same
    arithmetic per cell whatever the thread count), and `steps_single` steps on one thread."""
    from oracle import bnref

    def timed(n, threads):
        bnref.set_threads(threads)
        q = s.q.copy()
        t0 = time.perf_counter()
        for _ in range(n):
            lam, dt = bnref.cfl(s, q)
            q = bnref.step(s, q, dt)
        return time.perf_counter() - t0

    threads = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit():
        threads = min(threads, int(omp))
    el1 = timed(steps_single, 1) if steps_single > 0 else None
    el = timed(steps, threads)
    used = bnref.threads()
    bnref.set_threads(threads)
    out = {"value": s.nx * s.ny * steps / el, "unit": "cell-updates/s", "cores": used, "kind": "oracle",
           "sample": f"{steps} full oracle steps of the {s.nx}x{s.ny} {s.name} from its initial state "
                     f"({el:.1f} s on {used} threads; {steps_single} steps on 1 thread"
                     + (f" in {el1:.1f} s)" if el1 else ")"),
           "host": host_info()}
    if el1:
        out["single_thread_value"] = s.nx * s.ny * steps_single / el1
    return out


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


def timed_parts(run, K, parts=5):
    """Time K steps (run(n) enqueues n steps on torch's current stream) as one region split into
    `parts` consecutive parts: events between them, no synchronisation inside the region.  Returns
    the whole region's ms and the ms per step of each part."""
    import torch
    sizes = [n for n in (K // parts + (1 if p < K % parts else 0) for p in range(parts)) if n > 0]
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(len(sizes) + 1)]
    torch.cuda.synchronize()
    evs[0].record()
    for p, n in enumerate(sizes):
        run(n)
        evs[p + 1].record()
    torch.cuda.synchronize()
    return evs[0].elapsed_time(evs[-1]), [evs[p].elapsed_time(evs[p + 1]) / n for p, n in enumerate(sizes)]


def median(v):
    v = sorted(v)
    n = len(v)
    return v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2])


def single_workload(s, steps, warmup, rows=None, wavefronts=None, traffic=None):
    """One grid: `warmup` steps, then `steps` timed steps (one launch each); throughput, the step
    kernel's roofline (algorithmic FLOPs counted on the first and last state of the run)."""
    import torch

    from paper_1806_04960_amd import bn2d, flops

    q0 = torch.from_numpy(s.q).cuda()
    with bn2d.Simulation(s, rows_per_block=rows, wavefronts=wavefronts) as sim:
        sim.set_state(q0)
        shape = sim.launch()
        y0_start = sim.y0()
        dt_start = sim.compute_dt()
        sim.run(warmup)
        sim.status()
        ms, parts = timed_parts(sim.run, steps)
        sim.status()
        q_end = sim.get_state().cpu().numpy()
        y0_end = sim.y0()
        t_end, dt_end = sim.time()
    del q0
    cells = s.nx * s.ny
    launch_ms = ms / steps
    f0 = flops.count(s, s.q, y0_start, dt_start)
    f1 = flops.count(s, q_end, y0_end, dt_end)
    flops_per_launch = 0.5 * (f0["total"] + f1["total"])
    fluid = 0.5 * (f0["fluid_cells"] + f1["fluid_cells"])
    achieved = flops_per_launch / (launch_ms / 1e3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VECTOR / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR, "traffic": traffic,
                "flops_per_cell_update": flops_per_launch / cells, "kernel_ms": launch_ms,
                "hbm_frac_at_algorithmic_bytes": cells * STATE_BYTES_PER_CELL / (launch_ms / 1e3) / PEAK_HBM}
    return {"value": cells * steps / (ms / 1e3), "ms_per_step": launch_ms,
            "ms_per_step_median_of_5": median(parts), "ms_per_step_parts": parts,
            "fluid_cell_updates_per_s": fluid * steps / (ms / 1e3),
            "config": {"workload": f"{s.name} {s.nx}x{s.ny} seed 0, CFL {s.cfl}", "nx": s.nx, "ny": s.ny,
                       "cells": cells, "simulated_time_s": t_end, "rows_per_block": shape[0],
                       "wavefronts": shape[1]},
            "roofline": roofline}


def ensemble_measure(steps, warmup, count=64, rows=None, wavefronts=None):
    """A batch of uneven dam breaks (sizes 256x128 .. 1024x512, seed 0) advanced together, one
    launch per step, each member with its own CFL step; against the same members run one after
    another as single grids (each with its own default launch) for the same number of steps."""
    import torch

    from paper_1806_04960_amd import bn2d, flops
    from paper_1806_04960_amd import scenarios as sc

    members = sc.ensemble(0, count)
    cells = sum(s.nx * s.ny for s in members)
    print(f"# ensemble of {len(members)} members, {cells} cells, warmup {warmup}, steps {steps}",
          file=sys.stderr, flush=True)
    with bn2d.Batch(members, rows_per_block=rows, wavefronts=wavefronts) as b:
        for k, s in enumerate(members):
            b.set_state(k, torch.from_numpy(s.q).cuda())
        shape = b.launch()
        start_info = [(b.y0(k), b.time(k)[1]) for k in range(len(members))]
        b.run(warmup)
        b.status()
        ms, parts = timed_parts(b.run, steps)
        b.status()
        end_info = [(b.get_state(k).cpu().numpy(), b.y0(k), b.time(k)[1]) for k in range(len(members))]
    seq_ms, seq_parts = 0.0, [0.0] * 5
    for s in members:
        with bn2d.Simulation(s, rows_per_block=rows, wavefronts=wavefronts) as sim:
            sim.set_state(torch.from_numpy(s.q).cuda())
            sim.run(warmup)
            m, p = timed_parts(sim.run, steps)
            seq_ms += m
            seq_parts = [a + b for a, b in zip(seq_parts, p)] if len(p) == 5 else seq_parts
            sim.status()
    launch_ms = ms / steps
    f = 0.0
    for s, (y0a, dta), (qe, y0e, dte) in zip(members, start_info, end_info):
        f += 0.5 * (flops.count(s, s.q, y0a, dta)["total"] + flops.count(s, qe, y0e, dte)["total"])
    achieved = f / (launch_ms / 1e3)
    print(f"# batch {launch_ms:.4f} ms per step, sequential {seq_ms / steps:.4f} ms", file=sys.stderr, flush=True)
    return {"value": cells * steps / (ms / 1e3), "ms_per_step": launch_ms,
            "ms_per_step_median_of_5": median(parts), "ms_per_step_parts": parts,
            "sequential": {"value": cells * steps / (seq_ms / 1e3), "ms_per_step": seq_ms / steps,
                           "ms_per_step_median_of_5": median(seq_parts) if len(parts) == 5 else None},
            "speedup_of_batch": seq_ms / ms,
            "config": {"workload": f"ensemble of {len(members)} uneven dam breaks (256x128..1024x512, seed 0), "
                                   f"one launch per step", "members": len(members), "cells": cells,
                       "rows_per_block": shape[0], "wavefronts": shape[1]},
            "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VECTOR / 1e12,
                         "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VECTOR, "traffic": None,
                         "flops_per_cell_update": f / cells, "kernel_ms": launch_ms}}


class WallLoad:
    """The differentiation workload: 512 x 256 wall impact (seed 0), N steps of fixed dt (the CFL
    step of the initial state), loss J = sum_n dt sum_j dy (alpha p)(Q^n) over the column in front
    of the wall, its gradient by checkpoints every 20 steps, each segment recomputed and reversed
    with bn_adjoint_step."""

    def __init__(self, N=400, seg=20):
        import torch

        from paper_1806_04960_amd import bn2d
        from paper_1806_04960_amd import scenarios as sc

        self.N, self.seg = N, seg
        self.s = s = sc.wall_impact(0)
        self.iw = iw = s.meta["wall_column"] - 1
        self.sim = bn2d.Simulation(s)
        self.q0 = torch.from_numpy(s.q).cuda()
        self.sim.set_state(self.q0)
        self.dt = dt = self.sim.compute_dt()
        w = torch.zeros((4, s.ny, s.nx), dtype=torch.float64, device="cuda")
        fl = torch.from_numpy(s.fluid()).cuda()
        w[0, :, iw] = dt * s.dy * s.k0 / s.rho0   # d(alpha p)/d(alpha rho) = k0/rho0
        w[3, :, iw] = -dt * s.dy * s.k0           # d(alpha p)/d(alpha) = -k0
        self.w = w * fl

    def loss(self, q_init, N=None):
        import torch
        self.sim.set_state(q_init)
        J = torch.zeros((), dtype=torch.float64, device="cuda")
        for _ in range(self.N if N is None else N):
            self.sim.step(self.dt)
            J += (self.w * self.sim.get_state()).sum()
        return float(J)

    def forward_plain(self):
        self.sim.set_state(self.q0)
        for _ in range(self.N):
            self.sim.step(self.dt)

    def gradient(self, q_init=None, N=None, store_all=False, bottom=False):
        """dJ/dq0 (and, with ``bottom``, dJ/dy_L of the columns' bottoms: the wall's height is its
        column's entry)."""
        from paper_1806_04960_amd import bn2d
        return bn2d.trajectory_gradient(self.sim, self.q0 if q_init is None else q_init, self.dt,
                                        self.N if N is None else N, self.w, self.seg, store_all=store_all,
                                        bottom=bottom)

    def measure(self, reps=5):
        """Whole-gradient cost (forward with checkpoints + recomputation + reverse) over a plain
        forward run of the same N steps, each the median of `reps` timed repeats; the same with every
        state kept; one adjoint step and one forward step on their own."""
        import torch
        ev = lambda: torch.cuda.Event(enable_timing=True)

        def med(fn, n):
            fn()
            torch.cuda.synchronize()
            out = []
            for _ in range(n):
                a, b = ev(), ev()
                a.record()
                fn()
                b.record()
                torch.cuda.synchronize()
                out.append(a.elapsed_time(b))
            return median(out)

        # the workload's gradient: the 64 profile values come from dJ/dq0 through the state's
        # construction (host), the wall's height from the summed bottom adjoints of its column
        fwd_ms = med(self.forward_plain, reps)
        grad_ms = med(lambda: self.gradient(bottom=True), reps)
        grad_all_ms = med(lambda: self.gradient(store_all=True, bottom=True), reps)
        g_all, gb_all = self.gradient(store_all=True, bottom=True)
        g_ck, gb_ck = self.gradient(bottom=True)
        assert torch.equal(g_all, g_ck) and torch.equal(gb_all, gb_ck)
        dj_dhw = float(gb_ck[self.s.meta["wall_column"]])
        lam = torch.randn((4, self.s.ny, self.s.nx), dtype=torch.float64, device="cuda")
        out = torch.empty_like(lam)

        def adj100():
            for _ in range(100):
                self.sim.adjoint_step(self.q0, lam, self.dt, out=out)

        def fwd100():
            self.sim.set_state(self.q0)
            for _ in range(100):
                self.sim.step(self.dt)

        adj_ms = med(adj100, 3) / 100
        step_ms = med(fwd100, 3) / 100
        print(f"# forward {fwd_ms:.2f} ms, gradient {grad_ms:.2f} ms (x{grad_ms / fwd_ms:.2f}), all states kept "
              f"{grad_all_ms:.2f} ms (x{grad_all_ms / fwd_ms:.2f}); step {step_ms * 1e3:.1f} us, "
              f"adjoint step {adj_ms * 1e3:.1f} us", file=sys.stderr, flush=True)
        return {"workload": f"discrete adjoint, wall impact {self.s.nx}x{self.s.ny} seed 0, {self.N} steps of "
                            f"fixed dt, checkpoints every {self.seg}",
                "forward_ms": fwd_ms, "gradient_ms": grad_ms, "cost_ratio": grad_ms / fwd_ms,
                "gradient_all_states_ms": grad_all_ms, "cost_ratio_all_states": grad_all_ms / fwd_ms,
                "step_us": step_ms * 1e3, "adjoint_step_us": adj_ms * 1e3, "timing": f"median of {reps} repeats",
                "dJ_dwall_height": dj_dhw}

    def close(self):
        self.sim.close()


def ensemble_main(args):
    ens = ensemble_measure(args.steps, args.warmup, args.members, args.rows, args.wavefronts)
    line = {
        "metric": "FP64 cell updates/sec", "value": ens["value"], "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ens["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": ens["config"], "roofline": ens["roofline"],
        "sequential": dict(ens["sequential"], speedup_of_batch=ens["speedup_of_batch"]),
        "ms_per_step_median_of_5": ens["ms_per_step_median_of_5"],
    }
    print(json.dumps(line), flush=True)


def adjoint_main(args):
    """The differentiation workload (see WallLoad): cost of the whole gradient against a plain
    forward run, the adjoint step's own throughput, and checks of the gradient along seeded
    directions against central differences of J."""
    import numpy as np
    import torch

    from paper_1806_04960_amd import scenarios as sc

    W = WallLoad(args.steps)
    s, N, seg = W.s, W.N, W.seg
    n = s.nx * s.ny
    print(f"# adjoint workload {s.nx}x{s.ny}, {N} steps, checkpoints every {seg}", file=sys.stderr, flush=True)
    cost = W.measure()
    g = W.gradient()

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
    g_of = {"initial": g.cpu().numpy(), "smooth": W.gradient(q_smooth).cpu().numpy()}
    q_of = {"initial": W.q0, "smooth": q_smooth}
    theta0 = np.asarray(s.meta["theta"])
    gth_of = {"initial": sc.wall_impact_theta_vjp(s, g_of["initial"]),
              "smooth": sc.wall_impact_theta_vjp(s, sc.smooth_state_vjp(s, g_of["smooth"]))}

    def q_theta(theta, kind):
        st = sc.wall_impact(0, theta=theta)
        return torch.from_numpy((sc.smooth_state(st) if kind == "smooth" else st).q).cuda()

    def record(entry, ad, fds, out):
        """fds: central-difference quotients at decreasing steps h (a sweep over three decades).
        Where the trajectory crosses one of the scheme's kinks within +-h (limiter min/max, the
        liquid/gas and second-order switches) the quotients move with h; they then approach the
        adjoint as h shrinks rather than agreeing with each other.  A defect of the adjoint shows as
        the opposite: quotients that agree with each other ten times better than with the adjoint."""
        hs = sorted(fds, reverse=True)
        vals = [fds[h] for h in hs]
        ref = vals[-1]
        rel = [abs(ad - v) / abs(v) if v else None for v in vals]
        spread = [abs(a - b) / abs(b) if b else None for a, b in zip(vals, vals[1:])]
        kink = any(x is None or x > 1e-4 for x in spread)
        err = min((r for r in rel if r is not None), default=None)
        sp = min((x for x in spread if x is not None), default=None)
        defect = err is not None and sp is not None and err > 1e-4 and sp < err / 10
        entry.update({"adjoint": ad, "fd": ref, "rel": rel[-1], "h": hs, "fd_sweep": vals, "rel_sweep": rel,
                      "spread_sweep": spread, "kink": kink, "defect": defect})
        out.append(entry)
        print(f"# check {len(out) - 1}: {entry}", file=sys.stderr, flush=True)

    for m in range(2 * args.fd_directions):
        kind = "smooth" if m % 2 else "initial"
        # a patch in the reservoir (rows below 0.75 m, left of the wall)
        j0, i0 = int(rng.integers(0, 96 - 24)), int(rng.integers(0, W.iw - 24))
        d = np.zeros_like(s.q)
        d[:, j0:j0 + 24, i0:i0 + 24] = rng.normal(size=(4, 24, 24))
        d *= scale
        dd = torch.from_numpy(d).cuda()
        qa = q_of[kind]
        fds = {h: (W.loss(qa + h * dd) - W.loss(qa - h * dd)) / (2 * h) for h in (1e-6, 1e-7, 1e-8)}
        record({"wrt": "q0", "state": kind, "patch": [j0, i0]}, float(np.sum(g_of[kind] * d)), fds, checks)
    for m in range(2 * args.fd_directions):
        kind = "smooth" if m % 2 else "initial"
        dth = rng.normal(size=theta0.size)
        fds = {h: (W.loss(q_theta(theta0 + h * dth, kind)) - W.loss(q_theta(theta0 - h * dth, kind))) / (2 * h)
               for h in (1e-5, 1e-6, 1e-7)}
        record({"wrt": "theta", "state": kind}, float(gth_of[kind] @ dth), fds, checks)
    # the wall's height (its column's bottom), from both states
    iwall = s.meta["wall_column"]
    hw0 = float(s.bottom[iwall])

    def loss_hw(hw, kind, N=None):
        b = s.bottom.copy()
        b[iwall] = hw
        W.sim.set_bottom(b)
        J = W.loss(q_of[kind], N)
        W.sim.set_bottom(s.bottom)
        return J

    for kind in ("initial", "smooth"):
        _, gb = W.gradient(q_of[kind], bottom=True)
        fds = {h: (loss_hw(hw0 + h, kind) - loss_hw(hw0 - h, kind)) / (2 * h) for h in (1e-5, 1e-6, 1e-7)}
        record({"wrt": "wall_height", "state": kind}, float(gb[iwall]), fds, checks)
    # the same theta directions over a horizon on which J is smooth in theta (40 steps)
    N_short = 40
    short = []
    rng = np.random.default_rng(1)
    for m in range(2 * args.fd_directions):
        kind = "smooth" if m % 2 else "initial"
        gq = W.gradient(q_of[kind], N=N_short).cpu().numpy()
        gth = sc.wall_impact_theta_vjp(s, sc.smooth_state_vjp(s, gq) if kind == "smooth" else gq)
        dth = rng.normal(size=theta0.size)
        fds = {h: (W.loss(q_theta(theta0 + h * dth, kind), N_short) - W.loss(q_theta(theta0 - h * dth, kind), N_short))
               / (2 * h) for h in (1e-6, 1e-7, 5e-8)}
        record({"wrt": "theta", "state": kind, "steps": N_short}, float(gth @ dth), fds, short)
    for kind in ("initial", "smooth"):
        _, gb = W.gradient(q_of[kind], N=N_short, bottom=True)
        fds = {h: (loss_hw(hw0 + h, kind, N_short) - loss_hw(hw0 - h, kind, N_short)) / (2 * h)
               for h in (1e-6, 1e-7, 5e-8)}
        record({"wrt": "wall_height", "state": kind, "steps": N_short}, float(gb[iwall]), fds, short)
    W.close()
    defects = [c for c in checks + short if c["defect"]]
    adj_ms = cost["adjoint_step_us"] / 1e3
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
        "config": {"workload": cost["workload"], "nx": s.nx, "ny": s.ny},
        "adjoint": dict(cost, grad_theta_norm=float(np.linalg.norm(gth_of["initial"])), fd_checks=checks,
                        fd_checks_40_steps=short, defects=len(defects)),
    }
    print(json.dumps(line), flush=True)
    if defects:
        print(f"# {len(defects)} gradient checks look like adjoint defects (difference quotients agree with "
              f"each other ten times better than with the adjoint)", file=sys.stderr, flush=True)
        sys.exit(3)


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
    ap.add_argument("--no-extras", action="store_true",
                    help="headline workload only (no drop, ensemble and gradient measurements)")
    ap.add_argument("--cpu-baseline-steps", type=int, default=20, help="oracle steps on all host threads")
    ap.add_argument("--cpu-baseline-single-steps", type=int, default=5, help="oracle steps on one thread")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run device-to-device copies of BYTES bytes (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (each GPU would own a strip "
              "of columns and exchange two halo columns a side per step). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

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
    # (the committed counter summary is of the dam break workload)
    traffic = measured_traffic() if args.workload == "dam_break" else None
    head = single_workload(s, args.steps, args.warmup, args.rows, args.wavefronts, traffic)
    roofline = head["roofline"]
    peaks = attainable_peaks()
    if peaks:
        roofline["attainable"] = peaks
        if "fp64_fma_tflops" in peaks:
            roofline["frac_of_attainable"] = roofline["achieved"] / peaks["fp64_fma_tflops"]
    line = {
        "metric": "FP64 cell updates/sec",
        "value": head["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "ms_per_step_median_of_5": head["ms_per_step_median_of_5"],
        "ms_per_step_parts": head["ms_per_step_parts"],
        "fluid_cell_updates_per_s": head["fluid_cell_updates_per_s"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": head["config"],
        "roofline": roofline,
    }
    if args.workload == "dam_break" and not args.no_extras:
        # each within its stated number of steps (the drop 1000, the ensemble 500)
        extras = {}
        from paper_1806_04960_amd import scenarios as sc
        d = sc.elliptic_drop(0)
        warm = min(args.warmup, 20)
        steps = min(args.steps, 1000 - warm)
        print(f"# workload {d.name} {d.nx}x{d.ny}, warmup {warm}, steps {steps}", file=sys.stderr, flush=True)
        extras["elliptic_drop_4096x4096"] = dict(single_workload(d, steps, warm), steps=steps, warmup=warm)
        del d
        torch.cuda.empty_cache()
        steps = min(args.steps, 500 - warm)
        extras["ensemble_64"] = dict(ensemble_measure(steps, warm), steps=steps, warmup=warm)
        W = WallLoad(400)
        extras["adjoint_wall_impact_512x256"] = W.measure()
        W.close()
        line["workloads"] = extras
    if not args.no_cpu_baseline and args.cpu_baseline_steps > 0:
        line["cpu_baseline"] = cpu_baseline(s, args.cpu_baseline_steps, args.cpu_baseline_single_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
