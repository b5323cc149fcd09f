"""Per-wavefront timeline of the step kernel, from the instrumented build ``libbn2d_timeline.so``
(``build.py`` compiles it with BN2D_TIMELINE; the default library has no instrumentation).

After ``--warmup`` steps of a workload, each of ``--steps`` single steps is traced: per wavefront the
real-time clock (100 MHz) at entry, after the strip totals, after its strip's table entry, after its
row costs, after locating its range, after its own range and at exit, its own range and its steals.
Printed per traced step (microseconds from the first wavefront's entry): medians and percentiles of
those points, the own ranges' rows and durations, the latest own ranges and exits, and the median end of the
own ranges per wavefront residue mod 8 (workgroups are dealt to the 8 XCDs in turn).  The
instrumentation adds its clock reads and one record store per wavefront, so its launches run a few
percent longer than the default library's.

    python -m paper_1806_04960_amd.timeline [--workload dam_break|elliptic_drop] [--warmup 20] [--steps 3]
"""
import argparse
import ctypes
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
WORDS = 16
TICK_US = 0.01  # 100 MHz


def quantile(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, int(q * len(v)))]


def summarise(rec):
    """rec: one list of WORDS words per wavefront (one step).  Returns a dict of figures in us."""
    t0 = min(r[0] for r in rec)
    us = lambda x: (x - t0) * TICK_US
    start = [us(r[0]) for r in rec]
    located = [us(r[4]) for r in rec]
    own_end = [us(r[5]) for r in rec]
    exit_ = [us(r[6]) for r in rec]
    split = [r for r in rec if r[2] and r[3]]
    parts = {
        "strip_totals": [(r[1] - r[0]) * TICK_US for r in split],
        "cut_search_and_strip_entry": [(r[2] - r[1]) * TICK_US for r in split],
        "row_costs": [(r[3] - r[2]) * TICK_US for r in split],
        "rest_of_locating": [(r[4] - r[3]) * TICK_US for r in split],
    }
    own = [r for r in rec if r[9] > 0]
    dur = [(r[5] - r[4]) * TICK_US for r in own]
    latest = sorted(((us(r[5]), w, int(r[7]), int(r[8]), int(r[8]) + int(r[9])) for w, r in enumerate(rec) if r[9] > 0),
                    reverse=True)[:8]
    last_exits = sorted(((us(r[6]), us(r[5]) if r[5] else None, w, int(r[10])) for w, r in enumerate(rec)),
                        reverse=True)[:8]
    by_xcd = [statistics.median([own_end[w] for w in range(x, len(rec), 8)]) for x in range(8)]
    pct = lambda v: {"median": statistics.median(v), "p90": quantile(v, 0.9), "p99": quantile(v, 0.99), "max": max(v)}
    return {
        "wavefronts": len(rec),
        "launch_end": max(exit_),
        "start": pct(start),
        "located": pct(located),
        "own_range_end": pct(own_end),
        "exit": pct(exit_),
        "locating_parts_median": {k: statistics.median(v) for k, v in parts.items() if v},
        "own_range_rows_median": statistics.median([int(r[9]) for r in own]),
        "own_range_duration": pct(dur),
        "steals_total": int(sum(r[10] for r in rec)),
        "latest_own_ranges": [{"end": e, "wavefront": w, "strip": g, "rows": [a, b]} for e, w, g, a, b in latest],
        "latest_exits": [{"exit": e, "own_range_end": o, "wavefront": w, "steals": n} for e, o, w, n in last_exits],
        "own_range_end_median_by_wavefront_mod_8": by_xcd,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="dam_break", choices=["dam_break", "elliptic_drop"])
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--steps", type=int, default=3)
    args = ap.parse_args()

    path = os.path.join(HERE, "libbn2d_timeline.so")
    if not os.path.exists(path):
        sys.exit(f"{path} is not built (python -m paper_1806_04960_amd.build)")
    os.environ["BN2D_LIB"] = path  # the binding loads the instrumented build
    import numpy as np
    import torch

    from paper_1806_04960_amd import bn2d
    from paper_1806_04960_amd import scenarios as sc

    if not torch.cuda.is_available():
        sys.exit("no GPU visible")
    L = bn2d.lib()
    L.bn_timeline_read.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.bn_timeline_read.restype = ctypes.c_int
    s = sc.dam_break(0) if args.workload == "dam_break" else sc.elliptic_drop(0)
    with bn2d.Simulation(s) as sim:
        sim.set_state(torch.from_numpy(s.q).cuda())
        sim.run(args.warmup)
        sim.status()
        P = sim.launch()[1]
        for k in range(args.steps):
            sim.run(1)
            torch.cuda.synchronize()
            buf = np.zeros(P * WORDS, dtype=np.uint64)
            if L.bn_timeline_read(buf.ctypes.data, P) != 0:
                sys.exit("bn_timeline_read failed")
            rec = buf.reshape(P, WORDS).astype(np.int64).tolist()
            out = {"workload": f"{s.name} {s.nx}x{s.ny}", "step": args.warmup + k + 1, **summarise(rec)}
            print(json.dumps(out), flush=True)
        sim.status()


if __name__ == "__main__":
    main()
