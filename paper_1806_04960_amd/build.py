"""Build the HIP library ``libbn2d.so`` for gfx950 (in-tree, so it travels with the sources), the
attainable-peak probes ``libbn2d_probe.so`` that ``bench.py`` uses for the roofline, and
``libbn2d_timeline.so``, the library with the step kernel's per-wavefront timeline compiled in
(``python -m paper_1806_04960_amd.timeline``)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "csrc", f) for f in ("bn2d_step.hip", "bn2d_adjoint.hip", "bn2d_api.hip")]
LIB = os.path.join(HERE, "libbn2d.so")
# attainable-peak probes for the roofline (measurement only)
PROBE_SRC = [os.path.join(HERE, "csrc", "bn2d_probe.hip")]
PROBE_LIB = os.path.join(HERE, "libbn2d_probe.so")
# the same library with the step kernel's per-wavefront timeline compiled in (measurement only)
TIMELINE_LIB = os.path.join(HERE, "libbn2d_timeline.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
]


def _compile(srcs, lib, verbose, extra=()):
    tmp = lib + ".tmp"
    cmd = [HIPCC, *FLAGS, *extra, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    _compile(SRC, LIB, verbose)
    _compile(PROBE_SRC, PROBE_LIB, verbose)
    _compile(SRC, TIMELINE_LIB, verbose, ["-DBN2D_TIMELINE"])
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
