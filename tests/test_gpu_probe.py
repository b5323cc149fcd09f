"""The reciprocal the physics uses on the GPU (the hardware estimate refined by one Newton step) against
the correctly rounded quotient 1/x, over 4 M log-uniformly spaced x in [1e-8, 1e8] (the range of
densities, volume fractions and their products that the scheme divides by): within 16 ulps, i.e.
3.6e-15 relative, far inside the 1e-11 parity budget.  (Probe library built beside the HIP library.)"""
import ctypes
import math
import os

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_reciprocal_is_within_16_ulps():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L = ctypes.CDLL(os.path.join(ROOT, "paper_1806_04960_amd", "libbn2d_probe.so"))
    L.bn_probe_rcp.argtypes = [ctypes.c_longlong, ctypes.c_double, ctypes.c_double,
                               ctypes.POINTER(ctypes.c_ulonglong)]
    L.bn_probe_rcp.restype = ctypes.c_int
    worst = ctypes.c_ulonglong()
    lo, hi = math.log2(1e-8), math.log2(1e8)
    assert L.bn_probe_rcp(1 << 22, lo, hi, ctypes.byref(worst)) == 0
    print(f"reciprocal: at most {worst.value} ulps over 4 M inputs in [1e-8, 1e8]", flush=True)
    assert worst.value <= 16
