"""The C-ABI library loads and exports every entry point include/bn2d.h declares; argument
checks that run before any HIP call behave as documented (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1806_04960_amd import bn2d, scenarios as sc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "bn2d.h")).read()
    return sorted(set(re.findall(r"\b(bn_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_binding_symbols():
    assert set(declared_symbols()) == set(bn2d.SYMBOLS)


def test_library_exports_every_declared_symbol():
    L = bn2d.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_strerror_names_every_code():
    L = bn2d.lib()
    for code in (0, -1, -2, -3, -4, -5, -6, -99):
        assert L.bn_strerror(code)


def _create(s, solid=None):
    ctx = ctypes.c_void_p()
    sp = None
    if solid is not None:
        solid = np.ascontiguousarray(solid, dtype=np.uint8)
        sp = solid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    rc = bn2d.lib().bn_create(ctypes.byref(bn2d.grid_of(s)), ctypes.byref(bn2d.params_of(s)), sp, None,
                              ctypes.byref(ctx))
    return rc, ctx


@pytest.mark.parametrize("field,value", [("nx", 0), ("ny", -3), ("cfl", 0.0), ("cfl", 1.5), ("k0", -1.0),
                                         ("alpha_gas", 0.0), ("alpha_liq", 1e-4), ("alpha_liq", 1.2)])
def test_create_rejects_bad_arguments(field, value):
    s = sc.uniform_tank(4, 4)
    setattr(s, field, value)
    rc, ctx = _create(s)
    assert rc == bn2d.BN_EINVAL and not ctx.value


def test_create_rejects_bad_boundary_code():
    s = sc.uniform_tank(4, 4, bc=(0, 2, 0, 0))
    rc, ctx = _create(s)
    assert rc == bn2d.BN_EINVAL


def test_create_rejects_solid_above_fluid():
    s = sc.uniform_tank(4, 4)
    solid = np.zeros((4, 4), np.uint8)
    solid[2, 1] = 1
    rc, ctx = _create(s, solid)
    assert rc == bn2d.BN_EUNSUPPORTED and not ctx.value


def test_null_arguments():
    L = bn2d.lib()
    assert L.bn_create(None, None, None, None, None) == bn2d.BN_EINVAL
    assert L.bn_step(None, 1.0) == bn2d.BN_EINVAL
    assert L.bn_run(None, 1) == bn2d.BN_EINVAL
    assert L.bn_set_state(None, None) == bn2d.BN_EINVAL
    assert L.bn_status(None) == bn2d.BN_EINVAL
    assert L.bn_set_launch(None, 0, 0) == bn2d.BN_EINVAL
    assert L.bn_get_launch(None, None, None) == bn2d.BN_EINVAL
    L.bn_destroy(None)
