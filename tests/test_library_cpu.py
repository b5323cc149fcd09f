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


def test_timeline_instrumentation_only_in_its_own_build():
    """The step kernel's per-wavefront timeline (BN2D_TIMELINE) is compiled into
    libbn2d_timeline.so alone: the default library neither exports its reader nor differs in ABI."""
    L = bn2d.lib()
    assert not hasattr(L, "bn_timeline_read")
    path = os.path.join(ROOT, "paper_1806_04960_amd", "libbn2d_timeline.so")
    if not os.path.exists(path):
        pytest.skip("libbn2d_timeline.so not built")
    T = ctypes.CDLL(path)
    assert hasattr(T, "bn_timeline_read")
    for name in declared_symbols():
        assert hasattr(T, name), name
    T.bn_timeline_read.argtypes = [ctypes.c_void_p, ctypes.c_int]
    assert T.bn_timeline_read(None, 1) == -1  # rejected before any HIP call


def test_binding_declares_every_signature():
    """Every entry point has its ctypes argument types (a call without them fails on a double
    argument), with as many arguments as the header's prototype."""
    L = bn2d.lib()
    text = open(os.path.join(ROOT, "include", "bn2d.h")).read()
    for name in bn2d.SYMBOLS:
        m = re.search(r"\b" + name + r"\s*\(([^)]*)\)", text)
        n_args = len([a for a in m.group(1).split(",") if a.strip() and a.strip() != "void"])
        assert getattr(L, name).argtypes is not None, name
        assert len(getattr(L, name).argtypes) == n_args, name


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


def _batch_create(scens, solids=None):
    L = bn2d.lib()
    n = len(scens)
    grids = (bn2d.Grid * n)(*[bn2d.grid_of(s) for s in scens])
    params = (bn2d.Params * n)(*[bn2d.params_of(s) for s in scens])
    sp = None
    keep = []
    if solids is not None:
        sp = (ctypes.POINTER(ctypes.c_uint8) * n)()
        for k, m in enumerate(solids):
            if m is not None:
                m = np.ascontiguousarray(m, dtype=np.uint8)
                keep.append(m)
                sp[k] = m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    out = ctypes.c_void_p()
    return L.bn_batch_create(n, grids, params, sp, None, ctypes.byref(out)), out


def test_batch_create_rejects_any_bad_member():
    good = sc.uniform_tank(4, 4)
    bad = sc.uniform_tank(4, 4)
    bad.cfl = 2.0
    rc, b = _batch_create([good, bad, good])
    assert rc == bn2d.BN_EINVAL and not b.value
    solid = np.zeros((4, 4), np.uint8)
    solid[3, 0] = 1  # solid above fluid in column 0
    rc, b = _batch_create([good, good], [None, solid])
    assert rc == bn2d.BN_EUNSUPPORTED and not b.value


def test_batch_null_arguments_and_bad_counts():
    L = bn2d.lib()
    out = ctypes.c_void_p()
    g = (bn2d.Grid * 1)(bn2d.grid_of(sc.uniform_tank(4, 4)))
    p = (bn2d.Params * 1)(bn2d.params_of(sc.uniform_tank(4, 4)))
    assert L.bn_batch_create(0, g, p, None, None, ctypes.byref(out)) == bn2d.BN_EINVAL
    assert L.bn_batch_create(-1, g, p, None, None, ctypes.byref(out)) == bn2d.BN_EINVAL
    assert L.bn_batch_create(1, None, p, None, None, ctypes.byref(out)) == bn2d.BN_EINVAL
    assert L.bn_batch_create(1, g, None, None, None, ctypes.byref(out)) == bn2d.BN_EINVAL
    assert L.bn_batch_create(1, g, p, None, None, None) == bn2d.BN_EINVAL
    assert L.bn_batch_set_state(None, 0, None) == bn2d.BN_EINVAL
    assert L.bn_batch_get_state(None, 0, None) == bn2d.BN_EINVAL
    assert L.bn_batch_run(None, 1) == bn2d.BN_EINVAL
    assert L.bn_batch_get_time(None, 0, None, None) == bn2d.BN_EINVAL
    assert L.bn_batch_get_y0(None, 0, None) == bn2d.BN_EINVAL
    assert L.bn_batch_status(None, None) == bn2d.BN_EINVAL
    assert L.bn_batch_set_launch(None, 0, 0) == bn2d.BN_EINVAL
    assert L.bn_batch_get_launch(None, None, None) == bn2d.BN_EINVAL
    L.bn_batch_destroy(None)


@pytest.mark.parametrize("nx,ny", [(0x7FFF * 60 + 1, 4), (4, 0xFF0000 + 1)])
def test_create_rejects_grids_beyond_the_descriptor_fields(nx, ny):
    s = sc.uniform_tank(4, 4)
    s.nx, s.ny = nx, ny
    rc, ctx = _create(s)
    assert rc == bn2d.BN_EINVAL and not ctx.value


def test_batch_create_rejects_too_many_strips_in_total():
    # each member alone is within the limit, together they are not; rejected before allocating
    a = sc.uniform_tank(4, 4)
    a.nx = 0x7FFF * 60
    rc, out = _batch_create([a, sc.uniform_tank(4, 4)])
    assert rc == bn2d.BN_EINVAL and not out.value


def test_trajectory_gradient_rejects_bad_arguments():
    import torch
    q = torch.zeros((4, 2, 2), dtype=torch.float64)
    with pytest.raises(ValueError, match="n_steps"):
        bn2d.trajectory_gradient(None, q, 1.0, -1, q)
    with pytest.raises(ValueError, match="segment"):
        bn2d.trajectory_gradient(None, q, 1.0, 3, q, segment=0)
    with pytest.raises(ValueError, match="CUDA"):
        bn2d.trajectory_gradient(None, q, 1.0, 3, q)
