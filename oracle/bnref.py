"""ctypes binding of the CPU oracle (``oracle/bnref.c``).

TEST INFRASTRUCTURE, NOT PRODUCT CODE: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this module.  The product path (the HIP library in
``paper_1806_04960_amd``) never imports, links or calls it.

Every function takes a *scenario*: any object with the attributes ``nx, ny, x0, x1, y0, y1``
(grid), ``g, k0, rho0, alpha_liq, alpha_gas, cfl, bc`` (parameters), ``solid``
(``uint8 [ny, nx]`` or ``None``) and optionally ``bottom`` (``float64 [nx]``: each column's bottom
height for the free-surface detector, or ``None``).  States are ``float64 [4, ny, nx]`` arrays holding
(alpha rho, alpha rho u, alpha rho v, alpha).
"""
from __future__ import annotations

import copy
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bnref.c")
LIB = os.path.join(HERE, "libbnref.so")

CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]

OK, EINVAL, ENONPHYS, EUNSUPPORTED = 0, -1, -3, -4


class OracleError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"oracle {where} failed with code {code}")
        self.code = code


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("x0", ctypes.c_double),
                ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("g", ctypes.c_double), ("k0", ctypes.c_double), ("rho0", ctypes.c_double),
                ("alpha_liq", ctypes.c_double), ("alpha_gas", ctypes.c_double),
                ("cfl", ctypes.c_double), ("bc", ctypes.c_int32 * 4)]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU code involved)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _bind(path):
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    dp = P(ctypes.c_double)
    u8p = P(ctypes.c_uint8)
    gp, pp = P(_Grid), P(_Params)
    L.bnref_detector.argtypes = [gp, pp, u8p, dp, dp, dp]
    L.bnref_cfl.argtypes = [gp, pp, u8p, dp, dp, dp]
    L.bnref_step.argtypes = [gp, pp, u8p, dp, dp, ctypes.c_double, dp]
    L.bnref_step_cells.argtypes = [gp, pp, u8p, dp, dp, ctypes.c_double, ctypes.c_int64,
                                   P(ctypes.c_int64), dp]
    L.bnref_run.argtypes = [gp, pp, u8p, dp, dp, ctypes.c_int32, dp, dp]
    L.bnref_flux.argtypes = [pp, ctypes.c_int32, dp, dp]
    L.bnref_matrix.argtypes = [pp, ctypes.c_int32, ctypes.c_int32, dp, dp]
    L.bnref_fluct.argtypes = [pp, ctypes.c_int32, dp, dp, dp, dp, dp, dp]
    L.bnref_reconstruct.argtypes = [gp, pp, u8p, dp, dp, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_double, dp, dp, dp, dp]
    for name in ("bnref_detector", "bnref_cfl", "bnref_step", "bnref_step_cells", "bnref_run",
                 "bnref_flux", "bnref_matrix", "bnref_fluct", "bnref_reconstruct"):
        getattr(L, name).restype = ctypes.c_int
    L.bnref_threads.argtypes = []
    L.bnref_threads.restype = ctypes.c_int
    L.bnref_set_threads.argtypes = [ctypes.c_int32]
    L.bnref_set_threads.restype = None
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = _bind(LIB)
    return _lib


def threads() -> int:
    """Threads the oracle's row sweeps use (OpenMP; results do not depend on it)."""
    return int(lib().bnref_threads())


def set_threads(n: int) -> None:
    lib().bnref_set_threads(int(n))


# The literal forms of three passages that the oracle reads differently (compile-time switches of
# bnref.c, off in the oracle itself); built on demand, for the tests that show why.
VARIANTS = {
    "roe_velocity": "BNREF_LITERAL_ROE_VELOCITY",
    "cell_switch": "BNREF_LITERAL_CELL_SWITCH",
    "own_equilibrium": "BNREF_LITERAL_OWN_EQUILIBRIUM",
}


class Variant:
    """The oracle built with one literal-form switch: the same functions as this module."""

    def __init__(self, name: str, out_dir: str):
        path = os.path.join(out_dir, f"libbnref_{name}.so")
        subprocess.check_call(["gcc", *CFLAGS, f"-D{VARIANTS[name]}", "-o", path, SRC, "-lm"])
        self.name = name
        self._L = _bind(path)

    def step(self, s, q, dt):
        return step(s, q, dt, L=self._L)

    def run(self, s, q, n_steps):
        return run(s, q, n_steps, L=self._L)

    def cfl(self, s, q):
        return cfl(s, q, L=self._L)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _grid(s) -> _Grid:
    return _Grid(int(s.nx), int(s.ny), float(s.x0), float(s.x1), float(s.y0), float(s.y1))


def params_struct(s) -> _Params:
    bc = (ctypes.c_int32 * 4)(*[int(b) for b in s.bc])
    return _Params(float(s.g), float(s.k0), float(s.rho0), float(s.alpha_liq), float(s.alpha_gas),
                   float(s.cfl), bc)


def _solid(s):
    if getattr(s, "solid", None) is None:
        return None, None
    a = np.ascontiguousarray(s.solid, dtype=np.uint8)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _bottom(s):
    b = getattr(s, "bottom", None)
    if b is None:
        return None, None
    b = np.ascontiguousarray(b, dtype=np.float64)
    if b.shape != (s.nx,):
        raise ValueError(f"bottom shape {b.shape} != ({s.nx},)")
    return b, _dp(b)


def _state(s, q) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float64)
    if q.shape != (4, s.ny, s.nx):
        raise ValueError(f"state shape {q.shape} != (4, {s.ny}, {s.nx})")
    return q


def _check(rc: int, where: str):
    if rc < 0:
        raise OracleError(rc, where)


def detector(s, q) -> np.ndarray:
    q = _state(s, q)
    keep, sp = _solid(s)
    keepb, bp = _bottom(s)
    y0 = np.zeros(s.nx)
    _check(lib().bnref_detector(_grid(s), params_struct(s), sp, bp, _dp(q), _dp(y0)), "detector")
    return y0


def cfl(s, q, L=None):
    """Return (lambda_max, dt)."""
    q = _state(s, q)
    keep, sp = _solid(s)
    lam, dt = ctypes.c_double(), ctypes.c_double()
    _check((L or lib()).bnref_cfl(_grid(s), params_struct(s), sp, _dp(q), ctypes.byref(lam), ctypes.byref(dt)),
           "cfl")
    return lam.value, dt.value


def step(s, q, dt: float, L=None) -> np.ndarray:
    q = _state(s, q)
    keep, sp = _solid(s)
    keepb, bp = _bottom(s)
    out = np.empty_like(q)
    _check((L or lib()).bnref_step(_grid(s), params_struct(s), sp, bp, _dp(q), float(dt), _dp(out)), "step")
    return out


def step_cells(s, q, dt: float, cells) -> np.ndarray:
    """Q^{n+1} at the flat cell indices ``cells`` (j*nx + i); returns [4, len(cells)]."""
    q = _state(s, q)
    keep, sp = _solid(s)
    keepb, bp = _bottom(s)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.empty((4, cells.size))
    _check(lib().bnref_step_cells(_grid(s), params_struct(s), sp, bp, _dp(q), float(dt), cells.size,
                                  cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(out)),
           "step_cells")
    return out


def run(s, q, n_steps: int, L=None):
    """Advance ``n_steps`` CFL steps; returns (state, elapsed time, last dt)."""
    q = _state(s, q).copy()
    keep, sp = _solid(s)
    keepb, bp = _bottom(s)
    t, dt = ctypes.c_double(), ctypes.c_double()
    _check((L or lib()).bnref_run(_grid(s), params_struct(s), sp, bp, _dp(q), int(n_steps), ctypes.byref(t),
                           ctypes.byref(dt)), "run")
    return q, t.value, dt.value


def adjoint_fd(s, q, lam, dt: float, h=1e-6) -> np.ndarray:
    """Adjoint of one step with time step dt at state q, by its definition: (dF/dq)^T lam with
    F = step(., dt), the Jacobian taken column by column by central differences.  The perturbation
    of an entry is h times its cell's own scale (|alpha rho| for alpha rho, |alpha rho| x 1 m/s for
    the momenta, so that it stays small against gas and liquid values alike; 1 for alpha, whose
    perturbation reaches every liquid cell of its column through the free surface);
    the truncation error is O(h^2) away from the scheme's non-smooth points.  One pair of full
    steps per state entry: small grids only.  h: one relative step, or one per component."""
    q = _state(s, q)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    hs = np.broadcast_to(np.asarray(h, dtype=np.float64), (4,))
    out = np.zeros_like(q)
    for k in range(4):
        for j in range(s.ny):
            for i in range(s.nx):
                hk = hs[k] * (1.0 if k == 3 else abs(q[0, j, i]))
                qp = q.copy()
                qm = q.copy()
                qp[k, j, i] += hk
                qm[k, j, i] -= hk
                diff = step(s, qp, dt) - step(s, qm, dt)
                out[k, j, i] = float(np.sum(lam * diff)) / (2.0 * hk)
    return out


def adjoint_fd_bottom(s, q, lam, dt: float, columns, h=1e-6) -> np.ndarray:
    """Gradient of <lam, step(q, dt)> with respect to the bottom heights of ``columns`` (the
    scenario's ``bottom``, the detector's y_L), by central differences of the step (h in metres).
    The bottoms must stay within half a cell of their solid runs' tops at +-h."""
    q = _state(s, q)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    base = np.asarray(s.bottom, dtype=np.float64)
    out = np.zeros(len(columns))
    for n, i in enumerate(columns):
        sp_, sm_ = copy.copy(s), copy.copy(s)
        sp_.bottom = base.copy()
        sm_.bottom = base.copy()
        sp_.bottom[i] += h
        sm_.bottom[i] -= h
        out[n] = float(np.sum(lam * (step(sp_, q, dt) - step(sm_, q, dt)))) / (2.0 * h)
    return out


# ---- pieces used by the oracle's own pins --------------------------------------------------

def flux(s, direction: int, q5) -> np.ndarray:
    q5 = np.ascontiguousarray(q5, dtype=np.float64)
    out = np.zeros(5)
    _check(lib().bnref_flux(params_struct(s), int(direction), _dp(q5), _dp(out)), "flux")
    return out


def matrix(s, direction: int, kind: str, q5) -> np.ndarray:
    kinds = {"A": 0, "R": 1, "lambda": 2, "Rinv": 3, "absA": 4, "signA": 5}
    q5 = np.ascontiguousarray(q5, dtype=np.float64)
    out = np.zeros(5 if kind == "lambda" else 25)
    _check(lib().bnref_matrix(params_struct(s), int(direction), kinds[kind], _dp(q5), _dp(out)), "matrix")
    return out if kind == "lambda" else out.reshape(5, 5)


def fluct(s, direction: int, qm, qp, em=None, ep=None):
    """Edge fluctuations (D-, D+) between 5-component states qm, qp (y also needs E-parts)."""
    qm = np.ascontiguousarray(qm, dtype=np.float64)
    qp = np.ascontiguousarray(qp, dtype=np.float64)
    em = None if em is None else np.ascontiguousarray(em, dtype=np.float64)
    ep = None if ep is None else np.ascontiguousarray(ep, dtype=np.float64)
    dm, dp = np.zeros(5), np.zeros(5)
    _check(lib().bnref_fluct(params_struct(s), int(direction), _dp(qm), _dp(em), _dp(qp), _dp(ep),
                             _dp(dm), _dp(dp)), "fluct")
    return dm, dp


def reconstruct(s, q, i: int, j: int, dt: float):
    """Reconstruction of cell (i, j): dict of faces [4,5] (W,E,S,N), eparts, centre, gx, gy, so."""
    q = _state(s, q)
    keep, sp = _solid(s)
    keepb, bp = _bottom(s)
    faces, ep, centre, grad = np.zeros((4, 5)), np.zeros((4, 5)), np.zeros(5), np.zeros(8)
    rc = lib().bnref_reconstruct(_grid(s), params_struct(s), sp, bp, _dp(q), int(i), int(j), float(dt),
                                 _dp(faces), _dp(ep), _dp(centre), _dp(grad))
    _check(rc, "reconstruct")
    return {"faces": faces, "eparts": ep, "centre": centre, "gx": grad[:4], "gy": grad[4:], "so": bool(rc)}
