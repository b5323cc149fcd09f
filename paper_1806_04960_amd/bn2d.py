"""ctypes binding of ``libbn2d.so`` (C ABI in ``include/bn2d.h``).

Argument marshalling only: every step of the scheme runs in the HIP kernels.  Device memory and
streams come from PyTorch (ROCm); states are ``torch.float64`` CUDA tensors of shape
``[4, ny, nx]``.  There is no CPU fallback: if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# BN2D_LIB selects another build of the same ABI (e.g. to compare two kernel versions).
LIB_PATH = os.environ.get("BN2D_LIB", os.path.join(HERE, "libbn2d.so"))

BN_OK, BN_EINVAL, BN_EHIP, BN_ENONPHYS, BN_EUNSUPPORTED, BN_ENOMEM, BN_EINTERNAL = 0, -1, -2, -3, -4, -5, -6

SYMBOLS = ("bn_create", "bn_set_state", "bn_get_state", "bn_compute_dt", "bn_step", "bn_run",
           "bn_get_time", "bn_get_y0", "bn_status", "bn_set_bottom", "bn_set_launch", "bn_get_launch",
           "bn_destroy", "bn_strerror", "bn_adjoint_step", "bn_adjoint_step_noalloc", "bn_get_column_sums",
           "bn_adjoint_step_sums", "bn_batch_create",
           "bn_batch_set_state", "bn_batch_get_state", "bn_batch_run", "bn_batch_get_time", "bn_batch_get_y0",
           "bn_batch_status", "bn_batch_set_bottom", "bn_batch_set_launch", "bn_batch_get_launch",
           "bn_batch_destroy")


class BnError(RuntimeError):
    def __init__(self, code: int, where: str, text: str):
        super().__init__(f"{where}: {text} (code {code})")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("x0", ctypes.c_double),
                ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("g", ctypes.c_double), ("k0", ctypes.c_double), ("rho0", ctypes.c_double),
                ("alpha_liq", ctypes.c_double), ("alpha_gas", ctypes.c_double),
                ("cfl", ctypes.c_double), ("bc", ctypes.c_int32 * 4)]


_lib = None


def lib():
    """Load the HIP library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1806_04960_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        L.bn_create.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_uint8), vp,
                                ctypes.POINTER(vp)]
        L.bn_set_state.argtypes = [vp, vp]
        L.bn_get_state.argtypes = [vp, vp]
        L.bn_compute_dt.argtypes = [vp, dp]
        L.bn_step.argtypes = [vp, ctypes.c_double]
        L.bn_run.argtypes = [vp, ctypes.c_int32]
        L.bn_get_time.argtypes = [vp, dp, dp]
        L.bn_get_y0.argtypes = [vp, dp]
        L.bn_status.argtypes = [vp]
        L.bn_set_launch.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
        L.bn_get_launch.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.bn_destroy.argtypes = [vp]
        L.bn_destroy.restype = None
        L.bn_set_bottom.argtypes = [vp, dp]
        L.bn_adjoint_step.argtypes = [vp, vp, vp, ctypes.c_double, vp, vp, vp]
        L.bn_adjoint_step_noalloc.argtypes = [vp, vp, vp, ctypes.c_double, vp, vp, vp]
        L.bn_get_column_sums.argtypes = [vp, vp]
        L.bn_adjoint_step_sums.argtypes = [vp, vp, vp, vp, ctypes.c_double, vp, vp, vp]
        L.bn_strerror.argtypes = [ctypes.c_int]
        L.bn_strerror.restype = ctypes.c_char_p
        i32, pi32 = ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)
        L.bn_batch_create.argtypes = [i32, ctypes.POINTER(Grid), ctypes.POINTER(Params),
                                      ctypes.POINTER(ctypes.POINTER(ctypes.c_uint8)), vp, ctypes.POINTER(vp)]
        L.bn_batch_set_state.argtypes = [vp, i32, vp]
        L.bn_batch_get_state.argtypes = [vp, i32, vp]
        L.bn_batch_run.argtypes = [vp, i32]
        L.bn_batch_get_time.argtypes = [vp, i32, dp, dp]
        L.bn_batch_get_y0.argtypes = [vp, i32, dp]
        L.bn_batch_status.argtypes = [vp, pi32]
        L.bn_batch_set_bottom.argtypes = [vp, i32, dp]
        L.bn_batch_set_launch.argtypes = [vp, i32, i32]
        L.bn_batch_get_launch.argtypes = [vp, pi32, pi32]
        L.bn_batch_destroy.argtypes = [vp]
        L.bn_batch_destroy.restype = None
        for name in SYMBOLS:
            if name not in ("bn_destroy", "bn_strerror", "bn_batch_destroy"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def check(code: int, where: str):
    if code != BN_OK:
        raise BnError(code, where, lib().bn_strerror(code).decode())


def grid_of(s) -> Grid:
    return Grid(int(s.nx), int(s.ny), float(s.x0), float(s.x1), float(s.y0), float(s.y1))


def params_of(s) -> Params:
    return Params(float(s.g), float(s.k0), float(s.rho0), float(s.alpha_liq), float(s.alpha_gas),
                  float(s.cfl), (ctypes.c_int32 * 4)(*[int(b) for b in s.bc]))


class Simulation:
    """One context of the library on the current CUDA (HIP) device and stream.

    ``scenario`` provides the grid (nx, ny, x0, x1, y0, y1), the parameters (g, k0, rho0,
    alpha_liq, alpha_gas, cfl, bc), the solid mask (uint8 [ny, nx] or None) and optionally the
    columns' bottom heights (``bottom``, float64 [nx] or None; ``bn_set_bottom``)."""

    def __init__(self, scenario, stream=None, rows_per_block: int | None = None, wavefronts: int | None = None):
        import numpy as np
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU")
        self.nx, self.ny = int(scenario.nx), int(scenario.ny)
        self._scenario = scenario
        self._bottom = getattr(scenario, "bottom", None)
        self._twin = None
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        solid = None
        self._solid_keep = None
        if getattr(scenario, "solid", None) is not None:
            self._solid_keep = np.ascontiguousarray(scenario.solid, dtype=np.uint8)
            solid = self._solid_keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        ctx = ctypes.c_void_p()
        check(lib().bn_create(ctypes.byref(grid_of(scenario)), ctypes.byref(params_of(scenario)), solid,
                              ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(ctx)), "bn_create")
        self._ctx = ctx
        if getattr(scenario, "bottom", None) is not None:
            self.set_bottom(scenario.bottom)
        if rows_per_block is not None or wavefronts is not None:
            self.set_launch(rows_per_block or 0, wavefronts or 0)

    def set_bottom(self, bottom):
        """Bottom height of each column for the free-surface detector (nx values; None resets)."""
        import numpy as np
        self._bottom = None if bottom is None else np.array(bottom, dtype=np.float64)
        if self._twin is not None:
            self._twin.set_bottom(bottom)
        if bottom is None:
            check(lib().bn_set_bottom(self._ctx, None), "bn_set_bottom")
            return
        b = np.ascontiguousarray(bottom, dtype=np.float64)
        if b.shape != (self.nx,):
            raise ValueError(f"bottom must hold {self.nx} values")
        check(lib().bn_set_bottom(self._ctx, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "bn_set_bottom")

    # -- state -------------------------------------------------------------------------------
    def set_state(self, q):
        import torch
        if not (q.is_cuda and q.dtype == torch.float64 and q.is_contiguous()
                and tuple(q.shape) == (4, self.ny, self.nx)):
            raise ValueError("state must be a contiguous float64 CUDA tensor of shape [4, ny, nx]")
        check(lib().bn_set_state(self._ctx, ctypes.c_void_p(q.data_ptr())), "bn_set_state")

    def get_state(self, out=None):
        import torch
        if out is None:
            out = torch.empty((4, self.ny, self.nx), dtype=torch.float64, device="cuda")
        check(lib().bn_get_state(self._ctx, ctypes.c_void_p(out.data_ptr())), "bn_get_state")
        return out

    # -- time stepping -------------------------------------------------------------------------
    def compute_dt(self) -> float:
        dt = ctypes.c_double()
        check(lib().bn_compute_dt(self._ctx, ctypes.byref(dt)), "bn_compute_dt")
        return dt.value

    def step(self, dt: float):
        check(lib().bn_step(self._ctx, float(dt)), "bn_step")

    def run(self, n_steps: int):
        check(lib().bn_run(self._ctx, int(n_steps)), "bn_run")

    def adjoint_step(self, q, lam_next, dt: float, out=None, grad_bottom=None, src=None, sums=None):
        """lambda^n = (dQ^{n+1}/dQ^n)^T lambda^{n+1} (+ src) for the step of length dt from state q
        (``bn_adjoint_step``).  q, lam_next, src: contiguous float64 CUDA tensors [4, ny, nx].  With
        ``grad_bottom`` (a float64 CUDA tensor [nx]) also (dQ^{n+1}/dy_L)^T lambda^{n+1} of the
        columns' bottom heights.  With ``sums`` (``column_sums()`` of a context of this grid whose
        state was q) the free surface of q is taken from it (``bn_adjoint_step_sums``): the same
        result, one kernel fewer."""
        import torch
        if sums is None:
            return self._adjoint(lib().bn_adjoint_step, "bn_adjoint_step", q, lam_next, dt, out, grad_bottom, src)
        if not (sums.is_cuda and sums.dtype == torch.int64 and sums.is_contiguous() and tuple(sums.shape) == (self.nx,)):
            raise ValueError(f"sums must be a contiguous int64 CUDA tensor of shape ({self.nx},)")
        fn = lib().bn_adjoint_step_sums
        return self._adjoint(lambda ctx, qp, *rest: fn(ctx, qp, ctypes.c_void_p(sums.data_ptr()), *rest),
                             "bn_adjoint_step_sums", q, lam_next, dt, out, grad_bottom, src)

    def column_sums(self, out=None):
        """The free-surface column integrals of the current state (``bn_get_column_sums``: int64
        fixed point, [nx]) for ``adjoint_step(..., sums=...)``."""
        import torch
        if out is None:
            out = torch.empty(self.nx, dtype=torch.int64, device="cuda")
        elif not (out.is_cuda and out.dtype == torch.int64 and out.is_contiguous() and tuple(out.shape) == (self.nx,)):
            raise ValueError(f"out must be a contiguous int64 CUDA tensor of shape ({self.nx},)")
        check(lib().bn_get_column_sums(self._ctx, ctypes.c_void_p(out.data_ptr())), "bn_get_column_sums")
        return out

    def adjoint_step_noalloc(self, q, lam_next, dt: float, out, grad_bottom=None, src=None):
        """The same adjoint through ``bn_adjoint_step_noalloc``: the library's fixed scratch array,
        no allocation (the caller passes ``out``)."""
        return self._adjoint(lib().bn_adjoint_step_noalloc, "bn_adjoint_step_noalloc", q, lam_next, dt, out,
                             grad_bottom, src)

    def _adjoint(self, fn, name, q, lam_next, dt, out, grad_bottom, src=None):
        import torch
        shape = (4, self.ny, self.nx)
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device="cuda")
        for arg, t in (("q", q), ("lam_next", lam_next), ("out", out)) + ((("src", src),) if src is not None else ()):
            if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == shape):
                raise ValueError(f"{arg} must be a contiguous float64 CUDA tensor of shape {shape}")
        gb = None
        if grad_bottom is not None:
            if not (grad_bottom.is_cuda and grad_bottom.dtype == torch.float64 and grad_bottom.is_contiguous()
                    and tuple(grad_bottom.shape) == (self.nx,)):
                raise ValueError(f"grad_bottom must be a contiguous float64 CUDA tensor of shape ({self.nx},)")
            gb = ctypes.c_void_p(grad_bottom.data_ptr())
        sp = None if src is None else ctypes.c_void_p(src.data_ptr())
        check(fn(self._ctx, ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(lam_next.data_ptr()), float(dt),
                 ctypes.c_void_p(out.data_ptr()), gb, sp), name)
        return out

    def time(self):
        t, dt = ctypes.c_double(), ctypes.c_double()
        check(lib().bn_get_time(self._ctx, ctypes.byref(t), ctypes.byref(dt)), "bn_get_time")
        return t.value, dt.value

    def y0(self):
        import numpy as np
        out = np.zeros(self.nx)
        check(lib().bn_get_y0(self._ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "bn_get_y0")
        return out

    def status(self):
        check(lib().bn_status(self._ctx), "bn_status")

    def set_launch(self, rows_per_block: int = 0, wavefronts: int = 0):
        """Launch shape of the step kernel (0 = default for either)."""
        check(lib().bn_set_launch(self._ctx, int(rows_per_block), int(wavefronts)), "bn_set_launch")

    def launch(self):
        """(rows per block, wavefronts) of the step kernel."""
        r, w = ctypes.c_int32(), ctypes.c_int32()
        check(lib().bn_get_launch(self._ctx, ctypes.byref(r), ctypes.byref(w)), "bn_get_launch")
        return r.value, w.value

    def twin(self):
        """A second context of the same grid, model and bottoms on a stream of its own (kept with
        this one): trajectory gradients recompute their segments on it while this context's stream
        runs the adjoint steps."""
        import torch
        if self._twin is None:
            t = Simulation(self._scenario, stream=torch.cuda.Stream(), rows_per_block=self.launch()[0],
                           wavefronts=self.launch()[1])
            if self._bottom is not None:
                t.set_bottom(self._bottom)
            self._twin = t
        return self._twin

    def close(self):
        if getattr(self, "_twin", None) is not None:
            self._twin.close()
            self._twin = None
        if getattr(self, "_ctx", None):
            lib().bn_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """A batch of independent grids advanced together (``bn_batch_*``): one launch per step,
    each member with its own CFL time step.  ``scenarios`` is a list of scenario objects as for
    ``Simulation``."""

    def __init__(self, scenarios, stream=None, rows_per_block: int | None = None, wavefronts: int | None = None):
        import numpy as np
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU")
        n = len(scenarios)
        self.shapes = [(int(s.ny), int(s.nx)) for s in scenarios]
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        grids = (Grid * n)(*[grid_of(s) for s in scenarios])
        params = (Params * n)(*[params_of(s) for s in scenarios])
        self._solid_keep = []
        solids = (ctypes.POINTER(ctypes.c_uint8) * n)()
        for k, s in enumerate(scenarios):
            if getattr(s, "solid", None) is not None:
                m = np.ascontiguousarray(s.solid, dtype=np.uint8)
                self._solid_keep.append(m)
                solids[k] = m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        b = ctypes.c_void_p()
        check(lib().bn_batch_create(n, grids, params, solids, ctypes.c_void_p(self._stream.cuda_stream),
                                    ctypes.byref(b)), "bn_batch_create")
        self._b = b
        for k, s in enumerate(scenarios):
            if getattr(s, "bottom", None) is not None:
                bot = np.ascontiguousarray(s.bottom, dtype=np.float64)
                check(lib().bn_batch_set_bottom(self._b, k, bot.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                      "bn_batch_set_bottom")
        if rows_per_block is not None or wavefronts is not None:
            check(lib().bn_batch_set_launch(self._b, int(rows_per_block or 0), int(wavefronts or 0)),
                  "bn_batch_set_launch")

    def __len__(self):
        return len(self.shapes)

    def set_state(self, member: int, q):
        import torch
        ny, nx = self.shapes[member]
        if not (q.is_cuda and q.dtype == torch.float64 and q.is_contiguous() and tuple(q.shape) == (4, ny, nx)):
            raise ValueError("state must be a contiguous float64 CUDA tensor of shape [4, ny, nx]")
        check(lib().bn_batch_set_state(self._b, int(member), ctypes.c_void_p(q.data_ptr())), "bn_batch_set_state")

    def get_state(self, member: int):
        import torch
        ny, nx = self.shapes[member]
        out = torch.empty((4, ny, nx), dtype=torch.float64, device="cuda")
        check(lib().bn_batch_get_state(self._b, int(member), ctypes.c_void_p(out.data_ptr())), "bn_batch_get_state")
        return out

    def run(self, n_steps: int):
        check(lib().bn_batch_run(self._b, int(n_steps)), "bn_batch_run")

    def time(self, member: int):
        t, dt = ctypes.c_double(), ctypes.c_double()
        check(lib().bn_batch_get_time(self._b, int(member), ctypes.byref(t), ctypes.byref(dt)), "bn_batch_get_time")
        return t.value, dt.value

    def y0(self, member: int):
        import numpy as np
        out = np.zeros(self.shapes[member][1])
        check(lib().bn_batch_get_y0(self._b, int(member), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
              "bn_batch_get_y0")
        return out

    def status(self):
        m = ctypes.c_int32(-1)
        code = lib().bn_batch_status(self._b, ctypes.byref(m))
        if code != BN_OK:
            raise BnError(code, f"bn_batch_status (member {m.value})", lib().bn_strerror(code).decode())

    def launch(self):
        r, w = ctypes.c_int32(), ctypes.c_int32()
        check(lib().bn_batch_get_launch(self._b, ctypes.byref(r), ctypes.byref(w)), "bn_batch_get_launch")
        return r.value, w.value

    def close(self):
        if getattr(self, "_b", None):
            lib().bn_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def step_function():
    """A ``torch.autograd.Function`` for one step of fixed length: ``StepFn.apply(sim, q, dt)``
    returns the state after one step from q (through ``bn_set_state`` and ``bn_step``, so it
    resets the context's state and time), and its backward is ``bn_adjoint_step``.  Long
    trajectories are differentiated with checkpoints and recomputation by the caller."""
    import torch

    class StepFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, sim, q, dt):
            q = q.detach().contiguous()
            sim.set_state(q)
            sim.step(float(dt))
            ctx.sim, ctx.dt = sim, float(dt)
            ctx.save_for_backward(q)
            return sim.get_state()

        @staticmethod
        def backward(ctx, grad_out):
            (q,) = ctx.saved_tensors
            lam = ctx.sim.adjoint_step(q, grad_out.contiguous(), ctx.dt)
            return None, lam, None

    return StepFn


def _segment_buffers(sim, like, seg: int):
    """Two sets of buffers for the states of a segment after its checkpoint (seg - 1 states) and the
    free-surface column sums of all its states (seg), one set per segment in flight."""
    import torch

    bufs = [[torch.empty_like(like) for _ in range(max(seg - 1, 0))] for _ in range(2)]
    sums = [[torch.empty(sim.nx, dtype=torch.int64, device=like.device) for _ in range(seg)] for _ in range(2)]
    return bufs, sums


def _trajectory_forward(sim, q0, dt: float, N: int, w, seg: int, with_loss: bool, last=None):
    """N steps of length dt from q0: the loss sum_n <w, Q^n> (if asked) and the checkpoints.  With
    ``last`` = (states, sums), one buffer set of ``_segment_buffers``, the states of the last segment
    and the column sums of its states are kept there as they are computed, so that the reverse sweep
    need not recompute that segment before it can start."""
    import torch

    C = 1 + (N - 1) // seg if N > 0 else 1
    n0 = (C - 1) * seg  # the last segment's first state
    ck = [q0.detach().clone()]
    sim.set_state(ck[0])
    if last is not None and n0 == 0:
        sim.column_sums(out=last[1][0])
    J = torch.zeros((), dtype=torch.float64, device=q0.device)
    for k in range(N):
        sim.step(dt)
        m = k + 1  # the state just computed
        keep = m % seg == 0 and m < N
        if with_loss or keep:
            q = sim.get_state()
            if with_loss:
                J += (w * q).sum()
            if keep:
                ck.append(q)
        if last is not None and n0 <= m < N:
            if m > n0:
                sim.get_state(out=last[0][m - n0 - 1])
            sim.column_sums(out=last[1][m - n0])
    return J, ck


def _trajectory_reverse(sim, ck, dt: float, N: int, w, seg: int, gbot=None, buffers=None, last_ready=False):
    """dJ/dq0 from the checkpoints: each segment, last first, recomputed and reversed (and, into
    ``gbot`` if given, the sum over the steps of the bottom heights' adjoints).  The segments are
    recomputed on the context's twin, on a stream of its own, one segment ahead of the reverse sweep
    on the context's stream: segment c - 1 is recomputed while segment c is reversed (two sets of
    state buffers; events order a set's reuse after the sweep that reads it).  ``buffers``: the sets
    of ``_segment_buffers``; with ``last_ready`` the last segment's set was filled by the forward run
    (``_trajectory_forward(..., last=...)``) and is not recomputed."""
    import torch

    twin = sim.twin()
    sa, sb = sim._stream, twin._stream
    lam = w.clone() if N > 0 else torch.zeros_like(w)  # dJ/dQ^N
    # one row of bottom adjoints per step, summed once at the end
    gsteps = None if gbot is None else torch.empty((N, gbot.numel()), dtype=gbot.dtype, device=gbot.device)
    C = len(ck)
    sizes = [min(seg, N - c * seg) for c in range(C)]
    # the free-surface column sums of every state of a segment come from the twin that recomputes it
    # (its step computed them), so that the reverse sweep does not compute them again
    bufs, sums = buffers if buffers is not None else _segment_buffers(sim, ck[0], seg)
    ev_rec = [torch.cuda.Event() for _ in range(C)]
    ev_rev = [torch.cuda.Event() for _ in range(C)]
    # (the checkpoints and weights were written on the context's stream)
    sb.wait_stream(sa)

    def recompute(c):
        twin.set_state(ck[c])
        twin.column_sums(out=sums[c % 2][0])
        for k in range(1, sizes[c]):
            twin.step(dt)
            twin.get_state(out=bufs[c % 2][k - 1])
            twin.column_sums(out=sums[c % 2][k])
        ev_rec[c].record(sb)

    if last_ready:
        ev_rec[C - 1].record(sa)
    else:
        recompute(C - 1)
    for c in range(C - 1, -1, -1):
        if c >= 1:
            if c + 1 < C:
                sb.wait_event(ev_rev[c + 1])  # set (c - 1) % 2 was read by the sweep of segment c + 1
            recompute(c - 1)
        sa.wait_event(ev_rec[c])
        n0 = c * seg
        for k in range(sizes[c] - 1, -1, -1):
            q = ck[c] if k == 0 else bufs[c % 2][k - 1]
            # lam = dJ/dQ^{n0+k+1} in; out dJ/dQ^{n0+k}, with that step's own term w added (none for q0)
            lam = sim.adjoint_step(q, lam, dt, grad_bottom=None if gsteps is None else gsteps[n0 + k],
                                   src=w if n0 + k > 0 else None, sums=sums[c % 2][k])
        ev_rev[c].record(sa)
    sa.wait_stream(sb)
    if gbot is not None and N > 0:
        gbot += gsteps.sum(dim=0)
    sim.set_state(ck[0])
    return lam


def _check_trajectory(N, seg, q0, weights):
    import torch

    if int(N) < 0 or int(seg) < 1:
        raise ValueError("n_steps >= 0 and segment >= 1 required")
    for name, t in (("q0", q0), ("weights", weights)):
        if t.dtype != torch.float64 or not t.is_cuda:
            raise ValueError(f"{name} must be a float64 CUDA tensor")
    if weights.shape != q0.shape:
        raise ValueError("weights must have the shape of the state")
    return int(N), int(seg)


def trajectory_gradient(sim, q0, dt: float, n_steps: int, weights, segment: int = 20, with_loss: bool = False,
                        store_all: bool = False, bottom: bool = False):
    """Gradient of J = sum_{n=1..N} <weights, Q^n> over N steps of fixed length dt from q0 with
    respect to q0, by the discrete adjoint (``bn_adjoint_step``): the forward run keeps the state
    every ``segment`` steps, then each segment, last first, is recomputed from its checkpoint and
    reversed step by step.  Memory: N/segment + segment states.  With ``store_all`` the forward run
    keeps every state instead (N states, no recomputation: one forward step fewer per step where
    device memory allows it).  Returns dJ/dq0, or (J, dJ/dq0) with ``with_loss`` (J then also costs a
    reduction per forward step); with ``bottom`` also dJ/dy_L of the columns' bottom heights
    (bn_set_bottom), appended to the result.  Leaves the context at q0 (its elapsed time
    restarted)."""
    import torch

    N, seg = _check_trajectory(n_steps, segment, q0, weights)
    w = weights.contiguous()
    dt = float(dt)
    gbot = torch.zeros(sim.nx, dtype=torch.float64, device=q0.device) if bottom else None

    def result(J, lam):
        out = (float(J), lam) if with_loss else (lam,)
        out = out + ((gbot,) if bottom else ())
        return out if len(out) > 1 else out[0]

    if store_all:
        states = [q0.detach().clone()]
        sim.set_state(states[0])
        sums = [sim.column_sums()]
        J = torch.zeros((), dtype=torch.float64, device=q0.device)
        for k in range(N):
            sim.step(dt)
            if with_loss or k + 1 < N:
                q = sim.get_state()
                if with_loss:
                    J += (w * q).sum()
                if k + 1 < N:
                    states.append(q)
                    sums.append(sim.column_sums())
        lam = w.clone() if N > 0 else torch.zeros_like(w)  # dJ/dQ^N
        gsteps = torch.empty((N, sim.nx), dtype=torch.float64, device=q0.device) if bottom else None
        for n in range(N - 1, -1, -1):
            lam = sim.adjoint_step(states[n], lam, dt, grad_bottom=None if gsteps is None else gsteps[n],
                                   src=w if n > 0 else None, sums=sums[n])
        if bottom and N > 0:
            gbot += gsteps.sum(dim=0)
        sim.set_state(states[0])
        return result(J, lam)
    buffers = _segment_buffers(sim, q0, seg)
    C = 1 + (N - 1) // seg if N > 0 else 1
    J, ck = _trajectory_forward(sim, q0, dt, N, w, seg, with_loss,
                                last=(buffers[0][(C - 1) % 2], buffers[1][(C - 1) % 2]))
    lam = _trajectory_reverse(sim, ck, dt, N, w, seg, gbot, buffers=buffers, last_ready=True)
    return result(J, lam)


def trajectory_loss_function():
    """A ``torch.autograd.Function`` for the same loss: ``TrajLoss.apply(sim, q0, dt, n_steps,
    weights, segment)`` returns J = sum_{n=1..N} <weights, Q^n> (a 0-dim tensor) from a forward run
    that keeps the checkpoints; its backward recomputes each segment and runs the discrete adjoint
    (the gradient reaches q0 only; weights, dt and the model are constants)."""
    import torch

    class TrajLoss(torch.autograd.Function):
        @staticmethod
        def forward(ctx, sim, q0, dt, n_steps, weights, segment=20):
            N, seg = _check_trajectory(n_steps, segment, q0, weights)
            w = weights.detach().contiguous()
            J, ck = _trajectory_forward(sim, q0.detach().contiguous(), float(dt), N, w, seg, True)
            ctx.sim, ctx.dt, ctx.N, ctx.seg, ctx.w, ctx.ck = sim, float(dt), N, seg, w, ck
            return J

        @staticmethod
        def backward(ctx, grad_out):
            lam = _trajectory_reverse(ctx.sim, ctx.ck, ctx.dt, ctx.N, ctx.w, ctx.seg)
            ctx.ck = None
            return None, grad_out * lam, None, None, None, None

    return TrajLoss


def tune_launch(obj, steps: int = 30, shapes=None):
    """Choose the launch shape (rows per claim, wavefronts) of a ``Simulation`` or ``Batch`` by
    timing ``steps`` steps of each candidate on its current state(s), set the fastest and restore
    the state(s) (through set_state, which also resets the elapsed times).  Results do not depend
    on the shape, only the time per step does.  Returns (rows_per_block, wavefronts, {shape: ms})."""
    import torch

    batch = isinstance(obj, Batch)
    members = range(len(obj)) if batch else [None]
    saved = [obj.get_state(k) for k in members] if batch else [obj.get_state()]

    def restore():
        if batch:
            for k, q in zip(members, saved):
                obj.set_state(k, q)
        else:
            obj.set_state(saved[0])

    set_launch = (lambda r, w: check(lib().bn_batch_set_launch(obj._b, r, w), "bn_batch_set_launch")) if batch \
        else obj.set_launch
    set_launch(0, 0)
    r0, w0 = obj.launch()
    if shapes is None:
        waves = sorted({max(64, w0 // 4), max(64, w0 // 2), w0, min(65536, 2 * w0)} | {w for w in (512, 1024, 2048)
                                                                                         if w <= 2 * w0})
        shapes = [(r, w) for w in waves for r in (2, 4, 8)]
    times = {}
    ev = lambda: torch.cuda.Event(enable_timing=True)
    for r, w in shapes:
        set_launch(int(r), int(w))
        restore()
        obj.run(3)
        a, b = ev(), ev()
        torch.cuda.synchronize()
        a.record()
        obj.run(steps)
        b.record()
        torch.cuda.synchronize()
        times[(r, w)] = a.elapsed_time(b) / steps
    best = min(times, key=times.get)
    set_launch(int(best[0]), int(best[1]))
    restore()
    return best[0], best[1], times
