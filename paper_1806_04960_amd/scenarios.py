"""Seeded synthetic initial conditions for the explicit well-balanced step.

This module produces *inputs only*: grids, parameters, solid masks and the initial state
Q = (alpha rho, alpha rho u, alpha rho v, alpha) laid out as ``float64 [4, ny, nx]`` (x fastest).
It holds none of the scheme's arithmetic; both the HIP library and the CPU oracle consume
what it writes.

Initial conditions follow the paper's test section (Sec. 5): two-level volume fraction
(1 - eps in the liquid, eps in the gas, or 1 where a test says so), u = 0 and rho = rho0 in
the gas, and in the liquid the water-at-rest density rho0 exp(-g rho0/k0 (y - y0(x)))
(Sec. 5.5, same profile as Sec. 2.1), where y0(x) is the free surface of the rasterised liquid
column.  A cell is solid / liquid iff its centre lies in the closed region.  The free-surface
height of a column is written as (y_lo + n_solid dy) + dy * n_liquid, which is the value the
free-surface detector returns for two-level alpha, so a liquid at rest starts exactly on the
discrete equilibrium.  The exponential is evaluated with the C library's ``exp``
(``math.exp``), the same routine the oracle calls.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

EPS = 1e-3      # alpha of the gas and 1 - alpha of the liquid (Sec. 5)
CFL = 0.9       # CFL number of every workload
RHO0 = 1000.0   # reference density (Sec. 5)
GRAV = 9.81


@dataclass
class Scenario:
    name: str
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float
    y1: float
    g: float = GRAV
    k0: float = 6.54e5
    rho0: float = RHO0
    alpha_liq: float = 1.0 - EPS
    alpha_gas: float = EPS
    cfl: float = CFL
    bc: tuple = (0, 0, 0, 0)          # W, E, S, N: 0 reflective, 1 transmissive
    solid: np.ndarray | None = None   # uint8 [ny, nx], 1 = solid
    bottom: np.ndarray | None = None  # float64 [nx]: bottom height of each column (obstacle tops) or None
    q: np.ndarray | None = None       # float64 [4, ny, nx]
    steps: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def dx(self) -> float:
        return (self.x1 - self.x0) / self.nx

    @property
    def dy(self) -> float:
        return (self.y1 - self.y0) / self.ny

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    def xc(self) -> np.ndarray:
        return self.x0 + (np.arange(self.nx) + 0.5) * self.dx

    def yc(self) -> np.ndarray:
        return self.y0 + (np.arange(self.ny) + 0.5) * self.dy

    def fluid(self) -> np.ndarray:
        return np.ones((self.ny, self.nx), bool) if self.solid is None else self.solid == 0

    def copy(self) -> "Scenario":
        return replace(self, solid=None if self.solid is None else self.solid.copy(),
                       bottom=None if self.bottom is None else self.bottom.copy(),
                       q=None if self.q is None else self.q.copy(), meta=dict(self.meta))

    def solid_tops(self) -> np.ndarray:
        """Top of each column's bottom-attached solid run (the grid-aligned bottom)."""
        if self.solid is None:
            return np.full(self.nx, self.y0)
        jb = np.where((self.solid == 0).any(axis=0), np.argmax(self.solid == 0, axis=0), self.ny)
        return self.y0 + jb * self.dy


def _rect(s: Scenario, xa, xb, ya, yb) -> np.ndarray:
    X, Y = np.meshgrid(s.xc(), s.yc())
    return (X >= xa) & (X <= xb) & (Y >= ya) & (Y <= yb)


def _fill(s: Scenario, liquid: np.ndarray, u=None, v=None) -> Scenario:
    """Two-level alpha, hydrostatic density in bottom-attached liquid columns, rho0 elsewhere."""
    fluid = s.fluid()
    liquid = liquid & fluid
    alpha = np.where(liquid, s.alpha_liq, s.alpha_gas)
    rho = np.full((s.ny, s.nx), s.rho0)
    a = s.g * s.rho0 / s.k0
    dy = s.dy
    yc = s.yc()
    for i in range(s.nx):
        col_f = fluid[:, i]
        jb = 0
        while jb < s.ny and not col_f[jb]:
            jb += 1
        if np.any(~col_f[jb:]):
            raise ValueError(f"column {i}: solid above fluid is not supported")
        n_liq = int(liquid[:, i].sum())
        y_surf = (s.y0 + jb * dy) + dy * float(n_liq)
        for j in range(jb, s.ny):
            if liquid[j, i]:
                if not yc[j] < y_surf:
                    raise ValueError(f"column {i}: liquid is not attached to the bottom")
                rho[j, i] = s.rho0 * math.exp(-a * (yc[j] - y_surf))
    q = np.zeros((4, s.ny, s.nx))
    q[0] = alpha * rho
    uu = np.zeros((s.ny, s.nx)) if u is None else np.where(liquid, u, 0.0)
    vv = np.zeros((s.ny, s.nx)) if v is None else np.where(liquid, v, 0.0)
    q[1] = q[0] * uu
    q[2] = q[0] * vv
    q[3] = alpha
    # solid cells hold a benign gas state; they are never read by the scheme
    gas = np.array([s.alpha_gas * s.rho0, 0.0, 0.0, s.alpha_gas])
    q[:, ~fluid] = gas[:, None]
    s.q = q
    return s


def _fill_free(s: Scenario, liquid: np.ndarray, u, v) -> Scenario:
    """Liquid region not attached to the bottom (g = 0 tests): rho = rho0 everywhere."""
    if s.g != 0.0:
        raise ValueError("a floating liquid region needs g = 0")
    fluid = s.fluid()
    liquid = liquid & fluid
    alpha = np.where(liquid, s.alpha_liq, s.alpha_gas)
    q = np.zeros((4, s.ny, s.nx))
    q[0] = alpha * s.rho0
    q[1] = q[0] * np.where(liquid, u, 0.0)
    q[2] = q[0] * np.where(liquid, v, 0.0)
    q[3] = alpha
    s.q = q
    return s


# ---------------------------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------------------------

def rest_with_obstacle(nx: int = 128, ny: int = 64) -> Scenario:
    """Water at rest in a closed 2 m x 1 m tank: liquid (alpha = 1) below y = 0.5 around a
    rectangular obstacle [0.8, 1.2] x [0, 0.3], gas (alpha = 1e-3) above.  k0 = 2.78e5 (the
    paper's equilibrium test, Sec. 5.1)."""
    s = Scenario("rest_obstacle", nx, ny, 0.0, 2.0, 0.0, 1.0, k0=2.78e5, alpha_liq=1.0, cfl=CFL,
                 steps=200)
    s.solid = _rect(s, 0.8, 1.2, 0.0, 0.3).astype(np.uint8)
    X, Y = np.meshgrid(s.xc(), s.yc())
    return _fill(s, Y < 0.5)


def rest_flat(nx: int = 128, ny: int = 64) -> Scenario:
    s = Scenario("rest_flat", nx, ny, 0.0, 2.0, 0.0, 1.0, k0=2.78e5, alpha_liq=1.0, cfl=CFL,
                 steps=200)
    X, Y = np.meshgrid(s.xc(), s.yc())
    return _fill(s, Y < 0.5)


def dam_break_small(nx: int = 128, ny: int = 64) -> Scenario:
    """128 x 64 dam break in a closed 2 m x 1 m tank, liquid column 0.5 m x 0.5 m in the left
    corner, alpha = 1 - eps in the liquid (Sec. 3.4), k0 = 2.78e5."""
    s = Scenario("dam_break_small", nx, ny, 0.0, 2.0, 0.0, 1.0, k0=2.78e5, steps=200)
    return _fill(s, _rect(s, 0.0, 0.5, 0.0, 0.5))


def dam_break(seed: int = 0, nx: int = 2048, ny: int = 1024) -> Scenario:
    """Dam break with an obstacle on a 4 m x 2 m closed tank (headline workload at 2048 x 1024).
    Column width W ~ U[0.8, 1.2], height H ~ U[0.5, 1.0] at the left wall; obstacle
    [3.0, 3.1] x [0, h], h ~ U[0.05, 0.2]; k0 = 6.54e5 (the M = 0.3 value of Sec. 5.5/5.6)."""
    rng = np.random.default_rng(seed)
    W, H, h = rng.uniform(0.8, 1.2), rng.uniform(0.5, 1.0), rng.uniform(0.05, 0.2)
    s = Scenario("dam_break", nx, ny, 0.0, 4.0, 0.0, 2.0, k0=6.54e5, steps=2000,
                 meta={"seed": seed, "W": W, "H": H, "h_obstacle": h})
    s.solid = _rect(s, 3.0, 3.1, 0.0, h).astype(np.uint8)
    return _fill(s, _rect(s, 0.0, W, 0.0, H))


def weir(nx: int = 800, ny: int = 250) -> Scenario:
    """Flow over a sharp-crested weir (Sec. 5.5 set-up): [-7.5, 7.5] x [0, 2.1], a one-cell-thick
    solid strip of height 0.7 in the first column right of x = 0, liquid (alpha = 1 - eps) at rest
    in [-7.5, 0] x [0, 1.5] with the hydrostatic density, dry (gas) right of the weir, k0 = 6.54e5,
    reflective walls.  The paper's 800 x 250 mesh by default."""
    s = Scenario("weir", nx, ny, -7.5, 7.5, 0.0, 2.1, k0=6.54e5, steps=0)
    solid = np.zeros((ny, nx), np.uint8)
    iw = int(np.searchsorted(s.xc(), 0.0))      # first cell whose centre is right of x = 0
    solid[s.yc() <= 0.7, iw] = 1
    s.solid = solid
    s.meta = {"weir_column": iw, "crest": 0.7}
    return _fill(s, _rect(s, -7.5, 0.0, 0.0, 1.5))


def elliptic_drop(seed: int = 0, nx: int = 4096, ny: int = 4096) -> Scenario:
    """Oscillating elliptical drop without gravity on [-1, 1]^2 (Sec. 5.2 set-up, rescaled):
    semi-axes 0.5 (1 + da) along x and 0.25 (1 + db) along y, d ~ U[-0.02, 0.02];
    u = -100 x, v = 100 y in the liquid, rho = rho0, k0 = 2.25e9 (c = 1500 m/s)."""
    rng = np.random.default_rng(seed)
    da, db = rng.uniform(-0.02, 0.02, size=2)
    a, b = 0.5 * (1 + da), 0.25 * (1 + db)
    s = Scenario("elliptic_drop", nx, ny, -1.0, 1.0, -1.0, 1.0, g=0.0, k0=2.25e9, steps=1000,
                 meta={"seed": seed, "a": a, "b": b})
    X, Y = np.meshgrid(s.xc(), s.yc())
    liquid = (X / a) ** 2 + (Y / b) ** 2 <= 1.0
    return _fill_free(s, liquid, -100.0 * X, 100.0 * Y)


def circular_drop(nx: int = 100, ny: int = 100, radius: float = 1.0, half_width: float = 3.0) -> Scenario:
    """The paper's drop (Sec. 5.2): circle r = 1 in [-3, 3]^2, u = (-100 x, 100 y), g = 0,
    k0 = 2.25e9, alpha = 1 - eps."""
    s = Scenario("circular_drop", nx, ny, -half_width, half_width, -half_width, half_width, g=0.0,
                 k0=2.25e9)
    X, Y = np.meshgrid(s.xc(), s.yc())
    return _fill_free(s, X ** 2 + Y ** 2 <= radius ** 2, -100.0 * X, 100.0 * Y)


def equilibrium_box(obstacle: bool, nx: int = 100, ny: int = 100) -> Scenario:
    """Sec. 5.1: [-0.5, 0.5] x [0, 1] full of liquid (alpha = 1), k0 = 2.78e5, optionally
    minus the obstacle [-0.25, 0.25] x [0, 0.33]."""
    s = Scenario("equilibrium_obstacle" if obstacle else "equilibrium_flat", nx, ny, -0.5, 0.5, 0.0, 1.0,
                 k0=2.78e5, alpha_liq=1.0, cfl=CFL)
    if obstacle:
        s.solid = _rect(s, -0.25, 0.25, 0.0, 0.33).astype(np.uint8)
    return _fill(s, np.ones((ny, nx), bool))


ENSEMBLE_SIZES = ((256, 128), (512, 256), (768, 384), (1024, 512))


def ensemble(seed: int = 0, count: int = 64, sizes=ENSEMBLE_SIZES):
    """Batch of uneven dam breaks on a 4 m x 2 m tank: sizes drawn from {256x128, 512x256,
    768x384, 1024x512} (or the given list); H ~ U[0.3, 1.0], W ~ U[0.3, 1.2]; 0-2 obstacles
    0.1 m wide at x ~ U[W + 0.2, 3.8] with heights U[0.05, 0.3]; k0 = 6.54e5; 500 steps each."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        nx, ny = sizes[int(rng.integers(0, len(sizes)))]
        H, W = rng.uniform(0.3, 1.0), rng.uniform(0.3, 1.2)
        n_obs = int(rng.integers(0, 3))
        s = Scenario(f"ensemble_{k}", nx, ny, 0.0, 4.0, 0.0, 2.0, k0=6.54e5, steps=500,
                     meta={"seed": seed, "member": k, "H": H, "W": W})
        solid = np.zeros((ny, nx), bool)
        for o in range(n_obs):
            xo, ho = rng.uniform(W + 0.2, 3.8), rng.uniform(0.05, 0.3)
            solid |= _rect(s, xo, xo + 0.1, 0.0, ho)
        s.solid = solid.astype(np.uint8) if solid.any() else None
        out.append(_fill(s, _rect(s, 0.0, W, 0.0, H)))
    return out


def wall_impact(seed: int = 0, nx: int = 512, ny: int = 256, n_theta: int = 64, theta=None,
                wall_height: float = 0.4):
    """Reservoir released against a wall, the adjoint workload: [0,4] x [0,2], free-surface profile
    h(x) piecewise linear through theta_k = 0.6 + 0.1 U(-1, 1) at x_k = 3.5 k / (n_theta - 1);
    alpha is the liquid volume fraction of each cell below h(x_i) (two-level away from the surface,
    fractional in the cell the surface cuts); a one-cell solid wall of height 0.4 in the first
    column right of x = 3.5 (cells whose centre lies below its top are solid; the free-surface
    detector takes the top itself as that column's bottom, so that the loss is differentiable in
    it); dry (gas) right of it.  Hydrostatic density below each column's free surface (the
    detector's value), k0 = 6.54e5, at rest.  The profile values are kept in meta["theta"];
    ``theta`` given replaces the seeded ones (gradient checks); ``wall_height`` moves the wall's
    top (within the cell that holds it)."""
    rng = np.random.default_rng(seed)
    theta = 0.6 + 0.1 * rng.uniform(-1.0, 1.0, n_theta) if theta is None else np.asarray(theta, float)
    n_theta = theta.size
    s = Scenario("wall_impact", nx, ny, 0.0, 4.0, 0.0, 2.0, k0=6.54e5, steps=400,
                 meta={"seed": seed, "theta": theta.tolist()})
    xc = s.xc()
    iw = int(np.nonzero(xc > 3.5)[0][0])
    solid = np.zeros((ny, nx), np.uint8)
    solid[s.yc() < 0.4, iw] = 1
    s.solid = solid
    s.meta["wall_column"] = iw
    s.meta["wall_height"] = float(wall_height)
    s.bottom = s.solid_tops()
    s.bottom[iw] = wall_height
    if not abs(wall_height - s.solid_tops()[iw]) < 0.5 * s.dy:
        raise ValueError("wall_height must lie within half a cell of the wall's rasterised top")
    hx = np.interp(xc, 3.5 * np.arange(n_theta) / (n_theta - 1), theta)
    hx[xc >= 3.5] = 0.0
    ybot = s.y0 + np.arange(ny) * s.dy
    frac = np.clip((hx[None, :] - ybot[:, None]) / s.dy, 0.0, 1.0)
    frac[solid == 1] = 0.0
    alpha = s.alpha_gas + frac * (s.alpha_liq - s.alpha_gas)
    a = s.g * s.rho0 / s.k0
    yc = s.yc()
    rho = np.full((ny, nx), s.rho0)
    for i in range(nx):
        col_f = solid[:, i] == 0
        jb = int(np.argmax(col_f)) if col_f.any() else ny
        base = s.y0 + jb * s.dy
        y_surf = base + s.dy * float(frac[:, i].sum())
        if jb < ny:  # the detector's value with the column's bottom (the wall's top)
            y_surf += (s.bottom[i] - base) * (1.0 - float(frac[jb, i]))
        liq = col_f & (yc < y_surf)
        rho[liq, i] = s.rho0 * np.exp(-a * (yc[liq] - y_surf))
    q = np.zeros((4, ny, nx))
    q[0] = alpha * rho
    q[3] = alpha
    gas = np.array([s.alpha_gas * s.rho0, 0.0, 0.0, s.alpha_gas])
    q[:, solid == 1] = gas[:, None]
    s.q = q
    return s


def tank_with_wall(top: float, surface: float = 0.5, nx: int = 40, ny: int = 32, column: int = 13,
                   offset: float = 0.0) -> Scenario:
    """Water at rest below ``surface`` in a closed 2 m x 1 m tank (g = 9.81, k0 = 2.78e5, alpha = 1 in
    the liquid), with a one-column wall in ``column`` whose cells below ``top`` (by their centres) are
    solid; the column's bottom height for the free-surface detector is the top of that solid run plus
    ``offset`` cells (a wall top off the grid)."""
    s = Scenario("tank_wall", nx, ny, 0.0, 2.0, 0.0, 1.0, k0=2.78e5, alpha_liq=1.0)
    solid = np.zeros((ny, nx), np.uint8)
    solid[s.yc() < top, column] = 1
    s.solid = solid
    X, Y = np.meshgrid(s.xc(), s.yc())
    s = _fill(s, Y <= surface)
    s.bottom = s.solid_tops()
    s.bottom[column] += offset * s.dy
    return s


def wall_impact_theta_vjp(s: Scenario, lam0) -> np.ndarray:
    """dJ/dtheta from dJ/dq0 (``lam0``, [4, ny, nx]) for a ``wall_impact`` state: the chain rule
    through its construction, with the same switches held fixed as it takes them (which cells the
    surface cuts, which cells are liquid).  h(x_i) = sum_k L_k(x_i) theta_k with the hat functions
    of the linear interpolation; in a column, d frac/dh = 1/dy in the cut cell, the surface height
    moves with h one for one, alpha = a_g + frac (a_l - a_g), and the liquid density
    rho0 exp(-a (y - y_surf)) moves by a rho per unit of surface height."""
    lam0 = np.asarray(lam0, dtype=float)
    theta = np.asarray(s.meta["theta"], dtype=float)
    n_theta = theta.size
    xk = 3.5 * np.arange(n_theta) / (n_theta - 1)
    xc, yc = s.xc(), s.yc()
    ybot = s.y0 + np.arange(s.ny) * s.dy
    a = s.g * s.rho0 / s.k0
    alpha, q0 = s.q[3], s.q[0]
    rho = q0 / alpha
    solid = s.solid if s.solid is not None else np.zeros((s.ny, s.nx), np.uint8)
    dJdh = np.zeros(s.nx)
    for i in range(s.nx):
        if xc[i] >= 3.5:
            continue
        h = float(np.interp(xc[i], xk, theta))
        z = (h - ybot) / s.dy
        cut = (z > 0.0) & (z < 1.0) & (solid[:, i] == 0)
        dfrac = np.where(cut, 1.0 / s.dy, 0.0)
        dalpha = dfrac * (s.alpha_liq - s.alpha_gas)
        col_f = solid[:, i] == 0
        jb = int(np.argmax(col_f)) if col_f.any() else s.ny
        y_surf = (s.y0 + jb * s.dy) + s.dy * float(np.clip(z[col_f], 0.0, 1.0).sum())
        dysurf = s.dy * float(dfrac.sum())
        liq = col_f & (yc < y_surf)
        drho = np.where(liq, a * rho[:, i] * dysurf, 0.0)
        dq0 = rho[:, i] * dalpha + alpha[:, i] * drho
        dJdh[i] = float(lam0[0, :, i] @ dq0 + lam0[3, :, i] @ dalpha)
    # h_i = sum_k L_k(x_i) theta_k: the transpose of the interpolation
    grad = np.zeros(n_theta)
    for i in range(s.nx):
        if xc[i] >= 3.5 or dJdh[i] == 0.0:
            continue
        k = min(int(np.searchsorted(xk, xc[i], side="right")) - 1, n_theta - 2)
        w1 = (xc[i] - xk[k]) / (xk[k + 1] - xk[k])
        grad[k] += (1.0 - w1) * dJdh[i]
        grad[k + 1] += w1 * dJdh[i]
    return grad


# ---------------------------------------------------------------------------------------------
# Small cases for the oracle's pins and the parity tests
# ---------------------------------------------------------------------------------------------

def uniform_tank(nx: int, ny: int, x0=0.0, x1=1.0, y0=0.0, y1=1.0, *, g=0.0, k0=2.78e5,
                 alpha=1.0, alpha_liq=1.0, alpha_gas=EPS, bc=(0, 0, 0, 0), rho=None, u=None,
                 v=None) -> Scenario:
    """A box full of one phase with prescribed primitive fields (arrays [ny, nx] or scalars)."""
    s = Scenario("uniform_tank", nx, ny, x0, x1, y0, y1, g=g, k0=k0, alpha_liq=alpha_liq,
                 alpha_gas=alpha_gas, bc=tuple(bc))
    shape = (ny, nx)
    al = np.broadcast_to(np.asarray(alpha, float), shape)
    r = np.broadcast_to(np.asarray(RHO0 if rho is None else rho, float), shape)
    uu = np.broadcast_to(np.asarray(0.0 if u is None else u, float), shape)
    vv = np.broadcast_to(np.asarray(0.0 if v is None else v, float), shape)
    q = np.zeros((4, ny, nx))
    q[0] = al * r
    q[1] = q[0] * uu
    q[2] = q[0] * vv
    q[3] = al
    s.q = q
    return s


def random_state(s: Scenario, seed: int, amp: float = 0.05, vel: float = 3.0) -> Scenario:
    """Perturb a scenario's fluid cells with seeded noise (parity of generic, non-equilibrium
    states): rho by +-amp relative, velocities by +-vel m/s in the liquid, alpha unchanged."""
    rng = np.random.default_rng(seed)
    q = s.q.copy()
    fluid = s.fluid()
    alpha = q[3]
    rho = q[0] / alpha
    rho = rho * (1.0 + amp * rng.uniform(-1, 1, rho.shape))
    liq = alpha > 10 * s.alpha_gas
    u = np.where(liq, vel * rng.uniform(-1, 1, rho.shape), 0.0)
    v = np.where(liq, vel * rng.uniform(-1, 1, rho.shape), 0.0)
    q[0] = np.where(fluid, alpha * rho, q[0])
    q[1] = np.where(fluid, q[0] * u, q[1])
    q[2] = np.where(fluid, q[0] * v, q[2])
    out = s.copy()
    out.q = q
    out.name = s.name + f"_noise{seed}"
    return out


def generic_state(s: Scenario, seed: int, rel: float = 1e-3, vel: float = 0.05) -> Scenario:
    """A state near s.q with no two cells alike (for derivative checks, which need the scheme to be
    differentiable: equal neighbours sit on the limiter's min/max ties, velocities near zero on the
    kinks of |u| and sign(v)): every fluid cell's alpha rho scaled by 1 + rel U(-1, 1), alpha by
    1 - rel U(0, 1), and u, v shifted by vel (1 + U(0, 1)), a drift away from zero."""
    rng = np.random.default_rng(seed)
    q = s.q.copy()
    fl = s.fluid()
    shape = (s.ny, s.nx)
    u = np.where(q[0] != 0, q[1] / q[0], 0.0) + vel * (1.0 + rng.uniform(0, 1, shape))
    v = np.where(q[0] != 0, q[2] / q[0], 0.0) + vel * (1.0 + rng.uniform(0, 1, shape))
    ar = q[0] * (1.0 + rel * rng.uniform(-1, 1, shape))
    al = q[3] * (1.0 - rel * rng.uniform(0, 1, shape))
    q[0] = np.where(fl, ar, q[0])
    q[1] = np.where(fl, ar * u, q[1])
    q[2] = np.where(fl, ar * v, q[2])
    q[3] = np.where(fl, al, q[3])
    out = s.copy()
    out.q = q
    out.name = s.name + f"_generic{seed}"
    return out


def smooth_state(s: Scenario, amp: float = 1e-3, vel: float = 0.05) -> Scenario:
    """A smooth, physically consistent departure from s.q for trajectory derivative checks: in
    liquid cells (alpha > 1/2) alpha and alpha rho both scaled by 1 - amp/10 (1 + sin(2 pi x / 0.31
    + 1.1) sin(2 pi y / 0.19 + 0.4)) (density unchanged), then alpha rho by 1 + amp sin(2 pi x /
    0.37 + 0.3) sin(2 pi y / 0.23 + 0.7), and a smooth velocity field (vel (1 + 0.5 sin), vel (1 +
    0.5 cos)); gas cells drift uniformly at (vel, vel).  Neighbouring liquid cells then differ in
    every component (no limiter min/max ties, as a fluid at rest has), while the gas keeps its
    density (a noisy gas density makes pressure jumps that the light phase cannot carry)."""
    X, Y = np.meshgrid(s.xc(), s.yc())
    q = s.q.copy()
    fl = s.fluid()
    liq = fl & (q[3] > 0.5)
    gas = fl & ~liq
    frac = 1.0 - 0.1 * amp * (1.0 + np.sin(2 * np.pi * X / 0.31 + 1.1) * np.sin(2 * np.pi * Y / 0.19 + 0.4))
    q[3] = np.where(liq, q[3] * frac, q[3])
    wave = np.sin(2 * np.pi * X / 0.37 + 0.3) * np.sin(2 * np.pi * Y / 0.23 + 0.7)
    ar = np.where(liq, q[0] * frac * (1.0 + amp * wave), q[0])
    u = np.where(liq, vel * (1.0 + 0.5 * np.sin(2 * np.pi * (X + Y) / 0.41)), np.where(gas, vel, 0.0))
    v = np.where(liq, vel * (1.0 + 0.5 * np.cos(2 * np.pi * (X - Y) / 0.29)), np.where(gas, vel, 0.0))
    q[0] = ar
    q[1] = np.where(fl, ar * u, q[1])
    q[2] = np.where(fl, ar * v, q[2])
    out = s.copy()
    out.q = q
    out.name = s.name + "_smooth"
    return out


def smooth_state_vjp(s: Scenario, lam, amp: float = 1e-3, vel: float = 0.05) -> np.ndarray:
    """dJ/d(s.q) from dJ/d(smooth_state(s).q): the transpose of smooth_state's Jacobian, with its
    liquid/gas split held fixed.  Liquid: alpha' = f alpha, (alpha rho)' = f w alpha rho and the
    momenta (alpha rho)' times the (fixed) velocity field; gas: momenta alpha rho times vel."""
    lam = np.asarray(lam, dtype=float)
    X, Y = np.meshgrid(s.xc(), s.yc())
    q = s.q
    fl = s.fluid()
    liq = fl & (q[3] > 0.5)
    gas = fl & ~liq
    frac = 1.0 - 0.1 * amp * (1.0 + np.sin(2 * np.pi * X / 0.31 + 1.1) * np.sin(2 * np.pi * Y / 0.19 + 0.4))
    wave = np.sin(2 * np.pi * X / 0.37 + 0.3) * np.sin(2 * np.pi * Y / 0.23 + 0.7)
    u = np.where(liq, vel * (1.0 + 0.5 * np.sin(2 * np.pi * (X + Y) / 0.41)), np.where(gas, vel, 0.0))
    v = np.where(liq, vel * (1.0 + 0.5 * np.cos(2 * np.pi * (X - Y) / 0.29)), np.where(gas, vel, 0.0))
    dar = np.where(liq, frac * (1.0 + amp * wave), 1.0)  # d(alpha rho)'/d(alpha rho)
    out = lam.copy()
    lam_ar = lam[0] + np.where(fl, lam[1] * u + lam[2] * v, 0.0)
    out[0] = np.where(fl, lam_ar * dar, lam[0])
    out[1] = np.where(fl, 0.0, lam[1])
    out[2] = np.where(fl, 0.0, lam[2])
    out[3] = np.where(liq, lam[3] * frac, lam[3])
    return out


def scaled(builder, nx: int, ny: int, **kw) -> Scenario:
    return builder(nx=nx, ny=ny, **kw)
