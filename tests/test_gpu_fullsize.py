"""GPU parity at the workloads' full sizes and stated step counts.

Each workload runs on the GPU for its stated number of steps (the 2048 x 1024 dam break 2000 CFL
steps, the 4096 x 4096 elliptical drop 1000, the 512 x 256 wall impact 400 steps of its fixed time
step, the 64-member ensemble 500 steps of each member's own CFL step).  From the GPU's state at
that point the GPU takes one more step, and the oracle takes the same step from the same state
(with its own CFL time step, or the fixed one) on sampled cells: at least half of them on the
liquid/gas band (all of it where it holds fewer cells), beside solid cells and at the domain
walls, the rest spread uniformly.  The
oracle's time step must match the GPU's next one.  Then full-grid trajectories from the initial
states: the dam break over 100 steps and the drop over 10 steps, every cell of every field.

Tolerance: max relative error 1e-11 per field, normalised as in the other parity tests (the
momenta by max |alpha rho u| of the oracle, at least rho0 alpha_l times 1 m/s).
"""
import time

import numpy as np
import pytest

from paper_1806_04960_amd import scenarios as sc
from tests.parity import TOL, field_errors

pytestmark = pytest.mark.gpu
N_SAMPLED = 6000


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def bn(torch_cuda):
    from paper_1806_04960_amd import bn2d
    bn2d.lib()
    return bn2d


def sample_cells(s, q, n, seed):
    """n cells of state q: half on the liquid/gas band (alpha strictly between the two levels, or
    a jump of alpha to a neighbour), a quarter beside solid cells or on the domain's walls, the
    rest uniform; fluid cells only."""
    rng = np.random.default_rng(seed)
    fluid = s.fluid()
    a = q[3]
    band = (a > 2 * s.alpha_gas) & (a < 0.5 * (1 + s.alpha_liq) - 0.01)
    jump = np.zeros_like(band)
    dx = np.abs(np.diff(a, axis=1)) > 0.05
    dyy = np.abs(np.diff(a, axis=0)) > 0.05
    jump[:, :-1] |= dx
    jump[:, 1:] |= dx
    jump[:-1, :] |= dyy
    jump[1:, :] |= dyy
    band = (band | jump) & fluid
    wall = np.zeros_like(band)
    wall[0, :] = wall[-1, :] = wall[:, 0] = wall[:, -1] = True
    if s.solid is not None:
        sol = s.solid.astype(bool)
        near = np.zeros_like(sol)
        near[:, :-1] |= sol[:, 1:]
        near[:, 1:] |= sol[:, :-1]
        near[:-1, :] |= sol[1:, :]
        near[1:, :] |= sol[:-1, :]
        near[:-1, :-1] |= sol[1:, 1:]
        near[1:, 1:] |= sol[:-1, :-1]
        near[:-1, 1:] |= sol[1:, :-1]
        near[1:, :-1] |= sol[:-1, 1:]
        wall |= near
    wall &= fluid

    def pick(mask, k):
        idx = np.flatnonzero(mask)
        return idx if idx.size <= k else rng.choice(idx, size=k, replace=False)

    b = pick(band, n // 2)
    w = pick(wall, n // 4)
    u = pick(fluid, n - b.size - w.size)
    cells = np.unique(np.concatenate([b, w, u]))
    return cells, b.size, w.size, int(np.count_nonzero(band))


def check_next_step(oracle, s, q, q1, dt_gpu, dt_fixed=None, seed=0, n=N_SAMPLED):
    """The GPU's step from q (its result q1, its time step dt_gpu) against the oracle's on
    sampled cells."""
    if dt_fixed is None:
        lam, dt = oracle.cfl(s, q)
        assert abs(dt - dt_gpu) <= 1e-11 * dt, (dt, dt_gpu)
    else:
        dt = dt_fixed
    cells, nb, nw, nband = sample_cells(s, q, n, seed)
    assert nb == min(n // 2, nband) and nb > 0  # half the sample, or the whole band where it is smaller
    ref = oracle.step_cells(s, q, dt, cells)
    got = q1.reshape(4, -1)[:, cells]
    e = field_errors(s, got, ref)
    print(f"{s.name} {s.nx}x{s.ny}: {cells.size} cells ({nb} band, {nw} wall/obstacle), field errors {e}",
          flush=True)
    assert np.all(e <= TOL), e
    return e


def run_then_step(bn, torch, s, n_steps, dt_fixed=None):
    with bn.Simulation(s) as sim:
        sim.set_state(torch.from_numpy(np.ascontiguousarray(s.q)).cuda())
        if dt_fixed is None:
            sim.run(n_steps)
        else:
            for _ in range(n_steps):
                sim.step(dt_fixed)
        t, dt_next = sim.time()
        q = sim.get_state().cpu().numpy()
        if dt_fixed is None:
            sim.run(1)
        else:
            sim.step(dt_fixed)
        t1, _ = sim.time()
        sim.status()
        q1 = sim.get_state().cpu().numpy()
    if dt_fixed is None:
        assert t1 - t == pytest.approx(dt_next, rel=1e-12)
    return q, q1, dt_next


@pytest.mark.parametrize("name,builder,n_steps", [
    ("dam_break_2048x1024", lambda: sc.dam_break(0), 2000),
    ("elliptic_drop_4096x4096", lambda: sc.elliptic_drop(0), 1000),
])
def test_step_after_the_stated_steps(oracle, bn, torch_cuda, name, builder, n_steps):
    s = builder()
    print(f"{name}: {n_steps} GPU steps, then one more against the oracle", flush=True)
    q, q1, dt_next = run_then_step(bn, torch_cuda, s, n_steps)
    fl = s.fluid()
    assert np.isfinite(q).all() and q[3][fl].min() > 0
    check_next_step(oracle, s, q, q1, dt_next, seed=n_steps)


def test_wall_impact_step_after_400_fixed_steps(oracle, bn, torch_cuda):
    s = sc.wall_impact(0)
    lam, dt = oracle.cfl(s, s.q)
    print(f"wall impact 512x256: 400 GPU steps of dt {dt}, then one more against the oracle", flush=True)
    q, q1, _ = run_then_step(bn, torch_cuda, s, 400, dt_fixed=dt)
    check_next_step(oracle, s, q, q1, None, dt_fixed=dt, seed=400)


def test_ensemble_members_after_500_steps(oracle, bn, torch_cuda):
    torch = torch_cuda
    members = sc.ensemble(0)
    big = max(range(len(members)), key=lambda k: members[k].cells)
    print(f"ensemble of {len(members)}: 500 steps, then one more (largest member {members[big].nx}x"
          f"{members[big].ny})", flush=True)
    with bn.Batch(members) as b:
        for k, s in enumerate(members):
            b.set_state(k, torch.from_numpy(np.ascontiguousarray(s.q)).cuda())
        b.run(500)
        dts = [b.time(k)[1] for k in range(len(members))]
        qs = [b.get_state(k).cpu().numpy() for k in range(len(members))]
        b.run(1)
        b.status()
        q1s = [b.get_state(k).cpu().numpy() for k in range(len(members))]
    check_next_step(oracle, members[big], qs[big], q1s[big], dts[big], seed=500)
    worst = np.zeros(4)
    for k, s in enumerate(members):
        if k == big:
            continue
        worst = np.maximum(worst, check_next_step(oracle, s, qs[k], q1s[k], dts[k], seed=k, n=200))
    print(f"other members: worst field errors {worst}", flush=True)


@pytest.mark.parametrize("name,builder,n_steps", [
    ("dam_break_2048x1024", lambda: sc.dam_break(0), 100),
    ("elliptic_drop_4096x4096", lambda: sc.elliptic_drop(0), 10),
])
def test_full_grid_trajectory(oracle, bn, torch_cuda, name, builder, n_steps):
    s = builder()
    with bn.Simulation(s) as sim:
        sim.set_state(torch_cuda.from_numpy(np.ascontiguousarray(s.q)).cuda())
        sim.run(n_steps)
        tg, dtg = sim.time()
        qg = sim.get_state().cpu().numpy()
    t0 = time.perf_counter()
    qo, to, dto = oracle.run(s, s.q, n_steps)
    print(f"{name}: oracle {n_steps} steps in {time.perf_counter() - t0:.1f} s on {oracle.threads()} threads",
          flush=True)
    e = field_errors(s, qg, qo)
    print(f"{name} after {n_steps} steps: field errors {e}, time {tg} vs {to}", flush=True)
    assert np.all(e <= TOL), e
    assert abs(tg - to) <= 1e-11 * to
