"""Batches (bn_batch_*): many grids of different sizes, parameters and masks advanced by one launch
per step, each with its own CFL time step.

Each member's results must be bitwise those of a single-grid run on the same input (the kernel
computes every cell with the same arithmetic whatever the partition), and within the parity
tolerance of the oracle.  Inputs: small members of the scenario families the tests and the
ensemble workload use (dam breaks with obstacles, drops, water at rest over a step, ragged sizes).
"""

import numpy as np
import pytest

from paper_1806_04960_amd import scenarios as sc
from tests.parity import field_errors

pytestmark = pytest.mark.gpu
TOL = 1e-11




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


def small_members():
    """Seven grids of different shapes, gravity, boundaries and masks (some narrower than one
    strip, some spanning several strips with a ragged last one)."""
    out = sc.ensemble(seed=6, count=4, sizes=((130, 47), (61, 90), (200, 33), (256, 128)))
    out += [sc.rest_with_obstacle(), sc.dam_break_small(97, 41), sc.circular_drop(64, 64),
            sc.uniform_tank(7, 5, u=0.3, bc=(1, 1, 0, 0)), sc.uniform_tank(1, 23, v=-0.2)]
    return out


def _run_single(bn, torch, s, n):
    with bn.Simulation(s) as sim:
        sim.set_state(torch.from_numpy(np.ascontiguousarray(s.q)).cuda())
        sim.run(n)
        t, dt = sim.time()
        return sim.get_state().cpu().numpy(), t, dt, sim.y0()


def _run_batch(bn, torch, members, n, rows=None, waves=None):
    with bn.Batch(members, rows_per_block=rows, wavefronts=waves) as b:
        for k, s in enumerate(members):
            b.set_state(k, torch.from_numpy(np.ascontiguousarray(s.q)).cuda())
        b.run(n)
        b.status()
        return [(b.get_state(k).cpu().numpy(), *b.time(k), b.y0(k)) for k in range(len(members))]


def test_batch_members_equal_single_runs_bitwise(bn, torch_cuda):
    members = small_members()
    print(f"{len(members)} members: {[(s.nx, s.ny) for s in members]}", flush=True)
    res = _run_batch(bn, torch_cuda, members, 40)
    for s, (q, t, dt, y0) in zip(members, res):
        q1, t1, dt1, y01 = _run_single(bn, torch_cuda, s, 40)
        assert np.array_equal(q, q1), s.name
        assert t == t1 and dt == dt1, s.name
        assert np.array_equal(y0, y01), s.name


def test_batch_members_match_the_oracle(oracle, bn, torch_cuda):
    members = small_members()
    res = _run_batch(bn, torch_cuda, members, 25)
    for s, (q, t, dt, y0) in zip(members, res):
        qo, to, dto = oracle.run(s, s.q, 25)
        e = field_errors(s, q, qo)
        print(f"{s.name} {s.nx}x{s.ny}: {e}", flush=True)
        assert np.all(e <= TOL), (s.name, e)
        assert abs(t - to) <= 1e-12 * to


@pytest.mark.parametrize("rows,waves", [(1, 3), (5, 17), (64, 1), (32, 4096)])
def test_batch_launch_shape_does_not_change_results(bn, torch_cuda, rows, waves):
    members = small_members()
    ref = _run_batch(bn, torch_cuda, members, 12)
    got = _run_batch(bn, torch_cuda, members, 12, rows=rows, waves=waves)
    for (q, t, dt, y0), (q1, t1, dt1, y01) in zip(ref, got):
        assert np.array_equal(q, q1) and t == t1 and dt == dt1 and np.array_equal(y0, y01)


def test_each_member_keeps_its_own_time_step(bn, torch_cuda):
    a = sc.uniform_tank(16, 16, k0=2.78e5)
    b = sc.uniform_tank(16, 16, k0=6.54e5)
    res = _run_batch(bn, torch_cuda, [a, b], 3)
    dta, dtb = res[0][2], res[1][2]
    c_a, c_b = np.sqrt(a.k0 / a.rho0), np.sqrt(b.k0 / b.rho0)
    # at rest the rate is the sound speed over the cell size (both directions)
    assert dta / dtb == pytest.approx(c_b / c_a, rel=1e-12)
    assert res[0][1] == pytest.approx(3 * dta, rel=1e-14)


def test_resetting_one_member_leaves_the_others(bn, torch_cuda):
    members = [sc.dam_break_small(97, 41), sc.circular_drop(64, 64)]
    with bn.Batch(members) as b:
        for k, s in enumerate(members):
            b.set_state(k, torch_cuda.from_numpy(s.q).cuda())
        b.run(10)
        b.set_state(0, torch_cuda.from_numpy(members[0].q).cuda())
        b.run(10)
        q0, q1 = b.get_state(0).cpu().numpy(), b.get_state(1).cpu().numpy()
        t0, t1 = b.time(0)[0], b.time(1)[0]
    r0 = _run_single(bn, torch_cuda, members[0], 10)
    r1 = _run_single(bn, torch_cuda, members[1], 20)
    assert np.array_equal(q0, r0[0]) and t0 == r0[1]
    assert np.array_equal(q1, r1[0]) and t1 == r1[1]


def test_nonphysical_member_is_named(bn, torch_cuda):
    good = sc.uniform_tank(8, 8)
    bad = sc.uniform_tank(8, 8)
    q = bad.q.copy()
    q[0, 3, 3] = -1.0
    bad.q = q
    with bn.Batch([good, bad]) as b:
        b.set_state(0, torch_cuda.from_numpy(good.q).cuda())
        b.set_state(1, torch_cuda.from_numpy(bad.q).cuda())
        with pytest.raises(bn.BnError, match="member 1"):
            b.status()


def test_run_before_every_member_has_a_state_is_rejected(bn, torch_cuda):
    members = [sc.uniform_tank(8, 8), sc.uniform_tank(9, 9)]
    with bn.Batch(members) as b:
        b.set_state(0, torch_cuda.from_numpy(members[0].q).cuda())
        with pytest.raises(bn.BnError):
            b.run(1)


def test_tuned_launch_is_the_fastest_candidate_and_changes_no_result(bn, torch_cuda):
    s = sc.dam_break(3, 300, 150)
    with bn.Simulation(s) as sim:
        sim.set_state(torch_cuda.from_numpy(s.q).cuda())
        rows, waves, times = bn.tune_launch(sim, steps=10, shapes=[(4, 256), (4, 2048), (2, 512)])
        assert (rows, waves) == min(times, key=times.get)
        assert sim.launch() == (rows, waves)
        sim.run(15)
        q = sim.get_state().cpu().numpy()
    with bn.Simulation(s) as ref:
        ref.set_state(torch_cuda.from_numpy(s.q).cuda())
        ref.run(15)
        assert np.array_equal(q, ref.get_state().cpu().numpy())
    members = small_members()[:3]
    with bn.Batch(members) as b:
        for k, m in enumerate(members):
            b.set_state(k, torch_cuda.from_numpy(m.q).cuda())
        rows, waves, times = bn.tune_launch(b, steps=5, shapes=[(4, 128), (8, 1024)])
        assert b.launch() == (rows, waves)
