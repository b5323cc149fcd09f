"""The oracle's sampled-cell entry point (used to check grids too large for a full oracle
step) computes exactly what its full step computes."""
import numpy as np

from paper_1806_04960_amd import scenarios as sc


def test_step_cells_matches_full_step_bitwise(oracle):
    s = sc.random_state(sc.dam_break(3, 96, 48), seed=5, amp=0.02, vel=1.0)
    lam, dt = oracle.cfl(s, s.q)
    full = oracle.step(s, s.q, dt)
    rng = np.random.default_rng(1)
    cells = rng.choice(s.nx * s.ny, size=300, replace=False)
    cells = np.concatenate([cells, [0, s.nx - 1, s.nx * (s.ny - 1), s.nx * s.ny - 1]])
    part = oracle.step_cells(s, s.q, dt, cells)
    ref = full.reshape(4, -1)[:, cells]
    assert np.array_equal(part, ref)


def test_run_equals_repeated_cfl_steps(oracle):
    s = sc.dam_break_small(40, 20)
    q = s.q.copy()
    t = 0.0
    for _ in range(7):
        lam, dt = oracle.cfl(s, q)
        q = oracle.step(s, q, dt)
        t += dt
    q2, t2, dt2 = oracle.run(s, s.q, 7)
    assert np.array_equal(q, q2) and t == t2
