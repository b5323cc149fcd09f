"""Pins of the oracle's reading of an obstacle top that lies off the grid (the free-surface detector
of Sec. 3.5 integrating alpha from the column's bottom y_L), on the CPU.

Cells stay whole (solid iff the centre lies below the obstacle's top); only the detector sees the
top itself.  What fixes the reading without restating its formula:
  * at the top of the solid run it is the grid-aligned detector, bit for bit;
  * the detector is the integral of the normalised volume fraction from y_L upwards, the first fluid
    cell's value standing for the whole interval from y_L to its top edge (checked by adaptive
    quadrature of that step function);
  * water at rest over such a wall, and a wall that stands above the water, stay at rest exactly
    (Sec. 3.5: the detector is exact at rest even with obstacles);
  * the bottom moves the step only through the free surface of its own column, and only where the
    first fluid cell is neither full nor empty.
"""
import numpy as np
import pytest
from scipy import integrate

from paper_1806_04960_amd import scenarios as sc


def tank_with_wall(top, surface=0.5, nx=40, ny=32, column=13):
    return sc.tank_with_wall(top, surface, nx, ny, column)


def test_bottom_at_the_solid_tops_is_the_grid_aligned_detector(oracle):
    s = sc.random_state(sc.wall_impact(0, 48, 24), seed=2, amp=0.002, vel=0.05)
    plain = s.copy()
    plain.bottom = None
    aligned = s.copy()
    aligned.bottom = s.solid_tops()
    assert np.array_equal(oracle.detector(aligned, s.q), oracle.detector(plain, s.q))
    _, dt = oracle.cfl(s, s.q)
    assert np.array_equal(oracle.step(aligned, s.q, dt), oracle.step(plain, s.q, dt))


@pytest.mark.parametrize("offset", [-0.45, -0.2, 0.3])
def test_detector_integrates_alpha_from_the_bottom(oracle, offset):
    s = tank_with_wall(0.3, nx=8, ny=16, column=3)
    iw = 3
    base = s.solid_tops()[iw]
    s.bottom[iw] = base + offset * s.dy
    rng = np.random.default_rng(5)
    q = s.q.copy()
    fluid = s.solid[:, iw] == 0
    # any alpha profile in the wall column (first fluid cell partly liquid)
    q[3, fluid, iw] = s.alpha_gas + rng.uniform(0, 1, fluid.sum()) * (s.alpha_liq - s.alpha_gas)
    q[0, fluid, iw] = q[3, fluid, iw] * s.rho0
    a = (q[3, :, iw] - s.alpha_gas) / (s.alpha_liq - s.alpha_gas)
    jb = int(np.argmax(fluid))
    edges = s.y0 + np.arange(s.ny + 1) * s.dy

    def profile(y):
        j = min(max(int(np.floor((y - s.y0) / s.dy)), jb), s.ny - 1)
        return a[j]

    y_l = s.bottom[iw]
    pts = [e for e in edges if y_l < e < s.y1]
    integral, err = integrate.quad(profile, y_l, s.y1, points=pts, limit=200, epsabs=1e-14, epsrel=1e-14)
    y0 = oracle.detector(s, q)[iw]
    assert y0 == pytest.approx(y_l + integral, abs=1e-13)


@pytest.mark.parametrize("offset", [-0.4, 0.3])
def test_water_at_rest_over_an_off_grid_wall_stays_at_rest(oracle, offset):
    s = tank_with_wall(0.3, surface=0.5)
    s.bottom[13] = s.solid_tops()[13] + offset * s.dy
    plain = s.copy()
    plain.bottom = None
    q, t, _ = oracle.run(s, s.q, 300)
    fl = s.fluid()
    assert np.abs(q[1])[fl].max() == 0.0 and np.abs(q[2] / q[0])[fl].max() < 1e-11
    assert np.abs(q[0] - s.q[0])[fl].max() / s.rho0 < 1e-12
    # the first fluid cell of the wall column is full: the state is bitwise that of the grid-aligned wall
    q_plain, _, _ = oracle.run(plain, plain.q, 300)
    assert np.array_equal(q, q_plain)


@pytest.mark.parametrize("offset", [-0.3, 0.45])
def test_a_wall_above_the_water_leaves_the_rest_state_unchanged(oracle, offset):
    s = tank_with_wall(0.7, surface=0.4)
    s.bottom[13] = s.solid_tops()[13] + offset * s.dy
    y0 = oracle.detector(s, s.q)
    assert y0[13] == s.bottom[13]  # an empty column's free surface is its bottom
    q, _, _ = oracle.run(s, s.q, 300)
    fl = s.fluid()
    assert np.abs(q[1])[fl].max() == 0.0 and np.abs(q[2] / q[0])[fl].max() < 1e-11


def test_bottom_acts_only_through_a_partly_liquid_first_cell(oracle):
    """d<lam, step>/dy_L by differences: exactly 0 where the column's first fluid cell is empty (the
    whole column is gas: no liquid-type cell) or full (the free surface does not move); non-zero where
    it is partly liquid, and then the change of the step stays in that column's reach."""
    s = sc.wall_impact(0, 32, 16)
    iw = s.meta["wall_column"]
    jb = int(np.argmax(s.solid[:, iw] == 0))
    lam = np.random.default_rng(3).normal(size=s.q.shape)
    _, dt = oracle.cfl(s, s.q)
    # the wall column is dry at t = 0
    assert oracle.adjoint_fd_bottom(s, s.q, lam, dt, [iw])[0] == 0.0
    for a_first, expect_zero in ((1.0, True), (0.35, False)):
        q = s.q.copy()
        # liquid up to two cells above the wall, its first cell filled to a_first
        q[3, jb:jb + 3, iw] = s.alpha_liq
        q[3, jb, iw] = s.alpha_gas + a_first * (s.alpha_liq - s.alpha_gas)
        q[0, jb:jb + 3, iw] = q[3, jb:jb + 3, iw] * s.rho0
        g = oracle.adjoint_fd_bottom(s, q, lam, dt, [iw], h=1e-7)[0]
        if expect_zero:
            assert g == 0.0
        else:
            assert abs(g) > 1e-3
            sp, sm = s.copy(), s.copy()
            sp.bottom[iw] += 1e-6
            sm.bottom[iw] -= 1e-6
            d = np.abs(oracle.step(sp, q, dt) - oracle.step(sm, q, dt)).max(axis=0)
            cols = np.nonzero(d.max(axis=0) > 0)[0]
            assert set(cols) <= {iw - 1, iw, iw + 1}


def test_bottom_beyond_half_a_cell_is_rejected(oracle):
    s = tank_with_wall(0.3)
    s.bottom[13] = s.solid_tops()[13] + 0.5 * s.dy
    with pytest.raises(oracle.OracleError):
        oracle.detector(s, s.q)
    s.bottom[13] = s.solid_tops()[13] - 0.51 * s.dy
    with pytest.raises(oracle.OracleError):
        oracle.detector(s, s.q)
