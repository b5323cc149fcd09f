"""Host-side checks of the seeded input builders (shapes, masks, rasterisation by cell centres)."""
import numpy as np

from paper_1806_04960_amd import scenarios as sc


def test_weir_geometry():
    s = sc.weir()
    assert (s.nx, s.ny) == (800, 250) and s.dx == 15.0 / 800 and s.dy == 2.1 / 250
    iw = s.meta["weir_column"]
    assert s.xc()[iw - 1] < 0.0 < s.xc()[iw]           # first column right of x = 0
    cols = np.nonzero(s.solid.any(axis=0))[0]
    assert list(cols) == [iw]                           # one cell thick
    rows = np.nonzero(s.solid[:, iw])[0]
    assert rows[0] == 0 and np.all(np.diff(rows) == 1)  # attached to the bottom
    assert s.yc()[rows[-1]] <= 0.7 < s.yc()[rows[-1] + 1]
    liq = s.q[3] > 0.5
    assert liq[:, : iw].any() and not liq[:, iw + 1:].any()   # dry right of the weir
    assert np.all(s.q[1] == 0.0) and np.all(s.q[2] == 0.0)    # at rest


def test_seeded_builders_are_reproducible():
    a, b = sc.dam_break(3, 64, 32), sc.dam_break(3, 64, 32)
    assert np.array_equal(a.q, b.q) and np.array_equal(a.solid, b.solid)
    assert not np.array_equal(a.q, sc.dam_break(4, 64, 32).q)


def test_wall_impact_theta_vjp_matches_differences_of_the_builder():
    """dJ/dtheta = (dq0/dtheta)^T lam0, against central differences of the initial state itself
    along random profile directions (the builder is smooth between cell edges; the steps are far too
    small to move the surface across one)."""
    s = sc.wall_impact(3, nx=96, ny=48)
    theta = np.asarray(s.meta["theta"])
    rng = np.random.default_rng(7)
    lam = rng.standard_normal((4, s.ny, s.nx))
    g = sc.wall_impact_theta_vjp(s, lam)
    assert g.shape == theta.shape and np.abs(g).max() > 0
    for _ in range(4):
        d = rng.standard_normal(theta.size)
        h = 1e-7
        qp = sc.wall_impact(3, nx=96, ny=48, theta=theta + h * d).q
        qm = sc.wall_impact(3, nx=96, ny=48, theta=theta - h * d).q
        fd = float((lam * (qp - qm)).sum()) / (2 * h)
        assert abs(g @ d - fd) <= 1e-6 * abs(fd), (g @ d, fd)


def test_wall_impact_rebuilds_from_its_own_theta():
    s = sc.wall_impact(2, nx=64, ny=32)
    s2 = sc.wall_impact(2, nx=64, ny=32, theta=s.meta["theta"])
    assert np.array_equal(s.q, s2.q)


def test_smooth_state_vjp_matches_differences():
    s = sc.wall_impact(4, nx=64, ny=32)
    rng = np.random.default_rng(8)
    lam = rng.standard_normal((4, s.ny, s.nx))
    g = sc.smooth_state_vjp(s, lam)
    scale = np.stack([np.abs(s.q[0]) + 1.0] * 3 + [np.ones_like(s.q[3])])
    for _ in range(3):
        d = rng.standard_normal(s.q.shape) * scale * s.fluid()
        h = 1e-7
        sp, sm = s.copy(), s.copy()
        sp.q = s.q + h * d
        sm.q = s.q - h * d
        fd = float((lam * (sc.smooth_state(sp).q - sc.smooth_state(sm).q)).sum()) / (2 * h)
        assert abs(float((g * d).sum()) - fd) <= 1e-7 * abs(fd), (float((g * d).sum()), fd)
