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
