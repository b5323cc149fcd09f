"""The adjoint oracle (the transpose of the oracle step's Jacobian by central differences) against
what the scheme fixes independently of any derivative code:

- conservation of alpha rho in a closed box (Sec. 3: every edge's D- and D+ of the first component
  sum to the flux jump, and walls mirror): sum_c (alpha rho)^{n+1}_c = sum_c (alpha rho)^n_c for
  every state, so the adjoint of lambda^{n+1} = (1, 0, 0, 0) everywhere is (1, 0, 0, 0) everywhere;
- solid cells keep their state and are never read (Sec. 5): their adjoint passes through;
- the stencil (Sec. 3.4, 3.1-3.3): an output cell depends on the states within two cells along x
  and y and one diagonally, plus the alpha of the columns whose free surface its edges use
  (its own and the two beside it, Sec. 3.5); every other entry of the adjoint is exactly zero.
"""
import numpy as np

from paper_1806_04960_amd import scenarios as sc


def _dt(oracle, s):
    return 0.9 * oracle.cfl(s, s.q)[1]


def test_mass_identity(oracle):
    s = sc.generic_state(sc.dam_break_small(7, 6), seed=1)
    lam = np.zeros_like(s.q)
    lam[0] = 1.0
    out = oracle.adjoint_fd(s, s.q, lam, _dt(oracle, s))
    # (the difference quotients' rounding: about 1e-13 per changed entry over steps of 1e-6 |alpha rho|)
    np.testing.assert_allclose(out[0], 1.0, atol=1e-6)
    np.testing.assert_allclose(out[1:], 0.0, atol=1e-6)


def test_solid_cells_pass_through(oracle):
    s = sc.generic_state(sc.rest_with_obstacle(10, 6), seed=2)
    rng = np.random.default_rng(5)
    lam = rng.normal(size=s.q.shape)
    out = oracle.adjoint_fd(s, s.q, lam, _dt(oracle, s))
    solid = s.solid == 1
    assert solid.any()
    np.testing.assert_allclose(out[:, solid], lam[:, solid], rtol=0, atol=1e-8)


def test_stencil_support(oracle):
    # a second-order cell (its 3 x 3 stencil is liquid) with gas two rows above it
    s = sc.generic_state(sc.rest_flat(11, 10), seed=3)
    i, j = 5, 3
    lam = np.zeros_like(s.q)
    lam[:, j, i] = [1.0, 0.3, -0.7, 2.0]
    out = oracle.adjoint_fd(s, s.q, lam, _dt(oracle, s))
    J, I = np.meshgrid(np.arange(s.ny), np.arange(s.nx), indexing="ij")
    di, dj = np.abs(I - i), np.abs(J - j)
    support = ((di + dj) <= 2) | ((di <= 1) & (dj <= 1))
    for k in range(3):
        assert np.all(out[k][~support] == 0.0), k
    assert np.all(out[3][~(support | (di <= 1))] == 0.0)
    # something flows to every cell of the 3 x 3 stencil, and through the free surface to the
    # alpha of the column's top cell
    assert np.all(np.abs(out[0][(di <= 1) & (dj <= 1)]) > 0)
    assert abs(out[3][s.ny - 1, i]) > 0


def test_each_component_matches_a_directional_difference(oracle):
    """<adjoint_fd(lambda), d> against <lambda, (step(q + e d) - step(q - e d)) / 2e>, one scalar step
    e along a random direction d in one component at a time (alpha rho, the two momenta, alpha):
    pins adjoint_fd's per-entry step sizes and signs for every component, which the mass identity
    above sees only for alpha rho."""
    s = sc.generic_state(sc.dam_break_small(7, 6), seed=7)
    rng = np.random.default_rng(11)
    dt = _dt(oracle, s)
    lam = rng.normal(size=s.q.shape)
    adj = oracle.adjoint_fd(s, s.q, lam, dt)
    fluid = s.fluid()
    scale = [np.abs(s.q[0]), np.abs(s.q[0]), np.abs(s.q[0]), np.ones_like(s.q[3])]
    for k in range(4):
        d = np.zeros_like(s.q)
        d[k] = rng.uniform(-1.0, 1.0, size=d[k].shape) * scale[k] * fluid
        e = 1e-6
        fd = float(np.sum(lam * (oracle.step(s, s.q + e * d, dt) - oracle.step(s, s.q - e * d, dt))) / (2 * e))
        ad = float(np.sum(adj * d))
        assert abs(ad - fd) <= 1e-6 * max(abs(fd), 1e-12), (k, ad, fd)
