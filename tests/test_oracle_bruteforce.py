"""The oracle's transcription of one step against an independent 40-digit restatement of the scheme
(``tests/bruteforce_mp.py``: system matrices from the Jacobians of the fluxes of Sec. 2.1 plus the
non-conservative products, |A| and sign(A) by Sylvester interpolation over numerically found
eigenvalues) on 6 x 6 grids with random admissible states: liquid and gas rows, a first-order cell
inside the liquid, liquid reaching into the gas, a solid cell on the bottom, gravity on, every cell
moving.  Agreement within 1e-13 relative per field (momenta relative to rho0 c) covers the
equations of Sec. 3 (scheme, b_4 in x and y, the final b_3^y, the Osher-Romberg viscosity) as the
oracle writes them."""
import math

import mpmath as mp
import numpy as np
import pytest

from paper_1806_04960_amd import scenarios as sc
from tests.bruteforce_mp import Scheme


def tiny_state(seed, bc=(0, 0, 0, 0)):
    rng = np.random.default_rng(seed)
    s = sc.uniform_tank(6, 6, 0.0, 0.6, 0.0, 0.6, g=9.81, k0=2.78e5, alpha_liq=1 - 1e-3, bc=bc)
    solid = np.zeros((6, 6), np.uint8)
    solid[0, 4] = 1
    s.solid = solid
    rows = np.arange(6)[:, None]
    al = np.where(rows < 3, rng.uniform(0.9, 0.999, (6, 6)), rng.uniform(1e-3, 4e-3, (6, 6)))
    al[2, 1] = 0.005   # first order inside the liquid rows
    al[3, 2] = 0.6     # liquid reaching into the gas rows
    rho = 1000.0 * (1.0 + 0.01 * rng.uniform(-1, 1, (6, 6)))
    u, v = rng.uniform(-1, 1, (6, 6)), rng.uniform(-1, 1, (6, 6))
    q = np.zeros((4, 6, 6))
    q[0] = al * rho
    q[1] = q[0] * u
    q[2] = q[0] * v
    q[3] = al
    q[:, solid == 1] = np.array([1000.0, 0.0, 0.0, 1.0])[:, None]
    s.q = q
    return s


@pytest.mark.parametrize("seed,bc", [(0, (0, 0, 0, 0)), (1, (0, 0, 0, 0)), (2, (1, 1, 0, 1))])
def test_one_step_matches_the_high_precision_restatement(oracle, seed, bc):
    s = tiny_state(seed, bc)
    _, dt = oracle.cfl(s, s.q)
    ref = oracle.step(s, s.q, dt)
    Q = [[[mp.mpf(float(s.q[k, j, i])) for i in range(s.nx)] for j in range(s.ny)] for k in range(4)]
    out = Scheme(s).step(Q, dt)
    hp = np.array([[[float(out[k][j][i]) for i in range(s.nx)] for j in range(s.ny)] for k in range(4)])
    c = math.sqrt(s.k0 / s.rho0)
    scales = [s.rho0, s.rho0 * c, s.rho0 * c, 1.0]
    for k in range(4):
        err = np.abs(hp[k] - ref[k]).max() / max(np.abs(ref[k]).max(), scales[k])
        assert err <= 1e-13, (k, err)
    # the step did something in every field
    assert all(np.abs(hp[k] - s.q[k]).max() > 1e-6 * scales[k] for k in range(4))
