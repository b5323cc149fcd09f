"""Parity measure shared by the GPU tests: per field k,

    e_k = max |Q_k^gpu - Q_k^oracle| / max(max |Q_k^oracle|, s_k),

with floors s = (rho0 alpha_l, rho0 alpha_l x 1 m/s, rho0 alpha_l x 1 m/s, 1).  A field is divided by
its own largest value; the floors only act where a field is small everywhere (the momenta of a fluid
at rest are zero, or round-off), and then measure the error against a liquid moving at 1 m/s.
The bar is 1e-11 on every field."""
import numpy as np

TOL = 1e-11
VELOCITY_FLOOR = 1.0  # m/s


def field_errors(s, q_gpu, q_ref):
    m = s.rho0 * s.alpha_liq
    floors = [m, m * VELOCITY_FLOOR, m * VELOCITY_FLOOR, 1.0]
    return np.array([np.abs(q_gpu[k] - q_ref[k]).max() / max(np.abs(q_ref[k]).max(), floors[k])
                     for k in range(4)])
