"""Exact solution of the 1D Riemann problem for isothermal gas dynamics, p'(rho) = c^2
(textbook: two genuinely non-linear waves, shock or rarefaction, joined at (rho*, u*)).
With alpha constant and g = 0 the reduced model with gamma = 1 is exactly this system:
alpha p = alpha (c^2 rho - k0), whose constant part carries no force.
Independent of the oracle: used to pin its edge fluctuations."""
import math

import numpy as np


def _wave(rho_star, rho_k, c):
    """Velocity change across a wave from rho_k to rho_star (shock if compressive)."""
    if rho_star > rho_k:
        r = rho_star / rho_k
        return c * (math.sqrt(r) - 1.0 / math.sqrt(r))
    return c * math.log(rho_star / rho_k)


def star_state(rl, ul, rr, ur, c):
    f = lambda r: _wave(r, rl, c) + _wave(r, rr, c) + (ur - ul)
    lo, hi = 1e-12, 1e12
    r = math.sqrt(rl * rr)
    for _ in range(200):                      # safeguarded secant / bisection
        a, b = r * 0.999999, r * 1.000001
        fa, fb = f(a), f(b)
        d = (fb - fa) / (b - a)
        fr = f(r)
        if fr > 0:
            hi = min(hi, r)
        else:
            lo = max(lo, r)
        rn = r - fr / d if d != 0 else 0.5 * (lo + hi)
        if not (lo < rn < hi):
            rn = 0.5 * (lo + hi)
        if abs(rn - r) < 1e-15 * r:
            r = rn
            break
        r = rn
    ustar = 0.5 * (ul + ur) + 0.5 * (_wave(r, rr, c) - _wave(r, rl, c))
    return r, ustar


def sample(rl, ul, rr, ur, c, xi):
    """(rho, u) at similarity coordinates xi = (x - x0)/t."""
    rs, us = star_state(rl, ul, rr, ur, c)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    for n, s in enumerate(xi):
        if s < us:  # left of contact: 1-wave
            if rs > rl:
                sh = ul - c * math.sqrt(rs / rl)
                rho[n], u[n] = (rl, ul) if s < sh else (rs, us)
            else:
                head, tail = ul - c, us - c
                if s < head:
                    rho[n], u[n] = rl, ul
                elif s > tail:
                    rho[n], u[n] = rs, us
                else:
                    u[n] = s + c
                    rho[n] = rl * math.exp((ul - u[n]) / c)
        else:
            if rs > rr:
                sh = ur + c * math.sqrt(rs / rr)
                rho[n], u[n] = (rs, us) if s < sh else (rr, ur)
            else:
                tail, head = us + c, ur + c
                if s > head:
                    rho[n], u[n] = rr, ur
                elif s < tail:
                    rho[n], u[n] = rs, us
                else:
                    u[n] = s - c
                    rho[n] = rr * math.exp((u[n] - ur) / c)
    return rho, u
