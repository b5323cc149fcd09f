"""One explicit step of the well-balanced Osher / Osher-Romberg scheme in high precision (mpmath),
written a second time, from the paper, to check the oracle's transcription on tiny grids.

TEST INFRASTRUCTURE.  It shares no code with ``oracle/`` or with the HIP library and takes a
different route wherever one exists:
  * the system matrices A1, A2 are not the printed ones: they are the Jacobians of the fluxes f, g
    of Sec. 2.1, taken by high-precision central differences, plus the non-conservative products
    B1, B2 read off the PDE (u d_x alpha, v d_y alpha, d_y(alpha p) and the weight alpha rho g d_y y);
  * |A| and sign(A) are not R diag R^{-1} with the printed eigenvectors: they are Sylvester's
    interpolation over the distinct eigenvalues that mpmath finds numerically, f(A) = sum_j
    f(l_j) prod_{i != j} (A - l_i)/(l_j - l_i), exact for a diagonalisable matrix;
  * everything is evaluated with 40 significant digits.
The scheme's readings (free-surface detector, two-level equilibrium, fluctuations against the
centre cell's profile, limiter and second-order switch over the 3x3 stencil, path velocity of b_4,
b_3 on fluctuations, wall ghosts, cell integral) are the same as the oracle's: the check is of the
arithmetic, not of the readings.
"""
from __future__ import annotations

import mpmath as mp

W, E, S, N = 0, 1, 2, 3


class Scheme:
    def __init__(self, s, dps: int = 40):
        mp.mp.dps = dps
        self.s = s
        m = mp.mpf
        self.nx, self.ny = s.nx, s.ny
        self.dx = (m(s.x1) - m(s.x0)) / s.nx
        self.dy = (m(s.y1) - m(s.y0)) / s.ny
        self.ylo = m(s.y0)
        self.g, self.k0, self.rho0 = m(s.g), m(s.k0), m(s.rho0)
        self.al, self.ag = m(s.alpha_liq), m(s.alpha_gas)
        self.bc = tuple(int(b) for b in s.bc)
        self.solid = s.solid
        # Gauss-Legendre on [0, 1]: roots of P3 mapped, weights 5/18, 8/18, 5/18
        r = mp.sqrt(m(3) / 5)
        self.gl = [((1 - r) / 2, m(5) / 18), (m(1) / 2, m(8) / 18), ((1 + r) / 2, m(5) / 18)]

    # ---- model (Sec. 2.1, gamma = 1) ------------------------------------------------------------
    def fluid(self, i, j):
        if not (0 <= i < self.nx and 0 <= j < self.ny):
            return False
        return self.solid is None or self.solid[j][i] == 0

    def alpha_p(self, q):
        return q[3] * self.k0 * (q[0] / q[3] / self.rho0 - 1)

    def f(self, q):
        u = q[1] / q[0]
        return [q[1], q[1] * u + self.alpha_p(q), q[2] * u, mp.mpf(0), mp.mpf(0)]

    def gflux(self, q):
        v = q[2] / q[0]
        return [q[2], q[1] * v, q[2] * v, mp.mpf(0), mp.mpf(0)]

    def jac(self, fun, q):
        h = mp.mpf(10) ** (-15)
        J = mp.matrix(5, 5)
        for b in range(5):
            hb = h * max(1, abs(q[b]))
            qp, qm = list(q), list(q)
            qp[b] += hb
            qm[b] -= hb
            fp, fm = fun(qp), fun(qm)
            for a in range(5):
                J[a, b] = (fp[a] - fm[a]) / (2 * hb)
        return J

    def A(self, direction, q):
        if direction == 0:
            M = self.jac(self.f, q)
            M[3, 3] += q[1] / q[0]                      # u d_x alpha
        else:
            M = self.jac(self.gflux, q)
            dp = self.jac(lambda z: [0, 0, self.alpha_p(z), 0, 0], q)
            for b in range(5):
                M[2, b] += dp[2, b]                      # d_y (alpha p)
            M[2, 4] += q[0] * self.g                     # alpha rho g d_y y
            M[3, 3] += q[2] / q[0]                       # v d_y alpha
        return M

    def matfun(self, M, fn):
        lams = mp.eig(M, left=False, right=False)
        distinct = []
        for lam in lams:
            lam = mp.re(lam)
            if all(abs(lam - d) > mp.mpf(10) ** (-20) * (1 + abs(d)) for d in distinct):
                distinct.append(lam)
        out = mp.zeros(5, 5)
        I = mp.eye(5)
        for j, lj in enumerate(distinct):
            P = mp.eye(5)
            for i, li in enumerate(distinct):
                if i != j:
                    P = P * (M - li * I) / (lj - li)
            out += fn(lj) * P
        return out

    def absA(self, q):
        return self.matfun(self.A(0, q), lambda x: abs(x))

    def signA(self, q):
        tiny = mp.mpf(10) ** (-25)
        return self.matfun(self.A(1, q), lambda x: mp.mpf(0) if abs(x) < tiny else mp.sign(x))

    # ---- free surface and equilibrium (Sec. 2.1, 3.5) -------------------------------------------
    def detector(self, Q):
        y0 = []
        for i in range(self.nx):
            jb = 0
            while jb < self.ny and not self.fluid(i, jb):
                jb += 1
            total = mp.fsum((Q[3][j][i] - self.ag) / (self.al - self.ag) for j in range(jb, self.ny))
            y0.append(self.ylo + jb * self.dy + self.dy * total)
        return y0

    def eq(self, liquid, y0, y):
        if liquid:
            a = self.g * self.rho0 / self.k0
            return [self.al * self.rho0 * mp.exp(-a * (y - y0)), mp.mpf(0), mp.mpf(0), self.al, y]
        return [self.ag * self.rho0, mp.mpf(0), mp.mpf(0), self.ag, y]

    def yc(self, j):
        return self.ylo + (j + mp.mpf(1) / 2) * self.dy

    # ---- reconstruction (Sec. 3.4) --------------------------------------------------------------
    def reconstruct(self, Q, y0, i, j, dt):
        yc = self.yc(j)
        liquid = yc < y0[i]
        qc = [Q[k][j][i] for k in range(4)] + [yc]
        ec = self.eq(liquid, y0[i], yc)
        thr = 10 * self.ag
        so = all(not self.fluid(i + di, j + dj) or Q[3][j + dj][i + di] > thr
                 for dj in (-1, 0, 1) for di in (-1, 0, 1))
        rec = {"so": so, "ec": ec}
        if not so:
            rec["face"] = {f: list(qc) for f in (W, E, S, N)}
            rec["efac"] = {f: list(ec) for f in (W, E, S, N)}
            return rec
        fc = [qc[k] - ec[k] for k in range(4)]
        phi = {}
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                ii, jj = i + di, j + dj
                if self.fluid(ii, jj):
                    en = self.eq(liquid, y0[i], self.yc(jj))
                    phi[di, dj] = [Q[k][jj][ii] - en[k] for k in range(4)]
                else:
                    outx, outy = not 0 <= ii < self.nx, not 0 <= jj < self.ny
                    inside = not outx and not outy
                    side_x = W if ii < 0 else E
                    side_y = S if jj < 0 else N
                    mx = di != 0 and (inside or (outx and self.bc[side_x] == 0))
                    my = dj != 0 and (inside or (outy and self.bc[side_y] == 0))
                    phi[di, dj] = [fc[0], -fc[1] if mx else fc[1], -fc[2] if my else fc[2], fc[3]]
        gx, gy = [], []
        for k in range(4):
            cx = (phi[1, 0][k] - phi[-1, 0][k]) / (2 * self.dx)
            cy = (phi[0, 1][k] - phi[0, -1][k]) / (2 * self.dy)
            hi = max(p[k] for p in phi.values())
            lo = min(p[k] for p in phi.values())
            psi = mp.mpf(1)
            for d in (cx * self.dx / 2, -cx * self.dx / 2, cy * self.dy / 2, -cy * self.dy / 2):
                if d > 0:
                    psi = min(psi, (hi - fc[k]) / d)
                elif d < 0:
                    psi = min(psi, (lo - fc[k]) / d)
            gx.append(psi * cx)
            gy.append(psi * cy)
        a = self.g * self.rho0 / self.k0
        dxq = gx + [mp.mpf(0)]
        dyq = [gy[0] + (ec[3] * (-a) * ec[0] / ec[3] if liquid else 0), gy[1], gy[2], gy[3], mp.mpf(1)]
        A1, A2 = self.A(0, qc), self.A(1, qc)
        dtq = [-(mp.fsum(A1[r, c] * dxq[c] for c in range(5)) + mp.fsum(A2[r, c] * dyq[c] for c in range(5)))
               for r in range(5)]
        off = {W: (-self.dx / 2, 0), E: (self.dx / 2, 0), S: (0, -self.dy / 2), N: (0, self.dy / 2)}
        rec["face"], rec["efac"] = {}, {}
        for f, (ox, oy) in off.items():
            ef = self.eq(liquid, y0[i], yc + oy)
            rec["efac"][f] = ef
            rec["face"][f] = [ef[k] + fc[k] + gx[k] * ox + gy[k] * oy + dt / 2 * dtq[k] for k in range(4)] + [yc + oy]
        qh = [qc[k] + dt / 2 * dtq[k] for k in range(4)]
        fE, fW = self.f(rec["face"][E]), self.f(rec["face"][W])
        gN, gS = self.gflux(rec["face"][N]), self.gflux(rec["face"][S])
        rec["fdiff"] = [fE[k] - fW[k] for k in range(4)]
        rec["gdiff"] = [gN[k] - gS[k] for k in range(4)]
        # cell integral of the non-conservative products at (x_c, t^{n+1/2}): d_y(alpha p)^f + g (alpha rho)^f,
        # and u d_x alpha + v d_y alpha
        rec["vol"] = [mp.mpf(0), mp.mpf(0),
                      self.k0 * (gy[0] / self.rho0 - gy[3]) + self.g * (qh[0] - ec[0]),
                      qh[1] / qh[0] * gx[3] + qh[2] / qh[0] * gy[3]]
        return rec

    # ---- edges (Sec. 3.1-3.3) -------------------------------------------------------------------
    def ghost(self, q, normal, transmissive):
        g = list(q)
        if not transmissive:
            g[normal] = -g[normal]
        return g

    def osher_x(self, qm, qp):
        d = [qp[k] - qm[k] for k in range(5)]
        V = [mp.mpf(0)] * 5
        ubar = mp.mpf(0)
        for s_, w in self.gl:
            ph = [qm[k] + s_ * d[k] for k in range(5)]
            M = self.absA(ph)
            for a in range(5):
                V[a] += w * mp.fsum(M[a, b] * d[b] for b in range(5))
            ubar += w * ph[1] / ph[0]
        fm, fp = self.f(qm), self.f(qp)
        cen = [fp[k] - fm[k] for k in range(5)]
        cen[3] += ubar * d[3]
        return [(cen[k] - V[k]) / 2 for k in range(5)], [(cen[k] + V[k]) / 2 for k in range(5)]

    def b3(self, a, ea, b, eb):
        rho = lambda z: z[0] / z[3]
        pa, pb = self.alpha_p(a), self.alpha_p(b)
        pea, peb = self.alpha_p(ea), self.alpha_p(eb)
        abar, rbar = (a[3] + b[3]) / 2, (rho(a) + rho(b)) / 2
        aebar, rebar = (ea[3] + eb[3]) / 2, (rho(ea) + rho(eb)) / 2
        return (pb - peb) - (pa - pea) + self.g * (b[4] - a[4]) * (abar * rbar - aebar * rebar)

    def residual(self, a, ea, b, eb, vbar):
        ga, gb = self.gflux(a), self.gflux(b)
        r = [gb[k] - ga[k] for k in range(5)]
        r[2] += self.b3(a, ea, b, eb)
        r[3] += vbar * (b[3] - a[3])
        return r

    def osher_romberg_y(self, qm, em, qp, ep):
        at = lambda s_: [qm[k] + s_ * (qp[k] - qm[k]) for k in range(5)]
        q14, q12, q34 = at(mp.mpf(1) / 4), at(mp.mpf(1) / 2), at(mp.mpf(3) / 4)
        eh = [(em[k] + ep[k]) / 2 for k in range(5)]
        v14, v34 = q14[2] / q14[0], q34[2] / q34[0]
        R1 = self.residual(qm, em, q12, eh, v14)
        R2 = self.residual(q12, eh, qp, ep, v34)
        R3 = self.residual(qm, em, qp, ep, (v14 + v34) / 2)
        S1, S2, S3 = self.signA(q14), self.signA(q34), self.signA(q12)
        V = [mp.fsum([mp.mpf(4) / 3 * S1[a, b] * R1[b] + mp.mpf(4) / 3 * S2[a, b] * R2[b]
                      - mp.mpf(1) / 3 * S3[a, b] * R3[b] for b in range(5)]) for a in range(5)]
        return [(R3[k] - V[k]) / 2 for k in range(5)], [(R3[k] + V[k]) / 2 for k in range(5)]

    # ---- one step (Sec. 3, eq. Scheme, with the cell's own flux difference) ----------------------
    def step(self, Q, dt):
        dt = mp.mpf(dt)
        y0 = self.detector(Q)
        rec = {(i, j): self.reconstruct(Q, y0, i, j, dt)
               for j in range(self.ny) for i in range(self.nx) if self.fluid(i, j)}
        Dx = {}
        for j in range(self.ny):
            for fi in range(self.nx + 1):
                lf, rt = rec.get((fi - 1, j)), rec.get((fi, j))
                if lf is None and rt is None:
                    continue
                qm = lf["face"][E] if lf else self.ghost(rt["face"][W], 1, fi == 0 and self.bc[W] == 1)
                qp = rt["face"][W] if rt else self.ghost(lf["face"][E], 1, fi == self.nx and self.bc[E] == 1)
                Dx[fi, j] = self.osher_x(qm, qp)
        Dy = {}
        for fj in range(self.ny + 1):
            for i in range(self.nx):
                bt, tp = rec.get((i, fj - 1)), rec.get((i, fj))
                if bt is None and tp is None:
                    continue
                if bt:
                    qm, em = bt["face"][N], bt["efac"][N]
                else:
                    qm, em = self.ghost(tp["face"][S], 2, fj == 0 and self.bc[S] == 1), tp["efac"][S]
                if tp:
                    qp, ep = tp["face"][S], tp["efac"][S]
                else:
                    qp, ep = self.ghost(bt["face"][N], 2, fj == self.ny and self.bc[N] == 1), bt["efac"][N]
                Dy[i, fj] = self.osher_romberg_y(qm, em, qp, ep)
        out = [[[Q[k][j][i] for i in range(self.nx)] for j in range(self.ny)] for k in range(4)]
        for (i, j), r in rec.items():
            DpW, DmE = Dx[i, j][1], Dx[i + 1, j][0]
            DpS, DmN = Dy[i, j][1], Dy[i, j + 1][0]
            for k in range(4):
                xs = DpW[k] + DmE[k] + (r["fdiff"][k] if r["so"] else 0)
                ys = DpS[k] + DmN[k] + (r["gdiff"][k] if r["so"] else 0)
                vol = r["vol"][k] if r["so"] else 0
                out[k][j][i] = Q[k][j][i] - dt / self.dx * xs - dt / self.dy * ys - dt * vol
        return out
