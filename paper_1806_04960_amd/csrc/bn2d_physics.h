// Device-side physics of the reduced Baer-Nunziato model and of the path-conservative edge
// solvers (Gaburro, Castro, Dumbser, arXiv:1806.04960, Sec. 2-3), FP64, gfx950.
//
// The gravity potential y (5th conserved variable of Sec. 2.1) never carries a jump through the
// edge viscosities (its row of A1/A2 is zero and x-edges join states at one height), so |A1| and
// sign(A2) act here on the four stored components only, in the closed form of the paper's
// eigenvectors R1, R1^{-1}, R2, R2^{-1} (Sec. 3).  With gamma = 1, rho c^2 - p = k0 and
// (rho c^2 - p)/c^2 = rho0 exactly.
#pragma once

// The same source also compiles on the host with a counting scalar type (bn2d_flops.cpp), which
// is how the algorithmic FLOP count per cell update is measured.
#ifdef BN2D_HOST_COUNT
#define BN_DEV inline
#else
#include <hip/hip_runtime.h>
#define BN_DEV __device__ __forceinline__
typedef double real_t;
#endif

namespace bn {

struct Consts {
    int nx, ny;
    double dx, dy, ylo;
    double g, k0, rho0, al, ag, cfl;
    int bc[4];             // W, E, S, N: 0 reflective, 1 transmissive
    double c, c2, inv_c2, inv2c, half_rho0;
    double a;              // g rho0 / k0, decay rate of the hydrostatic density (Sec. 2.1)
    double e_up1, e_dn1;   // exp(-a dy), exp(+a dy): density ratio one row up / down
    double e_uph, e_dnh;   // exp(-a dy/2), exp(+a dy/2): ratio to the upper / lower edge
    double so_thr;         // 10 alpha_gas: second-order threshold (Sec. 3.4)
    double inv_dx, inv_dy, inv2dx, inv2dy, inv_rho0;
    double inv_dal;        // 1 / (alpha_l - alpha_g)
};

// Cell flags: fluid, outside the grid on a side, and (F_TX, F_TY) outside across a transmissive
// side in x or y.  Solid cells and cells outside across a reflective wall are mirrored.
enum : int { F_FLUID = 1, F_OUTW = 2, F_OUTE = 4, F_OUTS = 8, F_OUTN = 16, F_TX = 32, F_TY = 64 };
// Bits that stencils with S::kRingFlags add to the flags of their cells once per cell: a fluid cell
// without liquid (alpha <= 10 alpha_gas, Sec. 3.4), so that the second-order test of a window is one
// test of its flags, and for a cell that is not fluid whether its mirror image negates the x (F_MX)
// and the y (F_MY) momentum of the centre (a solid cell, or one outside across a reflective side).
enum : int { F_LOWA = 128, F_MX = 256, F_MY = 512 };

BN_DEV int mirror_bits(int f)
{
    const bool outx = f & (F_OUTW | F_OUTE), outy = f & (F_OUTS | F_OUTN);
    const bool inside = !outx && !outy;
    return ((inside || (outx && !(f & F_TX))) ? F_MX : 0) | ((inside || (outy && !(f & F_TY))) ? F_MY : 0);
}

// Flags of cell (i, j) of an nx x ny grid with boundary types bc (W, E, S, N; 1 transmissive).
BN_DEV int cell_flags(int i, int j, int nx, int ny, const int bc[4], bool fluid)
{
    int f = fluid ? F_FLUID : 0;
    if (i < 0) f |= F_OUTW | (bc[0] == 1 ? F_TX : 0);
    if (i >= nx) f |= F_OUTE | (bc[1] == 1 ? F_TX : 0);
    if (j < 0) f |= F_OUTS | (bc[2] == 1 ? F_TY : 0);
    if (j >= ny) f |= F_OUTN | (bc[3] == 1 ? F_TY : 0);
    return f;
}

BN_DEV real_t sgn(real_t x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

// A constant read once for the whole wavefront and held in scalar registers.  A per-lane choice
// between two constants is then a register select: left to itself the compiler may turn it into a
// per-lane vector load from the chosen field's address, whose memory latency every later wait for
// vector memory then pays.
#ifdef BN2D_HOST_COUNT
BN_DEV real_t uniform(real_t x) { return x; }
#else
BN_DEV double uniform(double x)
{
    asm volatile("" : "+s"(x));
    return x;
}
#endif

// 1/x: the hardware reciprocal (relative error about 2^-24) refined by one Newton step, whose
// error is the square of that: within 16 ulps of the quotient (at most 11 measured over 4 M
// log-uniform inputs of 1e-8 ... 1e8; a second step makes it exact there but costs 2-3 % of the
// step's time, against a parity budget of 1e-11).
#ifdef BN2D_HOST_COUNT
BN_DEV real_t rcp(real_t x) { return 1.0 / x; }
#else
BN_DEV double rcp(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
#endif

// Physical flux f (x) of Sec. 2.1 with alpha p = alpha k0 (rho/rho0 - 1) = k0 (alpha rho / rho0 - alpha).
BN_DEV void flux_f(const Consts &K, const real_t q[4], real_t inv_q0, real_t f[4])
{
    const real_t u = q[1] * inv_q0, v = q[2] * inv_q0;
    f[0] = q[1];
    f[1] = q[1] * u + K.k0 * (q[0] * K.inv_rho0 - q[3]);
    f[2] = q[1] * v;
    f[3] = 0.0;
}

// Physical flux g (y): no pressure, d_y(alpha p) is part of B2 (Sec. 2.1).
BN_DEV void flux_g(const real_t q[4], real_t inv_q0, real_t g[4])
{
    const real_t u = q[1] * inv_q0, v = q[2] * inv_q0;
    g[0] = q[2];
    g[1] = q[2] * u;
    g[2] = q[2] * v;
    g[3] = 0.0;
}

// |A1(u, v)| d  =  sum_m r_m |lambda_m| (l_m . d),  lambda = (u-c, u, u, u+c)  (Sec. 3).
BN_DEV void abs_a1(const Consts &K, real_t u, real_t v, const real_t d[4], real_t out[4])
{
    const real_t c = K.c;
    const real_t l1 = ((c + u) * K.inv2c) * d[0] - d[1] * K.inv2c - K.half_rho0 * d[3];
    const real_t l2 = -v * d[0] + d[2] + v * K.rho0 * d[3];
    const real_t l3 = d[3] * K.inv_c2;
    const real_t l5 = ((c - u) * K.inv2c) * d[0] + d[1] * K.inv2c - K.half_rho0 * d[3];
    const real_t au = fabs(u);
    const real_t w1 = fabs(u - c) * l1, w2 = au * l2, w3 = au * l3, w5 = fabs(u + c) * l5;
    out[0] = w1 + K.k0 * w3 + w5;
    out[1] = (u - c) * w1 + u * K.k0 * w3 + (u + c) * w5;
    out[2] = v * w1 + w2 + v * w5;
    out[3] = K.c2 * w3;
}

// sign(A2(u, v)) r  =  sum_m r_m sign(lambda_m) (l_m . r),  lambda = (v-c, v, v, v+c), sign(0) = 0.
// `sub`: |v| < c is known (then sign(v - c) = -1 and sign(v + c) = 1 exactly).
BN_DEV void sign_a2(const Consts &K, real_t u, real_t v, const real_t r[4], real_t out[4], bool sub)
{
    const real_t c = K.c;
    const real_t l1 = ((c + v) * K.inv2c) * r[0] - r[2] * K.inv2c - K.half_rho0 * r[3];
    const real_t l2 = -u * r[0] + r[1] + u * K.rho0 * r[3];
    const real_t l3 = r[3] * K.inv_c2;
    const real_t l5 = ((c - v) * K.inv2c) * r[0] + r[2] * K.inv2c - K.half_rho0 * r[3];
    const real_t sv = sgn(v);
    real_t slo = -1.0, shi = 1.0;
    if (!sub) {
        slo = sgn(v - c);
        shi = sgn(v + c);
    }
    const real_t w1 = slo * l1, w2 = sv * l2, w3 = sv * l3, w5 = shi * l5;
    out[0] = w1 + K.k0 * w3 + w5;
    out[1] = u * w1 + w2 + u * w5;
    out[2] = (v - c) * w1 + v * K.k0 * w3 + (v + c) * w5;
    out[3] = K.c2 * w3;
}

// x-edge: D-+ = 1/2 [ f(q+) - f(q-) + (0,0,0, ubar dalpha) -+ V dq ], Osher viscosity and the
// alpha-advection velocity ubar both integrated along the segment path with 3-point
// Gauss-Legendre (Sec. 3.2).
BN_DEV void edge_x(const Consts &K, const real_t qm[4], const real_t qp[4], real_t Dm[4],
                                       real_t Dp[4])
{
    const real_t s_gl[3] = {0.5 - 0.3872983346207416885, 0.5, 0.5 + 0.3872983346207416885};
    const real_t w_gl[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    real_t d[4], fm[4], fp[4], V[4] = {0.0, 0.0, 0.0, 0.0};
    real_t ubar = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) d[k] = qp[k] - qm[k];
    flux_f(K, qm, rcp(qm[0]), fm);
    flux_f(K, qp, rcp(qp[0]), fp);
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        real_t phi[4], t[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) phi[k] = qm[k] + s_gl[n] * d[k];
        const real_t inv = rcp(phi[0]);
        const real_t u = phi[1] * inv, v = phi[2] * inv;
        abs_a1(K, u, v, d, t);
#pragma unroll
        for (int k = 0; k < 4; ++k) V[k] += w_gl[n] * t[k];
        ubar += w_gl[n] * u;
    }
    real_t B[4] = {0.0, 0.0, 0.0, ubar * d[3]};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const real_t cen = fp[k] - fm[k] + B[k];
        Dm[k] = 0.5 * (cen - V[k]);
        Dp[k] = 0.5 * (cen + V[k]);
    }
}

// alpha p - alpha^E p^E = k0 ((alpha rho - (alpha rho)^E)/rho0 - (alpha - alpha^E))  (gamma = 1).
BN_DEV real_t press_fluct(const Consts &K, const real_t q[4], real_t e1, real_t aE)
{
    return K.k0 * ((q[0] - e1) * K.inv_rho0 - (q[3] - aE));
}

// Well-balanced b_3 on one sub-interval (Sec. 3.3): fluctuation pressure jump plus the gravity
// term of the fluctuations, (mean(alpha) mean(rho) - mean(alpha^E) mean(rho^E)) g (y_b - y_a).
// `grav` is false when the gravity part vanishes exactly (ya == yb) wherever it is evaluated
// together (a whole wavefront on the device), which skips it.
BN_DEV real_t b3(const Consts &K, const real_t qa[4], real_t e1a, real_t aEa, real_t Pa,
                                     real_t ya, const real_t qb[4], real_t e1b, real_t aEb, real_t Pb, real_t yb,
                                     bool grav)
{
    if (!grav) return Pb - Pa;
    const real_t abar = 0.5 * (qa[3] + qb[3]);
    const real_t rbar = 0.5 * (qa[0] * rcp(qa[3]) + qb[0] * rcp(qb[3]));
    const real_t aEbar = 0.5 * (aEa + aEb);
    const real_t rEbar = 0.5 * (e1a * rcp(aEa) + e1b * rcp(aEb));
    return (Pb - Pa) + (abar * rbar - aEbar * rEbar) * K.g * (yb - ya);
}

// Whether the states of a y-edge sit at different heights: per lane on the host, for the whole
// wavefront on the device (a uniform branch).
#ifdef BN2D_HOST_COUNT
BN_DEV bool y_jump(real_t ym, real_t yp) { return ym != yp; }
BN_DEV bool any_lane(bool p) { return p; }
BN_DEV bool all_lanes(bool p) { return p; }
#else
BN_DEV bool y_jump(double ym, double yp) { return __ballot(ym != yp) != 0ull; }
// whether p holds in some (every) active lane of the wavefront: a uniform branch condition
BN_DEV bool any_lane(bool p) { return __ballot(p) != 0ull; }
BN_DEV bool all_lanes(bool p) { return __ballot(!p) == 0ull; }
#endif

// y-edge: well-balanced Osher-Romberg (Sec. 3.3, Romberg l = 3 of Sec. 3.1):
//   V = 4/3 sign(A2(Phi(1/4))) R(0,1/2) + 4/3 sign(A2(Phi(3/4))) R(1/2,1) - 1/3 sign(A2(Phi(1/2))) R(0,1)
//   D-+ = 1/2 [ R(0,1) -+ V ],  R(a,b) = g(b) - g(a) + (0, 0, b_3, vbar dalpha)
// with vbar = v(Phi(1/4)), v(Phi(3/4)) and their mean on [0,1] (midpoint rule per sub-interval).
BN_DEV void edge_y(const Consts &K, const real_t qm[4], real_t e1m, real_t aEm, real_t ym,
                                       const real_t qp[4], real_t e1p, real_t aEp, real_t yp, real_t Dm[4],
                                       real_t Dp[4])
{
    real_t d[4], q14[4], q12[4], q34[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        d[k] = qp[k] - qm[k];
        q14[k] = qm[k] + 0.25 * d[k];
        q12[k] = qm[k] + 0.5 * d[k];
        q34[k] = qm[k] + 0.75 * d[k];
    }
    const real_t e1h = e1m + 0.5 * (e1p - e1m), aEh = aEm + 0.5 * (aEp - aEm), yh = ym + 0.5 * (yp - ym);
    const real_t im = rcp(qm[0]), ip = rcp(qp[0]), i12 = rcp(q12[0]);
    const real_t i14 = rcp(q14[0]), i34 = rcp(q34[0]);
    real_t gm[4], gh[4], gp[4];
    flux_g(qm, im, gm);
    flux_g(q12, i12, gh);
    flux_g(qp, ip, gp);
    const real_t Pm = press_fluct(K, qm, e1m, aEm), Ph = press_fluct(K, q12, e1h, aEh),
                 Pp = press_fluct(K, qp, e1p, aEp);
    const real_t u14 = q14[1] * i14, v14 = q14[2] * i14;
    const real_t u34 = q34[1] * i34, v34 = q34[2] * i34;
    const real_t u12 = q12[1] * i12, v12 = q12[2] * i12;
    real_t R1[4], R2[4], R3[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        R1[k] = gh[k] - gm[k];
        R2[k] = gp[k] - gh[k];
        R3[k] = gp[k] - gm[k];
    }
    // both states at one height (every edge between second-order cells): no gravity term
    const bool grav = y_jump(ym, yp);
    R1[2] += b3(K, qm, e1m, aEm, Pm, ym, q12, e1h, aEh, Ph, yh, grav);
    R2[2] += b3(K, q12, e1h, aEh, Ph, yh, qp, e1p, aEp, Pp, yp, grav);
    R3[2] += b3(K, qm, e1m, aEm, Pm, ym, qp, e1p, aEp, Pp, yp, grav);
    R1[3] += v14 * (q12[3] - qm[3]);
    R2[3] += v34 * (qp[3] - q12[3]);
    R3[3] += 0.5 * (v14 + v34) * d[3];
    real_t S1[4], S2[4], S3[4];
    // subsonic in every lane at the three nodes (the usual case): the outer eigenvalues' signs are known
    const bool sub = all_lanes(fabs(v14) < K.c && fabs(v34) < K.c && fabs(v12) < K.c);
    sign_a2(K, u14, v14, R1, S1, sub);
    sign_a2(K, u34, v34, R2, S2, sub);
    sign_a2(K, u12, v12, R3, S3, sub);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const real_t V = (4.0 / 3.0) * S1[k] + (4.0 / 3.0) * S2[k] - (1.0 / 3.0) * S3[k];
        Dm[k] = 0.5 * (R3[k] - V);
        Dp[k] = 0.5 * (R3[k] + V);
    }
}

struct Rec {
    real_t qW[4], qE[4], qS[4], qN[4];  // edge-midpoint states at t^{n+1/2}
    real_t e1S, e1N, aE;                // equilibrium parts (alpha rho)^E, alpha^E of the S/N states
    real_t yS, yN;                      // heights of the S/N states
    real_t fdiff[4], gdiff[4];          // f(q_E) - f(q_W), g(q_N) - g(q_S)
    real_t vol2, vol3;                  // cell integral of B(q) grad q (components 3 and 4)
};

// Well-balanced second-order reconstruction with Hancock predictor of the window centre
// (Sec. 3.4): fluctuations of the 3 x 3 stencil with respect to the centre cell's water-at-rest
// profile (Sec. 2.1, free surface y0c of its column), Barth-Jespersen limited central
// gradients component by component, d_t Q = -(A1 d_x Q + A2 d_y Q) with grad Q = grad Q^E +
// Psi grad Q^f.  Second order only if the centre and every fluid stencil cell hold liquid
// (alpha > 10 alpha_gas); otherwise the first-order states of Sec. 3.2/3.3.
// The stencil is read through S: S.q(dj, di, k) is component k of the cell at row offset dj - 1 and
// column offset di - 1, S.f(dj, di) its F_* flags.
template <class S>
BN_DEV void reconstruct(const Consts &K, const S &st, int j, real_t y0c, real_t dt, Rec &r)
{
    real_t wq[3][3][4];
    int wf[3][3];
#pragma unroll
    for (int dj = 0; dj < 3; ++dj)
#pragma unroll
        for (int di = 0; di < 3; ++di) {
            wf[dj][di] = st.f(dj, di);
#pragma unroll
            for (int k = 0; k < 4; ++k) wq[dj][di][k] = st.q(dj, di, k);
        }
    const real_t *Qc = wq[1][1];
    const real_t yc = K.ylo + (j + 0.5) * K.dy;
    const bool liquid = yc < y0c;
    const real_t aE = liquid ? uniform(K.al) : uniform(K.ag);
    // (the exponential only where some lane holds a liquid-type cell: gas rows skip it)
    real_t rE0 = K.rho0;
    if (any_lane(liquid)) rE0 = liquid ? K.rho0 * exp(-K.a * (yc - y0c)) : K.rho0;
    const real_t e1c = aE * rE0;
    r.aE = aE;

    bool so;
    if constexpr (S::kRingFlags) {
        int any = 0;
#pragma unroll
        for (int dj = 0; dj < 3; ++dj)
#pragma unroll
            for (int di = 0; di < 3; ++di) any |= wf[dj][di];
        so = !(any & F_LOWA);
    } else {
        so = Qc[3] > K.so_thr;
#pragma unroll
        for (int dj = 0; dj < 3; ++dj)
#pragma unroll
            for (int di = 0; di < 3; ++di)
                if ((wf[dj][di] & F_FLUID) && !(wq[dj][di][3] > K.so_thr)) so = false;
    }

    if (!so) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            r.qW[k] = Qc[k]; r.qE[k] = Qc[k]; r.qS[k] = Qc[k]; r.qN[k] = Qc[k];
            r.fdiff[k] = 0.0; r.gdiff[k] = 0.0;
        }
        r.e1S = e1c; r.e1N = e1c; r.yS = yc; r.yN = yc;
        r.vol2 = 0.0; r.vol3 = 0.0;
        return;
    }

    const real_t e1row[3] = {aE * (liquid ? rE0 * K.e_dn1 : K.rho0), e1c, aE * (liquid ? rE0 * K.e_up1 : K.rho0)};
    const real_t fc[4] = {Qc[0] - e1c, Qc[1], Qc[2], Qc[3] - aE};

    // 3x3 fluctuations of all four components (neighbours with respect to this cell's profile;
    // solid/outside neighbours mirror the centre across each reflective wall), then per component
    // central gradients and the Barth-Jespersen limiter over the four edge midpoints, whose two
    // x (y) midpoints carry +-d so that their ratios are (max - c)/|d| and (c - min)/|d|.
    // (the centre is a fluid cell: its fluctuation is fc)
    real_t phi[3][3][4];
#pragma unroll
    for (int dj = 0; dj < 3; ++dj)
#pragma unroll
        for (int di = 0; di < 3; ++di) {
            if (dj == 1 && di == 1) {
#pragma unroll
                for (int k = 0; k < 4; ++k) phi[1][1][k] = fc[k];
                continue;
            }
            // (selects rather than branches: both forms are a few operations)
            const int f = wf[dj][di];
            const bool fluid = f & F_FLUID;
            const int mb = S::kRingFlags ? f : mirror_bits(f);
            const bool fx = (di != 1) && (mb & F_MX);
            const bool fy = (dj != 1) && (mb & F_MY);
            phi[dj][di][0] = fluid ? wq[dj][di][0] - e1row[dj] : fc[0];
            phi[dj][di][1] = fluid ? wq[dj][di][1] : (fx ? -fc[1] : fc[1]);
            phi[dj][di][2] = fluid ? wq[dj][di][2] : (fy ? -fc[2] : fc[2]);
            phi[dj][di][3] = fluid ? wq[dj][di][3] - aE : fc[3];
        }
    real_t gx[4], gy[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const real_t gxr = (phi[1][2][k] - phi[1][0][k]) * K.inv2dx;
        const real_t gyr = (phi[2][1][k] - phi[0][1][k]) * K.inv2dy;
        real_t mx = phi[1][1][k], mn = phi[1][1][k];
#pragma unroll
        for (int dj = 0; dj < 3; ++dj)
#pragma unroll
            for (int di = 0; di < 3; ++di) {
                mx = fmax(mx, phi[dj][di][k]);
                mn = fmin(mn, phi[dj][di][k]);
            }
        const real_t lim = fmin(mx - fc[k], fc[k] - mn);
        const real_t hx = fabs(gxr * (0.5 * K.dx)), hy = fabs(gyr * (0.5 * K.dy));
        // Psi = min over the four midpoints of min(1, lim / |d|) = min(1, lim / max(hx, hy)) (lim >= 0),
        // 1 where both differences vanish
        const real_t hm = fmax(hx, hy);
        const real_t r = fmin(1.0, lim * rcp(hm));  // discarded if hm = 0
        const real_t psi = hm > 0.0 ? r : 1.0;
        gx[k] = psi * gxr;
        gy[k] = psi * gyr;
    }

    // Hancock predictor with A1, A2 at the cell average (Sec. 3 matrices; rho c^2 - p = k0).
    const real_t inv0 = rcp(Qc[0]);
    const real_t u = Qc[1] * inv0, v = Qc[2] * inv0;
    const real_t qy0 = gy[0] + aE * (liquid ? -K.a * rE0 : 0.0);
    real_t hdt[4];
    {
        const real_t ax0 = gx[1];
        const real_t ax1 = (K.c2 - u * u) * gx[0] + 2.0 * u * gx[1] - K.k0 * gx[3];
        const real_t ax2 = -u * v * gx[0] + v * gx[1] + u * gx[2];
        const real_t ax3 = u * gx[3];
        const real_t ay0 = gy[2];
        const real_t ay1 = -u * v * qy0 + v * gy[1] + u * gy[2];
        const real_t ay2 = (K.c2 - v * v) * qy0 + 2.0 * v * gy[2] - K.k0 * gy[3] + Qc[0] * K.g;
        const real_t ay3 = v * gy[3];
        const real_t h = -0.5 * dt;
        hdt[0] = h * (ax0 + ay0);
        hdt[1] = h * (ax1 + ay1);
        hdt[2] = h * (ax2 + ay2);
        hdt[3] = h * (ax3 + ay3);
    }

    const real_t e1S = aE * (liquid ? rE0 * K.e_dnh : K.rho0);
    const real_t e1N = aE * (liquid ? rE0 * K.e_uph : K.rho0);
    const real_t ex[4] = {e1c, 0.0, 0.0, aE}, eS[4] = {e1S, 0.0, 0.0, aE}, eN[4] = {e1N, 0.0, 0.0, aE};
    const real_t hx = 0.5 * K.dx, hy = 0.5 * K.dy;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        r.qW[k] = (ex[k] + fc[k]) + gx[k] * (-hx) + hdt[k];
        r.qE[k] = (ex[k] + fc[k]) + gx[k] * hx + hdt[k];
        r.qS[k] = (eS[k] + fc[k]) + gy[k] * (-hy) + hdt[k];
        r.qN[k] = (eN[k] + fc[k]) + gy[k] * hy + hdt[k];
    }
    r.e1S = e1S;
    r.e1N = e1N;
    r.yS = K.ylo + j * K.dy;
    r.yN = K.ylo + (j + 1) * K.dy;

    // Cell terms: the flux differences of the cell's own linear reconstruction and the midpoint
    // rule for the cell integral of B(q) grad q at (x_c, t^{n+1/2}) (Sec. 3.4).
    real_t fE[4], fW[4], gN[4], gS[4];
    flux_f(K, r.qE, rcp(r.qE[0]), fE);
    flux_f(K, r.qW, rcp(r.qW[0]), fW);
    flux_g(r.qN, rcp(r.qN[0]), gN);
    flux_g(r.qS, rcp(r.qS[0]), gS);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        r.fdiff[k] = fE[k] - fW[k];
        r.gdiff[k] = gN[k] - gS[k];
    }
    const real_t qc0 = Qc[0] + hdt[0];
    const real_t ic = rcp(qc0);
    const real_t uc = (Qc[1] + hdt[1]) * ic, vc = (Qc[2] + hdt[2]) * ic;
    r.vol2 = K.k0 * (gy[0] * K.inv_rho0 - gy[3]) + (qc0 - e1c) * K.g;
    r.vol3 = uc * gx[3] + vc * gy[3];
}


// Cell update (Sec. 3, eq. Scheme, with the cell's own flux difference [full system matrix]):
//   Q^{n+1} = Q^n - dt/dx (D+_W + D-_E + f(q_E) - f(q_W)) - dt/dy (D+_S + D-_N + g(q_N) - g(q_S)) - dt B(q) grad q
// split into everything known once the row's x-edges are solved, X, and the y-edge terms.
BN_DEV void update_partial(const real_t Qn[4], const real_t DpW[4], const real_t DmE[4], const real_t fdiff[4],
                           const real_t gdiff[4], real_t vol2, real_t vol3, real_t dt, real_t dtdx, real_t dtdy,
                           real_t X[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) X[k] = Qn[k] - dtdx * ((DpW[k] + DmE[k]) + fdiff[k]) - dtdy * gdiff[k];
    X[2] = X[2] - dt * vol2;
    X[3] = X[3] - dt * vol3;
}

// The south edge's D+ applied to a partial update (when the row above is being solved), then the
// north edge's D- (when that edge is known): what the cell's update is waiting for is 4 values.
BN_DEV void update_south(const real_t X[4], const real_t DpS[4], real_t dtdy, real_t P[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) P[k] = X[k] - dtdy * DpS[k];
}

BN_DEV void update_finish(const real_t P[4], const real_t DmN[4], real_t dtdy, real_t q[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = P[k] - dtdy * DmN[k];
}

// Free-surface detector term of a fluid cell (Sec. 3.5) and its CFL rate (|u|+c)/dx + (|v|+c)/dy.
BN_DEV real_t detector_term(const Consts &K, const real_t q[4]) { return (q[3] - K.ag) * K.inv_dal; }

BN_DEV real_t cfl_rate(const Consts &K, const real_t q[4])
{
    const real_t iq = rcp(q[0]);
    return (fabs(q[1] * iq) + K.c) * K.inv_dx + (fabs(q[2] * iq) + K.c) * K.inv_dy;
}

}  // namespace bn
