// Device-side physics of the reduced Baer-Nunziato model and of the path-conservative edge
// solvers (Gaburro, Castro, Dumbser, arXiv:1806.04960, Sec. 2-3), FP64, gfx950.
//
// The gravity potential y (5th conserved variable of Sec. 2.1) never carries a jump through the
// edge viscosities (its row of A1/A2 is zero and x-edges join states at one height), so |A1| and
// sign(A2) act here on the four stored components only, in the closed form of the paper's
// eigenvectors R1, R1^{-1}, R2, R2^{-1} (Sec. 3).  With gamma = 1, rho c^2 - p = k0 and
// (rho c^2 - p)/c^2 = rho0 exactly.
#pragma once
#include <hip/hip_runtime.h>

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
};

enum : int { F_FLUID = 1, F_OUTW = 2, F_OUTE = 4, F_OUTS = 8, F_OUTN = 16 };

__device__ __forceinline__ double sgn(double x) { return (double)((x > 0.0) - (x < 0.0)); }

// Physical flux f (x) of Sec. 2.1 with alpha p = alpha k0 (rho/rho0 - 1) = k0 (alpha rho / rho0 - alpha).
__device__ __forceinline__ void flux_f(const Consts &K, const double q[4], double inv_q0, double f[4])
{
    const double u = q[1] * inv_q0, v = q[2] * inv_q0;
    f[0] = q[1];
    f[1] = q[1] * u + K.k0 * (q[0] / K.rho0 - q[3]);
    f[2] = q[1] * v;
    f[3] = 0.0;
}

// Physical flux g (y): no pressure, d_y(alpha p) is part of B2 (Sec. 2.1).
__device__ __forceinline__ void flux_g(const double q[4], double inv_q0, double g[4])
{
    const double u = q[1] * inv_q0, v = q[2] * inv_q0;
    g[0] = q[2];
    g[1] = q[2] * u;
    g[2] = q[2] * v;
    g[3] = 0.0;
}

// |A1(u, v)| d  =  sum_m r_m |lambda_m| (l_m . d),  lambda = (u-c, u, u, u+c)  (Sec. 3).
__device__ __forceinline__ void abs_a1(const Consts &K, double u, double v, const double d[4], double out[4])
{
    const double c = K.c;
    const double l1 = ((c + u) * K.inv2c) * d[0] - d[1] * K.inv2c - K.half_rho0 * d[3];
    const double l2 = -v * d[0] + d[2] + v * K.rho0 * d[3];
    const double l3 = d[3] * K.inv_c2;
    const double l5 = ((c - u) * K.inv2c) * d[0] + d[1] * K.inv2c - K.half_rho0 * d[3];
    const double au = fabs(u);
    const double w1 = fabs(u - c) * l1, w2 = au * l2, w3 = au * l3, w5 = fabs(u + c) * l5;
    out[0] = w1 + K.k0 * w3 + w5;
    out[1] = (u - c) * w1 + u * K.k0 * w3 + (u + c) * w5;
    out[2] = v * w1 + w2 + v * w5;
    out[3] = K.c2 * w3;
}

// sign(A2(u, v)) r  =  sum_m r_m sign(lambda_m) (l_m . r),  lambda = (v-c, v, v, v+c), sign(0) = 0.
__device__ __forceinline__ void sign_a2(const Consts &K, double u, double v, const double r[4], double out[4])
{
    const double c = K.c;
    const double l1 = ((c + v) * K.inv2c) * r[0] - r[2] * K.inv2c - K.half_rho0 * r[3];
    const double l2 = -u * r[0] + r[1] + u * K.rho0 * r[3];
    const double l3 = r[3] * K.inv_c2;
    const double l5 = ((c - v) * K.inv2c) * r[0] + r[2] * K.inv2c - K.half_rho0 * r[3];
    const double sv = sgn(v);
    const double w1 = sgn(v - c) * l1, w2 = sv * l2, w3 = sv * l3, w5 = sgn(v + c) * l5;
    out[0] = w1 + K.k0 * w3 + w5;
    out[1] = u * w1 + w2 + u * w5;
    out[2] = (v - c) * w1 + v * K.k0 * w3 + (v + c) * w5;
    out[3] = K.c2 * w3;
}

// x-edge: D-+ = 1/2 [ f(q+) - f(q-) + (0,0,0, ubar dalpha) -+ V dq ], Osher viscosity and the
// alpha-advection velocity ubar both integrated along the segment path with 3-point
// Gauss-Legendre (Sec. 3.2).
__device__ __forceinline__ void edge_x(const Consts &K, const double qm[4], const double qp[4], double Dm[4],
                                       double Dp[4])
{
    const double s_gl[3] = {0.5 - 0.3872983346207416885, 0.5, 0.5 + 0.3872983346207416885};
    const double w_gl[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    double d[4], fm[4], fp[4], V[4] = {0.0, 0.0, 0.0, 0.0};
    double ubar = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) d[k] = qp[k] - qm[k];
    flux_f(K, qm, 1.0 / qm[0], fm);
    flux_f(K, qp, 1.0 / qp[0], fp);
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        double phi[4], t[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) phi[k] = qm[k] + s_gl[n] * d[k];
        const double inv = 1.0 / phi[0];
        const double u = phi[1] * inv, v = phi[2] * inv;
        abs_a1(K, u, v, d, t);
#pragma unroll
        for (int k = 0; k < 4; ++k) V[k] += w_gl[n] * t[k];
        ubar += w_gl[n] * u;
    }
    double B[4] = {0.0, 0.0, 0.0, ubar * d[3]};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double cen = fp[k] - fm[k] + B[k];
        Dm[k] = 0.5 * (cen - V[k]);
        Dp[k] = 0.5 * (cen + V[k]);
    }
}

// alpha p - alpha^E p^E = k0 ((alpha rho - (alpha rho)^E)/rho0 - (alpha - alpha^E))  (gamma = 1).
__device__ __forceinline__ double press_fluct(const Consts &K, const double q[4], double e1, double aE)
{
    return K.k0 * ((q[0] - e1) / K.rho0 - (q[3] - aE));
}

// Well-balanced b_3 on one sub-interval (Sec. 3.3): fluctuation pressure jump plus the gravity
// term of the fluctuations, (mean(alpha) mean(rho) - mean(alpha^E) mean(rho^E)) g (y_b - y_a).
__device__ __forceinline__ double b3(const Consts &K, const double qa[4], double e1a, double aEa, double Pa,
                                     double ya, const double qb[4], double e1b, double aEb, double Pb, double yb)
{
    double r = Pb - Pa;
    if (yb != ya) {
        const double abar = 0.5 * (qa[3] + qb[3]);
        const double rbar = 0.5 * (qa[0] / qa[3] + qb[0] / qb[3]);
        const double aEbar = 0.5 * (aEa + aEb);
        const double rEbar = 0.5 * (e1a / aEa + e1b / aEb);
        r += (abar * rbar - aEbar * rEbar) * K.g * (yb - ya);
    }
    return r;
}

// y-edge: well-balanced Osher-Romberg (Sec. 3.3, Romberg l = 3 of Sec. 3.1):
//   V = 4/3 sign(A2(Phi(1/4))) R(0,1/2) + 4/3 sign(A2(Phi(3/4))) R(1/2,1) - 1/3 sign(A2(Phi(1/2))) R(0,1)
//   D-+ = 1/2 [ R(0,1) -+ V ],  R(a,b) = g(b) - g(a) + (0, 0, b_3, vbar dalpha)
// with vbar = v(Phi(1/4)), v(Phi(3/4)) and their mean on [0,1] (midpoint rule per sub-interval).
__device__ __forceinline__ void edge_y(const Consts &K, const double qm[4], double e1m, double aEm, double ym,
                                       const double qp[4], double e1p, double aEp, double yp, double Dm[4],
                                       double Dp[4])
{
    double d[4], q14[4], q12[4], q34[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        d[k] = qp[k] - qm[k];
        q14[k] = qm[k] + 0.25 * d[k];
        q12[k] = qm[k] + 0.5 * d[k];
        q34[k] = qm[k] + 0.75 * d[k];
    }
    const double e1h = e1m + 0.5 * (e1p - e1m), aEh = aEm + 0.5 * (aEp - aEm), yh = ym + 0.5 * (yp - ym);
    const double im = 1.0 / qm[0], ip = 1.0 / qp[0], i12 = 1.0 / q12[0];
    const double i14 = 1.0 / q14[0], i34 = 1.0 / q34[0];
    double gm[4], gh[4], gp[4];
    flux_g(qm, im, gm);
    flux_g(q12, i12, gh);
    flux_g(qp, ip, gp);
    const double Pm = press_fluct(K, qm, e1m, aEm), Ph = press_fluct(K, q12, e1h, aEh),
                 Pp = press_fluct(K, qp, e1p, aEp);
    const double u14 = q14[1] * i14, v14 = q14[2] * i14;
    const double u34 = q34[1] * i34, v34 = q34[2] * i34;
    const double u12 = q12[1] * i12, v12 = q12[2] * i12;
    double R1[4], R2[4], R3[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        R1[k] = gh[k] - gm[k];
        R2[k] = gp[k] - gh[k];
        R3[k] = gp[k] - gm[k];
    }
    R1[2] += b3(K, qm, e1m, aEm, Pm, ym, q12, e1h, aEh, Ph, yh);
    R2[2] += b3(K, q12, e1h, aEh, Ph, yh, qp, e1p, aEp, Pp, yp);
    R3[2] += b3(K, qm, e1m, aEm, Pm, ym, qp, e1p, aEp, Pp, yp);
    R1[3] += v14 * (q12[3] - qm[3]);
    R2[3] += v34 * (qp[3] - q12[3]);
    R3[3] += 0.5 * (v14 + v34) * d[3];
    double S1[4], S2[4], S3[4];
    sign_a2(K, u14, v14, R1, S1);
    sign_a2(K, u34, v34, R2, S2);
    sign_a2(K, u12, v12, R3, S3);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double V = (4.0 / 3.0) * S1[k] + (4.0 / 3.0) * S2[k] - (1.0 / 3.0) * S3[k];
        Dm[k] = 0.5 * (R3[k] - V);
        Dp[k] = 0.5 * (R3[k] + V);
    }
}

}  // namespace bn
