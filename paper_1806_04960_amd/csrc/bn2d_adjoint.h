// Reverse-mode (adjoint) counterparts of the device physics in bn2d_physics.h: for each forward
// function F(x) -> y, a function that, given the forward inputs and an output adjoint ybar,
// ADDS (dF/dx)^T ybar to the input adjoints.  The forward values needed on the way back are
// recomputed from the inputs.  Together they differentiate one explicit step of the scheme
// (Sec. 3, eq. Scheme; Sec. 3.1-3.5) with respect to the state at t^n for a fixed time step.
//
// Derivative conventions at the non-smooth points of the scheme (sets of measure zero that the
// step is piecewise smooth across): |x| and sign(x) differentiate as sign(x) and 0; min / max pass
// the adjoint to the argument that the forward selection returns (the first of equal ones in the
// order the forward visits them); the discrete switches (fluid / solid, liquid below the free
// surface, second order above 10 alpha_gas, a wall's mirror) are held fixed.  The free-surface
// height is differentiated as the real-valued column sum of Sec. 3.5 (dy / (alpha_l - alpha_g) per
// fluid cell's alpha), not as its fixed-point evaluation.
#pragma once
#include "bn2d_physics.h"

namespace bn {

// d(1/x) terms: the forward uses rcp(x), within an ulp of 1/x.

// f(q) = (q1, q1 u + k0 (q0/rho0 - q3), q1 v, 0), u = q1/q0, v = q2/q0.
BN_DEV void flux_f_rev(const Consts &K, const double q[4], const double fb[4], double qb[4])
{
    const double iq = rcp(q[0]), u = q[1] * iq, v = q[2] * iq;
    qb[0] += fb[1] * (K.k0 * K.inv_rho0 - u * u) - fb[2] * (u * v);
    qb[1] += fb[0] + 2.0 * u * fb[1] + v * fb[2];
    qb[2] += u * fb[2];
    qb[3] -= K.k0 * fb[1];
}

// g(q) = (q2, q2 u, q2 v, 0).
BN_DEV void flux_g_rev(const double q[4], const double gb[4], double qb[4])
{
    const double iq = rcp(q[0]), u = q[1] * iq, v = q[2] * iq;
    qb[0] -= gb[1] * (u * v) + gb[2] * (v * v);
    qb[1] += v * gb[1];
    qb[2] += gb[0] + u * gb[1] + 2.0 * v * gb[2];
}

// u = p1 / p0, v = p2 / p0  ->  adjoints of p from those of u and v.
BN_DEV void velocity_rev(const double p[4], double ub, double vb, double pb[4])
{
    const double ip = rcp(p[0]), u = p[1] * ip, v = p[2] * ip;
    pb[0] -= (u * ub + v * vb) * ip;
    pb[1] += ub * ip;
    pb[2] += vb * ip;
}

// out = |A1(u, v)| d (abs_a1): adjoints of d, u and v.
BN_DEV void abs_a1_rev(const Consts &K, double u, double v, const double d[4], const double ob[4], double db[4],
                       double &ub, double &vb)
{
    const double c = K.c;
    const double l1 = ((c + u) * K.inv2c) * d[0] - d[1] * K.inv2c - K.half_rho0 * d[3];
    const double l2 = -v * d[0] + d[2] + v * K.rho0 * d[3];
    const double l3 = d[3] * K.inv_c2;
    const double l5 = ((c - u) * K.inv2c) * d[0] + d[1] * K.inv2c - K.half_rho0 * d[3];
    const double au = fabs(u), am = fabs(u - c), ap = fabs(u + c);
    const double w1 = am * l1, w2 = au * l2, w3 = au * l3, w5 = ap * l5;
    // out0 = w1 + k0 w3 + w5; out1 = (u-c) w1 + u k0 w3 + (u+c) w5; out2 = v w1 + w2 + v w5; out3 = c^2 w3
    const double w1b = ob[0] + (u - c) * ob[1] + v * ob[2];
    const double w2b = ob[2];
    const double w3b = K.k0 * ob[0] + u * K.k0 * ob[1] + K.c2 * ob[3];
    const double w5b = ob[0] + (u + c) * ob[1] + v * ob[2];
    ub += ob[1] * (w1 + K.k0 * w3 + w5);
    vb += ob[2] * (w1 + w5);
    const double l1b = am * w1b, l2b = au * w2b, l3b = au * w3b, l5b = ap * w5b;
    ub += sgn(u - c) * l1 * w1b + sgn(u) * (l2 * w2b + l3 * w3b) + sgn(u + c) * l5 * w5b;
    db[0] += ((c + u) * K.inv2c) * l1b - v * l2b + ((c - u) * K.inv2c) * l5b;
    db[1] += K.inv2c * (l5b - l1b);
    db[2] += l2b;
    db[3] += -K.half_rho0 * (l1b + l5b) + v * K.rho0 * l2b + K.inv_c2 * l3b;
    ub += d[0] * K.inv2c * (l1b - l5b);
    vb += (K.rho0 * d[3] - d[0]) * l2b;
}

// out = sign(A2(u, v)) r (sign_a2): adjoints of r, u and v (the signs are locally constant).
BN_DEV void sign_a2_rev(const Consts &K, double u, double v, const double r[4], const double ob[4], double rb[4],
                        double &ub, double &vb)
{
    const double c = K.c;
    const double l1 = ((c + v) * K.inv2c) * r[0] - r[2] * K.inv2c - K.half_rho0 * r[3];
    const double l2 = -u * r[0] + r[1] + u * K.rho0 * r[3];
    const double l3 = r[3] * K.inv_c2;
    const double l5 = ((c - v) * K.inv2c) * r[0] + r[2] * K.inv2c - K.half_rho0 * r[3];
    const double sm = sgn(v - c), sv = sgn(v), sp = sgn(v + c);
    const double w1 = sm * l1, w3 = sv * l3, w5 = sp * l5;
    // out0 = w1 + k0 w3 + w5; out1 = u w1 + w2 + u w5; out2 = (v-c) w1 + v k0 w3 + (v+c) w5; out3 = c^2 w3
    const double w1b = ob[0] + u * ob[1] + (v - c) * ob[2];
    const double w2b = ob[1];
    const double w3b = K.k0 * ob[0] + v * K.k0 * ob[2] + K.c2 * ob[3];
    const double w5b = ob[0] + u * ob[1] + (v + c) * ob[2];
    ub += ob[1] * (w1 + w5);
    vb += ob[2] * (w1 + K.k0 * w3 + w5);
    const double l1b = sm * w1b, l2b = sv * w2b, l3b = sv * w3b, l5b = sp * w5b;
    rb[0] += ((c + v) * K.inv2c) * l1b - u * l2b + ((c - v) * K.inv2c) * l5b;
    rb[1] += l2b;
    rb[2] += K.inv2c * (l5b - l1b);
    rb[3] += -K.half_rho0 * (l1b + l5b) + u * K.rho0 * l2b + K.inv_c2 * l3b;
    vb += r[0] * K.inv2c * (l1b - l5b);
    ub += (K.rho0 * r[3] - r[0]) * l2b;
}

// x-edge (edge_x): adjoints of q- and q+ from those of D- and D+.
BN_DEV void edge_x_rev(const Consts &K, const double qm[4], const double qp[4], const double Dmb[4],
                       const double Dpb[4], double qmb[4], double qpb[4])
{
    const double s_gl[3] = {0.5 - 0.3872983346207416885, 0.5, 0.5 + 0.3872983346207416885};
    const double w_gl[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    double d[4], db[4] = {0.0, 0.0, 0.0, 0.0}, cb[4], Vb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        d[k] = qp[k] - qm[k];
        cb[k] = 0.5 * (Dmb[k] + Dpb[k]);
        Vb[k] = 0.5 * (Dpb[k] - Dmb[k]);
    }
    // cen = f(q+) - f(q-) + (0, 0, 0, ubar d3)
    flux_f_rev(K, qp, cb, qpb);
    const double ncb[4] = {-cb[0], -cb[1], -cb[2], -cb[3]};
    flux_f_rev(K, qm, ncb, qmb);
    double ubar = 0.0;
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        double phi[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) phi[k] = qm[k] + s_gl[n] * d[k];
        const double inv = rcp(phi[0]);
        const double u = phi[1] * inv, v = phi[2] * inv;
        ubar += w_gl[n] * u;
        double tb[4], ub = w_gl[n] * cb[3] * d[3], vb = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) tb[k] = w_gl[n] * Vb[k];
        abs_a1_rev(K, u, v, d, tb, db, ub, vb);
        double phib[4] = {0.0, 0.0, 0.0, 0.0};
        velocity_rev(phi, ub, vb, phib);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            qmb[k] += phib[k];
            db[k] += s_gl[n] * phib[k];
        }
    }
    db[3] += cb[3] * ubar;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        qpb[k] += db[k];
        qmb[k] -= db[k];
    }
}

// alpha p fluctuation (press_fluct): adjoints of q and e1 (alpha^E is a constant of the cell type).
BN_DEV void press_fluct_rev(const Consts &K, double Pb, double qb[4], double &e1b)
{
    qb[0] += K.k0 * K.inv_rho0 * Pb;
    e1b -= K.k0 * K.inv_rho0 * Pb;
    qb[3] -= K.k0 * Pb;
}

// b_3 (b3): adjoints of qa, e1a, Pa, qb, e1b, Pb.
BN_DEV void b3_rev(const Consts &K, const double qa[4], double e1a, double aEa, double ya, const double qb[4],
                   double e1b, double aEb, double yb, double ob, double qab[4], double &e1ab, double &Pab,
                   double qbb[4], double &e1bb, double &Pbb)
{
    Pbb += ob;
    Pab -= ob;
    const double G = K.g * (yb - ya);
    const double ia = rcp(qa[3]), ib = rcp(qb[3]);
    const double abar = 0.5 * (qa[3] + qb[3]);
    const double rbar = 0.5 * (qa[0] * ia + qb[0] * ib);
    const double aEbar = 0.5 * (aEa + aEb);
    const double abarb = ob * G * rbar, rbarb = ob * G * abar, rEbarb = -ob * G * aEbar;
    qab[3] += 0.5 * abarb - 0.5 * rbarb * qa[0] * ia * ia;
    qbb[3] += 0.5 * abarb - 0.5 * rbarb * qb[0] * ib * ib;
    qab[0] += 0.5 * rbarb * ia;
    qbb[0] += 0.5 * rbarb * ib;
    e1ab += 0.5 * rEbarb * rcp(aEa);
    e1bb += 0.5 * rEbarb * rcp(aEb);
}

// y-edge (edge_y): adjoints of q-, e1-, q+, e1+ from those of D- and D+.
BN_DEV void edge_y_rev(const Consts &K, const double qm[4], double e1m, double aEm, double ym, const double qp[4],
                       double e1p, double aEp, double yp, const double Dmb[4], const double Dpb[4], double qmb[4],
                       double &e1mb, double qpb[4], double &e1pb)
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
    const double i14 = rcp(q14[0]), i34 = rcp(q34[0]), i12 = rcp(q12[0]);
    const double u14 = q14[1] * i14, v14 = q14[2] * i14;
    const double u34 = q34[1] * i34, v34 = q34[2] * i34;
    const double u12 = q12[1] * i12, v12 = q12[2] * i12;
    // forward residuals (their values enter the adjoint of the sign matrices' eigenvector terms)
    double gm[4], gh[4], gp[4];
    flux_g(qm, rcp(qm[0]), gm);
    flux_g(q12, i12, gh);
    flux_g(qp, rcp(qp[0]), gp);
    const double Pm = press_fluct(K, qm, e1m, aEm), Ph = press_fluct(K, q12, e1h, aEh),
                 Pp = press_fluct(K, qp, e1p, aEp);
    double R1[4], R2[4], R3[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        R1[k] = gh[k] - gm[k];
        R2[k] = gp[k] - gh[k];
        R3[k] = gp[k] - gm[k];
    }
    const bool grav = y_jump(ym, yp);
    R1[2] += b3(K, qm, e1m, aEm, Pm, ym, q12, e1h, aEh, Ph, yh, grav);
    R2[2] += b3(K, q12, e1h, aEh, Ph, yh, qp, e1p, aEp, Pp, yp, grav);
    R3[2] += b3(K, qm, e1m, aEm, Pm, ym, qp, e1p, aEp, Pp, yp, grav);
    R1[3] += v14 * (q12[3] - qm[3]);
    R2[3] += v34 * (qp[3] - q12[3]);
    R3[3] += 0.5 * (v14 + v34) * d[3];

    // D-+ = 1/2 (R3 -+ V), V = 4/3 S1 + 4/3 S2 - 1/3 S3
    double R1b[4] = {0, 0, 0, 0}, R2b[4] = {0, 0, 0, 0}, R3b[4], S1b[4], S2b[4], S3b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        R3b[k] = 0.5 * (Dmb[k] + Dpb[k]);
        const double Vb = 0.5 * (Dpb[k] - Dmb[k]);
        S1b[k] = (4.0 / 3.0) * Vb;
        S2b[k] = (4.0 / 3.0) * Vb;
        S3b[k] = -(1.0 / 3.0) * Vb;
    }
    double u14b = 0.0, v14b = 0.0, u34b = 0.0, v34b = 0.0, u12b = 0.0, v12b = 0.0;
    sign_a2_rev(K, u14, v14, R1, S1b, R1b, u14b, v14b);
    sign_a2_rev(K, u34, v34, R2, S2b, R2b, u34b, v34b);
    sign_a2_rev(K, u12, v12, R3, S3b, R3b, u12b, v12b);

    double q12b[4] = {0, 0, 0, 0}, q14b[4] = {0, 0, 0, 0}, q34b[4] = {0, 0, 0, 0}, db[4] = {0, 0, 0, 0};
    double e1hb = 0.0, Pmb = 0.0, Phb = 0.0, Ppb = 0.0;
    // the alpha-advection terms
    v14b += R1b[3] * (q12[3] - qm[3]);
    q12b[3] += R1b[3] * v14;
    qmb[3] -= R1b[3] * v14;
    v34b += R2b[3] * (qp[3] - q12[3]);
    qpb[3] += R2b[3] * v34;
    q12b[3] -= R2b[3] * v34;
    v14b += 0.5 * d[3] * R3b[3];
    v34b += 0.5 * d[3] * R3b[3];
    db[3] += 0.5 * (v14 + v34) * R3b[3];
    // the b_3 terms
    b3_rev(K, qm, e1m, aEm, ym, q12, e1h, aEh, yh, R1b[2], qmb, e1mb, Pmb, q12b, e1hb, Phb);
    b3_rev(K, q12, e1h, aEh, yh, qp, e1p, aEp, yp, R2b[2], q12b, e1hb, Phb, qpb, e1pb, Ppb);
    b3_rev(K, qm, e1m, aEm, ym, qp, e1p, aEp, yp, R3b[2], qmb, e1mb, Pmb, qpb, e1pb, Ppb);
    press_fluct_rev(K, Pmb, qmb, e1mb);
    press_fluct_rev(K, Phb, q12b, e1hb);
    press_fluct_rev(K, Ppb, qpb, e1pb);
    // the flux differences: R1 = gh - gm, R2 = gp - gh, R3 = gp - gm
    double gmb[4], ghb[4], gpb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        gmb[k] = -R1b[k] - R3b[k];
        ghb[k] = R1b[k] - R2b[k];
        gpb[k] = R2b[k] + R3b[k];
    }
    flux_g_rev(qm, gmb, qmb);
    flux_g_rev(q12, ghb, q12b);
    flux_g_rev(qp, gpb, qpb);
    velocity_rev(q14, u14b, v14b, q14b);
    velocity_rev(q34, u34b, v34b, q34b);
    velocity_rev(q12, u12b, v12b, q12b);
    e1mb += 0.5 * e1hb;
    e1pb += 0.5 * e1hb;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        qmb[k] += q14b[k] + q12b[k] + q34b[k];
        db[k] += 0.25 * q14b[k] + 0.5 * q12b[k] + 0.75 * q34b[k];
        qpb[k] += db[k];
        qmb[k] -= db[k];
    }
}

// Adjoints of the reconstruction outputs that the step uses (the edge states, the S/N equilibrium
// densities, the cell's flux differences and cell integral).
struct RecBar {
    double qW[4], qE[4], qS[4], qN[4];
    double e1S, e1N;
    double fdiff[4], gdiff[4];
    double vol2, vol3;
};

// Reconstruction (reconstruct) of cell (i, j) from its 3 x 3 stencil wq (row dj - 1, column
// di - 1 relative to the cell; flags wf) and its column's free-surface height y0c: adds the
// adjoints of the stencil states to wqb and returns that of y0c.
BN_DEV double reconstruct_rev(const Consts &K, const double (&wq)[3][3][4], const int (&wf)[3][3], int j, double y0c,
                              double dt, const RecBar &rb, double (&wqb)[3][3][4])
{
    const double *Qc = wq[1][1];
    double Qcb[4] = {0, 0, 0, 0};
    const double yc = K.ylo + (j + 0.5) * K.dy;
    const bool liquid = yc < y0c;
    const double aE = liquid ? K.al : K.ag;
    const double rE0 = liquid ? K.rho0 * exp(-K.a * (yc - y0c)) : K.rho0;
    const double e1c = aE * rE0;
    double e1cb = 0.0, rE0b = 0.0;

    bool so = Qc[3] > K.so_thr;
#pragma unroll
    for (int dj = 0; dj < 3; ++dj)
#pragma unroll
        for (int di = 0; di < 3; ++di)
            if ((wf[dj][di] & F_FLUID) && !(wq[dj][di][3] > K.so_thr)) so = false;

    if (!so) {
        // first order: edge states are the cell average, S/N equilibria the cell's
#pragma unroll
        for (int k = 0; k < 4; ++k) Qcb[k] += rb.qW[k] + rb.qE[k] + rb.qS[k] + rb.qN[k];
        e1cb += rb.e1S + rb.e1N;
    } else {
        const double e1row[3] = {aE * (liquid ? rE0 * K.e_dn1 : K.rho0), e1c,
                                 aE * (liquid ? rE0 * K.e_up1 : K.rho0)};
        const double fc[4] = {Qc[0] - e1c, Qc[1], Qc[2], Qc[3] - aE};
        double phi[3][3][4];
#pragma unroll
        for (int dj = 0; dj < 3; ++dj)
#pragma unroll
            for (int di = 0; di < 3; ++di) {
                const int f = wf[dj][di];
                const bool fluid = f & F_FLUID;
                const bool outx = f & (F_OUTW | F_OUTE), outy = f & (F_OUTS | F_OUTN);
                const bool inside = !outx && !outy;
                const bool fx = (di != 1) && (inside || (outx && !(f & F_TX)));
                const bool fy = (dj != 1) && (inside || (outy && !(f & F_TY)));
                phi[dj][di][0] = fluid ? wq[dj][di][0] - e1row[dj] : fc[0];
                phi[dj][di][1] = fluid ? wq[dj][di][1] : (fx ? -fc[1] : fc[1]);
                phi[dj][di][2] = fluid ? wq[dj][di][2] : (fy ? -fc[2] : fc[2]);
                phi[dj][di][3] = fluid ? wq[dj][di][3] - aE : fc[3];
            }
        // forward: limited gradients
        double gxr[4], gyr[4], psi[4], gx[4], gy[4], lim[4], hm[4];
        int amx[4], amn[4];
        bool lim_hi[4], use_x[4], const1[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            gxr[k] = (phi[1][2][k] - phi[1][0][k]) * K.inv2dx;
            gyr[k] = (phi[2][1][k] - phi[0][1][k]) * K.inv2dy;
            double mx = phi[1][1][k], mn = phi[1][1][k];
            int imx = 4, imn = 4;  // index dj * 3 + di of the selected extreme
#pragma unroll
            for (int dj = 0; dj < 3; ++dj)
#pragma unroll
                for (int di = 0; di < 3; ++di) {
                    const double p = phi[dj][di][k];
                    if (p > mx) { mx = p; imx = dj * 3 + di; }
                    if (p < mn) { mn = p; imn = dj * 3 + di; }
                }
            amx[k] = imx;
            amn[k] = imn;
            const double up = mx - fc[k], dn = fc[k] - mn;
            lim_hi[k] = up <= dn;
            lim[k] = fmin(up, dn);
            const double hx = fabs(gxr[k] * (0.5 * K.dx)), hy = fabs(gyr[k] * (0.5 * K.dy));
            use_x[k] = hx >= hy;  // the difference max(hx, hy) selects
            hm[k] = fmax(hx, hy);
            const double r = fmin(1.0, lim[k] * rcp(hm[k]));
            psi[k] = hm[k] > 0.0 ? r : 1.0;
            const1[k] = !(hm[k] > 0.0) || !(lim[k] * rcp(hm[k]) < 1.0);  // psi is the constant 1
            gx[k] = psi[k] * gxr[k];
            gy[k] = psi[k] * gyr[k];
        }
        const double inv0 = rcp(Qc[0]);
        const double u = Qc[1] * inv0, v = Qc[2] * inv0;
        const double qy0 = gy[0] + aE * (liquid ? -K.a * rE0 : 0.0);
        const double h = -0.5 * dt;
        double hdt[4];
        {
            const double ax0 = gx[1];
            const double ax1 = (K.c2 - u * u) * gx[0] + 2.0 * u * gx[1] - K.k0 * gx[3];
            const double ax2 = -u * v * gx[0] + v * gx[1] + u * gx[2];
            const double ax3 = u * gx[3];
            const double ay0 = gy[2];
            const double ay1 = -u * v * qy0 + v * gy[1] + u * gy[2];
            const double ay2 = (K.c2 - v * v) * qy0 + 2.0 * v * gy[2] - K.k0 * gy[3] + Qc[0] * K.g;
            const double ay3 = v * gy[3];
            hdt[0] = h * (ax0 + ay0);
            hdt[1] = h * (ax1 + ay1);
            hdt[2] = h * (ax2 + ay2);
            hdt[3] = h * (ax3 + ay3);
        }
        const double e1S = aE * (liquid ? rE0 * K.e_dnh : K.rho0);
        const double e1N = aE * (liquid ? rE0 * K.e_uph : K.rho0);
        const double ex[4] = {e1c, 0.0, 0.0, aE}, eS[4] = {e1S, 0.0, 0.0, aE}, eN[4] = {e1N, 0.0, 0.0, aE};
        const double hxx = 0.5 * K.dx, hyy = 0.5 * K.dy;
        double qW[4], qE[4], qS[4], qN[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            qW[k] = (ex[k] + fc[k]) + gx[k] * (-hxx) + hdt[k];
            qE[k] = (ex[k] + fc[k]) + gx[k] * hxx + hdt[k];
            qS[k] = (eS[k] + fc[k]) + gy[k] * (-hyy) + hdt[k];
            qN[k] = (eN[k] + fc[k]) + gy[k] * hyy + hdt[k];
        }
        const double qc0 = Qc[0] + hdt[0];
        const double ic = rcp(qc0);
        const double uc = (Qc[1] + hdt[1]) * ic, vc = (Qc[2] + hdt[2]) * ic;

        // ---- reverse ----
        double gxb[4] = {0, 0, 0, 0}, gyb[4] = {0, 0, 0, 0}, hdtb[4] = {0, 0, 0, 0}, fcb[4] = {0, 0, 0, 0};
        double qWb[4], qEb[4], qSb[4], qNb[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            qWb[k] = rb.qW[k];
            qEb[k] = rb.qE[k];
            qSb[k] = rb.qS[k];
            qNb[k] = rb.qN[k];
        }
        // cell integral: vol3 = uc gx3 + vc gy3, vol2 = k0 (gy0/rho0 - gy3) + (qc0 - e1c) g
        {
            const double ucb = rb.vol3 * gx[3], vcb = rb.vol3 * gy[3];
            gxb[3] += rb.vol3 * uc;
            gyb[3] += rb.vol3 * vc;
            double qc0b = -(uc * ucb + vc * vcb) * ic;
            Qcb[1] += ucb * ic;
            hdtb[1] += ucb * ic;
            Qcb[2] += vcb * ic;
            hdtb[2] += vcb * ic;
            gyb[0] += rb.vol2 * K.k0 * K.inv_rho0;
            gyb[3] -= rb.vol2 * K.k0;
            qc0b += rb.vol2 * K.g;
            e1cb -= rb.vol2 * K.g;
            Qcb[0] += qc0b;
            hdtb[0] += qc0b;
        }
        // the cell's flux differences
        {
            const double nf[4] = {-rb.fdiff[0], -rb.fdiff[1], -rb.fdiff[2], -rb.fdiff[3]};
            const double ng[4] = {-rb.gdiff[0], -rb.gdiff[1], -rb.gdiff[2], -rb.gdiff[3]};
            flux_f_rev(K, qE, rb.fdiff, qEb);
            flux_f_rev(K, qW, nf, qWb);
            flux_g_rev(qN, rb.gdiff, qNb);
            flux_g_rev(qS, ng, qSb);
        }
        // the edge states
        double e1Sb = rb.e1S, e1Nb = rb.e1N;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double Ab = qWb[k] + qEb[k];
            gxb[k] += (qEb[k] - qWb[k]) * hxx;
            gyb[k] += (qNb[k] - qSb[k]) * hyy;
            hdtb[k] += qWb[k] + qEb[k] + qSb[k] + qNb[k];
            fcb[k] += Ab + qSb[k] + qNb[k];
            if (k == 0) {
                e1cb += Ab;
                e1Sb += qSb[0];
                e1Nb += qNb[0];
            }
        }
        if (liquid) rE0b += aE * (K.e_dnh * e1Sb + K.e_uph * e1Nb);
        // predictor
        {
            double ub = 0.0, vb = 0.0, qy0b = 0.0;
            const double axb = h * hdtb[0], a1 = h * hdtb[1], a2 = h * hdtb[2], a3 = h * hdtb[3];
            // x part
            gxb[1] += axb;
            gxb[0] += (K.c2 - u * u) * a1 - u * v * a2;
            gxb[1] += 2.0 * u * a1 + v * a2;
            gxb[2] += u * a2;
            gxb[3] += -K.k0 * a1 + u * a3;
            ub += (2.0 * gx[1] - 2.0 * u * gx[0]) * a1 + (gx[2] - v * gx[0]) * a2 + gx[3] * a3;
            vb += (gx[1] - u * gx[0]) * a2;
            // y part
            gyb[2] += axb;
            qy0b += -u * v * a1 + (K.c2 - v * v) * a2;
            gyb[1] += v * a1;
            gyb[2] += u * a1 + 2.0 * v * a2;
            gyb[3] += -K.k0 * a2 + v * a3;
            Qcb[0] += K.g * a2;
            ub += (gy[2] - v * qy0) * a1;
            vb += (gy[1] - u * qy0) * a1 + (2.0 * gy[2] - 2.0 * v * qy0) * a2 + gy[3] * a3;
            gyb[0] += qy0b;
            if (liquid) rE0b -= aE * K.a * qy0b;
            velocity_rev(Qc, ub, vb, Qcb);
        }
        // limiter: gx = psi gxr, gy = psi gyr
        double phib[3][3][4];
#pragma unroll
        for (int dj = 0; dj < 3; ++dj)
#pragma unroll
            for (int di = 0; di < 3; ++di)
#pragma unroll
                for (int k = 0; k < 4; ++k) phib[dj][di][k] = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double gxrb = psi[k] * gxb[k], gyrb = psi[k] * gyb[k];
            const double psib = gxr[k] * gxb[k] + gyr[k] * gyb[k];
            double limb = 0.0;
            // psi = min(1, lim / max(hx, hy)) unless that is the constant 1
            if (!const1[k]) {
                const double ih = rcp(hm[k]);
                limb += psib * ih;
                const double hmb = -psib * lim[k] * ih * ih;
                if (use_x[k]) gxrb += hmb * sgn(gxr[k]) * (0.5 * K.dx);
                else gyrb += hmb * sgn(gyr[k]) * (0.5 * K.dy);
            }
            // lim = min(max - fc, fc - min): to the selected extreme (a select per stencil entry, so
            // that phib stays in registers)
            const int ext = lim_hi[k] ? amx[k] : amn[k];
            const double eb = lim_hi[k] ? limb : -limb;
            fcb[k] -= eb;
#pragma unroll
            for (int dj = 0; dj < 3; ++dj)
#pragma unroll
                for (int di = 0; di < 3; ++di) phib[dj][di][k] += ext == dj * 3 + di ? eb : 0.0;
            phib[1][2][k] += gxrb * K.inv2dx;
            phib[1][0][k] -= gxrb * K.inv2dx;
            phib[2][1][k] += gyrb * K.inv2dy;
            phib[0][1][k] -= gyrb * K.inv2dy;
        }
        // fluctuations of the stencil
        double e1rowb[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int dj = 0; dj < 3; ++dj)
#pragma unroll
            for (int di = 0; di < 3; ++di) {
                const int f = wf[dj][di];
                const bool fluid = f & F_FLUID;
                const bool outx = f & (F_OUTW | F_OUTE), outy = f & (F_OUTS | F_OUTN);
                const bool inside = !outx && !outy;
                const bool fx = (di != 1) && (inside || (outx && !(f & F_TX)));
                const bool fy = (dj != 1) && (inside || (outy && !(f & F_TY)));
                if (fluid) {
                    wqb[dj][di][0] += phib[dj][di][0];
                    e1rowb[dj] -= phib[dj][di][0];
                    wqb[dj][di][1] += phib[dj][di][1];
                    wqb[dj][di][2] += phib[dj][di][2];
                    wqb[dj][di][3] += phib[dj][di][3];
                } else {
                    fcb[0] += phib[dj][di][0];
                    fcb[1] += fx ? -phib[dj][di][1] : phib[dj][di][1];
                    fcb[2] += fy ? -phib[dj][di][2] : phib[dj][di][2];
                    fcb[3] += phib[dj][di][3];
                }
            }
        e1cb += e1rowb[1];
        if (liquid) rE0b += aE * (K.e_dn1 * e1rowb[0] + K.e_up1 * e1rowb[2]);
        // fc = (Qc0 - e1c, Qc1, Qc2, Qc3 - alpha^E)
        Qcb[0] += fcb[0];
        e1cb -= fcb[0];
        Qcb[1] += fcb[1];
        Qcb[2] += fcb[2];
        Qcb[3] += fcb[3];
    }
    // e1c = alpha^E rho^E(y_c); rho^E = rho0 exp(-a (y_c - y0c)) in the liquid
    rE0b += aE * e1cb;
#pragma unroll
    for (int k = 0; k < 4; ++k) wqb[1][1][k] += Qcb[k];
    return liquid ? K.a * rE0 * rE0b : 0.0;
}

}  // namespace bn
