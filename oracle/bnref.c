/*
 * bnref.c -- CPU oracle for one explicit time step of the second-order, well-balanced,
 * path-conservative Osher / Osher-Romberg finite-volume scheme for the reduced
 * three-equation Baer-Nunziato model (Gaburro, Castro, Dumbser, arXiv:1806.04960).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no source, header, table
 * or helper with the HIP library: it is written from the paper alone, plainly and slowly,
 * in FP64, in the paper's order and notation, so that a reader can check it by eye.
 *
 * Build:  gcc -O2 -std=c99 -ffp-contract=off -fno-fast-math -fopenmp -fPIC -shared -o libbnref.so bnref.c -lm
 * (-fopenmp shares the rows of each sweep of a step out over threads: every cell is still
 * computed by the same arithmetic, so results do not depend on the thread count; without it
 * the same source builds a single-threaded oracle.)
 *
 * Where the paper is silent, ambiguous or garbled the oracle takes one reading; each reading
 * is tagged [Rn] where it is used and listed below with its justification.
 *
 *  [R1]  The cell integral of the scheme is taken of the full system matrix A = dF/dQ + B
 *        (Sec. 3, eq. "Scheme" together with the path-conservative form it cites): the cell's
 *        own flux difference f(q_E)-f(q_W), g(q_N)-g(q_S) is added to the B-part.
 *  [R2]  That integral is (1/|T|) * int_t int_T ... and is evaluated by the midpoint rule at
 *        the barycentre and t^{n+1/2} (Sec. 3.4), i.e. dt * B(q_c) grad q.
 *  [R3]  The pressure part of the y non-conservative term b_3 (Sec. 3.3) is the integral of a
 *        total s-derivative, d/ds(alpha p); with the equilibrium part removed this is
 *        Delta(aE pf) + Delta(af pE) + Delta(af pf).  The gravity part is as printed, with
 *        arithmetic means of the end states.
 *  [R4]  The cell integral of b_3 (Sec. 3.4) reads its "Delta" as the y-gradient of the
 *        reconstruction: d/dy(alpha p)^f + g (alpha rho)^f, midpoint rule.
 *  [R5]  The Hancock predictor is d_t Q = -(A1 d_x Q + A2 d_y Q) (the minus sign of the
 *        quasi-linear form, Sec. 1).
 *  [R6]  Free-surface detector (Sec. 3.5): y0_i = y_L(i) + dy * sum_j (alpha_ij - a_g)/(a_l - a_g)
 *        over the fluid cells of column i, summed in ascending j; y_L(i) is the top of the
 *        solid run attached to the bottom of the column.  It is exact for two-level alpha.
 *  [R7]  Equilibrium state of a cell: liquid (alpha_l, exponential density of Sec. 2.1 with
 *        gamma = 1) if its centre lies below y0 of its column, else gas (alpha_g, rho0); zero
 *        velocity.  Its "cell average" is its value at the cell centre (allowed by Sec. 3.3).
 *  [R8]  gamma = 1 throughout (as in every test of Sec. 5): p = k0 (rho/rho0 - 1), c^2 = k0/rho0.
 *  [R10] Time step: dt = CFL / max over fluid cells of ((|u|+c)/dx + (|v|+c)/dy) (the paper
 *        states no formula).
 *  [R11] MUSCL gradients are central differences of the fluctuations; the Barth-Jespersen
 *        limiter takes min/max over the 3x3 stencil (centre included) and is evaluated at
 *        the four edge midpoints, one limiter per conserved component.
 *  [R12] The fluctuations of the stencil are taken with respect to the centre cell's
 *        equilibrium profile evaluated at each neighbour's centre (Sec. 3.4, the stationary
 *        solution of the cell computed for its neighbours).
 *  [R13] A solid or out-of-domain stencil neighbour takes the centre's fluctuation, with
 *        the momentum component normal to each separating reflective wall negated.
 *  [R14] Second order iff alpha > 10 * alpha_gas (strict, Sec. 3.4) in the cell and in every
 *        fluid cell of its 3x3 stencil, so that the reconstruction never extrapolates across a
 *        liquid/gas interface; otherwise the face states are the cell average at the
 *        cell-centre height and there is no predictor and no cell integral.
 *  [R15] The path is the segment in conserved variables, its equilibrium part the segment
 *        between the two equilibrium parts; the equilibrium part of b_3 is dropped.
 *  [R16] Heights: x-face states sit at the cell-centre height; y-face states of a
 *        second-order cell at the edge height (computed from the edge index), of a
 *        first-order cell at the centre height.
 *  [R17] sign(0) = 0.
 *  [R18] The velocity of the alpha-advection term b_4 is the path integral of u (v) along the
 *        segment path taken with the viscosity's own nodes: the 3-point Gauss-Legendre mean in x,
 *        the midpoint rule on each Romberg sub-interval in y.  This replaces the printed Roe
 *        average, which is not additive over the Romberg sub-intervals and differs from the
 *        node velocities: the resulting non-upwind alpha flux drains the gas volume fraction.
 *  [R19] Reflective wall: the ghost state is the interior edge state with its normal
 *        momentum negated (E-part and height copied); transmissive: a copy.  Solid cells
 *        are never updated.
 *  [R21] A column's bottom y_L (the top of an obstacle, Sec. 3.5 and 5.7) may be given off the
 *        grid, within half a cell of the top of its whole-cell solid run: the detector then
 *        integrates alpha from y_L, the first fluid cell standing for the interval from y_L to
 *        its top edge.  The cells themselves stay whole (solid iff the centre lies below the
 *        obstacle's top).  Without given bottoms y_L is the top of the solid run.
 *
 * Literal forms (off by default; the test-suite builds them separately to show why [R12], [R14]
 * and [R18] depart from the printed text):
 *   -DBNREF_LITERAL_ROE_VELOCITY   b_4 velocity = the printed Roe average of u (v) with sqrt(rho)
 *                                  weights between the end states of each (sub-)interval
 *                                  (Sec. 3.2 and 3.3), instead of [R18];
 *   -DBNREF_LITERAL_CELL_SWITCH    second order iff the cell's own alpha > 10 alpha_gas (Sec. 3.4),
 *                                  instead of [R14];
 *   -DBNREF_LITERAL_OWN_EQUILIBRIUM  each stencil neighbour's fluctuation taken against its own
 *                                  equilibrium (its column's free surface), instead of [R12].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef BNREF_REAL_DEFINED
typedef double real;
#define TO_DOUBLE(x) (x)
#endif

#define NV 5 /* (alpha rho, alpha rho u, alpha rho v, alpha, y) -- Sec. 2.1 */
#define BNREF_PARALLEL_CELLS 65536 /* smaller grids run their sweeps on one thread */

typedef struct { int32_t nx, ny; double x0, x1, y0, y1; } bnref_grid;
typedef struct {
    double g, k0, rho0, alpha_liq, alpha_gas, cfl;
    int32_t bc[4]; /* W, E, S, N: 0 reflective wall, 1 transmissive */
} bnref_params;

enum { BNREF_OK = 0, BNREF_EINVAL = -1, BNREF_ENONPHYS = -3, BNREF_EUNSUPPORTED = -4 };
enum { W = 0, E = 1, S = 2, N = 3 };

typedef struct {
    int nx, ny;
    real dx, dy, ylo;
    real g, k0, rho0, al, ag;
    int bc[4];
    const uint8_t *solid;
    const double *ybot; /* bottom height y_L of each column [R21], or NULL */
} model_t;

/* ------------------------------------------------------------------------------------ */
/* Physical model, Sec. 2                                                               */
/* ------------------------------------------------------------------------------------ */

/* Tait equation of state with gamma = 1 [R8] (Sec. 2, Tait law). */
static real eos_p(const model_t *m, real rho) { return m->k0 * (rho / m->rho0 - 1.0); }
/* Sound speed squared, gamma k0/rho0 (rho/rho0)^(gamma-1) at gamma = 1 (Sec. 3). */
static real eos_c2(const model_t *m) { return m->k0 / m->rho0; }

#ifdef BNREF_LITERAL_ROE_VELOCITY
/* Roe average of velocity component k (1: u, 2: v) between states a and b, weights sqrt(rho),
 * rho = alpha rho / alpha (Sec. 3.2, 3.3 as printed). */
static real roe_velocity(const real a[NV], const real b[NV], int k)
{
    real sa = sqrt(a[0] / a[3]), sb = sqrt(b[0] / b[3]);
    return (sa * (a[k] / a[0]) + sb * (b[k] / b[0])) / (sa + sb);
}
#endif

/* Conservative fluxes f and g of the augmented system (Sec. 2.1, general form).
 * The y-flux carries no pressure: d_y(alpha p) is a non-conservative term of B2. */
static void flux_f(const model_t *m, const real q[NV], real f[NV])
{
    real rho = q[0] / q[3], u = q[1] / q[0], v = q[2] / q[0];
    real alpha_p = q[3] * eos_p(m, rho);
    f[0] = q[1];
    f[1] = q[1] * u + alpha_p;
    f[2] = q[1] * v;
    f[3] = 0.0;
    f[4] = 0.0;
}

static void flux_g(const model_t *m, const real q[NV], real g[NV])
{
    real u = q[1] / q[0], v = q[2] / q[0];
    (void)m;
    g[0] = q[2];
    g[1] = q[2] * u;
    g[2] = q[2] * v;
    g[3] = 0.0;
    g[4] = 0.0;
}

/* System matrices A1 = df/dQ + B1, A2 = dg/dQ + B2 as printed in Sec. 3. */
static void matrix_A(const model_t *m, int dir, const real q[NV], real A[NV][NV])
{
    real rho = q[0] / q[3], u = q[1] / q[0], v = q[2] / q[0];
    real p = eos_p(m, rho), c2 = eos_c2(m);
    int a, b;
    for (a = 0; a < NV; ++a)
        for (b = 0; b < NV; ++b) A[a][b] = 0.0;
    if (dir == 0) {
        A[0][1] = 1.0;
        A[1][0] = c2 - u * u; A[1][1] = 2.0 * u; A[1][3] = p - rho * c2;
        A[2][0] = -u * v;     A[2][1] = v;       A[2][2] = u;
        A[3][3] = u;
    } else {
        A[0][2] = 1.0;
        A[1][0] = -u * v;     A[1][1] = v;       A[1][2] = u;
        A[2][0] = c2 - v * v; A[2][2] = 2.0 * v; A[2][3] = p - rho * c2; A[2][4] = q[0] * m->g;
        A[3][3] = v;
    }
}

/* Right eigenvectors R, eigenvalues lam and R^{-1} of A1 (dir 0) or A2 (dir 1), Sec. 3. */
static void eigen(const model_t *m, int dir, const real q[NV], real R[NV][NV], real lam[NV],
                  real L[NV][NV])
{
    real rho = q[0] / q[3], u = q[1] / q[0], v = q[2] / q[0];
    real p = eos_p(m, rho), c2 = eos_c2(m), c = sqrt(c2);
    real K = rho * c2 - p;   /* rho c^2 - p */
    real arg = q[0] * m->g;  /* alpha rho g */
    int a, b;
    for (a = 0; a < NV; ++a)
        for (b = 0; b < NV; ++b) { R[a][b] = 0.0; L[a][b] = 0.0; }
    if (dir == 0) {
        R[0][0] = 1.0;   R[0][2] = K;     R[0][4] = 1.0;
        R[1][0] = u - c; R[1][2] = u * K; R[1][4] = u + c;
        R[2][0] = v;     R[2][1] = 1.0;   R[2][4] = v;
        R[3][2] = c2;
        R[4][3] = 1.0;
        lam[0] = u - c; lam[1] = u; lam[2] = u; lam[3] = 0.0; lam[4] = u + c;
        L[0][0] = 0.5 * (c + u) / c; L[0][1] = -0.5 / c; L[0][3] = -0.5 * K / c2;
        L[1][0] = -v;                L[1][2] = 1.0;      L[1][3] = v * K / c2;
        L[2][3] = 1.0 / c2;
        L[3][4] = 1.0;
        L[4][0] = 0.5 * (c - u) / c; L[4][1] = 0.5 / c;  L[4][3] = -0.5 * K / c2;
    } else {
        R[0][0] = 1.0;   R[0][2] = K;     R[0][3] = arg;     R[0][4] = 1.0;
        R[1][0] = u;     R[1][1] = 1.0;   R[1][3] = u * arg; R[1][4] = u;
        R[2][0] = v - c; R[2][2] = v * K; R[2][4] = v + c;
        R[3][2] = c2;
        R[4][3] = v * v - c2;
        lam[0] = v - c; lam[1] = v; lam[2] = v; lam[3] = 0.0; lam[4] = v + c;
        L[0][0] = 0.5 * (c + v) / c; L[0][2] = -0.5 / c; L[0][3] = -0.5 * K / c2;
        L[0][4] = 0.5 / c * arg / (c - v);
        L[1][0] = -u; L[1][1] = 1.0; L[1][3] = u * K / c2;
        L[2][3] = 1.0 / c2;
        L[3][4] = 1.0 / (v * v - c2);
        L[4][0] = 0.5 * (c - v) / c; L[4][2] = 0.5 / c;  L[4][3] = -0.5 * K / c2;
        L[4][4] = 0.5 / c * arg / (c + v);
    }
}

/* M = R diag(h) R^{-1} with h = |lam| (kind 0) or sign(lam) (kind 1), sign(0) = 0 [R17]
 * (Sec. 3.1: |A| = R |Lambda| R^{-1}, sign(A) = R sign(Lambda) R^{-1}). */
static void matrix_function(const model_t *m, int dir, int kind, const real q[NV], real M[NV][NV])
{
    real R[NV][NV], L[NV][NV], lam[NV], h[NV];
    int a, b, k;
    eigen(m, dir, q, R, lam, L);
    for (k = 0; k < NV; ++k) {
        if (kind == 0) h[k] = fabs(lam[k]);
        else h[k] = (lam[k] > 0.0) ? 1.0 : ((lam[k] < 0.0) ? -1.0 : 0.0);
    }
    for (a = 0; a < NV; ++a)
        for (b = 0; b < NV; ++b) {
            real s = 0.0;
            for (k = 0; k < NV; ++k) s += R[a][k] * h[k] * L[k][b];
            M[a][b] = s;
        }
}

/* ------------------------------------------------------------------------------------ */
/* First-order fluctuations, Sec. 3.2 (x) and Sec. 3.3 (y)                              */
/* ------------------------------------------------------------------------------------ */

/* x-direction: D^{+-} = 1/2 [ f(q+) - f(q-) + B~ dq +- V dq ] (Sec. 3, fluctuation form),
 * with b_4^x = ubar * dalpha and the Osher viscosity, both integrated along the segment path
 * by 3-point Gauss-Legendre (Sec. 3.2); ubar is the Gauss-Legendre mean of u on the path [R18]. */
static void fluct_x(const model_t *m, const real qm[NV], const real qp[NV], real Dm[NV], real Dp[NV])
{
    static const double s_gl[3] = {0.5 - 0.3872983346207416885, 0.5, 0.5 + 0.3872983346207416885};
    static const double w_gl[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    real dq[NV], fm[NV], fp[NV], Bdq[NV], V[NV][NV], Vdq[NV];
    real ubar;
    int a, b, k;

    for (k = 0; k < NV; ++k) dq[k] = qp[k] - qm[k];
    flux_f(m, qm, fm);
    flux_f(m, qp, fp);

    for (a = 0; a < NV; ++a)
        for (b = 0; b < NV; ++b) V[a][b] = 0.0;
    ubar = 0.0;
    for (k = 0; k < 3; ++k) {
        real phi[NV], Ak[NV][NV];
        for (a = 0; a < NV; ++a) phi[a] = qm[a] + s_gl[k] * dq[a];
        matrix_function(m, 0, 0, phi, Ak);
        for (a = 0; a < NV; ++a)
            for (b = 0; b < NV; ++b) V[a][b] += w_gl[k] * Ak[a][b];
        ubar += w_gl[k] * (phi[1] / phi[0]);
    }
#ifdef BNREF_LITERAL_ROE_VELOCITY
    ubar = roe_velocity(qm, qp, 1);
#endif
    for (k = 0; k < NV; ++k) Bdq[k] = 0.0;
    Bdq[3] = ubar * dq[3];
    for (a = 0; a < NV; ++a) {
        real s = 0.0;
        for (b = 0; b < NV; ++b) s += V[a][b] * dq[b];
        Vdq[a] = s;
    }
    for (k = 0; k < NV; ++k) {
        Dm[k] = 0.5 * (fp[k] - fm[k] + Bdq[k] - Vdq[k]);
        Dp[k] = 0.5 * (fp[k] - fm[k] + Bdq[k] + Vdq[k]);
    }
}

/* Well-balanced b_3^y between path states a and b with equilibrium parts ea, eb
 * (Sec. 3.3, midpoint-rule formula) [R3][R15].  Heights are the 5th components. */
static real b3_y(const model_t *m, const real a[NV], const real ea[NV], const real b[NV], const real eb[NV])
{
    real al_a = a[3], rho_a = a[0] / a[3], p_a = eos_p(m, rho_a);
    real al_b = b[3], rho_b = b[0] / b[3], p_b = eos_p(m, rho_b);
    real alE_a = ea[3], rhoE_a = ea[0] / ea[3], pE_a = eos_p(m, rhoE_a);
    real alE_b = eb[3], rhoE_b = eb[0] / eb[3], pE_b = eos_p(m, rhoE_b);
    real alF_a = al_a - alE_a, pF_a = p_a - pE_a, rhoF_a = rho_a - rhoE_a;
    real alF_b = al_b - alE_b, pF_b = p_b - pE_b, rhoF_b = rho_b - rhoE_b;

    real pressure = (alE_b * pF_b - alE_a * pF_a)
                  + (alF_b * pE_b - alF_a * pE_a)
                  + (alF_b * pF_b - alF_a * pF_a);

    real alE_bar = 0.5 * (alE_a + alE_b), alF_bar = 0.5 * (alF_a + alF_b);
    real rhoE_bar = 0.5 * (rhoE_a + rhoE_b), rhoF_bar = 0.5 * (rhoF_a + rhoF_b);
    real gravity = (alE_bar * rhoF_bar + alF_bar * rhoE_bar + alF_bar * rhoF_bar) * m->g * (b[4] - a[4]);
    return pressure + gravity;
}

/* Residual g(b) - g(a) + B~(b - a) on one sub-interval of the path (Sec. 3.3):
 * B~ = (0, 0, b_3^y, vbar dalpha, 0), vbar the path velocity of the sub-interval [R18]. */
static void residual_y(const model_t *m, const real a[NV], const real ea[NV], const real b[NV],
                       const real eb[NV], real vbar, real Rs[NV])
{
    real ga[NV], gb[NV];
    int k;
    flux_g(m, a, ga);
    flux_g(m, b, gb);
    for (k = 0; k < NV; ++k) Rs[k] = gb[k] - ga[k];
    Rs[2] += b3_y(m, a, ea, b, eb);
    Rs[3] += vbar * (b[3] - a[3]);
}

/* y-direction: D^{+-} = 1/2 [ R(q-, q+) +- V ] with the well-balanced Osher-Romberg
 * viscosity, Romberg l = 3 (Sec. 3.1 weights, Sec. 3.3 final viscosity):
 *   V = 4/3 sign(A2(Phi(1/4))) R(0,1/2) + 4/3 sign(A2(Phi(3/4))) R(1/2,1)
 *       - 1/3 sign(A2(Phi(1/2))) R(0,1).
 * The velocity of b_4^y on [0,1/2] and [1/2,1] is v at Phi(1/4) and Phi(3/4) (midpoint rule on
 * each sub-interval), on [0,1] their mean (the composite rule), so the three residuals add up [R18]. */
static void fluct_y(const model_t *m, const real qm[NV], const real em[NV], const real qp[NV],
                    const real ep[NV], real Dm[NV], real Dp[NV])
{
    real dq[NV], q14[NV], q12[NV], q34[NV], e12[NV];
    real R1[NV], R2[NV], R3[NV], S1[NV][NV], S2[NV][NV], S3[NV][NV], V[NV];
    real v14, v34;
    int a, b;

    for (a = 0; a < NV; ++a) {
        dq[a] = qp[a] - qm[a];
        q14[a] = qm[a] + 0.25 * dq[a];
        q12[a] = qm[a] + 0.5 * dq[a];
        q34[a] = qm[a] + 0.75 * dq[a];
        e12[a] = em[a] + 0.5 * (ep[a] - em[a]);
    }
    v14 = q14[2] / q14[0];
    v34 = q34[2] / q34[0];
#ifdef BNREF_LITERAL_ROE_VELOCITY
    residual_y(m, qm, em, q12, e12, roe_velocity(qm, q12, 2), R1);
    residual_y(m, q12, e12, qp, ep, roe_velocity(q12, qp, 2), R2);
    residual_y(m, qm, em, qp, ep, roe_velocity(qm, qp, 2), R3);
#else
    residual_y(m, qm, em, q12, e12, v14, R1);
    residual_y(m, q12, e12, qp, ep, v34, R2);
    residual_y(m, qm, em, qp, ep, 0.5 * (v14 + v34), R3);
#endif
    matrix_function(m, 1, 1, q14, S1);
    matrix_function(m, 1, 1, q34, S2);
    matrix_function(m, 1, 1, q12, S3);
    for (a = 0; a < NV; ++a) {
        real s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (b = 0; b < NV; ++b) {
            s1 += S1[a][b] * R1[b];
            s2 += S2[a][b] * R2[b];
            s3 += S3[a][b] * R3[b];
        }
        V[a] = (4.0 / 3.0) * s1 + (4.0 / 3.0) * s2 - (1.0 / 3.0) * s3;
    }
    for (a = 0; a < NV; ++a) {
        Dm[a] = 0.5 * (R3[a] - V[a]);
        Dp[a] = 0.5 * (R3[a] + V[a]);
    }
}

/* ------------------------------------------------------------------------------------ */
/* Equilibrium profile and free-surface detector, Sec. 2.1 and Sec. 3.5                 */
/* ------------------------------------------------------------------------------------ */

static int is_fluid(const model_t *m, int i, int j)
{
    if (i < 0 || i >= m->nx || j < 0 || j >= m->ny) return 0;
    return m->solid ? (m->solid[(size_t)j * m->nx + i] == 0) : 1;
}

static real y_centre(const model_t *m, int j) { return m->ylo + (j + 0.5) * m->dy; }
static real y_edge(const model_t *m, int j) { return m->ylo + j * m->dy; } /* bottom edge of row j */

/* Water-at-rest state of a column with free surface Y0 evaluated at height y [R7]:
 * rho(y) = rho0 exp(-g rho0 / k0 (y - Y0)) in the liquid (Sec. 2.1, gamma = 1). */
static void estate(const model_t *m, int liquid, real Y0, real y, real e[NV])
{
    real alpha = liquid ? m->al : m->ag;
    real rho = liquid ? m->rho0 * exp(-(m->g * m->rho0 / m->k0) * (y - Y0)) : m->rho0;
    e[0] = alpha * rho;
    e[1] = 0.0;
    e[2] = 0.0;
    e[3] = alpha;
    e[4] = y;
}

/* Free-surface detector [R6] (Sec. 3.5): y0 = y_L + the integral of the normalised volume fraction
 * from the column's bottom y_L upwards.  [R21] y_L may lie inside the first fluid cell (a cut cell)
 * or inside the solid cell below it: the first fluid cell's value then stands for the whole fluid
 * interval from y_L to its top edge.  Written as the grid-aligned sum plus the correction of the
 * bottom's offset d = y_L - (top of the solid run), weighted by the part of the first cell that is
 * not liquid: d (1 - a_first).  A column whose first cell is full (a_first = 1) thus gets bitwise the
 * grid-aligned value, so water at rest over a wall stays exactly at rest; an empty one gets y_L. */
static int detector(const model_t *m, const double *Q, real *Y0)
{
    size_t plane = (size_t)m->nx * m->ny;
    int i, j;
    for (i = 0; i < m->nx; ++i) {
        int jb = 0;
        real sum = 0.0, first = 0.0, base;
        while (jb < m->ny && !is_fluid(m, i, jb)) ++jb;
        for (j = jb; j < m->ny; ++j) {
            real a;
            if (!is_fluid(m, i, j)) return BNREF_EUNSUPPORTED; /* solid above fluid */
            a = (Q[3 * plane + (size_t)j * m->nx + i] - m->ag) / (m->al - m->ag);
            if (j == jb) first = a;
            sum += a;
        }
        base = m->ylo + jb * m->dy;
        Y0[i] = base + m->dy * sum;
        if (m->ybot) Y0[i] += (m->ybot[i] - base) * (1.0 - first);
    }
    return BNREF_OK;
}

static void load_q(const model_t *m, const double *Q, int i, int j, real q[NV])
{
    size_t plane = (size_t)m->nx * m->ny, c = (size_t)j * m->nx + i;
    int k;
    for (k = 0; k < 4; ++k) q[k] = Q[k * plane + c];
    q[4] = y_centre(m, j);
}

/* ------------------------------------------------------------------------------------ */
/* Second-order well-balanced reconstruction with Hancock predictor, Sec. 3.4           */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    int so;           /* second-order cell [R14] */
    real q[4][NV];    /* edge-midpoint states at t^{n+1/2}: W, E, S, N */
    real e[4][NV];    /* their equilibrium parts */
    real qc[NV];      /* barycentre state at t^{n+1/2} */
    real ec[NV];      /* equilibrium state at the barycentre */
    real gx[4], gy[4];/* limited gradients Psi grad Q^f */
} recon_t;

/* Barth-Jespersen ratio for one evaluation point with unlimited increment d [R11]. */
static real bj_ratio(real d, real qmax, real qmin, real qc)
{
    if (d > 0.0) return fmin(1.0, (qmax - qc) / d);
    if (d < 0.0) return fmin(1.0, (qmin - qc) / d);
    return 1.0;
}

static void reconstruct(const model_t *m, const double *Q, const real *Y0, int i, int j, real dt, recon_t *r)
{
    real Qc[NV], fc[4], phi[3][3][4];
    real yc = y_centre(m, j);
    real yf[4], dxf[4], dyf[4];
    int liquid = yc < Y0[i];
    int di, dj, k, f;

    load_q(m, Q, i, j, Qc);
    estate(m, liquid, Y0[i], yc, r->ec);
    /* second order only where the cell and every fluid cell of its 3x3 stencil hold liquid [R14] */
    r->so = Qc[3] > 10.0 * m->ag;
#ifndef BNREF_LITERAL_CELL_SWITCH
    for (dj = -1; dj <= 1; ++dj)
        for (di = -1; di <= 1; ++di)
            if (is_fluid(m, i + di, j + dj) && !(Q[3 * (size_t)m->nx * m->ny + (size_t)(j + dj) * m->nx + i + di] > 10.0 * m->ag))
                r->so = 0;
#endif

    yf[W] = yc; yf[E] = yc;
    if (r->so) { yf[S] = y_edge(m, j); yf[N] = y_edge(m, j + 1); }
    else { yf[S] = yc; yf[N] = yc; }

    if (!r->so) {
        for (f = 0; f < 4; ++f)
            for (k = 0; k < NV; ++k) { r->q[f][k] = Qc[k]; r->e[f][k] = r->ec[k]; }
        for (k = 0; k < NV; ++k) r->qc[k] = Qc[k];
        for (k = 0; k < 4; ++k) { r->gx[k] = 0.0; r->gy[k] = 0.0; }
        return;
    }

    for (k = 0; k < 4; ++k) fc[k] = Qc[k] - r->ec[k];

    /* 3x3 stencil of fluctuations with respect to this cell's equilibrium profile [R12][R13]. */
    for (dj = -1; dj <= 1; ++dj)
        for (di = -1; di <= 1; ++di) {
            int ii = i + di, jj = j + dj;
            if (is_fluid(m, ii, jj)) {
                real qn[NV], en[NV];
                load_q(m, Q, ii, jj, qn);
#ifdef BNREF_LITERAL_OWN_EQUILIBRIUM
                estate(m, qn[4] < Y0[ii], Y0[ii], qn[4], en);
#else
                estate(m, liquid, Y0[i], qn[4], en);
#endif
                for (k = 0; k < 4; ++k) phi[dj + 1][di + 1][k] = qn[k] - en[k];
            } else {
                int out_x = (ii < 0 || ii >= m->nx), out_y = (jj < 0 || jj >= m->ny);
                int inside = !out_x && !out_y;
                int flip_x = di != 0 && (inside || (out_x && m->bc[ii < 0 ? W : E] == 0));
                int flip_y = dj != 0 && (inside || (out_y && m->bc[jj < 0 ? S : N] == 0));
                phi[dj + 1][di + 1][0] = fc[0];
                phi[dj + 1][di + 1][1] = flip_x ? -fc[1] : fc[1];
                phi[dj + 1][di + 1][2] = flip_y ? -fc[2] : fc[2];
                phi[dj + 1][di + 1][3] = fc[3];
            }
        }

    /* MUSCL central gradients + Barth-Jespersen limiter, component by component [R11]. */
    for (k = 0; k < 4; ++k) {
        real gx = (phi[1][2][k] - phi[1][0][k]) / (2.0 * m->dx);
        real gy = (phi[2][1][k] - phi[0][1][k]) / (2.0 * m->dy);
        real qmax = phi[1][1][k], qmin = phi[1][1][k], psi = 1.0;
        real d[4];
        for (dj = 0; dj < 3; ++dj)
            for (di = 0; di < 3; ++di) {
                qmax = fmax(qmax, phi[dj][di][k]);
                qmin = fmin(qmin, phi[dj][di][k]);
            }
        d[W] = gx * (-0.5 * m->dx);
        d[E] = gx * (0.5 * m->dx);
        d[S] = gy * (-0.5 * m->dy);
        d[N] = gy * (0.5 * m->dy);
        for (f = 0; f < 4; ++f) psi = fmin(psi, bj_ratio(d[f], qmax, qmin, fc[k]));
        r->gx[k] = psi * gx;
        r->gy[k] = psi * gy;
    }

    /* Hancock predictor d_t Q = -(A1 d_xQ + A2 d_yQ), grad Q = grad Q^E + Psi grad Q^f [R5]. */
    {
        real A1[NV][NV], A2[NV][NV], qx[NV], qy[NV], dtQ[NV];
        real drhoE = liquid ? -(m->g * m->rho0 / m->k0) * (r->ec[0] / r->ec[3]) : 0.0;
        int a, b;
        matrix_A(m, 0, Qc, A1);
        matrix_A(m, 1, Qc, A2);
        for (k = 0; k < 4; ++k) { qx[k] = r->gx[k]; qy[k] = r->gy[k]; }
        qy[0] += r->ec[3] * drhoE;  /* d_y (alpha^E rho^E) */
        qx[4] = 0.0;
        qy[4] = 1.0;                /* d_y y */
        for (a = 0; a < NV; ++a) {
            real s = 0.0;
            for (b = 0; b < NV; ++b) s += A1[a][b] * qx[b] + A2[a][b] * qy[b];
            dtQ[a] = -s;
        }

        dxf[W] = -0.5 * m->dx; dxf[E] = 0.5 * m->dx; dxf[S] = 0.0;          dxf[N] = 0.0;
        dyf[W] = 0.0;          dyf[E] = 0.0;         dyf[S] = -0.5 * m->dy; dyf[N] = 0.5 * m->dy;
        for (f = 0; f < 4; ++f) {
            estate(m, liquid, Y0[i], yf[f], r->e[f]);
            for (k = 0; k < 4; ++k)
                r->q[f][k] = r->e[f][k] + fc[k] + (r->gx[k] * dxf[f] + r->gy[k] * dyf[f]) + 0.5 * dt * dtQ[k];
            r->q[f][4] = yf[f];
        }
        for (k = 0; k < 4; ++k) r->qc[k] = Qc[k] + 0.5 * dt * dtQ[k];
        r->qc[4] = yc;
    }
}

/* ------------------------------------------------------------------------------------ */
/* Edges, walls and the cell update, Sec. 3 (scheme)                                    */
/* ------------------------------------------------------------------------------------ */

static void wall_ghost(const real q[NV], int normal, int transmissive, real g[NV])
{
    int k;
    for (k = 0; k < NV; ++k) g[k] = q[k];
    if (!transmissive) g[normal] = -g[normal];
}

/* x-edge between left cell and right cell (either may be NULL = solid/outside) [R19].
 * at_w / at_e flag an edge on the domain's west / east side. */
static void edge_x(const model_t *m, const recon_t *lf, const recon_t *rt, int at_w, int at_e,
                   real Dm[NV], real Dp[NV])
{
    real qm[NV], qp[NV];
    int k;
    if (lf) for (k = 0; k < NV; ++k) qm[k] = lf->q[E][k];
    else wall_ghost(rt->q[W], 1, at_w && m->bc[W] == 1, qm);
    if (rt) for (k = 0; k < NV; ++k) qp[k] = rt->q[W][k];
    else wall_ghost(lf->q[E], 1, at_e && m->bc[E] == 1, qp);
    fluct_x(m, qm, qp, Dm, Dp);
}

static void edge_y(const model_t *m, const recon_t *bt, const recon_t *tp, int at_s, int at_n,
                   real Dm[NV], real Dp[NV])
{
    real qm[NV], qp[NV], em[NV], ep[NV];
    int k;
    if (bt) for (k = 0; k < NV; ++k) { qm[k] = bt->q[N][k]; em[k] = bt->e[N][k]; }
    else { wall_ghost(tp->q[S], 2, at_s && m->bc[S] == 1, qm); for (k = 0; k < NV; ++k) em[k] = tp->e[S][k]; }
    if (tp) for (k = 0; k < NV; ++k) { qp[k] = tp->q[S][k]; ep[k] = tp->e[S][k]; }
    else { wall_ghost(bt->q[N], 2, at_n && m->bc[N] == 1, qp); for (k = 0; k < NV; ++k) ep[k] = bt->e[N][k]; }
    fluct_y(m, qm, em, qp, ep, Dm, Dp);
}

/* Q^{n+1} = Q^n - dt/dx (D+_W + D-_E + f(q_E) - f(q_W)) - dt/dy (D+_S + D-_N + g(q_N) - g(q_S))
 *           - dt * B(q_c) grad q  [R1][R2][R4]. */
static void update_cell(const model_t *m, const real Qn[NV], const recon_t *r, const real DpW[NV],
                        const real DmE[NV], const real DpS[NV], const real DmN[NV], real dt, real out[4])
{
    real fdiff[NV], gdiff[NV], vol[NV];
    int k;
    for (k = 0; k < NV; ++k) { fdiff[k] = 0.0; gdiff[k] = 0.0; vol[k] = 0.0; }
    if (r->so) {
        real fE[NV], fW[NV], gN[NV], gS[NV];
        real uc = r->qc[1] / r->qc[0], vc = r->qc[2] / r->qc[0];
        real rhoc = r->qc[0] / r->qc[3], rhoE = r->ec[0] / r->ec[3];
        real alF = r->qc[3] - r->ec[3], rhoF = rhoc - rhoE, alE = r->ec[3];
        flux_f(m, r->q[E], fE);
        flux_f(m, r->q[W], fW);
        flux_g(m, r->q[N], gN);
        flux_g(m, r->q[S], gS);
        for (k = 0; k < NV; ++k) { fdiff[k] = fE[k] - fW[k]; gdiff[k] = gN[k] - gS[k]; }
        /* d_y (alpha p)^f of the linear reconstruction (gamma = 1: alpha p = k0 (alpha rho/rho0 - alpha))
         * plus the gravity part of the fluctuations, g (aE rhoF + aF rhoE + aF rhoF), at (x_c, t^{n+1/2}). */
        vol[2] = m->k0 * (r->gy[0] / m->rho0 - r->gy[3]) + (alE * rhoF + alF * rhoE + alF * rhoF) * m->g;
        vol[3] = uc * r->gx[3] + vc * r->gy[3];
    }
    for (k = 0; k < 4; ++k)
        out[k] = Qn[k] - dt / m->dx * (DpW[k] + DmE[k] + fdiff[k])
                       - dt / m->dy * (DpS[k] + DmN[k] + gdiff[k])
                       - dt * vol[k];
}

/* ------------------------------------------------------------------------------------ */
/* Public entry points (test infrastructure)                                            */
/* ------------------------------------------------------------------------------------ */

static int make_model(const bnref_grid *gr, const bnref_params *pa, const uint8_t *solid, const double *ybot,
                      model_t *m)
{
    int i, k;
    if (!gr || !pa || gr->nx <= 0 || gr->ny <= 0 || !(gr->x1 > gr->x0) || !(gr->y1 > gr->y0)) return BNREF_EINVAL;
    if (!(pa->k0 > 0.0) || !(pa->rho0 > 0.0) || !(pa->alpha_gas > 0.0) || !(pa->alpha_liq > pa->alpha_gas)
        || !(pa->alpha_liq <= 1.0) || !(pa->cfl > 0.0) || !(pa->cfl <= 1.0) || !(pa->g >= 0.0))
        return BNREF_EINVAL;
    m->nx = gr->nx; m->ny = gr->ny;
    m->dx = (gr->x1 - gr->x0) / gr->nx;
    m->dy = (gr->y1 - gr->y0) / gr->ny;
    m->ylo = gr->y0;
    m->g = pa->g; m->k0 = pa->k0; m->rho0 = pa->rho0; m->al = pa->alpha_liq; m->ag = pa->alpha_gas;
    for (k = 0; k < 4; ++k) {
        if (pa->bc[k] != 0 && pa->bc[k] != 1) return BNREF_EINVAL;
        m->bc[k] = pa->bc[k];
    }
    m->solid = solid;
    m->ybot = ybot;
    /* [R21] each bottom lies within half a cell of the top of its column's solid run */
    if (ybot)
        for (i = 0; i < m->nx; ++i) {
            int jb = 0;
            real d;
            while (jb < m->ny && !is_fluid(m, i, jb)) ++jb;
            d = ybot[i] - (m->ylo + jb * m->dy);
            if (!(d >= -0.5 * m->dy && d < 0.5 * m->dy)) return BNREF_EINVAL;
        }
    return BNREF_OK;
}

int bnref_detector(const bnref_grid *gr, const bnref_params *pa, const uint8_t *solid, const double *ybot,
                   const double *q, double *y0)
{
    model_t m;
    real *Y0;
    int rc = make_model(gr, pa, solid, ybot, &m), i;
    if (rc) return rc;
    Y0 = (real *)malloc(sizeof(real) * m.nx);
    rc = detector(&m, q, Y0);
    for (i = 0; i < m.nx; ++i) y0[i] = TO_DOUBLE(Y0[i]);
    free(Y0);
    return rc;
}

/* Largest characteristic rate over fluid cells and dt = CFL / rate [R10].  Flags states
 * that are not finite or have alpha rho <= 0 or alpha <= 0. */
int bnref_cfl(const bnref_grid *gr, const bnref_params *pa, const uint8_t *solid, const double *Q,
              double *lambda_out, double *dt_out)
{
    model_t m;
    size_t plane;
    real lam = 0.0, c;
    int rc = make_model(gr, pa, solid, NULL, &m), i, j;
    if (rc) return rc;
    plane = (size_t)m.nx * m.ny;
    c = sqrt(eos_c2(&m));
    for (j = 0; j < m.ny; ++j)
        for (i = 0; i < m.nx; ++i) {
            size_t idx = (size_t)j * m.nx + i;
            real q0, q1, q2, q3, u, v, l;
            if (!is_fluid(&m, i, j)) continue;
            q0 = Q[idx]; q1 = Q[plane + idx]; q2 = Q[2 * plane + idx]; q3 = Q[3 * plane + idx];
            if (!(q0 > 0.0) || !(q3 > 0.0) || !isfinite(TO_DOUBLE(q0)) || !isfinite(TO_DOUBLE(q1))
                || !isfinite(TO_DOUBLE(q2)) || !isfinite(TO_DOUBLE(q3)))
                return BNREF_ENONPHYS;
            u = q1 / q0;
            v = q2 / q0;
            l = (fabs(u) + c) / m.dx + (fabs(v) + c) / m.dy;
            lam = fmax(lam, l);
        }
    if (lambda_out) *lambda_out = TO_DOUBLE(lam);
    if (dt_out) *dt_out = TO_DOUBLE(pa->cfl / lam);
    return BNREF_OK;
}

/* One full explicit step Q^n -> Q^{n+1} with the given dt: detector, reconstruction of every
 * fluid cell, every edge fluctuation once, cell update.  Solid cells are copied. */
int bnref_step(const bnref_grid *gr, const bnref_params *pa, const uint8_t *solid, const double *ybot,
               const double *Qn, double dt_in, double *Qout)
{
    model_t m;
    real *Y0, dt = dt_in;
    recon_t *R;
    real *Dxm, *Dxp, *Dym, *Dyp;
    size_t plane;
    int rc = make_model(gr, pa, solid, ybot, &m), i, j, k;
    if (rc) return rc;
    if (!(dt_in > 0.0)) return BNREF_EINVAL;
    plane = (size_t)m.nx * m.ny;
    Y0 = (real *)malloc(sizeof(real) * m.nx);
    R = (recon_t *)calloc(plane, sizeof(recon_t));
    Dxm = (real *)calloc((size_t)(m.nx + 1) * m.ny * NV, sizeof(real));
    Dxp = (real *)calloc((size_t)(m.nx + 1) * m.ny * NV, sizeof(real));
    Dym = (real *)calloc((size_t)m.nx * (m.ny + 1) * NV, sizeof(real));
    Dyp = (real *)calloc((size_t)m.nx * (m.ny + 1) * NV, sizeof(real));
    rc = detector(&m, Qn, Y0);
    if (rc) goto done;

    /* Rows are independent within each of the four sweeps below: with OpenMP they are shared
     * out over threads, and every value is still computed by the same arithmetic. */
#pragma omp parallel for private(i) schedule(dynamic, 1) if (plane >= BNREF_PARALLEL_CELLS)
    for (j = 0; j < m.ny; ++j)
        for (i = 0; i < m.nx; ++i)
            if (is_fluid(&m, i, j)) reconstruct(&m, Qn, Y0, i, j, dt, &R[(size_t)j * m.nx + i]);

    /* x-edges: edge fi sits between cells fi-1 and fi of row j. */
#pragma omp parallel for private(i) schedule(dynamic, 1) if (plane >= BNREF_PARALLEL_CELLS)
    for (j = 0; j < m.ny; ++j)
        for (i = 0; i <= m.nx; ++i) {
            const recon_t *lf = is_fluid(&m, i - 1, j) ? &R[(size_t)j * m.nx + i - 1] : NULL;
            const recon_t *rt = is_fluid(&m, i, j) ? &R[(size_t)j * m.nx + i] : NULL;
            size_t e = ((size_t)j * (m.nx + 1) + i) * NV;
            if (lf || rt) edge_x(&m, lf, rt, i == 0, i == m.nx, &Dxm[e], &Dxp[e]);
        }
    /* y-edges: edge fj sits between rows fj-1 and fj of column i. */
#pragma omp parallel for private(i) schedule(dynamic, 1) if (plane >= BNREF_PARALLEL_CELLS)
    for (j = 0; j <= m.ny; ++j)
        for (i = 0; i < m.nx; ++i) {
            const recon_t *bt = is_fluid(&m, i, j - 1) ? &R[(size_t)(j - 1) * m.nx + i] : NULL;
            const recon_t *tp = is_fluid(&m, i, j) ? &R[(size_t)j * m.nx + i] : NULL;
            size_t e = ((size_t)j * m.nx + i) * NV;
            if (bt || tp) edge_y(&m, bt, tp, j == 0, j == m.ny, &Dym[e], &Dyp[e]);
        }

#pragma omp parallel for private(i, k) schedule(dynamic, 1) if (plane >= BNREF_PARALLEL_CELLS)
    for (j = 0; j < m.ny; ++j)
        for (i = 0; i < m.nx; ++i) {
            size_t c = (size_t)j * m.nx + i;
            real Qc[NV], out[4];
            if (!is_fluid(&m, i, j)) {
                for (k = 0; k < 4; ++k) Qout[k * plane + c] = Qn[k * plane + c];
                continue;
            }
            load_q(&m, Qn, i, j, Qc);
            update_cell(&m, Qc, &R[c],
                        &Dxp[((size_t)j * (m.nx + 1) + i) * NV],      /* D+ of the west edge */
                        &Dxm[((size_t)j * (m.nx + 1) + i + 1) * NV],  /* D- of the east edge */
                        &Dyp[((size_t)j * m.nx + i) * NV],            /* D+ of the south edge */
                        &Dym[((size_t)(j + 1) * m.nx + i) * NV],      /* D- of the north edge */
                        dt, out);
            for (k = 0; k < 4; ++k) Qout[k * plane + c] = TO_DOUBLE(out[k]);
        }
done:
    free(Y0); free(R); free(Dxm); free(Dxp); free(Dym); free(Dyp);
    return rc;
}

/* The same update for a list of cells only (flat indices j*nx+i), each computed on its own
 * from Q^n: the checker for samples of grids too large for a full oracle step.
 * out is [4][ncells].  Solid cells return their input. */
int bnref_step_cells(const bnref_grid *gr, const bnref_params *pa, const uint8_t *solid, const double *ybot,
                     const double *Qn, double dt_in, int64_t ncells, const int64_t *cells, double *out)
{
    model_t m;
    real *Y0, dt = dt_in;
    size_t plane;
    int64_t n;
    int rc = make_model(gr, pa, solid, ybot, &m), k;
    if (rc) return rc;
    if (!(dt_in > 0.0) || ncells < 0) return BNREF_EINVAL;
    plane = (size_t)m.nx * m.ny;
    Y0 = (real *)malloc(sizeof(real) * m.nx);
    rc = detector(&m, Qn, Y0);
    if (rc) { free(Y0); return rc; }
    for (n = 0; n < ncells; ++n)
        if (cells[n] < 0 || (size_t)cells[n] >= plane) { free(Y0); return BNREF_EINVAL; }
#pragma omp parallel for private(k) schedule(dynamic, 16) if (ncells >= 4096)
    for (n = 0; n < ncells; ++n) {
        int i, j;
        recon_t rc0, rw, re, rs, rn;
        real Qc[NV], res[4], DpW[NV], DmE[NV], DpS[NV], DmN[NV], dummy[NV];
        i = (int)(cells[n] % m.nx);
        j = (int)(cells[n] / m.nx);
        if (!is_fluid(&m, i, j)) {
            for (k = 0; k < 4; ++k) out[k * ncells + n] = Qn[k * plane + (size_t)cells[n]];
            continue;
        }
        reconstruct(&m, Qn, Y0, i, j, dt, &rc0);
        if (is_fluid(&m, i - 1, j)) reconstruct(&m, Qn, Y0, i - 1, j, dt, &rw);
        if (is_fluid(&m, i + 1, j)) reconstruct(&m, Qn, Y0, i + 1, j, dt, &re);
        if (is_fluid(&m, i, j - 1)) reconstruct(&m, Qn, Y0, i, j - 1, dt, &rs);
        if (is_fluid(&m, i, j + 1)) reconstruct(&m, Qn, Y0, i, j + 1, dt, &rn);
        edge_x(&m, is_fluid(&m, i - 1, j) ? &rw : NULL, &rc0, i == 0, 0, dummy, DpW);
        edge_x(&m, &rc0, is_fluid(&m, i + 1, j) ? &re : NULL, 0, i == m.nx - 1, DmE, dummy);
        edge_y(&m, is_fluid(&m, i, j - 1) ? &rs : NULL, &rc0, j == 0, 0, dummy, DpS);
        edge_y(&m, &rc0, is_fluid(&m, i, j + 1) ? &rn : NULL, 0, j == m.ny - 1, DmN, dummy);
        load_q(&m, Qn, i, j, Qc);
        update_cell(&m, Qc, &rc0, DpW, DmE, DpS, DmN, dt, res);
        for (k = 0; k < 4; ++k) out[k * ncells + n] = TO_DOUBLE(res[k]);
    }
    free(Y0);
    return BNREF_OK;
}

/* n_steps steps with the CFL time step of the current state before each step [R10].
 * Q is updated in place; t_out receives the elapsed time and dt_out the last dt. */
int bnref_run(const bnref_grid *gr, const bnref_params *pa, const uint8_t *solid, const double *ybot, double *Q,
              int32_t n_steps, double *t_out, double *dt_out)
{
    size_t plane;
    double *tmp, t = 0.0, dt = 0.0;
    int s, rc = BNREF_OK;
    if (!gr || gr->nx <= 0 || gr->ny <= 0 || n_steps < 0) return BNREF_EINVAL;
    plane = (size_t)gr->nx * gr->ny;
    tmp = (double *)malloc(sizeof(double) * 4 * plane);
    for (s = 0; s < n_steps; ++s) {
        rc = bnref_cfl(gr, pa, solid, Q, NULL, &dt);
        if (rc) break;
        rc = bnref_step(gr, pa, solid, ybot, Q, dt, tmp);
        if (rc) break;
        memcpy(Q, tmp, sizeof(double) * 4 * plane);
        t += dt;
    }
    free(tmp);
    if (t_out) *t_out = t;
    if (dt_out) *dt_out = dt;
    return rc;
}

/* Threads of the row sweeps (1 without OpenMP).  bnref_set_threads(n) with n >= 1 sets them;
 * results do not depend on the count. */
#ifdef _OPENMP
#include <omp.h>
int bnref_threads(void) { return omp_get_max_threads(); }
void bnref_set_threads(int32_t n) { if (n >= 1) omp_set_num_threads(n); }
#else
int bnref_threads(void) { return 1; }
void bnref_set_threads(int32_t n) { (void)n; }
#endif

/* ---- pieces exported for the oracle's own pins (unit tests) ---------------------------- */

static int pieces_model(const bnref_params *pa, model_t *m)
{
    bnref_grid gr = {1, 1, 0.0, 1.0, 0.0, 1.0};
    return make_model(&gr, pa, NULL, NULL, m);
}

int bnref_flux(const bnref_params *pa, int32_t dir, const double *q, double *out)
{
    model_t m;
    real qq[NV], f[NV];
    int k, rc = pieces_model(pa, &m);
    if (rc) return rc;
    for (k = 0; k < NV; ++k) qq[k] = q[k];
    if (dir == 0) flux_f(&m, qq, f); else flux_g(&m, qq, f);
    for (k = 0; k < NV; ++k) out[k] = TO_DOUBLE(f[k]);
    return BNREF_OK;
}

int bnref_matrix(const bnref_params *pa, int32_t dir, int32_t kind, const double *q, double *out)
{
    /* kind 0: A, 1: R, 2: lambda (5 values), 3: R^{-1}, 4: |A|, 5: sign(A) */
    model_t m;
    real qq[NV], M[NV][NV], R[NV][NV], L[NV][NV], lam[NV];
    int a, b, rc = pieces_model(pa, &m);
    if (rc) return rc;
    for (a = 0; a < NV; ++a) qq[a] = q[a];
    if (kind == 0) matrix_A(&m, dir, qq, M);
    else if (kind >= 1 && kind <= 3) {
        eigen(&m, dir, qq, R, lam, L);
        if (kind == 2) { for (a = 0; a < NV; ++a) out[a] = TO_DOUBLE(lam[a]); return BNREF_OK; }
        for (a = 0; a < NV; ++a)
            for (b = 0; b < NV; ++b) M[a][b] = (kind == 1) ? R[a][b] : L[a][b];
    } else if (kind == 4 || kind == 5) matrix_function(&m, dir, kind - 4, qq, M);
    else return BNREF_EINVAL;
    for (a = 0; a < NV; ++a)
        for (b = 0; b < NV; ++b) out[a * NV + b] = TO_DOUBLE(M[a][b]);
    return BNREF_OK;
}

int bnref_fluct(const bnref_params *pa, int32_t dir, const double *qm, const double *em, const double *qp,
                const double *ep, double *Dm, double *Dp)
{
    model_t m;
    real a[NV], b[NV], ea[NV], eb[NV], dm[NV], dp[NV];
    int k, rc = pieces_model(pa, &m);
    if (rc) return rc;
    for (k = 0; k < NV; ++k) {
        a[k] = qm[k]; b[k] = qp[k];
        ea[k] = em ? em[k] : 0.0; eb[k] = ep ? ep[k] : 0.0;
    }
    if (dir == 0) fluct_x(&m, a, b, dm, dp);
    else {
        if (!em || !ep) return BNREF_EINVAL;
        fluct_y(&m, a, ea, b, eb, dm, dp);
    }
    for (k = 0; k < NV; ++k) { Dm[k] = TO_DOUBLE(dm[k]); Dp[k] = TO_DOUBLE(dp[k]); }
    return BNREF_OK;
}

/* Reconstruction of cell (i, j): faces [4][5], E-parts [4][5], centre [5], limited
 * gradients gx[4], gy[4]; returns the second-order flag (0/1) or a negative error. */
int bnref_reconstruct(const bnref_grid *gr, const bnref_params *pa, const uint8_t *solid, const double *ybot,
                      const double *Q, int32_t i, int32_t j, double dt, double *faces, double *eparts,
                      double *centre, double *grad)
{
    model_t m;
    real *Y0;
    recon_t r;
    int rc = make_model(gr, pa, solid, ybot, &m), f, k;
    if (rc) return rc;
    if (!is_fluid(&m, i, j)) return BNREF_EINVAL;
    Y0 = (real *)malloc(sizeof(real) * m.nx);
    rc = detector(&m, Q, Y0);
    if (rc) { free(Y0); return rc; }
    reconstruct(&m, Q, Y0, i, j, dt, &r);
    free(Y0);
    for (f = 0; f < 4; ++f)
        for (k = 0; k < NV; ++k) {
            faces[f * NV + k] = TO_DOUBLE(r.q[f][k]);
            eparts[f * NV + k] = TO_DOUBLE(r.e[f][k]);
        }
    for (k = 0; k < NV; ++k) centre[k] = TO_DOUBLE(r.qc[k]);
    for (k = 0; k < 4; ++k) { grad[k] = TO_DOUBLE(r.gx[k]); grad[4 + k] = TO_DOUBLE(r.gy[k]); }
    return r.so;
}
