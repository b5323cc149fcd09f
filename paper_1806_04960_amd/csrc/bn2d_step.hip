// Fused explicit step of the well-balanced Osher-Romberg scheme (Gaburro, Castro, Dumbser,
// arXiv:1806.04960, Sec. 3) for gfx950, FP64 on the vector ALUs.
//
// Work decomposition.  One wavefront (64 lanes) owns a strip of 64 columns, lane L holding
// column i0 - 2 + L, and marches upwards through H rows.  Per row it loads one row of the
// state (coalesced, one 8-byte value per lane and plane), keeps the 3 x 3 stencil window of the
// state in registers (neighbour columns through cross-lane shuffles), reconstructs the row below
// the newest one, computes every x-edge of that row and the y-edge below it exactly once, and
// finishes the row below that: the edge fluctuations a row needs are all in its own lane or in
// the adjacent lane, so nothing but the state crosses HBM.  Lanes 2..61 produce output; lanes
// 0, 1, 62, 63 are the column halo (lanes 1 and 62 reconstruct, 0 and 63 only load).
//
// Besides Q^{n+1} the kernel writes, per column and row block, the partial sum of
// (alpha - alpha_g)/(alpha_l - alpha_g) over the fluid cells it updated (the free-surface
// detector of Sec. 3.5 for the next step, summed upward), and folds the CFL rate of every
// updated cell into one 64-bit atomic max.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bn2d_physics.h"

namespace bn {

__device__ __forceinline__ double shfl_from_left(double v) { return __shfl_up(v, 1, 64); }
__device__ __forceinline__ double shfl_from_right(double v) { return __shfl_down(v, 1, 64); }
__device__ __forceinline__ int shfl_from_left(int v) { return __shfl_up(v, 1, 64); }
__device__ __forceinline__ int shfl_from_right(int v) { return __shfl_down(v, 1, 64); }

__global__ __launch_bounds__(64) void step_kernel(const double *__restrict__ Q, double *__restrict__ Qn,
                                                   const uint8_t *__restrict__ solid, const double *__restrict__ Y0,
                                                   const double *__restrict__ dt_dev, double dt_arg,
                                                   double *__restrict__ partial, unsigned long long *lam_slot,
                                                   int *flag, Consts K, int H)
{
    const int lane = threadIdx.x;
    const int i = (int)blockIdx.x * 60 - 2 + lane;
    const int j0 = (int)blockIdx.y * H;
    const bool colin = i >= 0 && i < K.nx;
    const bool out_lane = colin && lane >= 2 && lane < 62;
    const bool rec_lane = lane >= 1 && lane <= 62;
    const size_t plane = (size_t)K.nx * K.ny;
    const double dt = dt_dev ? *dt_dev : dt_arg;
    const double dtdx = dt / K.dx, dtdy = dt / K.dy;
    const double y0c = colin ? Y0[i] : 0.0;

    double wq[3][3][4];
    int wf[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            wf[a][b] = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) wq[a][b][k] = 1.0;
        }

    // pending row (the one below the row being reconstructed)
    double pP[4] = {0, 0, 0, 0}, pDpS[4] = {0, 0, 0, 0}, pG[4] = {0, 0, 0, 0}, pV2 = 0.0, pV3 = 0.0;
    double nQ[4] = {1, 0, 0, 1}, nE1 = 1.0, nAE = 1.0, nY = 0.0;
    int nF = 0;
    double colsum = 0.0, lam = 0.0;
    int bad = 0;

    for (int r = j0 - 2; r <= j0 + H + 1; ++r) {
        // ---- shift the window and load row r --------------------------------------------
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                wf[a][b] = wf[a + 1][b];
#pragma unroll
                for (int k = 0; k < 4; ++k) wq[a][b][k] = wq[a + 1][b][k];
            }
        {
            const bool rowin = r >= 0 && r < K.ny;
            int f = 0;
            double q[4] = {1.0, 0.0, 0.0, 1.0};
            if (!colin) f |= (i < 0) ? F_OUTW : F_OUTE;
            if (!rowin) f |= (r < 0) ? F_OUTS : F_OUTN;
            if (colin && rowin) {
                const size_t cidx = (size_t)r * K.nx + i;
                if (!solid || solid[cidx] == 0) f |= F_FLUID;
#pragma unroll
                for (int k = 0; k < 4; ++k) q[k] = Q[k * plane + cidx];
            }
            wf[2][1] = f;
            wf[2][0] = shfl_from_left(f);
            wf[2][2] = shfl_from_right(f);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                wq[2][1][k] = q[k];
                wq[2][0][k] = shfl_from_left(q[k]);
                wq[2][2][k] = shfl_from_right(q[k]);
            }
        }
        if (r < j0) continue;

        // ---- reconstruct row jr = r - 1 ----------------------------------------------------
        const int jr = r - 1;
        const bool fl = rec_lane && (wf[1][1] & F_FLUID);
        Rec rc;
        if (fl) {
            reconstruct(K, wq, wf, jr, y0c, dt, rc);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                rc.qW[k] = wq[1][1][k]; rc.qE[k] = wq[1][1][k]; rc.qS[k] = wq[1][1][k]; rc.qN[k] = wq[1][1][k];
                rc.fdiff[k] = 0.0; rc.gdiff[k] = 0.0;
            }
            rc.e1S = 1.0; rc.e1N = 1.0; rc.aE = 1.0; rc.yS = 0.0; rc.yN = 0.0; rc.vol2 = 0.0; rc.vol3 = 0.0;
        }
        const bool jr_inside_block = jr >= j0 && jr < j0 + H;

        // ---- x-edges of row jr: lane L solves the edge between columns L and L+1 ------------
        double DpW[4] = {0, 0, 0, 0}, DmE[4] = {0, 0, 0, 0};
        if (jr_inside_block) {
            double qWr[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) qWr[k] = shfl_from_right(rc.qW[k]);
            const int fR = shfl_from_right(wf[1][1]);
            const bool rf = (lane <= 61) && (fR & F_FLUID);
            double Dm[4] = {0, 0, 0, 0}, Dp[4] = {0, 0, 0, 0};
            if (fl || rf) {
                double qm[4], qp[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    qm[k] = fl ? rc.qE[k] : qWr[k];
                    qp[k] = rf ? qWr[k] : rc.qE[k];
                }
                // wall: mirror state with negated normal momentum, or a copy on a transmissive side
                if (!fl && !((wf[1][1] & F_OUTW) && K.bc[0] == 1)) qm[1] = -qm[1];
                if (!rf && !((fR & F_OUTE) && K.bc[1] == 1)) qp[1] = -qp[1];
                edge_x(K, qm, qp, Dm, Dp);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                DmE[k] = Dm[k];
                DpW[k] = shfl_from_left(Dp[k]);
            }
        }

        // ---- y-edge between row jr-1 (pending north state) and row jr ----------------------
        double DyM[4] = {0, 0, 0, 0}, DyP[4] = {0, 0, 0, 0};
        if (r > j0) {
            const bool bf = rec_lane && (nF & F_FLUID);
            if (bf || fl) {
                double qm[4], qp[4], e1m, aEm, ym, e1p, aEp, yp;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    qm[k] = bf ? nQ[k] : rc.qS[k];
                    qp[k] = fl ? rc.qS[k] : nQ[k];
                }
                e1m = bf ? nE1 : rc.e1S; aEm = bf ? nAE : rc.aE; ym = bf ? nY : rc.yS;
                e1p = fl ? rc.e1S : nE1; aEp = fl ? rc.aE : nAE; yp = fl ? rc.yS : nY;
                if (!bf && !((nF & F_OUTS) && K.bc[2] == 1)) qm[2] = -qm[2];
                if (!fl && !((wf[1][1] & F_OUTN) && K.bc[3] == 1)) qp[2] = -qp[2];
                edge_y(K, qm, e1m, aEm, ym, qp, e1p, aEp, yp, DyM, DyP);
            }
        }

        // ---- finish row jr-1 ---------------------------------------------------------------
        const int jf = jr - 1;
        if (r > j0 && jf >= j0 && jf < j0 + H && out_lane && jf < K.ny) {
            const size_t cidx = (size_t)jf * K.nx + i;
            const int ff = wf[0][1];
            if (ff & F_FLUID) {
                double qn[4];
                update_finish(pP, pDpS, DyM, pG, pV2, pV3, dt, dtdy, qn);
#pragma unroll
                for (int k = 0; k < 4; ++k) Qn[k * plane + cidx] = qn[k];
                colsum += detector_term(K, qn);
                lam = fmax(lam, cfl_rate(K, qn));
                if (!(qn[0] > 0.0) || !(qn[3] > 0.0) || !isfinite(qn[0]) || !isfinite(qn[1]) ||
                    !isfinite(qn[2]) || !isfinite(qn[3]))
                    bad = 1;
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) Qn[k * plane + cidx] = wq[0][1][k];
            }
        }

        // ---- row jr becomes the pending row ------------------------------------------------
        if (jr_inside_block && fl) {
            update_x_part(wq[1][1], DpW, DmE, rc.fdiff, dtdx, pP);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                pDpS[k] = DyP[k];
                pG[k] = rc.gdiff[k];
            }
            pV2 = rc.vol2;
            pV3 = rc.vol3;
        }
        if (fl) {
#pragma unroll
            for (int k = 0; k < 4; ++k) nQ[k] = rc.qN[k];
            nE1 = rc.e1N;
            nAE = rc.aE;
            nY = rc.yN;
        }
        nF = wf[1][1];
    }

    if (out_lane) partial[(size_t)blockIdx.y * K.nx + i] = colsum;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        lam = fmax(lam, __shfl_xor(lam, off, 64));
        bad |= __shfl_xor(bad, off, 64);
    }
    if (lane == 0) {
        if (lam > 0.0) atomicMax(lam_slot, (unsigned long long)__double_as_longlong(lam));
        if (bad) atomicOr(flag, 1);
    }
}

// Detector partial sums and CFL rate of a state (used after bn_set_state), same layout as the
// step kernel's output: thread = column, blockIdx.y = row block.
__global__ __launch_bounds__(64) void reduce_kernel(const double *__restrict__ Q, const uint8_t *__restrict__ solid,
                                                     double *__restrict__ partial, unsigned long long *lam_slot,
                                                     int *flag, Consts K, int H)
{
    const int i = (int)blockIdx.x * 64 + threadIdx.x;
    const size_t plane = (size_t)K.nx * K.ny;
    double colsum = 0.0, lam = 0.0;
    int bad = 0;
    if (i < K.nx) {
        const int ja = (int)blockIdx.y * H, jb = min(K.ny, ja + H);
        for (int j = ja; j < jb; ++j) {
            const size_t cidx = (size_t)j * K.nx + i;
            if (solid && solid[cidx]) continue;
            const double q0 = Q[cidx], q1 = Q[plane + cidx], q2 = Q[2 * plane + cidx], q3 = Q[3 * plane + cidx];
            const double q[4] = {q0, q1, q2, q3};
            colsum += detector_term(K, q);
            lam = fmax(lam, cfl_rate(K, q));
            if (!(q0 > 0.0) || !(q3 > 0.0) || !isfinite(q0) || !isfinite(q1) || !isfinite(q2) || !isfinite(q3))
                bad = 1;
        }
        partial[(size_t)blockIdx.y * K.nx + i] = colsum;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        lam = fmax(lam, __shfl_xor(lam, off, 64));
        bad |= __shfl_xor(bad, off, 64);
    }
    if (threadIdx.x == 0) {
        if (lam > 0.0) atomicMax(lam_slot, (unsigned long long)__double_as_longlong(lam));
        if (bad) atomicOr(flag, 1);
    }
}

// Free-surface heights y0_i = y_L(i) + dy * sum of the column's partial sums (bottom to top), and
// dt = CFL / max rate; the elapsed time advances by the dt of the step just taken.
__global__ void finalize_kernel(const double *__restrict__ partial, int nseg, const int *__restrict__ jb,
                                double *__restrict__ Y0, unsigned long long *lam_slot, int *flag, double *dt_dev,
                                double *t_dev, double dt_used, int use_dev_dt, int advance_t, Consts K)
{
    const int i = (int)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < K.nx) {
        double s = 0.0;
        for (int seg = 0; seg < nseg; ++seg) s += partial[(size_t)seg * K.nx + i];
        Y0[i] = (K.ylo + jb[i] * K.dy) + K.dy * s;
    }
    if (i == 0) {
        const double used = use_dev_dt ? *dt_dev : dt_used;
        if (advance_t) *t_dev += used;
        const double lam = __longlong_as_double((long long)*lam_slot);
        *lam_slot = 0ull;
        if (lam > 0.0 && isfinite(lam)) {
            *dt_dev = K.cfl / lam;
        } else {
            *dt_dev = 0.0;
            atomicOr(flag, 2);
        }
    }
}

}  // namespace bn
