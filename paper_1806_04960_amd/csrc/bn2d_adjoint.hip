// Discrete adjoint of one explicit step (Sec. 3, eq. Scheme, with a given time step): from the
// state Q^n and the adjoint lambda^{n+1} of Q^{n+1}, lambda^n = (dQ^{n+1}/dQ^n)^T lambda^{n+1}.
//
// The step's data flow, cell c = (i, j):
//   y0_i        = free-surface height of column i (Sec. 3.5)
//   Rec_c       = reconstruct(3 x 3 stencil of c, y0_i)             edge states, S/N equilibria,
//                                                                   flux differences, cell integral
//   D-+(e)      = edge_x / edge_y of the two edge states of e (a wall or solid side mirrors the
//                 fluid side's state)
//   Q^{n+1}_c   = Q^n_c - dt/dx (D+_W + D-_E + fdiff) - dt/dy (D+_S + D-_N + gdiff) - dt vol
// is reversed in three launches through library-owned scratch:
//   1. adj_fused_kernel   per tile of 64 x 4 cells: recompute Rec of the tile and its one-cell halo
//                         into LDS, reverse every x- and y-edge touching the tile (recompute D-+ and
//                         reverse it with the adjoints of the two cells' updates; the adjoints of
//                         the tile cells' edge states go back into LDS: each edge state feeds exactly
//                         one edge, no accumulation), then reverse each tile cell's reconstruction
//                         (adjoints of its 3 x 3 stencil, of a first-order cell only its own entry,
//                         and of y0_i) and sum the stencil adjoints per target cell in LDS: the
//                         tile's cells' sums (4 planes), those falling on the halo (140 cells per
//                         tile) and the tile's share of each column's y0 adjoint
//   2. adj_col_kernel     add the tiles' shares of each column's y0 adjoint (fixed order); and (if
//                         asked) the adjoint of each column's bottom height: its y0 adjoint times
//                         dy0/dy_L = (alpha_l - alpha_first) / (alpha_l - alpha_g) (0 for a column
//                         without fluid cells)
//   3. adj_gather_kernel  lambda^n_c = lambda^{n+1}_c + the stencil adjoints of the (up to 9)
//                         fluid cells whose stencil holds c (the own tile's sum, then those the
//                         neighbouring tiles left on their halos) + the detector's
//                         dy/(alpha_l - alpha_g) times its column's y0 adjoint (alpha only;
//                         (dy - d)/(alpha_l - alpha_g) in the first fluid cell of a column whose
//                         bottom lies d off the grid); solid cells pass lambda through (their state
//                         is copied and never read); an optional source (e.g. dJ/dQ^n of a
//                         trajectory loss) is added to lambda^n last
// Every sum is taken in a fixed order: the result is deterministic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bn2d_adjoint.h"

namespace bn {

struct AdjArgs {
    Consts K;
    const double *q;        // Q^n, 4 planes
    const double *lam1;     // lambda^{n+1}, 4 planes
    double *lam;            // lambda^n, 4 planes
    const uint8_t *solid;   // nx*ny or null
    const int *jb;          // first fluid row per column
    const double *dbot;     // per column: bottom height minus the top of its solid run, or null
    const long long *Sp;    // fixed-point free-surface integral of Q^n per column: nSp partials [nSp][nx]
    int nSp;
    double fix_inv;
    double dt, dtdx, dtdy;
    double *own;            // 4 planes: per cell, the stencil adjoints of its own tile's cells
    double *ring;           // [tiles][4][kRing]: those falling on each tile's halo
    double *colb;           // [ceil(ny / kTY)][nx]: each tile's share of the columns' y0 adjoints
    double *colt;           // [nx]: the columns' y0 adjoints
    double *gbot;           // [nx] adjoint of the bottom heights, or null
    const double *src;      // 4 planes added to lambda^n, or null
};


// record planes of the fused pass's LDS: qW 0-3, qE 4-7, qS 8-11, qN 12-15, e1S 16, e1N 17, aE 18,
// yS 19, yN 20 (the heights of the S/N states: the edge's for a second-order cell, the centre's for a
// first-order one); the face adjoints take the first 18 of them afterwards
constexpr int kRecPlanes = 21;
enum : int { P_QW = 0, P_QE = 4, P_QS = 8, P_QN = 12, P_E1S = 16, P_E1N = 17, P_AE = 18, P_YS = 19, P_YN = 20 };

typedef const __attribute__((address_space(1))) double *GlobalD;
__device__ __forceinline__ bool fluid_at(const AdjArgs &a, int i, int j)
{
    if (i < 0 || i >= a.K.nx || j < 0 || j >= a.K.ny) return false;
    return !a.solid || a.solid[(size_t)j * a.K.nx + i] == 0;
}

// 1 - (alpha - alpha_g)/(alpha_l - alpha_g) of column i's first fluid cell (0 for a full cell)
__device__ __forceinline__ double first_gap(const AdjArgs &a, int i)
{
    const size_t n = (size_t)a.K.nx * a.K.ny;
    return (a.K.al - a.q[3 * n + (size_t)a.jb[i] * a.K.nx + i]) * a.K.inv_dal;
}

__device__ __forceinline__ double y0_of(const AdjArgs &a, int i)
{
    long long S = 0;
    for (int b = 0; b < a.nSp; ++b) S += a.Sp[(size_t)b * a.K.nx + i];  // exact: the order does not matter
    double v = (a.K.ylo + a.jb[i] * a.K.dy) + a.K.dy * ((double)S * a.fix_inv);
    if (a.dbot && a.jb[i] < a.K.ny) v += a.dbot[i] * first_gap(a, i);
    return v;
}

// the mask byte read for every cell when a grid has no solid cells
__device__ const uint8_t kNoSolid[1] = {0};

// The 3 x 3 stencil of cell (i, j): states (outside the grid: the benign (1, 0, 0, 1), never used)
// and flags.  Every load is issued before any is used (clamped addresses, values replaced outside
// the grid): a mask byte tested as soon as it is loaded would wait for it, and for every load before
// it.  (Through global-memory pointers: with a generic one the choice between the state and the
// default becomes one flat load from either address, which every later wait for an LDS or scalar
// load then also waits for.)
__device__ __forceinline__ void load_stencil(const AdjArgs &a, int i, int j, double (&wq)[3][3][4], int (&wf)[3][3])
{
    const int nx = a.K.nx, ny = a.K.ny;
    const size_t plane = (size_t)nx * ny;
    typedef const __attribute__((address_space(1))) uint8_t *GlobalMask;
    const GlobalD qg = (GlobalD)a.q;
    const GlobalMask sg = (GlobalMask)(a.solid ? a.solid : kNoSolid);
    int mb[3][3];
#pragma unroll
    for (int dj = 0; dj < 3; ++dj)
#pragma unroll
        for (int di = 0; di < 3; ++di) {
            const int ii = i + di - 1, jj = j + dj - 1;
            const bool in = ii >= 0 && ii < nx && jj >= 0 && jj < ny;
            const size_t c = (size_t)min(max(jj, 0), ny - 1) * nx + min(max(ii, 0), nx - 1);
            mb[dj][di] = (int)sg[a.solid ? c : 0];
            const double dflt[4] = {1.0, 0.0, 0.0, 1.0};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double v = qg[k * plane + c];
                wq[dj][di][k] = in ? v : dflt[k];
            }
        }
#pragma unroll
    for (int dj = 0; dj < 3; ++dj)
#pragma unroll
        for (int di = 0; di < 3; ++di) {
            const int ii = i + di - 1, jj = j + dj - 1;
            const bool in = ii >= 0 && ii < nx && jj >= 0 && jj < ny;
            wf[dj][di] = cell_flags(ii, jj, nx, ny, a.K.bc, in && mb[dj][di] == 0);
        }
}

struct ArrayStencil {
    static constexpr bool kRingFlags = false;
    const double (*wq)[3][4];
    const int (*wf)[3];
    __device__ __forceinline__ double q(int dj, int di, int k) const { return wq[dj][di][k]; }
    __device__ __forceinline__ int f(int dj, int di) const { return wf[dj][di]; }
};

// ---- pass 1: reconstruction, edges and cells, fused over 64 x 4 tiles ----------------------------
// One workgroup (a thread per cell) per tile of 64 columns x 4 rows.  (a) It recomputes the reconstruction
// of the tile's cells and of a one-cell halo around it (66 x 6 cells) into LDS; (b) every x- and y-edge
// touching a tile cell (65 x 4 and 64 x 5) is reversed from those records and the lambdas of its two
// cells, the adjoints of the tile cells' edge states going back into LDS (over the records, after a
// barrier); (c) each tile cell reverses its reconstruction; (d) the stencil adjoints are summed per
// target cell in LDS.  The edge-state records and their adjoints never reach HBM, nor do the
// per-stencil-entry adjoints.
constexpr int kTX = 64, kTY = 4, kHX = kTX + 2, kHY = kTY + 2, kHalo = kHX * kHY;  // 396 records
constexpr int kThreads = kTX * kTY;  // one thread per tile cell
static_assert((kTX + 1) * kTY <= 2 * kThreads && kTX * (kTY + 1) <= 2 * kThreads, "two rounds of edges");
// the halo's 140 cells in ring order: the row below (66), the row above (66), the column left of the
// tile's rows (4), the column right of them (4)
constexpr int kRing = 2 * kHX + 2 * kTY;
static_assert(kRing <= kThreads, "one ring cell per thread");
__device__ __forceinline__ int ring_cell(int r)
{
    if (r < kHX) return r;
    if (r < 2 * kHX) return (kHY - 1) * kHX + (r - kHX);
    if (r < 2 * kHX + kTY) return (r - 2 * kHX + 1) * kHX;
    return (r - 2 * kHX - kTY + 1) * kHX + kHX - 1;
}

// x-edge between local columns e-1 and e (e = 0..64) of tile row ty; qmb/qpb: the adjoints of the
// left cell's east state and of the right cell's west state (a missing side mirrors the fluid one,
// so its share is folded into the fluid side's)
__device__ __forceinline__ void fused_xedge(const AdjArgs &a, const double (*sr)[kHalo], const int *sf, int i0, int j0,
                                            int e, int ty, double qmb[4], double qpb[4], bool &flL, bool &flR)
{
    const int iL = i0 + e - 1, iR = i0 + e, j = j0 + ty;
    const int hL = (ty + 1) * kHX + e, hR = hL + 1;  // halo-record indices of the two cells
    const int fL = sf[hL], fR = sf[hR];
    flL = fL & F_FLUID;
    flR = fR & F_FLUID;
#pragma unroll
    for (int k = 0; k < 4; ++k) qmb[k] = qpb[k] = 0.0;
    if (!flL && !flR) return;
    const size_t n = (size_t)a.K.nx * a.K.ny;
    double qm[4], qp[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double qEL = flL ? sr[P_QE + k][hL] : 0.0, qWR = flR ? sr[P_QW + k][hR] : 0.0;
        qm[k] = flL ? qEL : qWR;
        qp[k] = flR ? qWR : qEL;
    }
    const double sL = (!flL && !(fL & F_TX)) ? -1.0 : 1.0, sR = (!flR && !(fR & F_TX)) ? -1.0 : 1.0;
    qm[1] *= sL;
    qp[1] *= sR;
    const size_t cL = flL ? (size_t)j * a.K.nx + iL : 0, cR = flR ? (size_t)j * a.K.nx + iR : 0;
    const GlobalD lg = (GlobalD)a.lam1;
    double Dmb[4], Dpb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double lL = lg[k * n + cL], lR = lg[k * n + cR];
        Dmb[k] = flL ? -a.dtdx * lL : 0.0;
        Dpb[k] = flR ? -a.dtdx * lR : 0.0;
    }
    double bm[4] = {0, 0, 0, 0}, bp[4] = {0, 0, 0, 0};
    edge_x_rev(a.K, qm, qp, Dmb, Dpb, bm, bp);
    bm[1] *= sL;
    bp[1] *= sR;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        qmb[k] = bm[k] + (flR ? 0.0 : bp[k]);
        qpb[k] = bp[k] + (flL ? 0.0 : bm[k]);
    }
}

// y-edge between local rows e-1 and e (e = 0..4) of tile column tx
__device__ __forceinline__ void fused_yedge(const AdjArgs &a, const double (*sr)[kHalo], const int *sf, int i0, int j0,
                                            int tx, int e, double qmb[5], double qpb[5], bool &flB, bool &flT)
{
    const int i = i0 + tx, jB = j0 + e - 1, jT = j0 + e;
    const int hB = e * kHX + tx + 1, hT = hB + kHX;
    const int fB = sf[hB], fT = sf[hT];
    flB = fB & F_FLUID;
    flT = fT & F_FLUID;
#pragma unroll
    for (int k = 0; k < 5; ++k) qmb[k] = qpb[k] = 0.0;
    if (!flB && !flT) return;
    const size_t n = (size_t)a.K.nx * a.K.ny;
    double qNB[4], qST[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        qNB[k] = flB ? sr[P_QN + k][hB] : 0.0;
        qST[k] = flT ? sr[P_QS + k][hT] : 0.0;
    }
    const double e1NB = flB ? sr[P_E1N][hB] : 0.0, e1ST = flT ? sr[P_E1S][hT] : 0.0;
    const double aEB = flB ? sr[P_AE][hB] : 0.0, aET = flT ? sr[P_AE][hT] : 0.0;
    const double yN = flB ? sr[P_YN][hB] : 0.0, yS = flT ? sr[P_YS][hT] : 0.0;
    const double sB = (!flB && !(fB & F_TY)) ? -1.0 : 1.0, sT = (!flT && !(fT & F_TY)) ? -1.0 : 1.0;
    double qm[4], qp[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        qm[k] = flB ? qNB[k] : qST[k];
        qp[k] = flT ? qST[k] : qNB[k];
    }
    qm[2] *= sB;
    qp[2] *= sT;
    const double e1m = flB ? e1NB : e1ST, aEm = flB ? aEB : aET, ym = flB ? yN : yS;
    const double e1p = flT ? e1ST : e1NB, aEp = flT ? aET : aEB, yp = flT ? yS : yN;
    const size_t cB = flB ? (size_t)jB * a.K.nx + i : 0, cT = flT ? (size_t)jT * a.K.nx + i : 0;
    const GlobalD lg = (GlobalD)a.lam1;
    double Dmb[4], Dpb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double lB = lg[k * n + cB], lT = lg[k * n + cT];
        Dmb[k] = flB ? -a.dtdy * lB : 0.0;
        Dpb[k] = flT ? -a.dtdy * lT : 0.0;
    }
    double bm[4] = {0, 0, 0, 0}, bp[4] = {0, 0, 0, 0}, e1mb = 0.0, e1pb = 0.0;
    edge_y_rev(a.K, qm, e1m, aEm, ym, qp, e1p, aEp, yp, Dmb, Dpb, bm, e1mb, bp, e1pb);
    bm[2] *= sB;
    bp[2] *= sT;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        qmb[k] = bm[k] + (flT ? 0.0 : bp[k]);
        qpb[k] = bp[k] + (flB ? 0.0 : bm[k]);
    }
    qmb[4] = e1mb + (flT ? 0.0 : e1pb);
    qpb[4] = e1pb + (flB ? 0.0 : e1mb);
}

__global__ __launch_bounds__(kThreads) void adj_fused_kernel(AdjArgs a)
{
    __shared__ double sr[kRecPlanes][kHalo];  // records, then (planes 0..17, first kThreads entries) face adjoints
    __shared__ double sy0[kHX];               // free-surface heights of the tile's columns and halo
    __shared__ int sf[kHalo];                 // flags of the tile's cells and halo
    const int t = threadIdx.x;
    const int i0 = (int)blockIdx.x * kTX, j0 = (int)blockIdx.y * kTY;
    if (t < kHX && i0 + t - 1 >= 0 && i0 + t - 1 < a.K.nx) sy0[t] = y0_of(a, i0 + t - 1);
    __syncthreads();

    // (a) records of the tile and its halo
    for (int h = t; h < kHalo; h += kThreads) {
        const int i = i0 + h % kHX - 1, j = j0 + h / kHX - 1;
        double wq[3][3][4];
        int wf[3][3];
        load_stencil(a, i, j, wq, wf);
        sf[h] = wf[1][1];
        if (!(wf[1][1] & F_FLUID)) continue;
        Rec r;
        ArrayStencil st{wq, wf};
        reconstruct(a.K, st, j, sy0[h % kHX], a.dt, r);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            sr[P_QW + k][h] = r.qW[k];
            sr[P_QE + k][h] = r.qE[k];
            sr[P_QS + k][h] = r.qS[k];
            sr[P_QN + k][h] = r.qN[k];
        }
        sr[P_E1S][h] = r.e1S;
        sr[P_E1N][h] = r.e1N;
        sr[P_AE][h] = r.aE;
        sr[P_YS][h] = r.yS;
        sr[P_YN][h] = r.yN;
    }
    __syncthreads();

    // (b) edges: thread t takes x-edges t and t + kThreads (of 65 x 4) and y-edges t and t + kThreads
    // (of 64 x 5)
    constexpr int nX = (kTX + 1) * kTY, nY = kTX * (kTY + 1);
    double xm[2][4], xp[2][4], ym[2][5], yp[2][5];
    bool xl[2], xr[2], yb[2], yt[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int ex = t + kThreads * u;
        xl[u] = xr[u] = false;
        if (ex < nX) fused_xedge(a, sr, sf, i0, j0, ex % (kTX + 1), ex / (kTX + 1), xm[u], xp[u], xl[u], xr[u]);
        const int ey = t + kThreads * u;
        yb[u] = yt[u] = false;
        if (ey < nY) fused_yedge(a, sr, sf, i0, j0, ey % kTX, ey / kTX, ym[u], yp[u], yb[u], yt[u]);
    }
    __syncthreads();  // every record read: the face adjoints go over them
    // face adjoint of tile cell c = ty * 64 + tx in sr[plane][c]; a cell outside the tile or not
    // fluid is skipped (a missing side's share is already in its fluid neighbour's)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int ex = t + kThreads * u;
        if (ex < nX) {
            const int e = ex % (kTX + 1), ty = ex / (kTX + 1);
            if (xl[u] && e >= 1) {
#pragma unroll
                for (int k = 0; k < 4; ++k) sr[P_QE + k][ty * kTX + e - 1] = xm[u][k];
            }
            if (xr[u] && e < kTX) {
#pragma unroll
                for (int k = 0; k < 4; ++k) sr[P_QW + k][ty * kTX + e] = xp[u][k];
            }
        }
        const int ey = t + kThreads * u;
        if (ey < nY) {
            const int tx = ey % kTX, e = ey / kTX;
            if (yb[u] && e >= 1) {
#pragma unroll
                for (int k = 0; k < 4; ++k) sr[P_QN + k][(e - 1) * kTX + tx] = ym[u][k];
                sr[P_E1N][(e - 1) * kTX + tx] = ym[u][4];
            }
            if (yt[u] && e < kTY) {
#pragma unroll
                for (int k = 0; k < 4; ++k) sr[P_QS + k][e * kTX + tx] = yp[u][k];
                sr[P_E1S][e * kTX + tx] = yp[u][4];
            }
        }
    }
    __syncthreads();

    // (c) the tile cell's reconstruction reversed (a cell outside the grid or not fluid adds nothing)
    const int tx = t % kTX, ty = t / kTX;
    const int i = i0 + tx, j = j0 + ty;
    const bool in = i < a.K.nx && j < a.K.ny;
    const size_t n = (size_t)a.K.nx * a.K.ny;
    const size_t c = in ? (size_t)j * a.K.nx + i : 0;
    double wqb[3][3][4];
#pragma unroll
    for (int dj = 0; dj < 3; ++dj)
#pragma unroll
        for (int di = 0; di < 3; ++di)
#pragma unroll
            for (int k = 0; k < 4; ++k) wqb[dj][di][k] = 0.0;
    bool act = false, so = false;
    double ybar = 0.0;
    if (in) {
        double wq[3][3][4];
        int wf[3][3];
        load_stencil(a, i, j, wq, wf);
        if (wf[1][1] & F_FLUID) {
            act = true;
            so = wq[1][1][3] > a.K.so_thr;
#pragma unroll
            for (int dj = 0; dj < 3; ++dj)
#pragma unroll
                for (int di = 0; di < 3; ++di)
                    if ((wf[dj][di] & F_FLUID) && !(wq[dj][di][3] > a.K.so_thr)) so = false;
            RecBar rb;
            const GlobalD lg = (GlobalD)a.lam1;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                rb.qW[k] = sr[P_QW + k][t];
                rb.qE[k] = sr[P_QE + k][t];
                rb.qS[k] = sr[P_QS + k][t];
                rb.qN[k] = sr[P_QN + k][t];
                const double l = lg[k * n + c];
                rb.fdiff[k] = -a.dtdx * l;
                rb.gdiff[k] = -a.dtdy * l;
            }
            rb.e1S = sr[P_E1S][t];
            rb.e1N = sr[P_E1N][t];
            rb.vol2 = -a.dt * lg[2 * n + c];
            rb.vol3 = -a.dt * lg[3 * n + c];
            ybar = reconstruct_rev(a.K, wq, wf, j, sy0[tx + 1], a.dt, rb, wqb);
        }
    }
    __syncthreads();  // every record read: the sums go over them

    // (d) the stencil adjoints summed per target cell in LDS (planes 0-3 over the tile and its halo),
    // one stencil entry after another: within one entry the targets of different cells differ, so
    // every sum is taken in the fixed order of the entries (deterministic).  A first-order cell
    // reaches only itself.  The y0 adjoints of the tile's cells go to plane 4.
    for (int h = t; h < kHalo; h += kThreads) {
#pragma unroll
        for (int k = 0; k < 4; ++k) sr[k][h] = 0.0;
    }
    sr[4][t] = ybar;
    __syncthreads();
#pragma unroll
    for (int dj = 0; dj < 3; ++dj)
#pragma unroll
        for (int di = 0; di < 3; ++di) {
            if (act && (so || (dj == 1 && di == 1))) {
                const int h = (ty + dj) * kHX + tx + di;
#pragma unroll
                for (int k = 0; k < 4; ++k) sr[k][h] += wqb[dj][di][k];
            }
            __syncthreads();
        }
    if (in) {
#pragma unroll
        for (int k = 0; k < 4; ++k) a.own[k * n + c] = sr[k][(ty + 1) * kHX + tx + 1];
    }
    // the sums that fall on the halo, for the neighbouring tiles' cells
    const size_t tile = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (t < kRing) {
        const int h = ring_cell(t);
#pragma unroll
        for (int k = 0; k < 4; ++k) a.ring[(tile * 4 + k) * kRing + t] = sr[k][h];
    }
    // the tile's share of each column's y0 adjoint (its rows in order; rows off the grid hold 0)
    if (t < kTX && i0 + t < a.K.nx) {
        double cs = sr[4][t];
#pragma unroll
        for (int r = 1; r < kTY; ++r) cs += sr[4][r * kTX + t];
        a.colb[(size_t)blockIdx.y * a.K.nx + i0 + t] = cs;
    }
}

// The y0 adjoint of column i, one wavefront per column: lane l adds the shares of tile rows l,
// l + 64, ... in order, then the lanes' sums are combined by a butterfly (every lane ends with the
// same total: a fixed order, deterministic); and the adjoint of the column's bottom height, its y0
// adjoint times dy0/dy_L (0 for a column without fluid cells).
constexpr int kColWaves = 4;
__global__ __launch_bounds__(64 * kColWaves) void adj_col_kernel(AdjArgs a)
{
    const int lane = (int)threadIdx.x & 63;
    const int i = (int)blockIdx.x * kColWaves + ((int)threadIdx.x >> 6);
    if (i >= a.K.nx) return;  // a whole wavefront
    const int nty = (a.K.ny + kTY - 1) / kTY;
    const GlobalD cb = (GlobalD)a.colb;
    double col = 0.0;
    for (int by = lane; by < nty; by += 64) col += cb[(size_t)by * a.K.nx + i];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) col += __shfl_xor(col, off);
    if (lane == 0) {
        a.colt[i] = col;
        if (a.gbot) a.gbot[i] = a.jb[i] < a.K.ny ? col * first_gap(a, i) : 0.0;
    }
}

__global__ __launch_bounds__(256) void adj_gather_kernel(AdjArgs a)
{
    const size_t n = (size_t)a.K.nx * a.K.ny;
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int i = (int)(c % a.K.nx), j = (int)(c / a.K.nx);
    double out[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = a.lam1[k * n + c];
    double add[4] = {0.0, 0.0, 0.0, 0.0};
    if (a.src) {
#pragma unroll
        for (int k = 0; k < 4; ++k) add[k] = a.src[k * n + c];
    }
    if (fluid_at(a, i, j)) {
        // the sums of the cell's own tile, then those the neighbouring tiles left on their halos
        // (left, right, below and its corners, above and its corners)
#pragma unroll
        for (int k = 0; k < 4; ++k) out[k] += a.own[k * n + c];
        const int ntx = (a.K.nx + kTX - 1) / kTX, nty = (a.K.ny + kTY - 1) / kTY;
        const int bx = i / kTX, tx = i % kTX, by = j / kTY, ty = j % kTY;
        const bool lf = tx == 0 && bx > 0, rt = tx == kTX - 1 && bx + 1 < ntx;
        auto take = [&](int tbx, int tby, int r) {
            const size_t tile = (size_t)tby * ntx + tbx;
#pragma unroll
            for (int k = 0; k < 4; ++k) out[k] += a.ring[(tile * 4 + k) * kRing + r];
        };
        if (lf) take(bx - 1, by, 2 * kHX + kTY + ty);
        if (rt) take(bx + 1, by, 2 * kHX + ty);
        if (ty == 0 && by > 0) {
            take(bx, by - 1, kHX + tx + 1);
            if (lf) take(bx - 1, by - 1, 2 * kHX - 1);
            if (rt) take(bx + 1, by - 1, kHX);
        }
        if (ty == kTY - 1 && by + 1 < nty) {
            take(bx, by + 1, tx + 1);
            if (lf) take(bx - 1, by + 1, kHX - 1);
            if (rt) take(bx + 1, by + 1, 0);
        }
        const double dy_eff = (a.dbot && j == a.jb[i]) ? a.K.dy - a.dbot[i] : a.K.dy;
        out[3] += dy_eff / (a.K.al - a.K.ag) * a.colt[i];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) a.lam[k * n + c] = out[k] + add[k];
}

}  // namespace bn

// Launch the passes on `stream`.  Scratch: bn_adjoint_scratch(nx, ny) doubles.
size_t bn_adjoint_scratch(int nx, int ny)
{
    const size_t ntx = (nx + bn::kTX - 1) / bn::kTX, nty = (ny + bn::kTY - 1) / bn::kTY;
    return 4 * (size_t)nx * ny + ntx * nty * 4 * bn::kRing + (size_t)nx * (nty + 1);
}

hipError_t bn_adjoint_launch(const bn::Consts &K, const double *q, const double *lam1, double *lam,
                             const uint8_t *solid, const int *jb, const double *dbot, const long long *Sp,
                             int nSp, double fix_inv, double dt, double *scratch, double *gbot, const double *src,
                             hipStream_t stream)
{
    bn::AdjArgs a;
    a.K = K;
    a.q = q;
    a.lam1 = lam1;
    a.lam = lam;
    a.solid = solid;
    a.jb = jb;
    a.dbot = dbot;
    a.gbot = gbot;
    a.src = src;
    a.Sp = Sp;
    a.nSp = nSp;
    a.fix_inv = fix_inv;
    a.dt = dt;
    a.dtdx = dt * K.inv_dx;
    a.dtdy = dt * K.inv_dy;
    const size_t n = (size_t)K.nx * K.ny;
    const size_t ntx = (K.nx + bn::kTX - 1) / bn::kTX, nty = (K.ny + bn::kTY - 1) / bn::kTY;
    a.own = scratch;
    a.ring = a.own + 4 * n;
    a.colb = a.ring + ntx * nty * 4 * bn::kRing;
    a.colt = a.colb + nty * K.nx;
    const unsigned gc = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(bn::adj_fused_kernel, dim3((unsigned)ntx, (unsigned)nty), dim3(bn::kThreads), 0, stream, a);
    hipLaunchKernelGGL(bn::adj_col_kernel, dim3((K.nx + bn::kColWaves - 1) / bn::kColWaves), dim3(64 * bn::kColWaves), 0,
                       stream, a);
    hipLaunchKernelGGL(bn::adj_gather_kernel, dim3(gc), dim3(256), 0, stream, a);
    return hipGetLastError();
}
