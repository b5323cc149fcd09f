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
// is reversed in five passes, one thread per cell, edge or column, through library-owned planes:
//   1. adj_rec_kernel     recompute Rec_c (the edge states the edges need), 21 planes
//   2. adj_edge_kernel    per x- and y-edge (one launch for both kinds): recompute D-+, reverse
//                         it with the adjoints of the two cells' updates, and write the adjoints
//                         of the edge states to their owners (each edge state feeds exactly one
//                         edge: no accumulation), 18 planes
//   3. adj_cell_kernel    reverse the reconstruction: adjoints of the 3 x 3 stencil (36 planes;
//                         a first-order cell reaches only itself and writes only that entry and a
//                         0 in the second-order flag plane) and of y0_i (1 plane)
//   4. adj_col_kernel     sum the y0 adjoints of each column, in blocks of kColRows rows (the
//                         gather adds the blocks' partial sums in order: deterministic)
//   5. adj_gather_kernel  lambda^n_c = lambda^{n+1}_c + the stencil adjoints of the (up to 9)
//                         fluid cells whose stencil holds c (of a first-order neighbour only
//                         c's own entry) + the detector's dy/(alpha_l -
//                         alpha_g) times its column's y0 adjoint (alpha only; (dy - d)/(alpha_l -
//                         alpha_g) in the first fluid cell of a column whose bottom lies d off the
//                         grid); solid cells pass lambda through (their state is copied and never
//                         read)
//                         and (if asked) the adjoint of each column's bottom height: its y0
//                         adjoint times dy0/dy_L = (alpha_l - alpha_first) / (alpha_l - alpha_g),
//                         written by the column's first fluid cell
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
    const long long *S;     // fixed-point free-surface integral of Q^n per column
    double fix_inv;
    double dt, dtdx, dtdy;
    double *rec;            // kRecPlanes planes
    double *fb;             // kFacePlanes planes
    double *wb;             // 36 planes (a first-order cell writes only its own entry, (1, 1))
    double *y0b;            // 1 plane (0 for solid cells)
    double *sob;            // 1 plane: 1 where the fluid cell's reconstruction is second order
    double *colb;           // [ceil(ny / kColRows)][nx] partial column sums
    double *gbot;           // [nx] adjoint of the bottom heights, or null
};

constexpr int kColRows = 32;

// plane layout of rec: qW 0-3, qE 4-7, qS 8-11, qN 12-15, e1S 16, e1N 17, aE 18, yS 19, yN 20
// (the heights of the S/N states: the edge's for a second-order cell, the centre's for a
// first-order one); fb: the adjoints of the first 18
constexpr int kRecPlanes = 21;
constexpr int kFacePlanes = 18;
enum : int { P_QW = 0, P_QE = 4, P_QS = 8, P_QN = 12, P_E1S = 16, P_E1N = 17, P_AE = 18, P_YS = 19, P_YN = 20 };

__device__ __forceinline__ bool fluid_at(const AdjArgs &a, int i, int j)
{
    if (i < 0 || i >= a.K.nx || j < 0 || j >= a.K.ny) return false;
    return !a.solid || a.solid[(size_t)j * a.K.nx + i] == 0;
}

__device__ __forceinline__ int flags_at(const AdjArgs &a, int i, int j)
{
    return cell_flags(i, j, a.K.nx, a.K.ny, a.K.bc, fluid_at(a, i, j));
}

// 1 - (alpha - alpha_g)/(alpha_l - alpha_g) of column i's first fluid cell (0 for a full cell)
__device__ __forceinline__ double first_gap(const AdjArgs &a, int i)
{
    const size_t n = (size_t)a.K.nx * a.K.ny;
    return (a.K.al - a.q[3 * n + (size_t)a.jb[i] * a.K.nx + i]) * a.K.inv_dal;
}

__device__ __forceinline__ double y0_of(const AdjArgs &a, int i)
{
    double v = (a.K.ylo + a.jb[i] * a.K.dy) + a.K.dy * ((double)a.S[i] * a.fix_inv);
    if (a.dbot && a.jb[i] < a.K.ny) v += a.dbot[i] * first_gap(a, i);
    return v;
}

// The 3 x 3 stencil of cell (i, j): states (outside the grid: the benign (1, 0, 0, 1), never used)
// and flags.
__device__ __forceinline__ void load_stencil(const AdjArgs &a, int i, int j, double (&wq)[3][3][4], int (&wf)[3][3])
{
    const size_t plane = (size_t)a.K.nx * a.K.ny;
#pragma unroll
    for (int dj = 0; dj < 3; ++dj)
#pragma unroll
        for (int di = 0; di < 3; ++di) {
            const int ii = i + di - 1, jj = j + dj - 1;
            const bool in = ii >= 0 && ii < a.K.nx && jj >= 0 && jj < a.K.ny;
            const size_t c = in ? (size_t)jj * a.K.nx + ii : 0;
            const double dflt[4] = {1.0, 0.0, 0.0, 1.0};
#pragma unroll
            for (int k = 0; k < 4; ++k) wq[dj][di][k] = in ? a.q[k * plane + c] : dflt[k];
            wf[dj][di] = flags_at(a, ii, jj);
        }
}

struct ArrayStencil {
    const double (*wq)[3][4];
    const int (*wf)[3];
    __device__ __forceinline__ double q(int dj, int di, int k) const { return wq[dj][di][k]; }
    __device__ __forceinline__ int f(int dj, int di) const { return wf[dj][di]; }
};

__global__ __launch_bounds__(256) void adj_rec_kernel(AdjArgs a)
{
    const size_t n = (size_t)a.K.nx * a.K.ny;
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int i = (int)(c % a.K.nx), j = (int)(c / a.K.nx);
    if (!fluid_at(a, i, j)) return;
    double wq[3][3][4];
    int wf[3][3];
    load_stencil(a, i, j, wq, wf);
    Rec r;
    ArrayStencil st{wq, wf};
    reconstruct(a.K, st, j, y0_of(a, i), a.dt, r);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        a.rec[(P_QW + k) * n + c] = r.qW[k];
        a.rec[(P_QE + k) * n + c] = r.qE[k];
        a.rec[(P_QS + k) * n + c] = r.qS[k];
        a.rec[(P_QN + k) * n + c] = r.qN[k];
    }
    a.rec[P_E1S * n + c] = r.e1S;
    a.rec[P_E1N * n + c] = r.e1N;
    a.rec[P_AE * n + c] = r.aE;
    a.rec[P_YS * n + c] = r.yS;
    a.rec[P_YN * n + c] = r.yN;
}

// x-edge e (between cells e-1 and e of row j), e = 0..nx; t = j (nx+1) + e.
__device__ __forceinline__ void adj_xedge(const AdjArgs &a, long long t)
{
    const int ne = a.K.nx + 1;
    if (t >= (long long)ne * a.K.ny) return;
    const int e = (int)(t % ne), j = (int)(t / ne);
    const int iL = e - 1, iR = e;
    const bool flL = fluid_at(a, iL, j), flR = fluid_at(a, iR, j);
    if (!flL && !flR) return;
    const int fL = flags_at(a, iL, j), fR = flags_at(a, iR, j);
    const size_t n = (size_t)a.K.nx * a.K.ny;
    const size_t cL = flL ? (size_t)j * a.K.nx + iL : 0, cR = flR ? (size_t)j * a.K.nx + iR : 0;
    double qEL[4], qWR[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        qEL[k] = flL ? a.rec[(P_QE + k) * n + cL] : 0.0;
        qWR[k] = flR ? a.rec[(P_QW + k) * n + cR] : 0.0;
    }
    // the edge's states: a missing side mirrors the other (normal momentum negated unless the
    // side is transmissive)
    const double sL = (!flL && !(fL & F_TX)) ? -1.0 : 1.0, sR = (!flR && !(fR & F_TX)) ? -1.0 : 1.0;
    double qm[4], qp[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        qm[k] = flL ? qEL[k] : qWR[k];
        qp[k] = flR ? qWR[k] : qEL[k];
    }
    qm[1] *= sL;
    qp[1] *= sR;
    double Dmb[4], Dpb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        Dmb[k] = flL ? -a.dtdx * a.lam1[k * n + cL] : 0.0;  // D- of this edge enters cell L (its D-_E)
        Dpb[k] = flR ? -a.dtdx * a.lam1[k * n + cR] : 0.0;  // D+ enters cell R (its D+_W)
    }
    double qmb[4] = {0, 0, 0, 0}, qpb[4] = {0, 0, 0, 0};
    edge_x_rev(a.K, qm, qp, Dmb, Dpb, qmb, qpb);
    qmb[1] *= sL;
    qpb[1] *= sR;
    if (flL) {
#pragma unroll
        for (int k = 0; k < 4; ++k) a.fb[(P_QE + k) * n + cL] = qmb[k] + (flR ? 0.0 : qpb[k]);
    }
    if (flR) {
#pragma unroll
        for (int k = 0; k < 4; ++k) a.fb[(P_QW + k) * n + cR] = qpb[k] + (flL ? 0.0 : qmb[k]);
    }
}

// y-edge e (between rows e-1 and e of column i), e = 0..ny; t = e nx + i.
__device__ __forceinline__ void adj_yedge(const AdjArgs &a, long long t)
{
    const int nx = a.K.nx;
    if (t >= (long long)nx * (a.K.ny + 1)) return;
    const int i = (int)(t % nx), e = (int)(t / nx);
    const int jB = e - 1, jT = e;
    const bool flB = fluid_at(a, i, jB), flT = fluid_at(a, i, jT);
    if (!flB && !flT) return;
    const int fB = flags_at(a, i, jB), fT = flags_at(a, i, jT);
    const size_t n = (size_t)nx * a.K.ny;
    const size_t cB = flB ? (size_t)jB * nx + i : 0, cT = flT ? (size_t)jT * nx + i : 0;
    double qNB[4], qST[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        qNB[k] = flB ? a.rec[(P_QN + k) * n + cB] : 0.0;
        qST[k] = flT ? a.rec[(P_QS + k) * n + cT] : 0.0;
    }
    const double e1NB = flB ? a.rec[P_E1N * n + cB] : 0.0, e1ST = flT ? a.rec[P_E1S * n + cT] : 0.0;
    const double aEB = flB ? a.rec[P_AE * n + cB] : 0.0, aET = flT ? a.rec[P_AE * n + cT] : 0.0;
    const double yN = flB ? a.rec[P_YN * n + cB] : 0.0, yS = flT ? a.rec[P_YS * n + cT] : 0.0;
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
    double Dmb[4], Dpb[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        Dmb[k] = flB ? -a.dtdy * a.lam1[k * n + cB] : 0.0;  // D- enters the cell below (its D-_N)
        Dpb[k] = flT ? -a.dtdy * a.lam1[k * n + cT] : 0.0;  // D+ enters the cell above (its D+_S)
    }
    double qmb[4] = {0, 0, 0, 0}, qpb[4] = {0, 0, 0, 0}, e1mb = 0.0, e1pb = 0.0;
    edge_y_rev(a.K, qm, e1m, aEm, ym, qp, e1p, aEp, yp, Dmb, Dpb, qmb, e1mb, qpb, e1pb);
    qmb[2] *= sB;
    qpb[2] *= sT;
    if (flB) {
#pragma unroll
        for (int k = 0; k < 4; ++k) a.fb[(P_QN + k) * n + cB] = qmb[k] + (flT ? 0.0 : qpb[k]);
        a.fb[P_E1N * n + cB] = e1mb + (flT ? 0.0 : e1pb);
    }
    if (flT) {
#pragma unroll
        for (int k = 0; k < 4; ++k) a.fb[(P_QS + k) * n + cT] = qpb[k] + (flB ? 0.0 : qmb[k]);
        a.fb[P_E1S * n + cT] = e1pb + (flB ? 0.0 : e1mb);
    }
}

// Both edge passes in one launch (they read the same reconstruction planes and write disjoint
// adjoint planes): the first nbx workgroups take the x-edges, the rest the y-edges, so that the two
// halves fill the GPU together instead of one after the other.
__global__ __launch_bounds__(64) void adj_edge_kernel(AdjArgs a, unsigned nbx)
{
    if (blockIdx.x < nbx)
        adj_xedge(a, (long long)blockIdx.x * blockDim.x + threadIdx.x);
    else
        adj_yedge(a, (long long)(blockIdx.x - nbx) * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(64) void adj_cell_kernel(AdjArgs a)
{
    const size_t n = (size_t)a.K.nx * a.K.ny;
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int i = (int)(c % a.K.nx), j = (int)(c / a.K.nx);
    if (!fluid_at(a, i, j)) {
        a.y0b[c] = 0.0;
        return;
    }
    double wq[3][3][4];
    int wf[3][3];
    load_stencil(a, i, j, wq, wf);
    // the reconstruction's second-order switch (as reconstruct_rev takes it): a first-order cell's
    // reverse reaches only the cell itself, so only that entry of its stencil adjoint is stored
    bool so = wq[1][1][3] > a.K.so_thr;
#pragma unroll
    for (int dj = 0; dj < 3; ++dj)
#pragma unroll
        for (int di = 0; di < 3; ++di)
            if ((wf[dj][di] & F_FLUID) && !(wq[dj][di][3] > a.K.so_thr)) so = false;
    RecBar rb;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        rb.qW[k] = a.fb[(P_QW + k) * n + c];
        rb.qE[k] = a.fb[(P_QE + k) * n + c];
        rb.qS[k] = a.fb[(P_QS + k) * n + c];
        rb.qN[k] = a.fb[(P_QN + k) * n + c];
        const double l = a.lam1[k * n + c];
        rb.fdiff[k] = -a.dtdx * l;
        rb.gdiff[k] = -a.dtdy * l;
    }
    rb.e1S = a.fb[P_E1S * n + c];
    rb.e1N = a.fb[P_E1N * n + c];
    rb.vol2 = -a.dt * a.lam1[2 * n + c];
    rb.vol3 = -a.dt * a.lam1[3 * n + c];
    double wqb[3][3][4];
#pragma unroll
    for (int dj = 0; dj < 3; ++dj)
#pragma unroll
        for (int di = 0; di < 3; ++di)
#pragma unroll
            for (int k = 0; k < 4; ++k) wqb[dj][di][k] = 0.0;
    const double yb = reconstruct_rev(a.K, wq, wf, j, y0_of(a, i), a.dt, rb, wqb);
    if (so) {
#pragma unroll
        for (int dj = 0; dj < 3; ++dj)
#pragma unroll
            for (int di = 0; di < 3; ++di)
#pragma unroll
                for (int k = 0; k < 4; ++k) a.wb[((dj * 3 + di) * 4 + k) * n + c] = wqb[dj][di][k];
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) a.wb[((1 * 3 + 1) * 4 + k) * n + c] = wqb[1][1][k];
    }
    a.sob[c] = so ? 1.0 : 0.0;
    a.y0b[c] = yb;
}

// partial sum of rows [kColRows y, kColRows (y+1)) of column i (grid: columns / 64 x row blocks)
__global__ __launch_bounds__(64) void adj_col_kernel(AdjArgs a)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= a.K.nx) return;
    const int j0 = (int)blockIdx.y * kColRows, j1 = min(a.K.ny, j0 + kColRows);
    double v[kColRows];
#pragma unroll
    for (int u = 0; u < kColRows; ++u) v[u] = j0 + u < j1 ? a.y0b[(size_t)(j0 + u) * a.K.nx + i] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kColRows; ++u) s += v[u];
    a.colb[(size_t)blockIdx.y * a.K.nx + i] = s;
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
    if (fluid_at(a, i, j)) {
        // stencil entry (dj, di) of the cell (i - di + 1, j - dj + 1) is this cell
#pragma unroll
        for (int dj = 0; dj < 3; ++dj)
#pragma unroll
            for (int di = 0; di < 3; ++di) {
                const int ii = i - di + 1, jj = j - dj + 1;
                if (!fluid_at(a, ii, jj)) continue;
                const size_t m = (size_t)jj * a.K.nx + ii;
                // a first-order cell stored only its own entry
                if (!(dj == 1 && di == 1) && !(a.sob[m] != 0.0)) continue;
#pragma unroll
                for (int k = 0; k < 4; ++k) out[k] += a.wb[((dj * 3 + di) * 4 + k) * n + m];
            }
        double col = 0.0;
        for (int y = 0; y * kColRows < a.K.ny; ++y) col += a.colb[(size_t)y * a.K.nx + i];
        const double dy_eff = (a.dbot && j == a.jb[i]) ? a.K.dy - a.dbot[i] : a.K.dy;
        out[3] += dy_eff / (a.K.al - a.K.ag) * col;
        // the column's bottom height reaches the step through its free surface only:
        // dy0/dy_L = 1 - a of the first fluid cell (written by that cell's thread)
        if (a.gbot && j == a.jb[i]) a.gbot[i] = col * first_gap(a, i);
    } else if (a.gbot && j == a.K.ny - 1 && a.jb[i] == a.K.ny) {
        a.gbot[i] = 0.0;  // a column without fluid cells
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) a.lam[k * n + c] = out[k];
}

}  // namespace bn

// Launch the passes on `stream`.  Scratch: bn_adjoint_scratch(nx, ny) doubles.
namespace bn {
constexpr int kAdjPlanes = kRecPlanes + kFacePlanes + 36 + 2;
}

size_t bn_adjoint_scratch(int nx, int ny)
{
    return (size_t)bn::kAdjPlanes * nx * ny + (size_t)nx * ((ny + bn::kColRows - 1) / bn::kColRows);
}

hipError_t bn_adjoint_launch(const bn::Consts &K, const double *q, const double *lam1, double *lam,
                             const uint8_t *solid, const int *jb, const double *dbot, const long long *S,
                             double fix_inv, double dt, double *scratch, double *gbot, hipStream_t stream)
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
    a.S = S;
    a.fix_inv = fix_inv;
    a.dt = dt;
    a.dtdx = dt * K.inv_dx;
    a.dtdy = dt * K.inv_dy;
    const size_t n = (size_t)K.nx * K.ny;
    a.rec = scratch;
    a.fb = a.rec + bn::kRecPlanes * n;
    a.wb = a.fb + bn::kFacePlanes * n;
    a.y0b = a.wb + 36 * n;
    a.sob = a.y0b + n;
    a.colb = a.sob + n;
    const unsigned gc = (unsigned)((n + 255) / 256), gc64 = (unsigned)((n + 63) / 64);
    hipLaunchKernelGGL(bn::adj_rec_kernel, dim3(gc), dim3(256), 0, stream, a);
    const size_t nxe = (size_t)(K.nx + 1) * K.ny, nye = (size_t)K.nx * (K.ny + 1);
    const unsigned nbx = (unsigned)((nxe + 63) / 64), nby = (unsigned)((nye + 63) / 64);
    hipLaunchKernelGGL(bn::adj_edge_kernel, dim3(nbx + nby), dim3(64), 0, stream, a, nbx);
    hipLaunchKernelGGL(bn::adj_cell_kernel, dim3(gc64), dim3(64), 0, stream, a);
    hipLaunchKernelGGL(bn::adj_col_kernel, dim3((K.nx + 63) / 64, (K.ny + bn::kColRows - 1) / bn::kColRows), dim3(64),
                       0, stream, a);
    hipLaunchKernelGGL(bn::adj_gather_kernel, dim3(gc), dim3(256), 0, stream, a);
    return hipGetLastError();
}
