// Algorithmic FLOP count of one explicit step on a given state (measurement tool for the roofline).
//
// The device physics of bn2d_physics.h is compiled here on the host with a scalar type that counts
// every +, -, *, /, sqrt and exp (1 each; an FMA in the kernel is a * and a + here; fabs, fmin,
// fmax, negation, comparisons and selects are free).  The step is then walked over the grid the
// way the kernel walks it, but without the kernel's redundant halo work: one reconstruction per
// fluid cell, one solve per x- and y-edge with a fluid side, one update and one detector/CFL term
// per fluid cell.  Loop-invariant constants (products of grid and model constants) are not
// counted.  Rows are walked in parallel (OpenMP), each thread counting its own; the counts are sums
// of integers, so they do not depend on the thread count.  Build: g++ -O2 -std=c++17 -fopenmp -fPIC -shared.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace bn {
struct Counted;
}
typedef bn::Counted real_t;
#define BN2D_HOST_COUNT 1

namespace bn {
static thread_local unsigned long long g_ops = 0;  // per thread: rows are counted in parallel
struct Counted {
    double v;
    Counted() : v(0.0) {}
    Counted(double x) : v(x) {}
};
inline Counted operator+(Counted a, Counted b) { ++g_ops; return Counted(a.v + b.v); }
inline Counted operator-(Counted a, Counted b) { ++g_ops; return Counted(a.v - b.v); }
inline Counted operator*(Counted a, Counted b) { ++g_ops; return Counted(a.v * b.v); }
inline Counted operator/(Counted a, Counted b) { ++g_ops; return Counted(a.v / b.v); }
inline Counted operator-(Counted a) { return Counted(-a.v); }
inline Counted &operator+=(Counted &a, Counted b) { a = a + b; return a; }
inline bool operator>(Counted a, Counted b) { return a.v > b.v; }
inline bool operator<(Counted a, Counted b) { return a.v < b.v; }
inline bool operator!=(Counted a, Counted b) { return a.v != b.v; }
inline bool operator==(Counted a, Counted b) { return a.v == b.v; }
inline Counted fabs(Counted a) { return Counted(std::fabs(a.v)); }
inline Counted fmin(Counted a, Counted b) { return Counted(std::fmin(a.v, b.v)); }
inline Counted fmax(Counted a, Counted b) { return Counted(std::fmax(a.v, b.v)); }
inline Counted exp(Counted a) { ++g_ops; return Counted(std::exp(a.v)); }
inline Counted sqrt(Counted a) { ++g_ops; return Counted(std::sqrt(a.v)); }
inline bool isfinite(Counted a) { return std::isfinite(a.v); }
}  // namespace bn

#include "bn2d_physics.h"

using namespace bn;

namespace {

Consts make_consts(int nx, int ny, double x0, double x1, double y0, double y1, double g, double k0, double rho0,
                   double al, double ag, double cfl, const int32_t *bc)
{
    Consts K;
    std::memset(&K, 0, sizeof(K));
    K.nx = nx; K.ny = ny;
    K.dx = (x1 - x0) / nx; K.dy = (y1 - y0) / ny; K.ylo = y0;
    K.g = g; K.k0 = k0; K.rho0 = rho0; K.al = al; K.ag = ag; K.cfl = cfl;
    for (int s = 0; s < 4; ++s) K.bc[s] = bc[s];
    K.c2 = k0 / rho0; K.c = std::sqrt(K.c2); K.inv_c2 = 1.0 / K.c2; K.inv2c = 0.5 / K.c; K.half_rho0 = 0.5 * rho0;
    K.a = g * rho0 / k0;
    K.e_up1 = std::exp(-K.a * K.dy); K.e_dn1 = std::exp(K.a * K.dy);
    K.e_uph = std::exp(-K.a * 0.5 * K.dy); K.e_dnh = std::exp(K.a * 0.5 * K.dy);
    K.so_thr = 10.0 * ag;
    K.inv_dx = 1.0 / K.dx; K.inv_dy = 1.0 / K.dy; K.inv2dx = 1.0 / (2.0 * K.dx); K.inv2dy = 1.0 / (2.0 * K.dy);
    K.inv_rho0 = 1.0 / rho0;
    K.inv_dal = 1.0 / (al - ag);
    return K;
}

struct ArrayStencil {
    static constexpr bool kRingFlags = false;
    const real_t (*wq)[3][4];
    const int (*wf)[3];
    real_t q(int dj, int di, int k) const { return wq[dj][di][k]; }
    int f(int dj, int di) const { return wf[dj][di]; }
};

}  // namespace

extern "C" int bn2d_count_flops(int nx, int ny, double x0, double x1, double y0, double y1, double g, double k0,
                                double rho0, double al, double ag, double cfl, const int32_t *bc,
                                const uint8_t *solid, const double *Q, const double *Y0, double dt,
                                unsigned long long *out /* [6]: recon, x-edges, y-edges, update, reductions, cells */)
{
    const Consts K = make_consts(nx, ny, x0, x1, y0, y1, g, k0, rho0, al, ag, cfl, bc);
    const size_t plane = (size_t)nx * ny;
    auto fluid = [&](int i, int j) {
        return i >= 0 && i < nx && j >= 0 && j < ny && (!solid || solid[(size_t)j * nx + i] == 0);
    };
    auto flags = [&](int i, int j) { return cell_flags(i, j, nx, ny, bc, fluid(i, j)); };
    std::vector<Rec> rec(plane);
    unsigned long long c_rec = 0, c_x = 0, c_y = 0, c_upd = 0, c_red = 0, cells = 0;

#pragma omp parallel for schedule(dynamic, 4) reduction(+ : c_rec)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (!fluid(i, j)) continue;
            real_t wq[3][3][4];
            int wf[3][3];
            for (int dj = 0; dj < 3; ++dj)
                for (int di = 0; di < 3; ++di) {
                    const int ii = i + di - 1, jj = j + dj - 1;
                    wf[dj][di] = flags(ii, jj);
                    for (int k = 0; k < 4; ++k)
                        wq[dj][di][k] = (ii >= 0 && ii < nx && jj >= 0 && jj < ny)
                                            ? Q[k * plane + (size_t)jj * nx + ii] : (k == 0 || k == 3 ? 1.0 : 0.0);
                }
            g_ops = 0;
            ArrayStencil st{wq, wf};
            reconstruct(K, st, j, real_t(Y0[i]), real_t(dt), rec[(size_t)j * nx + i]);
            c_rec += g_ops;
        }

    std::vector<real_t> DpW(4 * plane), DmE(4 * plane), DpS(4 * plane), DmN(4 * plane);
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : c_x)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            const bool lf = fluid(i - 1, j), rf = fluid(i, j);
            if (!lf && !rf) continue;
            real_t qm[4], qp[4], Dm[4], Dp[4];
            const Rec *L = lf ? &rec[(size_t)j * nx + i - 1] : nullptr, *R = rf ? &rec[(size_t)j * nx + i] : nullptr;
            for (int k = 0; k < 4; ++k) {
                qm[k] = lf ? L->qE[k] : R->qW[k];
                qp[k] = rf ? R->qW[k] : L->qE[k];
            }
            if (!lf && !(i == 0 && K.bc[0] == 1)) qm[1] = -qm[1];
            if (!rf && !(i == nx && K.bc[1] == 1)) qp[1] = -qp[1];
            g_ops = 0;
            edge_x(K, qm, qp, Dm, Dp);
            c_x += g_ops;
            for (int k = 0; k < 4; ++k) {
                if (lf) DmE[k * plane + (size_t)j * nx + i - 1] = Dm[k];
                if (rf) DpW[k * plane + (size_t)j * nx + i] = Dp[k];
            }
        }
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : c_y)
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const bool bf = fluid(i, j - 1), tf = fluid(i, j);
            if (!bf && !tf) continue;
            const Rec *B = bf ? &rec[(size_t)(j - 1) * nx + i] : nullptr, *T = tf ? &rec[(size_t)j * nx + i] : nullptr;
            real_t qm[4], qp[4], Dm[4], Dp[4];
            for (int k = 0; k < 4; ++k) {
                qm[k] = bf ? B->qN[k] : T->qS[k];
                qp[k] = tf ? T->qS[k] : B->qN[k];
            }
            real_t e1m = bf ? B->e1N : T->e1S, aEm = bf ? B->aE : T->aE, ym = bf ? B->yN : T->yS;
            real_t e1p = tf ? T->e1S : B->e1N, aEp = tf ? T->aE : B->aE, yp = tf ? T->yS : B->yN;
            if (!bf && !(j == 0 && K.bc[2] == 1)) qm[2] = -qm[2];
            if (!tf && !(j == ny && K.bc[3] == 1)) qp[2] = -qp[2];
            g_ops = 0;
            edge_y(K, qm, e1m, aEm, ym, qp, e1p, aEp, yp, Dm, Dp);
            c_y += g_ops;
            for (int k = 0; k < 4; ++k) {
                if (bf) DmN[k * plane + (size_t)(j - 1) * nx + i] = Dm[k];
                if (tf) DpS[k * plane + (size_t)j * nx + i] = Dp[k];
            }
        }
    const real_t dtv(dt), dtdx(dt / K.dx), dtdy(dt / K.dy);
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : c_upd, c_red, cells)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (!fluid(i, j)) continue;
            const size_t c = (size_t)j * nx + i;
            real_t qn[4], P[4], dpw[4], dme[4], dps[4], dmn[4], q[4];
            for (int k = 0; k < 4; ++k) {
                qn[k] = Q[k * plane + c];
                dpw[k] = DpW[k * plane + c]; dme[k] = DmE[k * plane + c];
                dps[k] = DpS[k * plane + c]; dmn[k] = DmN[k * plane + c];
            }
            g_ops = 0;
            update_partial(qn, dpw, dme, rec[c].fdiff, rec[c].gdiff, rec[c].vol2, rec[c].vol3, dtv, dtdx, dtdy, P);
            update_south(P, dps, dtdy, P);
            update_finish(P, dmn, dtdy, q);
            c_upd += g_ops;
            g_ops = 0;
            (void)detector_term(K, q);
            (void)cfl_rate(K, q);
            c_red += g_ops;
            ++cells;
        }
    out[0] = c_rec; out[1] = c_x; out[2] = c_y; out[3] = c_upd; out[4] = c_red; out[5] = cells;
    return 0;
}
