// Fused explicit step of the well-balanced Osher-Romberg scheme (Gaburro, Castro, Dumbser,
// arXiv:1806.04960, Sec. 3) for gfx950, FP64 on the vector ALUs.
//
// Batch.  One launch advances every member of a batch of grids (any sizes, parameters and
// masks; a single grid is a batch of one) by one step, each with its own time step.  The members'
// column strips are concatenated into one list of strips that the scheduling below distributes.
//
// Marching.  A wavefront (64 lanes) works on a strip of 64 columns, lane L holding column
// 60 s - 2 + L of strip s, and marches upwards through a range of rows.  Per row it loads one row
// of the state (coalesced, 8 bytes per lane and plane, prefetched one row ahead), keeps the last
// three rows in an LDS ring, reconstructs the row below the newest one, solves every x-edge of that
// row and the y-edge below it exactly once, and finishes the row below that: the edge
// fluctuations a cell needs come from its own lane or the adjacent lane, so nothing but the state
// crosses HBM.  Lanes 2..61 produce output; lanes 0, 1, 62, 63 are the column halo (1 and 62
// reconstruct).  A range that starts at row j0 first reconstructs row j0 - 1 (halo below) and
// ends by reconstructing the row above its last one (halo above).
//
// Scheduling.  The launch is persistent: as many wavefronts as the device holds at once (two per
// SIMD at this kernel's register use).  Every marched range records its duration per row; the
// next step cuts the strips into one range per wavefront of equal
// recorded cost (second-order liquid rows cost about 1.5x first-order gas rows, rows across the
// free surface more), so that all wavefronts finish together as long as the flow changes little
// from one step to the next; a wavefront whose share crosses into the next strip also owns that
// strip's head, which it marches second.  A wavefront
// claims B rows of its range at a time with an atomic add on the range's descriptor, issued a
// row ahead so that the claim does not stall the march, and keeps marching through consecutive
// claims without repeating the halo.  When its range is exhausted it takes an unowned range or
// splits a range still being marched, taking its upper half (one compare-and-swap on the
// descriptor), which absorbs what the recorded costs did not predict.  The partition depends on
// timing, the results do not: every cell is computed by the same arithmetic whoever marches it.
// No wavefront ever waits for another.
//
// Reductions.  The free-surface integral of the next step (Sec. 3.5) is accumulated per column in
// 64-bit fixed point with atomic adds, which makes it independent of the order in which rows are
// processed and so of the schedule; the CFL rate is folded into a 64-bit atomic max, which the
// next step turns into its dt.  Nothing at the end of a step waits for other wavefronts: every
// result that crosses wavefronts is an atomic, read by the next launch.  The fixed-point
// integrals, the CFL maxima and the per-strip cost totals are triple-buffered (read, accumulate,
// clear for the next step); the per-row costs and the range lists are double-buffered, each step
// clearing the next step's list.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bn2d_layout.h"

namespace bn {

// Members and the Control are read through an address the compiler must treat as new at every use
// site (an empty asm that "modifies" it), so their scalar loads are repeated where needed instead
// of being held in scalar registers across the march.
typedef const __attribute__((address_space(4))) Member *MemberPtr;
typedef const __attribute__((address_space(4))) Control *ControlPtr;
__device__ __forceinline__ const Member &member_at(unsigned long long base, int b)
{
    // b is the same in every lane (the compiler cannot always see it): take lane 0's
    unsigned long long addr = base + (unsigned long long)__builtin_amdgcn_readfirstlane(b) * sizeof(Member);
    asm volatile("" : "+s"(addr));
    return *(const Member *)(MemberPtr)addr;
}
// The same for a member whose record address was computed once (a march keeps it instead of the
// array base and the index: two scalar registers fewer to spill and restore in its row loop).
__device__ __forceinline__ const Member &member_ref(unsigned long long addr)
{
    asm volatile("" : "+s"(addr));
    return *(const Member *)(MemberPtr)addr;
}
__device__ __forceinline__ const Control &control_at(unsigned long long addr)
{
    asm volatile("" : "+s"(addr));
    return *(const Control *)(ControlPtr)addr;
}

// Range descriptor: one 64-bit word, [63] owned, [62:48] strip, [47:24] end row (exclusive),
// [23:0] next unclaimed row.  The owner claims with an atomic add of B; a thief lowers the end.
constexpr unsigned long long kOwned = 1ull << 63;

__host__ __device__ inline int d_cur(unsigned long long d) { return (int)(d & 0xFFFFFFull); }
__host__ __device__ inline int d_end(unsigned long long d) { return (int)((d >> 24) & 0xFFFFFFull); }
__host__ __device__ inline int d_strip(unsigned long long d) { return (int)((d >> 48) & 0x7FFFull); }
__host__ __device__ inline unsigned long long d_make(bool owned, int strip, int end, int cur)
{
    return (owned ? kOwned : 0ull) | ((unsigned long long)strip << 48) | ((unsigned long long)end << 24) |
           (unsigned long long)cur;
}

__device__ __forceinline__ unsigned long long load_word(unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Neighbour lanes through DPP whole-wavefront shifts (a VALU move, no LDS round trip): lane L
// receives lane L-1 (from_left) or L+1 (from_right); the end lanes keep their own value (they are
// halo lanes whose results are discarded).
__device__ __forceinline__ int shfl_from_left(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xF, 0xF, false); }
__device__ __forceinline__ int shfl_from_right(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x130, 0xF, 0xF, false); }
__device__ __forceinline__ double shfl_from_left(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = shfl_from_left((int)(b & 0xFFFFFFFFll)), hi = shfl_from_left((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double shfl_from_right(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = shfl_from_right((int)(b & 0xFFFFFFFFll)), hi = shfl_from_right((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// v from a lane src that is the same in every lane: scalar reads of its halves, no LDS round trip
__device__ __forceinline__ double lane_value(double v, int src)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ int lane_value(int v, int src) { return __builtin_amdgcn_readlane(v, src); }

// A DPP move of both halves of v (lanes the pattern does not reach, or rows outside row_mask, get 0).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_or_zero(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xFFFFFFFFll), kCtrl, kRowMask, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, kRowMask, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Inclusive prefix sum over the wavefront by DPP (a fixed order of additions, the same in every
// wavefront): within each row of 16 lanes by shifts of 1, 2, 4 and 8, then lane 15 of rows 0 and 2
// added to rows 1 and 3, then lane 31 to rows 2 and 3.
__device__ __forceinline__ double wave_incl_scan(double v)
{
    v += dpp_or_zero<0x111, 0xF>(v);  // row_shr:1
    v += dpp_or_zero<0x112, 0xF>(v);  // row_shr:2
    v += dpp_or_zero<0x114, 0xF>(v);  // row_shr:4
    v += dpp_or_zero<0x118, 0xF>(v);  // row_shr:8
    v += dpp_or_zero<0x142, 0xA>(v);  // row_bcast:15
    v += dpp_or_zero<0x143, 0xC>(v);  // row_bcast:31
    return v;
}

// Prefix sums of v[0..n) spread over the wavefront: lane l holds the contiguous entries
// [l m, (l+1) m), m = ceil(n / 64), their sum, and (one wave scan) the sums before and through
// them.  find(t) returns the index i with v[0] + ... + v[i-1] <= t < v[0] + ... + v[i] (n if there
// is none) and t minus that lower bound.  Every wavefront computing the same target on the same
// data gets the same answer (the summation order is fixed).  Up to kHeld entries per lane are kept
// in registers, so that finding needs no further loads; longer lists are walked again from memory.
template <class T>
struct Chunks {
    static constexpr int kHeld = 16;
    const T *v;
    int n, m, b, e;
    double vv[kHeld];
    double excl, incl, total;

    __device__ void load(const T *v_, int n_)
    {
        const int lane = threadIdx.x;
        v = v_;
        n = n_;
        m = (n + 63) / 64;
        b = min(lane * m, n);
        e = min(b + m, n);
        double sum = 0.0;
        // loads 16 at a time from clamped addresses (no branch, one wait per batch)
#pragma unroll
        for (int u = 0; u < kHeld; ++u) {
            const double x = (double)v[min(b + u, n - 1)];
            vv[u] = b + u < e ? x : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kHeld; ++u) sum += vv[u];
        if (sizeof(T) == sizeof(float) && m > kHeld && m <= 64) {
            // up to 64 single-precision entries a lane: the rest in one more round of loads, summed
            // in the same order
            T w[64 - kHeld];
#pragma unroll
            for (int u = 0; u < 64 - kHeld; ++u) w[u] = v[min(b + kHeld + u, n - 1)];
#pragma unroll
            for (int u = 0; u < 64 - kHeld; ++u) sum += b + kHeld + u < e ? (double)w[u] : 0.0;
        } else {
            for (int c = b + kHeld; c < e; c += 16) {
                double w[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const double x = (double)v[min(c + u, n - 1)];
                    w[u] = c + u < e ? x : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) sum += w[u];
            }
        }
        incl = wave_incl_scan(sum);
        excl = incl - sum;
        total = lane_value(incl, 63);
    }

    __device__ void find(double t, int &idx, double &off) const
    {
        const int lane = threadIdx.x;
        idx = n;
        off = 0.0;
        const unsigned long long mask = __ballot(b < e && excl <= t && t < incl);
        if (!mask) return;
        const int l = __ffsll((long long)mask) - 1;
        int found;
        double rem;
        if (m <= kHeld) {
            // every lane walks its own entries; lane l's answer is the one
            found = e - 1;
            rem = 0.0;
            double acc = excl;
            bool done = false;
#pragma unroll
            for (int u = 0; u < kHeld; ++u) {
                const double next = acc + vv[u];
                if (!done && b + u < e && t < next) {
                    found = b + u;
                    rem = t - acc;
                    done = true;
                }
                acc = next;
            }
            found = lane_value(found, l);
            rem = lane_value(rem, l);
        } else {
            // the wavefront walks lane l's entries 64 at a time
            const int lb = lane_value(b, l), le = lane_value(e, l);
            double acc = lane_value(excl, l);
            found = le - 1;
            rem = 0.0;
            for (int c = lb; c < le; c += 64) {
                const bool in = c + lane < le;
                const double x = in ? (double)v[c + lane] : 0.0;
                const double si = wave_incl_scan(x);
                const unsigned long long hit = __ballot(in && t < acc + si);
                if (hit) {
                    const int u = __ffsll((long long)hit) - 1;
                    found = c + u;
                    rem = t - (acc + lane_value(si - x, u));
                    break;
                }
                acc += lane_value(si, 63);
            }
        }
        idx = found;
        off = rem;
    }
};

// Stencil accessor over the LDS ring: rows s[0..2] (below, centre, above), lane offsets -1..1.
struct LdsStencil {
    static constexpr bool kRingFlags = true;
    const double (*sq)[4][64];
    const int (*sf)[64];
    int s[3];
    int lane;
    __device__ __forceinline__ double q(int dj, int di, int k) const { return sq[s[dj]][k][lane + di - 1]; }
    __device__ __forceinline__ int f(int dj, int di) const { return sf[s[dj]][lane + di - 1]; }
};

// The time step of member b for this launch.
__device__ double member_dt(const StepArgs &a, unsigned long long ma, int b)
{
    if (!a.cfl_dt) return a.dt_arg;
    const Member &M = member_at(ma, b);
    const double lmax = __longlong_as_double((long long)*M.lam[a.m3]);
    return (lmax > 0.0 && isfinite(lmax)) ? M.K.cfl / lmax : 0.0;
}

// March global strip g (member b, its strip `strip`) upwards from row j0, rows [j0, E) already
// claimed, claiming further rows through descriptor `slot` (none if slot < 0) until a claim fails.
__device__ void march(const StepArgs &a, unsigned long long ma, unsigned long long ca, double (*sq)[4][64],
                      int (*sf)[64], int b, int g, int strip, int j0, int E, int slot)
{
    const int lane = threadIdx.x;
    const unsigned long long mab = ma + (unsigned long long)__builtin_amdgcn_readfirstlane(b) * sizeof(Member);
    int nx, ny;
    const double *Qp;
    double *Qnp;
    const uint8_t *solid;
    {
        const Member &M = member_ref(mab);
        nx = M.K.nx;
        ny = M.K.ny;
        Qp = M.q[a.cur];
        Qnp = M.q[1 - a.cur];
        solid = M.solid;
    }
    const double dt = member_dt(a, ma, b);
    double dtdx, dtdy;
    {
        const Consts &K = member_ref(mab).K;
        dtdx = dt * K.inv_dx;
        dtdy = dt * K.inv_dy;
    }
    double lam = 0.0;
    int bad = 0;
    const int i = strip * 60 - 2 + lane;
    const bool colin = i >= 0 && i < nx;
    const bool out_lane = colin && lane >= 2 && lane < 62;
    const bool rec_lane = lane >= 1 && lane <= 62;
    const size_t plane = (size_t)nx * ny;
    const int fcol = cell_flags(i, 0, nx, 1, member_ref(mab).K.bc, false);
    double y0c = 0.0;
    if (colin) {
        const Member &M = member_ref(mab);
        const int jbi = M.jb[i];
        y0c = (M.K.ylo + jbi * M.K.dy) + M.K.dy * ((double)M.S[a.m3][i] * M.fix_inv);
        // a bottom off the grid (Sec. 3.5): the first fluid cell stands for the interval from the
        // bottom to its top edge; its offset counts where that cell is not liquid
        if (M.dbot && jbi < ny) y0c += M.dbot[i] * ((M.K.al - Qp[3 * plane + (size_t)jbi * nx + i]) * M.K.inv_dal);
    }
    unsigned long long *desc = slot >= 0 ? control_at(ca).desc + slot : nullptr;
    bool outstanding = false, last = slot < 0;
    const long long t_begin = clock64();
    unsigned long long claim = 0;
    // the least cost to record a row at (loaded now: at the range's end the recording would wait
    // for it)
    const double floor_cost = a.cost_floor > 0.0 ? a.cost_floor * (control_at(ca).Ts_in[g] / ny) : 0.0;

    // pending row (below the row being reconstructed): its update with every term but its north
    // edge's D-, and its north edge state
    double pX[4] = {0, 0, 0, 0};
    double nQ[4] = {1, 0, 0, 1}, nE1 = 1.0, nAE = 1.0, nY = 0.0;
    int nF = 0;
    long long colfix = 0;

    // row prefetch (through a global-memory pointer: a generic one makes flat loads, which count
    // against the same wait counter as scalar and LDS loads, so that the next wait for a constant
    // would also wait for the row)
    typedef const __attribute__((address_space(1))) double *GlobalRow;
    const GlobalRow Qg = (GlobalRow)Qp;
    double lq[4];
    int ls = 0;  // the row's mask byte, turned into cell flags only when the row is stored (a use
                 // right after the load would wait for it, and for every store still in flight)
    // (the address is clamped into the grid and the value replaced outside it, so that the load
    // needs no branch)
    auto load_row = [&](int r) {
        const bool in = colin && r >= 0 && r < ny;
        const size_t cidx = (size_t)min(max(r, 0), ny - 1) * nx + min(max(i, 0), nx - 1);
        if (solid) ls = solid[cidx];
        const double dflt[4] = {1.0, 0.0, 0.0, 1.0};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double v = Qg[k * plane + cidx];
            lq[k] = in ? v : dflt[k];
        }
    };
    load_row(j0 - 2);

    int s_hi = 2;  // ring slot that receives row r
    for (int r = j0 - 2;; ++r) {
        // the claim of the rows from E on is resolved when row E is about to be reconstructed,
        // and the next claim goes out a row before it is needed
        if (outstanding && r == E + 1) {
            const unsigned long long c = __shfl(claim, 0, 64);
            outstanding = false;
            if (d_cur(c) < d_end(c)) E = min(E + a.B, d_end(c));  // d_cur(c) == E: only the owner advances it
            else last = true;
        }
        if (!last && !outstanding && r >= E - 1) {
            if (lane == 0) claim = atomicAdd(desc, (unsigned long long)a.B);
            outstanding = true;
        }
        const bool final_row = last && r == E + 1;

        s_hi = (s_hi == 2) ? 0 : s_hi + 1;
        const int s_mid = (s_hi == 0) ? 2 : s_hi - 1;
        const int s_lo = (s_mid == 0) ? 2 : s_mid - 1;
        __syncthreads();  // the slot about to be overwritten is no longer read
#pragma unroll
        for (int k = 0; k < 4; ++k) sq[s_hi][k][lane] = lq[k];
        // (a cell's flags are its column's, fixed for the march, and its row's, the same in every
        // lane; and its low-alpha or mirror bits)
        {
            const Consts &K = member_ref(mab).K;
            const bool fluid = colin && r >= 0 && r < ny && ls == 0;
            const int f = fcol | cell_flags(0, r, 1, ny, K.bc, fluid);
            sf[s_hi][lane] = f | (fluid ? (lq[3] > K.so_thr ? 0 : F_LOWA) : mirror_bits(f));
        }
        if (!final_row) load_row(r + 1);
        __syncthreads();
        if (r < j0) continue;

        // ---- reconstruct row jr = r - 1 ----------------------------------------------------
        const int jr = r - 1;
        const int fc_mid = sf[s_mid][lane];
        const bool fl = rec_lane && (fc_mid & F_FLUID);
        Rec rc;
        if (fl) {
            const Consts &K = member_ref(mab).K;
            LdsStencil st{sq, sf, {s_lo, s_mid, s_hi}, lane};
            reconstruct(K, st, jr, y0c, dt, rc);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double v = sq[s_mid][k][lane];
                rc.qW[k] = v; rc.qE[k] = v; rc.qS[k] = v; rc.qN[k] = v;
                rc.fdiff[k] = 0.0; rc.gdiff[k] = 0.0;
            }
            rc.e1S = 1.0; rc.e1N = 1.0; rc.aE = 1.0; rc.yS = 0.0; rc.yN = 0.0; rc.vol2 = 0.0; rc.vol3 = 0.0;
        }
        const bool jr_inside = jr >= j0 && jr < E;

        // ---- x-edges of row jr: lane L solves the edge between columns L and L+1, then every
        // term of the update of row jr except those of its two y-edges.  Lanes whose edge or
        // cell is not needed compute on benign copies and discard the result. -----------------
        double X[4] = {0, 0, 0, 0};
        if (jr_inside) {
            const Consts &K = member_ref(mab).K;
            double qWr[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) qWr[k] = shfl_from_right(rc.qW[k]);
            const int fR = shfl_from_right(fc_mid);
            const bool rf = (lane <= 61) && (fR & F_FLUID);
            double qm[4], qp[4], Dm[4], Dp[4];
            // (every reconstructing lane fluid, the usual case: no mirror states, a uniform branch)
            if (all_lanes(!rec_lane || fl)) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    qm[k] = rc.qE[k];
                    qp[k] = qWr[k];
                }
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    qm[k] = fl ? rc.qE[k] : qWr[k];
                    qp[k] = rf ? qWr[k] : rc.qE[k];
                }
                // wall: mirror state with negated normal momentum, or a copy on a transmissive side
                if (!fl && !(fc_mid & F_TX)) qm[1] = -qm[1];
                if (!rf && !(fR & F_TX)) qp[1] = -qp[1];
            }
            edge_x(K, qm, qp, Dm, Dp);
            double DpW[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) DpW[k] = shfl_from_left(Dp[k]);
            const double Qm[4] = {sq[s_mid][0][lane], sq[s_mid][1][lane], sq[s_mid][2][lane], sq[s_mid][3][lane]};
            update_partial(Qm, DpW, Dm, rc.fdiff, rc.gdiff, rc.vol2, rc.vol3, dt, dtdx, dtdy, X);
        }

        // ---- y-edge between row jr-1 (pending north state) and row jr ----------------------
        double DyM[4] = {0, 0, 0, 0}, DyP[4] = {0, 0, 0, 0};
        if (r > j0) {
            const Consts &K = member_ref(mab).K;
            const bool bf = rec_lane && (nF & F_FLUID);
            double qm[4], qp[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                qm[k] = bf ? nQ[k] : rc.qS[k];
                qp[k] = fl ? rc.qS[k] : nQ[k];
            }
            const double e1m = bf ? nE1 : rc.e1S, aEm = bf ? nAE : rc.aE, ym = bf ? nY : rc.yS;
            const double e1p = fl ? rc.e1S : nE1, aEp = fl ? rc.aE : nAE, yp = fl ? rc.yS : nY;
            if (!bf && !(nF & F_TY)) qm[2] = -qm[2];
            if (!fl && !(fc_mid & F_TY)) qp[2] = -qp[2];
            edge_y(K, qm, e1m, aEm, ym, qp, e1p, aEp, yp, DyM, DyP);
        }

        // ---- finish row jr-1 ---------------------------------------------------------------
        const int jf = jr - 1;
        if (jf >= j0 && jf < ny && out_lane) {
            const Member &M = member_ref(mab);
            const Consts &K = M.K;
            const size_t cidx = (size_t)jf * nx + i;
            const bool fluid = sf[s_lo][lane] & F_FLUID;  // solid cells keep their values
            double qn[4];
            update_finish(pX, DyM, dtdy, qn);
#pragma unroll
            for (int k = 0; k < 4; ++k) Qnp[k * plane + cidx] = fluid ? qn[k] : sq[s_lo][k][lane];
            const long long term = __double2ll_rn(detector_term(K, qn) * M.fix_scale);
            const double rate = cfl_rate(K, qn);
            colfix += fluid ? term : 0ll;
            lam = fluid ? fmax(lam, rate) : lam;
            const bool ok = qn[0] > 0.0 && qn[3] > 0.0 && isfinite(qn[0]) && isfinite(qn[1]) && isfinite(qn[2]) &&
                            isfinite(qn[3]);
            bad |= (fluid && !ok) ? 1 : 0;
        }
        if (final_row) break;

        // ---- row jr becomes the pending row ------------------------------------------------
        update_south(X, DyP, dtdy, pX);
        if (fl) {
#pragma unroll
            for (int k = 0; k < 4; ++k) nQ[k] = rc.qN[k];
            nE1 = rc.e1N;
            nAE = rc.aE;
            nY = rc.yN;
        }
        nF = fc_mid;
    }
    {
        const Member &M = member_ref(mab);
        const int m_next = a.m3 == 2 ? 0 : a.m3 + 1;
        if (out_lane && colfix != 0) atomicAdd((unsigned long long *)&M.S[m_next][i], (unsigned long long)colfix);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            lam = fmax(lam, __shfl_xor(lam, off, 64));
            bad |= __shfl_xor(bad, off, 64);
        }
        if (lane == 0) {
            if (lam > 0.0) atomicMax(M.lam[m_next], (unsigned long long)__double_as_longlong(lam));
            if (bad) atomicOr(M.flag, 1);
        }
    }

    // recorded cost of the rows marched here, for the next step's partition: the range's time
    // spread evenly over its rows, but at least a.cost_floor of the strip's mean row cost of this
    // step's partition (rows recorded cheap are where a share packs the most rows, and where a
    // change of the flow since, a liquid front arriving, makes the share late)
    const Control &C = control_at(ca);
    const long long cbase = member_ref(mab).cost0 + (long long)strip * ny;  // (the strip's cost_base)
    const float per_row = (float)fmax((double)(clock64() - t_begin) / (E - j0), floor_cost);
    const double spent = (double)per_row * (E - j0);
    for (int rr = j0 + lane; rr < E; rr += 64) C.cost_out[cbase + rr] = per_row;
    if (lane == 0) atomicAdd(&C.Ts_out[g], spent);
}

// A split costs the thief a halo (two extra reconstructed rows and a row of loads), so only ranges
// with at least this many unclaimed rows are split.
constexpr int kMinSplit = 3;
constexpr int kScanBatch = 40;  // descriptors per lane loaded at once by a thief's full scan
constexpr int kSample = 2;      // descriptors per lane of a thief's first look

// Search key of descriptor word d in slot s for thief attempt `attempt`, 0 if it offers nothing:
// score << 40 | hash << 32 | (2^31 - 1 - slot), larger is better.  Unowned ranges first, then by size
// class (floor log2 of the unclaimed rows); within a class a hash of (slot, thief) spreads the
// thieves over the victims.
__device__ __forceinline__ long long steal_key(unsigned long long d, int s, int attempt)
{
    const int rem = d_end(d) - d_cur(d);
    long long score = 0;
    if (!(d & kOwned) && rem >= 1) score = 64 + (31 - __clz(rem));
    else if ((d & kOwned) && rem >= kMinSplit) score = 31 - __clz(rem);
    if (score == 0) return 0;
    const unsigned h = ((unsigned)s * 2654435761u) ^ ((unsigned)blockIdx.x * 40503u + attempt);
    return (score << 40) | ((long long)(h & 0xFFu) << 32) | (long long)(0x7FFFFFFF - s);
}

__device__ __forceinline__ long long wave_max(long long v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Find work: a range nobody owns (taken whole) or a large range being marched with at least
// kMinSplit unclaimed rows (upper half taken).  Returns false when there is none.  On success the
// caller has claimed rows [*j0, *E) of strip *strip and owns descriptor *slot (-1: the rows up to
// *E are all it gets, when the descriptor list is full).
// A thief first looks at 64 kSample descriptors spread over the list (a phase of its own per
// attempt) and takes the best of them; it scans every descriptor only when that look finds nothing
// while some range is still unowned.  (Near the end of a step most searches find nothing: a full
// scan by every finishing wavefront loads the whole list each time and delays the last ones.  An
// unowned range is always found: its publisher counted it before publishing it, and its own
// search, after its own range, scans everything while the count is positive.)
__device__ bool steal(unsigned long long ca, int B, int *strip, int *j0, int *E, int *slot)
{
    const int lane = threadIdx.x;
    const Control &a = control_at(ca);
    for (int attempt = 0; attempt < 4096; ++attempt) {
        int n = __hip_atomic_load(a.nranges, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        n = n < a.max_slots ? n : a.max_slots;
        if (n <= 0) return false;
        long long best = 0;
        {
            const int stride = max(1, n / (64 * kSample));
            const int phase = (int)(((unsigned)blockIdx.x * 2654435761u + (unsigned)attempt * 40503u) % (unsigned)n);
            unsigned long long wd[kSample];
            int ws[kSample];
#pragma unroll
            for (int u = 0; u < kSample; ++u) {
                ws[u] = (int)(((long long)phase + (long long)(u * 64 + lane) * stride) % n);
                wd[u] = load_word(a.desc + ws[u]);
            }
#pragma unroll
            for (int u = 0; u < kSample; ++u) {
                const long long key = steal_key(wd[u], ws[u], attempt);
                best = key > best ? key : best;
            }
            best = wave_max(best);
        }
        if (best == 0 && __hip_atomic_load(a.unowned, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > 0) {
            // (all of a batch's loads are in flight together: one batch covers a launch's initial
            // descriptors and its first splits)
            for (int base = 0; base < n; base += 64 * kScanBatch) {
                unsigned long long wd[kScanBatch];
#pragma unroll
                for (int u = 0; u < kScanBatch; ++u) {
                    const int s = base + u * 64 + lane;
                    wd[u] = s < n ? load_word(a.desc + s) : 0ull;
                }
#pragma unroll
                for (int u = 0; u < kScanBatch; ++u) {
                    const int s = base + u * 64 + lane;
                    const long long key = s < n ? steal_key(wd[u], s, attempt) : 0;
                    best = key > best ? key : best;
                }
            }
            best = wave_max(best);
        }
        if (best == 0) return false;
        const int s = 0x7FFFFFFF - (int)(best & 0xFFFFFFFFll);
        int ok = 0, st = 0, r0 = 0, r1 = 0, sl = 0;
        if (lane == 0) {
            unsigned long long *p = a.desc + s;
            const unsigned long long old = load_word(p);
            const int cur = d_cur(old), end = d_end(old);
            if (!(old & kOwned) && end - cur >= 1) {
                if (atomicCAS(p, old, (old | kOwned) + (unsigned long long)B) == old) {
                    ok = 1; st = d_strip(old); r0 = cur; r1 = min(cur + B, end); sl = s;
                    atomicSub(a.unowned, 1);
                }
            } else if ((old & kOwned) && end - cur >= kMinSplit) {
                const int mid = cur + (end - cur) / 2;
                const unsigned long long lowered = (old & ~(0xFFFFFFull << 24)) | ((unsigned long long)mid << 24);
                if (atomicCAS(p, old, lowered) == old) {
                    ok = 1; st = d_strip(old); r0 = mid;
                    const int k = atomicAdd(a.nranges, 1);
                    if (k < a.max_slots) {
                        atomicExch(a.desc + k, d_make(true, st, end, min(mid + B, end)));
                        r1 = min(mid + B, end); sl = k;
                    } else {
                        r1 = end; sl = -1;  // list full: march the whole upper half unpublished
                    }
                }
            }
        }
        ok = __shfl(ok, 0, 64);
        if (ok) {
            *strip = __shfl(st, 0, 64);
            *j0 = __shfl(r0, 0, 64);
            *E = __shfl(r1, 0, 64);
            *slot = __shfl(sl, 0, 64);
            return true;
        }
    }
    if (lane == 0) atomicOr(a.flag, 4);
    return false;
}

// The record of global strip g (read through the scalar cache).
typedef const __attribute__((address_space(4))) StripInfo *StripPtr;
__device__ __forceinline__ StripInfo strip_at(unsigned long long ca, int g)
{
    unsigned long long addr = (unsigned long long)(uintptr_t)(control_at(ca).strips +
                                                              __builtin_amdgcn_readfirstlane(g));
    asm volatile("" : "+s"(addr));
    return *(const StripInfo *)(StripPtr)addr;
}

#ifdef BN2D_TIMELINE
// Opt-in instrumentation, compiled only with -DBN2D_TIMELINE (the library libbn2d_timeline.so, never
// the default one): per wavefront w, record w of g_timeline holds the real-time clock (100 MHz) at
// entry, after the strip totals, after the strip's table entry, after its row costs, after locating
// its range, after its own range and at exit, then its own range (strip, first row, rows) and the
// number of ranges it stole; bn_timeline_read copies the records of the last step to the host.
constexpr int kTimelineWaves = 16384, kTimelineWords = 16;
__device__ unsigned long long g_timeline[kTimelineWaves * kTimelineWords];
#define BN_TIMELINE(...) __VA_ARGS__
#else
#define BN_TIMELINE(...)
#endif

__global__ __launch_bounds__(64, 2) void step_kernel(StepArgs a)
{
    __shared__ double sq[3][4][64];
    __shared__ int sf[3][64];

    const int lane = threadIdx.x, w = blockIdx.x;
    const unsigned long long ma = a.maddr, ca = a.caddr;
    BN_TIMELINE(unsigned long long tl[7] = {__builtin_amdgcn_s_memrealtime(), 0, 0, 0, 0, 0, 0};
                long long tl_own[3] = {-1, 0, 0}; long long tl_steals = 0;)
    int nm, P;
    {
        const Control &C = control_at(ca);
        nm = C.nmembers;
        P = C.P;
        // the next step's range list and strip totals (this step does not touch them otherwise)
        for (int s = w * 64 + lane; s < C.max_slots; s += P * 64) C.desc_next[s] = 0ull;
        for (int c = w * 64 + lane; c < C.nstrips; c += P * 64) C.Ts_clear[c] = 0.0;
        if (w == 0 && lane == 0) *C.nranges_next = C.R0;
    }
    // per member (wavefront b mod P): elapsed time, and the third rotation buffers cleared
    const int m_clear = a.m3 == 0 ? 2 : a.m3 - 1;
    for (int b = w; b < nm; b += P) {
        const double dt = member_dt(a, ma, b);
        const Member &M = member_at(ma, b);
        for (int c = lane; c < M.K.nx; c += 64) M.S[m_clear][c] = 0;
        if (lane == 0) {
            *M.t += dt;
            *M.lam[m_clear] = 0ull;
            if (!(dt > 0.0)) atomicOr(M.flag, 2);
        }
    }

    // ---- this wavefront's range: the cost interval [w, w+1) T/P of the recorded costs ---------
    int g = 0, j0 = 0, E = 0, slot = w, head_g = -1;
    double head_off = 0.0;
    bool have = false;
    {
        const Control &C = control_at(ca);
        Chunks<double> strips;
        strips.load(C.Ts_in, C.nstrips);
        BN_TIMELINE(tl[1] = __builtin_amdgcn_s_memrealtime() + (unsigned long long)(strips.total != strips.total);)
        const double step = strips.total / P;
        // (the last share ends beyond every strip: its end is not compared against the total)
        int g_w, g_next;
        double soff0, soff1;
        strips.find(w * step, g_w, soff0);
        strips.find(w + 1 < P ? (w + 1) * step : 1e300, g_next, soff1);
        if (g_w < C.nstrips) {
            const StripInfo si = strip_at(ca, g_w);
            BN_TIMELINE(tl[2] = __builtin_amdgcn_s_memrealtime() + (unsigned long long)(si.ny < 0);)
            Chunks<float> rows;
            rows.load(C.cost_in + si.cost_base, si.ny);
            BN_TIMELINE(tl[3] = __builtin_amdgcn_s_memrealtime() + (unsigned long long)(rows.total != rows.total);)
            int lo, hi;
            double roff;
            rows.find(soff0, lo, roff);
            if (g_next == g_w) rows.find(soff1, hi, roff);
            else hi = si.ny;
            // published with atomic stores: other wavefronts read and update them atomically
            if (lane == 0 && lo < hi) atomicExch(C.desc + w, d_make(true, g_w, hi, min(lo + a.B, hi)));
            if (lo < hi) {
                have = true;
                g = g_w;
                j0 = lo;
                E = min(lo + a.B, hi);
                BN_TIMELINE(tl_own[0] = g_w; tl_own[1] = lo; tl_own[2] = hi - lo;)
            }
            // strips the share spans whole are left unowned (a strip cheaper than a share), counted
            // first: thieves scan every descriptor while the count is positive
            const int n_unowned = min(g_next, C.nstrips) - (g_w + 1);
            if (lane == 0 && n_unowned > 0) atomicAdd(C.unowned, n_unowned);
            for (int s = g_w + 1 + lane; s < g_next && s < C.nstrips; s += 64)
                atomicExch(C.desc + P + s, d_make(false, s, C.strips[s].ny, 0));
            // the head of the strip the share ends in is this wavefront's too: published owned and
            // unclaimed once its extent is known (after the first range is marched)
            if (g_next > g_w && g_next < C.nstrips) {
                head_g = g_next;
                head_off = soff1;
            }
        }
    }

    // own range, then the owned head of the next strip, then whatever can be taken (one call site
    // of the march, so that its code exists once)
    BN_TIMELINE(tl[4] = __builtin_amdgcn_s_memrealtime();)
    for (int phase = 0;; ++phase) {
        if (phase == 1) {
            BN_TIMELINE(tl[5] = __builtin_amdgcn_s_memrealtime();)
            have = false;
            if (head_g >= 0) {
                const Control &C = control_at(ca);
                const StripInfo si = strip_at(ca, head_g);
                Chunks<float> rows;
                rows.load(C.cost_in + si.cost_base, si.ny);
                int hend;
                double hoff;
                rows.find(head_off, hend, hoff);
                if (hend > 0) {
                    // nobody else can know this range yet: it is claimed directly, then published
                    g = head_g;
                    j0 = 0;
                    E = min(a.B, hend);
                    slot = P + head_g;
                    if (lane == 0) atomicExch(C.desc + slot, d_make(true, g, hend, E));
                    have = true;
                }
            }
        } else if (phase >= 2) {
            have = steal(ca, a.B, &g, &j0, &E, &slot);
            if (!have) break;
            BN_TIMELINE(++tl_steals;)
        }
        if (have) {
            const StripInfo si = strip_at(ca, g);
            march(a, ma, ca, sq, sf, si.member, g, si.local, j0, E, slot);
        }
    }
#ifdef BN2D_TIMELINE
    tl[6] = __builtin_amdgcn_s_memrealtime();
    if (lane == 0 && w < kTimelineWaves) {
        unsigned long long *T = g_timeline + (size_t)w * kTimelineWords;
        for (int k = 0; k < 7; ++k) T[k] = tl[k];
        T[7] = (unsigned long long)tl_own[0];
        T[8] = (unsigned long long)tl_own[1];
        T[9] = (unsigned long long)tl_own[2];
        T[10] = (unsigned long long)tl_steals;
    }
#endif
}

// Fixed-point free-surface integral and CFL rate of a state given through bn_set_state (thread =
// column, blockIdx.y = block of H rows).  S must be zero on entry.
__global__ __launch_bounds__(64) void reduce_kernel(const double *__restrict__ Q, const uint8_t *__restrict__ solid,
                                                     long long *S, double fix_scale, unsigned long long *lam_slot,
                                                     int *flag, Consts K, int H)
{
    const int i = (int)blockIdx.x * 64 + threadIdx.x;
    const size_t plane = (size_t)K.nx * K.ny;
    long long colfix = 0;
    double lam = 0.0;
    int bad = 0;
    if (i < K.nx) {
        const int ja = (int)blockIdx.y * H, je = min(K.ny, ja + H);
#pragma unroll 8
        for (int j = ja; j < je; ++j) {
            const size_t cidx = (size_t)j * K.nx + i;
            if (solid && solid[cidx]) continue;
            const double q[4] = {Q[cidx], Q[plane + cidx], Q[2 * plane + cidx], Q[3 * plane + cidx]};
            colfix += __double2ll_rn(detector_term(K, q) * fix_scale);
            lam = fmax(lam, cfl_rate(K, q));
            if (!(q[0] > 0.0) || !(q[3] > 0.0) || !isfinite(q[0]) || !isfinite(q[1]) || !isfinite(q[2]) ||
                !isfinite(q[3]))
                bad = 1;
        }
        if (colfix != 0) atomicAdd((unsigned long long *)&S[i], (unsigned long long)colfix);
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

// The free-surface integral alone, in partial sums (the same fixed-point terms as reduce_kernel, so
// their exact sum is the same integral): the adjoint's view of a given state.  Thread = column,
// blockIdx.y = block of H rows, whose partial is stored at Sp[blockIdx.y * nx + column].
__global__ __launch_bounds__(64) void colsum_kernel(const double *__restrict__ Q, const uint8_t *__restrict__ solid,
                                                     long long *Sp, double fix_scale, Consts K, int H)
{
    const int i = (int)blockIdx.x * 64 + threadIdx.x;
    if (i >= K.nx) return;
    const size_t plane = (size_t)K.nx * K.ny;
    const int ja = (int)blockIdx.y * H, je = min(K.ny, ja + H);
    long long colfix = 0;
#pragma unroll 8
    for (int j = ja; j < je; ++j) {
        const size_t cidx = (size_t)j * K.nx + i;
        const bool fluid = !solid || solid[cidx] == 0;
        const double q[4] = {0.0, 0.0, 0.0, Q[3 * plane + cidx]};
        const long long term = __double2ll_rn(detector_term(K, q) * fix_scale);
        colfix += fluid ? term : 0ll;
    }
    Sp[(size_t)blockIdx.y * K.nx + i] = colfix;
}

// dt = CFL / max rate of the current state, for the host (bn_compute_dt, bn_get_time).
__global__ void dt_kernel(const unsigned long long *lam_slot, double *dt_out, int *flag, Consts K)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double lam = __longlong_as_double((long long)*lam_slot);
        const bool ok = lam > 0.0 && isfinite(lam);
        *dt_out = ok ? K.cfl / lam : 0.0;
        if (!ok) atomicOr(flag, 2);
    }
}

// Schedule state of the next step after bn_set_state or a change of the launch shape: empty
// descriptor list, uniform recorded costs (1 per row), cleared strip totals to accumulate into.
__global__ void init_schedule_kernel(unsigned long long *desc, int *nranges, int *unowned, int R0, int max_slots,
                                     float *cost, long long nrows, double *Ts_in, double *Ts_acc,
                                     const StripInfo *strips, int nstrips)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < max_slots) desc[s] = 0ull;
    if (s < nrows) cost[s] = 1.0f;
    if (s < nstrips) {
        Ts_in[s] = (double)strips[s].ny;
        Ts_acc[s] = 0.0;
    }
    if (s == 0) {
        *nranges = R0;
        *unowned = 0;
    }
}

__global__ void zero_kernel(long long *p, int n)
{
    const int s = (int)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) p[s] = 0;
}

// y0 = y_bottom + dy * integral per column (with the offset of a bottom off the grid, as the step
// forms it from state Q), for bn_get_y0.
__global__ void y0_kernel(const long long *S, const int *jb, const double *dbot, const double *Q, double fix_inv,
                          double *y0, Consts K)
{
    const int i = (int)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K.nx) return;
    double v = (K.ylo + jb[i] * K.dy) + K.dy * ((double)S[i] * fix_inv);
    if (dbot && jb[i] < K.ny) v += dbot[i] * ((K.al - Q[(size_t)3 * K.nx * K.ny + (size_t)jb[i] * K.nx + i]) * K.inv_dal);
    y0[i] = v;
}

}  // namespace bn

#ifdef BN2D_TIMELINE
// The instrumented build's records of the last step: `waves` records of 16 words (the layout above)
// into the caller's host buffer.  0, or -2 on a HIP error.  Exists only in libbn2d_timeline.so.
extern "C" int bn_timeline_read(unsigned long long *host, int waves)
{
    if (!host || waves < 0 || waves > bn::kTimelineWaves) return -1;
    return hipMemcpyFromSymbol(host, HIP_SYMBOL(bn::g_timeline),
                               sizeof(unsigned long long) * bn::kTimelineWords * (size_t)waves) == hipSuccess ? 0 : -2;
}
#endif
