// Host side of the C ABI declared in include/bn2d.h: batches of grids, their device buffers and
// the launches.  A single-grid context is a batch of one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/bn2d.h"
#include "bn2d_layout.h"

namespace bn {
__global__ void step_kernel(StepArgs a);
__global__ void reduce_kernel(const double *Q, const uint8_t *solid, long long *S, double fix_scale,
                              unsigned long long *lam_slot, int *flag, Consts K, int H);
__global__ void dt_kernel(const unsigned long long *lam_slot, double *dt_out, int *flag, Consts K);
__global__ void colsum_kernel(const double *Q, const uint8_t *solid, long long *S, double fix_scale, Consts K, int H);
__global__ void init_schedule_kernel(unsigned long long *desc, int *nranges, int *unowned, int R0, int max_slots,
                                     float *cost, long long nrows, double *Ts_in, double *Ts_acc, const bn::StripInfo *strips,
                                     int nstrips);
__global__ void zero_kernel(long long *p, int n);
__global__ void y0_kernel(const long long *S, const int *jb, const double *dbot, const double *Q, double fix_inv,
                          double *y0, Consts K);
}  // namespace bn

// the discrete adjoint's passes (bn2d_adjoint.hip)
size_t bn_adjoint_scratch(int nx, int ny);
hipError_t bn_adjoint_launch(const bn::Consts &K, const double *q, const double *lam1, double *lam,
                             const uint8_t *solid, const int *jb, const double *dbot, const long long *Sp,
                             int nSp, double fix_inv, double dt, double *scratch, double *gbot, const double *src,
                             hipStream_t stream);

namespace {

constexpr int kOutCols = 60;  // output columns per wavefront (64 lanes minus a 2-column halo each side)
constexpr int kDefaultRowsPerBlock = 4;
constexpr int kReduceRows = 8;  // rows per block of the free-surface / CFL reduction of a given state

thread_local std::string g_last_hip_error;

int hip_fail(hipError_t e, const char *what)
{
    g_last_hip_error = std::string(what) + ": " + hipGetErrorString(e);
    return BN_EHIP;
}

#define HIP_TRY(call)                                    \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

// As many wavefronts as the device holds at once (compute units x resident single-wavefront
// workgroups per unit, from the kernel's register use): the launch is persistent.
int default_wavefronts()
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bn::step_kernel, 64, 0) != hipSuccess || cus <= 0 ||
        per_cu <= 0)
        return 1024;
    return cus * per_cu;
}

// The default launch: all resident wavefronts, or fewer for little work, about one per 4.5 strip
// rows (a power of two, at least 256), since every range costs two halo rows (measured on dam
// breaks: 256 for 256x128, 512 for 512x256, all 2048 resident ones from 2048x1024 on).
int sized_wavefronts(int resident, long long strip_rows)
{
    long long p = 256;
    while (p * 2 <= (long long)(strip_rows / 4.5)) p *= 2;
    return (int)std::min<long long>(resident, p);
}

// One grid: its parameters and device buffers.  `dev` mirrors what the kernels read.
struct Grid {
    bn_grid grid;
    bn_params params;
    bn::Member dev;                     // host copy of the device Member (pointers filled in)
    double *q[2] = {nullptr, nullptr};
    uint8_t *solid = nullptr;
    int *jb = nullptr;
    std::vector<int> jb_host;           // first fluid row of each column
    double *dbot = nullptr;             // [nx] bottom offsets, allocated by bn_*set_bottom
    long long *S = nullptr;             // [3][nx]
    unsigned long long *lam = nullptr;  // [3]
    double *t = nullptr;
    int *flag = nullptr;
    double *y0 = nullptr;               // [nx] staging for bn_get_y0
    double *dt = nullptr;               // staging for dt queries
    double *adj = nullptr;              // adjoint scratch planes, allocated on first use
    long long *adjS = nullptr;          // [ceil(ny / 16)][nx] free-surface partial sums of the adjoint's state
    bool has_state = false;
};

// Validate one grid and its mask; fills the first fluid row of each column.
int check_grid(const bn_grid *grid, const bn_params *params, const uint8_t *solid, std::vector<int> &jb)
{
    if (!grid || !params) return BN_EINVAL;
    if (grid->nx <= 0 || grid->ny <= 0 || !(grid->x1 > grid->x0) || !(grid->y1 > grid->y0)) return BN_EINVAL;
    const bn_params &p = *params;
    if (!(p.k0 > 0.0) || !(p.rho0 > 0.0) || !(p.alpha_gas > 0.0) || !(p.alpha_liq > p.alpha_gas) ||
        !(p.alpha_liq <= 1.0) || !(p.cfl > 0.0) || !(p.cfl <= 1.0) || !(p.g >= 0.0) || !std::isfinite(p.g) ||
        !std::isfinite(p.k0) || !std::isfinite(p.rho0))
        return BN_EINVAL;
    for (int s = 0; s < 4; ++s)
        if (p.bc[s] != 0 && p.bc[s] != 1) return BN_EINVAL;
    const int nx = grid->nx, ny = grid->ny;
    if ((nx + kOutCols - 1) / kOutCols > 0x7FFF || ny > 0xFF0000) return BN_EINVAL;
    // first fluid row of each column; solid cells above a fluid cell are not supported (Sec. 3.5)
    jb.assign(nx, 0);
    if (solid) {
        for (int i = 0; i < nx; ++i) {
            int j = 0;
            while (j < ny && solid[(size_t)j * nx + i]) ++j;
            jb[i] = j;
            for (int jj = j; jj < ny; ++jj)
                if (solid[(size_t)jj * nx + i]) return BN_EUNSUPPORTED;
        }
    }
    return BN_OK;
}

bn::Consts make_consts(const bn_grid &grid, const bn_params &p)
{
    bn::Consts K;
    std::memset(&K, 0, sizeof(K));
    K.nx = grid.nx;
    K.ny = grid.ny;
    K.dx = (grid.x1 - grid.x0) / grid.nx;
    K.dy = (grid.y1 - grid.y0) / grid.ny;
    K.ylo = grid.y0;
    K.g = p.g;
    K.k0 = p.k0;
    K.rho0 = p.rho0;
    K.al = p.alpha_liq;
    K.ag = p.alpha_gas;
    K.cfl = p.cfl;
    for (int s = 0; s < 4; ++s) K.bc[s] = p.bc[s];
    K.c2 = p.k0 / p.rho0;
    K.c = std::sqrt(K.c2);
    K.inv_c2 = 1.0 / K.c2;
    K.inv2c = 0.5 / K.c;
    K.half_rho0 = 0.5 * p.rho0;
    K.a = p.g * p.rho0 / p.k0;
    K.e_up1 = std::exp(-K.a * K.dy);
    K.e_dn1 = std::exp(K.a * K.dy);
    K.e_uph = std::exp(-K.a * 0.5 * K.dy);
    K.e_dnh = std::exp(K.a * 0.5 * K.dy);
    K.so_thr = 10.0 * p.alpha_gas;
    K.inv_dx = 1.0 / K.dx;
    K.inv_dy = 1.0 / K.dy;
    K.inv2dx = 1.0 / (2.0 * K.dx);
    K.inv2dy = 1.0 / (2.0 * K.dy);
    K.inv_rho0 = 1.0 / p.rho0;
    K.inv_dal = 1.0 / (p.alpha_liq - p.alpha_gas);
    return K;
}

}  // namespace

// The batch: its grids, the shared scheduling buffers and the rotation state.  The state buffers
// (cur), range lists and row costs (par) rotate by 2, the free-surface integrals, CFL maxima and
// strip cost totals (m3) by 3; all members rotate together, one launch per step.
struct bn_batch {
    hipStream_t stream = nullptr;
    std::vector<Grid> g;
    int nstrips = 0;                     // global strips (all members)
    long long nrows = 0;                 // rows over all strips (cost array length)
    int cur = 0, par = 0, m3 = 0;
    int B = kDefaultRowsPerBlock;
    int P = 1024, P_default = 1024;
    int R0 = 0, max_slots = 0, slots_alloc = 0;
    bn::Member *members = nullptr;       // [count] on the device
    bn::Control *ctl = nullptr;          // [6] on the device: combination 3 par + m3
    unsigned long long *desc = nullptr;  // [2][max_slots]
    int *nranges = nullptr;              // [3]: range counts [2], unowned ranges
    float *cost = nullptr;               // [2][nrows]
    double *Ts = nullptr;                // [3][nstrips]
    bn::StripInfo *strips = nullptr;     // [nstrips]
    int *flag = nullptr;                 // scheduler error (4)
};

// The single-grid context: a batch of one.
struct bn_ctx {
    bn_batch *b = nullptr;
};

namespace {

void free_batch(bn_batch *b)
{
    for (Grid &g : b->g) {
        void *ptrs[] = {g.q[0], g.q[1], g.solid, g.jb, g.dbot, g.S, g.lam, g.t, g.flag, g.y0, g.dt, g.adj, g.adjS};
        for (void *p : ptrs)
            if (p) (void)hipFree(p);
    }
    void *ptrs[] = {b->members, b->ctl, b->desc, b->nranges, b->cost, b->Ts, b->strips, b->flag};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete b;
}

// Descriptors: one range per wavefront, one head per strip, and up to 16 splits per wavefront (a
// split beyond that is marched unpublished).
int set_shape(bn_batch *b)
{
    b->R0 = b->P + b->nstrips;
    const long long slots = (long long)b->R0 + 16ll * b->P;
    if (slots > (1ll << 30)) return BN_EINVAL;
    b->max_slots = (int)slots;
    if (b->max_slots > b->slots_alloc) {
        if (b->desc) {
            HIP_TRY(hipFree(b->desc));
            b->desc = nullptr;
        }
        hipError_t e = hipMalloc(&b->desc, sizeof(unsigned long long) * 2 * (size_t)b->max_slots);
        if (e != hipSuccess) {
            b->desc = nullptr;
            b->slots_alloc = 0;
            g_last_hip_error = std::string("hipMalloc(ranges): ") + hipGetErrorString(e);
            return BN_ENOMEM;
        }
        b->slots_alloc = b->max_slots;
    }
    return BN_OK;
}

// Device copies of the Member array and of the six Control blocks.
int write_tables(bn_batch *b)
{
    std::vector<bn::Member> m(b->g.size());
    for (size_t k = 0; k < b->g.size(); ++k) m[k] = b->g[k].dev;
    HIP_TRY(hipMemcpyAsync(b->members, m.data(), sizeof(bn::Member) * m.size(), hipMemcpyHostToDevice, b->stream));
    bn::Control h[6];
    for (int p = 0; p < 2; ++p)
        for (int mm = 0; mm < 3; ++mm) {
            bn::Control &C = h[3 * p + mm];
            const int q = p ^ 1;
            const size_t ns = b->nstrips;
            C.desc = b->desc + (size_t)p * b->max_slots;
            C.nranges = b->nranges + p;
            C.desc_next = b->desc + (size_t)q * b->max_slots;
            C.nranges_next = b->nranges + q;
            C.cost_in = b->cost + (size_t)p * b->nrows;
            C.cost_out = b->cost + (size_t)q * b->nrows;
            C.Ts_in = b->Ts + mm * ns;
            C.Ts_out = b->Ts + ((mm + 1) % 3) * ns;
            C.Ts_clear = b->Ts + ((mm + 2) % 3) * ns;
            C.strips = b->strips;
            C.flag = b->flag;
            C.unowned = b->nranges + 2;
            C.nstrips = b->nstrips;
            C.nmembers = (int)b->g.size();
            C.R0 = b->R0;
            C.max_slots = b->max_slots;
            C.P = b->P;
        }
    HIP_TRY(hipMemcpyAsync(b->ctl, h, sizeof(h), hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return BN_OK;
}

// Schedule state for the next step: empty range list, uniform recorded costs.
int init_schedule(bn_batch *b)
{
    const long long n = std::max<long long>(std::max<long long>(b->nrows, b->max_slots), b->nstrips);
    const size_t ns = b->nstrips;
    hipLaunchKernelGGL(bn::init_schedule_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, b->stream,
                       b->desc + (size_t)b->par * b->max_slots, b->nranges + b->par, b->nranges + 2, b->R0,
                       b->max_slots,
                       b->cost + (size_t)b->par * b->nrows, b->nrows, b->Ts + (size_t)b->m3 * ns,
                       b->Ts + (size_t)((b->m3 + 1) % 3) * ns, b->strips, b->nstrips);
    HIP_TRY(hipGetLastError());
    return BN_OK;
}

int zero_S(bn_batch *b, Grid &g, int m)
{
    const int nx = g.grid.nx;
    hipLaunchKernelGGL(bn::zero_kernel, dim3((nx + 255) / 256), dim3(256), 0, b->stream, g.S + (size_t)m * nx, nx);
    HIP_TRY(hipGetLastError());
    return BN_OK;
}

// One step of every member: reads state cur, S[m3], CFL max[m3], ranges[par]; writes state
// 1-cur, S[m3+1], CFL max[m3+1], ranges[par^1].
int launch_step(bn_batch *b, bool cfl_dt, double dt_arg)
{
    for (const Grid &g : b->g)
        if (!g.has_state) return BN_EINVAL;
    bn::StepArgs a;
    a.maddr = (unsigned long long)(uintptr_t)b->members;
    a.caddr = (unsigned long long)(uintptr_t)(b->ctl + 3 * b->par + b->m3);
    a.dt_arg = dt_arg;
    a.cfl_dt = cfl_dt ? 1 : 0;
    a.cur = b->cur;
    a.m3 = b->m3;
    a.B = b->B;
    a.cost_floor = b->nrows >= (long long)bn::kCostFloorRows * b->P ? bn::kCostFloor : 0.0;
    hipLaunchKernelGGL(bn::step_kernel, dim3(b->P), dim3(64), 0, b->stream, a);
    HIP_TRY(hipGetLastError());
    b->cur ^= 1;
    b->par ^= 1;
    b->m3 = (b->m3 + 1) % 3;
    return BN_OK;
}

int sync_flags(bn_batch *b, int32_t *member)
{
    std::vector<int> f(b->g.size() + 1, 0);
    for (size_t k = 0; k < b->g.size(); ++k)
        HIP_TRY(hipMemcpyAsync(&f[k], b->g[k].flag, sizeof(int), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipMemcpyAsync(&f[b->g.size()], b->flag, sizeof(int), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (member) *member = -1;
    if (f[b->g.size()] & 4) return BN_EINTERNAL;
    for (size_t k = 0; k < b->g.size(); ++k) {
        if (f[k] & 4) return BN_EINTERNAL;
        if (f[k]) {
            if (member) *member = (int32_t)k;
            return BN_ENONPHYS;
        }
    }
    return BN_OK;
}

// dt = CFL / max rate of a member's current state into its staging word (stream-ordered).
int query_dt(bn_batch *b, Grid &g)
{
    hipLaunchKernelGGL(bn::dt_kernel, dim3(1), dim3(64), 0, b->stream, g.lam + b->m3, g.dt, g.flag, g.dev.K);
    HIP_TRY(hipGetLastError());
    return BN_OK;
}

bool bad_member(const bn_batch *b, int32_t k) { return !b || k < 0 || k >= (int32_t)b->g.size(); }

// The fixed-point free-surface integral of a given state as colsum_blocks(ny) partial sums per
// column into Sp ([blocks][nx] words, overwritten: no clearing, no atomics).
constexpr int kColsumRows = 16;
int colsum_blocks(int ny) { return (ny + kColsumRows - 1) / kColsumRows; }
int adjoint_colsum(bn_batch *b, Grid &g, const double *q_dev, long long *Sp)
{
    const int nx = g.grid.nx, ny = g.grid.ny;
    hipLaunchKernelGGL(bn::colsum_kernel, dim3((nx + 63) / 64, colsum_blocks(ny)), dim3(64), 0, b->stream, q_dev,
                       g.solid, Sp, g.dev.fix_scale, g.dev.K, kColsumRows);
    HIP_TRY(hipGetLastError());
    return BN_OK;
}

}  // namespace

extern "C" {

int bn_batch_create(int32_t count, const bn_grid *grids, const bn_params *params, const uint8_t *const *solids,
                    void *hip_stream, bn_batch **out)
{
    if (!out) return BN_EINVAL;
    *out = nullptr;
    if (count <= 0 || count > 0x7FFF || !grids || !params) return BN_EINVAL;
    std::vector<std::vector<int>> jbs(count);
    long long total_strips = 0;
    for (int k = 0; k < count; ++k) {
        const int rc = check_grid(&grids[k], &params[k], solids ? solids[k] : nullptr, jbs[k]);
        if (rc) return rc;
        total_strips += (grids[k].nx + kOutCols - 1) / kOutCols;
    }
    if (total_strips > 0x7FFF) return BN_EINVAL;  // the strip field of a range descriptor
    bn_batch *b = new (std::nothrow) bn_batch();
    if (!b) return BN_ENOMEM;
    b->stream = (hipStream_t)hip_stream;
    b->g.resize(count);
    auto fail = [&](int code) {
        free_batch(b);
        return code;
    };
    hipError_t e = hipSuccess;
#define ALLOC(ptr, bytes)                                                          \
    e = hipMalloc(&(ptr), (bytes));                                                \
    if (e != hipSuccess) {                                                         \
        g_last_hip_error = std::string("hipMalloc: ") + hipGetErrorString(e);      \
        return fail(BN_ENOMEM);                                                    \
    }
    std::vector<bn::StripInfo> strips;
    for (int k = 0; k < count; ++k) {
        Grid &g = b->g[k];
        g.grid = grids[k];
        g.params = params[k];
        g.jb_host = jbs[k];
        const int nx = g.grid.nx, ny = g.grid.ny;
        const size_t plane = (size_t)nx * ny;
        ALLOC(g.q[0], sizeof(double) * 4 * plane);
        ALLOC(g.q[1], sizeof(double) * 4 * plane);
        ALLOC(g.jb, sizeof(int) * nx);
        ALLOC(g.S, sizeof(long long) * 3 * nx);
        ALLOC(g.lam, sizeof(unsigned long long) * 3);
        ALLOC(g.t, sizeof(double));
        ALLOC(g.flag, sizeof(int));
        ALLOC(g.y0, sizeof(double) * nx);
        ALLOC(g.dt, sizeof(double));
        const uint8_t *solid = solids ? solids[k] : nullptr;
        if (solid) {
            ALLOC(g.solid, plane);
            e = hipMemcpy(g.solid, solid, plane, hipMemcpyHostToDevice);
        }
        if (e == hipSuccess) e = hipMemcpy(g.jb, jbs[k].data(), sizeof(int) * nx, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(g.S, 0, sizeof(long long) * 3 * nx);
        if (e == hipSuccess) e = hipMemset(g.lam, 0, sizeof(unsigned long long) * 3);
        if (e == hipSuccess) e = hipMemset(g.t, 0, sizeof(double));
        if (e == hipSuccess) e = hipMemset(g.flag, 0, sizeof(int));
        if (e != hipSuccess) {
            g_last_hip_error = std::string("bn_batch_create: ") + hipGetErrorString(e);
            return fail(BN_EHIP);
        }
        bn::Member &M = g.dev;
        std::memset(&M, 0, sizeof(M));
        M.K = make_consts(g.grid, g.params);
        M.q[0] = g.q[0];
        M.q[1] = g.q[1];
        M.solid = g.solid;
        M.jb = g.jb;
        for (int r = 0; r < 3; ++r) {
            M.S[r] = g.S + (size_t)r * nx;
            M.lam[r] = g.lam + r;
        }
        M.t = g.t;
        M.flag = g.flag;
        // fixed point: terms (alpha - alpha_g)/(alpha_l - alpha_g) lie in about [0, 1]; 2^f
        // leaves a factor 2 of headroom for ny of them in a signed 64-bit integer
        int lg = 0;
        while ((1ll << lg) < (long long)ny + 1) ++lg;
        M.fix_scale = std::ldexp(1.0, 61 - lg);
        M.fix_inv = std::ldexp(1.0, lg - 61);
        M.nstrips = (nx + kOutCols - 1) / kOutCols;
        M.strip0 = b->nstrips;
        M.cost0 = b->nrows;
        b->nstrips += M.nstrips;
        b->nrows += (long long)M.nstrips * ny;
        for (int s = 0; s < M.nstrips; ++s) strips.push_back({k, s, ny, 0, M.cost0 + (long long)s * ny});
    }
    ALLOC(b->members, sizeof(bn::Member) * count);
    ALLOC(b->ctl, sizeof(bn::Control) * 6);
    ALLOC(b->nranges, sizeof(int) * 3);  // two range counts and the unowned count
    ALLOC(b->cost, sizeof(float) * 2 * (size_t)b->nrows);
    ALLOC(b->Ts, sizeof(double) * 3 * (size_t)b->nstrips);
    ALLOC(b->strips, sizeof(bn::StripInfo) * (size_t)b->nstrips);
    ALLOC(b->flag, sizeof(int));
#undef ALLOC
    e = hipMemcpy(b->strips, strips.data(), sizeof(bn::StripInfo) * strips.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(b->nranges, 0, sizeof(int) * 3);
    if (e == hipSuccess) e = hipMemset(b->flag, 0, sizeof(int));
    if (e == hipSuccess) e = hipMemset(b->Ts, 0, sizeof(double) * 3 * (size_t)b->nstrips);
    if (e != hipSuccess) {
        g_last_hip_error = std::string("bn_batch_create: ") + hipGetErrorString(e);
        return fail(BN_EHIP);
    }
    b->P_default = sized_wavefronts(default_wavefronts(), b->nrows);
    b->P = b->P_default;
    int rc = set_shape(b);
    if (!rc) rc = write_tables(b);
    if (rc) return fail(rc);
    *out = b;
    return BN_OK;
}

int bn_batch_set_state(bn_batch *b, int32_t member, const double *q_dev)
{
    if (bad_member(b, member) || !q_dev) return BN_EINVAL;
    Grid &g = b->g[member];
    const size_t bytes = sizeof(double) * 4 * (size_t)g.grid.nx * g.grid.ny;
    HIP_TRY(hipMemcpyAsync(g.q[b->cur], q_dev, bytes, hipMemcpyDeviceToDevice, b->stream));
    HIP_TRY(hipMemsetAsync(g.flag, 0, sizeof(int), b->stream));
    HIP_TRY(hipMemsetAsync(b->flag, 0, sizeof(int), b->stream));
    HIP_TRY(hipMemsetAsync(g.t, 0, sizeof(double), b->stream));
    HIP_TRY(hipMemsetAsync(g.lam, 0, sizeof(unsigned long long) * 3, b->stream));
    // free-surface integral S[m3] and CFL max[m3] of the given state; S[m3+1] cleared to accumulate
    int rc = zero_S(b, g, b->m3);
    if (!rc) rc = zero_S(b, g, (b->m3 + 1) % 3);
    if (rc) return rc;
    const int H = kReduceRows;
    const dim3 rgrid((g.grid.nx + 63) / 64, (g.grid.ny + H - 1) / H);
    hipLaunchKernelGGL(bn::reduce_kernel, rgrid, dim3(64), 0, b->stream, g.q[b->cur], g.solid,
                       g.S + (size_t)b->m3 * g.grid.nx, g.dev.fix_scale, g.lam + b->m3, g.flag, g.dev.K, H);
    HIP_TRY(hipGetLastError());
    rc = init_schedule(b);
    if (rc) return rc;
    g.has_state = true;
    return BN_OK;
}

int bn_batch_get_state(bn_batch *b, int32_t member, double *q_dev)
{
    if (bad_member(b, member) || !q_dev || !b->g[member].has_state) return BN_EINVAL;
    Grid &g = b->g[member];
    const size_t bytes = sizeof(double) * 4 * (size_t)g.grid.nx * g.grid.ny;
    HIP_TRY(hipMemcpyAsync(q_dev, g.q[b->cur], bytes, hipMemcpyDeviceToDevice, b->stream));
    return BN_OK;
}

int bn_batch_run(bn_batch *b, int32_t n_steps)
{
    if (!b || n_steps < 0) return BN_EINVAL;
    for (int32_t s = 0; s < n_steps; ++s) {
        const int rc = launch_step(b, true, 0.0);
        if (rc) return rc;
    }
    return BN_OK;
}

int bn_batch_get_time(bn_batch *b, int32_t member, double *t_host, double *next_dt_host)
{
    if (bad_member(b, member) || !b->g[member].has_state) return BN_EINVAL;
    Grid &g = b->g[member];
    double tmp[2];
    HIP_TRY(hipMemcpyAsync(&tmp[0], g.t, sizeof(double), hipMemcpyDeviceToHost, b->stream));
    int rc = query_dt(b, g);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(&tmp[1], g.dt, sizeof(double), hipMemcpyDeviceToHost, b->stream));
    rc = sync_flags(b, nullptr);
    if (t_host) *t_host = tmp[0];
    if (next_dt_host) *next_dt_host = tmp[1];
    return rc;
}

int bn_batch_get_y0(bn_batch *b, int32_t member, double *y0_host)
{
    if (bad_member(b, member) || !y0_host || !b->g[member].has_state) return BN_EINVAL;
    Grid &g = b->g[member];
    const int nx = g.grid.nx;
    hipLaunchKernelGGL(bn::y0_kernel, dim3((nx + 255) / 256), dim3(256), 0, b->stream, g.S + (size_t)b->m3 * nx,
                       g.jb, g.dbot, g.q[b->cur], g.dev.fix_inv, g.y0, g.dev.K);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(y0_host, g.y0, sizeof(double) * nx, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return BN_OK;
}

int bn_batch_set_bottom(bn_batch *b, int32_t member, const double *y_bottom_host)
{
    if (bad_member(b, member)) return BN_EINVAL;
    Grid &g = b->g[member];
    const int nx = g.grid.nx;
    const double dy = (g.grid.y1 - g.grid.y0) / g.grid.ny;
    std::vector<double> d(nx, 0.0);
    if (y_bottom_host) {
        for (int i = 0; i < nx; ++i) {
            d[i] = y_bottom_host[i] - (g.grid.y0 + g.jb_host[i] * dy);
            if (!(d[i] >= -0.5 * dy && d[i] < 0.5 * dy)) return BN_EINVAL;
        }
    }
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (!y_bottom_host) {
        if (g.dbot) HIP_TRY(hipFree(g.dbot));
        g.dbot = nullptr;
    } else {
        if (!g.dbot) {
            const hipError_t e = hipMalloc(&g.dbot, sizeof(double) * nx);
            if (e != hipSuccess) {
                g.dbot = nullptr;
                g_last_hip_error = std::string("hipMalloc(bottom): ") + hipGetErrorString(e);
                return BN_ENOMEM;
            }
        }
        HIP_TRY(hipMemcpy(g.dbot, d.data(), sizeof(double) * nx, hipMemcpyHostToDevice));
    }
    g.dev.dbot = g.dbot;
    return write_tables(b);
}

int bn_batch_status(bn_batch *b, int32_t *member)
{
    if (!b) return BN_EINVAL;
    return sync_flags(b, member);
}

int bn_batch_set_launch(bn_batch *b, int32_t rows_per_block, int32_t wavefronts)
{
    if (!b || rows_per_block < 0 || rows_per_block > 4096 || wavefronts < 0 || wavefronts > 65536) return BN_EINVAL;
    const int B = rows_per_block ? rows_per_block : kDefaultRowsPerBlock;
    const int P = wavefronts ? wavefronts : b->P_default;
    if (B == b->B && P == b->P) return BN_OK;
    HIP_TRY(hipStreamSynchronize(b->stream));
    const int oldB = b->B, oldP = b->P;
    b->B = B;
    b->P = P;
    int rc = set_shape(b);
    if (!rc) rc = write_tables(b);
    if (rc) {
        b->B = oldB;
        b->P = oldP;
        if (!set_shape(b)) (void)write_tables(b);
        return rc;
    }
    // the next step's range list follows the new shape; states, times and integrals stay
    return init_schedule(b);
}

int bn_batch_get_launch(bn_batch *b, int32_t *rows_per_block, int32_t *wavefronts)
{
    if (!b) return BN_EINVAL;
    if (rows_per_block) *rows_per_block = b->B;
    if (wavefronts) *wavefronts = b->P;
    return BN_OK;
}

void bn_batch_destroy(bn_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    free_batch(b);
}

// ---- single grid: a batch of one --------------------------------------------------------------

int bn_create(const bn_grid *grid, const bn_params *params, const uint8_t *solid, void *hip_stream, bn_ctx **out)
{
    if (!grid || !params || !out) return BN_EINVAL;
    *out = nullptr;
    bn_ctx *c = new (std::nothrow) bn_ctx();
    if (!c) return BN_ENOMEM;
    const uint8_t *solids[1] = {solid};
    const int rc = bn_batch_create(1, grid, params, solids, hip_stream, &c->b);
    if (rc) {
        delete c;
        return rc;
    }
    *out = c;
    return BN_OK;
}

int bn_set_state(bn_ctx *c, const double *q_dev)
{
    if (!c) return BN_EINVAL;
    return bn_batch_set_state(c->b, 0, q_dev);
}

int bn_get_state(bn_ctx *c, double *q_dev)
{
    if (!c) return BN_EINVAL;
    return bn_batch_get_state(c->b, 0, q_dev);
}

int bn_compute_dt(bn_ctx *c, double *dt_host)
{
    if (!c || !dt_host || !c->b->g[0].has_state) return BN_EINVAL;
    return bn_batch_get_time(c->b, 0, nullptr, dt_host);
}

int bn_step(bn_ctx *c, double dt)
{
    if (!c || !c->b->g[0].has_state || !(dt > 0.0) || !std::isfinite(dt)) return BN_EINVAL;
    return launch_step(c->b, false, dt);
}

int bn_run(bn_ctx *c, int32_t n_steps)
{
    if (!c || !c->b->g[0].has_state) return BN_EINVAL;
    return bn_batch_run(c->b, n_steps);
}

int bn_get_time(bn_ctx *c, double *t_host, double *next_dt_host)
{
    if (!c) return BN_EINVAL;
    return bn_batch_get_time(c->b, 0, t_host, next_dt_host);
}

int bn_get_y0(bn_ctx *c, double *y0_host)
{
    if (!c) return BN_EINVAL;
    return bn_batch_get_y0(c->b, 0, y0_host);
}

int bn_status(bn_ctx *c)
{
    if (!c) return BN_EINVAL;
    return bn_batch_status(c->b, nullptr);
}

int bn_set_bottom(bn_ctx *c, const double *y_bottom_host)
{
    if (!c) return BN_EINVAL;
    return bn_batch_set_bottom(c->b, 0, y_bottom_host);
}

int bn_set_launch(bn_ctx *c, int32_t rows_per_block, int32_t wavefronts)
{
    if (!c) return BN_EINVAL;
    return bn_batch_set_launch(c->b, rows_per_block, wavefronts);
}

int bn_get_launch(bn_ctx *c, int32_t *rows_per_block, int32_t *wavefronts)
{
    if (!c) return BN_EINVAL;
    return bn_batch_get_launch(c->b, rows_per_block, wavefronts);
}

}  // extern "C"

namespace {
// The adjoint's scratch, allocated on a context's first adjoint step and kept until bn_destroy.
int adjoint_scratch(Grid &g)
{
    const int nx = g.grid.nx, ny = g.grid.ny;
    if (!g.adj) {
        hipError_t e = hipMalloc(&g.adj, sizeof(double) * bn_adjoint_scratch(nx, ny));
        if (e == hipSuccess) e = hipMalloc(&g.adjS, sizeof(long long) * (size_t)nx * colsum_blocks(ny));
        if (e != hipSuccess) {
            if (g.adj) (void)hipFree(g.adj);
            g.adj = nullptr;
            g.adjS = nullptr;
            g_last_hip_error = std::string("hipMalloc(adjoint scratch): ") + hipGetErrorString(e);
            return BN_ENOMEM;
        }
    }
    return BN_OK;
}
}  // namespace

extern "C" {

int bn_adjoint_step(bn_ctx *c, const double *q_dev, const double *lam_next_dev, double dt, double *lam_dev,
                    double *grad_bottom_dev, const double *src_dev)
{
    if (!c || !q_dev || !lam_next_dev || !lam_dev || !(dt > 0.0) || !std::isfinite(dt)) return BN_EINVAL;
    bn_batch *b = c->b;
    Grid &g = b->g[0];
    int rc = adjoint_scratch(g);
    if (rc) return rc;
    // the free-surface integral of the given state, exactly as a step from it would use it
    long long *S = g.adjS;
    rc = adjoint_colsum(b, g, q_dev, S);
    if (rc) return rc;
    HIP_TRY(bn_adjoint_launch(g.dev.K, q_dev, lam_next_dev, lam_dev, g.solid, g.jb, g.dbot, S,
                              colsum_blocks(g.grid.ny), g.dev.fix_inv, dt, g.adj, grad_bottom_dev, src_dev, b->stream));
    return BN_OK;
}

int bn_get_column_sums(bn_ctx *c, int64_t *sums_dev)
{
    if (!c || !sums_dev) return BN_EINVAL;
    bn_batch *b = c->b;
    Grid &g = b->g[0];
    HIP_TRY(hipMemcpyAsync(sums_dev, g.S + (size_t)b->m3 * g.grid.nx, sizeof(long long) * g.grid.nx,
                           hipMemcpyDeviceToDevice, b->stream));
    return BN_OK;
}

int bn_adjoint_step_sums(bn_ctx *c, const double *q_dev, const int64_t *sums_dev, const double *lam_next_dev,
                         double dt, double *lam_dev, double *grad_bottom_dev, const double *src_dev)
{
    if (!c || !q_dev || !sums_dev || !lam_next_dev || !lam_dev || !(dt > 0.0) || !std::isfinite(dt))
        return BN_EINVAL;
    bn_batch *b = c->b;
    Grid &g = b->g[0];
    const int rc = adjoint_scratch(g);
    if (rc) return rc;
    // the given column sums are the whole integral: one partial per column
    HIP_TRY(bn_adjoint_launch(g.dev.K, q_dev, lam_next_dev, lam_dev, g.solid, g.jb, g.dbot,
                              reinterpret_cast<const long long *>(sums_dev), 1, g.dev.fix_inv, dt, g.adj,
                              grad_bottom_dev, src_dev, b->stream));
    return BN_OK;
}

}  // extern "C"

// ---- the adjoint step without allocation ------------------------------------------------------
// Scratch of bn_adjoint_step_noalloc: a file-scope device array, one copy per GPU, held until the
// process ends.  Host code never names it in a launch or copy: its device address, per device, comes
// from hipGetSymbolAddress on the first call on that device.
namespace {
constexpr size_t kNoAllocScratchDoubles = size_t(1) << 24;  // 128 MiB
}
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {
std::mutex g_scratch_mu;
std::vector<double *> g_scratch_ptr;  // per device, null until resolved

int scratch_address(double **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return hip_fail(hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return BN_OK;
}
}  // namespace

extern "C" {

int bn_adjoint_step_noalloc(bn_ctx *c, const double *q_dev, const double *lam_next_dev, double dt, double *lam_dev,
                            double *grad_bottom_dev, const double *src_dev)
{
    if (!c || !q_dev || !lam_next_dev || !lam_dev || !(dt > 0.0) || !std::isfinite(dt)) return BN_EINVAL;
    bn_batch *b = c->b;
    Grid &g = b->g[0];
    const int nx = g.grid.nx, ny = g.grid.ny;
    // the free-surface partial sums follow the adjoint's planes
    const size_t planes = bn_adjoint_scratch(nx, ny);
    if (planes + (size_t)nx * colsum_blocks(ny) > kNoAllocScratchDoubles) return BN_EINVAL;
    double *base = nullptr;
    const int rc = scratch_address(&base);
    if (rc) return rc;
    long long *S = reinterpret_cast<long long *>(base + planes);
    // (the array keeps the previous call's contents: every word used is written before it is read)
    const int rc2 = adjoint_colsum(b, g, q_dev, S);
    if (rc2) return rc2;
    HIP_TRY(bn_adjoint_launch(g.dev.K, q_dev, lam_next_dev, lam_dev, g.solid, g.jb, g.dbot, S, colsum_blocks(ny),
                              g.dev.fix_inv, dt, base, grad_bottom_dev, src_dev, b->stream));
    return BN_OK;
}

void bn_destroy(bn_ctx *c)
{
    if (!c) return;
    bn_batch_destroy(c->b);
    delete c;
}

const char *bn_strerror(int code)
{
    switch (code) {
    case BN_OK: return "ok";
    case BN_EINVAL: return "invalid argument";
    case BN_EHIP: return g_last_hip_error.empty() ? "HIP runtime error" : g_last_hip_error.c_str();
    case BN_ENONPHYS: return "non-physical state (alpha rho <= 0, alpha <= 0 or not finite)";
    case BN_EUNSUPPORTED: return "solid cell above a fluid cell in one column";
    case BN_ENOMEM: return "device allocation failed";
    case BN_EINTERNAL: return "internal error of the step kernel's work distribution";
    default: return "unknown error";
    }
}

}  // extern "C"
