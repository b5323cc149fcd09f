// Host side of the C ABI declared in include/bn2d.h: context, device buffers, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/bn2d.h"
#include "bn2d_physics.h"

namespace bn {
struct Control {
    const int *jb;
    const long long *S_in;
    long long *S_out;
    long long *S_clear;
    double fix_scale, fix_inv;
    unsigned long long *desc;
    int *nranges;
    unsigned long long *desc_next;
    int *nranges_next;
    const float *cost_in;
    float *cost_out;
    const double *Ts_in;
    double *Ts_out;
    double *Ts_clear;
    const unsigned long long *lam_in;
    unsigned long long *lam_out;
    unsigned long long *lam_clear;
    double *t;
    int *flag;
    int B;
    int ny;
    int nstrips;
    int R0;
    int max_slots;
    int P;
};
struct StepArgs {
    const double *Q;
    double *Qn;
    const uint8_t *solid;
    unsigned long long kaddr;
    unsigned long long caddr;
    double dt_arg;
    int cfl_dt;
    int nx, ny, B;
};
__global__ void step_kernel(StepArgs a);
__global__ void reduce_kernel(const double *Q, const uint8_t *solid, long long *S, double fix_scale,
                              unsigned long long *lam_slot, int *flag, Consts K, int H);
__global__ void dt_kernel(const unsigned long long *lam_slot, double *dt_out, int *flag, Consts K);
__global__ void init_schedule_kernel(unsigned long long *desc, int *nranges, int R0, int max_slots, float *cost,
                                     double *Ts_in, double *Ts_acc, int nstrips, int ny);
__global__ void zero_kernel(long long *p, int n);
__global__ void y0_kernel(const long long *S, const int *jb, double fix_inv, double *y0, Consts K);
}  // namespace bn

namespace {

constexpr int kOutCols = 60;  // output columns per wavefront (64 lanes minus a 2-column halo each side)
constexpr int kDefaultRowsPerBlock = 32;

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

thread_local std::string g_last_hip_error;

// Device buffers.  The fixed-point free-surface integrals rotate through three buffers (a step
// reads S[m], accumulates S[m+1], clears S[m+2], mod 3); dt, the CFL maximum and the range lists
// through two (a step reads slot p and writes slot p^1).
struct Dev {
    double *q[2] = {nullptr, nullptr};
    uint8_t *solid = nullptr;
    int *jb = nullptr;
    long long *S = nullptr;              // [3][nx]
    double *y0 = nullptr;                // [nx], bn_get_y0 staging
    unsigned long long *desc = nullptr;  // [2][max_slots]
    float *cost = nullptr;               // [2][nstrips][ny] recorded march cost per row
    double *Ts = nullptr;                // [3][nstrips] recorded march cost per strip
    int *nranges = nullptr;              // [2]
    unsigned long long *lam = nullptr;   // [3] CFL rate maxima
    int *flag = nullptr;
    double *dt = nullptr;                // dt query staging
    double *t = nullptr;
    bn::Consts *kc = nullptr;            // the physical constants, read by the step kernel
    bn::Control *ctl = nullptr;          // [6]: one per (slot parity, integral buffer) combination
};

}  // namespace

struct bn_ctx {
    bn_grid grid;
    bn_params params;
    bn::Consts K;
    hipStream_t stream;
    Dev d;
    int cur = 0;       // state buffer holding the current state
    int par = 0;       // slot of dt / CFL maximum / range list read by the next step
    int m3 = 0;        // fixed-point buffer holding the current state's free-surface integral
    int B = 32;        // rows per claim
    int P = 1024;      // wavefronts per launch
    int P_default = 1024;
    int nstrips = 0, R0 = 0, max_slots = 0, slots_alloc = 0;
    double fix_scale = 0.0, fix_inv = 0.0;
    bool has_state = false;
};

namespace {

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

// Launch shape: descriptors for one range per wavefront, one unowned strip head per strip, and
// up to 16 splits per wavefront (a split beyond that is marched unpublished).
int set_shape(bn_ctx *c)
{
    c->R0 = c->P + c->nstrips;
    const long long slots = (long long)c->R0 + 16ll * c->P;
    if (slots > (1ll << 30)) return BN_EINVAL;
    c->max_slots = (int)slots;
    if (c->max_slots > c->slots_alloc) {
        if (c->d.desc) {
            HIP_TRY(hipFree(c->d.desc));
            c->d.desc = nullptr;
        }
        hipError_t e = hipMalloc(&c->d.desc, sizeof(unsigned long long) * 2 * (size_t)c->max_slots);
        if (e != hipSuccess) {
            c->d.desc = nullptr;
            c->slots_alloc = 0;
            g_last_hip_error = std::string("hipMalloc(ranges): ") + hipGetErrorString(e);
            return BN_ENOMEM;
        }
        c->slots_alloc = c->max_slots;
    }
    return BN_OK;
}

// Control blocks of the six combinations of range/dt slot p (mod 2) and integral buffer m (mod 3);
// a step reads combination 3 p + m.
int write_controls(bn_ctx *c)
{
    bn::Control h[6];
    const size_t nx = c->grid.nx;
    for (int p = 0; p < 2; ++p)
        for (int m = 0; m < 3; ++m) {
            bn::Control &C = h[3 * p + m];
            const int q = p ^ 1;
            C.jb = c->d.jb;
            C.S_in = c->d.S + m * nx;
            C.S_out = c->d.S + ((m + 1) % 3) * nx;
            C.S_clear = c->d.S + ((m + 2) % 3) * nx;
            C.fix_scale = c->fix_scale;
            C.fix_inv = c->fix_inv;
            C.desc = c->d.desc + (size_t)p * c->max_slots;
            C.nranges = c->d.nranges + p;
            C.desc_next = c->d.desc + (size_t)q * c->max_slots;
            C.nranges_next = c->d.nranges + q;
            const size_t ns = c->nstrips, cells = ns * c->grid.ny;
            C.cost_in = c->d.cost + p * cells;
            C.cost_out = c->d.cost + q * cells;
            C.Ts_in = c->d.Ts + m * ns;
            C.Ts_out = c->d.Ts + ((m + 1) % 3) * ns;
            C.Ts_clear = c->d.Ts + ((m + 2) % 3) * ns;
            C.lam_in = c->d.lam + m;
            C.lam_out = c->d.lam + (m + 1) % 3;
            C.lam_clear = c->d.lam + (m + 2) % 3;
            C.t = c->d.t;
            C.flag = c->d.flag;
            C.B = c->B;
            C.ny = c->grid.ny;
            C.nstrips = c->nstrips;
            C.R0 = c->R0;
            C.max_slots = c->max_slots;
            C.P = c->P;
        }
    HIP_TRY(hipMemcpyAsync(c->d.ctl, h, sizeof(h), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return BN_OK;
}

// Schedule state for the next step (slot par, strip totals m3), after bn_set_state or a change of
// the launch shape: uniform recorded costs, so the next step cuts every strip evenly.
int init_ranges(bn_ctx *c)
{
    const long long n = std::max<long long>((long long)c->nstrips * c->grid.ny, c->max_slots);
    const size_t ns = c->nstrips;
    hipLaunchKernelGGL(bn::init_schedule_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                       c->d.desc + (size_t)c->par * c->max_slots, c->d.nranges + c->par, c->R0, c->max_slots,
                       c->d.cost + (size_t)c->par * ns * c->grid.ny, c->d.Ts + (size_t)c->m3 * ns,
                       c->d.Ts + (size_t)((c->m3 + 1) % 3) * ns, c->nstrips, c->grid.ny);
    HIP_TRY(hipGetLastError());
    return BN_OK;
}

int zero_S(bn_ctx *c, int m)
{
    const int nx = c->grid.nx;
    hipLaunchKernelGGL(bn::zero_kernel, dim3((nx + 255) / 256), dim3(256), 0, c->stream,
                       c->d.S + (size_t)m * nx, nx);
    HIP_TRY(hipGetLastError());
    return BN_OK;
}

// Free-surface integral S[m3] and CFL dt[par] of the current state (no time advance); S[m3+1]
// is cleared for the next step's accumulation.
int refresh_reductions(bn_ctx *c)
{
    const int m = c->m3;
    int rc = zero_S(c, m);
    if (!rc) rc = zero_S(c, (m + 1) % 3);
    if (rc) return rc;
    const int H = 64;
    const dim3 rgrid((c->grid.nx + 63) / 64, (c->grid.ny + H - 1) / H);
    hipLaunchKernelGGL(bn::reduce_kernel, rgrid, dim3(64), 0, c->stream, c->d.q[c->cur], c->d.solid,
                       c->d.S + (size_t)m * c->grid.nx, c->fix_scale, c->d.lam + m, c->d.flag, c->K, H);
    HIP_TRY(hipGetLastError());
    return init_ranges(c);
}

// One step: reads state cur, S[m3], dt[par], ranges[par]; writes state 1-cur, S[m3+1],
// dt[par^1], ranges[par^1], and clears S[m3+2].
int launch_step(bn_ctx *c, bool device_dt, double dt_arg)
{
    const int p = c->par, m = c->m3;
    bn::StepArgs a;
    a.Q = c->d.q[c->cur];
    a.Qn = c->d.q[1 - c->cur];
    a.solid = c->d.solid;
    a.kaddr = (unsigned long long)(uintptr_t)c->d.kc;
    a.caddr = (unsigned long long)(uintptr_t)(c->d.ctl + 3 * p + m);
    a.dt_arg = dt_arg;
    a.cfl_dt = device_dt ? 1 : 0;
    a.nx = c->grid.nx;
    a.ny = c->grid.ny;
    a.B = c->B;
    hipLaunchKernelGGL(bn::step_kernel, dim3(c->P), dim3(64), 0, c->stream, a);
    HIP_TRY(hipGetLastError());
    c->cur = 1 - c->cur;
    c->par = p ^ 1;
    c->m3 = (m + 1) % 3;
    return BN_OK;
}

void free_all(bn_ctx *c)
{
    Dev &d = c->d;
    void *ptrs[] = {d.q[0], d.q[1], d.solid, d.jb, d.S, d.y0, d.desc, d.cost, d.Ts, d.nranges, d.lam, d.flag,
                    d.dt, d.t, d.kc, d.ctl};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    d = Dev();
}

// dt = CFL / max rate of the current state into d.dt (stream-ordered).
int query_dt(bn_ctx *c)
{
    hipLaunchKernelGGL(bn::dt_kernel, dim3(1), dim3(64), 0, c->stream, c->d.lam + c->m3, c->d.dt, c->d.flag, c->K);
    HIP_TRY(hipGetLastError());
    return BN_OK;
}

int sync_flag(bn_ctx *c)
{
    int flag = 0;
    HIP_TRY(hipMemcpyAsync(&flag, c->d.flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (flag & 4) return BN_EINTERNAL;
    return flag ? BN_ENONPHYS : BN_OK;
}

}  // namespace

extern "C" {

int bn_create(const bn_grid *grid, const bn_params *params, const uint8_t *solid, void *hip_stream, bn_ctx **out)
{
    if (!grid || !params || !out) return BN_EINVAL;
    *out = nullptr;
    if (grid->nx <= 0 || grid->ny <= 0 || !(grid->x1 > grid->x0) || !(grid->y1 > grid->y0)) return BN_EINVAL;
    const bn_params &p = *params;
    if (!(p.k0 > 0.0) || !(p.rho0 > 0.0) || !(p.alpha_gas > 0.0) || !(p.alpha_liq > p.alpha_gas) ||
        !(p.alpha_liq <= 1.0) || !(p.cfl > 0.0) || !(p.cfl <= 1.0) || !(p.g >= 0.0) || !std::isfinite(p.g) ||
        !std::isfinite(p.k0) || !std::isfinite(p.rho0))
        return BN_EINVAL;
    for (int s = 0; s < 4; ++s)
        if (p.bc[s] != 0 && p.bc[s] != 1) return BN_EINVAL;

    const int nx = grid->nx, ny = grid->ny;
    // first fluid row of each column; solid cells above a fluid cell are not supported (Sec. 3.5)
    std::vector<int> jb(nx, 0);
    if (solid) {
        for (int i = 0; i < nx; ++i) {
            int j = 0;
            while (j < ny && solid[(size_t)j * nx + i]) ++j;
            jb[i] = j;
            for (int jj = j; jj < ny; ++jj)
                if (solid[(size_t)jj * nx + i]) return BN_EUNSUPPORTED;
        }
    }

    bn_ctx *c = new (std::nothrow) bn_ctx();
    if (!c) return BN_ENOMEM;
    c->grid = *grid;
    c->params = p;
    c->stream = (hipStream_t)hip_stream;

    bn::Consts &K = c->K;
    std::memset(&K, 0, sizeof(K));
    K.nx = nx;
    K.ny = ny;
    K.dx = (grid->x1 - grid->x0) / nx;
    K.dy = (grid->y1 - grid->y0) / ny;
    K.ylo = grid->y0;
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
    c->nstrips = (nx + kOutCols - 1) / kOutCols;
    if (c->nstrips > 0x7FFF || ny > 0xFF0000) {
        delete c;
        return BN_EINVAL;
    }
    c->P_default = default_wavefronts();
    c->P = c->P_default;
    // fixed point: terms (alpha - alpha_g)/(alpha_l - alpha_g) lie in about [0, 1]; 2^f leaves
    // a factor 2 of headroom for ny of them in a signed 64-bit integer
    int lg = 0;
    while ((1ll << lg) < (long long)ny + 1) ++lg;
    c->fix_scale = std::ldexp(1.0, 61 - lg);
    c->fix_inv = std::ldexp(1.0, lg - 61);

    const size_t plane = (size_t)nx * ny;
    auto fail = [&](int code) {
        free_all(c);
        delete c;
        return code;
    };
    hipError_t e;
#define ALLOC(ptr, bytes)                                                          \
    e = hipMalloc(&(ptr), (bytes));                                                \
    if (e != hipSuccess) {                                                         \
        g_last_hip_error = std::string("hipMalloc: ") + hipGetErrorString(e);      \
        return fail(BN_ENOMEM);                                                    \
    }
    ALLOC(c->d.q[0], sizeof(double) * 4 * plane);
    ALLOC(c->d.q[1], sizeof(double) * 4 * plane);
    ALLOC(c->d.jb, sizeof(int) * nx);
    ALLOC(c->d.S, sizeof(long long) * 3 * nx);
    ALLOC(c->d.cost, sizeof(float) * 2 * (size_t)c->nstrips * ny);
    ALLOC(c->d.Ts, sizeof(double) * 3 * (size_t)c->nstrips);
    ALLOC(c->d.y0, sizeof(double) * nx);
    ALLOC(c->d.nranges, sizeof(int) * 2);
    ALLOC(c->d.lam, sizeof(unsigned long long) * 3);
    ALLOC(c->d.flag, sizeof(int));
    ALLOC(c->d.dt, sizeof(double));
    ALLOC(c->d.t, sizeof(double));
    ALLOC(c->d.kc, sizeof(bn::Consts));
    ALLOC(c->d.ctl, sizeof(bn::Control) * 6);
    if (solid) {
        ALLOC(c->d.solid, plane);
    }
#undef ALLOC
    int rc = set_shape(c);
    if (rc) return fail(rc);
    e = hipMemcpy(c->d.jb, jb.data(), sizeof(int) * nx, hipMemcpyHostToDevice);
    if (e == hipSuccess && solid) e = hipMemcpy(c->d.solid, solid, plane, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(c->d.lam, 0, sizeof(unsigned long long) * 3);
    if (e == hipSuccess) e = hipMemset(c->d.flag, 0, sizeof(int));
    if (e == hipSuccess) e = hipMemset(c->d.dt, 0, sizeof(double));
    if (e == hipSuccess) e = hipMemset(c->d.t, 0, sizeof(double));
    if (e == hipSuccess) e = hipMemset(c->d.S, 0, sizeof(long long) * 3 * nx);
    if (e == hipSuccess) e = hipMemset(c->d.nranges, 0, sizeof(int) * 2);
    if (e == hipSuccess) e = hipMemcpy(c->d.kc, &c->K, sizeof(bn::Consts), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        g_last_hip_error = std::string("bn_create: ") + hipGetErrorString(e);
        return fail(BN_EHIP);
    }
    rc = write_controls(c);
    if (rc) return fail(rc);
    *out = c;
    return BN_OK;
}

int bn_set_state(bn_ctx *c, const double *q_dev)
{
    if (!c || !q_dev) return BN_EINVAL;
    const size_t bytes = sizeof(double) * 4 * (size_t)c->grid.nx * c->grid.ny;
    HIP_TRY(hipMemcpyAsync(c->d.q[c->cur], q_dev, bytes, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemsetAsync(c->d.flag, 0, sizeof(int), c->stream));
    HIP_TRY(hipMemsetAsync(c->d.t, 0, sizeof(double), c->stream));
    HIP_TRY(hipMemsetAsync(c->d.lam, 0, sizeof(unsigned long long) * 3, c->stream));
    int rc = refresh_reductions(c);
    if (rc) return rc;
    c->has_state = true;
    return BN_OK;
}

int bn_get_state(bn_ctx *c, double *q_dev)
{
    if (!c || !q_dev || !c->has_state) return BN_EINVAL;
    const size_t bytes = sizeof(double) * 4 * (size_t)c->grid.nx * c->grid.ny;
    HIP_TRY(hipMemcpyAsync(q_dev, c->d.q[c->cur], bytes, hipMemcpyDeviceToDevice, c->stream));
    return BN_OK;
}

int bn_compute_dt(bn_ctx *c, double *dt_host)
{
    if (!c || !dt_host || !c->has_state) return BN_EINVAL;
    int rc = query_dt(c);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(dt_host, c->d.dt, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    return sync_flag(c);
}

int bn_step(bn_ctx *c, double dt)
{
    if (!c || !c->has_state || !(dt > 0.0) || !std::isfinite(dt)) return BN_EINVAL;
    return launch_step(c, false, dt);
}

int bn_run(bn_ctx *c, int32_t n_steps)
{
    if (!c || !c->has_state || n_steps < 0) return BN_EINVAL;
    for (int32_t s = 0; s < n_steps; ++s) {
        int rc = launch_step(c, true, 0.0);
        if (rc) return rc;
    }
    return BN_OK;
}

int bn_get_time(bn_ctx *c, double *t_host, double *next_dt_host)
{
    if (!c || !c->has_state) return BN_EINVAL;
    double tmp[2];
    HIP_TRY(hipMemcpyAsync(&tmp[0], c->d.t, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    int rc = query_dt(c);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(&tmp[1], c->d.dt, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    rc = sync_flag(c);
    if (t_host) *t_host = tmp[0];
    if (next_dt_host) *next_dt_host = tmp[1];
    return rc;
}

int bn_get_y0(bn_ctx *c, double *y0_host)
{
    if (!c || !y0_host || !c->has_state) return BN_EINVAL;
    const int nx = c->grid.nx;
    hipLaunchKernelGGL(bn::y0_kernel, dim3((nx + 255) / 256), dim3(256), 0, c->stream,
                       c->d.S + (size_t)c->m3 * nx, c->d.jb, c->fix_inv, c->d.y0, c->K);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(y0_host, c->d.y0, sizeof(double) * nx, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return BN_OK;
}

int bn_status(bn_ctx *c)
{
    if (!c) return BN_EINVAL;
    return sync_flag(c);
}

int bn_set_launch(bn_ctx *c, int32_t rows_per_block, int32_t wavefronts)
{
    if (!c || rows_per_block < 0 || rows_per_block > 4096 || wavefronts < 0 || wavefronts > 65536) return BN_EINVAL;
    const int B = rows_per_block ? rows_per_block : kDefaultRowsPerBlock;
    const int P = wavefronts ? wavefronts : c->P_default;
    if (B == c->B && P == c->P) return BN_OK;
    HIP_TRY(hipStreamSynchronize(c->stream));
    const int oldB = c->B, oldP = c->P;
    c->B = B;
    c->P = P;
    int rc = set_shape(c);
    if (!rc) rc = write_controls(c);
    if (rc) {
        c->B = oldB;
        c->P = oldP;
        if (!set_shape(c)) (void)write_controls(c);
        return rc;
    }
    // the next step's range list follows the new shape; y0, dt and t of the current state stay
    return c->has_state ? init_ranges(c) : BN_OK;
}

int bn_get_launch(bn_ctx *c, int32_t *rows_per_block, int32_t *wavefronts)
{
    if (!c) return BN_EINVAL;
    if (rows_per_block) *rows_per_block = c->B;
    if (wavefronts) *wavefronts = c->P;
    return BN_OK;
}

void bn_destroy(bn_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
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
