// Host side of the C ABI declared in include/bn2d.h: context, device buffers, launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/bn2d.h"
#include "bn2d_physics.h"

namespace bn {
__global__ void step_kernel(const double *Q, double *Qn, const uint8_t *solid, const double *Y0,
                            const double *dt_dev, double dt_arg, double *partial, unsigned long long *lam_slot,
                            int *flag, Consts K, int H);
__global__ void reduce_kernel(const double *Q, const uint8_t *solid, double *partial,
                              unsigned long long *lam_slot, int *flag, Consts K, int H);
__global__ void finalize_kernel(const double *partial, int nseg, const int *jb, double *Y0,
                                unsigned long long *lam_slot, int *flag, double *dt_dev, double *t_dev,
                                double dt_used, int use_dev_dt, int advance_t, Consts K);
}  // namespace bn

namespace {

constexpr int kOutCols = 60;  // output columns per wavefront (64 lanes minus a 2-column halo each side)

thread_local std::string g_last_hip_error;

struct Dev {
    double *q[2] = {nullptr, nullptr};
    uint8_t *solid = nullptr;
    int *jb = nullptr;
    double *y0 = nullptr;
    double *partial = nullptr;
    unsigned long long *lam = nullptr;
    int *flag = nullptr;
    double *dt = nullptr;
    double *t = nullptr;
};

}  // namespace

struct bn_ctx {
    bn_grid grid;
    bn_params params;
    bn::Consts K;
    hipStream_t stream;
    Dev d;
    int cur = 0;
    int rows = 16;
    int nseg = 0;
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

int alloc_partial(bn_ctx *c)
{
    if (c->d.partial) {
        HIP_TRY(hipFree(c->d.partial));
        c->d.partial = nullptr;
    }
    c->nseg = (c->grid.ny + c->rows - 1) / c->rows;
    const size_t bytes = sizeof(double) * (size_t)c->nseg * c->grid.nx;
    hipError_t e = hipMalloc(&c->d.partial, bytes);
    if (e != hipSuccess) {
        c->d.partial = nullptr;
        g_last_hip_error = std::string("hipMalloc(partial): ") + hipGetErrorString(e);
        return BN_ENOMEM;
    }
    return BN_OK;
}

// Detector partials + CFL rate of the current state, then y0 and dt (no time advance).
int refresh_reductions(bn_ctx *c)
{
    const dim3 rgrid((c->grid.nx + 63) / 64, c->nseg);
    hipLaunchKernelGGL(bn::reduce_kernel, rgrid, dim3(64), 0, c->stream, c->d.q[c->cur], c->d.solid, c->d.partial,
                       c->d.lam, c->d.flag, c->K, c->rows);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(bn::finalize_kernel, dim3((c->grid.nx + 255) / 256), dim3(256), 0, c->stream, c->d.partial,
                       c->nseg, c->d.jb, c->d.y0, c->d.lam, c->d.flag, c->d.dt, c->d.t, 0.0, 0, 0, c->K);
    HIP_TRY(hipGetLastError());
    return BN_OK;
}

int launch_step(bn_ctx *c, const double *dt_dev, double dt_arg)
{
    const dim3 grid((c->grid.nx + kOutCols - 1) / kOutCols, c->nseg);
    hipLaunchKernelGGL(bn::step_kernel, grid, dim3(64), 0, c->stream, c->d.q[c->cur], c->d.q[1 - c->cur],
                       c->d.solid, c->d.y0, dt_dev, dt_arg, c->d.partial, c->d.lam, c->d.flag, c->K, c->rows);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(bn::finalize_kernel, dim3((c->grid.nx + 255) / 256), dim3(256), 0, c->stream, c->d.partial,
                       c->nseg, c->d.jb, c->d.y0, c->d.lam, c->d.flag, c->d.dt, c->d.t, dt_arg, dt_dev ? 1 : 0, 1,
                       c->K);
    HIP_TRY(hipGetLastError());
    c->cur = 1 - c->cur;
    return BN_OK;
}

void free_all(bn_ctx *c)
{
    Dev &d = c->d;
    void *ptrs[] = {d.q[0], d.q[1], d.solid, d.jb, d.y0, d.partial, d.lam, d.flag, d.dt, d.t};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    d = Dev();
}

int sync_flag(bn_ctx *c)
{
    int flag = 0;
    HIP_TRY(hipMemcpyAsync(&flag, c->d.flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
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
    ALLOC(c->d.y0, sizeof(double) * nx);
    ALLOC(c->d.lam, sizeof(unsigned long long));
    ALLOC(c->d.flag, sizeof(int));
    ALLOC(c->d.dt, sizeof(double));
    ALLOC(c->d.t, sizeof(double));
    if (solid) {
        ALLOC(c->d.solid, plane);
    }
#undef ALLOC
    int rc = alloc_partial(c);
    if (rc) return fail(rc);
    e = hipMemcpy(c->d.jb, jb.data(), sizeof(int) * nx, hipMemcpyHostToDevice);
    if (e == hipSuccess && solid) e = hipMemcpy(c->d.solid, solid, plane, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(c->d.lam, 0, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(c->d.flag, 0, sizeof(int));
    if (e == hipSuccess) e = hipMemset(c->d.dt, 0, sizeof(double));
    if (e == hipSuccess) e = hipMemset(c->d.t, 0, sizeof(double));
    if (e == hipSuccess) e = hipMemset(c->d.y0, 0, sizeof(double) * nx);
    if (e != hipSuccess) {
        g_last_hip_error = std::string("bn_create: ") + hipGetErrorString(e);
        return fail(BN_EHIP);
    }
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
    HIP_TRY(hipMemsetAsync(c->d.lam, 0, sizeof(unsigned long long), c->stream));
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
    HIP_TRY(hipMemcpyAsync(dt_host, c->d.dt, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    return sync_flag(c);
}

int bn_step(bn_ctx *c, double dt)
{
    if (!c || !c->has_state || !(dt > 0.0) || !std::isfinite(dt)) return BN_EINVAL;
    return launch_step(c, nullptr, dt);
}

int bn_run(bn_ctx *c, int32_t n_steps)
{
    if (!c || !c->has_state || n_steps < 0) return BN_EINVAL;
    for (int32_t s = 0; s < n_steps; ++s) {
        int rc = launch_step(c, c->d.dt, 0.0);
        if (rc) return rc;
    }
    return BN_OK;
}

int bn_get_time(bn_ctx *c, double *t_host, double *next_dt_host)
{
    if (!c || !c->has_state) return BN_EINVAL;
    double tmp[2];
    HIP_TRY(hipMemcpyAsync(&tmp[0], c->d.t, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(&tmp[1], c->d.dt, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    int rc = sync_flag(c);
    if (t_host) *t_host = tmp[0];
    if (next_dt_host) *next_dt_host = tmp[1];
    return rc;
}

int bn_get_y0(bn_ctx *c, double *y0_host)
{
    if (!c || !y0_host || !c->has_state) return BN_EINVAL;
    HIP_TRY(hipMemcpyAsync(y0_host, c->d.y0, sizeof(double) * c->grid.nx, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return BN_OK;
}

int bn_status(bn_ctx *c)
{
    if (!c) return BN_EINVAL;
    return sync_flag(c);
}

int bn_set_rows_per_block(bn_ctx *c, int32_t rows)
{
    if (!c || rows < 1 || rows > 4096) return BN_EINVAL;
    if (rows == c->rows) return BN_OK;
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->rows = rows;
    int rc = alloc_partial(c);
    if (rc) return rc;
    if (c->has_state) {
        // recompute the partial sums in the new layout (y0, dt and t do not change)
        rc = refresh_reductions(c);
        if (rc) return rc;
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
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
    default: return "unknown error";
    }
}

}  // extern "C"
