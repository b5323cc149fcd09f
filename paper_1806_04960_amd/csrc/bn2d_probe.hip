// Probes beside the library (measurement only, not part of the method's ABI): attainable peaks for
// the step kernel's roofline (FP64 FMA throughput on the vector ALUs, HBM bandwidth of a triad), and
// the accuracy of the reciprocal the physics uses (bn::rcp: the hardware estimate refined by one
// Newton step) against the correctly rounded quotient.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bn2d_physics.h"

namespace {

constexpr int kChains = 8;   // independent FMA chains per lane (hide the FMA latency)
constexpr int kUnroll = 16;

__global__ __launch_bounds__(256) void fma_kernel(double *out, double a, double b, int iters)
{
    double x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = threadIdx.x * 1e-3 + c;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int c = 0; c < kChains; ++c) x[c] = fma(x[c], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void triad_kernel(double *a, const double *b, const double *c, double s, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        a[i] = b[i] + s * c[i];
}

// distance in units of the last place between bn::rcp(x) and the correctly rounded 1/x, for n
// log-uniformly spaced x in [2^lo, 2^hi]; the largest into *worst
__global__ __launch_bounds__(256) void rcp_kernel(long long n, double lo, double hi, unsigned long long *worst)
{
    unsigned long long m = 0;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
        const double x = exp2(lo + (hi - lo) * ((double)k + 0.5) / (double)n);
        const double r = bn::rcp(x), q = 1.0 / x;
        const long long d = __double_as_longlong(r) - __double_as_longlong(q);
        const unsigned long long u = (unsigned long long)(d < 0 ? -d : d);
        m = u > m ? u : m;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(worst, m);
}

}  // namespace

extern "C" {

// Largest distance in ulps between the physics' reciprocal and 1/x over n log-uniform x in
// [2^lo, 2^hi] (x > 0): 0 and *max_ulps, or a negative code.
int bn_probe_rcp(long long n, double lo, double hi, unsigned long long *max_ulps)
{
    if (n <= 0 || !(hi > lo) || !max_ulps) return -1;
    unsigned long long *w = nullptr;
    if (hipMalloc(&w, sizeof(unsigned long long)) != hipSuccess) return -2;
    hipError_t e = hipMemset(w, 0, sizeof(unsigned long long));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(rcp_kernel, dim3(1024), dim3(256), 0, 0, n, lo, hi, w);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(max_ulps, w, sizeof(unsigned long long), hipMemcpyDeviceToHost);
    (void)hipFree(w);
    return e == hipSuccess ? 0 : -2;
}

// FP64 FMA rate: `blocks` x 256 threads, each `iters` x 16 x 8 dependent-free FMAs.  Returns 0 and
// the FLOP/s (2 per FMA) of the best of `reps` launches, or a HIP error code.
int bn_probe_fma(int blocks, int iters, int reps, double *flops_per_s)
{
    if (blocks <= 0 || iters <= 0 || reps <= 0 || !flops_per_s) return -1;
    double *out = nullptr;
    hipEvent_t e0, e1;
    if (hipMalloc(&out, sizeof(double) * (size_t)blocks * 256) != hipSuccess) return -2;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best = 1e30f;
    for (int r = 0; r < reps + 1; ++r) {
        (void)hipEventRecord(e0, 0);
        hipLaunchKernelGGL(fma_kernel, dim3(blocks), dim3(256), 0, 0, out, 0.999999, 1e-7, iters);
        (void)hipEventRecord(e1, 0);
        (void)hipEventSynchronize(e1);
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (r > 0 && ms < best) best = ms;  // the first launch warms up
    }
    const hipError_t err = hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (err != hipSuccess) return -3;
    *flops_per_s = 2.0 * kChains * kUnroll * (double)iters * blocks * 256 / (best * 1e-3);
    return 0;
}

// Triad a = b + s c over n doubles: bytes moved (24 n) per second, best of `reps`.
int bn_probe_triad(long long n, int reps, double *bytes_per_s)
{
    if (n <= 0 || reps <= 0 || !bytes_per_s) return -1;
    double *a = nullptr, *b = nullptr, *c = nullptr;
    if (hipMalloc(&a, sizeof(double) * n) != hipSuccess) return -2;
    if (hipMalloc(&b, sizeof(double) * n) != hipSuccess || hipMalloc(&c, sizeof(double) * n) != hipSuccess) {
        (void)hipFree(a);
        if (b) (void)hipFree(b);
        return -2;
    }
    (void)hipMemset(b, 0, sizeof(double) * n);
    (void)hipMemset(c, 0, sizeof(double) * n);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best = 1e30f;
    const int blocks = 256 * 32;
    for (int r = 0; r < reps + 1; ++r) {
        (void)hipEventRecord(e0, 0);
        hipLaunchKernelGGL(triad_kernel, dim3(blocks), dim3(256), 0, 0, a, b, c, 1.5, (size_t)n);
        (void)hipEventRecord(e1, 0);
        (void)hipEventSynchronize(e1);
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (r > 0 && ms < best) best = ms;
    }
    const hipError_t err = hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    (void)hipFree(c);
    if (err != hipSuccess) return -3;
    *bytes_per_s = 24.0 * (double)n / (best * 1e-3);
    return 0;
}

}  // extern "C"
