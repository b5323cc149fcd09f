// Attainable-peak probes for the roofline of the step kernel (measurement only, not part of the
// method's ABI): FP64 FMA throughput on the vector ALUs and HBM bandwidth of a triad.
#include <hip/hip_runtime.h>
#include <stdint.h>

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

}  // namespace

extern "C" {

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
