// Latency probe: the floor under which a streaming frame cannot go on this
// GPU, measured rather than assumed.  One lane walks a dependent chain
// (each address comes from the previous load) and reads the 100 MHz
// real-time counter around it; the same for a chain of returning atomics.
// Together with the duration of an empty kernel this bounds a frame built
// from two launches of a few dependent memory round trips each.
#include <hip/hip_runtime.h>

#include <vector>

#include "sta_internal.h"

namespace sta {

namespace {

// chase[i] = (i + stride) mod n, stride coprime with n and larger than a
// cache line, so consecutive hops hit different lines.
__global__ void k_chase_init(uint32_t* chase, uint32_t n, uint32_t stride)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        chase[i] = (uint32_t)(((uint64_t)i + stride) % n);
}

__global__ void k_chase(const uint32_t* __restrict__ chase, int hops, uint64_t* out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    uint32_t p = 0;
    for (int h = 0; h < 16; ++h)  // warm up along the start of the walk
        p = chase[p];
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (int h = 0; h < hops; ++h)
        p = chase[p];
    const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
    out[0] = t1 - t0;
    out[1] = p;  // keeps the chain live
}

// A chain of returning device-scope atomics: each target depends on the previous result.
__global__ void k_atomic_chain(uint32_t* __restrict__ chase, int hops, uint64_t* out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    uint32_t p = 0;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (int h = 0; h < hops; ++h)
        p = atomicAdd(chase + p, 0u);
    const uint64_t t1 = __builtin_amdgcn_s_memrealtime();
    out[0] = t1 - t0;
    out[1] = p;
}

__global__ void k_empty() {}

// One grid barrier (the fused frame's, grid_barrier) and nothing else.
__global__ __launch_bounds__(256) void k_barrier_only(Ctl* ctl, unsigned spin_limit)
{
    __shared__ int s_ok;
    (void)grid_barrier(ctl, gridDim.x, spin_limit, &s_ok);
}

// Streaming bandwidth kernels: 16-byte accesses, consecutive lanes on
// consecutive addresses, grid-stride over the buffer.
typedef double dvec2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void k_bw_read(const dvec2* __restrict__ src, int64_t n, double* out)
{
    double acc = 0.0;
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const dvec2 x = src[i];
        acc += x.x + x.y;
    }
    if (acc == -1.0)  // never true for the positive fill; keeps the loads live
        out[0] = acc;
}

__global__ __launch_bounds__(256) void k_bw_write(dvec2* __restrict__ dst, int64_t n)
{
    const dvec2 one = {1.0, 1.0};
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        dst[i] = one;
}

__global__ __launch_bounds__(256) void k_bw_copy(const dvec2* __restrict__ src, dvec2* __restrict__ dst, int64_t n)
{
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        dst[i] = src[i];
}

}  // namespace

}  // namespace sta

using namespace sta;

extern "C" sta_status sta_latency_probe(void* stream, double* out4)
{
    if (!out4)
        return STA_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint32_t n_big = 64u << 20;  // 256 MB of uint32: beyond L2 and the 256 MB Infinity Cache working set
    const uint32_t n_small = 256u << 10;  // 1 MB: L2 resident
    uint32_t *big = nullptr, *small = nullptr;
    uint64_t* dout = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipMalloc(&big, sizeof(uint32_t) * n_big);
    if (e == hipSuccess) e = hipMalloc(&small, sizeof(uint32_t) * n_small);
    if (e == hipSuccess) e = hipMalloc(&dout, 2 * sizeof(uint64_t));
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    const int hops = 2000;
    uint64_t h[2] = {0, 0};
    double res[4] = {0, 0, 0, 0};
    if (e == hipSuccess) {
        // strides of ~4 KB-2 MB so each hop lands on a new line (and mostly a new page)
        hipLaunchKernelGGL(k_chase_init, dim3(n_big / 256), dim3(256), 0, s, big, n_big, 1000003u);
        hipLaunchKernelGGL(k_chase_init, dim3(n_small / 256), dim3(256), 0, s, small, n_small, 1031u);
        e = hipStreamSynchronize(s);
    }
    // [1] dependent load, working set far beyond the caches
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_chase, dim3(1), dim3(64), 0, s, big, hops, dout);
        e = hipMemcpyAsync(h, dout, sizeof h, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        res[1] = (double)h[0] * 10.0 / hops;  // 100 MHz ticks -> ns per hop
    }
    // [2] dependent load, L2-resident (second walk over a 1 MB buffer)
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_chase, dim3(1), dim3(64), 0, s, small, hops, dout);
        hipLaunchKernelGGL(k_chase, dim3(1), dim3(64), 0, s, small, hops, dout);
        e = hipMemcpyAsync(h, dout, sizeof h, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        res[2] = (double)h[0] * 10.0 / hops;
    }
    // [3] dependent returning atomics on the L2-sized buffer
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_atomic_chain, dim3(1), dim3(64), 0, s, small, hops, dout);
        e = hipMemcpyAsync(h, dout, sizeof h, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        res[3] = (double)h[0] * 10.0 / hops;
    }
    // [0] an empty kernel, launch to completion, averaged over back-to-back launches
    if (e == hipSuccess) {
        const int reps = 200;
        hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, s);
        e = hipEventRecord(a, s);
        for (int r = 0; r < reps && e == hipSuccess; ++r) {
            hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, s);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        res[0] = ms * 1e3 / reps;  // us per back-to-back empty kernel
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (big) (void)hipFree(big);
    if (small) (void)hipFree(small);
    if (dout) (void)hipFree(dout);
    if (e != hipSuccess)
        return STA_EHIP;
    for (int k = 0; k < 4; ++k)
        out4[k] = res[k];
    return STA_OK;
}

extern "C" sta_status sta_bandwidth_probe(void* stream, double* out3)
{
    if (!out3)
        return STA_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t bytes = 1ll << 30;  // per buffer, far beyond the 256 MB Infinity Cache
    const int64_t n = bytes / 16;
    const unsigned grids[4] = {1024, 4096, 16384, 65536};
    const int reps = 10;
    dvec2 *a = nullptr, *b = nullptr;
    double* dout = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&a, bytes);
    if (e == hipSuccess) e = hipMalloc(&b, bytes);
    if (e == hipSuccess) e = hipMalloc(&dout, sizeof(double));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double res[3] = {0, 0, 0};
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_bw_write, dim3(grids[0]), dim3(256), 0, s, a, n);
        hipLaunchKernelGGL(k_bw_write, dim3(grids[0]), dim3(256), 0, s, b, n);
        e = hipGetLastError();
    }
    for (int which = 0; which < 3 && e == hipSuccess; ++which) {
        for (int gi = 0; gi < 4 && e == hipSuccess; ++gi) {
            const dim3 grid(grids[gi]);
            for (int r = -1; r < reps && e == hipSuccess; ++r) {  // r = -1: warm-up
                if (r == 0) e = hipEventRecord(e0, s);
                if (which == 0)
                    hipLaunchKernelGGL(k_bw_read, grid, dim3(256), 0, s, a, n, dout);
                else if (which == 1)
                    hipLaunchKernelGGL(k_bw_write, grid, dim3(256), 0, s, b, n);
                else
                    hipLaunchKernelGGL(k_bw_copy, grid, dim3(256), 0, s, a, b, n);
                if (e == hipSuccess) e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            const double moved = (double)bytes * (which == 2 ? 2 : 1) * reps;
            const double gbs = ms > 0.0f ? moved / (ms * 1e-3) / 1e9 : 0.0;
            if (gbs > res[which])
                res[which] = gbs;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (dout) (void)hipFree(dout);
    if (e != hipSuccess)
        return STA_EHIP;
    for (int k = 0; k < 3; ++k)
        out3[k] = res[k];
    return STA_OK;
}

// Per-unit time of `launch` captured `per` times into one HIP graph on stream s
// and replayed `reps` times, in microseconds.
template <class F>
static hipError_t graph_unit_us(hipStream_t s, int per, int reps, F&& launch, double* us)
{
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    for (int i = 0; i < per && e == hipSuccess; ++i)
        e = launch();
    hipError_t e2 = hipStreamEndCapture(s, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(ge, s);  // warm-up
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r)
        e = hipGraphLaunch(ge, s);
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    *us = ms * 1e3 / ((double)reps * per);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

extern "C" sta_status sta_barrier_probe(double* out7)
{
    if (!out7)
        return STA_EINVAL;
    hipStream_t s = nullptr;
    Ctl* ctl = nullptr;
    int cus = 0, per_cu = 0, dev = 0;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&ctl, sizeof(Ctl));
    if (e == hipSuccess) e = hipMemset(ctl, 0, sizeof(Ctl));
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_barrier_only, 256, 0);
    const int per = 50, reps = 20;
    double r[7];
    for (int k = 0; k < 7; ++k)
        r[k] = -1.0;
    if (e == hipSuccess)
        e = graph_unit_us(s, per, reps, [&] {
            hipLaunchKernelGGL(k_empty, dim3(64), dim3(256), 0, s);
            return hipGetLastError();
        }, &r[0]);
    if (e == hipSuccess)
        e = graph_unit_us(s, per, reps, [&] {
            hipLaunchKernelGGL(k_empty, dim3(64), dim3(256), 0, s);
            hipLaunchKernelGGL(k_empty, dim3(64), dim3(256), 0, s);
            return hipGetLastError();
        }, &r[1]);
    const int grids[5] = {8, 32, 64, 128, 256};
    for (int k = 0; k < 5 && e == hipSuccess; ++k) {
        if (grids[k] > cus * per_cu)
            continue;  // not co-resident: not measured
        e = graph_unit_us(s, per, reps, [&] {
            hipLaunchKernelGGL(k_barrier_only, dim3(grids[k]), dim3(256), 0, s, ctl, kBarrierSpinDefault);
            return hipGetLastError();
        }, &r[2 + k]);
    }
    int32_t err = 0;
    if (e == hipSuccess) e = hipMemcpy(&err, &ctl->err, sizeof(err), hipMemcpyDeviceToHost);
    if (ctl) (void)hipFree(ctl);
    if (s) (void)hipStreamDestroy(s);
    if (e != hipSuccess)
        return STA_EHIP;
    if (err & ERR_TIMEOUT)
        return STA_ETIMEOUT;
    for (int k = 0; k < 7; ++k)
        out7[k] = r[k];
    return STA_OK;
}
