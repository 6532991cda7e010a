// Connectivity of the active tetrahedra (paper Sec. 3.6: rebuilt from the
// current mask; Alg. 1 keeps it with the mask), on gfx950.
//
// Two active tets are connected when they share a vertex (the components of
// the assembled operator).  Components are found over the vertices by
// hooking roots and shortcutting (a Shiloach-Vishkin style iteration): every
// vertex keeps a parent pointer f, initially itself; in a hooking pass each
// active tet climbs from its four vertices to their roots and lowers the
// larger roots (and the vertices) to the smallest one with atomic minimum; a
// shortcut pass points every vertex at the root it reaches.  Pointers only
// decrease and stay inside the component, so when a hooking pass changes no
// root, every component is one tree whose root is its smallest vertex.  A
// tet's label is that vertex, independent of execution order.
//
// Each pass is its own launch: within a pass, loads may see another XCD's
// stale copy of a pointer, which only delays convergence (every update is a
// monotone atomic minimum); the launch boundary makes all updates visible to
// the next pass.  The host checks a change flag after each hooking pass.
#include <hip/hip_runtime.h>

#include "sta_internal.h"

namespace sta {
namespace {

constexpr int kBlock = 256;

unsigned blocks(int64_t n)
{
    return (unsigned)((n + kBlock - 1) / kBlock);
}

// flag[0]: changed in this pass; flag[1]: number of components
__global__ __launch_bounds__(kBlock) void k_cc_init(int n_nodes, int* f, uint32_t* mark)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n_nodes) {
        f[i] = i;
        mark[i] = 0u;
    }
}

// Follow parent pointers from x towards its root (at most kMaxSteps hops:
// any vertex reached is an ancestor, which is all the passes need).
constexpr int kMaxSteps = 1 << 16;

__device__ __forceinline__ int climb(const int* f, int x)
{
    for (int s = 0; s < kMaxSteps; ++s) {
        const int p = f[x];
        if (p == x)
            break;
        x = p;
    }
    return x;
}

// Hooking pass: each active tet lowers the roots of its four vertices (and
// the vertices themselves) to the smallest of those roots.
__global__ __launch_bounds__(kBlock) void k_cc_hook(DevView v, int* f, uint32_t* flag)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= v.n_tets || !v.mask[e])
        return;
    const int4 t = v.T[e];
    const int x[4] = {t.x, t.y, t.z, t.w};
    int r[4], m = INT32_MAX;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        r[k] = climb(f, x[k]);
        m = r[k] < m ? r[k] : m;
    }
    bool changed = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (r[k] > m) {
            changed |= atomicMin(f + r[k], m) > m;
            changed |= atomicMin(f + x[k], m) > m;
        }
    }
    if (changed)
        flag[0] = 1u;
}

// Shortcut pass: every pointer to the root it reaches (only thread i writes f[i]).
__global__ __launch_bounds__(kBlock) void k_cc_shortcut(int n_nodes, int* f, uint32_t* flag)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_nodes)
        return;
    const int p = f[i];
    const int r = climb(f, p);
    if (r < p) {
        f[i] = r;
        flag[0] = 1u;
    }
}

// Label every tet with its component's root (-1 if inactive) and mark the
// vertices of active tets (plain stores: many tets share a vertex).
__global__ __launch_bounds__(kBlock) void k_cc_label(DevView v, const int* __restrict__ f,
                                                     int32_t* __restrict__ label, uint32_t* mark)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= v.n_tets)
        return;
    int32_t l = -1;
    if (v.mask[e]) {
        const int4 t = v.T[e];
        l = f[t.x];
        mark[t.x] = 1u;
        mark[t.y] = 1u;
        mark[t.z] = 1u;
        mark[t.w] = 1u;
    }
    label[e] = l;
}

// Components = marked vertices that are their own root (each component's
// root is its smallest vertex, which belongs to an active tet).
__global__ __launch_bounds__(kBlock) void k_cc_count(int n_nodes, const int* __restrict__ f,
                                                     const uint32_t* __restrict__ mark, uint32_t* flag)
{
    __shared__ uint32_t s_count;
    if (threadIdx.x == 0)
        s_count = 0u;
    __syncthreads();
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n_nodes && mark[i] && f[i] == i)
        atomicAdd(&s_count, 1u);
    __syncthreads();
    if (threadIdx.x == 0 && s_count)
        atomicAdd(flag + 1, s_count);
}

}  // namespace

// Component labels into label (device, n_tets); *n_components on the host.
// Synchronises s.  Returns hipErrorUnknown if the iteration bound is hit.
hipError_t run_components(const DevView& v, int* f, uint32_t* mark, uint32_t* flag, uint32_t* host_flag,
                          int32_t* label, int64_t* n_components, int* passes, hipStream_t s)
{
    const unsigned gn = v.n_nodes > 0 ? blocks(v.n_nodes) : 1u;
    hipLaunchKernelGGL(k_cc_init, dim3(gn), dim3(kBlock), 0, s, v.n_nodes, f, mark);
    hipError_t e = hipGetLastError();
    *passes = 0;
    // hooking passes until one changes nothing (then its reads were exact, so
    // every active tet's vertices share one root), each followed by one
    // shortcut; then shortcuts until every tree is a star.  Every pass that
    // does not end its loop lowers some pointer, so the loop is bounded; the
    // bound below is far above what a correct pass sequence needs.
    for (int phase = 0; phase < 2 && e == hipSuccess; ++phase) {
        for (int it = 0;; ++it) {
            if (it > v.n_nodes + 2)
                return hipErrorUnknown;
            e = hipMemsetAsync(flag, 0, sizeof(uint32_t), s);
            if (e == hipSuccess && phase == 0 && v.n_tets > 0) {
                hipLaunchKernelGGL(k_cc_hook, dim3(blocks(v.n_tets)), dim3(kBlock), 0, s, v, f, flag);
                e = hipGetLastError();
            }
            if (e == hipSuccess && v.n_nodes > 0) {
                hipLaunchKernelGGL(k_cc_shortcut, dim3(gn), dim3(kBlock), 0, s, v.n_nodes, f, flag + (phase == 0));
                e = hipGetLastError();
            }
            if (e == hipSuccess)
                e = hipMemcpyAsync(host_flag, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess)
                e = hipStreamSynchronize(s);
            if (e != hipSuccess)
                return e;
            ++*passes;
            if (*host_flag == 0u)
                break;
        }
    }
    if (e == hipSuccess)
        e = hipMemsetAsync(flag + 1, 0, sizeof(uint32_t), s);
    if (e == hipSuccess && v.n_tets > 0) {
        hipLaunchKernelGGL(k_cc_label, dim3(blocks(v.n_tets)), dim3(kBlock), 0, s, v, f, label, mark);
        e = hipGetLastError();
    }
    if (e == hipSuccess && v.n_nodes > 0) {
        hipLaunchKernelGGL(k_cc_count, dim3(gn), dim3(kBlock), 0, s, v.n_nodes, f, mark, flag);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(host_flag, flag + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e == hipSuccess)
        *n_components = *host_flag;
    return e;
}

}  // namespace sta

using namespace sta;

extern "C" sta_status sta_components(sta_ctx* ctx, int32_t* labels_dev, int64_t* n_components, void* stream)
{
    if (!ctx || (ctx->n_tets > 0 && !labels_dev))
        return STA_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t n = (size_t)(ctx->n_nodes ? ctx->n_nodes : 1);
    hipError_t e = hipSuccess;
    if (!ctx->cc_ws) {
        void* q = nullptr;
        e = hipMalloc(&q, sizeof(int32_t) * 2 * n + 256);  // parent and mark per vertex, 2 flags
        if (e != hipSuccess) {
            ctx->errmsg = std::string("connectivity workspace: ") + hipGetErrorString(e);
            return STA_ENOMEM;
        }
        ctx->owned.push_back(q);
        ctx->cc_ws = static_cast<int32_t*>(q);
        e = hipHostMalloc((void**)&ctx->cc_host, sizeof(uint32_t), hipHostMallocDefault);
        if (e != hipSuccess) {
            ctx->cc_host = nullptr;
            ctx->errmsg = std::string("connectivity host flag: ") + hipGetErrorString(e);
            return STA_ENOMEM;
        }
    }
    int* f = ctx->cc_ws;
    uint32_t* mark = reinterpret_cast<uint32_t*>(ctx->cc_ws + n);
    uint32_t* flag = mark + n;
    int64_t k = 0;
    e = run_components(ctx->v, f, mark, flag, ctx->cc_host, labels_dev, &k, &ctx->cc_passes, s);
    if (e == hipErrorUnknown) {
        ctx->errmsg = "connectivity: pass bound exceeded (labels invalid)";
        return STA_EHIP;
    }
    if (e != hipSuccess) {
        ctx->errmsg = std::string("connectivity: ") + hipGetErrorString(e);
        return STA_EHIP;
    }
    if (n_components)
        *n_components = k;
    return STA_OK;
}
