// Connectivity of the active tetrahedra (paper Sec. 3.6: rebuilt from the
// current mask; Alg. 1 keeps it with the mask), on gfx950.
//
// The paper does not fix the adjacency; two are provided.  Vertex: two
// active tets are connected when they share a vertex (the components of the
// assembled operator), labelled by the component's smallest vertex.  Face:
// when they share a face (fragments in the sense of fracture), labelled by
// the component's smallest tet; the candidate pairs with a common vertex
// triple are found once on the host and kept on the device.
//
// Vertex adjacency: components are found over the vertices by
// hooking roots and shortcutting (a Shiloach-Vishkin style iteration): every
// vertex keeps a parent pointer f, initially the smallest vertex of its
// active tets (itself if smaller or isolated); in a hooking pass each
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
// the next pass.  Passes are queued a few at a time, each returning at once
// unless the pass before it changed something; after the batch the labels
// (each climbing to its root) and the component count follow, and the host
// reads the flags and the count back once.  If the batch's last pass still
// changed something, another batch follows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <vector>

#include "sta_internal.h"

namespace sta {
namespace {

constexpr int kBlock = 256;

unsigned blocks(int64_t n)
{
    return (unsigned)((n + kBlock - 1) / kBlock);
}

// Hooking passes per batch: the vertex rebuild mostly converges in two, the
// face rebuild in three (on the 384k-tet fracture stream: vertex 77 / 78 / 81
// / 91 us per rebuild at 2 / 3 / 4 / 6 passes per batch, face 147 / 117 /
// 122 / 126 us).  Flag words: [0, batch) set by hooking pass p when it
// changes a pointer; kMaxBatch: a climb of the labelling pass stopped short
// of a root; kMaxBatch + 1: the number of components.
constexpr int kVertexBatch = 2, kFaceBatch = 3;
constexpr int kMaxBatch = 3;
constexpr int kTruncWord = kMaxBatch, kCountWord = kMaxBatch + 1;
constexpr int kFlagWords = kMaxBatch + 2;

// Pass p > 0 of a batch runs only if pass p - 1 changed something (gate
// NULL: always).  The word is the same for every thread of the launch.
__device__ __forceinline__ bool gated_off(const uint32_t* gate)
{
    return gate && *gate == 0u;
}

// Seed (replaces the identity start): every vertex points at the smallest
// vertex of its active tets, or at itself if that is smaller or it has none,
// read from its diagonal incidence segment (dinc: the tet of each incidence).
// That vertex shares a tet with it, so the pointer stays inside the component
// and only decreases, as every later update does; the hooking passes then
// start from local minima and contend far less on their atomics.
__global__ __launch_bounds__(kBlock) void k_cc_seed(DevView v, const int32_t* __restrict__ dinc, int* f,
                                                    uint32_t* mark, uint32_t* flag)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < kFlagWords)
        flag[i] = 0u;  // the first batch's flags
    if (i >= v.n_nodes)
        return;
    int m = i;
    bool any = false;
    const int b = v.ndiag[i];
    if (b >= 0) {
        const BlockDesc d = v.desc[b];
        constexpr int kChunk = 8;
        for (int k0 = d.k0; k0 < d.k1; k0 += kChunk) {
            int e[kChunk];
#pragma unroll
            for (int j = 0; j < kChunk; ++j)
                e[j] = k0 + j < d.k1 ? dinc[k0 + j] : -1;
            bool on[kChunk];
#pragma unroll
            for (int j = 0; j < kChunk; ++j)
                on[j] = e[j] >= 0 && v.mask[e[j]];
#pragma unroll
            for (int j = 0; j < kChunk; ++j)
                if (on[j]) {
                    const int4 t = v.T[e[j]];
                    const int lo = min(min(t.x, t.y), min(t.z, t.w));
                    m = lo < m ? lo : m;
                    any = true;
                }
        }
    }
    f[i] = m;
    mark[i] = any ? 1u : 0u;  // a vertex of an active tet
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
__global__ __launch_bounds__(kBlock) void k_cc_hook(DevView v, int* f, const uint32_t* gate, uint32_t* changed_out)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (gated_off(gate) || e >= v.n_tets || !v.mask[e])
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
        changed_out[0] = 1u;
}

// Shortcut pass: every pointer to the root it reaches (only thread i writes f[i]).
__global__ __launch_bounds__(kBlock) void k_cc_shortcut(int n, int* f, const uint32_t* gate)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (gated_off(gate) || i >= n)
        return;
    const int p = f[i];
    const int r = climb(f, p);
    if (r < p)
        f[i] = r;
}

// After the hooking passes have converged (roots fixed): thread e < n_tets
// labels tet e with the root of its first vertex (-1 if inactive), climbing
// there itself; thread i < n_nodes counts vertex i if it is a root and a
// vertex of an active tet (each component's root is its smallest vertex,
// which belongs to an active tet).  A climb that stops at the step limit
// leaves a non-root, reported in *truncated (then another batch follows).
__global__ __launch_bounds__(kBlock) void k_cc_finish(DevView v, const int* __restrict__ f,
                                                      const uint32_t* __restrict__ mark, int32_t* __restrict__ label,
                                                      uint32_t* count, uint32_t* truncated)
{
    __shared__ uint32_t s_count;
    if (threadIdx.x == 0)
        s_count = 0u;
    __syncthreads();
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < v.n_tets) {
        int32_t l = -1;
        if (v.mask[t]) {
            l = climb(f, v.T[t].x);
            if (f[l] != l)
                truncated[0] = 1u;
        }
        label[t] = l;
    }
    if (t < v.n_nodes && mark[t] && f[t] == t)
        atomicAdd(&s_count, 1u);
    __syncthreads();
    if (threadIdx.x == 0 && s_count)
        atomicAdd(count, s_count);
}

// Face adjacency: parent pointers over tets, each starting at itself.
__global__ __launch_bounds__(kBlock) void k_ccf_init(int n_tets, int* f, uint32_t* flag)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e < kFlagWords)
        flag[e] = 0u;  // the first batch's flags
    if (e < n_tets)
        f[e] = e;
}

// Face adjacency, seed: across each active face pair inside one aligned group
// of 16 tet ids, the larger tet points at the smaller (atomic minimum).  Chains
// stay inside a group (at most 15 hops) and every pointer still goes to a tet
// of the same component with a smaller id; the hooking passes then start with
// most of each group merged.  (Seeding from every face neighbour instead made
// chains as long as the mesh and the first hooking pass slower.)
__global__ __launch_bounds__(kBlock) void k_ccf_seed(const uint8_t* __restrict__ mask, const int2* __restrict__ pairs,
                                                     int64_t n_pairs, int* f)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n_pairs)
        return;
    const int2 p = pairs[k];  // p.x < p.y
    if ((p.x >> 4) != (p.y >> 4) || !mask[p.x] || !mask[p.y])
        return;
    atomicMin(f + p.y, p.x);
}

// Hooking pass over the face pairs whose two tets are both active.
__global__ __launch_bounds__(kBlock) void k_ccf_hook(const uint8_t* __restrict__ mask, const int2* __restrict__ pairs,
                                                     int64_t n_pairs, int* f, const uint32_t* gate,
                                                     uint32_t* changed_out)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (gated_off(gate) || k >= n_pairs)
        return;
    const int2 p = pairs[k];
    if (!mask[p.x] || !mask[p.y])
        return;
    const int ra = climb(f, p.x), rb = climb(f, p.y);
    if (ra == rb)
        return;
    const int lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
    bool changed = atomicMin(f + hi, lo) > lo;
    changed |= atomicMin(f + p.x, lo) > lo;
    changed |= atomicMin(f + p.y, lo) > lo;
    if (changed)
        changed_out[0] = 1u;
}

// After the hooking passes have converged: label every tet with its root
// (-1 if inactive), climbing there itself; count the active roots; report a
// climb stopped at the step limit in *truncated.
__global__ __launch_bounds__(kBlock) void k_ccf_label(int n_tets, const uint8_t* __restrict__ mask,
                                                      const int* __restrict__ f, int32_t* __restrict__ label,
                                                      uint32_t* count, uint32_t* truncated)
{
    __shared__ uint32_t s_count;
    if (threadIdx.x == 0)
        s_count = 0u;
    __syncthreads();
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e < n_tets) {
        const bool on = mask[e] != 0;
        const int r = on ? climb(f, e) : -1;
        if (on && f[r] != r)
            truncated[0] = 1u;
        label[e] = r;
        if (on && r == e)
            atomicAdd(&s_count, 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_count)
        atomicAdd(count, s_count);
}

}  // namespace

// Candidate tet pairs with a common face (sorted vertex triple), every pair
// of tets on one triple, (smaller id, larger id), sorted.
std::vector<int2> host_face_pairs(const std::vector<int4>& T)
{
    struct Face {
        int a, b, c, e;
    };
    std::vector<Face> fs;
    fs.reserve(4 * T.size());
    for (size_t e = 0; e < T.size(); ++e) {
        std::array<int, 4> v = {T[e].x, T[e].y, T[e].z, T[e].w};
        std::sort(v.begin(), v.end());
        for (int skip = 0; skip < 4; ++skip) {
            int t[3], k = 0;
            for (int i = 0; i < 4; ++i)
                if (i != skip)
                    t[k++] = v[i];
            fs.push_back(Face{t[0], t[1], t[2], (int)e});
        }
    }
    std::sort(fs.begin(), fs.end(), [](const Face& x, const Face& y) {
        if (x.a != y.a) return x.a < y.a;
        if (x.b != y.b) return x.b < y.b;
        if (x.c != y.c) return x.c < y.c;
        return x.e < y.e;
    });
    std::vector<int2> pairs;
    for (size_t i = 0; i < fs.size();) {
        size_t j = i + 1;
        while (j < fs.size() && fs[j].a == fs[i].a && fs[j].b == fs[i].b && fs[j].c == fs[i].c)
            ++j;
        for (size_t u = i; u < j; ++u)
            for (size_t w = u + 1; w < j; ++w)
                if (fs[u].e != fs[w].e)
                    pairs.push_back(make_int2(fs[u].e, fs[w].e));
        i = j;
    }
    std::sort(pairs.begin(), pairs.end(),
              [](const int2& x, const int2& y) { return x.x != y.x ? x.x < y.x : x.y < y.y; });
    pairs.erase(std::unique(pairs.begin(), pairs.end(), [](const int2& x, const int2& y) { return x.x == y.x && x.y == y.y; }),
                pairs.end());
    return pairs;
}

// One read-back per batch: the flags and the component count; *passes
// counts the hooking passes that ran.  converged: the batch's last pass
// changed nothing and no labelling climb stopped short.
static hipError_t finish_batch(uint32_t* flag, uint32_t* host, int batch, int* passes, bool& converged,
                               hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(host, flag, sizeof(uint32_t) * kFlagWords, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return e;
    int ran = 1;
    for (int p = 0; p + 1 < batch; ++p)
        ran += host[p] != 0u;
    *passes += ran;
    converged = host[batch - 1] == 0u && host[kTruncWord] == 0u;
    return hipSuccess;
}

// Face-adjacency labels (smallest tet id of the component, -1 if inactive)
// into label; *n_components on the host.  f: n_tets ints; flag: kFlagWords
// words; host_flag: kFlagWords pinned words.  Synchronises s.
hipError_t run_face_components(const DevView& v, const int2* pairs, int64_t n_pairs, int* f, uint32_t* flag,
                               uint32_t* host_flag, int32_t* label, int64_t* n_components, int* passes,
                               hipStream_t s)
{
    const unsigned gt = v.n_tets > 0 ? blocks(v.n_tets) : 1u;
    const unsigned gp = n_pairs > 0 ? (unsigned)((n_pairs + kBlock - 1) / kBlock) : 1u;
    // init also clears the first batch's flags
    hipLaunchKernelGGL(k_ccf_init, dim3(gt), dim3(kBlock), 0, s, v.n_tets, f, flag);
    if (n_pairs > 0)
        hipLaunchKernelGGL(k_ccf_seed, dim3(gp), dim3(kBlock), 0, s, v.mask, pairs, n_pairs, f);
    hipError_t e = hipGetLastError();
    *passes = 0;
    // batches of hooking passes until one changes nothing (bounded: every pass
    // that does not end the loop lowers some pointer; the bound is far above
    // what a correct pass sequence needs), then the labels, in the same batch
    for (bool converged = false; e == hipSuccess && !converged;) {
        if (*passes > v.n_tets + 2)
            return hipErrorUnknown;
        if (*passes > 0)
            e = hipMemsetAsync(flag, 0, sizeof(uint32_t) * kFlagWords, s);
        for (int p = 0; p < kFaceBatch && e == hipSuccess; ++p) {
            const uint32_t* gate = p == 0 ? nullptr : flag + p - 1;
            if (n_pairs > 0)
                hipLaunchKernelGGL(k_ccf_hook, dim3(gp), dim3(kBlock), 0, s, v.mask, pairs, n_pairs, f, gate,
                                   flag + p);
            if (v.n_tets > 0)
                hipLaunchKernelGGL(k_cc_shortcut, dim3(gt), dim3(kBlock), 0, s, v.n_tets, f, gate);
            e = hipGetLastError();
        }
        if (e == hipSuccess && v.n_tets > 0) {
            hipLaunchKernelGGL(k_ccf_label, dim3(gt), dim3(kBlock), 0, s, v.n_tets, v.mask, f, label,
                               flag + kCountWord, flag + kTruncWord);
            e = hipGetLastError();
        }
        if (e == hipSuccess)
            e = finish_batch(flag, host_flag, kFaceBatch, passes, converged, s);
    }
    if (e == hipSuccess)
        *n_components = host_flag[kCountWord];
    return e;
}

// Component labels into label (device, n_tets); *n_components on the host.
// flag: kFlagWords words; host_flag: kFlagWords pinned words.  Synchronises
// s.  Returns hipErrorUnknown if the iteration bound is hit.
hipError_t run_components(const DevView& v, const int32_t* dinc, int* f, uint32_t* mark, uint32_t* flag,
                          uint32_t* host_flag, int32_t* label, int64_t* n_components, int* passes, hipStream_t s)
{
    const unsigned gn = v.n_nodes > 0 ? blocks(v.n_nodes) : 1u;
    const unsigned gt = v.n_tets > 0 ? blocks(v.n_tets) : 1u;
    const unsigned gf = blocks(std::max(v.n_tets, v.n_nodes) > 0 ? std::max(v.n_tets, v.n_nodes) : 1);
    // the seed also marks the vertices of active tets and clears the first batch's flags
    hipLaunchKernelGGL(k_cc_seed, dim3(gn), dim3(kBlock), 0, s, v, dinc, f, mark, flag);
    // one shortcut before the first hooking pass: every vertex climbs its seed
    // chain once, so that the tets' climbs in that pass are short (180 -> 122
    // us per rebuild; the face seeds' chains are short already, and there the
    // extra pass costs more than it saves)
    if (v.n_nodes > 0)
        hipLaunchKernelGGL(k_cc_shortcut, dim3(gn), dim3(kBlock), 0, s, v.n_nodes, f, nullptr);
    hipError_t e = hipGetLastError();
    *passes = 0;
    // batches of hooking passes, each followed by a shortcut, until one
    // changes nothing (then its reads were exact, so every active tet's
    // vertices share one root); then labels and count in the same batch.
    // Bounded as in the face variant.
    for (bool converged = false; e == hipSuccess && !converged;) {
        if (*passes > v.n_nodes + 2)
            return hipErrorUnknown;
        if (*passes > 0)
            e = hipMemsetAsync(flag, 0, sizeof(uint32_t) * kFlagWords, s);
        for (int p = 0; p < kVertexBatch && e == hipSuccess; ++p) {
            const uint32_t* gate = p == 0 ? nullptr : flag + p - 1;
            if (v.n_tets > 0)
                hipLaunchKernelGGL(k_cc_hook, dim3(gt), dim3(kBlock), 0, s, v, f, gate, flag + p);
            if (v.n_nodes > 0)
                hipLaunchKernelGGL(k_cc_shortcut, dim3(gn), dim3(kBlock), 0, s, v.n_nodes, f, gate);
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_cc_finish, dim3(gf), dim3(kBlock), 0, s, v, f, mark, label, flag + kCountWord,
                               flag + kTruncWord);
            e = hipGetLastError();
        }
        if (e == hipSuccess)
            e = finish_batch(flag, host_flag, kVertexBatch, passes, converged, s);
    }
    if (e == hipSuccess)
        *n_components = host_flag[kCountWord];
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
        e = hipMalloc(&q, sizeof(int32_t) * (2 * n + kFlagWords));  // parent and mark per vertex, the flags
        if (e != hipSuccess) {
            ctx->errmsg = std::string("connectivity workspace: ") + hipGetErrorString(e);
            return STA_ENOMEM;
        }
        ctx->owned.push_back(q);
        ctx->cc_ws = static_cast<int32_t*>(q);
    }
    if (!ctx->cc_host) {
        e = hipHostMalloc((void**)&ctx->cc_host, sizeof(uint32_t) * kFlagWords, hipHostMallocDefault);
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
    e = run_components(ctx->v, ctx->dinc, f, mark, flag, ctx->cc_host, labels_dev, &k, &ctx->cc_passes, s);
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

extern "C" sta_status sta_face_components(sta_ctx* ctx, int32_t* labels_dev, int64_t* n_components, void* stream)
{
    if (!ctx || (ctx->n_tets > 0 && !labels_dev))
        return STA_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (!ctx->ccf_ws) {
        // the candidate face pairs, once per context (the candidate pool is fixed)
        std::vector<int4> T((size_t)ctx->n_tets);
        if (ctx->n_tets > 0)
            e = hipMemcpy(T.data(), ctx->v.T, sizeof(int4) * T.size(), hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            ctx->errmsg = std::string("face connectivity: ") + hipGetErrorString(e);
            return STA_EHIP;
        }
        const std::vector<int2> pairs = host_face_pairs(T);
        void* q = nullptr;
        const size_t bytes = sizeof(int32_t) * ((size_t)ctx->n_tets + kFlagWords) + sizeof(int2) * (pairs.size() + 1);
        e = hipMalloc(&q, bytes);
        if (e != hipSuccess) {
            ctx->errmsg = std::string("face connectivity workspace: ") + hipGetErrorString(e);
            return STA_ENOMEM;
        }
        ctx->owned.push_back(q);
        int32_t* base = static_cast<int32_t*>(q);
        int2* pd = reinterpret_cast<int2*>(base + ((ctx->n_tets + kFlagWords + 1) / 2) * 2);  // 8-byte aligned after f and flags
        if (!pairs.empty())
            e = hipMemcpy(pd, pairs.data(), sizeof(int2) * pairs.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            ctx->errmsg = std::string("face pairs upload: ") + hipGetErrorString(e);
            return STA_EHIP;
        }
        ctx->ccf_ws = base;
        ctx->ccf_pairs = pd;
        ctx->ccf_npairs = (int64_t)pairs.size();
    }
    if (!ctx->cc_host) {
        e = hipHostMalloc((void**)&ctx->cc_host, sizeof(uint32_t) * kFlagWords, hipHostMallocDefault);
        if (e != hipSuccess) {
            ctx->cc_host = nullptr;
            ctx->errmsg = std::string("connectivity host flag: ") + hipGetErrorString(e);
            return STA_ENOMEM;
        }
    }
    int* f = ctx->ccf_ws;
    uint32_t* flag = reinterpret_cast<uint32_t*>(ctx->ccf_ws + ctx->n_tets);
    int64_t k = 0;
    e = run_face_components(ctx->v, ctx->ccf_pairs, ctx->ccf_npairs, f, flag, ctx->cc_host, labels_dev, &k,
                            &ctx->cc_passes, s);
    if (e == hipErrorUnknown) {
        ctx->errmsg = "face connectivity: pass bound exceeded (labels invalid)";
        return STA_EHIP;
    }
    if (e != hipSuccess) {
        ctx->errmsg = std::string("face connectivity: ") + hipGetErrorString(e);
        return STA_EHIP;
    }
    if (n_components)
        *n_components = k;
    return STA_OK;
}
