// The graph-Laplacian proxy operator of paper Sec. 3.1 on gfx950: edge
// multiplicities c_t (eq. (1)), binary edge activity a_t = [c_t > 0]
// (eq. (2)), the Laplacian L_t (eq. (3)) and A_t = L_t + eps I (eq. (4)),
// maintained by the count update of eq. (7) / Alg. 1.
//
// State (all in HBM, owned by the context): the mask, c_t per superset edge,
// the degree (number of active edges) per vertex and the CSR values of A_t
// over the fixed scalar superset pattern.  Counts and degrees are integers,
// so the streaming update applies the paper's +/- deltas directly with
// integer atomics and stays exactly equal to a rebuild, whatever order the
// atomics land in.
//
// A frame is two launches.  Phase 1, eight lanes per edit: validate, detect
// duplicates (a per-tet stamp), flip the mask, add +1 or -1 to the six edge
// counts, and on a 0 <-> >0 transition add the same to both endpoint degrees.
// Phase 2, after every count of the frame has landed: rewrite the six edge
// entries (-1.0 or +0.0 from the final count) and the four vertex diagonals
// (degree + eps) of every changed tet.  These writes are idempotent, so
// edits that share an edge or a vertex may write it concurrently.  An error
// found in phase 1 makes phase 2 undo the frame's count and degree deltas
// and mask flips instead (integer deltas undo exactly).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "sta_internal.h"

struct ProxyCtl {
    int32_t err;         // sticky error bits until sta_proxy_status_sync
    int32_t frame_err;   // error bits of the last frame
    int32_t last_n;      // edit count of the last frame
    int32_t pad;
    uint32_t trans;      // 0 <-> >0 transitions counted by the running frame's phase 1
    uint32_t last_trans; // transitions of the last frame (0 if it was rolled back)
    uint32_t changed;    // edits that changed a tet's state, running frame
    uint32_t last_changed;
};

struct ProxyView {
    int32_t n_nodes, n_tets, n_edges, pad;
    const int4* T;          // vertex ids per tet
    uint8_t* mask;          // active mask
    const int32_t* t2e;     // 6 per tet: edge ids of vertex pairs 01 02 03 12 13 23
    const int32_t* eseg;    // n_edges+1: incidence segment of each edge
    const int32_t* einc;    // candidate tets containing each edge
    const int32_t* epos;    // 2 per edge (u < v): CSR index of (u,v) and of (v,u)
    const int32_t* enode;   // 2 per edge: u, v
    const int32_t* rowptr;  // n_nodes+1
    const int32_t* ndpos;   // per vertex: CSR index of (u,u), -1 if u is in no candidate
    int32_t* c;             // c_t per edge
    int32_t* deg;           // active edges per vertex
    double* values;         // A_t over the pattern
    uint32_t* estamp;       // per tet, nonzero while an edit of this frame holds it
    uint8_t* undo;          // per edit: previous mask value, 0xFF = nothing to undo
    uint8_t* wg_err;        // phase 1: error bits per workgroup
    ProxyCtl* ctl;
    double eps;
};

struct sta_proxy {
    int device = 0;
    int64_t n_nodes = 0, n_tets = 0, n_edges = 0, nnz = 0;
    ProxyView v{};
    int32_t* colidx = nullptr;
    std::vector<void*> owned;
    std::string errmsg;
};

namespace sta {
namespace {

constexpr int kBlock = 256;
constexpr int kLanes = 8;  // per edit: lane r < 6 owns edge r, lanes r < 4 own vertex r in phase 2

__device__ __forceinline__ int tet_vertex(int4 t, int r)
{
    return r == 0 ? t.x : r == 1 ? t.y : r == 2 ? t.z : t.w;
}

__device__ __forceinline__ double off_value(int32_t count)
{
    return count > 0 ? -1.0 : 0.0;
}

// Segment and row loops load this many terms before using any of them.
constexpr int kChunk = 8;

// Rebuild, step 1: every edge's count from the mask over its incidence
// segment (eq. (1)), and its two off-diagonal entries (eqs. (2), (3)).
__global__ __launch_bounds__(kBlock) void k_proxy_counts(ProxyView v)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= v.n_edges)
        return;
    int32_t cnt = 0;
    const int k1 = v.eseg[e + 1];
    for (int k0 = v.eseg[e]; k0 < k1; k0 += kChunk) {  // loads in flight together
        int t[kChunk];
#pragma unroll
        for (int j = 0; j < kChunk; ++j)
            t[j] = k0 + j < k1 ? v.einc[k0 + j] : -1;
#pragma unroll
        for (int j = 0; j < kChunk; ++j)
            cnt += t[j] >= 0 ? v.mask[t[j]] : 0;
    }
    v.c[e] = cnt;
    const double x = off_value(cnt);
    v.values[v.epos[2 * e]] = x;
    v.values[v.epos[2 * e + 1]] = x;
}

// Rebuild, step 2: every vertex's degree = active off-diagonal entries in its
// row (eq. (3)), and its diagonal entry degree + eps (eq. (4)).
__global__ __launch_bounds__(kBlock) void k_proxy_diagonal(ProxyView v)
{
    const int u = blockIdx.x * kBlock + threadIdx.x;
    if (u >= v.n_nodes)
        return;
    const int p = v.ndpos[u];
    if (p < 0)
        return;
    int32_t d = 0;
    const int k1 = v.rowptr[u + 1];
    for (int k0 = v.rowptr[u]; k0 < k1; k0 += kChunk) {  // loads in flight together
        double x[kChunk];
#pragma unroll
        for (int j = 0; j < kChunk; ++j)
            x[j] = k0 + j < k1 ? v.values[k0 + j] : 0.0;
#pragma unroll
        for (int j = 0; j < kChunk; ++j)
            d += (k0 + j < k1 && k0 + j != p && x[j] == -1.0) ? 1 : 0;
    }
    v.deg[u] = d;
    v.values[p] = (double)d + v.eps;
}

__device__ __forceinline__ int edit_count(int32_t n_host, const int32_t* n_dev, bool& bad)
{
    bad = false;
    if (!n_dev)
        return n_host;
    const int n = *n_dev;
    if (n < 0 || n > n_host) {
        bad = true;
        return 0;
    }
    return n;
}

// Apply delta d (+1 adds the tet, -1 removes it) to edge ek's count; on a
// 0 <-> >0 transition move both endpoint degrees by d.  Returns 1 on a transition.
__device__ __forceinline__ unsigned count_delta(const ProxyView& v, int ek, int d)
{
    const int32_t old = atomicAdd(&v.c[ek], d);
    if (d > 0 ? old != 0 : old != 1)
        return 0u;
    atomicAdd(&v.deg[v.enode[2 * ek]], d);
    atomicAdd(&v.deg[v.enode[2 * ek + 1]], d);
    return 1u;
}

// Phase 1 (Alg. 1: mask update and count update of eq. (7)).
__global__ __launch_bounds__(kBlock) void k_proxy_edits(ProxyView v, const int32_t* __restrict__ ids,
                                                        const uint8_t* __restrict__ states, int32_t n_host,
                                                        const int32_t* __restrict__ n_dev)
{
    __shared__ int s_bits;
    __shared__ unsigned s_trans, s_changed;
    if (threadIdx.x == 0) {
        s_bits = 0;
        s_trans = 0u;
        s_changed = 0u;
    }
    const int gt = blockIdx.x * kBlock + threadIdx.x;
    const int i = gt / kLanes, r = gt % kLanes;
    int id = -1;
    unsigned st = 0;
    if (i < n_host) {
        id = ids[i];
        st = states[i];
    }
    bool bad_n;
    const int n = edit_count(n_host, n_dev, bad_n);
    int bits = (bad_n && gt == 0) ? ERR_RANGE : 0;
    unsigned trans = 0u, changed = 0u;
    if (i < n) {
        if (id < 0 || id >= v.n_tets || st > 1u) {
            if (r == 0) {
                v.undo[i] = 0xFF;
                bits |= ERR_RANGE;
            }
        } else {
            const int ek = r < 6 ? v.t2e[6 * (size_t)id + r] : 0;
            const uint8_t prev = v.mask[id];
            unsigned taken = 0u;
            if (r == 0)
                taken = atomicExch(&v.estamp[id], 1u);
            const bool owner = __shfl(taken, (threadIdx.x & 63) & ~(kLanes - 1), 64) == 0u;
            const bool change = prev != st;
            if (!owner) {
                if (r == 0)
                    bits |= ERR_DUP;
            } else if (change) {
                if (r == 0) {
                    v.mask[id] = (uint8_t)st;
                    changed = 1u;
                }
                if (r < 6)
                    trans = count_delta(v, ek, st ? 1 : -1);
            }
            if (r == 0)
                v.undo[i] = (owner && change) ? prev : (uint8_t)0xFF;
        }
    }
    __syncthreads();
    if (bits)
        atomicOr(&s_bits, bits);
    if (trans)
        atomicAdd(&s_trans, trans);
    if (changed)
        atomicAdd(&s_changed, changed);
    __syncthreads();
    if (threadIdx.x == 0) {
        v.wg_err[blockIdx.x] = (uint8_t)s_bits;
        if (s_trans)
            atomicAdd(&v.ctl->trans, s_trans);
        if (s_changed)
            atomicAdd(&v.ctl->changed, s_changed);
    }
}

// Phase 2 (Alg. 1: insert / remove off-diagonal entries, update the diagonal
// degree terms; "finalize A_t"), or the frame's rollback on an error.
__global__ __launch_bounds__(kBlock) void k_proxy_touched(ProxyView v, const int32_t* __restrict__ ids,
                                                          int32_t n_host, const int32_t* __restrict__ n_dev)
{
    __shared__ int s_bits;
    const int gt = blockIdx.x * kBlock + threadIdx.x;
    const int i = gt / kLanes, r = gt % kLanes;
    int id = -1;
    uint8_t u = 0xFF;
    if (i < n_host) {
        id = ids[i];
        u = v.undo[i];
    }
    bool bad_n;
    const int n = edit_count(n_host, n_dev, bad_n);
    // the error bytes of every workgroup of phase 1 (its grid is sized by n_host)
    const int g = n_host > 0 ? (n_host * kLanes + kBlock - 1) / kBlock : 1;
    int bits = 0;
    for (int w = threadIdx.x; w < g; w += kBlock)
        bits |= v.wg_err[w];
    if (threadIdx.x == 0)
        s_bits = 0;
    __syncthreads();
    if (bits)
        atomicOr(&s_bits, bits);
    __syncthreads();
    const int fe = s_bits;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t t = atomicExch(&v.ctl->trans, 0u);
        const uint32_t c = atomicExch(&v.ctl->changed, 0u);
        v.ctl->last_trans = fe ? 0u : t;
        v.ctl->last_changed = fe ? 0u : c;
        v.ctl->frame_err = fe;
        v.ctl->last_n = n;
        if (fe)
            atomicOr(&v.ctl->err, fe);
    }
    if (i >= n || id < 0 || id >= v.n_tets)
        return;
    if (u != 0xFF) {
        const int ek = r < 6 ? v.t2e[6 * (size_t)id + r] : 0;
        if (fe) {
            // restore state u: the same count delta as an edit to state u
            if (r == 0)
                v.mask[id] = u;
            if (r < 6)
                (void)count_delta(v, ek, u ? 1 : -1);
        } else {
            if (r < 6) {
                const double x = off_value(v.c[ek]);
                v.values[v.epos[2 * ek]] = x;
                v.values[v.epos[2 * ek + 1]] = x;
            }
            if (r < 4) {
                const int node = tet_vertex(v.T[id], r);
                v.values[v.ndpos[node]] = (double)v.deg[node] + v.eps;
            }
        }
    }
    if (r == 0)
        v.estamp[id] = 0u;
}

unsigned blocks(int64_t threads)
{
    return (unsigned)((threads + kBlock - 1) / kBlock);
}

thread_local std::string g_proxy_build_err;

sta_status pfail(sta_proxy* p, sta_status code, const std::string& msg)
{
    if (p)
        p->errmsg = msg;
    else
        g_proxy_build_err = msg;
    return code;
}

template <class T>
hipError_t palloc(sta_proxy* p, T** out, size_t count)
{
    void* q = nullptr;
    const size_t bytes = count ? count * sizeof(T) : 256;
    hipError_t e = hipMalloc(&q, bytes);
    if (e == hipSuccess) {
        p->owned.push_back(q);
        *out = static_cast<T*>(q);
    }
    return e;
}

template <class T>
hipError_t put(T* dst, const T* src, size_t count, hipStream_t s)
{
    return count ? hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, s) : hipSuccess;
}

void release(sta_proxy* p)
{
    for (void* q : p->owned)
        (void)hipFree(q);
    p->owned.clear();
}

hipError_t launch_rebuild(const ProxyView& v, hipStream_t s)
{
    if (v.n_edges > 0)
        hipLaunchKernelGGL(k_proxy_counts, dim3(blocks(v.n_edges)), dim3(kBlock), 0, s, v);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && v.n_nodes > 0) {
        hipLaunchKernelGGL(k_proxy_diagonal, dim3(blocks(v.n_nodes)), dim3(kBlock), 0, s, v);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_frame(const ProxyView& v, const int32_t* ids, const uint8_t* states, int32_t n_host,
                        const int32_t* n_dev, hipStream_t s)
{
    const unsigned g = n_host > 0 ? blocks((int64_t)n_host * kLanes) : 1u;
    hipLaunchKernelGGL(k_proxy_edits, dim3(g), dim3(kBlock), 0, s, v, ids, states, n_host, n_dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_proxy_touched, dim3(g), dim3(kBlock), 0, s, v, ids, n_host, n_dev);
    return hipGetLastError();
}

}  // namespace
}  // namespace sta

using namespace sta;

extern "C" sta_status sta_proxy_build(const int32_t* tets, int64_t n_nodes, int64_t n_tets, const uint8_t* mask0,
                                      double eps, void* stream, sta_proxy** out)
{
    if (!out)
        return pfail(nullptr, STA_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_nodes < 0 || n_tets < 0 || n_nodes > INT32_MAX || n_tets > INT32_MAX / 10 ||
        (n_tets > 0 && (!tets || !mask0)))
        return pfail(nullptr, STA_EINVAL, "bad sizes or NULL host arrays");
    if (!std::isfinite(eps) || eps < 0.0)
        return pfail(nullptr, STA_EINVAL, "eps must be finite and >= 0");
    for (int64_t e = 0; e < n_tets; ++e) {
        if (mask0[e] > 1)
            return pfail(nullptr, STA_EINVAL, "mask0 values must be 0 or 1");
        const int32_t* t = tets + 4 * e;
        for (int a = 0; a < 4; ++a) {
            if (t[a] < 0 || t[a] >= n_nodes)
                return pfail(nullptr, STA_EINVAL, "tet vertex id out of range");
            for (int b = 0; b < a; ++b)
                if (t[a] == t[b])
                    return pfail(nullptr, STA_EDEGENERATE, "tet with a repeated vertex");
        }
    }
    HostPattern P;
    const std::string perr = build_host_pattern(n_nodes, tets, n_tets, P, 1);
    if (!perr.empty())
        return pfail(nullptr, STA_EINVAL, perr);
    sta_proxy* p = new (std::nothrow) sta_proxy;
    if (!p)
        return pfail(nullptr, STA_ENOMEM, "host allocation");
    hipStream_t s = static_cast<hipStream_t>(stream);
    (void)hipGetDevice(&p->device);
    p->n_nodes = n_nodes;
    p->n_tets = n_tets;
    p->n_edges = P.no;
    p->nnz = P.nnz;
    std::vector<int32_t> t2e((size_t)n_tets * 6), epos((size_t)P.no * 2), ndpos((size_t)n_nodes, -1);
    for (int64_t e = 0; e < n_tets; ++e)
        for (int q = 0; q < 6; ++q)
            t2e[6 * e + q] = P.e2b[10 * e + 4 + q];
    for (int64_t b = 0; b < P.no; ++b) {
        epos[2 * b] = P.ometa[4 * b + 0];
        epos[2 * b + 1] = P.ometa[4 * b + 2];
    }
    for (int64_t u = 0; u < n_nodes; ++u)
        if (P.ndiag[u] >= 0)
            ndpos[u] = P.dmeta[2 * (size_t)P.ndiag[u]];
    ProxyView& v = p->v;
    v.n_nodes = (int32_t)n_nodes;
    v.n_tets = (int32_t)n_tets;
    v.n_edges = (int32_t)P.no;
    v.eps = eps;
    int4* T = nullptr;
    int32_t *t2e_d = nullptr, *eseg = nullptr, *einc = nullptr, *epos_d = nullptr, *enode = nullptr,
            *rowptr = nullptr, *ndpos_d = nullptr;
    const int64_t wg = n_tets > 0 ? blocks(n_tets * kLanes) : 1;
    hipError_t e = hipSuccess;
#define PALLOC(ptr, count) \
    if (e == hipSuccess)   \
        e = palloc(p, &ptr, (size_t)(count));
    PALLOC(T, n_tets)
    PALLOC(v.mask, n_tets)
    PALLOC(t2e_d, n_tets * 6)
    PALLOC(eseg, P.no + 1)
    PALLOC(einc, n_tets * 6)
    PALLOC(epos_d, P.no * 2)
    PALLOC(enode, P.no * 2)
    PALLOC(rowptr, n_nodes + 1)
    PALLOC(p->colidx, P.nnz)
    PALLOC(ndpos_d, n_nodes)
    PALLOC(v.c, P.no)
    PALLOC(v.deg, n_nodes)
    PALLOC(v.values, P.nnz)
    PALLOC(v.estamp, n_tets)
    PALLOC(v.undo, n_tets)
    PALLOC(v.wg_err, wg)
    PALLOC(v.ctl, 1)
#undef PALLOC
    if (e == hipSuccess) e = put(T, reinterpret_cast<const int4*>(tets), (size_t)n_tets, s);
    if (e == hipSuccess) e = put(v.mask, mask0, (size_t)n_tets, s);
    if (e == hipSuccess) e = put(t2e_d, t2e.data(), t2e.size(), s);
    if (e == hipSuccess) e = put(eseg, P.oseg.data(), P.oseg.size(), s);
    if (e == hipSuccess) e = put(einc, P.oinc.data(), P.oinc.size(), s);
    if (e == hipSuccess) e = put(epos_d, epos.data(), epos.size(), s);
    if (e == hipSuccess) e = put(enode, P.opair.data(), P.opair.size(), s);
    if (e == hipSuccess) e = put(rowptr, P.rowptr.data(), P.rowptr.size(), s);
    if (e == hipSuccess) e = put(p->colidx, P.colidx.data(), P.colidx.size(), s);
    if (e == hipSuccess) e = put(ndpos_d, ndpos.data(), ndpos.size(), s);
    if (e == hipSuccess) e = hipMemsetAsync(v.deg, 0, sizeof(int32_t) * (size_t)(n_nodes ? n_nodes : 1), s);
    if (e == hipSuccess) e = hipMemsetAsync(v.values, 0, sizeof(double) * (size_t)(P.nnz ? P.nnz : 1), s);
    if (e == hipSuccess) e = hipMemsetAsync(v.estamp, 0, sizeof(uint32_t) * (size_t)(n_tets ? n_tets : 1), s);
    if (e == hipSuccess) e = hipMemsetAsync(v.ctl, 0, sizeof(ProxyCtl), s);
    v.T = T;
    v.t2e = t2e_d;
    v.eseg = eseg;
    v.einc = einc;
    v.epos = epos_d;
    v.enode = enode;
    v.rowptr = rowptr;
    v.ndpos = ndpos_d;
    if (e == hipSuccess)
        e = launch_rebuild(v, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        const std::string msg = std::string("proxy build: ") + hipGetErrorString(e);
        release(p);
        delete p;
        return pfail(nullptr, e == hipErrorOutOfMemory ? STA_ENOMEM : STA_EHIP, msg);
    }
    *out = p;
    return STA_OK;
}

extern "C" sta_status sta_proxy_full_rebuild(sta_proxy* p, void* stream)
{
    if (!p)
        return STA_EINVAL;
    const hipError_t e = launch_rebuild(p->v, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? STA_OK : pfail(p, STA_EHIP, std::string("proxy rebuild: ") + hipGetErrorString(e));
}

extern "C" sta_status sta_proxy_apply_edits(sta_proxy* p, const int32_t* ids_dev, const uint8_t* states_dev,
                                            int64_t n_edits, void* stream)
{
    if (!p)
        return STA_EINVAL;
    if (n_edits < 0 || n_edits > p->n_tets)
        return pfail(p, STA_EINVAL, "n_edits must be in [0, n_tets]");
    if (n_edits > 0 && (!ids_dev || !states_dev))
        return pfail(p, STA_EINVAL, "NULL edit arrays");
    const hipError_t e =
        launch_frame(p->v, ids_dev, states_dev, (int32_t)n_edits, nullptr, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? STA_OK : pfail(p, STA_EHIP, std::string("proxy frame: ") + hipGetErrorString(e));
}

extern "C" sta_status sta_proxy_apply_edits_dev(sta_proxy* p, const int32_t* ids_dev, const uint8_t* states_dev,
                                                int64_t capacity, const int32_t* n_dev, void* stream)
{
    if (!p)
        return STA_EINVAL;
    if (capacity < 1 || capacity > p->n_tets || !ids_dev || !states_dev || !n_dev)
        return pfail(p, STA_EINVAL, "capacity must be in [1, n_tets] and the device arrays non-NULL");
    const hipError_t e =
        launch_frame(p->v, ids_dev, states_dev, (int32_t)capacity, n_dev, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? STA_OK : pfail(p, STA_EHIP, std::string("proxy frame: ") + hipGetErrorString(e));
}

extern "C" sta_status sta_proxy_sizes(const sta_proxy* p, int64_t* n_rows, int64_t* nnz, int64_t* n_edges)
{
    if (!p)
        return STA_EINVAL;
    if (n_rows)
        *n_rows = p->n_nodes;
    if (nnz)
        *nnz = p->nnz;
    if (n_edges)
        *n_edges = p->n_edges;
    return STA_OK;
}

extern "C" const double* sta_proxy_values_ptr(const sta_proxy* p)
{
    return p ? p->v.values : nullptr;
}

extern "C" const int32_t* sta_proxy_counts_ptr(const sta_proxy* p)
{
    return p ? p->v.c : nullptr;
}

extern "C" const int32_t* sta_proxy_degree_ptr(const sta_proxy* p)
{
    return p ? p->v.deg : nullptr;
}

extern "C" sta_status sta_proxy_copy_state(const sta_proxy* p, double* values, int32_t* counts, int32_t* degree,
                                           void* stream)
{
    if (!p)
        return STA_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (values && p->nnz)
        e = hipMemcpyAsync(values, p->v.values, sizeof(double) * p->nnz, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && counts && p->n_edges)
        e = hipMemcpyAsync(counts, p->v.c, sizeof(int32_t) * p->n_edges, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && degree && p->n_nodes)
        e = hipMemcpyAsync(degree, p->v.deg, sizeof(int32_t) * p->n_nodes, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? STA_OK : STA_EHIP;
}

extern "C" sta_status sta_proxy_pattern_ptrs(const sta_proxy* p, const int32_t** rowptr, const int32_t** colidx,
                                             const int32_t** edges)
{
    if (!p)
        return STA_EINVAL;
    if (rowptr)
        *rowptr = p->v.rowptr;
    if (colidx)
        *colidx = p->colidx;
    if (edges)
        *edges = p->v.enode;
    return STA_OK;
}

extern "C" sta_status sta_proxy_pattern_host(const sta_proxy* p, int32_t* rowptr, int32_t* colidx, int32_t* edges)
{
    if (!p || !rowptr || !colidx || !edges)
        return STA_EINVAL;
    hipError_t e = hipMemcpy(rowptr, p->v.rowptr, sizeof(int32_t) * (p->n_nodes + 1), hipMemcpyDeviceToHost);
    if (e == hipSuccess && p->nnz)
        e = hipMemcpy(colidx, p->colidx, sizeof(int32_t) * p->nnz, hipMemcpyDeviceToHost);
    if (e == hipSuccess && p->n_edges)
        e = hipMemcpy(edges, p->v.enode, sizeof(int32_t) * 2 * p->n_edges, hipMemcpyDeviceToHost);
    return e == hipSuccess ? STA_OK : pfail(const_cast<sta_proxy*>(p), STA_EHIP, "proxy pattern copy");
}

extern "C" sta_status sta_proxy_last_frame_stats(sta_proxy* p, void* stream, int64_t* out3)
{
    if (!p || !out3)
        return STA_EINVAL;
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    ProxyCtl h{};
    if (e == hipSuccess)
        e = hipMemcpy(&h, p->v.ctl, sizeof h, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return pfail(p, STA_EHIP, std::string("proxy stats: ") + hipGetErrorString(e));
    out3[0] = h.last_n;
    out3[1] = h.last_changed;
    out3[2] = h.last_trans;
    return STA_OK;
}

extern "C" sta_status sta_proxy_status_sync(sta_proxy* p, void* stream)
{
    if (!p)
        return STA_EINVAL;
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    int32_t bits = 0;
    if (e == hipSuccess)
        e = hipMemcpy(&bits, &p->v.ctl->err, sizeof bits, hipMemcpyDeviceToHost);
    if (e == hipSuccess && bits) {
        const int32_t zero = 0;
        e = hipMemcpy(&p->v.ctl->err, &zero, sizeof zero, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess)
        return pfail(p, STA_EHIP, std::string("proxy status: ") + hipGetErrorString(e));
    if (bits & ERR_RANGE)
        return pfail(p, STA_ERANGE, "an edit named a tet id outside [0, n_tets) or a state other than 0/1; "
                                    "frame rolled back");
    if (bits & ERR_DUP)
        return pfail(p, STA_EDUP, "an edit list named the same tet twice; frame rolled back");
    return STA_OK;
}

extern "C" const char* sta_proxy_last_error(const sta_proxy* p)
{
    return p ? p->errmsg.c_str() : g_proxy_build_err.c_str();
}

extern "C" void sta_proxy_destroy(sta_proxy* p)
{
    if (!p)
        return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != p->device)
        (void)hipSetDevice(p->device);
    release(p);
    if (cur != p->device)
        (void)hipSetDevice(cur);
    delete p;
}
