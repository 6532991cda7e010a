// C ABI of libstafem.so (declared in include/stafem.h): argument checks,
// device allocation, the host pattern hand-off and kernel sequencing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "sta_internal.h"

using namespace sta;

namespace {

thread_local std::string g_build_err;

sta_status fail(sta_ctx* ctx, sta_status code, const std::string& msg)
{
    if (ctx)
        ctx->errmsg = msg;
    else
        g_build_err = msg;
    return code;
}

sta_status hip_fail(sta_ctx* ctx, hipError_t e, const char* what)
{
    return fail(ctx, STA_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Failure injection for tests of STA_ENOMEM: when the environment variable
// STA_FAIL_ALLOC_AT is a number k >= 1, the k-th device allocation made by
// this process (counting from the first allocation after the variable is
// read as set) reports out-of-memory without allocating.
bool injected_alloc_failure()
{
    static thread_local long seen = 0;
    const char* at = std::getenv("STA_FAIL_ALLOC_AT");
    if (!at || !*at) {
        seen = 0;
        return false;
    }
    const long k = std::strtol(at, nullptr, 10);
    return k >= 1 && ++seen == k;
}

template <class T>
hipError_t dalloc(sta_ctx* c, T** p, size_t count)
{
    void* q = nullptr;
    size_t bytes = count * sizeof(T);
    if (bytes == 0)
        bytes = 256;
    if (injected_alloc_failure())
        return hipErrorOutOfMemory;
    hipError_t e = hipMalloc(&q, bytes);
    if (e == hipSuccess) {
        c->owned.push_back(q);
        *p = static_cast<T*>(q);
    }
    return e;
}

template <class T>
hipError_t upload(T* dst, const T* src, size_t count, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    return hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, s);
}

void free_all(sta_ctx* c)
{
    for (void* p : c->owned)
        (void)hipFree(p);
    c->owned.clear();
}

sta_status device_errors(int32_t bits)
{
    if (bits & ERR_RANGE)
        return STA_ERANGE;
    if (bits & ERR_DUP)
        return STA_EDUP;
    if (bits & ERR_DEGENERATE)
        return STA_EDEGENERATE;
    return STA_OK;
}

Material material(double nu, double rho, double dt)
{
    Material m;
    m.cdt = dt * dt;
    const double den = (1.0 + nu) * (1.0 - (2.0 * nu));
    m.clam = nu / den;
    m.cmu = 0.5 / (1.0 + nu);
    m.rho = rho;
    return m;
}

hipEvent_t take_event(sta_ctx* c)
{
    if (!c->event_pool.empty()) {
        hipEvent_t ev = c->event_pool.back();
        c->event_pool.pop_back();
        return ev;
    }
    hipEvent_t ev = nullptr;
    if (hipEventCreate(&ev) != hipSuccess)
        return nullptr;
    return ev;
}

// Run one launcher with kernel timing when it is on.  A launcher of a single
// kernel (single = true) gets the events attached to the dispatch, so they
// time the kernel alone; other launchers are bracketed by event records
// (which adds the launch gaps between their kernels).
template <class F>
hipError_t timed(sta_ctx* c, int kernel, hipStream_t s, F&& launch, bool single = false)
{
    if (!c->timing)
        return launch();
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b)
        return hipErrorOutOfMemory;
    hipError_t e = hipSuccess;
    if (single) {
        KernelEvents& ev = kernel_events();
        ev.start = a;
        ev.stop = b;
        ev.used = false;
        e = launch();
        const bool used = ev.used;
        ev = KernelEvents{};
        if (!used) {  // nothing was launched: nothing to time
            c->event_pool.push_back(a);
            c->event_pool.push_back(b);
            return e;
        }
    } else {
        e = hipEventRecord(a, s);
        if (e == hipSuccess)
            e = launch();
        if (e == hipSuccess)
            e = hipEventRecord(b, s);
    }
    c->timed.push_back({kernel, a, b});
    return e;
}

double host_seconds()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

namespace sta {

KernelEvents& kernel_events()
{
    thread_local KernelEvents ev;
    return ev;
}

std::string& build_error()
{
    return g_build_err;
}

// Spread the low 10 bits of v to every third bit (Morton interleave).
static uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffull;
    x = (x | (x << 8)) & 0x0300f00full;
    x = (x | (x << 4)) & 0x030c30c3ull;
    x = (x | (x << 2)) & 0x09249249ull;
    return x;
}

// The adjoint's chunk order: chunks of kAdjointChunk consecutive tet ids,
// sorted by (mesh of the chunk's first tet, Morton code of the chunk's
// centroid on a 1024^3 grid over that mesh's bounding box), ties by chunk id.
// x: n_nodes * 3 row-major; node_off / tet_off: the meshes' node and tet ranges.
static std::vector<int32_t> adjoint_chunk_order(const double* x, const std::vector<int4>& T,
                                                const std::vector<int64_t>& node_off,
                                                const std::vector<int64_t>& tet_off)
{
    const int64_t n_tets = (int64_t)T.size();
    const int64_t nc = (n_tets + kAdjointChunk - 1) / kAdjointChunk;
    const size_t n_mesh = tet_off.size() > 1 ? tet_off.size() - 1 : 0;
    std::vector<double> lo(3 * n_mesh, 0.0), span(3 * n_mesh, 0.0);
    for (size_t m = 0; m < n_mesh; ++m) {
        double l[3] = {INFINITY, INFINITY, INFINITY}, h[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t i = node_off[m]; i < node_off[m + 1]; ++i)
            for (int k = 0; k < 3; ++k) {
                l[k] = std::min(l[k], x[3 * i + k]);
                h[k] = std::max(h[k], x[3 * i + k]);
            }
        for (int k = 0; k < 3; ++k) {
            lo[3 * m + k] = std::isfinite(l[k]) ? l[k] : 0.0;
            span[3 * m + k] = h[k] > l[k] ? h[k] - l[k] : 0.0;
        }
    }
    std::vector<std::pair<uint64_t, int32_t>> key((size_t)nc);
    size_t m = 0;
    for (int64_t c = 0; c < nc; ++c) {
        const int64_t e0 = c * kAdjointChunk, e1 = std::min(n_tets, e0 + kAdjointChunk);
        while (m + 1 < n_mesh && tet_off[m + 1] <= e0)
            ++m;
        double s[3] = {0.0, 0.0, 0.0};
        for (int64_t e = e0; e < e1; ++e) {
            const int id[4] = {T[e].x, T[e].y, T[e].z, T[e].w};
            for (int a = 0; a < 4; ++a)
                for (int k = 0; k < 3; ++k)
                    s[k] += x[3 * (int64_t)id[a] + k];
        }
        uint64_t code = 0;
        for (int k = 0; k < 3 && n_mesh > 0; ++k) {
            const double sp = span[3 * m + k];
            const double t = sp > 0.0 ? (s[k] / (4.0 * (double)(e1 - e0)) - lo[3 * m + k]) / sp : 0.0;
            const uint32_t q = (uint32_t)std::min(1023.0, std::max(0.0, std::floor(t * 1024.0)));
            code |= spread3(q) << k;
        }
        key[(size_t)c] = {((uint64_t)m << 30) | code, (int32_t)c};
    }
    std::sort(key.begin(), key.end());
    std::vector<int32_t> order((size_t)nc);
    for (int64_t c = 0; c < nc; ++c)
        order[(size_t)c] = key[(size_t)c].second;
    return order;
}

// A batch whose contributions (78 doubles per tet) exceed the 256 MB Infinity Cache is rebuilt
// in groups of consecutive meshes of at most this many contribution bytes, element pass then
// reduce per group: the reduce then reads what the element pass just wrote from that cache (on
// the 64-mesh batch, 853 MB: 660 -> 580 us per rebuild, same bits; groups of at most 100 / 160 /
// 250 / 300 / 400 MB: 636 / 602 / 608 / 618 / 629 us).  A batch's meshes share no block, so
// every block's segment lies in one group.
constexpr double kRebuildGroupBytes = 200e6;
constexpr double kContributionBytesPerTet = 78 * 8;

// The rebuild groups of a batch (node_off / tet_off: k + 1 mesh offsets), or none when the
// whole batch fits one group.  Blocks are numbered diagonal first, then off-diagonal, each in
// row order, so each mesh's blocks of either kind form one range, found from the CSR position
// of each block's upper copy.
static std::vector<std::array<int64_t, 6>> rebuild_groups(const HostPattern& P, const std::vector<BlockDesc>& hd,
                                                          const std::vector<int64_t>& node_off,
                                                          const std::vector<int64_t>& tet_off)
{
    std::vector<std::array<int64_t, 6>> groups;
    const size_t k = tet_off.size() > 1 ? tet_off.size() - 1 : 0;
    if (k < 2 || (double)tet_off[k] * kContributionBytesPerTet <= kRebuildGroupBytes)
        return groups;
    std::vector<int64_t> first_value(k + 1);
    for (size_t j = 0; j <= k; ++j)
        first_value[j] = P.rowptr[3 * node_off[j]];
    auto mesh_of = [&](int64_t up) {
        return (int64_t)(std::upper_bound(first_value.begin(), first_value.end(), up) - first_value.begin()) - 1;
    };
    // start[j]: the first block of mesh j (the kind's block count if it has none)
    auto starts = [&](int64_t b0, int64_t nb, std::vector<int64_t>& start) {
        start.assign(k + 1, nb);
        int64_t prev = -1;
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t m = mesh_of(hd[b0 + b].up);
            if (m < prev)
                return false;
            for (int64_t q = prev + 1; q <= m; ++q)
                start[q] = b;
            prev = m;
        }
        return true;
    };
    std::vector<int64_t> dstart, ostart;
    if (!starts(0, P.nd, dstart) || !starts(P.nd, P.no, ostart))
        return groups;
    for (size_t j = 0; j < k;) {
        size_t j1 = j + 1;
        while (j1 < k && (double)(tet_off[j1 + 1] - tet_off[j]) * kContributionBytesPerTet <= kRebuildGroupBytes)
            ++j1;
        groups.push_back({tet_off[j], tet_off[j1], dstart[j], dstart[j1], ostart[j], ostart[j1]});
        j = j1;
    }
    if (groups.size() < 2)
        groups.clear();
    return groups;
}

sta_status build_context(const double* x, int64_t n_nodes, const int32_t* tets, int64_t n_tets, const double* E,
                         double nu, double rho, double dt, const uint8_t* mask0, void* stream,
                         const std::vector<int64_t>& node_off, const std::vector<int64_t>& tet_off, sta_ctx** out)
{
    g_build_err.clear();
    if (!out)
        return fail(nullptr, STA_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_nodes < 0 || n_tets < 0 || n_nodes > INT32_MAX / 3 || n_tets > INT32_MAX / 10)
        return fail(nullptr, STA_EINVAL, "n_nodes / n_tets out of range");
    if ((n_nodes > 0 && !x) || (n_tets > 0 && (!tets || !E || !mask0)))
        return fail(nullptr, STA_EINVAL, "NULL input array");
    if (!(nu > -1.0 && nu < 0.5) || !(rho >= 0.0) || !std::isfinite(rho) || !(dt > 0.0) || !std::isfinite(dt))
        return fail(nullptr, STA_EINVAL, "material parameters out of range (need -1 < nu < 0.5, rho >= 0, dt > 0)");
    for (int64_t i = 0; i < 3 * n_nodes; ++i)
        if (!std::isfinite(x[i]))
            return fail(nullptr, STA_EINVAL, "non-finite node coordinate");
    for (int64_t e = 0; e < n_tets; ++e) {
        const int32_t* t = tets + 4 * e;
        for (int a = 0; a < 4; ++a)
            if (t[a] < 0 || t[a] >= n_nodes)
                return fail(nullptr, STA_EINVAL, "tet " + std::to_string(e) + " has a vertex id out of range");
        for (int a = 0; a < 4; ++a)
            for (int b = a + 1; b < 4; ++b)
                if (t[a] == t[b])
                    return fail(nullptr, STA_EDEGENERATE, "tet " + std::to_string(e) + " repeats a vertex");
        if (!std::isfinite(E[e]))
            return fail(nullptr, STA_EINVAL, "non-finite Young's modulus");
        if (mask0[e] > 1)
            return fail(nullptr, STA_EINVAL, "mask0 values must be 0 or 1");
    }

    HostPattern P;
    std::string msg = build_host_pattern(n_nodes, tets, n_tets, P);
    if (!msg.empty())
        return fail(nullptr, STA_EINVAL, msg);

    sta_ctx* c = new (std::nothrow) sta_ctx();
    if (!c)
        return fail(nullptr, STA_ENOMEM, "host allocation failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    (void)hipGetDevice(&c->device);
    c->n_nodes = n_nodes;
    c->n_tets = n_tets;
    c->n_rows = 3 * n_nodes;
    c->nnz = P.nnz;
    c->nd = P.nd;
    c->no = P.no;
    for (int64_t b = 0; b < P.nd; ++b)
        c->bucket_blocks[diag_bucket(P.dseg[b + 1] - P.dseg[b])]++;
    for (int64_t o = 0; o < P.no; ++o)
        c->bucket_blocks[kDiagBuckets + off_bucket(P.oseg[o + 1] - P.oseg[o])]++;
    c->nu = nu;
    c->rho = rho;
    c->dt = dt;

    DevView& v = c->v;
    v.n_nodes = (int32_t)n_nodes;
    v.n_tets = (int32_t)n_tets;
    v.nd = (int32_t)P.nd;
    v.no = (int32_t)P.no;
    v.mat = material(nu, rho, dt);

    const int64_t nb = P.nd + P.no;
    double *xs, *E_d, *cd, *co, *values;
    int4* T;
    uint8_t *mask, *undo, *wg_err;
    int32_t *e2b, *e2p, *ndiag;
    BlockDesc *desc, *rec;
    uint32_t *estamp, *bstamp;
    Ctl* ctl;
    hipError_t e = hipSuccess;
#define ALLOC(ptr, count)                                  \
    if (e == hipSuccess)                                   \
        e = dalloc(c, &ptr, (size_t)(count));
    ALLOC(xs, 3 * n_nodes);
    ALLOC(T, n_tets);
    ALLOC(E_d, n_tets);
    ALLOC(mask, n_tets);
    ALLOC(c->rowptr, 3 * n_nodes + 1);
    ALLOC(c->colidx, P.nnz);
    ALLOC(values, P.nnz);
    ALLOC(desc, nb);
    ALLOC(ndiag, n_nodes);
    ALLOC(e2b, 10 * n_tets);
    ALLOC(e2p, 10 * n_tets);
    ALLOC(cd, 24 * n_tets);
    ALLOC(co, 54 * n_tets);
    ALLOC(estamp, n_tets);
    ALLOC(bstamp, nb);
    ALLOC(rec, 10 * n_tets + 160);
    int32_t* rcount = nullptr;
    ALLOC(rcount, 8 * ((16 * n_tets + 255) / 256 + 1));
    ALLOC(undo, n_tets);
    ALLOC(wg_err, 16 * n_tets / 256 + 4096);
    ALLOC(ctl, 1);
    ALLOC(c->dinc, 4 * n_tets);
    TetRecord* trec = nullptr;
    ALLOC(trec, n_tets);
    const int64_t n_chunks = (n_tets + kAdjointChunk - 1) / kAdjointChunk;
    ALLOC(c->adj_order, n_chunks);
#undef ALLOC
    if (e != hipSuccess) {
        free_all(c);
        delete c;
        return fail(nullptr, e == hipErrorOutOfMemory ? STA_ENOMEM : STA_EHIP,
                    std::string("device allocation: ") + hipGetErrorString(e));
    }

    // host-side SoA / int4 / descriptor staging
    std::vector<double> hx((size_t)3 * n_nodes);
    for (int64_t i = 0; i < n_nodes; ++i)
        for (int k = 0; k < 3; ++k)
            hx[(size_t)k * n_nodes + i] = x[3 * i + k];
    std::vector<int4> hT((size_t)n_tets);
    for (int64_t t = 0; t < n_tets; ++t)
        hT[t] = make_int4(tets[4 * t], tets[4 * t + 1], tets[4 * t + 2], tets[4 * t + 3]);
    std::vector<BlockDesc> hd((size_t)nb);
    for (int64_t b = 0; b < P.nd; ++b)
        hd[b] = BlockDesc{P.dseg[b], P.dseg[b + 1], P.dmeta[2 * b], P.dmeta[2 * b + 1],
                          P.dmeta[2 * b], P.dmeta[2 * b + 1], 0, (int32_t)b};
    for (int64_t o = 0; o < P.no; ++o)
        hd[P.nd + o] = BlockDesc{P.oseg[o], P.oseg[o + 1], P.ometa[4 * o], P.ometa[4 * o + 1],
                                 P.ometa[4 * o + 2], P.ometa[4 * o + 3], 1, (int32_t)(P.nd + o)};
    std::vector<int32_t> he2b(P.e2b);
    for (int64_t t = 0; t < n_tets; ++t)
        for (int j = 4; j < 10; ++j)
            he2b[10 * t + j] += (int32_t)P.nd;

    if (e == hipSuccess) e = upload(xs, hx.data(), hx.size(), s);
    if (e == hipSuccess) e = upload(T, hT.data(), hT.size(), s);
    if (e == hipSuccess) e = upload(E_d, E, (size_t)n_tets, s);
    if (e == hipSuccess) e = upload(mask, mask0, (size_t)n_tets, s);
    if (e == hipSuccess) e = upload(c->rowptr, P.rowptr.data(), P.rowptr.size(), s);
    if (e == hipSuccess) e = upload(c->colidx, P.colidx.data(), P.colidx.size(), s);
    if (e == hipSuccess) e = upload(desc, hd.data(), hd.size(), s);
    if (e == hipSuccess) e = upload(ndiag, P.ndiag.data(), P.ndiag.size(), s);
    if (e == hipSuccess) e = upload(e2b, he2b.data(), he2b.size(), s);
    if (e == hipSuccess) e = upload(e2p, P.e2p.data(), P.e2p.size(), s);
    if (e == hipSuccess) e = upload(c->dinc, P.dinc.data(), P.dinc.size(), s);
    const std::vector<int32_t> order = adjoint_chunk_order(x, hT, node_off, tet_off);
    if (e == hipSuccess) e = upload(c->adj_order, order.data(), order.size(), s);
    c->adj_chunks = (int32_t)n_chunks;
    {
        std::vector<TetRecord> hr((size_t)n_tets);
        for (int64_t t = 0; t < n_tets; ++t) {
            TetRecord& r = hr[t];
            std::memset(&r, 0, sizeof r);
            for (int j = 0; j < 10; ++j) {
                r.desc[j] = hd[he2b[10 * t + j]];
                r.pos[j] = P.e2p[10 * t + j];
            }
            r.T = hT[t];
        }
        if (e == hipSuccess) e = upload(trec, hr.data(), hr.size(), s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);  // hr is freed at the end of this block
    }
    if (e == hipSuccess && n_tets > 0) e = hipMemsetAsync(estamp, 0, sizeof(uint32_t) * n_tets, s);
    if (e == hipSuccess && nb > 0) e = hipMemsetAsync(bstamp, 0, sizeof(uint32_t) * nb, s);
    if (e == hipSuccess && P.nnz > 0) e = hipMemsetAsync(values, 0, sizeof(double) * P.nnz, s);
    if (e == hipSuccess) e = hipMemsetAsync(ctl, 0, sizeof(Ctl), s);

    v.xs = xs;
    v.ys = xs + n_nodes;
    v.zs = xs + 2 * n_nodes;
    v.T = T;
    v.E = E_d;
    v.mask = mask;
    v.desc = desc;
    v.ndiag = ndiag;
    v.e2b = e2b;
    v.e2p = e2p;
    v.trec = trec;
    v.cd = cd;
    v.co = co;
    v.values = values;
    v.estamp = estamp;
    v.bstamp = bstamp;
    v.rec = rec;
    v.rcount = rcount;
    v.undo = undo;
    v.wg_err = wg_err;
    v.ctl = ctl;

    // the records' geometry, computed on the device with the element kernel's routine
    if (e == hipSuccess) e = launch_refresh_records(v, trec, s);
    if (e == hipSuccess) e = launch_element(v, false, s);
    if (e == hipSuccess) e = launch_reduce_all(v, c->rebuild_map, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    int32_t bits = 0;
    if (e == hipSuccess) e = hipMemcpy(&bits, &ctl->err, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        free_all(c);
        delete c;
        return fail(nullptr, STA_EHIP, std::string("build: ") + hipGetErrorString(e));
    }
    if (bits & ERR_DEGENERATE) {
        free_all(c);
        delete c;
        return fail(nullptr, STA_EDEGENERATE, "a candidate tet has zero volume (det == 0)");
    }
    const char* tp = std::getenv("STA_TRACE");
    if (tp && *tp) {
        c->trace = std::fopen(tp, "a");
        if (!c->trace) {
            free_all(c);
            delete c;
            return fail(nullptr, STA_EINVAL, std::string("STA_TRACE: cannot open ") + tp + " for appending");
        }
        const char* ts = std::getenv("STA_TRACE_STATS");
        c->trace_stats = ts && std::atoi(ts) != 0;
        c->trace_t0 = host_seconds();
    }
    c->node_off = node_off;
    c->tet_off = tet_off;
    c->rebuild_groups = rebuild_groups(P, hd, node_off, tet_off);
    c->nnz_off.resize(node_off.size());
    for (size_t j = 0; j < node_off.size(); ++j)
        c->nnz_off[j] = P.rowptr[3 * node_off[j]];
    *out = c;
    return STA_OK;
}

}  // namespace sta

namespace {

// One JSON line per traced call (after the call's launches are queued).  With
// trace_stats the stream is synchronised and the frame's statistics added.
void trace_call(sta_ctx* ctx, const char* call, int64_t n, bool n_is_capacity, hipStream_t s)
{
    if (!ctx->trace)
        return;
    const char* mode = ctx->fused ? "one launch" : "two launches";
    std::fprintf(ctx->trace, "{\"seq\": %lld, \"call\": \"%s\", \"%s\": %lld, \"frame_mode\": \"%s\", "
                 "\"host_us\": %.1f",
                 (long long)ctx->trace_seq++, call, n_is_capacity ? "capacity" : "edits", (long long)n, mode,
                 (host_seconds() - ctx->trace_t0) * 1e6);
    if (ctx->trace_stats && std::strncmp(call, "apply_edits", 11) == 0) {
        int64_t st[STA_NUM_FRAME_STATS] = {0};
        if (sta_last_frame_stats(ctx, s, st, STA_NUM_FRAME_STATS) == STA_OK)
            std::fprintf(ctx->trace,
                         ", \"stats\": {\"diag_blocks\": %lld, \"off_blocks\": %lld, \"diag_incidences\": %lld, "
                         "\"off_incidences\": %lld, \"touched_slots\": %lld, \"changed\": %lld, "
                         "\"activated\": %lld, \"edits\": %lld, \"rolled_back\": %lld}",
                         (long long)st[0], (long long)st[1], (long long)st[2], (long long)st[3], (long long)st[4],
                         (long long)st[5], (long long)st[6], (long long)st[7], (long long)st[8]);
    }
    std::fprintf(ctx->trace, "}\n");
    std::fflush(ctx->trace);
}

// One frame: two launches, or one persistent launch.
sta_status run_frame(sta_ctx* ctx, const int32_t* ids, const uint8_t* states, int32_t n_host, const int32_t* n_dev,
                     hipStream_t s)
{
    hipError_t e = hipSuccess;
    if (ctx->fused) {
        if (ctx->frame_max_grid <= 0) {
            e = frame_max_grid(ctx->stream_map, ctx->device, &ctx->frame_max_grid);
            if (e != hipSuccess)
                return hip_fail(ctx, e, "occupancy query");
            if (ctx->frame_max_grid <= 0)
                return fail(ctx, STA_EINVAL, "fused frame kernel cannot be resident");
        }
        const int grid = frame_grid_for(ctx->stream_map, n_host, ctx->frame_max_grid, ctx->frame_grid_cap);
        e = timed(
            ctx, STA_KERNEL_FRAME, s,
            [&] {
                return launch_frame(ctx->v, ctx->stream_map, grid, ids, states, n_host, n_dev, ctx->barrier_spin, s);
            },
            true);
        ctx->fused_used = true;
    } else {
        e = timed(
            ctx, STA_KERNEL_EDITS, s, [&] { return launch_edit_phase(ctx->v, ids, states, n_host, n_dev, s); },
            true);
        if (e == hipSuccess)
            e = timed(
                ctx, STA_KERNEL_TOUCHED, s,
                [&] { return launch_touched_phase(ctx->v, ctx->stream_map, ids, n_host, n_dev, s); }, true);
    }
    if (e != hipSuccess)
        return hip_fail(ctx, e, "frame launch");
    return STA_OK;
}

bool valid_map(int qd, int qo)
{
    return (qd == 1 || qd == 4 || qd == 16) && (qo == 1 || qo == 4);
}

}  // namespace

extern "C" {

sta_status sta_build_pattern(const double* x, int64_t n_nodes, const int32_t* tets, int64_t n_tets,
                             const double* E, double nu, double rho, double dt, const uint8_t* mask0,
                             void* stream, sta_ctx** out)
{
    return sta::build_context(x, n_nodes, tets, n_tets, E, nu, rho, dt, mask0, stream, {0, n_nodes},
                              {0, n_tets}, out);
}

sta_status sta_full_rebuild(sta_ctx* ctx, void* stream)
{
    if (!ctx)
        return STA_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (ctx->fused_used) {
        // a fused frame whose grid barrier gave up leaves stamps taken: release them all
        e = launch_clear_stamps(ctx->v, s);
        if (e == hipSuccess)
            ctx->fused_used = ctx->fused != 0;
    }
    const bool nt = ctx->rebuild_map.nt != 0;
    if (ctx->rebuild_groups.empty()) {
        if (e == hipSuccess)
            e = timed(ctx, STA_KERNEL_ELEMENT, s, [&] { return launch_element(ctx->v, nt, s); }, true);
        if (e == hipSuccess)
            e = timed(ctx, STA_KERNEL_REDUCE, s, [&] { return launch_reduce_all(ctx->v, ctx->rebuild_map, s); }, true);
    }
    for (const auto& g : ctx->rebuild_groups) {
        // views of the group's tets, of its diagonal blocks and of its off-diagonal blocks (the
        // reduce takes the diagonal blocks at desc[0, nd) and the off-diagonal ones at desc[nd, nd + no))
        DevView vt = ctx->v;
        vt.n_tets = (int32_t)(g[1] - g[0]);
        vt.T += g[0];
        vt.E += g[0];
        vt.mask += g[0];
        vt.e2b += 10 * g[0];
        vt.e2p += 10 * g[0];
        vt.trec += g[0];
        vt.estamp += g[0];
        DevView vd = ctx->v;
        vd.desc += g[2];
        vd.nd = (int32_t)(g[3] - g[2]);
        vd.no = 0;
        DevView vo = ctx->v;
        vo.desc += ctx->v.nd + g[4];
        vo.nd = 0;
        vo.no = (int32_t)(g[5] - g[4]);
        if (e == hipSuccess)
            e = timed(ctx, STA_KERNEL_ELEMENT, s, [&] { return launch_element(vt, nt, s); }, true);
        if (e == hipSuccess)
            e = timed(ctx, STA_KERNEL_REDUCE, s, [&] { return launch_reduce_all(vd, ctx->rebuild_map, s); }, true);
        if (e == hipSuccess)
            e = timed(ctx, STA_KERNEL_REDUCE, s, [&] { return launch_reduce_all(vo, ctx->rebuild_map, s); }, true);
    }
    if (e != hipSuccess)
        return hip_fail(ctx, e, "full_rebuild launch");
    ctx->stale = false;
    trace_call(ctx, "full_rebuild", 0, false, s);
    return STA_OK;
}

sta_status sta_apply_edits(sta_ctx* ctx, const int32_t* ids_dev, const uint8_t* states_dev, int64_t n_edits,
                           void* stream)
{
    if (!ctx)
        return STA_EINVAL;
    if (n_edits < 0 || n_edits > ctx->n_tets)
        return fail(ctx, STA_EINVAL, "n_edits must be in [0, n_tets] (ids are distinct)");
    if (n_edits > 0 && (!ids_dev || !states_dev))
        return fail(ctx, STA_EINVAL, "NULL edit array");
    if (ctx->stale)
        return fail(ctx, STA_ESTALE, "parameters changed: call sta_full_rebuild before sta_apply_edits");
    const sta_status st = run_frame(ctx, ids_dev, states_dev, (int32_t)n_edits, nullptr,
                                    static_cast<hipStream_t>(stream));
    if (st == STA_OK)
        trace_call(ctx, "apply_edits", n_edits, false, static_cast<hipStream_t>(stream));
    return st;
}

sta_status sta_apply_edits_dev(sta_ctx* ctx, const int32_t* ids_dev, const uint8_t* states_dev, const int32_t* n_dev,
                               int64_t capacity, void* stream)
{
    if (!ctx)
        return STA_EINVAL;
    if (capacity < 1 || capacity > ctx->n_tets)
        return fail(ctx, STA_EINVAL, "capacity must be in [1, n_tets]");
    if (!ids_dev || !states_dev || !n_dev)
        return fail(ctx, STA_EINVAL, "NULL edit array or count");
    if (ctx->stale)
        return fail(ctx, STA_ESTALE, "parameters changed: call sta_full_rebuild before sta_apply_edits_dev");
    const sta_status st = run_frame(ctx, ids_dev, states_dev, (int32_t)capacity, n_dev,
                                    static_cast<hipStream_t>(stream));
    if (st == STA_OK)
        trace_call(ctx, "apply_edits_dev", capacity, true, static_cast<hipStream_t>(stream));
    return st;
}

sta_status sta_apply_edits_delta(sta_ctx* ctx, const int32_t* ids_dev, const uint8_t* states_dev, int64_t n_edits,
                                 const int32_t* n_dev, void* stream)
{
    if (!ctx)
        return STA_EINVAL;
    if (n_edits < 0 || n_edits > ctx->n_tets || (n_dev && n_edits < 1))
        return fail(ctx, STA_EINVAL, "n_edits must be in [0, n_tets] ([1, n_tets] as a capacity)");
    if (n_edits > 0 && (!ids_dev || !states_dev))
        return fail(ctx, STA_EINVAL, "NULL edit array");
    if (ctx->stale)
        return fail(ctx, STA_ESTALE, "parameters changed: call sta_full_rebuild before sta_apply_edits_delta");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const hipError_t e = timed(ctx, STA_KERNEL_DELTA, s, [&] {
        return launch_delta_frame(ctx->v, ids_dev, states_dev, (int32_t)n_edits, n_dev, s);
    });
    if (e != hipSuccess)
        return hip_fail(ctx, e, "delta frame");
    trace_call(ctx, "apply_edits_delta", n_edits, n_dev != nullptr, s);
    return STA_OK;
}

const double* sta_values_ptr(const sta_ctx* ctx)
{
    return ctx ? ctx->v.values : nullptr;
}

sta_status sta_copy_values(const sta_ctx* ctx, double* dst_dev, void* stream)
{
    if (!ctx || (ctx->nnz > 0 && !dst_dev))
        return STA_EINVAL;
    if (ctx->nnz == 0)
        return STA_OK;
    hipError_t e = hipMemcpyAsync(dst_dev, ctx->v.values, sizeof(double) * ctx->nnz, hipMemcpyDeviceToDevice,
                                  static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_fail(const_cast<sta_ctx*>(ctx), e, "copy values");
    return STA_OK;
}

sta_status sta_sizes(const sta_ctx* ctx, int64_t* n_rows, int64_t* nnz, int64_t* n_diag_blocks, int64_t* n_off_blocks)
{
    if (!ctx)
        return STA_EINVAL;
    if (n_rows) *n_rows = ctx->n_rows;
    if (nnz) *nnz = ctx->nnz;
    if (n_diag_blocks) *n_diag_blocks = ctx->nd;
    if (n_off_blocks) *n_off_blocks = ctx->no;
    return STA_OK;
}

sta_status sta_pattern_ptrs(const sta_ctx* ctx, const int32_t** rowptr_dev, const int32_t** colidx_dev,
                            const uint8_t** mask_dev)
{
    if (!ctx)
        return STA_EINVAL;
    if (rowptr_dev) *rowptr_dev = ctx->rowptr;
    if (colidx_dev) *colidx_dev = ctx->colidx;
    if (mask_dev) *mask_dev = ctx->v.mask;
    return STA_OK;
}

sta_status sta_pattern_host(const sta_ctx* ctx, int32_t* rowptr, int32_t* colidx)
{
    if (!ctx || !rowptr || (ctx->nnz > 0 && !colidx))
        return STA_EINVAL;
    hipError_t e = hipMemcpy(rowptr, ctx->rowptr, sizeof(int32_t) * (ctx->n_rows + 1), hipMemcpyDeviceToHost);
    if (e == hipSuccess && ctx->nnz > 0)
        e = hipMemcpy(colidx, ctx->colidx, sizeof(int32_t) * ctx->nnz, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_fail(const_cast<sta_ctx*>(ctx), e, "pattern copy");
    return STA_OK;
}

sta_status sta_last_frame_stats(sta_ctx* ctx, void* stream, int64_t* out, int n_out)
{
    if (!ctx || (n_out > 0 && !out))
        return STA_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(s);
    Ctl h{};
    if (e == hipSuccess)
        e = hipMemcpy(&h, ctx->v.ctl, sizeof(Ctl), hipMemcpyDeviceToHost);
    const int64_t n = (h.last_n >= 0 && h.last_n <= ctx->n_tets) ? h.last_n : 0;
    const int64_t max_regions = 4 * ((16 * ctx->n_tets + 255) / 256 + 1);
    const int64_t g = (h.last_regions >= 0 && h.last_regions <= max_regions) ? h.last_regions : 0;
    std::vector<BlockDesc> rc((size_t)g * 40);
    std::vector<int32_t> cnt((size_t)g * 2);
    std::vector<uint8_t> un((size_t)n);
    if (e == hipSuccess && g > 0)
        e = hipMemcpy(rc.data(), ctx->v.rec, sizeof(BlockDesc) * rc.size(), hipMemcpyDeviceToHost);
    if (e == hipSuccess && g > 0)
        e = hipMemcpy(cnt.data(), ctx->v.rcount, sizeof(int32_t) * cnt.size(), hipMemcpyDeviceToHost);
    if (e == hipSuccess && n > 0)
        e = hipMemcpy(un.data(), ctx->v.undo, un.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "stats copy");
    int64_t st[STA_NUM_FRAME_STATS] = {0};
    st[7] = n;
    st[8] = (n > 0 && h.frame_err != 0) ? 1 : 0;
    if (n > 0 && h.frame_err == 0) {
        for (int64_t w = 0; w < g; ++w) {
            for (int k = 0; k < cnt[2 * w] && k < 16; ++k) {
                const BlockDesc& d = rc[40 * w + k];
                st[0] += 1;
                st[2] += d.k1 - d.k0;
                st[4] += 9;
            }
            for (int k = 0; k < cnt[2 * w + 1] && k < 24; ++k) {
                const BlockDesc& d = rc[40 * w + 16 + k];
                st[1] += 1;
                st[3] += d.k1 - d.k0;
                st[4] += 18;
            }
        }
        for (int64_t i = 0; i < n; ++i)
            if (un[i] != 0xFF) {
                st[5] += 1;
                if (un[i] == 0)
                    st[6] += 1;
            }
    }
    for (int k = 0; k < n_out && k < STA_NUM_FRAME_STATS; ++k)
        out[k] = st[k];
    return STA_OK;
}

sta_status sta_enable_kernel_timing(sta_ctx* ctx, int on)
{
    if (!ctx)
        return STA_EINVAL;
    ctx->timing = on != 0;
    return STA_OK;
}

sta_status sta_kernel_times(sta_ctx* ctx, void* stream, int64_t* launches, double* ms)
{
    if (!ctx || !launches || !ms)
        return STA_EINVAL;
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    if (e != hipSuccess)
        return hip_fail(ctx, e, "kernel_times sync");
    for (int k = 0; k < STA_NUM_KERNELS; ++k) {
        launches[k] = 0;
        ms[k] = 0.0;
    }
    for (auto& t : ctx->timed) {
        float dt = 0.0f;
        if (hipEventElapsedTime(&dt, t.a, t.b) == hipSuccess && t.kernel >= 0 && t.kernel < STA_NUM_KERNELS) {
            launches[t.kernel] += 1;
            ms[t.kernel] += dt;
        }
        ctx->event_pool.push_back(t.a);
        ctx->event_pool.push_back(t.b);
    }
    ctx->timed.clear();
    return STA_OK;
}

sta_status sta_set_params(sta_ctx* ctx, const double* x_dev, const double* E_dev, void* stream)
{
    if (!ctx)
        return STA_EINVAL;
    if (!x_dev && !E_dev)
        return STA_OK;
    double* xs = const_cast<double*>(ctx->v.xs);
    hipError_t e = launch_set_params(ctx->v, x_dev, E_dev, xs, xs + ctx->n_nodes, xs + 2 * ctx->n_nodes,
                                     const_cast<double*>(ctx->v.E), static_cast<hipStream_t>(stream));
    if (e == hipSuccess)
        e = launch_refresh_records(ctx->v, const_cast<TetRecord*>(ctx->v.trec), static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_fail(ctx, e, "set_params launch");
    ctx->stale = true;
    ctx->tet_ml_stale = true;
    return STA_OK;
}

sta_status sta_status_sync(sta_ctx* ctx, void* stream)
{
    if (!ctx)
        return STA_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(s);
    int32_t bits = 0;
    if (e == hipSuccess)
        e = hipMemcpy(&bits, &ctx->v.ctl->err, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && bits != 0) {
        const int32_t zero = 0;
        e = hipMemcpy(&ctx->v.ctl->err, &zero, sizeof(int32_t), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess)
        return hip_fail(ctx, e, "status sync");
    if (bits & ERR_TIMEOUT) {
        // Workgroups that gave up left before phase 2: their share of the touched
        // blocks was not re-summed and the stamps it would have released stay
        // taken.  Release every stamp now and refuse frames until a rebuild.
        const uint32_t zero2[2] = {0u, 0u};
        e = hipMemcpy(&ctx->v.ctl->bar_count, zero2, sizeof(zero2), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_clear_stamps(ctx->v, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        ctx->stale = true;
        if (e != hipSuccess)
            return hip_fail(ctx, e, "status sync after a barrier timeout");
        ctx->errmsg = "a fused frame's grid barrier timed out (GPU shared with other work); the frame is "
                      "incomplete (the mask holds its edits): call sta_full_rebuild before the next frame";
        return STA_ETIMEOUT;
    }
    const sta_status st = device_errors(bits);
    if (st == STA_ERANGE)
        ctx->errmsg = "an edit named a tet id outside [0, n_tets) or a state other than 0/1; frame rolled back";
    else if (st == STA_EDUP)
        ctx->errmsg = "an edit list named the same tet twice; frame rolled back";
    else if (st == STA_EDEGENERATE)
        ctx->errmsg = "an element with det == 0 was assembled";
    return st;
}

sta_status sta_set_config(sta_ctx* ctx, int fused, int rebuild_qd, int rebuild_qo, int stream_qd, int stream_qo,
                          int grid_cap, int rebuild_nt)
{
    if (!ctx || (fused != 0 && fused != 1) || !valid_map(rebuild_qd, rebuild_qo) || !valid_map(stream_qd, stream_qo) ||
        grid_cap < 0 || (rebuild_nt != 0 && rebuild_nt != 1))
        return STA_EINVAL;
    ctx->frame_max_grid = 0;  // the fused kernel's occupancy depends on the mapping
    ctx->fused = fused;
    ctx->rebuild_map = uniform_map(rebuild_qd, rebuild_qo, rebuild_nt);
    ctx->stream_map = uniform_map(stream_qd, stream_qo, 0);
    ctx->frame_grid_cap = grid_cap;
    return STA_OK;
}

sta_status sta_get_config(const sta_ctx* ctx, int* out7)
{
    if (!ctx || !out7)
        return STA_EINVAL;
    int* out6 = out7;
    out6[0] = ctx->fused;
    out6[1] = ctx->rebuild_map.qd;
    out6[2] = ctx->rebuild_map.qo;
    out6[3] = ctx->stream_map.qd;
    out6[4] = ctx->stream_map.qo;
    out6[5] = ctx->frame_grid_cap;
    out6[6] = ctx->rebuild_map.nt;
    return STA_OK;
}

sta_status sta_audit(sta_ctx* ctx, void* stream, int64_t* out2)
{
    if (!ctx || !out2)
        return STA_EINVAL;
    if (ctx->stale)
        return fail(ctx, STA_ESTALE, "parameters changed: call sta_full_rebuild before sta_audit");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (!ctx->audit_ws) {
        // nnz doubles, then two 8-byte counters (the allocation is 256-byte aligned)
        e = dalloc(ctx, &ctx->audit_ws, (size_t)ctx->nnz + 2);
        if (e != hipSuccess) {
            ctx->audit_ws = nullptr;
            return fail(ctx, STA_ENOMEM, "audit workspace allocation failed");
        }
    }
    unsigned long long* counts = reinterpret_cast<unsigned long long*>(ctx->audit_ws + ctx->nnz);
    e = hipMemsetAsync(counts, 0, 2 * sizeof(unsigned long long), s);
    if (e == hipSuccess)
        e = launch_audit(ctx->v, ctx->rebuild_map, ctx->audit_ws, ctx->nnz, counts, s);
    unsigned long long h[2] = {0, 0};
    if (e == hipSuccess)
        e = hipMemcpyAsync(h, counts, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "audit");
    out2[0] = (int64_t)h[0];
    out2[1] = (int64_t)h[1];
    return STA_OK;
}

sta_status sta_set_barrier_spin_limit(sta_ctx* ctx, int64_t polls)
{
    if (!ctx || polls < 0 || polls > (int64_t)UINT32_MAX)
        return STA_EINVAL;
    ctx->barrier_spin = polls == 0 ? kBarrierSpinDefault : (unsigned)polls;
    return STA_OK;
}

sta_status sta_set_bucket_map(sta_ctx* ctx, int which, const int* qd3, const int* qo2)
{
    if (!ctx || (which != 0 && which != 1) || !qd3 || !qo2)
        return STA_EINVAL;
    MapConfig m = which == 0 ? ctx->rebuild_map : ctx->stream_map;
    m.qd = 1;
    m.qo = 1;
    for (int b = 0; b < kDiagBuckets; ++b) {
        if (!valid_map(qd3[b], 1))
            return STA_EINVAL;
        m.qdb[b] = qd3[b];
        m.qd = qd3[b] > m.qd ? qd3[b] : m.qd;
    }
    for (int b = 0; b < kOffBuckets; ++b) {
        if (!valid_map(1, qo2[b]))
            return STA_EINVAL;
        m.qob[b] = qo2[b];
        m.qo = qo2[b] > m.qo ? qo2[b] : m.qo;
    }
    if (which == 0) {
        ctx->rebuild_map = m;
    } else {
        ctx->stream_map = m;
        ctx->frame_max_grid = 0;
    }
    return STA_OK;
}

sta_status sta_get_bucket_map(const sta_ctx* ctx, int which, int* qd3, int* qo2, int64_t* blocks5)
{
    if (!ctx || (which != 0 && which != 1))
        return STA_EINVAL;
    const MapConfig& m = which == 0 ? ctx->rebuild_map : ctx->stream_map;
    for (int b = 0; b < kDiagBuckets; ++b)
        if (qd3) qd3[b] = m.qdb[b];
    for (int b = 0; b < kOffBuckets; ++b)
        if (qo2) qo2[b] = m.qob[b];
    for (int b = 0; b < kDiagBuckets + kOffBuckets; ++b)
        if (blocks5) blocks5[b] = ctx->bucket_blocks[b];
    return STA_OK;
}

sta_status sta_batch_offsets(const sta_ctx* ctx, int* k, int64_t* node_off, int64_t* tet_off, int64_t* row_off,
                             int64_t* nnz_off, int64_t capacity)
{
    if (!ctx || !k)
        return STA_EINVAL;
    const int64_t nk = (int64_t)ctx->node_off.size() - 1;
    *k = (int)nk;
    if (capacity < nk + 1)
        return capacity == 0 ? STA_OK : STA_EINVAL;
    for (int64_t j = 0; j <= nk; ++j) {
        if (node_off) node_off[j] = ctx->node_off[j];
        if (tet_off) tet_off[j] = ctx->tet_off[j];
        if (row_off) row_off[j] = 3 * ctx->node_off[j];
        if (nnz_off) nnz_off[j] = ctx->nnz_off[j];
    }
    return STA_OK;
}

sta_status sta_adjoint(sta_ctx* ctx, const double* gA_dev, double* g_logE_dev, double* g_x_dev, void* stream)
{
    if (!ctx || (ctx->nnz > 0 && !gA_dev) || (ctx->n_tets > 0 && !g_logE_dev) || (ctx->n_nodes > 0 && !g_x_dev))
        return STA_EINVAL;
    if (ctx->stale)
        return fail(ctx, STA_ESTALE, "parameters changed: call sta_full_rebuild before sta_adjoint");
    hipError_t e = hipSuccess;
    if (!ctx->adj_xbar)
        e = dalloc(ctx, &ctx->adj_xbar, (size_t)12 * ctx->n_tets);
    if (e != hipSuccess)
        return fail(ctx, STA_ENOMEM, "adjoint workspace allocation failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    e = timed(ctx, STA_KERNEL_ADJOINT, s,
              [&] {
                  return launch_adjoint(ctx->v, ctx->adj_order, ctx->adj_chunks, gA_dev, g_logE_dev, g_x_dev,
                                        ctx->adj_xbar, s);
              });
    if (e != hipSuccess)
        return hip_fail(ctx, e, "adjoint launch");
    return STA_OK;
}

sta_status sta_slot_outer(sta_ctx* ctx, const double* a_dev, const double* b_dev, double alpha, double* out_dev,
                          void* stream)
{
    if (!ctx || (ctx->n_rows > 0 && (!a_dev || !b_dev)) || (ctx->nnz > 0 && !out_dev))
        return STA_EINVAL;
    hipError_t e = launch_slot_outer((int)ctx->n_rows, ctx->rowptr, ctx->colidx, a_dev, b_dev, alpha, out_dev,
                                     static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_fail(ctx, e, "slot_outer launch");
    return STA_OK;
}

sta_status sta_cg_solve(sta_ctx* ctx, const double* values_dev, const double* b_dev, double* x_dev, double rtol,
                        int max_iter, void* stream, int* iters_out, double* relres_out)
{
    if (!ctx || (ctx->n_rows > 0 && (!b_dev || !x_dev)) || !(rtol >= 0.0) || max_iter < 0)
        return STA_EINVAL;
    if (ctx->n_rows == 0) {
        if (iters_out) *iters_out = 0;
        if (relres_out) *relres_out = 0.0;
        return STA_OK;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int n = (int)ctx->n_rows;
    const int nparts = cg_partials(n);
    hipError_t e = hipSuccess;
    if (!ctx->cg_ws) {
        e = dalloc(ctx, &ctx->cg_ws, (size_t)7 * n + nparts);
        if (e == hipSuccess)
            e = dalloc(ctx, &ctx->cg_dpos, (size_t)n);
        if (e == hipSuccess)
            e = dalloc(ctx, &ctx->cg_s, 1);
        if (e == hipSuccess)
            e = hipHostMalloc((void**)&ctx->cg_host, sizeof(CgScalars), hipHostMallocDefault);
        if (e == hipSuccess)
            e = launch_diag_positions(ctx->v, ctx->cg_dpos, s);
        if (e != hipSuccess) {
            ctx->cg_ws = nullptr;
            return fail(ctx, STA_ENOMEM, "CG workspace allocation failed");
        }
    }
    CgView c;
    c.n = n;
    c.nparts = (n + 255) / 256;
    c.nparts_s = spmv_grid(n);
    c.nparts_u = update_grid(n);
    c.rowptr = ctx->rowptr;
    c.colidx = ctx->colidx;
    c.vals = values_dev ? values_dev : ctx->v.values;
    c.dpos = ctx->cg_dpos;
    c.x = ctx->cg_ws;
    c.r = c.x + n;
    c.z = c.r + n;
    c.p = c.z + n;
    c.q = c.p + 2 * n;
    c.dinv = c.q + n;
    c.part = c.dinv + n;
    c.s = ctx->cg_s;
    e = launch_cg_init(c, b_dev, rtol, s);
    // iterations k = 0 .. max_iter (the last one only records the residual),
    // 16 at a time between host checks
    const int chunk = 16;
    int next = 0;
    while (e == hipSuccess) {
        const int count = max_iter + 1 - next < chunk ? max_iter + 1 - next : chunk;
        if (count > 0)
            e = timed(ctx, STA_KERNEL_SOLVE, s, [&] { return launch_cg_iterations(c, next, count, max_iter, s); });
        next += count;
        if (e == hipSuccess)
            e = hipMemcpyAsync(ctx->cg_host, ctx->cg_s, sizeof(CgScalars), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess || ctx->cg_host->done || next > max_iter)
            break;
    }
    if (e == hipSuccess)
        e = launch_cg_output(c, x_dev, s);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "cg");
    if (iters_out)
        *iters_out = ctx->cg_host->iters;
    if (relres_out)
        *relres_out = ctx->cg_host->bnorm2 > 0.0 ? std::sqrt(ctx->cg_host->rr / ctx->cg_host->bnorm2) : 0.0;
    return STA_OK;
}

const char* sta_last_error(const sta_ctx* ctx)
{
    if (!ctx)
        return g_build_err.c_str();
    return ctx->errmsg.c_str();
}

void sta_destroy(sta_ctx* ctx)
{
    if (!ctx)
        return;
    (void)hipDeviceSynchronize();
    for (auto& t : ctx->timed) {
        ctx->event_pool.push_back(t.a);
        ctx->event_pool.push_back(t.b);
    }
    for (hipEvent_t ev : ctx->event_pool)
        (void)hipEventDestroy(ev);
    if (ctx->cg_host)
        (void)hipHostFree(ctx->cg_host);
    if (ctx->cc_host)
        (void)hipHostFree(ctx->cc_host);
    if (ctx->trace)
        std::fclose(ctx->trace);
    free_all(ctx);
    delete ctx;
}

}  // extern "C"
