// Batched contexts (many independent meshes in one context) and the
// autotuner that picks the slot mapping and the frame execution mode.
//
// A batch of meshes is their disjoint union: node, tet, row and value ranges
// are concatenated, so every kernel of the single-mesh path applies
// unchanged, a frame over all meshes is one launch (or one graph replay),
// and each mesh's values are bitwise what it would get alone (its blocks only
// ever see its own tets, summed in the same order).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "sta_internal.h"

using namespace sta;

namespace {

sta_status tune_fail(sta_ctx* ctx, sta_status code, const std::string& msg)
{
    ctx->errmsg = msg;
    return code;
}

struct Cfg {
    int fused, rqd, rqo, sqd, sqo, cap, nt;
    int rdb[kDiagBuckets], rob[kOffBuckets];  // rebuild mapping per incidence-length bucket
    int sdb[kDiagBuckets], sob[kOffBuckets];  // streaming mapping per bucket
};

constexpr int kCfgInts = 7 + 2 * (kDiagBuckets + kOffBuckets);

void cfg_ints(const Cfg& c, int* x)
{
    const int head[7] = {c.fused, c.rqd, c.rqo, c.sqd, c.sqo, c.cap, c.nt};
    int k = 0;
    for (int v : head) x[k++] = v;
    for (int v : c.rdb) x[k++] = v;
    for (int v : c.rob) x[k++] = v;
    for (int v : c.sdb) x[k++] = v;
    for (int v : c.sob) x[k++] = v;
}

Cfg cfg_from(const int* x)
{
    Cfg c;
    c.fused = x[0], c.rqd = x[1], c.rqo = x[2], c.sqd = x[3], c.sqo = x[4], c.cap = x[5], c.nt = x[6];
    int k = 7;
    for (int& v : c.rdb) v = x[k++];
    for (int& v : c.rob) v = x[k++];
    for (int& v : c.sdb) v = x[k++];
    for (int& v : c.sob) v = x[k++];
    return c;
}

// Uniform mappings: every bucket as the allocation.
void set_uniform(Cfg& c)
{
    for (int& v : c.rdb) v = c.rqd;
    for (int& v : c.rob) v = c.rqo;
    for (int& v : c.sdb) v = c.sqd;
    for (int& v : c.sob) v = c.sqo;
}

Cfg current(const sta_ctx* ctx)
{
    Cfg c{ctx->fused, ctx->rebuild_map.qd, ctx->rebuild_map.qo, ctx->stream_map.qd, ctx->stream_map.qo,
          ctx->frame_grid_cap, ctx->rebuild_map.nt, {}, {}, {}, {}};
    for (int b = 0; b < kDiagBuckets; ++b) {
        c.rdb[b] = ctx->rebuild_map.qdb[b];
        c.sdb[b] = ctx->stream_map.qdb[b];
    }
    for (int b = 0; b < kOffBuckets; ++b) {
        c.rob[b] = ctx->rebuild_map.qob[b];
        c.sob[b] = ctx->stream_map.qob[b];
    }
    return c;
}

sta_status apply(sta_ctx* ctx, const Cfg& c)
{
    sta_status st = sta_set_config(ctx, c.fused, c.rqd, c.rqo, c.sqd, c.sqo, c.cap, c.nt);
    if (st == STA_OK)
        st = sta_set_bucket_map(ctx, 0, c.rdb, c.rob);
    if (st == STA_OK)
        st = sta_set_bucket_map(ctx, 1, c.sdb, c.sob);
    return st;
}

std::string describe(const Cfg& c)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "fused %d rebuild %dx%d nt %d [%d %d %d | %d %d] stream %dx%d cap %d [%d %d %d | %d %d]",
                  c.fused, c.rqd, c.rqo, c.nt, c.rdb[0], c.rdb[1], c.rdb[2], c.rob[0], c.rob[1], c.sqd, c.sqo, c.cap,
                  c.sdb[0], c.sdb[1], c.sdb[2], c.sob[0], c.sob[1]);
    return buf;
}

std::string cache_key(const sta_ctx* ctx, int64_t n_edits)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "stafem-tune-v3 %lld %lld %lld %lld %lld %lld", (long long)ctx->n_nodes,
                  (long long)ctx->n_tets, (long long)ctx->nnz, (long long)ctx->nd, (long long)ctx->no,
                  (long long)n_edits);
    return buf;
}

bool cache_lookup(const char* path, const std::string& key, Cfg& c)
{
    FILE* f = std::fopen(path, "r");
    if (!f)
        return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        const char* bar = std::strchr(line, '|');
        if (!bar)
            continue;
        std::string k(line, bar - line);
        while (!k.empty() && k.back() == ' ')
            k.pop_back();
        if (k != key)
            continue;
        int x[kCfgInts];
        int n = 0, used = 0;
        const char* p = bar + 1;
        while (n < kCfgInts && std::sscanf(p, "%d%n", &x[n], &used) == 1) {
            p += used;
            ++n;
        }
        if (n == kCfgInts) {
            c = cfg_from(x);  // the last matching line wins
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char* path, const std::string& key, const Cfg& c)
{
    FILE* f = std::fopen(path, "a");
    if (!f)
        return;
    int x[kCfgInts];
    cfg_ints(c, x);
    std::fprintf(f, "%s |", key.c_str());
    for (int v : x)
        std::fprintf(f, " %d", v);
    std::fprintf(f, "\n");
    std::fclose(f);
}

double median(std::vector<float> v)
{
    std::sort(v.begin(), v.end());
    return v.empty() ? 0.0 : v[v.size() / 2];
}

const int kMaps[6][2] = {{1, 1}, {1, 4}, {4, 1}, {4, 4}, {16, 1}, {16, 4}};

}  // namespace

extern "C" {

sta_status sta_batch_build(int k, const double* const* x, const int64_t* n_nodes, const int32_t* const* tets,
                           const int64_t* n_tets, const double* const* E, double nu, double rho, double dt,
                           const uint8_t* const* mask0, void* stream, sta_ctx** out)
{
    build_error().clear();
    if (!out || k < 1 || !x || !n_nodes || !tets || !n_tets || !E || !mask0) {
        build_error() = "sta_batch_build: bad arguments";
        return STA_EINVAL;
    }
    *out = nullptr;
    std::vector<int64_t> noff(k + 1, 0), toff(k + 1, 0);
    for (int j = 0; j < k; ++j) {
        if (n_nodes[j] < 0 || n_tets[j] < 0) {
            build_error() = "sta_batch_build: negative size";
            return STA_EINVAL;
        }
        noff[j + 1] = noff[j] + n_nodes[j];
        toff[j + 1] = toff[j] + n_tets[j];
    }
    if (noff[k] > INT32_MAX / 3 || toff[k] > INT32_MAX / 10) {
        build_error() = "sta_batch_build: batch too large";
        return STA_EINVAL;
    }
    std::vector<double> X((size_t)3 * noff[k]), Ev((size_t)toff[k]);
    std::vector<int32_t> T((size_t)4 * toff[k]);
    std::vector<uint8_t> M((size_t)toff[k]);
    for (int j = 0; j < k; ++j) {
        if ((n_nodes[j] > 0 && !x[j]) || (n_tets[j] > 0 && (!tets[j] || !E[j] || !mask0[j]))) {
            build_error() = "sta_batch_build: NULL mesh array";
            return STA_EINVAL;
        }
        if (n_nodes[j] > 0)
            std::memcpy(&X[3 * noff[j]], x[j], sizeof(double) * 3 * n_nodes[j]);
        for (int64_t t = 0; t < n_tets[j]; ++t)
            for (int a = 0; a < 4; ++a) {
                const int32_t v = tets[j][4 * t + a];
                if (v < 0 || v >= n_nodes[j]) {
                    build_error() = "sta_batch_build: mesh " + std::to_string(j) + " tet " + std::to_string(t) +
                                    " has a vertex id out of range";
                    return STA_EINVAL;
                }
                T[4 * (toff[j] + t) + a] = (int32_t)(v + noff[j]);
            }
        if (n_tets[j] > 0) {
            std::memcpy(&Ev[toff[j]], E[j], sizeof(double) * n_tets[j]);
            std::memcpy(&M[toff[j]], mask0[j], n_tets[j]);
        }
    }
    return build_context(X.data(), noff[k], T.data(), toff[k], Ev.data(), nu, rho, dt, M.data(), stream, noff, toff,
                         out);
}

sta_status sta_autotune(sta_ctx* ctx, const int32_t* ids_dev, const uint8_t* states_dev, int64_t n_edits, int reps,
                        void* stream, char* report, int64_t report_len)
{
    if (!ctx || n_edits < 1 || n_edits > ctx->n_tets || !ids_dev || !states_dev)
        return STA_EINVAL;
    if (ctx->stale)
        return tune_fail(ctx, STA_ESTALE, "parameters changed: call sta_full_rebuild before sta_autotune");
    if (reps < 1)
        reps = 7;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::string rep;
    char line[320];
    const char* cache = std::getenv("STA_TUNE_CACHE");
    const std::string key = cache_key(ctx, n_edits);
    Cfg best{};
    auto finish = [&](sta_status st) {
        if (report && report_len > 0) {
            std::strncpy(report, rep.c_str(), (size_t)report_len - 1);
            report[report_len - 1] = 0;
        }
        return st;
    };
    if (cache && cache_lookup(cache, key, best)) {
        const sta_status st = apply(ctx, best);
        std::snprintf(line, sizeof line, "cached %s: %s\n", cache, describe(best).c_str());
        rep += line;
        return finish(st);
    }

    // the inverse frame: same ids, each tet's current state
    std::vector<int32_t> ids((size_t)n_edits);
    std::vector<uint8_t> mask((size_t)ctx->n_tets), inv((size_t)n_edits);
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess)
        e = hipMemcpy(ids.data(), ids_dev, sizeof(int32_t) * n_edits, hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipMemcpy(mask.data(), ctx->v.mask, ctx->n_tets, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return tune_fail(ctx, STA_EHIP, "autotune copies failed");
    {
        std::vector<int32_t> sorted(ids);
        std::sort(sorted.begin(), sorted.end());
        if (sorted.front() < 0 || sorted.back() >= ctx->n_tets ||
            std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
            return tune_fail(ctx, STA_EINVAL, "autotune needs a valid frame (ids in range, distinct)");
    }
    for (int64_t i = 0; i < n_edits; ++i)
        inv[i] = mask[ids[i]];
    uint8_t* inv_dev = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    e = hipMalloc(&inv_dev, n_edits);
    if (e == hipSuccess)
        e = hipMemcpy(inv_dev, inv.data(), n_edits, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipEventCreate(&a);
    if (e == hipSuccess)
        e = hipEventCreate(&b);
    auto cleanup = [&]() {
        if (inv_dev)
            (void)hipFree(inv_dev);
        if (a)
            (void)hipEventDestroy(a);
        if (b)
            (void)hipEventDestroy(b);
    };
    if (e != hipSuccess) {
        cleanup();
        return tune_fail(ctx, STA_ENOMEM, "autotune workspace");
    }
    const Cfg saved = current(ctx);
    const int saved_timing = ctx->timing;
    ctx->timing = false;
    sta_status st = STA_OK;

    // median time of one rebuild / of one streaming frame (each undone by
    // its inverse) under configuration c, in microseconds
    auto time_rebuild = [&](const Cfg& c) {
        std::vector<float> t;
        if (st == STA_OK)
            st = apply(ctx, c);
        for (int r = 0; r <= reps && st == STA_OK; ++r) {
            float ms = 0.0f;
            (void)hipEventRecord(a, s);
            st = sta_full_rebuild(ctx, stream);
            (void)hipEventRecord(b, s);
            (void)hipEventSynchronize(b);
            (void)hipEventElapsedTime(&ms, a, b);
            if (r > 0)
                t.push_back(ms);
        }
        return median(t) * 1e3;
    };
    auto time_frame = [&](const Cfg& c) {
        std::vector<float> t;
        if (st == STA_OK)
            st = apply(ctx, c);
        for (int r = 0; r <= reps && st == STA_OK; ++r) {
            float ms = 0.0f;
            (void)hipEventRecord(a, s);
            st = sta_apply_edits(ctx, ids_dev, states_dev, n_edits, stream);
            (void)hipEventRecord(b, s);
            if (st == STA_OK)
                st = sta_apply_edits(ctx, ids_dev, inv_dev, n_edits, stream);
            (void)hipEventSynchronize(b);
            (void)hipEventElapsedTime(&ms, a, b);
            if (r > 0)
                t.push_back(ms);
        }
        return median(t) * 1e3;
    };
    // one bucket at a time, each group size of that bucket alone; a change
    // is kept only if it is at least 1% faster
    auto refine = [&](Cfg& c, double& t_best, bool rebuild) {
        const char* what = rebuild ? "rebuild" : "frame  ";
        for (int bk = 0; bk < kDiagBuckets + kOffBuckets && st == STA_OK; ++bk) {
            if (ctx->bucket_blocks[bk] == 0)
                continue;
            const bool diag = bk < kDiagBuckets;
            const int nq = diag ? 3 : 2;
            const int qs[3] = {1, 4, 16};
            int* slot = diag ? (rebuild ? &c.rdb[bk] : &c.sdb[bk])
                             : (rebuild ? &c.rob[bk - kDiagBuckets] : &c.sob[bk - kDiagBuckets]);
            const int keep = *slot;
            int chosen = keep;
            for (int k = 0; k < nq && st == STA_OK; ++k) {
                if (qs[k] == keep)
                    continue;
                *slot = qs[k];
                const double t = rebuild ? time_rebuild(c) : time_frame(c);
                std::snprintf(line, sizeof line, "%s  bucket %s%d (%lld blocks) q %2d: %9.2f us\n", what,
                              diag ? "d" : "o", diag ? bk : bk - kDiagBuckets, (long long)ctx->bucket_blocks[bk],
                              qs[k], t);
                rep += line;
                if (t < 0.99 * t_best) {
                    t_best = t;
                    chosen = qs[k];
                }
            }
            *slot = chosen;
        }
    };

    // 1. rebuild: uniform mappings, then per bucket
    double best_t = 1e30;
    best = saved;
    for (int nt = 0; nt <= 1 && st == STA_OK; ++nt)
        for (auto& m : kMaps) {
            Cfg c = saved;
            c.rqd = m[0], c.rqo = m[1], c.nt = nt;
            set_uniform(c);
            const double med = time_rebuild(c);
            std::snprintf(line, sizeof line, "rebuild  map %2dx%d nt %d: %9.2f us\n", m[0], m[1], nt, med);
            rep += line;
            if (med < best_t) {
                best_t = med;
                best.rqd = m[0];
                best.rqo = m[1];
                best.nt = nt;
            }
        }
    for (int bk = 0; bk < kDiagBuckets; ++bk)
        best.rdb[bk] = best.rqd;
    for (int bk = 0; bk < kOffBuckets; ++bk)
        best.rob[bk] = best.rqo;
    refine(best, best_t, true);
    // the allocation is the largest group of any bucket
    best.rqd = std::max({best.rdb[0], best.rdb[1], best.rdb[2]});
    best.rqo = std::max(best.rob[0], best.rob[1]);

    // 2. streaming frame: mapping x mode, then per bucket
    best_t = 1e30;
    const int caps[3] = {0, 256, 1024};
    for (int fused = 0; fused <= 1 && st == STA_OK; ++fused)
        for (auto& m : kMaps)
            for (int ci = 0; ci < (fused ? 3 : 1) && st == STA_OK; ++ci) {
                Cfg c = best;
                c.fused = fused, c.sqd = m[0], c.sqo = m[1], c.cap = caps[ci];
                for (int bk = 0; bk < kDiagBuckets; ++bk)
                    c.sdb[bk] = m[0];
                for (int bk = 0; bk < kOffBuckets; ++bk)
                    c.sob[bk] = m[1];
                const double med = time_frame(c);
                std::snprintf(line, sizeof line, "frame    %s map %2dx%d cap %4d: %9.2f us\n",
                              fused ? "fused" : "2-launch", m[0], m[1], caps[ci], med);
                rep += line;
                if (med < best_t) {
                    best_t = med;
                    best.fused = fused;
                    best.sqd = m[0];
                    best.sqo = m[1];
                    best.cap = caps[ci];
                }
            }
    for (int bk = 0; bk < kDiagBuckets; ++bk)
        best.sdb[bk] = best.sqd;
    for (int bk = 0; bk < kOffBuckets; ++bk)
        best.sob[bk] = best.sqo;
    refine(best, best_t, false);
    best.sqd = std::max({best.sdb[0], best.sdb[1], best.sdb[2]});
    best.sqo = std::max(best.sob[0], best.sob[1]);

    ctx->timing = saved_timing;
    if (st == STA_OK && hipStreamSynchronize(s) == hipSuccess && sta_status_sync(ctx, stream) == STA_OK) {
        st = apply(ctx, best);
        std::snprintf(line, sizeof line, "chosen: %s\n", describe(best).c_str());
        rep += line;
        if (cache && st == STA_OK)
            cache_store(cache, key, best);
    } else {
        (void)apply(ctx, saved);
        if (st == STA_OK)
            st = STA_EHIP;
    }
    cleanup();
    return finish(st);
}

}  // extern "C"
