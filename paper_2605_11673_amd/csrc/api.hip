// C ABI of libstafem.so (declared in include/stafem.h): argument checks,
// device allocation, the host pattern hand-off and kernel sequencing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>

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

template <class T>
hipError_t dalloc(sta_ctx* c, T** p, size_t count)
{
    void* q = nullptr;
    size_t bytes = count * sizeof(T);
    if (bytes == 0)
        bytes = 256;
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

}  // namespace

extern "C" {

sta_status sta_build_pattern(const double* x, int64_t n_nodes, const int32_t* tets, int64_t n_tets,
                             const double* E, double nu, double rho, double dt, const uint8_t* mask0,
                             void* stream, sta_ctx** out)
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
    c->nu = nu;
    c->rho = rho;
    c->dt = dt;
    c->h_dseg = P.dseg;
    c->h_oseg = P.oseg;

    DevView& v = c->v;
    v.n_nodes = (int32_t)n_nodes;
    v.n_tets = (int32_t)n_tets;
    v.nd = (int32_t)P.nd;
    v.no = (int32_t)P.no;
    v.mat = material(nu, rho, dt);

    double *xs, *E_d, *cd, *co, *values;
    int4* T;
    uint8_t *mask, *undo;
    int32_t *dseg, *dinc, *oseg, *oinc, *e2b, *e2p, *claims;
    int2* dmeta;
    int4* ometa;
    uint32_t *cver, *estamp, *dstamp, *ostamp;
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
    ALLOC(dseg, P.nd + 1);
    ALLOC(dinc, 4 * n_tets);
    ALLOC(dmeta, P.nd);
    ALLOC(oseg, P.no + 1);
    ALLOC(oinc, 6 * n_tets);
    ALLOC(ometa, P.no);
    ALLOC(e2b, 10 * n_tets);
    ALLOC(e2p, 10 * n_tets);
    ALLOC(cd, 24 * n_tets);
    ALLOC(co, 54 * n_tets);
    ALLOC(cver, n_tets);
    ALLOC(estamp, n_tets);
    ALLOC(dstamp, P.nd);
    ALLOC(ostamp, P.no);
    ALLOC(claims, 10 * n_tets);
    ALLOC(undo, n_tets);
    ALLOC(ctl, 1);
#undef ALLOC
    if (e != hipSuccess) {
        free_all(c);
        delete c;
        return fail(nullptr, e == hipErrorOutOfMemory ? STA_ENOMEM : STA_EHIP,
                    std::string("device allocation: ") + hipGetErrorString(e));
    }

    // host-side SoA / int4 staging
    std::vector<double> hx((size_t)3 * n_nodes);
    for (int64_t i = 0; i < n_nodes; ++i)
        for (int k = 0; k < 3; ++k)
            hx[(size_t)k * n_nodes + i] = x[3 * i + k];
    std::vector<int4> hT((size_t)n_tets);
    for (int64_t t = 0; t < n_tets; ++t)
        hT[t] = make_int4(tets[4 * t], tets[4 * t + 1], tets[4 * t + 2], tets[4 * t + 3]);
    std::vector<int2> hdm((size_t)P.nd);
    for (int64_t b = 0; b < P.nd; ++b)
        hdm[b] = make_int2(P.dmeta[2 * b], P.dmeta[2 * b + 1]);
    std::vector<int4> hom((size_t)P.no);
    for (int64_t b = 0; b < P.no; ++b)
        hom[b] = make_int4(P.ometa[4 * b], P.ometa[4 * b + 1], P.ometa[4 * b + 2], P.ometa[4 * b + 3]);

    if (e == hipSuccess) e = upload(xs, hx.data(), hx.size(), s);
    if (e == hipSuccess) e = upload(T, hT.data(), hT.size(), s);
    if (e == hipSuccess) e = upload(E_d, E, (size_t)n_tets, s);
    if (e == hipSuccess) e = upload(mask, mask0, (size_t)n_tets, s);
    if (e == hipSuccess) e = upload(c->rowptr, P.rowptr.data(), P.rowptr.size(), s);
    if (e == hipSuccess) e = upload(c->colidx, P.colidx.data(), P.colidx.size(), s);
    if (e == hipSuccess) e = upload(dseg, P.dseg.data(), P.dseg.size(), s);
    if (e == hipSuccess) e = upload(dinc, P.dinc.data(), P.dinc.size(), s);
    if (e == hipSuccess) e = upload(dmeta, hdm.data(), hdm.size(), s);
    if (e == hipSuccess) e = upload(oseg, P.oseg.data(), P.oseg.size(), s);
    if (e == hipSuccess) e = upload(oinc, P.oinc.data(), P.oinc.size(), s);
    if (e == hipSuccess) e = upload(ometa, hom.data(), hom.size(), s);
    if (e == hipSuccess) e = upload(e2b, P.e2b.data(), P.e2b.size(), s);
    if (e == hipSuccess) e = upload(e2p, P.e2p.data(), P.e2p.size(), s);
    if (e == hipSuccess && n_tets > 0) e = hipMemsetAsync(cver, 0, sizeof(uint32_t) * n_tets, s);
    if (e == hipSuccess && n_tets > 0) e = hipMemsetAsync(estamp, 0, sizeof(uint32_t) * n_tets, s);
    if (e == hipSuccess && P.nd > 0) e = hipMemsetAsync(dstamp, 0, sizeof(uint32_t) * P.nd, s);
    if (e == hipSuccess && P.no > 0) e = hipMemsetAsync(ostamp, 0, sizeof(uint32_t) * P.no, s);
    if (e == hipSuccess && P.nnz > 0) e = hipMemsetAsync(values, 0, sizeof(double) * P.nnz, s);
    if (e == hipSuccess) e = hipMemsetAsync(ctl, 0, sizeof(Ctl), s);

    v.xs = xs;
    v.ys = xs + n_nodes;
    v.zs = xs + 2 * n_nodes;
    v.T = T;
    v.E = E_d;
    v.mask = mask;
    v.dseg = dseg;
    v.dinc = dinc;
    v.dmeta = dmeta;
    v.oseg = oseg;
    v.oinc = oinc;
    v.ometa = ometa;
    v.e2b = e2b;
    v.e2p = e2p;
    v.cd = cd;
    v.co = co;
    v.cver = cver;
    v.values = values;
    v.estamp = estamp;
    v.dstamp = dstamp;
    v.ostamp = ostamp;
    v.claims = claims;
    v.undo = undo;
    v.ctl = ctl;

    if (e == hipSuccess) e = launch_element(v, true, c->ver, s);
    if (e == hipSuccess) e = launch_reduce_all(v, s);
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
    *out = c;
    return STA_OK;
}

sta_status sta_full_rebuild(sta_ctx* ctx, void* stream)
{
    if (!ctx)
        return STA_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = launch_element(ctx->v, false, ctx->ver, s);
    if (e == hipSuccess)
        e = launch_reduce_all(ctx->v, s);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "full_rebuild launch");
    ctx->stale = false;
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
    ctx->last_n_edits = n_edits;
    if (n_edits == 0)
        return STA_OK;
    hipError_t e = launch_edits(ctx->v, ids_dev, states_dev, (int32_t)n_edits, ctx->ver,
                                static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_fail(ctx, e, "apply_edits launch");
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

sta_status sta_last_frame_stats(sta_ctx* ctx, void* stream, int64_t* touched_blocks, int64_t* touched_slots,
                                int64_t* touched_incidences, int64_t* changed, int64_t* activated)
{
    if (!ctx)
        return STA_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(s);
    const int64_t n = ctx->last_n_edits;
    std::vector<int32_t> cl((size_t)n * 10);
    std::vector<uint8_t> un((size_t)n);
    int32_t ferr = 0;
    if (e == hipSuccess && n > 0)
        e = hipMemcpy(cl.data(), ctx->v.claims, sizeof(int32_t) * cl.size(), hipMemcpyDeviceToHost);
    if (e == hipSuccess && n > 0)
        e = hipMemcpy(un.data(), ctx->v.undo, un.size(), hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipMemcpy(&ferr, &ctx->v.ctl->frame_err, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_fail(ctx, e, "stats copy");
    int64_t nb = 0, ns = 0, ni = 0, nc = 0, na = 0;
    if (n > 0 && ferr == 0) {
        for (int64_t i = 0; i < n; ++i) {
            for (int j = 0; j < 10; ++j) {
                const int32_t b = cl[10 * i + j];
                if (b < 0)
                    continue;
                ++nb;
                if (j < 4) {
                    ns += 9;
                    ni += ctx->h_dseg[b + 1] - ctx->h_dseg[b];
                } else {
                    ns += 18;
                    ni += ctx->h_oseg[b + 1] - ctx->h_oseg[b];
                }
            }
            if (un[i] != 0xFF) {
                ++nc;
                if (un[i] == 0)
                    ++na;
            }
        }
    }
    if (touched_blocks) *touched_blocks = nb;
    if (touched_slots) *touched_slots = ns;
    if (touched_incidences) *touched_incidences = ni;
    if (changed) *changed = nc;
    if (activated) *activated = na;
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
    if (e != hipSuccess)
        return hip_fail(ctx, e, "set_params launch");
    ctx->ver += 1;
    ctx->stale = true;
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
    const sta_status st = device_errors(bits);
    if (st == STA_ERANGE)
        ctx->errmsg = "an edit named a tet id outside [0, n_tets) or a state other than 0/1; frame rolled back";
    else if (st == STA_EDUP)
        ctx->errmsg = "an edit list named the same tet twice; frame rolled back";
    else if (st == STA_EDEGENERATE)
        ctx->errmsg = "an element with det == 0 was assembled";
    return st;
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
    free_all(ctx);
    delete ctx;
}

}  // extern "C"
