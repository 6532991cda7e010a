// The maintained lumped mass M_t and one implicit-Euler step of paper
// Sec. 6.2 eq. (9): (M_t + h^2 K_t) u_{t+1} = M_t (u_t + h v_t) + h^2 f, with
// h the context's time step (the matrix A_t = M_t + dt^2 K_t is the one this
// library maintains), solved by the Jacobi-PCG of cg.hip, and
// v_{t+1} = (u_{t+1} - u_t) / h.
//
// M_t per node is the sum of (rho V_e) / 4 over its active tets in ascending
// tet id from +0.0, the same term and order as the mass part of the
// diagonal of A_t; each vertex's three dofs share it.
#include <hip/hip_runtime.h>

#include <cmath>

#include "sta_internal.h"

#pragma clang fp contract(off)

namespace sta {
namespace {

constexpr int kBlock = 256;

unsigned blocks(int64_t n)
{
    return (unsigned)((n + kBlock - 1) / kBlock);
}

// (rho V) / 4 of every candidate, V = |det| / 6 with det evaluated in the
// element formula's fixed order.
__global__ __launch_bounds__(kBlock) void k_tet_mass(DevView v, double* __restrict__ ml)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= v.n_tets)
        return;
    const int4 t = v.T[e];
    const int id[4] = {t.x, t.y, t.z, t.w};
    double X[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        X[a][0] = v.xs[id[a]];
        X[a][1] = v.ys[id[a]];
        X[a][2] = v.zs[id[a]];
    }
    double d[4][3];
#pragma unroll
    for (int k = 1; k <= 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i)
            d[k][i] = X[k][i] - X[0][i];
    const double c0 = (d[2][1] * d[3][2]) - (d[2][2] * d[3][1]);
    const double c1 = (d[2][2] * d[3][0]) - (d[2][0] * d[3][2]);
    const double c2 = (d[2][0] * d[3][1]) - (d[2][1] * d[3][0]);
    const double det = ((d[1][0] * c0) + (d[1][1] * c1)) + (d[1][2] * c2);
    const double V = fabs(det) / 6.0;
    ml[e] = (v.mat.rho * V) * 0.25;
}

// One thread per node: its diagonal block's incidence segment in ascending
// tet id, active terms only.  Tet ids, mask bytes and masses are loaded
// kChunk at a time and then added in order (a few memory round trips per
// segment instead of two per term).
__global__ __launch_bounds__(kBlock) void k_lumped_mass(DevView v, const int32_t* __restrict__ dinc,
                                                        const double* __restrict__ ml, double* __restrict__ m)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= v.n_nodes)
        return;
    double acc = 0.0;
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
            double w[kChunk];
#pragma unroll
            for (int j = 0; j < kChunk; ++j) {
                on[j] = e[j] >= 0 && v.mask[e[j]];
                w[j] = e[j] >= 0 ? ml[e[j]] : 0.0;
            }
#pragma unroll
            for (int j = 0; j < kChunk; ++j)
                if (on[j])
                    acc = acc + w[j];
        }
    }
    m[3 * (size_t)i + 0] = acc;
    m[3 * (size_t)i + 1] = acc;
    m[3 * (size_t)i + 2] = acc;
}

__global__ __launch_bounds__(kBlock) void k_euler_rhs(int n, const double* __restrict__ m,
                                                      const double* __restrict__ u, const double* __restrict__ vel,
                                                      const double* __restrict__ f, double h, double* __restrict__ b)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r < n)
        b[r] = (m[r] * (u[r] + (h * vel[r]))) + ((h * h) * f[r]);
}

__global__ __launch_bounds__(kBlock) void k_euler_update(int n, const double* __restrict__ u1, double* __restrict__ u,
                                                         double* __restrict__ vel, double h)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r < n) {
        const double x = u1[r];
        vel[r] = (x - u[r]) / h;
        u[r] = x;
    }
}

}  // namespace

hipError_t launch_tet_mass(const DevView& v, double* tet_ml, hipStream_t s)
{
    if (v.n_tets == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_tet_mass, dim3(blocks(v.n_tets)), dim3(kBlock), 0, s, v, tet_ml);
    return hipGetLastError();
}

hipError_t launch_lumped_mass(const DevView& v, const int32_t* dinc, const double* tet_ml, double* m, hipStream_t s)
{
    if (v.n_nodes == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_lumped_mass, dim3(blocks(v.n_nodes)), dim3(kBlock), 0, s, v, dinc, tet_ml, m);
    return hipGetLastError();
}

hipError_t launch_euler_rhs(int n, const double* m, const double* u, const double* v, const double* f, double h,
                            double* b, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_euler_rhs, dim3(blocks(n)), dim3(kBlock), 0, s, n, m, u, v, f, h, b);
    return hipGetLastError();
}

hipError_t launch_euler_update(int n, const double* u1, double* u, double* v, double h, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_euler_update, dim3(blocks(n)), dim3(kBlock), 0, s, n, u1, u, v, h);
    return hipGetLastError();
}

}  // namespace sta

using namespace sta;

namespace {

sta_status efail(sta_ctx* ctx, sta_status code, const char* what, hipError_t e)
{
    ctx->errmsg = std::string(what) + ": " + hipGetErrorString(e);
    return code;
}

// M_t of the current mask into m (device, n_rows), refreshing the per-tet
// masses first if the parameters changed.
sta_status lumped_mass_into(sta_ctx* ctx, double* m, hipStream_t s)
{
    hipError_t e = hipSuccess;
    if (!ctx->tet_ml) {
        void* q = nullptr;
        e = hipMalloc(&q, sizeof(double) * (size_t)(ctx->n_tets ? ctx->n_tets : 1));
        if (e != hipSuccess)
            return efail(ctx, STA_ENOMEM, "tet mass allocation", e);
        ctx->owned.push_back(q);
        ctx->tet_ml = static_cast<double*>(q);
        ctx->tet_ml_stale = true;
    }
    if (ctx->tet_ml_stale) {
        e = launch_tet_mass(ctx->v, ctx->tet_ml, s);
        if (e != hipSuccess)
            return efail(ctx, STA_EHIP, "tet mass", e);
        ctx->tet_ml_stale = false;
    }
    e = launch_lumped_mass(ctx->v, ctx->dinc, ctx->tet_ml, m, s);
    return e == hipSuccess ? STA_OK : efail(ctx, STA_EHIP, "lumped mass", e);
}

}  // namespace

extern "C" sta_status sta_lumped_mass(sta_ctx* ctx, double* m_dev, void* stream)
{
    if (!ctx || (ctx->n_rows > 0 && !m_dev))
        return STA_EINVAL;
    return lumped_mass_into(ctx, m_dev, static_cast<hipStream_t>(stream));
}

extern "C" sta_status sta_euler_step(sta_ctx* ctx, double* u_dev, double* v_dev, const double* f_dev, double rtol,
                                     int max_iter, void* stream, int* iters_out, double* relres_out)
{
    if (!ctx || (ctx->n_rows > 0 && (!u_dev || !v_dev || !f_dev)) || !(rtol >= 0.0) || max_iter < 0)
        return STA_EINVAL;
    if (ctx->stale) {
        ctx->errmsg = "parameters changed: call sta_full_rebuild before sta_euler_step";
        return STA_ESTALE;
    }
    const int n = (int)ctx->n_rows;
    if (n == 0) {
        if (iters_out) *iters_out = 0;
        if (relres_out) *relres_out = 0.0;
        return STA_OK;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!ctx->euler_ws) {
        void* q = nullptr;
        const hipError_t e = hipMalloc(&q, sizeof(double) * 3 * (size_t)n);
        if (e != hipSuccess)
            return efail(ctx, STA_ENOMEM, "Euler workspace allocation", e);
        ctx->owned.push_back(q);
        ctx->euler_ws = static_cast<double*>(q);
    }
    double* m = ctx->euler_ws;
    double* b = m + n;
    double* u1 = b + n;
    sta_status st = lumped_mass_into(ctx, m, s);
    if (st != STA_OK)
        return st;
    hipError_t e = launch_euler_rhs(n, m, u_dev, v_dev, f_dev, ctx->dt, b, s);
    if (e != hipSuccess)
        return efail(ctx, STA_EHIP, "Euler right-hand side", e);
    st = sta_cg_solve(ctx, nullptr, b, u1, rtol, max_iter, stream, iters_out, relres_out);
    if (st != STA_OK)
        return st;
    e = launch_euler_update(n, u1, u_dev, v_dev, ctx->dt, s);
    return e == hipSuccess ? STA_OK : efail(ctx, STA_EHIP, "Euler update", e);
}
