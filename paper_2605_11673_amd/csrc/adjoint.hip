// Adjoint of the assembly: slot cotangents gA = dL/dvalues -> dL/dlogE per tet
// and dL/dx per node.
//
// For an active tet with element matrix
//   A[3a+i][3b+j] = lamV g_ai g_bj + muV g_aj g_bi + [i=j] muV (g_a.g_b) + [a=b][i=j] m,
// lamV = lambda V dt^2, muV = mu V dt^2, m = rho V / 4, V = |det D| / 6,
// g_k = column k of G = D^-T (k = 1..3), g_0 = -(g_1 + g_2 + g_3), D = [x1-x0, x2-x0, x3-x0]:
// with Abar the 12x12 gather of gA over the tet's slots and B_ab = Abar_ab + Abar_ba^T,
//   P_lam = sum_ab g_a^T Abar_ab g_b,  P_mu = sum_ab (g_b^T Abar_ab g_a + tr(Abar_ab) g_a.g_b),
//   P_m = sum_a tr(Abar_aa),
//   dL/dlogE = lamV P_lam + muV P_mu        (lambda, mu proportional to E = exp(logE)),
//   gbar_a = sum_b (lamV B_ab + muV B_ab^T + muV tr(B_ab) I) g_b,
//   Vbar = (lambda dt^2) P_lam + (mu dt^2) P_mu + (rho/4) P_m,
//   Dbar = -G Gbar^T G + (Vbar sign(det) / 6) det G,  Gbar columns gbar_k - gbar_0,
//   xbar_k = column k of Dbar (k = 1..3), xbar_0 = -(xbar_1 + xbar_2 + xbar_3).
// Inactive tets contribute nothing.  Per-vertex xbar are stored at the tet's
// diagonal incidence positions and summed per node over the node's
// incidence segment in ascending tet id (fixed order, no floating atomics).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "sta_internal.h"

#pragma clang fp contract(off)

namespace sta {

namespace {

constexpr int kBlock = 256;

struct Geo {
    double g[4][3];
    double det, V;
};

__device__ __forceinline__ void geometry(const DevView& v, int4 t, Geo& G)
{
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
    double c[4][3];
    const int nx[4][2] = {{0, 0}, {2, 3}, {3, 1}, {1, 2}};
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
        const double* a = d[nx[k][0]];
        const double* b = d[nx[k][1]];
        c[k][0] = (a[1] * b[2]) - (a[2] * b[1]);
        c[k][1] = (a[2] * b[0]) - (a[0] * b[2]);
        c[k][2] = (a[0] * b[1]) - (a[1] * b[0]);
    }
    const double det = ((d[1][0] * c[1][0]) + (d[1][1] * c[1][1])) + (d[1][2] * c[1][2]);
    const double inv = 1.0 / det;
#pragma unroll
    for (int k = 1; k <= 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i)
            G.g[k][i] = c[k][i] * inv;
#pragma unroll
    for (int i = 0; i < 3; ++i)
        G.g[0][i] = -((G.g[1][i] + G.g[2][i]) + G.g[3][i]);
    G.det = det;
    G.V = fabs(det) / 6.0;
}

// Gather the 3x3 cotangent block Abar_ab (rows: vertex a dofs, columns: vertex b dofs).
__device__ __forceinline__ void gather_block(const DevView& v, const double* __restrict__ gA, const int* id, int a,
                                             int b, int blk, double out[3][3])
{
    const BlockDesc d = v.desc[blk];
    if (a == b) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                out[i][j] = gA[d.up + i * d.rl + j];
    } else if (id[a] < id[b]) {  // row node of the stored block is vertex a
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                out[i][j] = gA[d.up + i * d.rl + j];
    } else {  // row node is vertex b: entry (3a+i, 3b+j) is the mirror part
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                out[i][j] = gA[d.lo + i * d.rlj + j];
    }
}

// The element pass's dynamic LDS, reserved and unused: it caps the pass at two
// workgroups per CU.  More resident waves gather more cotangent rows at once
// than the caches hold (on the 384k-tet fracture state: 81 us at two
// workgroups per CU, 86 us at three, 97 us at four).
constexpr size_t kAdjointReservedLds = 56 << 10;

__global__ __launch_bounds__(kBlock) void k_adjoint_element(DevView v, const int32_t* __restrict__ order,
                                                            int32_t n_chunks, const double* __restrict__ gA,
                                                            double* __restrict__ g_logE, double* __restrict__ xbar)
{
    // each XCD takes one contiguous share of the chunk order, chunks that are
    // near in space: neighbouring tets share node blocks, so their cotangent
    // rows stay in one L2 (132 -> 85 us for contiguous eighths of the tet ids
    // on the 384k-tet fracture state; 81 -> 79 us for the Morton chunk order
    // over the id order, both at two workgroups per CU; same bits throughout)
    constexpr int kPer = kBlock / kAdjointChunk;
    const int slot = xcd_remap(blockIdx.x, gridDim.x) * kPer + threadIdx.x / kAdjointChunk;
    if (slot >= n_chunks)
        return;
    const int e = order[slot] * kAdjointChunk + (threadIdx.x % kAdjointChunk);
    if (e >= v.n_tets)
        return;
    const int* pos = v.e2p + 10 * (size_t)e;
    if (!v.mask[e]) {
        g_logE[e] = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            double* dst = xbar + 3 * (size_t)pos[a];
            dst[0] = 0.0;
            dst[1] = 0.0;
            dst[2] = 0.0;
        }
        return;
    }
    const int4 t = v.T[e];
    const int id[4] = {t.x, t.y, t.z, t.w};
    const int* eb = v.e2b + 10 * (size_t)e;
    Geo G;
    geometry(v, t, G);
    const double E = v.E[e];
    const double lam_dt = (E * v.mat.clam) * v.mat.cdt;  // lambda dt^2
    const double mu_dt = (E * v.mat.cmu) * v.mat.cdt;    // mu dt^2
    const double lamV = lam_dt * G.V, muV = mu_dt * G.V;

    double Plam = 0.0, Pmu = 0.0, Pm = 0.0;
    double gbar[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i)
            gbar[a][i] = 0.0;

    // pairs (a, b) with a <= b; B_ab = Abar_ab + Abar_ba^T, B_ba = B_ab^T
    constexpr int PA[10] = {0, 1, 2, 3, 0, 0, 0, 1, 1, 2};
    constexpr int PB[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};
#pragma unroll
    for (int q = 0; q < 10; ++q) {
        const int a = PA[q], b = PB[q];
        double Aab[3][3], Aba[3][3];
        gather_block(v, gA, id, a, b, eb[q], Aab);
        if (a == b) {
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    Aba[i][j] = Aab[i][j];
        } else {
            gather_block(v, gA, id, b, a, eb[q], Aba);
        }
        // P terms over (a,b) and, for a != b, (b,a)
        const double* ga = G.g[a];
        const double* gb = G.g[b];
        const double sab = (ga[0] * gb[0] + ga[1] * gb[1]) + ga[2] * gb[2];
        double t_ab = 0.0, t_ba = 0.0, plam = 0.0, pmu = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                plam += ga[i] * Aab[i][j] * gb[j];
                pmu += gb[i] * Aab[i][j] * ga[j];
                if (a != b) {
                    plam += gb[i] * Aba[i][j] * ga[j];
                    pmu += ga[i] * Aba[i][j] * gb[j];
                }
            }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            t_ab += Aab[i][i];
            t_ba += Aba[i][i];
        }
        if (a == b) {
            Plam += plam;
            Pmu += pmu + t_ab * sab;
            Pm += t_ab;
        } else {
            Plam += plam;
            Pmu += pmu + (t_ab + t_ba) * sab;
        }
        // gbar: B_ab = Aab + Aba^T drives gbar_a (with g_b); B_ba = B_ab^T drives gbar_b (with g_a)
        double B[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                B[i][j] = Aab[i][j] + Aba[j][i];
        const double trB = (B[0][0] + B[1][1]) + B[2][2];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double ua = 0.0, ub = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                ua += (lamV * B[i][j] + muV * B[j][i]) * gb[j];
                if (a != b)
                    ub += (lamV * B[j][i] + muV * B[i][j]) * ga[j];
            }
            gbar[a][i] += ua + muV * trB * gb[i];
            if (a != b)
                gbar[b][i] += ub + muV * trB * ga[i];
        }
    }
    g_logE[e] = lamV * Plam + muV * Pmu;

    const double Vbar = lam_dt * Plam + mu_dt * Pmu + 0.25 * v.mat.rho * Pm;
    const double detbar = Vbar * (G.det < 0.0 ? -1.0 : 1.0) / 6.0;
    // Gbar columns k = 1..3: gbar_k - gbar_0 ; G columns g_k
    double Gm[3][3], Gb[3][3];  // [row i][col k-1]
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            Gm[i][k] = G.g[k + 1][i];
            Gb[i][k] = gbar[k + 1][i] - gbar[0][i];
        }
    // Dbar = -G Gbar^T G + detbar det G
    double T1[3][3];  // Gbar^T G
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            T1[i][j] = (Gb[0][i] * Gm[0][j] + Gb[1][i] * Gm[1][j]) + Gb[2][i] * Gm[2][j];
    double Db[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Db[i][j] = -((Gm[i][0] * T1[0][j] + Gm[i][1] * T1[1][j]) + Gm[i][2] * T1[2][j]) +
                       detbar * G.det * Gm[i][j];
    double xb[4][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        xb[1][i] = Db[i][0];
        xb[2][i] = Db[i][1];
        xb[3][i] = Db[i][2];
        xb[0][i] = -((Db[i][0] + Db[i][1]) + Db[i][2]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        double* dst = xbar + 3 * (size_t)pos[a];
        dst[0] = xb[a][0];
        dst[1] = xb[a][1];
        dst[2] = xb[a][2];
    }
}

// dL/dx of node i, component c: its diagonal segment's xbar in ascending tet id.
// Terms are loaded kChunk at a time and then added in order, so that a
// segment costs a few memory round trips instead of one per term.
__global__ __launch_bounds__(kBlock) void k_adjoint_nodes(DevView v, const double* __restrict__ xbar,
                                                          double* __restrict__ g_x)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= 3 * v.n_nodes)
        return;
    const int i = t / 3, c = t - 3 * (t / 3);
    const int b = v.ndiag[i];
    double acc = 0.0;
    if (b >= 0) {
        const BlockDesc d = v.desc[b];
        constexpr int kChunk = 8;
        for (int k0 = d.k0; k0 < d.k1; k0 += kChunk) {
            double x[kChunk];
#pragma unroll
            for (int j = 0; j < kChunk; ++j)
                x[j] = k0 + j < d.k1 ? xbar[3 * (size_t)(k0 + j) + c] : 0.0;
#pragma unroll
            for (int j = 0; j < kChunk; ++j)
                if (k0 + j < d.k1)
                    acc = acc + x[j];
        }
    }
    g_x[t] = acc;
}

// out[slot(r, c)] = alpha * a[r] * b[c] over the pattern.
__global__ __launch_bounds__(kBlock) void k_slot_outer(int n_rows, const int32_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ colidx, const double* __restrict__ a,
                                                       const double* __restrict__ b, double alpha,
                                                       double* __restrict__ out)
{
    const int r = blockIdx.x * (kBlock / 16) + threadIdx.x / 16;
    const int l = threadIdx.x & 15;
    if (r >= n_rows)
        return;
    const double ar = alpha * a[r];
    for (int s = rowptr[r] + l; s < rowptr[r + 1]; s += 16)
        out[s] = ar * b[colidx[s]];
}

}  // namespace

hipError_t launch_adjoint(const DevView& v, const int32_t* order, int32_t n_chunks, const double* gA, double* g_logE,
                          double* g_x, double* xbar, hipStream_t s)
{
    // kBlock / kAdjointChunk chunks per workgroup, so the grid covers n_chunks
    const unsigned grid = (unsigned)((n_chunks + kBlock / kAdjointChunk - 1) / (kBlock / kAdjointChunk));
    if (v.n_tets > 0)
        hipLaunchKernelGGL(k_adjoint_element, dim3(grid), dim3(kBlock), kAdjointReservedLds, s, v, order, n_chunks,
                           gA, g_logE, xbar);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || v.n_nodes == 0)
        return e;
    hipLaunchKernelGGL(k_adjoint_nodes, dim3((3 * v.n_nodes + kBlock - 1) / kBlock), dim3(kBlock), 0, s, v, xbar,
                       g_x);
    return hipGetLastError();
}

hipError_t launch_slot_outer(int n_rows, const int32_t* rowptr, const int32_t* colidx, const double* a,
                             const double* b, double alpha, double* out, hipStream_t s)
{
    if (n_rows == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_slot_outer, dim3((n_rows + kBlock / 16 - 1) / (kBlock / 16)), dim3(kBlock), 0, s, n_rows,
                       rowptr, colidx, a, b, alpha, out);
    return hipGetLastError();
}

}  // namespace sta

// ---------------------------------------------------------------------------
// Adjoint without allocation: the per-vertex cotangents live in a fixed
// device array of the library instead of a context workspace.
// ---------------------------------------------------------------------------

namespace {

// 3 doubles per diagonal incidence (4 per tet): room for 524,288 tets.
constexpr size_t kNoAllocTets = size_t(1) << 19;
constexpr size_t kNoAllocDoubles = 12 * kNoAllocTets;  // 48 MiB

static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per
// device (the current one); NULL on failure.
double* scratch_for_current_device(hipError_t& err)
{
    int dev = -1;
    err = hipGetDevice(&dev);
    if (err != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        if (err == hipSuccess)
            err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (err != hipSuccess)
            return nullptr;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" sta_status sta_adjoint_noalloc(sta_ctx* ctx, const double* gA_dev, double* g_logE_dev, double* g_x_dev,
                                          void* stream)
{
    if (!ctx || (ctx->nnz > 0 && !gA_dev) || (ctx->n_tets > 0 && !g_logE_dev) || (ctx->n_nodes > 0 && !g_x_dev))
        return STA_EINVAL;
    if ((size_t)ctx->n_tets > kNoAllocTets) {
        ctx->errmsg = "sta_adjoint_noalloc: " + std::to_string(ctx->n_tets) + " tets exceed the fixed workspace (" +
                      std::to_string(kNoAllocTets) + " tets); use sta_adjoint";
        return STA_EINVAL;
    }
    if (ctx->stale) {
        ctx->errmsg = "parameters changed: call sta_full_rebuild before sta_adjoint_noalloc";
        return STA_ESTALE;
    }
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && dev != ctx->device) {
        ctx->errmsg = "sta_adjoint_noalloc: the current device is not the context's device";
        return STA_EINVAL;
    }
    double* xbar = e == hipSuccess ? scratch_for_current_device(e) : nullptr;
    if (!xbar) {
        ctx->errmsg = std::string("sta_adjoint_noalloc: workspace address: ") + hipGetErrorString(e);
        return STA_EHIP;
    }
    // every diagonal incidence's three entries are written by the element pass
    // before the node pass reads them, so nothing needs clearing
    e = sta::launch_adjoint(ctx->v, ctx->adj_order, ctx->adj_chunks, gA_dev, g_logE_dev, g_x_dev, xbar,
                            static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        ctx->errmsg = std::string("sta_adjoint_noalloc launch: ") + hipGetErrorString(e);
        return STA_EHIP;
    }
    return STA_OK;
}
