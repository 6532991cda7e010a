// gfx950 kernels for exact assembly of A_t = M_t + dt^2 K_t (paper Sec. 3.4
// eq. (8), implicit-Euler matrix of Sec. 6.2 eq. (9)).
//
// Data flow.  Each candidate tet's element matrix is split into its 10 node
// blocks (4 diagonal, 6 off-diagonal) and stored at the tet's position in
// each block's incidence segment: the persistent per-element contributions
// the paper's streaming policy keeps across frames (Sec. 3.5).  A matrix
// entry is then the sum of its segment's terms whose tet is active, taken in
// ascending tet id from +0.0.  The full rebuild re-sums every block; the
// streaming update re-sums only blocks covered by tets whose state changed.
// Both call the same reduction routine, so they agree bit for bit.
//
// Floating point: contraction is off for this file and the element formula
// is evaluated in a fixed order (see include/stafem.h); only IEEE + - * / and
// |.| are used.  Skipping an inactive term equals adding +0.0 because an
// accumulator that starts at +0.0 can never become -0.0.
#include <hip/hip_runtime.h>

#include "sta_internal.h"

#pragma clang fp contract(off)

namespace sta {

namespace {

constexpr int kBlock = 256;
constexpr int kXcds = 8;

// Workgroups are dispatched round-robin over the 8 XCDs.  Remap so that each
// XCD walks one contiguous range of the work: neighbouring blocks share
// segment, mask and CSR cache lines, and each XCD has its own L2.
__device__ __forceinline__ int xcd_remap(int wg, int G)
{
    const int q = G / kXcds, r = G % kXcds;
    const int x = wg % kXcds, idx = wg / kXcds;
    const int base = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return base + idx;
}

struct Geo {
    double g[4][3];
    double lamV, muV, ml, det;
};

__device__ __forceinline__ void cross3(const double* a, const double* b, double* c)
{
    c[0] = (a[1] * b[2]) - (a[2] * b[1]);
    c[1] = (a[2] * b[0]) - (a[0] * b[2]);
    c[2] = (a[0] * b[1]) - (a[1] * b[0]);
}

// Basis gradients, scaled moduli and lumped mass of tet e, in the fixed order.
__device__ __forceinline__ void element_geometry(const DevView& v, int e, int4 t, Geo& G)
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
    cross3(d[2], d[3], c[1]);
    cross3(d[3], d[1], c[2]);
    cross3(d[1], d[2], c[3]);
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
    const double V = fabs(det) / 6.0;
    const double E = v.E[e];
    const double lam = E * v.mat.clam;
    const double mu = E * v.mat.cmu;
    G.lamV = (lam * V) * v.mat.cdt;
    G.muV = (mu * V) * v.mat.cdt;
    G.ml = (v.mat.rho * V) * 0.25;
    G.det = det;
}

__device__ __forceinline__ double dot3(const double* a, const double* b)
{
    return ((a[0] * b[0]) + (a[1] * b[1])) + (a[2] * b[2]);
}

// Entry (i, j) of the 3x3 block of row vertex a (gradient ga) and column
// vertex b (gradient gb); s = ga . gb; diag: a == b.
__device__ __forceinline__ double entry(const double* ga, const double* gb, double s, const Geo& G, int i, int j,
                                        bool diag)
{
    double v = (G.lamV * (ga[i] * gb[j])) + (G.muV * (ga[j] * gb[i]));
    if (i == j)
        v = v + (G.muV * s);
    if (diag && i == j)
        v = v + G.ml;
    return v;
}

__constant__ int kDiagP[6] = {0, 0, 0, 1, 1, 2};
__constant__ int kDiagQ[6] = {0, 1, 2, 1, 2, 2};

// Compute tet e's element matrix and store its 78 distinct values at the
// tet's positions in its 10 block segments.  Off-diagonal blocks are stored
// in block orientation (row node = smaller node id).
__device__ __forceinline__ void store_element(const DevView& v, int e, int4 t, const Geo& G)
{
    const int id[4] = {t.x, t.y, t.z, t.w};
    const int* pos = v.e2p + 10 * (size_t)e;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const double s = dot3(G.g[a], G.g[a]);
        double2* dst = reinterpret_cast<double2*>(v.cd + 6 * (size_t)pos[a]);
        dst[0] = make_double2(entry(G.g[a], G.g[a], s, G, 0, 0, true), entry(G.g[a], G.g[a], s, G, 0, 1, true));
        dst[1] = make_double2(entry(G.g[a], G.g[a], s, G, 0, 2, true), entry(G.g[a], G.g[a], s, G, 1, 1, true));
        dst[2] = make_double2(entry(G.g[a], G.g[a], s, G, 1, 2, true), entry(G.g[a], G.g[a], s, G, 2, 2, true));
    }
    constexpr int PA[6] = {0, 0, 0, 1, 1, 2};
    constexpr int PB[6] = {1, 2, 3, 2, 3, 3};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const bool sw = id[PA[q]] > id[PB[q]];
        double ga[3], gb[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            ga[i] = sw ? G.g[PB[q]][i] : G.g[PA[q]][i];
            gb[i] = sw ? G.g[PA[q]][i] : G.g[PB[q]][i];
        }
        const double s = dot3(ga, gb);
        double* dst = v.co + 9 * (size_t)pos[4 + q];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                dst[3 * i + j] = entry(ga, gb, s, G, i, j, false);
    }
}

// The canonical sum of one value of one block: +0.0 plus the active terms in
// segment (ascending tet id) order.
__device__ __forceinline__ double reduce_terms(const int32_t* __restrict__ inc, const double* __restrict__ c,
                                               int stride, int v, int k0, int k1,
                                               const uint8_t* __restrict__ mask)
{
    double acc = 0.0;
    for (int k = k0; k < k1; ++k) {
        const int e = inc[k];
        const double t = c[(size_t)k * stride + v];
        if (mask[e])
            acc = acc + t;
    }
    return acc;
}

__device__ __forceinline__ void reduce_diag_value(const DevView& v, int b, int vi)
{
    const int k0 = v.dseg[b], k1 = v.dseg[b + 1];
    const int2 meta = v.dmeta[b];
    const double acc = reduce_terms(v.dinc, v.cd, 6, vi, k0, k1, v.mask);
    const int p = kDiagP[vi], q = kDiagQ[vi];
    v.values[meta.x + p * meta.y + q] = acc;
    if (p != q)
        v.values[meta.x + q * meta.y + p] = acc;
}

__device__ __forceinline__ void reduce_off_value(const DevView& v, int b, int vi)
{
    const int k0 = v.oseg[b], k1 = v.oseg[b + 1];
    const int4 meta = v.ometa[b];
    const double acc = reduce_terms(v.oinc, v.co, 9, vi, k0, k1, v.mask);
    const int p = vi / 3, q = vi - 3 * (vi / 3);
    v.values[meta.x + p * meta.y + q] = acc;
    v.values[meta.z + q * meta.w + p] = acc;
}

// ---------------------------------------------------------------------------
// Full rebuild
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_element(DevView v, int all_tets, uint32_t ver)
{
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int e = wg * kBlock + threadIdx.x;
    if (e >= v.n_tets)
        return;
    if (!all_tets && !v.mask[e])
        return;
    const int4 t = v.T[e];
    Geo G;
    element_geometry(v, e, t, G);
    if (G.det == 0.0)
        atomicOr(&v.ctl->err, ERR_DEGENERATE);
    store_element(v, e, t, G);
    v.cver[e] = ver;
}

__global__ __launch_bounds__(kBlock) void k_reduce_all(DevView v)
{
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t t = (int64_t)wg * kBlock + threadIdx.x;
    const int64_t nd6 = (int64_t)v.nd * 6;
    if (t < nd6) {
        reduce_diag_value(v, (int)(t / 6), (int)(t % 6));
    } else {
        const int64_t u = t - nd6;
        if (u < (int64_t)v.no * 9)
            reduce_off_value(v, (int)(u / 9), (int)(u % 9));
    }
}

// ---------------------------------------------------------------------------
// Streaming update
// ---------------------------------------------------------------------------

// Phase 1, one thread per edit: validate, de-duplicate the tet, flip its mask
// bit, refresh its contributions if they predate the current parameters,
// and claim each of its 10 blocks for this frame (the first claimant of a
// block records it; later ones see the frame's stamp).  The last workgroup
// to finish publishes the frame's error bits and advances the epoch.
__global__ __launch_bounds__(kBlock) void k_edits(DevView v, const int32_t* __restrict__ ids,
                                                  const uint8_t* __restrict__ states, int32_t n_host,
                                                  const int32_t* __restrict__ n_dev, uint32_t ver)
{
    const uint32_t epoch = v.ctl->epoch + 1u;
    const int n = n_dev ? *n_dev : n_host;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        int32_t* cl = v.claims + 10 * (size_t)i;
        int32_t mine[10];
#pragma unroll
        for (int j = 0; j < 10; ++j)
            mine[j] = -1;
        uint8_t undo = 0xFF;
        const int id = ids[i];
        const unsigned st = states[i];
        if (id < 0 || id >= v.n_tets || st > 1u) {
            atomicOr(&v.ctl->ferr, ERR_RANGE);
        } else if (atomicExch(&v.estamp[id], epoch) == epoch) {
            atomicOr(&v.ctl->ferr, ERR_DUP);
        } else {
            const uint8_t prev = v.mask[id];
            if (prev != st) {
                v.mask[id] = (uint8_t)st;
                undo = prev;
                if (st && v.cver[id] != ver) {
                    const int4 t = v.T[id];
                    Geo G;
                    element_geometry(v, id, t, G);
                    store_element(v, id, t, G);
                    v.cver[id] = ver;
                }
                const int32_t* eb = v.e2b + 10 * (size_t)id;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int b = eb[j];
                    if (atomicExch(&v.dstamp[b], epoch) != epoch)
                        mine[j] = b;
                }
#pragma unroll
                for (int j = 4; j < 10; ++j) {
                    const int b = eb[j];
                    if (atomicExch(&v.ostamp[b], epoch) != epoch)
                        mine[j] = b;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 10; ++j)
            cl[j] = mine[j];
        v.undo[i] = undo;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned arrived = atomicAdd(&v.ctl->done, 1u);
        if (arrived == gridDim.x - 1) {
            __threadfence();
            const int fe = atomicOr(&v.ctl->ferr, 0);
            v.ctl->frame_err = fe;
            atomicOr(&v.ctl->err, fe);
            atomicExch(&v.ctl->ferr, 0);
            atomicExch(&v.ctl->done, 0u);
            atomicExch(&v.ctl->epoch, epoch);
            __threadfence();
        }
    }
}

// Phase 2: 78 lanes per edit (4 diagonal blocks x 6 values, 6 off-diagonal
// blocks x 9 values); a lane recomputes its value if the edit claimed the
// block.  If the frame had an error, lane 0 of each edit restores the mask
// instead and nothing else changes.
__global__ __launch_bounds__(kBlock) void k_touched(DevView v, const int32_t* __restrict__ ids, int32_t n_host,
                                                    const int32_t* __restrict__ n_dev)
{
    const int n = n_dev ? *n_dev : n_host;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int i = (int)(t / 78);
    const int r = (int)(t - (int64_t)i * 78);
    if (i >= n)
        return;
    if (v.ctl->frame_err) {
        if (r == 0 && v.undo[i] != 0xFF)
            v.mask[ids[i]] = v.undo[i];
        return;
    }
    if (r < 24) {
        const int b = v.claims[10 * (size_t)i + r / 6];
        if (b >= 0)
            reduce_diag_value(v, b, r % 6);
    } else {
        const int rr = r - 24;
        const int b = v.claims[10 * (size_t)i + 4 + rr / 9];
        if (b >= 0)
            reduce_off_value(v, b, rr % 9);
    }
}

__global__ __launch_bounds__(kBlock) void k_set_params(int n_nodes, int n_tets, const double* __restrict__ x_aos,
                                                       const double* __restrict__ Ein, double* xs, double* ys,
                                                       double* zs, double* Eout)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (x_aos && i < n_nodes) {
        xs[i] = x_aos[3 * (size_t)i + 0];
        ys[i] = x_aos[3 * (size_t)i + 1];
        zs[i] = x_aos[3 * (size_t)i + 2];
    }
    if (Ein && i < n_tets)
        Eout[i] = Ein[i];
}

inline unsigned blocks_for(int64_t threads)
{
    return (unsigned)((threads + kBlock - 1) / kBlock);
}

}  // namespace

hipError_t launch_element(const DevView& v, bool all_tets, uint32_t ver, hipStream_t s)
{
    if (v.n_tets == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_element, dim3(blocks_for(v.n_tets)), dim3(kBlock), 0, s, v, all_tets ? 1 : 0, ver);
    return hipGetLastError();
}

hipError_t launch_reduce_all(const DevView& v, hipStream_t s)
{
    const int64_t threads = (int64_t)v.nd * 6 + (int64_t)v.no * 9;
    if (threads == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_reduce_all, dim3(blocks_for(threads)), dim3(kBlock), 0, s, v);
    return hipGetLastError();
}

hipError_t launch_edits(const DevView& v, const int32_t* ids, const uint8_t* states, int32_t n, uint32_t ver,
                        hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_edits, dim3(blocks_for(n)), dim3(kBlock), 0, s, v, ids, states, n,
                       (const int32_t*)nullptr, ver);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess)
        return err;
    hipLaunchKernelGGL(k_touched, dim3(blocks_for((int64_t)n * 78)), dim3(kBlock), 0, s, v, ids, n,
                       (const int32_t*)nullptr);
    return hipGetLastError();
}

hipError_t launch_set_params(const DevView& v, const double* x_aos, const double* E, double* xs, double* ys,
                             double* zs, double* Eout, hipStream_t s)
{
    const int64_t n = v.n_nodes > v.n_tets ? v.n_nodes : v.n_tets;
    hipLaunchKernelGGL(k_set_params, dim3(blocks_for(n)), dim3(kBlock), 0, s, v.n_nodes, v.n_tets, x_aos, E, xs,
                       ys, zs, Eout);
    return hipGetLastError();
}

}  // namespace sta
