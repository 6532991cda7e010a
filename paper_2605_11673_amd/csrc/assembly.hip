// gfx950 kernels for exact assembly of A_t = M_t + dt^2 K_t (paper Sec. 3.4
// eq. (8), implicit-Euler matrix of Sec. 6.2 eq. (9)).
//
// Data flow.  Each candidate tet's element matrix is split into its 10 node
// blocks (4 diagonal, 6 off-diagonal) and stored at the tet's position in
// each block's incidence segment: the persistent per-element contributions
// the paper's streaming policy keeps across frames (Sec. 3.5).  An inactive
// tet's slots hold +0.0.  A matrix entry is the sum of its segment's terms,
// taken in ascending tet id from +0.0.  The full rebuild recomputes every
// tet's slots (zero for inactive ones) and re-sums every block; the
// streaming update rewrites the slots of tets whose state changed and
// re-sums only the blocks they cover.  Both use the same summation routine,
// so they agree bit for bit with each other and with a rebuild that skips
// inactive tets (an accumulator that starts at +0.0 never becomes -0.0, so
// adding +0.0 changes nothing).
//
// Floating point: contraction is off for this file and the element formula
// is evaluated in a fixed order (see include/stafem.h); only IEEE + - * / and
// |.| are used.
#include <hip/hip_runtime.h>

#include "sta_internal.h"

#pragma clang fp contract(off)

namespace sta {

namespace {

constexpr int kBlock = 256;
constexpr int kXcds = 8;
constexpr int kLanesPerEdit = 78;  // phase 2: 4 diagonal blocks x 6 values + 6 off-diagonal blocks x 9 values
constexpr int kEditLanes = 16;     // phase 1: one lane per block slot (10 used), power of two

// Workgroups are dispatched round-robin over the 8 XCDs.  Remap so that each
// XCD walks one contiguous range of the work: neighbouring blocks share
// contribution, descriptor and CSR cache lines, and each XCD has its own L2.
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

constexpr int PA[6] = {0, 0, 0, 1, 1, 2};
constexpr int PB[6] = {1, 2, 3, 2, 3, 3};

// Compute tet e's element matrix and store its 78 distinct values at the
// tet's 10 incidence positions.  Off-diagonal blocks are stored in block
// orientation (row node = smaller node id).  pos: the tet's 10 positions.
__device__ __forceinline__ void store_element(const DevView& v, int e, int4 t, const int* pos)
{
    Geo G;
    element_geometry(v, e, t, G);
    if (G.det == 0.0)
        atomicOr(&v.ctl->err, ERR_DEGENERATE);
    const int id[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const double s = dot3(G.g[a], G.g[a]);
        double2* dst = reinterpret_cast<double2*>(v.cd + 6 * (size_t)pos[a]);
        dst[0] = make_double2(entry(G.g[a], G.g[a], s, G, 0, 0, true), entry(G.g[a], G.g[a], s, G, 0, 1, true));
        dst[1] = make_double2(entry(G.g[a], G.g[a], s, G, 0, 2, true), entry(G.g[a], G.g[a], s, G, 1, 1, true));
        dst[2] = make_double2(entry(G.g[a], G.g[a], s, G, 1, 2, true), entry(G.g[a], G.g[a], s, G, 2, 2, true));
    }
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

// Zero the 78 slots of an inactive tet.
__device__ __forceinline__ void zero_element(const DevView& v, const int* pos)
{
    const double2 z = make_double2(0.0, 0.0);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        double2* dst = reinterpret_cast<double2*>(v.cd + 6 * (size_t)pos[a]);
        dst[0] = z;
        dst[1] = z;
        dst[2] = z;
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        double* dst = v.co + 9 * (size_t)pos[4 + q];
#pragma unroll
        for (int j = 0; j < 9; ++j)
            dst[j] = 0.0;
    }
}

// The canonical sum of value vi of one block: +0.0 plus the segment's terms
// in ascending tet id.  Loads are issued CH at a time so that a whole
// segment (up to CH terms) is in flight at once; padding terms are +0.0.
template <int CH>
__device__ __forceinline__ double seg_sum(const double* __restrict__ c, int stride, int vi, int k0, int k1)
{
    double acc = 0.0;
    for (int base = k0; base < k1; base += CH) {
        double t[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j)
            t[j] = (base + j < k1) ? c[(size_t)(base + j) * stride + vi] : 0.0;
#pragma unroll
        for (int j = 0; j < CH; ++j)
            acc = acc + t[j];
    }
    return acc;
}

__device__ __constant__ int kDiagP[6] = {0, 0, 0, 1, 1, 2};
__device__ __constant__ int kDiagQ[6] = {0, 1, 2, 1, 2, 2};

// Recompute value vi (0..5 unique diagonal values, 0..8 off-diagonal) of the
// block described by d and write it (and its mirror) into the CSR values.
__device__ __forceinline__ void block_value(const DevView& v, const BlockDesc& d, int vi)
{
    if (d.kind == 0) {
        const double acc = seg_sum<32>(v.cd, 6, vi, d.k0, d.k1);
        const int p = kDiagP[vi], q = kDiagQ[vi];
        v.values[d.up + p * d.rl + q] = acc;
        if (p != q)
            v.values[d.up + q * d.rl + p] = acc;
    } else {
        const double acc = seg_sum<8>(v.co, 9, vi, d.k0, d.k1);
        const int p = vi / 3, q = vi - 3 * (vi / 3);
        v.values[d.up + p * d.rl + q] = acc;
        v.values[d.lo + q * d.rlj + p] = acc;
    }
}

__device__ __forceinline__ BlockDesc load_desc(const BlockDesc* p)
{
    const int4* q = reinterpret_cast<const int4*>(p);
    const int4 a = q[0], b = q[1];
    BlockDesc d;
    d.k0 = a.x;
    d.k1 = a.y;
    d.up = a.z;
    d.rl = a.w;
    d.lo = b.x;
    d.rlj = b.y;
    d.kind = b.z;
    d.block = b.w;
    return d;
}

__device__ __forceinline__ void store_desc(BlockDesc* p, const BlockDesc& d)
{
    int4* q = reinterpret_cast<int4*>(p);
    q[0] = make_int4(d.k0, d.k1, d.up, d.rl);
    q[1] = make_int4(d.lo, d.rlj, d.kind, d.block);
}

// ---------------------------------------------------------------------------
// Full rebuild
// ---------------------------------------------------------------------------

// Every candidate: active -> element matrix into its slots, inactive -> zeros.
__global__ __launch_bounds__(kBlock) void k_element(DevView v)
{
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int e = wg * kBlock + threadIdx.x;
    if (e >= v.n_tets)
        return;
    int pos[10];
#pragma unroll
    for (int j = 0; j < 10; ++j)
        pos[j] = v.e2p[10 * (size_t)e + j];
    if (v.mask[e])
        store_element(v, e, v.T[e], pos);
    else
        zero_element(v, pos);
}

// Lanes: 6 per diagonal block, then 9 per off-diagonal block.
__global__ __launch_bounds__(kBlock) void k_reduce_all(DevView v)
{
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t t = (int64_t)wg * kBlock + threadIdx.x;
    const int64_t nd6 = (int64_t)v.nd * 6;
    int b, vi;
    if (t < nd6) {
        b = (int)(t / 6);
        vi = (int)(t - 6 * (int64_t)b);
    } else {
        const int64_t u = t - nd6;
        if (u >= (int64_t)v.no * 9)
            return;
        const int o = (int)(u / 9);
        vi = (int)(u - 9 * (int64_t)o);
        b = v.nd + o;
    }
    block_value(v, load_desc(v.desc + b), vi);
}

// ---------------------------------------------------------------------------
// Streaming update
// ---------------------------------------------------------------------------

// Write the values of local block (A, B) of tet e (block orientation: row
// vertex = the one with the smaller node id; same arithmetic as store_element).
template <int A, int B>
__device__ __forceinline__ void store_slot_ab(const DevView& v, const Geo& G, const int* id, int pos)
{
    if (A == B) {
        const double s = dot3(G.g[A], G.g[A]);
        double2* dst = reinterpret_cast<double2*>(v.cd + 6 * (size_t)pos);
        dst[0] = make_double2(entry(G.g[A], G.g[A], s, G, 0, 0, true), entry(G.g[A], G.g[A], s, G, 0, 1, true));
        dst[1] = make_double2(entry(G.g[A], G.g[A], s, G, 0, 2, true), entry(G.g[A], G.g[A], s, G, 1, 1, true));
        dst[2] = make_double2(entry(G.g[A], G.g[A], s, G, 1, 2, true), entry(G.g[A], G.g[A], s, G, 2, 2, true));
    } else {
        const bool sw = id[A] > id[B];
        double ga[3], gb[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            ga[i] = sw ? G.g[B][i] : G.g[A][i];
            gb[i] = sw ? G.g[A][i] : G.g[B][i];
        }
        const double s = dot3(ga, gb);
        double* dst = v.co + 9 * (size_t)pos;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                dst[3 * i + j] = entry(ga, gb, s, G, i, j, false);
    }
}

// Write block slot r (0..3 diagonal a=r, 4..9 pairs 01 02 03 12 13 23) of tet
// e: its element-matrix values or, for an inactive tet, zeros.
__device__ __forceinline__ void store_slot(const DevView& v, int e, int4 t, int r, int pos, bool active)
{
    if (!active) {
        if (r < 4) {
            double2* dst = reinterpret_cast<double2*>(v.cd + 6 * (size_t)pos);
            const double2 z = make_double2(0.0, 0.0);
            dst[0] = z;
            dst[1] = z;
            dst[2] = z;
        } else {
            double* dst = v.co + 9 * (size_t)pos;
#pragma unroll
            for (int j = 0; j < 9; ++j)
                dst[j] = 0.0;
        }
        return;
    }
    Geo G;
    element_geometry(v, e, t, G);
    if (G.det == 0.0 && r == 0)
        atomicOr(&v.ctl->err, ERR_DEGENERATE);
    const int id[4] = {t.x, t.y, t.z, t.w};
    switch (r) {
    case 0: store_slot_ab<0, 0>(v, G, id, pos); break;
    case 1: store_slot_ab<1, 1>(v, G, id, pos); break;
    case 2: store_slot_ab<2, 2>(v, G, id, pos); break;
    case 3: store_slot_ab<3, 3>(v, G, id, pos); break;
    case 4: store_slot_ab<0, 1>(v, G, id, pos); break;
    case 5: store_slot_ab<0, 2>(v, G, id, pos); break;
    case 6: store_slot_ab<0, 3>(v, G, id, pos); break;
    case 7: store_slot_ab<1, 2>(v, G, id, pos); break;
    case 8: store_slot_ab<1, 3>(v, G, id, pos); break;
    default: store_slot_ab<2, 3>(v, G, id, pos); break;
    }
}

__device__ __forceinline__ BlockDesc empty_desc()
{
    return BlockDesc{0, 0, 0, 0, 0, 0, -1, -1};
}

// Edit count of this frame: *n_dev if given and within [0, n_host], else n_host.
__device__ __forceinline__ int frame_count(int32_t n_host, const int32_t* n_dev, bool& bad)
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

// Phase 1, 16 lanes per edit (lane r < 10 owns block slot r).  Validate the
// edit; lane 0 takes the tet's stamp (a second edit of the same tet in this
// frame finds it taken: duplicate) and reads its mask bit.  If the state
// changes, each slot lane claims its block (first claimant wins; the claim
// record carries the block descriptor), the owner flips the mask bit and the
// slot lanes rewrite the tet's 78 contribution slots (element matrix on
// activation, zeros on deactivation).  Each workgroup writes its error bits
// to its own byte, so no global word needs resetting between frames.
__global__ __launch_bounds__(kBlock) void k_edits(DevView v, const int32_t* __restrict__ ids,
                                                  const uint8_t* __restrict__ states, int32_t n_host,
                                                  const int32_t* __restrict__ n_dev)
{
    __shared__ int s_bits;
    if (threadIdx.x == 0)
        s_bits = 0;
    __syncthreads();
    bool bad_n;
    const int n = frame_count(n_host, n_dev, bad_n);
    const int gt = blockIdx.x * kBlock + threadIdx.x;
    const int i = gt / kEditLanes;
    const int r = gt - i * kEditLanes;
    int bits = (bad_n && gt == 0) ? ERR_RANGE : 0;
    if (i < n) {
        BlockDesc* rec = v.rec + 10 * (size_t)i;
        const int id = ids[i];
        const unsigned st = states[i];
        if (id < 0 || id >= v.n_tets || st > 1u) {
            if (r == 0) {
                bits |= ERR_RANGE;
                v.undo[i] = 0xFF;
            }
            if (r < 10)
                store_desc(rec + r, empty_desc());
        } else {
            int eb = 0, ep = 0;
            if (r < 10) {
                eb = v.e2b[10 * (size_t)id + r];
                ep = v.e2p[10 * (size_t)id + r];
            }
            const uint8_t prev = v.mask[id];
            int owner = 1;
            if (r == 0)
                owner = atomicExch(&v.estamp[id], 1u) == 0u ? 1 : 0;
            const int lane = threadIdx.x & 63;
            owner = __shfl(owner, lane & ~(kEditLanes - 1), 64);
            const bool change = prev != st;
            if (r < 10) {
                BlockDesc d = empty_desc();
                if (change) {
                    const BlockDesc bd = load_desc(v.desc + eb);
                    if (atomicExch(&v.bstamp[eb], 1u) == 0u)
                        d = bd;
                }
                store_desc(rec + r, d);
            }
            if (!owner) {
                if (r == 0)
                    bits |= ERR_DUP;
            } else if (change) {
                if (r == 0)
                    v.mask[id] = (uint8_t)st;
                if (r < 10)
                    store_slot(v, id, v.T[id], r, ep, st != 0u);
            }
            if (r == 0)
                v.undo[i] = (owner && change) ? prev : (uint8_t)0xFF;
        }
    }
    if (bits)
        atomicOr(&s_bits, bits);
    __syncthreads();
    if (threadIdx.x == 0)
        v.wg_err[blockIdx.x] = (uint8_t)s_bits;
}

// Phase 2: 78 lanes per edit (4 diagonal blocks x 6 values, 6 off-diagonal
// blocks x 9 values).  Every workgroup first ORs the edit workgroups' error
// bytes.  Without an error a lane re-sums its value if the edit claimed the
// block; with one, lane 0 of each edit undoes its mask flip and slot rewrite.
// Either way the frame's stamps are cleared for the next frame.
__global__ __launch_bounds__(kBlock) void k_touched(DevView v, const int32_t* __restrict__ ids, int32_t n_host,
                                                    const int32_t* __restrict__ n_dev)
{
    __shared__ int s_bits;
    if (threadIdx.x == 0)
        s_bits = 0;
    __syncthreads();
    bool bad_n;
    const int n = frame_count(n_host, n_dev, bad_n);
    const int g_edits = n > 0 ? (n * kEditLanes + kBlock - 1) / kBlock : 1;
    int bits = 0;
    for (int w = threadIdx.x; w < g_edits; w += kBlock)
        bits |= v.wg_err[w];
    if (bits)
        atomicOr(&s_bits, bits);
    __syncthreads();
    const int fe = s_bits;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        v.ctl->frame_err = fe;
        v.ctl->last_n = n;
        if (fe)
            atomicOr(&v.ctl->err, fe);
    }
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int i = (int)(t / kLanesPerEdit);
    const int r = (int)(t - (int64_t)i * kLanesPerEdit);
    if (i >= n)
        return;
    int j, vi;
    if (r < 24) {
        j = r / 6;
        vi = r - 6 * j;
    } else {
        j = 4 + (r - 24) / 9;
        vi = (r - 24) - 9 * (j - 4);
    }
    const BlockDesc d = load_desc(v.rec + 10 * (size_t)i + j);
    if (!fe && d.kind >= 0)
        block_value(v, d, vi);
    if (vi == 0 && d.kind >= 0)
        v.bstamp[d.block] = 0u;
    if (r == 0) {
        const int id = ids[i];
        if (id >= 0 && id < v.n_tets) {
            v.estamp[id] = 0u;
            const uint8_t u = v.undo[i];
            if (fe && u != 0xFF) {
                int ep[10];
#pragma unroll
                for (int q = 0; q < 10; ++q)
                    ep[q] = v.e2p[10 * (size_t)id + q];
                v.mask[id] = u;
                if (u)
                    store_element(v, id, v.T[id], ep);
                else
                    zero_element(v, ep);
            }
        }
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

hipError_t launch_element(const DevView& v, hipStream_t s)
{
    if (v.n_tets == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_element, dim3(blocks_for(v.n_tets)), dim3(kBlock), 0, s, v);
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

hipError_t launch_edit_phase(const DevView& v, const int32_t* ids, const uint8_t* states, int32_t n_host,
                             const int32_t* n_dev, hipStream_t s)
{
    // an empty list still runs one workgroup of each phase: they record the frame (count 0)
    hipLaunchKernelGGL(k_edits, dim3(n_host > 0 ? blocks_for((int64_t)n_host * kEditLanes) : 1u), dim3(kBlock), 0, s, v, ids, states, n_host, n_dev);
    return hipGetLastError();
}

hipError_t launch_touched_phase(const DevView& v, const int32_t* ids, int32_t n_host, const int32_t* n_dev,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_touched, dim3(n_host > 0 ? blocks_for((int64_t)n_host * kLanesPerEdit) : 1u), dim3(kBlock), 0, s, v, ids,
                       n_host, n_dev);
    return hipGetLastError();
}

hipError_t launch_set_params(const DevView& v, const double* x_aos, const double* E, double* xs, double* ys,
                             double* zs, double* Eout, hipStream_t s)
{
    const int64_t n = v.n_nodes > v.n_tets ? v.n_nodes : v.n_tets;
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_set_params, dim3(blocks_for(n)), dim3(kBlock), 0, s, v.n_nodes, v.n_tets, x_aos, E, xs,
                       ys, zs, Eout);
    return hipGetLastError();
}

}  // namespace sta
