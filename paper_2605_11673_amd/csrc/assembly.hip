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
constexpr int kEditLanes = 16;     // phase 1: one lane per block slot (10 used), power of two
// Claimed blocks are compacted per edit-phase wave (64 / kEditLanes = 4
// edits): at most 16 diagonal and 24 off-diagonal claims.
constexpr int kRegionDiag = 16, kRegionOff = 24, kRegion = kRegionDiag + kRegionOff;
constexpr int kRegionsPerBlock = kBlock / 64;

typedef double dvec2 __attribute__((ext_vector_type(2)));

// Loads and stores with an optional non-temporal (streaming) cache hint, for
// data touched exactly once per launch (the rebuild's contributions and values).
template <bool NT>
__device__ __forceinline__ double ld(const double* p)
{
    if (NT)
        return __builtin_nontemporal_load(p);
    return *p;
}
template <bool NT>
__device__ __forceinline__ void st(double* p, double x)
{
    if (NT)
        __builtin_nontemporal_store(x, p);
    else
        *p = x;
}
template <bool NT>
__device__ __forceinline__ void st2(double* p, double a, double b)
{
    const dvec2 x = {a, b};
    if (NT)
        __builtin_nontemporal_store(x, reinterpret_cast<dvec2*>(p));
    else
        *reinterpret_cast<dvec2*>(p) = x;
}

// The rebuild kernels remap workgroup ids so that neighbouring work, which
// shares contribution, descriptor and CSR cache lines, runs on one XCD: the
// element kernel gives each XCD one contiguous eighth of the tets (xcd_remap).
//
// Reduce: each XCD takes runs of kXcdRun consecutive workgroups in turn, so
// that the runs spread every part of the work (the diagonal blocks, then the
// off-diagonal ones) evenly over the XCDs.  One contiguous range per XCD put
// the whole diagonal section on three XCDs and was 4% slower; plain
// round-robin was 1% slower.  Workgroups past the last whole round of runs
// keep their ids, so the map is a permutation of [0, G).
constexpr int kXcdRun = 16;
__device__ __forceinline__ int xcd_remap_runs(int wg, int G)
{
    const int full = G / (kXcds * kXcdRun) * (kXcds * kXcdRun);
    if (wg >= full)
        return wg;
    const int x = wg % kXcds, idx = wg / kXcds;
    return ((idx / kXcdRun) * kXcds + x) * kXcdRun + idx % kXcdRun;
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

// Basis gradients, scaled moduli and lumped mass of a tet from its vertex
// coordinates X and Young's modulus E, in the fixed order.
__device__ __forceinline__ void geometry_from(const DevView& v, const double (&X)[4][3], double E, Geo& G)
{
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
    const double lam = E * v.mat.clam;
    const double mu = E * v.mat.cmu;
    G.lamV = (lam * V) * v.mat.cdt;
    G.muV = (mu * V) * v.mat.cdt;
    G.ml = (v.mat.rho * V) * 0.25;
    G.det = det;
}

__device__ __forceinline__ void load_vertices(const DevView& v, int4 t, double (&X)[4][3])
{
    const int id[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        X[a][0] = v.xs[id[a]];
        X[a][1] = v.ys[id[a]];
        X[a][2] = v.zs[id[a]];
    }
}

__device__ __forceinline__ void element_geometry(const DevView& v, int e, int4 t, Geo& G)
{
    double X[4][3];
    load_vertices(v, t, X);
    geometry_from(v, X, v.E[e], G);
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
template <bool NT = false>
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
        double* dst = v.cd + 6 * (size_t)pos[a];
        st2<NT>(dst + 0, entry(G.g[a], G.g[a], s, G, 0, 0, true), entry(G.g[a], G.g[a], s, G, 0, 1, true));
        st2<NT>(dst + 2, entry(G.g[a], G.g[a], s, G, 0, 2, true), entry(G.g[a], G.g[a], s, G, 1, 1, true));
        st2<NT>(dst + 4, entry(G.g[a], G.g[a], s, G, 1, 2, true), entry(G.g[a], G.g[a], s, G, 2, 2, true));
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
                st<NT>(dst + 3 * i + j, entry(ga, gb, s, G, i, j, false));
    }
}

// Zero the 78 slots of an inactive tet.
template <bool NT = false>
__device__ __forceinline__ void zero_element(const DevView& v, const int* pos)
{
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        double* dst = v.cd + 6 * (size_t)pos[a];
        st2<NT>(dst + 0, 0.0, 0.0);
        st2<NT>(dst + 2, 0.0, 0.0);
        st2<NT>(dst + 4, 0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        double* dst = v.co + 9 * (size_t)pos[4 + q];
#pragma unroll
        for (int j = 0; j < 9; ++j)
            st<NT>(dst + j, 0.0);
    }
}

// The canonical sum of value vi of one block: +0.0 plus the segment's terms
// in ascending tet id.  Q lanes share one value ("slot mapping": Q = 1
// thread-, 4 quad-, 16 wave-sixteenth-per-slot): lane q of the group loads
// terms q, q+Q, q+2Q, ... CH at a time (padding terms are +0.0), then every
// lane of the group adds all terms in ascending order, taking each from the
// lane that holds it.  The additions are the same whatever Q is, so the
// result is bit-identical across mappings.  src0: wave lane of the group's
// lane 0; groups of Q lanes never straddle a wave.
//
// Padding terms past the segment end load the segment's last term (always
// in range, and on a line the group loads anyway) and are then replaced by
// +0.0: the CH loads issue back to back with no branch around each, where a
// guarded load per term cost an exec-mask branch apiece.
template <int Q, int CH, bool NT = false>
__device__ __forceinline__ double seg_sum(const double* __restrict__ c, int stride, int vi, int k0, int k1, int q,
                                          int src0)
{
    double acc = 0.0;
    for (int base = k0; base < k1; base += Q * CH) {
        double t[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int k = base + q + j * Q;
            const int kc = k < k1 ? k : k1 - 1;  // base < k1, so kc is in [k0, k1)
            t[j] = ld<NT>(c + (size_t)kc * stride + vi);
        }
#pragma unroll
        for (int j = 0; j < CH; ++j)
            t[j] = base + q + j * Q < k1 ? t[j] : 0.0;
        if (Q == 1) {
#pragma unroll
            for (int j = 0; j < CH; ++j)
                acc = acc + t[j];
        } else {
#pragma unroll
            for (int j = 0; j < CH; ++j)
#pragma unroll
                for (int l = 0; l < Q; ++l)
                    acc = acc + __shfl(t[j], src0 + l, 64);
        }
    }
    return acc;
}

// Terms held per lane per chunk: about 32 loads in flight per diagonal value
// (64 with sixteen lanes, so that the long segments of refinement supersets,
// 48 tets, are read in one round).
template <int Q>
struct DiagChunk {
    static constexpr int CH = Q == 1 ? 32 : (Q == 4 ? 8 : 4);
};
template <int Q>
struct OffChunk {
    static constexpr int CH = Q == 1 ? 8 : 2;
};

__device__ __constant__ int kDiagP[6] = {0, 0, 0, 1, 1, 2};
__device__ __constant__ int kDiagQ[6] = {0, 1, 2, 1, 2, 2};

// Recompute value vi (0..5 unique diagonal values, 0..8 off-diagonal) of the
// block described by d and write it (and its mirror) into the CSR values.
// All QD (or QO) lanes of the group call this; lane q == 0 writes.
template <int QD, int QO, bool NT = false>
__device__ __forceinline__ void block_value(const DevView& v, const BlockDesc& d, int vi, int q, int src0)
{
    if (d.kind == 0) {
        const double acc = seg_sum<QD, DiagChunk<QD>::CH, NT>(v.cd, 6, vi, d.k0, d.k1, q, src0);
        if (q == 0) {
            const int p = kDiagP[vi], r = kDiagQ[vi];
            st<NT>(v.values + d.up + p * d.rl + r, acc);
            if (p != r)
                st<NT>(v.values + d.up + r * d.rl + p, acc);
        }
    } else {
        const double acc = seg_sum<QO, OffChunk<QO>::CH, NT>(v.co, 9, vi, d.k0, d.k1, q, src0);
        if (q == 0) {
            const int p = vi / 3, r = vi - 3 * (vi / 3);
            st<NT>(v.values + d.up + p * d.rl + r, acc);
            st<NT>(v.values + d.lo + r * d.rlj + p, acc);
        }
    }
}

// block_value with the lane group size Q of the block's incidence-length
// bucket (Q <= the allocation QD / QO; a power of four, so that groups
// aligned to Q never straddle a wave).  MIXED = false: every bucket uses the
// allocation, and only that code path is compiled (the smaller mappings'
// deeper load chunks would otherwise cost registers and occupancy).
template <int QD, int QO, bool MIXED, bool NT = false>
__device__ __forceinline__ void block_value_q(const DevView& v, const BlockDesc& d, int vi, int q, int src0, int Q)
{
    if (!MIXED) {
        block_value<QD, QO, NT>(v, d, vi, q, src0);
    } else if (d.kind == 0) {
        if (QD >= 16 && Q == 16)
            block_value<16, 1, NT>(v, d, vi, q, src0);
        else if (QD >= 4 && Q == 4)
            block_value<4, 1, NT>(v, d, vi, q, src0);
        else
            block_value<1, 1, NT>(v, d, vi, q, src0);
    } else {
        if (QO >= 4 && Q == 4)
            block_value<1, 4, NT>(v, d, vi, q, src0);
        else
            block_value<1, 1, NT>(v, d, vi, q, src0);
    }
}

// Lane group size of block d under mapping m (its incidence-length bucket's).
template <int QD, int QO, bool MIXED>
__device__ __forceinline__ int bucket_q(const MapConfig& m, const BlockDesc& d)
{
    if (!MIXED)
        return d.kind == 0 ? QD : QO;
    const int kappa = d.k1 - d.k0;
    return d.kind == 0 ? m.qdb[diag_bucket(kappa)] : m.qob[off_bucket(kappa)];
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
// One lane per tet.  A tet's ten slot chunks lie far apart (each in its
// block's incidence segment), so lanes storing their own chunks would send
// one partial-line request per lane and store.  Instead each wave stages one
// slot of its 64 tets at a time in LDS and stores it cooperatively:
// neighbouring lanes write neighbouring parts of the same chunk, and the
// memory pipeline merges them into a few line requests.
template <bool NT>
__global__ __launch_bounds__(kBlock) void k_element(DevView v)
{
    __shared__ double s_stage[kBlock / 64][64 * 9];
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int base = wg * kBlock + (threadIdx.x & ~63);  // the wave's first tet
    if (base >= v.n_tets)
        return;
    const int lane = threadIdx.x & 63;
    const int e = base + lane;
    const int nw = v.n_tets - base < 64 ? v.n_tets - base : 64;  // tets of this wave
    const bool valid = lane < nw;
    int pos[10];
#pragma unroll
    for (int j = 0; j < 10; ++j)
        pos[j] = valid ? v.e2p[10 * (size_t)e + j] : 0;
    const bool active = valid && v.mask[e];
    Geo G;
    int4 t = make_int4(0, 1, 2, 3);
    if (active) {
        t = v.T[e];
        element_geometry(v, e, t, G);
        if (G.det == 0.0)
            atomicOr(&v.ctl->err, ERR_DEGENERATE);
    }
    double* buf = s_stage[threadIdx.x >> 6];
    // LDS accesses of one wave complete in issue order; the wavefront-scope
    // fences only keep the compiler from moving them across the exchange
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        if (active) {
            const double s = dot3(G.g[a], G.g[a]);
            buf[6 * lane + 0] = entry(G.g[a], G.g[a], s, G, 0, 0, true);
            buf[6 * lane + 1] = entry(G.g[a], G.g[a], s, G, 0, 1, true);
            buf[6 * lane + 2] = entry(G.g[a], G.g[a], s, G, 0, 2, true);
            buf[6 * lane + 3] = entry(G.g[a], G.g[a], s, G, 1, 1, true);
            buf[6 * lane + 4] = entry(G.g[a], G.g[a], s, G, 1, 2, true);
            buf[6 * lane + 5] = entry(G.g[a], G.g[a], s, G, 2, 2, true);
        } else {
#pragma unroll
            for (int k = 0; k < 6; ++k)
                buf[6 * lane + k] = 0.0;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // 64 chunks of 48 B = 192 pieces of 16 B, three per lane
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int p = lane + 64 * j, m = p / 3, k = p - 3 * m;
            const int pm = __shfl(pos[a], m, 64);
            if (m < nw)
                st2<NT>(v.cd + 6 * (size_t)pm + 2 * k, buf[6 * m + 2 * k], buf[6 * m + 2 * k + 1]);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    const int id[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        if (active) {
            const bool sw = id[PA[q]] > id[PB[q]];
            double ga[3], gb[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                ga[i] = sw ? G.g[PB[q]][i] : G.g[PA[q]][i];
                gb[i] = sw ? G.g[PA[q]][i] : G.g[PB[q]][i];
            }
            const double s = dot3(ga, gb);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    buf[9 * lane + 3 * i + j] = entry(ga, gb, s, G, i, j, false);
        } else {
#pragma unroll
            for (int k = 0; k < 9; ++k)
                buf[9 * lane + k] = 0.0;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // 64 chunks of 72 B (8-byte aligned) = 576 doubles, nine per lane
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const int p = lane + 64 * j, m = p / 9, k = p - 9 * m;
            const int pm = __shfl(pos[4 + q], m, 64);
            if (m < nw)
                st<NT>(v.co + 9 * (size_t)pm + k, buf[9 * m + k]);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// Off-diagonal value vi of block d with one lane per value (QO = 1), the
// block's 9 lanes in one wave from wave lane b0.  The mirror is written
// transposed through a shuffle (lane (p, r) writes mirror entry (p, r), the
// value of lane (r, p)), so that lanes 3p..3p+2 write one 24-byte row piece
// of the block and one of its mirror.
template <bool NT>
__device__ __forceinline__ void off_value_rows(const DevView& v, const BlockDesc& d, int vi, int b0)
{
    const double acc = seg_sum<1, OffChunk<1>::CH, NT>(v.co, 9, vi, d.k0, d.k1, 0, b0 + vi);
    const int p = vi / 3, r = vi - 3 * (vi / 3);
    const double tr = __shfl(acc, b0 + 3 * r + p, 64);
    st<NT>(v.values + d.up + p * d.rl + r, acc);
    st<NT>(v.values + d.lo + p * d.rlj + r, tr);
}

// Lanes: 6*QD per diagonal block (section padded to whole waves), then the
// off-diagonal blocks: for QO = 1, 7 blocks of 9 lanes per wave (lane 63
// idle, so that a block never straddles two waves), else 9*QO per block.
// Each block's lanes use its incidence-length bucket's group size Q (at most
// the allocation); lanes past 6Q (9Q) of a block idle.
template <int QD, int QO, bool MIXED, bool NT>
__global__ __launch_bounds__(kBlock) void k_reduce_all(DevView v, int64_t diag_lanes, MapConfig m)
{
    const int wg = xcd_remap_runs(blockIdx.x, gridDim.x);
    const int64_t t = (int64_t)wg * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    if (t < diag_lanes) {
        const int b = (int)(t / (6 * QD));
        if (b >= v.nd)
            return;
        const int rem = (int)(t - (int64_t)b * (6 * QD));
        const BlockDesc d = load_desc(v.desc + b);
        const int Q = bucket_q<QD, QO, MIXED>(m, d);
        if (rem >= 6 * Q)
            return;
        const int q = rem & (Q - 1);
        block_value_q<QD, QO, MIXED, NT>(v, d, rem / Q, q, lane - q, Q);
    } else {
        const int64_t u = t - diag_lanes;
        if (QO == 1) {
            const int l = (int)(u & 63);  // = lane: diag_lanes is a multiple of 64
            const int o1 = (int)(u >> 6) * 7 + l / 9;
            if (l == 63 || o1 >= v.no)
                return;
            off_value_rows<NT>(v, load_desc(v.desc + v.nd + o1), l % 9, lane - l % 9);
            return;
        }
        const int o = (int)(u / (9 * QO));
        if (o >= v.no)
            return;
        const int rem = (int)(u - (int64_t)o * (9 * QO));
        const BlockDesc d = load_desc(v.desc + v.nd + o);
        const int Q = bucket_q<QD, QO, MIXED>(m, d);
        if (rem >= 9 * Q)
            return;
        const int q = rem & (Q - 1);
        block_value_q<QD, QO, MIXED, NT>(v, d, rem / Q, q, lane - q, Q);
    }
}

// ---------------------------------------------------------------------------
// Streaming update
// ---------------------------------------------------------------------------

// Gradient of local vertex a (0..3, not a compile-time constant) by
// selects, so that no register array is indexed at run time.
__device__ __forceinline__ void pick_gradient(const Geo& G, int a, double* g)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
        g[i] = a == 0 ? G.g[0][i] : (a == 1 ? G.g[1][i] : (a == 2 ? G.g[2][i] : G.g[3][i]));
}

__device__ __forceinline__ int tet_vertex(int4 t, int a)
{
    return a == 0 ? t.x : (a == 1 ? t.y : (a == 2 ? t.z : t.w));
}

// Local vertices (A, B) of block slot r: r < 4 diagonal (r, r); 4..9 the
// pairs 01 02 03 12 13 23.  Two bits per slot, packed.
constexpr uint32_t kSlotA = 0u | 1u << 2 | 2u << 4 | 3u << 6 | 0u << 8 | 0u << 10 | 0u << 12 | 1u << 14 | 1u << 16 |
                            2u << 18;
constexpr uint32_t kSlotB = 0u | 1u << 2 | 2u << 4 | 3u << 6 | 1u << 8 | 2u << 10 | 3u << 12 | 2u << 14 | 3u << 16 |
                            3u << 18;

// Write block slot r of a tet with vertex ids t: its element-matrix values
// (geometry G; block orientation: row vertex = the one with the smaller node
// id; same arithmetic as store_element) when active, zeros when not.  One
// code path serves all ten slots (the slot only selects gradients), which
// keeps the streaming kernels' instruction footprint small.
__device__ __forceinline__ void store_slot(const DevView& v, int4 t, const Geo& G, int r, int pos, bool active)
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
    if (G.det == 0.0 && r == 0)
        atomicOr(&v.ctl->err, ERR_DEGENERATE);
    int A = (int)(kSlotA >> (2 * r)) & 3, B = (int)(kSlotB >> (2 * r)) & 3;
    if (tet_vertex(t, A) > tet_vertex(t, B)) {
        const int c = A;
        A = B;
        B = c;
    }
    double ga[3], gb[3];
    pick_gradient(G, A, ga);
    pick_gradient(G, B, gb);
    const double s = dot3(ga, gb);
    if (r < 4) {
        double2* dst = reinterpret_cast<double2*>(v.cd + 6 * (size_t)pos);
        dst[0] = make_double2(entry(ga, ga, s, G, 0, 0, true), entry(ga, ga, s, G, 0, 1, true));
        dst[1] = make_double2(entry(ga, ga, s, G, 0, 2, true), entry(ga, ga, s, G, 1, 1, true));
        dst[2] = make_double2(entry(ga, ga, s, G, 1, 2, true), entry(ga, ga, s, G, 2, 2, true));
    } else {
        double* dst = v.co + 9 * (size_t)pos;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                dst[3 * i + j] = entry(ga, gb, s, G, i, j, false);
    }
}

__device__ BlockDesc kNoClaim = {0, 0, 0, 0, 0, 0, -1, -1};
__device__ int32_t kNoTet = -1;

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

// Phase 1 for lane r of edit i = (tet id, requested state st); 16 lanes per
// edit, lane r < 10 owns block slot r.  Validate the edit; lane 0 takes the
// tet's stamp (a second edit of the same tet in this frame finds it taken:
// duplicate).  If the state changes, each slot lane claims its block (first
// claimant wins; the claim's kind and block descriptor are returned in ckind
// (-1: no claim) and cbd for the wave's compaction), the owner
// flips the mask bit and the slot lanes rewrite the tet's 78 contribution
// slots (element matrix on activation, zeros on deactivation).  Returns the
// lane's error bits.  All 16 lanes of the edit must call it together.
//
// The frame is a short chain of dependent memory round trips, so its time is
// their latency: every load that needs only the tet id (incidence positions,
// mask bit, vertex ids, modulus) and then the block descriptors and vertex
// coordinates are issued before the first atomic or store, which the compiler
// could not move them across.
__device__ __forceinline__ int edit_lane(const DevView& v, int id, unsigned st, int i, int r, int& ckind,
                                         BlockDesc& cbd)
{
    if (id < 0 || id >= v.n_tets || st > 1u) {
        if (r == 0) {
            v.undo[i] = 0xFF;
            return ERR_RANGE;
        }
        return 0;
    }
    const bool slot = r < 10;
    const TetRecord* rc = v.trec + id;
    // round trip 1: the tet's record (this lane's block descriptor and
    // incidence position; vertex ids and geometry for an activation), its
    // mask bit and its stamp
    BlockDesc bd = empty_desc();
    int ep = 0;
    if (slot) {
        bd = load_desc(rc->desc + r);
        ep = rc->pos[r];
    }
    int4 t = make_int4(0, 0, 0, 0);
    Geo G;
    if (slot && st) {
        t = rc->T;
        const dvec2* gp = reinterpret_cast<const dvec2*>(rc->g);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const dvec2 q = gp[k];
            G.g[(2 * k) / 3][(2 * k) % 3] = q.x;
            G.g[(2 * k + 1) / 3][(2 * k + 1) % 3] = q.y;
        }
        const dvec2 lm = *reinterpret_cast<const dvec2*>(&rc->lamV);
        G.lamV = lm.x;
        G.muV = lm.y;
        G.ml = rc->ml;
        G.det = rc->degenerate ? 0.0 : 1.0;  // store_slot only tests det == 0
    }
    const uint8_t prev = v.mask[id];
    unsigned taken = 0u;
    if (r == 0)
        taken = atomicExch(&v.estamp[id], 1u);
    // round trip 2: the block claim (its result is needed only for the claim
    // record, written last)
    const bool change = prev != st;
    unsigned claimed = 1u;
    if (slot && change)
        claimed = atomicExch(&v.bstamp[bd.block], 1u);
    // the atomics' results pass through cross-lane moves, which the compiler
    // keeps in place, so their waits fall here and after the slot stores
    const int owner = __shfl(taken, (threadIdx.x & 63) & ~(kEditLanes - 1), 64) == 0u;
    int bits = 0;
    if (!owner) {
        if (r == 0)
            bits = ERR_DUP;
    } else if (change) {
        if (r == 0)
            v.mask[id] = (uint8_t)st;
        if (slot)
            store_slot(v, t, G, r, ep, st != 0u);
    }
    // the claim is consumed last, so the claim's round trip overlaps the slot
    // arithmetic; the caller compacts the wave's claims into its region
    claimed = __shfl(claimed, threadIdx.x & 63, 64);
    if (slot && claimed == 0u) {
        ckind = r < 4 ? 0 : 1;
        cbd = bd;
    }
    if (r == 0)
        v.undo[i] = (owner && change) ? prev : (uint8_t)0xFF;
    return bits;
}

// Phase 2 lanes: per claim region, 6 QD lanes for each of its 16 diagonal
// records then 9 QO lanes for each of its 24 off-diagonal records, padded to
// whole waves; after all regions, one lane per edit (stamp release,
// rollback).  Every lane group of Q starts at a multiple of Q, so it never
// crosses a wave boundary.  Lanes of records past a region's count have
// nothing to do, and since each region fills from its start, whole waves of
// them exit at once.
template <int QD, int QO>
struct Phase2 {
    static constexpr int LD = 6 * QD, LO = 9 * QO;
    static constexpr int kDiagLanes = kRegionDiag * LD;
    // padded to whole waves, so that every region starts at a wave boundary
    static constexpr int kRegionLanes = (kDiagLanes + kRegionOff * LO + 63) / 64 * 64;
};

// Decode phase-2 lane t: a record lane (region w, slot in the region, lane
// rem among the record's 6 QD or 9 QO lanes), an edit lane (edit = index
// into the edit list, returned in w with slot = -1) or a padding lane
// (slot = -2).
template <int QD, int QO>
__device__ __forceinline__ void touched_role(int64_t t, int regions, int& w, int& slot, int& rem)
{
    using P = Phase2<QD, QO>;
    const int64_t rl = (int64_t)regions * P::kRegionLanes;
    rem = 0;
    if (t >= rl) {
        w = (int)(t - rl);
        slot = -1;
        return;
    }
    w = (int)(t / P::kRegionLanes);
    const int u = (int)(t - (int64_t)w * P::kRegionLanes);
    if (u < P::kDiagLanes) {
        slot = u / P::LD;
        rem = u - slot * P::LD;
    } else {
        const int u2 = u - P::kDiagLanes;
        const int k = u2 / P::LO;
        if (k >= kRegionOff) {
            slot = -2;
            return;
        }
        slot = kRegionDiag + k;
        rem = u2 - k * P::LO;
    }
}

// Phase 2, record lane rem: re-sum value rem / Q of a claimed block, Q lanes
// per value (Q from the block's incidence-length bucket; lanes past the
// record's 6Q or 9Q idle) unless the frame has an error; the record's first
// lane releases the block's claim stamp either way.
template <int QD, int QO, bool MIXED>
__device__ __forceinline__ void touched_record(const DevView& v, const BlockDesc& d, int fe, int rem,
                                               const MapConfig& m)
{
    const int Q = bucket_q<QD, QO, MIXED>(m, d);
    if (rem >= (d.kind == 0 ? 6 : 9) * Q)
        return;
    const int q = rem & (Q - 1);
    if (!fe)
        block_value_q<QD, QO, MIXED>(v, d, rem / Q, q, (threadIdx.x & 63) - q, Q);
    if (rem == 0)
        v.bstamp[d.block] = 0u;
}

// Phase 2, edit lane for edit i (tet id, undo byte u): release the tet stamp
// and, if the frame has an error, undo the edit's mask flip and slot rewrite.
__device__ __forceinline__ void touched_edit(const DevView& v, int id, uint8_t u, int fe)
{
    if (id < 0 || id >= v.n_tets)
        return;
    v.estamp[id] = 0u;
    if (fe && u != 0xFF) {
        int ep[10];
#pragma unroll
        for (int k = 0; k < 10; ++k)
            ep[k] = v.e2p[10 * (size_t)id + k];
        v.mask[id] = u;
        if (u)
            store_element(v, id, v.T[id], ep);
        else
            zero_element(v, ep);
    }
}

// Workgroup-wide OR of error bits.
__device__ __forceinline__ int block_or(int bits, int* s_bits)
{
    if (threadIdx.x == 0)
        *s_bits = 0;
    __syncthreads();
    if (bits)
        atomicOr(s_bits, bits);
    __syncthreads();
    return *s_bits;
}

// OR of the first g error bytes of the edit phase.
__device__ __forceinline__ int frame_error(const DevView& v, int g, int* s_bits)
{
    int bits = 0;
    for (int w = threadIdx.x; w < g; w += kBlock)
        bits |= v.wg_err[w];
    return block_or(bits, s_bits);
}

__device__ __forceinline__ void publish_frame(const DevView& v, int fe, int n, int regions)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        v.ctl->frame_err = fe;
        v.ctl->last_n = n;
        v.ctl->last_regions = regions;
        if (fe)
            atomicOr(&v.ctl->err, fe);
    }
}

// Compact the wave's claims into claim region `region`: diagonal claims
// first, then off-diagonal ones, each in lane order; lane 0 records the two
// counts.  Called by every lane of the wave (ckind = -1: no claim).
__device__ __forceinline__ void compact_claims(const DevView& v, int64_t region, int ckind, const BlockDesc& cbd)
{
    const uint64_t dm = __ballot(ckind == 0);
    const uint64_t om = __ballot(ckind == 1);
    const uint64_t below = __lanemask_lt();
    BlockDesc* base = v.rec + region * kRegion;
    if (ckind == 0)
        store_desc(base + __popcll(dm & below), cbd);
    else if (ckind == 1)
        store_desc(base + kRegionDiag + __popcll(om & below), cbd);
    if ((threadIdx.x & 63) == 0) {
        v.rcount[2 * region] = __popcll(dm);
        v.rcount[2 * region + 1] = __popcll(om);
    }
}

// Phase 1 as its own kernel: one 16-lane group per edit.  Each workgroup
// writes its error bits to its own byte, so nothing needs resetting.
__global__ __launch_bounds__(kBlock) void k_edits(DevView v, const int32_t* __restrict__ ids,
                                                  const uint8_t* __restrict__ states, int32_t n_host,
                                                  const int32_t* __restrict__ n_dev)
{
    __shared__ int s_bits;
    const int gt = blockIdx.x * kBlock + threadIdx.x;
    const int i = gt / kEditLanes;
    // the edit itself is read while the device-side count is still in flight
    int id = -1;
    unsigned st = 0;
    if (i < n_host) {
        id = ids[i];
        st = states[i];
    }
    bool bad_n;
    const int n = frame_count(n_host, n_dev, bad_n);
    int bits = (bad_n && gt == 0) ? ERR_RANGE : 0;
    int ckind = -1;
    BlockDesc cbd;
    if (i < n)
        bits |= edit_lane(v, id, st, i, gt - i * kEditLanes, ckind, cbd);
    compact_claims(v, gt / 64, ckind, cbd);
    bits = block_or(bits, &s_bits);
    if (threadIdx.x == 0)
        v.wg_err[blockIdx.x] = (uint8_t)bits;
}

// Phase 2 as its own kernel.
template <int QD, int QO, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_touched(DevView v, const int32_t* __restrict__ ids, int32_t n_host,
                                                    const int32_t* __restrict__ n_dev, MapConfig m)
{
    __shared__ int s_bits;
    // the edit phase ran `edit_wgs` workgroups of kRegionsPerBlock waves, each wave one claim region
    const int edit_wgs = n_host > 0 ? (n_host * kEditLanes + kBlock - 1) / kBlock : 1;
    const int regions = edit_wgs * kRegionsPerBlock;
    int w, slot, rem;
    touched_role<QD, QO>((int64_t)blockIdx.x * kBlock + threadIdx.x, regions, w, slot, rem);
    // claim record and count, or the edit's id and undo byte, load together
    // with the error bytes and the device-side count; lanes without them read
    // fixed empty values instead, so the loads need no branch
    const bool rec_lane = slot >= 0;
    const bool edit_lane_ = slot == -1 && w < n_host;
    const BlockDesc d = load_desc(rec_lane ? v.rec + (size_t)w * kRegion + slot : &kNoClaim);
    const int cnt = rec_lane ? v.rcount[2 * w + (slot >= kRegionDiag ? 1 : 0)] : 0;
    const int id = *(edit_lane_ ? ids + w : &kNoTet);
    const uint8_t u = edit_lane_ ? v.undo[w] : (uint8_t)0xFF;
    // the error bytes of every workgroup of the edit phase
    int bits = threadIdx.x < edit_wgs ? v.wg_err[threadIdx.x] : 0;
    for (int k = threadIdx.x + kBlock; k < edit_wgs; k += kBlock)
        bits |= v.wg_err[k];
    bool bad_n;
    const int n = frame_count(n_host, n_dev, bad_n);
    const int fe = block_or(bits, &s_bits);
    publish_frame(v, fe, n, regions);
    if (rec_lane) {
        if (slot - (slot >= kRegionDiag ? kRegionDiag : 0) < cnt)
            touched_record<QD, QO, MIXED>(v, d, fe, rem, m);
    } else if (edit_lane_ && w < n) {
        touched_edit(v, id, u, fe);
    }
}

// ---------------------------------------------------------------------------
// +/- delta policy (the paper's streaming_update for element assembly:
// touched entries change by adding or removing the edited elements' local
// contributions, Sec. 3.4 / Sec. 3.5)
// ---------------------------------------------------------------------------

// Add s * (block slot r's values) into the CSR values of block d (and its
// mirror), with hardware FP64 atomics.  The order in which concurrent edits
// land is not fixed, so the result is reproducible only up to rounding.
__device__ __forceinline__ void delta_block(const DevView& v, const BlockDesc& d, const double* x, bool add)
{
    if (d.kind == 0) {
#pragma unroll
        for (int vi = 0; vi < 6; ++vi) {
            const int p = kDiagP[vi], q = kDiagQ[vi];
            const double y = add ? x[vi] : -x[vi];
            unsafeAtomicAdd(v.values + d.up + p * d.rl + q, y);
            if (p != q)
                unsafeAtomicAdd(v.values + d.up + q * d.rl + p, y);
        }
    } else {
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const double y = add ? x[3 * p + q] : -x[3 * p + q];
                unsafeAtomicAdd(v.values + d.up + p * d.rl + q, y);
                unsafeAtomicAdd(v.values + d.lo + q * d.rlj + p, y);
            }
    }
}

// Lane r of edit i under the delta policy (16 lanes per edit, lane r < 10
// owns block slot r).  A changed tet's slot values are added (activation:
// computed and stored in its slot first) or subtracted (deletion: read from
// its slot, which is then zeroed), so the per-element contributions stay as
// the exact policy expects and either policy may follow.  Invalid and
// duplicate edits are skipped and reported; nothing is rolled back.
__device__ __forceinline__ int delta_lane(const DevView& v, int id, unsigned st, int r)
{
    if (id < 0 || id >= v.n_tets || st > 1u)
        return r == 0 ? ERR_RANGE : 0;
    const bool slot = r < 10;
    uint32_t eb = 0;
    int ep = 0;
    if (slot) {
        eb = (uint32_t)v.e2b[10 * (size_t)id + r];
        ep = v.e2p[10 * (size_t)id + r];
    }
    int4 t = make_int4(0, 0, 0, 0);
    double E = 0.0;
    if (slot && st) {
        t = v.T[id];
        E = v.E[id];
    }
    const uint8_t prev = v.mask[id];
    unsigned taken = 0u;
    if (r == 0)
        taken = atomicExch(&v.estamp[id], 1u);
    BlockDesc bd = empty_desc();
    if (slot)
        bd = load_desc(v.desc + eb);
    double X[4][3];
    if (slot && st)
        load_vertices(v, t, X);
    const bool owner = __shfl(taken, (threadIdx.x & 63) & ~(kEditLanes - 1), 64) == 0u;
    if (!owner)
        return r == 0 ? ERR_DUP : 0;
    if (prev == st)
        return 0;
    if (r == 0)
        v.mask[id] = (uint8_t)st;
    if (!slot)
        return 0;
    const int nv = r < 4 ? 6 : 9;
    const double* src = r < 4 ? v.cd + 6 * (size_t)ep : v.co + 9 * (size_t)ep;
    double x[9];
    Geo G;
    if (st) {
        geometry_from(v, X, E, G);
        store_slot(v, t, G, r, ep, true);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k)
        x[k] = k < nv ? src[k] : 0.0;
    if (!st)
        store_slot(v, t, G, r, ep, false);
    delta_block(v, bd, x, st != 0u);
    return 0;
}

__global__ __launch_bounds__(kBlock) void k_delta_edits(DevView v, const int32_t* __restrict__ ids,
                                                        const uint8_t* __restrict__ states, int32_t n_host,
                                                        const int32_t* __restrict__ n_dev)
{
    const int gt = blockIdx.x * kBlock + threadIdx.x;
    const int i = gt / kEditLanes;
    int id = -1;
    unsigned st = 0;
    if (i < n_host) {
        id = ids[i];
        st = states[i];
    }
    bool bad_n;
    const int n = frame_count(n_host, n_dev, bad_n);
    int bits = (bad_n && gt == 0) ? ERR_RANGE : 0;
    if (i < n)
        bits |= delta_lane(v, id, st, gt - i * kEditLanes);
    if (bits)
        atomicOr(&v.ctl->err, bits);
    if (gt == 0) {
        v.ctl->last_n = n;
        v.ctl->frame_err = 0;
        v.ctl->last_regions = 0;  // the delta policy claims no blocks
    }
}

// Release the frame's tet stamps (one lane per edit).
__global__ __launch_bounds__(kBlock) void k_delta_clear(DevView v, const int32_t* __restrict__ ids, int32_t n_host,
                                                        const int32_t* __restrict__ n_dev)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    bool bad_n;
    const int n = frame_count(n_host, n_dev, bad_n);
    if (i < n) {
        const int id = ids[i];
        if (id >= 0 && id < v.n_tets)
            v.estamp[id] = 0u;
    }
}

// The whole frame in one persistent launch: phase 1 over the edits, grid
// barrier, phase 2 over the claimed blocks (grid-stride loops; lane groups
// stay aligned because the stride is a multiple of the workgroup size).
template <int QD, int QO, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_frame(DevView v, const int32_t* __restrict__ ids,
                                                  const uint8_t* __restrict__ states, int32_t n_host,
                                                  const int32_t* __restrict__ n_dev, MapConfig m,
                                                  unsigned spin_limit)
{
    __shared__ int s_bits;
    __shared__ int s_ok;
    bool bad_n;
    const int n = frame_count(n_host, n_dev, bad_n);
    const int regions = (n_host > 0 ? (n_host * kEditLanes + kBlock - 1) / kBlock : 1) * kRegionsPerBlock;
    int bits = (bad_n && blockIdx.x == 0 && threadIdx.x == 0) ? ERR_RANGE : 0;
    // phase 1 over whole waves (one claim region each), so that every lane of
    // a wave runs the compaction together
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < (int64_t)regions * 64;
         t += (int64_t)gridDim.x * kBlock) {
        const int i = (int)(t / kEditLanes);
        int ckind = -1;
        BlockDesc cbd;
        if (i < n)
            bits |= edit_lane(v, ids[i], states[i], i, (int)(t - (int64_t)i * kEditLanes), ckind, cbd);
        compact_claims(v, t / 64, ckind, cbd);
    }
    bits = block_or(bits, &s_bits);
    if (threadIdx.x == 0)
        v.wg_err[blockIdx.x] = (uint8_t)bits;
    if (!grid_barrier(v.ctl, gridDim.x, spin_limit, &s_ok))
        return;
    const int fe = frame_error(v, gridDim.x, &s_bits);
    publish_frame(v, fe, n, regions);
    const int64_t total = (int64_t)regions * Phase2<QD, QO>::kRegionLanes + n_host;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < total; t += (int64_t)gridDim.x * kBlock) {
        int w, slot, rem;
        touched_role<QD, QO>(t, regions, w, slot, rem);
        if (slot >= 0) {
            const int c = v.rcount[2 * w + (slot >= kRegionDiag ? 1 : 0)];
            if (slot - (slot >= kRegionDiag ? kRegionDiag : 0) < c)
                touched_record<QD, QO, MIXED>(v, load_desc(v.rec + (size_t)w * kRegion + slot), fe, rem, m);
        } else if (slot == -1 && w < n) {
            touched_edit(v, ids[w], v.undo[w], fe);
        }
    }
}

// Audit: 1 if tet e's 78 stored contribution slots differ in any bit from
// what the rebuild would store (its element matrix if active, +0.0 if not).
__device__ __forceinline__ int audit_element(const DevView& v, int e)
{
    int pos[10];
#pragma unroll
    for (int j = 0; j < 10; ++j)
        pos[j] = v.e2p[10 * (size_t)e + j];
    const bool active = v.mask[e] != 0;
    Geo G;
    const int4 t = v.T[e];
    if (active)
        element_geometry(v, e, t, G);
    const int id[4] = {t.x, t.y, t.z, t.w};
    bool bad = false;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const double* c = v.cd + 6 * (size_t)pos[a];
        double ga[3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
            ga[i] = active ? G.g[a][i] : 0.0;
        const double s = dot3(ga, ga);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double want = active ? entry(ga, ga, s, G, kDiagP[k], kDiagQ[k], true) : 0.0;
            bad = bad || __double_as_longlong(c[k]) != __double_as_longlong(want);
        }
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const bool sw = id[PA[q]] > id[PB[q]];
        double ga[3], gb[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            ga[i] = active ? (sw ? G.g[PB[q]][i] : G.g[PA[q]][i]) : 0.0;
            gb[i] = active ? (sw ? G.g[PA[q]][i] : G.g[PB[q]][i]) : 0.0;
        }
        const double s = dot3(ga, gb);
        const double* c = v.co + 9 * (size_t)pos[4 + q];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double want = active ? entry(ga, gb, s, G, i, j, false) : 0.0;
                bad = bad || __double_as_longlong(c[3 * i + j]) != __double_as_longlong(want);
            }
    }
    return bad ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_audit_tets(DevView v, unsigned long long* count)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    const int bad = e < v.n_tets ? audit_element(v, e) : 0;
    const uint64_t m = __ballot(bad != 0);
    if ((threadIdx.x & 63) == 0 && m)
        atomicAdd(count, (unsigned long long)__popcll(m));
}

// Audit: values whose bits differ between a and b.
__global__ __launch_bounds__(kBlock) void k_audit_values(const double* __restrict__ a, const double* __restrict__ b,
                                                         int64_t n, unsigned long long* count)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool bad = i < n && __double_as_longlong(a[i]) != __double_as_longlong(b[i]);
    const uint64_t m = __ballot(bad);
    if ((threadIdx.x & 63) == 0 && m)
        atomicAdd(count, (unsigned long long)__popcll(m));
}

// Release every tet and block stamp (after a fused frame whose grid barrier
// gave up, some workgroups left before phase 2 and their stamps stay taken).
__global__ __launch_bounds__(kBlock) void k_clear_stamps(DevView v)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < v.n_tets)
        v.estamp[i] = 0u;
    if (i < v.nd + v.no)
        v.bstamp[i] = 0u;
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

// The geometry part of every tet record, from the current coordinates and
// moduli, by the rebuild's own routine (element_geometry).
__global__ __launch_bounds__(kBlock) void k_refresh_records(DevView v, TetRecord* __restrict__ trec)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= v.n_tets)
        return;
    Geo G;
    element_geometry(v, e, v.T[e], G);
    TetRecord& rc = trec[e];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i)
            rc.g[3 * a + i] = G.g[a][i];
    rc.lamV = G.lamV;
    rc.muV = G.muV;
    rc.ml = G.ml;
    rc.degenerate = G.det == 0.0 ? 1 : 0;
}

inline unsigned blocks_for(int64_t threads)
{
    return (unsigned)((threads + kBlock - 1) / kBlock);
}

}  // namespace

// Dynamic LDS of the element kernel, reserved and unused: with its 18 KB of
// staging it makes 44 KB per workgroup, three workgroups per CU instead of
// the five its registers allow; fewer tets in flight keep their node
// coordinates and staged lines in cache (on the 384k-tet cube: 61.0 -> 57.4 us
// per rebuild, same bits; two per CU 58.6 us, four 60.0 us).
constexpr uint32_t kElementReservedLds = 26 << 10;

hipError_t launch_element(const DevView& v, bool nt, hipStream_t s)
{
    if (v.n_tets == 0)
        return hipSuccess;
    if (nt)
        launch_kernel(&k_element<true>, dim3(blocks_for(v.n_tets)), dim3(kBlock), kElementReservedLds, s, v);
    else
        launch_kernel(&k_element<false>, dim3(blocks_for(v.n_tets)), dim3(kBlock), kElementReservedLds, s, v);
    return hipGetLastError();
}

#define STA_MAPPINGS(X) X(1, 1) X(1, 4) X(4, 1) X(4, 4) X(16, 1) X(16, 4)

// Whether some incidence-length bucket uses fewer lanes than the allocation.
bool mixed_map(const MapConfig& m)
{
    for (int b = 0; b < kDiagBuckets; ++b)
        if (m.qdb[b] != m.qd)
            return true;
    for (int b = 0; b < kOffBuckets; ++b)
        if (m.qob[b] != m.qo)
            return true;
    return false;
}

hipError_t launch_reduce_all(const DevView& v, const MapConfig& m, hipStream_t s)
{
    const int64_t diag_lanes = ((int64_t)v.nd * 6 * m.qd + 63) / 64 * 64;
    const int64_t threads = diag_lanes + (m.qo == 1 ? ((int64_t)v.no + 6) / 7 * 64 : (int64_t)v.no * 9 * m.qo);
    if (v.nd + v.no == 0)
        return hipSuccess;
    const bool mixed = mixed_map(m);
#define LAUNCH(QD, QO)                                                                                    \
    if (m.qd == QD && m.qo == QO) {                                                                       \
        const dim3 g(blocks_for(threads));                                                                \
        if (mixed && m.nt)                                                                                \
            launch_kernel(&k_reduce_all<QD, QO, true, true>, g, dim3(kBlock), 0, s, v, diag_lanes, m);    \
        else if (mixed)                                                                                   \
            launch_kernel(&k_reduce_all<QD, QO, true, false>, g, dim3(kBlock), 0, s, v, diag_lanes, m);   \
        else if (m.nt)                                                                                    \
            launch_kernel(&k_reduce_all<QD, QO, false, true>, g, dim3(kBlock), 0, s, v, diag_lanes, m);   \
        else                                                                                              \
            launch_kernel(&k_reduce_all<QD, QO, false, false>, g, dim3(kBlock), 0, s, v, diag_lanes, m);  \
        return hipGetLastError();                                                                         \
    }
    STA_MAPPINGS(LAUNCH)
#undef LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_edit_phase(const DevView& v, const int32_t* ids, const uint8_t* states, int32_t n_host,
                             const int32_t* n_dev, hipStream_t s)
{
    // an empty list still runs one workgroup of each phase: they record the frame (count 0)
    launch_kernel(&k_edits, dim3(n_host > 0 ? blocks_for((int64_t)n_host * kEditLanes) : 1u), dim3(kBlock), 0,
                       s, v, ids, states, n_host, n_dev);
    return hipGetLastError();
}

hipError_t launch_delta_frame(const DevView& v, const int32_t* ids, const uint8_t* states, int32_t n_host,
                              const int32_t* n_dev, hipStream_t s)
{
    hipLaunchKernelGGL(k_delta_edits, dim3(n_host > 0 ? blocks_for((int64_t)n_host * kEditLanes) : 1u), dim3(kBlock),
                       0, s, v, ids, states, n_host, n_dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_host == 0)
        return e;
    hipLaunchKernelGGL(k_delta_clear, dim3(blocks_for(n_host)), dim3(kBlock), 0, s, v, ids, n_host, n_dev);
    return hipGetLastError();
}

hipError_t launch_touched_phase(const DevView& v, const MapConfig& m, const int32_t* ids, int32_t n_host,
                                const int32_t* n_dev, hipStream_t s)
{
#define LAUNCH(QD, QO)                                                                                      \
    if (m.qd == QD && m.qo == QO) {                                                                         \
        const int64_t regions = (n_host > 0 ? ((int64_t)n_host * kEditLanes + kBlock - 1) / kBlock : 1) * kRegionsPerBlock; \
        const int64_t lanes = regions * Phase2<QD, QO>::kRegionLanes + n_host;                              \
        if (mixed_map(m))                                                                                   \
            launch_kernel(&k_touched<QD, QO, true>, dim3(blocks_for(lanes)), dim3(kBlock), 0, s, v, ids,    \
                          n_host, n_dev, m);                                                                \
        else                                                                                                \
            launch_kernel(&k_touched<QD, QO, false>, dim3(blocks_for(lanes)), dim3(kBlock), 0, s, v, ids,   \
                          n_host, n_dev, m);                                                                \
        return hipGetLastError();                                                                           \
    }
    STA_MAPPINGS(LAUNCH)
#undef LAUNCH
    return hipErrorInvalidValue;
}

hipError_t frame_max_grid(const MapConfig& m, int device, int* max_grid)
{
    int cus = 0, per_cu = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess)
        return e;
#define OCC(QD, QO)                                                                                        \
    if (m.qd == QD && m.qo == QO)                                                                          \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(                                                  \
            &per_cu, mixed_map(m) ? (const void*)&k_frame<QD, QO, true> : (const void*)&k_frame<QD, QO, false>, \
            kBlock, 0);
    STA_MAPPINGS(OCC)
#undef OCC
    if (e != hipSuccess)
        return e;
    *max_grid = per_cu * cus;
    return hipSuccess;
}

int frame_grid_for(const MapConfig& m, int32_t n_host, int max_grid, int grid_cap)
{
    int L = 16;
#define LANES(QD, QO)                 \
    if (m.qd == QD && m.qo == QO)     \
        L = Phase2<QD, QO>::kRegionLanes;
    STA_MAPPINGS(LANES)
#undef LANES
    const int64_t regions = (n_host > 0 ? ((int64_t)n_host * kEditLanes + kBlock - 1) / kBlock : 1) * kRegionsPerBlock;
    const int64_t want = (regions * L + n_host + kBlock - 1) / kBlock;
    int64_t g = want < max_grid ? want : max_grid;
    if (grid_cap > 0 && g > grid_cap)
        g = grid_cap;
    return (int)(g < 1 ? 1 : g);
}

hipError_t launch_frame(const DevView& v, const MapConfig& m, int grid, const int32_t* ids, const uint8_t* states,
                        int32_t n_host, const int32_t* n_dev, unsigned spin_limit, hipStream_t s)
{
#define LAUNCH(QD, QO)                                                                                        \
    if (m.qd == QD && m.qo == QO) {                                                                           \
        if (mixed_map(m))                                                                                     \
            launch_kernel(&k_frame<QD, QO, true>, dim3(grid), dim3(kBlock), 0, s, v, ids, states, n_host,     \
                          n_dev, m, spin_limit);                                                              \
        else                                                                                                  \
            launch_kernel(&k_frame<QD, QO, false>, dim3(grid), dim3(kBlock), 0, s, v, ids, states, n_host,    \
                          n_dev, m, spin_limit);                                                              \
        return hipGetLastError();                                                                             \
    }
    STA_MAPPINGS(LAUNCH)
#undef LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_audit(const DevView& v, const MapConfig& m, double* scratch_values, int64_t nnz,
                        unsigned long long* counts, hipStream_t s)
{
    hipError_t e = hipSuccess;
    if (v.n_tets > 0) {
        hipLaunchKernelGGL(k_audit_tets, dim3(blocks_for(v.n_tets)), dim3(kBlock), 0, s, v, counts + 1);
        e = hipGetLastError();
    }
    if (e != hipSuccess || nnz == 0)
        return e;
    DevView w = v;
    w.values = scratch_values;
    e = launch_reduce_all(w, m, s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_audit_values, dim3(blocks_for(nnz)), dim3(kBlock), 0, s, v.values, scratch_values, nnz,
                       counts);
    return hipGetLastError();
}

hipError_t launch_clear_stamps(const DevView& v, hipStream_t s)
{
    const int64_t n = v.n_tets > v.nd + v.no ? v.n_tets : v.nd + v.no;
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_clear_stamps, dim3(blocks_for(n)), dim3(kBlock), 0, s, v);
    return hipGetLastError();
}

hipError_t launch_refresh_records(const DevView& v, TetRecord* trec, hipStream_t s)
{
    if (v.n_tets == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_refresh_records, dim3(blocks_for(v.n_tets)), dim3(kBlock), 0, s, v, trec);
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
