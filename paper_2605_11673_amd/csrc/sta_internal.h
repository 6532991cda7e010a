// Internal layout of a stafem context: host bookkeeping plus the device
// buffers the kernels read and write.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstddef>
#include <cstdio>
#include <cstdint>
#include <string>
#include <vector>

#include "stafem.h"
#include <hip/hip_ext.h>

namespace sta {

// Device-detected error bits (Ctl::ferr / Ctl::err).
enum : int32_t {
    ERR_RANGE = 1,       // edit id out of range or state not in {0, 1}
    ERR_DUP = 2,         // the same tet twice in one edit list
    ERR_DEGENERATE = 4,  // det == 0 in an element
    ERR_TIMEOUT = 8,     // a fused frame's grid barrier gave up (grid not co-resident)
};

// Control words kept in device memory so that a frame never needs the host
// (and can be replayed from a captured graph).
struct Ctl {
    int32_t err;         // sticky error bits, cleared by sta_status_sync
    int32_t frame_err;   // error bits of the last frame (written by the reduce phase)
    int32_t last_n;      // edit count of the last frame (statistics; also right under graph replay)
    uint32_t bar_count;  // grid barrier of the fused frame kernel: arrivals
    uint32_t bar_gen;    // and generation
    int32_t last_regions;  // claim regions of the last frame (one per edit-phase wave of 4 edits)
    int32_t pad;
};

// Polls of the fused frame's grid barrier before it reports ERR_TIMEOUT.
constexpr unsigned kBarrierSpinDefault = 1u << 24;

// Grid-wide barrier for a co-resident grid (the host sizes the grid from the
// occupancy so that every workgroup is resident).  The spin is bounded (at
// most spin_limit polls): a grid that is not co-resident reports ERR_TIMEOUT
// instead of hanging.

__device__ __forceinline__ bool grid_barrier(Ctl* ctl, unsigned G, unsigned spin_limit, int* s_ok)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned gen = __hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const unsigned arrived = atomicAdd(&ctl->bar_count, 1u);
        if (arrived == G - 1) {
            __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            __hip_atomic_fetch_add(&ctl->bar_gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins >= spin_limit) {
                    ok = 0;
                    atomicOr(&ctl->err, ERR_TIMEOUT);
                    break;
                }
            }
        }
        __threadfence();
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}


// Workgroups are dispatched round-robin over the 8 XCDs of the device, each
// with its own L2.  xcd_remap maps a dispatch index to a work index such
// that each XCD walks one contiguous share of the work (sizes differ by at
// most one), so that neighbouring work, which shares cache lines, stays in
// one L2.  A permutation of [0, G).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_remap(int wg, int G)
{
    const int q = G / kXcds, r = G % kXcds;
    const int x = wg % kXcds, idx = wg / kXcds;
    const int base = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return base + idx;
}

// Incidence-length buckets of the slot mapping: a block's segment length
// kappa (its number of candidate tets) puts a diagonal block in bucket 0
// (kappa <= 8), 1 (9..32) or 2 (> 32), an off-diagonal block in bucket 0
// (kappa <= 8) or 1 (> 8).
constexpr int kDiagBuckets = 3, kOffBuckets = 2;
__host__ __device__ inline int diag_bucket(int kappa)
{
    return kappa <= 8 ? 0 : (kappa <= 32 ? 1 : 2);
}
__host__ __device__ inline int off_bucket(int kappa)
{
    return kappa <= 8 ? 0 : 1;
}

// Slot mapping: lanes per block value (1 thread-, 4 quad-, 16
// wave-sixteenth-per-slot; diagonal 1/4/16, off-diagonal 1/4), chosen per
// incidence-length bucket (qdb, qob).  qd / qo are the lanes allocated per
// value, the largest bucket mapping; a block whose bucket uses fewer leaves
// the rest of its lanes idle.
struct MapConfig {
    int qd = 1, qo = 1;
    int nt = 0;  // non-temporal cache hints (rebuild only)
    int qdb[kDiagBuckets] = {1, 1, 1};
    int qob[kOffBuckets] = {1, 1};
};

// One mapping for every bucket.
inline MapConfig uniform_map(int qd, int qo, int nt)
{
    MapConfig m;
    m.qd = qd;
    m.qo = qo;
    m.nt = nt;
    for (int b = 0; b < kDiagBuckets; ++b)
        m.qdb[b] = qd;
    for (int b = 0; b < kOffBuckets; ++b)
        m.qob[b] = qo;
    return m;
}

// Material constants, evaluated once on the host in the fixed order.
struct Material {
    double cdt;   // dt*dt
    double clam;  // nu / ((1+nu)*(1-2nu))
    double cmu;   // 0.5 / (1+nu)
    double rho;
};

// One 3x3 node block of the matrix (diagonal blocks first, then the
// off-diagonal blocks i < j in ascending (i, j)).  32 bytes so a lane reads it
// with two 16-byte loads.
struct BlockDesc {
    int32_t k0, k1;  // incidence range: into cd (diagonal) or co (off-diagonal)
    int32_t up, rl;  // CSR index of entry (3i, 3j) and row length 3*deg(i)
    int32_t lo, rlj; // CSR index of entry (3j, 3i) and row length 3*deg(j) (diagonal: = up, rl)
    int32_t kind;    // 0 diagonal, 1 off-diagonal, -1 empty claim record
    int32_t block;   // block id
};

// Everything the edit phase reads about one candidate tet, packed in one
// 512-byte record so that an edit needs a single memory round trip before
// its atomics: the tet's 10 block descriptors (local pairs 00 11 22 33 | 01
// 02 03 12 13 23), its geometry as the element formula uses it (basis
// gradients g_0..g_3, lamV, muV and the lumped mass per vertex, computed on
// the device by the same routine as the rebuild's, so an activation
// reproduces the rebuild's bits without redoing the determinant and the
// inverse; refreshed by sta_set_params), a flag for det == 0, its vertex ids
// and its 10 incidence positions.
struct TetRecord {
    BlockDesc desc[10];
    double g[12];  // g_a component i at 3a + i
    int4 T;
    double lamV, muV, ml;  // lamV at a 16-byte boundary (read with muV as one 16-byte load)
    int32_t pos[10];
    int32_t degenerate;  // det == 0
    int32_t pad[3];
};
static_assert(sizeof(TetRecord) == 512, "tet record is 512 bytes");
static_assert(offsetof(TetRecord, lamV) % 16 == 0, "lamV and muV are read as one 16-byte load");

// Everything the kernels need, passed by value.
//
// Invariant kept by every kernel: the contributions of an inactive tet are
// +0.0 in all 78 of its incidence slots.  Block sums then run over the whole
// segment without looking at the mask, and adding those +0.0 terms gives the
// same bits as skipping them.
struct DevView {
    int32_t n_nodes, n_tets;
    int32_t nd, no;               // diagonal / off-diagonal 3x3 blocks
    const double* xs;             // SoA node coordinates
    const double* ys;
    const double* zs;
    const int4* T;                // tets
    const double* E;
    uint8_t* mask;
    const BlockDesc* desc;        // nd + no blocks
    const int32_t* ndiag;         // per node: its diagonal block id, -1 if in no candidate tet
    // per tet, local pair order 00 11 22 33 | 01 02 03 12 13 23: block ids and
    // incidence positions (into cd for the first 4, into co for the other 6)
    const int32_t* e2b;
    const int32_t* e2p;
    const TetRecord* trec;        // per tet: what the edit phase reads
    double* cd;                   // 6 unique values per diagonal incidence
    double* co;                   // 9 values per off-diagonal incidence (block orientation)
    double* values;               // CSR values
    // streaming state
    // Stamps are 1 only while a frame is in flight: the edit phase sets them,
    // the reduce phase clears the ones it set.
    uint32_t* estamp;             // per tet: taken by an edit of this frame
    uint32_t* bstamp;             // per block: claimed in this frame
    // Claimed blocks of the frame, compacted per edit-phase wave (4 edits):
    // region w holds up to 16 diagonal then 24 off-diagonal block
    // descriptors; rcount[2w], rcount[2w+1] say how many of each are valid.
    BlockDesc* rec;
    int32_t* rcount;
    uint8_t* undo;                // per edit: previous mask value, 0xFF = nothing to undo
    uint8_t* wg_err;              // per edit-phase workgroup: its error bits (always written)
    Ctl* ctl;
    Material mat;
};

// Conjugate-gradient workspace (cg.hip).
struct CgScalars {
    double rz, alpha, beta, rr, bnorm2, tol2;
    int32_t iters, done;
    double rzk[2];  // r_k . z_k by iteration parity (the product of iteration k reads k-1's, writes k's)
};

struct CgView {
    int32_t n;        // rows
    int32_t nparts;   // partial sums of the start kernels (one per 256 rows)
    int32_t nparts_s; // partial sums of the product (one per workgroup)
    int32_t nparts_u; // partial sums of the update (one per workgroup, two dot products)
    const int32_t* rowptr;
    const int32_t* colidx;
    const double* vals;
    const int32_t* dpos;  // diagonal position per row, -1 if none
    double *x, *r, *z, *p, *q, *dinv, *part;  // p: two copies of n (previous / new direction)
    CgScalars* s;
};

}  // namespace sta

struct sta_ctx {
    int64_t n_nodes = 0, n_tets = 0, n_rows = 0, nnz = 0, nd = 0, no = 0;
    double nu = 0, rho = 0, dt = 0;
    bool stale = false;
    int device = 0;
    sta::DevView v{};
    int32_t* rowptr = nullptr;  // device
    int32_t* colidx = nullptr;  // device
    std::vector<void*> owned;   // every device allocation
    // execution configuration (sta_set_config / sta_autotune)
    sta::MapConfig rebuild_map, stream_map;
    int64_t bucket_blocks[sta::kDiagBuckets + sta::kOffBuckets] = {};  // blocks per incidence-length bucket
    int fused = 0;          // 1: one persistent launch per frame
    int frame_grid_cap = 0; // 0: occupancy limit only
    int frame_max_grid = 0; // co-resident workgroups for the fused kernel (per stream_map)
    unsigned barrier_spin = sta::kBarrierSpinDefault;  // polls before the fused frame's barrier gives up
    bool fused_used = false;  // a fused frame ran since the last rebuild (stamps may be left taken)
    // per-call trace (environment variable STA_TRACE names a JSON-lines file)
    FILE* trace = nullptr;
    bool trace_stats = false;  // STA_TRACE_STATS=1: synchronise and add each frame's statistics
    int64_t trace_seq = 0;
    double trace_t0 = 0.0;     // host seconds at context build
    // lazily allocated workspaces
    double* cg_ws = nullptr;        // 7 vectors of n_rows (two copies of p) + partials
    int32_t* cg_dpos = nullptr;
    sta::CgScalars* cg_s = nullptr;
    sta::CgScalars* cg_host = nullptr;  // pinned
    double* adj_xbar = nullptr;     // 3 doubles per diagonal incidence
    int32_t* adj_order = nullptr;   // adjoint visiting order of the kAdjointChunk-tet chunks
    int32_t adj_chunks = 0;
    int32_t* dinc = nullptr;        // per diagonal incidence: its tet (segments in ascending tet id)
    double* tet_ml = nullptr;       // per tet: lumped mass per vertex dof, (rho V) / 4
    bool tet_ml_stale = true;
    double* euler_ws = nullptr;     // implicit Euler: M_t, right-hand side, new u (3 x n_rows)
    double* audit_ws = nullptr;     // audit: nnz re-summed values, then 2 counters
    int32_t* cc_ws = nullptr;       // connectivity: parent and mark per node, then the pass flags
    uint32_t* cc_host = nullptr;    // pinned copy of the pass flags, read back once per batch of passes
    int cc_passes = 0;              // passes of the last sta_components / sta_face_components
    int32_t* ccf_ws = nullptr;      // face connectivity: parent per tet, the pass flags, then the face pairs
    int2* ccf_pairs = nullptr;      // candidate tet pairs with a common face
    int64_t ccf_npairs = 0;
    // batch layout: per mesh node / tet / value offsets (k+1 entries)
    std::vector<int64_t> node_off, tet_off, nnz_off;
    // A batch rebuilt in groups of consecutive meshes (empty: in one pass): per group its tet
    // range, its diagonal block range and its off-diagonal block range, each [begin, end).
    std::vector<std::array<int64_t, 6>> rebuild_groups;
    std::string errmsg;
    // per-kernel event timing
    bool timing = false;
    struct TimedLaunch {
        int kernel;
        hipEvent_t a, b;
    };
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;
};

namespace sta {

// Per-kernel timing: while start is set, launch_kernel attaches the two
// events to the dispatch itself (hipExtLaunchKernel), so their interval is
// the kernel's execution, as a profiler reports it.  Thread-local.
struct KernelEvents {
    hipEvent_t start = nullptr, stop = nullptr;
    bool used = false;
};
KernelEvents& kernel_events();

template <typename... KArgs, typename... Args>
inline void launch_kernel(void (*k)(KArgs...), dim3 grid, dim3 block, uint32_t shmem, hipStream_t s, Args... args)
{
    KernelEvents& ev = kernel_events();
    if (ev.start) {
        ev.used = true;
        hipExtLaunchKernelGGL(k, grid, block, shmem, s, ev.start, ev.stop, 0u, static_cast<KArgs>(args)...);
    } else {
        hipLaunchKernelGGL(k, grid, block, shmem, s, static_cast<KArgs>(args)...);
    }
}

// Kernel launchers (assembly.hip).
hipError_t launch_element(const DevView& v, bool nt, hipStream_t s);
hipError_t launch_reduce_all(const DevView& v, const MapConfig& m, hipStream_t s);
// Streaming phases.  n_dev (device int32, may be NULL) overrides n_host, which
// then only sizes the grid (an upper bound on the edit count).
hipError_t launch_edit_phase(const DevView& v, const int32_t* ids, const uint8_t* states, int32_t n_host,
                             const int32_t* n_dev, hipStream_t s);
hipError_t launch_touched_phase(const DevView& v, const MapConfig& m, const int32_t* ids, int32_t n_host,
                                const int32_t* n_dev, hipStream_t s);
// +/- delta policy: one launch applying the edits' contributions with FP64
// atomics, one releasing the tet stamps.
hipError_t launch_delta_frame(const DevView& v, const int32_t* ids, const uint8_t* states, int32_t n_host,
                              const int32_t* n_dev, hipStream_t s);
// Fused frame: both phases in one persistent launch of `grid` co-resident workgroups.
hipError_t frame_max_grid(const MapConfig& m, int device, int* max_grid);
int frame_grid_for(const MapConfig& m, int32_t n_host, int max_grid, int grid_cap);
hipError_t launch_frame(const DevView& v, const MapConfig& m, int grid, const int32_t* ids, const uint8_t* states,
                        int32_t n_host, const int32_t* n_dev, unsigned spin_limit, hipStream_t s);
// Audit: counts[1] += tets whose stored contributions differ from the rebuild's,
// then the blocks re-summed from the stored contributions into scratch_values
// (nnz) and counts[0] += values differing from the maintained ones.
hipError_t launch_audit(const DevView& v, const MapConfig& m, double* scratch_values, int64_t nnz,
                        unsigned long long* counts, hipStream_t s);
// Release every tet and block stamp (a fill kernel, so that it can be captured).
hipError_t launch_clear_stamps(const DevView& v, hipStream_t s);
hipError_t launch_set_params(const DevView& v, const double* x_aos, const double* E, double* xs, double* ys,
                             double* zs, double* Eout, hipStream_t s);
// Copy the current coordinates and moduli into the tet records.
hipError_t launch_refresh_records(const DevView& v, TetRecord* trec, hipStream_t s);

// Adjoint and CG launchers (adjoint.hip, cg.hip).
// The adjoint visits the tets in chunks of kAdjointChunk consecutive ids, in
// an order fixed at context build (each mesh's chunks by the Morton code of
// their centroid), so that the chunks in flight together are near in space
// and their cotangent rows shared in cache.  Any order gives the same bits.
constexpr int kAdjointChunk = 16;
hipError_t launch_adjoint(const DevView& v, const int32_t* order, int32_t n_chunks, const double* gA, double* g_logE,
                          double* g_x, double* xbar, hipStream_t s);
hipError_t launch_slot_outer(int n_rows, const int32_t* rowptr, const int32_t* colidx, const double* a,
                             const double* b, double alpha, double* out, hipStream_t s);
hipError_t launch_diag_positions(const DevView& v, int32_t* dpos, hipStream_t s);
int cg_partials(int n);
int spmv_grid(int n);
int update_grid(int n);
hipError_t launch_cg_init(const CgView& c, const double* b, double rtol, hipStream_t s);
// Iterations first .. first+count-1 (the iteration index picks the copy of p).
hipError_t launch_cg_iterations(const CgView& c, int first, int count, int max_iter, hipStream_t s);
hipError_t launch_cg_output(const CgView& c, double* x, hipStream_t s);

// Lumped mass and implicit Euler (euler.hip).
hipError_t launch_tet_mass(const DevView& v, double* tet_ml, hipStream_t s);
hipError_t launch_lumped_mass(const DevView& v, const int32_t* dinc, const double* tet_ml, double* m, hipStream_t s);
hipError_t launch_euler_rhs(int n, const double* m, const double* u, const double* v, const double* f, double h,
                            double* b, hipStream_t s);
hipError_t launch_euler_update(int n, const double* u1, double* u, double* v, double h, hipStream_t s);

// Context construction shared by single and batched builds (api.hip).
sta_status build_context(const double* x, int64_t n_nodes, const int32_t* tets, int64_t n_tets, const double* E,
                         double nu, double rho, double dt, const uint8_t* mask0, void* stream,
                         const std::vector<int64_t>& node_off, const std::vector<int64_t>& tet_off, sta_ctx** out);
std::string& build_error();

// Host pattern builder (pattern.cpp).  Fills host arrays; returns "" or an error message.
struct HostPattern {
    int64_t nd = 0, no = 0, nnz = 0;
    std::vector<int32_t> rowptr, colidx;
    std::vector<int32_t> dseg, dinc, oseg, oinc;
    std::vector<int32_t> dmeta;  // 2 per block
    std::vector<int32_t> ometa;  // 4 per block
    std::vector<int32_t> opair;  // 2 per off-diagonal block: its nodes i < j
    std::vector<int32_t> e2b, e2p;  // 10 per element
    std::vector<int32_t> ndiag;     // per node: diagonal block id or -1
};
// bs: rows per node (3: elasticity, 1: scalar proxy operator).
std::string build_host_pattern(int64_t n_nodes, const int32_t* tets, int64_t n_tets, HostPattern& P, int bs = 3);

}  // namespace sta
