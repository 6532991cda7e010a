/*
 * stafem.h -- C ABI of libstafem.so: exact streaming assembly of the implicit
 * system matrix A_t = M_t + dt^2 K_t over a preallocated superset tet mesh,
 * on one AMD MI355X (gfx950).
 *
 * The method (Acharya & Hyde, "STA-FEM: Exact Streaming Assembly for
 * Preplanned Dynamic Tetrahedral Topology Edits"):
 *   - Sec. 3.1 / Sec. 3.3: a fixed superset of vertices and candidate tets, an
 *     active mask over the candidates, and per-frame edit sets of deleted and
 *     added tets (eqs. (5), (6)).
 *   - Sec. 3.4 eq. (8): A_t = sum over active tets tau of P_tau^T A_tau P_tau,
 *     here with A_tau = dt^2 K_tau + M_tau (the implicit-Euler matrix of
 *     Sec. 6.2 eq. (9)), K_tau the 12x12 P1 linear-elasticity stiffness and
 *     M_tau the lumped mass, and eps = 0.
 *   - Sec. 3.3 invariant: after every frame the maintained matrix equals a
 *     rebuild from scratch on the current active set.  Here "equals" is
 *     bitwise in IEEE binary64: every entry is the sum of its active element
 *     terms in ascending element id starting from +0.0, whether it comes from
 *     sta_full_rebuild or from sta_apply_edits.
 *   - Sec. 3.5: full_rebuild and the streaming update are the policies; the
 *     streaming update touches only entries covered by edited tets.
 *
 * Matrix layout (values are owned by the context, in HBM):
 *   CSR over 3n rows, int32 indices.  Row 3i+p is displacement component p of
 *   node i.  Row 3i+p holds columns 3j+q for every node j that shares a
 *   candidate tet with i (j = i included), ascending.  The pattern is that of
 *   the whole superset and never changes; entries with no active incident tet
 *   hold +0.0.  A node in no candidate tet has empty rows.
 *
 * Element arithmetic (fixed so results are reproducible bit for bit): for a
 * tet with vertices x0..x3 in its given order, d_k = x_k - x_0,
 * c1 = d2 x d3, c2 = d3 x d1, c3 = d1 x d2, det = d1 . c1,
 * g_k = c_k * (1/det), g_0 = -((g_1 + g_2) + g_3), V = |det| / 6,
 * lamV = (E*cl*V)*dt^2, muV = (E*cm*V)*dt^2 with cl = nu/((1+nu)(1-2nu)),
 * cm = 0.5/(1+nu), m = (rho*V)*0.25, and
 *   A[3a+i][3b+j] = lamV*(g_ai*g_bj) + muV*(g_aj*g_bi) [+ muV*(g_a.g_b) if i=j]
 *                   [+ m if a=b and i=j],
 * each operation rounded once, left to right, no fused multiply-add.
 *
 * Streams: every call that takes `stream` (a hipStream_t, NULL = default
 * stream) only enqueues work on it and returns without waiting, unless
 * documented as synchronising.  Results are visible to later work on the
 * same stream.
 *
 * Errors: functions return a sta_status (0 = STA_OK, negative = error).
 * Host-checkable errors return before anything is modified.  Errors that
 * only the device can see (edit ids held in device memory) are recorded in
 * the context; the affected frame is rolled back (mask and values unchanged)
 * and sta_status_sync reports the error.  sta_last_error gives a message.
 * No function throws.
 *
 * Threading: a context may be used by one host thread at a time.  Calls on
 * one context must be ordered on one stream (or synchronised by the caller).
 */
#ifndef STAFEM_H
#define STAFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sta_ctx sta_ctx;
typedef int sta_status;

#define STA_OK 0
#define STA_EINVAL (-1)       /* bad argument (null pointer, size, material) */
#define STA_ENOMEM (-2)       /* device or host allocation failed (tests can force it: with the
                                 environment variable STA_FAIL_ALLOC_AT=k the k-th device
                                 allocation of the library fails; the call frees what it had
                                 allocated and changes nothing) */
#define STA_EHIP (-3)         /* a HIP runtime call failed */
#define STA_EDEGENERATE (-4)  /* a candidate tet has det == 0 or a repeated node */
#define STA_ESTALE (-5)       /* parameters changed; call sta_full_rebuild first */
#define STA_ERANGE (-6)       /* an edit id is outside [0, n_tets) or a state is not 0/1 */
#define STA_EDUP (-7)         /* an edit list names the same tet twice */
#define STA_ETIMEOUT (-8)     /* a fused frame could not synchronise its grid (GPU shared with
                                 other work); the frame is incomplete (the mask holds its edits)
                                 and frames are refused (STA_ESTALE) until sta_full_rebuild */

/* Build the superset pattern and the initial matrix (Sec. 3.1 inputs:
 * vertices, candidate pool, initial mask; Alg. 1 initialisation).
 *   x      host, n_nodes*3 float64, row-major (x, y, z per node)
 *   tets   host, n_tets*4 int32, vertex ids in [0, n_nodes), 4 distinct
 *   E      host, n_tets float64 Young's modulus per candidate
 *   nu, rho, dt  Poisson ratio in (-1, 0.5), density >= 0, time step > 0
 *   mask0  host, n_tets uint8 in {0, 1}
 * Inputs are copied; the caller keeps ownership.  Synchronises `stream`.
 * On success *out owns all device memory until sta_destroy; values hold
 * rebuild(mask0).  Element matrices are computed for every candidate here, so
 * later activations need no recomputation unless parameters change.
 * Errors: STA_EINVAL, STA_EDEGENERATE, STA_ENOMEM, STA_EHIP; *out = NULL. */
sta_status sta_build_pattern(const double* x, int64_t n_nodes, const int32_t* tets, int64_t n_tets,
                             const double* E, double nu, double rho, double dt,
                             const uint8_t* mask0, void* stream, sta_ctx** out);

/* Policy full_rebuild (Sec. 3.5): recompute the element matrices of every
 * active tet and re-sum every entry of A from the current mask.  Clears
 * STA_ESTALE.  After fused frames (sta_set_config fused = 1) it also releases
 * every edit stamp, which a frame whose grid barrier gave up may have left
 * taken.  Asynchronous on `stream`. */
sta_status sta_full_rebuild(sta_ctx* ctx, void* stream);

/* Streaming update for one frame (Sec. 3.2, Alg. 1): edit k sets tet
 * ids_dev[k] to state states_dev[k] (1 = add, eq. (6); 0 = delete, eq. (5)).
 *   ids_dev     device, n_edits int32
 *   states_dev  device, n_edits uint8
 * Ids must be distinct within one call (the edits are sets); an edit to the
 * state a tet already has is allowed and changes nothing.  Only entries
 * covered by tets whose state changed are recomputed, each from its
 * incidence list in ascending element id, so the result is bitwise equal to
 * sta_full_rebuild on the new mask.  Asynchronous on `stream`; the edit
 * arrays must stay valid until the work completes.  Bad ids / states /
 * duplicates found on the device roll the whole frame back and are reported
 * by sta_status_sync.  Host errors: STA_EINVAL (n_edits < 0 or > n_tets),
 * STA_ESTALE (parameters changed without a rebuild). */
sta_status sta_apply_edits(sta_ctx* ctx, const int32_t* ids_dev, const uint8_t* states_dev,
                           int64_t n_edits, void* stream);

/* The paper's +/- delta policy for element assembly (Sec. 3.4, Sec. 3.5
 * streaming_update): each changed tet's local contributions are added to
 * (activation) or subtracted from (deletion) the touched entries directly,
 * with FP64 atomics, and nothing is re-summed.  Faster per touched entry
 * than sta_apply_edits, but the result depends on the order in which
 * concurrent edits land: it equals the rebuild only up to rounding, and the
 * difference can grow over many frames (drift).  The mask and per-element
 * contributions are kept as sta_apply_edits expects, so the exact policy or
 * sta_full_rebuild may follow at any time (a rebuild removes the drift).
 * Arguments as sta_apply_edits; if n_dev (device int32) is not NULL the edit
 * count is *n_dev and n_edits is the arrays' capacity (graph-capturable).
 * Invalid or duplicate edits are skipped (not rolled back) and reported by
 * sta_status_sync.  Host errors: STA_EINVAL, STA_ESTALE. */
sta_status sta_apply_edits_delta(sta_ctx* ctx, const int32_t* ids_dev, const uint8_t* states_dev, int64_t n_edits,
                                 const int32_t* n_dev, void* stream);

/* sta_apply_edits with the edit count read on the device: *n_dev (device
 * int32) edits are taken from ids_dev / states_dev, whose allocations hold
 * `capacity` entries (1 <= capacity <= n_tets).  Nothing on the host depends
 * on the count, so the call can be captured once into a HIP graph and the
 * graph replayed with new edit lists written into the same buffers.
 * *n_dev outside [0, capacity] is reported as STA_ERANGE by sta_status_sync
 * and the frame is skipped. */
sta_status sta_apply_edits_dev(sta_ctx* ctx, const int32_t* ids_dev, const uint8_t* states_dev,
                               const int32_t* n_dev, int64_t capacity, void* stream);

/* The maintained matrix A_t of Sec. 3.3 (the operator the streaming update
 * keeps equal to a rebuild from the current mask after every frame of
 * Alg. 1): device pointer to its nnz CSR values in the pattern of
 * sta_pattern_ptrs.  Borrowed: valid until sta_destroy and updated in place
 * by sta_full_rebuild / sta_apply_edits*; order reads after the producing work
 * on the stream.  NULL for a NULL context. */
const double* sta_values_ptr(const sta_ctx* ctx);

/* Copy the nnz values into a caller-owned device buffer (stream-ordered). */
sta_status sta_copy_values(const sta_ctx* ctx, double* dst_dev, void* stream);

/* Sizes: rows = 3*n_nodes, nnz, diagonal / off-diagonal 3x3 node blocks. */
sta_status sta_sizes(const sta_ctx* ctx, int64_t* n_rows, int64_t* nnz, int64_t* n_diag_blocks,
                     int64_t* n_off_blocks);

/* The fixed superset pattern (Sec. 3.1: every node pair that shares a
 * candidate tet, whatever the mask) and the active mask a_t of Sec. 3.1:
 * device pointers to the CSR row pointer (n_rows+1) and column index (nnz)
 * arrays, and to the mask (n_tets uint8).  Borrowed, valid until
 * sta_destroy; the pattern never changes, the mask is updated in place by
 * every frame. */
sta_status sta_pattern_ptrs(const sta_ctx* ctx, const int32_t** rowptr_dev, const int32_t** colidx_dev,
                            const uint8_t** mask_dev);

/* The same superset pattern copied to host arrays of n_rows+1 and nnz int32.
 * Synchronous. */
sta_status sta_pattern_host(const sta_ctx* ctx, int32_t* rowptr, int32_t* colidx);

/* Statistics of the last sta_apply_edits, written to out[0 .. n_out-1]:
 *   [0] diagonal 3x3 blocks recomputed   [1] off-diagonal blocks recomputed
 *   [2] incidences read for [0]          [3] incidences read for [1]
 *   [4] matrix slots written (both triangles)
 *   [5] tets whose state changed         [6] of those, tets activated
 *   [7] edits in the list                [8] 1 if the frame was rolled back
 * Synchronises `stream`. */
#define STA_NUM_FRAME_STATS 9
sta_status sta_last_frame_stats(sta_ctx* ctx, void* stream, int64_t* out, int n_out);

/* Per-kernel timing (tracing aid).  While enabled, every kernel this context
 * launches is timed by two HIP events on the launch stream: attached to the
 * dispatch itself for the single-kernel ids (element, reduce, edits,
 * touched, frame: the kernel's execution time, as a profiler reports it),
 * recorded around the launches for the others (adjoint, solve, delta).
 * sta_kernel_times synchronises `stream`, writes per kernel id the number of
 * launches and their summed event-to-event duration in milliseconds (arrays
 * of STA_NUM_KERNELS), and resets the counters. */
/* Per-call trace: when the environment variable STA_TRACE names a file at
 * context build, every sta_full_rebuild and sta_apply_edits* call on the
 * context appends one JSON line to it (a sequence number, the call, its edit
 * count or capacity, the frame mode and the host time since the build, in
 * microseconds), flushed at once.  With STA_TRACE_STATS=1 as well, each frame
 * call synchronises its stream and adds the frame's statistics (the nine
 * values of sta_last_frame_stats).  The file is closed by sta_destroy.  A
 * file that cannot be opened for appending fails the build with STA_EINVAL. */
#define STA_KERNEL_ELEMENT 0   /* element contributions (rebuild / activation) */
#define STA_KERNEL_REDUCE 1    /* re-sum of every block (rebuild) */
/* A batch whose contributions exceed 200 MB is rebuilt in groups of
 * consecutive meshes: each group counts one STA_KERNEL_ELEMENT launch and two
 * STA_KERNEL_REDUCE launches (diagonal, then off-diagonal blocks). */
#define STA_KERNEL_EDITS 2     /* streaming phase 1: validate, flip, claim */
#define STA_KERNEL_TOUCHED 3   /* streaming phase 2: re-sum claimed blocks */
#define STA_KERNEL_ADJOINT 4
#define STA_KERNEL_SOLVE 5     /* all kernels of one CG solve */
#define STA_KERNEL_FRAME 6     /* fused frame: both streaming phases in one launch */
#define STA_KERNEL_DELTA 7     /* +/- delta frame (sta_apply_edits_delta), both launches */
#define STA_NUM_KERNELS 8
sta_status sta_enable_kernel_timing(sta_ctx* ctx, int on);
sta_status sta_kernel_times(sta_ctx* ctx, void* stream, int64_t* launches, double* ms);

/* Replace node positions (device, n_nodes*3 float64 row-major) and Young's
 * moduli (device, n_tets float64); either may be NULL to keep the current
 * one.  The matrix is then stale: sta_apply_edits returns STA_ESTALE until
 * sta_full_rebuild.  Asynchronous on `stream`. */
sta_status sta_set_params(sta_ctx* ctx, const double* x_dev, const double* E_dev, void* stream);

/* Adjoint of the assembly (the differentiable-assembly extension; the paper
 * itself maintains A_t only): given gA_dev = dL/dvalues (device, nnz), write
 * g_logE_dev[e] = dL/dlog(E_e) (device, n_tets; 0 for inactive tets) and
 * g_x_dev[3i+k] = dL/dx_{i,k} (device, n_nodes*3) for the current mask and
 * parameters, by reverse differentiation of the element formula above.
 * Per-node sums run over the node's tets in ascending id (reproducible).
 * Asynchronous on `stream`.  STA_ESTALE after sta_set_params until a rebuild. */
sta_status sta_adjoint(sta_ctx* ctx, const double* gA_dev, double* g_logE_dev, double* g_x_dev, void* stream);

/* sta_adjoint for callers that cannot allocate device memory (code being
 * captured into a HIP graph, serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same results, bit for bit, but the per-vertex
 * cotangent workspace (12 doubles per tet) is a fixed 48 MiB array inside the
 * library, one per GPU, held until the process ends, instead of a buffer the
 * context allocates on first use.  Arguments and results as sta_adjoint.
 * Contexts of more than 524,288 tets are refused with STA_EINVAL (use
 * sta_adjoint).  The current device must be the context's device.  The
 * array is shared by every call on one GPU and keeps the last call's
 * contents (each call overwrites all it reads): calls that may overlap on
 * one GPU (other streams, other host threads) race and must be serialised
 * by the caller.  No allocation and no synchronisation; asynchronous on
 * `stream`.  STA_ESTALE after sta_set_params until a rebuild. */
sta_status sta_adjoint_noalloc(sta_ctx* ctx, const double* gA_dev, double* g_logE_dev, double* g_x_dev,
                               void* stream);

/* out_dev[s] = alpha * a_dev[row(s)] * b_dev[col(s)] for every pattern slot s
 * (e.g. the cotangent -lambda u^T of the values behind a linear solve).
 * a_dev, b_dev: device, n_rows; out_dev: device, nnz.  Asynchronous. */
sta_status sta_slot_outer(sta_ctx* ctx, const double* a_dev, const double* b_dev, double alpha, double* out_dev,
                          void* stream);

/* Jacobi-preconditioned CG (Sec. 4; Alg. 1 solve step) on A x = b with the
 * matrix values_dev (device, nnz, this context's pattern; NULL = the
 * context's own values).  Rows with a zero diagonal (nodes with no active
 * tet) are held at x = 0 and their b is ignored.  Stops when
 * ||r|| <= rtol ||b|| or after max_iter iterations.  b_dev, x_dev: device,
 * n_rows.  Synchronises `stream` (convergence is checked every 16
 * iterations).  *iters_out / *relres_out (may be NULL) report the result. */
sta_status sta_cg_solve(sta_ctx* ctx, const double* values_dev, const double* b_dev, double* x_dev, double rtol,
                        int max_iter, void* stream, int* iters_out, double* relres_out);

/* Lumped mass M_t of the current mask (the maintained mass of Sec. 6.2
 * eq. (9)): m_dev[3i+k] (device, n_rows) = sum over the active tets of node
 * i, in ascending tet id from +0.0, of (rho V) / 4, V = |det| / 6 as in the
 * element formula; equal bit for bit to the diagonal of A_t when E = 0.
 * Asynchronous. */
sta_status sta_lumped_mass(sta_ctx* ctx, double* m_dev, void* stream);

/* One implicit-Euler step (Sec. 6.2 eq. (9)) with h = the context's dt and
 * the current A_t = M_t + h^2 K_t:
 *   solve A_t u' = M_t (u + h v) + h^2 f by Jacobi-PCG (as sta_cg_solve,
 *   from u' = 0, relative residual rtol, at most max_iter iterations),
 *   then v := (u' - u) / h and u := u'.
 * u_dev, v_dev (device, n_rows, updated in place), f_dev (device, n_rows,
 * a fixed external load).  Dofs of nodes with no active tet get u' = 0.
 * Synchronises `stream` (the solver checks convergence on the host).
 * Errors: STA_EINVAL, STA_ESTALE, STA_ENOMEM, STA_EHIP. */
sta_status sta_euler_step(sta_ctx* ctx, double* u_dev, double* v_dev, const double* f_dev, double rtol,
                          int max_iter, void* stream, int* iters_out, double* relres_out);

/* Connectivity of the active tets (Sec. 3.6, Alg. 1: union-find rebuilt from
 * the current mask).  Two active tets are connected when they share a vertex
 * (the components of the assembled operator).  labels_dev (device, n_tets
 * int32) receives, per tet, its component's smallest vertex id, or -1 for an
 * inactive tet; labels do not depend on execution order.  *n_components
 * (may be NULL) receives the number of components.  Synchronises `stream`
 * (the host reads the convergence flags and the count once per batch of
 * passes, normally once per call). */
sta_status sta_components(sta_ctx* ctx, int32_t* labels_dev, int64_t* n_components, void* stream);

/* Connectivity over shared faces (Sec. 3.6 leaves the adjacency open; this
 * is the fragment notion of fracture): two active tets are connected when
 * they have three vertices in common, so pieces touching only along an edge
 * or at a vertex are apart, and a hanging-node interface of a refinement
 * superset separates.  labels_dev (device, n_tets int32) receives, per tet,
 * its component's smallest tet id, or -1 for an inactive tet;
 * *n_components (may be NULL) the number of components.  The candidate
 * pairs with a common face are found on the first call (a host sort of the
 * 4 n_tets vertex triples) and kept on the device with the context (8 B per
 * pair, 4 B per tet).  Synchronises `stream`.  Errors: STA_EINVAL,
 * STA_ENOMEM, STA_EHIP. */
sta_status sta_face_components(sta_ctx* ctx, int32_t* labels_dev, int64_t* n_components, void* stream);

/* Execution configuration.
 *   fused       0: a frame is two launches (edit phase, touched phase);
 *               1: one persistent launch (both phases, grid barrier between).
 *   rebuild_qd / rebuild_qo, stream_qd / stream_qo: slot mapping, i.e. lanes
 *               cooperating on one block value for diagonal / off-diagonal
 *               blocks in the rebuild and in the streaming update
 *               (diagonal: 1 = thread-, 4 = quad-, 16 = wave-sixteenth-per-slot;
 *               off-diagonal: 1 or 4), here for every incidence-length
 *               bucket alike (see sta_set_bucket_map).  Every mapping adds the
 *               same terms in the same order: results are bit-identical.
 *   grid_cap    upper bound on the fused kernel's workgroups (0 = the
 *               co-resident limit).
 *   rebuild_nt  1: the rebuild streams contributions and values with
 *               non-temporal cache hints (each byte is touched once).
 * sta_get_config writes the same 7 integers.  Defaults: 0, 1, 1, 1, 1, 0, 0. */
sta_status sta_set_config(sta_ctx* ctx, int fused, int rebuild_qd, int rebuild_qo, int stream_qd, int stream_qo,
                          int grid_cap, int rebuild_nt);
sta_status sta_get_config(const sta_ctx* ctx, int* out7);

/* Audit of the maintained state against the Sec. 3.3 invariant (the
 * maintained matrix equals a rebuild from the mask), without changing it:
 * out2[1] = tets whose 78 stored contribution slots differ in any bit from
 * what a rebuild would store (the element matrix of an active tet, +0.0 for
 * an inactive one); out2[0] = matrix values differing in any bit from a
 * re-sum of the stored contributions into a scratch copy (nnz doubles,
 * allocated on first use).  Both 0 for an intact context.  Synchronises
 * `stream`.  STA_ESTALE after sta_set_params until a rebuild. */
sta_status sta_audit(sta_ctx* ctx, void* stream, int64_t* out2);

/* Failure injection for the fused frame (tests of STA_ETIMEOUT): the grid
 * barrier between the two phases gives up after `polls` polls of its
 * release word (0 restores the default, 2^24, far beyond any co-resident
 * grid's wait).  A small value makes workgroups that arrive early give up
 * and leave; the device records STA_ETIMEOUT for sta_status_sync.
 * STA_EINVAL for polls < 0 or >= 2^32. */
sta_status sta_set_barrier_spin_limit(sta_ctx* ctx, int64_t polls);

/* Slot mapping per incidence-length bucket.  A block's incidence length
 * kappa is the number of candidate tets in its segment (paper Sec. 3.3:
 * the per-block work of a local recompute, O(|Delta| kappa) in Prop. 1).
 * Diagonal blocks fall in bucket 0 (kappa <= 8), 1 (9..32) or 2 (> 32);
 * off-diagonal blocks in bucket 0 (kappa <= 8) or 1 (> 8).  qd3[b] in
 * {1, 4, 16} and qo2[b] in {1, 4} give the lanes per value for each bucket;
 * which = 0 sets the rebuild's mapping, 1 the streaming update's.  The
 * kernels allocate the largest group per block and a block of a bucket with
 * a smaller group leaves the rest idle, so a mixed mapping trades idle lanes
 * for load depth where segment lengths differ; sta_autotune chooses it by
 * timing.  sta_set_config resets every bucket to one mapping.  Results are
 * bit-identical for every mapping.  sta_get_config reports the allocation
 * (the largest group).  STA_EINVAL on a value outside the sets above. */
sta_status sta_set_bucket_map(sta_ctx* ctx, int which, const int* qd3, const int* qo2);

/* The mapping per bucket (qd3, qo2; either may be NULL) and the number of
 * blocks in each bucket (blocks5: 3 diagonal then 2 off-diagonal counts;
 * may be NULL). */
sta_status sta_get_bucket_map(const sta_ctx* ctx, int which, int* qd3, int* qo2, int64_t* blocks5);

/* Autotuner: times every slot mapping for the full rebuild, and every
 * mapping x {two launches, fused with grid caps} for one streaming frame
 * (ids_dev / states_dev, device, n_edits; each timed application is undone
 * before the next), keeps the fastest of each, then, for every non-empty
 * incidence-length bucket in turn, tries each group size for that bucket
 * alone (sta_set_bucket_map) and keeps it where it is faster, and returns a
 * text report in report (may be NULL).  If the environment variable STA_TUNE_CACHE names a
 * file, a previous result for the same mesh sizes and frame size is reused
 * from it and new results are appended.  Synchronises `stream`. */
sta_status sta_autotune(sta_ctx* ctx, const int32_t* ids_dev, const uint8_t* states_dev, int64_t n_edits,
                        int reps, void* stream, char* report, int64_t report_len);

/* Batched build: k independent meshes become one context whose node, tet,
 * row and value ranges are the meshes' own, concatenated in order (mesh j's
 * tet t is global tet tet_off[j] + t).  Arguments as for sta_build_pattern,
 * per mesh (arrays of k host pointers and sizes); nu, rho, dt shared.  A
 * frame over all meshes is one sta_apply_edits / sta_apply_edits_dev call
 * with global tet ids; with fused = 1 it is one launch, and with
 * sta_apply_edits_dev it can be captured once into a HIP graph. */
sta_status sta_batch_build(int k, const double* const* x, const int64_t* n_nodes, const int32_t* const* tets,
                           const int64_t* n_tets, const double* const* E, double nu, double rho, double dt,
                           const uint8_t* const* mask0, void* stream, sta_ctx** out);

/* Per-mesh offsets of a batched context (k+1 entries each: node, tet, CSR
 * row and value offsets; entry k is the total).  A context from
 * sta_build_pattern is a batch of one. */
sta_status sta_batch_offsets(const sta_ctx* ctx, int* k, int64_t* node_off, int64_t* tet_off, int64_t* row_off,
                             int64_t* nnz_off, int64_t capacity);

/* Latency floor of this GPU (no context needed; allocates ~257 MB
 * temporarily; synchronises `stream`): out4[0] = microseconds per empty
 * kernel launched back to back on one stream, out4[1] = nanoseconds per
 * dependent global load over a 256 MB working set, out4[2] = the same over
 * an L2-resident 1 MB set, out4[3] = nanoseconds per dependent returning
 * device-scope atomic.  A streaming frame is two launches with a few
 * dependent round trips each, so these numbers bound its latency. */
sta_status sta_latency_probe(void* stream, double* out4);

/* Measured streaming bandwidth of this GPU's HBM, in GB/s (1e9 B/s), on
 * `stream`: out3[0] reading 1 GiB, out3[1] writing 1 GiB, out3[2] copying
 * 1 GiB (2 GiB moved), 16-byte accesses by consecutive lanes in a
 * grid-stride loop; each kind is timed over ten launches after one warm-up at
 * grids of 1,024, 4,096, 16,384 and 65,536 workgroups of 256 lanes, and the
 * best grid is reported (writes are fastest with many short-lived
 * workgroups, reads and copies with few).  Allocates and frees 2 GiB of
 * device memory; synchronises `stream`.  The achieved fractions of the rebuild
 * kernels are reported against the published 8 TB/s peak; these numbers
 * say what a plain streaming kernel reaches on the same device. */
sta_status sta_bandwidth_probe(void* stream, double* out3);

/* Cost of a grid barrier against a kernel boundary on this GPU (no context
 * needed; creates its own stream, allocates a few bytes, synchronises):
 * microseconds per unit with each unit captured 50 times into a HIP graph
 * and the graph replayed, out7[0] = one empty kernel, out7[1] = two empty
 * kernels (the boundary a two-launch frame pays), out7[2..6] = one kernel of
 * 8, 32, 64, 128, 256 workgroups that does nothing but the fused frame's grid
 * barrier (-1 where that grid would not be co-resident).  STA_ETIMEOUT if a
 * barrier gave up. */
sta_status sta_barrier_probe(double* out7);

/* Synchronise `stream`, return and clear the first error the device
 * recorded (STA_ETIMEOUT, STA_ERANGE, STA_EDUP, STA_EDEGENERATE), else
 * STA_OK.  On STA_ETIMEOUT it also releases every edit stamp and marks the
 * context stale, so that sta_apply_edits returns STA_ESTALE until
 * sta_full_rebuild re-sums the matrix from the mask. */
sta_status sta_status_sync(sta_ctx* ctx, void* stream);

/* Message for the last error on this context (or of the last failed
 * sta_build_pattern when ctx is NULL).  Never NULL. */
const char* sta_last_error(const sta_ctx* ctx);

/* Free everything the context owns.  NULL is ignored. */
void sta_destroy(sta_ctx* ctx);

/* ------------------------------------------------------------------------
 * Graph-Laplacian proxy operator (Sec. 3.1 eqs. (1)-(4), Sec. 3.2 eq. (7),
 * Sec. 3.3 maintained state, Alg. 1), on its own context.
 *
 *   c_t(u,v) = number of active tets with edge (u,v)          (eq. (1))
 *   a_t(u,v) = 1 if c_t(u,v) > 0 else 0                        (eq. (2))
 *   A_t      = L_t + eps I: off-diagonal -a_t(u,v), diagonal the number of
 *              active edges at u, plus eps                     (eqs. (3), (4))
 *
 * Layout: scalar CSR over n rows, int32 indices; row u holds the diagonal
 * and one entry per superset edge at u (columns ascending), for every
 * vertex in some candidate tet (other rows are empty).  The pattern never
 * changes: an inactive edge's two entries hold +0.0, an active one's -1.0;
 * a diagonal holds float64(degree) + eps.  Edges are numbered in ascending
 * (u, v), u < v.  Counts and degrees are maintained as int32 with the +1/-1
 * deltas of eq. (7); values are rewritten from them, so every frame leaves
 * the state exactly equal to sta_proxy_full_rebuild on the same mask.
 * Stream, error and threading rules as above.
 * ------------------------------------------------------------------------ */
typedef struct sta_proxy sta_proxy;

/* Build the scalar superset pattern, the edge incidence and A_0 (Alg. 1
 * initialisation).  tets host n_tets*4 int32 (4 distinct ids in
 * [0, n_nodes)), mask0 host n_tets uint8 in {0, 1}, eps finite >= 0.
 * Inputs are copied.  Synchronises `stream`.  Errors: STA_EINVAL,
 * STA_EDEGENERATE (repeated vertex), STA_ENOMEM, STA_EHIP; *out = NULL. */
sta_status sta_proxy_build(const int32_t* tets, int64_t n_nodes, int64_t n_tets, const uint8_t* mask0, double eps,
                           void* stream, sta_proxy** out);

/* Policy full_rebuild (Sec. 3.5): counts from the mask over each edge's
 * incidence list, then degrees and every value.  Asynchronous. */
sta_status sta_proxy_full_rebuild(sta_proxy* p, void* stream);

/* One frame of Alg. 1: edit k sets tet ids_dev[k] to states_dev[k] (device
 * int32 / uint8, n_edits of each, ids distinct).  Each changed tet adds +1
 * (activation) or -1 (deletion) to its six edge counts; a count moving
 * between 0 and > 0 inserts or removes the edge's two entries and moves both
 * endpoint degrees; then the entries and diagonals of changed tets are
 * rewritten.  Asynchronous.  Bad ids / states / duplicates found on the
 * device roll the frame back (sta_proxy_status_sync reports them).  Host
 * errors: STA_EINVAL. */
sta_status sta_proxy_apply_edits(sta_proxy* p, const int32_t* ids_dev, const uint8_t* states_dev, int64_t n_edits,
                                 void* stream);

/* As sta_proxy_apply_edits with the edit count read from *n_dev (device
 * int32) and the arrays holding `capacity` entries (1 <= capacity <=
 * n_tets): graph-capturable.  *n_dev outside [0, capacity] is STA_ERANGE. */
sta_status sta_proxy_apply_edits_dev(sta_proxy* p, const int32_t* ids_dev, const uint8_t* states_dev,
                                     int64_t capacity, const int32_t* n_dev, void* stream);

/* n_rows (= n_nodes), nnz and the number of superset edges (any may be NULL). */
sta_status sta_proxy_sizes(const sta_proxy* p, int64_t* n_rows, int64_t* nnz, int64_t* n_edges);

/* Borrowed device pointers, valid until sta_proxy_destroy: the nnz values,
 * c_t per edge (int32), the degree per vertex (int32). */
const double* sta_proxy_values_ptr(const sta_proxy* p);
const int32_t* sta_proxy_counts_ptr(const sta_proxy* p);
const int32_t* sta_proxy_degree_ptr(const sta_proxy* p);

/* Stream-ordered device-to-device copies of the current state into caller
 * buffers (any may be NULL): values (nnz float64), counts (n_edges int32),
 * degree (n_rows int32). */
sta_status sta_proxy_copy_state(const sta_proxy* p, double* values, int32_t* counts, int32_t* degree, void* stream);

/* Borrowed device pointers to the CSR (rowptr n+1, colidx nnz) and the edge
 * list (2 int32 per edge: u < v). */
sta_status sta_proxy_pattern_ptrs(const sta_proxy* p, const int32_t** rowptr, const int32_t** colidx,
                                  const int32_t** edges);

/* Host copies of the same (synchronous): rowptr n_rows+1, colidx nnz,
 * edges 2*n_edges int32. */
sta_status sta_proxy_pattern_host(const sta_proxy* p, int32_t* rowptr, int32_t* colidx, int32_t* edges);

/* Synchronises `stream`; out3 = {edit count of the last frame, edits that
 * changed a tet's state, edge transitions between 0 and > 0} (0, 0 if the
 * frame was rolled back). */
sta_status sta_proxy_last_frame_stats(sta_proxy* p, void* stream, int64_t* out3);

/* Synchronise `stream`, return and clear the device-recorded error
 * (STA_ERANGE, STA_EDUP), else STA_OK. */
sta_status sta_proxy_status_sync(sta_proxy* p, void* stream);

/* Message for the last error on p (or of the last failed sta_proxy_build
 * when p is NULL).  Never NULL. */
const char* sta_proxy_last_error(const sta_proxy* p);

/* Free everything p owns.  NULL is ignored. */
void sta_proxy_destroy(sta_proxy* p);

#ifdef __cplusplus
}
#endif

#endif /* STAFEM_H */
