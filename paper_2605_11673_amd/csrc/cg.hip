// Jacobi-preconditioned conjugate gradients on the assembled CSR matrix (the
// paper's solve step: Sec. 4 and Alg. 1 solve A_t x_t = b_t by CG with a
// diagonal preconditioner).  Dofs whose diagonal is zero (nodes with no
// active tet: their rows and columns are all zero) are held at 0.
//
// All scalars stay on the device; each kernel returns at once when the
// solve has converged, so the host only synchronises every few iterations.
// Dot products use fixed reduction trees (a per-workgroup tree, then a sum
// over the workgroups' partials in index order): results are reproducible
// run to run.
//
// One iteration is two launches.  The matrix-vector product first sums the
// previous update's partials of r.z and r.r (every workgroup the same way,
// so all get the same bits), checks convergence, forms beta, and builds the
// new search direction p = z + beta p on the fly from a second copy of p.
// The update then sums the product's partials of p.Ap into alpha and
// updates x, r, z with partials of r.z and r.r.  The product works per node:
// the three rows of a node share one column list (3x3 blocks), so a group of
// lanes walks the node's neighbours once, reading one column index and one
// 3-vector of p per neighbour for all three rows.  Both grids are capped, so
// that the partials every workgroup sums stay few.
#include <hip/hip_runtime.h>

#include "sta_internal.h"

namespace sta {

namespace {

constexpr int kBlock = 256;
constexpr int kNodeLanes = 16;  // lanes per node (three CSR rows) in the matrix-vector product
#ifndef STA_CG_SPMV_GRID
#define STA_CG_SPMV_GRID 2048
#endif
#ifndef STA_CG_UPDATE_GRID
#define STA_CG_UPDATE_GRID 256
#endif
constexpr int kSpmvGridMax = STA_CG_SPMV_GRID;
constexpr int kUpdateGridMax = STA_CG_UPDATE_GRID;

// Workgroup sum of one value per thread, fixed tree; result valid in thread 0.
__device__ __forceinline__ double block_sum(double x, double* sh)
{
    sh[threadIdx.x] = x;
    __syncthreads();
#pragma unroll
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

// Sum of partials[0..n) by one workgroup: thread t adds t, t+256, ... in order, then a tree.
// Eight loads are issued before their additions (same order of additions).
__device__ __forceinline__ double reduce_partials(const double* __restrict__ p, int n, double* sh)
{
    double acc = 0.0;
    int i = threadIdx.x;
    for (; i + 7 * kBlock < n; i += 8 * kBlock) {
        double t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            t[k] = p[i + k * kBlock];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            acc = acc + t[k];
    }
    for (; i < n; i += kBlock)
        acc = acc + p[i];
    return block_sum(acc, sh);
}

// Workgroup sums of two values per thread, fixed trees; results valid in every thread.
__device__ __forceinline__ void block_sum2(double x, double y, double* sh, double& sx, double& sy)
{
    sh[threadIdx.x] = x;
    sh[kBlock + threadIdx.x] = y;
    __syncthreads();
#pragma unroll
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + s];
            sh[kBlock + threadIdx.x] = sh[kBlock + threadIdx.x] + sh[kBlock + threadIdx.x + s];
        }
        __syncthreads();
    }
    sx = sh[0];
    sy = sh[kBlock];
}

// Sums of p[0..n) and q[0..n) in one pass, each in the order of reduce_partials.
__device__ __forceinline__ void reduce_partials2(const double* __restrict__ p, const double* __restrict__ q, int n,
                                                 double* sh, double& sp, double& sq)
{
    double a = 0.0, b = 0.0;
    int i = threadIdx.x;
    for (; i + 7 * kBlock < n; i += 8 * kBlock) {
        double t[8], u[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            t[k] = p[i + k * kBlock];
            u[k] = q[i + k * kBlock];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            a = a + t[k];
            b = b + u[k];
        }
    }
    for (; i < n; i += kBlock) {
        a = a + p[i];
        b = b + q[i];
    }
    block_sum2(a, b, sh, sp, sq);
}

__global__ __launch_bounds__(kBlock) void k_cg_init(CgView c, const double* __restrict__ b)
{
    __shared__ double sh[kBlock];
    const int r = blockIdx.x * kBlock + threadIdx.x;
    double rz = 0.0, bb = 0.0;
    if (r < c.n) {
        const int pos = c.dpos[r];
        const double d = pos >= 0 ? c.vals[pos] : 0.0;
        const double di = d != 0.0 ? 1.0 / d : 0.0;
        const double br = d != 0.0 ? b[r] : 0.0;
        c.dinv[r] = di;
        c.x[r] = 0.0;
        c.r[r] = br;
        const double z = br * di;
        c.z[r] = z;
        c.p[r] = 0.0;  // p_0 = z_0 + 0 * 0, formed by the first product
        c.p[c.n + r] = 0.0;
        rz = br * z;
        bb = br * br;
    }
    const double s1 = block_sum(rz, sh);
    __syncthreads();
    const double s2 = block_sum(bb, sh);
    if (threadIdx.x == 0) {
        c.part[blockIdx.x] = s1;
        c.part[c.nparts + blockIdx.x] = s2;
    }
}

__global__ __launch_bounds__(kBlock) void k_cg_init_finish(CgView c, double rtol)
{
    __shared__ double sh[kBlock];
    const double rz = reduce_partials(c.part, c.nparts, sh);
    __syncthreads();
    const double bb = reduce_partials(c.part + c.nparts, c.nparts, sh);
    if (threadIdx.x == 0) {
        c.s->rz = rz;
        c.s->rzk[0] = rz;
        c.s->bnorm2 = bb;
        c.s->rr = bb;
        c.s->beta = 0.0;
        c.s->tol2 = (rtol * rtol) * bb;
        c.s->iters = 0;
        c.s->done = bb == 0.0 ? 1 : 0;
    }
}

// Iteration k, first launch.  For k > 0: r_k.z_k and r_k.r_k from the update's
// partials; stop if converged or k reaches max_iter; beta = (r_k.z_k) /
// (r_{k-1}.z_{k-1}).  Then p_new = z + beta p_old and q = A p_new, with the
// partials of p_new . q.  kNodeLanes lanes per node; lane l takes neighbours
// l, l + kNodeLanes, ...; the three row sums are combined by a fixed shuffle
// tree.  p_old is read, p_new written only for the node's own rows, so the two
// never alias.
__global__ __launch_bounds__(kBlock) void k_cg_spmv(CgView c, int k, int cur, int max_iter)
{
    __shared__ double sh[2 * kBlock];
    if (c.s->done)
        return;
    double beta = 0.0;
    {
        double rz = c.s->rzk[0], rr = c.s->rr;
        if (k > 0)
            reduce_partials2(c.part + c.nparts_s, c.part + c.nparts_s + c.nparts_u, c.nparts_u, sh, rz, rr);
        if ((k > 0 && rr <= c.s->tol2) || k >= max_iter) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                c.s->rr = rr;
                c.s->iters = k;
                c.s->done = 1;
            }
            return;
        }
        if (k > 0) {
            beta = rz / c.s->rzk[(k - 1) & 1];
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                c.s->rzk[k & 1] = rz;
                c.s->rr = rr;
                c.s->iters = k;
            }
        }
    }
    const double* __restrict__ pold = c.p + (cur ? c.n : 0);
    double* __restrict__ pnew = c.p + (cur ? 0 : c.n);
    const int nn = c.n / 3;
    const int group = threadIdx.x / kNodeLanes, l = threadIdx.x & (kNodeLanes - 1);
    constexpr int kGroups = kBlock / kNodeLanes;
    double pq = 0.0;
    // Node groups of kGroups nodes: with at least kXcds workgroups each XCD walks one
    // contiguous share of them (its workgroups in turn), so that neighbouring
    // nodes, which gather the same entries of z and p, stay in one L2 (29.8 ->
    // 28.3 us per iteration on the 207k-row fracture system); otherwise a plain
    // grid-stride.  All groups of a workgroup run the same number of rounds.
    const int ngroups = (nn + kGroups - 1) / kGroups;
    int g0 = blockIdx.x, g1 = ngroups, gstep = gridDim.x;
    if ((int)gridDim.x >= kXcds) {
        const int xcd = blockIdx.x % kXcds, G = gridDim.x;
        g0 = (int)((int64_t)ngroups * xcd / kXcds) + blockIdx.x / kXcds;
        g1 = (int)((int64_t)ngroups * (xcd + 1) / kXcds);
        gstep = G / kXcds + (xcd < G % kXcds ? 1 : 0);  // workgroups on this XCD
    }
    for (int gi = g0; gi < g1; gi += gstep) {
        const int i = gi * kGroups + group;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        if (i < nn) {
            const int base = c.rowptr[3 * i];
            const int rl = c.rowptr[3 * i + 1] - base;
            const int deg = rl / 3;
            for (int kk = l; kk < deg; kk += kNodeLanes) {
                const int j = c.colidx[base + 3 * kk] / 3;
                const double* v = c.vals + base + 3 * kk;
                double pj[3];
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    pj[q] = c.z[3 * j + q] + beta * pold[3 * j + q];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    a0 = a0 + v[q] * pj[q];
                    a1 = a1 + v[rl + q] * pj[q];
                    a2 = a2 + v[2 * rl + q] * pj[q];
                }
            }
        }
#pragma unroll
        for (int o = kNodeLanes / 2; o > 0; o >>= 1) {
            a0 = a0 + __shfl_xor(a0, o, kNodeLanes);
            a1 = a1 + __shfl_xor(a1, o, kNodeLanes);
            a2 = a2 + __shfl_xor(a2, o, kNodeLanes);
        }
        if (i < nn && l < 3) {
            const int r = 3 * i + l;
            const double acc = l == 0 ? a0 : (l == 1 ? a1 : a2);
            const double q = c.dinv[r] != 0.0 ? acc : 0.0;
            const double pr = c.z[r] + beta * pold[r];
            pnew[r] = pr;
            c.q[r] = q;
            pq = pq + pr * q;
        }
    }
    __syncthreads();  // sh is reused
    const double s = block_sum(pq, sh);
    if (threadIdx.x == 0)
        c.part[blockIdx.x] = s;
}

// Iteration k, second launch: alpha = (r_k.z_k) / (p.Ap) from the product's
// partials; x += alpha p_new, r -= alpha q, z = Dinv r; partials of r.z and r.r
// (grid-stride, each thread in ascending row order).  Each thread loads up to
// kUpdateRows of its rows before it updates any of them, so that their loads
// are in flight together (the vectors are distinct buffers, but the compiler
// cannot know it and would not hoist a row's loads above the previous row's
// stores): 29.8 instead of 31.5 us per iteration on the 207k-row fracture
// system, same bits.
constexpr int kUpdateRows = 4;
__global__ __launch_bounds__(kBlock) void k_cg_update(CgView c, int k, int cur)
{
    __shared__ double sh[2 * kBlock];
    if (c.s->done)
        return;
    const double pq = reduce_partials(c.part, c.nparts_s, sh);
    const double alpha = c.s->rzk[k & 1] / pq;
    const double* __restrict__ pnew = c.p + (cur ? 0 : c.n);
    double rz = 0.0, rr = 0.0;
    const int stride = gridDim.x * kBlock;
    for (int i0 = blockIdx.x * kBlock + threadIdx.x; i0 < c.n; i0 += kUpdateRows * stride) {
        double xs[kUpdateRows], ps[kUpdateRows], rs[kUpdateRows], qs[kUpdateRows], ds[kUpdateRows];
#pragma unroll
        for (int u = 0; u < kUpdateRows; ++u) {
            const int i = i0 + u * stride;
            const bool on = i < c.n;
            xs[u] = on ? c.x[i] : 0.0;
            ps[u] = on ? pnew[i] : 0.0;
            rs[u] = on ? c.r[i] : 0.0;
            qs[u] = on ? c.q[i] : 0.0;
            ds[u] = on ? c.dinv[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kUpdateRows; ++u) {
            const int i = i0 + u * stride;
            if (i < c.n) {
                c.x[i] = xs[u] + alpha * ps[u];
                const double r = rs[u] - alpha * qs[u];
                c.r[i] = r;
                const double z = r * ds[u];
                c.z[i] = z;
                rz = rz + r * z;
                rr = rr + r * r;
            }
        }
    }
    __syncthreads();  // sh is reused
    double s1, s2;
    block_sum2(rz, rr, sh, s1, s2);
    if (threadIdx.x == 0) {
        c.part[c.nparts_s + blockIdx.x] = s1;
        c.part[c.nparts_s + c.nparts_u + blockIdx.x] = s2;
    }
}

__global__ __launch_bounds__(kBlock) void k_cg_output(CgView c, double* __restrict__ x)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < c.n)
        x[i] = c.x[i];
}

// Position of each row's diagonal entry in the CSR values (-1: unused node).
__global__ __launch_bounds__(kBlock) void k_diag_positions(DevView v, int32_t* __restrict__ dpos)
{
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= 3 * v.n_nodes)
        return;
    const int i = r / 3, p = r - 3 * (r / 3);
    const int b = v.ndiag[i];
    dpos[r] = b >= 0 ? v.desc[b].up + p * v.desc[b].rl + p : -1;
}

inline unsigned blocks(int64_t n, int per)
{
    return (unsigned)((n + per - 1) / per);
}

}  // namespace

hipError_t launch_diag_positions(const DevView& v, int32_t* dpos, hipStream_t s)
{
    if (v.n_nodes == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_diag_positions, dim3(blocks(3 * (int64_t)v.n_nodes, kBlock)), dim3(kBlock), 0, s, v, dpos);
    return hipGetLastError();
}

// Matrix-vector product grid: one workgroup per 16 nodes, at most
// kSpmvGridMax; update grid: one per 256 rows, at most kUpdateGridMax.
int spmv_grid(int n)
{
    const int g = (int)blocks(n / 3, kBlock / kNodeLanes);
    return g < 1 ? 1 : (g > kSpmvGridMax ? kSpmvGridMax : g);
}

int update_grid(int n)
{
    const int g = (int)blocks(n, kBlock);
    return g < 1 ? 1 : (g > kUpdateGridMax ? kUpdateGridMax : g);
}

// Size of the partial-sum buffer: the start kernels' two halves, or the
// product's partials followed by the update's two halves.
int cg_partials(int n)
{
    const int a = 2 * (int)blocks(n, kBlock);
    const int b = spmv_grid(n) + 2 * update_grid(n);
    return a > b ? a : b;
}

hipError_t launch_cg_init(const CgView& c, const double* b, double rtol, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_init, dim3(blocks(c.n, kBlock)), dim3(kBlock), 0, s, c, b);
    hipLaunchKernelGGL(k_cg_init_finish, dim3(1), dim3(kBlock), 0, s, c, rtol);
    return hipGetLastError();
}

// Iterations first .. first+count-1 (the solve launches k = 0 .. max_iter;
// the product of k = max_iter only records the final residual).
hipError_t launch_cg_iterations(const CgView& c, int first, int count, int max_iter, hipStream_t s)
{
    for (int k = first; k < first + count; ++k) {
        const int cur = k & 1;  // which copy of p holds the previous direction
        hipLaunchKernelGGL(k_cg_spmv, dim3(c.nparts_s), dim3(kBlock), 0, s, c, k, cur, max_iter);
        hipLaunchKernelGGL(k_cg_update, dim3(c.nparts_u), dim3(kBlock), 0, s, c, k, cur);
    }
    return hipGetLastError();
}

hipError_t launch_cg_output(const CgView& c, double* x, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_output, dim3(blocks(c.n, kBlock)), dim3(kBlock), 0, s, c, x);
    return hipGetLastError();
}

}  // namespace sta
