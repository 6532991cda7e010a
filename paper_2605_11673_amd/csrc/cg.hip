// Jacobi-preconditioned conjugate gradients on the assembled CSR matrix (the
// paper's solve step: Sec. 4 and Alg. 1 solve A_t x_t = b_t by CG with a
// diagonal preconditioner).  Dofs whose diagonal is zero (nodes with no
// active tet: their rows and columns are all zero) are held at 0.
//
// All scalars stay on the device; each kernel returns at once when the
// solve has converged, so the host only synchronises every few iterations.
// Dot products use a fixed reduction tree (per-workgroup tree, then one
// workgroup over the partials in index order): results are reproducible
// run to run.
//
// One iteration is four launches: the matrix-vector product (which also
// forms the new search direction p = z + beta p on the fly, from a second
// copy of p, so no separate direction pass is needed), alpha, the x / r / z
// update, beta.  The product works per node: the three rows of a node share
// one column list (3x3 blocks), so a group of lanes walks the node's
// neighbours once, reading one column index and one 3-vector of p per
// neighbour for all three rows.
#include <hip/hip_runtime.h>

#include "sta_internal.h"

namespace sta {

namespace {

constexpr int kBlock = 256;
constexpr int kNodeLanes = 16;  // lanes per node (three CSR rows) in the matrix-vector product

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
        c.s->bnorm2 = bb;
        c.s->rr = bb;
        c.s->beta = 0.0;
        c.s->tol2 = (rtol * rtol) * bb;
        c.s->iters = 0;
        c.s->done = bb == 0.0 ? 1 : 0;
    }
}

// p_new = z + beta p_old and q = A p_new, partial p_new . q.  kNodeLanes
// lanes per node; lane l takes neighbours l, l + kNodeLanes, ...; the three
// row sums are then combined by a fixed shuffle tree.  p_old is read, p_new
// written only for the node's own rows, so the two never alias.
__global__ __launch_bounds__(kBlock) void k_cg_spmv(CgView c, int cur)
{
    __shared__ double sh[kBlock];
    if (c.s->done)
        return;
    const double beta = c.s->beta;
    const double* __restrict__ pold = c.p + (cur ? c.n : 0);
    double* __restrict__ pnew = c.p + (cur ? 0 : c.n);
    const int nn = c.n / 3;
    const int group = threadIdx.x / kNodeLanes, l = threadIdx.x & (kNodeLanes - 1);
    constexpr int kGroups = kBlock / kNodeLanes;
    double pq = 0.0;
    // grid-stride over nodes (the grid is capped, which bounds the partials
    // alpha adds); every group of a workgroup runs the same number of rounds
    for (int base_node = blockIdx.x * kGroups; base_node < nn; base_node += gridDim.x * kGroups) {
        const int i = base_node + group;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        if (i < nn) {
            const int base = c.rowptr[3 * i];
            const int rl = c.rowptr[3 * i + 1] - base;
            const int deg = rl / 3;
            for (int k = l; k < deg; k += kNodeLanes) {
                const int j = c.colidx[base + 3 * k] / 3;
                const double* v = c.vals + base + 3 * k;
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
    const double s = block_sum(pq, sh);
    if (threadIdx.x == 0)
        c.part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_cg_alpha(CgView c, int nparts)
{
    __shared__ double sh[kBlock];
    if (c.s->done)
        return;
    const double pq = reduce_partials(c.part, nparts, sh);
    if (threadIdx.x == 0)
        c.s->alpha = c.s->rz / pq;
}

// x += alpha p_new, r -= alpha q, z = Dinv r; partial r.z and r.r
__global__ __launch_bounds__(kBlock) void k_cg_update(CgView c, int cur)
{
    __shared__ double sh[kBlock];
    if (c.s->done)
        return;
    const double alpha = c.s->alpha;
    const double* __restrict__ pnew = c.p + (cur ? 0 : c.n);
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (i < c.n) {
        c.x[i] = c.x[i] + alpha * pnew[i];
        const double r = c.r[i] - alpha * c.q[i];
        c.r[i] = r;
        const double z = r * c.dinv[i];
        c.z[i] = z;
        rz = r * z;
        rr = r * r;
    }
    const double s1 = block_sum(rz, sh);
    __syncthreads();
    const double s2 = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        c.part[blockIdx.x] = s1;
        c.part[c.nparts + blockIdx.x] = s2;
    }
}

__global__ __launch_bounds__(kBlock) void k_cg_beta(CgView c, int max_iter)
{
    __shared__ double sh[kBlock];
    if (c.s->done)
        return;
    const double rz = reduce_partials(c.part, c.nparts, sh);
    __syncthreads();
    const double rr = reduce_partials(c.part + c.nparts, c.nparts, sh);
    if (threadIdx.x == 0) {
        c.s->beta = rz / c.s->rz;
        c.s->rz = rz;
        c.s->rr = rr;
        c.s->iters += 1;
        if (rr <= c.s->tol2 || c.s->iters >= max_iter)
            c.s->done = 1;
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

// Matrix-vector product grid: one workgroup per 16 nodes, at most 8192 (a
// wider grid keeps more gathers in flight than fewer, longer-running groups).
int spmv_grid(int n)
{
    const int g = (int)blocks(n / 3, kBlock / kNodeLanes);
    return g < 1 ? 1 : (g > 8192 ? 8192 : g);
}

// Size of the partial-sum buffer: two vector-kernel halves or one SpMV grid.
int cg_partials(int n)
{
    const int a = 2 * (int)blocks(n, kBlock);
    const int b = spmv_grid(n);
    return a > b ? a : b;
}

hipError_t launch_cg_init(const CgView& c, const double* b, double rtol, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_init, dim3(blocks(c.n, kBlock)), dim3(kBlock), 0, s, c, b);
    hipLaunchKernelGGL(k_cg_init_finish, dim3(1), dim3(kBlock), 0, s, c, rtol);
    return hipGetLastError();
}

hipError_t launch_cg_iterations(const CgView& c, int first, int count, int max_iter, hipStream_t s)
{
    const unsigned gs = (unsigned)spmv_grid(c.n);
    const unsigned gv = blocks(c.n, kBlock);
    for (int k = first; k < first + count; ++k) {
        const int cur = k & 1;  // which copy of p holds the previous direction
        hipLaunchKernelGGL(k_cg_spmv, dim3(gs), dim3(kBlock), 0, s, c, cur);
        hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(kBlock), 0, s, c, (int)gs);
        hipLaunchKernelGGL(k_cg_update, dim3(gv), dim3(kBlock), 0, s, c, cur);
        hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(kBlock), 0, s, c, max_iter);
    }
    return hipGetLastError();
}

hipError_t launch_cg_output(const CgView& c, double* x, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_output, dim3(blocks(c.n, kBlock)), dim3(kBlock), 0, s, c, x);
    return hipGetLastError();
}

}  // namespace sta
