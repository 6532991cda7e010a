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
#include <hip/hip_runtime.h>

#include "sta_internal.h"

namespace sta {

namespace {

constexpr int kBlock = 256;
constexpr int kRowLanes = 8;  // lanes per CSR row in the matrix-vector product

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
__device__ __forceinline__ double reduce_partials(const double* __restrict__ p, int n, double* sh)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock)
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
        c.p[r] = z;
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
        c.s->tol2 = (rtol * rtol) * bb;
        c.s->iters = 0;
        c.s->done = bb == 0.0 ? 1 : 0;
    }
}

// q = A p, partial p.q.  kRowLanes lanes per row, fixed shuffle tree.
__global__ __launch_bounds__(kBlock) void k_cg_spmv(CgView c)
{
    __shared__ double sh[kBlock];
    if (c.s->done)
        return;
    const int r = blockIdx.x * (kBlock / kRowLanes) + threadIdx.x / kRowLanes;
    const int l = threadIdx.x & (kRowLanes - 1);
    double acc = 0.0;
    if (r < c.n) {
        const int s0 = c.rowptr[r], s1 = c.rowptr[r + 1];
        for (int s = s0 + l; s < s1; s += kRowLanes)
            acc = acc + c.vals[s] * c.p[c.colidx[s]];
    }
#pragma unroll
    for (int o = kRowLanes / 2; o > 0; o >>= 1)
        acc = acc + __shfl_xor(acc, o, kRowLanes);
    double pq = 0.0;
    if (r < c.n && l == 0) {
        const double q = c.dinv[r] != 0.0 ? acc : 0.0;
        c.q[r] = q;
        pq = c.p[r] * q;
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

// x += alpha p, r -= alpha q, z = Dinv r; partial r.z and r.r
__global__ __launch_bounds__(kBlock) void k_cg_update(CgView c)
{
    __shared__ double sh[kBlock];
    if (c.s->done)
        return;
    const double alpha = c.s->alpha;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (i < c.n) {
        c.x[i] = c.x[i] + alpha * c.p[i];
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

__global__ __launch_bounds__(kBlock) void k_cg_direction(CgView c)
{
    if (c.s->done)
        return;
    const double beta = c.s->beta;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < c.n)
        c.p[i] = c.z[i] + beta * c.p[i];
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

// Size of the partial-sum buffer: two vector-kernel halves or one SpMV grid.
int cg_partials(int n)
{
    const int a = 2 * (int)blocks(n, kBlock);
    const int b = (int)blocks(n, kBlock / kRowLanes);
    return a > b ? a : b;
}

hipError_t launch_cg_init(const CgView& c, const double* b, double rtol, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_init, dim3(blocks(c.n, kBlock)), dim3(kBlock), 0, s, c, b);
    hipLaunchKernelGGL(k_cg_init_finish, dim3(1), dim3(kBlock), 0, s, c, rtol);
    return hipGetLastError();
}

hipError_t launch_cg_iterations(const CgView& c, int count, int max_iter, hipStream_t s)
{
    const unsigned gs = blocks(c.n, kBlock / kRowLanes);
    const unsigned gv = blocks(c.n, kBlock);
    for (int k = 0; k < count; ++k) {
        hipLaunchKernelGGL(k_cg_spmv, dim3(gs), dim3(kBlock), 0, s, c);
        hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(kBlock), 0, s, c, (int)gs);
        hipLaunchKernelGGL(k_cg_update, dim3(gv), dim3(kBlock), 0, s, c);
        hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(kBlock), 0, s, c, max_iter);
        hipLaunchKernelGGL(k_cg_direction, dim3(gv), dim3(kBlock), 0, s, c);
    }
    return hipGetLastError();
}

hipError_t launch_cg_output(const CgView& c, double* x, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_output, dim3(blocks(c.n, kBlock)), dim3(kBlock), 0, s, c, x);
    return hipGetLastError();
}

}  // namespace sta
