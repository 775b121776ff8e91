// solve.hip -- supernodal sparse triangular solves on gfx950.
//
// Method (Sympiler, Section 3.1): for each column block, solve the small
// dense triangle on the diagonal first, then apply the result to the block's
// rows below the diagonal.  The forward sweep visits blocks in a
// topological order of the block elimination tree, level by level; the
// reach-pruned sweep (Section 1.1, the decoupled code) visits only the
// blocks that hold reached columns, and within a block only the columns
// from its first reached one on (a reach set is a union of
// elimination-tree paths; columns of a block that are not reached hold
// exact zeros and contribute nothing).
//
// Forward, one launch per level, one workgroup per (block, chunk of 256 of
// its rows below the diagonal): the block's diagonal triangle is staged in
// LDS with coalesced loads; wavefront 0 solves it with the block's values
// in registers (lane k owns y_k) -- every chunk of the block repeats this
// small solve, which saves a second launch per level; chunk 0 stores the
// solved values in the output vector; every thread then forms
// sum_k L_ik y_k for one row (column-major reads contiguous across the
// wavefront) and subtracts it from the accumulator entry of that row with
// one atomic add.  Inputs are read from the accumulator and results written
// to a separate output vector, so no task reads a value another task of the
// same launch writes.
// Backward (L^T x = y), two launches per level in reverse: chunks of each
// block's rows below the diagonal subtract their share of L_offdiag^T x from
// the block's entries (atomics), then one wavefront per block solves the
// transposed diagonal triangle from LDS.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace sym {

namespace {

constexpr int NT = 256;
constexpr int LDT = 65;                 // LDS stride of a staged diagonal triangle

__device__ __forceinline__ double lane_value(double v, int src)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Stage the lower triangle of a w x w diagonal block (global, leading
// dimension ld, columns from c0 on) into LDS as doubles.  All loads are
// issued before the first store (one memory latency per block).
template <typename T>
__device__ __forceinline__ void stage_tri(double *D, const T *__restrict__ L, int64_t ld, int w,
                                          int c0)
{
    const int i = threadIdx.x & 63, cq = threadIdx.x >> 6;
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int c = cq + 4 * u;
        const bool ok = i < w && c < w && i >= c && c >= c0;
        const T val = L[ok ? (int64_t)c * ld + i : 0];
        v[u] = ok ? (double)val : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int c = cq + 4 * u;
        if (i < w && c < w) D[c * LDT + i] = v[u];
    }
}

// sum_{k = c0}^{w-1} L[k * ld + i] * ys[k] with the loads of 16 columns
// issued together.
template <typename T>
__device__ __forceinline__ double row_dot(const T *__restrict__ L, int64_t ld, int64_t i,
                                          const double *ys, int c0, int w)
{
    double s = 0.0;
    for (int k0 = c0; k0 < w; k0 += 16) {
        double lv[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int k = k0 + j;
            const T val = L[(k < w ? (int64_t)k * ld : 0) + i];
            lv[j] = k < w ? (double)val : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (k0 + j < w) s += lv[j] * ys[k0 + j];
    }
    return s;
}

__global__ void k_gather(const double *__restrict__ b, const int32_t *__restrict__ perm,
                         double *__restrict__ y, int32_t n)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        y[i] = b[perm[i]];
}

__global__ void k_scatter_perm(const double *__restrict__ y, const int32_t *__restrict__ perm,
                               double *__restrict__ x, int32_t n)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        x[perm[i]] = y[i];
}

__global__ void k_zero2(double *__restrict__ a, double *__restrict__ b, int32_t n)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        a[i] = 0.0;
        b[i] = 0.0;
    }
}

__global__ void k_place(const double *__restrict__ bv, const int32_t *__restrict__ bpos,
                        double *__restrict__ y, int64_t nb)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nb;
         k += (int64_t)gridDim.x * blockDim.x)
        y[bpos[k]] = bv[k];
}

// Forward sweep tasks of one level.  acc: right-hand side plus the updates
// of earlier levels (read for the block's own columns, atomically updated
// for the rows below); out: solved values of the block's columns.
template <typename T>
__global__ __launch_bounds__(NT) void k_fwd(const SolveTask *__restrict__ tasks,
                                            const BlockDesc *__restrict__ blk,
                                            const int32_t *__restrict__ rows,
                                            const T *__restrict__ Lx, double *__restrict__ acc,
                                            double *__restrict__ out)
{
    __shared__ double D[64 * LDT];
    __shared__ double ys[64];
    const int tid = threadIdx.x;
    const SolveTask tk = tasks[blockIdx.x];
    const BlockDesc J = blk[tk.J];
    const int c0 = tk.c0;
    const T *L = Lx + J.valoff;
    const int64_t ld = J.ld;
    const int w = J.w;
    stage_tri(D, L, ld, w, c0);
    double v = 0.0;
    if (tid < 64 && tid >= c0 && tid < w) v = acc[J.col0 + tid];
    __syncthreads();
    if (tid < 64) {
        for (int k = c0; k < w; ++k) {
            const double xk = lane_value(v, k) / D[k * LDT + k];
            if (tid == k) v = xk;
            else if (tid > k && tid < w) v -= D[k * LDT + tid] * xk;
        }
        ys[tid] = v;
        if (tk.chunk == 0 && tid >= c0 && tid < w) out[J.col0 + tid] = v;
    }
    __syncthreads();
    const int i = w + tk.chunk * NT + tid;
    if (i < J.r) {
        const int32_t row = rows[J.rowoff + i];
        const double s = row_dot(L, ld, i, ys, c0, w);
        atomicAdd(&acc[row], -s);
    }
}

// Backward sweep, first half of a level: task (J, chunk) subtracts
// sum_{i in chunk} L_ik x[row_i] from x[J's column k] for every k.  Wavefront v
// takes columns k = v, v + 4, ..., lanes take rows (coalesced column-major
// reads), a wavefront reduction per column, one atomic per column.  Tasks of
// a level read only x of blocks of higher levels (already final) and write
// only their own block's columns.
template <typename T>
__global__ __launch_bounds__(NT) void k_bwd_gather(const SolveTask *__restrict__ tasks,
                                                   const BlockDesc *__restrict__ blk,
                                                   const int32_t *__restrict__ rows,
                                                   const T *__restrict__ Lx, double *__restrict__ x)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const SolveTask tk = tasks[blockIdx.x];
    const BlockDesc J = blk[tk.J];
    const T *L = Lx + J.valoff;
    const int64_t ld = J.ld;
    const int w = J.w;
    const int i0 = w + tk.chunk * NT;
    const int i1 = min(J.r, i0 + NT);
    const int32_t *rJ = rows + J.rowoff;
    double part[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) part[q] = 0.0;
    // the chunk's four rows per lane: indices, then x values, then L
    int32_t ri[4];
    double xr[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = i0 + lane + 64 * u;
        ri[u] = i < i1 ? rJ[i] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = i0 + lane + 64 * u;
        const double xv = x[ri[u]];
        xr[u] = i < i1 ? xv : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = i0 + lane + 64 * u;
        const int ic = i < i1 ? i : i0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int k = wave + 4 * q;
            const T val = L[(k < w ? (int64_t)k * ld : 0) + ic];
            part[q] += (k < w ? (double)val : 0.0) * xr[u];
        }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int k = wave + 4 * q;
        if (k < w) {
            double s2 = part[q];
            for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off);
            if (lane == 0) atomicAdd(&x[J.col0 + k], -s2);
        }
    }
}

// Backward sweep, second half of a level: each block solves its transposed
// diagonal triangle, staged in LDS, with one wavefront (lane k owns x_k).
template <typename T>
__global__ __launch_bounds__(NT) void k_bwd_diag(const int32_t *__restrict__ blocks,
                                                 const BlockDesc *__restrict__ blk,
                                                 const T *__restrict__ Lx, double *__restrict__ x)
{
    __shared__ double D[64 * LDT];
    const int tid = threadIdx.x;
    const BlockDesc J = blk[blocks[blockIdx.x]];
    const T *L = Lx + J.valoff;
    const int64_t ld = J.ld;
    const int w = J.w;
    stage_tri(D, L, ld, w, 0);
    double v = 0.0;
    if (tid < w) v = x[J.col0 + tid];
    __syncthreads();
    if (tid < 64) {
        for (int k = w - 1; k >= 0; --k) {
            const double xk = lane_value(v, k) / D[k * LDT + k];
            if (tid == k) v = xk;
            else if (tid < k) v -= D[tid * LDT + k] * xk;
        }
        if (tid < w) x[J.col0 + tid] = v;
    }
}

inline unsigned grid_for(int64_t count)
{
    int64_t g = (count + 255) / 256;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

template <typename T>
hipError_t fwd_impl(const std::vector<int64_t> &level_ptr, const SolveTask *tasks,
                    const DevicePlan &D, double *acc, double *out, hipStream_t s)
{
    for (size_t l = 0; l + 1 < level_ptr.size(); ++l) {
        const int64_t t0 = level_ptr[l], t1 = level_ptr[l + 1];
        if (t1 > t0)
            k_fwd<T><<<(unsigned)(t1 - t0), NT, 0, s>>>(tasks + t0, D.blk, D.rows, (const T *)D.Lx,
                                                        acc, out);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t bwd_impl(const Plan &P, const DevicePlan &D, double *y, hipStream_t s)
{
    for (int32_t l = P.nlevels - 1; l >= 0; --l) {
        const int64_t t0 = P.bwd_level_ptr[l], t1 = P.bwd_level_ptr[l + 1];
        if (t1 > t0)
            k_bwd_gather<T><<<(unsigned)(t1 - t0), NT, 0, s>>>(D.bwd_tasks + t0, D.blk, D.rows,
                                                               (const T *)D.Lx, y);
        const int32_t b0 = P.level_ptr[l], b1 = P.level_ptr[l + 1];
        if (b1 > b0)
            k_bwd_diag<T><<<(unsigned)(b1 - b0), NT, 0, s>>>(D.level_blocks + b0, D.blk,
                                                             (const T *)D.Lx, y);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_perm_gather(const Plan &P, const DevicePlan &D, const double *b, double *y,
                              hipStream_t s)
{
    if (P.n > 0) k_gather<<<grid_for(P.n), 256, 0, s>>>(b, D.perm, y, P.n);
    return hipGetLastError();
}

hipError_t launch_perm_scatter(const Plan &P, const DevicePlan &D, const double *y, double *x,
                               hipStream_t s)
{
    if (P.n > 0) k_scatter_perm<<<grid_for(P.n), 256, 0, s>>>(y, D.perm, x, P.n);
    return hipGetLastError();
}

hipError_t launch_fwd(const Plan &P, const DevicePlan &D, double *acc, double *out, hipStream_t s)
{
    return P.precision == 1 ? fwd_impl<float>(P.fwd_level_ptr, D.fwd_tasks, D, acc, out, s)
                            : fwd_impl<double>(P.fwd_level_ptr, D.fwd_tasks, D, acc, out, s);
}

hipError_t launch_bwd(const Plan &P, const DevicePlan &D, double *y, hipStream_t s)
{
    return P.precision == 1 ? bwd_impl<float>(P, D, y, s) : bwd_impl<double>(P, D, y, s);
}

hipError_t launch_fwd_sparse(const Plan &P, const DevicePlan &D, const DeviceRhs &R,
                             const std::vector<int64_t> &level_ptr, int64_t nbeta,
                             const double *bv, double *acc, double *out, hipStream_t s)
{
    if (P.n > 0) k_zero2<<<grid_for(P.n), 256, 0, s>>>(acc, out, P.n);
    if (nbeta > 0) k_place<<<grid_for(nbeta), 256, 0, s>>>(bv, R.bpos, acc, nbeta);
    return P.precision == 1 ? fwd_impl<float>(level_ptr, R.tasks, D, acc, out, s)
                            : fwd_impl<double>(level_ptr, R.tasks, D, acc, out, s);
}

}  // namespace sym
