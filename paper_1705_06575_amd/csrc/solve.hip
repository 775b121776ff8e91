// solve.hip -- supernodal sparse triangular solves on gfx950.
//
// Method (Sympiler, Section 3.1): for each column block, solve the small
// dense triangle on the diagonal first, then apply the result to the block's
// rows below the diagonal.  The forward sweep visits blocks in a
// topological order of the block elimination tree (level by level); the
// reach-pruned sweep (Section 1.1, the decoupled code) visits only the
// blocks that hold reached columns, and within a block only its reached
// columns, which are a suffix of the block: a reach set is a union of
// elimination-tree paths, and a supernode's columns form a chain.
//
// Forward, block J (one workgroup):  wavefront 0 solves the diagonal
// triangle with y_J in registers (lane k owns y_k); then every thread takes
// rows below the diagonal, forms sum_k L_ik y_k from column-major panel
// reads that are contiguous across the wavefront, and subtracts it from
// y[row] with one atomic add per row.
// Backward (L^T x = y), block J: each wavefront takes columns k and reduces
// sum_i L_ik x[row_i] over the rows below the diagonal, then wavefront 0
// solves the transposed diagonal triangle.  No atomics.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace sym {

namespace {

constexpr int NT = 256;

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

__global__ void k_zero(double *__restrict__ y, int32_t n)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        y[i] = 0.0;
}

__global__ void k_place(const double *__restrict__ bv, const int32_t *__restrict__ bpos,
                        double *__restrict__ y, int64_t nb)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nb;
         k += (int64_t)gridDim.x * blockDim.x)
        y[bpos[k]] = bv[k];
}

// Forward sweep over one level.  cstart (may be null) gives the first
// reached local column of each block; columns before it hold exact zeros
// and are skipped.
template <typename T>
__global__ __launch_bounds__(NT) void k_fwd(const int32_t *__restrict__ blocks,
                                            const int32_t *__restrict__ cstart,
                                            const BlockDesc *__restrict__ blk,
                                            const int32_t *__restrict__ rows,
                                            const T *__restrict__ Lx, double *__restrict__ y)
{
    __shared__ double ys[64];
    const int tid = threadIdx.x;
    const BlockDesc J = blk[blocks[blockIdx.x]];
    const int c0 = cstart ? cstart[blockIdx.x] : 0;
    const T *L = Lx + J.valoff;
    const int64_t ld = J.ld;
    const int w = J.w;
    if (tid < 64) {
        double v = (tid >= c0 && tid < w) ? y[J.col0 + tid] : 0.0;
        for (int k = c0; k < w; ++k) {
            const double vk = __shfl(v, k);
            const double xk = vk / (double)L[k * ld + k];
            if (tid == k) v = xk;
            else if (tid > k && tid < w) v -= (double)L[k * ld + tid] * xk;
        }
        if (tid < w) {
            ys[tid] = v;
            if (tid >= c0) y[J.col0 + tid] = v;
        }
    }
    __syncthreads();
    const int32_t *rJ = rows + J.rowoff;
    for (int i = w + tid; i < J.r; i += NT) {
        double acc = 0.0;
        for (int k = c0; k < w; ++k) acc += (double)L[k * ld + i] * ys[k];
        atomicAdd(&y[rJ[i]], -acc);
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_bwd(const int32_t *__restrict__ blocks,
                                            const BlockDesc *__restrict__ blk,
                                            const int32_t *__restrict__ rows,
                                            const T *__restrict__ Lx, double *__restrict__ x)
{
    __shared__ double ts[64];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const BlockDesc J = blk[blocks[blockIdx.x]];
    const T *L = Lx + J.valoff;
    const int64_t ld = J.ld;
    const int w = J.w;
    const int32_t *rJ = rows + J.rowoff;
    for (int k = wave; k < w; k += NT / 64) {
        double s = 0.0;
        for (int i = w + lane; i < J.r; i += 64) s += (double)L[k * ld + i] * x[rJ[i]];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) ts[k] = x[J.col0 + k] - s;
    }
    __syncthreads();
    if (tid < 64) {
        double v = tid < w ? ts[tid] : 0.0;
        for (int k = w - 1; k >= 0; --k) {
            const double vk = __shfl(v, k);
            const double xk = vk / (double)L[k * ld + k];
            if (tid == k) v = xk;
            else if (tid < k) v -= (double)L[tid * ld + k] * xk;
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
hipError_t fwd_impl(const Plan &P, const DevicePlan &D, double *y, hipStream_t s)
{
    for (int32_t l = 0; l < P.nlevels; ++l) {
        const int32_t b0 = P.level_ptr[l], b1 = P.level_ptr[l + 1];
        if (b1 > b0)
            k_fwd<T><<<(unsigned)(b1 - b0), NT, 0, s>>>(D.level_blocks + b0, nullptr, D.blk, D.rows,
                                                        (const T *)D.Lx, y);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t bwd_impl(const Plan &P, const DevicePlan &D, double *y, hipStream_t s)
{
    for (int32_t l = P.nlevels - 1; l >= 0; --l) {
        const int32_t b0 = P.level_ptr[l], b1 = P.level_ptr[l + 1];
        if (b1 > b0)
            k_bwd<T><<<(unsigned)(b1 - b0), NT, 0, s>>>(D.level_blocks + b0, D.blk, D.rows,
                                                        (const T *)D.Lx, y);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t fwd_sparse_impl(const Plan &P, const DevicePlan &D, const DeviceRhs &R,
                           const std::vector<int64_t> &level_ptr, int64_t nbeta,
                           const double *bv, double *y, hipStream_t s)
{
    if (P.n > 0) k_zero<<<grid_for(P.n), 256, 0, s>>>(y, P.n);
    if (nbeta > 0) k_place<<<grid_for(nbeta), 256, 0, s>>>(bv, R.bpos, y, nbeta);
    for (size_t l = 0; l + 1 < level_ptr.size(); ++l) {
        const int64_t b0 = level_ptr[l], b1 = level_ptr[l + 1];
        if (b1 > b0)
            k_fwd<T><<<(unsigned)(b1 - b0), NT, 0, s>>>(R.blocks + b0, R.cstart + b0, D.blk, D.rows,
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

hipError_t launch_fwd(const Plan &P, const DevicePlan &D, double *y, hipStream_t s)
{
    return P.precision == 1 ? fwd_impl<float>(P, D, y, s) : fwd_impl<double>(P, D, y, s);
}

hipError_t launch_bwd(const Plan &P, const DevicePlan &D, double *y, hipStream_t s)
{
    return P.precision == 1 ? bwd_impl<float>(P, D, y, s) : bwd_impl<double>(P, D, y, s);
}

hipError_t launch_fwd_sparse(const Plan &P, const DevicePlan &D, const DeviceRhs &R,
                             const std::vector<int64_t> &level_ptr, int64_t nbeta,
                             const double *bv, double *y, hipStream_t s)
{
    return P.precision == 1 ? fwd_sparse_impl<float>(P, D, R, level_ptr, nbeta, bv, y, s)
                            : fwd_sparse_impl<double>(P, D, R, level_ptr, nbeta, bv, y, s);
}

}  // namespace sym
