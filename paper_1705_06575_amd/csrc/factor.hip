// factor.hip -- numeric supernodal Cholesky on gfx950.
//
// Method (Sympiler, Section 3.2): left-looking supernodal Cholesky.  For
// each column block J in a topological order of the block elimination tree:
//   update:  J's panel -= L_K[rows >= f_J, :] * L_K[rows in J's columns, :]^T
//            for every descendant block K in J's prune set (the blocks whose
//            row pattern meets J's columns);
//   factor:  dense Cholesky of J's diagonal block, then dense triangular
//            solves of the rows below it.
//
// GPU mapping.  Blocks of one level of the block elimination tree are
// independent.  Each level runs as
//   k_update : one workgroup per (J, 64-row tile of J).  The tile lives in
//              LDS for the whole gather; each descendant's contribution is
//              formed from the two row ranges of K that meet the tile and
//              subtracted at the relative positions (positions found by a
//              64-wide wavefront search in K's row list and a binary search
//              among the tile's rows).  No atomics: each tile has one owner,
//              so the summation order is fixed and runs are bitwise
//              reproducible.  Tile 0 of a block then factors the diagonal
//              block and solves its own rows below it in LDS.
//   k_trsm   : tiles t >= 1 of blocks with more than 64 rows solve
//              X := X L_JJ^{-T} against the diagonal block written by
//              tile 0 in k_update.
// A non-positive (or NaN) pivot stores the smallest failing column in a
// device word; the factorization continues (results are then undefined).
// A second word records the first block whose descendant rows do not nest
// in its own (impossible for a plan built by the analysis; checked so that a
// corrupt plan cannot write outside a tile).
#include <hip/hip_runtime.h>

#include <climits>

#include "device.hpp"

namespace sym {

namespace {

constexpr int NT = 256;           // threads per workgroup (4 wavefronts)
constexpr int TR = kTileRows;     // tile rows (64)
constexpr int LDC = TR + 1;       // LDS column stride of a tile

template <typename T>
__global__ void k_fill_zero(T *__restrict__ x, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = T(0);
}

template <typename T>
__global__ void k_scatter_a(const double *__restrict__ Ax, const int64_t *__restrict__ amap,
                            T *__restrict__ Lx, int64_t nnz)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * blockDim.x)
        Lx[amap[k]] = (T)Ax[k];
}

__global__ void k_info_reset(int32_t *info) { info[0] = INT32_MAX; info[1] = INT32_MAX; }

// First position p in [lo, hi) with a[p] >= key (a sorted ascending); every
// lane of the calling wavefront gets the result.  64-ary search: each round
// samples 64 evenly spaced entries and keeps the bracket that holds the
// answer, so a list of up to 4096 entries takes two dependent loads.
__device__ __forceinline__ int wave_lower_bound(const int32_t *__restrict__ a, int lo, int hi,
                                                int key)
{
    const int lane = threadIdx.x & 63;
    while (hi - lo > 64) {
        const int step = (hi - lo + 63) >> 6;
        const int pos = lo + lane * step;
        const bool less = pos < hi && a[pos] < key;
        const int cnt = __popcll(__ballot(less));
        const int nlo = cnt > 0 ? lo + (cnt - 1) * step + 1 : lo;
        const int nhi = min(lo + cnt * step, hi);
        lo = nlo;
        hi = nhi;
    }
    const int pos = lo + lane;
    const bool less = pos < hi && a[pos] < key;
    return lo + __popcll(__ballot(less));
}

// Right-looking Cholesky of an nr x w panel held column-major in LDS
// (stride LDC): rows [0, w) are the diagonal block, rows [w, nr) the rows
// below it.  Each step takes the pivot's square root, divides the column
// below it and applies the rank-1 update to the columns to its right.
template <typename T>
__device__ void panel_factor(T *C, int nr, int w, int col0, int32_t *info)
{
    const int tid = threadIdx.x;
    for (int k = 0; k < w; ++k) {
        const T d = C[k * LDC + k];
        const T l = sqrt(d);
        __syncthreads();
        if (tid == 0) {
            C[k * LDC + k] = l;
            if (!(d > T(0))) atomicMin(info, col0 + k);
        }
        for (int i = k + 1 + tid; i < nr; i += NT) C[k * LDC + i] /= l;
        __syncthreads();
        const int nc = w - k - 1;
        const int nrow = nr - k - 1;
        for (int idx = tid; idx < nc * nrow; idx += NT) {
            const int c = k + 1 + idx / nrow;
            const int i = k + 1 + idx % nrow;
            if (i >= c) C[c * LDC + i] -= C[k * LDC + i] * C[k * LDC + c];
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_update(const Task *__restrict__ tasks,
                                               const BlockDesc *__restrict__ blk,
                                               const int32_t *__restrict__ rows,
                                               const int64_t *__restrict__ dptr,
                                               const Pair *__restrict__ pairs,
                                               T *__restrict__ Lx, int32_t *__restrict__ info)
{
    __shared__ T C[64 * LDC];
    __shared__ int32_t trow[TR];
    __shared__ int32_t s_lr[TR];
    __shared__ int32_t s_lc[64];

    const int tid = threadIdx.x;
    const Task tk = tasks[blockIdx.x];
    const BlockDesc J = blk[tk.J];
    const int r0 = tk.t * TR;
    const int nr = min(TR, J.r - r0);
    const int w = J.w;
    const int32_t *rJ = rows + J.rowoff;
    T *LJ = Lx + J.valoff;

    for (int idx = tid; idx < nr * w; idx += NT) {
        const int i = idx % nr, c = idx / nr;
        C[c * LDC + i] = LJ[(int64_t)c * J.ld + r0 + i];
    }
    if (tid < nr) trow[tid] = rJ[r0 + tid];
    __syncthreads();
    const int row_lo = trow[0];
    const int row_hi = trow[nr - 1];

    const int64_t pend = dptr[tk.J + 1];
    for (int64_t p = dptr[tk.J]; p < pend; ++p) {
        const Pair pr = pairs[p];
        const BlockDesc K = blk[pr.K];
        const int32_t *rK = rows + K.rowoff;
        // K's rows inside this tile: [b0, b1) (uniform over the workgroup)
        const int b0 = tk.t == 0 ? pr.a0 : wave_lower_bound(rK, pr.a1, K.r, row_lo);
        const int b1 = wave_lower_bound(rK, b0, K.r, row_hi + 1);
        if (b0 >= b1) continue;
        const int nI = b1 - b0;
        const int nJ = pr.a1 - pr.a0;
        if (nI > nr || nJ > w) {                   // violates Eq. (1) containment: plan is corrupt
            if (tid == 0) atomicMin(info + 1, tk.J);
            continue;
        }
        if (tid < nI) {
            const int key = rK[b0 + tid];
            int lo = 0, hi = nr;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (trow[mid] < key) lo = mid + 1; else hi = mid;
            }
            if (lo >= nr || trow[lo] != key) {     // K row missing from J: plan is corrupt
                atomicMin(info + 1, tk.J);
                lo = 0;
            }
            s_lr[tid] = lo;
        }
        if (tid >= 64 && tid < 64 + nJ) s_lc[tid - 64] = rK[pr.a0 + tid - 64] - J.col0;
        __syncthreads();
        const T *LK = Lx + K.valoff;
        const int64_t ldk = K.ld;
        const int wk = K.w;
        for (int idx = tid; idx < nI * nJ; idx += NT) {
            const int i = idx % nI, j = idx / nI;
            const int row = s_lr[i], col = s_lc[j];
            if (r0 + row < col) continue;          // upper triangle of the diagonal block
            T acc = T(0);
            const T *pa = LK + b0 + i;
            const T *pb = LK + pr.a0 + j;
            for (int k = 0; k < wk; ++k) acc += pa[k * ldk] * pb[k * ldk];
            C[col * LDC + row] -= acc;
        }
        __syncthreads();
    }

    if (tk.t == 0) panel_factor(C, nr, w, J.col0, info);

    for (int idx = tid; idx < nr * w; idx += NT) {
        const int i = idx % nr, c = idx / nr;
        LJ[(int64_t)c * J.ld + r0 + i] = C[c * LDC + i];
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_trsm(const Task *__restrict__ tasks,
                                             const BlockDesc *__restrict__ blk,
                                             T *__restrict__ Lx)
{
    __shared__ T D[64 * LDC];
    __shared__ T X[64 * LDC];
    const int tid = threadIdx.x;
    const Task tk = tasks[blockIdx.x];
    const BlockDesc J = blk[tk.J];
    const int r0 = tk.t * TR;
    const int nr = min(TR, J.r - r0);
    const int w = J.w;
    T *LJ = Lx + J.valoff;
    for (int idx = tid; idx < w * w; idx += NT) {
        const int i = idx % w, c = idx / w;
        D[c * LDC + i] = LJ[(int64_t)c * J.ld + i];
    }
    for (int idx = tid; idx < nr * w; idx += NT) {
        const int i = idx % nr, c = idx / nr;
        X[c * LDC + i] = LJ[(int64_t)c * J.ld + r0 + i];
    }
    __syncthreads();
    for (int k = 0; k < w; ++k) {
        const T dkk = D[k * LDC + k];
        for (int i = tid; i < nr; i += NT) X[k * LDC + i] /= dkk;
        __syncthreads();
        const int nc = w - k - 1;
        for (int idx = tid; idx < nc * nr; idx += NT) {
            const int c = k + 1 + idx / nr;
            const int i = idx % nr;
            X[c * LDC + i] -= X[k * LDC + i] * D[k * LDC + c];
        }
        __syncthreads();
    }
    for (int idx = tid; idx < nr * w; idx += NT) {
        const int i = idx % nr, c = idx / nr;
        LJ[(int64_t)c * J.ld + r0 + i] = X[c * LDC + i];
    }
}

inline unsigned grid_for(int64_t count, int per = 256)
{
    int64_t g = (count + per - 1) / per;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

template <typename T>
hipError_t factor_impl(const Plan &P, const DevicePlan &D, const double *Ax, hipStream_t s)
{
    T *Lx = (T *)D.Lx;
    if (P.panel_entries > 0)
        k_fill_zero<T><<<grid_for(P.panel_entries), 256, 0, s>>>(Lx, P.panel_entries);
    if (P.nnzA > 0)
        k_scatter_a<T><<<grid_for(P.nnzA), 256, 0, s>>>(Ax, D.amap, Lx, P.nnzA);
    k_info_reset<<<1, 1, 0, s>>>(D.info);
    for (int32_t l = 0; l < P.nlevels; ++l) {
        const int64_t t0 = P.task_ptr[l], t1 = P.task_ptr[l + 1];
        if (t1 > t0)
            k_update<T><<<(unsigned)(t1 - t0), NT, 0, s>>>(D.tasks + t0, D.blk, D.rows, D.dptr,
                                                           D.pairs, Lx, D.info);
        const int64_t u0 = P.task2_ptr[l], u1 = P.task2_ptr[l + 1];
        if (u1 > u0)
            k_trsm<T><<<(unsigned)(u1 - u0), NT, 0, s>>>(D.tasks2 + u0, D.blk, Lx);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_factor(const Plan &P, const DevicePlan &D, const double *Ax, hipStream_t s)
{
    if (P.precision == 1) return factor_impl<float>(P, D, Ax, s);
    return factor_impl<double>(P, D, Ax, s);
}

}  // namespace sym
