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
// GPU mapping.  Supernodes of one level of the supernodal elimination tree
// are independent; a supernode is cut into column blocks of at most 64
// columns and each block into 64-row tiles.  Each level runs as
//   k_external : one workgroup per (block, row tile) of the level's
//                supernodes; the tile lives in LDS while every descendant of
//                another supernode that meets it subtracts its product
//                (matrix cores, 16x16x4) at the relative positions of its
//                rows.  The (tile, descendant) incidences and the descendant
//                row ranges are computed by the analysis, so the kernel
//                does no searching in global memory.  Tile 0 of each
//                supernode's first block then factors that block in LDS.
//   k_trsm     : the remaining row tiles of a just-factored block solve
//                X := X L_JJ^{-T}.
//   k_internal : right-looking updates inside a wide supernode: once block
//                k-1 is final, every tile of blocks k, k+1, ... subtracts
//                its product with block k-1 (matrix cores, accumulators
//                seeded with the tile); tile 0 of block k then factors it.
// Every tile has exactly one writer per launch and a fixed summation order,
// so results are bitwise reproducible.
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

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// 16x16x4 matrix-core product per wavefront.  Operands: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator element v of lane l
// is D[row(l, v)][l % 16] (the FP64 and FP32 instructions place rows
// differently).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
    using acc_t = d4;
    __device__ static __forceinline__ acc_t mma(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct Mfma<float> {
    using acc_t = f4;
    __device__ static __forceinline__ acc_t mma(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// acc[m][n] += sgn * A[rows, :] * B[cols, :]^T for the 32 x 32 quadrant
// (wr, wc) of a product with nI x nJ valid entries and inner dimension wk.
// A and B are column-major panels with leading dimension ld; rows and
// columns of the quadrant are 32*wr + 16*m + (lane % 16) and
// 32*wc + 16*n + (lane % 16).  Entries outside the valid range read as 0.
template <typename T>
__device__ __forceinline__ void wave_product(const T *__restrict__ pa, const T *__restrict__ pb,
                                             int64_t ld, int nI, int nJ, int wk, int wr, int wc,
                                             T sgn, typename Mfma<T>::acc_t (&acc)[2][2])
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int ra0 = 32 * wr + li, ra1 = ra0 + 16;
    const int cb0 = 32 * wc + li, cb1 = cb0 + 16;
    const bool va0 = ra0 < nI, va1 = ra1 < nI, vb0 = cb0 < nJ, vb1 = cb1 < nJ;
    for (int k0 = 0; k0 < wk; k0 += 4) {
        const int k = k0 + lk;
        const bool vk = k < wk;
        const int64_t ko = (int64_t)k * ld;
        const T a0 = (va0 && vk) ? sgn * pa[ra0 + ko] : T(0);
        const T a1 = (va1 && vk) ? sgn * pa[ra1 + ko] : T(0);
        const T b0 = (vb0 && vk) ? pb[cb0 + ko] : T(0);
        const T b1 = (vb1 && vk) ? pb[cb1 + ko] : T(0);
        acc[0][0] = Mfma<T>::mma(a0, b0, acc[0][0]);
        acc[0][1] = Mfma<T>::mma(a0, b1, acc[0][1]);
        acc[1][0] = Mfma<T>::mma(a1, b0, acc[1][0]);
        acc[1][1] = Mfma<T>::mma(a1, b1, acc[1][1]);
    }
}

// External update of one row tile of block J: for every descendant K of
// another supernode that meets the tile, tile -= L_K[b0:b1, :] L_K[a0:a1, :]^T
// at the relative positions of K's rows in J.  The tile stays in LDS; the
// four wavefronts each own one 32 x 32 quadrant of every product, and
// distinct product entries land on distinct tile entries, so no atomics are
// needed and the summation order is fixed.  With kFuseFactor the tile is
// tile 0 of a supernode's first block, which is then factored in place.
template <typename T>
__global__ __launch_bounds__(NT) void k_external(const Task *__restrict__ tasks,
                                                 const int64_t *__restrict__ iptr,
                                                 const Incidence *__restrict__ incs,
                                                 const BlockDesc *__restrict__ blk,
                                                 const int32_t *__restrict__ rows,
                                                 T *__restrict__ Lx, int32_t *__restrict__ info)
{
    __shared__ T C[64 * LDC];
    __shared__ int32_t trow[TR];
    __shared__ int32_t s_lr[TR];
    __shared__ int32_t s_lc[64];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
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

    const int64_t qend = iptr[blockIdx.x + 1];
    for (int64_t q = iptr[blockIdx.x]; q < qend; ++q) {
        const Incidence in = incs[q];
        const BlockDesc K = blk[in.K];
        const int32_t *rK = rows + K.rowoff;
        const int nI = in.b1 - in.b0;
        const int nJ = in.a1 - in.a0;
        if (nI > nr || nJ > w || nI <= 0 || nJ <= 0) {   // corrupt plan: never write outside the tile
            if (tid == 0) atomicMin(info + 1, tk.J);
            continue;
        }
        if (tid < nI) {
            const int key = rK[in.b0 + tid];
            int lo = 0, hi = nr;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (trow[mid] < key) lo = mid + 1; else hi = mid;
            }
            if (lo >= nr || trow[lo] != key) {
                atomicMin(info + 1, tk.J);
                lo = 0;
            }
            s_lr[tid] = lo;
        } else if (tid >= 64 && tid < 64 + nJ) {
            int c = rK[in.a0 + tid - 64] - J.col0;
            if (c < 0 || c >= w) {
                atomicMin(info + 1, tk.J);
                c = 0;
            }
            s_lc[tid - 64] = c;
        }
        __syncthreads();
        if (32 * wr < nI && 32 * wc < nJ) {
            typename Mfma<T>::acc_t acc[2][2] = {};
            const T *LK = Lx + K.valoff;
            wave_product<T>(LK + in.b0, LK + in.a0, K.ld, nI, nJ, K.w, wr, wc, T(1), acc);
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int n = 0; n < 2; ++n)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = 32 * wr + 16 * m + Mfma<T>::row(lane, v);
                        const int col = 32 * wc + 16 * n + (lane & 15);
                        if (row < nI && col < nJ) {
                            const int R = s_lr[row], Cc = s_lc[col];
                            if (r0 + R >= Cc) C[Cc * LDC + R] -= acc[m][n][v];
                        }
                    }
        }
        __syncthreads();
    }

    if (tk.flags & kFuseFactor) panel_factor(C, nr, w, J.col0, info);

    for (int idx = tid; idx < nr * w; idx += NT) {
        const int i = idx % nr, c = idx / nr;
        LJ[(int64_t)c * J.ld + r0 + i] = C[c * LDC + i];
    }
}

// Internal (right-looking) update of one row tile of block J by the final
// block K of the same supernode: tile -= L_K[tile rows, :] L_K[J's columns, :]^T.
// J's local row 0 is K's local row d = col0_J - col0_K, so no index lookups
// are needed.  The accumulators start from the tile's current values.  With
// kFuseFactor (tile 0 of block K+1) the result is factored in LDS.
template <typename T>
__global__ __launch_bounds__(NT) void k_internal(const Task *__restrict__ tasks,
                                                 const BlockDesc *__restrict__ blk,
                                                 T *__restrict__ Lx, int32_t *__restrict__ info)
{
    __shared__ T C[64 * LDC];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const Task tk = tasks[blockIdx.x];
    const BlockDesc J = blk[tk.J];
    const BlockDesc K = blk[tk.K];
    const int d = J.col0 - K.col0;
    const int r0 = tk.t * TR;
    const int nr = min(TR, J.r - r0);
    const int w = J.w;
    T *LJ = Lx + J.valoff;
    const T *LK = Lx + K.valoff;
    const bool active = 32 * wr < nr && 32 * wc < w;

    typename Mfma<T>::acc_t acc[2][2] = {};
    if (active) {
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 32 * wr + 16 * m + Mfma<T>::row(lane, v);
                    const int col = 32 * wc + 16 * n + (lane & 15);
                    if (row < nr && col < w) acc[m][n][v] = LJ[(int64_t)col * J.ld + r0 + row];
                }
        wave_product<T>(LK + d + r0, LK + d, K.ld, nr, w, K.w, wr, wc, T(-1), acc);
    }
    if (tk.flags & kFuseFactor) {
        if (active) {
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int n = 0; n < 2; ++n)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = 32 * wr + 16 * m + Mfma<T>::row(lane, v);
                        const int col = 32 * wc + 16 * n + (lane & 15);
                        if (row < nr && col < w) C[col * LDC + row] = acc[m][n][v];
                    }
        }
        __syncthreads();
        panel_factor(C, nr, w, J.col0, info);
        for (int idx = tid; idx < nr * w; idx += NT) {
            const int i = idx % nr, c = idx / nr;
            LJ[(int64_t)c * J.ld + r0 + i] = C[c * LDC + i];
        }
    } else if (active) {
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 32 * wr + 16 * m + Mfma<T>::row(lane, v);
                    const int col = 32 * wc + 16 * n + (lane & 15);
                    if (row < nr && col < w) LJ[(int64_t)col * J.ld + r0 + row] = acc[m][n][v];
                }
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

struct Bracket {
    FactorProfile *prof;
    hipStream_t s;
    int32_t kind;
    Bracket(FactorProfile *p, hipStream_t st, int32_t k) : prof(p), s(st), kind(k)
    {
        if (prof && (size_t)(2 * prof->used + 1) < prof->ev.size())
            (void)hipEventRecord(prof->ev[2 * prof->used], s);
    }
    ~Bracket()
    {
        if (prof && (size_t)(2 * prof->used + 1) < prof->ev.size()) {
            (void)hipEventRecord(prof->ev[2 * prof->used + 1], s);
            prof->kind[prof->used] = kind;
            prof->used++;
        }
    }
};

template <typename T>
hipError_t factor_impl(const Plan &P, const DevicePlan &D, const double *Ax, hipStream_t s,
                       FactorProfile *prof)
{
    T *Lx = (T *)D.Lx;
    if (prof) prof->used = 0;
    {
        Bracket b(prof, s, 0);
        if (P.panel_entries > 0)
            k_fill_zero<T><<<grid_for(P.panel_entries), 256, 0, s>>>(Lx, P.panel_entries);
        if (P.nnzA > 0)
            k_scatter_a<T><<<grid_for(P.nnzA), 256, 0, s>>>(Ax, D.amap, Lx, P.nnzA);
        k_info_reset<<<1, 1, 0, s>>>(D.info);
    }
    for (const Phase &ph : P.phases) {
        const unsigned g = (unsigned)(ph.t1 - ph.t0);
        Bracket b(prof, s, ph.kind == kPhaseExternal ? 1 : ph.kind == kPhaseTrsm ? 2 : 3);
        if (ph.kind == kPhaseExternal)
            k_external<T><<<g, NT, 0, s>>>(D.tasks + ph.t0, D.iptr + ph.t0, D.incs, D.blk, D.rows, Lx,
                                           D.info);
        else if (ph.kind == kPhaseInternal)
            k_internal<T><<<g, NT, 0, s>>>(D.tasks + ph.t0, D.blk, Lx, D.info);
        else
            k_trsm<T><<<g, NT, 0, s>>>(D.tasks + ph.t0, D.blk, Lx);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_factor(const Plan &P, const DevicePlan &D, const double *Ax, hipStream_t s,
                         FactorProfile *prof)
{
    if (P.precision == 1) return factor_impl<float>(P, D, Ax, s, prof);
    return factor_impl<double>(P, D, Ax, s, prof);
}

}  // namespace sym
