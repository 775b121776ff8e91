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
//                X := X L_JJ^{-T} (16 x 16 diagonal triangles inverted, the
//                rest on matrix cores).
//   k_internal : right-looking updates inside a wide supernode: once block
//                k-1 is final, every tile of blocks k, k+1, ... subtracts
//                its product with block k-1 (matrix cores, accumulators
//                seeded with the tile); tile 0 of block k then factors it.
//   k_inverse_small / k_inverse_big : after the last level, the inverse of
//                every diagonal block, stored transposed in the block's
//                unused upper triangle for the triangular solves.
// Every tile has exactly one writer per launch and a fixed summation order,
// so results are bitwise reproducible.  A long external tile is split into
// parts that run as separate workgroups of the same launch: each stores its
// partial sum with device-coherent stores and counts its arrival with a
// device-scope atomic; the last part adds the partial sums in part order
// and finishes the tile (no workgroup waits for another).
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

// Loads and stores of panel values that another workgroup of the same
// launch writes or reads take the device-coherence bit (sc1): the form of a
// device-scope relaxed atomic access, coherent across the chip's per-die L2
// caches.  They go through a raw buffer resource over the 4 GiB from a base
// address (a device panel never reaches 4 GiB), so the address is a scalar
// base plus a 32-bit byte offset, as for the plain loads.
constexpr int kCoherentBit = 16;        // the cache-policy operand's sc1 bit

__device__ __forceinline__ __amdgpu_buffer_rsrc_t coherent_rsrc(const void *base)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, -1, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T coherent_ld(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kCoherentBit));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kCoherentBit));
}
template <typename T>
__device__ __forceinline__ void coherent_st(__amdgpu_buffer_rsrc_t r, uint32_t off, T v)
{
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v),
                                              r, off, 0, kCoherentBit);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, kCoherentBit);
}

// Copy the nr x w column-major block at src (leading dimension ld; nr, w
// <= 64) into LDS (stride LDC) with all threads.  Thread t moves row t % 64
// of columns t / 64 + 4u: every load is issued before the first store, so
// the block costs one memory latency, and each column's rows are contiguous
// across the wavefront.
template <typename T>
__device__ __forceinline__ void tile_in(T *dst, const T *__restrict__ src, int64_t ld, int nr, int w)
{
    const int i = threadIdx.x & 63, c0 = threadIdx.x >> 6;
    T v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int c = c0 + 4 * u;
        v[u] = (i < nr && c < w) ? src[(int64_t)c * ld + i] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int c = c0 + 4 * u;
        if (i < nr && c < w) dst[c * LDC + i] = v[u];
    }
}

// Two blocks of the same panel (rows [0, n1) at s1 and [0, n2) at s2, w
// columns each) into LDS with all loads issued before the first store; the
// rest of both 64 x 64 LDS blocks is set to zero.
template <typename T>
__device__ __forceinline__ void tile2_in(T *d1, const T *__restrict__ s1, int n1, T *d2,
                                         const T *__restrict__ s2, int n2, int64_t ld, int w)
{
    const int i = threadIdx.x & 63, c0 = threadIdx.x >> 6;
    T v[16], u2[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int c = c0 + 4 * u;
        v[u] = (i < n1 && c < w) ? s1[(int64_t)c * ld + i] : T(0);
        u2[u] = (i < n2 && c < w) ? s2[(int64_t)c * ld + i] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int c = c0 + 4 * u;
        d1[c * LDC + i] = v[u];
        d2[c * LDC + i] = u2[u];
    }
}

// The reverse of tile_in: LDS block to global memory (an FP64 block into
// FP32 panels is rounded once, here).
template <typename T, typename U>
__device__ __forceinline__ void tile_out(T *__restrict__ dst, const U *src, int64_t ld, int nr, int w)
{
    const int i = threadIdx.x & 63, c0 = threadIdx.x >> 6;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int c = c0 + 4 * u;
        if (i < nr && c < w) dst[(int64_t)c * ld + i] = (T)src[c * LDC + i];
    }
}

// An FP32 tile (the first half of an FP64-sized LDS buffer) widened in place
// to FP64, for the diagonal factorization; called by all threads.  Every
// entry is read before any is written.
template <typename T>
__device__ __forceinline__ void widen_tile(double *buf)
{
    if constexpr (sizeof(T) == sizeof(float)) {
        const float *f = reinterpret_cast<const float *>(buf);
        const int i = threadIdx.x & 63, c0 = threadIdx.x >> 6;
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = f[(c0 + 4 * u) * LDC + i];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; ++u) buf[(c0 + 4 * u) * LDC + i] = (double)v[u];
        __syncthreads();
    }
}

// Kernels of the factorization take the value set (instance) of a batch
// from blockIdx.y: its panels start lx_stride entries after the previous
// instance's, its A values nnzA after, its status words 4 after.
template <typename T>
__global__ void k_fill_zero(T *__restrict__ x, int64_t count)
{
    x += blockIdx.y * count;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = T(0);
}

// Ax into the panels; with scaling (dscale != null) the entry (i, j) of
// P A P^T goes in as d_i a_ij d_j (acoord: its permuted row and column).
template <typename T>
__global__ void k_scatter_a(const double *__restrict__ Ax, const int64_t *__restrict__ amap,
                            T *__restrict__ Lx, int64_t nnz, int64_t lx_stride,
                            const double *__restrict__ dscale, const int32_t *__restrict__ acoord,
                            int32_t n)
{
    Ax += blockIdx.y * nnz;
    Lx += blockIdx.y * lx_stride;
    if (dscale) dscale += (int64_t)blockIdx.y * n;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * blockDim.x) {
        double v = Ax[k];
        if (dscale) v *= dscale[acoord[2 * k]] * dscale[acoord[2 * k + 1]];
        Lx[amap[k]] = (T)v;
    }
}

// Per-supernode scaling of the factored matrix: D = diag(d) with d_j =
// 2^-e_s for every column j of device supernode s, e_s = floor(E / 2) where
// 2^(E-1) <= max_{j in s} c_jj < 2^E (c_jj: the diagonal of P A P^T), so the
// largest diagonal entry of the supernode's columns in D P A P^T D lies in
// [1/2, 2).  Powers of two scale exactly.  The pivot floor of column j, if
// asked for, is tau times its diagonal entry in the scaled matrix.  One
// thread per device supernode; adiag[j]: index of c_jj in Ax (-1 if absent).
__global__ void k_super_scale(const double *__restrict__ Ax, const int64_t *__restrict__ adiag,
                              const int32_t *__restrict__ dsptr, int32_t nds, int64_t nnz,
                              int32_t n, double *__restrict__ dscale, double *__restrict__ pfloor,
                              double tau)
{
    Ax += blockIdx.y * nnz;
    dscale += (int64_t)blockIdx.y * n;
    if (pfloor) pfloor += (int64_t)blockIdx.y * n;
    for (int32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < nds; s += gridDim.x * blockDim.x) {
        double m = 0.0;
        for (int32_t j = dsptr[s]; j < dsptr[s + 1]; ++j)
            if (adiag[j] >= 0) m = fmax(m, Ax[adiag[j]]);
        double d = 1.0;
        if (m > 0.0 && m < __builtin_huge_val()) {
            int E = 0;
            (void)frexp(m, &E);
            const int e = E >= 0 ? E / 2 : -((1 - E) / 2);   // floor(E / 2)
            d = ldexp(1.0, -e);
        }
        for (int32_t j = dsptr[s]; j < dsptr[s + 1]; ++j) {
            dscale[j] = d;
            if (pfloor) pfloor[j] = adiag[j] >= 0 ? tau * (d * d) * Ax[adiag[j]] : 0.0;
        }
    }
}

__global__ void k_info_reset(int32_t *info)
{
    info += 4 * blockIdx.y;
    info[0] = INT32_MAX;
    info[1] = INT32_MAX;
    info[2] = 0;
    info[3] = 0;
}

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

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));
typedef _Float16 h4v __attribute__((ext_vector_type(4)));

// Operand format of the update products (external and internal updates):
// the panels' own type, or FP32 panel values rounded (to nearest even) to
// bfloat16 or IEEE half on their way to the 16-bit matrix cores, which
// accumulate in FP32.  The tiles, the diagonal factorization and the
// off-diagonal solves never leave the panels' precision (or FP64).
constexpr int kOpNative = 0, kOpBF16 = 1, kOpF16 = 2;

// acc += A B over four k-steps in one 16 x 16 x 16 matrix-core product:
// lane l supplies a[s] = A[l % 16][k_s(l)] and b[s] = B[k_s(l)][l % 16] for
// s < 4.  Any map of (s, l / 16) to 16 distinct inner indices is valid as
// long as both operands use the same one, so the four k-steps of the
// 16 x 16 x 4 form (k = 4 s + l / 16) go into one instruction unchanged.
template <int OP>
__device__ __forceinline__ f4 mma_pack(const float (&a)[4], const float (&b)[4], f4 c)
{
    if constexpr (OP == kOpBF16) {
        s4v x, y;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            x[i] = __builtin_bit_cast(short, (__bf16)a[i]);
            y[i] = __builtin_bit_cast(short, (__bf16)b[i]);
        }
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(x, y, c, 0, 0, 0);
    } else {
        h4v x, y;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            x[i] = (_Float16)a[i];
            y[i] = (_Float16)b[i];
        }
        return __builtin_amdgcn_mfma_f32_16x16x16f16(x, y, c, 0, 0, 0);
    }
}

// Four values of one row (or column) packed for mma_pack's operand, and the
// packed product of two such operands.
template <int OP>
__device__ __forceinline__ uint64_t pack4(const float (&v)[4])
{
    uint64_t r = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint16_t h;
        if constexpr (OP == kOpBF16) h = __builtin_bit_cast(uint16_t, (__bf16)v[i]);
        else h = __builtin_bit_cast(uint16_t, (_Float16)v[i]);
        r |= (uint64_t)h << (16 * i);
    }
    return r;
}
template <int OP>
__device__ __forceinline__ f4 mma_packed(uint64_t a, uint64_t b, f4 c)
{
    if constexpr (OP == kOpBF16)
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4v, a),
                                                         __builtin_bit_cast(s4v, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(h4v, a),
                                                     __builtin_bit_cast(h4v, b), c, 0, 0, 0);
}

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

// acc[m][n] -= A[rows, 0:wk] * B[cols, 0:wk]^T for the 32 x 32 quadrant
// (wr, wc), inner dimension wk of any length: the operands stream in chunks
// of 16 inner indices through two register stages (the next chunk is in
// flight while the current one is multiplied).  Loads are unconditional
// (addresses clamped into the valid rows, columns and inner range), so
// every chunk issues the same 16 loads and each product waits for its own
// chunk only; the inner range is masked at the product.
template <typename T>
struct Chunk16 {
    T a0[4], a1[4], b0[4], b1[4];
};
template <typename T, int OP, bool COH = false>
__device__ __forceinline__ void wave_product_pipe(const T *__restrict__ pa, const T *__restrict__ pb,
                                                  int64_t ld, int nI, int nJ, int wk, int wr, int wc,
                                                  typename Mfma<T>::acc_t (&acc)[2][2])
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const uint32_t ra0 = sizeof(T) * min(32 * wr + li, nI - 1);
    const uint32_t ra1 = sizeof(T) * min(32 * wr + 16 + li, nI - 1);
    const uint32_t cb0 = sizeof(T) * min(32 * wc + li, nJ - 1);
    const uint32_t cb1 = sizeof(T) * min(32 * wc + 16 + li, nJ - 1);
    const uint32_t ldb = sizeof(T) * (uint32_t)ld;
    const char *ca = reinterpret_cast<const char *>(pa);
    const char *cbp = reinterpret_cast<const char *>(pb);
    const __amdgpu_buffer_rsrc_t rsa = coherent_rsrc(pa), rsb = coherent_rsrc(pb);
    auto load = [&](Chunk16<T> &x, int kc) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const uint32_t ko = (uint32_t)min(kc + 4 * st + lk, wk - 1) * ldb;
            if constexpr (COH) {
                x.a0[st] = coherent_ld<T>(rsa, ra0 + ko);
                x.a1[st] = coherent_ld<T>(rsa, ra1 + ko);
                x.b0[st] = coherent_ld<T>(rsb, cb0 + ko);
                x.b1[st] = coherent_ld<T>(rsb, cb1 + ko);
            } else {
                x.a0[st] = *reinterpret_cast<const T *>(ca + (ra0 + ko));
                x.a1[st] = *reinterpret_cast<const T *>(ca + (ra1 + ko));
                x.b0[st] = *reinterpret_cast<const T *>(cbp + (cb0 + ko));
                x.b1[st] = *reinterpret_cast<const T *>(cbp + (cb1 + ko));
            }
        }
    };
    auto compute = [&](const Chunk16<T> &x, int kc) {
        if constexpr (OP == kOpNative) {
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const bool vk = kc + 4 * st + lk < wk;
                const T x0 = vk ? -x.a0[st] : T(0), x1 = vk ? -x.a1[st] : T(0);
                acc[0][0] = Mfma<T>::mma(x0, x.b0[st], acc[0][0]);
                acc[0][1] = Mfma<T>::mma(x0, x.b1[st], acc[0][1]);
                acc[1][0] = Mfma<T>::mma(x1, x.b0[st], acc[1][0]);
                acc[1][1] = Mfma<T>::mma(x1, x.b1[st], acc[1][1]);
            }
        } else {
            // the chunk's four k-steps in one 16-bit product per quadrant
            float x0[4], x1[4], y0[4], y1[4];
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const bool vk = kc + 4 * st + lk < wk;
                x0[st] = vk ? -x.a0[st] : 0.0f;
                x1[st] = vk ? -x.a1[st] : 0.0f;
                y0[st] = x.b0[st];
                y1[st] = x.b1[st];
            }
            acc[0][0] = mma_pack<OP>(x0, y0, acc[0][0]);
            acc[0][1] = mma_pack<OP>(x0, y1, acc[0][1]);
            acc[1][0] = mma_pack<OP>(x1, y0, acc[1][0]);
            acc[1][1] = mma_pack<OP>(x1, y1, acc[1][1]);
        }
    };
    // an even number of chunks (at least two); the last pair has no loads
    const int nq = max(2, ((wk + 31) >> 5) << 1);
    Chunk16<T> s0, s1;
    load(s0, 0);
    load(s1, 16);
    for (int q = 0; q < nq - 2; q += 2) {
        compute(s0, 16 * q);
        load(s0, 16 * (q + 2));
        compute(s1, 16 * (q + 1));
        load(s1, 16 * (q + 3));
    }
    compute(s0, 16 * (nq - 2));
    compute(s1, 16 * (nq - 1));
}

// Value of v in lane `src` (a compile-time or wave-uniform lane index).
__device__ __forceinline__ double lane_value(double v, int src)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_value(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Reciprocal square root of a pivot: the hardware estimate (about 24
// correct bits) refined by one third-order step of the series of
// (1 - e)^(-1/2), y <- y (1 + e/2 + 3 e^2/8) with e = 1 - d y^2: the
// truncation is O(e^3), far below rounding, so the result is within about
// one ulp, as after two Newton steps, with four dependent operations
// instead of six (it sits on the factorization's critical chain).  A
// non-positive or NaN pivot gives NaN or infinity, and the pivot check
// reports it.
__device__ __forceinline__ double pivot_rsqrt(double d)
{
    const double y = __builtin_amdgcn_rsq(d);
    const double e = fma(-d * y, y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
}
__device__ __forceinline__ float pivot_rsqrt(float d)
{
    float y = __builtin_amdgcn_rsqf(d);
    const float e = fmaf(-d * y, y, 1.0f);
    return fmaf(0.5f * y, e, y);
}

// One wavefront factors the 16-column sub-panel C[c0 : nr, c0 : c0 + wb]
// (LDS, column-major, stride LDC) in place: lane i holds row c0 + i in
// registers.  Column k: the pivot's reciprocal square root r scales the
// whole column (the diagonal entry d becomes d r), then the later columns
// take the rank-1 update (no barriers): the multiplier of column k + 1,
// which the next pivot waits for, is read across lanes; the others are
// broadcast through LDS (every lane stores its entry, with no branch, and
// reads the ones it needs), which keeps the cross-lane reads (two per
// value) off the issue path.  Rows c0 .. c0 + wb - 1 form the diagonal block (Cholesky);
// the rows below get the triangular solve against it.  No lane masks: the
// entries above the diagonal receive harmless updates (they are stored and
// never read).  Columns past wb start at zero, never feed the real ones
// (only later columns depend on a column) and are not stored.
// With a pivot floor (floor != null: floor[c] for the block's column c), a
// pivot below its column's floor is replaced by the floor (the factor is
// then that of a matrix with a slightly larger diagonal; the count of
// replacements goes to info[3]); a NaN pivot is never replaced.
template <typename T, bool FLOOR>
__device__ __forceinline__ void wave_subpanel(T *C, int c0, int wb, int nr, int col0,
                                              int32_t *info, const double *floor, double *bcast)
{
    const int lane = threadIdx.x & 63;
    const int row = c0 + lane;
    const bool mine = row < nr;
    double r[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) r[c] = (mine && c < wb) ? (double)C[(c0 + c) * LDC + row] : 0.0;
    const double fl = (FLOOR && floor) ? floor[c0 + min(lane & 15, wb - 1)] : 0.0;
    int bad = INT_MAX, nrep = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        double d = lane_value(r[k], k);
        if (FLOOR && floor) {
            const double f = lane_value(fl, k);
            if (k < wb && d < f) {
                if (lane == k) r[k] = f;
                d = f;
                ++nrep;
            }
        }
        bad = (k < wb && !(d > 0.0)) ? min(bad, col0 + c0 + k) : bad;
        r[k] *= pivot_rsqrt(d);
        if (k + 1 < 16) r[k + 1] = fma(-r[k], lane_value(r[k], k + 1), r[k + 1]);
        if (k + 2 < 16) {
            bcast[lane] = r[k];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
            for (int c = k + 2; c < 16; ++c) r[c] = fma(-r[k], bcast[c], r[c]);
            // the words are read before the next column overwrites them
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
    }
    if (bad != INT_MAX && lane == 0) atomicMin(info, bad);
    if (FLOOR && nrep && lane == 0) atomicAdd(info + 3, nrep);
#pragma unroll
    for (int c = 0; c < 16; ++c)
        if (mine && c < wb) C[(c0 + c) * LDC + row] = (T)r[c];
}

// One wavefront inverts the wb x wb lower triangle D[c0 .., c0 ..] (LDS,
// column-major, stride LDC; wb <= 16, and D is zero outside its w x w
// block), padded to 16 x 16 with the identity:
// lane j < 16 forms column j of the inverse by forward substitution, the
// triangle's entries being read as LDS broadcasts.  The result goes to M
// (M[c * 17 + k] = inverse[c][k]).
template <typename T>
__device__ __forceinline__ void wave_tri_inverse(const T *D, int c0, int wb, T *M)
{
    const int lane = threadIdx.x & 63;
    const int j = lane & 15;
    T m[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        T s0 = i == j ? T(1) : T(0), s1 = T(0);
#pragma unroll
        for (int k = 0; k < i; ++k) {
            const T lik = D[(c0 + k) * LDC + c0 + i];
            if (k & 1) s1 -= lik * m[k];
            else s0 -= lik * m[k];
        }
        const T dii = D[(c0 + i) * LDC + c0 + i];
        m[i] = (s0 + s1) / (i < wb ? dii : T(1));
    }
    if (lane < 16) {
#pragma unroll
        for (int i = 0; i < 16; ++i) M[i * 17 + j] = m[i];
    }
}

// One wavefront solves rows [rw, rw + 16) of X := X D^{-T} (X: nr x w tile,
// D: the w x w factored diagonal block, both LDS column-major with stride
// LDC) one 16-column block at a time with matrix cores: block j is
// (X_j - sum_{i<j} X_i D_ji^T) Minv_j^T, Minv_j the inverted diagonal block
// j (M + 272 j).  A wavefront touches only its own rows, so the blocks need
// no barriers: its LDS writes are ordered before its later reads.
template <typename T>
__device__ __forceinline__ void wave_rows_solve(T *X, const T *D, const T *M, int rw, int w)
{
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, kq = lane >> 4;
    for (int cb = 0; cb < w; cb += 16) {
        typename Mfma<T>::acc_t acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = X[(cb + li) * LDC + rw + Mfma<T>::row(lane, v)];
        for (int ib = 0; ib < cb; ib += 16) {
#pragma unroll
            for (int ks = 0; ks < 16; ks += 4) {
                const T a = X[(ib + ks + kq) * LDC + rw + li];
                const T b = D[(ib + ks + kq) * LDC + cb + li];
                acc = Mfma<T>::mma(-a, b, acc);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) X[(cb + li) * LDC + rw + Mfma<T>::row(lane, v)] = acc[v];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const T *Mj = M + 272 * (cb >> 4);
        typename Mfma<T>::acc_t y = {};
#pragma unroll
        for (int ks = 0; ks < 16; ks += 4) {
            const T a = X[(cb + ks + kq) * LDC + rw + li];
            const T b = Mj[li * 17 + ks + kq];
            y = Mfma<T>::mma(a, b, y);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
        for (int v = 0; v < 4; ++v) X[(cb + li) * LDC + rw + Mfma<T>::row(lane, v)] = y[v];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_sched_barrier(0);
    }
}

// C[ra:nr, ca:w] -= X[ra:nr, k0:k0+kw] * Y[ca:w, k0:k0+kw]^T in 16 x 16
// matrix-core blocks shared by the four wavefronts.  X, Y and C are LDS
// panels (column-major, stride LDC); kw <= 16.  When rows and columns index
// the same panel (diag_off = 0), blocks entirely above the diagonal are
// skipped and entries above it inside a block receive harmless updates to
// never-read storage; a diag_off of 64 or more disables the skipping.
template <typename T>
__device__ __forceinline__ void block_update(T *C, const T *X, const T *Y, int ra, int nr,
                                             int ca, int w, int k0, int kw, int diag_off,
                                             int wave0 = 0)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nrb = (nr - ra + 15) >> 4;
    const int ncb = (w - ca + 15) >> 4;
    // blocks are shared by the wavefronts wave0 .. NT / 64 - 1
    if (wave < wave0) return;
    for (int blk = wave - wave0; blk < nrb * ncb; blk += NT / 64 - wave0) {
        const int rb = ra + 16 * (blk % nrb);
        const int cb = ca + 16 * (blk / nrb);
        if (rb + 15 + diag_off < cb) continue;
        typename Mfma<T>::acc_t acc = {};
        const int ar = rb + (lane & 15);
        const int bc = cb + (lane & 15);
#pragma unroll
        for (int ks = 0; ks < 16; ks += 4) {
            const int k = ks + (lane >> 4);
            const bool vk = k < kw;
            const T a = (vk && ar < nr) ? X[(k0 + k) * LDC + ar] : T(0);
            const T b = (vk && bc < w) ? Y[(k0 + k) * LDC + bc] : T(0);
            acc = Mfma<T>::mma(a, b, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = rb + Mfma<T>::row(lane, v);
            const int c = cb + (lane & 15);
            if (r < nr && c < w) C[c * LDC + r] -= acc[v];
        }
    }
}

// Cholesky of an nr x w panel (nr, w <= 64) held column-major in LDS:
// rows [0, w) are the diagonal block, rows [w, nr) the rows below it (their
// triangular solve is part of the same sweep).  Blocked by 16 columns with
// look-ahead: once sub-panel j is factored, all four wavefronts apply its
// update to sub-panel j + 1's columns; then wavefront 0 factors sub-panel
// j + 1 while wavefronts 1..3 apply sub-panel j's update to the columns
// beyond it (matrix-core products).  Every column still receives the
// sub-panels' updates in order.  Called by all threads of the workgroup.
// Every factorization of a diagonal block runs here in FP64 (FP32 panels
// are widened into an FP64 tile first and rounded once when stored).  The
// pivot floor exists only where FLOOR is set (the 16-bit update precisions).
template <bool FLOOR, typename T>
__device__ __forceinline__ void panel_factor(T *C, int nr, int w, int col0, int32_t *info,
                                             const double *floor)
{
    __shared__ double bcast[64];        // the sub-panel's column broadcasts
    const int wave = threadIdx.x >> 6;
    if (wave == 0) wave_subpanel<T, FLOOR>(C, 0, min(16, w), nr, col0, info, floor, bcast);
    __syncthreads();
    for (int c0 = 16; c0 < w; c0 += 16) {
        const int wb = min(16, w - c0);
        block_update(C, C, C, c0, nr, c0, c0 + wb, c0 - 16, 16, 0);
        __syncthreads();
        if (wave == 0)
            wave_subpanel<T, FLOOR>(C, c0, wb, nr, col0, info, floor, bcast);
        else if (c0 + wb < w)
            block_update(C, C, C, c0 + wb, nr, c0 + wb, w, c0 - 16, 16, 0, 1);
        __syncthreads();
    }
}

// External update of one row tile of block J: for every descendant K of
// another supernode that meets the tile, tile -= L_K[b0 .. b0+nI, :] *
// L_K[a0 .. a0+nJ, :]^T at the tile-relative rows and columns recorded by the
// analysis.  The tile stays in LDS.  Wavefront w owns tile columns
// [16w, 16w + 16) and walks the incidence list on its own: it skips
// incidences whose columns miss its range, otherwise forms the product of
// all nI rows with its (at most 16) columns on the matrix cores and
// subtracts it from its own columns.  No two wavefronts write the same
// entry, so the loop has no barriers and each entry is updated in list
// order (bitwise reproducible).  The next record is fetched one iteration
// ahead.  With kFuseFactor the tile is tile 0 of a supernode's first block,
// which is then factored in place.
// Large incidences of one tile, by the whole workgroup: the product's
// inner dimension is walked in chunks of KC staged through double-buffered
// LDS, each thread keeping the loads of the next two chunks in flight in
// registers; wavefront (wr, wc) owns the 32 x 32 quadrant (wr, wc) of the
// 64 x 64 product and subtracts it at the relative positions.  One barrier
// per chunk.  With KC = 8 the staging buffers are small enough for three
// workgroups per CU.
template <typename T, int KC>
__device__ __forceinline__ void load_chunk(T (&va)[KC / 4], T (&vb)[KC / 4], const T *__restrict__ LK,
                                           const Incidence &in, int kc)
{
    const int r = threadIdx.x & 63, kq = threadIdx.x >> 6;
    const int64_t ld = in.ld;
#pragma unroll
    for (int j = 0; j < KC / 4; ++j) {
        const int k = kc + kq + 4 * j;
        const bool vk = k < in.wk;
        const int64_t ko = vk ? (int64_t)k * ld : 0;
        const bool oa = vk && r < in.nI, ob = vk && r < in.nJ;
        const T x = LK[in.b0 + (oa ? r : 0) + ko];
        const T y = LK[in.a0 + (ob ? r : 0) + ko];
        va[j] = oa ? x : T(0);
        vb[j] = ob ? y : T(0);
    }
}

template <typename T, int KC>
__device__ __forceinline__ void coop_product(T *C, T (*As)[KC][64], T (*Bs)[KC][64], int32_t *s_rel,
                                             const Incidence &in, const uint8_t *__restrict__ imap,
                                             const T *__restrict__ Lx, int r0, int nr, int w)
{
    constexpr int J4 = KC / 4;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int r = tid & 63, kq = tid >> 6;
    const T *LK = Lx + in.valoff;
    const int nI = in.nI, nJ = in.nJ;
    const uint8_t *mp = imap + in.mapoff;
    if (tid < 64) s_rel[tid] = tid < nI ? (int)mp[tid] : 0;
    else if (tid < 128) s_rel[tid] = tid - 64 < nJ ? (int)mp[nI + tid - 64] : 0;
    const int nch = (in.wk + KC - 1) / KC;
    T pa[2][J4], pb[2][J4];
    load_chunk<T, KC>(pa[0], pb[0], LK, in, 0);
    if (nch > 1) load_chunk<T, KC>(pa[1], pb[1], LK, in, KC);
#pragma unroll
    for (int j = 0; j < J4; ++j) {
        As[0][kq + 4 * j][r] = pa[0][j];
        Bs[0][kq + 4 * j][r] = pb[0][j];
    }
    if (nch > 2) load_chunk<T, KC>(pa[0], pb[0], LK, in, 2 * KC);
    __syncthreads();
    const bool active = 32 * wr < nI && 32 * wc < nJ;
    // 16-row and 16-column blocks of the quadrant past the product's extent
    // are skipped (wave-uniform conditions)
    const bool a1v = 32 * wr + 16 < nI, b1v = 32 * wc + 16 < nJ;
    typename Mfma<T>::acc_t acc[2][2] = {};
    const int li = lane & 15;
    for (int c = 0; c < nch; ++c) {
        const int buf = c & 1;
        if (active) {
#pragma unroll
            for (int st = 0; st < KC / 4; ++st) {
                const int kl = 4 * st + (lane >> 4);
                const T a0 = As[buf][kl][32 * wr + li];
                const T a1 = As[buf][kl][32 * wr + 16 + li];
                const T b0 = Bs[buf][kl][32 * wc + li];
                const T b1 = Bs[buf][kl][32 * wc + 16 + li];
                acc[0][0] = Mfma<T>::mma(a0, b0, acc[0][0]);
                if (b1v) acc[0][1] = Mfma<T>::mma(a0, b1, acc[0][1]);
                if (a1v) acc[1][0] = Mfma<T>::mma(a1, b0, acc[1][0]);
                if (a1v && b1v) acc[1][1] = Mfma<T>::mma(a1, b1, acc[1][1]);
            }
        }
        if (c + 1 < nch) {
            // chunk c+1 sits in register stage (c+1) & 1; its buffer was last
            // read in iteration c-1, before the previous barrier
            const int rs = (c + 1) & 1;
#pragma unroll
            for (int j = 0; j < J4; ++j) {
                As[buf ^ 1][kq + 4 * j][r] = pa[rs][j];
                Bs[buf ^ 1][kq + 4 * j][r] = pb[rs][j];
            }
            if (c + 3 < nch) load_chunk<T, KC>(pa[rs], pb[rs], LK, in, KC * (c + 3));
        }
        __syncthreads();
    }
    if (active) {
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n2 = 0; n2 < 2; ++n2) {
                const int col = 32 * wc + 16 * n2 + li;
                const int Cc = s_rel[64 + (col < 64 ? col : 0)];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 32 * wr + 16 * m + Mfma<T>::row(lane, v);
                    if (row < nI && col < nJ) {
                        const int R = s_rel[row];
                        if (R < nr && Cc < w && r0 + R >= Cc) C[Cc * LDC + R] -= acc[m][n2][v];
                    }
                }
            }
    }
    __syncthreads();
}

// The same product with the operands on the 16-bit matrix cores (FP32
// panels): chunks of 16 inner indices; thread (r, kq) loads row r's values
// at k = kc + kq + 4 j (j < 4) -- exactly the four k-steps that lane
// 16 kq + r % 16 of a wavefront supplies to one 16 x 16 x 16 product -- and
// stores them packed (8 bytes) at stage[kq][r], so a wavefront's operand is
// one LDS read.  Rows and columns past the product's extent and inner
// indices past wk are zero in the stage.
template <int OP>
__device__ __forceinline__ void stage_packed(uint64_t (*As)[64], uint64_t (*Bs)[64],
                                             const float (&va)[4], const float (&vb)[4])
{
    const int r = threadIdx.x & 63, kq = threadIdx.x >> 6;
    As[kq][r] = pack4<OP>(va);
    Bs[kq][r] = pack4<OP>(vb);
}

template <int OP>
__device__ __forceinline__ void coop_product_packed(float *C, uint64_t (*As)[4][64],
                                                    uint64_t (*Bs)[4][64], int32_t *s_rel,
                                                    const Incidence &in,
                                                    const uint8_t *__restrict__ imap,
                                                    const float *__restrict__ Lx, int r0, int nr,
                                                    int w)
{
    constexpr int KC = 16;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const float *LK = Lx + in.valoff;
    const int nI = in.nI, nJ = in.nJ;
    const uint8_t *mp = imap + in.mapoff;
    if (tid < 64) s_rel[tid] = tid < nI ? (int)mp[tid] : 0;
    else if (tid < 128) s_rel[tid] = tid - 64 < nJ ? (int)mp[nI + tid - 64] : 0;
    const int nch = (in.wk + KC - 1) / KC;
    float pa[2][4], pb[2][4];
    load_chunk<float, KC>(pa[0], pb[0], LK, in, 0);
    if (nch > 1) load_chunk<float, KC>(pa[1], pb[1], LK, in, KC);
    stage_packed<OP>(As[0], Bs[0], pa[0], pb[0]);
    if (nch > 2) load_chunk<float, KC>(pa[0], pb[0], LK, in, 2 * KC);
    __syncthreads();
    const bool active = 32 * wr < nI && 32 * wc < nJ;
    const bool a1v = 32 * wr + 16 < nI, b1v = 32 * wc + 16 < nJ;
    f4 acc[2][2] = {};
    const int li = lane & 15, g = lane >> 4;
    for (int c = 0; c < nch; ++c) {
        const int buf = c & 1;
        if (active) {
            const uint64_t a0 = As[buf][g][32 * wr + li];
            const uint64_t a1 = As[buf][g][32 * wr + 16 + li];
            const uint64_t b0 = Bs[buf][g][32 * wc + li];
            const uint64_t b1 = Bs[buf][g][32 * wc + 16 + li];
            acc[0][0] = mma_packed<OP>(a0, b0, acc[0][0]);
            if (b1v) acc[0][1] = mma_packed<OP>(a0, b1, acc[0][1]);
            if (a1v) acc[1][0] = mma_packed<OP>(a1, b0, acc[1][0]);
            if (a1v && b1v) acc[1][1] = mma_packed<OP>(a1, b1, acc[1][1]);
        }
        if (c + 1 < nch) {
            const int rs = (c + 1) & 1;
            stage_packed<OP>(As[buf ^ 1], Bs[buf ^ 1], pa[rs], pb[rs]);
            if (c + 3 < nch) load_chunk<float, KC>(pa[rs], pb[rs], LK, in, KC * (c + 3));
        }
        __syncthreads();
    }
    if (active) {
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n2 = 0; n2 < 2; ++n2) {
                const int col = 32 * wc + 16 * n2 + li;
                const int Cc = s_rel[64 + (col < 64 ? col : 0)];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 32 * wr + 16 * m + Mfma<float>::row(lane, v);
                    if (row < nI && col < nJ) {
                        const int R = s_rel[row];
                        if (R < nr && Cc < w && r0 + R >= Cc) C[Cc * LDC + R] -= acc[m][n2][v];
                    }
                }
            }
    }
    __syncthreads();
}

// ---- wavefront items (small incidences)
//
// A wavefront runs its item list as up to four streams of operand batches,
// one per group of items with the same number NRB of 16-row blocks (the
// analysis groups them), so that no load or product is spent on row blocks
// an item does not have.  A batch covers kSteps k-steps of 4 (k = 4 (kb +
// s) + l / 16 for lane l): per step NRB A values (product rows 16m + l % 16,
// m < NRB) and one B value (product column l % 16).  Addresses are clamped
// into the item's rows, columns and
// k range, so every load is in bounds, none depends on another load's value
// and every batch issues the same loads unconditionally (the hardware's
// in-order load counter then lets the products of one batch wait for that
// batch alone): the k range is masked at the product, and rows and columns
// past the item's are dropped by the scatter.  The batch after the current
// one is always in flight while the current one is multiplied (two register
// sets used in turn), and the next item's record is fetched one item ahead.
constexpr int kSteps = 4;

// An item's record, read as whole dwords so that it can stay in scalar
// registers.
struct Item {
    int64_t valoff, mapoff;
    int ld, b0, a0, wk, nI, nJ;
};

__device__ __forceinline__ Item load_item(const WaveItem *__restrict__ items, int64_t i)
{
    const uint32_t *d = reinterpret_cast<const uint32_t *>(items + i);
    uint32_t x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = d[u];
    Item it;
    it.valoff = (int64_t)(((uint64_t)x[1] << 32) | x[0]);
    it.mapoff = (int64_t)(((uint64_t)x[3] << 32) | x[2]);
    it.ld = (int)x[4];
    it.b0 = (int)x[5];
    it.a0 = (int)x[6];
    it.wk = (int)(int16_t)(x[7] & 0xffffu);
    it.nI = (int)((x[7] >> 16) & 0xffu);
    it.nJ = (int)(x[7] >> 24);
    return it;
}

template <typename T, int NRB>
struct Batch {
    T a[kSteps][NRB];
    T b[kSteps];
    int lr, cc;         // tile row of product row `lane`, tile column of product column lane % 16
};

// The loads of one batch of an item with NRB blocks of 16 product rows.
template <typename T, int NRB>
__device__ __forceinline__ void issue(Batch<T, NRB> &r, const T *__restrict__ Lx,
                                      const uint8_t *__restrict__ wmap, const Item &it, int kb,
                                      int lane)
{
    const T *LK = Lx + it.valoff;
    const uint8_t *mp = wmap + it.mapoff;
    const int li = lane & 15, kq = lane >> 4;
    r.lr = mp[min(lane, it.nI - 1)];
    r.cc = mp[it.nI + min(li, it.nJ - 1)];
    // 32-bit byte offsets from the uniform panel base (a panel is far below
    // 4 GiB), so the loads take the scalar-base addressing form
    const char *base = reinterpret_cast<const char *>(LK);
    const uint32_t ldb = sizeof(T) * (uint32_t)it.ld;
    const int wk1 = it.wk - 1;
    const uint32_t ob = sizeof(T) * (uint32_t)(it.a0 + min(li, it.nJ - 1));
    uint32_t oa[NRB];
#pragma unroll
    for (int m = 0; m < NRB; ++m) oa[m] = sizeof(T) * (uint32_t)(it.b0 + min(16 * m + li, it.nI - 1));
#pragma unroll
    for (int s = 0; s < kSteps; ++s) {
        const uint32_t ko = (uint32_t)min(4 * (kb + s) + kq, wk1) * ldb;
#pragma unroll
        for (int m = 0; m < NRB; ++m) r.a[s][m] = *reinterpret_cast<const T *>(base + (oa[m] + ko));
        r.b[s] = *reinterpret_cast<const T *>(base + (ob + ko));
    }
}

template <typename T, int OP, int NRB>
__device__ __forceinline__ void compute(const Batch<T, NRB> &r, typename Mfma<T>::acc_t (&acc)[NRB],
                                        const Item &it, int kb, int lane)
{
    if constexpr (OP == kOpNative) {
#pragma unroll
        for (int s = 0; s < kSteps; ++s) {
            if (4 * (kb + s) < it.wk) {
                const bool vk = 4 * (kb + s) + (lane >> 4) < it.wk;
                const T b = vk ? r.b[s] : T(0);
#pragma unroll
                for (int m = 0; m < NRB; ++m) acc[m] = Mfma<T>::mma(r.a[s][m], b, acc[m]);
            }
        }
    } else {
        // the batch's four k-steps in one 16-bit product per row block
        // (a batch exists only while 4 kb < wk)
        static_assert(kSteps == 4, "one 16-bit product covers four k-steps");
        float b[4];
#pragma unroll
        for (int s = 0; s < kSteps; ++s) b[s] = 4 * (kb + s) + (lane >> 4) < it.wk ? r.b[s] : 0.0f;
#pragma unroll
        for (int m = 0; m < NRB; ++m) {
            const float a[4] = {r.a[0][m], r.a[1][m], r.a[2][m], r.a[3][m]};
            acc[m] = mma_pack<OP>(a, b, acc[m]);
        }
    }
}

// Subtract an item's finished product from the LDS tile and clear the
// accumulators.  The tile row of product row i is lane i's lr; the tile
// column of lane l's products is its own cc.
template <typename T, int NRB>
__device__ __forceinline__ void scatter(T *C, typename Mfma<T>::acc_t (&acc)[NRB],
                                        const Batch<T, NRB> &r, const Item &it, int r0, int nr,
                                        int w, int lane)
{
    const int cc = r.cc;
    const bool vc = (lane & 15) < it.nJ && cc < w;
#pragma unroll
    for (int m = 0; m < NRB; ++m) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * m + Mfma<T>::row(lane, v);
            const int R = __shfl(r.lr, row);
            if (vc && row < it.nI && R < nr && r0 + R >= cc) C[cc * LDC + R] -= acc[m][v];
        }
        acc[m] = typename Mfma<T>::acc_t{};
    }
}

// One wavefront's items of NRB blocks of 16 product rows each (the items
// of a group have 16 NRB - 15 to 16 NRB rows), as one pipelined stream.
template <typename T, int OP, int NRB>
__device__ __forceinline__ void wave_items(T *C, const WaveItem *__restrict__ items,
                                           const uint8_t *__restrict__ wmap,
                                           const T *__restrict__ Lx, int64_t i0, int64_t i1, int r0,
                                           int nr, int w)
{
    const int lane = threadIdx.x & 63;
    Batch<T, NRB> X, Y;
    typename Mfma<T>::acc_t acc[NRB] = {};
    Item cur = load_item(items, i0);
    int64_t inx = i0 + 1;                  // index of the prefetched record `nxt`
    Item nxt = load_item(items, min(inx, i1 - 1));
    int kb = 0;                            // first k-step of the batch being multiplied
    issue(X, Lx, wmap, cur, 0, lane);
    // multiply batch P (item cur, k-steps from kb) while the following batch
    // loads into Q (after the last batch, a harmless reload); false once P
    // was the last batch
    auto step = [&](Batch<T, NRB> &P, Batch<T, NRB> &Q) -> bool {
        const bool same = 4 * (kb + kSteps) < cur.wk;
        const bool more = same || inx < i1;
        const Item ni = same ? cur : nxt;
        const int nkb = same ? kb + kSteps : 0;
        issue(Q, Lx, wmap, ni, nkb, lane);
        if (!same) {
            ++inx;
            nxt = load_item(items, min(inx, i1 - 1));
        }
        compute<T, OP, NRB>(P, acc, cur, kb, lane);
        if (!same) scatter(C, acc, P, cur, r0, nr, w, lane);
        cur = ni;
        kb = nkb;
        return more;
    };
    while (step(X, Y) && step(Y, X)) {
    }
}

// ---- staged products
//
// A staged tile runs its incidences as one stream of chunks (at most
// kStageK inner indices of one incidence each; StageChunk).  Per chunk the
// whole workgroup stages K's product rows for the chunk's inner indices in
// LDS (thread (r, q) loads row r at inner indices q, q + 4, q + 8, q + 12),
// so each row value is read from memory once per tile; then wavefront v
// multiplies all product rows with the product columns landing in its 16
// tile columns (its slice of K's column rows, read by its own lanes) and
// accumulates over the incidence's chunks; after the incidence's last chunk
// it subtracts the product from its own tile columns.  Wavefronts write
// disjoint columns, so no barrier separates incidences; one barrier per
// chunk guards the double-buffered stage.  The next chunk's rows and
// columns are loaded while the current one is multiplied.

// A chunk record, read as whole dwords (scalar registers).
struct Chunk {
    int64_t valoff;
    int ld, b0, a0, kc, nI, nJ, nk, last, jlo, jhi;
    uint32_t map;
};

__device__ __forceinline__ Chunk load_chunk_rec(const StageChunk *__restrict__ ch, int64_t i, int wave)
{
    const uint32_t *d = reinterpret_cast<const uint32_t *>(ch + i);
    uint32_t x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = d[u];
    Chunk c;
    c.valoff = (int64_t)(((uint64_t)x[1] << 32) | x[0]);
    c.ld = (int)x[2];
    c.b0 = (int)x[3];
    c.a0 = (int)x[4];
    c.map = x[5];
    c.kc = (int)(int16_t)(x[6] & 0xffffu);
    c.nI = (int)((x[6] >> 16) & 0xffu);
    c.nJ = (int)(x[6] >> 24);
    c.nk = (int)(x[7] & 0x7fu);
    c.last = (int)((x[7] >> 7) & 1u);
    const int j1 = (int)((x[7] >> 8) & 0xffu), j2 = (int)((x[7] >> 16) & 0xffu), j3 = (int)(x[7] >> 24);
    c.jlo = wave == 0 ? 0 : wave == 1 ? j1 : wave == 2 ? j2 : j3;
    c.jhi = wave == 0 ? j1 : wave == 1 ? j2 : wave == 2 ? j3 : c.nJ;
    return c;
}

// This thread's four staged values of chunk c: row r = lane, inner indices
// q + 4 j (q = wavefront); zero outside the rows and the chunk (addresses
// clamped into them).
template <typename T>
__device__ __forceinline__ void stage_load(T (&va)[4], const T *__restrict__ Lx, const Chunk &c)
{
    const int r = threadIdx.x & 63, q = threadIdx.x >> 6;
    const T *LK = Lx + c.valoff;
    const int rr = min(r, c.nI - 1);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = q + 4 * j;
        const T x = LK[(int64_t)(c.kc + min(k, c.nk - 1)) * c.ld + c.b0 + rr];
        va[j] = (r < c.nI && k < c.nk) ? x : T(0);
    }
}

// This lane's column operand of chunk c for its wavefront: product column
// jlo + lane % 16 (clamped) at inner index 4 s + lane / 16, s < 4, zero
// past the chunk.
template <typename T>
__device__ __forceinline__ void stage_cols(T (&vb)[4], const T *__restrict__ Lx, const Chunk &c)
{
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const T *LK = Lx + c.valoff;
    const int j = c.jlo + min(li, max(c.jhi - c.jlo, 1) - 1);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k = 4 * s + lk;
        const T x = LK[(int64_t)(c.kc + min(k, c.nk - 1)) * c.ld + c.a0 + min(j, c.nJ - 1)];
        vb[s] = k < c.nk ? x : T(0);
    }
}

// The tile rows (lane i: product row i) and this lane's tile column of the
// incidence of chunk c.
__device__ __forceinline__ void stage_maps(int &lr, int &cc, const uint8_t *__restrict__ imap, const Chunk &c)
{
    const int lane = threadIdx.x & 63, li = lane & 15;
    const uint8_t *mp = imap + c.map;
    lr = mp[min(lane, c.nI - 1)];
    cc = mp[c.nI + min(c.jlo + li, c.nJ - 1)];
}

template <typename T, int OP>
__device__ __forceinline__ void staged_products(T *C, T (*As)[kStageK][64], const StageChunk *__restrict__ ch,
                                                int64_t c0, int64_t c1, const uint8_t *__restrict__ imap,
                                                const T *__restrict__ Lx, int r0, int nr, int w)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (c0 >= c1) return;
    // X: the chunk being multiplied (staged in As[buf]); Y: the next one
    Chunk X = load_chunk_rec(ch, c0, wave);
    T va[4], vb[4], vbn[4];
    stage_load(va, Lx, X);
#pragma unroll
    for (int j = 0; j < 4; ++j) As[0][(tid >> 6) + 4 * j][lane] = va[j];
    stage_cols(vb, Lx, X);
    int lr = 0, cc = 0, lrn = 0, ccn = 0;
    if (X.last) stage_maps(lr, cc, imap, X);
    int64_t i = c0;
    Chunk Y = load_chunk_rec(ch, min(i + 1, c1 - 1), wave);
    __syncthreads();
    typename Mfma<T>::acc_t acc[4] = {};
    for (;;) {
        const int buf = (int)(i - c0) & 1;
        const bool more = i + 1 < c1;
        // the next chunk's rows, columns and (at its incidence's end) maps
        if (more) {
            stage_load(va, Lx, Y);
            stage_cols(vbn, Lx, Y);
            if (Y.last) stage_maps(lrn, ccn, imap, Y);
        }
        const Chunk Z = load_chunk_rec(ch, min(i + 2, c1 - 1), wave);
        // multiply X: this wavefront's columns with every product row
        const int nrb = (X.nI + 15) >> 4;
        if (X.jhi > X.jlo) {
            if constexpr (OP == kOpNative) {
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2) {
                    if (4 * s2 < X.nk) {
#pragma unroll
                        for (int m = 0; m < 4; ++m)
                            if (m < nrb) acc[m] = Mfma<T>::mma(As[buf][4 * s2 + lk][16 * m + li], vb[s2], acc[m]);
                    }
                }
            } else {
                const float b4[4] = {vb[0], vb[1], vb[2], vb[3]};
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    if (m < nrb) {
                        const float a4[4] = {As[buf][lk][16 * m + li], As[buf][4 + lk][16 * m + li],
                                             As[buf][8 + lk][16 * m + li], As[buf][12 + lk][16 * m + li]};
                        acc[m] = mma_pack<OP>(a4, b4, acc[m]);
                    }
                }
            }
        }
        if (X.last) {
            // subtract the finished product from this wavefront's tile columns
            const int nc = X.jhi - X.jlo;
            const bool vc = li < nc && cc < w;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                if (m < nrb) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = 16 * m + Mfma<T>::row(lane, v);
                        const int R = __shfl(lr, row);
                        if (vc && row < X.nI && R < nr && r0 + R >= cc) C[cc * LDC + R] -= acc[m][v];
                    }
                }
                acc[m] = typename Mfma<T>::acc_t{};
            }
        }
        if (!more) break;
        // stage the next chunk in the other buffer (last read before the
        // previous barrier), then let every wavefront see it
#pragma unroll
        for (int j = 0; j < 4; ++j) As[buf ^ 1][(tid >> 6) + 4 * j][lane] = va[j];
        __syncthreads();
        ++i;
        X = Y;
        Y = Z;
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) vb[s2] = vbn[s2];
        lr = lrn;
        cc = ccn;
    }
}

template <typename T, bool COOP, int OP>
__global__ __launch_bounds__(NT, 3) void k_external(const Task *__restrict__ tasks,
                                                 const int64_t *__restrict__ iptr,
                                                 const int64_t *__restrict__ ibig,
                                                 const Incidence *__restrict__ incs,
                                                 const uint8_t *__restrict__ imap,
                                                 const int64_t *__restrict__ wptr,
                                                 const WaveItem *__restrict__ witems,
                                                 const uint8_t *__restrict__ wmap,
                                                 const BlockDesc *__restrict__ blk,
                                                 T *__restrict__ Lx, int32_t *__restrict__ info,
                                                 int64_t lx_stride,
                                                 unsigned long long *__restrict__ ttime,
                                                 const PartDesc *__restrict__ parts,
                                                 int32_t *pcount, T *pbuf, int32_t nsplit,
                                                 int64_t npartial, const double *__restrict__ pfloor,
                                                 int32_t n, const int64_t *__restrict__ cptr,
                                                 const StageChunk *__restrict__ chunks,
                                                 const int32_t *__restrict__ xslot)
{
    const unsigned long long t_start = ttime ? wall_clock64() : 0ull;
    // the tile, in the panels' precision; FP64-sized so that a fused
    // diagonal factorization can widen it in place
    __shared__ double Cbuf[64 * LDC];
    T *C = reinterpret_cast<T *>(Cbuf);
    // operand staging of the cooperative and the staged products (one or
    // the other per tile)
    __shared__ double stage_mem[2 * kStageK * 64];
    Lx += blockIdx.y * lx_stride;
    info += 4 * blockIdx.y;
    pcount += (int64_t)blockIdx.y * nsplit;
    pbuf += (int64_t)blockIdx.y * npartial * 4096;
    if (pfloor) pfloor += (int64_t)blockIdx.y * n;
    __shared__ int32_t s_rel[COOP ? 128 : 1];
    __shared__ int s_last;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    // this workgroup slot's task, or its narrow tiles
    const int32_t e0 = xslot[blockIdx.x], e1 = xslot[blockIdx.x + 1] & INT32_MAX;
    const int32_t tq = e0 & INT32_MAX;
    if (e0 < 0) {
        // up to four tiles of blocks of at most 16 columns, one per
        // wavefront, in its own 16 LDS columns: the tile, its item stream
        // (a narrow tile's products all belong to the first wavefront's
        // columns), then with kFuseFactor the diagonal factorization in
        // FP64; the whole-workgroup path's steps, so the same values.  No
        // barriers.
        const int wv = __builtin_amdgcn_readfirstlane(wave);
        const int32_t q = tq + wv;
        if (q >= e1) return;
        double *Cw = Cbuf + wv * 16 * LDC;
        T *Cn = reinterpret_cast<T *>(Cw);
        const Task tk = tasks[q];
        const BlockDesc J = blk[tk.J];
        const int r0 = tk.t * TR;
        const int nr = min(TR, J.r - r0);
        const int w = min(J.w, 16);
        T *LJ = Lx + J.valoff;
#pragma unroll
        for (int c = 0; c < 16; ++c)
            Cn[c * LDC + lane] = (lane < nr && c < w) ? LJ[(int64_t)c * J.ld + r0 + lane] : T(0);
        const int64_t *wg = wptr + 16 * q;
        if (wg[0] < wg[1]) wave_items<T, OP, 4>(Cn, witems, wmap, (const T *)Lx, wg[0], wg[1], r0, nr, w);
        if (wg[1] < wg[2]) wave_items<T, OP, 3>(Cn, witems, wmap, (const T *)Lx, wg[1], wg[2], r0, nr, w);
        if (wg[2] < wg[3]) wave_items<T, OP, 2>(Cn, witems, wmap, (const T *)Lx, wg[2], wg[3], r0, nr, w);
        if (wg[3] < wg[4]) wave_items<T, OP, 1>(Cn, witems, wmap, (const T *)Lx, wg[3], wg[4], r0, nr, w);
        if (tk.flags & kFuseFactor) {
            if constexpr (sizeof(T) != sizeof(double)) {
                T v[16];
#pragma unroll
                for (int c = 0; c < 16; ++c) v[c] = Cn[c * LDC + lane];
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
                for (int c = 0; c < 16; ++c) Cw[c * LDC + lane] = (double)v[c];
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
            wave_subpanel<double, OP != kOpNative>(Cw, 0, w, nr, J.col0, info,
                                                   pfloor ? pfloor + J.col0 : nullptr, stage_mem + 64 * wv);
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (lane < nr && c < w) LJ[(int64_t)c * J.ld + r0 + lane] = (T)Cw[c * LDC + lane];
        } else {
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (lane < nr && c < w) LJ[(int64_t)c * J.ld + r0 + lane] = Cn[c * LDC + lane];
        }
        if (ttime && blockIdx.y == 0 && lane == 0) ttime[q] = wall_clock64() - t_start;
        return;
    }
    const Task tk = tasks[tq];
    const BlockDesc J = blk[tk.J];
    const int r0 = tk.t * TR;
    const int nr = min(TR, J.r - r0);
    const int w = J.w;
    T *LJ = Lx + J.valoff;
    const bool partial = (tk.flags & kPartial) != 0;

    // a part of a split tile accumulates from zero; other tiles from their values
    if (partial) {
        for (int k = tid; k < 64 * LDC; k += NT) C[k] = T(0);
    } else {
        tile_in(C, LJ + r0, J.ld, nr, w);
    }
    __syncthreads();

    int64_t q = iptr[tq];
    if (tk.flags & kStaged) {
        staged_products<T, OP>(C, reinterpret_cast<T(*)[kStageK][64]>(stage_mem), chunks, cptr[tq],
                               cptr[tq + 1], imap, (const T *)Lx, r0, nr, w);
    } else if constexpr (COOP && OP == kOpNative) {
        constexpr int KC = 8;   // inner indices per staged chunk of the cooperative product
        T(*As)[KC][64] = reinterpret_cast<T(*)[KC][64]>(stage_mem);
        T(*Bs)[KC][64] = reinterpret_cast<T(*)[KC][64]>(stage_mem + KC * 64 * 2 * sizeof(T) / sizeof(double));
        const int64_t qb = ibig[tq];
        for (; q < qb; ++q) {
            const Incidence in = incs[q];
            if (in.nI > nr || in.nJ > w) {       // corrupt plan: never write outside the tile
                if (tid == 0) atomicMin(info + 1, tk.J);
                continue;
            }
            coop_product<T, KC>(C, As, Bs, s_rel, in, imap, Lx, r0, nr, w);
        }
    } else if constexpr (COOP) {
        uint64_t(*Ap)[4][64] = reinterpret_cast<uint64_t(*)[4][64]>(stage_mem);
        uint64_t(*Bp)[4][64] = reinterpret_cast<uint64_t(*)[4][64]>(stage_mem + 2 * 4 * 64);
        const int64_t qb = ibig[tq];
        for (; q < qb; ++q) {
            const Incidence in = incs[q];
            if (in.nI > nr || in.nJ > w) {
                if (tid == 0) atomicMin(info + 1, tk.J);
                continue;
            }
            coop_product_packed<OP>(C, Ap, Bp, s_rel, in, imap, Lx, r0, nr, w);
        }
    }

    // the small incidences: each wavefront runs its own item list
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const int64_t *wg = wptr + 16 * (int64_t)tq + 4 * wv;
    if (wg[0] < wg[1]) wave_items<T, OP, 4>(C, witems, wmap, (const T *)Lx, wg[0], wg[1], r0, nr, w);
    if (wg[1] < wg[2]) wave_items<T, OP, 3>(C, witems, wmap, (const T *)Lx, wg[1], wg[2], r0, nr, w);
    if (wg[2] < wg[3]) wave_items<T, OP, 2>(C, witems, wmap, (const T *)Lx, wg[2], wg[3], r0, nr, w);
    if (wg[3] < wg[4]) wave_items<T, OP, 1>(C, witems, wmap, (const T *)Lx, wg[3], wg[4], r0, nr, w);
    __syncthreads();

    bool finish = !partial;
    if (partial) {
        // store this part's sum (written through to the device-coherent
        // level), count arrivals; the last part adds every part's sum, in
        // part order, to the tile and finishes it
        const PartDesc pd = parts[tk.K];
        T *slot = pbuf + (int64_t)(pd.slot0 + pd.part) * 4096;
        for (int k = tid; k < 4096; k += NT) {
            const int c = k >> 6, r = k & 63;
            if (r < nr && c < w)
                __hip_atomic_store(slot + k, C[c * LDC + r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) s_last = atomicAdd(&pcount[pd.counter], 1) == pd.nparts - 1;
        __syncthreads();
        if (s_last) {
            tile_in(C, LJ + r0, J.ld, nr, w);
            __syncthreads();
            // each thread owns 16 fixed entries; per part its 16 loads are
            // issued together (slot entries outside the tile are loaded but
            // never used, so the loads stay unconditional and in bounds)
            constexpr int E = 4096 / NT;
            const T *base = pbuf + (int64_t)pd.slot0 * 4096 + tid;
            T acc[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = tid + e * NT;
                acc[e] = C[(k >> 6) * LDC + (k & 63)];
            }
            for (int p = 0; p < pd.nparts; ++p) {
                T v[E];
#pragma unroll
                for (int e = 0; e < E; ++e)
                    v[e] = __hip_atomic_load(base + (int64_t)p * 4096 + e * NT, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                for (int e = 0; e < E; ++e) acc[e] += v[e];
            }
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = tid + e * NT;
                if ((k & 63) < nr && (k >> 6) < w) C[(k >> 6) * LDC + (k & 63)] = acc[e];
            }
            __syncthreads();
            if (tid == 0)
                __hip_atomic_store(&pcount[pd.counter], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            finish = true;
        }
    }
    if (finish) {
        if (tk.flags & kFuseFactor) {
            widen_tile<T>(Cbuf);
            panel_factor<OP != kOpNative>(Cbuf, nr, w, J.col0, info, pfloor ? pfloor + J.col0 : nullptr);
            tile_out(LJ + r0, Cbuf, J.ld, nr, w);
        } else {
            tile_out(LJ + r0, C, J.ld, nr, w);
        }
    }
    if (ttime && blockIdx.y == 0) {
        __syncthreads();                    // every wavefront's work is issued
        if (threadIdx.x == 0) ttime[tq] = wall_clock64() - t_start;
    }
}

// Internal (right-looking) update of one row tile of block J by the final
// blocks K, ..., K + g - 1 of the same supernode (g from the task's flags):
// tile -= sum_k L_k[tile rows, :] L_k[J's columns, :]^T, one accumulation
// over all g blocks' columns, so each entry takes the same sequence of
// products as with one block per step.  J's local row 0 is block k's local
// row d = col0_J - col0_k, so no index lookups are needed.  The
// accumulators start from the tile's current values.  With kFuseFactor
// (tile 0 of the block after the last source) the result is factored in LDS.
template <typename T, int OP>
__global__ __launch_bounds__(NT, 3) void k_internal(const Task *__restrict__ tasks,
                                                 const BlockDesc *__restrict__ blk,
                                                 T *__restrict__ Lx, int32_t *__restrict__ info,
                                                 int64_t lx_stride, const double *__restrict__ pfloor,
                                                 int32_t n)
{
    Lx += blockIdx.y * lx_stride;
    info += 4 * blockIdx.y;
    if (pfloor) pfloor += (int64_t)blockIdx.y * n;
    __shared__ double C[64 * LDC];      // the fused tile, factored in FP64
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const Task tk = tasks[blockIdx.x];
    const BlockDesc J = blk[tk.J];
    const int r0 = tk.t * TR;
    const int nr = min(TR, J.r - r0);
    const int w = J.w;
    T *LJ = Lx + J.valoff;
    const bool active = 32 * wr < nr && 32 * wc < w;

    typename Mfma<T>::acc_t acc[2][2] = {};
    if (active) {
        // the tile's entries seed the accumulators (32-bit byte offsets
        // from the tile's first entry; clamped, then masked)
        const char *tb = reinterpret_cast<const char *>(LJ + r0);
        const uint32_t ldb = sizeof(T) * (uint32_t)J.ld;
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int n = 0; n < 2; ++n)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 32 * wr + 16 * m + Mfma<T>::row(lane, v);
                    const int col = 32 * wc + 16 * n + (lane & 15);
                    const bool ok = row < nr && col < w;
                    const uint32_t off = (uint32_t)min(col, w - 1) * ldb + sizeof(T) * (uint32_t)min(row, nr - 1);
                    const T val = *reinterpret_cast<const T *>(tb + off);
                    acc[m][n][v] = ok ? val : T(0);
                }
        const int32_t k1 = tk.K + (tk.flags >> kDepthShift);
        for (int32_t k = tk.K; k <= k1; ++k) {
            const BlockDesc K = blk[k];
            const T *LK = Lx + K.valoff + (J.col0 - K.col0);
            wave_product_pipe<T, OP>(LK + r0, LK, K.ld, nr, w, K.w, wr, wc, acc);
        }
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
                        if (row < nr && col < w) C[col * LDC + row] = (double)acc[m][n][v];
                    }
        }
        __syncthreads();
        panel_factor<OP != kOpNative>(C, nr, w, J.col0, info, pfloor ? pfloor + J.col0 : nullptr);
        tile_out(LJ + r0, C, J.ld, nr, w);
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

// Leaves of the supernodal tree whose block is a single tile of at most 16
// columns: no update reaches them, so the block is only factored, one
// wavefront per block, with the fused-tile path's steps (the values as
// stored, widened to FP64, the same pivot steps, rounded once on the way
// out), so the factor is the same bit for bit.
template <typename T, bool FLOOR>
__global__ __launch_bounds__(64) void k_leaf(const Task *__restrict__ tasks, const BlockDesc *__restrict__ blk,
                                             T *__restrict__ Lx, int32_t *__restrict__ info, int64_t lx_stride,
                                             const double *__restrict__ pfloor, int32_t n)
{
    Lx += blockIdx.y * lx_stride;
    info += 4 * blockIdx.y;
    if (pfloor) pfloor += (int64_t)blockIdx.y * n;
    __shared__ double C[16 * LDC];
    __shared__ double bcast[64];
    const BlockDesc J = blk[tasks[blockIdx.x].J];
    const int nr = min(J.r, 64), w = min(J.w, 16);
    T *LJ = Lx + J.valoff;
    const int i = threadIdx.x;
#pragma unroll
    for (int c = 0; c < 16; ++c) C[c * LDC + i] = (i < nr && c < w) ? (double)LJ[(int64_t)c * J.ld + i] : 0.0;
    __syncthreads();
    wave_subpanel<double, FLOOR>(C, 0, w, nr, J.col0, info, pfloor ? pfloor + J.col0 : nullptr, bcast);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 16; ++c)
        if (i < nr && c < w) LJ[(int64_t)c * J.ld + i] = (T)C[c * LDC + i];
}

// Row tile t >= 1 of block J solves X := X L_JJ^{-T} against J's factored
// diagonal block, blocked by 16 columns: the four wavefronts first invert
// one 16 x 16 diagonal triangle each, then each solves 16 of the tile's rows
// through all column blocks with matrix-core products (no barriers).  The
// zero padding of both LDS blocks keeps the padded lanes finite.
template <typename T>
__global__ __launch_bounds__(NT) void k_trsm(const Task *__restrict__ tasks,
                                             const BlockDesc *__restrict__ blk,
                                             T *__restrict__ Lx, int64_t lx_stride)
{
    Lx += blockIdx.y * lx_stride;
    __shared__ T D[64 * LDC];
    __shared__ T X[64 * LDC];
    __shared__ T M[4 * 272];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const Task tk = tasks[blockIdx.x];
    const BlockDesc J = blk[tk.J];
    const int r0 = tk.t * TR;
    const int nr = min(TR, J.r - r0);
    const int w = J.w;
    T *LJ = Lx + J.valoff;
    tile2_in(D, LJ, w, X, LJ + r0, nr, J.ld, w);
    __syncthreads();
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    if (16 * wv < w) wave_tri_inverse(D, 16 * wv, min(16, w - 16 * wv), M + 272 * wv);
    __syncthreads();
    if (16 * wv < nr) wave_rows_solve(X, D, M, 16 * wv, w);
    __syncthreads();
    tile_out(LJ + r0, X, J.ld, nr, w);
}

// ------------------------------------------------------------ chain launch
//
// The steps inside the supernodes of one level (off-diagonal solves of the
// first blocks, then for every later block: the update by the previous
// block, the factorization of its diagonal tile and the solves of its other
// tiles) as one persistent launch.  Workgroups take tasks in the analysis's
// order (every task after the tasks it waits for) from a device counter,
// and a task waits for the tile states it needs: its own tile's previous
// update and the final tiles of the source block it reads (tile states as
// in Plan::tbase).  Values handed between the tasks of the launch are
// loaded and stored with device-coherent accesses; a task's state is
// published only after all of its stores have completed.  So the next
// block's factorization starts as soon as the tiles it reads are final,
// while the rest of the previous step's updates still run.

constexpr int kChainSpin = 1 << 22;     // sleeps of ~0.2 us: about a second
constexpr int kChainGrid = 512;         // workgroups of one instance (two per compute unit)

// Spin until *p >= v (device-scope loads); false, with the error word set,
// if the bound runs out or another workgroup of the launch gave up.
__device__ __forceinline__ bool chain_wait(const int32_t *p, int32_t v, int32_t *err)
{
    int it = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v) {
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        if (++it > kChainSpin) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(8);
    }
    return true;
}

// Initial tile states and task counters of every chain launch, per instance.
__global__ void k_chain_reset(int32_t *__restrict__ tstate, const int32_t *__restrict__ tinit,
                              int32_t ntiles, int32_t *__restrict__ cticket, int32_t nchain)
{
    tstate += (int64_t)blockIdx.y * ntiles;
    cticket += (int64_t)blockIdx.y * nchain;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ntiles; i += gridDim.x * blockDim.x)
        tstate[i] = tinit[i];
    if (blockIdx.x == 0)
        for (int32_t i = threadIdx.x; i < nchain; i += blockDim.x) cticket[i] = 0;
}

// An nr x w block at src (leading dimension ld) into the 64 x 64 LDS block
// dst (stride LDC), zero elsewhere; device-coherent loads.
template <typename T>
__device__ __forceinline__ void tile_in_coherent(T *dst, const T *src, int64_t ld, int nr, int w)
{
    const int i = threadIdx.x & 63, c0 = threadIdx.x >> 6;
    const __amdgpu_buffer_rsrc_t rs = coherent_rsrc(src);
    const uint32_t ldb = sizeof(T) * (uint32_t)ld;
    T v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int c = c0 + 4 * u;
        const T x = coherent_ld<T>(rs, (uint32_t)min(c, w - 1) * ldb + sizeof(T) * (uint32_t)min(i, nr - 1));
        v[u] = (i < nr && c < w) ? x : T(0);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) dst[(c0 + 4 * u) * LDC + i] = v[u];
}

template <typename T, typename U>
__device__ __forceinline__ void tile_out_coherent(T *dst, const U *src, int64_t ld, int nr, int w)
{
    const int i = threadIdx.x & 63, c0 = threadIdx.x >> 6;
    const __amdgpu_buffer_rsrc_t rs = coherent_rsrc(dst);
    const uint32_t ldb = sizeof(T) * (uint32_t)ld;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int c = c0 + 4 * u;
        if (i < nr && c < w) coherent_st<T>(rs, (uint32_t)c * ldb + sizeof(T) * (uint32_t)i, (T)src[c * LDC + i]);
    }
}

template <typename T, int OP>
__global__ __launch_bounds__(NT, 2) void k_chain(const Task *__restrict__ tasks, int32_t ntasks,
                                              const BlockDesc *__restrict__ blk,
                                              const int32_t *__restrict__ tbase, int32_t *tstate,
                                              int32_t ntiles, int32_t *cticket, int32_t nchain,
                                              T *Lx, int32_t *__restrict__ info, int64_t lx_stride,
                                              const double *__restrict__ pfloor, int32_t n)
{
    Lx += blockIdx.y * lx_stride;
    info += 4 * blockIdx.y;
    if (pfloor) pfloor += (int64_t)blockIdx.y * n;
    tstate += (int64_t)blockIdx.y * ntiles;
    int32_t *ticket = cticket + (int64_t)blockIdx.y * nchain;
    int32_t *err = info + 2;
    __shared__ double C[64 * LDC];      // a diagonal tile factored in FP64, or the tile X to solve
    __shared__ T Dg[64 * LDC];          // the factored diagonal block of a solve
    __shared__ T M[4 * 272];            // its inverted 16 x 16 diagonal triangles
    __shared__ int s_t, s_ok;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    for (;;) {
        __syncthreads();                // the previous task's LDS and s_t reads are done
        if (tid == 0)
            s_t = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? ntasks
                                                                                   : atomicAdd(ticket, 1);
        __syncthreads();
        const int q = s_t;
        if (q >= ntasks) break;
        const Task tk = tasks[q];
        const BlockDesc J = blk[tk.J];
        const int r0 = tk.t * TR;
        const int nr = min(TR, J.r - r0);
        const int w = J.w;
        T *LJ = Lx + J.valoff;
        const int32_t tile = tbase[tk.J] + tk.t;
        const bool factor = tk.flags & kFuseFactor;
        const bool solve = tk.flags & kChainSolve;
        typename Mfma<T>::acc_t acc[2][2] = {};
        const bool active = 32 * wr < nr && 32 * wc < w;
        if (tk.K >= 0) {
            const BlockDesc K = blk[tk.K];
            const int d = J.col0 - K.col0;
            if (tid == 0) {
                const int32_t kb = tbase[tk.K];
                bool ok = chain_wait(&tstate[tile], tk.K, err);
                for (int x = d / TR; ok && x <= (d + w - 1) / TR; ++x) ok = chain_wait(&tstate[kb + x], tk.K + 1, err);
                for (int x = (d + r0) / TR; ok && x <= (d + r0 + nr - 1) / TR; ++x)
                    ok = chain_wait(&tstate[kb + x], tk.K + 1, err);
                s_ok = ok;
            }
            __syncthreads();
            if (!s_ok) break;
            if (active) {
                const __amdgpu_buffer_rsrc_t rt = coherent_rsrc(LJ + r0);
                const uint32_t ldb = sizeof(T) * (uint32_t)J.ld;
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int nn = 0; nn < 2; ++nn)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int row = 32 * wr + 16 * m + Mfma<T>::row(lane, v);
                            const int col = 32 * wc + 16 * nn + (lane & 15);
                            const bool ok = row < nr && col < w;
                            const T val = coherent_ld<T>(rt, (uint32_t)min(col, w - 1) * ldb +
                                                                 sizeof(T) * (uint32_t)min(row, nr - 1));
                            acc[m][nn][v] = ok ? val : T(0);
                        }
                const T *LK = Lx + K.valoff;
                wave_product_pipe<T, OP, true>(LK + d + r0, LK + d, K.ld, nr, w, K.w, wr, wc, acc);
            }
        }
        if (factor) {
            if (active) {
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int nn = 0; nn < 2; ++nn)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int row = 32 * wr + 16 * m + Mfma<T>::row(lane, v);
                            const int col = 32 * wc + 16 * nn + (lane & 15);
                            if (row < nr && col < w) C[col * LDC + row] = (double)acc[m][nn][v];
                        }
            }
            __syncthreads();
            panel_factor<OP != kOpNative>(C, nr, w, J.col0, info, pfloor ? pfloor + J.col0 : nullptr);
            tile_out_coherent(LJ + r0, C, J.ld, nr, w);
        } else if (solve) {
            T *X = reinterpret_cast<T *>(C);
            if (tk.K >= 0) {
                // the updated tile, zero outside its nr x w entries
#pragma unroll
                for (int m = 0; m < 2; ++m)
#pragma unroll
                    for (int nn = 0; nn < 2; ++nn)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int row = 32 * wr + 16 * m + Mfma<T>::row(lane, v);
                            const int col = 32 * wc + 16 * nn + (lane & 15);
                            X[col * LDC + row] = (active && row < nr && col < w) ? acc[m][nn][v] : T(0);
                        }
            } else {
                tile_in_coherent(X, LJ + r0, J.ld, nr, w);
            }
            if (tid == 0) s_ok = chain_wait(&tstate[tbase[tk.J]], tk.J + 1, err);
            __syncthreads();
            if (!s_ok) break;
            tile_in_coherent(Dg, LJ, J.ld, w, w);
            __syncthreads();
            const int wv = __builtin_amdgcn_readfirstlane(wave);
            if (16 * wv < w) wave_tri_inverse(Dg, 16 * wv, min(16, w - 16 * wv), M + 272 * wv);
            __syncthreads();
            if (16 * wv < nr) wave_rows_solve(X, Dg, M, 16 * wv, w);
            __syncthreads();
            tile_out_coherent(LJ + r0, X, J.ld, nr, w);
        } else if (active) {
            const __amdgpu_buffer_rsrc_t rt = coherent_rsrc(LJ + r0);
            const uint32_t ldb = sizeof(T) * (uint32_t)J.ld;
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int nn = 0; nn < 2; ++nn)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = 32 * wr + 16 * m + Mfma<T>::row(lane, v);
                        const int col = 32 * wc + 16 * nn + (lane & 15);
                        if (row < nr && col < w)
                            coherent_st<T>(rt, (uint32_t)col * ldb + sizeof(T) * (uint32_t)row, acc[m][nn][v]);
                    }
        }
        // every store of the task has completed before its state moves on
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0)
            __hip_atomic_store(&tstate[tile], (factor || solve) ? tk.J + 1 : tk.K + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The inverse of every diagonal block, for the triangular solves.  Its
// strictly lower part is stored transposed in the block's upper triangle
// (entry (i, j), i > j, at row j of column i), which the factorization
// leaves unused; its diagonal (1 / L_ii) is not stored.
// Blocks of at most 16 columns: one wavefront inverts the triangle.
template <typename T>
__global__ __launch_bounds__(64) void k_inverse_small(const int32_t *__restrict__ list,
                                                      const BlockDesc *__restrict__ blk,
                                                      T *__restrict__ Lx, int64_t lx_stride)
{
    __shared__ T D[16 * LDC];
    __shared__ T M[272];
    Lx += blockIdx.y * lx_stride;
    const BlockDesc J = blk[list[blockIdx.x]];
    const int w = J.w, lane = threadIdx.x;
    const int64_t ld = J.ld;
    T *L = Lx + J.valoff;
    const int r = lane & 15, cq = lane >> 4;
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int c = cq + 4 * u;
        const bool ok = r < w && c < w && r >= c;
        const T x = L[ok ? (int64_t)c * ld + r : 0];
        v[u] = ok ? x : T(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) D[(cq + 4 * u) * LDC + r] = v[u];
    __syncthreads();
    wave_tri_inverse(D, 0, w, M);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = cq + 4 * u;
        if (r < i && i < w) L[(int64_t)i * ld + r] = M[i * 17 + r];
    }
}

// Wider blocks: X := I L_JJ^{-T} = (L_JJ^{-1})^T with the off-diagonal
// solve's routines (16 x 16 diagonal triangles inverted by the four
// wavefronts, then each solves 16 rows on the matrix cores); X's strictly
// upper part is the stored layout.
template <typename T>
__global__ __launch_bounds__(NT) void k_inverse_big(const int32_t *__restrict__ list,
                                                    const BlockDesc *__restrict__ blk,
                                                    T *__restrict__ Lx, int64_t lx_stride)
{
    __shared__ T D[64 * LDC];
    __shared__ T X[64 * LDC];
    __shared__ T M[4 * 272];
    Lx += blockIdx.y * lx_stride;
    const BlockDesc J = blk[list[blockIdx.x]];
    const int w = J.w;
    const int64_t ld = J.ld;
    T *L = Lx + J.valoff;
    const int tid = threadIdx.x;
    {
        const int i = tid & 63, c0 = tid >> 6;
        T v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int c = c0 + 4 * u;
            const bool ok = i < w && c < w && i >= c;
            const T x = L[ok ? (int64_t)c * ld + i : 0];
            v[u] = ok ? x : T(0);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int c = c0 + 4 * u;
            D[c * LDC + i] = v[u];
            X[c * LDC + i] = (i == c && i < w) ? T(1) : T(0);
        }
    }
    __syncthreads();
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (16 * wv < w) wave_tri_inverse(D, 16 * wv, min(16, w - 16 * wv), M + 272 * wv);
    __syncthreads();
    if (16 * wv < w) wave_rows_solve(X, D, M, 16 * wv, w);
    __syncthreads();
    for (int k = tid; k < 4096; k += NT) {
        const int i = k & 63, c = k >> 6;
        if (i < c && c < w) L[(int64_t)c * ld + i] = X[c * LDC + i];
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

template <typename T, int OP>
hipError_t factor_impl(const Plan &P, const DevicePlan &D, const double *Ax, hipStream_t s,
                       FactorProfile *prof)
{
    T *Lx = (T *)D.Lx;
    const unsigned m = (unsigned)D.m;
    const int64_t lxs = P.panel_entries;
    const double *pfloor = P.pivot_floor > 0.0 ? D.pfloor : nullptr;
    // per-task durations are recorded while profiling a single factorization
    auto ttime = [&](const Phase &ph) {
        return (prof && D.ttime && D.m == 1) ? (unsigned long long *)(D.ttime + ph.t0) : nullptr;
    };
    if (prof) prof->used = 0;
    {
        Bracket b(prof, s, 0);
        if (D.dscale && P.nds > 0)
            k_super_scale<<<dim3(grid_for(P.nds), m), 256, 0, s>>>(Ax, D.adiag, D.dsptr, P.nds,
                                                                    P.nnzA, P.n, D.dscale,
                                                                    pfloor ? D.pfloor : nullptr,
                                                                    P.pivot_floor);
        if (P.panel_entries > 0)
            k_fill_zero<T><<<dim3(grid_for(P.panel_entries), m), 256, 0, s>>>(Lx, P.panel_entries);
        if (P.nnzA > 0)
            k_scatter_a<T><<<dim3(grid_for(P.nnzA), m), 256, 0, s>>>(Ax, D.amap, Lx, P.nnzA, lxs,
                                                                      D.dscale, D.acoord, P.n);
        k_info_reset<<<dim3(1, m), 1, 0, s>>>(D.info);
    }
    if (P.nchain > 0) {
        Bracket b(prof, s, 0);
        k_chain_reset<<<dim3(grid_for(P.tbase[P.nb]), m), 256, 0, s>>>(D.tstate, D.tinit, P.tbase[P.nb],
                                                                       D.cticket, P.nchain);
    }
    int32_t chain = 0;
    for (const Phase &ph : P.phases) {
        const dim3 g((unsigned)(ph.t1 - ph.t0), m);
        // profile kinds: external updates; off-diagonal solves; the
        // factorizations inside supernodes (internal steps, leaves)
        Bracket b(prof, s, ph.kind == kPhaseExternal ? 1 : ph.kind == kPhaseTrsm ? 2 : 3);
        if (ph.kind == kPhaseChain) {
            const int64_t nt = ph.t1 - ph.t0;
            const unsigned gx = (unsigned)std::min<int64_t>(nt, std::max(16, kChainGrid / (int)m));
            k_chain<T, OP><<<dim3(gx, m), NT, 0, s>>>(D.tasks + ph.t0, (int32_t)nt, D.blk, D.tbase, D.tstate,
                                                      P.tbase[P.nb], D.cticket + chain, P.nchain, Lx, D.info,
                                                      lxs, pfloor, P.n);
            ++chain;
            continue;
        }
        const dim3 gx((unsigned)ph.nslots, m);
        if (ph.kind == kPhaseExternal && P.phase_coop[&ph - P.phases.data()])
            k_external<T, true, OP><<<gx, NT, 0, s>>>(D.tasks + ph.t0, D.iptr + ph.t0, D.ibig + ph.t0,
                                                     D.incs, D.imap, D.wptr + 16 * ph.t0, D.witems,
                                                     D.wmap, D.blk, Lx, D.info, lxs, ttime(ph), D.parts,
                                                     D.pcount, (T *)D.pbuf, P.nsplit, P.npartial,
                                                     pfloor, P.n, D.cptr + ph.t0, D.chunks, D.xslot + ph.s0);
        else if (ph.kind == kPhaseExternal)
            k_external<T, false, OP><<<gx, NT, 0, s>>>(D.tasks + ph.t0, D.iptr + ph.t0, D.ibig + ph.t0,
                                                      D.incs, D.imap, D.wptr + 16 * ph.t0, D.witems,
                                                      D.wmap, D.blk, Lx, D.info, lxs, ttime(ph), D.parts,
                                                      D.pcount, (T *)D.pbuf, P.nsplit, P.npartial,
                                                      pfloor, P.n, D.cptr + ph.t0, D.chunks, D.xslot + ph.s0);
        else if (ph.kind == kPhaseLeaf)
            k_leaf<T, OP != kOpNative><<<g, 64, 0, s>>>(D.tasks + ph.t0, D.blk, Lx, D.info, lxs, pfloor, P.n);
        else if (ph.kind == kPhaseInternal)
            k_internal<T, OP><<<g, NT, 0, s>>>(D.tasks + ph.t0, D.blk, Lx, D.info, lxs, pfloor, P.n);
        else
            k_trsm<T><<<g, NT, 0, s>>>(D.tasks + ph.t0, D.blk, Lx, lxs);
    }
    if (P.nb > 0) {
        Bracket b(prof, s, 2);
        const int32_t nsm = P.inv_nsmall, nbig = P.nb - P.inv_nsmall;
        if (nsm > 0)
            k_inverse_small<T><<<dim3((unsigned)nsm, m), 64, 0, s>>>(D.inv_blocks, D.blk, Lx, lxs);
        if (nbig > 0)
            k_inverse_big<T><<<dim3((unsigned)nbig, m), NT, 0, s>>>(D.inv_blocks + nsm, D.blk, Lx, lxs);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_factor(const Plan &P, const DevicePlan &D, const double *Ax, hipStream_t s,
                         FactorProfile *prof)
{
    switch (P.precision) {
    case kPrecF32: return factor_impl<float, kOpNative>(P, D, Ax, s, prof);
    case kPrecBF16: return factor_impl<float, kOpBF16>(P, D, Ax, s, prof);
    case kPrecF16: return factor_impl<float, kOpF16>(P, D, Ax, s, prof);
    default: return factor_impl<double, kOpNative>(P, D, Ax, s, prof);
    }
}

}  // namespace sym
