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
// Each sweep is one persistent launch driven by data flow, not one launch
// per level.  Workgroups take tasks by ticket (an atomic counter) in a
// topological order (the tasks of wide levels several to a ticket); a task
// waits, with a bounded spin, until what it reads is final, and signals
// what it produced.  The diagonal triangles are solved with the inverse of
// each diagonal block, which the factorization stores in the block's unused
// upper triangle: one small matrix-vector product per block instead of a
// chain of w dependent steps.
//   forward, task (block J, chunk of 256 rows below its diagonal): waits
//   until every chunk whose rows meet J's columns has added its update into
//   the accumulator (a per-block counter reaching zero); stages J's
//   diagonal block in LDS and fetches its rows' L values before waiting;
//   wavefront 0 forms y_J = L_JJ^{-1} (accumulator) (every chunk of J
//   repeats this small product); chunk 0 stores y_J; every thread subtracts
//   sum_k L_ik y_k from its row's accumulator entry (one atomic add); then
//   it decrements the counter of every block its rows fall in.
//   backward (L^T x = y), levels from the top: chunk tasks of J wait for the
//   blocks owning their rows to be final, subtract their share of
//   L_offdiag^T x from J's entries (atomics) and decrement J's counter; the
//   chunk that empties the counter applies L_JJ^{-T} and marks J final (a
//   block without rows below its columns has a task of its own for that).
//   For one or two value sets, the widest supernodes' blocks are finished
//   by a walker instead: one workgroup walks the supernode's diagonal
//   blocks from the top and computes each block's rows that hold the next
//   block's columns itself, with that block's solution still in LDS.
// A task only waits for tasks with smaller tickets, which running
// workgroups hold, so the launch always drains; a wait that exceeds its
// bound (a corrupt plan) records an error and ends the launch.  Counters
// are reset by a small kernel before each sweep.  Every value one task
// hands to another within a launch (accumulator and solution entries,
// counters, flags) is written and read with device-scope atomic operations,
// which are coherent across the XCDs' separate L2 caches without cache-wide
// write-back or invalidation; a producer waits for its own memory
// operations to complete before it signals.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "device.hpp"

namespace sym {

// Scratch of the allocation-free full solve: the two n-vectors of the
// sweeps (accumulator and forward result), the per-block counters and done
// flags, and the ticket word, for n and block counts up to kStaticMaxN.
// One copy per GPU, held until the process ends; every call on a GPU
// shares it.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int NT = 256;
constexpr int LDT = 65;                 // LDS stride of a staged diagonal block

// Stage the upper triangle (diagonal included) of a w x w diagonal block,
// rows from c0 on, into LDS as doubles (column-major, stride LDT).  The
// factorization leaves there the inverse of the block's lower triangle,
// transposed: entry (j, i), j < i, holds (L_JJ^{-1})_ij.  All loads are
// issued before the first store (one memory latency per block).
template <typename T>
__device__ __forceinline__ void stage_inv(double *D, const T *__restrict__ L, int64_t ld, int w,
                                          int c0)
{
    const int i = threadIdx.x & 63, cq = threadIdx.x >> 6;
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int c = cq + 4 * u;
        const bool ok = i < w && c < w && i <= c && i >= c0;
        const T val = L[ok ? (int64_t)c * ld + i : 0];
        v[u] = ok ? (double)val : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int c = cq + 4 * u;
        if (i < w && c < w) D[c * LDT + i] = v[u];
    }
}

// The diagonal block's inverse applied to v (staged by stage_inv; v in
// vb, zero outside [c0, w)), by the whole workgroup: wavefront q forms, for
// every row i (its lane), the partial sum over the 16 columns
// [16q, 16q + 16) and leaves it in pp[q][i]; the caller adds the four
// partials and v_i / L_ii.  Forward: y = L_JJ^{-1} v, row i takes
// (L_JJ^{-1})_ij v_j for j < i (stored at D[i * LDT + j]).  Backward:
// x = L_JJ^{-T} v, row j takes (L_JJ^{-1})_ij v_i for i > j (stored at
// D[i * LDT + j]).
__device__ __forceinline__ void inv_partials(const double *D, const double *vb, double *pp, int c0,
                                             int w, bool transposed)
{
    const int lane = threadIdx.x & 63;
    const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int j0 = max(16 * q, c0 & ~3), j1 = min(16 * q + 16, w);
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int jb = j0; jb < j1; jb += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = min(jb + u, 63);
            const bool in = jb + u < j1 && (transposed ? jb + u > lane : jb + u < lane);
            const double c = in ? (transposed ? D[j * LDT + lane] : D[lane * LDT + j]) : 0.0;
            s[u] = fma(c, vb[j], s[u]);
        }
    }
    pp[q * 64 + lane] = (s[0] + s[1]) + (s[2] + s[3]);
}

// y = D P b and x = P^T D y; D = diag(dscale) is the factor's
// per-supernode scaling (identity when dscale is null): the factor is that
// of D P A P^T D, so A^{-1} = P^T D (D P A P^T D)^{-1} D P.
__global__ void k_gather(const double *__restrict__ b, const int32_t *__restrict__ perm,
                         double *__restrict__ y, int32_t n, const double *__restrict__ dscale)
{
    b += (int64_t)blockIdx.y * n;
    y += (int64_t)blockIdx.y * n;
    if (dscale) dscale += (int64_t)blockIdx.y * n;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        y[i] = dscale ? b[perm[i]] * dscale[i] : b[perm[i]];
}

__global__ void k_scatter_perm(const double *__restrict__ y, const int32_t *__restrict__ perm,
                               double *__restrict__ x, int32_t n, const double *__restrict__ dscale)
{
    y += (int64_t)blockIdx.y * n;
    x += (int64_t)blockIdx.y * n;
    if (dscale) dscale += (int64_t)blockIdx.y * n;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        x[perm[i]] = dscale ? y[i] * dscale[i] : y[i];
}

__global__ void k_scale(double *__restrict__ y, const double *__restrict__ dscale, int32_t n)
{
    y += (int64_t)blockIdx.y * n;
    dscale += (int64_t)blockIdx.y * n;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        y[i] *= dscale[i];
}

__global__ void k_zero2(double *__restrict__ a, double *__restrict__ b, int32_t n)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        a[i] = 0.0;
        b[i] = 0.0;
    }
}

__global__ void k_place(const double *__restrict__ bv, const int32_t *__restrict__ bpos,
                        double *__restrict__ y, int64_t nb, const double *__restrict__ dscale)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nb;
         k += (int64_t)gridDim.x * blockDim.x)
        y[bpos[k]] = dscale ? bv[k] * dscale[bpos[k]] : bv[k];
}

constexpr int kSpinLimit = 1 << 22;     // sleeps of ~0.2 us: about a second

// Device-scope (coherent) load and store of a value handed between tasks.
__device__ __forceinline__ double coherent_load(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void coherent_store(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every memory operation of the workgroup so far has completed (each
// wavefront waits for its own, then the barrier), so a signal sent after
// this is seen only after them.
__device__ __forceinline__ void complete_then_sync()
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// Spin until *p == 0; false, with the error word set, if the bound runs
// out.
__device__ __forceinline__ bool wait_zero(int32_t *p, int32_t *err)
{
    int it = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        if (++it > kSpinLimit) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(8);
    }
    return true;
}

// Spin until *p != 0.
__device__ __forceinline__ bool wait_set(int32_t *p, int32_t *err)
{
    int it = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        if (++it > kSpinLimit) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(8);
    }
    return true;
}

// Counters of a sweep from their initial values; done flags cleared.
__global__ void k_sync_reset(int32_t *__restrict__ pend, const int32_t *__restrict__ init,
                             int32_t *__restrict__ done, int32_t nb, int32_t *__restrict__ ticket)
{
    pend += (int64_t)blockIdx.y * nb;
    if (done) done += (int64_t)blockIdx.y * nb;
    ticket += 16 * blockIdx.y;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x) {
        pend[i] = init[i];
        if (done) done[i] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ticket[0] = 0;
}

// Next task of a persistent launch for the whole workgroup, or -1 when the
// list is exhausted or some wait of this launch ran out (then every
// workgroup stops taking tasks, so the launch ends promptly).
__device__ __forceinline__ int next_ticket(int32_t *ticket, int *s_t, int nslots, int32_t *err)
{
    __syncthreads();                        // s_t of the previous slot is no longer read
    if (threadIdx.x == 0)
        *s_t = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? nslots
                                                                                 : atomicAdd(ticket, 1);
    __syncthreads();
    const int t = *s_t;
    return t < nslots ? t : -1;
}

// Value of v in lane `src` of the wavefront (src wave-uniform).
__device__ __forceinline__ double wave_bcast(double v, int src)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One wavefront spins until *p == 0 (every lane reads the same word).
__device__ __forceinline__ bool wave_wait_zero(int32_t *p, int32_t *err)
{
    int it = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        if (++it > kSpinLimit) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(8);
    }
    return true;
}

// One wavefront spins until done[tgt[q]] != 0 for every q in [q0, q1).
__device__ __forceinline__ bool wave_wait_all_set(const int32_t *done, const int32_t *__restrict__ tgt,
                                                  int64_t q0, int64_t q1, int32_t *err)
{
    const int lane = threadIdx.x & 63;
    int it = 0;
    for (;;) {
        bool ready = true;
        for (int64_t q = q0 + lane; q < q1; q += 64)
            ready = ready && __hip_atomic_load(&done[tgt[q]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        if (__all(ready)) return true;
        if (++it > kSpinLimit) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(8);
    }
}

// Forward task of a narrow block (at most kWaveCols columns and kWaveRows
// rows below them: one chunk) by one wavefront, with no workgroup
// barrier: lane i < w holds row i of the diagonal block's inverse, lane l
// the block's row w + l below it.  As the workgroup task: wait for the
// block's counter, y_J = L_JJ^{-1} acc_J (columns from c0), the rows below
// take their products by atomic adds, then the counters of the blocks
// owning those rows drop.  False if the wait ran out.
template <typename T>
__device__ __forceinline__ bool wave_fwd_task(const SolveTask &tk, const BlockDesc &J,
                                              const T *__restrict__ L, const int32_t *__restrict__ rows,
                                              const int64_t *__restrict__ tptr,
                                              const int32_t *__restrict__ tgt, int32_t *pend,
                                              double *acc, double *__restrict__ out, int32_t *err)
{
    const int lane = threadIdx.x & 63;
    const int w = J.w, c0 = tk.c0;
    const int64_t ld = J.ld;
    // row il of the inverse: entries j < il, stored at (j, il); the diagonal L_ii
    const int il = min(lane, w - 1);
    const T *Lc = L + (int64_t)il * ld;
    double inv[kWaveCols];
#pragma unroll
    for (int j = 0; j < kWaveCols; ++j) {
        const T val = Lc[min(j, il)];
        inv[j] = j < il ? (double)val : 0.0;
    }
    const double dii = (double)Lc[il];
    const int ir = w + lane;
    const bool has_row = ir < J.r;
    const int ic = has_row ? ir : w - 1;
    const int32_t row = rows[J.rowoff + ic];
    double lv[kWaveCols];
#pragma unroll
    for (int k = 0; k < kWaveCols; ++k) {
        const T val = L[(int64_t)min(k, w - 1) * ld + ic];
        lv[k] = k < w ? (double)val : 0.0;
    }
    if (!wave_wait_zero(&pend[tk.J], err)) return false;
    const bool mine = lane >= c0 && lane < w;
    const double v = mine ? coherent_load(&acc[J.col0 + lane]) : 0.0;
    double y = v / dii;
#pragma unroll
    for (int j = 0; j < kWaveCols; ++j) y = fma(inv[j], wave_bcast(v, j), y);
    y = mine ? y : 0.0;
    if (mine) out[J.col0 + lane] = y;
    // the cross-lane reads run with every lane active (a lane outside a
    // branch does not keep its register for the others to read)
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kWaveCols; ++k) s4[k & 3] = fma(lv[k], wave_bcast(y, k), s4[k & 3]);
    if (has_row) atomicAdd(&acc[row], -((s4[0] + s4[1]) + (s4[2] + s4[3])));
    __builtin_amdgcn_s_waitcnt(0);          // this wavefront's additions have completed
    for (int64_t q = tptr[tk.list] + lane; q < tptr[tk.list + 1]; q += 64)
        __hip_atomic_fetch_add(&pend[tgt[q]], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Forward sweep, one persistent launch.  acc: right-hand side plus the
// updates of finished chunks (read for a block's own columns once its
// counter is zero, atomically updated for the rows below); out: solved
// values of the blocks' columns.
template <typename T>
__global__ __launch_bounds__(NT, 3) void k_fwd_df(const SolveTask *__restrict__ tasks,
                                               const int32_t *__restrict__ slot_start,
                                               const uint8_t *__restrict__ slot_quad, int nslots,
                                               const int64_t *__restrict__ tptr,
                                               const int32_t *__restrict__ tgt,
                                               int32_t *__restrict__ pend, int32_t *ticket,
                                               int32_t *err, const BlockDesc *__restrict__ blk,
                                               const int32_t *__restrict__ rows,
                                               const T *__restrict__ Lx, double *acc,
                                               double *__restrict__ out, int32_t n, int32_t nb,
                                               int64_t lx_stride)
{
    __shared__ double D[64 * LDT];
    __shared__ double ys[64], vb[64], pp[256];
    __shared__ int s_t, s_abort;
    const int tid = threadIdx.x;
    // instance blockIdx.y of a batch
    pend += (int64_t)blockIdx.y * nb;
    ticket += 16 * blockIdx.y;
    err += 4 * blockIdx.y;
    Lx += blockIdx.y * lx_stride;
    acc += (int64_t)blockIdx.y * n;
    out += (int64_t)blockIdx.y * n;
    if (tid == 0) s_abort = 0;
    for (;;) {
        const int sl = next_ticket(ticket, &s_t, nslots, err);
        if (sl < 0 || s_abort) break;
        const int64_t ta = slot_start[sl], tb = slot_start[sl + 1];
        if (slot_quad[sl]) {
            // one narrow task per wavefront; the next ticket's barrier joins them
            const int64_t t = ta + (tid >> 6);
            if (t < tb) {
                const SolveTask tk = tasks[t];
                const BlockDesc J = blk[tk.J];
                if (!wave_fwd_task(tk, J, Lx + J.valoff, rows, tptr, tgt, pend, acc, out, err) &&
                    (tid & 63) == 0)
                    s_abort = 1;
            }
            continue;
        }
        for (int64_t t = ta; t < tb; ++t) {
        __syncthreads();                    // the previous task's LDS reads are done
        const SolveTask tk = tasks[t];
        const BlockDesc J = blk[tk.J];
        const int c0 = tk.c0;
        const T *L = Lx + J.valoff;
        const int64_t ld = J.ld;
        const int w = J.w;
        // what does not depend on other tasks: the diagonal block, this thread's
        // row index and the row's values (columns past w repeat the last)
        stage_inv(D, L, ld, w, c0);
        const int i = w + tk.chunk * NT + tid;
        const bool has_row = i < J.r;
        const int ic = has_row ? i : w - 1;
        const int32_t row = rows[J.rowoff + ic];
        const bool wide = w > 16;
        double lv[64];
#pragma unroll
        for (int k = 0; k < 16; ++k) lv[k] = (double)L[(int64_t)min(k, w - 1) * ld + ic];
        if (wide) {
#pragma unroll
            for (int k = 16; k < 64; ++k) lv[k] = (double)L[(int64_t)min(k, w - 1) * ld + ic];
        } else {
#pragma unroll
            for (int k = 16; k < 64; ++k) lv[k] = 0.0;
        }
        __syncthreads();                    // the staged diagonal block is readable
        const double rd = (tid >= c0 && tid < w) ? 1.0 / D[tid * LDT + tid] : 1.0;
        if (tid == 0 && !wait_zero(&pend[tk.J], err)) s_abort = 1;
        __syncthreads();
        if (s_abort) break;
        if (tid < 64) vb[tid] = (tid >= c0 && tid < w) ? coherent_load(&acc[J.col0 + tid]) : 0.0;
        __syncthreads();
        inv_partials(D, vb, pp, c0, w, false);
        __syncthreads();
        if (tid < 64) {
            const double v = rd * vb[tid] + ((pp[tid] + pp[64 + tid]) + (pp[128 + tid] + pp[192 + tid]));
            ys[tid] = tid >= c0 && tid < w ? v : 0.0;
            if (tk.chunk == 0 && tid >= c0 && tid < w) out[J.col0 + tid] = v;
        }
        __syncthreads();
        if (has_row) {
            // y is 0 outside [c0, w): all 64 (narrow blocks: 16) columns
            // take part, branch-free
            double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 16; ++k) s4[k & 3] = fma(lv[k], ys[k], s4[k & 3]);
            if (wide) {
#pragma unroll
                for (int k = 16; k < 64; ++k) s4[k & 3] = fma(lv[k], ys[k], s4[k & 3]);
            }
            atomicAdd(&acc[row], -((s4[0] + s4[1]) + (s4[2] + s4[3])));
        }
        complete_then_sync();
        for (int64_t q = tptr[tk.list] + tid; q < tptr[tk.list + 1]; q += NT)
            __hip_atomic_fetch_add(&pend[tgt[q]], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Backward task of a narrow block by one wavefront: the block's single
// chunk (at most kWaveRows rows below it) or, for a block with no rows
// below, its diagonal solve alone.  Lane l holds row w + l below the block,
// lane j < w column j of the transposed inverse.  After the owners of its
// rows are final: x_J = L_JJ^{-T} (x_J - L_offdiag^T x[rows]), the column
// sums over the rows reduced across the wavefront (no other task touches
// x_J, so no atomic adds are needed), then J is marked final.
template <typename T>
__device__ __forceinline__ bool wave_bwd_task(const SolveTask &tk, const BlockDesc &J,
                                              const T *__restrict__ L, const int32_t *__restrict__ rows,
                                              const int64_t *__restrict__ tptr,
                                              const int32_t *__restrict__ tgt, int32_t *done, double *x,
                                              int32_t *err)
{
    const int lane = threadIdx.x & 63;
    const int w = J.w;
    const int64_t ld = J.ld;
    // column il of L_JJ^{-T}: (L_JJ^{-1})_{i il} for i > il, stored at (il, i)
    const int il = min(lane, w - 1);
    double invT[kWaveCols];
#pragma unroll
    for (int i = 0; i < kWaveCols; ++i) {
        const T val = L[(int64_t)min(i, w - 1) * ld + il];
        invT[i] = (i > il && i < w) ? (double)val : 0.0;
    }
    const double djj = (double)L[(int64_t)il * ld + il];
    const int ir = w + lane;
    const bool has_row = tk.chunk >= 0 && ir < J.r;
    const int ic = has_row ? ir : w - 1;
    const int32_t row = rows[J.rowoff + ic];
    double lv[kWaveCols];
#pragma unroll
    for (int k = 0; k < kWaveCols; ++k) {
        const T val = L[(int64_t)min(k, w - 1) * ld + ic];
        lv[k] = k < w ? (double)val : 0.0;
    }
    if (tk.chunk >= 0 && !wave_wait_all_set(done, tgt, tptr[tk.list], tptr[tk.list + 1], err))
        return false;
    const double xr = has_row ? coherent_load(&x[row]) : 0.0;
    double part[kWaveCols];
#pragma unroll
    for (int k = 0; k < kWaveCols; ++k) part[k] = lv[k] * xr;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < kWaveCols; ++k) part[k] += __shfl_xor(part[k], off);
    double pj = 0.0;
#pragma unroll
    for (int k = 0; k < kWaveCols; ++k) pj = lane == k ? part[k] : pj;
    const bool mine = lane < w;
    const double v = mine ? coherent_load(&x[J.col0 + lane]) - pj : 0.0;
    double xo = v / djj;
#pragma unroll
    for (int i = 0; i < kWaveCols; ++i) xo = fma(invT[i], wave_bcast(v, i), xo);
    if (mine) coherent_store(&x[J.col0 + lane], xo);
    __builtin_amdgcn_s_waitcnt(0);          // the block's values have completed
    if (lane == 0) __hip_atomic_store(&done[tk.J], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Spin until *p <= v; false, with the error word set, if the bound runs out.
__device__ __forceinline__ bool wait_at_most(int32_t *p, int32_t v, int32_t *err)
{
    int it = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > v) {
        if (++it > kSpinLimit) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(8);
    }
    return true;
}

// Backward walker of one wide supernode (the whole workgroup): blocks b =
// tk.J down to tk.c0, each followed by block b + 1.  Block b's rows that
// hold block b + 1's columns are the walker's, with x of block b + 1 kept
// in LDS (xs) from the step before (the first step reads it once block
// b + 1 is final); the chunk tasks of its other rows add their sums to x_b
// by atomics and decrement b's counter, which starts one above their
// number.  Once it is down to one: x_b = L_bb^{-T} (x_b - the chunks' sums
// - L_{b+1,b}^T x_{b+1}), stored, and b is marked final.  The rows' L
// values and the diagonal inverse are fetched before the wait.  False if
// a wait ran out.
template <typename T>
struct WalkStage {
    double dv[16];      // this thread's entries of the block's staged inverse
    T lv[16];           // its L values of the next block's rows
};

// The loads of walk step b into registers (issued before they are needed).
template <typename T>
__device__ __forceinline__ void walk_fetch(WalkStage<T> &st, const BlockDesc &J, int wn, const T *L)
{
    const int i = threadIdx.x & 63, cq = threadIdx.x >> 6;
    const int w = J.w;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int c = cq + 4 * u;
        const bool ok = i < w && c < w && i <= c;
        const T val = L[ok ? (int64_t)c * J.ld + i : 0];
        st.dv[u] = ok ? (double)val : 0.0;
    }
    const int kc = min(i, w - 1);
#pragma unroll
    for (int u = 0; u < 16; ++u) st.lv[u] = L[(int64_t)kc * J.ld + w + min(16 * cq + u, wn - 1)];
}

// Backward walker of one wide supernode (the whole workgroup): blocks b =
// tk.J down to tk.c0, each followed by block b + 1.  Block b's rows that
// hold block b + 1's columns are the walker's, with x of block b + 1 kept
// in LDS (xs) from the step before (the first step reads it once block
// b + 1 is final); the chunk tasks of its other rows add their sums to x_b
// by atomics and decrement b's counter, which starts one above their
// number.  Once it is down to one: x_b = L_bb^{-T} (x_b - the chunks' sums
// - L_{b+1,b}^T x_{b+1}), stored, and b is marked final.  The next step's
// L values and diagonal inverse are fetched into registers while this
// step waits and finishes.  False if a wait ran out.
template <typename T>
__device__ bool bwd_walk(const SolveTask &tk, const BlockDesc *__restrict__ blk,
                         const T *__restrict__ Lx, int32_t *pend, int32_t *done, double *x,
                         int32_t *err, double *D, double *vb, double *pp, double *xs, int *s_flag)
{
    const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
    const BlockDesc Jn = blk[tk.J + 1];
    WalkStage<T> st;
    BlockDesc J = blk[tk.J];
    walk_fetch(st, J, Jn.w, Lx + J.valoff);
    if (tid == 0) *s_flag = wait_set(&done[tk.J + 1], err);
    __syncthreads();
    if (!*s_flag) return false;
    if (tid < 64) xs[tid] = tid < Jn.w ? coherent_load(&x[Jn.col0 + tid]) : 0.0;
    int wn = Jn.w;
    for (int32_t b = tk.J; b >= tk.c0; --b) {
        __syncthreads();                    // xs is written; the last step's LDS reads are done
        const int w = J.w;
        // stage the inverse (as stage_inv) and form this thread's part of
        // L_{b+1,b}^T x_{b+1}: column lane, rows 16q .. 16q+15 of block b + 1
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int c = q + 4 * u;
            if (lane < w && c < w) D[c * LDT + lane] = st.dv[u];
        }
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int i = 16 * q + u;
            s = fma(i < wn ? (double)st.lv[u] : 0.0, xs[i], s);
        }
        pp[q * 64 + lane] = lane < w ? s : 0.0;
        const int32_t colb = J.col0;
        if (b > tk.c0) {
            const BlockDesc Jp = blk[b - 1];
            walk_fetch(st, Jp, w, Lx + Jp.valoff);      // the next step's loads, in flight
            J = Jp;
        }
        if (tid == 0) *s_flag = wait_at_most(&pend[b], 1, err);
        __syncthreads();
        if (!*s_flag) return false;
        if (tid < 64)
            vb[tid] = tid < w ? coherent_load(&x[colb + tid]) -
                                    ((pp[tid] + pp[64 + tid]) + (pp[128 + tid] + pp[192 + tid]))
                              : 0.0;
        __syncthreads();
        const double rd = (tid < 64 && tid < w) ? 1.0 / D[tid * LDT + tid] : 1.0;
        inv_partials(D, vb, pp, 0, w, true);
        __syncthreads();
        if (tid < 64) {
            const double v = rd * vb[tid] + ((pp[tid] + pp[64 + tid]) + (pp[128 + tid] + pp[192 + tid]));
            if (tid < w) coherent_store(&x[colb + tid], v);
            xs[tid] = tid < w ? v : 0.0;
        }
        complete_then_sync();
        if (tid == 0) __hip_atomic_store(&done[b], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wn = w;
    }
    return true;
}

// Backward sweep, one persistent launch over the tasks in ticket order
// (levels from the top; per level the off-diagonal chunks, then the
// diagonal solves).  x holds y on entry and the solution on exit.
template <typename T>
__global__ __launch_bounds__(NT, 2) void k_bwd_df(const SolveTask *__restrict__ tasks,
                                               const int32_t *__restrict__ slot_start,
                                               const uint8_t *__restrict__ slot_quad, int nslots,
                                               const int64_t *__restrict__ tptr,
                                               const int32_t *__restrict__ tgt,
                                               int32_t *__restrict__ pend, int32_t *done,
                                               int32_t *ticket, int32_t *err,
                                               const BlockDesc *__restrict__ blk,
                                               const int32_t *__restrict__ rows,
                                               const T *__restrict__ Lx, double *x, int32_t n,
                                               int32_t nb, int64_t lx_stride)
{
    __shared__ double D[64 * LDT];
    __shared__ double vb[64], pp[256], xs[64];
    __shared__ int s_t, s_abort, s_last;
    const int tid = threadIdx.x;
    // instance blockIdx.y of a batch
    pend += (int64_t)blockIdx.y * nb;
    done += (int64_t)blockIdx.y * nb;
    ticket += 16 * blockIdx.y;
    err += 4 * blockIdx.y;
    Lx += blockIdx.y * lx_stride;
    x += (int64_t)blockIdx.y * n;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    if (tid == 0) s_abort = 0;
    for (;;) {
        const int sl = next_ticket(ticket, &s_t, nslots, err);
        if (sl < 0 || s_abort) break;
        const int64_t ta = slot_start[sl], tb = slot_start[sl + 1];
        if (slot_quad[sl]) {
            // one narrow block per wavefront; the next ticket's barrier joins them
            const int64_t t = ta + wave;
            if (t < tb) {
                const SolveTask tk = tasks[t];
                const BlockDesc J = blk[tk.J];
                if (!wave_bwd_task(tk, J, Lx + J.valoff, rows, tptr, tgt, done, x, err) && lane == 0)
                    s_abort = 1;
            }
            continue;
        }
        for (int64_t t = ta; t < tb; ++t) {
        __syncthreads();                    // the previous task's LDS reads are done
        const SolveTask tk = tasks[t];
        if (tk.chunk == kWalkTask) {
            if (!bwd_walk(tk, blk, Lx, pend, done, x, err, D, vb, pp, xs, &s_last) && tid == 0) s_abort = 1;
            __syncthreads();
            if (s_abort) break;
            continue;
        }
        const BlockDesc J = blk[tk.J];
        const T *L = Lx + J.valoff;
        const int64_t ld = J.ld;
        const int w = J.w;
        // the diagonal block's inverse, for the task that finishes J
        stage_inv(D, L, ld, w, 0);
        bool finish = true;
        if (tk.chunk >= 0) {
            // subtract sum_{i in chunk} L_ik x[row_i] from x[J's column k]:
            // wavefront v takes columns v, v + 4, ..., lanes take rows; the
            // factor values are fetched before the wait
            const int i0 = w + tk.c0 + tk.chunk * NT;     // c0: rows a walker takes
            const int i1 = min(J.r, i0 + NT);
            const int32_t *rJ = rows + J.rowoff;
            int32_t ri[4];
            double lvv[4][16];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + lane + 64 * u;
                const int ic = i < i1 ? i : i0;
                ri[u] = rJ[ic];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int k = wave + 4 * q;
                    const T val = L[(k < w ? (int64_t)k * ld : 0) + ic];
                    lvv[u][q] = k < w ? (double)val : 0.0;
                }
            }
            // the blocks owning the chunk's rows must be final
            bool ok = true;
            for (int64_t q = tptr[tk.list] + tid; q < tptr[tk.list + 1]; q += NT)
                ok = ok && wait_set(&done[tgt[q]], err);
            if (!ok) s_abort = 1;
            __syncthreads();
            if (s_abort) break;
            double xr[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + lane + 64 * u;
                const double xv = coherent_load(&x[ri[u]]);
                xr[u] = i < i1 ? xv : 0.0;
            }
            double part[16];
#pragma unroll
            for (int q = 0; q < 16; ++q)
                part[q] = fma(lvv[0][q], xr[0], lvv[1][q] * xr[1]) + fma(lvv[2][q], xr[2], lvv[3][q] * xr[3]);
            // sums over the 64 lanes, then one atomic per column of J: for
            // wide blocks all 16 columns without branches between the
            // exchanges, for narrow ones only the columns the block has
            if (w > 32) {
#pragma unroll
                for (int off = 32; off > 0; off >>= 1)
#pragma unroll
                    for (int q = 0; q < 16; ++q) part[q] += __shfl_xor(part[q], off);
                if (lane == 0) {
#pragma unroll
                    for (int q = 0; q < 16; ++q)
                        if (wave + 4 * q < w) atomicAdd(&x[J.col0 + wave + 4 * q], -part[q]);
                }
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int k = wave + 4 * q;
                    if (k < w) {
                        double s2 = part[q];
                        for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off);
                        if (lane == 0) atomicAdd(&x[J.col0 + k], -s2);
                    }
                }
            }
            // the chunk whose decrement empties J's counter finishes J (the
            // others' updates completed before their decrements)
            complete_then_sync();
            if (tid == 0)
                s_last = __hip_atomic_fetch_add(&pend[tk.J], -1, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT) == 1;
            __syncthreads();
            finish = s_last != 0;
        } else {
            // a block without rows below its columns
            __syncthreads();
            if (tid == 0 && !wait_zero(&pend[tk.J], err)) s_abort = 1;
            __syncthreads();
            if (s_abort) break;
        }
        if (finish) {
            const double rd = (tid < 64 && tid < w) ? 1.0 / D[tid * LDT + tid] : 1.0;
            if (tid < 64) vb[tid] = tid < w ? coherent_load(&x[J.col0 + tid]) : 0.0;
            __syncthreads();
            inv_partials(D, vb, pp, 0, w, true);
            __syncthreads();
            if (tid < w) {
                const double v = rd * vb[tid] + ((pp[tid] + pp[64 + tid]) + (pp[128 + tid] + pp[192 + tid]));
                coherent_store(&x[J.col0 + tid], v);
            }
            complete_then_sync();
            if (tid == 0)
                __hip_atomic_store(&done[tk.J], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        }
    }
}

inline unsigned grid_for(int64_t count)
{
    int64_t g = (count + 255) / 256;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

// Workgroups of a persistent sweep: enough to fill the chip, at most one
// per task.
inline unsigned sweep_grid(int64_t ntasks, int32_t m)
{
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ntasks, 2048 / std::max(1, m)));
}

template <typename T>
hipError_t fwd_impl(const Plan &P, const DevicePlan &D, const SolveTask *tasks, const int32_t *slot_start,
                    const uint8_t *slot_quad, int64_t nslots, const int32_t *pend_init, double *acc,
                    double *out, hipStream_t s)
{
    if (nslots == 0) return hipGetLastError();
    const unsigned m = (unsigned)D.m;
    k_sync_reset<<<dim3(grid_for(P.nb), m), 256, 0, s>>>(D.pend, pend_init, nullptr, P.nb, D.ticket);
    k_fwd_df<T><<<dim3(sweep_grid(nslots, D.m), m), NT, 0, s>>>(
        tasks, slot_start, slot_quad, (int)nslots, D.chunk_tptr, D.chunk_tgt, D.pend, D.ticket, D.info + 2,
        D.blk, D.rows, (const T *)D.Lx, acc, out, P.n, P.nb, P.panel_entries);
    return hipGetLastError();
}

template <typename T>
hipError_t bwd_impl(const Plan &P, const DevicePlan &D, double *y, hipStream_t s)
{
    // walkers for few value sets (each holds a workgroup while it waits)
    const bool walk = P.nwalk > 0 && (int64_t)D.m * P.nwalk <= kWalkBudget;
    const int64_t nslots = walk ? P.bw_slots.count() : P.bwd_slots.count();
    if (nslots == 0) return hipGetLastError();
    const unsigned m = (unsigned)D.m;
    k_sync_reset<<<dim3(grid_for(P.nb), m), 256, 0, s>>>(D.pend, walk ? D.bw_pend : D.bwd_pend, D.done, P.nb,
                                                         D.ticket);
    k_bwd_df<T><<<dim3(sweep_grid(nslots, D.m), m), NT, 0, s>>>(
        walk ? D.bw_df : D.bwd_df, walk ? D.bw_slot_start : D.bwd_slot_start,
        walk ? D.bw_slot_quad : D.bwd_slot_quad, (int)nslots, walk ? D.bw_tptr : D.chunk_tptr,
        walk ? D.bw_tgt : D.chunk_tgt, D.pend,
        D.done, D.ticket, D.info + 2, D.blk, D.rows, (const T *)D.Lx, y, P.n, P.nb, P.panel_entries);
    return hipGetLastError();
}

std::mutex g_scratch_mu;
void *g_scratch_addr[kStaticMaxDevices] = {};

}  // namespace

hipError_t static_scratch(void **ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kStaticMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        // the array's name is a host-side stand-in: its device address on
        // the current GPU comes from the runtime, once per device
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[dev] = p;
    }
    *ptr = g_scratch_addr[dev];
    return hipSuccess;
}

hipError_t launch_perm_gather(const Plan &P, const DevicePlan &D, const double *b, double *y,
                              hipStream_t s)
{
    if (P.n > 0) k_gather<<<dim3(grid_for(P.n), (unsigned)D.m), 256, 0, s>>>(b, D.perm, y, P.n, D.dscale);
    return hipGetLastError();
}

hipError_t launch_perm_scatter(const Plan &P, const DevicePlan &D, const double *y, double *x,
                               hipStream_t s)
{
    if (P.n > 0)
        k_scatter_perm<<<dim3(grid_for(P.n), (unsigned)D.m), 256, 0, s>>>(y, D.perm, x, P.n, D.dscale);
    return hipGetLastError();
}

hipError_t launch_scale(const Plan &P, const DevicePlan &D, double *y, hipStream_t s)
{
    if (P.n > 0 && D.dscale) k_scale<<<dim3(grid_for(P.n), (unsigned)D.m), 256, 0, s>>>(y, D.dscale, P.n);
    return hipGetLastError();
}

hipError_t launch_fwd(const Plan &P, const DevicePlan &D, double *acc, double *out, hipStream_t s)
{
    const int64_t ns = P.fwd_slots.count();
    return prec_fp32_panels(P.precision)
               ? fwd_impl<float>(P, D, D.fwd_tasks, D.fwd_slot_start, D.fwd_slot_quad, ns, D.fwd_pend, acc,
                                 out, s)
               : fwd_impl<double>(P, D, D.fwd_tasks, D.fwd_slot_start, D.fwd_slot_quad, ns, D.fwd_pend, acc,
                                  out, s);
}

hipError_t launch_bwd(const Plan &P, const DevicePlan &D, double *y, hipStream_t s)
{
    return prec_fp32_panels(P.precision) ? bwd_impl<float>(P, D, y, s) : bwd_impl<double>(P, D, y, s);
}

hipError_t launch_fwd_sparse(const Plan &P, const DevicePlan &D, const DeviceRhs &R,
                             int64_t nbeta, const double *bv, double *acc, double *out,
                             hipStream_t s)
{
    if (P.n > 0) k_zero2<<<grid_for(P.n), 256, 0, s>>>(acc, out, P.n);
    if (nbeta > 0) k_place<<<grid_for(nbeta), 256, 0, s>>>(bv, R.bpos, acc, nbeta, D.dscale);
    return prec_fp32_panels(P.precision)
               ? fwd_impl<float>(P, D, R.tasks, R.slot_start, R.slot_quad, R.nslots, R.pend, acc, out, s)
               : fwd_impl<double>(P, D, R.tasks, R.slot_start, R.slot_quad, R.nslots, R.pend, acc, out, s);
}

}  // namespace sym
