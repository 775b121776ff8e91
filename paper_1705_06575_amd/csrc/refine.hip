// refine.hip -- FP64 residual and update kernels of mixed-precision
// iterative refinement: x0 = solve(b) with the (FP32 or FP64) factor, then
// r = b - A x in FP64, eta_inf = |r|_inf / (|A|_inf |x|_inf + |b|_inf), and
// x += solve(r) until eta_inf reaches the tolerance; plus the matrix-vector
// product, dot products and vector updates of the conjugate-gradient form
// of the refinement.  Dot products are reduced in two fixed-order passes.
//
// The residual runs over the full symmetric pattern of A stored by rows
// (built by the analysis from the lower-triangle input), one thread per row,
// so every entry of r has one writer and a fixed summation order.  The
// infinity norms are maxima of nonnegative doubles, taken with atomic
// maxima on their bit patterns (order-independent, so exact).  A NaN
// anywhere (a failed factor fills x with NaN) makes the norm NaN: the
// maxima keep NaN operands instead of dropping them, so a broken solve can
// never report a small backward error.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace sym {

namespace {

// max(a, b) that returns NaN when either operand is NaN (fmax would drop it)
__device__ __forceinline__ double nan_max(double a, double b)
{
    return (b > a || b != b) ? b : a;
}

__device__ __forceinline__ void atomic_max_nonneg(double *addr, double v)
{
    // nonnegative IEEE doubles order like their bit patterns as unsigned
    // integers, and the positive quiet NaN's pattern lies above +infinity's,
    // so a NaN (made positive here) wins every later maximum
    const unsigned long long bits = v != v ? 0x7ff8000000000000ull
                                           : (unsigned long long)__double_as_longlong(v);
    atomicMax((unsigned long long *)addr, bits);
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = nan_max(v, __shfl_xor(v, off));
    return v;
}

// Batched use: instance blockIdx.y owns 4 reduction words, its vectors
// start n entries apart, its A values nnzA apart.
__global__ void k_red_reset(double *red)
{
    if (threadIdx.x < 4) red[4 * blockIdx.y + threadIdx.x] = 0.0;
}

// Batched use: instance i owns 4 reduction words, its vectors start n
// entries apart, its A values nnzA apart.  A thread takes one row for G
// consecutive instances (workgroup row blockIdx.y holds instances
// G blockIdx.y ...), so the row's pattern (positions and columns) is read
// once for all G; each instance's sum runs over the row in the same order
// as with G = 1.
constexpr int kRun = 8;

template <int G>
__global__ __launch_bounds__(256) void k_residual(const int64_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col,
                                                  const int64_t *__restrict__ val,
                                                  const double *__restrict__ Ax,
                                                  const double *__restrict__ b,
                                                  const double *__restrict__ x,
                                                  double *__restrict__ r, double *__restrict__ red,
                                                  int32_t n, int with_anorm, int64_t nnzA, int32_t m)
{
    const int32_t g0 = (int32_t)blockIdx.y * G;
    double mr[G], ma[G], mx[G], mb[G];
#pragma unroll
    for (int g = 0; g < G; ++g) mr[g] = ma[g] = mx[g] = mb[g] = 0.0;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s[G], sa[G];
#pragma unroll
        for (int g = 0; g < G; ++g) s[g] = sa[g] = 0.0;
        // the row's entries in runs (kRun for one value set, four when the
        // thread holds four value sets): all loads of a run
        // are issued before its products (addresses clamped into the row),
        // which are then taken in entry order
        const int64_t pb = rowptr[i], pe = rowptr[i + 1];
        constexpr int R = G == 1 ? kRun : 4;
        for (int64_t p0 = pb; p0 < pe; p0 += R) {
            int64_t v[R];
            int32_t c[R];
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const int64_t p = min(p0 + u, pe - 1);
                v[u] = val[p];
                c[u] = col[p];
            }
            double a[R][G], xv[R][G];
#pragma unroll
            for (int u = 0; u < R; ++u)
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const int64_t gi = min(g0 + g, m - 1);
                    a[u][g] = Ax[gi * nnzA + v[u]];
                    xv[u][g] = x[gi * n + c[u]];
                }
#pragma unroll
            for (int u = 0; u < R; ++u)
                if (p0 + u < pe) {
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        s[g] += a[u][g] * xv[u][g];
                        sa[g] += fabs(a[u][g]);
                    }
                }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (g0 + g < m) {
                const int64_t o = (int64_t)(g0 + g) * n + i;
                const double ri = b[o] - s[g];
                r[o] = ri;
                mr[g] = nan_max(mr[g], fabs(ri));
                ma[g] = nan_max(ma[g], sa[g]);
                mx[g] = nan_max(mx[g], fabs(x[o]));
                mb[g] = nan_max(mb[g], fabs(b[o]));
            }
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const double wr = wave_max(mr[g]), wa = wave_max(ma[g]), wx = wave_max(mx[g]), wb = wave_max(mb[g]);
        if ((threadIdx.x & 63) == 0 && g0 + g < m) {
            double *rd = red + 4 * (int64_t)(g0 + g);
            atomic_max_nonneg(&rd[0], wr);
            if (with_anorm) atomic_max_nonneg(&rd[1], wa);
            atomic_max_nonneg(&rd[2], wx);
            atomic_max_nonneg(&rd[3], wb);
        }
    }
}

__global__ void k_axpy(double *__restrict__ x, const double *__restrict__ d, int32_t n)
{
    x += (int64_t)blockIdx.y * n;
    d += (int64_t)blockIdx.y * n;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        x[i] += d[i];
}

// q = A p over the full symmetric rows, one thread per row (entries in
// runs of kRun, loads before products, products in entry order).
__global__ __launch_bounds__(256) void k_spmv(const int64_t *__restrict__ rowptr,
                                              const int32_t *__restrict__ col,
                                              const int64_t *__restrict__ val,
                                              const double *__restrict__ Ax,
                                              const double *__restrict__ p,
                                              double *__restrict__ q, int32_t n)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s = 0.0;
        const int64_t kb = rowptr[i], ke = rowptr[i + 1];
        for (int64_t k0 = kb; k0 < ke; k0 += kRun) {
            double a[kRun], pv[kRun];
#pragma unroll
            for (int u = 0; u < kRun; ++u) {
                const int64_t k = min(k0 + u, ke - 1);
                a[u] = Ax[val[k]];
                pv[u] = p[col[k]];
            }
#pragma unroll
            for (int u = 0; u < kRun; ++u)
                if (k0 + u < ke) s += a[u] * pv[u];
        }
        q[i] = s;
    }
}

// Dot product, first pass: workgroup g sums entries g, g + G, ... (a fixed
// order per thread, then a fixed tree) into part[g].
__global__ __launch_bounds__(256) void k_dot_part(const double *__restrict__ u,
                                                  const double *__restrict__ v,
                                                  double *__restrict__ part, int32_t n)
{
    __shared__ double sh[4];
    double s = 0.0;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        s += u[i] * v[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Second pass: one workgroup sums the kDotParts partials in a fixed tree.
__global__ __launch_bounds__(256) void k_dot_final(const double *__restrict__ part,
                                                   double *__restrict__ out)
{
    __shared__ double sh[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < kDotParts; i += 256) s += part[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void k_axpy_s(double *__restrict__ y, double a, const double *__restrict__ x, int32_t n)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        y[i] += a * x[i];
}

__global__ void k_xpby(double *__restrict__ p, const double *__restrict__ z, double b, int32_t n)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = z[i] + b * p[i];
}

inline unsigned grid_for(int64_t count)
{
    int64_t g = (count + 255) / 256;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_residual(const Plan &P, const DevicePlan &D, const double *Ax, const double *b,
                           const double *x, double *r, bool with_anorm, hipStream_t s)
{
    const unsigned m = (unsigned)D.m;
    k_red_reset<<<dim3(1, m), 64, 0, s>>>(D.red);
    if (P.n > 0 && m >= 4)
        k_residual<4><<<dim3(grid_for(P.n), (m + 3) / 4), 256, 0, s>>>(
            D.arowptr, D.acol, D.aval, Ax, b, x, r, D.red, P.n, with_anorm ? 1 : 0, P.nnzA, (int32_t)m);
    else if (P.n > 0)
        k_residual<1><<<dim3(grid_for(P.n), m), 256, 0, s>>>(
            D.arowptr, D.acol, D.aval, Ax, b, x, r, D.red, P.n, with_anorm ? 1 : 0, P.nnzA, (int32_t)m);
    return hipGetLastError();
}

hipError_t launch_axpy(const Plan &P, const DevicePlan &D, double *x, const double *d, hipStream_t s)
{
    if (P.n > 0) k_axpy<<<dim3(grid_for(P.n), (unsigned)D.m), 256, 0, s>>>(x, d, P.n);
    return hipGetLastError();
}

hipError_t launch_spmv(const Plan &P, const DevicePlan &D, const double *Ax, const double *p,
                       double *q, hipStream_t s)
{
    if (P.n > 0) k_spmv<<<grid_for(P.n), 256, 0, s>>>(D.arowptr, D.acol, D.aval, Ax, p, q, P.n);
    return hipGetLastError();
}

hipError_t launch_dot(const Plan &P, const DevicePlan &D, const double *u, const double *v,
                      double *out, hipStream_t s)
{
    k_dot_part<<<kDotParts, 256, 0, s>>>(u, v, D.part, P.n);
    k_dot_final<<<1, 256, 0, s>>>(D.part, out);
    return hipGetLastError();
}

hipError_t launch_axpy_s(const Plan &P, double *y, double a, const double *x, hipStream_t s)
{
    if (P.n > 0) k_axpy_s<<<grid_for(P.n), 256, 0, s>>>(y, a, x, P.n);
    return hipGetLastError();
}

hipError_t launch_xpby(const Plan &P, double *p, const double *z, double b, hipStream_t s)
{
    if (P.n > 0) k_xpby<<<grid_for(P.n), 256, 0, s>>>(p, z, b, P.n);
    return hipGetLastError();
}

}  // namespace sym
