// refine.hip -- FP64 residual and update kernels of mixed-precision
// iterative refinement: x0 = solve(b) with the (FP32 or FP64) factor, then
// r = b - A x in FP64, eta_inf = |r|_inf / (|A|_inf |x|_inf + |b|_inf), and
// x += solve(r) until eta_inf reaches the tolerance.
//
// The residual runs over the full symmetric pattern of A stored by rows
// (built by the analysis from the lower-triangle input), one thread per row,
// so every entry of r has one writer and a fixed summation order.  The
// infinity norms are maxima of nonnegative doubles, taken with atomic
// maxima on their bit patterns (order-independent, so exact).
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace sym {

namespace {

__device__ __forceinline__ void atomic_max_nonneg(double *addr, double v)
{
    // nonnegative IEEE doubles order like their bit patterns as unsigned integers
    atomicMax((unsigned long long *)addr, (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

__global__ void k_red_reset(double *red)
{
    if (threadIdx.x < 4) red[threadIdx.x] = 0.0;
}

__global__ __launch_bounds__(256) void k_residual(const int64_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col,
                                                  const int64_t *__restrict__ val,
                                                  const double *__restrict__ Ax,
                                                  const double *__restrict__ b,
                                                  const double *__restrict__ x,
                                                  double *__restrict__ r, double *__restrict__ red,
                                                  int32_t n, int with_anorm)
{
    double mr = 0.0, ma = 0.0, mx = 0.0, mb = 0.0;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double s = 0.0, sa = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            const double a = Ax[val[p]];
            s += a * x[col[p]];
            sa += fabs(a);
        }
        const double ri = b[i] - s;
        r[i] = ri;
        mr = fmax(mr, fabs(ri));
        ma = fmax(ma, sa);
        mx = fmax(mx, fabs(x[i]));
        mb = fmax(mb, fabs(b[i]));
    }
    mr = wave_max(mr);
    ma = wave_max(ma);
    mx = wave_max(mx);
    mb = wave_max(mb);
    if ((threadIdx.x & 63) == 0) {
        atomic_max_nonneg(&red[0], mr);
        if (with_anorm) atomic_max_nonneg(&red[1], ma);
        atomic_max_nonneg(&red[2], mx);
        atomic_max_nonneg(&red[3], mb);
    }
}

__global__ void k_axpy(double *__restrict__ x, const double *__restrict__ d, int32_t n)
{
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        x[i] += d[i];
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
    k_red_reset<<<1, 64, 0, s>>>(D.red);
    if (P.n > 0)
        k_residual<<<grid_for(P.n), 256, 0, s>>>(D.arowptr, D.acol, D.aval, Ax, b, x, r, D.red,
                                                  P.n, with_anorm ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_axpy(const Plan &P, double *x, const double *d, hipStream_t s)
{
    if (P.n > 0) k_axpy<<<grid_for(P.n), 256, 0, s>>>(x, d, P.n);
    return hipGetLastError();
}

}  // namespace sym
