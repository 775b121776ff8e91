// device.hpp -- device view of a bound plan and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"

namespace sym {

// Pointers into the caller's workspace, filled by sym_bind.
struct DevicePlan {
    void *Lx = nullptr;             // panel values, double or float
    BlockDesc *blk = nullptr;       // nb
    int32_t *rows = nullptr;        // sum of supernode row counts
    int64_t *dptr = nullptr;        // nb+1
    Pair *pairs = nullptr;          // npairs, grouped by target
    Task *tasks = nullptr;          // all tiles, grouped by level
    Task *tasks2 = nullptr;         // row tiles t >= 1 of multi-tile blocks, grouped by level
    int32_t *level_blocks = nullptr;// nb, grouped by level
    int64_t *amap = nullptr;        // nnzA
    int32_t *perm = nullptr;        // n
    double *vec = nullptr;          // n scratch
    int32_t *info = nullptr;        // [0] = smallest failing column (permuted), INT32_MAX if none
};

// Reach-pruned forward sweep schedule, device view.
struct DeviceRhs {
    int32_t *blocks = nullptr;      // touched blocks grouped by level
    int32_t *cstart = nullptr;      // first reached local column of each touched block
    int32_t *bpos = nullptr;        // nb_rhs: permuted positions of b's nonzeros
};

// ---- factor (factor.hip)
hipError_t launch_factor(const Plan &P, const DevicePlan &D, const double *Ax, hipStream_t s);

// ---- solve (solve.hip)
hipError_t launch_perm_gather(const Plan &P, const DevicePlan &D, const double *b, double *y,
                              hipStream_t s);
hipError_t launch_perm_scatter(const Plan &P, const DevicePlan &D, const double *y, double *x,
                               hipStream_t s);
hipError_t launch_fwd(const Plan &P, const DevicePlan &D, double *y, hipStream_t s);
hipError_t launch_bwd(const Plan &P, const DevicePlan &D, double *y, hipStream_t s);
hipError_t launch_fwd_sparse(const Plan &P, const DevicePlan &D, const DeviceRhs &R,
                             const std::vector<int64_t> &level_ptr, int64_t nbeta,
                             const double *bv, double *y, hipStream_t s);

}  // namespace sym
