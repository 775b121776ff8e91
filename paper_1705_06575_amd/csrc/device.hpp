// device.hpp -- device view of a bound plan and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "plan.hpp"

namespace sym {

// Pointers into the caller's workspace, filled by sym_bind.
// With m > 1 (a batch of value sets on one pattern) every per-instance
// buffer below holds m consecutive copies (Lx: panel_entries each; the
// vectors: n; info and red: 4; pend and done: nb; ticket: 16), and every
// launch covers the m instances with its grid's second dimension.
struct DevicePlan {
    int32_t m = 1;                  // instances
    void *Lx = nullptr;             // panel values, double or float
    BlockDesc *blk = nullptr;       // nb
    int32_t *rows = nullptr;        // sum of supernode row counts
    Task *tasks = nullptr;          // factor tasks in launch order
    int32_t *xslot = nullptr;       // external launches' workgroup slots (Plan::xslot)
    int64_t *iptr = nullptr;        // tasks+1: incidence ranges of external-update tasks
    int64_t *ibig = nullptr;        // tasks: end of each task's leading large incidences
    Incidence *incs = nullptr;      // (tile, descendant) incidences
    uint8_t *imap = nullptr;        // their tile-relative rows and columns
    int64_t *wptr = nullptr;        // 16*tasks+1: wavefront item ranges by row-block group
    WaveItem *witems = nullptr;     // small incidences per wavefront
    uint8_t *wmap = nullptr;        // their tile-relative rows and columns
    int64_t *cptr = nullptr;        // tasks+1: staged chunk ranges
    StageChunk *chunks = nullptr;   // staged chunks of the staged tasks
    int32_t *level_blocks = nullptr;// nb, grouped by level
    int64_t *amap = nullptr;        // nnzA
    int32_t *perm = nullptr;        // n
    double *vec = nullptr;          // n scratch (forward accumulator)
    double *vec2 = nullptr;         // n scratch (forward output in full solves)
    SolveTask *fwd_tasks = nullptr; // forward-sweep tasks grouped by level
    SolveTask *bwd_tasks = nullptr; // backward off-diagonal chunk tasks grouped by level
    int32_t *info = nullptr;        // [0] = smallest failing column (permuted), INT32_MAX if none
    double *vec3 = nullptr;         // n scratch (refinement residual / correction)
    int64_t *arowptr = nullptr;     // full symmetric rows of A (original ordering)
    int32_t *acol = nullptr;
    int64_t *aval = nullptr;
    double *red = nullptr;          // reduction scalars of refinement
    double *vec4 = nullptr;         // n scratch: conjugate-gradient direction p
    double *vec5 = nullptr;         // n scratch: A p
    double *vec6 = nullptr;         // n scratch: preconditioned residual z
    double *part = nullptr;         // kDotParts partial sums of a dot product
    uint64_t *ttime = nullptr;      // tasks: duration of each profiled external task (100 MHz ticks)
    int32_t *inv_blocks = nullptr;  // nb: blocks for the diagonal inverses
    PartDesc *parts = nullptr;      // split external tiles' parts
    int32_t *pcount = nullptr;      // nsplit arrival counters (per instance)
    void *pbuf = nullptr;           // npartial 64 x 64 partial tiles, T (per instance)
    // dataflow sweeps
    int64_t *chunk_tptr = nullptr;  // fwd tasks+1
    int32_t *chunk_tgt = nullptr;   // target blocks of each chunk
    int32_t *fwd_pend = nullptr;    // nb: initial counters of the forward sweep
    int32_t *bwd_pend = nullptr;    // nb: initial counters of the backward sweep
    SolveTask *bwd_df = nullptr;    // backward tasks in ticket order
    SolveTask *bw_df = nullptr;     // the same with walkers (Plan::bw_df)
    int64_t *bw_tptr = nullptr;
    int32_t *bw_tgt = nullptr;
    int32_t *bw_pend = nullptr;
    int32_t *bw_slot_start = nullptr;
    uint8_t *bw_slot_quad = nullptr;
    int32_t *pend = nullptr;        // nb: live counters
    int32_t *done = nullptr;        // nb: blocks whose backward solve is final
    int32_t *ticket = nullptr;      // next task of a running sweep
    int32_t *fwd_slot_start = nullptr;  // ticket slots of the dense forward sweep
    uint8_t *fwd_slot_quad = nullptr;
    int32_t *bwd_slot_start = nullptr;  // ticket slots of the backward sweep
    uint8_t *bwd_slot_quad = nullptr;
    // per-supernode scaling (scaled precisions; null otherwise): the factor
    // is that of D P A P^T D, D = diag(dscale) in permuted numbering
    double *dscale = nullptr;       // n (per instance)
    double *pfloor = nullptr;       // n (per instance): pivot floors
    int64_t *adiag = nullptr;       // n
    int32_t *acoord = nullptr;      // 2 nnzA
    int32_t *dsptr = nullptr;       // nds + 1
    // chain launches
    int32_t *tbase = nullptr;       // nb + 1: first tile of each block
    int32_t *tinit = nullptr;       // tiles: initial tile states
    int32_t *tstate = nullptr;      // tiles (per instance): live tile states
    int32_t *cticket = nullptr;     // nchain (per instance): next task of each chain launch
};

// Reach-pruned forward sweep schedule, device view.
struct DeviceRhs {
    SolveTask *tasks = nullptr;     // forward tasks of the touched blocks, grouped by level
    int32_t *bpos = nullptr;        // nb_rhs: permuted positions of b's nonzeros
    int32_t *pend = nullptr;        // nb: initial counters of the pruned forward sweep
    int64_t ntasks = 0;
    int32_t *slot_start = nullptr;  // ticket slots of the pruned forward sweep
    uint8_t *slot_quad = nullptr;
    int64_t nslots = 0;
};

// Optional per-launch event pairs for measurement: ev[2*i], ev[2*i+1]
// bracket launch i; kind[i] is its launch kind (0 scatter, 1 external,
// 2 trsm, 3 internal).
struct FactorProfile {
    std::vector<hipEvent_t> ev;
    std::vector<int32_t> kind;
    int32_t used = 0;
};

// ---- factor (factor.hip)
hipError_t launch_factor(const Plan &P, const DevicePlan &D, const double *Ax, hipStream_t s,
                         FactorProfile *prof);

// ---- solve (solve.hip)
// Static scratch of the allocation-free full solve: accumulator and forward
// result (kStaticMaxN doubles each), live counters and done flags
// (kStaticMaxN int32 each), ticket words (64 bytes).
constexpr int64_t kStaticMaxN = int64_t(1) << 19;
constexpr int kStaticMaxDevices = 64;
constexpr size_t kStaticOffVec2 = 8 * (size_t)kStaticMaxN;
constexpr size_t kStaticOffPend = 16 * (size_t)kStaticMaxN;
constexpr size_t kStaticOffDone = 20 * (size_t)kStaticMaxN;
constexpr size_t kStaticOffTicket = 24 * (size_t)kStaticMaxN;
constexpr size_t kStaticScratchBytes = kStaticOffTicket + 256;
// Device address of the scratch on the current GPU (looked up once per
// device).
hipError_t static_scratch(void **ptr);
hipError_t launch_perm_gather(const Plan &P, const DevicePlan &D, const double *b, double *y,
                              hipStream_t s);
hipError_t launch_perm_scatter(const Plan &P, const DevicePlan &D, const double *y, double *x,
                               hipStream_t s);
hipError_t launch_fwd(const Plan &P, const DevicePlan &D, double *acc, double *out, hipStream_t s);
hipError_t launch_bwd(const Plan &P, const DevicePlan &D, double *y, hipStream_t s);
hipError_t launch_fwd_sparse(const Plan &P, const DevicePlan &D, const DeviceRhs &R,
                             int64_t nbeta, const double *bv, double *acc, double *out,
                             hipStream_t s);
// y *= dscale (permuted numbering, per instance): the scaling's half of a
// backward sweep's result
hipError_t launch_scale(const Plan &P, const DevicePlan &D, double *y, hipStream_t s);

// ---- iterative refinement (refine.hip)
// r = b - A x (FP64); red[0] = max |r_i|, red[1] = max_i sum_j |A_ij|,
// red[2] = max |x_i|, red[3] = max |b_i| (the norms of eta_inf).
hipError_t launch_residual(const Plan &P, const DevicePlan &D, const double *Ax, const double *b,
                           const double *x, double *r, bool with_anorm, hipStream_t s);
// x += d
hipError_t launch_axpy(const Plan &P, const DevicePlan &D, double *x, const double *d, hipStream_t s);
// q = A p (FP64, full symmetric rows of A)
hipError_t launch_spmv(const Plan &P, const DevicePlan &D, const double *Ax, const double *p,
                       double *q, hipStream_t s);
// *out (device) = u . v, reduced in a fixed order
constexpr int kDotParts = 1024;
hipError_t launch_dot(const Plan &P, const DevicePlan &D, const double *u, const double *v,
                      double *out, hipStream_t s);
// y += a x
hipError_t launch_axpy_s(const Plan &P, double *y, double a, const double *x, hipStream_t s);
// p = z + b p
hipError_t launch_xpby(const Plan &P, double *p, const double *z, double b, hipStream_t s);

// ---- cost-model network (mlp.hip)
constexpr int kMlpHidden = 64;      // units per hidden layer
constexpr int kMlpMaxIn = 32;       // input features at most
constexpr int kMlpGradChunks = 64;  // sample chunks of the gradient reduction
int64_t mlp_param_count(int D);
int64_t mlp_work_floats(int n, int D);   // backward scratch: per-sample values + chunk sums
hipError_t launch_mlp_forward(const float *params, const float *X, int n, int D, float *y,
                              hipStream_t s);
// grad = gradient of the mean squared error; work: mlp_work_floats(n, D) floats
hipError_t launch_mlp_backward(const float *params, const float *X, const float *t, int n, int D,
                               float *grad, float *work, hipStream_t s);
hipError_t launch_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t count,
                           int step, float lr, hipStream_t s);

}  // namespace sym
