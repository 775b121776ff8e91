// capi.cpp -- the extern "C" boundary: handles, workspace layout, binding
// and argument checks around the symbolic analysis and the device kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <stdexcept>
#include <vector>

#include "device.hpp"
#include "plan.hpp"
#include "sym.h"

static_assert(SYM_STATIC_MAX_N == sym::kStaticMaxN, "static scratch bound of the ABI");

struct sym_plan {
    sym::Plan P;
    size_t ws_bytes = 0;
    size_t off_Lx = 0, off_blk = 0, off_rows = 0, off_tasks = 0, off_xslot = 0, off_iptr = 0, off_ibig = 0, off_incs = 0, off_imap = 0,
           off_wptr = 0, off_witems = 0, off_wmap = 0,
           off_lvl = 0, off_amap = 0, off_perm = 0, off_vec = 0, off_vec2 = 0, off_ftk = 0, off_btk = 0,
           off_vec3 = 0, off_arp = 0, off_acol = 0, off_aval = 0, off_red = 0,
           off_ctp = 0, off_ctg = 0, off_fpend = 0, off_bpend = 0, off_bdf = 0, off_sync = 0,
           off_vec4 = 0, off_vec5 = 0, off_vec6 = 0, off_part = 0, off_ttime = 0,
           off_parts = 0, off_pcount = 0, off_pbuf = 0, off_invb = 0, off_tbase = 0, off_tinit = 0,
           off_tstate = 0, off_ctk = 0, off_bwdf = 0, off_bwtp = 0, off_bwtg = 0, off_bwpd = 0,
           off_bwss = 0, off_bwsq = 0,
           off_info = 0, off_dscale = 0, off_pfloor = 0, off_adiag = 0, off_acoord = 0,
           off_dsptr = 0, off_fss = 0, off_fsq = 0, off_bss = 0, off_bsq = 0, off_cptr = 0,
           off_chunks = 0;
    sym::DevicePlan D;
    bool bound = false;
    bool factored = false;
    // bumped whenever the device plan arrays move or the schedule changes
    // (sym_bind, sym_set_variants): a batch bound to an older generation
    // holds stale pointers and sizes and refuses to run
    uint64_t generation = 0;
    hipStream_t stream = nullptr;
    bool profiling = false;
    sym::FactorProfile prof;
    ~sym_plan()
    {
        for (hipEvent_t e : prof.ev) (void)hipEventDestroy(e);
    }
};

struct sym_rhs_plan {
    sym_plan *h = nullptr;
    std::vector<int32_t> reach;      // permuted columns, increasing
    std::vector<sym::SolveTask> tasks;  // forward tasks of the touched blocks, grouped by level
    std::vector<int32_t> bpos;       // permuted positions of b's nonzeros
    std::vector<int64_t> level_ptr;  // groups of `tasks` per nonempty level
    std::vector<int32_t> pend;       // nb: chunks of `tasks` whose rows meet each block
    sym::SweepSlots slots;           // ticket slots of the pruned sweep
    size_t ws_bytes = 0, off_tasks = 0, off_bpos = 0, off_pend = 0, off_ss = 0, off_sq = 0;
    sym::DeviceRhs R;
    bool bound = false;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t elem_size(const sym::Plan &P)
{
    return sym::prec_fp32_panels(P.precision) ? sizeof(float) : sizeof(double);
}

void layout(sym_plan *h)
{
    const sym::Plan &P = h->P;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    h->off_Lx = take((size_t)P.panel_entries * elem_size(P));
    h->off_blk = take(sizeof(sym::BlockDesc) * P.blk.size());
    h->off_rows = take(sizeof(int32_t) * P.dsrows.size());
    h->off_tasks = take(sizeof(sym::Task) * P.ftasks.size());
    h->off_xslot = take(sizeof(int32_t) * P.xslot.size());
    h->off_iptr = take(sizeof(int64_t) * P.iptr.size());
    h->off_ibig = take(sizeof(int64_t) * P.ibig.size());
    h->off_incs = take(sizeof(sym::Incidence) * P.incs.size());
    h->off_imap = take(P.imap.size());
    h->off_wptr = take(sizeof(int64_t) * P.wptr.size());
    h->off_witems = take(sizeof(sym::WaveItem) * P.witems.size());
    h->off_wmap = take(P.wmap.size());
    h->off_lvl = take(sizeof(int32_t) * P.level_blocks.size());
    h->off_amap = take(sizeof(int64_t) * P.amap.size());
    h->off_perm = take(sizeof(int32_t) * P.perm.size());
    h->off_vec = take(sizeof(double) * (size_t)P.n);
    h->off_vec2 = take(sizeof(double) * (size_t)P.n);
    h->off_ftk = take(sizeof(sym::SolveTask) * P.fwd_tasks.size());
    h->off_btk = take(sizeof(sym::SolveTask) * P.bwd_tasks.size());
    h->off_info = take(sizeof(int32_t) * 4);
    h->off_vec3 = take(sizeof(double) * (size_t)P.n);
    h->off_arp = take(sizeof(int64_t) * P.arowptr.size());
    h->off_acol = take(sizeof(int32_t) * P.acol.size());
    h->off_aval = take(sizeof(int64_t) * P.aval.size());
    h->off_red = take(sizeof(double) * 4);
    h->off_ctp = take(sizeof(int64_t) * P.chunk_tptr.size());
    h->off_ctg = take(sizeof(int32_t) * P.chunk_tgt.size());
    h->off_fpend = take(sizeof(int32_t) * P.fwd_pend.size());
    h->off_bpend = take(sizeof(int32_t) * P.bwd_pend.size());
    h->off_bdf = take(sizeof(sym::SolveTask) * P.bwd_df.size());
    h->off_sync = take(sizeof(int32_t) * (2 * (size_t)P.nb + 64));
    h->off_vec4 = take(sizeof(double) * (size_t)P.n);
    h->off_vec5 = take(sizeof(double) * (size_t)P.n);
    h->off_vec6 = take(sizeof(double) * (size_t)P.n);
    h->off_part = take(sizeof(double) * (sym::kDotParts + 8));
    h->off_ttime = take(sizeof(uint64_t) * P.ftasks.size());
    h->off_parts = take(sizeof(sym::PartDesc) * P.parts.size());
    h->off_pcount = take(sizeof(int32_t) * (size_t)P.nsplit);
    h->off_pbuf = take((size_t)P.npartial * 4096 * elem_size(P));
    h->off_invb = take(sizeof(int32_t) * P.inv_blocks.size());
    const bool sc = sym::prec_scaled(P.precision);
    h->off_dscale = take(sc ? sizeof(double) * (size_t)P.n : 0);
    h->off_pfloor = take(sc ? sizeof(double) * (size_t)P.n : 0);
    h->off_adiag = take(sc ? sizeof(int64_t) * P.adiag.size() : 0);
    h->off_acoord = take(sc ? sizeof(int32_t) * P.acoord.size() : 0);
    h->off_dsptr = take(sc ? sizeof(int32_t) * P.dsptr.size() : 0);
    h->off_cptr = take(sizeof(int64_t) * P.cptr.size());
    h->off_chunks = take(sizeof(sym::StageChunk) * P.chunks.size());
    h->off_fss = take(sizeof(int32_t) * P.fwd_slots.start.size());
    h->off_fsq = take(P.fwd_slots.quad.size());
    h->off_bss = take(sizeof(int32_t) * P.bwd_slots.start.size());
    h->off_bsq = take(P.bwd_slots.quad.size());
    h->off_tbase = take(sizeof(int32_t) * P.tbase.size());
    h->off_tinit = take(sizeof(int32_t) * P.tinit.size());
    h->off_tstate = take(sizeof(int32_t) * P.tinit.size());
    h->off_ctk = take(sizeof(int32_t) * (size_t)P.nchain);
    h->off_bwdf = take(sizeof(sym::SolveTask) * P.bw_df.size());
    h->off_bwtp = take(sizeof(int64_t) * P.bw_tptr.size());
    h->off_bwtg = take(sizeof(int32_t) * P.bw_tgt.size());
    h->off_bwpd = take(sizeof(int32_t) * P.bw_pend.size());
    h->off_bwss = take(sizeof(int32_t) * P.bw_slots.start.size());
    h->off_bwsq = take(P.bw_slots.quad.size());
    h->ws_bytes = o;
}

hipError_t upload(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
}

// eta_inf = ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf) from the residual
// kernel's maxima cur = {|r|, (unused), |x|, |b|}; NaN stays NaN.
double backward_error(double anorm, const double cur[4])
{
    const double den = anorm * cur[2] + cur[3];
    return den > 0.0 ? cur[0] / den : cur[0];
}

// Whether the last factorization recorded a non-positive pivot (its first
// status word); synchronizes the stream.  False if a HIP call failed.
bool read_pivot_failed(sym_plan *h, hipStream_t s, bool &failed)
{
    int32_t w = INT32_MAX;
    if (hipMemcpyAsync(&w, h->D.info, sizeof(w), hipMemcpyDeviceToHost, s) != hipSuccess) return false;
    if (hipStreamSynchronize(s) != hipSuccess) return false;
    failed = w != INT32_MAX;
    return true;
}

}  // namespace

extern "C" {

void sym_opts_default(sym_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->ordering = SYM_ORDER_ND;
    o->perm = nullptr;
    o->block_width = 64;
    o->precision = SYM_F64;
    o->nd_leaf = 24;
    o->amalgamate = 1;
    o->pivot_floor_exp = 0;
}

int sym_analyze(int64_t n, const int64_t *Ap, const int32_t *Ai, const sym_opts *opts,
                sym_handle *out)
{
    if (!out) return SYM_EINVAL;
    *out = nullptr;
    sym_opts o;
    sym_opts_default(&o);
    if (opts) o = *opts;
    if (o.precision < SYM_F64 || o.precision > SYM_F16) return SYM_EINVAL;
    if (o.pivot_floor_exp < -60 || o.pivot_floor_exp > 1) return SYM_EINVAL;
    if (o.split_share < 0 || o.split_share > (1 << 24)) return SYM_EINVAL;
    if (o.chain_launch != 0 && o.chain_launch != 1) return SYM_EINVAL;
    if (o.update_depth < 0 || o.update_depth > sym::kMaxUpdateDepth) return SYM_EINVAL;
    sym_plan *h = new (std::nothrow) sym_plan();
    if (!h) return SYM_ENOMEM;
    int rc;
    try {
        h->P.precision = o.precision;
        if (o.split_share > 0) h->P.split_share = o.split_share;
        h->P.chain_launch = o.chain_launch != 0;
        if (o.update_depth > 0) h->P.update_depth = o.update_depth;
        // pivot floor of the scaled precisions: 2^exp, the default by format
        // (SYM_PIVOT_FLOOR_DEFAULT_*), or none (exp = 1)
        if (sym::prec_scaled(o.precision) && o.pivot_floor_exp != 1) {
            const int e = o.pivot_floor_exp != 0 ? o.pivot_floor_exp
                          : o.precision == SYM_BF16 ? SYM_PIVOT_FLOOR_DEFAULT_BF16
                                                    : SYM_PIVOT_FLOOR_DEFAULT_F16;
            h->P.pivot_floor = std::ldexp(1.0, e);
        }
        rc = sym::analyze(n, Ap, Ai, o.ordering, o.perm, o.block_width ? o.block_width : 64,
                          o.nd_leaf > 0 ? o.nd_leaf : 24, o.amalgamate != 0,
                          o.max_super_width ? o.max_super_width : sym::kMaxDeviceWidth, h->P);
        if (rc == SYM_OK) layout(h);
    } catch (const std::bad_alloc &) {
        rc = SYM_ENOMEM;
    } catch (const std::length_error &) {
        rc = SYM_ENOMEM;
    } catch (const std::logic_error &) {           // a schedule that failed its own check
        rc = SYM_ESCHED;
    }
    if (rc != SYM_OK) {
        delete h;
        return rc;
    }
    *out = h;
    return SYM_OK;
}

int sym_workspace(sym_handle h, size_t *bytes)
{
    if (!h || !bytes) return SYM_EINVAL;
    *bytes = h->ws_bytes;
    return SYM_OK;
}

int sym_bind(sym_handle h, void *dev_ws, size_t bytes, void *stream)
{
    if (!h || (!dev_ws && h->ws_bytes)) return SYM_EINVAL;
    if (bytes < h->ws_bytes || ((uintptr_t)dev_ws & 255)) return SYM_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)dev_ws;
    sym::DevicePlan &D = h->D;
    const sym::Plan &P = h->P;
    D.Lx = base + h->off_Lx;
    D.blk = (sym::BlockDesc *)(base + h->off_blk);
    D.rows = (int32_t *)(base + h->off_rows);
    D.tasks = (sym::Task *)(base + h->off_tasks);
    D.xslot = (int32_t *)(base + h->off_xslot);
    D.iptr = (int64_t *)(base + h->off_iptr);
    D.ibig = (int64_t *)(base + h->off_ibig);
    D.incs = (sym::Incidence *)(base + h->off_incs);
    D.imap = (uint8_t *)(base + h->off_imap);
    D.wptr = (int64_t *)(base + h->off_wptr);
    D.witems = (sym::WaveItem *)(base + h->off_witems);
    D.wmap = (uint8_t *)(base + h->off_wmap);
    D.level_blocks = (int32_t *)(base + h->off_lvl);
    D.amap = (int64_t *)(base + h->off_amap);
    D.perm = (int32_t *)(base + h->off_perm);
    D.vec = (double *)(base + h->off_vec);
    D.vec2 = (double *)(base + h->off_vec2);
    D.fwd_tasks = (sym::SolveTask *)(base + h->off_ftk);
    D.bwd_tasks = (sym::SolveTask *)(base + h->off_btk);
    D.info = (int32_t *)(base + h->off_info);
    D.vec3 = (double *)(base + h->off_vec3);
    D.arowptr = (int64_t *)(base + h->off_arp);
    D.acol = (int32_t *)(base + h->off_acol);
    D.aval = (int64_t *)(base + h->off_aval);
    D.red = (double *)(base + h->off_red);
    D.chunk_tptr = (int64_t *)(base + h->off_ctp);
    D.chunk_tgt = (int32_t *)(base + h->off_ctg);
    D.fwd_pend = (int32_t *)(base + h->off_fpend);
    D.bwd_pend = (int32_t *)(base + h->off_bpend);
    D.bwd_df = (sym::SolveTask *)(base + h->off_bdf);
    D.pend = (int32_t *)(base + h->off_sync);
    D.done = D.pend + P.nb;
    D.ticket = D.done + P.nb;
    D.vec4 = (double *)(base + h->off_vec4);
    D.vec5 = (double *)(base + h->off_vec5);
    D.vec6 = (double *)(base + h->off_vec6);
    D.part = (double *)(base + h->off_part);
    D.ttime = (uint64_t *)(base + h->off_ttime);
    D.parts = (sym::PartDesc *)(base + h->off_parts);
    D.pcount = (int32_t *)(base + h->off_pcount);
    D.pbuf = base + h->off_pbuf;
    D.inv_blocks = (int32_t *)(base + h->off_invb);
    D.cptr = (int64_t *)(base + h->off_cptr);
    D.chunks = (sym::StageChunk *)(base + h->off_chunks);
    D.fwd_slot_start = (int32_t *)(base + h->off_fss);
    D.fwd_slot_quad = (uint8_t *)(base + h->off_fsq);
    D.bwd_slot_start = (int32_t *)(base + h->off_bss);
    D.bwd_slot_quad = (uint8_t *)(base + h->off_bsq);
    D.tbase = (int32_t *)(base + h->off_tbase);
    D.tinit = (int32_t *)(base + h->off_tinit);
    D.tstate = (int32_t *)(base + h->off_tstate);
    D.cticket = (int32_t *)(base + h->off_ctk);
    D.bw_df = (sym::SolveTask *)(base + h->off_bwdf);
    D.bw_tptr = (int64_t *)(base + h->off_bwtp);
    D.bw_tgt = (int32_t *)(base + h->off_bwtg);
    D.bw_pend = (int32_t *)(base + h->off_bwpd);
    D.bw_slot_start = (int32_t *)(base + h->off_bwss);
    D.bw_slot_quad = (uint8_t *)(base + h->off_bwsq);
    const bool sc = sym::prec_scaled(P.precision);
    D.dscale = sc ? (double *)(base + h->off_dscale) : nullptr;
    D.pfloor = sc ? (double *)(base + h->off_pfloor) : nullptr;
    D.adiag = sc ? (int64_t *)(base + h->off_adiag) : nullptr;
    D.acoord = sc ? (int32_t *)(base + h->off_acoord) : nullptr;
    D.dsptr = sc ? (int32_t *)(base + h->off_dsptr) : nullptr;
    hipError_t e = hipSuccess;
    e = upload(D.cptr, P.cptr.data(), sizeof(int64_t) * P.cptr.size(), s);
    if (e == hipSuccess) e = upload(D.chunks, P.chunks.data(), sizeof(sym::StageChunk) * P.chunks.size(), s);
    if (e == hipSuccess)
        e = upload(D.fwd_slot_start, P.fwd_slots.start.data(), sizeof(int32_t) * P.fwd_slots.start.size(), s);
    if (e == hipSuccess) e = upload(D.fwd_slot_quad, P.fwd_slots.quad.data(), P.fwd_slots.quad.size(), s);
    if (e == hipSuccess)
        e = upload(D.bwd_slot_start, P.bwd_slots.start.data(), sizeof(int32_t) * P.bwd_slots.start.size(), s);
    if (e == hipSuccess) e = upload(D.bwd_slot_quad, P.bwd_slots.quad.data(), P.bwd_slots.quad.size(), s);
    if (e == hipSuccess) e = upload(D.tbase, P.tbase.data(), sizeof(int32_t) * P.tbase.size(), s);
    if (e == hipSuccess) e = upload(D.tinit, P.tinit.data(), sizeof(int32_t) * P.tinit.size(), s);
    if (e == hipSuccess) e = upload(D.bw_df, P.bw_df.data(), sizeof(sym::SolveTask) * P.bw_df.size(), s);
    if (e == hipSuccess) e = upload(D.bw_tptr, P.bw_tptr.data(), sizeof(int64_t) * P.bw_tptr.size(), s);
    if (e == hipSuccess) e = upload(D.bw_tgt, P.bw_tgt.data(), sizeof(int32_t) * P.bw_tgt.size(), s);
    if (e == hipSuccess) e = upload(D.bw_pend, P.bw_pend.data(), sizeof(int32_t) * P.bw_pend.size(), s);
    if (e == hipSuccess)
        e = upload(D.bw_slot_start, P.bw_slots.start.data(), sizeof(int32_t) * P.bw_slots.start.size(), s);
    if (e == hipSuccess) e = upload(D.bw_slot_quad, P.bw_slots.quad.data(), P.bw_slots.quad.size(), s);
    if (sc && e == hipSuccess) {
        e = upload(D.adiag, P.adiag.data(), sizeof(int64_t) * P.adiag.size(), s);
        if (e == hipSuccess) e = upload(D.acoord, P.acoord.data(), sizeof(int32_t) * P.acoord.size(), s);
        if (e == hipSuccess) e = upload(D.dsptr, P.dsptr.data(), sizeof(int32_t) * P.dsptr.size(), s);
    }
    if (e == hipSuccess) e = upload(D.blk, P.blk.data(), sizeof(sym::BlockDesc) * P.blk.size(), s);
    if (e == hipSuccess) e = upload(D.rows, P.dsrows.data(), sizeof(int32_t) * P.dsrows.size(), s);
    if (e == hipSuccess) e = upload(D.tasks, P.ftasks.data(), sizeof(sym::Task) * P.ftasks.size(), s);
    if (e == hipSuccess) e = upload(D.xslot, P.xslot.data(), sizeof(int32_t) * P.xslot.size(), s);
    if (e == hipSuccess) e = upload(D.iptr, P.iptr.data(), sizeof(int64_t) * P.iptr.size(), s);
    if (e == hipSuccess) e = upload(D.ibig, P.ibig.data(), sizeof(int64_t) * P.ibig.size(), s);
    if (e == hipSuccess) e = upload(D.incs, P.incs.data(), sizeof(sym::Incidence) * P.incs.size(), s);
    if (e == hipSuccess) e = upload(D.imap, P.imap.data(), P.imap.size(), s);
    if (e == hipSuccess) e = upload(D.wptr, P.wptr.data(), sizeof(int64_t) * P.wptr.size(), s);
    if (e == hipSuccess)
        e = upload(D.witems, P.witems.data(), sizeof(sym::WaveItem) * P.witems.size(), s);
    if (e == hipSuccess) e = upload(D.wmap, P.wmap.data(), P.wmap.size(), s);
    if (e == hipSuccess) e = upload(D.level_blocks, P.level_blocks.data(), sizeof(int32_t) * P.level_blocks.size(), s);
    if (e == hipSuccess) e = upload(D.amap, P.amap.data(), sizeof(int64_t) * P.amap.size(), s);
    if (e == hipSuccess) e = upload(D.perm, P.perm.data(), sizeof(int32_t) * P.perm.size(), s);
    if (e == hipSuccess)
        e = upload(D.fwd_tasks, P.fwd_tasks.data(), sizeof(sym::SolveTask) * P.fwd_tasks.size(), s);
    if (e == hipSuccess)
        e = upload(D.bwd_tasks, P.bwd_tasks.data(), sizeof(sym::SolveTask) * P.bwd_tasks.size(), s);
    if (e == hipSuccess)
        e = upload(D.chunk_tptr, P.chunk_tptr.data(), sizeof(int64_t) * P.chunk_tptr.size(), s);
    if (e == hipSuccess)
        e = upload(D.chunk_tgt, P.chunk_tgt.data(), sizeof(int32_t) * P.chunk_tgt.size(), s);
    if (e == hipSuccess) e = upload(D.fwd_pend, P.fwd_pend.data(), sizeof(int32_t) * P.fwd_pend.size(), s);
    if (e == hipSuccess) e = upload(D.bwd_pend, P.bwd_pend.data(), sizeof(int32_t) * P.bwd_pend.size(), s);
    if (e == hipSuccess) e = upload(D.bwd_df, P.bwd_df.data(), sizeof(sym::SolveTask) * P.bwd_df.size(), s);
    if (e == hipSuccess && !P.ftasks.empty())
        e = hipMemsetAsync(D.ttime, 0, sizeof(uint64_t) * P.ftasks.size(), s);
    if (e == hipSuccess) e = upload(D.parts, P.parts.data(), sizeof(sym::PartDesc) * P.parts.size(), s);
    if (e == hipSuccess)
        e = upload(D.inv_blocks, P.inv_blocks.data(), sizeof(int32_t) * P.inv_blocks.size(), s);
    if (e == hipSuccess && P.nsplit > 0)
        e = hipMemsetAsync(D.pcount, 0, sizeof(int32_t) * (size_t)P.nsplit, s);
    if (e == hipSuccess) e = upload(D.arowptr, P.arowptr.data(), sizeof(int64_t) * P.arowptr.size(), s);
    if (e == hipSuccess) e = upload(D.acol, P.acol.data(), sizeof(int32_t) * P.acol.size(), s);
    if (e == hipSuccess) e = upload(D.aval, P.aval.data(), sizeof(int64_t) * P.aval.size(), s);
    h->generation++;
    if (e != hipSuccess) return SYM_EHIP;
    h->bound = true;
    h->factored = false;
    h->stream = s;
    return SYM_OK;
}

int sym_factor(sym_handle h, const double *Ax_dev, void *stream)
{
    if (!h || (!Ax_dev && h->P.nnzA)) return SYM_EINVAL;
    if (!h->bound) return SYM_ESTATE;
    hipStream_t s = (hipStream_t)stream;
    h->stream = s;
    if (sym::launch_factor(h->P, h->D, Ax_dev, s, h->profiling ? &h->prof : nullptr) != hipSuccess)
        return SYM_EHIP;
    h->factored = true;
    return SYM_OK;
}

int sym_solve_lower(sym_handle h, const double *b_dev, double *y_dev, void *stream)
{
    if (!h || ((!b_dev || !y_dev) && h->P.n)) return SYM_EINVAL;
    if (!h->bound || !h->factored) return SYM_ESTATE;
    hipStream_t s = (hipStream_t)stream;
    h->stream = s;
    if (b_dev == y_dev) return SYM_EINVAL;
    if (sym::launch_perm_gather(h->P, h->D, b_dev, h->D.vec, s) != hipSuccess) return SYM_EHIP;
    if (sym::launch_fwd(h->P, h->D, h->D.vec, y_dev, s) != hipSuccess) return SYM_EHIP;
    return SYM_OK;
}

int sym_solve_upper(sym_handle h, double *y_dev, void *stream)
{
    if (!h || (!y_dev && h->P.n)) return SYM_EINVAL;
    if (!h->bound || !h->factored) return SYM_ESTATE;
    hipStream_t s = (hipStream_t)stream;
    h->stream = s;
    if (sym::launch_bwd(h->P, h->D, y_dev, s) != hipSuccess) return SYM_EHIP;
    // L = D^{-1} L-hat for a scaled factor, so L^{-T} y = D L-hat^{-T} y
    if (sym::launch_scale(h->P, h->D, y_dev, s) != hipSuccess) return SYM_EHIP;
    return SYM_OK;
}

int sym_solve(sym_handle h, double *bx_dev, void *stream)
{
    if (!h || (!bx_dev && h->P.n)) return SYM_EINVAL;
    if (!h->bound || !h->factored) return SYM_ESTATE;
    hipStream_t s = (hipStream_t)stream;
    h->stream = s;
    double *acc = h->D.vec, *y = h->D.vec2;
    if (sym::launch_perm_gather(h->P, h->D, bx_dev, acc, s) != hipSuccess) return SYM_EHIP;
    if (sym::launch_fwd(h->P, h->D, acc, y, s) != hipSuccess) return SYM_EHIP;
    if (sym::launch_bwd(h->P, h->D, y, s) != hipSuccess) return SYM_EHIP;
    if (sym::launch_perm_scatter(h->P, h->D, y, bx_dev, s) != hipSuccess) return SYM_EHIP;
    return SYM_OK;
}

int sym_solve_static(sym_handle h, double *bx_dev, void *stream)
{
    if (!h || (!bx_dev && h->P.n)) return SYM_EINVAL;
    const sym::Plan &P = h->P;
    if ((int64_t)P.n > sym::kStaticMaxN || (int64_t)P.nb > sym::kStaticMaxN) return SYM_EWORKSPACE;
    if (!h->bound || !h->factored) return SYM_ESTATE;
    hipStream_t s = (hipStream_t)stream;
    h->stream = s;
    if (P.n == 0) return SYM_OK;
    void *base = nullptr;
    if (sym::static_scratch(&base) != hipSuccess) return SYM_EHIP;
    // the bound plan and factor, with the sweeps' scratch in the static array
    sym::DevicePlan D = h->D;
    char *sc = (char *)base;
    D.vec = (double *)sc;
    D.vec2 = (double *)(sc + sym::kStaticOffVec2);
    D.pend = (int32_t *)(sc + sym::kStaticOffPend);
    D.done = (int32_t *)(sc + sym::kStaticOffDone);
    D.ticket = (int32_t *)(sc + sym::kStaticOffTicket);
    if (sym::launch_perm_gather(P, D, bx_dev, D.vec, s) != hipSuccess) return SYM_EHIP;
    if (sym::launch_fwd(P, D, D.vec, D.vec2, s) != hipSuccess) return SYM_EHIP;
    if (sym::launch_bwd(P, D, D.vec2, s) != hipSuccess) return SYM_EHIP;
    if (sym::launch_perm_scatter(P, D, D.vec2, bx_dev, s) != hipSuccess) return SYM_EHIP;
    return SYM_OK;
}

int sym_refine(sym_handle h, const double *Ax_dev, const double *b_dev, double *x_dev, double tol,
               int32_t maxit, void *stream, int32_t *iters, double *eta)
{
    if (!h || ((!Ax_dev || !b_dev || !x_dev) && h->P.n) || maxit < 0 || !(tol >= 0.0)) return SYM_EINVAL;
    if (!h->bound || !h->factored) return SYM_ESTATE;
    hipStream_t s = (hipStream_t)stream;
    h->stream = s;
    const sym::Plan &P = h->P;
    const sym::DevicePlan &D = h->D;
    const size_t bytes = sizeof(double) * (size_t)P.n;
    if (P.n == 0) {
        if (iters) *iters = 0;
        if (eta) *eta = 0.0;
        return SYM_OK;
    }
    // x0 = solve(b)
    if (hipMemcpyAsync(x_dev, b_dev, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) return SYM_EHIP;
    int rc = sym_solve(h, x_dev, stream);
    if (rc != SYM_OK) return rc;
    double red[4] = {0, 0, 0, 0};
    double e = 0.0;
    int32_t it = 0;
    bool pivot_failed = false;
    for (;;) {
        if (sym::launch_residual(P, D, Ax_dev, b_dev, x_dev, D.vec3, it == 0, s) != hipSuccess) return SYM_EHIP;
        double cur[4];
        if (hipMemcpyAsync(cur, D.red, sizeof(cur), hipMemcpyDeviceToHost, s) != hipSuccess) return SYM_EHIP;
        if (it == 0 && !read_pivot_failed(h, s, pivot_failed)) return SYM_EHIP;
        if (hipStreamSynchronize(s) != hipSuccess) return SYM_EHIP;
        if (it == 0) red[1] = cur[1];
        e = backward_error(red[1], cur);
        if (!(e > tol) || it >= maxit || pivot_failed) break;      // also stops on NaN
        rc = sym_solve(h, D.vec3, stream);           // correction, in place
        if (rc != SYM_OK) return rc;
        if (sym::launch_axpy(P, D, x_dev, D.vec3, s) != hipSuccess) return SYM_EHIP;
        ++it;
    }
    if (iters) *iters = it;
    if (eta) *eta = e;
    return (pivot_failed || !std::isfinite(e)) ? SYM_ENUMERIC : SYM_OK;
}

int sym_set_variants(sym_handle h, const uint8_t *variant, int32_t count)
{
    if (!h || (!variant && count) || count != h->P.nds) return SYM_EINVAL;
    for (int32_t s2 = 0; s2 < count; ++s2)
        if (variant[s2] >= sym::kVariants) return SYM_EINVAL;
    try {
        h->P.svariant.assign(variant, variant + count);
        sym::build_schedule(h->P);
    } catch (const std::bad_alloc &) {
        return SYM_ENOMEM;
    } catch (const std::length_error &) {
        return SYM_ENOMEM;
    } catch (const std::logic_error &) {
        return SYM_ESCHED;
    }
    layout(h);
    h->bound = false;
    h->factored = false;
    h->generation++;
    return SYM_OK;
}

int sym_task_times(sym_handle h, double *us)
{
    if (!h || (!us && !h->P.ftasks.empty())) return SYM_EINVAL;
    if (!h->bound) return SYM_ESTATE;
    const size_t nt = h->P.ftasks.size();
    if (nt == 0) return SYM_OK;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return SYM_EHIP;
    std::vector<uint64_t> ticks(nt);
    if (hipMemcpy(ticks.data(), h->D.ttime, sizeof(uint64_t) * nt, hipMemcpyDeviceToHost) != hipSuccess)
        return SYM_EHIP;
    // the device's constant wall clock runs at 100 MHz
    for (size_t q = 0; q < nt; ++q) us[q] = (double)ticks[q] * 0.01;
    return SYM_OK;
}

int sym_refine_pcg(sym_handle h, const double *Ax_dev, const double *b_dev, double *x_dev,
                   double tol, int32_t maxit, void *stream, int32_t *iters, double *eta)
{
    if (!h || ((!Ax_dev || !b_dev || !x_dev) && h->P.n) || maxit < 0 || !(tol >= 0.0)) return SYM_EINVAL;
    if (!h->bound || !h->factored) return SYM_ESTATE;
    hipStream_t s = (hipStream_t)stream;
    h->stream = s;
    const sym::Plan &P = h->P;
    const sym::DevicePlan &D = h->D;
    const size_t bytes = sizeof(double) * (size_t)P.n;
    if (P.n == 0) {
        if (iters) *iters = 0;
        if (eta) *eta = 0.0;
        return SYM_OK;
    }
    double *r = D.vec3, *p = D.vec4, *q = D.vec5, *z = D.vec6;
    double *scal = D.part + sym::kDotParts;     // device slots of the dot products
    auto fetch = [&](const double *dev, double *host, size_t count) {
        if (hipMemcpyAsync(host, dev, sizeof(double) * count, hipMemcpyDeviceToHost, s) != hipSuccess)
            return false;
        return hipStreamSynchronize(s) == hipSuccess;
    };
    // x0 = M b
    if (hipMemcpyAsync(x_dev, b_dev, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) return SYM_EHIP;
    int rc = sym_solve(h, x_dev, stream);
    if (rc != SYM_OK) return rc;
    double anorm = 0.0, e = 0.0, rho = 0.0;
    int32_t it = 0;
    bool pivot_failed = false;
    for (;;) {
        // true residual and its backward error
        if (sym::launch_residual(P, D, Ax_dev, b_dev, x_dev, r, it == 0, s) != hipSuccess) return SYM_EHIP;
        double cur[4];
        if (it == 0 && !read_pivot_failed(h, s, pivot_failed)) return SYM_EHIP;
        if (!fetch(D.red, cur, 4)) return SYM_EHIP;
        if (it == 0) anorm = cur[1];
        e = backward_error(anorm, cur);
        if (!(e > tol) || it >= maxit || pivot_failed) break;      // also stops on NaN
        // z = M r, rho' = r . z, p = z + (rho' / rho) p
        if (hipMemcpyAsync(z, r, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) return SYM_EHIP;
        rc = sym_solve(h, z, stream);
        if (rc != SYM_OK) return rc;
        if (sym::launch_dot(P, D, r, z, scal, s) != hipSuccess) return SYM_EHIP;
        double rho_new;
        if (!fetch(scal, &rho_new, 1)) return SYM_EHIP;
        if (it == 0) {
            if (hipMemcpyAsync(p, z, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) return SYM_EHIP;
        } else if (sym::launch_xpby(P, p, z, rho_new / rho, s) != hipSuccess) {
            return SYM_EHIP;
        }
        rho = rho_new;
        // x += (rho / p.Ap) p
        if (sym::launch_spmv(P, D, Ax_dev, p, q, s) != hipSuccess) return SYM_EHIP;
        if (sym::launch_dot(P, D, p, q, scal + 1, s) != hipSuccess) return SYM_EHIP;
        double pq;
        if (!fetch(scal + 1, &pq, 1)) return SYM_EHIP;
        if (!(pq > 0.0)) break;                        // breakdown (not SPD, or converged to 0)
        if (sym::launch_axpy_s(P, x_dev, rho / pq, p, s) != hipSuccess) return SYM_EHIP;
        ++it;
    }
    if (iters) *iters = it;
    if (eta) *eta = e;
    return (pivot_failed || !std::isfinite(e)) ? SYM_ENUMERIC : SYM_OK;
}

int sym_rhs_analyze(sym_handle h, int64_t nb, const int32_t *bi, sym_rhs *out)
{
    if (!h || !out || nb < 0 || (nb > 0 && !bi)) return SYM_EINVAL;
    *out = nullptr;
    const sym::Plan &P = h->P;
    sym_rhs_plan *r = new (std::nothrow) sym_rhs_plan();
    if (!r) return SYM_ENOMEM;
    try {
        r->h = h;
        std::vector<char> seen((size_t)P.n, 0);
        std::vector<int32_t> beta;
        beta.reserve((size_t)nb);
        for (int64_t k = 0; k < nb; ++k) {
            int32_t i = bi[k];
            if (i < 0 || i >= P.n || seen[i]) { delete r; return SYM_EINVAL; }
            seen[i] = 1;
            beta.push_back(P.pinv[i]);
        }
        r->bpos = beta;
        sym::reach_etree(P, beta, r->reach);
        // touched blocks and their first reached column, grouped by level
        std::vector<int32_t> bfirst((size_t)P.nb, INT32_MAX);
        std::vector<int32_t> touched;
        for (int32_t c : r->reach) {
            int32_t b = P.col2blk[c];
            if (bfirst[b] == INT32_MAX) touched.push_back(b);
            bfirst[b] = std::min(bfirst[b], c - P.blk[b].col0);
        }
        std::stable_sort(touched.begin(), touched.end(),
                         [&](int32_t a, int32_t b) { return P.blevel[a] < P.blevel[b]; });
        r->level_ptr.push_back(0);
        int32_t cur = -1;
        for (int32_t b : touched) {
            if (P.blevel[b] != cur && !r->tasks.empty()) r->level_ptr.push_back((int64_t)r->tasks.size());
            cur = P.blevel[b];
            const int32_t nch =
                std::max(1, (P.blk[b].r - P.blk[b].w + sym::kSolveChunk - 1) / sym::kSolveChunk);
            for (int32_t ch = 0; ch < nch; ++ch)
                r->tasks.push_back(sym::SolveTask{b, ch, bfirst[b], P.fwd_first[b] + ch});
        }
        if (!r->tasks.empty()) r->level_ptr.push_back((int64_t)r->tasks.size());
        // counters of the pruned sweep: only its own chunks contribute (the
        // blocks they update hold ancestors of reached columns, so are
        // touched themselves)
        r->pend.assign((size_t)P.nb, 0);
        for (const sym::SolveTask &t : r->tasks)
            for (int64_t q = P.chunk_tptr[t.list]; q < P.chunk_tptr[t.list + 1]; ++q)
                r->pend[P.chunk_tgt[q]]++;
        size_t o = 0;
        auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
        r->off_tasks = take(sizeof(sym::SolveTask) * r->tasks.size());
        r->off_bpos = take(sizeof(int32_t) * r->bpos.size());
        r->off_pend = take(sizeof(int32_t) * r->pend.size());
        r->slots = sym::sweep_slots(P, r->tasks, true);
        r->off_ss = take(sizeof(int32_t) * r->slots.start.size());
        r->off_sq = take(r->slots.quad.size());
        r->ws_bytes = std::max<size_t>(o, 256);
    } catch (const std::bad_alloc &) {
        delete r;
        return SYM_ENOMEM;
    }
    *out = r;
    return SYM_OK;
}

int sym_rhs_workspace(sym_rhs r, size_t *bytes)
{
    if (!r || !bytes) return SYM_EINVAL;
    *bytes = r->ws_bytes;
    return SYM_OK;
}

int sym_rhs_bind(sym_rhs r, void *dev_ws, size_t bytes, void *stream)
{
    if (!r || !dev_ws) return SYM_EINVAL;
    if (bytes < r->ws_bytes || ((uintptr_t)dev_ws & 255)) return SYM_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)dev_ws;
    r->R.tasks = (sym::SolveTask *)(base + r->off_tasks);
    r->R.bpos = (int32_t *)(base + r->off_bpos);
    r->R.pend = (int32_t *)(base + r->off_pend);
    r->R.ntasks = (int64_t)r->tasks.size();
    r->R.slot_start = (int32_t *)(base + r->off_ss);
    r->R.slot_quad = (uint8_t *)(base + r->off_sq);
    r->R.nslots = r->slots.count();
    hipError_t e = upload(r->R.tasks, r->tasks.data(), sizeof(sym::SolveTask) * r->tasks.size(), s);
    if (e == hipSuccess)
        e = upload(r->R.slot_start, r->slots.start.data(), sizeof(int32_t) * r->slots.start.size(), s);
    if (e == hipSuccess) e = upload(r->R.slot_quad, r->slots.quad.data(), r->slots.quad.size(), s);
    if (e == hipSuccess) e = upload(r->R.bpos, r->bpos.data(), sizeof(int32_t) * r->bpos.size(), s);
    if (e == hipSuccess) e = upload(r->R.pend, r->pend.data(), sizeof(int32_t) * r->pend.size(), s);
    if (e != hipSuccess) return SYM_EHIP;
    r->bound = true;
    return SYM_OK;
}

int sym_solve_lower_sparse(sym_handle h, sym_rhs r, const double *bv_dev, double *y_dev,
                           void *stream)
{
    if (!h || !r || r->h != h || (!y_dev && h->P.n) || (!bv_dev && !r->bpos.empty()))
        return SYM_EINVAL;
    if (!h->bound || !h->factored || !r->bound) return SYM_ESTATE;
    hipStream_t s = (hipStream_t)stream;
    h->stream = s;
    if (sym::launch_fwd_sparse(h->P, h->D, r->R, (int64_t)r->bpos.size(), bv_dev, h->D.vec, y_dev,
                               s) != hipSuccess)
        return SYM_EHIP;
    return SYM_OK;
}

int sym_solve_sparse(sym_handle h, sym_rhs r, const double *bv_dev, double *x_dev, void *stream)
{
    if (!h || !r || r->h != h || (!x_dev && h->P.n) || (!bv_dev && !r->bpos.empty()))
        return SYM_EINVAL;
    if (!h->bound || !h->factored || !r->bound) return SYM_ESTATE;
    hipStream_t s = (hipStream_t)stream;
    h->stream = s;
    if (h->P.n == 0) return SYM_OK;
    double *y = h->D.vec2;
    if (sym::launch_fwd_sparse(h->P, h->D, r->R, (int64_t)r->bpos.size(), bv_dev, h->D.vec, y, s) !=
        hipSuccess)
        return SYM_EHIP;
    if (sym::launch_bwd(h->P, h->D, y, s) != hipSuccess) return SYM_EHIP;
    if (sym::launch_perm_scatter(h->P, h->D, y, x_dev, s) != hipSuccess) return SYM_EHIP;
    return SYM_OK;
}

int sym_status(sym_handle h, int64_t *info)
{
    if (!h || !info) return SYM_EINVAL;
    if (!h->bound || !h->factored) return SYM_ESTATE;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return SYM_EHIP;
    int32_t w[3];
    if (hipMemcpy(w, h->D.info, sizeof(w), hipMemcpyDeviceToHost) != hipSuccess) return SYM_EHIP;
    if (w[1] != INT32_MAX || w[2] != 0) return SYM_ESCHED;
    *info = w[0] == INT32_MAX ? 0 : 1 + (int64_t)h->P.perm[w[0]];
    return SYM_OK;
}

int sym_pivots_perturbed(sym_handle h, int64_t *count)
{
    if (!h || !count) return SYM_EINVAL;
    if (!h->bound || !h->factored) return SYM_ESTATE;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return SYM_EHIP;
    int32_t w[4];
    if (hipMemcpy(w, h->D.info, sizeof(w), hipMemcpyDeviceToHost) != hipSuccess) return SYM_EHIP;
    *count = w[3];
    return SYM_OK;
}

int sym_export_factor(sym_handle h, double *Lx_host, void *stream)
{
    if (!h || (!Lx_host && h->P.nnzL)) return SYM_EINVAL;
    if (!h->bound || !h->factored) return SYM_ESTATE;
    const sym::Plan &P = h->P;
    hipStream_t s = (hipStream_t)stream;
    if (hipStreamSynchronize(s) != hipSuccess) return SYM_EHIP;
    const size_t es = elem_size(P);
    std::vector<char> panel;
    try {
        panel.resize((size_t)P.panel_entries * es);
    } catch (const std::bad_alloc &) {
        return SYM_ENOMEM;
    }
    if (!panel.empty() &&
        hipMemcpy(panel.data(), h->D.Lx, panel.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return SYM_EHIP;
    // a scaled factor holds D L: row i divided by d_i gives L
    std::vector<double> dsc;
    if (h->D.dscale) {
        try {
            dsc.resize((size_t)P.n);
        } catch (const std::bad_alloc &) {
            return SYM_ENOMEM;
        }
        if (P.n > 0 && hipMemcpy(dsc.data(), h->D.dscale, sizeof(double) * (size_t)P.n,
                                 hipMemcpyDeviceToHost) != hipSuccess)
            return SYM_EHIP;
    }
    int64_t q = 0;
    for (int32_t s = 0; s < P.ns; ++s) {
        const int32_t *frows = P.srows.data() + P.srowptr[s];
        const int32_t fr = (int32_t)(P.srowptr[s + 1] - P.srowptr[s]);
        for (int32_t c = P.sptr[s]; c < P.sptr[s + 1]; ++c) {
            const sym::BlockDesc &d = P.blk[P.col2blk[c]];
            const int32_t *drows = P.dsrows.data() + d.rowoff;
            const int32_t lc = c - d.col0;
            for (int32_t p = c - P.sptr[s]; p < fr; ++p) {
                const int32_t lr = (int32_t)(std::lower_bound(drows + lc, drows + d.r, frows[p]) - drows);
                const int64_t off = d.valoff + (int64_t)lc * d.ld + lr;
                double v = es == sizeof(float) ? (double)((const float *)panel.data())[off]
                                               : ((const double *)panel.data())[off];
                if (!dsc.empty()) v /= dsc[frows[p]];
                Lx_host[q++] = v;
            }
        }
    }
    return SYM_OK;
}

int sym_get_size(sym_handle h, int what, int64_t *count)
{
    if (!h || !count) return SYM_EINVAL;
    const sym::Plan &P = h->P;
    switch (what) {
    case SYM_GET_PERM: case SYM_GET_PARENT: case SYM_GET_COLCOUNT: *count = P.n; break;
    case SYM_GET_LP: *count = (int64_t)P.n + 1; break;
    case SYM_GET_LI: *count = P.nnzL; break;
    case SYM_GET_SUPER: *count = (int64_t)P.ns + 1; break;
    case SYM_GET_SPARENT: *count = P.ns; break;
    case SYM_GET_BLOCKS: *count = (int64_t)P.nb + 1; break;
    case SYM_GET_BLEVEL: *count = P.nb; break;
    case SYM_GET_SUPER_FEAT: *count = (int64_t)P.nds * sym::kSuperFeatures; break;
    case SYM_GET_TASK_SUPER: *count = (int64_t)P.ftasks.size(); break;
    case SYM_GET_VARIANT: *count = P.nds; break;
    default: return SYM_EINVAL;
    }
    return SYM_OK;
}

int sym_get(sym_handle h, int what, void *out)
{
    if (!h || !out) return SYM_EINVAL;
    const sym::Plan &P = h->P;
    switch (what) {
    case SYM_GET_PERM: std::memcpy(out, P.perm.data(), sizeof(int32_t) * P.perm.size()); break;
    case SYM_GET_SUPER_FEAT: std::memcpy(out, P.sfeat.data(), sizeof(double) * P.sfeat.size()); break;
    case SYM_GET_TASK_SUPER:
        std::memcpy(out, P.task_super.data(), sizeof(int32_t) * P.task_super.size());
        break;
    case SYM_GET_VARIANT: std::memcpy(out, P.svariant.data(), P.svariant.size()); break;
    case SYM_GET_PARENT: std::memcpy(out, P.parent.data(), sizeof(int32_t) * P.parent.size()); break;
    case SYM_GET_COLCOUNT: std::memcpy(out, P.colcount.data(), sizeof(int64_t) * P.colcount.size()); break;
    case SYM_GET_LP: {
        int64_t *Lp = (int64_t *)out;
        Lp[0] = 0;
        for (int32_t j = 0; j < P.n; ++j) Lp[j + 1] = Lp[j] + P.colcount[j];
        break;
    }
    case SYM_GET_LI: {
        int32_t *Li = (int32_t *)out;
        int64_t q = 0;
        for (int32_t s = 0; s < P.ns; ++s) {
            const int32_t *frows = P.srows.data() + P.srowptr[s];
            const int32_t fr = (int32_t)(P.srowptr[s + 1] - P.srowptr[s]);
            for (int32_t c = P.sptr[s]; c < P.sptr[s + 1]; ++c)
                for (int32_t p = c - P.sptr[s]; p < fr; ++p) Li[q++] = frows[p];
        }
        break;
    }
    case SYM_GET_SUPER: std::memcpy(out, P.sptr.data(), sizeof(int32_t) * P.sptr.size()); break;
    case SYM_GET_SPARENT: std::memcpy(out, P.sparent.data(), sizeof(int32_t) * P.sparent.size()); break;
    case SYM_GET_BLOCKS: std::memcpy(out, P.bptr.data(), sizeof(int32_t) * P.bptr.size()); break;
    case SYM_GET_BLEVEL: std::memcpy(out, P.blevel.data(), sizeof(int32_t) * P.blevel.size()); break;
    default: return SYM_EINVAL;
    }
    return SYM_OK;
}

int sym_rhs_get(sym_rhs r, int64_t *count, int32_t *cols)
{
    if (!r || !count) return SYM_EINVAL;
    *count = (int64_t)r->reach.size();
    if (cols) std::memcpy(cols, r->reach.data(), sizeof(int32_t) * r->reach.size());
    return SYM_OK;
}

int sym_stat(sym_handle h, int what, double *v)
{
    if (!h || !v) return SYM_EINVAL;
    const sym::Plan &P = h->P;
    switch (what) {
    case SYM_STAT_N: *v = P.n; break;
    case SYM_STAT_NNZA: *v = (double)P.nnzA; break;
    case SYM_STAT_NNZL: *v = (double)P.nnzL; break;
    case SYM_STAT_FLOPS: *v = P.flops; break;
    case SYM_STAT_NSUPER: *v = P.ns; break;
    case SYM_STAT_NBLOCKS: *v = P.nb; break;
    case SYM_STAT_NLEVELS: *v = P.nlevels; break;
    case SYM_STAT_NPAIRS: *v = (double)P.pairs.size(); break;
    case SYM_STAT_PANEL_ENTRIES: *v = (double)P.panel_entries; break;
    case SYM_STAT_ANALYZE_MS: *v = P.analyze_ms; break;
    case SYM_STAT_NPHASES: *v = (double)P.phases.size(); break;
    case SYM_STAT_NINCIDENCES: *v = (double)P.incs.size(); break;
    case SYM_STAT_NSLEVELS: *v = P.nslevels; break;
    case SYM_STAT_NDSUPER: *v = P.nds; break;
    case SYM_STAT_EXT_OPERAND_ENTRIES: *v = P.ext_operand_entries; break;
    case SYM_STAT_WALKERS: *v = P.nwalk; break;
    case SYM_STAT_STORED_LOWER: {
        double st = 0;
        for (int32_t r = 0; r < P.nds; ++r) {
            const double W = P.dsptr[r + 1] - P.dsptr[r];
            const double R = (double)(P.dsrowptr[r + 1] - P.dsrowptr[r]);
            st += W * (W + 1) / 2 + W * (R - W);
        }
        *v = st;
        break;
    }
    case SYM_STAT_SUM_ROWS: {
        double s = 0;
        for (const auto &d : P.blk) s += d.r;
        *v = s;
        break;
    }
    default: return SYM_EINVAL;
    }
    return SYM_OK;
}

int sym_profile(sym_handle h, int enable)
{
    if (!h) return SYM_EINVAL;
    h->profiling = enable != 0;
    if (h->profiling) {
        // brackets: the scatter, every phase, the diagonal inverses
        const size_t need = 2 * (h->P.phases.size() + 2);
        while (h->prof.ev.size() < need) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return SYM_EHIP;
            h->prof.ev.push_back(e);
        }
        h->prof.kind.assign(h->P.phases.size() + 2, 0);
        h->prof.used = 0;
    }
    return SYM_OK;
}

int sym_profile_read(sym_handle h, double *ms, int64_t *launches, double *algorithmic_flops)
{
    if (!h || !ms || !launches) return SYM_EINVAL;
    for (int k = 0; k < SYM_PROFILE_KINDS; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
        if (algorithmic_flops) algorithmic_flops[k] = h->P.kind_flops[k];
    }
    if (!h->profiling || h->prof.used == 0) return SYM_ESTATE;
    if (hipEventSynchronize(h->prof.ev[2 * h->prof.used - 1]) != hipSuccess) return SYM_EHIP;
    for (int32_t i = 0; i < h->prof.used; ++i) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, h->prof.ev[2 * i], h->prof.ev[2 * i + 1]) != hipSuccess) return SYM_EHIP;
        ms[h->prof.kind[i]] += t;
        launches[h->prof.kind[i]] += 1;
    }
    return SYM_OK;
}

void sym_destroy(sym_handle h) { delete h; }
void sym_rhs_destroy(sym_rhs r) { delete r; }


// ------------------------------------------------------------ cost model

int sym_mlp_param_count(int32_t d_in, int64_t *count)
{
    if (!count || d_in < 1 || d_in > sym::kMlpMaxIn) return SYM_EINVAL;
    *count = sym::mlp_param_count(d_in);
    return SYM_OK;
}

int sym_mlp_work_size(int32_t n, int32_t d_in, int64_t *floats)
{
    if (!floats || n < 0 || d_in < 1 || d_in > sym::kMlpMaxIn) return SYM_EINVAL;
    *floats = sym::mlp_work_floats(n, d_in);
    return SYM_OK;
}

int sym_mlp_forward(const float *params_dev, const float *X_dev, int32_t n, int32_t d_in,
                    float *y_dev, void *stream)
{
    if (d_in < 1 || d_in > sym::kMlpMaxIn || n < 0 || !params_dev || (n && (!X_dev || !y_dev)))
        return SYM_EINVAL;
    return sym::launch_mlp_forward(params_dev, X_dev, n, d_in, y_dev, (hipStream_t)stream) == hipSuccess
               ? SYM_OK : SYM_EHIP;
}

int sym_mlp_backward(const float *params_dev, const float *X_dev, const float *t_dev, int32_t n,
                     int32_t d_in, float *grad_dev, float *work_dev, void *stream)
{
    if (d_in < 1 || d_in > sym::kMlpMaxIn || n < 1 || !params_dev || !X_dev || !t_dev || !grad_dev ||
        !work_dev)
        return SYM_EINVAL;
    return sym::launch_mlp_backward(params_dev, X_dev, t_dev, n, d_in, grad_dev, work_dev,
                                    (hipStream_t)stream) == hipSuccess ? SYM_OK : SYM_EHIP;
}

int sym_mlp_adam(float *params_dev, const float *grad_dev, float *m_dev, float *v_dev,
                 int64_t count, int32_t step, float lr, void *stream)
{
    if (!params_dev || !grad_dev || !m_dev || !v_dev || count < 1 || step < 1 || !(lr > 0.0f))
        return SYM_EINVAL;
    return sym::launch_mlp_adam(params_dev, grad_dev, m_dev, v_dev, count, step, lr,
                                (hipStream_t)stream) == hipSuccess ? SYM_OK : SYM_EHIP;
}

// ------------------------------------------------------------------ batches

struct sym_batch {
    sym_plan *h = nullptr;
    int32_t m = 0;
    size_t ws_bytes = 0, off_Lx = 0, off_vec = 0, off_vec2 = 0, off_vec3 = 0, off_info = 0,
           off_red = 0, off_sync = 0, off_pcount = 0, off_pbuf = 0, off_dscale = 0, off_pfloor = 0,
           off_tstate = 0, off_ctk = 0;
    sym::DevicePlan D;              // the analysis's plan arrays, the batch's own buffers
    bool bound = false, factored = false;
    uint64_t generation = 0;        // the analysis's generation when the batch was bound
    hipStream_t stream = nullptr;
};

// A batch runs only while the analysis is bound to the same workspace and
// schedule it copied at its own bind (the plan pointers and the split-tile
// buffer sizes come from there).
static bool batch_current(const sym_batch *b)
{
    return b->bound && b->h->bound && b->generation == b->h->generation;
}

int sym_batch_create(sym_handle h, int32_t m, sym_batch_t *out)
{
    if (!h || !out || m < 1 || m > 65535) return SYM_EINVAL;
    *out = nullptr;
    sym_batch *b = new (std::nothrow) sym_batch();
    if (!b) return SYM_ENOMEM;
    b->h = h;
    b->m = m;
    const sym::Plan &P = h->P;
    const size_t M = (size_t)m;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    b->off_Lx = take(M * (size_t)P.panel_entries * elem_size(P));
    b->off_vec = take(M * sizeof(double) * (size_t)P.n);
    b->off_vec2 = take(M * sizeof(double) * (size_t)P.n);
    b->off_vec3 = take(M * sizeof(double) * (size_t)P.n);
    b->off_info = take(M * sizeof(int32_t) * 4);
    b->off_red = take(M * sizeof(double) * 4);
    b->off_sync = take(M * sizeof(int32_t) * (2 * (size_t)P.nb + 16));
    b->off_pcount = take(M * sizeof(int32_t) * (size_t)P.nsplit);
    b->off_pbuf = take(M * (size_t)P.npartial * 4096 * elem_size(P));
    const bool sc = sym::prec_scaled(P.precision);
    b->off_dscale = take(sc ? M * sizeof(double) * (size_t)P.n : 0);
    b->off_pfloor = take(sc ? M * sizeof(double) * (size_t)P.n : 0);
    b->off_tstate = take(M * sizeof(int32_t) * P.tinit.size());
    b->off_ctk = take(M * sizeof(int32_t) * (size_t)P.nchain);
    b->ws_bytes = std::max<size_t>(o, 256);
    *out = b;
    return SYM_OK;
}

int sym_batch_workspace(sym_batch_t b, size_t *bytes)
{
    if (!b || !bytes) return SYM_EINVAL;
    *bytes = b->ws_bytes;
    return SYM_OK;
}

int sym_batch_bind(sym_batch_t b, void *dev_ws, size_t bytes, void *stream)
{
    if (!b || !dev_ws) return SYM_EINVAL;
    if (!b->h->bound) return SYM_ESTATE;
    if (bytes < b->ws_bytes || ((uintptr_t)dev_ws & 255)) return SYM_EWORKSPACE;
    const sym::Plan &P = b->h->P;
    char *base = (char *)dev_ws;
    sym::DevicePlan D = b->h->D;
    D.m = b->m;
    D.Lx = base + b->off_Lx;
    D.vec = (double *)(base + b->off_vec);
    D.vec2 = (double *)(base + b->off_vec2);
    D.vec3 = (double *)(base + b->off_vec3);
    D.info = (int32_t *)(base + b->off_info);
    D.red = (double *)(base + b->off_red);
    D.pend = (int32_t *)(base + b->off_sync);
    D.done = D.pend + (size_t)b->m * P.nb;
    D.ticket = D.done + (size_t)b->m * P.nb;
    D.pcount = (int32_t *)(base + b->off_pcount);
    D.pbuf = base + b->off_pbuf;
    if (sym::prec_scaled(P.precision)) {
        D.dscale = (double *)(base + b->off_dscale);
        D.pfloor = (double *)(base + b->off_pfloor);
    }
    D.tstate = (int32_t *)(base + b->off_tstate);
    D.cticket = (int32_t *)(base + b->off_ctk);
    // single-instance scratch of the analysis is not used by batches
    D.vec4 = D.vec5 = D.vec6 = D.part = nullptr;
    D.ttime = nullptr;
    b->D = D;
    if (P.nsplit > 0 &&
        hipMemsetAsync(D.pcount, 0, sizeof(int32_t) * (size_t)P.nsplit * (size_t)b->m,
                       (hipStream_t)stream) != hipSuccess)
        return SYM_EHIP;
    b->stream = (hipStream_t)stream;
    b->bound = true;
    b->factored = false;
    b->generation = b->h->generation;
    return SYM_OK;
}

int sym_batch_factor(sym_batch_t b, const double *Ax_dev, void *stream)
{
    if (!b || (!Ax_dev && b->h->P.nnzA)) return SYM_EINVAL;
    if (!batch_current(b)) return SYM_ESTATE;
    hipStream_t s = (hipStream_t)stream;
    b->stream = s;
    if (sym::launch_factor(b->h->P, b->D, Ax_dev, s, nullptr) != hipSuccess) return SYM_EHIP;
    b->factored = true;
    return SYM_OK;
}

int sym_batch_solve(sym_batch_t b, double *bx_dev, void *stream)
{
    if (!b || (!bx_dev && b->h->P.n)) return SYM_EINVAL;
    if (!batch_current(b) || !b->factored) return SYM_ESTATE;
    hipStream_t s = (hipStream_t)stream;
    b->stream = s;
    const sym::Plan &P = b->h->P;
    const sym::DevicePlan &D = b->D;
    if (P.n == 0) return SYM_OK;
    if (sym::launch_perm_gather(P, D, bx_dev, D.vec, s) != hipSuccess) return SYM_EHIP;
    if (sym::launch_fwd(P, D, D.vec, D.vec2, s) != hipSuccess) return SYM_EHIP;
    if (sym::launch_bwd(P, D, D.vec2, s) != hipSuccess) return SYM_EHIP;
    if (sym::launch_perm_scatter(P, D, D.vec2, bx_dev, s) != hipSuccess) return SYM_EHIP;
    return SYM_OK;
}

int sym_batch_refine(sym_batch_t b, const double *Ax_dev, const double *b_dev, double *x_dev,
                     int32_t steps, void *stream)
{
    if (!b || ((!Ax_dev || !b_dev || !x_dev) && b->h->P.n) || steps < 0) return SYM_EINVAL;
    if (!batch_current(b) || !b->factored) return SYM_ESTATE;
    hipStream_t s = (hipStream_t)stream;
    const sym::Plan &P = b->h->P;
    const sym::DevicePlan &D = b->D;
    if (P.n == 0) return SYM_OK;
    const size_t bytes = sizeof(double) * (size_t)P.n * (size_t)b->m;
    if (hipMemcpyAsync(x_dev, b_dev, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) return SYM_EHIP;
    int rc = sym_batch_solve(b, x_dev, stream);
    if (rc != SYM_OK) return rc;
    for (int32_t k = 0; k < steps; ++k) {
        if (sym::launch_residual(P, D, Ax_dev, b_dev, x_dev, D.vec3, false, s) != hipSuccess) return SYM_EHIP;
        rc = sym_batch_solve(b, D.vec3, stream);
        if (rc != SYM_OK) return rc;
        if (sym::launch_axpy(P, D, x_dev, D.vec3, s) != hipSuccess) return SYM_EHIP;
    }
    return SYM_OK;
}

int sym_batch_eta(sym_batch_t b, const double *Ax_dev, const double *b_dev, const double *x_dev,
                  double *eta_host, void *stream)
{
    if (!b || !eta_host || ((!Ax_dev || !b_dev || !x_dev) && b->h->P.n)) return SYM_EINVAL;
    if (!batch_current(b)) return SYM_ESTATE;
    hipStream_t s = (hipStream_t)stream;
    const sym::Plan &P = b->h->P;
    const sym::DevicePlan &D = b->D;
    if (P.n == 0) {
        for (int32_t i = 0; i < b->m; ++i) eta_host[i] = 0.0;
        return SYM_OK;
    }
    if (sym::launch_residual(P, D, Ax_dev, b_dev, x_dev, D.vec3, true, s) != hipSuccess) return SYM_EHIP;
    std::vector<double> red((size_t)b->m * 4);
    if (hipMemcpyAsync(red.data(), D.red, sizeof(double) * red.size(), hipMemcpyDeviceToHost, s) != hipSuccess)
        return SYM_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return SYM_EHIP;
    for (int32_t i = 0; i < b->m; ++i) {
        const double *c = red.data() + 4 * (size_t)i;
        const double den = c[1] * c[2] + c[3];
        eta_host[i] = den > 0.0 ? c[0] / den : c[0];
    }
    return SYM_OK;
}

int sym_batch_status(sym_batch_t b, int64_t *info_host)
{
    if (!b || !info_host) return SYM_EINVAL;
    if (!batch_current(b) || !b->factored) return SYM_ESTATE;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return SYM_EHIP;
    std::vector<int32_t> w((size_t)b->m * 4);
    if (hipMemcpy(w.data(), b->D.info, sizeof(int32_t) * w.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return SYM_EHIP;
    int rc = SYM_OK;
    for (int32_t i = 0; i < b->m; ++i) {
        const int32_t *c = w.data() + 4 * (size_t)i;
        if (c[1] != INT32_MAX || c[2] != 0) rc = SYM_ESCHED;
        info_host[i] = c[0] == INT32_MAX ? 0 : 1 + (int64_t)b->h->P.perm[c[0]];
    }
    return rc;
}

void sym_batch_destroy(sym_batch_t b) { delete b; }

}  // extern "C"
