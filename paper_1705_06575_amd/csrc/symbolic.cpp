// symbolic.cpp -- host symbolic analysis (the paper's symbolic inspector,
// Section 3.2): ordering, elimination tree, column counts, fundamental
// supernodes and their row patterns (Eq. (1) applied per supernode), device
// column blocks, level sets, descendant lists (the prune set of the update
// phase) and the map from A's entries into L's panels.
#include <algorithm>
#include <cmath>
#include <chrono>
#include <climits>
#include <cstring>
#include <numeric>
#include <stdexcept>

#include "plan.hpp"
#include "sym.h"

namespace sym {

namespace {

// Lower-triangular CSC of C = P A P^T plus, per entry, its index in A.
struct PermutedLower {
    std::vector<int64_t> cp;   // n+1
    std::vector<int32_t> ci;   // rows (>= column), sorted
    std::vector<int64_t> src;  // index of the entry in A's arrays
};

void permute_lower(int32_t n, const int64_t *Ap, const int32_t *Ai,
                   const std::vector<int32_t> &pinv, PermutedLower &C)
{
    int64_t nnz = Ap[n];
    C.cp.assign((size_t)n + 1, 0);
    for (int32_t j = 0; j < n; ++j)
        for (int64_t p = Ap[j]; p < Ap[j + 1]; ++p) {
            int32_t a = pinv[Ai[p]], b = pinv[j];
            C.cp[(size_t)std::min(a, b) + 1]++;
        }
    for (int32_t j = 0; j < n; ++j) C.cp[j + 1] += C.cp[j];
    C.ci.resize((size_t)nnz);
    C.src.resize((size_t)nnz);
    std::vector<int64_t> fill(C.cp.begin(), C.cp.end() - 1);
    for (int32_t j = 0; j < n; ++j)
        for (int64_t p = Ap[j]; p < Ap[j + 1]; ++p) {
            int32_t a = pinv[Ai[p]], b = pinv[j];
            int32_t col = std::min(a, b), row = std::max(a, b);
            int64_t q = fill[col]++;
            C.ci[q] = row;
            C.src[q] = p;
        }
    // sort rows within each column (carrying the source index)
    std::vector<std::pair<int32_t, int64_t>> tmp;
    for (int32_t j = 0; j < n; ++j) {
        int64_t b = C.cp[j], e = C.cp[j + 1];
        bool sorted = true;
        for (int64_t q = b + 1; q < e; ++q)
            if (C.ci[q] < C.ci[q - 1]) { sorted = false; break; }
        if (sorted) continue;
        tmp.clear();
        for (int64_t q = b; q < e; ++q) tmp.emplace_back(C.ci[q], C.src[q]);
        std::sort(tmp.begin(), tmp.end());
        for (int64_t q = b; q < e; ++q) { C.ci[q] = tmp[q - b].first; C.src[q] = tmp[q - b].second; }
    }
}

}  // namespace

// The factor schedule of a plan (tasks, launches, incidences and
// per-wavefront items) for its current per-supernode kernel variants;
// rerun whenever the variants change.
void build_schedule(Plan &P)
{
    const int32_t B = P.B;
    // blocks whose inverse one wavefront forms, then the wider ones
    P.inv_blocks.clear();
    for (int32_t b = 0; b < P.nb; ++b)
        if (P.blk[b].w <= 16) P.inv_blocks.push_back(b);
    P.inv_nsmall = (int32_t)P.inv_blocks.size();
    for (int32_t b = 0; b < P.nb; ++b)
        if (P.blk[b].w > 16) P.inv_blocks.push_back(b);
    P.parts.clear();
    P.nsplit = 0;
    P.npartial = 0;
    P.ext_operand_entries = 0.0;
    if ((int32_t)P.svariant.size() != P.nds) P.svariant.assign((size_t)P.nds, 1);
    P.sfeat.assign((size_t)P.nds * kSuperFeatures, 0.0);
    P.sbptr.assign((size_t)P.nds + 1, 0);
    for (int32_t s2 = 0; s2 < P.nds; ++s2) {
        int32_t w = P.dsptr[s2 + 1] - P.dsptr[s2];
        P.sbptr[s2 + 1] = P.sbptr[s2] + (w + B - 1) / B;
    }
    P.slevel.assign((size_t)P.nds, 0);
    for (int32_t s2 = 0; s2 < P.nds; ++s2)
        if (P.dsparent[s2] >= 0)
            P.slevel[P.dsparent[s2]] = std::max(P.slevel[P.dsparent[s2]], P.slevel[s2] + 1);
    P.nslevels = 0;
    for (int32_t s2 = 0; s2 < P.nds; ++s2) P.nslevels = std::max(P.nslevels, P.slevel[s2] + 1);
    std::vector<int32_t> sl_ptr((size_t)P.nslevels + 1, 0), sl_list((size_t)P.nds);
    for (int32_t s2 = 0; s2 < P.nds; ++s2) sl_ptr[P.slevel[s2] + 1]++;
    for (int32_t l = 0; l < P.nslevels; ++l) sl_ptr[l + 1] += sl_ptr[l];
    {
        std::vector<int32_t> fill(sl_ptr.begin(), sl_ptr.end() - 1);
        for (int32_t s2 = 0; s2 < P.nds; ++s2) sl_list[fill[P.slevel[s2]]++] = s2;
    }
    auto ntiles = [&](int32_t J) { return (P.blk[J].r + kTileRows - 1) / kTileRows; };
    P.ftasks.clear();
    P.phases.clear();
    P.incs.clear();
    P.iptr.assign(1, 0);
    std::vector<int32_t> blk2ds((size_t)P.nb);
    for (int32_t r = 0; r < P.nds; ++r)
        for (int32_t b = P.sbptr[r]; b < P.sbptr[r + 1]; ++b) blk2ds[b] = r;
    // K is a block; a descendant supernode's blocks share their rows below
    // its columns, so all of its blocks' contributions to a tile form one
    // product whose inner dimension is the supernode's width (wk)
    struct RawInc { int32_t K, a0, a1, b0, b1, wk; };
    std::vector<std::vector<RawInc>> per_tile;
    P.imap.clear();
    P.ibig.clear();
    P.wptr.assign(1, 0);
    P.witems.clear();
    P.wmap.clear();
    P.cptr.assign(1, 0);
    P.chunks.clear();
    // tasks without wavefront items or chunks push their (empty) ranges here
    auto push_task = [&](int32_t J, int32_t t, int32_t K, int32_t flags, int64_t big_end) {
        P.ftasks.push_back(Task{J, t, K, flags});
        P.iptr.push_back((int64_t)P.incs.size());
        P.ibig.push_back(big_end);
        P.cptr.push_back((int64_t)P.chunks.size());
        while ((int64_t)P.wptr.size() < 16 * (int64_t)P.ftasks.size() + 1)
            P.wptr.push_back((int64_t)P.witems.size());
    };
    // tile rows of K's rows [b0, b1) and tile columns of K's rows [a0, a1)
    std::vector<uint8_t> rrel, crel;
    auto relative = [&](int32_t J, int32_t t, const RawInc &ri) {
        const BlockDesc &dJ = P.blk[J];
        const BlockDesc &dK = P.blk[ri.K];
        const int32_t *rJ = P.dsrows.data() + dJ.rowoff;
        const int32_t *rK = P.dsrows.data() + dK.rowoff;
        const int32_t r0 = t * kTileRows;
        const int32_t nr = std::min(kTileRows, dJ.r - r0);
        rrel.clear();
        crel.clear();
        int32_t p = r0;
        for (int32_t q = ri.b0; q < ri.b1; ++q) {
            while (p < r0 + nr && rJ[p] < rK[q]) ++p;
            rrel.push_back((uint8_t)(p - r0));
        }
        for (int32_t q = ri.a0; q < ri.a1; ++q) crel.push_back((uint8_t)(rK[q] - dJ.col0));
    };
    // the wavefront items of one task's small incidences, wavefront-major
    // Each wavefront's items are grouped by their 16-row blocks (4, 3, 2,
    // then 1), so the kernel runs each group
    // with loads and products for exactly that many row blocks; wptr holds
    // 16 boundaries per task (wavefront v, group g: entry 4 v + g).
    // Within a group, items that meet more wavefronts come first (then by
    // the set of wavefronts they meet, then list order): the four
    // wavefronts start on the same products and meet their shared ones in
    // the same order, so a product's rows, read once per wavefront, are
    // read at nearly the same time and the later reads hit the cache.
    std::vector<WaveItem> wgroup[4];
    std::vector<std::pair<int32_t, int32_t>> worder;
    auto emit_wave_items = [&](int32_t J, int32_t t, const std::vector<const RawInc *> &small) {
        worder.clear();
        for (int32_t i = 0; i < (int32_t)small.size(); ++i) {
            relative(J, t, *small[i]);
            int32_t mask = 0;
            for (uint8_t c : crel) mask |= 1 << (c / 16);
            const int32_t met = __builtin_popcount(mask);
            worder.emplace_back(((4 - met) << 4) | mask, i);
        }
        std::stable_sort(worder.begin(), worder.end(),
                         [](const auto &x, const auto &y) { return x.first < y.first; });
        for (int32_t v = 0; v < 4; ++v) {
            for (auto &g : wgroup) g.clear();
            for (const auto &wo : worder) {
                const RawInc *ri = small[wo.second];
                relative(J, t, *ri);
                // columns are increasing: the wavefront's are a contiguous run
                int32_t jlo = 0, jhi = 0;
                while (jlo < (int32_t)crel.size() && crel[jlo] < 16 * v) ++jlo;
                jhi = jlo;
                while (jhi < (int32_t)crel.size() && crel[jhi] < 16 * v + 16) ++jhi;
                if (jlo == jhi) continue;
                WaveItem it{};
                it.valoff = P.blk[ri->K].valoff;
                it.mapoff = (int64_t)P.wmap.size();
                it.ld = P.blk[ri->K].ld;
                it.b0 = ri->b0;
                it.a0 = ri->a0 + jlo;
                it.wk = (int16_t)ri->wk;
                it.nI = (uint8_t)rrel.size();
                it.nJ = (uint8_t)(jhi - jlo);
                P.wmap.insert(P.wmap.end(), rrel.begin(), rrel.end());
                P.wmap.insert(P.wmap.end(), crel.begin() + jlo, crel.begin() + jhi);
                wgroup[4 - (it.nI + 15) / 16].push_back(it);
                P.ext_operand_entries += (double)(it.nI + it.nJ) * (double)ri->wk;
            }
            for (const auto &g : wgroup) {
                P.witems.insert(P.witems.end(), g.begin(), g.end());
                P.wptr.push_back((int64_t)P.witems.size());
            }
        }
    };
    // the staged chunks of one tile's incidences (all of them, list order)
    auto emit_chunks = [&](int32_t J, int32_t t, const std::vector<RawInc> &incs_t) {
        for (const RawInc &ri : incs_t) {
            relative(J, t, ri);
            if (P.imap.size() + rrel.size() + crel.size() > (size_t)UINT32_MAX)
                throw std::length_error("relative-index map beyond 4 GiB");
            StageChunk c{};
            c.valoff = P.blk[ri.K].valoff;
            c.ld = P.blk[ri.K].ld;
            c.b0 = ri.b0;
            c.a0 = ri.a0;
            c.map = (uint32_t)P.imap.size();
            c.nI = (uint8_t)rrel.size();
            c.nJ = (uint8_t)crel.size();
            for (int v = 1; v < 4; ++v) {
                int32_t j = 0;
                while (j < (int32_t)crel.size() && crel[j] < 16 * v) ++j;
                c.jw[v - 1] = (uint8_t)j;
            }
            P.imap.insert(P.imap.end(), rrel.begin(), rrel.end());
            P.imap.insert(P.imap.end(), crel.begin(), crel.end());
            P.ext_operand_entries += (double)(rrel.size() + crel.size()) * (double)ri.wk;
            for (int32_t kc = 0; kc < ri.wk; kc += kStageK) {
                const int32_t nk = std::min(kStageK, ri.wk - kc);
                c.kc = (int16_t)kc;
                c.nk_last = (uint8_t)(nk | (kc + kStageK >= ri.wk ? 0x80 : 0));
                P.chunks.push_back(c);
            }
        }
    };
    auto open_phase = [&](int32_t kind) { P.phases.push_back(Phase{kind, (int64_t)P.ftasks.size(), 0}); };
    auto close_phase = [&]() {
        P.phases.back().t1 = (int64_t)P.ftasks.size();
        if (P.phases.back().t1 == P.phases.back().t0) {
            if (P.phases.back().s0 >= 0) P.xslot.resize((size_t)P.phases.back().s0);
            P.phases.pop_back();
        }
    };
    // record one incidence of tile t of block J, with its relative indices
    auto emit_inc = [&](int32_t J, int32_t t, const RawInc &ri) {
        const BlockDesc &dJ = P.blk[J];
        const BlockDesc &dK = P.blk[ri.K];
        const int32_t *rJ = P.dsrows.data() + dJ.rowoff;
        const int32_t *rK = P.dsrows.data() + dK.rowoff;
        const int32_t r0 = t * kTileRows;
        const int32_t nr = std::min(kTileRows, dJ.r - r0);
        Incidence in{};
        in.valoff = dK.valoff;
        in.mapoff = (int64_t)P.imap.size();
        in.ld = dK.ld;
        in.wk = (int16_t)ri.wk;
        in.b0 = ri.b0;
        in.a0 = ri.a0;
        in.nI = (uint8_t)(ri.b1 - ri.b0);
        in.nJ = (uint8_t)(ri.a1 - ri.a0);
        // tile rows of K's rows [b0, b1): a merge along J's sorted rows
        int32_t p = r0;
        for (int32_t q = ri.b0; q < ri.b1; ++q) {
            while (p < r0 + nr && rJ[p] < rK[q]) ++p;
            P.imap.push_back((uint8_t)(p - r0));
        }
        for (int32_t q = ri.a0; q < ri.a1; ++q) P.imap.push_back((uint8_t)(rK[q] - dJ.col0));
        in.cmin = (uint8_t)(rK[ri.a0] - dJ.col0);
        in.cmax = (uint8_t)(rK[ri.a1 - 1] - dJ.col0);
        P.incs.push_back(in);
        P.ext_operand_entries += (double)(in.nI + in.nJ) * (double)ri.wk;
    };
    // tiles of the chain launches and their initial states
    P.tbase.assign((size_t)P.nb + 1, 0);
    for (int32_t J = 0; J < P.nb; ++J) P.tbase[J + 1] = P.tbase[J] + ntiles(J);
    P.tinit.assign((size_t)P.tbase[P.nb], 0);
    for (int32_t r = 0; r < P.nds; ++r) {
        const int32_t b0 = P.sbptr[r];
        for (int32_t J = b0; J < P.sbptr[r + 1]; ++J)
            for (int32_t q = P.tbase[J]; q < P.tbase[J + 1]; ++q) P.tinit[q] = b0;
        P.tinit[P.tbase[b0]] = b0 + 1;
    }
    P.nchain = 0;
    // One chain launch for level l: the off-diagonal tiles of each
    // supernode's first block solve against its diagonal block (factored by
    // the external launch), and for k = 1, 2, ... every tile of blocks
    // b0 + k, b0 + k + 1, ... subtracts block b0 + k - 1's product, block
    // b0 + k's tile 0 is then factored and its other tiles solved.  A task
    // needs its tile's previous update and the final tiles of the source
    // block it reads (those holding the target block's columns and the
    // tile's rows); a solve also needs the factored diagonal tile.  Tasks
    // are ordered by their earliest start when every task has a workgroup
    // (unit time per update, a factorization 3 more, a solve 1 more): the
    // critical chain of factorizations leads, and every task comes after
    // those it waits for, so a persistent launch that hands out tasks in
    // this order never waits for a task no workgroup holds.
    std::vector<double> tcur, tfin;
    std::vector<int32_t> chain_check;
    auto emit_chain = [&](int32_t l) {
        struct CT {
            Task tk;
            double start;
        };
        std::vector<CT> ct;
        tcur.assign((size_t)P.tbase[P.nb], 0.0);
        tfin.assign((size_t)P.tbase[P.nb], 0.0);
        constexpr double dU = 1.0, dF = 3.0, dT = 1.0;
        for (int32_t q = sl_ptr[l]; q < sl_ptr[l + 1]; ++q) {
            const int32_t s2 = sl_list[q];
            const int32_t b0 = P.sbptr[s2], nbs = P.sbptr[s2 + 1] - b0;
            for (int32_t t = 1; t < ntiles(b0); ++t) {
                ct.push_back(CT{Task{b0, t, -1, kChainSolve}, 0.0});
                tfin[P.tbase[b0] + t] = dT;
            }
            for (int32_t k = 1; k < nbs; ++k) {
                const int32_t K = b0 + k - 1;
                const BlockDesc &dK = P.blk[K];
                for (int32_t c = k; c < nbs; ++c) {
                    const int32_t J = b0 + c;
                    const BlockDesc &dJ = P.blk[J];
                    const int32_t d = dJ.col0 - dK.col0;
                    for (int32_t t = 0; t < ntiles(J); ++t) {
                        const int32_t r0 = t * kTileRows, nr = std::min(kTileRows, dJ.r - r0);
                        const int32_t tile = P.tbase[J] + t;
                        double st = tcur[tile];
                        for (int32_t x = d / kTileRows; x <= (d + dJ.w - 1) / kTileRows; ++x)
                            st = std::max(st, tfin[P.tbase[K] + x]);
                        for (int32_t x = (d + r0) / kTileRows; x <= (d + r0 + nr - 1) / kTileRows; ++x)
                            st = std::max(st, tfin[P.tbase[K] + x]);
                        int32_t flags = 0;
                        double dur = dU;
                        if (c == k && t == 0) {
                            flags = kFuseFactor;
                            dur += dF;
                        } else if (c == k) {
                            st = std::max(st, tfin[P.tbase[J]] - dU);   // the solve waits, not the update
                            flags = kChainSolve;
                            dur += dT;
                        }
                        ct.push_back(CT{Task{J, t, K, flags}, st});
                        tcur[tile] = st + dur;
                        if (c == k) tfin[tile] = std::max(st + dur, tfin[P.tbase[J]] + dT);
                    }
                }
            }
        }
        if (ct.empty()) return;
        std::stable_sort(ct.begin(), ct.end(), [](const CT &a, const CT &b) { return a.start < b.start; });
        // the launch's tasks run one after another in this order without a
        // wait that is not already met (so the persistent launch cannot
        // wait for a task that no workgroup holds)
        std::vector<int32_t> &st = chain_check;
        st = P.tinit;
        for (const CT &c : ct) {
            const Task &tk = c.tk;
            const BlockDesc &dJ = P.blk[tk.J];
            const int32_t tile = P.tbase[tk.J] + tk.t;
            bool ok = true;
            if (tk.K >= 0) {
                const int32_t d = dJ.col0 - P.blk[tk.K].col0, r0 = tk.t * kTileRows;
                const int32_t nr = std::min(kTileRows, dJ.r - r0);
                ok = st[tile] == tk.K;
                for (int32_t x = d / kTileRows; x <= (d + dJ.w - 1) / kTileRows; ++x)
                    ok = ok && st[P.tbase[tk.K] + x] >= tk.K + 1;
                for (int32_t x = (d + r0) / kTileRows; x <= (d + r0 + nr - 1) / kTileRows; ++x)
                    ok = ok && st[P.tbase[tk.K] + x] >= tk.K + 1;
            }
            if (tk.flags & kChainSolve) ok = ok && st[P.tbase[tk.J]] >= tk.J + 1;
            if (!ok) throw std::logic_error("chain launch order");
            st[tile] = (tk.flags & (kFuseFactor | kChainSolve)) ? tk.J + 1 : tk.K + 1;
        }
        open_phase(kPhaseChain);
        for (const CT &c : ct) push_task(c.tk.J, c.tk.t, c.tk.K, c.tk.flags, 0);
        close_phase();
        P.nchain++;
    };
    std::vector<const RawInc *> small;
    struct Pending {
        int32_t J, t, s2;
        bool fuse;
        double cost;
        std::vector<RawInc> incs;
    };
    std::vector<Pending> pending;
    std::vector<int32_t> leaves;
    P.xslot.clear();
    for (int32_t l = 0; l < P.nslevels; ++l) {
        int32_t maxnb = 0;
        pending.clear();
        leaves.clear();
        open_phase(kPhaseExternal);
        for (int32_t q = sl_ptr[l]; q < sl_ptr[l + 1]; ++q) {
            const int32_t s2 = sl_list[q];
            maxnb = std::max(maxnb, P.sbptr[s2 + 1] - P.sbptr[s2]);
            for (int32_t J = P.sbptr[s2]; J < P.sbptr[s2 + 1]; ++J) {
                const BlockDesc &dJ = P.blk[J];
                const int32_t *rJ = P.dsrows.data() + dJ.rowoff;
                const int32_t nt = ntiles(J);
                if ((int32_t)per_tile.size() < nt) per_tile.resize((size_t)nt);
                for (int32_t t = 0; t < nt; ++t) per_tile[t].clear();
                for (int64_t p = P.dptr[J]; p < P.dptr[J + 1]; ++p) {
                    const Pair &pr = P.pairs[p];
                    if (pr.K >= P.sbptr[s2]) break;     // internal pairs come last
                    const int32_t ks = blk2ds[pr.K];
                    if (pr.K != P.sbptr[ks]) continue;   // folded into the supernode's first block
                    const int32_t kw = P.dsptr[ks + 1] - P.dsptr[ks];
                    const BlockDesc &dK = P.blk[pr.K];
                    const int32_t *rK = P.dsrows.data() + dK.rowoff;
                    int32_t pos = pr.a0;
                    while (pos < dK.r) {
                        const int32_t li = (int32_t)(std::lower_bound(rJ, rJ + dJ.r, rK[pos]) - rJ);
                        const int32_t t = li / kTileRows;
                        const int32_t last = rJ[std::min((t + 1) * kTileRows, dJ.r) - 1];
                        const int32_t end = (int32_t)(std::upper_bound(rK + pos, rK + dK.r, last) - rK);
                        per_tile[t].push_back(RawInc{pr.K, pr.a0, pr.a1, pos, end, kw});
                        pos = end;
                    }
                }
                const bool first = J == P.sbptr[s2];
                if (first && nt == 1 && dJ.w <= 16 && per_tile[0].empty()) {
                    // a leaf of one narrow tile: factored by the level's
                    // one-wavefront launch, not as an update tile
                    leaves.push_back(J);
                    P.sfeat[(size_t)s2 * kSuperFeatures + 2] += 1.0;
                    continue;
                }
                for (int32_t t = 0; t < nt; ++t) {
                    const bool fuse = first && t == 0;
                    if (per_tile[t].empty() && !fuse) continue;
                    // an estimate of the tile's work: 16-wide k-batches of its
                    // products, plus the fused factorization
                    double cost = fuse ? 8.0 : 0.0;
                    for (const RawInc &ri : per_tile[t]) cost += (ri.wk + 15) / 16;
                    pending.push_back(Pending{J, t, s2, fuse, cost, per_tile[t]});
                }
            }
        }
        // longest tiles first, so that no long tile starts in the launch's
        // last wave of workgroups (ties keep the block order)
        std::stable_sort(pending.begin(), pending.end(),
                         [](const Pending &a, const Pending &b) { return a.cost > b.cost; });
        // a long tile becomes parts of about one split unit each, contiguous
        // in its incidence list; counters and partial-sum slots are per
        // launch, so every level reuses them from the start
        int32_t lv_counters = 0;
        int64_t lv_slots = 0;
        double lv_cost = 0.0;
        for (const Pending &pd : pending) lv_cost += pd.cost;
        const double unit = std::max(kSplitUnits, lv_cost / P.split_share);
        // tiles of blocks of at most 16 columns that are neither split nor
        // staged go to the level's one-wavefront launch (their products are
        // all per-wavefront items of the first wavefront)
        auto cut_of = [&](const Pending &pd) {
            int32_t np = 1;
            if (pd.cost > unit)
                np = std::min<int32_t>((int32_t)std::ceil(pd.cost / unit), (int32_t)pd.incs.size());
            std::vector<size_t> cut(1, 0);
            if (np > 1) {
                double acc = 0.0;
                const double share = pd.cost / np;
                for (size_t i = 0; i < pd.incs.size() && (int32_t)cut.size() < np; ++i) {
                    acc += (pd.incs[i].wk + 15) / 16;
                    if (acc >= share * (double)cut.size() && i + 1 < pd.incs.size()) cut.push_back(i + 1);
                }
            }
            cut.push_back(pd.incs.size());
            return cut;
        };
        auto emit_pending = [&](const Pending &pd, const std::vector<size_t> &cut) {
            const int32_t np = (int32_t)cut.size() - 1;
            const int32_t counter = np > 1 ? lv_counters++ : -1;
            const int64_t slot0 = lv_slots;
            if (np > 1) lv_slots += np;
            P.nsplit = std::max(P.nsplit, lv_counters);
            P.npartial = std::max(P.npartial, lv_slots);
            for (int32_t part = 0; part < np; ++part) {
                    const int32_t J = pd.J, t = pd.t, s2 = pd.s2;
                    const bool fuse = pd.fuse;
                    const std::vector<RawInc> incs_t(pd.incs.begin() + (ptrdiff_t)cut[part],
                                                     pd.incs.begin() + (ptrdiff_t)cut[part + 1]);
                    // large incidences first, then the rest (each keeps list order)
                    const int32_t lim = kVariantLarge[P.svariant[s2]];
                    auto large = [lim](const RawInc &ri) {
                        return ri.b1 - ri.b0 >= lim && ri.a1 - ri.a0 >= lim && ri.wk >= lim;
                    };
                    double *ft = P.sfeat.data() + (size_t)s2 * kSuperFeatures;
                    if (part == 0) ft[2] += 1.0;
                    for (const RawInc &ri : incs_t) {
                        const double fl = 2.0 * (ri.b1 - ri.b0) * (ri.a1 - ri.a0) * (double)ri.wk;
                        const int32_t mn = std::min(std::min(ri.b1 - ri.b0, ri.a1 - ri.a0), ri.wk);
                        ft[3] += 1.0;
                        ft[4] += fl;
                        if (mn >= 64) ft[5] += fl;
                        if (mn >= 32) ft[6] += fl;
                    }
                    const bool staged = P.svariant[s2] == kVariantStaged;
                    small.clear();
                    if (staged) {
                        emit_chunks(J, t, incs_t);
                    } else {
                        for (const RawInc &ri : incs_t) {
                            if (large(ri)) emit_inc(J, t, ri);
                            else small.push_back(&ri);
                        }
                    }
                    const int64_t big_end = (int64_t)P.incs.size();
                    emit_wave_items(J, t, small);
                    const int32_t sflag = staged ? kStaged : 0;
                    if (np > 1) {
                        P.parts.push_back(PartDesc{counter, part, np, (int32_t)slot0});
                        push_task(J, t, (int32_t)P.parts.size() - 1,
                                  (fuse ? kFuseFactor : 0) | kPartial | sflag, big_end);
                    } else {
                        push_task(J, t, -1, (fuse ? kFuseFactor : 0) | sflag, big_end);
                    }
            }
        };
        // Workgroup slots of the launch, longest first: a tile of its own,
        // or up to four tiles of blocks of at most 16 columns that are
        // neither split nor staged, one per wavefront (a narrow tile's
        // products all belong to the first wavefront's columns, so a whole
        // workgroup would idle three of its four); a slot of narrow tiles
        // takes the next ones in the launch's order.
        {
            const size_t np = pending.size();
            std::vector<std::vector<size_t>> cuts(np);
            std::vector<uint8_t> nar(np, 0), done(np, 0);
            for (size_t i = 0; i < np; ++i) {
                cuts[i] = cut_of(pending[i]);
                nar[i] = cuts[i].size() == 2 && P.blk[pending[i].J].w <= 16 &&
                         P.svariant[pending[i].s2] != kVariantStaged;
            }
            const int64_t t0 = P.phases.back().t0;
            P.phases.back().s0 = (int64_t)P.xslot.size();
            size_t pn = 0;
            for (size_t i = 0; i < np; ++i) {
                if (done[i]) continue;
                const int32_t first = (int32_t)((int64_t)P.ftasks.size() - t0);
                if (!nar[i]) {
                    // a slot per part of a split tile
                    emit_pending(pending[i], cuts[i]);
                    for (int32_t k = first; k < (int32_t)((int64_t)P.ftasks.size() - t0); ++k) P.xslot.push_back(k);
                    done[i] = 1;
                    continue;
                }
                P.xslot.push_back(first | kQuadSlot);
                emit_pending(pending[i], cuts[i]);
                done[i] = 1;
                int32_t taken = 1;
                pn = std::max(pn, i + 1);
                for (; pn < np && taken < 4; ++pn) {
                    if (!nar[pn] || done[pn]) continue;
                    emit_pending(pending[pn], cuts[pn]);
                    done[pn] = 1;
                    ++taken;
                }
            }
            P.phases.back().nslots = (int64_t)P.xslot.size() - P.phases.back().s0;
            P.xslot.push_back((int32_t)((int64_t)P.ftasks.size() - t0));
            // the slots cover the launch's tasks in order; a narrow slot
            // holds one to four single-part tiles of at most 16 columns
            const int64_t s0 = P.phases.back().s0, ns = P.phases.back().nslots;
            for (int64_t k = 0; k < ns; ++k) {
                const int32_t a = P.xslot[s0 + k] & INT32_MAX, b = P.xslot[s0 + k + 1] & INT32_MAX;
                const bool quad = P.xslot[s0 + k] < 0;
                if (b <= a || (!quad && b - a != 1) || b - a > 4) throw std::logic_error("launch slots");
                if (quad)
                    for (int32_t q = a; q < b; ++q) {
                        const Task &tk = P.ftasks[t0 + q];
                        if (P.blk[tk.J].w > 16 || (tk.flags & (kPartial | kStaged))) throw std::logic_error("launch slots");
                    }
            }
            if (ns > 0 && (P.xslot[s0] & INT32_MAX) != 0) throw std::logic_error("launch slots");
        }
        close_phase();
        if (!leaves.empty()) {
            open_phase(kPhaseLeaf);
            for (int32_t J : leaves) push_task(J, 0, -1, kFuseFactor, 0);
            close_phase();
        }
        if (P.chain_launch) {
            emit_chain(l);
            continue;
        }
        open_phase(kPhaseTrsm);
        for (int32_t q = sl_ptr[l]; q < sl_ptr[l + 1]; ++q) {
            const int32_t J = P.sbptr[sl_list[q]];
            for (int32_t t = 1; t < ntiles(J); ++t) push_task(J, t, -1, 0, 0);
        }
        close_phase();
        // Right-looking steps in groups of G blocks (local block indices):
        // step k with k % G != 0 updates the blocks of k's group from k on by
        // block k - 1, and the diagonal tile of the next group's first block
        // too; step k with k % G == 0 updates every block from k on by the
        // whole group [k - G, k), one product per tile, except its own
        // diagonal tile, which then lacks only block k - 1 (so the
        // factorization every step waits for multiplies one block, not G).
        // Either way block k has then been updated by every block before it.
        const int32_t G = std::max(1, P.update_depth);
        for (int32_t k = 1; k < maxnb; ++k) {
            open_phase(kPhaseInternal);
            const bool group_end = k % G == 0;
            const int32_t ksrc = group_end ? k - G : k - 1;
            const int32_t dflags = group_end ? (G - 1) << kDepthShift : 0;
            const int32_t gnext = (k / G + 1) * G;     // the next group's first block
            // the tiles fused with a factorization (the longest) lead the launch
            for (int32_t q = sl_ptr[l]; q < sl_ptr[l + 1]; ++q) {
                const int32_t s2 = sl_list[q];
                const int32_t b0 = P.sbptr[s2], nbs = P.sbptr[s2 + 1] - b0;
                if (nbs > k) push_task(b0 + k, 0, b0 + k - 1, kFuseFactor, 0);
            }
            for (int32_t q = sl_ptr[l]; q < sl_ptr[l + 1]; ++q) {
                const int32_t s2 = sl_list[q];
                const int32_t b0 = P.sbptr[s2], nbs = P.sbptr[s2 + 1] - b0;
                if (nbs <= k) continue;
                const int32_t cend = group_end ? nbs : std::min(nbs, gnext);
                for (int32_t c = k; c < cend; ++c)
                    for (int32_t t = (c == k ? 1 : 0); t < ntiles(b0 + c); ++t)
                        push_task(b0 + c, t, b0 + ksrc, dflags, 0);
                if (!group_end && gnext < nbs) push_task(b0 + gnext, 0, b0 + k - 1, 0, 0);
            }
            close_phase();
            open_phase(kPhaseTrsm);
            for (int32_t q = sl_ptr[l]; q < sl_ptr[l + 1]; ++q) {
                const int32_t s2 = sl_list[q];
                const int32_t b0 = P.sbptr[s2], nbs = P.sbptr[s2 + 1] - b0;
                if (nbs <= k) continue;
                for (int32_t t = 1; t < ntiles(b0 + k); ++t) push_task(b0 + k, t, -1, 0, 0);
            }
            close_phase();
        }
    }

    // external phases with large incidences use the cooperative kernel
    P.phase_coop.assign(P.phases.size(), 0);
    for (size_t ph = 0; ph < P.phases.size(); ++ph) {
        if (P.phases[ph].kind != kPhaseExternal) continue;
        for (int64_t q = P.phases[ph].t0; q < P.phases[ph].t1; ++q)
            if (P.ibig[q] > P.iptr[q]) { P.phase_coop[ph] = 1; break; }
    }
    // supernode features and the target supernode of every external task
    for (int32_t s2 = 0; s2 < P.nds; ++s2) {
        double *ft = P.sfeat.data() + (size_t)s2 * kSuperFeatures;
        ft[0] = P.dsptr[s2 + 1] - P.dsptr[s2];
        ft[1] = (double)(P.dsrowptr[s2 + 1] - P.dsrowptr[s2]);
        ft[5] = ft[4] > 0 ? ft[5] / ft[4] : 0.0;
        ft[6] = ft[4] > 0 ? ft[6] / ft[4] : 0.0;
        ft[7] = P.slevel[s2];
    }
    {
        std::vector<double> lflops((size_t)P.nslevels, 0.0), lcount((size_t)P.nslevels, 0.0),
            ltiles((size_t)P.nslevels, 0.0);
        for (int32_t s2 = 0; s2 < P.nds; ++s2) {
            const double *ft = P.sfeat.data() + (size_t)s2 * kSuperFeatures;
            lflops[P.slevel[s2]] += ft[4];
            lcount[P.slevel[s2]] += 1.0;
            ltiles[P.slevel[s2]] += ft[2];
        }
        for (int32_t s2 = 0; s2 < P.nds; ++s2) {
            double *ft = P.sfeat.data() + (size_t)s2 * kSuperFeatures;
            const int32_t l = P.slevel[s2];
            ft[8] = lflops[l];
            ft[9] = lcount[l];
            ft[10] = ltiles[l];
            ft[11] = lflops[l] > 0 ? ft[4] / lflops[l] : 0.0;
        }
    }
    P.task_super.assign(P.ftasks.size(), -1);
    for (const Phase &ph : P.phases)
        if (ph.kind == kPhaseExternal)
            for (int64_t q = ph.t0; q < ph.t1; ++q) P.task_super[q] = blk2ds[P.ftasks[q].J];

}

int analyze(int64_t n64, const int64_t *Ap, const int32_t *Ai, int ordering,
            const int32_t *user_perm, int block_width, int nd_leaf, bool relax, int max_width,
            Plan &P)
{
    auto t_start = std::chrono::steady_clock::now();
    if (n64 < 0 || n64 > INT32_MAX - 1) return SYM_EINVAL;
    if (n64 > 0 && (!Ap || !Ai)) return SYM_EINVAL;
    const int32_t n = (int32_t)n64;
    if (block_width < 16 || block_width > 64 || block_width % 16) return SYM_EINVAL;
    if (max_width < 1 || max_width > kMaxDeviceWidth) return SYM_EINVAL;
    P.n = n;
    P.B = block_width;

    // ---------------------------------------------------------- validation
    if (n > 0 && Ap[0] != 0) return SYM_EPATTERN;
    for (int32_t j = 0; j < n; ++j)
        if (Ap[j + 1] < Ap[j]) return SYM_EPATTERN;
    P.nnzA = n > 0 ? Ap[n] : 0;
    {
        std::vector<int32_t> mark((size_t)n, -1);
        for (int32_t j = 0; j < n; ++j)
            for (int64_t p = Ap[j]; p < Ap[j + 1]; ++p) {
                int32_t i = Ai[p];
                if (i < j || i >= n) return SYM_EPATTERN;
                if (mark[i] == j) return SYM_EPATTERN;
                mark[i] = j;
            }
    }

    // ------------------------------------------------------------ ordering
    P.perm.resize((size_t)n);
    if (ordering == SYM_ORDER_USER) {
        if (n > 0 && !user_perm) return SYM_EINVAL;
        std::vector<char> seen((size_t)n, 0);
        for (int32_t k = 0; k < n; ++k) {
            int32_t v = user_perm[k];
            if (v < 0 || v >= n || seen[v]) return SYM_EINVAL;
            seen[v] = 1;
            P.perm[k] = v;
        }
    } else if (ordering == SYM_ORDER_NATURAL) {
        std::iota(P.perm.begin(), P.perm.end(), 0);
    } else if (ordering == SYM_ORDER_ND) {
        std::vector<int64_t> xadj((size_t)n + 1, 0);
        for (int32_t j = 0; j < n; ++j)
            for (int64_t p = Ap[j]; p < Ap[j + 1]; ++p)
                if (Ai[p] != j) { xadj[Ai[p] + 1]++; xadj[j + 1]++; }
        for (int32_t j = 0; j < n; ++j) xadj[j + 1] += xadj[j];
        std::vector<int32_t> adj((size_t)xadj[n]);
        std::vector<int64_t> fill(xadj.begin(), xadj.end() - 1);
        for (int32_t j = 0; j < n; ++j)
            for (int64_t p = Ap[j]; p < Ap[j + 1]; ++p)
                if (Ai[p] != j) { adj[fill[Ai[p]]++] = j; adj[fill[j]++] = Ai[p]; }
        nested_dissection(n, xadj, adj, std::max(nd_leaf, 1), P.perm);
    } else {
        return SYM_EINVAL;
    }
    P.pinv.resize((size_t)n);
    for (int32_t k = 0; k < n; ++k) P.pinv[P.perm[k]] = k;

    PermutedLower C;
    permute_lower(n, Ap, Ai, P.pinv, C);

    // row lists of the strict lower triangle of C: for row i, columns j < i
    std::vector<int64_t> rp((size_t)n + 1, 0);
    for (int32_t j = 0; j < n; ++j)
        for (int64_t p = C.cp[j]; p < C.cp[j + 1]; ++p)
            if (C.ci[p] != j) rp[C.ci[p] + 1]++;
    for (int32_t i = 0; i < n; ++i) rp[i + 1] += rp[i];
    std::vector<int32_t> rj((size_t)rp[n]);
    {
        std::vector<int64_t> fill(rp.begin(), rp.end() - 1);
        for (int32_t j = 0; j < n; ++j)
            for (int64_t p = C.cp[j]; p < C.cp[j + 1]; ++p)
                if (C.ci[p] != j) rj[fill[C.ci[p]]++] = j;
    }

    // ----------------------------------------------- elimination tree (3.2)
    // parent[j] = min{i > j : L_ij != 0}; built row by row with path-compressed
    // virtual ancestors: every entry C_kj (j < k) makes k an ancestor of j.
    P.parent.assign((size_t)n, -1);
    {
        std::vector<int32_t> anc((size_t)n, -1);
        for (int32_t k = 0; k < n; ++k) {
            for (int64_t q = rp[k]; q < rp[k + 1]; ++q) {
                int32_t i = rj[q];
                while (i != -1 && i < k) {
                    int32_t next = anc[i];
                    anc[i] = k;
                    if (next == -1) { P.parent[i] = k; break; }
                    i = next;
                }
            }
        }
    }

    // --------------------------------------- column counts by row subtrees
    // Row k of L is the union of the tree paths from each j with C_kj != 0
    // up to k; each visited column j gains row k.
    P.colcount.assign((size_t)n, 1);
    {
        std::vector<int32_t> mark((size_t)n, -1);
        for (int32_t k = 0; k < n; ++k) {
            mark[k] = k;
            for (int64_t q = rp[k]; q < rp[k + 1]; ++q) {
                int32_t j = rj[q];
                while (mark[j] != k) {
                    mark[j] = k;
                    P.colcount[j]++;
                    j = P.parent[j];
                }
            }
        }
    }
    P.nnzL = 0;
    P.flops = 0.0;
    for (int32_t j = 0; j < n; ++j) {
        P.nnzL += P.colcount[j];
        P.flops += (double)P.colcount[j] * (double)P.colcount[j];
    }

    // ----------------------------------------------- fundamental supernodes
    {
        std::vector<int32_t> nchild((size_t)n, 0);
        for (int32_t j = 0; j < n; ++j)
            if (P.parent[j] >= 0) nchild[P.parent[j]]++;
        P.sptr.clear();
        for (int32_t j = 0; j < n; ++j) {
            bool merge = j > 0 && P.parent[j - 1] == j && nchild[j] == 1 &&
                         P.colcount[j - 1] - 1 == P.colcount[j];
            if (!merge) P.sptr.push_back(j);
        }
        P.sptr.push_back(n);
        P.ns = (int32_t)P.sptr.size() - 1;
    }
    const int32_t ns = P.ns;
    std::vector<int32_t> col2sn((size_t)n);
    for (int32_t s = 0; s < ns; ++s)
        for (int32_t j = P.sptr[s]; j < P.sptr[s + 1]; ++j) col2sn[j] = s;
    P.sparent.assign((size_t)ns, -1);
    for (int32_t s = 0; s < ns; ++s) {
        int32_t last = P.sptr[s + 1] - 1;
        if (P.parent[last] >= 0) P.sparent[s] = col2sn[P.parent[last]];
    }

    // ------------------------- supernodal row patterns: Eq. (1) per supernode
    // R_s = {own columns} u (rows of C in s's columns) u (R_t minus t's own
    // columns, for every child supernode t).
    P.srowptr.assign((size_t)ns + 1, 0);
    for (int32_t s = 0; s < ns; ++s) P.srowptr[s + 1] = P.srowptr[s] + P.colcount[P.sptr[s]];
    P.srows.resize((size_t)P.srowptr[ns]);
    {
        std::vector<int32_t> chead((size_t)ns, -1), cnext((size_t)ns, -1);
        for (int32_t s = ns - 1; s >= 0; --s)
            if (P.sparent[s] >= 0) { cnext[s] = chead[P.sparent[s]]; chead[P.sparent[s]] = s; }
        std::vector<int32_t> mark((size_t)n, -1);
        std::vector<int32_t> buf;
        for (int32_t s = 0; s < ns; ++s) {
            int32_t f = P.sptr[s], l = P.sptr[s + 1] - 1;
            buf.clear();
            for (int32_t j = f; j <= l; ++j) mark[j] = s;
            for (int32_t j = f; j <= l; ++j)
                for (int64_t p = C.cp[j]; p < C.cp[j + 1]; ++p) {
                    int32_t i = C.ci[p];
                    if (mark[i] != s) { mark[i] = s; buf.push_back(i); }
                }
            for (int32_t t = chead[s]; t != -1; t = cnext[t]) {
                int32_t wt = P.sptr[t + 1] - P.sptr[t];
                for (int64_t p = P.srowptr[t] + wt; p < P.srowptr[t + 1]; ++p) {
                    int32_t i = P.srows[p];
                    if (i > l && mark[i] != s) { mark[i] = s; buf.push_back(i); }
                }
            }
            std::sort(buf.begin(), buf.end());
            int64_t need = P.srowptr[s + 1] - P.srowptr[s];
            if ((int64_t)buf.size() + (l - f + 1) != need) return SYM_EPATTERN;  // internal inconsistency
            int64_t o = P.srowptr[s];
            for (int32_t j = f; j <= l; ++j) P.srows[o++] = j;
            for (int32_t i : buf) P.srows[o++] = i;
        }
    }
    // ------------------------------------------- relaxed device supernodes
    // Adjacent child supernodes are merged into their parent when the
    // explicit zeros this adds stay within the limits below (widths 4 / 16 /
    // 48 with zero fractions 0.8 / 0.1 / 0.05 of the stored lower
    // trapezoid).  The merged panel's row list is its columns followed by
    // the parent's rows below them; every child row is in it (Eq. (1): a
    // child's pattern below its columns lies in its parent's column pattern).
    // The fundamental supernodes above stay the reported partition; only the
    // device blocking uses the relaxed ones.  Stored zeros remain exactly
    // zero through the factorization and the solves.
    {
        std::vector<int32_t> top;      // fundamental supernode on top of each relaxed one
        std::vector<int32_t> first;    // first column
        std::vector<double> ztrue;     // true entries of its columns
        for (int32_t s = 0; s < ns; ++s) {
            const int32_t f = P.sptr[s], wS = P.sptr[s + 1] - f;
            const double rS = (double)(P.srowptr[s + 1] - P.srowptr[s]);
            double zS = 0;
            for (int32_t j = f; j < f + wS; ++j) zS += (double)P.colcount[j];
            bool merged = false;
            if (relax && !top.empty() && P.sparent[top.back()] == s && P.sptr[top.back() + 1] == f) {
                const double Wn = (double)(f + wS - first.back());
                const double E = rS - wS;                      // rows below the merged columns
                const double stored = Wn * (Wn + 1) / 2 + Wn * E;
                const double zeros = stored - (ztrue.back() + zS);
                const double frac = stored > 0 ? zeros / stored : 0.0;
                if (Wn <= 4 || (Wn <= 16 && frac < 0.8) || (Wn <= 48 && frac < 0.1) || frac < 0.05) {
                    top.back() = s;
                    ztrue.back() += zS;
                    merged = true;
                }
            }
            if (!merged) {
                top.push_back(s);
                first.push_back(f);
                ztrue.push_back(zS);
            }
        }
        // A device supernode wider than the kernels' limits is cut into
        // pieces of consecutive columns (a piece's rows: its own columns,
        // the later columns of the supernode, then the rows below): the
        // update products' inner dimension is a supernode's width, held in
        // 16 bits, and their byte offsets within a panel in 32 bits, so a
        // piece has at most max_width columns and w * r * 8 < 2^32.  Each
        // piece is the only child of the next; nothing else changes.
        std::vector<int32_t> dtop, dend;
        P.dsptr.clear();
        for (size_t r = 0; r < top.size(); ++r) {
            const int32_t t = top[r];
            const int32_t f = first[r], e = P.sptr[t + 1];
            const int64_t below = (P.srowptr[t + 1] - P.srowptr[t]) - (P.sptr[t + 1] - P.sptr[t]);
            int32_t c = f;
            while (c < e) {
                const int64_t rows = (int64_t)(e - c) + below;
                const int64_t by_bytes = (int64_t)((((uint64_t)1 << 32) - 1) / (8 * (uint64_t)rows));
                const int32_t wmax = (int32_t)std::max<int64_t>(1, std::min<int64_t>(max_width, by_bytes));
                P.dsptr.push_back(c);
                dtop.push_back(t);
                dend.push_back(e);
                c = (int32_t)std::min<int64_t>(e, (int64_t)c + wmax);
            }
        }
        P.nds = (int32_t)P.dsptr.size();
        P.dsptr.push_back(n);
        P.dsparent.assign((size_t)P.nds, -1);
        P.dsrowptr.assign((size_t)P.nds + 1, 0);
        for (int32_t r = 0; r < P.nds; ++r) {
            const int32_t t = dtop[r];
            const int32_t wt = P.sptr[t + 1] - P.sptr[t];
            const int64_t below = (P.srowptr[t + 1] - P.srowptr[t]) - wt;
            P.dsrowptr[r + 1] = P.dsrowptr[r] + (dend[r] - P.dsptr[r]) + below;
        }
        P.dsrows.resize((size_t)P.dsrowptr[P.nds]);
        std::vector<int32_t> col2ds((size_t)n);
        for (int32_t r = 0; r < P.nds; ++r) {
            const int32_t t = dtop[r];
            int64_t o = P.dsrowptr[r];
            for (int32_t j = P.dsptr[r]; j < dend[r]; ++j) P.dsrows[o++] = j;
            const int32_t wt = P.sptr[t + 1] - P.sptr[t];
            for (int64_t p = P.srowptr[t] + wt; p < P.srowptr[t + 1]; ++p) P.dsrows[o++] = P.srows[p];
            for (int32_t j = P.dsptr[r]; j < P.dsptr[r + 1]; ++j) col2ds[j] = r;
        }
        // parent: the device supernode holding the first row below the columns
        for (int32_t r = 0; r < P.nds; ++r) {
            const int32_t w = P.dsptr[r + 1] - P.dsptr[r];
            if (P.dsrowptr[r + 1] - P.dsrowptr[r] > w) P.dsparent[r] = col2ds[P.dsrows[P.dsrowptr[r] + w]];
        }
    }
    P.dsvaloff.assign((size_t)P.nds + 1, 0);
    for (int32_t s = 0; s < P.nds; ++s) {
        int64_t w = P.dsptr[s + 1] - P.dsptr[s];
        int64_t r = P.dsrowptr[s + 1] - P.dsrowptr[s];
        P.dsvaloff[s + 1] = P.dsvaloff[s] + w * r;
    }
    P.panel_entries = P.dsvaloff[P.nds];

    // ------------------------------------------------------- device blocks
    const int32_t B = P.B;
    P.blk.clear();
    P.bptr.clear();
    P.col2blk.resize((size_t)n);
    for (int32_t s = 0; s < P.nds; ++s) {
        int32_t f = P.dsptr[s], w = P.dsptr[s + 1] - f;
        int32_t r = (int32_t)(P.dsrowptr[s + 1] - P.dsrowptr[s]);
        for (int32_t k = 0; k * B < w; ++k) {
            BlockDesc d;
            d.col0 = f + k * B;
            d.w = std::min(B, w - k * B);
            d.r = r - k * B;
            d.ld = r;
            d.rowoff = P.dsrowptr[s] + (int64_t)k * B;
            d.valoff = P.dsvaloff[s] + (int64_t)k * B * r + (int64_t)k * B;
            int32_t id = (int32_t)P.blk.size();
            for (int32_t j = d.col0; j < d.col0 + d.w; ++j) P.col2blk[j] = id;
            P.blk.push_back(d);
            P.bptr.push_back(d.col0);
        }
    }
    P.bptr.push_back(n);
    P.nb = (int32_t)P.blk.size();
    const int32_t nb = P.nb;
    P.bparent.assign((size_t)nb, -1);
    for (int32_t b = 0; b < nb; ++b) {
        const BlockDesc &d = P.blk[b];
        if (d.r > d.w) P.bparent[b] = P.col2blk[P.dsrows[d.rowoff + d.w]];
    }
    P.blevel.assign((size_t)nb, 0);
    for (int32_t b = 0; b < nb; ++b)
        if (P.bparent[b] >= 0)
            P.blevel[P.bparent[b]] = std::max(P.blevel[P.bparent[b]], P.blevel[b] + 1);
    P.nlevels = 0;
    for (int32_t b = 0; b < nb; ++b) P.nlevels = std::max(P.nlevels, P.blevel[b] + 1);
    P.level_ptr.assign((size_t)P.nlevels + 1, 0);
    for (int32_t b = 0; b < nb; ++b) P.level_ptr[P.blevel[b] + 1]++;
    for (int32_t l = 0; l < P.nlevels; ++l) P.level_ptr[l + 1] += P.level_ptr[l];
    P.level_blocks.resize((size_t)nb);
    {
        std::vector<int32_t> fill(P.level_ptr.begin(), P.level_ptr.end() - 1);
        for (int32_t b = 0; b < nb; ++b) P.level_blocks[fill[P.blevel[b]]++] = b;
    }

    // forward-sweep tasks: every block of a level, in chunks of its rows
    P.fwd_level_ptr.assign((size_t)P.nlevels + 1, 0);
    P.fwd_tasks.clear();
    for (int32_t l = 0; l < P.nlevels; ++l) {
        for (int32_t q = P.level_ptr[l]; q < P.level_ptr[l + 1]; ++q) {
            const int32_t b = P.level_blocks[q];
            const int32_t nch = std::max(1, (P.blk[b].r - P.blk[b].w + kSolveChunk - 1) / kSolveChunk);
            for (int32_t c = 0; c < nch; ++c) P.fwd_tasks.push_back(SolveTask{b, c, 0, -1});
        }
        P.fwd_level_ptr[l + 1] = (int64_t)P.fwd_tasks.size();
    }
    P.bwd_level_ptr.assign((size_t)P.nlevels + 1, 0);
    P.bwd_tasks.clear();
    for (int32_t l = 0; l < P.nlevels; ++l) {
        for (int32_t q = P.level_ptr[l]; q < P.level_ptr[l + 1]; ++q) {
            const int32_t b = P.level_blocks[q];
            const int32_t nch = (P.blk[b].r - P.blk[b].w + kSolveChunk - 1) / kSolveChunk;
            for (int32_t c = 0; c < nch; ++c) P.bwd_tasks.push_back(SolveTask{b, c, 0, -1});
        }
        P.bwd_level_ptr[l + 1] = (int64_t)P.bwd_tasks.size();
    }
    // dataflow form: every chunk's distinct target blocks (its rows are
    // increasing, so equal blocks are adjacent), the number of chunks that
    // update each block, and the backward order
    P.fwd_first.assign((size_t)nb, 0);
    P.chunk_tptr.assign(1, 0);
    P.chunk_tgt.clear();
    P.fwd_pend.assign((size_t)nb, 0);
    for (size_t q = 0; q < P.fwd_tasks.size(); ++q) {
        SolveTask &t = P.fwd_tasks[q];
        const BlockDesc &d = P.blk[t.J];
        if (t.chunk == 0) P.fwd_first[t.J] = (int32_t)q;
        t.list = (int32_t)q;
        const int32_t i0 = d.w + t.chunk * kSolveChunk, i1 = std::min(d.r, i0 + kSolveChunk);
        int32_t last = -1;
        for (int32_t i = i0; i < i1; ++i) {
            const int32_t b2 = P.col2blk[P.dsrows[d.rowoff + i]];
            if (b2 != last) {
                P.chunk_tgt.push_back(b2);
                P.fwd_pend[b2]++;
                last = b2;
            }
        }
        P.chunk_tptr.push_back((int64_t)P.chunk_tgt.size());
    }
    P.bwd_pend.assign((size_t)nb, 0);
    P.bwd_df.clear();
    for (int32_t l = P.nlevels - 1; l >= 0; --l) {
        for (int32_t q = P.level_ptr[l]; q < P.level_ptr[l + 1]; ++q) {
            const int32_t b = P.level_blocks[q];
            const int32_t nch = (P.blk[b].r - P.blk[b].w + kSolveChunk - 1) / kSolveChunk;
            P.bwd_pend[b] = nch;
            for (int32_t c = 0; c < nch; ++c) P.bwd_df.push_back(SolveTask{b, c, 0, P.fwd_first[b] + c});
        }
        // the last of a block's chunks finishes it; blocks without chunks
        // get a task of their own
        for (int32_t q = P.level_ptr[l]; q < P.level_ptr[l + 1]; ++q)
            if (P.bwd_pend[P.level_blocks[q]] == 0)
                P.bwd_df.push_back(SolveTask{P.level_blocks[q], -1, 0, -1});
    }
    P.fwd_slots = sweep_slots(P, P.fwd_tasks, true);
    P.bwd_slots = sweep_slots(P, P.bwd_df, false);

    // backward sweep with walkers: device supernodes of three or more
    // blocks, none but the last a one-wavefront block
    {
        std::vector<int32_t> walk_end((size_t)nb, -1);   // at the walk's first block: its last
        std::vector<uint8_t> walked((size_t)nb, 0);
        std::vector<std::pair<int32_t, int32_t>> cand;    // (blocks, supernode)
        for (int32_t r = 0; r < P.nds; ++r) {
            if (P.dsptr[r + 1] <= P.dsptr[r]) continue;
            const int32_t b0 = P.col2blk[P.dsptr[r]], bl = P.col2blk[P.dsptr[r + 1] - 1];
            if (bl - b0 < 2) continue;
            bool ok = true;
            for (int32_t b = b0; b < bl; ++b) ok = ok && !wave_task_block(P.blk[b]);
            if (ok) cand.push_back({bl - b0 + 1, r});
        }
        // the longest chains, at most kWalkMax of them
        std::stable_sort(cand.begin(), cand.end(),
                         [](const std::pair<int32_t, int32_t> &x, const std::pair<int32_t, int32_t> &y) {
                             return x.first > y.first;
                         });
        if ((int32_t)cand.size() > kWalkMax) cand.resize(kWalkMax);
        P.nwalk = (int32_t)cand.size();
        for (const auto &c : cand) {
            const int32_t b0 = P.col2blk[P.dsptr[c.second]], bl = P.col2blk[P.dsptr[c.second + 1] - 1];
            walk_end[bl - 1] = b0;
            for (int32_t b = b0; b < bl; ++b) walked[b] = 1;
        }
        std::vector<int32_t> nchw((size_t)nb, 0), skip((size_t)nb, 0);
        for (int32_t b = 0; b < nb; ++b) {
            skip[b] = walked[b] ? P.blk[b + 1].w : 0;
            nchw[b] = (P.blk[b].r - P.blk[b].w - skip[b] + kSolveChunk - 1) / kSolveChunk;
        }
        P.bw_df.clear();
        P.bw_tptr.assign(1, 0);
        P.bw_tgt.clear();
        P.bw_pend.assign((size_t)nb, 0);
        for (int32_t l = P.nlevels - 1; l >= 0; --l) {
            for (int32_t q = P.level_ptr[l]; q < P.level_ptr[l + 1]; ++q) {
                const int32_t b = P.level_blocks[q];
                if (walk_end[b] >= 0) P.bw_df.push_back(SolveTask{b, kWalkTask, walk_end[b], -1});
            }
            for (int32_t q = P.level_ptr[l]; q < P.level_ptr[l + 1]; ++q) {
                const int32_t b = P.level_blocks[q];
                const BlockDesc &d = P.blk[b];
                P.bw_pend[b] = nchw[b] + (walked[b] ? 1 : 0);
                for (int32_t c = 0; c < nchw[b]; ++c) {
                    const int32_t i0 = d.w + skip[b] + c * kSolveChunk, i1 = std::min(d.r, i0 + kSolveChunk);
                    const int32_t list = (int32_t)P.bw_tptr.size() - 1;
                    int32_t last = -1;
                    for (int32_t i = i0; i < i1; ++i) {
                        const int32_t b2 = P.col2blk[P.dsrows[d.rowoff + i]];
                        if (b2 != last) {
                            P.bw_tgt.push_back(b2);
                            last = b2;
                        }
                    }
                    P.bw_tptr.push_back((int64_t)P.bw_tgt.size());
                    P.bw_df.push_back(SolveTask{b, c, skip[b], list});
                }
            }
            for (int32_t q = P.level_ptr[l]; q < P.level_ptr[l + 1]; ++q) {
                const int32_t b = P.level_blocks[q];
                if (!walked[b] && nchw[b] == 0) P.bw_df.push_back(SolveTask{b, -1, 0, -1});
            }
        }
        P.bw_slots = sweep_slots(P, P.bw_df, false);
    }

    // ------------------------------------------ descendant pairs (prune set)
    // Block K's rows below its own columns fall into runs of consecutive
    // local rows that lie in one target block's columns.
    P.dptr.assign((size_t)nb + 1, 0);
    P.tptr.assign((size_t)nb + 1, 0);
    for (int32_t K = 0; K < nb; ++K) {
        const BlockDesc &d = P.blk[K];
        const int32_t *rows = P.dsrows.data() + d.rowoff;
        int32_t p = d.w;
        while (p < d.r) {
            int32_t J = P.col2blk[rows[p]];
            int32_t end = P.blk[J].col0 + P.blk[J].w;
            int32_t q = p;
            while (q < d.r && rows[q] < end) ++q;
            P.dptr[J + 1]++;
            P.tptr[K + 1]++;
            p = q;
        }
    }
    for (int32_t b = 0; b < nb; ++b) { P.dptr[b + 1] += P.dptr[b]; P.tptr[b + 1] += P.tptr[b]; }
    P.pairs.resize((size_t)P.dptr[nb]);
    P.tJ.resize((size_t)P.tptr[nb]);
    {
        std::vector<int64_t> fill(P.dptr.begin(), P.dptr.end() - 1);
        int64_t tq = 0;
        for (int32_t K = 0; K < nb; ++K) {
            const BlockDesc &d = P.blk[K];
            const int32_t *rows = P.dsrows.data() + d.rowoff;
            int32_t p = d.w;
            while (p < d.r) {
                int32_t J = P.col2blk[rows[p]];
                int32_t end = P.blk[J].col0 + P.blk[J].w;
                int32_t q = p;
                while (q < d.r && rows[q] < end) ++q;
                Pair pr;
                pr.K = K; pr.a0 = p; pr.a1 = q; pr.pad = 0;
                P.pairs[fill[J]++] = pr;
                P.tJ[tq++] = J;
                p = q;
            }
        }
    }

    // ------------------------------------------------ factor schedule
    // Supernodes of one level of the supernodal elimination tree are
    // independent.  Per level:
    //   external: every row tile of every block of the level's supernodes
    //             gathers its descendants from other supernodes; tile 0 of
    //             each supernode's first block then factors that block;
    //   trsm:     the first block's other row tiles solve against it;
    //   for k = 1, 2, ...: internal updates of blocks c >= k by the now final
    //             block k-1 of the same supernode (right-looking), tile 0 of
    //             block k fused with its factorization; then block k's trsm.
    P.svariant.assign((size_t)P.nds, 1);
    build_schedule(P);

    // ----------------------------------- arithmetic per launch kind
    // The method's count sum_k |L_k|^2 split by the launch kind that performs
    // it, on the true pattern of L (stored zeros excluded).  Column k
    // contributes a square root, |L_k| - 1 divisions and 2 flops for every
    // pair j <= i of its rows below k; the pair (j, i) is done by an external
    // update if j lies in another device supernode, by an internal update if
    // j lies in another block of k's device supernode, and otherwise inside
    // k's block: by the fused factorization of its tile 0 (kind external
    // for a supernode's first block, internal otherwise) when row i is among
    // the block's first 64 rows, else by an off-diagonal tile solve.
    {
        for (double &f : P.kind_flops) f = 0.0;
        std::vector<int32_t> col2ds((size_t)n);
        for (int32_t r = 0; r < P.nds; ++r)
            for (int32_t j = P.dsptr[r]; j < P.dsptr[r + 1]; ++j) col2ds[j] = r;
        std::vector<int32_t> blk_first((size_t)P.nb, 0);
        for (int32_t r = 0; r < P.nds; ++r) blk_first[P.col2blk[P.dsptr[r]]] = 1;
        for (int32_t s2 = 0; s2 < ns; ++s2) {
            const int32_t *frows = P.srows.data() + P.srowptr[s2];
            const int32_t fr = (int32_t)(P.srowptr[s2 + 1] - P.srowptr[s2]);
            for (int32_t k = P.sptr[s2]; k < P.sptr[s2 + 1]; ++k) {
                const int32_t *r = frows + (k - P.sptr[s2]);
                const int64_t c = fr - (k - P.sptr[s2]);
                const int32_t bk = P.col2blk[k];
                const BlockDesc &d = P.blk[bk];
                const int fused = blk_first[bk] ? 1 : 3;
                const int32_t *drows = P.dsrows.data() + d.rowoff;
                const int32_t thr = d.r > kTileRows ? drows[kTileRows - 1] : INT32_MAX;
                const int64_t q1 = std::upper_bound(r, r + c, d.col0 + d.w - 1) - r;
                const int64_t q2 = std::upper_bound(r, r + c, P.dsptr[col2ds[k] + 1] - 1) - r;
                const int64_t t0 = std::upper_bound(r, r + c, thr) - r;
                P.kind_flops[fused] += 1.0 + (double)(t0 - 1);
                P.kind_flops[2] += (double)(c - t0);
                for (int64_t p = 1; p < q1; ++p) {
                    P.kind_flops[fused] += 2.0 * (double)std::max<int64_t>(0, t0 - p);
                    P.kind_flops[2] += 2.0 * (double)(c - std::max<int64_t>(p, t0));
                }
                // sum_{p=a}^{b-1} (c - p)
                auto tri = [c](int64_t a, int64_t b) -> double {
                    if (b <= a) return 0.0;
                    return (double)(b - a) * (double)c - ((double)(a + b - 1) * (double)(b - a)) / 2.0;
                };
                P.kind_flops[3] += 2.0 * tri(q1, q2);
                P.kind_flops[1] += 2.0 * tri(q2, c);
            }
        }
    }

    // ----------------------- permuted coordinates of A's entries, diagonal
    P.acoord.resize(2 * (size_t)P.nnzA);
    P.adiag.assign((size_t)n, -1);
    for (int32_t c = 0; c < n; ++c)
        for (int64_t p = C.cp[c]; p < C.cp[c + 1]; ++p) {
            P.acoord[2 * (size_t)C.src[p]] = C.ci[p];
            P.acoord[2 * (size_t)C.src[p] + 1] = c;
            if (C.ci[p] == c) P.adiag[c] = C.src[p];
        }

    // ------------------------------------------------------ A -> L map
    P.amap.resize((size_t)P.nnzA);
    for (int32_t c = 0; c < n; ++c) {
        const BlockDesc &d = P.blk[P.col2blk[c]];
        const int32_t *rows = P.dsrows.data() + d.rowoff;
        int32_t lc = c - d.col0;
        for (int64_t p = C.cp[c]; p < C.cp[c + 1]; ++p) {
            int32_t row = C.ci[p];
            const int32_t *it = std::lower_bound(rows, rows + d.r, row);
            if (it == rows + d.r || *it != row) return SYM_EPATTERN;   // internal inconsistency
            int64_t lr = it - rows;
            P.amap[C.src[p]] = d.valoff + (int64_t)lc * d.ld + lr;
        }
    }

    // ------------------------------------ full symmetric rows of A (residual)
    P.arowptr.assign((size_t)n + 1, 0);
    for (int32_t j = 0; j < n; ++j)
        for (int64_t p = Ap[j]; p < Ap[j + 1]; ++p) {
            P.arowptr[Ai[p] + 1]++;
            if (Ai[p] != j) P.arowptr[j + 1]++;
        }
    for (int32_t i = 0; i < n; ++i) P.arowptr[i + 1] += P.arowptr[i];
    P.acol.resize((size_t)P.arowptr[n]);
    P.aval.resize((size_t)P.arowptr[n]);
    {
        std::vector<int64_t> fill(P.arowptr.begin(), P.arowptr.end() - 1);
        for (int32_t j = 0; j < n; ++j)
            for (int64_t p = Ap[j]; p < Ap[j + 1]; ++p) {
                const int32_t i = Ai[p];
                P.acol[fill[i]] = j;
                P.aval[fill[i]++] = p;
                if (i != j) {
                    P.acol[fill[j]] = i;
                    P.aval[fill[j]++] = p;
                }
            }
    }

    P.analyze_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return SYM_OK;
}

SweepSlots sweep_slots(const Plan &P, const std::vector<SolveTask> &tasks, bool bottom_first)
{
    SweepSlots S;
    const int64_t n = (int64_t)tasks.size();
    // the run of wide levels: [wa, wb)
    std::vector<int64_t> run(1, 0);
    for (int64_t i = 1; i < n; ++i)
        if (P.blevel[tasks[i].J] != P.blevel[tasks[i - 1].J]) run.push_back(i);
    if (n > 0) run.push_back(n);
    const size_t nr = run.size() - 1;
    int64_t wa = 0, wb = 0;
    if (bottom_first) {
        size_t r = 0;
        while (r < nr && run[r + 1] - run[r] >= kWideLevel) ++r;
        wa = 0;
        wb = run[r];
    } else {
        size_t r = nr;
        while (r > 0 && run[r] - run[r - 1] >= kWideLevel) --r;
        wa = run[r];
        wb = n;
    }
    auto wave = [&](int64_t i) { return wave_task_block(P.blk[tasks[i].J]); };
    int64_t i = 0;
    S.start.push_back(0);
    while (i < n) {
        int64_t j = i;
        if (tasks[i].chunk == kWalkTask) {
            // a walker takes a workgroup for a whole supernode: alone
            j = i + 1;
            S.quad.push_back(0);
        } else if (wave(i)) {
            while (j < n && j - i < 4 && wave(j)) ++j;
            S.quad.push_back(1);
        } else {
            const int64_t cap = (i >= wa && i < wb) ? kSlotGroup : 1;
            while (j < n && j - i < cap && !wave(j) && tasks[j].chunk != kWalkTask) ++j;
            S.quad.push_back(0);
        }
        S.start.push_back((int32_t)j);
        i = j;
    }
    return S;
}

void reach_etree(const Plan &P, const std::vector<int32_t> &beta, std::vector<int32_t> &out)
{
    std::vector<char> seen((size_t)P.n, 0);
    out.clear();
    for (int32_t b : beta) {
        int32_t j = b;
        while (j >= 0 && !seen[j]) {
            seen[j] = 1;
            out.push_back(j);
            j = P.parent[j];
        }
    }
    std::sort(out.begin(), out.end());
}

}  // namespace sym
