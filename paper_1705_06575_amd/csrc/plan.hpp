// plan.hpp -- host-side symbolic plan and the device-side view of it.
//
// Storage of L: each fundamental supernode s (columns [f_s, f_s + w_s), row
// list R_s of length r_s, sorted, whose first w_s entries are the
// supernode's own columns) owns a dense column-major panel of r_s x w_s
// values with leading dimension r_s.  The upper triangle of the w_s x w_s
// diagonal block is stored but never read.
//
// Device tasks work on column blocks: a supernode is cut into blocks of at
// most `block_width` columns.  Block k of s covers columns
// [f_s + k*B, f_s + min((k+1)*B, w_s)) and rows R_s[k*B ...]; its panel is
// the sub-panel of s starting at local (row k*B, column k*B) with the same
// leading dimension.  Cutting changes only the blocking of the arithmetic,
// never the factor.
#pragma once

#include <climits>
#include <cstdint>
#include <vector>

namespace sym {

struct BlockDesc {      // 32 bytes, device-visible
    int64_t valoff;     // offset of the block's panel (its local (0,0)) in L's value array
    int64_t rowoff;     // offset of the block's first row index in the row-index array
    int32_t col0;       // first column (permuted numbering)
    int32_t w;          // number of columns
    int32_t r;          // number of rows, including the w diagonal rows
    int32_t ld;         // leading dimension of the panel (r of the supernode)
};

struct Pair {           // 16 bytes: descendant block K updates target block J
    int32_t K;          // descendant block id
    int32_t a0;         // first local row of K inside J's columns
    int32_t a1;         // one past the last local row of K inside J's columns
    int32_t pad;
};

struct Task {           // 16 bytes: one row tile of one block
    int32_t J;          // target block
    int32_t t;          // tile index: local rows [t*T, min((t+1)*T, r_J))
    int32_t K;          // source block (internal updates), PartDesc index (kPartial), else -1
    int32_t flags;      // kFuseFactor: the task also factors the block; internal
                        // updates: source block count - 1 from bit kDepthShift
};

// One descendant block K's contribution to one row tile of a target block
// J: K's local rows [a0, a0 + nJ) lie in J's columns and K's local rows
// [b0, b0 + nI) in the tile's rows.  map[mapoff ...] holds the nI
// tile-relative rows of the latter, then the nJ tile columns of the former
// (both increasing); cmin and cmax are the first and last of those columns.
struct Incidence {      // 40 bytes, device-visible
    int64_t valoff;     // K's panel offset
    int64_t mapoff;     // offset into the relative-index map
    int32_t ld;         // K's leading dimension
    int32_t b0;
    int32_t a0;
    int16_t wk;         // K's width
    uint8_t nI, nJ;
    uint8_t cmin, cmax;
    uint8_t pad[6];
};

// The same contribution as one wavefront sees it.  Wavefront v of a tile's
// workgroup owns the tile's columns [16v, 16v + 16); for every incidence
// that meets them it gets an item: the product rows are K's local rows
// [b0, b0 + nI), the product columns K's local rows [a0, a0 + nJ) (those
// landing in the wavefront's columns, nJ <= 16).  wmap[mapoff ...] holds
// the nI tile-relative rows, then the nJ tile columns.
struct WaveItem {       // 32 bytes, device-visible
    int64_t valoff;     // K's panel offset
    int64_t mapoff;     // offset into the wavefront map
    int32_t ld;         // K's leading dimension
    int32_t b0;
    int32_t a0;
    int16_t wk;         // K's width (inner dimension)
    uint8_t nI, nJ;
};

// One chunk of a staged external-update product (a tile's incidence
// split into runs of at most kStageK inner indices): the whole workgroup
// stages K's rows [b0, b0 + nI) of the chunk's inner indices in LDS once;
// wavefront v multiplies them with the product columns that land in its 16
// tile columns, [jw[v-1], jw[v]) (jw[-1] = 0, jw[3] = nJ).  map: byte
// offset in imap of the incidence's nI tile rows and nJ tile columns.
struct StageChunk {     // 32 bytes, device-visible
    int64_t valoff;     // K's panel offset
    int32_t ld;         // K's leading dimension
    int32_t b0;         // K's local row of the first product row
    int32_t a0;         // K's local row of the first product column
    uint32_t map;
    int16_t kc;         // first inner index of the chunk
    uint8_t nI, nJ;
    uint8_t nk_last;    // inner indices in the chunk (1..kStageK); bit 7: the incidence's last chunk
    uint8_t jw[3];
};
constexpr int kStageK = 16;
constexpr int32_t kStaged = 4;      // Task flag: the tile's products run as staged chunks

static_assert(sizeof(Incidence) == 40, "Incidence layout is shared with the device");
static_assert(sizeof(StageChunk) == 32, "StageChunk layout is shared with the device");
static_assert(sizeof(WaveItem) == 32, "WaveItem layout is shared with the device");
static_assert(sizeof(BlockDesc) == 32, "BlockDesc layout is shared with the device");

constexpr int32_t kQuadSlot = INT32_MIN;   // Plan::xslot: a slot of narrow tiles

constexpr int32_t kFuseFactor = 1;
// An internal update (kPhaseInternal) reads the source blocks K, K + 1, ...,
// K + (flags >> kDepthShift) of the target's supernode, one product of inner
// dimension up to kMaxUpdateDepth x 64 per tile (Plan::update_depth).
constexpr int32_t kDepthShift = 8;
constexpr int32_t kUpdateDepth = 4;
constexpr int32_t kMaxUpdateDepth = 16;
// A task of a chain launch (kPhaseChain) that ends by solving its tile
// against its block's factored diagonal block (X := X L_JJ^{-T}).
constexpr int32_t kChainSolve = 8;
// A long external-update tile is split into parts (tasks of the same launch
// with kPartial and K = index of their PartDesc): each part accumulates
// its share of the products into a partial tile; the part that finishes
// last adds all partials in part order to the tile (and factors it if the
// tile carries kFuseFactor).
constexpr int32_t kPartial = 2;
// A part holds about max(kSplitUnits, level cost / kSplitShare) estimated
// 16-wide k-batches: small levels split finely, so that their few long
// tiles spread over the chip; large levels split only where a tile would
// hold a workgroup far beyond the average share (12288 = 256 compute units
// x 3 resident workgroups x 16).
constexpr double kSplitUnits = 64.0;
constexpr double kSplitShare = 12288.0;

struct PartDesc {       // 16 bytes, device-visible
    int32_t counter;    // arrival counter of the split tile (zero between launches)
    int32_t part;       // this part's index
    int32_t nparts;
    int32_t slot0;      // partial-tile slot of part 0 (part p uses slot0 + p)
};
static_assert(sizeof(PartDesc) == 16, "PartDesc layout is shared with the device");

// Kernel variant of a target supernode's external update.  Variants 0-2:
// an incidence is "large" -- multiplied by the whole workgroup through LDS
// -- when its product has at least kVariantLarge[v] rows, columns and inner
// indices; the others run as per-wavefront items (variant 0 puts every
// incidence there, 1 uses 64, 2 uses 32).  Variant 3: every incidence runs
// as staged chunks (StageChunk): its rows are read once per tile, instead
// of once per wavefront whose columns it meets.
constexpr int kVariants = 4;
constexpr int32_t kVariantLarge[kVariants] = {1 << 30, 64, 32, 0};
constexpr uint8_t kVariantStaged = 3;
constexpr int kSuperFeatures = 12;  // features of a device supernode, see Plan::sfeat

// One kernel launch of the factorization.  A chain launch runs, for the
// supernodes of one level, the off-diagonal solves of their first blocks
// and every right-looking step inside them (update by the previous block,
// then factorization or solve of the next block's tiles) as one persistent
// launch whose tasks wait for the tiles they read (Plan::tbase; only with
// Plan::chain_launch); by default every step is a kPhaseInternal launch
// followed by a kPhaseTrsm launch.
// A kPhaseLeaf launch factors leaves of the supernodal tree whose block is
// one tile of at most 16 columns (no update reaches a leaf), one wavefront
// per block.  An external launch runs its tasks by workgroup slot
// (Plan::xslot): one task, or (kQuadSlot) up to four tiles of blocks of at
// most 16 columns (not split, not staged), one wavefront each.
enum PhaseKind : int32_t { kPhaseExternal = 0, kPhaseTrsm = 1, kPhaseInternal = 2, kPhaseChain = 3,
                           kPhaseLeaf = 4 };
struct Phase {
    int32_t kind;
    int64_t t0, t1;     // task range in Plan::ftasks
    int64_t s0 = -1;    // kPhaseExternal: its workgroup slots at Plan::xslot[s0 .. s0 + nslots]
    int64_t nslots = 0;
};

// Factor precisions (sym.h: SYM_F64, SYM_F32, SYM_BF16, SYM_F16).  FP32
// panels for all but the first; the last two scale the matrix per device
// supernode and run the update products on 16-bit matrix cores.
constexpr int32_t kPrecF64 = 0, kPrecF32 = 1, kPrecBF16 = 2, kPrecF16 = 3;
inline bool prec_fp32_panels(int32_t p) { return p != kPrecF64; }
inline bool prec_scaled(int32_t p) { return p == kPrecBF16 || p == kPrecF16; }

constexpr int kTileRows = 64;   // T: rows per factor task tile
constexpr int kSolveChunk = 256; // rows below the diagonal per forward-solve task

// Ticket slots of a persistent sweep.  A workgroup takes one slot per
// ticket and runs the slot's tasks [start[s], start[s + 1]): either in
// order, by the whole workgroup, or -- a quad slot -- one task per
// wavefront, all at once (the blocks of a quad's tasks are narrow: at most
// kWaveCols columns and kWaveRows rows below them, so one wavefront holds a
// task).  Consecutive narrow tasks form quads wherever they occur; in the
// run of wide levels (many independent tasks) the other tasks go up to
// kSlotGroup to a slot, so that the one ticket counter does not serialize
// them; elsewhere they keep one task per slot.  Slots are taken in task
// order and a task waits only on tasks before it (in earlier slots, or in
// the same quad, whose wavefronts run concurrently), so no wait is circular.
struct SweepSlots {
    std::vector<int32_t> start;     // slots + 1
    std::vector<uint8_t> quad;      // per slot: 1 = one task per wavefront
    int64_t count() const { return (int64_t)quad.size(); }
};
constexpr int32_t kSlotGroup = 4;      // tasks per slot in a wide level
constexpr int64_t kWideLevel = 2048;   // tasks that make a level wide
constexpr int32_t kWaveCols = 16;      // widest block of a wavefront task
constexpr int32_t kWaveRows = 64;      // most rows below a wavefront task's block

constexpr int32_t kWalkTask = -2;      // SolveTask::chunk of a backward walker
// walkers hold workgroups while they wait for chunk tasks of later tickets:
// the walker schedule runs only while value sets x walkers stays within this
constexpr int32_t kWalkBudget = 128;
constexpr int32_t kWalkMax = 64;        // walkers of a plan: the supernodes with the most blocks

struct SolveTask {      // 16 bytes: one chunk of one block in a sweep
    int32_t J;
    int32_t chunk;      // rows [w + chunk*kSolveChunk, ...) below the diagonal;
                        // -1: the block's diagonal solve (backward sweep)
    int32_t c0;         // first column of the block to solve (reach-pruned sweeps)
    int32_t list;       // the chunk's target-block list (chunk_tptr), -1 if none
};

struct Plan {
    // ---- input
    int32_t n = 0;
    int64_t nnzA = 0;
    int32_t B = 64;             // block width
    int32_t precision = 0;      // kPrec*
    double split_share = kSplitShare;  // a long external tile's part: max(kSplitUnits, level cost / share)
    double pivot_floor = 0.0;   // tau: pivots below tau times their scaled diagonal entry are
                                // replaced by it (scaled precisions only; 0 = never)
    bool chain_launch = false;  // the steps inside a level's supernodes as one persistent launch
    int32_t update_depth = kUpdateDepth;  // source blocks per grouped internal update
    double analyze_ms = 0.0;

    // ---- ordering and column structure (permuted numbering)
    std::vector<int32_t> perm, pinv;
    std::vector<int32_t> parent;
    std::vector<int64_t> colcount;
    double flops = 0.0;         // sum_j colcount_j^2
    int64_t nnzL = 0;

    // ---- fundamental supernodes
    int32_t ns = 0;
    std::vector<int32_t> sptr;      // ns+1
    std::vector<int32_t> sparent;   // ns
    std::vector<int64_t> srowptr;   // ns+1
    std::vector<int32_t> srows;     // sum r_s

    // ---- device supernodes: the fundamental ones after relaxed
    // amalgamation (explicit zeros); panels and blocks are built on these
    int32_t nds = 0;
    std::vector<int32_t> dsptr;     // nds+1
    std::vector<int32_t> dsparent;  // nds
    std::vector<int64_t> dsrowptr;  // nds+1
    std::vector<int32_t> dsrows;    // row lists (columns first, then the rows below)
    std::vector<int64_t> dsvaloff;  // nds+1, panel offsets
    int64_t panel_entries = 0;

    // ---- device blocks
    int32_t nb = 0;
    std::vector<BlockDesc> blk;
    std::vector<int32_t> bptr;      // nb+1 first column of each block, then n
    std::vector<int32_t> bparent;   // nb
    std::vector<int32_t> blevel;    // nb
    std::vector<int32_t> col2blk;   // n
    int32_t nlevels = 0;
    std::vector<int32_t> level_ptr;     // nlevels+1 into level_blocks
    std::vector<int32_t> level_blocks;  // nb, blocks sorted by level (stable in id)
    std::vector<int64_t> fwd_level_ptr; // nlevels+1 into fwd_tasks
    std::vector<SolveTask> fwd_tasks;   // forward-sweep tasks grouped by level
    std::vector<int64_t> bwd_level_ptr; // nlevels+1 into bwd_tasks
    std::vector<SolveTask> bwd_tasks;   // backward off-diagonal chunks (blocks with rows below)
    // dataflow form of the sweeps (one launch each): list q (= forward task
    // q) holds the distinct blocks owning the rows of that chunk
    std::vector<int32_t> fwd_first;     // nb: forward task of each block's chunk 0
    std::vector<int64_t> chunk_tptr;    // fwd_tasks.size()+1
    std::vector<int32_t> chunk_tgt;
    std::vector<int32_t> fwd_pend;      // nb: forward chunks whose rows meet the block
    std::vector<int32_t> bwd_pend;      // nb: off-diagonal chunks of the block
    std::vector<SolveTask> bwd_df;      // backward tasks, levels from the top: gathers (the last of a block finishes it), then blocks without rows below
    SweepSlots fwd_slots, bwd_slots;    // ticket slots of the two dense sweeps
    // the backward sweep with walkers (used for few value sets): one task
    // per wide supernode (chunk kWalkTask, J = the block it starts at, c0 =
    // the block it ends at) finishes its blocks but the last, from the top,
    // and computes their rows that hold the next block's columns itself;
    // the chunk tasks of those blocks skip those rows (c0 = their count) and
    // never finish the block (its counter starts one above their number)
    std::vector<SolveTask> bw_df;
    std::vector<int64_t> bw_tptr;       // bw_df chunks' target-block lists
    std::vector<int32_t> bw_tgt;
    std::vector<int32_t> bw_pend;       // nb
    SweepSlots bw_slots;
    int32_t nwalk = 0;                  // walker tasks

    // split external tiles: part descriptors, and the counts of arrival
    // counters and of 64 x 64 partial-tile slots they use
    std::vector<int32_t> inv_blocks;    // blocks of <= 16 columns, then the wider ones
    int32_t inv_nsmall = 0;             // blocks of <= 16 columns in inv_blocks
    std::vector<PartDesc> parts;
    int32_t nsplit = 0;
    int64_t npartial = 0;

    // per device supernode: kernel variant of its external update, and the
    // features a cost model sees (kSuperFeatures each): width, rows, row
    // tiles of its blocks, incidences it receives, their product flops,
    // the fractions of those flops in incidences of >= 64 and >= 32 rows,
    // columns and inner indices, its level; then the level's context (the
    // supernodes it shares its launches with): the level's update flops,
    // its supernode count, its row tiles receiving updates, and this
    // supernode's share of the level's update flops
    std::vector<uint8_t> svariant;
    std::vector<double> sfeat;
    std::vector<int32_t> task_super;    // ftasks.size(): target supernode of external tasks, else -1

    // descendant pairs, grouped by target block
    std::vector<int64_t> dptr;      // nb+1
    std::vector<Pair> pairs;
    // the same pairs grouped by descendant block (for the backward sweep)
    std::vector<int64_t> tptr;      // nb+1
    std::vector<int32_t> tJ;        // target block of each pair, grouped by K

    // supernodal schedule of the factorization
    std::vector<int32_t> sbptr;     // nds+1: first block of each device supernode
    std::vector<int32_t> slevel;    // nds
    int32_t nslevels = 0;
    std::vector<Task> ftasks;       // all factor tasks in launch order
    std::vector<Phase> phases;      // launches
    // tiles of the chain launches: tile t of block J is tile tbase[J] + t
    // (every block's 64-row tiles, ceil(r / 64) each); the state of a tile
    // counts the operations done on it: it starts at b0, the first block of
    // the tile's supernode (b0 + 1 for tile 0 of block b0, factored by the
    // external launch), becomes K + 1 once block K's update has been
    // applied, and J + 1 once the tile is final (factored or solved).
    // per external launch: its slots' first tasks (launch-relative; bit 31
    // marks a slot of narrow tiles), then its task count
    std::vector<int32_t> xslot;
    std::vector<int32_t> tbase;     // nb + 1
    std::vector<int32_t> tinit;     // tbase[nb]: initial states
    int32_t nchain = 0;             // chain launches
    std::vector<int64_t> iptr;      // ftasks.size()+1: incidences of external-update tasks
    std::vector<int64_t> ibig;      // ftasks.size(): end of each task's leading large incidences
    std::vector<uint8_t> phase_coop;// per phase: an external phase with large incidences
    std::vector<Incidence> incs;
    std::vector<uint8_t> imap;      // tile-relative rows and columns of every incidence
    // the remaining (small) incidences as per-wavefront items: wavefront v of
    // task q runs items [wptr[16q + 4v], wptr[16q + 4v + 4]), in four groups
    // by row blocks: [wptr[16q + 4v + g], wptr[16q + 4v + g + 1]) holds the
    // items of 4 - g blocks of 16 rows
    std::vector<int64_t> wptr;      // 16 * ftasks.size() + 1
    std::vector<WaveItem> witems;
    std::vector<uint8_t> wmap;
    // staged tasks: chunks [cptr[q], cptr[q + 1]) of task q
    std::vector<int64_t> cptr;      // ftasks.size() + 1
    std::vector<StageChunk> chunks;
    // arithmetic of each launch kind by the method's count (lower-triangle
    // products, one flop per multiply, add, divide and square root):
    // [0] scatter (none), [1] external, [2] trsm, [3] internal; the four sum
    // to `flops`.
    double kind_flops[4] = {0, 0, 0, 0};
    // operand entries the external-update products read, summed over the
    // incidences and per-wavefront items of the schedule ((rows + columns)
    // x inner dimension each): the external update's panel reads without
    // any cache reuse
    double ext_operand_entries = 0.0;

    // A -> L map (offset into L's values for every entry of A, input order)
    std::vector<int64_t> amap;
    // for the per-supernode scaling: every entry's permuted (row, column),
    // and the index in A of each permuted column's diagonal entry (-1 if
    // the pattern has none)
    std::vector<int32_t> acoord;    // 2 * nnzA
    std::vector<int64_t> adiag;     // n

    // full symmetric pattern of A in the original ordering, by rows, for the
    // FP64 residual of iterative refinement: row i holds the entries
    // (i, acol[p]) whose value is Ax[aval[p]] (the stored lower entry)
    std::vector<int64_t> arowptr;   // n+1
    std::vector<int32_t> acol;
    std::vector<int64_t> aval;
};

// Analysis entry point (symbolic.cpp).  Returns SYM_OK or a SYM_E* code.
// Device supernodes are at most kMaxDeviceWidth columns wide (and narrower
// where w * r * 8 bytes would reach 4 GiB): widths are 16-bit fields of the
// incidence records, panel offsets 32-bit byte offsets in the kernels.
constexpr int32_t kMaxDeviceWidth = 16384;

int analyze(int64_t n, const int64_t *Ap, const int32_t *Ai, int ordering,
            const int32_t *user_perm, int block_width, int nd_leaf, bool relax, int max_width,
            Plan &P);

// Factor schedule for the plan's current svariant (symbolic.cpp).
void build_schedule(Plan &P);

// Graph nested dissection on the symmetric pattern (ordering.cpp).
// adj: CSR adjacency without self loops.  Returns perm[new] = old.
void nested_dissection(int32_t n, const std::vector<int64_t> &xadj,
                       const std::vector<int32_t> &adj, int32_t leaf,
                       std::vector<int32_t> &perm);

// Reach set of beta (permuted numbering) in the dependence graph of L,
// using the fact that L's column patterns are cliques of the filled graph:
// Reach_L(beta) is the union of the elimination-tree paths from beta to the
// roots.  Output: increasing order.
void reach_etree(const Plan &P, const std::vector<int32_t> &beta, std::vector<int32_t> &out);

// Slots of a sweep over `tasks` (contiguous runs of equal block level):
// with bottom_first the leading run of wide levels is grouped, otherwise
// the trailing one.
SweepSlots sweep_slots(const Plan &P, const std::vector<SolveTask> &tasks, bool bottom_first);

// Whether a block's sweep tasks fit one wavefront.
inline bool wave_task_block(const BlockDesc &d) { return d.w <= kWaveCols && d.r - d.w <= kWaveRows; }

}  // namespace sym
