// Internal types of librv shared by the host planner (plan.cpp, api.cpp) and
// the gfx950 kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "rv.h"

namespace rv {

// ---------------------------------------------------------------- tuning
constexpr int EXP_WG = 256;              // expansion workgroup (4 waves)
constexpr int RPL = 16;                  // records per lane per work item
constexpr int TILE = EXP_WG * RPL;       // records per expansion work item
constexpr int BINCAP = 2048;             // LDS bins of one expansion tile (one window of buckets)
constexpr int BINWIN = 8;                // windows a tile may take on the LDS path
constexpr int NBMAX = 1 << 20;           // location buckets per key-range pass
constexpr int SMAX = 9;                  // a bucket spans at most 2^SMAX locations
constexpr int BKT_WG = 256;              // sort + scan workgroup (4 waves)
constexpr int BKT_RPL = 16;              // records per lane in one on-chip slice
constexpr int CAP = BKT_WG * BKT_RPL;    // records per on-chip slice
constexpr int DEFAULT_TARGET = 2048;     // planner: mean records per bucket
constexpr int FOLD_RPL = 8;              // fold: records per lane in one slice
constexpr uint32_t FOLD_CAP = 256 * FOLD_RPL;   // fold: buckets above this many records are medium
constexpr uint32_t HOT = 1u << 15;       // fold: buckets above this many records are split over workgroups
constexpr int TBL = 1 << SMAX;           // locations of one bucket (LDS table entries)
constexpr uint32_t SMALL_CAP = 2048;     // batched check: passes of at most this many instances run on chip
constexpr uint32_t DIR_CAP = 2048;       // block-local spaces: locations of one on-chip unit's LDS table

static_assert((1 << SMAX) % BKT_WG == 0, "bucket locations split evenly over sort+scan threads");
static_assert(BINCAP % EXP_WG == 0, "tile bins split evenly over expansion threads");

// ------------------------------------------- division by invariant integers
// floor(n / d) for 32-bit n and a divisor d >= 1 fixed at plan time:
// t = mulhi(n, m); q = (t + ((n - t) >> s1)) >> s2 with l = ceil(log2 d),
// m = floor(2^32 (2^l - d) / d) + 1, s1 = min(l, 1), s2 = max(l - 1, 0)
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, section 4).
struct Magic {
    uint32_t m, s1, s2, d;
};

__host__ __device__ inline uint32_t udiv(uint32_t n, Magic g) {
    uint32_t t = (uint32_t)(((uint64_t)n * g.m) >> 32);
    return (t + ((n - t) >> g.s1)) >> g.s2;
}

// floor division of a signed value: for n < 0, floor(n / d) = -(floor((-n-1)/d) + 1) = ~floor(~n / d).
__host__ __device__ inline int32_t fdiv(int32_t n, Magic g) {
    uint32_t u = n >= 0 ? (uint32_t)n : ~(uint32_t)n;
    uint32_t q = udiv(u, g);
    return n >= 0 ? (int32_t)q : (int32_t)~q;
}

// Euclidean remainder in [0, d).
__host__ __device__ inline int32_t emod(int32_t n, Magic g) {
    return n - (int32_t)g.d * fdiv(n, g);
}

Magic make_magic(uint32_t d);

// --------------------------------------------------------- device tables
// Coefficient slots of a device row; the segment variable k is folded into
// the constant because every entry belongs to one dynamic phase.
enum { C_TX = 0, C_TY, C_BX, C_BY, C_L0, C_L1, C_L2, C_A0, C_A1, C_C0, NC };

// One (dynamic phase, access) pair of one barrier interval.
struct DevEntry {
    int32_t row[5][NC];        // idx dim 0..2, aux0 numerator, aux1 numerator
    int32_t aux_kind[2];
    Magic aux_mg[2];
    uint32_t dim[3];           // unused dims hold 1 (their rows are zero)
    int32_t lo[3];             // unused loops: lo 0, ext 1
    uint32_t ext[3];
    uint32_t nloops;
    uint32_t box;              // loop points per thread
    uint32_t off;              // first instance id offset (interval: inside the per-thread range)
    uint32_t tmul;             // instance id = thread * tmul + off + loop index (interval: the
                               // per-thread instance count M; ordered: the phase's loop box)
    uint32_t loc_mul;          // location = block * loc_mul + loc_base + flat
    uint32_t loc_base;
    uint32_t rw;
    uint32_t guard_begin;      // rows (NC int32 each) in the kernel's guard table
    uint32_t guard_count;
    uint32_t lch;              // loop points per lane per work item
    uint32_t gt;               // threads per lane per work item
    uint32_t n_lchunks;        // loop chunks of lch points along the loop box
    // Work-item mapping.  flat = 0: the lanes of an item are 256 consecutive
    // thread groups at one loop chunk (loop counters wave-uniform).  flat = 1
    // (entries with few threads): lane q of the entry takes thread group
    // q / n_lchunks at loop chunk q % n_lchunks, so a kernel with a handful
    // of threads still fills the lanes.
    uint32_t flat;
    uint32_t nq;               // flat: thread groups x loop chunks
    // Flat entries of the general path: chunk-major lanes (lane q takes
    // thread group q % ntg at loop chunk q / ntg), so the lanes of a wave
    // mostly share their loop counters and step the loops together.
    uint32_t cmaj;
    uint32_t ntg;              // thread groups: ceil(threads / gt)
    Magic mg_ntg;
    Magic mg_nl, mg_e1, mg_e2; // divisions by n_lchunks, ext[1], ext[2]
    Magic mg_gt;               // division by gt
    // Fast path (no aux terms, no guards): the location as one affine row
    // modulo 2^32, loc = fr . (tx,ty,bx,by,l0,l1,l2) + fr[C_C0] + block *
    // loc_mul; exact for every in-bounds record.  2: fast and every index of
    // the entry is proven inside its dimension (the exact range of an affine
    // form over the box; an entry that stays 1 has an out-of-bounds instance).
    uint32_t fast;
    uint32_t ndim;
    uint32_t fr[NC];
    // General entries (aux terms or guards).  astep[x][k] = (q, r), the
    // change of aux numerator x when the outer (k = 0), middle (1) or inner
    // (2) loop advances, written as q * d + r with 0 <= r < d (q modulo
    // 2^32), so floor(n / d) and n mod d advance with adds and one carry.  gproven: no
    // guards, and every index stays inside its dimension over the value
    // ranges of the variables and of the aux terms (no per-record test; the
    // location comes from the flattened row, fr[C_A0] and fr[C_A1] included).
    uint32_t astep[2][3][2];
    uint32_t gproven;
    // Linear items (fast entries, one thread per lane, lch points of the
    // innermost non-trivial loop `linner` that never wrap inside a chunk):
    // every index and the location are affine in the point of the chunk.
    uint32_t lin;
    uint32_t linner;
    // The whole loop box is affine in the row-major point index (one loop
    // with points, or coefficients in mixed radix: an outer loop's
    // coefficient is the next inner one's times that loop's extent, for the
    // location and, unless proven, every index), with step fr[linner].
    uint32_t lflat;
    // Thread-linear items (fast entries of one instance per thread, flat
    // mapping, a lane's gt consecutive threads differ in tx alone): every
    // index and the location are affine in the slot.
    uint32_t tlin;
    // Sub-key: the location key is (location << wshift) | sub-interval; the
    // general path shifts its flattened index (loc_mul, loc_base and fr
    // already carry the shift and the sub-interval).
    uint32_t wshift;
};

struct DevKernel {
    uint32_t bdx, bdy, gdx, gdy, tpb, nthreads, nblocks, pad;
    Magic mg_tpb, mg_bdx, mg_gdx;
};

// One key-range pass over one interval (a "sub-interval").  Begin offsets are
// relative to the chunk the pass runs in.
struct DevSub {
    const DevEntry *entries;
    const int32_t *guards;
    const uint32_t *entry_items;   // exclusive prefix of work items per entry (n_entries + 1)
    const DevKernel *kc;
    uint32_t n_entries;
    uint32_t item_begin;
    uint32_t bucket_begin;
    uint32_t nb;                   // buckets
    uint32_t s;                    // bucket = (loc - klo) >> s
    uint32_t klo, khi;             // location range of the pass
    uint32_t M;                    // instances per thread in the interval
    Magic mgM;
    uint32_t interval;
    uint32_t res;                  // result slot
    // Sub-keys (warp barriers; strict semantics' global space): a location
    // spans 2^wshift consecutive keys, one per sub-interval.  Records of one
    // sub-interval are judged as usual; across sub-intervals only records of
    // different units conflict: unit(thread) = block * upb + tid / unit size
    // (warps, or blocks with upb = 1 and unit size = threads per block).
    uint32_t wshift;
    uint32_t upb;
    Magic mg_unit;
    // 1: no entry this pass expands in the HBM pipeline writes, so none of
    // its locations can conflict: the count pass counts its records and
    // out-of-bounds instances, and it has no records and no buckets.  2: as
    // 1, and the pass holds the whole key range of its entries, so the
    // records of proven entries (every index inside its array over the
    // launch and the loop box, no guards: box x threads each) are
    // static_records, added on the host; the count pass evaluates the others.
    uint32_t count_only;
    unsigned long long static_records;
};

// One unit of the on-chip check of block-local spaces: the shared-array
// locations [lo, hi) of consecutive blocks in one pass, whose records all
// come from the threads [t0, t1) (global thread numbers); `sub` indexes the
// chunk's pass table.
struct DevUnit {
    uint32_t sub, lo, hi, t0, t1;
    uint32_t pad[3];
};

// Per-pass result slot (device).
struct SubResult {
    unsigned long long records;
    unsigned long long conflicts;
    unsigned long long oob;        // (interval << 32) | instance id; ~0 when none
    unsigned long long unit_records;   // records checked on chip in block-local units (part of records)
    uint32_t first_bucket;         // chunk-relative; ~0 when none
    uint32_t first_unit;           // chunk-relative unit with the pass's first witness; ~0 when none
    uint32_t pad;                  // nonzero: an internal capacity was exceeded (the result is void)
    uint32_t pad2;
    uint32_t w[4];                 // location, first id, second id, second is_write
};
static_assert(sizeof(SubResult) == 64, "SubResult layout");

// A barrier that carries guards (the threads that reach it), at one dynamic
// phase: its scopes are the block (scope = threads per block, nscope = 1)
// or the block's warps (scope = warp size, nscope = warps per block).
struct DevBarrier {
    uint32_t dphase;
    uint32_t guard_begin, guard_count;   // rows (NC int32 each) in the kernel's guard table, k folded in
    uint32_t scope, nscope;
    uint32_t pad[3];
};

// Per guarded barrier: its divergent scope instances and the first of them
// in (block, scope) order with that instance's smallest reaching thread and
// smallest thread that does not reach it.
struct BarrierResult {
    unsigned long long divergent;
    unsigned long long first;            // block * nscope + scope; ~0 when none
    uint32_t arrive, skip;
    uint32_t pad[2];
};
static_assert(sizeof(BarrierResult) == 32, "BarrierResult layout");

// Per-pass exact counts (rv_check_counts): distinct-thread pairs of the
// interval semantics, or the ordered semantics' dependences.
struct PassCounts {
    unsigned long long pairs, raw, waw, war, deploc;
    unsigned long long pad[3];
};
static_assert(sizeof(PassCounts) == 64, "PassCounts layout");

// Device witness of the collect mode: the SubResult-style words plus the pass.
struct DevWitness {
    uint32_t w[4];
    uint32_t sub;
    uint32_t pad[3];
};

// ------------------------------------------------------------ host plan
struct HostEntry {
    uint32_t dphase, access;
    int32_t kval;
};

struct IntervalPlan {
    uint32_t entry_begin = 0, entry_count = 0;
    uint64_t M = 0;                // instances per thread
    uint64_t P = 0;                // instances (nthreads * M)
    uint64_t K = 0;                // locations
    uint64_t S = 0;                // shared elements per block in this interval's layout
    std::vector<int64_t> arr_off;  // per array: offset in its region, -1 when untouched
    uint32_t s = 0, nb = 0, nsub = 0;
    uint32_t items = 0;
    uint32_t items_begin = 0;      // offset into KernelPlan::entry_items
    uint32_t dphase_begin = 0, dphase_end = 0;
    uint32_t w = 0;                // sub-key bits below the location
    uint32_t unit = 0, upb = 0;    // unordered units across sub-intervals: threads per unit, units per block
    // Block-local spaces checked on chip: shared entries are left out of the
    // HBM pipeline's work items (items_g counts the others) and their
    // locations are grouped per unit of consecutive blocks in LDS.
    bool direct = false;
    uint32_t items_g = 0;
};

struct SubPlan {
    uint32_t interval;
    uint32_t klo, khi, s, nb;
    uint32_t unit_begin = 0, unit_end = 0;   // its block-local units in rv_kernel::units
};

struct ChunkPlan {
    uint32_t sub_begin, sub_end;
    uint64_t items, buckets, records_bound;
    // the same passes with block-local spaces on chip: HBM work items and
    // buckets, and the chunk's units in rv_kernel::units
    uint64_t items_d = 0, buckets_d = 0;
    uint32_t unit_begin = 0, unit_end = 0;
};

struct WorkspaceLayout {
    size_t cap_records = 0;        // records per chunk
    size_t cap_buckets = 0;        // buckets per chunk
    size_t off_counts = 0, off_starts = 0, off_cursor = 0, off_conf = 0, off_bsum = 0;
    // hot buckets (more than HOT records): their list, its length, a
    // completion counter and a four-table location summary per entry
    size_t cap_hot = 0;
    size_t off_hot_n = 0, off_hot_list = 0, off_hot_sub = 0, off_hot_tab = 0;
    // medium buckets (one fold slice < records <= HOT): their list and length
    size_t cap_mid = 0;
    size_t off_mid_n = 0, off_mid_list = 0, off_mid_sub = 0;
    size_t bytes = 0;
};

}  // namespace rv

// The opaque handles of rv.h.
struct rv_kernel {
    // copied description
    rv_launch launch{};
    std::vector<rv_array> arrays;
    std::vector<rv_access> accesses;
    std::vector<rv_guard> guards;
    std::vector<rv_phase> phases;
    std::vector<rv_segment> segments;
    // schedule
    std::vector<uint32_t> dyn_phase;
    std::vector<int32_t> dyn_k;
    std::vector<uint32_t> dyn_interval;
    uint32_t n_intervals = 0;      // barrier intervals (strict semantics plan one more space after them)
    int semantics = RV_SEM_INTERVAL;
    bool has_subkeys = false;      // some pass has sub-keys (judged by the fold kernels)
    // plan
    rv::DevKernel kc{};
    std::vector<rv::DevEntry> entries;
    std::vector<rv::HostEntry> hentries;
    std::vector<int32_t> guard_rows;
    std::vector<uint32_t> entry_items;
    std::vector<uint32_t> entry_items_g;   // the same prefixes with the shared entries of direct intervals empty
    std::vector<rv::IntervalPlan> intervals;
    std::vector<rv::SubPlan> subs;
    std::vector<rv::ChunkPlan> chunks;
    uint64_t n_instances = 0;
    uint64_t max_interval_instances = 0;
    uint64_t n_buckets = 0;
    int target = rv::DEFAULT_TARGET;
    // guarded barriers (divergence check) and the number of barrier instances
    std::vector<rv::DevBarrier> barriers;
    uint64_t barrier_instances = 0;
    // device copies
    void *d_mem = nullptr;
    rv::DevBarrier *d_barriers = nullptr;
    rv::DevKernel *d_kc = nullptr;
    rv::DevEntry *d_entries = nullptr;
    int32_t *d_guards = nullptr;
    uint32_t *d_entry_items = nullptr;
    uint32_t *d_entry_items_g = nullptr;
    rv::DevSub *d_subs = nullptr;   // all passes, begins relative to this kernel's own chunks
    std::vector<rv::DevSub> h_subs;
    // block-local spaces on chip: the passes with shared entries left out of
    // the HBM pipeline, and the units of each chunk
    std::vector<rv::DevUnit> units;
    std::vector<rv::DevSub> h_subs_dir;   // the passes as the HBM pipeline sees them with units on
    rv::DevSub *d_subs_dir = nullptr;
    rv::DevUnit *d_units = nullptr;
    uint32_t max_chunk_units = 0;
    size_t plan_cap_records = 0;     // the workspace layout `chunks` was planned for
    size_t plan_cap_buckets = 0;
    // the same passes chunked for the static scratch of rv_check_static
    std::vector<rv::ChunkPlan> chunks_static;
    rv::DevSub *d_subs_static = nullptr;
    bool static_ok = false;
    std::string static_msg;          // why static_ok is false
    rv_ctx *owner = nullptr;
    uint64_t serial = 0;             // unique per load in the process (batch table cache key)
};

namespace rv {

// plan.cpp
rv_status validate(const rv_kernel_desc *d, std::string &msg);
rv_status plan_kernel(const rv_kernel_desc *d, int target, rv_kernel &k, std::string &msg,
                      int semantics = RV_SEM_INTERVAL);
WorkspaceLayout layout_workspace(size_t bytes);
rv_status plan_chunks(rv_kernel &k, const WorkspaceLayout &L, std::string &msg);
// Append DevSub entries for passes [sb, se) of k.  Item and bucket begins
// continue from *items / *buckets (relative to the chunk); pass i gets result
// slot res0 + (i - sb).
// direct: block-local spaces of direct intervals are checked on chip (their
// shared entries get no work items, their buckets start after the shared
// locations).
void make_devsubs(const rv_kernel &k, uint32_t sb, uint32_t se, uint32_t res0,
                  std::vector<DevSub> &out, uint64_t &items, uint64_t &buckets, bool direct = false);
// Units of the block-local spaces of k's chunks (main workspace layout):
// fills k.units and each chunk's unit range, HBM items and buckets.
void plan_units(rv_kernel &k);
// Decode helpers (host)
void decode_instance(const rv_kernel &k, uint32_t interval, uint32_t id, rv_side &side,
                     uint32_t &gthread, uint32_t &lidx);
void decode_location(const rv_kernel &k, uint32_t interval, uint32_t loc, int32_t &space,
                     int32_t &array, uint32_t &block, int64_t &address);

// kernels.hip launchers (all asynchronous on `st`)
struct Timer;
void launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t st);
void launch_init_results(SubResult *r, size_t n, hipStream_t st);
void launch_hist(const DevSub *subs, uint32_t nsub, uint64_t items, uint32_t *counts, SubResult *res,
                 unsigned ncu, hipStream_t st);
void launch_scan(const uint32_t *in, uint32_t *starts, uint32_t *cursor, uint32_t *bsum, size_t n,
                 hipStream_t st);
void launch_scatter(const DevSub *subs, uint32_t nsub, uint64_t items, unsigned long long *rec,
                    uint32_t *cursor, unsigned ncu, hipStream_t st);
void launch_bucket(const DevSub *subs, uint32_t nsub, uint64_t nbuckets, unsigned long long *rec,
                   const uint32_t *starts, const uint32_t *counts, uint32_t *conf, int debug_sorted,
                   unsigned ncu, hipStream_t st);
struct HotArea {
    uint32_t *n, *list, *sub, *tab;     // hot buckets: count, bucket, its pass, merged summaries
    uint32_t cap;
    uint32_t *mid_n, *mid_list, *mid_sub;
    uint32_t mid_cap;
};
void launch_fold(const DevSub *subs, uint32_t nsub, uint64_t nbuckets, unsigned long long *rec,
                 const uint32_t *starts, const uint32_t *counts, uint32_t *conf, HotArea hot, SubResult *res,
                 unsigned ncu, hipStream_t st);
void launch_finish(const DevSub *subs, uint32_t nsub, uint64_t nbuckets, const uint32_t *conf,
                   SubResult *res, hipStream_t st);
void launch_first(const DevSub *subs, uint32_t nsub, const unsigned long long *rec,
                  const uint32_t *starts, const uint32_t *uwit, SubResult *res, hipStream_t st);
// On-chip check of block-local units[0..n) of a chunk (pass table subs):
// records, conflicts and out-of-bounds instances into the passes' slots,
// each unit's first witness into uwit[4 * unit].
void launch_direct(const DevSub *subs, const DevUnit *units, uint32_t n, SubResult *res, uint32_t *uwit,
                   unsigned ncu, hipStream_t st);
void launch_gather(const DevSub *subs, uint32_t nsub, uint64_t nbuckets, const unsigned long long *rec,
                   const uint32_t *starts, const uint32_t *conf, const uint32_t *wpos,
                   unsigned long long base, unsigned long long lo, unsigned long long hi,
                   DevWitness *out, hipStream_t st);
size_t scan_bsum_words(size_t n);
// Exact per-location counts of a chunk's buckets (after the expansion):
// pairs (ordered = 0) or dependences (ordered = 1) into out[pass result slot];
// tmp holds the chunk's records again (buckets above one LDS tile sort there).
void launch_counts(const DevSub *subs, uint32_t nsub, uint64_t nbuckets, unsigned long long *rec,
                   unsigned long long *tmp, const uint32_t *starts, const uint32_t *counts, int ordered,
                   PassCounts *out, unsigned ncu, hipStream_t st);
void launch_init_counts(PassCounts *p, size_t n, hipStream_t st);
// On-chip check of n small passes subs[0..n) (each at most SMALL_CAP instances).
void launch_small(const DevSub *subs, uint32_t n, SubResult *res, unsigned ncu, hipStream_t st);
// Divergence of the guarded barriers bars[0..n): res[0..n) receives the
// divergent scope instances of each (its first instance included).
void launch_barriers(const DevBarrier *bars, uint32_t n, const DevKernel *kc, const int32_t *guards,
                     uint32_t nblocks, BarrierResult *res, unsigned ncu, hipStream_t st);
constexpr uint32_t BARRIER_MAX_TPB = 4096;   // threads per block the divergence check handles

// The device scratch of rv_check_static (kernels.hip): its address on
// `device` is looked up once, with that device current (rv_ctx_create), and
// kept; static_scratch returns it, or null before a successful lookup.
hipError_t static_scratch_init(int device);
void *static_scratch(int device);
// Static scratch layout: RV_STATIC_MAX_PASSES result slots, then a workspace.
constexpr size_t STATIC_RES_BYTES = ((size_t)RV_STATIC_MAX_PASSES * sizeof(SubResult) + 255) & ~(size_t)255;

}  // namespace rv
