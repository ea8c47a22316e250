/*
 * rv.h -- C ABI of librv, a per-barrier-interval SIMT data-race checker for
 * AMD Instinct MI355X (gfx950).
 *
 * The operation (arXiv 2503.08946):
 *   The paper models a GPU kernel as integer sets: a Domain of statement
 *   instances, Read and Write access relations from instances to array
 *   elements, and a Schedule that orders the instances (Section 2.1, steps
 *   1-5; Appendix listings).  Its check intersects the read/write relations
 *   with the happens-before order to find RaW, WaW and WaR pairs (Section 2.1
 *   step 6).  A data race is one thread writing data another thread still
 *   uses (Abstract; Section 1).
 *
 *   librv evaluates that model concretely for a SIMT launch.  For every
 *   barrier interval (the accesses of a block between two barriers) it
 *   expands each thread's accesses into records (location, instance id,
 *   read/write) and reports every location that two different threads touch
 *   in the same interval with at least one write, with a canonical witness
 *   pair.  Records are grouped by location with a radix sort and reduced by
 *   a segmented scan on the GPU; nothing runs on the CPU but planning.
 *
 * Conventions
 *   - Every function returns rv_status: RV_OK (0) or a negative code; on an
 *     error, outputs are left untouched and rv_last_error(ctx) holds a
 *     message.  Nothing throws across this interface.
 *   - A context belongs to one device and one HIP stream.  Calls on one
 *     context must be serialised by the caller; several contexts may share a
 *     device.
 *   - Pointers in rv_kernel_desc are host memory owned by the caller and are
 *     copied by rv_load_kernel_desc.  The workspace passed to rv_ctx_create
 *     is device memory owned by the caller and must outlive the context.
 *   - The library allocates small device tables of its own (per kernel: the
 *     plan; per context: result slots) with hipMalloc.
 */
#ifndef RV_H
#define RV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rv_status;
enum {
    RV_OK = 0,
    RV_ERR_INVALID = -1,      /* malformed description or argument */
    RV_ERR_UNSUPPORTED = -2,  /* launch z-dimension > 1, or a feature outside this interface */
    RV_ERR_KEY_BITS = -3,     /* an interval's location space does not fit 31 bits */
    RV_ERR_RANGE = -4,        /* an affine value may leave int32 over the iteration box */
    RV_ERR_OOB = -5,          /* an element index left [0, dim) (found on the GPU) */
    RV_ERR_TOO_LARGE = -6,    /* >= 2^32 instances in one interval, or workspace too small */
    RV_ERR_BUDGET = -7,       /* a job exceeds a server's memory budget */
    RV_ERR_DEVICE = -8,       /* a HIP call failed (message carried) */
    RV_ERR_STATE = -9         /* call not valid in the object's current state */
};

/* Variables an affine form ranges over. */
enum {
    RV_V_TX = 0, RV_V_TY, RV_V_BX, RV_V_BY,   /* threadIdx.x/y, blockIdx.x/y */
    RV_V_K,                                   /* repetition variable of the enclosing segment */
    RV_V_L0, RV_V_L1, RV_V_L2,                /* the access's loop variables */
    RV_V_AUX0, RV_V_AUX1,                     /* auxiliary floor-div / mod terms */
    RV_NV
};
enum { RV_SHARED = 0, RV_GLOBAL = 1 };
enum { RV_AUX_NONE = 0, RV_AUX_FLOORDIV = 1, RV_AUX_EMOD = 2 };

/* ----------------------------------------------------------- description
 * The concrete counterpart of the paper's Domain / Read / Write / Schedule
 * (Section 2.1 steps 2-5; Section 2 lists what must be recovered from a
 * kernel: thread and block ids, barriers, shared allocations, indices into
 * arrays, reads and writes).
 */
typedef struct { int32_t block[3]; int32_t grid[3]; } rv_launch;     /* [2] must be 1 */

/* An array is a set of elements addressed by a row-major index; arrays never
 * alias (Section 1: each variable is an array, a set of its index values). */
typedef struct {
    int32_t space;            /* RV_SHARED: one copy per block; RV_GLOBAL: one per launch */
    int32_t ndim;             /* 1..3 */
    int64_t dim[3];           /* extents >= 1; product < 2^31 */
} rv_array;

typedef struct { int32_t coef[RV_NV]; int32_t c0; } rv_affine;   /* value = c0 + sum coef[v]*v */

/* aux = floor(e / d) or the Euclidean e mod d (result in [0, d)); e may not
 * use RV_V_AUX0/1 (Presburger quasi-affine terms, as in the paper's j % 32). */
typedef struct { int32_t kind; int32_t d; rv_affine e; } rv_aux;

/* One array access per point of the loop box [lo, hi) (nloops <= 3),
 * executed when every guard is >= 0 (a conjunction of affine constraints,
 * the paper's Domain restrictions).  idx[d] is the index along dim d. */
typedef struct {
    int32_t array;
    int32_t is_write;
    int32_t nloops;
    int32_t loop_lo[3], loop_hi[3];
    rv_aux aux[2];
    rv_affine idx[3];
    int32_t guard_begin, guard_count;        /* range in rv_kernel_desc.guards */
} rv_access;

typedef struct { rv_affine g; } rv_guard;   /* holds iff g >= 0 */

/* A run of accesses ("code section") that may end with a barrier
 * (Section 2, component (4)): RV_BARRIER_BLOCK orders every thread of the
 * block (__syncthreads); RV_BARRIER_WARP orders the threads of one warp
 * (__syncwarp over the whole warp: the warp-level synchronisation of
 * coarse-grained warp merging, Section 1.1.4).  guard_begin / guard_count
 * (a range in rv_kernel_desc.guards; affine in tx, ty, bx, by, k only) name
 * the threads that reach the barrier: they feed the divergence check
 * (rv_check_barriers); the race check treats every barrier as reached by
 * all threads of its scope. */
enum { RV_BARRIER_NONE = 0, RV_BARRIER_BLOCK = 1, RV_BARRIER_WARP = 2 };
typedef struct { int32_t access_begin, access_count, barrier_after, guard_begin, guard_count; } rv_phase;

/* A run of phases executed repeat times; RV_V_K = k_base + repetition.  The
 * order of segments, repetitions and phases is the schedule. */
typedef struct { int32_t phase_begin, phase_count, repeat, k_base; } rv_segment;

typedef struct {
    rv_launch launch;
    const rv_array *arrays;     int32_t n_arrays;
    const rv_access *accesses;  int32_t n_accesses;
    const rv_guard *guards;     int32_t n_guards;
    const rv_phase *phases;     int32_t n_phases;
    const rv_segment *segments; int32_t n_segments;
    int32_t warp_size;          /* threads per warp: consecutive linear thread ids of a block (0: 32) */
} rv_kernel_desc;

/* ---------------------------------------------------------------- results */
/* One side of a witness: which instance made the access.  loop[] holds the
 * loop variables' values (0 for unused loops). */
typedef struct {
    uint32_t block;        /* blockIdx.y * gridDim.x + blockIdx.x */
    uint32_t tid;          /* threadIdx.y * blockDim.x + threadIdx.x */
    uint32_t dyn_phase;    /* index of the executed phase (segments x repeats x phases, in order) */
    uint32_t access;       /* index into rv_kernel_desc.accesses */
    int32_t loop[3];
    int32_t is_write;
} rv_side;

/* A conflicting location and its canonical pair: `first` is the write with
 * the smallest instance id; `second` is the smallest-id record of the
 * location when its thread differs from first's, else the largest-id record.
 * Instance ids order by (global thread, dynamic phase, access, loop index). */
typedef struct {
    uint32_t interval;     /* barrier interval (barriers executed before the access) */
    int32_t space;         /* RV_SHARED / RV_GLOBAL */
    int32_t array;
    uint32_t block;        /* the block owning the shared copy; 0 for global arrays */
    int64_t address;       /* row-major element index */
    rv_side first, second;
} rv_witness;

typedef struct {
    uint64_t n_records;    /* records emitted (instances whose guards hold) */
    uint64_t n_conflicts;  /* conflicting locations */
    int32_t has_witness;
    int32_t reserved;
    rv_witness witness;    /* the smallest conflicting location in (interval, space, block, array, address) order */
} rv_result;

/* Per-stage GPU time, accumulated while timing is enabled (HIP events on the
 * context's stream around each launch). */
enum { RV_STAGE_FILL = 0, RV_STAGE_COUNT, RV_STAGE_SCAN, RV_STAGE_EXPAND, RV_STAGE_SORT_SCAN,
       RV_STAGE_FINISH, RV_STAGE_SMALL /* batched passes checked on chip */,
       RV_STAGE_DIRECT /* block-local units checked on chip */, RV_NSTAGE };
typedef struct {
    double ms[RV_NSTAGE];
    uint64_t launches[RV_NSTAGE];
    uint64_t small_records;   /* records of the batched passes checked on chip (RV_STAGE_SMALL) */
    uint64_t direct_records;  /* records of block-local units checked on chip (RV_STAGE_DIRECT) */
    uint64_t counted_records; /* records of passes without writes (no location there can conflict):
                                 counted by RV_STAGE_COUNT, never placed or grouped */
} rv_timing;

/* Static facts about a loaded kernel. */
typedef struct {
    uint64_t n_instances;      /* thread x access x loop-point instances before guards */
    uint32_t n_intervals;
    uint32_t n_subintervals;   /* key-range passes (an interval with a large location space gets several) */
    uint32_t n_chunks;         /* workspace-sized groups of passes */
    uint32_t n_buckets;        /* location buckets over all passes */
    uint64_t max_interval_instances;
    uint32_t n_entries;        /* (interval, dynamic phase, access) expansion entries */
    uint32_t n_flat_entries;   /* of which expanded with loop chunks across lanes (few threads) */
    uint32_t n_linear_entries; /* of which each lane's records in a work item are affine in the
                                  slot: one thread's consecutive innermost-loop points, or one
                                  instance each of consecutive threads differing in tx alone
                                  (ranked per lane or per run, not per record, when they can be) */
    uint32_t n_fast_entries;   /* entries with neither aux terms nor guards (affine indices) */
    uint32_t n_proven_entries; /* entries whose every index is proven inside its dimension (no
                                  per-record bounds test): fast ones by the exact index range
                                  over the launch and the loop box (a fast entry that is not
                                  proven has an out-of-bounds instance), and entries with aux
                                  terms and no guards by the value ranges of the variables and
                                  of the aux terms (n mod d in [0, d)) */
    uint32_t n_direct_intervals; /* intervals whose block-local (shared-array) locations are
                                  grouped on chip, a unit of blocks per LDS table, when
                                  rv_check runs with the tuning's `direct` on */
} rv_kernel_info;

/* A decoded record (debugging and expansion-parity tests). */
typedef struct {
    uint32_t interval;
    int32_t space;
    uint32_t block;        /* owning block if shared, else 0 */
    int32_t array;
    int64_t address;
    uint32_t gthread, dyn_phase, access, lidx;   /* instance id (lidx: row-major loop index) */
    int32_t loop[3];
    int32_t is_write;
} rv_record;

/* One finished job of a server.  Times are the host's steady clock in ns:
 * submission, the launch of the batch that carried the job, and the moment
 * the server saw that batch's results on the host. */
typedef struct {
    uint64_t job_id;
    int32_t status;        /* as rv_check would return for the kernel */
    int32_t reserved;
    rv_result result;      /* valid when status == RV_OK */
    uint64_t t_submit_ns, t_start_ns, t_done_ns;
} rv_job_result;

/* Counters of a server since its creation. */
typedef struct {
    uint64_t batches;             /* batched checks launched */
    uint64_t jobs;                /* jobs launched */
    uint64_t max_batch_jobs;      /* largest batch */
    uint64_t overlapped_batches;  /* batches launched while the other lane was still running */
} rv_server_stats;

typedef struct rv_ctx rv_ctx;
typedef struct rv_kernel rv_kernel;
typedef struct rv_server rv_server;

/* ------------------------------------------------------------- functions */

/* Check a description on the host only (no device).  Returns RV_OK or the
 * code rv_load_kernel_desc would return for a malformed / unsupported /
 * out-of-range description; a message is written to msg (cap bytes, always
 * NUL-terminated when cap > 0). */
rv_status rv_validate_desc(const rv_kernel_desc *desc, char *msg, size_t cap);

/* Plan a description on the host only (no device): the figures
 * rv_kernel_get_info would report for it after rv_load_kernel_desc, with
 * n_chunks = 0 (chunks depend on a context's workspace).  `target` is the
 * planner's mean records per bucket (0: the default).  Returns the code
 * rv_load_kernel_desc would return; on an error *out is untouched and msg
 * (cap bytes, NUL-terminated when cap > 0) says why. */
rv_status rv_plan_desc(const rv_kernel_desc *desc, int32_t target, rv_kernel_info *out, char *msg, size_t cap);

/* Create a context on `device` (hipSetDevice numbering) issuing work on
 * `hip_stream` (a hipStream_t; NULL = the null stream).  `workspace` is
 * device memory of `workspace_bytes` (>= 64 MiB) holding the records of one
 * chunk; larger workspaces allow larger chunks (fewer passes). */
rv_status rv_ctx_create(rv_ctx **out, int device, void *hip_stream, void *workspace,
                        size_t workspace_bytes);
rv_status rv_ctx_destroy(rv_ctx *ctx);
/* Message of the last failing call on ctx ("" if none).  Owned by ctx. */
const char *rv_last_error(const rv_ctx *ctx);

/* Load a kernel description: the paper's Domain, Read/Write relations and
 * Schedule of one kernel (Section 2.1, steps 1-5; the component list of
 * Section 2), given as host structures.  The description is validated,
 * its schedule expanded into dynamic phases and barrier intervals, each
 * interval's location space laid out, and the plan tables uploaded to the
 * context's device (hipMalloc, synchronous copy).  The description is
 * deep-copied: the caller may free it on return.  *out is owned by the
 * library until rv_free_kernel.  Errors: RV_ERR_INVALID (malformed),
 * RV_ERR_UNSUPPORTED (z > 1), RV_ERR_KEY_BITS, RV_ERR_RANGE (a value may
 * leave int32), RV_ERR_TOO_LARGE (an interval of >= 2^32 instances, or one
 * the context's workspace cannot hold), RV_ERR_DEVICE. */
rv_status rv_load_kernel_desc(rv_ctx *ctx, const rv_kernel_desc *desc, rv_kernel **out);

/* Which race a loaded kernel is checked for.
 *  RV_SEM_INTERVAL (rv_load_kernel_desc): two records of one location
 *    conflict when they come from different threads, one writes, and
 *    nothing orders them: they are in the same barrier interval, and not in
 *    the same warp on either side of a warp barrier.  Records of global
 *    arrays from different blocks are compared within one interval index.
 *  RV_SEM_STRICT: no barrier orders two blocks (Abstract; Section 1: a race
 *    is one thread overwriting data another still uses), so records of a
 *    global array from different blocks conflict across intervals; within
 *    one block the intervals still order them.  Shared arrays are checked
 *    per interval as above.  Witnesses of global locations follow every
 *    shared one, in (array, address) order; their interval is the first
 *    side's.  Kernels with warp barriers are RV_ERR_UNSUPPORTED here.
 * The canonical witness of a conflicting location is that of rv_witness
 * taken inside the smallest sub-interval (fine interval between warp
 * barriers; interval, in strict mode for global arrays) holding a
 * conflict; when only records of different units (warps; blocks) conflict,
 * `second` is the smallest-id record if its unit differs from first's, else
 * the largest-id record. */
/*  RV_SEM_ORDERED: the check of Section 2.1 step 6 on a sequential schedule
 *    (the appendix listings' Before = Schedule << Schedule): dynamic phases
 *    run one after another, inside one the threads in global-thread order,
 *    each walking its loop points in row-major order; the accesses of one
 *    phase at one (thread, loop index) form one statement instance.
 *    Barriers play no part.  Such a kernel is checked with
 *    rv_check_counts only (RaW, WaW, WaR; rv_check: RV_ERR_STATE).  The
 *    instance ids of all phases share 32 bits (RV_ERR_TOO_LARGE beyond). */
enum { RV_SEM_INTERVAL = 0, RV_SEM_STRICT = 1, RV_SEM_ORDERED = 2 };
typedef struct {
    int32_t semantics;       /* RV_SEM_* */
    int32_t reserved[3];     /* 0 */
} rv_load_options;
/* rv_load_kernel_desc with options (NULL: the defaults).  Errors as
 * rv_load_kernel_desc, and RV_ERR_UNSUPPORTED for a combination this build
 * does not check, RV_ERR_INVALID for unknown options. */
rv_status rv_load_kernel_desc_ex(rv_ctx *ctx, const rv_kernel_desc *desc, const rv_load_options *opt,
                                 rv_kernel **out);
rv_status rv_free_kernel(rv_ctx *ctx, rv_kernel *k);
rv_status rv_kernel_get_info(rv_ctx *ctx, const rv_kernel *k, rv_kernel_info *out);

/* The race check of one loaded kernel: every instance of every barrier
 * interval is expanded into a record (the access relations restricted to
 * the Domain, Section 2.1 steps 3-4), records are grouped by location and
 * every location touched by two different threads in one interval with at
 * least one write is counted (the unordered counterpart of the RaW, WaW
 * and WaR relations of Section 2.1 step 6; a race in the sense of the
 * Abstract and Section 1).  *out (host) receives the record and conflict
 * counts and the witness of the smallest conflicting location.  Work runs
 * on the context's stream and workspace; the call blocks until the result
 * is on the host (one stream sync).  A kernel with no records gives
 * n_conflicts = 0 and has_witness = 0.  Errors: RV_ERR_OOB (rv_last_error
 * names the smallest out-of-bounds instance; *out untouched), RV_ERR_STATE
 * (the context is serving, or k belongs to another context), RV_ERR_DEVICE. */
rv_status rv_check(rv_ctx *ctx, rv_kernel *k, rv_result *out);

/* The check of Section 2.1 step 6 (as rv_check) for n loaded kernels at
 * once: ks[0..n) (host array of handles of this context), out[0..n) (host
 * results).  Their intervals share the same launches; out[i] is
 * bit-identical to rv_check(ks[i]).  Returns the first error (its message
 * names the kernel); kernels before it have valid results. */
rv_status rv_check_batch(rv_ctx *ctx, rv_kernel *const *ks, size_t n, rv_result *out);

/* The conflicting locations themselves, each with its canonical pair of
 * instances: the concrete elements of the paper's dependence relations
 * (Section 2.1 step 6; the appendix listings print whole relations).
 * Writes the witnesses with list index in [first_index, first_index + cap)
 * to out (host, cap entries), in (interval, space, block, array, address)
 * order; *n_out = number written.  Re-runs the check in collect mode (the
 * result is deterministic, so windows are consistent); the window buffer on
 * the device is kept by the context between calls.  Errors as rv_check. */
rv_status rv_get_witnesses(rv_ctx *ctx, rv_kernel *k, uint64_t first_index, rv_witness *out,
                           size_t cap, size_t *n_out);

/* For callers that cannot allocate device memory while they check: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The same check as rv_check (same kernels, bit-identical
 * result), but its scratch -- the records of one chunk, the per-bucket
 * arrays, the hot-bucket lists and the per-pass result slots -- lives in a
 * library-owned device array of RV_STATIC_SCRATCH_BYTES, one per device,
 * held from the first rv_ctx_create on that device until the process ends;
 * the context's workspace is not used.  The kernel's pass table for that
 * array is built and uploaded by rv_load_kernel_desc, so this call makes no
 * allocation of any kind: it launches the kernels on the context's stream,
 * copies the per-pass results into a fixed host buffer of its own and
 * waits on the stream.  Every call on one device shares that device's
 * array, which keeps the last call's contents (each call clears what it
 * needs): calls that overlap on one device -- from different threads, or
 * from contexts on different streams -- race, and the caller must serialise
 * them.  Errors: RV_ERR_TOO_LARGE when one of k's passes needs more records
 * or buckets than the array holds, or k has more than RV_STATIC_MAX_PASSES
 * passes (rv_last_error gives the sizes); RV_ERR_DEVICE if the array's
 * address could not be obtained at context creation; otherwise as rv_check. */
#define RV_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
#define RV_STATIC_MAX_PASSES 8192
rv_status rv_check_static(rv_ctx *ctx, rv_kernel *k, rv_result *out);

/* Exact pair and dependence counts.  For a kernel loaded with interval
 * semantics and no warp barriers: n_pairs = the unordered pairs of
 * different threads that touch one location in one barrier interval, at
 * least one of them writing it, summed over (interval, location) -- the
 * distinct-thread pairs behind n_conflicts.  For a kernel loaded with
 * RV_SEM_ORDERED: the dependence relations of Section 2.1 step 6 (RaW =
 * (Write . Read^-1) * Before, WaW, WaR, with Before = earlier on the
 * sequential schedule) counted as (earlier instance, element, later
 * instance) triples, and the elements holding at least one of them.  Each
 * bucket's records are ordered on the GPU by (location, thread) or
 * (location, time) -- an LDS sort, or a radix sort in global memory for
 * buckets above 4096 records -- and scanned.  Errors: RV_ERR_UNSUPPORTED for
 * strict semantics or a kernel with warp barriers; otherwise as rv_check
 * (out of bounds: the message names an out-of-bounds instance). */
typedef struct {
    uint64_t n_records;
    uint64_t n_conflicts;        /* interval semantics: as rv_check; ordered: 0 */
    uint64_t n_pairs;            /* interval semantics */
    uint64_t n_raw, n_waw, n_war, n_dep_locations;   /* ordered semantics */
} rv_counts;
rv_status rv_check_counts(rv_ctx *ctx, rv_kernel *k, rv_counts *out);

/* Barrier divergence (Section 2, component (4): barriers; Section 1.1.4:
 * warp-level synchronisation).  A barrier whose rv_phase carries guards is
 * reached by the threads for which every guard is >= 0.  One instance of a
 * block barrier is (dynamic phase, block); of a warp barrier, (dynamic
 * phase, block, warp).  An instance is divergent when some but not all of
 * its threads reach it (undefined behaviour in CUDA).  The race check
 * itself treats every barrier as reached by all threads of its scope. */
typedef struct {
    uint64_t n_instances;    /* barrier instances of the kernel (guarded or not) */
    uint64_t n_divergent;    /* divergent instances */
    int32_t has_divergence;  /* the fields below describe the first divergent instance in
                                (dynamic phase, block, warp) order */
    uint32_t dyn_phase;      /* the phase the barrier ends */
    uint32_t block;
    int32_t warp;            /* -1 for a block barrier */
    uint32_t arrive_tid;     /* its smallest thread (linear id in the block) that reaches the barrier */
    uint32_t skip_tid;       /* its smallest thread that does not */
} rv_barrier_result;
/* Evaluate every guarded barrier of a loaded kernel on the GPU (one
 * workgroup per barrier and block) and report divergence into *out (host).
 * Blocks of more than 4096 threads: RV_ERR_UNSUPPORTED.  Errors as rv_check. */
rv_status rv_check_barriers(rv_ctx *ctx, rv_kernel *k, rv_barrier_result *out);

/* Records of one barrier interval as the expansion wrote them (sorted = 0)
 * or after the per-bucket sort (sorted = 1: location order; requires every
 * bucket to fit one on-chip slice, else RV_ERR_UNSUPPORTED).  *n_out is the
 * number of records; at most cap are written. */
rv_status rv_debug_records(rv_ctx *ctx, rv_kernel *k, uint32_t interval, int sorted,
                           rv_record *out, size_t cap, size_t *n_out);

/* Per-stage GPU timing (HIP events around each launch; adds one event pair
 * per launch).  enable = 0 stops timing; rv_get_timing copies and, if
 * reset != 0, clears the accumulators. */
rv_status rv_set_timing(rv_ctx *ctx, int enable);
rv_status rv_get_timing(rv_ctx *ctx, rv_timing *out, int reset);

/* ---------------------------------------------------------------- tuning
 * Three free parameters, none of which changes any result:
 *  - `target`, the planner's mean number of records per location bucket: it
 *    sets each interval's bucket width 2^s (s = floor(log2(target x
 *    locations / instances)), clamped to [0, 9]), trading the number of
 *    buckets (per-bucket overhead) against slices that overflow one on-chip
 *    tile.  It applies to kernels loaded after it is set.
 *  - `group`, the per-bucket grouping kernel: both build, per location, the
 *    summary (min id, max id, min write id, max write id) from which the
 *    conflict and its witness follow (Section 2.1 step 6 reduced to one
 *    location); FOLD reaches it with LDS atomics on per-location slots,
 *    SORT_SCAN by sorting the bucket in LDS and scanning runs of equal
 *    location.  It applies to the next checks.
 *  - `small_cap`, the batched checks' small-pass threshold: in
 *    rv_check_batch (and a server's batches) a pass of at most small_cap
 *    instances (at most 2048; 0 turns the path off) is checked entirely on
 *    chip by one workgroup -- its records folded into an LDS hash table of
 *    per-location summaries, then judged -- instead of going through the
 *    record buffer in HBM and the bucket kernels.  Passes whose interval has warp barriers never take it.
 *  - `direct`, block-local spaces on chip: shared arrays are allocated per
 *    block (Section 2, component 5), so in a barrier interval a block's
 *    shared locations are touched by its own threads only.  With `direct`
 *    on, rv_check groups them per unit of consecutive blocks whose shared
 *    locations (at most 2048) fit one LDS table -- the unit's threads'
 *    records expanded and folded into per-location summaries on chip, then
 *    judged -- and only global-array records go through the record buffer
 *    in HBM.  Intervals with warp barriers, and intervals whose blocks hold
 *    more than 2048 shared elements, keep the HBM path.  With `direct` on,
 *    a pass whose HBM-side accesses are all reads is only counted (its
 *    records and out-of-bounds instances): without a write no location
 *    conflicts (Section 2.1 step 6: RaW, WaW and WaR all need a write).
 *    rv_get_witnesses, rv_check_counts and rv_check_static do not use it. */
enum {
    RV_GROUP_FOLD = 0,       /* fold records into per-location LDS tables with atomics (default) */
    RV_GROUP_SORT_SCAN = 1   /* LDS counting sort of each bucket + DPP segmented scan */
};
typedef struct {
    int32_t target;          /* mean records per bucket, in [64, 4096]; default 2048 */
    int32_t group;           /* RV_GROUP_*: how a bucket's records are grouped by location */
    int32_t n_candidates;    /* rv_autotune: candidates measured */
    int32_t small_cap;       /* batched small-pass threshold in [0, 2048]; default 2048 */
    int32_t direct;          /* 1 (default): rv_check groups block-local locations on chip; 0: every
                                record goes through the HBM pipeline */
    int32_t reserved;        /* 0 */
    int32_t candidates[8];   /* rv_autotune: target of each candidate */
    int32_t cand_group[8];   /* rv_autotune: grouping of each candidate */
    int32_t cand_small[8];   /* rv_autotune: small-pass threshold of each candidate */
    double ms[8];            /* rv_autotune: median wall time of one batched check per candidate */
} rv_tuning;
rv_status rv_ctx_get_tuning(rv_ctx *ctx, rv_tuning *out);
rv_status rv_ctx_set_tuning(rv_ctx *ctx, const rv_tuning *t);   /* reads target, group, small_cap and direct */
/* Measure a batched check of descs[0..n) (host memory, as rv_load_kernel_desc
 * takes them) under each candidate (target in {1024, 2048}, group, small_cap
 * in {0, 2048}), `trials` timed runs after one
 * warm-up each (host wall time from launch to results on the host, median),
 * keep the fastest in the context and report all of them in *out.  A
 * description that fails to load or check fails the call with its code. */
rv_status rv_autotune(rv_ctx *ctx, const rv_kernel_desc *descs, size_t n, int32_t trials, rv_tuning *out);

/* ------------------------------------------------------------- serving
 * A server checks a stream of submitted kernels with continuous batching:
 * the caller's device memory of `budget_bytes` (>= 128 MiB) is split into
 * two lanes, each with a HIP stream of its own (default priority); a worker
 * thread gives every idle lane the waiting jobs in arrival order while their
 * records (instance upper bounds) fit the lane's half of the budget and
 * max_batch_records (0: no limit; a job larger than the limit runs alone),
 * and launches them as one batched check (as rv_check_batch).  The limit
 * bounds how long one batch holds its jobs: a job's latency is that of its
 * batch.  Jobs that arrive while both lanes are
 * busy join the next batch, so one lane's batch runs while the next one is
 * admitted and launched.  Each job's result is bit-identical to rv_check of
 * its kernel alone.
 *
 * While a server exists its context accepts no rv_check / rv_check_batch /
 * rv_get_witnesses / rv_debug_records (RV_ERR_STATE), timing is not
 * collected for server work, and submitted kernels must stay loaded until
 * their results have been polled.  submit, poll and drain may be called from
 * any host thread. */
rv_status rv_server_create(rv_ctx *ctx, void *workspace, size_t budget_bytes, uint64_t max_batch_records,
                           rv_server **out);
/* Finishes the jobs already submitted, stops the worker and frees the
 * server's streams and tables (not the workspace). */
rv_status rv_server_destroy(rv_server *s);
/* Queue k; non-blocking.  RV_ERR_BUDGET if one of k's passes cannot fit a
 * lane's half of the budget (such a job would never be admitted). */
rv_status rv_server_submit(rv_server *s, rv_kernel *k, uint64_t *job_id);
/* Move up to cap finished jobs (completion order) into out; *n_out = count. */
rv_status rv_server_poll(rv_server *s, rv_job_result *out, size_t cap, size_t *n_out);
/* Wait until every submitted job has finished (RV_ERR_STATE on timeout). */
rv_status rv_server_drain(rv_server *s, uint64_t timeout_ms);
rv_status rv_server_get_stats(rv_server *s, rv_server_stats *out);

/* Host-side self test of the library's integer helpers (division by
 * invariant integers, key layout); returns RV_OK or RV_ERR_STATE with a
 * message in msg. */
rv_status rv_selftest(char *msg, size_t cap);

#ifdef __cplusplus
}
#endif
#endif /* RV_H */
