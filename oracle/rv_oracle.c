/*
 * rv_oracle.c -- TEST INFRASTRUCTURE.  A plain, slow, CPU-only statement of
 * the per-barrier-interval SIMT data-race check.  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark call it; the checker
 * library never links, loads or calls it, and it shares no code with it.
 *
 * What it computes (the definition, written out):
 *
 *  1. Dynamic phases.  Segments are walked in order; a segment is repeated
 *     `repeat` times and in repetition r its phases run with k = k_base + r.
 *     This plays the part of the paper's Schedule (Section 2.1, step 5:
 *     every code section gets a time vector; sections run in that order).
 *
 *  2. Barrier intervals.  interval(d) = number of dynamic phases e < d whose
 *     phase ends with a barrier.  Two accesses in different intervals of the
 *     same block are ordered by a barrier; two accesses in the same interval
 *     are not ordered.  (The paper's Before relation orders sections by their
 *     schedule vectors; a SIMT block only orders them across a barrier.)
 *
 *  3. Records.  For every block, every thread, every dynamic phase, every
 *     access of that phase and every point of the access's loop box, the
 *     instance is in the Domain (Section 2.1, step 2) when every guard is
 *     >= 0.  Its location is (interval, space, block if the array is shared
 *     else 0, array, row-major element index): the access relation of
 *     Section 2.1 steps 3-4 applied to one instance.  An element index
 *     outside [0, dim) is an error (the instance that is smallest in
 *     (interval, gthread, dynamic phase, access, loop index) order is
 *     reported).
 *
 *  4. Conflict.  A location conflicts when two of its records come from
 *     different threads and at least one of them is a write: the unordered
 *     counterpart of the RaW / WaW / WaR relations (Section 2.1, step 6).
 *
 *     Equivalent test used below:  anyWrite && minThread != maxThread.
 *     Proof.  (=>) a conflicting pair contains a write, and two different
 *     threads make min and max differ.  (<=) take a write record w of thread
 *     t; since minThread != maxThread at least one of them differs from t;
 *     a record of that thread together with w is a conflicting pair.
 *
 *  5. Canonical witness of a conflicting location: `first` is the write with
 *     the smallest id; `second` is the smallest-id record when its thread
 *     differs from first's thread, otherwise the largest-id record.  Ids are
 *     the tuples (gthread, dynamic phase, access, loop index) compared
 *     lexicographically, so the smallest-id record has the smallest thread
 *     and the largest-id record the largest: one of the two differs from
 *     first's thread.
 *
 *  6. Warp-scope barriers.  A phase may end with a warp barrier instead of a
 *     block barrier: it orders only the threads of one warp (warp_size
 *     consecutive linear thread ids of a block).  interval(d) counts block
 *     barriers before d; fine(d) counts barriers of either kind.  Two
 *     records of one location in the same interval are ordered exactly when
 *     they come from the same warp and different fine intervals; a conflict
 *     is an unordered pair of different threads with a write.
 *
 *     Equivalent test (records of one location and interval, sorted by id):
 *     some fine interval j holds a write and two different threads, or the
 *     location has a write and warp(minThread) != warp(maxThread).
 *     Proof.  (<=) In the first case the argument of step 4 inside j gives a
 *     pair of different threads in the same fine interval with a write:
 *     unordered.  In the second, take a write w; min and max thread lie in
 *     different warps, so one of them lies in a warp other than w's; that
 *     record and w are in different warps, hence unordered.  (=>) Let (a, b)
 *     conflict.  If a and b are in one warp they are in one fine interval j,
 *     which then holds a write and two threads.  Otherwise warp(a) !=
 *     warp(b); warp() is monotone in the thread id (block-major, then
 *     threads of a block in order), so warp(min) <= both <= warp(max) and
 *     warp(min) != warp(max).
 *     Witness: the canonical witness of step 5 taken inside the smallest
 *     such fine interval j; if there is none, first = the write with the
 *     smallest id, second = the smallest-id record when its warp differs
 *     from first's warp, else the largest-id record.  Without warp barriers
 *     fine intervals are intervals and this is step 5 unchanged.
 *
 *  7. Strict semantics (orc_check_strict).  Blocks are never ordered with
 *     each other, so records of a global array conflict across intervals
 *     when they come from different blocks; within one block the barrier
 *     intervals still order them.  Shared arrays are per block and keep the
 *     per-interval check.  A global location (array, address) conflicts iff
 *     some interval i holds a write and two different threads there, or it
 *     has a write and block(minThread) != block(maxThread) (the proof of 6
 *     with blocks for warps and intervals for fine intervals).  Witness:
 *     step 5 inside the smallest such interval, else first = the write with
 *     the smallest id, second = the smallest-id record when its block
 *     differs from first's block, else the largest-id record.  Ids compare
 *     as (gthread, dynamic phase, access, loop index) across intervals.
 *
 *  8. Ordered dependences (orc_ordered), the check of Section 2.1 step 6 on
 *     a sequential schedule: dynamic phases (the code sections) run one
 *     after another; inside one, threads run in global-thread order and each
 *     thread walks its loop points in row-major order (the time vector of a
 *     statement instance is (dynamic phase, gthread, loop index), the
 *     paper's label-first schedules of the appendix listings).  The accesses
 *     of one phase at one (thread, loop index) are one statement instance.
 *     Barriers play no part.  With Before = strictly earlier time, per
 *     element e: RaW counts pairs (x, y), x before y, x writes e, y reads e;
 *     WaW: x and y write e; WaR: x reads e, y writes e.  Totals are summed
 *     over elements (a pair of instances sharing two elements counts twice:
 *     the relation with the element kept).
 *
 *  9. Barrier divergence (orc_divergence).  A barrier may carry guards
 *     (affine >= 0 in tx, ty, bx, by, k) naming the threads that reach it.
 *     A block barrier instance (dynamic phase, block) or a warp barrier
 *     instance (dynamic phase, warp) is divergent when some but not all of
 *     its scope's threads reach it.  The race check treats every barrier as
 *     reached by all threads.
 *
 * Arithmetic is exact int64: every product and sum is checked, and a value
 * that would leave int64 stops the check with status -4 (the instance is
 * reported as for an out-of-bounds index).  The paper's sets range over
 * unbounded integers; int64 holds every value of a description whose
 * variables and coefficients are int32 unless a sum of several large
 * products overflows, which is reported instead of wrapped.  qsort is the
 * only library step.
 */

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NV 10
#define V_TX 0
#define V_TY 1
#define V_BX 2
#define V_BY 3
#define V_K 4
#define V_L0 5
#define V_AUX0 8

/* ------------------------------------------------------------ input layout */
/* The Python side serialises a description into int64 words:
 *   header  : magic, bdx, bdy, gdx, gdy, n_arrays, n_accesses, n_guards, n_phases, n_segments,
 *             warp_size
 *   arrays  : space, ndim, dim0, dim1, dim2                                   (5 words)
 *   accesses: array, is_write, nloops, lo0, hi0, lo1, hi1, lo2, hi2,
 *             aux0 (kind, d, coef[10], c0), aux1 (same),
 *             idx0 (coef[10], c0), idx1, idx2, guard_begin, guard_count      (70 words)
 *   guards  : coef[10], c0                                                    (11 words)
 *   phases  : access_begin, access_count, barrier (0 none, 1 block, 2 warp),
 *             guard_begin, guard_count (barrier guards)                       (5 words)
 *   segments: phase_begin, phase_count, repeat, k_base                        (4 words)
 */
#define ORC_MAGIC 0x524f5256LL
#define HDR 11
#define ARR_W 5
#define ACC_W 70
#define GRD_W 11
#define PH_W 5
#define SEG_W 4

typedef struct { int64_t coef[NV]; int64_t c0; } aff_t;
typedef struct { int64_t kind, d; aff_t e; } aux_t;
typedef struct {
    int64_t array, is_write, nloops, lo[3], hi[3];
    aux_t aux[2];
    aff_t idx[3];
    int64_t guard_begin, guard_count;
} acc_t;
typedef struct { int64_t space, ndim, dim[3]; } arr_t;
typedef struct { int64_t access_begin, access_count, barrier_after, guard_begin, guard_count; } ph_t;
typedef struct { int64_t phase_begin, phase_count, repeat, k_base; } seg_t;

typedef struct {
    int64_t bdx, bdy, gdx, gdy, warp_size;
    int64_t n_arrays, n_accesses, n_guards, n_phases, n_segments;
    arr_t *arrays;
    acc_t *accesses;
    aff_t *guards;
    ph_t *phases;
    seg_t *segments;
    /* dynamic phases */
    int64_t n_dyn;
    int64_t *dyn_phase;     /* static phase of dynamic phase d */
    int64_t *dyn_k;         /* value of k in d */
    int64_t *dyn_interval;  /* barrier interval of d (block barriers before d) */
    int64_t *dyn_fine;      /* fine interval of d (barriers of either kind before d) */
    int64_t n_intervals;
    int64_t has_warp_barriers;
} kern_t;

/* ------------------------------------------------------------- public API */
typedef struct {
    int64_t interval, space, array, address, block;           /* block: if shared, else 0 */
    int64_t f_block, f_tid, f_dphase, f_access, f_loop[3], f_write;
    int64_t s_block, s_tid, s_dphase, s_access, s_loop[3], s_write;
} orc_witness;

typedef struct {
    int64_t status;          /* 0 ok, -1 invalid description, -4 a value left int64,
                                -5 index out of bounds, -10 no memory */
    int64_t n_records;
    int64_t n_conflicts;     /* conflicting locations */
    int64_t n_pairs;         /* unordered distinct-thread pairs with >= 1 write (diagnostic) */
    int64_t n_intervals;
    int64_t oob[5];          /* interval, gthread, dynamic phase, access, loop index of the
                                instance behind status -5 or -4 */
    int64_t n_witness;       /* witnesses written (<= capacity) */
} orc_result;

typedef struct {
    int64_t interval, space, block, array, address;
    int64_t gthread, dphase, access, lidx, loop[3], is_write;
} orc_record;

/* ---------------------------------------------------------------- parsing */
static void rd_aff(const int64_t *w, aff_t *a) {
    for (int v = 0; v < NV; v++) a->coef[v] = w[v];
    a->c0 = w[NV];
}

static void kern_free(kern_t *k) {
    free(k->arrays); free(k->accesses); free(k->guards); free(k->phases); free(k->segments);
    free(k->dyn_phase); free(k->dyn_k); free(k->dyn_interval); free(k->dyn_fine);
    memset(k, 0, sizeof(*k));
}

static int kern_parse(const int64_t *w, int64_t len, kern_t *k) {
    memset(k, 0, sizeof(*k));
    if (len < HDR || w[0] != ORC_MAGIC) return -1;
    k->bdx = w[1]; k->bdy = w[2]; k->gdx = w[3]; k->gdy = w[4];
    k->n_arrays = w[5]; k->n_accesses = w[6]; k->n_guards = w[7]; k->n_phases = w[8]; k->n_segments = w[9];
    k->warp_size = w[10];
    if (k->bdx < 1 || k->bdy < 1 || k->gdx < 1 || k->gdy < 1 || k->warp_size < 1) return -1;
    if (k->n_arrays < 0 || k->n_accesses < 0 || k->n_guards < 0 || k->n_phases < 0 || k->n_segments < 0) return -1;
    int64_t need = HDR + k->n_arrays * ARR_W + k->n_accesses * ACC_W + k->n_guards * GRD_W +
                   k->n_phases * PH_W + k->n_segments * SEG_W;
    if (len != need) return -1;
    k->arrays = calloc((size_t)k->n_arrays + 1, sizeof(arr_t));
    k->accesses = calloc((size_t)k->n_accesses + 1, sizeof(acc_t));
    k->guards = calloc((size_t)k->n_guards + 1, sizeof(aff_t));
    k->phases = calloc((size_t)k->n_phases + 1, sizeof(ph_t));
    k->segments = calloc((size_t)k->n_segments + 1, sizeof(seg_t));
    if (!k->arrays || !k->accesses || !k->guards || !k->phases || !k->segments) return -10;
    const int64_t *p = w + HDR;
    for (int64_t i = 0; i < k->n_arrays; i++, p += ARR_W) {
        arr_t *a = &k->arrays[i];
        a->space = p[0]; a->ndim = p[1];
        a->dim[0] = p[2]; a->dim[1] = p[3]; a->dim[2] = p[4];
        if (a->space != 0 && a->space != 1) return -1;
        if (a->ndim < 1 || a->ndim > 3) return -1;
        int64_t elems = 1;
        for (int d = 0; d < a->ndim; d++) {
            if (a->dim[d] < 1) return -1;
            if (__builtin_mul_overflow(elems, a->dim[d], &elems)) return -1;   /* flat index fits int64 */
        }
    }
    for (int64_t i = 0; i < k->n_accesses; i++, p += ACC_W) {
        acc_t *a = &k->accesses[i];
        a->array = p[0]; a->is_write = p[1]; a->nloops = p[2];
        for (int l = 0; l < 3; l++) { a->lo[l] = p[3 + 2 * l]; a->hi[l] = p[4 + 2 * l]; }
        for (int x = 0; x < 2; x++) {
            const int64_t *q = p + 9 + 13 * x;
            a->aux[x].kind = q[0]; a->aux[x].d = q[1];
            rd_aff(q + 2, &a->aux[x].e);
        }
        for (int d = 0; d < 3; d++) rd_aff(p + 35 + 11 * d, &a->idx[d]);
        a->guard_begin = p[68]; a->guard_count = p[69];
        if (a->array < 0 || a->array >= k->n_arrays) return -1;
        if (a->nloops < 0 || a->nloops > 3) return -1;
        for (int l = 0; l < a->nloops; l++) if (a->lo[l] > a->hi[l]) return -1;
        for (int x = 0; x < 2; x++) {
            if (a->aux[x].kind < 0 || a->aux[x].kind > 2) return -1;
            if (a->aux[x].kind && a->aux[x].d < 1) return -1;
            if (a->aux[x].e.coef[V_AUX0] || a->aux[x].e.coef[V_AUX0 + 1]) return -1;
        }
        if (a->guard_begin < 0 || a->guard_count < 0 || a->guard_begin + a->guard_count > k->n_guards) return -1;
    }
    for (int64_t i = 0; i < k->n_guards; i++, p += GRD_W) rd_aff(p, &k->guards[i]);
    for (int64_t i = 0; i < k->n_phases; i++, p += PH_W) {
        ph_t *h = &k->phases[i];
        h->access_begin = p[0]; h->access_count = p[1]; h->barrier_after = p[2];
        h->guard_begin = p[3]; h->guard_count = p[4];
        if (h->access_begin < 0 || h->access_count < 0 || h->access_begin + h->access_count > k->n_accesses) return -1;
        if (h->barrier_after < 0 || h->barrier_after > 2) return -1;
        if (h->guard_begin < 0 || h->guard_count < 0 || h->guard_begin + h->guard_count > k->n_guards) return -1;
        if (h->guard_count && !h->barrier_after) return -1;
        for (int64_t g = h->guard_begin; g < h->guard_begin + h->guard_count; g++)
            for (int v = V_L0; v < NV; v++)
                if (k->guards[g].coef[v]) return -1;       /* barrier guards: tx, ty, bx, by, k only */
        if (h->barrier_after == 2) k->has_warp_barriers = 1;
    }
    for (int64_t i = 0; i < k->n_segments; i++, p += SEG_W) {
        seg_t *s = &k->segments[i];
        s->phase_begin = p[0]; s->phase_count = p[1]; s->repeat = p[2]; s->k_base = p[3];
        if (s->phase_begin < 0 || s->phase_count < 0 || s->phase_begin + s->phase_count > k->n_phases) return -1;
        if (s->repeat < 1) return -1;
    }
    /* step 1-2: dynamic phases and their barrier intervals */
    int64_t nd = 0;
    for (int64_t i = 0; i < k->n_segments; i++) nd += k->segments[i].repeat * k->segments[i].phase_count;
    k->n_dyn = nd;
    k->dyn_phase = calloc((size_t)nd + 1, sizeof(int64_t));
    k->dyn_k = calloc((size_t)nd + 1, sizeof(int64_t));
    k->dyn_interval = calloc((size_t)nd + 1, sizeof(int64_t));
    k->dyn_fine = calloc((size_t)nd + 1, sizeof(int64_t));
    if (!k->dyn_phase || !k->dyn_k || !k->dyn_interval || !k->dyn_fine) return -10;
    int64_t d = 0, barriers = 0, fine = 0;
    for (int64_t i = 0; i < k->n_segments; i++) {
        const seg_t *s = &k->segments[i];
        for (int64_t r = 0; r < s->repeat; r++) {
            for (int64_t j = 0; j < s->phase_count; j++) {
                int64_t ph = s->phase_begin + j;
                k->dyn_phase[d] = ph;
                k->dyn_k[d] = s->k_base + r;
                k->dyn_interval[d] = barriers;          /* block barriers executed before d */
                k->dyn_fine[d] = fine;                  /* barriers of either kind before d */
                if (k->phases[ph].barrier_after == 1) barriers++;
                if (k->phases[ph].barrier_after) fine++;
                d++;
            }
        }
    }
    k->n_intervals = nd ? k->dyn_interval[nd - 1] + 1 : 0;
    return 0;
}

/* ------------------------------------------------------------- arithmetic */
/* Checked int64 operations: *ovf is set when the exact result leaves int64. */
static int64_t add_ck(int64_t a, int64_t b, int *ovf) {
    int64_t r;
    if (__builtin_add_overflow(a, b, &r)) *ovf = 1;
    return r;
}

static int64_t mul_ck(int64_t a, int64_t b, int *ovf) {
    int64_t r;
    if (__builtin_mul_overflow(a, b, &r)) *ovf = 1;
    return r;
}

static int64_t eval_aff(const aff_t *a, const int64_t *v, int *ovf) {
    int64_t s = a->c0;
    for (int i = 0; i < NV; i++) s = add_ck(s, mul_ck(a->coef[i], v[i], ovf), ovf);
    return s;
}

static int64_t floor_div(int64_t n, int64_t d) {      /* d >= 1: no overflow */
    int64_t q = n / d;                               /* C truncates toward zero */
    if ((n % d != 0) && (n < 0)) q -= 1;
    return q;
}

static int64_t euclid_mod(int64_t n, int64_t d) {     /* result in [0, d) */
    int64_t r = n % d;                               /* same sign as n, |r| < d */
    return r < 0 ? r + d : r;
}

/* ------------------------------------------------------------ enumeration */
typedef struct {
    int64_t space, block, array, address;            /* location (the interval is implicit) */
    int64_t gthread, dphase, access, lidx;           /* id */
    int64_t loop[3], is_write;
} rec_t;

typedef struct { rec_t *r; int64_t n, cap; } recvec_t;

static int push(recvec_t *v, const rec_t *x) {
    if (v->n == v->cap) {
        int64_t nc = v->cap ? v->cap * 2 : 1024;
        rec_t *p = realloc(v->r, (size_t)nc * sizeof(rec_t));
        if (!p) return -10;
        v->r = p; v->cap = nc;
    }
    v->r[v->n++] = *x;
    return 0;
}

/* Records of one interval, in (gthread, dphase, access, lidx) order.
 * Returns 0, -5 (out of bounds: oob[] filled) or -10. */
static int enumerate_interval(const kern_t *k, int64_t iv, recvec_t *out, int64_t *oob) {
    int64_t dlo = -1, dhi = -1;
    for (int64_t d = 0; d < k->n_dyn; d++)
        if (k->dyn_interval[d] == iv) { if (dlo < 0) dlo = d; dhi = d + 1; }
    if (dlo < 0) return 0;
    const int64_t tpb = k->bdx * k->bdy;
    const int64_t nblk = k->gdx * k->gdy;
    for (int64_t b = 0; b < nblk; b++) {
        const int64_t bx = b % k->gdx, by = b / k->gdx;
        for (int64_t t = 0; t < tpb; t++) {
            const int64_t tx = t % k->bdx, ty = t / k->bdx;
            const int64_t gthread = b * tpb + t;
            for (int64_t d = dlo; d < dhi; d++) {
                const ph_t *ph = &k->phases[k->dyn_phase[d]];
                for (int64_t a = ph->access_begin; a < ph->access_begin + ph->access_count; a++) {
                    const acc_t *ac = &k->accesses[a];
                    const arr_t *ar = &k->arrays[ac->array];
                    int64_t ext[3] = {1, 1, 1};
                    for (int l = 0; l < ac->nloops; l++) ext[l] = ac->hi[l] - ac->lo[l];
                    int64_t box;
                    if (__builtin_mul_overflow(ext[0], ext[1], &box) || __builtin_mul_overflow(box, ext[2], &box)) {
                        oob[0] = iv; oob[1] = gthread; oob[2] = d; oob[3] = a; oob[4] = 0;
                        return -4;
                    }
                    for (int64_t li = 0; li < box; li++) {
                        int64_t v[NV] = {0};
                        v[V_TX] = tx; v[V_TY] = ty; v[V_BX] = bx; v[V_BY] = by; v[V_K] = k->dyn_k[d];
                        /* row-major loop index -> loop values */
                        int64_t rem = li, lv[3] = {0, 0, 0};
                        for (int l = ac->nloops - 1; l >= 0; l--) {
                            lv[l] = ac->lo[l] + rem % ext[l];
                            rem /= ext[l];
                        }
                        for (int l = 0; l < 3; l++) v[V_L0 + l] = lv[l];
                        int ovf = 0;
                        for (int x = 0; x < 2; x++) {
                            const aux_t *u = &ac->aux[x];
                            if (u->kind == 1) v[V_AUX0 + x] = floor_div(eval_aff(&u->e, v, &ovf), u->d);
                            else if (u->kind == 2) v[V_AUX0 + x] = euclid_mod(eval_aff(&u->e, v, &ovf), u->d);
                        }
                        int ok = 1;
                        for (int64_t g = ac->guard_begin; g < ac->guard_begin + ac->guard_count && ok; g++)
                            if (eval_aff(&k->guards[g], v, &ovf) < 0) ok = 0;
                        if (ovf) {
                            oob[0] = iv; oob[1] = gthread; oob[2] = d; oob[3] = a; oob[4] = li;
                            return -4;
                        }
                        if (!ok) continue;
                        int64_t flat = 0;
                        for (int dd = 0; dd < ar->ndim; dd++) {
                            int64_t ix = eval_aff(&ac->idx[dd], v, &ovf);
                            if (ovf) {
                                oob[0] = iv; oob[1] = gthread; oob[2] = d; oob[3] = a; oob[4] = li;
                                return -4;
                            }
                            if (ix < 0 || ix >= ar->dim[dd]) {
                                oob[0] = iv; oob[1] = gthread; oob[2] = d; oob[3] = a; oob[4] = li;
                                return -5;
                            }
                            flat = flat * ar->dim[dd] + ix;      /* < product of dims: checked at parse */
                        }
                        rec_t r;
                        r.space = ar->space;
                        r.block = ar->space == 0 ? b : 0;
                        r.array = ac->array;
                        r.address = flat;
                        r.gthread = gthread; r.dphase = d; r.access = a; r.lidx = li;
                        r.loop[0] = lv[0]; r.loop[1] = lv[1]; r.loop[2] = lv[2];
                        r.is_write = ac->is_write ? 1 : 0;
                        int e = push(out, &r);
                        if (e) return e;
                    }
                }
            }
        }
    }
    return 0;
}

#define CMP(a, b) do { if ((a) < (b)) return -1; if ((a) > (b)) return 1; } while (0)
static int cmp_loc_id(const void *pa, const void *pb) {
    const rec_t *a = pa, *b = pb;
    CMP(a->space, b->space); CMP(a->block, b->block); CMP(a->array, b->array); CMP(a->address, b->address);
    CMP(a->gthread, b->gthread); CMP(a->dphase, b->dphase); CMP(a->access, b->access); CMP(a->lidx, b->lidx);
    return 0;
}
static int same_loc(const rec_t *a, const rec_t *b) {
    return a->space == b->space && a->block == b->block && a->array == b->array && a->address == b->address;
}

static void side(const kern_t *k, const rec_t *r, int64_t *blk, int64_t *tid, int64_t *dph, int64_t *acc,
                 int64_t *loop, int64_t *wr) {
    const int64_t tpb = k->bdx * k->bdy;
    *blk = r->gthread / tpb; *tid = r->gthread % tpb;
    *dph = r->dphase; *acc = r->access;
    loop[0] = r->loop[0]; loop[1] = r->loop[1]; loop[2] = r->loop[2];
    *wr = r->is_write;
}

/* Warp of a thread: warp_size consecutive linear thread ids of one block. */
static int64_t warp_of(const kern_t *k, int64_t gthread) {
    const int64_t tpb = k->bdx * k->bdy;
    const int64_t wpb = (tpb + k->warp_size - 1) / k->warp_size;
    return (gthread / tpb) * wpb + (gthread % tpb) / k->warp_size;
}

static int64_t block_of(const kern_t *k, int64_t gthread) { return gthread / (k->bdx * k->bdy); }

/* Step 5 inside the records i of g[0..n) (sorted by id) with sub[i] == j:
 * returns 1 with the canonical pair when they hold a write and two threads. */
static int step5(const rec_t *g, int64_t n, const int64_t *sub, int64_t j, const rec_t **f, const rec_t **s) {
    const rec_t *lo = 0, *hi = 0, *fw = 0;
    for (int64_t i = 0; i < n; i++) {
        if (sub[i] != j) continue;
        if (!lo) lo = &g[i];
        hi = &g[i];
        if (g[i].is_write && !fw) fw = &g[i];
    }
    if (!fw || lo->gthread == hi->gthread) return 0;
    *f = fw;
    *s = lo->gthread != fw->gthread ? lo : hi;
    return 1;
}

/* One location's records g[0..n), sorted by id.  sub[i] is the ordering
 * interval of record i (fine interval, or interval in strict mode); unit()
 * the unordered scope (warp, or block in strict mode).  Steps 6-7: a
 * conflict inside the smallest sub-interval that has one, else across
 * units.  Returns 1 and the canonical pair when the location conflicts. */
static int judge_location(const kern_t *k, const rec_t *g, int64_t n, const int64_t *sub,
                          int64_t (*unit)(const kern_t *, int64_t), const rec_t **f, const rec_t **s) {
    int64_t j = -1;
    for (;;) {                              /* sub-intervals present, in increasing order */
        int64_t next = INT64_MAX;
        for (int64_t i = 0; i < n; i++)
            if (sub[i] > j && sub[i] < next) next = sub[i];
        if (next == INT64_MAX) break;
        j = next;
        if (step5(g, n, sub, j, f, s)) return 1;
    }
    const rec_t *fw = 0;
    for (int64_t i = 0; i < n && !fw; i++)
        if (g[i].is_write) fw = &g[i];
    if (!fw || unit(k, g[0].gthread) == unit(k, g[n - 1].gthread)) return 0;
    *f = fw;
    *s = unit(k, g[0].gthread) != unit(k, fw->gthread) ? &g[0] : &g[n - 1];
    return 1;
}

/* Distinct threads n and writing threads w of a location (records sorted by
 * id, so one thread's records are adjacent): C(n,2) - C(n-w,2) unordered
 * pairs of different threads with at least one write. */
static int64_t distinct_pairs(const rec_t *g, int64_t cnt) {
    int64_t n = 0, nw = 0;
    for (int64_t i = 0; i < cnt;) {
        int64_t j = i, wrote = 0;
        while (j < cnt && g[j].gthread == g[i].gthread) { wrote |= g[j].is_write; j++; }
        n++; nw += wrote; i = j;
    }
    return n * (n - 1) / 2 - (n - nw) * (n - nw - 1) / 2;
}

static void put_witness(const kern_t *k, orc_result *res, orc_witness *wbuf, int64_t wcap, int64_t iv,
                        const rec_t *f, const rec_t *s) {
    if (res->n_conflicts < wcap && wbuf) {
        orc_witness *w = &wbuf[res->n_conflicts];
        w->interval = iv; w->space = f->space; w->array = f->array; w->address = f->address;
        w->block = f->block;
        side(k, f, &w->f_block, &w->f_tid, &w->f_dphase, &w->f_access, w->f_loop, &w->f_write);
        side(k, s, &w->s_block, &w->s_tid, &w->s_dphase, &w->s_access, w->s_loop, &w->s_write);
        res->n_witness++;
    }
    res->n_conflicts++;
}

static int grow_i64(int64_t **p, int64_t *cap, int64_t n) {
    if (n <= *cap) return 0;
    int64_t nc = n > 2 * *cap ? n : 2 * *cap;
    int64_t *q = realloc(*p, (size_t)nc * sizeof(int64_t));
    if (!q) return -10;
    *p = q; *cap = nc;
    return 0;
}

/* Check intervals [ilo, ihi) (clipped to the kernel's).  Witnesses of the
 * conflicting locations are written in (interval, space, block, array,
 * address) order, up to wcap of them.  n_pairs (steps 4-5 only) is -1 when
 * the kernel has warp barriers. */
int orc_check(const int64_t *desc, int64_t len, int64_t ilo, int64_t ihi, orc_result *res,
              orc_witness *wbuf, int64_t wcap) {
    memset(res, 0, sizeof(*res));
    kern_t k;
    int st = kern_parse(desc, len, &k);
    if (st) { kern_free(&k); res->status = st; return st; }
    res->n_intervals = k.n_intervals;
    if (ilo < 0) ilo = 0;
    if (ihi > k.n_intervals) ihi = k.n_intervals;
    recvec_t v = {0};
    int64_t *sub = 0, sub_cap = 0;
    for (int64_t iv = ilo; iv < ihi && !st; iv++) {
        v.n = 0;
        st = enumerate_interval(&k, iv, &v, res->oob);
        if (st) break;
        res->n_records += v.n;
        qsort(v.r, (size_t)v.n, sizeof(rec_t), cmp_loc_id);
        if ((st = grow_i64(&sub, &sub_cap, v.n))) break;
        for (int64_t i = 0; i < v.n; i++) sub[i] = k.dyn_fine[v.r[i].dphase];
        for (int64_t g0 = 0; g0 < v.n;) {
            int64_t g1 = g0 + 1;
            while (g1 < v.n && same_loc(&v.r[g0], &v.r[g1])) g1++;
            /* steps 4-6: the group [g0, g1) is one location, sorted by id */
            const rec_t *f, *s2;
            if (judge_location(&k, v.r + g0, g1 - g0, sub + g0, warp_of, &f, &s2)) {
                if (!k.has_warp_barriers) res->n_pairs += distinct_pairs(v.r + g0, g1 - g0);
                put_witness(&k, res, wbuf, wcap, iv, f, s2);
            }
            g0 = g1;
        }
    }
    if (k.has_warp_barriers) res->n_pairs = -1;
    free(v.r);
    free(sub);
    kern_free(&k);
    res->status = st;
    return st;
}

static int cmp_global_id(const void *pa, const void *pb) {
    const rec_t *a = pa, *b = pb;
    CMP(a->array, b->array); CMP(a->address, b->address);
    CMP(a->gthread, b->gthread); CMP(a->dphase, b->dphase); CMP(a->access, b->access); CMP(a->lidx, b->lidx);
    return 0;
}

/* Step 7: the whole kernel under strict semantics.  Shared-array conflicts
 * come first, in (interval, block, array, address) order, then global ones
 * in (array, address) order; a global witness's interval is its first
 * side's.  Status -2 for a kernel with warp barriers (not defined here). */
int orc_check_strict(const int64_t *desc, int64_t len, orc_result *res, orc_witness *wbuf, int64_t wcap) {
    memset(res, 0, sizeof(*res));
    kern_t k;
    int st = kern_parse(desc, len, &k);
    if (st) { kern_free(&k); res->status = st; return st; }
    res->n_intervals = k.n_intervals;
    res->n_pairs = -1;
    if (k.has_warp_barriers) { kern_free(&k); res->status = -2; return -2; }
    recvec_t v = {0}, glob = {0};
    int64_t *sub = 0, sub_cap = 0;
    for (int64_t iv = 0; iv < k.n_intervals && !st; iv++) {
        v.n = 0;
        st = enumerate_interval(&k, iv, &v, res->oob);
        if (st) break;
        res->n_records += v.n;
        int64_t ns = 0;
        for (int64_t i = 0; i < v.n && !st; i++) {
            if (v.r[i].space == 0) v.r[ns++] = v.r[i];
            else st = push(&glob, &v.r[i]);
        }
        if (st) break;
        v.n = ns;
        qsort(v.r, (size_t)v.n, sizeof(rec_t), cmp_loc_id);
        if ((st = grow_i64(&sub, &sub_cap, v.n))) break;
        for (int64_t i = 0; i < v.n; i++) sub[i] = 0;
        for (int64_t g0 = 0; g0 < v.n;) {
            int64_t g1 = g0 + 1;
            while (g1 < v.n && same_loc(&v.r[g0], &v.r[g1])) g1++;
            const rec_t *f, *s2;
            if (judge_location(&k, v.r + g0, g1 - g0, sub + g0, block_of, &f, &s2))
                put_witness(&k, res, wbuf, wcap, iv, f, s2);
            g0 = g1;
        }
    }
    if (!st) {
        qsort(glob.r, (size_t)glob.n, sizeof(rec_t), cmp_global_id);
        st = grow_i64(&sub, &sub_cap, glob.n);
    }
    if (!st) {
        for (int64_t i = 0; i < glob.n; i++) sub[i] = k.dyn_interval[glob.r[i].dphase];
        for (int64_t g0 = 0; g0 < glob.n;) {
            int64_t g1 = g0 + 1;
            while (g1 < glob.n && same_loc(&glob.r[g0], &glob.r[g1])) g1++;
            const rec_t *f, *s2;
            if (judge_location(&k, glob.r + g0, g1 - g0, sub + g0, block_of, &f, &s2))
                put_witness(&k, res, wbuf, wcap, k.dyn_interval[f->dphase], f, s2);
            g0 = g1;
        }
    }
    free(v.r);
    free(glob.r);
    free(sub);
    kern_free(&k);
    res->status = st;
    return st;
}

/* ------------------------------------------------ step 8: ordered dependences */
typedef struct {
    int64_t status, n_records;
    int64_t n_raw, n_waw, n_war;     /* (earlier instance, element, later instance) triples */
    int64_t n_dep_locations;         /* elements with at least one of them */
    int64_t oob[5];
} orc_deps;

static int cmp_loc_time(const void *pa, const void *pb) {
    const rec_t *a = pa, *b = pb;
    CMP(a->space, b->space); CMP(a->block, b->block); CMP(a->array, b->array); CMP(a->address, b->address);
    CMP(a->dphase, b->dphase); CMP(a->gthread, b->gthread); CMP(a->lidx, b->lidx);
    CMP(a->is_write, b->is_write);
    return 0;
}

int orc_ordered(const int64_t *desc, int64_t len, orc_deps *out) {
    memset(out, 0, sizeof(*out));
    kern_t k;
    int st = kern_parse(desc, len, &k);
    if (st) { kern_free(&k); out->status = st; return st; }
    recvec_t v = {0};
    for (int64_t iv = 0; iv < k.n_intervals && !st; iv++) st = enumerate_interval(&k, iv, &v, out->oob);
    if (!st) {
        out->n_records = v.n;
        qsort(v.r, (size_t)v.n, sizeof(rec_t), cmp_loc_time);
        for (int64_t g0 = 0; g0 < v.n;) {
            int64_t g1 = g0 + 1;
            while (g1 < v.n && same_loc(&v.r[g0], &v.r[g1])) g1++;
            /* one element, its records in time order; instances of equal time run together */
            int64_t earlier_w = 0, earlier_r = 0, raw = 0, waw = 0, war = 0;
            for (int64_t i = g0; i < g1;) {
                int64_t j = i, has_w = 0, has_r = 0;
                while (j < g1 && v.r[j].dphase == v.r[i].dphase && v.r[j].gthread == v.r[i].gthread &&
                       v.r[j].lidx == v.r[i].lidx) {
                    if (v.r[j].is_write) has_w = 1; else has_r = 1;
                    j++;
                }
                raw += has_r * earlier_w;
                waw += has_w * earlier_w;
                war += has_w * earlier_r;
                earlier_w += has_w;
                earlier_r += has_r;
                i = j;
            }
            out->n_raw += raw; out->n_waw += waw; out->n_war += war;
            if (raw || waw || war) out->n_dep_locations++;
            g0 = g1;
        }
    }
    free(v.r);
    kern_free(&k);
    out->status = st;
    return st;
}

/* ---------------------------------------------------- step 9: divergence */
typedef struct {
    int64_t status;
    int64_t n_instances;             /* barrier instances: (dphase, block) or (dphase, warp) */
    int64_t n_divergent;
    int64_t dphase, block, warp;     /* the first divergent instance (warp -1 for a block barrier) */
    int64_t arrive_tid, skip_tid;    /* its smallest thread that reaches it and that does not */
} orc_div;

int orc_divergence(const int64_t *desc, int64_t len, orc_div *out) {
    memset(out, 0, sizeof(*out));
    out->dphase = out->block = out->warp = out->arrive_tid = out->skip_tid = -1;
    kern_t k;
    int st = kern_parse(desc, len, &k);
    if (st) { kern_free(&k); out->status = st; return st; }
    const int64_t tpb = k.bdx * k.bdy, nblk = k.gdx * k.gdy;
    for (int64_t d = 0; d < k.n_dyn; d++) {
        const ph_t *ph = &k.phases[k.dyn_phase[d]];
        if (!ph->barrier_after) continue;
        const int64_t scope = ph->barrier_after == 1 ? tpb : k.warp_size;
        for (int64_t b = 0; b < nblk; b++) {
            for (int64_t t0 = 0; t0 < tpb; t0 += scope) {
                const int64_t t1 = t0 + scope < tpb ? t0 + scope : tpb;
                int64_t arrive = -1, skip = -1, reached = 0;
                for (int64_t t = t0; t < t1; t++) {
                    int64_t v[NV] = {0};
                    v[V_TX] = t % k.bdx; v[V_TY] = t / k.bdx; v[V_BX] = b % k.gdx; v[V_BY] = b / k.gdx;
                    v[V_K] = k.dyn_k[d];
                    int ovf = 0, ok = 1;
                    for (int64_t g = ph->guard_begin; g < ph->guard_begin + ph->guard_count; g++)
                        if (eval_aff(&k.guards[g], v, &ovf) < 0) ok = 0;
                    if (ovf) {                  /* a guard value left int64: name the thread */
                        out->dphase = d; out->block = b; out->arrive_tid = t;
                        kern_free(&k);
                        out->status = -4;
                        return -4;
                    }
                    if (ok) { reached++; if (arrive < 0) arrive = t; }
                    else if (skip < 0) skip = t;
                }
                out->n_instances++;
                if (reached && reached < t1 - t0) {
                    if (!out->n_divergent) {
                        out->dphase = d; out->block = b;
                        out->warp = ph->barrier_after == 1 ? -1 : t0 / k.warp_size;
                        out->arrive_tid = arrive; out->skip_tid = skip;
                    }
                    out->n_divergent++;
                }
            }
        }
    }
    kern_free(&k);
    return 0;
}

/* All records of one interval, in id order (for expansion parity tests). */
int orc_records(const int64_t *desc, int64_t len, int64_t interval, orc_record *out, int64_t cap,
                int64_t *n_out) {
    kern_t k;
    int64_t oob[5];
    *n_out = 0;
    int st = kern_parse(desc, len, &k);
    if (st) { kern_free(&k); return st; }
    recvec_t v = {0};
    st = enumerate_interval(&k, interval, &v, oob);
    if (!st) {
        *n_out = v.n;
        for (int64_t i = 0; i < v.n && i < cap; i++) {
            const rec_t *r = &v.r[i];
            orc_record *o = &out[i];
            o->interval = interval; o->space = r->space; o->block = r->block; o->array = r->array;
            o->address = r->address; o->gthread = r->gthread; o->dphase = r->dphase; o->access = r->access;
            o->lidx = r->lidx; o->loop[0] = r->loop[0]; o->loop[1] = r->loop[1]; o->loop[2] = r->loop[2];
            o->is_write = r->is_write;
        }
    }
    free(v.r);
    kern_free(&k);
    return st;
}

/* Number of barrier intervals and emitted records per interval (sizes only). */
int orc_intervals(const int64_t *desc, int64_t len, int64_t *n_intervals) {
    kern_t k;
    int st = kern_parse(desc, len, &k);
    *n_intervals = st ? 0 : k.n_intervals;
    kern_free(&k);
    return st;
}
