// gfx950 kernels of the per-barrier-interval race check.
//
// Pipeline for one chunk of passes (see plan.cpp):
//   k_hist     count: evaluate every instance (guards, bounds, location) and
//              histogram the records per location bucket           [ALU, no record traffic]
//   k_scan_*   exclusive scan of the bucket counts -> bucket starts
//   k_scatter  expansion: evaluate the instances again, build the 8-byte
//              records (location << 1 | rw, instance id) and write them
//              grouped by bucket through an LDS-staged counting sort (the
//              most significant radix digit of the location key); linear
//              items reserve per run of points or per lane      [writes 8 B / record]
//   k_fold     (default grouping) per bucket: fold each location's summary
//              (min id, max id, min write id, max write id + 1) in LDS
//              tables with atomics, judge every location, write canonical
//              witnesses in location order; k_mid / k_hot take buckets
//              above one slice / above 32K records (k_hot merges parts of
//              a bucket, k_hot_judge judges it)                   [reads 8 B / record]
//   k_bucket   (sort + scan grouping) per bucket: load the records on chip, LDS radix sort on the
//              bucket's low key bits, segmented scan (ballot heads, DPP
//              reductions) giving per location (min id, max id, min write
//              id, max write id + 1); flag conflicting locations, count them
//              and write canonical witnesses in location order     [reads 8 B / record]
//   k_finish / k_first   per-pass conflict totals and first witness.
//
// A location conflicts iff it has a write and two different threads touch
// it in the interval.  Instance ids are ordered thread-major, so that is
// (max write id + 1 != 0) && thread(min id) != thread(max id): the RaW / WaW /
// WaR relations of Section 2.1 restricted to one unordered barrier interval.
//
// Plan tables are read through the constant address space: they are
// read-only during a launch, so the compiler keeps them in scalar registers
// (s_load) even across the atomics of the loops.  Count, scatter and fold
// run as persistent grids that deal their work items (buckets for the fold)
// out in small chunks, cyclically; within a round, adjacent chunks go to the
// same XCD (workgroups are dealt round-robin over the 8 XCDs), so the bucket
// counters and partially written lines they share stay in one L2.

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "rv_internal.h"

namespace rv {

#define RV_CONST __attribute__((address_space(4)))
using CSub = const RV_CONST DevSub;
using CEnt = const RV_CONST DevEntry;
using CKer = const RV_CONST DevKernel;
using CI32 = const RV_CONST int32_t;
using CU32 = const RV_CONST uint32_t;

template <class T>
__device__ __forceinline__ const RV_CONST T *cptr(const T *p) {
    return (const RV_CONST T *)p;
}

__device__ __forceinline__ Magic ldm(const RV_CONST Magic &x) {
    Magic g;
    g.m = x.m; g.s1 = x.s1; g.s2 = x.s2; g.d = x.d;
    return g;
}

// ---------------------------------------------------------------- wave utils
__device__ __forceinline__ uint32_t lane() { return __lane_id(); }

__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, uint32_t l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}

// DPP move: lanes whose source is outside the row (or whose row is masked
// off) receive `old`.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint32_t dpp(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWMASK, 0xf, false);
}
constexpr int ROW_SHR1 = 0x111, ROW_SHR2 = 0x112, ROW_SHR4 = 0x114, ROW_SHR8 = 0x118;
constexpr int ROW_BCAST15 = 0x142, ROW_BCAST31 = 0x143;

// Inclusive wave64 scans: Hillis-Steele inside each row of 16 lanes, then
// row 0 -> 1 and row 2 -> 3 (bcast15), lane 31 -> rows 2 and 3 (bcast31).
__device__ __forceinline__ uint32_t wave_incl_add(uint32_t v) {
    v += dpp<ROW_SHR1, 0xf>(0u, v);
    v += dpp<ROW_SHR2, 0xf>(0u, v);
    v += dpp<ROW_SHR4, 0xf>(0u, v);
    v += dpp<ROW_SHR8, 0xf>(0u, v);
    v += dpp<ROW_BCAST15, 0xa>(0u, v);
    v += dpp<ROW_BCAST31, 0xc>(0u, v);
    return v;
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
    v = min(v, dpp<ROW_SHR1, 0xf>(0xFFFFFFFFu, v));
    v = min(v, dpp<ROW_SHR2, 0xf>(0xFFFFFFFFu, v));
    v = min(v, dpp<ROW_SHR4, 0xf>(0xFFFFFFFFu, v));
    v = min(v, dpp<ROW_SHR8, 0xf>(0xFFFFFFFFu, v));
    v = min(v, dpp<ROW_BCAST15, 0xa>(0xFFFFFFFFu, v));
    v = min(v, dpp<ROW_BCAST31, 0xc>(0xFFFFFFFFu, v));
    return readlane(v, 63);
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
    v = max(v, dpp<ROW_SHR1, 0xf>(0u, v));
    v = max(v, dpp<ROW_SHR2, 0xf>(0u, v));
    v = max(v, dpp<ROW_SHR4, 0xf>(0u, v));
    v = max(v, dpp<ROW_SHR8, 0xf>(0u, v));
    v = max(v, dpp<ROW_BCAST15, 0xa>(0u, v));
    v = max(v, dpp<ROW_BCAST31, 0xc>(0u, v));
    return readlane(v, 63);
}

// Exclusive prefix sum over a workgroup of NT threads; returns the prefix and
// writes the total to *total (all threads).  `red` holds NT/64 words.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_add(uint32_t v, uint32_t *red, uint32_t *total) {
    const uint32_t wid = threadIdx.x >> 6;
    uint32_t inc = wave_incl_add(v);
    if (lane() == 63) red[wid] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; w++) {
        uint32_t x = red[w];
        before += (w < (int)wid) ? x : 0u;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

// Workgroup min, max and sum (all threads get the results).  `red` holds
// 3 * NT/64 words.
template <int NT>
__device__ __forceinline__ void block_min_max_sum(uint32_t &mn, uint32_t &mx, uint32_t &sum, uint32_t *red) {
    const uint32_t wid = threadIdx.x >> 6;
    const uint32_t a = wave_min(mn), b = wave_max(mx), c = readlane(wave_incl_add(sum), 63);
    if (lane() == 0) { red[wid] = a; red[NT / 64 + wid] = b; red[2 * (NT / 64) + wid] = c; }
    __syncthreads();
    mn = 0xFFFFFFFFu; mx = 0; sum = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; w++) {
        mn = min(mn, red[w]);
        mx = max(mx, red[NT / 64 + w]);
        sum += red[2 * (NT / 64) + w];
    }
    __syncthreads();
}

// Rank of a record inside its bin counter h[b] (unique per valid lane).
// Waves whose records share one bin (the common case for structured
// kernels) take one atomic.
__device__ __forceinline__ uint32_t lds_rank(uint32_t *h, uint32_t b, bool v) {
    const uint64_t act = __ballot(v);
    if (act == 0) return 0;
    const uint32_t lead = (uint32_t)__builtin_ctzll(act);
    const uint32_t lb = readlane(b, lead);
    const uint64_t same = __ballot(v && b == lb);
    if (same == act) {
        uint32_t base = 0;
        if (lane() == lead) base = atomicAdd(&h[lb], (uint32_t)__popcll(act));
        base = readlane(base, lead);
        return base + mbcnt(act);
    }
    return v ? atomicAdd(&h[b], 1u) : 0u;
}

// ------------------------------------------------------------ work items
// A cursor over the work items of a chunk: pass, entry of the pass's
// interval, item inside the entry.
struct Cursor {
    uint32_t sub, e, li, e_items;
};

__device__ __forceinline__ void seek(CSub *subs, uint32_t nsub, uint32_t w, Cursor &c) {
    uint32_t lo = 0, hi = nsub;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (subs[mid].item_begin <= w) lo = mid; else hi = mid;
    }
    c.sub = lo;
    const uint32_t local = w - subs[lo].item_begin;
    CU32 *pre = cptr(subs[lo].entry_items);
    uint32_t elo = 0, ehi = subs[lo].n_entries;
    while (ehi - elo > 1) {
        const uint32_t mid = (elo + ehi) >> 1;
        if (pre[mid] <= local) elo = mid; else ehi = mid;
    }
    c.e = elo;
    c.li = local - pre[elo];
    c.e_items = pre[elo + 1] - pre[elo];
}

// Next item; only called while one exists.
__device__ __forceinline__ void advance(CSub *subs, Cursor &c) {
    c.li++;
    while (c.li >= c.e_items) {
        c.li = 0;
        c.e++;
        if (c.e >= subs[c.sub].n_entries) { c.sub++; c.e = 0; }
        CU32 *pre = cptr(subs[c.sub].entry_items);
        c.e_items = pre[c.e + 1] - pre[c.e];
    }
}

// Evaluate the RPL instance slots of this lane in one work item and call
// f(slot, valid, in_bounds, location, id) for each.  A work item covers
// `lch` consecutive loop points of `gt` threads per lane; the loop counters
// are wave-uniform, the thread decode is per lane and per thread.
// Where item `li` of an entry starts for this lane: the first loop point of
// its chunk (lstart, and its loop counters) and the global thread of its
// first thread group slot (g0; slot gi is g0 + gi * gstep).
template <bool FLAT>
struct ItemStart {
    uint32_t lstart, g0, gstep, c0, c1, c2;
};

template <bool FLAT>
__device__ __forceinline__ ItemStart<FLAT> item_start(CEnt &E, CKer &K, uint32_t li) {
    ItemStart<FLAT> a;
    const uint32_t nl = E.n_lchunks;
    if constexpr (!FLAT) {
        const uint32_t gtile = udiv(li, ldm(E.mg_nl));
        const uint32_t lchunk = li - gtile * nl;
        a.lstart = lchunk * E.lch;
        a.g0 = gtile * E.gt * EXP_WG + threadIdx.x;
        a.gstep = EXP_WG;
    } else {
        const uint32_t q = li * EXP_WG + threadIdx.x;
        const bool qv = q < E.nq;
        uint32_t tg, lchunk;
        if (E.cmaj) {       // chunk-major: neighbouring lanes take neighbouring thread groups
            lchunk = udiv(q, ldm(E.mg_ntg));
            tg = q - lchunk * E.ntg;
        } else {
            tg = udiv(q, ldm(E.mg_nl));
            lchunk = q - tg * nl;
        }
        a.lstart = qv ? lchunk * E.lch : 0u;
        a.g0 = qv ? tg * E.gt : K.nthreads;     // past the last thread: every slot invalid
        a.gstep = 1;
    }
    uint32_t r = a.lstart;
    uint32_t t = udiv(r, ldm(E.mg_e2));
    a.c2 = r - t * E.ext[2];
    r = t;
    t = udiv(r, ldm(E.mg_e1));
    a.c1 = r - t * E.ext[1];
    a.c0 = t;
    return a;
}

// General entries (aux terms or guards) advance with the loop.  A lane keeps
// n mod d of each aux numerator n and one running sum per row (the location
// when the entry is proven in bounds, else the three indices) that already
// holds the aux terms' share.  A step moves n by q * d + r (0 <= r < d, split
// on the host), so n mod d moves by r, less d on a carry, and floor(n / d) by
// q plus the carry; each row adds a constant for the step and, on a carry,
// the aux term's change.  A point takes the inner loop's step, or where the
// inner loop wraps the middle loop's, or where that wraps the outer loop's
// (each lane picks its own, so lanes at different points cost one step).
// The division itself runs once per thread of a work item.
template <bool FLAT, bool GP, bool AUX, class F>
__device__ __forceinline__ void expand_gen(CSub &S, CEnt &E, CKer &K, CI32 *G, uint32_t item, F &&f) {
    const uint32_t lch = E.lch, gt = E.gt;
    const ItemStart<FLAT> st = item_start<FLAT>(E, K, item);
    const uint32_t lstart = st.lstart;
    const uint32_t lcnt = min(lch, E.box - lstart);
    const uint32_t e1 = E.ext[1], e2 = E.ext[2];
    // an absent aux term has d = 1, a zero numerator and zero steps: it
    // stays 0 and never carries
    const bool fd[2] = {E.aux_kind[0] == RV_AUX_FLOORDIV, E.aux_kind[1] == RV_AUX_FLOORDIV};
    const uint32_t dv[2] = {E.aux_mg[0].d, E.aux_mg[1].d};
    const uint32_t L0s = (uint32_t)E.lo[0] + st.c0, L1s = (uint32_t)E.lo[1] + st.c1, L2s = (uint32_t)E.lo[2] + st.c2;
    constexpr int NR = GP ? 1 : 3;       // running sums: the location, or the three indices
    constexpr int NX = AUX ? 2 : 0;      // aux terms stepped (an entry of guards alone has none)
    // coefficient v of row r (GP: the flattened location row)
    auto cf = [&](int r, int v) -> uint32_t {
        if constexpr (GP) return E.fr[v];
        else return (uint32_t)E.row[r][v];
    };
    auto lpart = [&](CI32 *row) {
        return (uint32_t)row[C_L0] * L0s + (uint32_t)row[C_L1] * L1s + (uint32_t)row[C_L2] * L2s;
    };
    // per step form k (the outer (0), middle (1) or inner (2) loop
    // advances): the aux splits, and each row's constant
    uint32_t aq[2][3], ar[2][3], kc[NR][3], jc[2][NR], ts[NR];
#pragma unroll
    for (int x = 0; x < 2; x++)
#pragma unroll
        for (int k = 0; k < 3; k++) { aq[x][k] = E.astep[x][k][0]; ar[x][k] = E.astep[x][k][1]; }
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const uint32_t x2 = cf(r, C_L2), x1 = cf(r, C_L1) - cf(r, C_L2) * (e2 - 1);
        const uint32_t x0 = cf(r, C_L0) - cf(r, C_L1) * (e1 - 1) - cf(r, C_L2) * (e2 - 1);
        kc[r][2] = x2; kc[r][1] = x1; kc[r][0] = x0;
        ts[r] = cf(r, C_L0) * L0s + cf(r, C_L1) * L1s + cf(r, C_L2) * L2s;
#pragma unroll
        for (int x = 0; x < NX; x++) {
            const uint32_t ca = cf(r, C_A0 + x);
#pragma unroll
            for (int k = 0; k < 3; k++) kc[r][k] += ca * (fd[x] ? aq[x][k] : ar[x][k]);
            jc[x][r] = fd[x] ? ca : 0u - ca * dv[x];
        }
    }
    const uint32_t ns[2] = {lpart(E.row[3]), lpart(E.row[4])};
    uint32_t c0 = st.c0, c1 = st.c1, c2 = st.c2;
    uint32_t gi = 0, li = 0;
    int32_t tx = 0, ty = 0, bx = 0, by = 0;
    uint32_t t[NR], rm[2] = {0, 0}, qt[2] = {0, 0};
    uint32_t idbase = 0, locbase = 0;
    bool gval = false;
    // one step of form 0, 1 or 2 (w0: the outer loop advances, else w1: the
    // middle one, else the inner one)
    auto apply = [&](bool w0, bool w1) {
        auto pick = [&](uint32_t v0, uint32_t v1, uint32_t v2) { return w0 ? v0 : w1 ? v1 : v2; };
#pragma unroll
        for (int r = 0; r < NR; r++) t[r] += pick(kc[r][0], kc[r][1], kc[r][2]);
#pragma unroll
        for (int x = 0; x < NX; x++) {
            const uint32_t rr = rm[x] + pick(ar[x][0], ar[x][1], ar[x][2]);
            const bool cy = rr >= dv[x];
            rm[x] = cy ? rr - dv[x] : rr;
            if constexpr (!GP) qt[x] += pick(aq[x][0], aq[x][1], aq[x][2]) + (cy ? 1u : 0u);
#pragma unroll
            for (int r = 0; r < NR; r++) t[r] += cy ? jc[x][r] : 0u;
        }
    };
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const bool active = gi < gt;
        if (active && li == 0) {
            const uint32_t g = st.g0 + gi * st.gstep;
            gval = g < K.nthreads;
            const uint32_t gg = gval ? g : 0u;
            const uint32_t blk = udiv(gg, ldm(K.mg_tpb));
            const uint32_t tid = gg - blk * K.tpb;
            const uint32_t byy = udiv(blk, ldm(K.mg_gdx));
            const uint32_t tyy = udiv(tid, ldm(K.mg_bdx));
            tx = (int32_t)(tid - tyy * K.bdx);
            ty = (int32_t)tyy;
            bx = (int32_t)(blk - byy * K.gdx);
            by = (int32_t)byy;
            // thread part of a row plus its constant (modulo 2^32; the plan
            // proved every value the row takes inside int32)
            auto tpart = [&](int r) {
                return cf(r, C_TX) * (uint32_t)tx + cf(r, C_TY) * (uint32_t)ty + cf(r, C_BX) * (uint32_t)bx +
                       cf(r, C_BY) * (uint32_t)by + cf(r, C_C0);
            };
            uint32_t a[2] = {0, 0};
#pragma unroll
            for (int x = 0; x < NX; x++) {
                CI32 *row = E.row[3 + x];
                const int32_t n = (int32_t)((uint32_t)row[C_TX] * (uint32_t)tx + (uint32_t)row[C_TY] * (uint32_t)ty +
                                            (uint32_t)row[C_BX] * (uint32_t)bx + (uint32_t)row[C_BY] * (uint32_t)by +
                                            (uint32_t)row[C_C0] + ns[x]);
                const int32_t q = fdiv(n, ldm(E.aux_mg[x]));
                qt[x] = (uint32_t)q;
                rm[x] = (uint32_t)(n - q * (int32_t)dv[x]);
                a[x] = fd[x] ? qt[x] : rm[x];
            }
#pragma unroll
            for (int r = 0; r < NR; r++) t[r] = tpart(r) + ts[r] + cf(r, C_A0) * a[0] + cf(r, C_A1) * a[1];
            idbase = gg * E.tmul + E.off + lstart;
            locbase = blk * E.loc_mul;
        }
        bool ok = false, inb = false;
        uint32_t loc = 0, id = 0;
        if (active) {
            ok = gval && li < lcnt;
            if constexpr (GP) {
                inb = true;
                loc = locbase + t[0];
            } else {
                const int32_t L0 = E.lo[0] + (int32_t)c0, L1 = E.lo[1] + (int32_t)c1, L2 = E.lo[2] + (int32_t)c2;
                const int32_t a0 = (int32_t)(fd[0] ? qt[0] : rm[0]), a1 = (int32_t)(fd[1] ? qt[1] : rm[1]);
                for (uint32_t q = 0; q < E.guard_count; q++) {
                    CI32 *gr = G + (size_t)(E.guard_begin + q) * NC;
                    const int32_t gv = gr[C_TX] * tx + gr[C_TY] * ty + gr[C_BX] * bx + gr[C_BY] * by +
                                       gr[C_L0] * L0 + gr[C_L1] * L1 + gr[C_L2] * L2 + gr[C_A0] * a0 +
                                       gr[C_A1] * a1 + gr[C_C0];
                    ok = ok && gv >= 0;
                }
                inb = t[0] < E.dim[0] && t[1] < E.dim[1] && t[2] < E.dim[2];
                const uint32_t flat = (t[0] * E.dim[1] + t[1]) * E.dim[2] + t[2];
                loc = locbase + E.loc_base + (flat << E.wshift);
            }
            id = idbase + li;
        }
        f(s, ok, inb, loc, id);
        if (active) {
            li++;
            if (li == lch) {
                li = 0;
                gi++;
                c0 = st.c0; c1 = st.c1; c2 = st.c2;
            } else {
                c2++;
                const bool w1 = c2 == e2;
                c2 = w1 ? 0u : c2;
                c1 += w1 ? 1u : 0u;
                const bool w0 = w1 && c1 == e1;
                c1 = w0 ? 0u : c1;
                c0 += w0 ? 1u : 0u;
                apply(w0, w1);
            }
        }
    }
}

// Evaluate an entry with aux terms or guards (the general path).
template <bool FLAT, class F>
__device__ __forceinline__ void expand_item(CSub &S, CEnt &E, CKer &K, CI32 *G, uint32_t item, F &&f) {
    if (E.gproven) expand_gen<FLAT, true, true>(S, E, K, G, item, f);
    else if (E.aux_kind[0] != 0 || E.aux_kind[1] != 0) expand_gen<FLAT, false, true>(S, E, K, G, item, f);
    else expand_gen<FLAT, false, false>(S, E, K, G, item, f);
}

// Fast path of expand_item for entries without aux terms or guards: the
// per-thread index bases are exact modulo 2^32, the loop terms advance by
// precomputed steps (wave-uniform on the scalar unit unless FLAT), and the
// location is one add per record from the flattened row (exact modulo 2^32
// for in-bounds records).  PROVEN: the plan showed every index of the entry
// inside its dimension over the whole launch and loop box, so the per-record
// index evaluation and bounds test are skipped.
template <bool FLAT, bool PROVEN, class F>
__device__ __forceinline__ void expand_fast(CSub &S, CEnt &E, CKer &K, uint32_t item, F &&f) {
    const uint32_t lch = E.lch, gt = E.gt;
    const ItemStart<FLAT> st = item_start<FLAT>(E, K, item);
    const uint32_t lstart = st.lstart;
    const uint32_t lcnt = min(lch, E.box - lstart);
    const uint32_t e1 = E.ext[1], e2 = E.ext[2];
    const uint32_t L0s = (uint32_t)E.lo[0] + st.c0, L1s = (uint32_t)E.lo[1] + st.c1, L2s = (uint32_t)E.lo[2] + st.c2;
    // loop terms at the chunk start, and their steps when the inner loop
    // advances (x2), when the middle one does (x1), when the outer one does
    // (x0); all modulo 2^32
    uint32_t la[3], lb[3], lc[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
        la[r] = PROVEN ? 0u : (uint32_t)E.row[r][C_L0];
        lb[r] = PROVEN ? 0u : (uint32_t)E.row[r][C_L1];
        lc[r] = PROVEN ? 0u : (uint32_t)E.row[r][C_L2];
    }
    const uint32_t ts0 = la[0] * L0s + lb[0] * L1s + lc[0] * L2s;
    const uint32_t ts1 = la[1] * L0s + lb[1] * L1s + lc[1] * L2s;
    const uint32_t ts2 = la[2] * L0s + lb[2] * L1s + lc[2] * L2s;
    const uint32_t x2_0 = lc[0], x2_1 = lc[1], x2_2 = lc[2];
    const uint32_t x1_0 = lb[0] - lc[0] * (e2 - 1), x1_1 = lb[1] - lc[1] * (e2 - 1), x1_2 = lb[2] - lc[2] * (e2 - 1);
    const uint32_t x0_0 = la[0] - lb[0] * (e1 - 1) - lc[0] * (e2 - 1);
    const uint32_t x0_1 = la[1] - lb[1] * (e1 - 1) - lc[1] * (e2 - 1);
    const uint32_t x0_2 = la[2] - lb[2] * (e1 - 1) - lc[2] * (e2 - 1);
    const uint32_t fl0 = E.fr[C_L0], fl1 = E.fr[C_L1], fl2 = E.fr[C_L2];
    const uint32_t tls = fl0 * L0s + fl1 * L1s + fl2 * L2s;
    const uint32_t y2 = fl2, y1 = fl1 - fl2 * (e2 - 1), y0 = fl0 - fl1 * (e1 - 1) - fl2 * (e2 - 1);
    const uint32_t d0 = E.dim[0], d1 = E.dim[1], d2 = E.dim[2];
    const uint32_t ftx = E.fr[C_TX], fty = E.fr[C_TY], fbx = E.fr[C_BX], fby = E.fr[C_BY], fc0 = E.fr[C_C0];
    const uint32_t loc_mul = E.loc_mul, eoff = E.off;
    const uint32_t tpb = K.tpb, bdx = K.bdx, gdx = K.gdx, nthreads = K.nthreads, M = E.tmul;
    const Magic mg_tpb = ldm(K.mg_tpb), mg_gdx = ldm(K.mg_gdx), mg_bdx = ldm(K.mg_bdx);
    uint32_t c1 = st.c1, c2 = st.c2;
    uint32_t t0 = ts0, t1 = ts1, t2 = ts2, tl = tls;
    uint32_t gi = 0, li = 0;
    uint32_t base0 = 0, base1 = 0, base2 = 0;
    uint32_t lbase = 0, idbase = 0;
    bool gval = false;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const bool active = gi < gt;
        if (active && li == 0) {
            const uint32_t g = st.g0 + gi * st.gstep;
            gval = g < nthreads;
            const uint32_t gg = gval ? g : 0u;
            const uint32_t blk = udiv(gg, mg_tpb);
            const uint32_t tid = gg - blk * tpb;
            const uint32_t byy = udiv(blk, mg_gdx);
            const uint32_t tyy = udiv(tid, mg_bdx);
            const int32_t tx = (int32_t)(tid - tyy * bdx), ty = (int32_t)tyy;
            const int32_t bx = (int32_t)(blk - byy * gdx), by = (int32_t)byy;
            if constexpr (!PROVEN) {
                // full 32-bit products: thread and block ids reach 2^31 - 1,
                // and the plan proved every index value fits int32, so the
                // sums modulo 2^32 are the exact indices
                auto bse = [&](int r) {
                    return (uint32_t)E.row[r][C_TX] * (uint32_t)tx + (uint32_t)E.row[r][C_TY] * (uint32_t)ty +
                           (uint32_t)E.row[r][C_BX] * (uint32_t)bx + (uint32_t)E.row[r][C_BY] * (uint32_t)by +
                           (uint32_t)E.row[r][C_C0];
                };
                base0 = bse(0);
                base1 = bse(1);
                base2 = bse(2);
            }
            lbase = blk * loc_mul + ftx * (uint32_t)tx + fty * (uint32_t)ty + fbx * (uint32_t)bx +
                    fby * (uint32_t)by + fc0;
            idbase = gg * M + eoff + lstart;
        }
        bool ok = false, inb = false;
        uint32_t loc = 0, id = 0;
        if (active) {
            if constexpr (PROVEN) {
                inb = true;
            } else {
                inb = base0 + t0 < d0 && base1 + t1 < d1 && base2 + t2 < d2;
            }
            loc = lbase + tl;
            id = idbase + li;
            ok = gval && li < lcnt;
        }
        f(s, ok, inb, loc, id);
        if (active) {
            li++;
            if (li == lch) {
                li = 0;
                gi++;
                c1 = st.c1; c2 = st.c2;
                t0 = ts0; t1 = ts1; t2 = ts2; tl = tls;
            } else {
                c2++;
                if (c2 == e2) {
                    c2 = 0;
                    c1++;
                    if (c1 == e1) {
                        c1 = 0;
                        t0 += x0_0; t1 += x0_1; t2 += x0_2; tl += y0;
                    } else {
                        t0 += x1_0; t1 += x1_1; t2 += x1_2; tl += y1;
                    }
                } else {
                    t0 += x2_0; t1 += x2_1; t2 += x2_2; tl += y2;
                }
            }
        }
    }
}

// Expansion variants: FLAT x {proven fast, fast, general}.
template <int V>
using Variant = std::integral_constant<int, V>;

template <int V, class F>
__device__ __forceinline__ void expand_v(Variant<V>, CSub &S, CEnt &E, CKer &K, uint32_t li, F &&f) {
    constexpr bool FLAT = V >= 3;
    constexpr int P = V % 3;
    if constexpr (P == 0) expand_fast<FLAT, true>(S, E, K, li, f);
    else if constexpr (P == 1) expand_fast<FLAT, false>(S, E, K, li, f);
    else expand_item<FLAT>(S, E, K, cptr(S.guards), li, f);
}

// Per-wave binning (count pass and scatter): each wave takes WBIN bins of the
// shared area, over at most WWIN windows of its own bucket range.
constexpr int EXP_NW = EXP_WG / 64;
constexpr uint32_t WBIN = BINCAP / EXP_NW;
constexpr uint32_t WWIN = 16;

// Linear work items.  A lane's records in an item of a linear entry are
// one thread's lcnt consecutive points of the innermost loop, so each index
// and the location are affine in the point: an index lies inside its
// dimension at every point when it does at the first and the last (the plan
// proved every index value fits int32, so the unsigned tests are exact), and
// then the locations are exact and move by the same step dl in every lane.
// lin_probe succeeds (wave-uniformly) when every record of the wave is in
// bounds and inside the pass's key range, and
//  * thread-major items (every live lane has the same points): at each point
//    the lanes' records share one bucket.  Points then form runs that share
//    a bucket; lane j < cnt holds point j's bucket, `starts` marks the first
//    point of each run, and a run of m points holds m x popc(live) records.
//  * flat items (lanes differ in their points): all records of the wave
//    share one bucket (a single run starting at point 0).
// The caller then counts or places the records with one reservation per run
// instead of a per-record rank.
struct LinItem {
    uint32_t lcnt;      // records of this lane (0 past the last thread)
    uint32_t hi, dhi;   // first record's key half (loc << 1 | rw), step per point
    uint32_t id;        // first record's id (ids step by one)
    uint32_t pb;        // lane j < cnt: bucket of point j (relative to the pass)
    uint32_t cnt;       // points of the item (thread-major: every live lane's count)
    uint32_t n;         // records of the wave
    uint64_t live;      // lanes with records
    uint64_t starts;    // lanes j that start a run of points
};

// One lane of a linear item: its lcnt points start at location loc and
// instance id (gg * tmul + off + first point) and step by dl and by one;
// inb: every point is inside the array (tested at the first and the last).
struct LinLane {
    uint32_t lcnt, loc, dl, id;
    bool inb;
};

// The lane's records from loop point lstart (loop counters c0, c1, c2 from
// the lower bounds) of global thread g0: at most lmax points.
template <bool PROVEN>
__device__ __forceinline__ LinLane lin_lane_at(CEnt &E, CKer &K, uint32_t g0, uint32_t lstart, uint32_t c0,
                                               uint32_t c1, uint32_t c2, uint32_t lmax) {
    const bool gval = g0 < K.nthreads;
    const uint32_t gg = gval ? g0 : 0u;
    const uint32_t blk = udiv(gg, ldm(K.mg_tpb));
    const uint32_t tid = gg - blk * K.tpb;
    const uint32_t byy = udiv(blk, ldm(K.mg_gdx));
    const uint32_t tyy = udiv(tid, ldm(K.mg_bdx));
    const uint32_t tx = tid - tyy * K.bdx, ty = tyy, bx = blk - byy * K.gdx, by = byy;
    const uint32_t L0 = (uint32_t)E.lo[0] + c0, L1 = (uint32_t)E.lo[1] + c1, L2 = (uint32_t)E.lo[2] + c2;
    LinLane r;
    r.lcnt = gval ? min(lmax, E.box - lstart) : 0u;
    const uint32_t last = r.lcnt - 1u;
    const uint32_t inner = E.linner;
    r.loc = blk * E.loc_mul + E.fr[C_TX] * tx + E.fr[C_TY] * ty + E.fr[C_BX] * bx +
            E.fr[C_BY] * by + E.fr[C_C0] + E.fr[C_L0] * L0 + E.fr[C_L1] * L1 + E.fr[C_L2] * L2;
    r.dl = E.fr[C_L0 + inner];
    r.id = gg * E.tmul + E.off + lstart;
    bool good = true;
    if constexpr (!PROVEN) {
#pragma unroll
        for (int q = 0; q < 3; q++) {
            const uint32_t i0 = (uint32_t)E.row[q][C_TX] * tx + (uint32_t)E.row[q][C_TY] * ty +
                                (uint32_t)E.row[q][C_BX] * bx + (uint32_t)E.row[q][C_BY] * by +
                                (uint32_t)E.row[q][C_C0] + (uint32_t)E.row[q][C_L0] * L0 +
                                (uint32_t)E.row[q][C_L1] * L1 + (uint32_t)E.row[q][C_L2] * L2;
            const uint32_t iN = i0 + last * (uint32_t)E.row[q][C_L0 + inner];
            good = good && i0 < E.dim[q] && iN < E.dim[q];
        }
    }
    r.inb = good;
    return r;
}

template <bool FLAT, bool PROVEN>
__device__ __forceinline__ LinLane lin_lane(CEnt &E, CKer &K, uint32_t item) {
    const ItemStart<FLAT> st = item_start<FLAT>(E, K, item);
    return lin_lane_at<PROVEN>(E, K, st.g0, st.lstart, st.c0, st.c1, st.c2, E.lch);
}

template <bool FLAT, bool PROVEN>
__device__ __forceinline__ bool lin_probe(CSub &S, CEnt &E, CKer &K, uint32_t item, LinItem &L) {
    const LinLane ln = lin_lane<FLAT, PROVEN>(E, K, item);
    const uint32_t lcnt = ln.lcnt, last = lcnt - 1u, loc = ln.loc, dl = ln.dl;
    bool good = ln.inb;
    const uint32_t span = S.khi - S.klo;
    const uint32_t r0 = loc - S.klo, rN = loc + last * dl - S.klo;
    good = lcnt == 0u || (good && r0 < span && rN < span);
    if (__ballot(!good)) return false;
    const uint64_t live = __ballot(lcnt != 0u);
    L.lcnt = lcnt;
    L.hi = (loc << 1) | E.rw;
    L.dhi = dl << 1;
    L.id = ln.id;
    L.live = live;
    if (!live) {
        L.n = 0;
        return true;
    }
    const uint32_t sh = S.s;
    if constexpr (FLAT) {
        const uint32_t b0 = r0 >> sh, bN = rN >> sh;
        const uint32_t mn = wave_min(lcnt ? min(b0, bN) : 0xFFFFFFFFu);
        const uint32_t mx = wave_max(lcnt ? max(b0, bN) : 0u);
        if (mn != mx) return false;
        L.pb = mn;
        L.cnt = wave_max(lcnt);
        L.n = readlane(wave_incl_add(lcnt), 63);
        L.starts = 1;
    } else {
        // every lane's point j is at rel r0 + j * dl (exact: all inside the
        // pass), so the lanes' range at point j is [rmin, rmax] + j * dl
        const uint32_t rmin = wave_min(lcnt ? r0 : 0xFFFFFFFFu);
        const uint32_t rmax = wave_max(lcnt ? r0 : 0u);
        const uint32_t cnt = readlane(lcnt, (uint32_t)__builtin_ctzll(live));
        const uint32_t j = lane();
        const bool pj = j < cnt;
        const uint32_t blo = (rmin + j * dl) >> sh, bhi = (rmax + j * dl) >> sh;
        if (__ballot(pj && blo != bhi)) return false;
        const uint32_t bprev = (rmin + (j - 1u) * dl) >> sh;
        L.pb = blo;
        L.cnt = cnt;
        L.n = cnt * (uint32_t)__popcll(live);
        L.starts = __ballot(pj && (j == 0u || blo != bprev));
    }
    return true;
}

// Thread-linear work items (flat mapping, one instance per thread): lane q
// takes gt consecutive threads, which differ in tx alone, so each index and
// the location are affine in the slot (steps row[.][tx] and fr[tx], ids step
// by the interval's per-thread count M).  tlin_probe succeeds (wave-
// uniformly) when every record of the wave is in bounds and inside the
// pass's key range, every live lane holds gt records, each lane's records
// share one bucket and the wave's buckets span fewer than WBIN; a lane is
// then ranked among the wave's lanes of its bucket with one LDS atomic.
struct TLinItem {
    uint32_t lcnt;          // records of this lane
    uint32_t hi, dhi;       // first record's key half, step per slot
    uint32_t id, did;       // first record's id, step per slot
    uint32_t bin;           // this lane's bucket relative to the wave's first
    uint32_t mn, R;         // the wave's first bucket (relative to the pass) and bucket span
    uint32_t n;             // records of the wave
};

template <bool PROVEN>
__device__ __forceinline__ bool tlin_probe(CSub &S, CEnt &E, CKer &K, uint32_t item, TLinItem &L) {
    const ItemStart<true> st = item_start<true>(E, K, item);
    const bool gval = st.g0 < K.nthreads;
    const uint32_t gg = gval ? st.g0 : 0u;
    const uint32_t blk = udiv(gg, ldm(K.mg_tpb));
    const uint32_t tid = gg - blk * K.tpb;
    const uint32_t byy = udiv(blk, ldm(K.mg_gdx));
    const uint32_t tyy = udiv(tid, ldm(K.mg_bdx));
    const uint32_t tx = tid - tyy * K.bdx, ty = tyy, bx = blk - byy * K.gdx, by = byy;
    const uint32_t L0 = (uint32_t)E.lo[0] + st.c0, L1 = (uint32_t)E.lo[1] + st.c1, L2 = (uint32_t)E.lo[2] + st.c2;
    const uint32_t lcnt = gval ? min(E.gt, K.nthreads - gg) : 0u;
    const uint32_t last = lcnt - 1u;
    const uint32_t loc = blk * E.loc_mul + E.fr[C_TX] * tx + E.fr[C_TY] * ty + E.fr[C_BX] * bx +
                         E.fr[C_BY] * by + E.fr[C_C0] + E.fr[C_L0] * L0 + E.fr[C_L1] * L1 + E.fr[C_L2] * L2;
    const uint32_t dl = E.fr[C_TX];
    bool good = true;
    if constexpr (!PROVEN) {
#pragma unroll
        for (int r = 0; r < 3; r++) {
            const uint32_t i0 = (uint32_t)E.row[r][C_TX] * tx + (uint32_t)E.row[r][C_TY] * ty +
                                (uint32_t)E.row[r][C_BX] * bx + (uint32_t)E.row[r][C_BY] * by +
                                (uint32_t)E.row[r][C_C0] + (uint32_t)E.row[r][C_L0] * L0 +
                                (uint32_t)E.row[r][C_L1] * L1 + (uint32_t)E.row[r][C_L2] * L2;
            const uint32_t iN = i0 + last * (uint32_t)E.row[r][C_TX];
            good = good && i0 < E.dim[r] && iN < E.dim[r];
        }
    }
    const uint32_t span = S.khi - S.klo;
    const uint32_t r0 = loc - S.klo, rN = loc + last * dl - S.klo;
    const uint32_t b0 = r0 >> S.s;
    good = lcnt == 0u || (good && lcnt == E.gt && r0 < span && rN < span && b0 == (rN >> S.s));
    if (__ballot(!good)) return false;
    const uint32_t mn = wave_min(lcnt ? b0 : 0xFFFFFFFFu);
    const uint32_t mx = wave_max(lcnt ? b0 : 0u);
    L.n = readlane(wave_incl_add(lcnt), 63);
    if (L.n && mx - mn >= WBIN) return false;
    L.lcnt = lcnt;
    L.hi = (loc << 1) | E.rw;
    L.dhi = dl << 1;
    L.id = gg * E.tmul + E.off;
    L.did = E.tmul;
    L.bin = b0 - mn;
    L.mn = mn;
    L.R = mx - mn + 1u;
    return true;
}

// Points in the run that lane j starts (j is a run start).
__device__ __forceinline__ uint32_t run_points(const LinItem &L, uint32_t j) {
    const uint64_t after = (L.starts >> j) >> 1;
    return (after ? j + 1u + (uint32_t)__builtin_ctzll(after) : L.cnt) - j;
}

// Run body(S, E, K, li, variant) over this workgroup's work items: chunks of
// up to ITEM_CHUNK consecutive items dealt out cyclically, so that items of
// very different cost (linear items that place their records without a rank,
// one-record-per-thread items that decode a thread per slot) spread evenly
// over the workgroups; launches with fewer items than ITEM_CHUNK per
// workgroup take smaller chunks, so that every workgroup gets work.
// Workgroups of one XCD (blockIdx.x mod 8) take adjacent chunks of each
// round.  Items of one entry are consecutive, so the entry's variant is
// chosen (and its constants loaded) once per entry inside a chunk rather
// than once per item.
constexpr uint32_t ITEM_CHUNK = 4;

// Chunk size for n units dealt cyclically over G workgroups: at most `cap`,
// and no more than one round's share when the units are few.
__device__ __forceinline__ uint32_t deal_chunk(uint32_t n, uint32_t G, uint32_t cap) {
    return max(1u, min(cap, (n + G - 1) / G));
}

template <class Body>
__device__ __forceinline__ void for_my_items(CSub *subs, uint32_t nsub, uint32_t nitems, Body &&body) {
    const uint32_t G = gridDim.x;                  // multiple of 8
    const uint32_t r = (blockIdx.x & 7u) * (G >> 3) + (blockIdx.x >> 3);
    const uint32_t ch = deal_chunk(nitems, G, ITEM_CHUNK);
    for (uint32_t w0 = r * ch; w0 < nitems; w0 += G * ch) {
        const uint32_t w1 = min(nitems, w0 + ch);
        Cursor cur;
        seek(subs, nsub, w0, cur);
        uint32_t w = w0;
        for (;;) {
            CSub &S = subs[cur.sub];
            CEnt &E = cptr(S.entries)[cur.e];
            CKer &K = *cptr(S.kc);
            const uint32_t n = min(w1 - w, cur.e_items - cur.li);
            const uint32_t l0 = cur.li;
            auto run = [&](auto variant) {
                for (uint32_t i = 0; i < n; i++) body(S, E, K, l0 + i, variant);
            };
            const uint32_t v = (E.flat ? 3u : 0u) + (E.fast == 2 ? 0u : E.fast ? 1u : 2u);
            switch (v) {
                case 0: run(Variant<0>{}); break;
                case 1: run(Variant<1>{}); break;
                case 2: run(Variant<2>{}); break;
                case 3: run(Variant<3>{}); break;
                case 4: run(Variant<4>{}); break;
                default: run(Variant<5>{}); break;
            }
            w += n;
            if (w >= w1) break;
            cur.li = l0 + n - 1;
            advance(subs, cur);
        }
    }
}

// ------------------------------------------------------------- fill kernels
__global__ void k_fill_u32(uint32_t *p, size_t n, uint32_t v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_init_results(SubResult *r, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        SubResult z;
        z.records = 0; z.conflicts = 0; z.oob = ~0ull; z.unit_records = 0;
        z.first_bucket = ~0u; z.first_unit = ~0u; z.pad = 0; z.pad2 = 0;
        z.w[0] = z.w[1] = z.w[2] = z.w[3] = 0;
        r[i] = z;
    }
}

// --------------------------------------------------------------- count pass
__global__ void __launch_bounds__(EXP_WG) k_hist(const DevSub *subs_g, uint32_t nsub, uint32_t nitems,
                                                  uint32_t *__restrict__ counts, SubResult *__restrict__ res) {
    __shared__ uint32_t h[BINCAP];
    __shared__ uint32_t red[3 * (EXP_WG / 64)];
    CSub *subs = cptr(subs_g);
    uint32_t *const hw = h + (threadIdx.x >> 6) * WBIN;
    for_my_items(subs, nsub, nitems, [&](CSub &S, CEnt &E, CKer &K, uint32_t li, auto variant) {
        // Fast entries count per wave (wave barriers only), so a wave may
        // finish an item on its own (linear items in one bucket); general
        // entries count per workgroup.
        constexpr int V = decltype(variant)::value;
        constexpr bool WAVE = V % 3 != 2;
        if (S.count_only) {
            // a pass without writes: its records and out-of-bounds instances
            // are counted, nothing else (the whole workgroup takes this
            // branch); with count_only 2 the host adds the records of entries
            // proven in bounds (fast ones, and general ones without guards)
            if (S.count_only == 2 && (V % 3 == 0 || (V % 3 == 2 && E.gproven))) return;
            uint32_t n = 0;
            const uint32_t klo = S.klo, span = S.khi - S.klo;
            expand_v(variant, S, E, K, li, [&](int, bool ok, bool inb, uint32_t loc, uint32_t id) {
                if (ok && !inb) atomicMin(&res[S.res].oob, ((unsigned long long)S.interval << 32) | id);
                n += (ok && inb && loc - klo < span) ? 1u : 0u;
            });
            n = readlane(wave_incl_add(n), 63);
            if (lane() == 0 && n) atomicAdd(&res[S.res].records, (unsigned long long)n);
            return;
        }
        uint32_t *gc = counts + S.bucket_begin;
        if constexpr (V == 3 || V == 4) {
            TLinItem T;
            if (E.tlin && tlin_probe<(V == 3)>(S, E, K, li, T)) {
                if (!T.n) return;
                for (uint32_t i = lane(); i < T.R; i += 64) hw[i] = 0;
                __builtin_amdgcn_wave_barrier();
                if (T.lcnt) atomicAdd(&hw[T.bin], T.lcnt);
                __builtin_amdgcn_wave_barrier();
                for (uint32_t i = lane(); i < T.R; i += 64) {
                    const uint32_t c = hw[i];
                    if (c) atomicAdd(&gc[T.mn + i], c);
                }
                __builtin_amdgcn_wave_barrier();
                if (lane() == 0) atomicAdd(&res[S.res].records, (unsigned long long)T.n);
                return;
            }
        }
        if constexpr (WAVE) {
            LinItem L;
            if (E.lin && lin_probe<(V >= 3), (V % 3 == 0)>(S, E, K, li, L)) {
                if (!L.n) return;
                const uint32_t j = lane();
                if ((L.starts >> j) & 1u)   // flat items: one run of all L.n records
                    atomicAdd(&gc[L.pb], V >= 3 ? L.n : run_points(L, j) * (uint32_t)__popcll(L.live));
                if (j == 0) atomicAdd(&res[S.res].records, (unsigned long long)L.n);
                return;
            }
        }
        const uint32_t span = S.khi - S.klo;
        uint32_t bk[RPL];
        uint32_t mn = 0xFFFFFFFFu, mx = 0, n = 0;
        const uint32_t klo = S.klo, sh = S.s;
        auto on_rec = [&](int s, bool ok, bool inb, uint32_t loc, uint32_t id) {
            if (ok && !inb) atomicMin(&res[S.res].oob, ((unsigned long long)S.interval << 32) | id);
            const uint32_t rel = loc - klo;
            const bool v = ok && inb && rel < span;
            const uint32_t b = rel >> sh;
            bk[s] = v ? b : 0xFFFFFFFFu;
            if (v) { mn = min(mn, b); mx = max(mx, b); n++; }
        };
        expand_v(variant, S, E, K, li, on_rec);
        if constexpr (WAVE) {
            mn = wave_min(mn);
            mx = wave_max(mx);
            n = readlane(wave_incl_add(n), 63);
            if (!n) return;
            if (lane() == 0) atomicAdd(&res[S.res].records, (unsigned long long)n);
            if (mx - mn < WBIN * WWIN) {
                for (uint32_t w = mn;; w += WBIN) {
                    const uint32_t R = min(WBIN, mx - w + 1);
                    for (uint32_t i = lane(); i < R; i += 64) hw[i] = 0;
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int s = 0; s < RPL; s++) lds_rank(hw, bk[s] - w, bk[s] - w < R);
                    __builtin_amdgcn_wave_barrier();
                    for (uint32_t i = lane(); i < R; i += 64) {
                        const uint32_t c = hw[i];
                        if (c) atomicAdd(&gc[w + i], c);
                    }
                    __builtin_amdgcn_wave_barrier();
                    if (mx - w < WBIN) break;
                }
                return;
            }
        } else {
            block_min_max_sum<EXP_WG>(mn, mx, n, red);
            if (!n) return;
            if (threadIdx.x == 0) atomicAdd(&res[S.res].records, (unsigned long long)n);
            if (mx - mn < (uint32_t)(BINCAP * BINWIN)) {
                // LDS bins over windows of BINCAP buckets of the tile's range
                for (uint32_t w = mn;; w += BINCAP) {
                    const uint32_t R = min((uint32_t)BINCAP, mx - w + 1);
                    for (uint32_t i = threadIdx.x; i < R; i += EXP_WG) h[i] = 0;
                    __syncthreads();
#pragma unroll
                    for (int s = 0; s < RPL; s++) lds_rank(h, bk[s] - w, bk[s] - w < R);
                    __syncthreads();
                    for (uint32_t i = threadIdx.x; i < R; i += EXP_WG) {
                        const uint32_t c = h[i];
                        if (c) atomicAdd(&gc[w + i], c);
                    }
                    __syncthreads();
                    if (mx - w < (uint32_t)BINCAP) break;
                }
                return;
            }
        }
        // records spread over more buckets than the windows cover
#pragma unroll
        for (int s = 0; s < RPL; s++) {
            const bool v = bk[s] != 0xFFFFFFFFu;
            const uint64_t act = __ballot(v);
            if (!act) continue;
            const uint32_t lead = (uint32_t)__builtin_ctzll(act);
            const uint32_t lb = readlane(bk[s], lead);
            if (__ballot(v && bk[s] == lb) == act) {
                if (lane() == lead) atomicAdd(&gc[lb], (uint32_t)__popcll(act));
            } else if (v) {
                atomicAdd(&gc[bk[s]], 1u);
            }
        }
    });
}

// ------------------------------------------------------------------ scans
constexpr int SCAN_WG = 256, SCAN_PER = 16, SCAN_TILE = SCAN_WG * SCAN_PER;

__global__ void __launch_bounds__(SCAN_WG) k_scan_up(const uint32_t *__restrict__ in, size_t n,
                                                      uint32_t *__restrict__ bsum) {
    __shared__ uint32_t red[SCAN_WG / 64];
    const size_t base = (size_t)blockIdx.x * SCAN_TILE;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_PER; i++) {
        const size_t j = base + (size_t)i * SCAN_WG + threadIdx.x;
        s += j < n ? in[j] : 0u;
    }
    uint32_t tot;
    block_excl_add<SCAN_WG>(s, red, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of nb block sums in place; the grand total
// goes to bsum[nb].
__global__ void __launch_bounds__(SCAN_WG) k_scan_mid(uint32_t *bsum, uint32_t nb) {
    __shared__ uint32_t red[SCAN_WG / 64];
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += SCAN_WG) {
        const uint32_t j = b0 + threadIdx.x;
        const uint32_t v = j < nb ? bsum[j] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_add<SCAN_WG>(v, red, &tot);
        if (j < nb) bsum[j] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ void __launch_bounds__(SCAN_WG) k_scan_down(const uint32_t *__restrict__ in, size_t n,
                                                        const uint32_t *__restrict__ bsum,
                                                        uint32_t *__restrict__ out1, uint32_t *__restrict__ out2) {
    __shared__ uint32_t red[SCAN_WG / 64];
    // each thread owns SCAN_PER consecutive elements
    const size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_PER;
    uint32_t v[SCAN_PER];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_PER; i++) {
        v[i] = base + i < n ? in[base + i] : 0u;
        s += v[i];
    }
    uint32_t tot;
    uint32_t run = bsum[blockIdx.x] + block_excl_add<SCAN_WG>(s, red, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_PER; i++) {
        if (base + i < n) {
            out1[base + i] = run;
            if (out2) out2[base + i] = run;
        }
        run += v[i];
    }
}

// -------------------------------------------------------------- expansion
__global__ void __launch_bounds__(EXP_WG) __attribute__((amdgpu_waves_per_eu(5))) k_scatter(const DevSub *subs_g, uint32_t nsub, uint32_t nitems,
                                                     unsigned long long *__restrict__ rec,
                                                     uint32_t *__restrict__ cursor) {
    // One LDS area, used per workgroup (h, gb: BINCAP bins each) for entries
    // of the general expansion, or per wave (WBIN bins each) for fast ones.
    __shared__ uint32_t bins[2 * BINCAP];
    __shared__ uint32_t red[3 * (EXP_WG / 64)];
    CSub *subs = cptr(subs_g);
    uint32_t *const hw = bins + (threadIdx.x >> 6) * 2 * WBIN, *const gw = hw + WBIN;
    for_my_items(subs, nsub, nitems, [&](CSub &S, CEnt &E, CKer &K, uint32_t li, auto variant) {
        constexpr int V = decltype(variant)::value;
        if (S.count_only) return;          // a pass without writes has no records to place
        if constexpr (V == 3 || V == 4) {
            TLinItem T;
            if (E.tlin && tlin_probe<(V == 3)>(S, E, K, li, T)) {
                // one LDS rank per lane among the wave's lanes of its bucket,
                // one reservation per bucket (gt records per lane); slot q of
                // the lane ranked k goes to base + q x lanes + k, so the lanes
                // of a bucket store to consecutive addresses
                if (!T.n) return;
                for (uint32_t i = lane(); i < T.R; i += 64) hw[i] = 0;
                __builtin_amdgcn_wave_barrier();
                uint32_t rk = 0;
                if (T.lcnt) rk = atomicAdd(&hw[T.bin], 1u);
                __builtin_amdgcn_wave_barrier();
                for (uint32_t i = lane(); i < T.R; i += 64) {
                    const uint32_t c = hw[i];
                    if (c) gw[i] = atomicAdd(&cursor[S.bucket_begin + T.mn + i], c * E.gt);
                }
                __builtin_amdgcn_wave_barrier();
                if (T.lcnt) {
                    const uint32_t lanes = hw[T.bin];
                    unsigned long long *p = rec + gw[T.bin] + rk;
                    uint32_t hi = T.hi, id = T.id;
                    for (uint32_t q = 0; q < T.lcnt; q++) {
                        p[(size_t)q * lanes] = ((unsigned long long)hi << 32) | id;
                        hi += T.dhi;
                        id += T.did;
                    }
                }
                __builtin_amdgcn_wave_barrier();
                return;
            }
        }
        if constexpr (V % 3 != 2) {
            LinItem L;
            if (E.lin && lin_probe<(V >= 3), (V % 3 == 0)>(S, E, K, li, L)) {
                // one reservation per run of points; records go point by
                // point, each point's lanes to consecutive addresses
                if (!L.n) return;
                const uint32_t j = lane();
                uint32_t hi = L.hi, id = L.id;
                if constexpr (V < 3) {
                    const uint32_t P = (uint32_t)__popcll(L.live);
                    uint32_t rb = 0;
                    if ((L.starts >> j) & 1u) rb = atomicAdd(&cursor[S.bucket_begin + L.pb], run_points(L, j) * P);
                    // lane j < cnt: the first slot of point j
                    const uint64_t upto = L.starts & ((2ull << (j & 63u)) - 1ull);
                    const uint32_t sj = upto ? 63u - (uint32_t)__builtin_clzll(upto) : 0u;
                    const uint32_t pt = (uint32_t)__shfl((int)rb, (int)sj) + (j - sj) * P;
                    // every lane runs the loop (point bases are read from
                    // lanes that may hold no records); live lanes store
                    const uint32_t mb = mbcnt(L.live);
                    const bool mine = L.lcnt != 0u;
                    for (uint32_t q = 0; q < L.cnt; q++) {
                        const uint32_t at = readlane(pt, q) + mb;
                        if (mine) rec[at] = ((unsigned long long)hi << 32) | id;
                        hi += L.dhi;
                        id++;
                    }
                } else {
                    uint32_t base = 0;
                    if (j == 0) base = atomicAdd(&cursor[S.bucket_begin + L.pb], L.n);
                    base = readlane(base, 0);
                    for (uint32_t q = 0; q < L.cnt; q++) {
                        const bool v = q < L.lcnt;
                        const uint64_t act = __ballot(v);
                        if (v) rec[base + mbcnt(act)] = ((unsigned long long)hi << 32) | id;
                        base += (uint32_t)__popcll(act);
                        hi += L.dhi;
                        id++;
                    }
                }
                return;
            }
        }
        const uint32_t span = S.khi - S.klo;
        const uint32_t rwbit = E.rw;
        unsigned long long r[RPL];
        uint32_t bk[RPL];
        uint32_t mn = 0xFFFFFFFFu, mx = 0, n = 0;
        const uint32_t klo = S.klo, sh = S.s;
        auto on_rec = [&](int s, bool ok, bool inb, uint32_t loc, uint32_t id) {
            const uint32_t rel = loc - klo;
            const bool v = ok && inb && rel < span;
            const uint32_t b = rel >> sh;
            bk[s] = v ? b : 0xFFFFFFFFu;
            r[s] = ((unsigned long long)((loc << 1) | rwbit) << 32) | id;
            if (v) { mn = min(mn, b); mx = max(mx, b); n++; }
        };
        expand_v(variant, S, E, K, li, on_rec);
        // Fast entries (structured addresses: a wave's records span few
        // buckets) rank per wave, with no workgroup barrier; general entries
        // rank per workgroup, whose longer runs pay off for scattered ones.
        constexpr bool WAVE = decltype(variant)::value % 3 != 2;
        if constexpr (WAVE) {
            mn = wave_min(mn);
            mx = wave_max(mx);
            n = readlane(wave_incl_add(n), 63);
        } else {
            block_min_max_sum<EXP_WG>(mn, mx, n, red);
        }
        uint32_t *gcur = cursor + S.bucket_begin;
        // Rank every record inside its bucket (per wave or per workgroup),
        // reserve one run per bucket in the chunk, write each record to run
        // base + rank; a wave slot whose records share a bucket writes one
        // contiguous 512-byte run.  Windows of WBIN / BINCAP buckets.
        if constexpr (WAVE) {
            if (n && mx - mn < WBIN * WWIN) {
                for (uint32_t w = mn;; w += WBIN) {
                    const uint32_t R = min(WBIN, mx - w + 1);
                    for (uint32_t i = lane(); i < R; i += 64) hw[i] = 0;
                    __builtin_amdgcn_wave_barrier();
                    uint32_t rk[RPL];
#pragma unroll
                    for (int s = 0; s < RPL; s++) rk[s] = lds_rank(hw, bk[s] - w, bk[s] - w < R);
                    __builtin_amdgcn_wave_barrier();
                    for (uint32_t i = lane(); i < R; i += 64) {
                        const uint32_t c = hw[i];
                        if (c) gw[i] = atomicAdd(&gcur[w + i], c);
                    }
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int s = 0; s < RPL; s++)
                        if (bk[s] - w < R) rec[gw[bk[s] - w] + rk[s]] = r[s];
                    __builtin_amdgcn_wave_barrier();
                    if (mx - w < WBIN) break;
                }
                return;
            }
        } else {
            if (n && mx - mn < (uint32_t)(BINCAP * BINWIN)) {
                uint32_t *h = bins, *gb = bins + BINCAP;
                for (uint32_t w = mn;; w += BINCAP) {
                    const uint32_t R = min((uint32_t)BINCAP, mx - w + 1);
                    for (uint32_t i = threadIdx.x; i < R; i += EXP_WG) h[i] = 0;
                    __syncthreads();
                    uint32_t rk[RPL];
#pragma unroll
                    for (int s = 0; s < RPL; s++) rk[s] = lds_rank(h, bk[s] - w, bk[s] - w < R);
                    __syncthreads();
                    for (uint32_t i = threadIdx.x; i < R; i += EXP_WG) {
                        const uint32_t c = h[i];
                        if (c) gb[i] = atomicAdd(&gcur[w + i], c);
                    }
                    __syncthreads();
#pragma unroll
                    for (int s = 0; s < RPL; s++)
                        if (bk[s] - w < R) rec[gb[bk[s] - w] + rk[s]] = r[s];
                    __syncthreads();
                    if (mx - w < (uint32_t)BINCAP) break;
                }
                return;
            }
        }
        if (n) {
            // records spread over more buckets than the windows cover (so many
            // that their counters rarely collide): reserve per record
#pragma unroll
            for (int s = 0; s < RPL; s++) {
                const bool v = bk[s] != 0xFFFFFFFFu;
                const uint64_t act = __ballot(v);
                if (!act) continue;
                const uint32_t lead = (uint32_t)__builtin_ctzll(act);
                const uint32_t lb = readlane(bk[s], lead);
                uint32_t pos = 0;
                if (__ballot(v && bk[s] == lb) == act) {
                    if (lane() == lead) pos = atomicAdd(&gcur[lb], (uint32_t)__popcll(act));
                    pos = readlane(pos, lead) + mbcnt(act);
                } else if (v) {
                    pos = atomicAdd(&gcur[bk[s]], 1u);
                }
                if (v) rec[pos] = r[s];
            }
        }
    });
}

// ------------------------------------------------ sort + segmented scan
// Per-location summary: min id, max id, min write id, max write id + 1.
struct Seg {
    uint32_t f, mn, mx, mnw, mxw1;
};

__device__ __forceinline__ void seg_add(Seg &a, uint32_t id, uint32_t w) {
    a.mn = min(a.mn, id);
    a.mx = max(a.mx, id);
    a.mnw = min(a.mnw, w ? id : 0xFFFFFFFFu);
    a.mxw1 = max(a.mxw1, w ? id + 1 : 0u);
}

// a <- prev (+) a for the segmented operator: a.f ? a : reduce(prev, a).
template <int CTRL, int RM>
__device__ __forceinline__ void seg_dpp_step(Seg &a) {
    const uint32_t pf = dpp<CTRL, RM>(0u, a.f);
    const uint32_t pmn = dpp<CTRL, RM>(0xFFFFFFFFu, a.mn);
    const uint32_t pmx = dpp<CTRL, RM>(0u, a.mx);
    const uint32_t pmnw = dpp<CTRL, RM>(0xFFFFFFFFu, a.mnw);
    const uint32_t pmxw1 = dpp<CTRL, RM>(0u, a.mxw1);
    if (!a.f) {
        a.mn = min(a.mn, pmn);
        a.mx = max(a.mx, pmx);
        a.mnw = min(a.mnw, pmnw);
        a.mxw1 = max(a.mxw1, pmxw1);
    }
    a.f |= pf;
}

__device__ __forceinline__ Seg shfl_up1(const Seg &a) {
    Seg p;
    p.f = __shfl_up(a.f, 1);
    p.mn = __shfl_up(a.mn, 1);
    p.mx = __shfl_up(a.mx, 1);
    p.mnw = __shfl_up(a.mnw, 1);
    p.mxw1 = __shfl_up(a.mxw1, 1);
    if (lane() == 0) { p.f = 0; p.mn = 0xFFFFFFFFu; p.mx = 0; p.mnw = 0xFFFFFFFFu; p.mxw1 = 0; }
    return p;
}

__device__ __forceinline__ void seg_combine(Seg &acc, const Seg &b) {   // acc <- acc (+) b
    acc.mn = b.f ? b.mn : min(acc.mn, b.mn);
    acc.mx = b.f ? b.mx : max(acc.mx, b.mx);
    acc.mnw = b.f ? b.mnw : min(acc.mnw, b.mnw);
    acc.mxw1 = b.f ? b.mxw1 : max(acc.mxw1, b.mxw1);
    acc.f |= b.f;
}

constexpr int TPER = TBL / BKT_WG;           // table entries per thread
static_assert(TBL % BKT_WG == 0, "table split");

__device__ __forceinline__ void fold(uint32_t *t_mn, uint32_t *t_mx, uint32_t *t_mnw, uint32_t *t_mxw1,
                                     uint32_t k, const Seg &s) {
    atomicMin(&t_mn[k], s.mn);
    atomicMax(&t_mx[k], s.mx);
    atomicMin(&t_mnw[k], s.mnw);
    atomicMax(&t_mxw1[k], s.mxw1);
}

// Conflict test and canonical witness of one location's summary.
__device__ __forceinline__ bool judge(const Seg &s, Magic mgM, uint32_t &second, uint32_t &srw) {
    if (s.mxw1 == 0u || s.mn == s.mx) return false;          // no write, or one record
    const uint32_t th_mn = udiv(s.mn, mgM), th_mx = udiv(s.mx, mgM);
    if (th_mn == th_mx) return false;                         // one thread
    const uint32_t th_w = udiv(s.mnw, mgM);
    if (th_mn != th_w) { second = s.mn; srw = (s.mn == s.mnw) ? 1u : 0u; }
    else { second = s.mx; srw = (s.mx + 1 == s.mxw1) ? 1u : 0u; }
    return true;
}

__device__ __forceinline__ void put_witness(uint32_t *wout, uint32_t pos, uint32_t loc, const Seg &s,
                                            uint32_t second, uint32_t srw) {
    uint32_t *w = wout + 4 * (size_t)pos;    // the region start is 8-byte aligned: store words
    w[0] = loc; w[1] = s.mnw; w[2] = second; w[3] = srw;
}

// Sorted slice in LDS: element p (sorted position) lives at padded slot
// (p / rpl) * stride + p % rpl, so that lane t's run [t*rpl, t*rpl + rpl)
// starts at t*stride with an odd stride: the lanes of a wave then read
// different banks.  Each slot holds (local key | rw << 15) << 32 | id.
constexpr int SRT_SLOTS = CAP + BKT_WG;

__global__ void __launch_bounds__(BKT_WG) k_bucket(const DevSub *subs_g, uint32_t nsub, uint32_t nbuckets,
                                                    unsigned long long *__restrict__ rec,
                                                    const uint32_t *__restrict__ starts,
                                                    const uint32_t *__restrict__ counts,
                                                    uint32_t *__restrict__ conf, int debug_sorted) {
    __shared__ unsigned long long srt[SRT_SLOTS];
    __shared__ uint32_t bins[TBL];
    __shared__ uint32_t t_mn[TBL], t_mx[TBL], t_mnw[TBL], t_mxw1[TBL];
    __shared__ Seg wtot[BKT_WG / 64];
    __shared__ uint32_t red[BKT_WG / 64];
    CSub *subs = cptr(subs_g);
    const uint32_t t = threadIdx.x;
    const uint32_t wid = t >> 6;

    uint32_t lo_s = 0;      // pass of the current bucket: buckets only increase, so walk forward
    {
        uint32_t hi_s = nsub;
        while (hi_s - lo_s > 1) {
            const uint32_t mid = (lo_s + hi_s) >> 1;
            if (subs[mid].bucket_begin <= blockIdx.x) lo_s = mid; else hi_s = mid;
        }
    }
    for (uint32_t b = blockIdx.x; b < nbuckets; b += gridDim.x) {
        const uint32_t cnt = counts[b];
        if (cnt == 0) {
            if (t == 0) conf[b] = 0;
            continue;
        }
        while (b >= subs[lo_s].bucket_begin + subs[lo_s].nb) lo_s++;
        CSub &S = subs[lo_s];
        const Magic mgM = ldm(S.mgM);
        const uint32_t nbins = 1u << S.s;
        const uint32_t lo = S.klo + ((b - S.bucket_begin) << S.s);
        const uint32_t width = min(nbins, S.khi - lo);
        const uint32_t start = starts[b];
        const bool single = cnt <= (uint32_t)CAP;
        if (!single) {
#pragma unroll
            for (int i = 0; i < TPER; i++) {
                const uint32_t k = t * TPER + i;
                t_mn[k] = 0xFFFFFFFFu; t_mx[k] = 0; t_mnw[k] = 0xFFFFFFFFu; t_mxw1[k] = 0;
            }
        }
        uint32_t nconf = 0;      // conflicts this thread finalized (single-slice path)
        for (uint32_t slice = 0; slice < cnt; slice += CAP) {
            const uint32_t n = min((uint32_t)CAP, cnt - slice);
            const uint32_t rpl = (n + BKT_WG - 1) / BKT_WG;           // records per lane, 1..BKT_RPL
            const uint32_t stride = rpl | 1u;
            const uint32_t rdiv = ((1u << 20) + rpl - 1) / rpl;          // p / rpl == (p * rdiv) >> 20 for p < 2^12
            const uint32_t r0 = t * rpl;
            const uint32_t m = r0 < n ? min(rpl, n - r0) : 0u;          // this lane's records
            const unsigned long long *src = rec + start + slice + r0;
            // --- load a contiguous run per lane: ids and keys (local key | rw << 15)
            uint32_t kw[BKT_RPL], id[BKT_RPL];
#pragma unroll
            for (int i = 0; i < BKT_RPL; i++) {
                const unsigned long long x = (uint32_t)i < m ? src[i] : 0ull;
                const uint32_t hi = (uint32_t)(x >> 32);
                id[i] = (uint32_t)x;
                kw[i] = ((hi >> 1) - lo) | ((hi & 1u) << 15);
            }
            for (uint32_t k = t; k < nbins; k += BKT_WG) bins[k] = 0;
            __syncthreads();
            // --- LDS radix sort, one counting-sort digit of `s` bits.  Each
            // record takes its rank with one LDS atomic; lanes hold
            // contiguous runs, so the lanes of one atomic rarely share a key.
            uint32_t off[BKT_RPL];
#pragma unroll
            for (int i = 0; i < BKT_RPL; i++)
                off[i] = (uint32_t)i < m ? atomicAdd(&bins[kw[i] & 0x7FFFu], 1u) : 0u;
            __syncthreads();
            {
                uint32_t hv[TPER], sum = 0, tot;
#pragma unroll
                for (int i = 0; i < TPER; i++) {
                    const uint32_t k = t * TPER + i;
                    hv[i] = k < nbins ? bins[k] : 0u;
                    sum += hv[i];
                }
                uint32_t run = block_excl_add<BKT_WG>(sum, red, &tot);
#pragma unroll
                for (int i = 0; i < TPER; i++) {
                    const uint32_t k = t * TPER + i;
                    if (k < nbins) bins[k] = run;
                    run += hv[i];
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < BKT_RPL; i++) {
                if ((uint32_t)i < m) {
                    const uint32_t p = bins[kw[i] & 0x7FFFu] + off[i];
                    const uint32_t q = (p * rdiv) >> 20;
                    srt[q * stride + (p - q * rpl)] = ((unsigned long long)kw[i] << 32) | id[i];
                }
            }
            __syncthreads();
            if (debug_sorted) {
                for (uint32_t j = t; j < n; j += BKT_WG) {
                    const uint32_t q = (j * rdiv) >> 20;
                    const unsigned long long x = srt[q * stride + (j - q * rpl)];
                    const uint32_t key = (uint32_t)(x >> 32);
                    const uint32_t hi = ((lo + (key & 0x7FFFu)) << 1) | (key >> 15);
                    rec[start + slice + j] = ((unsigned long long)hi << 32) | (uint32_t)x;
                }
            }
            // --- segmented scan over this lane's sorted run (same positions r0 .. r0 + m)
            uint32_t kv[BKT_RPL], iv[BKT_RPL];
            const unsigned long long *mine = srt + t * stride;
#pragma unroll
            for (int i = 0; i < BKT_RPL; i++) {
                const unsigned long long x = (uint32_t)i < m ? mine[i] : 0ull;
                kv[i] = (uint32_t)(x >> 32);
                iv[i] = (uint32_t)x;
            }
            const uint32_t prevk = (t > 0 && m) ? ((uint32_t)(srt[(t - 1) * stride + rpl - 1] >> 32) & 0x7FFFu) : 0xFFFFu;
            const uint32_t nextk = (m && r0 + m < n) ? ((uint32_t)(srt[(t + 1) * stride] >> 32) & 0x7FFFu) : 0xFFFFu;
            Seg a{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
            {
                uint32_t pk = prevk;
#pragma unroll
                for (int j = 0; j < BKT_RPL; j++) {
                    if ((uint32_t)j < m) {
                        const uint32_t k = kv[j] & 0x7FFFu;
                        if (k != pk) { a.f = 1; a.mn = 0xFFFFFFFFu; a.mx = 0; a.mnw = 0xFFFFFFFFu; a.mxw1 = 0; }
                        seg_add(a, iv[j], kv[j] >> 15);
                        pk = k;
                    }
                }
            }
            Seg inc = a;
            seg_dpp_step<ROW_SHR1, 0xf>(inc);
            seg_dpp_step<ROW_SHR2, 0xf>(inc);
            seg_dpp_step<ROW_SHR4, 0xf>(inc);
            seg_dpp_step<ROW_SHR8, 0xf>(inc);
            seg_dpp_step<ROW_BCAST15, 0xa>(inc);
            seg_dpp_step<ROW_BCAST31, 0xc>(inc);
            if (lane() == 63) wtot[wid] = inc;
            Seg carry = shfl_up1(inc);
            __syncthreads();
            {
                Seg wc{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
                for (uint32_t w = 0; w < wid; w++) seg_combine(wc, wtot[w]);
                seg_combine(wc, carry);
                carry = wc;
            }
            // Walk the run and finalize the segments that end inside it.
            // pass 0: count (single slice) or fold (several slices); pass 1: write witnesses.
            auto walk = [&](int pass, uint32_t pos) {
                Seg cur;
                const bool head0 = m && ((kv[0] & 0x7FFFu) != prevk);
                cur.f = 0;
                cur.mn = head0 ? 0xFFFFFFFFu : carry.mn;
                cur.mx = head0 ? 0u : carry.mx;
                cur.mnw = head0 ? 0xFFFFFFFFu : carry.mnw;
                cur.mxw1 = head0 ? 0u : carry.mxw1;
                uint32_t pk = m ? (kv[0] & 0x7FFFu) : 0u;
                uint32_t *wout = reinterpret_cast<uint32_t *>(rec + start);
#pragma unroll
                for (int j = 0; j < BKT_RPL; j++) {
                    if ((uint32_t)j < m) {
                        const uint32_t k = kv[j] & 0x7FFFu;
                        if (j != 0 && k != pk) {
                            if (!single) {
                                fold(t_mn, t_mx, t_mnw, t_mxw1, pk, cur);
                            } else {
                                uint32_t sec = 0, srw = 0;
                                if (judge(cur, mgM, sec, srw)) {
                                    if (pass) put_witness(wout, pos++, lo + pk, cur, sec, srw);
                                    else nconf++;
                                }
                            }
                            cur.mn = 0xFFFFFFFFu; cur.mx = 0; cur.mnw = 0xFFFFFFFFu; cur.mxw1 = 0;
                        }
                        seg_add(cur, iv[j], kv[j] >> 15);
                        pk = k;
                    }
                }
                if (m && nextk != pk) {   // the last segment ends here too
                    if (!single) {
                        fold(t_mn, t_mx, t_mnw, t_mxw1, pk, cur);
                    } else {
                        uint32_t sec = 0, srw = 0;
                        if (judge(cur, mgM, sec, srw)) {
                            if (pass) put_witness(wout, pos++, lo + pk, cur, sec, srw);
                            else nconf++;
                        }
                    }
                }
            };
            walk(0, 0);
            if (single) {
                uint32_t total;
                const uint32_t pos = block_excl_add<BKT_WG>(nconf, red, &total);
                if (total && !debug_sorted) walk(1, pos);
                if (t == 0) conf[b] = total;
            }
            __syncthreads();
        }
        if (single) continue;

        // --- several slices: flag the folded locations, in key order
        bool c[TPER];
        Seg e[TPER];
        uint32_t second[TPER], srw[TPER];
        uint32_t nc = 0;
#pragma unroll
        for (int i = 0; i < TPER; i++) {
            const uint32_t k = t * TPER + i;
            c[i] = false; second[i] = 0; srw[i] = 0;
            e[i] = Seg{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
            if (k < width) {
                e[i].mn = t_mn[k]; e[i].mx = t_mx[k]; e[i].mnw = t_mnw[k]; e[i].mxw1 = t_mxw1[k];
                if (e[i].mn != 0xFFFFFFFFu) c[i] = judge(e[i], mgM, second[i], srw[i]);
            }
            nc += c[i] ? 1u : 0u;
        }
        uint32_t total;
        uint32_t pos = block_excl_add<BKT_WG>(nc, red, &total);
        if (!debug_sorted) {
            uint32_t *wout = reinterpret_cast<uint32_t *>(rec + start);
#pragma unroll
            for (int i = 0; i < TPER; i++)
                if (c[i]) put_witness(wout, pos++, lo + t * TPER + i, e[i], second[i], srw[i]);
        }
        if (t == 0) conf[b] = total;
    }
}

// Grouping without sorting.  Each location of a bucket owns one slot of four
// LDS tables (min id, max id, min write id, max write id + 1: the summary the
// segmented scan produces), and records are folded into their slot with LDS
// atomics.  A lane first merges consecutive records of equal location in
// registers (it loads a contiguous run), so a run of one location costs one
// set of atomics.  The judge and the witness order (location order, from a
// prefix sum of per-lane counts) match the sorting path exactly.
//
// k_fold gives each workgroup a contiguous range of buckets.  It reads the
// range's counts 256 at a time, lists the non-empty ones in LDS (a bucket of
// more than HOT records, a hot location, goes to the hot list for k_hot), and
// while it folds one bucket the records of the next are already loading into
// registers.

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Records of a lane's contiguous run of one slice: slice of n records, lane
// `me` of NL takes [me * rpl, me * rpl + m).
struct __attribute__((aligned(8))) RecPair {
    unsigned long long a, b;
};
static_assert(FOLD_RPL % 2 == 0, "fold runs load records in pairs");

template <int NL>
struct Run {
    uint32_t rpl, m;
    unsigned long long x[FOLD_RPL];
};

template <int NL>
__device__ __forceinline__ void run_load(Run<NL> &r, const unsigned long long *__restrict__ src, uint32_t n,
                                         uint32_t me) {
    r.rpl = (n + NL - 1) / NL;
    const uint32_t r0 = me * r.rpl;
    r.m = r0 < n ? min(r.rpl, n - r0) : 0u;
    // Every lane issues all its loads (indices clamped into its run, or to
    // the slice's first record), so the loads are unconditional and the
    // compiler can leave them in flight while the previous bucket is folded.
    // Entries at or past m are never read (run_fold stops at m).
    // Loads go in pairs of records (16 bytes, 8-byte aligned: one dwordx4
    // per pair), the last pair starting at the run's last even index; a pair
    // may read one record past the lane's run, at most one past the slice
    // (the record area keeps a record of slack at its end).
    const unsigned long long *p = src + (r.m ? r0 : 0u);
    const uint32_t lastp = r.m ? (r.m - 1u) & ~1u : 0u;
#pragma unroll
    for (int j = 0; j < FOLD_RPL / 2; j++) {
        const RecPair v = *reinterpret_cast<const RecPair *>(p + min((uint32_t)(2 * j), lastp));
        r.x[2 * j] = v.a;
        r.x[2 * j + 1] = v.b;
    }
}

// A lane's merge state: the summary of the run of equal location it is
// accumulating (location pk, 0xFFFF: none) and the flush of that run into
// the location's LDS slot.
struct Merge {
    Seg cur;
    uint32_t pk;
};

__device__ __forceinline__ void merge_init(Merge &g) {
    g.cur = Seg{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
    g.pk = 0xFFFFu;
}

__device__ __forceinline__ void merge_flush(Merge &g, uint32_t *t_mn, uint32_t *t_mx, uint32_t *t_mnw,
                                            uint32_t *t_mxw1) {
    if (g.pk == 0xFFFFu) return;
    const uint32_t k = g.pk;
    atomicMin(&t_mn[k], g.cur.mn);
    atomicMax(&t_mx[k], g.cur.mx);
    if (g.cur.mxw1) {
        atomicMin(&t_mnw[k], g.cur.mnw);
        atomicMax(&t_mxw1[k], g.cur.mxw1);
    }
}

// Fold one lane's run into the tables: consecutive records of equal location
// are merged in registers, one set of atomics per merged run.  The run in
// progress stays in `g` (the caller flushes it), so a location spanning
// several slices costs one set of atomics.
template <int NL>
__device__ __forceinline__ void run_merge(const Run<NL> &r, uint32_t lo, Merge &g, uint32_t *t_mn, uint32_t *t_mx,
                                          uint32_t *t_mnw, uint32_t *t_mxw1) {
#pragma unroll
    for (int j = 0; j < FOLD_RPL; j++) {
        if ((uint32_t)j < r.m) {
            const uint32_t hi = (uint32_t)(r.x[j] >> 32);
            const uint32_t k = (hi >> 1) - lo;
            if (k != g.pk) {
                merge_flush(g, t_mn, t_mx, t_mnw, t_mxw1);
                g.cur = Seg{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
                g.pk = k;
            }
            seg_add(g.cur, (uint32_t)r.x[j], hi & 1u);
        }
    }
}

template <int NL>
__device__ __forceinline__ void run_fold(const Run<NL> &r, uint32_t lo, uint32_t *t_mn, uint32_t *t_mx,
                                         uint32_t *t_mnw, uint32_t *t_mxw1) {
    Seg cur{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
    uint32_t pk = 0xFFFFu;
    auto flush = [&](uint32_t k) {
        atomicMin(&t_mn[k], cur.mn);
        atomicMax(&t_mx[k], cur.mx);
        if (cur.mxw1) {
            atomicMin(&t_mnw[k], cur.mnw);
            atomicMax(&t_mxw1[k], cur.mxw1);
        }
    };
#pragma unroll
    for (int j = 0; j < FOLD_RPL; j++) {
        if ((uint32_t)j < r.m) {
            const uint32_t hi = (uint32_t)(r.x[j] >> 32);
            const uint32_t k = (hi >> 1) - lo;
            if (k != pk) {
                if (pk != 0xFFFFu) flush(pk);
                cur.mn = 0xFFFFFFFFu; cur.mx = 0; cur.mnw = 0xFFFFFFFFu; cur.mxw1 = 0;
                pk = k;
            }
            seg_add(cur, (uint32_t)r.x[j], hi & 1u);
        }
    }
    if (pk != 0xFFFFu) flush(pk);
}

// Fold records [r_begin, r_end) of one bucket in slices of NL * FOLD_RPL.
// Each lane keeps its merge state from one slice to the next (its runs are
// consecutive records of consecutive slices only in hot, single-location
// stretches, which is where it matters: one flush per lane per call).
// Two register sets alternate, as in the fold: while one slice is merged
// the next one is loading.  A slice past r_end loads nothing of its own (its
// clamped loads read the first records, m = 0), so every load is issued
// unconditionally.
template <int NL>
__device__ __forceinline__ void fold_records(const unsigned long long *__restrict__ src, uint32_t r_begin,
                                             uint32_t r_end, uint32_t lo, uint32_t me, uint32_t *t_mn,
                                             uint32_t *t_mx, uint32_t *t_mnw, uint32_t *t_mxw1) {
    constexpr uint32_t SL = NL * FOLD_RPL;
    if (r_begin >= r_end) return;     // the clamped loads below read at r_begin
    auto load = [&](Run<NL> &R, uint32_t sl) {
        const bool in = sl < r_end;
        run_load(R, src + (in ? sl : r_begin), in ? min(SL, r_end - sl) : 0u, me);
    };
    Merge g;
    merge_init(g);
    Run<NL> A, B;
    load(A, r_begin);
    load(B, r_begin + SL);
    for (uint32_t sl = r_begin; sl < r_end; sl += 2 * SL) {
        run_merge(A, lo, g, t_mn, t_mx, t_mnw, t_mxw1);
        load(A, sl + 2 * SL);
        run_merge(B, lo, g, t_mn, t_mx, t_mnw, t_mxw1);
        load(B, sl + 3 * SL);
    }
    merge_flush(g, t_mn, t_mx, t_mnw, t_mxw1);
}

// The pass a bucket belongs to (bucket begins are increasing).
__device__ __forceinline__ uint32_t sub_of_bucket(CSub *subs, uint32_t nsub, uint32_t b) {
    uint32_t lo_s = 0, hi_s = nsub;
    while (hi_s - lo_s > 1) {
        const uint32_t mid = (lo_s + hi_s) >> 1;
        if (subs[mid].bucket_begin <= b) lo_s = mid; else hi_s = mid;
    }
    return lo_s;
}

// A value every lane of the wave holds alike (an LDS word all lanes read),
// moved to a scalar register so that what it indexes loads on the scalar unit.
__device__ __forceinline__ uint32_t uni(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// The pass of bucket b, searching from pass `from` (at or below it) on.
__device__ __forceinline__ uint32_t sub_from(CSub *subs, uint32_t from, uint32_t nsub, uint32_t b) {
    uint32_t lo_s = from, hi_s = nsub;
    if (lo_s + 1 >= hi_s || subs[lo_s + 1].bucket_begin > b) return lo_s;
    while (hi_s - lo_s > 1) {
        const uint32_t mid = (lo_s + hi_s) >> 1;
        if (subs[mid].bucket_begin <= b) lo_s = mid; else hi_s = mid;
    }
    return lo_s;
}

// Unordered unit of an instance id: its thread's warp, or its block (upb = 1,
// unit size = threads per block).
__device__ __forceinline__ uint32_t unit_of(uint32_t id, Magic mgM, Magic mg_tpb, uint32_t tpb, Magic mg_unit,
                                            uint32_t upb) {
    const uint32_t th = udiv(id, mgM);
    const uint32_t blk = udiv(th, mg_tpb);
    return blk * upb + udiv(th - blk * tpb, mg_unit);
}

// Conflict across units of a location's combined summary (no sub-interval
// holds a conflict of its own): ids are thread-major and units are
// monotone in the thread, so the units of the smallest and largest ids
// differ iff the location spans two units; with a write, one of those two
// records lies in a unit other than the first write's.
__device__ __forceinline__ bool judge_units(const Seg &s, Magic mgM, Magic mg_tpb, uint32_t tpb, Magic mg_unit,
                                            uint32_t upb, uint32_t &second, uint32_t &srw) {
    if (s.mxw1 == 0u) return false;
    const uint32_t u_mn = unit_of(s.mn, mgM, mg_tpb, tpb, mg_unit, upb);
    const uint32_t u_mx = unit_of(s.mx, mgM, mg_tpb, tpb, mg_unit, upb);
    if (u_mn == u_mx) return false;
    const uint32_t u_w = unit_of(s.mnw, mgM, mg_tpb, tpb, mg_unit, upb);
    if (u_mn != u_w) { second = s.mn; srw = (s.mn == s.mnw) ? 1u : 0u; }
    else { second = s.mx; srw = (s.mx + 1 == s.mxw1) ? 1u : 0u; }
    return true;
}

// judge_tables for a pass with sub-keys: a location is 2^wshift consecutive
// table entries, one per sub-interval (fine interval between warp barriers,
// or barrier interval).  Thread t judges location t: the smallest
// sub-interval with a conflict gives the witness; if there is none, the
// location's combined summary is judged across units.
template <bool RESET>
__device__ __noinline__ uint32_t judge_tables_sub(uint32_t *t_mn, uint32_t *t_mx, uint32_t *t_mnw, uint32_t *t_mxw1,
                                                  uint32_t width, uint32_t lo, CSub &S, uint32_t *wout,
                                                  uint32_t *red) {
    const uint32_t t = threadIdx.x;
    const uint32_t w = S.wshift, G = 1u << w, nloc = width >> w;     // nloc <= TBL / 2 = BKT_WG
    const Magic mgM = ldm(S.mgM), mg_unit = ldm(S.mg_unit);
    CKer &K = *cptr(S.kc);
    const Magic mg_tpb = ldm(K.mg_tpb);
    bool c = false;
    Seg e{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
    uint32_t second = 0, srw = 0, key = 0;
    if (t < nloc) {
        Seg comb{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
        for (uint32_t j = 0; j < G; j++) {
            const uint32_t k = t * G + j;
            const Seg x{0u, t_mn[k], t_mx[k], t_mnw[k], t_mxw1[k]};
            if (x.mn == 0xFFFFFFFFu) continue;
            if (RESET) { t_mn[k] = 0xFFFFFFFFu; t_mx[k] = 0; t_mnw[k] = 0xFFFFFFFFu; t_mxw1[k] = 0; }
            uint32_t sc, sr;
            if (!c && judge(x, mgM, sc, sr)) { c = true; e = x; second = sc; srw = sr; key = lo + k; }
            comb.mn = min(comb.mn, x.mn);
            comb.mx = max(comb.mx, x.mx);
            comb.mnw = min(comb.mnw, x.mnw);
            comb.mxw1 = max(comb.mxw1, x.mxw1);
        }
        if (!c && comb.mn != 0xFFFFFFFFu &&
            judge_units(comb, mgM, mg_tpb, K.tpb, mg_unit, S.upb, second, srw)) {
            c = true; e = comb; key = lo + t * G;
        }
    }
    uint32_t total;
    const uint32_t pos = block_excl_add<BKT_WG>(c ? 1u : 0u, red, &total);   // also orders the reads
    if (c) put_witness(wout, pos, key, e, second, srw);                     // before the next clear
    return total;
}

// Judge every location of a folded bucket and write its witnesses in
// location order at the start of the bucket's region; returns the count.
// With RESET, each entry read is set back to the empty summary, so the
// tables are ready for the next bucket once the judge's barriers are passed.
template <bool RESET = false>
__device__ __forceinline__ uint32_t judge_tables(uint32_t *t_mn, uint32_t *t_mx, uint32_t *t_mnw, uint32_t *t_mxw1,
                                                 uint32_t width, uint32_t lo, CSub &S, uint32_t *wout,
                                                 uint32_t *red) {
    if (S.wshift) return judge_tables_sub<RESET>(t_mn, t_mx, t_mnw, t_mxw1, width, lo, S, wout, red);
    const Magic mgM = ldm(S.mgM);
    constexpr int TP = TBL / BKT_WG;
    static_assert(TP == 2, "the judge packs the two halves' counts into one scan");
    const uint32_t t = threadIdx.x;
    bool c[TP];
    Seg e[TP];
    uint32_t second[TP], srw[TP];
    // thread t judges locations t and t + 256 (consecutive threads read
    // consecutive words: no bank conflicts); witnesses keep location order
    // by placing the first half's before the second half's
#pragma unroll
    for (int i = 0; i < TP; i++) {
        const uint32_t k = t + i * BKT_WG;
        c[i] = false; second[i] = 0; srw[i] = 0;
        e[i] = Seg{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
        if (k < width) {
            e[i].mn = t_mn[k]; e[i].mx = t_mx[k]; e[i].mnw = t_mnw[k]; e[i].mxw1 = t_mxw1[k];
            if (e[i].mn != 0xFFFFFFFFu) {
                c[i] = judge(e[i], mgM, second[i], srw[i]);
                if (RESET) { t_mn[k] = 0xFFFFFFFFu; t_mx[k] = 0; t_mnw[k] = 0xFFFFFFFFu; t_mxw1[k] = 0; }
            }
        }
    }
    uint32_t total;
    const uint32_t pre = block_excl_add<BKT_WG>((c[0] ? 1u : 0u) | (c[1] ? 0x10000u : 0u), red, &total);
    const uint32_t tot0 = total & 0xFFFFu;   // its barriers also order the table reads before anyone
    if (c[0]) put_witness(wout, pre & 0xFFFFu, lo + t, e[0], second[0], srw[0]);     // clears them again
    if (c[1]) put_witness(wout, tot0 + (pre >> 16), lo + t + BKT_WG, e[1], second[1], srw[1]);
    return tot0 + (total >> 16);
}

// Sparse buckets (at most WCAP records, no sub-keys) are folded by one wave
// each, four at a time per workgroup, with wave barriers only.  The fold
// also marks each location it touches in a bitmap, so the judge visits the
// touched locations alone, in location order, rather than the bucket's whole
// width: 64 at a time, a ballot of the conflicting ones gives each witness
// its place.
constexpr uint32_t WCAP = 64 * FOLD_RPL;

struct WaveTab {
    uint32_t *mn, *mx, *mnw, *mxw1;
    uint32_t *seen;         // TBL bits: the location was touched
    uint16_t *touched;      // the touched locations, ascending (at most WCAP)
};

__device__ __forceinline__ void wave_fold_touch(const Run<64> &r, uint32_t lo, const WaveTab &W) {
    Seg cur{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
    uint32_t pk = 0xFFFFu;
    auto flush = [&](uint32_t k) {
        atomicOr(&W.seen[k >> 5], 1u << (k & 31));
        atomicMin(&W.mn[k], cur.mn);
        atomicMax(&W.mx[k], cur.mx);
        if (cur.mxw1) {
            atomicMin(&W.mnw[k], cur.mnw);
            atomicMax(&W.mxw1[k], cur.mxw1);
        }
    };
#pragma unroll
    for (int j = 0; j < FOLD_RPL; j++) {
        if ((uint32_t)j < r.m) {
            const uint32_t hi = (uint32_t)(r.x[j] >> 32);
            const uint32_t k = (hi >> 1) - lo;
            if (k != pk) {
                if (pk != 0xFFFFu) flush(pk);
                cur.mn = 0xFFFFFFFFu; cur.mx = 0; cur.mnw = 0xFFFFFFFFu; cur.mxw1 = 0;
                pk = k;
            }
            seg_add(cur, (uint32_t)r.x[j], hi & 1u);
        }
    }
    if (pk != 0xFFFFu) flush(pk);
}

// Judge the touched locations of a wave's folded bucket, write its witnesses
// in location order at wout, leave the tables and the bitmap empty; returns
// the count.
__device__ __forceinline__ uint32_t wave_judge(const WaveTab &W, uint32_t lo, Magic mgM, uint32_t *wout) {
    constexpr uint32_t NW = TBL / 32;
    static_assert(NW <= 64, "one bitmap word per lane");
    const uint32_t ln = lane();
    wave_sync_lds();
    // the touched list: lane l < NW lists the set bits of word l at the
    // count of set bits in the words before it
    uint32_t w = ln < NW ? W.seen[ln] : 0u;
    const uint32_t cnt = (uint32_t)__builtin_popcount(w);
    const uint32_t inc = wave_incl_add(cnt);
    const uint32_t nt = readlane(inc, 63);
    if (ln < NW) {
        uint32_t at = inc - cnt;
        while (w) {
            W.touched[at++] = (uint16_t)(ln * 32u + (uint32_t)__builtin_ctz(w));
            w &= w - 1u;
        }
        W.seen[ln] = 0u;
    }
    wave_sync_lds();
    uint32_t total = 0;
    for (uint32_t j0 = 0; j0 < nt; j0 += 64) {
        const uint32_t j = j0 + ln;
        bool c = false;
        uint32_t k = 0, sc = 0, sr = 0;
        Seg e{0u, 0u, 0u, 0u, 0u};
        if (j < nt) {
            k = W.touched[j];
            e = Seg{0u, W.mn[k], W.mx[k], W.mnw[k], W.mxw1[k]};
            W.mn[k] = 0xFFFFFFFFu; W.mx[k] = 0; W.mnw[k] = 0xFFFFFFFFu; W.mxw1[k] = 0;
            c = judge(e, mgM, sc, sr);
        }
        const uint64_t m = __ballot(c);
        if (c) put_witness(wout, total + mbcnt(m), lo + k, e, sc, sr);
        total += (uint32_t)__popcll(m);
    }
    wave_sync_lds();
    return total;
}

// The fold deals groups of up to FOLD_GROUP consecutive buckets out
// cyclically (workgroups of one XCD take adjacent groups of each round),
// which evens out buckets of different sizes across workgroups; with few
// buckets the groups shrink so that every workgroup gets some.
constexpr uint32_t FOLD_GROUP = 64;
static_assert(FOLD_GROUP <= BKT_WG, "one listing thread per bucket of a group");

// GS > 0: groups of GS buckets (launches with at least GS groups per
// workgroup); GS = 0: groups of deal_chunk(nbuckets, grid, FOLD_GROUP).  The
// compile-time group size measured markedly faster on launches of millions
// of sparse buckets, hence two instances.
template <uint32_t GS>
__global__ void __launch_bounds__(BKT_WG) k_fold(const DevSub *subs_g, uint32_t nsub, uint32_t nbuckets,
                                                  unsigned long long *__restrict__ rec,
                                                  const uint32_t *__restrict__ starts,
                                                  const uint32_t *__restrict__ counts, uint32_t *__restrict__ conf,
                                                  HotArea hot) {
    // four waves' tables (the workgroup's buckets use wave 0's)
    __shared__ uint32_t wt[BKT_WG / 64][4][TBL];
    __shared__ uint16_t w_touched[BKT_WG / 64][WCAP];
    __shared__ uint32_t w_seen[BKT_WG / 64][TBL / 32];
    // a group lists at most FOLD_GROUP buckets
    __shared__ uint32_t l_b[FOLD_GROUP], l_cnt[FOLD_GROUP], l_st[FOLD_GROUP], l_hot[FOLD_GROUP], l_sub[FOLD_GROUP];
    __shared__ uint32_t v_b[FOLD_GROUP], v_cnt[FOLD_GROUP], v_st[FOLD_GROUP], v_sub[FOLD_GROUP];
    __shared__ uint32_t p_beg[FOLD_GROUP + 1];
    __shared__ uint32_t red[BKT_WG / 64];
    uint32_t *const t_mn = wt[0][0], *const t_mx = wt[0][1], *const t_mnw = wt[0][2], *const t_mxw1 = wt[0][3];
    CSub *subs = cptr(subs_g);
    const uint32_t t = threadIdx.x;
    const uint32_t G = gridDim.x;                  // multiple of 8
    const uint32_t r = (blockIdx.x & 7u) * (G >> 3) + (blockIdx.x >> 3);
    const uint32_t gsz = GS ? GS : deal_chunk(nbuckets, G, FOLD_GROUP);
    if (r * gsz >= nbuckets) return;
    uint32_t sidx = sub_of_bucket(subs, nsub, r * gsz);   // groups only increase: walk forward
    const uint32_t wv = t >> 6;
    const WaveTab W{wt[wv][0], wt[wv][1], wt[wv][2], wt[wv][3], w_seen[wv], w_touched[wv]};
    for (uint32_t k = t; k < (BKT_WG / 64) * TBL; k += BKT_WG) {
        const uint32_t q = k / TBL, e = k % TBL;
        wt[q][0][e] = 0xFFFFFFFFu; wt[q][1][e] = 0; wt[q][2][e] = 0xFFFFFFFFu; wt[q][3][e] = 0;
    }
    if (t < (BKT_WG / 64) * (TBL / 32)) w_seen[t / (TBL / 32)][t % (TBL / 32)] = 0;
    for (uint32_t base = r * gsz; base < nbuckets; base += G * gsz) {
        // --- list this group's non-empty buckets (in order): sparse ones of
        // passes without sub-keys for the waves, the others for the
        // workgroup, and the hot ones
        const uint32_t b1 = min(nbuckets, base + gsz);
        const uint32_t mb = base + t;
        const bool inr = t < gsz && mb < b1;
        const uint32_t c = inr ? counts[mb] : 0u;
        // the pass of each bucket: the last pass starting at or below it
        // (passes without buckets start where the next one does), from the
        // group's first pass and the starts of the FOLD_GROUP after it
        sidx = sub_from(subs, sidx, nsub, base);
        uint32_t ms = sidx;
        bool nosub = subs[sidx].wshift == 0;
        if (b1 > subs[sidx].bucket_begin + subs[sidx].nb) {     // the group spans passes
            if (t <= FOLD_GROUP) p_beg[t] = sidx + t < nsub ? subs[sidx + t].bucket_begin : 0xFFFFFFFFu;
            __syncthreads();
            if (inr) {
                if (mb >= p_beg[FOLD_GROUP]) {
                    ms = sub_from(subs, sidx + FOLD_GROUP, nsub, mb);    // many passes without buckets
                } else {
                    uint32_t lo2 = 0, hi2 = FOLD_GROUP;     // p_beg[lo2] <= mb < p_beg[hi2]
                    while (hi2 - lo2 > 1) {
                        const uint32_t mid = (lo2 + hi2) >> 1;
                        if (p_beg[mid] <= mb) lo2 = mid; else hi2 = mid;
                    }
                    ms = sidx + lo2;
                }
                nosub = subs[ms].wshift == 0;
            }
        }
        const bool wave = c != 0 && c <= WCAP && nosub;
        const bool take = c != 0 && c <= FOLD_CAP && !wave;
        const bool is_hot = c > HOT;
        if (c > FOLD_CAP && !is_hot) {                   // medium: k_mid folds it
            const uint32_t slot = atomicAdd(hot.mid_n, 1u);
            if (slot < hot.mid_cap) { hot.mid_list[slot] = mb; hot.mid_sub[slot] = ms; }
        }
        if (inr && !take && !wave) conf[mb] = 0;
        uint32_t all;      // fields of 10 bits: workgroup list, hot list, wave list
        const uint32_t pos = block_excl_add<BKT_WG>((take ? 1u : 0u) | (is_hot ? 1u << 10 : 0u) |
                                                    (wave ? 1u << 20 : 0u), red, &all);
        const uint32_t nl = all & 1023u, nh = (all >> 10) & 1023u, nv = all >> 20;
        if (take) {
            const uint32_t p = pos & 1023u;
            l_b[p] = mb; l_cnt[p] = c; l_st[p] = starts[mb]; l_sub[p] = ms;
        }
        if (wave) {
            const uint32_t p = pos >> 20;
            v_b[p] = mb; v_cnt[p] = c; v_st[p] = starts[mb]; v_sub[p] = ms;
        }
        if (is_hot) {
            const uint32_t slot = atomicAdd(hot.n, 1u);
            l_hot[(pos >> 10) & 1023u] = slot;
            if (slot < hot.cap) { hot.list[slot] = mb; hot.sub[slot] = ms; }
        }
        __syncthreads();
        for (uint32_t j = 0; j < nh; j++) {     // clear the hot buckets' summaries
            const uint32_t slot = l_hot[j];
            if (slot < hot.cap) {
                uint32_t *g = hot.tab + (size_t)slot * 4 * TBL;
                for (uint32_t k = t; k < 4u * TBL; k += BKT_WG) g[k] = (k / TBL) % 2 == 0 ? 0xFFFFFFFFu : 0u;
            }
        }
        // --- sparse buckets: wave wv folds list entries wv, wv + 4, ...; the
        // next one's records load while one is folded
        if (wv < nv) {
            auto wprocess = [&](uint32_t i, const Run<64> &cur) {
                CSub &S = subs[uni(v_sub[i])];
                const uint32_t b = uni(v_b[i]);
                const uint32_t lo = S.klo + ((b - S.bucket_begin) << S.s);
                wave_fold_touch(cur, lo, W);
                const uint32_t total = wave_judge(W, lo, ldm(S.mgM), reinterpret_cast<uint32_t *>(rec + uni(v_st[i])));
                if (lane() == 0) conf[b] = total;
            };
            constexpr uint32_t NWV = BKT_WG / 64;
            const uint32_t last = wv + (nv - 1 - wv) / NWV * NWV;     // this wave's last entry
            Run<64> A, B;
            run_load(A, rec + uni(v_st[wv]), uni(v_cnt[wv]), lane());
            run_load(B, rec + uni(v_st[min(wv + NWV, last)]), uni(v_cnt[min(wv + NWV, last)]), lane());
            for (uint32_t i = wv; i < nv; i += 2 * NWV) {
                wprocess(i, A);
                const uint32_t ja = min(i + 2 * NWV, last);
                run_load(A, rec + uni(v_st[ja]), uni(v_cnt[ja]), lane());
                if (i + NWV < nv) wprocess(i + NWV, B);
                const uint32_t jb = min(i + 3 * NWV, last);
                run_load(B, rec + uni(v_st[jb]), uni(v_cnt[jb]), lane());
            }
        }
        if (nv && nl) __syncthreads();      // wave 0's tables serve the workgroup next
        // --- fold the listed buckets; slice 0 of the next one loads meanwhile
        // Two register sets alternate: while bucket i is folded from one, the
        // other already holds (or is loading) bucket i + 1, and set A is
        // reloaded with bucket i + 2 as soon as bucket i is done.  Loads are
        // unconditional (the list index is clamped) so the compiler keeps
        // exactly the other set in flight.
        auto slice_of = [&](uint32_t j) { return min((uint32_t)(BKT_WG * FOLD_RPL), uni(l_cnt[j])); };
        auto process = [&](uint32_t i, const Run<BKT_WG> &cur) {
            const uint32_t b = uni(l_b[i]), start = uni(l_st[i]);
            CSub &S = subs[uni(l_sub[i])];
            const uint32_t lo = S.klo + ((b - S.bucket_begin) << S.s);
            const uint32_t width = min(1u << S.s, S.khi - lo);
            // the tables are empty here: cleared before the first bucket, and
            // reset entry by entry by the previous bucket's judge
            run_fold(cur, lo, t_mn, t_mx, t_mnw, t_mxw1);
            __syncthreads();
            const uint32_t total = judge_tables<true>(t_mn, t_mx, t_mnw, t_mxw1, width, lo, S,
                                                      reinterpret_cast<uint32_t *>(rec + start), red);
            if (t == 0) conf[b] = total;
        };
        if (nl) {
            Run<BKT_WG> A, B;
            run_load(A, rec + uni(l_st[0]), slice_of(0), t);
            run_load(B, rec + uni(l_st[min(1u, nl - 1)]), slice_of(min(1u, nl - 1)), t);
            for (uint32_t i = 0; i < nl; i += 2) {
                process(i, A);
                const uint32_t ja = min(i + 2, nl - 1);
                run_load(A, rec + uni(l_st[ja]), slice_of(ja), t);
                if (i + 1 < nl) process(i + 1, B);
                const uint32_t jb = min(i + 3, nl - 1);
                run_load(B, rec + uni(l_st[jb]), slice_of(jb), t);
            }
        }
        __syncthreads();     // the list is rebuilt for the next group
    }
}

// Medium buckets (more records than one fold slice, at most HOT): one
// workgroup per bucket, slice after slice.
__global__ void __launch_bounds__(BKT_WG) k_mid(const DevSub *subs_g, unsigned long long *__restrict__ rec,
                                                 const uint32_t *__restrict__ starts,
                                                 const uint32_t *__restrict__ counts, uint32_t *__restrict__ conf,
                                                 HotArea hot) {
    __shared__ uint32_t t_mn[TBL], t_mx[TBL], t_mnw[TBL], t_mxw1[TBL];
    __shared__ uint32_t red[BKT_WG / 64];
    CSub *subs = cptr(subs_g);
    const uint32_t t = threadIdx.x;
    const uint32_t nm = min(*hot.mid_n, hot.mid_cap);
    for (uint32_t i = blockIdx.x; i < nm; i += gridDim.x) {
        const uint32_t b = hot.mid_list[i];
        const uint32_t cnt = counts[b], start = starts[b];
        CSub &S = subs[hot.mid_sub[i]];
        const uint32_t lo = S.klo + ((b - S.bucket_begin) << S.s);
        const uint32_t width = min(1u << S.s, S.khi - lo);
#pragma unroll
        for (int k2 = 0; k2 < TBL / BKT_WG; k2++) {
            const uint32_t k = t + k2 * BKT_WG;
            t_mn[k] = 0xFFFFFFFFu; t_mx[k] = 0; t_mnw[k] = 0xFFFFFFFFu; t_mxw1[k] = 0;
        }
        __syncthreads();
        fold_records<BKT_WG>(rec + start, 0, cnt, lo, t, t_mn, t_mx, t_mnw, t_mxw1);
        __syncthreads();
        const uint32_t total = judge_tables(t_mn, t_mx, t_mnw, t_mxw1, width, lo, S,
                                            reinterpret_cast<uint32_t *>(rec + start), red);
        if (t == 0) conf[b] = total;
    }
}

// Hot buckets (more than HOT records): part q of a bucket (records
// [q * HOT_PART, (q + 1) * HOT_PART)) is folded by one workgroup in LDS and
// merged into the bucket's summary in global memory with atomics; k_hot_judge,
// the next launch, judges each bucket's summary and writes its witnesses (the
// launch boundary orders the merges before the judge, with no device-scope
// fence inside a kernel: those write back and invalidate the L2 and cost more
// than the merges).  Each part pays table set-up, barriers and the global
// merge, so parts are four times the hot threshold (measured best on the
// batched workload's 1,199 hot buckets).
constexpr uint32_t HOT_PART = 4 * HOT;
__global__ void __launch_bounds__(BKT_WG) k_hot(const DevSub *subs_g, uint32_t nsub,
                                                 unsigned long long *__restrict__ rec,
                                                 const uint32_t *__restrict__ starts,
                                                 const uint32_t *__restrict__ counts, HotArea hot,
                                                 SubResult *__restrict__ res) {
    __shared__ uint32_t t_mn[TBL], t_mx[TBL], t_mnw[TBL], t_mxw1[TBL];
    __shared__ uint32_t h_pre[BKT_WG + 1], h_b[BKT_WG], h_cnt[BKT_WG], h_sub[BKT_WG];
    __shared__ uint32_t red[BKT_WG / 64];
    CSub *subs = cptr(subs_g);
    const uint32_t t = threadIdx.x;
    const uint32_t nh = min(*hot.n, hot.cap);
    if (blockIdx.x == 0 && (*hot.n > hot.cap || *hot.mid_n > hot.mid_cap)) {
        // a list dropped buckets (the workspace layout sizes them so that
        // this cannot happen): every pass of the chunk reports the failure
        for (uint32_t j = t; j < nsub; j += BKT_WG) res[subs[j].res].pad = 1u;
    }
    uint32_t u = 0;      // parts of the list before this group of entries
    for (uint32_t base = 0; base < nh; base += BKT_WG) {
        // the group's entries and the prefix of their part counts
        const uint32_t i = base + t;
        uint32_t b = 0, cnt = 0, sb = 0;
        if (i < nh) { b = hot.list[i]; cnt = counts[b]; sb = hot.sub[i]; }
        const uint32_t parts = (cnt + HOT_PART - 1) / HOT_PART;
        uint32_t tot;
        const uint32_t pre = block_excl_add<BKT_WG>(parts, red, &tot);
        h_pre[t] = pre; h_b[t] = b; h_cnt[t] = cnt; h_sub[t] = sb;
        if (t == 0) h_pre[BKT_WG] = tot;
        __syncthreads();
        // parts u .. u + tot - 1 go to workgroups round-robin
        for (uint32_t p = (blockIdx.x + gridDim.x - u % gridDim.x) % gridDim.x; p < tot; p += gridDim.x) {
            uint32_t lo_e = 0, hi_e = BKT_WG;         // entry: the last with h_pre <= p
            while (hi_e - lo_e > 1) {
                const uint32_t mid = (lo_e + hi_e) >> 1;
                if (h_pre[mid] <= p) lo_e = mid; else hi_e = mid;
            }
            while (lo_e + 1 < BKT_WG && h_pre[lo_e + 1] <= p) lo_e++;     // skip entries with no parts
            const uint32_t e = lo_e, q = p - h_pre[e];
            const uint32_t bk = h_b[e], bcnt = h_cnt[e];
            const uint32_t start = starts[bk];
            CSub &S = subs[uni(h_sub[e])];
            const uint32_t lo = S.klo + ((bk - S.bucket_begin) << S.s);
            const uint32_t width = min(1u << S.s, S.khi - lo);
#pragma unroll
            for (int k2 = 0; k2 < TBL / BKT_WG; k2++) {
                const uint32_t k = t + k2 * BKT_WG;
                t_mn[k] = 0xFFFFFFFFu; t_mx[k] = 0; t_mnw[k] = 0xFFFFFFFFu; t_mxw1[k] = 0;
            }
            __syncthreads();
            fold_records<BKT_WG>(rec + start, q * HOT_PART, min(bcnt, (q + 1) * HOT_PART), lo, t, t_mn, t_mx, t_mnw, t_mxw1);
            __syncthreads();
            uint32_t *g = hot.tab + (size_t)(base + e) * 4 * TBL;
            for (uint32_t k = t; k < width; k += BKT_WG) {
                if (t_mn[k] != 0xFFFFFFFFu) {
                    atomicMin(&g[k], t_mn[k]);
                    atomicMax(&g[TBL + k], t_mx[k]);
                    if (t_mxw1[k]) {
                        atomicMin(&g[2 * TBL + k], t_mnw[k]);
                        atomicMax(&g[3 * TBL + k], t_mxw1[k]);
                    }
                }
            }
            __syncthreads();     // the tables are cleared for the next part
        }
        u += tot;
        __syncthreads();     // the group's LDS arrays are rebuilt next
    }
}

// Judge each hot bucket from its merged summary: one workgroup per bucket.
__global__ void __launch_bounds__(BKT_WG) k_hot_judge(const DevSub *subs_g, unsigned long long *__restrict__ rec,
                                                       const uint32_t *__restrict__ starts,
                                                       uint32_t *__restrict__ conf, HotArea hot) {
    __shared__ uint32_t t_mn[TBL], t_mx[TBL], t_mnw[TBL], t_mxw1[TBL];
    __shared__ uint32_t red[BKT_WG / 64];
    CSub *subs = cptr(subs_g);
    const uint32_t t = threadIdx.x;
    const uint32_t nh = min(*hot.n, hot.cap);
    for (uint32_t j = blockIdx.x; j < nh; j += gridDim.x) {
        const uint32_t bk = hot.list[j];
        CSub &S = subs[hot.sub[j]];
        const uint32_t lo = S.klo + ((bk - S.bucket_begin) << S.s);
        const uint32_t width = min(1u << S.s, S.khi - lo);
        const uint32_t *g = hot.tab + (size_t)j * 4 * TBL;
        for (uint32_t k = t; k < width; k += BKT_WG) {
            t_mn[k] = g[k]; t_mx[k] = g[TBL + k]; t_mnw[k] = g[2 * TBL + k]; t_mxw1[k] = g[3 * TBL + k];
        }
        __syncthreads();
        const uint32_t total = judge_tables(t_mn, t_mx, t_mnw, t_mxw1, width, lo, S,
                                            reinterpret_cast<uint32_t *>(rec + starts[bk]), red);
        if (t == 0) conf[bk] = total;
        __syncthreads();     // the tables are refilled for the next bucket
    }
}

// ------------------------------------------------------------- finishing
__global__ void k_finish(const DevSub *subs_g, uint32_t nsub, size_t nbuckets, const uint32_t *__restrict__ conf,
                         SubResult *__restrict__ res) {
    CSub *subs = cptr(subs_g);
    const size_t b = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbuckets) return;
    const uint32_t c = conf[b];
    if (!c) return;
    uint32_t lo = 0, hi = nsub;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (subs[mid].bucket_begin <= (uint32_t)b) lo = mid; else hi = mid;
    }
    const uint32_t slot = subs[lo].res;
    atomicAdd(&res[slot].conflicts, (unsigned long long)c);
    atomicMin(&res[slot].first_bucket, (uint32_t)b);
}

// The pass's first witness: from its first conflicting block-local unit
// (whose locations precede every bucket's), else from its first bucket.
__global__ void k_first(const DevSub *subs_g, uint32_t nsub, const unsigned long long *__restrict__ rec,
                        const uint32_t *__restrict__ starts, const uint32_t *__restrict__ uwit,
                        SubResult *__restrict__ res) {
    CSub *subs = cptr(subs_g);
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nsub) return;
    SubResult &R = res[subs[j].res];
    const uint32_t fu = R.first_unit;
    if (fu != 0xFFFFFFFFu) {
        const uint32_t *w = uwit + 4 * (size_t)fu;
        R.w[0] = w[0]; R.w[1] = w[1]; R.w[2] = w[2]; R.w[3] = w[3];
        return;
    }
    const uint32_t fb = R.first_bucket;
    if (fb == 0xFFFFFFFFu) return;
    const uint32_t *w = reinterpret_cast<const uint32_t *>(rec + starts[fb]);
    R.w[0] = w[0]; R.w[1] = w[1]; R.w[2] = w[2]; R.w[3] = w[3];
}

__global__ void k_gather(const DevSub *subs_g, uint32_t nsub, const unsigned long long *__restrict__ rec,
                         const uint32_t *__restrict__ starts, const uint32_t *__restrict__ conf,
                         const uint32_t *__restrict__ wpos, unsigned long long base, unsigned long long lo,
                         unsigned long long hi, DevWitness *__restrict__ out) {
    CSub *subs = cptr(subs_g);
    const uint32_t b = blockIdx.x;
    const uint32_t c = conf[b];
    if (!c) return;
    const unsigned long long first = base + wpos[b];
    if (first >= hi || first + c <= lo) return;
    uint32_t slo = 0, shi = nsub;
    while (shi - slo > 1) {
        const uint32_t mid = (slo + shi) >> 1;
        if (subs[mid].bucket_begin <= b) slo = mid; else shi = mid;
    }
    const uint32_t sub = subs[slo].res;
    const uint32_t *w = reinterpret_cast<const uint32_t *>(rec + starts[b]);
    for (uint32_t k = threadIdx.x; k < c; k += blockDim.x) {
        const unsigned long long g = first + k;
        if (g >= lo && g < hi) {
            DevWitness d;
            d.w[0] = w[4 * k]; d.w[1] = w[4 * k + 1]; d.w[2] = w[4 * k + 2]; d.w[3] = w[4 * k + 3];
            d.sub = sub; d.pad[0] = d.pad[1] = d.pad[2] = 0;
            out[g - lo] = d;
        }
    }
}

// ------------------------------------------------- small passes, on chip
// A pass of at most SMALL_CAP instances is checked by one workgroup without
// its records touching HBM.  The workgroup expands every work item of the
// pass and folds each record into a per-location summary held in an LDS
// hash table (open addressing on the location key, linear probing, at most
// half full: the table has the first power of two of at least twice the
// pass's instances, 64 to 2 SMALL_CAP slots); each lane first merges its
// consecutive records of one location in registers.  A slot keeps the
// smallest id, the largest 2 id + rw and the smallest write id (ids of a
// small pass are below SMALL_CAP), so two workgroups share a CU.  The judge
// then scans the table: the pass's conflict count, and the witness of its
// smallest conflicting location.  Passes are dealt to the persistent
// workgroups cyclically.
constexpr uint32_t SMALL_HASH = 2 * SMALL_CAP;
static_assert(SMALL_HASH == 4096, "small tables hash to at most 12 bits");

__device__ __forceinline__ uint32_t small_slot(uint32_t *keys, uint32_t loc, uint32_t hb, uint32_t &over) {
    const uint32_t mask = (1u << hb) - 1u;
    uint32_t h = (loc * 0x9E3779B1u) >> (32 - hb);
    for (uint32_t n = 0; n <= mask; n++) {
        const uint32_t k = atomicCAS(&keys[h], 0xFFFFFFFFu, loc);
        if (k == 0xFFFFFFFFu || k == loc) return h;
        h = (h + 1) & mask;
    }
    over = 1;
    return 0xFFFFFFFFu;
}

__global__ void __launch_bounds__(BKT_WG) k_small(const DevSub *subs_g, uint32_t nsub,
                                                  SubResult *__restrict__ res) {
    __shared__ uint32_t keys[SMALL_HASH], t_mn[SMALL_HASH], t_mx2[SMALL_HASH], t_mnw[SMALL_HASH];
    __shared__ uint32_t red[BKT_WG / 64];
    __shared__ uint32_t s_over, s_first;
    __shared__ unsigned long long s_oob;
    CSub *subs = cptr(subs_g);
    const uint32_t t = threadIdx.x;
    for (uint32_t j = blockIdx.x; j < nsub; j += gridDim.x) {
        CSub &S = subs[j];
        CKer &K = *cptr(S.kc);
        // table bits: 2^hb >= 2 x the pass's instances (M per thread)
        const uint32_t P = S.M * K.nthreads;
        uint32_t hb = 6;
        while (hb < 12 && (1u << hb) < 2u * P) hb++;
        const uint32_t slots = 1u << hb;
        for (uint32_t i = t; i < slots; i += BKT_WG) {
            keys[i] = 0xFFFFFFFFu;
            t_mn[i] = 0xFFFFFFFFu; t_mx2[i] = 0; t_mnw[i] = 0xFFFFFFFFu;
        }
        if (t == 0) { s_over = 0; s_first = 0xFFFFFFFFu; s_oob = ~0ull; }
        __syncthreads();
        // --- expansion, folded into the table
        const uint32_t klo = S.klo, span = S.khi - S.klo;
        uint32_t nrec = 0;
        CEnt *ents = cptr(S.entries);
        CU32 *eit = cptr(S.entry_items);
        for (uint32_t e = 0; e < S.n_entries; e++) {
            CEnt &E = ents[e];
            const uint32_t ni = eit[e + 1] - eit[e];
            const uint32_t rwbit = E.rw;
            const uint32_t v = (E.flat ? 3u : 0u) + (E.fast == 2 ? 0u : E.fast ? 1u : 2u);
            auto run = [&](auto variant) {
                for (uint32_t li = 0; li < ni; li++) {
                    Seg cur{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
                    uint32_t pk = 0xFFFFFFFFu;
                    auto flush = [&]() {
                        if (pk == 0xFFFFFFFFu) return;
                        const uint32_t h = small_slot(keys, pk, hb, s_over);
                        if (h == 0xFFFFFFFFu) return;
                        atomicMin(&t_mn[h], cur.mn);
                        atomicMax(&t_mx2[h], 2u * cur.mx + (cur.mxw1 == cur.mx + 1u ? 1u : 0u));
                        if (cur.mxw1) atomicMin(&t_mnw[h], cur.mnw);
                    };
                    expand_v(variant, S, E, K, li, [&](int, bool ok, bool inb, uint32_t loc, uint32_t id) {
                        if (ok && !inb) atomicMin(&s_oob, ((unsigned long long)S.interval << 32) | id);
                        if (!(ok && inb && loc - klo < span)) return;
                        nrec++;
                        if (loc != pk) {
                            flush();
                            cur = Seg{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
                            pk = loc;
                        }
                        seg_add(cur, id, rwbit);
                    });
                    flush();
                }
            };
            switch (v) {
                case 0: run(Variant<0>{}); break;
                case 1: run(Variant<1>{}); break;
                case 2: run(Variant<2>{}); break;
                case 3: run(Variant<3>{}); break;
                case 4: run(Variant<4>{}); break;
                default: run(Variant<5>{}); break;
            }
        }
        uint32_t total_rec;
        block_excl_add<BKT_WG>(nrec, red, &total_rec);      // its barriers also end the folding
        // --- judge: count, and the smallest conflicting location.  A slot
        // reads back as a summary whose mxw1 is max write id + 1 when the
        // largest id writes, 0 without writes, and otherwise a value that is
        // neither (the judge only tests it against 0 and mx + 1).
        auto get = [&](uint32_t i) {
            const uint32_t a = t_mn[i], m2 = t_mx2[i], w = t_mnw[i];
            const uint32_t mx = m2 >> 1;
            return Seg{0u, a, mx, w, w == 0xFFFFFFFFu ? 0u : ((m2 & 1u) ? mx + 1u : mx)};
        };
        const Magic mgM = ldm(S.mgM);
        uint32_t nc = 0;
        for (uint32_t i = t; i < slots; i += BKT_WG) {
            if (keys[i] == 0xFFFFFFFFu) continue;
            uint32_t sc, sr;
            if (judge(get(i), mgM, sc, sr)) { nc++; atomicMin(&s_first, keys[i]); }
        }
        uint32_t total;
        block_excl_add<BKT_WG>(nc, red, &total);
        if (total) {
            const uint32_t fl = s_first;
            for (uint32_t i = t; i < slots; i += BKT_WG) {
                if (keys[i] != fl) continue;
                const Seg x = get(i);
                uint32_t sc = 0, sr = 0;
                judge(x, mgM, sc, sr);
                SubResult &R = res[S.res];
                R.w[0] = fl; R.w[1] = x.mnw; R.w[2] = sc; R.w[3] = sr;
            }
        }
        if (t == 0) {
            SubResult &R = res[S.res];
            R.records += total_rec;
            R.conflicts += total;
            if (s_oob != ~0ull) R.oob = min(R.oob, s_oob);
            if (s_over) R.pad = 1u;
        }
        __syncthreads();     // the table is reset for the next pass
    }
}

// ------------------------------------- block-local spaces, on chip
// In a barrier interval, the shared-array locations of block b are the keys
// [b * S, (b + 1) * S) (S shared elements per block), and only block b's
// threads touch them (Section 2: shared memory is allocated per block).  So
// a unit -- consecutive blocks whose S-ranges together fit one LDS table --
// is grouped by location without any record reaching HBM: one workgroup
// expands the shared entries' work items that cover the unit's threads,
// folds each record of the unit's range into the table slot of its location
// and judges the table, as the fold does for a bucket.  Work items at the
// edge of the unit also hold other blocks' threads; their records fall
// outside the range and are left to those blocks' units.

// A unit's LDS table: per slot the smallest id, the largest 2 id + rw (the
// largest id and whether that record writes; ids of a unit-checked interval
// stay below 2^31) and the smallest write id.  Three words per location
// instead of the fold's four, so six units share a CU.
struct UnitTab {
    uint32_t *mn, *mx2, *mnw;
    // records of one kind (rw) at slot k with ids from a to b
    __device__ __forceinline__ void run(uint32_t k, uint32_t a, uint32_t b, uint32_t rw) const {
        atomicMin(&mn[k], a);
        atomicMax(&mx2[k], 2u * b + rw);
        if (rw) atomicMin(&mnw[k], a);
    }
    __device__ __forceinline__ void seg(uint32_t k, const Seg &x) const {
        atomicMin(&mn[k], x.mn);
        atomicMax(&mx2[k], 2u * x.mx + (x.mxw1 == x.mx + 1u ? 1u : 0u));
        if (x.mxw1) atomicMin(&mnw[k], x.mnw);
    }
    // the slot as the judge reads a summary: mxw1 is max write id + 1 when
    // the largest id writes, 0 without writes, and otherwise a value that is
    // neither (the judge only tests it against 0 and mx + 1)
    __device__ __forceinline__ Seg get(uint32_t k) const {
        const uint32_t a = mn[k], m2 = mx2[k], w = mnw[k];
        const uint32_t mx = m2 >> 1;
        return Seg{0u, a, mx, w, w == 0xFFFFFFFFu ? 0u : ((m2 & 1u) ? mx + 1u : mx)};
    }
};

// Linear records: lane j holds lcnt records at unit slots r0 + p * dl with
// ids id + p (p < lcnt), all inside the unit.  Lanes are in instance order,
// so neighbouring lanes with the same r0 and count hold the same locations at
// every point p; such a run of lanes folds as one summary per point (min id:
// its first lane's, max id: its last lane's).  When the two halves of a full
// wave hold the same locations lane for lane (two rows of a block reading
// locations that do not depend on the row), lane j + 32 joins lane j's run,
// its ids being the larger.  With few runs each run's points are spread over
// the lanes; with many, the runs' points are walked by their first lanes
// (and, for paired halves, by their upper partners, odd points).  UNIFORM:
// every live lane has the same count.
template <bool UNIFORM>
__device__ __forceinline__ void fold_lin(uint32_t r0, uint32_t lcnt, uint32_t id, uint32_t dl, uint32_t rw,
                                         const UnitTab &T) {
    const bool live = lcnt != 0u;
    const uint64_t lm = __ballot(live);
    if (!lm) return;
    const uint32_t j = lane();
    bool pair = false;
    if (UNIFORM && lm == ~0ull) pair = !__ballot(__shfl_xor(r0, 32) != r0);
    const uint32_t pr = __shfl_up(r0, 1u), pc = __shfl_up(lcnt, 1u);
    const bool head = live && (!pair || j < 32u) && (j == 0u || pr != r0 || pc != lcnt);
    const uint64_t hm = __ballot(head);
    // the run of a head ends before the next head, or at the last live lane
    // of its half (lanes without records only follow the live ones); with
    // paired halves the run's last id is the upper partner's
    const uint64_t after = j < 63u ? hm >> (j + 1u) : 0ull;
    const uint32_t last = pair ? 31u : 63u - (uint32_t)__builtin_clzll(lm);
    const uint32_t tail = (after ? j + (uint32_t)__builtin_ctzll(after) : last) + (pair ? 32u : 0u);
    const uint32_t idt = __shfl(id, (int)tail);
    if (dl == 0u) {
        // every point of a lane at one location
        if (head) T.run(r0, id, idt + lcnt - 1u, rw);
        return;
    }
    const uint32_t nh = (uint32_t)__popcll(hm);
    const uint32_t cnt = UNIFORM ? readlane(lcnt, (uint32_t)__builtin_ctzll(lm)) : wave_max(lcnt);
    if (2u * nh <= cnt) {
        for (uint64_t m = hm; m; m &= m - 1u) {
            const uint32_t h = (uint32_t)__builtin_ctzll(m);
            const uint32_t hr = readlane(r0, h), hid = readlane(id, h), hidt = readlane(idt, h),
                           hc = readlane(lcnt, h);
            for (uint32_t p = j; p < hc; p += 64u) T.run(hr + p * dl, hid + p, hidt + p, rw);
        }
        return;
    }
    // many runs: lane j walks the points p = p0, p0 + ps, ... of the run
    // headed by lane hl
    const uint32_t hl = pair ? (j & 31u) : j;
    const uint32_t p0 = pair ? (j >> 5) : 0u, ps = pair ? 2u : 1u;
    const uint32_t hr = pair ? __shfl(r0, (int)hl) : r0, hid = pair ? __shfl(id, (int)hl) : id,
                   hidt = pair ? __shfl(idt, (int)hl) : idt;
    if ((hm >> hl) & 1u) {
        const uint32_t n = UNIFORM ? cnt : lcnt;
        uint32_t k = hr + p0 * dl, a = hid + p0, b2 = 2u * (hidt + p0) + rw;
        const uint32_t dk = ps * dl, db2 = 2u * ps;
        if (rw) {
#pragma unroll 4
            for (uint32_t p = p0; p < n; p += ps, k += dk, a += ps, b2 += db2) {
                atomicMin(&T.mn[k], a);
                atomicMax(&T.mx2[k], b2);
                atomicMin(&T.mnw[k], a);
            }
        } else {
#pragma unroll 4
            for (uint32_t p = p0; p < n; p += ps, k += dk, a += ps, b2 += db2) {
                atomicMin(&T.mn[k], a);
                atomicMax(&T.mx2[k], b2);
            }
        }
    }
}

// Unit slots of a lane's linear records; false (wave-uniformly) when a
// record of the wave is out of bounds or outside the unit.
__device__ __forceinline__ bool lin_in_unit(const LinLane &L, uint32_t ulo, uint32_t width, uint32_t &r0) {
    r0 = L.loc - ulo;
    const uint32_t rN = r0 + (L.lcnt - 1u) * L.dl;
    return !__ballot(L.lcnt != 0u && !(L.inb && r0 < width && rN < width));
}

// A linear work item of the HBM pipeline's mapping, folded on chip; false
// when the per-record path has to take it.
template <bool FLAT, bool PROVEN>
__device__ __forceinline__ bool dir_lin(CEnt &E, CKer &K, uint32_t item, uint32_t ulo, uint32_t width,
                                        const UnitTab &T, uint32_t &nrec) {
    const LinLane L = lin_lane<FLAT, PROVEN>(E, K, item);
    uint32_t r0;
    if (!lin_in_unit(L, ulo, width, r0)) return false;
    fold_lin<!FLAT>(r0, L.lcnt, L.id, L.dl, E.rw, T);
    nrec += L.lcnt;
    return true;
}

// A thread-linear work item (one instance per thread, a lane's gt
// consecutive threads differ in tx alone; the loop box is one point), folded
// on chip: lane records s < lcnt at unit slot r0 + s * fr[tx] with ids id +
// s * tmul.  When every lane's records share one slot, the wave folds them
// as one summary.  False when a record of the wave is out of bounds or
// outside the unit.
template <bool PROVEN>
__device__ __forceinline__ bool dir_tlin(CEnt &E, CKer &K, uint32_t item, uint32_t ulo, uint32_t width,
                                         const UnitTab &T, uint32_t &nrec) {
    // flat mapping with one loop chunk: lane q of the entry takes threads q gt ..
    const uint32_t q = item * EXP_WG + threadIdx.x;
    const uint32_t g0 = q < E.nq ? q * E.gt : K.nthreads;
    const bool gval = g0 < K.nthreads;
    const uint32_t gg = gval ? g0 : 0u;
    const uint32_t blk = udiv(gg, ldm(K.mg_tpb));
    const uint32_t tid = gg - blk * K.tpb;
    const uint32_t byy = udiv(blk, ldm(K.mg_gdx));
    const uint32_t tyy = udiv(tid, ldm(K.mg_bdx));
    const uint32_t tx = tid - tyy * K.bdx, ty = tyy, bx = blk - byy * K.gdx, by = byy;
    const uint32_t L0 = (uint32_t)E.lo[0], L1 = (uint32_t)E.lo[1], L2 = (uint32_t)E.lo[2];
    const uint32_t lcnt = gval ? min(E.gt, K.nthreads - gg) : 0u;
    const uint32_t loc = blk * E.loc_mul + E.fr[C_TX] * tx + E.fr[C_TY] * ty + E.fr[C_BX] * bx +
                         E.fr[C_BY] * by + E.fr[C_C0] + E.fr[C_L0] * L0 + E.fr[C_L1] * L1 + E.fr[C_L2] * L2;
    const uint32_t dl = E.fr[C_TX], did = E.tmul;
    bool good = true;
    if constexpr (!PROVEN) {
#pragma unroll
        for (int r = 0; r < 3; r++) {
            const uint32_t i0 = (uint32_t)E.row[r][C_TX] * tx + (uint32_t)E.row[r][C_TY] * ty +
                                (uint32_t)E.row[r][C_BX] * bx + (uint32_t)E.row[r][C_BY] * by +
                                (uint32_t)E.row[r][C_C0] + (uint32_t)E.row[r][C_L0] * L0 +
                                (uint32_t)E.row[r][C_L1] * L1 + (uint32_t)E.row[r][C_L2] * L2;
            const uint32_t iN = i0 + (lcnt - 1u) * (uint32_t)E.row[r][C_TX];
            good = good && i0 < E.dim[r] && iN < E.dim[r];
        }
    }
    const uint32_t r0 = loc - ulo, rN = r0 + (lcnt - 1u) * dl;
    if (__ballot(lcnt != 0u && !(good && r0 < width && rN < width))) return false;
    const uint64_t lm = __ballot(lcnt != 0u);
    if (!lm) return true;
    const uint32_t id = gg * E.tmul + E.off, rw = E.rw;
    if (dl == 0u) {
        const uint32_t f = (uint32_t)__builtin_ctzll(lm), l = 63u - (uint32_t)__builtin_clzll(lm);
        const uint32_t rf = readlane(r0, f);
        if (!__ballot(lcnt != 0u && r0 != rf)) {
            // the wave's records all at one location: ids increase with the lane
            const uint32_t mn = readlane(id, f), mx = readlane(id + (lcnt - 1u) * did, l);
            if (lane() == f) T.run(rf, mn, mx, rw);
        } else if (lcnt) {
            T.run(r0, id, id + (lcnt - 1u) * did, rw);
        }
    } else {
        uint32_t k = r0, a = id;
        for (uint32_t s = 0; s < lcnt; s++, k += dl, a += did) T.run(k, a, a, rw);
    }
    nrec += lcnt;
    return true;
}

// A tile of 256 consecutive threads of an entry whose loop box is one loop
// (every point of a thread is linear): lane = thread, all the box's points
// at once.  False when the per-record path has to take the tile.
template <bool PROVEN>
__device__ __forceinline__ bool dir_lin_box(CEnt &E, CKer &K, uint32_t tile, uint32_t ulo, uint32_t width,
                                            const UnitTab &T, uint32_t &nrec) {
    const LinLane L = lin_lane_at<PROVEN>(E, K, tile * EXP_WG + threadIdx.x, 0u, 0u, 0u, 0u, E.box);
    uint32_t r0;
    if (!lin_in_unit(L, ulo, width, r0)) return false;
    fold_lin<true>(r0, L.lcnt, L.id, L.dl, E.rw, T);
    nrec += L.lcnt;
    return true;
}

__global__ void __launch_bounds__(BKT_WG) k_direct(const DevSub *subs_g, const DevUnit *__restrict__ units,
                                                   uint32_t nunits, SubResult *__restrict__ res,
                                                   uint32_t *__restrict__ uwit) {
    __shared__ __align__(16) uint32_t t_mn[DIR_CAP], t_mx2[DIR_CAP], t_mnw[DIR_CAP];
    __shared__ uint32_t red[BKT_WG / 64];
    __shared__ uint32_t s_first;
    __shared__ unsigned long long s_oob;
    static_assert(DIR_CAP % (4 * BKT_WG) == 0, "unit slots split evenly over the threads, four at a time");
    const UnitTab T{t_mn, t_mx2, t_mnw};
    CSub *subs = cptr(subs_g);
    const uint32_t t = threadIdx.x;
    // one workgroup per unit
    const uint32_t u = blockIdx.x;
    if (u >= nunits) return;
    const DevUnit U = units[u];
    CSub &S = subs[U.sub];
    CKer &K = *cptr(S.kc);
    const uint32_t ulo = U.lo, width = U.hi - U.lo;
    // empty summaries over the unit's slots, four at a time
    for (uint32_t k = 4u * t; k < width; k += 4u * BKT_WG) {
        *reinterpret_cast<uint4 *>(&t_mn[k]) = make_uint4(~0u, ~0u, ~0u, ~0u);
        *reinterpret_cast<uint4 *>(&t_mx2[k]) = make_uint4(0u, 0u, 0u, 0u);
        *reinterpret_cast<uint4 *>(&t_mnw[k]) = make_uint4(~0u, ~0u, ~0u, ~0u);
    }
    if (t == 0) { s_first = 0xFFFFFFFFu; s_oob = ~0ull; }
    __syncthreads();
    uint32_t nrec = 0;
    CEnt *ents = cptr(S.entries);
    for (uint32_t e = 0; e < S.n_entries; e++) {
        CEnt &E = ents[e];
        if (E.loc_mul == 0u || E.n_lchunks == 0u) continue;     // global array, or an empty loop box
        // the entry's work items holding threads [t0, t1): thread-major
        // items of 256 gt threads (x n_lchunks), or flat lanes of gt threads
        // each (x n_lchunks) in items of 256 lanes; all below 2^32
        const uint32_t nl = E.n_lchunks;
        const Magic mg_gt = ldm(E.mg_gt);
        uint32_t ia, ib;
        if (!E.flat) {
            ia = udiv(U.t0 >> 8, mg_gt) * nl;
            ib = udiv((U.t1 + (uint32_t)EXP_WG * E.gt - 1u) >> 8, mg_gt) * nl;
        } else {
            const uint32_t q0 = udiv(U.t0, mg_gt) * nl;
            const uint32_t q1 = min(udiv(U.t1 + E.gt - 1u, mg_gt) * nl, E.nq);
            ia = q0 >> 8;
            ib = (q1 >> 8) + ((q1 & 255u) ? 1u : 0u);
        }
        static_assert(EXP_WG == 256, "item ranges divide by 256 with shifts");
        const uint32_t rwbit = E.rw;
        const uint32_t v = (E.flat ? 3u : 0u) + (E.fast == 2 ? 0u : E.fast ? 1u : 2u);
        auto run = [&](auto variant) {
            constexpr int V = decltype(variant)::value;
            auto per_record = [&](uint32_t li) {
                Seg cur{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
                uint32_t pk = 0xFFFFFFFFu;
                expand_v(variant, S, E, K, li, [&](int, bool ok, bool inb, uint32_t loc, uint32_t id) {
                    if (ok && !inb) atomicMin(&s_oob, ((unsigned long long)S.interval << 32) | id);
                    const uint32_t rel = loc - ulo;
                    if (!(ok && inb && rel < width)) return;
                    nrec++;
                    if (rel != pk) {
                        if (pk != 0xFFFFFFFFu) T.seg(pk, cur);
                        cur = Seg{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
                        pk = rel;
                    }
                    seg_add(cur, id, rwbit);
                });
                if (pk != 0xFFFFFFFFu) T.seg(pk, cur);
            };
            if constexpr (V < 2) {
                // the whole box affine in the point: a tile of threads takes it at once
                if (E.lin && E.lflat) {
                    const uint32_t ta = U.t0 / EXP_WG, tb = (U.t1 + EXP_WG - 1u) / EXP_WG;
                    for (uint32_t tile = ta; tile < tb; tile++)
                        if (!dir_lin_box<(V == 0)>(E, K, tile, ulo, width, T, nrec))
                            for (uint32_t c = 0; c < nl; c++) per_record(tile * nl + c);
                    return;
                }
            }
            for (uint32_t li = ia; li < ib; li++) {
                if constexpr (V == 3 || V == 4) {
                    if (E.tlin && dir_tlin<(V == 3)>(E, K, li, ulo, width, T, nrec)) continue;
                }
                if constexpr (V % 3 != 2) {
                    if (E.lin && dir_lin<(V >= 3), (V % 3 == 0)>(E, K, li, ulo, width, T, nrec)) continue;
                }
                per_record(li);
            }
        };
        switch (v) {
            case 0: run(Variant<0>{}); break;
            case 1: run(Variant<1>{}); break;
            case 2: run(Variant<2>{}); break;
            case 3: run(Variant<3>{}); break;
            case 4: run(Variant<4>{}); break;
            default: run(Variant<5>{}); break;
        }
    }
    uint32_t total_rec;
    block_excl_add<BKT_WG>(nrec, red, &total_rec);      // its barriers also end the folding
    // judge each location (all of a thread's slots read first); keep this
    // thread's first conflict
    const Magic mgM = ldm(S.mgM);
    uint32_t nc = 0, fk = 0xFFFFFFFFu, fsc = 0, fsr = 0, fmnw = 0;
    constexpr int JPT = DIR_CAP / BKT_WG;
    Seg x[JPT];
#pragma unroll
    for (int i = 0; i < JPT; i++) x[i] = T.get(min(t + (uint32_t)i * BKT_WG, width - 1u));
#pragma unroll
    for (int i = 0; i < JPT; i++) {
        const uint32_t k = t + (uint32_t)i * BKT_WG;
        uint32_t sc, sr;
        if (k < width && x[i].mn != 0xFFFFFFFFu && judge(x[i], mgM, sc, sr)) {
            if (!nc) { fk = k; fsc = sc; fsr = sr; fmnw = x[i].mnw; }
            nc++;
        }
    }
    if (nc) atomicMin(&s_first, fk);
    uint32_t total;
    block_excl_add<BKT_WG>(nc, red, &total);           // its barriers order s_first
    if (nc && fk == s_first) {
        uint32_t *w = uwit + 4 * (size_t)u;
        w[0] = ulo + fk; w[1] = fmnw; w[2] = fsc; w[3] = fsr;
    }
    if (t == 0) {
        SubResult &R = res[S.res];
        if (total_rec) {
            atomicAdd(&R.records, (unsigned long long)total_rec);
            atomicAdd(&R.unit_records, (unsigned long long)total_rec);
        }
        if (total) {
            atomicAdd(&R.conflicts, (unsigned long long)total);
            atomicMin(&R.first_unit, u);
        }
        if (s_oob != ~0ull) atomicMin(&R.oob, s_oob);
    }
}

// ----------------------------------------- exact counts per location
// Counts that need a location's records in order: distinct-thread pairs
// (interval semantics) and RaW / WaW / WaR (ordered semantics).  Each
// bucket's records are ordered by a count key -- in LDS for buckets of at
// most CNT_TILE records, by a workgroup radix sort in global memory for
// larger ones -- and scanned tile by tile with carries:
//  PAIRS   key = (location, thread, not rw): the first record of each
//          (location, thread) run says whether that thread writes there;
//          with n threads and w writers a location holds C(n,2) - C(n-w,2)
//          unordered pairs of different threads with at least one write.
//  ORDERED key = (location, time, rw), time = the phase-major instance id:
//          records of one statement instance are adjacent (reads first);
//          an instance reads the location iff its first record is a read
//          ("R head") and writes it iff its last record is a write ("W
//          tail").  Before an instance g of a location: eW = W tails, eR =
//          R heads of earlier instances of that location; g adds
//          RaW += hasR(g) eW, WaW += hasW(g) eW, WaR += hasW(g) eR.
constexpr uint32_t CNT_TILE = 4096;
enum { CNT_PAIRS = 0, CNT_ORDERED = 1 };

__device__ __forceinline__ unsigned long long count_key(unsigned long long r, uint32_t lo, Magic mgM, int mode) {
    const uint32_t hi = (uint32_t)(r >> 32), id = (uint32_t)r;
    const uint32_t locl = (hi >> 1) - lo, rw = hi & 1u;
    if (mode == CNT_PAIRS) return ((((unsigned long long)locl << 32) | udiv(id, mgM)) << 1) | (rw ^ 1u);
    return ((unsigned long long)locl << 33) | ((unsigned long long)id << 1) | rw;
}

// Inclusive max over a wave, and the exclusive max over a workgroup of NT
// threads (identity 0).
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v) {
    v = max(v, dpp<ROW_SHR1, 0xf>(0u, v));
    v = max(v, dpp<ROW_SHR2, 0xf>(0u, v));
    v = max(v, dpp<ROW_SHR4, 0xf>(0u, v));
    v = max(v, dpp<ROW_SHR8, 0xf>(0u, v));
    v = max(v, dpp<ROW_BCAST15, 0xa>(0u, v));
    v = max(v, dpp<ROW_BCAST31, 0xc>(0u, v));
    return v;
}

template <int NT>
__device__ __forceinline__ uint32_t block_excl_max(uint32_t v, uint32_t *red, uint32_t *total) {
    const uint32_t wid = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_max(v);
    const uint32_t prev_lane = __shfl_up(inc, 1);
    if (lane() == 63) red[wid] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; w++) {
        const uint32_t x = red[w];
        if (w < (int)wid) before = max(before, x);
        tot = max(tot, x);
    }
    __syncthreads();
    *total = tot;
    return max(before, lane() ? prev_lane : 0u);
}

// State carried from one tile of a bucket's ordered records to the next.
struct CountCarry {
    unsigned long long prev;   // last key of the previous tile (~0: none)
    uint32_t w_before, r_before;   // W tails / R heads before the tile (ordered)
    uint32_t open_has_r;       // ordered: the group the tile starts inside has a read
};

struct CountTables {
    uint32_t *a, *b, *c;       // per location: pairs n / w; ordered lstart W / lstart R / dependence flag
};

// Scan one tile of m ordered records; get(i) returns the key of record i of
// the tile, next_key the key after the tile (~0 when the bucket ends).
template <class Get>
__device__ __forceinline__ void count_tile(Get &&get, uint32_t m, unsigned long long next_key, int mode,
                                           CountCarry &cc, CountTables T, uint32_t *red,
                                           unsigned long long &raw, unsigned long long &waw,
                                           unsigned long long &war) {
    const uint32_t t = threadIdx.x;
    const uint32_t c = (m + BKT_WG - 1) / BKT_WG;
    const uint32_t b0 = min(m, t * c), b1 = min(m, b0 + c);
    auto prev_of = [&](uint32_t i) { return i ? get(i - 1) : cc.prev; };
    auto next_of = [&](uint32_t i) { return i + 1 < m ? get(i + 1) : next_key; };
    if (mode == CNT_PAIRS) {
        for (uint32_t i = b0; i < b1; i++) {
            const unsigned long long k = get(i), p = prev_of(i);
            if ((k >> 1) != (p >> 1) || p == ~0ull) {
                const uint32_t l = (uint32_t)(k >> 33);
                atomicAdd(&T.a[l], 1u);
                if (!(k & 1ull)) atomicAdd(&T.b[l], 1u);
            }
        }
        __syncthreads();
        if (t == 0) cc.prev = m ? get(m - 1) : cc.prev;
        __syncthreads();
        return;
    }
    // ordered: W tails and R heads of the chunk, and its last group head
    uint32_t cw = 0, cr = 0, last_gh = 0;
    for (uint32_t i = b0; i < b1; i++) {
        const unsigned long long k = get(i), p = prev_of(i), n = next_of(i);
        const bool gh = (k >> 1) != (p >> 1) || p == ~0ull;
        const bool gt = (k >> 1) != (n >> 1) || n == ~0ull;
        if (gt && (k & 1ull)) cw++;
        if (gh && !(k & 1ull)) cr++;
        if (gh) last_gh = ((i + 1) << 1) | ((k & 1ull) ? 0u : 1u);    // (index + 1, has a read)
    }
    uint32_t tot;
    const uint32_t pre = block_excl_add<BKT_WG>(cw | (cr << 16), red, &tot);
    uint32_t gmax;
    const uint32_t gh_before = block_excl_max<BKT_WG>(last_gh, red, &gmax);
    // running prefixes; location heads record theirs
    uint32_t pw = cc.w_before + (pre & 0xFFFFu), pr = cc.r_before + (pre >> 16);
    for (uint32_t i = b0; i < b1; i++) {
        const unsigned long long k = get(i), p = prev_of(i), n = next_of(i);
        const bool gh = (k >> 1) != (p >> 1) || p == ~0ull;
        const bool gt = (k >> 1) != (n >> 1) || n == ~0ull;
        if ((k >> 33) != (p >> 33) || p == ~0ull) {
            const uint32_t l = (uint32_t)(k >> 33);
            T.a[l] = pw;
            T.b[l] = pr;
        }
        if (gt && (k & 1ull)) pw++;
        if (gh && !(k & 1ull)) pr++;
    }
    __syncthreads();
    // contributions at the group tails
    pw = cc.w_before + (pre & 0xFFFFu);
    pr = cc.r_before + (pre >> 16);
    // the group open at the chunk start: its head is the latest one before the
    // chunk in this tile, else it began in an earlier tile
    bool open_r = gh_before ? (gh_before & 1u) != 0u : cc.open_has_r != 0u;
    uint32_t open_idx = gh_before ? (gh_before >> 1) - 1u : 0xFFFFFFFFu;     // tile index of the head
    for (uint32_t i = b0; i < b1; i++) {
        const unsigned long long k = get(i), p = prev_of(i), n = next_of(i);
        const bool gh = (k >> 1) != (p >> 1) || p == ~0ull;
        const bool gt = (k >> 1) != (n >> 1) || n == ~0ull;
        if (gh) { open_r = !(k & 1ull); open_idx = i; }
        if (gt) {
            const uint32_t l = (uint32_t)(k >> 33);
            const bool has_w = (k & 1ull) != 0;
            const bool has_r = open_r;
            // prefixes exclusive of this record; the group's own R head precedes
            // it unless the group is this one record
            const uint32_t ew = pw - T.a[l];
            const uint32_t er = pr - T.b[l] - ((has_r && !(gh && open_idx == i)) ? 1u : 0u);
            const unsigned long long d_raw = has_r ? ew : 0u, d_waw = has_w ? ew : 0u, d_war = has_w ? er : 0u;
            raw += d_raw; waw += d_waw; war += d_war;
            if (d_raw | d_waw | d_war) T.c[l] = 1u;
        }
        if (gt && (k & 1ull)) pw++;
        if (gh && !(k & 1ull)) pr++;
    }
    __syncthreads();
    if (t == 0) {
        cc.w_before += tot & 0xFFFFu;
        cc.r_before += tot >> 16;
        if (gmax) cc.open_has_r = gmax & 1u;
        if (m) cc.prev = get(m - 1);
    }
    __syncthreads();
}

// Stable LSD radix sort of the n records at a by their count key (8-bit
// digits over the key's nbits, digits that every record shares skipped),
// ping-ponging with b; one workgroup.  Returns the buffer holding the result.
__device__ unsigned long long *wg_radix_sort(unsigned long long *a, unsigned long long *b, uint32_t n, uint32_t nbits,
                                             uint32_t lo, Magic mgM, int mode, uint32_t *hist, uint32_t *base,
                                             uint32_t *wcnt, uint32_t *red) {
    const uint32_t t = threadIdx.x, w = t >> 6;
    for (uint32_t shift = 0; shift < nbits; shift += 8) {
        hist[t] = 0;
        __syncthreads();
        for (uint32_t i = t; i < n; i += BKT_WG)
            atomicAdd(&hist[(uint32_t)(count_key(a[i], lo, mgM, mode) >> shift) & 255u], 1u);
        __syncthreads();
        uint32_t tot;
        const uint32_t h = hist[t];
        base[t] = block_excl_add<BKT_WG>(h, red, &tot);
        const uint64_t uniform = __ballot(h == n);
        red[w] = uniform ? 1u : 0u;            // block_excl_add is done with red
        __syncthreads();
        const bool skip = red[0] | red[1] | red[2] | red[3];
        __syncthreads();
        if (skip) continue;
        for (uint32_t r0 = 0; r0 < n; r0 += BKT_WG) {
            const uint32_t i = r0 + t;
            const bool valid = i < n;
            const unsigned long long r = valid ? a[i] : 0ull;
            const uint32_t d = valid ? ((uint32_t)(count_key(r, lo, mgM, mode) >> shift) & 255u) : 0u;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int bit = 0; bit < 8; bit++) {
                const uint64_t m1 = __ballot(valid && ((d >> bit) & 1u));
                peers &= ((d >> bit) & 1u) ? m1 : ~m1;
            }
            for (uint32_t q = t; q < 4 * 256; q += BKT_WG) wcnt[q] = 0;
            __syncthreads();
            const uint32_t below = (uint32_t)__popcll(peers & ((1ull << lane()) - 1ull));
            if (valid && below == 0) wcnt[w * 256 + d] = (uint32_t)__popcll(peers);
            __syncthreads();
            if (valid) {
                uint32_t pos = base[d] + below;
                for (uint32_t x = 0; x < w; x++) pos += wcnt[x * 256 + d];
                b[pos] = r;
            }
            __syncthreads();
            base[t] += wcnt[t] + wcnt[256 + t] + wcnt[512 + t] + wcnt[768 + t];
            __syncthreads();
        }
        unsigned long long *x = a; a = b; b = x;
    }
    return a;
}

__global__ void __launch_bounds__(BKT_WG) k_counts(const DevSub *subs_g, uint32_t nsub, uint32_t nbuckets,
                                                   unsigned long long *__restrict__ rec,
                                                   unsigned long long *__restrict__ tmp,
                                                   const uint32_t *__restrict__ starts,
                                                   const uint32_t *__restrict__ counts, int mode,
                                                   PassCounts *__restrict__ out) {
    __shared__ unsigned long long keys[CNT_TILE];
    __shared__ uint32_t ta[TBL], tb[TBL], tc[TBL];
    __shared__ uint32_t hist[256], base[256], wcnt[4 * 256];
    __shared__ uint32_t red[BKT_WG / 64];
    __shared__ CountCarry cc;
    CSub *subs = cptr(subs_g);
    const uint32_t t = threadIdx.x;
    for (uint32_t bk = blockIdx.x; bk < nbuckets; bk += gridDim.x) {
        const uint32_t cnt = counts[bk];
        if (!cnt) continue;
        CSub &S = subs[sub_of_bucket(subs, nsub, bk)];
        const uint32_t lo = S.klo + ((bk - S.bucket_begin) << S.s);
        const uint32_t width = min(1u << S.s, S.khi - lo);
        const Magic mgM = ldm(S.mgM);
        const uint32_t start = starts[bk];
        for (uint32_t i = t; i < TBL; i += BKT_WG) { ta[i] = 0; tb[i] = 0; tc[i] = 0; }
        if (t == 0) { cc.prev = ~0ull; cc.w_before = 0; cc.r_before = 0; cc.open_has_r = 0; }
        __syncthreads();
        unsigned long long raw = 0, waw = 0, war = 0;
        CountTables T{ta, tb, tc};
        if (cnt <= CNT_TILE) {
            uint32_t np = 2;
            while (np < cnt) np <<= 1;
            for (uint32_t i = t; i < np; i += BKT_WG)
                keys[i] = i < cnt ? count_key(rec[start + i], lo, mgM, mode) : ~0ull;
            __syncthreads();
            for (uint32_t kk = 2; kk <= np; kk <<= 1) {
                for (uint32_t jj = kk >> 1; jj > 0; jj >>= 1) {
                    for (uint32_t i = t; i < np; i += BKT_WG) {
                        const uint32_t x = i ^ jj;
                        if (x > i) {
                            const unsigned long long a = keys[i], b = keys[x];
                            if ((a > b) == ((i & kk) == 0)) { keys[i] = b; keys[x] = a; }
                        }
                    }
                    __syncthreads();
                }
            }
            count_tile([&](uint32_t i) { return keys[i]; }, cnt, ~0ull, mode, cc, T, red, raw, waw, war);
        } else {
            const uint32_t nbits = 33u + S.s;      // location bits above 33 bits of (thread or time, rw)
            const unsigned long long *srt = wg_radix_sort(rec + start, tmp + start, cnt, nbits, lo, mgM, mode,
                                                          hist, base, wcnt, red);
            for (uint32_t t0 = 0; t0 < cnt; t0 += CNT_TILE) {
                const uint32_t m = min(CNT_TILE, cnt - t0);
                const unsigned long long nk = t0 + m < cnt ? count_key(srt[t0 + m], lo, mgM, mode) : ~0ull;
                count_tile([&](uint32_t i) { return count_key(srt[t0 + i], lo, mgM, mode); }, m, nk, mode, cc, T,
                           red, raw, waw, war);
            }
        }
        // per-location totals and the bucket's sums into its pass
        unsigned long long pairs = 0, deploc = 0;
        for (uint32_t l = t; l < width; l += BKT_WG) {
            if (mode == CNT_PAIRS) {
                const unsigned long long n = ta[l], w = tb[l];
                pairs += n * (n - 1) / 2 - (n - w) * (n - w - 1) / 2;
            } else {
                deploc += tc[l];
            }
        }
        // wave sums, added into the pass's counters by each wave's lane 0
        unsigned long long v0 = pairs, v1 = raw, v2 = waw, v3 = war, v4 = deploc;
        for (int off = 32; off > 0; off >>= 1) {
            v0 += __shfl_xor(v0, off); v1 += __shfl_xor(v1, off); v2 += __shfl_xor(v2, off);
            v3 += __shfl_xor(v3, off); v4 += __shfl_xor(v4, off);
        }
        if (lane() == 0) {
            PassCounts &P = out[S.res];
            if (v0) atomicAdd(&P.pairs, v0);
            if (v1) atomicAdd(&P.raw, v1);
            if (v2) atomicAdd(&P.waw, v2);
            if (v3) atomicAdd(&P.war, v3);
            if (v4) atomicAdd(&P.deploc, v4);
        }
        __syncthreads();     // tables and keys are reused by the next bucket
    }
}

// ------------------------------------------------------ barrier divergence
// One workgroup per (guarded barrier, block) item, dealt out cyclically: the
// threads of the block evaluate the barrier's guards into an LDS byte map,
// then each scope (the block, or one warp) is scanned for a thread that
// reaches the barrier and one that does not.  A scope with both is a
// divergent instance: counted, and the smallest (block, scope) kept.
__global__ void __launch_bounds__(256) k_barriers(const DevBarrier *__restrict__ bars, uint32_t nbar,
                                                  const DevKernel *__restrict__ kc_g,
                                                  const int32_t *__restrict__ guards, uint32_t nblocks,
                                                  BarrierResult *__restrict__ res) {
    __shared__ uint8_t reach[BARRIER_MAX_TPB];
    const DevKernel K = *kc_g;
    const uint32_t t = threadIdx.x;
    const uint64_t items = (uint64_t)nbar * nblocks;
    for (uint64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const uint32_t g = (uint32_t)(it / nblocks), blk = (uint32_t)(it % nblocks);
        const DevBarrier B = bars[g];
        const int32_t bx = (int32_t)(blk % K.gdx), by = (int32_t)(blk / K.gdx);
        for (uint32_t tid = t; tid < K.tpb; tid += blockDim.x) {
            const int32_t tx = (int32_t)(tid % K.bdx), ty = (int32_t)(tid / K.bdx);
            bool ok = true;
            for (uint32_t q = 0; q < B.guard_count; q++) {
                const int32_t *gr = guards + (size_t)(B.guard_begin + q) * NC;
                ok = ok && gr[C_TX] * tx + gr[C_TY] * ty + gr[C_BX] * bx + gr[C_BY] * by + gr[C_C0] >= 0;
            }
            reach[tid] = ok ? 1 : 0;
        }
        __syncthreads();
        for (uint32_t sc = t; sc < B.nscope; sc += blockDim.x) {
            const uint32_t t0 = sc * B.scope, t1 = min(K.tpb, t0 + B.scope);
            bool any = false, all = true;
            for (uint32_t x = t0; x < t1; x++) { any = any || reach[x]; all = all && reach[x]; }
            if (any && !all) {
                atomicAdd(&res[g].divergent, 1ull);
                atomicMin(&res[g].first, (unsigned long long)blk * B.nscope + sc);
            }
        }
        __syncthreads();     // the map is rewritten for the next item
    }
}

// The first divergent instance of each guarded barrier: its smallest thread
// that reaches the barrier and smallest that does not (one workgroup per
// barrier, after k_barriers).
__global__ void __launch_bounds__(256) k_barriers_first(const DevBarrier *__restrict__ bars,
                                                        const DevKernel *__restrict__ kc_g,
                                                        const int32_t *__restrict__ guards,
                                                        BarrierResult *__restrict__ res) {
    __shared__ uint32_t red[2 * (256 / 64)];
    const DevKernel K = *kc_g;
    const uint32_t g = blockIdx.x, t = threadIdx.x;
    const unsigned long long first = res[g].first;
    if (first == ~0ull) return;
    const DevBarrier B = bars[g];
    const uint32_t blk = (uint32_t)(first / B.nscope), sc = (uint32_t)(first % B.nscope);
    const int32_t bx = (int32_t)(blk % K.gdx), by = (int32_t)(blk / K.gdx);
    const uint32_t t0 = sc * B.scope, t1 = min(K.tpb, t0 + B.scope);
    uint32_t arrive = 0xFFFFFFFFu, skip = 0xFFFFFFFFu;
    for (uint32_t tid = t0 + t; tid < t1; tid += blockDim.x) {
        const int32_t tx = (int32_t)(tid % K.bdx), ty = (int32_t)(tid / K.bdx);
        bool ok = true;
        for (uint32_t q = 0; q < B.guard_count; q++) {
            const int32_t *gr = guards + (size_t)(B.guard_begin + q) * NC;
            ok = ok && gr[C_TX] * tx + gr[C_TY] * ty + gr[C_BX] * bx + gr[C_BY] * by + gr[C_C0] >= 0;
        }
        if (ok) arrive = min(arrive, tid); else skip = min(skip, tid);
    }
    arrive = wave_min(arrive);
    skip = wave_min(skip);
    if (lane() == 0) { red[t >> 6] = arrive; red[4 + (t >> 6)] = skip; }
    __syncthreads();
    if (t == 0) {
        for (int w = 1; w < 4; w++) { arrive = min(arrive, red[w]); skip = min(skip, red[4 + w]); }
        res[g].arrive = arrive;
        res[g].skip = skip;
    }
}

// ------------------------------------------------ static scratch (no-alloc)
// Scratch of rv_check_static: per-pass result slots, then one chunk's
// workspace (records, bucket arrays, hot lists).  Each device holds its own
// copy from the moment the library's code object is loaded on it until the
// process ends.  Host code must never pass `scratch` itself to a kernel (in
// host code the name is a stand-in, not a device address): it uses the
// address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[RV_STATIC_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[SCRATCH_DEVICES];
hipError_t g_scratch_err[SCRATCH_DEVICES];
bool g_scratch_done[SCRATCH_DEVICES];
}  // namespace

hipError_t static_scratch_init(int device) {
    if (device < 0 || device >= SCRATCH_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_err[device] = e;
        g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
        g_scratch_done[device] = true;
    }
    return g_scratch_err[device];
}

void *static_scratch(int device) {
    if (device < 0 || device >= SCRATCH_DEVICES) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    return g_scratch_done[device] ? g_scratch_ptr[device] : nullptr;
}

// --------------------------------------------------------------- launchers
static inline unsigned grid_for(size_t n, unsigned per) {
    size_t g = (n + per - 1) / per;
    return (unsigned)(g < 1 ? 1 : (g > 65535u * 16 ? 65535u * 16 : g));
}

// Resident workgroups per CU of a kernel (queried once).
template <class K>
static unsigned occupancy(K kern, int block, unsigned fallback) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, block, 0) != hipSuccess || n < 1) return fallback;
    return (unsigned)n;
}

// persistent grid: a multiple of 8 workgroups, no more than one per item
static inline unsigned persistent_grid(uint64_t items, unsigned ncu, unsigned per_cu) {
    uint64_t g = (uint64_t)ncu * per_cu;
    if (g > items) g = items;
    g = (g + 7) & ~7ull;
    return (unsigned)(g < 8 ? 8 : g);
}

void launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256 * 4)), dim3(256), 0, st, p, n, v);
}

void launch_init_results(SubResult *r, size_t n, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_init_results, dim3(grid_for(n, 256)), dim3(256), 0, st, r, n);
}

void launch_hist(const DevSub *subs, uint32_t nsub, uint64_t items, uint32_t *counts, SubResult *res,
                 unsigned ncu, hipStream_t st) {
    if (!items) return;
    static const unsigned occ = occupancy(k_hist, EXP_WG, 4);
    hipLaunchKernelGGL(k_hist, dim3(persistent_grid(items, ncu, occ)), dim3(EXP_WG), 0, st, subs, nsub,
                       (uint32_t)items, counts, res);
}

size_t scan_bsum_words(size_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

void launch_scan(const uint32_t *in, uint32_t *starts, uint32_t *cursor, uint32_t *bsum, size_t n,
                 hipStream_t st) {
    const uint32_t nb = (uint32_t)((n + SCAN_TILE - 1) / SCAN_TILE);
    if (nb) hipLaunchKernelGGL(k_scan_up, dim3(nb), dim3(SCAN_WG), 0, st, in, n, bsum);
    hipLaunchKernelGGL(k_scan_mid, dim3(1), dim3(SCAN_WG), 0, st, bsum, nb);
    if (nb) hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(SCAN_WG), 0, st, in, n, bsum, starts, cursor);
}

void launch_scatter(const DevSub *subs, uint32_t nsub, uint64_t items, unsigned long long *rec, uint32_t *cursor,
                    unsigned ncu, hipStream_t st) {
    if (!items) return;
    static const unsigned occ = occupancy(k_scatter, EXP_WG, 2);
    hipLaunchKernelGGL(k_scatter, dim3(persistent_grid(items, ncu, occ)), dim3(EXP_WG), 0, st, subs, nsub,
                       (uint32_t)items, rec, cursor);
}

void launch_bucket(const DevSub *subs, uint32_t nsub, uint64_t nbuckets, unsigned long long *rec,
                   const uint32_t *starts, const uint32_t *counts, uint32_t *conf, int debug_sorted,
                   unsigned ncu, hipStream_t st) {
    if (!nbuckets) return;
    static const unsigned occ = occupancy(k_bucket, BKT_WG, 2);
    uint64_t g = (uint64_t)ncu * occ;
    if (g > nbuckets) g = nbuckets;
    hipLaunchKernelGGL(k_bucket, dim3((unsigned)g), dim3(BKT_WG), 0, st, subs, nsub, (uint32_t)nbuckets, rec,
                       starts, counts, conf, debug_sorted);
}

void launch_fold(const DevSub *subs, uint32_t nsub, uint64_t nbuckets, unsigned long long *rec,
                 const uint32_t *starts, const uint32_t *counts, uint32_t *conf, HotArea hot, SubResult *res,
                 unsigned ncu, hipStream_t st) {
    if (!nbuckets) return;
    static const unsigned occ = occupancy(k_fold<FOLD_GROUP>, BKT_WG, 4);
    static const unsigned occ_hot = occupancy(k_hot, BKT_WG, 4);
    static const unsigned occ_mid = occupancy(k_mid, BKT_WG, 4);
    launch_fill_u32(hot.n, 1, 0u, st);
    launch_fill_u32(hot.mid_n, 1, 0u, st);
    const unsigned G = persistent_grid(nbuckets, ncu, occ);
    if (nbuckets >= (uint64_t)FOLD_GROUP * G)
        hipLaunchKernelGGL(k_fold<FOLD_GROUP>, dim3(G), dim3(BKT_WG), 0, st, subs, nsub, (uint32_t)nbuckets, rec,
                           starts, counts, conf, hot);
    else
        hipLaunchKernelGGL(k_fold<0>, dim3(G), dim3(BKT_WG), 0, st, subs, nsub, (uint32_t)nbuckets, rec, starts,
                           counts, conf, hot);
    hipLaunchKernelGGL(k_mid, dim3(ncu * occ_mid), dim3(BKT_WG), 0, st, subs, rec, starts, counts, conf, hot);
    hipLaunchKernelGGL(k_hot, dim3(ncu * occ_hot), dim3(BKT_WG), 0, st, subs, nsub, rec, starts, counts, hot, res);
    hipLaunchKernelGGL(k_hot_judge, dim3(ncu), dim3(BKT_WG), 0, st, subs, rec, starts, conf, hot);
}

void launch_small(const DevSub *subs, uint32_t n, SubResult *res, unsigned ncu, hipStream_t st) {
    if (!n) return;
    static const unsigned occ = occupancy(k_small, BKT_WG, 1);
    const unsigned grid = (unsigned)std::min<uint64_t>(n, (uint64_t)ncu * occ);
    hipLaunchKernelGGL(k_small, dim3(grid), dim3(BKT_WG), 0, st, subs, n, res);
}

void launch_counts(const DevSub *subs, uint32_t nsub, uint64_t nbuckets, unsigned long long *rec,
                   unsigned long long *tmp, const uint32_t *starts, const uint32_t *counts, int ordered,
                   PassCounts *out, unsigned ncu, hipStream_t st) {
    if (!nbuckets) return;
    static const unsigned occ = occupancy(k_counts, BKT_WG, 2);
    const unsigned grid = (unsigned)std::min<uint64_t>(nbuckets, (uint64_t)ncu * occ);
    hipLaunchKernelGGL(k_counts, dim3(grid), dim3(BKT_WG), 0, st, subs, nsub, (uint32_t)nbuckets, rec, tmp, starts,
                       counts, ordered ? (int)CNT_ORDERED : (int)CNT_PAIRS, out);
}

__global__ void k_fill_counts(PassCounts *p, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { PassCounts z{}; p[i] = z; }
}

void launch_init_counts(PassCounts *p, size_t n, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_fill_counts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, (uint32_t)n);
}

__global__ void k_init_barrier_results(BarrierResult *r, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { r[i].divergent = 0; r[i].first = ~0ull; r[i].arrive = r[i].skip = 0xFFFFFFFFu; }
}

void launch_barriers(const DevBarrier *bars, uint32_t n, const DevKernel *kc, const int32_t *guards,
                     uint32_t nblocks, BarrierResult *res, unsigned ncu, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_init_barrier_results, dim3((n + 255) / 256), dim3(256), 0, st, res, n);
    const uint64_t items = (uint64_t)n * nblocks;
    const unsigned grid = (unsigned)std::min<uint64_t>(items, (uint64_t)ncu * 8);
    hipLaunchKernelGGL(k_barriers, dim3(grid), dim3(256), 0, st, bars, n, kc, guards, nblocks, res);
    hipLaunchKernelGGL(k_barriers_first, dim3(n), dim3(256), 0, st, bars, kc, guards, res);
}

void launch_finish(const DevSub *subs, uint32_t nsub, uint64_t nbuckets, const uint32_t *conf, SubResult *res,
                   hipStream_t st) {
    if (!nbuckets) return;
    hipLaunchKernelGGL(k_finish, dim3((unsigned)((nbuckets + 255) / 256)), dim3(256), 0, st, subs, nsub,
                       (size_t)nbuckets, conf, res);
}

void launch_first(const DevSub *subs, uint32_t nsub, const unsigned long long *rec, const uint32_t *starts,
                  const uint32_t *uwit, SubResult *res, hipStream_t st) {
    if (!nsub) return;
    hipLaunchKernelGGL(k_first, dim3((nsub + 63) / 64), dim3(64), 0, st, subs, nsub, rec, starts, uwit, res);
}

void launch_direct(const DevSub *subs, const DevUnit *units, uint32_t n, SubResult *res, uint32_t *uwit,
                   unsigned ncu, hipStream_t st) {
    if (!n) return;
    // one workgroup per unit, not a persistent grid: as units retire, the
    // dispatcher can hand their slots to the HBM pipeline's kernels running
    // beside them on the other stream (measured faster than 2, 3 or 4
    // persistent workgroups per CU)
    (void)ncu;
    hipLaunchKernelGGL(k_direct, dim3(n), dim3(BKT_WG), 0, st, subs, units, n, res, uwit);
}

void launch_gather(const DevSub *subs, uint32_t nsub, uint64_t nbuckets, const unsigned long long *rec,
                   const uint32_t *starts, const uint32_t *conf, const uint32_t *wpos, unsigned long long base,
                   unsigned long long lo, unsigned long long hi, DevWitness *out, hipStream_t st) {
    if (!nbuckets) return;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)nbuckets), dim3(64), 0, st, subs, nsub, rec, starts, conf, wpos,
                       base, lo, hi, out);
}

}  // namespace rv
