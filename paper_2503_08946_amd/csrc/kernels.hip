// gfx950 kernels of the per-barrier-interval race check.
//
// Pipeline for one chunk of key-range passes (see plan.cpp):
//   k_hist     count: evaluate every instance (guards, bounds, location),
//              histogram the records per location bucket        [ALU, no record traffic]
//   k_scan_*   exclusive scan of the bucket counts -> bucket starts
//   k_scatter  expansion: evaluate the instances again, build the records
//              (location << 1 | rw, instance id) and write them grouped by
//              bucket through an LDS-staged counting sort (the most
//              significant radix digit of the location key)       [writes 8 B / record]
//   k_bucket   per bucket: load the records on chip, LDS radix sort on the
//              bucket's low key bits, segmented scan (ballot heads, DPP
//              reductions) giving per location (min id, max id, min write
//              id, max write id); flag conflicting locations, count them and
//              write canonical witnesses in location order           [reads 8 B / record]
//   k_finish / k_first   per-pass conflict totals and first witness.
//
// A location conflicts iff it has a write and two different threads touch
// it in the interval; with instance ids ordered thread-major that is
// (max write id + 1 != 0) && thread(min id) != thread(max id)  (the RaW / WaW /
// WaR relations of Section 2.1 restricted to one unordered barrier interval).

#include "rv_internal.h"

namespace rv {

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

// Inclusive wave64 prefix sum: Hillis-Steele inside each row of 16 lanes,
// then row 0 -> 1, row 2 -> 3 (bcast15) and lane 31 -> rows 2, 3 (bcast31).
__device__ __forceinline__ uint32_t wave_incl_add(uint32_t v) {
    v += dpp<ROW_SHR1, 0xf>(0u, v);
    v += dpp<ROW_SHR2, 0xf>(0u, v);
    v += dpp<ROW_SHR4, 0xf>(0u, v);
    v += dpp<ROW_SHR8, 0xf>(0u, v);
    v += dpp<ROW_BCAST15, 0xa>(0u, v);
    v += dpp<ROW_BCAST31, 0xc>(0u, v);
    return v;
}

// Exclusive prefix sum over a workgroup of NT threads; returns the prefix and
// writes the total to *total (all threads).  `red` holds NT/64 + 1 words.
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

// Rank of a record inside its bucket counter h[b] (unique per valid lane).
// All-equal waves (the common case for structured kernels) take one atomic.
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
__device__ __forceinline__ uint32_t sub_by_item(const DevSub *subs, uint32_t n, uint32_t w) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (subs[mid].item_begin <= w) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t sub_by_bucket(const DevSub *subs, uint32_t n, uint32_t b) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (subs[mid].bucket_begin <= b) lo = mid; else hi = mid;
    }
    return lo;
}

struct Item {
    const DevSub *S;
    const DevEntry *E;
    uint32_t gtile, lchunk;
};

__device__ __forceinline__ Item resolve_item(const DevSub *subs, uint32_t nsub, uint32_t w) {
    Item it;
    it.S = subs + sub_by_item(subs, nsub, w);
    const uint32_t local = w - it.S->item_begin;
    const uint32_t *pre = it.S->entry_items;
    uint32_t lo = 0, hi = it.S->n_entries;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= local) lo = mid; else hi = mid;
    }
    it.E = it.S->entries + lo;
    const uint32_t li = local - pre[lo];
    const uint32_t nl = it.E->n_lchunks;
    it.gtile = li / nl;
    it.lchunk = li - it.gtile * nl;
    return it;
}

// Evaluate the RPL instance slots of this lane in one work item and call
// f(slot, valid, in_bounds, location, id) for each.  A work item covers
// `lch` consecutive loop points of `gt` threads per lane; the loop counters
// are wave-uniform, the thread decode is per lane and per thread.
template <class F>
__device__ __forceinline__ void expand_item(const Item &it, F &&f) {
    const DevSub &S = *it.S;
    const DevEntry &E = *it.E;
    const DevKernel &K = *S.kc;
    const int32_t *__restrict__ G = S.guards;
    const uint32_t lch = E.lch, gt = E.gt;
    const uint32_t lstart = it.lchunk * lch;
    const uint32_t lcnt = min(lch, E.box - lstart);
    const uint32_t e1 = E.ext[1], e2 = E.ext[2];
    uint32_t c0s, c1s, c2s;
    {
        uint32_t r = lstart;
        c2s = r % e2; r /= e2;
        c1s = r % e1; r /= e1;
        c0s = r;
    }
    uint32_t c0 = c0s, c1 = c1s, c2 = c2s;
    uint32_t gi = 0, li = 0;
    int32_t tx = 0, ty = 0, bx = 0, by = 0;
    int32_t base[5] = {0, 0, 0, 0, 0};
    uint32_t idbase = 0, locbase = 0;
    bool gval = false;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const bool active = gi < gt;
        if (active && li == 0) {
            const uint32_t g = (it.gtile * gt + gi) * EXP_WG + threadIdx.x;
            gval = g < K.nthreads;
            const uint32_t gg = gval ? g : 0u;
            const uint32_t blk = udiv(gg, K.mg_tpb);
            const uint32_t tid = gg - blk * K.tpb;
            const uint32_t byy = udiv(blk, K.mg_gdx);
            const uint32_t tyy = udiv(tid, K.mg_bdx);
            tx = (int32_t)(tid - tyy * K.bdx);
            ty = (int32_t)tyy;
            bx = (int32_t)(blk - byy * K.gdx);
            by = (int32_t)byy;
#pragma unroll
            for (int r = 0; r < 5; r++)
                base[r] = E.row[r][C_TX] * tx + E.row[r][C_TY] * ty + E.row[r][C_BX] * bx +
                          E.row[r][C_BY] * by + E.row[r][C_C0];
            idbase = gg * S.M + E.off + lstart;
            locbase = blk * E.loc_mul + E.loc_base;
        }
        bool ok = false, inb = false;
        uint32_t loc = 0, id = 0;
        if (active) {
            const int32_t L0 = E.lo[0] + (int32_t)c0, L1 = E.lo[1] + (int32_t)c1, L2 = E.lo[2] + (int32_t)c2;
            int32_t a[2] = {0, 0};
#pragma unroll
            for (int x = 0; x < 2; x++) {
                if (E.aux_kind[x]) {
                    const int32_t n = base[3 + x] + E.row[3 + x][C_L0] * L0 + E.row[3 + x][C_L1] * L1 +
                                      E.row[3 + x][C_L2] * L2;
                    a[x] = E.aux_kind[x] == RV_AUX_FLOORDIV ? fdiv(n, E.aux_mg[x]) : emod(n, E.aux_mg[x]);
                }
            }
            ok = gval && li < lcnt;
            for (uint32_t q = 0; q < E.guard_count; q++) {
                const int32_t *gr = G + (size_t)(E.guard_begin + q) * NC;
                const int32_t gv = gr[C_TX] * tx + gr[C_TY] * ty + gr[C_BX] * bx + gr[C_BY] * by +
                                   gr[C_L0] * L0 + gr[C_L1] * L1 + gr[C_L2] * L2 + gr[C_A0] * a[0] +
                                   gr[C_A1] * a[1] + gr[C_C0];
                ok = ok && gv >= 0;
            }
            int32_t ix[3];
#pragma unroll
            for (int r = 0; r < 3; r++)
                ix[r] = base[r] + E.row[r][C_L0] * L0 + E.row[r][C_L1] * L1 + E.row[r][C_L2] * L2 +
                        E.row[r][C_A0] * a[0] + E.row[r][C_A1] * a[1];
            inb = (uint32_t)ix[0] < E.dim[0] && (uint32_t)ix[1] < E.dim[1] && (uint32_t)ix[2] < E.dim[2];
            const uint32_t flat = ((uint32_t)ix[0] * E.dim[1] + (uint32_t)ix[1]) * E.dim[2] + (uint32_t)ix[2];
            loc = locbase + flat;
            id = idbase + li;
        }
        f(s, ok, inb, loc, id);
        if (active) {
            li++;
            if (li == lch) {
                li = 0;
                gi++;
                c0 = c0s; c1 = c1s; c2 = c2s;
            } else {
                c2++;
                if (c2 == e2) { c2 = 0; c1++; if (c1 == e1) { c1 = 0; c0++; } }
            }
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
        z.records = 0; z.conflicts = 0; z.oob = ~0ull; z.first_bucket = ~0u; z.pad = 0;
        z.w[0] = z.w[1] = z.w[2] = z.w[3] = 0;
        r[i] = z;
    }
}

// --------------------------------------------------------------- count pass
__global__ void __launch_bounds__(EXP_WG) k_hist(const DevSub *__restrict__ subs, uint32_t nsub,
                                                  uint32_t *__restrict__ counts, SubResult *__restrict__ res) {
    __shared__ uint32_t h[NBMAX];
    __shared__ uint32_t red[EXP_WG / 64 + 1];
    const Item it = resolve_item(subs, nsub, blockIdx.x);
    const DevSub &S = *it.S;
    for (uint32_t i = threadIdx.x; i < S.nb; i += EXP_WG) h[i] = 0;
    __syncthreads();
    const uint32_t span = S.khi - S.klo;
    uint32_t mine = 0;
    expand_item(it, [&](int, bool ok, bool inb, uint32_t loc, uint32_t id) {
        if (ok && !inb) atomicMin(&res[S.res].oob, ((unsigned long long)S.interval << 32) | id);
        const uint32_t rel = loc - S.klo;
        const bool v = ok && inb && rel < span;
        lds_rank(h, rel >> S.s, v);
        mine += v ? 1u : 0u;
    });
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < S.nb; i += EXP_WG) {
        const uint32_t c = h[i];
        if (c) atomicAdd(&counts[S.bucket_begin + i], c);
    }
    uint32_t tot;
    block_excl_add<EXP_WG>(mine, red, &tot);
    if (threadIdx.x == 0 && tot) atomicAdd(&res[S.res].records, (unsigned long long)tot);
}

// ------------------------------------------------------------------ scans
constexpr int SCAN_WG = 256, SCAN_PER = 16, SCAN_TILE = SCAN_WG * SCAN_PER;

__global__ void __launch_bounds__(SCAN_WG) k_scan_up(const uint32_t *__restrict__ in, size_t n,
                                                      uint32_t *__restrict__ bsum) {
    __shared__ uint32_t red[SCAN_WG / 64 + 1];
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
    __shared__ uint32_t red[SCAN_WG / 64 + 1];
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
    __shared__ uint32_t red[SCAN_WG / 64 + 1];
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
__global__ void __launch_bounds__(EXP_WG) k_scatter(const DevSub *__restrict__ subs, uint32_t nsub,
                                                     unsigned long long *__restrict__ rec,
                                                     uint32_t *__restrict__ cursor) {
    __shared__ unsigned long long stage[TILE];
    __shared__ uint32_t h[NBMAX];
    __shared__ uint32_t dl[NBMAX];
    __shared__ uint32_t red[EXP_WG / 64 + 1];
    const Item it = resolve_item(subs, nsub, blockIdx.x);
    const DevSub &S = *it.S;
    const uint32_t nb = S.nb;
    for (uint32_t i = threadIdx.x; i < nb; i += EXP_WG) h[i] = 0;
    __syncthreads();
    const uint32_t span = S.khi - S.klo;
    const uint32_t rwbit = it.E->rw;
    unsigned long long r[RPL];
    uint32_t bk[RPL], rk[RPL];
    expand_item(it, [&](int s, bool ok, bool inb, uint32_t loc, uint32_t id) {
        const uint32_t rel = loc - S.klo;
        const bool v = ok && inb && rel < span;
        const uint32_t b = rel >> S.s;
        rk[s] = lds_rank(h, b, v);
        bk[s] = v ? b : 0xFFFFFFFFu;
        r[s] = ((unsigned long long)((loc << 1) | rwbit) << 32) | id;
    });
    __syncthreads();
    // exclusive scan of the tile histogram (each thread owns a run of bins)
    constexpr int PER = NBMAX / EXP_WG;
    const uint32_t b0 = threadIdx.x * PER;
    uint32_t hv[PER];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < PER; i++) {
        hv[i] = (b0 + i < nb) ? h[b0 + i] : 0u;
        sum += hv[i];
    }
    uint32_t total;
    uint32_t run = block_excl_add<EXP_WG>(sum, red, &total);
#pragma unroll
    for (int i = 0; i < PER; i++) {
        if (b0 + i < nb) h[b0 + i] = run;
        run += hv[i];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < RPL; s++)
        if (bk[s] != 0xFFFFFFFFu) stage[h[bk[s]] + rk[s]] = r[s];
    // reserve the bucket ranges in the chunk: one atomic per nonempty bucket
#pragma unroll
    for (int i = 0; i < PER; i++) {
        const uint32_t b = b0 + i;
        if (b < nb && hv[i]) dl[b] = atomicAdd(&cursor[S.bucket_begin + b], hv[i]) - h[b];
    }
    __syncthreads();
    for (uint32_t p = threadIdx.x; p < total; p += EXP_WG) {
        const unsigned long long v = stage[p];
        const uint32_t b = ((uint32_t)(v >> 33) - S.klo) >> S.s;
        rec[dl[b] + p] = v;
    }
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
    if (b.f) {
        acc = b;
    } else {
        acc.mn = min(acc.mn, b.mn);
        acc.mx = max(acc.mx, b.mx);
        acc.mnw = min(acc.mnw, b.mnw);
        acc.mxw1 = max(acc.mxw1, b.mxw1);
    }
}

constexpr int TBL = 1 << SMAX;

__global__ void __launch_bounds__(BKT_WG) k_bucket(const DevSub *__restrict__ subs, uint32_t nsub,
                                                    unsigned long long *__restrict__ rec,
                                                    const uint32_t *__restrict__ starts,
                                                    const uint32_t *__restrict__ counts,
                                                    uint32_t *__restrict__ conf, int debug_sorted) {
    __shared__ uint32_t sid[CAP];
    __shared__ uint16_t sk[CAP];
    __shared__ uint32_t bins[TBL];
    __shared__ uint32_t t_mn[TBL], t_mx[TBL], t_mnw[TBL], t_mxw1[TBL];
    __shared__ Seg wtot[BKT_WG / 64];
    __shared__ uint32_t red[BKT_WG / 64 + 1];

    const uint32_t b = blockIdx.x;
    const uint32_t cnt = counts[b];
    if (cnt == 0) {
        if (threadIdx.x == 0) conf[b] = 0;
        return;
    }
    const DevSub &S = subs[sub_by_bucket(subs, nsub, b)];
    const uint32_t lo = S.klo + ((b - S.bucket_begin) << S.s);
    const uint32_t width = min(1u << S.s, S.khi - lo);
    const uint32_t start = starts[b];
    const uint32_t t = threadIdx.x;
    const uint32_t wid = t >> 6;
    if (t < TBL) {
        t_mn[t] = 0xFFFFFFFFu; t_mx[t] = 0; t_mnw[t] = 0xFFFFFFFFu; t_mxw1[t] = 0;
    }

    for (uint32_t slice = 0; slice < cnt; slice += CAP) {
        const uint32_t n = min((uint32_t)CAP, cnt - slice);
        const unsigned long long *src = rec + start + slice;
        unsigned long long r[BKT_RPL];
#pragma unroll
        for (int i = 0; i < BKT_RPL; i++) {
            const uint32_t j = (uint32_t)i * BKT_WG + t;
            r[i] = j < n ? src[j] : 0ull;
        }
        if (t < TBL) bins[t] = 0;
        __syncthreads();
        // --- LDS radix sort, one digit of `s` bits (the bucket's local key)
        uint32_t kk[BKT_RPL], off[BKT_RPL];
#pragma unroll
        for (int i = 0; i < BKT_RPL; i++) {
            const bool v = (uint32_t)i * BKT_WG + t < n;
            kk[i] = v ? ((uint32_t)(r[i] >> 33) - lo) : 0u;
            off[i] = lds_rank(bins, kk[i], v);
        }
        __syncthreads();
        {
            uint32_t tot;
            const uint32_t x = t < TBL ? bins[t] : 0u;
            const uint32_t ex = block_excl_add<BKT_WG>(x, red, &tot);
            if (t < TBL) bins[t] = ex;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < BKT_RPL; i++) {
            if ((uint32_t)i * BKT_WG + t < n) {
                const uint32_t pos = bins[kk[i]] + off[i];
                sid[pos] = (uint32_t)r[i];
                sk[pos] = (uint16_t)(kk[i] | (((uint32_t)(r[i] >> 32) & 1u) << 15));
            }
        }
        __syncthreads();
        if (debug_sorted) {
            for (uint32_t j = t; j < n; j += BKT_WG) {
                const uint32_t key = sk[j];
                const uint32_t hi = ((lo + (key & 0x7FFFu)) << 1) | (key >> 15);
                rec[start + slice + j] = ((unsigned long long)hi << 32) | sid[j];
            }
        }
        // --- segmented scan over runs of equal key
        const uint32_t r0 = t * BKT_RPL;
        const uint32_t r1 = min(r0 + BKT_RPL, n);
        Seg a{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
        uint32_t prevk = r0 > 0 && r0 < n ? (sk[r0 - 1] & 0x7FFFu) : 0xFFFFu;
        for (uint32_t j = r0; j < r1; j++) {
            const uint32_t key = sk[j];
            const uint32_t k = key & 0x7FFFu;
            if (k != prevk) {   // head (j == 0 always is: prevk starts out of range)
                a.f = 1; a.mn = 0xFFFFFFFFu; a.mx = 0; a.mnw = 0xFFFFFFFFu; a.mxw1 = 0;
            }
            seg_add(a, sid[j], key >> 15);
            prevk = k;
        }
        // inclusive segmented scan across the wave (DPP), then exclusive
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
        // finalize segments that end in this run
        if (r0 < r1) {
            const uint32_t k0 = sk[r0] & 0x7FFFu;
            const bool head0 = (r0 == 0) || ((sk[r0 - 1] & 0x7FFFu) != k0);
            Seg cur = head0 ? Seg{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u} : carry;
            uint32_t pk = k0;
            for (uint32_t j = r0; j < r1; j++) {
                const uint32_t key = sk[j];
                const uint32_t k = key & 0x7FFFu;
                if (j != r0 && k != pk) {
                    atomicMin(&t_mn[pk], cur.mn);
                    atomicMax(&t_mx[pk], cur.mx);
                    atomicMin(&t_mnw[pk], cur.mnw);
                    atomicMax(&t_mxw1[pk], cur.mxw1);
                    cur = Seg{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu, 0u};
                }
                seg_add(cur, sid[j], key >> 15);
                pk = k;
            }
            const bool ends = (r1 == n) || ((sk[r1] & 0x7FFFu) != pk);
            if (ends) {
                atomicMin(&t_mn[pk], cur.mn);
                atomicMax(&t_mx[pk], cur.mx);
                atomicMin(&t_mnw[pk], cur.mnw);
                atomicMax(&t_mxw1[pk], cur.mxw1);
            }
        }
        __syncthreads();
    }

    // --- flag conflicting locations, in key order
    bool c = false;
    uint32_t mnw = 0, second = 0, srw = 0;
    if (t < width) {
        const uint32_t mn = t_mn[t];
        const uint32_t mxw1 = t_mxw1[t];
        if (mn != 0xFFFFFFFFu && mxw1 != 0u) {
            const uint32_t mx = t_mx[t];
            mnw = t_mnw[t];
            const uint32_t th_mn = udiv(mn, S.mgM), th_mx = udiv(mx, S.mgM);
            if (th_mn != th_mx) {
                c = true;
                const uint32_t th_w = udiv(mnw, S.mgM);
                if (th_mn != th_w) { second = mn; srw = (mn == mnw) ? 1u : 0u; }
                else { second = mx; srw = (mx + 1 == mxw1) ? 1u : 0u; }
            }
        }
    }
    uint32_t total;
    const uint32_t pos = block_excl_add<BKT_WG>(c ? 1u : 0u, red, &total);
    if (c && !debug_sorted) {   // the region start is 8-byte aligned: store words
        uint32_t *w = reinterpret_cast<uint32_t *>(rec + start) + 4 * (size_t)pos;
        w[0] = lo + t; w[1] = mnw; w[2] = second; w[3] = srw;
    }
    if (t == 0) conf[b] = total;
}

// ------------------------------------------------------------- finishing
__global__ void k_finish(const DevSub *__restrict__ subs, uint32_t nsub, size_t nbuckets,
                         const uint32_t *__restrict__ conf, SubResult *__restrict__ res) {
    const size_t b = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbuckets) return;
    const uint32_t c = conf[b];
    if (!c) return;
    const DevSub &S = subs[sub_by_bucket(subs, nsub, (uint32_t)b)];
    atomicAdd(&res[S.res].conflicts, (unsigned long long)c);
    atomicMin(&res[S.res].first_bucket, (uint32_t)b);
}

__global__ void k_first(const DevSub *__restrict__ subs, uint32_t nsub, const unsigned long long *__restrict__ rec,
                        const uint32_t *__restrict__ starts, SubResult *__restrict__ res) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nsub) return;
    SubResult &R = res[subs[j].res];
    const uint32_t fb = R.first_bucket;
    if (fb == 0xFFFFFFFFu) return;
    const uint32_t *w = reinterpret_cast<const uint32_t *>(rec + starts[fb]);
    R.w[0] = w[0]; R.w[1] = w[1]; R.w[2] = w[2]; R.w[3] = w[3];
}

__global__ void k_gather(const DevSub *__restrict__ subs, uint32_t nsub, const unsigned long long *__restrict__ rec,
                         const uint32_t *__restrict__ starts, const uint32_t *__restrict__ conf,
                         const uint32_t *__restrict__ wpos, unsigned long long base, unsigned long long lo,
                         unsigned long long hi, DevWitness *__restrict__ out) {
    const uint32_t b = blockIdx.x;
    const uint32_t c = conf[b];
    if (!c) return;
    const unsigned long long first = base + wpos[b];
    if (first >= hi || first + c <= lo) return;
    const uint32_t sub = subs[sub_by_bucket(subs, nsub, b)].res;
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

// --------------------------------------------------------------- launchers
static inline unsigned grid_for(size_t n, unsigned per) {
    size_t g = (n + per - 1) / per;
    return (unsigned)(g < 1 ? 1 : (g > 65535u * 16 ? 65535u * 16 : g));
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
                 hipStream_t st) {
    if (!items) return;
    hipLaunchKernelGGL(k_hist, dim3((unsigned)items), dim3(EXP_WG), 0, st, subs, nsub, counts, res);
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
                    hipStream_t st) {
    if (!items) return;
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)items), dim3(EXP_WG), 0, st, subs, nsub, rec, cursor);
}

void launch_bucket(const DevSub *subs, uint32_t nsub, uint64_t nbuckets, unsigned long long *rec,
                   const uint32_t *starts, const uint32_t *counts, uint32_t *conf, int debug_sorted,
                   hipStream_t st) {
    if (!nbuckets) return;
    hipLaunchKernelGGL(k_bucket, dim3((unsigned)nbuckets), dim3(BKT_WG), 0, st, subs, nsub, rec, starts, counts,
                       conf, debug_sorted);
}

void launch_finish(const DevSub *subs, uint32_t nsub, uint64_t nbuckets, const uint32_t *conf, SubResult *res,
                   hipStream_t st) {
    if (!nbuckets) return;
    hipLaunchKernelGGL(k_finish, dim3((unsigned)((nbuckets + 255) / 256)), dim3(256), 0, st, subs, nsub,
                       (size_t)nbuckets, conf, res);
}

void launch_first(const DevSub *subs, uint32_t nsub, const unsigned long long *rec, const uint32_t *starts,
                  SubResult *res, hipStream_t st) {
    if (!nsub) return;
    hipLaunchKernelGGL(k_first, dim3((nsub + 63) / 64), dim3(64), 0, st, subs, nsub, rec, starts, res);
}

void launch_gather(const DevSub *subs, uint32_t nsub, uint64_t nbuckets, const unsigned long long *rec,
                   const uint32_t *starts, const uint32_t *conf, const uint32_t *wpos, unsigned long long base,
                   unsigned long long lo, unsigned long long hi, DevWitness *out, hipStream_t st) {
    if (!nbuckets) return;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)nbuckets), dim3(64), 0, st, subs, nsub, rec, starts, conf, wpos,
                       base, lo, hi, out);
}

}  // namespace rv
