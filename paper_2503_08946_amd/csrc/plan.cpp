// Host planner: validates a description, expands its schedule into dynamic
// phases and barrier intervals, lays out each interval's location space and
// splits the work into key-range passes and workspace-sized chunks.
//
// Schedule and intervals: the paper orders code sections by schedule vectors
// and derives happens-before from that order (Section 2.1 step 5; the Before
// relation of the appendix listings).  In a SIMT block only a barrier orders
// the accesses of different threads, so the unit of the check is the barrier
// interval: interval(d) = number of barriers executed before dynamic phase d.

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "rv_internal.h"

namespace rv {

Magic make_magic(uint32_t d) {
    Magic g{};
    uint32_t l = 0;
    while (l < 32 && (uint64_t(1) << l) < d) l++;
    // m = floor(2^32 * (2^l - d) / d) + 1 ; fits 32 bits for d <= 2^31
    uint64_t m = ((((uint64_t)1 << l) - d) << 32) / d + 1;
    g.m = (uint32_t)m;
    g.s1 = l ? 1u : 0u;
    g.s2 = l ? l - 1 : 0u;
    g.d = d;
    return g;
}

static std::string fmt(const char *f, long long a = 0, long long b = 0, long long c = 0) {
    char buf[256];
    snprintf(buf, sizeof buf, f, a, b, c);
    return buf;
}

rv_status validate(const rv_kernel_desc *d, std::string &msg) {
    if (!d) { msg = "null description"; return RV_ERR_INVALID; }
    const rv_launch &L = d->launch;
    for (int i = 0; i < 2; i++)
        if (L.block[i] < 1 || L.grid[i] < 1) { msg = "launch dimensions must be >= 1"; return RV_ERR_INVALID; }
    if (L.block[2] < 1 || L.grid[2] < 1) { msg = "launch z dimension must be 1"; return RV_ERR_INVALID; }
    if (L.block[2] > 1 || L.grid[2] > 1) { msg = "launch z dimension > 1 is not supported"; return RV_ERR_UNSUPPORTED; }
    if (d->n_arrays < 0 || d->n_accesses < 0 || d->n_guards < 0 || d->n_phases < 0 || d->n_segments < 0) {
        msg = "negative count"; return RV_ERR_INVALID;
    }
    if ((d->n_arrays && !d->arrays) || (d->n_accesses && !d->accesses) || (d->n_guards && !d->guards) ||
        (d->n_phases && !d->phases) || (d->n_segments && !d->segments)) {
        msg = "null table with a nonzero count"; return RV_ERR_INVALID;
    }
    for (int i = 0; i < d->n_arrays; i++) {
        const rv_array &a = d->arrays[i];
        if (a.space != RV_SHARED && a.space != RV_GLOBAL) { msg = fmt("array %lld: bad space", i); return RV_ERR_INVALID; }
        if (a.ndim < 1 || a.ndim > 3) { msg = fmt("array %lld: ndim must be 1..3", i); return RV_ERR_INVALID; }
        long double n = 1;
        for (int j = 0; j < a.ndim; j++) {
            if (a.dim[j] < 1) { msg = fmt("array %lld: dims must be >= 1", i); return RV_ERR_INVALID; }
            n *= (long double)a.dim[j];
        }
        if (n >= 2147483648.0L) { msg = fmt("array %lld: more than 2^31-1 elements", i); return RV_ERR_KEY_BITS; }
    }
    for (int i = 0; i < d->n_accesses; i++) {
        const rv_access &a = d->accesses[i];
        if (a.array < 0 || a.array >= d->n_arrays) { msg = fmt("access %lld: bad array", i); return RV_ERR_INVALID; }
        if (a.nloops < 0 || a.nloops > 3) { msg = fmt("access %lld: nloops must be 0..3", i); return RV_ERR_INVALID; }
        for (int l = 0; l < a.nloops; l++)
            if (a.loop_lo[l] > a.loop_hi[l]) { msg = fmt("access %lld: loop %lld has lo > hi", i, l); return RV_ERR_INVALID; }
        for (int x = 0; x < 2; x++) {
            const rv_aux &u = a.aux[x];
            if (u.kind < RV_AUX_NONE || u.kind > RV_AUX_EMOD) { msg = fmt("access %lld: bad aux kind", i); return RV_ERR_INVALID; }
            if (u.kind != RV_AUX_NONE && u.d < 1) { msg = fmt("access %lld: aux divisor must be >= 1", i); return RV_ERR_INVALID; }
            if (u.e.coef[RV_V_AUX0] || u.e.coef[RV_V_AUX1]) {
                msg = fmt("access %lld: an aux numerator may not use aux variables", i); return RV_ERR_INVALID;
            }
        }
        if (a.guard_begin < 0 || a.guard_count < 0 || (int64_t)a.guard_begin + a.guard_count > d->n_guards) {
            msg = fmt("access %lld: bad guard range", i); return RV_ERR_INVALID;
        }
    }
    if (d->warp_size < 0) { msg = "warp_size must be >= 0 (0: 32)"; return RV_ERR_INVALID; }
    for (int i = 0; i < d->n_phases; i++) {
        const rv_phase &p = d->phases[i];
        if (p.access_begin < 0 || p.access_count < 0 || (int64_t)p.access_begin + p.access_count > d->n_accesses) {
            msg = fmt("phase %lld: bad access range", i); return RV_ERR_INVALID;
        }
        if (p.barrier_after < RV_BARRIER_NONE || p.barrier_after > RV_BARRIER_WARP) {
            msg = fmt("phase %lld: bad barrier kind", i); return RV_ERR_INVALID;
        }
        if (p.guard_begin < 0 || p.guard_count < 0 || (int64_t)p.guard_begin + p.guard_count > d->n_guards ||
            (p.guard_count && p.barrier_after == RV_BARRIER_NONE)) {
            msg = fmt("phase %lld: bad barrier guard range", i); return RV_ERR_INVALID;
        }
        for (int g = p.guard_begin; g < p.guard_begin + p.guard_count; g++)
            for (int v = RV_V_L0; v < RV_NV; v++)
                if (d->guards[g].g.coef[v]) {
                    msg = fmt("phase %lld: a barrier guard may use tx, ty, bx, by and k only", i);
                    return RV_ERR_INVALID;
                }
    }
    for (int i = 0; i < d->n_segments; i++) {
        const rv_segment &s = d->segments[i];
        if (s.phase_begin < 0 || s.phase_count < 0 || (int64_t)s.phase_begin + s.phase_count > d->n_phases) {
            msg = fmt("segment %lld: bad phase range", i); return RV_ERR_INVALID;
        }
        if (s.repeat < 1) { msg = fmt("segment %lld: repeat must be >= 1", i); return RV_ERR_INVALID; }
    }
    return RV_OK;
}

static uint64_t arr_size(const rv_array &a) {
    uint64_t n = 1;
    for (int j = 0; j < a.ndim; j++) n *= (uint64_t)a.dim[j];
    return n;
}

// Upper bound of |value| of an affine row over the iteration box.
static long double row_bound(const int32_t *row, const long double *vmax) {
    long double b = std::fabs((long double)row[C_C0]);
    for (int v = 0; v < C_C0; v++) b += std::fabs((long double)row[v]) * vmax[v];
    return b;
}

static uint32_t ceil_log2(uint64_t n) {
    uint32_t w = 0;
    while ((1ull << w) < n) w++;
    return w;
}

rv_status plan_kernel(const rv_kernel_desc *d, int target, rv_kernel &k, std::string &msg, int semantics) {
    rv_status st = validate(d, msg);
    if (st) return st;
    if (semantics != RV_SEM_INTERVAL && semantics != RV_SEM_STRICT && semantics != RV_SEM_ORDERED) {
        msg = "unknown semantics"; return RV_ERR_INVALID;
    }
    k.semantics = semantics;
    k.launch = d->launch;
    k.arrays.assign(d->arrays, d->arrays + d->n_arrays);
    k.accesses.assign(d->accesses, d->accesses + d->n_accesses);
    k.guards.assign(d->guards, d->guards + d->n_guards);
    k.phases.assign(d->phases, d->phases + d->n_phases);
    k.segments.assign(d->segments, d->segments + d->n_segments);
    k.target = target > 0 ? target : DEFAULT_TARGET;

    const uint64_t bdx = d->launch.block[0], bdy = d->launch.block[1];
    const uint64_t gdx = d->launch.grid[0], gdy = d->launch.grid[1];
    const uint64_t tpb = bdx * bdy, nblocks = gdx * gdy, nthreads = tpb * nblocks;
    if (nthreads >= (1ull << 31)) { msg = "more than 2^31 threads"; return RV_ERR_TOO_LARGE; }
    k.kc.bdx = (uint32_t)bdx; k.kc.bdy = (uint32_t)bdy; k.kc.gdx = (uint32_t)gdx; k.kc.gdy = (uint32_t)gdy;
    k.kc.tpb = (uint32_t)tpb; k.kc.nthreads = (uint32_t)nthreads; k.kc.nblocks = (uint32_t)nblocks;
    k.kc.mg_tpb = make_magic((uint32_t)tpb);
    k.kc.mg_bdx = make_magic((uint32_t)bdx);
    k.kc.mg_gdx = make_magic((uint32_t)gdx);

    // ---- dynamic phases and barrier intervals
    uint64_t ndyn = 0;
    for (auto &s : k.segments) ndyn += (uint64_t)s.repeat * s.phase_count;
    if (ndyn >= (1ull << 31)) { msg = "too many dynamic phases"; return RV_ERR_TOO_LARGE; }
    k.dyn_phase.clear(); k.dyn_k.clear(); k.dyn_interval.clear();
    std::vector<uint32_t> dyn_fine;   // barriers of either kind before each dynamic phase
    uint32_t barriers = 0, fine = 0;
    for (auto &s : k.segments)
        for (int r = 0; r < s.repeat; r++)
            for (int j = 0; j < s.phase_count; j++) {
                uint32_t ph = s.phase_begin + j;
                k.dyn_phase.push_back(ph);
                k.dyn_k.push_back(s.k_base + r);
                k.dyn_interval.push_back(barriers);
                dyn_fine.push_back(fine);
                if (k.phases[ph].barrier_after == RV_BARRIER_BLOCK) barriers++;
                if (k.phases[ph].barrier_after != RV_BARRIER_NONE) fine++;
                if (k.phases[ph].barrier_after == RV_BARRIER_WARP && semantics == RV_SEM_STRICT) {
                    msg = "strict semantics with warp barriers are not supported";
                    return RV_ERR_UNSUPPORTED;
                }
            }
    k.n_intervals = k.dyn_phase.empty() ? 0 : k.dyn_interval.back() + 1;
    const uint32_t warp = d->warp_size > 0 ? (uint32_t)d->warp_size : 32u;

    // ---- barriers: their instances, and the guarded ones for the divergence
    // check (guard rows over tx, ty, bx, by with k folded into the constant)
    k.guard_rows.clear();
    k.barriers.clear();
    k.barrier_instances = 0;
    for (size_t dd = 0; dd < k.dyn_phase.size(); dd++) {
        const rv_phase &ph = k.phases[k.dyn_phase[dd]];
        if (ph.barrier_after == RV_BARRIER_NONE) continue;
        const uint32_t scope = ph.barrier_after == RV_BARRIER_BLOCK ? (uint32_t)tpb
                                                                     : std::min<uint32_t>(warp, (uint32_t)tpb);
        const uint32_t nscope = (uint32_t)((tpb + scope - 1) / scope);
        k.barrier_instances += nblocks * nscope;
        if (!ph.guard_count) continue;
        DevBarrier B{};
        B.dphase = (uint32_t)dd;
        B.guard_begin = (uint32_t)(k.guard_rows.size() / NC);
        B.guard_count = (uint32_t)ph.guard_count;
        B.scope = scope;
        B.nscope = nscope;
        for (int g = ph.guard_begin; g < ph.guard_begin + ph.guard_count; g++) {
            const rv_affine &f = k.guards[g].g;
            int32_t row[NC] = {0};
            const int64_t c0 = (int64_t)f.c0 + (int64_t)f.coef[RV_V_K] * k.dyn_k[dd];
            row[C_TX] = f.coef[RV_V_TX]; row[C_TY] = f.coef[RV_V_TY];
            row[C_BX] = f.coef[RV_V_BX]; row[C_BY] = f.coef[RV_V_BY];
            long double b = std::fabs((long double)c0) + std::fabs((long double)row[C_TX]) * (long double)(bdx - 1) +
                            std::fabs((long double)row[C_TY]) * (long double)(bdy - 1) +
                            std::fabs((long double)row[C_BX]) * (long double)(gdx - 1) +
                            std::fabs((long double)row[C_BY]) * (long double)(gdy - 1);
            if (b > 2147483647.0L) {
                msg = fmt("dynamic phase %lld: a barrier guard may leave int32", (long long)dd);
                return RV_ERR_RANGE;
            }
            row[C_C0] = (int32_t)c0;
            k.guard_rows.insert(k.guard_rows.end(), row, row + NC);
        }
        k.barriers.push_back(B);
    }

    // ---- the planned location spaces ("virtual intervals").  Interval
    // semantics: one per barrier interval; the fine interval of each dynamic
    // phase inside it (warp barriers) becomes a sub-key below the location,
    // and warps are the unordered units.  Strict semantics: the barrier
    // intervals keep the shared arrays only, and one more space holds the
    // global arrays of the whole kernel with the interval as the sub-key and
    // blocks as the units (blocks are never ordered).
    struct Virt { uint32_t d0, d1, space_mask; bool strict_global; };
    std::vector<Virt> virt;
    if (semantics == RV_SEM_ORDERED) {
        // the sequential schedule: one space over every dynamic phase
        virt.push_back(Virt{0, (uint32_t)k.dyn_phase.size(), 3u, false});
    } else {
        uint32_t d0 = 0;
        for (uint32_t iv = 0; iv < k.n_intervals; iv++) {
            uint32_t d1 = d0;
            while (d1 < k.dyn_phase.size() && k.dyn_interval[d1] == iv) d1++;
            virt.push_back(Virt{d0, d1, semantics == RV_SEM_STRICT ? 1u : 3u, false});
            d0 = d1;
        }
        if (semantics == RV_SEM_STRICT) virt.push_back(Virt{0, (uint32_t)k.dyn_phase.size(), 2u, true});
    }

    // ---- per planned space: entries, layout, ranges, buckets
    k.entries.clear(); k.hentries.clear(); k.entry_items.clear(); k.entry_items_g.clear();
    k.intervals.assign(virt.size(), IntervalPlan());
    k.subs.clear();
    k.n_instances = 0; k.max_interval_instances = 0; k.n_buckets = 0;
    k.has_subkeys = false;
    for (uint32_t iv = 0; iv < virt.size(); iv++) {
        IntervalPlan &I = k.intervals[iv];
        const uint32_t d0 = virt[iv].d0, d1 = virt[iv].d1, smask = virt[iv].space_mask;
        auto in_space = [&](int a) { return (smask >> k.arrays[k.accesses[a].array].space) & 1u; };
        I.dphase_begin = d0; I.dphase_end = d1;
        I.entry_begin = (uint32_t)k.entries.size();
        I.arr_off.assign(k.arrays.size(), -1);
        // sub-key of each dynamic phase and its width, and the unordered units
        uint32_t nsubk = 1, sub0 = 0;
        if (virt[iv].strict_global) {
            nsubk = std::max<uint32_t>(k.n_intervals, 1);
            I.unit = (uint32_t)tpb; I.upb = 1;
        } else if (d1 > d0) {
            sub0 = dyn_fine[d0];
            nsubk = dyn_fine[d1 - 1] - sub0 + 1;
            I.unit = std::min<uint32_t>(warp, (uint32_t)tpb); I.upb = (uint32_t)((tpb + warp - 1) / warp);
        }
        I.w = ceil_log2(nsubk);
        if (I.w > (uint32_t)SMAX) {
            msg = fmt("interval %lld: %lld barrier-separated parts exceed the sub-key (at most 512)", iv, nsubk);
            return RV_ERR_UNSUPPORTED;
        }
        if (semantics == RV_SEM_ORDERED) { I.w = 0; nsubk = 1; }
        if (I.w) k.has_subkeys = true;
        auto subkey = [&](uint32_t dd) {
            return virt[iv].strict_global ? k.dyn_interval[dd] : dyn_fine[dd] - sub0;
        };
        // touched arrays
        std::vector<char> touched(k.arrays.size(), 0);
        for (uint32_t dd = d0; dd < d1; dd++) {
            const rv_phase &ph = k.phases[k.dyn_phase[dd]];
            for (int a = ph.access_begin; a < ph.access_begin + ph.access_count; a++)
                if (in_space(a)) touched[k.accesses[a].array] = 1;
        }
        uint64_t S = 0, G = 0;
        for (size_t a = 0; a < k.arrays.size(); a++)
            if (touched[a] && k.arrays[a].space == RV_SHARED) { I.arr_off[a] = (int64_t)S; S += arr_size(k.arrays[a]); }
        for (size_t a = 0; a < k.arrays.size(); a++)
            if (touched[a] && k.arrays[a].space == RV_GLOBAL) { I.arr_off[a] = (int64_t)G; G += arr_size(k.arrays[a]); }
        I.S = S;
        I.K = (nblocks * S + G) << I.w;
        if (I.K >= (1ull << 31)) {
            msg = fmt("interval %lld: %lld location keys do not fit 31 bits", iv, (long long)I.K);
            return RV_ERR_KEY_BITS;
        }
        // Block-local spaces on chip are considered when the shared
        // locations of a block (S, no sub-keys) fit one unit's LDS table; a
        // unit then spans Tu threads (DIR_CAP / S blocks).  Ordered
        // semantics keep one space of kernel-wide time order.
        const bool dcand = semantics != RV_SEM_ORDERED && I.w == 0 && S > 0 && S <= DIR_CAP;
        const uint64_t Tu = dcand ? std::max<uint64_t>(1, DIR_CAP / S) * tpb : 0;
        // entries
        uint64_t M = 0;
        uint64_t obase = 0;     // ordered: id base of the dynamic phase (phase-major ids)
        for (uint32_t dd = d0; dd < d1; dd++) {
            const rv_phase &ph = k.phases[k.dyn_phase[dd]];
            const int32_t kval = k.dyn_k[dd];
            uint64_t pbox = 0;  // ordered: the phase's statement instances per thread
            if (semantics == RV_SEM_ORDERED) {
                for (int a = ph.access_begin; a < ph.access_begin + ph.access_count; a++) {
                    const rv_access &ac = k.accesses[a];
                    uint64_t b = 1;
                    for (int l = 0; l < ac.nloops; l++) b *= (uint64_t)((int64_t)ac.loop_hi[l] - ac.loop_lo[l]);
                    pbox = std::max(pbox, b);
                }
            }
            for (int a = ph.access_begin; a < ph.access_begin + ph.access_count; a++) {
                if (!in_space(a)) continue;
                const rv_access &ac = k.accesses[a];
                const rv_array &ar = k.arrays[ac.array];
                DevEntry E{};
                uint64_t box = 1;
                for (int l = 0; l < 3; l++) {
                    if (l < ac.nloops) {
                        E.lo[l] = ac.loop_lo[l];
                        E.ext[l] = (uint32_t)((int64_t)ac.loop_hi[l] - ac.loop_lo[l]);
                    } else {
                        E.lo[l] = 0;
                        E.ext[l] = 1;
                    }
                    box *= E.ext[l];
                }
                if (box >= (1ull << 32)) { msg = fmt("access %lld: loop box too large", a); return RV_ERR_TOO_LARGE; }
                E.nloops = ac.nloops;
                E.box = (uint32_t)box;
                E.off = (uint32_t)M;   // checked below through P
                if (semantics == RV_SEM_ORDERED) {
                    E.off = (uint32_t)obase;     // checked below through obase
                    E.tmul = (uint32_t)pbox;
                }
                E.rw = ac.is_write ? 1u : 0u;
                for (int j = 0; j < 3; j++) E.dim[j] = j < ar.ndim ? (uint32_t)ar.dim[j] : 1u;
                if (ar.space == RV_SHARED) { E.loc_mul = (uint32_t)S; E.loc_base = (uint32_t)I.arr_off[ac.array]; }
                else { E.loc_mul = 0; E.loc_base = (uint32_t)(nblocks * S + I.arr_off[ac.array]); }
                // value bounds of the variables over the box
                long double vmax[NC] = {0};
                vmax[C_TX] = (long double)(bdx - 1); vmax[C_TY] = (long double)(bdy - 1);
                vmax[C_BX] = (long double)(gdx - 1); vmax[C_BY] = (long double)(gdy - 1);
                for (int l = 0; l < ac.nloops; l++)
                    if (E.ext[l] > 0)
                        vmax[C_L0 + l] = std::max(std::fabs((long double)ac.loop_lo[l]),
                                                  std::fabs((long double)ac.loop_hi[l] - 1));
                auto fold = [&](const rv_affine &f, int32_t *row, bool &ok) {
                    int64_t c0 = (int64_t)f.c0 + (int64_t)f.coef[RV_V_K] * kval;
                    ok = c0 >= INT32_MIN && c0 <= INT32_MAX;
                    row[C_TX] = f.coef[RV_V_TX]; row[C_TY] = f.coef[RV_V_TY];
                    row[C_BX] = f.coef[RV_V_BX]; row[C_BY] = f.coef[RV_V_BY];
                    row[C_L0] = f.coef[RV_V_L0]; row[C_L1] = f.coef[RV_V_L1]; row[C_L2] = f.coef[RV_V_L2];
                    row[C_A0] = f.coef[RV_V_AUX0]; row[C_A1] = f.coef[RV_V_AUX1];
                    row[C_C0] = (int32_t)c0;
                };
                const long double LIM = 2147483647.0L;
                bool ok = true;
                for (int x = 0; x < 2; x++) {
                    const rv_aux &u = ac.aux[x];
                    E.aux_kind[x] = u.kind;
                    if (u.kind == RV_AUX_NONE) { E.aux_mg[x] = make_magic(1); continue; }
                    fold(u.e, E.row[3 + x], ok);
                    long double b = row_bound(E.row[3 + x], vmax);
                    if (!ok || b > LIM) { msg = fmt("access %lld: aux term may leave int32", a); return RV_ERR_RANGE; }
                    E.aux_mg[x] = make_magic((uint32_t)u.d);
                    vmax[C_A0 + x] = u.kind == RV_AUX_FLOORDIV ? b / (long double)u.d + 1 : (long double)(u.d - 1);
                }
                for (int j = 0; j < ar.ndim; j++) {
                    fold(ac.idx[j], E.row[j], ok);
                    if (!ok || row_bound(E.row[j], vmax) > LIM) {
                        msg = fmt("access %lld: index %lld may leave int32", a, j); return RV_ERR_RANGE;
                    }
                }
                E.guard_begin = (uint32_t)(k.guard_rows.size() / NC);
                E.guard_count = (uint32_t)ac.guard_count;
                for (int g = ac.guard_begin; g < ac.guard_begin + ac.guard_count; g++) {
                    int32_t row[NC];
                    fold(k.guards[g].g, row, ok);
                    if (!ok || row_bound(row, vmax) > LIM) { msg = fmt("access %lld: guard may leave int32", a); return RV_ERR_RANGE; }
                    k.guard_rows.insert(k.guard_rows.end(), row, row + NC);
                }
                // fast path: no aux terms, no guards (indices are affine in
                // the variables; the range proof above makes them exact in
                // 32-bit arithmetic)
                E.ndim = (uint32_t)ar.ndim;
                const bool fast = E.aux_kind[0] == RV_AUX_NONE && E.aux_kind[1] == RV_AUX_NONE && E.guard_count == 0;
                E.fast = fast ? 1u : 0u;
                if (fast && box > 0) {
                    // exact index range over the launch and the loop box; when
                    // every dimension stays inside [0, dim) no record of the
                    // entry can be out of bounds (fast = 2: no per-record test)
                    int64_t vlo[NC] = {0}, vhi[NC] = {0};
                    vhi[C_TX] = (int64_t)bdx - 1; vhi[C_TY] = (int64_t)bdy - 1;
                    vhi[C_BX] = (int64_t)gdx - 1; vhi[C_BY] = (int64_t)gdy - 1;
                    for (int l = 0; l < 3; l++) {
                        vlo[C_L0 + l] = E.lo[l];
                        vhi[C_L0 + l] = (int64_t)E.lo[l] + (int64_t)E.ext[l] - 1;
                    }
                    bool proven = true;
                    for (int j = 0; j < 3 && proven; j++) {
                        int64_t mn = E.row[j][C_C0], mx = E.row[j][C_C0];
                        for (int v : {C_TX, C_TY, C_BX, C_BY, C_L0, C_L1, C_L2}) {
                            const int64_t cf = E.row[j][v];
                            mn += cf >= 0 ? cf * vlo[v] : cf * vhi[v];
                            mx += cf >= 0 ? cf * vhi[v] : cf * vlo[v];
                        }
                        proven = mn >= 0 && mx < (int64_t)E.dim[j];
                    }
                    if (proven) E.fast = 2u;
                }
                if (!fast && box > 0) {
                    // floor division of a step by d, split into (q mod 2^32, r)
                    auto split = [](int64_t s, int64_t d, uint32_t *qr) {
                        int64_t q = s / d, r = s % d;
                        if (r < 0) { r += d; q -= 1; }
                        qr[0] = (uint32_t)(uint64_t)q;
                        qr[1] = (uint32_t)r;
                    };
                    const int64_t e1 = E.ext[1], e2 = E.ext[2];
                    int64_t alo[2] = {0, 0}, ahi[2] = {0, 0};
                    int64_t vlo[NC] = {0}, vhi[NC] = {0};
                    vhi[C_TX] = (int64_t)bdx - 1; vhi[C_TY] = (int64_t)bdy - 1;
                    vhi[C_BX] = (int64_t)gdx - 1; vhi[C_BY] = (int64_t)gdy - 1;
                    for (int l = 0; l < 3; l++) {
                        vlo[C_L0 + l] = E.lo[l];
                        vhi[C_L0 + l] = (int64_t)E.lo[l] + (int64_t)E.ext[l] - 1;
                    }
                    auto range = [&](const int32_t *row, int64_t &mn, int64_t &mx) {
                        mn = mx = row[C_C0];
                        for (int v = C_TX; v <= C_A1; v++) {
                            const int64_t cf = row[v];
                            mn += cf >= 0 ? cf * vlo[v] : cf * vhi[v];
                            mx += cf >= 0 ? cf * vhi[v] : cf * vlo[v];
                        }
                    };
                    for (int x = 0; x < 2; x++) {
                        if (E.aux_kind[x] == RV_AUX_NONE) continue;
                        const int64_t d = ac.aux[x].d;
                        const int32_t *r = E.row[3 + x];
                        // the numerator's change when the inner, middle or outer
                        // loop advances (the inner ones wrapping to their start)
                        const int64_t x2 = r[C_L2], x1 = (int64_t)r[C_L1] - (int64_t)r[C_L2] * (e2 - 1);
                        const int64_t x0 = (int64_t)r[C_L0] - (int64_t)r[C_L1] * (e1 - 1) - (int64_t)r[C_L2] * (e2 - 1);
                        split(x0, d, E.astep[x][0]);
                        split(x1, d, E.astep[x][1]);
                        split(x2, d, E.astep[x][2]);
                        // value range of the aux term (its numerator uses no aux variable)
                        int64_t mn, mx;
                        range(r, mn, mx);
                        auto fl = [&](int64_t n) { return n >= 0 ? n / d : -((-n + d - 1) / d); };
                        if (E.aux_kind[x] == RV_AUX_FLOORDIV) { alo[x] = fl(mn); ahi[x] = fl(mx); }
                        else { alo[x] = 0; ahi[x] = d - 1; }
                    }
                    vlo[C_A0] = alo[0]; vhi[C_A0] = ahi[0];
                    vlo[C_A1] = alo[1]; vhi[C_A1] = ahi[1];
                    bool proven = E.guard_count == 0;
                    for (int j = 0; j < 3 && proven; j++) {
                        int64_t mn, mx;
                        range(E.row[j], mn, mx);
                        proven = mn >= 0 && mx < (int64_t)E.dim[j];
                    }
                    E.gproven = proven ? 1u : 0u;
                }
                // the flattened location row, modulo 2^32: sum over dims of stride * row
                uint32_t stride = 1;
                for (int v = 0; v < NC; v++) E.fr[v] = 0;
                for (int j = ar.ndim - 1; j >= 0; j--) {
                    for (int v = 0; v < NC; v++) E.fr[v] += stride * (uint32_t)E.row[j][v];
                    stride *= (uint32_t)ar.dim[j];
                }
                E.fr[C_C0] += E.loc_base;
                // sub-key below the location: key = location << w | sub
                const uint32_t sk = subkey(dd);
                E.wshift = I.w;
                if (I.w) {
                    for (int v = 0; v < NC; v++) E.fr[v] <<= I.w;
                    E.fr[C_C0] += sk;
                    E.loc_mul <<= I.w;
                    E.loc_base = (E.loc_base << I.w) + sk;
                }
                // work items: lch loop points x gt threads per lane
                if (E.box > 0) {
                    E.lch = std::min<uint32_t>(E.box, RPL);
                    E.gt = RPL / E.lch;
                    // a shared entry of a unit-checked interval: work items of
                    // at most one unit's threads where it can, so that a unit
                    // does not expand threads of its neighbours
                    if (dcand && ar.space == RV_SHARED && Tu < (uint64_t)EXP_WG * E.gt)
                        E.gt = (uint32_t)std::max<uint64_t>(1, Tu / EXP_WG);
                    E.n_lchunks = (E.box + E.lch - 1) / E.lch;
                } else {
                    E.lch = 1; E.gt = 1; E.n_lchunks = 0;
                }
                {
                    // linear items: chunks of one thread never cross a step of
                    // an outer loop (the innermost loop's extent is a multiple
                    // of the chunk, or it is the only loop with extent > 1)
                    const uint32_t inner = E.ext[2] > 1 ? 2u : E.ext[1] > 1 ? 1u : 0u;
                    const bool only = E.box == E.ext[inner];
                    // mixed radix over the loops with points (outer to inner):
                    // then any run of consecutive points is affine too
                    bool radix = true;
                    int prev = -1;
                    for (int l = 0; l < 3; l++) {
                        if (E.ext[l] <= 1) continue;
                        if (prev >= 0) {
                            radix = radix && E.fr[C_L0 + prev] == E.fr[C_L0 + l] * E.ext[l];
                            if (E.fast != 2)
                                for (int r = 0; r < 3; r++)
                                    radix = radix && (int64_t)E.row[r][C_L0 + prev] ==
                                                         (int64_t)E.row[r][C_L0 + l] * (int64_t)E.ext[l];
                        }
                        prev = l;
                    }
                    E.linner = inner;
                    E.lflat = (only || radix) ? 1u : 0u;
                    E.lin = (E.fast != 0 && E.box > 0 && E.gt == 1 &&
                             (E.lflat || E.ext[inner] % E.lch == 0)) ? 1u : 0u;
                }
                E.mg_nl = make_magic(std::max<uint32_t>(E.n_lchunks, 1));
                E.mg_gt = make_magic(std::max<uint32_t>(E.gt, 1));
                E.mg_e1 = make_magic(std::max<uint32_t>(E.ext[1], 1));
                E.mg_e2 = make_magic(std::max<uint32_t>(E.ext[2], 1));
                {
                    // flat mapping when it needs clearly fewer items than the
                    // thread-major one (few threads: most lanes would idle)
                    const uint64_t ntg = (nthreads + E.gt - 1) / E.gt;
                    const uint64_t per = (uint64_t)EXP_WG * E.gt;
                    const uint64_t thr_items = (uint64_t)E.n_lchunks * ((nthreads + per - 1) / per);
                    const uint64_t nq = ntg * E.n_lchunks;
                    const uint64_t flat_items = (nq + EXP_WG - 1) / EXP_WG;
                    E.flat = (flat_items * 8 < thr_items * 7) ? 1u : 0u;
                    // thread-linear: one instance per thread and rows of a
                    // multiple of gt threads, so the gt consecutive threads of
                    // a lane (flat mapping) differ in tx alone and every
                    // index and the location are affine in the slot
                    E.tlin = (E.fast != 0 && E.box == 1 && bdx % E.gt == 0) ? 1u : 0u;
                    if (E.tlin) E.flat = 1;
                    E.nq = E.flat ? (uint32_t)nq : 0u;
                    E.cmaj = (E.flat && E.fast == 0) ? 1u : 0u;
                    E.ntg = (uint32_t)ntg;
                    E.mg_ntg = make_magic((uint32_t)std::max<uint64_t>(ntg, 1));
                }
                M += box;
                k.entries.push_back(E);
                k.hentries.push_back(HostEntry{dd, (uint32_t)a, kval});
            }
            if (semantics == RV_SEM_ORDERED) {
                obase += pbox * nthreads;
                if (obase >= (1ull << 32)) {
                    msg = "the sequential schedule has 2^32 or more statement instances";
                    return RV_ERR_TOO_LARGE;
                }
            }
        }
        if (semantics != RV_SEM_ORDERED)
            for (uint32_t e = I.entry_begin; e < (uint32_t)k.entries.size(); e++) k.entries[e].tmul = (uint32_t)M;
        I.entry_count = (uint32_t)k.entries.size() - I.entry_begin;
        I.M = M;
        I.P = M * nthreads;
        if (I.P >= (1ull << 32)) {
            msg = fmt("interval %lld: %lld instances (must be < 2^32)", iv, (long long)I.P);
            return RV_ERR_TOO_LARGE;
        }
        k.n_instances += I.P;
        k.max_interval_instances = std::max(k.max_interval_instances, I.P);
        // A unit expands every work item holding one of its threads; an item
        // of `per` threads at the unit's edges is expanded by each unit it
        // overlaps, so a shared entry costs about (1 + per / Tu) times its
        // records.  Units take the interval when that averages at most 2.
        // Units also need every shared entry on a fast path (no aux terms, no
        // guards): those fold runs of records; the per-record path of general
        // entries (measured on the batched and served random kernels) costs a
        // unit more than the HBM pipeline costs the same records.
        if (dcand) {
            long double recs = 0, work = 0;
            bool fast = true;
            for (uint32_t e = 0; e < I.entry_count; e++) {
                const DevEntry &E = k.entries[I.entry_begin + e];
                if (E.loc_mul == 0 || E.box == 0) continue;
                fast = fast && E.fast != 0;
                const long double per = E.flat ? std::max(1.0L, (long double)EXP_WG / E.n_lchunks) * E.gt
                                               : (long double)EXP_WG * E.gt;
                const long double w = (long double)E.box * (long double)nthreads;
                recs += w;
                work += w * (1.0L + per / (long double)Tu);
            }
            // (the unit tables keep 2 id + rw in 32 bits: ids below 2^31)
            I.direct = fast && recs > 0 && work <= 2.0L * recs && I.P < (1ull << 31);
        }
        // entry work-item prefix (and the one without the shared entries of
        // a direct interval)
        I.items_begin = (uint32_t)k.entry_items.size();
        uint64_t items = 0, items_g = 0;
        for (uint32_t e = 0; e < I.entry_count; e++) {
            DevEntry &E = k.entries[I.entry_begin + e];
            k.entry_items.push_back((uint32_t)items);
            k.entry_items_g.push_back((uint32_t)items_g);
            uint64_t ei;
            if (E.flat) {
                ei = ((uint64_t)E.nq + EXP_WG - 1) / EXP_WG;
            } else {
                uint64_t per = (uint64_t)EXP_WG * E.gt;
                uint64_t gtiles = (nthreads + per - 1) / per;
                ei = (uint64_t)E.n_lchunks * gtiles;
            }
            items += ei;
            if (!(I.direct && E.loc_mul != 0)) items_g += ei;
        }
        k.entry_items.push_back((uint32_t)items);
        k.entry_items_g.push_back((uint32_t)items_g);
        I.items_g = (uint32_t)items_g;
        if (items >= (1ull << 31)) { msg = "too many work items"; return RV_ERR_TOO_LARGE; }
        I.items = (uint32_t)items;
        // buckets: aim for `target` records per bucket on average
        if (I.P > 0 && I.K > 0) {
            long double ratio = (long double)k.target * (long double)I.K / (long double)I.P;
            int s = ratio >= 1 ? (int)std::floor(std::log2((double)ratio)) : 0;
            s = std::max((int)I.w, std::min(SMAX, s));     // a bucket holds whole locations
            I.s = (uint32_t)s;
            uint64_t span = (uint64_t)NBMAX << s;   // locations per pass
            I.nsub = (uint32_t)((I.K + span - 1) / span);
            I.nb = (uint32_t)((I.K + (1ull << s) - 1) >> s);
            for (uint32_t q = 0; q < I.nsub; q++) {
                SubPlan sp{};
                sp.interval = iv;
                sp.klo = (uint32_t)(q * span);
                sp.khi = (uint32_t)std::min<uint64_t>(I.K, (q + 1) * span);
                sp.s = (uint32_t)s;
                sp.nb = (uint32_t)(((uint64_t)sp.khi - sp.klo + (1ull << s) - 1) >> s);
                k.n_buckets += sp.nb;
                k.subs.push_back(sp);
            }
        }
    }
    return RV_OK;
}

WorkspaceLayout layout_workspace(size_t bytes) {
    const size_t reserve = 1 << 20;
    if (bytes < reserve + (size_t)TILE * 8 * 4) return WorkspaceLayout{};
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    auto place = [&](size_t R) {
        WorkspaceLayout L{};
        const size_t BC = std::max<size_t>((size_t)NBMAX, R / 256);
        const size_t H = R / HOT + 1;    // at most this many buckets exceed HOT records
        size_t off = al(R * 8 + 8);      // one record of slack: the fold's pair loads may read it
        L.off_counts = off; off = al(off + BC * 4);
        L.off_starts = off; off = al(off + BC * 4);
        L.off_cursor = off; off = al(off + BC * 4);
        L.off_conf = off; off = al(off + BC * 4);
        L.off_bsum = off; off = al(off + scan_bsum_words(BC) * 4);
        L.off_hot_n = off; off = al(off + 4);
        L.off_hot_list = off; off = al(off + H * 4);
        L.off_hot_sub = off; off = al(off + H * 4);
        L.off_hot_tab = off; off = al(off + H * 4 * TBL * 4);
        const size_t Mc = R / FOLD_CAP + 1;   // at most this many buckets exceed one fold slice
        L.off_mid_n = off; off = al(off + 4);
        L.off_mid_list = off; off = al(off + Mc * 4);
        L.off_mid_sub = off; off = al(off + Mc * 4);
        L.cap_mid = Mc;
        L.cap_records = R;
        L.cap_buckets = BC;
        L.cap_hot = H;
        L.bytes = off;
        return L;
    };
    // per record: 8 B, bucket arrays 16 B per 256 records, hot tables 8 KiB per HOT records
    const long double per = 8.0L + 16.0L / 256.0L + (16.0L * TBL + 8.0L) / (long double)HOT + 4.0L / FOLD_CAP;
    size_t R = (size_t)(((long double)(bytes - reserve)) / per);
    R = std::min<size_t>(R, (size_t)0xFFF00000u);
    WorkspaceLayout L = place(R);
    while (L.bytes > bytes) {   // shrink the record area until it fits
        const size_t over = L.bytes - bytes;
        const size_t dr = (over + 7) / 8 + 64;
        if (dr >= R) return WorkspaceLayout{};
        R -= dr;
        L = place(R);
    }
    return L;
}

rv_status plan_chunks(rv_kernel &k, const WorkspaceLayout &L, std::string &msg) {
    k.chunks.clear();
    ChunkPlan cur{0, 0, 0, 0, 0};
    for (uint32_t i = 0; i < k.subs.size(); i++) {
        const SubPlan &sp = k.subs[i];
        const IntervalPlan &I = k.intervals[sp.interval];
        if (I.P > L.cap_records || sp.nb > L.cap_buckets) {
            msg = fmt("interval %lld needs %lld records of workspace; the workspace holds %lld",
                      sp.interval, (long long)I.P, (long long)L.cap_records);
            return RV_ERR_TOO_LARGE;
        }
        if (cur.sub_end > cur.sub_begin &&
            (cur.records_bound + I.P > L.cap_records || cur.buckets + sp.nb > L.cap_buckets ||
             cur.items + I.items >= (1ull << 31))) {
            k.chunks.push_back(cur);
            cur = ChunkPlan{i, i, 0, 0, 0};
        }
        cur.sub_end = i + 1;
        cur.records_bound += I.P;
        cur.buckets += sp.nb;
        cur.items += I.items;
    }
    if (cur.sub_end > cur.sub_begin) k.chunks.push_back(cur);
    return RV_OK;
}

// The part of pass sp left to the HBM pipeline when block-local spaces are
// checked on chip: in a unit-checked interval, the locations from the end of
// the shared ones, and their buckets.  count_only: none of the entries the
// pipeline expands for the pass writes (a location without a write never
// conflicts), so the pass is counted and has no buckets.
static void hbm_part(const rv_kernel &k, const SubPlan &sp, uint32_t &klo, uint32_t &nb, uint32_t &count_only,
                     unsigned long long &static_records) {
    const IntervalPlan &I = k.intervals[sp.interval];
    const uint64_t hbm_begin = I.direct ? (uint64_t)k.kc.nblocks * I.S : 0;
    klo = sp.klo;
    nb = sp.nb;
    if (I.direct) {
        klo = (uint32_t)std::min<uint64_t>(sp.khi, std::max<uint64_t>(sp.klo, hbm_begin));
        nb = (uint32_t)(((uint64_t)sp.khi - klo + (1ull << sp.s) - 1) >> sp.s);
    }
    bool writes = false;
    uint64_t proven = 0;
    for (uint32_t e = I.entry_begin; e < I.entry_begin + I.entry_count; e++) {
        const DevEntry &E = k.entries[e];
        if (!(!I.direct || E.loc_mul == 0) || E.box == 0) continue;
        if (E.rw) writes = true;
        if (E.fast == 2 || E.gproven) proven += (uint64_t)E.box * k.kc.nthreads;
    }
    count_only = writes ? 0u : 1u;
    static_records = 0;
    if (count_only) {
        nb = 0;
        // the pass holds every location its entries can reach
        if (sp.klo <= hbm_begin && (uint64_t)sp.khi >= I.K) {
            count_only = 2;
            static_records = proven;
        }
    }
}

void plan_units(rv_kernel &k) {
    k.units.clear();
    k.max_chunk_units = 0;
    const uint32_t tpb = k.kc.tpb;
    for (ChunkPlan &ch : k.chunks) {
        ch.unit_begin = (uint32_t)k.units.size();
        ch.items_d = ch.buckets_d = 0;
        for (uint32_t i = ch.sub_begin; i < ch.sub_end; i++) {
            SubPlan &sp = k.subs[i];
            const IntervalPlan &I = k.intervals[sp.interval];
            sp.unit_begin = sp.unit_end = (uint32_t)k.units.size();
            uint32_t hlo, hnb, co;
            unsigned long long sr;
            hbm_part(k, sp, hlo, hnb, co, sr);
            ch.items_d += I.direct ? I.items_g : I.items;
            ch.buckets_d += hnb;
            if (!I.direct) continue;
            // units of nbu consecutive blocks over the pass's shared locations [klo, hlo)
            const uint64_t S = I.S;
            const uint64_t nbu = std::max<uint64_t>(1, DIR_CAP / S);
            if (sp.klo >= hlo) continue;
            const uint64_t bf = sp.klo / S, bl = (hlo - 1) / S;
            for (uint64_t b0 = bf; b0 <= bl; b0 += nbu) {
                const uint64_t b1 = std::min<uint64_t>(b0 + nbu, bl + 1);
                DevUnit U{};
                U.sub = i - ch.sub_begin;
                U.lo = (uint32_t)std::max<uint64_t>(sp.klo, b0 * S);
                U.hi = (uint32_t)std::min<uint64_t>(hlo, b1 * S);
                U.t0 = (uint32_t)(b0 * tpb);
                U.t1 = (uint32_t)(b1 * tpb);
                k.units.push_back(U);
            }
            sp.unit_end = (uint32_t)k.units.size();
        }
        ch.unit_end = (uint32_t)k.units.size();
        k.max_chunk_units = std::max(k.max_chunk_units, ch.unit_end - ch.unit_begin);
    }
}

void make_devsubs(const rv_kernel &k, uint32_t sb, uint32_t se, uint32_t res0, std::vector<DevSub> &out,
                  uint64_t &items, uint64_t &buckets, bool direct) {
    for (uint32_t i = sb; i < se; i++) {
        const SubPlan &sp = k.subs[i];
        const IntervalPlan &I = k.intervals[sp.interval];
        const bool dir = direct && I.direct;
        DevSub D{};
        D.entries = k.d_entries + I.entry_begin;
        D.guards = k.d_guards;
        D.entry_items = (dir ? k.d_entry_items_g : k.d_entry_items) + I.items_begin;
        D.kc = k.d_kc;
        D.n_entries = I.entry_count;
        D.item_begin = (uint32_t)items;
        D.bucket_begin = (uint32_t)buckets;
        D.nb = sp.nb;
        D.s = sp.s;
        D.klo = sp.klo;
        D.khi = sp.khi;
        if (direct) hbm_part(k, sp, D.klo, D.nb, D.count_only, D.static_records);
        D.M = (uint32_t)I.M;
        D.mgM = make_magic((uint32_t)I.M);
        D.interval = sp.interval;
        D.res = res0 + (i - sb);
        D.wshift = I.w;
        D.upb = I.upb ? I.upb : 1u;
        D.mg_unit = make_magic(I.unit ? I.unit : 1u);
        items += dir ? I.items_g : I.items;
        buckets += D.nb;
        out.push_back(D);
    }
}

void decode_instance(const rv_kernel &k, uint32_t interval, uint32_t id, rv_side &side, uint32_t &gthread,
                     uint32_t &lidx) {
    const IntervalPlan &I = k.intervals[interval];
    gthread = (uint32_t)(id / I.M);
    uint32_t r = (uint32_t)(id % I.M);
    // entries are in increasing offset order
    uint32_t lo = I.entry_begin, hi = I.entry_begin + I.entry_count;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) / 2;
        if (k.entries[mid].off <= r) lo = mid; else hi = mid;
    }
    while (lo + 1 < I.entry_begin + I.entry_count && k.entries[lo].box == 0) lo++;
    const DevEntry &E = k.entries[lo];
    lidx = r - E.off;
    side.block = gthread / k.kc.tpb;
    side.tid = gthread % k.kc.tpb;
    side.dyn_phase = k.hentries[lo].dphase;
    side.access = k.hentries[lo].access;
    uint32_t rem = lidx;
    int32_t lv[3] = {0, 0, 0};
    for (int l = (int)E.nloops - 1; l >= 0; l--) {
        lv[l] = E.lo[l] + (int32_t)(rem % E.ext[l]);
        rem /= E.ext[l];
    }
    side.loop[0] = lv[0]; side.loop[1] = lv[1]; side.loop[2] = lv[2];
    side.is_write = (int32_t)E.rw;
}

void decode_location(const rv_kernel &k, uint32_t interval, uint32_t loc, int32_t &space, int32_t &array,
                     uint32_t &block, int64_t &address) {
    const IntervalPlan &I = k.intervals[interval];
    loc >>= I.w;                      // the sub-key below the location
    uint64_t shared_end = (uint64_t)k.kc.nblocks * I.S;
    uint64_t rem;
    if (loc < shared_end) {
        space = RV_SHARED;
        block = (uint32_t)(loc / I.S);
        rem = loc % I.S;
    } else {
        space = RV_GLOBAL;
        block = 0;
        rem = loc - shared_end;
    }
    array = -1;
    address = 0;
    for (size_t a = 0; a < k.arrays.size(); a++) {
        if (I.arr_off[a] < 0 || k.arrays[a].space != space) continue;
        uint64_t off = (uint64_t)I.arr_off[a], n = arr_size(k.arrays[a]);
        if (rem >= off && rem < off + n) { array = (int32_t)a; address = (int64_t)(rem - off); break; }
    }
}

}  // namespace rv
