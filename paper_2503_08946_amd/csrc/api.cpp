// C ABI of librv (declared in include/rv.h).  Host orchestration only: every
// step of the check runs in the gfx950 kernels of kernels.hip.

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <random>

#include "rv_internal.h"

using namespace rv;

struct rv_ctx {
    int device = 0;
    unsigned ncu = 256;             // compute units of the device (persistent grids)
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    WorkspaceLayout L;
    std::string err;
    // context-owned device buffers (grown on demand)
    SubResult *d_res = nullptr;
    size_t res_cap = 0;
    DevSub *d_bsubs = nullptr;
    size_t bsubs_cap = 0;
    void *h_pin = nullptr;
    size_t pin_cap = 0;
    // timing
    bool timing = false;
    struct Ev { int stage; hipEvent_t a, b; };
    std::vector<Ev> pending;
    std::vector<hipEvent_t> pool;
    rv_timing acc{};

    unsigned long long *rec() { return reinterpret_cast<unsigned long long *>(ws); }
    uint32_t *counts() { return reinterpret_cast<uint32_t *>(ws + L.off_counts); }
    uint32_t *starts() { return reinterpret_cast<uint32_t *>(ws + L.off_starts); }
    uint32_t *cursor() { return reinterpret_cast<uint32_t *>(ws + L.off_cursor); }
    uint32_t *conf() { return reinterpret_cast<uint32_t *>(ws + L.off_conf); }
    uint32_t *bsum() { return reinterpret_cast<uint32_t *>(ws + L.off_bsum); }
};

namespace {

rv_status fail(rv_ctx *c, rv_status st, const std::string &m) {
    if (c) c->err = m;
    return st;
}

#define HIP_TRY(c, call)                                                                      \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail((c), RV_ERR_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

hipEvent_t get_event(rv_ctx *c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

template <class F>
void timed(rv_ctx *c, int stage, F &&f) {
    if (!c->timing) { f(); return; }
    hipEvent_t a = get_event(c), b = get_event(c);
    if (!a || !b) { f(); return; }
    (void)hipEventRecord(a, c->stream);
    f();
    (void)hipEventRecord(b, c->stream);
    c->pending.push_back({stage, a, b});
}

rv_status drain_timing(rv_ctx *c) {
    for (auto &e : c->pending) {
        HIP_TRY(c, hipEventSynchronize(e.b));
        float ms = 0;
        HIP_TRY(c, hipEventElapsedTime(&ms, e.a, e.b));
        c->acc.ms[e.stage] += ms;
        c->acc.launches[e.stage] += 1;
        c->pool.push_back(e.a);
        c->pool.push_back(e.b);
    }
    c->pending.clear();
    return RV_OK;
}

rv_status ensure_res(rv_ctx *c, size_t n) {
    if (n <= c->res_cap) return RV_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->d_res) HIP_TRY(c, hipFree(c->d_res));
    c->d_res = nullptr;
    size_t cap = std::max<size_t>(n, 2 * c->res_cap);
    HIP_TRY(c, hipMalloc(&c->d_res, cap * sizeof(SubResult)));
    c->res_cap = cap;
    return RV_OK;
}

rv_status ensure_bsubs(rv_ctx *c, size_t n) {
    if (n <= c->bsubs_cap) return RV_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->d_bsubs) HIP_TRY(c, hipFree(c->d_bsubs));
    c->d_bsubs = nullptr;
    size_t cap = std::max<size_t>(n, 2 * c->bsubs_cap);
    HIP_TRY(c, hipMalloc(&c->d_bsubs, cap * sizeof(DevSub)));
    c->bsubs_cap = cap;
    return RV_OK;
}

rv_status ensure_pin(rv_ctx *c, size_t bytes) {
    if (bytes <= c->pin_cap) return RV_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->h_pin) HIP_TRY(c, hipHostFree(c->h_pin));
    c->h_pin = nullptr;
    size_t cap = std::max<size_t>(bytes, 2 * c->pin_cap);
    HIP_TRY(c, hipHostMalloc(&c->h_pin, cap, hipHostMallocDefault));
    c->pin_cap = cap;
    return RV_OK;
}

rv_status check_launch(rv_ctx *c) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, RV_ERR_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return RV_OK;
}

// count -> scan -> expansion for one chunk
void run_expand(rv_ctx *c, const DevSub *subs, uint32_t nsub, uint64_t items, uint64_t buckets) {
    timed(c, RV_STAGE_FILL, [&] { launch_fill_u32(c->counts(), buckets, 0u, c->stream); });
    timed(c, RV_STAGE_COUNT, [&] { launch_hist(subs, nsub, items, c->counts(), c->d_res, c->ncu, c->stream); });
    timed(c, RV_STAGE_SCAN, [&] { launch_scan(c->counts(), c->starts(), c->cursor(), c->bsum(), buckets, c->stream); });
    timed(c, RV_STAGE_EXPAND, [&] { launch_scatter(subs, nsub, items, c->rec(), c->cursor(), c->ncu, c->stream); });
}

void run_check_chunk(rv_ctx *c, const DevSub *subs, uint32_t nsub, uint64_t items, uint64_t buckets) {
    run_expand(c, subs, nsub, items, buckets);
    timed(c, RV_STAGE_SORT_SCAN, [&] {
        launch_bucket(subs, nsub, buckets, c->rec(), c->starts(), c->counts(), c->conf(), 0, c->ncu, c->stream);
    });
    timed(c, RV_STAGE_FINISH, [&] {
        launch_finish(subs, nsub, buckets, c->conf(), c->d_res, c->stream);
        launch_first(subs, nsub, c->rec(), c->starts(), c->d_res, c->stream);
    });
}

void decode_witness(const rv_kernel &k, uint32_t interval, const uint32_t w[4], rv_witness &out) {
    memset(&out, 0, sizeof out);
    out.interval = interval;
    decode_location(k, interval, w[0], out.space, out.array, out.block, out.address);
    uint32_t g, l;
    decode_instance(k, interval, w[1], out.first, g, l);
    decode_instance(k, interval, w[2], out.second, g, l);
}

// Per-kernel result from its passes' slots hr[0 .. k.subs.size()).
rv_status assemble(rv_ctx *c, const rv_kernel &k, const SubResult *hr, rv_result *out) {
    rv_result r;
    memset(&r, 0, sizeof r);
    unsigned long long oob = ~0ull;
    for (size_t i = 0; i < k.subs.size(); i++) {
        r.n_records += hr[i].records;
        r.n_conflicts += hr[i].conflicts;
        oob = std::min(oob, hr[i].oob);
    }
    if (oob != ~0ull) {
        uint32_t iv = (uint32_t)(oob >> 32), id = (uint32_t)oob;
        rv_side s;
        uint32_t g, l;
        decode_instance(k, iv, id, s, g, l);
        char buf[256];
        snprintf(buf, sizeof buf,
                 "index out of bounds: interval %u, block %u, thread %u, dynamic phase %u, access %u, loop (%d,%d,%d)",
                 iv, s.block, s.tid, s.dyn_phase, s.access, s.loop[0], s.loop[1], s.loop[2]);
        return fail(c, RV_ERR_OOB, buf);
    }
    for (size_t i = 0; i < k.subs.size(); i++) {
        if (hr[i].conflicts) {
            decode_witness(k, k.subs[i].interval, hr[i].w, r.witness);
            r.has_witness = 1;
            break;
        }
    }
    *out = r;
    return RV_OK;
}

}  // namespace

// ===================================================================== API
extern "C" {

rv_status rv_validate_desc(const rv_kernel_desc *desc, char *msg, size_t cap) {
    std::string m;
    rv_status st;
    try {
        rv_kernel k;
        st = plan_kernel(desc, DEFAULT_TARGET, k, m);
    } catch (const std::bad_alloc &) {
        st = RV_ERR_TOO_LARGE;
        m = "out of host memory";
    }
    if (msg && cap) {
        strncpy(msg, st ? m.c_str() : "", cap - 1);
        msg[cap - 1] = 0;
    }
    return st;
}

rv_status rv_ctx_create(rv_ctx **out, int device, void *hip_stream, void *workspace, size_t workspace_bytes) {
    if (!out || !workspace) return RV_ERR_INVALID;
    if (workspace_bytes < (64u << 20)) return RV_ERR_TOO_LARGE;
    rv_ctx *c = new (std::nothrow) rv_ctx;
    if (!c) return RV_ERR_TOO_LARGE;
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->ws = reinterpret_cast<char *>(workspace);
    c->ws_bytes = workspace_bytes;
    c->L = layout_workspace(workspace_bytes);
    if (!c->L.cap_records) { delete c; return RV_ERR_TOO_LARGE; }
    if (hipSetDevice(device) != hipSuccess) { delete c; return RV_ERR_DEVICE; }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        c->ncu = (unsigned)ncu;
    *out = c;
    return RV_OK;
}

rv_status rv_ctx_destroy(rv_ctx *c) {
    if (!c) return RV_ERR_INVALID;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto &e : c->pending) { c->pool.push_back(e.a); c->pool.push_back(e.b); }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    if (c->d_res) (void)hipFree(c->d_res);
    if (c->d_bsubs) (void)hipFree(c->d_bsubs);
    if (c->h_pin) (void)hipHostFree(c->h_pin);
    delete c;
    return RV_OK;
}

const char *rv_last_error(const rv_ctx *c) { return c ? c->err.c_str() : "null context"; }

rv_status rv_load_kernel_desc(rv_ctx *c, const rv_kernel_desc *desc, rv_kernel **out) {
    if (!c || !out) return RV_ERR_INVALID;
    c->err.clear();
    rv_kernel *k = new (std::nothrow) rv_kernel;
    if (!k) return fail(c, RV_ERR_TOO_LARGE, "out of host memory");
    std::string m;
    rv_status st;
    try {
        st = plan_kernel(desc, DEFAULT_TARGET, *k, m);
        if (!st) st = plan_chunks(*k, c->L, m);
    } catch (const std::bad_alloc &) {
        st = RV_ERR_TOO_LARGE;
        m = "out of host memory";
    }
    if (st) { delete k; return fail(c, st, m); }
    HIP_TRY(c, hipSetDevice(c->device));
    // one device block: kernel constants, entries, guard rows, entry prefixes, passes
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_kc = 0;
    const size_t o_en = al(o_kc + sizeof(DevKernel));
    const size_t o_gr = al(o_en + k->entries.size() * sizeof(DevEntry));
    const size_t o_ei = al(o_gr + k->guard_rows.size() * sizeof(int32_t));
    const size_t o_sb = al(o_ei + k->entry_items.size() * sizeof(uint32_t));
    const size_t total = al(o_sb + k->subs.size() * sizeof(DevSub) + 1);
    hipError_t e = hipMalloc(&k->d_mem, total);
    if (e != hipSuccess) { delete k; return fail(c, RV_ERR_DEVICE, std::string("hipMalloc: ") + hipGetErrorString(e)); }
    char *base = reinterpret_cast<char *>(k->d_mem);
    k->d_kc = reinterpret_cast<DevKernel *>(base + o_kc);
    k->d_entries = reinterpret_cast<DevEntry *>(base + o_en);
    k->d_guards = reinterpret_cast<int32_t *>(base + o_gr);
    k->d_entry_items = reinterpret_cast<uint32_t *>(base + o_ei);
    k->d_subs = reinterpret_cast<DevSub *>(base + o_sb);
    k->h_subs.clear();
    for (auto &ch : k->chunks) {
        uint64_t items = 0, buckets = 0;
        make_devsubs(*k, ch.sub_begin, ch.sub_end, ch.sub_begin, k->h_subs, items, buckets);
    }
    std::vector<char> host(total, 0);
    memcpy(host.data() + o_kc, &k->kc, sizeof(DevKernel));
    if (!k->entries.empty()) memcpy(host.data() + o_en, k->entries.data(), k->entries.size() * sizeof(DevEntry));
    if (!k->guard_rows.empty()) memcpy(host.data() + o_gr, k->guard_rows.data(), k->guard_rows.size() * 4);
    if (!k->entry_items.empty()) memcpy(host.data() + o_ei, k->entry_items.data(), k->entry_items.size() * 4);
    if (!k->h_subs.empty()) memcpy(host.data() + o_sb, k->h_subs.data(), k->h_subs.size() * sizeof(DevSub));
    e = hipMemcpy(k->d_mem, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(k->d_mem);
        delete k;
        return fail(c, RV_ERR_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    k->owner = c;
    *out = k;
    return RV_OK;
}

rv_status rv_free_kernel(rv_ctx *c, rv_kernel *k) {
    if (!c || !k) return RV_ERR_INVALID;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (k->d_mem) (void)hipFree(k->d_mem);
    delete k;
    return RV_OK;
}

rv_status rv_kernel_get_info(rv_ctx *c, const rv_kernel *k, rv_kernel_info *out) {
    if (!c || !k || !out) return RV_ERR_INVALID;
    out->n_instances = k->n_instances;
    out->n_intervals = k->n_intervals;
    out->n_subintervals = (uint32_t)k->subs.size();
    out->n_chunks = (uint32_t)k->chunks.size();
    out->n_buckets = (uint32_t)k->n_buckets;
    out->max_interval_instances = k->max_interval_instances;
    return RV_OK;
}

rv_status rv_check(rv_ctx *c, rv_kernel *k, rv_result *out) {
    if (!c || !k || !out) return RV_ERR_INVALID;
    if (k->owner != c) return fail(c, RV_ERR_STATE, "kernel was loaded on another context");
    c->err.clear();
    HIP_TRY(c, hipSetDevice(c->device));
    const size_t ns = k->subs.size();
    rv_status st = ensure_res(c, std::max<size_t>(ns, 1));
    if (st) return st;
    st = ensure_pin(c, std::max<size_t>(ns, 1) * sizeof(SubResult));
    if (st) return st;
    timed(c, RV_STAGE_FILL, [&] { launch_init_results(c->d_res, ns, c->stream); });
    for (auto &ch : k->chunks)
        run_check_chunk(c, k->d_subs + ch.sub_begin, ch.sub_end - ch.sub_begin, ch.items, ch.buckets);
    if ((st = check_launch(c))) return st;
    if (ns) HIP_TRY(c, hipMemcpyAsync(c->h_pin, c->d_res, ns * sizeof(SubResult), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return assemble(c, *k, reinterpret_cast<SubResult *>(c->h_pin), out);
}

rv_status rv_check_batch(rv_ctx *c, rv_kernel *const *ks, size_t n, rv_result *out) {
    if (!c || (n && (!ks || !out))) return RV_ERR_INVALID;
    c->err.clear();
    if (!n) return RV_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    std::vector<size_t> res0(n + 1, 0);
    for (size_t j = 0; j < n; j++) {
        if (!ks[j]) return fail(c, RV_ERR_INVALID, "null kernel in batch");
        if (ks[j]->owner != c) return fail(c, RV_ERR_STATE, "kernel was loaded on another context");
        res0[j + 1] = res0[j] + ks[j]->subs.size();
    }
    const size_t ns = res0[n];
    // chunks across kernels: passes in (kernel, pass) order, greedy by capacity
    struct Chunk { size_t sub_begin, sub_end; uint64_t items, buckets; };
    std::vector<Chunk> chunks;
    std::vector<DevSub> table;
    table.reserve(ns);
    Chunk cur{0, 0, 0, 0};
    uint64_t rec_bound = 0;
    for (size_t j = 0; j < n; j++) {
        const rv_kernel &k = *ks[j];
        for (uint32_t i = 0; i < k.subs.size(); i++) {
            const IntervalPlan &I = k.intervals[k.subs[i].interval];
            const uint32_t nb = k.subs[i].nb;
            if (cur.sub_end > cur.sub_begin &&
                (rec_bound + I.P > c->L.cap_records || cur.buckets + nb > c->L.cap_buckets ||
                 cur.items + I.items >= (1ull << 31))) {
                chunks.push_back(cur);
                cur = Chunk{table.size(), table.size(), 0, 0};
                rec_bound = 0;
            }
            make_devsubs(k, i, i + 1, (uint32_t)(res0[j] + i), table, cur.items, cur.buckets);
            cur.sub_end = table.size();
            rec_bound += I.P;
        }
    }
    if (cur.sub_end > cur.sub_begin) chunks.push_back(cur);
    rv_status st = ensure_res(c, std::max<size_t>(ns, 1));
    if (st) return st;
    st = ensure_bsubs(c, std::max<size_t>(table.size(), 1));
    if (st) return st;
    const size_t pin_bytes = std::max(table.size() * sizeof(DevSub), ns * sizeof(SubResult));
    st = ensure_pin(c, std::max<size_t>(pin_bytes, 64));
    if (st) return st;
    if (!table.empty()) {
        memcpy(c->h_pin, table.data(), table.size() * sizeof(DevSub));
        HIP_TRY(c, hipMemcpyAsync(c->d_bsubs, c->h_pin, table.size() * sizeof(DevSub), hipMemcpyHostToDevice,
                                  c->stream));
    }
    timed(c, RV_STAGE_FILL, [&] { launch_init_results(c->d_res, ns, c->stream); });
    for (auto &ch : chunks)
        run_check_chunk(c, c->d_bsubs + ch.sub_begin, (uint32_t)(ch.sub_end - ch.sub_begin), ch.items, ch.buckets);
    if ((st = check_launch(c))) return st;
    // the pinned buffer is reused for results once the upload has completed (stream order)
    if (ns) HIP_TRY(c, hipMemcpyAsync(c->h_pin, c->d_res, ns * sizeof(SubResult), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const SubResult *hr = reinterpret_cast<const SubResult *>(c->h_pin);
    for (size_t j = 0; j < n; j++) {
        st = assemble(c, *ks[j], hr + res0[j], &out[j]);
        if (st) {
            c->err = "kernel " + std::to_string(j) + ": " + c->err;
            return st;
        }
    }
    return RV_OK;
}

rv_status rv_get_witnesses(rv_ctx *c, rv_kernel *k, uint64_t first_index, rv_witness *out, size_t cap,
                           size_t *n_out) {
    if (!c || !k || !n_out || (cap && !out)) return RV_ERR_INVALID;
    if (k->owner != c) return fail(c, RV_ERR_STATE, "kernel was loaded on another context");
    c->err.clear();
    *n_out = 0;
    HIP_TRY(c, hipSetDevice(c->device));
    const size_t ns = k->subs.size();
    rv_status st = ensure_res(c, std::max<size_t>(ns, 1));
    if (st) return st;
    st = ensure_pin(c, std::max<size_t>(std::max<size_t>(cap, 1) * sizeof(DevWitness), ns * sizeof(SubResult)));
    if (st) return st;
    DevWitness *d_win = nullptr;
    if (cap) HIP_TRY(c, hipMalloc(&d_win, cap * sizeof(DevWitness)));
    const unsigned long long lo = first_index, hi = first_index + cap;
    unsigned long long base = 0;
    launch_init_results(c->d_res, ns, c->stream);
    for (auto &ch : k->chunks) {
        const DevSub *subs = k->d_subs + ch.sub_begin;
        const uint32_t nsub = ch.sub_end - ch.sub_begin;
        run_expand(c, subs, nsub, ch.items, ch.buckets);
        launch_bucket(subs, nsub, ch.buckets, c->rec(), c->starts(), c->counts(), c->conf(), 0, c->ncu, c->stream);
        launch_finish(subs, nsub, ch.buckets, c->conf(), c->d_res, c->stream);
        // exclusive scan of per-bucket conflict counts -> list positions (cursor area)
        launch_scan(c->conf(), c->cursor(), nullptr, c->bsum(), ch.buckets, c->stream);
        const size_t nbk = (ch.buckets + 4095) / 4096;
        uint32_t total = 0;
        hipError_t e = hipMemcpyAsync(&total, c->bsum() + nbk, 4, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            if (d_win) (void)hipFree(d_win);
            return fail(c, RV_ERR_DEVICE, std::string("witness collect: ") + hipGetErrorString(e));
        }
        if (cap && base < hi && base + total > lo)
            launch_gather(subs, nsub, ch.buckets, c->rec(), c->starts(), c->conf(), c->cursor(), base, lo, hi, d_win,
                          c->stream);
        base += total;
    }
    if ((st = check_launch(c))) { if (d_win) (void)hipFree(d_win); return st; }
    // OOB check through the pass results
    hipError_t e = hipMemcpyAsync(c->h_pin, c->d_res, ns * sizeof(SubResult), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        if (d_win) (void)hipFree(d_win);
        return fail(c, RV_ERR_DEVICE, std::string("witness collect: ") + hipGetErrorString(e));
    }
    rv_result tmp;
    st = assemble(c, *k, reinterpret_cast<const SubResult *>(c->h_pin), &tmp);
    if (st) { if (d_win) (void)hipFree(d_win); return st; }
    const size_t got = base > lo ? (size_t)std::min<unsigned long long>(cap, base - lo) : 0;
    if (got) {
        std::vector<DevWitness> hw(got);
        e = hipMemcpy(hw.data(), d_win, got * sizeof(DevWitness), hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            (void)hipFree(d_win);
            return fail(c, RV_ERR_DEVICE, std::string("witness copy: ") + hipGetErrorString(e));
        }
        for (size_t i = 0; i < got; i++) decode_witness(*k, k->subs[hw[i].sub].interval, hw[i].w, out[i]);
    }
    if (d_win) (void)hipFree(d_win);
    *n_out = got;
    return RV_OK;
}

rv_status rv_debug_records(rv_ctx *c, rv_kernel *k, uint32_t interval, int sorted, rv_record *out, size_t cap,
                           size_t *n_out) {
    if (!c || !k || !n_out || (cap && !out)) return RV_ERR_INVALID;
    if (k->owner != c) return fail(c, RV_ERR_STATE, "kernel was loaded on another context");
    c->err.clear();
    *n_out = 0;
    if (interval >= k->n_intervals) return fail(c, RV_ERR_INVALID, "no such interval");
    HIP_TRY(c, hipSetDevice(c->device));
    uint32_t sb = 0;
    while (sb < k->subs.size() && k->subs[sb].interval < interval) sb++;
    uint32_t se = sb;
    while (se < k->subs.size() && k->subs[se].interval == interval) se++;
    if (se == sb) return RV_OK;
    std::vector<DevSub> table;
    uint64_t items = 0, buckets = 0;
    make_devsubs(*k, sb, se, 0, table, items, buckets);
    const IntervalPlan &I = k->intervals[interval];
    if ((se - sb) * I.P > c->L.cap_records || buckets > c->L.cap_buckets)
        return fail(c, RV_ERR_TOO_LARGE, "interval does not fit the workspace");
    rv_status st = ensure_res(c, se - sb);
    if (st) return st;
    st = ensure_bsubs(c, table.size());
    if (st) return st;
    HIP_TRY(c, hipMemcpy(c->d_bsubs, table.data(), table.size() * sizeof(DevSub), hipMemcpyHostToDevice));
    launch_init_results(c->d_res, se - sb, c->stream);
    run_expand(c, c->d_bsubs, se - sb, items, buckets);
    if ((st = check_launch(c))) return st;
    std::vector<uint32_t> cnt(buckets);
    HIP_TRY(c, hipMemcpyAsync(cnt.data(), c->counts(), buckets * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    uint64_t total = 0;
    for (uint32_t x : cnt) {
        total += x;
        if (sorted && x > (uint32_t)CAP) return fail(c, RV_ERR_UNSUPPORTED, "a bucket exceeds one on-chip slice");
    }
    if (sorted) {
        launch_bucket(c->d_bsubs, se - sb, buckets, c->rec(), c->starts(), c->counts(), c->conf(), 1, c->ncu, c->stream);
        if ((st = check_launch(c))) return st;
    }
    std::vector<unsigned long long> recs(total);
    if (total)
        HIP_TRY(c, hipMemcpyAsync(recs.data(), c->rec(), total * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const size_t m = std::min<size_t>(cap, total);
    for (size_t i = 0; i < m; i++) {
        const uint32_t hiw = (uint32_t)(recs[i] >> 32), id = (uint32_t)recs[i];
        rv_record &o = out[i];
        memset(&o, 0, sizeof o);
        o.interval = interval;
        decode_location(*k, interval, hiw >> 1, o.space, o.array, o.block, o.address);
        rv_side s;
        decode_instance(*k, interval, id, s, o.gthread, o.lidx);
        o.dyn_phase = s.dyn_phase;
        o.access = s.access;
        o.loop[0] = s.loop[0]; o.loop[1] = s.loop[1]; o.loop[2] = s.loop[2];
        o.is_write = (int32_t)(hiw & 1u);
    }
    *n_out = total;
    return RV_OK;
}

rv_status rv_set_timing(rv_ctx *c, int enable) {
    if (!c) return RV_ERR_INVALID;
    c->timing = enable != 0;
    return RV_OK;
}

rv_status rv_get_timing(rv_ctx *c, rv_timing *out, int reset) {
    if (!c || !out) return RV_ERR_INVALID;
    rv_status st = drain_timing(c);
    if (st) return st;
    *out = c->acc;
    if (reset) memset(&c->acc, 0, sizeof c->acc);
    return RV_OK;
}

rv_status rv_selftest(char *msg, size_t cap) {
    std::string m;
    auto check_div = [&](uint32_t d, uint32_t n) -> bool {
        Magic g = make_magic(d);
        if (udiv(n, g) != n / d) {
            m = "udiv " + std::to_string(n) + "/" + std::to_string(d);
            return false;
        }
        int32_t sn = (int32_t)n;
        int64_t q = (int64_t)sn / (int64_t)d;
        if ((int64_t)sn % (int64_t)d != 0 && sn < 0) q -= 1;
        if (fdiv(sn, g) != q) { m = "fdiv " + std::to_string(sn) + "/" + std::to_string(d); return false; }
        int64_t r = (int64_t)sn - q * (int64_t)d;
        if (emod(sn, g) != r || r < 0 || r >= (int64_t)d) { m = "emod " + std::to_string(sn); return false; }
        return true;
    };
    std::mt19937_64 rng(12345);
    bool ok = true;
    for (uint32_t d = 1; d <= 4096 && ok; d++)
        for (uint32_t n : {0u, 1u, 2u, d - 1, d, d + 1, 2 * d - 1, 2 * d, 0x7FFFFFFFu, 0x80000000u, 0xFFFFFFFFu,
                           0xFFFFFFFEu, (uint32_t)-(int32_t)d, (uint32_t)(-(int32_t)d - 1)})
            if (!(ok = check_div(d, n))) break;
    for (int i = 0; i < 2000000 && ok; i++) {
        uint32_t d = (uint32_t)(rng() % 0x7FFFFFFFu) + 1;
        if (i & 1) d = (uint32_t)(rng() % 70000) + 1;
        uint32_t n = (uint32_t)rng();
        ok = check_div(d, n);
    }
    for (uint32_t d : {3u, 7u, 641u, 1000u, 65537u, 0x7FFFFFFFu, 0x40000000u})
        for (uint64_t n = 0; n < (1ull << 32) && ok; n += 9973) ok = check_div(d, (uint32_t)n);
    if (msg && cap) {
        strncpy(msg, ok ? "" : m.c_str(), cap - 1);
        msg[cap - 1] = 0;
    }
    return ok ? RV_OK : RV_ERR_STATE;
}

}  // extern "C"
