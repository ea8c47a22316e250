"""GPU parity: the HIP checker against the CPU oracle, bit-exact.

Every test runs librv through its C ABI (the ctypes binding) on cuda:0 and
compares counts, records and canonical witnesses with ``oracle`` on the same
seeded descriptions."""

import sys

import numpy as np
import pytest

import oracle
from cases import large_grid, linear_case
from workloads import kernels as K
from workloads import random_affine as RA
from workloads.desc import AUX_EMOD, AUX_FLOORDIV, GLOBAL, SHARED, Aux, Builder, aff, rw

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=["fold", "sort_scan"])
def ctx(request):
    # every parity case runs with both per-bucket grouping kernels
    import paper_2503_08946_amd as rv
    c = rv.Context(0, workspace_bytes=1 << 30)
    c.group = request.param
    yield c
    c.close()


def _wkey(w):
    return (w.interval, w.space, w.block, w.array, w.address,
            (w.first.block, w.first.tid, w.first.dphase, w.first.access, tuple(w.first.loop), w.first.is_write),
            (w.second.block, w.second.tid, w.second.dphase, w.second.access, tuple(w.second.loop),
             w.second.is_write))


def compare(ctx, desc, max_list=1 << 16, list_all=True):
    say(f"[parity] {desc.name} instances={desc.instances_upper_bound()}")
    o = oracle.check(desc, max_witnesses=max_list)
    assert o.status == 0
    k = ctx.load(desc)
    g = ctx.check(k)
    assert g.n_records == o.n_records
    assert g.n_conflicts == o.n_conflicts
    if o.n_conflicts:
        assert g.witness is not None
        assert _wkey(g.witness) == _wkey(o.witnesses[0])
    else:
        assert g.witness is None
    if list_all and o.n_conflicts:
        n = min(o.n_conflicts, max_list)
        ws = ctx.witnesses(k, 0, n)
        assert [_wkey(w) for w in ws] == [_wkey(w) for w in o.witnesses[:n]]
    return k, g, o


# ----------------------------------------------------------------- pins
@pytest.mark.parametrize("name", ["tiny_fixed", "polynomial_product", "stride1_shared", "stride1_global",
                                  "half_index_shared", "half_index_global", "gespmm_crc"])
def test_pin_kernels(ctx, name):
    compare(ctx, getattr(K, name)())


@pytest.mark.parametrize("mid,trail", [(True, True), (False, True), (True, False), (False, False)])
def test_gespmm_variants(ctx, mid, trail):
    compare(ctx, K.gespmm_crc(M=8, N=96, T=4, K=3, middle_barrier=mid, trailing_barrier=trail))


def test_tiny_random(ctx):
    for d in K.tiny_random(seed=1, count=32):
        compare(ctx, d)


@pytest.mark.parametrize("k", [-1] + list(range(10)))
def test_tree_reduction_full_size(ctx, k):
    _, g, o = compare(ctx, K.tree_reduction(k))
    assert g.n_records == 392832
    assert g.n_conflicts == (128 * (256 >> k) if 0 <= k <= 8 else 0)


@pytest.mark.parametrize("d", [-1, 0, 1, 6, 7])
def test_matmul_small(ctx, d):
    compare(ctx, K.tiled_matmul(grid=2, k_iters=4, drop_dynamic=d))


@pytest.mark.parametrize("s", ["load", "compute"])
def test_matmul_static(ctx, s):
    compare(ctx, K.tiled_matmul(grid=3, k_iters=3, drop_static=s))


# ------------------------------------------------------ expansion / sort
@pytest.mark.parametrize("desc", [K.tiny_fixed(), K.tree_reduction(2, block=256, grid=6),
                                  K.tiled_matmul(grid=2, k_iters=2, drop_dynamic=1),
                                  K.gespmm_crc(), K.polynomial_product(48)], ids=lambda d: d.name)
def test_expansion_record_multiset(ctx, desc):
    k = ctx.load(desc)
    for iv in range(oracle.n_intervals(desc)):
        say(f"[expand] {desc.name} interval {iv}")
        ref = oracle.records(desc, iv)
        got = ctx.debug_records(k, iv, sorted=False)
        # (interval, space, block, array, address, gthread, dphase, access, lidx, loops, rw)
        a = ref[np.lexsort(ref.T[::-1])]
        b = got[np.lexsort(got.T[::-1])]
        assert a.shape == b.shape
        assert np.array_equal(a, b)


def test_expansion_flat_mapping(ctx):
    # kernels with a few threads and long loops: their entries spread loop
    # chunks across the lanes of a work item
    descs = [d for d in RA.batch_kernels(seed=4, count=64)
             if d.instances_upper_bound() < 3_000_000][:12]
    b = Builder((3, 1), (1, 1), "three-threads")
    s = b.array(SHARED, (64, 64))
    g = b.array(GLOBAL, (4096,))
    p = b.phase([rw(s, True, aff(l0=1), aff(tx=1, l1=1), loops=((0, 64), (0, 61))),
                 rw(g, False, aff(tx=1000, l0=1), loops=((0, 37),)),
                 rw(g, True, aff(l0=3, tx=1), loops=((5, 9),)),
                 rw(s, False, aff(tx=1), aff(l0=1), loops=((0, 64),), guards=(aff(40, l0=-1),))], False)
    b.segment([p])
    descs.append(b.build())
    n_flat = 0
    for desc in descs:
        k = ctx.load(desc)
        n_flat += k.info().n_flat_entries
        for iv in range(oracle.n_intervals(desc)):
            say(f"[expand-flat] {desc.name} interval {iv}")
            ref = oracle.records(desc, iv)
            got = ctx.debug_records(k, iv, sorted=False)
            a = ref[np.lexsort(ref.T[::-1])]
            b2 = got[np.lexsort(got.T[::-1])]
            assert np.array_equal(a, b2)
        compare(ctx, desc, list_all=False)
    assert n_flat > 0


@pytest.mark.parametrize("desc", [K.tiny_fixed(), K.tree_reduction(4, block=512, grid=3),
                                  K.tiled_matmul(grid=2, k_iters=2), K.half_index_global(block=256, grid=8),
                                  K.polynomial_product(64)],
                         ids=lambda d: d.name)
def test_sort_output_is_sorted_permutation(ctx, desc):
    k = ctx.load(desc)
    for iv in range(oracle.n_intervals(desc)):
        say(f"[sort] {desc.name} interval {iv}")
        got = ctx.debug_records(k, iv, sorted=True)
        ref = oracle.records(desc, iv)
        loc = got[:, 1:5]
        # location order: (space, block, array, address) non-decreasing
        lk = [tuple(r) for r in loc]
        assert lk == sorted(lk)
        a = ref[np.lexsort(ref.T[::-1])]
        b = got[np.lexsort(got.T[::-1])]
        assert np.array_equal(a, b)


# ------------------------------------------------- linear work items
def _records_equal(ctx, k, desc):
    for iv in range(oracle.n_intervals(desc)):
        ref = oracle.records(desc, iv)
        got = ctx.debug_records(k, iv, sorted=False)
        assert np.array_equal(ref[np.lexsort(ref.T[::-1])], got[np.lexsort(got.T[::-1])])


@pytest.mark.parametrize("name", ["partial-chunk", "descending", "two-loops", "stride-buckets",
                                  "flat-few-threads", "pass-boundary", "thread-linear"])
def test_linear_items(ctx, name):
    desc = linear_case(name)
    k, r, o = compare(ctx, desc)
    info = k.info()
    say(f"[linear] {name}: {info.n_linear_entries} of {info.n_entries} entries linear")
    assert info.n_linear_entries > 0
    if name == "two-loops":
        assert info.n_linear_entries < info.n_entries
    if name == "pass-boundary":
        # the record dump needs every pass of an interval in one workspace
        # (two passes of 2^20 buckets do not fit): counts and witnesses above
        assert info.n_subintervals >= 2
        return
    _records_equal(ctx, k, desc)


def test_thread_linear_out_of_bounds(ctx):
    import paper_2503_08946_amd as rv
    desc = linear_case("thread-linear-oob")
    o = oracle.check(desc)
    assert o.status == -5
    k = ctx.load(desc)
    assert k.info().n_linear_entries == 1
    with pytest.raises(rv.RVError) as e:
        ctx.check(k)
    assert e.value.status == -5
    # first out-of-bounds instance: index 40 + 2 tx + 4 bx >= 100 at tx = 30 of block 0
    iv, gthread, dphase, access, lidx = o.oob
    assert (iv, gthread) == (0, 30)
    assert f"interval {iv}, block 0, thread 30, dynamic phase {dphase}, access {access}" in e.value.message


def test_linear_items_out_of_bounds(ctx):
    import paper_2503_08946_amd as rv
    desc = linear_case("edge-out-of-bounds")
    o = oracle.check(desc)
    assert o.status == -5
    k = ctx.load(desc)
    assert k.info().n_linear_entries == 1
    with pytest.raises(rv.RVError) as e:
        ctx.check(k)
    assert e.value.status == -5
    # the oracle's first out-of-bounds instance: thread 60 of block 1 at l0 = 6
    # (index 60 * 16 + 1024 + 6 = 1990)
    iv, gthread, dphase, access, lidx = o.oob
    assert (iv, gthread, lidx) == (0, 124, 6)
    say(f"[linear] {e.value.message}")
    assert f"interval {iv}, block 1, thread 60, dynamic phase {dphase}, access {access}" in e.value.message


# ------------------------------------------------------------- edge cases
def test_large_grid_out_of_bounds(ctx):
    # block ids reach 2^23 + 63: g[bx + 2^23] leaves g[2^24] from block 2^23
    # on; the fast path's index arithmetic must see that (a 24-bit product
    # wraps block 2^23 to -2^23 and reads index 0)
    import paper_2503_08946_amd as rv
    desc = large_grid(1 << 23, 1 << 24)
    o = oracle.check(desc, max_witnesses=1)
    assert o.status == -5 and o.oob == (0, 1 << 23, 0, 0, 0)
    k = ctx.load(desc)
    assert (k.info().n_fast_entries, k.info().n_proven_entries) == (1, 0)
    with pytest.raises(rv.RVError) as e:
        ctx.check(k)
    assert e.value.status == -5
    say(f"[large-grid] {e.value.message}")
    assert f"interval 0, block {1 << 23}, thread 0, dynamic phase 0, access 0" in e.value.message


def test_large_grid_in_bounds(ctx):
    # the same launch in bounds, with writes: block x writes g[x + 2^23 - 64]
    # and block x + 1 reads it, so every location but the ends conflicts
    desc = large_grid((1 << 23) - 63, (1 << 24) + 1, write_offset=(1 << 23) - 64)
    k, r, o = compare(ctx, desc, max_list=1 << 12)
    assert r.n_records == 2 * ((1 << 23) + 64)
    assert r.n_conflicts == (1 << 23) + 63



def test_empty_kernel(ctx):
    b = Builder((4, 1), (1, 1), "empty")
    b.array(SHARED, (4,))
    k = ctx.load(b.build())
    r = ctx.check(k)
    assert (r.n_records, r.n_conflicts, r.witness) == (0, 0, None)


def test_zero_trip_loops_and_false_guards(ctx):
    b = Builder((16, 2), (2, 1), "degenerate")
    s = b.array(SHARED, (40,))
    p = b.phase([rw(s, True, aff(tx=1), loops=((3, 3),)),                 # empty loop
                 rw(s, True, aff(0), guards=(aff(-1),)),                  # guard never holds
                 rw(s, False, aff(tx=1, l0=1), loops=((0, 2),))], False)
    b.segment([p])
    compare(ctx, b.build())


def test_single_thread(ctx):
    b = Builder((1, 1), (1, 1), "one-thread")
    g = b.array(GLOBAL, (8,))
    p = b.phase([rw(g, True, aff(l0=1), loops=((0, 8),)), rw(g, False, aff(l0=1), loops=((0, 8),))], False)
    b.segment([p])
    k, r, _ = compare(ctx, b.build())
    assert r.n_conflicts == 0


def test_out_of_bounds_reports_smallest_instance(ctx):
    import paper_2503_08946_amd as rv
    b = Builder((8, 1), (2, 1), "oob")
    s = b.array(SHARED, (8,))
    p0 = b.phase([rw(s, True, aff(tx=1))], True)
    p1 = b.phase([rw(s, False, aff(0, tx=1)), rw(s, False, aff(5, tx=1))], False)
    b.segment([p0, p1])
    desc = b.build()
    o = oracle.check(desc)
    assert o.status == -5
    k = ctx.load(desc)
    with pytest.raises(rv.RVError) as e:
        ctx.check(k)
    assert e.value.status == -5
    # oracle: (interval 1, gthread 3, dyn phase 1, access 2, loop index 0)
    assert "interval 1, block 0, thread 3, dynamic phase 1, access 2" in e.value.message


def test_hot_location_exceeds_one_slice(ctx):
    # every thread of 64 blocks x 256 reads g[0] 4 times and thread 7 of block 3 writes it:
    # one location with 65537 records, far above one on-chip slice
    b = Builder((256, 1), (64, 1), "hot-location")
    g = b.array(GLOBAL, (4,))
    who = 3 * 256 + 7
    # the guard pair pins tx + 256*bx == who (>= and <=)
    p = b.phase([rw(g, False, aff(0), loops=((0, 4),)),
                 rw(g, True, aff(0), guards=(aff(-who, tx=1, bx=256), aff(who, tx=-1, bx=-256)))], False)
    b.segment([p])
    k, r, o = compare(ctx, b.build())
    assert r.n_records == 64 * 256 * 4 + 1 and r.n_conflicts == 1


def test_hot_buckets_split_over_workgroups(ctx):
    # two locations with 262,144 and 131,073 records (buckets far above one
    # workgroup's share, folded in parts) next to ordinary buckets
    b = Builder((256, 1), (256, 1), "hot-buckets")
    g = b.array(GLOBAL, (4096,))
    who = 77 * 256 + 5
    p = b.phase([rw(g, False, aff(0), loops=((0, 4),)),
                 rw(g, False, aff(2048), loops=((0, 2),)),
                 rw(g, True, aff(2048), guards=(aff(-who, tx=1, bx=256), aff(who, tx=-1, bx=-256))),
                 rw(g, True, aff(1024, tx=1))], False)
    b.segment([p])
    k, r, o = compare(ctx, b.build())
    assert r.n_records == 256 * 256 * 4 + 256 * 256 * 2 + 1 + 256 * 256
    assert r.n_conflicts == 1 + 256


@pytest.mark.parametrize("log_dim", [22, 25])
def test_tile_spanning_many_buckets(ctx, log_dim):
    # pseudo-random addresses over a large global array: one expansion tile
    # touches thousands of buckets (LDS bins in windows at 2^22, per-record
    # reservations at 2^25)
    b = Builder((256, 1), (1, 1), f"wide-tile-{log_dim}")
    g = b.array(GLOBAL, (1 << log_dim,))
    h = Aux(AUX_EMOD, 1 << log_dim, aff(13, tx=7919, l0=104729))
    h2 = Aux(AUX_EMOD, 1 << log_dim, aff(13 + 7919, tx=7919, l0=104729))    # thread tx + 1's address
    p = b.phase([rw(g, False, aff(aux0=1), loops=((0, 256),), aux=(h, Aux())),
                 rw(g, True, aff(aux0=1), loops=((0, 8),), aux=(h, Aux())),
                 rw(g, True, aff(aux0=1), loops=((0, 4),), aux=(h2, Aux()))], False)
    b.segment([p])
    k, r, o = compare(ctx, b.build())
    assert r.n_conflicts > 0


def test_key_range_passes(ctx):
    # a 2^30-element global array touched sparsely: the interval's location
    # space needs more than one key-range pass
    b = Builder((64, 1), (32, 1), "wide-global")
    g = b.array(GLOBAL, (1 << 30,))
    stride = (1 << 30) // 32
    p = b.phase([rw(g, True, aff(tx=1, bx=stride)),
                 rw(g, False, aff(7, tx=1, bx=stride)),
                 rw(g, True, aff(3 << 28, tx=2)),
                 rw(g, False, aff(3 << 28, tx=1))], False)
    b.segment([p])
    desc = b.build()
    k = ctx.load(desc)
    assert k.info().n_subintervals >= 2
    compare(ctx, desc)


def test_many_chunks_small_workspace():
    import paper_2503_08946_amd as rv
    c = rv.Context(0, workspace_bytes=64 << 20)
    desc = K.tiled_matmul(grid=4, k_iters=8, drop_dynamic=5)
    k = c.load(desc)
    assert k.info().n_chunks > 1
    compare(c, desc)
    c.close()


# -------------------------------------------------------------- batches
def test_batch_equals_single(ctx):
    descs = [K.tiny_fixed(), K.tree_reduction(3, block=256, grid=4), K.gespmm_crc(middle_barrier=False),
             K.tiled_matmul(grid=2, k_iters=2, drop_dynamic=2)] + K.tiny_random(seed=9, count=12)
    descs += RA.batch_kernels(seed=4, count=24)
    ks = [ctx.load(d) for d in descs]
    single = [ctx.check(k) for k in ks]
    batch = ctx.check_batch(ks)
    for d, s, bt in zip(descs, single, batch):
        say(f"[batch] {d.name}")
        assert (s.n_records, s.n_conflicts) == (bt.n_records, bt.n_conflicts)
        assert (s.witness is None) == (bt.witness is None)
        if s.witness:
            assert _wkey(s.witness) == _wkey(bt.witness)
    for d in descs[:20]:
        o = oracle.check(d, max_witnesses=1)
        s = single[descs.index(d)]
        assert (s.n_records, s.n_conflicts) == (o.n_records, o.n_conflicts)


def test_batched_workload_sample(ctx):
    # the batched workload's first kernels (seed 4), all of them checked against the oracle
    descs = RA.batch_kernels(seed=4, count=48)
    ks = [ctx.load(d) for d in descs]
    res = ctx.check_batch(ks)
    for d, r in zip(descs, res):
        say(f"[batch-c4] {d.name} {r.n_records}")
        o = oracle.check(d, max_witnesses=1)
        assert (r.n_records, r.n_conflicts) == (o.n_records, o.n_conflicts)
        if o.n_conflicts:
            assert _wkey(r.witness) == _wkey(o.witnesses[0])


def test_witness_windows(ctx):
    desc = K.tree_reduction(1)
    k = ctx.load(desc)
    o = oracle.check(desc, max_witnesses=1 << 15)
    full = ctx.witnesses(k, 0, 1 << 15)
    assert len(full) == o.n_conflicts == 16384
    mid = ctx.witnesses(k, 1000, 77)
    assert [_wkey(w) for w in mid] == [_wkey(w) for w in full[1000:1077]]
    tail = ctx.witnesses(k, 16380, 100)
    assert len(tail) == 4


def _read_only(i):
    # 4,096 global reads, no write: a pass of the HBM pipeline (above the
    # small-pass threshold) that is counted only and has no buckets
    b = Builder((64, 1), (16, 1), f"read-only-{i}")
    g = b.array(GLOBAL, (1024,), "g")
    b.segment([b.phase([rw(g, False, aff(i, tx=3, bx=5), loops=((0, 4),))], barrier_after=False)])
    return b.build()


def _writer(i):
    # 3,072 records over a 4M-element array (8,192 buckets, most of them
    # empty): thread t reads what thread t + 1 writes
    b = Builder((64, 1), (16, 1), f"writer-{i}")
    g = b.array(GLOBAL, (1 << 22,), "g")
    b.segment([b.phase([rw(g, True, aff(i, tx=1024, bx=65536), loops=((0, 2),)),
                        rw(g, False, aff(1024 + i, tx=1024, bx=65536))], barrier_after=False)])
    return b.build()


def test_batch_groups_spanning_many_passes_without_buckets(ctx):
    """A batch where more than one fold group's worth of bucket-less passes
    (read-only kernels, counted only) lies between two kernels with buckets:
    the fold finds each bucket's pass past its table of the group's next
    passes.  Every kernel's counts and first witness equal the oracle's."""
    descs = [_writer(0)] + [_read_only(i) for i in range(80)] + [_writer(1)] + \
        [_read_only(80 + i) for i in range(3)] + [_writer(2)]
    want = []
    for d in descs:
        o = oracle.check(d, max_witnesses=1)
        assert o.status == 0
        want.append((o.n_records, o.n_conflicts, _wkey(o.witnesses[0]) if o.n_conflicts else None))
    assert all(w[1] > 0 for w, d in zip(want, descs) if d.name.startswith("writer"))
    ks = [ctx.load(d) for d in descs]
    try:
        got = [(r.n_records, r.n_conflicts, _wkey(r.witness) if r.witness is not None else None)
               for r in ctx.check_batch(ks)]
        assert got == want
    finally:
        for k in ks:
            k.free()
