"""GPU parity of the exact counts (rv_check_counts) against the oracle:

* distinct-thread pairs under interval semantics (the oracle's n_pairs,
  itself pinned by the brute force and by closed forms: 31 per conflicting
  location of the tiled matmul, 85,344 for the polynomial product);
* RaW / WaW / WaR and the elements holding a dependence on the sequential
  schedule (oracle.ordered, pinned by App.1's closed forms).

Buckets up to one LDS tile are ordered in LDS; larger ones (hot locations)
by the workgroup radix sort in global memory: both are covered."""

import sys

import numpy as np
import pytest

import oracle
from cases import rand_medium, rand_scoped, rand_small
from workloads import kernels as K
from workloads.desc import BARRIER_WARP, GLOBAL, SHARED, Builder, aff, rw

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2503_08946_amd as rv
    c = rv.Context(0, workspace_bytes=1 << 30)
    yield c
    c.close()


def pairs_vs_oracle(ctx, desc):
    o = oracle.check(desc, max_witnesses=1)
    say(f"[counts] pairs {desc.name}: records={o.n_records} pairs={o.n_pairs}")
    assert o.status == 0
    k = ctx.load(desc)
    try:
        g = ctx.check_counts(k)
    finally:
        k.free()
    assert (g["n_records"], g["n_conflicts"], g["n_pairs"]) == (o.n_records, o.n_conflicts, o.n_pairs)
    return g


def ordered_vs_oracle(ctx, desc):
    o = oracle.ordered(desc)
    say(f"[counts] ordered {desc.name}: records={o.n_records} raw={o.n_raw} waw={o.n_waw} war={o.n_war}")
    k = ctx.load(desc, semantics="ordered")
    try:
        if o.status == -5:
            import paper_2503_08946_amd as rv
            with pytest.raises(rv.RVError) as e:
                ctx.check_counts(k)
            assert e.value.status == -5
            return None
        assert o.status == 0
        g = ctx.check_counts(k)
    finally:
        k.free()
    assert (g["n_records"], g["n_raw"], g["n_waw"], g["n_war"], g["n_dep_locations"]) == \
        (o.n_records, o.n_raw, o.n_waw, o.n_war, o.n_dep_locations)
    return g


def hot_location(threads=1024, grid=8, loops=8):
    """Every thread of every block reads and writes g[0] `loops` times: one
    location of threads x grid x 2 x loops records (beyond one LDS tile)."""
    b = Builder((threads, 1), (grid, 1), f"hot-location-{threads * grid * 2 * loops}")
    g = b.array(GLOBAL, (4,))
    p = b.phase([rw(g, False, aff(0), loops=((0, loops),)), rw(g, True, aff(0), loops=((0, loops),))], False)
    b.segment([p])
    return b.build()


def hot_mixed():
    """A few hot locations in one bucket and many cold ones."""
    b = Builder((256, 1), (16, 1), "hot-mixed")
    g = b.array(GLOBAL, (64,))
    s = b.array(SHARED, (256,))
    p0 = b.phase([rw(g, True, aff(0, tx=0), loops=((0, 2),)), rw(g, False, aff(1), loops=((0, 3),)),
                  rw(s, True, aff(tx=1)), rw(g, False, aff(2, bx=1))], True)
    p1 = b.phase([rw(g, True, aff(1), guards=(aff(3, tx=-1),)), rw(s, False, aff(255, tx=-1))], False)
    b.segment([p0, p1])
    return b.build()


# ---------------------------------------------------------------- pairs
@pytest.mark.parametrize("name", ["tiny_fixed", "polynomial_product", "half_index_shared", "half_index_global",
                                  "gespmm_crc", "stride1_global"])
def test_pairs_pins(ctx, name):
    pairs_vs_oracle(ctx, getattr(K, name)())


def test_pairs_closed_forms(ctx):
    assert pairs_vs_oracle(ctx, K.polynomial_product(64))["n_pairs"] == 85344
    g = pairs_vs_oracle(ctx, K.tiled_matmul(grid=2, k_iters=4, drop_dynamic=2))
    assert g["n_pairs"] == 31 * g["n_conflicts"]
    for k in (-1, 0, 4):
        pairs_vs_oracle(ctx, K.tree_reduction(k))


def test_pairs_hot_buckets(ctx):
    pairs_vs_oracle(ctx, hot_location())
    pairs_vs_oracle(ctx, hot_mixed())


@pytest.mark.parametrize("seed", range(2))
def test_pairs_fuzz(ctx, seed):
    rng = np.random.Generator(np.random.PCG64(9700 + seed))
    for i in range(40):
        d = rand_small(rng, i)
        if oracle.check(d, max_witnesses=1).status == 0:
            pairs_vs_oracle(ctx, d)
    for i in range(15):
        pairs_vs_oracle(ctx, rand_medium(rng, i, oob_rate=0.0))


def test_pairs_refused(ctx):
    import paper_2503_08946_amd as rv
    for desc, sem in ((K.warp_exchange(BARRIER_WARP), "interval"), (K.cross_block_global(), "strict")):
        k = ctx.load(desc, semantics=sem)
        try:
            with pytest.raises(rv.RVError) as e:
                ctx.check_counts(k)
            assert e.value.status == -2
        finally:
            k.free()


# -------------------------------------------------------------- ordered
@pytest.mark.parametrize("full", [False, True])
def test_ordered_polynomial(ctx, full):
    g = ordered_vs_oracle(ctx, K.polynomial_product_full(64) if full else K.polynomial_product(64))
    assert g["n_war"] == 85344 and g["n_raw"] == 85344 + (4096 if full else 0)


@pytest.mark.parametrize("desc", [K.tiny_fixed(), K.gespmm_crc(), K.tiled_matmul(grid=2, k_iters=3),
                                  K.tree_reduction(3, block=256, grid=4), K.warp_reduction(1),
                                  K.cross_block_global()], ids=lambda d: d.name)
def test_ordered_kernels(ctx, desc):
    ordered_vs_oracle(ctx, desc)


def test_ordered_hot_buckets(ctx):
    ordered_vs_oracle(ctx, hot_location())
    ordered_vs_oracle(ctx, hot_mixed())
    ordered_vs_oracle(ctx, hot_location(threads=512, grid=3, loops=5))


@pytest.mark.parametrize("seed", range(2))
def test_ordered_fuzz(ctx, seed):
    rng = np.random.Generator(np.random.PCG64(9800 + seed))
    for i in range(40):
        ordered_vs_oracle(ctx, rand_small(rng, i))
    for i in range(20):
        ordered_vs_oracle(ctx, rand_scoped(rng, i))
    for i in range(12):
        ordered_vs_oracle(ctx, rand_medium(rng, i, oob_rate=0.0))


def test_ordered_refuses_race_entry_points(ctx):
    import paper_2503_08946_amd as rv
    k = ctx.load(K.polynomial_product(8), semantics="ordered")
    try:
        for f in (lambda: ctx.check(k), lambda: ctx.check_batch([k]), lambda: ctx.check_static(k),
                  lambda: ctx.witnesses(k, 0, 4)):
            with pytest.raises(rv.RVError) as e:
                f()
            assert e.value.status == -9
    finally:
        k.free()
