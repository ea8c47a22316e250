"""The batched check's on-chip path for small passes (one workgroup per
pass: expansion folded into an LDS hash table, judge) against the oracle and against
the bucket path, bit-exact: records, conflicts, first witnesses, and the
first out-of-bounds instance of a failing kernel in the batch."""

import sys

import numpy as np
import pytest

import oracle
from cases import rand_medium, rand_small
from workloads import kernels as K
from workloads import random_affine as RA

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _wkey(w):
    return None if w is None else (
        w.interval, w.space, w.block, w.array, w.address,
        (w.first.block, w.first.tid, w.first.dphase, w.first.access, tuple(w.first.loop), w.first.is_write),
        (w.second.block, w.second.tid, w.second.dphase, w.second.access, tuple(w.second.loop),
         w.second.is_write))


@pytest.fixture(scope="module")
def ctx():
    import paper_2503_08946_amd as rv
    c = rv.Context(0, workspace_bytes=1 << 30)
    yield c
    c.close()


def _batch_vs_oracle(ctx, descs):
    refs = [oracle.check(d, max_witnesses=1) for d in descs]
    ks = [ctx.load(d) for d in descs]
    try:
        out = {}
        for small in (2048, 0):
            ctx.small_cap = small
            out[small] = ctx.check_batch(ks)
            for d, o, r in zip(descs, refs, out[small]):
                assert o.status == 0, d.name
                assert (r.n_records, r.n_conflicts) == (o.n_records, o.n_conflicts), (small, d.name)
                assert _wkey(r.witness) == (_wkey(o.witnesses[0]) if o.n_conflicts else None), (small, d.name)
    finally:
        ctx.small_cap = 2048
        for k in ks:
            k.free()


def test_small_pins(ctx):
    say("[small] pin kernels")
    _batch_vs_oracle(ctx, [K.tiny_fixed(), K.polynomial_product(48), K.stride1_shared(), K.stride1_global(),
                           K.half_index_shared(), K.half_index_global(), K.gespmm_crc(),
                           K.tree_reduction(2, block=64, grid=1)] + K.tiny_random(seed=1, count=32))


@pytest.mark.parametrize("seed", range(3))
def test_small_random(ctx, seed):
    rng = np.random.Generator(np.random.PCG64(9500 + seed))
    ds = [rand_small(rng, i) for i in range(60)]
    ds = [d for d in ds if oracle.check(d, max_witnesses=1).status == 0]
    say(f"[small] random small seed {seed}: {len(ds)} kernels")
    _batch_vs_oracle(ctx, ds)


@pytest.mark.parametrize("seed", range(2))
def test_small_mixed_sizes(ctx, seed):
    # passes on both sides of the threshold in one batch
    rng = np.random.Generator(np.random.PCG64(9600 + seed))
    ds = [rand_medium(rng, i, oob_rate=0.0) for i in range(30)] + RA.batch_kernels(seed=4, count=64)
    say(f"[small] mixed seed {seed}")
    _batch_vs_oracle(ctx, ds)


def test_small_location_with_every_record(ctx):
    # all 2048 records of the pass at one location (every lane folds into one
    # hash slot)
    from workloads.desc import GLOBAL, Builder, aff, rw
    b = Builder((64, 1), (2, 1), "one-location-2048")
    g = b.array(GLOBAL, (1,))
    p = b.phase([rw(g, False, aff(0), loops=((0, 8),)), rw(g, True, aff(0), loops=((0, 8),))], False)
    b.segment([p])
    _batch_vs_oracle(ctx, [b.build(), K.tiny_fixed()])


def test_small_out_of_bounds_in_batch(ctx):
    import paper_2503_08946_amd as rv
    from workloads.desc import SHARED, Builder, aff, rw
    b = Builder((32, 1), (2, 1), "oob-small")
    s = b.array(SHARED, (16,))
    p = b.phase([rw(s, True, aff(tx=1))], False)
    b.segment([p])
    bad = b.build()
    o = oracle.check(bad, max_witnesses=1)
    assert o.status == -5
    ks = [ctx.load(K.tiny_fixed()), ctx.load(bad)]
    try:
        msgs = []
        for small in (2048, 0):
            ctx.small_cap = small
            with pytest.raises(rv.RVError) as e:
                ctx.check_batch(ks)
            assert e.value.status == -5
            msgs.append(e.value.message)
        assert msgs[0] == msgs[1]
        iv, gthread, dphase, access, lidx = o.oob
        assert f"interval {iv}, block {gthread // 32}, thread {gthread % 32}, dynamic phase {dphase}" in msgs[0]
    finally:
        ctx.small_cap = 2048
        for k in ks:
            k.free()


def test_batch_table_reuse(ctx):
    # the pass table of a batch stays on the device and is reused by the next
    # batch of the same kernels; a reloaded kernel (even at a freed one's
    # address), another threshold, or a call that rewrites the table must not
    # reuse it
    descs = RA.batch_kernels(seed=4, count=24) + [K.tiny_fixed(), K.tree_reduction(1, block=128, grid=3)]
    refs = {d.name: oracle.check(d, max_witnesses=1) for d in descs}

    def check(ks, ds):
        for d, r in zip(ds, ctx.check_batch(ks)):
            o = refs[d.name]
            assert (r.n_records, r.n_conflicts) == (o.n_records, o.n_conflicts), d.name
            assert _wkey(r.witness) == (_wkey(o.witnesses[0]) if o.n_conflicts else None), d.name

    ks = [ctx.load(d) for d in descs]
    try:
        say("[small] table reuse")
        check(ks, descs)
        check(ks, descs)                       # reused
        ks[3].free()
        ks[3] = ctx.load(descs[-1])            # another kernel, perhaps at the freed address
        ds = descs[:3] + [descs[-1]] + descs[4:]
        check(ks, ds)
        check(ks, ds)
        ctx.small_cap = 0
        check(ks, ds)
        ctx.small_cap = 2048
        ctx.debug_records(ks[0], 0)            # rewrites the context's pass table
        check(ks, ds)
        check(ks[::-1], ds[::-1])
    finally:
        ctx.small_cap = 2048
        for k in ks:
            k.free()
