"""GPU parity of the further check modes against the oracle, bit-exact:

* warp-scope barriers (interval semantics with fine intervals inside a
  barrier interval; warps as the unordered units);
* strict semantics (global records of different blocks conflict across
  intervals).

Per kernel: status, record and conflict counts, the whole witness list and
the record multiset, with both settings of the grouping kernel (passes with
sub-keys are always judged by the fold kernels)."""

import sys

import numpy as np
import pytest

import oracle
from cases import rand_medium, rand_scoped, rand_small
from workloads import kernels as K
from workloads.desc import BARRIER_BLOCK, BARRIER_WARP

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=["fold", "sort_scan"])
def ctx(request):
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


def _sorted_rows(a):
    return a[np.lexsort(a.T[::-1])] if len(a) else a.reshape(0, 13)


def compare(ctx, desc, strict=False, records=True):
    import paper_2503_08946_amd as rv
    sem = "strict" if strict else "interval"
    o = oracle.check(desc, max_witnesses=1 << 16, strict=strict)
    say(f"[modes] {ctx.group} {sem} {desc.name} records={o.n_records} conflicts={o.n_conflicts} status={o.status}")
    k = ctx.load(desc, semantics=sem)
    try:
        if o.status == -5:
            with pytest.raises(rv.RVError) as e:
                ctx.check(k)
            assert e.value.status == -5
            return o
        assert o.status == 0
        g = ctx.check(k)
        assert (g.n_records, g.n_conflicts) == (o.n_records, o.n_conflicts)
        if o.n_conflicts:
            n = min(o.n_conflicts, 1 << 16)
            assert _wkey(g.witness) == _wkey(o.witnesses[0])
            assert [_wkey(w) for w in ctx.witnesses(k, 0, n)] == [_wkey(w) for w in o.witnesses[:n]]
        else:
            assert g.witness is None
        if records:
            n_iv = oracle.n_intervals(desc)
            spaces = n_iv + (1 if strict else 0)
            got = np.concatenate([ctx.debug_records(k, s) for s in range(spaces)] or [np.zeros((0, 13), np.int64)])
            ref = np.concatenate([oracle.records(desc, iv) for iv in range(n_iv)] or [np.zeros((0, 13), np.int64)])
            assert np.array_equal(_sorted_rows(ref), _sorted_rows(got))
        return o
    finally:
        k.free()


# ------------------------------------------------------- warp barriers
@pytest.mark.parametrize("dropped", [-1, 0, 1, 2, 3, 4])
def test_warp_reduction(ctx, dropped):
    o = compare(ctx, K.warp_reduction(dropped))
    assert o.n_conflicts == (32 >> dropped if 0 <= dropped <= 3 else 0)


@pytest.mark.parametrize("dropped", [-1, 0, 3])
def test_warp_reduction_large(ctx, dropped):
    # 32 warps per block, 128 blocks: 1.5e5 records, many buckets
    o = compare(ctx, K.warp_reduction(dropped, block=1024, grid=128), records=False)
    assert o.n_conflicts == ((8 >> dropped) * 32 * 128 if 0 <= dropped <= 3 else 0)


@pytest.mark.parametrize("kind,warp", [(BARRIER_BLOCK, 32), (BARRIER_WARP, 32), (BARRIER_WARP, 64),
                                       (BARRIER_WARP, 16), (BARRIER_WARP, 1)])
def test_warp_exchange(ctx, kind, warp):
    compare(ctx, K.warp_exchange(kind, warp=warp))


@pytest.mark.parametrize("seed", range(3))
def test_warp_scopes_fuzz(ctx, seed):
    rng = np.random.Generator(np.random.PCG64(9100 + seed))
    for i in range(50):
        compare(ctx, rand_scoped(rng, i))


# -------------------------------------------------------------- strict
def test_cross_block_global(ctx):
    assert compare(ctx, K.cross_block_global(), strict=True).n_conflicts == 32
    assert compare(ctx, K.cross_block_global()).n_conflicts == 0


@pytest.mark.parametrize("d", [-1, 0, 6, 7])
def test_strict_matmul(ctx, d):
    compare(ctx, K.tiled_matmul(grid=2, k_iters=4, drop_dynamic=d), strict=True)


def test_strict_gespmm(ctx):
    compare(ctx, K.gespmm_crc(M=8, N=96, T=4, K=3, middle_barrier=False, kb_on_all=False), strict=True)


@pytest.mark.parametrize("seed", range(3))
def test_strict_fuzz_small(ctx, seed):
    rng = np.random.Generator(np.random.PCG64(9200 + seed))
    for i in range(50):
        d = rand_small(rng, i)
        compare(ctx, d.replace(warp_size=int(rng.integers(1, 5))), strict=True)


@pytest.mark.parametrize("seed", range(2))
def test_strict_fuzz_medium(ctx, seed):
    rng = np.random.Generator(np.random.PCG64(9300 + seed))
    for i in range(25):
        compare(ctx, rand_medium(rng, i, oob_rate=0.0), strict=True, records=(i % 5 == 0))


def test_strict_refuses_warp_barriers(ctx):
    import paper_2503_08946_amd as rv
    with pytest.raises(rv.RVError) as e:
        ctx.load(K.warp_exchange(BARRIER_WARP), semantics="strict")
    assert e.value.status == -2


# ---------------------------------------------------------- divergence
def _div_compare(ctx, desc):
    o = oracle.divergence(desc)
    assert o.status == 0
    k = ctx.load(desc)
    try:
        g = ctx.check_barriers(k)
    finally:
        k.free()
    say(f"[modes] barriers {desc.name}: {g['n_divergent']} of {g['n_instances']}")
    assert (g["n_instances"], g["n_divergent"]) == (o.n_instances, o.n_divergent)
    if o.n_divergent:
        assert g["first"] == (o.dphase, o.block, o.warp, o.arrive_tid, o.skip_tid)
    else:
        assert g["first"] is None


@pytest.mark.parametrize("case", ["block-half", "warp-tail", "block-uniform", "k-uniform"])
def test_guarded_barriers(ctx, case):
    _div_compare(ctx, K.guarded_barrier(case))


@pytest.mark.parametrize("seed", range(2))
def test_divergence_fuzz(ctx, seed):
    rng = np.random.Generator(np.random.PCG64(9400 + seed))
    for i in range(60):
        _div_compare(ctx, rand_scoped(rng, i))


def test_divergence_large_block(ctx):
    # 1024-thread blocks, 64 blocks, warp barrier reached by tid <= 700 in
    # repetition k = 0 only: warp 21 of every block diverges once
    from workloads.desc import Builder, aff, rw
    b = Builder((1024, 1), (64, 1), "guarded-warp-1024")
    s = b.array(0, (1024,))
    p = b.phase([rw(s, True, aff(tx=1))], barrier_after=BARRIER_WARP, barrier_guards=(aff(700, tx=-1, k=-1000),))
    b.segment([p], repeat=2)
    _div_compare(ctx, b.build())
