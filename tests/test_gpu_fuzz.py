"""GPU fuzz: random kernels covering every description feature against the
oracle, bit-exact, with both per-bucket grouping kernels.

150 small kernels (a few threads: guards with auxiliary terms, floor
division, 3-D arrays, the segment variable, negative loop bounds, repeated
segments) and 150 medium ones (up to a few million records: several tiles
and buckets, plain affine indices on the fast paths next to auxiliary terms
and guards, about 5% out of bounds).  Per kernel: the status (and, out of
bounds, the first offending instance), record and conflict counts, the whole
witness list, and the record multiset of every interval."""

import sys

import numpy as np
import pytest

import oracle
from cases import rand_medium, rand_small

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


def _loops_of(desc, access, lidx):
    """Loop values of row-major loop index lidx of an access."""
    ext = [hi - lo for lo, hi in desc.accesses[access].loops]
    vals = [0, 0, 0]
    for j in range(len(ext) - 1, -1, -1):
        vals[j] = desc.accesses[access].loops[j][0] + lidx % ext[j]
        lidx //= ext[j]
    return tuple(vals)


def _fuzz_one(ctx, desc):
    import paper_2503_08946_amd as rv
    o = oracle.check(desc, max_witnesses=1 << 16)
    say(f"[fuzz] {ctx.group} {desc.name} records={o.n_records} status={o.status}")
    k = ctx.load(desc)
    try:
        if o.status == -5:
            with pytest.raises(rv.RVError) as e:
                ctx.check(k)
            assert e.value.status == -5
            iv, gthread, dphase, access, lidx = o.oob
            tpb = desc.block[0] * desc.block[1]
            lv = _loops_of(desc, access, lidx)
            want = (f"interval {iv}, block {gthread // tpb}, thread {gthread % tpb}, dynamic phase {dphase}, "
                    f"access {access}, loop ({lv[0]},{lv[1]},{lv[2]})")
            assert want in e.value.message, (want, e.value.message)
            return
        assert o.status == 0
        g = ctx.check(k)
        assert (g.n_records, g.n_conflicts) == (o.n_records, o.n_conflicts)
        if o.n_conflicts:
            assert _wkey(g.witness) == _wkey(o.witnesses[0])
            n = min(o.n_conflicts, 1 << 16)
            assert [_wkey(w) for w in ctx.witnesses(k, 0, n)] == [_wkey(w) for w in o.witnesses[:n]]
        else:
            assert g.witness is None
        for iv in range(oracle.n_intervals(desc)):
            ref = oracle.records(desc, iv)
            got = ctx.debug_records(k, iv, sorted=False)
            assert np.array_equal(ref[np.lexsort(ref.T[::-1])], got[np.lexsort(got.T[::-1])]), iv
    finally:
        k.free()


@pytest.mark.parametrize("seed", range(3))
def test_fuzz_small(ctx, seed):
    rng = np.random.Generator(np.random.PCG64(7000 + seed))
    for i in range(50):
        _fuzz_one(ctx, rand_small(rng, i))


@pytest.mark.parametrize("seed", range(3))
def test_fuzz_medium(ctx, seed):
    rng = np.random.Generator(np.random.PCG64(8000 + seed))
    for i in range(50):
        _fuzz_one(ctx, rand_medium(rng, i))
