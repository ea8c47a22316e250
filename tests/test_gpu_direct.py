"""GPU parity of the on-chip check of block-local spaces.

With the context's `direct` switch on (the default), rv_check groups the
shared-array locations of each unit of blocks in LDS and sends only the
global-array records through HBM; with it off, every record goes through the
HBM pipeline.  Both must give the oracle's record and conflict counts and
canonical first witness, bit-exact, on the same seeded descriptions; an
out-of-bounds kernel must name the same first offending instance."""

import sys

import numpy as np
import pytest

import oracle
from cases import rand_affine_units, rand_medium, rand_scoped, rand_small
from workloads import kernels as K
from workloads.desc import GLOBAL, SHARED, Builder, aff, rw

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2503_08946_amd as rv
    c = rv.Context(0, workspace_bytes=1 << 30)
    yield c
    c.direct = True
    c.close()


def _wkey(w):
    return (w.interval, w.space, w.block, w.array, w.address,
            (w.first.block, w.first.tid, w.first.dphase, w.first.access, tuple(w.first.loop), w.first.is_write),
            (w.second.block, w.second.tid, w.second.dphase, w.second.access, tuple(w.second.loop),
             w.second.is_write))


def _run(ctx, k, direct):
    import paper_2503_08946_amd as rv
    ctx.direct = direct
    try:
        g = ctx.check(k)
    except rv.RVError as e:
        return ("error", e.status, e.message)
    return (g.n_records, g.n_conflicts, _wkey(g.witness) if g.witness is not None else None)


def check_both(ctx, desc, semantics="interval"):
    strict = semantics == "strict"
    import paper_2503_08946_amd as rv
    o = oracle.check(desc, max_witnesses=1, strict=strict)
    say(f"[direct] {desc.name} {semantics} records={o.n_records} status={o.status}")
    if o.status not in (0, -5):
        # a description the oracle refuses (strict semantics with warp
        # barriers) is refused at load time with the same code
        with pytest.raises(rv.RVError) as e:
            ctx.load(desc, semantics=semantics)
        assert e.value.status == o.status
        return None
    k = ctx.load(desc, semantics=semantics)
    try:
        on = _run(ctx, k, True)
        off = _run(ctx, k, False)
        assert on == off, (on, off)
        if o.status == -5:
            assert on[0] == "error" and on[1] == -5, on
        else:
            assert o.status == 0
            want = (o.n_records, o.n_conflicts, _wkey(o.witnesses[0]) if o.n_conflicts else None)
            assert on == want, (on, want)
        return k.info()
    finally:
        ctx.direct = True
        k.free()


PINS = [K.tiny_fixed(), K.polynomial_product(), K.stride1_shared(), K.half_index_shared(),
        K.tiled_matmul(grid=2, k_iters=4), K.tiled_matmul(grid=3, k_iters=4, drop_static="compute"),
        K.tiled_matmul(grid=2, k_iters=4, drop_static="load")] + \
    [K.tree_reduction(d, block=256, grid=3) for d in (-1, 0, 3, 7)] + \
    [K.tiled_matmul(grid=2, k_iters=4, drop_dynamic=d) for d in (0, 1, 4, 6, 7)]


@pytest.mark.parametrize("i", range(len(PINS)))
def test_pins(ctx, i):
    import paper_2503_08946_amd as rv
    info = check_both(ctx, PINS[i])
    # the host plan decides which intervals take units: those of the tiled
    # matmuls, the stride-1 writes and the tiny kernel's first interval
    # (plain affine shared accesses) do; a[tid/2] (floor division), the tree
    # reduction (guards) and the polynomial product (global arrays) do not
    assert info.n_direct_intervals == rv.plan(PINS[i]).n_direct_intervals
    assert (info.n_direct_intervals > 0) == PINS[i].name.startswith(("matmul", "stride1", "tiny"))


def test_direct_records_are_the_shared_records(ctx):
    desc = K.tiled_matmul(grid=3, k_iters=4, drop_dynamic=2)
    k = ctx.load(desc)
    try:
        info = k.info()
        assert info.n_direct_intervals == info.n_intervals - 1     # the last interval writes C only
        ctx.set_timing(True)
        ctx.timing(reset=True)
        g = ctx.check(k)
        t = ctx.timing(reset=True)
        ctx.set_timing(False)
        shared = sum(int(np.count_nonzero(oracle.records(desc, iv)[:, 1] == SHARED))
                     for iv in range(oracle.n_intervals(desc)))
        assert t["direct_records"] == shared
        assert t["direct"][1] > 0
        assert g.n_records == oracle.check(desc, max_witnesses=1).n_records
    finally:
        k.free()


@pytest.mark.parametrize("seed", range(2))
def test_fuzz_medium(ctx, seed):
    rng = np.random.Generator(np.random.PCG64(9100 + seed))
    for i in range(60):
        check_both(ctx, rand_medium(rng, i, oob_rate=0.02))


@pytest.mark.parametrize("seed", range(2))
def test_fuzz_small(ctx, seed):
    rng = np.random.Generator(np.random.PCG64(9200 + seed))
    for i in range(60):
        check_both(ctx, rand_small(rng, i))


@pytest.mark.parametrize("seed,semantics", [(0, "interval"), (1, "interval"), (2, "strict")])
def test_fuzz_units(ctx, seed, semantics):
    # plain affine kernels with small shared arrays: almost all take units
    rng = np.random.Generator(np.random.PCG64(9500 + seed))
    n_units = 0
    for i in range(60):
        info = check_both(ctx, rand_affine_units(rng, i), semantics)
        n_units += info is not None and info.n_direct_intervals > 0
    assert n_units >= 40


@pytest.mark.parametrize("semantics", ["interval", "strict"])
def test_fuzz_scoped(ctx, semantics):
    # warp barriers give an interval sub-keys (no units); the others keep them
    rng = np.random.Generator(np.random.PCG64(9300))
    for i in range(40):
        check_both(ctx, rand_scoped(rng, i), semantics)


def _edge_kernel(bdx, bdy, gdx, gdy, name):
    """Blocks of bdx*bdy threads (not a multiple of a work item's 256) and a
    shared array of tpb + 5 elements: units of several blocks whose edges
    cut work items.  Over a 5-point loop each thread writes s[tid + l0] and
    reads s[tpb - 1 - tid + l0] (plain affine indices, so the units take
    them); a global stride-1 write; then a read of s[tx]."""
    b = Builder((bdx, bdy), (gdx, gdy), name)
    tpb = bdx * bdy
    s = b.array(SHARED, (tpb + 5,), "s")
    g = b.array(GLOBAL, (tpb * gdx * gdy,), "g")
    ph = b.phase([
        rw(s, True, aff(0, tx=1, ty=bdx, l0=1), loops=((0, 5),)),
        rw(s, False, aff(tpb - 1, tx=-1, ty=-bdx, l0=1), loops=((0, 5),)),
        rw(g, True, aff(0, tx=1, ty=bdx, bx=tpb, by=tpb * gdx)),
    ], barrier_after=True)
    ph2 = b.phase([rw(s, False, aff(0, tx=1), loops=((0, 1),))], barrier_after=False)
    b.segment([ph, ph2])
    return b.build()


@pytest.mark.parametrize("shape", [(48, 4, 40, 3), (100, 1, 30, 5), (10, 7, 60, 4), (32, 8, 5, 5)])
def test_unit_edges(ctx, shape):
    info = check_both(ctx, _edge_kernel(*shape, name=f"edge-{'-'.join(map(str, shape))}"))
    assert info.n_direct_intervals >= 1


def test_large_shared_space_keeps_hbm_path(ctx):
    # 4096 shared elements per block exceed one unit's table
    b = Builder((64, 2), (3, 2), "shared-4096")
    s = b.array(SHARED, (64, 64), "s")
    b.segment([b.phase([rw(s, True, aff(0, ty=1), aff(0, tx=1)), rw(s, False, aff(1, ty=1), aff(0, tx=1))],
                       barrier_after=False)])
    desc = b.build()
    info = check_both(ctx, desc)
    assert info.n_direct_intervals == 0


def test_two_passes_split_the_shared_locations():
    """262,656 blocks of 256 threads with 2048 shared elements each: the
    interval's 537,919,488 locations span two key-range passes, the second
    starting inside the shared locations.  Each block writes s[t] and reads
    s[t + 1]: 255 conflicting locations per block, s[1] .. s[255] (closed
    form); with units and without, the same counts and first witness."""
    import paper_2503_08946_amd as rv
    gdx, gdy = 512, 513
    b = Builder((256, 1), (gdx, gdy), "two-pass-shared")
    s = b.array(SHARED, (2048,), "s")
    b.segment([b.phase([rw(s, True, aff(0, tx=1)), rw(s, False, aff(1, tx=1))], barrier_after=False)])
    desc = b.build()
    c = rv.Context(0, workspace_bytes=3 << 30)
    try:
        k = c.load(desc)
        info = k.info()
        say(f"[direct] two-pass subs={info.n_subintervals} direct={info.n_direct_intervals}")
        assert info.n_subintervals == 2 and info.n_direct_intervals == 1
        on = _run(c, k, True)
        off = _run(c, k, False)
        nblocks = gdx * gdy
        assert on == off
        assert on[0] == 2 * 256 * nblocks and on[1] == 255 * nblocks
        w = on[2]
        assert (w[0], w[1], w[2], w[3], w[4]) == (0, SHARED, 0, 0, 1)
        k.free()
    finally:
        c.close()


def test_witness_lists_and_static_with_units_on(ctx):
    # rv_get_witnesses and rv_check_static take the HBM path whatever the switch
    desc = K.tiled_matmul(grid=2, k_iters=4, drop_dynamic=3)
    o = oracle.check(desc, max_witnesses=1 << 16)
    assert o.n_conflicts == len(o.witnesses) == 2048 * 4
    k = ctx.load(desc)
    try:
        ctx.direct = True
        ws = ctx.witnesses(k, 0, o.n_conflicts)
        assert [_wkey(w) for w in ws] == [_wkey(w) for w in o.witnesses[:o.n_conflicts]]
        gs = ctx.check_static(k)
        g = ctx.check(k)
        assert (gs.n_records, gs.n_conflicts, _wkey(gs.witness)) == (g.n_records, g.n_conflicts, _wkey(g.witness))
    finally:
        k.free()


def _batch_results(ctx, ks, direct):
    import paper_2503_08946_amd as rv
    ctx.direct = direct
    b = rv.Batch(ctx, ks)
    b.run()
    return [(r.n_records, r.n_conflicts, _wkey(r.witness) if r.witness is not None else None) for r in b.results()]


@pytest.mark.parametrize("small_cap", [0, 2048])
def test_batch_units(ctx, small_cap):
    """rv_check_batch with units on and off: every kernel's counts and first
    witness equal the oracle's (units re-based onto the batch's passes,
    small passes on chip beside them); the same batch twice reuses its
    table."""
    rng = np.random.Generator(np.random.PCG64(9400))
    descs = PINS + [rand_medium(rng, i, oob_rate=0.0) for i in range(12)] + \
        [rand_affine_units(rng, i) for i in range(12)] + \
        [_edge_kernel(*sh, name=f"edge-b{j}") for j, sh in enumerate([(48, 4, 40, 3), (10, 7, 60, 4)])]
    want = []
    for d in descs:
        o = oracle.check(d, max_witnesses=1)
        assert o.status == 0
        want.append((o.n_records, o.n_conflicts, _wkey(o.witnesses[0]) if o.n_conflicts else None))
    ks = [ctx.load(d) for d in descs]
    try:
        ctx.small_cap = small_cap
        ctx.set_timing(True)
        ctx.timing(reset=True)
        on = _batch_results(ctx, ks, True)
        t = ctx.timing(reset=True)
        ctx.set_timing(False)
        assert t["direct_records"] > 0
        assert on == want
        assert _batch_results(ctx, ks, True) == want      # cached table
        assert _batch_results(ctx, ks, False) == want
    finally:
        ctx.small_cap = 2048
        ctx.direct = True
        for k in ks:
            k.free()
