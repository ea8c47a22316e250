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
from cases import rand_medium, rand_scoped, rand_small
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
    info = check_both(ctx, PINS[i])
    # every kernel here but the polynomial product (global arrays only) has
    # intervals with shared arrays of at most 2048 elements per block
    assert (info.n_direct_intervals > 0) == (PINS[i].name != "polynomial-product-64")


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


@pytest.mark.parametrize("semantics", ["interval", "strict"])
def test_fuzz_scoped(ctx, semantics):
    # warp barriers give an interval sub-keys (no units); the others keep them
    rng = np.random.Generator(np.random.PCG64(9300))
    for i in range(40):
        check_both(ctx, rand_scoped(rng, i), semantics)


def _edge_kernel(bdx, bdy, gdx, gdy, sdim, name):
    """Blocks of bdx*bdy threads (not a multiple of a work item's 256) and a
    shared array of sdim elements: units of several blocks whose edges cut
    work items.  s[(tid + l0) % sdim] written, s[(2 tid + 1 + l0) % sdim]
    read over a 5-point loop, and a global stride-1 write."""
    from workloads.desc import AUX_EMOD, Aux
    b = Builder((bdx, bdy), (gdx, gdy), name)
    s = b.array(SHARED, (sdim,), "s")
    g = b.array(GLOBAL, (bdx * bdy * gdx * gdy,), "g")
    tpb = bdx * bdy
    ph = b.phase([
        rw(s, True, aff(aux1=1), loops=((0, 5),), aux=(Aux(), Aux(AUX_EMOD, sdim, aff(0, tx=1, ty=bdx, l0=1)))),
        rw(s, False, aff(aux1=1), loops=((0, 5),), aux=(Aux(), Aux(AUX_EMOD, sdim, aff(1, tx=2, ty=2 * bdx, l0=1)))),
        rw(g, True, aff(0, tx=1, ty=bdx, bx=tpb, by=tpb * gdx)),
    ], barrier_after=True)
    ph2 = b.phase([rw(s, False, aff(0, tx=1), loops=((0, 1),)) if bdx <= sdim else rw(s, False, aff(0))],
                  barrier_after=False)
    b.segment([ph, ph2])
    return b.build()


@pytest.mark.parametrize("shape", [(48, 4, 40, 3, 64), (100, 1, 30, 5, 100), (10, 7, 60, 4, 300),
                                   (32, 8, 5, 5, 130)])
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
    s[(t + 1) mod 256]: 256 conflicting locations per block (closed form);
    with units and without, the same counts and first witness."""
    import paper_2503_08946_amd as rv
    from workloads.desc import AUX_EMOD, Aux
    gdx, gdy = 512, 513
    b = Builder((256, 1), (gdx, gdy), "two-pass-shared")
    s = b.array(SHARED, (2048,), "s")
    b.segment([b.phase([rw(s, True, aff(0, tx=1)),
                        rw(s, False, aff(aux1=1), aux=(Aux(), Aux(AUX_EMOD, 256, aff(1, tx=1))))],
                       barrier_after=False)])
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
        assert on[0] == 2 * 256 * nblocks and on[1] == 256 * nblocks
        w = on[2]
        assert (w[0], w[1], w[2], w[3], w[4]) == (0, SHARED, 0, 0, 0)
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
