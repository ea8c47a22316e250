"""Parity at the benchmark's full size, in the launch configuration bench.py
times (one context, 16 GiB workspace, default planner settings).

The 1,141,112,832-record tiled-matmul configuration: record and conflict
counts equal their closed forms, and the first witness and three windows of
the witness list equal the oracle's list for the one interval that holds the
conflicts (the interval where the dropped barrier merges two phases; the
oracle enumerates that interval alone, 17.8M records).  The same pattern at
gridDim (64, 64), 18,257,805,312 records, runs through several workspace
chunks and is checked against its closed forms."""

import sys

import pytest

import oracle
from workloads import kernels as K

pytestmark = pytest.mark.gpu

GRID16_RECORDS = 1_141_112_832
GRID64_RECORDS = 18_257_805_312
CONFLICTS_PER_BLOCK = 2048      # dropped dynamic barrier: every As/Bs element of a block


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _wkey(w):
    return (w.interval, w.space, w.block, w.array, w.address,
            (w.first.block, w.first.tid, w.first.dphase, w.first.access, tuple(w.first.loop), w.first.is_write),
            (w.second.block, w.second.tid, w.second.dphase, w.second.access, tuple(w.second.loop),
             w.second.is_write))


@pytest.fixture(scope="module")
def big_ctx():
    import paper_2503_08946_amd as rv
    c = rv.Context(0, workspace_bytes=16 << 30)
    yield c
    c.close()


def test_matmul_grid16_full_size(big_ctx):
    desc = K.tiled_matmul(grid=16, k_iters=64, drop_dynamic=64)
    k = big_ctx.load(desc)
    say("[full] grid 16 check")
    r = big_ctx.check(k)
    assert r.n_records == GRID16_RECORDS
    assert r.n_conflicts == 16 * 16 * CONFLICTS_PER_BLOCK
    # the conflicts all sit in one interval; the oracle enumerates it alone
    iv = r.witness.interval
    say(f"[full] oracle on interval {iv}")
    o = oracle.check(desc, max_witnesses=1 << 20, ilo=iv, ihi=iv + 1)
    assert o.n_conflicts == r.n_conflicts
    assert _wkey(r.witness) == _wkey(o.witnesses[0])
    for first, count in ((0, 2048), (300_000, 1024), (r.n_conflicts - 1000, 1000)):
        say(f"[full] witnesses {first} + {count}")
        got = big_ctx.witnesses(k, first, count)
        assert [_wkey(w) for w in got] == [_wkey(w) for w in o.witnesses[first:first + count]]


def test_matmul_grid64_multi_chunk(big_ctx):
    desc = K.tiled_matmul(grid=64, k_iters=64, drop_dynamic=64)
    k = big_ctx.load(desc)
    assert k.info().n_chunks > 1
    say("[full] grid 64 check")
    r = big_ctx.check(k)
    assert r.n_records == GRID64_RECORDS
    assert r.n_conflicts == 64 * 64 * CONFLICTS_PER_BLOCK
    # the smallest conflicting location is block 0's first shared element
    assert r.witness.block == 0 and r.witness.address == 0


@pytest.mark.parametrize("drop", [-1] + K.matmul_mutants(seed=3))
def test_matmul_grid16_mutants(big_ctx, drop):
    # the unmutated kernel, the fixed dropped barriers {0, 1, 64, 126, 127}
    # and three drawn from seed 3: counts against the closed forms (a dropped
    # barrier d < 127 merges two phases of one K-iteration, or a compute phase
    # with the next load: every As/Bs element of every block conflicts; d = 127
    # merges the last compute phase with the C write: no conflict), and the
    # witnesses against the oracle's list for the merged interval
    desc = K.tiled_matmul(grid=16, k_iters=64, drop_dynamic=drop)
    k = big_ctx.load(desc)
    say(f"[full] grid 16 drop {drop}")
    r = big_ctx.check(k)
    assert r.n_records == GRID16_RECORDS
    expect = 16 * 16 * CONFLICTS_PER_BLOCK if 0 <= drop < 127 else 0
    assert r.n_conflicts == expect
    if not expect:
        assert r.witness is None
        k.free()
        return
    assert r.witness.interval == drop
    o = oracle.check(desc, max_witnesses=1 << 20, ilo=drop, ihi=drop + 1)
    assert o.n_conflicts == expect
    assert _wkey(r.witness) == _wkey(o.witnesses[0])
    for first, count in ((0, 4096), (expect // 2, 512), (expect - 512, 512)):
        got = big_ctx.witnesses(k, first, count)
        assert [_wkey(w) for w in got] == [_wkey(w) for w in o.witnesses[first:first + count]]
    k.free()
