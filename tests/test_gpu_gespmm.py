"""The Ge-SpMM staging workload (Section 2.1.2's relations of Algorithm 2,
coalesced row caching, superset domain of Section 2.1.1) on the GPU:

* at small sizes, bit-exact against the oracle (counts, whole witness lists,
  record multisets) in all four barrier variants, with both grouping kernels;
* at every size the benchmark sweeps, in the launch configuration it times
  (16 GiB workspace), counts and first witnesses against the closed forms:
  race-free with both barriers (the verdict of Section 3's results table),
  64 T blocks conflicts without the middle barrier, 64 (T-1) blocks without
  the trailing one."""

import sys

import numpy as np
import pytest

import oracle
from cases import gespmm_closed_form
from workloads import kernels as K

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _wkey(w):
    return (w.interval, w.space, w.block, w.array, w.address,
            (w.first.block, w.first.tid, w.first.dphase, w.first.access, tuple(w.first.loop), w.first.is_write),
            (w.second.block, w.second.tid, w.second.dphase, w.second.access, tuple(w.second.loop),
             w.second.is_write))


@pytest.fixture(scope="module", params=["fold", "sort_scan"])
def ctx(request):
    import paper_2503_08946_amd as rv
    c = rv.Context(0, workspace_bytes=1 << 30)
    c.group = request.param
    yield c
    c.close()


@pytest.mark.parametrize("size", [(8, 96, 4, 3), (33, 64, 2, 5)])
@pytest.mark.parametrize("mid,trail", [(True, True), (False, True), (True, False), (False, False)])
def test_gespmm_small_oracle(ctx, size, mid, trail):
    M, N, T, Kb = size
    desc = K.gespmm_crc(M, N, T, Kb, middle_barrier=mid, trailing_barrier=trail, kb_on_all=False)
    say(f"[gespmm] {ctx.group} {desc.name}")
    o = oracle.check(desc, max_witnesses=1 << 16)
    cf = gespmm_closed_form(M, N, T, Kb)
    tag = "both" if mid and trail else ("no_middle" if trail else ("no_trailing" if mid else None))
    assert o.n_records == cf["records"]
    if tag:
        assert o.n_conflicts == cf["conflicts"][tag]
    k = ctx.load(desc)
    try:
        g = ctx.check(k)
        assert (g.n_records, g.n_conflicts) == (o.n_records, o.n_conflicts)
        if o.n_conflicts:
            ws = ctx.witnesses(k, 0, o.n_conflicts)
            assert [_wkey(w) for w in ws] == [_wkey(w) for w in o.witnesses[:o.n_conflicts]]
        else:
            assert g.witness is None
        for iv in range(oracle.n_intervals(desc)):
            ref = oracle.records(desc, iv)
            got = ctx.debug_records(k, iv, sorted=False)
            assert np.array_equal(ref[np.lexsort(ref.T[::-1])], got[np.lexsort(got.T[::-1])]), iv
    finally:
        k.free()


@pytest.fixture(scope="module")
def big_ctx():
    import paper_2503_08946_amd as rv
    c = rv.Context(0, workspace_bytes=16 << 30)
    yield c
    c.close()


@pytest.mark.parametrize("size", list(K.GESPMM_SWEEP), ids=lambda s: "M%d-N%d-T%d-K%d" % s)
def test_gespmm_sweep_closed_forms(big_ctx, size):
    M, N, T, Kb = size
    cf = gespmm_closed_form(M, N, T, Kb)
    for tag, mid, trail in (("both", True, True), ("no_middle", False, True), ("no_trailing", True, False)):
        desc = K.gespmm_crc(M, N, T, Kb, middle_barrier=mid, trailing_barrier=trail, kb_on_all=False)
        say(f"[gespmm] {desc.name}: expecting {cf['records']} records, {cf['conflicts'][tag]} conflicts")
        k = big_ctx.load(desc)
        try:
            g = big_ctx.check(k)
        finally:
            k.free()
        assert (g.n_records, g.n_conflicts) == (cf["records"], cf["conflicts"][tag])
        if tag == "both":
            assert g.witness is None
            continue
        # sm_k[0] of block 0: thread 0's staging write and thread 31's read of kk = 0
        w = g.witness
        iv = 0 if tag == "no_middle" else 1
        assert (w.interval, w.space, w.block, w.array, w.address) == (iv, 0, 0, 4, 0)
        first_dphase = 0 if tag == "no_middle" else 2
        assert (w.first.block, w.first.tid, w.first.dphase, w.first.access, w.first.loop, w.first.is_write) == \
            (0, 0, first_dphase, 2, (0, 0, 0), 1)
        assert (w.second.block, w.second.tid, w.second.dphase, w.second.access, w.second.loop,
                w.second.is_write) == (0, 31, 1, 4, (0, 0, 0), 0)
