"""CPU pins of the oracle's further modes (test infrastructure: no GPU).

* warp-scope barriers inside the per-interval check, and barrier divergence;
* strict semantics: blocks never ordered, so global records of different
  blocks conflict across intervals;
* ordered dependences: RaW / WaW / WaR on the sequential schedule.

Each mode is pinned twice: by hand-derived results (golden/modes.json) and
by the O(N^2) brute force of tests/brute.py on random kernels that use
every description feature (warp sizes of 1-4 threads, guarded barriers)."""

import json
import os

import numpy as np
import pytest

import oracle
from brute import brute_check, brute_divergence, brute_ordered
from cases import rand_scoped, rand_small
from workloads import kernels as K
from workloads.desc import BARRIER_BLOCK, BARRIER_WARP

PINS = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "modes.json")))


def _side(s):
    return [s.block, s.tid, s.dphase, s.access, list(s.loop), s.is_write]


def _loc(w):
    return [w.interval, w.space, w.block, w.array, w.address]


# --------------------------------------------------------- warp barriers
@pytest.mark.parametrize("dropped", [-1, 0, 1, 2, 3, 4])
def test_warp_reduction(dropped):
    pin = PINS["warp_reduction"]
    r = oracle.check(K.warp_reduction(dropped))
    assert r.status == 0 and r.n_records == pin["n_records"]
    assert r.n_conflicts == pin["conflicts_by_dropped"][str(dropped)]
    assert r.n_pairs == -1          # pairs are defined without warp barriers only
    if dropped == 0:
        w, wp = r.witnesses[0], pin["witness_dropped_0"]
        assert _loc(w) == wp["loc"] and _side(w.first) == wp["first"] and _side(w.second) == wp["second"]


def test_warp_exchange():
    pin = PINS["warp_exchange"]
    assert oracle.check(K.warp_exchange(BARRIER_BLOCK)).n_conflicts == pin["conflicts"]["block_barrier"]
    assert oracle.check(K.warp_exchange(BARRIER_WARP, warp=64)).n_conflicts == pin["conflicts"]["warp_barrier_w64"]
    r = oracle.check(K.warp_exchange(BARRIER_WARP, warp=32))
    assert r.n_conflicts == pin["conflicts"]["warp_barrier_w32"]
    w, wp = r.witnesses[0], pin["witness_warp_barrier_w32"]
    assert _loc(w) == wp["loc"] and _side(w.first) == wp["first"] and _side(w.second) == wp["second"]


def test_warp_barriers_change_nothing_without_them():
    # a kernel without warp barriers gives the same result whatever the warp size
    d = K.tree_reduction(3, block=64, grid=2)
    ref = oracle.check(d)
    for ws in (1, 4, 32, 64):
        r = oracle.check(d.replace(warp_size=ws))
        assert (r.n_records, r.n_conflicts, r.n_pairs) == (ref.n_records, ref.n_conflicts, ref.n_pairs)
        assert [(_loc(a), _side(a.first), _side(a.second)) for a in r.witnesses] == \
            [(_loc(a), _side(a.first), _side(a.second)) for a in ref.witnesses]


# -------------------------------------------------------------- strict
def test_cross_block_global():
    pin = PINS["cross_block_global"]
    d = K.cross_block_global()
    assert oracle.check(d).n_conflicts == pin["conflicts"]["interval"]
    r = oracle.check(d, strict=True)
    assert r.status == 0 and r.n_conflicts == pin["conflicts"]["strict"]
    w, wp = r.witnesses[0], pin["witness_strict"]
    assert w.interval == wp["interval"] and [w.space, w.array, w.address] == wp["loc"]
    assert _side(w.first) == wp["first"] and _side(w.second) == wp["second"]


@pytest.mark.parametrize("drop", [-1, 3, 7])
def test_strict_matmul_adds_nothing(drop):
    # the tiled matmul's global arrays are read-only except C, written once by
    # its own thread: strict semantics find the per-interval shared conflicts
    d = K.tiled_matmul(grid=2, k_iters=4, drop_dynamic=drop)
    a, b = oracle.check(d), oracle.check(d, strict=True)
    assert (a.n_records, a.n_conflicts) == (b.n_records, b.n_conflicts)
    assert a.n_conflicts == (2048 * 4 if 0 <= drop < 7 else 0)


def test_strict_refuses_warp_barriers():
    assert oracle.check(K.warp_exchange(BARRIER_WARP), strict=True).status == -2


# ------------------------------------------------------------- ordered
@pytest.mark.parametrize("full", [False, True])
def test_polynomial_product_ordered(full):
    pin = PINS["polynomial_product"]
    n = pin["n"]
    d = K.polynomial_product_full(n) if full else K.polynomial_product(n)
    r = oracle.ordered(d)
    want = pin["with_S" if full else "T_only"]
    assert r.status == 0
    assert (r.n_raw, r.n_waw, r.n_war, r.n_dep_locations) == \
        (want["n_raw"], want["n_waw"], want["n_war"], want["n_dep_locations"])
    if full:
        assert r.n_records == want["n_records"]
    # closed forms in n
    s = 2 * (n * (n - 1) * (n - 2) // 6) + n * (n - 1) // 2
    assert r.n_war == s and r.n_raw == s + (n * n if full else 0)


# ---------------------------------------------------------- divergence
@pytest.mark.parametrize("case", ["block-half", "warp-tail", "block-uniform", "k-uniform"])
def test_guarded_barriers(case):
    pin = PINS["guarded_barrier"][case]
    r = oracle.divergence(K.guarded_barrier(case))
    assert r.status == 0 and (r.n_instances, r.n_divergent) == (pin["n_instances"], pin["n_divergent"])
    if "first" in pin:
        assert [r.dphase, r.block, r.warp, r.arrive_tid, r.skip_tid] == pin["first"]


# -------------------------------------------------------- brute force
def _brute_compare(desc, strict=False):
    n, confl = brute_check(desc, strict=strict)
    r = oracle.check(desc, max_witnesses=1 << 14, strict=strict)
    assert r.status == 0, (desc.name, r.status)
    assert r.n_records == n
    assert r.n_conflicts == len(confl)
    tpb = desc.block[0] * desc.block[1]
    for w, (loc, first, second, _) in zip(r.witnesses, confl):
        assert tuple(_loc(w)) == loc, desc.name
        for s, rec in ((w.first, first), (w.second, second)):
            thread, dyn, acc, _li = rec[5]
            assert (s.block * tpb + s.tid, s.dphase, s.access, s.loop, s.is_write) == \
                (thread, dyn, acc, rec[8], rec[7]), desc.name


def _scoped(seed, count):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    while len(out) < count:
        d = rand_scoped(rng, len(out))
        if oracle.check(d, max_witnesses=1).status == 0:      # skip out-of-bounds draws
            out.append(d)
    return out


def _small(seed, count):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    while len(out) < count:
        d = rand_small(rng, len(out))
        if oracle.check(d, max_witnesses=1).status == 0:
            out.append(d)
    return out


@pytest.mark.parametrize("seed", range(4))
def test_brute_warp_scopes(seed):
    ds = _scoped(600 + seed, 40)
    assert any(any(int(p.barrier_after) == 2 for p in d.phases) for d in ds)
    for d in ds:
        _brute_compare(d)


@pytest.mark.parametrize("seed", range(4))
def test_brute_strict(seed):
    # warps of 1-4 threads: a block holds several warps, and strict mode must
    # order records of one block (not of one warp) across intervals
    rng = np.random.Generator(np.random.PCG64(750 + seed))
    for d in _small(700 + seed, 40):
        _brute_compare(d.replace(warp_size=int(rng.integers(1, 5))), strict=True)


@pytest.mark.parametrize("seed", range(3))
def test_brute_ordered(seed):
    for d in _small(800 + seed, 25) + _scoped(850 + seed, 15):
        r = oracle.ordered(d)
        assert r.status == 0
        assert (r.n_records, r.n_raw, r.n_waw, r.n_war, r.n_dep_locations) == brute_ordered(d), d.name


@pytest.mark.parametrize("seed", range(3))
def test_brute_divergence(seed):
    for d in _scoped(900 + seed, 40):
        r = oracle.divergence(d)
        n, nd, first = brute_divergence(d)
        assert (r.status, r.n_instances, r.n_divergent) == (0, n, nd), d.name
        if nd:
            assert (r.dphase, r.block, r.warp, r.arrive_tid, r.skip_tid) == first, d.name
