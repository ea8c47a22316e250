"""Pins of the CPU oracle: hand-derived closed forms (tests/golden) and an
O(N^2) brute force on small random kernels.  CPU only."""

import json
import os

import numpy as np
import pytest

import oracle
from brute import brute_check
from cases import rand_small
from workloads import kernels as K
from workloads import random_affine as RA
from workloads.desc import AUX_EMOD, AUX_FLOORDIV, GLOBAL, SHARED, Aux, Builder, aff, rw

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))
PINS = {p["name"]: p for p in GOLD["pins"]}


def _side(s):
    return [s.block, s.tid, s.dphase, s.access, list(s.loop), s.is_write]


def _loc(w):
    return [w.interval, w.space, w.block, w.array, w.address]


def _check_fixed(name):
    p = PINS[name]
    desc = getattr(K, p["builder"])(**p["args"])
    r = oracle.check(desc)
    assert r.status == 0
    assert r.n_records == p["n_records"]
    assert r.n_conflicts == p["n_conflicts"]
    assert r.n_pairs == p["pairs"]
    if "witness" in p:
        w = r.witnesses[0]
        assert _loc(w) == p["witness"]["loc"]
        assert _side(w.first) == p["witness"]["first"]
        assert _side(w.second) == p["witness"]["second"]


@pytest.mark.parametrize("name", ["stride1-shared", "stride1-global", "half-index-shared",
                                  "half-index-global", "tiny-fixed", "tree-reduction-correct",
                                  "polynomial-product", "matmul-correct"])
def test_fixed_pin(name):
    _check_fixed(name)


@pytest.mark.parametrize("k", range(10))
def test_tree_reduction_deleted_barrier(k):
    r = oracle.check(K.tree_reduction(k))
    expect = 128 * (256 >> k) if k <= 8 else 0
    assert r.n_records == PINS["tree-reduction-nobar-k"]["n_records"]
    assert r.n_conflicts == expect and r.n_pairs == expect
    if k <= 8:
        h2 = 256 >> k
        w = r.witnesses[0]
        assert _loc(w) == [k, 0, 0, 0, h2]
        assert _side(w.first) == [0, h2, k, 3 * k + 2, [0, 0, 0], 1]
        assert _side(w.second) == [0, 0, k + 1, 3 * (k + 1) + 1, [0, 0, 0], 0]
        # every witness: written by x in phase k, read by x - h/2 in phase k+1
        for w in r.witnesses[:50]:
            assert h2 <= w.address < 2 * h2
            assert w.first.tid == w.address and w.second.tid == w.address - h2


@pytest.mark.parametrize("d", range(8))
def test_matmul_drop_dynamic(d):
    desc = K.tiled_matmul(grid=2, k_iters=4, drop_dynamic=d)
    r = oracle.check(desc)
    assert r.n_records == 1118208
    expect = 2048 * 4 if d < 7 else 0
    assert r.n_conflicts == expect and r.n_pairs == 31 * expect
    if d < 7:
        w = r.witnesses[0]
        assert _loc(w) == [d, 0, 0, 3, 0]
        if d % 2 == 0:
            assert _side(w.first) == [0, 0, d, 2, [0, 0, 0], 1]
            assert _side(w.second) == [0, 31, d + 1, 4, [0, 0, 0], 0]
        else:
            assert _side(w.first) == [0, 0, d + 1, 2, [0, 0, 0], 1]
            assert _side(w.second) == [0, 31, d, 4, [0, 0, 0], 0]
        # all conflicts of the merged interval; As first, then Bs, per block
        assert {w.interval for w in r.witnesses} == {d}


@pytest.mark.parametrize("s,expect", [("load", 4 * 2048 * 4), ("compute", 3 * 2048 * 4)])
def test_matmul_drop_static(s, expect):
    r = oracle.check(K.tiled_matmul(grid=2, k_iters=4, drop_static=s))
    assert r.n_conflicts == expect and r.n_pairs == 31 * expect


@pytest.mark.parametrize("mid,trail,expect", [tuple(v) for v in PINS["gespmm-crc"]["variants"]])
def test_gespmm_crc(mid, trail, expect):
    desc = K.gespmm_crc(M=4, N=64, T=3, K=2, middle_barrier=mid, trailing_barrier=trail)
    r = oracle.check(desc)
    assert r.n_records == PINS["gespmm-crc"]["n_records"]
    assert r.n_conflicts == expect and r.n_pairs == 31 * expect
    if not mid and trail:
        w = r.witnesses[0]
        wp = PINS["gespmm-crc"]["witness_middle_dropped"]
        assert _loc(w) == wp["loc"] and _side(w.first) == wp["first"] and _side(w.second) == wp["second"]


@pytest.mark.parametrize("mid,trail,expect", [tuple(v) for v in PINS["gespmm-crc-b-only"]["variants"]])
def test_gespmm_crc_b_only(mid, trail, expect):
    pin = PINS["gespmm-crc-b-only"]
    desc = K.gespmm_crc(M=4, N=64, T=3, K=2, middle_barrier=mid, trailing_barrier=trail, kb_on_all=False)
    r = oracle.check(desc)
    assert r.n_records == pin["n_records"] == 4 * 64 * 3 * (4 + 32 * (4 + 2))
    assert r.n_conflicts == expect and r.n_pairs == 31 * expect
    if not mid and trail:
        w = r.witnesses[0]
        wp = pin["witness_middle_dropped"]
        assert _loc(w) == wp["loc"] and _side(w.first) == wp["first"] and _side(w.second) == wp["second"]


# ----------------------------------------------------------- brute force
def _brute_compare(desc):
    n, confl = brute_check(desc)
    r = oracle.check(desc, max_witnesses=1 << 14)
    assert r.status == 0
    assert r.n_records == n
    assert r.n_conflicts == len(confl)
    assert r.n_pairs == sum(c[3] for c in confl)
    for w, (loc, first, second, _) in zip(r.witnesses, confl):
        assert tuple(_loc(w)) == loc
        tpb = desc.block[0] * desc.block[1]
        for s, rec in ((w.first, first), (w.second, second)):
            thread, dyn, acc, _li = rec[5]
            assert (s.block * tpb + s.tid, s.dphase, s.access, s.loop, s.is_write) == \
                (thread, dyn, acc, rec[8], rec[7])


@pytest.mark.parametrize("seed", range(4))
def test_brute_tiny_random(seed):
    for desc in K.tiny_random(seed=100 + seed, count=8):
        _brute_compare(desc)


@pytest.mark.parametrize("seed", range(6))
def test_brute_random_features(seed):
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    for i in range(25):
        _brute_compare(rand_small(rng, i))


def test_brute_batch_like():
    # two of the batched workload's kernel shapes, shrunk to brute-force size
    rng = np.random.Generator(np.random.PCG64(77))
    for i in range(3):
        desc = RA.random_kernel(rng, 200, 600, name=f"bl-{i}")
        if desc.instances_upper_bound() <= 3000:
            _brute_compare(desc)


def test_oob_reports_smallest_instance():
    b = Builder((8, 1), (2, 1), "oob")
    s = b.array(SHARED, (8,))
    p0 = b.phase([rw(s, True, aff(tx=1))], barrier_after=True)
    # second phase: s[tx + 5] overflows for tx >= 3; smallest offender: block 0, tid 3
    p1 = b.phase([rw(s, False, aff(0, tx=1)), rw(s, False, aff(5, tx=1))], barrier_after=False)
    b.segment([p0, p1])
    r = oracle.check(b.build())
    assert r.status == -5
    assert r.oob == (1, 3, 1, 2, 0)


def test_pair_count_is_diagnostic_only():
    # two readers and one writer of one element: 1 location, 2 pairs
    b = Builder((3, 1), (1, 1), "pairs")
    s = b.array(SHARED, (1,))
    p = b.phase([rw(s, False, aff(0), guards=(aff(1, tx=-1),)),        # tid <= 1 read
                 rw(s, True, aff(0), guards=(aff(-2, tx=1),))], False)  # tid == 2 writes
    b.segment([p])
    r = oracle.check(b.build())
    assert r.n_conflicts == 1 and r.n_pairs == 2
