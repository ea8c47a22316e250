"""Pins of the oracle's record enumeration and of its interval window, CPU only.

``oracle.records(desc, iv)`` is the reference of every expansion-parity test
on the GPU, and ``oracle.check(desc, ilo=, ihi=)`` (a window of intervals) is
what the full-size GPU tests and the CPU baseline run.  Both are compared
here with things other than themselves:

* records, field by field, against ``brute.simulate`` -- an independent
  thread-by-thread interpreter of the description (Section 2.1, steps 3-4:
  the access relations restricted to the Domain, applied instance by
  instance), on every interval of random kernels covering every description
  feature, of the closed-form kernels and of the linear-item kernels;
* a window of intervals against the whole check: the windows of a partition
  of the intervals add up to the whole result (counts, pairs) and their
  witness lists concatenate to the whole list, because a conflict never
  spans two intervals (two accesses separated by a barrier are ordered).
"""

import numpy as np
import pytest

import oracle
from brute import simulate
from cases import linear_case, rand_small
from workloads import kernels as K
from workloads import random_affine as RA


def _brute_records(desc):
    """Per interval: the simulated records as rows of oracle.RECORD_COLUMNS."""
    out = {}
    for r in simulate(desc):
        interval, space, blk, array, address, (thread, dyn, acc, li), _thr, is_write, loops, _fine = r
        out.setdefault(interval, []).append(
            (interval, space, blk, array, address, thread, dyn, acc, li) + tuple(loops) + (is_write,))
    return out


def _compare_records(desc):
    ref = _brute_records(desc)
    n_iv = oracle.n_intervals(desc)
    assert set(ref) <= set(range(n_iv))
    total = 0
    for iv in range(n_iv):
        got = oracle.records(desc, iv)
        assert got.shape[1] == len(oracle.RECORD_COLUMNS)
        want = sorted(ref.get(iv, []))
        have = sorted(tuple(int(x) for x in row) for row in got)
        assert have == want, (desc.name, iv)
        # the oracle lists an interval's records in instance-id order
        ids = [tuple(row[5:9]) for row in got.tolist()]
        assert ids == sorted(ids)
        total += len(have)
    assert total == oracle.check(desc, max_witnesses=1).n_records


@pytest.mark.parametrize("seed", range(4))
def test_records_match_simulation_random(seed):
    rng = np.random.Generator(np.random.PCG64(2000 + seed))
    for i in range(30):
        _compare_records(rand_small(rng, i))


@pytest.mark.parametrize("desc", [K.tiny_fixed(), K.stride1_shared(), K.stride1_global(),
                                  K.half_index_shared(block=16, grid=3), K.half_index_global(block=16, grid=3),
                                  K.tree_reduction(2, block=64, grid=2, levels=6),
                                  K.tiled_matmul(grid=1, k_iters=2, drop_dynamic=1),
                                  K.polynomial_product(16), K.gespmm_crc(M=2, N=32, T=2, K=2)],
                         ids=lambda d: d.name)
def test_records_match_simulation_fixed(desc):
    _compare_records(desc)


@pytest.mark.parametrize("name", ["partial-chunk", "descending", "two-loops", "stride-buckets",
                                  "flat-few-threads", "pass-boundary", "thread-linear"])
def test_records_match_simulation_linear_cases(name):
    _compare_records(linear_case(name))


def test_records_match_simulation_batch_shapes():
    rng = np.random.Generator(np.random.PCG64(31))
    n = 0
    while n < 4:
        desc = RA.random_kernel(rng, 300, 3000, name=f"bs-{n}")
        if desc.instances_upper_bound() <= 20000:
            _compare_records(desc)
            n += 1


def _wkeys(res):
    return [(w.key(), w.first, w.second) for w in res.witnesses]


def _window_kernels():
    rng = np.random.Generator(np.random.PCG64(77))
    ds = [rand_small(rng, i) for i in range(40)]
    ds = [d for d in ds if oracle.n_intervals(d) >= 2]
    ds += [K.tree_reduction(k, block=64, grid=2, levels=6) for k in (-1, 0, 3)]
    ds += [K.tiled_matmul(grid=1, k_iters=3, drop_dynamic=d) for d in (-1, 0, 3)]
    ds += [K.gespmm_crc(M=2, N=32, T=3, K=2, middle_barrier=False)]
    return ds


@pytest.mark.parametrize("desc", _window_kernels(), ids=lambda d: d.name)
def test_interval_windows_partition_the_check(desc):
    full = oracle.check(desc)
    n_iv = oracle.n_intervals(desc)
    assert full.status == 0 and full.n_intervals == n_iv
    # one interval at a time
    parts = [oracle.check(desc, ilo=iv, ihi=iv + 1) for iv in range(n_iv)]
    assert sum(p.n_records for p in parts) == full.n_records
    assert sum(p.n_conflicts for p in parts) == full.n_conflicts
    assert sum(p.n_pairs for p in parts) == full.n_pairs
    assert [w for p in parts for w in _wkeys(p)] == _wkeys(full)
    for iv, p in enumerate(parts):
        assert all(w.interval == iv for w in p.witnesses)
        # the window's records are exactly the interval's records
        assert p.n_records == len(oracle.records(desc, iv))
    # a partition into two windows, and windows clipped at both ends
    cut = n_iv // 2
    a, b = oracle.check(desc, ilo=-5, ihi=cut), oracle.check(desc, ilo=cut, ihi=n_iv + 7)
    assert (a.n_records + b.n_records, a.n_conflicts + b.n_conflicts) == (full.n_records, full.n_conflicts)
    assert _wkeys(a) + _wkeys(b) == _wkeys(full)
    # an empty window
    e = oracle.check(desc, ilo=n_iv, ihi=n_iv + 3)
    assert (e.n_records, e.n_conflicts, e.witnesses) == (0, 0, [])


# ----------------------------------------------------- exact int64 arithmetic
def _big_kernel(coef, c0, kind, d, nterms, lo):
    """One write per thread of g[aux0], aux0 = emod or floordiv of
    c0 + coef * (l0 + ... ), every loop a single point at lo."""
    from workloads.desc import AUX_EMOD, AUX_FLOORDIV, GLOBAL, Aux, Builder, aff, rw
    b = Builder((2, 1), (1, 1), f"big-{kind}-{nterms}")
    g = b.array(GLOBAL, (1_000_003,))
    e = aff(c0, **{f"l{j}": coef for j in range(nterms)})
    loops = tuple((lo, lo + 1) for _ in range(nterms))
    kindc = {"emod": AUX_EMOD, "floordiv": AUX_FLOORDIV}[kind]
    p = b.phase([rw(g, True, aff(aux0=1), loops=loops, aux=(Aux(kindc, d, e), Aux()))], False)
    b.segment([p])
    return b.build()


@pytest.mark.parametrize("coef,c0,lo", [((1 << 31) - 1, (1 << 31) - 1, (1 << 31) - 2),
                                        (-(1 << 31), -(1 << 31), (1 << 31) - 1),
                                        (-(1 << 31), 12345, -(1 << 31) + 1)])
def test_large_values_are_exact(coef, c0, lo):
    # two products of about 2^62 each: the sum fits int64 and the Euclidean
    # remainder of it must be Python's exact one (the brute force)
    desc = _big_kernel(coef, c0, "emod", 1_000_003, 2, lo)
    exact = coef * lo * 2 + c0
    assert -(1 << 63) <= exact < (1 << 63)
    _compare_records(desc)
    recs = oracle.records(desc, 0)
    assert sorted(int(a) for a in recs[:, 4]) == [exact % 1_000_003] * 2


def test_large_floor_division_is_exact():
    desc = _big_kernel(-(1 << 31), 7, "floordiv", 1 << 40, 2, (1 << 31) - 1)
    # floor((-2^32 (2^31 - 1) + 7) / 2^40) = -2^23 + ... is out of bounds for an
    # index; the brute force and the oracle must both call it that instance
    exact = (-(1 << 31) * ((1 << 31) - 1) * 2 + 7) // (1 << 40)
    assert exact < 0
    r = oracle.check(desc)
    assert r.status == -5 and r.oob == (0, 0, 0, 0, 0)
    with pytest.raises(IndexError):
        list(simulate(desc))


def test_int64_overflow_is_reported():
    # three products of about 2^62: the exact sum leaves int64
    coef, lo = (1 << 31) - 1, (1 << 31) - 2
    desc = _big_kernel(coef, 0, "emod", 7, 3, lo)
    assert 3 * coef * lo >= (1 << 63)
    r = oracle.check(desc)
    assert r.status == -4
    assert r.oob == (0, 0, 0, 0, 0)       # the very first instance
