"""The planner target (mean records per bucket) changes the bucket widths,
never the results: every target gives the oracle's counts and witnesses, and
the autotuner keeps one of its candidates."""

import json
import sys

import pytest

import oracle
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


def test_targets_give_identical_results():
    import paper_2503_08946_amd as rv
    descs = [K.tree_reduction(3), K.tiled_matmul(grid=2, k_iters=4, drop_dynamic=2), K.polynomial_product(64),
             K.gespmm_crc()] + RA.batch_kernels(seed=4, count=16)
    refs = [oracle.check(d, max_witnesses=1) for d in descs]
    ctx = rv.Context(0, workspace_bytes=256 << 20)
    for target in (64, 512, 2048, 4096):
        ctx.target = target
        assert ctx.target == target
        ks = [ctx.load(d) for d in descs]
        for group in ("fold", "sort_scan"):
            ctx.group = group
            for small in (0, 1000, 2048):
                ctx.small_cap = small
                res = ctx.check_batch(ks)
                for d, o, r in zip(descs, refs, res):
                    say(f"[target {target} {group} small {small}] {d.name}")
                    assert (r.n_records, r.n_conflicts) == (o.n_records, o.n_conflicts)
                    assert _wkey(r.witness) == (_wkey(o.witnesses[0]) if o.n_conflicts else None)
        for k in ks:
            k.free()
    with pytest.raises(rv.RVError):
        ctx.target = 5000
    with pytest.raises(rv.RVError):
        ctx.small_cap = 3000
    ctx.close()


def test_autotune_and_cache(tmp_path):
    import paper_2503_08946_amd as rv
    descs = RA.batch_kernels(seed=4, count=32)
    ctx = rv.Context(0, workspace_bytes=256 << 20)
    cache = str(tmp_path / "tune.json")
    rec = ctx.autotune(descs, trials=2, cache=cache)
    say(f"[autotune] {rec}")
    assert f"{rec['target']}/{rec['group']}/{rec['small_cap']}" in rec["ms"]
    assert len(rec["ms"]) == 8 and all(v > 0 for v in rec["ms"].values())
    assert ctx.target == rec["target"] and ctx.group == rec["group"] and ctx.small_cap == rec["small_cap"]
    db = json.load(open(cache))
    assert len(db) == 1
    ctx.target = 2048
    ctx.group = "sort_scan" if rec["group"] == "fold" else "fold"
    again = ctx.autotune(descs, trials=2, cache=cache)     # served from the cache
    assert again["target"] == rec["target"] and ctx.target == rec["target"] and ctx.group == rec["group"]
    ks = [ctx.load(d) for d in descs[:8]]
    for d, r in zip(descs[:8], ctx.check_batch(ks)):
        o = oracle.check(d, max_witnesses=1)
        assert (r.n_records, r.n_conflicts) == (o.n_records, o.n_conflicts)
    ctx.close()
