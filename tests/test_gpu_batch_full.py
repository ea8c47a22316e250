"""The whole batched workload against the oracle: all 4096 random affine
kernels (seed 4, records log-uniform in [1e2, 1e6], 432,085,651 records),
checked in one rv_check_batch in the launch configuration bench.py times
(16 GiB workspace, default planner settings), and each kernel's record
count, conflict count and first witness compared with the oracle's.  The
oracle runs on the host in a pool of threads (its C code holds no global
state; ctypes releases the interpreter lock during the call)."""

import os
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

import oracle
from workloads import random_affine as RA

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _okey(w):
    return (w.interval, w.space, w.block, w.array, w.address,
            (w.first.block, w.first.tid, w.first.dphase, w.first.access, tuple(w.first.loop), w.first.is_write),
            (w.second.block, w.second.tid, w.second.dphase, w.second.access, tuple(w.second.loop),
             w.second.is_write))


def test_batched_workload_all_kernels():
    import paper_2503_08946_amd as rv
    descs = RA.batch_kernels(seed=4, count=4096)
    say("[batch-full] generated 4096 kernels")
    ctx = rv.Context(0, workspace_bytes=16 << 30)
    ks = [ctx.load(d) for d in descs]
    res = ctx.check_batch(ks)
    say(f"[batch-full] GPU: {sum(r.n_records for r in res)} records, "
        f"{sum(1 for r in res if r.n_conflicts)} kernels with conflicts")
    workers = max(1, min(16, (os.cpu_count() or 1)))
    with ThreadPoolExecutor(workers) as ex:
        ref = list(ex.map(lambda d: oracle.check(d, max_witnesses=1), descs))
    say(f"[batch-full] oracle done ({workers} threads)")
    assert sum(r.n_records for r in ref) == 432_085_651
    for d, r, o in zip(descs, res, ref):
        assert o.status == 0, d.name
        assert (r.n_records, r.n_conflicts) == (o.n_records, o.n_conflicts), d.name
        if o.n_conflicts:
            assert r.witness is not None and _okey(r.witness) == _okey(o.witnesses[0]), d.name
        else:
            assert r.witness is None, d.name
    ctx.close()
