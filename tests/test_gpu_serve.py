"""Served check: each job's result in the mix equals its result alone, and
both equal the oracle's.

A server over a small budget receives a seeded mix of kernels (random affine
jobs of the served workload's shape, one of about 1e7 records -- the top of
the served size range -- the pin kernels, a kernel whose index leaves its
array and an empty kernel) and every polled result is compared with rv_check
of the same kernel on a plain context, field by field, and with the oracle.
While the server runs, another thread loads kernels on the same context."""

import sys
import threading
import time

import pytest

import oracle
from workloads import kernels as K
from workloads import random_affine as RA
from workloads.desc import GLOBAL, SHARED, Builder, aff, rw

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _owkey(w):
    return (w.interval, w.space, w.block, w.array, w.address,
            (w.first.block, w.first.tid, w.first.dphase, w.first.access, tuple(w.first.loop), w.first.is_write),
            (w.second.block, w.second.tid, w.second.dphase, w.second.access, tuple(w.second.loop),
             w.second.is_write))


def _wkey(w):
    return None if w is None else (
        w.interval, w.space, w.block, w.array, w.address,
        (w.first.block, w.first.tid, w.first.dphase, w.first.access, tuple(w.first.loop), w.first.is_write),
        (w.second.block, w.second.tid, w.second.dphase, w.second.access, tuple(w.second.loop),
         w.second.is_write))


def _oob_kernel():
    b = Builder((8, 1), (2, 1), "oob")
    s = b.array(SHARED, (8,))
    p0 = b.phase([rw(s, True, aff(tx=1))], True)
    p1 = b.phase([rw(s, False, aff(5, tx=1))], False)
    b.segment([p0, p1])
    return b.build()


def _empty_kernel():
    b = Builder((4, 1), (1, 1), "empty")
    b.array(GLOBAL, (4,))
    return b.build()


def _mix():
    descs = list(RA.serving_stream(seed=5, count=40, lo=1e3, hi=2e6))
    descs += list(RA.serving_stream(seed=55, count=1, lo=9e6, hi=1e7))
    descs += [K.tiny_fixed(), K.tree_reduction(2), K.tiled_matmul(grid=2, k_iters=4, drop_dynamic=3),
              K.gespmm_crc(middle_barrier=False), _oob_kernel(), _empty_kernel(), K.polynomial_product(48)]
    return descs


@pytest.mark.parametrize("max_batch_records", [0, 100_000])
def test_served_equals_alone(max_batch_records):
    import paper_2503_08946_amd as rv
    descs = _mix()
    ctx = rv.Context(0, workspace_bytes=256 << 20)
    ks = [ctx.load(d) for d in descs]
    alone = []
    for d, k in zip(descs, ks):
        try:
            alone.append((0, ctx.check(k)))
        except rv.RVError as e:
            alone.append((e.status, None))
    say(f"[serve] {len(descs)} jobs checked alone")
    assert max(d.instances_upper_bound() for d in descs) >= 9_000_000
    for d, (st, ref) in zip(descs, alone):
        o = oracle.check(d, max_witnesses=1)
        say(f"[serve] oracle {d.name}: status {o.status} records {o.n_records}")
        assert st == o.status
        if st == 0:
            assert (ref.n_records, ref.n_conflicts) == (o.n_records, o.n_conflicts)
            assert _wkey(ref.witness) == (_owkey(o.witnesses[0]) if o.n_conflicts else None)
    srv = rv.Server(ctx, budget_bytes=256 << 20, max_batch_records=max_batch_records)
    # a second host thread loads (and frees) kernels on the serving context
    # while jobs run, the out-of-bounds one included
    loads = []

    def loader():
        for d in [K.tiny_fixed(), _oob_kernel(), K.tree_reduction(1)] * 3:
            kk = ctx.load(d)
            loads.append(kk.info().n_instances)
            kk.free()

    th = threading.Thread(target=loader)
    th.start()
    # submit in three waves with pauses so batches form at different points
    ids = {}
    order = list(range(len(ks))) + list(range(0, len(ks), 3))   # some kernels twice
    for n, j in enumerate(order):
        ids[srv.submit(ks[j])] = j
        if n % 17 == 16:
            time.sleep(0.002)
    th.join()
    assert len(loads) == 9
    srv.drain(120000)
    got = srv.poll(cap=4096)
    assert len(got) == len(order)
    assert sorted(r.job_id for r in got) == sorted(ids)
    for r in got:
        j = ids[r.job_id]
        st, ref = alone[j]
        say(f"[serve] job {r.job_id} kernel {descs[j].name} status {r.status}")
        assert r.status == st
        assert r.t_submit_ns <= r.t_start_ns <= r.t_done_ns
        if st == 0:
            assert (r.result.n_records, r.result.n_conflicts) == (ref.n_records, ref.n_conflicts)
            assert _wkey(r.result.witness) == _wkey(ref.witness)
    assert alone[-3][0] == -5          # the out-of-bounds kernel fails in the mix as alone
    st = srv.stats()
    say(f"[serve] {st}")
    assert st["jobs"] == len(order)
    if max_batch_records:
        assert st["batches"] > 3
    srv.close()
    # the context works normally again once the server is gone
    r = ctx.check(ks[0])
    assert r.n_records == alone[0][1].n_records
    ctx.close()


def test_server_budget_and_state():
    import paper_2503_08946_amd as rv
    ctx = rv.Context(0, workspace_bytes=256 << 20)
    big = ctx.load(K.tiled_matmul(grid=12, k_iters=2))       # compute intervals of about 9.6M records
    assert big.info().max_interval_instances > 8_000_000
    small = ctx.load(K.tiny_fixed())
    srv = rv.Server(ctx, budget_bytes=128 << 20)
    with pytest.raises(rv.RVError) as e:
        srv.submit(big)                                       # a 64 MiB lane holds < 8M records
    assert e.value.status == -7
    with pytest.raises(rv.RVError) as e:
        ctx.check(small)                                      # the context is serving
    assert e.value.status == -9
    jid = srv.submit(small)
    srv.drain(60000)
    (r,) = srv.poll()
    assert r.job_id == jid and r.status == 0 and r.result.n_conflicts == 62
    srv.close()
    ctx.close()
