"""rv_check_static, the check that allocates nothing: its results equal
rv_check's (bit-exact, every field of rv_result) on two calls in a row, the
second with a smaller kernel, across chunks of the static scratch; kernels
larger than the scratch are refused with RV_ERR_TOO_LARGE, and an
out-of-bounds kernel fails as rv_check fails."""

import sys

import pytest

from workloads import kernels as K
from cases import large_grid

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same(a, b):
    assert (a.n_records, a.n_conflicts) == (b.n_records, b.n_conflicts)
    assert a.witness == b.witness


@pytest.fixture(scope="module")
def ctx():
    import paper_2503_08946_amd as rv
    c = rv.Context(0, workspace_bytes=1 << 30)
    yield c
    c.close()


def test_static_equals_check_larger_then_smaller(ctx):
    # several static chunks (7.2e7 records), then one chunk, then a tiny kernel
    for desc in (K.tiled_matmul(grid=4, k_iters=64, drop_dynamic=5), K.tree_reduction(3), K.tiny_fixed()):
        say(f"[no-alloc] {desc.name}")
        k = ctx.load(desc)
        try:
            ref = ctx.check(k)
            got = ctx.check_static(k)
            _same(got, ref)
            assert got.n_conflicts > 0
        finally:
            k.free()


def test_static_twice_same_kernel_then_smaller(ctx):
    big, small = K.tree_reduction(0), K.tree_reduction(8)
    kb, ks = ctx.load(big), ctx.load(small)
    try:
        rb, rs = ctx.check(kb), ctx.check(ks)
        say("[no-alloc] repeated calls")
        _same(ctx.check_static(kb), rb)
        _same(ctx.check_static(kb), rb)
        _same(ctx.check_static(ks), rs)
        assert (rb.n_conflicts, rs.n_conflicts) == (32768, 128)
    finally:
        kb.free()
        ks.free()


def test_static_refuses_kernels_beyond_scratch(ctx):
    import paper_2503_08946_amd as rv
    k = ctx.load(K.tiled_matmul(grid=16, k_iters=64, drop_dynamic=64))
    try:
        with pytest.raises(rv.RVError) as e:
            ctx.check_static(k)
        assert e.value.status == -6 and "static scratch" in e.value.message
    finally:
        k.free()


def test_static_out_of_bounds_as_check(ctx):
    import paper_2503_08946_amd as rv
    k = ctx.load(large_grid(1 << 23, 1 << 24))
    try:
        with pytest.raises(rv.RVError) as e1:
            ctx.check(k)
        with pytest.raises(rv.RVError) as e2:
            ctx.check_static(k)
        assert e1.value.status == e2.value.status == -5
        assert e1.value.message == e2.value.message
    finally:
        k.free()
