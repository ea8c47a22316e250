"""Host-only checks of the C ABI: the library loads, exports every function
declared in include/rv.h, its integer helpers pass their self test and the
host validator returns the documented codes.  No compute call needs a GPU."""

import ctypes
import os
import re

import pytest

import paper_2503_08946_amd as rv
from workloads import kernels as K
from workloads import random_affine as RA
from cases import large_grid
from workloads.desc import AUX_EMOD, AUX_FLOORDIV, GLOBAL, SHARED, Aux, Builder, aff, rw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:rv_status|const char \*)\s*(rv_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_function():
    lib = rv.lib()
    declared = _declared()
    assert len(declared) >= 14
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(rv.EXPORTED) == declared


def test_host_selftest():
    st, msg = rv.selftest()
    assert st == 0, msg


@pytest.mark.parametrize("desc", [K.tiny_fixed(), K.tree_reduction(3), K.tiled_matmul(16, 64, 5),
                                  K.polynomial_product(), K.gespmm_crc(), K.half_index_global()],
                         ids=lambda d: d.name)
def test_validate_ok(desc):
    assert rv.validate(desc) == (0, "")


def test_validate_batch_kernels_ok():
    for d in RA.batch_kernels(seed=4, count=64):
        assert rv.validate(d)[0] == 0, d.name


def _one(access, arrays=((SHARED, (8,)),), block=(8, 1), grid=(1, 1)):
    b = Builder(block, grid)
    for sp, dims in arrays:
        b.array(sp, dims)
    p = b.phase([access], False)
    b.segment([p])
    return b.build()


def test_validate_errors():
    ok = _one(rw(0, True, aff(tx=1)))
    assert rv.validate(ok)[0] == 0
    # bad array index
    assert rv.validate(_one(rw(3, True, aff(tx=1))))[0] == -1
    # aux divisor < 1
    assert rv.validate(_one(rw(0, True, aff(aux0=1), aux=(Aux(AUX_FLOORDIV, 0, aff(tx=1)), Aux()))))[0] == -1
    # aux numerator uses an aux variable
    assert rv.validate(_one(rw(0, True, aff(aux0=1), aux=(Aux(AUX_EMOD, 4, aff(aux1=1)), Aux()))))[0] == -1
    # loop lo > hi
    assert rv.validate(_one(rw(0, True, aff(tx=1), loops=((3, 1),))))[0] == -1
    # value range: coefficient * tid may leave int32
    st, msg = rv.validate(_one(rw(0, True, aff(tx=1 << 29)), block=(8, 1)))
    assert st == -4, msg
    # location space beyond 31 bits
    st, _ = rv.validate(_one(rw(0, True, aff(tx=1)), arrays=((GLOBAL, (1 << 30,)), (GLOBAL, (1 << 30,))),
                              block=(8, 1)).replace(
        accesses=[rw(0, True, aff(tx=1)), rw(1, True, aff(tx=1))],
        phases=[__import__("workloads").Phase(0, 2, False)]))
    assert st == -3
    # too many instances in one interval
    big = _one(rw(0, False, aff(0), loops=((0, 1 << 16), (0, 1 << 10))), block=(32, 32), grid=(4, 1))
    assert rv.validate(big)[0] == -6
    # empty description is valid (no records)
    empty = Builder((1, 1), (1, 1)).build()
    assert rv.validate(empty)[0] == 0


def test_validate_z_dimension_unsupported():
    m = rv.Marshalled(K.tiny_fixed())
    m.desc.launch.block[2] = 2
    buf = ctypes.create_string_buffer(256)
    assert rv.lib().rv_validate_desc(ctypes.byref(m.desc), buf, 256) == -2
    m.desc.launch.block[2] = 0
    assert rv.lib().rv_validate_desc(ctypes.byref(m.desc), buf, 256) == -1


def test_context_needs_gpu_or_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        rv.Context(0, 64 << 20)


def test_plan_flags_large_grid():
    # in bounds: the index bx + 2^23 - 64 stays below 2^24 over the whole grid,
    # so the entry is proven (no per-record bounds test)
    ok = rv.plan(large_grid((1 << 23) - 64, 1 << 24))
    assert (ok.n_entries, ok.n_fast_entries, ok.n_proven_entries) == (1, 1, 1)
    # out of bounds from block 2^23 on: the entry stays on the fast path with
    # a per-record bounds test, whose index arithmetic must be exact for
    # block ids up to 2^23 + 63 (a 24-bit product would wrap 2^23 to -2^23)
    bad = rv.plan(large_grid(1 << 23, 1 << 24))
    assert (bad.n_entries, bad.n_fast_entries, bad.n_proven_entries) == (1, 1, 0)
    assert bad.n_instances == (1 << 23) + 64


def test_plan_matches_validate_errors():
    big = _one(rw(0, False, aff(0), loops=((0, 1 << 16), (0, 1 << 10))), block=(32, 32), grid=(4, 1))
    with pytest.raises(rv.RVError) as e:
        rv.plan(big)
    assert e.value.status == rv.validate(big)[0] == -6
    info = rv.plan(K.tiled_matmul(grid=16, k_iters=64, drop_dynamic=64))
    assert info.n_instances == 1_141_112_832 and info.n_intervals == 128
    assert info.n_chunks == 0 and info.n_fast_entries == info.n_proven_entries == info.n_entries


@pytest.mark.parametrize("size", list(K.GESPMM_SWEEP), ids=lambda s: "M%d-N%d-T%d-K%d" % s)
def test_plan_gespmm_sweep_sizes(size):
    # every size the Ge-SpMM benchmark sweeps plans in all three variants,
    # with the hand-derived record count (no guards: instances = records)
    from cases import gespmm_closed_form
    M, N, T, Kb = size
    cf = gespmm_closed_form(M, N, T, Kb)
    for mid, trail in ((True, True), (False, True), (True, False)):
        info = rv.plan(K.gespmm_crc(M, N, T, Kb, middle_barrier=mid, trailing_barrier=trail, kb_on_all=False))
        assert info.n_instances == cf["records"]


def test_plan_warp_barriers_and_strict():
    from workloads.desc import BARRIER_WARP
    # warp barriers: one barrier interval, 5 fine intervals -> 3 sub-key bits
    info = rv.plan(K.warp_reduction(-1))
    assert info.n_intervals == 1 and info.n_instances == 128 * 5 * 3      # before the guards
    assert rv.validate(K.cross_block_global())[0] == 0
    # warp barriers are refused in strict mode only at load (a context is
    # needed), validation accepts them
    assert rv.validate(K.warp_exchange(BARRIER_WARP))[0] == 0
    # a barrier guard may not use loop variables
    d = K.guarded_barrier("block-half")
    bad = d.replace(phases=[d.phases[0].__class__(0, 1, 1, (aff(l0=1),)), d.phases[1]])
    assert rv.validate(bad)[0] == -1
    # a barrier kind outside 0..2
    bad = d.replace(phases=[d.phases[0].__class__(0, 1, 3), d.phases[1]])
    assert rv.validate(bad)[0] == -1


def test_plan_proves_aux_indices():
    """An entry with aux terms and no guards is proven in bounds from the
    value ranges of its variables and aux terms: n mod d lies in [0, d), and
    floor(n / d) between the quotients of the numerator's extremes."""
    def one(idx, aux, dim=64, guards=()):
        aux = tuple(aux) + (Aux(),) * (2 - len(aux))
        return _one(rw(0, True, idx, loops=((0, 8),), aux=aux, guards=guards), arrays=((SHARED, (dim,)),))
    emod = (Aux(AUX_EMOD, 64, aff(3, tx=5, l0=-7)),)
    assert rv.plan(one(aff(aux0=1), emod)).n_proven_entries == 1
    # s[aux0 + 1] reaches 64 when aux0 = 63
    assert rv.plan(one(aff(1, aux0=1), emod)).n_proven_entries == 0
    # a divisor above the dimension leaves the entry to the per-record test
    assert rv.plan(one(aff(aux0=1), (Aux(AUX_EMOD, 65, aff(tx=1)),))).n_proven_entries == 0
    # floor((tx + 8 l0) / 2) over tx in [0, 8), l0 in [0, 8): [0, 31]
    fl = (Aux(AUX_FLOORDIV, 2, aff(tx=1, l0=8)),)
    assert rv.plan(one(aff(aux0=1), fl, dim=32)).n_proven_entries == 1
    assert rv.plan(one(aff(aux0=1), fl, dim=31)).n_proven_entries == 0
    # guards keep the per-record path
    assert rv.plan(one(aff(aux0=1), emod, guards=(aff(tx=1),))).n_proven_entries == 0
    # the batched workload's kernels: every index is n mod dim of its dimension
    for d in RA.batch_kernels(count=8):
        info = rv.plan(d)
        assert info.n_fast_entries == 0 and info.n_proven_entries == info.n_entries
