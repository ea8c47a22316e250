"""GPU parity of the general expansion (aux terms, guards) at its edges.

The general path divides each aux numerator once per thread of a work item
and then steps it with the loop: the change of the numerator for the inner,
middle and outer loop's step is split as q * d + r on the host, and each
point adds r to n mod d with one carry.  These descriptions aim at that
stepping: three loops whose inner two wrap inside a work item, divisors of
1 and of 2^16 (steps of many multiples), floor division of negative
numerators, both aux terms in one index, guards on aux terms, and an index
that leaves its array.  Each runs with few threads (lanes of a work item
take loop chunks of a handful of threads) and with many (lanes take
threads), under both grouping kernels; counts, the full witness list,
record multisets and the first out-of-bounds instance must equal the
oracle's."""

import sys

import pytest

import oracle
from test_gpu_fuzz import _fuzz_one
from workloads.desc import AUX_EMOD, AUX_FLOORDIV, GLOBAL, SHARED, Aux, Builder, aff, rw

pytestmark = pytest.mark.gpu

LOOPS = ((0, 3), (-2, 2), (0, 6))     # l1 runs over negative values; the inner loop wraps inside a chunk


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=["fold", "sort_scan"])
def ctx(request):
    import paper_2503_08946_amd as rv
    c = rv.Context(0, workspace_bytes=1 << 30)
    c.group = request.param
    yield c
    c.close()


def _case(name, shape, space, dims, idx, aux, guards=()):
    """Phase 0 writes the array through the general index under test; phase
    1 (same barrier interval) reads it through a plain Euclidean remainder,
    so the locations the writes reach conflict."""
    block, grid = shape
    b = Builder(block, grid, f"{name}-{block[0]}x{block[1]}-{grid[0]}x{grid[1]}")
    a = b.array(space, dims, "a")
    aux = tuple(aux) + (Aux(),) * (2 - len(aux))
    wr = rw(a, True, *idx, loops=LOOPS, aux=aux, guards=guards)
    rd_aux = tuple(Aux(AUX_EMOD, d, aff(j, tx=1 + j, ty=2, l0=3, l2=1)) for j, d in enumerate(dims[:2]))
    rd_aux = rd_aux + (Aux(),) * (2 - len(rd_aux))
    rd_idx = (aff(aux0=1), aff(aux1=1))[:len(dims)]
    rd = rw(a, False, *rd_idx, loops=((0, 2), (0, 5)), aux=rd_aux)
    b.segment([b.phase([wr], False), b.phase([rd], False)])
    return b.build()


SHAPES = [((3, 1), (1, 1)), ((32, 4), (3, 2))]

CASES = {
    # d = 1: the remainder is always 0, the quotient is the numerator itself
    "divisor-1": dict(space=GLOBAL, dims=(2, 128),
                      idx=(aff(aux0=1), aff(50, aux1=1)),
                      aux=(Aux(AUX_EMOD, 1, aff(tx=1, l0=3, l1=-2, l2=1)),
                           Aux(AUX_FLOORDIV, 1, aff(ty=1, l1=5, l2=-7)))),
    # floor division of negative numerators
    "negative-floor": dict(space=SHARED, dims=(32,),
                           idx=(aff(10, aux0=1),),
                           aux=(Aux(AUX_FLOORDIV, 7, aff(-20, tx=1, l0=2, l1=-3, l2=-1)),)),
    # steps of many multiples of a large divisor, quotient and remainder both used
    "large-divisor": dict(space=GLOBAL, dims=(16, 65536),
                          idx=(aff(2, aux0=1), aff(aux1=1)),
                          aux=(Aux(AUX_FLOORDIV, 65536, aff(tx=3, bx=7, l0=4096, l1=300, l2=50000)),
                               Aux(AUX_EMOD, 65536, aff(tx=17, l1=-1000, l2=-50000)))),
    # both aux terms in one index, plus loop terms
    "two-aux-one-index": dict(space=SHARED, dims=(256,),
                              idx=(aff(100, aux0=3, aux1=-2, l2=1),),
                              aux=(Aux(AUX_EMOD, 13, aff(tx=1, l0=3, l1=5, l2=-2)),
                                   Aux(AUX_FLOORDIV, 3, aff(-1, tx=-1, l1=1, l2=7)))),
    # guards on aux terms and loops (the per-record guard path)
    "guards-on-aux": dict(space=GLOBAL, dims=(13, 40),
                          idx=(aff(aux0=1), aff(15, aux1=1)),
                          aux=(Aux(AUX_EMOD, 13, aff(tx=1, l0=3, l1=5, l2=-2)),
                               Aux(AUX_FLOORDIV, 3, aff(-1, tx=-1, l1=1, l2=7))),
                          guards=(aff(-4, aux0=1), aff(l1=1, l0=-1))),
    # an index below 0 when the remainder is 0: out of bounds
    "out-of-bounds": dict(space=SHARED, dims=(8,),
                          idx=(aff(-1, aux0=1),),
                          aux=(Aux(AUX_EMOD, 8, aff(5, tx=1, l1=3, l2=1)),)),
}


@pytest.mark.parametrize("shape", SHAPES, ids=["few-threads", "many-threads"])
@pytest.mark.parametrize("name", list(CASES))
def test_general_stepping(ctx, name, shape):
    desc = _case(name, shape, **CASES[name])
    o = oracle.check(desc, max_witnesses=1)
    assert o.status == (-5 if name == "out-of-bounds" else 0)
    assert o.n_records > 0 or o.status == -5
    _fuzz_one(ctx, desc)
