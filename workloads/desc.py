"""Kernel descriptions: the input both the checker and the oracle consume.

A description is pure data.  It models what the paper extracts from a GPU
kernel before building its integer-set model (Section 2, the component list:
thread/block ids, barriers, shared-memory allocations, array indices, reads
and writes; Section 2.1, the Domain / Read / Write / Schedule sets):

* ``arrays``    -- each array is ``shared`` (one copy per thread block) or
                   ``global`` (one copy for the launch), with 1-3 dimensions.
* ``accesses``  -- one read or write of one array per loop point.  Each
                   index is an affine form over the variables listed in
                   ``VARS``; loops are constant boxes ``[lo, hi)``; guards are
                   affine forms that must be ``>= 0`` (a conjunction).  Two
                   auxiliary variables may hold ``floor(e / d)`` or the
                   Euclidean ``e mod d`` of an affine ``e``.
* ``phases``    -- runs of accesses; ``barrier_after`` ends the phase with a
                   barrier: ``BARRIER_BLOCK`` (all threads of the block,
                   ``__syncthreads``) or ``BARRIER_WARP`` (the threads of one
                   warp, ``__syncwarp``; warps are ``warp_size`` consecutive
                   linear thread ids of a block).  ``barrier_guards`` (affine
                   forms over tx, ty, bx, by, k that must be ``>= 0``) say which
                   threads reach the barrier; the race check treats every
                   barrier as reached by all threads, the divergence check
                   reports barriers that only part of their scope reaches.
* ``segments``  -- runs of phases repeated ``repeat`` times; the variable
                   ``k`` holds ``k_base + r`` in repetition ``r``.

Nothing in this module evaluates a description: it only builds and stores
them.  The checker library and the oracle each read these fields with their
own code.
"""

from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

# Variable slots of an affine form, in the order of the C structure.
VARS = ("tx", "ty", "bx", "by", "k", "l0", "l1", "l2", "aux0", "aux1")
NV = len(VARS)
V_TX, V_TY, V_BX, V_BY, V_K, V_L0, V_L1, V_L2, V_AUX0, V_AUX1 = range(NV)

SHARED, GLOBAL = 0, 1
AUX_NONE, AUX_FLOORDIV, AUX_EMOD = 0, 1, 2
BARRIER_NONE, BARRIER_BLOCK, BARRIER_WARP = 0, 1, 2


def aff(c0: int = 0, **terms: int) -> Tuple[int, ...]:
    """Affine form ``c0 + sum(coef * var)`` as a tuple ``(coef[0..9], c0)``."""
    coef = [0] * NV
    for name, c in terms.items():
        coef[VARS.index(name)] = int(c)
    return tuple(coef) + (int(c0),)


def aff_from(coef: Sequence[int], c0: int) -> Tuple[int, ...]:
    coef = [int(c) for c in coef]
    assert len(coef) == NV
    return tuple(coef) + (int(c0),)


ZERO = aff()


@dataclass(frozen=True)
class Array:
    space: int                      # SHARED or GLOBAL
    dims: Tuple[int, ...]           # 1-3 extents, row-major
    name: str = ""


@dataclass(frozen=True)
class Aux:
    kind: int = AUX_NONE            # AUX_NONE / AUX_FLOORDIV / AUX_EMOD
    d: int = 1                      # divisor, >= 1
    e: Tuple[int, ...] = ZERO       # affine numerator; may not use aux0/aux1


@dataclass(frozen=True)
class Access:
    array: int
    is_write: bool
    idx: Tuple[Tuple[int, ...], ...]             # one affine row per array dim
    loops: Tuple[Tuple[int, int], ...] = ()      # up to 3 boxes [lo, hi) -> l0, l1, l2
    aux: Tuple[Aux, Aux] = (Aux(), Aux())
    guards: Tuple[Tuple[int, ...], ...] = ()     # each affine >= 0
    name: str = ""


@dataclass(frozen=True)
class Phase:
    access_begin: int
    access_count: int
    barrier_after: int                           # BARRIER_NONE / BARRIER_BLOCK / BARRIER_WARP (True = block)
    barrier_guards: Tuple[Tuple[int, ...], ...] = ()   # who reaches the barrier: each affine >= 0


@dataclass(frozen=True)
class Segment:
    phase_begin: int
    phase_count: int
    repeat: int = 1
    k_base: int = 0


@dataclass
class KernelDesc:
    block: Tuple[int, int]
    grid: Tuple[int, int]
    arrays: List[Array]
    accesses: List[Access]
    phases: List[Phase]
    segments: List[Segment]
    name: str = ""
    warp_size: int = 32                          # threads per warp (CUDA: 32)

    # ------------------------------------------------------------ sizes
    @property
    def n_threads(self) -> int:
        return self.block[0] * self.block[1] * self.grid[0] * self.grid[1]

    def instances_upper_bound(self) -> int:
        """Thread x access x loop-point instances before guards (a count, no
        evaluation): the number of records when no access has guards."""
        total = 0
        for s in self.segments:
            for p in self.phases[s.phase_begin:s.phase_begin + s.phase_count]:
                for a in self.accesses[p.access_begin:p.access_begin + p.access_count]:
                    box = 1
                    for lo, hi in a.loops:
                        box *= max(0, hi - lo)
                    total += box * s.repeat
        return total * self.n_threads

    def replace(self, **kw) -> "KernelDesc":
        return dataclasses.replace(self, **kw)


class Builder:
    """Convenience builder: phases are appended in order and a segment covers
    a contiguous run of phases."""

    def __init__(self, block, grid, name="", warp_size=32):
        self.block = tuple(block)
        self.grid = tuple(grid)
        self.name = name
        self.warp_size = int(warp_size)
        self.arrays: List[Array] = []
        self.accesses: List[Access] = []
        self.phases: List[Phase] = []
        self.segments: List[Segment] = []
        self._open_segment = None

    def array(self, space, dims, name="") -> int:
        self.arrays.append(Array(space, tuple(int(d) for d in dims), name))
        return len(self.arrays) - 1

    def phase(self, accesses: Sequence[Access], barrier_after, barrier_guards=()) -> int:
        """``barrier_after``: False / True (block barrier) or a BARRIER_* kind."""
        begin = len(self.accesses)
        self.accesses.extend(accesses)
        self.phases.append(Phase(begin, len(accesses), int(barrier_after), tuple(barrier_guards)))
        return len(self.phases) - 1

    def phase_like(self, phase_id: int, barrier_after) -> int:
        """A new phase over the same accesses as ``phase_id`` (used to peel
        one iteration of a repeated segment with a different barrier flag)."""
        src = self.phases[phase_id]
        self.phases.append(Phase(src.access_begin, src.access_count, int(barrier_after), src.barrier_guards))
        return len(self.phases) - 1

    def segment(self, phase_ids: Sequence[int], repeat=1, k_base=0):
        phase_ids = list(phase_ids)
        assert phase_ids == list(range(phase_ids[0], phase_ids[0] + len(phase_ids))), \
            "a segment covers a contiguous run of phases"
        self.segments.append(Segment(phase_ids[0], len(phase_ids), repeat, k_base))

    def build(self) -> KernelDesc:
        return KernelDesc(self.block, self.grid, list(self.arrays), list(self.accesses),
                          list(self.phases), list(self.segments), self.name, self.warp_size)


def rw(array: int, is_write: bool, *idx, loops=(), aux=(Aux(), Aux()), guards=(), name=""):
    """Shorthand for an :class:`Access`."""
    return Access(array, bool(is_write), tuple(idx), tuple(loops), tuple(aux), tuple(guards), name)
