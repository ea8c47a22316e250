"""TEST INFRASTRUCTURE: the CPU oracle of the per-barrier-interval SIMT
data-race check.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The checker library (the
``paper_2503_08946_amd`` package and its HIP code) never imports, links or
runs anything here, and this package imports nothing from it.

The arithmetic lives in ``rv_oracle.c`` (plain C, int64, one ``qsort``);
this module serialises a :class:`workloads.KernelDesc` into the oracle's own
int64 word layout and calls it through ctypes.  See the header of
``rv_oracle.c`` for the definition it implements.

Every function here is pinned by the ``-m "not gpu"`` tests: closed forms
derived by hand (stride-1, ``a[tid/2]``, tree reduction, tiled matmul,
polynomial product, Ge-SpMM staging) and an O(N^2) brute-force pair search on
small random kernels.  The paper prints no output of its own ISCC runs, so no
value here is pinned to a number the paper prints.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MAGIC = 0x524F5256


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math: integer code only)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class OrcWitness(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "interval", "space", "array", "address", "block",
        "f_block", "f_tid", "f_dphase", "f_access")] + [("f_loop", ctypes.c_int64 * 3), ("f_write", ctypes.c_int64)] + \
        [(n, ctypes.c_int64) for n in ("s_block", "s_tid", "s_dphase", "s_access")] + \
        [("s_loop", ctypes.c_int64 * 3), ("s_write", ctypes.c_int64)]


class OrcResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int64), ("n_records", ctypes.c_int64),
                ("n_conflicts", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
                ("n_intervals", ctypes.c_int64), ("oob", ctypes.c_int64 * 5),
                ("n_witness", ctypes.c_int64)]


class OrcRecord(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "interval", "space", "block", "array", "address", "gthread", "dphase", "access", "lidx")] + \
        [("loop", ctypes.c_int64 * 3), ("is_write", ctypes.c_int64)]


class OrcDeps(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "status", "n_records", "n_raw", "n_waw", "n_war", "n_dep_locations")] + [("oob", ctypes.c_int64 * 5)]


class OrcDiv(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "status", "n_instances", "n_divergent", "dphase", "block", "warp", "arrive_tid", "skip_tid")]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        lib.orc_check.argtypes = [P(ctypes.c_int64), ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                  P(OrcResult), P(OrcWitness), ctypes.c_int64]
        lib.orc_check.restype = ctypes.c_int
        lib.orc_records.argtypes = [P(ctypes.c_int64), ctypes.c_int64, ctypes.c_int64, P(OrcRecord),
                                    ctypes.c_int64, P(ctypes.c_int64)]
        lib.orc_records.restype = ctypes.c_int
        lib.orc_intervals.argtypes = [P(ctypes.c_int64), ctypes.c_int64, P(ctypes.c_int64)]
        lib.orc_intervals.restype = ctypes.c_int
        lib.orc_check_strict.argtypes = [P(ctypes.c_int64), ctypes.c_int64, P(OrcResult), P(OrcWitness),
                                         ctypes.c_int64]
        lib.orc_check_strict.restype = ctypes.c_int
        lib.orc_ordered.argtypes = [P(ctypes.c_int64), ctypes.c_int64, P(OrcDeps)]
        lib.orc_ordered.restype = ctypes.c_int
        lib.orc_divergence.argtypes = [P(ctypes.c_int64), ctypes.c_int64, P(OrcDiv)]
        lib.orc_divergence.restype = ctypes.c_int
        _lib = lib
    return _lib


def serialize(desc) -> np.ndarray:
    """Description -> the oracle's int64 word layout (see rv_oracle.c)."""
    w = [MAGIC, desc.block[0], desc.block[1], desc.grid[0], desc.grid[1],
         len(desc.arrays), len(desc.accesses), 0, len(desc.phases), len(desc.segments),
         getattr(desc, "warp_size", 32)]
    guards = []
    for a in desc.arrays:
        dims = list(a.dims) + [1] * (3 - len(a.dims))
        w += [a.space, len(a.dims)] + dims
    for ac in desc.accesses:
        lo_hi = []
        for l in range(3):
            lo_hi += list(ac.loops[l]) if l < len(ac.loops) else [0, 1]
        w += [ac.array, int(ac.is_write), len(ac.loops)] + lo_hi
        for x in ac.aux:
            w += [x.kind, x.d] + list(x.e)
        for d in range(3):
            w += list(ac.idx[d]) if d < len(ac.idx) else [0] * 11
        w += [len(guards), len(ac.guards)]
        guards += list(ac.guards)
    ph_words = []
    for p in desc.phases:
        bg = tuple(getattr(p, "barrier_guards", ()))
        ph_words += [p.access_begin, p.access_count, int(p.barrier_after), len(guards), len(bg)]
        guards += list(bg)
    for g in guards:
        w += list(g)
    w += ph_words
    for s in desc.segments:
        w += [s.phase_begin, s.phase_count, s.repeat, s.k_base]
    w[7] = len(guards)
    return np.asarray(w, dtype=np.int64)


@dataclass
class Side:
    block: int
    tid: int
    dphase: int
    access: int
    loop: tuple
    is_write: int


@dataclass
class Witness:
    interval: int
    space: int
    array: int
    address: int
    block: int
    first: Side
    second: Side

    def key(self):
        return (self.interval, self.space, self.block, self.array, self.address)


@dataclass
class Result:
    status: int
    n_records: int
    n_conflicts: int
    n_pairs: int
    n_intervals: int
    oob: tuple
    witnesses: List[Witness]


def check(desc, max_witnesses: int = 1 << 16, ilo: int = 0, ihi: Optional[int] = None,
          strict: bool = False) -> Result:
    """Run the oracle on intervals [ilo, ihi) (default: all).  ``strict``:
    blocks are never ordered (global records of different blocks conflict
    across intervals); the whole kernel is checked and ilo/ihi are ignored."""
    lib = _load()
    words = serialize(desc)
    res = OrcResult()
    buf = (OrcWitness * max(1, max_witnesses))()
    hi = (1 << 62) if ihi is None else ihi
    wp = words.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    if strict:
        lib.orc_check_strict(wp, len(words), ctypes.byref(res), buf, max_witnesses)
    else:
        lib.orc_check(wp, len(words), ilo, hi, ctypes.byref(res), buf, max_witnesses)
    ws = []
    for i in range(res.n_witness):
        b = buf[i]
        ws.append(Witness(b.interval, b.space, b.array, b.address, b.block,
                          Side(b.f_block, b.f_tid, b.f_dphase, b.f_access, tuple(b.f_loop), b.f_write),
                          Side(b.s_block, b.s_tid, b.s_dphase, b.s_access, tuple(b.s_loop), b.s_write)))
    return Result(res.status, res.n_records, res.n_conflicts, res.n_pairs, res.n_intervals,
                  tuple(res.oob), ws)


def records(desc, interval: int) -> np.ndarray:
    """All records of one interval as a structured numpy array (id order)."""
    lib = _load()
    words = serialize(desc)
    n = ctypes.c_int64()
    cap = desc.instances_upper_bound()
    buf = (OrcRecord * max(1, cap))()
    st = lib.orc_records(words.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(words), interval,
                         buf, cap, ctypes.byref(n))
    if st:
        raise ValueError(f"oracle status {st}")
    arr = np.frombuffer(buf, dtype=np.int64).reshape(-1, 13)[: n.value]
    return arr.copy()


RECORD_COLUMNS = ("interval", "space", "block", "array", "address", "gthread", "dphase", "access",
                  "lidx", "loop0", "loop1", "loop2", "is_write")


def n_intervals(desc) -> int:
    lib = _load()
    words = serialize(desc)
    n = ctypes.c_int64()
    st = lib.orc_intervals(words.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(words), ctypes.byref(n))
    if st:
        raise ValueError(f"oracle status {st}")
    return n.value


@dataclass
class Deps:
    status: int
    n_records: int
    n_raw: int
    n_waw: int
    n_war: int
    n_dep_locations: int


def ordered(desc) -> Deps:
    """RaW / WaW / WaR counts of the kernel run on its sequential schedule
    (dynamic phase, global thread, loop index); see rv_oracle.c step 8."""
    lib = _load()
    words = serialize(desc)
    out = OrcDeps()
    lib.orc_ordered(words.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(words), ctypes.byref(out))
    return Deps(out.status, out.n_records, out.n_raw, out.n_waw, out.n_war, out.n_dep_locations)


@dataclass
class Divergence:
    status: int
    n_instances: int
    n_divergent: int
    dphase: int
    block: int
    warp: int
    arrive_tid: int
    skip_tid: int


def divergence(desc) -> Divergence:
    """Barrier instances reached by part of their scope (rv_oracle.c step 9)."""
    lib = _load()
    words = serialize(desc)
    out = OrcDiv()
    lib.orc_divergence(words.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(words), ctypes.byref(out))
    return Divergence(*(getattr(out, n) for n, _ in OrcDiv._fields_))
