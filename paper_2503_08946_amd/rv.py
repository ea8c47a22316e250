"""ctypes binding of librv (include/rv.h).

Argument marshalling only: every step of the check runs in librv's gfx950
kernels.  There is no CPU path; if librv.so is missing or no GPU is present,
the calls fail.  PyTorch is used for one thing: allocating the device
workspace and naming the current HIP stream.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librv.so")

RV_NV = 10
STATUS = {0: "RV_OK", -1: "RV_ERR_INVALID", -2: "RV_ERR_UNSUPPORTED", -3: "RV_ERR_KEY_BITS",
          -4: "RV_ERR_RANGE", -5: "RV_ERR_OOB", -6: "RV_ERR_TOO_LARGE", -7: "RV_ERR_BUDGET",
          -8: "RV_ERR_DEVICE", -9: "RV_ERR_STATE"}
STAGES = ("fill", "count", "scan", "expand", "sort_scan", "finish", "small", "direct")


class RVError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


# ----------------------------------------------------------- C structures
i32, i64, u32, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64


class rv_launch(ctypes.Structure):
    _fields_ = [("block", i32 * 3), ("grid", i32 * 3)]


class rv_array(ctypes.Structure):
    _fields_ = [("space", i32), ("ndim", i32), ("dim", i64 * 3)]


class rv_affine(ctypes.Structure):
    _fields_ = [("coef", i32 * RV_NV), ("c0", i32)]


class rv_aux(ctypes.Structure):
    _fields_ = [("kind", i32), ("d", i32), ("e", rv_affine)]


class rv_access(ctypes.Structure):
    _fields_ = [("array", i32), ("is_write", i32), ("nloops", i32), ("loop_lo", i32 * 3),
                ("loop_hi", i32 * 3), ("aux", rv_aux * 2), ("idx", rv_affine * 3),
                ("guard_begin", i32), ("guard_count", i32)]


class rv_guard(ctypes.Structure):
    _fields_ = [("g", rv_affine)]


class rv_phase(ctypes.Structure):
    _fields_ = [("access_begin", i32), ("access_count", i32), ("barrier_after", i32),
                ("guard_begin", i32), ("guard_count", i32)]


class rv_segment(ctypes.Structure):
    _fields_ = [("phase_begin", i32), ("phase_count", i32), ("repeat", i32), ("k_base", i32)]


class rv_kernel_desc(ctypes.Structure):
    _fields_ = [("launch", rv_launch),
                ("arrays", ctypes.POINTER(rv_array)), ("n_arrays", i32),
                ("accesses", ctypes.POINTER(rv_access)), ("n_accesses", i32),
                ("guards", ctypes.POINTER(rv_guard)), ("n_guards", i32),
                ("phases", ctypes.POINTER(rv_phase)), ("n_phases", i32),
                ("segments", ctypes.POINTER(rv_segment)), ("n_segments", i32),
                ("warp_size", i32)]


class rv_side(ctypes.Structure):
    _fields_ = [("block", u32), ("tid", u32), ("dyn_phase", u32), ("access", u32),
                ("loop", i32 * 3), ("is_write", i32)]


class rv_witness(ctypes.Structure):
    _fields_ = [("interval", u32), ("space", i32), ("array", i32), ("block", u32),
                ("address", i64), ("first", rv_side), ("second", rv_side)]


class rv_result(ctypes.Structure):
    _fields_ = [("n_records", u64), ("n_conflicts", u64), ("has_witness", i32),
                ("reserved", i32), ("witness", rv_witness)]


class rv_timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 8), ("launches", u64 * 8), ("small_records", u64),
                ("direct_records", u64), ("counted_records", u64)]


class rv_kernel_info(ctypes.Structure):
    _fields_ = [("n_instances", u64), ("n_intervals", u32), ("n_subintervals", u32),
                ("n_chunks", u32), ("n_buckets", u32), ("max_interval_instances", u64),
                ("n_entries", u32), ("n_flat_entries", u32), ("n_linear_entries", u32),
                ("n_fast_entries", u32), ("n_proven_entries", u32), ("n_direct_intervals", u32)]


class rv_record(ctypes.Structure):
    _fields_ = [("interval", u32), ("space", i32), ("block", u32), ("array", i32), ("address", i64),
                ("gthread", u32), ("dyn_phase", u32), ("access", u32), ("lidx", u32),
                ("loop", i32 * 3), ("is_write", i32)]


class rv_barrier_result(ctypes.Structure):
    _fields_ = [("n_instances", u64), ("n_divergent", u64), ("has_divergence", i32), ("dyn_phase", u32),
                ("block", u32), ("warp", i32), ("arrive_tid", u32), ("skip_tid", u32)]


class rv_load_options(ctypes.Structure):
    _fields_ = [("semantics", i32), ("reserved", i32 * 3)]


SEMANTICS = {"interval": 0, "strict": 1, "ordered": 2}


class rv_counts(ctypes.Structure):
    _fields_ = [("n_records", u64), ("n_conflicts", u64), ("n_pairs", u64), ("n_raw", u64), ("n_waw", u64),
                ("n_war", u64), ("n_dep_locations", u64)]


class rv_tuning(ctypes.Structure):
    _fields_ = [("target", i32), ("group", i32), ("n_candidates", i32), ("small_cap", i32),
                ("direct", i32), ("reserved", i32), ("candidates", i32 * 8), ("cand_group", i32 * 8), ("cand_small", i32 * 8),
                ("ms", ctypes.c_double * 8)]


GROUPS = {"fold": 0, "sort_scan": 1}


class rv_server_stats(ctypes.Structure):
    _fields_ = [("batches", u64), ("jobs", u64), ("max_batch_jobs", u64), ("overlapped_batches", u64)]


class rv_job_result(ctypes.Structure):
    _fields_ = [("job_id", u64), ("status", i32), ("reserved", i32), ("result", rv_result),
                ("t_submit_ns", u64), ("t_start_ns", u64), ("t_done_ns", u64)]


# --------------------------------------------------------------- library
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"librv.so is not built ({LIB_PATH}); run __graft_entry__.build() "
                               "or python -m paper_2503_08946_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, V, S = ctypes.POINTER, ctypes.c_void_p, ctypes.c_size_t
        sig = {
            "rv_validate_desc": [P(rv_kernel_desc), ctypes.c_char_p, S],
            "rv_plan_desc": [P(rv_kernel_desc), i32, P(rv_kernel_info), ctypes.c_char_p, S],
            "rv_ctx_create": [P(V), ctypes.c_int, V, V, S],
            "rv_ctx_destroy": [V],
            "rv_load_kernel_desc": [V, P(rv_kernel_desc), P(V)],
            "rv_load_kernel_desc_ex": [V, P(rv_kernel_desc), P(rv_load_options), P(V)],
            "rv_free_kernel": [V, V],
            "rv_kernel_get_info": [V, V, P(rv_kernel_info)],
            "rv_check": [V, V, P(rv_result)],
            "rv_check_batch": [V, P(V), S, P(rv_result)],
            "rv_check_static": [V, V, P(rv_result)],
            "rv_check_barriers": [V, V, P(rv_barrier_result)],
            "rv_check_counts": [V, V, P(rv_counts)],
            "rv_get_witnesses": [V, V, u64, P(rv_witness), S, P(S)],
            "rv_debug_records": [V, V, u32, ctypes.c_int, P(rv_record), S, P(S)],
            "rv_set_timing": [V, ctypes.c_int],
            "rv_get_timing": [V, P(rv_timing), ctypes.c_int],
            "rv_selftest": [ctypes.c_char_p, S],
            "rv_ctx_get_tuning": [V, P(rv_tuning)],
            "rv_ctx_set_tuning": [V, P(rv_tuning)],
            "rv_autotune": [V, P(rv_kernel_desc), S, i32, P(rv_tuning)],
            "rv_server_create": [V, V, S, u64, P(V)],
            "rv_server_destroy": [V],
            "rv_server_submit": [V, V, P(u64)],
            "rv_server_poll": [V, P(rv_job_result), S, P(S)],
            "rv_server_drain": [V, u64],
            "rv_server_get_stats": [V, P(rv_server_stats)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = i32
        L.rv_last_error.argtypes = [V]
        L.rv_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


EXPORTED = ("rv_validate_desc", "rv_plan_desc", "rv_ctx_create", "rv_ctx_destroy", "rv_last_error", "rv_load_kernel_desc",
            "rv_load_kernel_desc_ex",
            "rv_free_kernel", "rv_kernel_get_info", "rv_check", "rv_check_batch", "rv_check_static",
            "rv_check_barriers", "rv_check_counts",
            "rv_get_witnesses",
            "rv_debug_records", "rv_set_timing", "rv_get_timing", "rv_selftest", "rv_ctx_get_tuning",
            "rv_ctx_set_tuning", "rv_autotune", "rv_server_create",
            "rv_server_destroy", "rv_server_submit", "rv_server_poll", "rv_server_drain", "rv_server_get_stats")


# -------------------------------------------------------------- marshalling
def _affine(a, out: rv_affine):
    for v in range(RV_NV):
        out.coef[v] = int(a[v])
    out.c0 = int(a[RV_NV])


class Marshalled:
    """A description laid out as the C structures of rv.h (owns the arrays)."""

    def __init__(self, desc):
        arrays = (rv_array * max(1, len(desc.arrays)))()
        for i, a in enumerate(desc.arrays):
            arrays[i].space = int(a.space)
            arrays[i].ndim = len(a.dims)
            for j in range(3):
                arrays[i].dim[j] = int(a.dims[j]) if j < len(a.dims) else 1
        guards_list = []
        accesses = (rv_access * max(1, len(desc.accesses)))()
        for i, ac in enumerate(desc.accesses):
            c = accesses[i]
            c.array = int(ac.array)
            c.is_write = int(bool(ac.is_write))
            c.nloops = len(ac.loops)
            for l, (lo, hi) in enumerate(ac.loops):
                c.loop_lo[l] = int(lo)
                c.loop_hi[l] = int(hi)
            for x in range(2):
                c.aux[x].kind = int(ac.aux[x].kind)
                c.aux[x].d = int(ac.aux[x].d)
                _affine(ac.aux[x].e, c.aux[x].e)
            for d in range(len(ac.idx)):
                _affine(ac.idx[d], c.idx[d])
            c.guard_begin = len(guards_list)
            c.guard_count = len(ac.guards)
            guards_list.extend(ac.guards)
        phases = (rv_phase * max(1, len(desc.phases)))()
        for i, p in enumerate(desc.phases):
            phases[i].access_begin = int(p.access_begin)
            phases[i].access_count = int(p.access_count)
            phases[i].barrier_after = int(p.barrier_after)
            bg = tuple(getattr(p, "barrier_guards", ()))
            phases[i].guard_begin = len(guards_list)
            phases[i].guard_count = len(bg)
            guards_list.extend(bg)
        guards = (rv_guard * max(1, len(guards_list)))()
        for i, g in enumerate(guards_list):
            _affine(g, guards[i].g)
        segs = (rv_segment * max(1, len(desc.segments)))()
        for i, s in enumerate(desc.segments):
            segs[i].phase_begin = int(s.phase_begin)
            segs[i].phase_count = int(s.phase_count)
            segs[i].repeat = int(s.repeat)
            segs[i].k_base = int(s.k_base)
        d = rv_kernel_desc()
        d.launch.block[0], d.launch.block[1], d.launch.block[2] = int(desc.block[0]), int(desc.block[1]), 1
        d.launch.grid[0], d.launch.grid[1], d.launch.grid[2] = int(desc.grid[0]), int(desc.grid[1]), 1
        d.arrays, d.n_arrays = arrays, len(desc.arrays)
        d.accesses, d.n_accesses = accesses, len(desc.accesses)
        d.guards, d.n_guards = guards, len(guards_list)
        d.phases, d.n_phases = phases, len(desc.phases)
        d.segments, d.n_segments = segs, len(desc.segments)
        d.warp_size = int(getattr(desc, "warp_size", 32))
        self._keep = (arrays, accesses, guards, phases, segs)
        self.desc = d

    def desc_bytes(self) -> bytes:
        """The description's contents (not its addresses), for fingerprints."""
        d = self.desc
        parts = [bytes(d.launch)]
        for arr, n in zip(self._keep, (d.n_arrays, d.n_accesses, d.n_guards, d.n_phases, d.n_segments)):
            parts.append(bytes(memoryview(arr))[:n * ctypes.sizeof(arr._type_)])
        return b"".join(parts)


# ------------------------------------------------------------ Python types
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
    n_records: int
    n_conflicts: int
    witness: Optional[Witness]


def _side(s: rv_side) -> Side:
    return Side(s.block, s.tid, s.dyn_phase, s.access, tuple(s.loop), s.is_write)


def _witness(w: rv_witness) -> Witness:
    return Witness(w.interval, w.space, w.array, w.address, w.block, _side(w.first), _side(w.second))


def _result(r: rv_result) -> Result:
    return Result(r.n_records, r.n_conflicts, _witness(r.witness) if r.has_witness else None)


def validate(desc) -> tuple:
    """Host-only validation: (status, message)."""
    m = Marshalled(desc)
    buf = ctypes.create_string_buffer(512)
    st = lib().rv_validate_desc(ctypes.byref(m.desc), buf, 512)
    return st, buf.value.decode()


def plan(desc, target: int = 0) -> rv_kernel_info:
    """Host-only planning (no device): the kernel's plan figures.  Raises
    RVError with the planner's code and message for a rejected description."""
    m = Marshalled(desc)
    buf = ctypes.create_string_buffer(512)
    out = rv_kernel_info()
    st = lib().rv_plan_desc(ctypes.byref(m.desc), int(target), ctypes.byref(out), buf, 512)
    if st:
        raise RVError(st, buf.value.decode())
    return out


def selftest() -> tuple:
    buf = ctypes.create_string_buffer(256)
    st = lib().rv_selftest(buf, 256)
    return st, buf.value.decode()


class Kernel:
    def __init__(self, ctx: "Context", handle: ctypes.c_void_p, desc):
        self.ctx = ctx
        self.handle = handle
        self.desc = desc

    def info(self) -> rv_kernel_info:
        out = rv_kernel_info()
        self.ctx._call(lib().rv_kernel_get_info, self.ctx.handle, self.handle, ctypes.byref(out))
        return out

    def free(self):
        if self.handle:
            lib().rv_free_kernel(self.ctx.handle, self.handle)
            self.handle = None

    def __del__(self):
        try:
            if self.handle and self.ctx.handle:
                self.free()
        except Exception:
            pass


class Batch:
    """The marshalled arguments of rv_check_batch for a fixed list of
    kernels: run() calls the library and leaves the rv_result array in
    ``out``; results() converts it."""

    def __init__(self, ctx: "Context", ks: Sequence[Kernel]):
        self.ctx = ctx
        self.ks = list(ks)
        n = len(self.ks)
        self.handles = (ctypes.c_void_p * max(1, n))(*[k.handle for k in self.ks])
        self.out = (rv_result * max(1, n))()

    def run(self):
        self.ctx._call(lib().rv_check_batch, self.ctx.handle, self.handles, len(self.ks), self.out)

    def results(self) -> List[Result]:
        return [_result(self.out[i]) for i in range(len(self.ks))]


class Context:
    """A librv context on one device with a caller-owned workspace.

    ``workspace``: a torch uint8 CUDA tensor, or None to allocate
    ``workspace_bytes`` with torch.  ``stream``: a torch.cuda.Stream or None
    for the current stream."""

    def __init__(self, device: int = 0, workspace_bytes: int = 1 << 30, workspace=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("librv needs a GPU: torch.cuda.is_available() is False")
        self.device = device
        if workspace is None:
            workspace = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=f"cuda:{device}")
        self.workspace = workspace
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        st = lib().rv_ctx_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.c_void_p(workspace.data_ptr()), workspace.numel())
        if st:
            raise RVError(st, "rv_ctx_create failed")
        self.handle = h

    def _call(self, f, *args):
        st = f(*args)
        if st:
            raise RVError(st, lib().rv_last_error(self.handle).decode())
        return st

    def close(self):
        if self.handle:
            lib().rv_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- API
    def load(self, desc, semantics: str = "interval") -> Kernel:
        """Load a description; ``semantics`` "interval" (the default),
        "strict" (blocks are never ordered) or "ordered" (the sequential
        schedule, for rv_check_counts): rv_load_kernel_desc_ex."""
        m = Marshalled(desc)
        h = ctypes.c_void_p()
        if semantics == "interval":
            self._call(lib().rv_load_kernel_desc, self.handle, ctypes.byref(m.desc), ctypes.byref(h))
        else:
            o = rv_load_options()
            o.semantics = SEMANTICS[semantics]
            self._call(lib().rv_load_kernel_desc_ex, self.handle, ctypes.byref(m.desc), ctypes.byref(o),
                       ctypes.byref(h))
        return Kernel(self, h, desc)

    def check(self, k: Kernel) -> Result:
        out = rv_result()
        self._call(lib().rv_check, self.handle, k.handle, ctypes.byref(out))
        return _result(out)

    def check_static(self, k: Kernel) -> Result:
        """rv_check_static: the check with the library's static device
        scratch instead of the context's workspace (no allocation)."""
        out = rv_result()
        self._call(lib().rv_check_static, self.handle, k.handle, ctypes.byref(out))
        return _result(out)

    def check_counts(self, k: Kernel) -> dict:
        """rv_check_counts: distinct-thread pairs (interval semantics) or
        RaW / WaW / WaR dependences (a kernel loaded with semantics="ordered")."""
        out = rv_counts()
        self._call(lib().rv_check_counts, self.handle, k.handle, ctypes.byref(out))
        return {name: getattr(out, name) for name, _ in rv_counts._fields_}

    def check_barriers(self, k: Kernel) -> dict:
        """rv_check_barriers: divergent barrier instances of a kernel."""
        out = rv_barrier_result()
        self._call(lib().rv_check_barriers, self.handle, k.handle, ctypes.byref(out))
        d = {name: getattr(out, name) for name, _ in rv_barrier_result._fields_}
        d["first"] = ((out.dyn_phase, out.block, out.warp, out.arrive_tid, out.skip_tid)
                      if out.has_divergence else None)
        return d

    def check_batch(self, ks: Sequence[Kernel]) -> List[Result]:
        b = Batch(self, ks)
        b.run()
        return b.results()

    def witnesses(self, k: Kernel, first: int = 0, cap: int = 1 << 16) -> List[Witness]:
        buf = (rv_witness * max(1, cap))()
        n = ctypes.c_size_t()
        self._call(lib().rv_get_witnesses, self.handle, k.handle, first, buf, cap, ctypes.byref(n))
        return [_witness(buf[i]) for i in range(n.value)]

    def debug_records(self, k: Kernel, interval: int, sorted: bool = False, cap: Optional[int] = None):
        """Records of one interval as an int64 array with columns
        (interval, space, block, array, address, gthread, dyn_phase, access,
        lidx, loop0, loop1, loop2, is_write)."""
        if cap is None:
            cap = int(k.info().max_interval_instances)
        buf = (rv_record * max(1, cap))()
        n = ctypes.c_size_t()
        self._call(lib().rv_debug_records, self.handle, k.handle, interval, int(sorted), buf, cap,
                   ctypes.byref(n))
        m = min(n.value, cap)
        raw = np.frombuffer(buf, dtype=np.dtype([
            ("interval", "<u4"), ("space", "<i4"), ("block", "<u4"), ("array", "<i4"), ("address", "<i8"),
            ("gthread", "<u4"), ("dyn_phase", "<u4"), ("access", "<u4"), ("lidx", "<u4"),
            ("loop", "<i4", (3,)), ("is_write", "<i4")]))[:m]
        out = np.empty((m, 13), dtype=np.int64)
        for j, name in enumerate(("interval", "space", "block", "array", "address", "gthread", "dyn_phase",
                                  "access", "lidx")):
            out[:, j] = raw[name]
        out[:, 9:12] = raw["loop"]
        out[:, 12] = raw["is_write"]
        return out

    # ------------------------------------------------------------- tuning
    @property
    def target(self) -> int:
        t = rv_tuning()
        self._call(lib().rv_ctx_get_tuning, self.handle, ctypes.byref(t))
        return t.target

    @target.setter
    def target(self, value: int):
        t = rv_tuning()
        self._call(lib().rv_ctx_get_tuning, self.handle, ctypes.byref(t))
        t.target = int(value)
        self._call(lib().rv_ctx_set_tuning, self.handle, ctypes.byref(t))

    @property
    def small_cap(self) -> int:
        """Batched checks: passes of at most this many instances run on chip."""
        t = rv_tuning()
        self._call(lib().rv_ctx_get_tuning, self.handle, ctypes.byref(t))
        return t.small_cap

    @small_cap.setter
    def small_cap(self, value: int):
        t = rv_tuning()
        self._call(lib().rv_ctx_get_tuning, self.handle, ctypes.byref(t))
        t.small_cap = int(value)
        self._call(lib().rv_ctx_set_tuning, self.handle, ctypes.byref(t))

    @property
    def direct(self) -> bool:
        """rv_check groups block-local (shared-array) locations on chip."""
        t = rv_tuning()
        self._call(lib().rv_ctx_get_tuning, self.handle, ctypes.byref(t))
        return bool(t.direct)

    @direct.setter
    def direct(self, value: bool):
        t = rv_tuning()
        self._call(lib().rv_ctx_get_tuning, self.handle, ctypes.byref(t))
        t.direct = 1 if value else 0
        self._call(lib().rv_ctx_set_tuning, self.handle, ctypes.byref(t))

    @property
    def group(self) -> str:
        """Per-bucket grouping kernel: "fold" or "sort_scan"."""
        t = rv_tuning()
        self._call(lib().rv_ctx_get_tuning, self.handle, ctypes.byref(t))
        return {v: k for k, v in GROUPS.items()}[t.group]

    @group.setter
    def group(self, value: str):
        t = rv_tuning()
        self._call(lib().rv_ctx_get_tuning, self.handle, ctypes.byref(t))
        t.group = GROUPS[value]
        self._call(lib().rv_ctx_set_tuning, self.handle, ctypes.byref(t))

    def autotune(self, descs, trials: int = 3, cache: Optional[str] = None) -> dict:
        """Pick the planner target for this context by timing a batched
        check of ``descs`` under each candidate (rv_autotune).  With
        ``cache``, a JSON file keyed by the device name and the batch's
        description fingerprint is read first and written after a
        measurement."""
        import hashlib
        import json
        import torch
        ms = [Marshalled(d) for d in descs]
        fp = hashlib.sha256(b"".join(bytes(m.desc_bytes()) for m in ms)).hexdigest()[:16]
        key = f"{torch.cuda.get_device_name(self.device)}/{fp}"
        if cache and os.path.exists(cache):
            with open(cache) as f:
                db = json.load(f)
            if key in db:
                self.target = db[key]["target"]
                self.group = db[key]["group"]
                self.small_cap = db[key].get("small_cap", self.small_cap)
                return db[key]
        arr = (rv_kernel_desc * max(1, len(ms)))(*[m.desc for m in ms])
        t = rv_tuning()
        self._call(lib().rv_autotune, self.handle, arr, len(ms), int(trials), ctypes.byref(t))
        names = {v: k for k, v in GROUPS.items()}
        rec = {"target": t.target, "group": names[t.group], "small_cap": t.small_cap,
               "ms": {f"{t.candidates[i]}/{names[t.cand_group[i]]}/{t.cand_small[i]}": t.ms[i]
                      for i in range(t.n_candidates)}}
        if cache:
            db = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    db = json.load(f)
            db[key] = rec
            with open(cache, "w") as f:
                json.dump(db, f, indent=1)
        return rec

    def set_timing(self, on: bool):
        self._call(lib().rv_set_timing, self.handle, int(on))

    def timing(self, reset: bool = True) -> dict:
        t = rv_timing()
        self._call(lib().rv_get_timing, self.handle, ctypes.byref(t), int(reset))
        out = {name: (t.ms[i], t.launches[i]) for i, name in enumerate(STAGES)}
        out["small_records"] = t.small_records
        out["direct_records"] = t.direct_records
        out["counted_records"] = t.counted_records
        return out


@dataclass
class JobResult:
    job_id: int
    status: int
    result: Optional[Result]
    t_submit_ns: int
    t_start_ns: int
    t_done_ns: int

    @property
    def latency_ns(self) -> int:
        return self.t_done_ns - self.t_submit_ns


class Server:
    """Continuous-batching server over a context (see rv_server_* in rv.h).

    ``workspace``: a torch uint8 CUDA tensor of the budget, or None to
    allocate ``budget_bytes``."""

    def __init__(self, ctx: Context, budget_bytes: int = 1 << 30, workspace=None, max_batch_records: int = 1 << 26):
        import torch
        self.ctx = ctx
        if workspace is None:
            workspace = torch.empty(int(budget_bytes), dtype=torch.uint8, device=f"cuda:{ctx.device}")
        self.workspace = workspace
        h = ctypes.c_void_p()
        ctx._call(lib().rv_server_create, ctx.handle, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                  int(max_batch_records), ctypes.byref(h))
        self.handle = h
        self._keep = {}

    def submit(self, k: Kernel) -> int:
        jid = ctypes.c_uint64()
        st = lib().rv_server_submit(self.handle, k.handle, ctypes.byref(jid))
        if st:
            raise RVError(st, "rv_server_submit failed")
        self._keep[jid.value] = k
        return jid.value

    def poll(self, cap: int = 4096) -> List[JobResult]:
        buf = (rv_job_result * cap)()
        n = ctypes.c_size_t()
        st = lib().rv_server_poll(self.handle, buf, cap, ctypes.byref(n))
        if st:
            raise RVError(st, "rv_server_poll failed")
        out = []
        for i in range(n.value):
            r = buf[i]
            self._keep.pop(r.job_id, None)
            out.append(JobResult(r.job_id, r.status, _result(r.result) if r.status == 0 else None,
                                 r.t_submit_ns, r.t_start_ns, r.t_done_ns))
        return out

    def stats(self) -> dict:
        st = rv_server_stats()
        if lib().rv_server_get_stats(self.handle, ctypes.byref(st)):
            raise RVError(-1, "rv_server_get_stats failed")
        return {name: getattr(st, name) for name, _ in rv_server_stats._fields_}

    def drain(self, timeout_ms: int = 600000):
        st = lib().rv_server_drain(self.handle, int(timeout_ms))
        if st:
            raise RVError(st, "rv_server_drain timed out")

    def close(self):
        if self.handle:
            lib().rv_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
