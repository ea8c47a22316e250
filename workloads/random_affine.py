"""Seeded random affine 2-D kernels for the batched and served workloads.

Shape of one kernel (all draws from one ``PCG64`` stream per kernel), in
draw order:

* a record-count target drawn log-uniformly in ``[lo, hi]``;
* 1-6 phases, a barrier after each but the last; 1-8 accesses per phase;
  0-2 loops per access with trip counts in [1, 64] (this fixes the records
  per thread, m);
* blockDim (bx, by): bx uniform in [1, min(32, 1.1 target / m)], by uniform
  in [1, min(32, that bound / bx)]; gridDim up to (64, 64) scaled so the
  record count lands within 10 % of the target (everything above is redrawn
  until that is possible);
* 1-4 two-dimensional int arrays, each shared (256-4096 elements) or global
  (2^10-2^20 elements) with probability 1/2;
* each access: writes with p = 1/2; per array dimension an index
  ``emod(c . v + c0, dim)`` with coefficients
  uniform in [-4, 4] over (tx, ty, bx, by, l0, l1) and ``c0`` uniform in
  [0, dim); no guards.

Without guards the record count of a kernel is the plain product
``threads x sum over accesses of loop-box sizes``, so the target can be hit
exactly when the kernel is drawn.
"""

from __future__ import annotations

import math

import numpy as np

from .desc import AUX_EMOD, GLOBAL, SHARED, Aux, Builder, KernelDesc, aff, aff_from, NV


def _dims_for(rng, n_elems: int):
    # split n_elems = rows * cols with rows a power of two
    r = 1 << int(rng.integers(0, int(math.log2(n_elems)) + 1))
    return (r, n_elems // r)


def random_kernel(rng: np.random.Generator, lo: float, hi: float, name: str = "") -> KernelDesc:
    target = math.exp(rng.uniform(math.log(lo), math.log(hi)))
    while True:
        n_ph = int(rng.integers(1, 7))
        accs_per_phase = [int(rng.integers(1, 9)) for _ in range(n_ph)]
        n_acc = sum(accs_per_phase)
        loops = []
        m = 0
        for _ in range(n_acc):
            nl = int(rng.integers(0, 3))
            trips = [int(rng.integers(1, 65)) for _ in range(nl)]
            loops.append(trips)
            m += int(np.prod(trips)) if trips else 1
        # block dims drawn among those that can still reach the target
        cap = int(1.1 * target / m)
        if cap < 1:
            continue
        bdx = int(rng.integers(1, min(32, cap) + 1))
        bdy = int(rng.integers(1, min(32, max(1, cap // bdx)) + 1))
        tpb = bdx * bdy
        per_block = tpb * m
        nblk = target / per_block
        if nblk < 1 or nblk > 64 * 64:
            continue
        gy = max(1, math.ceil(nblk / 64))
        gx = max(1, min(64, round(nblk / gy)))
        rec = gx * gy * per_block
        if abs(rec - target) <= 0.1 * target:
            break
    b = Builder((bdx, bdy), (gx, gy), name)
    n_arr = int(rng.integers(1, 5))
    for a in range(n_arr):
        if rng.random() < 0.5:
            n = 1 << int(rng.integers(8, 13))          # 256 .. 4096
            b.array(SHARED, _dims_for(rng, n), f"s{a}")
        else:
            n = 1 << int(rng.integers(10, 21))         # 2^10 .. 2^20
            b.array(GLOBAL, _dims_for(rng, n), f"g{a}")
    pids = []
    ai = 0
    for p, na in enumerate(accs_per_phase):
        acc = []
        for _ in range(na):
            arr = int(rng.integers(0, n_arr))
            dims = b.arrays[arr].dims
            trips = loops[ai]
            ai += 1
            auxes = []
            for d in range(2):
                c = [0] * NV
                for v in (0, 1, 2, 3):                # tx ty bx by
                    c[v] = int(rng.integers(-4, 5))
                for li in range(len(trips)):          # l0 l1
                    c[5 + li] = int(rng.integers(-4, 5))
                auxes.append(Aux(AUX_EMOD, int(dims[d]), aff_from(c, int(rng.integers(0, dims[d])))))
            acc.append(b_access(arr, bool(rng.random() < 0.5), trips, auxes))
        pids.append(b.phase(acc, barrier_after=(p < n_ph - 1)))
    b.segment(pids)
    return b.build()


def b_access(arr, is_write, trips, auxes):
    from .desc import rw
    return rw(arr, is_write, aff(aux0=1), aff(aux1=1),
              loops=tuple((0, t) for t in trips), aux=tuple(auxes))


def batch_kernels(seed: int = 4, count: int = 4096, lo: float = 1e2, hi: float = 1e6):
    """``count`` kernels; kernel ``i`` draws from ``PCG64(SeedSequence(seed).spawn(count)[i])``."""
    out = []
    for i, child in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.Generator(np.random.PCG64(child))
        out.append(random_kernel(rng, lo, hi, name=f"batch-{seed}-{i}"))
    return out


def serving_stream(seed: int = 5, count: int = 10500, lo: float = 1e3, hi: float = 1e7):
    """Jobs for the served workload, drawn like :func:`batch_kernels` with
    record counts log-uniform in [lo, hi].  Returns a generator of kernels."""
    for i, child in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.Generator(np.random.PCG64(child))
        yield random_kernel(rng, lo, hi, name=f"serve-{seed}-{i}")


def poisson_arrivals(seed: int, count: int, rate_per_s: float):
    """Arrival offsets (seconds) of a Poisson process of the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))
