"""O(N^2) brute force for tiny kernels: an independent statement of the race
definition, used to pin the oracle.

It shares nothing with the oracle's C code.  Records come from simulating the
kernel thread by thread, the way a sequential interpreter would run it: walk
the segments, count the barriers a thread passes (its current barrier
interval), and at each access evaluate the index expressions with Python's
own ``//`` and ``%`` (floor division and, for a positive divisor, the
Euclidean remainder).  The conflict test is the pairwise definition itself:
two records of the same location in the same interval, from different
threads, at least one a write.  No sorting and no min/max shortcut.
"""

from __future__ import annotations

from itertools import product

from workloads.desc import VARS


def _ev(a, env):
    return a[-1] + sum(c * env[v] for c, v in zip(a[:-1], VARS))


def simulate(desc):
    """Yield records (interval, space, block_if_shared, array, address,
    id_tuple, thread, is_write, loop_values)."""
    bdx, bdy = desc.block
    gdx, gdy = desc.grid
    tpb = bdx * bdy
    for by, bx in product(range(gdy), range(gdx)):
        blk = by * gdx + bx
        for ty, tx in product(range(bdy), range(bdx)):
            tid = ty * bdx + tx
            thread = blk * tpb + tid
            interval = 0
            dyn = 0
            for seg in desc.segments:
                for r in range(seg.repeat):
                    for p in range(seg.phase_begin, seg.phase_begin + seg.phase_count):
                        ph = desc.phases[p]
                        for a in range(ph.access_begin, ph.access_begin + ph.access_count):
                            acc = desc.accesses[a]
                            arr = desc.arrays[acc.array]
                            ranges = [range(lo, hi) for lo, hi in acc.loops]
                            for li, lv in enumerate(product(*ranges)):
                                env = dict(tx=tx, ty=ty, bx=bx, by=by, k=seg.k_base + r,
                                           l0=0, l1=0, l2=0, aux0=0, aux1=0)
                                for j, val in enumerate(lv):
                                    env[f"l{j}"] = val
                                for j, x in enumerate(acc.aux):
                                    if x.kind == 1:
                                        env[f"aux{j}"] = _ev(x.e, env) // x.d
                                    elif x.kind == 2:
                                        env[f"aux{j}"] = _ev(x.e, env) % x.d
                                if any(_ev(g, env) < 0 for g in acc.guards):
                                    continue
                                idx = [_ev(e, env) for e in acc.idx]
                                for i, n in zip(idx, arr.dims):
                                    if not 0 <= i < n:
                                        raise IndexError((interval, thread, dyn, a, li))
                                flat = 0
                                for i, n in zip(idx, arr.dims):
                                    flat = flat * n + i
                                yield (interval, arr.space, blk if arr.space == 0 else 0, acc.array,
                                       flat, (thread, dyn, a, li), thread, int(acc.is_write),
                                       tuple(lv) + (0,) * (3 - len(lv)))
                        dyn += 1
                        if ph.barrier_after:
                            interval += 1


def brute_check(desc):
    """Return (n_records, conflicts) with conflicts an ordered list of
    (location, first, second, n_pairs); first/second are records."""
    recs = list(simulate(desc))
    by_loc = {}
    for r in recs:
        by_loc.setdefault(r[:5], []).append(r)
    out = []
    for loc in sorted(by_loc):
        rs = by_loc[loc]
        pairs = set()
        for i in range(len(rs)):
            for j in range(i + 1, len(rs)):
                a, b = rs[i], rs[j]
                if a[6] != b[6] and (a[7] or b[7]):
                    pairs.add((min(a[6], b[6]), max(a[6], b[6])))
        if pairs:
            writes = [r for r in rs if r[7]]
            first = min(writes, key=lambda r: r[5])
            lo = min(rs, key=lambda r: r[5])
            hi = max(rs, key=lambda r: r[5])
            second = lo if lo[6] != first[6] else hi
            out.append((loc, first, second, len(pairs)))
    return len(recs), out
