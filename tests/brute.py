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
    id_tuple, thread, is_write, loop_values, fine_interval).  The interval
    counts the block barriers a thread has passed, the fine interval the
    barriers of either kind (block or warp)."""
    bdx, bdy = desc.block
    gdx, gdy = desc.grid
    tpb = bdx * bdy
    for by, bx in product(range(gdy), range(gdx)):
        blk = by * gdx + bx
        for ty, tx in product(range(bdy), range(bdx)):
            tid = ty * bdx + tx
            thread = blk * tpb + tid
            interval = 0
            fine = 0
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
                                       tuple(lv) + (0,) * (3 - len(lv)), fine)
                        dyn += 1
                        if int(ph.barrier_after) == 1:
                            interval += 1
                        if int(ph.barrier_after):
                            fine += 1


def _canonical(rs, sub, unit):
    """The canonical pair of a conflicting location's records rs: inside the
    smallest sub-interval holding a write and two threads, the write with
    the smallest id and the smallest-id record of that sub-interval if its
    thread differs, else its largest-id record; with no such sub-interval,
    the same across units (warps or blocks) over all records."""
    for j in sorted({sub(r) for r in rs}):
        part = [r for r in rs if sub(r) == j]
        writes = [r for r in part if r[7]]
        if writes and len({r[6] for r in part}) > 1:
            first = min(writes, key=lambda r: r[5])
            lo, hi = min(part, key=lambda r: r[5]), max(part, key=lambda r: r[5])
            return first, (lo if lo[6] != first[6] else hi)
    first = min((r for r in rs if r[7]), key=lambda r: r[5])
    lo, hi = min(rs, key=lambda r: r[5]), max(rs, key=lambda r: r[5])
    return first, (lo if unit(lo[6]) != unit(first[6]) else hi)


def brute_check(desc, strict=False):
    """Return (n_records, conflicts) with conflicts an ordered list of
    (location, first, second, n_pairs); first/second are records.

    A pair of records of one location conflicts when it comes from two
    threads, one of them writes, and nothing orders it: in the same barrier
    interval, records of one warp in different fine intervals are ordered
    by a warp barrier.  ``strict``: global records are grouped across
    intervals, and two of them are ordered only when they come from one
    block and different intervals."""
    bdx, bdy = desc.block
    tpb = bdx * bdy
    ws = getattr(desc, "warp_size", 32)
    wpb = (tpb + ws - 1) // ws

    def warp(t):
        return (t // tpb) * wpb + (t % tpb) // ws

    def block(t):
        return t // tpb

    recs = list(simulate(desc))
    by_loc = {}
    for r in recs:
        if strict and r[1] == 1:
            key = (1, 1, 0, r[3], r[4])          # global: every interval together, after shared
        else:
            key = (0,) + r[:5]
        by_loc.setdefault(key, []).append(r)
    out = []
    for key in sorted(by_loc):
        rs = by_loc[key]
        glob = key[0] == 1
        pairs = set()
        for i in range(len(rs)):
            for j in range(i + 1, len(rs)):
                a, b = rs[i], rs[j]
                if a[6] == b[6] or not (a[7] or b[7]):
                    continue
                if glob:
                    ordered = block(a[6]) == block(b[6]) and a[0] != b[0]
                else:
                    ordered = warp(a[6]) == warp(b[6]) and a[9] != b[9]
                if not ordered:
                    pairs.add((min(a[6], b[6]), max(a[6], b[6])))
        if pairs:
            if glob:
                first, second = _canonical(rs, lambda r: r[0], block)
                loc = (first[0],) + key[1:]
            else:
                first, second = _canonical(rs, lambda r: r[9], warp)
                loc = key[1:]
            out.append((loc, first, second, len(pairs)))
    return len(recs), out


def brute_ordered(desc):
    """(records, RaW, WaW, WaR, locations with a dependence) of the kernel
    run sequentially: dynamic phase by dynamic phase, threads in order, loop
    points in order.  The accesses of one (dynamic phase, thread, loop index)
    are one statement instance.  Every ordered pair of instances that touch
    one element is tested."""
    recs = list(simulate(desc))
    by_loc = {}
    for r in recs:
        thread, dyn, _a, li = r[5]
        inst = by_loc.setdefault(r[1:5], {}).setdefault((dyn, thread, li), [False, False])
        inst[0 if r[7] else 1] = True
    raw = waw = war = nloc = 0
    for insts in by_loc.values():
        times = sorted(insts)
        lr = lw = lwr = 0
        for i, t1 in enumerate(times):
            for t2 in times[i + 1:]:
                w1, r1 = insts[t1]
                w2, r2 = insts[t2]
                lr += w1 and r2
                lw += w1 and w2
                lwr += r1 and w2
        raw += lr
        waw += lw
        war += lwr
        nloc += bool(lr or lw or lwr)
    return len(recs), raw, waw, war, nloc


def brute_divergence(desc):
    """(barrier instances, divergent ones, the first as (dynamic phase, block,
    warp or -1, smallest thread reaching it, smallest thread not))."""
    bdx, bdy = desc.block
    gdx, gdy = desc.grid
    tpb = bdx * bdy
    ws = getattr(desc, "warp_size", 32)
    n = nd = 0
    first = None
    dyn = 0
    for seg in desc.segments:
        for r in range(seg.repeat):
            for p in range(seg.phase_begin, seg.phase_begin + seg.phase_count):
                ph = desc.phases[p]
                kind = int(ph.barrier_after)
                if kind:
                    size = tpb if kind == 1 else ws
                    for blk in range(gdx * gdy):
                        for t0 in range(0, tpb, size):
                            reach = []
                            for t in range(t0, min(t0 + size, tpb)):
                                env = dict(tx=t % bdx, ty=t // bdx, bx=blk % gdx, by=blk // gdx,
                                           k=seg.k_base + r, l0=0, l1=0, l2=0, aux0=0, aux1=0)
                                reach.append(all(_ev(g, env) >= 0 for g in ph.barrier_guards))
                            n += 1
                            if any(reach) and not all(reach):
                                if first is None:
                                    first = (dyn, blk, -1 if kind == 1 else t0 // ws,
                                             t0 + reach.index(True), t0 + reach.index(False))
                                nd += 1
                dyn += 1
    return n, nd, first
