"""Description builders shared by the CPU and GPU tests.

Pure data: these functions lay out kernel descriptions (the same builders
the workloads use) and evaluate nothing.  ``rand_small`` draws small random
kernels exercising every description feature; ``linear_case`` builds the
kernels that drive the expansion's linear work-item paths and their
fallbacks."""

from workloads.desc import AUX_EMOD, AUX_FLOORDIV, GLOBAL, SHARED, Aux, Builder, aff, rw


def rand_small(rng, i):
    """Small random kernels exercising every description feature: 2-D blocks
    and grids, shared and global arrays of 1-3 dims, floordiv and emod aux
    terms, loops, the segment variable, guards, repeated segments and
    barrier-free phases."""
    bdx, bdy = int(rng.integers(1, 5)), int(rng.integers(1, 4))
    gdx, gdy = int(rng.integers(1, 3)), int(rng.integers(1, 3))
    b = Builder((bdx, bdy), (gdx, gdy), f"rand-small-{i}")
    n_arr = int(rng.integers(1, 4))
    for a in range(n_arr):
        nd = int(rng.integers(1, 4))
        dims = tuple(int(rng.integers(1, 5)) for _ in range(nd))
        b.array(SHARED if rng.random() < 0.5 else GLOBAL, dims)
    pids = []
    n_ph = int(rng.integers(1, 4))
    for p in range(n_ph):
        acc = []
        for _ in range(int(rng.integers(1, 4))):
            arr = int(rng.integers(0, n_arr))
            dims = b.arrays[arr].dims
            nl = int(rng.integers(0, 3))
            loops = tuple((int(lo), int(lo) + int(rng.integers(0, 3))) for lo in rng.integers(-1, 2, size=nl))

            def rnd_e(use_aux):
                terms = dict(tx=rng.integers(-2, 3), ty=rng.integers(-2, 3), bx=rng.integers(-2, 3),
                             by=rng.integers(-2, 3), k=rng.integers(-1, 2))
                for j in range(nl):
                    terms[f"l{j}"] = rng.integers(-2, 3)
                if use_aux:
                    terms["aux0"] = rng.integers(-1, 2)
                    terms["aux1"] = rng.integers(-1, 2)
                return aff(int(rng.integers(-3, 4)), **{k: int(v) for k, v in terms.items()})

            aux = (Aux(AUX_FLOORDIV, int(rng.integers(1, 4)), rnd_e(False)),
                   Aux(AUX_EMOD, int(rng.integers(1, 5)), rnd_e(False)))
            # per dim: emod into range so most kernels stay in bounds; aux vars mixed in
            idx = []
            for d, n in enumerate(dims):
                if d == 0:
                    idx.append(aff(aux1=1) if n >= 4 else aff(0))
                else:
                    idx.append(aff(0))
            guards = tuple(rnd_e(True) for _ in range(int(rng.integers(0, 2))))
            if dims[0] >= 4:
                aux = (aux[0], Aux(AUX_EMOD, dims[0], rnd_e(False)))
            acc.append(rw(arr, bool(rng.random() < 0.5), *idx, loops=loops, aux=aux, guards=guards))
        pids.append(b.phase(acc, barrier_after=bool(rng.random() < 0.6)))
    b.segment(pids[:1], repeat=int(rng.integers(1, 3)), k_base=int(rng.integers(0, 2)))
    if len(pids) > 1:
        b.segment(pids[1:], repeat=int(rng.integers(1, 3)))
    return b.build()

def rand_scoped(rng, i):
    """``rand_small`` kernels with barrier scopes: each phase ends with no
    barrier, a block barrier or a warp barrier, barriers may carry guards
    (affine in tx, ty, bx, by, k) and warps hold 1-4 threads (or 32), so
    small blocks span several warps."""
    import dataclasses
    d = rand_small(rng, i)
    phases = []
    for ph in d.phases:
        kind = int(rng.choice([0, 1, 2, 2]))
        guards = ()
        if kind and rng.random() < 0.4:
            guards = (aff(int(rng.integers(-1, 4)), tx=int(rng.integers(-2, 3)), ty=int(rng.integers(-1, 2)),
                          bx=int(rng.integers(-1, 2)), k=int(rng.integers(-1, 2))),)
        phases.append(dataclasses.replace(ph, barrier_after=kind, barrier_guards=guards))
    return d.replace(phases=phases, warp_size=int(rng.choice([1, 2, 3, 4, 32])), name=f"rand-scoped-{i}")


def rand_medium(rng, i, oob_rate=0.01):
    """Random kernels of a few thousand to a few hundred thousand records,
    spanning several expansion tiles and location buckets: 2-D launches up
    to (48, 4) x (5, 3), 1-4 shared or global arrays of 1-3 dims, 0-2 loops
    of up to 16 points, repeated segments (the segment variable k), guards,
    floor-division and Euclidean-remainder terms, and plain affine indices
    (the expansion's fast paths).  A plain affine index is placed inside
    its dimension over the whole launch and loop box; with probability
    ``oob_rate`` it is shifted out of it, so the kernel reports its first
    out-of-bounds instance."""
    bdx, bdy = int(rng.integers(1, 49)), int(rng.integers(1, 5))
    gdx, gdy = int(rng.integers(1, 6)), int(rng.integers(1, 4))
    b = Builder((bdx, bdy), (gdx, gdy), f"rand-medium-{i}")
    n_arr = int(rng.integers(1, 5))
    for a in range(n_arr):
        nd = int(rng.integers(1, 4))
        dims = tuple(int(rng.integers(4, 65)) for _ in range(nd))
        b.array(SHARED if rng.random() < 0.5 else GLOBAL, dims)
    n_ph = int(rng.integers(1, 5))
    reps = int(rng.integers(1, 4))
    vmax = dict(tx=bdx - 1, ty=bdy - 1, bx=gdx - 1, by=gdy - 1, k=reps - 1)
    pids = []
    for p in range(n_ph):
        acc = []
        for _ in range(int(rng.integers(1, 6))):
            arr = int(rng.integers(0, n_arr))
            dims = b.arrays[arr].dims
            nl = int(rng.integers(0, 3))
            trips = [int(rng.integers(1, 17)) for _ in range(nl)]
            loops = tuple((0, t) for t in trips)
            ranges = dict(vmax, **{f"l{j}": trips[j] - 1 for j in range(nl)})
            names = list(ranges)
            aux = [Aux(), Aux()]
            free_aux = [0, 1]
            idx = []
            for n in dims:
                kind = rng.random()
                if kind < 0.55:
                    # plain affine: coefficients in [-2, 2]; exact range over the box
                    terms = {v: int(rng.integers(-2, 3)) for v in names if rng.random() < 0.5}
                    lo = sum(min(0, c * ranges[v]) for v, c in terms.items())
                    hi = sum(max(0, c * ranges[v]) for v, c in terms.items())
                    if hi - lo < n:
                        c0 = -lo + int(rng.integers(0, n - (hi - lo)))
                        if rng.random() < oob_rate:
                            c0 += n - (hi - lo) if rng.random() < 0.5 else -(hi - lo) - 1
                        idx.append(aff(c0, **terms))
                        continue
                if free_aux:
                    x = free_aux.pop(0)
                    terms = {v: int(rng.integers(-3, 4)) for v in names}
                    e = aff(int(rng.integers(-8, 9)), **terms)
                    if rng.random() < 0.3:
                        # floor division of a non-negative numerator, kept in range
                        d = int(rng.integers(1, 5))
                        span = sum(abs(c) * ranges[v] for v, c in terms.items())
                        e = aff(span + 8, **terms)
                        aux[x] = Aux(AUX_FLOORDIV, d, e)
                        idx.append(aff(aux0=1) if x == 0 else aff(aux1=1))
                        if (2 * span + 16) // d >= n:
                            aux[x] = Aux(AUX_EMOD, n, e)
                    else:
                        aux[x] = Aux(AUX_EMOD, n, e)
                        idx.append(aff(aux0=1) if x == 0 else aff(aux1=1))
                else:
                    idx.append(aff(int(rng.integers(0, n))))
            guards = []
            for _ in range(int(rng.integers(0, 3)) if rng.random() < 0.35 else 0):
                terms = {v: int(rng.integers(-2, 3)) for v in names if rng.random() < 0.5}
                guards.append(aff(int(rng.integers(-2, 2 * max(1, bdx))), **terms))
            acc.append(rw(arr, bool(rng.random() < 0.5), *idx, loops=loops, aux=tuple(aux), guards=tuple(guards)))
        pids.append(b.phase(acc, barrier_after=bool(rng.random() < 0.6)))
    b.segment(pids, repeat=reps)
    return b.build()


def linear_case(name):
    # Entries whose lanes each take one thread and consecutive points of the
    # innermost loop: the records of a chunk are placed per run of points
    # sharing a bucket, with a fallback to the per-record rank when a chunk
    # leaves the bounds, the key range or a common bucket.  Each case pairs
    # accesses without thread terms (all lanes of a wave at one location per
    # point: the run path by construction) with accesses whose lanes spread
    # over several buckets per point (the fallback).
    if name == "partial-chunk":          # 40 points: chunks of 16, 16, 8
        b = Builder((64, 2), (3, 1), name)
        s = b.array(SHARED, (2, 40))
        t = b.array(SHARED, (2, 64, 40))
        p = b.phase([rw(s, True, aff(ty=1), aff(l0=1), loops=((0, 40),)),
                     rw(s, False, aff(1, ty=-1), aff(39, l0=-1), loops=((0, 40),)),
                     rw(t, True, aff(ty=1), aff(tx=1), aff(l0=1), loops=((0, 40),)),
                     rw(t, False, aff(1, ty=-1), aff(63, tx=-1), aff(l0=1), loops=((0, 40),))], False)
        b.segment([p])
    elif name == "descending":           # location falls by 33 per point, crossing buckets
        b = Builder((128, 1), (4, 1), name)
        g = b.array(GLOBAL, (200000,))
        p = b.phase([rw(g, True, aff(190000, bx=128, l0=-33), loops=((0, 48),)),
                     rw(g, False, aff(190000, bx=128, l0=-33), loops=((0, 48),)),
                     rw(g, True, aff(100000, tx=1, bx=128, l0=-33), loops=((0, 48),)),
                     rw(g, False, aff(100001, tx=1, bx=128, l0=-33), loops=((0, 48),))], False)
        b.segment([p])
    elif name == "two-loops":            # inner extent 32 (linear) and 20 (wraps: not linear)
        b = Builder((32, 4), (2, 2), name)
        s = b.array(SHARED, (8, 40))
        g = b.array(GLOBAL, (64, 64))
        p = b.phase([rw(s, True, aff(l0=1), aff(l1=1), loops=((0, 8), (0, 32))),
                     rw(s, False, aff(l0=1), aff(l1=1), loops=((0, 8), (3, 23))),
                     rw(g, False, aff(ty=1, by=4, l0=1), aff(tx=1, bx=32), loops=((0, 16),))], True)
        q = b.phase([rw(g, True, aff(ty=1, by=4, l0=1), aff(tx=1, bx=32), loops=((0, 16),)),
                     rw(g, False, aff(ty=1, by=4, l0=1), aff(63, tx=-1, bx=-32), loops=((0, 16),))], False)
        b.segment([p, q])
    elif name == "stride-buckets":       # 37 locations per point: runs of points per bucket
        b = Builder((64, 1), (8, 1), name)
        g = b.array(GLOBAL, (1 << 16,))
        p = b.phase([rw(g, False, aff(2048, bx=4096, l0=37), loops=((0, 64),)),
                     rw(g, True, aff(2048, bx=4096, l0=37), loops=((0, 64),)),
                     rw(g, False, aff(tx=1, bx=4096, l0=7), loops=((0, 64),)),
                     rw(g, True, aff(5, tx=1, bx=4096, l0=7), loops=((0, 64),))], False)
        b.segment([p])
    elif name == "flat-few-threads":     # 3 threads: loop chunks spread over the lanes
        b = Builder((3, 1), (1, 1), name)
        g = b.array(GLOBAL, (2000,))
        p = b.phase([rw(g, True, aff(7, l0=1), loops=((0, 40),)),
                     rw(g, False, aff(l0=1), loops=((0, 40),)),
                     rw(g, True, aff(tx=500, l0=1), loops=((0, 500),)),
                     rw(g, False, aff(tx=500, l0=2), loops=((0, 500),))], False)
        b.segment([p])
    elif name == "pass-boundary":        # chunks straddle the first key-range pass's end (2^29)
        b = Builder((64, 1), (2, 1), name)
        g = b.array(GLOBAL, (1 << 30,))
        p = b.phase([rw(g, True, aff((1 << 29) - 8, bx=1, l0=1), loops=((0, 16),)),
                     rw(g, False, aff((1 << 29) - 8, l0=1), loops=((0, 16),)),
                     rw(g, True, aff(3 << 28, l0=1), loops=((0, 32),)),
                     rw(g, False, aff(3 << 28, tx=3, l0=1), loops=((0, 32),))], False)
        b.segment([p])
    elif name == "thread-linear":        # no loops: a lane takes 16 consecutive threads (tx alone varies)
        b = Builder((64, 2), (4, 2), name)
        g = b.array(GLOBAL, (4096,))
        s = b.array(SHARED, (2, 64))
        p = b.phase([rw(g, True, aff(tx=1, ty=64, bx=128, by=512)),
                     rw(g, False, aff(5, tx=3, ty=192, bx=384, by=1536)),     # 3 locations per thread
                     rw(s, True, aff(ty=1), aff(7)),                          # broadcast: one location
                     rw(s, False, aff(ty=1), aff(63, tx=-1)),                 # descending
                     rw(g, False, aff(tx=60, bx=1)),                          # lanes over many buckets
                     rw(s, False, aff(1, ty=-1), aff(tx=1), guards=(aff(30, tx=-1),))], True)
        q = b.phase([rw(s, True, aff(ty=1), aff(tx=1)), rw(g, True, aff(2048, tx=1, by=64))], False)
        b.segment([p, q])
    elif name == "thread-linear-oob":    # a lane's 16 threads run off the array
        b = Builder((32, 1), (2, 1), name)
        g = b.array(GLOBAL, (100,))
        p = b.phase([rw(g, False, aff(40, tx=2, bx=4))], False)
        b.segment([p])
    elif name == "edge-out-of-bounds":   # block 1's last threads leave the array mid-chunk: fallback
        b = Builder((64, 1), (2, 1), name)
        g = b.array(GLOBAL, (1990,))
        p = b.phase([rw(g, False, aff(tx=16, bx=1024, l0=1), loops=((0, 16),))], False)
        b.segment([p])
    else:
        raise ValueError(name)
    return b.build()


def large_grid(offset, dim, write_offset=None):
    """One-thread blocks beyond 2^23 (block ids no longer fit 24 bits):
    every block reads g[bx + offset] of g[dim]; with ``write_offset`` it also
    writes g[bx + write_offset]."""
    b = Builder((1, 1), ((1 << 23) + 64, 1), f"large-grid-{offset}")
    g = b.array(GLOBAL, (dim,))
    acc = [rw(g, False, aff(offset, bx=1))]
    if write_offset is not None:
        acc.append(rw(g, True, aff(write_offset, bx=1)))
    p = b.phase(acc, False)
    b.segment([p])
    return b.build()


def gespmm_closed_form(M, N, T, K):
    """Hand-derived figures of ``gespmm_crc(M, N, T, K, kb_on_all=False)``
    (the derivation is in golden/closed_forms.json, entry gespmm-crc-b-only):
    records, and conflicts with both barriers, without the middle one and
    without the trailing one."""
    threads = M * N
    blocks = M * (N // 32)
    return {"records": threads * T * (4 + 32 * (4 + K)),
            "conflicts": {"both": 0, "no_middle": 64 * T * blocks, "no_trailing": 64 * (T - 1) * blocks}}


def rand_affine_units(rng, i):
    """Random kernels whose accesses are all plain affine (no aux terms, no
    guards) and in bounds, with shared arrays of at most 2048 elements per
    block: the kernels the on-chip block-local units take.  Blocks of 8-64 x
    1-8 threads, grids up to 6 x 4, 1-3 shared and 0-2 global arrays of 1-2
    dims, 1-4 phases of 1-5 accesses with 0-2 loops of 1-16 points,
    coefficients in [-2, 2], half of the accesses writes."""
    bdx, bdy = int(rng.integers(8, 65)), int(rng.integers(1, 9))
    gdx, gdy = int(rng.integers(1, 7)), int(rng.integers(1, 5))
    b = Builder((bdx, bdy), (gdx, gdy), f"rand-units-{i}")
    n_sh, n_gl = int(rng.integers(1, 4)), int(rng.integers(0, 3))
    budget = 2048
    for a in range(n_sh):
        nd = int(rng.integers(1, 3))
        cap = max(4, budget // (n_sh - a) // 2)
        dims = (int(rng.integers(4, min(64, cap) + 1)),) if nd == 1 else \
            (int(rng.integers(2, 17)), int(rng.integers(2, max(3, min(64, cap // 16)) + 1)))
        size = dims[0] * (dims[1] if nd == 2 else 1)
        budget -= size
        b.array(SHARED, dims)
    for a in range(n_gl):
        b.array(GLOBAL, tuple(int(rng.integers(4, 129)) for _ in range(int(rng.integers(1, 3)))))
    reps = int(rng.integers(1, 3))
    vmax = dict(tx=bdx - 1, ty=bdy - 1, bx=gdx - 1, by=gdy - 1, k=reps - 1)
    pids = []
    for p in range(int(rng.integers(1, 5))):
        acc = []
        for _ in range(int(rng.integers(1, 6))):
            arr = int(rng.integers(0, n_sh + n_gl))
            dims = b.arrays[arr].dims
            nl = int(rng.integers(0, 3))
            trips = [int(rng.integers(1, 17)) for _ in range(nl)]
            loops = tuple((0, t) for t in trips)
            ranges = dict(vmax, **{f"l{j}": trips[j] - 1 for j in range(nl)})
            idx = []
            for n in dims:
                for _try in range(20):
                    terms = {v: int(rng.integers(-2, 3)) for v in ranges if rng.random() < 0.5}
                    lo = sum(min(0, c * ranges[v]) for v, c in terms.items())
                    hi = sum(max(0, c * ranges[v]) for v, c in terms.items())
                    if hi - lo < n:
                        break
                else:
                    terms, lo, hi = {}, 0, 0
                idx.append(aff(-lo + int(rng.integers(0, n - (hi - lo))), **terms))
            acc.append(rw(arr, bool(rng.random() < 0.5), *idx, loops=loops))
        pids.append(b.phase(acc, barrier_after=bool(rng.random() < 0.7)))
    b.segment(pids, repeat=reps)
    return b.build()
