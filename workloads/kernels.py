"""Fixed and seeded kernel descriptions.

Each builder returns a :class:`~workloads.desc.KernelDesc`.  The builders
only lay out data; none of them computes records, locations or conflicts.

* ``tiny_fixed``            -- one 64-thread block: ``s[tid] = ..``; barrier;
                               ``.. = s[63 - tid]; s[(tid + 1) % 64] = ..``.
* ``tiny_random``           -- 64-thread single-block kernels with random
                               affine addresses taken mod 64 (seeded).
* ``tree_reduction``        -- a shared-memory tree reduction over 1024
                               threads, optionally with one barrier deleted.
* ``tiled_matmul``          -- the access pattern of a 32x32 shared-memory
                               tiled matrix product, optionally with one
                               dynamic barrier (or one static barrier) removed.
* ``polynomial_product``    -- the paper's polynomial-product example
                               (Section 2.1) with ``i`` mapped to ``tid.x``.
* ``gespmm_crc``            -- the access relations the paper writes for the
                               shared-memory staging of Ge-SpMM's Algorithm 2
                               (Section 2.1.2), as a looped SIMT kernel.
* ``stride1_*`` / ``half_index_*`` -- the two textbook patterns: stride-1
                               writes and ``a[tid / 2]`` writes.
* ``polynomial_product_full`` -- the same example with its zeroing statement
                               ``S: C[k] = 0`` as a phase of its own.
* ``warp_reduction``        -- per-warp tree reduction ordered by warp barriers
                               (coarse-grained warp merging), optionally with
                               one warp barrier dropped.
* ``warp_exchange``         -- a warp barrier (or a block barrier) between
                               writes and reads that cross warps.
* ``cross_block_global``    -- global elements written by block 0 and read by
                               every block after a barrier.
* ``guarded_barrier``       -- barriers reached by part of a block or warp.
"""

from __future__ import annotations

import numpy as np

from .desc import (AUX_EMOD, AUX_FLOORDIV, BARRIER_BLOCK, BARRIER_WARP, GLOBAL, SHARED, Aux, Builder,
                   KernelDesc, Phase, Segment, aff, aff_from, rw)


# --------------------------------------------------------------------- tiny
def tiny_fixed() -> KernelDesc:
    b = Builder((64, 1), (1, 1), "tiny-fixed")
    s = b.array(SHARED, (64,), "s")
    p0 = b.phase([rw(s, True, aff(tx=1), name="W s[tid]")], barrier_after=True)
    p1 = b.phase([
        rw(s, False, aff(63, tx=-1), name="R s[63-tid]"),
        rw(s, True, aff(aux0=1), aux=(Aux(AUX_EMOD, 64, aff(1, tx=1)), Aux()),
           name="W s[(tid+1)%64]"),
    ], barrier_after=False)
    b.segment([p0, p1])
    return b.build()


def tiny_random(seed: int = 1, count: int = 32):
    """``count`` single-block kernels: blockDim (64,1), one shared int[64];
    1-3 phases of 1-4 accesses; address ``emod(c . (tx,ty,bx,by) + c0, 64)``
    with ``c`` uniform in [-2, 2] and ``c0`` in [0, 64); writes with p = 0.5."""
    out = []
    for i, child in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.Generator(np.random.PCG64(child))
        b = Builder((64, 1), (1, 1), f"tiny-random-{seed}-{i}")
        s = b.array(SHARED, (64,), "s")
        n_ph = int(rng.integers(1, 4))
        pids = []
        for p in range(n_ph):
            acc = []
            for _ in range(int(rng.integers(1, 5))):
                c = rng.integers(-2, 3, size=4)
                c0 = int(rng.integers(0, 64))
                e = aff(c0, tx=int(c[0]), ty=int(c[1]), bx=int(c[2]), by=int(c[3]))
                acc.append(rw(s, bool(rng.random() < 0.5), aff(aux0=1),
                              aux=(Aux(AUX_EMOD, 64, e), Aux())))
            pids.append(b.phase(acc, barrier_after=(p < n_ph - 1)))
        b.segment(pids)
        out.append(b.build())
    return out


# ------------------------------------------------------------ tree reduction
def tree_reduction(deleted_barrier: int = -1, block: int = 1024, grid: int = 128,
                   levels: int = 10) -> KernelDesc:
    """Phase ``k`` (0 <= k < levels): threads ``tid < h`` with ``h = block/2 >> k``
    read ``s[tid]`` and ``s[tid + h]`` and write ``s[tid]``; a barrier follows
    every phase unless ``k == deleted_barrier``."""
    name = "tree-reduction" + ("" if deleted_barrier < 0 else f"-nobar{deleted_barrier}")
    b = Builder((block, 1), (grid, 1), name)
    s = b.array(SHARED, (block,), "s")
    pids = []
    for k in range(levels):
        h = (block // 2) >> k
        guard = aff(h - 1, tx=-1)                      # tid < h  <=>  h - 1 - tid >= 0
        pids.append(b.phase([
            rw(s, False, aff(tx=1), guards=(guard,), name="R s[tid]"),
            rw(s, False, aff(h, tx=1), guards=(guard,), name="R s[tid+h]"),
            rw(s, True, aff(tx=1), guards=(guard,), name="W s[tid]"),
        ], barrier_after=(k != deleted_barrier)))
    b.segment(pids)
    return b.build()


# --------------------------------------------------------------- tiled matmul
def tiled_matmul(grid: int = 16, k_iters: int = 64, drop_dynamic: int = -1,
                 drop_static: str = "") -> KernelDesc:
    """blockDim (32,32), gridDim (grid,grid).  For k in [0, k_iters):
    load   R A[by*32+ty][k*32+tx], R B[k*32+ty][bx*32+tx], W As[ty][tx], W Bs[ty][tx]; barrier
    compute (j in [0,32))  R As[ty][j], R Bs[j][tx]; barrier
    then W C[by*32+ty][bx*32+tx].

    ``drop_dynamic = d`` removes the d-th executed barrier (d = 2k after the
    load of iteration k, d = 2k+1 after its compute) by peeling iteration k.
    ``drop_static`` in {"load", "compute"} removes that barrier in every
    iteration."""
    T = 32
    n = T * grid
    kk = T * k_iters
    tag = f"matmul-{grid}x{grid}"
    if drop_dynamic >= 0:
        tag += f"-drop{drop_dynamic}"
    if drop_static:
        tag += f"-static-{drop_static}"
    b = Builder((T, T), (grid, grid), tag)
    A = b.array(GLOBAL, (n, kk), "A")
    B = b.array(GLOBAL, (kk, n), "B")
    C = b.array(GLOBAL, (n, n), "C")
    As = b.array(SHARED, (T, T), "As")
    Bs = b.array(SHARED, (T, T), "Bs")
    load = [
        rw(A, False, aff(by=T, ty=1), aff(k=T, tx=1), name="R A[by*32+ty][k*32+tx]"),
        rw(B, False, aff(k=T, ty=1), aff(bx=T, tx=1), name="R B[k*32+ty][bx*32+tx]"),
        rw(As, True, aff(ty=1), aff(tx=1), name="W As[ty][tx]"),
        rw(Bs, True, aff(ty=1), aff(tx=1), name="W Bs[ty][tx]"),
    ]
    comp = [
        rw(As, False, aff(ty=1), aff(l0=1), loops=((0, T),), name="R As[ty][j]"),
        rw(Bs, False, aff(l0=1), aff(tx=1), loops=((0, T),), name="R Bs[j][tx]"),
    ]
    p_load = b.phase(load, barrier_after=(drop_static != "load"))
    p_comp = b.phase(comp, barrier_after=(drop_static != "compute"))
    final = [rw(C, True, aff(by=T, ty=1), aff(bx=T, tx=1), name="W C[by*32+ty][bx*32+tx]")]
    if drop_dynamic < 0:
        b.segment([p_load, p_comp], repeat=k_iters)
    else:
        k0, which = divmod(drop_dynamic, 2)
        assert 0 <= k0 < k_iters
        if k0 > 0:
            b.segment([p_load, p_comp], repeat=k0, k_base=0)
        # the peeled iteration shares the access lists and clears one flag
        pl = b.phase_like(p_load, barrier_after=(which != 0))
        pc = b.phase_like(p_comp, barrier_after=(which != 1))
        b.segment([pl, pc], repeat=1, k_base=k0)
        if k0 + 1 < k_iters:
            pl2 = b.phase_like(p_load, barrier_after=True)
            pc2 = b.phase_like(p_comp, barrier_after=True)
            b.segment([pl2, pc2], repeat=k_iters - k0 - 1, k_base=k0 + 1)
    p_fin = b.phase(final, barrier_after=False)
    b.segment([p_fin])
    return b.build()


def matmul_mutants(seed: int = 3, k_iters: int = 64, extra: int = 3):
    """The fixed dropped-barrier indices {0, 1, 64, 126, 127} plus ``extra``
    drawn from ``PCG64(seed)`` in [0, 2*k_iters)."""
    fixed = [0, 1, k_iters, 2 * k_iters - 2, 2 * k_iters - 1]
    rng = np.random.Generator(np.random.PCG64(seed))
    pool = [d for d in range(2 * k_iters) if d not in fixed]
    drawn = sorted(int(x) for x in rng.choice(pool, size=extra, replace=False))
    return fixed + drawn


# --------------------------------------------------------- paper's examples
def polynomial_product(n: int = 64) -> KernelDesc:
    """Section 2.1's example ``C[i+j] += A[i] * B[j]`` as one SIMT phase:
    ``i`` is ``tid.x`` (n threads, one block) and ``j`` the loop ``l0`` in [0, n).
    Per loop point the thread reads C[i+j], A[i], B[j] and writes C[i+j]."""
    b = Builder((n, 1), (1, 1), f"polynomial-product-{n}")
    A = b.array(GLOBAL, (n,), "A")
    B = b.array(GLOBAL, (n,), "B")
    C = b.array(GLOBAL, (2 * n - 1,), "C")
    loop = ((0, n),)
    p = b.phase([
        rw(C, False, aff(tx=1, l0=1), loops=loop, name="R C[i+j]"),
        rw(A, False, aff(tx=1), loops=loop, name="R A[i]"),
        rw(B, False, aff(l0=1), loops=loop, name="R B[j]"),
        rw(C, True, aff(tx=1, l0=1), loops=loop, name="W C[i+j]"),
    ], barrier_after=False)
    b.segment([p])
    return b.build()


def polynomial_product_full(n: int = 64) -> KernelDesc:
    """Section 2.1's example with both statements: S (``C[k] = 0`` for k in
    [0, 2n-1)) is phase 0, run by thread 0 (its loop is ``l0``); T is
    ``polynomial_product``'s phase.  No barrier: the phases are the code
    sections of the sequential schedule (S before T)."""
    b = Builder((n, 1), (1, 1), f"polynomial-product-full-{n}")
    A = b.array(GLOBAL, (n,), "A")
    B = b.array(GLOBAL, (n,), "B")
    C = b.array(GLOBAL, (2 * n - 1,), "C")
    s = b.phase([rw(C, True, aff(l0=1), loops=((0, 2 * n - 1),), guards=(aff(tx=-1),), name="W C[k]")],
                barrier_after=False)
    loop = ((0, n),)
    t = b.phase([
        rw(C, False, aff(tx=1, l0=1), loops=loop, name="R C[i+j]"),
        rw(A, False, aff(tx=1), loops=loop, name="R A[i]"),
        rw(B, False, aff(l0=1), loops=loop, name="R B[j]"),
        rw(C, True, aff(tx=1, l0=1), loops=loop, name="W C[i+j]"),
    ], barrier_after=False)
    b.segment([s, t])
    return b.build()


def warp_reduction(dropped: int = -1, block: int = 64, grid: int = 2, warp: int = 32) -> KernelDesc:
    """Coarse-grained warp merging: each warp reduces its own slice of a
    shared array with warp barriers only.  Phase k (h = warp/2 >> k): lanes
    ``lane < h`` (lane = tid mod warp) read s[tid] and s[tid + h] and write
    s[tid]; a warp barrier follows every phase except ``dropped``."""
    levels = warp.bit_length() - 1
    b = Builder((block, 1), (grid, 1), f"warp-reduction-w{warp}" + ("" if dropped < 0 else f"-drop{dropped}"),
                warp_size=warp)
    s = b.array(SHARED, (block,), "s")
    lane = (Aux(AUX_EMOD, warp, aff(tx=1)), Aux())
    pids = []
    for k in range(levels):
        h = (warp // 2) >> k
        g = aff(h - 1, aux0=-1)                               # lane < h
        pids.append(b.phase([
            rw(s, False, aff(tx=1), aux=lane, guards=(g,), name="R s[tid]"),
            rw(s, False, aff(h, tx=1), aux=lane, guards=(g,), name="R s[tid+h]"),
            rw(s, True, aff(tx=1), aux=lane, guards=(g,), name="W s[tid]"),
        ], barrier_after=0 if k == dropped else BARRIER_WARP))
    b.segment(pids)
    return b.build()


def warp_exchange(kind: int = BARRIER_WARP, block: int = 64, grid: int = 2, warp: int = 32) -> KernelDesc:
    """s[tid] written, then a barrier of ``kind``, then s[block-1-tid] read:
    every element is read by a thread of the other half of the block."""
    b = Builder((block, 1), (grid, 1), f"warp-exchange-{'warp' if kind == BARRIER_WARP else 'block'}-w{warp}",
                warp_size=warp)
    s = b.array(SHARED, (block,), "s")
    p0 = b.phase([rw(s, True, aff(tx=1), name="W s[tid]")], barrier_after=kind)
    p1 = b.phase([rw(s, False, aff(block - 1, tx=-1), name="R s[block-1-tid]")], barrier_after=False)
    b.segment([p0, p1])
    return b.build()


def cross_block_global(block: int = 32, grid: int = 4) -> KernelDesc:
    """Block 0 writes g[tid]; block barrier; every block reads g[tid]."""
    b = Builder((block, 1), (grid, 1), "cross-block-global")
    g = b.array(GLOBAL, (block,), "g")
    p0 = b.phase([rw(g, True, aff(tx=1), guards=(aff(bx=-1),), name="W g[tid] (block 0)")], barrier_after=True)
    p1 = b.phase([rw(g, False, aff(tx=1), name="R g[tid]")], barrier_after=False)
    b.segment([p0, p1])
    return b.build()


def guarded_barrier(case: str) -> KernelDesc:
    """Barriers that carry guards.  ``block-half``: blockDim 32, gridDim 3, a
    block barrier reached by tid <= 15.  ``warp-tail``: blockDim 64 (two warps
    of 32), gridDim 2, a warp barrier reached by tid <= 47.  ``block-uniform``:
    gridDim 4, a block barrier reached by the blocks bx <= 1 (all their
    threads).  ``k-uniform``: a barrier in a segment repeated 3 times,
    reached while k <= 1."""
    if case == "block-half":
        b = Builder((32, 1), (3, 1), "guarded-barrier-block-half")
        s = b.array(SHARED, (32,))
        p0 = b.phase([rw(s, True, aff(tx=1))], barrier_after=BARRIER_BLOCK, barrier_guards=(aff(15, tx=-1),))
        p1 = b.phase([rw(s, False, aff(31, tx=-1))], barrier_after=False)
        b.segment([p0, p1])
    elif case == "warp-tail":
        b = Builder((64, 1), (2, 1), "guarded-barrier-warp-tail")
        s = b.array(SHARED, (64,))
        p0 = b.phase([rw(s, True, aff(tx=1))], barrier_after=BARRIER_WARP, barrier_guards=(aff(47, tx=-1),))
        p1 = b.phase([rw(s, False, aff(tx=1))], barrier_after=False)
        b.segment([p0, p1])
    elif case == "block-uniform":
        b = Builder((32, 1), (4, 1), "guarded-barrier-block-uniform")
        s = b.array(SHARED, (32,))
        p0 = b.phase([rw(s, True, aff(tx=1))], barrier_after=BARRIER_BLOCK, barrier_guards=(aff(1, bx=-1),))
        p1 = b.phase([rw(s, False, aff(tx=1))], barrier_after=False)
        b.segment([p0, p1])
    elif case == "k-uniform":
        b = Builder((16, 1), (2, 1), "guarded-barrier-k-uniform")
        s = b.array(SHARED, (16,))
        p0 = b.phase([rw(s, True, aff(tx=1))], barrier_after=BARRIER_BLOCK, barrier_guards=(aff(1, k=-1),))
        b.segment([p0], repeat=3)
    else:
        raise ValueError(case)
    return b.build()


def gespmm_crc(M: int = 4, N: int = 64, T: int = 3, K: int = 2,
               middle_barrier: bool = True, trailing_barrier: bool = True,
               kb_on_all: bool = True) -> KernelDesc:
    """The shared-memory staging pattern of Ge-SpMM's Algorithm 2 written from
    the access relations of Section 2.1.2, as a SIMT kernel.

    Thread mapping: ``i = bid.x`` (rows, M), ``j = bid.y * 32 + tid.x``
    (columns, N), blockDim (32, 1).  The data-dependent row range is replaced
    by a superset (Section 2.1.1): ``T`` chunks of 32 nonzeros, all guards
    true.  Chunk ``k`` (the segment variable):

    F: R A_colInd[32k + tid], R A_val[32k + tid], W sm_k[tid], W sm_val[tid]
       [barrier]
    T: for kk in [0,32), kb in [0,K):  R sm_k[kk], R sm_val[kk], R B[kb][j],
       R C[i][j], W C[i][j]       (kb is the existential row index of B)
       [barrier]

    With ``kb_on_all = False`` only the read of B ranges over ``kb`` (the
    relation of Section 2.1.2 quantifies k in the B read alone); the other
    T accesses loop over ``kk`` only.  The races are the same either way:
    only the number of repeated reads differs.
    """
    assert N % 32 == 0
    tag = f"gespmm-crc-M{M}-N{N}-T{T}" + ("" if kb_on_all else f"-K{K}")
    tag += ("" if middle_barrier else "-nomid") + ("" if trailing_barrier else "-notrail")
    b = Builder((32, 1), (M, N // 32), tag)
    colInd = b.array(GLOBAL, (32 * T,), "A_colInd")
    val = b.array(GLOBAL, (32 * T,), "A_val")
    Bm = b.array(GLOBAL, (K, N), "B")
    Cm = b.array(GLOBAL, (M, N), "C")
    sm_k = b.array(SHARED, (32,), "sm_k")
    sm_v = b.array(SHARED, (32,), "sm_val")
    f_acc = [
        rw(colInd, False, aff(k=32, tx=1), name="R A_colInd[ptr+tid]"),
        rw(val, False, aff(k=32, tx=1), name="R A_val[ptr+tid]"),
        rw(sm_k, True, aff(tx=1), name="W sm_k[tid]"),
        rw(sm_v, True, aff(tx=1), name="W sm_val[tid]"),
    ]
    loops = ((0, 32), (0, K))
    lk = loops if kb_on_all else ((0, 32),)
    t_acc = [
        rw(sm_k, False, aff(l0=1), loops=lk, name="R sm_k[kk]"),
        rw(sm_v, False, aff(l0=1), loops=lk, name="R sm_val[kk]"),
        rw(Bm, False, aff(l1=1), aff(by=32, tx=1), loops=loops, name="R B[kb][j]"),
        rw(Cm, False, aff(bx=1), aff(by=32, tx=1), loops=lk, name="R C[i][j]"),
        rw(Cm, True, aff(bx=1), aff(by=32, tx=1), loops=lk, name="W C[i][j]"),
    ]
    pf = b.phase(f_acc, barrier_after=middle_barrier)
    pt = b.phase(t_acc, barrier_after=trailing_barrier)
    b.segment([pf, pt], repeat=T)
    return b.build()


# Sizes of the Ge-SpMM staging benchmark: (M rows, N columns, T chunks of 32
# nonzeros per row, K candidate rows of B).  Every row holds the superset of
# T chunks (Section 2.1.1), so a size is a record count, not a sparsity
# pattern; the largest barrier interval stays below 2^32 instances.
GESPMM_SWEEP = ((1024, 64, 4, 8), (4096, 128, 4, 16), (16384, 256, 2, 8), (65536, 64, 8, 4))


# ------------------------------------------------------ textbook patterns
def stride1_shared(block=(64, 2), grid=(3, 2)) -> KernelDesc:
    b = Builder(block, grid, "stride1-shared")
    s = b.array(SHARED, (block[1], block[0]), "s")
    p = b.phase([rw(s, True, aff(ty=1), aff(tx=1))], barrier_after=False)
    b.segment([p])
    return b.build()


def stride1_global(block=(64, 2), grid=(3, 2)) -> KernelDesc:
    bx, by = block
    gx, gy = grid
    tpb = bx * by
    b = Builder(block, grid, "stride1-global")
    g = b.array(GLOBAL, (gx * gy * tpb,), "g")
    # gthread = (by*gx + bx) * tpb + ty*bdx + tx
    p = b.phase([rw(g, True, aff(by=gx * tpb, bx=tpb, ty=bx, tx=1))], barrier_after=False)
    b.segment([p])
    return b.build()


def half_index_shared(block=128, grid=4) -> KernelDesc:
    b = Builder((block, 1), (grid, 1), "half-index-shared")
    a = b.array(SHARED, (block // 2,), "a")
    p = b.phase([rw(a, True, aff(aux0=1), aux=(Aux(AUX_FLOORDIV, 2, aff(tx=1)), Aux()))],
                barrier_after=False)
    b.segment([p])
    return b.build()


def half_index_global(block=128, grid=4) -> KernelDesc:
    b = Builder((block, 1), (grid, 1), "half-index-global")
    a = b.array(GLOBAL, (block * grid // 2,), "a")
    e = aff(bx=block, tx=1)
    p = b.phase([rw(a, True, aff(aux0=1), aux=(Aux(AUX_FLOORDIV, 2, e), Aux()))],
                barrier_after=False)
    b.segment([p])
    return b.build()
