"""Summation orders of the library's dot products, for bitwise comparisons.

Test infrastructure. The library sums every dot product in a fixed order that
depends only on sizes and launch shapes, and evaluates everything else (sparse
products, vector updates, Jacobi divisions, scalar recurrences) in the oracle's
order without contraction. Running the oracle with `oracle.bicgstab.dot`
replaced by one of the functions below therefore reproduces the library's
arithmetic bit for bit. Nothing here computes a step of the method: these are
models of summation order only, written from the kernels' documented reduction
structure (not shared with them).
"""
from __future__ import annotations

import contextlib

import numpy as np


def _pad_pow2(k):
    kp = 1
    while kp < k:
        kp *= 2
    return kp


def _wave_tree(t):
    """Pairwise tree over the last axis (the row slots of a wave): adjacent
    slots first; with an odd count the last slot passes up unpaired."""
    while t.shape[-1] > 1:
        odd = t.shape[-1] % 2
        pairs = t[..., 0:t.shape[-1] - odd:2] + t[..., 1::2]
        t = np.concatenate([pairs, t[..., -1:]], axis=-1) if odd else pairs
    return t[..., 0]


def group_dot(n, k, grid_cap=512, block=256, fin_lanes=16):
    """Dot of two length-n columns as a vector pass computes it: a grid of
    nb = min(grid_cap, ceil(n / (block / kp))) workgroups; thread (b, slot)
    sums rows b*rpb + slot + j*nb*rpb in order of j; the row slots of a wave
    by a pairwise tree; the waves of a workgroup in order; then the finalize
    kernel: lane g of `fin_lanes` sums workgroups g, g + fin_lanes, ... in
    order, and the lane sums are added in lane order."""
    kp = _pad_pow2(k)
    rpb = block // kp
    waves = block // 64
    slots = 64 // kp
    nb = max(1, min(grid_cap, -(-n // rpb)))
    stride = nb * rpb
    m = max(1, -(-n // stride))
    mb = -(-nb // fin_lanes)

    def dot(u, w):
        p = np.zeros(m * stride)
        p[:n] = np.multiply(u, w)
        acc = np.add.accumulate(p.reshape(m, nb, rpb), axis=0)[-1]   # (nb, rpb)
        wv = _wave_tree(acc.reshape(nb, waves, slots))                # (nb, waves)
        part = np.add.accumulate(wv, axis=1)[:, -1]                   # (nb,)
        q = np.zeros(mb * fin_lanes)
        q[:nb] = part
        lanes = np.add.accumulate(q.reshape(mb, fin_lanes), axis=0)[-1]
        return float(np.add.accumulate(lanes)[-1])

    return dot


def batched_dot(n, k, nw, block):
    """Dot of two length-n columns as the batched kernel computes it for a
    system of n rows and k columns on nw workgroups of `block` threads: a
    wave holds 64 // k rows of k lanes; per thread over its rows (a stride of
    (block / 64) * (64 // k) rows through the workgroup's contiguous chunk of
    ceil(n / nw) rows), a pairwise tree over the row slots of a wave (adjacent
    first, an odd last slot unpaired), the waves in order, then the
    workgroups in order."""
    slots, waves = 64 // k, block // 64
    rpp = waves * slots
    chunk = (n + nw - 1) // nw
    m = (chunk + rpp - 1) // rpp

    def dot(u, w):
        p = np.zeros(nw * chunk)
        p[:n] = np.multiply(u, w)
        q = np.zeros((nw, m * rpp))
        q[:, :chunk] = p.reshape(nw, chunk)
        acc = np.add.accumulate(q.reshape(nw, m, rpp), axis=1)[:, -1, :]
        wv = _wave_tree(acc.reshape(nw, waves, slots))
        wg = np.add.accumulate(wv, axis=1)[:, -1]
        return float(np.add.accumulate(wg)[-1])

    return dot


@contextlib.contextmanager
def oracle_dot(dotf):
    """Run the oracle with its dot product replaced by `dotf`."""
    import oracle.bicgstab as ob

    saved = ob.dot
    ob.dot = dotf
    try:
        yield
    finally:
        ob.dot = saved


def _spmm_cols_per_lane(k):
    """Columns per lane of the sparse product: two for even k, else one."""
    return 2 if k % 2 == 0 else 1


def spmm_row_blocks(row_ptr, k, block=256, nnz_max=4096, rows_max=1024):
    """Row blocks of the sparse product: contiguous rows, at most
    block * cpl * rpl / kp rows (cpl columns per lane; rows per lane rpl = 2
    when cpl = 2, else 8 for kp >= 8 and kp below) and nnz_max entries unless
    one row is longer."""
    kp = _pad_pow2(k)
    cpl = _spmm_cols_per_lane(k)
    rpl = 2 if cpl == 2 else (8 if kp >= 8 else kp)
    target = max(1, min(rows_max, block * cpl * rpl // kp))
    n = len(row_ptr) - 1
    blk, r0 = [0], 0
    while r0 < n:
        r = r0 + 1
        while r < n and r - r0 < target and row_ptr[r + 1] - row_ptr[r0] <= nnz_max:
            r += 1
        blk.append(r)
        r0 = r
    return blk


def tile_order(grid, tile):
    """Rows of a natural-order nz x ny x nx grid (x fastest) in the order
    of a tile-by-tile copy: tiles of tz x ty x tx points in the natural order
    of their first point, the points of a tile in natural order within it."""
    nz, ny, nx = grid
    tz, ty, tx = tile
    z, y, x = np.meshgrid(np.arange(tz), np.arange(ty), np.arange(tx), indexing="ij")
    inner = ((z * ny + y) * nx + x).ravel()
    Z, Y, X = np.meshgrid(np.arange(0, nz, tz), np.arange(0, ny, ty), np.arange(0, nx, tx), indexing="ij")
    corner = ((Z * ny + Y) * nx + X).ravel()
    return (corner[:, None] + inner[None, :]).ravel()


def spmm_epilogue_dot(row_ptr, k, block=256, runs_max=256, fin_lanes=16, perm=None):
    """Dot of two length-n columns as the product's epilogue forms it: in row
    block L, row slot s (a group of kp / cpl lanes) sums rows
    r0 + s + j * (block * cpl / kp) in order of j; the row slots of a wave by a
    pairwise tree; the waves in order; then the G = min(#blocks, runs_max)
    runs of consecutive blocks in block order; then the finalize kernel's
    lanes over the runs. perm: the stored order of the rows when the matrix
    is kept permuted (row i of the copy is row perm[i]); the blocks and sums
    then run over the stored rows."""
    if perm is not None:
        perm = np.asarray(perm)
        cnt = np.diff(np.asarray(row_ptr))[perm]
        row_ptr = np.concatenate(([0], np.cumsum(cnt)))
        inner = spmm_epilogue_dot(row_ptr, k, block, runs_max, fin_lanes)
        return lambda u, w: inner(np.asarray(u)[perm], np.asarray(w)[perm])
    kp = _pad_pow2(k)
    cpl = _spmm_cols_per_lane(k)
    rpp, slots, waves = block * cpl // kp, 64 * cpl // kp, block // 64
    blk = spmm_row_blocks(row_ptr, k, block)
    nb = len(blk) - 1
    G = max(1, min(nb, runs_max))
    mg = -(-G // fin_lanes)

    sizes = np.diff(np.asarray(blk))
    uniform = nb > 0 and bool(np.all(sizes == sizes[0])) and sizes[0] % rpp == 0

    def block_partials(p):
        if uniform:
            # every block holds m whole passes of rpp rows: the same sums as
            # the loop below, for all blocks at once
            m = int(sizes[0]) // rpp
            acc = np.add.accumulate(p.reshape(nb, m, rpp), axis=1)[:, -1, :]
            wv = _wave_tree(acc.reshape(nb, waves, slots))
            return np.add.accumulate(wv, axis=1)[:, -1]
        part = np.zeros(nb)
        for L in range(nb):
            r0, r1 = blk[L], blk[L + 1]
            m = -(-(r1 - r0) // rpp)
            q = np.zeros(m * rpp)
            q[: r1 - r0] = p[r0:r1]
            acc = np.add.accumulate(q.reshape(m, rpp), axis=0)[-1]
            wv = _wave_tree(acc.reshape(waves, slots))
            part[L] = np.add.accumulate(wv)[-1]
        return part

    def dot(u, w):
        part = block_partials(np.multiply(u, w))
        runs = np.zeros(mg * fin_lanes)
        for g in range(G):
            b0, b1 = nb * g // G, nb * (g + 1) // G
            runs[g] = np.add.accumulate(np.concatenate(([0.0], part[b0:b1])))[-1]
        lanes = np.add.accumulate(runs.reshape(mg, fin_lanes), axis=0)[-1]
        return float(np.add.accumulate(lanes)[-1])

    return dot


def scheduled_dot(first, cycle):
    """A dot product that applies the functions of `first` to the first calls
    in order and then those of `cycle` round and round (the passes of a plan
    form their dots in a fixed sequence)."""
    state = {"i": 0}

    def dot(u, w):
        i = state["i"]
        state["i"] = i + 1
        f = first[i] if i < len(first) else cycle[(i - len(first)) % len(cycle)]
        return f(u, w)

    return dot


def host_dot(n, threads):
    """Dot of two length-n columns as the host executor sums it: range t of
    `threads` holds rows [n t / T, n (t+1) / T) and sums them in row order
    from 0; the range sums are added in order from 0."""
    bounds = [n * t // threads for t in range(threads + 1)]

    def dot(u, w):
        p = np.multiply(u, w)
        parts = [np.add.accumulate(np.concatenate(([0.0], p[bounds[t]:bounds[t + 1]])))[-1] for t in range(threads)]
        return float(np.add.accumulate(np.concatenate(([0.0], parts)))[-1])

    return dot
