"""CPU checks of the summation-order models in kernel_order.py: the
vectorised path of the product-epilogue dot (row blocks of equal length)
against a plain loop over blocks, row slots and waves."""
import numpy as np

from kernel_order import _pad_pow2, _wave_tree, spmm_epilogue_dot, spmm_row_blocks, tile_order
from workloads import conv_diff, random_sparse


def _loop_epilogue_dot(row_ptr, k, u, w, block=256, runs_max=256, fin_lanes=16):
    kp = _pad_pow2(k)
    cpl = 2 if k % 2 == 0 else 1
    rpp, slots, waves = block * cpl // kp, 64 * cpl // kp, block // 64
    blk = spmm_row_blocks(row_ptr, k, block)
    nb = len(blk) - 1
    p = u * w
    part = []
    for L in range(nb):
        r0, r1 = blk[L], blk[L + 1]
        slot_sums = np.zeros(rpp)
        for s in range(rpp):
            acc = 0.0
            for r in range(r0 + s, r1, rpp):
                acc += p[r]
            slot_sums[s] = acc
        wave = _wave_tree(slot_sums.reshape(waves, slots))
        tot = 0.0
        for x in wave:
            tot += x
        part.append(tot)
    G = max(1, min(nb, runs_max))
    runs = []
    for g in range(G):
        acc = 0.0
        for b in range(nb * g // G, nb * (g + 1) // G):
            acc += part[b]
        runs.append(acc)
    lanes = [0.0] * fin_lanes
    for i, v in enumerate(runs):
        lanes[i % fin_lanes] += v
    tot = 0.0
    for v in lanes:
        tot += v
    return tot


def test_epilogue_dot_uniform_and_ragged_blocks():
    rng = np.random.default_rng(4)
    for A, k in ((conv_diff(16, 3, (1.0, 0.7, 0.3)), 32), (conv_diff(16, 3, (1.0, 0.7, 0.3)), 5),
                 (conv_diff(13, 3, (0.3, 0.2, 0.1)), 32), (random_sparse(3001, 9, seed=1), 8)):
        u, w = rng.uniform(-1, 1, A.n), rng.uniform(-1, 1, A.n)
        assert spmm_epilogue_dot(A.row_ptr, k)(u, w) == _loop_epilogue_dot(A.row_ptr, k, u, w)


def test_tile_order_and_permuted_epilogue_dot():
    """The tile order is a permutation whose first block is the first tile
    (z, y, x nested in that order); the permuted epilogue dot equals the
    plain loop over the permuted rows."""
    g, t = (4, 8, 8), (2, 4, 4)
    perm = tile_order(g, t)
    assert sorted(perm.tolist()) == list(range(4 * 8 * 8))
    first = [(z * 8 + y) * 8 + x for z in range(2) for y in range(4) for x in range(4)]
    assert perm[:32].tolist() == first
    assert perm[32:36].tolist() == [4, 5, 6, 7]  # the next tile along x
    A = conv_diff(8, 3, (1.0, 0.7, 0.3))
    perm = tile_order((8, 8, 8), t)
    rng = np.random.default_rng(9)
    u, w = rng.uniform(-1, 1, A.n), rng.uniform(-1, 1, A.n)
    rp = np.concatenate(([0], np.cumsum(np.diff(A.row_ptr)[perm])))
    assert spmm_epilogue_dot(A.row_ptr, 32, perm=perm)(u, w) == _loop_epilogue_dot(rp, 32, u[perm], w[perm])


def _loop_batched_dot(n, k, nw, block, u, w):
    """The batched kernel's dot order written out lane by lane: lane l of
    wave q holds row slot l // k, column l % k (lanes past 64 // k whole rows
    idle); each thread adds its rows in order; the shuffle tree adds slot
    s + off into slot s when s is a multiple of 2 off and s + off < 64 // k;
    the waves and then the workgroups are added in order."""
    rpw = 64 // k
    waves = block // 64
    rpp = waves * rpw
    chunk = -(-n // nw)
    p = u * w
    tot = 0.0
    for g in range(nw):
        r0, r1 = min(n, g * chunk), min(n, (g + 1) * chunk)
        wave_sums = []
        for q in range(waves):
            lanes = [0.0] * rpw
            for s in range(rpw):
                for r in range(r0 + q * rpw + s, r1, rpp):
                    lanes[s] += p[r]
            off = 1
            while off < rpw:
                for s in range(0, rpw, 2 * off):
                    if s + off < rpw:
                        lanes[s] = lanes[s] + lanes[s + off]
                off *= 2
            wave_sums.append(lanes[0])
        v = wave_sums[0]
        for x in wave_sums[1:]:
            v += x
        tot += v
    return tot


def test_batched_dot_model_matches_lane_loop():
    from kernel_order import batched_dot

    rng = np.random.default_rng(3)
    for k in range(1, 9):
        for n, nw, block in ((1000, 3, 256), (4093, 5, 512), (777, 1, 1024)):
            u = rng.standard_normal(n)
            w = rng.standard_normal(n)
            assert batched_dot(n, k, nw, block)(u, w) == _loop_batched_dot(n, k, nw, block, u, w), (k, n, nw, block)
