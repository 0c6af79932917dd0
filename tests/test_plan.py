"""The tile plan (top_plan_tiles, host only): how one sweep's per-segment solves are laid out in
workgroup tiles, checked against rules stated independently of the packing code.

- every segment is solved exactly once (one core lane), halo lanes are copies;
- a trajectory of at most tile_lanes segments sits whole, in order, in one tile; those tiles are
  filled first-fit in decreasing length (each trajectory did not fit any earlier tile at the moment
  it was placed), so at most one of them is half full or less;
- a longer trajectory runs over consecutive tiles whose cores partition it, each core flanked by
  exactly `halo` copies on each side that has a neighbour;
- the chain table (several halo epochs in one launch) exists exactly when every halo copy and the
  segment before it are in the published edge of a neighbouring tile, which for this tiling has the
  closed form: no split trajectory has a middle tile, or tile_lanes >= 3 halo + 1.
"""
import ctypes

import numpy as np
import pytest

from paper_2507_10290_amd import binding
from paper_2507_10290_amd.binding import TOP_E_INVALID, TOP_HALO_BIT, TopError, top_plan_tiles
from paper_2507_10290_amd.workloads import make_config

SEG_MASK = TOP_HALO_BIT - 1


def _offsets(lengths):
    return np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)


def _check_plan(lengths, W, halo):
    off = _offsets(lengths)
    S = int(off[-1])
    info, lanes, chain, tail = top_plan_tiles(off, W, halo)
    assert info["tail_tiles"] == 0 and tail.shape[0] == 0
    assert info["tile_lanes"] == W and info["n_seg"] == S and info["n_traj"] == len(lengths)
    assert lanes.shape == (info["n_tiles"], W)
    assert info["used_lanes"] == int((lanes >= 0).sum())
    traj_of = np.repeat(np.arange(len(lengths)), lengths)

    # every segment has exactly one core lane
    core_count = np.zeros(S, dtype=np.int64)
    for t in range(info["n_tiles"]):
        for x in lanes[t]:
            if x >= 0 and not (x & TOP_HALO_BIT):
                core_count[x] += 1
    assert (core_count == 1).all()

    # occupied lanes form one prefix per tile; segments of a tile run in order within a trajectory
    tiles_of = {}
    for t in range(info["n_tiles"]):
        row = lanes[t]
        occ = row >= 0
        n = int(occ.sum())
        assert occ[:n].all() and not occ[n:].any(), t
        segs = row[:n] & SEG_MASK
        for b in np.unique(traj_of[segs]):
            tiles_of.setdefault(int(b), []).append(t)
            run = segs[traj_of[segs] == b]
            assert (np.diff(run) == 1).all(), (t, b)

    long_traj = [b for b, n in enumerate(lengths) if n > W]
    assert info["halo"] == (halo if long_traj else 0)

    # short trajectories: whole in one tile, no copies; first-fit in decreasing length
    short_tiles = sorted({t for b, n in enumerate(lengths) if n <= W for t in tiles_of[b]})
    for b, n in enumerate(lengths):
        if n <= W:
            assert len(tiles_of[b]) == 1
            row = lanes[tiles_of[b][0]]
            assert not (row[row >= 0] & TOP_HALO_BIT).any()
    order = sorted((b for b, n in enumerate(lengths) if n <= W), key=lambda b: (-lengths[b], b))
    index = {t: j for j, t in enumerate(short_tiles)}
    content = {t: [] for t in short_tiles}
    fill = np.zeros(len(short_tiles), dtype=np.int64)
    for b in order:  # in placement order: b fits no tile before its own at that moment
        j = index[tiles_of[b][0]]
        assert (fill[:j] + lengths[b] > W).all(), b
        fill[j] += lengths[b]
        content[short_tiles[j]].append(b)
    assert (fill <= W).all()
    fills = list(fill)
    assert sum(2 * f <= W for f in fills) <= 1
    # first trajectories of consecutive short tiles are non-increasing in length
    firsts = [lengths[content[t][0]] for t in short_tiles]
    assert firsts == sorted(firsts, reverse=True)

    # long trajectories: consecutive tiles, cores partition the trajectory, `halo` copies per side
    middle = False
    for b in long_traj:
        ts = tiles_of[b]
        assert ts == list(range(ts[0], ts[0] + len(ts))) and len(ts) >= 2
        next_core = int(off[b])
        for k, t in enumerate(ts):
            row = lanes[t]
            segs = row[row >= 0]
            assert (traj_of[segs & SEG_MASK] == b).all()
            is_halo = (segs & TOP_HALO_BIT) != 0
            n_left = int(np.argmax(~is_halo))
            n_right = int(np.argmax(~is_halo[::-1]))
            assert n_left == (halo if k > 0 else 0), (b, t)
            assert n_right == (halo if k < len(ts) - 1 else 0), (b, t)
            assert not is_halo[n_left:len(segs) - n_right].any()
            core = segs[n_left:len(segs) - n_right]
            assert core[0] == next_core
            next_core = int(core[-1]) + 1
            if k < len(ts) - 1:
                assert len(segs) == W
            if 0 < k < len(ts) - 1:
                middle = True
        assert next_core == int(off[b + 1])

    # chain table against the published-edge rule, lane by lane, and its closed form
    expect_chain = bool(long_traj) and (not middle or W >= 3 * halo + 1)
    assert info["chained"] == int(expect_chain)
    if long_traj:
        assert _chain_rule_holds(lanes, off, halo) == expect_chain
    if expect_chain:
        assert chain.shape == (info["n_tiles"], 4)
        for t in range(info["n_tiles"]):
            row = lanes[t]
            core_lanes = np.nonzero((row >= 0) & ((row & TOP_HALO_BIT) == 0))[0]
            left = row[0] >= 0 and bool(row[0] & TOP_HALO_BIT)
            last = row[row >= 0][-1]
            right = bool(last & TOP_HALO_BIT)
            assert list(chain[t]) == [t - 1 if left else -1, t + 1 if right else -1,
                                      core_lanes[0], core_lanes[-1] + 1], t
    else:
        assert chain.shape == (0, 4)
    return info, lanes, chain


def _chain_rule_holds(lanes, off, halo):
    """Every halo copy of tile t is a core segment of the neighbour on its side, within `halo` of a
    core edge of that neighbour that has a neighbour itself (one more on the right edge), and the
    segment before it (unless the copy starts its trajectory) is likewise published by t or a
    neighbour."""
    n_tiles, W = lanes.shape
    S = int(off[-1])
    owner = -np.ones(S, dtype=np.int64)
    pos = -np.ones(S, dtype=np.int64)
    edges = []
    for t in range(n_tiles):
        row = lanes[t]
        core = np.nonzero((row >= 0) & ((row & TOP_HALO_BIT) == 0))[0]
        owner[row[core]] = t
        pos[row[core]] = core
        has_l = row[0] >= 0 and bool(row[0] & TOP_HALO_BIT)
        has_r = bool(row[row >= 0][-1] & TOP_HALO_BIT)
        edges.append((has_l, has_r, core[0], core[-1] + 1))
    first = set(int(x) for x in off[:-1])

    def published(s):
        t = owner[s]
        has_l, has_r, lo, hi = edges[t]
        return (has_l and pos[s] < lo + halo) or (has_r and pos[s] >= hi - halo - 1)

    for t in range(n_tiles):
        row = lanes[t]
        has_l, has_r, lo, hi = edges[t]
        for i, x in enumerate(row):
            if x < 0 or not (x & TOP_HALO_BIT):
                continue
            s = int(x & SEG_MASK)
            side = t - 1 if i < lo else t + 1
            if owner[s] != side or not published(s):
                return False
            if s not in first and (owner[s - 1] not in (t - 1, t, t + 1) or not published(s - 1)):
                return False
    return True


@pytest.mark.parametrize("W,halo", [(64, 8), (64, 21), (64, 22), (128, 16), (256, 32), (320, 32), (512, 32),
                                    (512, 170), (512, 171), (128, 63)])
def test_random_batches(W, halo):
    rng = np.random.default_rng(W * 1000 + halo)
    for trial in range(4):
        B = int(rng.integers(1, 60))
        kind = rng.integers(0, 3, size=B)
        lengths = np.where(kind == 0, rng.integers(1, W + 1, size=B),
                           np.where(kind == 1, rng.integers(1, 17, size=B), rng.integers(W + 1, 6 * W, size=B)))
        _check_plan([int(x) for x in lengths], W, halo)


@pytest.mark.parametrize("lengths,W,halo", [
    ([1], 64, 1),                       # one segment
    ([64], 64, 8),                      # exactly one tile
    ([65], 64, 8),                      # one more: two tiles, the last core halo + 1
    ([64 + 64 - 16 + 1], 64, 8),        # three tiles, a middle one
    ([1] * 200, 64, 8),                 # many one-segment trajectories
    ([63, 1, 62, 2, 33, 31], 64, 4),    # pairs that fill tiles exactly
    ([300, 1, 2, 63, 64, 65], 64, 24),  # cores shorter than halo + 1: not chained
    ([300, 1, 2, 63, 64, 65], 64, 21),  # W = 3 halo + 1: chained
])
def test_edge_cases(lengths, W, halo):
    _check_plan(lengths, W, halo)


def test_exact_fill_and_tile_counts():
    info, lanes, _ = _check_plan([32] * 16, 64, 8)
    assert info["n_tiles"] == 8 and info["used_lanes"] == 512
    # a trajectory of N > W segments takes 1 + ceil((N - W) / (W - 2 halo)) tiles
    for N, W, h in [(65, 64, 8), (1000, 64, 8), (67259, 512, 32), (5000, 128, 60)]:
        info, _, _ = _check_plan([N], W, h)
        assert info["n_tiles"] == 1 + -(-(N - W) // (W - 2 * h)), (N, W, h)


@pytest.mark.parametrize("i", [2, 3])
def test_benchmark_shapes(i):
    # the 65,536-segment trajectory and the 4,096-trajectory batch at their full sizes
    w = make_config(i)
    lengths = [int(x) for x in np.diff(w.seg_offsets)]
    _check_plan(lengths, 512, 32)
    _check_plan(lengths, 320, 32)


def test_argument_errors():
    off = _offsets([10, 20])
    for W, h in [(0, 1), (96, 8), (1024, 8), (64, 0), (64, 32), (128, 64)]:
        with pytest.raises(TopError) as ei:
            top_plan_tiles(off, W, h)
        assert ei.value.status == TOP_E_INVALID, (W, h)
    for bad in ([1, 10], [0, 5, 5], [0, 7, 3]):
        with pytest.raises(TopError) as ei:
            top_plan_tiles(np.array(bad, dtype=np.int64), 64, 8)
        assert ei.value.status == TOP_E_INVALID
    # arrays smaller than the plan are refused, and nothing is written to them
    L = binding.lib()
    off = _offsets([100])
    offp = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    info = binding.TopPlanInfo()
    assert L.top_plan_tiles(1, offp, 64, 8, 0, 0, None, 0, None, 0, ctypes.byref(info)) == 0
    lanes = np.full(info.n_tiles * 64 - 1, 7, dtype=np.int32)
    assert L.top_plan_tiles(1, offp, 64, 8, 0, 0, lanes.ctypes.data, lanes.size, None, 0,
                            ctypes.byref(info)) == TOP_E_INVALID
    assert (lanes == 7).all()
    chain = np.full(4 * info.n_tiles - 1, 7, dtype=np.int32)
    assert L.top_plan_tiles(1, offp, 64, 8, 0, 0, None, 0, chain.ctypes.data, chain.size,
                            ctypes.byref(info)) == TOP_E_INVALID
    assert (chain == 7).all()


def _batched_lengths(n=4096):
    # the batched workload's trajectory lengths: uniform in [8, 512]
    return [int(x) for x in np.random.Generator(np.random.PCG64(3)).integers(8, 512, size=n, endpoint=True)[:n]]


def test_tail_split():
    # 4,096 trajectories make 2,056 tiles of 512: eight rounds of 256 tiles and a ninth of 8.  With a
    # tail, the main plan keeps 2,048 of the tiles (in order); the trajectories of the other 8 --
    # those whose longest trajectory is shortest, then the least filled -- are repacked first-fit
    # decreasing into tail tiles as wide as that longest trajectory rounded up to 64.
    lengths = _batched_lengths()
    off = _offsets(lengths)
    base, blanes, _, _ = top_plan_tiles(off, 512, 32)
    info, lanes, chain, tail = top_plan_tiles(off, 512, 32, 256, 320)
    assert base["n_tiles"] == 2056 and info["n_tiles"] == 2048
    assert info["used_lanes"] == int((lanes >= 0).sum() + (tail >= 0).sum()) == off[-1]
    traj_of = np.repeat(np.arange(len(lengths)), lengths)
    # the kept tiles are base tiles, in order
    key = lambda row: (max(lengths[b] for b in np.unique(traj_of[row[row >= 0]])), int((row >= 0).sum()))
    kept, j = [], 0
    for i in range(base["n_tiles"]):
        if j < info["n_tiles"] and np.array_equal(blanes[i], lanes[j]):
            kept.append(i)
            j += 1
    assert j == info["n_tiles"]
    moved = sorted(set(range(base["n_tiles"])) - set(kept))
    assert len(moved) == 8
    assert max(key(blanes[i]) for i in moved) <= min(key(blanes[i]) for i in kept)
    # the tail holds exactly the moved tiles' trajectories, whole and in order
    msegs = np.concatenate([blanes[i][blanes[i] >= 0] for i in moved])
    assert np.array_equal(np.sort(tail[tail >= 0]), np.sort(msegs))
    longest = max(key(blanes[i])[0] for i in moved)
    assert info["tail_tile_lanes"] == (longest + 63) // 64 * 64 and tail.shape == (info["tail_tiles"], info["tail_tile_lanes"])
    fill = []
    for row in tail:
        n = int((row >= 0).sum())
        assert (row[:n] >= 0).all() and (row[n:] < 0).all() and not (row[:n] & TOP_HALO_BIT).any()
        for b in np.unique(traj_of[row[:n]]):
            seg = row[:n][traj_of[row[:n]] == b]
            assert len(seg) == lengths[b] and (np.diff(seg) == 1).all()
        fill.append(n)
    assert sum(2 * f <= info["tail_tile_lanes"] for f in fill) <= 1   # first fit: at most one half-full tile


@pytest.mark.parametrize("case", ["exact", "too_many", "split", "long_tail", "no_round"])
def test_no_tail_split(case):
    lengths = _batched_lengths(4080)                       # exactly 2,048 tiles of 512
    W, halo, rnd, tw = 512, 32, 256, 320
    if case == "too_many":
        lengths = _batched_lengths(4096)
        rnd = 32                                           # 2,056 = 64 rounds of 32 and 8: a quarter round
    elif case == "split":
        lengths = _batched_lengths(4096) + [2000]          # a trajectory longer than a tile: halo tiles
    elif case == "long_tail":
        lengths = _batched_lengths(4096)
        tw = 64                                            # the tail's trajectories do not fit its tiles
    elif case == "no_round":
        lengths = _batched_lengths(4096)
        rnd = 0
    off = _offsets(lengths)
    base, blanes, _, _ = top_plan_tiles(off, W, halo)
    info, lanes, _, tail = top_plan_tiles(off, W, halo, rnd, tw)
    assert info["tail_tiles"] == 0 and tail.shape[0] == 0
    assert info["n_tiles"] == base["n_tiles"] and np.array_equal(lanes, blanes)


def test_tail_argument_errors():
    off = _offsets([10, 20])
    for rnd, tw in [(-1, 320), (4, 0), (4, 96), (4, 384)]:
        with pytest.raises(TopError) as ei:
            top_plan_tiles(off, 64, 8, rnd, tw)
        assert ei.value.status == TOP_E_INVALID, (rnd, tw)
