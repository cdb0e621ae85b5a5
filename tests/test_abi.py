"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/idm.h declares, validates problems, sizes workspaces
and packs lanes into work-group bundles correctly."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2412_16750_amd import _lib
    return _lib.load()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "idm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(idm_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    from paper_2412_16750_amd import _lib
    assert sorted(_lib.EXPORTS) == names


def _problem(offsets, S=100, K=16, delta=4.0, dt=0.1, bound=0, a_min=-10.0, gap_floor=1e-3):
    from paper_2412_16750_amd._lib import IdmProblem
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32))
    pb = IdmProblem(int(off[-1]), len(off) - 1, S, K, dt, delta, a_min, gap_floor, bound,
                    off.ctypes.data_as(ctypes.c_void_p))
    return pb, off


def _check(L, offsets, tuning=None, **kw):
    from paper_2412_16750_amd._lib import IdmPlanInfo, IdmTuning
    pb, off = _problem(offsets, **kw)
    info = IdmPlanInfo()
    ws = ctypes.c_size_t()
    tu = IdmTuning(*tuning) if tuning else None
    st = L.idm_problem_check(ctypes.byref(pb), ctypes.byref(tu) if tu else None, ctypes.byref(info),
                             ctypes.byref(ws))
    return st, info, ws.value


def test_valid_problem_shape_and_workspace(L):
    off = np.arange(0, 2000 * 1000 + 1, 1000)
    st, info, ws = _check(L, off, S=100, K=32)
    assert st == 0
    assert (info.threads, info.per_thread, info.ckpt_every, info.block) == (1024, 1, 32, 16)
    assert info.n_bundles == 2000 and info.max_lane == 1000
    assert abs(info.fill - 1000 / 1024) < 1e-12
    N, S, K = 2_000_000, 100, 32
    align = lambda x: (x + 255) // 256 * 256
    # loss partials, diagnostic counts (two per bundle), fit gradients, checkpoints
    expect = (align(8 * 2000) + align(16 * 2000) + align(8 * 7 * N)
              + align(((S + K - 1) // K) * 2 * 4 * N))
    assert ws == expect


@pytest.mark.parametrize("case, status", [
    (dict(offsets=[0, 5, 3, 10]), -2),            # decreasing
    (dict(offsets=[1, 5]), -2),                   # does not start at 0
    (dict(offsets=[0, 5000], K=12), -3),          # pieces need 1 vehicle/thread; K=12 needs 4
    (dict(offsets=[0, 10], delta=2.0), -3),       # only delta = 4
    (dict(offsets=[0, 10], dt=0.0), -1),
    (dict(offsets=[0, 10], dt=float("nan")), -1),
    (dict(offsets=[0, 10], a_min=1.0), -1),
    (dict(offsets=[0, 10], gap_floor=-1.0), -1),
    (dict(offsets=[0, 10], bound=7), -1),
    (dict(offsets=[0, 10], S=-1), -1),
    (dict(offsets=[0, 10], K=-3), -1),
    (dict(offsets=[0, 10], K=6), -3),             # no backward block divides K
    (dict(offsets=[0, (1 << 29) + 1]), -1),       # N above IDM_MAX_VEHICLES
    (dict(offsets=[0, 10], S=(1 << 27) + 1), -1),  # S above IDM_MAX_STEPS
])
def test_invalid_problems_are_rejected(L, case, status):
    st, _, _ = _check(L, **case)
    assert st == status
    assert len(L.idm_last_error()) > 0


def test_invalid_tuning(L):
    assert _check(L, [0, 100], tuning=(100, 1, 0, 0))[0] == -3
    assert _check(L, [0, 100], tuning=(64, 3, 0, 0))[0] == -3
    st, info, _ = _check(L, [0, 100], tuning=(64, 1, 0, 0))    # 100 > 64 slots: two pieces
    assert st == 0 and (info.n_levels, info.n_boundaries, info.n_bundles) == (2, 1, 2)
    assert _check(L, [0, 200], tuning=(64, 2, 0, 0))[0] == -3   # pieces need 1 vehicle/thread
    assert _check(L, [0, 100], tuning=(128, 1, 0, -1))[0] == -1
    assert _check(L, [0, 100], tuning=(64, 4, 32, 0, 16))[0] == -3  # block 16 not for R=4
    assert _check(L, [0, 100], tuning=(128, 1, 24, 0, 16))[0] == -3  # 16 does not divide 24
    assert _check(L, [0, 100], tuning=(128, 1, 0, 0, -1))[0] == -1
    st, info, _ = _check(L, [0, 100], tuning=(64, 4, 32, 0))
    assert st == 0 and (info.per_thread, info.ckpt_every, info.block) == (4, 32, 8)
    st, info, _ = _check(L, [0, 100], tuning=(64, 2, 8, 0))
    assert st == 0 and (info.threads, info.per_thread, info.ckpt_every, info.block) == (64, 2, 8, 8)
    # K = 12: only 4 vehicles per thread (block 4) divides it
    st, info, _ = _check(L, [0, 10], K=12)
    assert st == 0 and (info.per_thread, info.block) == (4, 4)
    st, info, _ = _check(L, [0, 10], K=48)
    assert st == 0 and (info.per_thread, info.block) == (1, 16)


def test_store_states_workspace_and_limits(L):
    """A plan that keeps every step's states: the workspace has no
    checkpoints and holds (S+1) x N displacements and speeds; lanes cut into
    pieces and values other than 0, 1 and 2 (the autotuner chooses; the
    plan starts with checkpoints) are rejected."""
    off = np.arange(0, 2000 * 1000 + 1, 1000)
    N, S, K = 2_000_000, 100, 32
    align = lambda x: (x + 255) // 256 * 256
    st, info, ws = _check(L, off, tuning=(0, 0, 0, 0, 0, 1), S=S, K=K)
    assert st == 0 and info.store_states == 1 and info.n_boundaries == 0
    expect = (align(8 * 2000) + align(16 * 2000) + align(8 * 7 * N)
              + 2 * align((S + 1) * 4 * N))
    assert ws == expect
    st, info, _ = _check(L, off, tuning=(0, 0, 0, 0, 0, 0), S=S, K=K)
    assert st == 0 and info.store_states == 0
    # a 1500-vehicle lane needs a 1024-slot bundle cut in two
    st, _, _ = _check(L, [0, 1500, 1600], tuning=(0, 0, 0, 0, 0, 1))
    assert st == -3 and b"pieces" in L.idm_last_error()
    assert _check(L, [0, 100], tuning=(0, 0, 0, 0, 0, 3))[0] == -1
    st, info, _ = _check(L, [0, 100], tuning=(0, 0, 0, 0, 0, 2))   # the autotuner chooses
    assert st == 0 and info.store_states == 0


def _tile_layout(L, offsets, threads, J, K=16, S=100):
    """Both slot tables of a halo-tile plan: [2][tiles][threads] (forward, then
    backward)."""
    from paper_2412_16750_amd._lib import IdmTuning
    tuning = (threads, 1, K, 0, 0, 1, J)
    st, info, ws = _check(L, offsets, tuning=tuning, S=S, K=K)
    assert st == 0, L.idm_last_error()
    assert info.tile_steps == J and info.store_states == 1 and info.n_levels == 1
    pb, off = _problem(offsets, S=S, K=K)
    tu = IdmTuning(*tuning)
    n = 2 * info.n_slots
    gidx = np.empty(n, dtype=np.int32)
    flags = np.empty(n, dtype=np.uint8)
    args = (ctypes.byref(pb), ctypes.byref(tu), gidx.ctypes.data_as(ctypes.c_void_p),
            flags.ctypes.data_as(ctypes.c_void_p))
    assert L.idm_problem_layout(*args, n - 1) == -1
    assert L.idm_problem_layout(*args, n) == 0
    nt = info.n_bundles
    return info, ws, gidx.reshape(2, nt, threads), flags.reshape(2, nt, threads)


@pytest.mark.parametrize("threads, J, K", [(256, 64, 16), (512, 128, 32), (256, 32, 16),
                                           (1024, 256, 32), (512, 64, 64), (768, 256, 32),
                                           (640, 256, 32), (576, 128, 32)])
def test_halo_tile_layout(L, threads, J, K):
    """Halo tiles (Sec. III-B: a step moves information one vehicle).  In each
    direction every vehicle is owned by exactly one tile.  Lanes of at most
    `threads` vehicles share tiles, packed best-fit decreasing: such a tile is
    the same in both tables, holds whole lanes one after another (head and
    tail flags exact, every vehicle owned), and any two of them together would
    overflow a work-group (when the later one was opened, the earlier lacked
    room for its first lane).  A longer lane is cut into m = ceil((n - J) /
    (threads - 1 - J)) tiles of its own, tile b of the forward and of the
    backward on the same lane; a cut tile's owned vehicles are consecutive; its
    forward slots are up to J vehicles ahead (fewer only where the lane starts,
    the first slot flagged as a lane head) and the owned ones; its backward
    slots the owned ones and up to J behind (fewer only where the lane ends,
    flagged as a head only on a true lane head); its slot counts within one of
    each other in each direction and at most threads - 1 (the slot after a cut
    tile's last vehicle is padding, whose contribution to a lane tail the
    backward's last thread gathers).  The workspace adds the carried adjoints
    and sums (68 B per vehicle) to the kept states."""
    import scenarios
    sizes = scenarios.lognormal_lane_sizes(300, np.log(threads) + 0.3, 1.0, 1, 6 * threads, 41)
    # lane 40: n + (m - 1) J divisible by m with T slots per tile (a tile
    # would exactly fill its work-group without the T - 1 cap)
    sizes[[2, 9, 17, 30, 31, 40]] = [threads, threads + 1, 5 * threads, threads - J,
                                     2 * threads - J, 3 * threads - 2 * J]
    # short lanes to share tiles, two of which fill one exactly
    sizes[[50, 51, 52, 53, 54]] = [1, 2, threads // 2, threads // 2, 3]
    sizes[::37] = 0
    off = scenarios.offsets_from_sizes(sizes)
    S = 100
    info, ws, gidx, flags = _tile_layout(L, off, threads, J, K=K, S=S)
    N = int(off[-1])
    sz = np.asarray(sizes, dtype=np.int64)
    need = np.where(sz > threads, -(-(sz - J) // (threads - 1 - J)), 0)
    lane_of = np.repeat(np.arange(len(sizes)), sizes)
    owned = {0: [], 1: []}
    tiles_of_lane = np.zeros(len(sizes), dtype=np.int64)
    whole_seen = np.zeros(len(sizes), dtype=np.int64)
    shared_fill = []
    counts = {}
    for b in range(info.n_bundles):
        g0 = gidx[0, b]
        if sz[lane_of[g0[0]]] <= threads:
            # a shared tile of whole lanes
            assert np.array_equal(gidx[0, b], gidx[1, b]) and np.array_equal(flags[0, b], flags[1, b])
            k = int(np.sum(g0 >= 0))
            assert 1 <= k <= threads
            assert np.all(g0[k:] == -1) and np.all(flags[0, b, k:] == 0)
            i = 0
            while i < k:
                lane = lane_of[g0[i]]
                ls, le = int(off[lane]), int(off[lane + 1])
                assert g0[i] == ls and le - ls <= threads
                seg, f = g0[i:i + le - ls], flags[0, b, i:i + le - ls]
                assert np.array_equal(seg, np.arange(ls, le))
                assert np.all((f & 8) != 0) and np.all((f & 4) != 0)   # owned, valid
                assert np.array_equal(np.nonzero(f & 1)[0], [0])          # head
                assert np.array_equal(np.nonzero(f & 2)[0], [le - ls - 1])  # tail
                whole_seen[lane] += 1
                i += le - ls
            for d in (0, 1):
                owned[d].append(g0[:k])
            shared_fill.append(k)
            continue
        lanes = []
        for d in (0, 1):
            g, f = gidx[d, b], flags[d, b]
            k = int(np.sum(g >= 0))
            assert 1 <= k <= threads - 1
            assert np.all(g[k:] == -1) and np.all(f[k:] == 0)
            seg = g[:k]
            assert np.array_equal(seg, np.arange(seg[0], seg[0] + k))
            lane = lane_of[seg[0]]
            assert lane_of[seg[-1]] == lane and sz[lane] > threads
            lanes.append(lane)
            ls, le = off[lane], off[lane + 1]
            own = seg[(f[:k] & 8) != 0]
            assert len(own) >= 1
            lo, hi = int(own[0]), int(own[-1]) + 1
            assert np.array_equal(own, np.arange(lo, hi))
            if d == 0:   # halo ahead, then owned; head flag on the first slot only
                assert seg[0] == max(ls, lo - J) and seg[-1] == hi - 1
                assert (f[0] & 1) and not np.any(f[1:k] & 1)
            else:        # owned, then the halo behind; head flag only on a lane head
                assert seg[0] == lo and seg[-1] == min(le, hi + J) - 1
                heads = seg[(f[:k] & 1) != 0]
                assert np.array_equal(heads, [ls] if lo == ls else [])
            owned[d].append(own)
            counts.setdefault((lane, d), []).append(k)
        assert lanes[0] == lanes[1]
        tiles_of_lane[lanes[0]] += 1
    assert np.array_equal(tiles_of_lane, need)
    assert np.array_equal(whole_seen, ((sz > 0) & (sz <= threads)).astype(np.int64))
    fill = np.asarray(shared_fill)
    assert len(fill) >= 1 and threads in fill
    pair = fill[:, None] + fill[None, :]
    np.fill_diagonal(pair, threads + 1)
    assert np.all(pair > threads)
    for d in (0, 1):
        o = np.concatenate(owned[d])
        assert len(o) == N and np.array_equal(np.sort(o), np.arange(N))
    for (lane, d), ks in counts.items():
        assert max(ks) - min(ks) <= 1, (lane, d, ks)
    align = lambda x: (x + 255) // 256 * 256
    nt = info.n_bundles
    expect = (align(8 * nt) + align(16 * nt) + align(8 * 7 * N) + 2 * align((S + 1) * 4 * N)
              + 2 * align(8 * N) + align(4 * N) + align(48 * N))
    assert ws == expect


def test_halo_tile_tuning_limits(L):
    """Halo tiles need kept states, one vehicle per thread, explicit threads of
    256, 512, 576, 640, 768 or 1024 (576, 640 and 768 for tiles only), an
    even J that is a multiple of K and below the work-group, and one
    work-group per tile."""
    off = [0, 3000, 3500]
    ok = (512, 1, 32, 0, 0, 1, 64)
    assert _check(L, off, tuning=ok, K=32)[0] == 0
    for bad in [(512, 1, 32, 0, 0, 0, 64),     # checkpoints
                (512, 1, 32, 0, 0, 2, 64),     # autotuner's choice pending
                (512, 2, 32, 0, 0, 1, 64),     # two vehicles per thread
                (0, 0, 32, 0, 0, 1, 64),       # no explicit shape
                (128, 1, 32, 0, 0, 1, 64),     # no 128-thread tile kernels
                (512, 1, 32, 0, 0, 1, 512),    # J >= threads
                (512, 1, 32, 0, 0, 1, 48),     # not a multiple of K
                (512, 1, 8, 0, 0, 1, 36),      # not a multiple of K = 8 (the tuning K)
                (512, 1, 32, 64, 0, 1, 64)]:   # persistent grid
        st = _check(L, off, tuning=bad, K=32)[0]
        assert st == -3, (bad, st)
    assert _check(L, off, tuning=(512, 1, 32, 0, 0, 1, -64), K=32)[0] == -1
    for t in (576, 640, 768):
        assert _check(L, off, tuning=(t, 1, 32, 0, 0, 1, 256), K=32)[0] == 0
        assert _check(L, off, tuning=(t, 1, 32, 0, 0, 1, 0), K=32)[0] == -3
    assert _check(L, off, tuning=(384, 1, 32, 0, 0, 1, 128), K=32)[0] == -3


def test_backward_entry_points_reject_null_arguments(L):
    """Argument checks that run before any device work: a null plan, and
    (through a null plan) the stored-state backward's required trajectories."""
    from paper_2412_16750_amd._lib import IdmParams
    prm = IdmParams(1, 1, 1, 1, 1, 1)
    for call in (lambda: L.idm_sim_backward_stored(None, ctypes.byref(prm), 8, 8, 8, None, None,
                                                   None, 8, 8, 8, None, 8, None),
                 lambda: L.idm_sim_backward(None, ctypes.byref(prm), 8, 8, None, None, None, 8, 8,
                                            8, None, 8, None),
                 lambda: L.idm_sim_backward_noalloc(None, ctypes.byref(prm), 8, 8, None, None,
                                                    None, 8, 8, 8, None, None)):
        assert call() == -1
        assert b"plan is null" in L.idm_last_error()


def _layout(L, offsets, tuning):
    from paper_2412_16750_amd._lib import IdmTuning
    st, info, _ = _check(L, offsets, tuning=tuning)
    assert st == 0
    pb, off = _problem(offsets)
    tu = IdmTuning(*tuning)
    n = info.n_slots
    gidx = np.empty(n, dtype=np.int32)
    flags = np.empty(n, dtype=np.uint8)
    assert L.idm_problem_layout(ctypes.byref(pb), ctypes.byref(tu), gidx.ctypes.data_as(ctypes.c_void_p),
                                flags.ctypes.data_as(ctypes.c_void_p), n - 1) == -1
    assert L.idm_problem_layout(ctypes.byref(pb), ctypes.byref(tu), gidx.ctypes.data_as(ctypes.c_void_p),
                                flags.ctypes.data_as(ctypes.c_void_p), n) == 0
    return info, gidx, flags


@pytest.mark.parametrize("tuning", [(64, 1, 8, 0, 0), (64, 2, 8, 0, 0), (256, 4, 4, 0, 0),
                                    (1024, 4, 8, 0, 0)])
def test_layout_packs_whole_lanes(L, tuning):
    import scenarios
    sizes = scenarios.lognormal_lane_sizes(3000, 3.0, 1.2, 1, tuning[0] * tuning[1], 99)
    sizes[::97] = 0
    off = scenarios.offsets_from_sizes(sizes)
    info, gidx, flags = _layout(L, off, tuning)
    cap = tuning[0] * tuning[1]
    N = int(off[-1])
    valid = gidx >= 0
    # every vehicle exactly once
    assert np.array_equal(np.sort(gidx[valid]), np.arange(N))
    assert np.all((flags[valid] & 4) == 4) and np.all(flags[~valid] == 0)
    lane_of = np.repeat(np.arange(len(sizes)), sizes)
    fills = []
    for b in range(info.n_bundles):
        g = gidx[b * cap:(b + 1) * cap]
        f = flags[b * cap:(b + 1) * cap]
        k = int(np.sum(g >= 0))
        fills.append(k)
        assert np.all(g[k:] == -1)          # padding only at the end
        seg = g[:k]
        # lanes are contiguous, head -> tail, flags mark heads and tails
        heads = np.flatnonzero(f[:k] & 1)
        tails = np.flatnonzero(f[:k] & 2)
        assert heads[0] == 0 and len(heads) == len(tails)
        for h, t in zip(heads, tails):
            lane = lane_of[seg[h]]
            assert seg[h] == off[lane] and seg[t] == off[lane + 1] - 1
            assert np.array_equal(seg[h:t + 1], np.arange(off[lane], off[lane + 1]))
    assert fills == sorted(fills, reverse=True)
    # best-fit decreasing: no two bundles could be merged
    assert sum(1 for f in fills if f <= cap // 2) <= 1


def test_python_binding_rejects_bad_tensors():
    """The Python binding validates shapes, dtypes and devices before calling."""
    import torch
    from paper_2412_16750_amd import sim
    with pytest.raises(ValueError):
        sim._need(torch.zeros(3), "x", torch.float32, 3)   # CPU tensor
    with pytest.raises(TypeError):
        sim._need(np.zeros(3), "x", torch.float32, 3)         # not a tensor


def _bundles(L, offsets, tuning):
    from paper_2412_16750_amd._lib import IdmTuning
    st, info, ws = _check(L, offsets, tuning=tuning)
    assert st == 0
    pb, off = _problem(offsets)
    tu = IdmTuning(*tuning) if tuning else None
    nb = info.n_bundles
    bin_, bout, lvl = (np.empty(nb, dtype=np.int32) for _ in range(3))
    args = [ctypes.byref(pb), ctypes.byref(tu) if tu else None] + \
        [a.ctypes.data_as(ctypes.c_void_p) for a in (bin_, bout, lvl)]
    assert L.idm_problem_bundles(*args, nb - 1) == -1
    assert L.idm_problem_bundles(*args, nb) == 0
    return info, ws, bin_, bout, lvl


@pytest.mark.parametrize("tuning", [(64, 1, 8, 0, 0), (256, 1, 16, 0, 0), None])
def test_long_lanes_are_cut_into_pieces(L, tuning):
    """Lanes longer than a bundle: pieces of a whole bundle each plus a
    remainder, piece j in launch level j, every boundary linking the last
    slot of piece j-1 to the first slot of piece j; short lanes fill the
    remainders' room and spread over the levels."""
    import scenarios
    cap = tuning[0] * tuning[1] if tuning else 1024
    sizes = scenarios.lognormal_lane_sizes(400, np.log(cap) - 0.5, 1.0, 1, 5 * cap, 77)
    sizes[[3, 50]] = [4 * cap, cap + 1]
    sizes[::53] = 0
    off = scenarios.offsets_from_sizes(sizes)
    info, gidx, flags = _layout(L, off, tuning) if tuning else (None, None, None)
    if tuning is None:
        from paper_2412_16750_amd._lib import IdmTuning
        st, info, _ = _check(L, off)
        assert st == 0 and (info.threads, info.per_thread) == (1024, 1)
        tuning = (1024, 1, 0, 0, 0)
        info, gidx, flags = _layout(L, off, tuning)
    info, ws, bin_, bout, lvl = _bundles(L, off, tuning)
    N = int(off[-1])
    pieces = np.where(sizes > cap, -(-sizes // cap), 1)
    assert info.n_levels == pieces.max() == 5
    assert info.n_boundaries == int(np.sum(pieces[sizes > 0] - 1))
    valid = gidx >= 0
    assert np.array_equal(np.sort(gidx[valid]), np.arange(N))
    # only a lane's own first and last vehicles carry head / tail flags
    heads = np.zeros(N, dtype=bool)
    tails = np.zeros(N, dtype=bool)
    heads[gidx[valid & ((flags & 1) == 1)]] = True
    tails[gidx[valid & ((flags & 2) == 2)]] = True
    ne = sizes > 0
    assert np.array_equal(np.flatnonzero(heads), off[:-1][ne])
    assert np.array_equal(np.flatnonzero(tails), off[1:][ne] - 1)
    g = gidx.reshape(-1, cap)
    # levels ascend through the bundle list
    assert np.all(np.diff(lvl) >= 0) and lvl[0] == 0 and lvl[-1] == info.n_levels - 1
    seen = set()
    for b in range(info.n_bundles):
        if bin_[b] >= 0:
            j = bin_[b]
            src = np.flatnonzero(bout == j)
            assert len(src) == 1 and j not in seen
            seen.add(j)
            a = src[0]
            # the leader bundle is a full piece whose last slot leads slot 0 here
            assert np.all(g[a] >= 0) and g[a, -1] + 1 == g[b, 0]
            assert not heads[g[b, 0]] and lvl[b] == lvl[a] + 1
        if bout[b] >= 0:
            assert np.all(g[b] >= 0) and not tails[g[b, -1]]
    assert seen == set(range(info.n_boundaries))
    # bundles of whole lanes only fill the levels' last rounds of resident
    # work-groups (256 CUs x 2048 threads): as few rounds as possible
    counts = np.bincount(lvl, minlength=info.n_levels)
    fixed = np.zeros(info.n_levels, dtype=int)
    for b in range(info.n_bundles):
        if bin_[b] >= 0 or bout[b] >= 0:
            fixed[lvl[b]] += 1
    q = 256 * max(1, 2048 // tuning[0])
    rounds = lambda c: int(np.sum(-(-c // q)))
    assert rounds(counts) == max(rounds(fixed), -(-info.n_bundles // q))
    # workspace: loss partials per lane and piece, fit buffer, checkpoints,
    # boundary rows (S + 1 states and S adjoint contributions of 8 B)
    S, K = 100, info.ckpt_every
    align = lambda x: (x + 255) // 256 * 256
    nbnd = info.n_boundaries
    expect = (align(8 * (len(sizes) + nbnd)) + align(16 * (len(sizes) + nbnd)) + align(8 * 7 * N)
              + align(-(-S // K) * 8 * N)
              + align(nbnd * (S + 1) * 8) + align(nbnd * S * 8))
    assert ws == expect


def test_level_rounds_on_the_uneven_workload(L):
    """The 10,000-lane uneven workload at 1024 x 1: 4 levels whose sizes are
    whole rounds of 512 resident forward work-groups but for one."""
    import scenarios
    sc = scenarios.uneven()
    info, ws, bin_, bout, lvl = _bundles(L, sc.lane_offsets, (1024, 1, 32, 0, 16))
    counts = np.bincount(lvl)
    assert info.n_levels == 4 and len(counts) == 4
    assert np.sum(counts % 512 != 0) <= 1
    assert int(np.sum(-(-counts // 512))) == -(-info.n_bundles // 512)


@pytest.mark.parametrize("seed", range(12))
def test_random_layouts_keep_every_invariant(L, seed):
    """Random lane-size mixes (empty lanes, singletons, exact multiples of the
    bundle, long lanes) and random one-vehicle-per-thread shapes: every
    vehicle in exactly one slot, lanes contiguous head -> tail across their
    pieces, each boundary joining a full bundle's last slot to the next
    piece's first slot one level up, and levels ascending."""
    rng = np.random.default_rng(seed)
    threads = int(rng.choice([64, 128, 256, 512, 1024]))
    cap = threads
    n_lanes = int(rng.integers(1, 120))
    kind = rng.integers(0, 4, n_lanes)
    sizes = np.where(kind == 0, rng.integers(0, 3, n_lanes),                 # empty / tiny
             np.where(kind == 1, rng.integers(1, cap + 1, n_lanes),          # fits
             np.where(kind == 2, cap * rng.integers(1, 4, n_lanes),          # exact multiples
                      rng.integers(cap + 1, 5 * cap, n_lanes)))).astype(np.int64)
    if sizes.sum() == 0:
        sizes[0] = 1
    off = scenarios_offsets(sizes)
    tuning = (threads, 1, 8, 0, 0)
    info, gidx, flags = _layout(L, off, tuning)
    info, ws, bin_, bout, lvl = _bundles(L, off, tuning)
    N = int(off[-1])
    valid = gidx >= 0
    assert np.array_equal(np.sort(gidx[valid]), np.arange(N))
    g = gidx.reshape(-1, cap)
    assert np.all(np.diff(lvl) >= 0)
    pieces = np.where(sizes > cap, -(-sizes // cap), 1)
    assert info.n_levels == max(1, int(pieces[sizes > 0].max()))
    assert info.n_boundaries == int(np.sum(pieces[sizes > 0] - 1))
    # within a bundle, occupied slots come first; consecutive slots of one
    # lane hold consecutive vehicles
    lane_of = np.repeat(np.arange(len(sizes)), sizes)
    for b in range(info.n_bundles):
        row = g[b]
        k = int(np.sum(row >= 0))
        assert np.all(row[k:] == -1)
        seg = row[:k]
        same = lane_of[seg[1:]] == lane_of[seg[:-1]]
        assert np.all(seg[1:][same] == seg[:-1][same] + 1)
        if bin_[b] >= 0:
            a = int(np.flatnonzero(bout == bin_[b])[0])
            assert np.all(g[a] >= 0) and g[a, -1] + 1 == g[b, 0] and lvl[b] == lvl[a] + 1
        elif k:
            # a bundle without an incoming boundary starts with a lane head
            assert seg[0] == off[lane_of[seg[0]]]


def scenarios_offsets(sizes):
    import scenarios
    return scenarios.offsets_from_sizes(np.asarray(sizes, dtype=np.int64))


def test_mlp_entry_points_validate_before_touching_the_device(L):
    """The warm-start network's entry points check their pointers, sizes and
    alignments on the host and return IDM_ERR_INVALID_ARG (nothing launched)."""
    from paper_2412_16750_amd._lib import IdmMlpState
    assert L.idm_mlp_param_count() == 160 * 256 + 256 + 256 * 256 + 256 + 256 * 16 + 16
    # plain copies of W1, W2, W3 and their transposes
    assert L.idm_mlp_weight_bf16_count() == 2 * (160 * 256 + 256 * 256 + 256 * 16)
    assert L.idm_mlp_workspace_bytes(0) == 0
    assert L.idm_mlp_workspace_bytes(4096) > 0

    def state(params, w16, m=0, v=0):
        st = IdmMlpState()
        st.params, st.weights_bf16, st.adam_m, st.adam_v = params, w16, m, v
        st.lr, st.beta1, st.beta2, st.eps = 1e-3, 0.9, 0.999, 1e-8
        return st

    good = state(0x10000, 0x20000, 0x30000, 0x40000)
    X, U, Y, ws = 0x50000, 0x60000, 0x70000, 0x80000
    cases = [
        (L.idm_mlp_forward, (ctypes.byref(state(0, 0x20000)), X, 1, Y, None, None)),
        (L.idm_mlp_forward, (ctypes.byref(state(0x10000, 0x20002)), X, 1, Y, None, None)),
        (L.idm_mlp_forward, (ctypes.byref(state(0x10004, 0x20000)), X, 1, Y, None, None)),
        (L.idm_mlp_forward, (ctypes.byref(good), X, 0, Y, None, None)),
        (L.idm_mlp_forward, (ctypes.byref(good), None, 1, Y, None, None)),
        (L.idm_mlp_gradients, (ctypes.byref(good), X, U, 1, 0x90000, None, ws + 8, None)),
        (L.idm_mlp_gradients, (ctypes.byref(good), X, U, 1, None, None, ws, None)),
        (L.idm_mlp_train_step, (ctypes.byref(state(0x10000, 0x20000)), X, U, 1, 1, None, ws, None)),
        (L.idm_mlp_train_step, (ctypes.byref(good), X, U, 1, 0, None, ws, None)),
        (L.idm_mlp_train_step, (ctypes.byref(good), X, U, 1, 1, None, ws + 4, None)),
        (L.idm_mlp_train_step, (ctypes.byref(good), X, U, (1 << 30) + 1, 1, None, ws, None)),
    ]
    for fn, args in cases:
        assert fn(*args) == -1, (fn.__name__, args)
        assert len(L.idm_last_error()) > 0
