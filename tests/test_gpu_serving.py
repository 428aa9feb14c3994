"""GPU tests of the serving loop (``mfs_server_*`` through the C ABI).

A request's result is the same alone and in the mix: frames solved by the
server while other requests join and leave the batch, some with workspaces
lent from the server's arena, equal bitwise the same frames solved one at a
time with ``mfs_solve_frame`` (the batch kernels keep per-character scalars
and fixed-order reductions, so the tolerance of the claim is zero).
"""

import sys
import time

import numpy as np
import pytest

from workloads import NH, COROT, humanoid, random_pose, animation_pose

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

OPTS = dict(precision=1, cg_tol=1e-5, step_tol=1e-9, cg_adaptive=1)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture()
def mfs_ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2408_04066_amd as mfs
    c = mfs.Context(0)
    yield mfs, c
    c.close()


def _chars(mfs, ctx, specs, seed0):
    probs = [humanoid(seed0 + i, target_tets=t, n_bones=b, models=(NH, COROT))
             for i, (t, b) in enumerate(specs)]
    return probs, [mfs.Character(ctx, p) for p in probs]


def test_served_equals_alone_with_arena_admission(mfs_ctx):
    mfs, ctx = mfs_ctx
    probs, chars = _chars(mfs, ctx, [(1500, 8), (3000, 12), (800, 10), (2200, 9), (1200, 14)], 300)
    poses = [random_pose(p, 400 + i) for i, p in enumerate(probs)]
    alone = []
    for ch, pose in zip(chars, poses):
        _say(f"alone: n={ch.n}")
        x, st, rc = ch.solve(*pose, **OPTS)
        alone.append((x, st))
    # three characters borrow workspaces; the arena holds the largest of
    # them but not all three at once, so admission must wait for memory
    ws = [ch.footprint()[1] for ch in chars[:3]]
    budget = max(ws) + min(ws) + 4096
    assert budget < sum(ws) + 3 * 256
    for ch in chars[:3]:
        ch.release_workspace()
    _say(f"server: slots 3, arena {budget} bytes (workspaces {ws})")
    srv = mfs.Server(ctx, slots=3, workspace_budget_bytes=budget, **OPTS)
    order = [0, 1, 2, 0]
    tickets = [(k, srv.submit(chars[k], *poses[k])) for k in order]
    t0 = time.time()
    while srv.info()["running"] == 0 and time.time() - t0 < 30:
        time.sleep(0.001)
    for k in (3, 4, 1):  # arrive while others are on the GPU
        tickets.append((k, srv.submit(chars[k], *poses[k])))
    got = []
    for k, tk in tickets:
        x, st, times, rc = srv.wait(tk)
        got.append((k, x, st, times))
    info = srv.info()
    srv.close()
    _say(f"server info {info}")
    assert info["completed"] == len(tickets) and info["queued"] == 0 and info["running"] == 0
    assert 0 < info["arena_peak"] <= budget and info["arena_in_use"] == 0
    assert info["slot_steps"] / info["steps"] > 1.0  # requests overlapped in the batch
    for j, (k, x, st, times) in enumerate(got):
        ref_x, ref_st = alone[k]
        assert np.array_equal(x, ref_x), (
            f"request {j} (character {k}) differs from its solve alone: max |dx| "
            f"{np.max(np.abs(x - ref_x)):.3e}; served {st}; alone {ref_st}; times {times}; info {info}")
        assert st["iterations"] == ref_st["iterations"] and st["cg_iterations"] == ref_st["cg_iterations"]
        assert st["status"] == ref_st["status"]
        assert times["submit_s"] <= times["admit_s"] <= times["done_s"]
    # frames of one character ran in submission order
    done0 = [t["done_s"] for k, _, _, t in got if k == 0]
    admit0 = [t["admit_s"] for k, _, _, t in got if k == 0]
    assert admit0[1] >= done0[0]
    # a released character solves standalone again (own workspace re-made)
    x, _, _ = chars[0].solve(*poses[0], **OPTS)
    assert np.array_equal(x, alone[0][0])
    for ch in chars:
        ch.close()


def test_served_warm_start_sequence_equals_standalone(mfs_ctx):
    """Animation frames with warm start from the previous frame: served in
    order per character, interleaved across characters, equal to the same
    sequence solved standalone on fresh copies of the characters."""
    mfs, ctx = mfs_ctx
    specs = [(1500, 10), (2500, 12)]
    probs, ref_chars = _chars(mfs, ctx, specs, 500)
    frames = [[animation_pose(p, 600 + i, f / 24.0) for f in range(3)] for i, p in enumerate(probs)]
    opts = dict(OPTS, warm_start=mfs.WARM_PREVIOUS)
    ref = []
    for ch, fr in zip(ref_chars, frames):
        seq = []
        for pose in fr:
            x, st, rc = ch.solve(*pose, **opts)
            seq.append(x)
        ref.append(seq)
        ch.close()
    _, chars = _chars(mfs, ctx, specs, 500)
    _say("server: warm-started animation, 2 characters x 3 frames")
    srv = mfs.Server(ctx, slots=4, **opts)
    tickets = [(i, f, srv.submit(chars[i], *frames[i][f])) for f in range(3) for i in range(2)]
    out = {(i, f): srv.wait(tk)[0] for i, f, tk in tickets}
    srv.close()
    for i in range(2):
        for f in range(3):
            assert np.array_equal(out[(i, f)], ref[i][f])
    for ch in chars:
        ch.close()


def test_server_rejects_bad_requests(mfs_ctx):
    mfs, ctx = mfs_ctx
    probs, chars = _chars(mfs, ctx, [(800, 8)], 700)
    ch = chars[0]
    srv = mfs.Server(ctx, slots=2, queue_capacity=1, **OPTS)
    R, t = random_pose(probs[0], 701)
    bad = R.copy()
    bad[0] *= 2.0
    with pytest.raises(mfs.MfsError) as e:
        srv.submit(ch, bad, t)
    assert e.value.code == -1
    ch.release_workspace()  # no arena: its workspace can never be lent
    with pytest.raises(mfs.MfsError) as e:
        srv.submit(ch, R, t)
    assert e.value.code == -6
    srv.close()
    ch.close()


def test_one_slot_reoccupied_by_other_characters(mfs_ctx):
    """Regression: with one slot, every request reoccupies slot 0 with the
    same slot list but another character (larger and smaller by turns, own
    and lent workspaces); each must run on its own tiles and equal its solve
    alone."""
    mfs, ctx = mfs_ctx
    probs, chars = _chars(mfs, ctx, [(3000, 12), (800, 8), (2000, 10)], 1000)
    poses = [random_pose(p, 1100 + i) for i, p in enumerate(probs)]
    alone = [ch.solve(*pose, **OPTS)[0] for ch, pose in zip(chars, poses)]
    chars[1].release_workspace()
    budget = chars[1].footprint()[1] + 4096
    _say("server: one slot, characters 0 1 2 1 0 2")
    srv = mfs.Server(ctx, slots=1, workspace_budget_bytes=budget, **OPTS)
    order = [0, 1, 2, 1, 0, 2]
    tickets = [(k, srv.submit(chars[k], *poses[k])) for k in order]
    for k, tk in tickets:
        x, st, _, rc = srv.wait(tk)
        assert np.array_equal(x, alone[k]), f"character {k} differs from its solve alone"
    srv.close()
    for ch in chars:
        ch.close()


def test_served_with_loads_and_smoothed_rotations(mfs_ctx):
    """Characters with external loads and smoothed rotations served in a mix
    with a plain one: each result equals its solve alone bitwise."""
    mfs, ctx = mfs_ctx
    probs, chars = _chars(mfs, ctx, [(1500, 8), (2000, 10), (1000, 9)], 1200)
    p0, p1 = probs[0], probs[1]
    H, W = ctx.blend_weights(p0["X"], p0["T"], p0["seg_a"], p0["seg_b"], p0["seg_handle"], p0["n_handles"],
                             0.05 * p0["bbox_diag"], 3)
    chars[0].set_rotation_blend(H, W)
    rng = np.random.default_rng(1201)
    fv = rng.choice(len(p1["X"]), 20, replace=False).astype(np.int32)
    chars[1].set_forces(fv, rng.normal(scale=1e-4 * float(np.max(p1["youngs"])) * p1["bbox_diag"] ** 2 / len(p1["X"]),
                                       size=(20, 3)))
    poses = [random_pose(p, 1300 + i) for i, p in enumerate(probs)]
    alone = [ch.solve(*pose, **OPTS)[0] for ch, pose in zip(chars, poses)]
    _say("server: smoothed, loaded and plain characters")
    srv = mfs.Server(ctx, slots=3, **OPTS)
    tickets = [(k, srv.submit(chars[k], *poses[k])) for k in (0, 1, 2, 1, 0)]
    for k, tk in tickets:
        x, st, _, rc = srv.wait(tk)
        assert np.array_equal(x, alone[k]), f"character {k} differs from its solve alone"
    srv.close()
    for ch in chars:
        ch.close()


def test_lanes_route_by_size_and_equal_alone(mfs_ctx):
    """Three lanes (size classes up to 1200 tets, up to 4000, larger), each
    a batch on a stream of its own: small, medium and large characters (one
    with smoothed rotations, one on a lent workspace) served in a mix equal
    their solves alone bitwise, and the server's counters add up over the
    lanes."""
    mfs, ctx = mfs_ctx
    probs, chars = _chars(mfs, ctx, [(800, 8), (1000, 10), (2500, 12), (3000, 9), (6000, 14)], 1400)
    p2 = probs[2]
    H, W = ctx.blend_weights(p2["X"], p2["T"], p2["seg_a"], p2["seg_b"], p2["seg_handle"], p2["n_handles"],
                             0.05 * p2["bbox_diag"], 3)
    chars[2].set_rotation_blend(H, W)
    poses = [random_pose(p, 1500 + i) for i, p in enumerate(probs)]
    alone = [ch.solve(*pose, **OPTS)[0] for ch, pose in zip(chars, poses)]
    # the large lane runs another PCG schedule: its reference is solved under it
    base = ctx.tuning()
    alt = 8 if base["pcg_lanes_per_row"] != 8 else 4
    ctx.set_tuning(pcg_lanes_per_row=alt)
    alone[4] = chars[4].solve(*poses[4], **OPTS)[0]
    ctx.set_tuning(**base)
    chars[0].release_workspace()
    budget = chars[0].footprint()[1] + 4096
    with pytest.raises(mfs.MfsError) as e:
        mfs.Server(ctx, lane_max_tets=(4000, 1200), **OPTS)
    assert e.value.code == -1
    _say(f"server: 3 lanes, tets {[ch.info()['n_tets'] for ch in chars]}")
    srv = mfs.Server(ctx, slots=2, workspace_budget_bytes=budget, lane_max_tets=(1200, 4000), **OPTS)
    with pytest.raises(mfs.MfsError) as e:
        srv.set_lane_tuning(3, pcg_lanes_per_row=alt)
    assert e.value.code == -1
    with pytest.raises(mfs.MfsError) as e:
        srv.set_lane_tuning(2, pcg_lanes_per_row=3)
    assert e.value.code == -1
    srv.set_lane_tuning(2, pcg_lanes_per_row=alt)
    order = [4, 0, 2, 1, 3, 0, 4, 2]
    tickets = [(k, srv.submit(chars[k], *poses[k])) for k in order]
    for k, tk in tickets:
        x, st, times, rc = srv.wait(tk)
        assert np.array_equal(x, alone[k]), f"character {k} differs from its solve alone"
        assert times["submit_s"] <= times["admit_s"] <= times["done_s"]
    info = srv.info()
    srv.close()
    _say(f"server info {info}")
    assert info["submitted"] == info["completed"] == len(order)
    assert info["queued"] == 0 and info["running"] == 0 and info["arena_in_use"] == 0
    assert info["arena_bytes"] >= 3 * (budget // 256 * 256)
    # the caller's context is usable again after the server is gone, with its
    # own schedule
    assert ctx.tuning() == base
    x, _, _ = chars[3].solve(*poses[3], **OPTS)
    assert np.array_equal(x, alone[3])
    for ch in chars:
        ch.close()
