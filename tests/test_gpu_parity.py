"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Every case builds seeded synthetic inputs, runs the library on the GPU and
compares element by element with the oracle on the same inputs.
Tolerances: FP64 frame solves within 1e-9 * bbox diagonal of the oracle's
positions; FP32 + FP64 refinement within 1e-7 * bbox diagonal; per-element
and assembled FP64 quantities within a relative 1e-12 of the oracle's (the
two sides round in different orders); rotation clusters bit-exact.
"""

import sys

import numpy as np
import pytest

import oracle
from workloads import (ARAP, COROT, NH, beam, beam_pose, humanoid, random_pose, euler_xyz)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2408_04066_amd as mfs
    c = mfs.Context(0)
    yield c
    c.close()


def _mfs():
    import paper_2408_04066_amd as mfs
    return mfs


def _small_humanoid(seed=21, tets=4000, bones=15):
    return humanoid(seed, target_tets=tets, n_bones=bones)


# --------------------------------------------------------------------------
# helpers / standalone kernels
# --------------------------------------------------------------------------
def test_cluster_kernel_bit_exact(ctx):
    from oracle.mfem import _barycenters, _segment_dist2
    from workloads.humanoid import _pool_member
    # a member of the batched workload's pool with tets exactly as far from
    # two segments of different handles (at shared joints): regression test
    # of ties decided differently when the distances were fused-multiply-added
    tied = _pool_member((27, 4001, (5000, 200000), (8, 30), (NH, COROT)))
    d2 = _segment_dist2(_barycenters(np.asarray(tied["X"], dtype=np.float64), np.asarray(tied["T"])),
                        tied["seg_a"], tied["seg_b"])
    best = d2.min(axis=1, keepdims=True)
    sh = np.asarray(tied["seg_handle"])
    ties = [k for k in np.nonzero(np.sum(d2 == best, axis=1) > 1)[0]
            if len(set(sh[d2[k] == best[k, 0]].tolist())) > 1]
    assert len(ties) >= 1
    for prob in (beam(), _small_humanoid(), tied):
        _say(f"cluster kernel: {prob['name']}")
        ref = oracle.cluster_by_segments(prob["X"], prob["T"], prob["seg_a"], prob["seg_b"],
                                         prob["seg_handle"])
        got = ctx.cluster_by_segments(prob["X"], prob["T"], prob["seg_a"], prob["seg_b"],
                                      prob["seg_handle"])
        assert np.array_equal(ref, got), f"{int(np.sum(ref != got))} tets differ (exact ties: {len(ties)})"


def test_polar_kernel_matches_oracle(ctx):
    mfs = _mfs()
    rng = np.random.default_rng(4)
    F = rng.normal(size=(1000, 3, 3))
    F[np.linalg.det(F) < 0, :, 0] *= -1.0
    # near-singular and near-identity members
    F[:20] = np.eye(3) + 1e-6 * rng.normal(size=(20, 3, 3))
    Q = np.stack([euler_xyz(*rng.uniform(-3, 3, 3)) for _ in range(20)])
    F[20:40] = Q @ np.diag([1.0, 0.5, 2e-4])
    F[40:45] = -np.eye(3)        # det < 0: warm start falls back to identity
    _say("polar kernel FP64")
    U, P, smin, routed = ctx.polar(F, mfs.FP64)
    Uo, Po = oracle.polar(F[45:])
    assert np.allclose(U[45:], Uo, atol=1e-12)
    assert np.allclose(P[45:], oracle.vech(Po), atol=1e-12 * np.abs(Po).max())
    sig = np.linalg.svd(F[45:], compute_uv=False)
    assert np.allclose(smin[45:], sig[:, 2], rtol=1e-9, atol=1e-13)
    assert np.all(P[40:45] == np.array([1.0, 1, 1, 0, 0, 0]))
    assert not routed.any()
    _say("polar kernel FP32 with FP64 re-route")
    U32, P32, smin32, routed32 = ctx.polar(F, mfs.FP32_REFINED)
    r45 = routed32[45:].astype(bool)
    assert np.all(r45[sig[:, 2] < 0.9e-3]) and not np.any(r45[sig[:, 2] > 1.1e-3])
    assert routed32[20:40].all()               # sigma_min = 2e-4 -> FP64
    assert np.allclose(P32[20:40], P[20:40], atol=1e-13)
    far = ~routed32.astype(bool)
    far[40:45] = False
    scale = np.abs(P).max(axis=1)
    assert np.max(np.abs(P32[far] - P[far]) / scale[far, None]) < 2e-6


# --------------------------------------------------------------------------
# element pass, assembly and SpMV against the oracle's Frame
# --------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["beam", "humanoid"])
def test_evaluate_matches_oracle(ctx, which):
    mfs = _mfs()
    if which == "beam":
        prob = beam()
        pose = beam_pose(prob)
    else:
        prob = _small_humanoid()
        prob["model"] = np.array([(ARAP, COROT, NH)[k % 3] for k in range(len(prob["T"]))],
                                 dtype=np.int32)
        pose = random_pose(prob, 77, amp_deg=20.0)
    fr = oracle.Frame(prob, pose)
    rng = np.random.default_rng(1)
    # a feasible deformed state near the rigidly skinned pose
    x = oracle.solve_frame(prob, pose, iterations=1, frame=fr)["x"]
    if not fr.feasible(x.reshape(-1)):
        x = prob["X"].copy()
    x = x + 1e-5 * prob["bbox_diag"] * rng.normal(size=x.shape)
    assert fr.feasible(x.reshape(-1))
    v = rng.normal(size=x.shape)
    _say(f"evaluate: {which} n={fr.n} m={fr.m}")
    ch = mfs.Character(ctx, prob)
    assert np.array_equal(ch.cluster, fr.cluster)
    out = ch.evaluate(*pose, x, v)
    E = fr.energy(x.reshape(-1))
    g = fr.gradient(x.reshape(-1)).reshape(-1, 3)
    s = fr.stretch(x.reshape(-1))
    Kv = (fr.hessian(s) @ v.reshape(-1)).reshape(-1, 3)
    assert abs(out["energy"] - E) <= 1e-12 * abs(E)
    assert np.max(np.abs(out["grad"] - g)) <= 1e-11 * np.abs(g).max()
    assert np.max(np.abs(out["stretch"] - s)) <= 1e-13 * max(1.0, np.abs(s).max())
    assert np.max(np.abs(out["Kv"] - Kv)) <= 1e-12 * np.abs(Kv).max()
    ch.close()


# --------------------------------------------------------------------------
# frame solves
# --------------------------------------------------------------------------
def _err(x, ref, prob):
    return float(np.max(np.linalg.norm(x - ref, axis=1))) / prob["bbox_diag"]


def test_beam_fp64_ten_iterations(ctx):
    mfs = _mfs()
    prob = beam()
    pose = beam_pose(prob)
    ref = oracle.solve_frame(prob, pose, iterations=10)
    _say("solve: beam 16x4x4 neo-Hookean, FP64, 10 iterations, cg_tol 1e-10")
    ch = mfs.Character(ctx, prob)
    x, st, rc = ch.solve(*pose, max_newton=10, fixed_newton=1, cg_tol=1e-10)
    _say(f"  stats {st}")
    assert rc == 0 and st["iterations"] == 10
    assert _err(x, ref["x"], prob) <= 1e-9
    # the same solve twice is bitwise identical (fixed-order reductions)
    x2, _, _ = ch.solve(*pose, max_newton=10, fixed_newton=1, cg_tol=1e-10)
    assert np.array_equal(x, x2)
    # the pipelined PCG form in FP64 (an autotuner candidate for FP64 solves)
    base = ctx.tuning()
    try:
        for lpr in (2, 4, 8):
            ctx.set_tuning(pcg_pipelined=1, pcg_persistent=0, pcg_lanes_per_row=lpr)
            xp, stp, rcp = ch.solve(*pose, max_newton=10, fixed_newton=1, cg_tol=1e-10)
            _say(f"  pipelined FP64, lanes {lpr}: stats {stp} err/bbox={_err(xp, ref['x'], prob):.3e}")
            assert rcp == 0 and stp["iterations"] == 10 and stp["cg_not_converged"] == 0
            assert _err(xp, ref["x"], prob) <= 1e-9
    finally:
        ctx.set_tuning(**base)
    ch.close()


@pytest.mark.parametrize("model", [ARAP, COROT, NH])
def test_rest_and_rigid_invariants(ctx, model):
    mfs = _mfs()
    prob = beam(8, 2, 2, model=model, pin_stiffness=3e3)
    ch = mfs.Character(ctx, prob)
    _say(f"solve: rest pose, model {model}")
    x, st, rc = ch.solve(np.stack([np.eye(3)] * 2), np.zeros((2, 3)))
    assert rc == 0
    assert np.max(np.abs(x - prob["X"])) <= 1e-14 * prob["bbox_diag"]
    Q = euler_xyz(0.9, -0.6, 2.1)
    c = np.array([3.0, -1.0, 2.0])
    _say(f"solve: rigid pose, model {model}")
    x, st, rc = ch.solve(np.stack([Q, Q]), np.stack([c, c]), cg_tol=1e-12, step_tol=1e-13,
                         max_newton=10)
    assert rc == 0
    assert np.max(np.abs(x - (prob["X"] @ Q.T + c))) <= 1e-11 * prob["bbox_diag"]
    ch.close()


@pytest.mark.parametrize("precision,tol", [(0, 1e-9), (1, 1e-7)])
def test_humanoid_frame(ctx, precision, tol):
    mfs = _mfs()
    prob = _small_humanoid(21, 4000, 15)
    pose = random_pose(prob, 22)
    ref = oracle.solve_frame(prob, pose)
    assert ref["status"] == "ok"
    _say(f"solve: humanoid m={len(prob['T'])} precision={precision}")
    ch = mfs.Character(ctx, prob)
    kw = dict(precision=precision)
    if precision == mfs.FP32_REFINED:
        kw.update(cg_tol=1e-5, step_tol=1e-9)
    x, st, rc = ch.solve(*pose, **kw)
    _say(f"  stats {st}  err/bbox={_err(x, ref['x'], prob):.3e}")
    assert rc == 0
    assert _err(x, ref["x"], prob) <= tol
    if precision == mfs.FP64:  # the pipelined PCG form in FP64 as well
        base = ctx.tuning()
        try:
            ctx.set_tuning(pcg_pipelined=1, pcg_persistent=0)
            xp, stp, rcp = ch.solve(*pose, **kw)
            _say(f"  pipelined FP64: stats {stp}  err/bbox={_err(xp, ref['x'], prob):.3e}")
            assert rcp == 0 and _err(xp, ref["x"], prob) <= tol
        finally:
            ctx.set_tuning(**base)
    ch.close()


def test_batch_equals_alone(ctx):
    """A batch's frames are bitwise those of the same frames solved alone,
    with the same statistics, whether the batch runs each character's Newton
    steps on its own (batch_async) or every character through the same
    Newton iteration; with a small FP32 PCG cap (FP64 re-solves in most
    Newton steps) the asynchronous batch still equals the solves alone."""
    mfs = _mfs()
    probs = [humanoid(100 + i, target_tets=t, n_bones=b, models=(NH, COROT))
             for i, (t, b) in enumerate([(1500, 8), (3000, 12), (800, 10)])]
    poses = [random_pose(p, 200 + i) for i, p in enumerate(probs)]
    chars = [mfs.Character(ctx, p) for p in probs]
    keys = ("status", "iterations", "mixed_iterations", "cg_iterations", "halvings", "fp64_resolves")
    base = ctx.tuning()
    assert base["pcg_pipelined"] == 0 and base["batch_async"] == 1
    opts = dict(precision=mfs.FP32_REFINED, cg_tol=1e-5, step_tol=1e-9)
    try:
        runs = {}
        for mode in (1, 0):
            ctx.set_tuning(batch_async=mode)
            alone = []
            for ch, pose in zip(chars, poses):
                _say(f"batch_async={mode}: solve alone n={ch.n}")
                x, st, rc = ch.solve(*pose, **opts)
                assert rc == 0
                alone.append((x, st))
            _say(f"batch_async={mode}: solve batch of 3")
            xs, sts, rc = mfs.solve_batch(ctx, chars, poses, **opts)
            assert rc == 0
            runs[mode] = (alone, list(zip(xs, sts)))
        ref = runs[1][0]
        for mode in (1, 0):
            for which in (0, 1):
                for (xa, sa), (xb, sb) in zip(ref, runs[mode][which]):
                    assert np.array_equal(xa, xb)
                    assert all(sa[k] == sb[k] for k in keys), (mode, which, sa, sb)
        ctx.set_tuning(batch_async=1)
        capped = dict(opts, fp32_cg_max=30)
        alone = []
        for ch, pose in zip(chars, poses):
            x, st, rc = ch.solve(*pose, **capped)
            alone.append((x, st))
        _say(f"FP32 cap 30 alone: {[st for _, st in alone]}")
        assert any(st["fp64_resolves"] > 0 for _, st in alone)
        xs, sts, rc = mfs.solve_batch(ctx, chars, poses, **capped)
        for (xa, sa), xb, sb in zip(alone, xs, sts):
            assert np.array_equal(xa, xb)
            assert all(sa[k] == sb[k] for k in keys), (sa, sb)
    finally:
        ctx.set_tuning(**base)
    for ch in chars:
        ch.close()


def test_pipelined_batch_equals_alone(ctx):
    """With the pipelined PCG a batch runs the asynchronous form (direct
    launches; each system's iteration parity offset by the launch its solve
    began at) while a character solved alone runs the lockstep form (graph
    replays from iteration 0): positions and statistics agree bitwise, in
    FP32 + refinement, with a small FP32 cap (FP64 re-solves in the
    two-kernel form beside pipelined FP32 solves), and in FP64."""
    mfs = _mfs()
    probs = [humanoid(100 + i, target_tets=t, n_bones=b, models=(NH, COROT))
             for i, (t, b) in enumerate([(1500, 8), (3000, 12), (800, 10)])]
    poses = [random_pose(p, 200 + i) for i, p in enumerate(probs)]
    chars = [mfs.Character(ctx, p) for p in probs]
    keys = ("status", "iterations", "mixed_iterations", "cg_iterations", "halvings", "fp64_resolves")
    base = ctx.tuning()
    cases = [("fp32", dict(precision=mfs.FP32_REFINED, cg_tol=1e-5, step_tol=1e-9)),
             ("fp32 cap 30", dict(precision=mfs.FP32_REFINED, cg_tol=1e-5, step_tol=1e-9, fp32_cg_max=30)),
             ("fp64", dict(precision=mfs.FP64, cg_tol=1e-8, step_tol=1e-9))]
    try:
        ctx.set_tuning(pcg_pipelined=1, pcg_persistent=0, batch_async=1, use_graphs=1, graph_iterations=8)
        for name, opts in cases:
            alone, worst = [], 0
            for ch, pose in zip(chars, poses):
                _say(f"pipelined {name}: solve alone n={ch.n}")
                x, st, rc = ch.solve(*pose, **opts)
                assert rc >= 0, (name, st)
                worst = max(worst, rc)
                alone.append((x, st))
            _say(f"pipelined {name}: alone {[st for _, st in alone]}")
            if name == "fp32 cap 30":
                assert any(st["fp64_resolves"] > 0 for _, st in alone)
            _say(f"pipelined {name}: solve batch of 3")
            xs, sts, rc = mfs.solve_batch(ctx, chars, poses, **opts)
            assert rc == worst
            for (xa, sa), xb, sb in zip(alone, xs, sts):
                assert np.array_equal(xa, xb), name
                assert all(sa[k] == sb[k] for k in keys), (name, sa, sb)
    finally:
        ctx.set_tuning(**base)
    for ch in chars:
        ch.close()


def test_graph_replay_and_lane_counts(ctx):
    """Replayed PCG graphs give bitwise the same frame as direct launches;
    other SpMV lane counts agree to the FP64 tolerance."""
    mfs = _mfs()
    prob = _small_humanoid(31, 3000, 12)
    pose = random_pose(prob, 32)
    ch = mfs.Character(ctx, prob)
    base = ctx.tuning()
    try:
        _say("solve: graphs on")
        ctx.set_tuning(use_graphs=1, graph_iterations=8)
        xg, _, rc = ch.solve(*pose)
        assert rc == 0
        _say("solve: graphs off")
        ctx.set_tuning(use_graphs=0)
        xd, _, rc = ch.solve(*pose)
        assert rc == 0
        assert np.array_equal(xg, xd)
        for lpr in (2, 8):
            _say(f"solve: lanes per row {lpr}")
            ctx.set_tuning(use_graphs=1, pcg_lanes_per_row=lpr)
            xl, _, rc = ch.solve(*pose)
            assert rc == 0
            assert _err(xl, xd, prob) <= 1e-9
    finally:
        ctx.set_tuning(**base)
        ch.close()


def test_full_size_humanoid_matches_golden(ctx):
    """~50k-tet humanoid at its benchmark launch shape: FP64 within 1e-9 and
    FP32 + refinement within 1e-7 of the oracle's stored solution."""
    import os
    mfs = _mfs()
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, os.path.join(here, "golden"))
    from make_golden import input_hash
    g = np.load(os.path.join(here, "golden", "humanoid50k_pose2002.npz"))
    prob = humanoid(2001, target_tets=50000, n_bones=20)
    pose = random_pose(prob, 2002)
    assert str(g["input_hash"]) == input_hash(prob, pose), "rebuilt inputs differ from the golden's"
    ch = mfs.Character(ctx, prob)
    _say("solve: humanoid 50k FP64")
    x64, st, rc = ch.solve(*pose, precision=mfs.FP64, cg_tol=1e-10, step_tol=1e-10, max_newton=60)
    _say(f"  stats {st} err/bbox={_err(x64, g['x'], prob):.3e}")
    assert rc == 0 and _err(x64, g["x"], prob) <= 1e-9
    _say("solve: humanoid 50k FP32 + refinement")
    x32, st, rc = ch.solve(*pose, precision=mfs.FP32_REFINED, cg_tol=1e-5, step_tol=1e-8, max_newton=60)
    _say(f"  stats {st} err/bbox={_err(x32, g['x'], prob):.3e}")
    assert rc == 0 and _err(x32, g["x"], prob) <= 1e-7
    # the benchmark's configuration: inexact Newton with Eisenstat-Walker forcing
    for prec in (mfs.FP32_REFINED, mfs.FP64):
        _say(f"solve: humanoid 50k precision {prec}, adaptive PCG tolerance")
        xa, st, rc = ch.solve(*pose, precision=prec, cg_tol=1e-5, step_tol=1e-8, max_newton=60,
                              cg_adaptive=1)
        _say(f"  stats {st} err/bbox={_err(xa, g['x'], prob):.3e}")
        assert rc == 0 and _err(xa, g["x"], prob) <= 1e-7
    ch.close()


def test_pipelined_pcg(ctx):
    """The pipelined one-kernel PCG (FP32 + refinement): the 4k humanoid and
    the full-size 50k golden within 1e-7 * bbox of the oracle, graph replay
    bitwise equal to direct launches (odd and even run starts), and a batch
    bitwise equal to its members solved alone."""
    import os
    mfs = _mfs()
    base = ctx.tuning()
    kw = dict(precision=mfs.FP32_REFINED, cg_tol=1e-5, step_tol=1e-9, max_newton=60, cg_adaptive=1)
    try:
        prob = _small_humanoid(21, 4000, 15)
        pose = random_pose(prob, 22)
        ref = oracle.solve_frame(prob, pose)
        ch = mfs.Character(ctx, prob)
        for lpr in (2, 4, 8):
            ctx.set_tuning(pcg_pipelined=1, pcg_persistent=0, pcg_lanes_per_row=lpr, use_graphs=1,
                           graph_iterations=8, first_check=31, min_run=7)
            _say(f"pipelined PCG: humanoid m={len(prob['T'])} lanes {lpr}, graphs")
            xg, st, rc = ch.solve(*pose, **kw)
            _say(f"  stats {st} err/bbox={_err(xg, ref['x'], prob):.3e}")
            assert rc == 0 and _err(xg, ref["x"], prob) <= 1e-7
            ctx.set_tuning(use_graphs=0)
            xd, _, rc = ch.solve(*pose, **kw)
            assert rc == 0 and np.array_equal(xg, xd)
        ch.close()
        ctx.set_tuning(pcg_pipelined=1, pcg_persistent=0, pcg_lanes_per_row=4, use_graphs=1, graph_iterations=8)
        probs = [humanoid(100 + i, target_tets=t, n_bones=b, models=(NH, COROT))
                 for i, (t, b) in enumerate([(1500, 8), (3000, 12), (800, 10)])]
        poses = [random_pose(p, 200 + i) for i, p in enumerate(probs)]
        chars = [mfs.Character(ctx, p) for p in probs]
        alone = [c.solve(*q, **kw)[0] for c, q in zip(chars, poses)]
        _say("pipelined PCG: batch of 3")
        xs, _, rc = mfs.solve_batch(ctx, chars, poses, **kw)
        assert rc == 0
        for a, b in zip(alone, xs):
            assert np.array_equal(a, b)
        for c in chars:
            c.close()
        here = os.path.dirname(os.path.abspath(__file__))
        g = np.load(os.path.join(here, "golden", "humanoid50k_pose2002.npz"))
        prob = humanoid(2001, target_tets=50000, n_bones=20)
        pose = random_pose(prob, 2002)
        ch = mfs.Character(ctx, prob)
        _say("pipelined PCG: humanoid 50k golden")
        x, st, rc = ch.solve(*pose, precision=mfs.FP32_REFINED, cg_tol=1e-5, step_tol=1e-8, max_newton=60,
                             cg_adaptive=1)
        _say(f"  stats {st} err/bbox={_err(x, g['x'], prob):.3e}")
        assert rc == 0 and _err(x, g["x"], prob) <= 1e-7
        ch.close()
    finally:
        ctx.set_tuning(**base)


def test_external_forces(ctx):
    """External vertex forces (mfs_character_set_forces): E, grad E at a
    perturbed state within 1e-12 relative of the oracle, FP64 frames within
    1e-9 * bbox and FP32 + refinement within 1e-7 * bbox of the oracle's
    solution with the same forces; clearing the forces restores the plain
    frame."""
    mfs = _mfs()
    rng = np.random.default_rng(77)
    cases = [(beam(), None), (_small_humanoid(21, 4000, 15), 22)]
    for prob, seed in cases:
        pose = beam_pose(prob) if seed is None else random_pose(prob, seed)
        n = len(prob["X"])
        fv = rng.choice(n, 12, replace=False).astype(np.int32)
        fv = np.concatenate([fv, fv[:3]])  # repeats add up
        ff = rng.normal(scale=5e-4 * float(np.max(prob["youngs"])) * prob["bbox_diag"] ** 2 / n, size=(len(fv), 3))
        pf = dict(prob, force_vertex=fv, force=ff)
        ch = mfs.Character(ctx, prob)
        ch.set_forces(fv, ff)
        _say(f"forces: {prob['name']} ({len(fv)} forces)")
        fr = oracle.Frame(pf, pose)
        x = oracle.solve_frame(pf, pose, iterations=1, frame=fr)["x"].reshape(n, 3)
        x = x + rng.normal(scale=1e-5 * prob["bbox_diag"], size=(n, 3))
        assert fr.feasible(x.reshape(-1))
        ev = ch.evaluate(*pose, x)
        assert abs(ev["energy"] - fr.energy(x)) <= 1e-12 * abs(fr.energy(x))
        g = fr.gradient(x).reshape(-1, 3)
        assert np.max(np.abs(ev["grad"] - g)) <= 1e-12 * np.max(np.abs(g))
        ref = oracle.solve_frame(pf, pose, step_tol=1e-12)
        assert ref["status"] == "ok"
        x64, st, rc = ch.solve(*pose, precision=mfs.FP64, step_tol=1e-10, cg_tol=1e-10, max_newton=60)
        _say(f"  FP64 stats {st} err/bbox={_err(x64, ref['x'], prob):.3e}")
        assert rc == 0 and _err(x64, ref["x"], prob) <= 1e-9
        x32, st, rc = ch.solve(*pose, precision=mfs.FP32_REFINED, step_tol=1e-9, cg_tol=1e-5, max_newton=60)
        assert rc == 0 and _err(x32, ref["x"], prob) <= 1e-7
        plain = oracle.solve_frame(prob, pose, step_tol=1e-12)
        assert _err(ref["x"], plain["x"], prob) > 1e-6  # the forces matter
        ch.set_forces(None)
        x0, _, rc = ch.solve(*pose, precision=mfs.FP64, step_tol=1e-10, cg_tol=1e-10, max_newton=60)
        assert rc == 0 and _err(x0, plain["x"], prob) <= 1e-9
        ch.close()


def test_stress_matches_oracle(ctx):
    """Stress recovery (mfs_stress): P_k and lambda_k = W_k R_k P_k within a
    relative 1e-12 of the oracle's on a mixed-material humanoid near a solved
    frame; an inverted neo-Hookean tet gives NaN in both outputs."""
    mfs = _mfs()
    prob = _small_humanoid(31, 4000, 12)
    prob["model"] = np.array([(ARAP, COROT, NH)[k % 3] for k in range(len(prob["T"]))], dtype=np.int32)
    pose = random_pose(prob, 32, amp_deg=25.0)
    rng = np.random.default_rng(33)
    x = oracle.solve_frame(prob, pose, iterations=4)["x"].reshape(-1, 3)
    x = x + 1e-4 * prob["bbox_diag"] * rng.normal(size=x.shape)
    fr = oracle.Frame(prob, pose)
    assert fr.feasible(x.reshape(-1))
    _say(f"stress: n={fr.n} m={fr.m}")
    ch = mfs.Character(ctx, prob)
    P, L = ch.stress(*pose, x)
    Pr, Lr = oracle.stress(prob, pose, x)
    assert np.max(np.abs(P - Pr)) <= 1e-12 * np.max(np.abs(Pr))
    assert np.max(np.abs(L - Lr)) <= 1e-12 * np.max(np.abs(Lr))
    # device-memory path: same values bitwise
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    Pd = torch.empty((len(prob["T"]), 6), dtype=torch.float64, device="cuda")
    Ld = torch.empty((len(prob["T"]), 3, 3), dtype=torch.float64, device="cuda")
    ch.stress(*pose, xd, out=(Pd, Ld))
    assert np.array_equal(Pd.cpu().numpy(), P) and np.array_equal(Ld.cpu().numpy(), L)
    k = int(np.flatnonzero(fr.model == NH)[0])
    a, b = prob["T"][k][:2]
    xb = x.copy()
    xb[[a, b]] = xb[[b, a]]
    Pb, Lb = ch.stress(*pose, xb)
    Pbr, _ = oracle.stress(prob, pose, xb)
    bad = np.isnan(Pbr[:, 0])
    assert bad[k] and np.array_equal(np.isnan(Pb[:, 0]), bad) and np.all(np.isnan(Lb[bad]))
    ok = ~bad
    assert np.max(np.abs(Pb[ok] - Pbr[ok])) <= 1e-12 * np.max(np.abs(Pbr[ok]))
    ch.close()


def test_persistent_pcg(ctx):
    """The persistent pipelined PCG (one cooperative launch per Newton step):
    bitwise the iterates of the one-kernel-per-iteration form for every lane
    count (same frame, same statistics), one SpMV-family launch per Newton
    step, a batch bitwise equal to its members solved alone, and the
    full-size 50k golden within 1e-7 * bbox of the oracle."""
    import os
    mfs = _mfs()
    base = ctx.tuning()
    kw = dict(precision=mfs.FP32_REFINED, cg_tol=1e-5, step_tol=1e-9, max_newton=60, cg_adaptive=1)
    try:
        prob = _small_humanoid(21, 4000, 15)
        pose = random_pose(prob, 22)
        ch = mfs.Character(ctx, prob)
        for lpr in (2, 4, 8):
            ctx.set_tuning(pcg_pipelined=1, pcg_persistent=0, pcg_lanes_per_row=lpr, use_graphs=1,
                           graph_iterations=8)
            x0, st0, rc0 = ch.solve(*pose, **kw)
            assert rc0 == 0
            ctx.set_tuning(pcg_persistent=1)
            _say(f"persistent PCG: humanoid m={len(prob['T'])} lanes {lpr}")
            ctx.profile_enable(1)
            ctx.profile_read(reset=True)
            x1, st1, rc1 = ch.solve(*pose, **kw)
            prof = ctx.profile_read(reset=True)
            ctx.profile_enable(0)
            _say(f"  stats {st1}; spmv launches {prof['spmv'][2]}")
            assert rc1 == 0 and np.array_equal(x0, x1)
            for key in ("iterations", "cg_iterations", "status", "fp64_resolves"):
                assert st0[key] == st1[key], key
            assert prof["spmv"][2] == st1["iterations"] and prof["spmv"][3] > 0
        ch.close()
        ctx.set_tuning(pcg_pipelined=1, pcg_persistent=1, pcg_lanes_per_row=4)
        probs = [humanoid(100 + i, target_tets=t, n_bones=b, models=(NH, COROT))
                 for i, (t, b) in enumerate([(1500, 8), (3000, 12), (800, 10)])]
        poses = [random_pose(p, 200 + i) for i, p in enumerate(probs)]
        chars = [mfs.Character(ctx, p) for p in probs]
        alone = [c.solve(*q, **kw)[0] for c, q in zip(chars, poses)]
        _say("persistent PCG: batch of 3")
        xs, _, rc = mfs.solve_batch(ctx, chars, poses, **kw)
        assert rc == 0
        for a, b in zip(alone, xs):
            assert np.array_equal(a, b)
        for c in chars:
            c.close()
        here = os.path.dirname(os.path.abspath(__file__))
        g = np.load(os.path.join(here, "golden", "humanoid50k_pose2002.npz"))
        prob = humanoid(2001, target_tets=50000, n_bones=20)
        pose = random_pose(prob, 2002)
        ch = mfs.Character(ctx, prob)
        _say("persistent PCG: humanoid 50k golden")
        x, st, rc = ch.solve(*pose, precision=mfs.FP32_REFINED, cg_tol=1e-5, step_tol=1e-8, max_newton=60,
                             cg_adaptive=1)
        _say(f"  stats {st} err/bbox={_err(x, g['x'], prob):.3e}")
        assert rc == 0 and _err(x, g["x"], prob) <= 1e-7
        ch.close()
    finally:
        ctx.set_tuning(**base)


def test_rotation_smoothing(ctx):
    """Rotation smoothing (mfs_blend_weights, mfs_character_set_rotation_blend):
    blend handles equal to the oracle's and weights within 1e-12; with the
    oracle's blend, E, grad E and S within 1e-12 relative, stress and
    multipliers within 1e-12, FP64 frames within 1e-9 * bbox and FP32 +
    refinement within 1e-7 * bbox of the oracle's smoothed solution; clearing
    the blend gives the cluster solve again."""
    mfs = _mfs()
    prob = _small_humanoid(21, 4000, 15)
    pose = random_pose(prob, 22, amp_deg=30.0)
    width = 0.3
    _say(f"rotation smoothing: humanoid m={len(prob['T'])}, width {width}")
    Hr, Wr = oracle.blend_weights(prob["X"], prob["T"], prob["seg_a"], prob["seg_b"], prob["seg_handle"], width, 3)
    Hg, Wg = ctx.blend_weights(prob["X"], prob["T"], prob["seg_a"], prob["seg_b"], prob["seg_handle"],
                               prob["n_handles"], width, 3)
    assert np.array_equal(Hg, Hr)
    assert np.max(np.abs(Wg - Wr)) <= 1e-12
    assert np.mean(Hr[:, 1] >= 0) > 0.05  # a real share of tets blends
    pb = dict(prob, blend_handles=Hr, blend_weights=Wr)
    fr = oracle.Frame(pb, pose)
    rng = np.random.default_rng(5)
    ref = oracle.solve_frame(pb, pose, step_tol=1e-12, frame=fr)
    assert ref["status"] == "ok"
    x = ref["x"].reshape(-1, 3) + 1e-5 * prob["bbox_diag"] * rng.normal(size=(len(prob["X"]), 3))
    assert fr.feasible(x.reshape(-1))
    ch = mfs.Character(ctx, prob)
    x_cluster, _, rc = ch.solve(*pose, precision=mfs.FP64, step_tol=1e-10, cg_tol=1e-10, max_newton=60)
    ch.set_rotation_blend(Hr, Wr)
    ev = ch.evaluate(*pose, x)
    E = fr.energy(x.reshape(-1))
    g = fr.gradient(x.reshape(-1)).reshape(-1, 3)
    s = fr.stretch(x.reshape(-1))
    assert abs(ev["energy"] - E) <= 1e-12 * abs(E)
    assert np.max(np.abs(ev["grad"] - g)) <= 1e-11 * np.max(np.abs(g))
    assert np.max(np.abs(ev["stretch"] - s)) <= 1e-12 * max(1.0, np.abs(s).max())
    P, L = ch.stress(*pose, x)
    Pr, Lr = oracle.stress(pb, pose, x)
    assert np.max(np.abs(P - Pr)) <= 1e-12 * np.max(np.abs(Pr))
    assert np.max(np.abs(L - Lr)) <= 1e-12 * np.max(np.abs(Lr))
    x64, st, rc = ch.solve(*pose, precision=mfs.FP64, step_tol=1e-10, cg_tol=1e-10, max_newton=60)
    _say(f"  FP64 stats {st} err/bbox={_err(x64, ref['x'], prob):.3e}")
    assert rc == 0 and _err(x64, ref["x"], prob) <= 1e-9
    x32, st, rc = ch.solve(*pose, precision=mfs.FP32_REFINED, step_tol=1e-9, cg_tol=1e-5, max_newton=60,
                           cg_adaptive=1)
    assert rc == 0 and _err(x32, ref["x"], prob) <= 1e-7
    assert _err(x64, x_cluster, prob) > 1e-6  # smoothing changes the frame
    ch.set_rotation_blend(None)
    x0, _, rc = ch.solve(*pose, precision=mfs.FP64, step_tol=1e-10, cg_tol=1e-10, max_newton=60)
    assert rc == 0 and np.array_equal(x0, x_cluster)
    ch.close()


def test_two_contexts_concurrently(ctx):
    """Two contexts (two HIP streams) solving batches from two host threads at
    once give bitwise the results of the same batches solved one after the
    other: the library keeps no state across contexts."""
    from concurrent.futures import ThreadPoolExecutor
    mfs = _mfs()
    kw = dict(precision=mfs.FP32_REFINED, cg_tol=1e-5, step_tol=1e-9, max_newton=60, cg_adaptive=1)
    groups = [[(1500, 8), (900, 9)], [(3500, 12), (2500, 10)]]
    ctxs = [mfs.Context(0), mfs.Context(0)]
    probs = [[humanoid(1400 + 10 * g + i, target_tets=t, n_bones=b, models=(NH, COROT))
              for i, (t, b) in enumerate(spec)] for g, spec in enumerate(groups)]
    chars = [[mfs.Character(c, p) for p in ps] for c, ps in zip(ctxs, probs)]
    poses = [[random_pose(p, 1500 + i) for i, p in enumerate(ps)] for ps in probs]
    seq = [mfs.solve_batch(c, ch, po, **kw)[0] for c, ch, po in zip(ctxs, chars, poses)]
    _say("two contexts from two threads")
    with ThreadPoolExecutor(max_workers=2) as ex:
        par = list(ex.map(lambda g: mfs.solve_batch(ctxs[g], chars[g], poses[g], **kw)[0], range(2)))
    for a, b in zip(seq, par):
        for xa, xb in zip(a, b):
            assert np.array_equal(xa, xb)
    for ch in chars:
        for c in ch:
            c.close()
    for c in ctxs:
        c.close()
