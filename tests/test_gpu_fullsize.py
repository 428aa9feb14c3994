"""Parity at the benchmark's full sizes, in the launch configuration the bench
times (its workload definitions and solve options, the autotuned PCG
schedule), where the oracle cannot solve the frame itself in seconds.

What the oracle checks there is what holds at any size: its energy and
gradient evaluated at the GPU's solution equal the library's own evaluation
of the same state (the full-size element pass); the solution is stationary
(the oracle's largest residual force there is orders below the largest pin
force at the rest shape, the load the elastic forces balance); and the
FP32 + refinement solution lies within 1e-7 of the bbox diagonal of a tight
FP64 solve continued from it, itself stationary by the oracle's gradient.
The batched workload is checked on a sample of its members after one
batched solve of all of them, and its positions are compared with the
oracle's own solutions of a size-stratified subset of the members.
"""

import os
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# a tight FP64 solve continued from the character's last solution (a pose
# far from the rest shape need not converge from there at all)
TIGHT = dict(precision=0, cg_tol=1e-10, step_tol=1e-12, cg_adaptive=0, max_newton=200, warm_start=1)
# largest per-vertex residual force at the solution over the applied force scale
# (measured: at most 8e-15 for the tight solves and 1.1e-11 with the bench's
# options, over the five solutions checked here)
R_TIGHT = 1e-12  # tight FP64 solve
R_BENCH = 1e-9  # the bench's options (Newton step below 1e-8 of the bbox)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mfs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2408_04066_amd as m
    return m


def _tight(ctx, ch, pose):
    """The tight FP64 solve, continued from ch's last solution, in the
    two-kernel PCG form (the pipelined recurrences can drift from the true
    residual near a 1e-10 tolerance); the context's schedule is restored."""
    saved = ctx.tuning()
    ctx.set_tuning(pcg_pipelined=0, pcg_persistent=0)
    try:
        return ch.solve(*pose, **TIGHT)
    finally:
        ctx.set_tuning(**saved)


def _err(x, ref, bbox):
    return float(np.max(np.linalg.norm(x - ref, axis=1))) / bbox


def _force_scale(fr, prob):
    """Largest pin force at the rest shape under the pose, k_s |P X - y|: the
    applied load that the elastic forces balance at the solution."""
    X = np.asarray(prob["X"], dtype=np.float64).reshape(-1)
    return fr.ks * float(np.max(np.linalg.norm(fr.pin_residual(X), axis=1)))


def _check_state(fr, scale, ch, pose, x, label):
    """Oracle energy and gradient at x against the library's evaluation of the
    same state; returns (E(x), max |grad E(x)| / scale) by the oracle."""
    xf = x.reshape(-1)
    E = fr.energy(xf)
    g = fr.gradient(xf).reshape(-1, 3)
    out = ch.evaluate(*pose, x, want_stretch=False)
    rel_e = abs(out["energy"] - E) / abs(E)
    rel_g = float(np.max(np.abs(out["grad"] - g))) / scale
    ratio = float(np.max(np.linalg.norm(g, axis=1))) / scale
    _say(f"  {label}: energy {E:.9e} (library rel diff {rel_e:.2e}), gradient diff / scale {rel_g:.2e}, "
         f"max |grad E(x)| / scale {ratio:.2e}")
    assert rel_e <= 1e-10
    assert rel_g <= 1e-11
    return E, ratio


def test_large_character_at_full_size(mfs):
    """The 505k-tet character of the warm-started animation as the bench runs
    it (autotuned schedule, frames warm-started from the previous one): the
    third frame, the first the bench times."""
    from bench import make_workload
    probs, pose_of, wname, opts = make_workload("c3")
    prob = probs[0]
    _say(f"{wname}: m={len(prob['T'])} n={len(prob['X'])}")
    ctx = mfs.Context(0)
    ch = mfs.Character(ctx, prob)
    t, _ = mfs.autotune(ctx, [ch], [pose_of(0)[0]], newton_iterations=2, **opts)
    _say(f"  schedule {t}")
    for f in range(3):
        pose = pose_of(f)[0]
        x32, st32, rc32 = ch.solve(*pose, **opts)
        _say(f"  frame {f}, FP32 + refinement: {st32}")
    xt, stt, rct = _tight(ctx, ch, pose)
    _say(f"  tight FP64: {stt}")
    assert rc32 == 0 and rct == 0
    e = _err(x32, xt, prob["bbox_diag"])
    _say(f"  |x32 - x_tight| / bbox = {e:.3e}")
    assert e <= 1e-7
    fr = oracle.Frame(prob, pose)
    scale = _force_scale(fr, prob)
    E_t, r_t = _check_state(fr, scale, ch, pose, xt, "tight FP64")
    E_32, r_32 = _check_state(fr, scale, ch, pose, x32, "FP32 + refinement")
    assert r_t <= R_TIGHT and r_32 <= R_BENCH
    assert abs(E_32 - E_t) <= 1e-9 * abs(E_t)
    ch.close()
    ctx.close()


GOLDEN_C4 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c4_oracle_subset.npz")


@pytest.fixture(scope="module")
def c4_batch(mfs):
    """The 64-character batch, autotuned and solved once in one batched run
    with the bench's options: (probs, poses, ctx, chars, xs, stats, opts)."""
    import bench
    # the pool does not depend on the worker count; this process already
    # holds the GPU, so few forked builders keep the count of processes low
    bench._workers = lambda: 8
    probs, pose_of, wname, opts = bench.make_workload("c4")
    poses = pose_of(0)
    _say(f"{wname}: {len(probs)} characters, {sum(len(p['T']) for p in probs)} tets")
    ctx = mfs.Context(0)
    chars = [mfs.Character(ctx, p) for p in probs]
    t, _ = mfs.autotune(ctx, chars, poses, newton_iterations=2, **opts)
    _say(f"  schedule {t}")
    xs, sts, rc = mfs.solve_batch(ctx, chars, poses, **opts)
    yield probs, poses, ctx, chars, [x.copy() for x in xs], sts, opts
    for c in chars:
        c.close()
    ctx.close()


def test_batched_positions_match_oracle_solutions(c4_batch):
    """The oracle's solved positions x* of a size-stratified subset of the
    batch's members (smallest, quartiles, largest and three random ones,
    written by tests/golden/make_golden_c4.py from the oracle alone) against
    the batched FP32 + refinement result, within 1e-7 of the bbox diagonal,
    and a tight FP64 solve continued from it, within 1e-9 (Algorithm 1's
    output: the deformed positions)."""
    probs, poses, ctx, chars, xs, sts, _ = c4_batch
    sys.path.insert(0, os.path.dirname(GOLDEN_C4))
    from make_golden_c4 import input_hash
    gold = np.load(GOLDEN_C4, allow_pickle=False)
    for k in gold["members"]:
        k = int(k)
        prob, pose = probs[k], poses[k]
        assert str(gold[f"hash_{k}"]) == input_hash(prob, pose), f"member {k}: inputs differ from the golden's"
        idx = gold[f"idx_{k}"]
        xo = gold[f"x_{k}"]
        bbox = prob["bbox_diag"]
        _say(f"  member {k}: m={len(prob['T'])} oracle {int(gold[f'iterations_{k}'])} iterations, "
             f"batch {sts[k]}")
        assert sts[k]["status"] == 0, f"member {k} did not converge in the batch"
        e32 = _err(xs[k][idx], xo, bbox)
        xt, stt, rct = _tight(ctx, chars[k], pose)
        e64 = _err(xt[idx], xo, bbox)
        _say(f"  member {k}: |x_batch - x*| / bbox = {e32:.3e}, |x_tight_fp64 - x*| / bbox = {e64:.3e}")
        assert rct == 0
        assert e32 <= 1e-7
        assert e64 <= 1e-9


# Members of the 64-character batch (first poses) that are known not to
# converge, with the reason.  The oracle's own solve (exact sparse LU solves,
# up to 100 Newton iterations, tests/golden/c4_oracle_summary.json) does not
# converge on these poses either.  Each uses all six load-step bisections:
# in the mixed phase a few tens of neo-Hookean tets keep the stretch step
# below 1/4 (the poses turn some element clusters by more than 90 degrees
# against their neighbours, where the neo-Hookean energy of the rig-fixed
# rotations is infinite).
KNOWN_UNCONVERGED_C4 = {
    26: "reaches the final pose after 78 iterations (67 mixed), then converges "
        "linearly (step ratio about 0.56) past the iteration cap",
    29: "mixed phase stalls at 28% of the pose (78 of 100 iterations mixed)",
    50: "mixed phase stalls at 72% of the pose (87 of 100 iterations mixed)",
    52: "mixed phase stalls at 97% of the pose (90 of 100 iterations mixed)",
    53: "mixed phase stalls at the final pose (77 of 100 iterations mixed)",
    59: "mixed phase stalls at 81% of the pose (89 of 100 iterations mixed)",
}


def test_batched_characters_at_full_size(c4_batch):
    """Members of the same batched run (smallest, largest and two between)
    checked by the oracle's energy and gradient against a tight FP64 solve;
    every member outside the known unconverged ones converges."""
    probs, poses, ctx, chars, xs, sts, _ = c4_batch
    sizes = np.array([len(p["T"]) for p in probs])
    order = np.argsort(sizes)
    conv = [k for k in order if sts[k]["status"] == 0]
    unconv = sorted(int(k) for k in range(len(probs)) if sts[k]["status"] != 0)
    _say(f"  unconverged: {[(k, sts[k]['iterations'], sts[k]['mixed_iterations']) for k in unconv]}")
    surprise = [k for k in unconv if k not in KNOWN_UNCONVERGED_C4]
    assert not surprise, f"members {surprise} did not converge: {[sts[k] for k in surprise]}"
    # four members spread over the sizes; a member whose tight solve does not
    # converge either (a pose that leaves elements inverted) gives way to the
    # next converged member in size order.  A converged member whose Newton
    # systems needed FP64 re-solves (the FP32 PCG stagnated; the FP64 PCG
    # starts from the FP32 iterate) is checked too when the batch has one.
    resolved = [k for k in conv if sts[k]["fp64_resolves"] > 0]
    _say(f"  converged {len(conv)} of {len(probs)}; with FP64 re-solves: {resolved}")
    groups = [conv[0:], conv[len(conv) // 3:], conv[2 * len(conv) // 3:], conv[::-1]]
    if resolved:
        groups.append(resolved)
    checked = 0
    for group in groups:
        for k in group:
            prob, pose = probs[k], poses[k]
            _say(f"  member {k}: m={sizes[k]} stats {sts[k]}")
            xt, stt, rct = _tight(ctx, chars[k], pose)
            if rct != 0:
                _say(f"  member {k}: tight FP64 did not converge ({stt}); next member")
                continue
            e = _err(xs[k], xt, prob["bbox_diag"])
            _say(f"  member {k}: |x_batch - x_tight| / bbox = {e:.3e}")
            assert e <= 1e-7
            fr = oracle.Frame(prob, pose)
            scale = _force_scale(fr, prob)
            E_t, r_t = _check_state(fr, scale, chars[k], pose, xt, f"member {k} tight FP64")
            E_b, r_b = _check_state(fr, scale, chars[k], pose, xs[k], f"member {k} batched FP32 + refinement")
            assert r_t <= R_TIGHT and r_b <= R_BENCH
            assert abs(E_b - E_t) <= 1e-9 * abs(E_t)
            checked += 1
            break
    assert checked == len(groups)


def test_served_positions_match_oracle_solutions(c4_batch, mfs):
    """The serving path on the same size-stratified subset: the eight members
    with oracle solutions, each next to another converging member, submitted
    in one burst to a server with two size-class lanes (the serving
    workload's layout, four slots per lane), solved from the rest shape with
    the bench's options.  Each served result against the oracle's x* within
    1e-7 of the bbox diagonal (Algorithm 1's output for every request), and
    bitwise equal to the same member's result in the batched run: the lanes
    take the context's PCG schedule, and a solve's arithmetic does not
    depend on the solves beside it."""
    probs, poses, ctx, chars, xs, sts, opts = c4_batch
    gold = np.load(GOLDEN_C4, allow_pickle=False)
    members = [int(k) for k in gold["members"]]
    others = [k for k in range(len(probs)) if k not in members and k not in KNOWN_UNCONVERGED_C4][:len(members)]
    order = [k for pair in zip(members, others) for k in pair]
    sizes = sorted(len(probs[k]["T"]) for k in order)
    bound = sizes[len(sizes) // 2]
    _say(f"  serving {len(order)} requests, lanes split at {bound} tets")
    srv = mfs.Server(ctx, slots=4, lane_max_tets=(bound,), **opts)
    try:
        tickets = [(k, srv.submit(chars[k], *poses[k])) for k in order]
        res = {k: srv.wait(t) for k, t in tickets}
        info = srv.info()
    finally:
        srv.close()
    _say(f"  server: {info}")
    assert info["completed"] == len(order)
    for k in members:
        x, st, tm, rc = res[k]
        idx = gold[f"idx_{k}"]
        e = _err(x[idx], gold[f"x_{k}"], probs[k]["bbox_diag"])
        d = _err(x, xs[k], probs[k]["bbox_diag"])
        _say(f"  member {k}: served {st}; |x_served - x*| / bbox = {e:.3e}, |x_served - x_batch| / bbox = {d:.3e}")
        assert rc == 0 and st["status"] == 0
        assert e <= 1e-7
        assert np.array_equal(x, xs[k])
