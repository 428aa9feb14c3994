"""GPU test of the PCG schedule autotuner (``mfs_autotune`` through the C ABI).

The tuner must apply its choice to the context, keep it per size class in
the context and in the cache file, reuse it without re-timing, and leave
solves correct: a frame solved under the tuned schedule matches the one
solved under the default schedule within the FP64 tolerance (only the SpMV
summation order may change), and a batch under it still equals its members
solved alone bitwise.
"""

import sys
import time

import numpy as np
import pytest

from workloads import NH, COROT, humanoid, random_pose

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_autotune_applies_caches_and_keeps_results(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2408_04066_amd as mfs
    ctx = mfs.Context(0)
    probs = [humanoid(800 + i, target_tets=t, n_bones=b, models=(NH, COROT))
             for i, (t, b) in enumerate([(2500, 10), (1200, 8)])]
    poses = [random_pose(p, 900 + i) for i, p in enumerate(probs)]
    chars = [mfs.Character(ctx, p) for p in probs]
    default = ctx.tuning()
    ref = [ch.solve(*pose)[0] for ch, pose in zip(chars, poses)]
    cache = tmp_path / "tune.txt"
    _say("autotune: 2 characters, FP32 + refinement")
    opts = dict(precision=mfs.FP32_REFINED, cg_tol=1e-5, step_tol=1e-9, cg_adaptive=1)
    best, ms = mfs.autotune(ctx, chars, poses, newton_iterations=3, cache_path=str(cache), **opts)
    _say(f"  best {best} {ms:.2f} ms (default {default})")
    assert ms > 0 and ctx.tuning() == best
    assert best["pcg_lanes_per_row"] in (2, 4, 8) and best["use_graphs"] == 1
    lines = cache.read_text().split("\n")
    assert len([ln for ln in lines if ln.strip()]) == 1 and lines[0].startswith("gfx950 ")
    # a fresh context takes the cached choice without timing
    ctx.set_tuning(**default)
    ctx2 = mfs.Context(0)
    chars2 = [mfs.Character(ctx2, p) for p in probs]
    t0 = time.time()
    best2, ms2 = mfs.autotune(ctx2, chars2, poses, newton_iterations=3, cache_path=str(cache), **opts)
    assert best2 == best and ms2 == pytest.approx(ms, rel=1e-6)
    assert ctx2.tuning() == best and time.time() - t0 < 5.0
    # tuned schedule: same frames (FP64 tolerance), batch == alone bitwise
    xs = [ch.solve(*pose)[0] for ch, pose in zip(chars2, poses)]
    for a, b, p in zip(xs, ref, probs):
        assert np.max(np.linalg.norm(a - b, axis=1)) / p["bbox_diag"] <= 1e-9
    alone = [ch.solve(*pose, **opts)[0] for ch, pose in zip(chars2, poses)]
    batch, _, rc = mfs.solve_batch(ctx2, chars2, poses, **opts)
    assert rc == 0
    for a, b in zip(alone, batch):
        assert np.array_equal(a, b)
    for ch in chars + chars2:
        ch.close()
    ctx2.close()
    ctx.close()
