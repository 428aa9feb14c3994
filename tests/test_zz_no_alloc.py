"""The allocation-free evaluation (mfs_evaluate_noalloc) against mfs_evaluate.

Through the C ABI: two allocation-free calls in a row on one GPU, the second
on a smaller character (so the shared scratch array holds the first call's
data when the second starts), each compared with mfs_evaluate of the same
state: energy, gradient, stretches and K v, host and device memory; and a
character too large for the scratch array is rejected before any GPU work.
"""

import sys

import numpy as np
import pytest

from workloads import beam, humanoid

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mfs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2408_04066_amd as m
    return m


def _state(prob, seed):
    """A feasible state: every handle on one random rigid motion (R, c), and x
    that motion applied to the rest shape perturbed by 1% of the bbox
    diagonal over sqrt(n); a random probe vector v."""
    from workloads import euler_xyz
    rng = np.random.default_rng(seed)
    X = np.asarray(prob["X"], dtype=np.float64)
    R = euler_xyz(*rng.uniform(-np.pi, np.pi, 3))
    c = rng.standard_normal(3)
    nh = int(prob["n_handles"])
    pose = (np.tile(R, (nh, 1, 1)), np.tile(c, (nh, 1)))
    Xp = X + 0.01 * prob["bbox_diag"] * rng.standard_normal(X.shape) / np.sqrt(len(X))
    x = Xp @ R.T + c
    v = rng.standard_normal(X.shape)
    return pose, x, v


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b))) / max(float(np.max(np.abs(b))), 1e-300)


def test_noalloc_evaluation_equals_evaluate(mfs):
    ctx = mfs.Context(0)
    big = humanoid(2001, target_tets=20000, n_bones=20)
    small = humanoid(21, target_tets=4000, n_bones=15)
    cases = []
    for prob, seed in ((big, 1), (small, 2)):
        ch = mfs.Character(ctx, prob)
        pose, x, v = _state(prob, seed)
        cases.append((prob, ch, pose, x, v))
    # two allocation-free calls in a row, the second on the smaller character
    got = []
    for prob, ch, pose, x, v in cases:
        _say(f"noalloc evaluation: m={len(prob['T'])} n={len(prob['X'])}")
        got.append(ch.evaluate(*pose, x, v=v, noalloc=True))
    for (prob, ch, pose, x, v), g in zip(cases, got):
        ref = ch.evaluate(*pose, x, v=v)
        e_rel = abs(g["energy"] - ref["energy"]) / abs(ref["energy"])
        errs = {k: _rel(g[k], ref[k]) for k in ("grad", "stretch", "Kv")}
        same = all(np.array_equal(g[k], ref[k]) for k in ("grad", "stretch", "Kv")) and g["energy"] == ref["energy"]
        _say(f"  m={len(prob['T'])}: energy rel {e_rel:.2e}, {errs}, bitwise {same}")
        assert np.isfinite(ref["energy"])
        assert e_rel <= 1e-12
        assert all(e <= 1e-12 for e in errs.values())
    # device memory: the smaller character again, inputs and outputs on the GPU
    prob, ch, pose, x, v = cases[1]
    ref = ch.evaluate(*pose, x, v=v)
    import ctypes
    R, t = ch._pose(*pose)
    xd = torch.as_tensor(x, device="cuda")
    vd = torch.as_tensor(v, device="cuda")
    gd = torch.empty_like(xd)
    kd = torch.empty_like(xd)
    sd = torch.empty((ch.m, 6), dtype=torch.float64, device="cuda")
    E = ctypes.c_double()
    rc = mfs.lib().mfs_evaluate_noalloc(ch.handle, R.ctypes.data, t.ctypes.data, xd.data_ptr(), vd.data_ptr(),
                                        mfs.MEM_DEVICE, ctypes.byref(E), gd.data_ptr(), sd.data_ptr(), kd.data_ptr())
    assert rc == 0
    torch.cuda.synchronize()
    assert abs(E.value - ref["energy"]) <= 1e-12 * abs(ref["energy"])
    assert _rel(gd.cpu().numpy(), ref["grad"]) <= 1e-12
    assert _rel(sd.cpu().numpy(), ref["stretch"]) <= 1e-12
    assert _rel(kd.cpu().numpy(), ref["Kv"]) <= 1e-12
    for _, ch, _, _, _ in cases:
        ch.close()
    # a character beyond the scratch array: a clear error, nothing run
    huge = beam(128, 8, 8)
    ch = mfs.Character(ctx, huge)
    pose, x, v = _state(huge, 3)
    with pytest.raises(mfs.MfsError) as e:
        ch.evaluate(*pose, x, v=v, noalloc=True)
    assert e.value.code == -1 and "scratch" in str(e.value)
    _say(f"  m={len(huge['T'])} rejected: {e.value}")
    ch.close()
    ctx.close()
