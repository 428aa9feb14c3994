"""Host-side checks of the benchmark (no GPU): the multi-GPU request is
refused with a message, and the workload definitions the bench times are the
configurations they are named for (sizes, handles, materials, options)."""

import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_beam_workload():
    """16 x 4 x 4 unit cubes split into 6 tets each, neo-Hookean E = 1e5,
    nu = 0.45, two handles; FP64, exactly 10 Newton iterations, PCG to 1e-10;
    the far cap turned 30 degrees about the beam axis and moved 2 units."""
    from bench import make_workload
    from workloads import NH
    probs, pose_of, name, opts = make_workload("c1")
    p = probs[0]
    assert len(p["T"]) == 16 * 4 * 4 * 6 and len(p["X"]) == 17 * 5 * 5
    assert p["n_handles"] == 2
    assert np.all(np.asarray(p["model"]) == NH)
    assert np.all(np.asarray(p["youngs"]) == 1e5) and np.all(np.asarray(p["poisson"]) == 0.45)
    assert opts == dict(precision=0, cg_tol=1e-10, max_newton=10, fixed_newton=1)
    R, t = pose_of(0)[0]
    moved = [h for h in range(2) if not np.allclose(R[h], np.eye(3))]
    assert len(moved) == 1
    h = moved[0]
    assert np.isclose(np.degrees(np.arccos((np.trace(R[h]) - 1.0) / 2.0)), 30.0)
    assert np.allclose(R[h] @ [1.0, 0.0, 0.0], [1.0, 0.0, 0.0])  # about the beam (x) axis


def test_humanoid_workload():
    """About 50k tets and 20 bone handles; neo-Hookean or ARAP per limb, E
    log-uniform in [1e4, 1e6], nu uniform in [0.3, 0.49]; the bench's
    FP32 + refinement options."""
    from bench import make_workload
    from workloads import ARAP, NH
    probs, pose_of, name, opts = make_workload("c2")
    p = probs[0]
    assert 0.9 * 50000 <= len(p["T"]) <= 1.1 * 50000
    assert p["n_handles"] == 20
    assert set(np.asarray(p["model"]).tolist()) <= {NH, ARAP}
    assert 1e4 <= np.min(p["youngs"]) and np.max(p["youngs"]) <= 1e6
    assert 0.3 <= np.min(p["poisson"]) and np.max(p["poisson"]) <= 0.49
    assert opts["precision"] == 1 and opts["max_newton"] == 60 and opts["step_tol"] == 1e-8
    assert pose_of(0)[0][0].shape == (20, 3, 3)


def test_batch_pool_members():
    """Members of the batched pool: sizes log-uniform in 5k-200k tets,
    8-30 handles, neo-Hookean or co-rotated per limb; each member is built
    from its own seed, so the first three come out the same alone."""
    from workloads import COROT, NH
    from workloads.humanoid import _pool_member
    for k in range(3):
        q = _pool_member((k, 4001, (5000, 200000), (8, 30), (NH, COROT)))
        assert 0.8 * 5000 <= len(q["T"]) <= 1.2 * 200000
        assert 8 <= q["n_handles"] <= 30
        assert set(np.asarray(q["model"]).tolist()) <= {NH, COROT}


def test_large_animation_workload():
    """About 500k tets and 30 handles, frames warm-started from the previous
    one, with the same FP32 + refinement options; consecutive frames of the
    animation are close (smooth joint angles at 30 frames per second)."""
    from bench import make_workload
    probs, pose_of, name, opts = make_workload("c3")
    p = probs[0]
    assert 0.9 * 500000 <= len(p["T"]) <= 1.1 * 500000
    assert p["n_handles"] == 30
    assert opts["warm_start"] == 1 and opts["precision"] == 1
    # each joint's rotation relative to its parent moves by at most three
    # Euler angles of a 60-degree sinusoid with a period of at least 2 s over
    # one frame at 30 frames per second: 3 * 60 * 2 pi / (2 * 30) degrees
    parent = np.asarray(p["handle_parent"])

    def local(R):
        return [R[h] if parent[h] < 0 else R[parent[h]].T @ R[h] for h in range(len(R))]

    def angle(a, b):
        return np.degrees(np.arccos(np.clip((np.trace(a.T @ b) - 1.0) / 2.0, -1.0, 1.0)))

    bound = 3 * 60.0 * 2 * np.pi / (2.0 * 30.0)
    for f in range(3):
        L0, L1 = local(pose_of(f)[0][0]), local(pose_of(f + 1)[0][0])
        steps = [angle(a, b) for a, b in zip(L0, L1)]
        assert 0.0 < max(steps) <= bound


def test_roofline_byte_count_and_traffic_summaries():
    """The algorithmic bytes of one SpMV-family launch follow the block-sparse
    count (every block's nine values and column, the row pointers, one input
    and one output vector; the pipelined kernel adds twelve vector passes and
    the preconditioner rows): the C1 beam's 425 vertices and 4,921 blocks
    give 208,744 bytes in FP32.  A committed counter summary is read back
    only while the kernel sources hash to the value it records, and then its
    counted and algorithmic bytes are the ones its table states."""
    sys.path.insert(0, ROOT)
    import bench
    info = {"n_vertices": 425, "n_blocks": 4921}
    assert bench.spmv_algorithmic_bytes(info, 4, False) == 4921 * 40 + 4 * 426 + 24 * 425 == 208744
    assert bench.spmv_algorithmic_bytes(info, 8, True) == 4921 * 76 + 4 * 426 + 48 * 425 + 336 * 425
    import glob
    for path in glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.md")):
        text = open(path).read()
        fields = dict(line[2:].split(": ", 1) for line in text.splitlines() if line.startswith("- ") and ": " in line)
        fields = {k.strip("`"): v.strip().strip("`") for k, v in fields.items()}
        got = bench.counted_traffic(fields["workload"], fields["kernel"])
        if fields["kernel_sources_sha256"] != bench.kernel_source_hash():
            assert got is None
            continue
        assert got["counted_bytes_per_dispatch"] == float(fields["traffic_bytes_per_launch"])
        assert got["algorithmic_bytes_per_dispatch"] == float(fields["algorithmic_bytes_per_launch"])
        ratio = [line for line in text.splitlines() if line.startswith("| traffic / algorithmic |")][0]
        stated = float(ratio.split("|")[2])
        assert abs(got["counted_bytes_per_dispatch"] / got["algorithmic_bytes_per_dispatch"] - stated) < 1e-3


def test_ordinals():
    sys.path.insert(0, ROOT)
    import bench
    assert [bench.ordinal(k) for k in (1, 2, 3, 4, 11, 12, 13, 21, 22, 32, 111, 112)] == \
        ["1st", "2nd", "3rd", "4th", "11th", "12th", "13th", "21st", "22nd", "32nd", "111th", "112th"]
