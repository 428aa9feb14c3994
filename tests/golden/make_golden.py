"""Write the oracle's expected frame solutions for the full-size parity tests.

Calls only the FP64 oracle and the seeded workload builders.  Output:
tests/golden/humanoid50k_pose2002.npz with the converged positions x* of
the ~50k-tet humanoid (mesh seed 2001, 20 handles) at random pose seed 2002,
the oracle's per-iteration history, and a hash of the inputs so a test can
tell that it rebuilt the same mesh.

Run: python tests/golden/make_golden.py   (about a minute on one core)
"""

import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workloads import humanoid, random_pose  # noqa: E402


def input_hash(prob, pose):
    h = hashlib.sha256()
    for a in (prob["X"], prob["T"], prob["model"], prob["youngs"], prob["poisson"],
              prob["pin_vertex"], prob["pin_handle"], pose[0], pose[1]):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    prob = humanoid(2001, target_tets=50000, n_bones=20)
    pose = random_pose(prob, 2002)
    r = oracle.solve_frame(prob, pose)
    assert r["status"] == "ok", r["status"]
    out = os.path.join(HERE, "humanoid50k_pose2002.npz")
    np.savez_compressed(out, x=r["x"], energy=np.array(r["energy"]),
                        grad_norm=np.array(r["grad_norm"]), alpha=np.array(r["alpha"]),
                        iterations=r["iterations"], input_hash=input_hash(prob, pose))
    print(f"wrote {out}: {r['iterations']} iterations, final |grad E| = {r['grad_norm'][-1]:.3e}")


if __name__ == "__main__":
    main()
