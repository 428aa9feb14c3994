"""Write the oracle's solutions of the 64-character batch (one frame each).

Calls only the FP64 oracle and the seeded workload builders.  Every member of
the batch (64 humanoids of 5k-200k tets, log-uniform, 8-30 handles, mixed
neo-Hookean / co-rotated limbs; member k has mesh seed 4001 + k and pose seed
41000 + k, the batch's first step) is solved by ``oracle.solve_frame`` from
the rest shape with load stepping, to a Newton step below 1e-12 of the bbox
diagonal, with at most 100 iterations.

Outputs (tests/golden/):
  c4_oracle_summary.json  per member: size, handles, status, iterations, the
                          phases, step lengths, load-step fractions and
                          clamped-element counts of every iteration, and the
                          final gradient norm (the data behind the analysis of
                          members that do not converge);
  c4_oracle_subset.npz    x* of a size-stratified subset of the members the
                          oracle solves within 60 iterations (the batch's
                          Newton cap): the smallest, the three quartiles, the
                          largest and three seeded random others.  Positions
                          are stored for every vertex of members up to 4096
                          vertices and for a seeded sample of 4096 vertices
                          otherwise (with the sampled indices), plus a hash of
                          each member's inputs.

Run: python tests/golden/make_golden_c4.py [workers]   (about 30 minutes on
six cores; each worker holds at most about 2 GB)
"""

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

import oracle  # noqa: E402
from workloads import NH, COROT, pool_member, random_pose  # noqa: E402

COUNT, SEED0, TETS, HANDLES, MODELS = 64, 4001, (5000, 200000), (8, 30), (NH, COROT)
POSE_SEED0 = 41000
MAX_IT = 100
SUBSET_CAP = 60
SAMPLE = 4096


def input_hash(prob, pose):
    h = hashlib.sha256()
    for a in (prob["X"], prob["T"], prob["model"], prob["youngs"], prob["poisson"],
              prob["pin_vertex"], prob["pin_handle"], pose[0], pose[1]):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def solve_member(k):
    prob = pool_member(k, SEED0, TETS, HANDLES, MODELS)
    pose = random_pose(prob, POSE_SEED0 + k)
    t0 = time.time()
    r = oracle.solve_frame(prob, pose, max_iterations=MAX_IT)
    dt = time.time() - t0
    info = {
        "member": k, "m": int(len(prob["T"])), "n": int(len(prob["X"])),
        "handles": int(prob["n_handles"]), "status": r["status"], "iterations": int(r["iterations"]),
        "seconds": round(dt, 1),
        "phase": r["phase"], "alpha": [float(a) for a in r["alpha"]],
        "tau": [float(t) for t in r["tau"]], "clamped": [int(c) for c in r["clamped"]],
        "step": [float(s) for s in r["step"]],
        "final_grad_norm": float(r["grad_norm"][-1]),
        "final_energy": float(r["energy"][-1]),
        "bbox_diag": float(prob["bbox_diag"]),
        "input_hash": input_hash(prob, pose),
    }
    print(f"member {k}: m={info['m']} {r['status']} in {r['iterations']} iterations, {dt:.0f} s",
          flush=True)
    return info, r["x"]


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 6
    from concurrent.futures import ProcessPoolExecutor
    rng = np.random.default_rng(SEED0)
    sizes = [float(np.exp(np.random.default_rng(SEED0 + k).uniform(np.log(TETS[0]), np.log(TETS[1]))))
             for k in range(COUNT)]
    order = sorted(range(COUNT), key=lambda k: -sizes[k])  # longest first
    infos, xs = {}, {}
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for info, x in ex.map(solve_member, order):
            infos[info["member"]] = info
            xs[info["member"]] = x
    summary = [infos[k] for k in range(COUNT)]
    with open(os.path.join(HERE, "c4_oracle_summary.json"), "w") as f:
        json.dump(summary, f, indent=0)
    ok = sorted((k for k in range(COUNT)
                 if infos[k]["status"] == "ok" and infos[k]["iterations"] <= SUBSET_CAP),
                key=lambda k: (infos[k]["m"], k))
    picks = [ok[0], ok[len(ok) // 4], ok[len(ok) // 2], ok[(3 * len(ok)) // 4], ok[-1]]
    rest = [k for k in ok if k not in picks]
    picks += [int(k) for k in rng.choice(rest, size=3, replace=False)]
    out = {"members": np.array(picks, dtype=np.int32)}
    srng = np.random.default_rng(SEED0 + 1)
    for k in picks:
        n = infos[k]["n"]
        idx = np.arange(n) if n <= SAMPLE else np.sort(srng.choice(n, SAMPLE, replace=False))
        out[f"x_{k}"] = xs[k][idx]
        out[f"idx_{k}"] = idx.astype(np.int32)
        out[f"hash_{k}"] = np.array(infos[k]["input_hash"])
        out[f"iterations_{k}"] = np.array(infos[k]["iterations"])
    np.savez_compressed(os.path.join(HERE, "c4_oracle_subset.npz"), **out)
    bad = [k for k in range(COUNT) if infos[k]["status"] != "ok"]
    print(f"subset {picks}; not converged within {MAX_IT}: {bad}")


if __name__ == "__main__":
    main()
