"""Benchmark of the mixed-FEM skinning frame solve on one MI355X.

Default workload (``--workload c2``): a seeded procedural humanoid of ~50k
tets / ~10k vertices with 20 bone handles, neo-Hookean or ARAP per limb
(E log-uniform in [1e4, 1e6], nu uniform in [0.3, 0.49]); each step solves
one frame at a fresh random pose (joint Euler angles uniform in +-45 degrees)
from the rest shape.  ``c1`` is the 16x4x4 neo-Hookean beam, ``c3`` the same
humanoid generator at ~500k tets / 30 handles, ``c4`` a batch of 64 humanoids
of 5k-200k tets (log-uniform), 8-30 handles, neo-Hookean / co-rotated per
limb, solved together in one batched run per step.

The timed path is the FP32 + FP64-refinement form (FP32 Hessian values and
PCG; FP64 residual, energies and updates), inexact Newton (Eisenstat-Walker
forcing over a 1e-5 PCG floor), stopped at a 1e-8 * bbox Newton step.  The
FP64 form of the same solve (identical options, FP64 Hessian and PCG) runs
beside it on the first poses and the two results are compared.  Characters
are resident in HBM before timing; a step uploads only handle transforms
and writes positions to device tensors.

Prints one JSON line: throughput in tet * Newton-iterations / s, frames/s,
p50/p99 frame latency, the roofline entry of the dominant kernel (the PCG
block-sparse matrix-vector product; algorithmic bytes over HIP-event time,
measured in a second pass over the same frames with the event profiler on)
and the FP64 CPU oracle timed on this host on a bounded sample.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def make_workload(name):
    """(problems, pose_of(step) -> list of poses, workload name)."""
    from workloads import NH, COROT, humanoid, random_pose, beam, beam_pose, character_pool
    if name == "c1":
        p = beam()
        return [p], (lambda i: [beam_pose(p)]), "beam_16x4x4_neohookean_twist30_stretch2"
    if name == "c2":
        p = humanoid(2001, target_tets=50000, n_bones=20)
        return [p], (lambda i: [random_pose(p, 2002 + i)]), "humanoid_50k_tets_20_handles_random_pose"
    if name == "c3":
        p = humanoid(3001, target_tets=500000, n_bones=30)
        return [p], (lambda i: [random_pose(p, 3002 + i)]), "humanoid_500k_tets_30_handles_random_pose"
    if name == "c4":
        ps = character_pool(64, 4001, (5000, 200000), (8, 30), (NH, COROT))
        return ps, (lambda i: [random_pose(p, 41000 + 100 * i + k) for k, p in enumerate(ps)]), \
            "batch_64_humanoids_5k_200k_tets_8_30_handles"
    raise SystemExit(f"unknown workload {name}")


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "hbm_traffic_spmv_humanoid50k.md")
TRAFFIC_SOURCES = ("paper_2408_04066_amd/csrc/kernels_cg.hip", "paper_2408_04066_amd/csrc/common.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counted_traffic(workload):
    """HBM bytes per SpMV launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (copy-kernel scaled), or None when that summary is
    for another workload or the kernel sources changed since it was taken."""
    try:
        lines = open(TRAFFIC_SUMMARY).read().splitlines()
    except OSError:
        return None
    kv = {}
    for line in lines:
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            kv[k.strip("`")] = v.strip().strip("`")
    if kv.get("workload") != workload or kv.get("kernel_sources_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(prob, pose, iterations=2):
    """The FP64 oracle, single-threaded, on the first `iterations` Newton
    iterations of one frame (rest -> pose)."""
    import oracle
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(1)
    except Exception:
        limiter = None
    t0 = time.perf_counter()
    fr = oracle.Frame(prob, pose)
    t1 = time.perf_counter()
    r = oracle.solve_frame(prob, pose, iterations=iterations, frame=fr)
    t2 = time.perf_counter()
    if limiter is not None and hasattr(limiter, "unregister"):
        limiter.unregister()
    m = len(prob["T"])
    return {
        "value": m * r["iterations"] / (t2 - t1),
        "unit": "tet*Newton-iter/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"first {r['iterations']} Newton iterations of one frame of a {m}-tet character, "
                   f"FP64 numpy/scipy SuperLU, 1 thread; {t2 - t1:.1f} s solve + {t1 - t0:.1f} s "
                   f"setup (setup excluded)"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--profile-stride", type=int, default=8)
    ap.add_argument("--roofline-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB (the reference kernel "
                         "that scales HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: one character's frame solve is not split across "
              "GPUs in this build (DESIGN.md describes how it would shard)", file=sys.stderr)
        return 2
    if int(os.environ.get("RANK", "0")) != 0:
        return 0

    import torch
    import paper_2408_04066_amd as mfs

    if args.copy_mb > 0:
        src = torch.ones(args.copy_mb << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    probs, pose_of, wname = make_workload(args.workload)
    ctx = mfs.Context(0)
    chars = [mfs.Character(ctx, p) for p in probs]
    infos = [c.info() for c in chars]
    m_tot = sum(i["n_tets"] for i in infos)
    outs = [torch.empty((i["n_vertices"], 3), dtype=torch.float64, device="cuda") for i in infos]
    steps = [pose_of(i) for i in range(args.warmup + args.steps)]
    common = dict(cg_tol=1e-5, step_tol=1e-8, max_newton=60, cg_adaptive=1)
    fp32_opts = dict(precision=mfs.FP32_REFINED, **common)
    fp64_opts = dict(precision=mfs.FP64, **common)

    def frame(poses, opts):
        if len(chars) == 1:
            _, st, rc = chars[0].solve(*poses[0], out=outs[0], **opts)
            return [st], rc
        _, sts, rc = mfs.solve_batch(ctx, chars, poses, outs=outs, **opts)
        return sts, rc

    for i in range(args.warmup):
        frame(steps[i], fp32_opts)
    torch.cuda.synchronize()

    # ---- timed region: FP32 + FP64 refinement (PCG runs replayed as graphs) ----
    lat, tet_iters, iters, cgs, rcs, conv = [], 0, [], [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        sts, rc = frame(steps[args.warmup + i], fp32_opts)
        lat.append(time.perf_counter() - ts)
        tet_iters += sum(inf["n_tets"] * st["iterations"] for inf, st in zip(infos, sts))
        iters.append(np.mean([st["iterations"] for st in sts]))
        cgs.append(np.mean([st["cg_iterations"] for st in sts]))
        rcs.append(rc)
        conv += [st["status"] == 0 for st in sts]
    torch.cuda.synchronize()
    total = time.perf_counter() - t0

    # ---- roofline pass: the same frames with sampled HIP-event timing of
    # every kernel family (direct launches; one event pair per timed launch) ----
    x32 = []
    ctx.profile_enable(args.profile_stride)
    ctx.profile_read(reset=True)
    for i in range(max(min(args.steps, args.roofline_steps), min(args.steps, args.fp64_steps))):
        sts32, _ = frame(steps[args.warmup + i], fp32_opts)
        if i < args.fp64_steps:
            x32.append(([o.cpu().numpy().copy() for o in outs], [st["status"] for st in sts32]))
    prof = ctx.profile_read(reset=True)
    ctx.profile_enable(0)

    # ---- the FP64 form of the same solve on the first poses ----
    lat64, tet_iters64, err = [], 0, []
    for i in range(min(args.fp64_steps, args.steps)):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        sts, rc = frame(steps[args.warmup + i], fp64_opts)
        torch.cuda.synchronize()
        lat64.append(time.perf_counter() - ts)
        tet_iters64 += sum(inf["n_tets"] * st["iterations"] for inf, st in zip(infos, sts))
        # compared where both forms converged (a frame stopped by the Newton
        # cap is an unconverged iterate in either precision)
        for o, a, s32, st, inf in zip(outs, x32[i][0], x32[i][1], sts, infos):
            if s32 == 0 and st["status"] == 0:
                err.append(float(np.max(np.linalg.norm(a - o.cpu().numpy(), axis=1))) / inf["bbox_diag"])

    spmv_ms, spmv_timed, spmv_launches, spmv_bytes = prof["spmv"]
    achieved = spmv_bytes / (spmv_ms * 1e-3) / 1e9 if spmv_ms > 0 else None
    nchar = len(chars)
    result = {
        "metric": "tet*Newton-iter/s (frames/s at 1e-7 rel err; p50/p99 frame latency)",
        "value": tet_iters / total,
        "unit": "tet*Newton-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "frames_per_s": nchar * args.steps / total,
        "latency_ms_p50": 1e3 * float(np.percentile(lat, 50)),
        "latency_ms_p99": 1e3 * float(np.percentile(lat, 99)),
        "newton_iters_per_frame": float(np.mean(iters)),
        "cg_iters_per_frame": float(np.mean(cgs)),
        "status_codes": sorted(set(int(r) for r in rcs)),
        "converged_fraction": float(np.mean(conv)),
        "fp64": {
            "frames_per_s": nchar * len(lat64) / sum(lat64) if lat64 else None,
            "tet_newton_iter_per_s": tet_iters64 / sum(lat64) if lat64 else None,
            "max_rel_diff_fp32_vs_fp64": max(err) if err else None,
        },
        "config": {"workload": wname, "characters": nchar, "tets": m_tot,
                   "vertices": sum(i["n_vertices"] for i in infos),
                   "blocks": sum(i["n_blocks"] for i in infos),
                   "handles": [i["n_handles"] for i in infos] if nchar > 1 else infos[0]["n_handles"],
                   "precision": "fp32 pcg + fp64 refinement", "cg_tol_floor": common["cg_tol"],
                   "cg_forcing": "eisenstat-walker", "step_tol_bbox": common["step_tol"]},
        "roofline": {
            "bound": "hbm",
            "kernel": "k_cg_spmv<float>",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": counted_traffic(wname),
            "bytes_per_launch": spmv_bytes / max(spmv_timed, 1),
            "avg_launch_us": 1e3 * spmv_ms / max(spmv_timed, 1),
            "timed_launches": spmv_timed,
            "launches": spmv_launches,
        },
        "kernel_ms_sampled": {k: v[0] for k, v in prof.items()},
        "kernel_timed": {k: v[1] for k, v in prof.items()},
        "kernel_launches": {k: v[2] for k, v in prof.items()},
    }
    if not args.no_cpu_baseline:
        k = int(np.argmin([len(p["T"]) for p in probs]))
        result["cpu_baseline"] = cpu_baseline(probs[k], steps[args.warmup][k])
    print(json.dumps(result), flush=True)
    for c in chars:
        c.close()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
