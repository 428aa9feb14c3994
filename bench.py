"""Benchmark of the mixed-FEM skinning frame solve on one MI355X.

Workloads (``--workload``; seeded synthetic inputs, resident in HBM before
timing):

* ``c4`` (default): 64 procedural humanoids of 5k-200k tets (log-uniform,
  2.82M tets in all), 8-30 bone handles, neo-Hookean / co-rotated per limb
  (E log-uniform in [1e4, 1e6], nu uniform in [0.3, 0.49]), solved together
  in one batched run per step, each at a fresh random pose (joint Euler
  angles uniform in +-45 degrees) from the rest shape.  The largest
  configuration that one launch covers.
* ``c2``: one such humanoid of ~50k tets / ~10k vertices with 20 handles,
  neo-Hookean or ARAP per limb; one frame per step.
* ``c2x``: the c2 frame with the adjacent features on: rotations smoothed
  across cluster boundaries (width 5% of the bounding-box diagonal, up to 3
  handles per tet), constant loads on 200 seeded vertices, and stress and
  multiplier recovery into device memory after every frame.
* ``c1``: the 16x4x4 neo-Hookean beam (1536 tets), FP64, exactly 10 Newton
  iterations with PCG tolerance 1e-10 per step.
* ``c3``: the humanoid generator at ~500k tets / 30 handles; an animation of
  seeded sinusoidal joint angles (60 degrees, periods 2-5 s, 30 fps), each
  frame warm-started from the previous one (a step is one frame).
* ``c5``: serving: a pool of characters of 2k-300k tets and a Poisson stream
  of frame requests (fresh random pose of a uniformly chosen character)
  through the continuous-batching server; reports p50/p99 latency.  By
  default the pool is split at its median size into two classes, each served
  by its own lane (batch, context and HIP stream) with half the slots and
  half the queue (``--size-classes 1``: one lane for the whole pool).

Before timing, the autotuner picks the PCG schedule (two-kernel or
pipelined form, lanes per row, graph length, run sizing) on the first
step's frames (``--no-autotune`` keeps the default).

The timed path (c2-c5) is the FP32 + FP64-refinement form (FP32 Hessian
values and PCG; FP64 residual, energies and updates), inexact Newton
(Eisenstat-Walker forcing over a 1e-5 PCG floor), stopped at a 1e-8 * bbox
Newton step.  The FP64 form of the same solve runs beside it on the first
poses and the two results are compared.  A step uploads only handle
transforms and writes positions to device tensors.

Prints one JSON line: throughput in tet * Newton-iterations / s and frames/s,
both over the frames that converged (a frame stopped by the Newton cap is
not a solution at 1e-7 and counts nothing; the all-frames figures and the
unconverged members are reported beside them), p50/p99 frame latency, the
roofline entry of the dominant kernel (the PCG block-sparse matrix-vector
product: the least bytes such a product moves, over its average kernel
duration from HIP events carried by the sampled dispatches in a second pass
over the same kind of frames) and the FP64 CPU oracle timed on this host on
a bounded sample, on all cores and on one.

``--counter-pass N`` replaces the timed run by a fixed-work run for HBM
counters: one Newton step in which every character's FP32 PCG runs exactly N
iterations (so every SpMV dispatch covers every character), printing the
algorithmic bytes per dispatch; run it under rocprofv3 --pmc with the
autotuned schedule from ``--tune-cache``.
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


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name):
    """(problems, poses_of(step) -> list of poses, workload name, options)."""
    from workloads import (NH, COROT, humanoid, random_pose, animation_pose, beam, beam_pose,
                           character_pool)
    fp32 = dict(precision=1, cg_tol=1e-5, step_tol=1e-8, max_newton=60, cg_adaptive=1)
    if name == "c1":
        p = beam()
        return [p], (lambda i: [beam_pose(p)]), "beam_16x4x4_neohookean_twist30_stretch2", \
            dict(precision=0, cg_tol=1e-10, max_newton=10, fixed_newton=1)
    if name == "c2":
        p = humanoid(2001, target_tets=50000, n_bones=20)
        return [p], (lambda i: [random_pose(p, 2002 + i)]), "humanoid_50k_tets_20_handles_random_pose", fp32
    if name == "c2x":  # the C2 frame with the adjacent features on: rotation smoothing, loads, stress
        p = humanoid(2001, target_tets=50000, n_bones=20)
        rng = np.random.default_rng(2003)
        n = len(p["X"])
        p["force_vertex"] = rng.choice(n, 200, replace=False).astype(np.int32)
        p["force"] = rng.normal(scale=5e-4 * float(np.max(p["youngs"])) * p["bbox_diag"] ** 2 / n, size=(200, 3))
        p["smooth_width"] = 0.05 * p["bbox_diag"]
        return [p], (lambda i: [random_pose(p, 2002 + i)]), \
            "humanoid_50k_tets_20_handles_random_pose_smoothed_rotations_200_loads_stress", fp32
    if name == "c3":
        p = humanoid(3001, target_tets=500000, n_bones=30)
        return [p], (lambda i: [animation_pose(p, 3002, i)]), \
            "humanoid_500k_tets_30_handles_animation_30fps_warm_started", dict(fp32, warm_start=1)
    if name == "c4":
        ps = character_pool(64, 4001, (5000, 200000), (8, 30), (NH, COROT), workers=_workers())
        return ps, (lambda i: [random_pose(p, 41000 + 100 * i + k) for k, p in enumerate(ps)]), \
            "batch_64_humanoids_5k_200k_tets_8_30_handles", fp32
    raise SystemExit(f"unknown workload {name}")


def _workers():
    return max(1, min(16, os.cpu_count() or 1))


TRAFFIC_SUMMARIES = os.path.join(ROOT, "profiles")
TRAFFIC_SOURCES = ("paper_2408_04066_amd/csrc/kernels_cg.hip", "paper_2408_04066_amd/csrc/common.h")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counted_traffic(workload, kernel):
    """The committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary of the dominant
    kernel for this workload (profiles/hbm_traffic_*.md, copy-kernel scaled,
    taken on the fixed-work counter pass): a dict with the counted and the
    algorithmic bytes per dispatch of that run, or None when there is none or
    the kernel sources changed since it was taken."""
    import glob
    kv = {}
    for path in sorted(glob.glob(os.path.join(TRAFFIC_SUMMARIES, "hbm_traffic_*.md"))):
        fields = {}
        for line in open(path).read().splitlines():
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                fields[k.strip("`")] = v.strip().strip("`")
        if fields.get("workload") == workload and fields.get("kernel") == kernel:
            kv = fields
            kv["file"] = os.path.relpath(path, ROOT)
            break
    if kv.get("kernel_sources_sha256") != kernel_source_hash():
        return None
    try:
        return {"counted_bytes_per_dispatch": float(kv["traffic_bytes_per_launch"]),
                "algorithmic_bytes_per_dispatch": float(kv["algorithmic_bytes_per_launch"]),
                "file": kv["file"]}
    except (KeyError, ValueError):
        return None


def host_cpu():
    """The host's CPU model and how many logical CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0))}


# Newton iterations per autotuning run of a frame workload: about a
# converged frame's length (4 misjudged the asynchronous batch, whose first
# iterations are mostly long mixed-phase solves; whole frames take minutes
# on the 64-character batch, where unconverged frames run 60 iterations)
TUNE_NEWTON = 12
SERVE_STALL_S = 120.0  # a serving run that completes no request for this long is reported as stalled
CPU_BASELINE_MAX_TETS = 200_000  # largest single character whose oracle frame is a bounded sample
# Newton iterations of the oracle's sample: about ten seconds per run on a
# 16-core host (the oracle does about 4e4 tet Newton iterations per second
# there): the quartile members of a batch (about 94k tets together), or one
# character of up to 50k tets
CPU_BASELINE_ITERS_BATCH = 5
CPU_BASELINE_ITERS_ONE = 8


def ordinal(k):
    """1st, 2nd, 3rd, 4th, ..., 32nd."""
    suffix = "th" if 10 <= k % 100 <= 20 else {1: "st", 2: "nd", 3: "rd"}.get(k % 10, "th")
    return f"{k}{suffix}"


def cpu_baseline(sample, iterations, what):
    """The FP64 oracle (numpy/scipy, SuperLU) on this host over a bounded
    sample: the first `iterations` Newton iterations of each (problem, pose)
    in `sample`, first with the BLAS thread pool at its default size (every
    core the process may use), then limited to one thread."""
    import oracle
    from threadpoolctl import threadpool_info, threadpool_limits

    def run():
        secs, work = 0.0, 0
        for prob, pose in sample:
            fr = oracle.Frame(prob, pose)
            t0 = time.perf_counter()
            r = oracle.solve_frame(prob, pose, iterations=iterations, frame=fr)
            secs += time.perf_counter() - t0
            work += len(prob["T"]) * r["iterations"]
        return work / secs, secs

    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    v_all, s_all = run()
    with threadpool_limits(1):
        v_one, s_one = run()
    return {
        "value": v_all,
        "unit": "tet*Newton-iter/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"first {iterations} Newton iteration(s) of {what} ({sum(len(p['T']) for p, _ in sample)} "
                   f"tets), FP64 numpy/scipy with SuperLU solves (sequential); {s_all:.1f} s with the "
                   f"{threads}-thread BLAS pool, {s_one:.1f} s on one thread; frame set-up excluded"),
        "single_thread_value": v_one,
        "host": host_cpu(),
    }


def spmv_algorithmic_bytes(info, word, pipelined):
    """Least bytes one PCG SpMV-family dispatch moves for one system: every
    block value and column index, the row pointers and one input and one
    output vector; the pipelined kernel also fuses the PCG vector updates
    and the block-Jacobi preconditioner (twelve passes over 3n values and
    six preconditioner values per row)."""
    n, nnzb = info["n_vertices"], info["n_blocks"]
    return nnzb * (9 * word + 4) + 4 * (n + 1) + 6 * word * n + (42 * word * n if pipelined else 0)


def counter_pass(args, mfs, torch, ctxs, chars, probs, infos, steps, opts, frame, wname, tuned):
    """Fixed work for hardware counters: one Newton step in which every
    character's FP32 PCG runs exactly args.counter_pass iterations (tolerance
    0, so no system stops early and every SpMV dispatch covers all of them);
    the FP32 PCG then counts as stalled and the same step re-solves in FP64
    (a different kernel instantiation, left out of the FP32 counts)."""
    ctx = ctxs[0]
    n_it = args.counter_pass
    fixed = dict(opts, fixed_newton=1, max_newton=1, cg_tol=0.0, cg_adaptive=0, cg_max=n_it, fp32_cg_max=n_it)
    torch.cuda.synchronize()
    sts, rc = frame(steps[0], fixed)
    torch.cuda.synchronize()
    pipelined = ctx.tuning()["pcg_pipelined"] == 1
    per_dispatch = sum(spmv_algorithmic_bytes(i, 4, pipelined) for i in infos)
    kernel = "k_pcg_iter<float>" if pipelined else "k_cg_spmv<float>"
    return {"counter_pass": True, "workload": wname, "kernel": kernel, "fp32_pcg_iterations": n_it,
            "fp32_dispatches_expected": n_it, "algorithmic_bytes_per_dispatch": per_dispatch,
            "pcg_schedule": tuned or ctx.tuning(), "cg_iterations": [st["cg_iterations"] for st in sts]}


def frame_bench(args, mfs, torch):
    probs, pose_of, wname, opts = make_workload(args.workload)
    if args.opts:  # stated solve options over the workload's (mfs_solve_opts names)
        for kv in args.opts.split(","):
            k, v = kv.split("=")
            opts[k] = float(v) if ("." in v or "e" in v) else int(v)
    # size classes (batches only): each class is solved as its own batch on its
    # own context (HIP stream) from its own host thread, so a small
    # character's Newton steps do not wait for a large one's PCG runs
    K = max(1, min(args.size_classes, len(probs)))
    sizes = np.array([len(p["T"]) for p in probs])
    edges = np.quantile(sizes, np.linspace(0, 1, K + 1))[1:-1] if K > 1 else []
    cls = np.searchsorted(edges, sizes, side="right") if K > 1 else np.zeros(len(probs), dtype=int)
    ctxs = [mfs.Context(0) for _ in range(K)]
    ctx = ctxs[0]
    chars = [mfs.Character(ctxs[c], p) for c, p in zip(cls, probs)]
    members = [[i for i in range(len(chars)) if cls[i] == g] for g in range(K)]
    infos = [c.info() for c in chars]
    m_tot = sum(i["n_tets"] for i in infos)
    extended = {}
    stress_out = None
    for p, c in zip(probs, chars):
        if p.get("smooth_width"):
            H, W = c.ctx.blend_weights(p["X"], p["T"], p["seg_a"], p["seg_b"], p["seg_handle"], p["n_handles"],
                                       p["smooth_width"], 3)
            c.set_rotation_blend(H, W)
            extended["smoothing_width"] = p["smooth_width"]
            extended["blended_tet_fraction"] = float(np.mean(H[:, 1] >= 0))
        if p.get("force_vertex") is not None:
            c.set_forces(p["force_vertex"], p["force"])
            extended["loaded_vertices"] = len(p["force_vertex"])
    if extended:
        extended["stress_recovery"] = "per frame, P (m x 6) and W R P (m x 9) to device memory"
        stress_out = [(torch.empty((i["n_tets"], 6), dtype=torch.float64, device="cuda"),
                       torch.empty((i["n_tets"], 3, 3), dtype=torch.float64, device="cuda")) for i in infos]
    outs = [torch.empty((i["n_vertices"], 3), dtype=torch.float64, device="cuda") for i in infos]
    steps = [pose_of(i) for i in range(args.warmup + args.steps + args.roofline_steps + args.fp64_steps)]
    fp64_opts = dict(opts, precision=mfs.FP64)
    warm = opts.get("warm_start", 0) == mfs.WARM_PREVIOUS
    _progress(f"{wname}: {len(chars)} characters resident, {m_tot} tets")
    tuned = None
    if not args.no_autotune:
        tuned = []
        for g in range(K):
            t, tms = mfs.autotune(ctxs[g], [chars[i] for i in members[g]], [steps[0][i] for i in members[g]],
                                  newton_iterations=TUNE_NEWTON, cache_path=args.tune_cache, **opts)
            tuned.append(t)
            _progress(f"class {g}: autotuned PCG schedule {t} ({tms:.1f} ms per {TUNE_NEWTON} Newton iterations)")
        tuned = tuned[0] if K == 1 else tuned
    fixed = dict(kv.split("=") for kv in args.tuning.split(",")) if args.tuning else {}
    for c in ctxs:  # batches: each character's Newton steps on its own (1) or in lockstep (0)
        c.set_tuning(batch_async=args.batch_async, **{k: int(v) for k, v in fixed.items()})
    if fixed:
        tuned = ctxs[0].tuning() if K == 1 else [c.tuning() for c in ctxs]
    pool = None
    if K > 1:
        from concurrent.futures import ThreadPoolExecutor
        pool = ThreadPoolExecutor(max_workers=K)

    def batch(g, poses, o):
        ids = members[g]
        _, sts, rc = mfs.solve_batch(ctxs[g], [chars[i] for i in ids], [poses[i] for i in ids],
                                     outs=[outs[i] for i in ids], **o)
        return ids, sts, rc

    def frame(poses, o):
        if len(chars) == 1:
            _, st, rc = chars[0].solve(*poses[0], out=outs[0], **o)
            if stress_out is not None:
                chars[0].stress(*poses[0], outs[0], out=stress_out[0])
            return [st], rc
        if K == 1:
            _, sts, rc = mfs.solve_batch(ctx, chars, poses, outs=outs, **o)
            return sts, rc
        sts, rc = [None] * len(chars), 0
        for ids, s_, r_ in pool.map(lambda g: batch(g, poses, o), range(K)):
            for i, st in zip(ids, s_):
                sts[i] = st
            rc = max(rc, r_)
        return sts, rc

    if args.counter_pass:
        return counter_pass(args, mfs, torch, ctxs, chars, probs, infos, steps, opts, frame, wname, tuned)

    for i in range(args.warmup):
        frame(steps[i], opts)
    torch.cuda.synchronize()
    _progress("warmup done")

    # ---- timed region.  The library's profiler times every stride-th launch
    # of each kernel family with a HIP event pair recorded around it on the
    # library's stream.  Where every launch is direct (the asynchronous batch
    # form) it samples the timed launches themselves; where PCG runs replay
    # as HIP graphs (the lockstep form: a single character, or the
    # asynchronous form switched off) sampling needs direct launches, so it
    # runs on the next frames of the same kind after the timed region and the
    # timed frames keep their graphs ----
    def graphs_replayed(t, count):
        asynchronous = bool(t["batch_async"]) and not t["pcg_persistent"] and count > 1
        return bool(t["use_graphs"]) and not asynchronous
    sample_timed = not any(graphs_replayed(c.tuning(), len(members[g])) for g, c in enumerate(ctxs))
    if sample_timed:
        for c in ctxs:
            c.profile_enable(args.profile_stride)
            c.profile_read(reset=True)
    lat, rcs, per_frame = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        sts, rc = frame(steps[args.warmup + i], opts)
        lat.append(time.perf_counter() - ts)
        if lat[-1] > 5.0:  # a long step says so as it ends
            _progress(f"timed step {i}: {lat[-1]:.1f} s")
        rcs.append(rc)
        per_frame += [(i, j, st) for j, st in enumerate(sts)]
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    _progress(f"timed {args.steps} steps in {total:.2f} s")
    nxt = args.warmup + args.steps
    if not sample_timed:  # sampled pass over the next frames, direct launches
        for c in ctxs:
            c.profile_enable(args.profile_stride)
            c.profile_read(reset=True)
        for i in range(args.roofline_steps):
            frame(steps[nxt + i], opts)
        nxt += args.roofline_steps
        _progress("sampled roofline pass done")
    prof = {}
    for c in ctxs:
        for fam, v in c.profile_read(reset=True).items():
            prof[fam] = tuple(a + b for a, b in zip(prof.get(fam, (0.0, 0, 0, 0.0)), v))
        c.profile_enable(0)
    # a frame counts when it converged (status 0); a frame stopped by the
    # Newton cap (or a failed line search) is not a solution at 1e-7
    conv = [st["status"] == 0 for _, _, st in per_frame]
    tet_iters_conv = sum(infos[j]["n_tets"] * st["iterations"] for _, j, st in per_frame if st["status"] == 0)
    tet_iters_all = sum(infos[j]["n_tets"] * st["iterations"] for _, j, st in per_frame)
    unconverged = [{"step": i, "member": j, "tets": infos[j]["n_tets"], "status": st["status"],
                    "newton": st["iterations"], "mixed": st["mixed_iterations"],
                    "grad_norm": st["grad_norm"], "last_step_bbox": st["last_step"] / infos[j]["bbox_diag"]}
                   for i, j, st in per_frame if st["status"] != 0]
    conv_iters = [st["iterations"] for _, _, st in per_frame if st["status"] == 0]
    conv_mixed = [st["mixed_iterations"] for _, _, st in per_frame if st["status"] == 0]


    # ---- FP32 + refinement against the FP64 form of the same solve, both
    # from the rest shape, and both against a tight FP64 solve (Newton step
    # below 1e-12 bbox, PCG to 1e-10, up to 200 Newton iterations): the two
    # forms stop on the same step test, which a slowly converging frame can
    # pass far from its solution, so their difference alone does not say
    # which of them is off ----
    lat64, tet_iters64, err, err32, err64 = [], 0, [], [], []
    rest_opts = dict(opts, warm_start=mfs.WARM_REST)
    tight_opts = dict(fp64_opts, warm_start=mfs.WARM_REST, step_tol=1e-12, cg_tol=1e-10, cg_adaptive=0,
                      max_newton=200, fixed_newton=0)
    if opts.get("fixed_newton"):  # a fixed iteration count is the workload itself: no tight reference
        tight_opts = None
    for i in range(args.fp64_steps):
        poses = steps[nxt + i]
        s32, _ = frame(poses, rest_opts)
        x32 = [o.cpu().numpy().copy() for o in outs]
        torch.cuda.synchronize()
        ts = time.perf_counter()
        s64, _ = frame(poses, dict(fp64_opts, warm_start=mfs.WARM_REST))
        torch.cuda.synchronize()
        lat64.append(time.perf_counter() - ts)
        x64 = [o.cpu().numpy().copy() for o in outs]
        tet_iters64 += sum(inf["n_tets"] * st["iterations"] for inf, st in zip(infos, s64))
        _progress(f"fp64 step {i}: FP32 + refinement and FP64 forms done")
        if tight_opts is not None:
            # the reference runs the two-kernel PCG (the pipelined recurrences
            # can drift from the true residual near a 1e-10 tolerance), and
            # only for the frames that one of the forms solved: the others
            # are not compared, and a frame that never converges would run
            # its 200 Newton steps of 1e-10 solves for nothing
            saved = [c.tuning() for c in ctxs]
            for c in ctxs:
                c.set_tuning(pcg_pipelined=0, pcg_persistent=0)
            st_t = [{"status": -1}] * len(chars)
            xt = [None] * len(chars)
            for g in range(K):
                ids = [j for j in members[g] if s32[j]["status"] == 0 or s64[j]["status"] == 0]
                if not ids:
                    continue
                _, sts_t, _ = mfs.solve_batch(ctxs[g], [chars[j] for j in ids], [poses[j] for j in ids],
                                              outs=[outs[j] for j in ids], **tight_opts)
                for j, st in zip(ids, sts_t):
                    st_t[j] = st
                    xt[j] = outs[j].cpu().numpy().copy()
            for c, t in zip(ctxs, saved):
                c.set_tuning(**t)
            _progress(f"fp64 step {i}: tight FP64 reference done")
        # compared where the forms converged (a frame stopped by the Newton
        # cap is an unconverged iterate in either precision)
        for j, (st32, st64, inf) in enumerate(zip(s32, s64, infos)):
            d = lambda a, b: float(np.max(np.linalg.norm(a - b, axis=1))) / inf["bbox_diag"]
            if st32["status"] == 0 and st64["status"] == 0:
                err.append(d(x32[j], x64[j]))
            if tight_opts is not None and st_t[j]["status"] == 0:
                def entry(x, st):
                    return (d(x, xt[j]), {"step": i, "member": j, "newton": st["iterations"],
                                          "tight_newton": st_t[j]["iterations"],
                                          "last_step_bbox": st["last_step"] / inf["bbox_diag"],
                                          "last_cg_rel_residual": st["cg_rel_residual"],
                                          "grad_norm": st["grad_norm"], "clamped": st["clamped"]})
                if st32["status"] == 0:
                    err32.append(entry(x32[j], st32))
                if st64["status"] == 0:
                    err64.append(entry(x64[j], st64))

    spmv_ms, spmv_timed, spmv_launches, spmv_bytes = prof["spmv"]
    achieved = spmv_bytes / (spmv_ms * 1e-3) / 1e9 if spmv_ms > 0 else None
    nchar = len(chars)
    fp32 = opts["precision"] == mfs.FP32_REFINED
    big = max(range(K), key=lambda g: sum(sizes[i] for i in members[g]))  # the class with most tets
    pipelined = ctxs[big].tuning()["pcg_pipelined"] == 1
    kernel = f"{'k_pcg_iter' if pipelined else 'k_cg_spmv'}<{'float' if fp32 else 'double'}>"
    traffic = counted_traffic(wname, kernel)
    result = {
        "metric": "tet*Newton-iter/s (frames/s at 1e-7 rel err; p50/p99 frame latency)",
        "value": tet_iters_conv / total,
        "unit": "tet*Newton-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if opts["precision"] == mfs.FP32_REFINED else "f64",
        "data": "synthetic",
        "frames_per_s": sum(conv) / total,
        "counted": "converged frames only (status 0); value and frames_per_s leave out the "
                   "unconverged frames, whose GPU time stays in the wall time",
        "all_frames": {"frames_per_s": len(per_frame) / total, "tet_newton_iter_per_s": tet_iters_all / total},
        "converged_fraction": float(np.mean(conv)),
        "unconverged": unconverged,
        "latency_ms_p50": 1e3 * float(np.percentile(lat, 50)),
        "latency_ms_p99": 1e3 * float(np.percentile(lat, 99)),
        "latency_unit": "one step: one batched solve of every character" if nchar > 1 else "one frame",
        "newton_iters_per_frame": float(np.mean([st["iterations"] for _, _, st in per_frame])),
        "newton_iters_converged": {"mean": float(np.mean(conv_iters)) if conv_iters else None,
                                   "max": int(max(conv_iters)) if conv_iters else None},
        "mixed_iters_converged": {"mean": float(np.mean(conv_mixed)) if conv_mixed else None,
                                  "max": int(max(conv_mixed)) if conv_mixed else None},
        "cg_iters_per_frame": float(np.mean([st["cg_iterations"] for _, _, st in per_frame])),
        "cg_iters_per_newton": float(sum(st["cg_iterations"] for _, _, st in per_frame)
                                     / max(1, sum(st["iterations"] for _, _, st in per_frame))),
        "fp64_resolves": {"newton_steps": sum(st["fp64_resolves"] for _, _, st in per_frame),
                          "pcg_iterations": sum(st["fp64_resolve_cg_iterations"] for _, _, st in per_frame),
                          "frames": sum(st["fp64_resolves"] > 0 for _, _, st in per_frame)},
        "status_codes": sorted(set(int(r) for r in rcs)),
        "fp64": {
            "frames_per_s": nchar * len(lat64) / sum(lat64) if lat64 else None,
            "tet_newton_iter_per_s": tet_iters64 / sum(lat64) if lat64 else None,
            "max_rel_diff_fp32_vs_fp64": (max(err) if err else None) if opts["precision"] else None,
            "max_rel_err_vs_tight_fp64": {"fp32_refined": max(e[0] for e in err32) if err32 else None,
                                          "fp64": max(e[0] for e in err64) if err64 else None,
                                          "frames_compared": len(err32),
                                          "frames_above_1e-7": {"fp32_refined": sum(e[0] > 1e-7 for e in err32),
                                                                "fp64": sum(e[0] > 1e-7 for e in err64)},
                                          "above_1e-7_fp32_refined": [dict(e[1], err=e[0]) for e in err32 if e[0] > 1e-7][:10],
                                          "above_1e-7_fp64": [dict(e[1], err=e[0]) for e in err64 if e[0] > 1e-7][:10]},
        },
        "config": {"workload": wname, "characters": nchar, "tets": m_tot,
                   "vertices": sum(i["n_vertices"] for i in infos),
                   "blocks": sum(i["n_blocks"] for i in infos),
                   "handles": [i["n_handles"] for i in infos] if nchar > 1 else infos[0]["n_handles"],
                   "precision": "fp32 pcg + fp64 refinement" if opts["precision"] else "fp64",
                   "cg_tol_floor": opts["cg_tol"],
                   "cg_forcing": "eisenstat-walker" if opts.get("cg_adaptive") else "fixed",
                   "step_tol_bbox": opts.get("step_tol"),
                   "newton": "fixed 10" if opts.get("fixed_newton") else f"max {opts['max_newton']}",
                   "warm_start": "previous frame" if warm else "rest",
                   "pcg_schedule": tuned or ctx.tuning(),
                   **({"solve_option_overrides": args.opts} if args.opts else {}),
                   **({"size_classes": K, "class_tet_edges": [float(e) for e in edges],
                       "class_sizes": [len(m_) for m_ in members]} if K > 1 else {}),
                   **({"extended": extended} if extended else {})},
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "sampled_over": (f"every {ordinal(args.profile_stride)} launch of the timed steps" if sample_timed else
                             f"every {ordinal(args.profile_stride)} launch of {args.roofline_steps} frames after the timed steps, "
                             f"launched directly (the timed steps replay their PCG runs as graphs)"),
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            # counted HBM bytes per launch: the counted / algorithmic ratio of
            # the committed counter pass times this run's algorithmic bytes
            # per timed launch (the launch sets differ: the counter pass keeps
            # every system in every dispatch)
            "traffic": (traffic["counted_bytes_per_dispatch"] / traffic["algorithmic_bytes_per_dispatch"]
                        * spmv_bytes / max(spmv_timed, 1)) if traffic else None,
            "traffic_counter_pass": traffic,
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
        if nchar >= 4:  # the members at the three quartiles of size, first Newton iteration each
            order = list(np.argsort(sizes, kind="stable"))
            pick = [int(order[(q * nchar) // 4]) for q in (1, 2, 3)]
            sample = [(probs[k], steps[args.warmup][k]) for k in pick]
            what = (f"the frames of the members at the three quartiles of size ({', '.join(str(sizes[k]) for k in pick)} "
                    f"tets) of the first timed step")
            result["cpu_baseline"] = cpu_baseline(sample, CPU_BASELINE_ITERS_BATCH, what)
        elif sizes[0] <= CPU_BASELINE_MAX_TETS:
            sample = [(probs[0], steps[args.warmup][0])]
            result["cpu_baseline"] = cpu_baseline(sample, CPU_BASELINE_ITERS_ONE, f"one frame of the {sizes[0]}-tet character")
        else:  # the oracle's sparse LU of one Newton step alone runs for minutes here
            result["cpu_baseline"] = None
            result["cpu_baseline_skipped"] = (f"the {sizes[0]}-tet character is above {CPU_BASELINE_MAX_TETS} tets, "
                                              f"where one oracle Newton step (sparse LU) exceeds a bounded sample")
        _progress("oracle baseline done")
    for c in chars:
        c.close()
    if pool is not None:
        pool.shutdown()
    for c in ctxs:
        c.close()
    return result


def serve_bench(args, mfs, torch):
    """Poisson stream of frame requests through the serving loop.  With
    ``--size-classes K`` > 1 the pool is split by tet count into K classes,
    each served by its own lane of one server (a batch on its own context and
    HIP stream, with the PCG schedule autotuned for that class), so the small
    characters' frames do not wait for the large ones' PCG runs and the
    streams overlap on the GPU; the slots are divided between the classes."""
    from workloads import NH, COROT, ARAP, character_pool, random_pose
    probs = character_pool(args.pool, 5001, (2000, 300000), (8, 30), (NH, COROT, ARAP),
                           workers=_workers())
    K = max(1, args.size_classes)
    sizes = np.array([len(p["T"]) for p in probs])
    edges = np.quantile(sizes, np.linspace(0, 1, K + 1))[1:-1] if K > 1 else []
    cls = np.searchsorted(edges, sizes, side="right") if K > 1 else np.zeros(len(probs), dtype=int)
    ctx = mfs.Context(0)
    chars = [mfs.Character(ctx, p) for p in probs]
    infos = [c.info() for c in chars]
    lane_max = [int(sizes[cls == g].max()) for g in range(K - 1)]  # lane g takes tets <= lane_max[g]
    slots = [max(1, args.slots // K)] * K
    budgets = []
    for g in range(K):
        ws = sorted((chars[k].footprint()[1] for k in range(len(chars)) if cls[k] == g), reverse=True)
        budgets.append(2 * sum(ws[:slots[g]]))
    for c in chars:
        c.release_workspace()
    opts = dict(precision=1, cg_tol=1e-5, step_tol=1e-8, max_newton=60, cg_adaptive=1)
    rng = np.random.default_rng(5002)
    n_req = int(args.rate * args.duration)
    arrivals = np.cumsum(rng.exponential(1.0 / args.rate, size=n_req))
    who = rng.integers(0, len(chars), size=n_req)
    poses = [random_pose(probs[k], 50000 + j) for j, k in enumerate(who)]
    tuned = []
    if not args.no_autotune:  # schedule for a batch like each served mix: a sample of the class
        for g in range(K):
            members = [k for k in range(len(chars)) if cls[k] == g]
            sample = members[::max(1, len(members) // slots[g])][:slots[g]]
            for k in sample:
                chars[k].solve(*random_pose(probs[k], 1), **opts)  # re-creates the released workspace
            t, tms = mfs.autotune(ctx, [chars[k] for k in sample], [random_pose(probs[k], 1) for k in sample],
                                  newton_iterations=4, cache_path=args.tune_cache, **opts)
            for k in sample:
                chars[k].release_workspace()
            tuned.append(t)
            _progress(f"class {g}: autotuned PCG schedule {t} ({tms:.1f} ms per 4 Newton iterations)")
    queue = max(1, args.queue // K)  # the same total queue capacity however the pool is split
    srv = mfs.Server(ctx, slots=slots[0], queue_capacity=queue, workspace_budget_bytes=max(budgets),
                     lane_max_tets=lane_max, **opts)
    fixed = {k: int(v) for k, v in (kv.split("=") for kv in args.tuning.split(","))} if args.tuning else {}
    if fixed:  # stated schedule fields over the autotuned ones (or the defaults)
        tuned = [dict(t, **fixed) for t in tuned] if tuned else [dict(ctx.tuning(), **fixed) for _ in range(K)]
    for g, t in enumerate(tuned):
        srv.set_lane_tuning(g, **t)
    for j in range(min(args.warmup, n_req)):  # warm the kernels and graphs
        srv.wait(srv.submit(chars[who[j]], *poses[j]))
    info0 = srv.info()
    tickets, rejected = [], 0
    t0 = time.perf_counter()
    _progress(f"pool of {len(chars)} characters resident in {K} size class(es); streaming {n_req} requests")
    for j in range(n_req):
        if j % 1000 == 0 and j:
            _progress(f"submitted {j} requests, {srv.info()['completed']} completed")
        delay = arrivals[j] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        k = who[j]
        try:
            tickets.append((k, srv.submit(chars[k], *poses[j])))
        except mfs.MfsError as e:
            if e.code != -6:
                raise
            rejected += 1
    lat, tet_iters, tet_iters_all, done_t, conv, first_submit = [], 0, 0, [], [], None
    # drain: poll the tickets in order, reporting progress; a server that
    # completes nothing for SERVE_STALL_S seconds ends the run with an error
    last_done, last_change = srv.info()["completed"], time.perf_counter()
    for n_done, (k, tk) in enumerate(tickets):
        while True:
            res = srv.poll(tk)
            if res is not None:
                break
            time.sleep(0.01)
            c = srv.info()["completed"]
            if c != last_done:
                last_done, last_change = c, time.perf_counter()
            elif time.perf_counter() - last_change > SERVE_STALL_S:
                raise RuntimeError(f"serving stalled: no request completed in {SERVE_STALL_S} s "
                                   f"({c} completed, {len(tickets)} accepted)")
        if n_done % 1000 == 0 and n_done:
            _progress(f"collected {n_done} of {len(tickets)} results")
        _, st, tm, _ = res
        lat.append(tm["done_s"] - tm["submit_s"])
        first_submit = tm["submit_s"] if first_submit is None else min(first_submit, tm["submit_s"])
        done_t.append(tm["done_s"])
        tet_iters_all += infos[k]["n_tets"] * st["iterations"]
        if st["status"] == 0:  # only converged frames count
            tet_iters += infos[k]["n_tets"] * st["iterations"]
        conv.append(st["status"] == 0)
    info = srv.info()
    srv.close()
    span = max(done_t) - first_submit
    steps = info["steps"] - info0["steps"]
    slot_steps = info["slot_steps"] - info0["slot_steps"]
    result = {
        "metric": "tet*Newton-iter/s (frames/s at 1e-7 rel err; p50/p99 frame latency)",
        "value": tet_iters / span,
        "unit": "tet*Newton-iter/s",
        "n_gpus": 1,
        "steps": len(tickets),
        "warmup": args.warmup,
        "ms_per_step": 1e3 * span / max(len(tickets), 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "frames_per_s": sum(conv) / span,
        "counted": "converged frames only (status 0); the latencies cover every served request",
        "served_per_s": len(tickets) / span,
        "all_frames": {"frames_per_s": len(tickets) / span, "tet_newton_iter_per_s": tet_iters_all / span},
        "latency_ms_p50": 1e3 * float(np.percentile(lat, 50)),
        "latency_ms_p99": 1e3 * float(np.percentile(lat, 99)),
        "offered_rate_per_s": args.rate,
        "requests": n_req,
        "served": len(tickets),
        "rejected_queue_full": rejected,
        "rejected_fraction": rejected / max(n_req, 1),
        "converged_fraction": float(np.mean(conv)),
        "mean_batch_width": slot_steps / max(steps, 1),
        "arena_peak_bytes": info["arena_peak"],
        "config": {"workload": f"serving_pool_{args.pool}_humanoids_2k_300k_tets_poisson_{args.rate:g}_per_s",
                   "characters": len(chars), "tets": int(sizes.sum()),
                   "size_classes": K, "lane_max_tets": lane_max,
                   "slots_per_lane": slots[0], "queue_capacity_per_lane": queue, "arena_bytes_per_lane": max(budgets),
                   "duration_s": args.duration, "precision": "fp32 pcg + fp64 refinement",
                   "pcg_schedule": tuned or [ctx.tuning()]},
    }
    for c in chars:
        c.close()
    ctx.close()
    return result

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--counter-pass", type=int, default=0,
                    help="fixed-work run for HBM counters: one Newton step with exactly this many FP32 PCG "
                         "iterations per character (no timed run)")
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--profile-stride", type=int, default=32,
                    help="time every N-th launch of each kernel family (0: off); on the 64-character batch "
                         "a stride of 8 slowed the timed batches by 6%%, 32 by under 1%%")
    ap.add_argument("--roofline-steps", type=int, default=2,
                    help="frames of the sampled pass that follows the timed region where PCG runs replay "
                         "as graphs (the asynchronous batch form samples its timed launches instead)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default PCG schedule")
    ap.add_argument("--tuning", default="",
                    help="PCG schedule fields set after autotuning, KEY=VALUE,... (mfs_tuning names), e.g. "
                         "with --no-autotune to run a stated schedule")
    ap.add_argument("--opts", default="",
                    help="solve options over the workload's, KEY=VALUE,... (mfs_solve_opts names, e.g. "
                         "fp32_cg_max=4000)")
    ap.add_argument("--batch-async", type=int, default=1, choices=(0, 1),
                    help="batches with the two-kernel PCG: each character runs its own Newton steps (1) or "
                         "all run the same Newton iteration (0)")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file: reuse a choice made for this GPU and size class")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB (the reference kernel "
                         "that scales HBM byte counters)")
    ap.add_argument("--pool", type=int, default=200, help="c5: resident characters")
    ap.add_argument("--rate", type=float, default=300.0, help="c5: Poisson arrivals per second")
    ap.add_argument("--duration", type=float, default=60.0, help="c5: seconds of arrivals")
    ap.add_argument("--slots", type=int, default=16, help="c5: requests in flight at once")
    ap.add_argument("--queue", type=int, default=512, help="c5: queued requests before rejection")
    ap.add_argument("--size-classes", type=int, default=None,
                    help="c4, c5: batches / servers by tet-count class, each on its own context and stream "
                         "(default: 3 for c5, 1 otherwise)")
    args = ap.parse_args()
    if args.size_classes is None:
        args.size_classes = 3 if args.workload == "c5" else 1
    if args.gpus != 1:
        print("bench.py measures one GPU: each frame solve runs on a single device and "
              "multi-GPU sharding is not implemented", file=sys.stderr)
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

    result = serve_bench(args, mfs, torch) if args.workload == "c5" else frame_bench(args, mfs, torch)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
