"""Python binding of ``libmfs`` (mixed-FEM skinning solve on MI355X, gfx950).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels behind the C ABI declared in ``include/mfs.h``.  PyTorch is used, when
present, only for device buffers and the current HIP stream.  The library is
loaded on first use; a missing build raises ``MfsUnavailable`` (there is no
fallback implementation).
"""

import ctypes
import os

import numpy as np

__all__ = ["MfsError", "MfsUnavailable", "Context", "Character", "SolveOpts", "SolveStats",
           "solve_batch", "autotune", "mesh_footprint", "Server", "lib", "EXPORTED", "ARAP", "COROT", "NEOHOOKEAN", "FP64", "FP32_REFINED",
           "MEM_HOST", "MEM_DEVICE", "WARM_REST", "WARM_PREVIOUS"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmfs.so")

OK, W_NOT_CONVERGED = 0, 1
ARAP, COROT, NEOHOOKEAN = 0, 1, 2
FP64, FP32_REFINED = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
WARM_REST, WARM_PREVIOUS = 0, 1

# Every function the header declares.
EXPORTED = ("mfs_default_opts", "mfs_status_string", "mfs_last_error", "mfs_context_create",
            "mfs_context_destroy", "mfs_character_create", "mfs_character_destroy",
            "mfs_character_footprint", "mfs_cluster_by_segments", "mfs_solve_frame",
            "mfs_solve_batch", "mfs_evaluate", "mfs_polar", "mfs_blend_weights",
            "mfs_character_set_rotation_blend", "mfs_character_get_info",
            "mfs_profile_enable", "mfs_profile_read", "mfs_context_get_tuning",
            "mfs_context_set_tuning", "mfs_character_release_workspace", "mfs_default_server_opts",
            "mfs_server_create", "mfs_server_destroy", "mfs_server_submit", "mfs_server_poll",
            "mfs_server_set_lane_tuning",
            "mfs_server_wait", "mfs_server_get_info", "mfs_autotune", "mfs_character_set_forces",
            "mfs_stress", "mfs_character_get_footprint", "mfs_evaluate_noalloc")

KERNEL_FAMILIES = ("warm_start", "element", "assemble", "spmv", "cg_update", "linesearch", "update",
                   "other")


class MfsUnavailable(ImportError):
    pass


class MfsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mfs error {code}: {msg}")
        self.code = code


c_i32, c_i64, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_vertices", c_i64), ("rest_positions", c_vp), ("n_tets", c_i64), ("tets", c_vp),
                ("material_model", c_vp), ("youngs", c_vp), ("poisson", c_vp),
                ("n_handles", c_i32), ("tet_cluster", c_vp), ("n_pins", c_i64),
                ("pin_vertex", c_vp), ("pin_handle", c_vp), ("pin_stiffness", c_dbl),
                ("memory_space", c_i32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("precision", c_i32), ("max_newton", c_i32), ("fixed_newton", c_i32),
                ("step_tol", c_dbl), ("cg_tol", c_dbl), ("cg_max", c_i32), ("warm_start", c_i32),
                ("output_memory", c_i32), ("cg_adaptive", c_i32), ("load_bisections", c_i32),
                ("fp32_cg_max", c_i32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("status", c_i32), ("iterations", c_i32), ("mixed_iterations", c_i32),
                ("cg_iterations", c_i32), ("halvings", c_i32), ("clamped", c_i32),
                ("fp64_routed", c_i32), ("cg_not_converged", c_i32), ("energy", c_dbl),
                ("grad_norm", c_dbl), ("last_step", c_dbl), ("cg_rel_residual", c_dbl),
                ("fp64_resolves", c_i32), ("fp64_resolve_cg_iterations", c_i32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class CharacterInfo(ctypes.Structure):
    _fields_ = [("n_vertices", c_i64), ("n_tets", c_i64), ("n_blocks", c_i64), ("n_pins", c_i64),
                ("n_handles", c_i32), ("reserved", c_i32), ("bbox_diag", c_dbl), ("mean_edge", c_dbl)]


class Tuning(ctypes.Structure):
    _fields_ = [("pcg_lanes_per_row", c_i32), ("use_graphs", c_i32), ("graph_iterations", c_i32),
                ("first_check", c_i32), ("min_run", c_i32), ("max_run", c_i32), ("pcg_pipelined", c_i32),
                ("allread_max_tiles", c_i32), ("pcg_persistent", c_i32), ("batch_async", c_i32)]


class Profile(ctypes.Structure):
    _fields_ = [("gpu_ms", c_dbl * 8), ("timed", c_i64 * 8), ("launches", c_i64 * 8),
                ("bytes", c_dbl * 8)]


_lib = None


class ServerOpts(ctypes.Structure):
    _fields_ = [("slots", c_i32), ("queue_capacity", c_i32), ("workspace_budget_bytes", ctypes.c_uint64),
                ("solve", SolveOpts), ("lanes", c_i32), ("reserved", c_i32), ("lane_max_tets", c_i64 * 3)]


class RequestTimes(ctypes.Structure):
    _fields_ = [("submit_s", c_dbl), ("admit_s", c_dbl), ("done_s", c_dbl)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("submitted", c_i64), ("completed", c_i64), ("steps", c_i64), ("queued", c_i32),
                ("running", c_i32), ("arena_bytes", ctypes.c_uint64), ("arena_in_use", ctypes.c_uint64),
                ("arena_peak", ctypes.c_uint64), ("slot_steps", c_dbl)]


def lib():
    """The loaded library (loads it on first call)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise MfsUnavailable(f"{LIB_PATH} is not built; run `python -m paper_2408_04066_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    sig = {
        "mfs_default_opts": (None, [P(SolveOpts)]),
        "mfs_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "mfs_last_error": (ctypes.c_char_p, []),
        "mfs_context_create": (ctypes.c_int, [ctypes.c_int, c_vp, P(c_vp)]),
        "mfs_context_destroy": (ctypes.c_int, [c_vp]),
        "mfs_character_create": (ctypes.c_int, [c_vp, P(MeshDesc), P(c_vp)]),
        "mfs_character_destroy": (ctypes.c_int, [c_vp]),
        "mfs_character_footprint": (ctypes.c_int, [P(MeshDesc), P(ctypes.c_size_t), P(ctypes.c_size_t)]),
        "mfs_character_get_footprint": (ctypes.c_int, [c_vp, P(ctypes.c_size_t), P(ctypes.c_size_t)]),
        "mfs_cluster_by_segments": (ctypes.c_int, [c_vp, c_vp, c_i64, c_vp, c_i64, c_i32, c_vp, c_vp,
                                                   c_vp, c_vp, c_i32]),
        "mfs_solve_frame": (ctypes.c_int, [c_vp, c_vp, c_vp, P(SolveOpts), c_vp, P(SolveStats)]),
        "mfs_solve_batch": (ctypes.c_int, [c_vp, c_i32, c_vp, c_vp, c_vp, P(SolveOpts), c_vp,
                                           P(SolveStats)]),
        "mfs_evaluate": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp]),
        "mfs_evaluate_noalloc": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp]),
        "mfs_polar": (ctypes.c_int, [c_vp, c_vp, c_i64, c_i32, c_vp, c_vp, c_vp, c_vp, c_i32]),
        "mfs_blend_weights": (ctypes.c_int, [c_vp, c_vp, c_i64, c_vp, c_i64, c_i32, c_vp, c_vp, c_vp, c_i32,
                                             c_dbl, c_i32, c_vp, c_vp, c_i32]),
        "mfs_character_set_rotation_blend": (ctypes.c_int, [c_vp, c_i32, c_vp, c_vp, c_i32]),
        "mfs_character_get_info": (ctypes.c_int, [c_vp, P(CharacterInfo)]),
        "mfs_profile_enable": (ctypes.c_int, [c_vp, c_i32]),
        "mfs_profile_read": (ctypes.c_int, [c_vp, P(Profile), c_i32]),
        "mfs_context_get_tuning": (ctypes.c_int, [c_vp, P(Tuning)]),
        "mfs_context_set_tuning": (ctypes.c_int, [c_vp, P(Tuning)]),
        "mfs_character_release_workspace": (ctypes.c_int, [c_vp]),
        "mfs_character_set_forces": (ctypes.c_int, [c_vp, c_vp, c_vp, c_i64, c_i32]),
        "mfs_stress": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, c_i32, c_vp, c_vp]),
        "mfs_default_server_opts": (None, [P(ServerOpts)]),
        "mfs_server_create": (ctypes.c_int, [c_vp, P(ServerOpts), P(c_vp)]),
        "mfs_server_destroy": (ctypes.c_int, [c_vp]),
        "mfs_server_submit": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, P(ctypes.c_uint64)]),
        "mfs_server_poll": (ctypes.c_int, [c_vp, ctypes.c_uint64, c_vp, P(SolveStats), P(RequestTimes),
                                           P(c_i32)]),
        "mfs_server_wait": (ctypes.c_int, [c_vp, ctypes.c_uint64, c_vp, P(SolveStats), P(RequestTimes)]),
        "mfs_server_get_info": (ctypes.c_int, [c_vp, P(ServerInfo)]),
        "mfs_server_set_lane_tuning": (ctypes.c_int, [c_vp, c_i32, P(Tuning)]),
        "mfs_autotune": (ctypes.c_int, [c_vp, c_i32, c_vp, c_vp, c_vp, P(SolveOpts), c_i32, ctypes.c_char_p,
                                        c_i32, P(Tuning), P(c_dbl)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc, allow_warning=True):
    if rc < 0 or (rc > 0 and not allow_warning):
        raise MfsError(rc, lib().mfs_last_error().decode())
    return rc


def _host(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()   # torch tensor on the device


def default_opts(**kw):
    o = SolveOpts()
    lib().mfs_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown solve option {k}")
        setattr(o, k, v)
    return o


class Context:
    """One GPU and one HIP stream.  ``stream``: "current" (torch's current
    stream), None (a stream owned by the context) or a raw hipStream_t."""

    def __init__(self, device=0, stream="current"):
        raw = None
        if stream == "current":
            import torch
            raw = torch.cuda.current_stream(device).cuda_stream
        elif stream is not None:
            raw = int(stream)
        h = c_vp()
        _check(lib().mfs_context_create(device, raw, ctypes.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib().mfs_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tuning(self):
        t = Tuning()
        _check(lib().mfs_context_get_tuning(self.handle, ctypes.byref(t)))
        return {name: getattr(t, name) for name, _ in t._fields_}

    def set_tuning(self, **kw):
        t = Tuning()
        _check(lib().mfs_context_get_tuning(self.handle, ctypes.byref(t)))
        for k, v in kw.items():
            if not hasattr(t, k):
                raise TypeError(f"unknown tuning field {k}")
            setattr(t, k, int(v))
        _check(lib().mfs_context_set_tuning(self.handle, ctypes.byref(t)))

    def profile_enable(self, stride=1):
        """Time every `stride`-th launch of each kernel family with HIP events
        (0 = off)."""
        _check(lib().mfs_profile_enable(self.handle, stride))

    def profile_read(self, reset=False):
        """{family: (gpu_ms, timed launches, all launches, algorithmic bytes of
        the timed launches)}."""
        p = Profile()
        _check(lib().mfs_profile_read(self.handle, ctypes.byref(p), int(reset)))
        return {f: (p.gpu_ms[i], p.timed[i], p.launches[i], p.bytes[i])
                for i, f in enumerate(KERNEL_FAMILIES)}

    def cluster_by_segments(self, X, T, seg_a, seg_b, seg_handle):
        X = _host(X, np.float64)
        T = _host(T, np.int32)
        sa, sb = _host(seg_a, np.float64), _host(seg_b, np.float64)
        sh = _host(seg_handle, np.int32)
        out = np.empty(T.shape[0], dtype=np.int32)
        _check(lib().mfs_cluster_by_segments(self.handle, _ptr(X), X.shape[0], _ptr(T), T.shape[0],
                                             len(sh), _ptr(sa), _ptr(sb), _ptr(sh), _ptr(out), MEM_HOST))
        return out

    def blend_weights(self, X, T, seg_a, seg_b, seg_handle, n_handles, width, kmax=3):
        """Rotation-smoothing weights (``mfs_blend_weights``): (handles, weights),
        each (m, kmax)."""
        X = _host(X, np.float64)
        T = _host(T, np.int32)
        sa, sb = _host(seg_a, np.float64), _host(seg_b, np.float64)
        sh = _host(seg_handle, np.int32)
        m = T.shape[0]
        H = np.empty((m, kmax), dtype=np.int32)
        W = np.empty((m, kmax))
        _check(lib().mfs_blend_weights(self.handle, _ptr(X), X.shape[0], _ptr(T), m, len(sh), _ptr(sa), _ptr(sb),
                                       _ptr(sh), int(n_handles), float(width), int(kmax), _ptr(H), _ptr(W),
                                       MEM_HOST))
        return H, W

    def polar(self, F, precision=FP64):
        F = _host(F, np.float64).reshape(-1, 9)
        c = F.shape[0]
        U = np.empty((c, 9))
        P = np.empty((c, 6))
        s = np.empty(c)
        routed = np.empty(c, dtype=np.uint8)
        _check(lib().mfs_polar(self.handle, _ptr(F), c, precision, _ptr(U), _ptr(P), _ptr(s),
                               _ptr(routed), MEM_HOST))
        return U.reshape(c, 3, 3), P, s, routed


def mesh_footprint(prob):
    """(resident bytes, workspace bytes) that a Character of ``prob`` would
    allocate, computed on the host before any upload
    (``mfs_character_footprint``)."""
    X = _host(prob["X"], np.float64)
    T = _host(prob["T"], np.int32)
    d = MeshDesc()
    d.n_vertices, d.n_tets, d.tets = X.shape[0], T.shape[0], _ptr(T)
    d.n_pins = len(prob["pin_vertex"])
    d.memory_space = MEM_HOST
    r, w = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().mfs_character_footprint(ctypes.byref(d), ctypes.byref(r), ctypes.byref(w)))
    return r.value, w.value


def autotune(ctx, chars, poses, newton_iterations=4, cache_path=None, force=False, **opts):
    """Pick and apply the PCG launch schedule for a batch like ``chars``
    (``mfs_autotune``).  Returns (tuning dict, best milliseconds)."""
    k = len(chars)
    Rs, ts = zip(*[ch._pose(R, t) for ch, (R, t) in zip(chars, poses)])
    arr = lambda vals: (c_vp * k)(*vals)
    o = default_opts(**opts)
    best, ms = Tuning(), c_dbl()
    path = cache_path.encode() if cache_path else None
    _check(lib().mfs_autotune(ctx.handle, k, arr([c.handle.value for c in chars]), arr([_ptr(R) for R in Rs]),
                              arr([_ptr(t) for t in ts]), ctypes.byref(o), newton_iterations, path,
                              1 if force else 0, ctypes.byref(best), ctypes.byref(ms)))
    return {name: getattr(best, name) for name, _ in best._fields_}, ms.value


class Character:
    """A character resident on the context's GPU.

    ``prob`` holds the arrays of a problem: ``X`` (n, 3), ``T`` (m, 4),
    ``model``, ``youngs``, ``poisson`` (m,), ``n_handles``, ``pin_vertex``,
    ``pin_handle``, ``pin_stiffness`` and either ``cluster`` (m,) or the bone
    segments ``seg_a``, ``seg_b``, ``seg_handle`` (clusters are then computed
    by the library's nearest-segment kernel).
    """

    def __init__(self, ctx, prob, cluster=None):
        self.ctx = ctx
        X = _host(prob["X"], np.float64)
        T = _host(prob["T"], np.int32)
        if cluster is None:
            cluster = prob.get("cluster")
        if cluster is None:
            cluster = ctx.cluster_by_segments(X, T, prob["seg_a"], prob["seg_b"], prob["seg_handle"])
        self.cluster = _host(cluster, np.int32)
        keep = [X, T, _host(prob["model"], np.int32), _host(prob["youngs"], np.float64),
                _host(prob["poisson"], np.float64), self.cluster,
                _host(prob["pin_vertex"], np.int32), _host(prob["pin_handle"], np.int32)]
        d = MeshDesc()
        d.n_vertices, d.rest_positions = X.shape[0], _ptr(keep[0])
        d.n_tets, d.tets = T.shape[0], _ptr(keep[1])
        d.material_model, d.youngs, d.poisson = _ptr(keep[2]), _ptr(keep[3]), _ptr(keep[4])
        d.n_handles = int(prob["n_handles"])
        d.tet_cluster = _ptr(keep[5])
        d.n_pins, d.pin_vertex, d.pin_handle = len(keep[6]), _ptr(keep[6]), _ptr(keep[7])
        d.pin_stiffness = float(prob["pin_stiffness"])
        d.memory_space = MEM_HOST
        h = c_vp()
        _check(lib().mfs_character_create(ctx.handle, ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        self.n, self.m, self.n_handles = X.shape[0], T.shape[0], d.n_handles
        if prob.get("blend_handles") is not None:
            self.set_rotation_blend(prob["blend_handles"], prob["blend_weights"])

    def close(self):
        if getattr(self, "handle", None):
            lib().mfs_character_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        i = CharacterInfo()
        _check(lib().mfs_character_get_info(self.handle, ctypes.byref(i)))
        return {name: getattr(i, name) for name, _ in i._fields_ if name != "reserved"}

    def footprint(self):
        """(resident bytes, workspace bytes) as allocated."""
        r, w = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().mfs_character_get_footprint(self.handle, ctypes.byref(r), ctypes.byref(w)))
        return r.value, w.value

    def set_rotation_blend(self, handles=None, weights=None):
        """Smoothed tet rotations (m x kmax handles and weights, caller order)
        for later solves; None returns to cluster rotations."""
        if handles is None:
            _check(lib().mfs_character_set_rotation_blend(self.handle, 0, None, None, MEM_HOST))
            return
        H = _host(handles, np.int32)
        W = _host(weights, np.float64)
        if H.shape != W.shape or H.ndim != 2 or H.shape[0] != self.m:
            raise ValueError("handles and weights must both be (m, kmax)")
        _check(lib().mfs_character_set_rotation_blend(self.handle, H.shape[1], _ptr(H), _ptr(W), MEM_HOST))

    def set_forces(self, vertices=None, forces=None):
        """External vertex forces (count x 3) for later solves; None clears."""
        if vertices is None or len(vertices) == 0:
            _check(lib().mfs_character_set_forces(self.handle, None, None, 0, MEM_HOST))
            return
        v = _host(vertices, np.int32).reshape(-1)
        f = _host(forces, np.float64).reshape(len(v), 3)
        _check(lib().mfs_character_set_forces(self.handle, _ptr(v), _ptr(f), len(v), MEM_HOST))

    def release_workspace(self):
        """Free the solve workspace; a server lends one per admitted frame."""
        _check(lib().mfs_character_release_workspace(self.handle))

    def _pose(self, R, t):
        R = _host(R, np.float64).reshape(self.n_handles, 9)
        t = _host(t, np.float64).reshape(self.n_handles, 3)
        return R, t

    def solve(self, R, t, out=None, **opts):
        """Solve one frame.  Returns (x, stats, rc); x is (n, 3) float64 in
        ``out`` (a numpy array, or a CUDA torch tensor for device output) or
        a new numpy array."""
        R, t = self._pose(R, t)
        if out is None:
            out = np.empty((self.n, 3))
        o = default_opts(**opts)
        o.output_memory = MEM_HOST if isinstance(out, np.ndarray) else MEM_DEVICE
        st = SolveStats()
        rc = _check(lib().mfs_solve_frame(self.handle, _ptr(R), _ptr(t), ctypes.byref(o), _ptr(out),
                                          ctypes.byref(st)))
        return out, st.as_dict(), rc

    def stress(self, R, t, x, out=None):
        """Per-tet stress P (m, 6) and world multiplier W R P (m, 3, 3) at x.
        With x a CUDA torch tensor (n, 3) float64 and ``out`` = (P, L) CUDA
        tensors of those shapes, everything stays in device memory."""
        R, t = self._pose(R, t)
        if out is not None:
            P, L = out
            _check(lib().mfs_stress(self.handle, _ptr(R), _ptr(t), _ptr(x), MEM_DEVICE, _ptr(P), _ptr(L)))
            return P, L
        x = _host(x, np.float64).reshape(self.n, 3)
        P = np.empty((self.m, 6))
        L = np.empty((self.m, 3, 3))
        _check(lib().mfs_stress(self.handle, _ptr(R), _ptr(t), _ptr(x), MEM_HOST, _ptr(P), _ptr(L)))
        return P, L

    def evaluate(self, R, t, x, v=None, want_grad=True, want_stretch=True, noalloc=False):
        """Energy, gradient, stretches and K v at positions x (host arrays);
        ``noalloc`` calls the allocation-free entry point."""
        fn = lib().mfs_evaluate_noalloc if noalloc else lib().mfs_evaluate
        R, t = self._pose(R, t)
        x = _host(x, np.float64).reshape(self.n, 3)
        E = ctypes.c_double()
        g = np.empty((self.n, 3)) if want_grad else None
        s = np.empty((self.m, 6)) if want_stretch else None
        vv = _host(v, np.float64).reshape(self.n, 3) if v is not None else None
        kv = np.empty((self.n, 3)) if v is not None else None
        _check(fn(self.handle, _ptr(R), _ptr(t), _ptr(x), _ptr(vv), MEM_HOST, ctypes.byref(E), _ptr(g), _ptr(s),
                  _ptr(kv)))
        return {"energy": E.value, "grad": g, "stretch": s, "Kv": kv}


def solve_batch(ctx, chars, poses, outs=None, **opts):
    """Solve one frame for each character in one batched run.  ``poses`` is
    a list of (R, t); returns (list of x, list of stats dicts, rc)."""
    k = len(chars)
    Rs, ts = [], []
    for ch, (R, t) in zip(chars, poses):
        R, t = ch._pose(R, t)
        Rs.append(R)
        ts.append(t)
    if outs is None:
        outs = [np.empty((ch.n, 3)) for ch in chars]
    o = default_opts(**opts)
    o.output_memory = MEM_HOST if isinstance(outs[0], np.ndarray) else MEM_DEVICE
    arr = lambda vals: (c_vp * k)(*vals)
    st = (SolveStats * k)()
    rc = _check(lib().mfs_solve_batch(ctx.handle, k, arr([c.handle.value for c in chars]),
                                      arr([_ptr(R) for R in Rs]), arr([_ptr(t) for t in ts]),
                                      ctypes.byref(o), arr([_ptr(x) for x in outs]), st))
    return outs, [s.as_dict() for s in st], rc


class Server:
    """Request loop with continuous batching (``mfs_server_*``).

    While the server exists its worker thread owns the context: use the
    context and its characters only through the server.  ``submit`` returns
    a ticket at once; ``poll`` returns None until the frame is done, then
    (x, stats, times, rc); ``wait`` blocks for it.  ``times`` holds submit,
    admit and completion times in seconds on the server's clock.

    ``lane_max_tets`` (a list of up to three increasing tet counts) splits the
    server into ``len(lane_max_tets) + 1`` lanes, each a batch of its own on a
    stream of its own: a character goes to the first lane whose bound is at
    least its tet count, else to the last.  ``slots``, ``queue_capacity`` and
    ``workspace_budget_bytes`` hold per lane."""

    def __init__(self, ctx, slots=16, queue_capacity=4096, workspace_budget_bytes=0, lane_max_tets=(),
                 **solve_opts):
        o = ServerOpts()
        lib().mfs_default_server_opts(ctypes.byref(o))
        o.slots, o.queue_capacity = slots, queue_capacity
        bounds = [int(v) for v in lane_max_tets]
        if len(bounds) > 3:
            raise ValueError("at most three lane bounds (four lanes)")
        o.lanes = len(bounds) + 1
        for i, v in enumerate(bounds):
            o.lane_max_tets[i] = v
        o.workspace_budget_bytes = int(workspace_budget_bytes)
        o.solve = default_opts(**solve_opts)
        o.solve.output_memory = MEM_HOST
        h = c_vp()
        _check(lib().mfs_server_create(ctx.handle, ctypes.byref(o), ctypes.byref(h)))
        self.handle, self.ctx = h, ctx
        self._n = {}

    def close(self):
        if getattr(self, "handle", None):
            lib().mfs_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, ch, R, t):
        R, t = ch._pose(R, t)
        tk = ctypes.c_uint64()
        _check(lib().mfs_server_submit(self.handle, ch.handle, _ptr(R), _ptr(t), ctypes.byref(tk)))
        self._n[tk.value] = ch.n
        return tk.value

    def _result(self, ticket, fn, *extra):
        x = np.empty((self._n[ticket], 3))
        st, tm = SolveStats(), RequestTimes()
        rc = fn(self.handle, ticket, _ptr(x), ctypes.byref(st), ctypes.byref(tm), *extra)
        return x, st, tm, rc

    def poll(self, ticket):
        done = c_i32()
        x, st, tm, rc = self._result(ticket, lib().mfs_server_poll, ctypes.byref(done))
        if not done.value:
            _check(rc)
            return None
        del self._n[ticket]
        _check(rc)
        return x, st.as_dict(), {k: getattr(tm, k) for k, _ in tm._fields_}, rc

    def wait(self, ticket):
        x, st, tm, rc = self._result(ticket, lib().mfs_server_wait)
        del self._n[ticket]
        _check(rc)
        return x, st.as_dict(), {k: getattr(tm, k) for k, _ in tm._fields_}, rc

    def info(self):
        i = ServerInfo()
        _check(lib().mfs_server_get_info(self.handle, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in i._fields_}

    def set_lane_tuning(self, lane, **tuning):
        """PCG schedule of one lane (fields as ``Context.tuning()``; the ones
        not given keep the caller's context's values), applied by the lane
        before its next Newton step."""
        t = Tuning()
        _check(lib().mfs_context_get_tuning(self.ctx.handle, ctypes.byref(t)))
        for k, v in tuning.items():
            if not hasattr(t, k):
                raise TypeError(f"unknown tuning field {k}")
            setattr(t, k, int(v))
        _check(lib().mfs_server_set_lane_tuning(self.handle, int(lane), ctypes.byref(t)))
