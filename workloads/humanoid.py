"""Procedural humanoid characters: 15 capsule limbs, jittered Delaunay fill.

A character is the union of 15 capsules (pelvis, abdomen, chest, neck, head,
and left/right upper arm, forearm, hand, thigh, shin) with seeded radii in
[0.1, 0.4] and lengths in [0.5, 1.5].  Its volume is filled by the Delaunay
tetrahedralisation of a jittered grid plus capsule-surface samples; tets whose
centroid lies outside the union and low-quality slivers are dropped, and the
largest face-connected piece is kept.

The rig has one handle per bone.  Bones start as the capsule axes; the
longest are split into collinear halves to reach more handles, or the
shortest leaves are merged into their parents to reach fewer.  Each handle
pins the three rest vertices nearest its joint and the three nearest the
midpoint of its first segment.  Materials are drawn per limb.

Everything is a function of the seed: the same arguments give bit-identical
arrays.
"""

import numpy as np
from scipy.spatial import Delaunay, cKDTree
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

from .common import ARAP, COROT, NH, euler_xyz, forward_kinematics, mean_edge_length, bbox_diag

CAPSULE_NAMES = ("pelvis", "abdomen", "chest", "neck", "head",
                 "l_upperarm", "l_forearm", "l_hand", "r_upperarm", "r_forearm", "r_hand",
                 "l_thigh", "l_shin", "r_thigh", "r_shin")
CAPSULE_PARENT = (-1, 0, 1, 2, 3, 2, 5, 6, 2, 8, 9, 0, 11, 0, 13)
LEG_SPLAY_DEG = 25.0
# Tets per h^3 of union volume for the jittered-grid fill (calibrated).
_TETS_PER_CELL = 6.45


def _capsules(rng):
    L = rng.uniform(0.5, 1.5, size=15)
    r = rng.uniform(0.1, 0.4, size=15)
    up = np.array([0.0, 0.0, 1.0])
    s = np.sin(np.deg2rad(LEG_SPLAY_DEG))
    c = np.cos(np.deg2rad(LEG_SPLAY_DEG))
    dirs = [up, up, up, up, up,
            np.array([1.0, 0, 0]), np.array([1.0, 0, 0]), np.array([1.0, 0, 0]),
            np.array([-1.0, 0, 0]), np.array([-1.0, 0, 0]), np.array([-1.0, 0, 0]),
            np.array([s, 0, -c]), np.array([s, 0, -c]),
            np.array([-s, 0, -c]), np.array([-s, 0, -c])]
    a = np.zeros((15, 3))
    b = np.zeros((15, 3))
    for i in range(15):
        p = CAPSULE_PARENT[i]
        if i in (11, 13):          # thighs start at the pelvis start (hip)
            start = a[0]
        elif p < 0:
            start = np.zeros(3)
        else:
            start = b[p]
        a[i] = start
        b[i] = start + L[i] * dirs[i]
    return a, b, r


def _seg_dist(P, a, b):
    """Distance from points P (k, 3) to segment [a, b]."""
    d = b - a
    dd = float(d @ d)
    if dd == 0.0:
        return np.linalg.norm(P - a, axis=1)
    u = np.clip((P - a) @ d / dd, 0.0, 1.0)
    return np.linalg.norm(P - (a + u[:, None] * d), axis=1)


def _capsule_sd(P, a, b, r):
    """Signed distance of points to each capsule, shape (k, ncaps)."""
    return np.stack([_seg_dist(P, a[i], b[i]) - r[i] for i in range(len(r))], axis=1)


def _surface_samples(a, b, r, h):
    pts = []
    golden = np.pi * (3.0 - np.sqrt(5.0))
    for i in range(len(r)):
        d = b[i] - a[i]
        L = np.linalg.norm(d)
        ax = d / L
        e1 = np.cross(ax, [0.0, 0.0, 1.0])
        if np.linalg.norm(e1) < 1e-8:
            e1 = np.cross(ax, [0.0, 1.0, 0.0])
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(ax, e1)
        n_len = max(1, int(round(L / h)))
        n_circ = max(6, int(round(2 * np.pi * r[i] / h)))
        for u in range(n_len):
            base = a[i] + d * (u + 0.5) / n_len
            ph = 2 * np.pi * (np.arange(n_circ) + 0.5 * (u % 2)) / n_circ
            pts.append(base + r[i] * (np.cos(ph)[:, None] * e1 + np.sin(ph)[:, None] * e2))
        n_sph = max(8, int(round(4 * np.pi * r[i] ** 2 / h ** 2)))
        k = np.arange(n_sph)
        z = 1.0 - 2.0 * (k + 0.5) / n_sph
        rho = np.sqrt(1.0 - z * z)
        th = golden * k
        dirs = (rho * np.cos(th))[:, None] * e1 + (rho * np.sin(th))[:, None] * e2 + z[:, None] * ax
        low = dirs @ ax < 0
        pts.append(a[i] + r[i] * dirs[low])
        pts.append(b[i] + r[i] * dirs[~low])
    return np.concatenate(pts)


def _thin(P, rmin):
    """Greedy removal of points closer than rmin to an earlier kept point."""
    tree = cKDTree(P)
    pairs = tree.query_pairs(rmin, output_type="ndarray")
    keep = np.ones(len(P), dtype=bool)
    if len(pairs):
        pairs = pairs[np.lexsort((pairs[:, 1], pairs[:, 0]))]
        for i, j in pairs:
            if keep[i]:
                keep[j] = False
    return P[keep]


def _tet_quality(X, T):
    """6*sqrt(2)*|V| / rms(edge)^3: 1 for a regular tet, 0 for a flat one."""
    p = X[T]
    vol = np.abs(np.einsum("ij,ij->i", p[:, 1] - p[:, 0],
                           np.cross(p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]))) / 6.0
    e2 = sum(((p[:, a] - p[:, b]) ** 2).sum(1) for a in range(4) for b in range(a + 1, 4))
    lrms = np.sqrt(e2 / 6.0)
    return 6.0 * np.sqrt(2.0) * vol / lrms ** 3


def _largest_face_component(T):
    m = len(T)
    faces = np.concatenate([np.sort(T[:, [1, 2, 3]], 1), np.sort(T[:, [0, 2, 3]], 1),
                            np.sort(T[:, [0, 1, 3]], 1), np.sort(T[:, [0, 1, 2]], 1)])
    owner = np.tile(np.arange(m), 4)
    order = np.lexsort((faces[:, 2], faces[:, 1], faces[:, 0]))
    f = faces[order]
    o = owner[order]
    same = np.all(f[1:] == f[:-1], axis=1)
    i = np.nonzero(same)[0]
    g = coo_matrix((np.ones(len(i)), (o[i], o[i + 1])), shape=(m, m))
    _, lab = connected_components(g, directed=False)
    big = np.argmax(np.bincount(lab))
    return lab == big


def _mesh_union(a, b, r, target_tets, rng):
    lo = np.min(np.minimum(a, b) - r[:, None], axis=0)
    hi = np.max(np.maximum(a, b) + r[:, None], axis=0)
    mc = rng.uniform(lo, hi, size=(200000, 3))
    vol = np.prod(hi - lo) * np.mean(_capsule_sd(mc, a, b, r).min(1) < 0)
    h = (_TETS_PER_CELL * vol / target_tets) ** (1.0 / 3.0)
    # jittered interior grid
    n = np.ceil((hi - lo) / h).astype(int) + 1
    gi = np.stack(np.meshgrid(*[np.arange(k) for k in n], indexing="ij"), -1).reshape(-1, 3)
    G = lo + h * gi + rng.uniform(-0.25, 0.25, size=gi.shape) * h
    G = G[_capsule_sd(G, a, b, r).min(1) < -0.4 * h]
    S = _surface_samples(a, b, r, h)
    S = S[_capsule_sd(S, a, b, r).min(1) > -0.3 * h]
    P = _thin(np.concatenate([S, G]), 0.6 * h)
    T = Delaunay(P).simplices.astype(np.int64)
    cen = P[T].mean(1)
    T = T[_capsule_sd(cen, a, b, r).min(1) < 0]
    T = T[_tet_quality(P, T) > 0.12]
    T = T[_largest_face_component(T)]
    used = np.unique(T)
    remap = np.full(len(P), -1, dtype=np.int64)
    remap[used] = np.arange(len(used))
    return P[used], remap[T].astype(np.int32), h


def _bones(a, b, n_bones):
    """Bone list [(segments, joint, parent)] with parents before children."""
    bones = [{"segs": [(a[i].copy(), b[i].copy())], "parent": CAPSULE_PARENT[i]} for i in range(15)]
    while len(bones) < n_bones:
        lens = [np.linalg.norm(bn["segs"][0][1] - bn["segs"][0][0]) for bn in bones]
        k = int(np.argmax(lens))
        s0, s1 = bones[k]["segs"][0]
        mid = 0.5 * (s0 + s1)
        bones[k]["segs"][0] = (s0, mid)
        new = {"segs": [(mid, s1)], "parent": k}
        j = len(bones)
        for bn in bones:           # children of k now hang off the distal half
            if bn["parent"] == k:
                bn["parent"] = j
        new["parent"] = k
        bones.append(new)
    while len(bones) > n_bones:
        children = {bn["parent"] for bn in bones}
        leaves = [i for i in range(len(bones)) if i not in children and bones[i]["parent"] >= 0]
        lens = [np.linalg.norm(bones[i]["segs"][0][1] - bones[i]["segs"][0][0]) for i in leaves]
        k = leaves[int(np.argmin(lens))]
        p = bones[k]["parent"]
        bones[p]["segs"].extend(bones[k]["segs"])
        del bones[k]
        for bn in bones:
            if bn["parent"] > k:
                bn["parent"] -= 1
    # order parents before children (breadth-first from the roots)
    order, frontier = [], [i for i, bn in enumerate(bones) if bn["parent"] < 0]
    while frontier:
        order.extend(frontier)
        frontier = [i for i, bn in enumerate(bones) if bn["parent"] in frontier]
    new_id = {old: new for new, old in enumerate(order)}
    out = []
    for old in order:
        bn = bones[old]
        out.append({"segs": bn["segs"], "joint": bn["segs"][0][0].copy(),
                    "parent": -1 if bn["parent"] < 0 else new_id[bn["parent"]]})
    return out


def _nearest_vertices(X, p, k):
    d = np.linalg.norm(X - p, axis=1)
    return np.lexsort((np.arange(len(X)), d))[:k]


def humanoid(seed, target_tets=50000, n_bones=20, models=(NH, ARAP),
             youngs_range=(1e4, 1e6), poisson_range=(0.3, 0.49), name=None):
    """Seeded procedural humanoid problem (see module docstring)."""
    rng = np.random.default_rng(seed)
    a, b, r = _capsules(rng)
    X, T, h = _mesh_union(a, b, r, target_tets, rng)
    m = len(T)
    # materials per limb: each tet takes the capsule nearest its centroid
    limb = np.argmin(_capsule_sd(X[T].mean(1), a, b, r), axis=1)
    limb_model = rng.choice(np.asarray(models, dtype=np.int32), size=15)
    limb_E = np.exp(rng.uniform(np.log(youngs_range[0]), np.log(youngs_range[1]), size=15))
    limb_nu = rng.uniform(poisson_range[0], poisson_range[1], size=15)
    bones = _bones(a, b, n_bones)
    seg_a, seg_b, seg_h = [], [], []
    for hdl, bn in enumerate(bones):
        for s0, s1 in bn["segs"]:
            seg_a.append(s0)
            seg_b.append(s1)
            seg_h.append(hdl)
    pins = []
    for hdl, bn in enumerate(bones):
        s0, s1 = bn["segs"][0]
        for v in _nearest_vertices(X, bn["joint"], 3):
            pins.append((int(v), hdl))
        for v in _nearest_vertices(X, 0.5 * (s0 + s1), 3):
            pins.append((int(v), hdl))
    pins = sorted(set(pins), key=lambda p: (p[1], p[0]))
    youngs = limb_E[limb]
    return {
        "name": name or f"humanoid_s{seed}_m{m}",
        "X": X, "T": T,
        "model": limb_model[limb].astype(np.int32),
        "youngs": youngs.astype(np.float64),
        "poisson": limb_nu[limb].astype(np.float64),
        "n_handles": len(bones),
        "seg_a": np.array(seg_a), "seg_b": np.array(seg_b),
        "seg_handle": np.array(seg_h, dtype=np.int32),
        "pin_vertex": np.array([p[0] for p in pins], dtype=np.int32),
        "pin_handle": np.array([p[1] for p in pins], dtype=np.int32),
        "pin_stiffness": 100.0 * float(youngs.max()) * mean_edge_length(X, T),
        "bbox_diag": bbox_diag(X),
        "handle_parent": np.array([bn["parent"] for bn in bones], dtype=np.int32),
        "handle_joint": np.array([bn["joint"] for bn in bones]),
        "grid_spacing": h,
        "capsules": (a, b, r),
    }


def random_pose(prob, seed, amp_deg=45.0):
    """Joint Euler angles uniform in +-amp (intrinsic XYZ, local to the
    parent); root handles stay at the identity."""
    rng = np.random.default_rng(seed)
    nh = prob["n_handles"]
    ang = np.deg2rad(rng.uniform(-amp_deg, amp_deg, size=(nh, 3)))
    local = np.stack([np.eye(3) if prob["handle_parent"][h] < 0 else euler_xyz(*ang[h])
                      for h in range(nh)])
    return forward_kinematics(prob["handle_parent"], prob["handle_joint"], local)


def animation_pose(prob, seed, frame, fps=30.0, amp_deg=60.0, period=(2.0, 5.0)):
    """Frame of a smooth animation: each joint angle follows
    amp * sin(2 pi t / P + phi) with seeded P ~ U[period] and phi ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    nh = prob["n_handles"]
    P = rng.uniform(period[0], period[1], size=(nh, 3))
    phi = rng.uniform(0.0, 2 * np.pi, size=(nh, 3))
    t = frame / fps
    ang = np.deg2rad(amp_deg) * np.sin(2 * np.pi * t / P + phi)
    local = np.stack([np.eye(3) if prob["handle_parent"][h] < 0 else euler_xyz(*ang[h])
                      for h in range(nh)])
    return forward_kinematics(prob["handle_parent"], prob["handle_joint"], local)


def _pool_member(args):
    i, seed0, tets_range, handles_range, models = args
    rng = np.random.default_rng(seed0 + i)
    m = float(np.exp(rng.uniform(np.log(tets_range[0]), np.log(tets_range[1]))))
    nh = int(rng.integers(handles_range[0], handles_range[1] + 1))
    return humanoid(seed0 + i, target_tets=m, n_bones=nh, models=models, name=f"char{i}_s{seed0 + i}")


def pool_member(i, seed0, tets_range, handles_range, models):
    """Member i of ``character_pool(count, seed0, ...)`` built on its own."""
    return _pool_member((i, seed0, tets_range, handles_range, tuple(models)))


def character_pool(count, seed0, tets_range, handles_range, models, workers=1):
    """Characters with log-uniform sizes and uniform handle counts.

    Character i uses seed ``seed0 + i`` for its size, handle count, mesh and
    materials, so the list does not depend on ``workers`` (processes that
    build members in parallel).  Returns a list of problems.
    """
    jobs = [(i, seed0, tets_range, handles_range, tuple(models)) for i in range(count)]
    if workers <= 1:
        return [_pool_member(j) for j in jobs]
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_pool_member, jobs))
