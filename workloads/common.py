"""Shared constants and small geometric helpers for building problems.

Only rig/pose construction lives here (axis rotations, Euler angles, the mean
edge length used to scale the pin stiffness).  Nothing in this file evaluates
the skinning method itself.
"""

import numpy as np

# Material model identifiers (per element), matching the C-ABI enumeration.
ARAP = 0    # as-rigid-as-possible stretch energy
COROT = 1   # co-rotated linear elasticity
NH = 2      # compressible neo-Hookean
MODEL_NAMES = {ARAP: "arap", COROT: "corot", NH: "neohookean"}

problem_keys = (
    "name",          # str
    "X",             # (n, 3) float64 rest positions
    "T",             # (m, 4) int32 tetrahedra (vertex indices)
    "model",         # (m,) int32 material model id per element
    "youngs",        # (m,) float64 Young's modulus per element
    "poisson",       # (m,) float64 Poisson ratio per element
    "n_handles",     # int, number of rig handles (bones)
    "seg_a",         # (ns, 3) float64 bone segment start points (rest)
    "seg_b",         # (ns, 3) float64 bone segment end points (rest)
    "seg_handle",    # (ns,) int32 handle owning each segment
    "pin_vertex",    # (np,) int32 pinned vertex
    "pin_handle",    # (np,) int32 handle whose transform the pin follows
    "pin_stiffness", # float, penalty stiffness k_s
    "bbox_diag",     # float, rest bounding-box diagonal
    "handle_parent", # (nh,) int32 parent handle (-1 for roots)
    "handle_joint",  # (nh, 3) float64 rest joint (pivot) of each handle
)


def rot_x(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def rot_y(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def rot_z(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def euler_xyz(ax, ay, az):
    """Intrinsic X-Y-Z Euler rotation (radians): R = Rx(ax) Ry(ay) Rz(az)."""
    return rot_x(ax) @ rot_y(ay) @ rot_z(az)


def mean_edge_length(X, T):
    """Mean length of the unique edges of a tet mesh."""
    T = np.asarray(T, dtype=np.int64)
    pairs = np.concatenate([T[:, [a, b]] for a in range(4) for b in range(a + 1, 4)])
    pairs.sort(axis=1)
    pairs = np.unique(pairs, axis=0)
    return float(np.linalg.norm(X[pairs[:, 0]] - X[pairs[:, 1]], axis=1).mean())


def bbox_diag(X):
    return float(np.linalg.norm(X.max(axis=0) - X.min(axis=0)))


def forward_kinematics(parent, joint, local_R):
    """Rest->posed rigid transforms of a joint hierarchy.

    Each handle h rotates by ``local_R[h]`` about its rest joint, composed
    with its parent's transform: M_h(X) = M_parent(R_loc (X - j_h) + j_h).
    Parents must precede children.
    """
    nh = len(parent)
    R = np.zeros((nh, 3, 3))
    t = np.zeros((nh, 3))
    for h in range(nh):
        Rl = local_R[h]
        j = joint[h]
        if parent[h] < 0:
            Rp, tp = np.eye(3), np.zeros(3)
        else:
            assert parent[h] < h
            Rp, tp = R[parent[h]], t[parent[h]]
        R[h] = Rp @ Rl
        t[h] = Rp @ (j - Rl @ j) + tp
    return R, t
