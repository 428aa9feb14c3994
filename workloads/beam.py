"""Box-beam problems: unit cubes split into six Kuhn tetrahedra.

The standard instance is a 16 x 4 x 4 beam (425 vertices, 1536 tets) whose
x = 0 end cap follows handle 0 and whose x = 16 end cap follows handle 1; it
is the deterministic bending/twisting case used to exercise the solver on a
mesh with a known, exact layout.
"""

import numpy as np

from .common import NH, rot_x, mean_edge_length, bbox_diag

# Axis orders of the six Kuhn tetrahedra of a cube: a tet walks from the
# cube's low corner to its high corner, stepping one axis at a time.
KUHN_PERMUTATIONS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def _kuhn_block(nx, ny, nz):
    sx, sy = nx + 1, (nx + 1) * (ny + 1)

    def vid(i, j, k):
        return i + sx * j + sy * k

    X = np.array([[i, j, k] for k in range(nz + 1) for j in range(ny + 1)
                  for i in range(nx + 1)], dtype=np.float64)
    T = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for perm in KUHN_PERMUTATIONS:
                    c = [i, j, k]
                    tet = [vid(*c)]
                    for ax in perm:
                        c = list(c)
                        c[ax] += 1
                        tet.append(vid(*c))
                    T.append(tet)
    return X, np.array(T, dtype=np.int32)


def beam(nx=16, ny=4, nz=4, model=NH, youngs=1e5, poisson=0.45,
         pin_stiffness=None, name=None):
    """Kuhn-split box beam with both end caps pinned.

    ``model``, ``youngs`` and ``poisson`` may be scalars or per-tet arrays.
    Handle 0 owns the x = 0 cap, handle 1 the x = nx cap; each handle is a
    point (a zero-length segment) at its cap's centroid.  The pin stiffness
    defaults to 100 * max(E) * (mean rest edge length).
    """
    X, T = _kuhn_block(nx, ny, nz)
    m = T.shape[0]
    model = np.broadcast_to(np.asarray(model, dtype=np.int32), (m,)).copy()
    youngs = np.broadcast_to(np.asarray(youngs, dtype=np.float64), (m,)).copy()
    poisson = np.broadcast_to(np.asarray(poisson, dtype=np.float64), (m,)).copy()
    c0 = np.array([0.0, ny / 2.0, nz / 2.0])
    c1 = np.array([float(nx), ny / 2.0, nz / 2.0])
    cap0 = np.nonzero(X[:, 0] == 0.0)[0]
    cap1 = np.nonzero(X[:, 0] == float(nx))[0]
    pin_vertex = np.concatenate([cap0, cap1]).astype(np.int32)
    pin_handle = np.concatenate([np.zeros(len(cap0)), np.ones(len(cap1))]).astype(np.int32)
    if pin_stiffness is None:
        pin_stiffness = 100.0 * float(youngs.max()) * mean_edge_length(X, T)
    return {
        "name": name or f"beam_{nx}x{ny}x{nz}",
        "X": X, "T": T, "model": model, "youngs": youngs, "poisson": poisson,
        "n_handles": 2,
        "seg_a": np.stack([c0, c1]), "seg_b": np.stack([c0, c1]),
        "seg_handle": np.array([0, 1], dtype=np.int32),
        "pin_vertex": pin_vertex, "pin_handle": pin_handle,
        "pin_stiffness": float(pin_stiffness),
        "bbox_diag": bbox_diag(X),
        "handle_parent": np.array([-1, -1], dtype=np.int32),
        "handle_joint": np.stack([c0, c1]),
    }


def beam_pose(prob, angle_deg=30.0, translate=(2.0, 0.0, 0.0)):
    """Handle 0 fixed; handle 1 rotated about the beam axis through its cap
    centroid by ``angle_deg`` (right-hand rule about +x), then translated."""
    c = prob["handle_joint"][1]
    R1 = rot_x(np.deg2rad(angle_deg))
    R = np.stack([np.eye(3), R1])
    t = np.stack([np.zeros(3), c - R1 @ c + np.asarray(translate, dtype=np.float64)])
    return R, t


def tiny_mesh(kind="one", model=NH, youngs=1e5, poisson=0.45, pin_stiffness=1e6):
    """Meshes of one to six tets for brute-force checks.

    ``"one"``: a single tet with three of its vertices pinned (two handles);
    ``"cube"``: one cube split into six Kuhn tets, x = 0 face on handle 0 and
    one x = 1 vertex on handle 1, leaving three vertices free.
    """
    if kind == "one":
        X = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 1.1, 0.1], [0.3, 0.2, 0.9]])
        T = np.array([[0, 1, 2, 3]], dtype=np.int32)
        pin_vertex = np.array([0, 1, 2], dtype=np.int32)
        pin_handle = np.array([0, 0, 1], dtype=np.int32)
    elif kind == "cube":
        X, T = _kuhn_block(1, 1, 1)
        pin_vertex = np.array([0, 2, 4, 6, 7], dtype=np.int32)
        pin_handle = np.array([0, 0, 0, 0, 1], dtype=np.int32)
    else:
        raise ValueError(kind)
    m = T.shape[0]
    joint = np.array([[0.0, 0.5, 0.5], [1.0, 0.5, 0.5]])
    return {
        "name": f"tiny_{kind}",
        "X": X, "T": T,
        "model": np.full(m, model, dtype=np.int32),
        "youngs": np.full(m, youngs, dtype=np.float64),
        "poisson": np.full(m, poisson, dtype=np.float64),
        "n_handles": 2,
        "seg_a": joint.copy(), "seg_b": joint.copy(),
        "seg_handle": np.array([0, 1], dtype=np.int32),
        "pin_vertex": pin_vertex, "pin_handle": pin_handle,
        "pin_stiffness": float(pin_stiffness),
        "bbox_diag": bbox_diag(X),
        "handle_parent": np.array([-1, -1], dtype=np.int32),
        "handle_joint": joint,
    }
