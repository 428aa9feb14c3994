"""Seeded synthetic inputs for the mixed-FEM skinning per-frame solve.

This package only *builds problems*: rest tetrahedral meshes, per-element
material parameters, rig handles (bone segments, joints, pinned vertices) and
handle poses (rest -> posed rigid transforms).  It holds none of the solver's
arithmetic: no deformation gradients, stretch energies, rotation clusters,
pin targets or linear algebra of the method.  The CPU oracle and the GPU
library both consume its output and share nothing else.

A problem is a plain dict (see ``problem_keys``); a pose is a pair of arrays
``(R, t)`` with ``R`` of shape (n_handles, 3, 3) and ``t`` of shape
(n_handles, 3), mapping a rest point X of handle h to ``R[h] @ X + t[h]``.
"""

from .common import (ARAP, COROT, NH, MODEL_NAMES, problem_keys,
                     rot_x, rot_y, rot_z, euler_xyz, mean_edge_length)
from .beam import beam, beam_pose, tiny_mesh
from .humanoid import humanoid, random_pose, animation_pose, character_pool, pool_member

__all__ = [
    "ARAP", "COROT", "NH", "MODEL_NAMES", "problem_keys",
    "rot_x", "rot_y", "rot_z", "euler_xyz", "mean_edge_length",
    "beam", "beam_pose", "tiny_mesh",
    "humanoid", "random_pose", "animation_pose", "character_pool", "pool_member",
]
