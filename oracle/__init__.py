"""Plain, slow FP64 CPU oracle of the mixed-FEM skinning per-frame solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product package
never imports it, and it imports nothing from the product: the two share no
code beyond the seeded input builders in ``workloads``.

Every function follows the paper ("Automatic Skinning using the Mixed Finite
Element Method", Song et al.): Section 3 (Method), its discrete mixed energy,
KKT system and Schur condensation, Section 3.1 (Final Algorithm, Algorithm 1)
and Section 3.2 (Implementation details, "Initial shape preservation").  The
readings taken where the paper is silent or garbled are listed in the module
docstring of ``oracle.mfem``.

Parity pins (tests/test_oracle_*.py) tie each function to something other than
itself: finite differences, closed forms at S = I, numpy's pseudo-inverse,
scipy's polar decomposition, a brute-force dense KKT solve, rest and rigid
invariants, posed-space equivariance and dense-vs-sparse solves.
"""

from .mfem import (ARAP, COROT, NH, lame, vech, unvech, sym_basis, rest_shape,
                   shape_gradients, deformation_operator, rotation_operator,
                   mixed_operator, psi, dpsi, d2psi, stretch_gradient, stretch_hessian,
                   polar, polar_stretch, cluster_by_segments, blend_weights, blend_rotations,
                   pin_targets, Frame,
                   solve_frame, interpolate_pose, energy, gradient, hessian, stress,
                   DegenerateElement)

__all__ = [
    "ARAP", "COROT", "NH", "lame", "vech", "unvech", "sym_basis", "rest_shape",
    "shape_gradients", "deformation_operator", "rotation_operator", "mixed_operator",
    "psi", "dpsi", "d2psi", "stretch_gradient", "stretch_hessian", "polar",
    "polar_stretch", "cluster_by_segments", "pin_targets", "Frame", "solve_frame",
    "interpolate_pose", "stress", "blend_weights", "blend_rotations",
    "energy", "gradient", "hessian", "DegenerateElement",
]
