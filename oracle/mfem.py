"""FP64 oracle of the mixed-FEM skinning per-frame solve (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py; never by the product package.

What it computes (paper Section 3).  Each tet k carries a symmetric stretch
S_k (6-vector s_k), a rotation R_k fixed by the rig, and the volume W_k.  The
discrete mixed energy (eq. 5, vectorised as eq. 6) couples them through the
constraint B_k x = R_k s_k, enforced by multipliers.  Condensing s and the
multipliers with the pseudo-inverse of the block-diagonal [R] (eqs. 10-12 and
the text after eq. 12) leaves a vertex-only problem whose solution is the
minimiser of

    E(x) = sum_k W_k Psi_k(S_k(x)) + k_s/2 ||P x - x_p||^2,
    s_k(x) = R_k^+ B_k x   (= vech(sym(R_k^T F_k)), F_k = B_k x).

For energies quadratic in S (ARAP, co-rotated linear) E is quadratic and one
linear solve reaches the optimum (end of Section 3).  For neo-Hookean the
condensed system of eq. 12 is the Newton system of E, iterated with a line
search.

Readings taken where the paper is silent, garbled or inconsistent:
  R1  R_k is the rig rotation of the tet's cluster (Section 3.1); the polar
      decomposition of F only supplies the mixed warm start s0 = stretch of
      F(x0) (identity for inverted elements).
  R2  The KKT system (eqs. 8-9) is read as a Newton increment: K dx = -grad E
      (the printed right-hand sides mix absolute values and increments).
  R3  [R] H_s^-1 [R]^T in eq. 11 is singular (9 rows, 6 unknowns per tet); the
      constraint is taken in least squares through the pseudo-inverse R_k^+,
      i.e. s_k = sym(R_k^T F_k).
  R4  B_k is the 9x12 per-tet operator (the printed "3x4" is the shape-
      gradient matrix); s in R^{6m}, lambda in R^{9m}.
  R5  s = (S00, S11, S22, S12, S02, S01), plain entries.
  R6  Materials: ARAP Psi = mu ||S - I||^2; co-rotated Psi = mu ||S - I||^2 +
      lam/2 tr(S - I)^2; compressible neo-Hookean Psi = mu/2 (tr(S S) - 3) -
      mu ln J + lam/2 (ln J)^2 with J = det S and S positive definite (else
      +inf).  Lame parameters from (E, nu).
  R7  Pin targets follow the pin's handle: x_p = R_h X_p + t_h (Section 3.2,
      "Initial shape preservation").
  R8  Rotation clusters: nearest bone segment to the tet barycenter (Section
      3.1), ties to the lowest segment index; a handle given as a point is a
      zero-length segment.
  R9  Neo-Hookean Hessian clamp: (mu - lam ln J) -> max(mu - lam ln J, 0) in
      the Hessian only, so every element block is positive semidefinite.
  R10 Line search (absent from the paper): alpha = 1, 1/2, ... (40 halvings).
      Newton phase (s = J x): accept when every neo-Hookean S_k(x + a dx) is
      positive definite and Armijo holds, E(x + a dx) <= E(x) + 1e-4 a
      gradE.dx + 1e-12 |E(x)| (the last term absorbs FP64 rounding of E).
      Mixed phase (s != J x, the predictor steps): the largest halving for
      which every neo-Hookean s_k + a ds_k is positive definite, with no
      energy test.  The mixed step is a Newton step of the mixed problem in
      (x, s) with the constraint linearised, not a descent step of E(x): at
      an iterate with s != J x the condensed energy E(x) is not the function
      being minimised, so asking E(x1) <= E(x0) would reject steps of the
      method itself (a full step lands on the constraint s = J x, where the
      Newton phase and its Armijo test take over).
  R11 Stop after a fixed iteration count (predictor counts as iteration 1),
      or when max_v ||alpha dx_v|| <= step_tol * bbox_diag.
  R12 Mixed phase, then Newton phase: s starts at the polar stretch of F(x0)
      (R1) and moves by alpha (J(x + dx) - s) under the mixed rule of R10;
      alpha = 1 puts s on the constraint and starts the Newton phase.  Load
      stepping for poses whose mixed phase stalls (see solve_frame).

Extension beyond the paper's per-frame statement: external vertex forces
f_ext (the local-perturbation experiment of Section 4) enter as the
potential -f_ext . x, i.e. b += f_ext in the Newton system; problems carry
them as ``force_vertex`` (indices, repeats add up) and ``force`` (k x 3).

Rotation smoothing (reading R15; the paper names rotation discontinuities at
cluster boundaries as its main limitation and leaves smoothing to future
work): with ``blend_handles``/``blend_weights`` (m x K, from blend_weights) a
tet's rotation is the rotation factor of the polar decomposition of the
weighted sum of its handles' rotations, instead of its cluster's rotation.

Stress recovery (f2): ``stress`` returns P_k = dPsi/dS at S_k(x) and the
world-frame multiplier W_k R_k P_k.
"""

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

ARAP, COROT, NH = 0, 1, 2

# 6-vector coordinates of a symmetric 3x3 matrix (reading R5).
SYM_INDEX = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


class DegenerateElement(ValueError):
    pass


def lame(youngs, poisson):
    """Lame parameters (mu, lambda) of isotropic linear elasticity from Young's
    modulus E and Poisson ratio nu: mu = E / (2 (1 + nu)) and
    lambda = E nu / ((1 + nu)(1 - 2 nu)) (reading R6; the paper gives
    stiffnesses, not formulas)."""
    E = np.asarray(youngs, dtype=np.float64)
    nu = np.asarray(poisson, dtype=np.float64)
    return E / (2.0 * (1.0 + nu)), E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))


def sym_basis():
    """E^(c) = dS/ds_c for the 6-vector coordinates (reading R5)."""
    E = np.zeros((6, 3, 3))
    for c, (i, j) in enumerate(SYM_INDEX):
        E[c, i, j] = 1.0
        E[c, j, i] = 1.0
    return E


def vech(S):
    S = np.asarray(S)
    return np.stack([S[..., i, j] for i, j in SYM_INDEX], axis=-1)


def unvech(s):
    return np.einsum("...c,cij->...ij", s, sym_basis())


# ----------------------------------------------------------------------------
# Rest shape: deformation-gradient operator F = B x (Section 3, after eq. 4)
# and element volumes W_k (after eq. 5).
# ----------------------------------------------------------------------------

def _mean_edge(X, T):
    e = np.concatenate([T[:, [a, b]] for a in range(4) for b in range(a + 1, 4)])
    e = np.unique(np.sort(e, axis=1), axis=0)
    return float(np.linalg.norm(X[e[:, 0]] - X[e[:, 1]], axis=1).mean())


def rest_shape(X, T):
    """Dm_k = [X1-X0, X2-X0, X3-X0] (columns); G_k = Dm_k^-1; W_k = |det Dm_k|/6.

    Raises DegenerateElement when |det Dm_k| <= 1e-12 * (mean edge)^3.
    """
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.int64)
    Dm = np.stack([X[T[:, 1]] - X[T[:, 0]], X[T[:, 2]] - X[T[:, 0]],
                   X[T[:, 3]] - X[T[:, 0]]], axis=-1)
    det = np.linalg.det(Dm)
    tol = 1e-12 * _mean_edge(X, T) ** 3
    bad = np.nonzero(np.abs(det) <= tol)[0]
    if len(bad):
        raise DegenerateElement(f"degenerate rest tets: {bad[:8].tolist()}")
    return np.linalg.inv(Dm), np.abs(det) / 6.0


def shape_gradients(G):
    """Gradients of the four linear shape functions, (m, 4, 3): rows of G for
    vertices 1..3 and minus their sum for vertex 0."""
    gN = np.empty((G.shape[0], 4, 3))
    gN[:, 1:, :] = G
    gN[:, 0, :] = -G.sum(axis=1)
    return gN


def deformation_operator(G):
    """B_k (m, 9, 12) with vec(F_k) = B_k x_k; vec is row-major (index 3i+j)
    and x_k stacks the tet's four vertex positions (index 3a+i)."""
    gN = shape_gradients(G)
    m = G.shape[0]
    B = np.zeros((m, 9, 12))
    for i in range(3):
        for j in range(3):
            for a in range(4):
                B[:, 3 * i + j, 3 * a + i] = gN[:, a, j]
    return B


def rotation_operator(Rk):
    """R_k (m, 9, 6): the map s -> vec(R_k S(s)) (Section 3, after eq. 6)."""
    E = sym_basis()
    cols = np.einsum("kij,cjl->kcil", Rk, E).reshape(Rk.shape[0], 6, 9)
    return np.transpose(cols, (0, 2, 1))


def mixed_operator(Rk, G):
    """J_k = R_k^+ B_k (m, 6, 12): the condensed stretch s_k = J_k x_k, with
    R_k^+ the pseudo-inverse of the 9x6 rotation block (text after eq. 12)."""
    return np.einsum("kcr,krj->kcj", np.linalg.pinv(rotation_operator(Rk)),
                     deformation_operator(G))


# ----------------------------------------------------------------------------
# Materials (reading R6): Psi(S), dPsi/dS and the Hessian bilinear form.
# ----------------------------------------------------------------------------

def _spd(S):
    """Sylvester's criterion on each 3x3 symmetric matrix."""
    m1 = S[:, 0, 0]
    m2 = S[:, 0, 0] * S[:, 1, 1] - S[:, 0, 1] * S[:, 1, 0]
    return (m1 > 0) & (m2 > 0) & (np.linalg.det(S) > 0)


def psi(S, model, mu, lam):
    """Stretch energy density per element; +inf for infeasible neo-Hookean."""
    I = np.eye(3)
    D = S - I
    dev = np.einsum("kij,kij->k", D, D)
    tr = np.trace(D, axis1=1, axis2=2)
    out = np.where(model == ARAP, mu * dev, mu * dev + 0.5 * lam * tr * tr)
    nh = model == NH
    if np.any(nh):
        Sn = S[nh]
        ok = _spd(Sn)
        J = np.linalg.det(Sn)
        lnJ = np.log(np.where(ok, J, 1.0))
        val = (0.5 * mu[nh] * (np.einsum("kij,kji->k", Sn, Sn) - 3.0) - mu[nh] * lnJ
               + 0.5 * lam[nh] * lnJ * lnJ)
        out = out.copy()
        out[nh] = np.where(ok, val, np.inf)
    return out


def _nh_parts(S, model):
    nh = model == NH
    Sinv = np.zeros_like(S)
    lnJ = np.zeros(S.shape[0])
    if np.any(nh):
        if not np.all(_spd(S[nh])):
            raise ValueError("neo-Hookean derivative at a non-positive-definite stretch")
        Sinv[nh] = np.linalg.inv(S[nh])
        lnJ[nh] = np.log(np.linalg.det(S[nh]))
    return nh, Sinv, lnJ


def dpsi(S, model, mu, lam):
    """P = dPsi/dS (symmetric 3x3 per element)."""
    I = np.eye(3)
    tr = np.trace(S - I, axis1=1, axis2=2)
    P = 2.0 * mu[:, None, None] * (S - I)
    P = P + np.where(model == COROT, lam * tr, 0.0)[:, None, None] * I
    nh, Sinv, lnJ = _nh_parts(S, model)
    Pn = mu[:, None, None] * S - mu[:, None, None] * Sinv + (lam * lnJ)[:, None, None] * Sinv
    return np.where(nh[:, None, None], Pn, P)


def d2psi(S, A, Bm, model, mu, lam, clamp=True, nh_parts=None):
    """Second derivative of Psi at S along symmetric directions A and Bm.

    ``nh_parts`` optionally passes the (mask, S^-1, ln J) triple of
    ``_nh_parts(S, model)`` so repeated calls at one S share it."""
    AB = np.einsum("kij,kij->k", A, Bm)
    trA = np.trace(A, axis1=1, axis2=2)
    trB = np.trace(Bm, axis1=1, axis2=2)
    out = np.where(model == COROT, 2.0 * mu * AB + lam * trA * trB, 2.0 * mu * AB)
    nh, Sinv, lnJ = nh_parts if nh_parts is not None else _nh_parts(S, model)
    if np.any(nh):
        c = mu - lam * lnJ
        if clamp:
            c = np.maximum(c, 0.0)
        SA = np.einsum("kij,kjl->kil", Sinv, A)
        SB = np.einsum("kij,kjl->kil", Sinv, Bm)
        val = (mu * AB + c * np.einsum("kij,kji->k", SA, SB)
               + lam * np.trace(SA, axis1=1, axis2=2) * np.trace(SB, axis1=1, axis2=2))
        out = np.where(nh, val, out)
    return out


def stretch_gradient(s, model, mu, lam):
    """g_k = dPsi/ds_k (m, 6): P : E^(c)."""
    P = dpsi(unvech(s), model, mu, lam)
    return np.einsum("kij,cij->kc", P, sym_basis())


def stretch_hessian(s, model, mu, lam, clamp=True):
    """H_k = d2Psi/ds_k^2 (m, 6, 6): the bilinear form on E^(c), E^(d)."""
    S = unvech(s)
    E = sym_basis()
    m = S.shape[0]
    parts = _nh_parts(S, model)
    H = np.empty((m, 6, 6))
    for c in range(6):
        for d in range(6):
            H[:, c, d] = d2psi(S, np.broadcast_to(E[c], S.shape), np.broadcast_to(E[d], S.shape),
                               model, mu, lam, clamp, nh_parts=parts)
    return H


# ----------------------------------------------------------------------------
# Polar decomposition (mixed warm start, reading R1) via the SVD.
# ----------------------------------------------------------------------------

def polar(F):
    """F = U P with U a proper rotation and P symmetric (SVD based)."""
    W, sig, Vt = np.linalg.svd(F)
    flip = np.linalg.det(W) * np.linalg.det(Vt) < 0
    W = W.copy()
    sig = sig.copy()
    W[flip, :, 2] *= -1.0
    sig[flip, 2] *= -1.0
    U = W @ Vt
    P = np.einsum("kji,kj,kjl->kil", Vt, sig, Vt)
    return U, 0.5 * (P + np.transpose(P, (0, 2, 1)))


def polar_stretch(F):
    """s0: stretch factor of F where det F > 0, identity otherwise."""
    _, P = polar(F)
    P[np.linalg.det(F) <= 0] = np.eye(3)
    return vech(P)


# ----------------------------------------------------------------------------
# Rig: rotation clusters (Section 3.1) and offset pin targets (Section 3.2).
# ----------------------------------------------------------------------------

def _barycenters(X, T):
    """((x0 + x1) + x2) + x3, times 1/4, per tet."""
    return (((X[T[:, 0]] + X[T[:, 1]]) + X[T[:, 2]]) + X[T[:, 3]]) * 0.25


def _segment_dist2(P, seg_a, seg_b):
    """Squared distances (len(P), nseg) from points to segments, every sum
    written out in one order with each product rounded on its own (no fused
    multiply-adds, no library dot products): a point as far from two segments
    as from their shared joint then ties exactly, and the tie goes to the lower
    segment index however the arithmetic is carried out elsewhere."""
    d2 = np.empty((P.shape[0], len(seg_a)))
    for s in range(len(seg_a)):
        a = np.asarray(seg_a[s], dtype=np.float64)
        d = np.asarray(seg_b[s], dtype=np.float64) - a
        dd = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
        if dd == 0.0:
            u = np.zeros(P.shape[0])
        else:
            r = P - a
            u = np.clip(((r[:, 0] * d[0] + r[:, 1] * d[1]) + r[:, 2] * d[2]) / dd, 0.0, 1.0)
        e = P - (a + u[:, None] * d)
        d2[:, s] = (e[:, 0] * e[:, 0] + e[:, 1] * e[:, 1]) + e[:, 2] * e[:, 2]
    return d2


def cluster_by_segments(X, T, seg_a, seg_b, seg_handle):
    """Handle of the bone segment nearest each tet's barycenter (reading R8;
    ties to the lowest segment index)."""
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.int64)
    d2 = _segment_dist2(_barycenters(X, T), seg_a, seg_b)
    return np.asarray(seg_handle, dtype=np.int32)[np.argmin(d2, axis=1)]


# ----------------------------------------------------------------------------
# Rotation smoothing across cluster boundaries (the paper's stated limitation
# and future work; reading R15): a tet blends the rotations of the handles
# whose bone segments lie within `width` of its nearest one, and the blend is
# projected back onto the rotations by the polar decomposition.
# ----------------------------------------------------------------------------

def blend_weights(X, T, seg_a, seg_b, seg_handle, width, kmax):
    """Per tet, kmax (handle, weight) pairs.  Distances d are from the tet's
    barycenter to the bone segments (as cluster_by_segments); a handle's
    distance is that of its nearest segment.  The handle of the nearest
    segment (the cluster rule, ties to the lowest segment index) comes first
    with weight 1; every other handle h with d_h - d_min < width follows with
    weight 1 - (d_h - d_min) / width, in decreasing weight (ties: lower handle
    index first); the first kmax are kept and divided by their sum (added in
    that order).  Unused entries: handle -1, weight 0."""
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.int64)
    seg_handle = np.asarray(seg_handle, dtype=np.int64)
    m = T.shape[0]
    d2 = _segment_dist2(_barycenters(X, T), seg_a, seg_b)
    handles = np.full((m, kmax), -1, dtype=np.int32)
    weights = np.zeros((m, kmax))
    hs = sorted(set(seg_handle.tolist()))
    for k in range(m):
        s0 = int(np.argmin(d2[k]))
        h0 = int(seg_handle[s0])
        dmin = math.sqrt(d2[k, s0])
        cand = []
        for h in hs:
            if h == h0:
                continue
            dh = math.sqrt(min(d2[k, s] for s in range(len(seg_a)) if seg_handle[s] == h))
            if width > 0.0 and dh - dmin < width:
                cand.append((1.0 - (dh - dmin) / width, h))
        cand.sort(key=lambda c: (-c[0], c[1]))
        chosen = [(1.0, h0)] + cand[: kmax - 1]
        total = 0.0
        for w, _ in chosen:
            total += w
        for j, (w, h) in enumerate(chosen):
            handles[k, j] = h
            weights[k, j] = w / total
    return handles, weights


def blend_rotations(R, handles, weights):
    """R_k = polar(sum_j w_kj R_{h_kj}) (the rotation factor).  A tet with a
    single handle takes that handle's rotation as it is; where the blend has
    det <= 0 the tet keeps the rotation of its first handle."""
    R = np.asarray(R, dtype=np.float64)
    handles = np.asarray(handles)
    M = np.zeros((handles.shape[0], 3, 3))
    for j in range(handles.shape[1]):
        ok = handles[:, j] >= 0
        M[ok] += weights[ok, j, None, None] * R[handles[ok, j]]
    U, _ = polar(M)
    keep = (np.linalg.det(M) <= 0.0) | (np.sum(handles >= 0, axis=1) == 1)
    U[keep] = R[handles[keep, 0]]
    return U


def pin_targets(X, pin_vertex, pin_handle, R, t):
    """x_p = R_h X_p + t_h for each pin (reading R7)."""
    Xp = np.asarray(X)[pin_vertex]
    return np.einsum("pij,pj->pi", R[pin_handle], Xp) + t[pin_handle]


# ----------------------------------------------------------------------------
# The condensed problem for one frame.
# ----------------------------------------------------------------------------

class Frame:
    """E(x), grad E(x) and the condensed matrix of eq. 12 for one rig pose."""

    def __init__(self, prob, pose, clusters=None):
        R, t = pose
        self.X = np.asarray(prob["X"], dtype=np.float64)
        self.T = np.asarray(prob["T"], dtype=np.int64)
        self.n = self.X.shape[0]
        self.m = self.T.shape[0]
        self.model = np.asarray(prob["model"], dtype=np.int32)
        self.mu, self.lam = lame(prob["youngs"], prob["poisson"])
        self.G, self.W = rest_shape(self.X, self.T)
        if clusters is None:
            clusters = prob.get("cluster")  # given clusters (user-defined rule)
        if clusters is None:
            clusters = cluster_by_segments(self.X, self.T, prob["seg_a"], prob["seg_b"],
                                           prob["seg_handle"])
        self.cluster = np.asarray(clusters, dtype=np.int32)
        if prob.get("blend_handles") is not None:  # rotation smoothing (R15)
            self.Rk = blend_rotations(R, prob["blend_handles"], prob["blend_weights"])
        else:
            self.Rk = np.asarray(R, dtype=np.float64)[self.cluster]
        self.B = deformation_operator(self.G)
        self.J = mixed_operator(self.Rk, self.G)
        self.pin_vertex = np.asarray(prob["pin_vertex"], dtype=np.int64)
        self.y = pin_targets(self.X, self.pin_vertex, np.asarray(prob["pin_handle"]), R, t)
        self.ks = float(prob["pin_stiffness"])
        self.bbox_diag = float(prob["bbox_diag"])
        self.dof = (3 * self.T[:, :, None] + np.arange(3)).reshape(self.m, 12)
        self.fext = np.zeros((self.n, 3))
        fv = prob.get("force_vertex")
        if fv is not None and len(fv):
            np.add.at(self.fext, np.asarray(fv, dtype=np.int64),
                      np.asarray(prob["force"], dtype=np.float64).reshape(-1, 3))

    def local(self, x):
        return np.asarray(x, dtype=np.float64).reshape(-1)[self.dof]

    def stretch(self, x):
        """s_k(x) = J_k x_k, (m, 6)."""
        return (self.J @ self.local(x)[:, :, None])[:, :, 0]

    def deformation_gradient(self, x):
        return np.einsum("krj,kj->kr", self.B, self.local(x)).reshape(self.m, 3, 3)

    def pin_residual(self, x):
        return np.asarray(x).reshape(-1, 3)[self.pin_vertex] - self.y

    def element_energy(self, x):
        return self.W * psi(unvech(self.stretch(x)), self.model, self.mu, self.lam)

    def energy(self, x):
        r = self.pin_residual(x)
        return float(self.element_energy(x).sum() + 0.5 * self.ks * (r * r).sum()
                     - (self.fext * np.asarray(x).reshape(-1, 3)).sum())

    def feasible(self, x):
        return bool(np.all(np.isfinite(self.element_energy(x))))

    def _scatter(self, local12):
        out = np.zeros(3 * self.n)
        np.add.at(out, self.dof, local12)
        return out

    def gradient(self, x, s_lin=None, clamp=True):
        """grad E(x); with s_lin, the mixed-predictor force of Section 3's KKT
        system linearised at s = s_lin instead of s = s(x)."""
        s = self.stretch(x)
        if s_lin is None:
            g = stretch_gradient(s, self.model, self.mu, self.lam)
        else:
            g = stretch_gradient(s_lin, self.model, self.mu, self.lam)
            H = stretch_hessian(s_lin, self.model, self.mu, self.lam, clamp)
            g = g + (H @ (s - s_lin)[:, :, None])[:, :, 0]
        Jt = np.transpose(self.J, (0, 2, 1))
        f = self._scatter((Jt @ (self.W[:, None] * g)[:, :, None])[:, :, 0])
        pin = np.zeros((self.n, 3))
        np.add.at(pin, self.pin_vertex, self.ks * self.pin_residual(x))
        return f + pin.reshape(-1) - self.fext.reshape(-1)

    def hessian(self, s, clamp=True):
        """K = H_x + sum_k W_k J_k^T H_k J_k (eq. 12 left-hand side), CSR."""
        H = stretch_hessian(s, self.model, self.mu, self.lam, clamp)
        Jt = np.transpose(self.J, (0, 2, 1))
        Kl = Jt @ (self.W[:, None, None] * H) @ self.J
        rows = np.repeat(self.dof, 12, axis=1).reshape(-1)
        cols = np.tile(self.dof, (1, 12)).reshape(-1)
        pd = (3 * self.pin_vertex[:, None] + np.arange(3)).reshape(-1)
        rows = np.concatenate([rows, pd])
        cols = np.concatenate([cols, pd])
        vals = np.concatenate([Kl.reshape(-1), np.full(len(pd), self.ks)])
        n3 = 3 * self.n
        return sp.coo_matrix((vals, (rows, cols)), shape=(n3, n3)).tocsr()


def stress(prob, pose, x):
    """Stress recovery (back-substitution of the stretch equations of
    Section 3): per tet, P_k = dPsi/dS at S_k = sym(R_k^T F_k(x)) as a
    6-vector (plain entries) and the volume-weighted world-frame multiplier
    lambda_k = W_k R_k P_k (3 x 3) of the constraint F_k = R_k S_k; NaN for an
    infeasible neo-Hookean tet."""
    fr = Frame(prob, pose)
    S = unvech(fr.stretch(x))
    m = fr.m
    P = np.full((m, 3, 3), np.nan)
    ok = np.ones(m, dtype=bool)
    nh = fr.model == NH
    if np.any(nh):
        ok[nh] = _spd(S[nh])
    if np.any(ok):
        P[ok] = dpsi(S[ok], fr.model[ok], fr.mu[ok], fr.lam[ok])
    lam = fr.W[:, None, None] * np.einsum("kij,kjl->kil", fr.Rk, P)
    return vech(P), lam


def energy(prob, pose, x):
    return Frame(prob, pose).energy(x)


def gradient(prob, pose, x):
    return Frame(prob, pose).gradient(x)


def hessian(prob, pose, x, clamp=True):
    fr = Frame(prob, pose)
    return fr.hessian(fr.stretch(x), clamp)


def _linear_solve(K, b, method):
    if method == "dense":
        return np.linalg.solve(K.toarray(), b)
    return spla.splu(K.tocsc()).solve(b)


def _se3_V(w):
    """V(w) = I + (1 - cos th)/th^2 [w] + (th - sin th)/th^3 [w]^2 (SE(3) exp)."""
    th = np.linalg.norm(w)
    K = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    if th < 1e-8:
        return np.eye(3) + 0.5 * K
    return np.eye(3) + (1 - np.cos(th)) / th ** 2 * K + (th - np.sin(th)) / th ** 3 * (K @ K)


def interpolate_pose(pose0, pose1, tau):
    """Handle transforms a fraction tau of the way from pose0 to pose1 along
    each handle's screw motion: T(tau) = T0 exp(tau log(T0^-1 T1)) in SE(3)
    (a rotation about a fixed joint keeps that joint fixed); tau = 1 gives
    pose1 exactly."""
    from scipy.spatial.transform import Rotation
    R0, t0 = (np.asarray(a, dtype=np.float64) for a in pose0)
    R1, t1 = (np.asarray(a, dtype=np.float64) for a in pose1)
    if tau >= 1.0:
        return R1.copy(), t1.copy()
    R = np.empty_like(R1)
    t = np.empty_like(t1)
    for h in range(R1.shape[0]):
        Rr = R0[h].T @ R1[h]
        tr = R0[h].T @ (t1[h] - t0[h])
        w = Rotation.from_matrix(Rr).as_rotvec()
        v = np.linalg.solve(_se3_V(w), tr)
        Re = Rotation.from_rotvec(tau * w).as_matrix()
        te = _se3_V(tau * w) @ (tau * v)
        R[h] = R0[h] @ Re
        t[h] = R0[h] @ te + t0[h]
    return R, t


def solve_frame(prob, pose, x0=None, iterations=None, max_iterations=50, step_tol=1e-12,
                linear_solver="splu", frame=None, load_bisections=6, pose0=None):
    """One frame of Algorithm 1 as a Newton iteration on the mixed problem.

    State: vertex positions x and per-element stretches s (the mixed variable
    of eq. 6).  Each iteration solves the condensed system (eq. 12) of the KKT
    Newton step (eqs. 8-11, reading R2) linearised at s:

        K(s) dx = -[grad C(x) + sum_k W_k J_k^T (g_k(s) + H_k(s)(J_k x - s_k))]
        ds_k    = J_k (x + dx) - s_k

    While s differs from J x (the "mixed" phase, which starts from s0 = the
    stretch factor of F(x0), reading R1) the step length is the first
    alpha = 1, 1/2, ... for which every neo-Hookean s_k + alpha ds_k is positive
    definite.  A full step satisfies the linear constraint s = J x exactly;
    from then on s = J x and the iteration is Newton's method on E with the
    Armijo line search of reading R10 ("newton" phase).  For ARAP and
    co-rotated elements the first step is already the optimum (end of
    Section 3).

    Load stepping (reading R12, not in the paper; off for a fixed iteration
    count): if the mixed phase of a load step takes more than 6 steps or no
    step is feasible, x returns to the last converged state and the pose is
    approached through intermediate poses (``interpolate_pose``: screw
    motion of each handle from ``pose0``, the identity pose by default, whose
    solution is the rest shape); the increment is halved at most
    ``load_bisections`` times and doubled after each intermediate pose
    converges to a 1e-4 * bbox step.

    Returns a dict with the final positions ``x`` (n, 3), the final stretches
    ``s`` (m, 6), per-iteration energies E(x) (+inf where infeasible) of the
    pose being solved, gradient norms, step lengths, step sizes, phases and
    load-step fractions, the iteration count, the number of clamped
    neo-Hookean elements per iteration, and ``status`` ("ok" or
    "not_converged").
    """
    nh = int(prob["n_handles"])
    if pose0 is None:
        pose0 = (np.tile(np.eye(3), (nh, 1, 1)), np.zeros((nh, 3)))
    loadstep = load_bisections > 0 and iterations is None
    fr = frame if frame is not None else Frame(prob, pose)
    x = (fr.X if x0 is None else np.asarray(x0, dtype=np.float64)).reshape(-1).copy()
    x_backup = x.copy()
    tau, tau_done, delta, bisections, load_mixed = 1.0, 0.0, 1.0, 0, 0
    s = polar_stretch(fr.deformation_gradient(x))
    s0 = s.copy()
    on_constraint = False
    nh_mask = fr.model == NH
    hist = {"energy": [], "grad_norm": [], "alpha": [], "step": [], "clamped": [], "phase": [],
            "tau": []}
    status = "ok"
    n_iter = iterations if iterations is not None else max_iterations
    converged = False

    def restart(new_tau):
        nonlocal fr, x, s, on_constraint, load_mixed, tau
        tau = new_tau
        fr = Frame(prob, interpolate_pose(pose0, pose, tau), clusters=fr.cluster)
        x = x_backup.copy()
        s = polar_stretch(fr.deformation_gradient(x))
        on_constraint = False
        load_mixed = 0

    it = -1
    for it in range(n_iter):
        E0 = fr.energy(x)
        grad = fr.gradient(x) if np.isfinite(E0) else None
        rhs = -fr.gradient(x, s_lin=s)
        K = fr.hessian(s)
        if np.any(nh_mask):
            _, _, lnJ = _nh_parts(unvech(s), fr.model)
            hist["clamped"].append(int(np.sum(nh_mask & (fr.mu - fr.lam * lnJ < 0))))
        else:
            hist["clamped"].append(0)
        dx = _linear_solve(K, rhs, linear_solver)
        ds = fr.stretch(x + dx) - s
        hist["energy"].append(E0)
        hist["grad_norm"].append(float(np.linalg.norm(grad)) if grad is not None else float("inf"))
        hist["phase"].append("newton" if on_constraint else "mixed")
        hist["tau"].append(tau)
        alpha, accepted = 1.0, False
        for _ in range(41):
            if on_constraint:
                Et = fr.energy(x + alpha * dx)
                accepted = bool(np.isfinite(Et)) and (
                    Et <= E0 + 1e-4 * alpha * float(grad @ dx) + 1e-12 * abs(E0))
            else:
                st = s + alpha * ds
                accepted = bool(np.all(_spd(unvech(st[nh_mask])))) if np.any(nh_mask) else True
            if accepted:
                break
            alpha *= 0.5
        was_newton = on_constraint
        if not was_newton:
            load_mixed += 1
        stalled = (not accepted) or (not was_newton and alpha < 1.0 and load_mixed > 6)
        if stalled and loadstep and bisections < load_bisections and it + 1 < n_iter:
            bisections += 1
            delta *= 0.5
            hist["alpha"].append(0.0)
            hist["step"].append(0.0)
            restart(tau_done + delta)
            continue
        if not accepted:
            status = "not_converged"
            hist["alpha"].append(0.0)
            hist["step"].append(0.0)
            break
        x = x + alpha * dx
        if on_constraint or alpha == 1.0:
            s = fr.stretch(x)
            on_constraint = True
        else:
            s = s + alpha * ds
        step = float(np.max(np.linalg.norm((alpha * dx).reshape(-1, 3), axis=1)))
        hist["alpha"].append(alpha)
        hist["step"].append(step)
        if iterations is None and was_newton:
            tol = step_tol if tau >= 1.0 else 1e-4
            if step <= tol * fr.bbox_diag:
                if tau >= 1.0:
                    converged = True
                    break
                x_backup = x.copy()
                tau_done = tau
                delta *= 2.0
                restart(min(1.0, tau_done + delta))
    if iterations is None and not converged and status == "ok":
        status = "not_converged"
    Ef = fr.energy(x)
    hist["energy"].append(Ef)
    hist["grad_norm"].append(float(np.linalg.norm(fr.gradient(x))) if np.isfinite(Ef)
                             else float("inf"))
    out = {"x": x.reshape(-1, 3), "s": s, "iterations": it + 1, "status": status,
           "cluster": fr.cluster, "s0": s0}
    out.update(hist)
    return out
