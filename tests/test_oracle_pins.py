"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test ties one oracle function to something other than itself: central
finite differences, closed forms at S = I, numpy's pseudo-inverse, scipy's
polar decomposition, a dense brute-force KKT solve, rest/rigid invariants,
posed-space equivariance, dense-vs-sparse solves and brute-force clustering.
"""

import math

import numpy as np
import pytest
import scipy.linalg

import oracle
from oracle.mfem import _spd
from workloads import (ARAP, COROT, NH, beam, beam_pose, tiny_mesh, humanoid,
                       random_pose, euler_xyz)

MODELS = (ARAP, COROT, NH)


def _rand_spd(rng, m, spread=0.3):
    """Q diag(sigma) Q^T with sigma in [1 - spread, 1 + spread]."""
    Q = _rand_rot(rng, m)
    sig = rng.uniform(1.0 - spread, 1.0 + spread, size=(m, 3))
    S = np.einsum("kij,kj,klj->kil", Q, sig, Q)
    S = 0.5 * (S + np.transpose(S, (0, 2, 1)))
    assert np.all(_spd(S))
    return S


def _rand_rot(rng, m):
    return np.stack([euler_xyz(*rng.uniform(-np.pi, np.pi, 3)) for _ in range(m)])


# --------------------------------------------------------------------------
# P1: per-element gradient and (unclamped) Hessian vs central differences.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("where", ["random", "near_identity"])
def test_material_derivatives_match_finite_differences(model, where):
    rng = np.random.default_rng(7 + model)
    m = 16
    S = _rand_spd(rng, m, 0.3 if where == "random" else 1e-3)
    s = oracle.vech(S)
    mod = np.full(m, model, dtype=np.int32)
    mu, lam = oracle.lame(rng.uniform(1e4, 1e6, m), rng.uniform(0.3, 0.49, m))
    g = oracle.stretch_gradient(s, mod, mu, lam)
    H = oracle.stretch_hessian(s, mod, mu, lam, clamp=False)
    g_fd = np.zeros_like(g)
    H_fd = np.zeros_like(H)
    for c in range(6):
        h = 1e-6 * np.maximum(1.0, np.abs(s[:, c]))
        sp, sm = s.copy(), s.copy()
        sp[:, c] += h
        sm[:, c] -= h
        g_fd[:, c] = (oracle.psi(oracle.unvech(sp), mod, mu, lam)
                      - oracle.psi(oracle.unvech(sm), mod, mu, lam)) / (2 * h)
        H_fd[:, :, c] = (oracle.stretch_gradient(sp, mod, mu, lam)
                         - oracle.stretch_gradient(sm, mod, mu, lam)) / (2 * h)[:, None]
    gscale = np.abs(g).max(axis=1, keepdims=True) + mu[:, None] * 1e-3
    assert np.max(np.abs(g - g_fd) / gscale) < 1e-6
    Hscale = np.abs(H).max(axis=(1, 2), keepdims=True)
    assert np.max(np.abs(H - H_fd) / Hscale) < 1e-6
    # the Hessian is symmetric
    assert np.allclose(H, np.transpose(H, (0, 2, 1)), rtol=0, atol=1e-9 * Hscale.max())


def test_clamped_hessian_is_psd_and_matches_unclamped_when_inactive():
    rng = np.random.default_rng(3)
    m = 64
    S = _rand_spd(rng, m, 0.35) * rng.uniform(0.8, 1.4, (m, 1, 1))
    s = oracle.vech(S)
    mod = np.full(m, NH, dtype=np.int32)
    mu, lam = oracle.lame(np.full(m, 1e5), np.full(m, 0.45))
    Hc = oracle.stretch_hessian(s, mod, mu, lam, clamp=True)
    Hu = oracle.stretch_hessian(s, mod, mu, lam, clamp=False)
    lnJ = np.log(np.linalg.det(S))
    active = mu - lam * lnJ < 0
    assert active.any() and (~active).any()
    assert np.allclose(Hc[~active], Hu[~active], rtol=0, atol=0)
    assert np.all(np.linalg.eigvalsh(Hc).min(axis=1) > -1e-9 * np.abs(Hc).max())


# --------------------------------------------------------------------------
# P2: closed forms at S = I (the linear-elasticity tensor).
# --------------------------------------------------------------------------
def test_closed_forms_at_identity():
    m = 3
    s = np.tile([1.0, 1.0, 1.0, 0.0, 0.0, 0.0], (m, 1))
    mu = np.array([1.0, 2.5, 7.0])
    lam = np.array([3.0, 0.5, 11.0])
    ones = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
    metric = np.diag([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])
    for model in MODELS:
        mod = np.full(m, model, dtype=np.int32)
        assert np.all(oracle.stretch_gradient(s, mod, mu, lam) == 0.0)
        H = oracle.stretch_hessian(s, mod, mu, lam)
        for k in range(m):
            want = 2 * mu[k] * metric
            if model != ARAP:
                want = want + lam[k] * np.outer(ones, ones)
            assert np.allclose(H[k], want, rtol=1e-15, atol=1e-15)
        assert np.all(oracle.psi(np.tile(np.eye(3), (m, 1, 1)), mod, mu, lam) == 0.0)


# --------------------------------------------------------------------------
# P3: F = B x against Ds Dm^-1, and the pseudo-inverse of the 9x6 rotation
# block against the closed form sym(R^T F).
# --------------------------------------------------------------------------
def test_deformation_operator_and_pseudo_inverse():
    rng = np.random.default_rng(11)
    prob = tiny_mesh("cube")
    X, T = prob["X"], prob["T"].astype(np.int64)
    x = X + rng.normal(scale=0.2, size=X.shape)
    G, W = oracle.rest_shape(X, T)
    F_direct = np.stack([np.column_stack([x[t[1]] - x[t[0]], x[t[2]] - x[t[0]],
                                          x[t[3]] - x[t[0]]])
                         @ np.linalg.inv(np.column_stack([X[t[1]] - X[t[0]], X[t[2]] - X[t[0]],
                                                          X[t[3]] - X[t[0]]]))
                         for t in T])
    B = oracle.deformation_operator(G)
    xl = x[T].reshape(len(T), 12)
    F_op = np.einsum("krj,kj->kr", B, xl).reshape(-1, 3, 3)
    assert np.allclose(F_op, F_direct, rtol=0, atol=1e-13)
    vol = np.array([abs(np.linalg.det(np.column_stack([X[t[1]] - X[t[0]], X[t[2]] - X[t[0]],
                                                        X[t[3]] - X[t[0]]]))) / 6 for t in T])
    assert np.allclose(W, vol, rtol=1e-15) and abs(W.sum() - 1.0) < 1e-14
    Rk = _rand_rot(rng, len(T))
    J = oracle.mixed_operator(Rk, G)
    s = np.einsum("kcj,kj->kc", J, xl)
    RtF = np.einsum("kji,kjl->kil", Rk, F_direct)
    sym = 0.5 * (RtF + np.transpose(RtF, (0, 2, 1)))
    want = np.stack([sym[:, 0, 0], sym[:, 1, 1], sym[:, 2, 2], sym[:, 1, 2], sym[:, 0, 2],
                     sym[:, 0, 1]], axis=1)
    assert np.allclose(s, want, rtol=0, atol=1e-13)
    # R_k maps s to vec(R S): check one column by hand
    Rop = oracle.rotation_operator(Rk)
    E01 = np.zeros((3, 3))
    E01[0, 1] = E01[1, 0] = 1.0
    assert np.allclose(Rop[0][:, 5], (Rk[0] @ E01).reshape(-1), atol=1e-15)


def test_degenerate_rest_tet_rejected():
    X = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0.5, 0.5, 0.0]])
    with pytest.raises(oracle.DegenerateElement):
        oracle.rest_shape(X, np.array([[0, 1, 2, 3]]))


# --------------------------------------------------------------------------
# Whole-energy gradient and Hessian vs finite differences of E (assembly).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["one", "cube"])
def test_energy_gradient_and_hessian_match_finite_differences(kind):
    rng = np.random.default_rng(5)
    prob = tiny_mesh(kind, model=NH, youngs=1e3, poisson=0.4, pin_stiffness=50.0)
    prob["model"] = np.array([MODELS[k % 3] for k in range(len(prob["T"]))], dtype=np.int32)
    R = _rand_rot(rng, 2) * 0 + np.stack([np.eye(3), euler_xyz(0.3, -0.2, 0.25)])
    t = rng.normal(scale=0.1, size=(2, 3))
    fr = oracle.Frame(prob, (R, t))
    x = fr.X.reshape(-1) + rng.normal(scale=0.03, size=3 * fr.n)
    assert fr.feasible(x)
    g = fr.gradient(x)
    K = fr.hessian(fr.stretch(x), clamp=False).toarray()
    h = 1e-6
    g_fd = np.zeros_like(g)
    K_fd = np.zeros_like(K)
    for i in range(3 * fr.n):
        e = np.zeros_like(x)
        e[i] = h
        g_fd[i] = (fr.energy(x + e) - fr.energy(x - e)) / (2 * h)
        K_fd[:, i] = (fr.gradient(x + e) - fr.gradient(x - e)) / (2 * h)
    assert np.max(np.abs(g - g_fd)) < 1e-6 * np.abs(g).max()
    assert np.max(np.abs(K - K_fd)) < 1e-6 * np.abs(K).max()
    assert np.allclose(K, K.T, atol=1e-10 * np.abs(K).max())


# --------------------------------------------------------------------------
# P4: the condensed step equals a dense solve of the full KKT Newton system.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["one", "cube"])
def test_condensed_step_equals_bruteforce_kkt(kind):
    rng = np.random.default_rng(17)
    prob = tiny_mesh(kind, model=NH, youngs=2e3, poisson=0.45, pin_stiffness=300.0)
    prob["model"] = np.array([MODELS[(k + 2) % 3] for k in range(len(prob["T"]))], dtype=np.int32)
    R = np.stack([euler_xyz(0.1, 0.2, -0.3), euler_xyz(0.7, -0.4, 0.2)])
    t = rng.normal(scale=0.2, size=(2, 3))
    fr = oracle.Frame(prob, (R, t))
    m, n = fr.m, fr.n
    x = fr.X.reshape(-1) + rng.normal(scale=0.05, size=3 * n)
    s = oracle.vech(_rand_spd(rng, m, 0.2))        # mixed variable off the constraint
    # condensed (oracle)
    dx = np.linalg.solve(fr.hessian(s).toarray(), -fr.gradient(x, s_lin=s))
    # brute force: unknowns (ds, dx, lambda); L = sum W (Psi(s) + lambda.(J x - s)) + C(x)
    g = oracle.stretch_gradient(s, fr.model, fr.mu, fr.lam)
    H = oracle.stretch_hessian(s, fr.model, fr.mu, fr.lam)
    Jg = np.zeros((6 * m, 3 * n))
    for k in range(m):
        Jg[6 * k:6 * k + 6][:, fr.dof[k]] += fr.J[k]
    Wd = np.kron(np.diag(fr.W), np.eye(6))
    Hs = np.zeros((6 * m, 6 * m))
    for k in range(m):
        Hs[6 * k:6 * k + 6, 6 * k:6 * k + 6] = fr.W[k] * H[k]
    HC = np.zeros((3 * n, 3 * n))
    gC = np.zeros(3 * n)
    for p, v in enumerate(fr.pin_vertex):
        HC[3 * v:3 * v + 3, 3 * v:3 * v + 3] += fr.ks * np.eye(3)
        gC[3 * v:3 * v + 3] += fr.ks * (x[3 * v:3 * v + 3] - fr.y[p])
    Z = np.zeros
    KKT = np.block([[Hs, Z((6 * m, 3 * n)), -Wd],
                    [Z((3 * n, 6 * m)), HC, Jg.T @ Wd],
                    [-Wd, Wd @ Jg, Z((6 * m, 6 * m))]])
    rhs = np.concatenate([-(Wd @ g.reshape(-1)), -gC, -(Wd @ (Jg @ x - s.reshape(-1)))])
    sol = np.linalg.solve(KKT, rhs)
    dx_kkt = sol[6 * m:6 * m + 3 * n]
    assert np.allclose(dx, dx_kkt, rtol=0, atol=1e-10 * np.abs(dx).max())
    # the recovered stretch step closes the linearised constraint
    ds = sol[:6 * m]
    assert np.allclose(s.reshape(-1) + ds, Jg @ (x + dx_kkt), atol=1e-10)


# --------------------------------------------------------------------------
# P5/P6/P7/P9: invariants of the frame solve.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("model", MODELS)
def test_rest_pose_gives_zero_displacement(model):
    prob = beam(8, 2, 2, model=model)
    R = np.stack([np.eye(3)] * 2)
    t = np.zeros((2, 3))
    r = oracle.solve_frame(prob, (R, t), iterations=3)
    assert r["status"] == "ok"
    assert np.max(np.abs(r["x"] - prob["X"])) <= 1e-14 * prob["bbox_diag"]


@pytest.mark.parametrize("model", MODELS)
def test_rigid_handles_give_rigid_mesh(model):
    prob = beam(8, 2, 2, model=model, pin_stiffness=3e3)
    Q = euler_xyz(0.9, -0.6, 2.1)
    c = np.array([3.0, -1.0, 2.0])
    R = np.stack([Q, Q])
    t = np.stack([c, c])
    r = oracle.solve_frame(prob, (R, t), iterations=4)
    assert r["status"] == "ok"
    want = prob["X"] @ Q.T + c
    assert np.max(np.abs(r["x"] - want)) <= 1e-13 * prob["bbox_diag"]


@pytest.mark.parametrize("model", [ARAP, COROT])
def test_quadratic_materials_need_one_solve(model):
    prob = beam(8, 2, 2, model=model, youngs=1e5, poisson=0.45)
    r = oracle.solve_frame(prob, beam_pose(prob, 60.0, (1.0, 0.5, 0.0)), iterations=3)
    assert r["status"] == "ok" and r["alpha"][0] == 1.0
    assert r["step"][1] <= 1e-12 * prob["bbox_diag"]


def test_posed_space_equivariance():
    prob = humanoid(31, target_tets=3000, n_bones=15)
    R, t = random_pose(prob, 32)
    Q = euler_xyz(0.4, 1.1, -0.7)
    c = np.array([0.5, -2.0, 1.0])
    r1 = oracle.solve_frame(prob, (R, t))
    r2 = oracle.solve_frame(prob, (np.einsum("ij,hjk->hik", Q, R), t @ Q.T + c),
                            x0=prob["X"] @ Q.T + c)
    assert r1["status"] == "ok" and r2["status"] == "ok"
    assert np.max(np.abs(r1["x"] @ Q.T + c - r2["x"])) <= 1e-9 * prob["bbox_diag"]


# --------------------------------------------------------------------------
# P8: Newton-phase energies never increase; the result is stationary; the
# unclamped Hessian at the result is positive semidefinite.
# --------------------------------------------------------------------------
def test_beam_neohookean_converges_monotonically():
    prob = beam()
    pose = beam_pose(prob)
    r = oracle.solve_frame(prob, pose, iterations=10)
    assert r["status"] == "ok"
    E = [e for e, ph in zip(r["energy"], r["phase"] + ["newton"]) if ph == "newton"]
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(E[:-1], E[1:]))
    first = r["phase"].index("newton")
    assert r["grad_norm"][-1] <= 1e-9 * r["grad_norm"][first]
    fr = oracle.Frame(prob, pose)
    x = r["x"].reshape(-1)
    K = fr.hessian(fr.stretch(x), clamp=False).toarray()
    ev = np.linalg.eigvalsh(K)
    assert ev.min() > -1e-10 * ev.max()
    # dense and sparse linear solves agree (P11)
    rd = oracle.solve_frame(prob, pose, iterations=10, linear_solver="dense")
    assert np.max(np.abs(rd["x"] - r["x"])) <= 1e-12 * prob["bbox_diag"]


def test_humanoid_mixed_phase_reaches_feasible_stationary_point():
    prob = humanoid(21, target_tets=4000, n_bones=15)
    pose = random_pose(prob, 22)
    r = oracle.solve_frame(prob, pose)
    assert r["status"] == "ok"
    assert r["phase"][0] == "mixed" and r["phase"][-1] == "newton"
    fr = oracle.Frame(prob, pose)
    x = r["x"].reshape(-1)
    assert fr.feasible(x)
    assert np.allclose(r["s"], fr.stretch(x), atol=1e-12)
    first = r["phase"].index("newton")
    assert r["grad_norm"][-1] <= 1e-8 * r["grad_norm"][first]
    E = r["energy"][first:]
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(E[:-1], E[1:]))


# --------------------------------------------------------------------------
# P10: polar decomposition vs scipy.linalg.polar.
# --------------------------------------------------------------------------
def test_polar_matches_scipy():
    rng = np.random.default_rng(9)
    F = rng.normal(size=(50, 3, 3))
    F[np.linalg.det(F) < 0, :, 0] *= -1.0
    U, P = oracle.polar(F)
    for k in range(len(F)):
        u, p = scipy.linalg.polar(F[k])
        assert np.allclose(U[k], u, atol=1e-12) and np.allclose(P[k], p, atol=1e-12)
    assert np.allclose(np.einsum("kji,kjl->kil", U, U), np.eye(3), atol=1e-14)
    assert np.allclose(np.linalg.det(U), 1.0, atol=1e-14)
    assert np.allclose(U @ P, F, atol=1e-13)
    assert np.all(np.linalg.eigvalsh(P) > 0)
    # inverted F: proper rotation, and the warm-start stretch falls back to I
    Fi = F.copy()
    Fi[:, :, 0] *= -1.0
    Ui, Pi = oracle.polar(Fi)
    assert np.allclose(np.linalg.det(Ui), 1.0) and np.allclose(Ui @ Pi, Fi, atol=1e-13)
    assert np.all(oracle.polar_stretch(Fi) == np.array([1.0, 1, 1, 0, 0, 0]))


# --------------------------------------------------------------------------
# P12: rotation clusters vs a brute-force loop.
# --------------------------------------------------------------------------
def test_clusters_match_bruteforce():
    prob = humanoid(11, target_tets=600, n_bones=9)
    cl = oracle.cluster_by_segments(prob["X"], prob["T"], prob["seg_a"], prob["seg_b"],
                                    prob["seg_handle"])
    X = prob["X"]
    for k, tet in enumerate(prob["T"]):
        c = sum(X[v] for v in tet) / 4.0
        best, arg = np.inf, -1
        for sidx, (a, b) in enumerate(zip(prob["seg_a"], prob["seg_b"])):
            # closest point by dense sampling refined with the exact projection
            d = b - a
            u = 0.0 if d @ d == 0 else min(1.0, max(0.0, (c - a) @ d / (d @ d)))
            samples = [a + w * d for w in np.linspace(0, 1, 41)] + [a + u * d]
            dist = min(np.linalg.norm(c - q) for q in samples)
            if dist < best - 1e-12:
                best, arg = dist, sidx
        assert cl[k] == prob["seg_handle"][arg]
    # beam: tets left of the middle take handle 0, right of it handle 1
    bm = beam()
    cb = oracle.cluster_by_segments(bm["X"], bm["T"], bm["seg_a"], bm["seg_b"], bm["seg_handle"])
    bx = bm["X"][bm["T"]].mean(axis=1)[:, 0]
    assert np.array_equal(cb, (bx > 8).astype(np.int32))


def test_interpolate_pose_is_the_matrix_exponential_screw():
    """Load-stepping poses: T(tau) = T0 expm(tau logm(T0^-1 T1)) on 4x4
    homogeneous matrices (scipy's general matrix exp/log), the one-parameter
    subgroup property (T0^-1 T(1/2))^2 = T0^-1 T1, and a handle rotated
    about a fixed point keeps that point fixed at every tau."""
    import scipy.linalg as sla
    from workloads.common import euler_xyz
    rng = np.random.default_rng(11)
    nh = 5
    R0 = np.stack([euler_xyz(*rng.uniform(-1.0, 1.0, 3)) for _ in range(nh)])
    t0 = rng.normal(size=(nh, 3))
    R1 = np.stack([euler_xyz(*rng.uniform(-1.2, 1.2, 3)) for _ in range(nh)])
    t1 = rng.normal(size=(nh, 3))
    # handle 0: relative motion is a pure rotation about the point c
    c = np.array([0.3, -0.7, 1.1])
    Rrel = R1[0] @ R0[0].T
    t1[0] = Rrel @ (t0[0] - c) + c  # T1 = Rot_c o T0  =>  T1 (T0^-1 c) = c
    def hom(R, t):
        M = np.eye(4)
        M[:3, :3], M[:3, 3] = R, t
        return M
    for tau in (0.0, 0.25, 0.5, 0.8125, 1.0):
        R, t = oracle.interpolate_pose((R0, t0), (R1, t1), tau)
        for h in range(nh):
            T0, T1 = hom(R0[h], t0[h]), hom(R1[h], t1[h])
            ref = T0 @ np.real(sla.expm(tau * sla.logm(np.linalg.solve(T0, T1))))
            assert np.abs(hom(R[h], t[h]) - ref).max() < 1e-10
        # the rotation centre of handle 0 stays where T0 put its preimage
        p = np.linalg.solve(R0[0], c - t0[0])
        assert np.abs(R[0] @ p + t[0] - c).max() < 1e-10
    Rh, th = oracle.interpolate_pose((R0, t0), (R1, t1), 0.5)
    for h in range(nh):
        A = np.linalg.solve(hom(R0[h], t0[h]), hom(Rh[h], th[h]))
        B = np.linalg.solve(hom(R0[h], t0[h]), hom(R1[h], t1[h]))
        assert np.abs(A @ A - B).max() < 1e-10


def test_external_forces_gradient_and_superposition():
    """External vertex forces (-f . x in E): the gradient matches central
    differences of E, and for a quadratic (co-rotated) energy the response
    superposes exactly: x*(f_a + f_b) - x*(0) = (x*(f_a) - x*(0)) + (x*(f_b) - x*(0))."""
    from workloads import beam, beam_pose
    rng = np.random.default_rng(5)
    prob = dict(beam(8, 2, 2, model=oracle.COROT))
    pose = beam_pose(prob, 20.0)
    n = len(prob["X"])
    va = rng.choice(n, 4, replace=False)
    fa = rng.normal(scale=1e3, size=(4, 3))
    vb = np.concatenate([va[:2], rng.choice(n, 3, replace=False)])
    fb = rng.normal(scale=1e3, size=(5, 3))
    # gradient vs central differences at a perturbed state
    pf = dict(prob, force_vertex=va, force=fa)
    fr = oracle.Frame(pf, pose)
    x = prob["X"].reshape(-1) + rng.normal(scale=1e-3, size=3 * n)
    g = fr.gradient(x)
    for _ in range(4):  # directional derivatives (E ~ 1e7: componentwise steps lose to roundoff)
        d = rng.normal(size=3 * n)
        d /= np.linalg.norm(d)
        h = 1e-4
        fd = (fr.energy(x + h * d) - fr.energy(x - h * d)) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * np.linalg.norm(g)
    # the force term alone: E(x) - E_without(x) = -f . x
    fr0 = oracle.Frame(prob, pose)
    fx = np.zeros((n, 3))
    np.add.at(fx, va, fa)
    assert abs((fr.energy(x) - fr0.energy(x)) + float((fx.reshape(-1) * x).sum())) <= 1e-9 * abs(fr0.energy(x))
    # superposition (quadratic energy: one Newton step reaches x*)
    def sol(fv, ff):
        p = dict(prob, force_vertex=fv, force=ff) if fv is not None else prob
        r = oracle.solve_frame(p, pose, step_tol=1e-13, linear_solver="dense")
        assert r["status"] == "ok"
        return r["x"]
    x0 = sol(None, None)
    xa = sol(va, fa)
    xb = sol(vb, fb)
    xab = sol(np.concatenate([va, vb]), np.concatenate([fa, fb]))
    lhs, rhs = xab - x0, (xa - x0) + (xb - x0)
    assert np.max(np.abs(lhs - rhs)) <= 1e-9 * np.max(np.abs(lhs))
    assert np.max(np.abs(xa - x0)) > 1e-6 * prob["bbox_diag"]  # the forces do move the beam


def test_stress_recovery_balances_element_forces():
    """Stress recovery: the multipliers lambda_k = W_k R_k P_k, applied as
    vertex forces lambda_k n_a, sum to the element part of grad E (the oracle
    computes that gradient through J_k^T g_k, a different route); P_k equals
    2 mu (S - I) for ARAP; NaN marks infeasible neo-Hookean tets."""
    from workloads import humanoid, random_pose
    rng = np.random.default_rng(9)
    prob = humanoid(31, target_tets=1500, n_bones=10, models=(oracle.NH, oracle.ARAP))
    pose = random_pose(prob, 32, amp_deg=25)
    fr = oracle.Frame(prob, pose)
    x0 = oracle.solve_frame(prob, pose, iterations=4)["x"].reshape(-1, 3)
    x = x0 + rng.normal(scale=1e-4 * prob["bbox_diag"], size=x0.shape)
    assert fr.feasible(x)
    P6, lam = oracle.stress(prob, pose, x)
    G, W = oracle.rest_shape(prob["X"], prob["T"])
    n = oracle.shape_gradients(G)  # (m, 4, 3) rest-frame gradients of the shape functions
    forces = np.zeros((len(prob["X"]), 3))
    np.add.at(forces, prob["T"], np.einsum("kij,kaj->kai", lam, n))
    pin = np.zeros_like(forces)
    np.add.at(pin, fr.pin_vertex, fr.ks * fr.pin_residual(x))
    g_elem = fr.gradient(x).reshape(-1, 3) - pin
    assert np.max(np.abs(forces - g_elem)) <= 1e-10 * np.max(np.abs(g_elem))
    arap = fr.model == oracle.ARAP
    S = oracle.unvech(fr.stretch(x))
    assert np.allclose(oracle.unvech(P6[arap]), 2 * fr.mu[arap, None, None] * (S[arap] - np.eye(3)), rtol=0, atol=1e-9 * fr.mu.max())
    # an inverted neo-Hookean tet gives NaN
    xb = x.copy()
    k = int(np.flatnonzero(fr.model == oracle.NH)[0])
    a, b = prob["T"][k][:2]
    xb[[a, b]] = xb[[b, a]]
    P6b, _ = oracle.stress(prob, pose, xb)
    assert np.all(np.isnan(P6b[k]))


def _axis_rot(axis, ang):
    axis = np.asarray(axis, dtype=np.float64) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def test_blend_rotations_closed_form_about_one_axis():
    """Rotation smoothing (R15): blending rotations about one axis by angles a
    and b with weights w, 1 - w gives the rotation by arg(w e^{ia} + (1-w) e^{ib})
    about that axis (the in-plane part is a scaled rotation); one handle
    reproduces its rotation; the result is a proper rotation."""
    rng = np.random.default_rng(3)
    axis = rng.normal(size=3)
    cases = [(0.3, -0.5, 0.5), (1.1, 0.2, 0.25), (-0.7, 0.9, 0.8), (2.0, 2.6, 0.6)]
    R = np.stack([_axis_rot(axis, a) for a, _, _ in cases] + [_axis_rot(axis, b) for _, b, _ in cases])
    nc = len(cases)
    handles = np.array([[i, nc + i] for i in range(nc)] + [[i, -1] for i in range(nc)], dtype=np.int32)
    weights = np.array([[w, 1 - w] for _, _, w in cases] + [[1.0, 0.0]] * nc)
    U = oracle.blend_rotations(R, handles, weights)
    for i, (a, b, w) in enumerate(cases):
        ang = np.angle(w * np.exp(1j * a) + (1 - w) * np.exp(1j * b))
        assert np.allclose(U[i], _axis_rot(axis, ang), atol=1e-13)
        assert np.allclose(U[nc + i], R[i], atol=1e-15)
    assert np.allclose(np.einsum("kji,kjl->kil", U, U), np.eye(3), atol=1e-13)
    assert np.all(np.linalg.det(U) > 0)
    # a blend with det <= 0 keeps the first handle's rotation
    Rb = np.stack([np.eye(3), np.diag([1.0, -1.0, -1.0]), np.diag([-1.0, 1.0, -1.0])])
    Ub = oracle.blend_rotations(Rb, np.array([[0, 1, 2], [1, 0, 2]], dtype=np.int32),
                                np.array([[0.2, 0.4, 0.4], [0.4, 0.2, 0.4]]))
    assert np.array_equal(Ub[0], np.eye(3)) and np.array_equal(Ub[1], Rb[1])


def test_blend_weights_brute_force_and_cluster_limit():
    """blend_weights against a per-tet brute force written from its
    definition on a small mesh with several segments per handle, and the
    cluster rule in the limit of zero width."""
    from workloads import humanoid
    prob = humanoid(61, target_tets=600, n_bones=6)
    X, T = prob["X"], prob["T"]
    sa, sb, sh = prob["seg_a"], prob["seg_b"], prob["seg_handle"]
    width = 0.3
    H, Wt = oracle.blend_weights(X, T, sa, sb, sh, width, 3)
    bary = X[T].mean(axis=1)
    def dist(p, a, b):
        a, b = np.asarray(a, float), np.asarray(b, float)
        d = b - a
        u = 0.0 if d @ d == 0 else min(1.0, max(0.0, (p - a) @ d / (d @ d)))
        return float(np.linalg.norm(p - (a + u * d)))
    for k in range(0, len(T), 7):
        ds = [dist(bary[k], sa[s], sb[s]) for s in range(len(sa))]
        s0 = int(np.argmin(ds))
        per_h = {}
        for s, d in enumerate(ds):
            per_h[int(sh[s])] = min(per_h.get(int(sh[s]), np.inf), d)
        h0 = int(sh[s0])
        others = sorted(((1 - (d - ds[s0]) / width, h) for h, d in per_h.items() if h != h0 and d - ds[s0] < width),
                        key=lambda c: (-c[0], c[1]))[:2]
        exp_h = [h0] + [h for _, h in others]
        exp_w = np.array([1.0] + [w for w, _ in others])
        exp_w /= exp_w.sum()
        got_h = [h for h in H[k] if h >= 0]
        assert got_h == exp_h, (k, got_h, exp_h)
        assert np.allclose(Wt[k, :len(exp_h)], exp_w, rtol=0, atol=1e-12)
        assert np.all(Wt[k, len(exp_h):] == 0)
    H0, W0 = oracle.blend_weights(X, T, sa, sb, sh, 0.0, 3)
    assert np.array_equal(H0[:, 0], oracle.cluster_by_segments(X, T, sa, sb, sh))
    assert np.all(W0[:, 0] == 1.0) and np.all(H0[:, 1:] == -1)


def test_smoothed_rotations_rigid_pose_and_zero_width():
    """A frame with smoothed rotations: a rigid pose (every handle at the same
    transform) still gives the rigidly moved rest shape, and zero blend width
    gives exactly the cluster frame's solution."""
    prob = humanoid(63, target_tets=1200, n_bones=8)
    H, Wt = oracle.blend_weights(prob["X"], prob["T"], prob["seg_a"], prob["seg_b"], prob["seg_handle"], 0.4, 3)
    assert np.any(H[:, 1] >= 0)  # some tets blend
    pb = dict(prob, blend_handles=H, blend_weights=Wt)
    nh = prob["n_handles"]
    Q = euler_xyz(0.5, -0.3, 1.2)
    c = np.array([0.2, 1.0, -0.5])
    r = oracle.solve_frame(pb, (np.stack([Q] * nh), np.stack([c] * nh)), iterations=4)
    assert r["status"] == "ok"
    assert np.max(np.abs(r["x"] - (prob["X"] @ Q.T + c))) <= 1e-12 * prob["bbox_diag"]
    pose = random_pose(prob, 64, amp_deg=20)
    H0, W0 = oracle.blend_weights(prob["X"], prob["T"], prob["seg_a"], prob["seg_b"], prob["seg_handle"], 0.0, 3)
    r0 = oracle.solve_frame(dict(prob, blend_handles=H0, blend_weights=W0), pose, iterations=3)
    rc = oracle.solve_frame(prob, pose, iterations=3)
    assert np.array_equal(r0["x"], rc["x"])
    rs = oracle.solve_frame(pb, pose, iterations=3)
    assert np.max(np.abs(rs["x"] - rc["x"])) > 1e-6 * prob["bbox_diag"]  # smoothing changes the frame


# --------------------------------------------------------------------------
# Lame parameters (reading R6): the values of the 1536-tet beam's material
# (E = 1e5, nu = 0.45), and a uniaxial-stress test through the co-rotated
# element, whose small-strain response is isotropic linear elasticity: with
# the lateral stresses zero, stress / axial strain must be E and the lateral
# contraction nu.
# --------------------------------------------------------------------------
def test_lame_values_and_uniaxial_stress():
    mu, lam = oracle.lame(np.array([1e5]), np.array([0.45]))
    assert abs(mu[0] - 34482.75862068966) <= 1e-9 * 34482.75862068966
    assert abs(lam[0] - 310344.8275862069) <= 1e-9 * 310344.8275862069
    assert abs(lam[0] / mu[0] - 9.0) <= 1e-12
    rng = np.random.default_rng(11)
    E = rng.uniform(1e3, 1e7, 8)
    nu = np.concatenate([[0.0, 0.25, 0.3, 0.49, 0.499], rng.uniform(-0.9, 0.49, 3)])
    mu, lam = oracle.lame(E, nu)
    mod = np.full(len(E), COROT, dtype=np.int32)
    # diagonal strain e -> diagonal stress P_ii = g_i(I + diag(e)); linear for
    # the co-rotated energy, so unit strains give its 3x3 stiffness columns
    C = np.zeros((len(E), 3, 3))
    for j in range(3):
        s = np.tile([1.0, 1.0, 1.0, 0.0, 0.0, 0.0], (len(E), 1))
        s[:, j] += 1.0
        C[:, :, j] = oracle.stretch_gradient(s, mod, mu, lam)[:, :3]
    for k in range(len(E)):
        # axial strain 1, lateral strains (l, l) with zero lateral stress
        lat = np.linalg.solve(C[k, 1:, 1:], -C[k, 1:, 0])
        axial_stress = C[k, 0, 0] + C[k, 0, 1:] @ lat
        assert abs(axial_stress - E[k]) <= 1e-11 * E[k]
        assert np.allclose(-lat, nu[k], rtol=0, atol=1e-12)


# --------------------------------------------------------------------------
# Mixed-phase step rule (reading R10): the accepted step is the largest
# halving of 1 that keeps every neo-Hookean s + alpha ds positive definite
# (checked by eigenvalues, not the oracle's Sylvester test), and there is no
# energy test: E(x) may even leave the feasible set during the mixed phase.
# --------------------------------------------------------------------------
def test_mixed_step_is_largest_feasible_halving():
    prob = humanoid(21, target_tets=4000, n_bones=15)
    for seed, finite_then_infinite in ((25, False), (22, True)):
        pose = random_pose(prob, seed)
        r = oracle.solve_frame(prob, pose, iterations=2)
        assert r["phase"] == ["mixed", "mixed"]
        fr = oracle.Frame(prob, pose)
        nh = fr.model == NH
        x = fr.X.reshape(-1).copy()
        s = oracle.polar_stretch(fr.deformation_gradient(x))
        for it in range(2):
            dx = oracle.mfem._linear_solve(fr.hessian(s), -fr.gradient(x, s_lin=s), "splu")
            ds = fr.stretch(x + dx) - s
            a = r["alpha"][it]

            def min_eig(alpha):
                return np.linalg.eigvalsh(oracle.unvech((s + alpha * ds)[nh])).min()
            assert a > 0.0 and math.log2(a) == round(math.log2(a))
            assert min_eig(a) > 0.0
            assert a == 1.0 or min_eig(2.0 * a) <= 0.0
            x = x + a * dx
            s = s + a * ds
        assert np.allclose(x.reshape(-1, 3), r["x"], rtol=0, atol=1e-12 * prob["bbox_diag"])
        # the step rule ignores E(x): the rest shape is infeasible for these
        # poses, and in one of them the second mixed step goes from a finite
        # E(x1) to E(x2) = +inf
        assert r["energy"][0] == np.inf
        if finite_then_infinite:
            assert np.isfinite(r["energy"][1]) and r["energy"][2] == np.inf
