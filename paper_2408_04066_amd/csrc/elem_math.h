// Per-element math of the mixed-FEM skinning solve (device, header-only).
//
// Notation.  For tet k with rest shape-gradient matrix G = Dm^-1 (rows are
// the gradients n_1..n_3 of the linear shape functions, n_0 = -(n_1+n_2+n_3))
// and deformed vertices x_0..x_3, the deformation gradient is
// F = sum_a x_a n_a^T.  The rig fixes the tet's rotation R (its cluster's
// handle), and the condensed stretch is S = sym(R^T F): the least-squares
// solution of F = R S, which is the pseudo-inverse of the 9x6 rotation block
// applied to F (Section 3, text after the condensed system).  Symmetric 3x3
// matrices are stored as 6-vectors (S00, S11, S22, S12, S02, S01).
//
// The Hessian of W Psi(S(x)) with respect to vertex a (row) and b (column) is
// R Kt_ab R^T, where in the rotated frame
//   Kt_ab = cI [(n_a.n_b) I + n_b n_a^T] + c2 n_a n_b^T
//         + c3 [(T n_b)(T n_a)^T + (n_a . T n_b) T] + c4 (T n_a)(T n_b)^T,
// with T = S^-1 and the coefficients of each material listed at
// element_state().  The force on vertex a is R (W P) n_a with W P the
// (linearised) stress.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace mfs {

enum Material : int { kArap = 0, kCorot = 1, kNeoHookean = 2 };

// ---- small symmetric / general 3x3 helpers (row-major 9, symmetric 6) ----

template <typename R>
__device__ __forceinline__ R det3(const R a[9]) {
  return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
         a[2] * (a[3] * a[7] - a[4] * a[6]);
}

// Full 3x3 from the 6-vector.
template <typename R>
__device__ __forceinline__ void sym_full(const R s[6], R a[9]) {
  a[0] = s[0]; a[4] = s[1]; a[8] = s[2];
  a[5] = a[7] = s[3];
  a[2] = a[6] = s[4];
  a[1] = a[3] = s[5];
}

template <typename R>
__device__ __forceinline__ R sym_det(const R s[6]) {
  return s[0] * (s[1] * s[2] - s[3] * s[3]) - s[5] * (s[5] * s[2] - s[3] * s[4]) +
         s[4] * (s[5] * s[3] - s[1] * s[4]);
}

// Inverse of a symmetric matrix via the adjugate.
template <typename R>
__device__ __forceinline__ void sym_inv(const R s[6], R det, R t[6]) {
  const R id = R(1) / det;
  t[0] = (s[1] * s[2] - s[3] * s[3]) * id;
  t[1] = (s[0] * s[2] - s[4] * s[4]) * id;
  t[2] = (s[0] * s[1] - s[5] * s[5]) * id;
  t[3] = (s[5] * s[4] - s[0] * s[3]) * id;
  t[4] = (s[5] * s[3] - s[1] * s[4]) * id;
  t[5] = (s[4] * s[3] - s[5] * s[2]) * id;
}

// Sylvester's criterion: leading principal minors positive.
template <typename R>
__device__ __forceinline__ bool sym_spd(const R s[6]) {
  return s[0] > R(0) && (s[0] * s[1] - s[5] * s[5]) > R(0) && sym_det(s) > R(0);
}

// y = A v for symmetric A.
template <typename R>
__device__ __forceinline__ void sym_mv(const R s[6], const R v[3], R y[3]) {
  y[0] = s[0] * v[0] + s[5] * v[1] + s[4] * v[2];
  y[1] = s[5] * v[0] + s[1] * v[1] + s[3] * v[2];
  y[2] = s[4] * v[0] + s[3] * v[1] + s[2] * v[2];
}

// A : B for symmetric 6-vectors (Frobenius).
template <typename R>
__device__ __forceinline__ R sym_ddot(const R a[6], const R b[6]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + R(2) * (a[3] * b[3] + a[4] * b[4] + a[5] * b[5]);
}

// T D T for symmetric T, D (result symmetric).
__device__ __forceinline__ void sym_sandwich(const double t[6], const double d[6], double out[6]) {
  double T[9], D[9], TD[9];
  sym_full(t, T);
  sym_full(d, D);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      TD[3 * i + j] = T[3 * i] * D[j] + T[3 * i + 1] * D[3 + j] + T[3 * i + 2] * D[6 + j];
  // (TD) T, only the six unique entries
  auto e = [&](int i, int j) {
    return TD[3 * i] * T[j] + TD[3 * i + 1] * T[3 + j] + TD[3 * i + 2] * T[6 + j];
  };
  out[0] = e(0, 0); out[1] = e(1, 1); out[2] = e(2, 2);
  out[3] = e(1, 2); out[4] = e(0, 2); out[5] = e(0, 1);
}

// ---- tet geometry ----

// Shape-function gradients n_0..n_3 (rest frame) from the 9 planes of G.
__device__ __forceinline__ void load_grads(const double* __restrict__ G, int m, int k, double n[4][3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) n[r + 1][c] = G[(3 * r + c) * (size_t)m + k];
#pragma unroll
  for (int c = 0; c < 3; ++c) n[0][c] = -(n[1][c] + n[2][c] + n[3][c]);
}

// F = sum_a x_a n_a^T (row-major).
__device__ __forceinline__ void deformation_gradient(const double x[4][3], const double n[4][3], double F[9]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      F[3 * i + j] = x[0][i] * n[0][j] + x[1][i] * n[1][j] + x[2][i] * n[2][j] + x[3][i] * n[3][j];
}

// s = vech(sym(R^T F)).
__device__ __forceinline__ void rotated_stretch(const double R[9], const double F[9], double s[6]) {
  double A[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) A[3 * i + j] = R[i] * F[j] + R[3 + i] * F[3 + j] + R[6 + i] * F[6 + j];
  s[0] = A[0];
  s[1] = A[4];
  s[2] = A[8];
  s[3] = 0.5 * (A[5] + A[7]);
  s[4] = 0.5 * (A[2] + A[6]);
  s[5] = 0.5 * (A[1] + A[3]);
}

// ---- materials ----

// W Psi(S); returns false (and +inf) for an infeasible neo-Hookean stretch.
__device__ __forceinline__ double element_energy(int model, double wmu, double wlam, const double s[6],
                                                 bool* feasible) {
  *feasible = true;
  if (model != kNeoHookean) {
    const double d0 = s[0] - 1.0, d1 = s[1] - 1.0, d2 = s[2] - 1.0;
    const double dev = d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]);
    const double tr = d0 + d1 + d2;
    return model == kArap ? wmu * dev : wmu * dev + 0.5 * wlam * tr * tr;
  }
  if (!sym_spd(s)) {
    *feasible = false;
    return INFINITY;
  }
  const double lnJ = log(sym_det(s));
  const double trSS = s[0] * s[0] + s[1] * s[1] + s[2] * s[2] + 2.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]);
  return 0.5 * wmu * (trSS - 3.0) - wmu * lnJ + 0.5 * wlam * lnJ * lnJ;
}

// Linearised stress and Hessian coefficients of one element.
//   sl: stretch the material is linearised at (SPD for neo-Hookean);
//   sx: current condensed stretch sym(R^T F(x)).
// Outputs (all premultiplied by the volume W):
//   WP = W [dPsi/dS(sl) + H(sl)[sx - sl]]   (the mixed-predictor stress; equal
//        to W dPsi/dS(sx) when sl = sx or Psi is quadratic),
//   T  = sl^-1 (neo-Hookean, else 0),
//   c  = {cI, c2, c3, c4}:
//     ARAP:        {W mu,   0,        0,            0}
//     co-rotated:  {W mu,   W lambda, 0,            0}
//     neo-Hookean: {W mu/2, 0,        W chat/2,     W lambda},
//   chat = max(mu - lambda ln J, 0) (Hessian clamp; the stress is not
//   clamped).  Returns true when the clamp is active.
__device__ __forceinline__ bool element_state(int model, double wmu, double wlam, const double sl[6],
                                              const double sx[6], double WP[6], double T[6], double c[4]) {
  if (model != kNeoHookean) {
    const double tr = (sx[0] - 1.0) + (sx[1] - 1.0) + (sx[2] - 1.0);
    const double lt = model == kCorot ? wlam * tr : 0.0;
    WP[0] = 2.0 * wmu * (sx[0] - 1.0) + lt;
    WP[1] = 2.0 * wmu * (sx[1] - 1.0) + lt;
    WP[2] = 2.0 * wmu * (sx[2] - 1.0) + lt;
    WP[3] = 2.0 * wmu * sx[3];
    WP[4] = 2.0 * wmu * sx[4];
    WP[5] = 2.0 * wmu * sx[5];
#pragma unroll
    for (int i = 0; i < 6; ++i) T[i] = 0.0;
    c[0] = wmu;
    c[1] = model == kCorot ? wlam : 0.0;
    c[2] = 0.0;
    c[3] = 0.0;
    return false;
  }
  const double J = sym_det(sl);
  sym_inv(sl, J, T);
  const double lnJ = log(J);
  const double craw = wmu - wlam * lnJ;
  const double chat = craw > 0.0 ? craw : 0.0;
  double d[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) d[i] = sx[i] - sl[i];
  double TdT[6];
  sym_sandwich(T, d, TdT);
  const double trTd = T[0] * d[0] + T[1] * d[1] + T[2] * d[2] + 2.0 * (T[3] * d[3] + T[4] * d[4] + T[5] * d[5]);
  const double a = wlam * lnJ - wmu + wlam * trTd;
#pragma unroll
  for (int i = 0; i < 6; ++i) WP[i] = wmu * sl[i] + a * T[i] + wmu * d[i] + chat * TdT[i];
  c[0] = 0.5 * wmu;
  c[1] = 0.0;
  c[2] = 0.5 * chat;
  c[3] = wlam;
  return craw < 0.0;
}

// Rotated-frame block Kt_ab (row-major 9) from the state of one element.
__device__ __forceinline__ void element_block(const double na[3], const double nb[3], const double T[6],
                                              const double c[4], double K[9]) {
  const double dab = na[0] * nb[0] + na[1] * nb[1] + na[2] * nb[2];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) K[3 * i + j] = c[0] * nb[i] * na[j] + c[1] * na[i] * nb[j];
  K[0] += c[0] * dab;
  K[4] += c[0] * dab;
  K[8] += c[0] * dab;
  if (c[2] != 0.0 || c[3] != 0.0) {
    double ma[3], mb[3], Tf[9];
    sym_mv(T, na, ma);
    sym_mv(T, nb, mb);
    sym_full(T, Tf);
    const double amb = na[0] * mb[0] + na[1] * mb[1] + na[2] * mb[2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        K[3 * i + j] += c[2] * (mb[i] * ma[j] + amb * Tf[3 * i + j]) + c[3] * ma[i] * mb[j];
  }
}

// Index of the unique block (a, b), a <= b, among the 10 blocks of a tet:
// (0,0) (0,1) (0,2) (0,3) (1,1) (1,2) (1,3) (2,2) (2,3) (3,3).
__host__ __device__ constexpr int pair_index(int a, int b) { return a * 4 - (a * (a - 1)) / 2 + (b - a); }

// R S R^T for symmetric S (6-vector in, 6-vector out).
__device__ __forceinline__ void sym_rotate(const double R[9], const double s[6], double out[6]) {
  double S[9], RS[9];
  sym_full(s, S);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) RS[3 * i + j] = R[3 * i] * S[j] + R[3 * i + 1] * S[3 + j] + R[3 * i + 2] * S[6 + j];
  auto e = [&](int i, int j) { return RS[3 * i] * R[3 * j] + RS[3 * i + 1] * R[3 * j + 1] + RS[3 * i + 2] * R[3 * j + 2]; };
  out[0] = e(0, 0); out[1] = e(1, 1); out[2] = e(2, 2);
  out[3] = e(1, 2); out[4] = e(0, 2); out[5] = e(0, 1);
}

// World-frame block K_ab = R Kt_ab R^T written with the rotated shape
// gradients p = R n, q = (R T R^T) p and Tw = R T R^T:
//   K_ab = cI [(p_a.p_b) I + p_b p_a^T] + c2 p_a p_b^T
//        + c3 [q_b q_a^T + (p_a . q_b) Tw] + c4 q_a q_b^T.
__device__ __forceinline__ void world_block(const double pa[3], const double pb[3], const double qa[3],
                                            const double qb[3], const double Tw[6], const double c[4],
                                            bool nh, double K[9]) {
  const double dab = pa[0] * pb[0] + pa[1] * pb[1] + pa[2] * pb[2];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) K[3 * i + j] = c[0] * pb[i] * pa[j] + c[1] * pa[i] * pb[j];
  K[0] += c[0] * dab;
  K[4] += c[0] * dab;
  K[8] += c[0] * dab;
  if (nh) {
    double Tf[9];
    sym_full(Tw, Tf);
    const double aqb = pa[0] * qb[0] + pa[1] * qb[1] + pa[2] * qb[2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        K[3 * i + j] += c[2] * (qb[i] * qa[j] + aqb * Tf[3 * i + j]) + c[3] * qa[i] * qb[j];
  }
}

// K <- R K R^T
__device__ __forceinline__ void rotate_block(const double R[9], const double Kt[9], double K[9]) {
  double RK[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) RK[3 * i + j] = R[3 * i] * Kt[j] + R[3 * i + 1] * Kt[3 + j] + R[3 * i + 2] * Kt[6 + j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) K[3 * i + j] = RK[3 * i] * R[3 * j] + RK[3 * i + 1] * R[3 * j + 1] + RK[3 * i + 2] * R[3 * j + 2];
}

// ---- polar decomposition: Higham's scaled Newton iteration (1986) ----
//
// U_{k+1} = (zeta U_k + U_k^{-T} / zeta) / 2 with the Frobenius-norm scaling
// zeta = sqrt(|U_k^-1|_F / |U_k|_F), switched off once the update is below
// 1e-2 so the last steps converge quadratically.  For det F > 0 the limit is
// the proper rotation of F = U P; P = sym(U^T F).  The smallest singular value
// is the smallest eigenvalue of P, from the trigonometric closed form for
// symmetric 3x3 eigenvalues (Smith 1961).
template <typename R>
__device__ __forceinline__ R sym_eig_min(const R s[6]) {
  const R q = (s[0] + s[1] + s[2]) / R(3);
  const R p1 = s[3] * s[3] + s[4] * s[4] + s[5] * s[5];
  const R a0 = s[0] - q, a1 = s[1] - q, a2 = s[2] - q;
  const R p2 = a0 * a0 + a1 * a1 + a2 * a2 + R(2) * p1;
  if (p2 <= R(0)) return q;
  const R p = sqrt(p2 / R(6));
  const R ip = R(1) / p;
  R b[6] = {a0 * ip, a1 * ip, a2 * ip, s[3] * ip, s[4] * ip, s[5] * ip};
  R r = sym_det(b) / R(2);
  r = r < R(-1) ? R(-1) : (r > R(1) ? R(1) : r);
  const R phi = acos(r) / R(3);
  return q + R(2) * p * cos(phi + R(2.0943951023931954923));  // + 2 pi / 3
}

template <typename R>
__device__ __forceinline__ bool polar_newton(const R F[9], R U[9], R P[6], R* smin) {
  const R d = det3(F);
  if (!(d > R(0))) {
#pragma unroll
    for (int i = 0; i < 9; ++i) U[i] = (i % 4 == 0) ? R(1) : R(0);
    P[0] = P[1] = P[2] = R(1);
    P[3] = P[4] = P[5] = R(0);
    *smin = R(0);
    return false;
  }
  const R eps = sizeof(R) == 8 ? R(2.220446049250313e-16) : R(1.1920929e-07);
#pragma unroll
  for (int i = 0; i < 9; ++i) U[i] = F[i];
  bool scale = true;
  for (int it = 0; it < 30; ++it) {
    const R du = det3(U);
    // U^-T = cofactor(U) / det(U)
    R C[9];
    C[0] = U[4] * U[8] - U[5] * U[7];
    C[1] = U[5] * U[6] - U[3] * U[8];
    C[2] = U[3] * U[7] - U[4] * U[6];
    C[3] = U[2] * U[7] - U[1] * U[8];
    C[4] = U[0] * U[8] - U[2] * U[6];
    C[5] = U[1] * U[6] - U[0] * U[7];
    C[6] = U[1] * U[5] - U[2] * U[4];
    C[7] = U[2] * U[3] - U[0] * U[5];
    C[8] = U[0] * U[4] - U[1] * U[3];
    R nu = 0, ni = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      C[i] /= du;
      nu += U[i] * U[i];
      ni += C[i] * C[i];
    }
    const R zeta = scale ? sqrt(sqrt(ni / nu)) : R(1);
    R diff = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const R un = R(0.5) * (zeta * U[i] + C[i] / zeta);
      diff += (un - U[i]) * (un - U[i]);
      U[i] = un;
    }
    diff = sqrt(diff);
    if (diff < R(1e-2)) scale = false;
    if (diff <= R(8) * eps) break;
  }
  // P = sym(U^T F)
  R A[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) A[3 * i + j] = U[i] * F[j] + U[3 + i] * F[3 + j] + U[6 + i] * F[6 + j];
  P[0] = A[0];
  P[1] = A[4];
  P[2] = A[8];
  P[3] = R(0.5) * (A[5] + A[7]);
  P[4] = R(0.5) * (A[2] + A[6]);
  P[5] = R(0.5) * (A[1] + A[3]);
  *smin = sym_eig_min(P);
  return true;
}

}  // namespace mfs
