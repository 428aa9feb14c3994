// Newton-iteration kernels: mixed warm start, element pass, Schur-complement
// assembly, line-search evaluations and updates.  All reductions are per
// tile in a fixed order (no atomics); a finalize kernel folds each system's
// tiles in a fixed order as well, so results do not depend on the batch.
#include "common.h"
#include "elem_math.h"
#include "launch.h"

namespace mfs {

__device__ __forceinline__ void load_rot(const double* __restrict__ Rh, int h, double R[9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) R[i] = Rh[9 * h + i];
}

// The rotation of tet k: its smoothed rotation when the character blends
// rotations across cluster boundaries, else its cluster handle's rotation.
__device__ __forceinline__ void tet_rot(const SysDesc& S, int k, int info, double R[9]) {
  if (S.Rt) {
#pragma unroll
    for (int i = 0; i < 9; ++i) R[i] = S.Rt[(size_t)i * S.m + k];
  } else {
    load_rot(S.Rh, info & 0xffff, R);
  }
}

__device__ __forceinline__ void gather4(const double* __restrict__ x, int4 t, double out[4][3]) {
  const int v[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) out[a][i] = x[3 * v[a] + i];
}

// ---------------------------------------------------------------------------
// Mixed warm start: s0_k = stretch factor of the polar decomposition of
// F_k(x0) (identity when det F <= 0).  FP32 mode runs the iteration in FP32
// and re-routes tets whose smallest singular value is below 1e-3 to FP64;
// the routed count goes to the P_ROUTED partial plane.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_warm_start(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
                                                       int ntiles, int fp32) {
  __shared__ double red[4];
  const Tile t = tiles[xcd_tile(blockIdx.x, ntiles)];
  const SysDesc& S = sd[t.sys];
  const int k = t.begin + threadIdx.x;
  double routed = 0.0;
  if (k < t.end) {
    double x[4][3], n[4][3], F[9];
    gather4(S.x, S.tets[k], x);
    load_grads(S.G, S.m, k, n);
    deformation_gradient(x, n, F);
    double U[9], P[6], sm;
    bool done = false;
    if (fp32) {
      float Ff[9], Uf[9], Pf[6], smf;
#pragma unroll
      for (int i = 0; i < 9; ++i) Ff[i] = (float)F[i];
      const bool ok = polar_newton<float>(Ff, Uf, Pf, &smf);
      if (!ok || smf >= 1e-3f) {
        done = true;
#pragma unroll
        for (int i = 0; i < 6; ++i) P[i] = ok ? (double)Pf[i] : (i < 3 ? 1.0 : 0.0);
      }
    }
    if (!done) {
      polar_newton<double>(F, U, P, &sm);
      routed = fp32 ? 1.0 : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) S.s[(size_t)i * S.m + k] = P[i];
  }
  const double tot = block_sum(routed, red);
  if (threadIdx.x == 0) S.part[P_ROUTED * S.ptile + t.local] = tot;
}

// ---------------------------------------------------------------------------
// Element pass (per Newton iteration).  For each tet: F = sum_a x_a n_a^T,
// condensed stretch sx = sym(R^T F), then the material linearised at
// sl = s (mixed phase, the stored mixed variable) or sl = sx (Newton phase).
// Writes the tet's record: its 10 unique world-frame Hessian blocks
// (precision T) and its four corner forces (FP64), and in the Newton phase
// s = sx.  World frame: p_a = R n_a, Tw = R S_lin^-1 R^T, q_a = Tw p_a, and
// the corner force R (W P) n_a = (R W P R^T) p_a.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_element(const SysDesc* __restrict__ sd, const Ctrl* __restrict__ ctrl,
                                                    const Tile* __restrict__ tiles, int ntiles) {
  __shared__ double red[4];
  const Tile t = tiles[xcd_tile(blockIdx.x, ntiles)];
  const SysDesc& S = sd[t.sys];
  const bool mixed = ctrl[t.sys].phase == 0;
  const int k = t.begin + threadIdx.x;
  double clamped = 0.0;
  if (k < t.end) {
    const size_t m = S.m;
    const int info = S.info[k];
    const int model = info >> 16;
    double R[9], x[4][3], n[4][3], F[9], sx[6], sl[6];
    tet_rot(S, k, info, R);
    gather4(S.x, S.tets[k], x);
    load_grads(S.G, S.m, k, n);
    deformation_gradient(x, n, F);
    rotated_stretch(R, F, sx);
    if (mixed) {
#pragma unroll
      for (int i = 0; i < 6; ++i) sl[i] = S.s[i * m + k];
    } else {
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        sl[i] = sx[i];
        S.s[i * m + k] = sx[i];
      }
    }
    double WP[6], Ti[6], c[4];
    clamped = element_state(model, S.wmu[k], S.wlam[k], sl, sx, WP, Ti, c) ? 1.0 : 0.0;
    const bool nh = model == kNeoHookean;
    double p[4][3], q[4][3], Tw[6] = {0, 0, 0, 0, 0, 0}, Pw[6];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i) p[a][i] = R[3 * i] * n[a][0] + R[3 * i + 1] * n[a][1] + R[3 * i + 2] * n[a][2];
    if (nh) sym_rotate(R, Ti, Tw);
#pragma unroll
    for (int a = 0; a < 4; ++a) sym_mv(Tw, p[a], q[a]);
    sym_rotate(R, WP, Pw);
    double* fr = S.frc + 12 * (size_t)k;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      double f[3];
      sym_mv(Pw, p[a], f);
#pragma unroll
      for (int i = 0; i < 3; ++i) fr[3 * a + i] = f[i];
    }
    T* bk = (T*)S.blk + 90 * (size_t)k;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = a; b < 4; ++b) {
        double K[9];
        world_block(p[a], p[b], q[a], q[b], Tw, c, nh, K);
        const int pi = pair_index(a, b);
#pragma unroll
        for (int i = 0; i < 9; ++i) bk[9 * pi + i] = (T)K[i];
      }
  }
  const double tot = block_sum(clamped, red);
  if (threadIdx.x == 0) S.part[P_CLAMP * S.ptile + t.local] = tot;
}

// ---------------------------------------------------------------------------
// Assembly of the condensed system (eq. 12 read as a Newton increment):
//   K = k_s P^T P + sum_k W_k J_k^T H_k J_k,  b = -grad C - sum_k W_k J_k^T g_k + f_ext,
// gathered per 3x3 block slot from the slot's list of (tet, a, b)
// contributions (no atomics); each contribution is one block of the tet's
// record (transposed when a > b).  The diagonal slot of vertex r also adds
// the pins of r, writes b_r and the inverse diagonal block (block Jacobi).
// Contributions are taken in batches of kBatch: the batch's codes, then all
// its blocks (and forces), are loaded before any is added, so a batch costs
// two dependent memory latencies instead of two per contribution (a
// diagonal slot has about twenty); they are still added in list order.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_assemble(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
                                                     int ntiles) {
  const Tile t = tiles[xcd_tile(blockIdx.x, ntiles)];
  const SysDesc& S = sd[t.sys];
  const int slot = t.begin + threadIdx.x;
  if (slot >= t.end) return;
  const T* blk = (const T*)S.blk;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double f[3] = {0, 0, 0};
  const int c0 = S.slot_ptr[slot], c1 = S.slot_ptr[slot + 1];  // c1 > c0: every slot has a contribution
  const int code0 = S.contrib[c0];
  const int a0 = (code0 >> 2) & 3;
  const bool diag = a0 == (code0 & 3);
  constexpr int kBatch = 4;
  for (int cb = c0; cb < c1; cb += kBatch) {
    int code[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) code[u] = S.contrib[cb + u < c1 ? cb + u : c1 - 1];  // past the end: reload the last
    T v[kBatch][9];
    double fr[kBatch][3];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int k = code[u] >> 4, a = (code[u] >> 2) & 3, b = code[u] & 3;
      const T* bp = blk + 90 * (size_t)k + 9 * pair_index(a <= b ? a : b, a <= b ? b : a);
#pragma unroll
      for (int i = 0; i < 9; ++i) v[u][i] = bp[i];
      if (diag) {
        const double* fp = S.frc + 12 * (size_t)k + 3 * a;
#pragma unroll
        for (int i = 0; i < 3; ++i) fr[u][i] = fp[i];
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      if (cb + u >= c1) break;
      const int a = (code[u] >> 2) & 3, b = code[u] & 3;
      if (a <= b) {
#pragma unroll
        for (int i = 0; i < 9; ++i) acc[i] += (double)v[u][i];
      } else {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) acc[3 * i + j] += (double)v[u][3 * j + i];
      }
      if (diag) {
#pragma unroll
        for (int i = 0; i < 3; ++i) f[i] += fr[u][i];
      }
    }
  }
  if (diag) {
    const int4 tv = S.tets[code0 >> 4];
    const int v[4] = {tv.x, tv.y, tv.z, tv.w};
    const int row = v[a0];
    // pins of this vertex: stiffness k_s I each, target R_h X_r + t_h
    double cnt = 0.0, ys[3] = {0, 0, 0};
    for (int pi = S.vpin_ptr[row]; pi < S.vpin_ptr[row + 1]; ++pi) {
      const int h = S.vpin_h[pi];
      double R[9];
      load_rot(S.Rh, h, R);
      cnt += 1.0;
#pragma unroll
      for (int i = 0; i < 3; ++i)
        ys[i] += R[3 * i] * S.X[3 * row] + R[3 * i + 1] * S.X[3 * row + 1] + R[3 * i + 2] * S.X[3 * row + 2] +
                 S.th[3 * h + i];
    }
    const double kc = S.ks * cnt;
    acc[0] += kc;
    acc[4] += kc;
    acc[8] += kc;
#pragma unroll
    for (int i = 0; i < 3; ++i)
      S.b[3 * row + i] = -f[i] - (kc * S.x[3 * row + i] - S.ks * ys[i]) + (S.fext ? S.fext[3 * row + i] : 0.0);
    // inverse of the symmetrised diagonal block
    double d6[6] = {acc[0], acc[4], acc[8], 0.5 * (acc[5] + acc[7]), 0.5 * (acc[2] + acc[6]),
                    0.5 * (acc[1] + acc[3])};
    double inv[6];
    sym_inv(d6, sym_det(d6), inv);
    T* mi = (T*)S.minv;
#pragma unroll
    for (int i = 0; i < 6; ++i) mi[6 * row + i] = (T)inv[i];
  }
  store_block((T*)S.vals, slot, acc, S.colidx[slot]);
}

// ---------------------------------------------------------------------------
// Line search, Newton phase: element energies at x + alpha_i dx for the
// trial step lengths of this pass, with neo-Hookean feasibility.
// Mixed phase: the number of halvings h (0..41) each neo-Hookean tet needs
// for s + 2^-h (sym(R^T F(x + dx)) - s) to be positive definite; the step is
// the one needed by the worst tet (the positive-definite set is convex and
// contains s, so every smaller step stays feasible).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_linesearch_tets(const SysDesc* __restrict__ sd,
                                                            const Ctrl* __restrict__ ctrl,
                                                            const Tile* __restrict__ tiles, int ntiles) {
  __shared__ double red[4];
  const Tile t = tiles[xcd_tile(blockIdx.x, ntiles)];
  const SysDesc& S = sd[t.sys];
  const Ctrl& C = ctrl[t.sys];
  const int k = t.begin + threadIdx.x;
  const bool valid = k < t.end;
  double s0[6] = {0, 0, 0, 0, 0, 0}, s1[6] = {0, 0, 0, 0, 0, 0};
  int model = 0;
  double wmu = 0.0, wlam = 0.0;
  if (valid) {
    const int info = S.info[k];
    model = info >> 16;
    wmu = S.wmu[k];
    wlam = S.wlam[k];
    double R[9], x[4][3], d[4][3], n[4][3], F[9];
    const int4 tv = S.tets[k];
    tet_rot(S, k, info, R);
    load_grads(S.G, S.m, k, n);
    gather4(S.x, tv, x);
    gather4(S.dx, tv, d);
    deformation_gradient(x, n, F);
    rotated_stretch(R, F, s0);
    deformation_gradient(d, n, F);
    rotated_stretch(R, F, s1);
  }
  if (C.phase == 0) {
    double h = 0.0;
    if (valid && model == kNeoHookean) {
      double sm[6], ds[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        sm[i] = S.s[(size_t)i * S.m + k];
        ds[i] = (s0[i] + s1[i]) - sm[i];
      }
      double a = 1.0;
      int hh = 0;
      for (; hh <= 40; ++hh, a *= 0.5) {
        double st[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) st[i] = sm[i] + a * ds[i];
        if (sym_spd(st)) break;
      }
      h = (double)hh;
    }
    const double hm = block_max(h, red);
    if (threadIdx.x == 0) S.part[P_HMAX * S.ptile + t.local] = hm;
    return;
  }
#pragma unroll
  for (int j = 0; j < kNumTrials; ++j) {
    double e = 0.0, inf = 0.0;
    if (valid) {
      double st[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) st[i] = s0[i] + C.trials[j] * s1[i];
      bool ok;
      const double v = element_energy(model, wmu, wlam, st, &ok);
      if (ok) e = v; else inf = 1.0;
    }
    const double es = block_sum(e, red);
    const double is = block_sum(inf, red);
    if (threadIdx.x == 0) {
      S.part[(P_E0 + j) * S.ptile + t.local] = es;
      S.part[(P_INF0 + j) * S.ptile + t.local] = is;
    }
  }
}

// Vertex part of the line search: b . dx, max_v |dx_v| and the pin energy
// k_s/2 |x_r + alpha_i dx_r - (R_h X_r + t_h)|^2 at each trial step.
__global__ __launch_bounds__(64) void k_linesearch_verts(const SysDesc* __restrict__ sd,
                                                         const Ctrl* __restrict__ ctrl,
                                                         const Tile* __restrict__ tiles, int ntiles) {
  const Tile t = tiles[xcd_tile(blockIdx.x, ntiles)];
  const SysDesc& S = sd[t.sys];
  const Ctrl& C = ctrl[t.sys];
  const int r = t.begin + threadIdx.x;
  double slope = 0.0, dmax = 0.0, pe[kNumTrials];
#pragma unroll
  for (int j = 0; j < kNumTrials; ++j) pe[j] = 0.0;
  if (r < t.end) {
    double x[3], d[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      x[i] = S.x[3 * r + i];
      d[i] = S.dx[3 * r + i];
      slope += S.b[3 * r + i] * d[i];
    }
    dmax = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int pi = S.vpin_ptr[r]; pi < S.vpin_ptr[r + 1]; ++pi) {
      const int h = S.vpin_h[pi];
      double R[9], y[3];
      load_rot(S.Rh, h, R);
#pragma unroll
      for (int i = 0; i < 3; ++i)
        y[i] = R[3 * i] * S.X[3 * r] + R[3 * i + 1] * S.X[3 * r + 1] + R[3 * i + 2] * S.X[3 * r + 2] + S.th[3 * h + i];
#pragma unroll
      for (int j = 0; j < kNumTrials; ++j) {
        double e2 = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const double e = x[i] + C.trials[j] * d[i] - y[i];
          e2 += e * e;
        }
        pe[j] += 0.5 * S.ks * e2;
      }
    }
    if (S.fext) {  // potential of the external forces, -f . x
      const double f0 = S.fext[3 * r], f1 = S.fext[3 * r + 1], f2 = S.fext[3 * r + 2];
#pragma unroll
      for (int j = 0; j < kNumTrials; ++j)
        pe[j] -= f0 * (x[0] + C.trials[j] * d[0]) + f1 * (x[1] + C.trials[j] * d[1]) + f2 * (x[2] + C.trials[j] * d[2]);
    }
  }
  const double ss = wave_sum(slope);
  const double dm = wave_max(dmax);
  if (threadIdx.x == 0) {
    S.part[P_SLOPE * S.ptile + t.local] = ss;
    S.part[P_DXMAX * S.ptile + t.local] = dm;
  }
#pragma unroll
  for (int j = 0; j < kNumTrials; ++j) {
    const double ps = wave_sum(pe[j]);
    if (threadIdx.x == 0) S.part[(P_PIN0 + j) * S.ptile + t.local] = ps;
  }
}

// Mixed-phase stretch update s <- s + alpha (sym(R^T F(x + dx)) - s), run
// before the position update (it reads the old x).
__global__ __launch_bounds__(kBlock) void k_update_s(const SysDesc* __restrict__ sd, const Ctrl* __restrict__ ctrl,
                                                     const Tile* __restrict__ tiles, int ntiles) {
  const Tile t = tiles[xcd_tile(blockIdx.x, ntiles)];
  const SysDesc& S = sd[t.sys];
  const Ctrl& C = ctrl[t.sys];
  const int k = t.begin + threadIdx.x;
  if (C.phase != 0 || C.update_s == 0 || k >= t.end) return;
  const int info = S.info[k];
  double R[9], x[4][3], n[4][3], F[9], sx[6];
  const int4 tv = S.tets[k];
  tet_rot(S, k, info, R);
  load_grads(S.G, S.m, k, n);
  gather4(S.x, tv, x);
  double d[4][3];
  gather4(S.dx, tv, d);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) x[a][i] += d[a][i];
  deformation_gradient(x, n, F);
  rotated_stretch(R, F, sx);
  const size_t m = S.m;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const double so = S.s[i * m + k];
    S.s[i * m + k] = so + C.alpha * (sx[i] - so);
  }
}

__global__ __launch_bounds__(64) void k_update_x(const SysDesc* __restrict__ sd, const Ctrl* __restrict__ ctrl,
                                                     const Tile* __restrict__ tiles, int ntiles) {
  const Tile t = tiles[xcd_tile(blockIdx.x, ntiles)];
  const SysDesc& S = sd[t.sys];
  const double a = ctrl[t.sys].alpha;
  const int r = t.begin + threadIdx.x;
  if (r >= t.end || a == 0.0) return;
#pragma unroll
  for (int i = 0; i < 3; ++i) S.x[3 * r + i] += a * S.dx[3 * r + i];
}

// Fold each system's partial planes over its tiles (fixed order): one
// workgroup per system, one wave per plane.
constexpr int kFinalizeThreads = 512;
__global__ __launch_bounds__(kFinalizeThreads) void k_finalize(const SysDesc* __restrict__ sd,
                                                              const int32_t* __restrict__ sys_ids) {
  const SysDesc& S = sd[sys_ids[blockIdx.x]];
  // the pipelined-PCG planes (from P_G0 on) are folded by the PCG kernels
  for (int p = threadIdx.x >> 6; p < P_G0; p += kFinalizeThreads / 64) {
    const bool vert = (p == P_PQ || p == P_RZ0 || p == P_RZ1 || p == P_RR || p == P_BB || p == P_SLOPE ||
                       p == P_DXMAX || (p >= P_PIN0 && p < P_PIN0 + kNumTrials));
    const int cnt = vert ? S.ntv : S.ntt;
    const double* plane = S.part + (size_t)p * S.ptile;
    const double v = (p == P_DXMAX || p == P_HMAX) ? sys_max(plane, cnt) : sys_sum(plane, cnt);
    if ((threadIdx.x & 63) == 0) S.red[p] = v;
  }
}

// ---------------------------------------------------------------------------
// Stress recovery at positions x (FP64): per tet, the stress P = dPsi/dS at
// S = sym(R^T F(x)) and the volume-weighted world-frame multiplier
// lambda = W R P of the constraint F = R S (Section 3: at a solution the
// stretch equations give W dPsi/ds = [R]^T lambda, and the element's vertex
// forces are lambda n_a).  Written in the caller's tet order; infeasible
// neo-Hookean elements give NaN.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_stress(const SysDesc* __restrict__ sd, const int32_t* __restrict__ tperm,
                                                   double* __restrict__ P6, double* __restrict__ L9) {
  const SysDesc& S = sd[0];
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= S.m) return;
  const int4 tv = S.tets[k];
  const int vi[4] = {tv.x, tv.y, tv.z, tv.w};
  double n[4][3], xv[4][3];
  load_grads(S.G, S.m, k, n);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) xv[a][i] = S.x[3 * vi[a] + i];
  double F[9], R[9], sx[6];
  deformation_gradient(xv, n, F);
  const int info = S.info[k];
  const int model = info >> 16;
  tet_rot(S, k, info, R);
  rotated_stretch(R, F, sx);
  const bool ok = model != kNeoHookean || sym_spd(sx);
  double WP[6] = {0, 0, 0, 0, 0, 0}, T[6], c[4];
  if (ok) element_state(model, S.wmu[k], S.wlam[k], sx, sx, WP, T, c);
  // W = |det Dm| / 6 = 1 / (6 |det G|), G = Dm^-1 with rows n_1..n_3
  const double Gm[9] = {n[1][0], n[1][1], n[1][2], n[2][0], n[2][1], n[2][2], n[3][0], n[3][1], n[3][2]};
  const double W = 1.0 / (6.0 * fabs(det3(Gm)));
  const int o = tperm[k];
  const double nan = __builtin_nan("");
  if (P6) {
#pragma unroll
    for (int i = 0; i < 6; ++i) P6[6 * (size_t)o + i] = ok ? WP[i] / W : nan;
  }
  if (L9) {
    double Pf[9];
    sym_full(WP, Pf);  // W P
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        L9[9 * (size_t)o + 3 * i + j] =
            ok ? R[3 * i] * Pf[j] + R[3 * i + 1] * Pf[3 + j] + R[3 * i + 2] * Pf[6 + j] : nan;
  }
}

// ---- launchers ----
void launch_warm_start(hipStream_t st, const SysDesc* sd, const Tile* tiles, int ntiles, int fp32) {
  if (ntiles) MFS_LAUNCH(k_warm_start, dim3(ntiles), dim3(kBlock), 0, st, sd, tiles, ntiles, fp32);
}
void launch_element(hipStream_t st, const SysDesc* sd, const Ctrl* ctrl, const Tile* tiles, int ntiles, int fp32) {
  if (!ntiles) return;
  if (fp32)
    MFS_LAUNCH(k_element<float>, dim3(ntiles), dim3(kBlock), 0, st, sd, ctrl, tiles, ntiles);
  else
    MFS_LAUNCH(k_element<double>, dim3(ntiles), dim3(kBlock), 0, st, sd, ctrl, tiles, ntiles);
}
void launch_assemble(hipStream_t st, const SysDesc* sd, const Tile* tiles, int ntiles, int fp32) {
  if (!ntiles) return;
  if (fp32)
    MFS_LAUNCH(k_assemble<float>, dim3(ntiles), dim3(kBlock), 0, st, sd, tiles, ntiles);
  else
    MFS_LAUNCH(k_assemble<double>, dim3(ntiles), dim3(kBlock), 0, st, sd, tiles, ntiles);
}
void launch_linesearch(hipStream_t st, const SysDesc* sd, const Ctrl* ctrl, const Tile* tt, int ntt, const Tile* tv,
                       int ntv) {
  if (ntt) MFS_LAUNCH(k_linesearch_tets, dim3(ntt), dim3(kBlock), 0, st, sd, ctrl, tt, ntt);
  if (ntv) MFS_LAUNCH(k_linesearch_verts, dim3(ntv), dim3(64), 0, st, sd, ctrl, tv, ntv);
}
void launch_update(hipStream_t st, const SysDesc* sd, const Ctrl* ctrl, const Tile* tt, int ntt, const Tile* tv,
                   int ntv) {
  if (ntt) MFS_LAUNCH(k_update_s, dim3(ntt), dim3(kBlock), 0, st, sd, ctrl, tt, ntt);
  if (ntv) MFS_LAUNCH(k_update_x, dim3(ntv), dim3(64), 0, st, sd, ctrl, tv, ntv);
}
void launch_stress(hipStream_t st, const SysDesc* sd, int m, const int32_t* tperm, double* P6, double* L9) {
  if (m > 0) MFS_LAUNCH(k_stress, dim3((m + kBlock - 1) / kBlock), dim3(kBlock), 0, st, sd, tperm, P6, L9);
}
void launch_finalize(hipStream_t st, const SysDesc* sd, const int32_t* sys_ids, int nsys) {
  if (nsys) MFS_LAUNCH(k_finalize, dim3(nsys), dim3(kFinalizeThreads), 0, st, sd, sys_ids);
}

}  // namespace mfs
