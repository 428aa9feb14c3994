// Per-character setup kernels and standalone helpers: rest shape, rotation
// clusters, polar decomposition, and the vertex / tet permutations between
// the caller's order and the library's bandwidth-reduced order.
#include "common.h"
#include "elem_math.h"
#include "launch.h"

namespace mfs {

// Rest shape (Section 3: F = B x with B built from Dm^-1; element volumes
// W_k of the discrete mixed energy).  Dm = [X1-X0, X2-X0, X3-X0] as columns;
// G = Dm^-1 (rows are the shape-function gradients n_1..n_3); W = |det Dm|/6;
// Lame parameters mu = E / (2 (1 + nu)), lambda = E nu / ((1 + nu)(1 - 2 nu)).
// bad[k] = 1 when |det Dm| <= det_tol.
__global__ __launch_bounds__(kBlock) void k_rest(const int4* __restrict__ tets, const double* __restrict__ X,
                                                 const double* __restrict__ youngs,
                                                 const double* __restrict__ poisson, int m, double det_tol,
                                                 double* __restrict__ G, double* __restrict__ wmu,
                                                 double* __restrict__ wlam, uint8_t* __restrict__ bad) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= m) return;
  const int4 t = tets[k];
  const int v[4] = {t.x, t.y, t.z, t.w};
  double D[9];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int i = 0; i < 3; ++i) D[3 * i + c] = X[3 * v[c + 1] + i] - X[3 * v[0] + i];
  const double det = det3(D);
  bad[k] = fabs(det) <= det_tol ? 1 : 0;
  const double id = 1.0 / det;
  double inv[9];
  inv[0] = (D[4] * D[8] - D[5] * D[7]) * id;
  inv[1] = (D[2] * D[7] - D[1] * D[8]) * id;
  inv[2] = (D[1] * D[5] - D[2] * D[4]) * id;
  inv[3] = (D[5] * D[6] - D[3] * D[8]) * id;
  inv[4] = (D[0] * D[8] - D[2] * D[6]) * id;
  inv[5] = (D[2] * D[3] - D[0] * D[5]) * id;
  inv[6] = (D[3] * D[7] - D[4] * D[6]) * id;
  inv[7] = (D[1] * D[6] - D[0] * D[7]) * id;
  inv[8] = (D[0] * D[4] - D[1] * D[3]) * id;
#pragma unroll
  for (int i = 0; i < 9; ++i) G[(size_t)i * m + k] = inv[i];
  const double W = fabs(det) / 6.0;
  const double E = youngs[k], nu = poisson[k];
  wmu[k] = W * (E / (2.0 * (1.0 + nu)));
  wlam[k] = W * (E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)));
}

// Tet barycenter ((X0 + X1) + X2) + X3) / 4 and squared distance to bone
// segment sg (a zero-length segment is a point).
// The barycenter and the segment distance are evaluated in one written-out
// order with every product rounded on its own (contraction off): a tet as far
// from two segments as from their shared joint must tie exactly, so that the
// nearest-segment rule (ties to the lower segment) gives the same cluster as
// any other evaluation in this order.  With fused multiply-adds the two
// distances of such a tet can differ in the last bit either way.
__device__ __forceinline__ void tet_barycenter(const double* __restrict__ X, const int32_t* __restrict__ tets,
                                               int64_t k, double c[3]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int i = 0; i < 3; ++i)
    c[i] = (((X[3 * (int64_t)tets[4 * k] + i] + X[3 * (int64_t)tets[4 * k + 1] + i]) +
             X[3 * (int64_t)tets[4 * k + 2] + i]) +
            X[3 * (int64_t)tets[4 * k + 3] + i]) * 0.25;
}

__device__ __forceinline__ double segment_dist2(const double c[3], const double* __restrict__ sa,
                                                const double* __restrict__ sb, int sg) {
#pragma clang fp contract(off)
  double a[3], d[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    a[i] = sa[3 * sg + i];
    d[i] = sb[3 * sg + i] - a[i];
  }
  const double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  double u = 0.0;
  if (dd != 0.0) {
    u = ((c[0] - a[0]) * d[0] + (c[1] - a[1]) * d[1] + (c[2] - a[2]) * d[2]) / dd;
    u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
  }
  double e2 = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double e = c[i] - (a[i] + u * d[i]);
    e2 += e * e;
  }
  return e2;
}

// Rotation clusters (Section 3.1): handle of the bone segment nearest the
// tet barycenter; strict '<' keeps the lowest segment index on ties.
__global__ __launch_bounds__(kBlock) void k_cluster(const double* __restrict__ X, const int32_t* __restrict__ tets,
                                                    int64_t m, int nseg, const double* __restrict__ sa,
                                                    const double* __restrict__ sb,
                                                    const int32_t* __restrict__ sh, int32_t* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= m) return;
  double c[3];
  tet_barycenter(X, tets, k, c);
  double best = INFINITY;
  int arg = 0;
  for (int sg = 0; sg < nseg; ++sg) {
    const double e2 = segment_dist2(c, sa, sb, sg);
    if (e2 < best) {
      best = e2;
      arg = sg;
    }
  }
  out[k] = sh[arg];
}

// Rotation smoothing weights (the paper leaves smoothing across cluster
// boundaries to future work; this is one reading of it).  Per tet: the
// handle of the nearest segment (the cluster rule) with weight 1, then the
// other handles h whose nearest segment lies at d_h < d_min + width, with
// weight 1 - (d_h - d_min) / width, in decreasing weight (ties: lower handle
// first), at most kmax in all, divided by their sum.  Unused entries get
// handle -1 and weight 0.  Row-major outputs: out_h[kmax k + j].
constexpr int kMaxBlend = 4;
__global__ __launch_bounds__(kBlock) void k_blend_weights(const double* __restrict__ X,
                                                          const int32_t* __restrict__ tets, int64_t m, int nseg,
                                                          const double* __restrict__ sa,
                                                          const double* __restrict__ sb,
                                                          const int32_t* __restrict__ sh, int nh, double width,
                                                          int kmax, int32_t* __restrict__ out_h,
                                                          double* __restrict__ out_w) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= m) return;
  double c[3];
  tet_barycenter(X, tets, k, c);
  double best = INFINITY;
  int arg = 0;
  for (int sg = 0; sg < nseg; ++sg) {
    const double e2 = segment_dist2(c, sa, sb, sg);
    if (e2 < best) {
      best = e2;
      arg = sg;
    }
  }
  const int h0 = sh[arg];
  const double dmin = sqrt(best);
  double cw[kMaxBlend - 1];
  int ch[kMaxBlend - 1];
  int nc = 0;
  for (int h = 0; h < nh && width > 0.0; ++h) {
    if (h == h0) continue;
    double dh2 = INFINITY;
    for (int sg = 0; sg < nseg; ++sg)
      if (sh[sg] == h) dh2 = fmin(dh2, segment_dist2(c, sa, sb, sg));
    if (!(dh2 < INFINITY)) continue;  // a handle with no segment
    const double dh = sqrt(dh2);
    if (!(dh - dmin < width)) continue;
    const double w = 1.0 - (dh - dmin) / width;
    // insertion into the first kmax - 1 places, by weight then handle
    int pos = nc;
    while (pos > 0 && (w > cw[pos - 1] || (w == cw[pos - 1] && h < ch[pos - 1]))) --pos;
    if (pos >= kmax - 1) continue;
    const int last = nc < kmax - 1 ? nc : kmax - 2;
    for (int j = last; j > pos; --j) {
      cw[j] = cw[j - 1];
      ch[j] = ch[j - 1];
    }
    cw[pos] = w;
    ch[pos] = h;
    if (nc < kmax - 1) ++nc;
  }
  double total = 1.0;
  for (int j = 0; j < nc; ++j) total += cw[j];
  out_h[kmax * k] = h0;
  out_w[kmax * k] = 1.0 / total;
  for (int j = 1; j < kmax; ++j) {
    out_h[kmax * k + j] = j - 1 < nc ? ch[j - 1] : -1;
    out_w[kmax * k + j] = j - 1 < nc ? cw[j - 1] / total : 0.0;
  }
}

// Smoothed tet rotations for the current pose: R_k = polar(sum_j w_kj R_h),
// the handle rotation itself for a tet with one handle or a blend with
// det <= 0.  bh, bw: kmax planes of m; Rt: 9 planes of m.
__global__ __launch_bounds__(kBlock) void k_blend_rot(const double* __restrict__ Rh, int m, int kmax,
                                                      const int32_t* __restrict__ bh,
                                                      const double* __restrict__ bw, double* __restrict__ Rt) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= m) return;
  double M[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  int cnt = 0;
  for (int j = 0; j < kmax; ++j) {
    const int h = bh[(size_t)j * m + k];
    if (h < 0) continue;
    const double w = bw[(size_t)j * m + k];
#pragma unroll
    for (int i = 0; i < 9; ++i) M[i] += w * Rh[9 * h + i];
    ++cnt;
  }
  const int h0 = bh[k];
  double U[9];
  bool ok = false;
  if (cnt > 1 && det3(M) > 0.0) {
    double P[6], smin;
    ok = polar_newton(M, U, P, &smin);
  }
  if (!ok) {
#pragma unroll
    for (int i = 0; i < 9; ++i) U[i] = Rh[9 * h0 + i];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) Rt[(size_t)i * m + k] = U[i];
}


// Standalone polar decomposition (FP64, or FP32 with FP64 re-route).
__global__ __launch_bounds__(kBlock) void k_polar(const double* __restrict__ F, int64_t count, int fp32,
                                                  double* __restrict__ U, double* __restrict__ P,
                                                  double* __restrict__ smin, uint8_t* __restrict__ routed) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= count) return;
  double f[9], u[9], p[6], sm;
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = F[9 * k + i];
  bool r64 = true;
  if (fp32) {
    float ff[9], uf[9], pf[6], smf;
#pragma unroll
    for (int i = 0; i < 9; ++i) ff[i] = (float)f[i];
    const bool ok = polar_newton<float>(ff, uf, pf, &smf);
    if (ok && smf >= 1e-3f) {
      r64 = false;
#pragma unroll
      for (int i = 0; i < 9; ++i) u[i] = uf[i];
#pragma unroll
      for (int i = 0; i < 6; ++i) p[i] = pf[i];
      sm = smf;
    }
  }
  if (r64) polar_newton<double>(f, u, p, &sm);
#pragma unroll
  for (int i = 0; i < 9; ++i) U[9 * k + i] = u[i];
#pragma unroll
  for (int i = 0; i < 6; ++i) P[6 * k + i] = p[i];
  smin[k] = sm;
  if (routed) routed[k] = (fp32 && r64) ? 1 : 0;
}

// dst[i] = src[perm[i]] for `width`-wide rows (caller order -> internal).
__global__ __launch_bounds__(kBlock) void k_gather_rows(const double* __restrict__ src, const int32_t* __restrict__ perm,
                                                        int count, int width, double* __restrict__ dst) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= count) return;
  const int64_t o = perm[i];
  for (int c = 0; c < width; ++c) dst[(int64_t)width * i + c] = src[o * width + c];
}

// dst[perm[i]] = sign * src[i] (internal -> caller order).
__global__ __launch_bounds__(kBlock) void k_scatter_rows(const double* __restrict__ src, const int32_t* __restrict__ perm,
                                                         int count, int width, double sign, double* __restrict__ dst) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= count) return;
  const int64_t o = perm[i];
  for (int c = 0; c < width; ++c) dst[o * width + c] = sign * src[(int64_t)width * i + c];
}

// Per-tet 6-vector planes (6 x m, internal order) -> m x 6 rows, caller order.
__global__ __launch_bounds__(kBlock) void k_scatter_planes6(const double* __restrict__ planes, int m,
                                                            const int32_t* __restrict__ tperm, double* __restrict__ dst) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= m) return;
  const int64_t o = tperm[k];
#pragma unroll
  for (int c = 0; c < 6; ++c) dst[6 * o + c] = planes[(size_t)c * m + k];
}

// ---- launchers ----
static inline int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

void launch_rest(hipStream_t st, const int4* tets, const double* X, const double* youngs, const double* poisson,
                 int m, double det_tol, double* G, double* wmu, double* wlam, uint8_t* bad) {
  MFS_LAUNCH(k_rest, dim3(blocks_for(m)), dim3(kBlock), 0, st, tets, X, youngs, poisson, m, det_tol, G, wmu,
                     wlam, bad);
}

void launch_cluster(hipStream_t st, const double* X, const int32_t* tets, int64_t m, int nseg, const double* sa,
                    const double* sb, const int32_t* sh, int32_t* out) {
  MFS_LAUNCH(k_cluster, dim3(blocks_for(m)), dim3(kBlock), 0, st, X, tets, m, nseg, sa, sb, sh, out);
}

void launch_blend_weights(hipStream_t st, const double* X, const int32_t* tets, int64_t m, int nseg,
                          const double* sa, const double* sb, const int32_t* sh, int nh, double width, int kmax,
                          int32_t* out_h, double* out_w) {
  MFS_LAUNCH(k_blend_weights, dim3(blocks_for(m)), dim3(kBlock), 0, st, X, tets, m, nseg, sa, sb, sh, nh, width,
             kmax, out_h, out_w);
}

void launch_blend_rot(hipStream_t st, const double* Rh, int m, int kmax, const int32_t* bh, const double* bw,
                      double* Rt) {
  if (m > 0) MFS_LAUNCH(k_blend_rot, dim3(blocks_for(m)), dim3(kBlock), 0, st, Rh, m, kmax, bh, bw, Rt);
}

void launch_polar(hipStream_t st, const double* F, int64_t count, int fp32, double* U, double* P, double* smin,
                  uint8_t* routed) {
  MFS_LAUNCH(k_polar, dim3(blocks_for(count)), dim3(kBlock), 0, st, F, count, fp32, U, P, smin, routed);
}

void launch_gather_rows(hipStream_t st, const double* src, const int32_t* perm, int count, int width, double* dst) {
  MFS_LAUNCH(k_gather_rows, dim3(blocks_for(count)), dim3(kBlock), 0, st, src, perm, count, width, dst);
}

void launch_scatter_rows(hipStream_t st, const double* src, const int32_t* perm, int count, int width, double sign,
                         double* dst) {
  MFS_LAUNCH(k_scatter_rows, dim3(blocks_for(count)), dim3(kBlock), 0, st, src, perm, count, width, sign, dst);
}

void launch_scatter_planes6(hipStream_t st, const double* planes, int m, const int32_t* tperm, double* dst) {
  MFS_LAUNCH(k_scatter_planes6, dim3(blocks_for(m)), dim3(kBlock), 0, st, planes, m, tperm, dst);
}

}  // namespace mfs
