// Preconditioned conjugate gradients on the condensed 3x3-block system
// (the global sparse SPD solve of each Newton step).
//
// Two kernels per iteration.  k_cg_spmv(it) forms the search direction
// p_it = z + beta p_{it-1} on the fly (double-buffered p, so the gathers of
// neighbouring rows read the previous buffer) and q = K p_it, with LPR lanes
// per block row reading the 9 value planes of consecutive slots (coalesced).
// k_cg_update(it) applies alpha, the block-Jacobi preconditioner and the
// next dot products.  Dot products are per-tile partials in FP64, folded per
// system in a fixed order by every workgroup that needs them.  Convergence
// (||r|| <= tol ||b||) is decided identically by every workgroup of a system
// from those partials.
#include "common.h"
#include "elem_math.h"
#include "launch.h"

namespace mfs {

template <typename T>
__device__ __forceinline__ T shfl_xor_t(T v, int o) {
  return __shfl_xor(v, o, 64);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_init(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
                                                    int ntiles) {
  __shared__ double red[4];
  const Tile t = tiles[xcd_tile(blockIdx.x, ntiles)];
  const SysDesc& S = sd[t.sys];
  const int row = t.begin + threadIdx.x;
  double rz = 0.0, rr = 0.0, bb = 0.0;
  if (row < t.end) {
    T* r = (T*)S.r;
    T* z = (T*)S.z;
    T* xc = (T*)S.xc;
    const T* mi = (const T*)S.minv + 6 * row;
    T rv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double bv = S.b[3 * row + i];
      bb += bv * bv;
      rv[i] = (T)bv;
      r[3 * row + i] = rv[i];
      xc[3 * row + i] = (T)0;
    }
    T zv[3];
    zv[0] = mi[0] * rv[0] + mi[5] * rv[1] + mi[4] * rv[2];
    zv[1] = mi[5] * rv[0] + mi[1] * rv[1] + mi[3] * rv[2];
    zv[2] = mi[4] * rv[0] + mi[3] * rv[1] + mi[2] * rv[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      z[3 * row + i] = zv[i];
      rz += (double)rv[i] * (double)zv[i];
      rr += (double)rv[i] * (double)rv[i];
    }
  }
  const double s_rz = block_sum(rz, red);
  const double s_rr = block_sum(rr, red);
  const double s_bb = block_sum(bb, red);
  if (threadIdx.x == 0) {
    S.part[P_RZ0 * S.ptile + t.local] = s_rz;
    S.part[P_RR * S.ptile + t.local] = s_rr;
    S.part[P_BB * S.ptile + t.local] = s_bb;
    if (t.local == 0) {
      S.flags[F_CG_DONE] = 0;
      S.flags[F_CG_ITERS] = 0;
    }
  }
}

template <typename T, int LPR>
__global__ __launch_bounds__(kBlock) void k_cg_spmv(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
                                                    int ntiles, int it, double tol2) {
  __shared__ double red[4];
  const Tile t = tiles[xcd_tile(blockIdx.x, ntiles)];
  const SysDesc& S = sd[t.sys];
  const double* part = S.part;
  const double rr = sys_sum(part + P_RR * S.ptile, S.ntv);
  const double bb = sys_sum(part + P_BB * S.ptile, S.ntv);
  if (rr <= tol2 * bb) {
    if (t.local == 0 && threadIdx.x == 0 && S.flags[F_CG_DONE] == 0) {
      S.flags[F_CG_DONE] = 1;
      S.flags[F_CG_ITERS] = it;
    }
    return;
  }
  const double rz = sys_sum(part + (P_RZ0 + (it & 1)) * S.ptile, S.ntv);
  const double beta = it == 0 ? 0.0 : rz / sys_sum(part + (P_RZ0 + ((it + 1) & 1)) * S.ptile, S.ntv);
  const T tb = (T)beta;
  T* pn = (T*)((it & 1) ? S.p1 : S.p0);
  const T* po = (const T*)((it & 1) ? S.p0 : S.p1);
  const T* z = (const T*)S.z;
  const T* vals = (const T*)S.vals;
  T* q = (T*)S.q;
  const size_t nz = S.nnzb;
  const int lane = threadIdx.x % LPR;
  constexpr int RPP = kBlock / LPR;
  double dot = 0.0;
  for (int r0 = t.begin; r0 < t.end; r0 += RPP) {
    const int row = r0 + threadIdx.x / LPR;
    T a0 = 0, a1 = 0, a2 = 0;
    if (row < t.end) {
      const int e = S.rowptr[row + 1];
      for (int sl = S.rowptr[row] + lane; sl < e; sl += LPR) {
        const int c = S.colidx[sl];
        T v0 = z[3 * c], v1 = z[3 * c + 1], v2 = z[3 * c + 2];
        if (it) {
          v0 += tb * po[3 * c];
          v1 += tb * po[3 * c + 1];
          v2 += tb * po[3 * c + 2];
        }
        a0 += vals[sl] * v0 + vals[nz + sl] * v1 + vals[2 * nz + sl] * v2;
        a1 += vals[3 * nz + sl] * v0 + vals[4 * nz + sl] * v1 + vals[5 * nz + sl] * v2;
        a2 += vals[6 * nz + sl] * v0 + vals[7 * nz + sl] * v1 + vals[8 * nz + sl] * v2;
      }
    }
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) {
      a0 += shfl_xor_t(a0, o);
      a1 += shfl_xor_t(a1, o);
      a2 += shfl_xor_t(a2, o);
    }
    if (row < t.end && lane == 0) {
      T p0 = z[3 * row], p1 = z[3 * row + 1], p2 = z[3 * row + 2];
      if (it) {
        p0 += tb * po[3 * row];
        p1 += tb * po[3 * row + 1];
        p2 += tb * po[3 * row + 2];
      }
      pn[3 * row] = p0;
      pn[3 * row + 1] = p1;
      pn[3 * row + 2] = p2;
      q[3 * row] = a0;
      q[3 * row + 1] = a1;
      q[3 * row + 2] = a2;
      dot += (double)p0 * (double)a0 + (double)p1 * (double)a1 + (double)p2 * (double)a2;
    }
  }
  const double tot = block_sum(dot, red);
  if (threadIdx.x == 0) S.part[P_PQ * S.ptile + t.local] = tot;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_update(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
                                                      int ntiles, int it) {
  __shared__ double red[4];
  const Tile t = tiles[xcd_tile(blockIdx.x, ntiles)];
  const SysDesc& S = sd[t.sys];
  if (S.flags[F_CG_DONE]) return;
  const double pq = sys_sum(S.part + P_PQ * S.ptile, S.ntv);
  const double rz = sys_sum(S.part + (P_RZ0 + (it & 1)) * S.ptile, S.ntv);
  const T alpha = (T)(rz / pq);
  const T* pn = (const T*)((it & 1) ? S.p1 : S.p0);
  const T* q = (const T*)S.q;
  T* r = (T*)S.r;
  T* z = (T*)S.z;
  T* xc = (T*)S.xc;
  const int row = t.begin + threadIdx.x;
  double rzn = 0.0, rrn = 0.0;
  if (row < t.end) {
    T rv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      xc[3 * row + i] += alpha * pn[3 * row + i];
      rv[i] = r[3 * row + i] - alpha * q[3 * row + i];
      r[3 * row + i] = rv[i];
    }
    const T* mi = (const T*)S.minv + 6 * row;
    T zv[3];
    zv[0] = mi[0] * rv[0] + mi[5] * rv[1] + mi[4] * rv[2];
    zv[1] = mi[5] * rv[0] + mi[1] * rv[1] + mi[3] * rv[2];
    zv[2] = mi[4] * rv[0] + mi[3] * rv[1] + mi[2] * rv[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      z[3 * row + i] = zv[i];
      rzn += (double)rv[i] * (double)zv[i];
      rrn += (double)rv[i] * (double)rv[i];
    }
  }
  const double s_rz = block_sum(rzn, red);
  const double s_rr = block_sum(rrn, red);
  if (threadIdx.x == 0) {
    S.part[(P_RZ0 + ((it + 1) & 1)) * S.ptile + t.local] = s_rz;
    S.part[P_RR * S.ptile + t.local] = s_rr;
  }
}

// dx (FP64) <- PCG iterate.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_finish(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
                                                      int ntiles) {
  const Tile t = tiles[xcd_tile(blockIdx.x, ntiles)];
  const SysDesc& S = sd[t.sys];
  const int row = t.begin + threadIdx.x;
  if (row >= t.end) return;
  const T* xc = (const T*)S.xc;
#pragma unroll
  for (int i = 0; i < 3; ++i) S.dx[3 * row + i] = (double)xc[3 * row + i];
}

// y = K v for one system (FP64 values and vectors), one thread per block row.
__global__ __launch_bounds__(kBlock) void k_spmv_plain(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                                                       const double* __restrict__ vals, int nnzb, int n,
                                                       const double* __restrict__ v, double* __restrict__ y) {
  const int row = blockIdx.x * kBlock + threadIdx.x;
  if (row >= n) return;
  double a[3] = {0, 0, 0};
  for (int sl = rowptr[row]; sl < rowptr[row + 1]; ++sl) {
    const int c = colidx[sl];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) a[i] += vals[(size_t)(3 * i + j) * nnzb + sl] * v[3 * c + j];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) y[3 * row + i] = a[i];
}

// ---- launchers ----
template <typename T>
static void cg_spmv_t(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int it, double tol2, int lpr) {
  switch (lpr) {
    case 4:
      hipLaunchKernelGGL((k_cg_spmv<T, 4>), dim3(ntv), dim3(kBlock), 0, st, sd, tv, ntv, it, tol2);
      break;
    case 16:
      hipLaunchKernelGGL((k_cg_spmv<T, 16>), dim3(ntv), dim3(kBlock), 0, st, sd, tv, ntv, it, tol2);
      break;
    default:
      hipLaunchKernelGGL((k_cg_spmv<T, 8>), dim3(ntv), dim3(kBlock), 0, st, sd, tv, ntv, it, tol2);
      break;
  }
}

void launch_cg_init(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32) {
  if (!ntv) return;
  if (fp32)
    hipLaunchKernelGGL(k_cg_init<float>, dim3(ntv), dim3(kBlock), 0, st, sd, tv, ntv);
  else
    hipLaunchKernelGGL(k_cg_init<double>, dim3(ntv), dim3(kBlock), 0, st, sd, tv, ntv);
}

void launch_cg_spmv(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int it, double tol2, int fp32,
                    int lpr) {
  if (!ntv) return;
  if (fp32)
    cg_spmv_t<float>(st, sd, tv, ntv, it, tol2, lpr);
  else
    cg_spmv_t<double>(st, sd, tv, ntv, it, tol2, lpr);
}

void launch_cg_update(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int it, int fp32) {
  if (!ntv) return;
  if (fp32)
    hipLaunchKernelGGL(k_cg_update<float>, dim3(ntv), dim3(kBlock), 0, st, sd, tv, ntv, it);
  else
    hipLaunchKernelGGL(k_cg_update<double>, dim3(ntv), dim3(kBlock), 0, st, sd, tv, ntv, it);
}

void launch_cg_finish(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32) {
  if (!ntv) return;
  if (fp32)
    hipLaunchKernelGGL(k_cg_finish<float>, dim3(ntv), dim3(kBlock), 0, st, sd, tv, ntv);
  else
    hipLaunchKernelGGL(k_cg_finish<double>, dim3(ntv), dim3(kBlock), 0, st, sd, tv, ntv);
}

void launch_spmv_plain(hipStream_t st, const int32_t* rowptr, const int32_t* colidx, const double* vals, int nnzb,
                       int n, const double* v, double* y) {
  hipLaunchKernelGGL(k_spmv_plain, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, rowptr, colidx, vals, nnzb,
                     n, v, y);
}

}  // namespace mfs
