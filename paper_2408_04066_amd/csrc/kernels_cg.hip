// Preconditioned conjugate gradients on the condensed 3x3-block system
// (the global sparse SPD solve of each Newton step).
//
// Standard form: two kernels per iteration.  k_cg_spmv forms the search direction
// p_it = z + beta p_{it-1} on the fly (double-buffered p, so the gathers of
// neighbouring rows read the previous buffer) and q = K p_it, with LPR lanes
// per block row reading the 9 value planes of consecutive slots (coalesced).
// k_cg_update applies alpha, the block-Jacobi preconditioner and the next
// dot products.  Dot products are per-tile partials in FP64, folded in a
// fixed order: for systems with many tiles by the last workgroup to finish
// each kernel (arrival ticket) into the system's PCG state, which the next
// kernel reads as a few scalars; for systems with few tiles by every
// workgroup of the next kernel ("all-read", no fences).  Convergence
// (||r|| <= tol ||b||) is decided from those folds.
//
// The iteration index and the per-step tolerance live in device memory: the
// launch arguments of an iteration do not depend on its index, and a run of
// iterations can be captured once as a HIP graph and replayed.
#include "common.h"
#include "elem_math.h"
#include "launch.h"

namespace mfs {

// z = M_row^-1 r with the symmetric 3x3 inverse block stored in precision T
// and the vectors in precision V (the product runs in V).
template <typename T, typename V>
__device__ __forceinline__ void precondition(const T* __restrict__ mi, const V rv[3], V zv[3]) {
  const V m0 = (V)mi[0], m1 = (V)mi[1], m2 = (V)mi[2], m3 = (V)mi[3], m4 = (V)mi[4], m5 = (V)mi[5];
  zv[0] = m0 * rv[0] + m5 * rv[1] + m4 * rv[2];
  zv[1] = m5 * rv[0] + m1 * rv[1] + m3 * rv[2];
  zv[2] = m4 * rv[0] + m3 * rv[1] + m2 * rv[2];
}

// ONE: a single system whose descriptor is the kernel argument `one` and
// whose tiles are implicit (tile j = rows [64 j, 64 j + 64)); saves the two
// dependent loads (tile, descriptor) at the head of every workgroup.
template <bool ONE>
__device__ __forceinline__ Tile vertex_tile(const Tile* __restrict__ tiles, int ntiles, const SysDesc& one) {
  const int j = xcd_tile(blockIdx.x, ntiles);
  if (ONE) return Tile{0, j * kVTile, min(one.n, (j + 1) * kVTile), j};
  return tiles[j];
}

// r = b, x = 0, z = M^-1 r; partials r.z, r.r, b.b.  Ticket mode: the last
// workgroup of a system sets its PCG state (and `done` when b is already
// within tolerance).  All-read mode: tile 0 resets the state; the first SpMV
// folds the partials and tests convergence.
template <typename T, typename V = T>
__global__ __launch_bounds__(64) void k_cg_init(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
                                                int ntiles) {
  __shared__ int last;
  const Tile t = tiles[xcd_tile(blockIdx.x, ntiles)];
  const SysDesc& S = sd[t.sys];
  const int row = t.begin + threadIdx.x;
  double rz = 0.0, rr = 0.0, bb = 0.0;
  if (row < t.end) {
    V* r = (V*)S.r;
    V* z = (V*)S.z;
    V* xc = (V*)S.xc;
    V rv[3], zv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double bv = S.b[3 * row + i];
      bb += bv * bv;
      rv[i] = (V)bv;
      r[3 * row + i] = rv[i];
      xc[3 * row + i] = (V)0;
    }
    precondition((const T*)S.minv + 6 * row, rv, zv);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      z[3 * row + i] = zv[i];
      rz += (double)rv[i] * (double)zv[i];
      rr += (double)rv[i] * (double)rv[i];
    }
  }
  rz = wave_sum(rz);
  rr = wave_sum(rr);
  bb = wave_sum(bb);
  if (threadIdx.x == 0) {
    S.part[P_RZ0 * S.ptile + t.local] = rz;
    S.part[P_RR * S.ptile + t.local] = rr;
    S.part[P_BB * S.ptile + t.local] = bb;
  }
  CgState* st = S.cg;
  if (!S.ticket) {
    if (t.local == 0 && threadIdx.x == 0) {
      st->done = 0;
      st->iters = 0;
      st->it_a = 0;
      st->it_b = 0;
    }
    return;
  }
  if (last_arrival(&st->arrive_init, S.ntv, &last)) {
    const double srz = coherent_sum(S.part + P_RZ0 * S.ptile, S.ntv);
    const double srr = coherent_sum(S.part + P_RR * S.ptile, S.ntv);
    const double sbb = coherent_sum(S.part + P_BB * S.ptile, S.ntv);
    if (threadIdx.x == 0) {
      st->rz = srz;
      st->rz_prev = 0.0;
      st->rr = srr;
      st->bb = sbb;
      st->pq = 0.0;
      st->it = 0;
      st->iters = 0;
      st->done = srr <= pcg_tol2(*S.ctrl, sbb) * sbb ? 1 : 0;
      st->arrive_init = 0;
    }
  }
}

// Search direction p_it = z + beta p_{it-1} and q = K p_it: one pass of 64
// rows, LPR lanes per row; partial p.q.
template <typename T, int LPR, bool ONE>
__global__ __launch_bounds__(64 * LPR) void k_cg_spmv(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
                                                      int ntiles, const SysDesc one) {
  __shared__ double red[LPR];
  __shared__ double bcast[2];
  __shared__ int last;
  const Tile t = vertex_tile<ONE>(tiles, ntiles, one);
  const SysDesc& S = ONE ? one : sd[t.sys];
  CgState* st = S.cg;
  int it;
  double beta;
  if (S.ticket) {
    if (st->done) return;
    it = st->it;
    beta = it == 0 ? 0.0 : st->rz / st->rz_prev;
  } else {
    // all-read: wave 0 folds this system's partials, the workgroup shares them
    it = st->it_a;
    if (threadIdx.x < 64) {
      const double* part = S.part;
      const double rr = sys_sum(part + P_RR * S.ptile, S.ntv);
      const double bb = sys_sum(part + P_BB * S.ptile, S.ntv);
      const bool conv = rr <= pcg_tol2(*S.ctrl, bb) * bb;
      double b = 0.0;
      if (!conv && it > 0)
        b = sys_sum(part + (P_RZ0 + (it & 1)) * S.ptile, S.ntv) /
            sys_sum(part + (P_RZ0 + ((it + 1) & 1)) * S.ptile, S.ntv);
      if (threadIdx.x == 0) {
        bcast[0] = conv ? 1.0 : 0.0;
        bcast[1] = b;
        if (t.local == 0) {
          st->rr = rr;
          st->bb = bb;
          if (conv && st->done == 0) {
            st->done = 1;
            st->iters = it;
          }
          if (!conv) st->it_b = it;
        }
      }
    }
    __syncthreads();
    if (bcast[0] != 0.0) return;
    beta = bcast[1];
  }
  const T tb = (T)beta;
  T* pn = (T*)((it & 1) ? S.p1 : S.p0);
  const T* po = (const T*)((it & 1) ? S.p0 : S.p1);
  const T* z = (const T*)S.z;
  const T* vals = (const T*)S.vals;
  T* q = (T*)S.q;
  const size_t nz = S.nnzb;
  const int lane = threadIdx.x % LPR;
  const int row = t.begin + threadIdx.x / LPR;
  T a0 = 0, a1 = 0, a2 = 0;
  if (row < t.end) {
    // batches of U blocks per lane: indices and values first, then the
    // gathers (two dependent latencies per batch, not per block)
    constexpr int U = LPR >= 16 ? 1 : 16 / LPR;
    const int e = S.rowptr[row + 1];
    for (int base = S.rowptr[row] + lane; base < e; base += U * LPR) {
      int c[U];
      T a[U][9];
#pragma unroll
      for (int u = 0; u < U; ++u) {  // past the row's end: reload its last block, weight 0
        const int sl = base + u * LPR;
        const int sc = sl < e ? sl : e - 1;
        c[u] = S.colidx[sc];
#pragma unroll
        for (int k = 0; k < 9; ++k) a[u][k] = vals[k * nz + sc];
      }

      T g[U][3];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        g[u][0] = z[3 * c[u]];
        g[u][1] = z[3 * c[u] + 1];
        g[u][2] = z[3 * c[u] + 2];
        if (it) {
          g[u][0] += tb * po[3 * c[u]];
          g[u][1] += tb * po[3 * c[u] + 1];
          g[u][2] += tb * po[3 * c[u] + 2];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {  // weight 1 (exact) or 0 for slots past the row's end
        const T w = base + u * LPR < e ? (T)1 : (T)0;
        a0 += w * (a[u][0] * g[u][0] + a[u][1] * g[u][1] + a[u][2] * g[u][2]);
        a1 += w * (a[u][3] * g[u][0] + a[u][4] * g[u][1] + a[u][5] * g[u][2]);
        a2 += w * (a[u][6] * g[u][0] + a[u][7] * g[u][1] + a[u][8] * g[u][2]);
      }
    }
  }
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) {
    a0 += __shfl_xor(a0, o, 64);
    a1 += __shfl_xor(a1, o, 64);
    a2 += __shfl_xor(a2, o, 64);
  }
  double dot = 0.0;
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
    dot = (double)p0 * (double)a0 + (double)p1 * (double)a1 + (double)p2 * (double)a2;
  }
  const double tot = block_sum<LPR>(dot, red);
  if (threadIdx.x == 0) S.part[P_PQ * S.ptile + t.local] = tot;
  if (S.ticket && last_arrival(&st->arrive_spmv, S.ntv, &last) && threadIdx.x < 64) {
    const double pq = coherent_sum(S.part + P_PQ * S.ptile, S.ntv);
    if (threadIdx.x == 0) {
      st->pq = pq;
      st->arrive_spmv = 0;
    }
  }
}

// alpha = r.z / p.q; x += alpha p; r -= alpha q; z = M^-1 r; partials r.z
// and r.r.  Ticket mode: the last workgroup folds them, advances the
// iteration and decides convergence with this Newton step's tolerance.
template <typename T, bool ONE>
__global__ __launch_bounds__(64) void k_cg_update(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
                                                  int ntiles, const SysDesc one) {
  __shared__ int last;
  const Tile t = vertex_tile<ONE>(tiles, ntiles, one);
  const SysDesc& S = ONE ? one : sd[t.sys];
  CgState* st = S.cg;
  if (st->done) return;
  int it;
  double rz_old, pq;
  if (S.ticket) {
    it = st->it;
    rz_old = st->rz;
    pq = st->pq;
  } else {
    it = st->it_b;
    pq = sys_sum(S.part + P_PQ * S.ptile, S.ntv);
    rz_old = sys_sum(S.part + (P_RZ0 + (it & 1)) * S.ptile, S.ntv);
  }
  const T alpha = (T)(rz_old / pq);
  const T* pn = (const T*)((it & 1) ? S.p1 : S.p0);
  const T* q = (const T*)S.q;
  T* r = (T*)S.r;
  T* z = (T*)S.z;
  T* xc = (T*)S.xc;
  const int row = t.begin + threadIdx.x;
  double rzn = 0.0, rrn = 0.0;
  if (row < t.end) {
    T rv[3], zv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      xc[3 * row + i] += alpha * pn[3 * row + i];
      rv[i] = r[3 * row + i] - alpha * q[3 * row + i];
      r[3 * row + i] = rv[i];
    }
    precondition((const T*)S.minv + 6 * row, rv, zv);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      z[3 * row + i] = zv[i];
      rzn += (double)rv[i] * (double)zv[i];
      rrn += (double)rv[i] * (double)rv[i];
    }
  }
  rzn = wave_sum(rzn);
  rrn = wave_sum(rrn);
  const int rz_plane = S.ticket ? P_RZ0 : P_RZ0 + ((it + 1) & 1);
  if (threadIdx.x == 0) {
    S.part[rz_plane * S.ptile + t.local] = rzn;
    S.part[P_RR * S.ptile + t.local] = rrn;
    if (!S.ticket && t.local == 0) st->it_a = it + 1;
  }
  if (S.ticket && last_arrival(&st->arrive_update, S.ntv, &last)) {
    const double srz = coherent_sum(S.part + P_RZ0 * S.ptile, S.ntv);
    const double srr = coherent_sum(S.part + P_RR * S.ptile, S.ntv);
    if (threadIdx.x == 0) {
      const double bb = st->bb;
      st->rz_prev = rz_old;
      st->rz = srz;
      st->rr = srr;
      st->it = it + 1;
      if (srr <= pcg_tol2(*S.ctrl, bb) * bb) {
        st->done = 1;
        st->iters = it + 1;
      }
      st->arrive_update = 0;
    }
  }
}

// ---- pipelined PCG (Ghysels and Vanroose, "Hiding global synchronization
// latency in the preconditioned conjugate gradient algorithm", 2014) ----
//
// One kernel per iteration.  Besides x and r it carries u = M^-1 r (in z),
// w = K u (v0) and the recurrences p (p0), s = K p (v3), q = M^-1 s (v2) and
// z = K q (v1); m = M^-1 w is double-buffered by iteration parity (buffer 0
// in p1, buffer 1 in q) because iteration i gathers neighbouring rows of m_i
// while writing m_{i+1}.  gamma = r.u, delta = w.u and r.r of the next
// iteration are per-tile partials double-buffered by parity.  The SpMV of
// iteration i gathers m_i, which is final when the launch starts, so it does
// not wait for the fold that gives alpha_i and beta_i.  In exact arithmetic
// the iterates equal those of the two-kernel PCG.  The matrix values and
// preconditioner blocks are read in precision T, every vector and recurrence
// is kept in V: with T = float the extra recurrences of the pipelined form
// lose the residual in FP32 rounding well before 1e-5 (its three-term
// updates break down), so the FP32 path runs them in FP64.  The parity is a launch
// argument: a captured run of an even number of iterations replays from any
// even iteration.

// acc = (K v)_row over this lane's share of the row's blocks, then summed
// over the LPR lanes of the row (every lane of the row gets the sum).  The
// lane's blocks are taken in batches of U: all column indices and values of a
// batch are loaded first (unconditionally: slots past the row's end reload its
// last block and are weighted 0, so no branch splits the loads), then all gathers are
// issued, so a batch costs two dependent memory latencies instead of two per
// block.
template <typename T, typename V, int LPR>
__device__ __forceinline__ void row_product(const SysDesc& S, const V* __restrict__ v, int row, bool valid, int lane,
                                            V acc[3]) {
  constexpr int U = LPR >= 16 ? 1 : 16 / LPR;
  acc[0] = acc[1] = acc[2] = (V)0;
  if (valid) {
    const T* vals = (const T*)S.vals;
    const size_t nz = S.nnzb;
    const int e = S.rowptr[row + 1];
    for (int base = S.rowptr[row] + lane; base < e; base += U * LPR) {
      int c[U];
      T a[U][9];
#pragma unroll
      for (int u = 0; u < U; ++u) {  // past the row's end: reload its last block, weight 0
        const int sl = base + u * LPR;
        const int sc = sl < e ? sl : e - 1;
        c[u] = S.colidx[sc];
#pragma unroll
        for (int k = 0; k < 9; ++k) a[u][k] = vals[k * nz + sc];
      }

      V g[U][3];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        g[u][0] = v[3 * c[u]];
        g[u][1] = v[3 * c[u] + 1];
        g[u][2] = v[3 * c[u] + 2];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {  // weight 1 (exact) or 0 for slots past the row's end
        const V w = base + u * LPR < e ? (V)1 : (V)0;
        acc[0] += w * ((V)a[u][0] * g[u][0] + (V)a[u][1] * g[u][1] + (V)a[u][2] * g[u][2]);
        acc[1] += w * ((V)a[u][3] * g[u][0] + (V)a[u][4] * g[u][1] + (V)a[u][5] * g[u][2]);
        acc[2] += w * ((V)a[u][6] * g[u][0] + (V)a[u][7] * g[u][1] + (V)a[u][8] * g[u][2]);
      }
    }
  }
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) {
    acc[0] += __shfl_xor(acc[0], o, 64);
    acc[1] += __shfl_xor(acc[1], o, 64);
    acc[2] += __shfl_xor(acc[2], o, 64);
  }
}

// After k_cg_init (r = b, x = 0, u = M^-1 r, partials r.r and b.b):
// w = K u, m_0 = M^-1 w, recurrences cleared, partials gamma_0 and delta_0.
template <typename T, typename V, int LPR, bool ONE>
__global__ __launch_bounds__(64 * LPR) void k_pcg_start(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
                                                        int ntiles, const SysDesc one) {
  __shared__ double red[2][LPR];
  __shared__ int conv;
  __shared__ int last;
  const Tile t = vertex_tile<ONE>(tiles, ntiles, one);
  const SysDesc& S = ONE ? one : sd[t.sys];
  CgState* st = S.cg;
  if (S.ticket) {
    if (st->done) return;
  } else {
    if (threadIdx.x < 64) {
      const double rr = sys_sum(S.part + P_RR * S.ptile, S.ntv);
      const double bb = sys_sum(S.part + P_BB * S.ptile, S.ntv);
      const bool c = rr <= pcg_tol2(*S.ctrl, bb) * bb;
      if (threadIdx.x == 0) {
        conv = c ? 1 : 0;
        if (t.local == 0) {
          st->rr = rr;
          st->bb = bb;
          if (c) {
            st->done = 1;
            st->iters = 0;
          }
        }
      }
    }
    __syncthreads();
    if (conv) return;
  }
  if (t.local == 0 && threadIdx.x == 0) {
    st->a_prev[1] = 1.0;       // alpha_{-1}: any non-zero value
    st->g_prev[1] = INFINITY;  // gamma_{-1}: beta_0 = 0
  }
  const int lane = threadIdx.x % LPR;
  const int row = t.begin + threadIdx.x / LPR;
  const bool valid = row < t.end;
  const V* u = (const V*)S.z;
  V w[3];
  row_product<T, V, LPR>(S, u, row, valid, lane, w);
  double g = 0.0, dl = 0.0;
  if (valid && lane == 0) {
    V m[3];
    precondition((const T*)S.minv + 6 * row, w, m);
    V* wv = (V*)S.v0;
    V* mv = (V*)S.p1;
    V* zv = (V*)S.v1;
    V* qv = (V*)S.v2;
    V* sv = (V*)S.v3;
    V* pv = (V*)S.p0;
    const V* r = (const V*)S.r;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int k = 3 * row + i;
      wv[k] = w[i];
      mv[k] = m[i];
      zv[k] = qv[k] = sv[k] = pv[k] = (V)0;
      const double uk = (double)u[k];
      g += (double)r[k] * uk;
      dl += (double)w[i] * uk;
    }
  }
  const double tg = block_sum<LPR>(g, red[0]);
  const double td = block_sum<LPR>(dl, red[1]);
  if (threadIdx.x == 0) {
    S.part[P_G0 * S.ptile + t.local] = tg;
    S.part[P_D0 * S.ptile + t.local] = td;
  }
  if (S.ticket && last_arrival(&st->arrive_pipe, S.ntv, &last) && threadIdx.x < 64) {
    const double sg = coherent_sum(S.part + P_G0 * S.ptile, S.ntv);
    const double sdl = coherent_sum(S.part + P_D0 * S.ptile, S.ntv);
    if (threadIdx.x == 0) {
      st->g = sg;
      st->d = sdl;
      st->arrive_pipe = 0;
    }
  }
}

// Iteration i (parity = i & 1) of the pipelined PCG.
template <typename T, typename V, int LPR, bool ONE>
__global__ __launch_bounds__(64 * LPR) void k_pcg_iter(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
                                                       int ntiles, const SysDesc one, int parity) {
  __shared__ double red[3][LPR];
  __shared__ double bcast[3];
  __shared__ int last;
  const Tile t = vertex_tile<ONE>(tiles, ntiles, one);
  const SysDesc& S = ONE ? one : sd[t.sys];
  CgState* st = S.cg;
  // A run of launches goes on after convergence (or a breakdown) while its
  // parity argument keeps alternating; the planes of the other parity still
  // hold the previous iteration's sums, so every later launch must stop here.
  // (Within the launch that sets `done`, every workgroup stops anyway.)
  if (st->done) return;
  const int par = parity & 1;
  const int lane = threadIdx.x % LPR;
  const int row = t.begin + threadIdx.x / LPR;
  const bool valid = row < t.end;
  const V* mi = (const V*)(par ? S.q : S.p1);
  V* mn = (V*)(par ? S.p1 : S.q);
  // n_i = K m_i: needs nothing from the fold below
  V nv[3];
  row_product<T, V, LPR>(S, mi, row, valid, lane, nv);
  double gam, del;
  if (S.ticket) {
    gam = st->g;
    del = st->d;
  } else {
    if (threadIdx.x < 64) {
      const double rr = sys_sum(S.part + (par ? P_RR1 : P_RR) * S.ptile, S.ntv);
      const double bb = st->bb;
      const bool c = rr <= pcg_tol2(*S.ctrl, bb) * bb;
      const double g = sys_sum(S.part + (P_G0 + par) * S.ptile, S.ntv);
      const double d = sys_sum(S.part + (P_D0 + par) * S.ptile, S.ntv);
      if (threadIdx.x == 0) {
        bcast[0] = c ? 1.0 : 0.0;
        bcast[1] = g;
        bcast[2] = d;
        if (t.local == 0) {
          st->rr = rr;
          if (c) st->done = 1;
        }
      }
    }
    __syncthreads();
    if (bcast[0] != 0.0) return;
    gam = bcast[1];
    del = bcast[2];
  }
  const double beta = gam / st->g_prev[par ^ 1];
  const double den = del - beta * gam / st->a_prev[par ^ 1];
  if (!(den > 0.0) || !(gam > 0.0)) {  // breakdown (lost positive definiteness in rounding): stop here
    if (t.local == 0 && threadIdx.x == 0) st->done = 2;  // reported as not converged
    return;
  }
  const double alpha = gam / den;
  if (t.local == 0 && threadIdx.x == 0) {
    st->a_prev[par] = alpha;
    st->g_prev[par] = gam;
    if (!S.ticket) st->iters += 1;
  }
  const V ta = (V)alpha, tb = (V)beta;
  double g = 0.0, dl = 0.0, rr = 0.0;
  if (valid && lane == 0) {
    V* zv = (V*)S.v1;
    V* qv = (V*)S.v2;
    V* sv = (V*)S.v3;
    V* pv = (V*)S.p0;
    V* xv = (V*)S.xc;
    V* rv = (V*)S.r;
    V* uv = (V*)S.z;
    V* wv = (V*)S.v0;
    V w[3], mnew[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int k = 3 * row + i;
      const V z = nv[i] + tb * zv[k];
      const V q = mi[k] + tb * qv[k];
      const V sk = wv[k] + tb * sv[k];
      const V pk = uv[k] + tb * pv[k];
      zv[k] = z;
      qv[k] = q;
      sv[k] = sk;
      pv[k] = pk;
      xv[k] += ta * pk;
      const V r = rv[k] - ta * sk;
      const V u = uv[k] - ta * q;
      w[i] = wv[k] - ta * z;
      rv[k] = r;
      uv[k] = u;
      wv[k] = w[i];
      g += (double)r * (double)u;
      dl += (double)w[i] * (double)u;
      rr += (double)r * (double)r;
    }
    precondition((const T*)S.minv + 6 * row, w, mnew);
#pragma unroll
    for (int i = 0; i < 3; ++i) mn[3 * row + i] = mnew[i];
  }
  const int nx = par ^ 1;
  const double tg = block_sum<LPR>(g, red[0]);
  const double td = block_sum<LPR>(dl, red[1]);
  const double tr = block_sum<LPR>(rr, red[2]);
  if (threadIdx.x == 0) {
    S.part[(P_G0 + nx) * S.ptile + t.local] = tg;
    S.part[(P_D0 + nx) * S.ptile + t.local] = td;
    S.part[(nx ? P_RR1 : P_RR) * S.ptile + t.local] = tr;
  }
  if (S.ticket && last_arrival(&st->arrive_pipe, S.ntv, &last) && threadIdx.x < 64) {
    const double sg = coherent_sum(S.part + (P_G0 + nx) * S.ptile, S.ntv);
    const double sdl = coherent_sum(S.part + (P_D0 + nx) * S.ptile, S.ntv);
    const double srr = coherent_sum(S.part + (nx ? P_RR1 : P_RR) * S.ptile, S.ntv);
    if (threadIdx.x == 0) {
      st->g = sg;
      st->d = sdl;
      st->rr = srr;
      st->iters += 1;
      if (srr <= pcg_tol2(*S.ctrl, st->bb) * st->bb) st->done = 1;
      st->arrive_pipe = 0;
    }
  }
}

// dx (FP64) <- PCG iterate.
template <typename T>
__global__ __launch_bounds__(64) void k_cg_finish(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
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
template <typename T, bool ONE>
static void cg_spmv_t(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int lpr, const SysDesc& one) {
  switch (lpr) {
    case 2:
      MFS_LAUNCH((k_cg_spmv<T, 2, ONE>), dim3(ntv), dim3(128), 0, st, sd, tv, ntv, one);
      break;
    case 8:
      MFS_LAUNCH((k_cg_spmv<T, 8, ONE>), dim3(ntv), dim3(512), 0, st, sd, tv, ntv, one);
      break;
    default:
      MFS_LAUNCH((k_cg_spmv<T, 4, ONE>), dim3(ntv), dim3(256), 0, st, sd, tv, ntv, one);
      break;
  }
}

void launch_cg_init(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32) {
  if (!ntv) return;
  if (fp32)
    MFS_LAUNCH(k_cg_init<float>, dim3(ntv), dim3(64), 0, st, sd, tv, ntv);
  else
    MFS_LAUNCH(k_cg_init<double>, dim3(ntv), dim3(64), 0, st, sd, tv, ntv);
}

void launch_cg_spmv(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32, int lpr,
                    const SysDesc* one) {
  if (!ntv) return;
  static const SysDesc none{};
  const SysDesc& o = one ? *one : none;
  if (fp32) {
    if (one) cg_spmv_t<float, true>(st, sd, tv, ntv, lpr, o);
    else cg_spmv_t<float, false>(st, sd, tv, ntv, lpr, o);
  } else {
    if (one) cg_spmv_t<double, true>(st, sd, tv, ntv, lpr, o);
    else cg_spmv_t<double, false>(st, sd, tv, ntv, lpr, o);
  }
}

void launch_cg_update(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32, const SysDesc* one) {
  if (!ntv) return;
  static const SysDesc none{};
  const SysDesc& o = one ? *one : none;
  if (fp32) {
    if (one) MFS_LAUNCH((k_cg_update<float, true>), dim3(ntv), dim3(64), 0, st, sd, tv, ntv, o);
    else MFS_LAUNCH((k_cg_update<float, false>), dim3(ntv), dim3(64), 0, st, sd, tv, ntv, o);
  } else {
    if (one) MFS_LAUNCH((k_cg_update<double, true>), dim3(ntv), dim3(64), 0, st, sd, tv, ntv, o);
    else MFS_LAUNCH((k_cg_update<double, false>), dim3(ntv), dim3(64), 0, st, sd, tv, ntv, o);
  }
}

template <typename T, typename V, bool ONE>
static void pcg_start_t(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int lpr, const SysDesc& one) {
  switch (lpr) {
    case 2:
      MFS_LAUNCH((k_pcg_start<T, V, 2, ONE>), dim3(ntv), dim3(128), 0, st, sd, tv, ntv, one);
      break;
    case 8:
      MFS_LAUNCH((k_pcg_start<T, V, 8, ONE>), dim3(ntv), dim3(512), 0, st, sd, tv, ntv, one);
      break;
    default:
      MFS_LAUNCH((k_pcg_start<T, V, 4, ONE>), dim3(ntv), dim3(256), 0, st, sd, tv, ntv, one);
      break;
  }
}

template <typename T, typename V, bool ONE>
static void pcg_iter_t(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int lpr, const SysDesc& one,
                       int parity) {
  switch (lpr) {
    case 2:
      MFS_LAUNCH((k_pcg_iter<T, V, 2, ONE>), dim3(ntv), dim3(128), 0, st, sd, tv, ntv, one, parity);
      break;
    case 8:
      MFS_LAUNCH((k_pcg_iter<T, V, 8, ONE>), dim3(ntv), dim3(512), 0, st, sd, tv, ntv, one, parity);
      break;
    default:
      MFS_LAUNCH((k_pcg_iter<T, V, 4, ONE>), dim3(ntv), dim3(256), 0, st, sd, tv, ntv, one, parity);
      break;
  }
}

// The pipelined form keeps FP64 vectors; fp32 selects FP32 matrix values.
void launch_pcg_init(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32) {
  if (!ntv) return;
  if (fp32)
    MFS_LAUNCH((k_cg_init<float, double>), dim3(ntv), dim3(64), 0, st, sd, tv, ntv);
  else
    MFS_LAUNCH((k_cg_init<double, double>), dim3(ntv), dim3(64), 0, st, sd, tv, ntv);
}

void launch_pcg_start(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32, int lpr,
                      const SysDesc* one) {
  if (!ntv) return;
  static const SysDesc none{};
  const SysDesc& o = one ? *one : none;
  if (fp32) {
    if (one) pcg_start_t<float, double, true>(st, sd, tv, ntv, lpr, o);
    else pcg_start_t<float, double, false>(st, sd, tv, ntv, lpr, o);
  } else {
    if (one) pcg_start_t<double, double, true>(st, sd, tv, ntv, lpr, o);
    else pcg_start_t<double, double, false>(st, sd, tv, ntv, lpr, o);
  }
}

void launch_pcg_iter(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32, int lpr,
                     const SysDesc* one, int parity) {
  if (!ntv) return;
  static const SysDesc none{};
  const SysDesc& o = one ? *one : none;
  if (fp32) {
    if (one) pcg_iter_t<float, double, true>(st, sd, tv, ntv, lpr, o, parity);
    else pcg_iter_t<float, double, false>(st, sd, tv, ntv, lpr, o, parity);
  } else {
    if (one) pcg_iter_t<double, double, true>(st, sd, tv, ntv, lpr, o, parity);
    else pcg_iter_t<double, double, false>(st, sd, tv, ntv, lpr, o, parity);
  }
}

void launch_cg_finish(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32) {
  if (!ntv) return;
  if (fp32)
    MFS_LAUNCH(k_cg_finish<float>, dim3(ntv), dim3(64), 0, st, sd, tv, ntv);
  else
    MFS_LAUNCH(k_cg_finish<double>, dim3(ntv), dim3(64), 0, st, sd, tv, ntv);
}

void launch_spmv_plain(hipStream_t st, const int32_t* rowptr, const int32_t* colidx, const double* vals, int nnzb,
                       int n, const double* v, double* y) {
  MFS_LAUNCH(k_spmv_plain, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, rowptr, colidx, vals, nnzb,
                     n, v, y);
}

}  // namespace mfs
