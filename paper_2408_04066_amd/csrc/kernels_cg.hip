// Preconditioned conjugate gradients on the condensed 3x3-block system
// (the global sparse SPD solve of each Newton step).
//
// Standard form: two kernels per iteration.  k_cg_spmv forms the search direction
// p_it = z + beta p_{it-1} row by row (double-buffered p) and q = K p_it as
// K z + beta q_{it-1}, the product of the matrix with z alone (one gathered
// vector per neighbouring block instead of two), with LPR lanes per block
// row reading the block records of consecutive slots.
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

// Row i (i = lane < 3) of the packed symmetric 3x3 block of row `row` of
// M^-1, in the order precondition() takes it: (m0 m5 m4), (m5 m1 m3),
// (m4 m3 m2).
template <typename T>
__device__ __forceinline__ void precond_row(const SysDesc& S, int row, int lane, T mb[3]) {
  const T* m = (const T*)S.minv + 6 * row;
  mb[0] = m[lane == 0 ? 0 : (lane == 1 ? 5 : 4)];
  mb[1] = m[lane == 0 ? 5 : (lane == 1 ? 1 : 3)];
  mb[2] = m[lane == 0 ? 4 : (lane == 1 ? 3 : 2)];
}

// Component i = lane of a row's 3-vector.
template <typename V>
__device__ __forceinline__ V component(const V v[3], int lane) {
  return lane == 0 ? v[0] : (lane == 1 ? v[1] : v[2]);
}

// (M^-1 w)_i on lane i < 3 of a row group aligned to four lanes, lane j
// holding w_j and row i of the block (precond_row): the three components
// are broadcast within the quad by DPP, and the products are added in
// precondition()'s order.  Called with all 64 lanes active (lanes that hold
// no component pass zeros).
template <typename T, typename V>
__device__ __forceinline__ V precondition_component(const T mb[3], V wi) {
  constexpr int kQuadLane0 = 0x00, kQuadLane1 = 0x55, kQuadLane2 = 0xAA;  // quad_perm [j,j,j,j]
  const V w0 = dpp<kQuadLane0>(wi), w1 = dpp<kQuadLane1>(wi), w2 = dpp<kQuadLane2>(wi);
  return (V)mb[0] * w0 + (V)mb[1] * w1 + (V)mb[2] * w2;
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
// folds the partials and tests convergence.  warm != 0: x starts from the
// system's dx (the iterate an FP32 solve of the same Newton system left
// there, non-finite entries read as 0) and r = b - K x, a sequential sum of
// the row's blocks in block order; the tolerance stays relative to |b|.
template <typename T, typename V = T>
__global__ __launch_bounds__(64) void k_cg_init(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
                                                int ntiles, int warm) {
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
    double kx[3] = {0.0, 0.0, 0.0}, x0[3] = {0.0, 0.0, 0.0};
    if (warm) {
      auto start = [&](int k) {
        const double v = S.dx[k];
        return isfinite(v) ? v : 0.0;
      };
      const T* vals = (const T*)S.vals;
      for (int blk = S.rowptr[row]; blk < S.rowptr[row + 1]; ++blk) {
        T a[9];
        int c;
        load_block(vals, blk, a, c);
        const double g[3] = {start(3 * c), start(3 * c + 1), start(3 * c + 2)};
#pragma unroll
        for (int i = 0; i < 3; ++i)
          kx[i] += (double)a[3 * i] * g[0] + (double)a[3 * i + 1] * g[1] + (double)a[3 * i + 2] * g[2];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) x0[i] = start(3 * row + i);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double bv = S.b[3 * row + i];
      bb += bv * bv;
      rv[i] = (V)(bv - kx[i]);
      r[3 * row + i] = rv[i];
      xc[3 * row + i] = (V)x0[i];
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
      if (st->done) signal_stop(S);
    }
  }
}

// This lane's terms of four partial planes over the share of wave w of W:
// tiles l + 64 (w + W k), k = 0, 1, ... (l = lane), added in sequence, the
// loads of four terms per plane issued before their additions.
template <int W>
__device__ __forceinline__ void share_sums4(const double* a, const double* b, const double* c, const double* d,
                                            int count, double s[4]) {
  s[0] = s[1] = s[2] = s[3] = 0.0;
  for (int i0 = (threadIdx.x & 63) + 64 * (threadIdx.x >> 6); i0 < count; i0 += 256 * W) {
    double v[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + 64 * W * u < count ? i0 + 64 * W * u : i0;
      v[0][u] = gld(a)[i];
      v[1][u] = gld(b)[i];
      v[2][u] = gld(c)[i];
      v[3][u] = gld(d)[i];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (i0 + 64 * W * u < count) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s[k] += v[k][u];
      }
    }
  }
}

// share_sums4 for two planes.
template <int W>
__device__ __forceinline__ void share_sums2(const double* a, const double* b, int count, double s[4]) {
  s[0] = s[1] = s[2] = s[3] = 0.0;
  for (int i0 = (threadIdx.x & 63) + 64 * (threadIdx.x >> 6); i0 < count; i0 += 256 * W) {
    double v[2][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + 64 * W * u < count ? i0 + 64 * W * u : i0;
      v[0][u] = gld(a)[i];
      v[1][u] = gld(b)[i];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (i0 + 64 * W * u < count) {
        s[0] += v[0][u];
        s[1] += v[1][u];
      }
    }
  }
}

// Search direction p_it = z + beta p_{it-1} and q = K p_it, formed as
// K z + beta q_{it-1} (algebraically the same: K p_{it-1} is the previous
// q): one pass of 64 rows, LPR lanes per row; partial p.q.  What the launch
// reads and no workgroup of it writes (the PCG state, the row's block range,
// the row's z, both p buffers and q, the partial sums of the previous
// launch) is loaded at
// its head, so those loads overlap, before a system whose PCG has stopped
// returns.  In all-read mode the LPR waves of a workgroup fold the sums
// together: wave w adds the tiles of its share in sequence (share_sums4), the
// shares meet in LDS in wave order and each wave sums the 64 lanes itself.
// Every workgroup takes the same order, so all of them reach the same beta
// and convergence decision.  Only the planes the previous update wrote are
// folded (r.r and the new r.z; b.b too in the first iteration): b.b and the
// previous r.z come from the PCG state, where tile 0 of the launch that
// folded them stored them.
template <typename T, int LPR, bool ONE>
__global__ __launch_bounds__(64 * LPR, sizeof(T) == 4 && LPR >= 4 ? 6 : 1) void k_cg_spmv(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
                                                      int ntiles, const SysDesc one) {
  __shared__ double red[LPR];
  __shared__ int last;
  const Tile t = vertex_tile<ONE>(tiles, ntiles, one);
  const SysDesc& S = ONE ? one : sd[t.sys];
  CgState* st = S.cg;
  const int lane = threadIdx.x % LPR;
  const int row = t.begin + threadIdx.x / LPR;
  const bool valid = row < t.end;
  const T* z = (const T*)S.z;
  const int rb = valid ? gld(S.rowptr)[row] : 0;
  const int re = valid ? gld(S.rowptr)[row + 1] : 0;
  const int stopped = st->done;
  const int it_t = st->it, it_all = st->it_a;
  const int it = S.ticket ? it_t : it_all;
  T* q = (T*)S.q;
  T oz[3] = {0, 0, 0}, op0[3] = {0, 0, 0}, op1[3] = {0, 0, 0}, oq[3] = {0, 0, 0};
  // with LPR >= 4, lane i < 3 of the row's group keeps component i of z,
  // both p buffers and the previous q (entry 0) and writes component i of p
  // and q
  constexpr bool CL = LPR >= 4;
  const bool comp = valid && lane < 3;
  if (CL) {
    if (comp) {
      oz[0] = gld(z)[3 * row + lane];
      op0[0] = gld((const T*)S.p0)[3 * row + lane];
      op1[0] = gld((const T*)S.p1)[3 * row + lane];
      oq[0] = gld((const T*)q)[3 * row + lane];
    }
  } else if (valid && lane == 0) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      oz[i] = z[3 * row + i];
      op0[i] = ((const T*)S.p0)[3 * row + i];
      op1[i] = ((const T*)S.p1)[3 * row + i];
      oq[i] = q[3 * row + i];
    }
  }
  double beta;
  const Ctrl ctrl = *S.ctrl;
  if (S.ticket) {
    const double rz_t = st->rz, rzp_t = st->rz_prev;
    if (stopped) return;
    beta = it == 0 ? 0.0 : rz_t / rzp_t;
  } else {
    // it = 0: r.r, r.z and b.b from the start kernel; later: r.r and the new
    // r.z (plane it & 1), with b.b and the previous r.z from the state
    double ls[4] = {0.0, 0.0, 0.0, 0.0};
    const double* prr = S.part + P_RR * S.ptile;
    const double* prz = S.part + (P_RZ0 + (it & 1)) * S.ptile;
    if (it == 0)
      share_sums4<LPR>(prr, prz, S.part + P_BB * S.ptile, prr, S.ntv, ls);
    else
      share_sums2<LPR>(prr, prz, S.ntv, ls);
    const double bb_s = st->bb, rzo_s = st->rz_par[(it + 1) & 1];
    if (stopped) return;  // this system's PCG has stopped
    __shared__ double share[3][LPR][64];
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int nf = it == 0 ? 3 : 2;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (k < nf) share[k][wv][ln] = ls[k];
    __syncthreads();
    double f[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k >= nf) continue;
      f[k] = share[k][0][ln];
#pragma unroll
      for (int j = 1; j < LPR; ++j) f[k] += share[k][j][ln];
      f[k] = wave_sum(f[k]);
    }
    const double rr = f[0], rz = f[1], bb = it == 0 ? f[2] : bb_s;
    const bool conv = rr <= pcg_tol2(ctrl, bb) * bb;
    if (t.local == 0 && threadIdx.x == 0) {
      st->rr = rr;
      if (it == 0) st->bb = bb;
      st->rz_par[it & 1] = rz;
      if (conv && st->done == 0) {
        st->done = 1;
        st->iters = it;
        signal_stop(S);
      }
      if (!conv) st->it_b = it;
    }
    if (conv) return;
    beta = it == 0 ? 0.0 : rz / rzo_s;
  }
  const T tb = (T)beta;
  T* pn = (T*)((it & 1) ? S.p1 : S.p0);
  const T* vals = (const T*)S.vals;
  T a0 = 0, a1 = 0, a2 = 0;
  {
    // K z: batches of U blocks per lane, indices and values first, then the
    // gathers of z (two dependent latencies per batch, not per block)
    constexpr int U = LPR >= 16 ? 1 : 16 / LPR;
    const int e = re;
    for (int base = rb + lane; base < e; base += U * LPR) {
      int c[U];
      T a[U][9];
#pragma unroll
      for (int u = 0; u < U; ++u) {  // past the row's end: reload its last block, weight 0
        const int sl = base + u * LPR;
        load_block(vals, sl < e ? sl : e - 1, a[u], c[u]);
      }

      T g[U][3];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const Triple<T> zc = gather3(z, c[u]);
        g[u][0] = zc.x;
        g[u][1] = zc.y;
        g[u][2] = zc.z;
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
  a0 = group_sum<LPR>(a0);
  a1 = group_sum<LPR>(a1);
  a2 = group_sum<LPR>(a2);
  // p = z + beta p_old and q = K z + beta q_old (= K p)
  double dot = 0.0;
  if (CL) {
    if (comp) {
      T p = oz[0];
      T qv = lane == 0 ? a0 : (lane == 1 ? a1 : a2);
      if (it) {
        p += tb * ((it & 1) ? op0[0] : op1[0]);
        qv += tb * oq[0];
      }
      gst(pn)[3 * row + lane] = p;
      gst(q)[3 * row + lane] = qv;
      dot = (double)p * (double)qv;
    }
  } else if (valid && lane == 0) {
    const T* pold = (it & 1) ? op0 : op1;
    T p0 = oz[0], p1 = oz[1], p2 = oz[2];
    if (it) {
      p0 += tb * pold[0];
      p1 += tb * pold[1];
      p2 += tb * pold[2];
      a0 += tb * oq[0];
      a1 += tb * oq[1];
      a2 += tb * oq[2];
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
// iteration and decides convergence with this Newton step's tolerance.  The
// row's vectors, its preconditioner block and the PCG state are loaded at
// the head, before the convergence flag is tested; in all-read mode the
// workgroup folds p.q and takes r.z from the state.
template <typename T, bool ONE>
__global__ __launch_bounds__(64) void k_cg_update(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
                                                  int ntiles, const SysDesc one) {
  __shared__ int last;
  const Tile t = vertex_tile<ONE>(tiles, ntiles, one);
  const SysDesc& S = ONE ? one : sd[t.sys];
  CgState* st = S.cg;
  const int row = t.begin + threadIdx.x;
  const bool valid = row < t.end;
  T* r = (T*)S.r;
  T* z = (T*)S.z;
  T* xc = (T*)S.xc;
  const T* q = (const T*)S.q;
  T oq[3] = {0, 0, 0}, orr[3] = {0, 0, 0}, ox[3] = {0, 0, 0}, op0[3] = {0, 0, 0}, op1[3] = {0, 0, 0};
  T mb[6] = {0, 0, 0, 0, 0, 0};
  if (valid) {
    const Triple<T> tq = gather3(q, row), tr = gather3((const T*)r, row), tx = gather3((const T*)xc, row);
    const Triple<T> t0 = gather3((const T*)S.p0, row), t1 = gather3((const T*)S.p1, row);
    oq[0] = tq.x, oq[1] = tq.y, oq[2] = tq.z;
    orr[0] = tr.x, orr[1] = tr.y, orr[2] = tr.z;
    ox[0] = tx.x, ox[1] = tx.y, ox[2] = tx.z;
    op0[0] = t0.x, op0[1] = t0.y, op0[2] = t0.z;
    op1[0] = t1.x, op1[1] = t1.y, op1[2] = t1.z;
    __builtin_memcpy(mb, (const T*)S.minv + 6 * (size_t)row, sizeof mb);
  }
  const int stopped = st->done;
  const int it_t = st->it, it_all = st->it_b;
  const double rz_t = st->rz, pq_t = st->pq;
  if (stopped) return;
  int it;
  double rz_old, pq;
  if (S.ticket) {
    it = it_t;
    rz_old = rz_t;
    pq = pq_t;
  } else {
    // p.q from this iteration's SpMV partials; r.z of the iterate as the
    // SpMV kernel folded it
    it = it_all;
    pq = sys_sum(S.part + P_PQ * S.ptile, S.ntv);
    rz_old = st->rz_par[it & 1];
  }
  const T alpha = (T)(rz_old / pq);
  double rzn = 0.0, rrn = 0.0;
  if (valid) {
    const T* pn = (it & 1) ? op1 : op0;
    T rv[3], zv[3], xv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      xv[i] = ox[i] + alpha * pn[i];
      rv[i] = orr[i] - alpha * oq[i];
    }
    scatter3(xc, row, xv[0], xv[1], xv[2]);
    scatter3(r, row, rv[0], rv[1], rv[2]);
    precondition(mb, rv, zv);
    scatter3(z, row, zv[0], zv[1], zv[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
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
        signal_stop(S);
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
// even iteration.  A launch over systems whose solves began at different
// launches (the asynchronous batch form) gives each system the parity of its
// own iteration: the launch's parity xor the system's par0, the parity of the
// launch that ran its iteration 0.

// acc = (K v)_row over this lane's share of the row's blocks, then summed
// over the LPR lanes of the row (every lane of the row gets the sum).  The
// lane's blocks are taken in batches of U: all column indices and values of a
// batch are loaded first (unconditionally: slots past the row's end reload its
// last block and are weighted 0, so no branch splits the loads), then all gathers are
// issued, so a batch costs two dependent memory latencies instead of two per
// block.  The blocks are added in index order whatever U is; a smaller
// batch only holds fewer registers (more waves per SIMD on large meshes).
// The row's block range [rb, re) is passed in (re = rb for no row).
template <typename T, typename V, int LPR>
__device__ __forceinline__ void row_range_product(const SysDesc& S, const V* __restrict__ v, int rb, int re, int lane,
                                                  V acc[3]) {
  constexpr int U = LPR >= 8 ? 1 : 8 / LPR;  // 8 blocks per row in flight (rows average about 15)
  acc[0] = acc[1] = acc[2] = (V)0;
  {
    const T* vals = (const T*)S.vals;
    const int e = re;
    for (int base = rb + lane; base < e; base += U * LPR) {
      int c[U];
      T a[U][9];
#pragma unroll
      for (int u = 0; u < U; ++u) {  // past the row's end: reload its last block, weight 0
        const int sl = base + u * LPR;
        load_block(vals, sl < e ? sl : e - 1, a[u], c[u]);
      }

      V g[U][3];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const Triple<V> vc = gather3(v, c[u]);
        g[u][0] = vc.x;
        g[u][1] = vc.y;
        g[u][2] = vc.z;
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
  acc[0] = group_sum<LPR>(acc[0]);
  acc[1] = group_sum<LPR>(acc[1]);
  acc[2] = group_sum<LPR>(acc[2]);
}

template <typename T, typename V, int LPR>
__device__ __forceinline__ void row_product(const SysDesc& S, const V* __restrict__ v, int row, bool valid, int lane,
                                            V acc[3]) {
  const int rb = valid ? S.rowptr[row] : 0;
  const int re = valid ? S.rowptr[row + 1] : 0;
  row_range_product<T, V, LPR>(S, v, rb, re, lane, acc);
}


// After k_cg_init (r = b, x = 0, u = M^-1 r, partials r.r and b.b):
// w = K u, m_0 = M^-1 w, recurrences cleared, partials gamma_0 and delta_0.
template <typename T, typename V, int LPR, bool ONE>
__global__ __launch_bounds__(64 * LPR) void k_pcg_start(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
                                                        int ntiles, const SysDesc one) {
  __shared__ double red[3][LPR];
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
            signal_stop(S);
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
    st->bar = 0;               // persistent form: no barrier passed yet
    st->abort = 0;
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
  double tg = g, td = dl, tz = 0.0;
  block_sum3<LPR>(tg, td, tz, &red[0][0]);
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

// Iteration i (parity ^ par0 = i & 1) of the pipelined PCG.  Everything the launch
// reads that no workgroup of it writes (the row's block range, the row's own
// vector entries, the partial sums of the previous launch, the PCG state) is
// loaded at its head, before the convergence flag is tested, so the loads
// overlap instead of forming a chain; a launch for a stopped system reads
// them and discards them.  In all-read mode the first wave folds the partial
// sums (every workgroup in the same fixed order) and hands them to the other
// waves through LDS after the SpMV: one fold per workgroup rather than one
// per wave, which at a thousand tiles was more L2 traffic than the
// iteration's own bytes.  The waves of a workgroup may read the convergence
// flag on either side of its setting (it is set during the launch that
// converges), so the folding wave never leaves before the hand-over and the
// stop decision after it is the folding wave's, taken by every wave.  The
// flag changes only in a launch whose fold tells every workgroup to stop.
template <typename T, typename V, int LPR, bool ONE>
__global__ __launch_bounds__(64 * LPR) void k_pcg_iter(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
                                                       int ntiles, const SysDesc one, int parity) {
  __shared__ double red[3][LPR];
  __shared__ int last;
  const Tile t = vertex_tile<ONE>(tiles, ntiles, one);
  const SysDesc& S = ONE ? one : sd[t.sys];
  CgState* st = S.cg;
  const int par = (parity ^ S.par0) & 1;
  const int lane = threadIdx.x % LPR;
  const int row = t.begin + threadIdx.x / LPR;
  const bool valid = row < t.end;
  const bool owner = valid && lane == 0;
  const V* mi = (const V*)(par ? S.q : S.p1);
  V* mn = (V*)(par ? S.p1 : S.q);
  V* zv = (V*)S.v1;
  V* qv = (V*)S.v2;
  V* sv = (V*)S.v3;
  V* pv = (V*)S.p0;
  V* xv = (V*)S.xc;
  V* rv = (V*)S.r;
  V* uv = (V*)S.z;
  V* wv = (V*)S.v0;
  const int rb = valid ? S.rowptr[row] : 0;
  const int re = valid ? S.rowptr[row + 1] : 0;
  // Row vectors: with LPR >= 4, lane i < 3 of the row's group keeps component
  // i of every vector (entry 0 of the arrays) and the row i of its 3x3
  // preconditioner block, so each vector moves in one load or store per
  // row-group instead of three from lane 0; with LPR = 2 lane 0 keeps all
  // three.
  constexpr bool CL = LPR >= 4;
  const bool comp = valid && lane < 3;
  V oz[3], oq[3], os[3], op[3], ox[3], orr[3], ou[3], ow[3], om[3];
  T mb[6];
  if (CL) {
    if (comp) {
      const int k = 3 * row + lane;
      oz[0] = zv[k];
      oq[0] = qv[k];
      os[0] = sv[k];
      op[0] = pv[k];
      ox[0] = xv[k];
      orr[0] = rv[k];
      ou[0] = uv[k];
      ow[0] = wv[k];
      om[0] = mi[k];
      precond_row(S, row, lane, mb);
    } else {
      mb[0] = mb[1] = mb[2] = (T)0;
    }
  } else if (owner) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int k = 3 * row + i;
      oz[i] = zv[k];
      oq[i] = qv[k];
      os[i] = sv[k];
      op[i] = pv[k];
      ox[i] = xv[k];
      orr[i] = rv[k];
      ou[i] = uv[k];
      ow[i] = wv[k];
      om[i] = mi[k];
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) mb[i] = ((const T*)S.minv)[6 * row + i];
  }
  const bool folder = !S.ticket && threadIdx.x < 64;
  double lr = 0.0, lg = 0.0, ld = 0.0;
  if (folder)
    lane_sums3(S.part + (par ? P_RR1 : P_RR) * S.ptile, S.part + (P_G0 + par) * S.ptile,
               S.part + (P_D0 + par) * S.ptile, S.ntv, lr, lg, ld);
  const int stopped = st->done;
  const double g_prev = st->g_prev[par ^ 1], a_prev = st->a_prev[par ^ 1];
  const double bb = st->bb;
  const double g_t = st->g, d_t = st->d;
  const Ctrl ctrl = *S.ctrl;
  // A run of launches goes on after convergence (or a breakdown) while its
  // parity argument keeps alternating; the planes of the other parity still
  // hold the previous iteration's sums, so every later launch must stop here.
  if (stopped && !folder) return;
  // n_i = K m_i: needs nothing from the fold below
  V nv[3] = {(V)0, (V)0, (V)0};
  if (!stopped) row_range_product<T, V, LPR>(S, mi, rb, re, lane, nv);
  double gam, del;
  if (S.ticket) {
    gam = g_t;
    del = d_t;
  } else {
    __shared__ double fold[4];
    if (folder) {
      const double f0 = wave_sum(lr), f1 = wave_sum(lg), f2 = wave_sum(ld);
      if (threadIdx.x == 0) {
        fold[0] = f0;
        fold[1] = f1;
        fold[2] = f2;
        fold[3] = stopped ? 1.0 : 0.0;
      }
    }
    __syncthreads();  // waves that saw the flag set may have left; the barrier waits for the others only
    if (fold[3] != 0.0) return;
    const double rr = fold[0];
    gam = fold[1];
    del = fold[2];
    if (rr <= pcg_tol2(ctrl, bb) * bb) {
      if (t.local == 0 && threadIdx.x == 0) {
        st->rr = rr;
        st->done = 1;
        signal_stop(S);
      }
      return;
    }
    if (t.local == 0 && threadIdx.x == 0) st->rr = rr;
  }
  const double beta = gam / g_prev;
  const double den = del - beta * gam / a_prev;
  if (!(den > 0.0) || !(gam > 0.0)) {  // breakdown (lost positive definiteness in rounding): stop here
    if (t.local == 0 && threadIdx.x == 0) {
      st->done = 2;  // reported as not converged
      signal_stop(S);
    }
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
  if (CL) {
    V wi = (V)0;
    if (comp) {
      const int k = 3 * row + lane;
      const V z = component(nv, lane) + tb * oz[0];
      const V q = om[0] + tb * oq[0];
      const V sk = ow[0] + tb * os[0];
      const V pk = ou[0] + tb * op[0];
      zv[k] = z;
      qv[k] = q;
      sv[k] = sk;
      pv[k] = pk;
      xv[k] = ox[0] + ta * pk;
      const V r = orr[0] - ta * sk;
      const V u = ou[0] - ta * q;
      wi = ow[0] - ta * z;
      rv[k] = r;
      uv[k] = u;
      wv[k] = wi;
      g = (double)r * (double)u;
      dl = (double)wi * (double)u;
      rr = (double)r * (double)r;
    }
    const V mnew = precondition_component<T>(mb, wi);
    if (comp) mn[3 * row + lane] = mnew;
  } else if (owner) {
    V w[3], mnew[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int k = 3 * row + i;
      const V z = nv[i] + tb * oz[i];
      const V q = om[i] + tb * oq[i];
      const V sk = ow[i] + tb * os[i];
      const V pk = ou[i] + tb * op[i];
      zv[k] = z;
      qv[k] = q;
      sv[k] = sk;
      pv[k] = pk;
      xv[k] = ox[i] + ta * pk;
      const V r = orr[i] - ta * sk;
      const V u = ou[i] - ta * q;
      w[i] = ow[i] - ta * z;
      rv[k] = r;
      uv[k] = u;
      wv[k] = w[i];
      g += (double)r * (double)u;
      dl += (double)w[i] * (double)u;
      rr += (double)r * (double)r;
    }
    precondition(mb, w, mnew);
#pragma unroll
    for (int i = 0; i < 3; ++i) mn[3 * row + i] = mnew[i];
  }
  const int nx = par ^ 1;
  double tg = g, td = dl, tr = rr;
  block_sum3<LPR>(tg, td, tr, &red[0][0]);
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
      if (srr <= pcg_tol2(*S.ctrl, st->bb) * st->bb) {
        st->done = 1;
        signal_stop(S);
      }
      st->arrive_pipe = 0;
    }
  }
}

// ---- persistent pipelined PCG ----
//
// The whole pipelined PCG of a Newton step in one cooperative launch: one
// workgroup per vertex tile, every workgroup of the launch resident at once
// (the host launches it only when the device can hold them all).  A
// workgroup copies its tile's rows of the matrix (values, column indices,
// row offsets) into LDS once and keeps its rows' vectors and recurrences in
// registers, so an iteration reads from memory only the gathered
// neighbours of m_i and the previous iteration's partial sums.  Iterations
// of a system are separated by a barrier over that system's workgroups (an
// arrival counter with release/acquire fences); the fold, the convergence
// test and the breakdown test are computed identically by every
// workgroup, so all of a system's workgroups leave the loop at the same
// iteration.  The arithmetic, and its order, is that of k_pcg_iter, so the
// iterates are bitwise those of the one-kernel-per-iteration form.
//
// The values other workgroups read (the rows of m and the partial sums) are
// stored with device-scope atomic stores; the workgroup barrier orders them
// before thread 0's release fence, which (with the acquire fence after the
// wait) makes them visible to the other workgroups of the system.  One fence
// pair per workgroup and iteration: fences issued by every wave cost several
// microseconds per iteration more.
//
// Every spin on the barrier is bounded: a workgroup that waits longer than
// kBarrierSpins polls marks the system aborted (CgState::abort), and every
// workgroup of that system leaves at its next barrier or poll.
constexpr int kBarrierSpins = 1 << 22;

__device__ __forceinline__ void st_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier over the `count` workgroups of one system; `target` is
// count x (barriers passed + 1).  Returns false when the system aborted.
__device__ __forceinline__ bool system_barrier(CgState* st, uint32_t target, int* lds_ok) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();  // release the workgroup's m rows and partial sums
    atomicAdd(&st->bar, 1u);
    int ok = 1;
    for (int spins = 0;; ++spins) {
      if (__hip_atomic_load(&st->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (spins >= kBarrierSpins || __hip_atomic_load(&st->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        __hip_atomic_store(&st->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __threadfence();  // acquire the other workgroups' stores
    *lds_ok = ok;
  }
  __syncthreads();
  return *lds_ok != 0;
}

// Loads of values written by other workgroups of the running launch, at
// device scope (they do not hit stale lines of this CU's caches).
__device__ __forceinline__ double ld_dev(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// lane_sums3 with device-scope loads.
__device__ __forceinline__ void lane_sums3_dev(const double* a, const double* b, const double* c, int count,
                                               double& sa, double& sb, double& sc) {
  sa = sb = sc = 0.0;
  for (int i0 = threadIdx.x & 63; i0 < count; i0 += 256) {
    double va[4], vb[4], vc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + 64 * u < count ? i0 + 64 * u : i0;
      va[u] = ld_dev(a + i);
      vb[u] = ld_dev(b + i);
      vc[u] = ld_dev(c + i);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (i0 + 64 * u < count) {
        sa += va[u];
        sb += vb[u];
        sc += vc[u];
      }
    }
  }
}

// LDS bytes of one tile of `blocks` matrix blocks in precision T.
template <typename T>
__host__ __device__ constexpr size_t persist_lds_bytes(int blocks) {
  return ((size_t)(kVTile + 1) * 4 + 15) / 16 * 16 + ((size_t)blocks * 4 + 15) / 16 * 16 + (size_t)9 * blocks * sizeof(T);
}

template <typename T, typename V, int LPR>
__global__ __launch_bounds__(64 * LPR) void k_pcg_persist(const SysDesc* __restrict__ sd, const Tile* __restrict__ tiles,
                                                          int ntiles) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ double red[3][LPR];
  __shared__ int bar_ok;
  const Tile t = tiles[xcd_tile(blockIdx.x, ntiles)];
  const SysDesc& S = sd[t.sys];
  CgState* st = S.cg;
  if (st->done) return;  // converged at the start (set by the start kernel)
  const int cap = S.ctrl->cg_cap;
  const Ctrl ctrl = *S.ctrl;
  const double bb = st->bb;
  // ---- the tile's matrix rows into LDS ----
  const int rows = t.end - t.begin;
  const int base = S.rowptr[t.begin];
  const int nbt = S.rowptr[t.end] - base;
  int* lrow = (int*)lds_raw;
  int* lcol = (int*)(lds_raw + ((size_t)(kVTile + 1) * 4 + 15) / 16 * 16);
  T* lval = (T*)((unsigned char*)lcol + ((size_t)nbt * 4 + 15) / 16 * 16);
  {
    const T* vals = (const T*)S.vals;
    for (int i = threadIdx.x; i <= rows; i += blockDim.x) lrow[i] = S.rowptr[t.begin + i] - base;
    for (int i = threadIdx.x; i < nbt; i += blockDim.x) {
      T a[9];
      load_block(vals, base + i, a, lcol[i]);
#pragma unroll
      for (int k = 0; k < 9; ++k) lval[k * nbt + i] = a[k];
    }
  }
  const int lane = threadIdx.x % LPR;
  const int lr = threadIdx.x / LPR;
  const int row = t.begin + lr;
  const bool valid = row < t.end;
  const bool owner = valid && lane == 0;
  V* xv = (V*)S.xc;
  // ---- the rows' vectors and recurrences, kept in registers (split by
  // component over lanes 0-2 of the row's group as in k_pcg_iter) ----
  constexpr bool CL = LPR >= 4;
  const bool comp = valid && lane < 3;
  V oz[3], oq[3], os[3], op[3], ox[3], orr[3], ou[3], ow[3], om[3];
  T mb[6];
  if (CL) {
    if (comp) {
      const int k = 3 * row + lane;
      oz[0] = ((const V*)S.v1)[k];
      oq[0] = ((const V*)S.v2)[k];
      os[0] = ((const V*)S.v3)[k];
      op[0] = ((const V*)S.p0)[k];
      ox[0] = xv[k];
      orr[0] = ((const V*)S.r)[k];
      ou[0] = ((const V*)S.z)[k];
      ow[0] = ((const V*)S.v0)[k];
      om[0] = ((const V*)S.p1)[k];  // m_0 (iteration 0 has parity 0)
      precond_row(S, row, lane, mb);
    } else {
      mb[0] = mb[1] = mb[2] = (T)0;
    }
  } else if (owner) {
    const V* zv = (const V*)S.v1;
    const V* qv = (const V*)S.v2;
    const V* sv = (const V*)S.v3;
    const V* pv = (const V*)S.p0;
    const V* rv = (const V*)S.r;
    const V* uv = (const V*)S.z;
    const V* wv = (const V*)S.v0;
    const V* m0 = (const V*)S.p1;  // m_0 (iteration 0 has parity 0)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int k = 3 * row + i;
      oz[i] = zv[k];
      oq[i] = qv[k];
      os[i] = sv[k];
      op[i] = pv[k];
      ox[i] = xv[k];
      orr[i] = rv[k];
      ou[i] = uv[k];
      ow[i] = wv[k];
      om[i] = m0[k];
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) mb[i] = ((const T*)S.minv)[6 * row + i];
  }
  __syncthreads();
  const int rb = valid ? lrow[lr] : 0;
  const int re = valid ? lrow[lr + 1] : 0;
  double a_prev = 1.0, g_prev = INFINITY;  // alpha_{-1}, gamma_{-1}: beta_0 = 0
  double rr_last = st->rr;
  int it = 0;
  int state = 0;  // 0: running/capped, 1: converged, 2: breakdown, 3: aborted
  for (;; ++it) {
    const int par = it & 1;
    const V* mi = (const V*)(par ? S.q : S.p1);
    V* mn = (V*)(par ? S.p1 : S.q);
    // n_i = K m_i: blocks from LDS, m_i gathered (same order as row_range_product)
    V nv[3] = {(V)0, (V)0, (V)0};
    {
      constexpr int U = LPR >= 16 ? 1 : 16 / LPR;
      for (int b0 = rb + lane; b0 < re; b0 += U * LPR) {
        int c[U];
        T a[U][9];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int sl = b0 + u * LPR;
          const int sc = sl < re ? sl : re - 1;
          c[u] = lcol[sc];
#pragma unroll
          for (int k = 0; k < 9; ++k) a[u][k] = lval[k * nbt + sc];
        }
        V g[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          g[u][0] = ld_dev(mi + 3 * c[u]);
          g[u][1] = ld_dev(mi + 3 * c[u] + 1);
          g[u][2] = ld_dev(mi + 3 * c[u] + 2);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const V w = b0 + u * LPR < re ? (V)1 : (V)0;
          nv[0] += w * ((V)a[u][0] * g[u][0] + (V)a[u][1] * g[u][1] + (V)a[u][2] * g[u][2]);
          nv[1] += w * ((V)a[u][3] * g[u][0] + (V)a[u][4] * g[u][1] + (V)a[u][5] * g[u][2]);
          nv[2] += w * ((V)a[u][6] * g[u][0] + (V)a[u][7] * g[u][1] + (V)a[u][8] * g[u][2]);
        }
      }
      nv[0] = group_sum<LPR>(nv[0]);
      nv[1] = group_sum<LPR>(nv[1]);
      nv[2] = group_sum<LPR>(nv[2]);
    }
    // fold of the previous iteration's partial sums (every wave, same order)
    double lsr, lsg, lsd;
    lane_sums3_dev(S.part + (par ? P_RR1 : P_RR) * S.ptile, S.part + (P_G0 + par) * S.ptile,
               S.part + (P_D0 + par) * S.ptile, S.ntv, lsr, lsg, lsd);
    const double rr = wave_sum(lsr);
    const double gam = wave_sum(lsg);
    const double del = wave_sum(lsd);
    rr_last = rr;
    if (rr <= pcg_tol2(ctrl, bb) * bb) {
      state = 1;
      break;
    }
    if (it >= cap) break;
    const double beta = gam / g_prev;
    const double den = del - beta * gam / a_prev;
    if (!(den > 0.0) || !(gam > 0.0)) {
      state = 2;
      break;
    }
    const double alpha = gam / den;
    a_prev = alpha;
    g_prev = gam;
    const V ta = (V)alpha, tb = (V)beta;
    double g = 0.0, dl = 0.0, r2 = 0.0;
    if (CL) {
      V wi = (V)0;
      if (comp) {
        const V z = component(nv, lane) + tb * oz[0];
        const V q = om[0] + tb * oq[0];
        const V sk = ow[0] + tb * os[0];
        const V pk = ou[0] + tb * op[0];
        oz[0] = z;
        oq[0] = q;
        os[0] = sk;
        op[0] = pk;
        ox[0] = ox[0] + ta * pk;
        const V r = orr[0] - ta * sk;
        const V u = ou[0] - ta * q;
        wi = ow[0] - ta * z;
        orr[0] = r;
        ou[0] = u;
        ow[0] = wi;
        g = (double)r * (double)u;
        dl = (double)wi * (double)u;
        r2 = (double)r * (double)r;
      }
      const V mnew = precondition_component<T>(mb, wi);
      if (comp) {
        st_dev(mn + 3 * row + lane, mnew);
        om[0] = mnew;
      }
    } else if (owner) {
      V w[3], mnew[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const V z = nv[i] + tb * oz[i];
        const V q = om[i] + tb * oq[i];
        const V sk = ow[i] + tb * os[i];
        const V pk = ou[i] + tb * op[i];
        oz[i] = z;
        oq[i] = q;
        os[i] = sk;
        op[i] = pk;
        ox[i] = ox[i] + ta * pk;
        const V r = orr[i] - ta * sk;
        const V u = ou[i] - ta * q;
        w[i] = ow[i] - ta * z;
        orr[i] = r;
        ou[i] = u;
        ow[i] = w[i];
        g += (double)r * (double)u;
        dl += (double)w[i] * (double)u;
        r2 += (double)r * (double)r;
      }
      precondition(mb, w, mnew);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        st_dev(mn + 3 * row + i, mnew[i]);
        om[i] = mnew[i];
      }
    }
    const int nx = par ^ 1;
    double tg = g, td = dl, tr = r2;
    block_sum3<LPR>(tg, td, tr, &red[0][0]);
    if (threadIdx.x == 0) {
      st_dev(S.part + (P_G0 + nx) * S.ptile + t.local, tg);
      st_dev(S.part + (P_D0 + nx) * S.ptile + t.local, td);
      st_dev(S.part + (nx ? P_RR1 : P_RR) * S.ptile + t.local, tr);
    }
    if (!system_barrier(st, (uint32_t)S.ntv * (uint32_t)(it + 1), &bar_ok)) {
      state = 3;
      break;
    }
  }
  if (CL) {
    if (comp) xv[3 * row + lane] = ox[0];
  } else if (owner) {
#pragma unroll
    for (int i = 0; i < 3; ++i) xv[3 * row + i] = ox[i];
  }
  if (t.local == 0 && threadIdx.x == 0) {
    st->iters = it;
    st->rr = rr_last;
    st->done = state;
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

// y = K v for one system (FP64 block records and vectors), one thread per
// block row.
__global__ __launch_bounds__(kBlock) void k_spmv_plain(const int32_t* __restrict__ rowptr,
                                                       const double* __restrict__ vals, int n,
                                                       const double* __restrict__ v, double* __restrict__ y) {
  const int row = blockIdx.x * kBlock + threadIdx.x;
  if (row >= n) return;
  double a[3] = {0, 0, 0};
  for (int sl = rowptr[row]; sl < rowptr[row + 1]; ++sl) {
    double b[9];
    int c;
    load_block(vals, sl, b, c);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) a[i] += b[3 * i + j] * v[3 * c + j];
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

void launch_cg_init(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32, int warm) {
  if (!ntv) return;
  if (fp32)
    MFS_LAUNCH(k_cg_init<float>, dim3(ntv), dim3(64), 0, st, sd, tv, ntv, warm);
  else
    MFS_LAUNCH(k_cg_init<double>, dim3(ntv), dim3(64), 0, st, sd, tv, ntv, warm);
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
    MFS_LAUNCH((k_cg_init<float, double>), dim3(ntv), dim3(64), 0, st, sd, tv, ntv, 0);
  else
    MFS_LAUNCH((k_cg_init<double, double>), dim3(ntv), dim3(64), 0, st, sd, tv, ntv, 0);
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

// ---- persistent pipelined PCG launch ----
template <int LPR>
static const void* persist_kernel() {
  return reinterpret_cast<const void*>(&k_pcg_persist<float, double, LPR>);
}
static const void* persist_fn(int lpr) {
  return lpr == 2 ? persist_kernel<2>() : (lpr == 8 ? persist_kernel<8>() : persist_kernel<4>());
}

size_t pcg_persist_lds(int max_tile_blocks) { return persist_lds_bytes<float>(max_tile_blocks); }

int pcg_persist_capacity(int lpr, size_t lds_bytes) {
  int dev = 0, per_cu = 0, cus = 0, lds_max = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
  const size_t static_lds = sizeof(double) * 3 * 8 + 16;
  if (lds_bytes + static_lds > (size_t)lds_max) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persist_fn(lpr), 64 * (lpr == 2 || lpr == 8 ? lpr : 4),
                                                   lds_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return per_cu * cus;
}

hipError_t launch_pcg_persist(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int lpr, size_t lds_bytes) {
  if (!ntv) return hipSuccess;
  const int L = (lpr == 2 || lpr == 8) ? lpr : 4;
  void* args[] = {(void*)&sd, (void*)&tv, (void*)&ntv};
  LaunchEvents& le = launch_events();
  if (le.stop && !le.started) {
    (void)hipEventRecord(le.start, st);
    le.started = true;
    le.where = st;
  }
  return hipLaunchCooperativeKernel(persist_fn(L), dim3(ntv), dim3(64 * L), args, (unsigned)lds_bytes, st);
}

void launch_cg_finish(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32) {
  if (!ntv) return;
  if (fp32)
    MFS_LAUNCH(k_cg_finish<float>, dim3(ntv), dim3(64), 0, st, sd, tv, ntv);
  else
    MFS_LAUNCH(k_cg_finish<double>, dim3(ntv), dim3(64), 0, st, sd, tv, ntv);
}

void launch_spmv_plain(hipStream_t st, const int32_t* rowptr, const double* vals, int n, const double* v,
                       double* y) {
  MFS_LAUNCH(k_spmv_plain, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, rowptr, vals, n, v, y);
}

}  // namespace mfs
