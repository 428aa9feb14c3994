// Shared device-side structures of the mixed-FEM skinning library (gfx950).
//
// Every kernel works on "tiles" of one system (one character's frame solve):
// a workgroup of 256 threads takes one tile, loads its system descriptor with
// scalar loads, and works on a contiguous range of vertices, tets or
// matrix-block slots of that system.  A batch is just a longer tile list over
// several descriptors, so one launch covers every character still iterating
// and each character keeps its own scalars and reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mfs {

constexpr int kBlock = 256;      // threads per workgroup of tet and slot kernels (4 wave64)
constexpr int kVTile = 64;       // block rows per vertex tile (vertex kernels run one wave64)
constexpr int kTTile = 256;      // tets per tile
constexpr int kSTile = 256;      // matrix-block slots per tile
constexpr int kMaxHandles = 256;
constexpr int kNumTrials = 5;    // line-search step lengths evaluated per energy pass

// Per-tile partial-result planes (index into SysDesc::part).
enum PartSlot : int {
  P_PQ = 0,      // p . K p
  P_RZ0 = 1,     // r . z, even iterations
  P_RZ1 = 2,     // r . z, odd iterations
  P_RR = 3,      // r . r
  P_BB = 4,      // b . b
  P_SLOPE = 5,   // b . dx
  P_DXMAX = 6,   // max_v |dx_v|
  P_HMAX = 7,    // largest halving count of the mixed line search
  P_INF0 = 8,    // infeasible element count per trial (kNumTrials planes)
  P_E0 = 8 + kNumTrials,        // element energy per trial
  P_PIN0 = 8 + 2 * kNumTrials,  // pin energy per trial
  P_CLAMP = 8 + 3 * kNumTrials, // clamped neo-Hookean elements
  P_ROUTED = 9 + 3 * kNumTrials, // warm-start polar decompositions re-run in FP64
  // pipelined PCG: gamma = r . u, delta = w . u and r . r of the next
  // iteration, by iteration parity (P_RR holds parity 0)
  P_G0 = 10 + 3 * kNumTrials,
  P_G1 = 11 + 3 * kNumTrials,
  P_D0 = 12 + 3 * kNumTrials,
  P_D1 = 13 + 3 * kNumTrials,
  P_RR1 = 14 + 3 * kNumTrials,
  P_COUNT = 15 + 3 * kNumTrials
};

// Per-system PCG scalars.  Every PCG kernel ends with an arrival ticket:
// the last workgroup of a system to finish folds that system's per-tile
// partials in a fixed order and writes the sums here, so the next kernel
// reads a few scalars instead of every tile's partial.  Each field is written
// only by that last workgroup, after every workgroup of the system has read
// the old values.
//
// Systems with at most a tuned number of vertex tiles (default
// kAllReadTiles) skip the tickets (whose release fence costs a few
// microseconds per workgroup): there every workgroup folds the partials
// itself ("all-read" mode, O(tiles) reads per workgroup) and the iteration
// index is double-buffered in it_a / it_b (each written only by the other
// kernel of the PCG pair).
constexpr int kAllReadTiles = 256;

struct CgState {
  double rz;       // r . z of the current iterate (ticket mode)
  double rz_prev;  // r . z of the previous iterate (ticket mode; beta = rz / rz_prev)
  double rr;       // r . r of the current iterate (both modes; for the host)
  double bb;       // b . b (both modes)
  double pq;       // p . K p of the last SpMV (ticket mode)
  int32_t it;      // iterations completed (ticket mode)
  int32_t done;    // 1 once r . r <= tol^2 b . b; 2 after a breakdown (stopped, not converged)
  int32_t iters;   // iterations at convergence
  uint32_t arrive_init, arrive_spmv, arrive_update;  // arrival tickets (0 between kernels)
  int32_t it_a;    // all-read mode: iteration index read by the SpMV kernel
  int32_t it_b;    // all-read mode: iteration index read by the update kernel
  // pipelined PCG (one kernel per iteration)
  double g, d;          // gamma_i, delta_i folded for the next iteration (ticket mode)
  double a_prev[2];     // alpha of the iterations of each parity
  double g_prev[2];     // gamma of the iterations of each parity
  uint32_t arrive_pipe; // arrival ticket of the pipelined kernels
  uint32_t bar;         // persistent form: barrier arrivals of this solve
  int32_t abort;        // persistent form: set when a barrier wait timed out
  int32_t pad1;
  // two-kernel PCG, all-read mode: r . z of iteration it, as the SpMV kernel
  // of that iteration folded it (tile 0 stores it in slot it & 1; the update
  // kernel of iteration it and the SpMV kernel of it + 1 read it instead of
  // folding the plane again)
  double rz_par[2];
};

// Per-system control block, written by the host driver each iteration.
struct Ctrl {
  int32_t phase;     // 0: mixed phase (s != J x), 1: Newton phase (s = J x)
  int32_t update_s;  // mixed phase: apply the stretch update this iteration
  double alpha;      // accepted step length (0 = no update)
  double cg_tol2;    // squared relative PCG tolerance (floor when adaptive)
  int32_t cg_adaptive;  // 1: Eisenstat-Walker forcing on top of the floor
  int32_t cg_cap;       // persistent PCG: iteration cap of this solve
  int32_t cg_epoch;     // number of this PCG solve, stored to SysDesc::stop_flag when it stops
  int32_t pad2;
  double cg_g2prev;  // |g|^2 of the previous Newton step (0: first step)
  double cg_eta_min; // safeguard lower bound on the forcing term
  double cg_eta_max; // upper bound on the forcing term (0: 0.1)
  double trials[kNumTrials];  // step lengths evaluated by the energy pass
};

// PCG stopping threshold on |r|^2 / |b|^2 for one Newton step: the floor
// cg_tol^2, raised in adaptive mode to the Eisenstat-Walker (choice 2) forcing
// eta^2 with eta = min(eta_max, 0.9 (|b| / |b_prev|)^2), eta_max = 0.1 except
// in a step that checks a stop (a smaller cg_eta_max), never below the safeguard
// eta_min; the first step uses eta = eta_max.
__host__ __device__ inline double pcg_tol2(const Ctrl& C, double bb) {
  double tol2 = C.cg_tol2;
  if (C.cg_adaptive) {
    const double cap = C.cg_eta_max > 0.0 ? C.cg_eta_max : 0.1;
    double eta2 = cap * cap;
    if (C.cg_g2prev > 0.0) {
      const double ratio = bb / C.cg_g2prev;
      eta2 = 0.81 * ratio * ratio;
      eta2 = eta2 < cap * cap ? eta2 : cap * cap;
      const double lo = C.cg_eta_min * C.cg_eta_min;
      eta2 = eta2 > lo ? eta2 : lo;
    }
    tol2 = tol2 > eta2 ? tol2 : eta2;
  }
  return tol2;
}

// Global-memory views of the generic pointers the descriptors carry: loads
// and stores through them compile to global_* instructions (a scalar base
// plus a 32-bit lane offset where the base is uniform) instead of flat_*
// ones, which also test the LDS and scratch apertures and wait on both
// memory counters.  Every buffer of the solver is device memory.
// (Host compilation, which never runs these functions, keeps plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
#define MFS_GLOBAL __attribute__((address_space(1)))
#else
#define MFS_GLOBAL
#endif
template <typename T>
__device__ __forceinline__ const MFS_GLOBAL T* gld(const T* p) {
  return (const MFS_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ MFS_GLOBAL T* gst(T* p) {
  return (MFS_GLOBAL T*)p;
}

// A 3x3 matrix block of the condensed system is stored as one record: its
// nine values row-major, then its column (block-row index of the gathered
// vector) as the bits of the tenth word, then zero padding.  FP32: 12 floats
// (48 bytes, read as two 16-byte loads and one 8-byte load); FP64: 10 doubles
// (80 bytes, five 16-byte loads).  A lane reads a whole block, column included, in a few wide loads
// instead of ten single-word loads from ten arrays.
template <typename T>
struct BlockRec;
template <>
struct BlockRec<float> {
  static constexpr int kWords = 12;
};
template <>
struct BlockRec<double> {
  static constexpr int kWords = 10;
};
constexpr int kBlockRecBytes = 80;  // the larger record: a workspace holds either precision

__device__ __forceinline__ void load_block(const float* __restrict__ recs, size_t slot, float a[9], int& col) {
  const MFS_GLOBAL float4* p = (const MFS_GLOBAL float4*)(recs + 12 * slot);
  const float4 r0 = p[0], r1 = p[1];
  const float2 r2 = *(const MFS_GLOBAL float2*)(recs + 12 * slot + 8);  // the padding is not read
  a[0] = r0.x;
  a[1] = r0.y;
  a[2] = r0.z;
  a[3] = r0.w;
  a[4] = r1.x;
  a[5] = r1.y;
  a[6] = r1.z;
  a[7] = r1.w;
  a[8] = r2.x;
  col = __float_as_int(r2.y);
}

__device__ __forceinline__ void load_block(const double* __restrict__ recs, size_t slot, double a[9], int& col) {
  const MFS_GLOBAL double2* p = (const MFS_GLOBAL double2*)(recs + 10 * slot);
  const double2 r0 = p[0], r1 = p[1], r2 = p[2], r3 = p[3], r4 = p[4];
  a[0] = r0.x;
  a[1] = r0.y;
  a[2] = r1.x;
  a[3] = r1.y;
  a[4] = r2.x;
  a[5] = r2.y;
  a[6] = r3.x;
  a[7] = r3.y;
  a[8] = r4.x;
  col = (int)__double_as_longlong(r4.y);
}

__device__ __forceinline__ void store_block(float* recs, size_t slot, const double v[9], int col) {
  MFS_GLOBAL float4* p = (MFS_GLOBAL float4*)(recs + 12 * slot);
  p[0] = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
  p[1] = make_float4((float)v[4], (float)v[5], (float)v[6], (float)v[7]);
  p[2] = make_float4((float)v[8], __int_as_float(col), 0.0f, 0.0f);
}

__device__ __forceinline__ void store_block(double* recs, size_t slot, const double v[9], int col) {
  MFS_GLOBAL double2* p = (MFS_GLOBAL double2*)(recs + 10 * slot);
  p[0] = make_double2(v[0], v[1]);
  p[1] = make_double2(v[2], v[3]);
  p[2] = make_double2(v[4], v[5]);
  p[3] = make_double2(v[6], v[7]);
  p[4] = make_double2(v[8], __longlong_as_double((long long)col));
}

// The three components of block row `row` of a 3n vector, gathered (or
// stored) as one triple: one 12-byte access for FP32, a 16-byte and an 8-byte
// one for FP64, instead of three single-word accesses.
template <typename T>
struct Triple {
  T x, y, z;
};
template <typename T>
__device__ __forceinline__ Triple<T> gather3(const T* __restrict__ v, int row) {
  const MFS_GLOBAL T* p = gld(v) + 3 * (size_t)row;
  return Triple<T>{p[0], p[1], p[2]};
}

template <typename T>
__device__ __forceinline__ void scatter3(T* __restrict__ v, int row, T x, T y, T z) {
  MFS_GLOBAL T* p = gst(v) + 3 * (size_t)row;
  p[0] = x;
  p[1] = y;
  p[2] = z;
}

struct Tile {
  int32_t sys;     // system (descriptor) index
  int32_t begin;   // first vertex / tet / slot
  int32_t end;     // one past the last
  int32_t local;   // tile index within its system (partial-result column)
};

struct SysDesc {
  int32_t n, m, nnzb, nh;
  int32_t ntv, ntt, nts, ptile;   // tiles per system: vertex, tet, slot; partial stride
  int32_t ticket;                 // PCG reductions by arrival ticket (ntv above the all-read limit)
  int32_t par0;                   // pipelined PCG: parity of the launch that runs this system's iteration 0
  double ks;                      // pin stiffness
  // resident (reordered) mesh data
  const int4* tets;        // m
  const double* G;         // 9 planes of m: G[(3r+c)*m + k] = (Dm_k^-1)[r][c]
  const double* wmu;       // m: W_k mu_k
  const double* wlam;      // m: W_k lambda_k
  const int32_t* info;     // m: cluster | model << 16
  const double* X;         // 3n rest positions
  const int32_t* rowptr;   // n + 1
  const int32_t* colidx;   // nnzb
  const int32_t* slot_ptr; // nnzb + 1
  const int32_t* contrib;  // 16 m: (tet << 4) | (a << 2) | b, grouped by slot
  const int32_t* diag;     // n: slot of block (r, r)
  const int32_t* vpin_ptr; // n + 1
  const int32_t* vpin_h;   // pins grouped by vertex: their handles
  const double* fext;      // 3n external vertex forces, or null (none)
  const double* Rt;        // 9 planes of m: smoothed tet rotations of the pose, or null (cluster rotations)
  // per-frame rig
  const double* Rh;        // nh x 9
  const double* th;        // nh x 3
  // state (double)
  double* x;     // 3n positions
  double* s;     // 6 planes of m: mixed stretches
  void* blk;     // m records of 90 (precision T): the tet's 10 unique world-frame 3x3 Hessian blocks
  double* frc;   // m records of 12: the tet's four corner forces (gradient of W Psi)
  double* b;     // 3n right-hand side (-grad)
  double* dx;    // 3n step (double)
  // state (precision T of the linear solve)
  void* vals;    // nnzb block records (BlockRec<T>: nine values and the column)
  void* minv;    // 6 n: inverse diagonal blocks (symmetric)
  void* r;
  void* z;
  void* p0;
  void* p1;
  void* q;
  void* xc;      // PCG iterate
  void* v0;      // pipelined PCG: w = K u
  void* v1;      // pipelined PCG: z = K q (recurrence)
  void* v2;      // pipelined PCG: q = M^-1 s (recurrence)
  void* v3;      // pipelined PCG: s = K p (recurrence)
  // reductions
  double* part;  // P_COUNT planes of ptile
  double* red;   // P_COUNT per-system results of the finalize kernel
  CgState* cg;   // PCG scalars of this system
  const Ctrl* ctrl;  // this system's control block (per-step PCG tolerance)
  int32_t* stop_flag;  // host-mapped word set to ctrl->cg_epoch when the PCG stops, or null
};

// Workgroup -> tile map that keeps consecutive tiles on one XCD: workgroups
// are dealt round-robin over the 8 XCDs, so workgroup b runs on XCD b % 8;
// XCD j gets the j-th contiguous chunk of the tile list (neighbouring tiles
// share vertex gathers and sit in that XCD's L2).
__device__ __forceinline__ int xcd_tile(int b, int ntiles) {
  const int j = b & 7, i = b >> 3;
  const int q = ntiles >> 3, rem = ntiles & 7;
  return j * q + (j < rem ? j : rem) + i;
}

// Cross-lane moves through DPP (data-parallel primitives of GFX9): quad
// permutations, mirrors within 8 and 16 lanes, and the broadcasts of lane 15
// and lane 31 to the following rows.  A lane whose row is outside ROW_MASK
// receives 0.  Each move is a VALU operation; a ds_bpermute shuffle goes
// through the LDS crossbar and costs several times as long.
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppMirror8 = 0x141;    // row_half_mirror: lane j <- lane 7 - j within 8
constexpr int kDppMirror16 = 0x140;   // row_mirror: lane j <- lane 15 - j within 16
constexpr int kDppBcast15 = 0x142;    // row_bcast:15
constexpr int kDppBcast31 = 0x143;    // row_bcast:31

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

__device__ __forceinline__ double lane63(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

// Sum over the G consecutive lanes of a group (G = 1, 2, 4 or 8, groups
// aligned to G); every lane of the group gets the sum.  Called with all 64
// lanes active.
template <int G, typename R>
__device__ __forceinline__ R group_sum(R v) {
  if (G >= 2) v += dpp<kDppXor1>(v);
  if (G >= 4) v += dpp<kDppXor2>(v);
  if (G >= 8) v += dpp<kDppMirror8>(v);
  return v;
}

// Sum over the 64 lanes in a fixed order (quads, eighths, rows of 16, then
// the rows in order); every lane gets the sum.  Called with all 64 lanes
// active.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp<kDppXor1>(v);
  v += dpp<kDppXor2>(v);
  v += dpp<kDppMirror8>(v);
  v += dpp<kDppMirror16>(v);
  v += dpp<kDppBcast15, 0xA>(v);
  v += dpp<kDppBcast31, 0xC>(v);
  return lane63(v);
}

// Maximum over the 64 lanes of values >= 0 (a masked-off row contributes 0).
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp<kDppXor1>(v));
  v = fmax(v, dpp<kDppXor2>(v));
  v = fmax(v, dpp<kDppMirror8>(v));
  v = fmax(v, dpp<kDppMirror16>(v));
  v = fmax(v, dpp<kDppBcast15, 0xA>(v));
  v = fmax(v, dpp<kDppBcast31, 0xC>(v));
  return lane63(v);
}

// Fixed-order workgroup sum: butterfly within each wave, then the wave
// totals in order.  Every thread returns the same value.
template <int NW = 4>
__device__ __forceinline__ double block_sum(double v, double* lds) {
  v = wave_sum(v);
  if (NW == 1) return v;
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  double acc = lds[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) acc += lds[i];
  return acc;
}

// Three fixed-order workgroup sums with one pair of barriers (lds: 3 x NW).
template <int NW = 4>
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* lds) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  if (NW == 1) return;
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    lds[w] = a;
    lds[NW + w] = b;
    lds[2 * NW + w] = c;
  }
  __syncthreads();
  a = lds[0];
  b = lds[NW];
  c = lds[2 * NW];
#pragma unroll
  for (int i = 1; i < NW; ++i) {
    a += lds[i];
    b += lds[NW + i];
    c += lds[2 * NW + i];
  }
}

__device__ __forceinline__ double block_max(double v, double* lds4) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds4[w] = v;
  __syncthreads();
  return fmax(fmax(lds4[0], lds4[1]), fmax(lds4[2], lds4[3]));
}

// Sum of one partial plane over a system's tiles in a fixed order: lane l
// adds tiles l, l + 64, ... in sequence, then the wave butterfly.  Every lane
// of every wave returns the same value, independent of which workgroup asks.
// The loads of four terms are issued before their additions.
__device__ __forceinline__ double sys_sum(const double* plane, int count) {
  double acc = 0.0;
  for (int i0 = threadIdx.x & 63; i0 < count; i0 += 256) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = gld(plane)[i0 + 64 * u < count ? i0 + 64 * u : i0];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + 64 * u < count) acc += v[u];
  }
  return wave_sum(acc);
}

// Arrival ticket at the end of a kernel: thread 0 has stored this
// workgroup's partial; returns true (in every thread) in the workgroup that
// arrives last among `count`.  The release fence orders the partial store
// before the ticket; the last workgroup then reads the partials coherently.
__device__ __forceinline__ bool last_arrival(uint32_t* ticket, uint32_t count, int* lds_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t t = atomicAdd(ticket, 1u);
    *lds_flag = (t == count - 1) ? 1 : 0;
  }
  __syncthreads();
  const bool last = *lds_flag != 0;
  if (last) __threadfence();
  return last;
}

// Tells the host that this system's PCG has stopped (converged, or broke
// down): the solve's epoch, stored to the host-mapped flag at system scope.
// Called by the one thread that sets CgState::done.
__device__ __forceinline__ void signal_stop(const SysDesc& S) {
  if (S.stop_flag) __hip_atomic_store(S.stop_flag, S.ctrl->cg_epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Fixed-order sum of one partial plane with device-coherent loads (the
// partials were written by other workgroups of the running kernel, possibly
// on other XCDs).  Lane l adds entries l, l + 64, ...; then the butterfly.
__device__ __forceinline__ double coherent_sum(const double* plane, int count) {
  double acc = 0.0;
  for (int i = threadIdx.x & 63; i < count; i += 64)
    acc += __hip_atomic_load(plane + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return wave_sum(acc);
}

// This lane's terms of the fixed-order sums of three partial planes (lane l
// adds tiles l, l + 64, ... in sequence, as sys_sum does), with the loads of
// four terms per plane issued before their additions.
__device__ __forceinline__ void lane_sums3(const double* a, const double* b, const double* c, int count,
                                           double& sa, double& sb, double& sc) {
  sa = sb = sc = 0.0;
  for (int i0 = threadIdx.x & 63; i0 < count; i0 += 256) {
    double va[4], vb[4], vc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + 64 * u < count ? i0 + 64 * u : i0;
      va[u] = a[i];
      vb[u] = b[i];
      vc[u] = c[i];
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

__device__ __forceinline__ double sys_max(const double* plane, int count) {
  double acc = 0.0;
  for (int i0 = threadIdx.x & 63; i0 < count; i0 += 256) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = plane[i0 + 64 * u < count ? i0 + 64 * u : i0];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + 64 * u < count) acc = fmax(acc, v[u]);
  }
  return wave_max(acc);
}

}  // namespace mfs
