// Host-side launchers of the library's kernels (one per kernel family).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace mfs {

// Event pair of a sampled profiler scope.  While `stop` is set, the first
// launch through MFS_LAUNCH records `start` on its stream just before it; the
// scope records `stop` on the same stream when it closes, after its last
// launch, so the interval spans the scope's kernels (and the small gaps
// between them).
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
  bool started = false;
  hipStream_t where = nullptr;  // the stream of the first launch
};
LaunchEvents& launch_events();  // this host thread's pair

#define MFS_LAUNCH(kernel, grid, block, shmem, stream, ...)                                            \
  do {                                                                                               \
    ::mfs::LaunchEvents& le_ = ::mfs::launch_events();                                               \
    if (le_.stop && !le_.started) {                                                                  \
      (void)hipEventRecord(le_.start, stream);                                                       \
      le_.started = true;                                                                            \
      le_.where = stream;                                                                            \
    }                                                                                                \
    hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                             \
  } while (0)

// setup and helpers
void launch_rest(hipStream_t st, const int4* tets, const double* X, const double* youngs, const double* poisson,
                 int m, double det_tol, double* G, double* wmu, double* wlam, uint8_t* bad);
void launch_cluster(hipStream_t st, const double* X, const int32_t* tets, int64_t m, int nseg, const double* sa,
                    const double* sb, const int32_t* sh, int32_t* out);
// Rotation smoothing: per-tet blend weights from segment distances (kmax <= 4),
// and the blended, polar-projected tet rotations of the current pose.
void launch_blend_weights(hipStream_t st, const double* X, const int32_t* tets, int64_t m, int nseg,
                          const double* sa, const double* sb, const int32_t* sh, int nh, double width, int kmax,
                          int32_t* out_h, double* out_w);
void launch_blend_rot(hipStream_t st, const double* Rh, int m, int kmax, const int32_t* bh, const double* bw,
                      double* Rt);
void launch_polar(hipStream_t st, const double* F, int64_t count, int fp32, double* U, double* P, double* smin,
                  uint8_t* routed);
void launch_gather_rows(hipStream_t st, const double* src, const int32_t* perm, int count, int width, double* dst);
void launch_scatter_rows(hipStream_t st, const double* src, const int32_t* perm, int count, int width, double sign,
                         double* dst);
void launch_scatter_planes6(hipStream_t st, const double* planes, int m, const int32_t* tperm, double* dst);

// Newton iteration
void launch_warm_start(hipStream_t st, const SysDesc* sd, const Tile* tiles, int ntiles, int fp32);
void launch_element(hipStream_t st, const SysDesc* sd, const Ctrl* ctrl, const Tile* tiles, int ntiles, int fp32);
void launch_assemble(hipStream_t st, const SysDesc* sd, const Tile* tiles, int ntiles, int fp32);
void launch_linesearch(hipStream_t st, const SysDesc* sd, const Ctrl* ctrl, const Tile* tt, int ntt, const Tile* tv,
                       int ntv);
void launch_update(hipStream_t st, const SysDesc* sd, const Ctrl* ctrl, const Tile* tt, int ntt, const Tile* tv,
                   int ntv);
// per-tet stress and multiplier at the descriptor's positions (system 0), in
// the caller's tet order (tperm: internal -> caller)
void launch_stress(hipStream_t st, const SysDesc* sd, int m, const int32_t* tperm, double* P6, double* L9);
void launch_finalize(hipStream_t st, const SysDesc* sd, const int32_t* sys_ids, int nsys);

// PCG
// warm != 0: start from each system's dx (see k_cg_init) instead of 0
void launch_cg_init(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32, int warm = 0);
// `one`: non-null when the launch covers a single system, whose descriptor
// is then passed by value and whose tiles are implicit.
void launch_cg_spmv(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32, int lpr,
                    const SysDesc* one);
void launch_cg_update(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32, const SysDesc* one);
// pipelined PCG (FP64 vectors; fp32 selects FP32 matrix values): init
// (r = b, x = 0, u = M^-1 r), start (w = K u, m_0) and one iteration of
// parity i & 1; finish with launch_cg_finish(..., fp32 = 0)
void launch_pcg_init(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32);
void launch_pcg_start(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32, int lpr,
                      const SysDesc* one);
void launch_pcg_iter(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32, int lpr,
                     const SysDesc* one, int parity);
// Persistent pipelined PCG (FP32 matrix, FP64 vectors): LDS bytes for tiles
// of at most `max_tile_blocks` blocks, the number of its workgroups the
// device holds at once (0: cannot run), and the cooperative launch (one
// workgroup per vertex tile, after launch_pcg_start).
size_t pcg_persist_lds(int max_tile_blocks);
int pcg_persist_capacity(int lpr, size_t lds_bytes);
hipError_t launch_pcg_persist(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int lpr, size_t lds_bytes);
void launch_cg_finish(hipStream_t st, const SysDesc* sd, const Tile* tv, int ntv, int fp32);
// y = K v for one system with FP64 block records (v, y: 3n in the internal order)
void launch_spmv_plain(hipStream_t st, const int32_t* rowptr, const double* vals, int n, const double* v, double* y);

}  // namespace mfs
