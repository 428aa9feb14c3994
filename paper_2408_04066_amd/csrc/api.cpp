#include <cmath>
// C ABI: library-level calls, contexts and the standalone helpers (rotation
// clusters, polar decomposition).
#include <cstring>

#include "internal.h"
#include "launch.h"

using namespace mfs;

extern "C" void mfs_default_opts(mfs_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->precision = MFS_FP64;
  o->max_newton = 50;
  o->fixed_newton = 0;
  o->step_tol = 1e-10;
  o->cg_tol = 1e-10;
  o->cg_max = 20000;
  o->warm_start = MFS_WARM_REST;
  o->output_memory = MFS_MEM_HOST;
  o->cg_adaptive = 0;
  o->load_bisections = 6;
}

extern "C" const char* mfs_status_string(int s) {
  switch (s) {
    case MFS_OK: return "ok";
    case MFS_W_NOT_CONVERGED: return "not converged (best iterate returned)";
    case MFS_E_INVALID: return "invalid argument";
    case MFS_E_DEGENERATE: return "degenerate rest element";
    case MFS_E_SINGULAR: return "pins cannot remove rigid motion";
    case MFS_E_OOM: return "out of device memory";
    case MFS_E_HIP: return "HIP runtime error";
    case MFS_E_BUSY: return "busy";
    case MFS_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

extern "C" const char* mfs_last_error(void) { return last_error_text(); }

extern "C" int mfs_context_create(int device, void* hip_stream, mfs_context** out) {
  clear_error();
  if (!out) return set_error(MFS_E_INVALID, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  MFS_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return set_error(MFS_E_INVALID, "device %d not present (%d devices)", device, ndev);
  MFS_HIP(hipSetDevice(device));
  MFS_TRY(scratch_init(device));
  auto ctx = new mfs_context();
  ctx->device = device;
  if (hip_stream) {
    ctx->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&ctx->stream) != hipSuccess) {
      delete ctx;
      return set_error(MFS_E_HIP, "hipStreamCreate failed");
    }
    ctx->own_stream = true;
  }
  *out = ctx;
  return MFS_OK;
}

extern "C" int mfs_context_destroy(mfs_context* ctx) {
  if (!ctx) return MFS_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return MFS_OK;
}

// Copy host or device input into device memory owned by `buf`.
static int stage_in(mfs_context* ctx, DevBuf& buf, const void* src, size_t bytes, int mem, const void** dptr) {
  if (mem == MFS_MEM_DEVICE) {
    *dptr = src;
    return MFS_OK;
  }
  MFS_TRY(buf.alloc(std::max<size_t>(bytes, 1)));
  MFS_HIP(hipMemcpyAsync(buf.p, src, bytes, hipMemcpyHostToDevice, ctx->stream));
  *dptr = buf.p;
  return MFS_OK;
}

extern "C" int mfs_cluster_by_segments(mfs_context* ctx, const double* X, int64_t n, const int32_t* tets, int64_t m,
                                       int32_t nseg, const double* seg_a, const double* seg_b,
                                       const int32_t* seg_handle, int32_t* out, int32_t memory_space) {
  clear_error();
  if (!ctx || !X || !tets || !seg_a || !seg_b || !seg_handle || !out) return set_error(MFS_E_INVALID, "null argument");
  if (n < 1 || m < 1 || nseg < 1) return set_error(MFS_E_INVALID, "empty mesh or no segments");
  if (memory_space != MFS_MEM_HOST && memory_space != MFS_MEM_DEVICE)
    return set_error(MFS_E_INVALID, "invalid memory space");
  MFS_HIP(hipSetDevice(ctx->device));
  if (memory_space == MFS_MEM_HOST) {
    for (int64_t i = 0; i < 4 * m; ++i)
      if (tets[i] < 0 || tets[i] >= n) return set_error(MFS_E_INVALID, "tet vertex index out of range");
  }
  DevBuf bX, bT, ba, bb, bh, bo;
  const void *dX, *dT, *da, *db, *dh;
  MFS_TRY(stage_in(ctx, bX, X, 3 * sizeof(double) * n, memory_space, &dX));
  MFS_TRY(stage_in(ctx, bT, tets, 4 * sizeof(int32_t) * m, memory_space, &dT));
  MFS_TRY(stage_in(ctx, ba, seg_a, 3 * sizeof(double) * nseg, memory_space, &da));
  MFS_TRY(stage_in(ctx, bb, seg_b, 3 * sizeof(double) * nseg, memory_space, &db));
  MFS_TRY(stage_in(ctx, bh, seg_handle, sizeof(int32_t) * nseg, memory_space, &dh));
  int32_t* dout = out;
  if (memory_space == MFS_MEM_HOST) {
    MFS_TRY(bo.alloc(sizeof(int32_t) * m));
    dout = bo.as<int32_t>();
  }
  launch_cluster(ctx->stream, (const double*)dX, (const int32_t*)dT, m, nseg, (const double*)da, (const double*)db,
                 (const int32_t*)dh, dout);
  MFS_HIP(hipGetLastError());
  if (memory_space == MFS_MEM_HOST)
    MFS_HIP(hipMemcpyAsync(out, dout, sizeof(int32_t) * m, hipMemcpyDeviceToHost, ctx->stream));
  MFS_HIP(hipStreamSynchronize(ctx->stream));
  return MFS_OK;
}

extern "C" int mfs_blend_weights(mfs_context* ctx, const double* X, int64_t n, const int32_t* tets, int64_t m,
                                 int32_t nseg, const double* seg_a, const double* seg_b, const int32_t* seg_handle,
                                 int32_t n_handles, double width, int32_t kmax, int32_t* out_handles,
                                 double* out_weights, int32_t memory_space) {
  clear_error();
  if (!ctx || !X || !tets || !seg_a || !seg_b || !seg_handle || !out_handles || !out_weights)
    return set_error(MFS_E_INVALID, "null argument");
  if (n < 1 || m < 1 || nseg < 1) return set_error(MFS_E_INVALID, "empty mesh or no segments");
  if (n_handles < 1 || n_handles > kMaxHandles) return set_error(MFS_E_INVALID, "n_handles out of range");
  if (kmax < 1 || kmax > 4) return set_error(MFS_E_INVALID, "kmax must be in 1..4");
  if (!(width >= 0.0) || !std::isfinite(width)) return set_error(MFS_E_INVALID, "width must be finite and >= 0");
  if (memory_space != MFS_MEM_HOST && memory_space != MFS_MEM_DEVICE)
    return set_error(MFS_E_INVALID, "invalid memory space");
  MFS_HIP(hipSetDevice(ctx->device));
  if (memory_space == MFS_MEM_HOST) {
    for (int64_t i = 0; i < 4 * m; ++i)
      if (tets[i] < 0 || tets[i] >= n) return set_error(MFS_E_INVALID, "tet vertex index out of range");
    for (int32_t i = 0; i < nseg; ++i)
      if (seg_handle[i] < 0 || seg_handle[i] >= n_handles) return set_error(MFS_E_INVALID, "segment handle out of range");
  }
  DevBuf bX, bT, ba, bb, bh, boh, bow;
  const void *dX, *dT, *da, *db, *dh;
  MFS_TRY(stage_in(ctx, bX, X, 3 * sizeof(double) * n, memory_space, &dX));
  MFS_TRY(stage_in(ctx, bT, tets, 4 * sizeof(int32_t) * m, memory_space, &dT));
  MFS_TRY(stage_in(ctx, ba, seg_a, 3 * sizeof(double) * nseg, memory_space, &da));
  MFS_TRY(stage_in(ctx, bb, seg_b, 3 * sizeof(double) * nseg, memory_space, &db));
  MFS_TRY(stage_in(ctx, bh, seg_handle, sizeof(int32_t) * nseg, memory_space, &dh));
  int32_t* doh = out_handles;
  double* dow = out_weights;
  const size_t mk = (size_t)m * kmax;
  if (memory_space == MFS_MEM_HOST) {
    MFS_TRY(boh.alloc(sizeof(int32_t) * mk));
    MFS_TRY(bow.alloc(sizeof(double) * mk));
    doh = boh.as<int32_t>();
    dow = bow.as<double>();
  }
  launch_blend_weights(ctx->stream, (const double*)dX, (const int32_t*)dT, m, nseg, (const double*)da,
                       (const double*)db, (const int32_t*)dh, n_handles, width, kmax, doh, dow);
  MFS_HIP(hipGetLastError());
  if (memory_space == MFS_MEM_HOST) {
    MFS_HIP(hipMemcpyAsync(out_handles, doh, sizeof(int32_t) * mk, hipMemcpyDeviceToHost, ctx->stream));
    MFS_HIP(hipMemcpyAsync(out_weights, dow, sizeof(double) * mk, hipMemcpyDeviceToHost, ctx->stream));
  }
  MFS_HIP(hipStreamSynchronize(ctx->stream));
  return MFS_OK;
}

extern "C" int mfs_polar(mfs_context* ctx, const double* F, int64_t count, int32_t precision, double* U, double* P,
                         double* sigma_min, uint8_t* routed, int32_t memory_space) {
  clear_error();
  if (!ctx || !F || !U || !P || !sigma_min) return set_error(MFS_E_INVALID, "null argument");
  if (count < 1) return set_error(MFS_E_INVALID, "count must be >= 1");
  if (precision != MFS_FP64 && precision != MFS_FP32_REFINED) return set_error(MFS_E_INVALID, "unknown precision");
  if (memory_space != MFS_MEM_HOST && memory_space != MFS_MEM_DEVICE)
    return set_error(MFS_E_INVALID, "invalid memory space");
  MFS_HIP(hipSetDevice(ctx->device));
  const bool host = memory_space == MFS_MEM_HOST;
  DevBuf bF, bU, bP, bS, bR;
  const void* dF;
  MFS_TRY(stage_in(ctx, bF, F, 9 * sizeof(double) * count, memory_space, &dF));
  double *dU = U, *dP = P, *dS = sigma_min;
  uint8_t* dR = routed;
  if (host) {
    MFS_TRY(bU.alloc(9 * sizeof(double) * count));
    MFS_TRY(bP.alloc(6 * sizeof(double) * count));
    MFS_TRY(bS.alloc(sizeof(double) * count));
    dU = bU.as<double>();
    dP = bP.as<double>();
    dS = bS.as<double>();
    if (routed) {
      MFS_TRY(bR.alloc(count));
      dR = bR.as<uint8_t>();
    }
  }
  launch_polar(ctx->stream, (const double*)dF, count, precision == MFS_FP32_REFINED, dU, dP, dS, dR);
  MFS_HIP(hipGetLastError());
  if (host) {
    MFS_HIP(hipMemcpyAsync(U, dU, 9 * sizeof(double) * count, hipMemcpyDeviceToHost, ctx->stream));
    MFS_HIP(hipMemcpyAsync(P, dP, 6 * sizeof(double) * count, hipMemcpyDeviceToHost, ctx->stream));
    MFS_HIP(hipMemcpyAsync(sigma_min, dS, sizeof(double) * count, hipMemcpyDeviceToHost, ctx->stream));
    if (routed) MFS_HIP(hipMemcpyAsync(routed, dR, count, hipMemcpyDeviceToHost, ctx->stream));
  }
  MFS_HIP(hipStreamSynchronize(ctx->stream));
  return MFS_OK;
}

extern "C" int mfs_context_get_tuning(const mfs_context* ctx, mfs_tuning* out) {
  clear_error();
  if (!ctx || !out) return set_error(MFS_E_INVALID, "null argument");
  out->pcg_lanes_per_row = ctx->lpr;
  out->use_graphs = ctx->use_graphs ? 1 : 0;
  out->graph_iterations = ctx->graph_iters;
  out->first_check = ctx->cg_first_run;
  out->min_run = ctx->cg_min_run;
  out->max_run = ctx->cg_max_run;
  out->pcg_pipelined = ctx->pipelined ? 1 : 0;
  out->allread_max_tiles = ctx->allread_tiles;
  out->pcg_persistent = ctx->persistent ? 1 : 0;
  out->batch_async = ctx->batch_async ? 1 : 0;
  return MFS_OK;
}

int mfs::check_tuning(const mfs_tuning* t) {
  if (!t) return set_error(MFS_E_INVALID, "null tuning");
  if (t->pcg_lanes_per_row != 2 && t->pcg_lanes_per_row != 4 && t->pcg_lanes_per_row != 8)
    return set_error(MFS_E_INVALID, "pcg_lanes_per_row must be 2, 4 or 8");
  if (t->graph_iterations < 1 || t->graph_iterations > 64)
    return set_error(MFS_E_INVALID, "graph_iterations must be in [1, 64]");
  if (t->first_check < 1 || t->min_run < 1 || t->max_run < t->min_run)
    return set_error(MFS_E_INVALID, "invalid PCG run bounds");
  if (t->pcg_pipelined != 0 && t->pcg_pipelined != 1) return set_error(MFS_E_INVALID, "pcg_pipelined must be 0 or 1");
  if (t->allread_max_tiles < 0) return set_error(MFS_E_INVALID, "allread_max_tiles must be >= 0");
  if (t->pcg_persistent != 0 && t->pcg_persistent != 1)
    return set_error(MFS_E_INVALID, "pcg_persistent must be 0 or 1");
  if (t->batch_async != 0 && t->batch_async != 1) return set_error(MFS_E_INVALID, "batch_async must be 0 or 1");
  return MFS_OK;
}

extern "C" int mfs_context_set_tuning(mfs_context* ctx, const mfs_tuning* t) {
  clear_error();
  if (!ctx || !t) return set_error(MFS_E_INVALID, "null argument");
  MFS_TRY(check_tuning(t));
  MFS_HIP(hipSetDevice(ctx->device));
  MFS_HIP(hipStreamSynchronize(ctx->stream));
  for (const CgGraph& g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
  ctx->graphs.clear();
  ctx->lpr = t->pcg_lanes_per_row;
  ctx->use_graphs = t->use_graphs != 0;
  ctx->graph_iters = t->graph_iterations;
  ctx->cg_first_run = t->first_check;
  ctx->cg_min_run = t->min_run;
  ctx->cg_max_run = t->max_run;
  ctx->pipelined = t->pcg_pipelined != 0;
  ctx->allread_tiles = t->allread_max_tiles;
  ctx->persistent = t->pcg_persistent != 0;
  ctx->batch_async = t->batch_async != 0;
  return MFS_OK;
}
