// Batch engine: one Newton iteration per step() over the occupied slots.
//
// Iteration (state x, s; s is the mixed stretch variable of the paper's
// Section 3):
//   solve K(s) dx = -[grad C(x) + sum_k W_k J_k^T (g_k(s) + H_k(s)(J_k x - s_k))]
//   mixed phase (s != J x): alpha = the step the worst neo-Hookean tet allows
//     along s + alpha (J(x + dx) - s) while staying positive definite
//     (halvings of 1); s <- s + alpha (J(x + dx) - s); alpha = 1 lands on the
//     constraint s = J x and starts the Newton phase.
//   Newton phase (s = J x): Armijo on E, E(x + a dx) <= E(x) + 1e-4 a gradE.dx
//     + 1e-12 |E(x)|, with every neo-Hookean stretch positive definite.
//   stop: fixed iteration count, or a Newton-phase step with
//     max_v |alpha dx_v| <= step_tol * bbox diagonal.
// The host reads back only per-slot scalars: PCG flags and residuals after
// each run of PCG iterations, and the line-search reductions.
#include "engine.h"

#include <algorithm>
#include <deque>
#include <cmath>
#include <cstring>

#include "launch.h"

namespace mfs {

int upload_ctrl(mfs_context* ctx, int count) {
  return ctx->up.upload(ctx->stream, ctx->ctrl.p, ctx->h_ctrl.data(), count * sizeof(Ctrl));
}

int ensure_stop_flags(mfs_context* ctx, int slots) {
  if (slots <= ctx->stop_slots) return MFS_OK;
  MFS_HIP(hipStreamSynchronize(ctx->stream));
  if (ctx->h_stop) (void)hipHostFree(ctx->h_stop);
  ctx->h_stop = nullptr;
  ctx->d_stop = nullptr;
  ctx->stop_slots = 0;
  void* p = nullptr;
  if (hipHostMalloc(&p, sizeof(int32_t) * slots, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(MFS_E_OOM, "host-mapped PCG flags for %d slots", slots);
  }
  std::memset(p, 0, sizeof(int32_t) * slots);
  void* d = nullptr;
  if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipHostFree(p);
    return set_error(MFS_E_HIP, "no device address for the host-mapped PCG flags");
  }
  ctx->h_stop = static_cast<int32_t*>(p);
  ctx->d_stop = static_cast<int32_t*>(d);
  ctx->stop_slots = slots;
  return MFS_OK;
}

int sync_event(mfs_context* ctx, hipEvent_t* out) {
  if (!ctx->sync_events.empty()) {
    *out = ctx->sync_events.back();
    ctx->sync_events.pop_back();
    return MFS_OK;
  }
  MFS_HIP(hipEventCreateWithFlags(out, hipEventDisableTiming));
  return MFS_OK;
}

int wait_stream(mfs_context* ctx) {
  hipEvent_t e = nullptr;
  MFS_TRY(sync_event(ctx, &e));
  MFS_HIP(hipEventRecord(e, ctx->stream));
  PollPacer pacer;
  for (;;) {
    const hipError_t r = hipEventQuery(e);
    if (r == hipSuccess) break;
    if (r != hipErrorNotReady) return set_error(MFS_E_HIP, "stream wait: %s", hipGetErrorString(r));
    if (!pacer.pace())
      return set_error(MFS_E_HIP, "stream wait: not done in %d s", PollPacer::kLimitSeconds);
  }
  ctx->sync_events.push_back(e);
  return MFS_OK;
}

int read_cg(mfs_context* ctx, int count, bool resolve) {
  MFS_HIP(hipMemcpyAsync(ctx->h_cg.p, ctx->cg.p, count * sizeof(CgState), hipMemcpyDeviceToHost, ctx->stream));
  MFS_TRY(wait_stream(ctx));
  if (resolve) prof_resolve(ctx);
  return MFS_OK;
}

int wait_event(mfs_context* ctx, hipEvent_t e) {
  PollPacer pacer;
  for (;;) {
    const hipError_t r = hipEventQuery(e);
    if (r == hipSuccess) break;
    if (r != hipErrorNotReady) return set_error(MFS_E_HIP, "event wait: %s", hipGetErrorString(r));
    if (!pacer.pace()) return set_error(MFS_E_HIP, "event wait: not done in %d s", PollPacer::kLimitSeconds);
  }
  ctx->sync_events.push_back(e);
  return MFS_OK;
}

int read_red(mfs_context* ctx, int count, const std::function<int()>& fill) {
  MFS_HIP(hipMemcpyAsync(ctx->h_red.p, ctx->red.p, count * P_COUNT * sizeof(double), hipMemcpyDeviceToHost,
                         ctx->stream));
  if (fill) {
    // wait for the copy only; the work `fill` queues behind it runs meanwhile
    hipEvent_t e = nullptr;
    MFS_TRY(sync_event(ctx, &e));
    MFS_HIP(hipEventRecord(e, ctx->stream));
    MFS_TRY(fill());
    MFS_TRY(wait_event(ctx, e));
  } else {
    MFS_TRY(wait_stream(ctx));
  }
  prof_resolve(ctx);
  return MFS_OK;
}

int build_tile_list(mfs_context* ctx, const std::vector<mfs_character*>& by_slot, const std::vector<int>& ids,
                    TileSet* ts) {
  size_t total = 0;
  for (int i : ids) total += by_slot[i]->ntv + by_slot[i]->ntt + by_slot[i]->nts;
  ctx->h_tiles.resize(std::max<size_t>(total, 1));
  // growing a buffer frees the old one: no queued launch may still read it
  if (std::max<size_t>(total, 1) * sizeof(Tile) > ctx->tiles.bytes ||
      std::max<size_t>(ids.size(), 1) * sizeof(int32_t) > ctx->sys_ids.bytes)
    MFS_HIP(hipStreamSynchronize(ctx->stream));
  MFS_TRY(ctx->tiles.reserve(std::max<size_t>(total, 1) * sizeof(Tile)));
  Tile* h = ctx->h_tiles.data();
  size_t pos = 0;
  int counts[3] = {0, 0, 0};
  for (int kind = 0; kind < 3; ++kind) {
    for (int i : ids) {
      const mfs_character* c = by_slot[i];
      const int items = kind == 0 ? c->n : (kind == 1 ? c->m : c->nnzb);
      const int nt = kind == 0 ? c->ntv : (kind == 1 ? c->ntt : c->nts);
      const int size = kind == 0 ? kVTile : (kind == 1 ? kTTile : kSTile);
      for (int j = 0; j < nt; ++j) {
        h[pos++] = Tile{i, j * size, std::min(items, (j + 1) * size), j};
        counts[kind]++;
      }
    }
  }
  MFS_TRY(ctx->up.upload(ctx->stream, ctx->tiles.p, h, pos * sizeof(Tile)));
  Tile* d = ctx->tiles.as<Tile>();
  ts->nv = counts[0];
  ts->nt = counts[1];
  ts->ns = counts[2];
  ts->dv = d;
  ts->dt = d + counts[0];
  ts->ds = d + counts[0] + counts[1];
  MFS_TRY(ctx->sys_ids.reserve(std::max<size_t>(ids.size(), 1) * sizeof(int32_t)));
  return ctx->up.upload(ctx->stream, ctx->sys_ids.p, ids.data(), ids.size() * sizeof(int32_t));
}

// A run of PCG iterations captured once as a HIP graph per (tiles, sizes,
// precision, launch shape, single-system descriptor) and replayed; the
// kernels take no per-iteration arguments (the iteration index and the
// per-step tolerance live in device memory).
static int cg_graph(mfs_context* ctx, const SysDesc* sd, const TileSet& ts, int fp32, int iters,
                    const SysDesc* one, bool pipe, hipGraphExec_t* out) {
  for (CgGraph& g : ctx->graphs) {
    if (g.sd == sd && g.tiles == ts.dv && g.ntv == ts.nv && g.fp32 == fp32 && g.lpr == ctx->lpr &&
        g.iters == iters && g.pipelined == pipe && g.has_one == (one != nullptr) &&
        (!one || std::memcmp(&g.one, one, sizeof(SysDesc)) == 0)) {
      *out = g.exec;
      return MFS_OK;
    }
  }
  hipGraph_t graph = nullptr;
  MFS_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  for (int j = 0; j < iters; ++j) {
    if (pipe) {
      launch_pcg_iter(ctx->stream, sd, ts.dv, ts.nv, fp32, ctx->lpr, one, j & 1);
    } else {
      launch_cg_spmv(ctx->stream, sd, ts.dv, ts.nv, fp32, ctx->lpr, one);
      launch_cg_update(ctx->stream, sd, ts.dv, ts.nv, fp32, one);
    }
  }
  MFS_HIP(hipStreamEndCapture(ctx->stream, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return set_error(MFS_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  if (ctx->graphs.size() >= 8) {
    (void)hipGraphExecDestroy(ctx->graphs.front().exec);
    ctx->graphs.erase(ctx->graphs.begin());
  }
  CgGraph g{sd, ts.dv, ts.nv, fp32, ctx->lpr, iters, pipe, one != nullptr, SysDesc{}, exec};
  if (one) g.one = *one;
  ctx->graphs.push_back(g);
  *out = exec;
  return MFS_OK;
}

// Enqueue `run` PCG iterations starting at iteration `start`: replayed
// graphs when enabled and the profiler is off, direct launches (each family
// timed by the profiler) otherwise.  A pipelined graph holds an even number
// of iterations and starts at an even one (the kernels take the parity as
// an argument).
static int enqueue_cg(mfs_context* ctx, const SysDesc* sd, const TileSet& ts, int fp32, int run,
                      const SysDesc* one, bool pipe, int start) {
  const int G = ctx->graph_iters;
  int done = 0;
  // timed SpMV-family launches carry their iteration index; their bytes are
  // set once the run's convergence counts are known (run_cg)
  auto direct = [&](int it) {
    if (pipe) {
      ProfScope ps(ctx, MFS_K_SPMV, 0.0, it);
      launch_pcg_iter(ctx->stream, sd, ts.dv, ts.nv, fp32, ctx->lpr, one, it & 1);
      return;
    }
    {
      ProfScope ps(ctx, MFS_K_SPMV, 0.0, it);
      launch_cg_spmv(ctx->stream, sd, ts.dv, ts.nv, fp32, ctx->lpr, one);
    }
    ProfScope ps(ctx, MFS_K_CG_UPDATE);
    launch_cg_update(ctx->stream, sd, ts.dv, ts.nv, fp32, one);
  };
  if (ctx->use_graphs && ctx->prof_stride == 0 && G > 0 && (!pipe || G % 2 == 0)) {
    if (pipe && (start & 1) && run > 0) direct(start + done++);  // graphs start at even iterations
    hipGraphExec_t exec;
    MFS_TRY(cg_graph(ctx, sd, ts, fp32, G, one, pipe, &exec));
    for (; done + G <= run; done += G) {
      MFS_HIP(hipGraphLaunch(exec, ctx->stream));
      ctx->prof_launches[MFS_K_SPMV] += G;
      if (!pipe) ctx->prof_launches[MFS_K_CG_UPDATE] += G;
    }
  }
  for (; done < run; ++done) direct(start + done);
  return MFS_OK;
}

// ---- rigid-motion interpolation of handle poses (load stepping) ----

static void rot_log(const double R[9], double w[3]) {
  const double c = std::min(1.0, std::max(-1.0, 0.5 * (R[0] + R[4] + R[8] - 1.0)));
  const double th = std::acos(c);
  const double v[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};  // 2 sin(th) * axis
  if (th < 1e-6) {
    for (int i = 0; i < 3; ++i) w[i] = 0.5 * v[i];
    return;
  }
  if (M_PI - th < 1e-6) {  // axis from (R + I) / 2 = a a^T
    int k = 0;
    for (int i = 1; i < 3; ++i)
      if (R[4 * i] > R[4 * k]) k = i;
    double a[3];
    for (int i = 0; i < 3; ++i) a[i] = 0.5 * (R[3 * i + k] + (i == k ? 1.0 : 0.0));
    const double nrm = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    for (int i = 0; i < 3; ++i) w[i] = th * a[i] / nrm;
    return;
  }
  const double f = th / (2.0 * std::sin(th));
  for (int i = 0; i < 3; ++i) w[i] = f * v[i];
}

static void rot_exp(const double w[3], double R[9]) {
  const double th = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  const double K[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
  double K2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
  double a = 1.0, b = 0.5;  // sin(th)/th, (1 - cos(th))/th^2
  if (th > 1e-8) {
    a = std::sin(th) / th;
    b = (1.0 - std::cos(th)) / (th * th);
  }
  for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0 ? 1.0 : 0.0) + a * K[i] + b * K2[i];
}

// V(w) = I + (1 - cos th)/th^2 [w] + (th - sin th)/th^3 [w]^2, the
// translation part of the SE(3) exponential.
static void se3_V(const double w[3], double V[9]) {
  const double th = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  const double K[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
  double K2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
  double a = 0.5, b = 1.0 / 6.0;
  if (th > 1e-8) {
    a = (1.0 - std::cos(th)) / (th * th);
    b = (th - std::sin(th)) / (th * th * th);
  }
  for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0 ? 1.0 : 0.0) + a * K[i] + b * K2[i];
}

static void solve3(const double A[9], const double b[3], double x[3]) {  // Cramer's rule
  const double d = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                   A[2] * (A[3] * A[7] - A[4] * A[6]);
  for (int c = 0; c < 3; ++c) {
    double M[9];
    for (int i = 0; i < 9; ++i) M[i] = A[i];
    for (int r = 0; r < 3; ++r) M[3 * r + c] = b[r];
    x[c] = (M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
            M[2] * (M[3] * M[7] - M[4] * M[6])) / d;
  }
}

// Handle transforms a fraction tau of the way from (R0, t0) to (R1, t1)
// along each handle's screw motion, T(tau) = T0 exp(tau log(T0^-1 T1)) in
// SE(3): a rotation about a fixed joint keeps the joint fixed on the way.
int Engine::set_pose(int i, double tau) {
  SlotState& S = slot_[i];
  const int nh = S.ch->nh;
  S.tau = tau;
  if (tau >= 1.0) {
    S.Rc = S.R1;
    S.tc = S.t1;
  } else {
    S.Rc.assign(9 * nh, 0.0);
    S.tc.assign(3 * nh, 0.0);
    for (int h = 0; h < nh; ++h) {
      const double* A = &S.R0[9 * h];
      const double* B = &S.R1[9 * h];
      const double* a = &S.t0[3 * h];
      const double* bt = &S.t1[3 * h];
      double D[9], dt[3], w[3], v[3], V[9], E[9], Vt[9], te[3];
      for (int r = 0; r < 3; ++r) {  // relative motion: D = A^T B, dt = A^T (t1 - t0)
        for (int c = 0; c < 3; ++c) D[3 * r + c] = A[r] * B[c] + A[3 + r] * B[3 + c] + A[6 + r] * B[6 + c];
        dt[r] = A[r] * (bt[0] - a[0]) + A[3 + r] * (bt[1] - a[1]) + A[6 + r] * (bt[2] - a[2]);
      }
      rot_log(D, w);
      se3_V(w, V);
      solve3(V, dt, v);
      for (int k = 0; k < 3; ++k) {
        w[k] *= tau;
        v[k] *= tau;
      }
      rot_exp(w, E);
      se3_V(w, Vt);
      for (int r = 0; r < 3; ++r) te[r] = Vt[3 * r] * v[0] + Vt[3 * r + 1] * v[1] + Vt[3 * r + 2] * v[2];
      for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c)
          S.Rc[9 * h + 3 * r + c] = A[3 * r] * E[c] + A[3 * r + 1] * E[3 + c] + A[3 * r + 2] * E[6 + c];
        S.tc[3 * h + r] = A[3 * r] * te[0] + A[3 * r + 1] * te[1] + A[3 * r + 2] * te[2] + a[r];
      }
    }
  }
  return upload_pose(ctx_, S.ch, S.Rc.data(), S.tc.data());
}

// Start a new load step from the state in xb: the slot re-enters the mixed
// phase with a fresh warm start and restarted forcing.
int Engine::restart_load_step(int i) {
  SlotState& S = slot_[i];
  mfs_character* ch = S.ch;
  MFS_HIP(hipMemcpyAsync(ch->x.p, ch->xb.p, 3 * sizeof(double) * ch->n, hipMemcpyDeviceToDevice, ctx_->stream));
  S.phase = 0;
  S.fresh = true;
  S.load_mixed = 0;
  S.newton_prev = 0.0;
  S.E_known = false;
  Ctrl& c = ctx_->h_ctrl.data()[i];
  c.cg_g2prev = 0.0;
  c.cg_eta_min = 0.0;
  return MFS_OK;
}

int Engine::configure(const mfs_solve_opts* opts) {
  mfs_default_opts(&o_);
  if (opts) o_ = *opts;
  if (o_.precision != MFS_FP64 && o_.precision != MFS_FP32_REFINED)
    return set_error(MFS_E_INVALID, "unknown precision %d", o_.precision);
  if (o_.max_newton < 1 || o_.cg_max < 1 || !(o_.cg_tol >= 0.0) || !(o_.step_tol >= 0.0))
    return set_error(MFS_E_INVALID, "invalid solve options");
  if (o_.output_memory != MFS_MEM_HOST && o_.output_memory != MFS_MEM_DEVICE)
    return set_error(MFS_E_INVALID, "invalid output memory space");
  if (o_.warm_start != MFS_WARM_REST && o_.warm_start != MFS_WARM_PREVIOUS)
    return set_error(MFS_E_INVALID, "invalid warm-start option");
  fp32_ = o_.precision == MFS_FP32_REFINED;
  return MFS_OK;
}

int Engine::reserve(int n) {
  if (n < 1) return set_error(MFS_E_INVALID, "engine needs at least one slot");
  MFS_HIP(hipSetDevice(ctx_->device));
  MFS_HIP(hipStreamSynchronize(ctx_->stream));  // staging buffers may be reallocated
  MFS_TRY(ctx_->desc.reserve(n * sizeof(SysDesc)));
  MFS_TRY(ctx_->ctrl.reserve(n * sizeof(Ctrl)));
  MFS_TRY(ctx_->red.reserve(n * P_COUNT * sizeof(double)));
  MFS_TRY(ctx_->cg.reserve(n * sizeof(CgState)));
  ctx_->h_ctrl.assign(n, Ctrl{});
  MFS_TRY(ctx_->h_red.reserve(n * P_COUNT * sizeof(double)));
  MFS_TRY(ctx_->h_cg.reserve(n * sizeof(CgState)));
  MFS_TRY(ensure_stop_flags(ctx_, n));
  // arrival tickets start at zero (each kernel's last workgroup resets its own)
  MFS_HIP(hipMemsetAsync(ctx_->cg.p, 0, n * sizeof(CgState), ctx_->stream));
  slot_.assign(n, SlotState());
  hd_.assign(n, SysDesc{});
  desc_dirty_ = true;
  tiles_valid_ = false;
  for (int p = 0; p < 2; ++p) {
    live_[p].clear();
    launched_[p] = 0;
    gen_[p] = -1;
  }
  for (hipEvent_t e : queued_) ctx_->sync_events.push_back(e);
  queued_.clear();
  spans_.clear();
  gens_.clear();
  timed_.clear();
  return MFS_OK;
}

bool Engine::any_busy() const {
  for (const SlotState& s : slot_)
    if (s.used && !s.done) return true;
  return false;
}

int Engine::attach(int i, mfs_character* ch, const double* R, const double* t) {
  if (i < 0 || i >= (int)slot_.size() || slot_[i].used) return set_error(MFS_E_INVALID, "slot %d unavailable", i);
  // A character may come from another context on the same device (a server
  // lane runs on a context of its own); its frame then runs on this stream.
  if (!ch || ch->ctx->device != ctx_->device)
    return set_error(MFS_E_INVALID, "character is null or on another device");
  for (const SlotState& s : slot_)
    if (s.used && s.ch == ch) return set_error(MFS_E_INVALID, "character already has a frame in flight");
  MFS_TRY(check_pose(ch, R, t));
  const bool warm = o_.warm_start == MFS_WARM_PREVIOUS && ch->has_solution;
  if (!warm)
    MFS_HIP(hipMemcpyAsync(ch->x.p, ch->X.p, 3 * sizeof(double) * ch->n, hipMemcpyDeviceToDevice, ctx_->stream));
  MFS_HIP(hipMemcpyAsync(ch->xb.p, ch->x.p, 3 * sizeof(double) * ch->n, hipMemcpyDeviceToDevice, ctx_->stream));
  ch->has_solution = false;
  SlotState& S = slot_[i];
  S = SlotState();
  S.ch = ch;
  S.used = true;
  S.fresh = true;
  const int nh = ch->nh;
  S.R1.assign(R, R + 9 * nh);
  S.t1.assign(t, t + 3 * nh);
  if (warm && (int)ch->last_R.size() == 9 * nh) {
    S.R0 = ch->last_R;
    S.t0 = ch->last_t;
  } else {  // the rest shape is the solution of the identity pose
    S.R0.assign(9 * nh, 0.0);
    S.t0.assign(3 * nh, 0.0);
    for (int h = 0; h < nh; ++h) S.R0[9 * h] = S.R0[9 * h + 4] = S.R0[9 * h + 8] = 1.0;
  }
  MFS_TRY(set_pose(i, 1.0));
  tiles_valid_ = false;  // the slot's occupant changed
  SysDesc& d = hd_[i];
  d = ch->desc;
  d.ticket = ch->ntv > ctx_->allread_tiles ? 1 : 0;
  d.red = ctx_->red.as<double>() + P_COUNT * i;
  d.cg = ctx_->cg.as<CgState>() + i;
  d.ctrl = ctx_->ctrl.as<Ctrl>() + i;
  d.stop_flag = ctx_->d_stop + i;
  Ctrl& c = ctx_->h_ctrl.data()[i];
  std::memset(&c, 0, sizeof c);
  c.cg_tol2 = o_.cg_tol * o_.cg_tol;
  c.cg_adaptive = o_.cg_adaptive ? 1 : 0;
  desc_dirty_ = true;
  return MFS_OK;
}

int Engine::bind_workspace(int i, char* base) {
  if (i < 0 || i >= (int)slot_.size() || !slot_[i].used) return set_error(MFS_E_INVALID, "slot %d is empty", i);
  if (!base) return set_error(MFS_E_INVALID, "null workspace");
  SysDesc& d = hd_[i];
  double* red = d.red;
  mfs::bind_workspace(slot_[i].ch, base, &d);
  d.red = red;  // the slot's reduction row stays in the context
  desc_dirty_ = true;
  return MFS_OK;
}

int Engine::upload_desc() {
  if (!desc_dirty_) return MFS_OK;
  const int n = (int)slot_.size();
  MFS_TRY(ctx_->up.upload(ctx_->stream, ctx_->desc.p, hd_.data(), n * sizeof(SysDesc)));
  desc_dirty_ = false;
  return MFS_OK;
}

// The tile list is cached for the last (slot, character) set; a slot that
// changed occupant must never reuse its previous occupant's tile ranges.
int Engine::tiles_for(const std::vector<int>& ids) {
  std::vector<const mfs_character*> chars(ids.size());
  for (size_t k = 0; k < ids.size(); ++k) chars[k] = slot_[ids[k]].ch;
  if (tiles_valid_ && ids == tile_ids_ && chars == tile_chars_) return MFS_OK;
  std::vector<mfs_character*> by_slot(slot_.size(), nullptr);
  for (size_t i = 0; i < slot_.size(); ++i) by_slot[i] = slot_[i].ch;
  for (int i : ids)
    if (i < 0 || i >= (int)slot_.size() || !slot_[i].used || !slot_[i].ch)
      return set_error(MFS_E_INVALID, "tile list asked for empty slot %d", i);
  MFS_TRY(build_tile_list(ctx_, by_slot, ids, &ts_));
  tile_ids_ = ids;
  tile_chars_ = chars;
  tiles_valid_ = true;
  return MFS_OK;
}

int Engine::fp32_cap(const mfs_character* ch) const {
  if (o_.fp32_cg_max > 0) return std::min(o_.cg_max, o_.fp32_cg_max);
  return std::min(o_.cg_max, std::max(8000, (int)(100.0 * std::cbrt((double)ch->n))));
}

int Engine::run_cg(const std::vector<int>& act, bool fp32, std::vector<int>* failed,
                   const std::function<int()>& before_wait) {
  mfs_context* ctx = ctx_;
  const SysDesc* dsd = ctx->desc.as<SysDesc>();
  const int n = (int)slot_.size();
  const CgState* hg = ctx->h_cg.as<CgState>();
  int cit = 0;
  // launch set: the slots whose PCG still iterates.  It shrinks when stopped
  // systems hold a quarter of its tiles (or a system reaches its cap), so
  // the tiles of converged systems leave the grid, and a single remaining
  // system runs with its descriptor as the kernel argument.  A slot's
  // arithmetic does not depend on the set.
  std::vector<int> live = act;
  const SysDesc* one = live.size() == 1 ? &hd_[live[0]] : nullptr;
  // the pipelined form runs FP32 solves and FP64 solves; the FP64 re-solves
  // inside an FP32 solve keep the two-kernel form (started from the FP32
  // iterate), and the persistent kernel exists in the FP32 form only
  const bool pipe = ctx->pipelined && (fp32 || !fp32_);
  // per-slot iteration caps: the FP32 pass stops early where FP32 stalls
  std::vector<int> cap(slot_.size(), o_.cg_max);
  int max_cap = 0;
  for (int i : act) {
    cap[i] = failed ? fp32_cap(slot_[i].ch) : o_.cg_max;
    max_cap = std::max(max_cap, cap[i]);
  }
  std::vector<int> stopped_at(slot_.size(), -1);
  // algorithmic bytes of one SpMV-family launch over the slots still in
  // PCG, for the profiler's roofline figures: the least a block-sparse
  // product must move, every block value and column index, the row
  // pointers, one input and one output vector (nnzb (9w + 4) + 4 (n + 1) +
  // 6 w n, w the solve's word size); the pipelined form fuses the PCG
  // vector work and the block-Jacobi preconditioner into the same launch,
  // which adds twelve passes over 3n values and the 6 preconditioner values
  // per row (42 w n)
  const double word = fp32 ? 4.0 : 8.0;
  const double per_row = pipe ? (6.0 + 42.0) * word : 6.0 * word;
  // A launch at iteration index `it` does work for a slot whose PCG had not
  // stopped before it (a stopped slot's launches return at once).
  auto attribute_bytes = [&]() {
    for (ProfPending& p : ctx->pending) {
      if (p.fam != MFS_K_SPMV || p.tag < 0) continue;
      double by = 0.0;
      for (int i : act)
        if (!hg[i].done || p.tag < hg[i].iters) {
          const mfs_character* c = slot_[i].ch;
          by += c->nnzb * (9.0 * word + 4.0) + (c->n + 1) * 4.0 + c->n * per_row;
        }
      p.bytes = by;
      p.tag = -1;
    }
  };
  if (pipe) {
    // iteration j runs with parity j & 1 here (a slot that last solved in
    // the asynchronous form may carry another offset)
    for (int i : act)
      if (hd_[i].par0 != 0) {
        hd_[i].par0 = 0;
        desc_dirty_ = true;
      }
    MFS_TRY(upload_desc());
    ProfScope ps(ctx, MFS_K_OTHER);
    launch_pcg_start(ctx->stream, dsd, ts_.dv, ts_.nv, fp32, ctx->lpr, one);
  }
  // Persistent form: when the device holds every workgroup of the set at
  // once, the whole solve is one cooperative launch that stops each system
  // at its convergence, breakdown or cap (Ctrl::cg_cap) by itself.
  if (pipe && fp32 && ctx->persistent) {
    int maxb = 0;
    for (int i : act) maxb = std::max(maxb, slot_[i].ch->max_tile_blocks);
    const size_t lds = pcg_persist_lds(maxb);
    if (ctx->persist_lpr != ctx->lpr || ctx->persist_lds != lds) {
      ctx->persist_capacity = pcg_persist_capacity(ctx->lpr, lds);
      ctx->persist_lpr = ctx->lpr;
      ctx->persist_lds = lds;
    }
    if (ts_.nv <= ctx->persist_capacity) {
      constexpr int kPersistTag = -2;
      {
        ProfScope ps(ctx, MFS_K_SPMV, 0.0, kPersistTag);
        MFS_HIP(launch_pcg_persist(ctx->stream, dsd, ts_.dv, ts_.nv, ctx->lpr, lds));
      }
      MFS_TRY(read_cg(ctx, n, false));
      // algorithmic bytes: those of one pipelined launch (FP32, above) per
      // iteration, as for the per-launch form (the persistent kernel keeps
      // the matrix rows in LDS and moves less)
      for (ProfPending& p : ctx->pending) {
        if (p.fam != MFS_K_SPMV || p.tag != kPersistTag) continue;
        double by = 0.0;
        for (int i : act) {
          const mfs_character* c = slot_[i].ch;
          by += (double)hg[i].iters * (c->nnzb * (9.0 * 4.0 + 4.0) + (c->n + 1) * 4.0 + c->n * 48.0 * 4.0);
        }
        p.bytes = by;
        p.tag = -1;
      }
      prof_resolve(ctx);
      for (int i : act) {
        if (hg[i].abort)
          return set_error(MFS_E_HIP, "persistent PCG: a barrier wait timed out (slot %d)", i);
        const bool ok = hg[i].done == 1;
        slot_[i].cg += hg[i].iters;
        if (!fp32 && fp32_) slot_[i].cg_resolve += hg[i].iters;
        if (ok) continue;
        if (failed)
          failed->push_back(i);
        else
          slot_[i].cg_fail++;
      }
      ProfScope ps(ctx, MFS_K_OTHER);
      launch_cg_finish(ctx->stream, dsd, ts_.dv, ts_.nv, 0);
      return MFS_OK;
    }
  }
  // PCG in chunks: first_check iterations, then min_run (at most max_run),
  // one chunk queued ahead of the running one.  The PCG kernels store the
  // solve's epoch to a system's host-mapped stop flag when it stops; the
  // host polls the flags and the oldest chunk's completion event, so the
  // device never idles waiting for the host between chunks, and after the
  // last stop only the queued launches run (they return at once).  The
  // stream is synchronised only to shrink the launch set.
  const int32_t epoch = cg_epoch_;
  const int32_t* flag = ctx->h_stop;
  auto stopped = [&](int i) { return __atomic_load_n(flag + i, __ATOMIC_ACQUIRE) == epoch; };
  const int steady = std::max(1, std::min(ctx->cg_min_run, ctx->cg_max_run));
  std::deque<std::pair<int, hipEvent_t>> queued;  // (iterations enqueued after the chunk, its completion)
  auto enqueue = [&](int run) -> int {
    MFS_TRY(enqueue_cg(ctx, dsd, ts_, fp32, run, one, pipe, cit));
    cit += run;
    MFS_HIP(hipGetLastError());
    hipEvent_t e = nullptr;
    MFS_TRY(sync_event(ctx, &e));
    MFS_HIP(hipEventRecord(e, ctx->stream));
    queued.emplace_back(cit, e);
    return MFS_OK;
  };
  auto drain = [&]() -> int {
    MFS_TRY(wait_stream(ctx));
    for (auto& qe : queued) ctx->sync_events.push_back(qe.second);
    queued.clear();
    return MFS_OK;
  };
  int live_tiles = ts_.nv;
  if (max_cap > 0) MFS_TRY(enqueue(std::min(ctx->cg_first_run, max_cap)));
  while (!queued.empty()) {
    if (cit < max_cap && queued.size() < 2) MFS_TRY(enqueue(std::min(steady, max_cap - cit)));
    bool all = false, shrink = false, front_done = false;
    PollPacer pacer;
    for (;;) {
      all = true;
      int stopped_tiles = 0;
      for (int i : live) {
        if (stopped(i))
          stopped_tiles += slot_[i].ch->ntv;
        else
          all = false;
      }
      shrink = live.size() > 1 && 4 * stopped_tiles >= live_tiles;
      const hipError_t e = hipEventQuery(queued.front().second);
      if (e != hipSuccess && e != hipErrorNotReady) return set_error(MFS_E_HIP, "PCG chunk: %s", hipGetErrorString(e));
      front_done = e == hipSuccess;
      if (all || shrink || front_done) break;
      if (!pacer.pace())
        return set_error(MFS_E_HIP, "PCG chunk: no stop flag and no completed chunk in %d s",
                         PollPacer::kLimitSeconds);
    }
    if (all) break;
    if (front_done) {
      ctx->sync_events.push_back(queued.front().second);
      queued.pop_front();
    }
    bool capped = false;
    for (int i : live)
      if (!stopped(i) && cit >= cap[i]) capped = true;
    if (shrink || capped) {
      MFS_TRY(drain());
      std::vector<int> still;
      for (int i : live) {
        if (stopped(i)) continue;
        if (cit >= cap[i]) {  // this slot's cap: stop iterating it
          stopped_at[i] = cit;
          continue;
        }
        still.push_back(i);
      }
      if (still.empty()) break;
      if (still.size() < live.size()) {
        live.swap(still);
        MFS_TRY(tiles_for(live));  // the stream is idle
        one = live.size() == 1 ? &hd_[live[0]] : nullptr;
        live_tiles = ts_.nv;
      }
      if (cit < max_cap) MFS_TRY(enqueue(std::min(steady, max_cap - cit)));
    }
  }
  // The PCG state to the host (behind every queued chunk), the iterates into
  // dx (FP64; a pipelined iterate is FP64 already), and the caller's next
  // work, all queued before the host waits for the state: the GPU goes on
  // while the host reads it.
  MFS_HIP(hipMemcpyAsync(ctx->h_cg.p, ctx->cg.p, n * sizeof(CgState), hipMemcpyDeviceToHost, ctx->stream));
  hipEvent_t state_read = nullptr;
  MFS_TRY(sync_event(ctx, &state_read));
  MFS_HIP(hipEventRecord(state_read, ctx->stream));
  if (live.size() != act.size()) MFS_TRY(tiles_for(act));
  {
    ProfScope ps(ctx, MFS_K_OTHER);
    launch_cg_finish(ctx->stream, dsd, ts_.dv, ts_.nv, pipe ? 0 : fp32);
  }
  MFS_HIP(hipGetLastError());
  if (before_wait) MFS_TRY(before_wait());
  MFS_TRY(wait_event(ctx, state_read));
  for (auto& qe : queued) ctx->sync_events.push_back(qe.second);
  queued.clear();
  attribute_bytes();
  prof_resolve(ctx);
  for (int i : act) {
    const bool ok = hg[i].done == 1;
    const int ran = hg[i].done ? hg[i].iters : (stopped_at[i] >= 0 ? stopped_at[i] : cit);
    slot_[i].cg += ran;
    if (!fp32 && fp32_) slot_[i].cg_resolve += ran;
    if (ok) continue;
    if (failed)
      failed->push_back(i);
    else
      slot_[i].cg_fail++;
  }
  return MFS_OK;
}

// first pass: Newton slots evaluate E at {0, 1, 1/2, 1/4, 1/8}; mixed slots
// get the halving count their worst tet needs
void Engine::ls_setup(const std::vector<int>& act) {
  Ctrl* hc = ctx_->h_ctrl.data();
  for (int i : act) {
    slot_[i].alpha = 0.0;
    hc[i].phase = slot_[i].phase;
    hc[i].trials[0] = 0.0;
    for (int j = 1; j < kNumTrials; ++j) hc[i].trials[j] = std::ldexp(1.0, -(j - 1));
  }
}

int Engine::ls_queue(const std::vector<int>& act) {
  mfs_context* ctx = ctx_;
  hipStream_t st = ctx->stream;
  const int n = (int)slot_.size();
  ls_setup(act);
  MFS_TRY(tiles_for(act));
  MFS_TRY(upload_ctrl(ctx, n));
  {
    ProfScope ps(ctx, MFS_K_LINESEARCH);
    launch_linesearch(st, ctx->desc.as<SysDesc>(), ctx->ctrl.as<Ctrl>(), ts_.dt, ts_.nt, ts_.dv, ts_.nv);
  }
  {
    ProfScope ps(ctx, MFS_K_OTHER);
    launch_finalize(st, ctx->desc.as<SysDesc>(), ctx->sys_ids.as<int32_t>(), (int)act.size());
  }
  MFS_HIP(hipGetLastError());
  MFS_HIP(hipMemcpyAsync(ctx->h_red.p, ctx->red.p, n * P_COUNT * sizeof(double), hipMemcpyDeviceToHost, st));
  MFS_TRY(sync_event(ctx, &ls_event_));
  MFS_HIP(hipEventRecord(ls_event_, st));
  return MFS_OK;
}

int Engine::linesearch(const std::vector<int>& act) {
  mfs_context* ctx = ctx_;
  hipStream_t st = ctx->stream;
  const SysDesc* dsd = ctx->desc.as<SysDesc>();
  const Ctrl* dctrl = ctx->ctrl.as<Ctrl>();
  Ctrl* hc = ctx->h_ctrl.data();
  const double* hr = ctx->h_red.as<double>();
  const int n = (int)slot_.size();
  const bool queued = ls_event_ != nullptr;  // the first pass is on its way (ls_queue)
  if (!queued) ls_setup(act);
  std::vector<int> srch = act;
  bool first_pass = true;
  while (!srch.empty()) {
    if (first_pass && queued) {
      const hipEvent_t e = ls_event_;
      ls_event_ = nullptr;
      MFS_TRY(wait_event(ctx, e));
      prof_resolve(ctx);
    } else {
      MFS_TRY(tiles_for(srch));
      MFS_TRY(upload_ctrl(ctx, n));
      {
        ProfScope ps(ctx, MFS_K_LINESEARCH);
        launch_linesearch(st, dsd, dctrl, ts_.dt, ts_.nt, ts_.dv, ts_.nv);
      }
      {
        ProfScope ps(ctx, MFS_K_OTHER);
        launch_finalize(st, dsd, ctx->sys_ids.as<int32_t>(), (int)srch.size());
      }
      MFS_HIP(hipGetLastError());
      MFS_TRY(read_red(ctx, n, first_pass ? ls_fill_ : std::function<int()>()));
    }
    std::vector<int> next;
    for (int i : srch) {
      SlotState& S = slot_[i];
      const double* rd = hr + P_COUNT * i;
      if (first_pass) {
        // forcing state for the next Newton step (Eisenstat-Walker safeguard)
        const double eta = std::sqrt(pcg_tol2(hc[i], rd[P_BB]));
        const double sg = 0.9 * eta * eta;
        hc[i].cg_eta_min = sg > 0.1 ? sg : 0.0;
        hc[i].cg_g2prev = rd[P_BB];
        S.grad = std::sqrt(rd[P_BB]);
        S.relres = rd[P_BB] > 0.0 ? std::sqrt(rd[P_RR] / rd[P_BB]) : 0.0;
        S.clamped = (int)rd[P_CLAMP];
        S.step = rd[P_DXMAX];  // scaled by alpha after the update
      }
      if (S.phase == 0) {
        const int h = (int)rd[P_HMAX];
        if (h <= 40) {
          S.alpha = std::ldexp(1.0, -h);
          S.halvings += h;
        }
        continue;
      }
      int j0 = 0;
      if (first_pass) {
        S.E = rd[P_INF0] > 0.0 ? INFINITY : rd[P_E0] + rd[P_PIN0];
        S.E_known = true;
        j0 = 1;
      }
      const double slope = -rd[P_SLOPE];  // grad E . dx, with b = -grad E
      const double E0 = S.E;
      bool acc = false;
      for (int j = j0; j < kNumTrials && !acc; ++j) {
        const double a = hc[i].trials[j];
        if (rd[P_INF0 + j] > 0.0) continue;
        const double Ej = rd[P_E0 + j] + rd[P_PIN0 + j];
        if (std::isfinite(E0) && Ej <= E0 + 1e-4 * a * slope + 1e-12 * std::fabs(E0)) {
          acc = true;
          S.alpha = a;
          S.E = Ej;
          S.halvings += (int)std::lround(-std::log2(a));
        }
      }
      if (!acc) {
        const double last = hc[i].trials[kNumTrials - 1];
        if (last > std::ldexp(1.0, -40) && std::isfinite(E0)) {
          for (int j = 0; j < kNumTrials; ++j) hc[i].trials[j] = last * std::ldexp(1.0, -(j + 1));
          next.push_back(i);
        }
      }
    }
    srch.swap(next);
    first_pass = false;
  }
  return MFS_OK;
}

int Engine::step() {
  mfs_context* ctx = ctx_;
  hipStream_t st = ctx->stream;
  MFS_HIP(hipSetDevice(ctx->device));
  const int n = (int)slot_.size();
  const SysDesc* dsd = ctx->desc.as<SysDesc>();
  const Ctrl* dctrl = ctx->ctrl.as<Ctrl>();
  Ctrl* hc = ctx->h_ctrl.data();
  const double* hr = ctx->h_red.as<double>();
  for (int i = 0; i < n; ++i)
    if (slot_[i].used && !slot_[i].done && !hd_[i].blk)
      return set_error(MFS_E_INVALID, "slot %d has no workspace bound", i);
  MFS_TRY(upload_desc());

  // mixed warm start of newly attached slots: s0 = stretch factor of F(x0)
  std::vector<int> fresh;
  for (int i = 0; i < n; ++i)
    if (slot_[i].used && slot_[i].fresh) fresh.push_back(i);
  if (!fresh.empty()) {
    MFS_TRY(tiles_for(fresh));
    {
      ProfScope ps(ctx, MFS_K_WARM_START);
      launch_warm_start(st, dsd, ts_.dt, ts_.nt, fp32_);
    }
    {
      ProfScope ps(ctx, MFS_K_OTHER);
      launch_finalize(st, dsd, ctx->sys_ids.as<int32_t>(), (int)fresh.size());
    }
    MFS_HIP(hipGetLastError());
    MFS_TRY(read_red(ctx, n));
    for (int i : fresh) {
      slot_[i].routed = (int)hr[P_COUNT * i + P_ROUTED];
      slot_[i].fresh = false;
    }
  }

  std::vector<int> act;
  for (int i = 0; i < n; ++i)
    if (slot_[i].used && !slot_[i].done) act.push_back(i);
  if (act.empty()) return MFS_OK;
  MFS_TRY(tiles_for(act));
  for (int i : act) {
    hc[i].phase = slot_[i].phase;
    hc[i].update_s = 0;
    hc[i].alpha = 0.0;
    // inexact Newton only on the constraint: mixed-phase solves use the floor
    // tolerance (a loose mixed step can leave the positive-definite cone in
    // single tets and stall the mixed line search)
    hc[i].cg_adaptive = (o_.cg_adaptive && slot_[i].phase == 1) ? 1 : 0;
    hc[i].cg_eta_max = slot_[i].check_next ? kCheckEta : 0.0;
    slot_[i].check_next = false;
    hc[i].cg_cap = fp32_ ? fp32_cap(slot_[i].ch) : o_.cg_max;
  }
  cg_epoch_ = ++ctx->cg_epoch;
  for (int i : act) hc[i].cg_epoch = cg_epoch_;
  MFS_TRY(upload_ctrl(ctx, n));
  {
    ProfScope ps(ctx, MFS_K_ELEMENT);
    launch_element(st, dsd, dctrl, ts_.dt, ts_.nt, fp32_);
  }
  {
    ProfScope ps(ctx, MFS_K_ASSEMBLE);
    launch_assemble(st, dsd, ts_.ds, ts_.ns, fp32_);
  }
  {
    ProfScope ps(ctx, MFS_K_OTHER);
    if (ctx->pipelined && fp32_)
      launch_pcg_init(st, dsd, ts_.dv, ts_.nv, fp32_);
    else
      launch_cg_init(st, dsd, ts_.dv, ts_.nv, fp32_);
  }
  MFS_HIP(hipGetLastError());
  std::vector<int> redo;
  // the first line-search pass is queued behind the PCG run, so the GPU
  // does not wait for the host to read the PCG state; it is dropped when
  // some Newton system needs its FP64 re-solve
  MFS_TRY(run_cg(act, fp32_, fp32_ ? &redo : nullptr, [&]() { return ls_queue(act); }));
  if (!redo.empty() && ls_event_) {
    const hipEvent_t e = ls_event_;
    ls_event_ = nullptr;
    MFS_TRY(wait_event(ctx, e));
    prof_resolve(ctx);
  }
  if (!redo.empty()) {
    // FP32 could not solve these Newton systems (ill-conditioned beyond
    // single precision): element records, assembly and PCG again in FP64,
    // the PCG started from the FP32 iterate (left in dx by run_cg) rather
    // than from zero
    MFS_TRY(tiles_for(redo));
    cg_epoch_ = ++ctx->cg_epoch;
    for (int i : redo) hc[i].cg_epoch = cg_epoch_;
    MFS_TRY(upload_ctrl(ctx, n));
    {
      ProfScope ps(ctx, MFS_K_ELEMENT);
      launch_element(st, dsd, dctrl, ts_.dt, ts_.nt, 0);
    }
    {
      ProfScope ps(ctx, MFS_K_ASSEMBLE);
      launch_assemble(st, dsd, ts_.ds, ts_.ns, 0);
    }
    {
      ProfScope ps(ctx, MFS_K_OTHER);
      launch_cg_init(st, dsd, ts_.dv, ts_.nv, 0, /*warm=*/1);
    }
    MFS_HIP(hipGetLastError());
    MFS_TRY(run_cg(redo, false, nullptr));
    for (int i : redo) slot_[i].resolves++;
  }
  MFS_TRY(linesearch(act));
  MFS_TRY(apply_update(act));
  for (int i : act) MFS_TRY(finish_newton(i));
  return MFS_OK;
}

int Engine::apply_update(const std::vector<int>& act) {
  mfs_context* ctx = ctx_;
  Ctrl* hc = ctx->h_ctrl.data();
  for (int i : act) {
    hc[i].alpha = slot_[i].alpha;
    hc[i].update_s = (slot_[i].phase == 0 && slot_[i].alpha > 0.0 && slot_[i].alpha < 1.0) ? 1 : 0;
    hc[i].phase = slot_[i].phase;
  }
  MFS_TRY(tiles_for(act));
  MFS_TRY(upload_ctrl(ctx, (int)slot_.size()));
  {
    ProfScope ps(ctx, MFS_K_UPDATE);
    launch_update(ctx->stream, ctx->desc.as<SysDesc>(), ctx->ctrl.as<Ctrl>(), ts_.dt, ts_.nt, ts_.dv, ts_.nv);
  }
  MFS_HIP(hipGetLastError());
  return MFS_OK;
}

int Engine::finish_newton(int i) {
  Ctrl* hc = ctx_->h_ctrl.data();
  const bool loadstep = o_.load_bisections > 0 && !o_.fixed_newton;
  SlotState& S = slot_[i];
  const bool was_newton = S.phase == 1;
  S.iters++;
  S.step = S.alpha * S.step;
  if (!was_newton) {
    S.mixed++;
    S.load_mixed++;
    S.E_known = false;
  }
  const bool stalled = S.alpha == 0.0 || (!was_newton && S.alpha < 1.0 && S.load_mixed > 6);
  if (stalled && loadstep && S.bisections < o_.load_bisections && S.iters < o_.max_newton) {
    // back to the last converged pose; approach the target in a shorter step
    S.bisections++;
    S.delta *= 0.5;
    MFS_TRY(restart_load_step(i));
    MFS_TRY(set_pose(i, S.tau_done + S.delta));
    return MFS_OK;
  }
  if (S.alpha == 0.0) {  // line search failed: keep the iterate
    S.done = true;
    S.status = MFS_W_NOT_CONVERGED;
    return MFS_OK;
  }
  if (!was_newton && S.alpha == 1.0) {
    S.phase = 1;
    hc[i].cg_g2prev = 0.0;  // forcing restarts at the first Newton-phase step
    hc[i].cg_eta_min = 0.0;
  }
  const bool final_pose = S.tau >= 1.0;
  const double tol = final_pose ? o_.step_tol : 1e-4;
  // Step test.  Near a solution where clamped element Hessians remain, Newton
  // converges only linearly, at the rate rho of successive full steps; the
  // distance left is then about step * rho / (1 - rho), which exceeds the
  // step once rho > 1/2, so the step must be that much shorter.  Steps below
  // 1/20 of the tolerance pass whatever their ratio (rounding-level steps).
  // Intermediate poses of load stepping keep the plain test.
  double need = tol * S.ch->bbox_diag;
  const bool full = was_newton && S.alpha == 1.0;
  const double rho = full && S.newton_prev > 0.0 ? S.step / S.newton_prev : NAN;
  if (final_pose && full && S.newton_prev > 0.0 && S.step > 0.05 * need) {
    if (rho >= 1.0)
      need = 0.0;
    else if (rho > 0.5)
      need *= (1.0 - rho) / rho;
  }
  S.newton_prev = full ? S.step : 0.0;
  // A short step also says little when its PCG stopped on a loose forcing
  // term (near 0.1 when the gradient stalls): the solve can leave a soft
  // mode of the Newton step unsolved, so the steps shrink while the
  // iterate stays where it is.  A stop after a solve looser than the check
  // tolerance is taken only after one more step whose forcing term is at
  // most that tolerance.
  const bool check = final_pose && was_newton && o_.cg_adaptive && S.relres > kCheckEta;
  if (o_.fixed_newton) {
    if (S.iters >= o_.max_newton) S.done = true;
  } else if (was_newton && S.step <= need && check) {
    S.check_next = true;
  } else if (was_newton && S.step <= need) {
    if (final_pose) {
      S.done = true;
    } else {  // intermediate pose reached: keep it, lengthen the next step
      MFS_HIP(hipMemcpyAsync(S.ch->xb.p, S.ch->x.p, 3 * sizeof(double) * S.ch->n, hipMemcpyDeviceToDevice,
                             ctx_->stream));
      S.tau_done = S.tau;
      S.delta *= 2.0;
      MFS_TRY(restart_load_step(i));
      MFS_TRY(set_pose(i, std::min(1.0, S.tau_done + S.delta)));
    }
  }
  // The step that will likely be the last (this one times its contraction
  // rate, at least 0.1, is within the tolerance) is solved to the check
  // tolerance at once, so that a stop after it needs no extra check step.
  if (!S.done && !o_.fixed_newton && final_pose && was_newton && o_.cg_adaptive && S.phase == 1) {
    const double r = rho < 1.0 ? std::max(rho, 0.1) : 1.0;  // no rate yet: as if 1
    if (S.step * r <= tol * S.ch->bbox_diag) S.check_next = true;
  }
  if (!S.done && S.iters >= o_.max_newton) {
    S.done = true;
    S.status = MFS_W_NOT_CONVERGED;
  }
  return MFS_OK;
}

int Engine::finish_energies() {
  const int n = (int)slot_.size();
  std::vector<int> need;
  for (int i = 0; i < n; ++i)
    if (slot_[i].used && slot_[i].done && !slot_[i].E_known) need.push_back(i);
  if (need.empty()) return MFS_OK;
  mfs_context* ctx = ctx_;
  Ctrl* hc = ctx->h_ctrl.data();
  MFS_TRY(upload_desc());
  MFS_TRY(tiles_for(need));
  for (int i : need) {
    hc[i].phase = 1;
    for (int j = 0; j < kNumTrials; ++j) hc[i].trials[j] = 0.0;
  }
  MFS_TRY(upload_ctrl(ctx, n));
  launch_linesearch(ctx->stream, ctx->desc.as<SysDesc>(), ctx->ctrl.as<Ctrl>(), ts_.dt, ts_.nt, ts_.dv, ts_.nv);
  launch_finalize(ctx->stream, ctx->desc.as<SysDesc>(), ctx->sys_ids.as<int32_t>(), (int)need.size());
  MFS_HIP(hipGetLastError());
  MFS_TRY(read_red(ctx, n));
  const double* hr = ctx->h_red.as<double>();
  for (int i : need) {
    const double* rd = hr + P_COUNT * i;
    slot_[i].E = rd[P_INF0] > 0.0 ? INFINITY : rd[P_E0] + rd[P_PIN0];
    slot_[i].E_known = true;
  }
  return MFS_OK;
}

int Engine::output(int i, double* x_out, int mem) {
  mfs_character* ch = slot_[i].ch;
  hipStream_t st = ctx_->stream;
  if (mem == MFS_MEM_DEVICE) {
    launch_scatter_rows(st, ch->x.as<double>(), ch->perm_d.as<int32_t>(), ch->n, 3, 1.0, x_out);
  } else {
    double* stage = static_cast<double*>(hd_[i].r);  // the slot's PCG residual, free after the solve
    launch_scatter_rows(st, ch->x.as<double>(), ch->perm_d.as<int32_t>(), ch->n, 3, 1.0, stage);
    MFS_HIP(hipMemcpyAsync(x_out, stage, 3 * sizeof(double) * ch->n, hipMemcpyDeviceToHost, st));
  }
  MFS_HIP(hipGetLastError());
  MFS_HIP(hipStreamSynchronize(st));
  prof_resolve(ctx_);
  ch->has_solution = true;
  ch->last_R = slot_[i].R1;
  ch->last_t = slot_[i].t1;
  return MFS_OK;
}

void Engine::stats(int i, mfs_solve_stats* s) const {
  const SlotState& S = slot_[i];
  s->status = S.status;
  s->iterations = S.iters;
  s->mixed_iterations = S.mixed;
  s->cg_iterations = S.cg;
  s->halvings = S.halvings;
  s->clamped = S.clamped;
  s->fp64_routed = S.routed;
  s->cg_not_converged = S.cg_fail;
  s->fp64_resolves = S.resolves;
  s->fp64_resolve_cg_iterations = S.cg_resolve;
  s->energy = S.E;
  s->grad_norm = S.grad;
  s->last_step = S.step;
  s->cg_rel_residual = S.relres;
}

}  // namespace mfs
