// Newton driver of the per-frame solve (Algorithm 1, one pose per call) for
// one character or a batch of characters.
//
// Per iteration, for every character still iterating: element pass ->
// assembly -> PCG -> line search -> update, each a single launch over the
// tiles of all those characters.  The host reads back only per-character
// scalars: PCG convergence flags every few iterations and the line-search
// results once per iteration.
//
// Iteration (state x, s; s is the mixed stretch variable):
//   solve K(s) dx = -[grad C(x) + sum_k W_k J_k^T (g_k(s) + H_k(s)(J_k x - s_k))]
//   mixed phase (s != J x): alpha = the step the worst neo-Hookean tet allows
//     along s + alpha (J(x + dx) - s) while staying positive definite
//     (halvings of 1); s <- s + alpha (J(x + dx) - s); alpha = 1 lands on the
//     constraint s = J x and starts the Newton phase.
//   Newton phase (s = J x): Armijo on E, E(x + a dx) <= E(x) + 1e-4 a gradE.dx
//     + 1e-12 |E(x)|, with every neo-Hookean stretch positive definite.
//   stop: fixed iteration count, or a Newton-phase step with
//     max_v |alpha dx_v| <= step_tol * bbox diagonal.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"
#include "launch.h"

namespace mfs {

int check_pose(const mfs_character* ch, const double* R, const double* t) {
  if (!R || !t) return set_error(MFS_E_INVALID, "null handle transforms");
  for (int h = 0; h < ch->nh; ++h) {
    const double* r = R + 9 * h;
    for (int i = 0; i < 9; ++i)
      if (!std::isfinite(r[i])) return set_error(MFS_E_INVALID, "handle %d: non-finite rotation", h);
    for (int i = 0; i < 3; ++i)
      if (!std::isfinite(t[3 * h + i])) return set_error(MFS_E_INVALID, "handle %d: non-finite translation", h);
    double err = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double v = r[i] * r[j] + r[3 + i] * r[3 + j] + r[6 + i] * r[6 + j] - (i == j ? 1.0 : 0.0);
        err += v * v;
      }
    const double det = r[0] * (r[4] * r[8] - r[5] * r[7]) - r[1] * (r[3] * r[8] - r[5] * r[6]) +
                       r[2] * (r[3] * r[7] - r[4] * r[6]);
    if (std::sqrt(err) > 1e-9 || !(det > 0.0))
      return set_error(MFS_E_INVALID, "handle %d: not a rotation (|R^T R - I| = %.3g, det = %.6g)", h, std::sqrt(err), det);
  }
  return MFS_OK;
}

int upload_pose(mfs_character* ch, const double* R, const double* t) {
  hipStream_t st = ch->ctx->stream;
  MFS_HIP(hipMemcpyAsync(ch->Rh.p, R, 9 * sizeof(double) * ch->nh, hipMemcpyHostToDevice, st));
  MFS_HIP(hipMemcpyAsync(ch->th.p, t, 3 * sizeof(double) * ch->nh, hipMemcpyHostToDevice, st));
  return MFS_OK;
}

namespace {

struct HostSys {
  mfs_character* ch = nullptr;
  int phase = 0;  // 0 mixed, 1 Newton
  bool done = false;
  int status = MFS_OK;
  int iters = 0, mixed = 0, cg = 0, halvings = 0, clamped = 0, routed = 0, cg_fail = 0;
  double E = INFINITY;
  bool E_known = false;
  double grad = NAN, step = NAN, relres = NAN;
  // PCG residual history (run sizing)
  double rho_prev = -1.0;
  int it_prev = 0;
  // line search
  bool searching = false;
  double alpha = 0.0;
  int pass = 0;
};

enum TileKind { kVert = 0, kTet = 1, kSlot = 2 };

struct TileSet {
  int nv = 0, nt = 0, ns = 0;
  Tile* dv = nullptr;
  Tile* dt = nullptr;
  Tile* ds = nullptr;
};

// Tiles of the listed systems (indices into the batch), uploaded to the
// context's tile buffer.  The caller has synchronised the stream, so the
// pinned staging area is free.
int build_tiles(mfs_context* ctx, const std::vector<HostSys>& sys, const std::vector<int>& ids, TileSet* ts) {
  size_t total = 0;
  for (int i : ids) total += sys[i].ch->ntv + sys[i].ch->ntt + sys[i].ch->nts;
  MFS_TRY(ctx->h_tiles.reserve(std::max<size_t>(total, 1) * sizeof(Tile)));
  MFS_TRY(ctx->tiles.reserve(std::max<size_t>(total, 1) * sizeof(Tile)));
  Tile* h = ctx->h_tiles.as<Tile>();
  size_t pos = 0;
  int counts[3] = {0, 0, 0};
  for (int kind = 0; kind < 3; ++kind) {
    for (int i : ids) {
      const mfs_character* c = sys[i].ch;
      const int total_items = kind == kVert ? c->n : (kind == kTet ? c->m : c->nnzb);
      const int nt = kind == kVert ? c->ntv : (kind == kTet ? c->ntt : c->nts);
      const int size = kind == kVert ? kVTile : (kind == kTet ? kTTile : kSTile);
      for (int j = 0; j < nt; ++j) {
        h[pos++] = Tile{i, j * size, std::min(total_items, (j + 1) * size), j};
        counts[kind]++;
      }
    }
  }
  MFS_HIP(hipMemcpyAsync(ctx->tiles.p, h, pos * sizeof(Tile), hipMemcpyHostToDevice, ctx->stream));
  Tile* d = ctx->tiles.as<Tile>();
  ts->nv = counts[0];
  ts->nt = counts[1];
  ts->ns = counts[2];
  ts->dv = d;
  ts->dt = d + counts[0];
  ts->ds = d + counts[0] + counts[1];
  // system ids for the finalize kernel
  MFS_TRY(ctx->sys_ids.reserve(std::max<size_t>(ids.size(), 1) * sizeof(int32_t)));
  MFS_TRY(ctx->h_stage.reserve(std::max<size_t>(ids.size(), 1) * sizeof(int32_t)));
  std::memcpy(ctx->h_stage.p, ids.data(), ids.size() * sizeof(int32_t));
  MFS_HIP(hipMemcpyAsync(ctx->sys_ids.p, ctx->h_stage.p, ids.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                         ctx->stream));
  return MFS_OK;
}

int upload_ctrl(mfs_context* ctx, int count) {
  MFS_HIP(hipMemcpyAsync(ctx->ctrl.p, ctx->h_ctrl.p, count * sizeof(Ctrl), hipMemcpyHostToDevice, ctx->stream));
  return MFS_OK;
}

int read_flags(mfs_context* ctx, int count) {
  MFS_HIP(hipMemcpyAsync(ctx->h_flags.p, ctx->flags.p, count * F_COUNT * sizeof(int32_t), hipMemcpyDeviceToHost,
                         ctx->stream));
  MFS_HIP(hipMemcpyAsync(ctx->h_cgres.p, ctx->cgres.p, count * 2 * sizeof(double), hipMemcpyDeviceToHost,
                         ctx->stream));
  MFS_HIP(hipStreamSynchronize(ctx->stream));
  prof_resolve(ctx);
  return MFS_OK;
}

// A run of PCG iterations captured once as a HIP graph per (tiles, sizes,
// tolerance, precision) and replayed; the kernels take no per-iteration
// arguments (the iteration index lives in device memory).
int cg_graph(mfs_context* ctx, const SysDesc* sd, const TileSet& ts, int fp32, int iters, const SysDesc* one,
             hipGraphExec_t* out) {
  for (CgGraph& g : ctx->graphs) {
    if (g.sd == sd && g.tiles == ts.dv && g.ntv == ts.nv && g.fp32 == fp32 &&
        g.lpr == ctx->lpr && g.iters == iters && g.has_one == (one != nullptr) &&
        (!one || std::memcmp(&g.one, one, sizeof(SysDesc)) == 0)) {
      *out = g.exec;
      return MFS_OK;
    }
  }
  hipGraph_t graph = nullptr;
  MFS_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  for (int j = 0; j < iters; ++j) {
    launch_cg_spmv(ctx->stream, sd, ts.dv, ts.nv, fp32, ctx->lpr, one);
    launch_cg_update(ctx->stream, sd, ts.dv, ts.nv, fp32, one);
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
  CgGraph g{sd, ts.dv, ts.nv, fp32, ctx->lpr, iters, one != nullptr, SysDesc{}, exec};
  if (one) g.one = *one;
  ctx->graphs.push_back(g);
  *out = exec;
  return MFS_OK;
}

// Enqueue `run` PCG iterations: replayed graphs when enabled and the
// profiler is off, direct launches (each family timed by the profiler)
// otherwise.
int run_cg(mfs_context* ctx, const SysDesc* sd, const TileSet& ts, int fp32, int run, const SysDesc* one,
           double spmv_bytes) {
  const int G = ctx->graph_iters;
  int done = 0;
  if (ctx->use_graphs && ctx->prof_stride == 0 && G > 0) {
    hipGraphExec_t exec;
    MFS_TRY(cg_graph(ctx, sd, ts, fp32, G, one, &exec));
    for (; done + G <= run; done += G) {
      MFS_HIP(hipGraphLaunch(exec, ctx->stream));
      ctx->prof_launches[MFS_K_SPMV] += G;
      ctx->prof_launches[MFS_K_CG_UPDATE] += G;
    }
  }
  for (; done < run; ++done) {
    {
      ProfScope ps(ctx, MFS_K_SPMV, spmv_bytes);
      launch_cg_spmv(ctx->stream, sd, ts.dv, ts.nv, fp32, ctx->lpr, one);
    }
    ProfScope ps(ctx, MFS_K_CG_UPDATE);
    launch_cg_update(ctx->stream, sd, ts.dv, ts.nv, fp32, one);
  }
  return MFS_OK;
}

int read_red(mfs_context* ctx, int count) {
  MFS_HIP(hipMemcpyAsync(ctx->h_red.p, ctx->red.p, count * P_COUNT * sizeof(double), hipMemcpyDeviceToHost,
                         ctx->stream));
  MFS_HIP(hipStreamSynchronize(ctx->stream));
  prof_resolve(ctx);
  return MFS_OK;
}

}  // namespace

int solve_systems(mfs_context* ctx, int count, mfs_character* const* chars, const double* const* R,
                  const double* const* t, const mfs_solve_opts* opts, double* const* x_out, mfs_solve_stats* stats) {
  if (!ctx || count < 1 || !chars || !R || !t || !x_out)
    return set_error(MFS_E_INVALID, "null argument or empty batch");
  mfs_solve_opts o;
  mfs_default_opts(&o);
  if (opts) o = *opts;
  if (o.precision != MFS_FP64 && o.precision != MFS_FP32_REFINED)
    return set_error(MFS_E_INVALID, "unknown precision %d", o.precision);
  if (o.max_newton < 1 || o.cg_max < 1 || !(o.cg_tol >= 0.0) || !(o.step_tol >= 0.0))
    return set_error(MFS_E_INVALID, "invalid solve options");
  if (o.output_memory != MFS_MEM_HOST && o.output_memory != MFS_MEM_DEVICE)
    return set_error(MFS_E_INVALID, "invalid output memory space");
  const int fp32 = o.precision == MFS_FP32_REFINED;
  MFS_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;

  std::vector<HostSys> sys(count);
  for (int i = 0; i < count; ++i) {
    if (!chars[i] || chars[i]->ctx != ctx) return set_error(MFS_E_INVALID, "character %d is null or of another context", i);
    for (int j = 0; j < i; ++j)
      if (chars[j] == chars[i]) return set_error(MFS_E_INVALID, "character %d appears twice in the batch", i);
    if (!x_out[i]) return set_error(MFS_E_INVALID, "x_out[%d] is NULL", i);
    MFS_TRY(check_pose(chars[i], R[i], t[i]));
    sys[i].ch = chars[i];
  }

  // batch scratch: descriptors with batch-owned flags / reductions
  MFS_TRY(ctx->desc.reserve(count * sizeof(SysDesc)));
  MFS_TRY(ctx->ctrl.reserve(count * sizeof(Ctrl)));
  MFS_TRY(ctx->flags.reserve(count * F_COUNT * sizeof(int32_t)));
  MFS_TRY(ctx->red.reserve(count * P_COUNT * sizeof(double)));
  MFS_TRY(ctx->h_ctrl.reserve(count * sizeof(Ctrl)));
  MFS_TRY(ctx->h_flags.reserve(count * F_COUNT * sizeof(int32_t)));
  MFS_TRY(ctx->h_red.reserve(count * P_COUNT * sizeof(double)));
  MFS_TRY(ctx->cgres.reserve(count * 2 * sizeof(double)));
  MFS_TRY(ctx->h_cgres.reserve(count * 2 * sizeof(double)));
  MFS_HIP(hipStreamSynchronize(st));  // staging buffers may be reused below
  std::vector<SysDesc> hd(count);
  {
    for (int i = 0; i < count; ++i) {
      hd[i] = chars[i]->desc;
      hd[i].flags = ctx->flags.as<int32_t>() + F_COUNT * i;
      hd[i].red = ctx->red.as<double>() + P_COUNT * i;
      hd[i].cgres = ctx->cgres.as<double>() + 2 * i;
      hd[i].ctrl = ctx->ctrl.as<Ctrl>() + i;
    }
    MFS_HIP(hipMemcpyAsync(ctx->desc.p, hd.data(), count * sizeof(SysDesc), hipMemcpyHostToDevice, st));
    MFS_HIP(hipStreamSynchronize(st));
  }
  const SysDesc* dsd = ctx->desc.as<SysDesc>();
  const Ctrl* dctrl = ctx->ctrl.as<Ctrl>();
  Ctrl* hc = ctx->h_ctrl.as<Ctrl>();
  std::memset(hc, 0, count * sizeof(Ctrl));
  const int32_t* hf = ctx->h_flags.as<int32_t>();
  const double* hr = ctx->h_red.as<double>();

  // pose upload and warm start x0
  for (int i = 0; i < count; ++i) {
    mfs_character* ch = chars[i];
    MFS_TRY(upload_pose(ch, R[i], t[i]));
    if (o.warm_start != MFS_WARM_PREVIOUS || !ch->has_solution)
      MFS_HIP(hipMemcpyAsync(ch->x.p, ch->X.p, 3 * sizeof(double) * ch->n, hipMemcpyDeviceToDevice, st));
    ch->has_solution = false;
  }

  std::vector<int> ids(count);
  for (int i = 0; i < count; ++i) ids[i] = i;
  TileSet ts;
  MFS_TRY(build_tiles(ctx, sys, ids, &ts));
  std::vector<int> tile_ids = ids;

  // mixed warm start s0 = stretch factor of F(x0)
  {
    ProfScope ps(ctx, MFS_K_WARM_START);
    launch_warm_start(st, dsd, ts.dt, ts.nt, fp32);
  }
  {
    ProfScope ps(ctx, MFS_K_OTHER);
    launch_finalize(st, dsd, ctx->sys_ids.as<int32_t>(), (int)ids.size());
  }
  MFS_HIP(hipGetLastError());
  MFS_TRY(read_red(ctx, count));
  for (int i = 0; i < count; ++i) sys[i].routed = (int)hr[P_COUNT * i + P_ROUTED];

  for (int i = 0; i < count; ++i) {
    hc[i].cg_tol2 = o.cg_tol * o.cg_tol;
    hc[i].cg_adaptive = o.cg_adaptive ? 1 : 0;
    hc[i].cg_g2prev = 0.0;
    hc[i].cg_eta_min = 0.0;
  }
  for (int it = 0; it < o.max_newton; ++it) {
    std::vector<int> act;
    for (int i = 0; i < count; ++i)
      if (!sys[i].done) act.push_back(i);
    if (act.empty()) break;
    if (act != tile_ids) {
      MFS_TRY(build_tiles(ctx, sys, act, &ts));
      tile_ids = act;
    }
    for (int i : act) {
      hc[i].phase = sys[i].phase;
      hc[i].update_s = 0;
      hc[i].alpha = 0.0;
    }
    MFS_TRY(upload_ctrl(ctx, count));
    {
      ProfScope ps(ctx, MFS_K_ELEMENT);
      launch_element(st, dsd, dctrl, ts.dt, ts.nt, fp32);
    }
    {
      ProfScope ps(ctx, MFS_K_ASSEMBLE);
      launch_assemble(st, dsd, ts.ds, ts.ns, fp32);
    }
    {
      ProfScope ps(ctx, MFS_K_OTHER);
      launch_cg_init(st, dsd, ts.dv, ts.nv, fp32);
    }
    MFS_HIP(hipGetLastError());

    // PCG in runs of iterations; after each run the host reads the
    // convergence flags and residuals and sizes the next run from the
    // observed residual decay of the slowest character.
    int cit = 0;
    int chunk = ctx->cg_first_run;
    for (int i : act) {
      sys[i].rho_prev = -1.0;
      sys[i].it_prev = 0;
    }
    const SysDesc* one = act.size() == 1 ? &hd[act[0]] : nullptr;
    // algorithmic bytes of one SpMV launch over the characters still in PCG
    // (blocks + column indices + row pointers + 2 gathered inputs and 2
    // outputs per row), for the profiler's roofline figures
    const double word = fp32 ? 4.0 : 8.0;
    auto spmv_bytes = [&]() {
      double by = 0.0;
      for (int i : act)
        if (!hf[F_COUNT * i + F_CG_DONE] || cit == 0)
          by += chars[i]->nnzb * (9.0 * word + 4.0) + (chars[i]->n + 1) * 4.0 + chars[i]->n * 12.0 * word;
      return by;
    };
    while (cit < o.cg_max) {
      const int run = std::min(chunk, o.cg_max - cit);
      MFS_TRY(run_cg(ctx, dsd, ts, fp32, run, one, spmv_bytes()));
      cit += run;
      MFS_HIP(hipGetLastError());
      MFS_TRY(read_flags(ctx, count));
      const double* hres = ctx->h_cgres.as<double>();
      bool all = true;
      int need = 0;
      for (int i : act) {
        if (hf[F_COUNT * i + F_CG_DONE]) continue;
        all = false;
        const double rr = hres[2 * i], bb = hres[2 * i + 1];
        const double rho = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
        const double tol_i = std::sqrt(pcg_tol2(hc[i], bb));
        int est = ctx->cg_first_run;
        HostSys& S = sys[i];
        if (S.rho_prev > 0.0 && rho > 0.0 && rho < S.rho_prev && cit > S.it_prev) {
          const double rate = std::pow(rho / S.rho_prev, 1.0 / (cit - S.it_prev));
          const double left = std::log(tol_i / rho) / std::log(rate);
          est = (int)std::ceil(1.1 * left) + 2;
        }
        S.rho_prev = rho;
        S.it_prev = cit;
        need = std::max(need, est);
      }
      if (all) break;
      chunk = std::min(std::max(need, ctx->cg_min_run), ctx->cg_max_run);
    }
    for (int i : act) {
      if (hf[F_COUNT * i + F_CG_DONE]) {
        sys[i].cg += hf[F_COUNT * i + F_CG_ITERS];
      } else {
        sys[i].cg += o.cg_max;
        sys[i].cg_fail++;
      }
    }
    {
      ProfScope ps(ctx, MFS_K_OTHER);
      launch_cg_finish(st, dsd, ts.dv, ts.nv, fp32);
    }

    // line search, first pass: Newton systems evaluate E at {0, 1, 1/2, 1/4, 1/8}
    for (int i : act) {
      sys[i].searching = true;
      sys[i].alpha = 0.0;
      sys[i].pass = 0;
      hc[i].phase = sys[i].phase;
      hc[i].trials[0] = 0.0;
      for (int j = 1; j < kNumTrials; ++j) hc[i].trials[j] = std::ldexp(1.0, -(j - 1));
    }
    std::vector<int> srch = act;
    bool first_pass = true;
    while (!srch.empty()) {
      if (srch != tile_ids) {
        MFS_TRY(build_tiles(ctx, sys, srch, &ts));
        tile_ids = srch;
      }
      MFS_TRY(upload_ctrl(ctx, count));
      {
        ProfScope ps(ctx, MFS_K_LINESEARCH);
        launch_linesearch(st, dsd, dctrl, ts.dt, ts.nt, ts.dv, ts.nv);
      }
      {
        ProfScope ps(ctx, MFS_K_OTHER);
        launch_finalize(st, dsd, ctx->sys_ids.as<int32_t>(), (int)srch.size());
      }
      MFS_HIP(hipGetLastError());
      MFS_TRY(read_red(ctx, count));
      std::vector<int> next;
      for (int i : srch) {
        HostSys& S = sys[i];
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
          S.step = rd[P_DXMAX];  // scaled by alpha below
        }
        if (S.phase == 0) {
          const int h = (int)rd[P_HMAX];
          S.searching = false;
          if (h > 40) {
            S.alpha = 0.0;
          } else {
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
          if (last <= std::ldexp(1.0, -40) || !std::isfinite(E0)) {
            S.alpha = 0.0;
            S.searching = false;
          } else {
            for (int j = 0; j < kNumTrials; ++j) hc[i].trials[j] = last * std::ldexp(1.0, -(j + 1));
            next.push_back(i);
          }
        } else {
          S.searching = false;
        }
      }
      srch.swap(next);
      first_pass = false;
    }

    // updates
    for (int i : act) {
      hc[i].alpha = sys[i].alpha;
      hc[i].update_s = (sys[i].phase == 0 && sys[i].alpha > 0.0 && sys[i].alpha < 1.0) ? 1 : 0;
      hc[i].phase = sys[i].phase;
    }
    if (act != tile_ids) {
      MFS_TRY(build_tiles(ctx, sys, act, &ts));
      tile_ids = act;
    }
    MFS_TRY(upload_ctrl(ctx, count));
    {
      ProfScope ps(ctx, MFS_K_UPDATE);
      launch_update(st, dsd, dctrl, ts.dt, ts.nt, ts.dv, ts.nv);
    }
    MFS_HIP(hipGetLastError());

    for (int i : act) {
      HostSys& S = sys[i];
      const bool was_newton = S.phase == 1;
      S.iters = it + 1;
      S.step = S.alpha * S.step;
      if (!was_newton) {
        S.mixed++;
        S.E_known = false;
      }
      if (S.alpha == 0.0) {
        S.done = true;
        S.status = MFS_W_NOT_CONVERGED;
        continue;
      }
      if (!was_newton && S.alpha == 1.0) S.phase = 1;
      if (o.fixed_newton) {
        if (it + 1 == o.max_newton) S.done = true;
      } else if (was_newton && S.step <= o.step_tol * S.ch->bbox_diag) {
        S.done = true;
      } else if (it + 1 == o.max_newton) {
        S.done = true;
        S.status = MFS_W_NOT_CONVERGED;
      }
    }
  }
  for (int i = 0; i < count; ++i)
    if (!sys[i].done) sys[i].status = MFS_W_NOT_CONVERGED;

  // energies at the returned positions where the last step did not give them
  if (stats) {
    std::vector<int> need;
    for (int i = 0; i < count; ++i)
      if (!sys[i].E_known) need.push_back(i);
    if (!need.empty()) {
      MFS_TRY(build_tiles(ctx, sys, need, &ts));
      tile_ids = need;
      for (int i : need) {
        hc[i].phase = 1;
        for (int j = 0; j < kNumTrials; ++j) hc[i].trials[j] = 0.0;
      }
      MFS_TRY(upload_ctrl(ctx, count));
      launch_linesearch(st, dsd, dctrl, ts.dt, ts.nt, ts.dv, ts.nv);
      launch_finalize(st, dsd, ctx->sys_ids.as<int32_t>(), (int)need.size());
      MFS_HIP(hipGetLastError());
      MFS_TRY(read_red(ctx, count));
      for (int i : need) {
        const double* rd = hr + P_COUNT * i;
        sys[i].E = rd[P_INF0] > 0.0 ? INFINITY : rd[P_E0] + rd[P_PIN0];
      }
    }
  }

  // outputs in the caller's vertex order
  int worst = MFS_OK;
  for (int i = 0; i < count; ++i) {
    mfs_character* ch = chars[i];
    if (o.output_memory == MFS_MEM_DEVICE) {
      launch_scatter_rows(st, ch->x.as<double>(), ch->perm_d.as<int32_t>(), ch->n, 3, 1.0, x_out[i]);
    } else {
      launch_scatter_rows(st, ch->x.as<double>(), ch->perm_d.as<int32_t>(), ch->n, 3, 1.0, ch->r.as<double>());
      MFS_HIP(hipMemcpyAsync(x_out[i], ch->r.p, 3 * sizeof(double) * ch->n, hipMemcpyDeviceToHost, st));
    }
    ch->has_solution = true;
    if (sys[i].status > worst) worst = sys[i].status;
  }
  MFS_HIP(hipGetLastError());
  MFS_HIP(hipStreamSynchronize(st));
  prof_resolve(ctx);
  if (stats) {
    for (int i = 0; i < count; ++i) {
      mfs_solve_stats& s = stats[i];
      const HostSys& S = sys[i];
      s.status = S.status;
      s.iterations = S.iters;
      s.mixed_iterations = S.mixed;
      s.cg_iterations = S.cg;
      s.halvings = S.halvings;
      s.clamped = S.clamped;
      s.fp64_routed = S.routed;
      s.cg_not_converged = S.cg_fail;
      s.energy = S.E;
      s.grad_norm = S.grad;
      s.last_step = S.step;
      s.cg_rel_residual = S.relres;
    }
  }
  if (worst == MFS_W_NOT_CONVERGED) set_error(MFS_W_NOT_CONVERGED, "frame solve did not converge");
  return worst;
}

}  // namespace mfs

using namespace mfs;

extern "C" int mfs_solve_frame(mfs_character* ch, const double* handle_R, const double* handle_t,
                               const mfs_solve_opts* opts, double* x_out, mfs_solve_stats* stats) {
  clear_error();
  if (!ch) return set_error(MFS_E_INVALID, "null character");
  return solve_systems(ch->ctx, 1, &ch, &handle_R, &handle_t, opts, &x_out, stats);
}

extern "C" int mfs_solve_batch(mfs_context* ctx, int32_t count, mfs_character* const* chars,
                               const double* const* handle_R, const double* const* handle_t,
                               const mfs_solve_opts* opts, double* const* x_out, mfs_solve_stats* stats) {
  clear_error();
  return solve_systems(ctx, count, chars, handle_R, handle_t, opts, x_out, stats);
}

extern "C" int mfs_evaluate(mfs_character* ch, const double* handle_R, const double* handle_t, const double* x,
                            const double* v, int32_t memory_space, double* energy_out, double* grad_out,
                            double* stretch_out, double* Kv_out) {
  clear_error();
  if (!ch || !x) return set_error(MFS_E_INVALID, "null character or positions");
  if (memory_space != MFS_MEM_HOST && memory_space != MFS_MEM_DEVICE)
    return set_error(MFS_E_INVALID, "invalid memory space");
  if ((v == nullptr) != (Kv_out == nullptr)) return set_error(MFS_E_INVALID, "v and Kv_out must both be given");
  mfs_context* ctx = ch->ctx;
  MFS_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  MFS_TRY(check_pose(ch, handle_R, handle_t));
  const bool host = memory_space == MFS_MEM_HOST;
  const size_t n3 = 3 * sizeof(double) * (size_t)ch->n;
  const size_t m6 = 6 * sizeof(double) * (size_t)ch->m;
  MFS_TRY(ctx->tmp.reserve(std::max(n3, m6)));
  MFS_TRY(ctx->desc.reserve(sizeof(SysDesc)));
  MFS_TRY(ctx->ctrl.reserve(sizeof(Ctrl)));
  MFS_TRY(ctx->flags.reserve(F_COUNT * sizeof(int32_t)));
  MFS_TRY(ctx->red.reserve(P_COUNT * sizeof(double)));
  MFS_TRY(ctx->cgres.reserve(2 * sizeof(double)));
  MFS_TRY(ctx->h_ctrl.reserve(sizeof(Ctrl)));
  MFS_TRY(ctx->h_red.reserve(P_COUNT * sizeof(double)));
  MFS_HIP(hipStreamSynchronize(st));
  SysDesc hd = ch->desc;
  hd.flags = ctx->flags.as<int32_t>();
  hd.red = ctx->red.as<double>();
  hd.cgres = ctx->cgres.as<double>();
  hd.ctrl = ctx->ctrl.as<Ctrl>();
  MFS_HIP(hipMemcpyAsync(ctx->desc.p, &hd, sizeof(SysDesc), hipMemcpyHostToDevice, st));
  MFS_TRY(upload_pose(ch, handle_R, handle_t));
  double* tmp = ctx->tmp.as<double>();
  const double* xs = x;
  if (host) {
    MFS_HIP(hipMemcpyAsync(tmp, x, n3, hipMemcpyHostToDevice, st));
    xs = tmp;
  }
  launch_gather_rows(st, xs, ch->perm_d.as<int32_t>(), ch->n, 3, ch->x.as<double>());
  ch->has_solution = false;
  std::vector<HostSys> sys(1);
  sys[0].ch = ch;
  TileSet ts;
  MFS_TRY(build_tiles(ctx, sys, std::vector<int>{0}, &ts));
  Ctrl* hc = ctx->h_ctrl.as<Ctrl>();
  std::memset(hc, 0, sizeof(Ctrl));
  hc->phase = 1;
  MFS_TRY(upload_ctrl(ctx, 1));
  const SysDesc* dsd = ctx->desc.as<SysDesc>();
  const Ctrl* dctrl = ctx->ctrl.as<Ctrl>();
  launch_element(st, dsd, dctrl, ts.dt, ts.nt, 0);
  launch_assemble(st, dsd, ts.ds, ts.ns, 0);
  MFS_HIP(hipMemsetAsync(ch->dx.p, 0, n3, st));
  launch_linesearch(st, dsd, dctrl, ts.dt, ts.nt, ts.dv, ts.nv);
  launch_finalize(st, dsd, ctx->sys_ids.as<int32_t>(), 1);
  MFS_HIP(hipGetLastError());
  if (grad_out) {
    double* dst = host ? tmp : grad_out;
    launch_scatter_rows(st, ch->b.as<double>(), ch->perm_d.as<int32_t>(), ch->n, 3, -1.0, dst);
    if (host) MFS_HIP(hipMemcpyAsync(grad_out, tmp, n3, hipMemcpyDeviceToHost, st));
  }
  if (stretch_out) {
    double* dst = host ? tmp : stretch_out;
    launch_scatter_planes6(st, ch->s.as<double>(), ch->m, ch->tperm_d.as<int32_t>(), dst);
    if (host) MFS_HIP(hipMemcpyAsync(stretch_out, tmp, m6, hipMemcpyDeviceToHost, st));
  }
  if (v) {
    const double* vs = v;
    if (host) {
      MFS_HIP(hipMemcpyAsync(tmp, v, n3, hipMemcpyHostToDevice, st));
      vs = tmp;
    }
    launch_gather_rows(st, vs, ch->perm_d.as<int32_t>(), ch->n, 3, ch->p0.as<double>());
    launch_spmv_plain(st, ch->rowptr.as<int32_t>(), ch->colidx.as<int32_t>(), ch->vals.as<double>(), ch->nnzb, ch->n,
                      ch->p0.as<double>(), ch->q.as<double>());
    double* dst = host ? tmp : Kv_out;
    launch_scatter_rows(st, ch->q.as<double>(), ch->perm_d.as<int32_t>(), ch->n, 3, 1.0, dst);
    if (host) MFS_HIP(hipMemcpyAsync(Kv_out, tmp, n3, hipMemcpyDeviceToHost, st));
  }
  MFS_HIP(hipGetLastError());
  MFS_TRY(read_red(ctx, 1));
  if (energy_out) {
    const double* rd = ctx->h_red.as<double>();
    *energy_out = rd[P_INF0] > 0.0 ? INFINITY : rd[P_E0] + rd[P_PIN0];
  }
  return MFS_OK;
}
