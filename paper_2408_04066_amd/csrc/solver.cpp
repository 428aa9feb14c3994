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

#include "engine.h"
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

int upload_pose(mfs_context* ctx, mfs_character* ch, const double* R, const double* t) {
  hipStream_t st = ctx->stream;
  MFS_TRY(ctx->up.upload(st, ch->Rh.p, R, 9 * sizeof(double) * ch->nh));
  MFS_TRY(ctx->up.upload(st, ch->th.p, t, 3 * sizeof(double) * ch->nh));
  if (ch->blend_k > 0)  // smoothed tet rotations follow every pose (and load step)
    launch_blend_rot(st, ch->Rh.as<double>(), ch->m, ch->blend_k, ch->blend_h.as<int32_t>(), ch->blend_w.as<double>(),
                     ch->Rt.as<double>());
  return MFS_OK;
}

int solve_systems(mfs_context* ctx, int count, mfs_character* const* chars, const double* const* R,
                  const double* const* t, const mfs_solve_opts* opts, double* const* x_out, mfs_solve_stats* stats) {
  if (!ctx || count < 1 || !chars || !R || !t || !x_out)
    return set_error(MFS_E_INVALID, "null argument or empty batch");
  for (int i = 0; i < count; ++i)
    if (!x_out[i]) return set_error(MFS_E_INVALID, "x_out[%d] is NULL", i);
  MFS_HIP(hipSetDevice(ctx->device));
  Engine eng(ctx);
  MFS_TRY(eng.configure(opts));
  MFS_TRY(eng.reserve(count));
  for (int i = 0; i < count; ++i) {
    if (!chars[i] || chars[i]->ctx != ctx) return set_error(MFS_E_INVALID, "character %d is null or of another context", i);
    MFS_TRY(ensure_workspace(chars[i]));
    MFS_TRY(eng.attach(i, chars[i], R[i], t[i]));
  }
  for (int idle = 0; eng.any_busy();) {
    const uint64_t before = eng.progress_key();
    MFS_TRY(eng.run_once());
    idle = eng.progress_key() == before ? idle + 1 : 0;
    if (idle > 8) return set_error(MFS_E_HIP, "frame solve: scheduling calls make no progress");
  }
  if (stats) MFS_TRY(eng.finish_energies());
  mfs_solve_opts o;
  mfs_default_opts(&o);
  if (opts) o = *opts;
  int worst = MFS_OK;
  for (int i = 0; i < count; ++i) {
    MFS_TRY(eng.output(i, x_out[i], o.output_memory));
    if (stats) eng.stats(i, &stats[i]);
    worst = std::max(worst, eng.state(i).status);
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
  MFS_TRY(ensure_workspace(ch));
  const bool host = memory_space == MFS_MEM_HOST;
  const size_t n3 = 3 * sizeof(double) * (size_t)ch->n;
  const size_t m6 = 6 * sizeof(double) * (size_t)ch->m;
  MFS_TRY(ctx->tmp.reserve(std::max(n3, m6)));
  MFS_TRY(ctx->desc.reserve(sizeof(SysDesc)));
  MFS_TRY(ctx->ctrl.reserve(sizeof(Ctrl)));
  MFS_TRY(ctx->red.reserve(P_COUNT * sizeof(double)));
  MFS_TRY(ctx->cg.reserve(sizeof(CgState)));
  if (ctx->h_ctrl.empty()) ctx->h_ctrl.resize(1);
  MFS_TRY(ctx->h_red.reserve(P_COUNT * sizeof(double)));
  MFS_HIP(hipStreamSynchronize(st));
  SysDesc hd = ch->desc;
  hd.red = ctx->red.as<double>();
  hd.cg = ctx->cg.as<CgState>();
  hd.ctrl = ctx->ctrl.as<Ctrl>();
  MFS_TRY(ctx->up.upload(st, ctx->desc.p, &hd, sizeof(SysDesc)));
  MFS_TRY(upload_pose(ctx, ch, handle_R, handle_t));
  double* tmp = ctx->tmp.as<double>();
  const double* xs = x;
  if (host) {
    MFS_HIP(hipMemcpyAsync(tmp, x, n3, hipMemcpyHostToDevice, st));
    xs = tmp;
  }
  launch_gather_rows(st, xs, ch->perm_d.as<int32_t>(), ch->n, 3, ch->x.as<double>());
  ch->has_solution = false;
  TileSet ts;
  MFS_TRY(build_tile_list(ctx, std::vector<mfs_character*>{ch}, std::vector<int>{0}, &ts));
  Ctrl* hc = ctx->h_ctrl.data();
  std::memset(hc, 0, sizeof(Ctrl));
  hc->phase = 1;
  MFS_TRY(upload_ctrl(ctx, 1));
  const SysDesc* dsd = ctx->desc.as<SysDesc>();
  const Ctrl* dctrl = ctx->ctrl.as<Ctrl>();
  launch_element(st, dsd, dctrl, ts.dt, ts.nt, 0);
  launch_assemble(st, dsd, ts.ds, ts.ns, 0);
  MFS_HIP(hipMemsetAsync(ch->desc.dx, 0, n3, st));
  launch_linesearch(st, dsd, dctrl, ts.dt, ts.nt, ts.dv, ts.nv);
  launch_finalize(st, dsd, ctx->sys_ids.as<int32_t>(), 1);
  MFS_HIP(hipGetLastError());
  if (grad_out) {
    double* dst = host ? tmp : grad_out;
    launch_scatter_rows(st, ch->desc.b, ch->perm_d.as<int32_t>(), ch->n, 3, -1.0, dst);
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
    launch_gather_rows(st, vs, ch->perm_d.as<int32_t>(), ch->n, 3, static_cast<double*>(ch->desc.p0));
    launch_spmv_plain(st, ch->rowptr.as<int32_t>(), static_cast<const double*>(ch->desc.vals), ch->n,
                      static_cast<const double*>(ch->desc.p0), static_cast<double*>(ch->desc.q));
    double* dst = host ? tmp : Kv_out;
    launch_scatter_rows(st, static_cast<const double*>(ch->desc.q), ch->perm_d.as<int32_t>(), ch->n, 3, 1.0, dst);
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

extern "C" int mfs_stress(mfs_character* ch, const double* handle_R, const double* handle_t, const double* x,
                          int32_t memory_space, double* stress_out, double* multiplier_out) {
  clear_error();
  if (!ch || !x) return set_error(MFS_E_INVALID, "null character or positions");
  if (memory_space != MFS_MEM_HOST && memory_space != MFS_MEM_DEVICE)
    return set_error(MFS_E_INVALID, "invalid memory space");
  if (!stress_out && !multiplier_out) return MFS_OK;
  mfs_context* ctx = ch->ctx;
  MFS_HIP(hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  MFS_TRY(check_pose(ch, handle_R, handle_t));
  const bool host = memory_space == MFS_MEM_HOST;
  const size_t n3 = 3 * sizeof(double) * (size_t)ch->n;
  const size_t m6 = 6 * sizeof(double) * (size_t)ch->m, m9 = 9 * sizeof(double) * (size_t)ch->m;
  MFS_TRY(ctx->tmp.reserve(std::max(n3, m6 + m9)));
  MFS_TRY(ctx->desc.reserve(sizeof(SysDesc)));
  MFS_HIP(hipStreamSynchronize(st));
  MFS_TRY(ctx->up.upload(st, ctx->desc.p, &ch->desc, sizeof(SysDesc)));
  MFS_TRY(upload_pose(ctx, ch, handle_R, handle_t));
  double* tmp = ctx->tmp.as<double>();
  const double* xs = x;
  if (host) {
    MFS_HIP(hipMemcpyAsync(tmp, x, n3, hipMemcpyHostToDevice, st));
    xs = tmp;
  }
  launch_gather_rows(st, xs, ch->perm_d.as<int32_t>(), ch->n, 3, ch->x.as<double>());
  ch->has_solution = false;
  double* P6 = stress_out ? (host ? tmp : stress_out) : nullptr;
  double* L9 = multiplier_out ? (host ? tmp + 6 * (size_t)ch->m : multiplier_out) : nullptr;
  launch_stress(st, ctx->desc.as<SysDesc>(), ch->m, ch->tperm_d.as<int32_t>(), P6, L9);
  MFS_HIP(hipGetLastError());
  if (host) {
    if (stress_out) MFS_HIP(hipMemcpyAsync(stress_out, P6, m6, hipMemcpyDeviceToHost, st));
    if (multiplier_out) MFS_HIP(hipMemcpyAsync(multiplier_out, L9, m9, hipMemcpyDeviceToHost, st));
  }
  MFS_HIP(hipStreamSynchronize(st));
  return MFS_OK;
}
