// Autotuner of the PCG launch schedule.
//
// The schedule knobs are the PCG form (two kernels per iteration, the
// pipelined one-kernel form, or its persistent launch for FP32 solves), the
// SpMV lanes per block row
// (2, 4 or 8 lanes of a 64-row tile), the number of PCG iterations per
// captured graph, the lengths of the first and shortest runs between host
// convergence checks, and for large systems the reduction mode (all-read
// folds or fenced arrival tickets).  Candidates
// are timed on the caller's own systems: each runs the same fixed number of
// Newton iterations from the rest shape (the same launches for every
// candidate, up to summation order), timed on the host clock around the
// synchronous solve.  Summation order alone moves the PCG iteration counts of
// a candidate's runs by a few percent either way, so a candidate's time is
// scaled by the reference schedule's total PCG iteration count over its own
// before it is compared: the ranking is by time per unit of the same PCG work,
// which carries over to other frames.  The fastest is applied to the context and cached per
// (GPU architecture, size class), where the size class is the bit length of
// the total block-row count of the batch; a cache file keeps the choices
// across processes.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace mfs {
namespace {

struct Entry {
  std::string arch;
  int size_class;
  mfs_tuning t;
  double ms;
};

int size_class_of(int count, mfs_character* const* chars) {
  long long rows = 0;
  for (int i = 0; i < count; ++i) rows += chars[i]->n;
  int c = 0;
  while (rows > 0) {
    ++c;
    rows >>= 1;
  }
  return c;
}

std::vector<Entry> read_cache(const char* path) {
  std::vector<Entry> out;
  if (!path) return out;
  FILE* f = std::fopen(path, "r");
  if (!f) return out;
  char line[512], arch[128];
  while (std::fgets(line, sizeof line, f)) {
    Entry e{};
    e.t.batch_async = 1;
    double v[12];
    const int k = std::sscanf(line, "%127s %d %d %d %d %d %d %d %d %d %d %lf %lf", arch, &e.size_class,
                              &e.t.pcg_lanes_per_row, &e.t.use_graphs, &e.t.graph_iterations, &e.t.first_check,
                              &e.t.min_run, &e.t.max_run, &e.t.pcg_pipelined, &e.t.allread_max_tiles,
                              &e.t.pcg_persistent, &v[0], &v[1]);
    if (k == 12) {  // written before the batch_async field
      e.ms = v[0];
    } else if (k == 13) {  // ... batch_async ms
      e.t.batch_async = (int)v[0];
      e.ms = v[1];
    } else {
      continue;
    }
    e.arch = arch;
    out.push_back(e);
  }
  std::fclose(f);
  return out;
}

int write_cache(const char* path, const std::vector<Entry>& entries) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return set_error(MFS_E_INVALID, "cannot write tuning cache %s", tmp.c_str());
  for (const Entry& e : entries)
    std::fprintf(f, "%s %d %d %d %d %d %d %d %d %d %d %d %.6f\n", e.arch.c_str(), e.size_class,
                 e.t.pcg_lanes_per_row, e.t.use_graphs, e.t.graph_iterations, e.t.first_check, e.t.min_run,
                 e.t.max_run, e.t.pcg_pipelined, e.t.allread_max_tiles, e.t.pcg_persistent, e.t.batch_async, e.ms);
  std::fclose(f);
  if (std::rename(tmp.c_str(), path) != 0) return set_error(MFS_E_INVALID, "cannot replace tuning cache %s", path);
  return MFS_OK;
}

}  // namespace
}  // namespace mfs

using namespace mfs;

extern "C" int mfs_autotune(mfs_context* ctx, int32_t count, mfs_character* const* chars,
                            const double* const* handle_R, const double* const* handle_t,
                            const mfs_solve_opts* opts, int32_t newton_iterations, const char* cache_path,
                            int32_t flags, mfs_tuning* best, double* best_ms) {
  clear_error();
  if (!ctx || count < 1 || !chars || !handle_R || !handle_t)
    return set_error(MFS_E_INVALID, "null argument or empty batch");
  if (newton_iterations < 0) return set_error(MFS_E_INVALID, "newton_iterations must be >= 0");
  for (int i = 0; i < count; ++i)
    if (!chars[i] || chars[i]->ctx != ctx) return set_error(MFS_E_INVALID, "character %d is null or of another context", i);
  MFS_HIP(hipSetDevice(ctx->device));
  hipDeviceProp_t prop;
  MFS_HIP(hipGetDeviceProperties(&prop, ctx->device));
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  const int cls = size_class_of(count, chars);

  std::vector<Entry> cache = read_cache(cache_path);
  if (!(flags & MFS_AUTOTUNE_FORCE)) {
    for (const mfs_context::TuneEntry& e : ctx->tune_cache)
      if (e.size_class == cls) {
        MFS_TRY(mfs_context_set_tuning(ctx, &e.tuning));
        if (best) *best = e.tuning;
        if (best_ms) *best_ms = e.ms;
        return MFS_OK;
      }
    for (const Entry& e : cache)
      if (e.arch == arch && e.size_class == cls) {
        MFS_TRY(mfs_context_set_tuning(ctx, &e.t));
        ctx->tune_cache.push_back(mfs_context::TuneEntry{cls, e.t, e.ms});
        if (best) *best = e.t;
        if (best_ms) *best_ms = e.ms;
        return MFS_OK;
      }
  }

  mfs_solve_opts o;
  mfs_default_opts(&o);
  if (opts) o = *opts;
  o.warm_start = MFS_WARM_REST;
  // a fixed number of Newton iterations, or (0) whole frames with the
  // caller's stop rule and Newton cap: the asynchronous batch form's launch
  // sets change over a frame, so its first iterations alone misjudge it
  if (newton_iterations > 0) {
    o.fixed_newton = 1;
    o.max_newton = newton_iterations;
  }
  o.output_memory = MFS_MEM_DEVICE;
  std::vector<DevBuf> outs(count);
  std::vector<double*> xo(count);
  for (int i = 0; i < count; ++i) {
    MFS_TRY(outs[i].alloc(3 * sizeof(double) * (size_t)chars[i]->n));
    xo[i] = outs[i].as<double>();
  }
  mfs_tuning base;
  MFS_TRY(mfs_context_get_tuning(ctx, &base));

  // A candidate qualifies only if its solves are as good as the default
  // schedule's: no PCG solve stopped unconverged (or by breakdown) where the
  // default had none, and every final gradient within 10x the default's.
  std::vector<mfs_solve_stats> ref(count), got(count);
  auto time_one = [&](const mfs_tuning& t, double* ms, std::vector<mfs_solve_stats>& st) -> int {
    MFS_TRY(mfs_context_set_tuning(ctx, &t));
    // first run captures this schedule's graphs; the second is timed
    for (int rep = 0; rep < 2; ++rep) {
      const auto t0 = std::chrono::steady_clock::now();
      const int rc = solve_systems(ctx, count, chars, handle_R, handle_t, &o, xo.data(), st.data());
      if (rc < 0) return rc;
      MFS_HIP(hipStreamSynchronize(ctx->stream));
      *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return MFS_OK;
  };
  auto cg_total = [&](const std::vector<mfs_solve_stats>& st) {
    double n = 0.0;
    for (int i = 0; i < count; ++i) n += st[i].cg_iterations;
    return n;
  };
  // time scaled to the reference schedule's PCG work (ref must be filled)
  auto scaled = [&](double ms) {
    const double r = cg_total(ref), g = cg_total(got);
    return (r > 0.0 && g > 0.0) ? ms * r / g : ms;
  };
  auto qualifies = [&]() {
    for (int i = 0; i < count; ++i) {
      if (got[i].cg_not_converged > ref[i].cg_not_converged) return false;
      if (!(got[i].grad_norm <= 10.0 * ref[i].grad_norm + 1e-300)) return false;
    }
    return true;
  };

  mfs_tuning win = base;
  win.use_graphs = 1;
  win.pcg_pipelined = 0;
  win.pcg_persistent = 0;
  double win_ms = INFINITY;
  {
    double ms;
    const int rc = time_one(win, &ms, ref);
    if (rc < 0) {
      (void)mfs_context_set_tuning(ctx, &base);
      return rc;
    }
    win_ms = ms;
  }
  // stage 1: PCG form x lanes per row x graph length (the persistent launch
  // of the pipelined form, FP32 solves only, has no graphs)
  const int forms = o.precision == MFS_FP32_REFINED ? 3 : 2;
  for (int form = 0; form < forms; ++form)
  for (int lpr : {2, 4, 8})
    for (int gi : {4, 8, 16}) {
      if (form == 2 && gi != 8) continue;
      // the asynchronous batch form (batches) launches directly, so the
      // graph length does not matter
      if (win.batch_async && count > 1 && form < 2 && gi != 8) continue;
      // batches: the persistent launch holds one system's tiles only, and the
      // shortest graphs lose to longer ones at batch sizes
      if (count > 1 && (form == 2 || gi == 4)) continue;
      mfs_tuning t = win;
      t.pcg_pipelined = form > 0 ? 1 : 0;
      t.pcg_persistent = form == 2 ? 1 : 0;
      t.pcg_lanes_per_row = lpr;
      t.graph_iterations = gi;
      double ms;
      const int rc = time_one(t, &ms, got);
      if (rc < 0) {
        (void)mfs_context_set_tuning(ctx, &base);
        return rc;
      }
      ms = scaled(ms);
      if (ms < win_ms && qualifies()) {
        win_ms = ms;
        win = t;
      }
    }
  // stage 2: first convergence check and the shortest later run
  const mfs_tuning stage1 = win;
  for (int first : {16, 32, 64})
    for (int minrun : {4, 8, 16}) {
      if (first == stage1.first_check && minrun == stage1.min_run) continue;
      mfs_tuning t = stage1;
      t.first_check = first;
      t.min_run = minrun;
      if (t.max_run < t.min_run) t.max_run = t.min_run;
      double ms;
      const int rc = time_one(t, &ms, got);
      if (rc < 0) {
        (void)mfs_context_set_tuning(ctx, &base);
        return rc;
      }
      ms = scaled(ms);
      if (ms < win_ms && qualifies()) {
        win_ms = ms;
        win = t;
      }
    }
  // stage 3: reduction mode of the large systems (all-read folds instead of
  // fenced arrival tickets), when the batch has any
  int max_tiles = 0;
  for (int i = 0; i < count; ++i) max_tiles = std::max(max_tiles, chars[i]->ntv);
  if (max_tiles > win.allread_max_tiles) {
    const mfs_tuning stage2 = win;
    for (int lim : {1024, 4096, 1 << 20}) {
      if (lim <= stage2.allread_max_tiles) continue;
      mfs_tuning t = stage2;
      t.allread_max_tiles = lim;
      double ms;
      const int rc = time_one(t, &ms, got);
      if (rc < 0) {
        (void)mfs_context_set_tuning(ctx, &base);
        return rc;
      }
      ms = scaled(ms);
      if (ms < win_ms && qualifies()) {
        win_ms = ms;
        win = t;
      }
      if (max_tiles <= lim) break;
    }
  }
  MFS_TRY(mfs_context_set_tuning(ctx, &win));
  bool replaced = false;
  for (auto& e : ctx->tune_cache)
    if (e.size_class == cls) {
      e = mfs_context::TuneEntry{cls, win, win_ms};
      replaced = true;
    }
  if (!replaced) ctx->tune_cache.push_back(mfs_context::TuneEntry{cls, win, win_ms});
  if (cache_path) {
    bool found = false;
    for (Entry& e : cache)
      if (e.arch == arch && e.size_class == cls) {
        e.t = win;
        e.ms = win_ms;
        found = true;
      }
    if (!found) cache.push_back(Entry{arch, cls, win, win_ms});
    MFS_TRY(write_cache(cache_path, cache));
  }
  if (best) *best = win;
  if (best_ms) *best_ms = win_ms;
  return MFS_OK;
}
