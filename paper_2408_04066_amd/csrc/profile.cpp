// Context profiler: for every stride-th launch group of a kernel family, a
// HIP event pair recorded on the group's stream around its launches (before
// its first kernel, after its last), folded into per-family totals at stream
// syncs.
#include <cstring>

#include "internal.h"
#include "launch.h"

namespace mfs {

static hipEvent_t get_event(mfs_context* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

LaunchEvents& launch_events() {
  static thread_local LaunchEvents ev;
  return ev;
}

// A sampled scope hands its event pair to the launches inside it (see
// MFS_LAUNCH); the pair is kept only if a kernel was launched.
ProfScope::ProfScope(mfs_context* ctx, int family, double algorithmic_bytes, int iteration_tag)
    : c(ctx), fam(family), bytes(algorithmic_bytes), tag(iteration_tag) {
  const int64_t k = c->prof_launches[fam]++;
  if (c->prof_stride > 0 && k % c->prof_stride == 0) {
    a = get_event(c);
    b = a ? get_event(c) : nullptr;
    if (!b) {
      if (a) c->ev_pool.push_back(a);
      a = nullptr;
      return;
    }
    LaunchEvents& le = launch_events();
    le.start = a;
    le.stop = b;
    le.started = false;
  }
}

ProfScope::~ProfScope() {
  if (!a) return;
  LaunchEvents& le = launch_events();
  const bool launched = le.started;
  const hipStream_t st = le.where;
  le = LaunchEvents();
  if (!launched) {
    c->ev_pool.push_back(a);
    c->ev_pool.push_back(b);
    return;
  }
  (void)hipEventRecord(b, st);  // after the scope's last launch
  c->pending.push_back(ProfPending{fam, bytes, a, b, tag, -1.0f});
}

// Each pair whose launches have completed gives up its time and its events
// (a pair still in flight keeps both: its events must not be recorded again
// before its dispatches end).  Launch groups whose algorithmic bytes are not
// known yet (tag >= 0: the PCG solves they served have not all ended) stay
// pending with their time alone, so the events held at any moment are those
// of launches since the last stream synchronisation.
void prof_resolve(mfs_context* c) {
  std::vector<ProfPending> keep;
  for (ProfPending p : c->pending) {
    if (p.a) {
      float ms = 0.0f;
      const hipError_t e = hipEventElapsedTime(&ms, p.a, p.b);
      if (e == hipErrorNotReady) {
        keep.push_back(p);
        continue;
      }
      p.ms = e == hipSuccess ? ms : -1.0f;
      c->ev_pool.push_back(p.a);
      c->ev_pool.push_back(p.b);
      p.a = p.b = nullptr;
    }
    if (p.tag >= 0) {
      keep.push_back(p);
      continue;
    }
    if (p.tag == -1 && p.ms >= 0.0f) {
      c->prof_ms[p.fam] += p.ms;
      c->prof_timed[p.fam]++;
      c->prof_bytes[p.fam] += p.bytes;
    }
  }
  c->pending.swap(keep);
}

}  // namespace mfs

mfs_context::~mfs_context() {
  for (const mfs::CgGraph& g : graphs) (void)hipGraphExecDestroy(g.exec);
  for (const mfs::ProfPending& p : pending) {
    if (p.a) (void)hipEventDestroy(p.a);
    if (p.b) (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : sync_events) (void)hipEventDestroy(e);
  if (h_stop) (void)hipHostFree(h_stop);
}

using namespace mfs;

extern "C" int mfs_profile_enable(mfs_context* ctx, int32_t stride) {
  clear_error();
  if (!ctx || stride < 0) return set_error(MFS_E_INVALID, "null context or negative stride");
  MFS_HIP(hipSetDevice(ctx->device));
  MFS_HIP(hipStreamSynchronize(ctx->stream));
  prof_resolve(ctx);
  ctx->prof_stride = stride;
  if (stride == 0) {
    std::memset(ctx->prof_ms, 0, sizeof ctx->prof_ms);
    std::memset(ctx->prof_timed, 0, sizeof ctx->prof_timed);
    std::memset(ctx->prof_launches, 0, sizeof ctx->prof_launches);
    std::memset(ctx->prof_bytes, 0, sizeof ctx->prof_bytes);
  }
  return MFS_OK;
}

extern "C" int mfs_profile_read(mfs_context* ctx, mfs_profile* out, int32_t reset) {
  clear_error();
  if (!ctx || !out) return set_error(MFS_E_INVALID, "null argument");
  MFS_HIP(hipSetDevice(ctx->device));
  MFS_HIP(hipStreamSynchronize(ctx->stream));
  prof_resolve(ctx);
  for (int f = 0; f < MFS_K_FAMILIES; ++f) {
    out->gpu_ms[f] = ctx->prof_ms[f];
    out->timed[f] = ctx->prof_timed[f];
    out->launches[f] = ctx->prof_launches[f];
    out->bytes[f] = ctx->prof_bytes[f];
  }
  if (reset) {
    std::memset(ctx->prof_ms, 0, sizeof ctx->prof_ms);
    std::memset(ctx->prof_timed, 0, sizeof ctx->prof_timed);
    std::memset(ctx->prof_launches, 0, sizeof ctx->prof_launches);
    std::memset(ctx->prof_bytes, 0, sizeof ctx->prof_bytes);
  }
  return MFS_OK;
}

extern "C" int mfs_character_get_info(const mfs_character* ch, mfs_character_info* info) {
  clear_error();
  if (!ch || !info) return set_error(MFS_E_INVALID, "null argument");
  std::memset(info, 0, sizeof *info);
  info->n_vertices = ch->n;
  info->n_tets = ch->m;
  info->n_blocks = ch->nnzb;
  info->n_pins = ch->npin;
  info->n_handles = ch->nh;
  info->bbox_diag = ch->bbox_diag;
  info->mean_edge = ch->lbar;
  return MFS_OK;
}
