// Asynchronous batch form of the engine (two-kernel or pipelined PCG).
//
// In step() every slot of a batch runs the same Newton iteration: the batch
// waits for the slowest slot's PCG solve before any slot takes its line
// search, so the tail of every Newton step is a few slots' PCG iterations in
// launches that are mostly empty.  Here each slot moves through its own
// Newton steps:
//
//   head (element pass, assembly, PCG start) -> PCG -> [FP64 re-solve of a
//   stalled FP32 solve] -> tail (line search, update, stop test) -> head ...
//
// and every PCG launch covers all slots that are solving at that moment, in
// each precision.  A slot's PCG stops by itself (its kernels return at once
// after it converges); the host watches the host-mapped stop flags, and when
// enough slots have stopped it drains the stream, moves them on, and queues
// one more chunk for the slots still solving before it takes the stopped
// slots' line searches, so the GPU keeps working through the host's
// decisions.  Per slot, the launches it takes part in and their arithmetic
// are those of step() and of a solve alone; only the company in each launch
// changes, so results are bitwise the same.
#include <algorithm>
#include <cstring>

#include "engine.h"
#include "launch.h"

namespace mfs {

bool Engine::async_mode() const {
  if (!async_ok_ || !ctx_->batch_async || ctx_->persistent) return false;
  int used = 0;
  for (const SlotState& S : slot_) used += S.used ? 1 : 0;
  return used > 1;
}

uint64_t Engine::progress_key() const {
  uint64_t k = (uint64_t)launched_[0] * 0x9E3779B97F4A7C15ull + (uint64_t)launched_[1];
  for (const SlotState& S : slot_)
    k = k * 1000003ull + (uint64_t)S.iters * 64 + (uint64_t)S.stage * 2 + (S.done ? 1 : 0) +
        ((uint64_t)S.resolves << 32);
  return k;
}

bool Engine::async_pending() const {
  for (const SlotState& S : slot_)
    if (S.used && !S.done && (S.stage == kPcg32 || S.stage == kPcg64 || S.stage == kRedo)) return true;
  return false;
}

// Vertex tiles of the listed slots into precision prec's own tile buffer (the
// PCG launches of the two live sets and the engine's other launches each keep
// their tile list, so none overwrites another's between chunks).
int Engine::vertex_tiles(int prec, const std::vector<int>& ids) {
  size_t total = 0;
  for (int i : ids) total += slot_[i].ch->ntv;
  std::vector<Tile> h;
  h.reserve(std::max<size_t>(total, 1));
  for (int i : ids) {
    const mfs_character* c = slot_[i].ch;
    for (int j = 0; j < c->ntv; ++j) h.push_back(Tile{i, j * kVTile, std::min(c->n, (j + 1) * kVTile), j});
  }
  if (h.empty()) h.push_back(Tile{0, 0, 0, 0});
  // growing the buffer frees the old one: no queued launch may still read it
  if (h.size() * sizeof(Tile) > ltiles_[prec].bytes) MFS_HIP(hipStreamSynchronize(ctx_->stream));
  MFS_TRY(ltiles_[prec].reserve(h.size() * sizeof(Tile)));
  MFS_TRY(ctx_->up.upload(ctx_->stream, ltiles_[prec].p, h.data(), h.size() * sizeof(Tile)));
  lts_[prec].dv = ltiles_[prec].as<Tile>();
  lts_[prec].nv = (int)total;
  return MFS_OK;
}

// Start a PCG solve for each listed slot: the Newton step's element pass,
// assembly and PCG start in precision prec (1 FP32, 0 FP64), or with `redo`
// the FP64 re-solve of a stalled FP32 solve, started from its FP32 iterate.
int Engine::async_head(const std::vector<int>& ids, int prec, bool redo) {
  mfs_context* ctx = ctx_;
  hipStream_t st = ctx->stream;
  Ctrl* hc = ctx->h_ctrl.data();
  const int32_t epoch = ++ctx->cg_epoch;
  for (int i : ids) {
    SlotState& S = slot_[i];
    if (!redo) {
      hc[i].phase = S.phase;
      hc[i].update_s = 0;
      hc[i].alpha = 0.0;
      // inexact Newton only on the constraint (as in step())
      hc[i].cg_adaptive = (o_.cg_adaptive && S.phase == 1) ? 1 : 0;
      hc[i].cg_eta_max = S.check_next ? kCheckEta : 0.0;
      S.check_next = false;
      hc[i].cg_cap = fp32_ ? fp32_cap(S.ch) : o_.cg_max;
    }
    hc[i].cg_epoch = epoch;
    S.epoch = epoch;
    S.pcg_cap = (prec == 1) ? fp32_cap(S.ch) : o_.cg_max;
  }
  // a pipelined solve's iteration j runs in the live set's launch
  // launched_[prec] + j, whose parity argument is that launch's: the system's
  // par0 maps it back to j's parity
  const bool pipe = pipe_set(prec);
  if (pipe)
    for (int i : ids)
      if (hd_[i].par0 != (int)(launched_[prec] & 1)) {
        hd_[i].par0 = (int)(launched_[prec] & 1);
        desc_dirty_ = true;
      }
  MFS_TRY(upload_desc());  // stream-ordered: in-flight launches read the old, equal, entries of other slots
  MFS_TRY(upload_ctrl(ctx, (int)slot_.size()));
  MFS_TRY(tiles_for(ids));
  const SysDesc* dsd = ctx->desc.as<SysDesc>();
  {
    ProfScope ps(ctx, MFS_K_ELEMENT);
    launch_element(st, dsd, ctx->ctrl.as<Ctrl>(), ts_.dt, ts_.nt, prec);
  }
  {
    ProfScope ps(ctx, MFS_K_ASSEMBLE);
    launch_assemble(st, dsd, ts_.ds, ts_.ns, prec);
  }
  {
    ProfScope ps(ctx, MFS_K_OTHER);
    // the FP32 pipelined solve keeps its vectors in FP64 (k_pcg_init)
    if (pipe && prec == 1)
      launch_pcg_init(st, dsd, ts_.dv, ts_.nv, 1);
    else
      launch_cg_init(st, dsd, ts_.dv, ts_.nv, prec, redo ? 1 : 0);
    if (pipe) launch_pcg_start(st, dsd, ts_.dv, ts_.nv, prec, ctx->lpr, nullptr);
  }
  MFS_HIP(hipGetLastError());
  const double word = prec ? 4.0 : 8.0;
  const double per_row = (pipe ? 48.0 : 6.0) * word;  // as in run_cg
  for (int i : ids) {
    SlotState& S = slot_[i];
    S.stage = prec ? kPcg32 : kPcg64;
    S.pcg_base = launched_[prec];
    S.span = -1;
    if (ctx->prof_stride > 0) {  // the profiler attributes timed launches to solve spans
      const mfs_character* c = S.ch;
      S.span = (int)spans_.size();
      spans_.push_back(SolveSpan{prec, launched_[prec], -1,
                                 c->nnzb * (9.0 * word + 4.0) + (c->n + 1) * 4.0 + c->n * per_row});
    }
    live_[prec].push_back(i);
  }
  gen_[prec] = -1;  // the live set changed
  return vertex_tiles(prec, live_[prec]);
}

// `run` iterations over precision prec's live set, launched directly (the live
// set changes too often for captured graphs to pay).
int Engine::async_enqueue(int prec, int run) {
  mfs_context* ctx = ctx_;
  const std::vector<int>& live = live_[prec];
  if (live.empty() || run <= 0) return MFS_OK;
  if (gen_[prec] < 0 && ctx->prof_stride > 0) {
    std::vector<int> g;
    for (int i : live) g.push_back(slot_[i].span);
    gen_[prec] = (int)gens_.size();
    gens_.push_back(std::move(g));
  }
  const SysDesc* dsd = ctx->desc.as<SysDesc>();
  const SysDesc* one = live.size() == 1 ? &hd_[live[0]] : nullptr;
  const bool pipe = pipe_set(prec);
  for (int j = 0; j < run; ++j) {
    {
      ProfScope ps(ctx, MFS_K_SPMV, 0.0, (int)timed_.size());
      if (ps.a && gen_[prec] >= 0)
        timed_.push_back(TimedLaunch{launched_[prec] + j, prec, gen_[prec]});
      else
        ps.tag = -1;
      if (pipe)
        launch_pcg_iter(ctx->stream, dsd, lts_[prec].dv, lts_[prec].nv, prec, ctx->lpr, one,
                        (int)((launched_[prec] + j) & 1));
      else
        launch_cg_spmv(ctx->stream, dsd, lts_[prec].dv, lts_[prec].nv, prec, ctx->lpr, one);
    }
    if (pipe) continue;
    ProfScope ps(ctx, MFS_K_CG_UPDATE);
    launch_cg_update(ctx->stream, dsd, lts_[prec].dv, lts_[prec].nv, prec, one);
  }
  launched_[prec] += run;
  MFS_HIP(hipGetLastError());
  return MFS_OK;
}

// Bytes of the timed SpMV launches whose every slot's solve has ended: the
// solves in the launch's live set that had not stopped before it.
void Engine::async_attribute() {
  for (ProfPending& p : ctx_->pending) {
    if (p.fam != MFS_K_SPMV || p.tag < 0 || p.tag >= (int)timed_.size()) continue;
    const TimedLaunch& t = timed_[p.tag];
    double by = 0.0;
    bool known = true;
    for (int sp : gens_[t.gen]) {
      if (sp < 0) continue;  // a solve started while the profiler was off
      const SolveSpan& s = spans_[sp];
      if (s.end < 0) {
        known = false;
        break;
      }
      if (t.g >= s.base && t.g < s.end) by += s.bytes;
    }
    if (!known) continue;
    p.bytes = by;
    p.tag = -1;
  }
}

// Run PCG chunks over the live sets until enough slots have stopped (or
// reached their cap), then drain and move the stopped slots on: a stalled
// FP32 solve to the FP64 re-solve queue, every other one to its tail.
int Engine::async_pcg() {
  mfs_context* ctx = ctx_;
  const int steady = std::max(1, std::min(ctx->cg_min_run, ctx->cg_max_run));
  const int32_t* flag = ctx->h_stop;
  auto stopped = [&](int i) { return __atomic_load_n(flag + i, __ATOMIC_ACQUIRE) == slot_[i].epoch; };
  // a chunk never takes a slot past its cap
  auto chunk = [&](int prec) {
    int run = steady;
    for (int i : live_[prec])
      run = std::min<int64_t>(run, slot_[i].pcg_base + slot_[i].pcg_cap - launched_[prec]);
    return std::max(run, 0);
  };
  auto enqueue_round = [&]() -> int {
    MFS_TRY(async_enqueue(1, chunk(1)));
    MFS_TRY(async_enqueue(0, chunk(0)));
    hipEvent_t e = nullptr;
    MFS_TRY(sync_event(ctx, &e));
    MFS_HIP(hipEventRecord(e, ctx->stream));
    queued_.push_back(e);
    return MFS_OK;
  };
  int total_tiles = 0;
  for (int p = 0; p < 2; ++p)
    for (int i : live_[p]) total_tiles += slot_[i].ch->ntv;
  if (total_tiles == 0) return MFS_OK;
  for (;;) {
    while (queued_.size() < 2) MFS_TRY(enqueue_round());
    // wait for: every slot stopped, stopped slots holding an eighth of the
    // live tiles or a quarter of the live slots, a slot at its cap, or the
    // oldest queued chunk done (then queue the next one)
    bool event = false;
    PollPacer pacer;
    for (;;) {
      int stopped_tiles = 0, stopped_slots = 0, live_slots = 0;
      bool capped = false;
      for (int p = 0; p < 2; ++p)
        for (int i : live_[p]) {
          ++live_slots;
          if (stopped(i)) {
            stopped_tiles += slot_[i].ch->ntv;
            ++stopped_slots;
          } else if (launched_[p] >= slot_[i].pcg_base + slot_[i].pcg_cap) {
            capped = true;
          }
        }
      if (stopped_slots == live_slots || 8 * stopped_tiles >= total_tiles || 4 * stopped_slots >= live_slots ||
          capped) {
        event = true;
        break;
      }
      const hipError_t e = hipEventQuery(queued_.front());
      if (e != hipSuccess && e != hipErrorNotReady) return set_error(MFS_E_HIP, "PCG chunk: %s", hipGetErrorString(e));
      if (e == hipSuccess) break;
      if (!pacer.pace())
        return set_error(MFS_E_HIP, "PCG chunk: no stop flag and no completed chunk in %d s",
                         PollPacer::kLimitSeconds);
    }
    if (event) break;
    ctx->sync_events.push_back(queued_.front());
    queued_.erase(queued_.begin());
  }
  // drain, then read every slot's PCG state (the read waits for every
  // queued chunk)
  MFS_TRY(read_cg(ctx, (int)slot_.size(), false));
  for (hipEvent_t e : queued_) ctx->sync_events.push_back(e);
  queued_.clear();
  const CgState* hg = ctx->h_cg.as<CgState>();
  for (int p = 1; p >= 0; --p) {
    std::vector<int> still, out;
    for (int i : live_[p]) {
      SlotState& S = slot_[i];
      const int64_t ran = launched_[p] - S.pcg_base;
      const int before = S.cg;
      if (hg[i].done) {
        S.cg += hg[i].iters;
        if (S.span >= 0) spans_[S.span].end = S.pcg_base + hg[i].iters;
      } else if (ran >= S.pcg_cap) {
        S.cg += (int)ran;
        if (S.span >= 0) spans_[S.span].end = launched_[p];
      } else {
        still.push_back(i);
        continue;
      }
      if (p == 0 && fp32_) S.cg_resolve += S.cg - before;  // an FP64 re-solve's iterations
      out.push_back(i);
      const bool ok = hg[i].done == 1;
      if (!ok && p == 1) {
        S.stage = kRedo;  // FP32 could not solve this Newton system
      } else {
        if (!ok) S.cg_fail++;
        S.stage = kTail;
      }
    }
    if (out.empty()) continue;
    // the solves' iterates into dx (FP64), per precision
    MFS_TRY(tiles_for(out));
    {
      ProfScope ps(ctx, MFS_K_OTHER);
      // (a pipelined iterate is FP64 in both precisions)
      launch_cg_finish(ctx->stream, ctx->desc.as<SysDesc>(), ts_.dv, ts_.nv, pipe_set(p) ? 0 : p);
    }
    MFS_HIP(hipGetLastError());
    live_[p].swap(still);
    gen_[p] = -1;
    MFS_TRY(vertex_tiles(p, live_[p]));
  }
  async_attribute();
  prof_resolve(ctx);
  return MFS_OK;
}

int Engine::advance() {
  mfs_context* ctx = ctx_;
  hipStream_t st = ctx->stream;
  MFS_HIP(hipSetDevice(ctx->device));
  const int n = (int)slot_.size();
  const SysDesc* dsd = ctx->desc.as<SysDesc>();
  const double* hr = ctx->h_red.as<double>();
  for (int i = 0; i < n; ++i)
    if (slot_[i].used && !slot_[i].done && !hd_[i].blk)
      return set_error(MFS_E_INVALID, "slot %d has no workspace bound", i);
  MFS_TRY(upload_desc());

  // mixed warm start of newly attached slots (as in step())
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
      slot_[i].stage = kHead;
    }
  }

  // slots starting a Newton step, and stalled FP32 solves to redo in FP64
  std::vector<int> heads, redo;
  for (int i = 0; i < n; ++i) {
    if (!slot_[i].used || slot_[i].done) continue;
    if (slot_[i].stage == kHead) heads.push_back(i);
    if (slot_[i].stage == kRedo) redo.push_back(i);
  }
  // (a context that left the asynchronous form only finishes the solves in flight)
  if (!heads.empty() && async_mode()) MFS_TRY(async_head(heads, fp32_ ? 1 : 0, false));
  if (!redo.empty()) {
    MFS_TRY(async_head(redo, 0, true));
    for (int i : redo) slot_[i].resolves++;
  }

  MFS_TRY(async_pcg());

  std::vector<int> tails;
  for (int i = 0; i < n; ++i)
    if (slot_[i].used && !slot_[i].done && slot_[i].stage == kTail) tails.push_back(i);
  if (tails.empty()) return MFS_OK;
  // keep the GPU on the slots still solving while the host takes the line
  // searches: a chunk queued behind the first pass's reduction copy runs
  // while the host reads the reductions and decides the steps
  if (!live_[0].empty() || !live_[1].empty()) {
    ls_fill_ = [this, ctx]() -> int {
      const int steady = std::max(1, std::min(ctx->cg_min_run, ctx->cg_max_run));
      for (int p = 1; p >= 0; --p) {
        int run = steady;
        for (int i : live_[p])
          run = std::min<int64_t>(run, slot_[i].pcg_base + slot_[i].pcg_cap - launched_[p]);
        MFS_TRY(async_enqueue(p, std::max(run, 0)));
      }
      return MFS_OK;
    };
  }
  const int ls = linesearch(tails);
  ls_fill_ = nullptr;
  MFS_TRY(ls);
  MFS_TRY(apply_update(tails));
  for (int i : tails) {
    MFS_TRY(finish_newton(i));
    slot_[i].stage = kHead;
  }
  // a finished batch leaves nothing behind: spans and timed launches end
  // with the solves they describe
  bool any = false;
  for (int i = 0; i < n; ++i) any = any || (slot_[i].used && !slot_[i].done);
  if (!any) {
    MFS_HIP(hipStreamSynchronize(st));
    async_attribute();
    // every solve has ended, so every timed launch is attributed; one that
    // is not (no span recorded for it) is dropped with the spans
    for (ProfPending& p : ctx->pending)
      if (p.tag >= 0) p.tag = kProfDropped;
    prof_resolve(ctx);
    spans_.clear();
    gens_.clear();
    timed_.clear();
    gen_[0] = gen_[1] = -1;
  }
  return MFS_OK;
}

}  // namespace mfs
