// Batch engine of the per-frame Newton solve.
//
// A fixed number of slots; each slot holds one character's frame solve
// (Algorithm 1, one pose).  step() runs one Newton iteration for every
// occupied, unfinished slot: element pass -> assembly -> PCG -> line search ->
// update, each one launch over the tiles of all those slots, with
// per-slot scalars, flags and fixed-order reductions, so a slot's result
// does not depend on which other slots are occupied.  Slots can be attached
// and retired between steps, which is how the serving loop batches
// continuously; mfs_solve_frame / mfs_solve_batch attach everything, step
// until all slots finish, and copy the results out.
#pragma once

#include <chrono>
#include <functional>
#include <thread>
#include <vector>

#include "internal.h"

namespace mfs {

// Largest PCG forcing term of a Newton step that checks a stop (see
// Engine::finish_newton).
constexpr double kCheckEta = 1e-2;

// Host side of a wait for the GPU (a stop flag, or the event behind a chunk
// of PCG launches): polls back to back for the first kSpinMicros, since a
// chunk usually ends within it and the GPU may have only a few tens of
// microseconds of queued work left (a sleep wakes up late), then sleeps
// between polls so that a long wait does not keep the HIP runtime busy with
// queries; a wait that sees nothing for kLimitSeconds is given up (the
// caller returns an error).
struct PollPacer {
  static constexpr int kSpinMicros = 2000;
  static constexpr int kLimitSeconds = 120;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  void reset() { t0 = std::chrono::steady_clock::now(); }
  // false once the wait has lasted longer than the limit
  bool pace() {
    const auto waited = std::chrono::steady_clock::now() - t0;
    if (waited < std::chrono::microseconds(kSpinMicros)) return true;
    std::this_thread::sleep_for(std::chrono::microseconds(20));
    return waited < std::chrono::seconds(kLimitSeconds);
  }
};

struct SlotState {
  mfs_character* ch = nullptr;
  bool used = false, fresh = false, done = false;
  int phase = 0;  // 0 mixed (s != J x), 1 Newton (s = J x)
  int status = MFS_OK;
  int iters = 0, mixed = 0, cg = 0, halvings = 0, clamped = 0, routed = 0, cg_fail = 0, resolves = 0;
  int cg_resolve = 0;  // PCG iterations of the FP64 re-solves (counted in cg too)
  double E = INFINITY;
  bool E_known = false;
  double grad = NAN, step = NAN, relres = NAN;
  // the previous full (alpha = 1) Newton-phase step at this pose, 0 if none:
  // with it the stop test sees how fast the steps contract
  double newton_prev = 0.0;
  // the next Newton step checks a stop: its PCG forcing term is at most
  // 1e-3 (see finish_newton)
  bool check_next = false;
  // PCG residual history (run sizing)
  // line search
  double alpha = 0.0;
  // pose homotopy (load stepping): start pose (R0, t0), target (R1, t1),
  // current pose (Rc, tc) at fraction tau, last converged fraction tau_done
  std::vector<double> R0, t0, R1, t1, Rc, tc;
  double tau = 1.0, tau_done = 0.0, delta = 1.0;
  int bisections = 0, load_mixed = 0;
  // asynchronous batch form: where the slot is in its own Newton step, and
  // its running PCG solve (global iteration index of its first iteration in
  // its precision's launch sequence, iteration cap, stop-flag epoch, span)
  int stage = 0;  // Engine::Stage
  int64_t pcg_base = 0;
  int pcg_cap = 0;
  int32_t epoch = 0;
  int span = -1;
};

struct TileSet {
  int nv = 0, nt = 0, ns = 0;
  Tile* dv = nullptr;
  Tile* dt = nullptr;
  Tile* ds = nullptr;
};

// Asynchronous batch form: one PCG solve of one slot, [base, end) in its
// precision's global launch sequence (end < 0 while it runs), with the
// algorithmic bytes one SpMV launch moves for it.
struct SolveSpan {
  int prec;
  int64_t base, end;
  double bytes;
};
// A timed SpMV launch of the asynchronous form: its global index, precision
// and the live set (span ids) it covered.
struct TimedLaunch {
  int64_t g;
  int prec;
  int gen;
};

int upload_ctrl(mfs_context* ctx, int count);
// Host-mapped PCG stop flags for `slots` slots (grow-only; zeroed when made).
int ensure_stop_flags(mfs_context* ctx, int slots);
// An event (no timing) from the context's pool.
int sync_event(mfs_context* ctx, hipEvent_t* out);
// Wait until the work queued on the context's stream is done, polling an
// event with a PollPacer (a stream synchronisation can return well after
// the work ends).
int wait_stream(mfs_context* ctx);
// Wait for an event recorded on the context's stream (polled with a
// PollPacer), then return it to the context's pool.
int wait_event(mfs_context* ctx, hipEvent_t e);
int read_cg(mfs_context* ctx, int count, bool resolve = true);
// The per-system reductions to the host.  With `fill`, the host waits for
// the copy only: fill() queues more work behind it first (work that neither
// the copy nor the host's use of the reductions depends on).
int read_red(mfs_context* ctx, int count, const std::function<int()>& fill = std::function<int()>());
// Tiles of the listed slots (indices into by_slot), uploaded in stream order
// to the context's tile buffer, plus the slot-id list of the finalize kernel
// (a buffer that must grow is replaced only after the stream drains).
int build_tile_list(mfs_context* ctx, const std::vector<mfs_character*>& by_slot, const std::vector<int>& ids,
                    TileSet* ts);

class Engine {
 public:
  explicit Engine(mfs_context* ctx) : ctx_(ctx) {}
  // Validate and adopt solve options (before any attach).
  int configure(const mfs_solve_opts* opts);
  // Size the per-slot device arrays; drops all slots.
  int reserve(int nslots);
  int slots() const { return (int)slot_.size(); }
  // Occupy a free slot with one frame solve; the pose is validated and
  // uploaded, x0 set per the warm-start option.  The warm start runs at the
  // slot's first step.
  int attach(int slot, mfs_character* ch, const double* R, const double* t);
  // Points the slot's workspace (element records, BSR values, PCG vectors)
  // at `base`, workspace_layout(ch) bytes of device memory that stay valid
  // until the slot retires; by default a slot uses the character's own.
  int bind_workspace(int slot, char* base);
  // One Newton iteration for every occupied, unfinished slot.
  int step();
  // Asynchronous batch form: each slot runs its own Newton steps.  One call is one scheduling event: slots at the start of a Newton
  // step get their element pass, assembly and PCG start; PCG chunks run over
  // every slot then solving, in each precision, until enough of them stop;
  // stopped FP32 solves that stalled are queued for an FP64 re-solve, and the
  // others take their line search and update and start their next step (or
  // finish).  A slot's arithmetic is the same as in step() and as alone; only
  // which slots share a launch changes.
  int advance();
  // advance() applies: the context has the asynchronous batch form enabled,
  // the engine's driver allows it, the engine holds more than one slot (a
  // single system gains nothing from it, and the lockstep form replays its
  // PCG runs as graphs), and the PCG form launches per iteration (the
  // persistent launch holds one set of systems for a whole solve, so it
  // keeps the lockstep form).
  bool async_mode() const;
  // The serving lanes keep the lockstep form (see server.cpp).
  void allow_async(bool on) { async_ok_ = on; }
  // Some slot is inside an asynchronous Newton step (solving, or waiting for
  // its FP64 re-solve): advance() must run until none is, even after the
  // context left the asynchronous form.
  bool async_pending() const;
  // The driver's next scheduling call: advance() or step().
  int run_once() { return (async_mode() || async_pending()) ? advance() : step(); }
  // E(x) for finished slots whose last step did not produce it.
  int finish_energies();
  bool busy(int slot) const { return slot_[slot].used && !slot_[slot].done; }
  bool finished(int slot) const { return slot_[slot].used && slot_[slot].done; }
  bool any_busy() const;
  // Changes whenever a scheduling call moved any slot on or launched PCG
  // iterations (the drive loops stop with an error after calls that do
  // neither).
  uint64_t progress_key() const;
  // Copy a finished slot's positions to x_out (caller's vertex order), host
  // or device; synchronises the stream.
  int output(int slot, double* x_out, int mem);
  void stats(int slot, mfs_solve_stats* s) const;
  void retire(int slot) {
    slot_[slot] = SlotState();
    desc_dirty_ = true;
    tiles_valid_ = false;
  }
  const SlotState& state(int slot) const { return slot_[slot]; }

  enum Stage { kHead = 0, kPcg32 = 1, kPcg64 = 2, kRedo = 3, kTail = 4 };

 private:
  int upload_desc();
  // the end of a Newton step for slot i after its update: counters, stop
  // test, load stepping; sets done/status
  int finish_newton(int i);
  // x (and s in the mixed phase) updated by each listed slot's accepted step
  int apply_update(const std::vector<int>& act);
  // asynchronous form
  int async_head(const std::vector<int>& ids, int prec, bool redo);
  int async_pcg();
  int async_enqueue(int prec, int run);
  // precision prec's live set runs the pipelined PCG (else the two-kernel
  // form; FP64 re-solves of stalled FP32 solves always do)
  bool pipe_set(int prec) const { return ctx_->pipelined && (prec == 1 || !fp32_); }
  void async_attribute();
  int vertex_tiles(int prec, const std::vector<int>& ids);
  int set_pose(int slot, double tau);
  int restart_load_step(int slot);
  int tiles_for(const std::vector<int>& ids);
  // PCG for the listed slots in the given precision; with `failed`, slots
  // whose solve stops unconverged (cap or breakdown) are listed there instead
  // of counted as failures (the FP32 pass, re-solved in FP64).
  // `before_wait`, when given, queues more work behind the run's last
  // launches (after the iterates go to dx) before the host waits for the
  // PCG state; the persistent launch does not call it.
  int run_cg(const std::vector<int>& act, bool fp32, std::vector<int>* failed,
             const std::function<int()>& before_wait = std::function<int()>());
  int fp32_cap(const mfs_character* ch) const;
  // The line search of the listed slots; its first pass may have been
  // queued already by ls_queue (then ls_event_ is set).
  int linesearch(const std::vector<int>& act);
  // Queue the first line-search pass of the listed slots (launches and the
  // copy of its reductions, ls_event_ recorded after it) without waiting.
  int ls_queue(const std::vector<int>& act);
  void ls_setup(const std::vector<int>& act);

  mfs_context* ctx_;
  mfs_solve_opts o_{};
  int fp32_ = 0;
  int32_t cg_epoch_ = 0;  // epoch of the PCG solve being run
  std::vector<SlotState> slot_;
  std::vector<SysDesc> hd_;
  bool desc_dirty_ = true;
  TileSet ts_;
  std::vector<int> tile_ids_;
  std::vector<const mfs_character*> tile_chars_;
  bool tiles_valid_ = false;
  // asynchronous form: per precision (0 FP64, 1 FP32) the live set, its
  // vertex tiles, the launches enqueued so far, the queued chunks' completion
  // events; solve spans and timed launches for the profiler
  std::vector<int> live_[2];
  TileSet lts_[2];
  DevBuf ltiles_[2];
  int64_t launched_[2] = {0, 0};
  bool async_ok_ = true;
  std::vector<hipEvent_t> queued_;
  std::vector<SolveSpan> spans_;
  std::vector<std::vector<int>> gens_;
  int gen_[2] = {-1, -1};
  std::vector<TimedLaunch> timed_;
  // asynchronous form: PCG work for the slots still solving, queued behind
  // the first line-search pass's reduction copy (see linesearch)
  std::function<int()> ls_fill_;
  // lockstep form: event behind a queued first line-search pass, or null
  hipEvent_t ls_event_ = nullptr;
};

}  // namespace mfs
