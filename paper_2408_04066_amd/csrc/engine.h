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

#include <vector>

#include "internal.h"

namespace mfs {

struct SlotState {
  mfs_character* ch = nullptr;
  bool used = false, fresh = false, done = false;
  int phase = 0;  // 0 mixed (s != J x), 1 Newton (s = J x)
  int status = MFS_OK;
  int iters = 0, mixed = 0, cg = 0, halvings = 0, clamped = 0, routed = 0, cg_fail = 0, resolves = 0;
  double E = INFINITY;
  bool E_known = false;
  double grad = NAN, step = NAN, relres = NAN;
  // PCG residual history (run sizing)
  // line search
  double alpha = 0.0;
  // pose homotopy (load stepping): start pose (R0, t0), target (R1, t1),
  // current pose (Rc, tc) at fraction tau, last converged fraction tau_done
  std::vector<double> R0, t0, R1, t1, Rc, tc;
  double tau = 1.0, tau_done = 0.0, delta = 1.0;
  int bisections = 0, load_mixed = 0;
};

struct TileSet {
  int nv = 0, nt = 0, ns = 0;
  Tile* dv = nullptr;
  Tile* dt = nullptr;
  Tile* ds = nullptr;
};

int upload_ctrl(mfs_context* ctx, int count);
// Host-mapped PCG stop flags for `slots` slots (grow-only; zeroed when made).
int ensure_stop_flags(mfs_context* ctx, int slots);
// An event (no timing) from the context's pool.
int sync_event(mfs_context* ctx, hipEvent_t* out);
int read_cg(mfs_context* ctx, int count, bool resolve = true);
int read_red(mfs_context* ctx, int count);
// Tiles of the listed slots (indices into by_slot), uploaded to the
// context's tile buffer, plus the slot-id list of the finalize kernel.  The
// caller has synchronised the stream since the staging buffers were last used.
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
  // E(x) for finished slots whose last step did not produce it.
  int finish_energies();
  bool busy(int slot) const { return slot_[slot].used && !slot_[slot].done; }
  bool finished(int slot) const { return slot_[slot].used && slot_[slot].done; }
  bool any_busy() const;
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

 private:
  int upload_desc();
  int set_pose(int slot, double tau);
  int restart_load_step(int slot);
  int tiles_for(const std::vector<int>& ids);
  // PCG for the listed slots in the given precision; with `failed`, slots
  // whose solve stops unconverged (cap or breakdown) are listed there instead
  // of counted as failures (the FP32 pass, re-solved in FP64).
  int run_cg(const std::vector<int>& act, bool fp32, std::vector<int>* failed);
  int fp32_cap(const mfs_character* ch) const;
  int linesearch(const std::vector<int>& act);

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
};

}  // namespace mfs
