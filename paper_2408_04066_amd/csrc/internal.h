// Host-side internals shared by the library's C++ translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mfs.h"
#include "common.h"

namespace mfs {

int set_error(int code, const char* fmt, ...);
void clear_error();
const char* last_error_text();  // this thread's last error

#define MFS_HIP(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return ::mfs::set_error(MFS_E_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                              __LINE__);                                                       \
  } while (0)

#define MFS_TRY(expr)           \
  do {                          \
    int rc_ = (expr);           \
    if (rc_ < 0) return rc_;    \
  } while (0)

// Owned device allocation.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  int alloc(size_t nbytes);              // exact size, old contents dropped
  int reserve(size_t nbytes);            // grow-only
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Grow-only pinned host buffer.
struct PinnedBuf {
  void* p = nullptr;
  size_t bytes = 0;
  PinnedBuf() = default;
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
  int reserve(size_t nbytes);
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Pinned staging for host-to-device uploads on one stream.  A copy from
// pinned memory reads its source when it executes, not when it is enqueued,
// so a chunk is rewritten only after the copy that last read it has
// completed (an event recorded behind that copy).  The caller's source may be
// reused as soon as upload() returns.  Eight chunks let several uploads be in
// flight without waiting.
struct UploadRing {
  static constexpr int kChunks = 8;
  PinnedBuf chunk[kChunks];
  hipEvent_t ev[kChunks] = {};
  bool in_flight[kChunks] = {};
  int next = 0;
  UploadRing() = default;
  UploadRing(const UploadRing&) = delete;
  UploadRing& operator=(const UploadRing&) = delete;
  ~UploadRing();
  int upload(hipStream_t st, void* dst, const void* src, size_t bytes);
};

}  // namespace mfs

namespace mfs {
constexpr int kProfDropped = -2;
struct ProfPending {
  int fam;
  double bytes;
  hipEvent_t a, b;  // the launch group's event pair, until its time is read (then null)
  int tag;          // index of an SpMV-family launch whose bytes are set after its run (-1: none,
                    // kProfDropped: never attributed, not counted)
  float ms = -1.0f; // the group's time once read (negative: not read, or not measurable)
};
struct CgGraph {
  const SysDesc* sd;
  const Tile* tiles;
  int ntv;
  int fp32, lpr, iters;
  bool pipelined;    // pipelined PCG kernels
  bool has_one;      // captured with a single system's descriptor as kernel argument
  SysDesc one;       // that descriptor (compared bytewise on lookup)
  hipGraphExec_t exec;
};
}  // namespace mfs

struct mfs_context {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int lpr = 4;                       // PCG lanes per block row (2, 4 or 8)
  int cg_first_run = 32;             // PCG iterations before the first convergence check
  int cg_min_run = 8, cg_max_run = 512;
  bool use_graphs = true;            // replay captured runs of PCG iterations
  int graph_iters = 8;               // PCG iterations per captured graph
  bool pipelined = false;            // FP32 solves: pipelined PCG, one kernel per iteration
  bool persistent = false;           // pipelined solves that fit the device: one cooperative launch
  int persist_lpr = 0;               // launch shape of the cached capacity below
  size_t persist_lds = 0;
  int persist_capacity = 0;          // workgroups of the persistent PCG the device holds at once
  int allread_tiles = mfs::kAllReadTiles;  // largest system (vertex tiles) with all-read PCG sums
  bool batch_async = true;           // batches (two-kernel or pipelined PCG): each system runs its own Newton steps
  std::vector<mfs::CgGraph> graphs;
  // batch scratch
  mfs::DevBuf desc, ctrl, red, cg, tiles, sys_ids, tmp;
  mfs::PinnedBuf h_red, h_cg;              // device-to-host reads (synchronised at once)
  std::vector<mfs::Ctrl> h_ctrl;           // host copies of the per-slot controls
  std::vector<mfs::Tile> h_tiles;          // host copy of the current tile list
  mfs::UploadRing up;                      // every host-to-device upload of the stream
  int32_t* h_stop = nullptr;               // host-mapped PCG stop flags, one per slot
  int32_t* d_stop = nullptr;               // their device address
  int stop_slots = 0;
  int32_t cg_epoch = 0;                    // last PCG solve number handed out
  std::vector<hipEvent_t> sync_events;     // completion events of queued PCG chunks
  // HIP-event profiler (mfs_profile_enable)
  int prof_stride = 0;
  double prof_ms[MFS_K_FAMILIES] = {};
  int64_t prof_timed[MFS_K_FAMILIES] = {};
  int64_t prof_launches[MFS_K_FAMILIES] = {};
  double prof_bytes[MFS_K_FAMILIES] = {};
  std::vector<hipEvent_t> ev_pool;
  std::vector<mfs::ProfPending> pending;
  // autotuned PCG schedules of this context, per size class
  struct TuneEntry {
    int size_class;
    mfs_tuning tuning;
    double ms;
  };
  std::vector<TuneEntry> tune_cache;
  ~mfs_context();
};

struct mfs_character {
  mfs_context* ctx = nullptr;
  int32_t n = 0, m = 0, nh = 0, nnzb = 0, npin = 0;
  double ks = 0.0, bbox_diag = 0.0, lbar = 0.0;
  std::vector<int32_t> perm;   // internal vertex -> caller vertex
  std::vector<int32_t> tperm;  // internal tet -> caller tet
  int ntv = 0, ntt = 0, nts = 0, ptile = 0;
  int max_tile_blocks = 0;     // matrix blocks of the densest 64-row vertex tile
  int blend_k = 0;             // rotation smoothing: handles per tet (0: cluster rotations)
  mfs::DevBuf blend_h, blend_w, Rt;  // blend handles / weights (blend_k planes of m), smoothed rotations (9 planes)
  bool has_solution = false;
  // resident mesh data
  mfs::DevBuf tets, G, wmu, wlam, info, X, rowptr, colidx, slot_ptr, contrib, diag, vpin_ptr, vpin_h, perm_d,
      tperm_d;
  // per-frame rig and solver state
  mfs::DevBuf Rh, th, x, xb, s;
  mfs::DevBuf fext;  // external vertex forces (internal order), allocated on first use
  // per-frame workspace (element records, BSR values, PCG vectors, partials):
  // one allocation carved by workspace_layout; empty after
  // mfs_character_release_workspace until a standalone solve needs it again
  mfs::DevBuf ws;
  std::vector<double> last_R, last_t;  // pose of the last solved frame (warm-start homotopy origin)
  mfs::SysDesc desc;  // resident pointers + the own workspace's, host copy
  size_t resident_bytes = 0, workspace_bytes = 0;
};

namespace mfs {

// Driver entry used by mfs_solve_frame / mfs_solve_batch.
int solve_systems(mfs_context* ctx, int count, mfs_character* const* chars, const double* const* R,
                  const double* const* t, const mfs_solve_opts* opts, double* const* x_out, mfs_solve_stats* stats);

int check_pose(const mfs_character* ch, const double* R, const double* t);

// Workspace of one frame solve of `ch`: total bytes (pieces 256-byte
// aligned), and the SysDesc workspace pointers carved from `base`.
size_t workspace_layout(const mfs_character* ch);
// Device bytes of a character with n vertices, m tets, nnzb matrix blocks and
// np pins: its resident data, and one frame solve's workspace.
size_t resident_bytes_of(int64_t n, int64_t m, int64_t nnzb, int64_t np);

// The allocation-free evaluation's per-device scratch array: its device
// address on `device` (which must be current), taken once per process by
// context creation.
int scratch_init(int device);
size_t workspace_bytes_of(int64_t n, int64_t m, int64_t nnzb);
void bind_workspace(const mfs_character* ch, char* base, SysDesc* d);
// Re-allocates the character's own workspace after a release.
int ensure_workspace(mfs_character* ch);

// Brackets one launch group of kernel family `fam` with an event pair when
// the context profiler samples it.  prof_resolve reads the times of pairs
// that have completed and returns their events to the pool at once (the
// events of a pair still in flight stay with it), and folds in the launch
// groups whose bytes are known.
struct ProfScope {
  mfs_context* c;
  int fam;
  double bytes;
  hipEvent_t a = nullptr, b = nullptr;
  int tag = -1;
  ProfScope(mfs_context* ctx, int family, double algorithmic_bytes = 0.0, int iteration_tag = -1);
  ~ProfScope();
};
// Fold completed event pairs into the counters (call after a stream sync).
void prof_resolve(mfs_context* c);
// MFS_OK when every field of t is in its documented range.
int check_tuning(const mfs_tuning* t);

// Uploads a validated pose into the character's pose buffers on ctx's stream
// (and smooths the per-tet rotations there when the character has a blend).
int upload_pose(mfs_context* ctx, mfs_character* ch, const double* R, const double* t);

}  // namespace mfs
