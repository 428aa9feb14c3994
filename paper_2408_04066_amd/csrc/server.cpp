// Serving loop: continuous batching of frame-solve requests.
//
// A worker thread owns the context's stream and one batch Engine with a
// fixed number of slots.  Between Newton steps it admits queued requests:
// a request takes a free slot when its character has no frame in flight
// (frames of one character run in submission order, so a warm start from
// the previous frame sees that frame's result) and, for a character whose
// own workspace was released, when its workspace fits in the server's
// device arena.  Admitted requests join the running batch at the next
// step, so new work overlaps work already on the GPU; finished slots are
// copied out and retired after every step.  A request's result does not
// depend on what else is in the batch (per-slot scalars and fixed-order
// reductions in every kernel).
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>

#include "engine.h"
#include "internal.h"

namespace mfs {

namespace {

// First-fit allocator over one device allocation (offsets in bytes, 256-byte
// granules), neighbours coalesced on release.
class Arena {
 public:
  int init(size_t bytes) {
    cap_ = bytes / kGranule * kGranule;
    free_.clear();
    if (cap_ == 0) return MFS_OK;
    MFS_TRY(buf_.alloc(cap_));
    free_[0] = cap_;
    return MFS_OK;
  }
  size_t capacity() const { return cap_; }
  size_t in_use() const { return used_; }
  size_t peak() const { return peak_; }
  char* base() const { return buf_.as<char>(); }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + kGranule - 1) / kGranule * kGranule;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + kGranule - 1) / kGranule * kGranule;
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  static constexpr size_t kGranule = 256;
  DevBuf buf_;
  size_t cap_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

enum ReqState { kQueued = 0, kRunning = 1, kDone = 2 };

struct Request {
  mfs_character* ch = nullptr;
  std::vector<double> R, t, x;
  int state = kQueued;
  int status = MFS_OK;
  std::string error;
  mfs_solve_stats stats{};
  mfs_request_times times{};
  int slot = -1;
  bool arena = false;
  size_t ws_off = 0, ws_bytes = 0;
};

}  // namespace
}  // namespace mfs

using namespace mfs;

namespace mfs {
namespace {

// One lane: a worker thread, its context's stream and one batch Engine.
struct ServerLane {
  mfs_context* ctx = nullptr;
  mfs_server_opts o{};
  Engine eng;
  Arena arena;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Request> reqs;
  std::vector<uint64_t> slot_req;  // ticket per slot, 0 = free
  std::unordered_set<const mfs_character*> in_flight;
  uint64_t next_ticket = 1;
  bool stop = false;
  int fatal = MFS_OK;
  std::string fatal_msg;
  int64_t submitted = 0, completed = 0, steps = 0;
  double slot_steps = 0.0;
  std::chrono::steady_clock::time_point origin = std::chrono::steady_clock::now();
  std::thread worker;
  bool retune = false;  // a PCG schedule waits to be applied between steps
  mfs_tuning tuning{};

  // The lanes run the lockstep batch form: with the asynchronous one, a C5
  // serving run (two lanes, 300 requests/s) stopped completing requests
  // after 6,577 of them, and the cause is not known.
  explicit ServerLane(mfs_context* c) : ctx(c), eng(c) { eng.allow_async(false); }
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - origin).count();
  }
  void run();
  void admit_locked();
  void fail_all_locked(int code, const std::string& msg);
  int complete_finished();
};

void ServerLane::fail_all_locked(int code, const std::string& msg) {
  fatal = code;
  fatal_msg = msg;
  for (auto& kv : reqs) {
    Request& r = kv.second;
    if (r.state == kDone) continue;
    r.state = kDone;
    r.status = code;
    r.error = msg;
    r.stats.status = code;
    r.times.done_s = now();
  }
  queue.clear();
  cv_done.notify_all();
}

// Under the lock: move queued requests into free slots, in queue order,
// skipping requests whose character has a frame in flight; stop at the
// first request whose workspace does not fit the arena (so a large request
// is not starved by smaller ones behind it).
void ServerLane::admit_locked() {
  for (auto it = queue.begin(); it != queue.end();) {
    int slot = -1;
    for (int i = 0; i < (int)slot_req.size(); ++i)
      if (slot_req[i] == 0) {
        slot = i;
        break;
      }
    if (slot < 0) return;
    const uint64_t tk = *it;
    Request& r = reqs[tk];
    if (in_flight.count(r.ch)) {
      ++it;
      continue;
    }
    if (!r.ch->ws.p) {
      if (!arena.alloc(r.ws_bytes, &r.ws_off)) return;
      r.arena = true;
    }
    int rc = eng.attach(slot, r.ch, r.R.data(), r.t.data());
    if (rc >= 0 && r.arena) rc = eng.bind_workspace(slot, arena.base() + r.ws_off);
    if (rc < 0) {
      if (eng.state(slot).used) eng.retire(slot);
      if (r.arena) arena.release(r.ws_off, r.ws_bytes);
      r.arena = false;
      r.state = kDone;
      r.status = rc;
      r.error = last_error_text();
      r.stats.status = rc;
      r.times.admit_s = r.times.done_s = now();
      it = queue.erase(it);
      cv_done.notify_all();
      continue;
    }
    r.state = kRunning;
    r.slot = slot;
    r.times.admit_s = now();
    slot_req[slot] = tk;
    in_flight.insert(r.ch);
    it = queue.erase(it);
  }
}

// Worker only: copy out and retire every finished slot.
int ServerLane::complete_finished() {
  bool any = false;
  for (int i = 0; i < eng.slots(); ++i) any = any || eng.finished(i);
  if (!any) return MFS_OK;
  MFS_TRY(eng.finish_energies());
  for (int i = 0; i < eng.slots(); ++i) {
    if (!eng.finished(i)) continue;
    uint64_t tk;
    Request* r;
    {
      std::lock_guard<std::mutex> lk(mu);
      tk = slot_req[i];
      r = &reqs[tk];
    }
    r->x.resize(3 * (size_t)r->ch->n);
    MFS_TRY(eng.output(i, r->x.data(), MFS_MEM_HOST));  // synchronises the stream
    mfs_solve_stats st{};
    eng.stats(i, &st);
    const int status = eng.state(i).status;
    eng.retire(i);
    std::lock_guard<std::mutex> lk(mu);
    if (r->arena) arena.release(r->ws_off, r->ws_bytes);
    r->arena = false;
    r->stats = st;
    r->status = status;
    r->state = kDone;
    r->times.done_s = now();
    slot_req[i] = 0;
    in_flight.erase(r->ch);
    ++completed;
    cv_done.notify_all();
  }
  return MFS_OK;
}

void ServerLane::run() {
  (void)hipSetDevice(ctx->device);
  int idle = 0;  // scheduling calls in a row that moved no slot on
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !queue.empty() || eng.any_busy(); });
      if (stop) return;
      if (retune) {  // between steps: no kernel of this lane is in flight after the sync inside
        retune = false;
        const int rc = mfs_context_set_tuning(ctx, &tuning);
        if (rc < 0) {
          fail_all_locked(rc, last_error_text());
          return;
        }
      }
      admit_locked();
      if (!eng.any_busy()) continue;  // everything admitted this round failed
      int occupied = 0;
      for (uint64_t tk : slot_req) occupied += tk != 0;
      slot_steps += occupied;
      ++steps;
    }
    const uint64_t before = eng.progress_key();
    int rc = eng.run_once();
    if (rc >= 0) {
      idle = eng.progress_key() == before ? idle + 1 : 0;
      if (idle > 8) rc = set_error(MFS_E_HIP, "serving lane: scheduling calls make no progress");
    }
    if (rc >= 0) rc = complete_finished();
    if (rc < 0) {
      const std::string msg = last_error_text();
      std::lock_guard<std::mutex> lk(mu);
      fail_all_locked(rc, msg);
      return;
    }
  }
}

}  // namespace
}  // namespace mfs

extern "C" void mfs_default_server_opts(mfs_server_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->slots = 16;
  o->queue_capacity = 4096;
  o->workspace_budget_bytes = 0;
  mfs_default_opts(&o->solve);
  o->lanes = 1;
}

// The server: lanes of their own (lane 0 on the caller's context, the others
// on contexts of their own on the same device, each with its own stream),
// a request going to the lane of its character's size class.  Tickets carry
// the lane in their low bits.
constexpr int kMaxLanes = 4;

struct mfs_server {
  mfs_context* ctx = nullptr;  // the caller's context (characters belong to it)
  std::vector<std::unique_ptr<mfs::ServerLane>> lanes;
  std::vector<mfs_context*> own_ctx;  // contexts made for lanes 1.. (destroyed with the server)
  std::vector<int64_t> max_tets;      // lane i < lanes - 1 takes characters of at most max_tets[i] tets
  int lane_of(const mfs_character* ch) const {
    for (size_t i = 0; i < max_tets.size(); ++i)
      if (ch->m <= max_tets[i]) return (int)i;
    return (int)lanes.size() - 1;
  }
  ~mfs_server();
};

namespace mfs {
namespace {

int lane_start(mfs_context* ctx, const mfs_server_opts& o, std::unique_ptr<ServerLane>* out) {
  MFS_HIP(hipSetDevice(ctx->device));
  std::unique_ptr<ServerLane> s(new ServerLane(ctx));
  s->o = o;
  MFS_TRY(s->eng.configure(&o.solve));
  MFS_TRY(s->eng.reserve(o.slots));
  MFS_TRY(s->arena.init(o.workspace_budget_bytes));
  s->slot_req.assign(o.slots, 0);
  MFS_HIP(hipStreamSynchronize(ctx->stream));
  ServerLane* raw = s.get();
  try {
    s->worker = std::thread([raw] { raw->run(); });
  } catch (...) {
    return set_error(MFS_E_UNSUPPORTED, "could not start a server thread");
  }
  *out = std::move(s);
  return MFS_OK;
}

void lane_stop(ServerLane* s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->ctx->device);
  (void)hipStreamSynchronize(s->ctx->stream);
}

int lane_submit(ServerLane* s, mfs_character* ch, const double* R, const double* t, uint64_t* ticket) {
  Request r;
  r.ch = ch;
  r.R.assign(R, R + 9 * (size_t)ch->nh);
  r.t.assign(t, t + 3 * (size_t)ch->nh);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->fatal < 0) return set_error(s->fatal, "server stopped: %s", s->fatal_msg.c_str());
  if (!ch->ws.p) {
    r.ws_bytes = ch->workspace_bytes;
    if (r.ws_bytes > s->arena.capacity())
      return set_error(MFS_E_BUSY, "request workspace of %zu bytes exceeds the server budget of %zu bytes",
                       r.ws_bytes, s->arena.capacity());
  }
  if ((int64_t)s->queue.size() >= s->o.queue_capacity) return set_error(MFS_E_BUSY, "request queue is full");
  r.times.submit_s = s->now();
  const uint64_t tk = s->next_ticket++;
  s->reqs.emplace(tk, std::move(r));
  s->queue.push_back(tk);
  ++s->submitted;
  s->cv_work.notify_one();
  *ticket = tk;
  return MFS_OK;
}

int take_result(ServerLane* s, std::unique_lock<std::mutex>& lk, uint64_t ticket, double* x_out,
                mfs_solve_stats* stats, mfs_request_times* times) {
  auto it = s->reqs.find(ticket);
  Request& r = it->second;
  const int status = r.status;
  if (x_out && !r.x.empty()) std::memcpy(x_out, r.x.data(), r.x.size() * sizeof(double));
  if (stats) *stats = r.stats;
  if (times) *times = r.times;
  const std::string err = r.error;
  s->reqs.erase(it);
  lk.unlock();
  if (status < 0) return set_error(status, "%s", err.c_str());
  if (status == MFS_W_NOT_CONVERGED) set_error(status, "frame solve did not converge");
  return status;
}

int decode(mfs_server* s, uint64_t ticket, ServerLane** lane, uint64_t* lane_ticket) {
  const uint64_t l = ticket % kMaxLanes;
  if (l >= s->lanes.size()) return set_error(MFS_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  *lane = s->lanes[l].get();
  *lane_ticket = ticket / kMaxLanes;
  return MFS_OK;
}

}  // namespace
}  // namespace mfs

mfs_server::~mfs_server() {
  for (auto& l : lanes) mfs::lane_stop(l.get());
  lanes.clear();
  for (mfs_context* c : own_ctx) (void)mfs_context_destroy(c);
}

extern "C" int mfs_server_create(mfs_context* ctx, const mfs_server_opts* opts, mfs_server** out) {
  clear_error();
  if (!ctx || !out) return set_error(MFS_E_INVALID, "null context or output");
  *out = nullptr;
  mfs_server_opts o;
  mfs_default_server_opts(&o);
  if (opts) o = *opts;
  if (o.slots < 1 || o.slots > 1024) return set_error(MFS_E_INVALID, "slots must be in 1..1024");
  if (o.queue_capacity < 1) return set_error(MFS_E_INVALID, "queue capacity must be positive");
  if (o.lanes < 1 || o.lanes > kMaxLanes) return set_error(MFS_E_INVALID, "lanes must be in 1..%d", kMaxLanes);
  for (int i = 0; i + 1 < o.lanes; ++i)
    if (o.lane_max_tets[i] < 1 || (i > 0 && o.lane_max_tets[i] <= o.lane_max_tets[i - 1]))
      return set_error(MFS_E_INVALID, "lane_max_tets must be positive and increasing");
  if (o.solve.output_memory != MFS_MEM_HOST)
    return set_error(MFS_E_UNSUPPORTED, "server results are returned in host memory");
  MFS_HIP(hipSetDevice(ctx->device));
  std::unique_ptr<mfs_server> s(new mfs_server());
  s->ctx = ctx;
  s->max_tets.assign(o.lane_max_tets, o.lane_max_tets + (o.lanes - 1));
  mfs_tuning tuning;
  MFS_TRY(mfs_context_get_tuning(ctx, &tuning));
  for (int l = 0; l < o.lanes; ++l) {
    mfs_context* lc = ctx;
    if (l > 0) {  // a context of its own (own stream), with the caller's PCG schedule
      MFS_TRY(mfs_context_create(ctx->device, nullptr, &lc));
      s->own_ctx.push_back(lc);
      MFS_TRY(mfs_context_set_tuning(lc, &tuning));
    }
    std::unique_ptr<ServerLane> lane;
    MFS_TRY(lane_start(lc, o, &lane));
    s->lanes.push_back(std::move(lane));
  }
  *out = s.release();
  return MFS_OK;
}

extern "C" int mfs_server_destroy(mfs_server* s) {
  if (!s) return MFS_OK;
  delete s;
  return MFS_OK;
}

extern "C" int mfs_server_submit(mfs_server* s, mfs_character* ch, const double* R, const double* t,
                                 uint64_t* ticket) {
  clear_error();
  if (!s || !ch || !ticket) return set_error(MFS_E_INVALID, "null server, character or ticket");
  if (ch->ctx != s->ctx) return set_error(MFS_E_INVALID, "character belongs to another context");
  MFS_TRY(check_pose(ch, R, t));
  const int l = s->lane_of(ch);
  uint64_t tk = 0;
  MFS_TRY(lane_submit(s->lanes[l].get(), ch, R, t, &tk));
  *ticket = tk * kMaxLanes + (uint64_t)l;
  return MFS_OK;
}

extern "C" int mfs_server_poll(mfs_server* s, uint64_t ticket, double* x_out, mfs_solve_stats* stats,
                               mfs_request_times* times, int32_t* done) {
  clear_error();
  if (!s || !done) return set_error(MFS_E_INVALID, "null server or done flag");
  ServerLane* lane;
  uint64_t tk;
  MFS_TRY(decode(s, ticket, &lane, &tk));
  std::unique_lock<std::mutex> lk(lane->mu);
  auto it = lane->reqs.find(tk);
  if (it == lane->reqs.end()) return set_error(MFS_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  if (it->second.state != kDone) {
    *done = 0;
    return MFS_OK;
  }
  *done = 1;
  return take_result(lane, lk, tk, x_out, stats, times);
}

extern "C" int mfs_server_wait(mfs_server* s, uint64_t ticket, double* x_out, mfs_solve_stats* stats,
                               mfs_request_times* times) {
  clear_error();
  if (!s) return set_error(MFS_E_INVALID, "null server");
  ServerLane* lane;
  uint64_t tk;
  MFS_TRY(decode(s, ticket, &lane, &tk));
  std::unique_lock<std::mutex> lk(lane->mu);
  auto it = lane->reqs.find(tk);
  if (it == lane->reqs.end()) return set_error(MFS_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  lane->cv_done.wait(lk, [&] {
    auto j = lane->reqs.find(tk);
    return j == lane->reqs.end() || j->second.state == kDone;
  });
  if (lane->reqs.find(tk) == lane->reqs.end())
    return set_error(MFS_E_INVALID, "ticket %llu was taken by another caller", (unsigned long long)ticket);
  return take_result(lane, lk, tk, x_out, stats, times);
}

extern "C" int mfs_server_set_lane_tuning(mfs_server* s, int32_t lane, const mfs_tuning* t) {
  clear_error();
  if (!s || !t) return set_error(MFS_E_INVALID, "null server or tuning");
  if (lane < 0 || lane >= (int)s->lanes.size()) return set_error(MFS_E_INVALID, "lane %d out of range", lane);
  MFS_TRY(check_tuning(t));
  mfs::ServerLane* l = s->lanes[lane].get();
  std::lock_guard<std::mutex> lk(l->mu);
  if (l->fatal < 0) return set_error(l->fatal, "server stopped: %s", l->fatal_msg.c_str());
  l->tuning = *t;
  l->retune = true;
  l->cv_work.notify_one();
  return MFS_OK;
}

extern "C" int mfs_server_get_info(mfs_server* s, mfs_server_info* info) {
  clear_error();
  if (!s || !info) return set_error(MFS_E_INVALID, "null server or info");
  std::memset(info, 0, sizeof *info);
  int fatal = MFS_OK;
  std::string msg;
  for (auto& lp : s->lanes) {
    ServerLane* l = lp.get();
    std::lock_guard<std::mutex> lk(l->mu);
    info->submitted += l->submitted;
    info->completed += l->completed;
    info->steps += l->steps;
    info->queued += (int32_t)l->queue.size();
    for (uint64_t tk : l->slot_req) info->running += tk != 0;
    info->arena_bytes += l->arena.capacity();
    info->arena_in_use += l->arena.in_use();
    info->arena_peak += l->arena.peak();
    info->slot_steps += l->slot_steps;
    if (l->fatal < 0 && fatal == MFS_OK) {
      fatal = l->fatal;
      msg = l->fatal_msg;
    }
  }
  return fatal < 0 ? set_error(fatal, "server stopped: %s", msg.c_str()) : MFS_OK;
}
