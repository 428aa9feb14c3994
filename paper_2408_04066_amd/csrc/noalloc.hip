// Allocation-free evaluation entry point (mfs_evaluate_noalloc).
//
// mfs_evaluate runs the element pass, the assembly, the energy reduction and
// a block-sparse product over the character's solve workspace (element
// records, matrix values, right-hand side, partial sums), which it allocates
// when the character released it, and it stages host arrays and the
// descriptor through context buffers that grow on demand.  Callers that may
// not allocate device memory get the same evaluation here with every one of
// those buffers carved from one file-scope device array, `scratch`, of fixed
// size.  Each GPU holds its own copy of the array from the library's load
// until the process ends; its address on a device is taken once, at context
// creation on that device (scratch_init), and only that address is used from
// the host.  Calls on one GPU share the array: calls that overlap on one GPU
// (two streams, two threads) race on it.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "internal.h"
#include "launch.h"

namespace {
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;
}  // namespace

// The allocation-free entry point's workspace.  In host code this name is a
// host-side stand-in, not a device address: host code uses the per-device
// address from hipGetSymbolAddress (g_scratch_ptr) instead.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Tile list of one system (vertex, tet and slot tiles in that order, as the
// engine lays them out), one thread per tile.
__global__ void k_one_system_tiles(mfs::Tile* out, int n, int m, int nnzb, int ntv, int ntt, int nts) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntv + ntt + nts) return;
  int j, items, size;
  if (i < ntv) {
    j = i;
    items = n;
    size = mfs::kVTile;
  } else if (i < ntv + ntt) {
    j = i - ntv;
    items = m;
    size = mfs::kTTile;
  } else {
    j = i - ntv - ntt;
    items = nnzb;
    size = mfs::kSTile;
  }
  const int end = (j + 1) * size < items ? (j + 1) * size : items;
  out[i] = mfs::Tile{0, j * size, end, j};
}

__global__ void k_fill_zero(double* p, size_t count) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

__global__ void k_fill_int(int32_t* p, int32_t value) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = value;
}
}  // namespace

namespace mfs {

// Called by mfs_context_create with `device` current: the device address of
// this GPU's copy of `scratch`, kept for the rest of the process.
int scratch_init(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return set_error(MFS_E_INVALID, "device %d beyond %d", device, kMaxDevices);
  if (g_scratch_ptr[device]) return MFS_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return set_error(MFS_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
  g_scratch_ptr[device] = p;
  return MFS_OK;
}

}  // namespace mfs

using namespace mfs;

extern "C" int mfs_evaluate_noalloc(mfs_character* ch, const double* handle_R, const double* handle_t,
                                    const double* x, const double* v, int32_t memory_space, double* energy_out,
                                    double* grad_out, double* stretch_out, double* Kv_out) {
  clear_error();
  if (!ch || !x) return set_error(MFS_E_INVALID, "null character or positions");
  if (memory_space != MFS_MEM_HOST && memory_space != MFS_MEM_DEVICE)
    return set_error(MFS_E_INVALID, "invalid memory space");
  if ((v == nullptr) != (Kv_out == nullptr)) return set_error(MFS_E_INVALID, "v and Kv_out must both be given");
  mfs_context* ctx = ch->ctx;
  const int dev = ctx->device;
  MFS_TRY(check_pose(ch, handle_R, handle_t));

  // carve: descriptor | control block | tile list | system id | host staging | workspace
  const size_t n3 = 3 * sizeof(double) * (size_t)ch->n;
  const size_t m6 = 6 * sizeof(double) * (size_t)ch->m;
  const int ntiles = ch->ntv + ch->ntt + ch->nts;
  const bool host = memory_space == MFS_MEM_HOST;
  const size_t off_ctrl = align_up(sizeof(SysDesc));
  const size_t off_tiles = off_ctrl + align_up(sizeof(Ctrl));
  const size_t off_ids = off_tiles + align_up(sizeof(Tile) * (size_t)ntiles);
  const size_t off_tmp = off_ids + align_up(sizeof(int32_t));
  const size_t off_ws = off_tmp + (host ? align_up(std::max(n3, m6)) : 0);
  const size_t total = off_ws + workspace_layout(ch);
  if (total > kScratchBytes)
    return set_error(MFS_E_INVALID,
                     "character of %d tets needs %zu bytes of evaluation scratch; the allocation-free "
                     "evaluation holds at most %zu bytes (use mfs_evaluate)",
                     ch->m, total, kScratchBytes);
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev >= 0 && dev < kMaxDevices) base = static_cast<char*>(g_scratch_ptr[dev]);
  }
  if (!base) return set_error(MFS_E_INVALID, "no scratch address for device %d (no context was created on it)", dev);
  MFS_HIP(hipSetDevice(dev));
  hipStream_t st = ctx->stream;

  SysDesc* dsd = reinterpret_cast<SysDesc*>(base);
  Ctrl* dctrl = reinterpret_cast<Ctrl*>(base + off_ctrl);
  Tile* tiles = reinterpret_cast<Tile*>(base + off_tiles);
  int32_t* ids = reinterpret_cast<int32_t*>(base + off_ids);
  double* tmp = reinterpret_cast<double*>(base + off_tmp);

  // descriptor with the workspace in scratch (the character's own stays as it is)
  SysDesc hd = ch->desc;
  bind_workspace(ch, base + off_ws, &hd);
  hd.cg = nullptr;
  hd.stop_flag = nullptr;
  hd.ctrl = dctrl;
  Ctrl hc;
  std::memset(&hc, 0, sizeof hc);
  hc.phase = 1;  // s = J x; every trial step is 0: energy at x itself
  // the host sources below stay alive until the stream is synchronised at the end
  MFS_HIP(hipMemcpyAsync(dsd, &hd, sizeof(SysDesc), hipMemcpyHostToDevice, st));
  MFS_HIP(hipMemcpyAsync(dctrl, &hc, sizeof(Ctrl), hipMemcpyHostToDevice, st));
  MFS_HIP(hipMemcpyAsync(ch->Rh.p, handle_R, 9 * sizeof(double) * ch->nh, hipMemcpyHostToDevice, st));
  MFS_HIP(hipMemcpyAsync(ch->th.p, handle_t, 3 * sizeof(double) * ch->nh, hipMemcpyHostToDevice, st));
  if (ch->blend_k > 0)
    launch_blend_rot(st, ch->Rh.as<double>(), ch->m, ch->blend_k, ch->blend_h.as<int32_t>(), ch->blend_w.as<double>(),
                     ch->Rt.as<double>());
  hipLaunchKernelGGL(k_one_system_tiles, dim3((ntiles + 255) / 256), dim3(256), 0, st, tiles, ch->n, ch->m, ch->nnzb,
                     ch->ntv, ch->ntt, ch->nts);
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, ids, 0);
  // every trial energy is taken at x + 0 dx: dx starts at zero, whatever the
  // array held from the last call
  hipLaunchKernelGGL(k_fill_zero, dim3((3 * (size_t)ch->n + 255) / 256), dim3(256), 0, st, hd.dx, 3 * (size_t)ch->n);
  const double* xs = x;
  if (host) {
    MFS_HIP(hipMemcpyAsync(tmp, x, n3, hipMemcpyHostToDevice, st));
    xs = tmp;
  }
  launch_gather_rows(st, xs, ch->perm_d.as<int32_t>(), ch->n, 3, ch->x.as<double>());
  ch->has_solution = false;
  const Tile* tv = tiles;
  const Tile* tt = tiles + ch->ntv;
  const Tile* ts = tiles + ch->ntv + ch->ntt;
  launch_element(st, dsd, dctrl, tt, ch->ntt, 0);
  launch_assemble(st, dsd, ts, ch->nts, 0);
  launch_linesearch(st, dsd, dctrl, tt, ch->ntt, tv, ch->ntv);
  launch_finalize(st, dsd, ids, 1);
  MFS_HIP(hipGetLastError());
  if (grad_out) {
    double* dst = host ? tmp : grad_out;
    launch_scatter_rows(st, hd.b, ch->perm_d.as<int32_t>(), ch->n, 3, -1.0, dst);
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
    launch_gather_rows(st, vs, ch->perm_d.as<int32_t>(), ch->n, 3, static_cast<double*>(hd.p0));
    launch_spmv_plain(st, ch->rowptr.as<int32_t>(), static_cast<const double*>(hd.vals), ch->n,
                      static_cast<const double*>(hd.p0), static_cast<double*>(hd.q));
    double* dst = host ? tmp : Kv_out;
    launch_scatter_rows(st, static_cast<const double*>(hd.q), ch->perm_d.as<int32_t>(), ch->n, 3, 1.0, dst);
    if (host) MFS_HIP(hipMemcpyAsync(Kv_out, tmp, n3, hipMemcpyDeviceToHost, st));
  }
  MFS_HIP(hipGetLastError());
  double red[P_COUNT];
  MFS_HIP(hipMemcpyAsync(red, hd.red, sizeof red, hipMemcpyDeviceToHost, st));
  MFS_HIP(hipStreamSynchronize(st));
  if (energy_out) *energy_out = red[P_INF0] > 0.0 ? INFINITY : red[P_E0] + red[P_PIN0];
  return MFS_OK;
}
