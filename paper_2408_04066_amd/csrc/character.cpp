// Character creation: input validation, bandwidth-reducing vertex order,
// 3x3-block sparsity pattern of the condensed matrix with its
// element-to-block assembly map, pin grouping, and upload of the resident
// mesh data.  Runs once per character (not per frame).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <numeric>

#include "internal.h"
#include "launch.h"

namespace mfs {

static thread_local std::string g_last_error;

int set_error(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

void clear_error() { g_last_error.clear(); }

const char* last_error_text() { return g_last_error.c_str(); }

int DevBuf::alloc(size_t nbytes) {
  release();
  if (nbytes == 0) return MFS_OK;
  if (hipMalloc(&p, nbytes) != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    return set_error(MFS_E_OOM, "device allocation of %zu bytes failed", nbytes);
  }
  bytes = nbytes;
  return MFS_OK;
}

int DevBuf::reserve(size_t nbytes) { return nbytes <= bytes ? MFS_OK : alloc(nbytes); }

int PinnedBuf::reserve(size_t nbytes) {
  if (nbytes <= bytes) return MFS_OK;
  if (p) hipHostFree(p);
  p = nullptr;
  bytes = 0;
  if (hipHostMalloc(&p, nbytes, hipHostMallocDefault) != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    return set_error(MFS_E_OOM, "pinned host allocation of %zu bytes failed", nbytes);
  }
  bytes = nbytes;
  return MFS_OK;
}

UploadRing::~UploadRing() {
  for (int k = 0; k < kChunks; ++k) {
    if (in_flight[k]) (void)hipEventSynchronize(ev[k]);
    if (ev[k]) (void)hipEventDestroy(ev[k]);
  }
}

int UploadRing::upload(hipStream_t st, void* dst, const void* src, size_t bytes) {
  if (!bytes) return MFS_OK;
  const int k = next;
  next = (next + 1) % kChunks;
  if (!ev[k]) MFS_HIP(hipEventCreateWithFlags(&ev[k], hipEventDisableTiming));
  if (in_flight[k]) {
    MFS_HIP(hipEventSynchronize(ev[k]));
    in_flight[k] = false;
  }
  MFS_TRY(chunk[k].reserve(bytes));
  std::memcpy(chunk[k].p, src, bytes);
  MFS_HIP(hipMemcpyAsync(dst, chunk[k].p, bytes, hipMemcpyHostToDevice, st));
  MFS_HIP(hipEventRecord(ev[k], st));
  in_flight[k] = true;
  return MFS_OK;
}

// Copy `count` elements from host or device memory into a host vector.
template <class T>
static int fetch(const T* src, size_t count, int mem, std::vector<T>& dst) {
  if (count && !src) return set_error(MFS_E_INVALID, "null input array");
  dst.resize(count);
  if (!count) return MFS_OK;
  if (mem == MFS_MEM_DEVICE) {
    MFS_HIP(hipMemcpy(dst.data(), src, count * sizeof(T), hipMemcpyDeviceToHost));
  } else if (mem == MFS_MEM_HOST) {
    std::memcpy(dst.data(), src, count * sizeof(T));
  } else {
    return set_error(MFS_E_INVALID, "memory_space must be MFS_MEM_HOST or MFS_MEM_DEVICE");
  }
  return MFS_OK;
}

template <class T>
static int upload(DevBuf& buf, const T* src, size_t count) {
  MFS_TRY(buf.alloc(std::max<size_t>(count, 1) * sizeof(T)));
  if (count) MFS_HIP(hipMemcpy(buf.p, src, count * sizeof(T), hipMemcpyHostToDevice));
  return MFS_OK;
}

// Reverse Cuthill-McKee order (order[new] = old) of an undirected graph in
// CSR form (no self loops); each component starts from a pseudo-peripheral
// vertex found by repeated breadth-first search (George-Liu).
static void rcm_order(int n, const std::vector<int32_t>& ptr, const std::vector<int32_t>& adj,
                      std::vector<int32_t>& order) {
  std::vector<int32_t> deg(n), level(n, -1), stamp(n, -1);
  for (int v = 0; v < n; ++v) deg[v] = ptr[v + 1] - ptr[v];
  std::vector<char> placed(n, 0);
  std::vector<int32_t> queue(n), nb;
  order.clear();
  order.reserve(n);
  int bfs_id = 0;
  auto bfs = [&](int root, int& last_begin, int& count) {
    // returns eccentricity; queue[0..count) is the BFS order of the component
    ++bfs_id;
    int head = 0;
    count = 0;
    queue[count++] = root;
    stamp[root] = bfs_id;
    level[root] = 0;
    int ecc = 0;
    last_begin = 0;
    while (head < count) {
      const int v = queue[head++];
      for (int e = ptr[v]; e < ptr[v + 1]; ++e) {
        const int w = adj[e];
        if (stamp[w] != bfs_id) {
          stamp[w] = bfs_id;
          level[w] = level[v] + 1;
          if (level[w] > ecc) {
            ecc = level[w];
            last_begin = count;
          }
          queue[count++] = w;
        }
      }
    }
    return ecc;
  };
  for (int start = 0; start < n; ++start) {
    if (placed[start]) continue;
    int last_begin, count;
    int root = start;
    int ecc = bfs(root, last_begin, count);
    // start from the minimum-degree vertex of the component
    for (int i = 0; i < count; ++i)
      if (deg[queue[i]] < deg[root] || (deg[queue[i]] == deg[root] && queue[i] < root)) root = queue[i];
    ecc = bfs(root, last_begin, count);
    for (int rep = 0; rep < 8; ++rep) {
      int cand = queue[last_begin];
      for (int i = last_begin; i < count; ++i)
        if (deg[queue[i]] < deg[cand] || (deg[queue[i]] == deg[cand] && queue[i] < cand)) cand = queue[i];
      int lb2, c2;
      const int e2 = bfs(cand, lb2, c2);
      if (e2 <= ecc) break;
      root = cand;
      ecc = e2;
      last_begin = lb2;
      count = c2;
    }
    // Cuthill-McKee from root: neighbours by increasing degree, then index
    size_t head = order.size();
    order.push_back(root);
    placed[root] = 1;
    while (head < order.size()) {
      const int v = order[head++];
      nb.clear();
      for (int e = ptr[v]; e < ptr[v + 1]; ++e)
        if (!placed[adj[e]]) nb.push_back(adj[e]);
      std::sort(nb.begin(), nb.end(), [&](int a, int b) { return deg[a] != deg[b] ? deg[a] < deg[b] : a < b; });
      for (int w : nb) {
        placed[w] = 1;
        order.push_back(w);
      }
    }
  }
  std::reverse(order.begin(), order.end());
}

static bool finite_all(const std::vector<double>& v) {
  for (double d : v)
    if (!std::isfinite(d)) return false;
  return true;
}

}  // namespace mfs

using namespace mfs;

namespace mfs {

namespace {
// Tiles per system: the partial-result stride of a character of these sizes.
int64_t partial_tiles(int64_t n, int64_t m, int64_t nnzb) {
  const int64_t ntv = (n + kVTile - 1) / kVTile, ntt = (m + kTTile - 1) / kTTile, nts = (nnzb + kSTile - 1) / kSTile;
  return std::max(ntv, std::max(ntt, nts));
}

// Byte sizes of the workspace pieces, in carving order.
int workspace_pieces(int64_t n, int64_t m_, int64_t nnzb, size_t* sz) {
  const size_t n3 = 3 * sizeof(double) * (size_t)n;
  const size_t m = (size_t)m_;
  int k = 0;
  sz[k++] = 90 * sizeof(double) * m;                          // blk
  sz[k++] = 12 * sizeof(double) * m;                          // frc
  sz[k++] = n3;                                               // b
  sz[k++] = n3;                                               // dx
  sz[k++] = (size_t)kBlockRecBytes * (size_t)nnzb;              // vals (block records, either precision)
  sz[k++] = 6 * sizeof(double) * (size_t)n;                   // minv
  for (int v = 0; v < 10; ++v) sz[k++] = n3;                  // r z p0 p1 q xc v0 v1 v2 v3
  sz[k++] = sizeof(double) * P_COUNT * (size_t)partial_tiles(n, m_, nnzb);  // part
  sz[k++] = sizeof(double) * P_COUNT;                         // red
  return k;
}
constexpr size_t kWsAlign = 256;
size_t align_up(size_t v) { return (v + kWsAlign - 1) / kWsAlign * kWsAlign; }
}  // namespace

size_t workspace_bytes_of(int64_t n, int64_t m, int64_t nnzb) {
  size_t sz[24];
  const int k = workspace_pieces(n, m, nnzb, sz);
  size_t total = 0;
  for (int i = 0; i < k; ++i) total += align_up(sz[i]);
  return total;
}

// Every resident device buffer of mfs_character_create, by its exact size.
// Per tet: tets 16, G 72, W mu 8, W lambda 8, info 4, tet order 4, s 48 and
// the 16 slot contributions 64 bytes.  Per vertex: X 24, diagonal slot 4,
// vertex order 4, x 24 and its backup 24, plus row pointers and pin pointers
// (4 per vertex and one more each).  Per block: column index 4 and slot
// pointer 4 (one more).  Per pin: its handle 4.  And the pose tables for the
// largest handle count.
size_t resident_bytes_of(int64_t n_, int64_t m_, int64_t nnzb_, int64_t np_) {
  const size_t n = (size_t)n_, m = (size_t)m_, nnzb = (size_t)nnzb_, np = (size_t)np_;
  return m * (16 + 72 + 8 + 8 + 4 + 4 + 48 + 64) + n * (24 + 4 + 4 + 24 + 24) + 4 * (n + 1) * 2 +
         4 * nnzb + 4 * (nnzb + 1) + 4 * np + (9 + 3) * sizeof(double) * kMaxHandles;
}

size_t workspace_layout(const mfs_character* ch) { return workspace_bytes_of(ch->n, ch->m, ch->nnzb); }

void bind_workspace(const mfs_character* ch, char* base, SysDesc* d) {
  size_t sz[24];
  const int k = workspace_pieces(ch->n, ch->m, ch->nnzb, sz);
  void* ptr[24];
  size_t off = 0;
  for (int i = 0; i < k; ++i) {
    ptr[i] = base ? base + off : nullptr;
    off += align_up(sz[i]);
  }
  d->blk = ptr[0];
  d->frc = static_cast<double*>(ptr[1]);
  d->b = static_cast<double*>(ptr[2]);
  d->dx = static_cast<double*>(ptr[3]);
  d->vals = ptr[4];
  d->minv = ptr[5];
  d->r = ptr[6];
  d->z = ptr[7];
  d->p0 = ptr[8];
  d->p1 = ptr[9];
  d->q = ptr[10];
  d->xc = ptr[11];
  d->v0 = ptr[12];
  d->v1 = ptr[13];
  d->v2 = ptr[14];
  d->v3 = ptr[15];
  d->part = static_cast<double*>(ptr[16]);
  d->red = static_cast<double*>(ptr[17]);
}

int ensure_workspace(mfs_character* ch) {
  if (ch->ws.p) return MFS_OK;
  MFS_HIP(hipSetDevice(ch->ctx->device));
  MFS_TRY(ch->ws.alloc(ch->workspace_bytes));
  bind_workspace(ch, ch->ws.as<char>(), &ch->desc);
  return MFS_OK;
}

}  // namespace mfs

extern "C" int mfs_character_create(mfs_context* ctx, const mfs_mesh_desc* d, mfs_character** out) {
  clear_error();
  if (!out) return set_error(MFS_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!ctx || !d) return set_error(MFS_E_INVALID, "null context or descriptor");
  if (d->n_vertices < 4 || d->n_vertices > (1LL << 30)) return set_error(MFS_E_INVALID, "n_vertices out of range");
  if (d->n_tets < 1 || d->n_tets > (1LL << 27)) return set_error(MFS_E_INVALID, "n_tets out of range");
  if (d->n_handles < 1 || d->n_handles > kMaxHandles)
    return set_error(MFS_E_INVALID, "n_handles must be in [1, %d]", kMaxHandles);
  if (d->n_pins < 1 || d->n_pins > (1LL << 30)) return set_error(MFS_E_INVALID, "n_pins out of range");
  if (!(d->pin_stiffness > 0.0) || !std::isfinite(d->pin_stiffness))
    return set_error(MFS_E_INVALID, "pin_stiffness must be finite and > 0");
  MFS_HIP(hipSetDevice(ctx->device));
  const int n = (int)d->n_vertices, m = (int)d->n_tets, nh = d->n_handles, np = (int)d->n_pins;
  const int mem = d->memory_space;

  std::vector<double> X, E, nu;
  std::vector<int32_t> T, model, cluster, pv, ph;
  MFS_TRY(fetch(d->rest_positions, 3 * (size_t)n, mem, X));
  MFS_TRY(fetch(d->tets, 4 * (size_t)m, mem, T));
  MFS_TRY(fetch(d->material_model, (size_t)m, mem, model));
  MFS_TRY(fetch(d->youngs, (size_t)m, mem, E));
  MFS_TRY(fetch(d->poisson, (size_t)m, mem, nu));
  MFS_TRY(fetch(d->tet_cluster, (size_t)m, mem, cluster));
  MFS_TRY(fetch(d->pin_vertex, (size_t)np, mem, pv));
  MFS_TRY(fetch(d->pin_handle, (size_t)np, mem, ph));

  // ---- validation ----
  if (!finite_all(X)) return set_error(MFS_E_INVALID, "non-finite rest position");
  std::vector<char> used(n, 0);
  for (int k = 0; k < m; ++k) {
    const int32_t* t = &T[4 * (size_t)k];
    for (int a = 0; a < 4; ++a) {
      if (t[a] < 0 || t[a] >= n) return set_error(MFS_E_INVALID, "tet %d: vertex index %d out of range", k, t[a]);
      used[t[a]] = 1;
      for (int b = 0; b < a; ++b)
        if (t[a] == t[b]) return set_error(MFS_E_INVALID, "tet %d repeats vertex %d", k, t[a]);
    }
    if (model[k] < MFS_ARAP || model[k] > MFS_NEOHOOKEAN)
      return set_error(MFS_E_INVALID, "tet %d: unknown material model %d", k, model[k]);
    if (!(E[k] > 0.0) || !std::isfinite(E[k])) return set_error(MFS_E_INVALID, "tet %d: Young's modulus must be > 0", k);
    if (!(nu[k] > -1.0 && nu[k] < 0.5)) return set_error(MFS_E_INVALID, "tet %d: Poisson ratio outside (-1, 0.5)", k);
    if (cluster[k] < 0 || cluster[k] >= nh) return set_error(MFS_E_INVALID, "tet %d: cluster %d out of range", k, cluster[k]);
  }
  for (int v = 0; v < n; ++v)
    if (!used[v]) return set_error(MFS_E_INVALID, "vertex %d belongs to no tet", v);
  for (int p = 0; p < np; ++p) {
    if (pv[p] < 0 || pv[p] >= n) return set_error(MFS_E_INVALID, "pin %d: vertex out of range", p);
    if (ph[p] < 0 || ph[p] >= nh) return set_error(MFS_E_INVALID, "pin %d: handle out of range", p);
  }

  auto ch = new mfs_character();
  std::unique_ptr<mfs_character> guard(ch);
  ch->ctx = ctx;
  ch->n = n;
  ch->m = m;
  ch->nh = nh;
  ch->npin = np;
  ch->ks = d->pin_stiffness;

  // ---- vertex adjacency and reverse Cuthill-McKee order ----
  std::vector<int64_t> keys;
  keys.reserve(12 * (size_t)m);
  for (int k = 0; k < m; ++k)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        if (a != b) keys.push_back((int64_t)T[4 * (size_t)k + a] * n + T[4 * (size_t)k + b]);
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  std::vector<int32_t> aptr(n + 1, 0), adj(keys.size());
  for (size_t i = 0; i < keys.size(); ++i) {
    aptr[keys[i] / n + 1]++;
    adj[i] = (int32_t)(keys[i] % n);
  }
  for (int v = 0; v < n; ++v) aptr[v + 1] += aptr[v];
  rcm_order(n, aptr, adj, ch->perm);
  std::vector<int32_t> iperm(n);
  for (int i = 0; i < n; ++i) iperm[ch->perm[i]] = i;

  // mean rest edge length (degeneracy tolerance) and bounding box
  double lsum = 0.0;
  size_t ecount = 0;
  for (size_t i = 0; i < keys.size(); ++i) {
    const int64_t r = keys[i] / n, c = keys[i] % n;
    if (r < c) {
      double e2 = 0.0;
      for (int j = 0; j < 3; ++j) {
        const double dd = X[3 * r + j] - X[3 * c + j];
        e2 += dd * dd;
      }
      lsum += std::sqrt(e2);
      ++ecount;
    }
  }
  ch->lbar = lsum / (double)ecount;
  {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int v = 0; v < n; ++v)
      for (int j = 0; j < 3; ++j) {
        lo[j] = std::min(lo[j], X[3 * (size_t)v + j]);
        hi[j] = std::max(hi[j], X[3 * (size_t)v + j]);
      }
    ch->bbox_diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                              (hi[2] - lo[2]) * (hi[2] - lo[2]));
  }

  // ---- rigid-motion check: >= 3 non-collinear pinned vertices ----
  {
    const double* p0 = &X[3 * (size_t)pv[0]];
    double best = 0.0;
    int far = pv[0];
    for (int p = 0; p < np; ++p) {
      const double* q = &X[3 * (size_t)pv[p]];
      const double dd = (q[0] - p0[0]) * (q[0] - p0[0]) + (q[1] - p0[1]) * (q[1] - p0[1]) + (q[2] - p0[2]) * (q[2] - p0[2]);
      if (dd > best) {
        best = dd;
        far = pv[p];
      }
    }
    const double* p1 = &X[3 * (size_t)far];
    double u[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
    double area = 0.0;
    for (int p = 0; p < np; ++p) {
      const double* q = &X[3 * (size_t)pv[p]];
      const double w[3] = {q[0] - p0[0], q[1] - p0[1], q[2] - p0[2]};
      const double c[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
      area = std::max(area, std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]));
    }
    if (!(best > 0.0) || !(area > 1e-9 * best))
      return set_error(MFS_E_SINGULAR, "pins cannot fix rigid motion: fewer than 3 non-collinear pinned vertices");
  }

  // ---- tets in the new vertex order, sorted by their smallest vertex ----
  std::vector<int32_t> Tn(4 * (size_t)m), tmin(m);
  for (int k = 0; k < m; ++k) {
    int mn = n;
    for (int a = 0; a < 4; ++a) {
      Tn[4 * (size_t)k + a] = iperm[T[4 * (size_t)k + a]];
      mn = std::min(mn, Tn[4 * (size_t)k + a]);
    }
    tmin[k] = mn;
  }
  ch->tperm.resize(m);
  std::iota(ch->tperm.begin(), ch->tperm.end(), 0);
  std::stable_sort(ch->tperm.begin(), ch->tperm.end(), [&](int a, int b) { return tmin[a] < tmin[b]; });
  std::vector<int32_t> Ts(4 * (size_t)m), info(m);
  std::vector<double> Es(m), nus(m);
  for (int k = 0; k < m; ++k) {
    const int o = ch->tperm[k];
    for (int a = 0; a < 4; ++a) Ts[4 * (size_t)k + a] = Tn[4 * (size_t)o + a];
    info[k] = cluster[o] | (model[o] << 16);
    Es[k] = E[o];
    nus[k] = nu[o];
  }

  // ---- block pattern (both triangles) and assembly map ----
  std::vector<int32_t> rowptr(n + 1, 0), colidx;
  {
    std::vector<int64_t> bk;
    bk.reserve(16 * (size_t)m);
    for (int k = 0; k < m; ++k)
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) bk.push_back((int64_t)Ts[4 * (size_t)k + a] * n + Ts[4 * (size_t)k + b]);
    std::sort(bk.begin(), bk.end());
    bk.erase(std::unique(bk.begin(), bk.end()), bk.end());
    colidx.resize(bk.size());
    for (size_t i = 0; i < bk.size(); ++i) {
      rowptr[bk[i] / n + 1]++;
      colidx[i] = (int32_t)(bk[i] % n);
    }
    for (int v = 0; v < n; ++v) rowptr[v + 1] += rowptr[v];
  }
  const int nnzb = (int)colidx.size();
  ch->nnzb = nnzb;
  auto find_slot = [&](int r, int c) {
    const int32_t* lo = colidx.data() + rowptr[r];
    const int32_t* hi = colidx.data() + rowptr[r + 1];
    return (int)(std::lower_bound(lo, hi, c) - colidx.data());
  };
  std::vector<int32_t> slot_of(16 * (size_t)m), slot_ptr(nnzb + 1, 0), contrib(16 * (size_t)m), diag(n);
  for (int k = 0; k < m; ++k)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        const int sl = find_slot(Ts[4 * (size_t)k + a], Ts[4 * (size_t)k + b]);
        slot_of[16 * (size_t)k + 4 * a + b] = sl;
        slot_ptr[sl + 1]++;
      }
  for (int i = 0; i < nnzb; ++i) slot_ptr[i + 1] += slot_ptr[i];
  {
    std::vector<int32_t> fill(slot_ptr.begin(), slot_ptr.end() - 1);
    for (int k = 0; k < m; ++k)
      for (int ab = 0; ab < 16; ++ab) contrib[fill[slot_of[16 * (size_t)k + ab]]++] = (k << 4) | ab;
  }
  for (int r = 0; r < n; ++r) diag[r] = find_slot(r, r);

  // ---- pins grouped by (new) vertex ----
  std::vector<int32_t> pin_order(np), vpin_ptr(n + 1, 0), vpin_h(np);
  std::iota(pin_order.begin(), pin_order.end(), 0);
  std::stable_sort(pin_order.begin(), pin_order.end(), [&](int a, int b) { return iperm[pv[a]] < iperm[pv[b]]; });
  for (int i = 0; i < np; ++i) {
    vpin_ptr[iperm[pv[pin_order[i]]] + 1]++;
    vpin_h[i] = ph[pin_order[i]];
  }
  for (int v = 0; v < n; ++v) vpin_ptr[v + 1] += vpin_ptr[v];

  std::vector<double> Xn(3 * (size_t)n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < 3; ++j) Xn[3 * (size_t)i + j] = X[3 * (size_t)ch->perm[i] + j];

  // ---- upload resident data ----
  MFS_TRY(upload(ch->tets, Ts.data(), 4 * (size_t)m));
  MFS_TRY(upload(ch->info, info.data(), (size_t)m));
  MFS_TRY(upload(ch->X, Xn.data(), 3 * (size_t)n));
  MFS_TRY(upload(ch->rowptr, rowptr.data(), (size_t)n + 1));
  ch->max_tile_blocks = 0;
  for (int b = 0; b < n; b += kVTile)
    ch->max_tile_blocks = std::max(ch->max_tile_blocks, rowptr[std::min(n, b + kVTile)] - rowptr[b]);
  MFS_TRY(upload(ch->colidx, colidx.data(), (size_t)nnzb));
  MFS_TRY(upload(ch->slot_ptr, slot_ptr.data(), (size_t)nnzb + 1));
  MFS_TRY(upload(ch->contrib, contrib.data(), 16 * (size_t)m));
  MFS_TRY(upload(ch->diag, diag.data(), (size_t)n));
  MFS_TRY(upload(ch->vpin_ptr, vpin_ptr.data(), (size_t)n + 1));
  MFS_TRY(upload(ch->vpin_h, vpin_h.data(), (size_t)np));
  MFS_TRY(upload(ch->perm_d, ch->perm.data(), (size_t)n));
  MFS_TRY(upload(ch->tperm_d, ch->tperm.data(), (size_t)m));
  MFS_TRY(ch->G.alloc(9 * sizeof(double) * (size_t)m));
  MFS_TRY(ch->wmu.alloc(sizeof(double) * (size_t)m));
  MFS_TRY(ch->wlam.alloc(sizeof(double) * (size_t)m));
  {
    DevBuf dE, dnu, dbad;
    MFS_TRY(upload(dE, Es.data(), (size_t)m));
    MFS_TRY(upload(dnu, nus.data(), (size_t)m));
    MFS_TRY(dbad.alloc((size_t)m));
    const double tol = 1e-12 * ch->lbar * ch->lbar * ch->lbar;
    launch_rest(ctx->stream, ch->tets.as<int4>(), ch->X.as<double>(), dE.as<double>(), dnu.as<double>(), m, tol,
                ch->G.as<double>(), ch->wmu.as<double>(), ch->wlam.as<double>(), dbad.as<uint8_t>());
    MFS_HIP(hipGetLastError());
    std::vector<uint8_t> bad(m);
    MFS_HIP(hipMemcpyAsync(bad.data(), dbad.p, (size_t)m, hipMemcpyDeviceToHost, ctx->stream));
    MFS_HIP(hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < m; ++k)
      if (bad[k])
        return set_error(MFS_E_DEGENERATE, "tet %d is degenerate (|det Dm| <= 1e-12 * mean_edge^3)", ch->tperm[k]);
  }

  // ---- per-frame and solver state ----
  ch->ntv = (n + kVTile - 1) / kVTile;
  ch->ntt = (m + kTTile - 1) / kTTile;
  ch->nts = (nnzb + kSTile - 1) / kSTile;
  ch->ptile = std::max(ch->ntv, std::max(ch->ntt, ch->nts));
  const size_t n3 = 3 * (size_t)n * sizeof(double);
  MFS_TRY(ch->Rh.alloc(9 * sizeof(double) * kMaxHandles));
  MFS_TRY(ch->th.alloc(3 * sizeof(double) * kMaxHandles));
  MFS_TRY(ch->x.alloc(n3));
  MFS_TRY(ch->xb.alloc(n3));
  MFS_TRY(ch->s.alloc(6 * sizeof(double) * (size_t)m));
  ch->workspace_bytes = workspace_layout(ch);
  MFS_TRY(ch->ws.alloc(ch->workspace_bytes));
  MFS_HIP(hipMemcpyAsync(ch->x.p, ch->X.p, n3, hipMemcpyDeviceToDevice, ctx->stream));
  MFS_HIP(hipStreamSynchronize(ctx->stream));

  SysDesc& s = ch->desc;
  std::memset(&s, 0, sizeof s);
  s.n = n;
  s.m = m;
  s.nnzb = nnzb;
  s.nh = nh;
  s.ntv = ch->ntv;
  s.ntt = ch->ntt;
  s.nts = ch->nts;
  s.ptile = ch->ptile;
  s.ticket = ch->ntv > kAllReadTiles ? 1 : 0;
  s.ks = ch->ks;
  s.tets = ch->tets.as<int4>();
  s.G = ch->G.as<double>();
  s.wmu = ch->wmu.as<double>();
  s.wlam = ch->wlam.as<double>();
  s.info = ch->info.as<int32_t>();
  s.X = ch->X.as<double>();
  s.rowptr = ch->rowptr.as<int32_t>();
  s.colidx = ch->colidx.as<int32_t>();
  s.slot_ptr = ch->slot_ptr.as<int32_t>();
  s.contrib = ch->contrib.as<int32_t>();
  s.diag = ch->diag.as<int32_t>();
  s.vpin_ptr = ch->vpin_ptr.as<int32_t>();
  s.vpin_h = ch->vpin_h.as<int32_t>();
  s.Rh = ch->Rh.as<double>();
  s.th = ch->th.as<double>();
  s.x = ch->x.as<double>();
  s.s = ch->s.as<double>();
  bind_workspace(ch, ch->ws.as<char>(), &s);

  // the sizes actually allocated (mfs_character_footprint predicts them from
  // a descriptor with resident_bytes_of)
  ch->resident_bytes = ch->tets.bytes + ch->G.bytes + ch->wmu.bytes + ch->wlam.bytes + ch->info.bytes + ch->X.bytes +
                       ch->rowptr.bytes + ch->colidx.bytes + ch->slot_ptr.bytes + ch->contrib.bytes +
                       ch->diag.bytes + ch->vpin_ptr.bytes + ch->vpin_h.bytes + ch->perm_d.bytes +
                       ch->tperm_d.bytes + ch->x.bytes + ch->xb.bytes + ch->s.bytes + ch->Rh.bytes + ch->th.bytes;
  *out = guard.release();
  return MFS_OK;
}

extern "C" int mfs_character_destroy(mfs_character* ch) {
  if (!ch) return MFS_OK;
  if (ch->ctx) (void)hipSetDevice(ch->ctx->device);
  delete ch;
  return MFS_OK;
}

extern "C" int mfs_character_set_forces(mfs_character* ch, const int32_t* vertices, const double* forces,
                                        int64_t count, int32_t memory_space) {
  clear_error();
  if (!ch) return set_error(MFS_E_INVALID, "null character");
  if (count < 0) return set_error(MFS_E_INVALID, "negative force count");
  if (memory_space != MFS_MEM_HOST && memory_space != MFS_MEM_DEVICE)
    return set_error(MFS_E_INVALID, "invalid memory space");
  mfs_context* ctx = ch->ctx;
  MFS_HIP(hipSetDevice(ctx->device));
  MFS_HIP(hipStreamSynchronize(ctx->stream));  // no solve is reading the old forces
  if (count == 0) {
    ch->desc.fext = nullptr;
    return MFS_OK;
  }
  if (!vertices || !forces) return set_error(MFS_E_INVALID, "null vertices or forces");
  std::vector<int32_t> hv(count);
  std::vector<double> hf(3 * (size_t)count);
  if (memory_space == MFS_MEM_DEVICE) {
    MFS_HIP(hipMemcpy(hv.data(), vertices, sizeof(int32_t) * count, hipMemcpyDeviceToHost));
    MFS_HIP(hipMemcpy(hf.data(), forces, sizeof(double) * 3 * count, hipMemcpyDeviceToHost));
  } else {
    std::memcpy(hv.data(), vertices, sizeof(int32_t) * count);
    std::memcpy(hf.data(), forces, sizeof(double) * 3 * count);
  }
  std::vector<int32_t> inv(ch->n);
  for (int i = 0; i < ch->n; ++i) inv[ch->perm[i]] = i;
  std::vector<double> f(3 * (size_t)ch->n, 0.0);
  for (int64_t k = 0; k < count; ++k) {
    if (hv[k] < 0 || hv[k] >= ch->n) return set_error(MFS_E_INVALID, "force %lld: vertex %d out of range", (long long)k, hv[k]);
    for (int i = 0; i < 3; ++i) {
      const double v = hf[3 * k + i];
      if (!std::isfinite(v)) return set_error(MFS_E_INVALID, "force %lld is not finite", (long long)k);
      f[3 * (size_t)inv[hv[k]] + i] += v;  // repeated vertices add up
    }
  }
  if (!ch->fext.p) MFS_TRY(ch->fext.alloc(3 * sizeof(double) * (size_t)ch->n));
  MFS_HIP(hipMemcpy(ch->fext.p, f.data(), f.size() * sizeof(double), hipMemcpyHostToDevice));
  ch->desc.fext = ch->fext.as<double>();
  return MFS_OK;
}

extern "C" int mfs_character_set_rotation_blend(mfs_character* ch, int32_t kmax, const int32_t* handles,
                                                const double* weights, int32_t memory_space) {
  clear_error();
  if (!ch) return set_error(MFS_E_INVALID, "null character");
  if (memory_space != MFS_MEM_HOST && memory_space != MFS_MEM_DEVICE)
    return set_error(MFS_E_INVALID, "invalid memory space");
  mfs_context* ctx = ch->ctx;
  MFS_HIP(hipSetDevice(ctx->device));
  MFS_HIP(hipStreamSynchronize(ctx->stream));  // no solve is reading the old rotations
  if (!handles) {
    ch->blend_k = 0;
    ch->desc.Rt = nullptr;
    return MFS_OK;
  }
  if (kmax < 1 || kmax > 4) return set_error(MFS_E_INVALID, "kmax must be in 1..4");
  if (!weights) return set_error(MFS_E_INVALID, "null weights");
  const size_t mk = (size_t)ch->m * kmax;
  std::vector<int32_t> hh(mk);
  std::vector<double> hw(mk);
  if (memory_space == MFS_MEM_DEVICE) {
    MFS_HIP(hipMemcpy(hh.data(), handles, sizeof(int32_t) * mk, hipMemcpyDeviceToHost));
    MFS_HIP(hipMemcpy(hw.data(), weights, sizeof(double) * mk, hipMemcpyDeviceToHost));
  } else {
    std::memcpy(hh.data(), handles, sizeof(int32_t) * mk);
    std::memcpy(hw.data(), weights, sizeof(double) * mk);
  }
  // caller's tet order, row-major (m x kmax) -> internal order, kmax planes of m
  std::vector<int32_t> ph(mk);
  std::vector<double> pw(mk);
  for (int k = 0; k < ch->m; ++k) {
    const size_t src = (size_t)ch->tperm[k] * kmax;
    if (hh[src] < 0 || hh[src] >= ch->nh)
      return set_error(MFS_E_INVALID, "tet %d: first blend handle %d out of range", ch->tperm[k], hh[src]);
    for (int j = 0; j < kmax; ++j) {
      const int32_t h = hh[src + j];
      const double w = hw[src + j];
      if (h < -1 || h >= ch->nh) return set_error(MFS_E_INVALID, "tet %d: blend handle %d out of range", ch->tperm[k], h);
      if (!(w >= 0.0) || !std::isfinite(w))
        return set_error(MFS_E_INVALID, "tet %d: blend weight must be finite and >= 0", ch->tperm[k]);
      ph[(size_t)j * ch->m + k] = h;
      pw[(size_t)j * ch->m + k] = h >= 0 ? w : 0.0;
    }
  }
  MFS_TRY(ch->blend_h.alloc(sizeof(int32_t) * mk));
  MFS_TRY(ch->blend_w.alloc(sizeof(double) * mk));
  if (!ch->Rt.p) MFS_TRY(ch->Rt.alloc(9 * sizeof(double) * (size_t)ch->m));
  MFS_HIP(hipMemcpy(ch->blend_h.p, ph.data(), sizeof(int32_t) * mk, hipMemcpyHostToDevice));
  MFS_HIP(hipMemcpy(ch->blend_w.p, pw.data(), sizeof(double) * mk, hipMemcpyHostToDevice));
  ch->blend_k = kmax;
  ch->desc.Rt = ch->Rt.as<double>();
  return MFS_OK;
}

extern "C" int mfs_character_release_workspace(mfs_character* ch) {
  if (!ch) return set_error(MFS_E_INVALID, "null character");
  if (!ch->ws.p) return MFS_OK;
  MFS_HIP(hipSetDevice(ch->ctx->device));
  MFS_HIP(hipStreamSynchronize(ch->ctx->stream));
  ch->ws.release();
  bind_workspace(ch, nullptr, &ch->desc);
  return MFS_OK;
}

extern "C" int mfs_character_get_footprint(const mfs_character* ch, size_t* resident, size_t* workspace) {
  clear_error();
  if (!ch) return set_error(MFS_E_INVALID, "null character");
  if (resident) *resident = ch->resident_bytes;
  if (workspace) *workspace = ch->workspace_bytes;
  return MFS_OK;
}

// The byte counts of mfs_character_create for a mesh not yet uploaded: the
// block count of the condensed matrix is one diagonal block per vertex plus
// two per mesh edge (both triangles), the edges being the distinct vertex
// pairs of the tets.
extern "C" int mfs_character_footprint(const mfs_mesh_desc* d, size_t* resident, size_t* workspace) {
  clear_error();
  if (!d) return set_error(MFS_E_INVALID, "null descriptor");
  if (d->n_vertices < 4 || d->n_vertices > (1LL << 30)) return set_error(MFS_E_INVALID, "n_vertices out of range");
  if (d->n_tets < 1 || d->n_tets > (1LL << 27)) return set_error(MFS_E_INVALID, "n_tets out of range");
  if (d->n_pins < 1 || d->n_pins > (1LL << 30)) return set_error(MFS_E_INVALID, "n_pins out of range");
  if (!d->tets) return set_error(MFS_E_INVALID, "null tets");
  const int64_t n = d->n_vertices, m = d->n_tets;
  std::vector<int32_t> T;
  MFS_TRY(fetch(d->tets, 4 * (size_t)m, d->memory_space, T));
  std::vector<char> used((size_t)n, 0);
  std::vector<int64_t> edges;
  edges.reserve(6 * (size_t)m);
  for (int64_t k = 0; k < m; ++k) {
    const int32_t* t = &T[4 * (size_t)k];
    for (int a = 0; a < 4; ++a) {
      if (t[a] < 0 || t[a] >= n)
        return set_error(MFS_E_INVALID, "tet %lld: vertex index %d out of range", (long long)k, t[a]);
      used[t[a]] = 1;
      for (int b = 0; b < a; ++b) {
        if (t[a] == t[b]) return set_error(MFS_E_INVALID, "tet %lld repeats vertex %d", (long long)k, t[a]);
        const int64_t lo = std::min(t[a], t[b]), hi = std::max(t[a], t[b]);
        edges.push_back(lo * n + hi);
      }
    }
  }
  for (int64_t v = 0; v < n; ++v)
    if (!used[v]) return set_error(MFS_E_INVALID, "vertex %lld belongs to no tet", (long long)v);
  std::sort(edges.begin(), edges.end());
  const int64_t ne = std::unique(edges.begin(), edges.end()) - edges.begin();
  const int64_t nnzb = n + 2 * ne;
  if (resident) *resident = resident_bytes_of(n, m, nnzb, d->n_pins);
  if (workspace) *workspace = workspace_bytes_of(n, m, nnzb);
  return MFS_OK;
}
