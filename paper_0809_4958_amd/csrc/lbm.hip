// lbm.hip -- host side of the C ABI declared in include/lbm.h.
//
// A context owns two structure-of-arrays population arenas (all boxes back to
// back), the boundary histories, the chain state (double-buffered by step
// parity) and a work list of items (interior tiles and boundary chunks) for the
// fused kernel.  Per step it launches k_chain (when chains exist) and k_lb on
// the context stream; every per-step quantity (time index, buffer parity,
// check steps) is read on the device from DevState, so a chunk of steps can
// be captured once into a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "lbm.h"
#include "lb_io_kernels.hpp"
#include "lb_vort_kernels.hpp"
#include "lb_launch.hpp"

using namespace lbdev;

namespace {

constexpr int BND_CHUNK = 512;

struct BoxHost {
  lb_box dim;
  int64_t nn = 0, off = 0;
  int64_t interior = 0;
  int ox = 1, oy = 1, oz = 1;  // first interior coordinate per axis
  int ix = 0, iy = 0, iz = 0;  // interior extent per axis
  bool has_layer = false;
  bool has_bc = false;
  int bc_mode = -1, bc_dt = 1, bc_ns = 0, bc_res = 0;
  int64_t bc_t0 = 0;
  void* d_bc = nullptr;
  const void* ring = nullptr;  // LEARNED: caller-owned device ring (not freed here)
  int ex = 0, ey = 0, ez = 0;  // tile shape
  int n_rect = 0;
  int rect_face[MAX_RECT] = {};
  int rect_cnt[MAX_RECT] = {};
  int rect_start[MAX_RECT][3] = {};
  int rect_len[MAX_RECT][3] = {};
  int nbnd = 0;
  bool vec = false;  // interior rows as lane vectors (ITEM_ROWS), x-face nodes included
  int ylog = 0;      // log2 of the y lines interleaved per population row
  int xf_off = -1;   // row boxes: first float of the x-face velocities
  int vw = 0;        // row boxes: 32-bit words per lane vector
  // accelerated-frame body force: tracer acceleration samples on the device
  double* d_body = nullptr;
  int body_dt = 1, body_ns = 0;
  int64_t body_t0 = 0;
};

struct ChainHost {
  lb_chain p;
  int box;
  std::vector<double> pos, vel;
  bool pos_is_rel = false;  // pos holds positions minus the anchor (exact restore)
};

using lbhost::ChainLaunch;
using lbhost::LbLaunch;

template <int S>
void launch_read(bool per, int nblk, hipStream_t s, const BoxDesc& d, const void* src, double* out,
                 int what, int pre, double r0) {
  using T = typename Store<S>::T;
  if (per)
    hipLaunchKernelGGL((k_read<S, true>), dim3(nblk), dim3(WG), 0, s, d, (const T*)src, out, what, pre, r0);
  else
    hipLaunchKernelGGL((k_read<S, false>), dim3(nblk), dim3(WG), 0, s, d, (const T*)src, out, what, pre, r0);
}

template <int S>
void launch_sites(bool per, int nblk, hipStream_t s, const BoxDesc& d, const void* src,
                  const int* xyz, int n, double* out, int pre, double r0) {
  using T = typename Store<S>::T;
  if (per)
    hipLaunchKernelGGL((k_read_sites<S, true>), dim3(nblk), dim3(WG), 0, s, d, (const T*)src, xyz, n, out, pre, r0);
  else
    hipLaunchKernelGGL((k_read_sites<S, false>), dim3(nblk), dim3(WG), 0, s, d, (const T*)src, xyz, n, out, pre, r0);
}

using CheckLaunch = void (*)(int, hipStream_t, const LbArgs&);

template <int S, bool P>
void launch_check(int n, hipStream_t s, const LbArgs& a) {
  hipLaunchKernelGGL((k_check<S, P>), dim3(n), dim3(WG), 0, s, a);
}

template <int S>
CheckLaunch pick_check(bool per) {
  return per ? launch_check<S, true> : launch_check<S, false>;
}

// coll: 0 BGK, 1 MRT, 2 MRT with ghost relaxation rate 1 (ghost moments not formed)
template <int S>
LbLaunch pick_lb(int coll, bool per, bool ext, bool aa) {
  if (coll == 0) return lbhost::pick_lb<S, 0>(per, ext, aa);
  if (coll == 1) return lbhost::pick_lb<S, 1>(per, ext, aa);
  return lbhost::pick_lb<S, 2>(per, ext, aa);
}

template <int S>
LbLaunch pick_force(int coll, bool per, bool ext) {
  if (coll == 0) return lbhost::pick_force<S, 0>(per, ext);
  if (coll == 1) return lbhost::pick_force<S, 1>(per, ext);
  return lbhost::pick_force<S, 2>(per, ext);
}

size_t store_bytes(int s) { return s == LB_STORE_F64 ? 8 : (s == LB_STORE_F32 ? 4 : 2); }
// nodes per lane of the row items with w 32-bit words per lane
int row_nodes(int s, int w) { return w * 4 / (int)store_bytes(s); }

// Lane-vector width of a row box: prefer 2 words, then 3, among the widths
// whose lane groups per row divide a wavefront (or fill whole wavefronts) --
// groups of a row that straddle wavefronts need a halo load per wavefront
// edge; then any width that divides the row.  0 = no row path.
int pick_row_words(int storage, int nx) {
  int fallback = 0;
  for (int w : {2, 3}) {
    const int V = row_nodes(storage, w);
    if (nx % V != 0 || nx < 2 * V) continue;
    const int L = nx / V;
    if (64 % L == 0 || L % 64 == 0) return w;
    if (!fallback) fallback = w;
  }
  return fallback;
}

// Staging of the allocation-free site readout (lb_read_sites_noalloc): the
// site list (int32 [n][3]) followed, at a 256-byte boundary, by the output
// populations (FP64 [n][19]) of at most NOALLOC_SITES sites.  One copy per
// GPU the library runs on, held until the process ends.  In host code its
// name is not a device address: host code uses only the address that
// hipGetSymbolAddress returned for the current device (scratch_ptr below).
constexpr int NOALLOC_SITES = 32768;
constexpr size_t NOALLOC_XYZ_BYTES = ((size_t)3 * NOALLOC_SITES * sizeof(int) + 255) / 256 * 256;
constexpr size_t NOALLOC_BYTES = NOALLOC_XYZ_BYTES + (size_t)Q * NOALLOC_SITES * sizeof(double);
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// device address of `scratch` per device, looked up once per device by lb_init
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_dev[MAX_DEVICES] = {};

// Looks up (once per device, with that device current) the device address of
// the staging array; nullptr if the lookup fails.
void* scratch_ptr(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    scratch_dev[dev] = p;
  }
  return scratch_dev[dev];
}

}  // namespace

struct lb_ctx {
  lb_config cfg{};
  std::vector<BoxHost> bx;
  std::vector<ChainHost> ch;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  int S = 0, coll = 0;
  bool per = false;
  int fp16_exp = 14;
  int dev = 0;                    // device current at lb_init
  void* noalloc = nullptr;        // that device's address of the static staging array
  bool aa = false;                // in-place streaming on one population buffer
  double kT = 0.0;                // thermal fluctuations (lb_set_thermal)
  uint64_t seed = 0;              // their Philox key
  void* arena[2] = {nullptr, nullptr};
  int64_t arena_elems = 0;
  // device tables
  BoxDesc* d_boxes = nullptr;
  Item* d_items = nullptr;
  int* d_order = nullptr;
  int4* d_check_items = nullptr;   // k_check workgroups: box, first plane, end plane
  int* d_check_off = nullptr;      // [n_boxes + 1]
  double* d_partials = nullptr;    // [n_check][4]
  int n_check = 0;
  double* d_mass_mom = nullptr;
  float* d_xface = nullptr;        // x-face velocities of the row boxes (k_xface)
  int4* d_xf_items = nullptr;      // x-face work items (one wavefront each): box, first node, count
  int n_xf_items = 0;
  DevState* d_st = nullptr;
  ChainDesc* d_chains = nullptr;
  void* d_pos = nullptr;
  void* d_vel = nullptr;
  int4* d_rec_base = nullptr;
  void* d_rec_d = nullptr;
  void* d_rec_dp = nullptr;
  int* d_bbox = nullptr;
  int total_beads = 0;
  int n_items = 0, n_entries = 0, grid = 0;
  std::vector<Item> items;
  std::vector<BoxDesc> h_boxes;
  bool tables_ready = false;
  bool chains_ready = false;
  bool state_pre = true;
  int64_t host_step = 0;
  lb_status latched = LB_OK;
  hipGraphExec_t gexec = nullptr;
  int gsteps = 0;
  int gphase = -1;  // check phase the graphs were captured for (-1: checks decided on the device)
  // timed graphs: two instances with their own event-record nodes, replayed
  // alternately so the host reads one chunk's events while the next runs
  hipGraphExec_t gexec_t[2] = {nullptr, nullptr};
  long long* d_stamps = nullptr;     // [2][3 * gsteps_t] device timestamps
  long long* h_stamps = nullptr;     // pinned copy
  hipEvent_t stamp_ev[2] = {nullptr, nullptr};
  double clock_khz = 0;
  int gsteps_t = 0;
  LbLaunch lb_fn = nullptr;
  LbLaunch force_fn = nullptr;
  ChainLaunch chain_fn = nullptr;
  CheckLaunch check_fn = nullptr;
  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev;
  int ev_used = 0;
  int t_steps = 0;
  // event times accumulated from timed graph chunks
  double acc_lb = 0, acc_ch = 0, acc_step = 0;
  int acc_n = 0, acc_step_n = 0;
  std::string err, desc;
  std::vector<void*> owned;
};

namespace {

lb_status fail(lb_ctx* c, lb_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

#define HIPCHK(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, LB_ERR_HIP, std::string(#call " failed: ") + hipGetErrorString(e_)); \
  } while (0)

void* dalloc(lb_ctx* ctx, size_t bytes) {
  if (bytes == 0) bytes = 8;
  void* p = nullptr;
  if (ctx->cfg.dev_alloc) {
    p = ctx->cfg.dev_alloc(bytes, ctx->cfg.alloc_user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  return p;
}

void dfree(lb_ctx* ctx, void* p) {
  if (!p) return;
  if (ctx->cfg.dev_free)
    ctx->cfg.dev_free(p, ctx->cfg.alloc_user);
  else
    (void)hipFree(p);
}

// All initialisation is ordered on the context stream: null-stream memsets and
// copies do not order against a non-blocking stream.
hipError_t h2d(lb_ctx* ctx, void* dst, const void* src, size_t bytes) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(ctx->stream);
}

hipError_t copy_sync(lb_ctx* ctx, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, ctx->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(ctx->stream);
}

hipError_t dzero(lb_ctx* ctx, void* dst, size_t bytes) {
  return hipMemsetAsync(dst, 0, bytes, ctx->stream);
}

template <typename X>
X* dalloc_t(lb_ctx* ctx, size_t n, bool* ok) {
  X* p = (X*)dalloc(ctx, n * sizeof(X));
  if (!p) *ok = false;
  return p;
}

void drop_graph(lb_ctx* ctx) {
  if (ctx->gexec) {
    (void)hipGraphExecDestroy(ctx->gexec);
    ctx->gexec = nullptr;
  }
  for (int x = 0; x < 2; x++)
    if (ctx->gexec_t[x]) {
      (void)hipGraphExecDestroy(ctx->gexec_t[x]);
      ctx->gexec_t[x] = nullptr;
    }
}

void drop_stamps(lb_ctx* ctx) {
  if (ctx->d_stamps) dfree(ctx, ctx->d_stamps);
  if (ctx->h_stamps) (void)hipHostFree(ctx->h_stamps);
  for (auto& e : ctx->stamp_ev)
    if (e) (void)hipEventDestroy(e);
  ctx->d_stamps = nullptr;
  ctx->h_stamps = nullptr;
  ctx->stamp_ev[0] = ctx->stamp_ev[1] = nullptr;
}

// Default tile: whole interior rows in x (coalesced, one box row per wave
// segment), about 512 (x, y) positions per workgroup (two per thread) and a
// deep z march so that the z+-1 planes a node pulls from are re-read from
// cache by the same thread; y halo overhead (ey+2)/ey, z halo (ez+2)/ez.
void default_tile(BoxHost& b) {
  const int ix = b.ix;
  b.ex = ix <= 128 ? ix : 64;
  b.ey = std::max(1, std::min(b.iy, 512 / std::max(1, b.ex)));
  while (b.ex * b.ey > WG * MAX_SLOTS) b.ey--;
  // tiles: planes per item; row boxes: workgroup iterations per item (short
  // items keep the tail of a launch short)
  b.ez = b.vec ? 4 : std::min(b.iz, 16);
}

std::string box_key(const lb_ctx* ctx, const BoxHost& b) {
  std::ostringstream s;
  s << "S" << ctx->S << "C" << ctx->coll << "_" << b.dim.nx << "x" << b.dim.ny << "x" << b.dim.nz
    << "p" << b.dim.periodic_mask;
  return s.str();
}

// key of a whole context's launch grid: its box-size classes and their counts
std::string grid_key(lb_ctx* ctx) {
  std::map<std::string, int> cnt;
  for (auto& b : ctx->bx) cnt[box_key(ctx, b)]++;
  std::ostringstream s;
  s << "grid";
  for (auto& kv : cnt) s << "_" << kv.first << "n" << kv.second;
  return s.str();
}

void load_tune_cache(lb_ctx* ctx) {
  if (!ctx->cfg.tune_cache) return;
  std::ifstream in(ctx->cfg.tune_cache);
  if (!in) return;
  std::map<std::string, std::vector<int>> entries;
  std::string line;
  while (std::getline(in, line)) {
    // {"key": "...", "ex": a, "ey": b, "ez": c}
    auto kp = line.find("\"key\"");
    if (kp == std::string::npos) continue;
    auto q1 = line.find('"', line.find(':', kp) + 1);
    auto q2 = line.find('"', q1 + 1);
    if (q1 == std::string::npos || q2 == std::string::npos) continue;
    std::string key = line.substr(q1 + 1, q2 - q1 - 1);
    auto num = [&](const char* name) {
      auto p = line.find(std::string("\"") + name + "\"");
      if (p == std::string::npos) return -1;
      return atoi(line.c_str() + line.find(':', p) + 1);
    };
    entries[key] = {num("ex"), num("ey"), num("ez"), num("grid"), num("vw")};
  }
  auto g = entries.find(grid_key(ctx));
  if (g != entries.end() && g->second[3] >= 8) ctx->grid = g->second[3];
  for (auto& b : ctx->bx) {
    auto it = entries.find(box_key(ctx, b));
    if (it == entries.end()) continue;
    const auto& v = it->second;
    if (v[0] >= 1 && v[1] >= 1 && v[2] >= 1 && v[0] <= b.ix && v[1] <= b.iy && v[2] <= b.iz &&
        v[0] * v[1] <= WG * MAX_SLOTS) {
      b.ex = v[0];
      b.ey = v[1];
      b.ez = v[2];
    }
    if (b.vec && (v[4] == 2 || v[4] == 3)) {
      const int V = row_nodes(ctx->S, v[4]);
      if (b.dim.nx % V == 0 && b.dim.nx >= 2 * V) b.vw = v[4];
    }
  }
}

void free_tables(lb_ctx* ctx) {
  dfree(ctx, ctx->d_items);
  dfree(ctx, ctx->d_order);
  dfree(ctx, ctx->d_check_items);
  dfree(ctx, ctx->d_check_off);
  dfree(ctx, ctx->d_partials);
  ctx->d_items = nullptr;
  ctx->d_order = nullptr;
  ctx->d_check_items = nullptr;
  ctx->d_check_off = nullptr;
  ctx->d_partials = nullptr;
  ctx->tables_ready = false;
  drop_graph(ctx);
}

// Work list: items numbered box by box (box order), so each box owns a
// contiguous item range (fixed-order reduction); the launch order places boxes
// largest first and cuts the sequence into 8 contiguous pieces of equal work,
// one per XCD (workgroup w runs on XCD w % 8), so tiles that share halo rows
// share an L2.
lb_status build_tables(lb_ctx* ctx, int grid_override) {
  free_tables(ctx);
  std::vector<Item> items;
  std::vector<int> box_off(ctx->bx.size() + 1, 0);
  std::vector<double> work;
  for (size_t bi = 0; bi < ctx->bx.size(); bi++) {
    BoxHost& b = ctx->bx[bi];
    box_off[bi] = (int)items.size();
    for (int k = 0; k < b.nbnd; k += BND_CHUNK) {
      Item it{};
      it.box = (int)bi;
      it.kind = ITEM_BOUNDARY;
      it.x0 = k;
      it.ex = std::min(BND_CHUNK, b.nbnd - k);
      items.push_back(it);
      work.push_back(0.25 * it.ex);
    }
    if (b.vec) {
      // interior rows cut into lane groups of V nodes, numbered row by row
      // (y fastest, then z); an item is b.ez workgroup iterations of WG groups
      const int V = row_nodes(ctx->S, b.vw);
      const int L = b.dim.nx / V, nyi = b.dim.ny - 2;
      const int64_t groups = (int64_t)L * nyi * (b.dim.nz - 2);
      const int64_t per = (int64_t)WG * std::max(1, b.ez);
      for (int64_t g0 = 0; g0 < groups; g0 += per) {
        const int64_t g1 = std::min(groups, g0 + per);
        const int r0 = (int)(g0 / L), r1 = (int)((g1 - 1) / L);
        const int z0 = r0 / nyi, z1 = r1 / nyi;
        Item it{};
        it.box = (int)bi;
        it.kind = ITEM_ROWS;
        it.x0 = (int)g0;
        it.ex = (int)(g1 - g0);
        // bounding box of the item's rows (chain overlap test)
        it.z0 = 1 + z0;
        it.ez = z1 - z0 + 1;
        it.y0 = z0 == z1 ? 1 + (r0 - z0 * nyi) : 1;
        it.ey = z0 == z1 ? r1 - r0 + 1 : nyi;
        items.push_back(it);
        work.push_back((double)it.ex * V);
      }
      // face rows: planes z = 0 and nz-1, then rows y = 0 and ny-1 of each
      // interior plane
      const int64_t fgroups = (int64_t)L * (2 * b.dim.ny + 2 * (b.dim.nz - 2));
      const int64_t fper = (int64_t)WG * 4;
      for (int64_t g0 = 0; g0 < fgroups; g0 += fper) {
        Item it{};
        it.box = (int)bi;
        it.kind = ITEM_FACE_ROWS;
        it.x0 = (int)g0;
        it.ex = (int)std::min(fper, fgroups - g0);
        items.push_back(it);
        work.push_back(0.5 * it.ex * V);
      }
      continue;
    }
    for (int z = 0; z < b.iz; z += b.ez)
      for (int y = 0; y < b.iy; y += b.ey)
        for (int x = 0; x < b.ix; x += b.ex) {
          Item it{};
          it.box = (int)bi;
          it.kind = ITEM_TILE;
          it.x0 = b.ox + x;
          it.y0 = b.oy + y;
          it.z0 = b.oz + z;
          it.ex = std::min(b.ex, b.ix - x);
          it.ey = std::min(b.ey, b.iy - y);
          it.ez = std::min(b.ez, b.iz - z);
          items.push_back(it);
          work.push_back((double)it.ex * it.ey * it.ez);
        }
  }
  box_off[ctx->bx.size()] = (int)items.size();
  const int n_items = (int)items.size();
  // launch sequence: boxes by decreasing interior volume (stable)
  std::vector<int> boxes(ctx->bx.size());
  std::iota(boxes.begin(), boxes.end(), 0);
  std::stable_sort(boxes.begin(), boxes.end(),
                   [&](int a, int b) { return ctx->bx[a].interior > ctx->bx[b].interior; });
  std::vector<int> seq;
  seq.reserve(n_items);
  for (int b : boxes)
    for (int i = box_off[b]; i < box_off[b + 1]; i++) seq.push_back(i);
  double total = 0;
  for (double w : work) total += w;
  std::vector<std::vector<int>> piece(8);
  double acc = 0;
  for (int i : seq) {
    int x = (int)std::min(7.0, std::floor(acc / (total / 8.0 + 1e-30)));
    piece[x].push_back(i);
    acc += work[i];
  }
  size_t maxlen = 0;
  for (auto& p : piece) maxlen = std::max(maxlen, p.size());
  std::vector<int> order(8 * maxlen, -1);
  for (int x = 0; x < 8; x++)
    for (size_t j = 0; j < piece[x].size(); j++) order[8 * j + x] = piece[x][j];
  ctx->n_items = n_items;
  ctx->n_entries = (int)order.size();
  int g = grid_override > 0 ? grid_override : ctx->n_entries;
  g = std::max(8, (g + 7) / 8 * 8);
  ctx->grid = std::min(g, std::max(8, ctx->n_entries));
  bool ok = true;
  ctx->d_items = dalloc_t<Item>(ctx, items.size(), &ok);
  ctx->d_order = dalloc_t<int>(ctx, order.size(), &ok);
  // mass/momentum check work list: slabs of whole planes, about 64k nodes each
  std::vector<int4> check;
  std::vector<int> check_off(ctx->bx.size() + 1, 0);
  for (size_t bi = 0; bi < ctx->bx.size(); bi++) {
    const BoxHost& b = ctx->bx[bi];
    check_off[bi] = (int)check.size();
    // whole planes of about 64k nodes; a slab stays below 2^31 nodes (32-bit
    // indices in k_check)
    const int zc = std::max(1, 65536 / std::max(1, b.dim.nx * b.dim.ny));
    for (int z = 0; z < b.dim.nz; z += zc) check.push_back(make_int4((int)bi, z, std::min(b.dim.nz, z + zc), 0));
  }
  check_off[ctx->bx.size()] = (int)check.size();
  ctx->n_check = (int)check.size();
  ctx->d_check_items = dalloc_t<int4>(ctx, check.size(), &ok);
  ctx->d_check_off = dalloc_t<int>(ctx, check_off.size(), &ok);
  ctx->d_partials = dalloc_t<double>(ctx, 4 * check.size(), &ok);
  if (!ok) return fail(ctx, LB_ERR_OOM, "work-list allocation failed");
  HIPCHK(h2d(ctx, ctx->d_items, items.data(), items.size() * sizeof(Item)));
  HIPCHK(h2d(ctx, ctx->d_order, order.data(), order.size() * sizeof(int)));
  HIPCHK(h2d(ctx, ctx->d_check_items, check.data(), check.size() * sizeof(int4)));
  HIPCHK(h2d(ctx, ctx->d_check_off, check_off.data(), check_off.size() * sizeof(int)));
  HIPCHK(dzero(ctx, ctx->d_partials, 4 * sizeof(double) * check.size()));
  ctx->items = items;
  ctx->tables_ready = true;
  std::ostringstream d;
  d << "items=" << n_items << " entries=" << ctx->n_entries << " grid=" << ctx->grid << " tiles:";
  std::map<std::string, int> seen;
  for (auto& b : ctx->bx) {
    std::ostringstream k;
    k << " " << b.dim.nx << "x" << b.dim.ny << "x" << b.dim.nz << "->" << b.ex << "x" << b.ey << "x"
      << b.ez;
    if (!seen.count(k.str())) {
      seen[k.str()] = 1;
      d << k.str();
    }
  }
  ctx->desc = d.str();
  return LB_OK;
}

lb_status upload_boxes(lb_ctx* ctx) {
  ctx->h_boxes.resize(ctx->bx.size());
  // chains sorted by box, stable
  std::vector<int> corder(ctx->ch.size());
  std::iota(corder.begin(), corder.end(), 0);
  std::stable_sort(corder.begin(), corder.end(),
                   [&](int a, int b) { return ctx->ch[a].box < ctx->ch[b].box; });
  std::vector<int> cfirst(ctx->bx.size(), 0), ccount(ctx->bx.size(), 0);
  for (size_t k = 0; k < corder.size(); k++) {
    int b = ctx->ch[corder[k]].box;
    if (ccount[b] == 0) cfirst[b] = (int)k;
    ccount[b]++;
  }
  const double s2 = std::ldexp(1.0, ctx->fp16_exp);
  for (size_t i = 0; i < ctx->bx.size(); i++) {
    const BoxHost& b = ctx->bx[i];
    BoxDesc d{};
    d.off = b.off;
    d.nn = b.nn;
    d.nx = b.dim.nx;
    d.ny = b.dim.ny;
    d.nz = b.dim.nz;
    d.pmask = (int)(b.dim.periodic_mask & 7u);
    d.bc_mode = b.has_bc ? b.bc_mode : -1;
    d.bc_dt = b.bc_dt;
    d.bc_ns = b.bc_ns;
    d.bc_res = b.bc_res;
    d.bc_t0 = b.bc_t0;
    d.bc = b.bc_mode == LB_BC_LEARNED ? b.ring : b.d_bc;
    d.chain_first = cfirst[i];
    d.chain_count = ccount[i];
    d.nbnd = b.nbnd;
    d.n_rect = b.n_rect;
    for (int r = 0; r < MAX_RECT; r++) {
      d.rect_face[r] = b.rect_face[r];
      d.rect_cnt[r] = b.rect_cnt[r];
      for (int a = 0; a < 3; a++) {
        d.rect_start[r][a] = b.rect_start[r][a];
        d.rect_len[r][a] = b.rect_len[r][a];
      }
    }
    d.vec = b.vec ? 1 : 0;
    d.ylog = b.ylog;
    d.vw = b.vw;
    d.xf_off = b.xf_off;
    d.index = (int)i;
    d.body = b.body_ns > 0 ? b.d_body : nullptr;
    d.body_dt = b.body_dt;
    d.body_ns = b.body_ns;
    d.body_t0 = b.body_t0;
    for (int c = 0; c < 3; c++) {
      d.enc[c] = (float)(s2 / WD[c]);
      d.dec[c] = (float)(WD[c] / s2);
    }
    d.s2 = (float)s2;
    d.interior = (double)b.interior;
    d.fast = (!ctx->aa && b.dim.periodic_mask == 0 &&
              (double)Q * (double)b.nn * (double)store_bytes(ctx->S) < 4294967296.0) ? 1 : 0;
    ctx->h_boxes[i] = d;
  }
  HIPCHK(h2d(ctx, ctx->d_boxes, ctx->h_boxes.data(), ctx->h_boxes.size() * sizeof(BoxDesc)));
  return LB_OK;
}

// chain tables, bead state (into the parity buffer of the current step),
// spreading records
lb_status upload_chains(lb_ctx* ctx) {
  dfree(ctx, ctx->d_chains);
  dfree(ctx, ctx->d_pos);
  dfree(ctx, ctx->d_vel);
  dfree(ctx, ctx->d_rec_base);
  dfree(ctx, ctx->d_rec_d);
  dfree(ctx, ctx->d_rec_dp);
  dfree(ctx, ctx->d_bbox);
  ctx->d_chains = nullptr;
  ctx->d_pos = ctx->d_vel = nullptr;
  ctx->d_rec_base = nullptr;
  ctx->d_rec_d = ctx->d_rec_dp = nullptr;
  ctx->d_bbox = nullptr;
  std::vector<int> corder(ctx->ch.size());
  std::iota(corder.begin(), corder.end(), 0);
  std::stable_sort(corder.begin(), corder.end(),
                   [&](int a, int b) { return ctx->ch[a].box < ctx->ch[b].box; });
  std::vector<ChainDesc> cd;
  std::vector<double> rel, vel;
  int first = 0;
  std::vector<int> box_beads(ctx->bx.size(), 0);
  for (int k : corder) {
    const ChainHost& c = ctx->ch[k];
    ChainDesc d{};
    d.box = c.box;
    d.first = first;
    d.bead0 = box_beads[c.box];
    box_beads[c.box] += c.p.n_beads;
    {
      const double h = 1.0 / c.p.md_substeps;
      d.kick = ctx->kT > 0.0 ? std::sqrt(ctx->kT / c.p.mass * (1.0 - std::exp(-2.0 * c.p.zeta * h / c.p.mass)))
                             : 0.0;
    }
    d.nb = c.p.n_beads;
    d.substeps = c.p.md_substeps;
    d.fix_com = c.p.fix_com;
    d.zeta = c.p.zeta;
    d.mass = c.p.mass;
    d.fene_k = c.p.fene_k;
    d.fene_r0 = c.p.fene_r0;
    d.decay = std::exp(-c.p.zeta * (1.0 / c.p.md_substeps) / c.p.mass);
    for (int a = 0; a < 3; a++) {
      const double fl = std::floor(c.p.anchor[a]);
      d.ai[a] = (int)fl;
      d.af[a] = c.p.anchor[a] - fl;
    }
    for (int j = 0; j < d.nb; j++)
      for (int a = 0; a < 3; a++) {
        rel.push_back(c.pos_is_rel ? c.pos[3 * j + a] : (c.pos[3 * j + a] - d.ai[a]) - d.af[a]);
        vel.push_back(c.vel[3 * j + a]);
      }
    first += d.nb;
    cd.push_back(d);
  }
  ctx->total_beads = first;
  bool ok = true;
  const size_t rb = sizeof(double);  // bead state and records: FP64 for every storage
  const size_t nbd = std::max(1, first);
  ctx->d_chains = dalloc_t<ChainDesc>(ctx, std::max<size_t>(1, cd.size()), &ok);
  ctx->d_pos = dalloc(ctx, 2 * 3 * nbd * rb);
  ctx->d_vel = dalloc(ctx, 2 * 3 * nbd * rb);
  ctx->d_rec_base = dalloc_t<int4>(ctx, nbd, &ok);
  ctx->d_rec_d = dalloc(ctx, 3 * nbd * rb);
  ctx->d_rec_dp = dalloc(ctx, 3 * nbd * rb);
  ctx->d_bbox = dalloc_t<int>(ctx, 6 * std::max<size_t>(1, cd.size()), &ok);
  if (!ok || !ctx->d_pos || !ctx->d_vel || !ctx->d_rec_d || !ctx->d_rec_dp)
    return fail(ctx, LB_ERR_OOM, "chain allocation failed");
  if (!cd.empty())
    HIPCHK(h2d(ctx, ctx->d_chains, cd.data(), cd.size() * sizeof(ChainDesc)));
  const int par = (int)(ctx->host_step & 1);
  char* pbase = (char*)ctx->d_pos + (size_t)par * 3 * nbd * rb;
  char* vbase = (char*)ctx->d_vel + (size_t)par * 3 * nbd * rb;
  if (first) {
    HIPCHK(h2d(ctx, pbase, rel.data(), rel.size() * sizeof(double)));
    HIPCHK(h2d(ctx, vbase, vel.data(), vel.size() * sizeof(double)));
  }
  // empty bounding boxes until the first chain step
  std::vector<int> bb(6 * std::max<size_t>(1, cd.size()));
  for (size_t c = 0; c < bb.size() / 6; c++) {
    bb[6 * c] = bb[6 * c + 1] = bb[6 * c + 2] = 1 << 30;
    bb[6 * c + 3] = bb[6 * c + 4] = bb[6 * c + 5] = -(1 << 30);
  }
  HIPCHK(h2d(ctx, ctx->d_bbox, bb.data(), bb.size() * sizeof(int)));
  HIPCHK(dzero(ctx, ctx->d_rec_base, nbd * sizeof(int4)));
  HIPCHK(dzero(ctx, ctx->d_rec_d, 3 * nbd * rb));
  HIPCHK(dzero(ctx, ctx->d_rec_dp, 3 * nbd * rb));
  // chain kernel: one wavefront per chain when every chain fits in one
  int max_nb = 0;
  for (auto& c : ctx->ch) max_nb = std::max(max_nb, c.p.n_beads);
  const bool th = ctx->kT > 0.0;
  if (ctx->S == 0)
    ctx->chain_fn = lbhost::pick_chain<0>(ctx->per, max_nb, th);
  else if (ctx->S == 1)
    ctx->chain_fn = lbhost::pick_chain<1>(ctx->per, max_nb, th);
  else
    ctx->chain_fn = lbhost::pick_chain<2>(ctx->per, max_nb, th);
  ctx->chains_ready = true;
  return upload_boxes(ctx);
}

// Step and force-pass kernels: the extended collision when a box has a body
// force or the context is thermal, the plain one otherwise.
void select_launchers(lb_ctx* ctx) {
  bool ext = ctx->kT > 0.0;
  for (auto& b : ctx->bx) ext = ext || b.body_ns > 0;
  const int kc = ctx->coll == LB_BGK ? 0 : (ctx->cfg.ghost_rate == 1.0 ? 2 : 1);
  const bool aa = ctx->aa;
  switch (ctx->S) {
    case 0: ctx->lb_fn = pick_lb<0>(kc, ctx->per, ext, aa); ctx->force_fn = pick_force<0>(kc, ctx->per, ext); break;
    case 1: ctx->lb_fn = pick_lb<1>(kc, ctx->per, ext, aa); ctx->force_fn = pick_force<1>(kc, ctx->per, ext); break;
    default: ctx->lb_fn = pick_lb<2>(kc, ctx->per, ext, aa); ctx->force_fn = pick_force<2>(kc, ctx->per, ext); break;
  }
}

// Layout of the current state in the buffer of its parity, for readers:
// two buffers hold it pulled, or in place right after an upload; one buffer
// (in-place streaming) holds it as the step's parity says.
int read_layout(const lb_ctx* ctx, int64_t step) {
  if (ctx->aa) return aa_layout(step);
  return ctx->state_pre ? LAYOUT_PLACE : LAYOUT_PULL;
}

lb_status prepare(lb_ctx* ctx) {
  if (!ctx->chains_ready) {
    lb_status s = upload_chains(ctx);
    if (s) return s;
  }
  if (!ctx->tables_ready) {
    lb_status s = build_tables(ctx, ctx->grid > 0 ? ctx->grid : 0);
    if (s) return s;
  }
  return LB_OK;
}

LbArgs make_args(lb_ctx* ctx, int pre, int advance, int reduce_every) {
  LbArgs a{};
  a.boxes = ctx->d_boxes;
  a.items = ctx->d_items;
  a.order = ctx->d_order;
  a.n_entries = ctx->n_entries;
  a.a0 = ctx->arena[0];
  a.a1 = ctx->arena[1];
  a.chains = ctx->d_chains;
  a.rec_base = ctx->d_rec_base;
  a.rec_d = ctx->d_rec_d;
  a.rec_dp = ctx->d_rec_dp;
  a.bbox = ctx->d_bbox;
  a.st = ctx->d_st;
  a.partials = ctx->d_partials;
  a.check_items = ctx->d_check_items;
  a.check_off = ctx->d_check_off;
  a.mass_mom = ctx->d_mass_mom;
  a.xface = ctx->d_xface;
  a.xf_items = ctx->d_xf_items;
  a.n_xf_items = ctx->n_xf_items;
  a.n_boxes = (int)ctx->bx.size();
  a.reduce_every = reduce_every;
  a.rho0 = ctx->cfg.rho0;
  a.omega = 1.0 / ctx->cfg.tau;
  a.om_bulk = 1.0 / ctx->cfg.tau_bulk;
  a.om_ghost = ctx->cfg.ghost_rate;
  a.pre = pre;
  a.advance = advance;
  a.aa = ctx->aa ? 1 : 0;
  if (ctx->aa) a.pre = 0;  // the layout follows from the step's parity
  a.kT = ctx->kT;
  a.key0 = (unsigned)(ctx->seed & 0xffffffffu);
  a.key1 = (unsigned)(ctx->seed >> 32);
  return a;
}

hipEvent_t next_event(lb_ctx* ctx) {
  if (ctx->ev_used >= (int)ctx->ev.size()) {
    hipEvent_t e;
    (void)hipEventCreate(&e);
    ctx->ev.push_back(e);
  }
  return ctx->ev[ctx->ev_used++];
}

// x-face velocities of the row boxes at the current device step, on their own
// (with chains, k_chain's extra workgroups compute them)
void launch_xface(lb_ctx* ctx, hipStream_t s, const LbArgs& a) {
  const dim3 g((unsigned)((ctx->n_xf_items + WG / 64 - 1) / (WG / 64)));
  if (ctx->S == 1)
    hipLaunchKernelGGL(k_xface<1>, g, dim3(WG), 0, s, a);
  else
    hipLaunchKernelGGL(k_xface<2>, g, dim3(WG), 0, s, a);
}

// One step on stream s: k_chain (whose workgroups after the chains compute the
// x-face velocities; k_xface alone when there are no chains), k_lb, k_force
// (chains), k_check, k_finalize.  ev3
// (optional) receives event records before the first kernel, before k_lb and
// after k_lb; st3 (optional, inside captured graphs) receives device
// timestamps from the kernels themselves: the start of the step's first
// kernel, of k_lb, and of the kernel after k_lb.
void enqueue_step(lb_ctx* ctx, hipStream_t s, int pre, const hipEvent_t* ev3,
                  long long* st3, int chk) {
  const bool xf = ctx->n_xf_items > 0, chains = !ctx->ch.empty();
  if (ev3) (void)hipEventRecord(ev3[0], s);
  if (chains) {  // chains and x-face velocities in one launch
    ctx->chain_fn((int)ctx->ch.size(), s, ctx->d_boxes, ctx->d_chains, ctx->arena[0], ctx->arena[1],
                  ctx->d_pos, ctx->d_vel, ctx->total_beads, ctx->d_rec_base, ctx->d_rec_d,
                  ctx->d_rec_dp, ctx->d_bbox, ctx->d_st, ctx->cfg.rho0, ctx->aa ? 2 : pre, st3,
                  ctx->d_xf_items, ctx->n_xf_items, ctx->d_xface,
                  (unsigned)(ctx->seed & 0xffffffffu), (unsigned)(ctx->seed >> 32));
  } else if (xf) {
    LbArgs xa = make_args(ctx, pre, 0, 0);
    if (st3) xa.stamp_first = st3;
    launch_xface(ctx, s, xa);
  }
  if (ev3) (void)hipEventRecord(ev3[1], s);
  LbArgs a = make_args(ctx, pre, 1, ctx->cfg.reduce_every);
  if (st3) {
    a.stamp_lb = st3 + 1;
    if (!xf && !chains) a.stamp_first = st3;
  }
  ctx->lb_fn(dim3(ctx->grid), s, a);
  if (ev3) (void)hipEventRecord(ev3[2], s);
  LbArgs t = make_args(ctx, pre, 1, ctx->cfg.reduce_every);
  if (st3) t.stamp_after = st3 + 2;  // by the first kernel after k_lb
  // on a step known to have no check pass, k_force's last workgroup ends it
  // (in-place streaming: the fused step gathers every chain's force itself)
  const bool force_ends = chains && chk == 0 && !ctx->aa;
  if (chains && !ctx->aa) {  // spread force of the chains of non-periodic boxes
    LbArgs f = t;
    f.advance = force_ends ? 1 : 0;
    ctx->force_fn(dim3((unsigned)ctx->ch.size()), s, f);
    t.stamp_after = nullptr;
  }
  if (force_ends) return;
  if (ctx->cfg.reduce_every > 0 && chk != 0) {
    ctx->check_fn(ctx->n_check, s, t);
    t.stamp_after = nullptr;
  }
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(WG), 0, s, t);
}

void enqueue_step(lb_ctx* ctx, hipStream_t s, int pre, bool timed, int chk) {
  hipEvent_t ev3[3];
  if (timed)
    for (auto& e : ev3) e = next_event(ctx);
  enqueue_step(ctx, s, pre, timed ? ev3 : nullptr, nullptr, chk);
}

// Whether the step that starts at time index n is a check step: 1 or 0 (its
// k_check launch is left out; the kernel would find nothing to do).  The
// host's step count follows the device's until an error latches, after which
// every kernel returns at once.
int check_mode(const lb_ctx* ctx, int64_t n) {
  const int K = ctx->cfg.reduce_every;
  return K > 0 && (n + 1) % K == 0 ? 1 : 0;
}

// Check phase of a graph of gs steps starting at time index n: replays of it
// start at n + j gs, the same phase when K divides gs; otherwise -1 (every
// step launches k_check, which decides on the device)
int graph_phase(const lb_ctx* ctx, int64_t n, int gs) {
  const int K = ctx->cfg.reduce_every;
  if (K <= 0) return 0;
  return gs % K == 0 ? (int)(n % K) : -1;
}

// add the timestamps of one finished timed graph chunk x (copied to pinned
// host memory behind the chunk on the context stream)
lb_status accumulate_chunk(lb_ctx* ctx, int x) {
  const int n = ctx->gsteps_t;
  HIPCHK(hipEventSynchronize(ctx->stamp_ev[x]));
  const long long* t = ctx->h_stamps + (size_t)x * 3 * n;
  const double ms = 1.0 / ctx->clock_khz;  // one clock tick in ms
  for (int k = 0; k < n; k++) {
    ctx->acc_ch += (double)(t[3 * k + 1] - t[3 * k]) * ms;
    ctx->acc_lb += (double)(t[3 * k + 2] - t[3 * k + 1]) * ms;
    if (k + 1 < n) {
      ctx->acc_step += (double)(t[3 * (k + 1)] - t[3 * k]) * ms;
      ctx->acc_step_n++;
    }
  }
  ctx->acc_n += n;
  return LB_OK;
}

// Boundary nodes enumerated by boundary items, as rectangles.  Face priority
// -x, +x, -y, +y, -z, +z: a face excludes the nodes of earlier (lower-axis)
// faces.  Row boxes have none: their x-face nodes are written by the interior
// row items and every other boundary node by the face-row items.
void add_rect(BoxHost& b, int f, int x0, int lx, int y0, int ly, int z0, int lz) {
  if (lx <= 0 || ly <= 0 || lz <= 0) return;
  const int r = b.n_rect++;
  b.rect_face[r] = f;
  b.rect_start[r][0] = x0;
  b.rect_start[r][1] = y0;
  b.rect_start[r][2] = z0;
  b.rect_len[r][0] = lx;
  b.rect_len[r][1] = ly;
  b.rect_len[r][2] = lz;
  b.rect_cnt[r] = lx * ly * lz;
  b.nbnd += lx * ly * lz;
}

void face_tables(BoxHost& b) {
  const int n3[3] = {b.dim.nx, b.dim.ny, b.dim.nz};
  const unsigned pm = b.dim.periodic_mask;
  b.nbnd = 0;
  b.n_rect = 0;
  if (b.vec) return;
  for (int f = 0; f < 6; f++) {
    const int a = f / 2;
    if ((pm >> a) & 1u) continue;
    int st[3], ln[3];
    for (int k = 0; k < 3; k++) {
      if (k == a) {
        st[k] = (f % 2) ? n3[k] - 1 : 0;
        ln[k] = 1;
      } else if (k < a && !((pm >> k) & 1u)) {
        st[k] = 1;
        ln[k] = n3[k] - 2;
      } else {
        st[k] = 0;
        ln[k] = n3[k];
      }
    }
    add_rect(b, f, st[0], ln[0], st[1], ln[1], st[2], ln[2]);
  }
}

lb_status check_box(lb_ctx* ctx, int32_t box) {
  if (!ctx) return LB_ERR_ARG;
  if (box < 0 || box >= (int)ctx->bx.size()) return fail(ctx, LB_ERR_ARG, "box index out of range");
  return LB_OK;
}

lb_status decode_error(lb_ctx* ctx, int key, int64_t step) {
  const int code = key & 15, owner = key >> 4;
  std::ostringstream m;
  lb_status st = LB_ERR_UNSTABLE;
  if (code == EC_BEAD_OUT) {
    st = LB_ERR_BEAD_OUT;
    m << "bead stencil left the interior (chain " << owner << ") at step " << step;
  } else if (code == EC_FENE) {
    st = LB_ERR_FENE;
    m << "FENE bond reached R0 (chain " << owner << ") at step " << step;
  } else {
    m << "non-finite mass or momentum in box " << owner << " at step " << step;
  }
  ctx->err = m.str();
  ctx->latched = st;
  return st;
}

lb_status sync_state(lb_ctx* ctx, DevState* out) {
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(copy_sync(ctx, out, ctx->d_st, sizeof(DevState), hipMemcpyDeviceToHost));
  if (out->err_key != ERR_NONE && ctx->latched == LB_OK) decode_error(ctx, out->err_key, out->step);
  return LB_OK;
}

lb_status vorticity_run(lb_ctx* ctx, int32_t box, int32_t n_vol, const int32_t* vol,
                        double* mean_host, double* field_dev);

// Upload of a box's pre-collision state (k_set_pre modes 0-3) into the buffer
// of the current parity, in the layout that parity expects.
void launch_set_pre(lb_ctx* ctx, int box, const double* in, int mode) {
  const BoxHost& b = ctx->bx[box];
  const int par = (int)(ctx->host_step & 1);
  const int nblk = (int)std::min<int64_t>((b.nn + WG - 1) / WG, 65535);
  const BoxDesc& d = ctx->h_boxes[box];
  const size_t sb = store_bytes(ctx->S);
  void* dst = (char*)ctx->arena[par] + (size_t)b.off * sb;
  const int swap = ctx->aa && aa_layout(ctx->host_step) == LAYOUT_SWAP ? 1 : 0;
  switch (ctx->S) {
    case 0: hipLaunchKernelGGL(k_set_pre<0>, dim3(nblk), dim3(WG), 0, ctx->stream, d, (double*)dst, in, mode, ctx->cfg.rho0, swap); break;
    case 1: hipLaunchKernelGGL(k_set_pre<1>, dim3(nblk), dim3(WG), 0, ctx->stream, d, (float*)dst, in, mode, ctx->cfg.rho0, swap); break;
    default: hipLaunchKernelGGL(k_set_pre<2>, dim3(nblk), dim3(WG), 0, ctx->stream, d, (_Float16*)dst, in, mode, ctx->cfg.rho0, swap); break;
  }
}

}  // namespace

// =========================================================== C ABI
extern "C" {

lb_status lb_init(const lb_config* cfg, lb_ctx** out) {
  if (!cfg || !out) return LB_ERR_ARG;
  *out = nullptr;
  if (cfg->n_boxes < 1 || !cfg->boxes) return LB_ERR_ARG;
  if (!(cfg->tau > 0.5) || (cfg->collision == LB_MRT && !(cfg->tau_bulk > 0.5))) return LB_ERR_ARG;
  if (cfg->collision != LB_BGK && cfg->collision != LB_MRT) return LB_ERR_ARG;
  if (cfg->storage < LB_STORE_F64 || cfg->storage > LB_STORE_F16DEV) return LB_ERR_ARG;
  if (!(cfg->rho0 > 0) || cfg->reduce_every < 0 || cfg->fp16_exp < 0 || cfg->fp16_exp > 24)
    return LB_ERR_ARG;
  if ((cfg->dev_alloc == nullptr) != (cfg->dev_free == nullptr)) return LB_ERR_ARG;
  lb_ctx* ctx = new lb_ctx();
  ctx->cfg = *cfg;
  if (cfg->collision == LB_BGK) {
    ctx->cfg.tau_bulk = cfg->tau;
    ctx->cfg.ghost_rate = 1.0 / cfg->tau;
  }
  ctx->cfg.boxes = nullptr;
  ctx->S = cfg->storage;
  ctx->coll = cfg->collision;
  ctx->fp16_exp = cfg->fp16_exp ? cfg->fp16_exp : 10;
  if (cfg->streaming != LB_STREAM_AB && cfg->streaming != LB_STREAM_AA) {
    delete ctx;
    return LB_ERR_ARG;
  }
  ctx->aa = cfg->streaming == LB_STREAM_AA;
  // one periodic box makes the whole context take the periodic kernel
  // instantiations, which carry only the tile items: no box of such a
  // context may then be a row box
  for (int i = 0; i < cfg->n_boxes; i++)
    if (cfg->boxes[i].periodic_mask & 7u) ctx->per = true;
  int64_t off = 0;
  for (int i = 0; i < cfg->n_boxes; i++) {
    BoxHost b;
    b.dim = cfg->boxes[i];
    const int n3[3] = {b.dim.nx, b.dim.ny, b.dim.nz};
    int64_t nn = 1;
    for (int a = 0; a < 3; a++) {
      const bool p = (b.dim.periodic_mask >> a) & 1u;
      if (n3[a] < (p ? 1 : 3) || n3[a] > 4096) {
        delete ctx;
        return LB_ERR_ARG;
      }
      nn *= n3[a];
    }
    if (nn * Q >= ((int64_t)1 << 40) || nn >= ((int64_t)1 << 31)) {
      delete ctx;
      return LB_ERR_ARG;
    }
    const unsigned pm = b.dim.periodic_mask & 7u;
    b.dim.periodic_mask = pm;
    b.ox = (pm & 1) ? 0 : 1;
    b.oy = (pm & 2) ? 0 : 1;
    b.oz = (pm & 4) ? 0 : 1;
    b.ix = (pm & 1) ? n3[0] : n3[0] - 2;
    b.iy = (pm & 2) ? n3[1] : n3[1] - 2;
    b.iz = (pm & 4) ? n3[2] : n3[2] - 2;
    b.interior = (int64_t)b.ix * b.iy * b.iz;
    b.has_layer = pm != 7u;
    b.nn = nn;
    // every box starts on a 128-element boundary (aligned vector access)
    off = (off + 127) / 128 * 128;
    b.off = off;
    off += nn * Q;
    {
      b.vw = cfg->storage == LB_STORE_F64 ? 0 : pick_row_words(cfg->storage, n3[0]);
      const int V = b.vw ? row_nodes(cfg->storage, b.vw) : 1;
      const double groups = (double)(n3[0] / V) * (n3[1] - 2) * (n3[2] - 2);
      // 32-bit buffer offsets: the planes one workgroup iteration touches
      const double plane = (double)Q * n3[0] * n3[1] * (double)store_bytes(cfg->storage);
      const double span = (WG / ((double)(n3[0] / V) * (n3[1] - 2)) + 4.0) * plane;
      b.vec = b.vw != 0 && !ctx->per && !ctx->aa && groups < 2.0e9 && span < 2147483648.0 && !getenv("LBM_NO_VEC");
      // interleave Y = 2^ylog lines per population row so that a row of a
      // block spans whole 128-byte lines (row boxes only)
      b.ylog = 0;
      if (b.vec) {
        const int rowb = n3[0] * (int)store_bytes(cfg->storage);
        for (int yl = 0; yl <= 2; yl++)
          if ((rowb << yl) % 128 == 0 && n3[1] % (1 << yl) == 0) {
            b.ylog = yl;
            break;
          }
      }
    }
    face_tables(b);
    default_tile(b);
    ctx->bx.push_back(b);
  }
  ctx->arena_elems = off;
  // x-face velocity blocks of the row boxes (2 sides x interior y, z x 3
  // floats) and the x-face work list: chunks of at most XF_ITEM nodes of a box,
  // one per wavefront (each lane evaluates XF_NODES nodes with their loads
  // overlapped)
  int64_t xf_floats = 0;
  std::vector<int4> xf_items;
  for (size_t bi = 0; bi < ctx->bx.size(); bi++) {
    BoxHost& b = ctx->bx[bi];
    if (!b.vec) continue;
    const int64_t nodes = 2LL * (b.dim.ny - 2) * (b.dim.nz - 2);
    if (xf_floats + 3 * nodes >= (1LL << 31)) {  // 32-bit offsets
      lb_free(ctx);
      return LB_ERR_ARG;
    }
    b.xf_off = (int)xf_floats;
    xf_floats += 3 * nodes;
    for (int64_t k = 0; k < nodes; k += XF_ITEM)
      xf_items.push_back(make_int4((int)bi, (int)k, (int)std::min<int64_t>(XF_ITEM, nodes - k), 0));
  }
  // the device this context lives on, and its copy of the static staging
  // array of the allocation-free readout
  if (hipGetDevice(&ctx->dev) != hipSuccess) {
    lb_free(ctx);
    return LB_ERR_HIP;
  }
  ctx->noalloc = scratch_ptr(ctx->dev);
  if (!ctx->noalloc) {
    lb_free(ctx);
    return LB_ERR_HIP;
  }
  // NULL is HIP's null stream (ordered with PyTorch's default stream)
  ctx->stream = (hipStream_t)cfg->stream;
  if (hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    lb_free(ctx);
    return LB_ERR_HIP;
  }
  const size_t sb = store_bytes(ctx->S);
  ctx->arena[0] = dalloc(ctx, (size_t)off * sb);
  // in-place streaming: one buffer serves as both
  ctx->arena[1] = ctx->aa ? ctx->arena[0] : dalloc(ctx, (size_t)off * sb);
  bool ok = ctx->arena[0] && ctx->arena[1];
  ctx->d_boxes = dalloc_t<BoxDesc>(ctx, ctx->bx.size(), &ok);
  ctx->d_mass_mom = dalloc_t<double>(ctx, 5 * ctx->bx.size(), &ok);
  ctx->d_st = dalloc_t<DevState>(ctx, 1, &ok);
  if (!xf_items.empty()) {
    ctx->d_xface = dalloc_t<float>(ctx, (size_t)xf_floats, &ok);
    ctx->d_xf_items = dalloc_t<int4>(ctx, xf_items.size(), &ok);
    ctx->n_xf_items = (int)xf_items.size();
  }
  if (!ok) {
    lb_free(ctx);
    return LB_ERR_OOM;
  }
  if (!xf_items.empty() &&
      (dzero(ctx, ctx->d_xface, (size_t)xf_floats * sizeof(float)) != hipSuccess ||
       h2d(ctx, ctx->d_xf_items, xf_items.data(), xf_items.size() * sizeof(int4)) != hipSuccess)) {
    lb_free(ctx);
    return LB_ERR_HIP;
  }
  // rest state: all deviations zero, in both buffers
  if (dzero(ctx, ctx->arena[0], (size_t)off * sb) != hipSuccess ||
      dzero(ctx, ctx->arena[1], (size_t)off * sb) != hipSuccess ||
      dzero(ctx, ctx->d_mass_mom, 5 * sizeof(double) * ctx->bx.size()) != hipSuccess) {
    lb_free(ctx);
    return LB_ERR_HIP;
  }
  DevState st{};
  st.step = 0;
  st.err_key = ERR_NONE;
  if (h2d(ctx, ctx->d_st, &st, sizeof(st)) != hipSuccess) {
    lb_free(ctx);
    return LB_ERR_HIP;
  }
  select_launchers(ctx);
  ctx->check_fn = ctx->S == 0 ? pick_check<0>(ctx->per)
                              : (ctx->S == 1 ? pick_check<1>(ctx->per) : pick_check<2>(ctx->per));
  load_tune_cache(ctx);
  if (upload_boxes(ctx) != LB_OK) {
    lb_free(ctx);
    return LB_ERR_HIP;
  }
  *out = ctx;
  return LB_OK;
}

lb_status lb_set_initial(lb_ctx* ctx, int32_t box, const double* u) {
  lb_status s = check_box(ctx, box);
  if (s) return s;
  if (!ctx->state_pre) return fail(ctx, LB_ERR_STATE, "lb_set_initial after the first lb_step");
  BoxHost& b = ctx->bx[box];
  double* d_u = nullptr;
  if (u) {
    d_u = (double*)dalloc(ctx, 3 * sizeof(double) * b.nn);
    if (!d_u) return fail(ctx, LB_ERR_OOM, "initial-field staging allocation failed");
    HIPCHK(hipMemcpyAsync(d_u, u, 3 * sizeof(double) * b.nn, hipMemcpyHostToDevice, ctx->stream));
  }
  launch_set_pre(ctx, box, d_u, u ? 1 : 2);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  dfree(ctx, d_u);
  return LB_OK;
}

lb_status lb_set_boundary(lb_ctx* ctx, int32_t box, const lb_boundary* bc) {
  lb_status s = check_box(ctx, box);
  if (s) return s;
  if (!bc || !bc->data || bc->dt < 1 || bc->n_samples < 1)
    return fail(ctx, LB_ERR_ARG, "invalid boundary description");
  if (bc->mode != LB_BC_AFFINE && bc->mode != LB_BC_SAMPLED && bc->mode != LB_BC_LEARNED)
    return fail(ctx, LB_ERR_ARG, "unknown boundary mode");
  if (bc->mode != LB_BC_AFFINE && (bc->res < 2 || bc->res > 8192))
    return fail(ctx, LB_ERR_ARG, "sampled boundary needs res >= 2");
  BoxHost& b = ctx->bx[box];
  if (bc->mode != LB_BC_AFFINE) {
    // the face-grid cell is found in 32-bit integer arithmetic
    const int64_t nmax = std::max(b.dim.nx, std::max(b.dim.ny, b.dim.nz));
    if ((nmax - 1) * (int64_t)(bc->res - 1) >= (int64_t)1 << 31)
      return fail(ctx, LB_ERR_ARG, "(box edge - 1) * (res - 1) must stay below 2^31");
  }
  if (bc->mode == LB_BC_LEARNED) {
    // caller-owned device ring, read in place
    if (ctx->S == LB_STORE_F64 || bc->data_is_f64)
      return fail(ctx, LB_ERR_ARG, "learned boundary rings are FP32 (FP32/FP16 storage)");
    HIPCHK(hipStreamSynchronize(ctx->stream));
    dfree(ctx, b.d_bc);
    b.d_bc = nullptr;
    b.ring = bc->data;
    b.has_bc = true;
    b.bc_mode = bc->mode;
    b.bc_t0 = bc->t0;
    b.bc_dt = bc->dt;
    b.bc_ns = bc->n_samples;
    b.bc_res = bc->res;
    drop_graph(ctx);
    return upload_boxes(ctx);
  }
  size_t per = bc->mode == LB_BC_AFFINE ? 9 : (size_t)6 * bc->res * bc->res * 3;
  size_t n = per * bc->n_samples;
  void* dptr = nullptr;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (bc->mode == LB_BC_AFFINE || ctx->S == LB_STORE_F64) {
    std::vector<double> v(n);
    if (bc->mode == LB_BC_SAMPLED && !bc->data_is_f64) {
      const float* f = (const float*)bc->data;
      for (size_t i = 0; i < n; i++) v[i] = f[i];
    } else {
      std::memcpy(v.data(), bc->data, n * sizeof(double));
    }
    dptr = dalloc(ctx, n * sizeof(double));
    if (!dptr) return fail(ctx, LB_ERR_OOM, "boundary allocation failed");
    HIPCHK(h2d(ctx, dptr, v.data(), n * sizeof(double)));
  } else {
    std::vector<float> v(n);
    if (bc->data_is_f64) {
      const double* f = (const double*)bc->data;
      for (size_t i = 0; i < n; i++) v[i] = (float)f[i];
    } else {
      std::memcpy(v.data(), bc->data, n * sizeof(float));
    }
    dptr = dalloc(ctx, n * sizeof(float));
    if (!dptr) return fail(ctx, LB_ERR_OOM, "boundary allocation failed");
    HIPCHK(h2d(ctx, dptr, v.data(), n * sizeof(float)));
  }
  dfree(ctx, b.d_bc);
  b.d_bc = dptr;
  b.ring = nullptr;
  b.has_bc = true;
  b.bc_mode = bc->mode;
  b.bc_t0 = bc->t0;
  b.bc_dt = bc->dt;
  b.bc_ns = bc->n_samples;
  b.bc_res = bc->res;
  drop_graph(ctx);
  return upload_boxes(ctx);
}

lb_status lb_couple_chain(lb_ctx* ctx, int32_t box, const lb_chain* chain, const double* pos,
                          const double* vel) {
  lb_status s = check_box(ctx, box);
  if (s) return s;
  if (!ctx->state_pre) return fail(ctx, LB_ERR_STATE, "lb_couple_chain after the first lb_step");
  if (!chain || !pos || chain->n_beads < 1 || chain->n_beads > WG || chain->md_substeps < 1 ||
      !(chain->zeta > 0) || !(chain->mass > 0) || !(chain->fene_r0 > 0) || chain->fene_k < 0)
    return fail(ctx, LB_ERR_ARG, "invalid chain (1 <= n_beads <= 256, zeta, mass, R0 > 0)");
  int count = 0;
  for (auto& c : ctx->ch) count += c.box == box;
  if (count >= MAX_BOX_CHAINS) return fail(ctx, LB_ERR_ARG, "at most 64 chains per box");
  ChainHost c;
  c.p = *chain;
  c.box = box;
  c.pos.assign(pos, pos + 3 * chain->n_beads);
  c.vel.assign(3 * chain->n_beads, 0.0);
  if (vel) c.vel.assign(vel, vel + 3 * chain->n_beads);
  ctx->ch.push_back(c);
  ctx->chains_ready = false;
  drop_graph(ctx);
  return LB_OK;
}

lb_status lb_set_body_force(lb_ctx* ctx, int32_t box, int64_t t0, int32_t dt, int32_t n_samples,
                            const double* accel) {
  lb_status s = check_box(ctx, box);
  if (s) return s;
  BoxHost& b = ctx->bx[box];
  if (n_samples < 0 || (n_samples > 0 && (!accel || dt < 1)))
    return fail(ctx, LB_ERR_ARG, "invalid body-force samples");
  for (int64_t k = 0; k < 3 * (int64_t)n_samples; k++)
    if (!std::isfinite(accel[k])) return fail(ctx, LB_ERR_ARG, "non-finite body-force sample");
  HIPCHK(hipStreamSynchronize(ctx->stream));
  double* d = nullptr;
  if (n_samples > 0) {
    d = (double*)dalloc(ctx, (size_t)3 * n_samples * sizeof(double));
    if (!d) return fail(ctx, LB_ERR_OOM, "body-force allocation failed");
    if (h2d(ctx, d, accel, (size_t)3 * n_samples * sizeof(double)) != hipSuccess) {
      dfree(ctx, d);
      return fail(ctx, LB_ERR_HIP, "body-force upload failed");
    }
  }
  dfree(ctx, b.d_body);
  b.d_body = d;
  b.body_ns = n_samples;
  b.body_dt = n_samples > 0 ? dt : 1;
  b.body_t0 = t0;
  select_launchers(ctx);
  drop_graph(ctx);
  return upload_boxes(ctx);
}

lb_status lb_set_thermal(lb_ctx* ctx, double kT, uint64_t seed) {
  if (!ctx) return LB_ERR_ARG;
  if (!(kT >= 0.0) || !std::isfinite(kT)) return fail(ctx, LB_ERR_ARG, "kT must be finite and >= 0");
  if (kT > 0.0 && ctx->coll != LB_MRT)
    return fail(ctx, LB_ERR_ARG, "thermal fluctuations need the MRT collision");
  if (!ctx->state_pre) return fail(ctx, LB_ERR_STATE, "lb_set_thermal after the first lb_step");
  ctx->kT = kT;
  ctx->seed = seed;
  select_launchers(ctx);
  drop_graph(ctx);
  if (ctx->chains_ready && !ctx->ch.empty()) {
    // chains already on the device: refresh their Langevin kicks and the
    // chain kernel variant in place (their state may have been restored)
    std::vector<ChainDesc> cd(ctx->ch.size());
    HIPCHK(copy_sync(ctx, cd.data(), ctx->d_chains, cd.size() * sizeof(ChainDesc),
                     hipMemcpyDeviceToHost));
    int max_nb = 0;
    for (auto& d : cd) {
      const double h = 1.0 / d.substeps;
      d.kick = kT > 0.0 ? std::sqrt(kT / d.mass * (1.0 - std::exp(-2.0 * d.zeta * h / d.mass))) : 0.0;
      max_nb = std::max(max_nb, d.nb);
    }
    HIPCHK(h2d(ctx, ctx->d_chains, cd.data(), cd.size() * sizeof(ChainDesc)));
    const bool th = kT > 0.0;
    if (ctx->S == 0) ctx->chain_fn = lbhost::pick_chain<0>(ctx->per, max_nb, th);
    else if (ctx->S == 1) ctx->chain_fn = lbhost::pick_chain<1>(ctx->per, max_nb, th);
    else ctx->chain_fn = lbhost::pick_chain<2>(ctx->per, max_nb, th);
  }
  return LB_OK;
}

lb_status lb_load_subvolume(lb_ctx* ctx, int32_t box, const char* path, int32_t what) {
  lb_status s = check_box(ctx, box);
  if (s) return s;
  if (!path || (what & ~(LB_SUBVOL_INITIAL | LB_SUBVOL_BOUNDARY | LB_SUBVOL_BODY)))
    return fail(ctx, LB_ERR_ARG, "invalid sub-volume load request");
  std::ifstream in(path, std::ios::binary);
  if (!in) return fail(ctx, LB_ERR_ARG, std::string("cannot open sub-volume file ") + path);
  char magic[8];
  int32_t version = 0, R = 0, ns = 0, dt = 0, flags = 0, reserved = 0;
  int64_t t0 = 0;
  in.read(magic, 8);
  in.read((char*)&version, 4);
  in.read((char*)&R, 4);
  in.read((char*)&ns, 4);
  in.read((char*)&dt, 4);
  in.read((char*)&t0, 8);
  in.read((char*)&flags, 4);
  in.read((char*)&reserved, 4);
  if (!in || std::memcmp(magic, "LBSUBVOL", 8) != 0 || version != 1)
    return fail(ctx, LB_ERR_ARG, "not a version-1 sub-volume file");
  if (R < 2 || R > 1024 || ns < 1 || dt < 1 || (flags & ~1))
    return fail(ctx, LB_ERR_ARG, "invalid sub-volume header");
  const size_t per = (size_t)R * R * R * 3;
  std::vector<float> w(per * ns);
  in.read((char*)w.data(), (std::streamsize)(w.size() * sizeof(float)));
  std::vector<double> acc;
  if (flags & 1) {
    acc.resize((size_t)3 * ns);
    in.read((char*)acc.data(), (std::streamsize)(acc.size() * sizeof(double)));
  }
  if (!in) return fail(ctx, LB_ERR_ARG, "sub-volume file shorter than its header says");
  in.peek();
  if (!in.eof()) return fail(ctx, LB_ERR_ARG, "sub-volume file longer than its header says");
  if ((what & LB_SUBVOL_BODY) && !(flags & 1))
    return fail(ctx, LB_ERR_ARG, "sub-volume file holds no tracer accelerations");
  const BoxHost& b = ctx->bx[box];
  const int n3[3] = {b.dim.nx, b.dim.ny, b.dim.nz};
  // grid value of sample k at grid point (i, j, l) along x, y, z, component c
  auto W = [&](int k, int i, int j, int l, int c) -> float {
    return w[(((size_t)k * R + l) * R + j) * R * 3 + (size_t)i * 3 + c];
  };
  if (what & LB_SUBVOL_BOUNDARY) {
    // the six faces of the grid, corner-aligned with the box's faces: face f
    // lies on axis f/2 at grid index 0 or R-1, entry [v][u] with u the
    // lower-index tangential axis (the SAMPLED layout)
    std::vector<float> faces((size_t)ns * 6 * R * R * 3);
    for (int k = 0; k < ns; k++)
      for (int f = 0; f < 6; f++) {
        const int a = f / 2, au = a == 0 ? 1 : 0, av = a == 2 ? 1 : 2;
        for (int iv = 0; iv < R; iv++)
          for (int iu = 0; iu < R; iu++) {
            int g[3];
            g[a] = (f % 2) ? R - 1 : 0;
            g[au] = iu;
            g[av] = iv;
            for (int c = 0; c < 3; c++)
              faces[((((size_t)k * 6 + f) * R + iv) * R + iu) * 3 + c] = W(k, g[0], g[1], g[2], c);
          }
      }
    lb_boundary bc{};
    bc.mode = LB_BC_SAMPLED;
    bc.t0 = t0;
    bc.dt = dt;
    bc.n_samples = ns;
    bc.res = R;
    bc.data = faces.data();
    bc.data_is_f64 = 0;
    s = lb_set_boundary(ctx, box, &bc);
    if (s) return s;
  }
  if (what & LB_SUBVOL_INITIAL) {
    // Sec. 2: the sub-volume field linearly interpolated onto every site at
    // t = 0: grid point p of an axis sits at node coordinate p (n - 1)/(R - 1)
    if (n3[0] < 2 || n3[1] < 2 || n3[2] < 2)
      return fail(ctx, LB_ERR_ARG, "a sub-volume initial field needs two nodes per axis");
    std::vector<double> u((size_t)3 * b.nn);
    std::vector<int> cell[3];
    std::vector<double> frac[3];
    for (int a = 0; a < 3; a++) {
      cell[a].resize(n3[a]);
      frac[a].resize(n3[a]);
    }
    for (int a = 0; a < 3; a++)
      for (int q = 0; q < n3[a]; q++) {
        const int64_t sq = (int64_t)q * (R - 1);
        int p = (int)(sq / (n3[a] - 1));
        if (p > R - 2) p = R - 2;
        cell[a][q] = p;
        frac[a][q] = (double)(sq - (int64_t)p * (n3[a] - 1)) / (double)(n3[a] - 1);
      }
    for (int z = 0; z < n3[2]; z++)
      for (int y = 0; y < n3[1]; y++)
        for (int x = 0; x < n3[0]; x++) {
          const int ci = cell[0][x], cj = cell[1][y], cl = cell[2][z];
          const double fx = frac[0][x], fy = frac[1][y], fz = frac[2][z];
          for (int c = 0; c < 3; c++) {
            double v = 0.0;
            for (int o = 0; o < 8; o++) {
              const int ox = o & 1, oy = (o >> 1) & 1, oz = (o >> 2) & 1;
              const double wgt = (ox ? fx : 1.0 - fx) * (oy ? fy : 1.0 - fy) * (oz ? fz : 1.0 - fz);
              v += wgt * (double)W(0, ci + ox, cj + oy, cl + oz, c);
            }
            u[(((size_t)z * n3[1] + y) * n3[0] + x) * 3 + c] = v;
          }
        }
    s = lb_set_initial(ctx, box, u.data());
    if (s) return s;
  }
  if (what & LB_SUBVOL_BODY) {
    s = lb_set_body_force(ctx, box, t0, dt, ns, acc.data());
    if (s) return s;
  }
  return LB_OK;
}

lb_status lb_step(lb_ctx* ctx, int32_t n_steps) {
  if (!ctx || n_steps < 0) return LB_ERR_ARG;
  if (ctx->latched) return ctx->latched;
  if (n_steps == 0) return LB_OK;
  for (auto& b : ctx->bx) {
    if (!b.has_layer) continue;
    if (!b.has_bc) return fail(ctx, LB_ERR_STATE, "a box with a boundary layer has no boundary");
    const int64_t first = ctx->host_step, last = ctx->host_step + n_steps - 1;
    const int64_t end = b.bc_t0 + (int64_t)(b.bc_ns - 1) * b.bc_dt;
    if (first < b.bc_t0 || (b.bc_mode != LB_BC_LEARNED && last > end))
      return fail(ctx, LB_ERR_ARG, "steps beyond the boundary samples (no extrapolation)");
  }
  for (auto& b : ctx->bx) {
    if (b.body_ns <= 0) continue;
    const int64_t first = ctx->host_step, last = ctx->host_step + n_steps - 1;
    const int64_t end = b.body_t0 + (int64_t)(b.body_ns - 1) * b.body_dt;
    if (first < b.body_t0 || last > end)
      return fail(ctx, LB_ERR_ARG, "steps beyond the body-force samples (no extrapolation)");
  }
  lb_status s = prepare(ctx);
  if (s) return s;
  int left = n_steps;
  const bool timed = ctx->timing;
  if (timed) {
    ctx->ev_used = 0;
    ctx->t_steps = 0;
    ctx->acc_lb = ctx->acc_ch = ctx->acc_step = 0;
    ctx->acc_n = ctx->acc_step_n = 0;
  }
  int64_t hs = ctx->host_step;  // time index of the next step enqueued
  if (ctx->state_pre) {
    enqueue_step(ctx, ctx->stream, 1, timed, check_mode(ctx, hs));
    HIPCHK(hipGetLastError());
    ctx->state_pre = false;
    left--;
    hs++;
    if (timed) ctx->t_steps++;
  }
  const int gs = ctx->cfg.graph_steps;
  const int phase = gs > 0 ? graph_phase(ctx, hs, gs) : -1;
  auto graph_chk = [&](int k) { return phase < 0 ? -1 : check_mode(ctx, (int64_t)phase + k); };
  if (gs > 0 && ctx->gphase != phase) drop_graph(ctx);
  if (gs > 0 && timed && left >= gs) {
    // HIP events recorded inside a graph cannot be timed: in the timed graphs
    // the kernels record device timestamps themselves
    if (!ctx->gexec_t[0] || ctx->gsteps_t != gs) {
      drop_graph(ctx);
      drop_stamps(ctx);
      int dev = 0, khz = 0;
      HIPCHK(hipGetDevice(&dev));
      HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
      if (khz <= 0) return fail(ctx, LB_ERR_HIP, "device wall-clock rate unavailable");
      ctx->clock_khz = khz;
      bool ok = true;
      ctx->d_stamps = dalloc_t<long long>(ctx, 6 * (size_t)gs, &ok);
      if (!ok) return fail(ctx, LB_ERR_OOM, "timestamp buffer allocation failed");
      HIPCHK(hipHostMalloc((void**)&ctx->h_stamps, 6 * (size_t)gs * sizeof(long long),
                           hipHostMallocDefault));
      for (auto& e : ctx->stamp_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      for (int x = 0; x < 2; x++) {
        hipGraph_t g;
        HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
        for (int k = 0; k < gs; k++)
          enqueue_step(ctx, ctx->cap_stream, 0, nullptr, ctx->d_stamps + (size_t)x * 3 * gs + 3 * k,
                       graph_chk(k));
        HIPCHK(hipStreamEndCapture(ctx->cap_stream, &g));
        HIPCHK(hipGraphInstantiate(&ctx->gexec_t[x], g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
      }
      ctx->gsteps_t = gs;
      ctx->gphase = phase;
    }
    const size_t nb = 3 * (size_t)gs * sizeof(long long);
    int j = 0;
    for (; left >= gs; j++, left -= gs, hs += gs) {
      const int x = j & 1;
      if (j >= 2) {  // chunk j-2 used the same buffers: its stamps must be read first
        lb_status st = accumulate_chunk(ctx, x);
        if (st) return st;
      }
      HIPCHK(hipGraphLaunch(ctx->gexec_t[x], ctx->stream));
      HIPCHK(hipMemcpyAsync(ctx->h_stamps + (size_t)x * 3 * gs, ctx->d_stamps + (size_t)x * 3 * gs,
                            nb, hipMemcpyDeviceToHost, ctx->stream));
      HIPCHK(hipEventRecord(ctx->stamp_ev[x], ctx->stream));
    }
    for (int r = std::max(0, j - 2); r < j; r++) {
      lb_status st = accumulate_chunk(ctx, r & 1);
      if (st) return st;
    }
  }
  if (gs > 0 && !timed) {
    while (left >= gs) {
      if (!ctx->gexec || ctx->gsteps != gs) {
        drop_graph(ctx);
        hipGraph_t g;
        HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
        for (int k = 0; k < gs; k++) enqueue_step(ctx, ctx->cap_stream, 0, false, graph_chk(k));
        HIPCHK(hipStreamEndCapture(ctx->cap_stream, &g));
        HIPCHK(hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
        ctx->gsteps = gs;
        ctx->gphase = phase;
      }
      HIPCHK(hipGraphLaunch(ctx->gexec, ctx->stream));
      left -= gs;
      hs += gs;
    }
  }
  while (left > 0) {
    enqueue_step(ctx, ctx->stream, 0, timed, check_mode(ctx, hs));
    left--;
    hs++;
    if (timed) ctx->t_steps++;
  }
  HIPCHK(hipGetLastError());
  ctx->host_step += n_steps;
  return LB_OK;
}

lb_status lb_sync(lb_ctx* ctx) {
  if (!ctx) return LB_ERR_ARG;
  DevState st;
  lb_status s = sync_state(ctx, &st);
  if (s) return s;
  return ctx->latched;
}

lb_status lb_read_fields(lb_ctx* ctx, int32_t box, lb_field field, void* dst, size_t dst_bytes,
                         int32_t dst_on_device) {
  if (!ctx || !dst) return LB_ERR_ARG;
  if (field != LB_F_STEP) {
    lb_status s = check_box(ctx, box);
    if (s) return s;
  }
  lb_status s = prepare(ctx);
  if (s) return s;
  DevState st;
  s = sync_state(ctx, &st);
  if (s) return s;
  const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (field == LB_F_STEP) {
    if (dst_bytes != sizeof(int64_t)) return fail(ctx, LB_ERR_BUFSIZE, "LB_F_STEP needs 8 bytes");
    int64_t v = st.step;
    if (dst_on_device)
      HIPCHK(h2d(ctx, dst, &v, 8));
    else
      std::memcpy(dst, &v, 8);
    return ctx->latched;
  }
  BoxHost& b = ctx->bx[box];
  if (field == LB_F_MASS_MOM) {
    if (dst_bytes != 5 * sizeof(double)) return fail(ctx, LB_ERR_BUFSIZE, "LB_F_MASS_MOM needs 40 bytes");
    HIPCHK(copy_sync(ctx, dst, ctx->d_mass_mom + 5 * box, 5 * sizeof(double), kind));
    return ctx->latched;
  }
  const int par = (int)(st.step & 1);
  if (field == LB_F_BEAD_POS || field == LB_F_BEAD_VEL || field == LB_F_BEAD_REL) {
    int c0 = ctx->h_boxes[box].chain_first, c1 = c0 + ctx->h_boxes[box].chain_count;
    int nb = 0;
    for (auto& c : ctx->ch) nb += (c.box == box) ? c.p.n_beads : 0;
    if (dst_bytes != (size_t)nb * 3 * sizeof(double))
      return fail(ctx, LB_ERR_BUFSIZE, "bead buffer must be [beads][3] doubles");
    if (nb == 0) return ctx->latched;
    double* tmp = (double*)dalloc(ctx, (size_t)nb * 3 * sizeof(double));
    if (!tmp) return fail(ctx, LB_ERR_OOM, "readout allocation failed");
    const size_t nbd = std::max(1, ctx->total_beads);
    const bool is_pos = field != LB_F_BEAD_VEL;
    const void* src = (char*)(is_pos ? ctx->d_pos : ctx->d_vel) + (size_t)par * 3 * nbd * sizeof(double);
    hipLaunchKernelGGL(k_read_beads<double>, dim3(1), dim3(WG), 0, ctx->stream, ctx->d_chains, c0, c1,
                       (const double*)src, tmp, field == LB_F_BEAD_POS ? 1 : 0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(copy_sync(ctx, dst, tmp, (size_t)nb * 3 * sizeof(double), kind));
    dfree(ctx, tmp);
    return ctx->latched;
  }
  if (field == LB_F_VORT) {
    const size_t need = (size_t)b.nn * sizeof(double);
    if (dst_bytes != need) return fail(ctx, LB_ERR_BUFSIZE, "LB_F_VORT needs [nz][ny][nx] doubles");
    int v6[6];
    for (int a = 0; a < 3; a++) {
      const int n = a == 0 ? b.dim.nx : (a == 1 ? b.dim.ny : b.dim.nz);
      const bool p = (b.dim.periodic_mask >> a) & 1u;
      v6[a] = p ? 0 : 2;
      v6[3 + a] = p ? n - 1 : n - 3;
      if (v6[a] > v6[3 + a]) {  // no node with interior neighbours: all zero
        v6[0] = 1;
        v6[3] = 0;
      }
    }
    double* out = dst_on_device ? (double*)dst : (double*)dalloc(ctx, need);
    if (!out) return fail(ctx, LB_ERR_OOM, "readout allocation failed");
    lb_status r = dzero(ctx, out, need) == hipSuccess ? LB_OK : fail(ctx, LB_ERR_HIP, "zero fill failed");
    if (!r && v6[0] <= v6[3]) r = vorticity_run(ctx, box, 1, v6, nullptr, out);
    if (!r) r = hipStreamSynchronize(ctx->stream) == hipSuccess ? LB_OK : fail(ctx, LB_ERR_HIP, "sync failed");
    if (!r && !dst_on_device && copy_sync(ctx, dst, out, need, hipMemcpyDeviceToHost) != hipSuccess)
      r = fail(ctx, LB_ERR_HIP, "copy failed");
    if (!dst_on_device) dfree(ctx, out);
    return r ? r : ctx->latched;
  }
  int what;
  size_t need;
  if (field == LB_F_POP || field == LB_F_POP_DEV) {
    what = field == LB_F_POP ? 0 : 3;
    need = (size_t)Q * b.nn * sizeof(double);
  } else if (field == LB_F_RHO) {
    what = 1;
    need = (size_t)b.nn * sizeof(double);
  } else if (field == LB_F_U) {
    what = 2;
    need = (size_t)3 * b.nn * sizeof(double);
  } else {
    return fail(ctx, LB_ERR_ARG, "unknown field");
  }
  if (dst_bytes != need) return fail(ctx, LB_ERR_BUFSIZE, "field buffer size mismatch");
  double* out = dst_on_device ? (double*)dst : (double*)dalloc(ctx, need);
  if (!out) return fail(ctx, LB_ERR_OOM, "readout allocation failed");
  const size_t sb = store_bytes(ctx->S);
  const void* src = (char*)ctx->arena[par] + (size_t)b.off * sb;
  const int nblk = (int)std::min<int64_t>((b.nn + WG - 1) / WG, 65535);
  const int pre = read_layout(ctx, st.step);
  const BoxDesc& d = ctx->h_boxes[box];
  const double r0 = ctx->cfg.rho0;
  if (ctx->S == 0) launch_read<0>(ctx->per, nblk, ctx->stream, d, src, out, what, pre, r0);
  else if (ctx->S == 1) launch_read<1>(ctx->per, nblk, ctx->stream, d, src, out, what, pre, r0);
  else launch_read<2>(ctx->per, nblk, ctx->stream, d, src, out, what, pre, r0);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (!dst_on_device) {
    HIPCHK(copy_sync(ctx, dst, out, need, hipMemcpyDeviceToHost));
    dfree(ctx, out);
  }
  return ctx->latched;
}

}  // extern "C"

namespace {

template <int S>
void launch_vort(bool per, int grid, hipStream_t s, const VortArgs& a) {
  if (per)
    hipLaunchKernelGGL((k_vort<S, true>), dim3(grid), dim3(VT * VT), 0, s, a);
  else
    hipLaunchKernelGGL((k_vort<S, false>), dim3(grid), dim3(VT * VT), 0, s, a);
}

// Vorticity of n_vol control volumes of a box (vol: [n_vol][6] = lo x, y, z,
// hi x, y, z inclusive): their means to mean_host (may be NULL) and, when
// field_dev is given, |omega| per node into that device [nz][ny][nx] array.
// Every node of a volume needs its six axis neighbours in the interior.
lb_status vorticity_run(lb_ctx* ctx, int32_t box, int32_t n_vol, const int32_t* vol,
                        double* mean_host, double* field_dev) {
  const BoxHost& b = ctx->bx[box];
  const int n3[3] = {b.dim.nx, b.dim.ny, b.dim.nz};
  std::vector<int> off(1, 0);
  std::vector<double> count;
  std::vector<std::array<int, 4>> shape;  // tx, ty, zslab, grid per volume
  for (int v = 0; v < n_vol; v++) {
    const int* lo = vol + 6 * v;
    const int* hi = lo + 3;
    double cnt = 1.0;
    for (int a = 0; a < 3; a++) {
      const bool p = (b.dim.periodic_mask >> a) & 1u;
      const int mn = p ? 0 : 2, mx = p ? n3[a] - 1 : n3[a] - 3;
      if (lo[a] > hi[a] || lo[a] < mn || hi[a] > mx)
        return fail(ctx, LB_ERR_ARG, "control volume outside the nodes whose neighbours are interior");
      cnt *= (double)(hi[a] - lo[a] + 1);
    }
    const int tx = (hi[0] - lo[0] + VT) / VT, ty = (hi[1] - lo[1] + VT) / VT;
    const int ez = hi[2] - lo[2] + 1;
    const int zslab = std::max(4, std::min(32, (int)(((int64_t)ez * tx * ty + 2047) / 2048)));
    const int64_t grid = (int64_t)tx * ty * ((ez + zslab - 1) / zslab);
    if (grid + off.back() >= (1 << 30)) return fail(ctx, LB_ERR_ARG, "control volumes too large");
    shape.push_back({tx, ty, zslab, (int)grid});
    off.push_back(off.back() + (int)grid);
    count.push_back(cnt);
  }
  if (n_vol == 0) return LB_OK;
  lb_status s = prepare(ctx);
  if (s) return s;
  DevState st;
  s = sync_state(ctx, &st);
  if (s) return s;
  double* d_part = (double*)dalloc(ctx, (size_t)off.back() * sizeof(double));
  int* d_off = (int*)dalloc(ctx, off.size() * sizeof(int));
  double* d_cnt = (double*)dalloc(ctx, count.size() * sizeof(double));
  double* d_mean = (double*)dalloc(ctx, count.size() * sizeof(double));
  auto release = [&]() {
    dfree(ctx, d_part);
    dfree(ctx, d_off);
    dfree(ctx, d_cnt);
    dfree(ctx, d_mean);
  };
  if (!d_part || !d_off || !d_cnt || !d_mean) {
    release();
    return fail(ctx, LB_ERR_OOM, "vorticity work buffers");
  }
  if (h2d(ctx, d_off, off.data(), off.size() * sizeof(int)) != hipSuccess ||
      h2d(ctx, d_cnt, count.data(), count.size() * sizeof(double)) != hipSuccess) {
    release();
    return fail(ctx, LB_ERR_HIP, "vorticity tables upload failed");
  }
  const size_t sb = store_bytes(ctx->S);
  VortArgs a{};
  a.b = ctx->h_boxes[box];
  a.src = (char*)ctx->arena[(int)(st.step & 1)] + (size_t)b.off * sb;
  a.pre = read_layout(ctx, st.step);
  a.rho0 = ctx->cfg.rho0;
  a.field = field_dev;
  for (int v = 0; v < n_vol; v++) {
    for (int k = 0; k < 3; k++) {
      a.lo[k] = vol[6 * v + k];
      a.hi[k] = vol[6 * v + 3 + k];
    }
    a.tx = shape[v][0];
    a.ty = shape[v][1];
    a.zslab = shape[v][2];
    a.partials = d_part + off[v];
    if (ctx->S == 0) launch_vort<0>(ctx->per, shape[v][3], ctx->stream, a);
    else if (ctx->S == 1) launch_vort<1>(ctx->per, shape[v][3], ctx->stream, a);
    else launch_vort<2>(ctx->per, shape[v][3], ctx->stream, a);
  }
  hipLaunchKernelGGL(k_vort_sum, dim3(1), dim3(WG), 0, ctx->stream, d_part, d_off, d_cnt, n_vol, d_mean);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && mean_host)
    e = copy_sync(ctx, mean_host, d_mean, (size_t)n_vol * sizeof(double), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  release();
  if (e != hipSuccess) return fail(ctx, LB_ERR_HIP, std::string("vorticity: ") + hipGetErrorString(e));
  return ctx->latched;
}

lb_status check_sites(lb_ctx* ctx, int32_t box, int32_t n, const int32_t* xyz, const double* out) {
  lb_status s = check_box(ctx, box);
  if (s) return s;
  if (n < 0 || (n > 0 && (!xyz || !out))) return fail(ctx, LB_ERR_ARG, "invalid site list");
  const BoxHost& b = ctx->bx[box];
  for (int k = 0; k < n; k++) {
    const int x = xyz[3 * k], y = xyz[3 * k + 1], z = xyz[3 * k + 2];
    const bool in = ((b.dim.periodic_mask & 1) ? (x >= 0 && x < b.dim.nx) : (x >= 1 && x <= b.dim.nx - 2)) &&
                    ((b.dim.periodic_mask & 2) ? (y >= 0 && y < b.dim.ny) : (y >= 1 && y <= b.dim.ny - 2)) &&
                    ((b.dim.periodic_mask & 4) ? (z >= 0 && z < b.dim.nz) : (z >= 1 && z <= b.dim.nz - 2));
    if (!in) return fail(ctx, LB_ERR_ARG, "site outside the interior");
  }
  return LB_OK;
}

// Populations of n sites of a box at the current step: the site list is
// already in d_xyz (device), the kernel writes d_out (device, [n][19]), which
// is then copied to the host buffer out.
lb_status sites_to_host(lb_ctx* ctx, int32_t box, int32_t n, const DevState& st, const int* d_xyz,
                        double* d_out, double* out) {
  const BoxHost& b = ctx->bx[box];
  const int par = (int)(st.step & 1);
  const size_t sb = store_bytes(ctx->S);
  const void* src = (char*)ctx->arena[par] + (size_t)b.off * sb;
  const BoxDesc& d = ctx->h_boxes[box];
  const int pre = read_layout(ctx, st.step);
  const int nblk = (n + WG - 1) / WG;
  const double r0 = ctx->cfg.rho0;
  if (ctx->S == 0) launch_sites<0>(ctx->per, nblk, ctx->stream, d, src, d_xyz, n, d_out, pre, r0);
  else if (ctx->S == 1) launch_sites<1>(ctx->per, nblk, ctx->stream, d, src, d_xyz, n, d_out, pre, r0);
  else launch_sites<2>(ctx->per, nblk, ctx->stream, d, src, d_xyz, n, d_out, pre, r0);
  HIPCHK(hipGetLastError());
  HIPCHK(copy_sync(ctx, out, d_out, (size_t)Q * n * sizeof(double), hipMemcpyDeviceToHost));
  return LB_OK;
}

}  // namespace

extern "C" {

lb_status lb_read_sites(lb_ctx* ctx, int32_t box, int32_t n, const int32_t* xyz, double* out) {
  lb_status s = check_sites(ctx, box, n, xyz, out);
  if (s || n == 0) return s;
  s = prepare(ctx);
  if (s) return s;
  DevState st;
  s = sync_state(ctx, &st);
  if (s) return s;
  int* d_xyz = (int*)dalloc(ctx, (size_t)3 * n * sizeof(int));
  double* d_out = (double*)dalloc(ctx, (size_t)Q * n * sizeof(double));
  if (!d_xyz || !d_out) {
    dfree(ctx, d_xyz);
    dfree(ctx, d_out);
    return fail(ctx, LB_ERR_OOM, "site readout allocation failed");
  }
  s = h2d(ctx, d_xyz, xyz, (size_t)3 * n * sizeof(int)) == hipSuccess
          ? sites_to_host(ctx, box, n, st, d_xyz, d_out, out)
          : fail(ctx, LB_ERR_HIP, "site list upload failed");
  dfree(ctx, d_xyz);
  dfree(ctx, d_out);
  return s ? s : ctx->latched;
}

lb_status lb_vorticity(lb_ctx* ctx, int32_t box, int32_t n_vol, const int32_t* vol, double* mean) {
  lb_status s = check_box(ctx, box);
  if (s) return s;
  if (n_vol < 0 || (n_vol > 0 && (!vol || !mean))) return fail(ctx, LB_ERR_ARG, "invalid control volumes");
  return vorticity_run(ctx, box, n_vol, vol, mean, nullptr);
}

lb_status lb_read_sites_noalloc(lb_ctx* ctx, int32_t box, int32_t n, const int32_t* xyz, double* out) {
  lb_status s = check_sites(ctx, box, n, xyz, out);
  if (s || n == 0) return s;
  if (n > NOALLOC_SITES)
    return fail(ctx, LB_ERR_ARG, "lb_read_sites_noalloc reads at most 32768 sites per call");
  if (!ctx->chains_ready || !ctx->tables_ready)
    return fail(ctx, LB_ERR_STATE, "lb_read_sites_noalloc needs a context that has stepped or been "
                                   "read once (its device tables are built then)");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != ctx->dev)
    return fail(ctx, LB_ERR_STATE, "lb_read_sites_noalloc called with another device current");
  DevState st;
  s = sync_state(ctx, &st);
  if (s) return s;
  int* d_xyz = (int*)ctx->noalloc;
  double* d_out = (double*)((char*)ctx->noalloc + NOALLOC_XYZ_BYTES);
  HIPCHK(h2d(ctx, d_xyz, xyz, (size_t)3 * n * sizeof(int)));
  s = sites_to_host(ctx, box, n, st, d_xyz, d_out, out);
  return s ? s : ctx->latched;
}

lb_status lb_write_state(lb_ctx* ctx, int32_t box, lb_field field, const void* src, size_t bytes) {
  if (!ctx || !src) return LB_ERR_ARG;
  if (!ctx->state_pre) return fail(ctx, LB_ERR_STATE, "lb_write_state after the first lb_step");
  if (field == LB_F_STEP) {
    if (bytes != 8) return fail(ctx, LB_ERR_BUFSIZE, "LB_F_STEP needs 8 bytes");
    int64_t n;
    std::memcpy(&n, src, 8);
    if (n < 0) return fail(ctx, LB_ERR_ARG, "negative step");
    const int old_par = (int)(ctx->host_step & 1), new_par = (int)(n & 1);
    if (old_par != new_par && ctx->aa) {
      // one buffer: re-lay every box out as the new parity reads it (the
      // deviations through FP64, exactly as a checkpoint round trip)
      lb_status r = prepare(ctx);
      if (r) return r;
      for (int bi = 0; bi < (int)ctx->bx.size(); bi++) {
        const BoxHost& b = ctx->bx[bi];
        const size_t need = (size_t)Q * b.nn * sizeof(double);
        double* tmp = (double*)dalloc(ctx, need);
        if (!tmp) return fail(ctx, LB_ERR_OOM, "re-layout staging allocation failed");
        const size_t sb = store_bytes(ctx->S);
        const void* srcb = (char*)ctx->arena[0] + (size_t)b.off * sb;
        const int nblk = (int)std::min<int64_t>((b.nn + WG - 1) / WG, 65535);
        const int lay = aa_layout(ctx->host_step);
        const BoxDesc& d = ctx->h_boxes[bi];
        if (ctx->S == 0) launch_read<0>(ctx->per, nblk, ctx->stream, d, srcb, tmp, 3, lay, ctx->cfg.rho0);
        else if (ctx->S == 1) launch_read<1>(ctx->per, nblk, ctx->stream, d, srcb, tmp, 3, lay, ctx->cfg.rho0);
        else launch_read<2>(ctx->per, nblk, ctx->stream, d, srcb, tmp, 3, lay, ctx->cfg.rho0);
        const int64_t keep = ctx->host_step;
        ctx->host_step = n;
        launch_set_pre(ctx, bi, tmp, 3);
        ctx->host_step = keep;
        hipError_t e = hipStreamSynchronize(ctx->stream);
        dfree(ctx, tmp);
        if (e != hipSuccess) return fail(ctx, LB_ERR_HIP, "re-layout failed");
      }
      ctx->chains_ready = false;
    } else if (old_par != new_par) {
      const size_t sb = store_bytes(ctx->S);
      HIPCHK(copy_sync(ctx, ctx->arena[new_par], ctx->arena[old_par], (size_t)ctx->arena_elems * sb,
                       hipMemcpyDeviceToDevice));
      ctx->chains_ready = false;  // bead state is re-uploaded into the new parity
    }
    ctx->host_step = n;
    DevState st{};
    st.step = n;
    st.err_key = ERR_NONE;
    HIPCHK(h2d(ctx, ctx->d_st, &st, sizeof(st)));
    return LB_OK;
  }
  lb_status s = check_box(ctx, box);
  if (s) return s;
  BoxHost& b = ctx->bx[box];
  if (field == LB_F_BEAD_POS || field == LB_F_BEAD_VEL || field == LB_F_BEAD_REL) {
    size_t nb = 0;
    for (auto& c : ctx->ch) nb += (c.box == box) ? c.p.n_beads : 0;
    if (bytes != nb * 3 * sizeof(double)) return fail(ctx, LB_ERR_BUFSIZE, "bead state size mismatch");
    const double* p = (const double*)src;
    size_t o = 0;
    for (auto& c : ctx->ch) {
      if (c.box != box) continue;
      auto& v = field == LB_F_BEAD_VEL ? c.vel : c.pos;
      v.assign(p + o, p + o + 3 * c.p.n_beads);
      c.pos_is_rel = field == LB_F_BEAD_REL ? true : (field == LB_F_BEAD_POS ? false : c.pos_is_rel);
      o += 3 * c.p.n_beads;
    }
    ctx->chains_ready = false;
    return LB_OK;
  }
  if (field != LB_F_POP && field != LB_F_POP_DEV)
    return fail(ctx, LB_ERR_ARG, "only POP, POP_DEV, BEAD_POS, BEAD_VEL, STEP are writable");
  const int mode = field == LB_F_POP ? 0 : 3;
  if (bytes != (size_t)Q * b.nn * sizeof(double)) return fail(ctx, LB_ERR_BUFSIZE, "POP size mismatch");
  double* d_in = (double*)dalloc(ctx, bytes);
  if (!d_in) return fail(ctx, LB_ERR_OOM, "staging allocation failed");
  HIPCHK(h2d(ctx, d_in, src, bytes));
  launch_set_pre(ctx, box, d_in, mode);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  dfree(ctx, d_in);
  return LB_OK;
}

lb_status lb_set_timing(lb_ctx* ctx, int32_t on) {
  if (!ctx) return LB_ERR_ARG;
  ctx->timing = on != 0;
  return LB_OK;
}

lb_status lb_get_timing(lb_ctx* ctx, double out[4]) {
  if (!ctx || !out) return LB_ERR_ARG;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  double step_ms = ctx->acc_step, lb_ms = ctx->acc_lb, ch_ms = ctx->acc_ch;
  int n_step = ctx->acc_step_n;
  const int n_ev = ctx->ev_used / 3;
  for (int k = 0; k < n_ev; k++) {
    float a = 0, b = 0, c = 0;
    HIPCHK(hipEventElapsedTime(&a, ctx->ev[3 * k], ctx->ev[3 * k + 1]));
    HIPCHK(hipEventElapsedTime(&b, ctx->ev[3 * k + 1], ctx->ev[3 * k + 2]));
    ch_ms += a;
    lb_ms += b;
    if (k + 1 < n_ev) {
      HIPCHK(hipEventElapsedTime(&c, ctx->ev[3 * k], ctx->ev[3 * (k + 1)]));
      step_ms += c;
      n_step++;
    }
  }
  const int n = n_ev + ctx->acc_n;
  double bytes = 0;
  for (auto& b : ctx->bx) bytes += 2.0 * Q * store_bytes(ctx->S) * (double)b.interior;
  out[0] = n_step > 0 ? step_ms / n_step : (n ? (ch_ms + lb_ms) / n : 0);
  out[1] = n ? lb_ms / n : 0;
  out[2] = (n && (!ctx->ch.empty() || ctx->n_xf_items > 0)) ? ch_ms / n : 0;
  out[3] = bytes;
  return LB_OK;
}

lb_status lb_autotune(lb_ctx* ctx, int32_t trials) {
  if (!ctx || trials < 1) return LB_ERR_ARG;
  if (ctx->latched) return ctx->latched;
  if (ctx->aa)  // its trial launches rely on a step that leaves its input buffer intact
    return fail(ctx, LB_ERR_STATE, "the autotuner needs two population buffers (streaming LB_STREAM_AB)");
  lb_status s = prepare(ctx);
  if (s) return s;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // a candidate's time: the median of `samples` single launches (one warm-up
  // launch first), each between its own pair of events
  const int samples = std::max(7, (int)trials);
  auto time_now = [&](double* ms) -> lb_status {
    LbArgs a = make_args(ctx, 0, 0, 0);
    if (ctx->n_xf_items) launch_xface(ctx, ctx->stream, a);  // x-face velocities of this step
    ctx->lb_fn(dim3(ctx->grid), ctx->stream, a);  // warm-up
    std::vector<double> t(samples);
    for (int k = 0; k < samples; k++) {
      HIPCHK(hipEventRecord(e0, ctx->stream));
      ctx->lb_fn(dim3(ctx->grid), ctx->stream, a);
      HIPCHK(hipEventRecord(e1, ctx->stream));
      HIPCHK(hipEventSynchronize(e1));
      float f = 0;
      HIPCHK(hipEventElapsedTime(&f, e0, e1));
      t[k] = f;
    }
    std::sort(t.begin(), t.end());
    *ms = t[samples / 2];
    return LB_OK;
  };
  // Coordinate descent over box-size classes, then over the persistent grid
  // size.  Every candidate of a class is timed; the best two are then timed
  // again in alternation (three rounds) and the lower total wins, so one
  // noisy sample does not decide.  Row boxes try the workgroup iterations per
  // item and the lane-vector widths (2 or 3 words) that divide their rows.
  std::map<std::string, std::vector<int>> classes;
  for (size_t i = 0; i < ctx->bx.size(); i++) classes[box_key(ctx, ctx->bx[i])].push_back((int)i);
  using Cand = std::array<int, 4>;  // ex, ey, ez, vw
  auto apply = [&](const std::vector<int>& members, const Cand& c) -> lb_status {
    bool vw_changed = false;
    for (int i : members) {
      BoxHost& b = ctx->bx[i];
      b.ex = c[0];
      b.ey = c[1];
      b.ez = c[2];
      if (b.vec && b.vw != c[3]) {
        b.vw = c[3];
        vw_changed = true;
      }
    }
    if (vw_changed) {
      lb_status r = upload_boxes(ctx);
      if (r) return r;
    }
    return build_tables(ctx, 0);
  };
  auto pick_two = [&](const std::vector<double>& ms, int& i1, int& i2) {
    i1 = i2 = -1;
    for (int k = 0; k < (int)ms.size(); k++) {
      if (i1 < 0 || ms[k] < ms[i1]) {
        i2 = i1;
        i1 = k;
      } else if (i2 < 0 || ms[k] < ms[i2]) {
        i2 = k;
      }
    }
  };
  s = build_tables(ctx, 0);
  if (s) return s;
  for (auto& kv : classes) {
    BoxHost& ref = ctx->bx[kv.second[0]];
    std::vector<Cand> cands;
    std::vector<int> exs;
    if (ref.vec) {  // row boxes: workgroup iterations per item (ez) and lane-vector width
      for (int w : {2, 3}) {
        const int V = row_nodes(ctx->S, w);
        if (ref.dim.nx % V != 0 || ref.dim.nx < 2 * V) continue;
        // the 32-bit offsets of a workgroup iteration's planes (as lb_init checks)
        const double plane = (double)Q * ref.dim.nx * ref.dim.ny * (double)store_bytes(ctx->S);
        const double span = (WG / ((double)(ref.dim.nx / V) * (ref.dim.ny - 2)) + 4.0) * plane;
        if (span >= 2147483648.0) continue;
        for (int ez : {2, 4, 8, 16, 32, 64}) cands.push_back({ref.ex, ref.ey, ez, w});
      }
    } else {
      for (int ex : {ref.ix, 32, 64, 128, 256})
        if (ex >= 1 && ex <= ref.ix && std::find(exs.begin(), exs.end(), ex) == exs.end())
          exs.push_back(ex);
    }
    for (int ex : exs)
      for (int pl : {256, 512, 1024}) {
        int ey = std::max(1, std::min(ref.iy, pl / ex));
        if (ex * ey > WG * MAX_SLOTS) continue;
        for (int ez : {1, 2, 4, 8, 16}) {
          if (ez > ref.iz) continue;
          cands.push_back({ex, ey, ez, ref.vw});
        }
      }
    if (cands.empty()) continue;
    std::vector<double> ms(cands.size());
    for (size_t k = 0; k < cands.size(); k++) {
      s = apply(kv.second, cands[k]);
      if (s) return s;
      s = time_now(&ms[k]);
      if (s) return s;
    }
    int i1, i2;
    pick_two(ms, i1, i2);
    int win = i1;
    if (i2 >= 0) {
      double t1 = 0, t2 = 0;
      for (int r = 0; r < 3; r++) {
        double m;
        s = apply(kv.second, cands[i1]);
        if (s) return s;
        s = time_now(&m);
        if (s) return s;
        t1 += m;
        s = apply(kv.second, cands[i2]);
        if (s) return s;
        s = time_now(&m);
        if (s) return s;
        t2 += m;
      }
      win = t2 < t1 ? i2 : i1;
    }
    s = apply(kv.second, cands[win]);
    if (s) return s;
  }
  std::vector<int> grids = {0};
  for (int g : {2048, 4096, 8192, 16384})
    if (g < ctx->n_entries) grids.push_back(g);
  std::vector<double> gms(grids.size());
  std::vector<int> gsz(grids.size());
  for (size_t k = 0; k < grids.size(); k++) {
    s = build_tables(ctx, grids[k]);
    if (s) return s;
    gsz[k] = ctx->grid;
    s = time_now(&gms[k]);
    if (s) return s;
  }
  int g1, g2;
  pick_two(gms, g1, g2);
  int gwin = g1;
  if (g2 >= 0) {
    double t1 = 0, t2 = 0;
    for (int r = 0; r < 3; r++) {
      double m;
      s = build_tables(ctx, grids[g1]);
      if (s) return s;
      s = time_now(&m);
      if (s) return s;
      t1 += m;
      s = build_tables(ctx, grids[g2]);
      if (s) return s;
      s = time_now(&m);
      if (s) return s;
      t2 += m;
    }
    gwin = t2 < t1 ? g2 : g1;
  }
  s = build_tables(ctx, grids[gwin]);
  if (s) return s;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (ctx->cfg.tune_cache) {
    std::ofstream o(ctx->cfg.tune_cache, std::ios::app);
    for (auto& kv : classes) {
      const BoxHost& b = ctx->bx[kv.second[0]];
      o << "{\"key\": \"" << kv.first << "\", \"ex\": " << b.ex << ", \"ey\": " << b.ey
        << ", \"ez\": " << b.ez << ", \"vw\": " << b.vw << "}\n";
    }
    o << "{\"key\": \"" << grid_key(ctx) << "\", \"grid\": " << ctx->grid << "}\n";
  }
  return LB_OK;
}

lb_status lb_copy_probe(size_t bytes, int32_t iters, double* gbs) {
  if (!gbs || iters < 1 || bytes < 16) return LB_ERR_ARG;
  const size_t n = bytes / 16;
  void *a = nullptr, *b = nullptr;
  if (hipMalloc(&a, n * 16) != hipSuccess) return LB_ERR_OOM;
  if (hipMalloc(&b, n * 16) != hipSuccess) {
    (void)hipFree(a);
    return LB_ERR_OOM;
  }
  hipEvent_t e0, e1;
  lb_status st = LB_OK;
  if (hipMemset(a, 0, n * 16) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    st = LB_ERR_HIP;
  } else {
    // 256 KiB per workgroup: the fastest of the copy shapes measured (grid
    // strides and chunks of 64 KiB .. 1 MiB)
    const size_t per_block = 16384;
    const int grid = (int)std::min<size_t>((n + per_block - 1) / per_block, 1u << 30);
    const size_t nn = std::min(n, (size_t)grid * per_block);
    hipLaunchKernelGGL(k_copy, dim3(grid), dim3(WG), 0, nullptr, (const uint4*)a, (uint4*)b, nn, per_block);
    (void)hipEventRecord(e0, nullptr);
    for (int k = 0; k < iters; k++)
      hipLaunchKernelGGL(k_copy, dim3(grid), dim3(WG), 0, nullptr, (const uint4*)a, (uint4*)b, nn, per_block);
    (void)hipEventRecord(e1, nullptr);
    float ms = 0;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      st = LB_ERR_HIP;
    else
      *gbs = 2.0 * (double)nn * 16.0 * iters / (ms * 1e-3) / 1e9;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  (void)hipFree(a);
  (void)hipFree(b);
  return st;
}

lb_status lb_memcpy_probe(size_t bytes, int32_t iters, double* gbs) {
  if (!gbs || iters < 1 || bytes < 16) return LB_ERR_ARG;
  void *a = nullptr, *b = nullptr;
  if (hipMalloc(&a, bytes) != hipSuccess) return LB_ERR_OOM;
  if (hipMalloc(&b, bytes) != hipSuccess) {
    (void)hipFree(a);
    return LB_ERR_OOM;
  }
  hipEvent_t e0, e1;
  lb_status st = LB_OK;
  if (hipMemset(a, 0, bytes) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    st = LB_ERR_HIP;
  } else {
    bool ok = hipMemcpyAsync(b, a, bytes, hipMemcpyDeviceToDevice, nullptr) == hipSuccess;
    ok = ok && hipEventRecord(e0, nullptr) == hipSuccess;
    for (int k = 0; ok && k < iters; k++)
      ok = hipMemcpyAsync(b, a, bytes, hipMemcpyDeviceToDevice, nullptr) == hipSuccess;
    ok = ok && hipEventRecord(e1, nullptr) == hipSuccess;
    float ms = 0;
    if (!ok || hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      st = LB_ERR_HIP;
    else
      *gbs = 2.0 * (double)bytes * iters / (ms * 1e-3) / 1e9;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  (void)hipFree(a);
  (void)hipFree(b);
  return st;
}

const char* lb_describe(const lb_ctx* ctx) { return ctx ? ctx->desc.c_str() : ""; }

const char* lb_last_error(const lb_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void lb_free(lb_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  drop_graph(ctx);
  free_tables(ctx);
  for (auto& b : ctx->bx) {
    dfree(ctx, b.d_bc);
    dfree(ctx, b.d_body);
  }
  if (ctx->arena[1] == ctx->arena[0]) ctx->arena[1] = nullptr;
  dfree(ctx, ctx->arena[0]);
  dfree(ctx, ctx->arena[1]);
  dfree(ctx, ctx->d_boxes);
  dfree(ctx, ctx->d_mass_mom);
  dfree(ctx, ctx->d_xface);
  dfree(ctx, ctx->d_xf_items);
  dfree(ctx, ctx->d_st);
  dfree(ctx, ctx->d_chains);
  dfree(ctx, ctx->d_pos);
  dfree(ctx, ctx->d_vel);
  dfree(ctx, ctx->d_rec_base);
  dfree(ctx, ctx->d_rec_d);
  dfree(ctx, ctx->d_rec_dp);
  dfree(ctx, ctx->d_bbox);
  for (auto e : ctx->ev) (void)hipEventDestroy(e);
  drop_stamps(ctx);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  delete ctx;
}

}  // extern "C"
