// C ABI of the CADMM sweep library: argument checks, device buffers, the tile
// planner, launch sequencing (optionally replayed as hipGraphs), the tile
// autotuner and the output queries.  See include/top.h for the contract.
#include "top.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "adjoint_impl.h"
#include "api_internal.h"
#include "common.h"

namespace {

thread_local std::string g_err = "";

constexpr size_t kWsAlign = 256;  // alignment of every buffer carved from a caller's workspace

top_status fail(top_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define TOP_HIP(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return fail(TOP_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// SIMDs of the current device (four per compute unit), or 1024 if the runtime does not say.
int device_simds() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      cus > 0)
    return 4 * cus;
  return 1024;
}

int max_tile(const top::Variant& v) {
  if (v.num) return 64;
  if (v.faces) return (v.prec == 0 && v.p == 3) ? 512 : 256;  // the polytope kernel's LDS-matrix instance
  return (v.prec == 0 && v.p == 3 && v.s != 2 * v.p - 1) ? 512 : 256;
}
// Handles that keep a tape also run the adjoint kernel on the same tiles: it is built for tiles of up
// to top::adjoint_max_tile segments (three lanes each), and its LDS must fit the device's
// per-workgroup LDS.
int max_tile(const top::Variant& v, bool taped) {
  if (!taped) return max_tile(v);
  int lds = 65536;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int q = 0;
    if (hipDeviceGetAttribute(&q, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && q > 0) lds = q;
  }
  const size_t rsz = v.prec == 0 ? 4 : 8;
  // the kernel's LDS rows are strided by its largest tile, whatever the launch's W
  if (top::adjoint_lds_bytes(v, rsz, top::adjoint_max_tile(v.prec)) + top::kAdjointStaticLds > (size_t)lds) return 0;
  return std::min(top::adjoint_max_tile(v.prec), max_tile(v));
}

// Whether the sweep of this variant and these options can run one lane per segment and axis.
// (NumericSolve takes it as four lanes per segment: three axes and a spare.)
static bool axis_allowed(const top::Variant& v, const top_options& opt) {
  return !v.faces && v.s != 2 * v.p - 1 && opt.checkpoint_every == 0 && opt.check_every == 0;
}
// The tail launch of a plan (see make_plan): the tiles of one round, the tail tile width, its form.
struct TailSpec {
  int round = 0, W = 0, form = 0;
};

// Largest tile (segments) of that form.
static int axis_tile_max(const top::Variant& v) {
  return v.num ? top::num_quad_max_tile(v.prec) : top::axis_max_tile(v.prec);
}
// The tail of a plan of W-segment tiles in lane form `form` (see make_plan), or none (one lane per
// segment and axis already, NumericSolve, a tape, residual checks, or the runtime does not say how
// many tiles the device holds): the lane-per-axis kernel where it takes the variant, with tiles of
// up to its maximum; else the main kernel itself with tiles of at most W / 2 segments (half the
// waves).  With checks every launch covers only the sweeps up to the next check, and a tail launch
// after each cost more than the round it saves (adaptive batched solve: 8.4 against 7.7 ms).
static TailSpec tail_spec(const top::Variant& v, const top_options& opt, int W, int form) {
  TailSpec t;
  if (form != 1 || v.num || opt.checkpoint_every > 0 || opt.check_every > 0) return t;
  const int r = v.faces ? (v.prec == 0 ? top::poly_resident<float>(v, W) : top::poly_resident<double>(v, W))
                        : (v.prec == 0 ? top::sweep_resident<float>(v, W) : top::sweep_resident<double>(v, W));
  if (r <= 0) return t;
  t.round = r;
  if (axis_allowed(v, opt)) {
    t.W = top::axis_max_tile(v.prec);
    t.form = 3;
  } else {
    t.W = W / 2 >= 64 ? W / 2 / 64 * 64 : 0;
    t.form = 1;
    if (t.W == 0) t.round = 0;
  }
  return t;
}

struct Plan {
  int W = 0;
  int n_tiles = 0;
  int halo = 0;          // > 0 when some trajectory is split across tiles
  int64_t used = 0;
  std::vector<int32_t> lanes;
  // Chained launches (several halo epochs in one launch): per tile the left / right tile whose core
  // holds its halo copies (-1: none) and its core lane range [lo, hi); empty when the plan has no
  // halo or its tiles do not meet the conditions (checked by chain_table).
  std::vector<int32_t> chain;
  // Tail launch: when the tiles make a last round that holds only a few of them, the trajectories of
  // those tiles run in a second launch after the main one, one lane per segment and axis, in tiles
  // of tail_W segments (segment of each lane, -1 idle), instead of taking a whole round of the main
  // kernel's time (see make_plan).  Empty: no tail.
  int tail_W = 0, tail_tiles = 0;
  int tail_form = 0;   // 3: one lane per segment and axis; 1: the main kernel's own form, smaller tiles
  std::vector<int32_t> tail;
  size_t table_elems() const { return lanes.size() + chain.size() + tail.size(); }
  size_t tail_offset() const { return lanes.size() + chain.size(); }
};

// The chain table of a plan with halo tiles (see Plan::chain), or empty.  A chained epoch relies
// on every halo copy, and the start knot of every halo copy's segment, being published by a
// neighbouring tile: the core segments within `halo` of a core edge that has a neighbour, plus one
// more on the right.  The table is built from the tiles' core ranges and then checked against that
// rule lane by lane.
std::vector<int32_t> chain_table(const Plan& pl, const std::vector<int64_t>& off) {
  std::vector<int32_t> ch;
  const int W = pl.W, h = pl.halo;
  if (h <= 0 || pl.n_tiles <= 0) return ch;
  const int64_t S = off.back();
  ch.assign(4 * (size_t)pl.n_tiles, 0);
  std::vector<int32_t> owner((size_t)S, -1), owner_lane((size_t)S, -1);
  for (int t = 0; t < pl.n_tiles; ++t) {
    const int32_t* L = pl.lanes.data() + (size_t)t * W;
    int lo = -1, hi = -1;
    for (int i = 0; i < W; ++i) {
      if (L[i] < 0 || (L[i] & top::kHaloBit)) continue;
      if (lo < 0) lo = i;
      hi = i + 1;
      owner[L[i] & top::kSegMask] = t;
      owner_lane[L[i] & top::kSegMask] = i;
    }
    const bool left = W > 0 && L[0] >= 0 && (L[0] & top::kHaloBit);
    bool right = false;
    for (int i = W - 1; i >= 0; --i)
      if (L[i] >= 0) { right = (L[i] & top::kHaloBit) != 0; break; }
    int32_t* c = ch.data() + 4 * (size_t)t;
    c[0] = left ? t - 1 : -1;
    c[1] = right ? t + 1 : -1;
    c[2] = lo < 0 ? 0 : lo;
    c[3] = hi < 0 ? 0 : hi;
  }
  // whether tile t publishes segment s (its core lane i) at the end of an epoch
  auto published = [&](int64_t s) {
    const int t = owner[(size_t)s], i = owner_lane[(size_t)s];
    if (t < 0) return false;
    const int32_t* c = ch.data() + 4 * (size_t)t;
    return (c[0] >= 0 && i < c[2] + h) || (c[1] >= 0 && i >= c[3] - h - 1);
  };
  std::vector<uint8_t> first((size_t)S, 0);
  for (size_t b = 0; b + 1 < off.size(); ++b) first[(size_t)off[b]] = 1;
  for (int t = 0; t < pl.n_tiles; ++t) {
    const int32_t* L = pl.lanes.data() + (size_t)t * W;
    const int32_t* c = ch.data() + 4 * (size_t)t;
    for (int i = 0; i < W; ++i) {
      if (L[i] < 0 || !(L[i] & top::kHaloBit)) continue;
      const int64_t s = L[i] & top::kSegMask;
      const int dep = i < c[2] ? c[0] : c[1];
      if (dep < 0 || owner[(size_t)s] != dep || !published(s)) return {};
      // a copy reloads its start knot as the end knot of the segment before it, which must be
      // published too (by this tile or a neighbour)
      if (!first[(size_t)s]) {
        const int o = owner[(size_t)(s - 1)];
        if ((o != c[0] && o != c[1] && o != t) || !published(s - 1)) return {};
      }
    }
  }
  return ch;
}

// Trajectories `items` packed into bins of `cap` segments, first-fit in decreasing length (ties
// in index order).
static std::vector<std::vector<int>> pack_ffd(std::vector<int> items, const std::vector<int64_t>& off, int cap) {
  std::stable_sort(items.begin(), items.end(), [&](int x, int y) {
    return (off[x + 1] - off[x]) > (off[y + 1] - off[y]);
  });
  std::vector<int> fill;
  std::vector<std::vector<int>> bins;
  int first_open = 0;  // bins before this index are full to within the smallest length seen
  for (int b : items) {
    const int len = (int)(off[b + 1] - off[b]);
    int k = -1;
    for (int i = first_open; i < (int)bins.size(); ++i)
      if (fill[i] + len <= cap) { k = i; break; }
    if (k < 0) {
      k = (int)bins.size();
      bins.emplace_back();
      fill.push_back(0);
    }
    bins[k].push_back(b);
    fill[k] += len;
    while (first_open < (int)bins.size() && fill[first_open] == cap) ++first_open;
  }
  return bins;
}

// Pack whole trajectories of at most W segments into W-lane tiles (first-fit decreasing); split
// longer ones into tiles whose cores are flanked by up to `halo` copied neighbours.
//
// Tail: tiles run in rounds of `round` (the tiles the device holds at once), each round taking about
// the same time whatever it holds.  When nothing is split and the last round would hold only a few
// tiles (k, at most an eighth of a round), the trajectories of k tiles go to a tail plan instead:
// the k whose longest trajectory is shortest (then the least filled), repacked into tiles as wide as
// that longest trajectory rounded up to 64 (at most tail_W), which spread over the CUs with fewer
// waves each and finish in a fraction of a round (round = 0: no tail).  tail_form says which kernel
// runs them (3: one lane per segment and axis; 1: the main kernel with the narrower tiles).
Plan make_plan(const std::vector<int64_t>& off, int W, int halo, int round, int tail_W, int tail_form) {
  Plan pl;
  pl.W = W;
  const int B = (int)off.size() - 1;
  std::vector<int> shorts, longs;
  for (int b = 0; b < B; ++b) ((off[b + 1] - off[b]) <= W ? shorts : longs).push_back(b);
  std::vector<std::vector<int>> bins = pack_ffd(shorts, off, W);
  std::vector<int> tail_items;
  int tail_w = 0;
  if (longs.empty() && round > 0 && tail_W > 0 && (int)bins.size() > round) {
    const int k = (int)bins.size() % round;
    if (k > 0 && 8 * k <= round) {
      std::vector<int> order(bins.size());
      std::vector<int64_t> longest(bins.size(), 0), fill(bins.size(), 0);
      for (size_t i = 0; i < bins.size(); ++i) {
        order[i] = (int)i;
        for (int b : bins[i]) {
          longest[i] = std::max(longest[i], off[b + 1] - off[b]);
          fill[i] += off[b + 1] - off[b];
        }
      }
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return longest[x] != longest[y] ? longest[x] < longest[y] : fill[x] < fill[y];
      });
      int64_t tl = 0;
      for (int j = 0; j < k; ++j) tl = std::max(tl, longest[order[j]]);
      if (tl <= tail_W) {
        tail_w = (int)((tl + 63) / 64 * 64);
        std::vector<char> moved(bins.size(), 0);
        for (int j = 0; j < k; ++j) moved[order[j]] = 1;
        std::vector<std::vector<int>> kept;
        for (size_t i = 0; i < bins.size(); ++i) {
          if (moved[i]) tail_items.insert(tail_items.end(), bins[i].begin(), bins[i].end());
          else kept.push_back(std::move(bins[i]));
        }
        bins = std::move(kept);
      }
    }
  }
  for (size_t i = 0; i < bins.size(); ++i) {
    std::vector<int32_t> t(W, -1);
    int pos = 0;
    for (int b : bins[i])
      for (int64_t s = off[b]; s < off[b + 1]; ++s) t[pos++] = (int32_t)s;
    pl.used += pos;
    pl.lanes.insert(pl.lanes.end(), t.begin(), t.end());
  }
  if (!tail_items.empty()) {
    for (const std::vector<int>& bin : pack_ffd(tail_items, off, tail_w)) {
      std::vector<int32_t> t(tail_w, -1);
      int pos = 0;
      for (int b : bin)
        for (int64_t s = off[b]; s < off[b + 1]; ++s) t[pos++] = (int32_t)s;
      pl.used += pos;
      pl.tail.insert(pl.tail.end(), t.begin(), t.end());
    }
    pl.tail_W = tail_w;
    pl.tail_tiles = (int)(pl.tail.size() / tail_w);
    pl.tail_form = tail_form;
  }
  if (!longs.empty()) pl.halo = halo;
  for (int b : longs) {
    const int64_t N = off[b + 1] - off[b];
    int64_t c0 = 0;
    while (c0 < N) {
      const int64_t left = c0 > 0 ? halo : 0;
      int64_t c1;
      if (c0 - left + W >= N) c1 = N;
      else c1 = c0 + W - left - halo;
      const int64_t l0 = c0 - left, l1 = std::min<int64_t>(N, c1 + halo);
      std::vector<int32_t> t(W, -1);
      for (int64_t s = l0; s < l1; ++s) {
        const int64_t seg = off[b] + s;
        t[s - l0] = (int32_t)seg | ((s < c0 || s >= c1) ? top::kHaloBit : 0);
      }
      pl.used += l1 - l0;
      pl.lanes.insert(pl.lanes.end(), t.begin(), t.end());
      c0 = c1;
    }
  }
  pl.n_tiles = (int)(pl.lanes.size() / W);
  pl.chain = chain_table(pl, off);
  return pl;
}

// Shape class of a problem for the tuning cache.
std::string shape_key(const top::Variant& v, const std::vector<int64_t>& off) {
  int64_t mx = 0;
  for (size_t b = 0; b + 1 < off.size(); ++b) mx = std::max(mx, off[b + 1] - off[b]);
  const int64_t S = off.back();
  auto lg = [](int64_t x) { int r = 0; while (x > 1) { x >>= 1; ++r; } return r; };
  char buf[128];
  snprintf(buf, sizeof buf, "v2:prec%d:p%d:s%d:box%d:vel%d:logS%d:logmax%d", v.prec, v.p, v.s, v.box,
           v.vel, lg(S), lg(mx));
  return buf;
}

struct TuneChoice {
  int W = 0, halo = 0, form = 1;   // tile width, halo, lanes per segment
};
std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune;  // shape class -> tuned plan
bool g_tune_loaded = false;

void tune_cache_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("TOP_TUNE_CACHE");
  if (path == nullptr) return;
  FILE* f = std::fopen(path, "r");
  if (f == nullptr) return;
  char key[160];
  int W, h, form;
  while (std::fscanf(f, "%159s %d %d %d", key, &W, &h, &form) == 4) g_tune[key] = TuneChoice{W, h, form};
  std::fclose(f);
}

void tune_cache_store() {
  const char* path = std::getenv("TOP_TUNE_CACHE");
  if (path == nullptr) return;
  FILE* f = std::fopen(path, "w");
  if (f == nullptr) return;
  for (auto& kv : g_tune)
    std::fprintf(f, "%s %d %d %d\n", kv.first.c_str(), kv.second.W, kv.second.halo, kv.second.form);
  std::fclose(f);
}

// ---- device memory pool: blocks released by top_destroy are kept per (device, size class) and
// handed to the next handle that asks for the same size class, so repeated problems of one shape
// do not call hipMalloc/hipFree.  top_destroy does not wait for the handle's queued work: each
// released block carries the stream it was last used on and an event recorded there at release.
// A handle on the same stream reuses it at once (stream order puts its work after the old work);
// a handle on another stream first makes its stream wait for that event.
size_t size_class(size_t b) {
  const size_t g = b < (size_t(2) << 20) ? size_t(4096) : (size_t(2) << 20);
  return (b + g - 1) / g * g;
}

struct ReleaseEvent {  // shared by the blocks of one released handle
  hipEvent_t ev = nullptr;
  ~ReleaseEvent() {
    if (ev != nullptr) (void)hipEventDestroy(ev);
  }
};

struct PoolBlock {
  void* p;
  hipStream_t stream;                   // last used on this stream
  std::shared_ptr<ReleaseEvent> done;   // recorded there at release; null: no pending work
};

struct Pool {
  std::mutex mu;
  std::multimap<std::pair<int, size_t>, PoolBlock> blocks;
  size_t cached = 0;
  size_t cap() const {
    const char* e = std::getenv("TOP_POOL_MAX_BYTES");
    return e != nullptr ? std::strtoull(e, nullptr, 10) : (size_t(64) << 30);
  }
};
Pool g_pool;

hipError_t pool_get(size_t bytes, hipStream_t stream, void** out, int* dev_out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const size_t sc = size_class(bytes);
  *dev_out = dev;
  PoolBlock blk{nullptr, nullptr, nullptr};
  {
    std::lock_guard<std::mutex> lk(g_pool.mu);
    auto range = g_pool.blocks.equal_range({dev, sc});
    auto pick = range.first;
    for (auto it = range.first; it != range.second; ++it)
      if (it->second.stream == stream) { pick = it; break; }   // prefer a block of this stream
    if (pick != range.second) {
      blk = pick->second;
      g_pool.blocks.erase(pick);
      g_pool.cached -= sc;
    }
  }
  if (blk.p == nullptr) return hipMalloc(out, sc);
  if (blk.done && blk.stream != stream) {
    e = hipStreamWaitEvent(stream, blk.done->ev, 0);
    if (e != hipSuccess) {
      std::lock_guard<std::mutex> lk(g_pool.mu);
      g_pool.blocks.insert({{dev, sc}, blk});
      g_pool.cached += sc;
      return e;
    }
  }
  *out = blk.p;
  return hipSuccess;
}

void pool_put(void* p, size_t bytes, int dev, hipStream_t stream, const std::shared_ptr<ReleaseEvent>& done) {
  const size_t sc = size_class(bytes);
  std::lock_guard<std::mutex> lk(g_pool.mu);
  if (g_pool.cached + sc > g_pool.cap()) {
    (void)hipFree(p);  // hipFree waits for the device's queued work
    return;
  }
  g_pool.blocks.insert({{dev, sc}, PoolBlock{p, stream, done}});
  g_pool.cached += sc;
}

// ---- plan cache: the packed lane map of a CSR shape, on the device, shared by every handle of
// that shape (immutable once built).
struct PlanEntry {
  Plan plan;
  std::vector<int64_t> off;
  int device = 0;
  int32_t* dev = nullptr;
  ~PlanEntry() {
    if (dev != nullptr) (void)hipFree(dev);
  }
};

std::mutex g_plan_mu;
// Never destroyed: entries free device memory, which must not happen after the HIP runtime has
// shut down at process exit.
std::map<uint64_t, std::shared_ptr<PlanEntry>>& g_plans = *new std::map<uint64_t, std::shared_ptr<PlanEntry>>();

// Hash of the offsets and shape parameters (64-bit words folded in with a multiply-xorshift mix; the
// caches compare the offsets themselves on a hit, so collisions only cost a rebuild).
uint64_t offsets_hash(const std::vector<int64_t>& off, std::initializer_list<int64_t> extra) {
  uint64_t h = 0x9e3779b97f4a7c15ull;
  auto mix = [&](uint64_t v) {
    h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 33;
  };
  for (int64_t o : off) mix((uint64_t)o);
  for (int64_t x : extra) mix((uint64_t)x);
  return h;
}

uint64_t plan_key(const std::vector<int64_t>& off, int W, int halo, int round, int tail_W, int tail_form,
                  int device) {
  return offsets_hash(off, {W, halo, round, tail_W, tail_form, device});
}

// Copy the tables of plan pl (lane map, chain table, tail lane map) to dst, in that order.
hipError_t upload_plan(const Plan& pl, int32_t* dst, hipStream_t st, bool async) {
  auto put = [&](size_t at, const std::vector<int32_t>& v) -> hipError_t {
    if (v.empty()) return hipSuccess;
    return async ? hipMemcpyAsync(dst + at, v.data(), v.size() * sizeof(int32_t), hipMemcpyHostToDevice, st)
                 : hipMemcpy(dst + at, v.data(), v.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  };
  hipError_t e = put(0, pl.lanes);
  if (e == hipSuccess) e = put(pl.lanes.size(), pl.chain);
  if (e == hipSuccess) e = put(pl.tail_offset(), pl.tail);
  return e;
}

// The cached plan of this shape, building and uploading it on first use (the tail: see make_plan).
top_status get_plan(const std::vector<int64_t>& off, int W, int halo, const TailSpec& ts,
                    std::shared_ptr<PlanEntry>* out) {
  int dev = 0;
  TOP_HIP(hipGetDevice(&dev));
  const uint64_t key = plan_key(off, W, halo, ts.round, ts.W, ts.form, dev);
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end() && it->second->off == off && it->second->plan.W == W) {
      *out = it->second;
      return TOP_OK;
    }
  }
  auto e = std::make_shared<PlanEntry>();
  e->plan = make_plan(off, W, halo, ts.round, ts.W, ts.form);
  e->off = off;
  e->device = dev;
  const size_t bytes = e->plan.table_elems() * sizeof(int32_t);
  void* q = nullptr;
  hipError_t he = hipMalloc(&q, bytes);
  if (he != hipSuccess) return fail(TOP_E_NOMEM, "hipMalloc(%zu) for the lane map failed", bytes);
  e->dev = static_cast<int32_t*>(q);
  he = upload_plan(e->plan, e->dev, nullptr, false);
  if (he != hipSuccess) return fail(TOP_E_HIP, "lane map upload failed: %s", hipGetErrorString(he));
  std::lock_guard<std::mutex> lk(g_plan_mu);
  // keep at most 16 shapes; drop the ones no handle uses any more
  if (g_plans.size() >= 16) {
    for (auto it = g_plans.begin(); it != g_plans.end();) {
      if (it->second.use_count() == 1) it = g_plans.erase(it); else ++it;
    }
  }
  g_plans[key] = e;
  *out = e;
  return TOP_OK;
}

// ---- shape cache: the device copy of a CSR shape's offsets and the chunk tables of its
// per-trajectory reduction, shared (read-only) by every handle of that shape on a device.
struct ShapeEntry {
  std::vector<int64_t> off;
  int device = 0;
  int64_t* off_dev = nullptr;        // [B + 1]
  int32_t* chunk_off = nullptr;      // [B + 1] first reduction chunk of each trajectory
  int32_t* chunk_traj = nullptr;     // [n_chunks] trajectory of each chunk
  int n_chunks = 0;
  ~ShapeEntry() {
    for (void* q : {(void*)off_dev, (void*)chunk_off, (void*)chunk_traj})
      if (q != nullptr) (void)hipFree(q);
  }
};

// Reduction chunk tables of a CSR shape: first chunk of each trajectory, trajectory of each chunk.
void chunk_tables(const std::vector<int64_t>& off, std::vector<int32_t>* c_off, std::vector<int32_t>* c_traj) {
  const int B = (int)off.size() - 1;
  c_off->assign((size_t)B + 1, 0);
  c_traj->clear();
  for (int b = 0; b < B; ++b) {
    const int64_t nc = (off[b + 1] - off[b] + top::kReduceChunk - 1) / top::kReduceChunk;
    (*c_off)[b + 1] = (*c_off)[b] + (int32_t)nc;
    for (int64_t j = 0; j < nc; ++j) c_traj->push_back(b);
  }
}

std::mutex g_shape_mu;
std::map<uint64_t, std::shared_ptr<ShapeEntry>>& g_shapes = *new std::map<uint64_t, std::shared_ptr<ShapeEntry>>();

top_status get_shape(const std::vector<int64_t>& off, std::shared_ptr<ShapeEntry>* out) {
  int dev = 0;
  TOP_HIP(hipGetDevice(&dev));
  const uint64_t key = offsets_hash(off, {dev});
  {
    std::lock_guard<std::mutex> lk(g_shape_mu);
    auto it = g_shapes.find(key);
    if (it != g_shapes.end() && it->second->device == dev && it->second->off == off) {
      *out = it->second;
      return TOP_OK;
    }
  }
  auto e = std::make_shared<ShapeEntry>();
  e->off = off;
  e->device = dev;
  std::vector<int32_t> c_off, c_traj;
  chunk_tables(off, &c_off, &c_traj);
  e->n_chunks = (int)c_traj.size();
  hipError_t he = hipMalloc((void**)&e->off_dev, off.size() * sizeof(int64_t));
  if (he == hipSuccess) he = hipMalloc((void**)&e->chunk_off, c_off.size() * sizeof(int32_t));
  if (he == hipSuccess) he = hipMalloc((void**)&e->chunk_traj, std::max<size_t>(c_traj.size(), 1) * sizeof(int32_t));
  if (he != hipSuccess) return fail(TOP_E_NOMEM, "device allocation for the shape tables failed");
  he = hipMemcpy(e->off_dev, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(e->chunk_off, c_off.data(), c_off.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (he == hipSuccess && !c_traj.empty())
    he = hipMemcpy(e->chunk_traj, c_traj.data(), c_traj.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (he != hipSuccess) return fail(TOP_E_HIP, "shape table upload failed: %s", hipGetErrorString(he));
  std::lock_guard<std::mutex> lk(g_shape_mu);
  if (g_shapes.size() >= 16) {  // keep at most 16 shapes; drop the ones no handle uses any more
    for (auto it = g_shapes.begin(); it != g_shapes.end();) {
      if (it->second.use_count() == 1) it = g_shapes.erase(it); else ++it;
    }
  }
  g_shapes[key] = e;
  *out = e;
  return TOP_OK;
}

// ---- per-device second stream (default priority) and events of the reverse pass, created on first
// use and kept for the process's lifetime.
struct ReverseAux {
  std::mutex mu;
  hipStream_t stream = nullptr;
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};
std::mutex g_aux_mu;
std::map<int, ReverseAux*>& g_aux = *new std::map<int, ReverseAux*>();

top_status reverse_aux(ReverseAux** out) {
  int dev = 0;
  TOP_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_aux_mu);
  ReverseAux*& a = g_aux[dev];
  if (a == nullptr) {
    auto* n = new ReverseAux();
    hipError_t e = hipStreamCreateWithFlags(&n->stream, hipStreamNonBlocking);
    for (int k = 0; k < 5 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&n->ev[k], hipEventDisableTiming);
    if (e != hipSuccess) {
      delete n;  // its stream and events are left to the process's end
      return fail(TOP_E_HIP, "reverse-pass stream setup failed: %s", hipGetErrorString(e));
    }
    a = n;
  }
  *out = a;
  return TOP_OK;
}

// ---- pinned host words for the validation flags, so create can read them back without blocking
// the launches queued behind the check.
std::mutex g_pin_mu;
int* g_pin = nullptr;
std::vector<int> g_pin_free;
constexpr int kPinSlots = 1024;  // two words each

int* pin_get() {
  std::lock_guard<std::mutex> lk(g_pin_mu);
  if (g_pin == nullptr) {
    if (hipHostMalloc((void**)&g_pin, 2 * kPinSlots * sizeof(int), hipHostMallocDefault) != hipSuccess) {
      g_pin = nullptr;
      return nullptr;
    }
    for (int k = kPinSlots - 1; k >= 0; --k) g_pin_free.push_back(k);
  }
  if (g_pin_free.empty()) return nullptr;
  const int k = g_pin_free.back();
  g_pin_free.pop_back();
  return g_pin + 2 * k;
}

void pin_put(int* p) {
  if (p == nullptr) return;
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pin_free.push_back((int)((p - g_pin) / 2));
}

}  // namespace

struct top_problem {
  top_options opt{};
  top::Variant v{};
  int B = 0;
  int64_t S = 0, ld = 0;
  int nf = 0;
  size_t rsz = 4;
  std::vector<int64_t> off;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  struct Block { void* p; size_t bytes; int dev; };
  std::vector<Block> allocs;           // pool blocks (handles without a caller workspace)
  // Caller workspace: buffers are carved from it in order, kWsAlign-aligned.  `sizing` only counts
  // the bytes (top_workspace_bytes), handing out placeholder pointers that are never dereferenced.
  char* ws = nullptr;
  size_t ws_cap = 0, ws_used = 0;
  bool sizing = false;
  // device buffers
  void *Hr = nullptr, *iT = nullptr, *lo = nullptr, *hi = nullptr, *vmax = nullptr, *bcL = nullptr;
  void *Urot = nullptr, *fa = nullptr;  // polytope corridor: rotation and faces
  double* lam = nullptr;                // polytope corridor: eigenvalues of sum_k a_k a_k^T
  void* state[2] = {nullptr, nullptr};
  void *cbuf = nullptr, *zold = nullptr;
  uint8_t* flags = nullptr;
  int32_t* traj = nullptr;
  double *Tdev = nullptr, *rho_seg = nullptr, *part = nullptr, *out = nullptr;
  std::shared_ptr<ShapeEntry> shape;   // device offsets and reduction chunk tables of this CSR shape
  const int64_t* off_dev = nullptr;
  int* flag_dev = nullptr;
  int* pin = nullptr;                // pinned host words receiving the input check's flags
  hipEvent_t ev_valid = nullptr;     // recorded after their readback
  const int32_t *chunk_traj = nullptr, *chunk_off = nullptr;
  int n_chunks = 0;
  int64_t max_len = 0;                 // segments of the longest trajectory
  double* chunk_sum = nullptr;
  top::ReduceArgs reduce_args() const {
    top::ReduceArgs a{};
    a.part = part;
    a.S = S;
    a.off = off_dev;
    a.B = B;
    a.chunk_traj = chunk_traj;
    a.chunk_off = chunk_off;
    a.n_chunks = n_chunks;
    a.chunk_sum = chunk_sum;
    a.out = out;
    a.done = opt.check_every > 0 ? done_dev : nullptr;
    return a;
  }
  std::shared_ptr<PlanEntry> pe;
  // A handle on the static scratch keeps its shape tables and lane map in its own workspace: the
  // host copies they are uploaded from, and the plan.
  bool own_tables = false;
  Plan own_plan;
  int32_t* own_lanes = nullptr;
  std::vector<int32_t> own_chunk_off, own_chunk_traj;
  const Plan& plan_ref() const { return pe ? pe->plan : own_plan; }
  const int32_t* lanes() const { return pe ? pe->dev : own_lanes; }

  // The shape tables and the lane map in the handle's workspace (own_tables), after its buffers.
  top_status allocate_tables(int64_t n_chunks, size_t n_lanes) {
    top_status st;
    if ((st = alloc(&off_dev, (size_t)(B + 1) * sizeof(int64_t))) != TOP_OK) return st;
    if ((st = alloc(&chunk_off, (size_t)(B + 1) * sizeof(int32_t))) != TOP_OK) return st;
    if ((st = alloc(&chunk_traj, (size_t)std::max<int64_t>(n_chunks, 1) * sizeof(int32_t))) != TOP_OK) return st;
    return alloc(&own_lanes, n_lanes * sizeof(int32_t));
  }
  int cur = 0;
  int iters_done = 0;
  bool have_sweep = false;
  bool init_cost_ready = false;  // out[0] holds the Init guess's cost (computed on first request)
  bool explicit_tile = false;
  bool axis = false;             // sweep launches run one lane per segment and axis
  bool axis_ok = false;          // the variant and options allow that form
  // tape: slot j holds the state before sweep j * checkpoint_every
  void* tape = nullptr;
  int tape_slots = 0;
  // reverse pass: T-derivative of rho Htilde^-1, float64 copies of the inputs, work buffers
  void* Hd = nullptr;
  double *wp64 = nullptr, *lo64 = nullptr, *hi64 = nullptr, *vmax64 = nullptr, *bc64 = nullptr;
  void *blk = nullptr, *adjb[2] = {nullptr, nullptr}, *acc_iT = nullptr, *acc_hd = nullptr, *acc_z0 = nullptr;
  // The forward records the states of the block holding the last sweep of each top_iterate call into
  // block buffer (block % 2), so the reverse pass need not replay that block: rec_block is the block,
  // rec_upto the number of leading states of it present (state 0 is the block's checkpoint).
  int rec_block = -1, rec_upto = 0;
  double *dPL = nullptr, *dPR = nullptr, *dK = nullptr, *dK0 = nullptr;
  // residual checks: per-trajectory stop flag, sweep counters, current rho and the last change
  uint8_t *done_dev = nullptr, *fresh = nullptr;
  int32_t *swept = nullptr, *stop_at = nullptr;
  double *rho_traj = nullptr, *ratio = nullptr;
  int32_t *check_lists = nullptr, *check_counts = nullptr;  // [3][B] and [3]: per-check work lists
  // launch sequences replayed as graphs, keyed by (sweeps, start buffer, sweep index mod check_every)
  std::map<std::tuple<int, int, int>, hipGraphExec_t> graphs;
  std::set<std::tuple<int, int, int>> graph_seen;  // sequences launched once directly
  std::vector<hipGraph_t> graph_defs;

  template <typename T>
  top_status alloc(T** p, size_t bytes) {
    void* q = nullptr;
    if (bytes == 0) bytes = 256;
    if (sizing || ws != nullptr) {
      const size_t need = (bytes + kWsAlign - 1) / kWsAlign * kWsAlign;
      if (sizing) {
        ws_used += need;
        *p = reinterpret_cast<T*>(uintptr_t(kWsAlign));
        return TOP_OK;
      }
      if (ws_used + need > ws_cap)
        return fail(TOP_E_WORKSPACE, "workspace of %zu bytes exhausted (%zu more needed)", ws_cap,
                    ws_used + need - ws_cap);
      *p = reinterpret_cast<T*>(ws + ws_used);
      ws_used += need;
      return TOP_OK;
    }
    int dev = 0;
    hipError_t e = pool_get(bytes, stream, &q, &dev);
    if (e != hipSuccess) return fail(TOP_E_NOMEM, "device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    allocs.push_back({q, bytes, dev});
    *p = reinterpret_cast<T*>(q);
    return TOP_OK;
  }

  void drop_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
    for (auto g : graph_defs) (void)hipGraphDestroy(g);
    graph_defs.clear();
  }

  template <typename R>
  top::SweepArgs<R> sweep_args(const Plan& pl, const int32_t* lane_map) const {
    top::SweepArgs<R> a{};
    a.k.Hr = (const R*)Hr;
    a.k.iT = (const R*)iT;
    a.k.lo = (const R*)lo;
    a.k.hi = (const R*)hi;
    a.k.vmax = (const R*)vmax;
    a.k.flags = flags;
    a.k.traj = traj;
    a.k.bcL = (const R*)bcL;
    a.k.U = (const R*)Urot;
    a.k.fa = (const R*)fa;
    a.k.rho = rho_seg;
    a.k.ld = ld;
    a.lane_seg = lane_map;
    a.W = pl.W;
    a.fixpos = opt.fix_interior;
    a.c_out = (R*)cbuf;
    a.zold_out = (R*)zold;
    a.done = opt.check_every > 0 ? done_dev : nullptr;
    return a;
  }

  // The lane form of launches over plan pl: the handle's, for its own plan (tuning probes pass
  // candidate plans and set probe_axis).
  bool probe_axis = false;
  const Plan* probe_plan = nullptr;
  bool axis_of(const Plan& pl) const { return &pl == probe_plan ? probe_axis : axis; }

  template <typename R>
  top_status launch_one(const Plan& pl, const int32_t* lane_map, const void* in, void* outp, int n, bool fin,
                        hipStream_t st, bool store_frozen, void* rec, bool chain) {
    top::SweepArgs<R> a = sweep_args<R>(pl, lane_map);
    a.st_in = (const R*)in;
    a.st_out = (R*)outp;
    a.iters = n;
    a.final_out = fin ? 1 : 0;
    a.store_frozen = store_frozen ? 1 : 0;
    a.inner = opt.lbfgs_iters;
    if (chain) {  // the epochs of n sweeps in one launch; both state buffers are written
      a.chain_halo = pl.halo;
      a.chain = lane_map + pl.lanes.size();
      a.chain_flag = chain_flag;
      a.chain_err = flag_dev + 2;
      a.chain_spin = chain_spin;
    }
    if (rec != nullptr) {  // recording launch: the state after sweep i < n - 1 goes to slot i + 1
      a.rec = (R*)rec;
      a.rec_slot = (int64_t)nf * ld;
    }
    hipError_t e = v.num     ? (axis_of(pl) ? top::launch_numeric_quad<R>(v, a, pl.n_tiles, st)
                                          : top::launch_numeric_sweep<R>(v, a, pl.n_tiles, st))
                 : v.faces ? top::launch_poly_sweep<R>(v, a, pl.n_tiles, st)
                 : (axis_of(pl) && rec == nullptr) ? top::launch_sweep_axis<R>(v, a, pl.n_tiles, st)
                           : top::launch_sweep<R>(v, a, pl.n_tiles, st);
    if (e == hipSuccess && pl.tail_tiles > 0) {
      // the tail's trajectories: the same sweeps, with one lane per segment and axis (where that
      // kernel takes the variant: no checks) or with the main kernel on the tail's narrower tiles
      if (rec != nullptr || chain || (pl.tail_form == 3 && a.done != nullptr))
        return fail(TOP_E_STATE, "this plan's tail launch cannot record, chain or check");
      top::SweepArgs<R> t = a;
      t.lane_seg = lane_map + pl.tail_offset();
      t.W = pl.tail_W;
      e = pl.tail_form == 3 ? top::launch_sweep_axis<R>(v, t, pl.tail_tiles, st)
        : v.faces           ? top::launch_poly_sweep<R>(v, t, pl.tail_tiles, st)
                            : top::launch_sweep<R>(v, t, pl.tail_tiles, st);
    }
    if (e != hipSuccess) return fail(TOP_E_HIP, "sweep launch failed: %s", hipGetErrorString(e));
    return TOP_OK;
  }

  top_status sweep_launch(const Plan& pl, const int32_t* lane_map, const void* in, void* outp, int n, bool fin,
                          hipStream_t st, bool store_frozen = false, void* rec = nullptr, bool chain = false) {
    return v.prec == 0 ? launch_one<float>(pl, lane_map, in, outp, n, fin, st, store_frozen, rec, chain)
                       : launch_one<double>(pl, lane_map, in, outp, n, fin, st, store_frozen, rec, chain);
  }

  // Chained launches (SweepArgs::chain_halo): the epoch flags, the tiles they cover, and the
  // device's co-resident tile count for the plan's tile width (cached).
  unsigned long long* chain_flag = nullptr;
  int64_t chain_cap = 0;
  int chain_spin = top::kChainSpin;
  int resident_W = 0, resident_tiles = 0;
  // Whether plan pl (in the lane form `axis_form`) may chain on this handle: option, lane form,
  // chain table, flag room, residency.
  bool plan_chains(const Plan& pl, bool axis_form) {
    if (opt.chain != 0 || !axis_form || pl.chain.empty() || tape != nullptr || opt.check_every > 0 || v.num ||
        v.faces)
      return false;
    if (pl.n_tiles > chain_cap) return false;
    if (resident_W != pl.W) {
      resident_tiles = v.prec == 0 ? top::sweep_axis_resident<float>(v, pl.W) : top::sweep_axis_resident<double>(v, pl.W);
      resident_W = pl.W;
    }
    return pl.n_tiles <= resident_tiles;
  }
  bool can_chain() { return plan_chains(plan_ref(), axis); }
  // k sweeps as one chained launch: more than one epoch on a plan that can chain
  // (each edge's 32-bit export count reaches epochs times up to 15 waves)
  bool chains(int k) { return chains(plan_ref(), axis, k); }
  bool chains(const Plan& pl, bool axis_form, int k) {
    const int h = pl.halo;
    return h > 0 && k > h && k / h < (1 << 27) && plan_chains(pl, axis_form);
  }

  // Elements of the reverse pass's zero-initialised allocation: the adjoint of the state after the
  // last sweep (adjb[0]) and the per-segment accumulators (1/T, rho Htilde^-1, start knot).
  int64_t adjoint_zero_elems() const { return (int64_t)nf * ld + (2 + 3 * (int64_t)v.s) * ld; }

  // Every device buffer of the handle, in one fixed order (the workspace layout).  has_* say which
  // optional inputs were given; n_chunks is the number of reduction chunks of the shape.
  top_status allocate_buffers(bool has_box, bool has_vmax, bool has_bc, int64_t n_chunks) {
    top::Layout L{v.p, v.s, v.box, v.vel, v.faces, v.num};
    const size_t R = rsz, l = (size_t)ld, s = (size_t)v.s;
    top_status st;
#define TOP_ALLOC(ptr, bytes) \
  if ((st = alloc(&(ptr), (bytes))) != TOP_OK) return st
    TOP_ALLOC(Hr, L.nhr() * l * R);
    if (v.faces) {
      TOP_ALLOC(Urot, 9 * l * R);
      TOP_ALLOC(fa, 4 * (size_t)top::kFaces * l * R);
      TOP_ALLOC(lam, 3 * l * sizeof(double));
    }
    TOP_ALLOC(iT, l * R);
    TOP_ALLOC(lo, 3 * l * R);
    TOP_ALLOC(hi, 3 * l * R);
    TOP_ALLOC(vmax, l * R);
    TOP_ALLOC(bcL, (size_t)B * 3 * s * R);
    for (int q = 0; q < 2; ++q) TOP_ALLOC(state[q], (size_t)nf * l * R);  // setup zeroes the padding
    TOP_ALLOC(cbuf, 3 * (size_t)L.n() * l * R);
    TOP_ALLOC(zold, 3 * s * l * R);
    TOP_ALLOC(flags, l);
    TOP_ALLOC(traj, l * sizeof(int32_t));
    TOP_ALLOC(Tdev, l * sizeof(double));
    TOP_ALLOC(rho_seg, l * sizeof(double));
    TOP_ALLOC(part, 3 * (size_t)S * sizeof(double));
    TOP_ALLOC(out, 3 * (size_t)B * sizeof(double));
    TOP_ALLOC(flag_dev, 4 * sizeof(int));   // non-finite, invalid input, chained-launch wait
    // epoch flags of chained launches: one per tile of any plan whose tile cores hold 64 segments
    // or more (the lane-per-axis variants only)
    chain_cap = axis_allowed(v, opt) && !v.num ? S / 64 + B + 1 : 0;
    if (chain_cap > 0) TOP_ALLOC(chain_flag, (size_t)chain_cap * sizeof(unsigned long long));
    TOP_ALLOC(rho_traj, (size_t)B * sizeof(double));
    TOP_ALLOC(chunk_sum, 3 * (size_t)std::max<int64_t>(n_chunks, 1) * sizeof(double));
    if (opt.check_every > 0) {
      TOP_ALLOC(done_dev, (size_t)B);
      TOP_ALLOC(fresh, (size_t)B);
      TOP_ALLOC(swept, (size_t)B * sizeof(int32_t));
      TOP_ALLOC(stop_at, (size_t)B * sizeof(int32_t));
      TOP_ALLOC(ratio, (size_t)B * sizeof(double));
      TOP_ALLOC(check_lists, 3 * (size_t)B * sizeof(int32_t));
      TOP_ALLOC(check_counts, 3 * sizeof(int32_t));
    }
    if (opt.checkpoint_every > 0) {
      tape_slots = opt.max_taped_iters / opt.checkpoint_every + 1;
      TOP_ALLOC(tape, (size_t)tape_slots * nf * l * R);
      TOP_ALLOC(Hd, L.nh() * l * R);
      TOP_ALLOC(wp64, (size_t)(S + B) * 3 * sizeof(double));
      if (has_box) {
        TOP_ALLOC(lo64, (size_t)S * 3 * sizeof(double));
        TOP_ALLOC(hi64, (size_t)S * 3 * sizeof(double));
      }
      if (has_vmax) TOP_ALLOC(vmax64, (size_t)B * sizeof(double));
      if (has_bc) TOP_ALLOC(bc64, (size_t)B * 2 * v.p * 3 * sizeof(double));
      // reverse pass: two block buffers of checkpoint_every states, the zero-initialised adjoint
      // and accumulators, the second adjoint buffer, and the float64 per-segment waypoint terms
      TOP_ALLOC(blk, 2 * (size_t)opt.checkpoint_every * nf * l * R);
      TOP_ALLOC(adjb[0], (size_t)adjoint_zero_elems() * R);
      TOP_ALLOC(adjb[1], (size_t)nf * l * R);
      acc_iT = (char*)adjb[0] + (size_t)nf * l * R;
      acc_hd = (char*)acc_iT + l * R;
      acc_z0 = (char*)acc_hd + l * R;
      for (double** p : {&dPL, &dPR, &dK, &dK0}) TOP_ALLOC(*p, (size_t)S * 3 * sizeof(double));
    }
#undef TOP_ALLOC
    return TOP_OK;
  }

  // Block buffers of the reverse pass; allocated with the handle when it records a tape.
  top_status ensure_blk() {
    if (blk != nullptr) return TOP_OK;
    return fail(TOP_E_STATE, "the handle has no reverse-pass buffers");
  }

  template <typename R>
  top_status finalize_t(double* coeffs, bool with_res, bool write_part, hipStream_t st) {
    top::FinalArgs<R> a{};
    a.c = (const R*)cbuf;
    a.state = (const R*)state[cur];
    a.zold = (const R*)zold;
    a.bcL = (const R*)bcL;
    a.T = Tdev;
    a.rho = rho_seg;
    a.flags = flags;
    a.traj = traj;
    a.S = S;
    a.ld = ld;
    a.part = write_part ? part : nullptr;
    a.coeffs = coeffs;
    a.nonfinite = flag_dev;
    a.with_res = with_res ? 1 : 0;
    // stopped trajectories keep their partials; coefficient output needs every segment
    a.done = (opt.check_every > 0 && coeffs == nullptr) ? done_dev : nullptr;
    a.off = off_dev;
    a.B = B;
    a.max_len = max_len;
    a.live = check_lists != nullptr ? check_lists + 2 * B : nullptr;
    a.live_count = check_counts != nullptr ? check_counts + 2 : nullptr;
    hipError_t e = top::launch_finalize<R>(v, a, st);
    if (e != hipSuccess) return fail(TOP_E_HIP, "finalize launch failed: %s", hipGetErrorString(e));
    return TOP_OK;
  }

  top_status finalize(double* coeffs, bool with_res, bool write_part, hipStream_t st) {
    return v.prec == 0 ? finalize_t<float>(coeffs, with_res, write_part, st)
                       : finalize_t<double>(coeffs, with_res, write_part, st);
  }

  template <typename R>
  top_status backward_t(const double* dcost, double* dP, double* dT) {
    const int K = iters_done, m = opt.checkpoint_every;
    const size_t sl = (size_t)nf * ld;
    top::Layout L{v.p, v.s, v.box, v.vel, v.faces, v.num};
    top_status s;
    const int64_t nzero = adjoint_zero_elems();
    auto chk = [](hipError_t e) -> top_status {
      return e == hipSuccess ? TOP_OK : fail(TOP_E_HIP, "backward launch failed: %s", hipGetErrorString(e));
    };
    if ((s = chk(top::launch_fill<R>((R*)adjb[0], nzero, R(0), stream))) != TOP_OK) return s;
    // Block j is replayed from its checkpoint (read in place from the tape) into block buffer j % 2,
    // keeping the state before every sweep, then reversed.  The replay of block j - 1 needs only the
    // tape, so it runs on a second stream while block j is reversed; the buffer it fills was last
    // read by the reversal of block j + 1.
    // The second stream and the events are the device's (created once): a backward call holds them
    // while it queues its work; the waits it queues refer to the records it made.
    ReverseAux* aux = nullptr;
    if ((s = reverse_aux(&aux)) != TOP_OK) return s;
    std::lock_guard<std::mutex> aux_lock(aux->mu);
    hipStream_t rstream = aux->stream;
    hipEvent_t ev_start = aux->ev[0], ev_rep[2] = {aux->ev[1], aux->ev[2]}, ev_adj[2] = {aux->ev[3], aux->ev[4]};
    auto buf_of = [&](int q) { return (R*)blk + (size_t)q * m * sl; };
    auto replay = [&](int j, hipStream_t st) -> top_status {
      const int n = std::min(K, j * m + m) - j * m;
      R* b = buf_of(j % 2);
      const R* ckpt = (const R*)tape + (size_t)j * sl;
      // one recording launch per replay chunk (halo sweeps at most on split trajectories): the launch
      // from slot t0 stores the states after its sweeps in slots t0+1 .. t0+cnt (slot 0 stays unused)
      for (int t0 = 0; t0 < n - 1;) {
        const int cnt = plan_ref().halo > 0 ? std::min(n - 1 - t0, plan_ref().halo) : n - 1 - t0;
        top::SweepArgs<R> a = sweep_args<R>(plan_ref(), lanes());
        a.st_in = t0 == 0 ? ckpt : b + (size_t)t0 * sl;
        a.st_out = b + (size_t)(t0 + cnt) * sl;
        a.iters = cnt;
        a.final_out = 0;
        a.rec = b + (size_t)t0 * sl;
        a.rec_slot = (int64_t)sl;
        top_status r = chk(top::launch_sweep<R>(v, a, plan_ref().n_tiles, st));
        if (r != TOP_OK) return r;
        t0 += cnt;
      }
      return TOP_OK;
    };
    int ai = 0;
    const int nblk = (K + m - 1) / m;
    // the last block was recorded by the forward when its states are all in its buffer
    const bool recorded = rec_block == nblk - 1 && rec_upto >= K - (nblk - 1) * m;
    rec_block = -1;  // the replays below overwrite the block buffers
    TOP_HIP(hipEventRecord(ev_start, stream));
    TOP_HIP(hipStreamWaitEvent(rstream, ev_start, 0));
    if (!recorded) {
      if ((s = replay(nblk - 1, rstream)) != TOP_OK) return s;
      TOP_HIP(hipEventRecord(ev_rep[(nblk - 1) % 2], rstream));
    }
    for (int j = nblk - 1; j >= 0; --j) {
      const int k_lo = j * m;
      const int n = std::min(K, k_lo + m) - k_lo;
      const int q = j % 2;
      if (j >= 1) {
        if (j + 1 < nblk) TOP_HIP(hipStreamWaitEvent(rstream, ev_adj[(j - 1) % 2], 0));
        if ((s = replay(j - 1, rstream)) != TOP_OK) return s;
        TOP_HIP(hipEventRecord(ev_rep[(j - 1) % 2], rstream));
      }
      if (!(recorded && j == nblk - 1)) TOP_HIP(hipStreamWaitEvent(stream, ev_rep[q], 0));
      const R* ckpt = (const R*)tape + (size_t)j * sl;
      R* b = buf_of(q);
      int t_hi = n;
      while (t_hi > 0) {
        // Reverse steps per launch on split trajectories: halo - 1.  A wrong value entering at a
        // tile's right edge reaches one lane further than in the forward sweep (the adjoint of a
        // right knot also flows through the neighbour's solve into the next knot's u), so after
        // `halo` steps the last core lane's knot adjoint would be stale.
        const int cnt = plan_ref().halo > 0 ? std::min(t_hi, plan_ref().halo - 1) : t_hi;
        const int t_lo = t_hi - cnt;
        top::AdjArgs<R> a{};
        a.k = sweep_args<R>(plan_ref(), lanes()).k;
        a.Hd = (const R*)Hd;
        a.lane_seg = lanes();
        a.W = plan_ref().W;
        a.fixpos = opt.fix_interior;
        a.blk = b + (size_t)t_lo * sl;
        a.blk0 = t_lo == 0 ? ckpt : nullptr;
        a.slot = (int64_t)sl;
        a.steps = cnt;
        a.adj_in = (const R*)adjb[ai];
        a.adj_out = (R*)adjb[ai ^ 1];
        a.dcost = dcost;
        a.with_cost = (k_lo + t_hi == K) ? 1 : 0;
        a.acc_iT = (R*)acc_iT;
        a.acc_hd = (R*)acc_hd;
        a.acc_z0 = (R*)acc_z0;
        if ((s = chk(top::launch_adjoint<R>(v, a, plan_ref().n_tiles, stream))) != TOP_OK) return s;
        ai ^= 1;
        t_hi = t_lo;
      }
      TOP_HIP(hipEventRecord(ev_adj[q], stream));
    }
    top::InitAdjArgs<R> ia{};
    ia.waypoints = wp64;
    ia.durations = Tdev;
    ia.box_lo = lo64;
    ia.box_hi = hi64;
    ia.vmax = vmax64;
    ia.bc = bc64;
    ia.traj = traj;
    ia.flags = flags;
    ia.S = S;
    ia.ld = ld;
    ia.lam = (const R*)adjb[ai];
    ia.acc_iT = (const R*)acc_iT;
    ia.acc_hd = (const R*)acc_hd;
    ia.acc_z0 = (const R*)acc_z0;
    ia.dPL = dPL;
    ia.dPR = dPR;
    ia.dK = dK;
    ia.dK0 = dK0;
    ia.dT = dT;
    if ((s = chk(top::launch_init_adjoint<R>(v, ia, stream))) != TOP_OK) return s;
    if (dP != nullptr)
      if ((s = chk(top::launch_gather_waypoints(dPL, dPR, dK, dK0, off_dev, B, S + B, dP, stream))) != TOP_OK)
        return s;
    (void)L;
    return TOP_OK;
  }

  // Host bookkeeping after k sweeps were queued (mirrors the launch sequence of enqueue).
  void advance(int k) {
    int remaining = k, done = iters_done;
    while (remaining > 0) {
      const int n = chunk(remaining, done);
      cur ^= 1;
      remaining -= n;
      done += n;
    }
    iters_done = done;
    have_sweep = true;
  }

  // Sweeps per launch for the remaining count.
  int chunk(int remaining, int done) const {
    int n = remaining;
    if (plan_ref().halo > 0) n = std::min(n, plan_ref().halo);
    if (tape != nullptr) n = std::min(n, opt.checkpoint_every - (done % opt.checkpoint_every));
    if (opt.check_every > 0) n = std::min(n, opt.check_every - (done % opt.check_every));
    return n;
  }

  // Residuals of the sweep that just wrote buffer `c`, the stopping test and the penalty update.
  top_status run_check(int c, hipStream_t st) {
    const int save = cur;
    cur = c;
    top_status s = finalize(nullptr, true, true, st);
    cur = save;
    if (s != TOP_OK) return s;
    hipError_t e = top::launch_reduce(reduce_args(), st);
    if (e != hipSuccess) return fail(TOP_E_HIP, "reduce launch failed: %s", hipGetErrorString(e));
    top::CheckArgs ca{};
    ca.res = out;
    ca.off = off_dev;
    ca.B = B;
    ca.check_every = opt.check_every;
    ca.adapt = opt.adapt_rho;
    ca.tol = opt.tol;
    ca.mu = opt.mu;
    ca.tau_incr = opt.tau_incr;
    ca.tau_decr = opt.tau_decr;
    ca.done = done_dev;
    ca.fresh = fresh;
    ca.swept = swept;
    ca.stop_at = stop_at;
    ca.rho = rho_traj;
    ca.ratio = ratio;
    ca.lists = check_lists;
    ca.counts = check_counts;
    if ((e = top::launch_reset_counts(check_counts, st)) != hipSuccess)
      return fail(TOP_E_HIP, "check reset failed: %s", hipGetErrorString(e));
    if ((e = top::launch_check(ca, st)) != hipSuccess)
      return fail(TOP_E_HIP, "check launch failed: %s", hipGetErrorString(e));
    if ((e = top::launch_freeze_copy(state[c], state[c ^ 1], check_lists, check_counts, off_dev, B, max_len, nf,
                                     ld, rsz, st)) != hipSuccess)
      return fail(TOP_E_HIP, "freeze copy failed: %s", hipGetErrorString(e));
    if (!opt.adapt_rho) return TOP_OK;
    e = v.prec == 0 ? rescale_t<float>(c, st) : rescale_t<double>(c, st);
    if (e != hipSuccess) return fail(TOP_E_HIP, "rescale launch failed: %s", hipGetErrorString(e));
    return TOP_OK;
  }

  template <typename R>
  hipError_t rescale_t(int c, hipStream_t st) {
    top::RescaleArgs<R> ra{};
    ra.lam = lam;
    ra.state = (R*)state[c];
    ra.Hr = (R*)Hr;
    ra.rho_seg = rho_seg;
    ra.ratio = ratio;
    ra.rho = rho_traj;
    ra.T = Tdev;
    ra.flags = flags;
    ra.traj = traj;
    ra.vmax = (const R*)vmax;
    ra.S = S;
    ra.ld = ld;
    ra.off = off_dev;
    ra.B = B;
    ra.max_len = max_len;
    ra.list = check_lists + B;
    ra.count = check_counts + 1;
    return top::launch_rescale<R>(v, ra, st);
  }

  // The launch sequence of k sweeps starting from buffer `c0` and sweep index `done0`.
  top_status enqueue(int k, int c0, int done0, hipStream_t st, hipEvent_t ev0 = nullptr,
                     hipEvent_t ev1 = nullptr) {
    int remaining = k, c = c0, done = done0;
    const size_t sbytes = (size_t)nf * ld * rsz;
    if (ev0 != nullptr) TOP_HIP(hipEventRecord(ev0, st));
    bool checked_last = false;
    // (not while a caller captures the stream into a graph: a cooperative launch is not captured)
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    const bool capturing = hipStreamIsCapturing(st, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone;
    if (!capturing && chains(k)) {
      // all k sweeps in one launch; its epochs alternate the state buffers like separate launches
      const Plan& pl = plan_ref();
      hipError_t e = top::launch_zero_u64(chain_flag, pl.n_tiles, st);
      if (e != hipSuccess) return fail(TOP_E_HIP, "chain flag reset failed: %s", hipGetErrorString(e));
      top_status s = sweep_launch(pl, lanes(), state[c], state[c ^ 1], k, true, st, false, nullptr, true);
      if (s != TOP_OK) return s;
      const int epochs = (k + pl.halo - 1) / pl.halo;
      c ^= epochs & 1;
      remaining = 0;
    }
    const int m = opt.checkpoint_every;
    const int j_last = tape != nullptr ? (done0 + k - 1) / m : -1;  // block of this call's last sweep
    while (remaining > 0) {
      const int n = chunk(remaining, done);
      const bool check = opt.check_every > 0 && (done + n) % opt.check_every == 0;
      const bool fin = (n == remaining) || check;
      // record the states of block j_last (launches never cross a checkpoint boundary)
      void* rec = nullptr;
      const int t0 = tape != nullptr ? done - j_last * m : 0;
      if (tape != nullptr && done / m == j_last) {
        if (t0 == 0) {
          rec_block = j_last;
          rec_upto = 1;
        }
        if (rec_block == j_last && rec_upto == t0 + 1) {
          top_status s = ensure_blk();
          if (s != TOP_OK) return s;
          rec = (char*)blk + ((size_t)(j_last % 2) * m + t0) * sbytes;
        }
      }
      top_status s = sweep_launch(plan_ref(), lanes(), state[c], state[c ^ 1], n, fin, st, false, rec);
      if (s != TOP_OK) return s;
      c ^= 1;
      if (rec != nullptr) {
        if (t0 + n < m) {  // the block goes on in a later launch: keep the state it starts from
          TOP_HIP(hipMemcpyAsync((char*)rec + (size_t)n * sbytes, state[c], sbytes, hipMemcpyDeviceToDevice, st));
          rec_upto = t0 + n + 1;
        } else {
          rec_upto = m;
        }
      }
      remaining -= n;
      done += n;
      checked_last = check;
      if (check && (s = run_check(c, st)) != TOP_OK) return s;
      if (tape != nullptr && done % opt.checkpoint_every == 0) {
        const int slot = done / opt.checkpoint_every;
        if (slot < tape_slots)
          TOP_HIP(hipMemcpyAsync((char*)tape + (size_t)slot * sbytes, state[c], sbytes,
                                 hipMemcpyDeviceToDevice, st));
      }
    }
    if (ev1 != nullptr) TOP_HIP(hipEventRecord(ev1, st));
    // residual and cost partials of the last sweep, reduced per trajectory (a check just did that,
    // before any change of rho)
    if (checked_last) return TOP_OK;
    const int save = cur;
    cur = c;
    top_status s = finalize(nullptr, true, true, st);
    cur = save;
    if (s != TOP_OK) return s;
    hipError_t e = top::launch_reduce(reduce_args(), st);
    if (e != hipSuccess) return fail(TOP_E_HIP, "reduce launch failed: %s", hipGetErrorString(e));
    return TOP_OK;
  }
};

extern "C" {

void top_default_options(top_options* opt) {
  if (opt == nullptr) return;
  std::memset(opt, 0, sizeof *opt);
  opt->order = 3;
  opt->n_cont = 0;
  opt->fix_interior = 1;
  opt->n_samples = 8;
  opt->precision = TOP_FP32;
  opt->checkpoint_every = 0;
  opt->max_taped_iters = 0;
  opt->tile_lanes = 0;
  opt->halo = 0;
  opt->use_graph = 1;
  opt->check_every = 0;
  opt->adapt_rho = 0;
  opt->tol = 0.05;
  opt->mu = 10.0;
  opt->tau_incr = 1.1;
  opt->tau_decr = 1.1;
  opt->local_solve = 0;
  opt->lbfgs_iters = 10;
  opt->vel_norm = 2;
  opt->lane_form = 0;
}

const char* top_last_error(void) { return g_err.c_str(); }

void top_destroy(top_problem* h) {
  if (h == nullptr) return;
  // Handles with graphs wait for their work; a handle on the pool releases its buffers behind an
  // event recorded on its stream and returns at once; a handle on a caller's workspace leaves
  // the workspace's stream order to the caller.
  std::shared_ptr<ReleaseEvent> done;
  if (!h->graphs.empty() || h->cap_stream != nullptr) {
    (void)hipStreamSynchronize(h->stream);
  } else if (!h->allocs.empty()) {
    done = std::make_shared<ReleaseEvent>();
    if (hipEventCreateWithFlags(&done->ev, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(done->ev, h->stream) != hipSuccess) {
      (void)hipStreamSynchronize(h->stream);
      done.reset();
    }
  }
  h->drop_graphs();
  if (h->cap_stream != nullptr) (void)hipStreamDestroy(h->cap_stream);
  if (h->ev_valid != nullptr) {
    (void)hipEventSynchronize(h->ev_valid);  // the readback into the pinned word has landed
    (void)hipEventDestroy(h->ev_valid);
  }
  pin_put(h->pin);
  for (auto& b : h->allocs) pool_put(b.p, b.bytes, b.dev, h->stream, done);  // none on a caller workspace
  delete h;
}

void top_trim(void) {
  int dev0 = 0;
  const bool have_dev = hipGetDevice(&dev0) == hipSuccess;
  std::vector<std::pair<int, void*>> blocks;
  {
    std::lock_guard<std::mutex> lk(g_pool.mu);
    for (auto& kv : g_pool.blocks) blocks.push_back({kv.first.first, kv.second.p});
    g_pool.blocks.clear();
    g_pool.cached = 0;
  }
  for (auto& b : blocks) {
    (void)hipSetDevice(b.first);
    (void)hipFree(b.second);  // waits for the device's queued work
  }
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto it = g_plans.begin(); it != g_plans.end();) {
      if (it->second.use_count() == 1) {
        (void)hipSetDevice(it->second->device);
        it = g_plans.erase(it);
      } else {
        ++it;
      }
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_shape_mu);
    for (auto it = g_shapes.begin(); it != g_shapes.end();) {
      if (it->second.use_count() == 1) {
        (void)hipSetDevice(it->second->device);
        it = g_shapes.erase(it);
      } else {
        ++it;
      }
    }
  }
  if (have_dev) (void)hipSetDevice(dev0);
}

// Options after defaults, checked as far as they can be without the trajectory lengths, and the
// kernel variant they select.  box/vel/polytope say which corridor and bound are given.
static top_status resolve_options(const top_options* opt_in, bool box, bool vel, bool polytope, top_options* opt_out,
                                  top::Variant* v_out) {
  top_options opt;
  if (opt_in != nullptr) opt = *opt_in; else top_default_options(&opt);
  if (opt.order != 3 && opt.order != 4) return fail(TOP_E_UNSUPPORTED, "order must be 3 or 4 (got %d)", opt.order);
  const int s = opt.n_cont == 0 ? opt.order : opt.n_cont;
  if (s != opt.order && s != opt.order + 1 && s != 2 * opt.order - 1)
    return fail(TOP_E_UNSUPPORTED, "n_cont must be p, p+1 or 2p-1 (got %d for p = %d)", s, opt.order);
  if (s == 2 * opt.order - 1 && opt.checkpoint_every > 0)
    return fail(TOP_E_UNSUPPORTED, "n_cont = 2p-1 cannot be combined with a tape");
  if (opt.n_samples == 0) opt.n_samples = top::kSamples;
  if (opt.n_samples != top::kSamples) return fail(TOP_E_UNSUPPORTED, "only n_samples = 8 is built (got %d)", opt.n_samples);
  if (opt.precision != TOP_FP32 && opt.precision != TOP_FP64) return fail(TOP_E_INVALID, "precision must be TOP_FP32 or TOP_FP64");
  if (opt.fix_interior != 0 && opt.fix_interior != 1) return fail(TOP_E_INVALID, "fix_interior must be 0 or 1");
  if (opt.checkpoint_every < 0 || (opt.checkpoint_every > 0 && opt.max_taped_iters < 1))
    return fail(TOP_E_INVALID, "checkpoint_every >= 0, and max_taped_iters >= 1 when it is > 0");
  if (opt.local_solve != 0 && opt.local_solve != 1) return fail(TOP_E_INVALID, "local_solve must be 0 or 1");
  if (opt.vel_norm == 0) opt.vel_norm = 2;
  if (opt.vel_norm != 2 && opt.vel_norm != 4) return fail(TOP_E_INVALID, "vel_norm must be 2 or 4 (got %d)", opt.vel_norm);
  if (opt.vel_norm == 4 && opt.local_solve != 1)
    return fail(TOP_E_UNSUPPORTED, "the l4 speed bound needs NumericSolve (local_solve = 1)");
  top::Variant v{opt.precision == TOP_FP64 ? 1 : 0, opt.order, s, box, vel, polytope ? top::kFaces : 0,
                 opt.local_solve == 1 ? 1 : 0, opt.vel_norm};
  if (v.num) {
    if (!vel) return fail(TOP_E_UNSUPPORTED, "NumericSolve needs a velocity bound (vmax)");
    if (polytope || s != opt.order || opt.checkpoint_every > 0 || opt.check_every > 0)
      return fail(TOP_E_UNSUPPORTED, "NumericSolve takes s = p, a box or no corridor, no tape and no checks");
    if (opt.lbfgs_iters < 0) return fail(TOP_E_INVALID, "lbfgs_iters must be >= 0");
  }
  const bool taped = opt.checkpoint_every > 0;
  if (polytope && taped) return fail(TOP_E_UNSUPPORTED, "a polytope corridor cannot be combined with a tape");
  if (opt.lane_form != 0 && opt.lane_form != 1 && opt.lane_form != 3)
    return fail(TOP_E_INVALID, "lane_form must be 0, 1 or 3 (got %d)", opt.lane_form);
  if (opt.chain != 0 && opt.chain != 1) return fail(TOP_E_INVALID, "chain must be 0 or 1 (got %d)", opt.chain);
  if (opt.lane_form == 3 && !axis_allowed(v, opt))
    return fail(TOP_E_UNSUPPORTED, "one lane per axis needs n_cont < 2p-1, no polytope, no tape and no "
                                   "residual checks");
  if (opt.halo < 0) return fail(TOP_E_INVALID, "halo must be >= 0");
  if (opt.check_every < 0) return fail(TOP_E_INVALID, "check_every must be >= 0 (got %d)", opt.check_every);
  if (opt.check_every > 0) {
    if (taped) return fail(TOP_E_UNSUPPORTED, "residual checks cannot be combined with a tape");
    if (opt.adapt_rho != 0 && opt.adapt_rho != 1) return fail(TOP_E_INVALID, "adapt_rho must be 0 or 1");
    if (!std::isfinite(opt.tol)) return fail(TOP_E_INVALID, "tol must be finite");
    if (opt.adapt_rho && !(opt.mu > 1.0 && opt.tau_incr > 1.0 && opt.tau_decr > 1.0 && std::isfinite(opt.mu) &&
                           std::isfinite(opt.tau_incr) && std::isfinite(opt.tau_decr)))
      return fail(TOP_E_INVALID, "mu, tau_incr and tau_decr must be finite and > 1");
  }
  opt.n_cont = s;
  *opt_out = opt;
  *v_out = v;
  return TOP_OK;
}

// Reduction chunks of a CSR shape (chunk j of trajectory b covers kReduceChunk segments from
// off[b] + j * kReduceChunk).
static int64_t count_chunks(const int64_t* off, int B) {
  int64_t n = 0;
  for (int b = 0; b < B; ++b) n += (off[b + 1] - off[b] + top::kReduceChunk - 1) / top::kReduceChunk;
  return n;
}

// Fill the shape fields of a handle that has no buffers yet.
static void shape_handle(top_problem* h, const top_options& opt, const top::Variant& v, int B, int64_t S) {
  h->opt = opt;
  h->v = v;
  h->B = B;
  h->S = S;
  h->ld = (S + 63) / 64 * 64;
  h->rsz = v.prec == 0 ? sizeof(float) : sizeof(double);
  top::Layout L{v.p, v.s, v.box, v.vel, v.faces, v.num};
  h->nf = L.nf();
}

// Workspace bytes of a problem (exact for the given presence flags and chunk count), or 0 with the
// error set.
static size_t workspace_need(int32_t n_traj, int64_t S, const top_options& opt, const top::Variant& v, bool has_box,
                             bool has_vmax, bool has_bc, int64_t n_chunks) {
  top_problem sz;
  sz.sizing = true;
  shape_handle(&sz, opt, v, n_traj, S);
  if (sz.allocate_buffers(has_box, has_vmax, has_bc, n_chunks) != TOP_OK) return 0;
  return sz.ws_used;
}

static size_t workspace_bytes_impl(int32_t n_traj, int64_t n_seg_total, int32_t n_faces, const top_options* opt_in) {
  if (n_traj < 1) { fail(TOP_E_INVALID, "n_traj must be >= 1 (got %d)", n_traj); return 0; }
  if (n_seg_total < n_traj) {
    fail(TOP_E_INVALID, "n_seg_total must be >= n_traj (every trajectory has a segment; got %lld)",
         (long long)n_seg_total);
    return 0;
  }
  if (n_seg_total + n_traj >= (int64_t)top::kHaloBit) {
    fail(TOP_E_UNSUPPORTED, "too many segments (%lld)", (long long)n_seg_total);
    return 0;
  }
  top_options opt;
  top::Variant v;
  if (resolve_options(opt_in, n_faces == 0, true, n_faces > 0, &opt, &v) != TOP_OK) return 0;
  // chunks: sum over trajectories of ceil(len / c) <= (S + B (c - 1)) / c
  const int64_t c = top::kReduceChunk;
  const int64_t chunks = (n_seg_total + (int64_t)n_traj * (c - 1)) / c;
  const size_t need = workspace_need(n_traj, n_seg_total, opt, v, n_faces == 0, true, true, chunks);
  return need == 0 ? 0 : need + kWsAlign;  // room to align an arbitrary base
}

// The execution plan's tile width, halo and lane form for this shape and these options: explicit,
// tuned for the shape class (top_tune), or the default (see top_options.lane_form).
static top_status choose_plan(const top::Variant& v, const top_options& opt, const std::vector<int64_t>& off,
                              bool taped, int* W_out, int* halo_out, int* form_out) {
  const bool axis_ok = axis_allowed(v, opt);
  const int64_t S = off.back();
  int64_t longest = 0;
  for (size_t b = 0; b + 1 < off.size(); ++b) longest = std::max<int64_t>(longest, off[b + 1] - off[b]);
  int W = opt.tile_lanes, halo = opt.halo, form = opt.lane_form;
  if (W == 0 && form == 0) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_load();
    auto it = g_tune.find(shape_key(v, off));
    if (it != g_tune.end()) {
      const TuneChoice& t = it->second;
      const bool valid = t.form == 3 ? (axis_ok && t.W <= axis_tile_max(v)) : t.W <= max_tile(v, taped);
      if (valid) {
        W = t.W;
        form = t.form;
        if (halo == 0) halo = t.halo;
      }
    }
  }
  if (form == 0) {
    // NumericSolve: four lanes per segment where allowed (256 batched trajectories, 67,259 segments,
    // 50 sweeps of 10 L-BFGS iterations: 7.4 against 12.3 ms in float32, 15 against 62 ms in float64).
    // Closed form: three lanes per segment where allowed and either some trajectory is longer than a one-lane
    // tile, or (float32, no tile width given) one lane per segment would give fewer waves than half
    // the device's SIMDs: a small problem is latency-bound, and three times the waves each with a
    // third of the work finish sooner (a 64-segment trajectory: 0.60 against 1.44 ms for 1,000
    // sweeps; 15,384 segments in 64 trajectories: 0.64 against 0.77 ms for 200; at 67,259 segments,
    // one wave per SIMD with one lane, the one-lane form is ahead, 0.82 against 1.26 ms).
    const bool few_waves = opt.tile_lanes == 0 && v.prec == 0 && (S + 63) / 64 < device_simds() / 2;
    form = (axis_ok && (v.num || longest > max_tile(v, taped) || few_waves)) ? 3 : 1;
  }
  const int wmax = form == 3 ? axis_tile_max(v) : max_tile(v, taped);
  if (wmax < 64) return fail(TOP_E_UNSUPPORTED, "the device's per-workgroup LDS is too small for the adjoint kernel");
  if (opt.tile_lanes != 0 && (opt.tile_lanes < 64 || opt.tile_lanes > wmax || opt.tile_lanes % 64 != 0))
    return fail(TOP_E_INVALID, "tile_lanes must be a multiple of 64 in [64, %d] (got %d)", wmax, opt.tile_lanes);
  // (NumericSolve's four-lane form: 64-segment tiles, three per CU, ahead of 128-segment ones)
  if (W == 0) W = (form == 3 && v.num) ? 64 : wmax;
  if (halo == 0) halo = std::max(1, std::min(32, W / 8));
  if (2 * halo >= W) return fail(TOP_E_INVALID, "halo %d too large for %d-lane tiles", halo, W);
  if (taped && halo < 2) {
    if (opt.halo != 0) return fail(TOP_E_INVALID, "a handle that records a tape needs halo >= 2 (got %d)", halo);
    halo = 2;
  }
  *W_out = W;
  *halo_out = halo;
  *form_out = form;
  return TOP_OK;
}

static top_status create_impl(int32_t n_traj, const int64_t* seg_offsets, const double* waypoints,
                              const double* durations, const double* bc, const double* box_lo,
                              const double* box_hi, int32_t n_faces, const double* faces, const double* vmax,
                              const double* rho, const top_options* opt_in, void* workspace, size_t workspace_bytes,
                              hipStream_t stream, top_problem** out, top::Mem mem = top::Mem::kCallerWs) {
  using top::Mem;
  if (out == nullptr) return fail(TOP_E_INVALID, "out is NULL");
  *out = nullptr;
  if (n_traj < 1) return fail(TOP_E_INVALID, "n_traj must be >= 1 (got %d)", n_traj);
  if (seg_offsets == nullptr) return fail(TOP_E_INVALID, "seg_offsets is NULL");
  if (waypoints == nullptr || durations == nullptr || rho == nullptr)
    return fail(TOP_E_INVALID, "waypoints, durations and rho are required");
  if ((box_lo == nullptr) != (box_hi == nullptr)) return fail(TOP_E_INVALID, "give both box_lo and box_hi, or neither");
  if ((workspace == nullptr) != (workspace_bytes == 0))
    return fail(TOP_E_INVALID, "give a workspace with its size, or NULL and 0 for the library's pool");
  if (seg_offsets[0] != 0) return fail(TOP_E_INVALID, "seg_offsets[0] must be 0");
  for (int b = 0; b < n_traj; ++b)
    if (seg_offsets[b + 1] <= seg_offsets[b])
      return fail(TOP_E_INVALID, "trajectory %d has no segment (seg_offsets must increase strictly)", b);
  const int64_t S = seg_offsets[n_traj];
  if (S + n_traj >= (int64_t)top::kHaloBit) return fail(TOP_E_UNSUPPORTED, "too many segments (%lld)", (long long)S);
  top_options opt;
  top::Variant v;
  top_status st = resolve_options(opt_in, box_lo != nullptr, vmax != nullptr, faces != nullptr, &opt, &v);
  if (st != TOP_OK) return st;
  const int s = opt.n_cont;
  const bool taped = opt.checkpoint_every > 0;
  if (opt.check_every > 0) {
    int64_t longest = 0;
    for (int b = 0; b < n_traj; ++b) longest = std::max<int64_t>(longest, seg_offsets[b + 1] - seg_offsets[b]);
    if (longest > 65535LL * 128)  // the check kernels' trajectory-major grids
      return fail(TOP_E_UNSUPPORTED, "residual checks support trajectories of at most %lld segments",
                  65535LL * 128);
  }
  if (mem == Mem::kPool) workspace = nullptr, workspace_bytes = 0;
  const std::vector<int64_t> off(seg_offsets, seg_offsets + n_traj + 1);
  const bool axis_ok = axis_allowed(v, opt);
  int W = 0, halo = 0, form = 0;
  if ((st = choose_plan(v, opt, off, taped, &W, &halo, &form)) != TOP_OK) return st;
  Plan own_plan;
  const TailSpec ts = tail_spec(v, opt, W, form);
  if (mem == Mem::kStatic) own_plan = make_plan(off, W, halo, ts.round, ts.W, ts.form);
  // The workspace must hold this problem's buffers (checked before any device work).
  size_t ws_pad = 0;
  const int64_t n_chunks = count_chunks(seg_offsets, n_traj);
  if (workspace != nullptr) {
    ws_pad = (kWsAlign - (uintptr_t)workspace % kWsAlign) % kWsAlign;
    size_t need = workspace_need(n_traj, S, opt, v, box_lo != nullptr, vmax != nullptr, bc != nullptr, n_chunks);
    if (need == 0) return fail(TOP_E_INVALID, "workspace sizing failed");
    if (mem == Mem::kStatic) {
      top_problem sz;
      sz.sizing = true;
      sz.B = n_traj;
      (void)sz.allocate_tables(n_chunks, own_plan.table_elems());
      need += sz.ws_used;
    }
    if (workspace_bytes < ws_pad + need)
      return fail(TOP_E_WORKSPACE, "workspace of %zu bytes is too small: this problem needs %zu (plus %zu to align it)",
                  workspace_bytes, need, ws_pad);
  }
  {
    // Several kernels keep spill areas or local arrays in per-lane scratch (the build refuses any
    // kernel above top::kScratchLimit bytes).  A kernel whose scratch exceeded the runtime's per-lane
    // stack limit was seen to compute wrong values, so the limit is raised first, and a device on
    // which it cannot be raised is refused.
    size_t lim = 0;
    hipError_t e = hipDeviceGetLimit(&lim, hipLimitStackSize);
    if (e == hipSuccess && lim < top::kScratchLimit) {
      e = hipDeviceSetLimit(hipLimitStackSize, top::kScratchLimit);
      if (e == hipSuccess) e = hipDeviceGetLimit(&lim, hipLimitStackSize);
    }
    if (e != hipSuccess) return fail(TOP_E_HIP, "per-lane stack limit: %s", hipGetErrorString(e));
    if (lim < top::kScratchLimit)
      return fail(TOP_E_HIP, "the per-lane stack limit stays at %zu bytes (kernels need %zu)", lim,
                  (size_t)top::kScratchLimit);
  }

  top_problem* h = new (std::nothrow) top_problem();
  if (h == nullptr) return fail(TOP_E_NOMEM, "host allocation failed");
  shape_handle(h, opt, v, n_traj, S);
  h->off = off;
  h->explicit_tile = opt.tile_lanes != 0 || opt.lane_form != 0;
  h->axis = form == 3;
  h->axis_ok = axis_ok;
  if (const char* e = std::getenv("TOP_CHAIN_SPIN")) {
    char* end = nullptr;
    const long n = std::strtol(e, &end, 10);
    if (end != e && n >= 0 && n < top::kChainSpin) h->chain_spin = (int)n;
  }
  for (int b = 0; b < n_traj; ++b) h->max_len = std::max<int64_t>(h->max_len, seg_offsets[b + 1] - seg_offsets[b]);
  h->stream = stream;
  if (workspace != nullptr) {
    h->ws = static_cast<char*>(workspace) + ws_pad;
    h->ws_cap = workspace_bytes - ws_pad;
  }

  auto bail = [&](top_status st) { top_destroy(h); return st; };
  const size_t R = h->rsz, ld = (size_t)h->ld;
  if (mem != Mem::kStatic) {
    if ((st = get_shape(h->off, &h->shape)) != TOP_OK) return bail(st);
    h->off_dev = h->shape->off_dev;
    h->chunk_off = h->shape->chunk_off;
    h->chunk_traj = h->shape->chunk_traj;
    h->n_chunks = h->shape->n_chunks;
  } else {
    h->n_chunks = (int)n_chunks;
  }
  if ((st = h->allocate_buffers(box_lo != nullptr, vmax != nullptr, bc != nullptr, h->n_chunks)) != TOP_OK)
    return bail(st);
  if (mem == Mem::kStatic) {
    // shape tables and lane map into the workspace, from host copies the handle keeps
    h->own_tables = true;
    h->own_plan = std::move(own_plan);
    chunk_tables(h->off, &h->own_chunk_off, &h->own_chunk_traj);
    if ((st = h->allocate_tables(h->n_chunks, h->own_plan.table_elems())) != TOP_OK) return bail(st);
    hipError_t e = hipMemcpyAsync(const_cast<int64_t*>(h->off_dev), h->off.data(), h->off.size() * sizeof(int64_t),
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(const_cast<int32_t*>(h->chunk_off), h->own_chunk_off.data(),
                         h->own_chunk_off.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !h->own_chunk_traj.empty())
      e = hipMemcpyAsync(const_cast<int32_t*>(h->chunk_traj), h->own_chunk_traj.data(),
                         h->own_chunk_traj.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = upload_plan(h->own_plan, h->own_lanes, stream, true);
    if (e != hipSuccess) return bail(fail(TOP_E_HIP, "table upload failed: %s", hipGetErrorString(e)));
  }
  if (opt.check_every > 0) {
    hipError_t e = hipMemsetAsync(h->done_dev, 0, (size_t)n_traj, stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->swept, 0, (size_t)n_traj * sizeof(int32_t), stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->stop_at, 0xff, (size_t)n_traj * sizeof(int32_t), stream);
    if (e == hipSuccess) e = top::launch_all_running(h->check_lists, h->check_counts, n_traj, stream);
    if (e != hipSuccess) return bail(fail(TOP_E_HIP, "check state reset failed: %s", hipGetErrorString(e)));
  }
  {
    hipError_t e = hipMemcpyAsync(h->rho_traj, rho, (size_t)n_traj * sizeof(double), hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return bail(fail(TOP_E_HIP, "rho copy failed: %s", hipGetErrorString(e)));
  }
  if (taped) {
    const size_t nwp = (size_t)(S + n_traj) * 3 * sizeof(double);
    hipError_t e = hipMemcpyAsync(h->wp64, waypoints, nwp, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess && box_lo != nullptr) {
      e = hipMemcpyAsync(h->lo64, box_lo, (size_t)S * 3 * sizeof(double), hipMemcpyDeviceToDevice, stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(h->hi64, box_hi, (size_t)S * 3 * sizeof(double), hipMemcpyDeviceToDevice, stream);
    }
    if (e == hipSuccess && vmax != nullptr)
      e = hipMemcpyAsync(h->vmax64, vmax, (size_t)n_traj * sizeof(double), hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess && bc != nullptr)
      e = hipMemcpyAsync(h->bc64, bc, (size_t)n_traj * 2 * v.p * 3 * sizeof(double), hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return bail(fail(TOP_E_HIP, "input copy failed: %s", hipGetErrorString(e)));
  }
  {
    hipError_t e = hipMemsetAsync(h->flag_dev, 0, 4 * sizeof(int), stream);
    if (e != hipSuccess) return bail(fail(TOP_E_HIP, "flag reset failed: %s", hipGetErrorString(e)));
  }
  top::SetupArgs sa{waypoints, durations, bc, box_lo, box_hi, faces, n_faces, vmax, rho, h->off_dev, n_traj, S,
                    opt.fix_interior};
  // The device-side input check runs first and its flags come back through a pinned host word behind
  // an event, so the setup is queued before the host waits for them (the setup is memory-safe
  // whatever the input values: every index it forms derives from the host-checked offsets).  Invalid
  // inputs then release the handle.
  {
    hipError_t e = top::launch_validate(sa, v.p, h->flag_dev, stream);
    if (e != hipSuccess) return bail(fail(TOP_E_HIP, "validation launch failed: %s", hipGetErrorString(e)));
    h->pin = mem == Mem::kStatic ? nullptr : pin_get();
    if (h->pin != nullptr) {
      e = hipMemcpyAsync(h->pin, h->flag_dev, 2 * sizeof(int), hipMemcpyDeviceToHost, stream);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_valid, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventRecord(h->ev_valid, stream);
      if (e != hipSuccess) return bail(fail(TOP_E_HIP, "validation readback failed: %s", hipGetErrorString(e)));
    }
  }
  {
    hipError_t e;
    if (v.prec == 0) {
      top::SetupOut<float> o{(float*)h->Hr, (float*)h->iT, (float*)h->lo, (float*)h->hi, (float*)h->vmax,
                             h->flags, h->traj, (float*)h->bcL, (float*)h->state[0], (float*)h->cbuf,
                             h->ld, h->Tdev, h->rho_seg, (float*)h->Hd, (float*)h->Urot, (float*)h->fa, h->lam,
                             (float*)h->state[1], h->nf};
      e = top::launch_setup<float>(v, sa, o, stream);
    } else {
      top::SetupOut<double> o{(double*)h->Hr, (double*)h->iT, (double*)h->lo, (double*)h->hi, (double*)h->vmax,
                              h->flags, h->traj, (double*)h->bcL, (double*)h->state[0], (double*)h->cbuf,
                              h->ld, h->Tdev, h->rho_seg, (double*)h->Hd, (double*)h->Urot, (double*)h->fa,
                              h->lam, (double*)h->state[1], h->nf};
      e = top::launch_setup<double>(v, sa, o, stream);
    }
    if (e != hipSuccess) return bail(fail(TOP_E_HIP, "setup launch failed: %s", hipGetErrorString(e)));
  }
  if (h->tape != nullptr) {
    hipError_t e = hipMemcpyAsync(h->tape, h->state[0], (size_t)h->nf * ld * R, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return bail(fail(TOP_E_HIP, "tape copy failed: %s", hipGetErrorString(e)));
  }
  if (mem != Mem::kStatic && (st = get_plan(h->off, W, halo, ts, &h->pe)) != TOP_OK) return bail(st);
  // the input check's verdict
  int bad = 0;
  {
    hipError_t e;
    if (h->pin != nullptr) {
      e = hipEventSynchronize(h->ev_valid);
      bad = h->pin[0];
    } else {  // no pinned word free: read back through pageable memory (waits for the setup too)
      int b2[2] = {0, 0};
      e = hipMemcpyAsync(b2, h->flag_dev, sizeof b2, hipMemcpyDeviceToHost, stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      bad = b2[0];
    }
    if (e != hipSuccess) return bail(fail(TOP_E_HIP, "validation failed: %s", hipGetErrorString(e)));
  }
  if (bad != 0) {
    std::string what;
    if (bad & 1) what += " durations (need finite T > 0);";
    if (bad & 2) what += " box (need finite lo < hi);";
    if (bad & 4) what += " waypoints (need finite);";
    if (bad & 8) what += " rho (need finite > 0);";
    if (bad & 16) what += " vmax (need finite > 0);";
    if (bad & 32) what += " bc (need finite);";
    if (bad & 64) what += " faces (need finite);";
    return bail(fail(TOP_E_INVALID, "invalid input:%s", what.c_str()));
  }
  *out = h;
  return TOP_OK;
}

top_status top_create(int32_t n_traj, const int64_t* seg_offsets, const double* waypoints,
                      const double* durations, const double* bc, const double* box_lo,
                      const double* box_hi, const double* vmax, const double* rho,
                      const top_options* opt, void* workspace, size_t workspace_bytes, hipStream_t stream,
                      top_problem** out) {
  return create_impl(n_traj, seg_offsets, waypoints, durations, bc, box_lo, box_hi, 0, nullptr, vmax, rho, opt,
                     workspace, workspace_bytes, stream, out);
}


size_t top_workspace_bytes(int32_t n_traj, int64_t n_seg_total, const top_options* opt) {
  return workspace_bytes_impl(n_traj, n_seg_total, 0, opt);
}

size_t top_workspace_bytes_polytope(int32_t n_traj, int64_t n_seg_total, int32_t n_faces, const top_options* opt) {
  if (n_faces < 1 || n_faces > top::kFaces) {
    fail(TOP_E_UNSUPPORTED, "n_faces must be in [1, %d] (got %d)", top::kFaces, n_faces);
    return 0;
  }
  return workspace_bytes_impl(n_traj, n_seg_total, n_faces, opt);
}

top_status top_create_polytope(int32_t n_traj, const int64_t* seg_offsets, const double* waypoints,
                               const double* durations, const double* bc, int32_t n_faces, const double* faces,
                               const double* vmax, const double* rho, const top_options* opt,
                               void* workspace, size_t workspace_bytes, hipStream_t stream, top_problem** out) {
  if (out != nullptr) *out = nullptr;
  if (faces == nullptr) return fail(TOP_E_INVALID, "faces is NULL");
  if (n_faces < 1 || n_faces > top::kFaces)
    return fail(TOP_E_UNSUPPORTED, "n_faces must be in [1, %d] (got %d)", top::kFaces, n_faces);
  return create_impl(n_traj, seg_offsets, waypoints, durations, bc, nullptr, nullptr, n_faces, faces, vmax, rho, opt,
                     workspace, workspace_bytes, stream, out);
}

top_status top_iterate(top_problem* h, int32_t k) {
  if (h == nullptr) return fail(TOP_E_INVALID, "handle is NULL");
  if (k < 0) return fail(TOP_E_INVALID, "k must be >= 0 (got %d)", k);
  if (k == 0) return TOP_OK;
  if (h->tape != nullptr && h->iters_done + k > h->opt.max_taped_iters)
    return fail(TOP_E_STATE, "the tape holds %d sweeps; %d done, %d more asked", h->opt.max_taped_iters,
                h->iters_done, k);
  // The sequence only depends on (k, start buffer) unless a tape is written.
  // A sequence is captured into a graph the second time it is asked for; the first call launches it
  // directly (a one-shot solve would only pay for the capture).
  const auto key = std::make_tuple(k, h->cur, h->opt.check_every > 0 ? h->iters_done % h->opt.check_every : 0);
  // (a chained launch is cooperative and is launched directly)
  const bool graph = h->opt.use_graph != 0 && h->tape == nullptr && !h->chains(k) &&
                     (h->graphs.count(key) != 0 || h->graph_seen.count(key) != 0);
  if (!graph) {
    top_status s = h->enqueue(k, h->cur, h->iters_done, h->stream);
    if (s != TOP_OK) return s;
    if (h->opt.use_graph != 0 && h->tape == nullptr && !h->chains(k)) h->graph_seen.insert(key);
  } else {
    auto it = h->graphs.find(key);
    if (it == h->graphs.end()) {
      if (h->cap_stream == nullptr) TOP_HIP(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
      TOP_HIP(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
      top_status s = h->enqueue(k, h->cur, h->iters_done, h->cap_stream);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
      if (s != TOP_OK) { if (g) (void)hipGraphDestroy(g); return s; }
      if (e != hipSuccess) return fail(TOP_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
      hipGraphExec_t ex = nullptr;
      e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      if (e != hipSuccess) { (void)hipGraphDestroy(g); return fail(TOP_E_HIP, "graph instantiate failed: %s", hipGetErrorString(e)); }
      h->graph_defs.push_back(g);
      it = h->graphs.emplace(key, ex).first;
    }
    TOP_HIP(hipGraphLaunch(it->second, h->stream));
  }
  h->advance(k);
  return TOP_OK;
}

top_status top_time_sweeps(top_problem* h, int32_t k, float* ms) {
  if (h == nullptr || ms == nullptr) return fail(TOP_E_INVALID, "handle and ms must be non-NULL");
  if (k < 1) return fail(TOP_E_INVALID, "k must be >= 1 (got %d)", k);
  if (h->tape != nullptr && h->iters_done + k > h->opt.max_taped_iters)
    return fail(TOP_E_STATE, "the tape holds %d sweeps; %d done, %d more asked", h->opt.max_taped_iters,
                h->iters_done, k);
  hipEvent_t e0, e1;
  TOP_HIP(hipEventCreate(&e0));
  TOP_HIP(hipEventCreate(&e1));
  top_status s = h->enqueue(k, h->cur, h->iters_done, h->stream, e0, e1);
  if (s == TOP_OK) {
    h->advance(k);
    hipError_t e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e != hipSuccess) s = fail(TOP_E_HIP, "sweep timing failed: %s", hipGetErrorString(e));
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return s;
}

top_status top_residuals(const top_problem* h, double* r_primal, double* r_dual) {
  if (h == nullptr) return fail(TOP_E_INVALID, "handle is NULL");
  if (!h->have_sweep) return fail(TOP_E_STATE, "no sweep has run yet");
  if (r_primal != nullptr)
    TOP_HIP(hipMemcpyAsync(r_primal, h->out + h->B, h->B * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  if (r_dual != nullptr)
    TOP_HIP(hipMemcpyAsync(r_dual, h->out + 2 * h->B, h->B * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  return TOP_OK;
}

top_status top_cost(const top_problem* h, double* cost) {
  if (h == nullptr || cost == nullptr) return fail(TOP_E_INVALID, "handle and cost must be non-NULL");
  if (!h->have_sweep && !h->init_cost_ready) {
    // before any sweep: the cost of the Init guess, reduced on first request only
    top_problem* m = const_cast<top_problem*>(h);
    top_status st = m->finalize(nullptr, false, true, h->stream);
    if (st != TOP_OK) return st;
    hipError_t e = top::launch_reduce(m->reduce_args(), h->stream);
    if (e != hipSuccess) return fail(TOP_E_HIP, "reduce launch failed: %s", hipGetErrorString(e));
    m->init_cost_ready = true;
  }
  TOP_HIP(hipMemcpyAsync(cost, h->out, h->B * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  return TOP_OK;
}

top_status top_coeffs(const top_problem* h, double* coeffs) {
  if (h == nullptr || coeffs == nullptr) return fail(TOP_E_INVALID, "handle and coeffs must be non-NULL");
  hipError_t e = h->v.prec == 0
      ? top::launch_coeffs<float>(h->v.p, (const float*)h->cbuf, h->Tdev, h->S, h->ld, coeffs, h->stream)
      : top::launch_coeffs<double>(h->v.p, (const double*)h->cbuf, h->Tdev, h->S, h->ld, coeffs, h->stream);
  if (e != hipSuccess) return fail(TOP_E_HIP, "coefficient output launch failed: %s", hipGetErrorString(e));
  return TOP_OK;
}

top_status top_backward(top_problem* h, const double* dcost, double* dwaypoints, double* ddurations) {
  if (h == nullptr || dcost == nullptr) return fail(TOP_E_INVALID, "handle and dcost must be non-NULL");
  if (h->tape == nullptr) return fail(TOP_E_STATE, "no tape: create with checkpoint_every > 0");
  if (h->iters_done < 1) return fail(TOP_E_STATE, "no sweep has run yet");
  if (h->iters_done > h->opt.max_taped_iters)
    return fail(TOP_E_STATE, "%d sweeps run but the tape holds %d", h->iters_done, h->opt.max_taped_iters);
  return h->v.prec == 0 ? h->backward_t<float>(dcost, dwaypoints, ddurations)
                        : h->backward_t<double>(dcost, dwaypoints, ddurations);
}

top_status top_convergence(const top_problem* h, int32_t* iters, double* rho, uint8_t* done) {
  if (h == nullptr) return fail(TOP_E_INVALID, "handle is NULL");
  hipError_t e = top::launch_conv_report(h->opt.check_every > 0 ? h->done_dev : nullptr, h->stop_at, h->rho_traj,
                                         h->B, h->iters_done, iters, rho, done, h->stream);
  if (e != hipSuccess) return fail(TOP_E_HIP, "convergence report failed: %s", hipGetErrorString(e));
  return TOP_OK;
}

top_status top_sync_status(top_problem* h) {
  if (h == nullptr) return fail(TOP_E_INVALID, "handle is NULL");
  int flag[4] = {0, 0, 0, 0};
  TOP_HIP(hipMemcpyAsync(flag, h->flag_dev, sizeof flag, hipMemcpyDeviceToHost, h->stream));
  TOP_HIP(hipStreamSynchronize(h->stream));
  if (flag[2] != 0) return fail(TOP_E_HIP, "a tile of a chained sweep launch gave up waiting for a neighbour");
  if (flag[0] != 0) return fail(TOP_E_NONFINITE, "a sweep produced a non-finite value");
  return TOP_OK;
}

top_status top_get_plan(const top_problem* h, top_plan_info* info) {
  if (h == nullptr || info == nullptr) return fail(TOP_E_INVALID, "handle and info must be non-NULL");
  info->tile_lanes = h->plan_ref().W;
  info->n_tiles = h->plan_ref().n_tiles;
  info->halo = h->plan_ref().halo;
  info->n_traj = h->B;
  info->n_seg = h->S;
  info->used_lanes = h->plan_ref().used;
  info->precision = h->opt.precision;
  info->order = h->opt.order;
  info->n_cont = h->opt.n_cont;
  info->iters_done = h->iters_done;
  info->n_fields = h->nf;
  info->ld = h->ld;
  info->lane_form = h->axis ? 3 : 1;
  info->chained = const_cast<top_problem*>(h)->can_chain() ? 1 : 0;
  info->tail_tiles = h->plan_ref().tail_tiles;
  info->tail_tile_lanes = h->plan_ref().tail_W;
  return TOP_OK;
}

top_status top_plan_tiles(int32_t n_traj, const int64_t* seg_offsets, int32_t tile_lanes, int32_t halo,
                          int32_t tiles_per_round, int32_t tail_tile_lanes, int32_t* lanes, int64_t lanes_cap,
                          int32_t* chain, int64_t chain_cap, top_plan_info* info) {
  if (n_traj <= 0 || seg_offsets == nullptr || info == nullptr)
    return fail(TOP_E_INVALID, "n_traj > 0, seg_offsets and info are required");
  if (seg_offsets[0] != 0) return fail(TOP_E_INVALID, "seg_offsets[0] must be 0");
  for (int b = 0; b < n_traj; ++b)
    if (seg_offsets[b + 1] <= seg_offsets[b])
      return fail(TOP_E_INVALID, "trajectory %d has no segment (seg_offsets must increase strictly)", b);
  const int64_t S = seg_offsets[n_traj];
  if (S + n_traj >= (int64_t)top::kHaloBit) return fail(TOP_E_UNSUPPORTED, "too many segments (%lld)", (long long)S);
  if (tile_lanes < 64 || tile_lanes > 512 || tile_lanes % 64 != 0)
    return fail(TOP_E_INVALID, "tile_lanes must be a multiple of 64 in [64, 512] (got %d)", tile_lanes);
  if (halo < 1 || 2 * halo >= tile_lanes)
    return fail(TOP_E_INVALID, "halo must be in [1, tile_lanes / 2) (got %d for %d-lane tiles)", halo, tile_lanes);
  if (tiles_per_round < 0 || (tiles_per_round > 0 && (tail_tile_lanes < 64 || tail_tile_lanes > top::kAxisTileMax ||
                                                      tail_tile_lanes % 64 != 0)))
    return fail(TOP_E_INVALID, "tiles_per_round must be >= 0, and with it tail_tile_lanes a multiple of 64 in [64, %d]",
                top::kAxisTileMax);
  const std::vector<int64_t> off(seg_offsets, seg_offsets + n_traj + 1);
  const Plan pl = make_plan(off, tile_lanes, halo, tiles_per_round, tiles_per_round > 0 ? tail_tile_lanes : 0, 3);
  const size_t n_lanes = pl.lanes.size() + pl.tail.size();
  if (lanes != nullptr && lanes_cap < (int64_t)n_lanes)
    return fail(TOP_E_INVALID, "lanes holds %lld entries; the plan has %zu", (long long)lanes_cap, n_lanes);
  if (chain != nullptr && chain_cap < (int64_t)pl.chain.size())
    return fail(TOP_E_INVALID, "chain holds %lld entries; the plan has %zu", (long long)chain_cap, pl.chain.size());
  *info = top_plan_info{};
  info->tile_lanes = pl.W;
  info->n_tiles = pl.n_tiles;
  info->halo = pl.halo;
  info->n_traj = n_traj;
  info->n_seg = S;
  info->used_lanes = pl.used;
  info->chained = pl.chain.empty() ? 0 : 1;
  info->tail_tiles = pl.tail_tiles;
  info->tail_tile_lanes = pl.tail_W;
  if (lanes != nullptr) {
    std::copy(pl.lanes.begin(), pl.lanes.end(), lanes);
    std::copy(pl.tail.begin(), pl.tail.end(), lanes + pl.lanes.size());
  }
  if (chain != nullptr) std::copy(pl.chain.begin(), pl.chain.end(), chain);
  return TOP_OK;
}

top_status top_get_state(const top_problem* h, void* state) {
  if (h == nullptr || state == nullptr) return fail(TOP_E_INVALID, "handle and state must be non-NULL");
  TOP_HIP(hipMemcpyAsync(state, h->state[h->cur], (size_t)h->nf * h->ld * h->rsz, hipMemcpyDeviceToDevice,
                         h->stream));
  return TOP_OK;
}

top_status top_set_state(top_problem* h, const void* state) {
  if (h == nullptr || state == nullptr) return fail(TOP_E_INVALID, "handle and state must be non-NULL");
  if (h->tape != nullptr) return fail(TOP_E_STATE, "the iterate of a handle that records a tape cannot be replaced");
  TOP_HIP(hipMemcpyAsync(h->state[h->cur], state, (size_t)h->nf * h->ld * h->rsz, hipMemcpyDeviceToDevice,
                         h->stream));
  return TOP_OK;
}

top_status top_tune(top_problem* h, int32_t k_probe) {
  if (h == nullptr) return fail(TOP_E_INVALID, "handle is NULL");
  if (k_probe < 1) return fail(TOP_E_INVALID, "k_probe must be >= 1");
  if (h->explicit_tile) return TOP_OK;
  // The probe sweeps write the state buffer the next sweep will overwrite anyway.  Lanes of stopped
  // trajectories store their unchanged state there (or nothing), so that buffer keeps holding it.
  void* probe_out = h->state[h->cur ^ 1];
  int64_t mx = 0;
  for (int b = 0; b < h->B; ++b) mx = std::max(mx, h->off[b + 1] - h->off[b]);
  std::vector<TuneChoice> cands;   // (W, halo or 0 when nothing is split, lane form)
  auto add = [&](int W, int form) {
    if (mx <= W) cands.push_back({W, 0, form});
    else
      for (int halo : {8, 16, 24, 32})
        if (4 * halo <= W) cands.push_back({W, halo, form});
  };
  for (int W = 64; W <= max_tile(h->v, h->tape != nullptr); W *= 2) add(W, 1);
  if (h->axis_ok)   // one lane per axis: for long trajectories, and small problems
    for (int W = h->v.num ? 64 : 128; W <= axis_tile_max(h->v); W += 64) add(W, 3);
  hipEvent_t e0, e1;
  TOP_HIP(hipEventCreate(&e0));
  TOP_HIP(hipEventCreate(&e1));
  float best = 1e30f, cur_ms = 1e30f;
  const TuneChoice curc{h->plan_ref().W, h->plan_ref().halo, h->axis ? 3 : 1};
  TuneChoice bestc = curc;
  top_status s = TOP_OK;
  // A candidate that would chain is timed as the chained launch an iterate call makes.  Its epochs
  // write both of its state buffers, so it runs on a copy of the iterate in a block taken from the
  // library's pool for the tuning (returned at the end) and the scratch buffer.
  const size_t sbytes = (size_t)h->nf * h->ld * h->rsz;
  void* probe_in = nullptr;
  int probe_dev = 0;
  for (const TuneChoice& c : cands) {
    std::shared_ptr<PlanEntry> cand;
    s = get_plan(h->off, c.W, c.halo > 0 ? c.halo : 1, tail_spec(h->v, h->opt, c.W, c.form), &cand);
    if (s != TOP_OK) break;
    const Plan& pl = cand->plan;
    h->probe_plan = &pl;
    h->probe_axis = c.form == 3;
    const bool chain = h->chains(pl, c.form == 3, k_probe);
    if (chain && probe_in == nullptr) {
      const hipError_t e = pool_get(sbytes, h->stream, &probe_in, &probe_dev);
      if (e != hipSuccess) {
        probe_in = nullptr;
        s = fail(TOP_E_NOMEM, "device allocation of %zu bytes for a tuning probe failed: %s", sbytes,
                 hipGetErrorString(e));
        break;
      }
    }
    float tbest = 1e30f;
    for (int rep = 0; rep < 3 && s == TOP_OK; ++rep) {
      if (chain) {
        hipError_t e = hipMemcpyAsync(probe_in, h->state[h->cur], sbytes, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
        if (e == hipSuccess) e = top::launch_zero_u64(h->chain_flag, pl.n_tiles, h->stream);
        if (e != hipSuccess) {
          s = fail(TOP_E_HIP, "tuning probe set-up failed: %s", hipGetErrorString(e));
          break;
        }
        s = h->sweep_launch(pl, cand->dev, probe_in, probe_out, k_probe, false, h->stream, true, nullptr, true);
      } else {
        const hipError_t e = hipEventRecord(e0, h->stream);
        if (e != hipSuccess) {
          s = fail(TOP_E_HIP, "hipEventRecord failed: %s", hipGetErrorString(e));
          break;
        }
        int remaining = k_probe;
        while (remaining > 0) {
          const int n = pl.halo > 0 ? std::min(remaining, pl.halo) : remaining;
          // probe sweeps read the live state; the iterate is not advanced
          s = h->sweep_launch(pl, cand->dev, h->state[h->cur], probe_out, n, false, h->stream, true);
          if (s != TOP_OK) break;
          remaining -= n;
        }
      }
      if (s != TOP_OK) break;
      float ms = 0.f;
      hipError_t e = hipEventRecord(e1, h->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        s = fail(TOP_E_HIP, "probe timing failed: %s", hipGetErrorString(e));
        break;
      }
      tbest = std::min(tbest, ms);
    }
    h->probe_plan = nullptr;
    if (s != TOP_OK) break;
    if (c.W == curc.W && c.form == curc.form && pl.halo == curc.halo) cur_ms = tbest;
    if (tbest < best) {
      best = tbest;
      bestc = {c.W, pl.halo, c.form};
    }
  }
  // the handle's plan stays unless another is faster by more than the timing noise (3 %)
  if (cur_ms < 1e30f && cur_ms <= 1.03f * best) bestc = curc;
  if (probe_in != nullptr) {   // back to the pool once the probes that used it have run
    (void)hipStreamSynchronize(h->stream);
    pool_put(probe_in, sbytes, probe_dev, h->stream, nullptr);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != TOP_OK) return s;
  s = get_plan(h->off, bestc.W, bestc.halo > 0 ? bestc.halo : std::max(1, std::min(32, bestc.W / 8)),
               tail_spec(h->v, h->opt, bestc.W, bestc.form), &h->pe);
  if (s != TOP_OK) return s;
  h->axis = bestc.form == 3;
  h->drop_graphs();
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[shape_key(h->v, h->off)] = TuneChoice{h->plan_ref().W, h->plan_ref().halo, bestc.form};
    tune_cache_store();
  }
  return TOP_OK;
}


}  // extern "C"

namespace top {
top_status internal_create(int32_t n_traj, const int64_t* seg_offsets, const double* waypoints,
                           const double* durations, const double* bc, const double* box_lo, const double* box_hi,
                           const double* vmax, const double* rho, const top_options* opt, void* workspace,
                           size_t workspace_bytes, hipStream_t stream, top_problem** out, Mem mem) {
  return create_impl(n_traj, seg_offsets, waypoints, durations, bc, box_lo, box_hi, 0, nullptr, vmax, rho, opt,
                     workspace, workspace_bytes, stream, out, mem);
}

top_status internal_error(top_status s, const char* text) { return fail(s, "%s", text); }
}  // namespace top
