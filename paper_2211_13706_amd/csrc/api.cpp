// C ABI of libposetx (declared in include/posetx.h): poset handles, device
// upload, workspaces and the drivers that sequence the kernels of one
// transform on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "kernels.h"
#include "niv_device.h"
#include "noalloc.h"
#include "posetx.h"
#include "prep.h"

namespace {

thread_local std::string g_err;

px_status fail(px_status s, const std::string& m) {
  g_err = m;
  return s;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Makes `dev` current for the scope of a call and restores the caller's device.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

template <typename T>
hipError_t upload(T** dst, const T* src, size_t count, int64_t& bytes) {
  *dst = nullptr;
  if (count == 0) return hipSuccess;
  hipError_t e = hipMalloc((void**)dst, count * sizeof(T));
  if (e != hipSuccess) return e;
  bytes += count * sizeof(T);
  return hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice);
}

size_t elem_size(int dtype) { return dtype == PX_F32 ? 4 : 8; }
px::ElemType etype(int dtype) { return dtype == PX_I64 ? px::E_I64 : dtype == PX_F32 ? px::E_F32 : px::E_F64; }
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Grow-only device workspace.
struct Workspace {
  void* p = nullptr;
  size_t bytes = 0;
  px_status ensure(size_t need) {
    if (need <= bytes) return PX_OK;
    if (p) {
      (void)hipDeviceSynchronize();
      (void)hipFree(p);
      p = nullptr;
      bytes = 0;
    }
    if (hipMalloc(&p, need) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return fail(PX_ENOMEM, "device workspace allocation of " + std::to_string(need) + " bytes failed");
    }
    bytes = need;
    return PX_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

// Tile offsets of the chain scan for each of the 7 tile heights.
void seg_tables(const std::vector<int32_t>& chain_off, std::vector<int32_t>& segoff, int64_t ntiles[7]) {
  const int64_t nc = (int64_t)chain_off.size() - 1;
  segoff.assign(7 * (nc + 1), 0);
  for (int i = 0; i < 7; ++i) {
    const int64_t seg = px::seg_rows(1 << i);
    int32_t* so = &segoff[i * (nc + 1)];
    for (int64_t c = 0; c < nc; ++c) {
      int64_t len = chain_off[c + 1] - chain_off[c];
      so[c + 1] = so[c] + (int32_t)((len + seg - 1) / seg);
    }
    ntiles[i] = so[nc];
  }
}

// Tile heights (bit i: seg_rows(1 << i), narrow blocks only) whose scan takes
// flat tiles (rows in fixed blocks, chain starts resetting the sum): where
// chain-aligned tiles would be at most 80% full and no chain spans more than
// 64 flat tiles (the carry of a flat tile folds the earlier tiles of its chain).
uint32_t flat_mask(int64_t n, int32_t max_chain, const int64_t ntiles[7], const int32_t max_chain_tiles[7]) {
  uint32_t m = 0;
  for (int i = 0; i < 6; ++i) {
    const int64_t H = px::seg_rows(1 << i);
    const int64_t nft = (n + H - 1) / H;
    if (max_chain_tiles[i] > 1 && 5 * nft <= 4 * ntiles[i] && max_chain <= 64 * H) m |= 1u << i;
  }
  return m;
}

// For each tile height (as seg_tables): {first row, end row of its chain} of
// every tile, concatenated over the heights, and the most tiles of any chain.
std::vector<int32_t> tile_tables(const std::vector<int32_t>& chain_off, int64_t off[8], int32_t maxt[7]) {
  const int64_t nc = (int64_t)chain_off.size() - 1;
  std::vector<int32_t> t;
  for (int i = 0; i < 7; ++i) {
    const int64_t seg = px::seg_rows(1 << i);
    off[i] = (int64_t)t.size() / 2;
    maxt[i] = 0;
    for (int64_t c = 0; c < nc; ++c) {
      const int64_t nt = (chain_off[c + 1] - chain_off[c] + seg - 1) / seg;
      maxt[i] = std::max<int32_t>(maxt[i], (int32_t)nt);
      for (int64_t r = chain_off[c]; r < chain_off[c + 1]; r += seg) {
        t.push_back((int32_t)r);
        t.push_back(chain_off[c + 1]);
      }
    }
  }
  off[7] = (int64_t)t.size() / 2;
  return t;
}

// Runs of the walking gather for one niv map (see px::WalkTables).  Every chain
// is cut into runs of at most T rows (T <= 255) and at most `emax` change
// events, so that no wavefront's serial event work is much longer than the
// average; the runs are then ordered by the relative height of their middle
// inside their chain (ties by chain), so that the waves resident together
// gather from one height band of every chain.  Defaults; px_autotune picks
// per poset and B.
constexpr int kWalkT = 128;
constexpr int kWalkEvents = 96;

// Host threads of the table builders (walk, compact and run tables): up to 16
// for posets of 2^15 rows or more; POSETX_PREP_THREADS overrides (1..64).
// The tables do not depend on the thread count.
int table_threads(int64_t n) {
  if (const char* v = std::getenv("POSETX_PREP_THREADS")) {
    const int t = std::atoi(v);
    if (t >= 1) return std::min(t, 64);
  }
  if (n < (1 << 15)) return 1;
  const unsigned hc = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(16u, hc ? hc : 1u));
}

// fn(t, lo, hi) over [0, count) in nt contiguous ascending parts, part t on
// thread t (part 0 on the caller's thread).
template <typename F>
void parallel_for(int64_t count, int nt, const F& fn) {
  nt = (int)std::max<int64_t>(1, std::min<int64_t>(nt, count));
  if (nt <= 1) {
    if (count > 0) fn(0, (int64_t)0, count);
    return;
  }
  const int64_t part = (count + nt - 1) / nt;
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) {
    const int64_t lo = t * part, hi = std::min(count, lo + part);
    if (lo < hi) th.emplace_back([&fn, t, lo, hi] { fn(t, lo, hi); });
  }
  fn(0, (int64_t)0, std::min(count, part));
  for (auto& x : th) x.join();
}

// The other-chain entries of every row that differ from the row below it in
// its chain (0 for a chain's first row).
std::vector<int32_t> row_changes(const px::Prep& P, const std::vector<int32_t>& nv, int nt) {
  const int64_t n = P.n, k = P.k;
  std::vector<int32_t> cnt(n, 0);
  parallel_for(n, nt, [&](int, int64_t lo, int64_t hi) {
    for (int64_t r = lo; r < hi; ++r) {
      const int32_t c = P.chain_of_row[r];
      if (r == P.chain_off[c]) continue;
      const int32_t* a = &nv[(size_t)r * k];
      const int32_t* b = a - k;
      int e = 0;
      for (int64_t j = 0; j < k; ++j) e += (j != c && a[j] != b[j]);
      cnt[r] = e;
    }
  });
  return cnt;
}

struct HostWalk {
  std::vector<int32_t> runs;  // pairs (r0, r1)
  std::vector<int32_t> ev;    // quadruples (new row, old row, (u << 8) | chain, 0), -1 = none
  std::vector<int32_t> ev_off, snap_off, snap_of_row;
  int32_t nsnap = 0;
  int64_t rows_distinct = 0, row_loads = 0;  // P rows the event kernel reads: distinct, and loads
};

void build_walk(const px::Prep& P, const std::vector<int32_t>& nv, HostWalk& W, int T, int emax) {
  const int64_t k = P.k, n = P.n;
  const int nt = table_threads(n);
  const std::vector<int32_t> ch = row_changes(P, nv, nt);
  struct Run {
    double h;
    int32_t c, r0, r1;
  };
  // runs chain by chain (each thread a contiguous range of chains, joined in order)
  std::vector<std::vector<Run>> part(std::max(1, nt));
  parallel_for(k, nt, [&](int t, int64_t c0, int64_t c1) {
    for (int64_t c = c0; c < c1; ++c) {
      const int32_t lo = P.chain_off[c], hi = P.chain_off[c + 1];
      int32_t r = lo;
      while (r < hi) {
        const int32_t r0 = r++;
        int ev = 0;
        while (r < hi && r - r0 < T) {
          const int e = ch[r];
          if (ev + e > emax && r > r0 + 1) break;
          ev += e;
          ++r;
        }
        part[t].push_back({(0.5 * (r0 + r) - lo) / (double)(hi - lo), (int32_t)c, r0, r});
      }
    }
  });
  std::vector<Run> runs;
  for (auto& v : part) runs.insert(runs.end(), v.begin(), v.end());
  std::stable_sort(runs.begin(), runs.end(), [](const Run& x, const Run& y) { return x.h < y.h; });
  const size_t nr = runs.size();
  W.runs.resize(2 * nr);
  W.ev_off.assign(nr + 1, 0);
  W.snap_off.assign(nr + 1, 0);
  W.snap_of_row.assign(n, 0);
  // events and snapshots per run, then their offsets
  for (size_t s = 0; s < nr; ++s) {
    int64_t e = 0, m = 1;  // the first row's snapshot, then one per row with events
    for (int32_t r = runs[s].r0 + 1; r < runs[s].r1; ++r) {
      e += ch[r];
      m += ch[r] > 0;
    }
    W.ev_off[s + 1] = (int32_t)(W.ev_off[s] + e);
    W.snap_off[s + 1] = (int32_t)(W.snap_off[s] + m);
  }
  W.ev.assign(4 * (size_t)W.ev_off[nr], 0);
  parallel_for((int64_t)nr, nt, [&](int, int64_t s0, int64_t s1) {
    for (int64_t s = s0; s < s1; ++s) {
      const Run& R = runs[s];
      W.runs[2 * s] = R.r0;
      W.runs[2 * s + 1] = R.r1;
      int32_t cur = W.snap_off[s];
      size_t o = 4 * (size_t)W.ev_off[s];
      W.snap_of_row[R.r0] = cur;
      for (int32_t r = R.r0 + 1; r < R.r1; ++r) {
        const int32_t* a = &nv[(size_t)r * k];
        const int32_t* b = &nv[(size_t)(r - 1) * k];
        for (int64_t j = 0; j < k; ++j)
          if (j != R.c && a[j] != b[j]) {
            W.ev[o++] = a[j];
            W.ev[o++] = b[j];
            W.ev[o++] = ((r - R.r0) << 8) | (int32_t)std::min<int64_t>(j, 255);
            W.ev[o++] = 0;
          }
        if (ch[r] > 0) ++cur;
        W.snap_of_row[r] = cur;
      }
    }
  });
  const int32_t m = W.snap_off[nr];
  W.nsnap = m;
  // P rows read by the event kernel: the other-chain entries of every run's
  // first row, and the new and old rows of every event
  std::vector<char> seen(n, 0);
  W.row_loads = 0;
  auto touch = [&](int32_t t) {
    if (t < 0) return;
    ++W.row_loads;
    seen[t] = 1;
  };
  for (size_t s = 0; s < runs.size(); ++s) {
    const int32_t r0 = runs[s].r0;
    for (int64_t j = 0; j < k; ++j)
      if (j != runs[s].c) touch(nv[(size_t)r0 * k + j]);
  }
  for (size_t e = 0; e < W.ev.size(); e += 4) {
    touch(W.ev[e]);
    touch(W.ev[e + 1]);
  }
  W.rows_distinct = 0;
  for (char c : seen) W.rows_distinct += c;
}

// Compact form of a walk (see px::WalkTables): the gathered rows numbered in
// row order inside the 64-row tiles of the 64-column scan, and the walk's
// first-row entries and events with slots instead of rows.
struct HostCompact {
  std::vector<uint64_t> tmask;
  std::vector<int32_t> qoff, tile_of_slot, init, evq;
  int32_t nslots = 0;
};

void build_compact(const px::Prep& P, const std::vector<int32_t>& nv, const HostWalk& W, HostCompact& H) {
  const int64_t k = P.k, seg = px::seg_rows(64);
  std::vector<int64_t> so(k + 1, 0);  // first tile of each chain
  for (int64_t c = 0; c < k; ++c) so[c + 1] = so[c] + (P.chain_off[c + 1] - P.chain_off[c] + seg - 1) / seg;
  const int64_t nt = so[k];
  auto tile_bit = [&](int32_t r, int64_t& t, int& b) {
    const int32_t c = P.chain_of_row[r];
    const int64_t pos = r - P.chain_off[c];
    t = so[c] + pos / seg;
    b = (int)(pos % seg);
  };
  const size_t nruns = W.runs.size() / 2;
  H.tmask.assign(nt, 0);
  auto mark = [&](int32_t r) {
    if (r < 0) return;
    int64_t t;
    int b;
    tile_bit(r, t, b);
    H.tmask[t] |= uint64_t(1) << b;
  };
  for (size_t s = 0; s < nruns; ++s) {
    const int32_t r0 = W.runs[2 * s], c = P.chain_of_row[r0];
    for (int64_t j = 0; j < k; ++j)
      if (j != c) mark(nv[(size_t)r0 * k + j]);
  }
  for (size_t e = 0; e < W.ev.size(); e += 4) {
    mark(W.ev[e]);
    mark(W.ev[e + 1]);
  }
  H.qoff.assign(nt + 1, 0);
  for (int64_t t = 0; t < nt; ++t) H.qoff[t + 1] = H.qoff[t] + __builtin_popcountll(H.tmask[t]);
  H.nslots = H.qoff[nt];
  H.tile_of_slot.resize(H.nslots);
  for (int64_t t = 0; t < nt; ++t)
    for (int32_t q = H.qoff[t]; q < H.qoff[t + 1]; ++q) H.tile_of_slot[q] = (int32_t)t;
  auto slot = [&](int32_t r) -> int32_t {
    if (r < 0) return H.nslots;
    int64_t t;
    int b;
    tile_bit(r, t, b);
    return H.qoff[t] + __builtin_popcountll(H.tmask[t] & ((uint64_t(1) << b) - 1));
  };
  H.init.assign(nruns * k, H.nslots);
  for (size_t s = 0; s < nruns; ++s) {
    const int32_t r0 = W.runs[2 * s], c = P.chain_of_row[r0];
    for (int64_t j = 0; j < k; ++j)
      if (j != c) H.init[s * k + j] = slot(nv[(size_t)r0 * k + j]);
  }
  H.evq = W.ev;
  for (size_t e = 0; e < H.evq.size(); e += 4) {
    H.evq[e] = slot(W.ev[e]);
    H.evq[e + 1] = slot(W.ev[e + 1]);
  }
}

// Every index the compact kernels derive from the tables stays inside Q, L
// and the tile arrays: slots counted per tile agree with the masks, every
// slot's tile holds it, and the walk names slots 0..nslots only.
bool compact_consistent(const HostCompact& H, int64_t ntiles) {
  const int64_t nt = (int64_t)H.tmask.size();
  if (nt != ntiles || (int64_t)H.qoff.size() != nt + 1 || H.qoff[0] != 0 || H.qoff[nt] != H.nslots) return false;
  for (int64_t t = 0; t < nt; ++t)
    if (H.qoff[t + 1] - H.qoff[t] != __builtin_popcountll(H.tmask[t])) return false;
  if ((int64_t)H.tile_of_slot.size() != H.nslots) return false;
  for (int32_t q = 0; q < H.nslots; ++q) {
    const int32_t t = H.tile_of_slot[q];
    if (t < 0 || t >= nt || q < H.qoff[t] || q >= H.qoff[t + 1]) return false;
  }
  for (int32_t v : H.init)
    if (v < 0 || v > H.nslots) return false;
  for (size_t e = 0; e < H.evq.size(); e += 4)
    if (H.evq[e] < 0 || H.evq[e] > H.nslots || H.evq[e + 1] < 0 || H.evq[e + 1] > H.nslots) return false;
  return true;
}

// Tile orders of the single-pass scan: for each tile height and direction, the
// tiles sorted by their position in the scan (from the bottom for prefix scans,
// from the top for suffix scans), then by chain.
std::vector<int32_t> scan_orders(const std::vector<int32_t>& segoff, int64_t nchains, const int64_t ntiles[7]) {
  std::vector<int32_t> out;
  for (int dir = 0; dir < 2; ++dir)
    for (int i = 0; i < 7; ++i) {
      const int32_t* so = &segoff[i * (nchains + 1)];
      std::vector<std::pair<int64_t, int32_t>> key;
      key.reserve(ntiles[i]);
      for (int64_t c = 0; c < nchains; ++c)
        for (int32_t t = so[c]; t < so[c + 1]; ++t) {
          const int32_t q = t - so[c], nq = so[c + 1] - so[c];
          key.push_back({(int64_t)(dir == 0 ? q : nq - 1 - q) * nchains + c, t});
        }
      std::sort(key.begin(), key.end());
      for (auto& kv : key) out.push_back(kv.second);
    }
  return out;
}

struct Layout {
  size_t y = 0, p64 = 0, r64 = 0, aux = 0, stats = 0, snaps = 0, sync = 0, lq = 0, part = 0, flow = 0, total = 0;
};

// Workspace layout of one call: a [n, B] matrix of the working type (P or Y),
// for float32 refinement two float64 [n, B] matrices (P64 and the residual),
// the scan's tile states and the refinement statistics.  nparts: chunk sums
// of the split long rows of a sparse level solve (8 bytes per column).
// With nslots >= 0 also the compact walk's L and Q ((2 * nslots + 1) rows of
// the working type: float64 for the residual of a refinement).  nflow: ints of
// the persistent int64 solve's error word and ready flags.
Layout layout(int64_t n, int64_t B, int dtype, bool refine, int64_t ntiles, int64_t nsnap = 0,
              int64_t nslots = -1, int64_t nparts = 0, int64_t nflow = 0) {
  Layout L;
  size_t o = 0;
  L.y = o;  // one row more: the scan's zero row
  o = align256(o + (size_t)(n + 1) * B * elem_size(dtype));
  if (refine) {
    L.p64 = o;
    o = align256(o + (size_t)(n + 1) * B * 8);
    L.r64 = o;
    o = align256(o + (size_t)n * B * 8);
  }
  L.aux = o;
  o = align256(o + (size_t)ntiles * B * 16 * 2);
  L.stats = o;
  o = align256(o + (size_t)(2 * B + 1) * 8);
  L.snaps = o;
  o = align256(o + (size_t)nsnap * B * (refine ? 8 : elem_size(dtype)));
  L.sync = o;
  o = align256(o + (size_t)(2 + ntiles * ((B + px::col_width(B) - 1) / px::col_width(B))) * 4);
  L.lq = o;
  if (nslots >= 0) o = align256(o + (size_t)(2 * nslots + 1) * B * (refine ? 8 : elem_size(dtype)));
  L.part = o;
  o = align256(o + (size_t)nparts * B * 8);
  L.flow = o;
  o = align256(o + (size_t)nflow * 4);
  L.total = o;
  return L;
}

px_status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return PX_OK;
  return fail(PX_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Opt-in per-kernel timing with HIP events recorded on the launch stream
// (px_profile / px_profile_read).  Off by default: then it costs one branch.
namespace prof {
enum Phase { SCAN_REDUCE = 0, SCAN_CARRY, SCAN_APPLY, GATHER, USOLVE, CHAIN_DIFF, ABSMAX, WALK_EVENTS, WALK_COMBINE,
             SCAN_ONEPASS, APPLY_COMBINE, NPH };
const char* const kNames[NPH] = {"scan_reduce", "scan_carry",   "scan_apply",  "gather",
                                 "usolve_level", "chain_diff",  "absmax",      "walk_events",
                                 "walk_combine", "scan_onepass", "apply_combine"};
std::mutex mu;
std::atomic<bool> on{false};
struct Rec {
  int ph;
  hipEvent_t a, b;
};
std::vector<Rec> pending;
double ms[NPH];
int64_t cnt[NPH];

void drain() {
  for (Rec& r : pending) {
    float t = 0;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
      ms[r.ph] += t;
      cnt[r.ph] += 1;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  pending.clear();
}

struct Scope {
  int ph;
  hipStream_t s;
  hipEvent_t a = nullptr;
  Scope(int p, hipStream_t st) : ph(p), s(st) {
    if (on && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, s);
  }
  ~Scope() {
    if (!a) return;
    hipEvent_t b;
    if (hipEventCreate(&b) != hipSuccess) return;
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(mu);
    pending.push_back({ph, a, b});
  }
};
// Times the two kernels of the walking gather separately.
struct WalkHook : px::LaunchHook {
  Scope* sc[2] = {nullptr, nullptr};
  void before(int k, hipStream_t s) override { sc[k] = new Scope(k ? WALK_COMBINE : WALK_EVENTS, s); }
  void after(int k, hipStream_t) override {
    delete sc[k];
    sc[k] = nullptr;
  }
};
// Times the four kernels of the compact walk.
struct CompactHook : px::LaunchHook {
  Scope* sc[4] = {nullptr, nullptr, nullptr, nullptr};
  void before(int k, hipStream_t s) override {
    static const int ph[4] = {SCAN_REDUCE, SCAN_CARRY, WALK_EVENTS, APPLY_COMBINE};
    sc[k] = new Scope(ph[k], s);
  }
  void after(int k, hipStream_t) override {
    delete sc[k];
    sc[k] = nullptr;
  }
};
}  // namespace prof

// Polls per look-back wait of the single-pass scan (about 30 ms by default;
// POSETX_LB_SPIN overrides it, e.g. 0 to exercise the direct-sum fallback).
int lb_spin_limit() {
  const char* v = std::getenv("POSETX_LB_SPIN");
  if (v && *v) return (int)std::min<long>(std::max<long>(std::strtol(v, nullptr, 10), 0), 1 << 30);
  return 1 << 16;
}

// The reduce / carry / apply scan is the default: at n = 2^20, k = 64, B = 64
// it takes 0.18 ms against 0.27 ms for the single-pass scan, whose tiles wait
// on their predecessors' flags.  POSETX_SCAN=onepass selects the single-pass
// scan (read on every call).
bool use_onepass() {
  const char* v = std::getenv("POSETX_SCAN");
  return v && std::strcmp(v, "onepass") == 0;
}

hipError_t run_scan(const px::DevPoset& d, int dir, px::ElemType tin, const void* x, int64_t ldx, px::ElemType tout,
                    void* P, int64_t B, void* aux, int64_t nt, int* sync, hipStream_t s) {
  if (sync && use_onepass() && d.scan_order[dir > 0 ? 0 : 1][px::seg_index(px::col_width(B))]) {
    prof::Scope sc(prof::SCAN_ONEPASS, s);
    return px::launch_chain_scan_onepass(d, dir, tin, x, ldx, tout, P, B, aux, nt, sync, lb_spin_limit(), s);
  }
  hipError_t e;
  {
    prof::Scope sc(prof::SCAN_REDUCE, s);
    e = px::launch_chain_scan_phase(0, d, dir, tin, x, ldx, tout, P, B, aux, nt, s);
  }
  if (e != hipSuccess) return e;
  {
    prof::Scope sc(prof::SCAN_CARRY, s);
    e = px::launch_chain_scan_phase(1, d, dir, tin, x, ldx, tout, P, B, aux, nt, s);
  }
  if (e != hipSuccess) return e;
  prof::Scope sc(prof::SCAN_APPLY, s);
  return px::launch_chain_scan_phase(2, d, dir, tin, x, ldx, tout, P, B, aux, nt, s);
}

hipError_t run_gather(const px::DevPoset& d, bool up, px::ElemType tp, const void* P, int64_t B, px::ElemType tout,
                      void* out, int64_t ldo, px::ElemType tres, const void* resid, int64_t ldr, void* snaps,
                      hipStream_t s) {
  if (prof::on) {
    prof::WalkHook hook;
    if (snaps && !d.nivp[up ? 1 : 0])
      return px::launch_gather(d, up, tp, P, B, tout, out, ldo, tres, resid, ldr, snaps, &hook, s);
    prof::Scope sc(prof::GATHER, s);  // (sparse rows: snaps holds the split gather's chunk sums)
    return px::launch_gather(d, up, tp, P, B, tout, out, ldo, tres, resid, ldr, snaps, nullptr, s);
  }
  return px::launch_gather(d, up, tp, P, B, tout, out, ldo, tres, resid, ldr, snaps, nullptr, s);
}

// The compact walk is the default wherever it applies (single poset, k <= 64,
// 64-column blocks); POSETX_WALK=rows (read on every call) selects the
// scan that writes P and the walk over P instead.
bool compact_enabled() {
  const char* v = std::getenv("POSETX_WALK");
  return !(v && std::strcmp(v, "rows") == 0);
}

hipError_t run_compact(const px::DevPoset& d, int dir, px::ElemType tin, const void* x, int64_t ldx,
                       px::ElemType tout, void* out, int64_t ldo, px::ElemType tres, const void* resid, int64_t ldr,
                       int64_t B, void* aux, int64_t nt, void* lq, void* snaps, hipStream_t s) {
  if (prof::on) {
    prof::CompactHook hook;
    return px::launch_zeta_compact(d, dir, tin, x, ldx, tout, out, ldo, tres, resid, ldr, B, aux, nt, lq, snaps,
                                   &hook, s);
  }
  return px::launch_zeta_compact(d, dir, tin, x, ldx, tout, out, ldo, tres, resid, ldr, B, aux, nt, lq, snaps,
                                 nullptr, s);
}

hipError_t run_chain_diff(const px::DevPoset& d, int dir, px::ElemType ty, const void* Y, int64_t B,
                          px::ElemType tout, void* out, int64_t ldo, bool acc, uint64_t* stats, hipStream_t s) {
  prof::Scope sc(prof::CHAIN_DIFF, s);
  return px::launch_chain_diff(d, dir, ty, Y, B, tout, out, ldo, acc, stats, s);
}

}  // namespace

struct px_poset {
  px::Prep prep;
  int device = 0;
  bool host_only = false, has_up = false, mirsky = false;
  int32_t *d_node_of_row = nullptr, *d_chain_of_row = nullptr, *d_chain_off = nullptr, *d_niv = nullptr,
          *d_niv_up = nullptr, *d_lev_down = nullptr, *d_lev_up = nullptr, *d_segoff = nullptr, *d_order = nullptr,
          *d_tiles = nullptr, *d_lev_niv[2] = {nullptr, nullptr}, *d_lev_node[2] = {nullptr, nullptr},
          *d_walk[2][5] = {{nullptr, nullptr, nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr, nullptr, nullptr}};
  int32_t* d_nivr[2] = {nullptr, nullptr};  // sparse niv rows: entries and row offsets
  // function-matrix layout (px_poset_set_layout); with rows, dp addresses user
  // matrices through the identity d_iota instead of node_of_row
  uint32_t layout = PX_LAYOUT_NODES;
  int32_t* d_iota = nullptr;
  // int64 level solve by runs: change events and per-level chunks (px::SegTables)
  int4* d_run_ev[2] = {nullptr, nullptr};
  int4* d_run_chunks[2] = {nullptr, nullptr};
  std::vector<int64_t> run_cptr[2];  // per level: offsets into d_run_chunks
  int64_t run_events[2] = {0, 0};
  int32_t* d_run_levn[2] = {nullptr, nullptr};  // per level: its first chunk (levels + 1 entries)
  // per level: its first position in d_lev_down / d_lev_up (levels + 1 entries; dense rows)
  int32_t* d_lev_ptr[2] = {nullptr, nullptr};
  uint64_t* d_lev_bits[2] = {nullptr, nullptr};  // bit p: position p starts a level
  int32_t* d_run_dep_ptr[2] = {nullptr, nullptr};  // per chunk: the chunks it reads from
  int32_t* d_run_deps[2] = {nullptr, nullptr};
  int64_t* d_nivp[2] = {nullptr, nullptr};
  int64_t ntiles[7] = {0, 0, 0, 0, 0, 0, 0};
  int64_t nevents[2] = {0, 0};
  int32_t nsnap[2] = {0, 0};
  std::vector<int32_t> hw_runs[2], hw_ev[2], hw_ev_off[2], hw_snap_off[2], hw_snap_of_row[2];
  int32_t walk_T = 0, walk_emax = 0;
  int64_t walk_rows[2][2] = {{0, 0}, {0, 0}};  // per map: distinct P rows read, P-row loads
  // compact walk tables per map (tmask, qoff, tile_of_slot, init, evq); nslots
  // is -1 where the map has none
  void* d_compact[2][5] = {{nullptr, nullptr, nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr, nullptr, nullptr}};
  int32_t nslots[2] = {-1, -1};
  // sparse level solves: per level, the short rows, and the long rows split
  // into chunks of consecutive entries (kSplitChunk), per map
  struct Split {
    bool on = false;
    std::vector<int32_t> sptr, lptr, cptr;  // per level: offsets into d_short, d_long, d_items
    int32_t* d_short = nullptr;
    int4* d_long = nullptr;
    int4* d_items = nullptr;
    int64_t max_items = 0;
    // the zeta gather's split (all rows at once)
    int32_t* d_gshort = nullptr;
    int4* d_glong = nullptr;
    int4* d_gitems = nullptr;
    int4* d_gitems8 = nullptr;
    int64_t gitems = 0;
  } split[2];
  px::DevPoset dp;
  Workspace ws;
  int64_t device_bytes = 0;
  double t_upload = 0;
};

struct px_batch {
  int device = 0;
  int count = 0;
  int64_t rows = 0;
  bool has_up = false;
  int32_t *d_node_of_row = nullptr, *d_chain_of_row = nullptr, *d_chain_off = nullptr, *d_niv = nullptr,
          *d_niv_up = nullptr, *d_segoff = nullptr, *d_tiles = nullptr, *d_poset_of_row = nullptr, *d_k = nullptr, *d_row_off = nullptr,
          *d_order = nullptr;
  int64_t* d_niv_off = nullptr;
  int32_t* d_walk[2][5] = {{nullptr, nullptr, nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr, nullptr, nullptr}};
  int32_t nsnap[2] = {0, 0};
  int64_t ntiles[7] = {0, 0, 0, 0, 0, 0, 0};
  std::vector<int32_t> node_of_row;  // batch node (poset offset + node) of every batch row
  uint32_t layout = PX_LAYOUT_NODES;  // px_batch_set_layout
  int32_t* d_iota = nullptr;          // identity row table of the row layout
  px::DevPoset dp;
  Workspace ws;
};

namespace {

void free_poset_device(px_poset* p) {
  int32_t* bufs[] = {p->d_node_of_row, p->d_chain_of_row, p->d_chain_off, p->d_niv, p->d_niv_up,
                     p->d_lev_down,     p->d_lev_up,       p->d_segoff,    p->d_order, p->d_tiles,
                     p->d_lev_niv[0],   p->d_lev_niv[1],   p->d_lev_node[0], p->d_lev_node[1], p->d_iota,
                     p->d_nivr[0],      p->d_nivr[1],      p->d_lev_ptr[0], p->d_lev_ptr[1]};
  for (int32_t* b : bufs)
    if (b) (void)hipFree(b);
  for (int64_t* b : p->d_nivp)
    if (b) (void)hipFree(b);
  for (uint64_t*& b : p->d_lev_bits) {
    if (b) (void)hipFree(b);
    b = nullptr;
  }
  for (int m = 0; m < 2; ++m) {
    if (p->d_run_ev[m]) (void)hipFree(p->d_run_ev[m]);
    if (p->d_run_chunks[m]) (void)hipFree(p->d_run_chunks[m]);
    if (p->d_run_levn[m]) (void)hipFree(p->d_run_levn[m]);
    if (p->d_run_dep_ptr[m]) (void)hipFree(p->d_run_dep_ptr[m]);
    if (p->d_run_deps[m]) (void)hipFree(p->d_run_deps[m]);
    p->d_run_ev[m] = p->d_run_chunks[m] = nullptr;
    p->d_run_levn[m] = p->d_run_dep_ptr[m] = p->d_run_deps[m] = nullptr;
  }
  for (auto& sp : p->split) {
    if (sp.d_short) (void)hipFree(sp.d_short);
    if (sp.d_long) (void)hipFree(sp.d_long);
    if (sp.d_items) (void)hipFree(sp.d_items);
    if (sp.d_gshort) (void)hipFree(sp.d_gshort);
    if (sp.d_glong) (void)hipFree(sp.d_glong);
    if (sp.d_gitems) (void)hipFree(sp.d_gitems);
    if (sp.d_gitems8) (void)hipFree(sp.d_gitems8);
    sp = px_poset::Split();
  }
  for (auto& dir : p->d_walk)
    for (int32_t*& b : dir)
      if (b) {
        (void)hipFree(b);
        b = nullptr;
      }
  for (auto& dir : p->d_compact)
    for (void*& b : dir)
      if (b) {
        (void)hipFree(b);
        b = nullptr;
      }
  p->ws.release();
}

px_status check_matrix_args(int64_t n, int dtype, const void* a, int64_t lda, const void* b, int64_t ldb,
                            int64_t B) {
  if (dtype != PX_I64 && dtype != PX_F32 && dtype != PX_F64) return fail(PX_EINVAL, "unknown dtype");
  if (B < 1) return fail(PX_EINVAL, "B must be >= 1");
  if (B > (int64_t)65535 * 64) return fail(PX_EINVAL, "B too large");
  if (lda < B || ldb < B) return fail(PX_EINVAL, "leading dimension smaller than B");
  if (n > 0 && (!a || !b)) return fail(PX_EINVAL, "null function matrix");
  return PX_OK;
}

int64_t max_slots(const px_poset* p) { return std::max(p->nslots[0], p->nslots[1]); }
int64_t max_parts(const px_poset* p) {
  return std::max({p->split[0].max_items, p->split[1].max_items, p->split[0].gitems, p->split[1].gitems});
}

// Entries per chunk of a split long row in a sparse level solve: a level waits
// for its longest row, and the rows of the last levels of a wide poset are
// long (thousands of entries in a handful of rows).
constexpr int64_t kSplitChunk = 256;

// Short rows and chunks of the long ones among rows[0 .. cnt) (host side).
// A row's chunks take consecutive slots (item.w, relative to the first item
// added here; longs[j].y is its first slot).  With by_entry the items are
// then ordered by the row of their first entry, so that chunks gathered
// together read nearby rows.  On the n = 2^18 ER DAG at B = 64 this made the
// int64 level solve 12% and the float64 residual gather about 10% faster but
// the float32 zeta gather 1.5% slower, so the gather keeps both orders and
// takes the ordered one for 8-byte elements.
void split_rows(const std::vector<int64_t>& ep, const std::vector<int32_t>& er, const int32_t* rows, int64_t cnt,
                bool by_entry, std::vector<int32_t>& shorts, std::vector<int4>& longs, std::vector<int4>& items) {
  const size_t c0 = items.size();
  for (int64_t i = 0; i < cnt; ++i) {
    const int32_t r = rows ? rows[i] : (int32_t)i;
    const int64_t e0 = ep[r], e1 = ep[r + 1];
    if (e1 - e0 <= kSplitChunk) {
      shorts.push_back(r);
      continue;
    }
    const int32_t first = (int32_t)(items.size() - c0);
    for (int64_t e = e0; e < e1; e += kSplitChunk) {
      const int32_t w = (int32_t)(items.size() - c0);
      items.push_back(make_int4(r, (int32_t)e, (int32_t)std::min(e + kSplitChunk, e1), w));
    }
    longs.push_back(make_int4(r, first, (int32_t)(items.size() - c0) - first, 0));
  }
  if (by_entry)
    std::stable_sort(items.begin() + c0, items.end(), [&](const int4& a, const int4& b) { return er[a.y] < er[b.y]; });
}

// The split schedules of map m of a sparse poset: per level for the solve,
// and over all rows for the zeta gather.
void build_split(const px::Prep& P, int m, px_poset::Split& sp, px::GatherSplit& gs) {
  const std::vector<int32_t>& lptr = m ? P.lev_up_ptr : P.lev_down_ptr;
  const std::vector<int32_t>& rows = m ? P.lev_up_rows : P.lev_down_rows;
  const std::vector<int64_t>& ep = P.nivp[m];
  std::vector<int32_t> shorts;
  std::vector<int4> longs, items;
  sp.sptr.assign(1, 0);
  sp.lptr.assign(1, 0);
  sp.cptr.assign(1, 0);
  sp.max_items = 0;
  for (size_t l = 0; l + 1 < lptr.size(); ++l) {
    const size_t c0 = items.size();
    split_rows(ep, P.nivr[m], rows.data() + lptr[l], lptr[l + 1] - lptr[l], true, shorts, longs, items);
    sp.sptr.push_back((int32_t)shorts.size());
    sp.lptr.push_back((int32_t)longs.size());
    sp.cptr.push_back((int32_t)items.size());
    sp.max_items = std::max<int64_t>(sp.max_items, (int64_t)(items.size() - c0));
  }
  sp.on = true;
  int64_t b = 0;
  hipError_t e = upload(&sp.d_short, shorts.data(), shorts.size(), b);
  if (e == hipSuccess) e = upload(&sp.d_long, longs.data(), longs.size(), b);
  if (e == hipSuccess) e = upload(&sp.d_items, items.data(), items.size(), b);
  if (e != hipSuccess) {
    sp.on = false;
    return;
  }
  shorts.clear();
  longs.clear();
  items.clear();
  split_rows(ep, P.nivr[m], nullptr, P.n, false, shorts, longs, items);
  e = upload(&sp.d_gshort, shorts.data(), shorts.size(), b);
  if (e == hipSuccess) e = upload(&sp.d_glong, longs.data(), longs.size(), b);
  if (e == hipSuccess) e = upload(&sp.d_gitems, items.data(), items.size(), b);
  if (e == hipSuccess) {
    std::stable_sort(items.begin(), items.end(),
                     [&](const int4& a, const int4& c) { return P.nivr[m][a.y] < P.nivr[m][c.y]; });
    e = upload(&sp.d_gitems8, items.data(), items.size(), b);
  }
  if (e != hipSuccess) return;
  sp.gitems = (int64_t)items.size();
  gs.shorts = sp.d_gshort;
  gs.nshorts = (int64_t)shorts.size();
  gs.items = sp.d_gitems;
  gs.items8 = sp.d_gitems8;
  gs.nitems = (int64_t)items.size();
  gs.longs = sp.d_glong;
  gs.nlongs = (int64_t)longs.size();
}

// Tables of the int64 level solve by runs for one niv map (dense rows, see
// px::SegTables): the change events of every row against the row below it in
// its chain, then per level the chunks of at most kSegRows consecutive rows of
// one chain with at most kSegEvents events in the rows after the first, each
// {first row, (level << 6) | rows, first event, end event}.
// Also, per chunk, the chunks it reads from (deps[dep_ptr[c] .. dep_ptr[c + 1])).
// Returns false (no tables) where the events, chunks or dependencies overflow
// 32-bit offsets or the levels 25 bits, or where the events would read more than
// half as many rows as the full sums.
bool build_runs(const px::Prep& P, bool up, std::vector<int4>& ev, std::vector<int4>& chunks,
                std::vector<int64_t>& cptr, std::vector<int32_t>& dep_ptr, std::vector<int32_t>& deps) {
  const int64_t n = P.n, k = P.k;
  const std::vector<int32_t>& nv = up ? P.niv_up : P.niv;
  const std::vector<int32_t>& ptr = up ? P.lev_up_ptr : P.lev_down_ptr;
  const std::vector<int32_t>& rows = up ? P.lev_up_rows : P.lev_down_rows;
  const int nt = table_threads(n);
  const std::vector<int32_t> ch = row_changes(P, nv, nt);
  std::vector<int32_t> ev_ptr(n + 1, 0);
  int64_t nev = 0;
  for (int64_t r = 0; r < n; ++r) {
    nev += ch[r];
    if (nev >= (int64_t)INT32_MAX) return false;
    ev_ptr[r + 1] = (int32_t)nev;
  }
  ev.assign((size_t)nev, make_int4(0, 0, 0, 0));
  parallel_for(n, nt, [&](int, int64_t lo, int64_t hi) {
    for (int64_t r = lo; r < hi; ++r) {
      if (ch[r] == 0) continue;
      const int32_t c = P.chain_of_row[r];
      const int32_t* a = &nv[(size_t)r * k];
      const int32_t* b = a - k;
      int64_t o = ev_ptr[r];
      for (int64_t j = 0; j < k; ++j)
        if (j != c && a[j] != b[j]) ev[o++] = make_int4(a[j] < 0 ? (int)n : a[j], b[j] < 0 ? (int)n : b[j], (int)r, 0);
    }
  });
  // deltas read two rows per event against k - 1 for a full sum: only worth it
  // where they read at most half as much (not on a grid, where row i of chain j
  // changes all j entries below it)
  if (n > k && 2 * 2 * (int64_t)ev.size() > (k - 1) * (n - k)) return false;
  chunks.clear();
  cptr.assign(1, 0);
  if (ptr.size() > ((size_t)1 << 25)) return false;  // levels packed in 25 bits
  for (size_t l = 0; l + 1 < ptr.size(); ++l) {
    for (int64_t i = ptr[l]; i < ptr[l + 1];) {
      const int32_t r0 = rows[i], c = P.chain_of_row[r0];
      int64_t j = i + 1;
      while (j < ptr[l + 1] && j - i < px::kSegRows && rows[j] == rows[j - 1] + 1 && P.chain_of_row[rows[j]] == c &&
             ev_ptr[rows[j] + 1] - ev_ptr[r0 + 1] <= px::kSegEvents)
        ++j;
      const int32_t r1 = rows[j - 1] + 1;
      chunks.push_back(make_int4(r0, (int)(l << 6) | (r1 - r0), ev_ptr[r0 + 1], ev_ptr[r1]));
      i = j;
    }
    cptr.push_back((int64_t)chunks.size());
  }
  if (chunks.size() >= (size_t)INT32_MAX) return false;
  // the chunks that each chunk reads from: those holding its first row's
  // other-chain entries and its events' rows (all at lower levels); each thread
  // a contiguous range of chunks, joined in order
  const int64_t nch = (int64_t)chunks.size();
  std::vector<int32_t> chunk_of(n, -1);
  for (int64_t c = 0; c < nch; ++c)
    for (int32_t r = chunks[c].x; r < chunks[c].x + (chunks[c].y & 63); ++r) chunk_of[r] = (int32_t)c;
  const int ntd = (int)std::max<int64_t>(1, std::min<int64_t>(nt, nch));
  std::vector<std::vector<int32_t>> dpart(ntd);
  std::vector<int32_t> dcnt(nch, 0);
  parallel_for(nch, ntd, [&](int t, int64_t c0, int64_t c1) {
    std::vector<int32_t> seen(nch, -1);
    std::vector<int32_t>& out = dpart[t];
    for (int64_t c = c0; c < c1; ++c) {
      const size_t before = out.size();
      auto add = [&](int32_t row) {
        if (row < 0 || row >= n) return;
        const int32_t q = chunk_of[row];
        if (q >= 0 && q != c && seen[q] != c) {
          seen[q] = (int32_t)c;
          out.push_back(q);
        }
      };
      const int4 chk = chunks[c];
      const int32_t* a = &nv[(size_t)chk.x * k];
      for (int64_t j = 0; j < k; ++j)
        if (a[j] != chk.x) add(a[j]);
      for (int32_t e = chk.z; e < chk.w; ++e) {
        add(ev[e].x);
        add(ev[e].y);
      }
      dcnt[c] = (int32_t)(out.size() - before);
    }
  });
  dep_ptr.assign(nch + 1, 0);
  int64_t nd = 0;
  for (int64_t c = 0; c < nch; ++c) {
    nd += dcnt[c];
    if (nd >= (int64_t)INT32_MAX) return false;
    dep_ptr[c + 1] = (int32_t)nd;
  }
  deps.clear();
  deps.reserve((size_t)nd);
  for (auto& v : dpart) deps.insert(deps.end(), v.begin(), v.end());
  return true;
}

// The int64 solve goes by runs wherever its tables exist and B >= 5, in one
// persistent launch.  POSETX_USOLVE (read on every call): "levels" runs the
// solve by runs one launch per level, "direct" the row-by-row solve.
int usolve_mode() {
  const char* v = std::getenv("POSETX_USOLVE");
  if (v && std::strcmp(v, "direct") == 0) return 0;
  if (v && std::strcmp(v, "levels") == 0) return 1;
  return 2;
}

// Polls per wait of the persistent solve (about a second); POSETX_FLOW_SPIN
// overrides it (a tiny value exercises the fallback).
int flow_spin_limit() {
  const char* v = std::getenv("POSETX_FLOW_SPIN");
  return v ? std::max(0, std::atoi(v)) : 1 << 20;
}

// Ints of the persistent solves' scratch for B columns (0 where neither is
// used): the error word and a ready flag per row and column block.
int64_t flow_ints(const px_poset* p, int64_t B) {
  const int64_t poll = p->d_lev_ptr[0] ? px::usolve_poll_ints(p->prep.n, B) : 0;
  if (!p->d_run_chunks[0]) return poll;
  const int cw = px::flow_col_width(B);
  const int64_t ncb = (B + cw - 1) / cw;
  const int64_t nch = std::max(p->run_cptr[0].empty() ? 0 : p->run_cptr[0].back(),
                               p->run_cptr[1].empty() ? 0 : p->run_cptr[1].back());
  return std::max(poll, 1 + ncb * std::max<int64_t>(p->prep.n + 1, nch));
}

// Row-by-row level solves (floating point, and int64 without runs) run every
// level in one persistent launch polling the values they read
// (px::launch_usolve_poll) where the rows are dense, there are at least two
// levels and the average level fits the resident wavefronts at one row (and
// 64-column block) each: n = 2^20, k = 64, 568 levels of 1,846 rows, float64
// B = 64: 3.9 ms against 5.4 ms with a launch per level; the 4096 x 64 grid,
// 64 levels of 4,096 rows: 0.83 against 0.46 ms (int64, B = 16), since each
// wavefront then takes two rows a level, one after the other.
// POSETX_LEVEL_POLL (read on every call): 0 launches one kernel per level,
// 2 takes the persistent launch whatever the level widths; POSETX_POLL_GRID
// caps its workgroups.
int level_poll_mode() {
  const char* v = std::getenv("POSETX_LEVEL_POLL");
  if (v && v[0] == '0') return 0;
  if (v && v[0] == '2') return 2;
  return 1;
}

// Narrow blocks (B <= 32).  With 8 to 32 columns per block, zeta values and
// refinement residuals take the compact walk with narrow kernels
// (k_scan_reduce_cn, k_scan_apply_cn and the walks on Q).
// POSETX_COMPACT_NARROW (read on every call): 0 never takes the compact walk
// for narrow blocks; 1 takes it for every narrow block, with 1 to 4 columns in
// 64-column tiles with the columns beyond B masked (slower: a masked tile
// spends a 64-lane wavefront on each row however narrow it is).
int compact_narrow_mode() {
  const char* v = std::getenv("POSETX_COMPACT_NARROW");
  if (v && v[0] == '0') return 0;
  if (v && v[0] == '1') return 2;
  return 1;
}

bool use_compact(const px_poset* p, bool up, int64_t B) {
  if (p->nslots[up ? 1 : 0] < 0 || !compact_enabled() || !px::compact_ok(p->dp, up, B)) return false;
  const int cw = px::col_width(B);
  if (cw == 64) return true;
  const int mode = compact_narrow_mode();
  return mode == 2 || (mode == 1 && cw >= 8);
}

// Tiles of the compact walk's scan (64-row tiles whatever B is), and the tile
// count a workspace for B columns must hold (either scan).
int64_t compact_tiles(const px_poset* p) { return p->ntiles[px::seg_index(64)]; }
int64_t ws_tiles(const px_poset* p, int64_t B) {
  return std::max(p->ntiles[px::seg_index(px::col_width(B))], p->nslots[0] >= 0 ? compact_tiles(p) : (int64_t)0);
}

// Level-scheduled solve U y' = g (Alg. 4, first loop; Alg. 5 schedule): each
// level sees the levels below it complete, by one launch per level or by the
// waits of a persistent launch.
hipError_t solve_levels(const px_poset* p, bool up, px::ElemType tin, const void* g, int64_t ldg, px::ElemType ty,
                        void* Y, int64_t B, void* part, void* flow, hipStream_t s) {
  const std::vector<int32_t>& ptr = up ? p->prep.lev_up_ptr : p->prep.lev_down_ptr;
  const int32_t* rows = up ? p->d_lev_up : p->d_lev_down;
  if (p->prep.n > 0) {
    hipError_t e = px::launch_usolve_begin(p->dp, ty, Y, B, s);
    if (e != hipSuccess) return e;
  }
  const px_poset::Split& sp = p->split[up ? 1 : 0];
  if (sp.on) {  // sparse rows: short rows whole, long rows in chunks
    for (size_t l = 0; l + 1 < ptr.size(); ++l) {
      prof::Scope sc(prof::USOLVE, s);
      hipError_t e = hipSuccess;
      const int64_t ns = sp.sptr[l + 1] - sp.sptr[l];
      if (ns)
        e = px::launch_usolve_level(p->dp, up, sp.d_short + sp.sptr[l], sp.sptr[l], ns, tin, g, ldg, ty, Y, B, s);
      const int64_t nl = sp.lptr[l + 1] - sp.lptr[l];
      if (e == hipSuccess && nl)
        e = px::launch_usolve_split(p->dp, up, sp.d_items + sp.cptr[l], sp.cptr[l + 1] - sp.cptr[l],
                                    sp.d_long + sp.lptr[l], nl, tin, g, ldg, ty, Y, B, part, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int m = up ? 1 : 0;
  const int mode = usolve_mode();
  if (tin == px::E_I64 && ty == px::E_I64 && p->d_run_chunks[m] && B >= 5 && mode > 0) {
    const std::vector<int64_t>& cp = p->run_cptr[m];
    if (mode == 2 && flow) {
      prof::Scope sc(prof::USOLVE, s);
      const char* wv = std::getenv("POSETX_FLOW_WAIT");
      const char* gv = std::getenv("POSETX_FLOW_GRID");
      // measured (n = 2^20, k = 64, B = 64): 64-column items waiting on the chunks read from
      // 3.3 ms, against 4.4 ms waiting on the rows read; with narrower items the row waits win
      // (32 columns: 3.0 against 3.4 ms; n = 2^23, k = 32, B = 16: 9.1 against 12.0 ms), and
      // polling the values read instead of flags is faster still (32 columns: 2.46 ms; 16: 2.04;
      // n = 2^23: 5.7 ms): no store acknowledgement, flag store and flag poll per level
      int wait = px::flow_col_width(B) == 64 ? px::kWaitDeps : px::kWaitValues;
      if (wv && std::strcmp(wv, "values") == 0) wait = px::kWaitValues;
      if (wv && std::strcmp(wv, "rows") == 0) wait = px::kWaitRows;
      if (wv && std::strcmp(wv, "level") == 0) wait = px::kWaitLevel;
      if (wv && std::strcmp(wv, "deps") == 0) wait = px::kWaitDeps;
      // workgroups: 256 per column block plus 256, at most 1024 (polling the values in 16-column
      // items: n = 2^20, B = 64, four blocks: 512 2.09 ms, 768 1.90, 1024 1.88; n = 2^23, B = 16,
      // one block: 384 5.76, 512 5.59, 640 5.69, 768 5.81); capped by the resident count
      const int64_t ncb = (B + px::flow_col_width(B) - 1) / px::flow_col_width(B);
      const int grid = gv ? std::atoi(gv) : (int)(256 * std::min<int64_t>(ncb + 1, 4));
      return px::launch_usolve_flow(p->dp, up, p->d_run_chunks[m], cp.back(), p->d_run_levn[m], p->d_run_dep_ptr[m],
                                    p->d_run_deps[m], wait, g, ldg, Y, B, (int*)flow, flow_spin_limit(), grid, s);
    }
    for (size_t l = 0; l + 1 < cp.size(); ++l) {
      prof::Scope sc(prof::USOLVE, s);
      hipError_t e = px::launch_usolve_runs(p->dp, up, p->d_run_chunks[m] + cp[l], cp[l + 1] - cp[l], g, ldg, Y, B, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int poll = level_poll_mode();
  const int64_t nlev = (int64_t)ptr.size() - 1;
  const int cwp = 64 / px::usolve_poll_rows_per_wave(B);
  const int64_t wave_items = ((int64_t)ptr.back() + 64 / cwp - 1) / (64 / cwp) * ((B + cwp - 1) / cwp);
  if (flow && p->d_lev_ptr[m] && p->d_lev_bits[m] && nlev >= 2 && poll > 0 &&
      (poll == 2 || wave_items <= nlev * px::usolve_poll_waves(tin, ty, p->prep.n, B))) {
    prof::Scope sc(prof::USOLVE, s);
    const char* gv = std::getenv("POSETX_POLL_GRID");
    return px::launch_usolve_poll(p->dp, up, rows, p->d_lev_ptr[m], p->d_lev_bits[m], (int)nlev, ptr.back(), tin, g,
                                  ldg, ty, Y, B, (int*)flow, flow_spin_limit(), gv ? std::atoi(gv) : 0, s);
  }
  for (size_t l = 0; l + 1 < ptr.size(); ++l) {
    prof::Scope sc(prof::USOLVE, s);
    hipError_t e =
        px::launch_usolve_level(p->dp, up, rows + ptr[l], ptr[l], ptr[l + 1] - ptr[l], tin, g, ldg, ty, Y, B, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The regions one zeta call uses, and nothing else: the compact walk takes the
// tile states, the snapshots and L / Q; the scan over P takes P, the tile
// states, the single-pass flags and the snapshots (sparse rows: the chunk sums).
Layout zeta_layout(const px_poset* p, bool up, int dtype, int64_t B, bool compact) {
  const int64_t n = p->prep.n;
  const size_t es = elem_size(dtype);
  const int cw = px::col_width(B);
  const int64_t nt = compact ? compact_tiles(p) : p->ntiles[px::seg_index(cw)];
  const int m = up ? 1 : 0;
  Layout L;
  size_t o = 0;
  if (!compact) {
    L.y = o;
    o = align256(o + (size_t)(n + 1) * B * es);
  }
  L.aux = o;
  o = align256(o + (size_t)nt * B * 16 * 2);
  if (!compact) {
    L.sync = o;
    o = align256(o + (size_t)(2 + nt * ((B + cw - 1) / cw)) * 4);
  }
  L.snaps = o;
  if (p->prep.sparse) {
    L.part = o;
    o = align256(o + (size_t)max_parts(p) * B * 8);
  } else {
    o = align256(o + (size_t)p->nsnap[m] * B * es);
  }
  if (compact) {
    L.lq = o;
    o = align256(o + (size_t)(2 * p->nslots[m] + 1) * B * es);
  }
  L.total = o;
  return L;
}

// ext (nullable): a caller-provided workspace of ext_bytes bytes, used instead
// of the handle's grow-only one (then nothing is allocated).
px_status zeta_impl(px_poset* p, bool up, int dtype, const void* f, int64_t ldf, void* g, int64_t ldg, int64_t B,
                    void* stream, void* ext = nullptr, size_t ext_bytes = 0) {
  if (!p) return fail(PX_EINVAL, "null poset");
  if (p->host_only) return fail(PX_EUNSUPPORTED, "poset was built with PX_BUILD_HOST_ONLY");
  if (up && !p->has_up) return fail(PX_EUNSUPPORTED, "poset was built with PX_BUILD_NO_ADJOINT");
  px_status st = check_matrix_args(p->prep.n, dtype, f, ldf, g, ldg, B);
  if (st != PX_OK) return st;
  if (p->prep.n == 0) return PX_OK;
  DeviceGuard dg(p->device);
  if (!dg.ok) return fail(PX_EHIP, "hipSetDevice failed");
  const int cw = px::col_width(B);
  const bool compact = use_compact(p, up, B);
  const int64_t nt = compact ? compact_tiles(p) : p->ntiles[px::seg_index(cw)];
  Layout L;
  char* w;
  if (ext) {
    L = zeta_layout(p, up, dtype, B, compact);
    if (L.total > ext_bytes)
      return fail(PX_EINVAL, "this call needs " + std::to_string(L.total) + " bytes of scratch; the static scratch holds " +
                                 std::to_string(ext_bytes));
    w = (char*)ext;
  } else {
    L = layout(p->prep.n, B, dtype, false, ws_tiles(p, B), std::max(p->nsnap[0], p->nsnap[1]), max_slots(p),
               max_parts(p));
    if ((st = p->ws.ensure(L.total)) != PX_OK) return st;
    w = (char*)p->ws.p;
  }
  hipStream_t s = (hipStream_t)stream;
  const px::ElemType T = etype(dtype);
  if (compact)
    return hip_status(run_compact(p->dp, up ? -1 : 1, T, f, ldf, T, g, ldg, T, nullptr, 0, B, w + L.aux, nt,
                                  w + L.lq, w + L.snaps, s),
                      "zeta launch");
  hipError_t e = run_scan(p->dp, up ? -1 : 1, T, f, ldf, T, w + L.y, B, w + L.aux, nt, (int*)(w + L.sync), s);
  // sparse rows: the chunk sums of the split gather take the snapshots' place
  if (e == hipSuccess)
    e = run_gather(p->dp, up, T, w + L.y, B, T, g, ldg, T, nullptr, 0, p->prep.sparse ? w + L.part : w + L.snaps, s);
  return hip_status(e, "zeta launch");
}

px_status mobius_impl(px_poset* p, bool up, int dtype, const void* g, int64_t ldg, void* f, int64_t ldf, int64_t B,
                      int max_refine, double tol, void* stream, px_refine_report* rep) {
  if (!p) return fail(PX_EINVAL, "null poset");
  if (p->host_only) return fail(PX_EUNSUPPORTED, "poset was built with PX_BUILD_HOST_ONLY");
  if (up && !p->has_up) return fail(PX_EUNSUPPORTED, "poset was built with PX_BUILD_NO_ADJOINT");
  px_status st = check_matrix_args(p->prep.n, dtype, g, ldg, f, ldf, B);
  if (st != PX_OK) return st;
  if (max_refine < 0) return fail(PX_EINVAL, "max_refine must be >= 0");
  const int64_t n = p->prep.n;
  if (rep) *rep = px_refine_report{0, 0, 0.0, 0.0};
  if (n == 0) return PX_OK;
  {
    const char* gb = (const char*)g;
    const char* fb = (const char*)f;
    const size_t es = elem_size(dtype);
    const char* ge = gb + ((n - 1) * ldg + B) * es;
    const char* fe = fb + ((n - 1) * ldf + B) * es;
    if (gb < fe && fb < ge) return fail(PX_EINVAL, "g and f must not overlap");
  }
  DeviceGuard dg(p->device);
  if (!dg.ok) return fail(PX_EHIP, "hipSetDevice failed");
  const bool refine = dtype == PX_F32;
  const int cw = px::col_width(B);
  const int64_t nt = p->ntiles[px::seg_index(cw)];
  Layout L = layout(n, B, dtype, refine, ws_tiles(p, B), std::max(p->nsnap[0], p->nsnap[1]), max_slots(p),
                    max_parts(p), flow_ints(p, B));
  if ((st = p->ws.ensure(L.total)) != PX_OK) return st;
  char* w = (char*)p->ws.p;
  hipStream_t s = (hipStream_t)stream;
  const px::ElemType T = etype(dtype);
  const int dir = up ? -1 : 1;
  // Floating-point results are checked for NaN / Inf unless tol < 0: once, after
  // the last chain difference, from the statistics it fuses (one synchronisation).
  const bool fp = dtype != PX_I64;
  const bool check_end = fp && tol >= 0;
  const bool check_steps = refine && (tol > 0 || rep);  // statistics read after every step
  uint64_t* dstats = (uint64_t*)(w + L.stats);
  std::vector<uint64_t> hstats(2 * B + 1);
  const bool stats0 = check_end && (!refine || max_refine == 0);
  hipError_t e = solve_levels(p, up, T, g, ldg, T, w + L.y, B, w + L.part, w + L.flow, s);
  if (e == hipSuccess) e = run_chain_diff(p->dp, dir, T, w + L.y, B, T, f, ldf, false, stats0 ? dstats : nullptr, s);
  if (e != hipSuccess) return hip_status(e, "mobius launch");
  auto read_nonfinite = [&](bool& nonfinite) -> px_status {
    hipError_t e2 = hipMemcpyAsync(hstats.data() + 2 * B, dstats + 2 * B, 8, hipMemcpyDeviceToHost, s);
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
    if (e2 != hipSuccess) return hip_status(e2, "non-finite check");
    nonfinite = hstats[2 * B] != 0;
    return PX_OK;
  };
  if (stats0) {
    bool bad = false;
    if ((st = read_nonfinite(bad)) != PX_OK) return st;
    if (bad) {
      if (rep) rep->nonfinite = 1;
      return fail(PX_ENONFINITE, "the Möbius transform met a non-finite value");
    }
  }
  if (!refine) return PX_OK;

  double* r64 = (double*)(w + L.r64);
  // Largest over columns of stats[col] / stats[B + col] (float64 bit patterns).
  auto read_ratio = [&](double& ratio, bool& nonfinite) -> px_status {
    hipError_t e2 = hipMemcpyAsync(hstats.data(), dstats, hstats.size() * 8, hipMemcpyDeviceToHost, s);
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
    if (e2 != hipSuccess) return hip_status(e2, "refinement statistics");
    nonfinite = nonfinite || hstats[2 * B] != 0;
    ratio = 0;
    for (int64_t c = 0; c < B; ++c) {
      double num, den;
      std::memcpy(&num, &hstats[c], 8);
      std::memcpy(&den, &hstats[B + c], 8);
      ratio = std::max(ratio, den > 0 ? num / den : num);
    }
    return PX_OK;
  };
  // r = g - zeta(f), zeta applied in float64 to the float32 iterate.
  auto residual = [&]() -> hipError_t {
    if (use_compact(p, up, B))
      return run_compact(p->dp, dir, px::E_F32, f, ldf, px::E_F64, r64, B, px::E_F32, g, ldg, B, w + L.aux,
                         compact_tiles(p), w + L.lq, w + L.snaps, s);
    hipError_t e2 = run_scan(p->dp, dir, px::E_F32, f, ldf, px::E_F64, w + L.p64, B, w + L.aux, nt, (int*)(w + L.sync), s);
    if (e2 == hipSuccess)
      e2 = run_gather(p->dp, up, px::E_F64, w + L.p64, B, px::E_F64, r64, B, px::E_F32, g, ldg,
                      p->prep.sparse ? w + L.part : w + L.snaps, s);
    return e2;
  };
  int it = 0;
  double corr = 0, resid = 0;
  bool nonfinite = false, converged = false;
  while (it < max_refine) {
    const bool last_check = check_end && it + 1 == max_refine;
    e = residual();
    if (e == hipSuccess) e = solve_levels(p, up, px::E_F64, r64, B, px::E_F32, w + L.y, B, w + L.part, w + L.flow, s);
    if (e == hipSuccess)
      e = run_chain_diff(p->dp, dir, px::E_F32, w + L.y, B, px::E_F32, f, ldf, true,
                         check_steps || last_check ? dstats : nullptr, s);
    if (e != hipSuccess) return hip_status(e, "refinement launch");
    ++it;
    if (!check_steps && last_check) {
      if ((st = read_nonfinite(nonfinite)) != PX_OK) return st;
    }
    if (check_steps) {
      // stop on the size of the correction relative to the iterate (forward error)
      if ((st = read_ratio(corr, nonfinite)) != PX_OK) return st;
      if (nonfinite) break;
      if (tol > 0 && corr <= tol) {
        converged = true;
        break;
      }
    }
  }
  if (rep) {
    // normwise backward error of the returned f
    e = residual();
    if (e == hipSuccess) {
      prof::Scope sc(prof::ABSMAX, s);
      e = px::launch_absmax(n, B, r64, px::E_F32, g, ldg, dstats, s);
    }
    if (e != hipSuccess) return hip_status(e, "residual statistics");
    if ((st = read_ratio(resid, nonfinite)) != PX_OK) return st;
    rep->iterations = it;
    rep->nonfinite = nonfinite ? 1 : 0;
    rep->residual = resid;
    rep->correction = corr;
  }
  if (nonfinite) return fail(PX_ENONFINITE, "refinement met a non-finite value");
  if (tol > 0 && max_refine > 0 && !converged)
    return fail(PX_ENOTCONV, "refinement stopped with correction " + std::to_string(corr) + " > tol");
  return PX_OK;
}

// (Re)build and upload the walk tables of both niv maps with run length T and
// event cap emax.
hipError_t set_walk(px_poset* p, int T, int emax) {
  const px::Prep& P = p->prep;
  hipError_t e = hipSuccess;
  for (int dir = 0; dir < 2 && e == hipSuccess; ++dir) {
    if (dir == 1 && !p->has_up) break;
    HostWalk W;
    build_walk(P, dir ? P.niv_up : P.niv, W, T, emax);
    int32_t** db = p->d_walk[dir];
    for (int i = 0; i < 5; ++i)
      if (db[i]) {
        (void)hipFree(db[i]);
        db[i] = nullptr;
      }
    px::WalkTables& t = p->dp.walk[dir];
    const int32_t keep_cw = t.cw;
    t = px::WalkTables();
    t.cw = keep_cw;
    int64_t b = 0;
    e = upload(&db[0], W.runs.data(), W.runs.size(), b);
    if (e == hipSuccess) {  // "no element" names the zero row n of P on the device
      std::vector<int32_t> evd(W.ev);
      for (size_t x = 0; x < evd.size(); x += 4) {
        if (evd[x] < 0) evd[x] = (int32_t)P.n;
        if (evd[x + 1] < 0) evd[x + 1] = (int32_t)P.n;
      }
      // one padding record (no event), so that record loads may clamp to a run's end
      evd.insert(evd.end(), {(int32_t)P.n, (int32_t)P.n, -1, 0});
      e = upload(&db[1], evd.data(), evd.size(), b);
    }
    if (e == hipSuccess) e = upload(&db[2], W.ev_off.data(), W.ev_off.size(), b);
    if (e == hipSuccess) e = upload(&db[3], W.snap_off.data(), W.snap_off.size(), b);
    if (e == hipSuccess) e = upload(&db[4], W.snap_of_row.data(), W.snap_of_row.size(), b);
    if (e != hipSuccess) break;
    p->nevents[dir] = (int64_t)W.ev.size() / 4;
    p->walk_rows[dir][0] = W.rows_distinct;
    p->walk_rows[dir][1] = W.row_loads;
    p->nsnap[dir] = W.nsnap;
    t.nruns = (int32_t)(W.runs.size() / 2);
    t.nsnap = W.nsnap;
    t.runs = (const int2*)db[0];
    t.ev = (const int4*)db[1];
    t.ev_off = db[2];
    t.snap_off = db[3];
    t.snap_of_row = db[4];
    // compact form (single poset, k <= 64)
    void** dc = p->d_compact[dir];
    for (int i = 0; i < 5; ++i)
      if (dc[i]) {
        (void)hipFree(dc[i]);
        dc[i] = nullptr;
      }
    p->nslots[dir] = -1;
    if (P.k <= 64) {
      HostCompact H;
      build_compact(P, dir ? P.niv_up : P.niv, W, H);
      if (!compact_consistent(H, p->ntiles[px::seg_index(64)])) {
        e = hipErrorInvalidValue;
        break;
      }
      uint64_t* tm = nullptr;
      int32_t *qo = nullptr, *ts = nullptr, *in = nullptr, *eq = nullptr;
      e = upload(&tm, H.tmask.data(), H.tmask.size(), b);
      dc[0] = tm;
      if (e == hipSuccess) e = upload(&qo, H.qoff.data(), H.qoff.size(), b);
      dc[1] = qo;
      if (e == hipSuccess) e = upload(&ts, H.tile_of_slot.data(), H.tile_of_slot.size(), b);
      dc[2] = ts;
      if (e == hipSuccess) e = upload(&in, H.init.data(), H.init.size(), b);
      dc[3] = in;
      // one padding record (no event) after the last run's, as for ev
      H.evq.insert(H.evq.end(), {H.nslots, H.nslots, -1, 0});
      if (e == hipSuccess) e = upload(&eq, H.evq.data(), H.evq.size(), b);
      dc[4] = eq;
      if (e != hipSuccess) break;
      t.tmask = tm;
      t.qoff = qo;
      t.tile_of_slot = ts;
      t.init = in;
      t.evq = (const int4*)eq;
      t.nslots = H.nslots;
      t.qoff_tiles = (int64_t)H.tmask.size();
      p->nslots[dir] = H.nslots;
    }
    p->hw_runs[dir] = std::move(W.runs);
    p->hw_ev[dir] = std::move(W.ev);
    p->hw_ev_off[dir] = std::move(W.ev_off);
    p->hw_snap_off[dir] = std::move(W.snap_off);
    p->hw_snap_of_row[dir] = std::move(W.snap_of_row);
  }
  p->walk_T = T;
  p->walk_emax = emax;
  return e;
}

// Autotuning: time candidate tile shapes of the walking gather on the device
// and keep the fastest.  Results are cached per shape (n, k, niv size, B,
// dtype) in the process and, if POSETX_TUNE_CACHE names a file, across
// processes (one "key T emax cw ms" line per tuned shape).
struct TuneResult {
  int T = kWalkT, emax = kWalkEvents, cw = 0;
  double ms = 0;
};
std::mutex tune_mu;
std::map<std::string, TuneResult> tune_cache;
bool tune_loaded = false;

void tune_load() {
  if (tune_loaded) return;
  tune_loaded = true;
  const char* path = std::getenv("POSETX_TUNE_CACHE");
  if (!path) return;
  FILE* fh = std::fopen(path, "r");
  if (!fh) return;
  char key[256];
  TuneResult r;
  while (std::fscanf(fh, "%255s %d %d %d %lf", key, &r.T, &r.emax, &r.cw, &r.ms) == 5) tune_cache[key] = r;
  std::fclose(fh);
}

void tune_store(const std::string& key, const TuneResult& r) {
  tune_cache[key] = r;
  const char* path = std::getenv("POSETX_TUNE_CACHE");
  if (!path) return;
  FILE* fh = std::fopen(path, "a");
  if (!fh) return;
  std::fprintf(fh, "%s %d %d %d %.6f\n", key.c_str(), r.T, r.emax, r.cw, r.ms);
  std::fclose(fh);
}

// Milliseconds of one zeta call (median of reps), on the null stream.
template <typename Run>
double time_ms(Run run, int reps) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return -1;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return -1;
  }
  std::vector<float> t;
  if (!run()) return -1;  // warm-up
  for (int i = 0; i < reps; ++i) {
    (void)hipEventRecord(a, nullptr);
    if (!run()) return -1;
    (void)hipEventRecord(b, nullptr);
    (void)hipEventSynchronize(b);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    t.push_back(ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  std::sort(t.begin(), t.end());
  return t[t.size() / 2];
}

}  // namespace

extern "C" {

const char* px_last_error(void) { return g_err.c_str(); }

px_status px_profile(int on) {
  std::lock_guard<std::mutex> lk(prof::mu);
  prof::drain();
  for (int i = 0; i < prof::NPH; ++i) {
    prof::ms[i] = 0;
    prof::cnt[i] = 0;
  }
  prof::on = on != 0;
  return PX_OK;
}

px_status px_profile_read(double* ms, int64_t* count, int nphases) {
  if (nphases < 0 || (nphases > 0 && (!ms || !count))) return fail(PX_EINVAL, "bad profile buffers");
  std::lock_guard<std::mutex> lk(prof::mu);
  prof::drain();
  for (int i = 0; i < nphases && i < prof::NPH; ++i) {
    ms[i] = prof::ms[i];
    count[i] = prof::cnt[i];
  }
  return PX_OK;
}

const char* px_profile_phase_name(int i) { return (i >= 0 && i < prof::NPH) ? prof::kNames[i] : ""; }
const char* px_version(void) { return "posetx 0.1 (gfx950)"; }

// Device side of a preprocessed handle (tables, uploads, walks); on failure
// the handle is freed.
static px_status finish_poset(px_poset* p, int device, px_poset** out) {
  const int64_t n = p->prep.n;
  std::vector<int32_t> segoff;
  seg_tables(p->prep.chain_off, segoff, p->ntiles);
  if (!p->host_only && n > 0) {
    double t0 = now_s();
    DeviceGuard dg(device);
    if (!dg.ok) {
      free_poset_device(p);
      delete p;
      return fail(PX_EHIP, "hipSetDevice(" + std::to_string(device) + ") failed");
    }
    const px::Prep& P = p->prep;
    int64_t& b = p->device_bytes;
    hipError_t e = upload(&p->d_node_of_row, P.node_of_row.data(), P.node_of_row.size(), b);
    if (e == hipSuccess) e = upload(&p->d_chain_of_row, P.chain_of_row.data(), P.chain_of_row.size(), b);
    if (e == hipSuccess) e = upload(&p->d_chain_off, P.chain_off.data(), P.chain_off.size(), b);
    if (!P.sparse && p->d_niv) {  // computed on the device
      b += (int64_t)(P.niv.size() + P.niv_up.size()) * 4;
    } else if (!P.sparse) {
      if (e == hipSuccess) e = upload(&p->d_niv, P.niv.data(), P.niv.size(), b);
      if (e == hipSuccess && p->has_up) e = upload(&p->d_niv_up, P.niv_up.data(), P.niv_up.size(), b);
    } else {
      for (int m = 0; m < (p->has_up ? 2 : 1) && e == hipSuccess; ++m) {
        if (p->d_nivp[m] && p->d_nivr[m]) {  // computed on the device
          b += (int64_t)(P.nivp[m].size() * 8 + P.nivr[m].size() * 4);
        } else {
          e = upload(&p->d_nivp[m], P.nivp[m].data(), P.nivp[m].size(), b);
          if (e == hipSuccess) e = upload(&p->d_nivr[m], P.nivr[m].data(), P.nivr[m].size(), b);
        }
        p->dp.nivp[m] = p->d_nivp[m];
        p->dp.nivr[m] = p->d_nivr[m];
      }
    }
    if (e == hipSuccess) e = upload(&p->d_lev_down, P.lev_down_rows.data(), P.lev_down_rows.size(), b);
    if (e == hipSuccess && p->has_up) e = upload(&p->d_lev_up, P.lev_up_rows.data(), P.lev_up_rows.size(), b);
    for (int dir = 0; dir < (p->has_up ? 2 : 1) && e == hipSuccess && !P.sparse; ++dir) {
      const std::vector<int32_t>& lp = dir ? P.lev_up_ptr : P.lev_down_ptr;
      std::vector<uint64_t> bits((size_t)(n + 64) / 64 + 1, 0);
      for (int32_t q : lp) bits[(size_t)q >> 6] |= 1ull << (q & 63);
      e = upload(&p->d_lev_ptr[dir], lp.data(), lp.size(), b);
      if (e == hipSuccess) e = upload(&p->d_lev_bits[dir], bits.data(), bits.size(), b);
    }
    // level-ordered niv rows and node ids for the uniform level solve, gathered
    // on the device from the maps and level orders already there
    for (int dir = 0; dir < 2 && e == hipSuccess && P.k <= 64 && !P.sparse; ++dir) {
      if (dir == 1 && !p->has_up) break;
      const int32_t* d_lr = dir ? p->d_lev_up : p->d_lev_down;
      const int32_t* d_nv = dir ? p->d_niv_up : p->d_niv;
      const int64_t cnt = (int64_t)(dir ? P.lev_up_rows.size() : P.lev_down_rows.size());
      if (!d_lr || !d_nv) {
        e = hipErrorInvalidValue;
        break;
      }
      e = hipMalloc((void**)&p->d_lev_niv[dir], std::max<int64_t>(cnt * P.k, 1) * sizeof(int32_t));
      if (e == hipSuccess) e = hipMalloc((void**)&p->d_lev_node[dir], std::max<int64_t>(cnt, 1) * sizeof(int32_t));
      if (e == hipSuccess) {
        b += (cnt * P.k + cnt) * (int64_t)sizeof(int32_t);
        e = px::device_gather_rows(d_nv, (int)P.k, d_lr, cnt, p->d_node_of_row, p->d_lev_niv[dir],
                                   p->d_lev_node[dir]);
      }
      p->dp.lev_niv[dir] = p->d_lev_niv[dir];
      p->dp.lev_node[dir] = p->d_lev_node[dir];
    }
    // int64 level solves by runs (dense rows)
    for (int m = 0; m < (p->has_up ? 2 : 1) && e == hipSuccess && !P.sparse; ++m) {
      std::vector<int4> ev, chunks;
      std::vector<int32_t> dep_ptr, deps;
      if (!build_runs(P, m == 1, ev, chunks, p->run_cptr[m], dep_ptr, deps)) {
        p->run_cptr[m].clear();
        continue;
      }
      if (deps.empty()) deps.push_back(0);  // a valid pointer for posets without dependencies
      p->run_events[m] = (int64_t)ev.size();
      if (ev.empty()) ev.push_back(make_int4((int)n, (int)n, 0, 0));  // a valid pointer for posets without events
      std::vector<int32_t> levn(p->run_cptr[m].begin(), p->run_cptr[m].end());  // first chunk of every level
      e = upload(&p->d_run_ev[m], ev.data(), ev.size(), b);
      if (e == hipSuccess) e = upload(&p->d_run_chunks[m], chunks.data(), chunks.size(), b);
      if (e == hipSuccess) e = upload(&p->d_run_levn[m], levn.data(), levn.size(), b);
      if (e == hipSuccess) e = upload(&p->d_run_dep_ptr[m], dep_ptr.data(), dep_ptr.size(), b);
      if (e == hipSuccess) e = upload(&p->d_run_deps[m], deps.data(), deps.size(), b);
      p->dp.seg[m].ev = p->d_run_ev[m];
    }
    if (e == hipSuccess) e = upload(&p->d_segoff, segoff.data(), segoff.size(), b);
    if (e == hipSuccess) {
      int64_t off[8];
      std::vector<int32_t> tt = tile_tables(P.chain_off, off, p->dp.max_chain_tiles);
      p->dp.max_chain = (int32_t)P.max_chain;
      p->dp.flat_mask = flat_mask(P.n, p->dp.max_chain, p->ntiles, p->dp.max_chain_tiles);
      for (int i = 0; i < 7; ++i)
        if (off[i + 1] - off[i] != p->ntiles[i]) e = hipErrorInvalidValue;
      if (e == hipSuccess) e = upload(&p->d_tiles, tt.data(), tt.size(), b);
      for (int i = 0; i < 7 && e == hipSuccess; ++i)
        p->dp.tiles[i] = p->d_tiles ? (const int2*)p->d_tiles + off[i] : nullptr;
    }
    if (e == hipSuccess) {
      std::vector<int32_t> ord = scan_orders(segoff, P.k, p->ntiles);
      e = upload(&p->d_order, ord.data(), ord.size(), b);
      int64_t o = 0;
      for (int dir = 0; dir < 2; ++dir)
        for (int i = 0; i < 7; ++i) {
          p->dp.scan_order[dir][i] = p->d_order ? p->d_order + o : nullptr;
          o += p->ntiles[i];
        }
    }
    // the walking gathers read dense niv rows; sparse rows take the plain gather,
    // and their level solves split long rows (entry offsets held in 32 bits)
    if (e == hipSuccess && !P.sparse) e = set_walk(p, kWalkT, kWalkEvents);
    if (e == hipSuccess && P.sparse && P.nnz_niv < INT32_MAX && P.nnz_niv_up < INT32_MAX)
      for (int m = 0; m < (p->has_up ? 2 : 1); ++m) build_split(P, m, p->split[m], p->dp.gsplit[m]);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      free_poset_device(p);
      delete p;
      return fail(e == hipErrorOutOfMemory ? PX_ENOMEM : PX_EHIP,
                  std::string("device upload failed: ") + hipGetErrorString(e));
    }
    p->t_upload = now_s() - t0;
  }
  px::DevPoset& d = p->dp;
  d.n = (int32_t)n;
  d.k = (int32_t)p->prep.k;
  d.nchains = (int32_t)p->prep.k;
  d.node_of_row = p->d_node_of_row;
  d.chain_of_row = p->d_chain_of_row;
  d.chain_off = p->d_chain_off;
  d.niv = p->d_niv;
  d.niv_up = p->d_niv_up;
  d.segoff = p->d_segoff;
  *out = p;
  return PX_OK;
}

px_status px_poset_build(int64_t n, const int64_t* indptr, const int32_t* indices, const int32_t* chain_of,
                         const int32_t* chain_pos, uint32_t flags, int device, px_poset** out) {
  if (!out) return fail(PX_EINVAL, "null output handle");
  *out = nullptr;
  px_poset* p = new (std::nothrow) px_poset();
  if (!p) return fail(PX_ENOMEM, "host allocation failed");
  p->host_only = flags & PX_BUILD_HOST_ONLY;
  p->has_up = !(flags & PX_BUILD_NO_ADJOINT);
  p->mirsky = flags & PX_BUILD_LEVELS_MIRSKY;
  p->device = device;
  std::string msg;
  int rc;
  // dense niv maps of at least 2^24 entries are computed on the device (smaller
  // ones are quicker on the host); POSETX_PREP=host / device forces either side
  const char* prep_env = std::getenv("POSETX_PREP");
  const bool force_host = prep_env && std::strcmp(prep_env, "host") == 0;
  const bool force_dev = prep_env && std::strcmp(prep_env, "device") == 0;
  const bool dev_niv = !p->host_only && n > 0 && !force_host;
  const int64_t min_dev_entries = force_dev ? 0 : (int64_t)1 << 24;
  px::NivHook hook = [&](px::Prep& P, const std::vector<int64_t>& rptr, const std::vector<int32_t>& ridx,
                         const px::Heights* heights, std::string& m) -> int {
    if (heights) {  // sparse rows: on the device from 2^16 elements (or when forced)
      if (P.n < (force_dev ? 0 : (int64_t)1 << 16)) return -1;
      DeviceGuard dg(device);
      if (!dg.ok) return -1;
      return px::device_niv_sparse(P, indptr, indices, rptr, ridx, *heights, p->has_up, p->d_nivp, p->d_nivr, m);
    }
    if (P.n * P.k < min_dev_entries) return -1;
    DeviceGuard dg(device);
    if (!dg.ok) return -1;
    int rounds = 0;
    const int r = px::device_niv(P, indptr, indices, rptr, ridx, p->has_up, &p->d_niv, &p->d_niv_up, &rounds, m);
    if (r == PX_OK) P.niv_rounds = rounds;
    return r;
  };
  // levels on the device wherever the map already is (device niv rows)
  px::LevelHook lhook = [&](const px::Prep& P, bool up, const std::vector<int64_t>& hptr,
                            const std::vector<int32_t>& hnodes, std::vector<int32_t>& lev) -> int {
    const int m = up ? 1 : 0;
    const int32_t* nv = P.sparse ? nullptr : (up ? p->d_niv_up : p->d_niv);
    if (!nv && !(P.sparse && p->d_nivp[m] && p->d_nivr[m])) return -1;
    DeviceGuard dg(device);
    if (!dg.ok) return -1;
    return px::device_udep_levels(P, hptr, hnodes, nv, p->d_nivp[m], p->d_nivr[m], lev);
  };
  try {
    rc = px::preprocess(n, indptr, indices, chain_of, chain_pos, p->has_up, p->mirsky,
                        (flags & PX_BUILD_SPARSE_NIV) != 0, p->prep, msg, dev_niv ? &hook : nullptr,
                        (flags & PX_BUILD_MIN_CHAINS) != 0, dev_niv ? &lhook : nullptr);
  } catch (const std::bad_alloc&) {
    rc = PX_ENOMEM;
    msg = "host allocation failed during preprocessing";
  }
  if (rc != PX_OK) {
    if (!p->host_only) free_poset_device(p);
    delete p;
    return fail((px_status)rc, msg);
  }
  return finish_poset(p, device, out);
}

// ------------------------------------------------ saved preprocessing
// File: "PXPOSET1", a byte-order word, flag bits, the scalars, then every
// array as (count, raw little-endian elements), then "PXEND\0\0\0".  Loading
// checks every index array against n and k before anything reaches a kernel.
extern "C++" {
namespace {
constexpr char kMagic[8] = {'P', 'X', 'P', 'O', 'S', 'E', 'T', '1'};
constexpr char kEnd[8] = {'P', 'X', 'E', 'N', 'D', 0, 0, 0};

struct Writer {
  FILE* f;
  bool ok = true;
  void raw(const void* p, size_t n) { ok = ok && (n == 0 || fwrite(p, 1, n, f) == n); }
  template <typename T> void val(T v) { raw(&v, sizeof(T)); }
  template <typename T> void vec(const std::vector<T>& v) {
    val<uint64_t>(v.size());
    raw(v.data(), v.size() * sizeof(T));
  }
};
struct Reader {
  FILE* f;
  bool ok = true;
  void raw(void* p, size_t n) { ok = ok && (n == 0 || fread(p, 1, n, f) == n); }
  template <typename T> T val() {
    T v{};
    raw(&v, sizeof(T));
    return v;
  }
  template <typename T> void vec(std::vector<T>& v, uint64_t max_count) {
    const uint64_t c = val<uint64_t>();
    if (!ok || c > max_count) {
      ok = false;
      return;
    }
    v.resize(c);
    raw(v.data(), c * sizeof(T));
  }
};

bool in_range(const std::vector<int32_t>& v, int64_t lo, int64_t hi) {
  for (int32_t x : v)
    if (x < lo || x >= hi) return false;
  return true;
}
bool offsets_ok(const std::vector<int32_t>& ptr, int64_t total) {
  if (ptr.empty() || ptr[0] != 0 || ptr.back() != total) return false;
  for (size_t i = 1; i < ptr.size(); ++i)
    if (ptr[i] < ptr[i - 1]) return false;
  return true;
}

// Every index the kernels derive from the preprocessing stays inside its array.
bool prep_consistent(const px::Prep& P, bool has_up, std::string& why) {
  const int64_t n = P.n, k = P.k;
  auto bad = [&](const char* w) {
    why = w;
    return false;
  };
  if (n < 0 || n >= INT32_MAX || k < 0 || k > n || (n > 0 && k == 0)) return bad("n or k out of range");
  if ((int64_t)P.chain_off.size() != k + 1 || !offsets_ok(P.chain_off, n)) return bad("chain offsets");
  if ((int64_t)P.chain_of.size() != n || (int64_t)P.chain_pos.size() != n || (int64_t)P.row_of_node.size() != n ||
      (int64_t)P.node_of_row.size() != n || (int64_t)P.chain_of_row.size() != n)
    return bad("per-node array sizes");
  for (int64_t x = 0; x < n; ++x) {
    const int32_t c = P.chain_of[x], r = P.row_of_node[x];
    if (c < 0 || c >= k || r < 0 || r >= n || P.node_of_row[r] != x || P.chain_of_row[r] != c ||
        r != P.chain_off[c] + P.chain_pos[x])
      return bad("chain numbering");
  }
  const int nm = has_up ? 2 : 1;
  if (!P.sparse) {
    if ((int64_t)P.niv.size() != n * k || (int64_t)P.niv_up.size() != (has_up ? n * k : 0)) return bad("niv sizes");
    if (!in_range(P.niv, -1, n) || !in_range(P.niv_up, -1, n)) return bad("niv entries");
  } else {
    if (!P.niv.empty() || !P.niv_up.empty()) return bad("niv sizes");
    for (int m = 0; m < nm; ++m) {
      const std::vector<int64_t>& ep = P.nivp[m];
      if ((int64_t)ep.size() != n + 1 || ep[0] != 0 || ep[n] != (int64_t)P.nivr[m].size()) return bad("sparse niv offsets");
      for (int64_t r = 0; r < n; ++r)
        if (ep[r + 1] < ep[r]) return bad("sparse niv offsets");
      if (!in_range(P.nivr[m], 0, n)) return bad("sparse niv entries");
    }
  }
  if ((int64_t)P.lev_down.size() != n || (int64_t)P.lev_down_rows.size() != n ||
      !offsets_ok(P.lev_down_ptr, n) || !in_range(P.lev_down_rows, 0, n))
    return bad("level schedule");
  if (has_up && ((int64_t)P.lev_up.size() != n || (int64_t)P.lev_up_rows.size() != n ||
                 !offsets_ok(P.lev_up_ptr, n) || !in_range(P.lev_up_rows, 0, n)))
    return bad("adjoint level schedule");
  return true;
}
}  // namespace
}  // extern "C++"

px_status px_poset_save(const px_poset* p, const char* path) {
  if (!p || !path) return fail(PX_EINVAL, "null argument");
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(PX_EINVAL, std::string("cannot open ") + path + " for writing");
  const px::Prep& P = p->prep;
  Writer w{f};
  w.raw(kMagic, 8);
  w.val<uint32_t>(0x01020304u);
  w.val<uint32_t>((p->has_up ? 1u : 0u) | (p->mirsky ? 2u : 0u) | (P.planted ? 4u : 0u) | (P.sparse ? 8u : 0u));
  for (int64_t v : {P.n, P.k, P.edges, P.nnz_niv, P.nnz_niv_up, P.max_chain, P.mirsky, P.udep}) w.val<int64_t>(v);
  w.val<int32_t>(P.niv_rounds);
  for (double v : {P.t_validate, P.t_chains, P.t_niv, P.t_levels}) w.val<double>(v);
  for (const std::vector<int32_t>* v : {&P.chain_of, &P.chain_pos, &P.chain_off, &P.row_of_node, &P.node_of_row,
                                        &P.chain_of_row, &P.niv, &P.niv_up, &P.nivr[0], &P.nivr[1], &P.lev_down,
                                        &P.lev_up, &P.lev_down_ptr, &P.lev_down_rows, &P.lev_up_ptr, &P.lev_up_rows})
    w.vec(*v);
  w.vec(P.nivp[0]);
  w.vec(P.nivp[1]);
  w.raw(kEnd, 8);
  const bool ok = w.ok && std::fclose(f) == 0;
  if (!ok) return fail(PX_EINVAL, std::string("writing ") + path + " failed");
  return PX_OK;
}

px_status px_poset_load(const char* path, uint32_t flags, int device, px_poset** out) {
  if (!path || !out) return fail(PX_EINVAL, "null argument");
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(PX_EINVAL, std::string("cannot open ") + path);
  px_poset* p = new (std::nothrow) px_poset();
  if (!p) {
    std::fclose(f);
    return fail(PX_ENOMEM, "host allocation failed");
  }
  px::Prep& P = p->prep;
  Reader rd{f};
  char magic[8], end[8];
  std::string why = "truncated or malformed file";
  try {
    rd.raw(magic, 8);
    const uint32_t order = rd.val<uint32_t>();
    const uint32_t bits = rd.val<uint32_t>();
    if (!rd.ok || std::memcmp(magic, kMagic, 8) != 0 || order != 0x01020304u) {
      rd.ok = false;
      why = "not a saved poset of this library and byte order";
    }
    p->has_up = bits & 1u;
    p->mirsky = bits & 2u;
    P.planted = bits & 4u;
    P.sparse = bits & 8u;
    int64_t* sc[] = {&P.n, &P.k, &P.edges, &P.nnz_niv, &P.nnz_niv_up, &P.max_chain, &P.mirsky, &P.udep};
    for (int64_t* v : sc) *v = rd.val<int64_t>();
    P.niv_rounds = rd.val<int32_t>();
    for (double* v : {&P.t_validate, &P.t_chains, &P.t_niv, &P.t_levels}) *v = rd.val<double>();
    const bool dims = rd.ok && P.n >= 0 && P.n < INT32_MAX && P.k >= 0 && P.k <= P.n;
    const uint64_t nk = dims ? (uint64_t)P.n * (uint64_t)P.k : 0, n1 = dims ? (uint64_t)P.n + 1 : 0;
    const uint64_t big = dims ? std::max<uint64_t>({nk, n1, (uint64_t)std::max<int64_t>(0, P.nnz_niv),
                                                   (uint64_t)std::max<int64_t>(0, P.nnz_niv_up)}) : 0;
    if (!dims) rd.ok = false;
    for (std::vector<int32_t>* v : {&P.chain_of, &P.chain_pos, &P.chain_off, &P.row_of_node, &P.node_of_row,
                                    &P.chain_of_row, &P.niv, &P.niv_up, &P.nivr[0], &P.nivr[1], &P.lev_down,
                                    &P.lev_up, &P.lev_down_ptr, &P.lev_down_rows, &P.lev_up_ptr, &P.lev_up_rows})
      rd.vec(*v, big);
    rd.vec(P.nivp[0], n1);
    rd.vec(P.nivp[1], n1);
    rd.raw(end, 8);
    if (rd.ok && std::memcmp(end, kEnd, 8) != 0) rd.ok = false;
  } catch (const std::bad_alloc&) {
    std::fclose(f);
    delete p;
    return fail(PX_ENOMEM, "host allocation failed while loading");
  }
  std::fclose(f);
  if (!rd.ok || !prep_consistent(P, p->has_up, why)) {
    delete p;
    return fail(PX_EINVAL, std::string(path) + ": " + why);
  }
  // the counts that size device work come from the arrays, not from the file's scalars
  P.max_chain = 0;
  for (int64_t c = 0; c < P.k; ++c) P.max_chain = std::max<int64_t>(P.max_chain, P.chain_off[c + 1] - P.chain_off[c]);
  if (P.sparse) {
    P.nnz_niv = (int64_t)P.nivr[0].size();
    P.nnz_niv_up = p->has_up ? (int64_t)P.nivr[1].size() : 0;
  } else {
    P.nnz_niv = P.nnz_niv_up = 0;
    for (int32_t v : P.niv) P.nnz_niv += v >= 0;
    for (int32_t v : P.niv_up) P.nnz_niv_up += v >= 0;
  }
  if (!p->has_up) P.lev_up_ptr.assign(1, 0);
  p->host_only = flags & PX_BUILD_HOST_ONLY;
  p->device = device;
  return finish_poset(p, device, out);
}

px_status px_poset_free(px_poset* p) {
  if (!p) return PX_OK;
  if (!p->host_only) {
    DeviceGuard dg(p->device);
    free_poset_device(p);
  }
  delete p;
  return PX_OK;
}

px_status px_poset_info(const px_poset* p, px_info* o) {
  if (!p || !o) return fail(PX_EINVAL, "null argument");
  const px::Prep& P = p->prep;
  o->n = P.n;
  o->k = P.k;
  o->edges = P.edges;
  o->nnz_niv = P.nnz_niv;
  o->nnz_niv_up = P.nnz_niv_up;
  o->max_chain = P.max_chain;
  o->levels_down = (int64_t)P.lev_down_ptr.size() - 1;
  o->levels_up = (int64_t)P.lev_up_ptr.size() - 1;
  o->mirsky_levels = P.mirsky;
  o->udep_levels = P.udep;
  o->device_bytes = p->device_bytes;
  o->walk_runs = p->dp.walk[0].nruns;
  o->walk_events = p->nevents[0];
  o->walk_snapshots = p->nsnap[0];
  o->walk_T = p->walk_T;
  o->walk_emax = p->walk_emax;
  o->walk_rows_distinct = p->walk_rows[0][0];
  o->walk_row_loads = p->walk_rows[0][1];
  o->chains_planted = P.planted ? 1 : 0;
  o->device = p->device;
  o->t_validate = P.t_validate;
  o->t_chains = P.t_chains;
  o->t_niv = P.t_niv;
  o->t_levels = P.t_levels;
  o->t_upload = p->t_upload;
  o->niv_sparse = P.sparse ? 1 : 0;
  o->niv_device_rounds = P.niv_rounds;
  o->run_chunks = p->run_cptr[0].empty() ? 0 : p->run_cptr[0].back();
  o->run_events = p->run_events[0];
  o->path_cover = P.path_cover;
  o->layout = p->layout;
  o->scan_flat = p->dp.flat_mask;
  return PX_OK;
}

px_status px_poset_chains(const px_poset* p, int32_t* chain_of, int32_t* chain_pos) {
  if (!p || (p->prep.n > 0 && (!chain_of || !chain_pos))) return fail(PX_EINVAL, "null argument");
  std::copy(p->prep.chain_of.begin(), p->prep.chain_of.end(), chain_of);
  std::copy(p->prep.chain_pos.begin(), p->prep.chain_pos.end(), chain_pos);
  return PX_OK;
}

px_status px_poset_set_layout(px_poset* p, uint32_t layout) {
  if (!p) return fail(PX_EINVAL, "null poset");
  if (layout != PX_LAYOUT_NODES && layout != PX_LAYOUT_ROWS) return fail(PX_EINVAL, "unknown layout");
  if (p->host_only) return fail(PX_EUNSUPPORTED, "poset was built with PX_BUILD_HOST_ONLY");
  const int64_t n = p->prep.n;
  if (layout == PX_LAYOUT_ROWS && n > 0) {
    if (!p->d_iota) {
      DeviceGuard dg(p->device);
      if (!dg.ok) return fail(PX_EHIP, "hipSetDevice failed");
      std::vector<int32_t> iota(n);
      for (int64_t r = 0; r < n; ++r) iota[r] = (int32_t)r;
      const hipError_t e = upload(&p->d_iota, iota.data(), iota.size(), p->device_bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        p->d_iota = nullptr;
        return fail(e == hipErrorOutOfMemory ? PX_ENOMEM : PX_EHIP, "row layout table");
      }
    }
    p->dp.node_of_row = p->d_iota;
    p->dp.ident = 1;
    // the uniform level solve's level-ordered ids: the rows themselves
    p->dp.lev_node[0] = p->d_lev_node[0] ? p->d_lev_down : nullptr;
    p->dp.lev_node[1] = p->d_lev_node[1] ? p->d_lev_up : nullptr;
  } else {
    p->dp.node_of_row = p->d_node_of_row;
    p->dp.ident = 0;
    p->dp.lev_node[0] = p->d_lev_node[0];
    p->dp.lev_node[1] = p->d_lev_node[1];
  }
  p->layout = layout;
  return PX_OK;
}

px_status px_poset_rows(const px_poset* p, int64_t* row_of_node) {
  if (!p || (p->prep.n > 0 && !row_of_node)) return fail(PX_EINVAL, "null argument");
  std::copy(p->prep.row_of_node.begin(), p->prep.row_of_node.end(), row_of_node);
  return PX_OK;
}

px_status px_poset_niv(const px_poset* p, int up, int32_t* out) {
  if (!p || (p->prep.n > 0 && !out)) return fail(PX_EINVAL, "null argument");
  if (up && !p->has_up) return fail(PX_EUNSUPPORTED, "poset was built with PX_BUILD_NO_ADJOINT");
  const px::Prep& P = p->prep;
  if (P.sparse) {
    std::fill(out, out + P.n * P.k, -1);
    const std::vector<int64_t>& ep = P.nivp[up ? 1 : 0];
    const std::vector<int32_t>& er = P.nivr[up ? 1 : 0];
    for (int64_t x = 0; x < P.n; ++x) {
      const int32_t r = P.row_of_node[x];
      for (int64_t e = ep[r]; e < ep[r + 1]; ++e) out[x * P.k + P.chain_of_row[er[e]]] = P.node_of_row[er[e]];
    }
    return PX_OK;
  }
  const std::vector<int32_t>& nv = up ? P.niv_up : P.niv;
  for (int64_t x = 0; x < P.n; ++x) {
    const int32_t* R = &nv[(size_t)P.row_of_node[x] * P.k];
    for (int64_t j = 0; j < P.k; ++j) out[x * P.k + j] = R[j] >= 0 ? P.node_of_row[R[j]] : -1;
  }
  return PX_OK;
}

px_status px_poset_niv_csr(const px_poset* p, int up, int64_t* ptr, int32_t* nodes) {
  if (!p || !ptr || (p->prep.n > 0 && !nodes && (up ? p->prep.nnz_niv_up : p->prep.nnz_niv) > 0))
    return fail(PX_EINVAL, "null argument");
  if (up && !p->has_up) return fail(PX_EUNSUPPORTED, "poset was built with PX_BUILD_NO_ADJOINT");
  const px::Prep& P = p->prep;
  const int m = up ? 1 : 0;
  int64_t o = 0;
  ptr[0] = 0;
  for (int64_t x = 0; x < P.n; ++x) {
    const int32_t r = P.row_of_node[x];
    if (P.sparse) {
      for (int64_t e = P.nivp[m][r]; e < P.nivp[m][r + 1]; ++e) nodes[o++] = P.node_of_row[P.nivr[m][e]];
    } else {
      const int32_t* R = &(up ? P.niv_up : P.niv)[(size_t)r * P.k];
      for (int64_t j = 0; j < P.k; ++j)
        if (R[j] >= 0) nodes[o++] = P.node_of_row[R[j]];
    }
    ptr[x + 1] = o;
  }
  return PX_OK;
}

px_status px_poset_levels(const px_poset* p, int up, int32_t* level) {
  if (!p || (p->prep.n > 0 && !level)) return fail(PX_EINVAL, "null argument");
  if (up && !p->has_up) return fail(PX_EUNSUPPORTED, "poset was built with PX_BUILD_NO_ADJOINT");
  const px::Prep& P = p->prep;
  const std::vector<int32_t>& lev = up ? P.lev_up : P.lev_down;
  for (int64_t x = 0; x < P.n; ++x) level[x] = lev[P.row_of_node[x]];
  return PX_OK;
}

px_status px_reserve(px_poset* p, int dtype, int64_t B) {
  if (!p) return fail(PX_EINVAL, "null poset");
  if (p->host_only) return fail(PX_EUNSUPPORTED, "poset was built with PX_BUILD_HOST_ONLY");
  if (dtype != PX_I64 && dtype != PX_F32 && dtype != PX_F64) return fail(PX_EINVAL, "unknown dtype");
  if (B < 1) return fail(PX_EINVAL, "B must be >= 1");
  DeviceGuard dg(p->device);
  return p->ws.ensure(
      layout(p->prep.n, B, dtype, dtype == PX_F32, ws_tiles(p, B), std::max(p->nsnap[0], p->nsnap[1]), max_slots(p),
             max_parts(p), flow_ints(p, B)).total);
}

px_status px_zeta(px_poset* p, int dtype, const void* f, int64_t ldf, void* g, int64_t ldg, int64_t B, void* stream) {
  return zeta_impl(p, false, dtype, f, ldf, g, ldg, B, stream);
}

px_status px_zeta_adjoint(px_poset* p, int dtype, const void* w, int64_t ldw, void* out, int64_t ldo, int64_t B,
                          void* stream) {
  return zeta_impl(p, true, dtype, w, ldw, out, ldo, B, stream);
}

px_status px_zeta_noalloc(px_poset* p, int dtype, const void* f, int64_t ldf, void* g, int64_t ldg, int64_t B,
                          void* stream) {
  if (!p) return fail(PX_EINVAL, "null poset");
  if (p->host_only) return fail(PX_EUNSUPPORTED, "poset was built with PX_BUILD_HOST_ONLY");
  DeviceGuard dg(p->device);
  if (!dg.ok) return fail(PX_EHIP, "hipSetDevice failed");
  void* scratch = nullptr;
  const hipError_t e = px::static_scratch(p->device, &scratch);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(PX_EHIP, std::string("address of the static scratch: ") + hipGetErrorString(e));
  }
  return zeta_impl(p, false, dtype, f, ldf, g, ldg, B, stream, scratch, px::kStaticScratchBytes);
}

px_status px_mobius(px_poset* p, int dtype, const void* g, int64_t ldg, void* f, int64_t ldf, int64_t B,
                    int max_refine, double tol, void* stream, px_refine_report* rep) {
  return mobius_impl(p, false, dtype, g, ldg, f, ldf, B, max_refine, tol, stream, rep);
}

px_status px_mobius_adjoint(px_poset* p, int dtype, const void* v, int64_t ldv, void* out, int64_t ldo, int64_t B,
                            int max_refine, double tol, void* stream, px_refine_report* rep) {
  return mobius_impl(p, true, dtype, v, ldv, out, ldo, B, max_refine, tol, stream, rep);
}

px_status px_autotune(px_poset* p, int dtype, int64_t B, px_tune_report* rep) {
  if (!p) return fail(PX_EINVAL, "null poset");
  if (p->host_only) return fail(PX_EUNSUPPORTED, "poset was built with PX_BUILD_HOST_ONLY");
  if (dtype != PX_I64 && dtype != PX_F32 && dtype != PX_F64) return fail(PX_EINVAL, "unknown dtype");
  if (B < 1) return fail(PX_EINVAL, "B must be >= 1");
  const int64_t n = p->prep.n;
  if (rep) *rep = px_tune_report{p->walk_T, p->walk_emax, p->dp.walk[0].cw, 0.0, 0.0, 0};
  if (n == 0 || p->prep.sparse) return PX_OK;  // sparse rows: nothing to tune
  DeviceGuard dg(p->device);
  if (!dg.ok) return fail(PX_EHIP, "hipSetDevice failed");
  std::lock_guard<std::mutex> lk(tune_mu);
  tune_load();
  const std::string key = "poset:" + std::to_string(n) + ":" + std::to_string(p->prep.k) + ":" +
                          std::to_string(p->prep.nnz_niv) + ":" + std::to_string(B) + ":" + std::to_string(dtype);
  auto apply = [&](const TuneResult& r) -> px_status {
    if (r.T != p->walk_T || r.emax != p->walk_emax) {
      hipError_t e = set_walk(p, r.T, r.emax);
      if (e != hipSuccess) return hip_status(e, "walk table upload");
    }
    p->dp.walk[0].cw = p->dp.walk[1].cw = r.cw;
    return PX_OK;
  };
  auto it = tune_cache.find(key);
  if (it != tune_cache.end()) {
    px_status st = apply(it->second);
    if (rep) *rep = px_tune_report{it->second.T, it->second.emax, it->second.cw, it->second.ms, 0.0, 1};
    return st;
  }
  const size_t bytes = (size_t)n * B * elem_size(dtype);
  void *f = nullptr, *g = nullptr;
  if (hipMalloc(&f, bytes) != hipSuccess || hipMalloc(&g, bytes) != hipSuccess) {
    (void)hipGetLastError();
    if (f) (void)hipFree(f);
    return fail(PX_ENOMEM, "autotune buffers");
  }
  (void)hipMemset(f, 0, bytes);
  auto run = [&]() { return zeta_impl(p, false, dtype, f, B, g, B, B, nullptr) == PX_OK; };
  const int T0 = p->walk_T, E0 = p->walk_emax;
  TuneResult best;
  best.ms = 1e30;
  double ms_default = -1;
  const int dcw = px::col_width(B);
  std::vector<int> cws{0};
  if (B < 32)
    for (int c = 2 * dcw; c <= 64 && c <= 4 * dcw; c *= 2) cws.push_back(c);
  px_status st = PX_OK;
  for (int T : {64, 128, 256}) {
    for (int E : {48, 96, 192}) {
      hipError_t e = set_walk(p, T, E);
      if (e != hipSuccess) {
        st = hip_status(e, "walk table upload");
        break;
      }
      for (int c : cws) {
        p->dp.walk[0].cw = p->dp.walk[1].cw = c;
        const double ms = time_ms(run, 5);
        if (ms < 0) {
          st = fail(PX_EHIP, "autotune run failed");
          break;
        }
        if (T == T0 && E == E0 && c == 0) ms_default = ms;
        if (ms < best.ms) best = TuneResult{T, E, c, ms};
      }
      if (st != PX_OK) break;
    }
    if (st != PX_OK) break;
  }
  (void)hipFree(f);
  (void)hipFree(g);
  if (st != PX_OK) return st;
  if ((st = apply(best)) != PX_OK) return st;
  tune_store(key, best);
  if (rep) *rep = px_tune_report{best.T, best.emax, best.cw, best.ms, ms_default, 0};
  return PX_OK;
}

// ------------------------------------------------------------------- batches
px_status px_batch_build(int count, px_poset* const* posets, px_batch** out) {
  if (!out || count < 1 || !posets) return fail(PX_EINVAL, "bad batch arguments");
  *out = nullptr;
  const int dev = posets[0] ? posets[0]->device : 0;
  bool has_up = true;
  for (int i = 0; i < count; ++i) {
    if (!posets[i]) return fail(PX_EINVAL, "null poset in batch");
    if (posets[i]->host_only) return fail(PX_EUNSUPPORTED, "host-only poset in batch");
    if (posets[i]->prep.sparse) return fail(PX_EUNSUPPORTED, "batches take posets with dense niv rows");
    if (posets[i]->device != dev) return fail(PX_EINVAL, "posets of a batch must share a device");
    has_up = has_up && posets[i]->has_up;
  }
  px_batch* b = new (std::nothrow) px_batch();
  if (!b) return fail(PX_ENOMEM, "host allocation failed");
  b->device = dev;
  b->count = count;
  b->has_up = has_up;
  std::vector<int32_t> node_of_row, chain_of_row, chain_off(1, 0), poset_of_row, kk(count), row_off(count + 1, 0);
  std::vector<int64_t> niv_off(count + 1, 0);
  int64_t rows = 0, chains = 0;
  for (int i = 0; i < count; ++i) {
    const px::Prep& P = posets[i]->prep;
    row_off[i] = (int32_t)rows;
    niv_off[i + 1] = niv_off[i] + P.n * P.k;
    kk[i] = (int32_t)P.k;
    rows += P.n;
    chains += P.k;
  }
  if (rows >= INT32_MAX) {
    delete b;
    return fail(PX_EINVAL, "batch has too many rows");
  }
  row_off[count] = (int32_t)rows;
  b->rows = rows;
  node_of_row.resize(rows);
  chain_of_row.resize(rows);
  poset_of_row.resize(rows);
  chain_off.reserve(chains + 1);
  std::vector<int32_t> niv((size_t)niv_off[count]), niv_up(has_up ? (size_t)niv_off[count] : 0);
  int32_t cbase = 0;
  for (int i = 0; i < count; ++i) {
    const px::Prep& P = posets[i]->prep;
    const int32_t o = row_off[i];
    for (int64_t r = 0; r < P.n; ++r) {
      node_of_row[o + r] = o + P.node_of_row[r];
      chain_of_row[o + r] = cbase + P.chain_of_row[r];
      poset_of_row[o + r] = i;
    }
    for (int64_t c = 0; c < P.k; ++c) chain_off.push_back(o + P.chain_off[c + 1]);
    for (size_t e = 0; e < P.niv.size(); ++e) niv[niv_off[i] + e] = P.niv[e] >= 0 ? P.niv[e] + o : -1;
    if (has_up)
      for (size_t e = 0; e < P.niv_up.size(); ++e) niv_up[niv_off[i] + e] = P.niv_up[e] >= 0 ? P.niv_up[e] + o : -1;
    cbase += (int32_t)P.k;
  }
  std::vector<int32_t> segoff;
  seg_tables(chain_off, segoff, b->ntiles);
  DeviceGuard dg(dev);
  int64_t bytes = 0;
  hipError_t e = upload(&b->d_node_of_row, node_of_row.data(), node_of_row.size(), bytes);
  if (e == hipSuccess) e = upload(&b->d_chain_of_row, chain_of_row.data(), chain_of_row.size(), bytes);
  if (e == hipSuccess) e = upload(&b->d_chain_off, chain_off.data(), chain_off.size(), bytes);
  if (e == hipSuccess) e = upload(&b->d_niv, niv.data(), niv.size(), bytes);
  if (e == hipSuccess && has_up) e = upload(&b->d_niv_up, niv_up.data(), niv_up.size(), bytes);
  if (e == hipSuccess) e = upload(&b->d_segoff, segoff.data(), segoff.size(), bytes);
  if (e == hipSuccess) {
    int64_t off[8];
    std::vector<int32_t> tt = tile_tables(chain_off, off, b->dp.max_chain_tiles);
    for (size_t c = 0; c + 1 < chain_off.size(); ++c)
      b->dp.max_chain = std::max(b->dp.max_chain, chain_off[c + 1] - chain_off[c]);
    b->dp.flat_mask = flat_mask(rows, b->dp.max_chain, b->ntiles, b->dp.max_chain_tiles);
    for (int i = 0; i < 7; ++i)
      if (off[i + 1] - off[i] != b->ntiles[i]) e = hipErrorInvalidValue;
    if (e == hipSuccess) e = upload(&b->d_tiles, tt.data(), tt.size(), bytes);
    for (int i = 0; i < 7 && e == hipSuccess; ++i)
      b->dp.tiles[i] = b->d_tiles ? (const int2*)b->d_tiles + off[i] : nullptr;
  }
  if (e == hipSuccess) {
    std::vector<int32_t> ord = scan_orders(segoff, chains, b->ntiles);
    e = upload(&b->d_order, ord.data(), ord.size(), bytes);
    int64_t o = 0;
    for (int dir = 0; dir < 2; ++dir)
      for (int i = 0; i < 7; ++i) {
        b->dp.scan_order[dir][i] = b->d_order ? b->d_order + o : nullptr;
        o += b->ntiles[i];
      }
  }
  if (e == hipSuccess) e = upload(&b->d_poset_of_row, poset_of_row.data(), poset_of_row.size(), bytes);
  if (e == hipSuccess) e = upload(&b->d_k, kk.data(), kk.size(), bytes);
  if (e == hipSuccess) e = upload(&b->d_row_off, row_off.data(), row_off.size(), bytes);
  if (e == hipSuccess) e = upload(&b->d_niv_off, niv_off.data(), niv_off.size(), bytes);
  // walk tables of every poset, rows, events and snapshots shifted into the batch
  for (int dir = 0; dir < 2 && e == hipSuccess; ++dir) {
    if (dir == 1 && !has_up) break;
    std::vector<int32_t> runs, ev, ev_off(1, 0), snap_off(1, 0), snap_of_row(rows);
    int32_t eo = 0, so = 0;
    for (int i = 0; i < count; ++i) {
      const px_poset* q = posets[i];
      const int32_t o = row_off[i];
      for (int32_t r : q->hw_runs[dir]) runs.push_back(r + o);
      const std::vector<int32_t>& qe = q->hw_ev[dir];
      for (size_t x = 0; x < qe.size(); x += 4) {  // "no element": the batch's zero row
        ev.push_back(qe[x] >= 0 ? qe[x] + o : (int32_t)rows);
        ev.push_back(qe[x + 1] >= 0 ? qe[x + 1] + o : (int32_t)rows);
        ev.push_back(qe[x + 2]);
        ev.push_back(0);
      }
      for (size_t x = 1; x < q->hw_ev_off[dir].size(); ++x) ev_off.push_back(q->hw_ev_off[dir][x] + eo);
      for (size_t x = 1; x < q->hw_snap_off[dir].size(); ++x) snap_off.push_back(q->hw_snap_off[dir][x] + so);
      for (int64_t r = 0; r < q->prep.n; ++r) snap_of_row[o + r] = q->hw_snap_of_row[dir][r] + so;
      eo += (int32_t)(qe.size() / 4);
      so += q->nsnap[dir];
    }
    ev.insert(ev.end(), {(int32_t)rows, (int32_t)rows, -1, 0});  // padding record, as for one poset
    b->nsnap[dir] = so;
    px::WalkTables& t = b->dp.walk[dir];
    t.nruns = (int32_t)(runs.size() / 2);
    t.nsnap = so;
    int32_t** db = b->d_walk[dir];
    e = upload(&db[0], runs.data(), runs.size(), bytes);
    if (e == hipSuccess) e = upload(&db[1], ev.data(), ev.size(), bytes);
    if (e == hipSuccess) e = upload(&db[2], ev_off.data(), ev_off.size(), bytes);
    if (e == hipSuccess) e = upload(&db[3], snap_off.data(), snap_off.size(), bytes);
    if (e == hipSuccess) e = upload(&db[4], snap_of_row.data(), snap_of_row.size(), bytes);
    t.runs = (const int2*)db[0];
    t.ev = (const int4*)db[1];
    t.ev_off = db[2];
    t.snap_off = db[3];
    t.snap_of_row = db[4];
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    px_batch_free(b);
    return fail(e == hipErrorOutOfMemory ? PX_ENOMEM : PX_EHIP, std::string("batch upload failed: ") + hipGetErrorString(e));
  }
  px::DevPoset& d = b->dp;
  d.n = (int32_t)rows;
  d.k = 0;
  d.nchains = (int32_t)chains;
  d.node_of_row = b->d_node_of_row;
  d.chain_of_row = b->d_chain_of_row;
  d.chain_off = b->d_chain_off;
  d.niv = b->d_niv;
  d.niv_up = b->d_niv_up;
  d.segoff = b->d_segoff;
  d.niv_off = b->d_niv_off;
  d.poset_of_row = b->d_poset_of_row;
  d.k_of_poset = b->d_k;
  d.row_off = b->d_row_off;
  b->node_of_row = std::move(node_of_row);
  *out = b;
  return PX_OK;
}

px_status px_batch_set_layout(px_batch* b, uint32_t layout) {
  if (!b) return fail(PX_EINVAL, "null batch");
  if (layout != PX_LAYOUT_NODES && layout != PX_LAYOUT_ROWS) return fail(PX_EINVAL, "unknown layout");
  if (layout == PX_LAYOUT_ROWS && b->rows > 0) {
    if (!b->d_iota) {
      DeviceGuard dg(b->device);
      if (!dg.ok) return fail(PX_EHIP, "hipSetDevice failed");
      std::vector<int32_t> iota(b->rows);
      for (int64_t r = 0; r < b->rows; ++r) iota[r] = (int32_t)r;
      int64_t bytes = 0;
      const hipError_t e = upload(&b->d_iota, iota.data(), iota.size(), bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        b->d_iota = nullptr;
        return fail(e == hipErrorOutOfMemory ? PX_ENOMEM : PX_EHIP, "row layout table");
      }
    }
    b->dp.node_of_row = b->d_iota;
    b->dp.ident = 1;
  } else {
    b->dp.node_of_row = b->d_node_of_row;
    b->dp.ident = 0;
  }
  b->layout = layout;
  return PX_OK;
}

px_status px_batch_row_order(const px_batch* b, int64_t* row_of_node) {
  if (!b || (b->rows > 0 && !row_of_node)) return fail(PX_EINVAL, "null argument");
  for (int64_t r = 0; r < b->rows; ++r) row_of_node[b->node_of_row[r]] = r;
  return PX_OK;
}

px_status px_batch_free(px_batch* b) {
  if (!b) return PX_OK;
  DeviceGuard dg(b->device);
  int32_t* bufs[] = {b->d_node_of_row, b->d_chain_of_row, b->d_chain_off, b->d_niv,     b->d_niv_up,
                     b->d_segoff,      b->d_poset_of_row,  b->d_k,         b->d_row_off, b->d_order,
                     b->d_tiles,       b->d_iota};
  for (int32_t* q : bufs)
    if (q) (void)hipFree(q);
  if (b->d_niv_off) (void)hipFree(b->d_niv_off);
  for (auto& dir : b->d_walk)
    for (int32_t* q : dir)
      if (q) (void)hipFree(q);
  b->ws.release();
  delete b;
  return PX_OK;
}

px_status px_batch_rows(const px_batch* b, int64_t* total_rows) {
  if (!b || !total_rows) return fail(PX_EINVAL, "null argument");
  *total_rows = b->rows;
  return PX_OK;
}

px_status px_batch_reserve(px_batch* b, int dtype, int64_t B) {
  if (!b) return fail(PX_EINVAL, "null batch");
  if (dtype != PX_I64 && dtype != PX_F32 && dtype != PX_F64) return fail(PX_EINVAL, "unknown dtype");
  if (B < 1) return fail(PX_EINVAL, "B must be >= 1");
  DeviceGuard dg(b->device);
  const int64_t nt = b->ntiles[px::seg_index(px::col_width(B))];
  return b->ws.ensure(layout(b->rows, B, dtype, false, nt, std::max(b->nsnap[0], b->nsnap[1])).total);
}

static px_status batch_zeta(px_batch* b, bool up, int dtype, const void* f, int64_t ldf, void* g, int64_t ldg,
                            int64_t B, void* stream) {
  if (!b) return fail(PX_EINVAL, "null batch");
  if (up && !b->has_up) return fail(PX_EUNSUPPORTED, "a poset of the batch was built with PX_BUILD_NO_ADJOINT");
  px_status st = check_matrix_args(b->rows, dtype, f, ldf, g, ldg, B);
  if (st != PX_OK) return st;
  DeviceGuard dg(b->device);
  if (!dg.ok) return fail(PX_EHIP, "hipSetDevice failed");
  const int64_t nt = b->ntiles[px::seg_index(px::col_width(B))];
  Layout L = layout(b->rows, B, dtype, false, nt, std::max(b->nsnap[0], b->nsnap[1]));
  if ((st = b->ws.ensure(L.total)) != PX_OK) return st;
  char* w = (char*)b->ws.p;
  hipStream_t s = (hipStream_t)stream;
  const px::ElemType T = etype(dtype);
  hipError_t e = run_scan(b->dp, up ? -1 : 1, T, f, ldf, T, w + L.y, B, w + L.aux, nt, (int*)(w + L.sync), s);
  if (e == hipSuccess) e = run_gather(b->dp, up, T, w + L.y, B, T, g, ldg, T, nullptr, 0, w + L.snaps, s);
  return hip_status(e, "batched zeta launch");
}

px_status px_batch_autotune(px_batch* b, int dtype, int64_t B, px_tune_report* rep) {
  if (!b) return fail(PX_EINVAL, "null batch");
  if (dtype != PX_I64 && dtype != PX_F32 && dtype != PX_F64) return fail(PX_EINVAL, "unknown dtype");
  if (B < 1) return fail(PX_EINVAL, "B must be >= 1");
  if (rep) *rep = px_tune_report{0, 0, b->dp.walk[0].cw, 0.0, 0.0, 0};
  DeviceGuard dg(b->device);
  if (!dg.ok) return fail(PX_EHIP, "hipSetDevice failed");
  std::lock_guard<std::mutex> lk(tune_mu);
  tune_load();
  const std::string key = "batch:" + std::to_string(b->count) + ":" + std::to_string(b->rows) + ":" +
                          std::to_string(b->nsnap[0]) + ":" + std::to_string(B) + ":" + std::to_string(dtype);
  auto it = tune_cache.find(key);
  if (it != tune_cache.end()) {
    b->dp.walk[0].cw = b->dp.walk[1].cw = it->second.cw;
    if (rep) *rep = px_tune_report{0, 0, it->second.cw, it->second.ms, 0.0, 1};
    return PX_OK;
  }
  const size_t bytes = (size_t)b->rows * B * elem_size(dtype);
  void *f = nullptr, *g = nullptr;
  if (hipMalloc(&f, bytes) != hipSuccess || hipMalloc(&g, bytes) != hipSuccess) {
    (void)hipGetLastError();
    if (f) (void)hipFree(f);
    return fail(PX_ENOMEM, "autotune buffers");
  }
  (void)hipMemset(f, 0, bytes);
  auto run = [&]() { return batch_zeta(b, false, dtype, f, B, g, B, B, nullptr) == PX_OK; };
  TuneResult best;
  best.ms = 1e30;
  double ms_default = -1;
  const int dcw = px::col_width(B);
  for (int c = dcw; c <= 64; c *= 2) {
    b->dp.walk[0].cw = b->dp.walk[1].cw = (c == dcw ? 0 : c);
    const double ms = time_ms(run, 5);
    if (ms < 0) {
      (void)hipFree(f);
      (void)hipFree(g);
      return fail(PX_EHIP, "autotune run failed");
    }
    if (c == dcw) ms_default = ms;
    if (ms < best.ms) best = TuneResult{0, 0, c == dcw ? 0 : c, ms};
  }
  (void)hipFree(f);
  (void)hipFree(g);
  b->dp.walk[0].cw = b->dp.walk[1].cw = best.cw;
  tune_store(key, best);
  if (rep) *rep = px_tune_report{0, 0, best.cw, best.ms, ms_default, 0};
  return PX_OK;
}

px_status px_zeta_batched(px_batch* b, int dtype, const void* f, int64_t ldf, void* g, int64_t ldg, int64_t B,
                          void* stream) {
  return batch_zeta(b, false, dtype, f, ldf, g, ldg, B, stream);
}

px_status px_zeta_adjoint_batched(px_batch* b, int dtype, const void* w, int64_t ldw, void* out, int64_t ldo,
                                  int64_t B, void* stream) {
  return batch_zeta(b, true, dtype, w, ldw, out, ldo, B, stream);
}

}  // extern "C"
