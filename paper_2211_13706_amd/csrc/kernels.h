// Launchers of the gfx950 kernels of the transforms (internal interface).
//
// Row = position in the chain-major renumbering: chain c owns rows
// [chain_off[c], chain_off[c+1]), bottom element first.  Device matrices P / Y
// are [n, B] chain-major and dense; user matrices are in node order with a
// leading dimension and are addressed through node_of_row.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace px {

enum ElemType { E_I64 = 0, E_F32 = 1, E_F64 = 2 };

// Runs of the walking gather (see k_walk_events): run s covers rows
// [runs[s].x, runs[s].y) of one chain; its niv change events are
// ev[ev_off[s] .. ev_off[s+1]), each {new row, old row, (row offset << 8) | chain, 0}
// (-1 = none), sorted by row offset, own chain excluded (ev keeps one padding
// record {n, n, -1, 0} after the last run's); it owns snapshots
// [snap_off[s], snap_off[s+1]) (first row, then every row with events), and
// snap_of_row[r] is the snapshot that row r adds to its own P[r].
// Event rows name row n (a zero row of P that the scan keeps zero) for "no
// element"; P therefore has n + 1 rows.
//
// Compact form (single poset, k <= 64): the event kernel reads P only at the
// rows it gathers (the other-chain niv entries of each run's first row and
// the rows of the events), so the scan can record P at those rows alone, in
// Q, and never write P.  The gathered rows are numbered ("slots") in row
// order within the 64-row scan tiles of 64-column blocks:
// slot(r) = qoff[t] + popcount(tmask[t] & ((1 << b) - 1)) for row r at bit b of
// tile t.  init[s * k + j] is the slot of niv_j(first row of run s) and evq
// are the events with slots; both name slot nslots (a zero row of Q) for the
// own chain and "no element".
struct WalkTables {
  const int2* runs = nullptr;
  const int4* ev = nullptr;
  const int32_t* ev_off = nullptr;
  const int32_t* snap_off = nullptr;
  const int32_t* snap_of_row = nullptr;
  int32_t nruns = 0, nsnap = 0;
  int32_t cw = 0;  // column tile of the lane-split form (0: the smallest power of two >= B)
  // compact form (absent: tmask == nullptr)
  const uint64_t* tmask = nullptr;       // [tiles of height 64]
  const int32_t* qoff = nullptr;         // [tiles of height 64 + 1]
  const int32_t* tile_of_slot = nullptr; // [nslots]
  const int32_t* init = nullptr;         // [nruns * k]
  const int4* evq = nullptr;             // as ev, rows replaced by slots
  int32_t nslots = 0;
  int64_t qoff_tiles = 0;                // tiles of height 64 that tmask / qoff cover
};

// The sparse gather's rows split by length: the short rows (taken whole) and
// the long ones in chunks, as for the level solve (see launch_usolve_split).
struct GatherSplit {
  const int32_t* shorts = nullptr;  // nullptr: no split, every row whole
  int64_t nshorts = 0;
  const int4* items = nullptr;    // chunk items in row order (4-byte elements)
  const int4* items8 = nullptr;   // the same ordered by first entry (8-byte elements)
  int64_t nitems = 0;
  const int4* longs = nullptr;
  int64_t nlongs = 0;
};

// Tables of the level solve by runs (int64, dense niv rows), per map:
// ev[e] = {new row, old row, row, 0}: the entries j != own chain in which row
// `row` differs from the row below it in its chain (row n, a zero row of Y,
// for "no element"), grouped by row in ascending row order.  A level's chunks
// are {first row, (level << 6) | rows, first event, end event}: at most
// kSegRows consecutive rows of one chain, all in that level, and the events of
// all but the first of them.
constexpr int kSegRows = 32;
// Events per chunk (beyond the second row): a chunk's row groups take its
// events in batches of 16, one batch at a time, so bursts are split over
// chunks instead.
constexpr int kSegEvents = 64;
struct SegTables {
  const int4* ev = nullptr;
};

// Static description of one poset (or a batch of posets) on the device.
struct DevPoset {
  int32_t n = 0, k = 0;           // for a batch: total rows; k = 0 (per-poset k)
  const int32_t* node_of_row = nullptr;
  // 1: node_of_row is the identity (matrices in row order): kernels use the
  // row itself and skip the table loads
  int32_t ident = 0;
  const int32_t* chain_of_row = nullptr;
  const int32_t* chain_off = nullptr;   // chains+1
  int32_t nchains = 0;
  const int32_t* niv = nullptr;         // [n*k] or, for a batch, at niv_off[poset]
  const int32_t* niv_up = nullptr;
  // sparse niv rows, [0] niv / [1] up-niv (single posets; nullptr: dense):
  // row r's finite entries are nivr[m][nivp[m][r] .. nivp[m][r + 1]), ascending
  const int64_t* nivp[2] = {nullptr, nullptr};
  const int32_t* nivr[2] = {nullptr, nullptr};
  GatherSplit gsplit[2];
  const int32_t* segoff = nullptr;      // [7][nchains+1] tile offsets per tile height
  // per tile height (as segoff): every tile's {first row, end row of its chain}
  // (nullable), and the most tiles any chain has
  const int2* tiles[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  int32_t max_chain_tiles[7] = {0, 0, 0, 0, 0, 0, 0};
  int32_t max_chain = 0;                // rows of the longest chain
  // tile heights (bit segi) whose narrow-block scan takes flat tiles: rows in
  // fixed blocks of seg_rows, a chain start resetting the sum (short chains)
  uint32_t flat_mask = 0;
  // tables of the walking gather, [0] for niv (zeta), [1] for the up-niv map
  WalkTables walk[2];
  // level solves, [0] down / [1] up: the niv rows (k entries each) and node ids
  // of the rows in level order (nullable; single posets with k <= 64)
  const int32_t* lev_niv[2] = {nullptr, nullptr};
  const int32_t* lev_node[2] = {nullptr, nullptr};
  SegTables seg[2];  // level solve by runs (nullable)
  // single-pass scan: tiles in scan-position-major order, [0] prefix / [1] suffix,
  // one table per tile height (as segoff)
  const int32_t* scan_order[2][7] = {{nullptr}};
  // batch only
  const int64_t* niv_off = nullptr;     // element offset of each poset's niv block
  const int32_t* poset_of_row = nullptr;
  const int32_t* k_of_poset = nullptr;
  const int32_t* row_off = nullptr;     // first row of each poset
};

// Column tile width used by every kernel for B right-hand sides, and the
// scan tile height derived from it.
int col_width(int64_t B);
int seg_index(int cw);     // 0..6
int seg_rows(int cw);      // rows of one scan tile
// Column tile of the persistent int64 solve (launch_usolve_flow): col_width(B)
// up to 32, or a narrower power of two from POSETX_FLOW_CW (read on every call).
int flow_col_width(int64_t B);

// Chain scan V x (forward, dir=+1, prefix from the bottom) or V^T x (dir=-1,
// suffix from the top), three deterministic phases.  x is node order
// (ld ldx, element type tin); P is chain-major dense [n + 1, B] of type tout,
// row n set to zero.
// Scan state: compensated float for E_F32 -> E_F32, compensated double when
// tout is E_F64, wrapping uint64 for E_I64.  aux must hold 2 * ntiles * B *
// 16 bytes.
// phase: 0 = tile totals, 1 = carries, 2 = scan and write (run in this order).
hipError_t launch_chain_scan_phase(int phase, const DevPoset& d, int dir, ElemType tin, const void* x,
                                   int64_t ldx, ElemType tout, void* P, int64_t B, void* aux,
                                   int64_t ntiles, hipStream_t s);

// The same scan in one pass with a deterministic look-back between tiles.
// sync: 2 + ntiles * ceil(B / cw) int words of scratch (cleared by the launch).
// spin_limit bounds each wait for an earlier tile (polls); a tile that gives up
// sums the missing tiles from the input instead.
hipError_t launch_chain_scan_onepass(const DevPoset& d, int dir, ElemType tin, const void* x, int64_t ldx,
                                     ElemType tout, void* P, int64_t B, void* aux, int64_t ntiles, int* sync,
                                     int spin_limit, hipStream_t s);

// Gather-reduce U c: out[node(r)] = Σ_j P[nv[r][j]] over finite entries, in
// chain order (dense rows, or the sparse rows nivp / nivr when present).  With
// resid != nullptr (float64 P only): out = resid[node] - Σ (residual of a
// refinement step; resid has element type tres, leading dim ldr).
// Called around the two kernels of the walking gather (0 = events, 1 = combine),
// e.g. to record timing events on the launch stream.
struct LaunchHook {
  virtual void before(int kernel, hipStream_t s) = 0;
  virtual void after(int kernel, hipStream_t s) = 0;
  virtual ~LaunchHook() = default;
};

// snaps: scratch for walk[up].nsnap * B values of type tp (nullable: one-thread-per-row gather);
// for sparse rows with a split (gsplit), gsplit.nitems * B 8-byte chunk sums.
hipError_t launch_gather(const DevPoset& d, bool up, ElemType tp, const void* P, int64_t B,
                         ElemType tout, void* out, int64_t ldo, ElemType tres, const void* resid,
                         int64_t ldr, void* snaps, LaunchHook* hook, hipStream_t s);

// Zeta (dir=+1, niv map) or its adjoint (dir=-1, up map) through the
// compact walk, for a single poset with k <= 64 whose walk tables have the
// compact form (64-column tiles; with B < 64 the columns beyond B are masked
// and ntiles is the count of 64-row tiles whatever B is):
//   0. tile totals, and the tile-local prefixes at the gathered rows (L);
//   1. tile carries, and Q = carry + L at the gathered rows, Q[nslots] = 0;
//   2. walk events on Q into snapshots;
//   3. the scan inside each tile fused with the combine:
//      out[node(r)] = P[r] + S[snap_of_row[r]]
//      (or resid[node(r)] minus that, for a refinement residual).
// P never exists.  tin -> tout as for the scan (E_F32 -> E_F64 only with resid).
// aux: 2 * ntiles * B * 16 bytes (tile states); lq: (2 * nslots + 1) * B
// elements of tout; snaps: nsnap * B elements of tout.
// hook (nullable) is called around the four kernels (0..3).
bool compact_ok(const DevPoset& d, bool up, int64_t B);
hipError_t launch_zeta_compact(const DevPoset& d, int dir, ElemType tin, const void* x, int64_t ldx, ElemType tout,
                               void* out, int64_t ldo, ElemType tres, const void* resid, int64_t ldr, int64_t B,
                               void* aux, int64_t ntiles, void* lq, void* snaps, LaunchHook* hook, hipStream_t s);

// One level of the solve U y' = g: for the rows lev_rows[0..cnt),
// Y[r] = g[node(r)] - Σ_{j: nv[r][j] != r} Y[nv[r][j]].
// Before the levels of a solve into Y ([n + 1, B] of type ty): row n of Y set
// to zero (the uniform solve reads it for the own and missing niv entries).
hipError_t launch_usolve_begin(const DevPoset& d, ElemType ty, void* Y, int64_t B, hipStream_t s);

// i0: the level's first position in the level order (lev_rows = rows + i0).
hipError_t launch_usolve_level(const DevPoset& d, bool up, const int32_t* lev_rows, int64_t i0, int64_t cnt,
                               ElemType tin, const void* g, int64_t ldg, ElemType ty, void* Y,
                               int64_t B, hipStream_t s);

// The whole int64 solve by runs in one persistent launch (plus a clear and a
// fallback kernel; see k_usolve_flow): the chunks of every level in level
// order (nchunks), lev_off[l] the first chunk of level l (levels + 1 entries),
// and the chunks each chunk reads from: deps[dep_ptr[c] .. dep_ptr[c + 1]).
// wait: what a chunk waits for before it reads Y:
//   kWaitRows   a ready flag of every row it reads;
//   kWaitLevel  every chunk of the level below (one done flag per chunk);
//   kWaitDeps   every chunk it reads from (one done flag per chunk);
//   kWaitValues nothing: it reads the rows' values themselves until none is
//               the unwritten mark (rows 0 .. n-1 of Y are filled with it
//               first), a value equal to the mark being taken once the
//               row's ready flag is set.
// sync: 1 + ceil(B / flow_col_width(B)) * (n + 1) ints of scratch (chunk
// flags: nchunks instead of n + 1), cleared by the launch.  spin_limit bounds
// each wait (polls); a wait that gives up makes the fallback recompute the
// solve in one workgroup.  max_grid > 0 caps the workgroups.  B >= 5.
constexpr int kWaitRows = 0, kWaitLevel = 1, kWaitDeps = 2, kWaitValues = 3;
hipError_t launch_usolve_flow(const DevPoset& d, bool up, const int4* chunks, int64_t nchunks, const int32_t* lev_off,
                              const int32_t* dep_ptr, const int32_t* deps, int wait, const void* g, int64_t ldg, void* Y,
                              int64_t B, int* sync, int spin_limit, int max_grid, hipStream_t s);

// The row-by-row level solve (dense niv rows, the per-level kernels' sums, so
// results equal them bit for bit) for every level in one persistent launch:
// rows, the level-ordered rows (cnt), lev_ptr (device, nlev + 1 entries) the
// first position of every level, lev_bits (device, one bit per position,
// ceil((cnt + 1) / 64) words) set at those first positions.  Rows 0 .. n-1 of
// Y are first filled with a mark; a row's lanes read the rows it needs until
// none holds the mark (int64: a legitimate value equal to it is taken once
// that row's ready flag is set).  One row per wavefront for B > 32, else 8,
// 16 or 32 columns per row and several rows per wavefront.  sync:
// usolve_poll_ints(n, B) ints of scratch, cleared by the launch.  spin_limit
// bounds each wait (polls); a wait that gives up makes a one-workgroup
// fallback solve again level by level.  max_grid > 0 caps the workgroups.
// Row n of Y must be zero (launch_usolve_begin).
int64_t usolve_poll_ints(int64_t n, int64_t B);
// Wavefronts of that launch the device holds resident at once (0: none), and
// the rows each takes at a time.
int64_t usolve_poll_waves(ElemType tin, ElemType ty, int64_t n, int64_t B);
int usolve_poll_rows_per_wave(int64_t B);
hipError_t launch_usolve_poll(const DevPoset& d, bool up, const int32_t* rows, const int32_t* lev_ptr,
                              const uint64_t* lev_bits, int nlev, int64_t cnt, ElemType tin, const void* g,
                              int64_t ldg, ElemType ty, void* Y, int64_t B, int* sync, int spin_limit, int max_grid,
                              hipStream_t s);

// One level of the int64 solve by runs (dense niv rows, B >= 5): the chunks
// of that level (see SegTables).
// g and Y are int64; the result equals launch_usolve_level's bit for bit.
hipError_t launch_usolve_runs(const DevPoset& d, bool up, const int4* chunks, int64_t nchunks, const void* g,
                              int64_t ldg, void* Y, int64_t B, hipStream_t s);

// The long rows of a level of a sparse solve, split into chunks: items =
// {row, first entry, end entry, w} (nitems, in any order; w: the chunk's slot
// in part), longs[j] = {row, first slot, chunks, 0} (nlongs; a row's chunks
// take consecutive slots in entry order).  Y[row] = g[node(row)] minus the
// chunk sums in order.  part: nitems * B 8-byte words of scratch.
hipError_t launch_usolve_split(const DevPoset& d, bool up, const int4* items, int64_t nitems, const int4* longs,
                               int64_t nlongs, ElemType tin, const void* g, int64_t ldg, ElemType ty, void* Y,
                               int64_t B, void* part, hipStream_t s);

// y = V^{-1} y' (dir=+1: minus the element below in the chain; dir=-1: minus the
// element above).  accumulate: out += result instead of out = result.
// stats (nullable, float32/float64 only): 2B+1 uint64 words that receive the
// per-column max |correction|, max |result| and a non-finite flag.
hipError_t launch_chain_diff(const DevPoset& d, int dir, ElemType ty, const void* Y, int64_t B,
                             ElemType tout, void* out, int64_t ldo, bool accumulate, uint64_t* stats,
                             hipStream_t s);

// Per-column max|r| (float64 [n, B], ld B) and max|g| (type tg, ld ldg) plus a
// non-finite flag into stats[2*B + 1] (as uint64 bit patterns / 0-1).
hipError_t launch_absmax(int64_t n, int64_t B, const double* r, ElemType tg, const void* g,
                         int64_t ldg, uint64_t* stats, hipStream_t s);

}  // namespace px
