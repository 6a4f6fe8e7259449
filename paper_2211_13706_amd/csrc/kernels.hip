// gfx950 kernels of the fast zeta / Möbius transforms.
//
// The transforms factor as Z = U V (§3): V sums every chain from the bottom
// up to each element (a prefix scan along chain-major rows), U gathers for
// every element x the chain prefixes ending at niv_j(x) (§2.4, Eq.
// zeta-fast).  The Möbius transform solves U y' = g by substitution,
// level by level, then applies V^{-1}, one subtraction per element (§3, Alg. 4).
//
// For a single poset with at most 64 chains and 64-column blocks the zeta
// transform never forms V f: the scan completes the prefixes only at the rows
// U reads, and U's own-chain term is added inside the scan's last pass (the
// compact walk: k_scan_reduce / k_scan_carry with MARK, k_walk_events with
// COMPACT, k_scan_apply modes 1 and 2).
//
// Thread layout shared by all kernels: a 256-thread workgroup covers `cw`
// consecutive right-hand-side columns (lanes) times 256/cw rows, so that the
// lanes of a wavefront read contiguous bytes of a row; B is padded to cw.
// Everything here is a scan or an integer-indexed gather: VALU + HBM work, no
// MFMA.
#include <atomic>
#include <cstring>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "kernels.h"

namespace px {

constexpr int WG = 256;
constexpr int RPT = 16;          // rows per thread in a scan tile
constexpr int COMBINE_ROWS = 8;  // rows per thread in the walk's combine pass

int col_width(int64_t B) {
  int cw = 1;
  while (cw < B && cw < 64) cw <<= 1;
  return cw;
}
int seg_index(int cw) {
  int i = 0;
  while ((1 << i) < cw) ++i;
  return i;
}
int seg_rows(int cw) { return (WG / cw) * RPT; }

// 16 columns at most.  Polling the values it reads (n = 2^20, k = 64, B = 64,
// 512 workgroups) the solve took 2.04 ms in 16-column items against 2.46 ms in
// 32-column ones (8: 2.54 ms; at n = 2^23, k = 32, B = 16, 16 columns 5.70 ms,
// 8 columns 5.64): a narrow item moves fewer bytes between its reads and its
// stores, and more items of a level run at once.
int flow_col_width(int64_t B) {
  const int cw = std::min(col_width(B), 16);
  const char* e = std::getenv("POSETX_FLOW_CW");
  if (e && *e) {
    const int v = std::atoi(e);
    if ((v == 8 || v == 16 || v == 32 || v == 64) && v <= cw) return v;
  }
  return cw;
}

// Every byte offset of a buffer of `bytes` fits an unsigned 32-bit offset
// (POSETX_O32=0, read on every call, takes 64-bit offsets everywhere).
bool fits32(int64_t bytes) {
  const char* e = std::getenv("POSETX_O32");
  if (e && e[0] == '0') return false;
  return bytes >= 0 && bytes <= (int64_t)0xffffffffu;
}

namespace {

constexpr int reduce_tiles(int cwt) { return cwt == 64 ? 1 : 2; }

// ------------------------------------------------------------------ scan state
// Wrapping 64-bit integer sum (two's complement modulo 2^64).
struct StateI {
  uint64_t s;
  __device__ void zero() { s = 0; }
  __device__ void add(uint64_t x) { s += x; }
  __device__ void combine(const StateI& o) { s += o.s; }
  __device__ uint64_t value() const { return s; }
};

// Compensated floating-point sum: s + e carries the running total, and each
// addition's rounding error (TwoSum, Knuth) is accumulated in e
// (Kahan-Babuska-Neumaier).  Order-independent combination lets tiles be
// summed in parallel.  No multiplications, so contraction cannot change it.
template <typename F>
struct StateF {
  F s, e;
  __device__ void zero() { s = F(0); e = F(0); }
  __device__ void add(F x) {
    F t = s + x;
    F bp = t - s;
    F err = (s - (t - bp)) + (x - bp);
    s = t;
    e += err;
  }
  __device__ void combine(const StateF& o) {
    F t = s + o.s;
    F bp = t - s;
    F err = (s - (t - bp)) + (o.s - bp);
    s = t;
    e += o.e + err;
  }
  __device__ F value() const { return s + e; }
};

template <typename Tin, typename Tout> struct ScanTraits;
template <> struct ScanTraits<int64_t, int64_t> {
  using St = StateI;
  __device__ static uint64_t in(int64_t x) { return (uint64_t)x; }
  __device__ static int64_t out(uint64_t v) { return (int64_t)v; }
};
template <> struct ScanTraits<float, float> {
  using St = StateF<float>;
  __device__ static float in(float x) { return x; }
  __device__ static float out(float v) { return v; }
};
template <> struct ScanTraits<double, double> {
  using St = StateF<double>;
  __device__ static double in(double x) { return x; }
  __device__ static double out(double v) { return v; }
};
template <> struct ScanTraits<float, double> {
  using St = StateF<double>;
  __device__ static double in(float x) { return (double)x; }
  __device__ static double out(double v) { return v; }
};

// accumulation type of sums of TP values (exact wrap for int64)
template <typename T> struct Wide;
template <> struct Wide<int64_t> { using W = uint64_t; };
template <> struct Wide<float> { using W = double; };
template <> struct Wide<double> { using W = double; };

__device__ inline int find_chain(const int32_t* so, int nchains, int t) {
  int lo = 0, hi = nchains;  // so[lo] <= t < so[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (so[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

// Address of element (row, col) of a matrix with leading dimension ld.  With
// O32 (the launcher checked that every offset of the matrix fits 32 bits) the
// offset is a 32-bit lane value from a scalar base: one register per address
// and no 64-bit multiply.
template <bool O32, typename T>
__device__ inline T* elem(T* base, int64_t row, int64_t ld, int64_t col) {
  if constexpr (O32)
    return (T*)((char*)base + ((uint32_t)row * (uint32_t)ld + (uint32_t)col) * (uint32_t)sizeof(T));
  else
    return base + row * ld + col;
}

// Matrix row of chain-major row r: the node, or r itself in the row layout
// (d.ident, uniform), where the table load is skipped.
__device__ inline int node_at(const DevPoset& d, int64_t r) { return d.ident ? (int)r : d.node_of_row[r]; }

// Phase 1: per tile and column, the compensated total of the tile's rows.  A
// workgroup reduces reduce_tiles(CWT) tiles: two for narrow column blocks, so
// that each thread has 2*RPT loads in flight; one for 64-column blocks, whose
// tile rows come from one scalar table load (measured faster at n = 2^20).
// With CWT = 64 a row group is one wavefront, so its row (and node) indices
// are wave-uniform and live in scalar registers.
//
// MARK (compact walk, 64-column blocks): also the tile-local prefix (from the
// tile's first row in scan order) at every gathered row, into L[slot].  Rows
// of a tile are marked in tmask[t]; their slots are consecutive from qoff[t].
// Each wavefront sums its rows in scan order and keeps its running sum at its
// first MK marked rows in LDS; after the barrier each of them is combined with
// the sum of the row groups before it.  A wavefront with more marks (rare)
// sums its rows again for the rest.
template <typename Tin, typename Tout, int CWT, bool MARK, bool O32 = false>
__global__ __launch_bounds__(WG) void k_scan_reduce(DevPoset d, int segi, int cw_rt, const Tin* __restrict__ x,
                                                    int64_t ldx, int64_t B, int64_t ntiles,
                                                    typename ScanTraits<Tin, Tout>::St* __restrict__ A, int dir,
                                                    const uint64_t* __restrict__ tmask,
                                                    const int32_t* __restrict__ qoff, Tout* __restrict__ L) {
  using Tr = ScanTraits<Tin, Tout>;
  using St = typename Tr::St;
  static_assert(!MARK || CWT == 64, "marked rows need wave-uniform row groups");
  constexpr int NT = reduce_tiles(CWT);
  const int cw = CWT ? CWT : cw_rt;
  __shared__ St sm[NT][WG];
  const int32_t* so = d.segoff + (int64_t)segi * (d.nchains + 1);
  const int seg = (WG / cw) * RPT;
  // with 64-wide column blocks the row group is the wavefront index: uniform
  const int lane = threadIdx.x % cw;
  const int rg = CWT == 64 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64)) : (int)(threadIdx.x / cw);
  const int64_t col = (int64_t)blockIdx.y * cw + lane;
  const int64_t colc = col < B ? col : 0;
  int64_t r0[NT], end[NT];
  uint64_t tm[NT];  // MARK: the tiles' marks and first slots, loaded with the rows
  int qo[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    const int t = min((int64_t)blockIdx.x * NT + q, ntiles - 1);
    if (MARK) {
      tm[q] = tmask[t];
      qo[q] = qoff[t];
    }
    if (d.tiles[segi]) {  // one (scalar) load instead of a search over the chains
      const int2 tr = d.tiles[segi][t];
      r0[q] = tr.x + (int64_t)rg * RPT;
      end[q] = tr.y;
    } else {
      const int c = find_chain(so, d.nchains, t);
      r0[q] = d.chain_off[c] + (int64_t)(t - so[c]) * seg + (int64_t)rg * RPT;
      end[q] = d.chain_off[c + 1];
    }
  }
  // row indices first, then every load unconditionally (rows clamped into the
  // chain, columns into the matrix), so that all loads are in flight together
  int32_t nodes[NT][RPT];
#pragma unroll
  for (int q = 0; q < NT; ++q)
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      nodes[q][i] = node_at(d, min(r0[q] + i, end[q] - 1));
      if (CWT == 64) nodes[q][i] = __builtin_amdgcn_readfirstlane(nodes[q][i]);
    }
  Tin v[NT][RPT];
#pragma unroll
  for (int q = 0; q < NT; ++q)
#pragma unroll
    for (int i = 0; i < RPT; ++i) v[q][i] = *elem<O32>(x, nodes[q][i], ldx, colc);
  // MARK: this wavefront's marked rows (bits of its RPT rows, scalar)
  constexpr int MK = 4;
  __shared__ St lm[MARK ? NT * MK : 1][WG];
  uint32_t wm[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q)
    wm[q] = (MARK && (int64_t)blockIdx.x * NT + q < ntiles) ? (uint32_t)(tm[q] >> (rg * RPT)) & ((1u << RPT) - 1)
                                                          : 0u;
#pragma unroll
  for (int q = 0; q < NT; ++q) {
    St st;
    st.zero();
    int m = 0;
    // MARK sums in scan order (dir < 0: from the top) and keeps the running sum at marks
    auto step = [&](int i) {
      if (r0[q] + i < end[q]) st.add(Tr::in(v[q][i]));
      if (MARK && ((wm[q] >> i) & 1)) {
        if (m < MK) lm[q * MK + m][threadIdx.x] = st;
        ++m;
      }
    };
    if (MARK && dir < 0) {
#pragma unroll
      for (int i = RPT - 1; i >= 0; --i) step(i);
    } else {
#pragma unroll
      for (int i = 0; i < RPT; ++i) step(i);
    }
    sm[q][threadIdx.x] = st;
  }
  __syncthreads();
  if constexpr (MARK) {
    constexpr int RG = WG / 64;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      if (wm[q] == 0) continue;
      const int nm = __popc(wm[q]);
      // slots of this wavefront's marks, in scan order: from first, by sgn
      const int below = __popcll(tm[q] & ((uint64_t(1) << (rg * RPT)) - 1));
      const int first = dir > 0 ? qo[q] + below : qo[q] + below + nm - 1;
      const int sgn = dir > 0 ? 1 : -1;
      St base;  // the row groups before this one in scan order
      base.zero();
      if (dir > 0) {
        for (int g = 0; g < rg; ++g) base.combine(sm[q][g * 64 + lane]);
      } else {
        for (int g = RG - 1; g > rg; --g) base.combine(sm[q][g * 64 + lane]);
      }
      for (int m = 0; m < min(nm, MK); ++m) {
        St pre = base;
        pre.combine(lm[q * MK + m][threadIdx.x]);
        if (col < B) __builtin_nontemporal_store(Tr::out(pre.value()), &L[(int64_t)(first + sgn * m) * B + col]);
      }
      if (nm > MK) {
        St pre = base;
        int m = 0;
        auto step = [&](int i) {
          if (r0[q] + i < end[q]) pre.add(Tr::in(v[q][i]));
          if ((wm[q] >> i) & 1) {
            if (m >= MK && col < B)
              __builtin_nontemporal_store(Tr::out(pre.value()), &L[(int64_t)(first + sgn * m) * B + col]);
            ++m;
          }
        };
        if (dir < 0) {
#pragma unroll
          for (int i = RPT - 1; i >= 0; --i) step(i);
        } else {
#pragma unroll
          for (int i = 0; i < RPT; ++i) step(i);
        }
      }
    }
  }
  if (rg == 0 && col < B) {
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int64_t t = (int64_t)blockIdx.x * NT + q;
      if (t < ntiles) {
        St tot = sm[q][lane];
        for (int g = 1; g < WG / cw; ++g) tot.combine(sm[q][g * cw + lane]);
        A[t * B + col] = tot;
      }
    }
  }
}

// Phase 2: exclusive scan of the tile totals along every chain, per column.
// One workgroup per (chain, 16 columns): windows of 128 tile totals are staged
// in LDS, each of 16 thread groups combines 8 of them, the group totals are
// combined in order, and the carries are written; a running carry links the
// windows.  The combination order is fixed, so results are reproducible.
//
// MARK (compact walk): the carries of a window stay in LDS and the gathered
// rows of its tiles are completed, Q[slot] = carry(tile) + L[slot].  The
// gridDim.z workgroups of one (chain, column block) each scan the chain's
// tile totals (LDS work) and complete their share of the slots; the first of
// them writes the carries.
template <typename St, typename Tout, bool MARK>
__global__ __launch_bounds__(WG) void k_scan_carry(DevPoset d, int segi, int dir, int64_t B,
                                                   const St* __restrict__ A, St* __restrict__ C,
                                                   Tout* __restrict__ P, const int32_t* __restrict__ qoff,
                                                   const int32_t* __restrict__ tile_of_slot,
                                                   const Tout* __restrict__ L, int32_t nslots) {
  constexpr int CB = 16, NS = WG / CB, TPS = 16, WIN = NS * TPS;
  __shared__ St sh[WIN * CB];
  __shared__ St tot[NS * CB];
  const int c = blockIdx.x;
  const int64_t c0 = (int64_t)blockIdx.y * CB;
  const int lc = threadIdx.x % CB, sg = threadIdx.x / CB;
  const int64_t col = c0 + lc;
  const bool lead = blockIdx.z == 0;
  // the zero row (row n of P, or slot nslots of Q) stays zero: the walk reads
  // it for "no element"
  if (c == 0 && lead && sg == 0 && col < B) P[(int64_t)(MARK ? nslots : d.n) * B + col] = Tout(0);
  const int32_t* so = d.segoff + (int64_t)segi * (d.nchains + 1);
  const int t0 = so[c], t1 = so[c + 1], nt = t1 - t0;
  St carry;
  carry.zero();
  constexpr int U = 8;  // MARK: slots completed per thread and batch, loads in flight together
  for (int w0 = 0; w0 < nt; w0 += WIN) {
    // MARK: this workgroup's share [a0, a0 + cnt / CB) of the window's slots; the
    // first batch of their tiles and L values loads together with the window
    int a0 = 0, cnt = 0;
    int ti[U];
    Tout lv[U];
    auto load_batch = [&](int x0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int x = min(x0 + u * WG, cnt - 1);
        ti[u] = tile_of_slot[a0 + x / CB];
        lv[u] = L[(int64_t)(a0 + x / CB) * B + (col < B ? col : 0)];
      }
    };
    if constexpr (MARK) {
      const int wn = min(WIN, nt - w0);
      const int tlo = dir > 0 ? t0 + w0 : t1 - w0 - wn;  // the window's tiles in index order
      const int s0 = qoff[tlo], s1 = qoff[tlo + wn];
      const int per = (s1 - s0 + (int)gridDim.z - 1) / (int)gridDim.z;
      a0 = s0 + (int)blockIdx.z * per;
      cnt = max(min(s1, a0 + per) - a0, 0) * CB;
      if ((int)threadIdx.x < cnt) load_batch(threadIdx.x);
    }
    {
      // the window's WIN * CB totals, WIN * CB / WG per thread, all loads in
      // flight before the LDS stores (addresses clamped, outside values zero)
      constexpr int PER = WIN * CB / WG;
      St v[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int x = (int)threadIdx.x + u * WG;
        const int i = w0 + x / CB;
        const int64_t cc = c0 + x % CB;
        const int ic = min(i, nt - 1);
        const int64_t ccc = cc < B ? cc : B - 1;
        v[u] = A[(int64_t)(dir > 0 ? t0 + ic : t1 - 1 - ic) * B + ccc];
        if (i >= nt || cc >= B) v[u].zero();
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) sh[threadIdx.x + u * WG] = v[u];
    }
    __syncthreads();
    St part;
    part.zero();
#pragma unroll
    for (int u = 0; u < TPS; ++u) part.combine(sh[(sg * TPS + u) * CB + lc]);
    tot[sg * CB + lc] = part;
    __syncthreads();
    St pre = carry;
    for (int g = 0; g < sg; ++g) pre.combine(tot[g * CB + lc]);
#pragma unroll
    for (int u = 0; u < TPS; ++u) {
      const int i = w0 + sg * TPS + u;
      if (lead && i < nt && col < B) C[(int64_t)(dir > 0 ? t0 + i : t1 - 1 - i) * B + col] = pre;
      const St a = sh[(sg * TPS + u) * CB + lc];
      if (MARK) sh[(sg * TPS + u) * CB + lc] = pre;  // this thread's own entry: read just before
      pre.combine(a);
    }
    for (int g = 0; g < NS; ++g) carry.combine(tot[g * CB + lc]);
    if constexpr (MARK) {
      __syncthreads();
      // Q[slot] = carry of the slot's tile (in sh) + L[slot]
      for (int x0 = threadIdx.x; x0 < cnt; x0 += WG * U) {
        if (x0 != (int)threadIdx.x) load_batch(x0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int x = x0 + u * WG;
          if (x < cnt && col < B) {
            const int i = (dir > 0 ? ti[u] - t0 : t1 - 1 - ti[u]) - w0;  // position in the window
            St q = sh[i * CB + lc];
            q.add((decltype(q.value()))lv[u]);
            P[(int64_t)(a0 + x / CB) * B + col] = (Tout)q.value();
          }
        }
      }
    }
    __syncthreads();
  }
}

// Phase 2 for posets whose chains have few tiles (at most kShortCarry): one
// thread per (chain, column) folds the chain's tile totals in scan order,
// eight loads in flight, instead of a workgroup staging windows in LDS.  The
// combination order is that of the windowed kernel's prefix, so both are
// reproducible (they may differ from each other in the last bits).
constexpr int kShortCarry = 64;
template <typename St, typename Tout>
__global__ __launch_bounds__(WG) void k_scan_carry_short(DevPoset d, int segi, int dir, int64_t B,
                                                         const St* __restrict__ A, St* __restrict__ C,
                                                         Tout* __restrict__ P) {
  const int64_t idx = (int64_t)blockIdx.x * WG + threadIdx.x;
  const int64_t c = idx / B, col = idx % B;
  if (c >= d.nchains) return;
  if (c == 0) P[(int64_t)d.n * B + col] = Tout(0);  // the walk's zero row
  const int32_t* so = d.segoff + (int64_t)segi * (d.nchains + 1);
  const int t0 = so[c], t1 = so[c + 1], nt = t1 - t0;
  St carry;
  carry.zero();
  for (int i0 = 0; i0 < nt; i0 += 8) {
    St a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = min(i0 + u, nt - 1);
      a[u] = A[(int64_t)(dir > 0 ? t0 + i : t1 - 1 - i) * B + col];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u;
      if (i < nt) {
        C[(int64_t)(dir > 0 ? t0 + i : t1 - 1 - i) * B + col] = carry;
        carry.combine(a[u]);
      }
    }
  }
}

// Phase 3: scan inside the tile from its carry; write P chain-major.  This is
// the last read of f and P is not read back soon: both streams are
// non-temporal, so that f read by phase 1 stays in the MALL for this read and
// the next call's phase 1.
//
// MODE 1 / 2 (compact walk, 64-column blocks): instead of writing P[r], add
// the other chains' sum S[snap_of_row[r]] (from the walk) and write the zeta
// value out[node(r)] = P[r] + S (MODE 1), or the refinement residual
// out[node(r)] = res[node(r)] - (P[r] + S) (MODE 2).
template <typename Tin, typename Tout, int CWT, int MODE, typename Tres, bool O32 = false>
__global__ __launch_bounds__(WG) void k_scan_apply(DevPoset d, int segi, int cw_rt, int dir,
                                                   const Tin* __restrict__ x, int64_t ldx, int64_t B,
                                                   const typename ScanTraits<Tin, Tout>::St* __restrict__ C,
                                                   Tout* __restrict__ P, const int32_t* __restrict__ snap_of_row,
                                                   const Tout* __restrict__ S, int64_t ldo,
                                                   const Tres* __restrict__ res, int64_t ldr) {
  using Tr = ScanTraits<Tin, Tout>;
  using St = typename Tr::St;
  using W = typename Wide<Tout>::W;
  static_assert(MODE == 0 || CWT == 64, "the fused combine needs wave-uniform rows");
  const int cw = CWT ? CWT : cw_rt;
  using Tv = decltype(Tr::in(Tin()));
  __shared__ St sm[WG];
  const int t = blockIdx.x;
  const int RG = WG / cw;
  int64_t base, end;
  if (d.tiles[segi]) {  // one (scalar) load instead of a search over the chains
    const int2 tr = d.tiles[segi][t];
    base = tr.x;
    end = tr.y;
  } else {
    const int32_t* so = d.segoff + (int64_t)segi * (d.nchains + 1);
    const int c = find_chain(so, d.nchains, t);
    base = d.chain_off[c] + (int64_t)(t - so[c]) * (RG * RPT);
    end = d.chain_off[c + 1];
  }
  // with 64-wide column blocks the row group is the wavefront index: uniform
  const int lane = threadIdx.x % cw;
  const int rg = CWT == 64 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64)) : (int)(threadIdx.x / cw);
  const int64_t col = (int64_t)blockIdx.y * cw + lane;
  const int64_t r0 = base + (int64_t)rg * RPT;
  const int64_t colc = col < B ? col : 0;
  int32_t nodes[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    nodes[i] = node_at(d, min(r0 + i, end - 1));
    if (CWT == 64) nodes[i] = __builtin_amdgcn_readfirstlane(nodes[i]);
  }
  Tin raw[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) raw[i] = __builtin_nontemporal_load(elem<O32>(x, nodes[i], ldx, colc));
  // MODE != 0: the rows' snapshots; consecutive rows mostly share one, which
  // is loaded once (scalar tests) and copied once the loads have returned
  Tout sv[MODE ? RPT : 1];
  int32_t sn[MODE ? RPT : 1];
  Tres rv[MODE == 2 ? RPT : 1];  // MODE 2: the residual's right-hand side, loaded with f
  if constexpr (MODE != 0) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) sn[i] = __builtin_amdgcn_readfirstlane(snap_of_row[min(r0 + i, end - 1)]);
#pragma unroll
    for (int i = 0; i < RPT; ++i)
      if (i == 0 || sn[i] != sn[i - 1]) sv[i] = (S + (int64_t)sn[i] * B)[colc];
  }
  if constexpr (MODE == 2) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) rv[i] = res[(int64_t)nodes[i] * ldr + colc];
  }
  // row i's result: P[r] itself, or the combined zeta value / residual
  auto put = [&](int i, const St& st) {
    const int64_t r = r0 + i;
    if (r >= end) return;
    if constexpr (MODE == 0) {
      // a narrow tile's store covers pieces of several lines: leave it to L2 to merge them
      if (CWT == 64)
        __builtin_nontemporal_store(Tr::out(st.value()), &P[r * B + col]);
      else
        *elem<O32>(P, r, B, col) = Tr::out(st.value());
    } else if constexpr (MODE == 1) {
      __builtin_nontemporal_store((Tout)((W)Tr::out(st.value()) + (W)sv[i]), &P[(int64_t)nodes[i] * ldo + col]);
    } else {
      __builtin_nontemporal_store((Tout)((double)rv[i] - ((W)Tr::out(st.value()) + (W)sv[i])),
                                  &P[(int64_t)nodes[i] * ldo + col]);
    }
  };
  Tv v[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) v[i] = (r0 + i < end) ? Tr::in(raw[i]) : Tv(0);
  St loc;
  loc.zero();
  if (dir > 0) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) loc.add(v[i]);
  } else {
#pragma unroll
    for (int i = RPT - 1; i >= 0; --i) loc.add(v[i]);
  }
  sm[threadIdx.x] = loc;
  __syncthreads();
  // the row groups before this one in scan order: folded one by one for a few
  // groups; for narrow column tiles (up to 32 groups) an inclusive scan over the
  // groups in LDS, log2(RG) steps in a fixed order
  St pre;
  pre.zero();
  if (RG <= 4) {
    if (dir > 0) {
      for (int g = 0; g < rg; ++g) pre.combine(sm[g * cw + lane]);
    } else {
      for (int g = RG - 1; g > rg; --g) pre.combine(sm[g * cw + lane]);
    }
  } else {
    for (int off = 1; off < RG; off <<= 1) {
      const int src = dir > 0 ? rg - off : rg + off;
      const bool has = src >= 0 && src < RG;
      St a;
      if (has) a = sm[src * cw + lane];
      __syncthreads();
      if (has) {
        a.combine(sm[threadIdx.x]);
        sm[threadIdx.x] = a;
      }
      __syncthreads();
    }
    const int src = dir > 0 ? rg - 1 : rg + 1;
    if (src >= 0 && src < RG) pre = sm[src * cw + lane];
  }
  if (col >= B) return;
  if constexpr (MODE != 0) {
#pragma unroll
    for (int i = 1; i < RPT; ++i)
      if (sn[i] == sn[i - 1]) sv[i] = sv[i - 1];
  }
  St st;
  if (C) {
    st = C[(int64_t)t * B + col];
  } else {  // every chain fits one tile: no carries; this kernel keeps row n of P zero
    st.zero();
    if (MODE == 0 && t == 0 && rg == 0) P[(int64_t)d.n * B + col] = Tout(0);
  }
  st.combine(pre);
  if (dir > 0) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      st.add(v[i]);
      put(i, st);
    }
  } else {
#pragma unroll
    for (int i = RPT - 1; i >= 0; --i) {
      st.add(v[i]);
      put(i, st);
    }
  }
}

// Flat tiles (narrow column blocks of posets with short chains, such as
// batches of small posets): tile t holds rows [t * H, min(n, t * H + H)),
// H = seg_rows(cw), whatever chains they belong to, so every tile but the last
// is full; chain-aligned tiles of chains much shorter than H are mostly empty.
// The scan is segmented: a chain's first row in scan order (its bottom row for
// dir > 0, its top row for dir < 0) starts a new sum.  Phases as for the
// chain-aligned scan:
//   0. A[t]: the compensated total of tile t's last segment in scan order;
//   1. C[t]: the fold, in scan order, of A over the earlier tiles of the chain
//      open at tile t's first row in scan order (zero when it starts there);
//   2. the segmented scan inside each tile from C[t], written to P.
// Row r starts a segment when its neighbour below (dir > 0) or above (dir < 0)
// belongs to another chain.
__device__ inline bool flat_seg_start(const int32_t* __restrict__ cor, int64_t n, int64_t r, int dir) {
  const int64_t q = r - dir;
  return q < 0 || q >= n || cor[q] != cor[r];
}

// Segmented fold: (seen, st) after (f, x) is x when f (a start inside x), else st + x.
template <typename St>
__device__ inline void seg_fold(St& st, bool f, const St& x) {
  if (f) st = x;
  else st.combine(x);
}

template <typename Tin, typename Tout>
struct FlatRows {
  using Tr = ScanTraits<Tin, Tout>;
  using Tv = decltype(Tr::in(Tin()));
  Tv v[RPT];
  bool seg[RPT];
  // the RPT rows of row group rg of tile t: values (zero beyond n) and segment starts
  template <bool O32>
  __device__ void load(const DevPoset& d, int64_t t, int H, int rg, int dir, const Tin* __restrict__ x, int64_t ldx,
                       int64_t colc) {
    const int64_t n = d.n;
    const int64_t r0 = t * H + (int64_t)rg * RPT;
    int32_t nodes[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) nodes[i] = node_at(d, min(r0 + i, n - 1));
    Tin raw[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) raw[i] = __builtin_nontemporal_load(elem<O32>(x, nodes[i], ldx, colc));
#pragma unroll
    for (int i = 0; i < RPT; ++i) seg[i] = r0 + i < n && flat_seg_start(d.chain_of_row, n, r0 + i, dir);
#pragma unroll
    for (int i = 0; i < RPT; ++i) v[i] = r0 + i < n ? Tr::in(raw[i]) : Tv(0);
  }
  // this row group's own (seen, total of its last segment) in scan order
  template <typename St>
  __device__ void local(int dir, bool& seen, St& st) const {
    seen = false;
    st.zero();
    auto step = [&](int i) {
      if (seg[i]) {
        st.zero();
        seen = true;
      }
      st.add(v[i]);
    };
    if (dir > 0) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) step(i);
    } else {
#pragma unroll
      for (int i = RPT - 1; i >= 0; --i) step(i);
    }
  }
};

template <typename Tin, typename Tout, bool O32>
__global__ __launch_bounds__(WG) void k_scan_reduce_flat(DevPoset d, int cw, int dir, const Tin* __restrict__ x,
                                                         int64_t ldx, int64_t B,
                                                         typename ScanTraits<Tin, Tout>::St* __restrict__ A) {
  using St = typename ScanTraits<Tin, Tout>::St;
  __shared__ St sm[WG];
  __shared__ int sf[WG];
  const int RG = WG / cw, H = RG * RPT;
  const int64_t t = blockIdx.x;
  const int lane = threadIdx.x % cw, rg = threadIdx.x / cw;
  const int64_t col = (int64_t)blockIdx.y * cw + lane;
  FlatRows<Tin, Tout> fr;
  fr.template load<O32>(d, t, H, rg, dir, x, ldx, col < B ? col : 0);
  bool seen;
  St st;
  fr.local(dir, seen, st);
  sm[threadIdx.x] = st;
  sf[threadIdx.x] = seen;
  __syncthreads();
  if (rg == 0 && col < B) {
    St acc;
    acc.zero();
    if (dir > 0) {
      for (int g = 0; g < RG; ++g) seg_fold(acc, sf[g * cw + lane] != 0, sm[g * cw + lane]);
    } else {
      for (int g = RG - 1; g >= 0; --g) seg_fold(acc, sf[g * cw + lane] != 0, sm[g * cw + lane]);
    }
    A[t * B + col] = acc;
  }
}

// One thread per (tile, column); also clears row n of P (the walk's zero row).
template <typename St, typename Tout>
__global__ __launch_bounds__(WG) void k_scan_carry_flat(DevPoset d, int H, int64_t ntiles, int dir, int64_t B,
                                                        const St* __restrict__ A, St* __restrict__ C,
                                                        Tout* __restrict__ P) {
  const int64_t idx = (int64_t)blockIdx.x * WG + threadIdx.x;
  const int64_t t = idx / B, col = idx % B;
  if (t >= ntiles) return;
  const int64_t n = d.n;
  if (t == 0) P[n * B + col] = Tout(0);
  const int64_t first = dir > 0 ? t * H : min(n, t * H + H) - 1;  // the tile's first row in scan order
  const int c = d.chain_of_row[first];
  const int64_t start = dir > 0 ? d.chain_off[c] : d.chain_off[c + 1] - 1;
  const int64_t u0 = start / H;
  St acc;
  acc.zero();
  if (u0 != t) {
    acc = A[u0 * B + col];
    for (int64_t u = u0 + dir; u != t; u += dir) acc.combine(A[u * B + col]);
  }
  C[t * B + col] = acc;
}

template <typename Tin, typename Tout, bool O32>
__global__ __launch_bounds__(WG) void k_scan_apply_flat(DevPoset d, int cw, int dir, const Tin* __restrict__ x,
                                                        int64_t ldx, int64_t B,
                                                        const typename ScanTraits<Tin, Tout>::St* __restrict__ C,
                                                        Tout* __restrict__ P) {
  using Tr = ScanTraits<Tin, Tout>;
  using St = typename Tr::St;
  __shared__ St sm[WG];
  __shared__ int sf[WG];
  const int RG = WG / cw, H = RG * RPT;
  const int64_t t = blockIdx.x;
  const int lane = threadIdx.x % cw, rg = threadIdx.x / cw;
  const int64_t col = (int64_t)blockIdx.y * cw + lane;
  FlatRows<Tin, Tout> fr;
  fr.template load<O32>(d, t, H, rg, dir, x, ldx, col < B ? col : 0);
  bool seen;
  St loc;
  fr.local(dir, seen, loc);
  sm[threadIdx.x] = loc;
  sf[threadIdx.x] = seen;
  __syncthreads();
  // inclusive segmented scan over the row groups in scan order, log2(RG) steps
  for (int off = 1; off < RG; off <<= 1) {
    const int src = dir > 0 ? rg - off : rg + off;
    const bool has = src >= 0 && src < RG;
    St a;
    int fa = 0;
    if (has) {
      a = sm[src * cw + lane];
      fa = sf[src * cw + lane];
    }
    __syncthreads();
    if (has) {
      seg_fold(a, sf[threadIdx.x] != 0, sm[threadIdx.x]);
      sm[threadIdx.x] = a;
      sf[threadIdx.x] = fa | sf[threadIdx.x];
    }
    __syncthreads();
  }
  if (col >= B) return;
  St st = C[t * B + col];
  const int src = dir > 0 ? rg - 1 : rg + 1;
  if (src >= 0 && src < RG) seg_fold(st, sf[src * cw + lane] != 0, sm[src * cw + lane]);
  const int64_t r0 = t * H + (int64_t)rg * RPT;
  auto step = [&](int i) {
    if (fr.seg[i]) st.zero();
    st.add(fr.v[i]);
    if (r0 + i < d.n) *elem<O32>(P, r0 + i, B, col) = Tr::out(st.value());
  };
  if (dir > 0) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) step(i);
  } else {
#pragma unroll
    for (int i = RPT - 1; i >= 0; --i) step(i);
  }
}

// Compact walk for narrow column blocks (8 <= cw <= 32): the scan kernels of
// the compact walk with cw-column blocks.  A workgroup covers TPW = WG / (4 cw)
// consecutive 64-row tiles of the compact tables (which may belong to
// different chains), 4 row groups of RPT = 16 rows per tile; a row group's
// marks are a 16-bit slice of its tile's mask.  The tile totals and the
// tile-local prefixes are those of the 64-column kernels, combined in the
// same order, so the carry kernel and the tables are shared.
template <typename Tin, typename Tout, bool O32>
__global__ __launch_bounds__(WG) void k_scan_reduce_cn(DevPoset d, int cw, int dir, const Tin* __restrict__ x,
                                                       int64_t ldx, int64_t B, int64_t ntiles,
                                                       typename ScanTraits<Tin, Tout>::St* __restrict__ A,
                                                       const uint64_t* __restrict__ tmask,
                                                       const int32_t* __restrict__ qoff, Tout* __restrict__ L) {
  using Tr = ScanTraits<Tin, Tout>;
  using St = typename Tr::St;
  using Tv = decltype(Tr::in(Tin()));
  __shared__ St sm[WG];
  const int RG = WG / cw, TPW = RG / 4;
  const int lane = threadIdx.x % cw, rg = threadIdx.x / cw;
  const int tq = rg >> 2, q = rg & 3;
  const int64_t t = (int64_t)blockIdx.x * TPW + tq;
  const bool tok = t < ntiles;
  const int64_t tc = tok ? t : ntiles - 1;
  const int2 tr = d.tiles[6][tc];  // 64-row tiles: {first row, end row of its chain}
  const int64_t r0 = tr.x + (int64_t)q * RPT, end = tr.y;
  const int64_t col = (int64_t)blockIdx.y * cw + lane;
  const int64_t colc = col < B ? col : 0;
  const uint64_t tm = tmask[tc];
  int32_t nodes[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) nodes[i] = node_at(d, min(r0 + i, end - 1));
  Tin raw[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) raw[i] = *elem<O32>(x, nodes[i], ldx, colc);
  Tv v[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) v[i] = (tok && r0 + i < end) ? Tr::in(raw[i]) : Tv(0);
  St st;
  st.zero();
#pragma unroll
  for (int i = 0; i < RPT; ++i) st.add(v[dir > 0 ? i : RPT - 1 - i]);
  sm[threadIdx.x] = st;
  __syncthreads();
  const int g0 = tq * 4;  // this tile's first row group
  if (q == 0 && tok && col < B) {
    St tot;
    tot.zero();
    for (int u = 0; u < 4; ++u) tot.combine(sm[(g0 + (dir > 0 ? u : 3 - u)) * cw + lane]);
    A[t * B + col] = tot;
  }
  const uint32_t m16 = tok ? (uint32_t)(tm >> (q * RPT)) & 0xffffu : 0u;
  if (m16 == 0 || col >= B) return;
  // the row groups of this tile before this one in scan order, then this one's rows
  St pre;
  pre.zero();
  if (dir > 0) {
    for (int u = 0; u < q; ++u) pre.combine(sm[(g0 + u) * cw + lane]);
  } else {
    for (int u = 3; u > q; --u) pre.combine(sm[(g0 + u) * cw + lane]);
  }
  const int32_t qo = qoff[tc];
  auto step = [&](int i) {
    pre.add(v[i]);
    if ((m16 >> i) & 1u) {
      const int b = q * RPT + i;  // the row's bit in its tile; slots run in row order
      const int slot = qo + __popcll(tm & ((uint64_t(1) << b) - 1));
      L[(int64_t)slot * B + col] = Tr::out(pre.value());
    }
  };
  if (dir > 0) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) step(i);
  } else {
#pragma unroll
    for (int i = RPT - 1; i >= 0; --i) step(i);
  }
}

// The last pass of the narrow compact walk: the scan inside each 64-row tile
// from its carry, fused with the combine: out[node(r)] = P[r] + S[snap_of_row[r]]
// (MODE 1), or the refinement residual res[node(r)] - (P[r] + S[...]) (MODE 2).
template <typename Tin, typename Tout, int MODE, typename Tres, bool O32>
__global__ __launch_bounds__(WG) void k_scan_apply_cn(DevPoset d, int cw, int dir, const Tin* __restrict__ x,
                                                      int64_t ldx, int64_t B, int64_t ntiles,
                                                      const typename ScanTraits<Tin, Tout>::St* __restrict__ C,
                                                      Tout* __restrict__ out, int64_t ldo,
                                                      const int32_t* __restrict__ snap_of_row,
                                                      const Tout* __restrict__ S, const Tres* __restrict__ res,
                                                      int64_t ldr) {
  using Tr = ScanTraits<Tin, Tout>;
  using St = typename Tr::St;
  using Tv = decltype(Tr::in(Tin()));
  using W = typename Wide<Tout>::W;
  __shared__ St sm[WG];
  const int RG = WG / cw, TPW = RG / 4;
  const int lane = threadIdx.x % cw, rg = threadIdx.x / cw;
  const int tq = rg >> 2, q = rg & 3;
  const int64_t t = (int64_t)blockIdx.x * TPW + tq;
  const bool tok = t < ntiles;
  const int64_t tc = tok ? t : ntiles - 1;
  const int2 tr = d.tiles[6][tc];
  const int64_t r0 = tr.x + (int64_t)q * RPT, end = tr.y;
  const int64_t col = (int64_t)blockIdx.y * cw + lane;
  const int64_t colc = col < B ? col : 0;
  int32_t nodes[RPT], sn[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    nodes[i] = node_at(d, min(r0 + i, end - 1));
    sn[i] = snap_of_row[min(r0 + i, end - 1)];
  }
  Tin raw[RPT];
  Tout sv[RPT];
  Tres rv[MODE == 2 ? RPT : 1];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    raw[i] = __builtin_nontemporal_load(elem<O32>(x, nodes[i], ldx, colc));
    sv[i] = *elem<O32>(S, sn[i], B, colc);
    if constexpr (MODE == 2) rv[i] = *elem<O32>(res, nodes[i], ldr, colc);
  }
  Tv v[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) v[i] = (tok && r0 + i < end) ? Tr::in(raw[i]) : Tv(0);
  St loc;
  loc.zero();
#pragma unroll
  for (int i = 0; i < RPT; ++i) loc.add(v[dir > 0 ? i : RPT - 1 - i]);
  sm[threadIdx.x] = loc;
  __syncthreads();
  if (!tok || col >= B) return;
  const int g0 = tq * 4;
  St pre;
  pre.zero();
  if (dir > 0) {
    for (int u = 0; u < q; ++u) pre.combine(sm[(g0 + u) * cw + lane]);
  } else {
    for (int u = 3; u > q; --u) pre.combine(sm[(g0 + u) * cw + lane]);
  }
  St st = C[t * B + col];
  st.combine(pre);
  auto step = [&](int i) {
    st.add(v[i]);
    if (r0 + i < end) {
      if constexpr (MODE == 2)
        *elem<O32>(out, nodes[i], ldo, col) = (Tout)((double)rv[i] - ((W)Tr::out(st.value()) + (W)sv[i]));
      else
        *elem<O32>(out, nodes[i], ldo, col) = (Tout)((W)Tr::out(st.value()) + (W)sv[i]);
    }
  };
  if (dir > 0) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) step(i);
  } else {
#pragma unroll
    for (int i = RPT - 1; i >= 0; --i) step(i);
  }
}

// Single-pass chain scan with a deterministic multi-level look-back.
//
// Workgroups take tiles (and column blocks) in scan-position-major order of
// their index, so a tile only waits for tiles of its chain held by workgroups
// of lower index.  Workgroups are dispatched in index order on each XCD, so
// the lowest unfinished workgroup is always resident and never waits for a
// later one: every wait ends.  (A single claim counter would serialise all
// workgroups on one device-scope atomic, about 20 ns each.)  Positions
// along a chain are read as base-16 numbers; the level-m group of a position is
// the run of 16^m positions sharing its digits above m.  Each tile publishes
// exactly one state: the total of the largest group it closes (its own total
// when its lowest digit is below 15; the total of its 16-tile group when it is
// the group's last tile, and so on up).  The carry of the tile at position p is
// the fold, in a fixed order, of the totals of the complete groups before it:
// at every level m, the d_m(p) earlier sibling groups (d_m = digit m of p).
// All waits of a tile are issued together, one lane per awaited flag, and the
// dependency depth is the number of levels, so no serial chain of waits runs
// along the scan.  The fold order depends on p alone, so results are
// bit-reproducible from run to run.
//
// Publication: states are stored with relaxed device-scope atomics, which are
// coherent across the per-XCD L2s without cache maintenance, and the publishing
// wave waits until those stores have completed (vmcnt 0) before it stores the
// flag.  A release fence would write back the whole L2, holding the tile
// outputs, once per tile; with no wait at all the flag may overtake the last
// quarter-wave line of the state.  Readers load states with relaxed
// device-scope atomics after their flag loads have returned.
//
// Waits are bounded (spin_limit polls).  A tile that gives up sums the missing
// groups straight from the input rows instead (slower, still correct, no longer
// bit-reproducible) and sets the error word so that other waits give up early.
constexpr int LB_LG = 4;
constexpr int LB_G = 1 << LB_LG;
constexpr int LB_LEVELS = 8;  // chain positions < 2^31

// Tile states travel as relaxed device-scope atomics, which are coherent
// across the per-XCD L2s without a cache write-back or invalidate.  A release
// fence would write back the whole L2 (the tile outputs are in it) once per
// tile; instead the publishing wave waits until its own state stores have
// completed (vmcnt reaches zero) before it stores the flag.  Without that wait
// the flag store may overtake the last quarter-wave line of the state.  The
// reader's loads are issued after its flag load has returned the flag.
template <typename St>
__device__ inline void st_put(St* p, const St& v) {
  static_assert(sizeof(St) % 8 == 0, "tile state is whole 64-bit words");
  uint64_t w[sizeof(St) / 8];
  __builtin_memcpy(w, &v, sizeof(St));
#pragma unroll
  for (int i = 0; i < (int)(sizeof(St) / 8); ++i)
    __hip_atomic_store(reinterpret_cast<uint64_t*>(p) + i, w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename St>
__device__ inline St st_get(const St* p) {
  uint64_t w[sizeof(St) / 8];
#pragma unroll
  for (int i = 0; i < (int)(sizeof(St) / 8); ++i)
    w[i] = __hip_atomic_load(reinterpret_cast<const uint64_t*>(p) + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  St v;
  __builtin_memcpy(&v, w, sizeof(St));
  return v;
}

// This wave's earlier vector-memory operations have completed; also a compiler
// barrier, so no memory access moves across it.
__device__ inline void wait_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

template <typename Tin, typename Tout, int CWT>
__global__ __launch_bounds__(WG) void k_scan_onepass(DevPoset d, int segi, int cw_rt, int dir,
                                                     const Tin* __restrict__ x, int64_t ldx, int64_t B,
                                                     int64_t ntiles, const int32_t* __restrict__ order,
                                                     typename ScanTraits<Tin, Tout>::St* __restrict__ Val,
                                                     int* __restrict__ flags, int* __restrict__ err,
                                                     int spin_limit, Tout* __restrict__ P) {
  using Tr = ScanTraits<Tin, Tout>;
  using St = typename Tr::St;
  using Tv = decltype(Tr::in(Tin()));
  const int cw = CWT ? CWT : cw_rt;
  __shared__ St sm[WG];
  __shared__ St carry_sh[64];
  const int64_t ncb = (B + cw - 1) / cw;
  const int64_t item = blockIdx.x;
  if (item >= ntiles * ncb) return;
  // row n of P stays zero: the walk reads it for "no element"
  if (item < ncb && threadIdx.x < cw && item * cw + threadIdx.x < B)
    P[(int64_t)d.n * B + item * cw + threadIdx.x] = Tout(0);
  const int64_t cb = item % ncb;
  const int t = order[item / ncb];
  const int32_t* so = d.segoff + (int64_t)segi * (d.nchains + 1);
  const int c = find_chain(so, d.nchains, t);
  const int RG = WG / cw;
  const int seg = RG * RPT;
  const int q = t - so[c];
  const int nq = so[c + 1] - so[c];
  const int pos = dir > 0 ? q : nq - 1 - q;
  const int64_t base = d.chain_off[c] + (int64_t)q * seg;
  const int64_t end = d.chain_off[c + 1];
  // with 64-wide column blocks the row group is the wavefront index: uniform
  const int lane = threadIdx.x % cw;
  const int rg = CWT == 64 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64)) : (int)(threadIdx.x / cw);
  const int64_t col = cb * cw + lane;
  const int64_t colc = col < B ? col : 0;
  const int64_t r0 = base + (int64_t)rg * RPT;

  // load the tile and scan each thread's rows
  int32_t nodes[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    nodes[i] = node_at(d, min(r0 + i, end - 1));
    if (CWT == 64) nodes[i] = __builtin_amdgcn_readfirstlane(nodes[i]);
  }
  Tin raw[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) raw[i] = x[(int64_t)nodes[i] * ldx + colc];
  Tv v[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) v[i] = (r0 + i < end) ? Tr::in(raw[i]) : Tv(0);
  St loc;
  loc.zero();
  if (dir > 0) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) loc.add(v[i]);
  } else {
#pragma unroll
    for (int i = RPT - 1; i >= 0; --i) loc.add(v[i]);
  }
  sm[threadIdx.x] = loc;
  __syncthreads();

  // wave 0 handles the look-back; its lanes with rg == 0 hold one column each
  if (threadIdx.x < 64) {
    const int wl = threadIdx.x;
    const bool own = rg == 0 && col < B;
    St tot;
    tot.zero();
    if (rg == 0) {
      if (dir > 0)
        for (int g = 0; g < RG; ++g) tot.combine(sm[g * cw + lane]);
      else
        for (int g = RG - 1; g >= 0; --g) tot.combine(sm[g * cw + lane]);
    }
    auto tile_at = [&](int64_t pp) { return dir > 0 ? so[c] + (int)pp : so[c + 1] - 1 - (int)pp; };
    auto digit = [&](int m) { return (int)(((int64_t)pos >> (LB_LG * m)) & (LB_G - 1)); };
    // sum of the tiles at positions [p0, p1), read from the input (fallback)
    auto direct = [&](int64_t p0, int64_t p1) {
      St acc;
      acc.zero();
      for (int64_t pp = p0; pp < p1; ++pp) {
        const int64_t rb = d.chain_off[c] + (int64_t)(tile_at(pp) - so[c]) * seg;
        const int64_t re = min(rb + seg, end);
        if (dir > 0)
          for (int64_t r = rb; r < re; ++r) acc.add(Tr::in(x[(int64_t)d.node_of_row[r] * ldx + colc]));
        else
          for (int64_t r = re - 1; r >= rb; --r) acc.add(Tr::in(x[(int64_t)d.node_of_row[r] * ldx + colc]));
      }
      return acc;
    };
    int lam = 0;  // number of trailing 15 digits: this tile closes its level-lam group
    while (lam < LB_LEVELS && digit(lam) == LB_G - 1) ++lam;
    const bool publish = pos != nq - 1;  // nobody reads the last tile of a chain
    const int64_t me = (int64_t)t * ncb + cb;
    auto put = [&](const St& v) {
      if (own) st_put(&Val[(int64_t)t * B + col], v);
      wait_vmem();
      if (wl == 0) __hip_atomic_store(&flags[me], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    if (lam == 0 && publish) put(tot);
    // Awaited groups, in fold order: the tail (levels lam-1 .. 0, 15 siblings
    // each) and then the head (levels LB_LEVELS-1 .. lam, digit(m) each).
    const int ntail = (LB_G - 1) * lam;
    int nhead = 0;
    for (int m = lam; m < LB_LEVELS; ++m) nhead += digit(m);
    // item j -> position of the last tile of that group, and its level m
    auto item = [&](int j, int& m) -> int64_t {
      int i;
      if (j < ntail) {
        m = lam - 1 - j / (LB_G - 1);
        i = j % (LB_G - 1);
      } else {
        j -= ntail;
        for (m = LB_LEVELS - 1; m > lam && j >= digit(m); --m) j -= digit(m);
        i = j;
      }
      const int64_t base = ((int64_t)pos >> (LB_LG * (m + 1))) << (LB_LG * (m + 1));
      return base + ((int64_t)(i + 1) << (LB_LG * m)) - 1;
    };
    // wait for items [j0, j1) (at most 64); returns the mask of items given up on
    auto await_items = [&](int j0, int j1) -> uint64_t {
      const int j = j0 + wl;
      bool ok = j >= j1;
      const int* fl = flags;
      if (!ok) {
        int m;
        fl = &flags[(int64_t)tile_at(item(j, m)) * ncb + cb];
      }
      for (int spin = 0;; ++spin) {
        if (!ok) ok = __hip_atomic_load(fl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= 1;
        if (__all(ok)) break;
        bool give_up = spin >= spin_limit;
        if ((spin & 255) == 255 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) give_up = true;
        if (__any(give_up)) {
          if (wl == 0 && spin >= spin_limit) atomicOr(err, 1);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      return __ballot(!ok);
    };
    // fold of items [j0, j1) in order; loads go out eight at a time
    auto fold = [&](int j0, int j1, uint64_t miss) {
      St acc;
      acc.zero();
      for (int j = j0; j < j1; j += 8) {
        St v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          v[u].zero();
          const int jj = j + u;
          if (jj < j1 && !((miss >> (jj - j0)) & 1) && own) {
            int m;
            v[u] = st_get(&Val[(int64_t)tile_at(item(jj, m)) * B + col]);
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int jj = j + u;
          if (jj >= j1) break;
          if ((miss >> (jj - j0)) & 1) {
            int m;
            const int64_t q = item(jj, m);
            acc.combine(direct(q + 1 - ((int64_t)1 << (LB_LG * m)), q + 1));
          } else {
            acc.combine(v[u]);
          }
        }
      }
      return acc;
    };
    St tail;
    tail.zero();
    for (int j0 = 0; j0 < ntail; j0 += 64) {
      const int j1 = min(ntail, j0 + 64);
      tail.combine(fold(j0, j1, await_items(j0, j1)));
    }
    if (lam > 0 && publish) {
      St closed = tail;
      closed.combine(tot);
      put(closed);
    }
    St carry;
    carry.zero();
    for (int j0 = ntail; j0 < ntail + nhead; j0 += 64) {
      const int j1 = min(ntail + nhead, j0 + 64);
      carry.combine(fold(j0, j1, await_items(j0, j1)));
    }
    carry.combine(tail);
    if (rg == 0) carry_sh[lane] = carry;
  }
  __syncthreads();
  if (col >= B) return;
  St st = carry_sh[lane];
  if (dir > 0) {
    for (int g = 0; g < rg; ++g) st.combine(sm[g * cw + lane]);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      st.add(v[i]);
      const int64_t r = r0 + i;
      if (r < end) P[r * B + col] = Tr::out(st.value());
    }
  } else {
    for (int g = RG - 1; g > rg; --g) st.combine(sm[g * cw + lane]);
#pragma unroll
    for (int i = RPT - 1; i >= 0; --i) {
      st.add(v[i]);
      const int64_t r = r0 + i;
      if (r < end) P[r * B + col] = Tr::out(st.value());
    }
  }
}

__global__ void k_fill_i32(int* p, int64_t cnt, int v) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i < cnt) p[i] = v;
}

// cnt 64-bit words set to v, two per thread (16-byte stores when p is 16-byte
// aligned).
__global__ void k_fill_i64x2(int64_t* __restrict__ p, int64_t cnt, int64_t v) {
  const int64_t i = ((int64_t)blockIdx.x * WG + threadIdx.x) * 2;
  if (i + 1 < cnt && (uintptr_t)p % 16 == 0) {
    reinterpret_cast<longlong2*>(p + i)[0] = make_longlong2(v, v);
  } else {
    if (i < cnt) p[i] = v;
    if (i + 1 < cnt) p[i + 1] = v;
  }
}

// ------------------------------------------------------------ gather-reduce

__device__ inline double fmax_(double a, double b) { return a > b ? a : b; }

// acc plus (SUB: minus) M[entry][col] for a row's k niv entries in chain
// order, one at a time, skipping -1 and `skip`: 32 entries load together,
// then their 32 rows together, instead of one entry and one dependent row at a
// time.  Skipped entries read row zr of M, which every producer of M keeps
// zero, so that no load is behind a branch (adding or subtracting that zero
// leaves acc unchanged).
template <typename TM, typename W, bool SUB = false>
__device__ inline W niv_sum(const int32_t* __restrict__ nr, int k, int64_t skip, int64_t zr,
                            const TM* __restrict__ M, int64_t B, int64_t col, W acc = W(0)) {
  for (int j0 = 0; j0 < k; j0 += 32) {
    int32_t t[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) t[u] = j0 + u < k ? nr[j0 + u] : -1;
    TM v[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) v[u] = M[(t[u] >= 0 && t[u] != skip ? (int64_t)t[u] : zr) * B + col];
#pragma unroll
    for (int u = 0; u < 32; ++u) acc = SUB ? acc - (W)v[u] : acc + (W)v[u];
  }
  return acc;
}

// The same over a sparse row: its finite entries er[e0 .. e1) (ascending
// chain order), 16 at a time.  The terms and their order are those of the
// dense row, so results agree bit for bit with niv_sum.
template <typename TM, typename W, bool SUB = false>
__device__ inline W csr_sum(const int32_t* __restrict__ er, int64_t e0, int64_t e1, int64_t skip, int64_t zr,
                            const TM* __restrict__ M, int64_t B, int64_t col, W acc = W(0)) {
  for (int64_t e = e0; e < e1; e += 16) {
    int32_t t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) t[u] = e + u < e1 ? er[e + u] : -1;
    TM v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = M[(t[u] >= 0 && t[u] != skip ? (int64_t)t[u] : zr) * B + col];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc = SUB ? acc - (W)v[u] : acc + (W)v[u];
  }
  return acc;
}

template <typename TP, typename Tout, typename Tres, bool RESID>
__global__ __launch_bounds__(WG) void k_gather(DevPoset d, const int32_t* __restrict__ nv, int cw,
                                               const TP* __restrict__ P, int64_t B, Tout* __restrict__ out,
                                               int64_t ldo, const Tres* __restrict__ res, int64_t ldr) {
  using W = typename Wide<TP>::W;
  const int RG = WG / cw;
  const int64_t r = (int64_t)blockIdx.x * RG + threadIdx.x / cw;
  const int64_t col = (int64_t)blockIdx.y * cw + threadIdx.x % cw;
  if (r >= d.n || col >= B) return;
  const int k = d.k;
  const W acc = niv_sum<TP, W>(nv + r * k, k, -1, d.n, P, B, col);  // row n of P is zero
  const int64_t node = d.node_of_row[r];
  if constexpr (RESID) {
    out[node * ldo + col] = (Tout)((double)res[node * ldr + col] - (double)acc);
  } else {
    out[node * ldo + col] = (Tout)acc;
  }
}

// The gather over sparse niv rows (CSR: ep[r] .. ep[r + 1] index er), one
// thread per (row, column), over all rows or the listed ones (rows != nullptr).
// The entries are vector loads even where a row is a whole wavefront: scalar
// loads of them made this kernel 13% slower.
template <typename TP, typename Tout, typename Tres, bool RESID>
__global__ __launch_bounds__(WG) void k_gather_csr(DevPoset d, const int64_t* __restrict__ ep,
                                                   const int32_t* __restrict__ er, const int32_t* __restrict__ rows,
                                                   int64_t nrows, int cw, const TP* __restrict__ P, int64_t B,
                                                   Tout* __restrict__ out, int64_t ldo, const Tres* __restrict__ res,
                                                   int64_t ldr) {
  using W = typename Wide<TP>::W;
  const int RG = WG / cw;
  const int64_t i = (int64_t)blockIdx.x * RG + threadIdx.x / cw;
  const int64_t col = (int64_t)blockIdx.y * cw + threadIdx.x % cw;
  if (i >= nrows || col >= B) return;
  const int64_t r = rows ? rows[i] : i;
  const W acc = csr_sum<TP, W>(er, ep[r], ep[r + 1], -1, d.n, P, B, col);  // row n of P is zero
  const int64_t node = d.node_of_row[r];
  if constexpr (RESID) {
    out[node * ldo + col] = (Tout)((double)res[node * ldr + col] - (double)acc);
  } else {
    out[node * ldo + col] = (Tout)acc;
  }
}

// Gather-reduce by walking chains (two kernels).  Along a chain the niv rows
// change little from one element to the next (x below y implies
// out(x) ⊆ out(y), Theorem 4): at n = 2^20, k = 64 a row differs from the one
// below in about one other-chain entry.  Preprocessing cuts every chain into
// runs of at most 128 rows and a bounded number of change events and encodes
// each run as the niv row of its first element plus the events of its later
// rows, {new row, old row, (row offset << 8) | chain}, own chain excluded
// (-1 = none).
//
// G1 keeps, for each run and right-hand side, acc = Σ_{j != own} P[niv_j(r)]
// in float64 (exact int64 wrap): a full gather for the first row, then
// acc += P[new] - P[old] per event, 16 (uniform form) or 8 (lane-split form)
// events with their gathers in flight together.  It stores acc as a snapshot
// after the first row and after every row with events: S[snap_off[s] + m].
// G2 is a streaming pass: out[node(r)] = P[r] + S[snap_of_row[r]] (the own
// chain contributes the row itself), or resid[node(r)] minus that for a
// refinement residual.  Snapshots are stored in the P type; for float32 this
// adds one rounding of |acc| <= (Z|f|)(x).
//
// Uniform form (k_walk_events, single poset, B >= 32, k <= 64): one wavefront
// per run, lanes = 64 columns; event fields are read with readlane, so all
// control flow is scalar.
//
// COMPACT: P is the compact Q of the gathered rows (slots), the first row's
// entries come from w.init and the events from w.evq; slot nslots is the zero
// row.
template <typename TP, bool OFF32, bool COMPACT>
__global__ __launch_bounds__(WG) void k_walk_events(DevPoset d, const int32_t* __restrict__ nv, WalkTables w,
                                                    const TP* __restrict__ P, int64_t B, TP* __restrict__ S) {
  using W = typename Wide<TP>::W;
  const int lane = threadIdx.x & 63;
  const int ncb = (int)((B + 63) >> 6);
  // Wave-uniform values go through readfirstlane so that they live in scalar
  // registers: every gather is then one load from a scalar base at a per-lane
  // offset.  Row n of P is a zero row: the tables name it for "no element",
  // so that every event adds P[new] - P[old] without a predicate.
  // Workgroups are dispatched round-robin over the 8 XCDs, each with its own
  // L2: XCD x takes a contiguous slice of the height-ordered runs, so that its
  // L2 holds one height band instead of every band at once (a bijection of
  // the block indices).
  const int nblk = (int)gridDim.x, q8 = nblk >> 3, r8 = nblk & 7;
  const int xcd = (int)(blockIdx.x & 7), slot = (int)(blockIdx.x >> 3);
  const int blk = xcd * q8 + min(xcd, r8) + slot;
  const int gw = __builtin_amdgcn_readfirstlane(blk * (WG / 64) + (int)(threadIdx.x >> 6));
  if ((int64_t)gw >= (int64_t)w.nruns * ncb) return;
  const int run = gw / ncb;
  const int col = (gw % ncb) * 64 + lane;
  const bool colok = col < B;
  const int colc = colok ? col : 0;
  const int r0 = __builtin_amdgcn_readfirstlane(w.runs[run].x);
  const int k = d.k;
  const int zr = COMPACT ? w.nslots : d.n;
  const int4* __restrict__ evs = COMPACT ? w.evq : w.ev;
  const int e0 = __builtin_amdgcn_readfirstlane(w.ev_off[run]);
  const int e1 = __builtin_amdgcn_readfirstlane(w.ev_off[run + 1]);
  // P[t][col]: with OFF32 (all of P within 2^31 bytes) one scalar 32-bit
  // multiply per row and a 32-bit lane offset from P's base
  const uint32_t rowb = (uint32_t)(B * sizeof(TP));
  const uint32_t lofs = (uint32_t)colc * (uint32_t)sizeof(TP);
  auto ld = [&](int t) -> TP {
    if (OFF32) return *(const TP*)((const char*)P + ((uint32_t)t * rowb + lofs));
    return (P + (int64_t)t * B)[colc];
  };

  // the first row's niv entries and the first batch of events load together
  const int cur = COMPACT ? (lane < k ? w.init[(int64_t)run * k + lane] : zr)
                          : (lane < k ? nv[(int64_t)r0 * k + lane] : -1);
  const int4 ev_first = lane < e1 - e0 ? evs[e0 + lane] : make_int4(zr, zr, -1, 0);
  // full gather of the first row, 32 loads in flight (64 cost more in occupancy
  // than they save); missing entries and the own chain read the zero row
  constexpr int PG = 32;
  W acc = W(0);
  for (int j0 = 0; j0 < k; j0 += PG) {
    TP v[PG];
#pragma unroll
    for (int u = 0; u < PG; ++u) {
      const int j = j0 + u;
      const int t = __builtin_amdgcn_readlane(cur, j & 63);
      v[u] = ld(COMPACT ? t : (j < k && t >= 0 && t != r0 ? t : zr));
    }
#pragma unroll
    for (int u = 0; u < PG; ++u) acc += (W)v[u];
  }
  int m = __builtin_amdgcn_readfirstlane(w.snap_off[run]);
  const int mlast = __builtin_amdgcn_readfirstlane(w.snap_off[run + 1]) - 1;  // the run's own snapshots only
  if (colok) (S + (int64_t)m * B)[col] = (TP)acc;

  constexpr int EG = 16;  // events per group, both gathers of each in flight
  for (int eb = e0; eb < e1; eb += 64) {
    const int ne = min(64, e1 - eb);
    const int4 evl = eb == e0 ? ev_first : (lane < ne ? evs[eb + lane] : make_int4(zr, zr, -1, 0));
    for (int g0 = 0; g0 < ne; g0 += EG) {
      TP vn[EG], vo[EG];
      int ue[EG + 1];  // row offset of each event (-1: none); the last entry looks one event ahead
#pragma unroll
      for (int q = 0; q < EG; ++q) {
        const int i = g0 + q;  // lanes >= ne hold the zero row and offset -1
        vn[q] = ld(__builtin_amdgcn_readlane(evl.x, i));
        vo[q] = ld(__builtin_amdgcn_readlane(evl.y, i));
        ue[q] = __builtin_amdgcn_readlane(evl.z, i) >> 8;
      }
      // the row offset of the event after this group (-1 at the end of the run)
      const int inext = g0 + EG;
      ue[EG] = inext < ne ? (__builtin_amdgcn_readlane(evl.z, inext) >> 8)
                          : (eb + 64 < e1 ? (__builtin_amdgcn_readfirstlane(evs[eb + 64].z) >> 8) : -1);
#pragma unroll
      for (int q = 0; q < EG; ++q) {
        acc += (W)vn[q] - (W)vo[q];
        if (ue[q] >= 0 && ue[q + 1] != ue[q]) {  // last event of its row: snapshot
          m = min(m + 1, mlast);
          if (colok) (S + (int64_t)m * B)[col] = (TP)acc;
        }
      }
    }
  }
}

// Lane-split form (any B <= 64, batches of posets, any k): a wavefront runs
// 64/cw runs side by side, cw lanes (columns) each; every lane follows its own
// run's events with per-lane predication.  The own-chain entry of the first
// row is the row itself, which identifies it without chain numbers.  As in the
// uniform form, XCD x takes a contiguous slice of the runs: for a batch, whose
// runs are poset after poset, each XCD's L2 then holds the P rows of the few
// posets it is working on instead of all of them.
// COMPACT (one poset, k <= 64, cw >= 8): P is the compact Q, as in the
// vector-lane form.
template <typename TP, bool COMPACT = false>
__global__ __launch_bounds__(WG) void k_walk_events_split(DevPoset d, const int32_t* __restrict__ nv, WalkTables w,
                                                          int cw, const TP* __restrict__ P, int64_t B,
                                                          TP* __restrict__ S) {
  using W = typename Wide<TP>::W;
  if (COMPACT && cw < 8) return;  // not launched: the compact form needs cw >= 8
  const int lane = threadIdx.x & 63;
  const int nsub = 64 / cw;
  const int nblk = (int)gridDim.x, q8 = nblk >> 3, r8 = nblk & 7;
  const int xcd = (int)(blockIdx.x & 7), slot = (int)(blockIdx.x >> 3);
  const int blk = xcd * q8 + min(xcd, r8) + slot;
  const int64_t run = ((int64_t)blk * (WG / 64) + (threadIdx.x >> 6)) * nsub + lane / cw;
  const int col = lane % cw;
  const bool active = run < w.nruns;
  const bool colok = active && col < B;
  const int64_t colc = col < B ? col : 0;
  const int64_t runc = active ? run : 0;
  const int r0 = w.runs[runc].x;
  int k;
  const int32_t* nr;
  if (COMPACT) {
    k = d.k;
    nr = w.init + runc * k;
  } else if (d.poset_of_row) {
    const int p = d.poset_of_row[r0];
    k = d.k_of_poset[p];
    nr = nv + d.niv_off[p] + (int64_t)(r0 - d.row_off[p]) * k;
  } else {
    k = d.k;
    nr = nv + (int64_t)r0 * k;
  }
  const int zrow = COMPACT ? w.nslots : r0;  // a row to load for masked entries
  const int klast = k - 1;  // entries load from nr[min(j, klast)] (k >= 1) and are masked after
  if (!active) k = 0;
  int kmax = k;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) kmax = max(kmax, __shfl_xor(kmax, off));

  W acc = W(0);
  if (cw >= 8) {
    // the first row's entries 16 at a time, two per lane of the run's group,
    // shared by lane shuffles; the next 16 load with this group's gathers
    const int sub = lane % cw, base = lane - sub, s8 = sub & 7;
    auto ent = [&](int j) {  // OR-ing the mask keeps the load unconditional (no branch)
      return nr[min(j, klast)] | (j < k ? 0 : -1);
    };
    int ta = ent(s8), tb = ent(8 + s8);
    for (int j0 = 0; j0 < kmax; j0 += 16) {
      const int na = ent(j0 + 16 + s8), nb = ent(j0 + 24 + s8);
      TP v[16];
      bool ok[16];
      int t[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) t[u] = __shfl(u < 8 ? ta : tb, base + (u & 7));
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        ok[u] = t[u] >= 0 && (COMPACT || t[u] != r0);
        v[u] = P[(int64_t)(ok[u] ? t[u] : zrow) * B + colc];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (ok[u]) acc += (W)v[u];
      ta = na;
      tb = nb;
    }
  } else {
    for (int j0 = 0; j0 < kmax; j0 += 16) {
      TP v[16];
      bool ok[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int j = j0 + u;
        const int t = j < k ? nr[j] : -1;
        ok[u] = t >= 0 && t != r0;
        v[u] = P[(int64_t)(ok[u] ? t : r0) * B + colc];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (ok[u]) acc += (W)v[u];
    }
  }
  int64_t m = w.snap_off[runc];
  const int64_t mlast = w.snap_off[runc + 1] - 1;
  if (colok) S[m * B + col] = (TP)acc;

  const int e0 = w.ev_off[runc];
  const int ne = active ? w.ev_off[runc + 1] - e0 : 0;
  int nemax = ne;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) nemax = max(nemax, __shfl_xor(nemax, off));
  if (cw >= 8) {
    // Groups of 16 events: lane j of the run's cw lanes holds records j & 7 and
    // 8 + (j & 7), the fields go round the group by lane shuffles, and the next
    // group's records load behind this group's 32 gathers, so that their wait
    // overlaps this group's sums.  A row's snapshot is stored when the first
    // event of a later row comes (or after the last event), which needs nothing
    // of the next group.  Record indices clamp to the run's end: the tables
    // keep one padding record after the last run.
    const int sub = lane % cw, base = lane - sub, s8 = sub & 7;
    const int4* __restrict__ evs = COMPACT ? w.evq : w.ev;
    auto rec = [&](int i) {  // OR-ing the mask keeps the load unconditional (no branch)
      const int4 r = evs[e0 + min(i, ne)];
      const int no = i < ne ? 0 : -1;
      return make_int4(r.x | no, r.y | no, r.z | no, 0);
    };
    int4 ra = rec(s8), rb = rec(8 + s8);
    int uprev = -1;  // row offset of the last event applied (-1: none yet)
    for (int g0 = 0; g0 < nemax; g0 += 16) {
      TP vn[16], vo[16];
      bool okn[16], oko[16];
      int ue[16], ex[16], ey[16];
      // all shuffles first (one wait for the lot), then all gathers
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int4& r = q < 8 ? ra : rb;
        ex[q] = __shfl(r.x, base + (q & 7));
        ey[q] = __shfl(r.y, base + (q & 7));
        ue[q] = __shfl(r.z, base + (q & 7)) >> 8;  // -1: no event
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        okn[q] = ex[q] >= 0;
        oko[q] = ey[q] >= 0;
        vn[q] = P[(int64_t)(okn[q] ? ex[q] : zrow) * B + colc];
        vo[q] = P[(int64_t)(oko[q] ? ey[q] : zrow) * B + colc];
      }
      ra = rec(g0 + 16 + s8);
      rb = rec(g0 + 24 + s8);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        if (ue[q] >= 0) {
          if (uprev >= 0 && ue[q] != uprev) {  // row uprev is complete
            m = min(m + 1, mlast);
            if (colok) S[m * B + col] = (TP)acc;
          }
          if (okn[q]) acc += (W)vn[q];
          if (oko[q]) acc -= (W)vo[q];
          uprev = ue[q];
        }
      }
    }
    if (uprev >= 0) {
      m = min(m + 1, mlast);
      if (colok) S[m * B + col] = (TP)acc;
    }
    return;
  }
  for (int g0 = 0; g0 < nemax; g0 += 8) {
    TP vn[8], vo[8];
    bool okn[8], oko[8];
    int ue[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const int i = g0 + q;
      ue[q] = i < ne ? (w.ev[e0 + i].z >> 8) : -1;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = g0 + q;
      const bool has = i < ne;
      const int4 e = has ? w.ev[e0 + i] : make_int4(-1, -1, 0, 0);
      okn[q] = e.x >= 0;
      oko[q] = e.y >= 0;
      vn[q] = P[(int64_t)(okn[q] ? e.x : r0) * B + colc];
      vo[q] = P[(int64_t)(oko[q] ? e.y : r0) * B + colc];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (ue[q] >= 0) {
        if (okn[q]) acc += (W)vn[q];
        if (oko[q]) acc -= (W)vo[q];
        if (ue[q + 1] != ue[q]) {
          m = min(m + 1, mlast);
          if (colok) S[m * B + col] = (TP)acc;
        }
      }
    }
  }
}

// Vector-lane form of the lane-split walk (B a multiple of V = 16 / sizeof(TP)):
// a lane carries V consecutive columns, so each gathered row is one 16-byte
// load and a wavefront gathers 64 / L rows per load instruction, L = cw / V
// lanes per run (2 <= L <= 16), instead of 64 / cw.  The vector memory unit
// of a compute unit spends its time per row touched, so narrow blocks gather
// several times faster this way.  Events and first-row entries are shared by
// the run's L lanes as in the lane-split form; EG events per group.
//
// COMPACT (one poset, k <= 64): P is the compact Q of the gathered rows; the
// first row's entries come from w.init and the events from w.evq, as slots
// (slot nslots, a zero row, for the own chain and "no element").
template <typename TP, int L, int EG, bool COMPACT = false>
__global__ __launch_bounds__(WG) void k_walk_events_vec(DevPoset d, const int32_t* __restrict__ nv, WalkTables w,
                                                        const TP* __restrict__ P, int64_t B, TP* __restrict__ S) {
  using W = typename Wide<TP>::W;
  constexpr int V = 16 / sizeof(TP);
  using VT = TP __attribute__((ext_vector_type(V)));
  static_assert(L >= 2 && L <= 16 && EG % L == 0 && 16 % L == 0, "lanes per run");
  constexpr int NSUB = 64 / L;  // runs per wavefront
  const int lane = threadIdx.x & 63;
  const int nblk = (int)gridDim.x, q8 = nblk >> 3, r8 = nblk & 7;
  const int xcd = (int)(blockIdx.x & 7), slot = (int)(blockIdx.x >> 3);
  const int blk = xcd * q8 + min(xcd, r8) + slot;
  const int64_t run = ((int64_t)blk * (WG / 64) + (threadIdx.x >> 6)) * NSUB + lane / L;
  const int sub = lane % L, base = lane - sub;
  const int64_t col = (int64_t)sub * V;  // B % V == 0: the lane's V columns are all in or all out
  const bool active = run < w.nruns;
  const bool colok = active && col < B;
  const int64_t colc = col < B ? col : 0;
  const int64_t runc = active ? run : 0;
  const int r0 = w.runs[runc].x;
  int k;
  const int32_t* nr;
  if (COMPACT) {
    k = d.k;
    nr = w.init + runc * k;
  } else if (d.poset_of_row) {
    const int p = d.poset_of_row[r0];
    k = d.k_of_poset[p];
    nr = nv + d.niv_off[p] + (int64_t)(r0 - d.row_off[p]) * k;
  } else {
    k = d.k;
    nr = nv + (int64_t)r0 * k;
  }
  const int4* __restrict__ evs = COMPACT ? w.evq : w.ev;
  const int klast = k - 1;
  if (!active) k = 0;
  int kmax = k;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) kmax = max(kmax, __shfl_xor(kmax, off));
  auto row = [&](int t) { return *(const VT*)(P + (int64_t)t * B + colc); };

  W acc[V];
#pragma unroll
  for (int v = 0; v < V; ++v) acc[v] = W(0);
  // first row: 16 entries at a time, 16 / L per lane, shared by shuffles (the
  // mask is OR-ed in so that the loads stay unconditional)
  for (int j0 = 0; j0 < kmax; j0 += 16) {
    int e[16 / L];
#pragma unroll
    for (int i = 0; i < 16 / L; ++i) {
      const int j = j0 + sub + L * i;
      e[i] = nr[min(j, klast)] | (j < k ? 0 : -1);
    }
    int t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) t[u] = __shfl(e[u / L], base + u % L);
    __builtin_amdgcn_sched_barrier(0);
    VT vv[16];
    bool ok[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      // compact slots name the zero row for the own chain; masked entries are -1
      ok[u] = t[u] >= 0 && (COMPACT || t[u] != r0);
      vv[u] = row(ok[u] ? t[u] : (COMPACT ? w.nslots : r0));
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (ok[u])
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] += (W)vv[u][v];
  }
  int64_t m = w.snap_off[runc];
  const int64_t mlast = w.snap_off[runc + 1] - 1;
  auto snap = [&]() {
    VT o;
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = (TP)acc[v];
    if (colok) *(VT*)(S + m * B + col) = o;
  };
  snap();

  const int e0 = w.ev_off[runc];
  const int ne = active ? w.ev_off[runc + 1] - e0 : 0;
  int nemax = ne;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) nemax = max(nemax, __shfl_xor(nemax, off));
  // record i of this run (clamped to the padding record after the last run)
  auto rec = [&](int i) {
    const int4 r = evs[e0 + min(i, ne)];
    const int no = i < ne ? 0 : -1;
    return make_int4(r.x | no, r.y | no, r.z | no, 0);
  };
  constexpr int RL = EG / L;  // records per lane and group
  int4 ra[RL];
#pragma unroll
  for (int i = 0; i < RL; ++i) ra[i] = rec(sub + L * i);
  int uprev = -1;  // row offset of the last event applied (-1: none yet)
  for (int g0 = 0; g0 < nemax; g0 += EG) {
    int ex[EG], ey[EG], ue[EG];
#pragma unroll
    for (int q = 0; q < EG; ++q) {
      ex[q] = __shfl(ra[q / L].x, base + q % L);
      ey[q] = __shfl(ra[q / L].y, base + q % L);
      ue[q] = __shfl(ra[q / L].z, base + q % L) >> 8;  // -1: no event
    }
    __builtin_amdgcn_sched_barrier(0);
    VT vn[EG], vo[EG];
    bool okn[EG], oko[EG];
#pragma unroll
    for (int q = 0; q < EG; ++q) {
      okn[q] = ex[q] >= 0;
      oko[q] = ey[q] >= 0;
      vn[q] = row(okn[q] ? ex[q] : (COMPACT ? w.nslots : r0));
      vo[q] = row(oko[q] ? ey[q] : (COMPACT ? w.nslots : r0));
    }
#pragma unroll
    for (int i = 0; i < RL; ++i) ra[i] = rec(g0 + EG + sub + L * i);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < EG; ++q) {
      if (ue[q] >= 0) {
        if (uprev >= 0 && ue[q] != uprev) {  // row uprev is complete
          m = min(m + 1, mlast);
          snap();
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
          if (okn[q]) acc[v] += (W)vn[q][v];
          if (oko[q]) acc[v] -= (W)vo[q][v];
        }
        uprev = ue[q];
      }
    }
  }
  if (uprev >= 0) {
    m = min(m + 1, mlast);
    snap();
  }
}

// UNI: cw == 64, so each wavefront owns whole rows and row quantities are
// wave-uniform (kept in scalar registers, loads from scalar row bases).
// P is read here for the last time and g is written once: both streams are
// non-temporal, so that they do not evict f and P's gathered rows from the
// caches (f stays in the 256 MB MALL between its two reads by the scan).
template <typename TP, typename Tres, bool RESID, bool UNI, bool O32 = false>
__global__ __launch_bounds__(WG) void k_walk_combine(DevPoset d, const int32_t* __restrict__ snap_of_row, int cw_rt,
                                                     const TP* __restrict__ P, const TP* __restrict__ S, int64_t B,
                                                     TP* __restrict__ out, int64_t ldo, const Tres* __restrict__ res,
                                                     int64_t ldr) {
  using W = typename Wide<TP>::W;
  constexpr int RPC = COMBINE_ROWS;
  const int cw = UNI ? 64 : cw_rt;
  auto uni = [](int v) { return UNI ? __builtin_amdgcn_readfirstlane(v) : v; };
  const int RG = WG / cw;
  // row of step i: UNI, a wavefront's RPC consecutive rows; narrow tiles, the
  // block's row groups side by side at every step (RG consecutive rows), so
  // that each load of P covers whole lines
  const int g = (int)(threadIdx.x / cw);
  const int rb = UNI ? uni((int)((blockIdx.x * RG + g) * RPC)) : (int)(blockIdx.x * RG * RPC) + g;
  const int rs = UNI ? 1 : RG;
  const int col = (int)blockIdx.y * cw + (int)(threadIdx.x % cw);
  if (rb >= d.n) return;
  const int colc = col < B ? col : 0;
  int32_t nd[RPC], sm[RPC];
#pragma unroll
  for (int i = 0; i < RPC; ++i) {
    const int r = min(rb + i * rs, d.n - 1);
    nd[i] = uni(node_at(d, r));
    sm[i] = uni(snap_of_row[r]);
  }
  TP pv[RPC], sv[RPC];
  Tres rv[RESID ? RPC : 1];
#pragma unroll
  for (int i = 0; i < RPC; ++i) {
    const int r = min(rb + i * rs, d.n - 1);
    pv[i] = __builtin_nontemporal_load(elem<O32>(P, r, B, colc));
    sv[i] = *elem<O32>(S, sm[i], B, colc);
    if constexpr (RESID) rv[i] = (res + (int64_t)nd[i] * ldr)[colc];
  }
  if (col >= B) return;
#pragma unroll
  for (int i = 0; i < RPC; ++i) {
    if (rb + i * rs < d.n) {
      if constexpr (RESID)
        (out + (int64_t)nd[i] * ldo)[col] = (TP)((double)rv[i] - ((W)pv[i] + (W)sv[i]));
      else if (UNI)
        __builtin_nontemporal_store((TP)((W)pv[i] + (W)sv[i]), &(out + (int64_t)nd[i] * ldo)[col]);
      else
        *elem<O32>(out, nd[i], ldo, col) = (TP)((W)pv[i] + (W)sv[i]);
    }
  }
}

// The vector-lane walk takes B a multiple of 16 / sizeof(TP) with 2 to 16 lanes
// per run, and enough runs for 2048 wavefronts (it holds twice the registers of
// the lane-split form, so fewer waves are resident; with few runs, as for one
// poset of 2^20 elements at B = 8, the lane-split form is faster).
// POSETX_WALK_VEC=0 / 1 (read on every call) never / always takes it.
template <typename TP>
bool walk_vec_ok(int cw, int64_t B, int64_t nruns) {
  constexpr int V = 16 / sizeof(TP);
  const int L = cw / V;
  if (B % V != 0 || L < 2 || L > 16) return false;
  const char* e = std::getenv("POSETX_WALK_VEC");
  if (e && e[0] == '0') return false;
  if (e && e[0] == '1') return true;
  return nruns / (64 / L) >= 2048;
}

template <typename TP>
hipError_t walk_typed(const DevPoset& d, const int32_t* nv, const WalkTables& w, const void* P, int64_t B, void* out,
                      int64_t ldo, ElemType tres, const void* resid, int64_t ldr, void* snaps, LaunchHook* hook,
                      hipStream_t s) {
  const bool uniform = !d.poset_of_row && d.k <= 64 && B >= 32;
  int cw = col_width(B);
  if (w.cw > cw && w.cw <= 64 && (w.cw & (w.cw - 1)) == 0) cw = w.cw;
  if (hook) hook->before(0, s);
  if (uniform) {
    const int64_t waves = (int64_t)w.nruns * ((B + 63) / 64);
    const dim3 g((unsigned)((waves + (WG / 64) - 1) / (WG / 64)));
    if (((int64_t)d.n + 1) * B * (int64_t)sizeof(TP) < ((int64_t)1 << 31))
      hipLaunchKernelGGL((k_walk_events<TP, true, false>), g, dim3(WG), 0, s, d, nv, w, (const TP*)P, B,
                         (TP*)snaps);
    else
      hipLaunchKernelGGL((k_walk_events<TP, false, false>), g, dim3(WG), 0, s, d, nv, w, (const TP*)P, B,
                         (TP*)snaps);
  } else if (walk_vec_ok<TP>(cw, B, w.nruns)) {
    constexpr int V = 16 / sizeof(TP);
    const int L = cw / V;
    const int64_t waves = (w.nruns + (64 / L) - 1) / (64 / L);
    const dim3 g((unsigned)((waves + (WG / 64) - 1) / (WG / 64)));
    const TP* p = (const TP*)P;
    TP* sn = (TP*)snaps;
    if (L == 2) hipLaunchKernelGGL((k_walk_events_vec<TP, 2, 16>), g, dim3(WG), 0, s, d, nv, w, p, B, sn);
    else if (L == 4) hipLaunchKernelGGL((k_walk_events_vec<TP, 4, 16>), g, dim3(WG), 0, s, d, nv, w, p, B, sn);
    else if (L == 8) hipLaunchKernelGGL((k_walk_events_vec<TP, 8, 16>), g, dim3(WG), 0, s, d, nv, w, p, B, sn);
    else hipLaunchKernelGGL((k_walk_events_vec<TP, 16, 16>), g, dim3(WG), 0, s, d, nv, w, p, B, sn);
  } else {
    const int64_t waves = (w.nruns + (64 / cw) - 1) / (64 / cw);
    hipLaunchKernelGGL((k_walk_events_split<TP>), dim3((unsigned)((waves + (WG / 64) - 1) / (WG / 64))), dim3(WG),
                       0, s, d, nv, w, cw, (const TP*)P, B, (TP*)snaps);
  }
  if (hook) hook->after(0, s);
  if (hook) hook->before(1, s);
  const int ccw = uniform ? 64 : cw;
  const int64_t rows_per_block = (WG / ccw) * COMBINE_ROWS;
  const dim3 gc((unsigned)((d.n + rows_per_block - 1) / rows_per_block), (unsigned)((B + ccw - 1) / ccw));
  if (ccw == 64) {
    if (resid && tres == E_F32)
      hipLaunchKernelGGL((k_walk_combine<TP, float, true, true>), gc, dim3(WG), 0, s, d, w.snap_of_row, ccw,
                         (const TP*)P, (const TP*)snaps, B, (TP*)out, ldo, (const float*)resid, ldr);
    else if (resid)
      hipLaunchKernelGGL((k_walk_combine<TP, double, true, true>), gc, dim3(WG), 0, s, d, w.snap_of_row, ccw,
                         (const TP*)P, (const TP*)snaps, B, (TP*)out, ldo, (const double*)resid, ldr);
    else
      hipLaunchKernelGGL((k_walk_combine<TP, TP, false, true>), gc, dim3(WG), 0, s, d, w.snap_of_row, ccw,
                         (const TP*)P, (const TP*)snaps, B, (TP*)out, ldo, (const TP*)nullptr, 0);
  } else {
    if (resid && tres == E_F32)
      hipLaunchKernelGGL((k_walk_combine<TP, float, true, false>), gc, dim3(WG), 0, s, d, w.snap_of_row, ccw,
                         (const TP*)P, (const TP*)snaps, B, (TP*)out, ldo, (const float*)resid, ldr);
    else if (resid)
      hipLaunchKernelGGL((k_walk_combine<TP, double, true, false>), gc, dim3(WG), 0, s, d, w.snap_of_row, ccw,
                         (const TP*)P, (const TP*)snaps, B, (TP*)out, ldo, (const double*)resid, ldr);
    else if (fits32(((int64_t)d.n + 1) * B * (int64_t)sizeof(TP)) && fits32((int64_t)w.nsnap * B * (int64_t)sizeof(TP)) &&
             fits32((int64_t)d.n * ldo * (int64_t)sizeof(TP)))
      hipLaunchKernelGGL((k_walk_combine<TP, TP, false, false, true>), gc, dim3(WG), 0, s, d, w.snap_of_row, ccw,
                         (const TP*)P, (const TP*)snaps, B, (TP*)out, ldo, (const TP*)nullptr, 0);
    else
      hipLaunchKernelGGL((k_walk_combine<TP, TP, false, false>), gc, dim3(WG), 0, s, d, w.snap_of_row, ccw,
                         (const TP*)P, (const TP*)snaps, B, (TP*)out, ldo, (const TP*)nullptr, 0);
  }
  if (hook) hook->after(1, s);
  return hipGetLastError();
}

// Batched gather over many posets of different width: row r belongs to
// poset p = poset_of_row[r] whose niv block (k_p entries per row, global row
// ids) starts at niv_off[p].
template <typename TP, typename Tout>
__global__ __launch_bounds__(WG) void k_gather_batched(DevPoset d, const int32_t* __restrict__ nv, int cw,
                                                       const TP* __restrict__ P, int64_t B,
                                                       Tout* __restrict__ out, int64_t ldo) {
  using W = typename Wide<TP>::W;
  const int RG = WG / cw;
  const int64_t r = (int64_t)blockIdx.x * RG + threadIdx.x / cw;
  const int64_t col = (int64_t)blockIdx.y * cw + threadIdx.x % cw;
  if (r >= d.n || col >= B) return;
  const int p = d.poset_of_row[r];
  const int k = d.k_of_poset[p];
  const W acc = niv_sum<TP, W>(nv + d.niv_off[p] + (r - d.row_off[p]) * k, k, -1, d.n, P, B, col);
  out[(int64_t)d.node_of_row[r] * ldo + col] = (Tout)acc;
}

// ------------------------------------------------------------- U-solve level
template <typename Tin, typename TY>
__global__ __launch_bounds__(WG) void k_usolve(DevPoset d, const int32_t* __restrict__ nv,
                                               const int32_t* __restrict__ rows, int64_t cnt, int cw,
                                               const Tin* __restrict__ g, int64_t ldg, TY* __restrict__ Y,
                                               int64_t B) {
  using W = typename Wide<TY>::W;
  const int RG = WG / cw;
  const int64_t i = (int64_t)blockIdx.x * RG + threadIdx.x / cw;
  const int64_t col = (int64_t)blockIdx.y * cw + threadIdx.x % cw;
  if (i >= cnt || col >= B) return;
  const int64_t r = rows[i];
  const int64_t node = d.node_of_row[r];
  const W acc = niv_sum<TY, W, true>(nv + r * d.k, d.k, r, d.n, Y, B, col, (W)g[node * ldg + col]);
  Y[r * B + col] = (TY)acc;
}

// Long sparse rows of a level are split into chunks of consecutive entries:
// item {row, first entry, end entry, w} gets part[w] = Σ Y[entry] over
// its chunk (own row skipped), one item per row group; then each long row
// {row, first item, items, 0} takes g minus its chunks' sums in chunk order.
// A row's result depends only on its chunking, which the host fixes.
// (SKIP_OWN: the solve, which leaves the row's own entry out; the zeta gather
// keeps it.)
//
// The host may order the items by the row of their first entry, so that
// chunks taken together gather from the same chains near the same heights;
// item.w is the chunk's place in its row's run of chunk sums.  Workgroups are
// dispatched round-robin over the 8 XCDs; a bijection of the block indices
// gives each XCD a contiguous slice of the ordered items, so that its L2 sees
// one band of P.
template <typename TY, bool SKIP_OWN>
__global__ __launch_bounds__(WG) void k_csr_part(DevPoset d, const int4* __restrict__ items, int64_t cnt, int cw,
                                                 const int32_t* __restrict__ er, const TY* __restrict__ Y, int64_t B,
                                                 typename Wide<TY>::W* __restrict__ part) {
  using W = typename Wide<TY>::W;
  const int RG = WG / cw;
  const int64_t nblk = gridDim.x, q8 = nblk >> 3, r8 = nblk & 7;
  const int64_t xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int64_t blk = xcd * q8 + min(xcd, r8) + slot;
  const int64_t i = blk * RG + threadIdx.x / cw;
  const int64_t col = (int64_t)blockIdx.y * cw + threadIdx.x % cw;
  if (i >= cnt || col >= B) return;
  const int4 it = items[i];
  part[(int64_t)it.w * B + col] = csr_sum<TY, W>(er, it.y, it.z, SKIP_OWN ? it.x : -1, d.n, Y, B, col);
}

// The zeta gather's long rows: out[node(row)] = Σ of the chunk sums in order
// (or resid minus that for a refinement residual).
template <typename TP, typename Tout, typename Tres, bool RESID>
__global__ __launch_bounds__(WG) void k_gather_csr_fin(DevPoset d, const int4* __restrict__ longs, int64_t cnt,
                                                       int cw, const typename Wide<TP>::W* __restrict__ part,
                                                       int64_t B, Tout* __restrict__ out, int64_t ldo,
                                                       const Tres* __restrict__ res, int64_t ldr) {
  using W = typename Wide<TP>::W;
  const int RG = WG / cw;
  const int64_t i = (int64_t)blockIdx.x * RG + threadIdx.x / cw;
  const int64_t col = (int64_t)blockIdx.y * cw + threadIdx.x % cw;
  if (i >= cnt || col >= B) return;
  const int4 lr = longs[i];
  W acc = W(0);
  for (int c = 0; c < lr.z; ++c) acc += part[(int64_t)(lr.y + c) * B + col];
  const int64_t node = d.node_of_row[lr.x];
  if constexpr (RESID) {
    out[node * ldo + col] = (Tout)((double)res[node * ldr + col] - (double)acc);
  } else {
    out[node * ldo + col] = (Tout)acc;
  }
}

template <typename Tin, typename TY>
__global__ __launch_bounds__(WG) void k_usolve_csr_fin(DevPoset d, const int4* __restrict__ longs, int64_t cnt,
                                                       int cw, const Tin* __restrict__ g, int64_t ldg,
                                                       const typename Wide<TY>::W* __restrict__ part,
                                                       TY* __restrict__ Y, int64_t B) {
  using W = typename Wide<TY>::W;
  const int RG = WG / cw;
  const int64_t i = (int64_t)blockIdx.x * RG + threadIdx.x / cw;
  const int64_t col = (int64_t)blockIdx.y * cw + threadIdx.x % cw;
  if (i >= cnt || col >= B) return;
  const int4 lr = longs[i];
  W acc = (W)g[(int64_t)d.node_of_row[lr.x] * ldg + col];
  for (int c = 0; c < lr.z; ++c) acc -= part[(int64_t)(lr.y + c) * B + col];
  Y[(int64_t)lr.x * B + col] = (TY)acc;
}

// The same over sparse niv rows (CSR ep / er).
template <typename Tin, typename TY>
__global__ __launch_bounds__(WG) void k_usolve_csr(DevPoset d, const int64_t* __restrict__ ep,
                                                   const int32_t* __restrict__ er, const int32_t* __restrict__ rows,
                                                   int64_t cnt, int cw, const Tin* __restrict__ g, int64_t ldg,
                                                   TY* __restrict__ Y, int64_t B) {
  using W = typename Wide<TY>::W;
  const int RG = WG / cw;
  const int64_t i = (int64_t)blockIdx.x * RG + threadIdx.x / cw;
  const int64_t col = (int64_t)blockIdx.y * cw + threadIdx.x % cw;
  if (i >= cnt || col >= B) return;
  const int64_t r = rows[i];
  const int64_t node = d.node_of_row[r];
  const W acc = csr_sum<TY, W, true>(er, ep[r], ep[r + 1], r, d.n, Y, B, col, (W)g[node * ldg + col]);
  Y[r * B + col] = (TY)acc;
}

// With 64-wide column blocks each wavefront solves one row: the row and its
// niv entries are wave-uniform (scalar registers), its k - 1 dependencies go
// out all at once from scalar row bases, and the own and missing entries read
// row n of Y, which launch_usolve_begin sets to zero.  Same subtraction order
// as k_usolve (g minus one entry at a time, in chain order; a zero row
// subtracts nothing), so results are identical.
//
// With level-ordered copies of the niv rows and node ids (lnv, lnode; the
// level starts at position i0), a row's entries, node and index load together
// instead of after the row index: one dependent memory round trip less per
// level.
template <typename Tin, typename TY>
__global__ __launch_bounds__(WG) void k_usolve_uni(DevPoset d, const int32_t* __restrict__ nv,
                                                   const int32_t* __restrict__ rows, int cnt,
                                                   const Tin* __restrict__ g, int64_t ldg, TY* __restrict__ Y,
                                                   int64_t B, const int32_t* __restrict__ lnv,
                                                   const int32_t* __restrict__ lnode, int64_t i0) {
  using W = typename Wide<TY>::W;
  const int lane = threadIdx.x & 63;
  const int i = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (WG / 64) + (threadIdx.x >> 6)));
  if (i >= cnt) return;
  const int col = (int)blockIdx.y * 64 + lane;
  const bool colok = col < B;
  const int colc = colok ? col : 0;
  const int k = d.k, zr = d.n;
  const int r = __builtin_amdgcn_readfirstlane(rows[i]);
  int node, cur;
  if (lnv) {
    node = __builtin_amdgcn_readfirstlane(lnode[i0 + i]);
    cur = lane < k ? lnv[(i0 + i) * k + lane] : -1;
  } else {
    node = __builtin_amdgcn_readfirstlane(d.node_of_row[r]);
    cur = lane < k ? nv[(int64_t)r * k + lane] : -1;
  }
  W acc = (W)(g + (int64_t)node * ldg)[colc];
  // levels hold few rows, so occupancy matters little: all k loads in flight
  TY v[64];
#pragma unroll
  for (int j = 0; j < 64; ++j) {
    const int t = __builtin_amdgcn_readlane(cur, j);
    v[j] = (Y + (int64_t)(j < k && t >= 0 && t != r ? t : zr) * B)[colc];
  }
#pragma unroll
  for (int j = 0; j < 64; ++j) acc -= (W)v[j];
  if (colok) (Y + (int64_t)r * B)[col] = (TY)acc;
}

// Level solve by runs (int64).  The rows of one chain that share a level are
// consecutive, and along them S(r) = Σ_{j != own} Y[niv_j(r)] changes only at
// the entries that differ from the row below: S(r) - S(r - 1) = Σ over those
// entries of Y[new] - Y[old].  Both rows of every such pair are entries of r
// or of r - 1, so they lie at lower levels and are final.  A workgroup takes a
// chunk {first row, (level << 6) | rows, first event, end event} of at most
// kSegRows consecutive rows of one chain in one level (see SegTables):
//   1. its row groups split the full sum S(first row) (entries rg, rg + RG, ...)
//      and the chunk's change events, adding each into its row's slot in LDS;
//   2. an inclusive scan of the slots over the rows gives every S(r), and
//      Y[r] = g[node(r)] - S(r).
// Wrapping 64-bit arithmetic is exact in any order, so the result equals the
// row-by-row solve bit for bit.  Loads of one batch are all in flight together.
template <typename TY, int CW>
__global__ __launch_bounds__(WG) void k_usolve_seg(DevPoset d, const int32_t* __restrict__ nv,
                                                   const int4* __restrict__ chunks, const int4* __restrict__ ev,
                                                   const TY* __restrict__ g, int64_t ldg, TY* __restrict__ Y,
                                                   int64_t B) {
  using W = typename Wide<TY>::W;
  constexpr int RG = WG / CW;       // row groups (4 .. 32)
  constexpr int SR = kSegRows / RG; // rows per row group in the scan (8 .. 1)
  static_assert(SR >= 1 && SR * RG == kSegRows, "kSegRows must be a multiple of the row groups");
  __shared__ W s_d[kSegRows][CW];
  __shared__ W s_t[RG][CW];
  auto uni = [](int v) { return CW == 64 ? __builtin_amdgcn_readfirstlane(v) : v; };
  const int lane = threadIdx.x % CW;
  const int rg = uni((int)(threadIdx.x / CW));
  const int64_t col = (int64_t)blockIdx.y * CW + lane;
  const bool colok = col < B;
  const int64_t colc = colok ? col : 0;
  const int4 c = chunks[blockIdx.x];
  const int r0 = uni(c.x), nrows = uni(c.y & 63), e0 = uni(c.z), e1 = uni(c.w);
  const int k = d.k;
  const int64_t zr = d.n;
#pragma unroll
  for (int i = 0; i < SR; ++i) s_d[rg * SR + i][lane] = W(0);
  __syncthreads();
  // g of this row group's scan rows
  W gv[SR];
#pragma unroll
  for (int i = 0; i < SR; ++i) {
    const int ri = rg * SR + i;
    const int node = uni(d.node_of_row[r0 + (ri < nrows ? ri : 0)]);
    gv[i] = (W)g[(int64_t)node * ldg + colc];
  }
  // the first row's full sum, entries rg, rg + RG, ... (own entry and -1 read the zero row)
  W part = W(0);
  const int32_t* __restrict__ nr0 = nv + (int64_t)r0 * k;
  for (int jb = rg; jb < k; jb += RG * 16) {
    int32_t t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int j = jb + u * RG;
      t[u] = j < k ? uni(nr0[j]) : -1;
    }
    TY v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = Y[(t[u] >= 0 && t[u] != r0 ? (int64_t)t[u] : zr) * B + colc];
#pragma unroll
    for (int u = 0; u < 16; ++u) part += (W)v[u];
  }
  // the change events of the later rows, e0 + rg, e0 + rg + RG, ...
  for (int eb = e0 + rg; eb < e1; eb += RG * 16) {
    int4 q[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = eb + u * RG;
      q[u] = e < e1 ? ev[e] : make_int4((int)zr, (int)zr, r0, 0);
      q[u].x = uni(q[u].x);
      q[u].y = uni(q[u].y);
      q[u].z = uni(q[u].z);
    }
    TY vn[16], vo[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      vn[u] = Y[(int64_t)q[u].x * B + colc];
      vo[u] = Y[(int64_t)q[u].y * B + colc];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (eb + u * RG < e1) atomicAdd(&s_d[q[u].z - r0][lane], (W)vn[u] - (W)vo[u]);
  }
  atomicAdd(&s_d[0][lane], part);
  __syncthreads();
  W sv[SR];
  W run = W(0);
#pragma unroll
  for (int i = 0; i < SR; ++i) {
    run += s_d[rg * SR + i][lane];
    sv[i] = run;
  }
  s_t[rg][lane] = run;
  __syncthreads();
  W base = W(0);
  for (int q = 0; q < rg; ++q) base += s_t[q][lane];
#pragma unroll
  for (int i = 0; i < SR; ++i) {
    const int ri = rg * SR + i;
    if (ri < nrows && colok) Y[(int64_t)(r0 + ri) * B + col] = (TY)(gv[i] - (base + sv[i]));
  }
}

// Relaxed device-scope loads and stores: coherent across the per-XCD L2s
// without cache maintenance (as the single-pass scan's tile states).
template <typename T>
__device__ inline T ld_dev(const T* p) {
  static_assert(sizeof(T) == 8, "64-bit elements");
  const uint64_t w = __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  T v;
  __builtin_memcpy(&v, &w, 8);
  return v;
}
template <typename T>
__device__ inline void st_dev(T* p, T v) {
  static_assert(sizeof(T) == 8, "64-bit elements");
  uint64_t w;
  __builtin_memcpy(&w, &v, 8);
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Longest wait of the persistent solve, in ticks of the 100 MHz real-time
// counter (2 s), whatever the polls cost.
constexpr uint64_t kFlowWaitTicks = 200000000ull;

// Waits until the flags fl[idx] of every index a lane holds (-1 = none) are
// set, all of them polled together in each round; exits are uniform over the
// active lanes.  Returns false when it gives up: after spin_limit polls, after
// kFlowWaitTicks, or when the error word is set.
template <int M>
__device__ inline bool await_idx(const int* __restrict__ fl, int (&idx)[M], const int* __restrict__ err,
                                 int spin_limit) {
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  for (int spin = 0;; ++spin) {
    int v[M];
#pragma unroll
    for (int m = 0; m < M; ++m)
      v[m] = idx[m] >= 0 ? __hip_atomic_load(fl + idx[m], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 1;
    bool pend = false;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (v[m] != 0) idx[m] = -1;
      pend = pend || idx[m] >= 0;
    }
    if (!__any(pend)) return true;
    if (spin >= spin_limit) return false;
    if ((spin & 15) == 15) {
      if (__builtin_amdgcn_readfirstlane(__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0)
        return false;
      if (__builtin_amdgcn_s_memrealtime() - t0 > kFlowWaitTicks) return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// The ready flags of up to N rows (row-group-uniform, -1 = none), lane l of a
// row group polling rows l, l + CW, ...
template <int CW, int N>
__device__ inline bool await_rows(const int* __restrict__ fl, const int32_t (&rows)[N], int lane,
                                  const int* __restrict__ err, int spin_limit) {
  constexpr int M = (N + CW - 1) / CW;
  int mine[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    int r = -1;
#pragma unroll
    for (int u = 0; u < N; ++u)
      if (u == lane + m * CW) r = rows[u];
    mine[m] = r;
  }
  return await_idx<M>(fl, mine, err, spin_limit);
}

// The ready flags of the rows of Q lists of N rows each at once (all polls of
// one round in flight together rather than one list after another).
template <int CW, int N, int Q>
__device__ inline bool await_rows_n(const int* __restrict__ fl, const int32_t* const (&lists)[Q], int lane,
                                    const int* __restrict__ err, int spin_limit) {
  constexpr int M = (N + CW - 1) / CW;
  int mine[Q * M];
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int m = 0; m < M; ++m) {
      int r = -1;
#pragma unroll
      for (int u = 0; u < N; ++u)
        if (u == lane + m * CW) r = lists[q][u];
      mine[q * M + m] = r;
    }
  return await_idx<Q * M>(fl, mine, err, spin_limit);
}

// Rows of Y not yet written by the persistent solve hold this mark.
constexpr int64_t kUnwritten = INT64_MIN;

// Reads the values of the lane's column in Q lists of N rows of Y (-1 = the
// zero row zr) into vals, until none is kUnwritten.  A round reads every value
// (a written value never changes, so settled entries just read the same word;
// the loads of a round are all in flight together).  While some entry is
// still marked, the wavefront polls only the first such entry (one load per
// lane and poll, so waiting workgroups add little traffic) and reads all
// again once it has been written.  A row's value can equal the mark
// legitimately: every fourth poll also reads the polled row's ready flag (set
// after the row's stores completed), and once it reads as set the next
// round's read of that entry, issued after the flag arrived, is taken as it
// is.  Exits are uniform over the active lanes; false when the wait gives up.
template <int N, int Q>
__device__ inline bool await_vals(const int64_t* __restrict__ Y, int64_t B, int64_t colc, int zr,
                                  const int32_t* const (&rows)[Q], int64_t* const (&vals)[Q],
                                  const int* __restrict__ fl, const int* __restrict__ err, int spin_limit) {
  uint32_t seen[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) seen[q] = 0;
  int spin = 0;
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  for (;;) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int u = 0; u < N; ++u) {
        int r = rows[q][u] >= 0 ? rows[q][u] : zr;
        asm volatile("" : "+v"(r));  // addresses formed in each round, not held across rounds
        vals[q][u] = ld_dev(&Y[(int64_t)r * B + colc]);
      }
    uint32_t pend[Q];
    bool any = false;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      pend[q] = 0;
#pragma unroll
      for (int u = 0; u < N; ++u)
        if (rows[q][u] >= 0 && !((seen[q] >> u) & 1) && vals[q][u] == kUnwritten) pend[q] |= 1u << u;
      any = any || pend[q] != 0;
    }
    if (!__any(any)) return true;
    // the first entry still pending in some lane (the same for the whole wavefront)
    int qs = -1, us = -1;
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int u = 0; u < N; ++u)
        if (qs < 0 && __any((pend[q] >> u) & 1)) {
          qs = q;
          us = u;
        }
    int rs = zr;
    bool mine = false;
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int u = 0; u < N; ++u)
        if (q == qs && u == us && ((pend[q] >> u) & 1)) {
          rs = rows[q][u];
          mine = true;
        }
    for (int poll = 0;; ++poll, ++spin) {
      if (spin >= spin_limit) return false;
      if ((spin & 15) == 15) {
        if (__builtin_amdgcn_readfirstlane(__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0)
          return false;
        if (__builtin_amdgcn_s_memrealtime() - t0 > kFlowWaitTicks) return false;
      }
      __builtin_amdgcn_s_sleep(1);
      if ((poll & 3) == 3) {
        const int f = __hip_atomic_load(fl + rs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wait_vmem();  // the flag has arrived before the next round's reads are issued
        const bool set = mine && f != 0;
#pragma unroll
        for (int q = 0; q < Q; ++q)
          if (q == qs && set) seen[q] |= 1u << us;
        if (__any(set)) break;
      }
      if (!__any(mine && ld_dev(&Y[(int64_t)rs * B + colc]) == kUnwritten)) break;
    }
  }
}

// One wavefront (all lanes active): the flags fl[a .. b), 512 at a time.
__device__ inline bool await_range(const int* __restrict__ fl, int a, int b, const int* __restrict__ err,
                                   int spin_limit) {
  const int lane = (int)(threadIdx.x & 63);
  for (int w = a; w < b; w += 512) {
    int idx[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) idx[m] = w + lane + 64 * m < b ? w + lane + 64 * m : -1;
    if (!await_idx<8>(fl, idx, err, spin_limit)) return false;
  }
  return true;
}

// The int64 solve by runs in one persistent launch: a dataflow over the chunks
// instead of one launch per level.  Workgroup b takes the (chunk, column
// block) items b, b + G, b + 2G, ... of the level-ordered list, G workgroups
// being at most what the device holds resident at once.  VALS (the default):
// a row group reads the rows of Y it needs until none holds the unwritten mark
// (await_vals; rows 0 .. n-1 of Y are filled with it before the launch).
// Otherwise, before it reads a row of Y a row group waits for that row's
// ready flag (one per row and column block), set by the chunk that wrote it
// (LEVEL: instead one wavefront waits for the done flags of every chunk of the
// level below, which are contiguous; those chunks waited for their own level
// below, so all lower levels are then complete; DEPS: for the done flags of
// the chunks it reads from).  A chunk reads only rows of lower levels, which come earlier in
// the list; a workgroup takes its items in order, so the unfinished item of
// lowest index always has every row it reads finished, and with all
// workgroups resident every wait ends.  Everything that does not depend on Y
// (the chunk, g, the first row's entries, the events) is loaded before the
// waits.
//
// Y and the flags travel as relaxed device-scope stores and loads, which are
// coherent across the per-XCD L2s (as the single-pass scan's tile states); a
// row group sets its rows' flags after its wave's Y stores have completed
// (vmcnt 0).  No read-modify-write atomics cross workgroups.
//
// Waits are bounded (spin_limit polls, and 2 s of real time).  A workgroup
// that gives up (also when some workgroups could not be resident) stores the
// error word and stops, and so does every waiter that sees it; then
// k_usolve_flow_fix recomputes the whole solve in one workgroup.  flags:
// ncb * (n + 1) ints (chunk flags: ncb * nchunks) and err, cleared before the
// launch; the row flags are set in VALS mode too, for values equal to the mark.
template <typename TY, int CW, int WAIT>
__global__ __launch_bounds__(WG) void k_usolve_flow(DevPoset d, const int32_t* __restrict__ nv,
                                                    const int4* __restrict__ chunks, int nchunks,
                                                    const int32_t* __restrict__ lev_off,
                                                    const int32_t* __restrict__ dep_ptr,
                                                    const int32_t* __restrict__ deps,
                                                    const int4* __restrict__ ev, const TY* __restrict__ g,
                                                    int64_t ldg, TY* __restrict__ Y, int64_t B,
                                                    int* __restrict__ flags, int* __restrict__ err, int spin_limit) {
  using W = typename Wide<TY>::W;
  constexpr int RG = WG / CW;
  constexpr int SR = kSegRows / RG;
  constexpr bool LEVEL = WAIT == kWaitLevel || WAIT == kWaitDeps;  // chunk done flags
  constexpr bool VALS = WAIT == kWaitValues;  // polls the values (no flag waits before the reads)
  // entries and events per row group and batch: 16; polling the values, 64 per
  // workgroup (fewer registers in flight, so that two workgroups fit per CU)
  constexpr int NB = !VALS ? 16 : 64 / RG < 2 ? 2 : 64 / RG > 16 ? 16 : 64 / RG;
  static_assert(SR >= 1 && SR * RG == kSegRows, "kSegRows must be a multiple of the row groups");
  __shared__ W s_d[kSegRows][CW];
  __shared__ W s_t[RG][CW];
  __shared__ int s_bad;
  auto uni = [](int v) { return CW == 64 ? __builtin_amdgcn_readfirstlane(v) : v; };
  const int lane = threadIdx.x % CW;
  const int rg = uni((int)(threadIdx.x / CW));
  const int ncb = (int)((B + CW - 1) / CW);
  const int total = nchunks * ncb;
  const int k = d.k;
  const int zr = d.n;
  for (int tk = blockIdx.x; tk < total; tk += gridDim.x) {
    const int ci = tk / ncb, cb = tk - ci * ncb;
    // LEVEL: one done flag per chunk; otherwise one ready flag per row
    int* const fl = flags + (int64_t)cb * (LEVEL ? nchunks : zr + 1);
    const int64_t col = (int64_t)cb * CW + lane;
    const bool colok = col < B;
    const int64_t colc = colok ? col : 0;
    const int4 c = chunks[ci];
    const int r0 = uni(c.x), nrows = uni(c.y & 63), e0 = uni(c.z), e1 = uni(c.w);
#pragma unroll
    for (int i = 0; i < SR; ++i) s_d[rg * SR + i][lane] = W(0);
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    W gv[SR];
#pragma unroll
    for (int i = 0; i < SR; ++i) {
      const int ri = rg * SR + i;
      const int node = uni(d.node_of_row[r0 + (ri < nrows ? ri : 0)]);
      gv[i] = (W)g[(int64_t)node * ldg + colc];
    }
    // the first batches of the first row's entries (rg, rg + RG, ...; own entry
    // and -1 skipped) and of the events (e0 + rg, e0 + rg + RG, ...), loaded
    // before the wait like g
    const int32_t* __restrict__ nr0 = nv + (int64_t)r0 * k;
    int32_t t[NB], a[NB], b[NB], rr[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int j = rg + u * RG;
      const int tt = j < k ? uni(nr0[j]) : -1;
      t[u] = tt != r0 ? tt : -1;
    }
    auto load_events = [&](int eb) {
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int e = eb + u * RG;
        const int4 q = e < e1 ? ev[e] : make_int4(zr, zr, r0, 0);
        a[u] = uni(q.x) != zr ? uni(q.x) : -1;
        b[u] = uni(q.y) != zr ? uni(q.y) : -1;
        rr[u] = uni(q.z);
      }
    };
    load_events(e0 + rg);
    // WAIT == kWaitDeps: the chunks this one reads from, up to 128 loaded now
    int dp0 = 0, dp1 = 0, dv[2] = {-1, -1};
    const int wl = (int)(threadIdx.x & 63);
    if (WAIT == kWaitDeps && threadIdx.x < 64) {
      dp0 = __builtin_amdgcn_readfirstlane(dep_ptr[ci]);
      dp1 = __builtin_amdgcn_readfirstlane(dep_ptr[ci + 1]);
#pragma unroll
      for (int m = 0; m < 2; ++m) dv[m] = dp0 + wl + 64 * m < dp1 ? deps[dp0 + wl + 64 * m] : -1;
    }
    bool ok = true;
    if (LEVEL) {
      if (WAIT == kWaitLevel) {  // every chunk of the level below (and so every lower level) is done
        const int lev = uni(c.y >> 6);
        if (lev > 0 && threadIdx.x < 64)
          if (!await_range(fl, lev_off[lev - 1], lev_off[lev], err, spin_limit)) s_bad = 1;
      } else if (threadIdx.x < 64) {  // every chunk holding a row this one reads is done
        bool good = await_idx<2>(fl, dv, err, spin_limit);
        for (int w = dp0 + 128; w < dp1 && good; w += 128) {
          int more[2];
#pragma unroll
          for (int m = 0; m < 2; ++m) more[m] = w + wl + 64 * m < dp1 ? deps[w + wl + 64 * m] : -1;
          good = await_idx<2>(fl, more, err, spin_limit);
        }
        if (!good) s_bad = 1;
      }
      __syncthreads();
      if (__builtin_amdgcn_readfirstlane(s_bad)) {
        if (threadIdx.x == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    } else if (!VALS) {
      const int32_t* const lists[3] = {t, a, b};
      ok = await_rows_n<CW, NB, 3>(fl, lists, lane, err, spin_limit);
    }
    W part = W(0);
    if (ok) {  // the first batches' rows of Y, all in flight together
      TY v[NB], vn[NB], vo[NB];
      if (VALS) {
        const int32_t* const lists[3] = {t, a, b};
        int64_t* const outs[3] = {v, vn, vo};
        ok = await_vals<NB, 3>(Y, B, colc, zr, lists, outs, fl, err, spin_limit);
      } else {
#pragma unroll
        for (int u = 0; u < NB; ++u) {
          v[u] = ld_dev(&Y[(int64_t)(t[u] >= 0 ? t[u] : zr) * B + colc]);
          vn[u] = ld_dev(&Y[(int64_t)(a[u] >= 0 ? a[u] : zr) * B + colc]);
          vo[u] = ld_dev(&Y[(int64_t)(b[u] >= 0 ? b[u] : zr) * B + colc]);
        }
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) part += (W)v[u];
#pragma unroll
      for (int u = 0; u < NB; ++u)
        if (e0 + rg + u * RG < e1) atomicAdd(&s_d[rr[u] - r0][lane], (W)vn[u] - (W)vo[u]);
    }
    // later batches (k > NB * RG, or more than NB events per row group)
    for (int jb = rg + NB * RG; jb < k && ok; jb += RG * NB) {
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int j = jb + u * RG;
        const int tt = j < k ? uni(nr0[j]) : -1;
        t[u] = tt != r0 ? tt : -1;
      }
      if (!LEVEL && !VALS) ok = await_rows<CW, NB>(fl, t, lane, err, spin_limit);
      if (!ok) break;
      TY v[NB];
      if (VALS) {
        const int32_t* const lists[1] = {t};
        int64_t* const outs[1] = {v};
        if (!await_vals<NB, 1>(Y, B, colc, zr, lists, outs, fl, err, spin_limit)) {
          ok = false;
          break;
        }
      } else {
#pragma unroll
        for (int u = 0; u < NB; ++u) v[u] = ld_dev(&Y[(int64_t)(t[u] >= 0 ? t[u] : zr) * B + colc]);
      }
#pragma unroll
      for (int u = 0; u < NB; ++u) part += (W)v[u];
    }
    for (int eb = e0 + rg + NB * RG; eb < e1 && ok; eb += RG * NB) {
      load_events(eb);
      if (!LEVEL && !VALS) {
        const int32_t* const lists[2] = {a, b};
        ok = await_rows_n<CW, NB, 2>(fl, lists, lane, err, spin_limit);
      }
      if (!ok) break;
      TY vn[NB], vo[NB];
      if (VALS) {
        const int32_t* const lists[2] = {a, b};
        int64_t* const outs[2] = {vn, vo};
        if (!await_vals<NB, 2>(Y, B, colc, zr, lists, outs, fl, err, spin_limit)) {
          ok = false;
          break;
        }
      } else {
#pragma unroll
        for (int u = 0; u < NB; ++u) {
          vn[u] = ld_dev(&Y[(int64_t)(a[u] >= 0 ? a[u] : zr) * B + colc]);
          vo[u] = ld_dev(&Y[(int64_t)(b[u] >= 0 ? b[u] : zr) * B + colc]);
        }
      }
#pragma unroll
      for (int u = 0; u < NB; ++u)
        if (eb + u * RG < e1) atomicAdd(&s_d[rr[u] - r0][lane], (W)vn[u] - (W)vo[u]);
    }
    if (ok)
      atomicAdd(&s_d[0][lane], part);
    else
      s_bad = 1;
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s_bad)) {
      if (threadIdx.x == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    W sv[SR];
    W run = W(0);
#pragma unroll
    for (int i = 0; i < SR; ++i) {
      run += s_d[rg * SR + i][lane];
      sv[i] = run;
    }
    s_t[rg][lane] = run;
    __syncthreads();
    W base = W(0);
    for (int z = 0; z < rg; ++z) base += s_t[z][lane];
#pragma unroll
    for (int i = 0; i < SR; ++i) {
      const int ri = rg * SR + i;
      if (ri < nrows && colok) st_dev(&Y[(int64_t)(r0 + ri) * B + col], (TY)(gv[i] - (base + sv[i])));
    }
    wait_vmem();
    if (LEVEL) {
      __syncthreads();  // every wave's Y stores have completed
      if (threadIdx.x == 0) __hip_atomic_store(&fl[ci], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (lane == 0) {
#pragma unroll
      for (int i = 0; i < SR; ++i) {
        const int ri = rg * SR + i;
        if (ri < nrows) __hip_atomic_store(&fl[r0 + ri], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// Fallback of k_usolve_flow: when its error word is set, one workgroup solves
// again from scratch, chunk after chunk in level order with a barrier between
// levels, every row by its full sum; otherwise it returns at once.
template <typename TY>
__global__ __launch_bounds__(WG) void k_usolve_flow_fix(DevPoset d, const int32_t* __restrict__ nv,
                                                        const int4* __restrict__ chunks, int nchunks,
                                                        const TY* __restrict__ g, int64_t ldg, TY* __restrict__ Y,
                                                        int64_t B, const int* __restrict__ err) {
  using W = typename Wide<TY>::W;
  if (__builtin_amdgcn_readfirstlane(__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 0) return;
  const int k = d.k;
  const int64_t zr = d.n;
  const int64_t nel = (int64_t)kSegRows * B;
  int lev = -1;
  for (int ci = 0; ci < nchunks; ++ci) {
    const int4 c = chunks[ci];
    if ((c.y >> 6) != lev) {
      __syncthreads();
      lev = c.y >> 6;
    }
    const int nrows = c.y & 63;
    for (int64_t i = threadIdx.x; i < nel; i += WG) {
      const int ri = (int)(i / B);
      const int64_t col = i - (int64_t)ri * B;
      if (ri >= nrows) continue;
      const int64_t r = (int64_t)c.x + ri;
      W acc = (W)g[(int64_t)d.node_of_row[r] * ldg + col];
      for (int j = 0; j < k; ++j) {
        const int tt = nv[r * k + j];
        if (tt >= 0 && tt != r) acc -= (W)ld_dev(&Y[(int64_t)tt * B + col]);
      }
      st_dev(&Y[r * B + col], (TY)acc);
    }
  }
}

__global__ void k_zero_bytes(uint32_t* p, int64_t words) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i < words) p[i] = 0u;
}

// ------------------------------------------------------------ chain difference
// With stats != nullptr (refinement, accumulate mode): per column the largest
// |correction| into stats[col], the largest |updated value| into stats[B+col]
// (float64 bit patterns, non-negative so integer max orders them), and a
// non-finite flag into stats[2B]; reduced over the workgroup's rows in LDS
// first, one atomic per column per workgroup.
template <typename TY, typename Tout, int CWT>
__global__ __launch_bounds__(WG) void k_chain_diff(DevPoset d, int dir, int cw_rt, const TY* __restrict__ Y, int64_t B,
                                                   Tout* __restrict__ out, int64_t ldo, int accumulate,
                                                   uint64_t* __restrict__ stats) {
  using W = typename Wide<TY>::W;
  constexpr int RPC = 8;  // rows per thread, loads in flight together
  const int cw = CWT ? CWT : cw_rt;
  const int RG = WG / cw;
  // with 64-wide column blocks a row group is one wavefront: rows are uniform
  auto uni = [](int v) { return CWT == 64 ? __builtin_amdgcn_readfirstlane(v) : v; };
  const int rbase = uni((int)((blockIdx.x * RG + threadIdx.x / cw) * RPC));
  const int64_t col = (int64_t)blockIdx.y * cw + threadIdx.x % cw;
  const int64_t colc = col < B ? col : 0;
  const int n = d.n;
  int nd[RPC], nb[RPC], bound[RPC];
  TY y[RPC], yb[RPC];
  // in phases, so that each phase's loads are in flight together: the rows'
  // chains and nodes, the chains' end rows, then the rows of Y
#pragma unroll
  for (int i = 0; i < RPC; ++i) {
    const int r = min(rbase + i, n - 1);
    bound[i] = uni(d.chain_of_row[r]) + (dir > 0 ? 0 : 1);
    nd[i] = uni(d.node_of_row[r]);
  }
#pragma unroll
  for (int i = 0; i < RPC; ++i) bound[i] = uni(d.chain_off[bound[i]]);
#pragma unroll
  for (int i = 0; i < RPC; ++i) {
    const int r = min(rbase + i, n - 1);
    // the neighbour in the chain (below for dir > 0, above otherwise); the
    // chain's end rows take the row itself and subtract nothing
    const int rb = dir > 0 ? (r > bound[i] ? r - 1 : -1) : (r + 1 < bound[i] ? r + 1 : -1);
    nb[i] = uni(rb);
    y[i] = Y[(int64_t)r * B + colc];
    yb[i] = Y[(int64_t)(rb >= 0 ? rb : r) * B + colc];
  }
  // the iterate, when accumulating a correction, loads with the rows above
  Tout ov[RPC];
  if (accumulate) {
#pragma unroll
    for (int i = 0; i < RPC; ++i) ov[i] = out[(int64_t)nd[i] * ldo + colc];
  }
  double dmax = 0, fmax = 0;
  bool bad = false;
  if (col < B) {
#pragma unroll
    for (int i = 0; i < RPC; ++i) {
      if (rbase + i >= n) break;
      W v = (W)y[i];
      if (nb[i] >= 0) v -= (W)yb[i];
      Tout* o = out + (int64_t)nd[i] * ldo + col;
      const Tout nvv = accumulate ? (Tout)((W)ov[i] + v) : (Tout)v;
      *o = nvv;
      if constexpr (std::is_floating_point<W>::value) {
        const double a1 = fabs((double)v), a2 = fabs((double)nvv);
        bad = bad || !isfinite(a1) || !isfinite(a2);
        dmax = fmax_(dmax, a1);
        fmax = fmax_(fmax, a2);
      }
    }
  }
  if (!stats) return;
  __shared__ double sd[WG], sf[WG];
  __shared__ int sb;
  if (threadIdx.x == 0) sb = 0;
  __syncthreads();
  sd[threadIdx.x] = bad ? 0.0 : dmax;
  sf[threadIdx.x] = bad ? 0.0 : fmax;
  if (bad) sb = 1;
  __syncthreads();
  if ((int)threadIdx.x < cw && col < B) {
    double a = 0, bb = 0;
    for (int g = 0; g < RG; ++g) {
      a = fmax_(a, sd[g * cw + threadIdx.x]);
      bb = fmax_(bb, sf[g * cw + threadIdx.x]);
    }
    atomicMax((unsigned long long*)&stats[col], (unsigned long long)__double_as_longlong(a));
    atomicMax((unsigned long long*)&stats[B + col], (unsigned long long)__double_as_longlong(bb));
  }
  if (threadIdx.x == 0 && sb) atomicMax((unsigned long long*)&stats[2 * B], 1ull);
}

// --------------------------------------------------------------- statistics
template <typename TG>
__global__ __launch_bounds__(WG) void k_absmax(int64_t n, int64_t B, int cw, const double* __restrict__ r,
                                               const TG* __restrict__ g, int64_t ldg, uint64_t* stats) {
  // each thread keeps the maxima of its rows of one column; the row groups of a
  // workgroup are folded in LDS and one lane per column updates the totals
  // (bit patterns of non-negative doubles order as unsigned integers)
  __shared__ double sa[WG], sb[WG];
  const int RG = WG / cw;
  const int rg = threadIdx.x / cw;
  const int64_t col = (int64_t)blockIdx.y * cw + threadIdx.x % cw;
  double ma = 0, mb = 0;
  bool bad = false;
  if (col < B) {
    for (int64_t x = (int64_t)blockIdx.x * RG + rg; x < n; x += (int64_t)gridDim.x * RG) {
      const double a = fabs(r[x * B + col]);
      const double b = fabs((double)g[x * ldg + col]);
      if (!isfinite(a) || !isfinite(b)) {
        bad = true;
        continue;
      }
      ma = fmax_(ma, a);
      mb = fmax_(mb, b);
    }
  }
  sa[threadIdx.x] = ma;
  sb[threadIdx.x] = mb;
  if (bad) atomicMax((unsigned long long*)&stats[2 * B], 1ull);
  __syncthreads();
  if (rg == 0 && col < B) {
    for (int q = 1; q < RG; ++q) {
      ma = fmax_(ma, sa[q * cw + threadIdx.x]);
      mb = fmax_(mb, sb[q * cw + threadIdx.x]);
    }
    atomicMax((unsigned long long*)&stats[col], (unsigned long long)__double_as_longlong(ma));
    atomicMax((unsigned long long*)&stats[B + col], (unsigned long long)__double_as_longlong(mb));
  }
}

__global__ void k_fill_u64(uint64_t* p, int64_t cnt, uint64_t v) {
  int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i < cnt) p[i] = v;
}

inline dim3 grid2(int64_t rows, int cw, int64_t B) {
  const int64_t RG = WG / cw;
  return dim3((unsigned)((rows + RG - 1) / RG), (unsigned)((B + cw - 1) / cw));
}

// Short chains (every chain within one scan tile and at most kShortChain
// rows): one thread per (chain, column) scans its chain's rows in order, 16
// loads in flight, instead of a 64-row tile per chain of which wide sparse
// posets (chains of ~5 rows) fill a twelfth.  Row n of P is set to zero here.
constexpr int kShortChain = 256;
template <typename Tin, typename Tout>
__global__ __launch_bounds__(WG) void k_scan_chains(DevPoset d, int dir, int cw, const Tin* __restrict__ x,
                                                    int64_t ldx, int64_t B, Tout* __restrict__ P) {
  using Tr = ScanTraits<Tin, Tout>;
  using St = typename Tr::St;
  const int RG = WG / cw;
  const int64_t c = (int64_t)blockIdx.x * RG + threadIdx.x / cw;
  const int64_t col = (int64_t)blockIdx.y * cw + threadIdx.x % cw;
  if (col >= B) return;
  if (c == 0) P[(int64_t)d.n * B + col] = Tout(0);
  if (c >= d.nchains) return;
  const int64_t r0 = d.chain_off[c], r1 = d.chain_off[c + 1], len = r1 - r0;
  St st;
  st.zero();
  for (int64_t i0 = 0; i0 < len; i0 += 16) {
    int32_t nodes[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int64_t i = min(i0 + u, len - 1);
      nodes[u] = node_at(d, dir > 0 ? r0 + i : r1 - 1 - i);
    }
    Tin raw[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) raw[u] = x[(int64_t)nodes[u] * ldx + col];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if (i0 + u >= len) break;
      st.add(Tr::in(raw[u]));
      const int64_t r = dir > 0 ? r0 + i0 + u : r1 - 1 - i0 - u;
      P[r * B + col] = Tr::out(st.value());
    }
  }
}

// Flat tiles for tile height segi when the host chose them (d.flat_mask);
// POSETX_SCAN_FLAT=0 / 1 (read on every call) never / always takes them.
bool flat_scan(const DevPoset& d, int segi) {
  const char* e = std::getenv("POSETX_SCAN_FLAT");
  if (e && e[0] == '0') return false;
  if (e && e[0] == '1') return d.chain_of_row && d.chain_off;
  return (d.flat_mask >> segi) & 1u;
}

template <typename Tin, typename Tout>
hipError_t scan_typed(int phase, const DevPoset& d, int dir, const void* x, int64_t ldx, void* P, int64_t B,
                      void* aux, int64_t ntiles, hipStream_t s) {
  using St = typename ScanTraits<Tin, Tout>::St;
  const int cw = col_width(B);
  const int segi = seg_index(cw);
  St* A = (St*)aux;
  // 32-bit offsets for f (node order, n rows of ldx) and P (n + 1 rows of B)
  const bool o32 = fits32((int64_t)d.n * ldx * (int64_t)sizeof(Tin)) &&
                   fits32(((int64_t)d.n + 1) * B * (int64_t)sizeof(Tout));
  if (cw < 64 && flat_scan(d, segi)) {  // flat tiles (see k_scan_reduce_flat)
    const int H = seg_rows(cw);
    const int64_t nft = ((int64_t)d.n + H - 1) / H;
    if (nft > ntiles) return hipErrorInvalidValue;  // aux holds ntiles tile states per column
    St* Cf = A + ntiles * B;
    const dim3 gf((unsigned)nft, (unsigned)((B + cw - 1) / cw));
    if (phase == 0) {
      if (o32)
        hipLaunchKernelGGL((k_scan_reduce_flat<Tin, Tout, true>), gf, dim3(WG), 0, s, d, cw, dir, (const Tin*)x, ldx, B, A);
      else
        hipLaunchKernelGGL((k_scan_reduce_flat<Tin, Tout, false>), gf, dim3(WG), 0, s, d, cw, dir, (const Tin*)x, ldx, B,
                           A);
    } else if (phase == 1) {
      const int64_t threads = nft * B;
      hipLaunchKernelGGL((k_scan_carry_flat<St, Tout>), dim3((unsigned)((threads + WG - 1) / WG)), dim3(WG), 0, s, d,
                         H, nft, dir, B, (const St*)A, Cf, (Tout*)P);
    } else if (o32) {
      hipLaunchKernelGGL((k_scan_apply_flat<Tin, Tout, true>), gf, dim3(WG), 0, s, d, cw, dir, (const Tin*)x, ldx, B,
                         (const St*)Cf, (Tout*)P);
    } else {
      hipLaunchKernelGGL((k_scan_apply_flat<Tin, Tout, false>), gf, dim3(WG), 0, s, d, cw, dir, (const Tin*)x, ldx, B,
                         (const St*)Cf, (Tout*)P);
    }
    return hipGetLastError();
  }
  // when every chain fits one tile (short chains, e.g. wide sparse posets) there
  // are no carries: phases 0 and 1 do nothing and phase 2 scans each tile alone
  const bool one_tile = d.max_chain_tiles[segi] == 1;
  if (one_tile && phase < 2) return hipSuccess;
  St* C = one_tile ? nullptr : A + ntiles * B;
  if (one_tile && d.max_chain <= kShortChain) {
    const dim3 gc((unsigned)((d.nchains + WG / cw - 1) / (WG / cw)), (unsigned)((B + cw - 1) / cw));
    hipLaunchKernelGGL((k_scan_chains<Tin, Tout>), gc, dim3(WG), 0, s, d, dir, cw, (const Tin*)x, ldx, B, (Tout*)P);
    return hipGetLastError();
  }
  dim3 g((unsigned)ntiles, (unsigned)((B + cw - 1) / cw));
  if (phase == 0) {
    const int nt = reduce_tiles(cw == 64 ? 64 : 0);
    const dim3 g2((unsigned)((ntiles + nt - 1) / nt), (unsigned)((B + cw - 1) / cw));
    if (cw == 64)
      hipLaunchKernelGGL((k_scan_reduce<Tin, Tout, 64, false>), g2, dim3(WG), 0, s, d, segi, cw, (const Tin*)x,
                         ldx, B, ntiles, A, dir, (const uint64_t*)nullptr, (const int32_t*)nullptr, (Tout*)nullptr);
    else if (o32)
      hipLaunchKernelGGL((k_scan_reduce<Tin, Tout, 0, false, true>), g2, dim3(WG), 0, s, d, segi, cw, (const Tin*)x,
                         ldx, B, ntiles, A, dir, (const uint64_t*)nullptr, (const int32_t*)nullptr, (Tout*)nullptr);
    else
      hipLaunchKernelGGL((k_scan_reduce<Tin, Tout, 0, false>), g2, dim3(WG), 0, s, d, segi, cw, (const Tin*)x,
                         ldx, B, ntiles, A, dir, (const uint64_t*)nullptr, (const int32_t*)nullptr, (Tout*)nullptr);
  } else if (phase == 1) {
    if (d.max_chain_tiles[segi] <= kShortCarry) {
      const int64_t threads = (int64_t)d.nchains * B;
      hipLaunchKernelGGL((k_scan_carry_short<St, Tout>), dim3((unsigned)((threads + WG - 1) / WG)), dim3(WG), 0, s,
                         d, segi, dir, B, (const St*)A, C, (Tout*)P);
    } else {
      hipLaunchKernelGGL((k_scan_carry<St, Tout, false>), dim3((unsigned)d.nchains, (unsigned)((B + 15) / 16)),
                         dim3(WG), 0, s, d, segi, dir, B, (const St*)A, C, (Tout*)P, (const int32_t*)nullptr,
                         (const int32_t*)nullptr, (const Tout*)nullptr, 0);
    }
  } else if (cw == 64) {
    hipLaunchKernelGGL((k_scan_apply<Tin, Tout, 64, 0, Tout>), g, dim3(WG), 0, s, d, segi, cw, dir, (const Tin*)x,
                       ldx, B, (const St*)C, (Tout*)P, (const int32_t*)nullptr, (const Tout*)nullptr, 0,
                       (const Tout*)nullptr, 0);
  } else if (o32) {
    hipLaunchKernelGGL((k_scan_apply<Tin, Tout, 0, 0, Tout, true>), g, dim3(WG), 0, s, d, segi, cw, dir, (const Tin*)x,
                       ldx, B, (const St*)C, (Tout*)P, (const int32_t*)nullptr, (const Tout*)nullptr, 0,
                       (const Tout*)nullptr, 0);
  } else {
    hipLaunchKernelGGL((k_scan_apply<Tin, Tout, 0, 0, Tout>), g, dim3(WG), 0, s, d, segi, cw, dir, (const Tin*)x,
                       ldx, B, (const St*)C, (Tout*)P, (const int32_t*)nullptr, (const Tout*)nullptr, 0,
                       (const Tout*)nullptr, 0);
  }
  return hipGetLastError();
}

// Workgroups per (chain, 16 columns) of the compact carry: each completes a
// quarter of the chain's gathered rows.
constexpr int kCarrySplit = 4;

// The narrow compact walk (8 <= cw <= 32): k_scan_reduce_cn, the shared
// carry, the vector-lane or lane-split walk on Q, k_scan_apply_cn (MODE 1: zeta
// values; MODE 2: refinement residuals against resid, type Tres).
template <typename Tin, typename Tout, int MODE, typename Tres>
hipError_t compact_narrow_typed(const DevPoset& d, int dir, const void* x, int64_t ldx, void* out, int64_t ldo,
                                const void* resid, int64_t ldr, int64_t B, void* aux, int64_t ntiles, void* lq,
                                void* snaps, LaunchHook* hook, hipStream_t s) {
  using St = typename ScanTraits<Tin, Tout>::St;
  const WalkTables& w = d.walk[dir > 0 ? 0 : 1];
  const int cw = col_width(B);
  St* A = (St*)aux;
  St* C = A + ntiles * B;
  Tout* L = (Tout*)lq;
  Tout* Q = L + (int64_t)w.nslots * B;
  const int tpw = WG / cw / 4;
  const dim3 g((unsigned)((ntiles + tpw - 1) / tpw));
  const bool o32 = fits32((int64_t)d.n * ldx * (int64_t)sizeof(Tin)) &&
                   fits32((int64_t)d.n * ldo * (int64_t)sizeof(Tout)) &&
                   fits32((int64_t)w.nsnap * B * (int64_t)sizeof(Tout)) &&
                   (MODE != 2 || fits32((int64_t)d.n * ldr * (int64_t)sizeof(Tres)));
  if (hook) hook->before(0, s);
  if (o32)
    hipLaunchKernelGGL((k_scan_reduce_cn<Tin, Tout, true>), g, dim3(WG), 0, s, d, cw, dir, (const Tin*)x, ldx, B,
                       ntiles, A, w.tmask, w.qoff, L);
  else
    hipLaunchKernelGGL((k_scan_reduce_cn<Tin, Tout, false>), g, dim3(WG), 0, s, d, cw, dir, (const Tin*)x, ldx, B,
                       ntiles, A, w.tmask, w.qoff, L);
  if (hook) hook->after(0, s);
  if (hook) hook->before(1, s);
  hipLaunchKernelGGL((k_scan_carry<St, Tout, true>),
                     dim3((unsigned)d.nchains, (unsigned)((B + 15) / 16), (unsigned)kCarrySplit), dim3(WG), 0, s, d,
                     seg_index(64), dir, B, (const St*)A, C, Q, w.qoff, w.tile_of_slot, (const Tout*)L, w.nslots);
  if (hook) hook->after(1, s);
  if (hook) hook->before(2, s);
  if (walk_vec_ok<Tout>(cw, B, w.nruns)) {
    constexpr int V = 16 / sizeof(Tout);
    const int Lr = cw / V;
    const int64_t waves = (w.nruns + (64 / Lr) - 1) / (64 / Lr);
    const dim3 gw((unsigned)((waves + (WG / 64) - 1) / (WG / 64)));
    const Tout* q = Q;
    Tout* sn = (Tout*)snaps;
    if (Lr == 2) hipLaunchKernelGGL((k_walk_events_vec<Tout, 2, 16, true>), gw, dim3(WG), 0, s, d, nullptr, w, q, B, sn);
    else if (Lr == 4) hipLaunchKernelGGL((k_walk_events_vec<Tout, 4, 16, true>), gw, dim3(WG), 0, s, d, nullptr, w, q, B, sn);
    else if (Lr == 8) hipLaunchKernelGGL((k_walk_events_vec<Tout, 8, 16, true>), gw, dim3(WG), 0, s, d, nullptr, w, q, B, sn);
    else hipLaunchKernelGGL((k_walk_events_vec<Tout, 16, 16, true>), gw, dim3(WG), 0, s, d, nullptr, w, q, B, sn);
  } else {
    const int64_t waves = (w.nruns + (64 / cw) - 1) / (64 / cw);
    hipLaunchKernelGGL((k_walk_events_split<Tout, true>), dim3((unsigned)((waves + (WG / 64) - 1) / (WG / 64))),
                       dim3(WG), 0, s, d, nullptr, w, cw, (const Tout*)Q, B, (Tout*)snaps);
  }
  if (hook) hook->after(2, s);
  if (hook) hook->before(3, s);
  if (o32)
    hipLaunchKernelGGL((k_scan_apply_cn<Tin, Tout, MODE, Tres, true>), g, dim3(WG), 0, s, d, cw, dir, (const Tin*)x,
                       ldx, B, ntiles, (const St*)C, (Tout*)out, ldo, w.snap_of_row, (const Tout*)snaps,
                       (const Tres*)resid, ldr);
  else
    hipLaunchKernelGGL((k_scan_apply_cn<Tin, Tout, MODE, Tres, false>), g, dim3(WG), 0, s, d, cw, dir, (const Tin*)x,
                       ldx, B, ntiles, (const St*)C, (Tout*)out, ldo, w.snap_of_row, (const Tout*)snaps,
                       (const Tres*)resid, ldr);
  if (hook) hook->after(3, s);
  return hipGetLastError();
}

template <typename Tin, typename Tout, int MODE, typename Tres>
hipError_t compact_typed(const DevPoset& d, int dir, const void* x, int64_t ldx, void* out, int64_t ldo,
                         const void* resid, int64_t ldr, int64_t B, void* aux, int64_t ntiles, void* lq,
                         void* snaps, LaunchHook* hook, hipStream_t s) {
  using St = typename ScanTraits<Tin, Tout>::St;
  const WalkTables& w = d.walk[dir > 0 ? 0 : 1];
  const int segi = seg_index(64);
  {
    const int cw = col_width(B);
    if (cw >= 8 && cw <= 32)
      return compact_narrow_typed<Tin, Tout, MODE, Tres>(d, dir, x, ldx, out, ldo, resid, ldr, B, aux, ntiles, lq,
                                                         snaps, hook, s);
  }
  St* A = (St*)aux;
  St* C = A + ntiles * B;
  Tout* L = (Tout*)lq;
  Tout* Q = L + (int64_t)w.nslots * B;
  const unsigned ncb = (unsigned)((B + 63) / 64);
  if (hook) hook->before(0, s);
  hipLaunchKernelGGL((k_scan_reduce<Tin, Tout, 64, true>), dim3((unsigned)((ntiles + reduce_tiles(64) - 1) / reduce_tiles(64)), ncb), dim3(WG), 0, s,
                     d, segi, 64, (const Tin*)x, ldx, B, ntiles, A, dir, w.tmask, w.qoff, L);
  if (hook) hook->after(0, s);
  if (hook) hook->before(1, s);
  hipLaunchKernelGGL((k_scan_carry<St, Tout, true>),
                     dim3((unsigned)d.nchains, (unsigned)((B + 15) / 16), (unsigned)kCarrySplit), dim3(WG), 0, s, d,
                     segi, dir, B, (const St*)A, C, Q, w.qoff, w.tile_of_slot, (const Tout*)L, w.nslots);
  if (hook) hook->after(1, s);
  if (hook) hook->before(2, s);
  {
    const int64_t waves = (int64_t)w.nruns * ncb;
    const dim3 g((unsigned)((waves + (WG / 64) - 1) / (WG / 64)));
    if (((int64_t)w.nslots + 1) * B * (int64_t)sizeof(Tout) < ((int64_t)1 << 31))
      hipLaunchKernelGGL((k_walk_events<Tout, true, true>), g, dim3(WG), 0, s, d, (const int32_t*)nullptr, w,
                         (const Tout*)Q, B, (Tout*)snaps);
    else
      hipLaunchKernelGGL((k_walk_events<Tout, false, true>), g, dim3(WG), 0, s, d, (const int32_t*)nullptr, w,
                         (const Tout*)Q, B, (Tout*)snaps);
  }
  if (hook) hook->after(2, s);
  if (hook) hook->before(3, s);
  hipLaunchKernelGGL((k_scan_apply<Tin, Tout, 64, MODE, Tres>), dim3((unsigned)ntiles, ncb), dim3(WG), 0, s, d, segi,
                     64, dir, (const Tin*)x, ldx, B, (const St*)C, (Tout*)out, w.snap_of_row, (const Tout*)snaps,
                     ldo, (const Tres*)resid, ldr);
  if (hook) hook->after(3, s);
  return hipGetLastError();
}

}  // namespace

namespace {
template <typename Tin, typename Tout>
hipError_t onepass_typed(const DevPoset& d, int dir, const void* x, int64_t ldx, void* P, int64_t B, void* aux,
                         int64_t ntiles, int* sync, int spin_limit, hipStream_t s) {
  using St = typename ScanTraits<Tin, Tout>::St;
  const int cw = col_width(B);
  const int segi = seg_index(cw);
  const int64_t ncb = (B + cw - 1) / cw;
  const int32_t* order = d.scan_order[dir > 0 ? 0 : 1][segi];
  if (!order) return hipErrorInvalidValue;
  St* Val = (St*)aux;
  // sync words: [0] unused, [1] error, [2..] one flag per (tile, column block)
  const int64_t nsync = 2 + ntiles * ncb;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((nsync + WG - 1) / WG)), dim3(WG), 0, s, sync, nsync, 0);
  const dim3 g((unsigned)(ntiles * ncb));
  if (cw == 64)
    hipLaunchKernelGGL((k_scan_onepass<Tin, Tout, 64>), g, dim3(WG), 0, s, d, segi, cw, dir, (const Tin*)x, ldx, B,
                       ntiles, order, Val, sync + 2, sync + 1, spin_limit, (Tout*)P);
  else
    hipLaunchKernelGGL((k_scan_onepass<Tin, Tout, 0>), g, dim3(WG), 0, s, d, segi, cw, dir, (const Tin*)x, ldx, B,
                       ntiles, order, Val, sync + 2, sync + 1, spin_limit, (Tout*)P);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_chain_scan_onepass(const DevPoset& d, int dir, ElemType tin, const void* x, int64_t ldx,
                                     ElemType tout, void* P, int64_t B, void* aux, int64_t ntiles, int* sync,
                                     int spin_limit, hipStream_t s) {
  if (d.n == 0 || ntiles == 0) return hipSuccess;
  if (tin == E_I64 && tout == E_I64) return onepass_typed<int64_t, int64_t>(d, dir, x, ldx, P, B, aux, ntiles, sync, spin_limit, s);
  if (tin == E_F32 && tout == E_F32) return onepass_typed<float, float>(d, dir, x, ldx, P, B, aux, ntiles, sync, spin_limit, s);
  if (tin == E_F64 && tout == E_F64) return onepass_typed<double, double>(d, dir, x, ldx, P, B, aux, ntiles, sync, spin_limit, s);
  if (tin == E_F32 && tout == E_F64) return onepass_typed<float, double>(d, dir, x, ldx, P, B, aux, ntiles, sync, spin_limit, s);
  return hipErrorInvalidValue;
}

hipError_t launch_chain_scan_phase(int phase, const DevPoset& d, int dir, ElemType tin, const void* x, int64_t ldx,
                                   ElemType tout, void* P, int64_t B, void* aux, int64_t ntiles, hipStream_t s) {
  if (d.n == 0 || ntiles == 0) return hipSuccess;
  if (tin == E_I64 && tout == E_I64) return scan_typed<int64_t, int64_t>(phase, d, dir, x, ldx, P, B, aux, ntiles, s);
  if (tin == E_F32 && tout == E_F32) return scan_typed<float, float>(phase, d, dir, x, ldx, P, B, aux, ntiles, s);
  if (tin == E_F64 && tout == E_F64) return scan_typed<double, double>(phase, d, dir, x, ldx, P, B, aux, ntiles, s);
  if (tin == E_F32 && tout == E_F64) return scan_typed<float, double>(phase, d, dir, x, ldx, P, B, aux, ntiles, s);
  return hipErrorInvalidValue;
}

bool compact_ok(const DevPoset& d, bool up, int64_t B) {
  const WalkTables& w = d.walk[up ? 1 : 0];
  return d.n > 0 && B >= 1 && !d.poset_of_row && d.k <= 64 && w.runs && w.tmask && w.qoff && w.init &&
         w.snap_of_row;
}

hipError_t launch_zeta_compact(const DevPoset& d, int dir, ElemType tin, const void* x, int64_t ldx, ElemType tout,
                               void* out, int64_t ldo, ElemType tres, const void* resid, int64_t ldr, int64_t B,
                               void* aux, int64_t ntiles, void* lq, void* snaps, LaunchHook* hook, hipStream_t s) {
  if (!compact_ok(d, dir < 0, B) || ntiles != d.walk[dir > 0 ? 0 : 1].qoff_tiles) return hipErrorInvalidValue;
  if (!resid) {
    if (tin != tout) return hipErrorInvalidValue;
    if (tin == E_I64)
      return compact_typed<int64_t, int64_t, 1, int64_t>(d, dir, x, ldx, out, ldo, nullptr, 0, B, aux, ntiles, lq,
                                                         snaps, hook, s);
    if (tin == E_F32)
      return compact_typed<float, float, 1, float>(d, dir, x, ldx, out, ldo, nullptr, 0, B, aux, ntiles, lq, snaps,
                                                   hook, s);
    if (tin == E_F64)
      return compact_typed<double, double, 1, double>(d, dir, x, ldx, out, ldo, nullptr, 0, B, aux, ntiles, lq,
                                                      snaps, hook, s);
    return hipErrorInvalidValue;
  }
  if (tin != E_F32 || tout != E_F64) return hipErrorInvalidValue;
  if (tres == E_F32)
    return compact_typed<float, double, 2, float>(d, dir, x, ldx, out, ldo, resid, ldr, B, aux, ntiles, lq, snaps,
                                                  hook, s);
  if (tres == E_F64)
    return compact_typed<float, double, 2, double>(d, dir, x, ldx, out, ldo, resid, ldr, B, aux, ntiles, lq, snaps,
                                                   hook, s);
  return hipErrorInvalidValue;
}

namespace {
hipError_t gather_csr(const DevPoset& d, const int64_t* ep, const int32_t* er, const int32_t* rows, int64_t nrows,
                      ElemType tp, const void* P, int64_t B, ElemType tout, void* out, int64_t ldo, ElemType tres,
                      const void* resid, int64_t ldr, hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  const int cw = col_width(B);
  const dim3 g = grid2(nrows, cw, B);
  if (resid && tres == E_F32)
    hipLaunchKernelGGL((k_gather_csr<double, double, float, true>), g, dim3(WG), 0, s, d, ep, er, rows, nrows, cw,
                       (const double*)P, B, (double*)out, ldo, (const float*)resid, ldr);
  else if (resid && tres == E_F64)
    hipLaunchKernelGGL((k_gather_csr<double, double, double, true>), g, dim3(WG), 0, s, d, ep, er, rows, nrows, cw,
                       (const double*)P, B, (double*)out, ldo, (const double*)resid, ldr);
  else if (resid)
    return hipErrorInvalidValue;
  else if (tp == E_I64 && tout == E_I64)
    hipLaunchKernelGGL((k_gather_csr<int64_t, int64_t, int64_t, false>), g, dim3(WG), 0, s, d, ep, er, rows, nrows,
                       cw, (const int64_t*)P, B, (int64_t*)out, ldo, (const int64_t*)nullptr, 0);
  else if (tp == E_F32 && tout == E_F32)
    hipLaunchKernelGGL((k_gather_csr<float, float, float, false>), g, dim3(WG), 0, s, d, ep, er, rows, nrows, cw,
                       (const float*)P, B, (float*)out, ldo, (const float*)nullptr, 0);
  else if (tp == E_F64 && tout == E_F64)
    hipLaunchKernelGGL((k_gather_csr<double, double, double, false>), g, dim3(WG), 0, s, d, ep, er, rows, nrows, cw,
                       (const double*)P, B, (double*)out, ldo, (const double*)nullptr, 0);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// The long rows of the sparse gather: chunk sums, then each row's total.
template <typename TP, typename Tout, typename Tres, bool RESID>
hipError_t gather_split_typed(const DevPoset& d, int m, const void* P, int64_t B, void* out, int64_t ldo,
                              const void* resid, int64_t ldr, void* part, hipStream_t s) {
  using W = typename Wide<TP>::W;
  const int cw = col_width(B);
  const GatherSplit& gs = d.gsplit[m];
  const int4* items = sizeof(TP) == 8 && gs.items8 ? gs.items8 : gs.items;
  hipLaunchKernelGGL((k_csr_part<TP, false>), grid2(gs.nitems, cw, B), dim3(WG), 0, s, d, items, gs.nitems, cw,
                     d.nivr[m], (const TP*)P, B, (W*)part);
  hipLaunchKernelGGL((k_gather_csr_fin<TP, Tout, Tres, RESID>), grid2(gs.nlongs, cw, B), dim3(WG), 0, s, d,
                     gs.longs, gs.nlongs, cw, (const W*)part, B, (Tout*)out, ldo, (const Tres*)resid, ldr);
  return hipGetLastError();
}

hipError_t gather_split(const DevPoset& d, int m, ElemType tp, const void* P, int64_t B, ElemType tout, void* out,
                        int64_t ldo, ElemType tres, const void* resid, int64_t ldr, void* part, hipStream_t s) {
  if (d.gsplit[m].nlongs == 0) return hipSuccess;
  if (resid && tres == E_F32)
    return gather_split_typed<double, double, float, true>(d, m, P, B, out, ldo, resid, ldr, part, s);
  if (resid && tres == E_F64)
    return gather_split_typed<double, double, double, true>(d, m, P, B, out, ldo, resid, ldr, part, s);
  if (resid) return hipErrorInvalidValue;
  if (tp == E_I64 && tout == E_I64)
    return gather_split_typed<int64_t, int64_t, int64_t, false>(d, m, P, B, out, ldo, nullptr, 0, part, s);
  if (tp == E_F32 && tout == E_F32)
    return gather_split_typed<float, float, float, false>(d, m, P, B, out, ldo, nullptr, 0, part, s);
  if (tp == E_F64 && tout == E_F64)
    return gather_split_typed<double, double, double, false>(d, m, P, B, out, ldo, nullptr, 0, part, s);
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_gather(const DevPoset& d, bool up, ElemType tp, const void* P, int64_t B, ElemType tout,
                         void* out, int64_t ldo, ElemType tres, const void* resid, int64_t ldr, void* snaps,
                         LaunchHook* hook, hipStream_t s) {
  if (d.n == 0) return hipSuccess;
  const int cw = col_width(B);
  const dim3 g = grid2(d.n, cw, B);
  const int32_t* nv = up ? d.niv_up : d.niv;
  if (resid && (tp != E_F64 || tout != E_F64)) return hipErrorInvalidValue;
  if (const int64_t* ep = d.nivp[up ? 1 : 0]) {  // sparse niv rows
    const int m = up ? 1 : 0;
    const int32_t* er = d.nivr[m];
    const GatherSplit& gs = d.gsplit[m];
    if (!gs.shorts || !snaps) return gather_csr(d, ep, er, nullptr, d.n, tp, P, B, tout, out, ldo, tres, resid, ldr, s);
    // short rows whole, long rows in chunks (snaps: the chunk sums)
    hipError_t e = gather_csr(d, ep, er, gs.shorts, gs.nshorts, tp, P, B, tout, out, ldo, tres, resid, ldr, s);
    if (e == hipSuccess) e = gather_split(d, m, tp, P, B, tout, out, ldo, tres, resid, ldr, snaps, s);
    return e;
  }
  // the walking gather when its tables and snapshot scratch are there
  const WalkTables& w = d.walk[up ? 1 : 0];
  if (w.runs && snaps && tp == tout && (B <= 64 || (!d.poset_of_row && d.k <= 64))) {
    if (tp == E_F32) return walk_typed<float>(d, nv, w, P, B, out, ldo, tres, resid, ldr, snaps, hook, s);
    if (tp == E_F64) return walk_typed<double>(d, nv, w, P, B, out, ldo, tres, resid, ldr, snaps, hook, s);
    if (tp == E_I64) return walk_typed<int64_t>(d, nv, w, P, B, out, ldo, tres, resid, ldr, snaps, hook, s);
    return hipErrorInvalidValue;
  }
  // otherwise one thread per (row, column) over all k niv entries
  if (resid) {
    if (tres == E_F32)
      hipLaunchKernelGGL((k_gather<double, double, float, true>), g, dim3(WG), 0, s, d, nv, cw, (const double*)P, B,
                         (double*)out, ldo, (const float*)resid, ldr);
    else if (tres == E_F64)
      hipLaunchKernelGGL((k_gather<double, double, double, true>), g, dim3(WG), 0, s, d, nv, cw, (const double*)P,
                         B, (double*)out, ldo, (const double*)resid, ldr);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (d.poset_of_row) {
    if (tp == E_F32 && tout == E_F32)
      hipLaunchKernelGGL((k_gather_batched<float, float>), g, dim3(WG), 0, s, d, nv, cw, (const float*)P, B,
                         (float*)out, ldo);
    else if (tp == E_F64 && tout == E_F64)
      hipLaunchKernelGGL((k_gather_batched<double, double>), g, dim3(WG), 0, s, d, nv, cw, (const double*)P, B,
                         (double*)out, ldo);
    else if (tp == E_I64 && tout == E_I64)
      hipLaunchKernelGGL((k_gather_batched<int64_t, int64_t>), g, dim3(WG), 0, s, d, nv, cw, (const int64_t*)P,
                         B, (int64_t*)out, ldo);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (tp == E_I64 && tout == E_I64)
    hipLaunchKernelGGL((k_gather<int64_t, int64_t, int64_t, false>), g, dim3(WG), 0, s, d, nv, cw,
                       (const int64_t*)P, B, (int64_t*)out, ldo, (const int64_t*)nullptr, 0);
  else if (tp == E_F32 && tout == E_F32)
    hipLaunchKernelGGL((k_gather<float, float, float, false>), g, dim3(WG), 0, s, d, nv, cw, (const float*)P, B,
                       (float*)out, ldo, (const float*)nullptr, 0);
  else if (tp == E_F64 && tout == E_F64)
    hipLaunchKernelGGL((k_gather<double, double, double, false>), g, dim3(WG), 0, s, d, nv, cw, (const double*)P,
                       B, (double*)out, ldo, (const double*)nullptr, 0);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_usolve_begin(const DevPoset& d, ElemType ty, void* Y, int64_t B, hipStream_t s) {
  const int64_t words = B * (ty == E_F32 ? 1 : 2);
  hipLaunchKernelGGL(k_zero_bytes, dim3((unsigned)((words + WG - 1) / WG)), dim3(WG), 0, s,
                     (uint32_t*)((char*)Y + (int64_t)d.n * B * (ty == E_F32 ? 4 : 8)), words);
  return hipGetLastError();
}

namespace {
hipError_t usolve_csr(const DevPoset& d, const int64_t* ep, const int32_t* er, const int32_t* rows, int64_t cnt,
                            ElemType tin, const void* g, int64_t ldg, ElemType ty, void* Y, int64_t B,
                            hipStream_t s) {
  const int cw = col_width(B);
  const dim3 gr = grid2(cnt, cw, B);
  if (tin == E_I64 && ty == E_I64)
    hipLaunchKernelGGL((k_usolve_csr<int64_t, int64_t>), gr, dim3(WG), 0, s, d, ep, er, rows, cnt, cw,
                       (const int64_t*)g, ldg, (int64_t*)Y, B);
  else if (tin == E_F32 && ty == E_F32)
    hipLaunchKernelGGL((k_usolve_csr<float, float>), gr, dim3(WG), 0, s, d, ep, er, rows, cnt, cw,
                       (const float*)g, ldg, (float*)Y, B);
  else if (tin == E_F64 && ty == E_F32)
    hipLaunchKernelGGL((k_usolve_csr<double, float>), gr, dim3(WG), 0, s, d, ep, er, rows, cnt, cw,
                       (const double*)g, ldg, (float*)Y, B);
  else if (tin == E_F64 && ty == E_F64)
    hipLaunchKernelGGL((k_usolve_csr<double, double>), gr, dim3(WG), 0, s, d, ep, er, rows, cnt, cw,
                       (const double*)g, ldg, (double*)Y, B);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
}  // namespace

namespace {
template <typename Tin, typename TY>
hipError_t usolve_split_typed(const DevPoset& d, const int32_t* er, const int4* items, int64_t nitems,
                              const int4* longs, int64_t nlongs, const void* g, int64_t ldg, void* Y, int64_t B,
                              void* part, hipStream_t s) {
  using W = typename Wide<TY>::W;
  const int cw = col_width(B);
  hipLaunchKernelGGL((k_csr_part<TY, true>), grid2(nitems, cw, B), dim3(WG), 0, s, d, items, nitems, cw, er,
                     (const TY*)Y, B, (W*)part);
  hipLaunchKernelGGL((k_usolve_csr_fin<Tin, TY>), grid2(nlongs, cw, B), dim3(WG), 0, s, d, longs, nlongs, cw,
                     (const Tin*)g, ldg, (const W*)part, (TY*)Y, B);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_usolve_split(const DevPoset& d, bool up, const int4* items, int64_t nitems, const int4* longs,
                               int64_t nlongs, ElemType tin, const void* g, int64_t ldg, ElemType ty, void* Y,
                               int64_t B, void* part, hipStream_t s) {
  if (nlongs == 0) return hipSuccess;
  const int32_t* er = d.nivr[up ? 1 : 0];
  if (!er) return hipErrorInvalidValue;
  if (tin == E_I64 && ty == E_I64)
    return usolve_split_typed<int64_t, int64_t>(d, er, items, nitems, longs, nlongs, g, ldg, Y, B, part, s);
  if (tin == E_F32 && ty == E_F32)
    return usolve_split_typed<float, float>(d, er, items, nitems, longs, nlongs, g, ldg, Y, B, part, s);
  if (tin == E_F64 && ty == E_F32)
    return usolve_split_typed<double, float>(d, er, items, nitems, longs, nlongs, g, ldg, Y, B, part, s);
  if (tin == E_F64 && ty == E_F64)
    return usolve_split_typed<double, double>(d, er, items, nitems, longs, nlongs, g, ldg, Y, B, part, s);
  return hipErrorInvalidValue;
}

hipError_t launch_usolve_runs(const DevPoset& d, bool up, const int4* chunks, int64_t nchunks, const void* g,
                              int64_t ldg, void* Y, int64_t B, hipStream_t s) {
  if (nchunks == 0) return hipSuccess;
  const int32_t* nv = up ? d.niv_up : d.niv;
  const SegTables& t = d.seg[up ? 1 : 0];
  if (!nv || !t.ev || nchunks > INT32_MAX) return hipErrorInvalidValue;
  const int cw = col_width(B);
  const dim3 gr((unsigned)nchunks, (unsigned)((B + cw - 1) / cw));
  const int64_t* gi = (const int64_t*)g;
  int64_t* Yi = (int64_t*)Y;
  switch (cw) {
    case 64: hipLaunchKernelGGL((k_usolve_seg<int64_t, 64>), gr, dim3(WG), 0, s, d, nv, chunks, t.ev, gi, ldg, Yi, B); break;
    case 32: hipLaunchKernelGGL((k_usolve_seg<int64_t, 32>), gr, dim3(WG), 0, s, d, nv, chunks, t.ev, gi, ldg, Yi, B); break;
    case 16: hipLaunchKernelGGL((k_usolve_seg<int64_t, 16>), gr, dim3(WG), 0, s, d, nv, chunks, t.ev, gi, ldg, Yi, B); break;
    case 8: hipLaunchKernelGGL((k_usolve_seg<int64_t, 8>), gr, dim3(WG), 0, s, d, nv, chunks, t.ev, gi, ldg, Yi, B); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

namespace {
// Workgroups of k_usolve_flow<TY, CW> the device holds resident at once.
template <int CW, int WAIT>
int flow_resident() {
  static std::atomic<int> cached[64];  // per device; builds may run on several threads
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (int c = cached[dev].load(std::memory_order_relaxed); c > 0) return c;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_usolve_flow<int64_t, CW, WAIT>, WG, 0) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  const int r = std::max(1, per_cu) * std::max(1, cus);
  cached[dev].store(r, std::memory_order_relaxed);
  return r;
}

template <int CW, int WAIT>
hipError_t flow_typed(const DevPoset& d, const int32_t* nv, const int4* chunks, int nchunks, const int32_t* lev_off,
                      const int32_t* dep_ptr, const int32_t* deps, const int4* ev, const int64_t* g, int64_t ldg,
                      int64_t* Y, int64_t B, int* flags, int* err, int spin_limit, int64_t total, int max_grid,
                      hipStream_t s) {
  const int res = flow_resident<CW, WAIT>();
  if (res <= 0) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)std::min<int64_t>(std::min<int64_t>(total, res), max_grid > 0 ? max_grid : res);
  hipLaunchKernelGGL((k_usolve_flow<int64_t, CW, WAIT>), dim3(grid), dim3(WG), 0, s, d, nv, chunks, nchunks, lev_off,
                     dep_ptr, deps, ev, g, ldg, Y, B, flags, err, spin_limit);
  return hipGetLastError();
}

template <int CW>
hipError_t flow_wait(int wait, const DevPoset& d, const int32_t* nv, const int4* chunks, int nchunks,
                     const int32_t* lev_off, const int32_t* dep_ptr, const int32_t* deps, const int4* ev,
                     const int64_t* g, int64_t ldg, int64_t* Y, int64_t B, int* flags, int* err, int spin_limit,
                     int64_t total, int max_grid, hipStream_t s) {
  switch (wait) {
    case kWaitRows:
      return flow_typed<CW, kWaitRows>(d, nv, chunks, nchunks, lev_off, dep_ptr, deps, ev, g, ldg, Y, B, flags, err,
                                       spin_limit, total, max_grid, s);
    case kWaitLevel:
      return flow_typed<CW, kWaitLevel>(d, nv, chunks, nchunks, lev_off, dep_ptr, deps, ev, g, ldg, Y, B, flags, err,
                                        spin_limit, total, max_grid, s);
    case kWaitDeps:
      return flow_typed<CW, kWaitDeps>(d, nv, chunks, nchunks, lev_off, dep_ptr, deps, ev, g, ldg, Y, B, flags, err,
                                       spin_limit, total, max_grid, s);
    default:
      return flow_typed<CW, kWaitValues>(d, nv, chunks, nchunks, lev_off, dep_ptr, deps, ev, g, ldg, Y, B, flags, err,
                                         spin_limit, total, max_grid, s);
  }
}
}  // namespace

hipError_t launch_usolve_flow(const DevPoset& d, bool up, const int4* chunks, int64_t nchunks, const int32_t* lev_off,
                              const int32_t* dep_ptr, const int32_t* deps, int wait, const void* g, int64_t ldg, void* Y,
                              int64_t B, int* sync, int spin_limit, int max_grid, hipStream_t s) {
  if (nchunks == 0) return hipSuccess;
  const int32_t* nv = up ? d.niv_up : d.niv;
  const SegTables& t = d.seg[up ? 1 : 0];
  const int cw = flow_col_width(B);
  const int64_t ncb = (B + cw - 1) / cw;
  if (!nv || !t.ev || !lev_off || (wait == kWaitDeps && (!dep_ptr || !deps)) || nchunks * ncb >= INT32_MAX ||
      (int64_t)d.n + 1 >= INT32_MAX || cw < 8 || wait < kWaitRows || wait > kWaitValues)
    return hipErrorInvalidValue;
  int* err = sync;
  int* flags = sync + 1;
  const bool chunk_flags = wait == kWaitLevel || wait == kWaitDeps;
  const int64_t nsync = 1 + ncb * (chunk_flags ? nchunks : (int64_t)d.n + 1);
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((nsync + WG - 1) / WG)), dim3(WG), 0, s, sync, nsync, 0);
  if (wait == kWaitValues) {  // rows 0 .. n-1 of Y unwritten (row n, the zero row, stays 0)
    const int64_t words = (int64_t)d.n * B;
    hipLaunchKernelGGL(k_fill_i64x2, dim3((unsigned)((words + 2 * WG - 1) / (2 * WG))), dim3(WG), 0, s, (int64_t*)Y,
                       words, kUnwritten);
  }
  const int nc = (int)nchunks;
  const int64_t* gi = (const int64_t*)g;
  int64_t* Yi = (int64_t*)Y;
  const int64_t tot = nchunks * ncb;
  hipError_t e;
  switch (cw) {
    case 64: e = flow_wait<64>(wait, d, nv, chunks, nc, lev_off, dep_ptr, deps, t.ev, gi, ldg, Yi, B, flags, err, spin_limit, tot, max_grid, s); break;
    case 32: e = flow_wait<32>(wait, d, nv, chunks, nc, lev_off, dep_ptr, deps, t.ev, gi, ldg, Yi, B, flags, err, spin_limit, tot, max_grid, s); break;
    case 16: e = flow_wait<16>(wait, d, nv, chunks, nc, lev_off, dep_ptr, deps, t.ev, gi, ldg, Yi, B, flags, err, spin_limit, tot, max_grid, s); break;
    case 8: e = flow_wait<8>(wait, d, nv, chunks, nc, lev_off, dep_ptr, deps, t.ev, gi, ldg, Yi, B, flags, err, spin_limit, tot, max_grid, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_usolve_flow_fix<int64_t>), dim3(1), dim3(WG), 0, s, d, nv, chunks, nc, gi, ldg, Yi, B,
                     (const int*)err);
  return hipGetLastError();
}

// ------------------------------------------- row-by-row solve in one launch

// Bit pattern of an unwritten value of Y in the value-polling row solve: the
// int64 minimum, and signalling NaNs with a payload for float32 and float64
// (arithmetic returns quiet NaNs).  A legitimate value equal to the mark is
// handled through the row's ready flag.
template <typename T> struct PollMark;
template <> struct PollMark<int64_t> { using U = uint64_t; static constexpr U bits = 0x8000000000000000ull; };
template <> struct PollMark<double> { using U = uint64_t; static constexpr U bits = 0x7FF4A5A5A5A5A5A5ull; };
template <> struct PollMark<float> { using U = uint32_t; static constexpr U bits = 0x7FA5A5A5u; };

template <typename T>
__device__ inline typename PollMark<T>::U ld_bits(const T* p) {
  using U = typename PollMark<T>::U;
  return __hip_atomic_load(reinterpret_cast<const U*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ inline void st_bits(T* p, T v) {
  using U = typename PollMark<T>::U;
  U w;
  __builtin_memcpy(&w, &v, sizeof(U));
  __hip_atomic_store(reinterpret_cast<U*>(p), w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One wavefront, one row: lane j < KB holds entry j of a batch (-1: none or
// the own chain).  Reads Y at those rows, column colc of each lane, into v,
// until no value is the mark.  A round reads all KB entries (unconditional
// loads, all in flight together; a written value never changes, so settled
// entries just read the same word).  While some entry is still marked, the
// wavefront polls only the lowest such entry (one load per poll, so waiting
// wavefronts add little traffic) and reads all again once it has been
// written.  With FLAGS (int64, whose results can equal the mark) every fourth
// poll also reads that row's ready flag; once the flag reads as set, the next
// round's read of it (issued after the flag arrived) is taken as it is.
// Without FLAGS (floating point: arithmetic never yields the signalling-NaN
// mark) a wait for such a value would end at the spin limit and the fallback.
// Exits are wave-uniform; false when it gives up.
template <typename TY, int KB, bool FLAGS, bool O32>
__device__ inline bool poll_row(const TY* __restrict__ Y, int64_t B, int64_t colc, int zr, int cur, TY (&v)[KB],
                                const int* __restrict__ fl, const int* __restrict__ err, int spin_limit) {
  using U = typename PollMark<TY>::U;
  // O32: Y spans less than 4 GiB, so each load is Y plus a 32-bit byte offset
  auto at = [&](int t) -> const TY* {
    if (O32)
      return reinterpret_cast<const TY*>(reinterpret_cast<const char*>(Y) +
                                         (uint32_t)(((uint32_t)t * (uint32_t)B + (uint32_t)colc) * sizeof(TY)));
    return Y + (int64_t)t * B + colc;
  };
  U b[KB];
  uint64_t seen = 0;
  int spin = 0;
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  for (;;) {
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int t = __builtin_amdgcn_readlane(cur, j);
      b[j] = ld_bits(at(t >= 0 ? t : zr));
    }
    uint64_t pend = 0;  // wave-uniform: entries still marked in some lane
#pragma unroll
    for (int j = 0; j < KB; ++j)
      if (__any(b[j] == PollMark<TY>::bits) && !((seen >> j) & 1) && __builtin_amdgcn_readlane(cur, j) >= 0)
        pend |= 1ull << j;
    if (pend == 0) break;
    const int js = __builtin_amdgcn_readfirstlane(__builtin_ctzll(pend));
    const int ts = __builtin_amdgcn_readlane(cur, js);
    for (int poll = 0;; ++poll, ++spin) {
      if (spin >= spin_limit) return false;
      if ((spin & 15) == 15) {
        if (__builtin_amdgcn_readfirstlane(__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0)
          return false;
        if (__builtin_amdgcn_s_memrealtime() - t0 > kFlowWaitTicks) return false;
      }
      __builtin_amdgcn_s_sleep(2);
      if (FLAGS && (poll & 3) == 3) {
        const int f = __hip_atomic_load(fl + ts, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wait_vmem();  // the flag has arrived before the next round's reads are issued
        if (__builtin_amdgcn_readfirstlane(f) != 0) {
          seen |= 1ull << js;
          break;
        }
      }
      if (!__any(ld_bits(at(ts)) == PollMark<TY>::bits)) break;
    }
  }
#pragma unroll
  for (int j = 0; j < KB; ++j) __builtin_memcpy(&v[j], &b[j], sizeof(U));
  return true;
}

// The row-by-row level solve (k_usolve_uni's sums: g minus one entry at a time
// in chain order, the own and missing entries reading the zero row n) for all
// levels in one launch.  Each wavefront takes the items gw, gw + W, ... (gw its
// index over the grid, W the wavefronts of the grid) of the level-ordered list
// of (row, 64-column block) items; it reads the Y rows it needs by polling
// their values (rows 0 .. n-1 of Y hold the mark until written), stores its
// row's values and (int64) once they have completed sets the row's ready flag.  A row
// reads only rows of lower levels, which come earlier in the list; a
// wavefront takes its items in order, so with every wavefront resident the
// unfinished item of lowest index has all it reads and every wait ends.  One
// row per wavefront: a wavefront never holds a row and one of its readers.
// Waits are bounded; a wavefront that gives up stores the error word and
// stops, and k_usolve_poll_fix then solves again level by level.  Results
// equal the per-level kernels' bit for bit.
template <typename Tin, typename TY, bool O32>
__global__ __launch_bounds__(WG) void k_usolve_poll(DevPoset d, const int32_t* __restrict__ nv,
                                                    const int32_t* __restrict__ rows, const int32_t* __restrict__ lnv,
                                                    const int32_t* __restrict__ lnode, int cnt,
                                                    const Tin* __restrict__ g, int64_t ldg, TY* __restrict__ Y,
                                                    int64_t B, int* __restrict__ flags, int* __restrict__ err,
                                                    int spin_limit) {
  using W = typename Wide<TY>::W;
  constexpr bool FLAGS = std::is_same<TY, int64_t>::value;  // integer results can equal the mark
  constexpr int KB = sizeof(TY) == 4 ? 64 : 32;               // entries per batch (registers in flight)
  const int lane = threadIdx.x & 63;
  const int ncb = (int)((B + 63) / 64);
  const int64_t total = (int64_t)cnt * ncb;
  const int64_t nw = (int64_t)gridDim.x * (WG / 64);
  const int k = d.k, zr = d.n;
  for (int64_t it = (int64_t)blockIdx.x * (WG / 64) + (threadIdx.x >> 6); it < total; it += nw) {
    const int i = __builtin_amdgcn_readfirstlane((int)(it / ncb));
    const int cb = __builtin_amdgcn_readfirstlane((int)(it - (int64_t)i * ncb));
    int* const fl = flags + (int64_t)cb * (zr + 1);
    const int64_t col = (int64_t)cb * 64 + lane;
    const bool colok = col < B;
    const int64_t colc = colok ? col : 0;
    const int r = __builtin_amdgcn_readfirstlane(rows[i]);
    const int node = __builtin_amdgcn_readfirstlane(lnode ? lnode[i] : d.node_of_row[r]);
    const int32_t* __restrict__ nr = lnv ? lnv + (int64_t)i * k : nv + (int64_t)r * k;
    W acc = (W)g[(int64_t)node * ldg + colc];
    bool ok = true;
    for (int j0 = 0; j0 < k; j0 += KB) {
      int cur = lane < KB && j0 + lane < k ? nr[j0 + lane] : -1;
      if (cur == r) cur = -1;
      TY v[KB];
      if (!poll_row<TY, KB, FLAGS, O32>(Y, B, colc, zr, cur, v, fl, err, spin_limit)) {
        ok = false;
        break;
      }
#pragma unroll
      for (int j = 0; j < KB; ++j) acc -= (W)v[j];
    }
    if (!ok) {
      if (lane == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    if (colok) st_bits(&Y[(int64_t)r * B + col], (TY)acc);
    if (FLAGS) {
      wait_vmem();
      if (lane == 0) __hip_atomic_store(&fl[r], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// The same poll for row groups of fewer than 64 lanes: every lane holds its
// row's entries t[0 .. KB) (-1: none), so rows differ across the wavefront.
// The lowest entry still marked in some lane is polled (lanes whose row has
// no such entry read the zero row); with FLAGS a lane that reads its entry's
// ready flag as set takes that entry's next read as it is.
template <typename TY, int KB, bool FLAGS, bool O32>
__device__ inline bool poll_lanes(const TY* __restrict__ Y, int64_t B, int64_t colc, int zr, const int32_t (&t)[KB],
                                  TY (&v)[KB], const int* __restrict__ fl, const int* __restrict__ err,
                                  int spin_limit) {
  using U = typename PollMark<TY>::U;
  auto at = [&](int r) -> const TY* {
    if (O32)
      return reinterpret_cast<const TY*>(reinterpret_cast<const char*>(Y) +
                                         (uint32_t)(((uint32_t)r * (uint32_t)B + (uint32_t)colc) * sizeof(TY)));
    return Y + (int64_t)r * B + colc;
  };
  U b[KB];
  uint64_t seen = 0;  // per lane
  int spin = 0;
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  for (;;) {
#pragma unroll
    for (int j = 0; j < KB; ++j) b[j] = ld_bits(at(t[j] >= 0 ? t[j] : zr));
    uint64_t pend = 0;  // wave-uniform
#pragma unroll
    for (int j = 0; j < KB; ++j)
      if (__any(b[j] == PollMark<TY>::bits && t[j] >= 0 && !((seen >> j) & 1))) pend |= 1ull << j;
    if (pend == 0) break;
    const int js = __builtin_amdgcn_readfirstlane(__builtin_ctzll(pend));
    int ts = -1;
#pragma unroll
    for (int j = 0; j < KB; ++j)
      if (j == js) ts = t[j];
    const bool mine = ts >= 0 && !((seen >> js) & 1);
    for (int poll = 0;; ++poll, ++spin) {
      if (spin >= spin_limit) return false;
      if ((spin & 15) == 15) {
        if (__builtin_amdgcn_readfirstlane(__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0)
          return false;
        if (__builtin_amdgcn_s_memrealtime() - t0 > kFlowWaitTicks) return false;
      }
      __builtin_amdgcn_s_sleep(2);
      if (FLAGS && (poll & 3) == 3) {
        const int f = __hip_atomic_load(fl + (mine ? ts : zr), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        wait_vmem();  // the flag has arrived before the next round's reads are issued
        if (mine && f != 0) seen |= 1ull << js;
        if (__any(mine && f != 0)) break;
      }
      if (!__any(mine && ld_bits(at(mine ? ts : zr)) == PollMark<TY>::bits)) break;
    }
  }
#pragma unroll
  for (int j = 0; j < KB; ++j) __builtin_memcpy(&v[j], &b[j], sizeof(U));
  return true;
}

// k_usolve_poll for narrow blocks (CW = 8, 16 or 32 columns): a wavefront
// takes 64 / CW consecutive positions of the level-ordered list at a time, one
// row per group of CW lanes, and a block of CW columns.  Rows of one
// wavefront item that lie in different levels are solved one level after the
// other (sub-batches; lev_bits marks the first position of every level), so a
// wavefront never waits on a row it holds itself.  Same sums as the per-level
// kernels.
template <typename Tin, typename TY, int CW, bool O32>
__global__ __launch_bounds__(WG) void k_usolve_poll_n(DevPoset d, const int32_t* __restrict__ nv,
                                                      const int32_t* __restrict__ rows,
                                                      const int32_t* __restrict__ lnv,
                                                      const int32_t* __restrict__ lnode,
                                                      const uint64_t* __restrict__ lev_bits, int cnt,
                                                      const Tin* __restrict__ g, int64_t ldg, TY* __restrict__ Y,
                                                      int64_t B, int* __restrict__ flags, int* __restrict__ err,
                                                      int spin_limit) {
  using W = typename Wide<TY>::W;
  constexpr bool FLAGS = std::is_same<TY, int64_t>::value;
  constexpr int KB = 32;
  constexpr int RPW = 64 / CW;  // rows per wavefront item
  const int lane = threadIdx.x % CW;
  const int rgw = (threadIdx.x & 63) / CW;
  const int ncb = (int)((B + CW - 1) / CW);
  const int64_t nwi = ((int64_t)cnt + RPW - 1) / RPW;
  const int64_t total = nwi * ncb;
  const int64_t nw = (int64_t)gridDim.x * (WG / 64);
  const int k = d.k, zr = d.n;
  for (int64_t it = (int64_t)blockIdx.x * (WG / 64) + (threadIdx.x >> 6); it < total; it += nw) {
    const int wi = __builtin_amdgcn_readfirstlane((int)(it / ncb));
    const int cb = __builtin_amdgcn_readfirstlane((int)(it - (int64_t)wi * ncb));
    const int p0 = wi * RPW;  // a multiple of RPW: the item's positions share one 64-bit word of lev_bits
    const int pos = p0 + rgw;
    const bool act = pos < cnt;
    int* const fl = flags + (int64_t)cb * (zr + 1);
    const int64_t col = (int64_t)cb * CW + lane;
    const bool colok = col < B;
    const int64_t colc = colok ? col : 0;
    // level of each position relative to the item's first: the level starts in (p0, pos]
    const uint64_t word = lev_bits[p0 >> 6];
    const int sh = p0 & 63;
    const uint64_t within = RPW == 64 ? word : (word >> sh) & ((1ull << RPW) - 1);
    const int sub = __builtin_popcountll(within & ((2ull << rgw) - 1) & ~1ull);
    const int nsub = __builtin_popcountll(within & ~1ull);
    const int r = act ? rows[pos] : 0;
    const int node = act ? (lnode ? lnode[pos] : d.node_of_row[r]) : 0;
    const int32_t* __restrict__ nr = lnv ? lnv + (int64_t)(act ? pos : 0) * k : nv + (int64_t)r * k;
    W acc = act ? (W)g[(int64_t)node * ldg + colc] : W(0);
    for (int sb = 0; sb <= nsub; ++sb) {
      if (!act || sub != sb) continue;
      bool ok = true;
      for (int j0 = 0; j0 < k; j0 += KB) {
        int32_t t[KB];
#pragma unroll
        for (int u = 0; u < KB; ++u) {
          const int e = j0 + u < k ? nr[j0 + u] : -1;
          t[u] = e != r ? e : -1;
        }
        TY v[KB];
        if (!poll_lanes<TY, KB, FLAGS, O32>(Y, B, colc, zr, t, v, fl, err, spin_limit)) {
          ok = false;
          break;
        }
#pragma unroll
        for (int u = 0; u < KB; ++u) acc -= (W)v[u];
      }
      if (!ok) {
        if (lane == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
      }
      if (colok) st_bits(&Y[(int64_t)r * B + col], (TY)acc);
      if (FLAGS || nsub > 0) wait_vmem();  // (the next sub-batch may read these rows)
      if (FLAGS && lane == 0) __hip_atomic_store(&fl[r], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Fallback of k_usolve_poll: when its error word is set, one workgroup solves
// again, level after level with a barrier in between, a row per wavefront with
// the same sums; otherwise it returns at once.  Reads and writes are
// device-scope, so nothing stale from the persistent launch is seen.
template <typename Tin, typename TY>
__global__ __launch_bounds__(WG) void k_usolve_poll_fix(DevPoset d, const int32_t* __restrict__ nv,
                                                        const int32_t* __restrict__ rows,
                                                        const int32_t* __restrict__ lev_ptr, int nlev,
                                                        const Tin* __restrict__ g, int64_t ldg, TY* __restrict__ Y,
                                                        int64_t B, const int* __restrict__ err) {
  using W = typename Wide<TY>::W;
  if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int k = d.k, zr = d.n;
  for (int l = 0; l < nlev; ++l) {
    const int a = lev_ptr[l], b = lev_ptr[l + 1];
    for (int i = a + wv; i < b; i += WG / 64) {
      const int r = __builtin_amdgcn_readfirstlane(rows[i]);
      const int node = __builtin_amdgcn_readfirstlane(d.node_of_row[r]);
      for (int64_t c0 = 0; c0 < B; c0 += 64) {
        const int64_t col = c0 + lane;
        const bool colok = col < B;
        const int64_t colc = colok ? col : 0;
        W acc = (W)g[(int64_t)node * ldg + colc];
        for (int j0 = 0; j0 < k; j0 += 64) {  // 64 entries in flight at a time
          int cur = j0 + lane < k ? nv[(int64_t)r * k + j0 + lane] : -1;
          if (cur == r) cur = -1;
          typename PollMark<TY>::U w[64];
#pragma unroll
          for (int j = 0; j < 64; ++j) {
            const int t = __builtin_amdgcn_readlane(cur, j);
            w[j] = ld_bits(Y + (int64_t)(t >= 0 ? t : zr) * B + colc);
          }
#pragma unroll
          for (int j = 0; j < 64; ++j) {
            TY v;
            __builtin_memcpy(&v, &w[j], sizeof(v));
            acc -= (W)v;
          }
        }
        if (colok) st_bits(&Y[(int64_t)r * B + col], (TY)acc);
      }
    }
    wait_vmem();
    __syncthreads();
  }
}

namespace {
// Columns per row group of the persistent row solve: 64 (one row per
// wavefront) for B > 32, else 8, 16 or 32 (several rows per wavefront).
int poll_col_width(int64_t B) { return std::max(8, col_width(B)); }

template <typename Tin, typename TY, int CW, bool O32>
const void* poll_kernel() {
  if constexpr (CW == 64)
    return reinterpret_cast<const void*>(&k_usolve_poll<Tin, TY, O32>);
  else
    return reinterpret_cast<const void*>(&k_usolve_poll_n<Tin, TY, CW, O32>);
}

template <typename Tin, typename TY, int CW, bool O32>
int poll_resident() {
  static std::atomic<int> cached[64];  // per device; builds may run on several threads
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (int c = cached[dev].load(std::memory_order_relaxed); c > 0) return c;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, poll_kernel<Tin, TY, CW, O32>(), WG, 0) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  const int r = std::max(1, per_cu) * std::max(1, cus);
  cached[dev].store(r, std::memory_order_relaxed);
  return r;
}

template <typename Tin, typename TY, bool O32>
int poll_resident_cw(int cw) {
  switch (cw) {
    case 64: return poll_resident<Tin, TY, 64, O32>();
    case 32: return poll_resident<Tin, TY, 32, O32>();
    case 16: return poll_resident<Tin, TY, 16, O32>();
    default: return poll_resident<Tin, TY, 8, O32>();
  }
}

template <typename Tin, typename TY, bool O32>
void poll_launch(int cw, unsigned grid, hipStream_t s, const DevPoset& d, const int32_t* nv, const int32_t* rows,
                 const int32_t* lnv, const int32_t* lnode, const uint64_t* lev_bits, int cnt, const void* g,
                 int64_t ldg, void* Y, int64_t B, int* sync, int spin_limit) {
  const Tin* gt = (const Tin*)g;
  TY* Yt = (TY*)Y;
  switch (cw) {
    case 64:
      hipLaunchKernelGGL((k_usolve_poll<Tin, TY, O32>), dim3(grid), dim3(WG), 0, s, d, nv, rows, lnv, lnode, cnt, gt,
                         ldg, Yt, B, sync + 1, sync, spin_limit);
      break;
    case 32:
      hipLaunchKernelGGL((k_usolve_poll_n<Tin, TY, 32, O32>), dim3(grid), dim3(WG), 0, s, d, nv, rows, lnv, lnode,
                         lev_bits, cnt, gt, ldg, Yt, B, sync + 1, sync, spin_limit);
      break;
    case 16:
      hipLaunchKernelGGL((k_usolve_poll_n<Tin, TY, 16, O32>), dim3(grid), dim3(WG), 0, s, d, nv, rows, lnv, lnode,
                         lev_bits, cnt, gt, ldg, Yt, B, sync + 1, sync, spin_limit);
      break;
    default:
      hipLaunchKernelGGL((k_usolve_poll_n<Tin, TY, 8, O32>), dim3(grid), dim3(WG), 0, s, d, nv, rows, lnv, lnode,
                         lev_bits, cnt, gt, ldg, Yt, B, sync + 1, sync, spin_limit);
      break;
  }
}

template <typename Tin, typename TY>
hipError_t poll_typed(const DevPoset& d, const int32_t* nv, const int32_t* rows, const int32_t* lnv,
                      const int32_t* lnode, const uint64_t* lev_bits, const int32_t* lev_ptr, int nlev, int cnt,
                      const void* g, int64_t ldg, void* Y, int64_t B, int* sync, int spin_limit, int max_grid,
                      hipStream_t s) {
  using U = typename PollMark<TY>::U;
  const int cw = poll_col_width(B);
  const int64_t ncb = (B + cw - 1) / cw;
  const int64_t nsync = 1 + ncb * ((int64_t)d.n + 1);
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((nsync + WG - 1) / WG)), dim3(WG), 0, s, sync, nsync, 0);
  const int64_t words = (int64_t)d.n * B;  // rows 0 .. n-1 unwritten; row n, the zero row, stays 0
  if (sizeof(U) == 8) {
    int64_t m;
    const U bits = PollMark<TY>::bits;
    std::memcpy(&m, &bits, 8);
    hipLaunchKernelGGL(k_fill_i64x2, dim3((unsigned)((words + 2 * WG - 1) / (2 * WG))), dim3(WG), 0, s, (int64_t*)Y,
                       words, m);
  } else {
    int m;
    const U bits = PollMark<TY>::bits;
    std::memcpy(&m, &bits, 4);
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((words + WG - 1) / WG)), dim3(WG), 0, s, (int*)Y, words, m);
  }
  const bool o32 = ((int64_t)d.n + 1) * B * (int64_t)sizeof(TY) < ((int64_t)1 << 32);
  const int res = o32 ? poll_resident_cw<Tin, TY, true>(cw) : poll_resident_cw<Tin, TY, false>(cw);
  if (res <= 0) return hipErrorInvalidValue;
  const int64_t waves = ((int64_t)cnt + 64 / cw - 1) / (64 / cw) * ncb;
  const int64_t need = (waves + (WG / 64) - 1) / (WG / 64);
  const unsigned grid =
      (unsigned)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(need, res), max_grid > 0 ? max_grid : res));
  if (o32)
    poll_launch<Tin, TY, true>(cw, grid, s, d, nv, rows, lnv, lnode, lev_bits, cnt, g, ldg, Y, B, sync, spin_limit);
  else
    poll_launch<Tin, TY, false>(cw, grid, s, d, nv, rows, lnv, lnode, lev_bits, cnt, g, ldg, Y, B, sync, spin_limit);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_usolve_poll_fix<Tin, TY>), dim3(1), dim3(WG), 0, s, d, nv, rows, lev_ptr, nlev,
                     (const Tin*)g, ldg, (TY*)Y, B, (const int*)sync);
  return hipGetLastError();
}
}  // namespace

int64_t usolve_poll_ints(int64_t n, int64_t B) {
  const int cw = poll_col_width(B);
  return 1 + (B + cw - 1) / cw * (n + 1);
}

int64_t usolve_poll_waves(ElemType tin, ElemType ty, int64_t n, int64_t B) {
  const int64_t span = ((int64_t)n + 1) * B * (ty == E_F32 ? 4 : 8);
  const bool o32 = span < ((int64_t)1 << 32);
  const int cw = poll_col_width(B);
  int res = 0;
  if (tin == E_I64 && ty == E_I64)
    res = o32 ? poll_resident_cw<int64_t, int64_t, true>(cw) : poll_resident_cw<int64_t, int64_t, false>(cw);
  else if (tin == E_F32 && ty == E_F32)
    res = o32 ? poll_resident_cw<float, float, true>(cw) : poll_resident_cw<float, float, false>(cw);
  else if (tin == E_F64 && ty == E_F32)
    res = o32 ? poll_resident_cw<double, float, true>(cw) : poll_resident_cw<double, float, false>(cw);
  else if (tin == E_F64 && ty == E_F64)
    res = o32 ? poll_resident_cw<double, double, true>(cw) : poll_resident_cw<double, double, false>(cw);
  return (int64_t)res * (WG / 64);
}

int usolve_poll_rows_per_wave(int64_t B) { return 64 / poll_col_width(B); }

hipError_t launch_usolve_poll(const DevPoset& d, bool up, const int32_t* rows, const int32_t* lev_ptr,
                              const uint64_t* lev_bits, int nlev, int64_t cnt, ElemType tin, const void* g,
                              int64_t ldg, ElemType ty, void* Y, int64_t B, int* sync, int spin_limit, int max_grid,
                              hipStream_t s) {
  if (cnt == 0) return hipSuccess;
  const int32_t* nv = up ? d.niv_up : d.niv;
  if (!nv || !rows || !lev_ptr || !lev_bits || !sync || d.nivp[up ? 1 : 0] || cnt >= INT32_MAX ||
      (int64_t)d.n + 1 >= INT32_MAX || (int64_t)d.n * ((B + 7) / 8) >= INT32_MAX || d.poset_of_row)
    return hipErrorInvalidValue;
  const int32_t* lnv = d.lev_niv[up ? 1 : 0];
  const int32_t* lnode = d.lev_node[up ? 1 : 0];
  if (!lnv || !lnode) lnv = lnode = nullptr;
  const int c = (int)cnt;
  if (tin == E_I64 && ty == E_I64)
    return poll_typed<int64_t, int64_t>(d, nv, rows, lnv, lnode, lev_bits, lev_ptr, nlev, c, g, ldg, Y, B, sync,
                                        spin_limit, max_grid, s);
  if (tin == E_F32 && ty == E_F32)
    return poll_typed<float, float>(d, nv, rows, lnv, lnode, lev_bits, lev_ptr, nlev, c, g, ldg, Y, B, sync,
                                    spin_limit, max_grid, s);
  if (tin == E_F64 && ty == E_F32)
    return poll_typed<double, float>(d, nv, rows, lnv, lnode, lev_bits, lev_ptr, nlev, c, g, ldg, Y, B, sync,
                                     spin_limit, max_grid, s);
  if (tin == E_F64 && ty == E_F64)
    return poll_typed<double, double>(d, nv, rows, lnv, lnode, lev_bits, lev_ptr, nlev, c, g, ldg, Y, B, sync,
                                      spin_limit, max_grid, s);
  return hipErrorInvalidValue;
}

hipError_t launch_usolve_level(const DevPoset& d, bool up, const int32_t* lev_rows, int64_t i0, int64_t cnt,
                               ElemType tin, const void* g, int64_t ldg, ElemType ty, void* Y, int64_t B,
                               hipStream_t s) {
  if (cnt == 0) return hipSuccess;
  const int cw = col_width(B);
  const dim3 gr = grid2(cnt, cw, B);
  const int32_t* nv = up ? d.niv_up : d.niv;
  if (const int64_t* ep = d.nivp[up ? 1 : 0]) {  // sparse niv rows
    const int32_t* er = d.nivr[up ? 1 : 0];
    return usolve_csr(d, ep, er, lev_rows, cnt, tin, g, ldg, ty, Y, B, s);
  }
  if (cw == 64 && d.k <= 64 && !d.poset_of_row && cnt < INT32_MAX) {
    const dim3 gu((unsigned)((cnt + (WG / 64) - 1) / (WG / 64)), (unsigned)((B + 63) / 64));
    const int c = (int)cnt;
    const int32_t* lnv = d.lev_niv[up ? 1 : 0];
    const int32_t* lnode = d.lev_node[up ? 1 : 0];
    if (tin == E_I64 && ty == E_I64)
      hipLaunchKernelGGL((k_usolve_uni<int64_t, int64_t>), gu, dim3(WG), 0, s, d, nv, lev_rows, c, (const int64_t*)g,
                         ldg, (int64_t*)Y, B, lnv, lnode, i0);
    else if (tin == E_F32 && ty == E_F32)
      hipLaunchKernelGGL((k_usolve_uni<float, float>), gu, dim3(WG), 0, s, d, nv, lev_rows, c, (const float*)g, ldg,
                         (float*)Y, B, lnv, lnode, i0);
    else if (tin == E_F64 && ty == E_F32)
      hipLaunchKernelGGL((k_usolve_uni<double, float>), gu, dim3(WG), 0, s, d, nv, lev_rows, c, (const double*)g, ldg,
                         (float*)Y, B, lnv, lnode, i0);
    else if (tin == E_F64 && ty == E_F64)
      hipLaunchKernelGGL((k_usolve_uni<double, double>), gu, dim3(WG), 0, s, d, nv, lev_rows, c, (const double*)g,
                         ldg, (double*)Y, B, lnv, lnode, i0);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (tin == E_I64 && ty == E_I64)
    hipLaunchKernelGGL((k_usolve<int64_t, int64_t>), gr, dim3(WG), 0, s, d, nv, lev_rows, cnt, cw,
                       (const int64_t*)g, ldg, (int64_t*)Y, B);
  else if (tin == E_F32 && ty == E_F32)
    hipLaunchKernelGGL((k_usolve<float, float>), gr, dim3(WG), 0, s, d, nv, lev_rows, cnt, cw, (const float*)g,
                       ldg, (float*)Y, B);
  else if (tin == E_F64 && ty == E_F32)
    hipLaunchKernelGGL((k_usolve<double, float>), gr, dim3(WG), 0, s, d, nv, lev_rows, cnt, cw, (const double*)g,
                       ldg, (float*)Y, B);
  else if (tin == E_F64 && ty == E_F64)
    hipLaunchKernelGGL((k_usolve<double, double>), gr, dim3(WG), 0, s, d, nv, lev_rows, cnt, cw,
                       (const double*)g, ldg, (double*)Y, B);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

namespace {
template <typename TY, typename Tout>
void chain_diff_typed(const DevPoset& d, int dir, int cw, const void* Y, int64_t B, void* out, int64_t ldo,
                      bool accumulate, uint64_t* stats, hipStream_t s) {
  const int64_t rows_per_block = (WG / cw) * 8;
  const dim3 g((unsigned)((d.n + rows_per_block - 1) / rows_per_block), (unsigned)((B + cw - 1) / cw));
  if (cw == 64)
    hipLaunchKernelGGL((k_chain_diff<TY, Tout, 64>), g, dim3(WG), 0, s, d, dir, cw, (const TY*)Y, B, (Tout*)out, ldo,
                       (int)accumulate, stats);
  else
    hipLaunchKernelGGL((k_chain_diff<TY, Tout, 0>), g, dim3(WG), 0, s, d, dir, cw, (const TY*)Y, B, (Tout*)out, ldo,
                       (int)accumulate, stats);
}
}  // namespace

hipError_t launch_chain_diff(const DevPoset& d, int dir, ElemType ty, const void* Y, int64_t B, ElemType tout,
                             void* out, int64_t ldo, bool accumulate, uint64_t* stats, hipStream_t s) {
  if (d.n == 0) return hipSuccess;
  const int cw = col_width(B);
  if (stats) {
    const int64_t cnt = 2 * B + 1;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((cnt + WG - 1) / WG)), dim3(WG), 0, s, stats, cnt, (uint64_t)0);
  }
  if (ty == E_I64 && tout == E_I64)
    chain_diff_typed<int64_t, int64_t>(d, dir, cw, Y, B, out, ldo, accumulate, stats, s);
  else if (ty == E_F32 && tout == E_F32)
    chain_diff_typed<float, float>(d, dir, cw, Y, B, out, ldo, accumulate, stats, s);
  else if (ty == E_F64 && tout == E_F64)
    chain_diff_typed<double, double>(d, dir, cw, Y, B, out, ldo, accumulate, stats, s);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_absmax(int64_t n, int64_t B, const double* r, ElemType tg, const void* g, int64_t ldg,
                         uint64_t* stats, hipStream_t s) {
  const int64_t cnt = 2 * B + 1;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((cnt + WG - 1) / WG)), dim3(WG), 0, s, stats, cnt, (uint64_t)0);
  if (n == 0) return hipGetLastError();
  const int cw = col_width(B);
  const int64_t rows_per_block = WG / cw;
  int64_t blocks = (n + rows_per_block - 1) / rows_per_block;
  if (blocks > 2048) blocks = 2048;
  const dim3 grid((unsigned)blocks, (unsigned)((B + cw - 1) / cw));
  if (tg == E_F32)
    hipLaunchKernelGGL((k_absmax<float>), grid, dim3(WG), 0, s, n, B, cw, r, (const float*)g, ldg, stats);
  else if (tg == E_F64)
    hipLaunchKernelGGL((k_absmax<double>), grid, dim3(WG), 0, s, n, B, cw, r, (const double*)g, ldg, stats);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace px
