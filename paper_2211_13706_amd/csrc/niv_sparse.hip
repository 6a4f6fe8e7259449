// The niv maps as rows of their finite entries (N of §2.4 by rows), computed
// on the device.
//
// Theorem 5: row x of the map is the per-chain max (min for the dual map) over
// the rows of its children (parents), and x itself on its own chain.  A row
// lists its entries in ascending row order of the chain-major numbering, which
// is ascending chain order with one entry per chain.  So a row is a merge of
// its neighbours' sorted rows in which the entries of one chain, adjacent in
// the merged order, collapse to their max (min), with the own chain's entry
// replaced by x's row.  Rows of one height (longest path down to a leaf; up to
// a root for the dual map) depend only on lower heights, as in the host
// recursion, so one launch per height merges all of its rows:
//   * a wavefront per row, a lane per neighbour: lanes hold the heads of their
//     neighbours' rows (and those heads' chains, eight at a time), the wave
//     minimum picks the next chain, and the lanes whose head lies on it
//     advance;
//   * a count pass, an exclusive scan of the counts on the host (which also
//     reads the planted-chain check of the height), then a fill pass into a
//     pool; at the end one kernel lays the rows out by row.
// The planted-chain check is the host recursion's: for the map below, the
// largest own-chain entry over the children must be the row just below x (or
// none at the bottom of its chain).  Nodes with more than 64 neighbours send
// the map back to the host recursion.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cstdint>
#include <string>
#include <vector>

#include "niv_device.h"
#include "posetx.h"

namespace px {
namespace {

constexpr int SWG = 256;     // threads per workgroup: 4 wavefronts, a row each
constexpr int kMaxNbr = 64;  // neighbours per node (a lane each)
constexpr int kPf = 8;       // heads a lane holds

__device__ inline int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// One height: FILL = false counts every row's entries into count[i] and
// records failing planted chains in *bad (smallest node); FILL = true writes
// them to out[dst[i] ..].
template <bool UP, bool FILL>
__global__ __launch_bounds__(SWG) void k_sparse_rows(int64_t cnt, const int32_t* __restrict__ hn,
                                                     const int64_t* __restrict__ nptr,
                                                     const int32_t* __restrict__ nidx,
                                                     const int32_t* __restrict__ row_of_node,
                                                     const int32_t* __restrict__ chain_of_row,
                                                     const int32_t* __restrict__ chain_off,
                                                     const int64_t* __restrict__ st, const int32_t* __restrict__ ln,
                                                     const int32_t* __restrict__ pool, int32_t* __restrict__ count,
                                                     const int64_t* __restrict__ dst, int32_t* __restrict__ out,
                                                     int* __restrict__ bad) {
  const int lane = (int)(threadIdx.x & 63);
  const int64_t i = (int64_t)blockIdx.x * (SWG / 64) + (threadIdx.x >> 6);
  if (i >= cnt) return;
  const int x = __builtin_amdgcn_readfirstlane(hn[i]);
  const int r = __builtin_amdgcn_readfirstlane(row_of_node[x]);
  const int c = __builtin_amdgcn_readfirstlane(chain_of_row[r]);
  const bool bottom = r == __builtin_amdgcn_readfirstlane(chain_off[c]);
  const int64_t e0 = nptr[x];
  const int d = (int)(nptr[x + 1] - e0);
  // this lane's neighbour row: entries pool[p .. pe)
  int64_t p = 0, pe = 0;
  if (lane < d) {
    const int rz = row_of_node[nidx[e0 + lane]];
    p = st[rz];
    pe = p + ln[rz];
  }
  int hv[kPf], hc[kPf];  // the next heads and their chains (INT_MAX: none)
  auto refill = [&]() {
#pragma unroll
    for (int u = 0; u < kPf; ++u) hv[u] = p + u < pe ? pool[p + u] : INT_MAX;
#pragma unroll
    for (int u = 0; u < kPf; ++u) hc[u] = hv[u] != INT_MAX ? chain_of_row[hv[u]] : INT_MAX;
    p = min(p + kPf, pe);
  };
  refill();
  int64_t base = FILL ? dst[i] : 0;
  int n_out = 0, ob = 0;
  bool own_done = false, fail = false;
  auto emit = [&](int v) {
    if (FILL) {
      if (lane == (n_out & 63)) ob = v;
      if (((n_out + 1) & 63) == 0) out[base + (n_out + 1 - 64) + lane] = ob;
    }
    ++n_out;
  };
  for (;;) {
    const int head = hv[0];
    const int m = wave_min(head);
    if (m == INT_MAX) break;
    const uint64_t mb = __ballot(head == m);
    const int jm = __builtin_amdgcn_readlane(hc[0], (int)__builtin_ctzll(mb));
    if (!own_done && c < jm) {  // no neighbour entry on the own chain
      if (!UP && !bottom) fail = true;
      emit(r);
      own_done = true;
    }
    const bool mine = hc[0] == jm;
    const int v = UP ? m : wave_max(mine ? head : -1);
    if (jm == c) {
      if (!UP && (bottom || v != r - 1)) fail = true;
      emit(r);
      own_done = true;
    } else {
      emit(v);
    }
    if (mine) {  // advance past the head
#pragma unroll
      for (int u = 0; u + 1 < kPf; ++u) {
        hv[u] = hv[u + 1];
        hc[u] = hc[u + 1];
      }
      hv[kPf - 1] = INT_MAX;
      hc[kPf - 1] = INT_MAX;
      if (hv[0] == INT_MAX && p < pe) refill();
    }
  }
  if (!own_done) {
    if (!UP && !bottom) fail = true;
    emit(r);
  }
  if (FILL) {
    if (lane < (n_out & 63)) out[base + (n_out & ~63) + lane] = ob;
  } else {
    if (lane == 0) {
      count[i] = n_out;
      if (fail) atomicMin(bad, x);
    }
  }
}

// st / ln of the rows of one height from their counts and pool offsets.
__global__ __launch_bounds__(SWG) void k_sparse_place(int64_t cnt, const int32_t* __restrict__ hn,
                                                      const int32_t* __restrict__ row_of_node,
                                                      const int32_t* __restrict__ count,
                                                      const int64_t* __restrict__ dst, int64_t* __restrict__ st,
                                                      int32_t* __restrict__ ln) {
  const int64_t i = (int64_t)blockIdx.x * SWG + threadIdx.x;
  if (i >= cnt) return;
  const int r = row_of_node[hn[i]];
  st[r] = dst[i];
  ln[r] = count[i];
}

// The rows laid out by row: out[ptr[r] ..] = pool[st[r] ..], a wavefront per row.
__global__ __launch_bounds__(SWG) void k_sparse_layout(int64_t n, const int64_t* __restrict__ ptr,
                                                       const int64_t* __restrict__ st,
                                                       const int32_t* __restrict__ pool, int32_t* __restrict__ out) {
  const int lane = (int)(threadIdx.x & 63);
  const int64_t r = (int64_t)blockIdx.x * (SWG / 64) + (threadIdx.x >> 6);
  if (r >= n) return;
  const int64_t a = ptr[r], len = ptr[r + 1] - a, s = st[r];
  for (int64_t j = lane; j < len; j += 64) out[a + j] = pool[s + j];
}

// One height of the U-dependency levels, a wavefront per row: lev[r] = 1 + the
// largest level among the row's other-chain entries (dense rows nv [n, k], or
// the sparse rows ep / er), 0 without any.  Entries lie at lower heights.
__global__ __launch_bounds__(SWG) void k_udep_level(int64_t cnt, const int32_t* __restrict__ hn,
                                                    const int32_t* __restrict__ row_of_node, int k,
                                                    const int32_t* __restrict__ nv, const int64_t* __restrict__ ep,
                                                    const int32_t* __restrict__ er, int32_t* __restrict__ lev) {
  const int lane = (int)(threadIdx.x & 63);
  const int64_t i = (int64_t)blockIdx.x * (SWG / 64) + (threadIdx.x >> 6);
  if (i >= cnt) return;
  const int r = __builtin_amdgcn_readfirstlane(row_of_node[hn[i]]);
  const int32_t* row = nv ? nv + (int64_t)r * k : er + ep[r];
  const int64_t len = nv ? k : ep[r + 1] - ep[r];
  int m = 0;
  for (int64_t j = lane; j < len; j += 64) {
    const int t = row[j];
    if (t >= 0 && t != r) m = max(m, lev[t] + 1);
  }
  m = wave_max(m);
  if (lane == 0) lev[r] = m;
}

// All U-dependency levels in one persistent launch.  lev starts at -1
// (unknown).  Wavefront w takes the positions w, w + W, ... of the height
// order (W the wavefronts of the grid), one row each: its lanes read the row's
// other-chain entries (64 at a time), poll their levels until none is -1, and
// lane 0 stores 1 + the largest (0 without entries).  An entry lies at a
// lower height, so earlier in the order; a wavefront takes its positions in
// order, so with every wavefront resident the unfinished position of lowest
// index has all it reads and every wait ends.  Levels travel as relaxed
// device-scope loads and stores (coherent across the per-XCD caches).  A
// wait is bounded by spin_limit polls and about 2 s; one that gives up stores
// err and stops, and the caller computes the levels height by height instead.
__global__ __launch_bounds__(SWG) void k_udep_poll(int64_t n, const int32_t* __restrict__ hn,
                                                   const int32_t* __restrict__ row_of_node, int k,
                                                   const int32_t* __restrict__ nv, const int64_t* __restrict__ ep,
                                                   const int32_t* __restrict__ er, int32_t* lev, int* err,
                                                   int spin_limit) {
  const int lane = (int)(threadIdx.x & 63);
  const int64_t nw = (int64_t)gridDim.x * (SWG / 64);
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  for (int64_t i = (int64_t)blockIdx.x * (SWG / 64) + (threadIdx.x >> 6); i < n; i += nw) {
    const int r = __builtin_amdgcn_readfirstlane(row_of_node[hn[i]]);
    const int32_t* row = nv ? nv + (int64_t)r * k : er + ep[r];
    const int64_t len = nv ? k : ep[r + 1] - ep[r];
    int m = 0;
    for (int64_t j0 = 0; j0 < len; j0 += 64) {
      int t = j0 + lane < len ? row[j0 + lane] : -1;
      if (t == r) t = -1;
      int v = __hip_atomic_load(lev + (t >= 0 ? t : r), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (int spin = 0; __any(t >= 0 && v < 0); ++spin) {
        if (spin >= spin_limit || ((spin & 15) == 15 && (__hip_atomic_load(err, __ATOMIC_RELAXED,
                                                                             __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                                                          __builtin_amdgcn_s_memrealtime() - t0 > 200000000ull))) {
          if (lane == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          return;
        }
        __builtin_amdgcn_s_sleep(1);
        if (t >= 0 && v < 0) v = __hip_atomic_load(lev + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (t >= 0) m = max(m, v + 1);
    }
    m = wave_max(m);
    if (lane == 0) __hip_atomic_store(lev + r, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// A run of narrow heights (few rows each, such as the one row per chain of a
// poset of long chains) in one launch, for dense rows: a single workgroup
// takes heights h0 .. h1 - 1 in order.  The rows of height h are R[hptr[h] ..
// hptr[h + 1]) and E holds their other-chain entries (-1 for none and for the
// own chain), k per row, in the same order, so that a height's entries load
// while the height before it is summed: only the levels themselves wait.
// Each thread takes up to SEQ_PP (row, entry) pairs of a height, the rows'
// maxima meet in LDS (two buffers, alternating by height), and a workgroup
// barrier orders one height's level stores before the next height's loads
// (all wavefronts share one compute unit and its cache).  Measured per height:
// one launch about 3.4 to 4.7 us, this loop 1.9 us with 1,024 pairs (n = 2^23,
// k = 32) but 4.2 us with 4,096 (n = 2^20, k = 64: 64 atomics on each row's
// maximum), so heights of more than SEQ_WG * SEQ_PP pairs take a launch each.
constexpr int SEQ_WG = 1024, SEQ_PP = 2, SEQ_ROWS = 128;
__global__ __launch_bounds__(SEQ_WG) void k_udep_levels_seq(int64_t h0, int64_t h1, const int64_t* __restrict__ hptr,
                                                           const int32_t* __restrict__ R, int k,
                                                           const int32_t* __restrict__ E, int32_t* lev) {
  __shared__ int mx[2][SEQ_ROWS];
  int tc[SEQ_PP], tn[SEQ_PP];
  auto load = [&](int64_t h, int* t) {
    const int64_t i0 = hptr[h], pairs = (hptr[h + 1] - i0) * k;
#pragma unroll
    for (int u = 0; u < SEQ_PP; ++u) {
      const int64_t q = threadIdx.x + (int64_t)u * SEQ_WG;
      t[u] = q < pairs ? E[i0 * k + q] : -1;
    }
  };
  load(h0, tc);
  for (int64_t h = h0; h < h1; ++h) {
    const int b = (int)(h & 1);
    const int64_t i0 = hptr[h], c = hptr[h + 1] - i0;
    if (threadIdx.x < c) mx[b][threadIdx.x] = 0;
    if (h + 1 < h1) load(h + 1, tn);
    __syncthreads();  // the maxima cleared; the levels of earlier heights stored
#pragma unroll
    for (int u = 0; u < SEQ_PP; ++u) {
      const int q = (int)threadIdx.x + u * SEQ_WG;
      if (tc[u] >= 0) atomicMax(&mx[b][q / k], lev[tc[u]] + 1);
    }
    __syncthreads();
    if (threadIdx.x < c) lev[R[i0 + threadIdx.x]] = mx[b][threadIdx.x];
#pragma unroll
    for (int u = 0; u < SEQ_PP; ++u) tc[u] = tn[u];
  }
}

// E for k_udep_levels_seq: R[i] = row of the i-th node in height order, and its
// k entries with the own chain and missing entries as -1.
__global__ __launch_bounds__(SWG) void k_udep_entries(int64_t n, int k, const int32_t* __restrict__ hn,
                                                      const int32_t* __restrict__ row_of_node,
                                                      const int32_t* __restrict__ nv, int32_t* __restrict__ R,
                                                      int32_t* __restrict__ E) {
  const int64_t q = (int64_t)blockIdx.x * SWG + threadIdx.x;
  if (q >= n * k) return;
  const int64_t i = q / k, j = q % k;
  const int r = row_of_node[hn[i]];
  if (j == 0) R[i] = r;
  const int t = nv[(int64_t)r * k + j];
  E[q] = (t >= 0 && t != r) ? t : -1;
}

unsigned nblocks(int64_t items, int per) { return (unsigned)((items + per - 1) / per); }

struct Held {
  std::vector<void*> bufs;
  hipError_t err = hipSuccess;
  template <typename T>
  T* get(size_t count) {
    void* q = nullptr;
    if (err == hipSuccess) err = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (err == hipSuccess) bufs.push_back(q);
    return (T*)q;
  }
  template <typename T>
  T* put(const T* h, size_t count) {
    T* q = get<T>(count);
    if (err == hipSuccess && count) err = hipMemcpy(q, h, count * sizeof(T), hipMemcpyHostToDevice);
    return q;
  }
  void drop(void* q) {
    for (size_t j = 0; j < bufs.size(); ++j)
      if (bufs[j] == q) {
        (void)hipFree(q);
        bufs.erase(bufs.begin() + j);
        return;
      }
  }
  void release(void* keep1 = nullptr, void* keep2 = nullptr, void* keep3 = nullptr, void* keep4 = nullptr) {
    for (void* q : bufs)
      if (q != keep1 && q != keep2 && q != keep3 && q != keep4) (void)hipFree(q);
    bufs.clear();
  }
};

}  // namespace

int device_niv_sparse(Prep& P, const int64_t* indptr, const int32_t* indices, const std::vector<int64_t>& rptr,
                      const std::vector<int32_t>& ridx, const Heights& H, bool want_up, int64_t* out_ptr[2],
                      int32_t* out_rows[2], std::string& msg) {
  const int64_t n = P.n;
  out_ptr[0] = out_ptr[1] = nullptr;
  out_rows[0] = out_rows[1] = nullptr;
  for (int64_t x = 0; x < n; ++x)
    if (indptr[x + 1] - indptr[x] > kMaxNbr || (want_up && rptr[x + 1] - rptr[x] > kMaxNbr)) return -1;
  Held hb;
  const int32_t* d_ron = hb.put(P.row_of_node.data(), (size_t)n);
  const int32_t* d_cor = hb.put(P.chain_of_row.data(), (size_t)n);
  const int32_t* d_coff = hb.put(P.chain_off.data(), P.chain_off.size());
  int* d_bad = hb.get<int>(1);
  int32_t* d_cnt = hb.get<int32_t>((size_t)n);
  int64_t* d_dst = hb.get<int64_t>((size_t)n);
  int64_t* d_st = hb.get<int64_t>((size_t)n);
  int32_t* d_ln = hb.get<int32_t>((size_t)n);
  if (hb.err != hipSuccess) {
    hb.release();
    return -1;
  }
  int32_t* kept_rows[2] = {nullptr, nullptr};
  int64_t* kept_ptr[2] = {nullptr, nullptr};
  int rc = PX_OK;
  for (int m = 0; m < (want_up ? 2 : 1) && rc == PX_OK; ++m) {
    const bool up = m == 1;
    Held mb;  // this map's buffers
    const int64_t* d_nptr = up ? mb.put(rptr.data(), rptr.size()) : mb.put(indptr, (size_t)n + 1);
    const int32_t* d_nidx = up ? mb.put(ridx.data(), ridx.size()) : mb.put(indices, (size_t)indptr[n]);
    const int32_t* d_hn = mb.put(H.nodes[m].data(), H.nodes[m].size());
    size_t cap = (size_t)std::max<int64_t>(n * 4, 1 << 20);
    int32_t* d_pool = mb.get<int32_t>(cap);
    int64_t used = 0;
    const int bad0 = INT_MAX;
    hipError_t e = mb.err != hipSuccess ? mb.err : hb.err;
    if (e == hipSuccess) e = hipMemcpy(d_bad, &bad0, sizeof(int), hipMemcpyHostToDevice);
    std::vector<int32_t> cnt;
    std::vector<int64_t> dst;
    const std::vector<int64_t>& hp = H.ptr[m];
    for (size_t h = 0; h + 1 < hp.size() && e == hipSuccess; ++h) {
      const int64_t c = hp[h + 1] - hp[h];
      const int32_t* hn = d_hn + hp[h];
      if (up)
        hipLaunchKernelGGL((k_sparse_rows<true, false>), dim3(nblocks(c, SWG / 64)), dim3(SWG), 0, 0, c, hn, d_nptr,
                           d_nidx, d_ron, d_cor, d_coff, d_st, d_ln, d_pool, d_cnt, nullptr, nullptr, d_bad);
      else
        hipLaunchKernelGGL((k_sparse_rows<false, false>), dim3(nblocks(c, SWG / 64)), dim3(SWG), 0, 0, c, hn, d_nptr,
                           d_nidx, d_ron, d_cor, d_coff, d_st, d_ln, d_pool, d_cnt, nullptr, nullptr, d_bad);
      e = hipGetLastError();
      cnt.resize(c);
      int bad = INT_MAX;
      if (e == hipSuccess) e = hipMemcpy(cnt.data(), d_cnt, c * sizeof(int32_t), hipMemcpyDeviceToHost);
      if (e == hipSuccess) e = hipMemcpy(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost);
      if (e != hipSuccess) break;
      if (bad != INT_MAX) {
        msg = "chain " + std::to_string(P.chain_of[bad]) + " is not totally ordered at position " +
              std::to_string(P.chain_pos[bad]) + " (node " + std::to_string(bad) + ")";
        rc = PX_ECHAIN;
        break;
      }
      dst.resize(c);
      int64_t total = 0;
      for (int64_t j = 0; j < c; ++j) {
        dst[j] = used + total;
        total += cnt[j];
      }
      if ((size_t)(used + total) > cap) {  // grow the pool
        size_t ncap = std::max(cap * 3 / 2, (size_t)(used + total));
        int32_t* np = mb.get<int32_t>(ncap);
        if (mb.err != hipSuccess) {
          e = mb.err;
          break;
        }
        if (used) e = hipMemcpy(np, d_pool, used * sizeof(int32_t), hipMemcpyDeviceToDevice);
        mb.drop(d_pool);
        d_pool = np;
        cap = ncap;
      }
      if (e == hipSuccess) e = hipMemcpy(d_dst, dst.data(), c * sizeof(int64_t), hipMemcpyHostToDevice);
      if (e != hipSuccess) break;
      hipLaunchKernelGGL(k_sparse_place, dim3(nblocks(c, SWG)), dim3(SWG), 0, 0, c, hn, d_ron, d_cnt, d_dst, d_st,
                         d_ln);
      if (up)
        hipLaunchKernelGGL((k_sparse_rows<true, true>), dim3(nblocks(c, SWG / 64)), dim3(SWG), 0, 0, c, hn, d_nptr,
                           d_nidx, d_ron, d_cor, d_coff, d_st, d_ln, d_pool, nullptr, d_dst, d_pool, d_bad);
      else
        hipLaunchKernelGGL((k_sparse_rows<false, true>), dim3(nblocks(c, SWG / 64)), dim3(SWG), 0, 0, c, hn, d_nptr,
                           d_nidx, d_ron, d_cor, d_coff, d_st, d_ln, d_pool, nullptr, d_dst, d_pool, d_bad);
      e = hipGetLastError();
      used += total;
    }
    if (rc == PX_OK && e == hipSuccess) {  // lay the rows out by row
      std::vector<int32_t> lens(n);
      e = hipMemcpy(lens.data(), d_ln, n * sizeof(int32_t), hipMemcpyDeviceToHost);
      std::vector<int64_t>& ptr = P.nivp[m];
      std::vector<int32_t>& ent = P.nivr[m];
      ptr.assign(n + 1, 0);
      for (int64_t r = 0; r < n; ++r) ptr[r + 1] = ptr[r] + lens[r];
      int64_t* d_ptr = e == hipSuccess ? mb.put(ptr.data(), ptr.size()) : nullptr;
      int32_t* d_rows = e == hipSuccess ? mb.get<int32_t>((size_t)ptr[n]) : nullptr;
      if (e == hipSuccess) e = mb.err;
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_sparse_layout, dim3(nblocks(n, SWG / 64)), dim3(SWG), 0, 0, n, d_ptr, d_st, d_pool,
                           d_rows);
        e = hipGetLastError();
      }
      ent.resize(ptr[n]);
      if (e == hipSuccess && ptr[n]) e = hipMemcpy(ent.data(), d_rows, ptr[n] * sizeof(int32_t), hipMemcpyDeviceToHost);
      if (e == hipSuccess) {
        (up ? P.nnz_niv_up : P.nnz_niv) = ptr[n];
        kept_ptr[m] = d_ptr;
        kept_rows[m] = d_rows;
        mb.release(d_ptr, d_rows);
      }
    }
    if (e != hipSuccess && rc == PX_OK) {
      (void)hipGetLastError();
      rc = e == hipErrorOutOfMemory ? PX_ENOMEM : PX_EHIP;
      msg = std::string("device niv rows: ") + hipGetErrorString(e);
    }
    if (rc != PX_OK) mb.release();
  }
  hb.release();
  if (rc != PX_OK) {
    for (int m = 0; m < 2; ++m) {
      if (kept_ptr[m]) (void)hipFree(kept_ptr[m]);
      if (kept_rows[m]) (void)hipFree(kept_rows[m]);
    }
    P.nivp[0].clear();
    P.nivp[1].clear();
    P.nivr[0].clear();
    P.nivr[1].clear();
    return rc;
  }
  for (int m = 0; m < 2; ++m) {
    out_ptr[m] = kept_ptr[m];
    out_rows[m] = kept_rows[m];
  }
  P.niv_rounds = (int32_t)(H.ptr[0].size() - 1);
  return PX_OK;
}

int device_udep_levels(const Prep& P, const std::vector<int64_t>& hptr, const std::vector<int32_t>& hnodes,
                       const int32_t* nv, const int64_t* ep, const int32_t* er, std::vector<int32_t>& lev) {
  const int64_t n = P.n;
  if (n == 0 || (!nv && (!ep || !er))) return -1;
  Held hb;
  const int32_t* d_hn = hb.put(hnodes.data(), hnodes.size());
  const int32_t* d_ron = hb.put(P.row_of_node.data(), (size_t)n);
  const int64_t* d_hptr = hb.put(hptr.data(), hptr.size());
  int32_t* d_lev = hb.get<int32_t>((size_t)n);
  hipError_t e = hb.err;
  if (e == hipSuccess) e = hipMemset(d_lev, 0, n * sizeof(int32_t));
  const int64_t nh = (int64_t)hptr.size() - 1;
  // all levels in one persistent launch, unless POSETX_UDEP=heights; if a wait
  // gave up there, height by height below
  bool done = false;
  const char* mode = std::getenv("POSETX_UDEP");
  if (e == hipSuccess && !(mode && std::string(mode) == "heights")) {
    int* d_err = hb.get<int>(1);
    int per_cu = 0, cus = 0, dev = 0;
    e = hb.err;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_udep_poll, SWG, 0);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipMemset(d_lev, 0xFF, n * sizeof(int32_t));
    if (e == hipSuccess) e = hipMemset(d_err, 0, sizeof(int));
    if (e == hipSuccess) {
      const int64_t res = (int64_t)std::max(1, per_cu) * std::max(1, cus);
      const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(res, (n + SWG / 64 - 1) / (SWG / 64)));
      const char* sv = std::getenv("POSETX_FLOW_SPIN");
      const int spin = sv ? std::max(0, std::atoi(sv)) : 1 << 20;
      hipLaunchKernelGGL(k_udep_poll, dim3(grid), dim3(SWG), 0, 0, n, d_hn, d_ron, (int)P.k, nv, ep, er, d_lev, d_err,
                         spin);
      e = hipGetLastError();
    }
    int herr = 1;
    if (e == hipSuccess) e = hipMemcpy(&herr, d_err, sizeof(int), hipMemcpyDeviceToHost);
    done = e == hipSuccess && herr == 0;
    if (e == hipSuccess && !done) e = hipMemset(d_lev, 0, n * sizeof(int32_t));
  }
  // height by height: for dense rows, heights of at most SEQ_ROWS rows and
  // SEQ_WG * SEQ_PP entries go in runs through k_udep_levels_seq, wider ones
  // (and sparse rows) one launch each
  int32_t* d_R = nullptr;
  int32_t* d_E = nullptr;
  if (nv && e == hipSuccess && !done) {
    d_R = hb.get<int32_t>((size_t)n);
    d_E = hb.get<int32_t>((size_t)(n * P.k));
    e = hb.err;
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_udep_entries, dim3(nblocks(n * P.k, SWG)), dim3(SWG), 0, 0, n, (int)P.k, d_hn, d_ron, nv,
                         d_R, d_E);
      e = hipGetLastError();
    }
  }
  int64_t h0 = 0;  // first height of the pending run of narrow heights
  for (int64_t h = 0; h <= nh && e == hipSuccess && !done; ++h) {
    const int64_t c = h < nh ? hptr[h + 1] - hptr[h] : 0;
    const bool narrow = h < nh && d_E && c <= SEQ_ROWS && c * P.k <= (int64_t)SEQ_WG * SEQ_PP;
    if (narrow) continue;
    if (h > h0) {
      hipLaunchKernelGGL(k_udep_levels_seq, dim3(1), dim3(SEQ_WG), 0, 0, h0, h, d_hptr, d_R, (int)P.k, d_E, d_lev);
      e = hipGetLastError();
    }
    if (h < nh && e == hipSuccess) {
      hipLaunchKernelGGL(k_udep_level, dim3(nblocks(c, SWG / 64)), dim3(SWG), 0, 0, c, d_hn + hptr[h], d_ron,
                         (int)P.k, nv, ep, er, d_lev);
      e = hipGetLastError();
    }
    h0 = h + 1;
  }
  lev.resize(n);
  if (e == hipSuccess) e = hipMemcpy(lev.data(), d_lev, n * sizeof(int32_t), hipMemcpyDeviceToHost);
  hb.release();
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return -1;
  }
  return PX_OK;
}

__global__ __launch_bounds__(SWG) void k_gather_rows(const int32_t* __restrict__ src, int k,
                                                     const int32_t* __restrict__ rows, int64_t cnt,
                                                     const int32_t* __restrict__ node_of_row,
                                                     int32_t* __restrict__ dst, int32_t* __restrict__ nodes) {
  const int64_t q = (int64_t)blockIdx.x * SWG + threadIdx.x;
  if (q >= cnt * k) return;
  const int64_t i = q / k, j = q % k;
  const int r = rows[i];
  dst[q] = src[(int64_t)r * k + j];
  if (j == 0) nodes[i] = node_of_row[r];
}

hipError_t device_gather_rows(const int32_t* src, int k, const int32_t* rows, int64_t cnt,
                              const int32_t* node_of_row, int32_t* dst, int32_t* nodes) {
  if (cnt == 0 || k == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3(nblocks(cnt * k, SWG)), dim3(SWG), 0, 0, src, k, rows, cnt, node_of_row,
                     dst, nodes);
  return hipGetLastError();
}

}  // namespace px
