// The niv maps (§2.4) computed on the device, for dense rows.
//
// Theorem 5 defines niv(x) through the children of x: niv_j(x) is the largest
// niv_j over the children, and x itself on its own chain.  Along a chain that
// is totally ordered the element below x is one of those descendants, and every
// other same-chain descendant lies below it, so
//
//   niv(r) = max( niv(r - 1), max over the other-chain children z of niv(z) ),
//   niv_{own}(r) = r                                    (rows chain-major),
//
// i.e. niv is the fixed point of X -> PrefixMax_chain(C(X)) with
// C(X)(r) = max(e_own(r), max over other-chain children z of X(z)).  The host
// evaluates the recursion node by node in topological order; here it is
// iterated as a whole: from X_0 = e_own (its own chain prefix max), each round
// is one gather over the other-chain children and one prefix max along every
// chain (a three-pass tile scan), until a round changes nothing.  Every X_t
// lies below the unique fixed point and the rounds increase, so the result is
// exactly the recursion's.  A round is needed per chain change along the
// paths that realise niv, and such a path never needs to come back to a chain
// (from its first element on a chain it can go down that chain instead), so
// k + 1 rounds always suffice: ten per map on random-height posets with 64
// chains, 64 on a 64-column grid.  The cap kMaxRounds (above the 256 chains of
// dense rows) sends a poset back to the host recursion should it be reached.
// The dual map is the same with min, parents and suffixes.
//
// Planted chains are checked afterwards, as the host recursion checks them:
// for every row, the largest own-chain entry over all of its children must be
// the row just below it (or none at the chain's bottom).  Where a chain is not
// totally ordered, the descendants of the lowest offending element still get
// their true niv rows, so that element fails the check.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <string>
#include <vector>

#include "niv_device.h"
#include "posetx.h"

namespace px {
namespace {

constexpr int NWG = 256;         // threads per workgroup: 4 wavefronts
constexpr int kTileRows = 256;   // rows per tile of the chain prefix max
constexpr int kMaxRounds = 512;

template <bool UP> __device__ inline int32_t comb(int32_t a, int32_t b) { return UP ? min(a, b) : max(a, b); }
template <bool UP> __device__ inline int32_t none_v() { return UP ? INT32_MAX : -1; }

// X_0: own entry only (already its own chain prefix).
template <bool UP>
__global__ __launch_bounds__(NWG) void k_niv_init(int64_t n, int k, const int32_t* __restrict__ cor,
                                                  int32_t* __restrict__ X) {
  const int64_t i = (int64_t)blockIdx.x * NWG + threadIdx.x;
  if (i >= n * k) return;
  const int64_t r = i / k;
  X[i] = (int)(i % k) == cor[r] ? (int32_t)r : none_v<UP>();
}

// C(X): one wavefront per row, lanes over 64 entries of it.
template <bool UP>
__global__ __launch_bounds__(NWG) void k_niv_cross(int64_t n, int k, const int64_t* __restrict__ xp,
                                                   const int32_t* __restrict__ xr, const int32_t* __restrict__ cor,
                                                   const int32_t* __restrict__ X, int32_t* __restrict__ C) {
  const int64_t r = (int64_t)blockIdx.x * (NWG / 64) + (threadIdx.x >> 6);
  const int j = (int)blockIdx.y * 64 + (int)(threadIdx.x & 63);
  if (r >= n || j >= k) return;
  int32_t v = j == cor[r] ? (int32_t)r : none_v<UP>();
  const int64_t e1 = xp[r + 1];
  int64_t e = xp[r];
  for (; e + 4 <= e1; e += 4) {
    int32_t z[4], w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) z[u] = xr[e + u];
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = X[(int64_t)z[u] * k + j];
#pragma unroll
    for (int u = 0; u < 4; ++u) v = comb<UP>(v, w[u]);
  }
  for (; e < e1; ++e) v = comb<UP>(v, X[(int64_t)xr[e] * k + j]);
  C[r * k + j] = v;
}

// Tile totals of C; tiles[t] = {first row, end row, chain, 0}.
template <bool UP>
__global__ __launch_bounds__(NWG) void k_niv_tile(int k, int64_t ntiles, const int4* __restrict__ tiles,
                                                  const int32_t* __restrict__ C, int32_t* __restrict__ TM) {
  const int64_t t = (int64_t)blockIdx.x * (NWG / 64) + (threadIdx.x >> 6);
  const int j = (int)blockIdx.y * 64 + (int)(threadIdx.x & 63);
  if (t >= ntiles || j >= k) return;
  const int4 tt = tiles[t];
  int32_t acc = none_v<UP>();
  int r = tt.x;
  for (; r + 8 <= tt.y; r += 8) {
    int32_t w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) w[u] = C[(int64_t)(r + u) * k + j];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = comb<UP>(acc, w[u]);
  }
  for (; r < tt.y; ++r) acc = comb<UP>(acc, C[(int64_t)r * k + j]);
  TM[t * k + j] = acc;
}

// Exclusive scan of the tile totals along every chain (UP: from the top).
template <bool UP>
__global__ __launch_bounds__(NWG) void k_niv_carry(int k, int nchains, const int32_t* __restrict__ ctile,
                                                   const int32_t* __restrict__ TM, int32_t* __restrict__ CA) {
  const int64_t i = (int64_t)blockIdx.x * NWG + threadIdx.x;
  const int64_t c = i / k;
  const int j = (int)(i % k);
  if (c >= nchains) return;
  const int t0 = ctile[c], t1 = ctile[c + 1];
  int32_t acc = none_v<UP>();
  for (int q = 0; q < t1 - t0; ++q) {
    const int64_t t = UP ? t1 - 1 - q : t0 + q;
    const int32_t w = TM[t * k + j];
    CA[t * k + j] = acc;
    acc = comb<UP>(acc, w);
  }
}

// X' = PrefixMax_chain(C) tile by tile from the carries; flags a change.
template <bool UP>
__global__ __launch_bounds__(NWG) void k_niv_apply(int k, int64_t ntiles, const int4* __restrict__ tiles,
                                                   const int32_t* __restrict__ C, const int32_t* __restrict__ CA,
                                                   const int32_t* __restrict__ X, int32_t* __restrict__ Xn,
                                                   int* __restrict__ changed) {
  const int64_t t = (int64_t)blockIdx.x * (NWG / 64) + (threadIdx.x >> 6);
  const int j = (int)blockIdx.y * 64 + (int)(threadIdx.x & 63);
  if (t >= ntiles || j >= k) return;
  const int4 tt = tiles[t];
  int32_t acc = CA[t * k + j];
  bool ch = false;
  const int len = tt.y - tt.x;
  for (int q = 0; q < len; ++q) {
    const int64_t r = UP ? tt.y - 1 - q : tt.x + q;
    acc = comb<UP>(acc, C[r * k + j]);
    ch = ch || acc != X[r * k + j];
    Xn[r * k + j] = acc;
  }
  if (ch) *changed = 1;  // every writer stores the same value
}

__global__ __launch_bounds__(NWG) void k_niv_none(int64_t cnt, int32_t* __restrict__ X) {
  const int64_t i = (int64_t)blockIdx.x * NWG + threadIdx.x;
  if (i < cnt && X[i] == INT32_MAX) X[i] = -1;
}

// The planted-chain check: row r's largest own-chain entry over all of its
// children must be r - 1 (or -1 at the chain's bottom).  bad: smallest failing row.
__global__ __launch_bounds__(NWG) void k_niv_check(int64_t n, int k, const int64_t* __restrict__ cp,
                                                   const int32_t* __restrict__ cr, const int32_t* __restrict__ cor,
                                                   const int32_t* __restrict__ coff, const int32_t* __restrict__ X,
                                                   int* __restrict__ bad) {
  const int64_t r = (int64_t)blockIdx.x * NWG + threadIdx.x;
  if (r >= n) return;
  const int c = cor[r];
  const int32_t expect = r > coff[c] ? (int32_t)r - 1 : -1;
  int32_t m = -1;
  for (int64_t e = cp[r]; e < cp[r + 1]; ++e) m = max(m, X[(int64_t)cr[e] * k + c]);
  if (m != expect) atomicMin(bad, (int)r);
}

unsigned blocks(int64_t items, int per) { return (unsigned)((items + per - 1) / per); }

// Device buffers of one call, freed on every exit.
struct Bufs {
  std::vector<void*> held;
  hipError_t err = hipSuccess;
  template <typename T>
  T* get(size_t count) {
    void* p = nullptr;
    if (err == hipSuccess) err = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
    if (err == hipSuccess) held.push_back(p);
    return (T*)p;
  }
  template <typename T>
  T* put(const std::vector<T>& h) {
    T* p = get<T>(h.size());
    if (err == hipSuccess && !h.empty()) err = hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    return p;
  }
  void release(void* keep1, void* keep2) {
    for (void* p : held)
      if (p != keep1 && p != keep2) (void)hipFree(p);
    held.clear();
  }
};

// Rows of the neighbours in CSR (children or parents), in row order; with
// cross_only, those on other chains only.
void row_csr(const Prep& P, const int64_t* ptr, const int32_t* idx, bool cross_only, std::vector<int64_t>& rp,
             std::vector<int32_t>& rr) {
  const int64_t n = P.n;
  rp.assign(n + 1, 0);
  rr.clear();
  rr.reserve((size_t)ptr[n]);
  for (int64_t r = 0; r < n; ++r) {
    const int32_t x = P.node_of_row[r];
    for (int64_t e = ptr[x]; e < ptr[x + 1]; ++e) {
      const int32_t z = idx[e];
      if (!cross_only || P.chain_of[z] != P.chain_of[x]) rr.push_back(P.row_of_node[z]);
    }
    rp[r + 1] = (int64_t)rr.size();
  }
}

}  // namespace

int device_niv(Prep& P, const int64_t* indptr, const int32_t* indices, const std::vector<int64_t>& rptr,
               const std::vector<int32_t>& ridx, bool want_up, int32_t** out_niv, int32_t** out_up, int* rounds,
               std::string& msg) {
  *out_niv = *out_up = nullptr;
  const int64_t n = P.n, k = P.k;
  if (n == 0 || k == 0 || k > 1024) return -1;
  // tiles of at most kTileRows rows inside every chain
  std::vector<int4> tiles;
  std::vector<int32_t> ctile(k + 1, 0);
  for (int64_t c = 0; c < k; ++c) {
    for (int32_t r = P.chain_off[c]; r < P.chain_off[c + 1]; r += kTileRows)
      tiles.push_back(make_int4(r, std::min<int32_t>(r + kTileRows, P.chain_off[c + 1]), (int)c, 0));
    ctile[c + 1] = (int32_t)tiles.size();
  }
  const int64_t nt = (int64_t)tiles.size();
  std::vector<int64_t> dp, cp, up;
  std::vector<int32_t> dr, cr, ur;
  row_csr(P, indptr, indices, true, dp, dr);
  row_csr(P, indptr, indices, false, cp, cr);
  if (want_up) row_csr(P, rptr.data(), ridx.data(), true, up, ur);

  Bufs b;
  const int32_t* d_cor = b.put(P.chain_of_row);
  const int32_t* d_coff = b.put(P.chain_off);
  const int4* d_tiles = b.put(tiles);
  const int32_t* d_ctile = b.put(ctile);
  int32_t* d_niv = b.get<int32_t>((size_t)n * k);
  int32_t* d_up = want_up ? b.get<int32_t>((size_t)n * k) : nullptr;
  int32_t* d_tmp = b.get<int32_t>((size_t)n * k);
  int32_t* d_C = b.get<int32_t>((size_t)n * k);
  int32_t* d_TM = b.get<int32_t>((size_t)nt * k);
  int32_t* d_CA = b.get<int32_t>((size_t)nt * k);
  int* d_flag = b.get<int>(2);
  if (b.err != hipSuccess) {
    const hipError_t e = b.err;
    b.release(nullptr, nullptr);
    (void)hipGetLastError();
    msg = std::string("device niv buffers: ") + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? PX_ENOMEM : PX_EHIP;
  }
  const dim3 grow(blocks(n, NWG / 64), (unsigned)((k + 63) / 64));
  const dim3 gtile(blocks(nt, NWG / 64), (unsigned)((k + 63) / 64));
  int total_rounds = 0;
  // one map: the fixed point into dst (X alternates between dst and d_tmp)
  auto run = [&](bool upm, const std::vector<int64_t>& hp, const std::vector<int32_t>& hr, int32_t* dst) -> int {
    Bufs nb;
    const int64_t* d_xp = nb.put(hp);
    const int32_t* d_xr = nb.put(hr);
    if (nb.err != hipSuccess) {
      nb.release(nullptr, nullptr);
      return nb.err == hipErrorOutOfMemory ? PX_ENOMEM : PX_EHIP;
    }
    int32_t* X = dst;
    int32_t* Xn = d_tmp;
    if (upm)
      hipLaunchKernelGGL(k_niv_init<true>, dim3(blocks(n * k, NWG)), dim3(NWG), 0, 0, n, (int)k, d_cor, X);
    else
      hipLaunchKernelGGL(k_niv_init<false>, dim3(blocks(n * k, NWG)), dim3(NWG), 0, 0, n, (int)k, d_cor, X);
    int flag = 1, round = 0;
    hipError_t e = hipGetLastError();
    while (e == hipSuccess && flag && round < kMaxRounds) {
      e = hipMemset(d_flag, 0, sizeof(int));
      if (e != hipSuccess) break;
      if (upm) {
        hipLaunchKernelGGL(k_niv_cross<true>, grow, dim3(NWG), 0, 0, n, (int)k, d_xp, d_xr, d_cor, X, d_C);
        hipLaunchKernelGGL(k_niv_tile<true>, gtile, dim3(NWG), 0, 0, (int)k, nt, d_tiles, d_C, d_TM);
        hipLaunchKernelGGL(k_niv_carry<true>, dim3(blocks(k * k, NWG)), dim3(NWG), 0, 0, (int)k, (int)k, d_ctile,
                           d_TM, d_CA);
        hipLaunchKernelGGL(k_niv_apply<true>, gtile, dim3(NWG), 0, 0, (int)k, nt, d_tiles, d_C, d_CA, X, Xn, d_flag);
      } else {
        hipLaunchKernelGGL(k_niv_cross<false>, grow, dim3(NWG), 0, 0, n, (int)k, d_xp, d_xr, d_cor, X, d_C);
        hipLaunchKernelGGL(k_niv_tile<false>, gtile, dim3(NWG), 0, 0, (int)k, nt, d_tiles, d_C, d_TM);
        hipLaunchKernelGGL(k_niv_carry<false>, dim3(blocks(k * k, NWG)), dim3(NWG), 0, 0, (int)k, (int)k, d_ctile,
                           d_TM, d_CA);
        hipLaunchKernelGGL(k_niv_apply<false>, gtile, dim3(NWG), 0, 0, (int)k, nt, d_tiles, d_C, d_CA, X, Xn,
                           d_flag);
      }
      e = hipGetLastError();
      if (e == hipSuccess) e = hipMemcpy(&flag, d_flag, sizeof(int), hipMemcpyDeviceToHost);
      std::swap(X, Xn);
      ++round;
    }
    total_rounds += round;
    if (e == hipSuccess && X != dst) e = hipMemcpy(dst, X, (size_t)n * k * sizeof(int32_t), hipMemcpyDeviceToDevice);
    if (e == hipSuccess && upm)
      hipLaunchKernelGGL(k_niv_none, dim3(blocks(n * k, NWG)), dim3(NWG), 0, 0, n * k, dst);
    if (e == hipSuccess) e = hipGetLastError();
    nb.release(nullptr, nullptr);
    if (e != hipSuccess) {
      msg = std::string("device niv: ") + hipGetErrorString(e);
      return PX_EHIP;
    }
    return flag ? -1 : PX_OK;  // -1: not converged within kMaxRounds
  };
  int rc = run(false, dp, dr, d_niv);
  if (rc == PX_OK) {  // planted-chain check on the down map
    Bufs cb;
    const int64_t* d_cp = cb.put(cp);
    const int32_t* d_cr = cb.put(cr);
    int bad = INT32_MAX;
    hipError_t e = cb.err;
    if (e == hipSuccess) e = hipMemcpy(d_flag + 1, &bad, sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_niv_check, dim3(blocks(n, NWG)), dim3(NWG), 0, 0, n, (int)k, d_cp, d_cr, d_cor, d_coff,
                         d_niv, d_flag + 1);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(&bad, d_flag + 1, sizeof(int), hipMemcpyDeviceToHost);
    cb.release(nullptr, nullptr);
    if (e != hipSuccess) {
      msg = std::string("device niv check: ") + hipGetErrorString(e);
      rc = PX_EHIP;
    } else if (bad < n) {
      const int32_t x = P.node_of_row[bad];
      msg = "chain " + std::to_string(P.chain_of[x]) + " is not totally ordered at position " +
            std::to_string(P.chain_pos[x]) + " (node " + std::to_string(x) + ")";
      rc = PX_ECHAIN;
    }
  }
  if (rc == PX_OK && want_up) rc = run(true, up, ur, d_up);
  if (rc == PX_OK) {  // host copies for the level schedules and the walk tables
    P.niv.resize((size_t)n * k);
    hipError_t e = hipMemcpy(P.niv.data(), d_niv, (size_t)n * k * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && want_up) {
      P.niv_up.resize((size_t)n * k);
      e = hipMemcpy(P.niv_up.data(), d_up, (size_t)n * k * sizeof(int32_t), hipMemcpyDeviceToHost);
    }
    if (e != hipSuccess) {
      msg = std::string("device niv download: ") + hipGetErrorString(e);
      rc = PX_EHIP;
    }
  }
  if (rc != PX_OK) {
    P.niv.clear();
    P.niv_up.clear();
    b.release(nullptr, nullptr);
    (void)hipGetLastError();
    return rc;
  }
  b.release(d_niv, d_up);
  *out_niv = d_niv;
  *out_up = d_up;
  if (rounds) *rounds = total_rounds;
  return PX_OK;
}

}  // namespace px
