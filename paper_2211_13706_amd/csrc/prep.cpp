// One-time host preprocessing of a poset; see prep.h.
#include "prep.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>

#include "posetx.h"

namespace px {
namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// A fixed team of threads (the caller's included) that runs fn(thread, lo, hi)
// over chunks of [0, count) per call of run(); workers persist across calls.
class Workers {
 public:
  explicit Workers(int nt) : nt_(std::max(1, nt)) {
    for (int t = 1; t < nt_; ++t) th_.emplace_back([this, t] { loop(t); });
  }
  ~Workers() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
      ++gen_;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  int size() const { return nt_; }
  using Fn = std::function<void(int, int64_t, int64_t)>;
  void run(int64_t count, int64_t chunk, const Fn& fn) {
    if (nt_ == 1 || count <= chunk) {
      if (count > 0) fn(0, 0, count);
      return;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      fn_ = &fn;
      count_ = count;
      chunk_ = chunk;
      next_.store(0);
      busy_ = nt_ - 1;
      ++gen_;
    }
    cv_.notify_all();
    work(0);
    std::unique_lock<std::mutex> lk(mu_);
    done_.wait(lk, [this] { return busy_ == 0; });
    fn_ = nullptr;
  }

 private:
  void work(int t) {
    for (;;) {
      const int64_t lo = next_.fetch_add(chunk_);
      if (lo >= count_) return;
      (*fn_)(t, lo, std::min(lo + chunk_, count_));
    }
  }
  void loop(int t) {
    uint64_t seen = 0;
    for (;;) {
      std::unique_lock<std::mutex> lk(mu_);
      cv_.wait(lk, [&] { return gen_ != seen; });
      seen = gen_;
      if (stop_) return;
      lk.unlock();
      work(t);
      lk.lock();
      if (--busy_ == 0) done_.notify_one();
    }
  }
  int nt_;
  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable cv_, done_;
  uint64_t gen_ = 0;
  bool stop_ = false;
  int busy_ = 0;
  const Fn* fn_ = nullptr;
  int64_t count_ = 0, chunk_ = 1;
  std::atomic<int64_t> next_{0};
};

// Threads for the host recursion by heights: up to 16; one for small posets
// and for posets whose heights hold fewer than 256 rows on average (the rows
// of a narrow height run on the calling thread anyway).  POSETX_PREP_THREADS
// overrides (1..64).
int prep_threads(int64_t n, int64_t heights) {
  if (const char* v = std::getenv("POSETX_PREP_THREADS")) {
    const int t = std::atoi(v);
    if (t >= 1) return std::min(t, 64);
  }
  if (n < (1 << 15) || n < 256 * heights) return 1;
  const unsigned hc = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(16u, hc ? hc : 1u));
}

// Nodes grouped by height, ascending node id within a height: for the down
// map the longest path down to a leaf (mir), for the dual map the longest path
// up to a root.  Rows of one height depend only on rows of lower heights in
// the recursion of Theorem 5 and in the U-dependency levels.
void by_height(int64_t n, const int64_t* indptr, const int32_t* indices, const std::vector<int32_t>& order,
               const std::vector<int32_t>& mir, bool up, std::vector<int64_t>& hptr, std::vector<int32_t>& hnodes) {
  std::vector<int32_t> height;
  if (!up) {
    height = mir;
  } else {
    height.assign(n, 0);
    for (int64_t h = n; h-- > 0;) {
      const int32_t x = order[h];
      for (int64_t e = indptr[x]; e < indptr[x + 1]; ++e)
        height[indices[e]] = std::max(height[indices[e]], height[x] + 1);
    }
  }
  int32_t H = 0;
  for (int64_t x = 0; x < n; ++x) H = std::max(H, height[x] + 1);
  hptr.assign(H + 1, 0);
  for (int64_t x = 0; x < n; ++x) hptr[height[x] + 1]++;
  for (int32_t h = 0; h < H; ++h) hptr[h + 1] += hptr[h];
  hnodes.resize(n);
  std::vector<int64_t> fill(hptr.begin(), hptr.end() - 1);
  for (int64_t x = 0; x < n; ++x) hnodes[fill[height[x]]++] = (int32_t)x;
}

// Parent lists (reversed CSR) of the child lists, each in ascending parent
// order.  Graphs of 2^22 edges or more (or any, with POSETX_PREP_THREADS)
// split the targets into ranges, one per thread: every thread reads all edges
// in order and handles those into its range, so the lists are the same for any
// thread count.
void reverse_csr(int64_t n, const int64_t* indptr, const int32_t* indices, std::vector<int64_t>& rptr,
                 std::vector<int32_t>& ridx) {
  rptr.assign(n + 1, 0);
  const int64_t m = indptr[n];
  const unsigned hc = std::thread::hardware_concurrency();
  int nt = m >= ((int64_t)1 << 22) ? (int)std::max(1u, std::min(16u, hc ? hc : 1u)) : 1;
  if (const char* v = std::getenv("POSETX_PREP_THREADS"))
    if (std::atoi(v) >= 1) nt = std::min(std::atoi(v), 64);
  auto each = [&](const std::function<void(int32_t, int32_t)>& fn) {
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
      th.emplace_back([&, t] { fn((int32_t)(n * t / nt), (int32_t)(n * (t + 1) / nt)); });
    for (auto& x : th) x.join();
  };
  if (nt == 1) {
    for (int64_t e = 0; e < m; ++e) rptr[indices[e] + 1]++;
  } else {
    each([&](int32_t v0, int32_t v1) {
      for (int64_t e = 0; e < m; ++e) {
        const int32_t v = indices[e];
        if (v >= v0 && v < v1) rptr[v + 1]++;
      }
    });
  }
  for (int64_t i = 0; i < n; ++i) rptr[i + 1] += rptr[i];
  ridx.resize(m);
  std::vector<int64_t> fill(rptr.begin(), rptr.end() - 1);
  if (nt == 1) {
    for (int64_t u = 0; u < n; ++u)
      for (int64_t e = indptr[u]; e < indptr[u + 1]; ++e) ridx[fill[indices[e]]++] = (int32_t)u;
  } else {
    each([&](int32_t v0, int32_t v1) {
      for (int64_t u = 0; u < n; ++u)
        for (int64_t e = indptr[u]; e < indptr[u + 1]; ++e) {
          const int32_t v = indices[e];
          if (v >= v0 && v < v1) ridx[fill[v]++] = (int32_t)u;
        }
    });
  }
}

// Maximum matching of the bipartite graph with an edge (v1, u2) per DAG edge v -> u
// (Alg. 1): Hopcroft-Karp with iterative searches.  next[v] = u when matched.
void hopcroft_karp(int64_t n, const int64_t* indptr, const int32_t* indices, std::vector<int32_t>& matchL,
                   std::vector<int32_t>& matchR) {
  matchL.assign(n, -1);
  matchR.assign(n, -1);
  for (int64_t v = 0; v < n; ++v)  // greedy start
    for (int64_t e = indptr[v]; e < indptr[v + 1]; ++e)
      if (matchR[indices[e]] < 0) {
        matchL[v] = indices[e];
        matchR[indices[e]] = (int32_t)v;
        break;
      }
  const int32_t INF = INT32_MAX;
  std::vector<int32_t> dist(n), queue(n), stack, via;
  std::vector<int64_t> it(n);
  for (;;) {
    int64_t qh = 0, qt = 0;
    for (int64_t v = 0; v < n; ++v) {
      if (matchL[v] < 0) {
        dist[v] = 0;
        queue[qt++] = (int32_t)v;
      } else {
        dist[v] = INF;
      }
    }
    bool found = false;
    while (qh < qt) {
      int32_t v = queue[qh++];
      for (int64_t e = indptr[v]; e < indptr[v + 1]; ++e) {
        int32_t w = matchR[indices[e]];
        if (w < 0) {
          found = true;
        } else if (dist[w] == INF) {
          dist[w] = dist[v] + 1;
          queue[qt++] = w;
        }
      }
    }
    if (!found) break;
    for (int64_t v = 0; v < n; ++v) it[v] = indptr[v];
    for (int64_t s = 0; s < n; ++s) {
      if (matchL[s] >= 0) continue;
      stack.assign(1, (int32_t)s);
      via.clear();
      while (!stack.empty()) {
        int32_t x = stack.back();
        if (it[x] == indptr[x + 1]) {
          dist[x] = INF;
          stack.pop_back();
          if (!via.empty()) via.pop_back();
          continue;
        }
        int32_t u = indices[it[x]++];
        int32_t w = matchR[u];
        if (w < 0) {
          via.push_back(u);
          for (size_t d = stack.size(); d-- > 0;) {
            matchL[stack[d]] = via[d];
            matchR[via[d]] = stack[d];
          }
          break;
        }
        if (dist[w] == dist[x] + 1) {
          via.push_back(u);
          stack.push_back(w);
        }
      }
    }
  }
}

}  // namespace

int preprocess(int64_t n, const int64_t* indptr, const int32_t* indices, const int32_t* chain_of,
               const int32_t* chain_pos, bool want_up, bool mirsky_schedule, bool want_sparse, Prep& P,
               std::string& msg, const NivHook* niv_hook, bool min_chains, const LevelHook* level_hook) {
  double t0 = now_s();
  if (n < 0 || n >= INT32_MAX) {
    msg = "n out of range";
    return PX_EINVAL;
  }
  if (n > 0 && (!indptr || (!indices && indptr[n] > 0))) {
    msg = "null CSR array";
    return PX_EINVAL;
  }
  if ((chain_of == nullptr) != (chain_pos == nullptr)) {
    msg = "chain_of and chain_pos must both be given or both be NULL";
    return PX_EINVAL;
  }
  P = Prep();
  P.n = n;
  if (n == 0) {
    P.chain_off.assign(1, 0);
    P.lev_down_ptr.assign(1, 0);
    P.lev_up_ptr.assign(1, 0);
    return PX_OK;
  }
  if (indptr[0] != 0) {
    msg = "indptr[0] must be 0";
    return PX_EINVAL;
  }
  for (int64_t u = 0; u < n; ++u)
    if (indptr[u + 1] < indptr[u]) {
      msg = "indptr is not non-decreasing";
      return PX_EINVAL;
    }
  const int64_t m = indptr[n];
  P.edges = m;
  for (int64_t u = 0; u < n; ++u)
    for (int64_t e = indptr[u]; e < indptr[u + 1]; ++e) {
      int32_t v = indices[e];
      if (v < 0 || v >= n) {
        msg = "edge target out of range at edge " + std::to_string(e);
        return PX_EINVAL;
      }
      if (v == u) {
        msg = "self-loop at node " + std::to_string(u);
        return PX_EINVAL;
      }
    }

  // Topological order, children before parents (Kahn; leaves first as in Alg. 6).
  std::vector<int64_t> rptr;
  std::vector<int32_t> ridx;
  reverse_csr(n, indptr, indices, rptr, ridx);
  std::vector<int32_t> order;
  order.reserve(n);
  // a node's remaining out-degree and its longest path down to a leaf (Mirsky
  // level) side by side: one cache line per visit of a parent
  struct alignas(16) KahnState {
    int64_t deg;
    int32_t mir;
  };
  std::vector<KahnState> st(n);
  for (int64_t u = 0; u < n; ++u) {
    st[u] = {indptr[u + 1] - indptr[u], 0};
    if (st[u].deg == 0) order.push_back((int32_t)u);
  }
  for (size_t h = 0; h < order.size(); ++h) {
    const int32_t v = order[h];
    const int32_t up = st[v].mir + 1;
    for (int64_t e = rptr[v]; e < rptr[v + 1]; ++e) {
      KahnState& s = st[ridx[e]];
      s.mir = std::max(s.mir, up);
      if (--s.deg == 0) order.push_back(ridx[e]);
    }
  }
  if ((int64_t)order.size() != n) {
    msg = "the graph has a directed cycle";
    return PX_ECYCLE;
  }
  std::vector<int32_t> mir(n);
  for (int64_t v = 0; v < n; ++v) {
    mir[v] = st[v].mir;
    P.mirsky = std::max<int64_t>(P.mirsky, mir[v] + 1);
  }
  std::vector<KahnState>().swap(st);
  double t1 = now_s();
  P.t_validate = t1 - t0;

  // Chain decomposition (Definition 1): planted or by maximum matching (Alg. 1).
  P.chain_of.resize(n);
  P.chain_pos.resize(n);
  if (chain_of) {
    P.planted = true;
    int64_t k = 0;
    for (int64_t x = 0; x < n; ++x) {
      if (chain_of[x] < 0 || chain_pos[x] < 0) {
        msg = "negative chain id or position at node " + std::to_string(x);
        return PX_EINVAL;
      }
      k = std::max<int64_t>(k, (int64_t)chain_of[x] + 1);
    }
    P.k = k;
    std::copy(chain_of, chain_of + n, P.chain_of.begin());
    std::copy(chain_pos, chain_pos + n, P.chain_pos.begin());
  } else {
    std::vector<int32_t> matchL, matchR;
    hopcroft_karp(n, indptr, indices, matchL, matchR);
    int32_t k = 0;
    std::vector<int32_t> path;
    for (int64_t top = 0; top < n; ++top) {
      if (matchR[top] >= 0) continue;  // someone's successor: not a chain top
      path.clear();
      for (int32_t x = (int32_t)top; x >= 0; x = matchL[x]) path.push_back(x);
      for (size_t i = 0; i < path.size(); ++i) {
        P.chain_of[path[i]] = k;
        P.chain_pos[path[i]] = (int32_t)(path.size() - 1 - i);
      }
      ++k;
    }
    P.k = k;
    P.path_cover = k;
    if (min_chains) {  // refine to as many chains as the width
      std::vector<int32_t> co, cp;
      const int64_t km = min_chain_decomposition(n, indptr, indices, matchL, co, cp);
      if (km > 0 && km <= k) {
        P.chain_of.swap(co);
        P.chain_pos.swap(cp);
        P.k = km;
      }
    }
  }
  const int64_t k = P.k;
  P.chain_off.assign(k + 1, 0);
  for (int64_t x = 0; x < n; ++x) P.chain_off[P.chain_of[x] + 1]++;
  for (int64_t c = 0; c < k; ++c) {
    P.max_chain = std::max<int64_t>(P.max_chain, P.chain_off[c + 1]);
    P.chain_off[c + 1] += P.chain_off[c];
  }
  P.row_of_node.resize(n);
  P.node_of_row.assign(n, -1);
  P.chain_of_row.resize(n);
  for (int64_t x = 0; x < n; ++x) {
    int32_t c = P.chain_of[x];
    int64_t len = P.chain_off[c + 1] - P.chain_off[c];
    if (P.chain_pos[x] >= len) {
      msg = "chain position out of range at node " + std::to_string(x);
      return PX_EINVAL;
    }
    int32_t r = P.chain_off[c] + P.chain_pos[x];
    if (P.node_of_row[r] >= 0) {
      msg = "chain " + std::to_string(c) + " uses position " + std::to_string(P.chain_pos[x]) + " twice";
      return PX_EINVAL;
    }
    P.node_of_row[r] = (int32_t)x;
    P.row_of_node[x] = r;
    P.chain_of_row[r] = c;
  }
  double t2 = now_s();
  P.t_chains = t2 - t1;

  // niv by the recursion of Theorem 5 over rows in chain-major order.  Within a
  // chain, rows grow with the position, so the highest element of chain j below x
  // is the largest row of chain j reachable from x: a row-wise max over the
  // children, and x itself on its own chain.  The own-chain entry before x is
  // inserted must be the row just below x: this checks planted chains.
  auto chain_error = [&](int64_t x) {
    msg = "chain " + std::to_string(P.chain_of[x]) + " is not totally ordered at position " +
          std::to_string(P.chain_pos[x]) + " (node " + std::to_string(x) + ")";
    return PX_ECHAIN;
  };
  P.sparse = want_sparse || k > kSparseNivChains;
  int hook_rc = -1;
  if (!P.sparse && niv_hook && *niv_hook) hook_rc = (*niv_hook)(P, rptr, ridx, nullptr, msg);
  if (P.sparse && niv_hook && *niv_hook) {
    Heights hs;
    for (int m = 0; m < (want_up ? 2 : 1); ++m) by_height(n, indptr, indices, order, mir, m == 1, hs.ptr[m], hs.nodes[m]);
    hook_rc = (*niv_hook)(P, rptr, ridx, &hs, msg);
  }
  if (hook_rc > 0) return hook_rc;
  if (P.sparse && hook_rc == PX_OK) {
    // rows computed elsewhere
  } else if (!P.sparse && hook_rc == PX_OK) {
    // finite entries of the maps computed elsewhere, counted on a team of threads
    // (n = 2^23, k = 32: two maps of 2^28 entries)
    const unsigned hc = std::thread::hardware_concurrency();
    Workers team(P.niv.size() >= ((size_t)1 << 24) ? (int)std::max(1u, std::min(16u, hc ? hc : 1u)) : 1);
    for (int m = 0; m < 2; ++m) {
      const std::vector<int32_t>& v = m ? P.niv_up : P.niv;
      std::vector<int64_t> part(team.size(), 0);
      team.run((int64_t)v.size(), (int64_t)1 << 20, [&](int t, int64_t lo, int64_t hi) {
        int64_t c = 0;
        for (int64_t i = lo; i < hi; ++i) c += v[(size_t)i] >= 0;
        part[t] += c;
      });
      int64_t total = 0;
      for (int64_t c : part) total += c;
      (m ? P.nnz_niv_up : P.nnz_niv) = total;
    }
  } else if (!P.sparse) {
    // Rows of one height (the longest path down to a leaf; up to a root for
    // the dual map) depend only on lower ones, so a team of threads takes the
    // rows of a height together; the maps do not depend on the thread count.
    P.niv_rounds = 0;
    Workers team(prep_threads(n, P.mirsky));
    auto heights = [&](bool up, std::vector<int64_t>& hp, std::vector<int32_t>& hn) {
      by_height(n, indptr, indices, order, mir, up, hp, hn);
    };
    std::vector<int64_t> hptr;
    std::vector<int32_t> hnodes;
    P.niv.assign((size_t)n * k, -1);
    heights(false, hptr, hnodes);
    std::atomic<int64_t> bad{INT64_MAX};  // smallest node whose chain check fails
    for (size_t h = 0; h + 1 < hptr.size(); ++h) {
      team.run(hptr[h + 1] - hptr[h], 64, [&](int, int64_t lo, int64_t hi) {
        for (int64_t i = hptr[h] + lo; i < hptr[h] + hi; ++i) {
          const int32_t x = hnodes[i];
          const int32_t r = P.row_of_node[x];
          int32_t* R = &P.niv[(size_t)r * k];
          for (int64_t e = indptr[x]; e < indptr[x + 1]; ++e) {
            const int32_t* Rz = &P.niv[(size_t)P.row_of_node[indices[e]] * k];
            for (int64_t j = 0; j < k; ++j) R[j] = std::max(R[j], Rz[j]);
          }
          const int32_t c = P.chain_of[x];
          if (R[c] != (P.chain_pos[x] > 0 ? r - 1 : -1)) {
            int64_t cur = bad.load();
            while (x < cur && !bad.compare_exchange_weak(cur, x)) {
            }
          }
          R[c] = r;
        }
      });
      if (bad.load() != INT64_MAX) return chain_error(bad.load());
    }
    for (size_t i = 0; i < P.niv.size(); ++i) P.nnz_niv += P.niv[i] >= 0;
    if (want_up) {
      // Dual order: the lowest element of chain j above x is a row-wise min over parents.
      P.niv_up.assign((size_t)n * k, INT32_MAX);
      heights(true, hptr, hnodes);
      for (size_t h = 0; h + 1 < hptr.size(); ++h) {
        team.run(hptr[h + 1] - hptr[h], 64, [&](int, int64_t lo, int64_t hi) {
          for (int64_t i = hptr[h] + lo; i < hptr[h] + hi; ++i) {
            const int32_t x = hnodes[i];
            const int32_t r = P.row_of_node[x];
            int32_t* R = &P.niv_up[(size_t)r * k];
            for (int64_t e = rptr[x]; e < rptr[x + 1]; ++e) {
              const int32_t* Rp = &P.niv_up[(size_t)P.row_of_node[ridx[e]] * k];
              for (int64_t j = 0; j < k; ++j) R[j] = std::min(R[j], Rp[j]);
            }
            R[P.chain_of[x]] = r;
          }
        });
      }
      for (size_t i = 0; i < P.niv_up.size(); ++i) {
        if (P.niv_up[i] == INT32_MAX) P.niv_up[i] = -1;
        P.nnz_niv_up += P.niv_up[i] >= 0;
      }
    }
  } else {
    // The same recursion on rows that list only their finite entries (nnz(N)
    // instead of n * k storage): a row is the per-chain max (min for the dual
    // map) over its children's (parents') rows, merged through a k-wide
    // scratch row, plus its own entry.  Rows depend only on rows of lower
    // height (the longest path down to a leaf, or up to a root for the dual
    // map), so the rows of one height are merged by a team of threads into
    // per-thread buffers and then appended to a pool; at the end the rows are
    // laid out by row.  The maps do not depend on the number of threads.
    Workers team(prep_threads(n, P.mirsky));
    const int nt = team.size();
    struct Local {
      std::vector<int32_t> acc, touched, buf;
      std::vector<int64_t> rec;  // (row, offset in buf, length) triples
    };
    std::vector<Local> loc(nt);
    for (Local& L : loc) L.acc.assign(k, -1);
    auto build = [&](bool up) -> int {
      // the nodes of each height, ascending node id
      std::vector<int64_t> hptr;
      std::vector<int32_t> hnodes;
      by_height(n, indptr, indices, order, mir, up, hptr, hnodes);
      const int32_t H = (int32_t)hptr.size() - 1;
      std::vector<int64_t> st(n), ln(n);
      std::vector<int32_t> pool;
      pool.reserve((size_t)n * 4);
      std::atomic<int64_t> bad{INT64_MAX};  // smallest node whose chain check fails
      std::atomic<bool> oom{false};
      const Workers::Fn merge = [&](int t, int64_t lo, int64_t hi) {
        Local& L = loc[t];
        try {
          for (int64_t i = lo; i < hi; ++i) {
            const int32_t x = hnodes[i];
            const int32_t r = P.row_of_node[x];
            L.touched.clear();
            const int64_t e0 = up ? rptr[x] : indptr[x], e1 = up ? rptr[x + 1] : indptr[x + 1];
            for (int64_t e = e0; e < e1; ++e) {
              const int32_t rz = P.row_of_node[up ? ridx[e] : indices[e]];
              for (int64_t j = st[rz], je = st[rz] + ln[rz]; j < je; ++j) {
                const int32_t v = pool[j];
                int32_t& a = L.acc[P.chain_of_row[v]];
                if (a < 0) {
                  L.touched.push_back(P.chain_of_row[v]);
                  a = v;
                } else {
                  a = up ? std::min(a, v) : std::max(a, v);
                }
              }
            }
            const int32_t c = P.chain_of[x];
            if (!up && L.acc[c] != (P.chain_pos[x] > 0 ? r - 1 : -1)) {
              int64_t cur = bad.load();
              while (x < cur && !bad.compare_exchange_weak(cur, x)) {
              }
            }
            if (L.acc[c] < 0) L.touched.push_back(c);
            L.acc[c] = r;
            std::sort(L.touched.begin(), L.touched.end());
            L.rec.push_back(r);
            L.rec.push_back((int64_t)L.buf.size());
            L.rec.push_back((int64_t)L.touched.size());
            for (int32_t j : L.touched) {
              L.buf.push_back(L.acc[j]);
              L.acc[j] = -1;
            }
          }
        } catch (const std::bad_alloc&) {
          oom = true;
        }
      };
      for (int32_t h = 0; h < H; ++h) {
        team.run(hptr[h + 1] - hptr[h], 64, [&](int t, int64_t lo, int64_t hi) { merge(t, hptr[h] + lo, hptr[h] + hi); });
        if (oom) throw std::bad_alloc();
        if (bad.load() != INT64_MAX) return chain_error(bad.load());
        for (Local& L : loc) {  // append this height's rows to the pool
          const int64_t base = (int64_t)pool.size();
          pool.insert(pool.end(), L.buf.begin(), L.buf.end());
          for (size_t q = 0; q < L.rec.size(); q += 3) {
            st[L.rec[q]] = base + L.rec[q + 1];
            ln[L.rec[q]] = L.rec[q + 2];
          }
          L.buf.clear();
          L.rec.clear();
        }
      }
      std::vector<int64_t>& ptr = P.nivp[up ? 1 : 0];
      std::vector<int32_t>& ent = P.nivr[up ? 1 : 0];
      ptr.assign(n + 1, 0);
      for (int64_t r = 0; r < n; ++r) ptr[r + 1] = ptr[r] + ln[r];
      ent.resize(pool.size());
      for (int64_t r = 0; r < n; ++r) std::copy_n(pool.begin() + st[r], ln[r], ent.begin() + ptr[r]);
      (up ? P.nnz_niv_up : P.nnz_niv) = (int64_t)ent.size();
      return PX_OK;
    };
    int rc = build(false);
    if (rc == PX_OK && want_up) rc = build(true);
    if (rc != PX_OK) return rc;
  }
  double t3 = now_s();
  P.t_niv = t3 - t2;

  // Level schedules.  U-dependency levels: the solve at x reads the rows
  // niv_j(x), j != id(x), all strictly below x, so level(x) = 1 + the largest
  // level among them.  Mirsky levels (§4) are the longest path to a leaf.
  auto bucket = [n](const std::vector<int32_t>& lev, std::vector<int32_t>& ptr, std::vector<int32_t>& rows) {
    int32_t L = 0;
    for (int64_t r = 0; r < n; ++r) L = std::max(L, lev[r] + 1);
    ptr.assign(L + 1, 0);
    for (int64_t r = 0; r < n; ++r) ptr[lev[r] + 1]++;
    for (int32_t l = 0; l < L; ++l) ptr[l + 1] += ptr[l];
    rows.resize(n);
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t r = 0; r < n; ++r) rows[fill[lev[r]]++] = (int32_t)r;
  };
  // (the entries of a row lie at lower heights, so a height's rows are taken
  // together by a thread team, as in the recursion)
  Workers lteam(prep_threads(n, P.mirsky));
  auto udep_levels = [&](bool up, std::vector<int32_t>& lev) {
    lev.assign(n, 0);
    const std::vector<int32_t>& nv = up ? P.niv_up : P.niv;
    std::vector<int64_t> hptr;
    std::vector<int32_t> hnodes;
    by_height(n, indptr, indices, order, mir, up, hptr, hnodes);
    if (level_hook && *level_hook && (*level_hook)(P, up, hptr, hnodes, lev) == PX_OK) return;
    for (size_t h = 0; h + 1 < hptr.size(); ++h) {
      lteam.run(hptr[h + 1] - hptr[h], 256, [&](int, int64_t lo, int64_t hi) {
        for (int64_t i = hptr[h] + lo; i < hptr[h] + hi; ++i) {
          const int32_t r = P.row_of_node[hnodes[i]];
          const int32_t* R = P.sparse ? P.nivr[up ? 1 : 0].data() + P.nivp[up ? 1 : 0][r] : &nv[(size_t)r * k];
          const int64_t len = P.sparse ? P.nivp[up ? 1 : 0][r + 1] - P.nivp[up ? 1 : 0][r] : k;
          int32_t l = 0;
          for (int64_t j = 0; j < len; ++j)
            if (R[j] >= 0 && R[j] != r) l = std::max(l, lev[R[j]] + 1);
          lev[r] = l;
        }
      });
    }
  };
  std::vector<int32_t> ud;
  udep_levels(false, ud);
  for (int64_t r = 0; r < n; ++r) P.udep = std::max<int64_t>(P.udep, ud[r] + 1);
  if (mirsky_schedule) {
    P.lev_down.resize(n);
    for (int64_t x = 0; x < n; ++x) P.lev_down[P.row_of_node[x]] = mir[x];
  } else {
    P.lev_down.swap(ud);
  }
  bucket(P.lev_down, P.lev_down_ptr, P.lev_down_rows);
  if (want_up) {
    if (mirsky_schedule) {
      std::vector<int32_t> comir(n, 0);  // longest path up to a root
      for (int64_t h = n; h-- > 0;) {
        int32_t x = order[h];
        for (int64_t e = indptr[x]; e < indptr[x + 1]; ++e)
          comir[indices[e]] = std::max(comir[indices[e]], comir[x] + 1);
      }
      P.lev_up.resize(n);
      for (int64_t x = 0; x < n; ++x) P.lev_up[P.row_of_node[x]] = comir[x];
    } else {
      udep_levels(true, P.lev_up);
    }
    bucket(P.lev_up, P.lev_up_ptr, P.lev_up_rows);
  } else {
    P.lev_up_ptr.assign(1, 0);
  }
  P.t_levels = now_s() - t3;
  return PX_OK;
}

}  // namespace px
