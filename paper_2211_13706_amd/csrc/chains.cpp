// Minimum chain decomposition of a DAG (§2.3, Theorem 2: the fewest chains
// equal the width).  The path cover of Alg. 1 matches on the edges only, so it
// can need more chains than the width when the edge set is not transitively
// closed; §4 names better decompositions as the lever on the cost, which grows
// with k.
//
// Method: minimum flow with a lower bound of one unit on every vertex.  The
// network has a source s, a sink t and per vertex v an arc v_in -> v_out
// (lower bound 1); s -> v_in and v_out -> t for every v, and u_out -> v_in for
// every DAG edge u -> v (v below u); all upper bounds are infinite.  A unit of
// flow is a path of the DAG from a top to a bottom, paths may share vertices,
// and a feasible flow covers every vertex.  Its minimum value is the width
// (the min-flow / max-antichain duality of Dilworth's theorem in Fulkerson's
// form, here on the DAG's own edges: flow can pass through a vertex that
// another path covers, which is what lets a chain skip elements).
//
// The flow starts as the given path cover (value = its number of paths) and
// is decreased by a maximum flow from t to s in the residual network (Dinic):
// every original arc a -> b with flow f and lower bound l gives the residual
// arcs a -> b (infinite) and b -> a (capacity f - l).  Paths of the final flow
// are then taken one unit at a time from s, and each vertex joins the chain of
// the first path that reaches it; the vertices of one path are totally
// ordered, so every chain is, and since no partition has fewer chains than the
// width, exactly that many chains are non-empty.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "prep.h"

namespace px {

namespace {

constexpr int64_t kInf = INT64_MAX / 4;

struct Net {
  // original arcs: from, to, lower bound, flow; residual arc 2e runs from -> to
  // (capacity infinite), 2e + 1 runs to -> from (capacity flow - lower)
  std::vector<int32_t> from, to;
  std::vector<int8_t> lower;
  std::vector<int64_t> flow;
  std::vector<int64_t> adj_ptr;  // residual arcs leaving each node
  std::vector<int32_t> adj;

  int32_t head(int32_t ra) const { return (ra & 1) ? from[ra >> 1] : to[ra >> 1]; }
  int64_t cap(int32_t ra) const { return (ra & 1) ? flow[ra >> 1] - lower[ra >> 1] : kInf; }
  void push(int32_t ra, int64_t x) {
    if (ra & 1)
      flow[ra >> 1] -= x;
    else
      flow[ra >> 1] += x;
  }
  int32_t add(int32_t a, int32_t b, int8_t lb, int64_t f) {
    from.push_back(a);
    to.push_back(b);
    lower.push_back(lb);
    flow.push_back(f);
    return (int32_t)from.size() - 1;
  }
  void finish(int64_t nodes) {
    adj_ptr.assign(nodes + 1, 0);
    const int64_t m = (int64_t)from.size();
    for (int64_t e = 0; e < m; ++e) {
      adj_ptr[from[e] + 1]++;
      adj_ptr[to[e] + 1]++;
    }
    for (int64_t v = 0; v < nodes; ++v) adj_ptr[v + 1] += adj_ptr[v];
    adj.resize(2 * m);
    std::vector<int64_t> fill(adj_ptr.begin(), adj_ptr.end() - 1);
    for (int64_t e = 0; e < m; ++e) {
      adj[fill[from[e]]++] = (int32_t)(2 * e);
      adj[fill[to[e]]++] = (int32_t)(2 * e + 1);
    }
  }
};

// Maximum flow from src to dst on the residual network (Dinic: a BFS level
// graph, then blocking flow by iterative depth-first search).
int64_t dinic(Net& g, int64_t nodes, int32_t src, int32_t dst) {
  std::vector<int32_t> level(nodes), queue(nodes), stack, arcs;
  std::vector<int64_t> it(nodes);
  int64_t total = 0;
  for (;;) {
    std::fill(level.begin(), level.end(), -1);
    int64_t qh = 0, qt = 0;
    level[src] = 0;
    queue[qt++] = src;
    while (qh < qt && level[dst] < 0) {
      const int32_t a = queue[qh++];
      for (int64_t i = g.adj_ptr[a]; i < g.adj_ptr[a + 1]; ++i) {
        const int32_t ra = g.adj[i];
        const int32_t b = g.head(ra);
        if (level[b] < 0 && g.cap(ra) > 0) {
          level[b] = level[a] + 1;
          queue[qt++] = b;
        }
      }
    }
    if (level[dst] < 0) return total;
    for (int64_t v = 0; v < nodes; ++v) it[v] = g.adj_ptr[v];
    stack.assign(1, src);
    arcs.clear();
    while (!stack.empty()) {
      const int32_t a = stack.back();
      if (a == dst) {  // augment along the stack by its bottleneck
        int64_t x = kInf;
        for (int32_t ra : arcs) x = std::min(x, g.cap(ra));
        for (int32_t ra : arcs) g.push(ra, x);
        total += x;
        // back up to the first arc left without capacity
        size_t keep = arcs.size();
        for (size_t j = 0; j < arcs.size(); ++j)
          if (g.cap(arcs[j]) == 0) {
            keep = j;
            break;
          }
        arcs.resize(keep);
        stack.resize(keep + 1);
        continue;
      }
      bool advanced = false;
      for (; it[a] < g.adj_ptr[a + 1]; ++it[a]) {
        const int32_t ra = g.adj[it[a]];
        const int32_t b = g.head(ra);
        if (level[b] == level[a] + 1 && g.cap(ra) > 0) {
          arcs.push_back(ra);
          stack.push_back(b);
          advanced = true;
          break;
        }
      }
      if (!advanced) {  // dead end: leave it out of this phase
        level[a] = -1;
        stack.pop_back();
        if (!arcs.empty()) {
          arcs.pop_back();
          ++it[stack.back()];
        }
      }
    }
  }
}

}  // namespace

int64_t min_chain_decomposition(int64_t n, const int64_t* indptr, const int32_t* indices,
                                const std::vector<int32_t>& next, std::vector<int32_t>& chain_of,
                                std::vector<int32_t>& chain_pos) {
  // nodes: v_in = 2v, v_out = 2v + 1, s = 2n, t = 2n + 1; residual arcs 2 per arc
  const int64_t nodes = 2 * n + 2;
  if (nodes >= INT32_MAX || 2 * (3 * n + indptr[n]) >= INT32_MAX) return -1;
  const int32_t s = (int32_t)(2 * n), t = s + 1;
  Net g;
  const int64_t m = indptr[n];
  g.from.reserve(3 * n + m);
  g.to.reserve(3 * n + m);
  g.lower.reserve(3 * n + m);
  g.flow.reserve(3 * n + m);
  std::vector<int32_t> is_next(n, 0);  // some path continues into v
  for (int64_t v = 0; v < n; ++v)
    if (next[v] >= 0) is_next[next[v]] = 1;
  // the starting flow: one unit along every path of the cover
  for (int64_t v = 0; v < n; ++v) g.add(s, (int32_t)(2 * v), 0, is_next[v] ? 0 : 1);
  for (int64_t v = 0; v < n; ++v) g.add((int32_t)(2 * v), (int32_t)(2 * v + 1), 1, 1);
  for (int64_t v = 0; v < n; ++v) g.add((int32_t)(2 * v + 1), t, 0, next[v] >= 0 ? 0 : 1);
  for (int64_t u = 0; u < n; ++u) {
    bool used = false;  // the path's own edge carries its unit (once, even with duplicate edges)
    for (int64_t e = indptr[u]; e < indptr[u + 1]; ++e) {
      const int32_t v = indices[e];
      const bool mine = !used && v == next[u];
      used = used || mine;
      g.add((int32_t)(2 * u + 1), (int32_t)(2 * v), 0, mine ? 1 : 0);
    }
  }
  g.finish(nodes);
  dinic(g, nodes, t, s);

  // the paths of the final flow, one unit at a time from s
  std::vector<int64_t> out_it(nodes);
  for (int64_t v = 0; v < nodes; ++v) out_it[v] = g.adj_ptr[v];
  auto next_arc = [&](int32_t a) -> int32_t {  // an original arc out of a with flow left
    for (; out_it[a] < g.adj_ptr[a + 1]; ++out_it[a]) {
      const int32_t ra = g.adj[out_it[a]];
      if (!(ra & 1) && g.flow[ra >> 1] > 0) return ra >> 1;
    }
    return -1;
  };
  chain_of.assign(n, -1);
  chain_pos.assign(n, 0);
  std::vector<int32_t> path, mine;
  int64_t k = 0;
  for (int32_t e0; (e0 = next_arc(s)) >= 0;) {
    path.clear();
    int32_t e = e0;
    for (;;) {
      --g.flow[e];
      const int32_t b = g.to[e];
      if (b == t) break;
      if ((b & 1) == 0) path.push_back(b >> 1);  // entering v_in: vertex v
      e = next_arc(b);
      if (e < 0) return -1;  // flow not conserved: cannot happen
    }
    mine.clear();
    for (int32_t v : path)
      if (chain_of[v] < 0) mine.push_back(v);
    if (mine.empty()) continue;
    // the path runs from a top down to a bottom: position 0 is its lowest vertex
    for (size_t i = 0; i < mine.size(); ++i) {
      chain_of[mine[i]] = (int32_t)k;
      chain_pos[mine[i]] = (int32_t)(mine.size() - 1 - i);
    }
    ++k;
  }
  for (int64_t v = 0; v < n; ++v)
    if (chain_of[v] < 0) return -1;  // a vertex without flow: cannot happen
  return k;
}

}  // namespace px
