// Host-side, one-time preprocessing of a poset (§2.3-§2.4 and §4 of the paper):
// validation, topological order, chain decomposition, chain-major renumbering,
// the niv map and its dual, and the level schedules of the Möbius solves.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace px {

struct Prep {
  int64_t n = 0, k = 0, edges = 0;
  bool planted = false;
  std::vector<int32_t> chain_of, chain_pos;       // per node
  std::vector<int32_t> chain_off;                 // k+1 row offsets of the chains
  std::vector<int32_t> row_of_node, node_of_row;  // chain-major renumbering
  std::vector<int32_t> chain_of_row;              // per row
  // niv[r*k + j]: row of the highest element of chain j below row r, or -1.
  std::vector<int32_t> niv;
  // niv_up[r*k + j]: row of the lowest element of chain j above row r, or -1.
  std::vector<int32_t> niv_up;
  // Sparse form (sparse == true; niv and niv_up then stay empty): the finite
  // entries of row r of map m (0 = niv, 1 = niv_up) are
  // nivr[m][nivp[m][r] .. nivp[m][r+1]), in ascending chain order, which in the
  // chain-major numbering is ascending row order.
  bool sparse = false;
  std::vector<int64_t> nivp[2];
  std::vector<int32_t> nivr[2];
  // level schedules: rows of level l are lev_rows[lev_ptr[l] .. lev_ptr[l+1])
  std::vector<int32_t> lev_down, lev_up;          // level per row
  std::vector<int32_t> lev_down_ptr, lev_down_rows, lev_up_ptr, lev_up_rows;
  int64_t nnz_niv = 0, nnz_niv_up = 0, max_chain = 0, mirsky = 0, udep = 0;
  int64_t path_cover = 0;  // chains of the matching's path cover (Alg. 1), before any refinement
  int32_t niv_rounds = 0;  // rounds of a device computation of niv (0: the host recursion)
  double t_validate = 0, t_chains = 0, t_niv = 0, t_levels = 0;
};

// Decompositions with more chains than this keep the niv maps sparse.
constexpr int64_t kSparseNivChains = 256;

// The nodes of every height (longest path down to a leaf for map 0, up to a
// root for map 1), height after height: nodes[m][ptr[m][h] .. ptr[m][h + 1]).
struct Heights {
  std::vector<int64_t> ptr[2];
  std::vector<int32_t> nodes[2];
};

// Computes the niv maps elsewhere (on a device) once the chains are known,
// given the parent lists: returns PX_OK with P.niv (and P.niv_up) filled, or
// for sparse rows (P.sparse; heights non-null) P.nivp / P.nivr, -1 to let the
// host recursion run instead, or an error status with msg set.
using NivHook = std::function<int(Prep& P, const std::vector<int64_t>& rptr, const std::vector<int32_t>& ridx,
                                  const Heights* heights, std::string& msg)>;

// A minimum chain decomposition (as many chains as the width) starting from
// the path cover next[v] (the element after v on its path, -1 at a path's
// end; see chains.cpp).  Returns the number of chains with chain_of /
// chain_pos filled (position 0 the lowest element), or -1 where the network
// would not fit 32-bit indices.
int64_t min_chain_decomposition(int64_t n, const int64_t* indptr, const int32_t* indices,
                                const std::vector<int32_t>& next, std::vector<int32_t>& chain_of,
                                std::vector<int32_t>& chain_pos);

// Computes the U-dependency levels of one map elsewhere (on a device, where
// the map already is): lev[r] = 1 + the largest level among the other-chain
// entries of row r (0 without any), rows taken height by height (hptr /
// hnodes as in Heights).  Returns PX_OK with lev filled (n entries) or -1 to
// let the host compute them.
using LevelHook = std::function<int(const Prep& P, bool up, const std::vector<int64_t>& hptr,
                                    const std::vector<int32_t>& hnodes, std::vector<int32_t>& lev)>;

// Returns a px_status value; on failure `msg` says why.  want_sparse forces
// the sparse form of the niv maps; niv_hook (nullable) is tried for dense ones.
// min_chains: without planted chains, refine the matching's path cover to a
// minimum chain decomposition.
int preprocess(int64_t n, const int64_t* indptr, const int32_t* indices, const int32_t* chain_of,
               const int32_t* chain_pos, bool want_up, bool mirsky_schedule, bool want_sparse, Prep& out,
               std::string& msg, const NivHook* niv_hook = nullptr, bool min_chains = false,
               const LevelHook* level_hook = nullptr);

}  // namespace px
