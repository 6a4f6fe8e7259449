// The niv maps computed on the device (dense rows); see niv_device.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "prep.h"

namespace px {

// Computes P.niv (and P.niv_up if want_up) for the chains already in P, on
// the current device, as the fixed point of the chain recursion, and checks
// planted chains.  rptr / ridx: the parent lists (reversed CSR).  On success
// returns PX_OK, leaves the device copies in *out_niv / *out_up (hipMalloc'd,
// owned by the caller; rows as in P, -1 = none), fills P.niv / P.niv_up on the
// host and the number of rounds taken.  Returns -1 (nothing allocated, nothing
// changed) where the rounds do not settle within their cap, so that the caller
// runs the host recursion instead; PX_ECHAIN for a chain that is not totally
// ordered; PX_ENOMEM / PX_EHIP with msg set.
int device_niv(Prep& P, const int64_t* indptr, const int32_t* indices, const std::vector<int64_t>& rptr,
               const std::vector<int32_t>& ridx, bool want_up, int32_t** out_niv, int32_t** out_up, int* rounds,
               std::string& msg);

// The niv maps as rows of their finite entries (P.sparse), on the current
// device, height after height (see niv_sparse.hip).  On success returns
// PX_OK, fills P.nivp / P.nivr (and the dual map's if want_up) on the host and
// leaves device copies in out_ptr[m] / out_rows[m] (hipMalloc'd, owned by the
// caller).  Returns -1 (nothing kept) for a node with more than 64 neighbours
// or where device memory runs out, so that the host recursion runs instead;
// PX_ECHAIN for a chain that is not totally ordered; PX_EHIP with msg set.
int device_niv_sparse(Prep& P, const int64_t* indptr, const int32_t* indices, const std::vector<int64_t>& rptr,
                      const std::vector<int32_t>& ridx, const Heights& heights, bool want_up, int64_t* out_ptr[2],
                      int32_t* out_rows[2], std::string& msg);

// The U-dependency levels of one map on the current device from the map's
// device rows (dense [n, k] nv, or sparse ep / er), copied into lev: in one
// persistent launch over the rows in height order (hnodes) polling the levels
// they read; if a wait gives up there (or POSETX_UDEP=heights), height after
// height (hptr: runs of narrow heights in one single-workgroup launch, wider
// heights a launch each).  Returns PX_OK, or -1 on any HIP error (the caller
// computes them on the host instead).
int device_udep_levels(const Prep& P, const std::vector<int64_t>& hptr, const std::vector<int32_t>& hnodes,
                       const int32_t* nv, const int64_t* ep, const int32_t* er, std::vector<int32_t>& lev);

// Rows of a dense device map in a given order, on the current device (all
// pointers device memory): dst[i * k + j] = src[rows[i] * k + j] and
// nodes[i] = node_of_row[rows[i]] for i < cnt.  Returns the launch status.
hipError_t device_gather_rows(const int32_t* src, int k, const int32_t* rows, int64_t cnt,
                              const int32_t* node_of_row, int32_t* dst, int32_t* nodes);

}  // namespace px
