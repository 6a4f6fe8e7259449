/*
 * posetx — fast zeta and Möbius transforms on posets, MI355X (gfx950) native.
 *
 * C ABI of the library libposetx.so.  The operations follow Pegolotti,
 * Seifert and Püschel, "Fast Möbius and Zeta Transforms":
 *
 *   zeta      g(x) = Σ_{y ⪯ x} f(y)                    (Theorem 1, Corollary 1, §2.2)
 *   mobius    f(x) = Σ_{y ⪯ x} μ(y, x) g(y),  i.e. f = Z^{-1} g   (Theorem 1)
 *   adjoints  Z^T and M^T = (Z^T)^{-1}: the same transforms on the dual order
 *
 * computed through the factorisation Z = U V of §3: V is the chain-wise
 * prefix sum over a chain decomposition (Definition 1, §2.3) and U gathers,
 * for every element x and chain j, the prefix of chain j ending at
 * niv_j(x), the highest element of chain j below x (§2.4).  The Möbius
 * transform solves U y' = g by substitution and then takes the first
 * difference along every chain (V^{-1}, §3 and §4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - The poset is a DAG in CSR form: indices[indptr[u] .. indptr[u+1]) are the
 *    children of u; an edge u -> v means v ⪯ u (§2.1).  Duplicate edges and
 *    transitive edges are allowed, self-loops and cycles are errors.  The DAG
 *    need not be connected.
 *  - Function matrices are [n, B] row-major in NODE order: element (x, b) of a
 *    matrix with leading dimension ld (in elements, ld >= B) sits at
 *    ptr[x * ld + b].  They are DEVICE pointers on the poset's device and stay
 *    owned by the caller.
 *  - dtype PX_I64 computes in two's-complement int64 with wrap-around
 *    (exact modulo 2^64); PX_F32 computes in float32 with compensated chain
 *    scans and float64 accumulation of the gathered terms; PX_F64 in float64.
 *  - Compute calls are asynchronous on `stream` (a hipStream_t, NULL = the
 *    null stream) unless stated otherwise.  Argument errors are reported
 *    synchronously; launch errors as PX_EHIP.  The poset handle owns a device
 *    workspace that grows on demand (hipMalloc); call px_reserve() first to
 *    keep later calls allocation-free, e.g. before HIP graph capture.  Calls
 *    on one handle must be ordered (same stream or explicit synchronisation):
 *    they share that workspace.
 *  - Every call returns a px_status; px_last_error() gives a thread-local
 *    message for the last failure on the calling thread.  No C++ exception
 *    crosses this interface.
 *  - Execution paths (results agree to rounding; int64 bit for bit), read from
 *    the environment on every call: for a single poset with at most 64 chains
 *    and B >= 5, zeta, its adjoint and the residual of the refined Mobius
 *    transform complete the chain prefixes only at the rows the gather reads
 *    and never form the full prefix matrix (POSETX_COMPACT_NARROW=0 keeps that
 *    to B > 32, =2 extends it to every B); POSETX_WALK=rows forms it
 *    instead.  POSETX_SCAN=onepass selects the single-pass chain scan for the
 *    paths that form it, with POSETX_LB_SPIN bounding its waits (polls; 0
 *    makes every wait give up and sum its predecessors from the input).
 *    POSETX_TUNE_CACHE: see px_autotune.  The Möbius level solve runs every
 *    level in one persistent launch whose workgroups poll the values they
 *    read (bounded waits; a wait that gives up makes a one-workgroup fallback
 *    solve again): int64 with dense rows and B >= 5 by runs of rows
 *    (POSETX_USOLVE=levels: a launch per level, =direct: row by row), other
 *    dense solves row by row where the average level fits the resident
 *    wavefronts (POSETX_LEVEL_POLL=0: a launch per level, =2: always
 *    persistent); floating-point results do not depend on the choice.
 *    POSETX_FLOW_SPIN bounds the polls of each wait.  A persistent launch
 *    sizes its grid to what the device holds resident; other work running
 *    at the same time on other streams (another persistent solve, say) can
 *    keep some of its workgroups from starting, and its waits then give up
 *    after about 2 s and the fallback solves again: results stay the same,
 *    only slower.
 *    Posets with sparse niv rows (PX_BUILD_SPARSE_NIV, or more than 256
 *    chains) take the chain scan, a gather over their rows and a level solve
 *    with a launch per level, rows of more than 256 entries summed in fixed
 *    chunks.  Preprocessing:
 *    POSETX_PREP (see px_poset_build) and POSETX_PREP_THREADS (host threads of
 *    the recursion, default up to 16 for posets with wide levels).
 */
#ifndef POSETX_H
#define POSETX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct px_poset px_poset;
typedef struct px_batch px_batch;

typedef enum { PX_I64 = 0, PX_F32 = 1, PX_F64 = 2 } px_dtype;

typedef enum {
  PX_OK = 0,
  PX_EINVAL = 1,        /* bad argument: sizes, ranges, self-loop, malformed chains   */
  PX_ECYCLE = 2,        /* the edge list has a directed cycle                         */
  PX_ECHAIN = 3,        /* a planted chain is not totally ordered by the DAG          */
  PX_ENOMEM = 4,        /* host or device allocation failed                           */
  PX_EHIP = 5,          /* a HIP runtime call or kernel launch failed                 */
  PX_EUNSUPPORTED = 6,  /* operation not available for this handle or dtype           */
  PX_ENONFINITE = 7,    /* a floating-point Möbius result or refinement held NaN / Inf */
  PX_ENOTCONV = 8       /* refinement did not reach the tolerance                     */
} px_status;

/* px_poset_build flags */
#define PX_BUILD_HOST_ONLY 0x1u      /* preprocess on the host only: no device buffers, no compute  */
#define PX_BUILD_NO_ADJOINT 0x2u     /* skip the up-niv map and its levels (adjoints unavailable)   */
#define PX_BUILD_LEVELS_MIRSKY 0x4u  /* schedule Möbius over Mirsky antichains (§4, Alg. 5/6)       */
#define PX_BUILD_SPARSE_NIV 0x8u     /* keep the niv maps as rows of their finite entries (nnz(N)
                                        storage, §2.4) instead of dense [n, k] rows; automatic for
                                        more than 256 chains.  Such posets take gathers and level
                                        solves over their rows (long rows in fixed chunks) and
                                        cannot join a batch                                      */
#define PX_BUILD_MIN_CHAINS 0x10u    /* without planted chains: refine the matching's path cover
                                        (Alg. 1) to a minimum chain decomposition, as many chains
                                        as the width (Theorem 2), by minimum flow; k and so every
                                        transform's work can only drop (px_info.path_cover keeps
                                        the cover's count)                                      */

typedef struct {
  int64_t n;              /* elements                                                   */
  int64_t k;              /* chains in the decomposition                                */
  int64_t edges;          /* CSR edges                                                  */
  int64_t nnz_niv;        /* finite entries of niv, own chain included (nnz(N), §2.4)   */
  int64_t nnz_niv_up;     /* the same for the up-niv map of the dual order             */
  int64_t max_chain;      /* longest chain of the decomposition                         */
  int64_t levels_down;    /* levels scheduling the Möbius solve                         */
  int64_t levels_up;      /* levels scheduling the adjoint Möbius solve                 */
  int64_t mirsky_levels;  /* length of the longest chain of the poset (Mirsky, §4)      */
  int64_t udep_levels;    /* levels of the U-solve dependency DAG                       */
  int64_t device_bytes;   /* device memory held by the handle, workspace excluded       */
  int64_t walk_runs;      /* runs of the walking gather over the niv map (0: not used)  */
  int64_t walk_events;    /* niv change events inside those runs                        */
  int64_t walk_snapshots; /* running-sum snapshots those runs store                     */
  int64_t walk_T;         /* their run length and event cap (see px_autotune)            */
  int64_t walk_emax;
  int64_t walk_rows_distinct; /* distinct P rows those runs read (each counted once)     */
  int64_t walk_row_loads;     /* P-row loads they issue (first rows' gathers, both rows
                                 of every event)                                        */
  int32_t chains_planted; /* 1 if the caller supplied the chains                        */
  int32_t device;
  double t_validate, t_chains, t_niv, t_levels, t_upload;  /* preprocessing seconds      */
  int32_t niv_sparse;     /* 1 if the niv maps are kept sparse (PX_BUILD_SPARSE_NIV)    */
  int32_t niv_device_rounds; /* rounds of the device computation of the dense niv maps
                                (0: the host recursion computed them)                    */
  int64_t run_chunks;     /* chunks of the int64 level solve by runs (niv map; 0: that
                             solve is not used and int64 solves row by row)              */
  int64_t run_events;     /* change events those chunks read (niv map)                   */
  int64_t path_cover;     /* chains of the matching's path cover when the library chose
                             the chains (k is smaller with PX_BUILD_MIN_CHAINS); 0 for
                             planted or loaded chains                                    */
  int64_t layout;         /* PX_LAYOUT_NODES or PX_LAYOUT_ROWS (px_poset_set_layout)     */
  int64_t scan_flat;      /* bit i set: the chain scan for blocks of 2^i columns
                             (i < 6) runs over fixed blocks of rows, a chain start
                             resetting the sum, instead of tiles cut per chain (chosen
                             when most chains are short)                               */
} px_info;

typedef struct {
  int32_t iterations;     /* refinement steps taken                                        */
  int32_t nonfinite;      /* 1 if a correction, the iterate or the residual held NaN or Inf */
  double residual;        /* max over columns of ||g - zeta(f)||_inf / ||g||_inf, float64,
                             for the returned f (normwise backward error)                  */
  double correction;      /* max over columns of ||delta||_inf / ||f||_inf of the last step */
} px_refine_report;

/*
 * Build a poset handle (one-time preprocessing, §4: chain decomposition,
 * niv map by the recursion of Theorem 5, levels; then upload).  For a device
 * handle with dense niv rows of at least 2^24 entries (n * k) the two niv maps
 * are computed on the device as the fixed point of that recursion (the same
 * maps; POSETX_PREP=host or =device forces the host recursion or the device
 * for any size); the rest of the preprocessing runs on the host.
 *   n          elements, 0 <= n < 2^31
 *   indptr     host, n+1 entries, indptr[0] = 0, non-decreasing
 *   indices    host, indptr[n] entries in [0, n)
 *   chain_of   host, n entries or NULL.  With chain_pos: a planted chain
 *   chain_pos  decomposition, chain_of[x] in [0, k), positions 0..len-1 of
 *              each chain used exactly once, position 0 the minimal element.
 *              It is validated (PX_ECHAIN if a chain is not totally ordered).
 *              NULL: chains come from a maximum matching on the edges
 *              (Alg. 1, Hopcroft-Karp), a minimum path cover of the DAG.
 *   flags      PX_BUILD_* bits
 *   device     HIP device ordinal (ignored with PX_BUILD_HOST_ONLY)
 *   out        receives the handle; free it with px_poset_free
 * Host arrays are copied.  Synchronous.  Builds share no state: calls on
 * several host threads may run at once, each returning its own handle, with
 * the same result as one call after another.
 */
px_status px_poset_build(int64_t n, const int64_t* indptr, const int32_t* indices,
                         const int32_t* chain_of, const int32_t* chain_pos, uint32_t flags,
                         int device, px_poset** out);
px_status px_poset_free(px_poset* p);

/* Save the preprocessing of a handle (chains, niv maps, level schedules) to a
 * file, and build a handle from such a file without preprocessing again (the
 * preprocessing is the one-time cost that the transforms amortise, §5).  The
 * file is raw arrays in this machine's byte order.  px_poset_load checks every
 * array against n and k (PX_EINVAL for a file that is not a saved poset or is
 * inconsistent); flags: PX_BUILD_HOST_ONLY or 0 (the other build choices come
 * from the file); device as for px_poset_build.  Synchronous. */
px_status px_poset_save(const px_poset* p, const char* path);
px_status px_poset_load(const char* path, uint32_t flags, int device, px_poset** out);
px_status px_poset_info(const px_poset* p, px_info* out);

/* Host copies of the preprocessing products, in NODE order (for inspection and tests).
 *   chains: chain_of[n], chain_pos[n]
 *   niv:    out[n * k]; out[x*k + j] = node id of niv_j(x), or -1 (the paper's ∞);
 *           up != 0 gives the dual map: the lowest element of chain j above x.  For a
 *           handle with sparse rows this expands them to n * k entries (see
 *           px_poset_niv_csr for the compact form).
 *   levels: level[n] of every node in the Möbius schedule (up != 0: adjoint schedule). */
px_status px_poset_chains(const px_poset* p, int32_t* chain_of, int32_t* chain_pos);
/* The chain-major numbering the kernels work in: row_of_node[x] = first row of
 * x's chain + its position (chains in order, bottom first), n entries.  Function
 * matrices stay in node order at this interface; the numbering lets a caller
 * relate them to the chain-major prefix matrix V f (§3). */
px_status px_poset_rows(const px_poset* p, int64_t* row_of_node);
px_status px_poset_niv(const px_poset* p, int up, int32_t* out);

/* Function-matrix layout of every later transform on this handle.
 *   PX_LAYOUT_NODES (default): row x of f, g, w, v, out is node x.
 *   PX_LAYOUT_ROWS: row r is the element at chain-major row r (px_poset_rows), the
 *     order in which the chain scans and level solves run, so that every
 *     kernel streams the matrices instead of visiting them in node order.  A
 *     caller that keeps its functions permuted this way gets the same values, bit
 *     for bit, permuted the same way (§3: Z = U V acts on that numbering).
 * The first switch to rows allocates one int32 table of n entries (not under
 * graph capture).  Not to be called while a transform on the handle is in
 * flight.  Batches built from the handle keep node order. */
#define PX_LAYOUT_NODES 0u
#define PX_LAYOUT_ROWS 1u
px_status px_poset_set_layout(px_poset* p, uint32_t layout);
/* The same map by rows of its finite entries (N of §2.4 in CSR form, node order):
 * the entries of node x are nodes[ptr[x] .. ptr[x+1]), the node ids niv_j(x) in
 * ascending chain j.  ptr: n+1 entries; nodes: px_info.nnz_niv (up: nnz_niv_up)
 * entries.  Available for dense and sparse handles. */
px_status px_poset_niv_csr(const px_poset* p, int up, int64_t* ptr, int32_t* nodes);
px_status px_poset_levels(const px_poset* p, int up, int32_t* level);

/* Grow the workspace for dtype and B right-hand sides now, so that later calls with
 * at most B columns allocate nothing.  Synchronous. */
px_status px_reserve(px_poset* p, int dtype, int64_t B);

/*
 * g = Z f  (fast zeta transform, §3 Eq. zeta-fast / Alg. 3): chain-wise prefix sums
 * followed by the niv gather-reduce.  f, g: device [n, B] with leading dims ldf, ldg.
 * f == g (same pointer and ld) is allowed.  B >= 1.
 */
px_status px_zeta(px_poset* p, int dtype, const void* f, int64_t ldf, void* g, int64_t ldg,
                  int64_t B, void* stream);

/* out = Z^T w: chain-wise suffix sums and the up-niv gather (zeta on the dual order).
 * Requires a handle built without PX_BUILD_NO_ADJOINT. */
px_status px_zeta_adjoint(px_poset* p, int dtype, const void* w, int64_t ldw, void* out,
                          int64_t ldo, int64_t B, void* stream);

/*
 * g = Z f exactly as px_zeta computes it (the same kernels, bit-identical results),
 * for callers that cannot allocate device memory: code recorded under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  It calls no
 * hipMalloc, hipFree or other allocating routine.  Its scratch (the prefixes,
 * tile states and walk snapshots that px_zeta keeps in the handle's workspace)
 * is a static device array of 64 MiB that every GPU running the library holds
 * until the process ends; its device address is looked up once per device, on
 * the first call there.
 *   Returns PX_EINVAL, before launching anything, when the call needs more than
 *   64 MiB of scratch (the message says how much).  The scratch of the compact
 *   walk (one poset, k <= 64, B >= 5) is small: at n = 2^20, k = 64, B = 64 float32
 *   it needs about 97 MiB, so that size is rejected while n = 2^19 fits; the scan
 *   over P (other shapes) needs (n + 1) * B * elem bytes for P and fits while
 *   n * B * elem stays below about 60 MiB.
 *   Every call on one GPU shares that GPU's array and leaves its contents behind;
 *   nothing in it needs to start at zero (the kernels write every word they read).
 *   Calls that overlap in time on one GPU (on different streams or from different
 *   threads) race on it: serialise them.
 * Other arguments, errors and the asynchronous behaviour are those of px_zeta.
 */
px_status px_zeta_noalloc(px_poset* p, int dtype, const void* f, int64_t ldf, void* g,
                          int64_t ldg, int64_t B, void* stream);

/*
 * f = M g = Z^{-1} g  (fast Möbius transform, §3 and Alg. 4): level-scheduled solve
 * of U y' = g, then f = V^{-1} y' (first difference along every chain).
 *   PX_I64: exact; max_refine and tol are ignored; never synchronises.
 *   PX_F64: float64 solve; no refinement.
 *   PX_F32: float32 solve, then up to max_refine steps of iterative refinement:
 *           r = g - zeta(f) with zeta applied in float64, delta = M r (float32
 *           solve), f += delta.
 *   tol (floating-point dtypes):
 *     > 0   PX_F32 stops early once every column has ||delta||_inf <= tol *
 *           ||f||_inf (a forward-error test: the residual itself is floored by
 *           the float32 rounding of f summed over down-sets); this check
 *           synchronises the stream after each step.
 *     = 0   runs exactly max_refine steps; then synchronises the stream once and
 *           checks the result for NaN / Inf.
 *     < 0   runs exactly max_refine steps asynchronously: no value checks and no
 *           host synchronisation (the form to record under HIP graph capture).
 *   rep        NULL or receives the refinement report (PX_F32; computes the final
 *              residual; synchronises).
 * g and f must not overlap.  Returns PX_ENONFINITE if tol >= 0 (or rep != NULL) and
 * the result, a correction or the residual holds a NaN or Inf (f is still written),
 * and PX_ENOTCONV if tol > 0 and max_refine > 0 and the correction test was not met
 * within max_refine steps (f is still written).
 */
px_status px_mobius(px_poset* p, int dtype, const void* g, int64_t ldg, void* f, int64_t ldf,
                    int64_t B, int max_refine, double tol, void* stream, px_refine_report* rep);

/* out = M^T v = (Z^T)^{-1} v: the Möbius transform of the dual order, same contract as
 * px_mobius.  Requires a handle built without PX_BUILD_NO_ADJOINT. */
px_status px_mobius_adjoint(px_poset* p, int dtype, const void* v, int64_t ldv, void* out,
                            int64_t ldo, int64_t B, int max_refine, double tol, void* stream,
                            px_refine_report* rep);

/*
 * Batches of independent posets of uneven size (all on one device).  A batch
 * function matrix stacks the posets' [n_i, B] matrices in order: rows
 * [o_i, o_i + n_i) belong to poset i, o_i = n_0 + ... + n_{i-1}.  Each batched
 * call runs every poset in one launch per phase.  The batch keeps its own
 * device copy of the posets' maps; the poset handles may be freed afterwards.
 */
px_status px_batch_build(int count, px_poset* const* posets, px_batch** out);
px_status px_batch_free(px_batch* b);
px_status px_batch_reserve(px_batch* b, int dtype, int64_t B);
px_status px_batch_rows(const px_batch* b, int64_t* total_rows);
px_status px_zeta_batched(px_batch* b, int dtype, const void* f, int64_t ldf, void* g,
                          int64_t ldg, int64_t B, void* stream);
px_status px_zeta_adjoint_batched(px_batch* b, int dtype, const void* w, int64_t ldw, void* out,
                                  int64_t ldo, int64_t B, void* stream);
/* Layout of the batch's function matrices, as px_poset_set_layout for one poset:
 * PX_LAYOUT_NODES (default) stacks each poset's matrix in node order;
 * PX_LAYOUT_ROWS stacks each poset's chain-major rows (px_poset_rows), so that
 * the scans read and the gathers write the matrices in order.  Results are the
 * same values, bit for bit, permuted the same way.  The first switch to rows
 * allocates one int32 table of px_batch_rows entries; not to be called while a
 * transform on the batch is in flight or under graph capture.
 * px_batch_row_order: row_of_node[x] = batch row of batch node x (o_i + node),
 * px_batch_rows entries (the permutation a caller applies to switch layouts). */
px_status px_batch_set_layout(px_batch* b, uint32_t layout);
px_status px_batch_row_order(const px_batch* b, int64_t* row_of_node);

/* Report of an autotuning call. */
typedef struct {
  int32_t walk_T;         /* run length of the walking gather (rows)                     */
  int32_t walk_emax;      /* change events per run at most                               */
  int32_t rhs_tile;       /* column tile of the lane-split gather (0 = smallest >= B)   */
  double ms_best;         /* one zeta call with the chosen shape, milliseconds           */
  double ms_default;      /* the same with the default shape (-1 if not timed)           */
  int32_t from_cache;     /* 1 if the shape came from the cache without timing           */
} px_tune_report;

/*
 * Autotuner of the gather tile shapes: for a poset, the chain tile (walk run
 * length 64/128/256 rows x event cap 48/96/192) and, for B < 32, the RHS tile
 * (columns per lane group); for a batch, the RHS tile.  Every candidate is
 * timed on the device with HIP events (median of 5 zeta calls on the null
 * stream) and the fastest is kept in the handle.  Results are cached per
 * shape for the process and, when the environment variable POSETX_TUNE_CACHE
 * names a file, appended there and reused by later processes.  Synchronous;
 * allocates two [n, B] scratch matrices while it runs.  rep may be NULL.
 */
px_status px_autotune(px_poset* p, int dtype, int64_t B, px_tune_report* rep);
px_status px_batch_autotune(px_batch* b, int dtype, int64_t B, px_tune_report* rep);

/* Optional per-kernel timing.  px_profile(1) resets the totals and starts recording a
 * pair of HIP events on the launch stream around every kernel launch of every handle;
 * px_profile(0) stops.  px_profile_read synchronises on the recorded events and returns,
 * for each of the first nphases phases, the summed milliseconds and the launch count.
 * Phase names: px_profile_phase_name(i) (scan_reduce, scan_carry, scan_apply, gather,
 * usolve_level, chain_diff, absmax, walk_events, walk_combine, scan_onepass, apply_combine).
 * Not for use under HIP graph capture. */
px_status px_profile(int on);
px_status px_profile_read(double* ms, int64_t* count, int nphases);
const char* px_profile_phase_name(int i);

/* Thread-local message of the last failure on this thread ("" if none). */
const char* px_last_error(void);
const char* px_version(void);

#ifdef __cplusplus
}
#endif

#endif /* POSETX_H */
