/*
 * knng.h -- C ABI of the MI355X (gfx950) k-NN graph construction library.
 *
 * The library builds an approximate k-nearest-neighbour graph over n points
 * x_1..x_n in R^d (Definition 1 of Wang et al., "Scalable k-NN graph
 * construction", arXiv 1307.7852: a directed graph with an edge <x_i, x_j>
 * when the distance from x_i to x_j is among the k smallest from x_i).  The
 * distance is the squared Euclidean distance, which ranks exactly like the
 * Euclidean metric.
 *
 * The method (Section 3) is
 *   1. T random hierarchical divisions of the point set (Section 3.1,
 *      appendix; principal-direction variant in Section 3.4),
 *   2. an exact brute-force k-NN subgraph inside every leaf subset
 *      (Section 3.1),
 *   3. the combination of the T base graphs: unite each point's adjacency
 *      lists and keep the k nearest (Section 3.1),
 *   4. neighbourhood propagation rounds (Section 3.2, first-order form of
 *      Theorem 1) with pairwise updating (Section 3.4).
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers owned by the caller unless a
 *     parameter says "host".  The library never allocates or frees device
 *     memory: scratch space comes from the caller's workspace `ws` of
 *     `ws_bytes` bytes, which must be at least knng_workspace_bytes(p, op)
 *     and 256-byte aligned.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued asynchronously; an entry point may wait for the stream to
 *     reach its own first copy (host-to-device upload of the data-independent
 *     tree plan) but never for work enqueued after it.
 *   - Arguments are validated on the host before anything is enqueued.  On a
 *     negative return nothing was enqueued, except KNNG_EHIP, after which the
 *     outputs are unspecified.  knng_last_error() describes the last failure
 *     of the calling thread.
 *   - X is row-major n x d float32, rows contiguous, 16-byte aligned, finite;
 *     d must be a multiple of 4 (pad with zero columns otherwise: that keeps
 *     every distance and projection unchanged).
 *   - Neighbour lists are n x k: row i belongs to point id i, entries sorted
 *     ascending by (distance, id); a row with fewer than k candidates is
 *     padded with (KNNG_NONE, +inf).  Ids are uint32, distances float32.
 *   - Requirements: 1 <= n < 2^32 - 1, 4 <= d <= 4096, 1 <= k <= 64,
 *     1 <= T <= 4096, leaf_max >= 2, 0 < q_lo_pm <= q_hi_pm < 1000,
 *     every leaf at most 2048 points, tree depth at most 31.
 *   - Deterministic: identical inputs and parameters give bitwise-identical
 *     outputs.
 */
#ifndef KNNG_H
#define KNNG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KNNG_NONE 0xFFFFFFFFu
#define KNNG_MAX_LEAF 2048

typedef enum {
  KNNG_OK = 0,
  KNNG_EINVAL = -1,      /* invalid argument or parameter                      */
  KNNG_ENOMEM = -2,      /* workspace smaller than knng_workspace_bytes()      */
  KNNG_EHIP = -3,        /* a HIP runtime call failed                          */
  KNNG_EUNSUPPORTED = -4 /* valid but not supported by this build              */
} knng_status;

typedef enum {
  KNNG_SPLIT_RP = 0,  /* random projection, median split (appendix)          */
  KNNG_SPLIT_PCA = 1  /* principal direction of a node sample (Section 3.4)  */
} knng_split;

typedef enum {
  KNNG_FP32 = 0,  /* leaf Gram on FP32 MFMA                                   */
  KNNG_BF16 = 1   /* leaf Gram on BF16 MFMA with FP32 accumulation            */
} knng_precision;

typedef enum {
  KNNG_OP_DIVIDE = 0,
  KNNG_OP_LEAF = 1,
  KNNG_OP_MERGE = 2,
  KNNG_OP_PROPAGATE = 3,
  KNNG_OP_BUILD = 4
} knng_op;

typedef struct {
  int64_t n;              /* number of points                                  */
  int32_t d;              /* dimension (multiple of 4)                         */
  int32_t k;              /* neighbours per point                              */
  int32_t T;              /* number of random divisions (the paper's M or L)   */
  int32_t leaf_max;       /* a node with more points is split (paper's g - 1)  */
  int32_t leaf_cap_cycle; /* 0: every division uses leaf_max; 3: division t
                             uses {leaf_max/2, leaf_max, 2 leaf_max}[t mod 3]  */
  int32_t q_lo_pm;        /* split count range in permille of the node size;   */
  int32_t q_hi_pm;        /*   500/500 is the median split                      */
  int32_t rounds;         /* propagation rounds run by knng_build              */
  int32_t pairwise;       /* 1: pairwise updating (Section 3.4)                */
  int32_t split;          /* knng_split                                        */
  int32_t precision;      /* knng_precision of the leaf Gram                   */
  int32_t rerank_m;       /* extra leaf candidates re-ranked exactly (>= 0)    */
  int32_t pca_iters;      /* power iterations for KNNG_SPLIT_PCA (e.g. 16)     */
  uint64_t seed;          /* seed of every random draw                         */
} knng_params;

/* Diagnostics a call leaves in its workspace (read with knng_read_diag). */
typedef struct {
  int64_t leaf_rows_fallback;   /* leaf rows redone exactly (uncertified)     */
  int64_t leaf_rows;            /* leaf rows processed                        */
  int64_t prop_candidates;      /* sum over points of |C_p| in the last round */
  int64_t prop_proposals;       /* reverse proposals kept in the last round   */
} knng_diag;

/* Human-readable name of a status code (static string). */
const char* knng_status_str(int status);

/* Description of the calling thread's last failure (static thread-local). */
const char* knng_last_error(void);

/* Bytes of workspace entry point `op` needs for parameters `p`
 * (0 on invalid parameters; knng_last_error() then says why).  Host only. */
size_t knng_workspace_bytes(const knng_params* p, int op);

/* Shape of division t's random partition tree, which depends only on
 * (n, leaf_max, leaf_cap_cycle, q range, seed) and never on the data
 * (Section 3.1 recursion; the appendix's median bipartition).  Host only.
 *   n_leaves, n_internal, depth (host, non-null): sizes of the tree.
 *   leaf_off_host (host, nullable): receives n_leaves + 1 offsets into the
 *     permutation; `cap` is its capacity in elements.                      */
int knng_tree_shape(const knng_params* p, int t, int64_t* leaf_off_host, int64_t cap, int64_t* n_leaves,
                    int64_t* n_internal, int32_t* depth);

/* One random division (Section 3.1; appendix for the random-projection
 * median split; Section 3.4 for the principal direction).  Every node with
 * more points than the cap is split: points are ordered by (key, id), with
 * key = a_v . x in float32 summed left to right without fused multiply-add,
 * and the first `left` go to the left child; each child keeps its parent's
 * relative order.
 *   X            (n x d)  points.
 *   dir_override (nullable, n_internal x d): directions to use instead of
 *                drawing them, one per internal node in level order, left to
 *                right within a level.
 *   dirs_out     (nullable, n_internal x d): receives the directions used.
 *   perm         (n) receives the point ids leaf by leaf.
 *   leaf_off     (n_leaves + 1, int64) receives the leaves' offsets.       */
int knng_divide(const knng_params* p, int t, const float* X, const float* dir_override, float* dirs_out,
                uint32_t* perm, int64_t* leaf_off, void* ws, size_t ws_bytes, void* stream);

/* Exact k-NN inside every leaf (Section 3.1's brute-force subgraph): for
 * each member i of a leaf, the first min(k, m-1) other members by
 * (distance, id).  The Gram matrix runs on MFMA (p->precision); the best
 * k + rerank_m candidates are re-scored with the exact float32 distance and
 * any row whose choice the Gram error could have changed is redone exactly.
 *   perm (n), leaf_off (n_leaves + 1): as written by knng_divide; every
 *   leaf must hold 1..KNNG_MAX_LEAF points.
 *   ids, dist (n x k): rows of points that are members of a leaf.          */
int knng_leaf_knn(const knng_params* p, const float* X, const uint32_t* perm, const int64_t* leaf_off,
                  int64_t n_leaves, uint32_t* ids, float* dist, void* ws, size_t ws_bytes, void* stream);

/* Combination of base graphs (Section 3.1): per point, unite n_lists lists,
 * drop duplicate ids, keep the first k by (distance, id).
 *   ids_in, dist_in (n_lists x n x k); ids_out, dist_out (n x k), which must
 *   not overlap the inputs.                                                */
int knng_merge(const knng_params* p, int n_lists, const uint32_t* ids_in, const float* dist_in,
               uint32_t* ids_out, float* dist_out, void* stream);

/* `rounds` rounds of neighbourhood propagation (Section 3.2) in the
 * first-order form of Theorem 1: each round reads the graph G frozen and
 * gives every p the first k by (distance, id) of N(p), the neighbours of its
 * neighbours and, when p->pairwise (Section 3.4), the points that evaluated
 * p as such a candidate.
 *   ids, dist (n x k, in/out).                                             */
int knng_propagate(const knng_params* p, const float* X, uint32_t* ids, float* dist, int rounds, void* ws,
                   size_t ws_bytes, void* stream);

/* The whole method: p->T divisions (advanced level by level together),
 * leaf k-NN of every leaf of every division in one persistent launch
 * (largest leaves first), merge, p->rounds propagation rounds.
 * ids, dist (n x k) receive the graph.                                     */
int knng_build(const knng_params* p, const float* X, uint32_t* ids, float* dist, void* ws, size_t ws_bytes,
               void* stream);

/* knng_build with a HIP event at every stage boundary; waits for the stream
 * at the end.  ms_out (host, at least 3 + rounds entries) receives the GPU
 * time of: all T divisions (entry 0, the batched divide launches), the leaf
 * k-NN of every leaf of every division (1, one persistent launch plus its
 * exact-row pass), the merge (2), then each propagation round (3 + r).     */
int knng_build_timed(const knng_params* p, const float* X, uint32_t* ids, float* dist, void* ws, size_t ws_bytes,
                     void* stream, float* ms_out, int ms_cap);

/* Copies the diagnostics of the last call that used workspace `ws` to the
 * host; waits for `stream`.                                                */
int knng_read_diag(const knng_params* p, const void* ws, int op, knng_diag* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* KNNG_H */
