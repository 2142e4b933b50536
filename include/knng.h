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
 *   4. neighbourhood propagation (Section 3.2): first-order rounds
 *      (Theorem 1) or best-first passes with a budget of visited points,
 *      with pairwise updating (Section 3.4).
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers owned by the caller unless a
 *     parameter says "host".  The library never allocates or frees device
 *     memory: scratch space comes from the caller's workspace `ws` of
 *     `ws_bytes` bytes, which must be at least knng_workspace_bytes(p, op)
 *     and 256-byte aligned.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued asynchronously and the entry points do not wait for the
 *     stream (the data-independent tree plan is copied from pinned host
 *     memory the library keeps until the copy has completed), except those
 *     documented as returning host results or timings.
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
  KNNG_EUNSUPPORTED = -4 /* valid but not supported by the library            */
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
  KNNG_METRIC_L2 = 0,     /* squared Euclidean distance                        */
  KNNG_METRIC_COSINE = 1  /* cosine: the method runs on rows scaled to unit
                             length (knng_normalize); distances are the
                             squared distances of the unit rows,
                             2 (1 - cos theta), which rank like 1 - cos theta */
} knng_metric;

typedef enum {
  KNNG_OP_DIVIDE = 0,
  KNNG_OP_LEAF = 1,
  KNNG_OP_MERGE = 2,
  KNNG_OP_PROPAGATE = 3,
  KNNG_OP_BUILD = 4,
  KNNG_OP_COLEAF = 5
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
  int32_t metric;         /* knng_metric, honoured by knng_build* and the graph
                             entry points; the stage entry points measure
                             distances between the rows they are given       */
  int32_t visit_max;      /* propagation form: 0 = first-order rounds
                             (Theorem 1); > 0 = best-first passes (Section
                             3.2) evaluating at most visit_max new points per
                             point and pass (<= 1024)                        */
  int32_t rate_permille;  /* 0: knng_build runs all T divisions; > 0: it stops
                             them at the first division m whose effective rate
                             r_m (Section 3.2) is below rate_permille / 1000
                             (Section 4 starts propagation at r_m < 0.05,
                             i.e. 50); T is then the largest number          */
  int32_t reserved;       /* must be 0                                         */
} knng_params;

/* Diagnostics a call leaves in its workspace (read with knng_read_diag). */
typedef struct {
  int64_t leaf_rows_fallback;   /* leaf rows redone exactly (uncertified)     */
  int64_t leaf_rows;            /* leaf rows processed                        */
  int64_t prop_candidates;      /* sum over points of |C_p| in the last round */
  int64_t prop_proposals;       /* reverse proposals kept in the last round   */
  int64_t divisions_used;       /* knng_build: divisions run (T unless the
                                   effective-rate rule stopped them earlier) */
  int64_t rate_new[64];         /* knng_build with rate_permille > 0: per
                                   division m < 64, sum over p of the ids of
                                   p's list m in none of its earlier lists   */
  int64_t rate_total[64];       /* ... and of |union of p's lists 0..m|; r_m =
                                   rate_new[m] / rate_total[m]               */
} knng_diag;

/* Human-readable name of a status code (static string). */
const char* knng_status_str(int status);

/* Description of the calling thread's last failure (static thread-local). */
const char* knng_last_error(void);

/* Host-side fault injection, for callers that test their own handling of a
 * failed launch (re-issuing a stage: every entry point is a pure function
 * of its inputs, parameters and seed).  mode 1 arms a one-shot fault: the
 * next kernel launch of any entry point, in any thread, returns KNNG_EHIP
 * without enqueueing that launch or anything after it (work the same call
 * enqueued before it stays enqueued; outputs are unspecified); mode 0
 * disarms.  Setting KNNG_FAULT=launch in the environment arms it once when
 * the library is loaded.  Nothing reaches the GPU.  Returns the previous
 * state (0 or 1), or KNNG_EINVAL for another mode.  Host only. */
int knng_inject_fault(int32_t mode);

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

/* Rows scaled to unit length, for the cosine distance of Definition 1:
 * Xn[i] = X[i] / |X[i]| with |X[i]|^2 summed over the features left to
 * right in float32 (each product and sum rounded), a correctly rounded
 * square root and correctly rounded quotients; a zero row stays zero.
 * X, Xn: n x d (d a multiple of 4; Xn may equal X).  Asynchronous.          */
int knng_normalize(int64_t n, int32_t d, const float* X, float* Xn, void* stream);

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

/* knng_leaf_knn for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): it
 * takes no workspace and allocates nothing.  Its scratch (diagnostics,
 * fallback rows, member norms) is one array inside the library of
 * 12 bytes per point for KNNG_NOALLOC_MAX_N points (about 25 MB) per GPU,
 * held until the process ends, so n is at most KNNG_NOALLOC_MAX_N (larger
 * n: KNNG_EINVAL, nothing enqueued).
 * Every call on one GPU shares that array: calls that overlap on a GPU
 * (other threads, other streams) race and must be serialised by the caller.
 * Arguments and results as knng_leaf_knn.                                   */
#define KNNG_NOALLOC_MAX_N ((int64_t)1 << 21)
int knng_leaf_knn_noalloc(const knng_params* p, const float* X, const uint32_t* perm, const int64_t* leaf_off,
                          int64_t n_leaves, uint32_t* ids, float* dist, void* stream);

/* Combination of base graphs (Section 3.1): per point, unite n_lists lists,
 * drop duplicate ids, keep the first k by (distance, id).  Every input list
 * is sorted by (distance, id) with its padding at the tail, as the other
 * entry points write them, and one id carries one distance.
 *   ids_in, dist_in (n_lists x n x k); ids_out, dist_out (n x k), which must
 *   not overlap the inputs.                                                */
int knng_merge(const knng_params* p, int n_lists, const uint32_t* ids_in, const float* dist_in,
               uint32_t* ids_out, float* dist_out, void* stream);

/* `rounds` rounds of neighbourhood propagation (Section 3.2).  Each round
 * reads the graph G frozen.  With p->visit_max == 0 it is the first-order
 * form of Theorem 1: every p gets the first k by (distance, id) of N(p) and
 * the neighbours of its neighbours.  With p->visit_max > 0 it is a
 * best-first pass: a queue ordered by (distance to p, id) starts with N(p);
 * the nearest queued point is popped and its neighbours not seen yet are
 * evaluated (distance to p) and queued, in its list order, until visit_max
 * points have been evaluated or the queue is empty; p keeps the first k of
 * N(p) and the evaluated points.  Either way, when p->pairwise (Section
 * 3.4), the points that evaluated p are candidates of p too.
 * First-order rounds take k <= 31 in one fast kernel and 31 < k <= 64 in the
 * queue kernel; best-first passes take any k <= 64.
 *   ids, dist (n x k, in/out).                                             */
int knng_propagate(const knng_params* p, const float* X, uint32_t* ids, float* dist, int rounds, void* ws,
                   size_t ws_bytes, void* stream);

/* The whole method: p->T divisions (advanced level by level together),
 * leaf k-NN of every leaf of every division in one persistent launch
 * (largest leaves first), merge, p->rounds propagation rounds.  One pass
 * over X first records whether its values are integers (and whether all lie
 * in 0..255, when the divisions and propagation read a one-byte copy of X
 * kept in the workspace); the output is the same either way.
 * ids, dist (n x k) receive the graph.                                     */
int knng_build(const knng_params* p, const float* X, uint32_t* ids, float* dist, void* ws, size_t ws_bytes,
               void* stream);

/* knng_build with a HIP event at every stage boundary; waits for the stream
 * at the end.  ms_out (host, at least 3 + rounds entries) receives the GPU
 * time of: all T divisions (entry 0, the batched divide launches, and the
 * row scaling of the cosine metric), the leaf k-NN of every leaf of every
 * division (1, one persistent launch plus its exact-row pass), the merge
 * (2), then each propagation round (3 + r).  With rate_permille > 0 the
 * divisions run one at a time: entry 0 then holds the divide, leaf k-NN and
 * rate test of every division and entry 1 is zero.                         */
int knng_build_timed(const knng_params* p, const float* X, uint32_t* ids, float* dist, void* ws, size_t ws_bytes,
                     void* stream, float* ms_out, int ms_cap);

/* knng_build with the T divisions computed on other rows: point i is placed
 * in the trees by row i of S (n x ds float32, ds a multiple of 4 with
 * 4 <= ds <= p->d; p->split applies in R^ds), while the leaf k-NN, the merge
 * and the propagation measure distances between rows of X.  With S the
 * embedding of a trained partitioner (knng_mlp_forward) this is the learned
 * division: random-projection splits of the embedded points.  S = X and
 * ds = p->d give knng_build exactly.  Workspace: knng_workspace_bytes(p,
 * KNNG_OP_BUILD).  ms_out may be NULL; otherwise it receives stage times as
 * in knng_build_timed and the call waits for the stream.                   */
int knng_build_split(const knng_params* p, const float* X, const float* S, int32_t ds, uint32_t* ids, float* dist,
                     void* ws, size_t ws_bytes, void* stream, float* ms_out, int ms_cap);

/* Share of n_pairs point pairs (device uint32 [2 n_pairs], pair j =
 * (pairs[2j], pairs[2j+1])) whose two points land in the same leaf of
 * division t computed on S (n x ds, as in knng_build_split).  For exact
 * neighbour pairs this is the single-tree co-leaf probability that Lemma 1
 * multiplies over trees.  *rate is written on the host; waits for the
 * stream.  Workspace: knng_workspace_bytes(p, KNNG_OP_COLEAF).             */
int knng_coleaf_rate(const knng_params* p, int t, const float* S, int32_t ds, const uint32_t* pairs, int64_t n_pairs,
                     double* rate, void* ws, size_t ws_bytes, void* stream);

/* The learned division's fallback rule: computes the co-leaf rate of the
 * held-out pairs (knng_coleaf_rate, division 0) for plain random division
 * of X (random projection in R^d) and for the learned division (p->split
 * applied to the embedding Z in R^KNNG_MLP_EMB), and sets *use_learned to
 * 1 only if the learned rate is strictly higher.  Rates are written to the
 * host; waits for the stream.  Workspace: knng_workspace_bytes(p,
 * KNNG_OP_COLEAF).                                                          */
int knng_learned_choice(const knng_params* p, const float* X, const float* Z, const uint32_t* pairs, int64_t n_pairs,
                        int32_t* use_learned, double* rate_plain, double* rate_learned, void* ws, size_t ws_bytes,
                        void* stream);

/* ---------------------------------------------------------------------------
 * Learned partitioner (an added form of the method; not in the paper).
 * A two-layer network z = W2 relu(W1 (scale x) + b1) + b2 maps a point of
 * R^d to R^KNNG_MLP_EMB through KNNG_MLP_HIDDEN hidden units.  Parameters
 * are one float32 device array of knng_mlp_param_count(d) entries laid out
 * as W1 [H][d] row-major | b1 [H] | W2 [E][H] row-major | b2 [E].  The
 * matrix products run on MFMA: KNNG_BF16 rounds both operands to bfloat16
 * (round to nearest even) and accumulates in float32; KNNG_FP32 keeps
 * float32 throughout.  d must be a multiple of 16 with 16 <= d <= 256.
 *
 * Training minimises the contrastive loss of Hadsell, Chopra and LeCun
 * (CVPR 2006) over P positive pairs (a, b) and N negative pairs (a, u):
 *   L = mean_P |z_a - z_b|^2 + lam * mean_N max(0, margin - |z_a - z_u|^2)
 * with Adam (Kingma and Ba, ICLR 2015).  Positives are edges of a k-NN
 * graph the method produced, negatives uniform random pairs.
 * ------------------------------------------------------------------------- */
#define KNNG_MLP_HIDDEN 256
#define KNNG_MLP_EMB 16

/* Number of float32 parameters for input dimension d (0 if d is invalid). */
int64_t knng_mlp_param_count(int32_t d);

/* Initial parameters: W1 ~ U(-sqrt(6/d), sqrt(6/d)), W2 ~ U(-sqrt(6/(H+E)),
 * sqrt(6/(H+E))) from 24-bit uniforms of the library's counter generator
 * (tag 4, index = parameter position), biases zero.                        */
int knng_mlp_init(int32_t d, uint64_t seed, float* params, void* stream);

/* Z (n x KNNG_MLP_EMB float32, 16-byte aligned) = network(X) for n rows. */
int knng_mlp_forward(int32_t d, int32_t precision, float scale, const float* params, const float* X, int64_t n,
                     float* Z, void* stream);

/* Workspace for knng_mlp_grad / knng_mlp_train with n_pos + n_neg pairs. */
size_t knng_mlp_workspace_bytes(int32_t d, int32_t n_pos, int32_t n_neg);

/* Gradient of L with respect to every parameter (grads: param_count
 * float32, device) and L itself (loss: one float32, device; may be NULL)
 * for the pairs in rows (device uint32 [2 (n_pos + n_neg)]: pair j =
 * (rows[2j], rows[2j+1]), positives first).  Per-chunk partial sums are
 * added in a fixed order, so the result is deterministic.                 */
int knng_mlp_grad(int32_t d, int32_t precision, float scale, const float* params, const float* X,
                  const uint32_t* rows, int32_t n_pos, int32_t n_neg, float lam, float margin, float* grads,
                  float* loss, void* ws, size_t ws_bytes, void* stream);

/* One Adam step (t = step >= 1) on n parameters with moments m, v.        */
int knng_mlp_adam(int64_t n, float* params, const float* grads, float* m, float* v, int32_t step, float lr,
                  float beta1, float beta2, float eps, void* stream);

/* Training pairs of step `step` from a k-NN graph ids (n x k): pair j <
 * n_pos is (i, ids[i][s]) with i, s drawn uniformly; the others (a, b)
 * uniform over [0, n).  Draw j uses the counter generator with tag 5
 * (positives) or 6 (negatives), division field step mod 4096, node field j,
 * index field step / 4096; i = hi32(r) * n >> 32, s = lo32(r) * k >> 32,
 * b = lo32(r) * n >> 32.  A padded slot (KNNG_NONE) pairs i with itself.  */
int knng_mlp_sample_pairs(int64_t n, int32_t k, const uint32_t* ids, uint64_t seed, uint32_t step, int32_t n_pos,
                          int32_t n_neg, uint32_t* rows, void* stream);

/* steps iterations of (sample pairs, gradient, Adam) starting at Adam step
 * step0 + 1, all enqueued on the stream.  losses (device, steps float32)
 * receives each step's loss and may be NULL.  Workspace:
 * knng_mlp_workspace_bytes(d, n_pos, n_neg).                              */
int knng_mlp_train(int32_t d, int32_t precision, float scale, float* params, float* m, float* v, const float* X,
                   int64_t n, int32_t k, const uint32_t* graph_ids, uint64_t seed, int32_t step0, int32_t steps,
                   int32_t n_pos, int32_t n_neg, float lam, float margin, float lr, float* losses, void* ws,
                   size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Leaf tile configuration (the batched leaf launch of added form (2)).
 * The leaf kernel runs one workgroup per leaf with `waves` waves (4 or 8)
 * and stages `kc` features of 32 candidates per tile (32, 64 or 128).  A
 * configuration applies to one shape class: input dimension d, precision,
 * list length class kp (k + rerank_m rounded up to 16, 32 or 64) and leaf
 * bucket (the largest leaf of the launch rounded up to a power of two in
 * [64, 2048]).  Classes without one use the defaults (8 waves, 4 for
 * kp = 64; kc = 32, 64 or 128 as d <= 32, <= 64, larger).  The table is
 * process-wide and shared by all threads.
 * ------------------------------------------------------------------------- */

/* Sets (waves, kc) for a shape class; waves = kc = 0 restores the default. */
int knng_leaf_set_config(int32_t d, int32_t precision, int32_t kp, int32_t leaf_bucket, int32_t waves, int32_t kc);

/* Autotuner: runs the T divisions of p on X once, then times the batched
 * leaf launch over those leaves for every configuration that fits (waves
 * in {8, 4}; kc from {64, 128} for d > 64, {32, 64} for 32 < d <= 64, 32
 * otherwise; one warm-up and the mean of 3 timed launches each), stores
 * the fastest for p's shape class and returns it with its time and the
 * leaf bucket.  Needs a non-null stream; waits for it.  Workspace:
 * knng_workspace_bytes(p, KNNG_OP_BUILD).                                  */
int knng_leaf_tune(const knng_params* p, const float* X, void* ws, size_t ws_bytes, void* stream, int32_t* waves_out,
                   int32_t* kc_out, float* ms_out, int32_t* leaf_bucket_out);

/* HIP-graph form of knng_build_split (S = X, ds = p->d for knng_build):
 * runs the build once eagerly (which uploads the tree plans into ws and
 * performs every lazy kernel set-up), then captures the same launch
 * sequence (kernels and device-to-device copies only) on `stream` (non-null)
 * and instantiates it.  *graph receives an opaque handle.  X, S, ids, dist
 * and ws are baked into the graph: they must stay allocated, and ws must not
 * be used by another call, until knng_graph_destroy.                       */
int knng_graph_create(const knng_params* p, const float* X, const float* S, int32_t ds, uint32_t* ids, float* dist,
                      void* ws, size_t ws_bytes, void* stream, void** graph);

/* Enqueues one replay of the captured build on `stream`.                  */
int knng_graph_launch(void* graph, void* stream);

/* Frees a graph (NULL is accepted).                                        */
int knng_graph_destroy(void* graph);

/* Copies the diagnostics of the last call that used workspace `ws` to the
 * host; waits for `stream`.                                                */
int knng_read_diag(const knng_params* p, const void* ws, int op, knng_diag* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* KNNG_H */
