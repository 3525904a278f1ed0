/*
 * drgraph.h -- C ABI of libdrgraph.so, the MI355X (gfx950) implementation of
 * DRGraph's layout hot path (Zhu et al., "DRGraph: An Efficient Graph Layout
 * Algorithm for Large-scale Graphs by Dimensionality Reduction").
 *
 * Problem (Sec. 3.1): an undirected, unweighted graph G = (V, E) is mapped to
 * positions Y in R^2 or R^3.  The library takes the graph as CSR in device
 * memory and writes FP32 coordinates [n][dim] into caller-owned device
 * memory.  3-D layouts (dim = 3 in the parameters) run the row-form sweep;
 * the column-blocked copy, the batched form and the quality evaluators are
 * 2-D only.
 *
 * General conventions
 *   - Every pointer named *_dev is device memory on the context's device;
 *     every pointer named *_host (or documented as host) is host memory.
 *   - Inputs are borrowed for the duration of the call and never retained;
 *     drg_sim and drg_hier copy what they need.  Opaque objects are owned by
 *     the library and released by their *_destroy call (NULL-safe).
 *   - Work is enqueued on the context's HIP stream and is asynchronous unless
 *     a function says it synchronises.  drg_build_similarity and drg_coarsen
 *     synchronise internally (they size allocations from device counts).
 *   - Errors are status codes; no C++ exception crosses this boundary.  On
 *     error the outputs are unspecified, owned state is unchanged and
 *     drg_last_error() describes the failure (thread-local string, valid
 *     until the next call on the same thread).
 *   - Input CSR contract (Sec. 3.1, undirected unweighted): row_ptr int32
 *     [n+1] with row_ptr[0] = 0, col int32 [row_ptr[n]]; symmetric, rows
 *     sorted ascending, no self-loops, no duplicates.  DRG_VALIDATE checks
 *     this on the device and returns DRG_E_GRAPH if it does not hold.
 *   - Randomness is a Philox4x64-10 counter generator (Salmon et al., SC'11)
 *     keyed by {seed, stream tag}; every random choice is a pure function of
 *     (seed, tag, counter), so results do not depend on launch shapes.
 */
#ifndef DRGRAPH_H
#define DRGRAPH_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif
#pragma GCC visibility push(default)

typedef int32_t drg_status;
#define DRG_OK 0
#define DRG_E_INVALID -1     /* bad argument (null pointer, out-of-range value) */
#define DRG_E_GRAPH -2       /* input CSR breaks the contract (DRG_VALIDATE) */
#define DRG_E_OOM -3         /* device allocation failed; partial allocations freed */
#define DRG_E_DEVICE -4      /* a HIP runtime call failed */
#define DRG_E_UNSUPPORTED -5 /* valid request outside the implemented range */

#define DRG_VALIDATE 1u      /* flag: validate the input CSR on the device */

#define DRG_MODE_SYNC 0      /* Jacobi: all steps from one snapshot, deterministic */
#define DRG_MODE_ASYNC 1     /* Hogwild: steps applied in place while others read */

/* Sweep forms of the FP32 layout step (drg_ctx_last_sweep) */
#define DRG_SWEEP_ROW 0           /* a group of lanes per row, gathered records */
#define DRG_SWEEP_WINDOW 1        /* same sums, records staged in LDS windows */
#define DRG_SWEEP_BLOCKED 2       /* column-blocked copy, LDS-staged blocks */
#define DRG_SWEEP_ROW_ASYNC 3     /* Hogwild, a group of lanes per row */
#define DRG_SWEEP_BLOCKED_ASYNC 4 /* column-blocked copy, rows moved per row stage */

typedef struct drg_ctx drg_ctx;
typedef struct drg_sim drg_sim;
typedef struct drg_hier drg_hier;
typedef struct drg_batch drg_batch;

/* Undirected graph in CSR form (device pointers, borrowed). */
typedef struct {
    int32_t n;
    int32_t nnz;             /* = row_ptr[n] = 2|E| */
    const int32_t* row_ptr;  /* device, [n+1] */
    const int32_t* col;      /* device, [nnz] */
} drg_csr;

/* Parameters of one optimisation iteration (Sec. 3.2.2, Eq. gradient). */
typedef struct {
    int32_t M;               /* negative samples per node, >= 0 */
    int32_t b;               /* proximity shape parameter, 1..3 (Sec. 4.2); with b_half
                                set, b + 1/2.  A half b runs the row-form sweep */
    float gamma;             /* weight of negative samples */
    float eta;               /* step size of this iteration */
    float clip;              /* per-pair, per-component force clip, > 0 */
    int32_t level;           /* hierarchy level being laid out (0 = finest) */
    int32_t mode;            /* DRG_MODE_SYNC or DRG_MODE_ASYNC */
    int32_t dim;             /* 2 (or 0): positions in R^2, y [n][2]; 3: R^3, y [n][3] */
    uint64_t seed;
    uint64_t iter;           /* global iteration index; keys the negatives */
    int32_t b_half;          /* 1: the shape is b + 1/2 (b = 1 or 2: 1.5, 2.5); 0: b */
    int32_t _pad;
} drg_step_params;

/* Parameters of the whole multilevel layout (Sec. 3.2, Sec. 4 defaults). */
typedef struct {
    int32_t k;               /* order of the neighbourhoods NNG(v, k), 1..4 */
    int32_t M;
    int32_t b;
    int32_t T;               /* total iterations, split over levels */
    double sigma;            /* Gaussian width of the similarity */
    float gamma;             /* weight of negatives on all but the coarsest level */
    float gamma_coarsest;    /* on the coarsest level when there are >= 2 levels */
    float eta0;              /* initial step size, decays linearly per level */
    float clip;
    double rho;              /* coarsening stops when |V^{l+1}| > rho |V^l| */
    int32_t min_nodes;       /* do not coarsen a level with fewer active nodes */
    int32_t max_levels;      /* at most this many levels (1 = single level) */
    int32_t mode;            /* DRG_MODE_SYNC or DRG_MODE_ASYNC */
    int32_t dim;             /* 2 (or 0) or 3: coordinates [n][dim] (Sec. 3.1) */
    uint64_t seed;
    int32_t b_half;          /* 1: the shape is b + 1/2 (b = 1 or 2) */
    int32_t _pad;
    double perplexity;       /* 0: one sigma for all nodes; >= 1: node-wise sigma_i
                                calibrated to it (drg_build_similarity_perplexity) */
} drg_layout_params;

/* Parameters of the sampled objective (Eq. objectfunction). */
typedef struct {
    int32_t M;               /* negatives per node, >= 0 */
    int32_t b;               /* 1..3 */
    double gamma;
    uint64_t seed;
    uint64_t iter;           /* keys the negatives like drg_layout_step */
    int32_t dim;             /* 2 (or 0) or 3: coordinates [n][dim] */
    int32_t b_half;          /* 1: the shape is b + 1/2 (b = 1 or 2) */
} drg_obj_params;

const char* drg_last_error(void);
const char* drg_version(void);

/* Fills *p with the paper's defaults: k=1, M=5, b=2, T=400, sigma=1,
 * gamma=0.1, gamma_coarsest=0.01, eta0=1, clip=4, rho=0.8, min_nodes=1000,
 * max_levels=64, sync mode, seed 0 (Sec. 4 "Parameters", Sec. 3.2.3). */
drg_status drg_layout_params_default(drg_layout_params* p);

/* Source of device memory: alloc(bytes, user) returns device memory of the
 * context's device, at least `bytes` bytes, 256-byte aligned, or NULL when it
 * cannot; free(ptr, user) releases what alloc returned.  Both are called on
 * the thread of the drg_* call that needs them (destroy calls included). */
typedef struct {
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* ptr, void* user);
    void* user;
} drg_allocator;

/* Creates a context on `device` that enqueues on `hip_stream` (a hipStream_t;
 * NULL = the null stream).  The stream is borrowed and must outlive ctx.
 * alloc (nullable; copied): every device buffer that calls on this context
 * create -- similarities, hierarchies, batches and per-call scratch -- comes
 * from it and goes back to it, also when the object is destroyed after the
 * context; NULL = hipMalloc / hipFree.  When it returns NULL the call fails
 * with DRG_E_OOM after freeing what it had allocated.  DRG_E_INVALID when
 * alloc lacks a function. */
drg_status drg_ctx_create(int32_t device, void* hip_stream, const drg_allocator* alloc,
                          drg_ctx** out);
void drg_ctx_destroy(drg_ctx* ctx);
drg_status drg_ctx_synchronize(drg_ctx* ctx);
/* Kernel timing: when on, the library brackets every launch of the layout
 * iteration's sweep kernel with HIP events on the context's stream.
 * drg_ctx_kernel_stats synchronises and returns the launch count and the
 * summed duration in milliseconds since the last reset. */
drg_status drg_ctx_set_profiling(drg_ctx* ctx, int32_t on);
drg_status drg_ctx_kernel_stats(drg_ctx* ctx, int64_t* launches, double* total_ms);
/* *form = the DRG_SWEEP_* form that the latest drg_layout_step (or layout
 * run) on this context launched, -1 before the first. */
drg_status drg_ctx_last_sweep(const drg_ctx* ctx, int32_t* form);

/* Sparse distance matrix and node similarity (Sec. 3.2.1, Eq. NS):
 * for every node i the set NNG(i, k) = {j != i : SPD(i, j) <= k} with hop
 * d_ij = SPD(i, j), by bounded breadth-first search; then
 *   e_d = exp(-d^2 / (2 sigma^2)),  Z_i = sum_{j in NNG(i,k)} e_{d_ij},
 *   P~_ij = e_{d_ij} (1/Z_i + 1/Z_j) / 2   (= N_a * NS_ij, symmetric),
 *   qt_i  = sum_j P~_ij                     (node weight, Sec. 3.2.2),
 * plus the integer table used to draw negatives with probability
 * proportional to the node weight.  k in 1..4, n < 2^30.
 * Synchronises.  The result lives in device memory owned by *out. */
drg_status drg_build_similarity(drg_ctx* ctx, const drg_csr* g, int32_t k, double sigma,
                                uint32_t flags, drg_sim** out);
/* The same similarity with one sigma_i per node (Eq. NS writes sigma_i), each
 * chosen so that the conditional distribution NS_{.|i} over NNG(i, k) has
 * the given perplexity exp(H_i), H_i its entropy in nats (the calibration
 * of t-SNE, on which the method builds).  With t_i = exp(-1/(2 sigma_i^2))
 * the Gaussian of hop d is t_i^(d^2); t_i is found by 64 bisection steps
 * on (0, 1) (the entropy grows with t), or is 1 (uniform over NNG(i, k))
 * when ln(perplexity) >= ln |NNG(i, k)|.  Then
 *   NS_{j|i} = t_i^(d_ij^2) / Z_i,  P~_ij = (NS_{j|i} + NS_{i|j}) / 2,
 * with qt, the sampling table and 1/Z as for drg_build_similarity.  The
 * calibration uses IEEE-754 operations only (its logarithm is the atanh
 * series), so its results are reproducible bit for bit.  Such a similarity
 * is swept by the row-form kernels (no column-blocked copy).
 * perplexity >= 1 and finite; k in 1..4.  Synchronises. */
drg_status drg_build_similarity_perplexity(drg_ctx* ctx, const drg_csr* g, int32_t k,
                                           double perplexity, uint32_t flags, drg_sim** out);
/* The similarity of a weighted graph (weighted graphs are named as future
 * work in Sec. 6; Eq. NS is written with the graph distance GD).
 * length_dev[nnz] (device, FP64): one positive finite length per CSR entry,
 * equal for (u, v) and (v, u).  NNG(i, k) is the hop-defined pattern; GD_ij
 * is the length of the shortest i-j path of at most k edges (k rounds of
 * Bellman-Ford from each source, each round from the previous round's
 * distances), the smaller of the two directions; then
 *   E_ij = exp(-GD_ij^2 / (2 sigma^2)),  Z_i = sum_l E_il,
 *   P~_ij = E_ij (1/Z_i + 1/Z_j) / 2,
 * with qt, the sampling table and 1/Z as for drg_build_similarity (unit
 * lengths give that similarity up to the order of Z's sum).  The exponential
 * is computed from IEEE-754 operations only (Cody-Waite reduction, Taylor
 * series), so the results are reproducible bit for bit.  The structure is
 * always validated (as with DRG_VALIDATE); DRG_E_INVALID for a bad length or
 * asymmetric lengths.  Swept by the row-form kernels (no column-blocked
 * copy); coarsening (drg_coarsen) uses the structure only.  Peak device
 * memory of the build: 24 bytes per pattern entry besides the pattern.
 * Synchronises. */
drg_status drg_build_similarity_weighted(drg_ctx* ctx, const drg_csr* g,
                                         const double* length_dev, int32_t k, double sigma,
                                         uint32_t flags, drg_sim** out);
/* sigma_i of every node into sigma_host[n] (host; synchronises): the global
 * sigma, or for a node-wise similarity sqrt(-1/(2 ln t_i)) (+inf where t_i = 1);
 * 0 for isolated nodes. */
drg_status drg_sim_node_sigma(const drg_sim* s, double* sigma_host);
/* Host-side sizes (no synchronisation needed); *blocked (nullable) is 1 when
 * the synchronous FP32 sweep runs over the column-blocked copy of P~. */
drg_status drg_sim_info(const drg_sim* s, int32_t* n, int64_t* nnz, int32_t* n_active,
                        int32_t* k, int32_t* blocked);
/* Copies the similarity to host arrays (each nullable; synchronises):
 * row_ptr[n+1], col[nnz], hop[nnz] (1..k), P[nnz] (FP64 P~_ij), qt[n] (FP64),
 * W[n] (uint64 sampling weights), e[k] (FP64 exp(-d^2 / (2 sigma^2)) per
 * hop d; zeros for a node-wise similarity; for a weighted similarity the same
 * hop values, which its P~ does not use), invZ[n] (FP64). */
drg_status drg_sim_export(const drg_sim* s, int64_t* row_ptr, int32_t* col, uint8_t* hop,
                          double* P, double* qt, uint64_t* W, double* e, double* invZ);
/* Copies the rows rows[0..nrows) of the similarity to host arrays (each
 * nullable; synchronises), for graphs whose whole pattern is too large to
 * copy: row_len[nrows] entries per row; col, hop (1..k) and P (FP64 P~_ij)
 * of the rows one after another in the order of `rows`, each row in
 * ascending column order; qt[nrows], W[nrows], invZ[nrows] of the rows.
 * cap = capacity of col/hop/P in entries.  DRG_E_INVALID when a row index is
 * out of range or the rows hold more than cap entries (row_len is still
 * written). */
drg_status drg_sim_export_rows(const drg_sim* s, int32_t nrows, const int32_t* rows,
                               int64_t cap, int64_t* row_len, int32_t* col, uint8_t* hop,
                               double* P, double* qt, uint64_t* W, double* invZ);
/* Layout quality: neighbourhood preservation (Sec. 4.1, Eq. NP) of the nodes
 * nodes[0..count) (device int32).  For node v with graph neighbourhood
 * N_G(v) = NNG(v, k) -- the rows of `s`, so build it with k = k_eval -- and
 * m = |N_G(v)| > 0, N_L(v) is the set of the m nodes u != v nearest to y_v
 * (squared distance in FP64 from the FP32 coordinates y [n][2], device;
 * ties by smaller id), and np_out[t] (device double) = |N_G & N_L| /
 * |N_G | N_L| for v = nodes[t]; -1 when m = 0.  Exact selection, one
 * workgroup per node, O(n) work per node.  Enqueued on the context's stream
 * (asynchronous; np_out is ready after drg_ctx_synchronize).  DRG_E_INVALID
 * for a node id out of range, DRG_E_UNSUPPORTED for n >= 2^24. */
drg_status drg_neighbourhood_preservation(drg_ctx* ctx, const drg_sim* s, const float* y,
                                          int32_t count, const int32_t* nodes, double* np_out);
/* Layout quality: sampled normalised stress (Sec. 4.1).  The stress with
 * weights 1/SPD^2 and the best scale alpha is (P - A^2/B) / |V|^2, with
 * A = sum L/D, B = sum L^2/D^2 over the P pairs summed (L = layout distance,
 * D = shortest-path distance; unreachable pairs carry weight 0).  For each
 * source sources[t] (device int32, count of them) this writes, over the
 * pairs (source, j) with j reachable and j != source, sums_out[3t..3t+2] =
 * (A, B, P) (device double); the sampled estimate of the stress is then
 * (n / count) (sum P - (sum A)^2 / sum B) / n^2.  Distances by breadth-first
 * search over the whole graph g (device CSR, as for drg_build_similarity);
 * y [n][2] FP32 device coordinates, L in FP64.  Sums in ascending node id:
 * repeatable.  *estimate (host, nullable) receives that sampled estimate,
 * the sums added over the sources in the order given.  Scratch: 8 n bytes
 * per concurrently searched source.  Synchronises.  DRG_E_INVALID for a
 * source id out of range. */
drg_status drg_stress_sampled(drg_ctx* ctx, const drg_csr* g, const float* y, int32_t count,
                              const int32_t* sources, double* sums_out, double* estimate);
void drg_sim_destroy(drg_sim* s);

/* Multilevel coarsening (Sec. 3.2.3, Fig. 3): repeatedly groups a randomly
 * chosen node with its unassigned first-order neighbours into one coarse node
 * until every node is assigned; edges inside a group disappear.  Levels are
 * added while the level has at least min_nodes non-isolated nodes and fewer
 * than max_levels levels exist; a new level with more than rho times the
 * non-isolated nodes of its parent is discarded and coarsening stops.
 * Random choices come from `seed`.  Synchronises. */
drg_status drg_coarsen(drg_ctx* ctx, const drg_csr* g, uint64_t seed, double rho,
                       int32_t min_nodes, int32_t max_levels, drg_hier** out);
/* levels (>= 1) and, if sizes_host is non-null, sizes_host[levels] node counts. */
drg_status drg_hier_info(const drg_hier* h, int32_t* levels, int32_t* sizes_host);
/* For level >= 1 (host arrays, each nullable; synchronises):
 * map[n_{level-1}]: node of level-1 -> node of level; cmap[n_0]: finest node
 * -> node of level; coarse_rp[n_level+1] and coarse_col[nnz_level]: the
 * contracted graph G^level.  coarse_nnz (nullable) receives nnz_level. */
drg_status drg_hier_export(const drg_hier* h, int32_t level, int32_t* map, int32_t* cmap,
                           int32_t* coarse_rp, int32_t* coarse_col, int64_t* coarse_nnz);
/* fine_to_level[n_0] (host): the node of `level` that each finest node
 * belongs to (the composed grouping of Sec. 3.2.3); level 0 is refused
 * (DRG_E_INVALID), its map being the identity.  Synchronises. */
drg_status drg_hier_export_map(const drg_hier* h, int32_t level, int32_t* fine_to_level);
void drg_hier_destroy(drg_hier* h);

/* Random layout of a level (Sec. 3.2.3): y[v] = (2u-1, 2u-1) with 24-bit
 * uniform fractions u from Philox(seed, node v, level).  y_dev: [n][2]. */
drg_status drg_init_layout(drg_ctx* ctx, int32_t n, uint64_t seed, int32_t level, float* y_dev);
/* Refinement (Sec. 3.2.3): y_finer[u] = y_level[map_level(u)] for every node u
 * of level-1.  level >= 1. */
drg_status drg_prolong(drg_ctx* ctx, const drg_hier* h, int32_t level, const float* y_level_dev,
                       float* y_finer_dev);
/* The same in R^3 (Sec. 3.1): coordinates [n][3]; coordinate c of node v is
 * (2u-1) with u from Philox word c of (seed, node v, level), so the first
 * two are those of drg_init_layout.  FP64 instances for trajectory checks. */
drg_status drg_init_layout_3d(drg_ctx* ctx, int32_t n, uint64_t seed, int32_t level,
                              float* y_dev);
drg_status drg_prolong_3d(drg_ctx* ctx, const drg_hier* h, int32_t level,
                          const float* y_level_dev, float* y_finer_dev);
drg_status drg_init_layout_3d_f64(drg_ctx* ctx, int32_t n, uint64_t seed, int32_t level,
                                  double* y_dev);
drg_status drg_prolong_3d_f64(drg_ctx* ctx, const drg_hier* h, int32_t level,
                              const double* y_level_dev, double* y_finer_dev);

/* One optimisation iteration at level p->level (Sec. 3.2.2 with the
 * gradient sharing of Sec. 3.2.3).  For every non-isolated finest node i,
 * with a = c(i) its node on the level:
 *   g_i = sum_j P~_ij clip(A(y_a - y_c(j))) + gamma qt_i sum_{m<M} clip(R(y_a - y_c(v_im)))
 *   A(D) = -2b |D|^{2b-2} D / (1 + |D|^{2b}),  R(D) = 2b D / (|D|^2 (1 + |D|^{2b}))
 * (the attractive and repulsive forces of Eq. gradient) with v_im the
 * negatives drawn by node weight from (seed, iter, i, m); clip is per pair and
 * per component; a pair at distance 0 contributes nothing.  Node i is selected
 * about qt_i times per iteration by the paper's SGD, so a level node moves by
 * the average of its members' selections:
 *   sync : y_a += eta * (sum_{c(i)=a} g_i) / (sum_{c(i)=a} qt_i), all g_i from
 *          one snapshot (deterministic, bit-for-bit repeatable);
 *   async: eta * g_i / (sum_{c(j)=c(i)} qt_j) is added to y_c(i) as soon as g_i
 *          is computed, while other nodes read y (Hogwild-style: not
 *          repeatable).  On a similarity with the column-blocked copy the
 *          rows are cut into DRG_ASYNC_STAGES (environment, default 4)
 *          equal ranges, moved range by range once all their pairs are
 *          summed; later ranges see the moves of earlier ones.
 * h may be NULL for level 0.  y_level_dev: [n_level][dim], in/out (p->dim
 * 3: the same step in R^3, row-form sweep). */
drg_status drg_layout_step(drg_ctx* ctx, const drg_sim* s, const drg_hier* h,
                           const drg_step_params* p, float* y_level_dev);

/* FP64 instances of drg_init_layout, drg_prolong and drg_layout_step (sync
 * mode only; async returns DRG_E_UNSUPPORTED): the same kernels and the same
 * order of operations with double coordinates, for trajectory checks against
 * an FP64 reference. */
drg_status drg_init_layout_f64(drg_ctx* ctx, int32_t n, uint64_t seed, int32_t level,
                               double* y_dev);
drg_status drg_prolong_f64(drg_ctx* ctx, const drg_hier* h, int32_t level,
                           const double* y_level_dev, double* y_finer_dev);
drg_status drg_layout_step_f64(drg_ctx* ctx, const drg_sim* s, const drg_hier* h,
                               const drg_step_params* p, double* y_level_dev);

/* Sampled objective (Eq. objectfunction), the form used with an autograd
 * system (Sec. 5: further cost terms can be added to the objective):
 *   L^(Y) = sum_i sum_j P~_ij log w_ij + gamma sum_i qt_i sum_{m<M} log(1 - w_{i v_im})
 * with w = 1/(1 + |y_i - y_j|^{2b}) and the negatives v_im of drg_layout_step
 * for (seed, iter); a negative equal to its node or at distance 0 adds 0.
 * y_dev: [n][2] finest-level coordinates.  loss_dev: one device scalar
 * (the row values summed in a fixed order), or NULL; rows_dev: [n] the value
 * of each row i (its attraction terms plus gamma qt_i times its negatives'
 * terms), or NULL; not both NULL.  Synchronises.  No clipping (this is the
 * objective, not the step). */
drg_status drg_objective_fwd(drg_ctx* ctx, const drg_sim* s, const drg_obj_params* p,
                             const float* y_dev, float* loss_dev, float* rows_dev);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the loss of
 * drg_objective_fwd (same kernels, same fixed-order sum, so the same bits)
 * with no allocation of any kind.  Its scratch -- the n row values and the
 * block sums of the reduction, 4 (2^20 + 2048) bytes -- is a static device
 * array that each GPU the library runs on holds until the process ends;
 * every call on a GPU reuses that GPU's array, so calls that overlap on one
 * GPU (other streams, other threads) race and must be serialised by the
 * caller.  The array needs no clearing: every value in it is written before
 * it is read.  Enqueued on the context's stream, no synchronisation: the
 * loss is in loss_dev (one device float) once the stream reaches it.
 * DRG_E_INVALID when the similarity has more than 2^20 nodes (the size of
 * the static scratch), or for a NULL argument, M < 0 or b outside 1..3. */
drg_status drg_objective_fwd_noalloc(drg_ctx* ctx, const drg_sim* s, const drg_obj_params* p,
                                     const float* y_dev, float* loss_dev);
/* dy_dev[n][2] = dloss * dL^/dY (exact gradient of the sampled objective).
 * The negatives are drawn again from their counters (nothing is stored by
 * the forward); contributions to a drawn node are summed in a fixed order,
 * so the result is deterministic.  dloss_dev: device scalar or NULL (= 1).
 * Synchronises. */
drg_status drg_objective_bwd(drg_ctx* ctx, const drg_sim* s, const drg_obj_params* p,
                             const float* y_dev, const float* dloss_dev, float* dy_dev);
/* FP64 instances (double coordinates, loss and gradient; FP64 P~ and qt). */
drg_status drg_objective_fwd_f64(drg_ctx* ctx, const drg_sim* s, const drg_obj_params* p,
                                 const double* y_dev, double* loss_dev, double* rows_dev);
drg_status drg_objective_bwd_f64(drg_ctx* ctx, const drg_sim* s, const drg_obj_params* p,
                                 const double* y_dev, const double* dloss_dev, double* dy_dev);
/* The negatives of (seed, iter): out_dev[n][M] node ids, -1 for an isolated
 * anchor.  For checks and for reference implementations. */
drg_status drg_sample_negatives(drg_ctx* ctx, const drg_sim* s, int32_t M, uint64_t seed,
                                uint64_t iter, int32_t* out_dev);
/* P~ as device COO in CSR order (each pointer nullable): rows_dev[nnz],
 * cols_dev[nnz], P_dev[nnz] (FP32, from the FP32 1/Z). */
drg_status drg_sim_coo(drg_ctx* ctx, const drg_sim* s, int32_t* rows_dev, int32_t* cols_dev,
                       float* P_dev);

/* The multilevel layout of Sec. 3.2.3 on a built similarity and hierarchy:
 * random layout of the coarsest level, the iterations of Sec. 3.2.2 level by
 * level from the coarsest down, each level's result copied to the next finer
 * level (refinement).  T (Sec. 4.2: iteration number) is the total over the
 * levels, split evenly, the finest taking the remainder; the step is
 * eta0 (1 - t/T_l), restarting per level; the coarsest of two or more levels
 * uses gamma_coarsest (Sec. 4.2, weight of negative samples).  Iteration t of
 * level l has the global index (iterations of the coarser levels) + t, which
 * keys its negatives.  y_out_dev: [n][2].  Synchronises. */
drg_status drg_layout_run(drg_ctx* ctx, const drg_sim* s, const drg_hier* h,
                          const drg_layout_params* p, float* y_out_dev);
/* Checkpoint and resume of that schedule.  drg_layout_run_until runs it from
 * the start until t iterations of `level` are done (0 <= t <= T_level; t =
 * T_level is before the refinement to level-1) and writes that level's
 * coordinates to y_level_dev [n_level][2].  drg_layout_resume continues from
 * such a state (level, t, y_level_dev) to the end and writes the finest
 * coordinates to y_out_dev [n][2].  In sync mode a run cut anywhere and
 * resumed gives the same bits as drg_layout_run.  DRG_E_INVALID for a point
 * outside the schedule.  Both synchronise. */
drg_status drg_layout_run_until(drg_ctx* ctx, const drg_sim* s, const drg_hier* h,
                                const drg_layout_params* p, int32_t level, int32_t t,
                                float* y_level_dev);
drg_status drg_layout_resume(drg_ctx* ctx, const drg_sim* s, const drg_hier* h,
                             const drg_layout_params* p, int32_t level, int32_t t,
                             const float* y_level_dev, float* y_out_dev);

/* End to end (Sec. 3.1: undirected graph in, positions out; Sec. 3.2 stages
 * in order): drg_build_similarity + drg_coarsen + drg_layout_run. */
drg_status drg_layout(drg_ctx* ctx, const drg_csr* g, const drg_layout_params* p,
                      float* y_out_dev);

/* ------------------------------------------------------------------ batches
 * Many independent graphs laid out together (Sec. 3.2.2 iteration, Sec. 3.2.3
 * multilevel scheme, synchronous mode).  graphs[count] and params[count] are
 * host arrays; each drg_csr holds DEVICE pointers of one graph (the same
 * contract as drg_layout: symmetric, sorted rows, no self-loops).  Every
 * graph keeps its own parameters (M, b, T, gamma, gamma_coarsest, eta0, clip,
 * rho, min_nodes, max_levels, seed); k and sigma must be equal over the batch
 * and mode must be DRG_MODE_SYNC (else DRG_E_INVALID / DRG_E_UNSUPPORTED).
 * The coordinates of graph c come out as the rows base_c .. base_c + n_c - 1
 * of y_out_dev (float [sum n_c][2], device), base_c = n_0 + ... + n_{c-1},
 * and equal, bit for bit, what drg_layout gives for that graph alone when its
 * single-graph sweep is the row-per-group one (graphs below the column-blocked
 * threshold).  The union must stay below 2^30 nodes and 2^31 input edges.
 *
 * drg_batch_create builds the similarity of all graphs at once, one hierarchy
 * per graph and the per-graph schedules, then records the whole run (initial
 * layout, T iterations, prolongations) into one hipGraph; the batch owns its
 * device memory and the input graphs are not read afterwards.
 * drg_batch_run replays that graph on the context's stream and copies the
 * finest coordinates to y_out_dev; it returns when they are there.  Runs of
 * one batch must not overlap. */
drg_status drg_batch_create(drg_ctx* ctx, const drg_csr* graphs, int32_t count,
                            const drg_layout_params* params, drg_batch** out);
/* Sizes: total nodes, total pattern entries, iterations of the longest
 * schedule; nodes_host[count] and levels_host[count] (host, optional). */
drg_status drg_batch_info(const drg_batch* b, int64_t* n_total, int64_t* nnz_total, int32_t* T,
                          int32_t* nodes_host, int32_t* levels_host);
/* The sweep forms drg_batch_create timed on the batch (it picks the fastest;
 * all give the same bits): *n candidates; for i < cap, rpl[i] = 0 for the row
 * form (a group of lanes per row, records gathered from global memory) or the
 * rows per group of the LDS-windowed form, ch[i] its LDS chunk in records,
 * ms[i] the time of one sweep; *chosen = index of the form in use (-1 when the
 * form was forced by the environment and nothing was timed).  Host arrays,
 * each optional. */
drg_status drg_batch_tuning(const drg_batch* b, int32_t cap, int32_t* n, int32_t* chosen,
                            int32_t* rpl, int32_t* ch, float* ms);
drg_status drg_batch_run(drg_ctx* ctx, drg_batch* b, float* y_out_dev);
void drg_batch_destroy(drg_batch* b);
/* One shot: create, run once, destroy. */
drg_status drg_layout_batched(drg_ctx* ctx, const drg_csr* graphs, int32_t count,
                              const drg_layout_params* params, float* y_out_dev);

#pragma GCC visibility pop
#ifdef __cplusplus
}
#endif
#endif
