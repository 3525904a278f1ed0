/*
 * drgo.h -- CPU oracle for the DRGraph layout hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded FP64
 * implementation of what the layout method computes, written from the
 * paper's definitions (Zhu et al., "DRGraph: An Efficient Graph Layout
 * Algorithm for Large-scale Graphs by Dimensionality Reduction").  It exists
 * to check the GPU library.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code with the GPU
 * library: no headers, no helpers, no tables.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared drgo.c -o libdrgo.so -lm
 * (-ffp-contract=off: every FP64 operation rounds on its own, so the values
 * that decide integers -- the sampling weights -- are reproducible.)
 *
 * Conventions shared with the GPU side by definition (not by code):
 *   - Philox4x64-10 counter RNG (Salmon et al., SC'11), key = {seed, tag},
 *     counter = {a, b, c, 0}; tags below.
 *   - e_d = exp(-d^2 / (2 sigma^2)), d = 1..k, computed with libm exp.
 *   - Z_i = sum_{d=1..k} cnt_i(d) * e_d, accumulated from 0 in d order.
 *   - invZ_i = 1 / Z_i (0 for an isolated node).
 *   - P~_ij = ((invZ_i + invZ_j) * e_d) * 0.5       (d = SPD(i, j) <= k)
 *   - W_i = sum_j trunc(P~_ij * 2^32)  (uint64), C = exclusive prefix of W.
 *   - negative draw from word w: r = floor(w * S / 2^64), S = C[n];
 *     node = smallest v with C[v+1] > r.
 */
#ifndef DRGO_H
#define DRGO_H
#include <stdint.h>

#define DRGO_TAG_INIT 1u
#define DRGO_TAG_COARSEN 2u
#define DRGO_TAG_NEG 3u

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x64-10: out = bijection_{key}(ctr). */
void drgo_philox(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* k-order neighbourhoods NNG(v, k) by breadth-first search (Sec. 3.2.1).
 * count: writes out_rp[0..n] (int64 row offsets), returns nnz.
 * fill : writes out_col[nnz] (ascending within each row) and out_hop[nnz]. */
int64_t drgo_khop_count(int32_t n, const int32_t* rp, const int32_t* col, int32_t k, int64_t* out_rp);
void drgo_khop_fill(int32_t n, const int32_t* rp, const int32_t* col, int32_t k,
                    const int64_t* out_rp, int32_t* out_col, uint8_t* out_hop);

/* Node similarity over the sparse distance matrix (Eq. NS and its sparse
 * form, Sec. 3.2.1), symmetrised and scaled so that P~ = N_a * NS. */
void drgo_similarity(int32_t n, int32_t k, double sigma, const int64_t* prp, const int32_t* pcol,
                     const uint8_t* phop, double* e, double* Z, double* invZ, double* P, double* qt,
                     uint64_t* W, uint64_t* C);

/* Node-wise sigma_i calibrated to a perplexity (Eq. NS with one sigma per
 * node; t-SNE's calibration): per node t_i = exp(-1/(2 sigma_i^2)) in
 * tnode[n], the conditional probabilities NS_{j|i} of hop d in A[i*k + d-1],
 * Z, invZ, and P~_ij = (NS_{j|i} + NS_{i|j}) / 2 with qt, W, C as in
 * drgo_similarity.  Returns -1 for k outside 1..8 or perplexity < 1. */
int32_t drgo_similarity_perplexity(int32_t n, int32_t k, double perplexity, const int64_t* prp,
                                   const int32_t* pcol, const uint8_t* phop, double* tnode,
                                   double* A, double* Z, double* invZ, double* P, double* qt,
                                   uint64_t* W, uint64_t* C);
/* Natural logarithm from IEEE operations only (atanh series), x > 0. */
double drgo_ln(double x);

/* Weighted graphs: len[e] > 0 per CSR entry (symmetric).  gd[x] = length of
 * the shortest path of at most k edges for pattern entry x, the smaller of
 * the two directions; then E = exp(-gd^2/(2 sigma^2)), Z, invZ, P~ = E (1/Z_i
 * + 1/Z_j)/2, qt, W, C as in drgo_similarity. */
void drgo_hop_bounded_dist(int32_t n, const int32_t* rp, const int32_t* col, const double* len,
                           int32_t k, const int64_t* prp, const int32_t* pcol, double* gd);
void drgo_similarity_weighted(int32_t n, double sigma, const int64_t* prp, const int32_t* pcol,
                              const double* gd, double* E, double* Z, double* invZ, double* P,
                              double* qt, uint64_t* W, uint64_t* C);
/* e^x for x <= 0 from IEEE operations only (0 below -708). */
double drgo_exp_neg(double x);

/* The same similarity for the rows srcs[0..nsrc) only (k <= 8): out_rp[nsrc+1]
 * row offsets; with out_col non-NULL also the rows' columns (ascending), hops,
 * P~ values, and per row 1/Z, qt and W.  Returns the number of entries. */
int64_t drgo_similarity_rows(int32_t n, const int32_t* rp, const int32_t* col, int32_t k,
                             double sigma, int32_t nsrc, const int32_t* srcs, int64_t* out_rp,
                             int32_t* out_col, uint8_t* out_hop, double* out_P, double* out_invZ,
                             double* out_qt, uint64_t* out_W);

/* Negative-sample draw from a 64-bit uniform word (node weight sampling). */
int32_t drgo_draw(const uint64_t* C, int32_t n, uint64_t w);
/* The word for slot m of node i at iteration it. */
uint64_t drgo_neg_word(uint64_t seed, uint64_t it, int32_t i, int32_t m);

/* One coarsening level (Sec. 3.2.3): returns n_coarse, writes map[n]. */
int32_t drgo_coarsen_level(int32_t n, const int32_t* rp, const int32_t* col, uint64_t seed,
                           int32_t level, int32_t* map);
/* Contract edges through map: returns coarse nnz; out_rp[nc+1], out_col cap >= rp[n]. */
int64_t drgo_contract(int32_t n, const int32_t* rp, const int32_t* col, const int32_t* map,
                      int32_t nc, int32_t* out_rp, int32_t* out_col);

/* Coordinates are points of R^dim, dim = 2 or 3 (Sec. 3.1), stored [n][dim].
 * b (the proximity shape of Eq. gradient) is a whole or half number. */
/* Random initial layout of the coarsest level. */
void drgo_init(int32_t nl, uint64_t seed, int32_t level, double* y, int32_t dim);

/* One-sided step direction g_i of every fine node i (attraction over row i
 * plus gamma * qt_i * M sampled repulsions), evaluated at level coordinates
 * y (fine node i sits at y[cmap[i]]; cmap NULL = identity).  Per-pair,
 * per-component clipping at +-clip (pass INFINITY for none). */
void drgo_step_direction(int32_t n0, const int64_t* prp, const int32_t* pcol, const double* P,
                         const double* qt, const uint64_t* C, const int32_t* cmap, const double* y,
                         int32_t M, double b, double gamma, double clip, uint64_t seed,
                         uint64_t it, double* g, int32_t dim);
/* Synchronous (Jacobi) iteration:
 * y[a] += eta * (sum_{cmap[i]=a} g_i) / (sum_{cmap[i]=a} qt_i). */
void drgo_iter_sync(int32_t n0, const int64_t* prp, const int32_t* pcol, const double* P,
                    const double* qt, const uint64_t* C, const int32_t* cmap, int32_t nl, double* y,
                    int32_t M, double b, double gamma, double eta, double clip, uint64_t seed,
                    uint64_t it, int32_t dim);
/* Sequential (Gauss-Seidel) iteration in ascending fine-node order. */
void drgo_iter_seq(int32_t n0, const int64_t* prp, const int32_t* pcol, const double* P,
                   const double* qt, const uint64_t* C, const int32_t* cmap, int32_t nl, double* y,
                   int32_t M, double b, double gamma, double eta, double clip, uint64_t seed,
                   uint64_t it, int32_t dim);

/* Sampled objective L^ (Eq. objectfunction with the expectation over
 * positives taken exactly and M negatives drawn per node) and its exact
 * two-sided gradient, unclipped, at level-0 coordinates y[n][dim]. */
double drgo_objective(int32_t n, const int64_t* prp, const int32_t* pcol, const double* P,
                      const double* qt, const uint64_t* C, const double* y, int32_t M, double b,
                      double gamma, uint64_t seed, uint64_t it, int32_t dim);
void drgo_objective_grad(int32_t n, const int64_t* prp, const int32_t* pcol, const double* P,
                         const double* qt, const uint64_t* C, const double* y, int32_t M, double b,
                         double gamma, uint64_t seed, uint64_t it, double* grad, int32_t dim);

/* Expected objective L (negatives averaged over the sampling distribution
 * W/S instead of drawn) and its gradient; O(n^2), tiny graphs only. */
double drgo_objective_exact(int32_t n, const int64_t* prp, const int32_t* pcol, const double* P,
                            const double* qt, const uint64_t* C, const double* y, int32_t M,
                            double b, double gamma, int32_t dim);
void drgo_objective_exact_grad(int32_t n, const int64_t* prp, const int32_t* pcol, const double* P,
                               const double* qt, const uint64_t* C, const double* y, int32_t M,
                               double b, double gamma, double* grad, int32_t dim);
/* Expectation of the one-sided step direction over the negative draws,
 * unclipped; O(n^2). */
void drgo_step_expected(int32_t n, const int64_t* prp, const int32_t* pcol, const double* P,
                        const double* qt, const uint64_t* C, const double* y, int32_t M, double b,
                        double gamma, double* g, int32_t dim);

#ifdef __cplusplus
}
#endif
#endif
