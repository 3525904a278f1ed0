/*
 * drgo.c -- CPU oracle for the DRGraph layout hot path (see drgo.h).
 *
 * TEST INFRASTRUCTURE ONLY: plain, slow, single-threaded FP64 code written
 * from the paper's definitions.  Each function names the passage it follows.
 * Parity pins for every function live in tests/ (marked "not gpu").
 */
#include "drgo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of two 64x64->128 multiplies with    */
/* the published multipliers and Weyl key increments.                        */
/* ------------------------------------------------------------------------ */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void drgo_philox(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, x0, &hi0, &lo0);
        mulhilo64(M1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

static void philox_stream(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b, uint64_t c,
                          uint64_t out[4]) {
    uint64_t ctr[4] = {a, b, c, 0};
    uint64_t key[2] = {seed, tag};
    drgo_philox(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* k-order nearest neighbours NNG(v_i, k) = {v : SPD(v_i, v) <= k, v != v_i} */
/* (Sec. 3.2.1), by plain breadth-first search bounded at depth k.           */
/* ------------------------------------------------------------------------ */
static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* BFS from src; fills q[0..ret) with reached nodes (q[0] = src) and dist[]. */
static int32_t bfs_bounded(const int32_t* rp, const int32_t* col, int32_t k, int32_t src,
                           int32_t* dist, int32_t* q) {
    int32_t head = 0, tail = 0;
    dist[src] = 0;
    q[tail++] = src;
    while (head < tail) {
        int32_t u = q[head++];
        if (dist[u] >= k) continue;
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
            int32_t v = col[e];
            if (dist[v] < 0) {
                dist[v] = dist[u] + 1;
                q[tail++] = v;
            }
        }
    }
    return tail;
}

int64_t drgo_khop_count(int32_t n, const int32_t* rp, const int32_t* col, int32_t k,
                        int64_t* out_rp) {
    int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* q = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t v = 0; v < n; ++v) dist[v] = -1;
    out_rp[0] = 0;
    for (int32_t s = 0; s < n; ++s) {
        int32_t t = bfs_bounded(rp, col, k, s, dist, q);
        out_rp[s + 1] = out_rp[s] + (t - 1);
        for (int32_t x = 0; x < t; ++x) dist[q[x]] = -1;
    }
    free(dist);
    free(q);
    return out_rp[n];
}

void drgo_khop_fill(int32_t n, const int32_t* rp, const int32_t* col, int32_t k,
                    const int64_t* out_rp, int32_t* out_col, uint8_t* out_hop) {
    int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* q = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t v = 0; v < n; ++v) dist[v] = -1;
    for (int32_t s = 0; s < n; ++s) {
        int32_t t = bfs_bounded(rp, col, k, s, dist, q);
        int64_t o = out_rp[s];
        /* reached nodes except the source, ascending by id */
        qsort(q + 1, (size_t)(t - 1), sizeof(int32_t), cmp_i32);
        for (int32_t x = 1; x < t; ++x) {
            out_col[o + x - 1] = q[x];
            out_hop[o + x - 1] = (uint8_t)dist[q[x]];
        }
        for (int32_t x = 0; x < t; ++x) dist[q[x]] = -1;
    }
    free(dist);
    free(q);
}

/* ------------------------------------------------------------------------ */
/* Node similarity (Eq. NS; sparse form in Sec. 3.2.1).                      */
/*   NS_{j|i} = e_{d_ij} / Z_i,  Z_i = sum_{l in NNG(i,k)} e_{d_il}          */
/*   NS_ij    = (NS_{i|j} + NS_{j|i}) / (2|V|)                               */
/* The Gaussian is precomputed for the k hop values; Z_i is the hop         */
/* histogram weighted by it.  We keep P~ = N_a * NS with N_a the number of  */
/* non-isolated nodes (the paper's graphs have none isolated, so N_a = |V|).*/
/* The node weight used for negative sampling is sum_l NS_{j,l} (Sec.       */
/* 3.2.2), i.e. qt_j / N_a; it is quantised per entry to 2^-32 so that the */
/* sampling distribution is an exact integer table.                         */
/* ------------------------------------------------------------------------ */
void drgo_similarity(int32_t n, int32_t k, double sigma, const int64_t* prp, const int32_t* pcol,
                     const uint8_t* phop, double* e, double* Z, double* invZ, double* P, double* qt,
                     uint64_t* W, uint64_t* C) {
    for (int32_t d = 1; d <= k; ++d) e[d - 1] = exp(-(double)(d * d) / (2.0 * sigma * sigma));
    int64_t* cnt = (int64_t*)calloc((size_t)(k > 0 ? k : 1), sizeof(int64_t));
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t d = 0; d < k; ++d) cnt[d] = 0;
        for (int64_t x = prp[i]; x < prp[i + 1]; ++x) cnt[phop[x] - 1] += 1;
        double z = 0.0;
        for (int32_t d = 0; d < k; ++d) {
            double term = (double)cnt[d] * e[d];
            z = z + term;
        }
        Z[i] = z;
        invZ[i] = (prp[i + 1] > prp[i]) ? 1.0 / z : 0.0;
    }
    free(cnt);
    C[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        double q = 0.0;
        uint64_t w = 0;
        for (int64_t x = prp[i]; x < prp[i + 1]; ++x) {
            int32_t j = pcol[x];
            double s = invZ[i] + invZ[j];
            double t = e[phop[x] - 1] * s;
            double p = t * 0.5;
            P[x] = p;
            q = q + p;
            w += (uint64_t)(p * 4294967296.0);
        }
        qt[i] = q;
        W[i] = w;
        C[i + 1] = C[i] + w;
    }
}

/* ------------------------------------------------------------------------ */
/* Node-wise sigma_i (Eq. NS gives each node its own Gaussian): sigma_i is    */
/* chosen so that the conditional distribution NS_{.|i} over NNG(i, k) has    */
/* a given perplexity exp(H_i), H_i its entropy in nats -- the calibration    */
/* of t-SNE (van der Maaten and Hinton, JMLR 2008), which the paper builds    */
/* on.  With t = exp(-1/(2 sigma_i^2)) in (0, 1] the Gaussian of hop d is    */
/* t^(d^2), so NS_{.|i} depends on t and the hop histogram c_d(i) only.     */
/* Every step uses IEEE operations only (frexp, +, -, *, / and comparisons) */
/* so that another program doing the same operations in the same order     */
/* obtains the same bits.                                                   */
/* ------------------------------------------------------------------------ */

/* Natural logarithm, x > 0 finite: x = m 2^e with m in [sqrt(1/2), sqrt(2)),  */
/* ln m = 2 atanh(s) with s = (m - 1)/(m + 1), |s| < 0.172, and              */
/* atanh(s) = s (1 + s^2/3 + s^4/5 + ...), summed by Horner's rule over the  */
/* first 13 terms (the rest is below 1e-20 of the sum); ln x = e ln2 + ln m. */
double drgo_ln(double x) {
    int e = 0;
    double m = frexp(x, &e); /* m in [1/2, 1) */
    if (m < 0.70710678118654752440) {
        m = m * 2.0;
        e = e - 1;
    }
    double s = (m - 1.0) / (m + 1.0);
    double s2 = s * s;
    double p = 1.0 / 25.0;
    for (int j = 11; j >= 0; --j) p = p * s2 + 1.0 / (double)(2 * j + 1);
    double lm = 2.0 * s * p;
    return (double)e * 0.69314718055994530942 + lm;
}

/* e[d-1] = t^(d^2), d = 1..k, as a running product of d^2 factors t */
static void hop_gauss_t(double t, int32_t k, double* e) {
    for (int32_t d = 1; d <= k; ++d) {
        double p = 1.0;
        for (int32_t r = 0; r < d * d; ++r) p = p * t;
        e[d - 1] = p;
    }
}

/* Z = sum_d c_d t^(d^2) and H = ln Z - ln(t) S / Z, S = sum_d c_d d^2 t^(d^2):  */
/* the entropy of p_j = t^(d_ij^2) / Z over the neighbourhood.                 */
static double entropy_t(const int64_t* cnt, int32_t k, double t, double* zout) {
    double e[8];
    hop_gauss_t(t, k, e);
    double z = 0.0, sw = 0.0;
    for (int32_t d = 0; d < k; ++d) {
        double c = (double)cnt[d];
        double term = c * e[d];
        z = z + term;
        double dd = (double)((d + 1) * (d + 1));
        sw = sw + term * dd;
    }
    if (zout) *zout = z;
    double lt = drgo_ln(t);
    return drgo_ln(z) - lt * (sw / z);
}

/* t of a node with a non-empty neighbourhood.  H grows with t (the entropy  */
/* of a Gibbs distribution falls as its inverse temperature -ln t grows);    */
/* its largest value, ln N at t = 1 (uniform), is taken when the target      */
/* reaches it; otherwise 64 halvings of (0, 1).                              */
static double calibrate_t(const int64_t* cnt, int32_t k, double target) {
    if (entropy_t(cnt, k, 1.0, NULL) <= target) return 1.0;
    double lo = 0.0, hi = 1.0;
    for (int r = 0; r < 64; ++r) {
        double mid = 0.5 * (lo + hi);
        if (entropy_t(cnt, k, mid, NULL) < target)
            lo = mid;
        else
            hi = mid;
    }
    return 0.5 * (lo + hi);
}

int32_t drgo_similarity_perplexity(int32_t n, int32_t k, double perplexity, const int64_t* prp,
                                   const int32_t* pcol, const uint8_t* phop, double* tnode,
                                   double* A, double* Z, double* invZ, double* P, double* qt,
                                   uint64_t* W, uint64_t* C) {
    if (k < 1 || k > 8 || !(perplexity >= 1.0) || !(perplexity < 1e300)) return -1;
    const double target = drgo_ln(perplexity);
    int64_t cnt[8];
    double e[8];
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t d = 0; d < k; ++d) cnt[d] = 0;
        for (int64_t x = prp[i]; x < prp[i + 1]; ++x) cnt[phop[x] - 1] += 1;
        if (prp[i + 1] == prp[i]) { /* isolated: no distribution */
            tnode[i] = 1.0;
            Z[i] = 0.0;
            invZ[i] = 0.0;
            for (int32_t d = 0; d < k; ++d) A[(int64_t)i * k + d] = 0.0;
            continue;
        }
        double t = calibrate_t(cnt, k, target);
        double z = 0.0;
        entropy_t(cnt, k, t, &z);
        hop_gauss_t(t, k, e);
        tnode[i] = t;
        Z[i] = z;
        invZ[i] = 1.0 / z;
        for (int32_t d = 0; d < k; ++d) A[(int64_t)i * k + d] = e[d] / z; /* NS_{j|i}, hop d+1 */
    }
    /* P~_ij = (NS_{j|i} + NS_{i|j}) / 2, scaled as in drgo_similarity */
    C[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        double q = 0.0;
        uint64_t w = 0;
        for (int64_t x = prp[i]; x < prp[i + 1]; ++x) {
            int32_t j = pcol[x];
            int32_t h = phop[x] - 1;
            double s = A[(int64_t)i * k + h] + A[(int64_t)j * k + h];
            double p = s * 0.5;
            P[x] = p;
            q = q + p;
            w += (uint64_t)(p * 4294967296.0);
        }
        qt[i] = q;
        W[i] = w;
        C[i + 1] = C[i] + w;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Weighted graphs (the paper names them as future work, Sec. 6).  Eq. NS is */
/* written with the graph distance GD; with positive symmetric edge lengths  */
/* GD_ij is taken as the length of the shortest i-j path of at most k edges */
/* for j in NNG(i, k) (the pattern stays the hop-defined one), made exactly  */
/* symmetric by taking the smaller of the two directions (the sums along a  */
/* path are rounded in path order); E_ij = exp(-GD_ij^2 / (2 sigma^2)),      */
/* Z_i = sum_l E_il, P~_ij = E_ij (1/Z_i + 1/Z_j) / 2.  With unit lengths    */
/* GD is the hop count and P~ the unweighted similarity.                     */
/* ------------------------------------------------------------------------ */

/* e^x for x <= 0 from IEEE operations only: Cody and Waite's reduction      */
/* n = floor(x / ln2 + 1/2), r = (x - n L1) - n L2 with ln 2 = L1 + L2 and   */
/* L1 holding 32 significant bits (n L1 exact), |r| <= 0.35; e^r by Taylor's */
/* series to r^13 (Horner's rule, coefficients 1/j! by successive division); */
/* e^x = 2^n e^r.  Below -708 (where 2^n e^r would leave the normal range)   */
/* the result is 0.                                                          */
double drgo_exp_neg(double x) {
    if (x < -708.0) return 0.0;
    double n = floor(x * 1.44269504088896340736 + 0.5);
    double r = (x - n * 6.93147180369123816490e-01) - n * 1.90821492927058770002e-10;
    double c[14];
    c[0] = 1.0;
    for (int j = 1; j < 14; ++j) c[j] = c[j - 1] / (double)j;
    double p = c[13];
    for (int j = 12; j >= 0; --j) p = p * r + c[j];
    return ldexp(p, (int)n);
}

static int64_t find_in_row(const int32_t* pcol, int64_t lo, int64_t hi, int32_t key) {
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (pcol[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

/* gd[x] of every pattern entry: Bellman-Ford from each source over k rounds, */
/* every round from the previous round's distances only (so round r allows   */
/* paths of at most r edges), then the smaller of gd_ij and gd_ji.           */
void drgo_hop_bounded_dist(int32_t n, const int32_t* rp, const int32_t* col, const double* len,
                           int32_t k, const int64_t* prp, const int32_t* pcol, double* gd) {
    double* prev = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* cur = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    char* inball = (char*)calloc((size_t)(n > 0 ? n : 1), 1);
    for (int32_t v = 0; v < n; ++v) prev[v] = cur[v] = INFINITY;
    for (int32_t i = 0; i < n; ++i) {
        for (int64_t x = prp[i]; x < prp[i + 1]; ++x) inball[pcol[x]] = 1;
        inball[i] = 1;
        prev[i] = 0.0;
        cur[i] = 0.0;
        for (int32_t r = 1; r <= k; ++r) {
            /* relax every edge out of a reached ball node, from prev into cur */
            for (int64_t x = prp[i] - 1; x < prp[i + 1]; ++x) {
                int32_t u = x < prp[i] ? i : pcol[x];
                if (prev[u] == INFINITY) continue;
                for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
                    int32_t v = col[e];
                    if (!inball[v] || v == i) continue;
                    double c = prev[u] + len[e];
                    if (c < cur[v]) cur[v] = c;
                }
            }
            for (int64_t x = prp[i]; x < prp[i + 1]; ++x) prev[pcol[x]] = cur[pcol[x]];
        }
        for (int64_t x = prp[i]; x < prp[i + 1]; ++x) {
            gd[x] = prev[pcol[x]];
            inball[pcol[x]] = 0;
            prev[pcol[x]] = cur[pcol[x]] = INFINITY;
        }
        inball[i] = 0;
        prev[i] = cur[i] = INFINITY;
    }
    for (int32_t i = 0; i < n; ++i) {
        for (int64_t x = prp[i]; x < prp[i + 1]; ++x) {
            int32_t j = pcol[x];
            if (j < i) continue;
            int64_t y = find_in_row(pcol, prp[j], prp[j + 1], i);
            double m = gd[x] < gd[y] ? gd[x] : gd[y];
            gd[x] = m;
            gd[y] = m;
        }
    }
    free(prev);
    free(cur);
    free(inball);
}

void drgo_similarity_weighted(int32_t n, double sigma, const int64_t* prp, const int32_t* pcol,
                              const double* gd, double* E, double* Z, double* invZ, double* P,
                              double* qt, uint64_t* W, uint64_t* C) {
    const double s2 = 2.0 * sigma * sigma;
    for (int32_t i = 0; i < n; ++i) {
        double z = 0.0;
        for (int64_t x = prp[i]; x < prp[i + 1]; ++x) {
            double a = gd[x] * gd[x];
            E[x] = drgo_exp_neg(-(a / s2));
            z = z + E[x];
        }
        Z[i] = z;
        invZ[i] = (prp[i + 1] > prp[i]) ? 1.0 / z : 0.0;
    }
    C[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        double q = 0.0;
        uint64_t w = 0;
        for (int64_t x = prp[i]; x < prp[i + 1]; ++x) {
            double s = invZ[i] + invZ[pcol[x]];
            double t = E[x] * s;
            double p = t * 0.5;
            P[x] = p;
            q = q + p;
            w += (uint64_t)(p * 4294967296.0);
        }
        qt[i] = q;
        W[i] = w;
        C[i + 1] = C[i] + w;
    }
}

/* ------------------------------------------------------------------------ */
/* The same similarity for a list of rows only, for graphs too large to take */
/* whole: row s is NNG(s, k) by the bounded BFS above, ascending; Z of every */
/* node involved is its own hop histogram weighted by e (each node's BFS run */
/* once); P~, qt and W of the listed rows follow the operations and order of */
/* drgo_similarity.  out_rp[r] .. out_rp[r+1] are the entries of srcs[r].    */
/* Returns the number of entries; with out_col == NULL only out_rp is set.   */
/* ------------------------------------------------------------------------ */
static double z_of(const int32_t* rp, const int32_t* col, int32_t k, const double* e, int32_t v,
                   int32_t* dist, int32_t* q, int64_t* cnt) {
    int32_t t = bfs_bounded(rp, col, k, v, dist, q);
    for (int32_t d = 0; d < k; ++d) cnt[d] = 0;
    for (int32_t x = 1; x < t; ++x) cnt[dist[q[x]] - 1] += 1;
    for (int32_t x = 0; x < t; ++x) dist[q[x]] = -1;
    double z = 0.0;
    for (int32_t d = 0; d < k; ++d) {
        double term = (double)cnt[d] * e[d];
        z = z + term;
    }
    return z;
}

int64_t drgo_similarity_rows(int32_t n, const int32_t* rp, const int32_t* col, int32_t k,
                             double sigma, int32_t nsrc, const int32_t* srcs, int64_t* out_rp,
                             int32_t* out_col, uint8_t* out_hop, double* out_P, double* out_invZ,
                             double* out_qt, uint64_t* out_W) {
    double e[8];
    if (k < 1 || k > 8) return -1;
    for (int32_t d = 1; d <= k; ++d) e[d - 1] = exp(-(double)(d * d) / (2.0 * sigma * sigma));
    int32_t* dist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* q = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t* cnt = (int64_t*)calloc((size_t)(k > 0 ? k : 1), sizeof(int64_t));
    for (int32_t v = 0; v < n; ++v) dist[v] = -1;
    out_rp[0] = 0;
    for (int32_t r = 0; r < nsrc; ++r) {
        int32_t t = bfs_bounded(rp, col, k, srcs[r], dist, q);
        out_rp[r + 1] = out_rp[r] + (t - 1);
        for (int32_t x = 0; x < t; ++x) dist[q[x]] = -1;
    }
    if (out_col) {
        double* Zc = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        for (int32_t v = 0; v < n; ++v) Zc[v] = -1.0;
        for (int32_t r = 0; r < nsrc; ++r) {
            int32_t s = srcs[r];
            int32_t t = bfs_bounded(rp, col, k, s, dist, q);
            int64_t o = out_rp[r];
            qsort(q + 1, (size_t)(t - 1), sizeof(int32_t), cmp_i32);
            for (int32_t x = 1; x < t; ++x) {
                out_col[o + x - 1] = q[x];
                out_hop[o + x - 1] = (uint8_t)dist[q[x]];
            }
            for (int32_t x = 0; x < t; ++x) dist[q[x]] = -1;
            if (Zc[s] < 0.0) Zc[s] = z_of(rp, col, k, e, s, dist, q, cnt);
            double izs = (out_rp[r + 1] > o) ? 1.0 / Zc[s] : 0.0;
            out_invZ[r] = izs;
            double qs = 0.0;
            uint64_t w = 0;
            for (int64_t x = o; x < out_rp[r + 1]; ++x) {
                int32_t j = out_col[x];
                if (Zc[j] < 0.0) Zc[j] = z_of(rp, col, k, e, j, dist, q, cnt);
                double sm = izs + 1.0 / Zc[j];
                double tt = e[out_hop[x] - 1] * sm;
                double p = tt * 0.5;
                out_P[x] = p;
                qs = qs + p;
                w += (uint64_t)(p * 4294967296.0);
            }
            out_qt[r] = qs;
            out_W[r] = w;
        }
        free(Zc);
    }
    free(cnt);
    free(dist);
    free(q);
    return out_rp[nsrc];
}

/* ------------------------------------------------------------------------ */
/* Negative sampling by node weight (Sec. 3.2.2): inverse of the integer   */
/* cumulative weight table.                                                  */
/* ------------------------------------------------------------------------ */
int32_t drgo_draw(const uint64_t* C, int32_t n, uint64_t w) {
    uint64_t hi, lo;
    mulhilo64(w, C[n], &hi, &lo);
    uint64_t r = hi; /* floor(w * S / 2^64) in [0, S) */
    int32_t a = 0, b = n - 1;
    while (a < b) { /* smallest v with C[v+1] > r */
        int32_t m = a + (b - a) / 2;
        if (C[m + 1] > r)
            b = m;
        else
            a = m + 1;
    }
    return a;
}

uint64_t drgo_neg_word(uint64_t seed, uint64_t it, int32_t i, int32_t m) {
    uint64_t out[4];
    philox_stream(seed, DRGO_TAG_NEG, (uint64_t)(uint32_t)i, it, (uint64_t)(m / 4), out);
    return out[m % 4];
}

/* ------------------------------------------------------------------------ */
/* Coarsening (Sec. 3.2.3, Fig. 3): pick a random unassigned node, group it */
/* with its unassigned first-order neighbours into one coarse node, repeat  */
/* until every node is assigned.  "Random" is a Philox priority per node,   */
/* visited in descending (priority, -id) order.                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t pri;
    int32_t id;
} prio_t;

static int cmp_prio_desc(const void* a, const void* b) {
    const prio_t* x = (const prio_t*)a;
    const prio_t* y = (const prio_t*)b;
    if (x->pri != y->pri) return (x->pri < y->pri) ? 1 : -1;
    return (x->id > y->id) - (x->id < y->id);
}

int32_t drgo_coarsen_level(int32_t n, const int32_t* rp, const int32_t* col, uint64_t seed,
                           int32_t level, int32_t* map) {
    prio_t* order = (prio_t*)malloc(sizeof(prio_t) * (size_t)(n > 0 ? n : 1));
    int32_t* owner = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t v = 0; v < n; ++v) {
        uint64_t out[4];
        philox_stream(seed, DRGO_TAG_COARSEN, (uint64_t)(uint32_t)v, (uint64_t)(uint32_t)level, 0,
                      out);
        order[v].pri = out[0];
        order[v].id = v;
        owner[v] = -1;
    }
    qsort(order, (size_t)n, sizeof(prio_t), cmp_prio_desc);
    for (int32_t x = 0; x < n; ++x) {
        int32_t v = order[x].id;
        if (owner[v] >= 0) continue;
        owner[v] = v;
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e)
            if (owner[col[e]] < 0) owner[col[e]] = v;
    }
    /* coarse ids: centres ranked by node id */
    int32_t* rank = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t nc = 0;
    for (int32_t v = 0; v < n; ++v) rank[v] = (owner[v] == v) ? nc++ : -1;
    for (int32_t v = 0; v < n; ++v) map[v] = rank[owner[v]];
    free(rank);
    free(owner);
    free(order);
    return nc;
}

static int cmp_i64(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

/* An edge of G^l survives into G^{l+1} between the two coarse nodes unless
 * both ends were grouped into the same coarse node (Sec. 3.2.3). */
int64_t drgo_contract(int32_t n, const int32_t* rp, const int32_t* col, const int32_t* map,
                      int32_t nc, int32_t* out_rp, int32_t* out_col) {
    int64_t m = rp[n];
    int64_t* key = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    int64_t t = 0;
    for (int32_t u = 0; u < n; ++u)
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
            int32_t a = map[u], b = map[col[e]];
            if (a != b) key[t++] = (int64_t)a * nc + b;
        }
    qsort(key, (size_t)t, sizeof(int64_t), cmp_i64);
    int64_t u = 0;
    for (int64_t x = 0; x < t; ++x)
        if (x == 0 || key[x] != key[x - 1]) key[u++] = key[x];
    for (int32_t a = 0; a <= nc; ++a) out_rp[a] = 0;
    for (int64_t x = 0; x < u; ++x) {
        out_rp[key[x] / nc + 1] += 1;
        out_col[x] = (int32_t)(key[x] % nc);
    }
    for (int32_t a = 0; a < nc; ++a) out_rp[a + 1] += out_rp[a];
    free(key);
    return u;
}

/* ------------------------------------------------------------------------ */
/* Layout of the coarsest graph: random initialisation (Sec. 3.2.3), each   */
/* coordinate uniform on [-1, 1) on a 2^-23 grid.  Positions are points of  */
/* R^dim, dim = 2 or 3 (Sec. 3.1); coordinate c of node v is word c of the   */
/* node's Philox block, so the 2-D layout is the first two coordinates of   */
/* the 3-D one.                                                              */
/* ------------------------------------------------------------------------ */
void drgo_init(int32_t nl, uint64_t seed, int32_t level, double* y, int32_t dim) {
    for (int32_t v = 0; v < nl; ++v) {
        uint64_t out[4];
        philox_stream(seed, DRGO_TAG_INIT, (uint64_t)(uint32_t)v, (uint64_t)(uint32_t)level, 0,
                      out);
        for (int32_t c = 0; c < dim; ++c) {
            double u = (double)(out[c] >> 40) * (1.0 / 16777216.0);
            y[(size_t)dim * v + c] = 2.0 * u - 1.0;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Forces (Eq. gradient).  With unnormalised proximity w = 1/(1 + d^{2b}),  */
/* d = ||y_i - y_j||:                                                        */
/*   d/dy_i log w       = -2b d^{2b-2} (y_i - y_j) / (1 + d^{2b})  (attract) */
/*   d/dy_i log(1 - w)  =  2b (y_i - y_j) / (d^2 (1 + d^{2b}))     (repel)   */
/* A pair at distance exactly zero contributes nothing.  Both act along the  */
/* offset, so they are the same in any dimension.                           */
/* ------------------------------------------------------------------------ */
static double ipow(double x, int32_t b) {
    double r = 1.0;
    for (int32_t t = 0; t < b; ++t) r = r * x;
    return r;
}

/* d^{2b} from d2 = d^2 for b a whole or half number (Sec. 4.2 tabulates b;
 * its supplement also uses 1.5 and 2.5): (d2)^floor(b), times sqrt(d2) when
 * b has a half.  For a whole b it is ipow(d2, b) exactly. */
static double powb(double d2, double b) {
    int32_t h = (int32_t)floor(b);
    double r = ipow(d2, h);
    if (b - (double)h == 0.5) r = r * sqrt(d2);
    return r;
}

static double clipd(double v, double c) { return v > c ? c : (v < -c ? -c : v); }

/* attraction coefficient: A = coef * delta */
static double attract_coef(double d2, double b) {
    double D = powb(d2, b);
    return -2.0 * b * powb(d2, b - 1.0) / (1.0 + D);
}

static double repel_coef(double d2, double b) {
    double D = powb(d2, b);
    return 2.0 * b / (d2 * (1.0 + D));
}

/* offset d = y_a - y_c (dim components) and its squared length, summed in
 * component order */
static double offset(const double* y, int32_t a, int32_t c, int32_t dim, double* d) {
    double d2 = 0.0;
    for (int32_t k = 0; k < dim; ++k) {
        d[k] = y[(size_t)dim * a + k] - y[(size_t)dim * c + k];
        d2 += d[k] * d[k];
    }
    return d2;
}

void drgo_step_direction(int32_t n0, const int64_t* prp, const int32_t* pcol, const double* P,
                         const double* qt, const uint64_t* C, const int32_t* cmap, const double* y,
                         int32_t M, double b, double gamma, double clip, uint64_t seed,
                         uint64_t it, double* g, int32_t dim) {
    for (int32_t i = 0; i < n0; ++i) {
        for (int32_t k = 0; k < dim; ++k) g[(size_t)dim * i + k] = 0.0;
        if (prp[i + 1] == prp[i]) continue; /* isolated: never anchors */
        int32_t a = cmap ? cmap[i] : i;
        double A[3] = {0.0, 0.0, 0.0}, R[3] = {0.0, 0.0, 0.0}, d[3];
        for (int64_t x = prp[i]; x < prp[i + 1]; ++x) {
            int32_t c = cmap ? cmap[pcol[x]] : pcol[x];
            double d2 = offset(y, a, c, dim, d);
            if (d2 == 0.0) continue;
            double k = attract_coef(d2, b);
            for (int32_t q = 0; q < dim; ++q) A[q] += P[x] * clipd(k * d[q], clip);
        }
        for (int32_t m = 0; m < M; ++m) {
            int32_t v = drgo_draw(C, n0, drgo_neg_word(seed, it, i, m));
            int32_t c = cmap ? cmap[v] : v;
            double d2 = offset(y, a, c, dim, d);
            if (d2 == 0.0) continue;
            double k = repel_coef(d2, b);
            for (int32_t q = 0; q < dim; ++q) R[q] += clipd(k * d[q], clip);
        }
        for (int32_t q = 0; q < dim; ++q) g[(size_t)dim * i + q] = A[q] + gamma * qt[i] * R[q];
    }
}

/* Anchor weight of every level node: w_a = sum_{cmap[i]=a} qt_i, the expected
 * number of times per iteration that one of its members is selected as the
 * node whose gradient is computed (qt_i = N_a * sum_j NS_ij, Sec. 3.2.2). */
static double* level_weights(int32_t n0, const double* qt, const int32_t* cmap, int32_t nl) {
    double* w = (double*)calloc((size_t)(nl > 0 ? nl : 1), sizeof(double));
    for (int32_t i = 0; i < n0; ++i) w[cmap ? cmap[i] : i] += qt[i];
    return w;
}

/* Synchronous (Jacobi) iteration.  In the paper's SGD (Sec. 3.2.2) a node is
 * selected about qt_i times per iteration and each selection applies its own
 * step; with gradient sharing (Sec. 3.2.3) the steps of all fine members are
 * applied to their level node.  Applied together from one snapshot, those
 * steps are replaced by one step along their average:
 *   y_a += eta * (sum_{cmap[i]=a} g_i) / (sum_{cmap[i]=a} qt_i). */
void drgo_iter_sync(int32_t n0, const int64_t* prp, const int32_t* pcol, const double* P,
                    const double* qt, const uint64_t* C, const int32_t* cmap, int32_t nl, double* y,
                    int32_t M, double b, double gamma, double eta, double clip, uint64_t seed,
                    uint64_t it, int32_t dim) {
    double* g = (double*)malloc(sizeof(double) * (size_t)dim * (size_t)(n0 > 0 ? n0 : 1));
    double* G = (double*)calloc((size_t)dim * (size_t)(nl > 0 ? nl : 1), sizeof(double));
    double* w = level_weights(n0, qt, cmap, nl);
    drgo_step_direction(n0, prp, pcol, P, qt, C, cmap, y, M, b, gamma, clip, seed, it, g, dim);
    for (int32_t i = 0; i < n0; ++i) {
        int32_t a = cmap ? cmap[i] : i;
        for (int32_t q = 0; q < dim; ++q) G[(size_t)dim * a + q] += g[(size_t)dim * i + q];
    }
    for (int32_t a = 0; a < nl; ++a) {
        if (w[a] <= 0.0) continue;
        for (int32_t q = 0; q < dim; ++q)
            y[(size_t)dim * a + q] += eta * (G[(size_t)dim * a + q] / w[a]);
    }
    free(w);
    free(g);
    free(G);
}

/* Sequential (Gauss-Seidel) iteration in ascending fine-node order: the
 * step of node i, computed from the current positions, is applied at once
 * with the same weighting as the synchronous iteration. */
void drgo_iter_seq(int32_t n0, const int64_t* prp, const int32_t* pcol, const double* P,
                   const double* qt, const uint64_t* C, const int32_t* cmap, int32_t nl, double* y,
                   int32_t M, double b, double gamma, double eta, double clip, uint64_t seed,
                   uint64_t it, int32_t dim) {
    double* w = level_weights(n0, qt, cmap, nl);
    for (int32_t i = 0; i < n0; ++i) {
        if (prp[i + 1] == prp[i]) continue;
        int32_t a = cmap ? cmap[i] : i;
        double A[3] = {0.0, 0.0, 0.0}, R[3] = {0.0, 0.0, 0.0}, d[3];
        for (int64_t x = prp[i]; x < prp[i + 1]; ++x) {
            int32_t c = cmap ? cmap[pcol[x]] : pcol[x];
            double d2 = offset(y, a, c, dim, d);
            if (d2 == 0.0) continue;
            double k = attract_coef(d2, b);
            for (int32_t q = 0; q < dim; ++q) A[q] += P[x] * clipd(k * d[q], clip);
        }
        for (int32_t m = 0; m < M; ++m) {
            int32_t v = drgo_draw(C, n0, drgo_neg_word(seed, it, i, m));
            int32_t c = cmap ? cmap[v] : v;
            double d2 = offset(y, a, c, dim, d);
            if (d2 == 0.0) continue;
            double k = repel_coef(d2, b);
            for (int32_t q = 0; q < dim; ++q) R[q] += clipd(k * d[q], clip);
        }
        for (int32_t q = 0; q < dim; ++q)
            y[(size_t)dim * a + q] += eta * ((A[q] + gamma * qt[i] * R[q]) / w[a]);
    }
    free(w);
}

/* ------------------------------------------------------------------------ */
/* Objective (Eq. objectfunction).  The expectation over positive pairs    */
/* (i, j) ~ NS is taken exactly (weights P~); the M negatives per anchor    */
/* are the drawn ones, each weighted gamma * qt_i.                          */
/*   L^ = sum_ij P~_ij log w_ij + gamma sum_i qt_i sum_m log(1 - w_{i v_im}) */
/* log w = -log1p(d^{2b}); log(1 - w) = b log d^2 - log1p(d^{2b}).           */
/* ------------------------------------------------------------------------ */
double drgo_objective(int32_t n, const int64_t* prp, const int32_t* pcol, const double* P,
                      const double* qt, const uint64_t* C, const double* y, int32_t M, double b,
                      double gamma, uint64_t seed, uint64_t it, int32_t dim) {
    double L = 0.0, d[3];
    for (int32_t i = 0; i < n; ++i) {
        if (prp[i + 1] == prp[i]) continue;
        double att = 0.0;
        for (int64_t x = prp[i]; x < prp[i + 1]; ++x) {
            double d2 = offset(y, i, pcol[x], dim, d);
            att += P[x] * (-log1p(powb(d2, b)));
        }
        double rep = 0.0;
        for (int32_t m = 0; m < M; ++m) {
            int32_t v = drgo_draw(C, n, drgo_neg_word(seed, it, i, m));
            double d2 = offset(y, i, v, dim, d);
            if (v == i || d2 == 0.0) continue;
            rep += b * log(d2) - log1p(powb(d2, b));
        }
        L += att + gamma * qt[i] * rep;
    }
    return L;
}

void drgo_objective_grad(int32_t n, const int64_t* prp, const int32_t* pcol, const double* P,
                         const double* qt, const uint64_t* C, const double* y, int32_t M, double b,
                         double gamma, uint64_t seed, uint64_t it, double* grad, int32_t dim) {
    double d[3];
    for (int64_t t = 0; t < (int64_t)dim * n; ++t) grad[t] = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        if (prp[i + 1] == prp[i]) continue;
        for (int64_t x = prp[i]; x < prp[i + 1]; ++x) {
            int32_t j = pcol[x];
            double d2 = offset(y, i, j, dim, d);
            if (d2 == 0.0) continue;
            double k = attract_coef(d2, b);
            /* the term P~_ij log w_ij depends on both y_i and y_j */
            for (int32_t q = 0; q < dim; ++q) {
                grad[(size_t)dim * i + q] += P[x] * k * d[q];
                grad[(size_t)dim * j + q] -= P[x] * k * d[q];
            }
        }
        for (int32_t m = 0; m < M; ++m) {
            int32_t v = drgo_draw(C, n, drgo_neg_word(seed, it, i, m));
            double d2 = offset(y, i, v, dim, d);
            if (v == i || d2 == 0.0) continue;
            double k = gamma * qt[i] * repel_coef(d2, b);
            for (int32_t q = 0; q < dim; ++q) {
                grad[(size_t)dim * i + q] += k * d[q];
                grad[(size_t)dim * v + q] -= k * d[q];
            }
        }
    }
}

/* probability that a draw returns v */
static double draw_prob(const uint64_t* C, int32_t n, int32_t v) {
    return (double)(C[v + 1] - C[v]) / (double)C[n];
}

double drgo_objective_exact(int32_t n, const int64_t* prp, const int32_t* pcol, const double* P,
                            const double* qt, const uint64_t* C, const double* y, int32_t M,
                            double b, double gamma, int32_t dim) {
    double L = 0.0, d[3];
    for (int32_t i = 0; i < n; ++i) {
        if (prp[i + 1] == prp[i]) continue;
        for (int64_t x = prp[i]; x < prp[i + 1]; ++x)
            L += P[x] * (-log1p(powb(offset(y, i, pcol[x], dim, d), b)));
        double rep = 0.0;
        for (int32_t v = 0; v < n; ++v) {
            double pv = draw_prob(C, n, v);
            double d2 = offset(y, i, v, dim, d);
            if (v == i || d2 == 0.0 || pv == 0.0) continue;
            rep += pv * (b * log(d2) - log1p(powb(d2, b)));
        }
        L += gamma * qt[i] * (double)M * rep;
    }
    return L;
}

void drgo_objective_exact_grad(int32_t n, const int64_t* prp, const int32_t* pcol, const double* P,
                               const double* qt, const uint64_t* C, const double* y, int32_t M,
                               double b, double gamma, double* grad, int32_t dim) {
    double d[3];
    for (int64_t t = 0; t < (int64_t)dim * n; ++t) grad[t] = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        if (prp[i + 1] == prp[i]) continue;
        for (int64_t x = prp[i]; x < prp[i + 1]; ++x) {
            int32_t j = pcol[x];
            double d2 = offset(y, i, j, dim, d);
            if (d2 == 0.0) continue;
            double k = P[x] * attract_coef(d2, b);
            for (int32_t q = 0; q < dim; ++q) {
                grad[(size_t)dim * i + q] += k * d[q];
                grad[(size_t)dim * j + q] -= k * d[q];
            }
        }
        for (int32_t v = 0; v < n; ++v) {
            double pv = draw_prob(C, n, v);
            double d2 = offset(y, i, v, dim, d);
            if (v == i || d2 == 0.0 || pv == 0.0) continue;
            double k = gamma * qt[i] * (double)M * pv * repel_coef(d2, b);
            for (int32_t q = 0; q < dim; ++q) {
                grad[(size_t)dim * i + q] += k * d[q];
                grad[(size_t)dim * v + q] -= k * d[q];
            }
        }
    }
}

void drgo_step_expected(int32_t n, const int64_t* prp, const int32_t* pcol, const double* P,
                        const double* qt, const uint64_t* C, const double* y, int32_t M, double b,
                        double gamma, double* g, int32_t dim) {
    double d[3];
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t q = 0; q < dim; ++q) g[(size_t)dim * i + q] = 0.0;
        if (prp[i + 1] == prp[i]) continue;
        double A[3] = {0.0, 0.0, 0.0}, R[3] = {0.0, 0.0, 0.0};
        for (int64_t x = prp[i]; x < prp[i + 1]; ++x) {
            double d2 = offset(y, i, pcol[x], dim, d);
            if (d2 == 0.0) continue;
            double k = attract_coef(d2, b);
            for (int32_t q = 0; q < dim; ++q) A[q] += P[x] * k * d[q];
        }
        for (int32_t v = 0; v < n; ++v) {
            double pv = draw_prob(C, n, v);
            double d2 = offset(y, i, v, dim, d);
            if (d2 == 0.0 || pv == 0.0) continue;
            double k = repel_coef(d2, b);
            for (int32_t q = 0; q < dim; ++q) R[q] += pv * k * d[q];
        }
        for (int32_t q = 0; q < dim; ++q)
            g[(size_t)dim * i + q] = A[q] + gamma * qt[i] * (double)M * R[q];
    }
}
