// drg_internal.hpp -- library-private state behind the opaque C handles.
#pragma once
#include <atomic>
#include <vector>

#include "../../include/drgraph.h"
#include "drg_common.hpp"
#include "drg_forces.hpp"
#include "drg_prims.hpp"

struct drg_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 0;
    int max_lds = 0;   // bytes of LDS one workgroup may use
    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    int64_t launches = 0;
    double total_ms = 0.0;
    int32_t last_sweep = -1;  // DRG_SWEEP_* form of the latest layout step
    drg::Allocator alloc;     // device memory of every object built on this context
};

// Sparse similarity P~ over the finest graph plus the sampling table.
namespace drg {
// a number no other object of the process gets (cache keys that must not
// match a later object allocated at a freed one's address)
inline uint64_t next_uid() {
    static std::atomic<uint64_t> counter{0};
    return ++counter;
}
}  // namespace drg

struct drg_sim {
    int device = 0;
    int32_t n = 0, k = 0, n_active = 0;
    int64_t nnz = 0;
    double len_wmean = 0.0;          // sum len^2 / sum len over the rows (sweep_group)
    double sigma = 1.0;              // 0 with node-wise sigma
    double perplexity = 0.0;         // > 0: node-wise sigma calibrated to it
    double e[4] = {0, 0, 0, 0};
    drg::DevBuf<int64_t> row_ptr;    // [n+1]
    drg::DevBuf<uint32_t> colhop;    // [nnz] col | (hop-1) << 30, ascending col per row
    drg::DevBuf<double> invZ;        // [n]
    drg::DevBuf<double> qt;          // [n]
    drg::DevBuf<uint64_t> W;         // [n]
    drg::DevBuf<uint64_t> C;         // [n+1]
    drg::DevBuf<int32_t> guide;      // [2^gbits + 1]
    int gbits = 1;
    uint64_t S = 0;                  // = C[n]
    drg::DevBuf<float> invZf;        // [n]
    drg::DevBuf<float> invZlo;       // [n] 1/Z - invZf (so hi + lo holds 1/Z to ~48 bits)
    drg::DevBuf<float> qtf;          // [n]
    // node-wise sigma only: A[i][d] = NS_{j|i} for j at hop d+1 (P~_ij =
    // (A_i[d] + A_j[d]) / 2), and t_i = exp(-1/(2 sigma_i^2))
    drg::DevBuf<double> A;           // [n][4]
    drg::DevBuf<double> tnode;       // [n]
    // weighted graph only: E_ij = exp(-GD_ij^2 / (2 sigma^2)) per entry, in
    // place of e_d (P~_ij = E_ij (1/Z_i + 1/Z_j) / 2)
    drg::DevBuf<double> Ex;          // [nnz]
    // per-iteration workspace of the layout step
    drg::DevBuf<float4> rec;         // [n] staged (y_c(j), invZ_j)
    drg::DevBuf<float2> g;           // [n] one-sided steps
    drg::DevBuf<float> wlev;         // [n] anchor weights of level nodes (async)
    uint64_t wlev_hier = 0;          // uid of the hierarchy whose level wlev holds (0: none)
    int32_t wlev_level = -1;
    drg::DevBuf<double4> rec64;      // FP64 instance workspace (allocated on use)
    drg::DevBuf<double2> g64;
    drg::DevBuf<float> g3;           // [n][3] steps of a 3-D layout (allocated on use)
    drg::DevBuf<double> g3_64;
    // column-blocked copy of the pattern for the LDS-staged sweep (blk_nb > 0)
    int32_t blk_nb = 0, blk_bits = 0, blk_nitems = 0;
    drg::DevBuf<int64_t> blk_base;   // [nb+1] first entry of each block
    drg::DevBuf<int32_t> blk_off;    // [nb][n+1] row offsets inside a block
    drg::DevBuf<uint16_t> blk_ent;   // [nnz] local col | (hop-1) << 13
    drg::DevBuf<int4> blk_items;     // (block, first row, end row)
    drg::DevBuf<float2> blk_partial; // [nb][n] partial attraction
    // asynchronous form on the blocked layout (built on first use): the work
    // items sorted by row stage, and the first item of each stage
    int32_t blk_stages = 0;
    drg::DevBuf<int4> blk_items_async;
    std::vector<int32_t> blk_stage_first;
    // work items of the windowed sweep (built on first use)
    drg::DevBuf<drg::WinItem> win_items;
    int32_t win_n = 0, win_rpl = 0;
};

struct drg_level {
    int32_t n = 0, n_active = 0;
    int64_t nnz = 0;
    drg::DevBuf<int32_t> rp, col;    // contracted graph G^l (level >= 1)
    drg::DevBuf<int32_t> map;        // [n_{l-1}] parent node -> node of this level
    drg::DevBuf<int32_t> cmap;       // [n_0] finest node -> node of this level
    drg::DevBuf<int32_t> perm;       // [n_0] finest nodes grouped by cmap, ascending within
    drg::DevBuf<int32_t> seg;        // [n+1] group offsets into perm
};

struct drg_hier {
    int device = 0;
    int32_t n0 = 0;
    uint64_t uid = drg::next_uid();  // distinct for every hierarchy of the process
    std::vector<drg_level> lv;       // lv[0] describes G^0 (sizes only)
};

namespace drg {
void set_error(const std::string& msg);

// A union of disjoint graphs: graph c owns the node ids base[c] .. base[c+1]-1
// and its edges stay inside that range.
struct UnionInfo {
    int32_t count = 0;
    std::vector<int32_t> base;            // [count+1], host
    const int32_t* node_base = nullptr;   // [n], device: base of the node's graph
    int32_t max_comp = 0;                 // largest graph
    std::vector<int64_t> nnz;             // out: pattern entries of each graph
};

// Lanes per row of the row-per-group sweep: about four entries per lane in
// the row a typical entry sits in.  wmean = sum len^2 / sum len, the mean row
// length seen from the entries, so a skewed graph (R-MAT hubs hold most
// entries) gets wide groups and an even one (an RGG, a grid) narrow ones,
// which share the per-row work (the butterflies, the negatives) among fewer
// lanes: on the 100k RGG (mean 65) 16 lanes sweep in 0.052 ms against 0.106
// ms for 64; on R-MAT 2^20 at k = 1 (mean 49) 64 lanes take 1.04 ms against
// 1.50 ms for 16.  A small graph keeps at least 2^14 lanes busy (the 32x32
// grid: 8.1 us per sweep with 16 lanes per row, 10.1 us with 4).
inline int sweep_group(double wmean, int64_t n_active) {
    int g = 4;
    while (g < 64 && 8.0 * g <= wmean) g *= 2;
    while (g < 64 && n_active > 0 && n_active * g < (int64_t)1 << 14) g *= 2;
    return g;
}

// similarity.hip
// With u, the pattern is built for every graph of the union at once, each
// graph's row weights with the launch shape of its own single-graph build;
// the sampling guide and the column-blocked copy are then left out.
// perplexity != 0: node-wise sigma_i calibrated to it (sigma unused).
// lengths (device, one per CSR entry): a weighted graph.
drg_sim* build_similarity(drg_ctx* ctx, const drg_csr* g, int k, double sigma, uint32_t flags,
                          UnionInfo* u = nullptr, double perplexity = 0.0,
                          const double* lengths = nullptr);
void sim_node_sigma(const drg_sim* s, double* sigma);
void validate_csr(drg_ctx* ctx, const drg_csr* g);
void validate_csr_impl(drg_ctx* ctx, const drg_csr* g, bool full);
void stress_sampled(drg_ctx* ctx, const drg_csr* g, const float* y, int32_t count,
                    const int32_t* sources, double* out, double* estimate);
void neighbourhood_preservation(drg_ctx* ctx, const drg_sim* s, const float* y, int32_t count,
                                const int32_t* nodes, double* out);
void sim_export_rows(const drg_sim* s, int32_t nrows, const int32_t* rows, int64_t cap,
                     int64_t* row_len, int32_t* col, uint8_t* hop, double* P, double* qt,
                     uint64_t* W, double* invZ);
void sim_export(const drg_sim* s, int64_t* row_ptr, int32_t* col, uint8_t* hop, double* P,
                double* qt, uint64_t* W, double* e, double* invZ);
// blocked.hip
// Column-blocked copy of a pattern (see blocked.hip).
struct BlkLayout {
    int32_t nb = 0, bits = 0, nitems = 0;
    int64_t chunk = 0;        // work per item the items were cut for
    DevBuf<int64_t> base;     // [nb+1] first entry of each block
    DevBuf<int32_t> off;      // [nb][n+1] row offsets inside a block
    DevBuf<uint16_t> ent;     // [nnz+8] block-local col | (hop-1) << 13
    DevBuf<int4> items;       // (block, first row, end row, -)
    DevBuf<float2> partial;   // [nb][n] partial attraction (zero where a row has no entry)
};
bool blocked_wanted(drg_ctx* ctx, const drg_sim* s);
bool blocked_wanted_for(drg_ctx* ctx, int32_t n, int64_t nnz);
void build_blocked(drg_ctx* ctx, drg_sim* s);
// rows prp[0..n] of a pattern whose columns are col_base .. col_base+n-1
void build_blocked_core(drg_ctx* ctx, int32_t n, int64_t nnz, const int64_t* prp,
                        const uint32_t* colhop, int32_t col_base, BlkLayout& L);
int blk_flat_cpl();  // chunks per lane and batch of the flat form (env DRG_BLK_FLAT: 2, 4; 0: row form)
int blk_lanes();
bool attract_clip_free(double b, double clip);
// b = whole in 1..3, or b + 1/2 (b_half = 1) for b in 1..2; else DRG_E_INVALID
inline void check_shape(int32_t b, int32_t b_half) {
    if (b < 1 || b > 3 || (b_half != 0 && b_half != 1) || (b_half && b > 2))
        throw Error(DRG_E_INVALID, "b must be 1, 1.5, 2, 2.5 or 3 (b in 1..3, b_half 0 or 1)");
}  // the attraction clip cannot bind     // row form: lanes per segment (env DRG_BLK_LANES; 0: per item)
// One FP32 sync sweep on the blocked layout: the one-sided steps into g.
void sweep_blocked(drg_ctx* ctx, drg_sim* s, int b, int M, float gamma, float clip,
                   uint64_t seed, uint64_t iter, float2* g, hipEvent_t e0, hipEvent_t e1);
// The objective's attraction terms per (block, row) into s->blk_partial from
// coordinates y: kind 0 = row values, 1 = attraction gradients.
// largest similarity (nodes) of the allocation-free objective forward
constexpr int64_t OBJ_NOALLOC_MAX_N = (int64_t)1 << 20;
void objective_fwd_noalloc(drg_ctx* ctx, drg_sim* s, const drg_obj_params* p, const float* y,
                           float* loss);
void sweep_blocked_async(drg_ctx* ctx, drg_sim* s, int b, int M, float gamma, float clip,
                         float eta, uint64_t seed, uint64_t iter, float* y, const int32_t* cmap,
                         const float* w, hipEvent_t e0, hipEvent_t e1);
void sweep_blocked_objective(drg_ctx* ctx, drg_sim* s, int b, const float* y, int kind);
// objective.hip
template <typename T>
void objective_fwd_t(drg_ctx* ctx, drg_sim* s, const drg_obj_params* p, const T* y, T* loss,
                     T* rows);
template <typename T>
void objective_bwd_t(drg_ctx* ctx, drg_sim* s, const drg_obj_params* p, const T* y,
                     const T* dloss, T* dy);
void sample_negatives(drg_ctx* ctx, drg_sim* s, int32_t M, uint64_t seed, uint64_t iter,
                      int32_t* out);
void sim_coo(drg_ctx* ctx, drg_sim* s, int32_t* rows, int32_t* cols, float* P);
// coarsen.hip
drg_hier* build_hierarchy(drg_ctx* ctx, const drg_csr* g, uint64_t seed, double rho,
                          int min_nodes, int max_levels);

// Hierarchies of all graphs of a union.  Level l >= 1 of graph c lives in
// pools shared by the graphs that have that level; its arrays hold the same
// (graph-local) values as the single-graph hierarchy:
//   map  at pool.map  + mo[c]  [n_{l-1}]   cmap at pool.cmap + co[c]  [n_0]
//   perm at pool.perm + co[c]  [n_0]       seg  at pool.seg  + so[c]  [n_l+1]
struct UnionHier {
    struct Pool {
        DevBuf<int32_t> map, cmap, perm, seg;
        std::vector<int64_t> mo, co, so;  // [count], -1: graph has no such level
    };
    std::vector<Pool> lv;                 // lv[0] unused
    std::vector<std::vector<int32_t>> n;  // [c][l] nodes per level
};
void build_hierarchy_union(drg_ctx* ctx, const drg_csr* g, const int32_t* gid,
                           const std::vector<int32_t>& base, const drg_layout_params* params,
                           UnionHier& out);
// layout.hip
void init_layout(drg_ctx* ctx, int32_t n, uint64_t seed, int32_t level, float* y);
void prolong(drg_ctx* ctx, const drg_hier* h, int32_t level, const float* yl, float* yf);
void layout_step(drg_ctx* ctx, drg_sim* s, const drg_hier* h, const drg_step_params* p,
                 float* y, bool staged = false, bool restage = false);
void prepare_sync_step(drg_ctx* ctx, drg_sim* s);
// layouts in R^3 (coordinates [n][3]; row-form sweep)
template <typename T>
void init_layout3_t(drg_ctx* ctx, int32_t n, uint64_t seed, int32_t level, T* y);
template <typename T>
void prolong3_t(drg_ctx* ctx, const drg_hier* h, int32_t level, const T* yl, T* yf);
template <typename T>
void layout_step3_t(drg_ctx* ctx, drg_sim* s, const drg_hier* h, const drg_step_params* p, T* y);
template <typename T>
void init_layout_t(drg_ctx* ctx, int32_t n, uint64_t seed, int32_t level, T* y);
template <typename T>
void prolong_t(drg_ctx* ctx, const drg_hier* h, int32_t level, const T* yl, T* yf);
template <typename T>
void layout_step_t(drg_ctx* ctx, drg_sim* s, const drg_hier* h, const drg_step_params* p, T* y,
                   bool staged = false, bool restage = false);
// window.hip
// Items of rows_per_item[c] consecutive rows of graph c (rows base[c] ..
// base[c+1]-1 of s) with the column window of their entries; returns the
// number of items.
int32_t build_window_items(drg_ctx* ctx, const drg_sim* s, const std::vector<int32_t>& base,
                           const std::vector<int32_t>& rows_per_item, DevBuf<WinItem>& out);
// Windowed sweep shape: lanes per workgroup and LDS records per chunk.
constexpr int WIN_BLOCK = 1024;
int win_rpl();        // rows per group (env DRG_WIN_RPL: 1, 2, 4, 8; default 4)
int win_chunk(drg_ctx* ctx);  // records per chunk (env DRG_WIN_CH; default fills 128 KB)
bool window_wanted(const drg_sim* s);  // env DRG_SWEEP_WINDOW=1 (default 0)

// batch.hip
void check_layout_params(const drg_layout_params* p);
drg_batch* batch_create(drg_ctx* ctx, const drg_csr* graphs, int32_t count,
                        const drg_layout_params* params);
void batch_run(drg_ctx* ctx, drg_batch* b, float* y_out);
void batch_destroy(drg_batch* b);
void batch_tuning(const drg_batch* b, int32_t cap, int32_t* n, int32_t* chosen, int32_t* rpl,
                  int32_t* ch, float* ms);
void batch_info(const drg_batch* b, int64_t* n_total, int64_t* nnz_total, int32_t* T,
                int32_t* nodes, int32_t* levels);
}  // namespace drg
