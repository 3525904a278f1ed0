// capi.hip -- the extern "C" boundary of libdrgraph.  Every entry point
// catches library errors and returns a status code; see include/drgraph.h.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>

#include "drg_internal.hpp"

namespace drg {
static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace drg

using drg::Error;

template <typename F>
static drg_status guarded(F&& f) {
    try {
        drg::g_last_error.clear();
        f();
        return DRG_OK;
    } catch (const Error& e) {
        drg::set_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        drg::set_error("host allocation failed");
        return DRG_E_OOM;
    } catch (const std::exception& e) {
        drg::set_error(e.what());
        return DRG_E_DEVICE;
    } catch (...) {
        drg::set_error("unknown error");
        return DRG_E_DEVICE;
    }
}

static void use_device(int dev) { DRG_HIP(hipSetDevice(dev)); }

// For the duration of a call on a context: its device is current and the
// device memory of whatever the call builds comes from its allocator.
struct CtxScope {
    drg::Allocator saved;
    explicit CtxScope(const drg_ctx* c) {
        use_device(c->device);
        saved = drg::thread_allocator();
        drg::thread_allocator() = c->alloc;
    }
    ~CtxScope() { drg::thread_allocator() = saved; }
    CtxScope(const CtxScope&) = delete;
    CtxScope& operator=(const CtxScope&) = delete;
};

static void need(const void* p, const char* what) {
    if (!p) throw Error(DRG_E_INVALID, std::string(what) + " is NULL");
}

extern "C" {

const char* drg_last_error(void) { return drg::g_last_error.c_str(); }

const char* drg_version(void) { return "drgraph-mi355x 0.1 (gfx950)"; }

drg_status drg_layout_params_default(drg_layout_params* p) {
    return guarded([&] {
        need(p, "params");
        std::memset(p, 0, sizeof(*p));
        p->k = 1;
        p->M = 5;
        p->b = 2;
        p->T = 400;
        p->sigma = 1.0;
        p->gamma = 0.1f;
        p->gamma_coarsest = 0.01f;
        p->eta0 = 1.0f;
        p->clip = 4.0f;
        p->rho = 0.8;
        p->min_nodes = 1000;
        p->max_levels = 64;
        p->mode = DRG_MODE_SYNC;
        p->seed = 0;
    });
}

drg_status drg_ctx_create(int32_t device, void* hip_stream, const drg_allocator* alloc,
                          drg_ctx** out) {
    return guarded([&] {
        need(out, "out");
        *out = nullptr;
        if (alloc && (!alloc->alloc || !alloc->free))
            throw Error(DRG_E_INVALID, "allocator needs both alloc and free");
        int count = 0;
        DRG_HIP(hipGetDeviceCount(&count));
        if (device < 0 || device >= count) throw Error(DRG_E_INVALID, "no such device");
        use_device(device);
        auto c = std::make_unique<drg_ctx>();
        c->device = device;
        c->stream = static_cast<hipStream_t>(hip_stream);
        DRG_HIP(hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, device));
        int lds = 0, lds_optin = 0;
        DRG_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
        if (hipDeviceGetAttribute(&lds_optin, hipDeviceAttributeSharedMemPerBlockOptin, device) !=
            hipSuccess) {
            (void)hipGetLastError();
            lds_optin = 0;
        }
        c->max_lds = std::max(lds, lds_optin);
        if (alloc) {
            c->alloc.alloc = alloc->alloc;
            c->alloc.free = alloc->free;
            c->alloc.user = alloc->user;
        }
        *out = c.release();
    });
}

void drg_ctx_destroy(drg_ctx* ctx) {
    if (!ctx) return;
    for (auto& e : ctx->events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    delete ctx;
}

drg_status drg_ctx_synchronize(drg_ctx* ctx) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        DRG_HIP(hipStreamSynchronize(ctx->stream));
    });
}

drg_status drg_ctx_set_profiling(drg_ctx* ctx, int32_t on) {
    return guarded([&] {
        need(ctx, "ctx");
        ctx->profiling = on != 0;
        for (auto& e : ctx->events) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        ctx->events.clear();
        ctx->launches = 0;
        ctx->total_ms = 0.0;
    });
}

drg_status drg_ctx_kernel_stats(drg_ctx* ctx, int64_t* launches, double* total_ms) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        DRG_HIP(hipStreamSynchronize(ctx->stream));
        for (auto& e : ctx->events) {
            float ms = 0.0f;
            DRG_HIP(hipEventElapsedTime(&ms, e.first, e.second));
            ctx->total_ms += ms;
            ctx->launches += 1;
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        ctx->events.clear();
        if (launches) *launches = ctx->launches;
        if (total_ms) *total_ms = ctx->total_ms;
    });
}

drg_status drg_ctx_last_sweep(const drg_ctx* ctx, int32_t* form) {
    return guarded([&] {
        need(ctx, "ctx");
        need(form, "form");
        *form = ctx->last_sweep;
    });
}

drg_status drg_build_similarity(drg_ctx* ctx, const drg_csr* g, int32_t k, double sigma,
                                uint32_t flags, drg_sim** out) {
    return guarded([&] {
        need(ctx, "ctx");
        need(out, "out");
        *out = nullptr;
        CtxScope scope(ctx);
        *out = drg::build_similarity(ctx, g, k, sigma, flags);
    });
}

drg_status drg_build_similarity_perplexity(drg_ctx* ctx, const drg_csr* g, int32_t k,
                                           double perplexity, uint32_t flags, drg_sim** out) {
    return guarded([&] {
        need(ctx, "ctx");
        need(out, "out");
        *out = nullptr;
        if (!(perplexity >= 1.0) || !(perplexity < 1e300))
            throw drg::Error(DRG_E_INVALID, "perplexity must be >= 1 and finite");
        CtxScope scope(ctx);
        *out = drg::build_similarity(ctx, g, k, 1.0, flags, nullptr, perplexity);
    });
}

drg_status drg_build_similarity_weighted(drg_ctx* ctx, const drg_csr* g,
                                         const double* length_dev, int32_t k, double sigma,
                                         uint32_t flags, drg_sim** out) {
    return guarded([&] {
        need(ctx, "ctx");
        need(out, "out");
        need(g, "graph");
        *out = nullptr;
        if (g->nnz > 0) need(length_dev, "length_dev");
        CtxScope scope(ctx);
        *out = drg::build_similarity(ctx, g, k, sigma, flags, nullptr, 0.0,
                                     g->nnz > 0 ? length_dev : nullptr);
    });
}

drg_status drg_sim_node_sigma(const drg_sim* s, double* sigma_host) {
    return guarded([&] {
        need(s, "sim");
        drg::sim_node_sigma(s, sigma_host);
    });
}

drg_status drg_sim_info(const drg_sim* s, int32_t* n, int64_t* nnz, int32_t* n_active,
                        int32_t* k, int32_t* blocked) {
    return guarded([&] {
        need(s, "sim");
        if (blocked) *blocked = s->blk_nb > 0 ? 1 : 0;
        if (n) *n = s->n;
        if (nnz) *nnz = s->nnz;
        if (n_active) *n_active = s->n_active;
        if (k) *k = s->k;
    });
}

drg_status drg_sim_export(const drg_sim* s, int64_t* row_ptr, int32_t* col, uint8_t* hop,
                          double* P, double* qt, uint64_t* W, double* e, double* invZ) {
    return guarded([&] {
        need(s, "sim");
        drg::sim_export(s, row_ptr, col, hop, P, qt, W, e, invZ);
    });
}

drg_status drg_sim_export_rows(const drg_sim* s, int32_t nrows, const int32_t* rows,
                               int64_t cap, int64_t* row_len, int32_t* col, uint8_t* hop,
                               double* P, double* qt, uint64_t* W, double* invZ) {
    return guarded([&] {
        need(s, "sim");
        drg::sim_export_rows(s, nrows, rows, cap, row_len, col, hop, P, qt, W, invZ);
    });
}

drg_status drg_neighbourhood_preservation(drg_ctx* ctx, const drg_sim* s, const float* y,
                                          int32_t count, const int32_t* nodes, double* np_out) {
    return guarded([&] {
        need(ctx, "ctx");
        need(s, "sim");
        CtxScope scope(ctx);
        drg::neighbourhood_preservation(ctx, s, y, count, nodes, np_out);
    });
}

drg_status drg_stress_sampled(drg_ctx* ctx, const drg_csr* g, const float* y, int32_t count,
                              const int32_t* sources, double* sums_out, double* estimate) {
    return guarded([&] {
        need(ctx, "ctx");
        need(g, "graph");
        CtxScope scope(ctx);
        drg::stress_sampled(ctx, g, y, count, sources, sums_out, estimate);
    });
}

void drg_sim_destroy(drg_sim* s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    (void)hipDeviceSynchronize();
    delete s;
}

drg_status drg_coarsen(drg_ctx* ctx, const drg_csr* g, uint64_t seed, double rho,
                       int32_t min_nodes, int32_t max_levels, drg_hier** out) {
    return guarded([&] {
        need(ctx, "ctx");
        need(out, "out");
        *out = nullptr;
        CtxScope scope(ctx);
        *out = drg::build_hierarchy(ctx, g, seed, rho, min_nodes, max_levels);
    });
}

drg_status drg_hier_info(const drg_hier* h, int32_t* levels, int32_t* sizes_host) {
    return guarded([&] {
        need(h, "hier");
        if (levels) *levels = (int32_t)h->lv.size();
        if (sizes_host)
            for (size_t l = 0; l < h->lv.size(); ++l) sizes_host[l] = h->lv[l].n;
    });
}

drg_status drg_hier_export_map(const drg_hier* h, int32_t level, int32_t* fine_to_level) {
    return drg_hier_export(h, level, nullptr, fine_to_level, nullptr, nullptr, nullptr);
}

drg_status drg_hier_export(const drg_hier* h, int32_t level, int32_t* map, int32_t* cmap,
                           int32_t* coarse_rp, int32_t* coarse_col, int64_t* coarse_nnz) {
    return guarded([&] {
        need(h, "hier");
        if (level < 1 || level >= (int32_t)h->lv.size())
            throw Error(DRG_E_INVALID, "level out of range");
        use_device(h->device);
        DRG_HIP(hipDeviceSynchronize());
        const drg_level& L = h->lv[level];
        const int32_t nf = h->lv[level - 1].n;
        if (map) DRG_HIP(hipMemcpy(map, L.map.get(), sizeof(int32_t) * nf, hipMemcpyDeviceToHost));
        if (cmap)
            DRG_HIP(hipMemcpy(cmap, L.cmap.get(), sizeof(int32_t) * h->n0, hipMemcpyDeviceToHost));
        if (coarse_rp)
            DRG_HIP(hipMemcpy(coarse_rp, L.rp.get(), sizeof(int32_t) * (L.n + 1),
                              hipMemcpyDeviceToHost));
        if (coarse_col && L.nnz > 0)
            DRG_HIP(hipMemcpy(coarse_col, L.col.get(), sizeof(int32_t) * L.nnz,
                              hipMemcpyDeviceToHost));
        if (coarse_nnz) *coarse_nnz = L.nnz;
    });
}

void drg_hier_destroy(drg_hier* h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    delete h;
}

drg_status drg_init_layout(drg_ctx* ctx, int32_t n, uint64_t seed, int32_t level, float* y_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        drg::init_layout(ctx, n, seed, level, y_dev);
    });
}

drg_status drg_prolong(drg_ctx* ctx, const drg_hier* h, int32_t level, const float* y_level_dev,
                       float* y_finer_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        drg::prolong(ctx, h, level, y_level_dev, y_finer_dev);
    });
}

// the coordinate dimension of a parameter block: 2 (0 means 2) or 3
static int32_t dim_of(int32_t d) {
    if (d == 0 || d == 2) return 2;
    if (d == 3) return 3;
    throw Error(DRG_E_INVALID, "dim must be 2 (or 0) or 3");
}

drg_status drg_layout_step(drg_ctx* ctx, const drg_sim* s, const drg_hier* h,
                           const drg_step_params* p, float* y_level_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        need(p, "params");
        CtxScope scope(ctx);
        if (dim_of(p->dim) == 3)
            drg::layout_step3_t<float>(ctx, const_cast<drg_sim*>(s), h, p, y_level_dev);
        else
            drg::layout_step(ctx, const_cast<drg_sim*>(s), h, p, y_level_dev);
    });
}

drg_status drg_init_layout_3d(drg_ctx* ctx, int32_t n, uint64_t seed, int32_t level,
                              float* y_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        drg::init_layout3_t<float>(ctx, n, seed, level, y_dev);
    });
}

drg_status drg_prolong_3d(drg_ctx* ctx, const drg_hier* h, int32_t level,
                          const float* y_level_dev, float* y_finer_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        drg::prolong3_t<float>(ctx, h, level, y_level_dev, y_finer_dev);
    });
}

drg_status drg_init_layout_3d_f64(drg_ctx* ctx, int32_t n, uint64_t seed, int32_t level,
                                  double* y_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        drg::init_layout3_t<double>(ctx, n, seed, level, y_dev);
    });
}

drg_status drg_prolong_3d_f64(drg_ctx* ctx, const drg_hier* h, int32_t level,
                              const double* y_level_dev, double* y_finer_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        drg::prolong3_t<double>(ctx, h, level, y_level_dev, y_finer_dev);
    });
}

drg_status drg_init_layout_f64(drg_ctx* ctx, int32_t n, uint64_t seed, int32_t level,
                               double* y_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        drg::init_layout_t<double>(ctx, n, seed, level, y_dev);
    });
}

drg_status drg_prolong_f64(drg_ctx* ctx, const drg_hier* h, int32_t level,
                           const double* y_level_dev, double* y_finer_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        drg::prolong_t<double>(ctx, h, level, y_level_dev, y_finer_dev);
    });
}

drg_status drg_layout_step_f64(drg_ctx* ctx, const drg_sim* s, const drg_hier* h,
                               const drg_step_params* p, double* y_level_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        need(p, "params");
        CtxScope scope(ctx);
        if (dim_of(p->dim) == 3)
            drg::layout_step3_t<double>(ctx, const_cast<drg_sim*>(s), h, p, y_level_dev);
        else
            drg::layout_step_t<double>(ctx, const_cast<drg_sim*>(s), h, p, y_level_dev);
    });
}

drg_status drg_objective_fwd(drg_ctx* ctx, const drg_sim* s, const drg_obj_params* p,
                             const float* y_dev, float* loss_dev, float* rows_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        drg::objective_fwd_t<float>(ctx, const_cast<drg_sim*>(s), p, y_dev, loss_dev, rows_dev);
    });
}

drg_status drg_objective_fwd_noalloc(drg_ctx* ctx, const drg_sim* s, const drg_obj_params* p,
                                     const float* y_dev, float* loss_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        drg::objective_fwd_noalloc(ctx, const_cast<drg_sim*>(s), p, y_dev, loss_dev);
    });
}

drg_status drg_objective_bwd(drg_ctx* ctx, const drg_sim* s, const drg_obj_params* p,
                             const float* y_dev, const float* dloss_dev, float* dy_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        drg::objective_bwd_t<float>(ctx, const_cast<drg_sim*>(s), p, y_dev, dloss_dev, dy_dev);
    });
}

drg_status drg_objective_fwd_f64(drg_ctx* ctx, const drg_sim* s, const drg_obj_params* p,
                                 const double* y_dev, double* loss_dev, double* rows_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        drg::objective_fwd_t<double>(ctx, const_cast<drg_sim*>(s), p, y_dev, loss_dev, rows_dev);
    });
}

drg_status drg_objective_bwd_f64(drg_ctx* ctx, const drg_sim* s, const drg_obj_params* p,
                                 const double* y_dev, const double* dloss_dev, double* dy_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        drg::objective_bwd_t<double>(ctx, const_cast<drg_sim*>(s), p, y_dev, dloss_dev, dy_dev);
    });
}

drg_status drg_sample_negatives(drg_ctx* ctx, const drg_sim* s, int32_t M, uint64_t seed,
                                uint64_t iter, int32_t* out_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        drg::sample_negatives(ctx, const_cast<drg_sim*>(s), M, seed, iter, out_dev);
    });
}

drg_status drg_sim_coo(drg_ctx* ctx, const drg_sim* s, int32_t* rows_dev, int32_t* cols_dev,
                       float* P_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        drg::sim_coo(ctx, const_cast<drg_sim*>(s), rows_dev, cols_dev, P_dev);
    });
}

using drg::check_layout_params;

// A point of the schedule: `t` iterations of level `level` done (levels run
// from the coarsest down to 0).
struct SchedPoint {
    int32_t level, t;
};

static int32_t level_iters(const drg_layout_params* p, int32_t Lc, int32_t l) {
    const int32_t base = p->T / Lc;
    return base + (l == 0 ? p->T - base * Lc : 0);
}

static void check_point(const drg_layout_params* p, int32_t Lc, const SchedPoint& q) {
    if (q.level < 0 || q.level >= Lc || q.t < 0 || q.t > level_iters(p, Lc, q.level))
        throw Error(DRG_E_INVALID, "schedule point: level in [0, levels), t in [0, T_level]");
}

// Whether a synchronous run is recorded into a graph and launched once
// (DRG_RUN_GRAPH=1; not while kernel timing is on).  Off by default: for a
// run made once, recording and instantiating its launches costs more than
// the launch overhead it saves (32x32 grid, 300 iterations: 5.9 ms recorded
// vs 5.1 ms launched one by one).
static bool run_as_graph(const drg_ctx* ctx, const drg_sim* s, const drg_layout_params* p) {
    (void)s;
    if (p->mode != DRG_MODE_SYNC || ctx->profiling) return false;
    const char* v = std::getenv("DRG_RUN_GRAPH");
    return v && *v == '1';
}

// The schedule of Sec. 3.2.3 / Sec. 4.2 on a built similarity and hierarchy:
// from `from` (coordinates y_from of that level; NULL: the random layout of
// the coarsest level at its first iteration) to `to` (the level's
// coordinates copied to y_to; NULL: to the end, the finest coordinates in
// y_out).  Iteration t of level l has step eta0 (1 - t/T_l) and global index
// (iterations of the coarser levels) + t, which keys its negatives; a split
// run therefore equals the whole one.
static void run_schedule(drg_ctx* ctx, drg_sim* s, const drg_hier* h, const drg_layout_params* p,
                         const SchedPoint* from, const float* y_from, const SchedPoint* to,
                         float* y_to, float* y_out) {
    check_layout_params(p);
    need(s, "sim");
    need(h, "hier");
    if (h->n0 != s->n) throw Error(DRG_E_INVALID, "hierarchy is of another graph");
    const int32_t Lc = (int32_t)h->lv.size();
    const SchedPoint start = from ? *from : SchedPoint{Lc - 1, 0};
    const SchedPoint stop = to ? *to : SchedPoint{0, level_iters(p, Lc, 0)};
    check_point(p, Lc, start);
    check_point(p, Lc, stop);
    if (start.level < stop.level || (start.level == stop.level && start.t > stop.t))
        throw Error(DRG_E_INVALID, "schedule point: the stop lies before the start");
    if (from) need(y_from, "y_from");
    if (to) need(y_to, "y_to");
    else need(y_out, "y_out");
    const int32_t D = dim_of(p->dim);
    // level buffers: the finest level of a run to the end is y_out, the others scratch
    std::vector<drg::DevBuf<float>> ybuf(Lc);
    auto ylev = [&](int32_t l) -> float* { return (l == 0 && !to) ? y_out : ybuf[l].get(); };
    for (int32_t l = stop.level; l <= start.level; ++l)
        if (!(l == 0 && !to)) ybuf[l].alloc((int64_t)D * h->lv[l].n);
    uint64_t git0 = 0;
    for (int32_t l = Lc - 1; l > start.level; --l) git0 += (uint64_t)level_iters(p, Lc, l);
    git0 += (uint64_t)start.t;
    // every launch of the run, in order; a level-0 sync step leaves the
    // records of the next one written, so only the first step of a level
    // (after the initial layout, a refinement or a resume) stages them
    const bool sync = p->mode == DRG_MODE_SYNC;
    auto issue = [&] {
        if (!from) {
            if (D == 3)
                drg::init_layout3_t<float>(ctx, h->lv[Lc - 1].n, p->seed, Lc - 1, ylev(Lc - 1));
            else
                drg::init_layout(ctx, h->lv[Lc - 1].n, p->seed, Lc - 1, ylev(Lc - 1));
        }
        uint64_t git = git0;
        for (int32_t l = start.level; l >= stop.level; --l) {
            const int32_t Tl = level_iters(p, Lc, l);
            const float gam = (l == Lc - 1 && Lc > 1) ? p->gamma_coarsest : p->gamma;
            drg_step_params sp{};
            sp.M = p->M;
            sp.b = p->b;
            sp.gamma = gam;
            sp.clip = p->clip;
            sp.level = l;
            sp.mode = p->mode;
            sp.dim = D;
            sp.b_half = p->b_half;
            sp.seed = p->seed;
            const int32_t t0 = l == start.level ? start.t : 0;
            const int32_t t1 = l == stop.level ? stop.t : Tl;
            for (int32_t t = t0; t < t1; ++t) {
                sp.eta = (float)((double)p->eta0 * (1.0 - (double)t / (double)Tl));
                sp.iter = git++;
                if (D == 3)
                    drg::layout_step3_t<float>(ctx, s, h, &sp, ylev(l));
                else
                    drg::layout_step(ctx, s, h, &sp, ylev(l), sync && t > t0, sync);
            }
            if (l == stop.level) break;
            if (D == 3)
                drg::prolong3_t<float>(ctx, h, l, ylev(l), ylev(l - 1));
            else
                drg::prolong(ctx, h, l, ylev(l), ylev(l - 1));
        }
    };
    if (from)
        DRG_HIP(hipMemcpyAsync(ylev(start.level), y_from,
                               sizeof(float) * D * h->lv[start.level].n, hipMemcpyDeviceToDevice,
                               ctx->stream));
    if (run_as_graph(ctx, s, p)) {
        // the launches of the whole run recorded into a graph, launched once
        drg::prepare_sync_step(ctx, s);
        hipStream_t cap = nullptr;
        DRG_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        struct Guard {
            hipStream_t& c;
            hipGraph_t& g;
            hipGraphExec_t& e;
            ~Guard() {
                if (e) (void)hipGraphExecDestroy(e);
                if (g) (void)hipGraphDestroy(g);
                if (c) (void)hipStreamDestroy(c);
            }
        } guard{cap, graph, exec};
        const hipStream_t user = ctx->stream;
        DRG_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        ctx->stream = cap;
        try {
            issue();
        } catch (...) {
            ctx->stream = user;
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(cap, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        ctx->stream = user;
        DRG_HIP(hipStreamEndCapture(cap, &graph));
        DRG_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        DRG_HIP(hipGraphLaunch(exec, user));
        DRG_HIP(hipStreamSynchronize(user));
    } else {
        issue();
    }
    if (to)
        DRG_HIP(hipMemcpyAsync(y_to, ylev(stop.level), sizeof(float) * D * h->lv[stop.level].n,
                               hipMemcpyDeviceToDevice, ctx->stream));
    DRG_HIP(hipStreamSynchronize(ctx->stream));
}

drg_status drg_layout_run(drg_ctx* ctx, const drg_sim* s, const drg_hier* h,
                          const drg_layout_params* p, float* y_out_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        run_schedule(ctx, const_cast<drg_sim*>(s), h, p, nullptr, nullptr, nullptr, nullptr,
                     y_out_dev);
    });
}

drg_status drg_layout_run_until(drg_ctx* ctx, const drg_sim* s, const drg_hier* h,
                                const drg_layout_params* p, int32_t level, int32_t t,
                                float* y_level_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        const SchedPoint to{level, t};
        run_schedule(ctx, const_cast<drg_sim*>(s), h, p, nullptr, nullptr, &to, y_level_dev,
                     nullptr);
    });
}

drg_status drg_layout_resume(drg_ctx* ctx, const drg_sim* s, const drg_hier* h,
                             const drg_layout_params* p, int32_t level, int32_t t,
                             const float* y_level_dev, float* y_out_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        const SchedPoint from{level, t};
        run_schedule(ctx, const_cast<drg_sim*>(s), h, p, &from, y_level_dev, nullptr, nullptr,
                     y_out_dev);
    });
}

drg_status drg_layout(drg_ctx* ctx, const drg_csr* g, const drg_layout_params* p,
                      float* y_out_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        need(g, "graph");
        check_layout_params(p);
        CtxScope scope(ctx);
        std::unique_ptr<drg_sim, void (*)(drg_sim*)> s(
            drg::build_similarity(ctx, g, p->k, p->sigma, 0, nullptr, p->perplexity),
            drg_sim_destroy);
        std::unique_ptr<drg_hier, void (*)(drg_hier*)> h(
            drg::build_hierarchy(ctx, g, p->seed, p->rho, p->min_nodes, p->max_levels),
            drg_hier_destroy);
        run_schedule(ctx, s.get(), h.get(), p, nullptr, nullptr, nullptr, nullptr, y_out_dev);
    });
}

drg_status drg_batch_create(drg_ctx* ctx, const drg_csr* graphs, int32_t count,
                            const drg_layout_params* params, drg_batch** out) {
    return guarded([&] {
        need(ctx, "ctx");
        need(out, "out");
        *out = nullptr;
        CtxScope scope(ctx);
        *out = drg::batch_create(ctx, graphs, count, params);
    });
}

drg_status drg_batch_info(const drg_batch* b, int64_t* n_total, int64_t* nnz_total, int32_t* T,
                          int32_t* nodes_host, int32_t* levels_host) {
    return guarded([&] { drg::batch_info(b, n_total, nnz_total, T, nodes_host, levels_host); });
}

drg_status drg_batch_tuning(const drg_batch* b, int32_t cap, int32_t* n, int32_t* chosen,
                            int32_t* rpl, int32_t* ch, float* ms) {
    return guarded([&] { drg::batch_tuning(b, cap, n, chosen, rpl, ch, ms); });
}

drg_status drg_batch_run(drg_ctx* ctx, drg_batch* b, float* y_out_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        CtxScope scope(ctx);
        drg::batch_run(ctx, b, y_out_dev);
    });
}

void drg_batch_destroy(drg_batch* b) { drg::batch_destroy(b); }

drg_status drg_layout_batched(drg_ctx* ctx, const drg_csr* graphs, int32_t count,
                              const drg_layout_params* params, float* y_out_dev) {
    return guarded([&] {
        need(ctx, "ctx");
        need(y_out_dev, "y_out");
        CtxScope scope(ctx);
        std::unique_ptr<drg_batch, void (*)(drg_batch*)> b(
            drg::batch_create(ctx, graphs, count, params), drg_batch_destroy);
        drg::batch_run(ctx, b.get(), y_out_dev);
    });
}

}  // extern "C"
