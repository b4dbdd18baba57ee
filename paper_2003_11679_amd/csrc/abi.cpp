// C ABI (include/sie.h): argument checking, error capture, dispatch.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "problem.h"
#include "tune.h"

using namespace sie;

static thread_local std::string g_err;

static sie_status fail(sie_status s, const std::string &m) {
    g_err = m;
    return s;
}

namespace sie {
void set_last_error(const std::string &m) { g_err = m; }
}  // namespace sie

template <typename F>
static sie_status guard(F &&f) {
    try {
        g_err.clear();
        f();
        return SIE_OK;
    } catch (const Error &e) {
        return fail(e.code, e.what());
    } catch (const std::bad_alloc &) {
        return fail(SIE_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(SIE_EINVAL, e.what());
    }
}

// The same, also recording a failure's message on the context.
template <typename F>
static sie_status guard(sie_ctx *ctx, F &&f) {
    const sie_status st = guard(std::forward<F>(f));
    if (st != SIE_OK && ctx) ctx_set_error(ctx, g_err);
    return st;
}
static sie_ctx *ctx_of(const sie_problem *p) { return p ? p->ctx : nullptr; }

// The library runs its own work (setup, solves) on the calling thread's
// default stream.  A null stream handed in by a caller means the caller's
// legacy default stream, so hot-path calls order with the caller's work.
static hipStream_t user_stream(void *stream) { return stream ? (hipStream_t)stream : hipStreamLegacy; }

// Entry points that run on the thread's own stream first wait for work the
// caller queued on the legacy default stream; server workers have no such
// caller (and the wait would order them behind every blocking stream).
static thread_local bool g_worker = false;
namespace sie {
void mark_worker_thread() { g_worker = true; }
}  // namespace sie
static void after_caller_work() {
    if (!g_worker) SIE_HIP(hipStreamSynchronize(hipStreamLegacy));
}

extern "C" {

const char *sie_last_error(void) { return g_err.c_str(); }

const char *sie_ctx_last_error(const sie_ctx *ctx) {
    if (!ctx) return "";
    sie_ctx *c = const_cast<sie_ctx *>(ctx);
    std::lock_guard<std::mutex> lk(c->mu);
    return c->err.c_str();
}

sie_status sie_ctx_create(int device, sie_ctx **out) {
    return guard([&] {
        SIE_CHECK(out, SIE_EINVAL, "out is NULL");
        int n = 0;
        SIE_HIP(hipGetDeviceCount(&n));
        SIE_CHECK(device >= 0 && device < n, SIE_EDEVICE, "no HIP device " + std::to_string(device));
        SIE_HIP(hipSetDevice(device));
        noalloc_init(device);
        auto *c = new sie_ctx;
        c->device = device;
        *out = c;
    });
}

void sie_ctx_destroy(sie_ctx *ctx) { delete ctx; }

sie_status sie_ctx_trim(sie_ctx *ctx) {
    return guard(ctx, [&] {
        SIE_CHECK(ctx, SIE_EINVAL, "NULL context");
        pool_trim(ctx->device);
    });
}

sie_status sie_set_tuning(int32_t mode) {
    return guard([&] { tune_set_mode(mode); });
}

sie_status sie_tuning_force(int32_t family, int32_t candidate) {
    return guard([&] { tune_force(family, candidate); });
}

sie_status sie_tuning_report(char *buf, size_t len, size_t *needed) {
    return guard([&] {
        SIE_CHECK(buf || len == 0, SIE_EINVAL, "NULL buffer with nonzero length");
        const std::string r = tune_report();
        if (needed) *needed = r.size() + 1;
        if (len) {
            const size_t n = std::min(len - 1, r.size());
            std::memcpy(buf, r.data(), n);
            buf[n] = '\0';
        }
    });
}

sie_status sie_tuning_clear(void) {
    return guard([&] { tune_clear(); });
}

sie_status sie_problem_create(sie_ctx *ctx, double freq_hz, double bg_eps_r, double bg_mu_r, sie_problem **out) {
    return guard(ctx, [&] {
        SIE_CHECK(ctx && out, SIE_EINVAL, "NULL argument");
        SIE_CHECK(freq_hz > 0 && std::isfinite(freq_hz), SIE_EINVAL, "frequency must be positive");
        SIE_CHECK(bg_eps_r > 0 && bg_mu_r > 0, SIE_EINVAL, "background must be lossless with positive eps, mu");
        auto *p = new sie_problem;
        p->ctx = ctx;
        p->freq = freq_hz;
        p->bg_eps_r = bg_eps_r;
        p->bg_mu_r = bg_mu_r;
        *out = p;
    });
}

sie_status sie_problem_add_object(sie_problem *p, const double *xyz, int64_t nv, const int32_t *tri, int64_t nt,
                                  double eps_r, double mu_r, double sigma, int32_t *obj_id) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p && xyz && tri, SIE_EINVAL, "NULL argument");
        SIE_CHECK(!p->is_setup, SIE_ESTATE, "problem already set up");
        SIE_CHECK(nv >= 4 && nt >= 4, SIE_EMESH, "a closed surface needs at least 4 vertices and 4 triangles");
        SIE_CHECK(eps_r > 0 && mu_r > 0 && sigma >= 0, SIE_EINVAL, "material needs eps_r > 0, mu_r > 0, sigma >= 0");
        for (int64_t i = 0; i < 3 * nv; ++i) SIE_CHECK(std::isfinite(xyz[i]), SIE_EMESH, "non-finite vertex");
        ObjIn o;
        o.xyz.assign(xyz, xyz + 3 * nv);
        o.tri.assign(tri, tri + 3 * nt);
        o.eps_r = eps_r; o.mu_r = mu_r; o.sigma = sigma;
        p->objs.push_back(std::move(o));
        p->obj_req.push_back(GridReq());
        if (obj_id) *obj_id = (int32_t)p->objs.size() - 1;
    });
}

sie_status sie_problem_set_grid(sie_problem *p, int32_t medium, int32_t n, int32_t near_radius, int32_t share) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p, SIE_EINVAL, "NULL problem");
        SIE_CHECK(!p->is_setup, SIE_ESTATE, "problem already set up");
        SIE_CHECK(n == 0 || (n >= 5 && n <= 1024), SIE_EINVAL, "grid points per axis must be 0 or in [5, 1024]");
        SIE_CHECK(near_radius >= 1 && near_radius <= 12, SIE_EINVAL, "near radius must be in [1, 12]");
        GridReq r;
        r.n = n; r.R = near_radius; r.share = share ? 1 : 0;
        if (medium == -1) { r.share = -1; p->ext_req = r; return; }
        SIE_CHECK(medium >= 0 && medium < (int)p->objs.size(), SIE_EINVAL, "medium out of range");
        p->obj_req[medium] = r;
    });
}

sie_status sie_grid_choose(double freq_hz, double eps_r, double mu_r, double sigma, double extent, double mean_edge,
                           int32_t near_radius, int32_t strict, sie_grid_params *out) {
    return guard([&] {
        SIE_CHECK(out, SIE_EINVAL, "out is NULL");
        choose_grid(freq_hz, eps_r, mu_r, sigma, extent, mean_edge, near_radius, strict, out);
    });
}

sie_status sie_problem_set_grid_params(sie_problem *p, int32_t medium, const sie_grid_params *g, int32_t share) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p && g, SIE_EINVAL, "NULL argument");
        SIE_CHECK(!p->is_setup, SIE_ESTATE, "problem already set up");
        SIE_CHECK(g->order == 0 || g->order == 2, SIE_EINVAL, "only stencil order 2 (3 points per axis) is built");
        const int R = g->near_radius == 0 ? 5 : g->near_radius;
        SIE_CHECK(R >= 1 && R <= 12, SIE_EINVAL, "near radius must be in [1, 12]");
        SIE_CHECK(g->n == 0 || (g->n >= 5 && g->n <= 1024), SIE_EINVAL, "grid points per axis must be 0 or in [5, 1024]");
        SIE_CHECK(g->h >= 0 && std::isfinite(g->h), SIE_EINVAL, "grid spacing must be finite and non-negative");
        GridReq r;
        r.n = g->n;
        r.R = R;
        r.h = g->n > 0 ? g->h : 0.0;
        r.has_origin = std::isfinite(g->origin[0]) && std::isfinite(g->origin[1]) && std::isfinite(g->origin[2]);
        for (int c = 0; c < 3; ++c) r.origin[c] = g->origin[c];
        r.share = share ? 1 : 0;
        if (medium == -1) { r.share = -1; p->ext_req = r; return; }
        SIE_CHECK(medium >= 0 && medium < (int)p->objs.size(), SIE_EINVAL, "medium out of range");
        p->obj_req[medium] = r;
    });
}

sie_status sie_problem_set_quadrature(sie_problem *p, const sie_quad_params *q) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p && q, SIE_EINVAL, "NULL argument");
        SIE_CHECK(!p->is_setup, SIE_ESTATE, "problem already set up");
        p->quad = *q;
    });
}

sie_status sie_problem_set_skin_cutoff(sie_problem *p, double skin_depths) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p, SIE_EINVAL, "NULL problem");
        SIE_CHECK(!p->is_setup, SIE_ESTATE, "problem already set up");
        SIE_CHECK(skin_depths >= 0.0 && std::isfinite(skin_depths), SIE_EINVAL, "cutoff must be finite and >= 0");
        p->cutoff_factor = skin_depths;
    });
}

sie_status sie_problem_set_augmented(sie_problem *p, int32_t on) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p, SIE_EINVAL, "NULL problem");
        SIE_CHECK(!p->is_setup, SIE_ESTATE, "problem already set up");
        SIE_CHECK(on == 0 || on == 1, SIE_EINVAL, "augmented must be 0 or 1");
        p->aug_mode = on;
    });
}

sie_status sie_problem_augmented_info(const sie_problem *p, int32_t *on, int64_t *factor_nnz, int32_t *levels,
                                      double *t_factor_s) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
        const bool a = (bool)p->aug;
        if (on) *on = a ? 1 : 0;
        if (factor_nnz) *factor_nnz = a ? p->aug->lu.nnz_factor : 0;
        if (levels) *levels = a ? (int32_t)p->aug->lu.lev_ptr.size() - 1 : 0;
        if (t_factor_s) *t_factor_s = a ? p->aug->t_factor_s : 0.0;
    });
}

sie_status sie_constraint_precond(sie_problem *p, int32_t nrhs, const void *x_dev, void *y_dev, void *stream) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
        SIE_CHECK(p->aug, SIE_ESTATE, "problem not set up for the augmented EFIE");
        SIE_CHECK(x_dev && y_dev && nrhs >= 1, SIE_EINVAL, "bad vectors");
        SIE_CHECK(x_dev != y_dev, SIE_EINVAL, "x and y must not alias");
        cp_apply(p, nrhs, (const c128 *)x_dev, (c128 *)y_dev, user_stream(stream));
    });
}

int32_t sie_medium_is_local(const sie_problem *p, int32_t medium) {
    int32_t out = SIE_EINVAL;
    const sie_status st = guard(ctx_of(p), [&] {
        SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
        out = p->medium(medium).local ? 1 : 0;
    });
    return st == SIE_OK ? out : st;
}

sie_status sie_problem_setup(sie_problem *p) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p, SIE_EINVAL, "NULL problem");
        SIE_CHECK(!p->is_setup, SIE_ESTATE, "problem already set up");
        after_caller_work();
        const auto t0 = std::chrono::steady_clock::now();
        problem_setup(p);
        p->t_setup_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    });
}

void sie_problem_destroy(sie_problem *p) {
    if (!p) return;
    if (p->solve) solver_destroy(p->solve);
    delete p;
}

int64_t sie_problem_num_rwg(const sie_problem *p) { return p && p->is_setup ? p->mesh.nrwg : -1; }
int64_t sie_problem_num_tri(const sie_problem *p) { return p && p->is_setup ? p->mesh.nt() : -1; }

sie_status sie_get_rwg(const sie_problem *p, int32_t *edge_v, int32_t *tpm) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
        if (edge_v) std::memcpy(edge_v, p->mesh.edge_v.data(), p->mesh.edge_v.size() * sizeof(int32_t));
        if (tpm) std::memcpy(tpm, p->mesh.tpm.data(), p->mesh.tpm.size() * sizeof(int32_t));
    });
}

sie_status sie_get_grid(const sie_problem *p, int32_t medium, double *origin, double *h, int32_t *n, int32_t *lo,
                        int32_t *nl, int32_t *m) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
        const Grid &g = *p->medium(medium).grid;
        for (int c = 0; c < 3; ++c) {
            if (origin) origin[c] = g.origin[c];
            if (n) n[c] = g.n[c];
            if (lo) lo[c] = g.lo[c];
            if (nl) nl[c] = g.nl[c];
            if (m) m[c] = g.m[c];
        }
        if (h) *h = g.h;
    });
}

sie_status sie_get_stencils(const sie_problem *p, int32_t medium, int32_t *out, int64_t *nt_grid) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
        const Grid &g = *p->medium(medium).grid;
        const int64_t ntg = (int64_t)g.tris.size();
        if (nt_grid) *nt_grid = ntg;
        if (!out) return;
        // ascending global triangle order
        std::vector<std::pair<int32_t, int64_t>> ord(ntg);
        for (int64_t i = 0; i < ntg; ++i) ord[i] = {g.tris[i], i};
        std::sort(ord.begin(), ord.end());
        for (int64_t j = 0; j < ntg; ++j)
            for (int c = 0; c < 3; ++c) out[3 * j + c] = g.centre[3 * ord[j].second + c];
    });
}

sie_status sie_stencil_assign(sie_problem *p, int32_t medium, int32_t *centre_dev, void *stream) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
        SIE_CHECK(centre_dev, SIE_EINVAL, "NULL pointer");
        const Grid &g = *p->medium(medium).grid;
        // the grid covers whole objects, whose triangles are contiguous
        const int64_t t0 = *std::min_element(g.tris.begin(), g.tris.end());
        const int64_t ntg = (int64_t)g.tris.size();
        launch_stencil_assign(p->d_centroid.p, nullptr, t0, ntg, g.origin, g.h, g.n, centre_dev, nullptr,
                              user_stream(stream));
    });
}

sie_status sie_get_near_pattern(const sie_problem *p, int32_t medium, int64_t *row_ptr, int32_t *cols, int64_t *nnz) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
        const Grid &g = *p->medium(medium).grid;
        if (nnz) *nnz = g.nnz;
        if (!row_ptr) return;
        const int64_t E = p->mesh.nrwg;
        std::vector<int64_t> rp = g.d_row_ptr.download(g.rwg1 - g.rwg0 + 1);
        for (int64_t r = 0; r <= E; ++r) {
            if (r <= g.rwg0) row_ptr[r] = 0;
            else if (r >= g.rwg1) row_ptr[r] = g.nnz;
            else row_ptr[r] = rp[r - g.rwg0];
        }
        if (cols && g.nnz) {
            std::vector<int32_t> c = g.d_cols.download(g.nnz);
            std::memcpy(cols, c.data(), g.nnz * sizeof(int32_t));
        }
    });
}

sie_status sie_get_near_values(const sie_problem *p, int32_t medium, sie_op op, sie_c128 *out) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
        SIE_CHECK(op == SIE_OP_L || op == SIE_OP_K, SIE_EINVAL, "near values exist for L and K");
        const Medium &md = p->medium(medium);
        const int64_t nnz = md.grid->nnz;
        std::vector<c128> v = (op == SIE_OP_L ? md.d_nL64 : md.d_nK64).download(nnz);
        std::memcpy(out, v.data(), nnz * sizeof(c128));
    });
}

sie_status sie_get_wavenumber(const sie_problem *p, int32_t medium, sie_c128 *k) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p && p->is_setup && k, SIE_ESTATE, "problem not set up");
        const c128 v = p->medium(medium).k;
        k->re = v.re; k->im = v.im;
    });
}

sie_status sie_matvec(sie_problem *p, int32_t medium, sie_op op, sie_precision prec, int32_t nrhs, const void *x_dev,
                      void *y_dev, void *stream) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
        SIE_CHECK(x_dev && y_dev && nrhs >= 1, SIE_EINVAL, "bad vectors");
        SIE_CHECK(x_dev != y_dev, SIE_EINVAL, "x and y must not alias");
        SIE_CHECK(op == SIE_OP_L || op == SIE_OP_K || op == SIE_OP_X || op == SIE_OP_AUG, SIE_EINVAL,
                  "unknown operator");
        hipStream_t st = user_stream(stream);
        if (op == SIE_OP_AUG) {
            SIE_CHECK(medium == -1, SIE_EINVAL, "the augmented product belongs to the exterior medium (-1)");
            SIE_CHECK(prec == SIE_FP64, SIE_EINVAL, "the augmented product runs in FP64");
            SIE_CHECK(p->aug, SIE_ESTATE, "problem not set up for the augmented EFIE");
            aug_product(p, nrhs, (const c128 *)x_dev, (c128 *)y_dev, st);
            return;
        }
        if (medium == SIE_INTERIORS && op != SIE_OP_X) {
            SIE_CHECK(prec == SIE_FP64 || prec == SIE_FP32, SIE_EINVAL, "unknown precision");
            for (auto &gp : p->groups) {
                if (prec == SIE_FP64)
                    group_product<double>(p, *gp, op, false, nrhs, (const c128 *)x_dev, (c128 *)y_dev, st);
                else
                    group_product<float>(p, *gp, op, false, nrhs, (const c64 *)x_dev, (c64 *)y_dev, st);
            }
            return;
        }
        Medium &md = p->medium(op == SIE_OP_X ? -1 : medium);
        if (prec == SIE_FP64)
            matvec<double>(p, md, op, nrhs, (const c128 *)x_dev, (c128 *)y_dev, st);
        else if (prec == SIE_FP32)
            matvec<float>(p, md, op, nrhs, (const c64 *)x_dev, (c64 *)y_dev, st);
        else
            throw Error(SIE_EINVAL, "unknown precision");
    });
}

sie_status sie_matvec_noalloc(sie_problem *p, int32_t medium, sie_op op, sie_precision prec, const void *x_dev,
                              void *y_dev, void *stream) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
        SIE_CHECK(x_dev && y_dev, SIE_EINVAL, "bad vectors");
        SIE_CHECK(x_dev != y_dev, SIE_EINVAL, "x and y must not alias");
        SIE_CHECK(op == SIE_OP_L || op == SIE_OP_K || op == SIE_OP_X, SIE_EINVAL, "unknown operator");
        SIE_CHECK(prec == SIE_FP64 || prec == SIE_FP32, SIE_EINVAL, "unknown precision");
        Medium &md = p->medium(op == SIE_OP_X ? -1 : medium);
        matvec_noalloc(p, md, op, prec, x_dev, y_dev, user_stream(stream));
    });
}

sie_status sie_nested_precond(sie_problem *p, int32_t precond, sie_precision prec, int32_t nrhs, const void *x_dev,
                              void *y_dev, void *stream) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p, SIE_EINVAL, "NULL problem");
        nested_precond_entry(p, precond, prec, nrhs, x_dev, y_dev, user_stream(stream));
    });
}

int32_t sie_nested_precond_factored(const sie_problem *p, int64_t *factor_nnz, double *t_factor_s) {
    if (!p) return -1;
    return nested_precond_factored(p, factor_nnz, t_factor_s);
}

int32_t sie_nested_precond_clusters(const sie_problem *p, int64_t *owned) {
    if (!p) return -1;
    return nested_precond_clusters(p, owned);
}

sie_status sie_project(sie_problem *p, int32_t medium, sie_precision prec, const void *x_dev, void *grid_dev,
                       void *stream) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
        SIE_CHECK(x_dev && grid_dev, SIE_EINVAL, "NULL pointer");
        Medium &md = p->medium(medium);
        if (prec == SIE_FP64) stage_project<double>(p, md, (const c128 *)x_dev, (c128 *)grid_dev, user_stream(stream));
        else stage_project<float>(p, md, (const c64 *)x_dev, (c64 *)grid_dev, user_stream(stream));
    });
}

sie_status sie_convolve(sie_problem *p, int32_t medium, sie_op op, sie_precision prec, int32_t nfields,
                        const void *in_dev, void *out_dev, void *stream) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
        SIE_CHECK(in_dev && out_dev, SIE_EINVAL, "NULL pointer");
        SIE_CHECK(op == SIE_OP_L || op == SIE_OP_K, SIE_EINVAL, "convolution op must be L (G) or K (grad G x)");
        Medium &md = p->medium(medium);
        if (prec == SIE_FP64)
            stage_convolve<double>(p, md, op, nfields, (const c128 *)in_dev, (c128 *)out_dev, user_stream(stream));
        else
            stage_convolve<float>(p, md, op, nfields, (const c64 *)in_dev, (c64 *)out_dev, user_stream(stream));
    });
}

sie_status sie_interpolate(sie_problem *p, int32_t medium, sie_precision prec, const void *grid_dev, void *y_dev,
                           void *stream) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
        SIE_CHECK(grid_dev && y_dev, SIE_EINVAL, "NULL pointer");
        Medium &md = p->medium(medium);
        if (prec == SIE_FP64)
            stage_interpolate<double>(p, md, (const c128 *)grid_dev, (c128 *)y_dev, user_stream(stream));
        else
            stage_interpolate<float>(p, md, (const c64 *)grid_dev, (c64 *)y_dev, user_stream(stream));
    });
}

sie_status sie_set_timing(sie_problem *p, int32_t on) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p, SIE_EINVAL, "NULL problem");
        SIE_CHECK(on >= 0 && on <= 2, SIE_EINVAL, "timing mode must be 0, 1 or 2");
        p->timer.reset();
        p->timer.on = on;
    });
}

sie_status sie_get_stage_time(sie_problem *p, int32_t stage, int64_t *launches, double *total_ms) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(p, SIE_EINVAL, "NULL problem");
        SIE_CHECK(stage >= 0 && stage < NSTAGE, SIE_EINVAL, "stage out of range");
        p->timer.flush();
        if (launches) *launches = p->timer.count[stage];
        if (total_ms) *total_ms = p->timer.total_ms[stage];
    });
}

sie_status sie_set_planewaves(sie_problem *p, int32_t nrhs, const double *khat, const sie_c128 *e0) {
    return guard(ctx_of(p), [&] {
        after_caller_work();
        planewaves_entry(p, nrhs, khat, e0);
    });
}

sie_status sie_solve(sie_problem *p, sie_precision prec, const sie_solver_opts *opts, sie_report *report) {
    return guard(ctx_of(p), [&] {
        after_caller_work();
        solve_entry(p, prec, opts, report);
    });
}

sie_status sie_get_currents(const sie_problem *p, int32_t rhs, sie_c128 *u, sie_c128 *v) {
    return guard(ctx_of(p), [&] { currents_entry(p, rhs, u, v); });
}

sie_status sie_get_charges(const sie_problem *p, int32_t rhs, sie_c128 *sigma) {
    return guard(ctx_of(p), [&] { charges_entry(p, rhs, sigma); });
}

sie_status sie_far_field(const sie_problem *p, int32_t rhs, int64_t ndir, const double *rhat, sie_c128 *F) {
    return guard(ctx_of(p), [&] { farfield_entry(p, rhs, ndir, rhat, F); });
}

sie_status sie_far_field_angles(const sie_problem *p, int32_t rhs, int64_t ndir, const double *theta,
                                const double *phi, sie_c128 *e_theta, sie_c128 *e_phi) {
    return guard(ctx_of(p), [&] {
        SIE_CHECK(ndir >= 0 && (ndir == 0 || (theta && phi && e_theta && e_phi)), SIE_EINVAL, "bad directions");
        if (ndir == 0) return;
        std::vector<double> rhat(3 * ndir);
        std::vector<sie_c128> F(3 * ndir);
        for (int64_t i = 0; i < ndir; ++i) {
            const double st = std::sin(theta[i]), ct = std::cos(theta[i]), sp = std::sin(phi[i]), cp = std::cos(phi[i]);
            rhat[3 * i] = st * cp; rhat[3 * i + 1] = st * sp; rhat[3 * i + 2] = ct;
        }
        farfield_entry(p, rhs, ndir, rhat.data(), F.data());
        for (int64_t i = 0; i < ndir; ++i) {
            const double st = std::sin(theta[i]), ct = std::cos(theta[i]), sp = std::sin(phi[i]), cp = std::cos(phi[i]);
            const double th[3] = {ct * cp, ct * sp, -st}, ph[3] = {-sp, cp, 0.0};
            sie_c128 a{0, 0}, b{0, 0};
            for (int c = 0; c < 3; ++c) {
                a.re += th[c] * F[3 * i + c].re; a.im += th[c] * F[3 * i + c].im;
                b.re += ph[c] * F[3 * i + c].re; b.im += ph[c] * F[3 * i + c].im;
            }
            e_theta[i] = a;
            e_phi[i] = b;
        }
    });
}

}  // extern "C"
