// Problem setup and the AIM operator product (Sec. III-D-1).
//
// Readings of what the paper leaves to its references:
//  * grid: isotropic spacing h = (largest bounding-box extent)/(n - 3), one
//    spare node on each side, centred on the bounding box;
//  * stencil: 3 points per axis (order n = 2, the order of Fig. R), anchored
//    at floor((c - x0)/h + 0.5) of the triangle centroid c, clamped to
//    [1, n - 2];
//  * projection: Galerkin moments of the tensor Lagrange polynomials (moment
//    matching up to degree 2 per axis), interpolation W = P^T;
//  * grid Green's function zero at zero offset (only near pairs see it, and
//    they are precorrected);
//  * near region: stencil centres within R cells per axis (R = 5: a near
//    region 11 grid points across, Sec. IV-A);
//  * scalar potential term subtracted (L = A - k^-2 Phi, eq. AIM_Lin with the
//    sign carried by W_phi).
#include <algorithm>
#include <cmath>
#include <numeric>

#include <atomic>
#include <chrono>
#include <exception>
#include <mutex>
#include <thread>
#include <cstdio>
#include <cstdlib>

#include "problem.h"

namespace sie {

static const double C0 = 299792458.0;
static const double MU0 = 4e-7 * 3.14159265358979323846;
static const double EPS0 = 1.0 / (MU0 * C0 * C0);

// k = sqrt(w mu (w eps - j sigma)), principal branch (Re k >= 0, Im k <= 0) (eq. kin)
static c128 wavenumber(double w, double eps_r, double mu_r, double sigma) {
    const double ar = w * MU0 * mu_r * w * EPS0 * eps_r, ai = -w * MU0 * mu_r * sigma;
    const double mod = std::sqrt(std::hypot(ar, ai));
    const double ang = 0.5 * std::atan2(ai, ar);
    c128 k(mod * std::cos(ang), mod * std::sin(ang));
    if (k.re < 0) k = -k;
    return k;
}

static int next_pow2(int v) {
    int m = 1;
    while (m < v) m <<= 1;
    return m;
}

// Largest vertex distance of every triangle from its centroid, in the
// arithmetic the near-list cutoff is compared with (no contraction).
static std::vector<double> bounding_radii(const Mesh &m) {
#pragma clang fp contract(off)
    const int64_t T = m.nt();
    std::vector<double> r(T);
    for (int64_t t = 0; t < T; ++t) {
        double best = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double *v = &m.xyz[3 * (int64_t)m.tri[3 * t + k]];
            const double *c = &m.centroid[3 * t];
            const double dx = v[0] - c[0], dy = v[1] - c[1], dz = v[2] - c[2];
            const double d2 = (dx * dx + dy * dy) + dz * dz;
            best = std::max(best, d2);
        }
        r[t] = std::sqrt(best);
    }
    return r;
}

// Grid geometry: explicit (h, n, origin) when given; otherwise n points per
// axis (n from the Sec. IV rule when 0: the finest spacing over the media
// that use the grid, at most 256 points per axis) over the largest
// bounding-box extent with one spare node a side, h = extent / (n - 3),
// centred on the bounding box.
struct MediumProps {
    double eps_r, mu_r, sigma;
};
static void build_grid_geometry(sie_problem *p, Grid &g, const GridReq &req, const std::vector<MediumProps> &media) {
    const Mesh &m = p->mesh;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    double esum = 0;
    int64_t ecnt = 0;
    for (int32_t t : g.tris)
        for (int k = 0; k < 3; ++k) {
            const double *v = &m.xyz[3 * (int64_t)m.tri[3 * (int64_t)t + k]];
            for (int c = 0; c < 3; ++c) { lo[c] = std::min(lo[c], v[c]); hi[c] = std::max(hi[c], v[c]); }
            const int e = m.tri_rwg[3 * (int64_t)t + k];
            esum += m.len[e]; ecnt++;
        }
    const double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    g.near_radius = req.R;
    if (req.h > 0 && req.n > 0) {
        g.h = req.h;
        for (int c = 0; c < 3; ++c) {
            g.n[c] = req.n;
            g.origin[c] = req.has_origin ? req.origin[c] : 0.5 * (lo[c] + hi[c]) - g.h * (req.n - 1) / 2.0;
        }
        return;
    }
    int n = req.n;
    if (n <= 0) {
        const double mean_edge = esum / std::max<int64_t>(ecnt, 1);
        n = 5;
        for (const MediumProps &md : media) {
            sie_grid_params gp;
            choose_grid(p->freq, md.eps_r, md.mu_r, md.sigma, std::max(ext, 1e-300), std::max(mean_edge, 1e-300),
                        req.R, 0, &gp);
            n = std::max(n, gp.n);
        }
        n = std::min(n, 256);
    }
    SIE_CHECK(n >= 4, SIE_EGRID, "grid needs at least 4 points per axis");
    g.h = ext / (n - 3);
    for (int c = 0; c < 3; ++c) {
        g.n[c] = n;
        g.origin[c] = 0.5 * (lo[c] + hi[c]) - g.h * (n - 1) / 2.0;
    }
}

// Stencil centres, live box, local (cell-sorted) triangle order, moments,
// projection lists, near pairs and the RWG near pattern of one grid.
// Setup phase timing on stderr when SIE_TRACE is set (waits for the device at
// every mark; silent and free otherwise).
static void setup_mark(const char *what) {
    static const bool trace = std::getenv("SIE_TRACE") != nullptr;
    if (!trace) return;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    static auto last = std::chrono::steady_clock::now();
    SIE_HIP(hipDeviceSynchronize());
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[setup] %-28s %8.1f ms\n", what, std::chrono::duration<double, std::milli>(now - last).count());
    last = now;
}

static void build_grid(sie_problem *p, Grid &g) {
    const Mesh &m = p->mesh;
    const int64_t ntg = (int64_t)g.tris.size();
    SIE_CHECK(ntg > 0, SIE_EINVAL, "grid without triangles");
    // 1. stencil assignment (ascending global order)
    {
        DBuf<int32_t> d_t(ntg), d_c(3 * ntg), d_raw(3 * ntg);
        d_t.upload(g.tris);
        launch_stencil_assign(p->d_centroid.p, d_t.p, 0, ntg, g.origin, g.h, g.n, d_c.p, d_raw.p, 0);
        std::vector<int32_t> c = d_c.download(), raw = d_raw.download();
        for (int64_t i = 0; i < 3 * ntg; ++i)
            SIE_CHECK(raw[i] >= 0 && raw[i] <= g.n[i % 3] - 1, SIE_EGRID, "triangle outside its grid");
        // 2. live box
        int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
        for (int64_t i = 0; i < ntg; ++i)
            for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], c[3 * i + k]); hi[k] = std::max(hi[k], c[3 * i + k]); }
        for (int k = 0; k < 3; ++k) {
            g.lo[k] = lo[k] - 1;
            g.nl[k] = hi[k] - lo[k] + 3;
            g.m[k] = std::max(2, next_pow2(2 * g.nl[k] - 1));
        }
        // every pair near: stencil centres within R of each other on every axis
        g.all_near = hi[0] - lo[0] <= g.near_radius && hi[1] - lo[1] <= g.near_radius &&
                     hi[2] - lo[2] <= g.near_radius;
        // 3. local order: sorted by live-box cell (z, y, x), then global id
        std::vector<int64_t> key(ntg);
        for (int64_t i = 0; i < ntg; ++i)
            key[i] = ((int64_t)(c[3 * i + 2] - g.lo[2]) * g.nl[1] + (c[3 * i + 1] - g.lo[1])) * g.nl[0] +
                     (c[3 * i] - g.lo[0]);
        std::vector<int64_t> ord(ntg);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });
        std::vector<int32_t> tris2(ntg), c2(3 * ntg);
        for (int64_t i = 0; i < ntg; ++i) {
            tris2[i] = g.tris[ord[i]];
            for (int k = 0; k < 3; ++k) c2[3 * i + k] = c[3 * ord[i] + k];
        }
        g.tris = tris2;
        g.centre = c2;
        g.d_tris.upload(g.tris);
        g.d_centre.upload(g.centre);
        // cell_ptr over live cells for the near search
        const int64_t nlive = g.nlive();
        std::vector<int32_t> cell_ptr(nlive + 1, 0);
        for (int64_t i = 0; i < ntg; ++i) cell_ptr[key[ord[i]] + 1]++;
        for (int64_t v = 0; v < nlive; ++v) cell_ptr[v + 1] += cell_ptr[v];
        // 4. near pairs
        DBuf<int32_t> d_cell(nlive + 1);
        d_cell.upload(cell_ptr);
        DBuf<int64_t> d_cnt(ntg);
        NearCut cut;
        cut.dc = g.cutoff;
        cut.centroid = p->d_centroid.p;
        cut.rho = p->d_rho.p;
        cut.tris = g.d_tris.p;
        launch_near_count(g.d_centre.p, ntg, d_cell.p, cut, g.lo, g.nl, g.near_radius, d_cnt.p, 0);
        std::vector<int64_t> cnt = d_cnt.download();
        std::vector<int64_t> pptr(ntg + 1, 0);
        for (int64_t i = 0; i < ntg; ++i) pptr[i + 1] = pptr[i] + cnt[i];
        g.npairs = pptr[ntg];
        g.d_pair_ptr.upload(pptr);
        g.d_pair_s.alloc(std::max<int64_t>(g.npairs, 1));
        launch_near_emit(g.d_centre.p, ntg, d_cell.p, cut, g.lo, g.nl, g.near_radius, g.d_pair_ptr.p,
                         g.d_pair_s.p, 0);
    }
    // 5. per-triangle coefficients and maps
    g.glob2loc.assign(m.nt(), -1);
    for (int64_t i = 0; i < ntg; ++i) g.glob2loc[g.tris[i]] = (int32_t)i;
    g.d_glob2loc.upload(g.glob2loc);
    g.tri_coef.assign(12 * ntg, 0.0);
    std::vector<float> coef32(12 * ntg);
    std::vector<int32_t> trirwg(3 * ntg);
    for (int64_t i = 0; i < ntg; ++i) {
        const int64_t t = g.tris[i];
        const double rc[3] = {g.origin[0] + g.h * g.centre[3 * i], g.origin[1] + g.h * g.centre[3 * i + 1],
                              g.origin[2] + g.h * g.centre[3 * i + 2]};
        for (int e = 0; e < 3; ++e) {
            const int32_t n = m.tri_rwg[3 * t + e];
            trirwg[3 * i + e] = n;
            const double ce = m.tri_sign[3 * t + e] * m.len[n] / (2.0 * m.area[t]);
            const double *pv = &m.xyz[3 * (int64_t)m.tri[3 * t + e]];
            double *o = &g.tri_coef[12 * i + 4 * e];
            o[0] = ce;
            for (int c = 0; c < 3; ++c) o[1 + c] = pv[c] - rc[c];
        }
    }
    for (int64_t i = 0; i < 12 * ntg; ++i) coef32[i] = (float)g.tri_coef[i];
    g.d_tri64.upload(g.tri_coef);
    g.d_tri32.upload(coef32);
    g.d_trirwg.upload(trirwg);
    // RWG rows of the grid's objects
    g.rwg0 = m.obj_rwg0[*std::min_element(g.objs.begin(), g.objs.end())];
    g.rwg1 = m.obj_rwg0[*std::max_element(g.objs.begin(), g.objs.end()) + 1];
    const int64_t nrow = g.rwg1 - g.rwg0;
    std::vector<int32_t> rwgloc(2 * nrow);
    for (int64_t r = 0; r < nrow; ++r) {
        const int64_t n = g.rwg0 + r;
        for (int s = 0; s < 2; ++s) {
            const int32_t tl = g.glob2loc[m.tpm[2 * n + s]];
            SIE_CHECK(tl >= 0, SIE_EINVAL, "RWG triangle not on its grid");
            rwgloc[2 * r + s] = (tl << 2) | m.epm[2 * n + s];
        }
    }
    g.d_rwgloc.upload(rwgloc);
    setup_mark("grid: stencils, near pairs");
    // 6. moments
    {
        Rule r = rule_collapsed(5);   // exact to degree 8 (integrands of degree 7)
        std::vector<double> packed(4 * r.size());
        for (int q = 0; q < r.size(); ++q) {
            for (int c = 0; c < 3; ++c) packed[4 * q + c] = r.bary[3 * q + c];
            packed[4 * q + 3] = r.w[q];
        }
        DBuf<double> d_rule;
        d_rule.upload(packed);
        g.d_mom64.alloc(27 * 4 * ntg);
        g.d_mom32.alloc(27 * 4 * ntg);
        launch_moments(p->d_xyz.p, p->d_tri.p, g.d_tris.p, g.d_centre.p, ntg, g.origin, g.h, d_rule.p, r.size(),
                       g.d_mom64.p, g.d_mom32.p, 0);
        SIE_HIP(hipStreamSynchronize(0));
    }
    // 7. projection gather lists: node -> (local triangle, slot)
    {
        const int64_t nlive = g.nlive();
        std::vector<int32_t> nptr(nlive + 1, 0), ent(27 * ntg);
        auto node_of = [&](int64_t i, int a) {
            const int dx = a % 3 - 1, dy = (a / 3) % 3 - 1, dz = a / 9 - 1;
            return ((int64_t)(g.centre[3 * i + 2] + dz - g.lo[2]) * g.nl[1] + (g.centre[3 * i + 1] + dy - g.lo[1])) *
                       g.nl[0] + (g.centre[3 * i] + dx - g.lo[0]);
        };
        for (int64_t i = 0; i < ntg; ++i)
            for (int a = 0; a < 27; ++a) nptr[node_of(i, a) + 1]++;
        for (int64_t v = 0; v < nlive; ++v) nptr[v + 1] += nptr[v];
        std::vector<int32_t> fill(nptr.begin(), nptr.end() - 1);
        for (int64_t i = 0; i < ntg; ++i)
            for (int a = 0; a < 27; ++a) ent[fill[node_of(i, a)]++] = (int32_t)((i << 5) | a);
        g.d_node_ptr.upload(nptr);
        g.d_node_ent.upload(ent);
    }
    setup_mark("grid: moments, gather lists");
    // 8. RWG near pattern
    {
        DBuf<int64_t> d_len(nrow), d_rp(nrow + 1);
        launch_rwg_pattern(nrow, g.rwg0, nrow, g.d_rwgloc.p, g.d_pair_ptr.p, g.d_pair_s.p, g.d_tris.p,
                           p->d_tri_rwg.p, d_len.p, nullptr, nullptr, 0, 0);
        std::vector<int64_t> len = d_len.download();
        std::vector<int64_t> rp(nrow + 1, 0);
        g.max_row = 0;
        for (int64_t r = 0; r < nrow; ++r) { rp[r + 1] = rp[r] + len[r]; g.max_row = std::max(g.max_row, len[r]); }
        g.nnz = rp[nrow];
        g.d_row_ptr.upload(rp);
        g.d_cols.alloc(std::max<int64_t>(g.nnz, 1));
        launch_rwg_pattern(nrow, g.rwg0, nrow, g.d_rwgloc.p, g.d_pair_ptr.p, g.d_pair_s.p, g.d_tris.p,
                           p->d_tri_rwg.p, nullptr, g.d_row_ptr.p, g.d_cols.p, 1, 0);
        // 16-bit column offsets for the near-field products
        g.d_row_base.alloc(std::max<int64_t>(nrow, 1));
        g.d_cols16.alloc(std::max<int64_t>(g.nnz, 1));
        DBuf<int> wide(1);
        SIE_HIP(hipMemsetAsync(wide.p, 0, sizeof(int), 0));
        launch_cols16(nrow, g.d_row_ptr.p, g.d_cols.p, g.d_row_base.p, g.d_cols16.p, wide.p, 0);
        int w = 0;
        SIE_HIP(hipMemcpyAsync(&w, wide.p, sizeof(int), hipMemcpyDeviceToHost, 0));
        SIE_HIP(hipStreamSynchronize(0));
        g.cols16 = w == 0;
        if (!g.cols16) {
            g.d_cols16 = DBuf<uint16_t>();
            g.d_row_base = DBuf<int32_t>();
        }
    }
}

static std::vector<double> pack_rule(const Rule &r) {
    std::vector<double> v(4 * r.size());
    for (int q = 0; q < r.size(); ++q) {
        for (int c = 0; c < 3; ++c) v[4 * q + c] = r.bary[3 * q + c];
        v[4 * q + 3] = r.w[q];
    }
    return v;
}

// A buffer that is already a large enough view into a group's array stays
// one; otherwise it gets memory of its own.
template <typename T>
static void keep_or_alloc(DBuf<T> &b, size_t n) {
    if (b.p && !b.own && b.n >= n) return;
    b.alloc(n);
}

// Kind of every near pair of a grid (self, edge, vertex, close, far), shared
// by the media on the grid.
static void pair_kinds(sie_problem *p, Grid &g, hipStream_t st) {
    g.d_pair_kind.alloc(std::max<int64_t>(g.npairs, 1));
    NearFillArgs a{};
    a.xyz = p->d_xyz.p; a.tri = p->d_tri.p; a.tris = g.d_tris.p; a.centroid = p->d_centroid.p;
    a.pair_ptr = g.d_pair_ptr.p; a.pair_s = g.d_pair_s.p; a.ntg = (int64_t)g.tris.size();
    launch_pair_kinds(a, g.d_pair_kind.p, st);
}

// Precorrected near values and Green's spectra of one medium on its grid.
static void build_medium(sie_problem *p, Medium &md, hipStream_t st) {
    Grid &g = *md.grid;
    const int64_t ntg = (int64_t)g.tris.size();
    // rules: 0 self, 1..3 edge, 4..6 vertex, 7 close, 8 far, 9 touch inner, 10 close inner, 11 far inner
    const sie_quad_params &q = p->quad;
    std::vector<Rule> rules;
    rules.push_back(rule_self(q.touch_out));
    for (int i = 0; i < 3; ++i) rules.push_back(rule_edge(q.touch_out, i));
    for (int i = 0; i < 3; ++i) rules.push_back(rule_vertex(q.touch_out, i));
    rules.push_back(rule_collapsed(q.close_out));
    rules.push_back(rule_collapsed(q.far_out));
    rules.push_back(rule_collapsed(q.touch_in));
    rules.push_back(rule_collapsed(q.close_in));
    rules.push_back(rule_collapsed(q.far_in));
    std::vector<double> packed;
    std::vector<int> off, num;
    for (auto &r : rules) {
        off.push_back((int)(packed.size() / 4));
        num.push_back(r.size());
        auto v = pack_rule(r);
        packed.insert(packed.end(), v.begin(), v.end());
    }
    DBuf<double> d_rules; d_rules.upload(packed, st);
    DBuf<int> d_off; d_off.upload(off, st);
    DBuf<int> d_num; d_num.upload(num, st);
    // radial Green's tables over squared node offsets of near pairs:
    // |d| <= R + 2 per axis
    const int W = g.near_radius + 2;
    const int nq = 3 * W * W + 1;
    DBuf<c128> d_grad(2 * nq);
    launch_green_radial(md.k, g.h, nq, d_grad.p, st);
    // strong-loss inner scheme: 8-point Gauss-Legendre on [-1, 1]
    std::vector<double> glx, glw, gl;
    gauss_legendre01(8, glx, glw);
    for (double x : glx) gl.push_back(2.0 * x - 1.0);
    for (double w : glw) gl.push_back(2.0 * w);
    DBuf<double> d_gl;
    d_gl.upload(gl, st);
    // strong-loss scheme: lossy enough a medium (|Im k| >= 0.38 |k|) and, for
    // some source triangle, |Im k| times its longest edge above 2 (the
    // per-pair test on the device; 1 % margin here so none is missed)
    double lmax_grid = 0.0;
    for (int32_t t : g.tris)
        for (int e = 0; e < 3; ++e) {
            const double *u = &p->mesh.xyz[3 * (int64_t)p->mesh.tri[3 * (int64_t)t + e]];
            const double *v = &p->mesh.xyz[3 * (int64_t)p->mesh.tri[3 * (int64_t)t + (e + 1) % 3]];
            lmax_grid = std::max(lmax_grid, std::sqrt((u[0] - v[0]) * (u[0] - v[0]) + (u[1] - v[1]) * (u[1] - v[1]) +
                                                      (u[2] - v[2]) * (u[2] - v[2])));
        }
    const int polar = std::fabs(md.k.im) >= 0.38 * std::hypot(md.k.re, md.k.im) &&
                              std::fabs(md.k.im) * lmax_grid > 0.99 * 2.0
                          ? 1
                          : 0;

    setup_mark("medium: rules, tables");
    // augmented EFIE: the exterior medium also yields the vector-potential
    // values, the pulse integrals and the preconditioner's diagonals
    const bool aug = p->aug && &md == &p->ext;
    if (aug) {
        AugState &A = *p->aug;
        SIE_CHECK(ntg == p->mesh.nt(), SIE_EINVAL, "augmented EFIE: exterior grid must hold every triangle");
        A.nA64.alloc(std::max<int64_t>(g.nnz, 1));
        A.gam64.alloc(std::max<int64_t>(g.npairs, 1));
        A.adiag.alloc(std::max<int64_t>(g.rwg1 - g.rwg0, 1));
        A.gself.alloc(std::max<int64_t>(ntg, 1));
        SIE_HIP(hipMemsetAsync(A.nA64.p, 0, A.nA64.bytes(), st));
        SIE_HIP(hipMemsetAsync(A.adiag.p, 0, A.adiag.bytes(), st));
        SIE_HIP(hipMemsetAsync(A.gself.p, 0, A.gself.bytes(), st));
    }
    const int bstride = aug ? 45 : 27;
    keep_or_alloc(md.d_nL64, std::max<int64_t>(g.nnz, 1));
    keep_or_alloc(md.d_nK64, std::max<int64_t>(g.nnz, 1));
    md.d_nLd64.alloc(std::max<int64_t>(g.nnz, 1));
    SIE_HIP(hipMemsetAsync(md.d_nL64.p, 0, md.d_nL64.bytes(), st));
    SIE_HIP(hipMemsetAsync(md.d_nK64.p, 0, md.d_nK64.bytes(), st));
    SIE_HIP(hipMemsetAsync(md.d_nLd64.p, 0, md.d_nLd64.bytes(), st));
    // process row triangles in chunks to bound the pair-block buffer
    setup_mark("medium: alloc + clear");
    std::vector<int64_t> pptr = g.d_pair_ptr.download();
    const int64_t max_chunk = 30000000 * 27 / bstride;  // pair blocks of one chunk: 13 GB of HBM at most
    DBuf<c128> blocks, ptab;
    DBuf<int64_t> d_pp;
    const int64_t nrow = g.rwg1 - g.rwg0;
    // precorrection tables: (2 (R + 1) + 1)^3 offsets x 10 sums per row, rows
    // of one chunk within 4 GB
    const int tab_w = g.near_radius + 1;
    const int64_t tab_row = (int64_t)(2 * tab_w + 1) * (2 * tab_w + 1) * (2 * tab_w + 1) * 10;
    const int64_t max_rows = std::max<int64_t>(1, (int64_t)(4e9 / (double)(tab_row * sizeof(c128))));
    SIE_CHECK(g.d_pair_kind.n == (size_t)std::max<int64_t>(g.npairs, 1), SIE_ESTATE, "pair kinds not classified");
    int64_t t0 = 0;
    while (t0 < ntg) {
        int64_t t1 = t0 + 1;
        while (t1 < ntg && pptr[t1 + 1] - pptr[t0] <= max_chunk && t1 - t0 < max_rows) ++t1;
        const int64_t np = pptr[t1] - pptr[t0];
        // chunk-relative pair pointers over all rows (rows outside the chunk empty)
        std::vector<int64_t> cp(ntg + 1);
        for (int64_t i = 0; i <= ntg; ++i) cp[i] = std::min(std::max(pptr[i], pptr[t0]), pptr[t1]) - pptr[t0];
        d_pp.upload(cp, st);
        blocks.alloc(std::max<int64_t>(np, 1) * bstride);
        setup_mark("fill: chunk buffers");
        NearFillArgs a;
        a.xyz = p->d_xyz.p; a.tri = p->d_tri.p; a.tris = g.d_tris.p; a.centre = g.d_centre.p;
        a.centroid = p->d_centroid.p; a.tri_coef = g.d_tri64.p; a.mom = g.d_mom64.p;
        a.pair_ptr = d_pp.p; a.pair_s = g.d_pair_s.p + pptr[t0]; a.ntg = ntg;
        a.rules = d_rules.p; a.rule_off = d_off.p; a.rule_n = d_num.p;
        a.gradial = d_grad.p; a.nq = nq; a.k = md.k; a.h = g.h;
        a.blocks = blocks.p;
        a.polar = polar;
        a.polar_gl = d_gl.p;
        a.tab_row0 = t0; a.tab_w = tab_w;
        a.pkind = g.d_pair_kind.p + pptr[t0];
        a.no_grid = md.local ? 1 : 0;
        a.bstride = bstride;
        a.gam = aug ? p->aug->gam64.p + pptr[t0] : nullptr;
        a.gself = aug ? p->aug->gself.p : nullptr;
        if (!md.local) {
            ptab.alloc((t1 - t0) * tab_row);
            a.ptab = ptab.p;
            launch_precorr_table(a, t0, t1 - t0, ptab.p, st);
        } else {
            a.ptab = nullptr;
        }
        setup_mark("fill: precorrection tables");
        launch_near_fill(a, np, st);
        setup_mark("fill: pair blocks");
        launch_near_gather(nrow, g.rwg0, g.max_row, g.d_row_ptr.p, g.d_cols.p, g.d_rwgloc.p, g.d_glob2loc.p,
                           p->d_tpm.p, p->d_epm.p, d_pp.p, g.d_pair_s.p + pptr[t0], blocks.p, bstride,
                           md.d_nL64.p, md.d_nK64.p, md.d_nLd64.p, aug ? p->aug->nA64.p : nullptr,
                           aug ? p->aug->adiag.p : nullptr, st);
        SIE_HIP(hipStreamSynchronize(st));
        t0 = t1;
    }
    setup_mark("medium: near fill");
    keep_or_alloc(md.d_nL32, std::max<int64_t>(g.nnz, 1));
    keep_or_alloc(md.d_nK32, std::max<int64_t>(g.nnz, 1));
    launch_convert<double, float>(md.d_nL64.p, md.d_nL32.p, g.nnz, st);
    launch_convert<double, float>(md.d_nK64.p, md.d_nK32.p, g.nnz, st);
    // spectra of G, dG/dx, dG/dy, dG/dz, folded to the octant, 1/(mx my mz) folded in
    setup_mark("medium: FP32 copies");
    DBuf<c128> d_vol, d_tmp;
    if (!md.local) {   // a medium without grid part needs no spectra
        const int64_t vol = g.mvol();
        d_vol.alloc(vol);
        d_tmp.alloc(vol);
        md.d_spec64.alloc(4 * g.oct());
        md.d_spec32.alloc(4 * g.oct());
        const double scale = 1.0 / (double)vol;
        for (int kind = 0; kind < 4; ++kind) {
            launch_green_sample(md.k, g.h, g.nl, g.m, kind, d_vol.p, st);
            fft3d_full_fwd(d_vol.p, d_tmp.p, g.m[0], g.m[1], g.m[2], st);
            launch_fold_octant(d_vol.p, g.m, kind, scale, md.d_spec64.p, md.d_spec32.p, st);
        }
    }
    SIE_HIP(hipStreamSynchronize(st));
    setup_mark("medium: spectra");
    // per-medium scalars of the products: -2 k^-2 (scalar term of L) and the
    // nested operator's factor -j w eps~
    const c128 ks = cdiv(c128(-2.0), md.k * md.k);
    const c128 al = c128(0.0, -p->w) * md.eps;
    md.d_ks64.upload(std::vector<c128>{ks}, st);
    md.d_ks32.upload(std::vector<c64>{c64((float)ks.re, (float)ks.im)}, st);
    md.d_alpha64.upload(std::vector<c128>{al}, st);
    md.d_alpha32.upload(std::vector<c64>{c64((float)al.re, (float)al.im)}, st);
    // every launch that used the temporaries has completed on st
    PoolSyncedFree synced;
    d_rules.release(); d_off.release(); d_num.release(); d_grad.release(); d_gl.release();
    blocks.release(); ptab.release(); d_pp.release(); d_vol.release(); d_tmp.release();
}

// Groups of interior media for batched products: consecutive objects whose
// own grids share the live-box and FFT shapes (at most kGroupMax per
// group); a medium on the exterior grid, or of a shape of its own, forms a
// group of one.  Media of larger groups get their near values as views into
// the group's arrays (filled in place by the near-field setup).
constexpr int kGroupMax = 4096;

static bool same_shape(const Grid &a, const Grid &b) {
    for (int c = 0; c < 3; ++c)
        if (a.nl[c] != b.nl[c] || a.m[c] != b.m[c]) return false;
    return true;
}

static void form_groups(sie_problem *p) {
    p->groups.clear();
    for (int i = 0; i < (int)p->ints.size(); ++i) {
        Medium &md = p->ints[i];
        const bool own = md.grid != p->ext.grid;
        if (own && !p->groups.empty()) {
            Group &last = *p->groups.back();
            const Medium &prev = p->ints[last.media.back()];
            if (prev.grid != p->ext.grid && last.media.back() == i - 1 && same_shape(*prev.grid, *md.grid) &&
                prev.local == md.local && (int)last.media.size() < kGroupMax) {
                last.media.push_back(i);
                md.group = (int)p->groups.size() - 1;
                continue;
            }
        }
        auto g = std::make_unique<Group>();
        g->media.push_back(i);
        md.group = (int)p->groups.size();
        p->groups.push_back(std::move(g));
    }
    for (auto &gp : p->groups) {
        Group &gr = *gp;
        if (gr.media.size() < 2) continue;
        int64_t nnz = 0;
        for (int i : gr.media) nnz += p->ints[i].grid->nnz;
        gr.nnz = nnz;
        gr.d_nL64.alloc(std::max<int64_t>(nnz, 1));
        gr.d_nK64.alloc(std::max<int64_t>(nnz, 1));
        gr.d_nL32.alloc(std::max<int64_t>(nnz, 1));
        gr.d_nK32.alloc(std::max<int64_t>(nnz, 1));
        int64_t off = 0;
        for (int i : gr.media) {
            Medium &md = p->ints[i];
            const int64_t n = std::max<int64_t>(md.grid->nnz, 1);
            md.d_nL64.view(gr.d_nL64.p + off, n);
            md.d_nK64.view(gr.d_nK64.p + off, n);
            md.d_nL32.view(gr.d_nL32.p + off, n);
            md.d_nK32.view(gr.d_nK32.p + off, n);
            off += md.grid->nnz;
        }
    }
}

template <typename T>
static void d2d(T *dst, const T *src, size_t n) {
    if (n) SIE_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToDevice, 0));
}

// Merged per-triangle, per-node and per-row arrays of the groups of several
// media, in slot order (slot s = the group's s-th medium); triangle, entry,
// row and nonzero indices offset by those of the earlier slots.
static void finalize_groups(sie_problem *p) {
    for (auto &gp : p->groups) {
        Group &gr = *gp;
        if (gr.media.size() < 2) {
            gr.grid0 = p->ints[gr.media[0]].grid;
            gr.view = view_of(*gr.grid0);
            continue;
        }
        const int S = (int)gr.media.size();
        const Grid &g0 = *p->ints[gr.media[0]].grid;
        int64_t ntg = 0, nrow = 0;
        bool c16 = true;
        for (int i : gr.media) {
            const Grid &g = *p->ints[i].grid;
            ntg += (int64_t)g.tris.size();
            nrow += g.rwg1 - g.rwg0;
            c16 = c16 && g.cols16;
        }
        const int64_t nlive = g0.nlive(), oct = g0.oct();
        std::vector<int32_t> centre(3 * ntg), slot(ntg), nptr((size_t)S * nlive + 1, 0), ent, rwgloc(2 * nrow);
        std::vector<int64_t> rptr(nrow + 1, 0);
        ent.reserve(27 * ntg);
        gr.d_trirwg.alloc(3 * ntg);
        gr.d_mom64.alloc(27 * 4 * ntg);
        gr.d_mom32.alloc(27 * 4 * ntg);
        gr.d_coef64.alloc(12 * ntg);
        gr.d_coef32.alloc(12 * ntg);
        gr.d_cols.alloc(std::max<int64_t>(gr.nnz, 1));
        if (c16) {
            gr.d_cols16.alloc(std::max<int64_t>(gr.nnz, 1));
            gr.d_row_base.alloc(std::max<int64_t>(nrow, 1));
        }
        const bool local = p->ints[gr.media[0]].local;
        if (!local) {
            gr.d_spec64.alloc((size_t)S * 4 * oct);
            gr.d_spec32.alloc((size_t)S * 4 * oct);
        }
        std::vector<c128> ks(S), al(S);
        int64_t toff = 0, roff = 0, zoff = 0, eoff = 0;
        for (int s = 0; s < S; ++s) {
            const Medium &md = p->ints[gr.media[s]];
            const Grid &g = *md.grid;
            const int64_t nt = (int64_t)g.tris.size(), nr = g.rwg1 - g.rwg0;
            for (int64_t t = 0; t < nt; ++t) {
                for (int c = 0; c < 3; ++c) centre[3 * (toff + t) + c] = g.centre[3 * t + c] - g.lo[c];
                slot[toff + t] = s;
            }
            const std::vector<int32_t> np = g.d_node_ptr.download(nlive + 1);
            for (int64_t v = 0; v < nlive; ++v) nptr[(size_t)s * nlive + v + 1] = (int32_t)(eoff + np[v + 1]);
            for (int32_t e : g.d_node_ent.download(np[nlive])) ent.push_back((int32_t)(((e >> 5) + toff) << 5 | (e & 31)));
            eoff += np[nlive];
            const std::vector<int32_t> rl = g.d_rwgloc.download(2 * nr);
            for (int64_t k = 0; k < 2 * nr; ++k) rwgloc[2 * roff + k] = (int32_t)((((rl[k] >> 2) + toff) << 2) | (rl[k] & 3));
            const std::vector<int64_t> rp = g.d_row_ptr.download(nr + 1);
            for (int64_t r = 0; r < nr; ++r) rptr[roff + r + 1] = zoff + rp[r + 1];
            d2d(gr.d_trirwg.p + 3 * toff, g.d_trirwg.p, 3 * nt);
            d2d(gr.d_mom64.p + 108 * toff, g.d_mom64.p, 108 * nt);
            d2d(gr.d_mom32.p + 108 * toff, g.d_mom32.p, 108 * nt);
            d2d(gr.d_coef64.p + 12 * toff, g.d_tri64.p, 12 * nt);
            d2d(gr.d_coef32.p + 12 * toff, g.d_tri32.p, 12 * nt);
            d2d(gr.d_cols.p + zoff, g.d_cols.p, g.nnz);
            if (c16) {
                d2d(gr.d_cols16.p + zoff, g.d_cols16.p, g.nnz);
                d2d(gr.d_row_base.p + roff, g.d_row_base.p, nr);
            }
            if (!local) {
                d2d(gr.d_spec64.p + (size_t)s * 4 * oct, md.d_spec64.p, 4 * oct);
                d2d(gr.d_spec32.p + (size_t)s * 4 * oct, md.d_spec32.p, 4 * oct);
            }
            ks[s] = cdiv(c128(-2.0), md.k * md.k);
            al[s] = c128(0.0, -p->w) * md.eps;
            toff += nt; roff += nr; zoff += g.nnz;
        }
        gr.d_centre.upload(centre);
        gr.d_tri_slot.upload(slot);
        gr.d_node_ptr.upload(nptr);
        gr.d_node_ent.upload(ent);
        gr.d_rwgloc.upload(rwgloc);
        gr.d_row_ptr.upload(rptr);
        gr.d_ks64.upload(ks);
        gr.d_alpha64.upload(al);
        std::vector<c64> ks32(S), al32(S);
        for (int s = 0; s < S; ++s) {
            ks32[s] = c64((float)ks[s].re, (float)ks[s].im);
            al32[s] = c64((float)al[s].re, (float)al[s].im);
        }
        gr.d_ks32.upload(ks32);
        gr.d_alpha32.upload(al32);
        SIE_HIP(hipStreamSynchronize(0));
        GridView v;
        v.nslot = S;
        v.ntg = ntg;
        v.nlive = nlive;
        for (int c = 0; c < 3; ++c) { v.nl[c] = g0.nl[c]; v.m[c] = g0.m[c]; v.lo[c] = 0; }
        v.rwg0 = g0.rwg0;
        v.rwg1 = g0.rwg0 + nrow;
        v.centre = gr.d_centre.p;
        v.tri_slot = gr.d_tri_slot.p;
        v.node_ptr = gr.d_node_ptr.p;
        v.node_ent = gr.d_node_ent.p;
        v.trirwg = gr.d_trirwg.p;
        v.rwgloc = gr.d_rwgloc.p;
        v.mom64 = gr.d_mom64.p; v.mom32 = gr.d_mom32.p;
        v.coef64 = gr.d_coef64.p; v.coef32 = gr.d_coef32.p;
        v.row_ptr = gr.d_row_ptr.p;
        v.cols = gr.d_cols.p;
        v.cols16 = c16 ? gr.d_cols16.p : nullptr;
        v.row_base = c16 ? gr.d_row_base.p : nullptr;
        v.c16 = c16;
        gr.view = v;
    }
}

static void build_x(sie_problem *p) {
    const Mesh &m = p->mesh;
    const int64_t E = m.nrwg;
    std::vector<std::vector<std::pair<int32_t, double>>> rows(E);
    for (int64_t t = 0; t < m.nt(); ++t) {
        const double *nn = &m.normal[3 * t];
        const double *c = &m.centroid[3 * t];
        double pr[3][3], ce[3];
        for (int e = 0; e < 3; ++e) {
            const double *pv = &m.xyz[3 * (int64_t)m.tri[3 * t + e]];
            for (int k = 0; k < 3; ++k) pr[e][k] = pv[k] - c[k];
            ce[e] = m.tri_sign[3 * t + e] * m.len[m.tri_rwg[3 * t + e]] / (2.0 * m.area[t]);
        }
        // int_t (n x f_e) . f_f dS = c_e c_f A n . (p_e' x p_f'), p' = p - centroid
        for (int e = 0; e < 3; ++e)
            for (int f = 0; f < 3; ++f) {
                const double cx_ = pr[e][1] * pr[f][2] - pr[e][2] * pr[f][1];
                const double cy = pr[e][2] * pr[f][0] - pr[e][0] * pr[f][2];
                const double cz = pr[e][0] * pr[f][1] - pr[e][1] * pr[f][0];
                const double v = ce[e] * ce[f] * m.area[t] * (nn[0] * cx_ + nn[1] * cy + nn[2] * cz);
                const int32_t a = m.tri_rwg[3 * t + e], b = m.tri_rwg[3 * t + f];
                bool found = false;
                for (auto &pr2 : rows[a])
                    if (pr2.first == b) { pr2.second += v; found = true; }
                if (!found) rows[a].push_back({b, v});
            }
    }
    std::vector<int32_t> ptr(E + 1, 0), col;
    std::vector<double> val;
    for (int64_t r = 0; r < E; ++r) {
        std::sort(rows[r].begin(), rows[r].end());
        for (auto &e : rows[r]) { col.push_back(e.first); val.push_back(e.second); }
        ptr[r + 1] = (int32_t)col.size();
    }
    std::vector<float> val32(val.begin(), val.end());
    p->d_xptr.upload(ptr);
    p->d_xcol.upload(col);
    p->d_xval64.upload(val);
    p->d_xval32.upload(val32);
}

GridView view_of(const Grid &g) {
    GridView v;
    v.nslot = 1;
    v.ntg = (int64_t)g.tris.size();
    v.nlive = g.nlive();
    for (int c = 0; c < 3; ++c) { v.nl[c] = g.nl[c]; v.m[c] = g.m[c]; v.lo[c] = g.lo[c]; }
    v.rwg0 = g.rwg0;
    v.rwg1 = g.rwg1;
    v.centre = g.d_centre.p;
    v.tri_slot = nullptr;
    v.node_ptr = g.d_node_ptr.p;
    v.node_ent = g.d_node_ent.p;
    v.trirwg = g.d_trirwg.p;
    v.rwgloc = g.d_rwgloc.p;
    v.mom64 = g.d_mom64.p; v.mom32 = g.d_mom32.p;
    v.coef64 = g.d_tri64.p; v.coef32 = g.d_tri32.p;
    v.row_ptr = g.d_row_ptr.p;
    v.cols = g.d_cols.p;
    v.cols16 = g.d_cols16.p;
    v.row_base = g.d_row_base.p;
    v.c16 = g.cols16;
    return v;
}

// Scratch for products of up to nrhs right-hand sides over a view (grown on
// demand; E is the number of RWG functions, for the transposed right-hand
// sides of a batched product).
template <typename T>
static void ensure_work(const GridView &v, Work<T> &w, int nrhs, int64_t E) {
    if (w.cap_rhs < nrhs) {
        const size_t F = 4, R = (size_t)nrhs, S = (size_t)v.nslot;
        w.grid.alloc(R * F * v.nnodes());
        w.bufA.alloc(R * F * S * v.nl[2] * v.nl[1] * v.m[0]);
        w.bufB.alloc(R * F * S * v.nl[2] * v.m[1] * v.m[0]);
        w.trisrc.alloc(R * 4 * v.ntg);
        w.tripot.alloc(R * 5 * v.ntg);
        w.cap_rhs = nrhs;
    }
    if (nrhs > 1 && w.xt.n < (size_t)nrhs * E) w.xt.alloc((size_t)nrhs * E);
}

template <> Work<double> &work_of<double>(Grid &g) { ensure_work(view_of(g), g.w64, 1, 0); return g.w64; }
template <> Work<float> &work_of<float>(Grid &g) { ensure_work(view_of(g), g.w32, 1, 0); return g.w32; }
template <typename T> static Work<T> &work_sel(Grid &g);
template <> Work<double> &work_sel<double>(Grid &g) { return g.w64; }
template <> Work<float> &work_sel<float>(Grid &g) { return g.w32; }
template <typename T> static Work<T> &work_sel(Group &g);
template <> Work<double> &work_sel<double>(Group &g) { return g.w64; }
template <> Work<float> &work_sel<float>(Group &g) { return g.w32; }

template <typename T> static const T *mom_v(const GridView &v);
template <> const double *mom_v<double>(const GridView &v) { return v.mom64; }
template <> const float *mom_v<float>(const GridView &v) { return v.mom32; }
template <typename T> static const T *coef_v(const GridView &v);
template <> const double *coef_v<double>(const GridView &v) { return v.coef64; }
template <> const float *coef_v<float>(const GridView &v) { return v.coef32; }
template <typename T> static const cx<T> *spec_of(const Medium &m);
template <> const c128 *spec_of<double>(const Medium &m) { return m.d_spec64.p; }
template <> const c64 *spec_of<float>(const Medium &m) { return m.d_spec32.p; }
template <typename T> static const T *xval_of(sie_problem *p);
template <> const double *xval_of<double>(sie_problem *p) { return p->d_xval64.p; }
template <> const float *xval_of<float>(sie_problem *p) { return p->d_xval32.p; }

// Medium-dependent arrays of a product of one medium on its own grid.
template <typename T> static MediaView<T> media_of(const Medium &m, bool scaled);
template <> MediaView<double> media_of<double>(const Medium &m, bool scaled) {
    MediaView<double> v;
    v.far = !m.local;
    v.spec = m.d_spec64.p; v.nL = m.d_nL64.p; v.nK = m.d_nK64.p; v.kscal = m.d_ks64.p;
    v.alpha = scaled ? m.d_alpha64.p : nullptr;
    return v;
}
template <> MediaView<float> media_of<float>(const Medium &m, bool scaled) {
    MediaView<float> v;
    v.far = !m.local;
    v.spec = m.d_spec32.p; v.nL = m.d_nL32.p; v.nK = m.d_nK32.p; v.kscal = m.d_ks32.p;
    v.alpha = scaled ? m.d_alpha32.p : nullptr;
    return v;
}
// ... and of a merged group (spectra [slot][4][oct]).
template <typename T> static MediaView<T> media_of(const Group &g, bool scaled);
template <> MediaView<double> media_of<double>(const Group &g, bool scaled) {
    MediaView<double> v;
    v.far = g.d_spec64.p != nullptr;
    v.spec = g.d_spec64.p; v.spec_stride = (int64_t)(g.d_spec64.n / g.view.nslot);
    v.nL = g.d_nL64.p; v.nK = g.d_nK64.p; v.kscal = g.d_ks64.p;
    v.alpha = scaled ? g.d_alpha64.p : nullptr;
    return v;
}
template <> MediaView<float> media_of<float>(const Group &g, bool scaled) {
    MediaView<float> v;
    v.far = g.d_spec32.p != nullptr;
    v.spec = g.d_spec32.p; v.spec_stride = (int64_t)(g.d_spec32.n / g.view.nslot);
    v.nL = g.d_nL32.p; v.nK = g.d_nK32.p; v.kscal = g.d_ks32.p;
    v.alpha = scaled ? g.d_alpha32.p : nullptr;
    return v;
}

// ---- stage timers
hipEvent_t StageTimer::get() {
    if (pool.empty()) {
        hipEvent_t e;
        SIE_HIP(hipEventCreate(&e));
        return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
}
void StageTimer::begin(int, hipStream_t st, hipEvent_t &a) {
    a = get();
    SIE_HIP(hipEventRecord(a, st));
}
void StageTimer::end(int stage, hipStream_t st, hipEvent_t a, int extra, int extra2) {
    hipEvent_t b = get();
    SIE_HIP(hipEventRecord(b, st));
    pending.push_back({stage, extra, extra2, a, b});
    if (pending.size() >= 4096) flush();
}
void StageTimer::flush() {
    for (auto &r : pending) {
        SIE_HIP(hipEventSynchronize(r.b));
        float ms = 0.f;
        SIE_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        total_ms[r.stage] += ms;
        count[r.stage] += 1;
        for (int x : {r.extra, r.extra2})
            if (x >= 0) {
                total_ms[x] += ms;
                count[x] += 1;
            }
        pool.push_back(r.a);
        pool.push_back(r.b);
    }
    pending.clear();
}
void StageTimer::reset() {
    flush();
    for (int i = 0; i < NSTAGE; ++i) { total_ms[i] = 0; count[i] = 0; }
}
StageTimer::~StageTimer() {
    for (auto &r : pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
}

// One AIM product over a view for nrhs right-hand sides [nrhs][E]: the rows
// of the view are written, others are not touched.  Every stage takes all
// right-hand sides and slots at once; with several right-hand sides the
// near-field values are streamed once for the whole batch.
template <typename T>
static void run_product(sie_problem *p, const GridView &v, const MediaView<T> &mv, sie_op op, int nrhs,
                        const cx<T> *x, cx<T> *y, const ProductBufs<T> &b, cx<T> *xt, StageTimer *tm,
                        hipStream_t st, bool interior = false) {
    // launches that skip the rows of inactive objects go to their own class
    const int x64 = v.active ? ST_SKIP : (sizeof(T) == 8 ? ST_SPMV64 : -1);
    const int xint = interior && !v.active ? (sizeof(T) == 8 ? ST_INT64 : ST_INT32) : -1;
    const int64_t E = p->mesh.nrwg;
    const int F = op == SIE_OP_L ? 4 : 3;
    const int nf = F * v.nslot * nrhs;
    const bool all = tm && tm->on == 1;   // every stage; otherwise the near-field CSR product only
    const bool csr = tm && tm->on;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const cx<T> *vals = op == SIE_OP_L ? mv.nL : mv.nK;
    if (!mv.far) {
        // local operator: the direct near-region values alone
        if (all) tm->begin(ST_PRODUCT, st, e0);
        if (csr) tm->begin(ST_SPMV, st, e1);
        if (nrhs == 1)
            launch_spmv_far<T>(v, coef_v<T>(v), (const cx<T> *)nullptr, (const cx<T> *)nullptr, mv.alpha, vals, x, y,
                               false, st);
        else
            launch_spmm_far<T>(v, E, nrhs, coef_v<T>(v), (const cx<T> *)nullptr, (const cx<T> *)nullptr, mv.alpha,
                               vals, x, xt, y, st);
        if (csr) tm->end(ST_SPMV, st, e1, x64, xint);
        if (all) tm->end(ST_PRODUCT, st, e0);
        return;
    }
    if (all) { tm->begin(ST_PRODUCT, st, e0); tm->begin(ST_PROJECT, st, e1); }
    launch_tri_sources<T>(v, coef_v<T>(v), x, E, nrhs, b.trisrc, st);
    launch_project<T>(v, mom_v<T>(v), b.trisrc, b.grid, F, nrhs, st);
    if (all) { tm->end(ST_PROJECT, st, e1); tm->begin(ST_FFT, st, e1); }
    fft_convolve<T>(v, mv.spec, mv.spec_stride, v.nslot > 1 ? F : nf, v.nslot, nf, op == SIE_OP_L ? 0 : 1, b.grid,
                    b.grid, b.bufA, b.bufB, st);
    if (all) { tm->end(ST_FFT, st, e1); tm->begin(ST_INTERP, st, e1); }
    launch_interp<T>(v, mom_v<T>(v), b.grid, F, nrhs, b.tripot, st);
    if (all) tm->end(ST_INTERP, st, e1);
    if (csr) tm->begin(ST_SPMV, st, e1);
    const cx<T> *ks = op == SIE_OP_L ? mv.kscal : nullptr;
    if (nrhs == 1)
        launch_spmv_far<T>(v, coef_v<T>(v), b.tripot, ks, mv.alpha, vals, x, y, true, st);
    else
        launch_spmm_far<T>(v, E, nrhs, coef_v<T>(v), b.tripot, ks, mv.alpha, vals, x, xt, y, st);
    if (csr) tm->end(ST_SPMV, st, e1, x64, xint);
    if (all) tm->end(ST_PRODUCT, st, e0);
}

template <typename T>
static ProductBufs<T> bufs_of(Work<T> &w) {
    return ProductBufs<T>{w.grid.p, w.bufA.p, w.bufB.p, w.trisrc.p, w.tripot.p};
}

template <typename T>
void matvec(sie_problem *p, Medium &md, sie_op op, int nrhs, const cx<T> *x, cx<T> *y, hipStream_t st) {
    const int64_t E = p->mesh.nrwg;
    if (op == SIE_OP_X) {
        for (int r = 0; r < nrhs; ++r)
            launch_x_apply<T>(E, p->d_xptr.p, p->d_xcol.p, xval_of<T>(p), x + r * E, y + r * E, st);
        return;
    }
    Grid &g = *md.grid;
    const GridView v = view_of(g);
    Work<T> &w = work_sel<T>(g);
    ensure_work(v, w, nrhs, E);
    // rows outside the medium's objects are zero
    if (v.rwg0 > 0 || v.rwg1 < E) launch_zero<T>((int64_t)nrhs * E, y, st);
    run_product<T>(p, v, media_of<T>(md, false), op, nrhs, x, y, bufs_of(w), w.xt.p, &p->timer, st);
}

template <typename T>
void group_product(sie_problem *p, Group &gr, sie_op op, bool scaled, int nrhs, const cx<T> *x, cx<T> *y,
                   hipStream_t st, const uint8_t *active) {
    const int64_t E = p->mesh.nrwg;
    if (gr.media.size() == 1) {
        Medium &md = p->ints[gr.media[0]];
        Grid &g = *md.grid;
        GridView v = view_of(g);
        if (nrhs == 1 && active) { v.active = active; v.obj0 = gr.media[0]; }
        Work<T> &w = work_sel<T>(g);
        ensure_work(v, w, nrhs, E);
        run_product<T>(p, v, media_of<T>(md, scaled), op, nrhs, x, y, bufs_of(w), w.xt.p, &p->timer, st, true);
        return;
    }
    Work<T> &w = work_sel<T>(gr);
    ensure_work(gr.view, w, nrhs, E);
    GridView v = gr.view;
    if (nrhs == 1 && active) { v.active = active; v.obj0 = gr.media[0]; }
    run_product<T>(p, v, media_of<T>(gr, scaled), op, nrhs, x, y, bufs_of(w), w.xt.p, &p->timer, st, true);
}

template <typename T>
void product_one(sie_problem *p, Medium &md, sie_op op, const cx<T> *x, cx<T> *y, const ProductBufs<T> &b,
                 StageTimer *tm, hipStream_t st) {
    const GridView v = view_of(*md.grid);
    const int64_t E = p->mesh.nrwg;
    if (v.rwg0 > 0 || v.rwg1 < E) launch_zero<T>(E, y, st);
    run_product<T>(p, v, media_of<T>(md, false), op, 1, x, y, b, nullptr, tm, st);
}

// Elements of cx<T> each buffer of one single-right-hand-side product needs
// (L-type, four fields; a K-type product uses the first three).
ProductSizes product_sizes(const Grid &g) {
    const int64_t F = 4;
    const int64_t ntg = (int64_t)g.tris.size();
    return {F * g.nlive(), F * g.nl[2] * g.nl[1] * g.m[0], F * g.nl[2] * g.m[1] * g.m[0], 4 * ntg, 5 * ntg};
}

template <typename T>
void stage_project(sie_problem *p, Medium &md, const cx<T> *x, cx<T> *grid, hipStream_t st) {
    Grid &g = *md.grid;
    const GridView v = view_of(g);
    Work<T> &w = work_of<T>(g);
    launch_tri_sources<T>(v, coef_v<T>(v), x, p->mesh.nrwg, 1, w.trisrc.p, st);
    launch_project<T>(v, mom_v<T>(v), w.trisrc.p, grid, 4, 1, st);
}

template <typename T>
void stage_convolve(sie_problem *p, Medium &md, sie_op op, int nf, const cx<T> *in, cx<T> *out, hipStream_t st) {
    Grid &g = *md.grid;
    Work<T> &w = work_of<T>(g);
    SIE_CHECK(!md.local, SIE_ESTATE, "the medium has no grid part (skin-depth cutoff or every pair near)");
    if (op == SIE_OP_K) SIE_CHECK(nf == 3, SIE_EINVAL, "the grad-G convolution takes 3 fields");
    else SIE_CHECK(nf >= 1 && nf <= 4, SIE_EINVAL, "nfields must be 1..4");
    fft_convolve<T>(view_of(g), spec_of<T>(md), 0, nf, 1, nf, op == SIE_OP_K ? 1 : 0, in, out, w.bufA.p, w.bufB.p,
                    st);
}

template <typename T>
void stage_interpolate(sie_problem *p, Medium &md, const cx<T> *grid, cx<T> *y, hipStream_t st) {
    Grid &g = *md.grid;
    const GridView v = view_of(g);
    Work<T> &w = work_of<T>(g);
    const int64_t E = p->mesh.nrwg;
    launch_interp<T>(v, mom_v<T>(v), grid, 4, 1, w.tripot.p, st);
    if (v.rwg0 > 0 || v.rwg1 < E) launch_zero<T>(E, y, st);
    const MediaView<T> mv = media_of<T>(md, false);
    launch_spmv_far<T>(v, coef_v<T>(v), w.tripot.p, mv.kscal, (const cx<T> *)nullptr, (const cx<T> *)nullptr,
                       (const cx<T> *)nullptr, y, true, st);
}

#define SIE_INST_MV(T)                                                                                     \
    template void matvec<T>(sie_problem *, Medium &, sie_op, int, const cx<T> *, cx<T> *, hipStream_t);    \
    template void group_product<T>(sie_problem *, Group &, sie_op, bool, int, const cx<T> *, cx<T> *,       \
                                   hipStream_t, const uint8_t *);                                          \
    template void product_one<T>(sie_problem *, Medium &, sie_op, const cx<T> *, cx<T> *, const ProductBufs<T> &, \
                                 StageTimer *, hipStream_t);                                               \
    template void stage_project<T>(sie_problem *, Medium &, const cx<T> *, cx<T> *, hipStream_t);          \
    template void stage_convolve<T>(sie_problem *, Medium &, sie_op, int, const cx<T> *, cx<T> *, hipStream_t); \
    template void stage_interpolate<T>(sie_problem *, Medium &, const cx<T> *, cx<T> *, hipStream_t);
SIE_INST_MV(float)
SIE_INST_MV(double)

// Constants of the augmented product and the factors of the constraint
// preconditioner's Schur complement (Sec. III-E).
static void aug_setup(sie_problem *p) {
    AugState &A = *p->aug;
    const Mesh &m = p->mesh;
    const int64_t E = m.nrwg, T = m.nt();
    const double k0 = p->ext.k.re;
    std::vector<double> sl(3 * T);
    for (int64_t i = 0; i < 3 * T; ++i) sl[i] = m.tri_sign[i] * m.len[m.tri_rwg[i]];
    A.sl.upload(sl);
    A.ks.upload(std::vector<c128>{c128(0.0, 2.0 / k0)});
    A.alpha.upload(std::vector<c128>{c128(0.0, k0)});
    const std::vector<c128> adiag = A.adiag.download(E), gself = A.gself.download(T);
    std::vector<c128> ad(E);
    for (int64_t n = 0; n < E; ++n) ad[n] = c128(0.0, k0) * adiag[n];
    A.ad.upload(ad);
    // S = j k0 I + Dv diag(ad)^-1 Dv^T diag(gself): the RWG function n couples
    // its two triangles
    std::vector<std::vector<std::pair<int32_t, c128>>> rows(T);
    for (int64_t t = 0; t < T; ++t) rows[t].push_back({(int32_t)t, c128(0.0, k0)});
    for (int64_t n = 0; n < E; ++n) {
        int32_t ts[2];
        double dv[2];
        for (int s = 0; s < 2; ++s) {
            ts[s] = m.tpm[2 * n + s];
            dv[s] = sl[3 * (int64_t)ts[s] + m.epm[2 * n + s]] / m.area[ts[s]];
        }
        const c128 w = cdiv(c128(1.0), ad[n]);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) rows[ts[a]].push_back({ts[b], (dv[a] * dv[b]) * (w * gself[ts[b]])});
    }
    std::vector<int64_t> rp(T + 1, 0);
    std::vector<int32_t> ci;
    std::vector<c128> val;
    for (int64_t t = 0; t < T; ++t) {
        auto &r = rows[t];
        std::sort(r.begin(), r.end(), [](const std::pair<int32_t, c128> &a, const std::pair<int32_t, c128> &b) {
            return a.first < b.first;
        });
        for (size_t i = 0; i < r.size(); ++i) {
            if (!ci.empty() && (int64_t)ci.size() > rp[t] && ci.back() == r[i].first) val.back() += r[i].second;
            else { ci.push_back(r[i].first); val.push_back(r[i].second); }
        }
        rp[t + 1] = (int64_t)ci.size();
        std::vector<std::pair<int32_t, c128>>().swap(r);
    }
    const auto t0 = std::chrono::steady_clock::now();
    lu_factor(A.lu, T, rp, ci, val, m.centroid, hipStreamPerThread);
    A.t_factor_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    setup_mark("augmented EFIE: Schur factors");
}

void aug_product(sie_problem *p, int nb, const c128 *x, c128 *y, hipStream_t st) {
    SIE_CHECK(p->aug, SIE_ESTATE, "problem not set up for the augmented EFIE");
    AugState &A = *p->aug;
    Medium &md = p->ext;
    Grid &g = *md.grid;
    const GridView v = view_of(g);
    const int64_t E = p->mesh.nrwg, T = p->mesh.nt(), ld = E + T;
    const double k0 = md.k.re;
    Work<double> &w = work_sel<double>(g);
    ensure_work(v, w, nb, E);
    const c128 *u = x;
    c128 *yu = y;
    if (nb > 1) {
        if (A.u.n < (size_t)nb * E) { A.u.alloc((size_t)nb * E); A.yu.alloc((size_t)nb * E); }
        SIE_HIP(hipMemcpy2DAsync(A.u.p, E * sizeof(c128), x, ld * sizeof(c128), E * sizeof(c128), nb,
                                 hipMemcpyDeviceToDevice, st));
        u = A.u.p;
        yu = A.yu.p;
    }
    StageTimer *tm = &p->timer;
    const bool all = tm->on == 1, csr = tm->on != 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (all) tm->begin(ST_PRODUCT, st, e0);
    const MediaView<double> mv = media_of<double>(md, false);
    if (mv.far) {
        // vector fields from u, the scalar field from the pulse charges
        if (all) tm->begin(ST_PROJECT, st, e1);
        launch_tri_sources<double>(v, v.coef64, u, E, nb, w.trisrc.p, st);
        launch_project<double>(v, v.mom64, w.trisrc.p, w.grid.p, 4, nb, st, x + E, ld, g.d_tris.p);
        if (all) { tm->end(ST_PROJECT, st, e1); tm->begin(ST_FFT, st, e1); }
        fft_convolve<double>(v, mv.spec, mv.spec_stride, 4 * nb, 1, 4 * nb, 0, w.grid.p, w.grid.p, w.bufA.p, w.bufB.p,
                             st);
        if (all) { tm->end(ST_FFT, st, e1); tm->begin(ST_INTERP, st, e1); }
        launch_interp<double>(v, v.mom64, w.grid.p, 4, nb, w.tripot.p, st);
        if (all) tm->end(ST_INTERP, st, e1);
    } else {
        launch_zero<double>((int64_t)nb * 5 * v.ntg, w.tripot.p, st);
    }
    // near part of the pulse potential joins the interpolated one per triangle
    launch_tri_near(v.ntg, g.d_pair_ptr.p, g.d_pair_s.p, g.d_tris.p, A.gam64.p, x + E, ld, nb, w.tripot.p, st);
    if (csr) tm->begin(ST_SPMV, st, e1);
    if (nb == 1)
        launch_spmv_far<double>(v, v.coef64, w.tripot.p, A.ks.p, A.alpha.p, A.nA64.p, u, yu, true, st);
    else
        launch_spmm_far<double>(v, E, nb, v.coef64, w.tripot.p, A.ks.p, A.alpha.p, A.nA64.p, u, w.xt.p, yu, st);
    if (csr) tm->end(ST_SPMV, st, e1, ST_SPMV64);
    launch_continuity(T, p->d_tri_rwg.p, A.sl.p, p->d_area.p, k0, u, E, x + E, ld, y + E, ld, nb, st);
    if (nb > 1)
        SIE_HIP(hipMemcpy2DAsync(y, ld * sizeof(c128), yu, E * sizeof(c128), E * sizeof(c128), nb,
                                 hipMemcpyDeviceToDevice, st));
    if (all) tm->end(ST_PRODUCT, st, e0);
}

void cp_apply(sie_problem *p, int nb, const c128 *x, c128 *y, hipStream_t st) {
    SIE_CHECK(p->aug, SIE_ESTATE, "problem not set up for the augmented EFIE");
    AugState &A = *p->aug;
    const int64_t E = p->mesh.nrwg, T = p->mesh.nt(), ld = E + T;
    const double k0 = p->ext.k.re;
    if (A.xnd.n < (size_t)nb * T) A.xnd.alloc((size_t)nb * T);
    launch_cp_pre(T, p->d_tri_rwg.p, A.sl.p, p->d_area.p, k0, A.ad.p, A.lu.iperm.p, x, ld, E, A.xnd.p, nb, st);
    lu_solve(A.lu, nb, A.xnd.p, st);
    launch_cp_post(E, T, p->d_tpm.p, p->d_epm.p, A.sl.p, p->d_area.p, A.gself.p, A.ad.p, A.lu.iperm.p, A.xnd.p, x,
                   ld, y, ld, nb, st);
}

// Host threads that build interior media concurrently.
constexpr int kBuildThreads = 8;

void problem_setup(sie_problem *p) {
    SIE_CHECK(!p->objs.empty(), SIE_ESTATE, "no objects");
    SIE_HIP(hipSetDevice(p->ctx->device));
    Mesh &m = p->mesh;
    m = Mesh();
    for (size_t i = 0; i < p->objs.size(); ++i) {
        const ObjIn &o = p->objs[i];
        const int32_t off = (int32_t)m.nv();
        m.xyz.insert(m.xyz.end(), o.xyz.begin(), o.xyz.end());
        for (int32_t v : o.tri) m.tri.push_back(v + off);
        for (size_t t = 0; t < o.tri.size() / 3; ++t) m.tri_obj.push_back((int32_t)i);
        for (int32_t v : o.tri) SIE_CHECK(v >= 0 && v < (int32_t)(o.xyz.size() / 3), SIE_EMESH, "vertex index out of range");
    }
    m.nobj = (int)p->objs.size();
    setup_mark("start");
    build_topology(m);
    setup_mark("topology");
    // quadrature defaults
    sie_quad_params &q = p->quad;
    if (q.touch_out <= 0) q.touch_out = 6;
    if (q.touch_in <= 0) q.touch_in = 6;
    if (q.close_out <= 0) q.close_out = 5;
    if (q.close_in <= 0) q.close_in = 5;
    if (q.far_out <= 0) q.far_out = 3;   // row-level error vs converged rules ~1e-5 on the copper bar
    if (q.far_in <= 0) q.far_in = 3;
    SIE_CHECK(q.touch_out <= 16 && q.touch_in <= 16 && q.close_out <= 16 && q.close_in <= 16 && q.far_out <= 16 &&
                  q.far_in <= 16, SIE_EINVAL, "quadrature order above 16");
    // device mesh arrays
    p->d_xyz.upload(m.xyz);
    p->d_centroid.upload(m.centroid);
    p->d_tri.upload(m.tri);
    p->d_tri_rwg.upload(m.tri_rwg);
    p->d_tpm.upload(m.tpm);
    p->d_epm.upload(m.epm);
    p->d_len.upload(m.len);
    p->d_area.upload(m.area);
    p->d_tri_sign.upload(m.tri_sign);
    build_x(p);
    setup_mark("mesh upload, X");
    // media
    p->w = 2.0 * 3.14159265358979323846 * p->freq;
    const double w = p->w;
    p->ext = Medium();
    p->ext.id = -1;
    p->ext.k = wavenumber(w, p->bg_eps_r, p->bg_mu_r, 0.0);
    p->ext.eps = c128(EPS0 * p->bg_eps_r);
    p->ext.mu = c128(MU0 * p->bg_mu_r);
    p->ints.clear();
    p->ints.resize(m.nobj);
    for (int i = 0; i < m.nobj; ++i) {
        Medium &md = p->ints[i];
        md.id = i;
        md.k = wavenumber(w, p->objs[i].eps_r, p->objs[i].mu_r, p->objs[i].sigma);
        md.eps = c128(EPS0 * p->objs[i].eps_r, -p->objs[i].sigma / w);
        md.mu = c128(MU0 * p->objs[i].mu_r);
    }
    // per-triangle bounding radius about the centroid, for the skin-depth
    // cutoff of the near lists
    p->rho = bounding_radii(m);
    p->d_rho.upload(p->rho);
    // cutoff distance of an interior medium (0: none): the chosen number of
    // skin depths, delta = -1 / Im k_i (Sec. V)
    auto cutoff_of = [&](int i) {
        const double ki = p->ints[i].k.im;
        return p->cutoff_factor > 0.0 && ki < 0.0 ? p->cutoff_factor / -ki : 0.0;
    };
    auto rho_max = [&](int obj) {
        double r = 0.0;
        for (int64_t t = 0; t < m.nt(); ++t)
            if (obj < 0 || m.tri_obj[t] == obj) r = std::max(r, p->rho[t]);
        return r;
    };
    // the cutoff removes the grid part when every far pair (centroids at
    // least R h apart along an axis) lies beyond it
    auto cut_local = [&](int i, double h, int R) {
        const double dc = cutoff_of(i);
        return dc > 0.0 && dc <= R * h - 2.0 * rho_max(i);
    };
    // grids
    p->grids.clear();
    auto shares = [&](int i) {
        const GridReq &rq = p->obj_req[i];
        return rq.share == 1 || (rq.share == -1 && m.nobj == 1);
    };
    std::vector<char> unshare(m.nobj, 0);   // local under the cutoff: a near list of its own
    {
        auto g = std::make_unique<Grid>();
        for (int64_t t = 0; t < m.nt(); ++t) g->tris.push_back((int32_t)t);
        for (int i = 0; i < m.nobj; ++i) g->objs.push_back(i);
        std::vector<MediumProps> users{{p->bg_eps_r, p->bg_mu_r, 0.0}};
        for (int i = 0; i < m.nobj; ++i)
            if (shares(i)) users.push_back({p->objs[i].eps_r, p->objs[i].mu_r, p->objs[i].sigma});
        build_grid_geometry(p, *g, p->ext_req, users);
        for (int i = 0; i < m.nobj; ++i)
            if (shares(i) && cut_local(i, g->h, p->obj_req[i].R)) unshare[i] = 1;
        build_grid(p, *g);
        setup_mark("exterior grid");
        p->ext.grid = g.get();
        p->ext.local = g->all_near;
        p->grids.push_back(std::move(g));
    }
    for (int i = 0; i < m.nobj; ++i) {
        GridReq rq = p->obj_req[i];
        Medium &md = p->ints[i];
        if (shares(i) && !unshare[i]) {
            SIE_CHECK(m.nobj == 1, SIE_EINVAL, "interior grids can share the exterior grid only for one object");
            md.grid = p->ext.grid;
            md.local = p->ext.grid->all_near;
            continue;
        }
        auto g = std::make_unique<Grid>();
        for (int64_t t = 0; t < m.nt(); ++t)
            if (m.tri_obj[t] == i) g->tris.push_back((int32_t)t);
        g->objs.push_back(i);
        if (unshare[i]) {
            // the exterior grid's geometry, the medium's own (cut) near list
            const Grid &ge = *p->ext.grid;
            rq.h = ge.h;
            rq.n = ge.n[0];
            rq.has_origin = true;
            for (int c = 0; c < 3; ++c) rq.origin[c] = ge.origin[c];
        }
        build_grid_geometry(p, *g, rq, {{p->objs[i].eps_r, p->objs[i].mu_r, p->objs[i].sigma}});
        const bool cut = cut_local(i, g->h, g->near_radius);
        if (cut) g->cutoff = cutoff_of(i);
        md.local = cut;   // or'ed with the grid's all-near flag below
        md.grid = g.get();
        p->grids.push_back(std::move(g));
    }
    // the interior grids (stencils, near lists, moments: host work with a
    // few launches each) from several host threads, each on its own default
    // stream
    {
        const int ng = (int)p->grids.size() - 1;   // [0]: the exterior grid, built above
        const int nthr = std::max(1, std::min(kBuildThreads, ng));
        std::atomic<int> next{0};
        std::exception_ptr err;
        std::mutex emu;
        auto work = [&]() {
            try {
                SIE_HIP(hipSetDevice(p->ctx->device));
                for (int k = next.fetch_add(1); k < ng; k = next.fetch_add(1)) build_grid(p, *p->grids[1 + k]);
            } catch (...) {
                std::lock_guard<std::mutex> lk(emu);
                if (!err) err = std::current_exception();
                next.store(ng);
            }
        };
        std::vector<std::thread> th;
        for (int t = 1; t < nthr; ++t) th.emplace_back(work);
        work();
        for (auto &t : th) t.join();
        if (err) std::rethrow_exception(err);
    }
    for (int i = 0; i < m.nobj; ++i)
        if (p->ints[i].grid != p->ext.grid) p->ints[i].local = p->ints[i].local || p->ints[i].grid->all_near;
    setup_mark("interior grids");
    form_groups(p);
    if (p->aug_mode == 1) p->aug.reset(new AugState);
    else p->aug.reset();
    // the exterior medium first (its fill fills the device by itself); then
    // the interior media, independent of each other, from several host
    // threads, each on a stream of its own, so that their fills (many small
    // launches per medium) overlap on the device, and beside them the host
    // factorisation of the augmented EFIE's Schur complement on a thread of
    // its own.  (Building the exterior medium beside the interior ones was
    // slower: the factorisation, which needs the exterior values, then
    // started later.)
    for (auto &g : p->grids) pair_kinds(p, *g, 0);
    setup_mark("pair kinds");
    build_medium(p, p->ext, 0);
    SIE_HIP(hipDeviceSynchronize());
    std::thread aug_thread;
    std::exception_ptr aug_err;
    if (p->aug)
        aug_thread = std::thread([&]() {
            try {
                SIE_HIP(hipSetDevice(p->ctx->device));
                aug_setup(p);
            } catch (...) {
                aug_err = std::current_exception();
            }
        });
    struct JoinAug {
        std::thread &t;
        ~JoinAug() { if (t.joinable()) t.join(); }
    } join_aug{aug_thread};
    {
        const int nthr = std::max(1, std::min(kBuildThreads, m.nobj));
        std::atomic<int> next{0};
        std::exception_ptr err;
        std::mutex emu;
        auto work = [&]() {
            hipStream_t st = nullptr;
            try {
                SIE_HIP(hipSetDevice(p->ctx->device));
                SIE_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
                for (int i = next.fetch_add(1); i < m.nobj; i = next.fetch_add(1)) build_medium(p, p->ints[i], st);
                SIE_HIP(hipStreamSynchronize(st));
            } catch (...) {
                std::lock_guard<std::mutex> lk(emu);
                if (!err) err = std::current_exception();
                next.store(m.nobj);
            }
            if (st) {
                (void)hipStreamSynchronize(st);
                (void)hipStreamDestroy(st);
            }
        };
        std::vector<std::thread> th;
        for (int t = 1; t < nthr; ++t) th.emplace_back(work);
        work();
        for (auto &t : th) t.join();
        if (aug_thread.joinable()) aug_thread.join();
        if (err) std::rethrow_exception(err);
        if (aug_err) std::rethrow_exception(aug_err);
    }
    finalize_groups(p);
    setup_mark("groups");
    p->is_setup = true;
}

}  // namespace sie

sie::Medium &sie_problem::medium(int id) {
    if (id == -1) return ext;
    SIE_CHECK(id >= 0 && id < (int)ints.size(), SIE_EINVAL, "medium index out of range");
    return ints[id];
}
const sie::Medium &sie_problem::medium(int id) const {
    if (id == -1) return ext;
    SIE_CHECK(id >= 0 && id < (int)ints.size(), SIE_EINVAL, "medium index out of range");
    return ints[id];
}
