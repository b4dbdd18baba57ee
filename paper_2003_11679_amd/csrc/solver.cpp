// GIBC solve with AIM-accelerated nested interior solves (Sec. III-C/D).
//
// Unknowns u = n x H, v = n x E (RWG coefficients).  Block equations (derived
// from the equivalence principle with e^{+j w t}; the printed half-term signs
// coincide with these for the source-gradient K and n0 x H = -u):
//   exterior:  j w mu0 L0 u - (K0 - X/2) v = e                    (eq. EFIE01dis)
//   interior:  -j w eps~_i L_i v - (K_i + X/2) u = 0              (eq. MFIE1dis)
// GIBC elimination v = Z u (eq. GIBCdef) gives the outer system
//   [j w mu0 L0 - (K0 - X/2) Z] u = e                             (eq. GIBCsys)
// whose product with u needs a = (K_i + X/2) u (eq. nest02) and a nested
// iterative solve of -j w eps~_i L_i (Z u) = a (eq. nest2), all products
// AIM-accelerated.  GMRES (right-preconditioned, restarted, classical
// Gram-Schmidt applied twice with FP64 dot products, Givens rotations and the
// triangular solve in FP64 on the host) drives both levels.
//
// Precision: SIE_FP64 runs every stage in complex128.  SIE_FP32 runs the
// interior work (K_i products and the nested L_i solves, which dominate the
// operator count) in complex64 inside FP64 iterative refinement: the residual
// of the block equations above (no nested solve needed) is formed in FP64 and
// the correction solved with FP64 exterior products and outer Krylov vectors
// (at low frequency the k0 operator's vector potential is ~(k0 h)^2 below its
// scalar potential and does not survive FP32) around FP32 nested solves.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>

#include "problem.h"
#include "solve_kernels.h"

namespace sie {

static const double PI = 3.14159265358979323846;

// ---------------------------------------------------------------- GMRES
template <typename T>
struct Gmres {
    int64_t n = 0;
    int m = 0;
    DBuf<cx<T>> V, Zb, w, r;
    DBuf<c128> part, hd;
    using Op = std::function<void(const cx<T> *, cx<T> *)>;

    void init(int64_t n_, int m_) {
        if (n == n_ && m == m_) return;
        n = n_; m = m_;
        V.alloc((size_t)(m + 1) * n);
        Zb.alloc((size_t)m * n);
        w.alloc(n);
        r.alloc(n);
        part.alloc((size_t)(m + 1) * DOT_BLOCKS);
        hd.alloc(m + 1);
    }

    std::vector<c128> dots(int J, const cx<T> *Vp, const cx<T> *x, hipStream_t st) {
        launch_dots<T>(n, J, Vp, n, x, part.p, DOT_BLOCKS, hd.p, st);
        std::vector<c128> h(J);
        SIE_HIP(hipMemcpyAsync(h.data(), hd.p, J * sizeof(c128), hipMemcpyDeviceToHost, st));
        SIE_HIP(hipStreamSynchronize(st));
        return h;
    }
    double norm(const cx<T> *x, hipStream_t st) { return std::sqrt(std::max(0.0, dots(1, x, x, st)[0].re)); }

    // Solves A x = b (x holds the initial guess).  Returns iterations; *relres
    // receives the final relative residual estimate.
    const char *tag = "gmres";
    // Stagnation window: a cycle that gains under 1 % over this many
    // iterations hands back to the caller (the precision floor of an FP32
    // correction); 0 disables it.
    int stag_window = 25;
    int solve(const Op &A, const Op &M, const cx<T> *b, cx<T> *x, double tol, int maxit, double *relres,
              hipStream_t st, int *napply = nullptr) {
        static const bool trace = std::getenv("SIE_TRACE") != nullptr;
        const double bn = norm(b, st);
        if (bn == 0.0) {
            SIE_HIP(hipMemsetAsync(x, 0, n * sizeof(cx<T>), st));
            if (relres) *relres = 0.0;
            return 0;
        }
        int it = 0;
        double res = 1.0;
        bool stagnated = false;
        std::vector<double> hist;
        std::vector<c128> H((size_t)(m + 1) * m), g(m + 1), sn(m);
        std::vector<double> cs(m);
        while (true) {
            // r = b - A x
            A(x, r.p);
            if (napply) ++*napply;
            launch_axpby<T>(n, c128(1.0), b, c128(-1.0), r.p, st);
            const double beta = norm(r.p, st);
            res = beta / bn;
            if (trace) std::fprintf(stderr, "[%s] restart at it %d true res %.3e\n", tag, it, res);
            if (res <= tol || it >= maxit) break;
            launch_scale_into<T>(n, c128(1.0 / beta), r.p, V.p, st);
            std::fill(g.begin(), g.end(), c128());
            g[0] = c128(beta);
            int j = 0;
            for (; j < m && it < maxit; ++j, ++it) {
                cx<T> *vj = V.p + (size_t)j * n, *zj = Zb.p + (size_t)j * n;
                M(vj, zj);
                A(zj, w.p);
                if (napply) ++*napply;
                std::vector<c128> h = dots(j + 1, V.p, w.p, st);
                launch_gemv_sub<T>(n, j + 1, V.p, n, hd.p, w.p, st);
                std::vector<c128> h2 = dots(j + 1, V.p, w.p, st);
                launch_gemv_sub<T>(n, j + 1, V.p, n, hd.p, w.p, st);
                for (int i = 0; i <= j; ++i) h[i] += h2[i];
                const double hn = norm(w.p, st);
                // Givens
                for (int i = 0; i < j; ++i) {
                    const c128 a = h[i], bb = h[i + 1];
                    h[i] = cs[i] * a + sn[i] * bb;
                    h[i + 1] = cs[i] * bb - conj(sn[i]) * a;
                }
                {
                    const c128 a = h[j];
                    const double aa = std::sqrt(norm2(a));
                    const double t = std::hypot(aa, hn);
                    if (aa == 0.0) { cs[j] = 0.0; sn[j] = c128(1.0); h[j] = c128(t); }
                    else {
                        const c128 ph = (1.0 / aa) * a;
                        cs[j] = aa / t;
                        sn[j] = (hn / t) * ph;
                        h[j] = t * ph;
                    }
                    g[j + 1] = -(conj(sn[j]) * g[j]);
                    g[j] = cs[j] * g[j];
                }
                for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i];
                res = std::sqrt(norm2(g[j + 1])) / bn;
                if (trace) std::fprintf(stderr, "[%s] it %d res %.3e\n", tag, it + 1, res);
                hist.push_back(res);
                if (stag_window > 0 && (int)hist.size() > stag_window &&
                    res > 0.99 * hist[hist.size() - 1 - stag_window])
                    stagnated = true;
                if (hn > 0.0 && hn > 1e-300) launch_scale_into<T>(n, c128(1.0 / hn), w.p, V.p + (size_t)(j + 1) * n, st);
                if (res <= tol || hn <= 1e-14 * beta || stagnated) { ++j; ++it; break; }
            }
            // y = H^-1 g ; x += Zb y
            const int k = j;
            std::vector<c128> y(k);
            for (int i = k - 1; i >= 0; --i) {
                c128 s = g[i];
                for (int l = i + 1; l < k; ++l) s -= H[(size_t)i * m + l] * y[l];
                y[i] = cdiv(s, H[(size_t)i * m + i]);
            }
            SIE_HIP(hipMemcpyAsync(hd.p, y.data(), k * sizeof(c128), hipMemcpyHostToDevice, st));
            launch_gemv_add<T>(n, k, Zb.p, n, hd.p, x, st);
            if (stagnated) {
                A(x, r.p);
                launch_axpby<T>(n, c128(1.0), b, c128(-1.0), r.p, st);
                res = norm(r.p, st) / bn;
                break;
            }
        }
        if (relres) *relres = res;
        return it;
    }
};

// ---------------------------------------------------------------- preconditioner
struct BlockJacobi {
    int B = 32;
    int nb = 0;
    DBuf<int32_t> perm;
    DBuf<c128> inv64;
    DBuf<c64> inv32;
};

// Blocks of B RWG functions in the spatial (cell-sorted) order of the grid,
// for the RWG rows [r0, r1) of that grid; entries from the direct near-region
// L of the medium times `scale`.
static void bj_add(sie_problem *p, BlockJacobi &bj, std::vector<int32_t> &perm_all, std::vector<int> &blk_medium,
                   Medium &md, int64_t r0, int64_t r1) {
    Grid &g = *md.grid;
    std::vector<std::pair<int32_t, int32_t>> key;
    for (int64_t r = r0; r < r1; ++r) key.push_back({g.glob2loc[p->mesh.tpm[2 * r]], (int32_t)r});
    std::sort(key.begin(), key.end());
    const int B = bj.B;
    const int nb = (int)((key.size() + B - 1) / B);
    for (int b = 0; b < nb; ++b) {
        for (int i = 0; i < B; ++i) {
            const size_t k = (size_t)b * B + i;
            perm_all.push_back(k < key.size() ? key[k].second : -1);
        }
        blk_medium.push_back(md.id);
    }
}

static void bj_build(sie_problem *p, BlockJacobi &bj, const std::vector<Medium *> &media,
                     const std::vector<std::pair<int64_t, int64_t>> &ranges, const std::vector<c128> &scales) {
    std::vector<int32_t> perm;
    std::vector<int> bm;
    std::vector<int> first;
    for (size_t i = 0; i < media.size(); ++i) {
        first.push_back((int)(perm.size() / bj.B));
        bj_add(p, bj, perm, bm, *media[i], ranges[i].first, ranges[i].second);
    }
    first.push_back((int)(perm.size() / bj.B));
    bj.nb = (int)(perm.size() / bj.B);
    bj.perm.upload(perm);
    bj.inv64.alloc((size_t)bj.nb * bj.B * bj.B);
    bj.inv32.alloc((size_t)bj.nb * bj.B * bj.B);
    for (size_t i = 0; i < media.size(); ++i) {
        Grid &g = *media[i]->grid;
        const int nbi = first[i + 1] - first[i];
        const size_t o = (size_t)first[i] * bj.B;
        launch_bj_setup(nbi, bj.B, bj.perm.p + o, g.rwg0, g.d_row_ptr.p, g.d_cols.p, media[i]->d_nLd64.p, scales[i],
                        bj.inv64.p + o * bj.B, bj.inv32.p + o * bj.B, 0);
    }
    SIE_HIP(hipDeviceSynchronize());
}

template <typename T> static const cx<T> *bj_inv(const BlockJacobi &bj);
template <> const c128 *bj_inv<double>(const BlockJacobi &bj) { return bj.inv64.p; }
template <> const c64 *bj_inv<float>(const BlockJacobi &bj) { return bj.inv32.p; }

// ---------------------------------------------------------------- solve state
struct SolveState {
    int nrhs = 0;
    int64_t E = 0;
    DBuf<c128> e, u, v;            // [nrhs][E]
    bool solved = false;
    BlockJacobi pin, pout;         // inner (interior L-hat) and outer (exterior) preconditioners
    bool pre_built = false;
    Gmres<double> go64, gi64;
    Gmres<float> go32, gi32;
    DBuf<c128> t64[6];
    DBuf<c64> t32[6];
    int matvecs = 0, inner_iters = 0, inner_max = 0;
};

void solver_destroy(SolveState *s) { delete s; }

template <typename T> static DBuf<cx<T>> *tmp_of(SolveState &s);
template <> DBuf<c128> *tmp_of<double>(SolveState &s) { return s.t64; }
template <> DBuf<c64> *tmp_of<float>(SolveState &s) { return s.t32; }
template <typename T> static Gmres<T> &outer_of(SolveState &s);
template <> Gmres<double> &outer_of<double>(SolveState &s) { return s.go64; }
template <> Gmres<float> &outer_of<float>(SolveState &s) { return s.go32; }
template <typename T> static Gmres<T> &inner_of(SolveState &s);
template <> Gmres<double> &inner_of<double>(SolveState &s) { return s.gi64; }
template <> Gmres<float> &inner_of<float>(SolveState &s) { return s.gi32; }

template <typename T>
struct Ops {
    sie_problem *p;
    SolveState &s;
    hipStream_t st;
    int64_t E;
    cx<T> *t[6];
    double inner_tol;
    int inner_max_iter;
    int restart;

    Ops(sie_problem *p_, SolveState &s_, hipStream_t st_, double itol, int imax, int rs)
        : p(p_), s(s_), st(st_), E(p_->mesh.nrwg), inner_tol(itol), inner_max_iter(imax), restart(rs) {
        DBuf<cx<T>> *tb = tmp_of<T>(s);
        for (int i = 0; i < 6; ++i) {
            if (tb[i].n != (size_t)E) tb[i].alloc(E);
            t[i] = tb[i].p;
        }
        inner_of<T>(s).init(E, restart);
        outer_of<T>(s).init(E, restart);
        inner_of<T>(s).tag = sizeof(T) == 8 ? "inner64" : "inner32";
        outer_of<T>(s).tag = sizeof(T) == 8 ? "outer64" : "outer32";
    }

    void mv(Medium &md, sie_op op, const cx<T> *x, cx<T> *y) {
        matvec<T>(p, md, op, 1, x, y, st);
        if (op != SIE_OP_X) s.matvecs++;
    }
    // y = sum_i (-j w eps~_i) L_i x   (block diagonal over objects)
    void Lhat(const cx<T> *x, cx<T> *y) {
        for (size_t i = 0; i < p->ints.size(); ++i) {
            Medium &md = p->ints[i];
            const c128 sc = c128(0.0, -p->w) * md.eps;
            if (i == 0) {
                mv(md, SIE_OP_L, x, y);
                launch_scale_into<T>(E, sc, y, y, st);
            } else {
                mv(md, SIE_OP_L, x, t[5]);
                launch_axpby<T>(E, sc, t[5], c128(1.0), y, st);
            }
        }
    }
    // y = sum_i K_i x + sgn X x / 2
    void KpX(bool interior, double sgn, const cx<T> *x, cx<T> *y) {
        if (interior) {
            for (size_t i = 0; i < p->ints.size(); ++i) {
                if (i == 0) mv(p->ints[i], SIE_OP_K, x, y);
                else {
                    mv(p->ints[i], SIE_OP_K, x, t[5]);
                    launch_axpby<T>(E, c128(1.0), t[5], c128(1.0), y, st);
                }
            }
        } else {
            mv(p->ext, SIE_OP_K, x, y);
        }
        mv(p->ext, SIE_OP_X, x, t[4]);
        launch_axpby<T>(E, c128(0.5 * sgn), t[4], c128(1.0), y, st);
    }
    bool use_bj_in = false, use_bj_out = false;
    void prec_inner(const cx<T> *x, cx<T> *y) {
        if (use_bj_in) launch_bj_apply<T>(s.pin.nb, s.pin.B, s.pin.perm.p, bj_inv<T>(s.pin), x, y, st);
        else SIE_HIP(hipMemcpyAsync(y, x, E * sizeof(cx<T>), hipMemcpyDeviceToDevice, st));
    }
    void prec_outer(const cx<T> *x, cx<T> *y) {
        if (use_bj_out) launch_bj_apply<T>(s.pout.nb, s.pout.B, s.pout.perm.p, bj_inv<T>(s.pout), x, y, st);
        else SIE_HIP(hipMemcpyAsync(y, x, E * sizeof(cx<T>), hipMemcpyDeviceToDevice, st));
    }
    // Mixed precision: an FP64 operator set may delegate the interior work
    // (K_i products and the nested L_i solves) to an FP32 one.
    Ops<float> *lo = nullptr;
    // v = Lhat^-1 a (nested solve, eq. nest2)
    void inner_solve(const cx<T> *a, cx<T> *v);
    void inner_solve_native(const cx<T> *a, cx<T> *v) {
        SIE_HIP(hipMemsetAsync(v, 0, E * sizeof(cx<T>), st));
        double rr;
        int it = inner_of<T>(s).solve([&](const cx<T> *x, cx<T> *y) { Lhat(x, y); },
                                      [&](const cx<T> *x, cx<T> *y) { prec_inner(x, y); }, a, v, inner_tol,
                                      inner_max_iter, &rr, st);
        s.inner_iters += it;
        s.inner_max = std::max(s.inner_max, it);
    }
    // v = Z u = Lhat^-1 (K_i + X/2) u
    void Z(const cx<T> *u, cx<T> *v);
    void Z_native(const cx<T> *u, cx<T> *v) {
        KpX(true, +1.0, u, t[0]);
        inner_solve_native(t[0], v);
    }
    // y = j w mu0 L0 u - (K0 - X/2) Z u
    void gibc(const cx<T> *u, cx<T> *y) {
        Z(u, t[1]);
        KpX(false, -1.0, t[1], t[2]);
        mv(p->ext, SIE_OP_L, u, y);
        launch_axpby<T>(E, c128(-1.0), t[2], c128(0.0, p->w) * p->ext.mu, y, st);
    }
};

template <> void Ops<float>::inner_solve(const c64 *a, c64 *v) { inner_solve_native(a, v); }
template <> void Ops<float>::Z(const c64 *u, c64 *v) { Z_native(u, v); }
template <> void Ops<double>::inner_solve(const c128 *a, c128 *v) {
    if (!lo) { inner_solve_native(a, v); return; }
    c64 *a32 = lo->t[1], *v32 = lo->t[2];
    launch_convert<double, float>(a, a32, E, st);
    lo->inner_solve_native(a32, v32);
    launch_convert<float, double>(v32, v, E, st);
}
template <> void Ops<double>::Z(const c128 *u, c128 *v) {
    if (!lo) { Z_native(u, v); return; }
    c64 *u32 = lo->t[1], *v32 = lo->t[2];
    launch_convert<double, float>(u, u32, E, st);
    lo->Z_native(u32, v32);
    launch_convert<float, double>(v32, v, E, st);
}

// FP64 residual of the block equations: r1 = e - [j w mu0 L0 u - (K0 - X/2) v],
// r2 = -[-(K_i + X/2) u + Lhat v]; returns ||r|| / ||e||.
static double block_residual(Ops<double> &o, const c128 *e, const c128 *u, const c128 *v, c128 *r1, c128 *r2) {
    const int64_t E = o.E;
    hipStream_t st = o.st;
    // r1
    o.KpX(false, -1.0, v, o.t[2]);
    o.mv(o.p->ext, SIE_OP_L, u, r1);
    launch_axpby<double>(E, c128(-1.0), o.t[2], c128(0.0, o.p->w) * o.p->ext.mu, r1, st);   // A1 x
    launch_axpby<double>(E, c128(1.0), e, c128(-1.0), r1, st);                              // e - A1 x
    // r2 = (K_i + X/2) u - Lhat v
    o.KpX(true, +1.0, u, r2);
    o.Lhat(v, o.t[3]);
    launch_axpby<double>(E, c128(-1.0), o.t[3], c128(1.0), r2, st);
    Gmres<double> &g = o.s.go64;
    const double n1 = g.norm(r1, st), n2 = g.norm(r2, st), ne = g.norm(e, st);
    return std::sqrt(n1 * n1 + n2 * n2) / ne;
}

static void build_preconditioners(sie_problem *p, SolveState &s) {
    if (s.pre_built) return;
    std::vector<Medium *> mi;
    std::vector<std::pair<int64_t, int64_t>> ri;
    std::vector<c128> si;
    for (size_t i = 0; i < p->ints.size(); ++i) {
        mi.push_back(&p->ints[i]);
        ri.push_back({p->mesh.obj_rwg0[i], p->mesh.obj_rwg0[i + 1]});
        si.push_back(c128(0.0, -p->w) * p->ints[i].eps);
    }
    bj_build(p, s.pin, mi, ri, si);
    bj_build(p, s.pout, {&p->ext}, {{0, p->mesh.nrwg}}, {c128(0.0, p->w) * p->ext.mu});
    s.pre_built = true;
}

static void solve_all(sie_problem *p, sie_precision prec, const sie_solver_opts &o, sie_report *rep) {
    SolveState &s = *p->solve;
    const int64_t E = s.E;
    hipStream_t st = 0;
    if (o.precond != 0) build_preconditioners(p, s);
    s.matvecs = s.inner_iters = s.inner_max = 0;
    int outer_total = 0, sweeps_total = 0;
    double worst = 0.0;
    bool all_conv = true;
    const auto t0 = std::chrono::steady_clock::now();
    Ops<double> o64(p, s, st, o.inner_tol, o.inner_max_iter, o.restart);
    o64.use_bj_in = (o.precond & 1) != 0;
    o64.use_bj_out = (o.precond & 2) != 0;
    for (int r = 0; r < s.nrhs; ++r) {
        c128 *e = s.e.p + r * E, *u = s.u.p + r * E, *v = s.v.p + r * E;
        double res = 1.0;
        // Refinement sweeps: residual of the block equations in FP64, correction
        // from the nested GIBC solve.  SIE_FP32 delegates the interior work to
        // complex64 (the exterior products and outer Krylov vectors stay FP64:
        // at low frequency the k0 operator's vector potential is ~(k0 h)^2
        // below its scalar potential and does not survive FP32).
        std::unique_ptr<Ops<float>> o32;
        if (prec == SIE_FP32) {
            o32.reset(new Ops<float>(p, s, st, std::max(o.inner_tol, 1e-5), o.inner_max_iter, o.restart));
            o32->use_bj_in = o64.use_bj_in;
            o32->use_bj_out = o64.use_bj_out;
            o64.lo = o32.get();
        }
        SIE_HIP(hipMemsetAsync(u, 0, E * sizeof(c128), st));
        SIE_HIP(hipMemsetAsync(v, 0, E * sizeof(c128), st));
        DBuf<c128> r1(E), r2(E), du(E), dv(E), sv(E);
        double prev = 2.0;
        for (int sw = 0; sw <= o.max_refine; ++sw) {
            res = block_residual(o64, e, u, v, r1.p, r2.p);
            // stop at the tolerance, at the sweep cap, or when a sweep no longer
            // halves the residual (the outer system itself has stagnated)
            if (res <= o.tol || sw == o.max_refine || res > 0.5 * prev) break;
            prev = res;
            ++sweeps_total;
            // s = Lhat^-1 r2 ; r1' = r1 + (K0 - X/2) s
            o64.inner_solve(r2.p, sv.p);
            o64.KpX(false, -1.0, sv.p, o64.t[3]);
            launch_axpby<double>(E, c128(1.0), o64.t[3], c128(1.0), r1.p, st);
            SIE_HIP(hipMemsetAsync(du.p, 0, E * sizeof(c128), st));
            // FP64: run through the plateaus of the low-frequency EFIE; FP32:
            // hand back when a correction stalls for longer than a plateau
            s.go64.stag_window = prec == SIE_FP32 ? 100 : 0;
            // relative tolerance of the correction solve: what is left to the
            // target, but at most three digits per FP32 sweep (its interior
            // products carry FP32 rounding)
            const double need = o.tol / res;
            const double sweep_tol = prec == SIE_FP32 ? std::max(need, 1e-3) : need;
            double rr;
            outer_total += s.go64.solve([&](const c128 *x, c128 *y) { o64.gibc(x, y); },
                                        [&](const c128 *x, c128 *y) { o64.prec_outer(x, y); }, r1.p, du.p,
                                        sweep_tol, o.max_iter, &rr, st);
            // dv = Lhat^-1 (r2 + (K_i + X/2) du)
            o64.KpX(true, +1.0, du.p, o64.t[3]);
            launch_axpby<double>(E, c128(1.0), r2.p, c128(1.0), o64.t[3], st);
            o64.inner_solve(o64.t[3], dv.p);
            launch_axpby<double>(E, c128(1.0), du.p, c128(1.0), u, st);
            launch_axpby<double>(E, c128(1.0), dv.p, c128(1.0), v, st);
        }
        o64.lo = nullptr;
        worst = std::max(worst, res);
        if (!(res <= o.tol)) all_conv = false;
    }
    SIE_HIP(hipStreamSynchronize(st));
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    s.solved = true;
    if (rep) {
        rep->outer_iters = outer_total;
        rep->inner_iters = s.inner_iters;
        rep->inner_iters_max = s.inner_max;
        rep->refine_sweeps = sweeps_total;
        rep->matvecs = s.matvecs;
        rep->residual = worst;
        rep->t_solve_s = dt;
    }
    if (!all_conv) throw Error(SIE_ENOCONV, "residual " + std::to_string(worst) + " above tolerance");
}

}  // namespace sie

namespace sie {
void planewaves_entry(sie_problem *p, int32_t nrhs, const double *khat, const sie_c128 *e0) {
    SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
    SIE_CHECK(nrhs >= 1 && khat && e0, SIE_EINVAL, "bad plane waves");
    if (!p->solve) p->solve = new SolveState;
    SolveState &s = *p->solve;
    const int64_t E = p->mesh.nrwg;
    s.nrhs = nrhs;
    s.E = E;
    s.e.alloc((size_t)nrhs * E);
    s.u.alloc((size_t)nrhs * E);
    s.v.alloc((size_t)nrhs * E);
    s.solved = false;
    Rule rq = rule_collapsed(6);
    std::vector<double> packed(4 * rq.size());
    for (int q = 0; q < rq.size(); ++q) {
        for (int c = 0; c < 3; ++c) packed[4 * q + c] = rq.bary[3 * q + c];
        packed[4 * q + 3] = rq.w[q];
    }
    DBuf<double> d_rule;
    d_rule.upload(packed);
    p->khat.assign(khat, khat + 3 * nrhs);
    p->e0.resize(3 * nrhs);
    for (int r = 0; r < nrhs; ++r) {
        const double *k = khat + 3 * r;
        const double kn = std::sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
        SIE_CHECK(kn > 0.0, SIE_EINVAL, "zero propagation direction");
        const double kh[3] = {k[0] / kn, k[1] / kn, k[2] / kn};
        c128 ee[3];
        for (int c = 0; c < 3; ++c) { ee[c] = c128(e0[3 * r + c].re, e0[3 * r + c].im); p->e0[3 * r + c] = ee[c]; }
        launch_excitation(p, d_rule.p, rq.size(), p->ext.k.re, kh, ee, s.e.p + r * E, 0);
    }
    SIE_HIP(hipDeviceSynchronize());
}
}  // namespace sie

namespace sie {
void solve_entry(sie_problem *p, sie_precision prec, const sie_solver_opts *opts, sie_report *rep) {
    SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
    SIE_CHECK(p->solve && p->solve->nrhs > 0, SIE_ESTATE, "no plane waves set");
    SIE_CHECK(prec == SIE_FP64 || prec == SIE_FP32, SIE_EINVAL, "unknown precision");
    sie_solver_opts o{1e-6, 1e-8, 100, 800, 800, 10, 0};
    if (opts) {
        if (opts->tol > 0) o.tol = opts->tol;
        if (opts->inner_tol > 0) o.inner_tol = opts->inner_tol;
        if (opts->restart > 0) o.restart = opts->restart;
        if (opts->max_iter > 0) o.max_iter = opts->max_iter;
        if (opts->inner_max_iter > 0) o.inner_max_iter = opts->inner_max_iter;
        if (opts->max_refine > 0) o.max_refine = opts->max_refine;
        o.precond = opts->precond;
    }
    SIE_CHECK(o.precond >= 0 && o.precond <= 3, SIE_EINVAL, "unknown preconditioner");
    SIE_CHECK(o.restart <= 1000, SIE_EINVAL, "restart above 1000");
    solve_all(p, prec, o, rep);
}

void currents_entry(const sie_problem *p, int32_t rhs, sie_c128 *u, sie_c128 *v) {
    SIE_CHECK(p && p->solve && p->solve->solved, SIE_ESTATE, "no solution");
    SIE_CHECK(rhs >= 0 && rhs < p->solve->nrhs, SIE_EINVAL, "rhs out of range");
    const int64_t E = p->solve->E;
    if (u) SIE_HIP(hipMemcpy(u, p->solve->u.p + rhs * E, E * sizeof(c128), hipMemcpyDeviceToHost));
    if (v) SIE_HIP(hipMemcpy(v, p->solve->v.p + rhs * E, E * sizeof(c128), hipMemcpyDeviceToHost));
}

void farfield_entry(const sie_problem *cp, int32_t rhs, int64_t ndir, const double *rhat, sie_c128 *F) {
    sie_problem *p = const_cast<sie_problem *>(cp);
    SIE_CHECK(p && p->solve && p->solve->solved, SIE_ESTATE, "no solution");
    SIE_CHECK(rhs >= 0 && rhs < p->solve->nrhs, SIE_EINVAL, "rhs out of range");
    SIE_CHECK(ndir >= 0 && (ndir == 0 || (rhat && F)), SIE_EINVAL, "bad directions");
    if (ndir == 0) return;
    SIE_CHECK(ndir <= (1 << 24), SIE_EINVAL, "too many directions");
    const int64_t E = p->solve->E;
    Rule rq = rule_collapsed(6);
    std::vector<double> packed(4 * rq.size());
    for (int q = 0; q < rq.size(); ++q) {
        for (int c = 0; c < 3; ++c) packed[4 * q + c] = rq.bary[3 * q + c];
        packed[4 * q + 3] = rq.w[q];
    }
    DBuf<double> d_rule, d_rhat;
    d_rule.upload(packed);
    d_rhat.upload(rhat, 3 * ndir);
    DBuf<c128> d_F(3 * ndir);
    const double eta0 = std::sqrt((p->ext.mu.re) / (p->ext.eps.re));
    launch_farfield(p, d_rule.p, rq.size(), p->ext.k.re, eta0, d_rhat.p, ndir, p->solve->u.p + rhs * E,
                    p->solve->v.p + rhs * E, d_F.p, 0);
    std::vector<c128> h = d_F.download(3 * ndir);
    std::memcpy(F, h.data(), 3 * ndir * sizeof(c128));
}
}  // namespace sie
