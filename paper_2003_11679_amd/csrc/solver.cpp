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
// Several right-hand sides are solved together: the Krylov solvers iterate
// them in lock step (one Hessenberg matrix per right-hand side) and every
// operator product takes the whole batch, so the near-field values are
// streamed once per batch (SpMM) and the FFTs run over all fields of all
// right-hand sides.
//
// Precision: SIE_FP64 runs every stage in complex128.  SIE_FP32 runs the
// interior work (K_i products and the nested L_i solves, which dominate the
// operator count) in complex64 inside FP64 iterative refinement: the residual
// of the block equations above (no nested solve needed) is formed in FP64 and
// the correction solved with FP64 exterior products and outer Krylov vectors
// (at low frequency the k0 operator's vector potential is ~(k0 h)^2 below its
// scalar potential and does not survive FP32) around FP32 nested solves.
#include <algorithm>
#include <atomic>
#include <exception>
#include <mutex>
#include <thread>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <numeric>
#include <type_traits>
#include <unordered_map>

#include "problem.h"
#include "solve_kernels.h"

namespace sie {

static const double PI = 3.14159265358979323846;

// ---------------------------------------------------------------- GMRES
// nb independent systems with the same operator iterate in lock step: every
// vector holds the nb systems [nb][n], one operator application serves all
// of them, and each keeps its own Hessenberg matrix, rotations, tolerance
// and convergence state.  A system that has converged (or stalled) in a
// cycle stops extending its basis; its next basis vectors are zero, so the
// shared products carry zeros for it.
// Page-locked host buffer (device-to-host results read after one stream
// synchronisation; host-to-device coefficients copied without staging).
struct PinnedC128 {
    c128 *p = nullptr;
    c128 *dev = nullptr;   // the device's address of the same memory
    size_t n = 0;
    void alloc(size_t k, unsigned flags = hipHostMallocDefault) {
        if (k <= n) return;
        release();
        SIE_HIP(hipHostMalloc((void **)&p, k * sizeof(c128), flags));
        n = k;
        SIE_HIP(hipHostGetDevicePointer((void **)&dev, p, 0));
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        dev = nullptr;
        n = 0;
    }
    PinnedC128() = default;
    PinnedC128(const PinnedC128 &) = delete;
    PinnedC128 &operator=(const PinnedC128 &) = delete;
    ~PinnedC128() { release(); }
};

template <typename T>
struct Gmres {
    int64_t n = 0;                  // length of one system
    int nb = 0;                     // systems
    int m = 0;                      // restart length
    int dblk = 1;                   // dot-product blocks per system
    DBuf<cx<T>> V, Zb, w, r;        // V: (m+1) x [nb][n], Zb: m x [nb][n], w, r: [nb][n]
    DBuf<c128> part, hd, cd;        // hd: 4 slots of [nb][m + 1] dot results
    PinnedC128 hh;                  // host copy of the 4 slots of hd (written by the dot kernels)
    PinnedC128 hc;                  // [nb] scaling coefficients (batches wider than kScaleArg)
    PinnedC128 hy;                  // [nb][m + 1] least-squares solutions
    hipEvent_t hc_done = nullptr;   // last copy out of hc
    hipEvent_t hy_done = nullptr;   // last copy out of hy
    hipEvent_t sync_ev = nullptr;   // host waits
    std::vector<c128> H;            // [nb][m + 1][m] Hessenberg matrices, kept between solves
    std::vector<double> live;       // [nb] residual estimate of the running solve, per step
    using Op = std::function<void(const cx<T> *, cx<T> *)>;
    // Called before the products of every Arnoldi step with the systems
    // still iterating (act[k] != 0); the others' basis vectors are zero, so
    // the products may write zeros for them without computing.
    std::function<void(const std::vector<char> &)> on_active;
    const char *tag = "gmres";
    // Stagnation window: a system that gains under 1 % over this many
    // iterations hands back to the caller (the precision floor of an FP32
    // correction); 0 disables it.
    int stag_window = 25;

    size_t slot() const { return (size_t)nb * (m + 1); }
    void init(int64_t n_, int nb_, int m_) {
        if (n == n_ && nb == nb_ && m == m_) return;
        if (hy_done) SIE_HIP(hipEventSynchronize(hy_done));   // hy is reallocated below
        n = n_; nb = nb_; m = m_;
        const size_t blk = (size_t)nb * n;
        V.alloc((size_t)(m + 1) * blk);
        Zb.alloc((size_t)m * blk);
        w.alloc(blk);
        r.alloc(blk);
        dblk = (int)std::min<int64_t>(DOT_BLOCKS, std::max<int64_t>(4, (n + 4095) / 4096));
        part.alloc((size_t)nb * (m + 1) * dblk);
        hd.alloc(4 * slot());
        cd.alloc(nb);
        hh.alloc(4 * slot(), hipHostMallocMapped | hipHostMallocCoherent);
        hy.alloc(slot());
        hc.alloc(nb);
        if (!hc_done) SIE_HIP(hipEventCreateWithFlags(&hc_done, hipEventDisableTiming));
        if (!hy_done) SIE_HIP(hipEventCreateWithFlags(&hy_done, hipEventDisableTiming));
        if (!sync_ev) SIE_HIP(hipEventCreateWithFlags(&sync_ev, hipEventDisableTiming));
        const size_t need = (size_t)nb * (m + 1) * m;
        if (H.size() < need) H.resize(need);
        live.assign(nb, 1.0);
    }
    Gmres() = default;
    Gmres(const Gmres &) = delete;
    Gmres &operator=(const Gmres &) = delete;
    ~Gmres() {
        if (hy_done) (void)hipEventSynchronize(hy_done);   // hy is freed with the object
        for (hipEvent_t e : {hc_done, hy_done, sync_ev})
            if (e) (void)hipEventDestroy(e);
    }
    // Host wait for the work queued on st so far.  It polls an event: a
    // blocking synchronisation sleeps and adds a wake-up latency to every
    // Arnoldi step.
    void wait(hipStream_t st) {
        SIE_HIP(hipEventRecord(sync_ev, st));
        hipError_t e;
        while ((e = hipEventQuery(sync_ev)) == hipErrorNotReady)
            for (int i = 0; i < 32; ++i) __builtin_ia32_pause();
        SIE_HIP(e);
    }
    // Device slot sl of hd receives h[s][j] = V_j[s]^H x[s], j < J
    // (V_j at Vp + j * nb * n), and so does the same slot of the host's hh
    // (the final dot kernel writes both: no copy launch); returns the device
    // slot.
    c128 *dots_dev(int J, const cx<T> *Vp, const cx<T> *x, int sl, hipStream_t st) {
        c128 *h = hd.p + (size_t)sl * slot();
        launch_dots_sys<T>(n, J, Vp, (int64_t)nb * n, nb, x, part.p, dblk, h, m + 1, st, hh.dev + (size_t)sl * slot());
        return h;
    }
    // h[s][j] = V_j[s]^H x[s], j < J
    std::vector<c128> dots(int J, const cx<T> *Vp, const cx<T> *x, hipStream_t st) {
        dots_dev(J, Vp, x, 0, st);
        wait(st);
        std::vector<c128> out(slot(), c128());
        for (int k = 0; k < nb; ++k)
            std::copy(hh.p + (size_t)k * (m + 1), hh.p + (size_t)k * (m + 1) + J, out.begin() + (size_t)k * (m + 1));
        return out;
    }
    std::vector<double> norms(const cx<T> *x, hipStream_t st) {
        std::vector<c128> h = dots(1, x, x, st);
        std::vector<double> out(nb);
        for (int k = 0; k < nb; ++k) out[k] = std::sqrt(std::max(0.0, h[(size_t)k * (m + 1)].re));
        return out;
    }
    void scale(const std::vector<c128> &c, const cx<T> *x, cx<T> *y, hipStream_t st) {
        if (nb <= kScaleArg) {
            ScaleArg a;
            for (int k = 0; k < nb; ++k) a.v[k] = c[k];
            launch_scale_val<T>(n, nb, a, x, y, st);
            return;
        }
        SIE_HIP(hipEventSynchronize(hc_done));     // hc no longer being copied
        std::copy(c.begin(), c.end(), hc.p);
        SIE_HIP(hipMemcpyAsync(cd.p, hc.p, nb * sizeof(c128), hipMemcpyHostToDevice, st));
        SIE_HIP(hipEventRecord(hc_done, st));
        launch_scale_sys<T>(n, nb, cd.p, x, y, st);
    }

    // Solves A x = b for the nb systems (x holds the initial guesses), each
    // to its own relative tolerance tol[k].  Returns the iterations of the
    // longest system; relres[k] receives the final relative residuals.
    // x_zero: the guesses are zero (the first residual is b, no product; its
    // norms are applied on the device and read with the first Arnoldi step).
    // trust_estimate: return when every system's Arnoldi residual estimate
    // meets its tolerance (or it stagnated) instead of confirming it with a
    // true residual; for solves inside an outer iteration whose own residual
    // is checked.  The host then returns without waiting for the device.
    int solve(const Op &A, const Op &M, const cx<T> *b, cx<T> *x, const std::vector<double> &tol, int maxit,
              std::vector<double> *relres, hipStream_t st, int *napply = nullptr, bool x_zero = false,
              bool trust_estimate = false) {
        static const bool trace = std::getenv("SIE_TRACE") != nullptr;
        static const bool trace_sys = std::getenv("SIE_TRACE_SYSTEMS") != nullptr;
        const size_t ld = (size_t)m + 1, sl = slot(), mm = ld * m;
        const bool defer = x_zero && maxit > 0;
        std::vector<char> fin(nb, 0);
        std::vector<double> res(nb, 0.0), bn(nb, 0.0);
        if (!defer) {
            bn = norms(b, st);
            bool any_zero = false;
            for (int k = 0; k < nb; ++k)
                if (bn[k] == 0.0) fin[k] = 1, any_zero = true;
            if (any_zero) {   // systems with a zero right-hand side: x = 0
                std::vector<c128> keep(nb);
                for (int k = 0; k < nb; ++k) keep[k] = c128(fin[k] ? 0.0 : 1.0);
                scale(keep, x, x, st);
            }
        }
        std::vector<c128> g((size_t)nb * ld), sn((size_t)nb * m);
        std::vector<double> cs((size_t)nb * m);
        std::vector<std::vector<double>> hist(nb);
        std::vector<char> stag(nb, 0);
        int it = 0;
        bool first = true;
        while (true) {
            std::vector<double> beta(nb, 0.0);
            std::vector<char> act(nb, 0);
            std::vector<int> kb(nb, 0);
            const bool pending = first && defer;   // ||b|| still on the device
            if (pending) {
                // V_0 = b / ||b|| on the device; the host reads ||b|| with
                // the first Arnoldi step
                const c128 *nd = dots_dev(1, b, b, 3, st);
                launch_scale_rnorm<T>(n, nb, nd, m + 1, b, V.p, st);
                std::fill(g.begin(), g.end(), c128());
                std::fill(act.begin(), act.end(), 1);
                std::fill(live.begin(), live.end(), 1.0);
            } else {
                // r = b - A x
                if (first && x_zero) {
                    SIE_HIP(hipMemcpyAsync(r.p, b, (size_t)nb * n * sizeof(cx<T>), hipMemcpyDeviceToDevice, st));
                } else {
                    if (on_active) on_active(std::vector<char>(nb, 1));   // the product of every system
                    A(x, r.p);
                    if (napply) ++*napply;
                    launch_axpby<T>((int64_t)nb * n, c128(1.0), b, c128(-1.0), r.p, st);
                }
                beta = norms(r.p, st);
                bool all = true;
                for (int k = 0; k < nb; ++k) {
                    if (bn[k] > 0.0) res[k] = beta[k] / bn[k];
                    if (!fin[k] && (res[k] <= tol[k] || stag[k])) fin[k] = 1;
                    all = all && fin[k];
                }
                live = res;
                if (trace) std::fprintf(stderr, "[%s] restart at it %d true res %.3e\n", tag, it, res[0]);
                if (all || it >= maxit) break;
                std::vector<c128> c0(nb);
                for (int k = 0; k < nb; ++k) {
                    act[k] = !fin[k];
                    c0[k] = act[k] ? c128(1.0 / beta[k]) : c128();
                    std::fill(g.begin() + (size_t)k * ld, g.begin() + (size_t)(k + 1) * ld, c128());
                    g[(size_t)k * ld] = c128(beta[k]);
                }
                scale(c0, r.p, V.p, st);
            }
            first = false;
            const int64_t blk = (int64_t)nb * n;
            int j = 0;
            for (; j < m && it < maxit; ++j, ++it) {
                cx<T> *vj = V.p + (size_t)j * blk, *zj = Zb.p + (size_t)j * blk;
                if (on_active) on_active(act);
                M(vj, zj);
                A(zj, w.p);
                if (napply) ++*napply;
                // classical Gram-Schmidt, twice (the projections use the
                // device copies of the coefficients; the host reads all
                // results after one copy and one wait)
                const c128 *d1 = dots_dev(j + 1, V.p, w.p, 0, st);
                launch_gemv_sys<T>(n, j + 1, V.p, blk, nb, d1, m + 1, w.p, false, st);
                const c128 *d2 = dots_dev(j + 1, V.p, w.p, 1, st);
                launch_gemv_sys<T>(n, j + 1, V.p, blk, nb, d2, m + 1, w.p, false, st);
                dots_dev(1, w.p, w.p, 2, st);
                const bool read_b = pending && j == 0;
                // the dot kernels have written the host's copies of the slots
                wait(st);
                c128 *h1 = hh.p;
                const c128 *h2 = hh.p + sl, *h3 = hh.p + 2 * sl;
                if (read_b) {
                    for (int k = 0; k < nb; ++k) {
                        bn[k] = std::sqrt(std::max(0.0, hh.p[3 * sl + (size_t)k * ld].re));
                        beta[k] = bn[k];
                        res[k] = 1.0;
                        if (bn[k] == 0.0) { fin[k] = 1; act[k] = 0; res[k] = 0.0; }   // x stays zero
                        else g[(size_t)k * ld] = c128(beta[k]);
                    }
                }
                std::vector<double> hn(nb);
                for (int k = 0; k < nb; ++k) hn[k] = std::sqrt(std::max(0.0, h3[(size_t)k * ld].re));
                std::vector<c128> cn(nb);
                bool any = false;
                for (int k = 0; k < nb; ++k) {
                    if (!act[k]) continue;
                    c128 *hk = h1 + (size_t)k * ld;
                    const c128 *h2k = h2 + (size_t)k * ld;
                    for (int i = 0; i <= j; ++i) hk[i] += h2k[i];
                    c128 *gk = g.data() + (size_t)k * ld;
                    double *csk = cs.data() + (size_t)k * m;
                    c128 *snk = sn.data() + (size_t)k * m;
                    for (int i = 0; i < j; ++i) {
                        const c128 a = hk[i], bb = hk[i + 1];
                        hk[i] = csk[i] * a + snk[i] * bb;
                        hk[i + 1] = csk[i] * bb - conj(snk[i]) * a;
                    }
                    {
                        const c128 a = hk[j];
                        const double aa = std::sqrt(norm2(a));
                        const double t = std::hypot(aa, hn[k]);
                        if (aa == 0.0) { csk[j] = 0.0; snk[j] = c128(1.0); hk[j] = c128(t); }
                        else {
                            const c128 ph = (1.0 / aa) * a;
                            csk[j] = aa / t;
                            snk[j] = (hn[k] / t) * ph;
                            hk[j] = t * ph;
                        }
                        gk[j + 1] = -(conj(snk[j]) * gk[j]);
                        gk[j] = csk[j] * gk[j];
                    }
                    c128 *Hk = H.data() + (size_t)k * mm;
                    for (int i = 0; i <= j; ++i) Hk[(size_t)i * m + j] = hk[i];
                    res[k] = std::sqrt(norm2(gk[j + 1])) / bn[k];
                    live[k] = res[k];
                    kb[k] = j + 1;
                    auto &hs = hist[k];
                    hs.push_back(res[k]);
                    if (stag_window > 0 && (int)hs.size() > stag_window &&
                        res[k] > 0.99 * hs[hs.size() - 1 - stag_window])
                        stag[k] = 1;
                    if (res[k] <= tol[k] || hn[k] <= 1e-14 * beta[k] || stag[k]) act[k] = 0;
                    if (act[k] && hn[k] > 1e-300) cn[k] = c128(1.0 / hn[k]);
                    any = any || act[k];
                }
                if (trace) std::fprintf(stderr, "[%s] it %d res %.3e\n", tag, it + 1, res[0]);
                if (!any) { ++j; ++it; break; }
                scale(cn, w.p, V.p + (size_t)(j + 1) * blk, st);
            }
            // y_k = H_k^-1 g_k ; x_k += Zb_k y_k
            int kmax = 0;
            for (int k = 0; k < nb; ++k) kmax = std::max(kmax, kb[k]);
            if (kmax > 0) {
                SIE_HIP(hipEventSynchronize(hy_done));   // hy no longer being copied
                c128 *y = hy.p;
                for (int k = 0; k < nb; ++k) {
                    const int kk = kb[k];
                    const c128 *Hk = H.data() + (size_t)k * mm;
                    const c128 *gk = g.data() + (size_t)k * ld;
                    c128 *yk = y + (size_t)k * ld;
                    std::fill(yk + kk, yk + kmax, c128());
                    for (int i = kk - 1; i >= 0; --i) {
                        c128 sacc = gk[i];
                        for (int l = i + 1; l < kk; ++l) sacc -= Hk[(size_t)i * m + l] * yk[l];
                        yk[i] = cdiv(sacc, Hk[(size_t)i * m + i]);
                    }
                }
                SIE_HIP(hipMemcpy2DAsync(hd.p, ld * sizeof(c128), y, ld * sizeof(c128), kmax * sizeof(c128), nb,
                                         hipMemcpyHostToDevice, st));
                SIE_HIP(hipEventRecord(hy_done, st));
                launch_gemv_sys<T>(n, kmax, Zb.p, blk, nb, hd.p, m + 1, x, true, st);
            }
            if (trust_estimate) {
                bool done = true;
                for (int k = 0; k < nb; ++k)
                    if (!fin[k] && !(res[k] <= tol[k] || stag[k])) done = false;
                if (done || it >= maxit) break;
            }
        }
        if (relres) *relres = res;
        int itmax = 0;
        int64_t itsum = 0;
        for (int k = 0; k < nb; ++k) {
            itmax = std::max(itmax, (int)hist[k].size());
            itsum += (int64_t)hist[k].size();
        }
        if (trace_sys)
            std::fprintf(stderr, "[%s] systems %d iterations max %d sum %lld\n", tag, nb, itmax, (long long)itsum);
        return itmax;
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
    SIE_HIP(hipStreamSynchronize(0));
}

template <typename T> static const cx<T> *bj_inv(const BlockJacobi &bj);
template <> const c128 *bj_inv<double>(const BlockJacobi &bj) { return bj.inv64.p; }
template <> const c64 *bj_inv<float>(const BlockJacobi &bj) { return bj.inv32.p; }

// Restricted additive Schwarz form of the near-region preconditioner
// M_i = -j w eps_i L_i,NR (eq. nest2pc): clusters of C^3 grid cells own their
// RWG functions (cell of the stencil centre of T+) and extend O cells beyond
// on every side; each cluster keeps the owned rows of the inverse of M_i
// restricted to its extended set.  The overlap spans about three mesh edges
// (O = max(1, round(3 l / h)) for mean RWG edge l and grid spacing h) and
// C = 2 O; clusters shrink when an extended one would exceed kRasMax.
struct Schwarz {
    int nc = 0;
    int max_own = 0;               // largest owned set of one cluster
    bool covers_all = false;       // every RWG row is owned by some cluster
    int64_t owned = 0;
    DBuf<int64_t> ext_off, m_off;  // [nc + 1]
    DBuf<int32_t> ext, own_off, own;
    DBuf<int32_t> cobj;            // [nc] object of each cluster
    DBuf<c128> m64;
    DBuf<c64> m32;
};

// Setup workspace (augmented cluster matrices in FP64) per launch: at most
// a quarter of the free device memory, between 2 and 12 GB.  One launch
// then holds the clusters of many small media (one workgroup per cluster,
// 128 KB of LDS each: the chip fills with 256 or more).
constexpr double kSchwarzWorkspaceMin = 2e9, kSchwarzWorkspaceMax = 12e9;

// The near-region operator carries the interior medium's interaction when
// the field decays within the near region: five skin depths fit within
// R grid spacings.  For low-loss media the near-region inverse is a poor
// approximation of the operator's inverse and the nested solve runs
// unpreconditioned.
static bool near_region_dominates(const Medium &md) {
    const double a = std::fabs(md.k.im);
    return a > 0.0 && 5.0 / a <= md.grid->near_radius * md.grid->h;
}

struct ClusterLists {
    std::vector<int64_t> ext_off{0}, m_off{0}, ws_off{0};
    std::vector<int32_t> ext, own_off{0}, own, own_pos;
};

// Clusters of one medium over its RWG rows [r0, r1), into L (lists of this
// medium alone, offsets from zero); false if an extended cluster would exceed
// kRasMax functions at this cluster size.
static bool cluster_medium(sie_problem *p, const Medium &md, int64_t r0, int64_t r1, int C, int O,
                           ClusterLists &L) {
    const Grid &g = *md.grid;
    auto cell = [&](int64_t r, int d) { return g.centre[3 * (size_t)g.glob2loc[p->mesh.tpm[2 * r]] + d]; };
    auto lin = [&](int64_t x, int64_t y, int64_t z) { return (z * g.n[1] + y) * g.n[0] + x; };
    std::unordered_map<int64_t, std::vector<int32_t>> bucket;
    std::map<int64_t, std::vector<int32_t>> clusters;   // ordered: deterministic numbering
    for (int64_t r = r0; r < r1; ++r) {
        const int x = cell(r, 0), y = cell(r, 1), z = cell(r, 2);
        bucket[lin(x, y, z)].push_back((int32_t)r);
        clusters[lin(x / C, y / C, z / C)].push_back((int32_t)r);
    }
    ClusterLists M;
    for (const auto &kv : clusters) {
        const std::vector<int32_t> &ow = kv.second;
        const int bx = cell(ow[0], 0) / C * C, by = cell(ow[0], 1) / C * C, bz = cell(ow[0], 2) / C * C;
        std::vector<int32_t> ex;
        for (int z = bz - O; z <= bz + C - 1 + O; ++z)
            for (int y = by - O; y <= by + C - 1 + O; ++y)
                for (int x = bx - O; x <= bx + C - 1 + O; ++x) {
                    if (x < 0 || y < 0 || z < 0 || x >= g.n[0] || y >= g.n[1] || z >= g.n[2]) continue;
                    auto it = bucket.find(lin(x, y, z));
                    if (it != bucket.end()) ex.insert(ex.end(), it->second.begin(), it->second.end());
                }
        std::sort(ex.begin(), ex.end());
        if (ex.size() > (size_t)kRasMax) return false;
        const int64_t n = (int64_t)ex.size(), no = (int64_t)ow.size();
        for (int32_t r : ow) {
            M.own.push_back(r);
            M.own_pos.push_back((int32_t)(std::lower_bound(ex.begin(), ex.end(), r) - ex.begin()));
        }
        M.ext.insert(M.ext.end(), ex.begin(), ex.end());
        M.ext_off.push_back((int64_t)M.ext.size());
        M.own_off.push_back((int32_t)M.own.size());
        M.m_off.push_back(M.m_off.back() + no * n);
        M.ws_off.push_back(M.ws_off.back() + n * (n + no));
    }
    L = std::move(M);
    return true;
}

// all_media: also the media whose field does not decay within the near
// region (dielectrics, weak conductors), with clusters of 4^3 cells and two
// cells of overlap (or smaller where an extended cluster would be too large);
// there the near-region operator still carries the strong (hypersingular)
// part of the interior EFIE that makes the nested solve slow.
static void schwarz_build(sie_problem *p, Schwarz &sw, const std::vector<Medium *> &media,
                          const std::vector<std::pair<int64_t, int64_t>> &ranges, const std::vector<c128> &scales,
                          bool all_media) {
    // each medium's clusters on the host threads, then joined in medium order
    std::vector<ClusterLists> per(media.size());
    {
        std::atomic<size_t> next{0};
        std::exception_ptr err;
        std::mutex emu;
        auto work = [&]() {
            for (size_t i = next.fetch_add(1); i < media.size(); i = next.fetch_add(1)) {
                try {
                    const bool dominated = near_region_dominates(*media[i]);
                    if (!dominated && !all_media) continue;
                    const int64_t r0 = ranges[i].first, r1 = ranges[i].second;
                    double l = 0.0;
                    for (int64_t r = r0; r < r1; ++r) l += p->mesh.len[r];
                    l /= (double)std::max<int64_t>(r1 - r0, 1);
                    const int O0 = dominated ? std::max(1, (int)std::lround(3.0 * l / media[i]->grid->h)) : 2;
                    bool done = false;
                    for (int O = O0; O >= 1 && !done; --O)
                        for (int C = 2 * O; C >= 1 && !done; --C)
                            done = cluster_medium(p, *media[i], r0, r1, C, O, per[i]);
                } catch (...) {
                    std::lock_guard<std::mutex> lk(emu);
                    if (!err) err = std::current_exception();
                }
            }
        };
        const int nthr = (int)std::max<size_t>(1, std::min<size_t>(16, media.size()));
        std::vector<std::thread> th;
        for (int t = 1; t < nthr; ++t) th.emplace_back(work);
        work();
        for (auto &t : th) t.join();
        if (err) std::rethrow_exception(err);
    }
    ClusterLists L;
    std::vector<int> first;
    for (size_t i = 0; i < media.size(); ++i) {
        first.push_back((int)L.own_off.size() - 1);
        const ClusterLists &M = per[i];
        const int64_t e0 = (int64_t)L.ext.size(), m0 = L.m_off.back(), w0 = L.ws_off.back();
        const int32_t o0 = (int32_t)L.own.size();
        L.ext.insert(L.ext.end(), M.ext.begin(), M.ext.end());
        L.own.insert(L.own.end(), M.own.begin(), M.own.end());
        L.own_pos.insert(L.own_pos.end(), M.own_pos.begin(), M.own_pos.end());
        for (size_t k = 1; k < M.ext_off.size(); ++k) {
            L.ext_off.push_back(e0 + M.ext_off[k]);
            L.own_off.push_back(o0 + M.own_off[k]);
            L.m_off.push_back(m0 + M.m_off[k]);
            L.ws_off.push_back(w0 + M.ws_off[k]);
        }
        ClusterLists().ext.swap(per[i].ext);
    }
    first.push_back((int)L.own_off.size() - 1);
    sw.nc = (int)L.own_off.size() - 1;
    sw.owned = (int64_t)L.own.size();
    for (int c = 0; c < sw.nc; ++c) sw.max_own = std::max(sw.max_own, L.own_off[c + 1] - L.own_off[c]);
    sw.covers_all = sw.owned == p->mesh.nrwg;
    if (sw.nc == 0) return;
    sw.ext_off.upload(L.ext_off);
    sw.ext.upload(L.ext);
    sw.own_off.upload(L.own_off);
    sw.own.upload(L.own);
    sw.m_off.upload(L.m_off);
    sw.m64.alloc((size_t)L.m_off.back());
    sw.m32.alloc((size_t)L.m_off.back());
    DBuf<int32_t> own_pos;
    own_pos.upload(L.own_pos);
    DBuf<int64_t> ws_off;
    ws_off.upload(L.ws_off);
    // the rows each cluster's matrix comes from
    std::vector<RasSource> src(media.size());
    std::vector<int32_t> cmed(sw.nc);
    for (size_t i = 0; i < media.size(); ++i) {
        const Grid &g = *media[i]->grid;
        src[i] = RasSource{g.rwg0, g.d_row_ptr.p, g.d_cols.p, media[i]->d_nLd64.p, scales[i]};
        for (int c = first[i]; c < first[i + 1]; ++c) cmed[c] = (int32_t)i;
    }
    DBuf<RasSource> d_src;
    d_src.upload(src);
    DBuf<int32_t> d_cmed;
    d_cmed.upload(cmed);
    std::vector<int32_t> cobj(sw.nc);
    for (int c = 0; c < sw.nc; ++c) cobj[c] = (int32_t)media[cmed[c]]->id;
    sw.cobj.upload(cobj);
    // batches of consecutive clusters (of any media) within the workspace
    // budget, at least one cluster each
    size_t fr = 0, tot = 0;
    SIE_HIP(hipMemGetInfo(&fr, &tot));
    const double budget = std::min(kSchwarzWorkspaceMax, std::max(kSchwarzWorkspaceMin, 0.25 * (double)fr));
    std::vector<std::pair<int, int>> batches;
    size_t ws_max = 0;
    for (int a = 0; a < sw.nc;) {
        int b = a + 1;
        while (b < sw.nc && (double)(L.ws_off[b + 1] - L.ws_off[a]) * sizeof(c128) <= budget) ++b;
        batches.push_back({a, b});
        ws_max = std::max(ws_max, (size_t)(L.ws_off[b] - L.ws_off[a]));
        a = b;
    }
    DBuf<c128> ws(ws_max);
    DBuf<int> fail(1);
    SIE_HIP(hipMemsetAsync(fail.p, 0, sizeof(int), 0));
    for (const auto &bt : batches)
        launch_ras_setup(bt.first, bt.second - bt.first, sw.ext_off.p, sw.ext.p, sw.own_off.p, own_pos.p, ws_off.p,
                         sw.m_off.p, d_cmed.p, d_src.p, ws.p, sw.m64.p, sw.m32.p, fail.p, 0);
    int bad = 0;
    SIE_HIP(hipMemcpyAsync(&bad, fail.p, sizeof(int), hipMemcpyDeviceToHost, 0));
    SIE_HIP(hipStreamSynchronize(0));
    SIE_CHECK(!bad, SIE_EINVAL, "near-region preconditioner: singular cluster matrix");
}

template <typename T> static const cx<T> *ras_m(const Schwarz &w);
template <> const c128 *ras_m<double>(const Schwarz &w) { return w.m64.p; }
template <> const c64 *ras_m<float>(const Schwarz &w) { return w.m32.p; }

// ---------------------------------------------------------------- exact near-region factorisation
// The preconditioner of eq. nest2pc as the paper applies it: a sparse LU of
// M_i = -j w eps_i L_i,NR over the object's RWG rows, factored in FP64
// (nested dissection and symbolic factorisation on the host, fronts
// eliminated on the device, no pivoting) and applied with the device's
// level-by-level triangular solves (in FP32 with FP32 copies of the factors
// for FP32 solves).  A medium whose near-region matrix is too dense to
// factor as a sparse matrix (more than kLUMeanRow nonzeros per row on
// average when above the supernode limit in size, a separator above that
// limit, or factors beyond the size and arithmetic limits of the sparse LU)
// gets none.
struct NearLU {
    int medium = 0;
    int64_t r0 = 0, n = 0;
    SparseLU f;
};
constexpr double kLUMeanRow = 1500.0;

static bool near_lu_build(sie_problem *p, int medium, int64_t r0, int64_t r1, c128 scale, NearLU &out) {
    const Medium &md = p->ints[medium];
    const Grid &g = *md.grid;
    const int64_t n = r1 - r0;
    if (n <= 0) return false;
    SIE_CHECK(r0 >= g.rwg0 && r1 <= g.rwg1, SIE_EINVAL, "object rows outside its grid's rows");
    const std::vector<int64_t> rp_all = g.d_row_ptr.download();
    const int64_t b = rp_all[r0 - g.rwg0], e = rp_all[r1 - g.rwg0];
    if (n > kLUMaxSupernode && (double)(e - b) > kLUMeanRow * (double)n) return false;
    std::vector<int32_t> cols(e - b);
    std::vector<c128> vals(e - b);
    if (e > b) {
        SIE_HIP(hipMemcpy(cols.data(), g.d_cols.p + b, (e - b) * sizeof(int32_t), hipMemcpyDeviceToHost));
        SIE_HIP(hipMemcpy(vals.data(), md.d_nLd64.p + b, (e - b) * sizeof(c128), hipMemcpyDeviceToHost));
    }
    // local rows and columns (the near pattern is symmetric, holds every
    // diagonal and lists each row's columns in ascending order)
    std::vector<int64_t> rp(n + 1, 0);
    std::vector<int32_t> ci;
    std::vector<c128> val;
    ci.reserve(e - b);
    val.reserve(e - b);
    for (int64_t i = 0; i < n; ++i) {
        bool diag = false;
        for (int64_t k = rp_all[r0 - g.rwg0 + i] - b; k < rp_all[r0 - g.rwg0 + i + 1] - b; ++k) {
            const int64_t c = (int64_t)cols[k] - r0;
            if (c < 0 || c >= n) continue;
            SIE_CHECK((int64_t)ci.size() == rp[i] || ci.back() < c, SIE_EINVAL, "near pattern not ascending");
            diag |= c == i;
            ci.push_back((int32_t)c);
            val.push_back(scale * vals[k]);
        }
        SIE_CHECK(diag, SIE_EINVAL, "near pattern without its diagonal");
        rp[i + 1] = (int64_t)ci.size();
    }
    // RWG edge midpoints place the unknowns for the dissection
    const Mesh &m = p->mesh;
    std::vector<double> xyz(3 * n);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t a = m.edge_v[2 * (r0 + i)], c = m.edge_v[2 * (r0 + i) + 1];
        for (int d = 0; d < 3; ++d) xyz[3 * i + d] = 0.5 * (m.xyz[3 * a + d] + m.xyz[3 * c + d]);
    }
    try {
        lu_factor(out.f, n, rp, ci, val, xyz, hipStreamPerThread);
    } catch (const Error &er) {
        if (er.code == SIE_EINVAL) return false;   // too dense, or a vanishing pivot
        throw;
    }
    lu_make_fp32(out.f, hipStreamPerThread);   // FP32 nested solves apply FP32 factors
    out.medium = medium;
    out.r0 = r0;
    out.n = n;
    return true;
}

// ---------------------------------------------------------------- solve state
struct SolveState {
    int nrhs = 0;
    int64_t E = 0;
    DBuf<c128> e, u, v;            // [nrhs][E]
    bool solved = false;
    BlockJacobi pin, pout;         // inner (interior L-hat) and outer (exterior) preconditioners
    bool pre_built = false;
    Schwarz sin;                   // near-region Schwarz preconditioner of the nested solves
    bool sin_built = false;
    int sin_bits = 0;              // preconditioner bits it was built for
    std::vector<std::unique_ptr<NearLU>> nlu;   // exact near-region factorisations (one per factored medium)
    bool nlu_built = false;
    bool nlu_covers_all = false;   // every RWG row belongs to a factored medium
    int64_t nlu_nnz = 0;
    double nlu_factor_s = 0.0;
    DBuf<c128> nlu_work;           // [nrhs][n] right-hand sides in position order
    DBuf<c64> nlu_work32;
    Gmres<double> go64, gi64;
    Gmres<float> go32, gi32;
    Gmres<double> goa;             // outer solve of the augmented EFIE (unknowns [u; sigma])
    DBuf<c128> sg;                 // [nrhs][T] charge unknowns sigma = c0 rho of the augmented EFIE
    DBuf<c128> t64[6];
    DBuf<c64> t32[6];
    int64_t matvecs = 0, kmatvecs = 0;   // L-type / K-type products, one per medium and right-hand side
    int inner_iters = 0, inner_max = 0;
};

void solver_destroy(SolveState *s) { delete s; }

template <typename T> static DBuf<cx<T>> &nlu_work_of(SolveState &s);
template <> DBuf<c128> &nlu_work_of<double>(SolveState &s) { return s.nlu_work; }
template <> DBuf<c64> &nlu_work_of<float>(SolveState &s) { return s.nlu_work32; }
template <typename T> static DBuf<cx<T>> *tmp_of(SolveState &s);
template <> DBuf<c128> *tmp_of<double>(SolveState &s) { return s.t64; }
template <> DBuf<c64> *tmp_of<float>(SolveState &s) { return s.t32; }
template <typename T> static Gmres<T> &outer_of(SolveState &s);
template <> Gmres<double> &outer_of<double>(SolveState &s) { return s.go64; }
template <> Gmres<float> &outer_of<float>(SolveState &s) { return s.go32; }
template <typename T> static Gmres<T> &inner_of(SolveState &s);
template <> Gmres<double> &inner_of<double>(SolveState &s) { return s.gi64; }
template <> Gmres<float> &inner_of<float>(SolveState &s) { return s.gi32; }

// Krylov dimension of the nested solves: the interior EFIE of a low-loss
// dielectric on a fine mesh needs a few hundred iterations, which restarts
// every `restart` iterations would multiply; restart only beyond 300.
static int nested_dim(int restart, int inner_max_iter) {
    return std::max(restart, std::min(inner_max_iter, 300));
}

// Operator set for nb right-hand sides at once: every vector is [nb][E].
// Nested-solve preconditioner on nrhs vectors [nrhs][E]: Schwarz clusters
// (rows of media without clusters copied) and/or the exact factorisations
// of the media that have one; x and y must not alias.
// active (optional, [nrhs][objects]): the Schwarz clusters of inactive
// objects write zeros (their rows of x are zero).
template <typename T>
static void nested_apply(sie_problem *p, SolveState &s, bool ras, bool lu, int nrhs, const cx<T> *x, cx<T> *y,
                         hipStream_t st, const uint8_t *active = nullptr) {
    const int64_t E = p->mesh.nrwg;
    const bool covered = (ras && s.sin.covers_all) || (lu && s.nlu_covers_all);
    if (!covered) SIE_HIP(hipMemcpyAsync(y, x, (size_t)nrhs * E * sizeof(cx<T>), hipMemcpyDeviceToDevice, st));
    if (ras) {
        const Schwarz &w = s.sin;
        launch_ras_apply<T>(w.nc, w.max_own, w.ext_off.p, w.ext.p, w.own_off.p, w.own.p, w.m_off.p, ras_m<T>(w), x, y,
                            E, nrhs, st, active, (int)p->ints.size(), w.cobj.p);
    }
    if (lu) {
        DBuf<cx<T>> &wk = nlu_work_of<T>(s);
        for (const auto &f : s.nlu) {
            const size_t need = (size_t)nrhs * f->n;
            if (wk.n < need) wk.alloc(need);
            launch_lu_gather<T>(f->n, f->r0, E, nrhs, f->f.iperm.p, x, wk.p, st);
            lu_solve(f->f, nrhs, wk.p, st);
            launch_lu_scatter<T>(f->n, f->r0, E, nrhs, f->f.iperm.p, wk.p, y, st);
        }
    }
}

template <typename T>
struct Ops {
    sie_problem *p;
    SolveState &s;
    hipStream_t st;
    int64_t E;
    int nb;
    int64_t NE;                    // nb * E
    cx<T> *t[6];
    double inner_tol;
    int inner_max_iter;
    int restart;

    // Nested systems per right-hand side: one per object when the objects
    // have equal RWG counts (their block-diagonal systems then iterate side
    // by side in lock step, each with its own Krylov basis, tolerance and
    // convergence), else one for all of them.
    int nsys = 1;
    Ops(sie_problem *p_, SolveState &s_, hipStream_t st_, double itol, int imax, int rs, int nb_, bool outer = true)
        : p(p_), s(s_), st(st_), E(p_->mesh.nrwg), nb(nb_), NE((int64_t)nb_ * p_->mesh.nrwg), inner_tol(itol),
          inner_max_iter(imax), restart(rs) {
        DBuf<cx<T>> *tb = tmp_of<T>(s);
        for (int i = 0; i < 6; ++i) {
            if (tb[i].n != (size_t)NE) tb[i].alloc(NE);
            t[i] = tb[i].p;
        }
        const std::vector<int64_t> &o0 = p->mesh.obj_rwg0;
        const int nobj = (int)o0.size() - 1;
        bool equal = nobj > 1;
        for (int i = 1; i < nobj && equal; ++i) equal = o0[i + 1] - o0[i] == o0[1] - o0[0];
        nsys = equal ? nobj : 1;
        inner_of<T>(s).init(E / nsys, nb * nsys, nested_dim(restart, imax));
        if (outer) outer_of<T>(s).init(E, nb, restart);
        inner_of<T>(s).tag = sizeof(T) == 8 ? "inner64" : "inner32";
        outer_of<T>(s).tag = sizeof(T) == 8 ? "outer64" : "outer32";
    }

    void count(sie_op op, int64_t n) {
        if (op == SIE_OP_L) s.matvecs += n;
        else if (op == SIE_OP_K) s.kmatvecs += n;
    }
    void mv(Medium &md, sie_op op, const cx<T> *x, cx<T> *y) {
        matvec<T>(p, md, op, nb, x, y, st);
        count(op, nb);
    }
    // Product of every interior medium on its own rows, one launch per stage
    // and group of media (the groups' rows cover all RWG functions).
    void interior(sie_op op, bool scaled, const cx<T> *x, cx<T> *y, const uint8_t *act = nullptr) {
        for (auto &gp : p->groups) {
            group_product<T>(p, *gp, op, scaled, nb, x, y, st, act);
            // products of objects that are skipped (zero rows) are not counted
            int64_t n = (int64_t)gp->media.size();
            if (act) {
                n = 0;
                for (int o : gp->media) n += act_last[o] ? 1 : 0;
            }
            count(op, (int64_t)nb * n);
        }
    }
    // Objects whose nested systems still iterate ([nb][objects], device),
    // while a nested solve with one system per object runs; null otherwise.
    const uint8_t *active = nullptr;
    bool skip_converged = true;
    DBuf<uint8_t> act_dev;
    PinnedC128 act_host;
    std::vector<char> act_last;
    // y = sum_i (-j w eps~_i) L_i x   (block diagonal over objects)
    void Lhat(const cx<T> *x, cx<T> *y) { interior(SIE_OP_L, true, x, y, active); }
    // y = sum_i K_i x + sgn X x / 2
    void KpX(bool interior_side, double sgn, const cx<T> *x, cx<T> *y) {
        if (interior_side) {
            interior(SIE_OP_K, false, x, y);
        } else {
            mv(p->ext, SIE_OP_K, x, y);
        }
        mv(p->ext, SIE_OP_X, x, t[4]);
        launch_axpby<T>(NE, c128(0.5 * sgn), t[4], c128(1.0), y, st);
    }
    bool use_bj_in = false, use_bj_out = false;
    void bj(bool on, const BlockJacobi &b, const cx<T> *x, cx<T> *y) {
        if (!on) {
            SIE_HIP(hipMemcpyAsync(y, x, NE * sizeof(cx<T>), hipMemcpyDeviceToDevice, st));
            return;
        }
        for (int k = 0; k < nb; ++k) launch_bj_apply<T>(b.nb, b.B, b.perm.p, bj_inv<T>(b), x + k * E, y + k * E, st);
    }
    bool use_ras_in = false, use_lu_in = false;
    void prec_inner(const cx<T> *x, cx<T> *y) {
        if (!use_ras_in && !use_lu_in) {
            bj(use_bj_in, s.pin, x, y);
            return;
        }
        nested_apply<T>(p, s, use_ras_in, use_lu_in, nb, x, y, st, active);
    }
    void prec_outer(const cx<T> *x, cx<T> *y) { bj(use_bj_out, s.pout, x, y); }
    // Mixed precision: an FP64 operator set may delegate the interior work
    // (K_i products and the nested L_i solves) to an FP32 one.
    Ops<float> *lo = nullptr;
    // v = Lhat^-1 a (nested solve, eq. nest2)
    void inner_solve(const cx<T> *a, cx<T> *v);
    // Relaxed nested tolerance (inexact Krylov): while relax_res points at
    // the enclosing solve's residual estimates, nested solve k runs to
    // relax_eps[k] / (*relax_res)[k] within [inner_tol, kRelaxCap].
    static constexpr double kRelaxCap = 1e-2;
    const std::vector<double> *relax_res = nullptr;
    std::vector<double> relax_eps;
    void inner_solve_native(const cx<T> *a, cx<T> *v) {
        SIE_HIP(hipMemsetAsync(v, 0, NE * sizeof(cx<T>), st));
        // system k of the nested solver: right-hand side k / nsys, object k mod nsys
        std::vector<double> tol((size_t)nb * nsys, inner_tol);
        if (relax_res)
            for (int k = 0; k < nb * nsys; ++k) {
                const int r = k / nsys;
                tol[k] = std::min(kRelaxCap, std::max(inner_tol, relax_eps[r] / std::max((*relax_res)[r], 1e-300)));
            }
        // with one nested system per object, the products skip the objects
        // whose systems have converged
        Gmres<T> &g = inner_of<T>(s);
        const int nobj = (int)p->ints.size();
        if (skip_converged && nsys == nobj && nobj > 1 && nb == 1) {
            if (act_dev.n < (size_t)nobj) {
                act_dev.alloc(nobj);
                act_host.alloc((nobj + 15) / 16);
            }
            act_last.assign(nobj, 2);
            g.on_active = [&](const std::vector<char> &act) {
                if (std::equal(act.begin(), act.end(), act_last.begin())) return;
                act_last.assign(act.begin(), act.end());
                if (std::find(act.begin(), act.end(), 0) == act.end()) {   // all iterate: no mask
                    active = nullptr;
                    return;
                }
                // the previous copy out of act_host ended before the last
                // Arnoldi step's host wait
                uint8_t *h = reinterpret_cast<uint8_t *>(act_host.p);
                for (int k = 0; k < nobj; ++k) h[k] = act[k] ? 1 : 0;
                SIE_HIP(hipMemcpyAsync(act_dev.p, h, nobj, hipMemcpyHostToDevice, st));
                active = act_dev.p;
            };
        }
        struct Reset {
            Gmres<T> &g;
            const uint8_t *&a;
            ~Reset() { g.on_active = nullptr; a = nullptr; }
        } reset{g, active};
        int it = g.solve([&](const cx<T> *x, cx<T> *y) { Lhat(x, y); },
                         [&](const cx<T> *x, cx<T> *y) { prec_inner(x, y); }, a, v, tol, inner_max_iter, nullptr, st,
                         nullptr, true, true);
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
    void gibc_mixed(const cx<T> *u, cx<T> *y);
    void gibc(const cx<T> *u, cx<T> *y) {
        if constexpr (std::is_same<T, double>::value) {
            if (lo) {
                gibc_mixed(u, y);
                return;
            }
        }
        Z(u, t[1]);
        KpX(false, -1.0, t[1], t[2]);
        mv(p->ext, SIE_OP_L, u, y);
        launch_axpby<T>(NE, c128(-1.0), t[2], c128(0.0, p->w) * p->ext.mu, y, st);
    }
};

// Mixed precision: v = Z u comes out of the FP32 nested solve, and
// (K0 - X/2) v is applied to it in FP32 as well (K0 has no cancellation
// between terms of different order in k0 h); j w mu0 L0 u stays FP64 (its
// vector potential is ~(k0 h)^2 below its scalar potential at low frequency).
template <> void Ops<float>::gibc_mixed(const c64 *, c64 *) {}
template <> void Ops<double>::gibc_mixed(const c128 *u, c128 *y) {
    c64 *u32 = lo->t[1], *v32 = lo->t[2], *k32 = lo->t[3];
    launch_convert<double, float>(u, u32, NE, st);
    lo->Z_native(u32, v32);
    lo->KpX(false, -1.0, v32, k32);
    launch_convert<float, double>(k32, t[2], NE, st);
    mv(p->ext, SIE_OP_L, u, y);
    launch_axpby<double>(NE, c128(-1.0), t[2], c128(0.0, p->w) * p->ext.mu, y, st);
}

template <> void Ops<float>::inner_solve(const c64 *a, c64 *v) { inner_solve_native(a, v); }
template <> void Ops<float>::Z(const c64 *u, c64 *v) { Z_native(u, v); }
template <> void Ops<double>::inner_solve(const c128 *a, c128 *v) {
    if (!lo) { inner_solve_native(a, v); return; }
    c64 *a32 = lo->t[1], *v32 = lo->t[2];
    launch_convert<double, float>(a, a32, NE, st);
    lo->inner_solve_native(a32, v32);
    launch_convert<float, double>(v32, v, NE, st);
}
template <> void Ops<double>::Z(const c128 *u, c128 *v) {
    if (!lo) { Z_native(u, v); return; }
    c64 *u32 = lo->t[1], *v32 = lo->t[2];
    launch_convert<double, float>(u, u32, NE, st);
    lo->Z_native(u32, v32);
    launch_convert<float, double>(v32, v, NE, st);
}

// FP64 residual of the block equations for the nb systems of o:
// r1 = e - [j w mu0 L0 u - (K0 - X/2) v], r2 = -[-(K_i + X/2) u + Lhat v];
// returns ||r_k|| / ||e_k|| per system.
static std::vector<double> block_residual(Ops<double> &o, const c128 *e, const c128 *u, const c128 *v, c128 *r1,
                                          c128 *r2) {
    const int64_t NE = o.NE;
    hipStream_t st = o.st;
    // r1
    o.KpX(false, -1.0, v, o.t[2]);
    o.mv(o.p->ext, SIE_OP_L, u, r1);
    launch_axpby<double>(NE, c128(-1.0), o.t[2], c128(0.0, o.p->w) * o.p->ext.mu, r1, st);   // A1 x
    launch_axpby<double>(NE, c128(1.0), e, c128(-1.0), r1, st);                              // e - A1 x
    // r2 = (K_i + X/2) u - Lhat v
    o.KpX(true, +1.0, u, r2);
    o.Lhat(v, o.t[3]);
    launch_axpby<double>(NE, c128(-1.0), o.t[3], c128(1.0), r2, st);
    Gmres<double> &g = o.s.go64;
    const std::vector<double> n1 = g.norms(r1, st), n2 = g.norms(r2, st), ne = g.norms(e, st);
    std::vector<double> out(o.nb);
    for (int k = 0; k < o.nb; ++k) out[k] = ne[k] > 0.0 ? std::sqrt(n1[k] * n1[k] + n2[k] * n2[k]) / ne[k] : 0.0;
    return out;
}

// ---------------------------------------------------------------- augmented EFIE
// Outer operator of eq. sys for x = [u; sigma] per right-hand side (stride
// E + T): the augmented exterior product minus (K0 - X/2) Z u / eta0 on the
// first E rows.  With an FP32 operator set, Z u and (K0 - X/2) Z u run in
// FP32 (as in the GIBC system); the augmented product stays FP64.
static double eta0_of(const sie_problem *p) { return std::sqrt(p->ext.mu.re / p->ext.eps.re); }

static const c128 *aug_u(Ops<double> &o, const c128 *x, c128 *tmp) {
    if (o.nb == 1) return x;
    const int64_t ld = o.E + o.p->mesh.nt();
    SIE_HIP(hipMemcpy2DAsync(tmp, o.E * sizeof(c128), x, ld * sizeof(c128), o.E * sizeof(c128), o.nb,
                             hipMemcpyDeviceToDevice, o.st));
    return tmp;
}

static void gibc_aug(Ops<double> &o, const c128 *x, c128 *y) {
    sie_problem *p = o.p;
    const int64_t E = o.E, ld = E + p->mesh.nt();
    aug_product(p, o.nb, x, y, o.st);
    o.count(SIE_OP_L, o.nb);
    const c128 *u = aug_u(o, x, o.t[5]);
    if (o.lo) {
        Ops<float> &l = *o.lo;
        launch_convert<double, float>(u, l.t[1], o.NE, o.st);
        l.Z_native(l.t[1], l.t[2]);
        l.KpX(false, -1.0, l.t[2], l.t[3]);
        launch_convert<float, double>(l.t[3], o.t[2], o.NE, o.st);
    } else {
        o.Z(u, o.t[1]);
        o.KpX(false, -1.0, o.t[1], o.t[2]);
    }
    const c128 a(-1.0 / eta0_of(p));
    for (int k = 0; k < o.nb; ++k) launch_axpby<double>(E, a, o.t[2] + k * E, c128(1.0), y + k * ld, o.st);
}

// FP64 residual of the augmented block equations (eq. sys with v kept, and
// the interior rows of eq. MFIE1dis): r1 [nb][E + T] = ea - [aug(u, sigma) -
// (K0 - X/2) v / eta0 on the first E rows], r2 = (K_i + X/2) u - Lhat v;
// returns sqrt(|r1|^2 + |r2|^2) / |ea| per system.
static std::vector<double> block_residual_aug(Ops<double> &o, Gmres<double> &ga, const c128 *ea, const c128 *xa,
                                              const c128 *v, c128 *r1, c128 *r2) {
    sie_problem *p = o.p;
    const int64_t E = o.E, ld = E + p->mesh.nt();
    hipStream_t st = o.st;
    aug_product(p, o.nb, xa, r1, st);
    o.count(SIE_OP_L, o.nb);
    o.KpX(false, -1.0, v, o.t[2]);
    const c128 a(-1.0 / eta0_of(p));
    for (int k = 0; k < o.nb; ++k) launch_axpby<double>(E, a, o.t[2] + k * E, c128(1.0), r1 + k * ld, st);
    launch_axpby<double>((int64_t)o.nb * ld, c128(1.0), ea, c128(-1.0), r1, st);
    const c128 *u = aug_u(o, xa, o.t[5]);
    o.KpX(true, +1.0, u, r2);
    o.Lhat(v, o.t[3]);
    launch_axpby<double>(o.NE, c128(-1.0), o.t[3], c128(1.0), r2, st);
    const std::vector<double> n1 = ga.norms(r1, st), n2 = o.s.go64.norms(r2, st), ne = ga.norms(ea, st);
    std::vector<double> out(o.nb);
    for (int k = 0; k < o.nb; ++k) out[k] = ne[k] > 0.0 ? std::sqrt(n1[k] * n1[k] + n2[k] * n2[k]) / ne[k] : 0.0;
    return out;
}

// precond bits: 1 block-Jacobi in the nested solves, 2 block-Jacobi in the
// outer solve, 4 near-region Schwarz clusters in the nested solves.
static void build_preconditioners(sie_problem *p, SolveState &s, int precond) {
    std::vector<Medium *> mi;
    std::vector<std::pair<int64_t, int64_t>> ri;
    std::vector<c128> si;
    for (size_t i = 0; i < p->ints.size(); ++i) {
        mi.push_back(&p->ints[i]);
        ri.push_back({p->mesh.obj_rwg0[i], p->mesh.obj_rwg0[i + 1]});
        si.push_back(c128(0.0, -p->w) * p->ints[i].eps);
    }
    if ((precond & 3) && !s.pre_built) {
        bj_build(p, s.pin, mi, ri, si);
        bj_build(p, s.pout, {&p->ext}, {{0, p->mesh.nrwg}}, {c128(0.0, p->w) * p->ext.mu});
        s.pre_built = true;
    }
    std::vector<char> factored(mi.size(), 0);
    if (precond & 16) {
        if (!s.nlu_built) {
            const auto t0 = std::chrono::steady_clock::now();
            int64_t rows = 0;
            for (size_t i = 0; i < mi.size(); ++i) {
                std::unique_ptr<NearLU> f(new NearLU);
                if (near_lu_build(p, (int)i, ri[i].first, ri[i].second, si[i], *f)) {
                    rows += f->n;
                    s.nlu_nnz += f->f.nnz_factor;
                    s.nlu.push_back(std::move(f));
                }
            }
            s.nlu_covers_all = rows == p->mesh.nrwg;
            s.nlu_built = true;
            s.nlu_factor_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (std::getenv("SIE_TRACE")) {
                double fl = 0.0;
                for (const auto &f : s.nlu) fl += f->f.est_flops;
                std::fprintf(stderr, "[setup] %-28s %8.1f ms (%zu media, %.3g Tflop)\n", "near-region LU",
                             1e3 * s.nlu_factor_s, s.nlu.size(), fl / 1e12);
            }
        }
        for (const auto &f : s.nlu) factored[f->medium] = 1;
    }
    const int sin_bits = precond & (4 | 8 | 16);
    if ((precond & 4) && (!s.sin_built || s.sin_bits != sin_bits)) {
        const auto t0 = std::chrono::steady_clock::now();
        // clusters for the media without an exact factorisation
        std::vector<Medium *> mr;
        std::vector<std::pair<int64_t, int64_t>> rr;
        std::vector<c128> sr;
        for (size_t i = 0; i < mi.size(); ++i)
            if (!factored[i]) { mr.push_back(mi[i]); rr.push_back(ri[i]); sr.push_back(si[i]); }
        s.sin = Schwarz();
        schwarz_build(p, s.sin, mr, rr, sr, (precond & 8) != 0);
        s.sin_built = true;
        s.sin_bits = sin_bits;
        if (std::getenv("SIE_TRACE"))
            std::fprintf(stderr, "[setup] %-28s %8.1f ms\n", "Schwarz clusters",
                         std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    }
}

// Relaxed nested tolerances inside one correction solve (res: the outer
// solve's residual estimates; null ends the relaxation).  The nested solves
// run in the FP32 operator set when there is one, else in the FP64 one.
// Not with the exact near-region factorisation: its nested solves reach a
// loose tolerance in one or two costly iterations, and the larger nested
// errors then cost more outer iterations than the relaxation saves (on
// dielectric requests 2-4 times the outer iterations and 1.3-4 times the
// solve time of fixed tolerances).
static void set_relax(Ops<double> &o64, Ops<float> *o32, double relax, const std::vector<double> &stol,
                      const std::vector<double> *res) {
    if (o64.use_lu_in) res = nullptr;
    std::vector<double> eps(stol.size());
    for (size_t k = 0; k < stol.size(); ++k) eps[k] = relax * stol[k];
    if (o32) {
        o32->relax_eps = eps;
        o32->relax_res = res;
    } else {
        o64.relax_eps = eps;
        o64.relax_res = res;
    }
}

// Refinement sweeps of the augmented EFIE for one batch: the residual of the
// augmented block equations in FP64, the correction [du; dsigma] from eq. sys
// (right-preconditioned with the constraint preconditioner) around nested
// solves as in the GIBC system.  u, v [cnt][E] and sg [cnt][T] receive the
// solution; res the final relative residuals.
static void refine_aug(sie_problem *p, SolveState &s, Ops<double> &o64, Ops<float> *o32, sie_precision prec,
                       const sie_solver_opts &o, const c128 *e, c128 *u, c128 *v, c128 *sg, int cnt,
                       std::vector<double> &res, int &outer_total, int &sweeps_total) {
    const int64_t E = o64.E, T = p->mesh.nt(), ld = E + T, NE = o64.NE, NA = (int64_t)cnt * ld;
    hipStream_t st = o64.st;
    Gmres<double> &ga = s.goa;
    ga.init(ld, cnt, o.restart);
    ga.tag = "outer_aug";
    s.go64.init(E, cnt, 1);   // norms and scaling of the interior rows
    DBuf<c128> ea(NA), xa(NA), r1(NA), dx(NA), r2(NE), dv(NE), sv(NE), du(NE);
    const double ie = 1.0 / eta0_of(p);
    launch_zero<double>(NA, ea.p, st);
    for (int k = 0; k < cnt; ++k) launch_axpby<double>(E, c128(ie), e + k * E, c128(0.0), ea.p + k * ld, st);
    launch_zero<double>(NA, xa.p, st);
    launch_zero<double>(NE, v, st);
    std::vector<double> prev(cnt, 2.0);
    std::vector<char> done(cnt, 0);
    for (int sw = 0; sw <= o.max_refine; ++sw) {
        res = block_residual_aug(o64, ga, ea.p, xa.p, v, r1.p, r2.p);
        bool all = true;
        std::vector<c128> keep(cnt);
        for (int k = 0; k < cnt; ++k) {
            if (!done[k] && (res[k] <= o.tol || sw == o.max_refine || res[k] > 0.5 * prev[k])) done[k] = 1;
            prev[k] = res[k];
            keep[k] = c128(done[k] ? 0.0 : 1.0);
            all = all && done[k];
        }
        if (all) break;
        ++sweeps_total;
        ga.scale(keep, r1.p, r1.p, st);
        s.go64.scale(keep, r2.p, r2.p, st);
        // sv = Lhat^-1 r2 ; the exterior rows take (K0 - X/2) sv / eta0
        o64.inner_solve(r2.p, sv.p);
        o64.KpX(false, -1.0, sv.p, o64.t[3]);
        for (int k = 0; k < cnt; ++k)
            launch_axpby<double>(E, c128(ie), o64.t[3] + k * E, c128(1.0), r1.p + k * ld, st);
        launch_zero<double>(NA, dx.p, st);
        ga.stag_window = prec == SIE_FP32 ? 100 : 0;
        const double floor32 = std::min(1e-3, std::max(2e-4, 0.63 * std::sqrt(o.tol)));
        std::vector<double> stol(cnt);
        for (int k = 0; k < cnt; ++k) {
            const double need = res[k] > 0.0 ? o.tol / res[k] : 1.0;
            stol[k] = prec == SIE_FP32 ? std::max(need, floor32) : need;
        }
        if (o.inner_relax > 0.0) set_relax(o64, o32, o.inner_relax, stol, &ga.live);
        outer_total += ga.solve([&](const c128 *x, c128 *y) { gibc_aug(o64, x, y); },
                                [&](const c128 *x, c128 *y) { cp_apply(p, cnt, x, y, st); }, r1.p, dx.p, stol,
                                o.max_iter, nullptr, st, nullptr, true);
        set_relax(o64, o32, 0.0, stol, nullptr);
        // dv = Lhat^-1 (r2 + (K_i + X/2) du)
        const c128 *dup = aug_u(o64, dx.p, du.p);
        o64.KpX(true, +1.0, dup, o64.t[3]);
        launch_axpby<double>(NE, c128(1.0), r2.p, c128(1.0), o64.t[3], st);
        o64.inner_solve(o64.t[3], dv.p);
        launch_axpby<double>(NA, c128(1.0), dx.p, c128(1.0), xa.p, st);
        launch_axpby<double>(NE, c128(1.0), dv.p, c128(1.0), v, st);
    }
    SIE_HIP(hipMemcpy2DAsync(u, E * sizeof(c128), xa.p, ld * sizeof(c128), E * sizeof(c128), cnt,
                             hipMemcpyDeviceToDevice, st));
    SIE_HIP(hipMemcpy2DAsync(sg, T * sizeof(c128), xa.p + E, ld * sizeof(c128), T * sizeof(c128), cnt,
                             hipMemcpyDeviceToDevice, st));
    SIE_HIP(hipStreamSynchronize(st));   // the batch's buffers are released on return
}

// Krylov storage of one batch of right-hand sides is kept within this many
// bytes (outer and nested bases, FP64 plus the FP32 nested copy).
constexpr double kKrylovBudget = 24e9;

static void solve_all(sie_problem *p, sie_precision prec, const sie_solver_opts &o, sie_report *rep) {
    SolveState &s = *p->solve;
    const int64_t E = s.E;
    hipStream_t st = 0;
    if (o.precond != 0) build_preconditioners(p, s, o.precond);
    s.matvecs = s.kmatvecs = 0;
    s.inner_iters = s.inner_max = 0;
    int outer_total = 0, sweeps_total = 0;
    double worst = 0.0;
    bool all_conv = true;
    const auto t0 = std::chrono::steady_clock::now();
    // right-hand sides per batch: all of them, unless the Krylov bases
    // (2 m + 1 vectors per level: FP64 and FP32 outer with m = restart, FP64
    // and FP32 nested with the nested dimension) would exceed the budget
    const int mi = nested_dim(o.restart, o.inner_max_iter);
    const bool augm = (bool)p->aug;
    const int64_t T = p->mesh.nt();
    const double Eo = augm ? (double)(E + T) : (double)E;   // outer unknowns per right-hand side
    const double per_rhs = Eo * (2.0 * o.restart + 1.0) * (augm ? 16.0 : 16.0 + 8.0) +
                           (double)E * (2.0 * mi + 1.0) * (16.0 + 8.0);
    if (augm && s.sg.n < (size_t)s.nrhs * T) s.sg.alloc((size_t)s.nrhs * T);
    const int nb = (int)std::max(1.0, std::min((double)s.nrhs, std::floor(kKrylovBudget / per_rhs)));
    for (int r0 = 0; r0 < s.nrhs; r0 += nb) {
        const int cnt = std::min(nb, s.nrhs - r0);
        Ops<double> o64(p, s, st, o.inner_tol, o.inner_max_iter, o.restart, cnt, !augm);
        o64.use_bj_in = (o.precond & 1) != 0;
        o64.use_bj_out = (o.precond & 2) != 0;
        o64.use_ras_in = (o.precond & 4) != 0 && s.sin.nc > 0;
        o64.use_lu_in = (o.precond & 16) != 0 && !s.nlu.empty();
        o64.skip_converged = o.keep_converged == 0;
        c128 *e = s.e.p + r0 * E, *u = s.u.p + r0 * E, *v = s.v.p + r0 * E;
        const int64_t NE = (int64_t)cnt * E;
        // Refinement sweeps: residual of the block equations in FP64, correction
        // from the nested GIBC solve.  SIE_FP32 delegates the interior work to
        // complex64 (the exterior products and outer Krylov vectors stay FP64:
        // at low frequency the k0 operator's vector potential is ~(k0 h)^2
        // below its scalar potential and does not survive FP32).
        std::unique_ptr<Ops<float>> o32;
        if (prec == SIE_FP32) {
            o32.reset(new Ops<float>(p, s, st, std::max(o.inner_tol, 1e-5), o.inner_max_iter, o.restart, cnt,
                                     !augm));
            o32->use_bj_in = o64.use_bj_in;
            o32->use_bj_out = o64.use_bj_out;
            o32->use_ras_in = o64.use_ras_in;
            o32->use_lu_in = o64.use_lu_in;
            o32->skip_converged = o64.skip_converged;
            o64.lo = o32.get();
        }
        SIE_HIP(hipMemsetAsync(u, 0, NE * sizeof(c128), st));
        SIE_HIP(hipMemsetAsync(v, 0, NE * sizeof(c128), st));
        std::vector<double> res(cnt, 1.0);
        if (augm) {
            refine_aug(p, s, o64, o32.get(), prec, o, e, u, v, s.sg.p + (int64_t)r0 * T, cnt, res, outer_total,
                       sweeps_total);
        } else {
        DBuf<c128> r1(NE), r2(NE), du(NE), dv(NE), sv(NE);
        std::vector<double> prev(cnt, 2.0);
        std::vector<char> done(cnt, 0);
        for (int sw = 0; sw <= o.max_refine; ++sw) {
            res = block_residual(o64, e, u, v, r1.p, r2.p);
            // a system stops at the tolerance, at the sweep cap, or when a
            // sweep no longer halves its residual (its outer system has
            // stagnated)
            bool all = true;
            std::vector<c128> keep(cnt);
            for (int k = 0; k < cnt; ++k) {
                if (!done[k] && (res[k] <= o.tol || sw == o.max_refine || res[k] > 0.5 * prev[k])) done[k] = 1;
                prev[k] = res[k];
                keep[k] = c128(done[k] ? 0.0 : 1.0);
                all = all && done[k];
            }
            if (all) break;
            ++sweeps_total;
            // finished systems take a zero correction
            Gmres<double> &g = s.go64;
            g.scale(keep, r1.p, r1.p, st);
            g.scale(keep, r2.p, r2.p, st);
            // s = Lhat^-1 r2 ; r1' = r1 + (K0 - X/2) s
            o64.inner_solve(r2.p, sv.p);
            o64.KpX(false, -1.0, sv.p, o64.t[3]);
            launch_axpby<double>(NE, c128(1.0), o64.t[3], c128(1.0), r1.p, st);
            SIE_HIP(hipMemsetAsync(du.p, 0, NE * sizeof(c128), st));
            // FP64: run through the plateaus of the low-frequency EFIE; FP32:
            // hand back when a correction stalls for longer than a plateau
            g.stag_window = prec == SIE_FP32 ? 100 : 0;
            // relative tolerance of each correction solve: what is left to the
            // target, but in FP32 (its interior products carry FP32 rounding)
            // no tighter than 0.63 sqrt(tol), so that two sweeps reach tol
            // with a margin of 2.5, clamped to [2e-4, 1e-3] (tighter FP32
            // corrections of the low-frequency EFIE stall and cost a sweep)
            const double floor32 = std::min(1e-3, std::max(2e-4, 0.63 * std::sqrt(o.tol)));
            std::vector<double> stol(cnt);
            for (int k = 0; k < cnt; ++k) {
                const double need = res[k] > 0.0 ? o.tol / res[k] : 1.0;
                stol[k] = prec == SIE_FP32 ? std::max(need, floor32) : need;
            }
            if (o.inner_relax > 0.0) set_relax(o64, o32.get(), o.inner_relax, stol, &g.live);
            outer_total += g.solve([&](const c128 *x, c128 *y) { o64.gibc(x, y); },
                                   [&](const c128 *x, c128 *y) { o64.prec_outer(x, y); }, r1.p, du.p, stol,
                                   o.max_iter, nullptr, st, nullptr, true);
            set_relax(o64, o32.get(), 0.0, stol, nullptr);
            // dv = Lhat^-1 (r2 + (K_i + X/2) du)
            o64.KpX(true, +1.0, du.p, o64.t[3]);
            launch_axpby<double>(NE, c128(1.0), r2.p, c128(1.0), o64.t[3], st);
            o64.inner_solve(o64.t[3], dv.p);
            launch_axpby<double>(NE, c128(1.0), du.p, c128(1.0), u, st);
            launch_axpby<double>(NE, c128(1.0), dv.p, c128(1.0), v, st);
        }
        }
        o64.lo = nullptr;
        for (int k = 0; k < cnt; ++k) {
            worst = std::max(worst, res[k]);
            if (!(res[k] <= o.tol)) all_conv = false;
        }
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
        rep->k_matvecs = s.kmatvecs;
        rep->t_setup_s = p->t_setup_s;
        rep->device_bytes = estimate_footprint(p, o.restart, o.inner_max_iter);
        rep->residual = worst;
        rep->t_solve_s = dt;
    }
    if (!all_conv) throw Error(SIE_ENOCONV, "residual " + std::to_string(worst) + " above tolerance");
}

}  // namespace sie

namespace sie {
template <typename T>
static void nested_precond_apply(sie_problem *p, SolveState &s, int precond, int nrhs, const cx<T> *x, cx<T> *y,
                                 hipStream_t st) {
    const int64_t E = p->mesh.nrwg;
    if (precond & (4 | 16)) {
        nested_apply<T>(p, s, (precond & 4) != 0, (precond & 16) != 0, nrhs, x, y, st);
    } else {
        for (int k = 0; k < nrhs; ++k)
            launch_bj_apply<T>(s.pin.nb, s.pin.B, s.pin.perm.p, bj_inv<T>(s.pin), x + k * E, y + k * E, st);
    }
}

void nested_precond_entry(sie_problem *p, int precond, sie_precision prec, int nrhs, const void *x, void *y,
                          hipStream_t st) {
    SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
    SIE_CHECK(precond == 1 || precond == 4 || precond == 12 || precond == 16 || precond == 20 || precond == 28,
              SIE_EINVAL,
              "nested preconditioner must be 1 (block-Jacobi), 4 or 12 (Schwarz clusters), 16 (near-region LU), "
              "20 or 28 (LU where it applies, Schwarz clusters elsewhere)");
    SIE_CHECK(x && y && nrhs >= 1, SIE_EINVAL, "bad vectors");
    SIE_CHECK(x != y, SIE_EINVAL, "x and y must not alias");
    SIE_CHECK(prec == SIE_FP64 || prec == SIE_FP32, SIE_EINVAL, "unknown precision");
    if (!p->solve) p->solve = new SolveState;
    SolveState &s = *p->solve;
    build_preconditioners(p, s, precond);
    if (prec == SIE_FP64)
        nested_precond_apply<double>(p, s, precond, nrhs, (const c128 *)x, (c128 *)y, st);
    else
        nested_precond_apply<float>(p, s, precond, nrhs, (const c64 *)x, (c64 *)y, st);
}

int nested_precond_factored(const sie_problem *p, int64_t *factor_nnz, double *t_factor_s) {
    if (!p->solve || !p->solve->nlu_built) return -1;
    if (factor_nnz) *factor_nnz = p->solve->nlu_nnz;
    if (t_factor_s) *t_factor_s = p->solve->nlu_factor_s;
    return (int)p->solve->nlu.size();
}

int nested_precond_clusters(const sie_problem *p, int64_t *owned) {
    if (!p->solve || !p->solve->sin_built) return -1;
    if (owned) *owned = p->solve->sin.owned;
    return p->solve->sin.nc;
}

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
    SIE_HIP(hipStreamSynchronize(0));
}
}  // namespace sie

namespace sie {
void solve_entry(sie_problem *p, sie_precision prec, const sie_solver_opts *opts, sie_report *rep) {
    SIE_CHECK(p && p->is_setup, SIE_ESTATE, "problem not set up");
    SIE_CHECK(p->solve && p->solve->nrhs > 0, SIE_ESTATE, "no plane waves set");
    SIE_CHECK(prec == SIE_FP64 || prec == SIE_FP32, SIE_EINVAL, "unknown precision");
    sie_solver_opts o{1e-6, 1e-8, 100, 800, 800, 10, 0, 0.0, 0};
    if (opts) {
        if (opts->tol > 0) o.tol = opts->tol;
        if (opts->inner_tol > 0) o.inner_tol = opts->inner_tol;
        if (opts->restart > 0) o.restart = opts->restart;
        if (opts->max_iter > 0) o.max_iter = opts->max_iter;
        if (opts->inner_max_iter > 0) o.inner_max_iter = opts->inner_max_iter;
        if (opts->max_refine > 0) o.max_refine = opts->max_refine;
        o.precond = opts->precond;
        SIE_CHECK(opts->inner_relax >= 0.0, SIE_EINVAL, "inner_relax must be non-negative");
        o.inner_relax = opts->inner_relax;
        SIE_CHECK(opts->keep_converged == 0 || opts->keep_converged == 1, SIE_EINVAL, "keep_converged must be 0 or 1");
        o.keep_converged = opts->keep_converged;
    }
    SIE_CHECK(!(o.precond & 8) || (o.precond & 4), SIE_EINVAL, "preconditioner bit 8 extends bit 4");
    SIE_CHECK((o.precond & 5) != 5, SIE_EINVAL, "nested block-Jacobi (1) and nested Schwarz clusters (4) exclude each other");
    SIE_CHECK((o.precond & 17) != 17, SIE_EINVAL,
              "nested block-Jacobi (1) and the near-region LU (16) exclude each other");
    SIE_CHECK(o.precond >= 0 && o.precond < 32, SIE_EINVAL, "unknown preconditioner bits");
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

void charges_entry(const sie_problem *p, int32_t rhs, sie_c128 *sg) {
    SIE_CHECK(p && p->solve && p->solve->solved, SIE_ESTATE, "no solution");
    SIE_CHECK(p->aug, SIE_ESTATE, "problem not set up for the augmented EFIE");
    SIE_CHECK(rhs >= 0 && rhs < p->solve->nrhs, SIE_EINVAL, "rhs out of range");
    SIE_CHECK(sg, SIE_EINVAL, "NULL output");
    const int64_t T = p->mesh.nt();
    SIE_HIP(hipMemcpy(sg, p->solve->sg.p + rhs * T, T * sizeof(c128), hipMemcpyDeviceToHost));
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
