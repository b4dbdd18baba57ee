// Multifrontal LU without pivoting in nested-dissection order (host, FP64).
//
// Ordering: the unknowns are bisected recursively at the median of the
// longest extent of their bounding box; the unknowns of the lower half with a
// neighbour in the upper half form the separator, numbered after both halves
// (leaves of at most kLeaf unknowns are numbered as they come).  Every
// separator and leaf is a supernode; a supernode's level is its height in the
// dissection tree, so supernodes of one level are never ancestor and
// descendant of each other.
//
// Factorisation: each supernode N assembles a dense front over its own
// positions and its boundary B (later positions coupled to N directly or
// through its descendants), eliminates its own positions (no pivoting: the
// matrices factored here are shifted surface Laplacians, diagonally dominant
// up to one eigenvalue per object that the shift moves off zero) and hands
// the Schur complement on B to its parent.  Kept: the inverses of the
// diagonal blocks L_NN (unit lower) and U_NN, and the blocks L_BN, U_NB,
// stored by rows so that a device solve gathers what a row needs:
//   forward  y_N = L_NN^-1 (b_N - sum_{descendants D} L_ND y_D)
//   backward x_N = U_NN^-1 (y_N - U_NB x_B)
// Supernodes of one level run concurrently on the host and on the device.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <exception>
#include <limits>
#include <mutex>
#include <thread>

#include "sparse_lu.h"

namespace sie {
namespace {

constexpr int kLeaf = 64;

struct Node {
    int p0 = 0, n = 0, height = 0;
    std::vector<int> children;
};

struct Dissection {
    const std::vector<int64_t> &rp;
    const std::vector<int32_t> &ci;
    const std::vector<double> &xyz;
    std::vector<int32_t> order;   // position -> unknown
    std::vector<Node> nodes;      // children before parents; the root is last
    std::vector<int64_t> mark;
    int64_t stamp = 0;

    Dissection(const std::vector<int64_t> &r, const std::vector<int32_t> &c, const std::vector<double> &x, int64_t n)
        : rp(r), ci(c), xyz(x), mark(n, -1) {}

    int build(std::vector<int32_t> &v) {
        Node nd;
        if ((int64_t)v.size() <= kLeaf) {
            nd.p0 = (int)order.size();
            nd.n = (int)v.size();
            order.insert(order.end(), v.begin(), v.end());
            nodes.push_back(nd);
            return (int)nodes.size() - 1;
        }
        double lo[3], hi[3];
        for (int c = 0; c < 3; ++c) { lo[c] = std::numeric_limits<double>::infinity(); hi[c] = -lo[c]; }
        for (int32_t u : v)
            for (int c = 0; c < 3; ++c) {
                lo[c] = std::min(lo[c], xyz[3 * (int64_t)u + c]);
                hi[c] = std::max(hi[c], xyz[3 * (int64_t)u + c]);
            }
        int ax = 0;
        for (int c = 1; c < 3; ++c)
            if (hi[c] - lo[c] > hi[ax] - lo[ax]) ax = c;
        const size_t mid = v.size() / 2;
        std::nth_element(v.begin(), v.begin() + mid, v.end(), [&](int32_t a, int32_t b) {
            const double xa = xyz[3 * (int64_t)a + ax], xb = xyz[3 * (int64_t)b + ax];
            return xa < xb || (xa == xb && a < b);
        });
        const int64_t s = ++stamp;
        for (size_t i = 0; i < v.size(); ++i) mark[v[i]] = 2 * s + (i < mid ? 0 : 1);
        std::vector<int32_t> left, right(v.begin() + mid, v.end()), sep;
        for (size_t i = 0; i < mid; ++i) {
            const int32_t u = v[i];
            bool cut = false;
            for (int64_t k = rp[u]; k < rp[u + 1] && !cut; ++k) cut = mark[ci[k]] == 2 * s + 1;
            (cut ? sep : left).push_back(u);
        }
        std::vector<int32_t>().swap(v);
        if (!left.empty()) nd.children.push_back(build(left));
        if (!right.empty()) nd.children.push_back(build(right));
        nd.p0 = (int)order.size();
        nd.n = (int)sep.size();
        SIE_CHECK(nd.n <= kLUMaxSupernode, SIE_EINVAL,
                  "sparse LU: separator of " + std::to_string(nd.n) + " unknowns exceeds " +
                      std::to_string(kLUMaxSupernode));
        order.insert(order.end(), sep.begin(), sep.end());
        for (int c : nd.children) nd.height = std::max(nd.height, nodes[c].height + 1);
        nodes.push_back(nd);
        return (int)nodes.size() - 1;
    }
};

struct Factor {
    std::vector<int32_t> B;        // boundary positions (ascending)
    std::vector<c128> upd;         // |B| x |B| Schur complement for the parent
    std::vector<c128> linv, uinv;  // n x n
    std::vector<c128> lb, ub;      // |B| x n and n x |B|
};

// Dense front of supernode `id`: assemble, eliminate its own positions.
void factor_node(int id, const std::vector<Node> &nodes, std::vector<Factor> &fac, const std::vector<int32_t> &order,
                 const std::vector<int32_t> &iperm, const std::vector<int64_t> &rp, const std::vector<int32_t> &ci,
                 const std::vector<c128> &val) {
    const Node &nd = nodes[id];
    const int n = nd.n, p0 = nd.p0, p1 = p0 + n;
    Factor &f = fac[id];
    std::vector<int32_t> B;
    for (int i = p0; i < p1; ++i) {
        const int32_t u = order[i];
        for (int64_t k = rp[u]; k < rp[u + 1]; ++k)
            if (iperm[ci[k]] >= p1) B.push_back(iperm[ci[k]]);
    }
    for (int c : nd.children)
        for (int32_t b : fac[c].B)
            if (b >= p1) B.push_back(b);
    std::sort(B.begin(), B.end());
    B.erase(std::unique(B.begin(), B.end()), B.end());
    const int nb = (int)B.size(), m = n + nb;
    auto loc = [&](int32_t pos) -> int {
        if (pos < p1) return pos - p0;
        return n + (int)(std::lower_bound(B.begin(), B.end(), pos) - B.begin());
    };
    std::vector<c128> F((size_t)m * m);
    // original entries whose smaller position lies in N
    for (int i = p0; i < p1; ++i) {
        const int32_t u = order[i];
        for (int64_t k = rp[u]; k < rp[u + 1]; ++k) {
            const int32_t pj = iperm[ci[k]];
            if (pj < p0) continue;
            F[(size_t)loc(i) * m + loc(pj)] += val[k];
            if (pj >= p1) {   // the transposed entry (row in B, column in N)
                const int32_t w = ci[k];
                const int32_t *b0 = ci.data() + rp[w], *b1 = ci.data() + rp[w + 1];
                const int32_t *q = std::lower_bound(b0, b1, u);
                SIE_CHECK(q != b1 && *q == u, SIE_EINVAL, "sparse LU: pattern not structurally symmetric");
                F[(size_t)loc(pj) * m + loc(i)] += val[q - ci.data()];
            }
        }
    }
    // children's Schur complements
    for (int c : nd.children) {
        Factor &fc = fac[c];
        const int bc = (int)fc.B.size();
        std::vector<int> lc(bc);
        for (int a = 0; a < bc; ++a) lc[a] = loc(fc.B[a]);
        for (int a = 0; a < bc; ++a)
            for (int b = 0; b < bc; ++b) F[(size_t)lc[a] * m + lc[b]] += fc.upd[(size_t)a * bc + b];
        std::vector<c128>().swap(fc.upd);
    }
    // eliminate the n own positions
    for (int k = 0; k < n; ++k) {
        const c128 piv = F[(size_t)k * m + k];
        const double pa = std::hypot(piv.re, piv.im);
        SIE_CHECK(pa > 0.0 && std::isfinite(pa), SIE_EINVAL, "sparse LU: zero pivot");
        const c128 ip = cdiv(c128(1.0), piv);
        for (int i = k + 1; i < m; ++i) F[(size_t)i * m + k] = F[(size_t)i * m + k] * ip;
        const c128 *fk = &F[(size_t)k * m];
        for (int i = k + 1; i < m; ++i) {
            const c128 l = F[(size_t)i * m + k];
            if (l.re == 0.0 && l.im == 0.0) continue;
            c128 *fi = &F[(size_t)i * m];
            for (int j = k + 1; j < m; ++j) {
                fi[j].re -= l.re * fk[j].re - l.im * fk[j].im;
                fi[j].im -= l.re * fk[j].im + l.im * fk[j].re;
            }
        }
    }
    // inverses of the diagonal blocks
    f.linv.assign((size_t)n * n, c128());
    f.uinv.assign((size_t)n * n, c128());
    for (int c = 0; c < n; ++c) {
        f.linv[(size_t)c * n + c] = c128(1.0);
        for (int i = c + 1; i < n; ++i) {
            c128 s;
            for (int k = c; k < i; ++k) s += F[(size_t)i * m + k] * f.linv[(size_t)k * n + c];
            f.linv[(size_t)i * n + c] = -s;
        }
        f.uinv[(size_t)c * n + c] = cdiv(c128(1.0), F[(size_t)c * m + c]);
        for (int i = c - 1; i >= 0; --i) {
            c128 s;
            for (int k = i + 1; k <= c; ++k) s += F[(size_t)i * m + k] * f.uinv[(size_t)k * n + c];
            f.uinv[(size_t)i * n + c] = cdiv(-s, F[(size_t)i * m + i]);
        }
    }
    f.lb.resize((size_t)nb * n);
    f.ub.resize((size_t)n * nb);
    for (int a = 0; a < nb; ++a)
        for (int k = 0; k < n; ++k) f.lb[(size_t)a * n + k] = F[(size_t)(n + a) * m + k];
    for (int k = 0; k < n; ++k)
        for (int b = 0; b < nb; ++b) f.ub[(size_t)k * nb + b] = F[(size_t)k * m + n + b];
    f.upd.resize((size_t)nb * nb);
    for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) f.upd[(size_t)a * nb + b] = F[(size_t)(n + a) * m + n + b];
    f.B = std::move(B);
}

}  // namespace

void lu_factor_host(SparseLUHost &h, int64_t n, const std::vector<int64_t> &rp, const std::vector<int32_t> &ci,
                    const std::vector<c128> &val, const std::vector<double> &coords) {
    SIE_CHECK(n > 0 && n < (int64_t(1) << 31), SIE_EINVAL, "sparse LU: bad size");
    SIE_CHECK((int64_t)rp.size() == n + 1 && (int64_t)coords.size() == 3 * n, SIE_EINVAL, "sparse LU: bad input");
    Dissection nd(rp, ci, coords, n);
    {
        std::vector<int32_t> all(n);
        for (int64_t i = 0; i < n; ++i) all[i] = (int32_t)i;
        nd.build(all);
    }
    SIE_CHECK((int64_t)nd.order.size() == n, SIE_EINVAL, "sparse LU: dissection lost unknowns");
    std::vector<int32_t> iperm(n);
    for (int64_t p = 0; p < n; ++p) iperm[nd.order[p]] = (int32_t)p;
    const int nn = (int)nd.nodes.size();
    int H = 0;
    for (const Node &x : nd.nodes) H = std::max(H, x.height + 1);
    std::vector<std::vector<int>> by_level(H);
    for (int i = 0; i < nn; ++i) by_level[nd.nodes[i].height].push_back(i);
    // numeric factorisation, the supernodes of a level in parallel
    std::vector<Factor> fac(nn);
    const int nthr = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    for (int l = 0; l < H; ++l) {
        const std::vector<int> &lv = by_level[l];
        std::atomic<size_t> next{0};
        std::exception_ptr err;
        std::mutex emu;
        auto work = [&]() {
            for (;;) {
                const size_t i = next.fetch_add(1);
                if (i >= lv.size()) return;
                try {
                    factor_node(lv[i], nd.nodes, fac, nd.order, iperm, rp, ci, val);
                } catch (...) {
                    std::lock_guard<std::mutex> lk(emu);
                    if (!err) err = std::current_exception();
                }
            }
        };
        const int nt = (int)std::min<size_t>(nthr, lv.size());
        std::vector<std::thread> th;
        for (int t = 1; t < nt; ++t) th.emplace_back(work);
        work();
        for (auto &t : th) t.join();
        if (err) std::rethrow_exception(err);
    }
    // device layout
    std::vector<int64_t> lcnt(n + 1, 0), ucnt(n + 1, 0);
    for (int id = 0; id < nn; ++id) {
        const Node &x = nd.nodes[id];
        for (int32_t b : fac[id].B) lcnt[b + 1] += x.n;
        for (int k = 0; k < x.n; ++k) ucnt[x.p0 + k + 1] += (int64_t)fac[id].B.size();
    }
    for (int64_t i = 0; i < n; ++i) { lcnt[i + 1] += lcnt[i]; ucnt[i + 1] += ucnt[i]; }
    std::vector<int32_t> lcol(lcnt[n]), ucol(ucnt[n]);
    std::vector<c128> lval(lcnt[n]), uval(ucnt[n]);
    std::vector<int64_t> lfill(lcnt.begin(), lcnt.end() - 1), ufill(ucnt.begin(), ucnt.end() - 1);
    std::vector<int32_t> sn_p0(nn), sn_n(nn);
    std::vector<int64_t> inv_off(nn);
    int64_t inv_total = 0;
    int max_sn = 0;
    for (int id = 0; id < nn; ++id) {
        const Node &x = nd.nodes[id];
        const Factor &fc = fac[id];
        const int nb = (int)fc.B.size();
        for (int a = 0; a < nb; ++a)
            for (int k = 0; k < x.n; ++k) {
                const int64_t q = lfill[fc.B[a]]++;
                lcol[q] = x.p0 + k;
                lval[q] = fc.lb[(size_t)a * x.n + k];
            }
        for (int k = 0; k < x.n; ++k)
            for (int b = 0; b < nb; ++b) {
                const int64_t q = ufill[x.p0 + k]++;
                ucol[q] = fc.B[b];
                uval[q] = fc.ub[(size_t)k * nb + b];
            }
        sn_p0[id] = x.p0;
        sn_n[id] = x.n;
        inv_off[id] = inv_total;
        inv_total += (int64_t)x.n * x.n;
        max_sn = std::max(max_sn, x.n);
    }
    std::vector<c128> linv(std::max<int64_t>(inv_total, 1)), uinv(std::max<int64_t>(inv_total, 1));
    for (int id = 0; id < nn; ++id) {
        std::copy(fac[id].linv.begin(), fac[id].linv.end(), linv.begin() + inv_off[id]);
        std::copy(fac[id].uinv.begin(), fac[id].uinv.end(), uinv.begin() + inv_off[id]);
    }
    h.lev_ptr.assign(1, 0);
    h.lev_sn.clear();
    for (int l = 0; l < H; ++l) {
        for (int id : by_level[l])
            if (nd.nodes[id].n > 0) h.lev_sn.push_back(id);
        h.lev_ptr.push_back((int)h.lev_sn.size());
    }
    h.n = n;
    h.sn_p0 = std::move(sn_p0);
    h.sn_n = std::move(sn_n);
    h.inv_off = std::move(inv_off);
    h.linv = std::move(linv);
    h.uinv = std::move(uinv);
    h.lrow_ptr = std::move(lcnt);
    h.urow_ptr = std::move(ucnt);
    h.lcol = std::move(lcol);
    h.ucol = std::move(ucol);
    h.lval = std::move(lval);
    h.uval = std::move(uval);
    h.perm = std::move(nd.order);
    h.iperm = std::move(iperm);
    (void)max_sn;
}

void lu_upload(const SparseLUHost &h, SparseLU &f) {
    auto up = [](auto &d, const auto &v, auto zero) {
        if (v.empty()) d.upload(&zero, 1);
        else d.upload(v);
    };
    f.n = h.n;
    f.nsn = (int)h.sn_n.size();
    f.max_sn = 0;
    for (int32_t x : h.sn_n) f.max_sn = std::max(f.max_sn, (int)x);
    f.nnz_factor = (int64_t)h.lcol.size() + (int64_t)h.ucol.size();
    f.lev_ptr = h.lev_ptr;
    up(f.lev_sn, h.lev_sn, int32_t(0));
    up(f.sn_p0, h.sn_p0, int32_t(0));
    up(f.sn_n, h.sn_n, int32_t(0));
    up(f.inv_off, h.inv_off, int64_t(0));
    up(f.linv, h.linv, c128());
    up(f.uinv, h.uinv, c128());
    up(f.lrow_ptr, h.lrow_ptr, int64_t(0));
    up(f.urow_ptr, h.urow_ptr, int64_t(0));
    up(f.lcol, h.lcol, int32_t(0));
    up(f.ucol, h.ucol, int32_t(0));
    up(f.lval, h.lval, c128());
    up(f.uval, h.uval, c128());
    up(f.perm, h.perm, int32_t(0));
    up(f.iperm, h.iperm, int32_t(0));
    std::vector<int32_t> bsn, brow;
    f.blk_ptr.assign(1, 0);
    for (size_t l = 0; l + 1 < h.lev_ptr.size(); ++l) {
        for (int q = h.lev_ptr[l]; q < h.lev_ptr[l + 1]; ++q) {
            const int32_t sn = h.lev_sn[q];
            for (int r = 0; r < h.sn_n[sn]; r += kLURowsPerBlock) {
                bsn.push_back(sn);
                brow.push_back(r);
            }
        }
        f.blk_ptr.push_back((int)bsn.size());
    }
    up(f.blk_sn, bsn, int32_t(0));
    up(f.blk_row0, brow, int32_t(0));
}

void lu_solve_host(const SparseLUHost &h, c128 *x) {
    const int64_t n = h.n;
    std::vector<c128> y(n), t;
    for (int64_t p = 0; p < n; ++p) y[p] = x[h.perm[p]];
    const int H = (int)h.lev_ptr.size() - 1;
    auto level = [&](int l, bool fwd) {
        const std::vector<int64_t> &rp = fwd ? h.lrow_ptr : h.urow_ptr;
        const std::vector<int32_t> &cc = fwd ? h.lcol : h.ucol;
        const std::vector<c128> &vv = fwd ? h.lval : h.uval;
        const std::vector<c128> &inv = fwd ? h.linv : h.uinv;
        for (int q = h.lev_ptr[l]; q < h.lev_ptr[l + 1]; ++q) {
            const int sn = h.lev_sn[q], p0 = h.sn_p0[sn], nn = h.sn_n[sn];
            t.assign(nn, c128());
            for (int i = 0; i < nn; ++i) {
                c128 acc = y[p0 + i];
                for (int64_t j = rp[p0 + i]; j < rp[p0 + i + 1]; ++j) acc -= vv[j] * y[cc[j]];
                t[i] = acc;
            }
            const c128 *M = inv.data() + h.inv_off[sn];
            for (int i = 0; i < nn; ++i) {
                c128 s;
                for (int k = fwd ? 0 : i; k < (fwd ? i + 1 : nn); ++k) s += M[(int64_t)i * nn + k] * t[k];
                y[p0 + i] = s;
            }
        }
    };
    for (int l = 0; l < H; ++l) level(l, true);
    for (int l = H - 1; l >= 0; --l) level(l, false);
    for (int64_t p = 0; p < n; ++p) x[h.perm[p]] = y[p];
}

void lu_solve(const SparseLU &f, int nrhs, c128 *x, hipStream_t st) {
    if (f.work.n < (size_t)nrhs * f.n) f.work.alloc((size_t)nrhs * f.n);
    const int H = (int)f.lev_ptr.size() - 1;
    for (int l = 0; l < H; ++l) launch_lu_level(f, l, true, nrhs, x, st);
    for (int l = H - 1; l >= 0; --l) launch_lu_level(f, l, false, nrhs, x, st);
}

}  // namespace sie
