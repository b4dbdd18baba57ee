// Multifrontal LU without pivoting in nested-dissection order (FP64): the
// ordering and the symbolic factorisation on the host, the numeric
// factorisation on the device.
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
// up to one eigenvalue per object that the shift moves off zero, and
// near-region operators dominated by their self and neighbour terms) and
// hands the Schur complement on B to its parent.  The symbolic pass finds
// every B first, so that the size of the factors and the arithmetic are
// known (and refused beyond the limits) before any front is factored, and
// lays out where every result goes; the fronts then run on the device in
// postorder (k_front.hip), their update matrices on a stack, or, when every
// front is small, on the host (the supernodes of a level in parallel).  Kept: the
// inverses of the diagonal blocks L_NN (unit lower) and U_NN, and the blocks
// L_BN, U_NB, stored by rows so that a device solve gathers what a row
// needs:
//   forward  y_N = L_NN^-1 (b_N - sum_{descendants D} L_ND y_D)
//   backward x_N = U_NN^-1 (y_N - U_NB x_B)
// Supernodes of one level run concurrently in the device solve.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <exception>
#include <limits>
#include <mutex>
#include <thread>

#include "sparse_lu.h"

namespace sie {
namespace {

constexpr int kLeaf = 128;

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

// Boundary of supernode `id` (its children's already found): the later
// positions coupled to its own directly or through a child's boundary.
// mark [n] holds, per position, the last supernode that listed it.
void front_boundary(int id, const std::vector<Node> &nodes, std::vector<std::vector<int32_t>> &Bs,
                    const std::vector<int32_t> &order, const std::vector<int32_t> &iperm,
                    const std::vector<int64_t> &rp, const std::vector<int32_t> &ci, std::vector<int32_t> &mark) {
    const Node &nd = nodes[id];
    const int p1 = nd.p0 + nd.n;
    std::vector<int32_t> &B = Bs[id];
    B.clear();
    auto add = [&](int32_t pos) {
        if (pos >= p1 && mark[pos] != id) {
            mark[pos] = id;
            B.push_back(pos);
        }
    };
    for (int i = nd.p0; i < p1; ++i) {
        const int32_t u = order[i];
        for (int64_t k = rp[u]; k < rp[u + 1]; ++k) add(iperm[ci[k]]);
    }
    for (int c : nd.children)
        for (int32_t b : Bs[c]) add(b);
    std::sort(B.begin(), B.end());
}

// f(i, t) for i in [0, count) on up to 16 host threads (t: the thread's
// index); the first exception is rethrown once all have joined.
template <typename F>
void parallel_for(int64_t count, int nthr, F &&f) {
    std::atomic<int64_t> next{0};
    std::exception_ptr err;
    std::mutex emu;
    auto work = [&](int t) {
        for (;;) {
            const int64_t i = next.fetch_add(1);
            if (i >= count) return;
            try {
                f(i, t);
            } catch (...) {
                std::lock_guard<std::mutex> lk(emu);
                if (!err) err = std::current_exception();
            }
        }
    };
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(nthr, count));
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(work, t);
    work(0);
    for (auto &t : th) t.join();
    if (err) std::rethrow_exception(err);
}

int host_threads() { return (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency())); }

// Dense elimination of the first n positions of the m x m front F on the
// host (the small fronts): the same results as the device's, multipliers of
// zero skipped.
void eliminate_host(c128 *F, int m, int n, c128 *linv, c128 *uinv) {
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
    for (int c = 0; c < n; ++c) {
        linv[(size_t)c * n + c] = c128(1.0);
        for (int i = c + 1; i < n; ++i) {
            c128 s;
            for (int k = c; k < i; ++k) s += F[(size_t)i * m + k] * linv[(size_t)k * n + c];
            linv[(size_t)i * n + c] = -s;
        }
        uinv[(size_t)c * n + c] = cdiv(c128(1.0), F[(size_t)c * m + c]);
        for (int i = c - 1; i >= 0; --i) {
            c128 s;
            for (int k = i + 1; k <= c; ++k) s += F[(size_t)i * m + k] * uinv[(size_t)k * n + c];
            uinv[(size_t)i * n + c] = cdiv(-s, F[(size_t)i * m + i]);
        }
    }
}

}  // namespace

void lu_factor(SparseLU &f, int64_t n, const std::vector<int64_t> &rp, const std::vector<int32_t> &ci,
               const std::vector<c128> &val, const std::vector<double> &coords, hipStream_t st) {
    SIE_CHECK(n > 0 && n < (int64_t(1) << 31), SIE_EINVAL, "sparse LU: bad size");
    SIE_CHECK((int64_t)rp.size() == n + 1 && (int64_t)coords.size() == 3 * n, SIE_EINVAL, "sparse LU: bad input");
    SIE_CHECK(rp[n] < (int64_t(1) << 31) && (int64_t)ci.size() == rp[n] && val.size() == ci.size(), SIE_EINVAL,
              "sparse LU: bad input");
    const auto t0 = std::chrono::steady_clock::now();
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
    const std::vector<Node> &nodes = nd.nodes;

    // symbolic factorisation: every front's boundary, the factors' size and
    // the arithmetic of the elimination (complex multiply-adds of 8 flops:
    // n m^2 - n^2 m + n^3 / 3 for the front, n^3 / 3 for the two inverses)
    std::vector<std::vector<int32_t>> Bs(nn);
    double bytes = 0.0, flops = 0.0;
    int64_t max_mm = 1;
    std::vector<int32_t> mark(n, -1);
    for (int id = 0; id < nn; ++id) {
        front_boundary(id, nodes, Bs, nd.order, iperm, rp, ci, mark);
        const double a = nodes[id].n, b = (double)Bs[id].size(), m = a + b;
        bytes += 16.0 * (2.0 * a * a + 2.0 * a * b);
        flops += 8.0 * (a * m * m - a * a * m + 2.0 * a * a * a / 3.0);
        max_mm = std::max<int64_t>(max_mm, (int64_t)(a + b) * (int64_t)(a + b));
    }
    SIE_CHECK(bytes <= kLUMaxBytes && flops <= kLUMaxFlops, SIE_EINVAL,
              "sparse LU: factors of " + std::to_string(bytes / 1e9) + " GB and " + std::to_string(flops / 1e12) +
                  " Tflop exceed the limits");

    // where each front's results go: rows of L gather the boundary rows of
    // every descendant front, rows of U the boundary of their own front
    std::vector<int64_t> lcnt(n + 1, 0), ucnt(n + 1, 0);
    for (int id = 0; id < nn; ++id) {
        for (int32_t b : Bs[id]) lcnt[b + 1] += nodes[id].n;
        for (int k = 0; k < nodes[id].n; ++k) ucnt[nodes[id].p0 + k + 1] += (int64_t)Bs[id].size();
    }
    for (int64_t i = 0; i < n; ++i) { lcnt[i + 1] += lcnt[i]; ucnt[i + 1] += ucnt[i]; }
    std::vector<int32_t> lcol(lcnt[n]), ucol(ucnt[n]);
    std::vector<int64_t> lfill(lcnt.begin(), lcnt.end() - 1);
    std::vector<int64_t> loff;                     // per front and boundary row: first L entry
    std::vector<int64_t> loff0(nn + 1, 0), inv_off(nn, 0), upd_off(nn, 0);
    std::vector<int32_t> sn_p0(nn), sn_n(nn);
    int64_t inv_total = 0, top = 0, peak = 1;
    for (int id = 0; id < nn; ++id) {
        const Node &x = nodes[id];
        const std::vector<int32_t> &B = Bs[id];
        const int nb = (int)B.size();
        for (int a = 0; a < nb; ++a) {
            loff.push_back(lfill[B[a]]);
            lfill[B[a]] += x.n;
        }
        loff0[id + 1] = (int64_t)loff.size();
        sn_p0[id] = x.p0;
        sn_n[id] = x.n;
        inv_off[id] = inv_total;
        inv_total += (int64_t)x.n * x.n;
        // update matrices on a stack: a front's children (consecutive
        // subtrees just before it) left theirs on top; it pops them once
        // assembled and pushes its own
        if (!x.children.empty()) top = upd_off[x.children.front()];
        upd_off[id] = top;
        top += (int64_t)nb * nb;
        peak = std::max(peak, top);
    }
    const int nthr = host_threads();
    // column indices of the factors (each front fills its own ranges)
    parallel_for(nn, nthr, [&](int64_t id, int) {
        const Node &x = nodes[id];
        const std::vector<int32_t> &B = Bs[id];
        const int64_t *lo = loff.data() + loff0[id];
        for (size_t a = 0; a < B.size(); ++a)
            for (int k = 0; k < x.n; ++k) lcol[lo[a] + k] = x.p0 + k;
        for (int k = 0; k < x.n; ++k) std::copy(B.begin(), B.end(), ucol.begin() + ucnt[x.p0 + k]);
    });
    // assembly lists: original entries (front-local row, column, value
    // index; every entry lands in exactly one front position) and the
    // positions of each child's boundary in its parent's front; counted
    // first, then filled per front
    std::vector<int64_t> asm0(nn + 1, 0), map0(nn + 1, 0);
    parallel_for(nn, nthr, [&](int64_t id, int) {
        const Node &x = nodes[id];
        const int p0 = x.p0, p1 = p0 + x.n;
        int64_t cnt = 0;
        for (int i = p0; i < p1; ++i) {
            const int32_t u = nd.order[i];
            for (int64_t k = rp[u]; k < rp[u + 1]; ++k) {
                const int32_t pj = iperm[ci[k]];
                if (pj >= p0) cnt += pj >= p1 ? 2 : 1;
            }
        }
        asm0[id + 1] = cnt;
        int64_t mc = 0;
        for (int c : x.children) mc += (int64_t)Bs[c].size();
        map0[id + 1] = mc;
    });
    for (int id = 0; id < nn; ++id) {
        asm0[id + 1] += asm0[id];
        map0[id + 1] += map0[id];
    }
    std::vector<int32_t> arow(asm0[nn]), acol(asm0[nn]), asrc(asm0[nn]), cmap(map0[nn]);
    std::vector<std::vector<int32_t>> lmap(nthr);   // per thread: front-local index of a boundary position
    parallel_for(nn, nthr, [&](int64_t id, int t) {
        const Node &x = nodes[id];
        const std::vector<int32_t> &B = Bs[id];
        const int p0 = x.p0, p1 = p0 + x.n;
        std::vector<int32_t> &mk = lmap[t];
        if (mk.size() != (size_t)n) mk.assign(n, -1);
        for (int a = 0; a < (int)B.size(); ++a) mk[B[a]] = x.n + a;
        auto loc = [&](int32_t pos) -> int32_t { return pos < p1 ? pos - p0 : mk[pos]; };
        int64_t e = asm0[id];
        for (int i = p0; i < p1; ++i) {
            const int32_t u = nd.order[i];
            for (int64_t k = rp[u]; k < rp[u + 1]; ++k) {
                const int32_t pj = iperm[ci[k]];
                if (pj < p0) continue;
                arow[e] = loc(i);
                acol[e] = loc(pj);
                asrc[e++] = (int32_t)k;
                if (pj >= p1) {   // the transposed entry (row in B, column in N)
                    const int32_t w = ci[k];
                    const int32_t *b0 = ci.data() + rp[w], *b1 = ci.data() + rp[w + 1];
                    const int32_t *q = std::lower_bound(b0, b1, u);
                    SIE_CHECK(q != b1 && *q == u, SIE_EINVAL, "sparse LU: pattern not structurally symmetric");
                    arow[e] = loc(pj);
                    acol[e] = loc(i);
                    asrc[e++] = (int32_t)(q - ci.data());
                }
            }
        }
        int64_t mo = map0[id];
        for (int c : x.children)
            for (int32_t b : Bs[c]) {   // a child couples only to its ancestors' positions
                SIE_CHECK(b >= p0, SIE_EINVAL, "sparse LU: child boundary outside its parent's front");
                cmap[mo++] = loc(b);
            }
    });

    const auto t1 = std::chrono::steady_clock::now();
    // device layout of the factors (what the level-by-level solve reads)
    auto up = [](auto &d, const auto &v, auto zero) {
        if (v.empty()) d.upload(&zero, 1);
        else d.upload(v);
    };
    f = SparseLU();
    f.n = n;
    f.nsn = nn;
    f.max_sn = 0;
    for (int32_t x : sn_n) f.max_sn = std::max(f.max_sn, (int)x);
    f.nnz_factor = (int64_t)lcol.size() + (int64_t)ucol.size();
    f.est_flops = flops;
    int H = 0;
    for (const Node &x : nodes) H = std::max(H, x.height + 1);
    std::vector<std::vector<int>> by_level(H);
    for (int i = 0; i < nn; ++i) by_level[nodes[i].height].push_back(i);
    std::vector<int32_t> lev_sn;
    f.lev_ptr.assign(1, 0);
    for (int l = 0; l < H; ++l) {
        for (int id : by_level[l])
            if (nodes[id].n > 0) lev_sn.push_back(id);
        f.lev_ptr.push_back((int)lev_sn.size());
    }
    up(f.lev_sn, lev_sn, int32_t(0));
    up(f.sn_p0, sn_p0, int32_t(0));
    up(f.sn_n, sn_n, int32_t(0));
    up(f.inv_off, inv_off, int64_t(0));
    up(f.lrow_ptr, lcnt, int64_t(0));
    up(f.urow_ptr, ucnt, int64_t(0));
    up(f.lcol, lcol, int32_t(0));
    up(f.ucol, ucol, int32_t(0));
    up(f.perm, nd.order, int32_t(0));
    up(f.iperm, iperm, int32_t(0));
    std::vector<int32_t> bsn, brow;
    f.blk_ptr.assign(1, 0);
    for (size_t l = 0; l + 1 < f.lev_ptr.size(); ++l) {
        for (int q = f.lev_ptr[l]; q < f.lev_ptr[l + 1]; ++q) {
            const int32_t sn = lev_sn[q];
            for (int r = 0; r < sn_n[sn]; r += kLURowsPerBlock) {
                bsn.push_back(sn);
                brow.push_back(r);
            }
        }
        f.blk_ptr.push_back((int)bsn.size());
    }
    up(f.blk_sn, bsn, int32_t(0));
    up(f.blk_row0, brow, int32_t(0));
    const auto t2 = std::chrono::steady_clock::now();
    int bad = 0;
    const bool on_host = max_mm <= (int64_t)kLUHostFront * kLUHostFront;
    if (on_host) {
        // small fronts only: numeric factorisation on the host, the
        // supernodes of a level in parallel, update matrices per supernode
        std::vector<c128> lval(std::max<size_t>(lcol.size(), 1)), uval(std::max<size_t>(ucol.size(), 1));
        std::vector<c128> linv((size_t)std::max<int64_t>(inv_total, 1)), uinv((size_t)std::max<int64_t>(inv_total, 1));
        std::vector<std::vector<c128>> upd(nn);
        auto front = [&](int id) {
            const Node &x = nodes[id];
            const int fn = x.n, nb = (int)Bs[id].size(), m = fn + nb;
            if (m == 0) return;
            std::vector<c128> F((size_t)m * m);
            for (int64_t e = asm0[id]; e < asm0[id + 1]; ++e) F[(size_t)arow[e] * m + acol[e]] = val[asrc[e]];
            int64_t mo = map0[id];
            for (int c : x.children) {
                const int bc = (int)Bs[c].size();
                const int32_t *mp = cmap.data() + mo;
                for (int a = 0; a < bc; ++a)
                    for (int b = 0; b < bc; ++b) F[(size_t)mp[a] * m + mp[b]] += upd[c][(size_t)a * bc + b];
                mo += bc;
                std::vector<c128>().swap(upd[c]);
            }
            if (fn > 0) {
                eliminate_host(F.data(), m, fn, linv.data() + inv_off[id], uinv.data() + inv_off[id]);
                const int64_t *lo = loff.data() + loff0[id];
                for (int a = 0; a < nb; ++a)
                    for (int k = 0; k < fn; ++k) lval[lo[a] + k] = F[(size_t)(fn + a) * m + k];
                for (int k = 0; k < fn; ++k)
                    for (int b = 0; b < nb; ++b) uval[ucnt[x.p0 + k] + b] = F[(size_t)k * m + fn + b];
            }
            upd[id].resize((size_t)nb * nb);
            for (int a = 0; a < nb; ++a)
                for (int b = 0; b < nb; ++b) upd[id][(size_t)a * nb + b] = F[(size_t)(fn + a) * m + fn + b];
        };
        for (int l = 0; l < H; ++l) {
            const std::vector<int> &lv = by_level[l];
            parallel_for((int64_t)lv.size(), nthr, [&](int64_t i, int) { front(lv[i]); });
        }
        f.lval.upload(lval);
        f.uval.upload(uval);
        f.linv.upload(linv);
        f.uinv.upload(uinv);
    } else {
        // numeric factorisation on the device, front by front in postorder
        // on one stream (one front buffer reused; update matrices on the
        // stack)
        f.lval.alloc(std::max<size_t>(lcol.size(), 1));
        f.uval.alloc(std::max<size_t>(ucol.size(), 1));
        f.linv.alloc((size_t)std::max<int64_t>(inv_total, 1));
        f.uinv.alloc((size_t)std::max<int64_t>(inv_total, 1));
        PoolSyncedFree synced;   // the blocks below are freed after the stream is drained
        DBuf<c128> dval, dF, dstack;
        DBuf<int32_t> darow, dacol, dasrc, dmap;
        DBuf<int64_t> dloff;
        DBuf<int> dbad;
        try {
            dval.upload(val, st);
            up(darow, arow, int32_t(0));
            up(dacol, acol, int32_t(0));
            up(dasrc, asrc, int32_t(0));
            up(dmap, cmap, int32_t(0));
            up(dloff, loff, int64_t(0));
            dbad.upload(std::vector<int>(1, 0), st);
            dF.alloc((size_t)max_mm);
            dstack.alloc((size_t)peak);
            for (int id = 0; id < nn; ++id) {
                const Node &x = nodes[id];
                const int nb = (int)Bs[id].size(), m = x.n + nb;
                if (m == 0) continue;
                FrontStep fs;
                fs.F = dF.p;
                fs.m = m;
                fs.n = x.n;
                fs.arow = darow.p + asm0[id];
                fs.acol = dacol.p + asm0[id];
                fs.asrc = dasrc.p + asm0[id];
                fs.nasm = asm0[id + 1] - asm0[id];
                fs.val = dval.p;
                int64_t mo = map0[id];
                for (int c : x.children) {
                    const int bc = (int)Bs[c].size();
                    if (bc == 0) continue;
                    fs.child_upd.push_back(dstack.p + upd_off[c]);
                    fs.child_nb.push_back(bc);
                    fs.child_map.push_back(dmap.p + mo);
                    mo += bc;
                }
                fs.linv = f.linv.p + inv_off[id];
                fs.uinv = f.uinv.p + inv_off[id];
                fs.lval = f.lval.p;
                fs.loff = dloff.p + loff0[id];
                fs.uval = f.uval.p;
                fs.urow = f.urow_ptr.p + x.p0;
                fs.upd = nb > 0 ? dstack.p + upd_off[id] : nullptr;
                fs.bad = dbad.p;
                launch_front_step(fs, st);
            }
            SIE_HIP(hipMemcpyAsync(&bad, dbad.p, sizeof(int), hipMemcpyDeviceToHost, st));
            SIE_HIP(hipStreamSynchronize(st));
        } catch (...) {
            (void)hipStreamSynchronize(st);
            throw;
        }
    }
    SIE_CHECK(bad == 0, SIE_EINVAL, "sparse LU: zero pivot");
    const auto t3 = std::chrono::steady_clock::now();
    f.t_factor_s = std::chrono::duration<double>(t3 - t0).count();
    if (std::getenv("SIE_TRACE")) {
        auto ms = [](auto a, auto b) { return std::chrono::duration<double, std::milli>(b - a).count(); };
        std::fprintf(stderr,
                     "[setup]   sparse LU n=%lld: ordering + symbolic %.1f ms, layout upload %.1f ms, fronts %.1f ms "
                     "(%d fronts, largest %lld, %.3g Tflop, factors %.3g GB)\n",
                     (long long)n, ms(t0, t1), ms(t1, t2), ms(t2, t3), nn,
                     (long long)std::llround(std::sqrt((double)max_mm)), flops / 1e12, bytes / 1e9);
    }
}

void lu_solve(const SparseLU &f, int nrhs, c128 *x, hipStream_t st) {
    if (f.work.n < (size_t)nrhs * f.n) f.work.alloc((size_t)nrhs * f.n);
    const int H = (int)f.lev_ptr.size() - 1;
    for (int l = 0; l < H; ++l) launch_lu_level<double>(f, l, true, nrhs, x, st);
    for (int l = H - 1; l >= 0; --l) launch_lu_level<double>(f, l, false, nrhs, x, st);
}

void lu_solve(const SparseLU &f, int nrhs, c64 *x, hipStream_t st) {
    SIE_CHECK(f.lval32.n == f.lval.n && f.linv32.n == f.linv.n, SIE_ESTATE, "sparse LU: no FP32 factors");
    if (f.work32.n < (size_t)nrhs * f.n) f.work32.alloc((size_t)nrhs * f.n);
    const int H = (int)f.lev_ptr.size() - 1;
    for (int l = 0; l < H; ++l) launch_lu_level<float>(f, l, true, nrhs, x, st);
    for (int l = H - 1; l >= 0; --l) launch_lu_level<float>(f, l, false, nrhs, x, st);
}

}  // namespace sie
