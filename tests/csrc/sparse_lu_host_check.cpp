// Host-logic check of the sparse LU (csrc/sparse_lu.cpp) without a device:
// the device entry points it calls are replaced by host code that performs
// the same operations on host memory and checks every access against the
// allocation it falls in.  The ordering, the symbolic factorisation (front
// boundaries, where each result goes, the update-matrix stack) and both
// numeric paths (host fronts, and the per-front steps the device would run)
// are exercised; the factors then solve the system with the level-by-level
// algorithm of the device solve, and the residual is printed.
//
// Usage: sparse_lu_host_check n radius seed
//   n points on the unit sphere, coupled when closer than radius, give a
//   structurally symmetric, diagonally dominant complex matrix.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>

#include "../../paper_2003_11679_amd/csrc/sparse_lu.h"

using namespace sie;

static std::map<const char *, size_t> g_alloc;
static int g_device_fronts = 0;

static void check(const void *base, int64_t idx, size_t elt) {
    const char *p = (const char *)base + idx * (int64_t)elt;
    auto it = g_alloc.upper_bound(p);
    if (it == g_alloc.begin()) {
        std::fprintf(stderr, "access outside every allocation\n");
        std::exit(3);
    }
    --it;
    if (!(p >= it->first && p + elt <= it->first + it->second)) {
        std::fprintf(stderr, "access beyond its allocation (index %lld)\n", (long long)idx);
        std::exit(3);
    }
}

namespace sie {
void *pool_alloc(size_t bytes) {
    void *p = std::malloc(bytes);
    std::memset(p, 0xcd, bytes);   // no block starts out zero
    g_alloc[(const char *)p] = bytes;
    return p;
}
void pool_free(void *p) {
    g_alloc.erase((const char *)p);
    std::free(p);
}
PoolSyncedFree::PoolSyncedFree() {}
PoolSyncedFree::~PoolSyncedFree() {}
template <typename T> void launch_lu_level(const SparseLU &, int, bool, int, cx<T> *, hipStream_t) { std::abort(); }
template void launch_lu_level<double>(const SparseLU &, int, bool, int, c128 *, hipStream_t);
template void launch_lu_level<float>(const SparseLU &, int, bool, int, c64 *, hipStream_t);

// One front, as the device kernels compute it (unblocked here).
void launch_front_step(const FrontStep &s, hipStream_t) {
    ++g_device_fronts;
    const int m = s.m, n = s.n, nb = m - n;
    auto F = [&](int64_t i, int64_t j) -> c128 & {
        check(s.F, i * m + j, sizeof(c128));
        return s.F[i * m + j];
    };
    for (int64_t e = 0; e < (int64_t)m * m; ++e) F(e / m, e % m) = c128();
    for (int64_t e = 0; e < s.nasm; ++e) {
        check(s.arow, e, 4);
        check(s.acol, e, 4);
        check(s.asrc, e, 4);
        check(s.val, s.asrc[e], sizeof(c128));
        if (s.arow[e] < 0 || s.arow[e] >= m || s.acol[e] < 0 || s.acol[e] >= m) std::exit(4);
        c128 &d = F(s.arow[e], s.acol[e]);
        if (d.re != 0.0 || d.im != 0.0) std::exit(5);   // two original entries in one position
        d = s.val[s.asrc[e]];
    }
    for (size_t c = 0; c < s.child_nb.size(); ++c) {
        const int bc = s.child_nb[c];
        for (int a = 0; a < bc; ++a) {
            check(s.child_map[c], a, 4);
            if (s.child_map[c][a] < 0 || s.child_map[c][a] >= m) std::exit(4);
        }
        for (int a = 0; a < bc; ++a)
            for (int b = 0; b < bc; ++b) {
                check(s.child_upd[c], (int64_t)a * bc + b, sizeof(c128));
                F(s.child_map[c][a], s.child_map[c][b]) += s.child_upd[c][(int64_t)a * bc + b];
            }
    }
    if (n > 0) {
        for (int k = 0; k < n; ++k) {
            const c128 ip = cdiv(c128(1.0), F(k, k));
            for (int i = k + 1; i < m; ++i) F(i, k) = F(i, k) * ip;
            for (int i = k + 1; i < m; ++i)
                for (int j = k + 1; j < m; ++j) F(i, j) -= F(i, k) * F(k, j);
        }
        auto L = [&](int64_t i, int64_t j) -> c128 & {
            check(s.linv, i * n + j, sizeof(c128));
            return s.linv[i * n + j];
        };
        auto U = [&](int64_t i, int64_t j) -> c128 & {
            check(s.uinv, i * n + j, sizeof(c128));
            return s.uinv[i * n + j];
        };
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) L(i, j) = U(i, j) = c128();
        for (int c = 0; c < n; ++c) {
            L(c, c) = c128(1.0);
            for (int i = c + 1; i < n; ++i) {
                c128 acc;
                for (int k = c; k < i; ++k) acc += F(i, k) * L(k, c);
                L(i, c) = -acc;
            }
            U(c, c) = cdiv(c128(1.0), F(c, c));
            for (int i = c - 1; i >= 0; --i) {
                c128 acc;
                for (int k = i + 1; k <= c; ++k) acc += F(i, k) * U(k, c);
                U(i, c) = cdiv(-acc, F(i, i));
            }
        }
        for (int a = 0; a < nb; ++a)
            for (int k = 0; k < n; ++k) {
                check(s.loff, a, 8);
                check(s.lval, s.loff[a] + k, sizeof(c128));
                s.lval[s.loff[a] + k] = F(n + a, k);
            }
        for (int k = 0; k < n; ++k)
            for (int b = 0; b < nb; ++b) {
                check(s.urow, k, 8);
                check(s.uval, s.urow[k] + b, sizeof(c128));
                s.uval[s.urow[k] + b] = F(k, n + b);
            }
    }
    for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) {
            check(s.upd, (int64_t)a * nb + b, sizeof(c128));
            s.upd[(int64_t)a * nb + b] = F(n + a, n + b);
        }
}
}  // namespace sie

extern "C" {
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
    std::memcpy(d, s, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) {
    std::memcpy(d, s, n);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
}

int main(int argc, char **argv) {
    if (argc < 4) return 2;
    const int n = std::atoi(argv[1]);
    const double r = std::atof(argv[2]);
    std::mt19937_64 gen((uint64_t)std::atoll(argv[3]));
    std::normal_distribution<double> gauss;
    std::uniform_real_distribution<double> uni(-1.0, 1.0);
    std::vector<double> xyz(3 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        double v[3] = {gauss(gen), gauss(gen), gauss(gen)};
        const double l = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        for (int d = 0; d < 3; ++d) xyz[3 * i + d] = v[d] / l;
    }
    // pattern: pairs closer than r (symmetric); values: random off-diagonal,
    // a diagonal above the row's absolute sum
    std::vector<std::vector<std::pair<int, c128>>> rows(n);
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double d2 = 0.0;
            for (int c = 0; c < 3; ++c) d2 += (xyz[3 * i + c] - xyz[3 * j + c]) * (xyz[3 * i + c] - xyz[3 * j + c]);
            if (d2 < r * r) {
                rows[i].push_back({j, c128(uni(gen), uni(gen))});
                rows[j].push_back({i, c128(uni(gen), uni(gen))});
            }
        }
    std::vector<int64_t> rp(n + 1, 0);
    std::vector<int32_t> ci;
    std::vector<c128> val;
    for (int i = 0; i < n; ++i) {
        double sum = 0.0;
        for (auto &kv : rows[i]) sum += std::hypot(kv.second.re, kv.second.im);
        rows[i].push_back({i, c128(sum + 1.0, 0.5)});
        std::sort(rows[i].begin(), rows[i].end(), [](const auto &a, const auto &b) { return a.first < b.first; });
        for (auto &kv : rows[i]) {
            ci.push_back(kv.first);
            val.push_back(kv.second);
        }
        rp[i + 1] = (int64_t)ci.size();
    }
    SparseLU f;
    lu_factor(f, n, rp, ci, val, xyz, nullptr);
    // the device solve's two sweeps, level by level, on the stored layout
    std::vector<c128> b(n), y(n), x(n);
    for (int i = 0; i < n; ++i) b[i] = c128(uni(gen), uni(gen));
    for (int p = 0; p < n; ++p) y[p] = b[f.perm.p[p]];
    const int H = (int)f.lev_ptr.size() - 1;
    auto level = [&](int l, bool fwd) {
        const int64_t *rpp = fwd ? f.lrow_ptr.p : f.urow_ptr.p;
        const int32_t *cc = fwd ? f.lcol.p : f.ucol.p;
        const c128 *vv = fwd ? f.lval.p : f.uval.p, *inv = fwd ? f.linv.p : f.uinv.p;
        for (int q = f.lev_ptr[l]; q < f.lev_ptr[l + 1]; ++q) {
            const int sn = f.lev_sn.p[q], p0 = f.sn_p0.p[sn], nn = f.sn_n.p[sn];
            std::vector<c128> t(nn);
            for (int i = 0; i < nn; ++i) {
                c128 acc = y[p0 + i];
                for (int64_t j = rpp[p0 + i]; j < rpp[p0 + i + 1]; ++j) acc -= vv[j] * y[cc[j]];
                t[i] = acc;
            }
            const c128 *M = inv + f.inv_off.p[sn];
            for (int i = 0; i < nn; ++i) {
                c128 acc;
                for (int k = fwd ? 0 : i; k < (fwd ? i + 1 : nn); ++k) acc += M[(int64_t)i * nn + k] * t[k];
                y[p0 + i] = acc;
            }
        }
    };
    for (int l = 0; l < H; ++l) level(l, true);
    for (int l = H - 1; l >= 0; --l) level(l, false);
    for (int p = 0; p < n; ++p) x[f.perm.p[p]] = y[p];
    double rn = 0.0, bn = 0.0;
    for (int i = 0; i < n; ++i) {
        c128 acc;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) acc += val[k] * x[ci[k]];
        acc -= b[i];
        rn += norm2(acc);
        bn += norm2(b[i]);
    }
    std::printf("n %d nnz %zu supernodes %d largest %d device_fronts %d residual %.3e\n", n, ci.size(), f.nsn,
                f.max_sn, g_device_fronts, std::sqrt(rn / bn));
    return 0;
}
