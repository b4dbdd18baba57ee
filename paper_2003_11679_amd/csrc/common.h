// Internal declarations of the SIE library (host C++ and HIP kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/sie.h"

namespace sie {

// ---------------------------------------------------------------- complex
template <typename T>
struct cx {
    T re, im;
    __host__ __device__ cx() : re(0), im(0) {}
    __host__ __device__ cx(T r, T i = 0) : re(r), im(i) {}
    template <typename U>
    __host__ __device__ explicit cx(const cx<U> &o) : re(T(o.re)), im(T(o.im)) {}
};
template <typename T> __host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __host__ __device__ inline cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <typename T> __host__ __device__ inline cx<T> operator*(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __host__ __device__ inline cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __host__ __device__ inline cx<T> operator*(cx<T> a, T s) { return {s * a.re, s * a.im}; }
template <typename T> __host__ __device__ inline cx<T> &operator+=(cx<T> &a, cx<T> b) { a.re += b.re; a.im += b.im; return a; }
template <typename T> __host__ __device__ inline cx<T> &operator-=(cx<T> &a, cx<T> b) { a.re -= b.re; a.im -= b.im; return a; }
template <typename T> __host__ __device__ inline cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
template <typename T> __host__ __device__ inline T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename T> __host__ __device__ inline cx<T> cdiv(cx<T> a, cx<T> b) {
    T d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
using c64 = cx<float>;
using c128 = cx<double>;

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
    sie_status code;
    Error(sie_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define SIE_HIP(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            throw ::sie::Error(SIE_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define SIE_CHECK(cond, code, msg)                                            \
    do {                                                                      \
        if (!(cond)) throw ::sie::Error(code, msg);                           \
    } while (0)

// ---------------------------------------------------------------- device memory
// Pool of device blocks (pool.cpp): pool_alloc throws SIE_ENOMEM; pool_free
// synchronises the device and keeps the block for reuse.
void *pool_alloc(size_t bytes);
void pool_free(void *p);
size_t pool_cached_bytes(int device);
void pool_trim(int device);
// While one is alive, pool_free on this host thread skips its device-wide
// synchronisation: the caller has completed every piece of work that used
// the blocks it frees.
struct PoolSyncedFree {
    PoolSyncedFree();
    ~PoolSyncedFree();
    PoolSyncedFree(const PoolSyncedFree &) = delete;
    PoolSyncedFree &operator=(const PoolSyncedFree &) = delete;
};

// ---------------------------------------------------------------- device buffer
// Owns its device memory, or (view) refers to a slice of another DBuf's.
template <typename T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    bool own = true;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n), own(o.own) { o.p = nullptr; o.n = 0; o.own = true; }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; own = o.own; o.p = nullptr; o.n = 0; o.own = true; }
        return *this;
    }
    ~DBuf() { release(); }
    // Refer to count elements at q (owned elsewhere; never freed here).
    void view(T *q, size_t count) {
        release();
        p = q; n = count; own = false;
    }
    void alloc(size_t count) {
        release();
        n = count;
        if (count) {
            try {
                p = static_cast<T *>(pool_alloc(count * sizeof(T)));
            } catch (...) {
                p = nullptr; n = 0;
                throw;
            }
        }
    }
    void release() {
        if (p && own) pool_free(p);
        p = nullptr; n = 0; own = true;
    }
    void upload(const T *h, size_t count) {
        if (count > n) alloc(count);
        if (count) SIE_HIP(hipMemcpy(p, h, count * sizeof(T), hipMemcpyHostToDevice));
    }
    void upload(const std::vector<T> &v) { upload(v.data(), v.size()); }
    // Ordered on stream st; returns once the copy is complete.
    void upload(const std::vector<T> &v, hipStream_t st) {
        if (v.size() > n) alloc(v.size());
        if (v.empty()) return;
        SIE_HIP(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
        SIE_HIP(hipStreamSynchronize(st));
    }
    std::vector<T> download(size_t count) const {
        std::vector<T> h(count);
        if (count) SIE_HIP(hipMemcpy(h.data(), p, count * sizeof(T), hipMemcpyDeviceToHost));
        return h;
    }
    std::vector<T> download() const { return download(n); }
    size_t bytes() const { return n * sizeof(T); }
};

// ---------------------------------------------------------------- mesh (host)
struct Mesh {
    // concatenated objects
    std::vector<double> xyz;        // [nv][3]
    std::vector<int32_t> tri;       // [nt][3]
    std::vector<int32_t> tri_obj;   // [nt]
    int nobj = 0;
    // geometry
    std::vector<double> area;       // [nt]
    std::vector<double> normal;     // [nt][3]
    std::vector<double> centroid;   // [nt][3], ((v0 + v1) + v2) / 3
    // RWG topology
    int64_t nrwg = 0;
    std::vector<int32_t> edge_v;    // [E][2] a < b
    std::vector<int32_t> tpm;       // [E][2] T+, T-
    std::vector<int32_t> epm;       // [E][2] local edge index in T+, T-
    std::vector<double> len;        // [E]
    std::vector<int32_t> tri_rwg;   // [nt][3]
    std::vector<double> tri_sign;   // [nt][3]
    std::vector<int64_t> obj_rwg0;  // [nobj + 1] first RWG of each object
    int64_t nt() const { return (int64_t)tri.size() / 3; }
    int64_t nv() const { return (int64_t)xyz.size() / 3; }
};
void build_topology(Mesh &m);   // throws Error(SIE_EMESH)

// ---------------------------------------------------------------- quadrature (host)
struct Rule {
    std::vector<double> bary;   // [q][3]
    std::vector<double> w;      // [q], sum = 1
    int size() const { return (int)w.size(); }
};
void gauss_legendre01(int n, std::vector<double> &x, std::vector<double> &w);
Rule rule_collapsed(int n);
Rule rule_self(int n);
Rule rule_edge(int n, int opp);
Rule rule_vertex(int n, int vtx);

enum PairKind { KIND_SELF = 0, KIND_EDGE = 1, KIND_VERTEX = 2, KIND_CLOSE = 3, KIND_FAR = 4 };
constexpr double CLOSE_FACTOR = 2.5;

// ---------------------------------------------------------------- grid + operators
template <typename T>
struct Work {       // per-medium, per-precision scratch for matvecs
    DBuf<cx<T>> grid;     // [rhs][F][nl_z][nl_y][nl_x] sources then potentials
    DBuf<cx<T>> bufA;     // [rhs][F][nl_z][nl_y][m_x]
    DBuf<cx<T>> bufB;     // [rhs][F][nl_z][m_y][m_x]
    DBuf<cx<T>> trisrc;   // [rhs][ntg][4]  per-triangle projection coefficients
    DBuf<cx<T>> tripot;   // [ntg][5]  per-triangle interpolation partials
    DBuf<cx<T>> xt;       // [E][nrhs] right-hand sides of a batched product
    int cap_rhs = 0;      // right-hand sides the buffers above hold
};

struct Grid {
    double origin[3] = {0, 0, 0};
    double h = 0;
    int n[3] = {0, 0, 0};      // full grid
    int lo[3] = {0, 0, 0};     // live box origin (node index)
    int nl[3] = {0, 0, 0};     // live box extent
    int m[3] = {0, 0, 0};      // FFT lengths (powers of two >= 2 nl - 1)
    int near_radius = 5;
    double cutoff = 0;         // skin-depth cutoff of the near list (0: none)
    bool all_near = false;     // every pair of the grid's triangles is near
    std::vector<int32_t> tris; // triangles (global ids) on this grid, ascending
    std::vector<int32_t> objs; // objects covered
    std::vector<int32_t> centre;  // [ntg][3] stencil centres (host copy)
    // device data
    DBuf<int32_t> d_tris;      // [ntg] global triangle id
    DBuf<int32_t> d_centre;    // [ntg][3]
    DBuf<double> d_mom64;      // [ntg][27][4] (M0, M1x, M1y, M1z)
    DBuf<float> d_mom32;
    DBuf<double> d_tri64;      // [ntg][3 edges][4]: coef c_e = s l/(2A), q_e (free vertex - centre)
    DBuf<float> d_tri32;
    // projection as a gather: node -> list of (local triangle, stencil slot)
    DBuf<int32_t> d_node_ptr;  // [nlive + 1]
    DBuf<int32_t> d_node_ent;  // [27 ntg]  (tl << 5) | slot
    // near triangle pairs (local indices), CSR over row triangle
    DBuf<int64_t> d_pair_ptr;  // [ntg + 1]
    DBuf<int32_t> d_pair_s;    // [npairs]
    int64_t npairs = 0;
    // kind | loc << 4 of every near pair (geometry only: built once, with
    // the first medium, and shared by the others)
    DBuf<uint8_t> d_pair_kind; // [npairs]
    // RWG near pattern (global RWG rows of the grid's objects)
    int64_t rwg0 = 0, rwg1 = 0; // RWG range [rwg0, rwg1)
    DBuf<int64_t> d_row_ptr;   // [nrow + 1] (row r = RWG rwg0 + r)
    DBuf<int32_t> d_cols;      // [nnz] global RWG column
    // the same columns as 16-bit offsets from the row's first column, when
    // every row spans fewer than 65536 columns (the products then stream
    // 2 bytes per index instead of 4)
    bool cols16 = false;
    DBuf<uint16_t> d_cols16;   // [nnz]
    DBuf<int32_t> d_row_base;  // [nrow]
    int64_t nnz = 0;
    int64_t max_row = 0;
    DBuf<int32_t> d_trirwg;    // [ntg][3] global RWG of each local triangle edge
    DBuf<int32_t> d_rwgloc;    // [nrow][2] (local triangle << 2) | local edge, for T+ and T-
    DBuf<int32_t> d_glob2loc;  // [nt] local index or -1
    std::vector<int32_t> glob2loc;
    std::vector<double> tri_coef;  // host copy of d_tri64
    Work<double> w64;
    Work<float> w32;
    int64_t nlive() const { return (int64_t)nl[0] * nl[1] * nl[2]; }
    int64_t mvol() const { return (int64_t)m[0] * m[1] * m[2]; }
    int64_t oct() const { return (int64_t)(m[0] / 2 + 1) * (m[1] / 2 + 1) * (m[2] / 2 + 1); }
};

struct Medium;
template <typename T> Work<T> &work_of(Grid &g);

// What one launch of the grid stages and the near-field product reads: one
// grid, or several grids of one live-box shape laid side by side ("slots",
// one object each).  Slot s owns live nodes [s nlive, (s + 1) nlive) of the
// node range, its triangles' centres are relative to its own live box, and
// grid fields are stored [rhs][slot][F][nl_z][nl_y][nl_x].  The near-field
// product covers the RWG rows [rwg0, rwg1) (the slots' objects, contiguous).
struct GridView {
    int nslot = 1;
    int64_t ntg = 0;                 // triangles of all slots
    int64_t nlive = 0;               // live nodes of one slot
    int nl[3] = {0, 0, 0}, m[3] = {0, 0, 0}, lo[3] = {0, 0, 0};
    int64_t rwg0 = 0, rwg1 = 0;
    const int32_t *centre = nullptr;     // [ntg][3], minus lo = live-box index
    const int32_t *tri_slot = nullptr;   // [ntg] slot of each triangle (null: one slot)
    const int32_t *node_ptr = nullptr;   // [nslot nlive + 1]
    const int32_t *node_ent = nullptr;   // (triangle << 5) | stencil slot
    const int32_t *trirwg = nullptr;     // [ntg][3] global RWG of each triangle edge
    const int32_t *rwgloc = nullptr;     // [nrow][2] (triangle << 2) | local edge
    const double *mom64 = nullptr, *coef64 = nullptr;
    const float *mom32 = nullptr, *coef32 = nullptr;
    const int64_t *row_ptr = nullptr;    // [nrow + 1]
    const int32_t *cols = nullptr;
    const uint16_t *cols16 = nullptr;
    const int32_t *row_base = nullptr;
    bool c16 = false;
    // optional: the near-field product writes zero rows, without reading
    // their values, for the slots s with !active[obj0 + s] (slot s holds
    // object obj0 + s; one right-hand side)
    const uint8_t *active = nullptr;
    int obj0 = 0;
    int64_t nrow() const { return rwg1 - rwg0; }
    int64_t nnodes() const { return nlive * nslot; }
};
GridView view_of(const Grid &g);

// Medium-dependent arrays of one launch, per slot: spectra ([slot][4][oct]),
// near values (CSR of the view), -2 k^-2 of the scalar term of L, and an
// optional per-slot factor on the whole result.
template <typename T>
struct MediaView {
    bool far = true;                     // grid part present
    const cx<T> *spec = nullptr;
    int64_t spec_stride = 0;
    const cx<T> *nL = nullptr, *nK = nullptr;
    const cx<T> *kscal = nullptr;        // [nslot]
    const cx<T> *alpha = nullptr;        // [nslot] or null (factor 1)
};

struct Medium {
    int id = -1;               // -1 exterior, else object index
    Grid *grid = nullptr;
    c128 k;                    // wavenumber
    c128 eps, mu;              // complex permittivity, permeability (absolute)
    // spectra (octant-folded, 1/(mx my mz) folded in): G, dG/dx, dG/dy, dG/dz
    DBuf<c128> d_spec64;       // [4][oct]
    DBuf<c64> d_spec32;
    // precorrected near values (CSR of the grid pattern)
    DBuf<c128> d_nL64, d_nK64;
    DBuf<c64> d_nL32, d_nK32;
    DBuf<c128> d_nLd64;        // direct near-region L (no precorrection): preconditioner source
    DBuf<c128> d_ks64, d_alpha64;   // [1]: -2 k^-2 and -j w eps~ (nested operator factor)
    DBuf<c64> d_ks32, d_alpha32;
    int group = -1;            // interior media: the product group it belongs to
    // no grid part (Sec. III-D-2 items a and b): the skin-depth cutoff lies
    // within the near region, or every pair of the grid is near; the
    // operator is then the direct near-region one
    bool local = false;
};

// Interior media whose grids share one live-box shape, batched into one
// launch per stage (Sec. III-D-1: one grid per object; the objects'
// products are independent and run side by side).  A group of one medium
// refers to that medium's own grid arrays; a larger one owns merged copies,
// and its media's near values are views into the group's arrays.
struct Group {
    std::vector<int> media;    // object ids, consecutive
    GridView view;
    const Grid *grid0 = nullptr;   // the grid of a one-medium group
    int64_t nnz = 0;
    // merged arrays (several slots)
    DBuf<int32_t> d_centre, d_tri_slot, d_node_ptr, d_node_ent, d_trirwg, d_rwgloc, d_cols, d_row_base;
    DBuf<uint16_t> d_cols16;
    DBuf<int64_t> d_row_ptr;
    DBuf<double> d_mom64, d_coef64;
    DBuf<float> d_mom32, d_coef32;
    DBuf<c128> d_spec64, d_ks64, d_alpha64, d_nL64, d_nK64;
    DBuf<c64> d_spec32, d_ks32, d_alpha32, d_nL32, d_nK32;
    Work<double> w64;
    Work<float> w32;
};

}  // namespace sie
