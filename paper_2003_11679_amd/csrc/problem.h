// Problem state: mesh, grids, media (exterior and interiors), operators.
#pragma once
#include "common.h"
#include "kernels.h"
#include "sparse_lu.h"

#include <mutex>

struct sie_ctx {
    int device = 0;
    std::mutex mu;
    std::string err;   // message of the last failing call on this context
};
inline void ctx_set_error(sie_ctx *c, const std::string &m) {
    std::lock_guard<std::mutex> lk(c->mu);
    c->err = m;
}

namespace sie {

struct ObjIn {
    std::vector<double> xyz;
    std::vector<int32_t> tri;
    double eps_r = 1, mu_r = 1, sigma = 0;
};

struct GridReq {
    int n = 0;         // 0 = rule
    int R = 5;
    int share = -1;    // -1 default, 0 own grid, 1 share exterior grid
    double h = 0;      // > 0 with n > 0: explicit spacing
    double origin[3] = {0, 0, 0};
    bool has_origin = false;
};
// host_grid.cpp: grid rule of Sec. IV (eq. LboundsD2, Ddef)
double loss_ratio(int n, double theta0, double s);
void choose_grid(double freq, double eps_r, double mu_r, double sigma, double extent, double mean_edge,
                 int near_radius, int strict, sie_grid_params *out);

struct SolveState;     // solver.cpp

// HIP-event timers of the operator stages (enabled per problem).
// ST_SPMV64 counts the FP64 near-field products a second time (they are in
// ST_SPMV as well).
// ST_INT32 / ST_INT64 count the interior media's near-field products (the
// nested operator's, through the product groups) once more, per precision.
// ST_SKIP counts, instead of ST_SPMV64 / ST_INT32 / ST_INT64, the interior
// products that skip the rows of objects whose nested systems have
// converged (in ST_SPMV as well).
enum Stage {
    ST_PROJECT = 0, ST_FFT = 1, ST_INTERP = 2, ST_SPMV = 3, ST_PRODUCT = 4, ST_SPMV64 = 5, ST_INT32 = 6,
    ST_INT64 = 7, ST_SKIP = 8, NSTAGE = 9
};
struct StageTimer {
    int on = 0;   // 0 off, 1 every stage, 2 the near-field CSR product alone
    struct Rec { int stage, extra, extra2; hipEvent_t a, b; };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double total_ms[NSTAGE] = {};
    int64_t count[NSTAGE] = {};
    hipEvent_t get();
    void begin(int stage, hipStream_t st, hipEvent_t &a);
    void end(int stage, hipStream_t st, hipEvent_t a, int extra = -1, int extra2 = -1);
    void flush();
    void reset();
    ~StageTimer();
};

// Augmented EFIE of the exterior medium (Sec. III-E, eq. sys): unknowns
// [u (E); sigma = c0 rho (T, one pulse per triangle)], continuity rows
// weighted by A_t / k0, and the constraint preconditioner
// [j k0 diag(A0), -Dv^T diag(Gam); W Dv, j k0 W] applied through the exact
// Schur complement S = j k0 I + Dv diag(j k0 A0)^-1 Dv^T diag(Gam).
struct AugState {
    DBuf<c128> nA64;     // precorrected vector-potential near values (exterior CSR)
    DBuf<c128> gam64;    // precorrected pulse integrals per exterior near pair
    DBuf<c128> adiag;    // direct A0_nn
    DBuf<c128> gself;    // direct int_t int_t G0 of every triangle
    DBuf<c128> ad;       // j k0 A0_nn
    DBuf<c128> ks, alpha;   // [1]: the far part's scalar weight 2 j / k0 and the row factor j k0
    DBuf<double> sl;     // [T][3] +-l of each triangle edge's RWG function
    SparseLU lu;         // factors of S
    DBuf<c128> xnd, u, yu;   // workspaces: Schur right-hand sides, u and y_u of nb > 1 products
    double t_factor_s = 0.0;
};

}  // namespace sie

struct sie_problem {
    sie_ctx *ctx = nullptr;
    double freq = 0, w = 0, bg_eps_r = 1, bg_mu_r = 1;
    std::vector<sie::ObjIn> objs;
    sie::GridReq ext_req;
    std::vector<sie::GridReq> obj_req;
    sie_quad_params quad{0, 0, 0, 0, 0, 0};
    bool is_setup = false;
    double t_setup_s = 0;
    double cutoff_factor = 0;       // skin-depth cutoff in skin depths (0: off)
    int aug_mode = 0;               // augmented EFIE: 1 on, 0 off
    std::unique_ptr<sie::AugState> aug;   // set up when aug_mode is 1

    sie::Mesh mesh;
    std::vector<std::unique_ptr<sie::Grid>> grids;
    sie::Medium ext;
    std::vector<sie::Medium> ints;
    std::vector<std::unique_ptr<sie::Group>> groups;   // interior media batched by grid shape
    // device mesh arrays
    sie::DBuf<double> d_xyz, d_centroid;
    sie::DBuf<int32_t> d_tri, d_tri_rwg, d_tpm, d_epm;
    sie::DBuf<double> d_len, d_area, d_tri_sign;
    sie::DBuf<double> d_rho;           // [nt] largest vertex distance from the centroid
    std::vector<double> rho;
    // X operator (CSR, real)
    sie::DBuf<int32_t> d_xptr, d_xcol;
    sie::DBuf<double> d_xval64;
    sie::DBuf<float> d_xval32;
    // plane waves
    std::vector<double> khat;          // [nrhs][3]
    std::vector<sie::c128> e0;         // [nrhs][3]
    sie::SolveState *solve = nullptr;   // owned; freed by solver_destroy
    sie::StageTimer timer;

    sie::Medium &medium(int id);
    const sie::Medium &medium(int id) const;
};

namespace sie {

void problem_setup(sie_problem *p);
// Augmented exterior product (eq. sys without the GIBC term), x and y
// [nb][E + T]: y_u = j k0 A0 u - Dv^T Gam0 sigma, y_s = W (Dv u + j k0 sigma).
void aug_product(sie_problem *p, int nb, const c128 *x, c128 *y, hipStream_t st);
// Constraint preconditioner y = P^-1 x, x and y [nb][E + T], not aliased.
void cp_apply(sie_problem *p, int nb, const c128 *x, c128 *y, hipStream_t st);
template <typename T>
void matvec(sie_problem *p, Medium &md, sie_op op, int nrhs, const cx<T> *x, cx<T> *y, hipStream_t st);
// The product of every medium of a group on the group's rows (others not
// written), times -j w eps~_i per medium when `scaled` (the nested
// operator of eq. nest2).  active (optional, one right-hand side, indexed
// by object): the near-field product writes zero rows for the objects with
// active[object] == 0, whose rows of x must be zero (their grid stages
// still run, on zero sources).
template <typename T>
void group_product(sie_problem *p, Group &gr, sie_op op, bool scaled, int nrhs, const cx<T> *x, cx<T> *y,
                   hipStream_t st, const uint8_t *active = nullptr);
// Stage intermediates of one single-right-hand-side product: grid sources
// and potentials [F][nlive], the FFT pass buffers, per-triangle projection
// coefficients [ntg][4] and interpolation partials [ntg][5].
template <typename T>
struct ProductBufs {
    cx<T> *grid, *bufA, *bufB, *trisrc, *tripot;
};
struct ProductSizes {
    int64_t grid, bufA, bufB, trisrc, tripot;   // elements
};
ProductSizes product_sizes(const Grid &g);
// One AIM product y = Op_medium x (one right-hand side) in the given
// buffers; tm (nullable) records stage timings.  Allocates nothing.
template <typename T>
void product_one(sie_problem *p, Medium &md, sie_op op, const cx<T> *x, cx<T> *y, const ProductBufs<T> &b,
                 StageTimer *tm, hipStream_t st);
template <typename T>
void stage_project(sie_problem *p, Medium &md, const cx<T> *x, cx<T> *grid, hipStream_t st);
template <typename T>
void stage_convolve(sie_problem *p, Medium &md, sie_op op, int nf, const cx<T> *in, cx<T> *out, hipStream_t st);
template <typename T>
void stage_interpolate(sie_problem *p, Medium &md, const cx<T> *grid, cx<T> *y, hipStream_t st);
void solver_destroy(SolveState *s);
// abi.cpp: the calling thread is a server worker (no caller work to wait for)
void mark_worker_thread();
// server.cpp: device bytes of a problem, estimated from its description
size_t estimate_footprint(const sie_problem *p, int restart, int inner_max_iter);
// noalloc.hip: device address of the allocation-free product's scratch on
// `device` (current), looked up once; the product itself.
void noalloc_init(int device);
void matvec_noalloc(sie_problem *p, Medium &md, sie_op op, sie_precision prec, const void *x, void *y,
                    hipStream_t st);
void planewaves_entry(sie_problem *p, int32_t nrhs, const double *khat, const sie_c128 *e0);
void solve_entry(sie_problem *p, sie_precision prec, const sie_solver_opts *opts, sie_report *rep);
void nested_precond_entry(sie_problem *p, int precond, sie_precision prec, int nrhs, const void *x, void *y,
                          hipStream_t st);
int nested_precond_clusters(const sie_problem *p, int64_t *owned);
int nested_precond_factored(const sie_problem *p, int64_t *factor_nnz, double *t_factor_s);
void currents_entry(const sie_problem *p, int32_t rhs, sie_c128 *u, sie_c128 *v);
void charges_entry(const sie_problem *p, int32_t rhs, sie_c128 *sg);
// Message returned by sie_last_error() on this thread.
void set_last_error(const std::string &m);
void farfield_entry(const sie_problem *p, int32_t rhs, int64_t ndir, const double *rhat, sie_c128 *F);

// ---- k_blas.hip
template <typename T> void launch_zero(int64_t n, cx<T> *y, hipStream_t st);
template <typename Ti, typename To> void launch_convert(const cx<Ti> *in, cx<To> *out, int64_t n, hipStream_t st);
template <typename T> void launch_axpby(int64_t n, c128 a, const cx<T> *x, c128 b, cx<T> *y, hipStream_t st);
template <typename T> void launch_scale_into(int64_t n, c128 a, const cx<T> *x, cx<T> *y, hipStream_t st);
// h[j] = sum_i conj(V[j][i]) w[i], j < J (FP64 accumulation); part: scratch [J][nb]
template <typename T> void launch_dots(int64_t n, int J, const cx<T> *V, int64_t ldv, const cx<T> *w, c128 *part,
                                       int nb, c128 *h, hipStream_t st);
// w -= sum_j V[j] h[j]
template <typename T> void launch_gemv_sub(int64_t n, int J, const cx<T> *V, int64_t ldv, const c128 *h, cx<T> *w,
                                           hipStream_t st);
// w += sum_j V[j] h[j]
template <typename T> void launch_gemv_add(int64_t n, int J, const cx<T> *V, int64_t ldv, const c128 *h, cx<T> *w,
                                           hipStream_t st);
// Batched forms for ns systems stored [ns][n] inside every vector (Krylov
// vector j at V + j * ldv): dots into h[s * hstride + j] (and, when hmirror
// is not null, the same entries of hmirror, e.g. mapped host memory),
// w[s] -+= V[s] h[s], y[s] = c[s] x[s].
template <typename T> void launch_dots_sys(int64_t n, int J, const cx<T> *V, int64_t ldv, int ns, const cx<T> *w,
                                           c128 *part, int nb, c128 *h, int hstride, hipStream_t st,
                                           c128 *hmirror = nullptr);
template <typename T> void launch_gemv_sys(int64_t n, int J, const cx<T> *V, int64_t ldv, int ns, const c128 *h,
                                           int hstride, cx<T> *w, bool add, hipStream_t st);
template <typename T> void launch_scale_sys(int64_t n, int ns, const c128 *c, const cx<T> *x, cx<T> *y,
                                            hipStream_t st);
// y[s] = c.v[s] x[s], coefficients passed by value (ns <= kScaleArg)
constexpr int kScaleArg = 64;
struct ScaleArg { c128 v[kScaleArg]; };
template <typename T> void launch_scale_val(int64_t n, int ns, const ScaleArg &c, const cx<T> *x, cx<T> *y,
                                            hipStream_t st);
// y[s] = x[s] / sqrt(Re d[s * dstride]) (zero where that is zero): scaling
// by a squared norm that stays on the device
template <typename T> void launch_scale_rnorm(int64_t n, int ns, const c128 *d, int dstride, const cx<T> *x,
                                              cx<T> *y, hipStream_t st);
// y[i] = d[i] * x[i] with per-element complex d (range [i0, i1), zero elsewhere if zero_out)
template <typename T> void launch_diag_mul(int64_t n, const c128 *d, const cx<T> *x, cx<T> *y, hipStream_t st);
constexpr int DOT_BLOCKS = 256;

}  // namespace sie
