// Launchers of the HIP kernels (definitions in k_*.hip).
#pragma once
#include "common.h"

namespace sie {

// ---- k_fft.hip
// nf fields [nf][nl_z][nl_y][nl_x] of the view's live-box shape.  The fields
// form runs of `fps` consecutive fields that share one spectrum; run j uses
// spec + ((j mod nspec) * spec_stride) (one spectrum for all: fps = nf,
// nspec = 1).  mode 0: each field times G; mode 1: triples (J_x, J_y, J_z) to
// grad G x J (fps and nf multiples of 3).
template <typename T>
void fft_convolve(const GridView &g, const cx<T> *spec, int64_t spec_stride, int fps, int nspec, int nf, int mode,
                  const cx<T> *in, cx<T> *out, cx<T> *bufA, cx<T> *bufB, hipStream_t st);
void fft3d_full_fwd(c128 *vol, c128 *tmp, int mx, int my, int mz, hipStream_t st);

// ---- k_grid.hip
void launch_stencil_assign(const double *centroids, const int32_t *tris, int64_t t0, int64_t ntg,
                           const double origin[3], double h, const int n[3], int32_t *centre_out, int32_t *raw_out,
                           hipStream_t st);
void launch_moments(const double *xyz, const int32_t *tri, const int32_t *tris, const int32_t *centre,
                    int64_t ntg, const double origin[3], double h, const double *rule, int nq,
                    double *mom64, float *mom32, hipStream_t st);
template <typename T>
void launch_tri_sources(const GridView &g, const T *tri_coef, const cx<T> *x, int64_t ldx, int nrhs,
                        cx<T> *trisrc, hipStream_t st);
template <typename T>
void launch_project(const GridView &g, const T *mom, const cx<T> *trisrc, cx<T> *grid, int nfields, int nrhs,
                    hipStream_t st, const cx<T> *rho = nullptr, int64_t ldr = 0, const int32_t *rho_tris = nullptr);
template <typename T>
void launch_interp(const GridView &g, const T *mom, const cx<T> *pot, int nfields, int nrhs, cx<T> *tripot,
                   hipStream_t st);
// y[r] = sum_j N[r,j] x[j] + sum over the row's triangles of the far part,
// times alpha[slot] (alpha null: 1), for the view's rows r in [rwg0, rwg1);
// other rows are not written.  kscal[slot] = -2 k^-2 (scalar part weight;
// null for K-type).  N may be null (far part only).
template <typename T>
void launch_spmv_far(const GridView &g, const T *tri_coef, const cx<T> *tripot, const cx<T> *kscal,
                     const cx<T> *alpha, const cx<T> *vals, const cx<T> *x, cx<T> *y, bool use_far, hipStream_t st);
template <typename T>
void launch_spmm_far(const GridView &g, int64_t E, int nrhs, const T *tri_coef, const cx<T> *tripot,
                     const cx<T> *kscal, const cx<T> *alpha, const cx<T> *vals, const cx<T> *x, cx<T> *xt, cx<T> *y,
                     hipStream_t st);
template <typename T>
void launch_x_apply(int64_t E, const int32_t *xptr, const int32_t *xcol, const T *xval, const cx<T> *x,
                    cx<T> *y, hipStream_t st);

// ---- k_aug.hip (augmented EFIE, Sec. III-E; FP64)
// tripot[r][t][4] += sum over the near pairs (t, s) of gam[p] rho[r][tris[s]]
// (t, s the grid's triangles, tris their global numbers).
void launch_tri_near(int64_t ntg, const int64_t *pair_ptr, const int32_t *pair_s, const int32_t *tris,
                     const c128 *gam, const c128 *rho, int64_t ldr, int nrhs, c128 *tripot, hipStream_t st);
// y[r][t] = sum_e sl[t][e] u[r][n_e] / k0 + j A_t sigma[r][t] (weighted continuity rows).
void launch_continuity(int64_t nt, const int32_t *tri_rwg, const double *sl, const double *area, double k0,
                       const c128 *u, int64_t ldu, const c128 *sg, int64_t lds, c128 *y, int64_t ldy, int nrhs,
                       hipStream_t st);
// Constraint preconditioner around the Schur solve (xnd [nrhs][nt] in the
// solver's position order).
void launch_cp_pre(int64_t nt, const int32_t *tri_rwg, const double *sl, const double *area, double k0, const c128 *ad,
                   const int32_t *iperm, const c128 *r, int64_t ldr, int64_t E, c128 *xnd, int nrhs, hipStream_t st);
void launch_cp_post(int64_t E, int64_t nt, const int32_t *tpm, const int32_t *epm, const double *sl, const double *area,
                    const c128 *gself, const c128 *ad, const int32_t *iperm, const c128 *xnd, const c128 *r,
                    int64_t ldr, c128 *y, int64_t ldy, int nrhs, hipStream_t st);

// ---- k_near.hip
// Skin-depth cutoff of a near search: dc > 0 keeps the pairs whose centroids
// (global arrays, triangle tris[local]) are at most dc + rho_t + rho_s apart.
struct NearCut {
    double dc = 0.0;
    const double *centroid = nullptr;
    const double *rho = nullptr;
    const int32_t *tris = nullptr;
};
void launch_near_count(const int32_t *centre, int64_t ntg, const int32_t *cell_ptr, const NearCut &cut,
                       const int lo[3], const int nl[3], int R, int64_t *count, hipStream_t st);
void launch_near_emit(const int32_t *centre, int64_t ntg, const int32_t *cell_ptr, const NearCut &cut,
                      const int lo[3], const int nl[3], int R, const int64_t *pair_ptr, int32_t *pair_s,
                      hipStream_t st);
// 16-bit column offsets from each row's first column; *wide is set when a
// row spans 65536 columns or more (the offsets are then unusable).
void launch_cols16(int64_t nrow, const int64_t *row_ptr, const int32_t *cols, int32_t *row_base, uint16_t *cols16,
                   int *wide, hipStream_t st);
void launch_rwg_pattern(int64_t nrow, int64_t rwg0, int64_t nbits, const int32_t *rwg_loc, const int64_t *pair_ptr,
                        const int32_t *pair_s, const int32_t *tris, const int32_t *tri_rwg, int64_t *row_len,
                        const int64_t *row_ptr, int32_t *cols, int pass, hipStream_t st);

struct NearFillArgs {
    const double *xyz; const int32_t *tri; const int32_t *tris; const int32_t *centre;
    const double *centroid; const double *tri_coef; const double *mom;
    const int64_t *pair_ptr; const int32_t *pair_s; int64_t ntg;
    const double *rules; const int *rule_off; const int *rule_n;   // packed rules
    const c128 *gradial; int nq;     // radial tables (G, grad G / (h d)) for |d|^2 < nq
    c128 k; double h;
    c128 *blocks;                    // [npairs][3][3][3]: L, K (precorrected), L direct
    int polar;                       // medium lossy enough for the strong-loss inner scheme
    const double *polar_gl;          // its Gauss-Legendre nodes [8] and weights [8] on [-1, 1]
    // precorrection test-node sums of rows [tab_row0, tab_row0 + rows):
    // [row][(2 tab_w + 1)^3 offsets][10], tab_w = near radius + 1
    const c128 *ptab; int64_t tab_row0; int tab_w;
    const uint8_t *pkind;            // kind | loc << 4 of pair slot p (same offset as pair_s)
    int no_grid;                     // medium without grid part: direct values, no precorrection
    // augmented EFIE (exterior medium, Sec. III-E): blocks of bstride = 45
    // values per pair also hold the precorrected and the direct vector
    // potential blocks; gam[p] receives the pair's precorrected pulse integral
    // int_t int_s G, gself[t] the direct self integral of global triangle t
    int bstride = 27;
    c128 *gam = nullptr;
    c128 *gself = nullptr;
};
// kinds[p] = kind | loc << 4 for every pair slot of a.pair_ptr / a.pair_s.
void launch_pair_kinds(const NearFillArgs &a, uint8_t *kinds, hipStream_t st);
// Fills ptab's rows (the test-node sums every pair of those rows reads).
void launch_precorr_table(const NearFillArgs &a, int64_t row0, int64_t nrows, c128 *tab, hipStream_t st);
void launch_near_fill(const NearFillArgs &a, int64_t npairs, hipStream_t st);
void launch_near_gather(int64_t nrow, int64_t rwg0, int64_t max_row, const int64_t *row_ptr, const int32_t *cols,
                        const int32_t *rwg_loc, const int32_t *glob2loc, const int32_t *tpm, const int32_t *epm,
                        const int64_t *pair_ptr, const int32_t *pair_s, const c128 *blocks, int bstride,
                        c128 *nL64, c128 *nK64, c128 *nLd64, c128 *nA64, c128 *adiag, hipStream_t st);
void launch_green_radial(c128 k, double h, int nq, c128 *gr, hipStream_t st);
void launch_green_sample(c128 k, double h, const int nl[3], const int m[3], int kind, c128 *vol, hipStream_t st);
void launch_fold_octant(const c128 *vol, const int m[3], int kind, double scale, c128 *spec64, c64 *spec32,
                        hipStream_t st);


}  // namespace sie
