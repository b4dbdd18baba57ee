/* sie.h - C ABI of the MI355X (gfx950) implementation of the AIM-accelerated
 * GIBC surface-integral-equation method of Sharma & Triverio, "An Accelerated
 * Surface Integral Equation Method for the Electromagnetic Modeling of
 * Dielectric and Lossy Objects of Arbitrary Conductivity" (arXiv:2003.11679).
 *
 * Conventions (all entry points)
 *   - Time dependence e^{+j omega t}; SI units.
 *   - Complex numbers are interleaved (re, im) pairs: sie_c128 on the host,
 *     complex64 (float re, im) or complex128 (double re, im) on the device.
 *   - Meshes: closed, oriented triangle surfaces; triangles counter-clockwise
 *     seen from outside (right-hand normal = outward normal n_i, Sec. II).
 *     0-based vertex indices.  A mesh that is not a closed consistently
 *     oriented 2-manifold is rejected with SIE_EMESH.
 *   - Unknowns: RWG coefficients (Sec. III-A) of u = n_i x H and v = n_i x E
 *     on each object.  RWG n is the interior edge {a, b}, a < b, in
 *     concatenated vertex numbering, sorted by (a, b); T+ is the triangle whose
 *     counter-clockwise order runs a -> b.  Objects are numbered in the order
 *     they are added and their RWG functions are contiguous in that order.
 *   - Media: medium -1 is the background (exterior problem, wavenumber k0);
 *     medium i >= 0 is the interior of object i (wavenumber k_i, eq. kin).
 *   - Ownership: host arrays passed in are read during the call and copied;
 *     host arrays passed out are written by the call and owned by the caller.
 *     Device pointers (hot-path calls) belong to the caller; the library never
 *     frees them and never synchronises the stream it is given except where
 *     stated.  Handles belong to the caller, who destroys them.
 *   - Errors: every call returns an sie_status; on failure nothing is thrown
 *     across the ABI, outputs are left unspecified and sie_last_error() holds a
 *     message (thread-local, valid until the next call on that thread);
 *     sie_ctx_last_error() keeps the last failure of a context.
 *   - Threads: one sie_problem is used by one host thread at a time.  Setup
 *     and solves run on the calling thread's default stream; a NULL stream
 *     passed to a hot-path call means the caller's legacy default stream.
 */
#ifndef SIE_H
#define SIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sie_ctx sie_ctx;
typedef struct sie_problem sie_problem;

typedef struct { double re, im; } sie_c128;

typedef enum {
    SIE_OK = 0,
    SIE_EINVAL = -1,     /* bad argument */
    SIE_ENOMEM = -2,     /* device or host allocation failed */
    SIE_EMESH = -3,      /* mesh not closed / not oriented / degenerate */
    SIE_EGRID = -4,      /* grid too small to hold the stencils */
    SIE_ENOCONV = -5,    /* iterative solve hit its iteration cap; best iterate kept */
    SIE_EDEVICE = -6,    /* HIP runtime error */
    SIE_ESTATE = -7      /* call out of order (e.g. matvec before setup) */
} sie_status;

typedef enum {
    SIE_FP64 = 0,        /* complex128 everywhere */
    SIE_FP32 = 1         /* complex64 projection / FFT / interpolation / SpMV;
                            solves refine in FP64 (Sec. V tolerances) */
} sie_precision;

/* Operators of one medium (Sec. III-A, eq. opL, opK; AIM form eq. AIM_Lin,
 * AIM_Kin):  A_mn = <f_m, G f_n>,  PHI_mn = <div f_m, G div f_n>,
 * L = A - k^-2 PHI,  K_mn = <f_m, PV grad G x f_n>.  X_mn = <n x f_m, f_n>
 * (the identity operator written I-cross in Sec. III-A) is medium-free. */
typedef enum {
    SIE_OP_L = 0,
    SIE_OP_K = 1,
    SIE_OP_X = 2,
    SIE_OP_AUG = 3   /* exterior rows of the augmented EFIE (sie_problem_set_augmented) */
} sie_op;

/* Quadrature orders (points per axis of the product rules) used for the
 * near-region direct integrals (Sec. III-D-1: near entries by direct
 * integration).  Pairs are classified as self / edge-adjacent /
 * vertex-adjacent ("touch"), close (centroid distance < 2.5 x longest edge)
 * and far; zeros select the defaults. */
typedef struct {
    int32_t touch_out, touch_in, close_out, close_in, far_out, far_in;
} sie_quad_params;

typedef struct {
    double tol;          /* relative residual of the outer (GIBC) system, default 1e-6 */
    double inner_tol;    /* nested solve (eq. nest2) tolerance, default 1e-8 (FP64) */
    int32_t restart;     /* GMRES restart length, default 100, at most 1000; the
                            nested solves restart after max(restart,
                            min(inner_max_iter, 300)) iterations */
    int32_t max_iter;    /* outer iteration cap, default 800 (Sec. V-A) */
    int32_t inner_max_iter; /* nested iteration cap, default 800 */
    int32_t max_refine;  /* FP64 refinement sweeps for SIE_FP32, default 10 */
    int32_t precond;     /* bit mask of preconditioners built from the direct
                            near-region operators (eq. nest2pc): 1 block-Jacobi
                            of -j w eps_i L_i,NR in the nested interior solves,
                            2 block-Jacobi of j w mu0 L0,NR in the outer solve,
                            4 the nested near-region preconditioner M_i applied
                            as restricted additive Schwarz over clusters of
                            C^3 grid cells with O cells of overlap (dense FP64
                            inverses of M_i on each extended cluster; O spans
                            about three mesh edges, C = 2 O, smaller when an
                            extended cluster would exceed 2048 functions);
                            only media whose field decays within the near
                            region (five skin depths within R grid spacings)
                            get it, the others run unpreconditioned; with 8
                            as well (12) every interior medium gets it, the
                            others with clusters of 4^3 cells and two cells
                            of overlap; 16 the same M_i factored exactly
                            (sparse LU without pivoting over the object's RWG
                            rows: FP64 multifrontal factorisation in
                            nested-dissection order, the large fronts
                            eliminated on the device, the small ones on the
                            host; device triangular solves), for each medium
                            whose M_i stays sparse enough (at most 4096 rows
                            or at most 1500 nonzeros per row on average, no
                            separator above 4096 unknowns, factors within
                            8 GB and 5e12 flops); with 4 as well (20, or 28
                            with 8) the media without a factorisation get
                            Schwarz clusters.  1 and 4 exclude each other, 1
                            and 16 too, 8 needs 4 (SIE_EINVAL); 0 none
                            (default) */
    double inner_relax;  /* relaxed nested tolerance inside each correction
                            solve (inexact Krylov relaxation, Simoncini and
                            Szyld): nested solve j runs to inner_relax x
                            (correction target) / (current outer residual
                            estimate), clamped to [t, 1e-2] with t the nested
                            tolerance (SIE_FP32: max(inner_tol, 1e-5)); 0 keeps
                            the fixed tolerance (default), and so does a
                            solve whose nested solves use the exact
                            factorisation (precond 16).  The FP64 block
                            residual of every refinement sweep still decides
                            convergence. */
    int32_t keep_converged; /* nested solves with one system per object
                            (objects of equal RWG counts) iterate the
                            objects' systems side by side; once a system has
                            converged its rows of the nested products are
                            zero and are skipped (near-field product and
                            Schwarz clusters write zeros without reading
                            their values; such products are not counted in
                            sie_report.matvecs).  1 keeps multiplying them
                            (same results, more work); default 0 */
} sie_solver_opts;

typedef struct {
    int32_t outer_iters;     /* total outer GMRES iterations (all sweeps) */
    int32_t inner_iters;     /* total nested GMRES iterations */
    int32_t inner_iters_max; /* largest nested count in one outer iteration */
    int32_t refine_sweeps;
    int64_t matvecs;         /* L-type AIM products (eq. AIM_Lin): one per medium
                                and right-hand side, FP32 and FP64 together */
    int64_t k_matvecs;       /* K-type AIM products (eq. AIM_Kin), counted alike */
    double residual;         /* final relative residual of the FP64 GIBC system */
    double t_setup_s;        /* duration of the problem's sie_problem_setup */
    double t_solve_s;
    size_t device_bytes;     /* the problem's device-memory estimate
                                (sie_problem_footprint with the solve's options) */
} sie_report;

/* ---- context --------------------------------------------------------- */

/* Binds HIP device `device`.  Returns SIE_EDEVICE if it does not exist. */
sie_status sie_ctx_create(int device, sie_ctx **out);
void sie_ctx_destroy(sie_ctx *ctx);
/* Frees the device memory the library keeps for reuse (see
 * sie_problem_destroy) on the context's device, e.g. before the caller
 * allocates much device memory of its own.  Kept blocks outlive contexts. */
sie_status sie_ctx_trim(sie_ctx *ctx);
const char *sie_last_error(void);

/* ---- launch-shape tuning (process-wide) ------------------------------ */
/* The grid stages of the AIM product (Sec. III-D-1: projection, the five
 * passes of the zero-padded FFT convolution, interpolation) run with launch
 * shapes chosen per problem shape: FFT tile shapes (threads and values per
 * thread of a block, hence the lines per LDS tile) of the strided y passes
 * and the fused z pass, and the block sizes of projection and
 * interpolation.  All candidates of a stage compute identical values; only
 * the time differs.  mode 1 (default): on the first product of a shape the
 * candidates are timed on the caller's stream (a few launches each, on the
 * product's own buffers before they hold data) and the fastest is kept per
 * device for the rest of the process; not while the stream is being
 * captured, not in sie_matvec_noalloc, and not while another thread tunes
 * (that product uses the built-in shapes).  mode 0: built-in shapes only
 * (choices already made are still used). */
sie_status sie_set_tuning(int32_t mode);
/* Testing: stage `family` (0 y forward, 1 y inverse, 2 z pass, 3
 * projection, 4 interpolation) always uses candidate `candidate` (-1:
 * choose as above).  SIE_EINVAL for an unknown family; a candidate beyond
 * the stage's list fails the next product of that stage with SIE_EINVAL. */
sie_status sie_tuning_force(int32_t family, int32_t candidate);
/* The choices made so far, one text line per stage and shape (candidate
 * times in microseconds, -1 where a candidate did not run).  Writes at most
 * len bytes including the terminating NUL into buf (may be NULL with len 0);
 * *needed (if not NULL) receives the full length including the NUL. */
sie_status sie_tuning_report(char *buf, size_t len, size_t *needed);
/* Forgets the choices made so far. */
sie_status sie_tuning_clear(void);
/* Message of the last failing call made with this context (through a
 * problem or server created on it); "" if none.  Valid until the next
 * failing call on the context. */
const char *sie_ctx_last_error(const sie_ctx *ctx);

/* ---- problem definition (Sec. II: objects with (eps_i, mu_i, sigma_i) in a
 * homogeneous background; Sec. III-A: triangle meshes) ------------------- */

sie_status sie_problem_create(sie_ctx *ctx, double freq_hz, double bg_eps_r, double bg_mu_r,
                              sie_problem **out);
/* xyz: [nv][3] float64 metres; tri: [nt][3] int32.  eps_r, mu_r relative;
 * sigma in S/m.  Writes the object index to *obj_id (may be NULL). */
sie_status sie_problem_add_object(sie_problem *p, const double *xyz, int64_t nv,
                                  const int32_t *tri, int64_t nt, double eps_r, double mu_r,
                                  double sigma, int32_t *obj_id);
/* Grid of medium `medium` (Sec. III-D-1: one Cartesian grid per object plus
 * one global exterior grid, eq. AIM_Lin): n points per axis (isotropic
 * spacing h = largest bounding-box extent / (n - 3)), Chebyshev near radius
 * in cells (5 = a near region 11 points across).  With `share` != 0 an
 * interior medium reuses the exterior grid (single-object problems).
 * Defaults: exterior n from the lambda_r/20 rule of Sec. IV, capped at 256;
 * interiors share the exterior grid when there is one object. */
sie_status sie_problem_set_grid(sie_problem *p, int32_t medium, int32_t n, int32_t near_radius,
                                int32_t share);

/* Grid parameters of one medium (Sec. III-D-1 grid, Sec. IV spacing).  As
 * input to sie_problem_set_grid_params: h > 0 and n > 0 fix the spacing and
 * the points per axis, with origin[] the grid's first node (zero h or n: the
 * rule below; an origin of NaN centres the grid on the medium's objects);
 * order is the stencil order (points per axis - 1; only 2 is built, anything
 * else is SIE_EINVAL; 0 means 2); near_radius the Chebyshev near radius in
 * cells (0 = 5, a near region 11 points across, Sec. IV-A).  As output of
 * sie_grid_choose every field is set. */
typedef struct {
    double h;
    int32_t n;
    double origin[3];
    int32_t order;
    int32_t near_radius;
    double loss_ratio;   /* out: worst Delta G_n / Delta G_n,lossless beyond the near region */
    double lambda_r;     /* out: 2 pi / k_r, the medium's wavelength without losses */
} sie_grid_params;

/* Grid rule of Sec. IV for a medium (eps_r, mu_r, sigma) at freq_hz, objects
 * of largest bounding-box extent `extent` and mean mesh edge `mean_edge`:
 * spacing lambda_r / 20 with lambda_r = 2 pi / (k0 sqrt(eps_r mu_r)) (the
 * lossy error bound of eq. LboundsD2 stays within ~1.5 of the lossless one
 * for one grid, so losses do not refine it), with strict != 0 further refined
 * by the (order+1)-th root of the worst lossy/lossless bound ratio (eq. Ddef)
 * beyond the near region, and never coarser than the mean edge (a stencil
 * spans a triangle); n = ceil(extent / h) + 3 points (one spare node a side),
 * clamped to [5, 1024], and h = extent / (n - 3).  Host-only; needs no device.
 * The library applies this rule to every grid whose n is 0, taking the finest
 * spacing over the media that share the grid. */
sie_status sie_grid_choose(double freq_hz, double eps_r, double mu_r, double sigma, double extent,
                           double mean_edge, int32_t near_radius, int32_t strict, sie_grid_params *out);
/* Grid of a medium from explicit parameters (see sie_grid_params); the
 * interior of a single object shares the exterior grid unless share == 0. */
sie_status sie_problem_set_grid_params(sie_problem *p, int32_t medium, const sie_grid_params *g,
                                       int32_t share);
sie_status sie_problem_set_quadrature(sie_problem *p, const sie_quad_params *q);
/* Skin-depth cutoff of the interior problem (Sec. V: interactions of
 * triangles more than `skin_depths` skin depths apart are ignored; the paper
 * uses 5; 0 turns it off, the default).  Two triangles are apart when their
 * centroids are farther than the cutoff plus both bounding radii about the
 * centroids (touching triangles never are).  The cutoff applies to an
 * interior medium whose cutoff lies within its near region (every far pair
 * beyond it): the medium then has no grid part, its near list keeps the pairs
 * within the cutoff and its operator is the direct near-region one
 * (Sec. III-D-2 item a); an interior that would share the exterior grid gets
 * the exterior grid's geometry with a near list of its own.  Elsewhere the
 * AIM operator is kept unchanged.  Independently of the cutoff, a medium
 * whose grid has every pair near (objects within the near region,
 * Sec. III-D-2 item b) also runs without grid part: the grid part would
 * equal its precorrection. */
sie_status sie_problem_set_skin_cutoff(sie_problem *p, double skin_depths);
/* Augmented EFIE for the exterior problem (Sec. III-E, eq. sys), set before
 * setup; on = 1 or 0 (default).  The surface charge becomes an unknown, one
 * pulse per triangle: with sigma = c0 rho, Dv[t][n] = div f_n on triangle t
 * (+-l_n / A_t) and Gam[t][s] = int_t int_s G0,
 *   [ j k0 A0 - (K0 - X/2) Z / eta0 , -Dv^T Gam ] [ u     ]   [ e / eta0 ]
 *   [ W Dv                          ,  j k0 W   ] [ sigma ] = [ 0        ]
 * (A0 the vector-potential part of L0, Z the GIBC operator of eq. GIBCdef,
 * W = diag(A_t / k0) weighting the continuity rows).  Eliminating sigma
 * gives the GIBC system divided by eta0, so u is the same.  Setup then also
 * keeps the precorrected A0 and pulse near values, and factors the Schur
 * complement S = j k0 I + Dv diag(j k0 A0_nn)^-1 Dv^T diag(Gam_tt) of the
 * constraint preconditioner (sparse LU, FP64, host and device fronts;
 * SIE_EINVAL from setup when a separator of its nested dissection exceeds
 * 4096 triangles or the factors exceed 8 GB or 5e12 flops).  Solves
 * then iterate on (u, sigma) with that preconditioner (the outer-solve
 * preconditioner bit 2 is ignored), and their residual is that of the
 * augmented block system. */
sie_status sie_problem_set_augmented(sie_problem *p, int32_t on);
/* After setup: *on (1 if set up augmented), stored off-diagonal entries of
 * the Schur factors, levels of the dissection tree, host factorisation time.
 * Any output may be NULL. */
sie_status sie_problem_augmented_info(const sie_problem *p, int32_t *on, int64_t *factor_nnz, int32_t *levels,
                                      double *t_factor_s);
/* 1 if the medium runs without grid part (see sie_problem_set_skin_cutoff),
 * 0 if it has one, negative sie_status on error. */
int32_t sie_medium_is_local(const sie_problem *p, int32_t medium);
/* Builds RWG topology, grids, stencils and projection moments, near lists,
 * precorrected near-field matrices (FP64 direct integrals on the device) and
 * Green's spectra for every medium.  Synchronous. */
sie_status sie_problem_setup(sie_problem *p);
/* Synchronises the device; the problem's device memory stays with the
 * library for reuse by later problems on the device (blocks beyond half of
 * the device's memory are freed), so that a request that repeats an earlier
 * one maps no new memory.  sie_ctx_trim frees what is kept. */
void sie_problem_destroy(sie_problem *p);

/* ---- queries --------------------------------------------------------- */

int64_t sie_problem_num_rwg(const sie_problem *p);      /* all objects; -1 before setup */
int64_t sie_problem_num_tri(const sie_problem *p);
/* RWG records (host arrays): edge_v [E][2] (a < b), tpm [E][2] (T+, T-). */
sie_status sie_get_rwg(const sie_problem *p, int32_t *edge_v, int32_t *tpm);
/* Grid of a medium: origin [3], h, n [3] (full grid), lo [3] and nl [3]
 * (live box of stencil nodes), m [3] (FFT lengths, powers of two >= 2 nl - 1). */
sie_status sie_get_grid(const sie_problem *p, int32_t medium, double *origin, double *h,
                        int32_t *n, int32_t *lo, int32_t *nl, int32_t *m);
/* Stencil centre (integer grid index, 3 per triangle) of every triangle of the
 * medium's grid, in the grid's triangle order (all triangles of the objects the
 * grid covers, ascending).  out: [nt_grid][3]; *nt_grid receives the count. */
sie_status sie_get_stencils(const sie_problem *p, int32_t medium, int32_t *out, int64_t *nt_grid);
/* Stencil assignment on the device (Sec. III-D-1, the integer grid index of
 * each triangle's stencil centre: floor((c - origin) / h + 0.5) of the centroid
 * c = ((v0 + v1) + v2) / 3, clamped to [1, n - 2]) for every triangle of the
 * medium's grid, in ascending global triangle order, into centre_dev [nt][3]
 * int32 (device memory of the caller, nt from sie_get_stencils) on the
 * caller's stream; recomputes what setup assigned. */
sie_status sie_stencil_assign(sie_problem *p, int32_t medium, int32_t *centre_dev, void *stream);
/* Near-field CSR of a medium (RWG rows/cols of the medium's objects, global
 * numbering): row_ptr [E+1] int64, cols [nnz] int32.  With row_ptr == NULL
 * only *nnz is written. */
sie_status sie_get_near_pattern(const sie_problem *p, int32_t medium, int64_t *row_ptr,
                                int32_t *cols, int64_t *nnz);
/* Precorrected near-field values (L or K, eq. LinNRP/KinNRP) in FP64, in the
 * CSR order of sie_get_near_pattern: out [nnz]. */
sie_status sie_get_near_values(const sie_problem *p, int32_t medium, sie_op op, sie_c128 *out);
/* Wavenumber of a medium (eq. kin, principal branch, Im k <= 0). */
sie_status sie_get_wavenumber(const sie_problem *p, int32_t medium, sie_c128 *k);

/* ---- hot path (device pointers, caller's stream, no host synchronisation) */

/* y = Op_medium x for nrhs right-hand sides stored [nrhs][E] contiguous
 * (E = sie_problem_num_rwg), complex64 for SIE_FP32 and complex128 for
 * SIE_FP64.  Op = L or K: AIM product near + W G P (eq. AIM_Lin / AIM_Kin);
 * rows and columns outside the medium's objects are zero.  Op = X: medium
 * ignored.  medium = SIE_INTERIORS: every object's interior operator on its
 * own rows (the block-diagonal operator whose blocks eq. nest2 inverts,
 * without its -j w eps_i factors), computed the way the solver does: the
 * objects whose grids share a shape in one launch per stage. */
#define SIE_INTERIORS (-2)
/* Op = SIE_OP_AUG (medium -1, SIE_FP64, problem set up augmented): x and y
 * are [nrhs][E + T] (T triangles), [u; sigma] in and
 * [j k0 A0 u - Dv^T Gam sigma; W (Dv u + j k0 sigma)] out, the AIM product
 * of the exterior rows of eq. sys without the GIBC term (the vector fields
 * projected from u, the scalar field from the pulse charges). */
sie_status sie_matvec(sie_problem *p, int32_t medium, sie_op op, sie_precision prec, int32_t nrhs,
                      const void *x_dev, void *y_dev, void *stream);
/* Allocation-free form of sie_matvec, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): one right-hand side [E], same operators and result as
 * sie_matvec, but the stage intermediates (grid sources and potentials, FFT
 * pass buffers, per-triangle partials) live in a library-owned device array of
 * SIE_NOALLOC_SCRATCH_BYTES per device (held from the first sie_ctx_create on
 * that device until the process ends) instead of buffers the problem
 * allocates.  The call allocates and frees nothing and does not synchronise.
 * SIE_EINVAL when the medium's intermediates exceed the array (about 64 MiB
 * holds an L product on a live box of ~1.6e6 complex64 nodes per field, or
 * half that in FP64); SIE_EDEVICE when the problem's device is not current.
 * All calls on one device share the array: calls that overlap on a device
 * (two streams, two threads) race and must be serialised by the caller. */
#define SIE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
sie_status sie_matvec_noalloc(sie_problem *p, int32_t medium, sie_op op, sie_precision prec,
                              const void *x_dev, void *y_dev, void *stream);
/* The stages of one AIM product, exposed for stage-level checks: grid
 * sources [4][nl_z][nl_y][nl_x] (J_x, J_y, J_z, charge; x fastest) from RWG
 * coefficients (projection P, P_phi); the zero-padded FFT convolution on the
 * live box (Sec. III-D-1), op = SIE_OP_L: each of nfields (1..4) grids with
 * G, op = SIE_OP_K: the 3 grids (J_x, J_y, J_z) to grad G x J (nfields = 3);
 * interpolation W back to RWG (vector fields minus k^-2 times the scalar
 * field).  in and out may be the same buffer. */
sie_status sie_project(sie_problem *p, int32_t medium, sie_precision prec, const void *x_dev,
                       void *grid_dev, void *stream);
sie_status sie_convolve(sie_problem *p, int32_t medium, sie_op op, sie_precision prec, int32_t nfields,
                        const void *grid_in_dev, void *grid_out_dev, void *stream);
sie_status sie_interpolate(sie_problem *p, int32_t medium, sie_precision prec,
                           const void *grid_dev, void *y_dev, void *stream);

/* Nested-solve preconditioner (eq. nest2pc, M_i = -j w eps_i L_i,NR of every
 * object's interior medium), applied to nrhs vectors [nrhs][E] on the
 * caller's stream: precond = 1 block-Jacobi, 4 or 12 restricted additive
 * Schwarz over grid-cell clusters, 16 the exact sparse LU of M_i, 20 or 28
 * the LU where it applies and clusters elsewhere (see
 * sie_solver_opts.precond; rows of media with neither are copied).  Built
 * on first use (host-synchronous); the same structure serves later solves.
 * x and y must not alias; complex64 for SIE_FP32 (Schwarz inverses and LU
 * factors in FP32 copies), complex128 for SIE_FP64.  SIE_ESTATE before
 * setup. */
sie_status sie_nested_precond(sie_problem *p, int32_t precond, sie_precision prec, int32_t nrhs,
                              const void *x_dev, void *y_dev, void *stream);
/* Clusters of the built Schwarz preconditioner (-1 if not built); *owned
 * (nullable) receives the number of RWG rows they own. */
int32_t sie_nested_precond_clusters(const sie_problem *p, int64_t *owned);
/* Interior media with an exact near-region factorisation (precond bit 16;
 * -1 if not built); *factor_nnz (nullable) receives the stored off-block
 * entries of their L and U factors, *t_factor_s (nullable) the wall time of
 * the factorisations (ordering and symbolic part on the host, fronts on the
 * device or the host). */
int32_t sie_nested_precond_factored(const sie_problem *p, int64_t *factor_nnz, double *t_factor_s);

/* Constraint preconditioner of the augmented EFIE (Sec. III-E), y = P^-1 x
 * for nrhs vectors [nrhs][E + T] complex128 on the caller's stream, with
 *   P = [ j k0 diag(A0_nn) , -Dv^T diag(Gam_tt) ]
 *       [ W Dv             ,  j k0 W            ]
 * applied by block elimination through the factored Schur complement (see
 * sie_problem_set_augmented).  x and y must not alias.  SIE_ESTATE unless
 * set up augmented. */
sie_status sie_constraint_precond(sie_problem *p, int32_t nrhs, const void *x_dev, void *y_dev, void *stream);

/* Stage timers (HIP events recorded on the stream of each product).
 * sie_set_timing(p, 1) starts recording every stage, sie_set_timing(p, 2)
 * the near-field CSR product alone (stages 3 and 5: two events per product
 * instead of ten), 0 stops; each call clears the totals.  Stages:
 * 0 projection, 1 FFT convolution, 2 interpolation, 3 near-field CSR product
 * (the k_spmv_far kernel alone), 4 whole operator product, 5 the FP64
 * near-field CSR products alone (also counted in 3), 6 and 7 the near-field
 * CSR products of the interior media inside solves (the nested operator of
 * eq. nest2, one launch per group of media) in FP32 and FP64 (also counted
 * in 3, and 7 in 5), 8 the interior near-field products of nested solves
 * that skip the rows of objects whose systems have converged (counted in 3
 * only, not in 5, 6 or 7).  Query returns the
 * number of timed launches and their summed duration (synchronises). */
sie_status sie_set_timing(sie_problem *p, int32_t on);
sie_status sie_get_stage_time(sie_problem *p, int32_t stage, int64_t *launches, double *total_ms);

/* ---- solve (Sec. III-C: GIBC with AIM-accelerated nested interior solves,
 * eq. GIBCsys, nest02, nest2) --------------------------------------------- */

/* Plane waves (Sec. II): E_inc = e0 exp(-j k0 khat . r); khat [nrhs][3] unit,
 * e0 [nrhs][3] complex (V/m). */
sie_status sie_set_planewaves(sie_problem *p, int32_t nrhs, const double *khat, const sie_c128 *e0);
/* Solves the GIBC system for every plane wave.  opts may be NULL (defaults);
 * report may be NULL.  Synchronous.  SIE_ENOCONV: cap reached, best iterate
 * kept and readable. */
sie_status sie_solve(sie_problem *p, sie_precision prec, const sie_solver_opts *opts,
                     sie_report *report);
/* Currents of right-hand side `rhs` (host arrays [E]). */
sie_status sie_get_currents(const sie_problem *p, int32_t rhs, sie_c128 *u, sie_c128 *v);
/* Charge unknowns sigma = c0 rho (one pulse per triangle, host array [T]) of
 * right-hand side `rhs` of an augmented solve (Sec. III-E); SIE_ESTATE if the
 * problem is not set up augmented or not solved. */
sie_status sie_get_charges(const sie_problem *p, int32_t rhs, sie_c128 *sigma);
/* Scattered far-field amplitude F (E_s ~ F exp(-j k0 r)/r) of right-hand side
 * `rhs` in the directions rhat [ndir][3]: F [ndir][3] (host). */
sie_status sie_far_field(const sie_problem *p, int32_t rhs, int64_t ndir, const double *rhat,
                         sie_c128 *F);
/* The same in spherical components (Sec. V-A far field / RCS): directions
 * (theta[i], phi[i]) in radians, e_theta[i] = F . theta-hat and
 * e_phi[i] = F . phi-hat (host arrays [ndir]); the RCS of unit incidence is
 * 4 pi (|e_theta|^2 + |e_phi|^2). */
sie_status sie_far_field_angles(const sie_problem *p, int32_t rhs, int64_t ndir, const double *theta,
                                const double *phi, sie_c128 *e_theta, sie_c128 *e_phi);

/* ---- serving: continuous batching of independent solve requests
 *
 * A server runs queued solve requests concurrently on worker threads of one
 * device (each on its own stream), admitting requests first-in first-out
 * while the sum of their device-memory footprint estimates stays within the
 * budget (a request larger than the budget still runs when nothing else
 * does).  A request is a problem with its objects and grids described
 * (sie_problem_setup not yet called, or already called), plus plane waves,
 * precision and solver options; the worker runs setup, plane waves and the
 * solve.  Serving is not described in the paper: it is the deployment form
 * of the per-request pipeline of Sec. III. */
typedef struct sie_server sie_server;

typedef struct {
    int32_t done;           /* 0 queued or running, 1 finished */
    int32_t running;        /* 1 while a worker holds the request */
    sie_status status;      /* result of the request once done (SIE_OK,
                               SIE_ENOCONV or the error of setup / solve) */
    double t_submit_s;      /* times on the server's clock (s since creation) */
    double t_start_s;
    double t_end_s;
    size_t footprint;       /* the estimate the request was admitted with */
    sie_report report;      /* the solve's report once done */
    char message[256];      /* error message of a failed request ("" if none) */
} sie_job_info;

/* Device-memory estimate (bytes) of a problem's setup and solve: near-field
 * CSR values of every medium (FP64 and FP32), grid buffers and spectra, the
 * largest near-field fill transient (pair blocks and precorrection tables of
 * one chunk), and the Krylov bases of the default solver options; available
 * before setup. */
sie_status sie_problem_footprint(const sie_problem *p, size_t *device_bytes);
/* hbm_budget_bytes 0: 80 % of the device memory free at creation (blocks
 * the library keeps for reuse count as free);
 * max_slots: concurrent requests (worker threads), 1..64. */
sie_status sie_server_create(sie_ctx *ctx, size_t hbm_budget_bytes, int32_t max_slots, sie_server **out);
/* Queues a request; the server owns p until sie_server_take.  khat / e0 as
 * in sie_set_planewaves (copied); opts may be NULL.  *ticket identifies the
 * request. */
sie_status sie_server_submit(sie_server *s, sie_problem *p, int32_t nrhs, const double *khat,
                             const sie_c128 *e0, sie_precision prec, const sie_solver_opts *opts,
                             uint64_t *ticket);
/* State of a request (non-blocking). */
sie_status sie_server_poll(sie_server *s, uint64_t ticket, sie_job_info *info);
/* Blocks until the request is done, then hands the problem back (currents
 * and far fields readable if its status allows) and forgets the ticket. */
sie_status sie_server_take(sie_server *s, uint64_t ticket, sie_problem **out);
/* Waits for the running requests, destroys the problems still owned by the
 * server and frees it. */
void sie_server_destroy(sie_server *s);

#ifdef __cplusplus
}
#endif
#endif /* SIE_H */
