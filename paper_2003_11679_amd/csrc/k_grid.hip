// Grid-side stages of the AIM product (Sec. III-D-1, eq. AIM_Lin / AIM_Kin):
// stencil assignment, projection moments, projection P / P_phi (a gather over
// per-node source lists, so results do not depend on thread scheduling),
// interpolation W = P^T and the near-field CSR product that also adds the
// interpolated far part.
//
// Projection weights of RWG n on triangle t at stencil node a (27 nodes,
// tensor Lagrange polynomials l_a of the 3-point stencil, moment matching up
// to degree 2 per axis):
//   P_n(a)     = c_e (M1_t[a] - q_e M0_t[a]),   P_phi,n(a) = 2 c_e M0_t[a]
//   M0_t[a] = int_t l_a dS,  M1_t[a] = int_t l_a (r - r_c) dS,
//   c_e = +-l/(2A),  q_e = (vertex opposite edge e) - r_c,  r_c = stencil centre.
#include "common.h"
#include "kernels.h"
#include "tune.h"

namespace sie {

// Triangle i of the launch is tris[i], or t0 + i without a list; raw
// (nullable) receives the unclamped index.
__global__ void k_stencil_assign(const double *__restrict__ centroids, const int32_t *__restrict__ tris,
                                 int64_t t0, int64_t ntg, double ox, double oy, double oz, double h, int nx, int ny,
                                 int nz, int32_t *__restrict__ centre, int32_t *__restrict__ raw) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= ntg) return;
    const int64_t t = tris ? tris[i] : t0 + i;
    const double o[3] = {ox, oy, oz};
    const int n[3] = {nx, ny, nz};
    for (int c = 0; c < 3; ++c) {
        // IEEE subtraction, division, addition; no contraction possible
        double q = (centroids[3 * t + c] - o[c]) / h;
        double f = floor(q + 0.5);
        int v = (int)f;
        if (raw) raw[3 * i + c] = v;
        centre[3 * i + c] = v < 1 ? 1 : (v > n[c] - 2 ? n[c] - 2 : v);
    }
}

void launch_stencil_assign(const double *centroids, const int32_t *tris, int64_t t0, int64_t ntg,
                           const double origin[3], double h, const int n[3], int32_t *centre_out, int32_t *raw_out,
                           hipStream_t st) {
    if (ntg == 0) return;
    hipLaunchKernelGGL(k_stencil_assign, dim3((unsigned)((ntg + 255) / 256)), dim3(256), 0, st, centroids, tris,
                       t0, ntg, origin[0], origin[1], origin[2], h, n[0], n[1], n[2], centre_out, raw_out);
    SIE_HIP(hipGetLastError());
}

// One thread per triangle: 27 x (M0, M1) by a quadrature rule exact for the
// degree-7 integrands (rule: [nq][4] = bary0, bary1, bary2, weight).
__global__ void k_moments(const double *__restrict__ xyz, const int32_t *__restrict__ tri,
                          const int32_t *__restrict__ tris, const int32_t *__restrict__ centre, int64_t ntg,
                          double ox, double oy, double oz, double h, const double *__restrict__ rule, int nq,
                          double *__restrict__ mom64, float *__restrict__ mom32) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= ntg) return;
    const int64_t t = tris[i];
    double v[3][3];
    for (int k = 0; k < 3; ++k)
        for (int c = 0; c < 3; ++c) v[k][c] = xyz[3 * (int64_t)tri[3 * t + k] + c];
    const double rc[3] = {ox + h * centre[3 * i], oy + h * centre[3 * i + 1], oz + h * centre[3 * i + 2]};
    double e1[3], e2[3];
    for (int c = 0; c < 3; ++c) { e1[c] = v[1][c] - v[0][c]; e2[c] = v[2][c] - v[0][c]; }
    double cr0 = e1[1] * e2[2] - e1[2] * e2[1], cr1 = e1[2] * e2[0] - e1[0] * e2[2], cr2 = e1[0] * e2[1] - e1[1] * e2[0];
    const double A = 0.5 * sqrt(cr0 * cr0 + cr1 * cr1 + cr2 * cr2);
    double M[27][4];
    for (int a = 0; a < 27; ++a) M[a][0] = M[a][1] = M[a][2] = M[a][3] = 0.0;
    for (int q = 0; q < nq; ++q) {
        const double b0 = rule[4 * q], b1 = rule[4 * q + 1], b2 = rule[4 * q + 2], w = rule[4 * q + 3] * A;
        double d[3], l[3][3];
        for (int c = 0; c < 3; ++c) {
            d[c] = b0 * v[0][c] + b1 * v[1][c] + b2 * v[2][c] - rc[c];
            const double xi = d[c] / h;
            l[c][0] = 0.5 * xi * (xi - 1.0);
            l[c][1] = 1.0 - xi * xi;
            l[c][2] = 0.5 * xi * (xi + 1.0);
        }
        for (int cz = 0; cz < 3; ++cz)
            for (int cy = 0; cy < 3; ++cy)
                for (int cx_ = 0; cx_ < 3; ++cx_) {
                    const int a = (cz * 3 + cy) * 3 + cx_;
                    const double wl = w * l[0][cx_] * l[1][cy] * l[2][cz];
                    M[a][0] += wl;
                    M[a][1] += wl * d[0];
                    M[a][2] += wl * d[1];
                    M[a][3] += wl * d[2];
                }
    }
    for (int a = 0; a < 27; ++a)
        for (int c = 0; c < 4; ++c) {
            mom64[(i * 27 + a) * 4 + c] = M[a][c];
            mom32[(i * 27 + a) * 4 + c] = (float)M[a][c];
        }
}

void launch_moments(const double *xyz, const int32_t *tri, const int32_t *tris, const int32_t *centre,
                    int64_t ntg, const double origin[3], double h, const double *rule, int nq,
                    double *mom64, float *mom32, hipStream_t st) {
    if (ntg == 0) return;
    hipLaunchKernelGGL(k_moments, dim3((unsigned)((ntg + 127) / 128)), dim3(128), 0, st, xyz, tri, tris, centre,
                       ntg, origin[0], origin[1], origin[2], h, rule, nq, mom64, mom32);
    SIE_HIP(hipGetLastError());
}

// Per-triangle projection coefficients: alpha = sum_e x_e c_e and
// beta = sum_e x_e c_e q_e (trisrc[t] = alpha, beta_x, beta_y, beta_z).
template <typename T>
__global__ void k_tri_sources(int64_t ntg, const int32_t *__restrict__ tri_rwg, const T *__restrict__ coef,
                              const cx<T> *__restrict__ x, int64_t ldx, cx<T> *__restrict__ src) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= ntg) return;
    x += blockIdx.y * ldx;                 // right-hand side blockIdx.y
    src += blockIdx.y * 4 * ntg;
    cx<T> a, bx, by, bz;
    for (int e = 0; e < 3; ++e) {
        const cx<T> xv = x[tri_rwg[3 * t + e]];
        const T *c = coef + (t * 3 + e) * 4;
        const cx<T> cxv = c[0] * xv;
        a += cxv;
        bx += c[1] * cxv; by += c[2] * cxv; bz += c[3] * cxv;
    }
    src[4 * t] = a; src[4 * t + 1] = bx; src[4 * t + 2] = by; src[4 * t + 3] = bz;
}

template <typename T>
void launch_tri_sources(const GridView &g, const T *tri_coef, const cx<T> *x, int64_t ldx, int nrhs, cx<T> *trisrc,
                        hipStream_t st) {
    const int32_t *tri_rwg_loc = g.trirwg;
    const int64_t ntg = g.ntg;
    if (!ntg || nrhs < 1) return;
    SIE_CHECK(nrhs <= 65535, SIE_EINVAL, "too many right-hand sides");
    hipLaunchKernelGGL(k_tri_sources<T>, dim3((unsigned)((ntg + 255) / 256), (unsigned)nrhs), dim3(256), 0, st, ntg,
                       tri_rwg_loc, tri_coef, x, ldx, trisrc);
    SIE_HIP(hipGetLastError());
}

// Threads per block the tuner chooses among for projection and
// interpolation (the first is the built-in size).
constexpr int kNumStageBlocks = 4;
constexpr int kStageBlocks[kNumStageBlocks] = {256, 128, 512, 64};

// Gather projection: `lpn` lanes (a power of two <= 64) per live node share
// its entry list and reduce with lane shuffles.  grid [F][nlive] with
// J_c = sum (alpha M1_c - beta_c M0) and (F == 4) Q = sum 2 alpha M0, the
// RWG divergences; with rho given (augmented EFIE, Sec. III-E), Q = sum
// rho_t M0 of the pulse charges instead (rho [rhs][T] in the global triangle
// numbering, stride ldr; rho_tris maps the view's triangles to it).
template <typename T>
__device__ inline T seg_sum(T v, int lpn) {
    for (int off = lpn >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T>
__global__ void k_project(int64_t nnodes, int64_t nlive, const int32_t *__restrict__ node_ptr,
                          const int32_t *__restrict__ ent, const T *__restrict__ mom, const cx<T> *__restrict__ src,
                          cx<T> *__restrict__ grid, int nf, int lpn, int64_t ntg, const cx<T> *__restrict__ rho,
                          int64_t ldr, const int32_t *__restrict__ rho_tris, const uint8_t *__restrict__ active,
                          int obj0) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t v = gid / lpn;
    // nodes of inactive slots are left as they are: nothing downstream
    // reads them (uniform over the node's lanes)
    if (active && v < nnodes && !active[obj0 + (int)(v / nlive)]) return;
    src += blockIdx.y * 4 * ntg;           // right-hand side blockIdx.y
    grid += blockIdx.y * nf * nnodes;
    if (rho) rho += blockIdx.y * ldr;
    const int sub = (int)(gid % lpn);
    // every lane of a wave takes part in the shuffles; out-of-range nodes add zeros
    T s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (v < nnodes) {
        for (int k = node_ptr[v] + sub; k < node_ptr[v + 1]; k += lpn) {
            const int32_t e = ent[k];
            const int64_t t = e >> 5;
            const int a = e & 31;
            const T *m = mom + (t * 27 + a) * 4;
            const cx<T> al = src[4 * t], bx = src[4 * t + 1], by = src[4 * t + 2], bz = src[4 * t + 3];
            s[0] += m[1] * al.re - m[0] * bx.re; s[1] += m[1] * al.im - m[0] * bx.im;
            s[2] += m[2] * al.re - m[0] * by.re; s[3] += m[2] * al.im - m[0] * by.im;
            s[4] += m[3] * al.re - m[0] * bz.re; s[5] += m[3] * al.im - m[0] * bz.im;
            if (rho) {
                const cx<T> q = rho[rho_tris[t]];
                s[6] += m[0] * q.re; s[7] += m[0] * q.im;
            } else {
                s[6] += m[0] * al.re; s[7] += m[0] * al.im;
            }
        }
    }
    for (int i = 0; i < 8; ++i) s[i] = seg_sum(s[i], lpn);
    if (v < nnodes && sub == 0) {
        // node v of slot v / nlive: fields of a slot are nf consecutive blocks
        const int64_t slot = v / nlive;
        cx<T> *o = grid + slot * (nf - 1) * nlive + v;
        o[0] = cx<T>(s[0], s[1]);
        o[nlive] = cx<T>(s[2], s[3]);
        o[2 * nlive] = cx<T>(s[4], s[5]);
        if (nf == 4) o[3 * nlive] = rho ? cx<T>(s[6], s[7]) : cx<T>(T(2) * s[6], T(2) * s[7]);
    }
}

template <typename T>
void launch_project(const GridView &g, const T *mom, const cx<T> *trisrc, cx<T> *grid, int nfields, int nrhs,
                    hipStream_t st, const cx<T> *rho, int64_t ldr, const int32_t *rho_tris) {
    SIE_CHECK(!rho || rho_tris, SIE_EINVAL, "pulse charges need the view's triangle numbers");
    const int64_t nnodes = g.nnodes();
    if (nrhs < 1) return;
    SIE_CHECK(nrhs <= 65535, SIE_EINVAL, "too many right-hand sides");
    // lanes per node: about two entries per lane on average
    const double avg = 27.0 * (double)g.ntg / (double)std::max<int64_t>(nnodes, 1);
    int lpn = 1;
    while (lpn < 64 && lpn * 2 <= avg / 2.0) lpn *= 2;
    const int64_t threads = nnodes * lpn;
    // block size: tuned among kStageBlocks (lpn divides each, so a node's
    // lanes stay in one wavefront)
    auto run = [&](int c) {
        const int bs = kStageBlocks[c];
        hipLaunchKernelGGL(k_project<T>, dim3((unsigned)((threads + bs - 1) / bs), (unsigned)nrhs), dim3(bs), 0, st,
                           nnodes, g.nlive, g.node_ptr, g.node_ent, mom, trisrc, grid, nfields, lpn, g.ntg, rho, ldr,
                           rho_tris, nrhs == 1 ? g.active : nullptr, g.obj0);
        SIE_HIP(hipGetLastError());
        return true;
    };
    int dev = 0;
    SIE_HIP(hipGetDevice(&dev));
    const TuneKey key{dev, TUNE_PROJECT, (int)sizeof(T), {nnodes, g.ntg, nfields, nrhs, lpn + (rho ? 1000 : 0)}};
    run(tune_pick(key, kNumStageBlocks, run, st));
}

// Interpolation partials per triangle: psi = sum_a M1[a] . F_vec(a),
// chi = sum_a M0[a] F_vec(a), zeta = sum_a M0[a] F_scal(a) (F == 4).
template <typename T>
__global__ void k_interp(int64_t ntg, const int32_t *__restrict__ centre, const int32_t *__restrict__ tri_slot,
                         int lox, int loy, int loz, int nlx, int nly, int64_t nlive, int64_t nnodes,
                         const T *__restrict__ mom, const cx<T> *__restrict__ pot, int nf, cx<T> *__restrict__ out,
                         const uint8_t *__restrict__ active, int obj0) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= ntg) return;
    // triangles of inactive slots: their rows of the near-field product are
    // zero and do not read these partials
    if (active && !active[obj0 + (tri_slot ? tri_slot[t] : 0)]) return;
    pot += blockIdx.y * nf * nnodes;       // right-hand side blockIdx.y
    if (tri_slot) pot += (int64_t)tri_slot[t] * nf * nlive;
    out += blockIdx.y * 5 * ntg;
    const int cxi = centre[3 * t] - lox, cyi = centre[3 * t + 1] - loy, czi = centre[3 * t + 2] - loz;
    cx<T> psi, chx, chy, chz, zeta;
    for (int dz = 0; dz < 3; ++dz)
        for (int dy = 0; dy < 3; ++dy)
            for (int dx = 0; dx < 3; ++dx) {
                const int a = (dz * 3 + dy) * 3 + dx;
                const int64_t v = ((int64_t)(czi + dz - 1) * nly + (cyi + dy - 1)) * nlx + (cxi + dx - 1);
                const T *m = mom + (t * 27 + a) * 4;
                const cx<T> fx = pot[v], fy = pot[nlive + v], fz = pot[2 * nlive + v];
                psi += m[1] * fx + m[2] * fy + m[3] * fz;
                chx += m[0] * fx; chy += m[0] * fy; chz += m[0] * fz;
                if (nf == 4) zeta += m[0] * pot[3 * nlive + v];
            }
    cx<T> *o = out + 5 * t;
    o[0] = psi; o[1] = chx; o[2] = chy; o[3] = chz; o[4] = zeta;
}

template <typename T>
void launch_interp(const GridView &g, const T *mom, const cx<T> *pot, int nfields, int nrhs, cx<T> *tripot,
                   hipStream_t st) {
    const int64_t ntg = g.ntg;
    if (!ntg || nrhs < 1) return;
    SIE_CHECK(nrhs <= 65535, SIE_EINVAL, "too many right-hand sides");
    auto run = [&](int c) {
        const int bs = kStageBlocks[c];
        hipLaunchKernelGGL(k_interp<T>, dim3((unsigned)((ntg + bs - 1) / bs), (unsigned)nrhs), dim3(bs), 0, st, ntg,
                           g.centre, g.tri_slot, g.lo[0], g.lo[1], g.lo[2], g.nl[0], g.nl[1], g.nlive, g.nnodes(),
                           mom, pot, nfields, tripot, nrhs == 1 ? g.active : nullptr, g.obj0);
        SIE_HIP(hipGetLastError());
        return true;
    };
    int dev = 0;
    SIE_HIP(hipGetDevice(&dev));
    const TuneKey key{dev, TUNE_INTERP, (int)sizeof(T), {ntg, g.nnodes(), nfields, nrhs, 0}};
    run(tune_pick(key, kNumStageBlocks, run, st));
}

template <typename T>
__device__ inline cx<T> wave_sum(cx<T> v) {
    for (int off = 32; off > 0; off >>= 1) {
        v.re += __shfl_xor(v.re, off, 64);
        v.im += __shfl_xor(v.im, off, 64);
    }
    return v;
}

// One wavefront per row.  Far part of row n from its two triangles:
// c_e (psi - q_e . chi) + kscal c_e zeta   (kscal = -2 k^-2 for L, 0 for K).
// Row base (first column) and 16-bit column offsets: one wave per row.
__global__ void k_cols16(int64_t nrow, const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ cols,
                         int32_t *__restrict__ row_base, uint16_t *__restrict__ cols16, int *__restrict__ wide) {
    const int lane = threadIdx.x & 63;
    const int64_t r = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    if (r >= nrow) return;
    const int64_t b = row_ptr[r], e = row_ptr[r + 1];
    const int32_t base = e > b ? cols[b] : 0;
    if (lane == 0) row_base[r] = base;
    if (e > b && cols[e - 1] - base > 65535) {      // columns ascend within a row
        if (lane == 0) atomicMax(wide, 1);
        return;
    }
    for (int64_t j = b + lane; j < e; j += 64) cols16[j] = (uint16_t)(cols[j] - base);
}

void launch_cols16(int64_t nrow, const int64_t *row_ptr, const int32_t *cols, int32_t *row_base, uint16_t *cols16,
                   int *wide, hipStream_t st) {
    if (nrow <= 0) return;
    hipLaunchKernelGGL(k_cols16, dim3((unsigned)((nrow + 3) / 4)), dim3(256), 0, st, nrow, row_ptr, cols, row_base,
                       cols16, wide);
    SIE_HIP(hipGetLastError());
}

// Rows rwg0 + r, r < nrow (the rows of the view; others are not touched).
// The far part's scalar weight kscal (-2 k^-2 for L, none for K) and the
// optional factor alpha on the row's result are taken per slot, the slot
// being that of the row's triangles.  Lanes 0 and 1 load the far-part
// operands of the row's two triangles before the near-field loop, so that
// those loads overlap it, and their contributions join the lane sum.
typedef float spmv_f4 __attribute__((ext_vector_type(4)));
typedef int spmv_i2 __attribute__((ext_vector_type(2)));

// Two consecutive FP32 nonzeros from position j (even, counted from arrays
// whose starts are aligned): both values in one 16-byte load and both column
// indices in one 4-byte (16-bit offsets) or 8-byte load, so that the lanes of
// a wave read one contiguous stretch per load; streamed once (non-temporal).
template <bool C16>
__device__ inline void load2(const c64 *__restrict__ vals, const int32_t *__restrict__ cols,
                             const uint16_t *__restrict__ cols16, int32_t base, int64_t j, c64 v[2], int32_t c[2]) {
    if constexpr (C16) {
        const unsigned w = __builtin_nontemporal_load(reinterpret_cast<const unsigned *>(cols16 + j));
        c[0] = base + (int32_t)(w & 0xffffu);
        c[1] = base + (int32_t)(w >> 16);
    } else {
        const spmv_i2 w = __builtin_nontemporal_load(reinterpret_cast<const spmv_i2 *>(cols + j));
        c[0] = w.x;
        c[1] = w.y;
    }
    const spmv_f4 a = __builtin_nontemporal_load(reinterpret_cast<const spmv_f4 *>(vals + j));
    v[0] = c64(a.x, a.y);
    v[1] = c64(a.z, a.w);
}

template <typename T, bool C16, bool VEC>
__global__ void k_spmv_far(int64_t nrow, int64_t rwg0, const int64_t *__restrict__ row_ptr,
                           const int32_t *__restrict__ cols, const uint16_t *__restrict__ cols16,
                           const int32_t *__restrict__ row_base, const cx<T> *__restrict__ vals,
                           const int32_t *__restrict__ rwg_loc, const T *__restrict__ coef,
                           const cx<T> *__restrict__ tripot, const int32_t *__restrict__ tri_slot,
                           const cx<T> *__restrict__ kscal, const cx<T> *__restrict__ alpha,
                           const cx<T> *__restrict__ x, cx<T> *__restrict__ y, int use_far,
                           const uint8_t *__restrict__ active, int obj0) {
    const int lane = threadIdx.x & 63;
    const int64_t r = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    if (r >= nrow) return;
    const int64_t row = rwg0 + r;
    if (active) {   // a row of an inactive slot is zero (uniform over the wavefront)
        const int slot = tri_slot ? tri_slot[rwg_loc[2 * r] >> 2] : 0;
        if (!active[obj0 + slot]) {
            if (lane == 0) y[row] = cx<T>();
            return;
        }
    }
    cx<T> acc;
    cx<T> al(T(1));
    if (lane < 2 && (use_far || alpha)) {
        const int32_t lc = rwg_loc[2 * r + lane];
        const int64_t t = lc >> 2;
        const int slot = tri_slot ? tri_slot[t] : 0;
        if (use_far) {
            const int ed = lc & 3;
            const T *c = coef + (t * 3 + ed) * 4;
            const cx<T> *p = tripot + 5 * t;
            const cx<T> ks = kscal ? kscal[slot] : cx<T>();
            cx<T> v = p[0] - (c[1] * p[1] + c[2] * p[2] + c[3] * p[3]);
            v += ks * p[4];
            acc = c[0] * v;
        }
        if (alpha) al = alpha[slot];
    }
    if (vals) {
        const int64_t b = row_ptr[r], e = row_ptr[r + 1];
        // four independent gathers in flight per lane; values and column
        // indices are streamed once (non-temporal), x stays cache-resident;
        // C16: columns as 16-bit offsets from the row's first column
        const int32_t base = C16 ? row_base[r] : 0;
        auto col = [&](int64_t jj) -> int32_t {
            if constexpr (C16) return base + (int32_t)__builtin_nontemporal_load(cols16 + jj);
            else return __builtin_nontemporal_load(cols + jj);
        };
        cx<T> a1, a2, a3;
        if constexpr (VEC && sizeof(T) == 4) {
            // VEC (FP32, aligned array starts): lane l takes the pair of
            // nonzeros 2 l, 2 l + 1 of each stretch of 128; an odd first or
            // last nonzero is taken alone
            const int64_t jb = min(e, (b + 1) & ~(int64_t)1);
            const int64_t je = max(jb, e & ~(int64_t)1);
            if (lane == 0 && b < jb) acc += vals[b] * x[col(b)];
            if (lane == 1 && je < e) a1 += vals[je] * x[col(je)];
            int64_t j = jb + 2 * lane;
            for (; j + 128 < je; j += 256) {
                c64 v[4];
                int32_t c[4];
                load2<C16>(reinterpret_cast<const c64 *>(vals), cols, cols16, base, j, v, c);
                load2<C16>(reinterpret_cast<const c64 *>(vals), cols, cols16, base, j + 128, v + 2, c + 2);
                acc += v[0] * x[c[0]];
                a1 += v[1] * x[c[1]];
                a2 += v[2] * x[c[2]];
                a3 += v[3] * x[c[3]];
            }
            if (j < je) {
                c64 v[2];
                int32_t c[2];
                load2<C16>(reinterpret_cast<const c64 *>(vals), cols, cols16, base, j, v, c);
                acc += v[0] * x[c[0]];
                a1 += v[1] * x[c[1]];
            }
        } else {
        int64_t j = b + lane;
        for (; j + 192 < e; j += 256) {
            const int32_t c0 = col(j);
            const int32_t c1 = col(j + 64);
            const int32_t c2 = col(j + 128);
            const int32_t c3 = col(j + 192);
            const T *vp = reinterpret_cast<const T *>(vals + j);
            const cx<T> v0(__builtin_nontemporal_load(vp), __builtin_nontemporal_load(vp + 1));
            const cx<T> v1(__builtin_nontemporal_load(vp + 128), __builtin_nontemporal_load(vp + 129));
            const cx<T> v2(__builtin_nontemporal_load(vp + 256), __builtin_nontemporal_load(vp + 257));
            const cx<T> v3(__builtin_nontemporal_load(vp + 384), __builtin_nontemporal_load(vp + 385));
            acc += v0 * x[c0];
            a1 += v1 * x[c1];
            a2 += v2 * x[c2];
            a3 += v3 * x[c3];
        }
        for (; j < e; j += 64) acc += vals[j] * x[col(j)];
        }
        acc += (a1 + a2) + a3;
    }
    acc = wave_sum(acc);
    if (lane == 0) y[row] = alpha ? al * acc : acc;
}

template <typename T>
void launch_spmv_far(const GridView &g, const T *tri_coef, const cx<T> *tripot, const cx<T> *kscal,
                     const cx<T> *alpha, const cx<T> *vals, const cx<T> *x, cx<T> *y, bool use_far, hipStream_t st) {
    const int64_t nrow = g.nrow();
    if (nrow <= 0) return;
    const int rows_per_block = 4;
    const dim3 grid((unsigned)((nrow + rows_per_block - 1) / rows_per_block));
    // paired loads: FP32 values, value and index arrays that start aligned
    // (a medium's values viewed inside a group's array may not)
    const bool vec = sizeof(T) == 4 && ((uintptr_t)vals % 16 == 0) &&
                     (g.c16 ? (uintptr_t)g.cols16 % 4 == 0 : (uintptr_t)g.cols % 8 == 0);
#define SIE_SPMV(C, V)                                                                                              \
    hipLaunchKernelGGL((k_spmv_far<T, C, V>), grid, dim3(256), 0, st, nrow, g.rwg0, g.row_ptr, g.cols, g.cols16,     \
                       g.row_base, vals, g.rwgloc, tri_coef, tripot, g.tri_slot, kscal, alpha, x, y, use_far ? 1 : 0, \
                       g.active, g.obj0)
    if constexpr (sizeof(T) == 4) {
        if (g.c16) {
            if (vec) SIE_SPMV(true, true);
            else SIE_SPMV(true, false);
        } else {
            if (vec) SIE_SPMV(false, true);
            else SIE_SPMV(false, false);
        }
    } else {
        (void)vec;
        if (g.c16) SIE_SPMV(true, false);
        else SIE_SPMV(false, false);
    }
#undef SIE_SPMV
    SIE_HIP(hipGetLastError());
}

// Right-hand-side transpose x [nrhs][E] -> xt [E][nrhs] through a 32 x 32
// LDS tile, so that the batched near-field product reads the nrhs values of
// one column as one contiguous row.
template <typename T>
__global__ void k_rhs_transpose(int64_t E, int nrhs, const cx<T> *__restrict__ x, cx<T> *__restrict__ xt) {
    __shared__ T tre[32][33], tim[32][33];
    const int64_t e0 = blockIdx.x * 32LL;
    const int r0 = blockIdx.y * 32;
    for (int i = threadIdx.y; i < 32; i += 8) {
        const int r = r0 + i;
        const int64_t e = e0 + threadIdx.x;
        if (r < nrhs && e < E) {
            const cx<T> v = x[r * E + e];
            tre[i][threadIdx.x] = v.re;
            tim[i][threadIdx.x] = v.im;
        }
    }
    __syncthreads();
    for (int i = threadIdx.y; i < 32; i += 8) {
        const int64_t e = e0 + i;
        const int r = r0 + threadIdx.x;
        if (r < nrhs && e < E) xt[e * nrhs + r] = cx<T>(tre[threadIdx.x][i], tim[threadIdx.x][i]);
    }
}

// Batched near-field product plus far part for nrhs right-hand sides:
// y[r][row] = sum_j N[row][j] xt[j][r] + c_e (psi - q_e . chi) + kscal c_e zeta
// (tripot of right-hand side r).  One 64-lane block per row; the lanes are
// SLOTS = 64 / RPW groups of RPW (a power of two >= nrhs of the slice, at
// most 64) lanes: group s takes the row's nonzeros s, s + SLOTS, ... and
// lane q of the group right-hand side q, so every lane is busy whatever
// nrhs is; the groups are summed with lane shuffles at the end.  The x
// values of one column are one contiguous row of xt.
template <typename T, int RPW, bool C16>
__global__ void __launch_bounds__(64) k_spmm_far(int64_t E, int64_t rwg0, int nrhs,
                                                 const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ cols,
                                                 const uint16_t *__restrict__ cols16,
                                                 const int32_t *__restrict__ row_base,
                                                 const cx<T> *__restrict__ vals, const int32_t *__restrict__ rwg_loc,
                                                 const T *__restrict__ coef, const cx<T> *__restrict__ tripot,
                                                 int64_t ntg, const int32_t *__restrict__ tri_slot,
                                                 const cx<T> *__restrict__ kscal, const cx<T> *__restrict__ alpha,
                                                 const cx<T> *__restrict__ xt, cx<T> *__restrict__ y) {
    constexpr int SLOTS = 64 / RPW;
    const int64_t rr = blockIdx.x;         // row rwg0 + rr of the view
    const int64_t row = rwg0 + rr;
    const int slot = threadIdx.x / RPW, q = threadIdx.x % RPW;
    const int r = blockIdx.y * RPW + q;
    const bool act = r < nrhs;
    // the far part of right-hand side r and the row's factor, loaded by the
    // lanes of group 0 before the near loop (their sums join the reduction)
    cx<T> acc;
    cx<T> al(T(1));
    if (act && slot == 0) {
        const int sl = tri_slot ? tri_slot[rwg_loc[2 * rr] >> 2] : 0;
        if (tripot) {
            const cx<T> ks = kscal ? kscal[sl] : cx<T>();
            const cx<T> *tp = tripot + (int64_t)r * 5 * ntg;
            for (int s2 = 0; s2 < 2; ++s2) {
                const int32_t lc = rwg_loc[2 * rr + s2];
                const int64_t t = lc >> 2;
                const int ed = lc & 3;
                const T *c = coef + (t * 3 + ed) * 4;
                const cx<T> *qq = tp + 5 * t;
                cx<T> v = qq[0] - (c[1] * qq[1] + c[2] * qq[2] + c[3] * qq[3]);
                v += ks * qq[4];
                acc += c[0] * v;
            }
        }
        if (alpha) al = alpha[sl];
    }
    if (vals) {
        const int64_t b = row_ptr[rr], e = row_ptr[rr + 1];
        const cx<T> *xr = xt + (act ? r : 0);
        const int32_t base = C16 ? row_base[rr] : 0;
        auto col = [&](int64_t jj) -> int32_t {
            if constexpr (C16) return base + (int32_t)cols16[jj];
            else return cols[jj];
        };
        cx<T> a1, a2, a3;
        int64_t j = b + slot;
        for (; j + 3 * SLOTS < e; j += 4 * SLOTS) {
            const int32_t c0 = col(j), c1 = col(j + SLOTS), c2 = col(j + 2 * SLOTS), c3 = col(j + 3 * SLOTS);
            const cx<T> v0 = vals[j], v1 = vals[j + SLOTS], v2 = vals[j + 2 * SLOTS], v3 = vals[j + 3 * SLOTS];
            acc += v0 * xr[(int64_t)c0 * nrhs];
            a1 += v1 * xr[(int64_t)c1 * nrhs];
            a2 += v2 * xr[(int64_t)c2 * nrhs];
            a3 += v3 * xr[(int64_t)c3 * nrhs];
        }
        for (; j < e; j += SLOTS) acc += vals[j] * xr[(int64_t)col(j) * nrhs];
        acc += (a1 + a2) + a3;
        for (int off = RPW; off < 64; off <<= 1) {
            acc.re += __shfl_xor(acc.re, off, 64);
            acc.im += __shfl_xor(acc.im, off, 64);
        }
    }
    if (!act || slot != 0) return;
    y[r * E + row] = alpha ? al * acc : acc;
}

// xt: scratch of E * nrhs values; x, y: [nrhs][E]; rows of the view only.
template <typename T>
void launch_spmm_far(const GridView &g, int64_t E, int nrhs, const T *tri_coef, const cx<T> *tripot,
                     const cx<T> *kscal, const cx<T> *alpha, const cx<T> *vals, const cx<T> *x, cx<T> *xt, cx<T> *y,
                     hipStream_t st) {
    if (E == 0 || nrhs < 1 || g.nrow() <= 0) return;
    SIE_CHECK(nrhs <= 65535 * 64, SIE_EINVAL, "too many right-hand sides");
    SIE_CHECK(E <= 0x7fffffffLL, SIE_EINVAL, "too many RWG functions for one launch");
    if (vals) {
        hipLaunchKernelGGL(k_rhs_transpose<T>, dim3((unsigned)((E + 31) / 32), (unsigned)((nrhs + 31) / 32)),
                           dim3(32, 8), 0, st, E, nrhs, x, xt);
        SIE_HIP(hipGetLastError());
    }
    int rpw = 1;
    while (rpw < nrhs && rpw < 64) rpw *= 2;
    const dim3 grid((unsigned)g.nrow(), (unsigned)((nrhs + rpw - 1) / rpw));
    const int64_t ntg = g.ntg;
#define SIE_SPMM(R)                                                                                              \
    if (g.c16)                                                                                                   \
        hipLaunchKernelGGL((k_spmm_far<T, R, true>), grid, dim3(64), 0, st, E, g.rwg0, nrhs, g.row_ptr, g.cols,  \
                           g.cols16, g.row_base, vals, g.rwgloc, tri_coef, tripot, ntg, g.tri_slot, kscal, alpha,\
                           xt, y);                                                                               \
    else                                                                                                         \
        hipLaunchKernelGGL((k_spmm_far<T, R, false>), grid, dim3(64), 0, st, E, g.rwg0, nrhs, g.row_ptr, g.cols, \
                           g.cols16, g.row_base, vals, g.rwgloc, tri_coef, tripot, ntg, g.tri_slot, kscal, alpha,\
                           xt, y)
    switch (rpw) {
    case 1: SIE_SPMM(1); break;
    case 2: SIE_SPMM(2); break;
    case 4: SIE_SPMM(4); break;
    case 8: SIE_SPMM(8); break;
    case 16: SIE_SPMM(16); break;
    case 32: SIE_SPMM(32); break;
    default: SIE_SPMM(64); break;
    }
#undef SIE_SPMM
    SIE_HIP(hipGetLastError());
}

// y = X x for the sparse X (real values, <= 5 per row, CSR int32).
template <typename T>
__global__ void k_x_apply(int64_t E, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                          const T *__restrict__ val, const cx<T> *__restrict__ x, cx<T> *__restrict__ y) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= E) return;
    cx<T> acc;
    for (int j = ptr[r]; j < ptr[r + 1]; ++j) acc += val[j] * x[col[j]];
    y[r] = acc;
}

template <typename T>
void launch_x_apply(int64_t E, const int32_t *xptr, const int32_t *xcol, const T *xval, const cx<T> *x, cx<T> *y,
                    hipStream_t st) {
    if (E == 0) return;
    hipLaunchKernelGGL(k_x_apply<T>, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, st, E, xptr, xcol, xval, x, y);
    SIE_HIP(hipGetLastError());
}

#define SIE_INST(T)                                                                                           \
    template void launch_tri_sources<T>(const GridView &, const T *, const cx<T> *, int64_t, int, cx<T> *,      \
                                        hipStream_t);                                                          \
    template void launch_project<T>(const GridView &, const T *, const cx<T> *, cx<T> *, int, int, hipStream_t, \
                                    const cx<T> *, int64_t, const int32_t *);                                    \
    template void launch_interp<T>(const GridView &, const T *, const cx<T> *, int, int, cx<T> *, hipStream_t); \
    template void launch_spmm_far<T>(const GridView &, int64_t, int, const T *, const cx<T> *, const cx<T> *,   \
                                     const cx<T> *, const cx<T> *, const cx<T> *, cx<T> *, cx<T> *, hipStream_t); \
    template void launch_spmv_far<T>(const GridView &, const T *, const cx<T> *, const cx<T> *, const cx<T> *,  \
                                     const cx<T> *, const cx<T> *, cx<T> *, bool, hipStream_t);                 \
    template void launch_x_apply<T>(int64_t, const int32_t *, const int32_t *, const T *, const cx<T> *, cx<T> *, \
                                    hipStream_t);
SIE_INST(float)
SIE_INST(double)

}  // namespace sie
