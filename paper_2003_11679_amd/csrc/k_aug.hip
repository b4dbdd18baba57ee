// Kernels of the augmented EFIE (Sec. III-E, eq. sys): the near part of the
// pulse-charge potential, the weighted continuity rows, and the two sides of
// the constraint preconditioner around its Schur-complement solve.
//
// Notation (per triangle t with local edges e and RWG functions n_e):
//   sl[t][e] = +-l of RWG n_e on t (sign + on T+), so div f_n = sl / A_t;
//   continuity row t, weighted by A_t / k0: sum_e sl[t][e] u[n_e] / k0 + j A_t sigma_t.
#include "common.h"
#include "kernels.h"

namespace sie {

__device__ inline c128 wsum64(c128 v) {
    for (int off = 32; off > 0; off >>= 1) {
        v.re += __shfl_xor(v.re, off, 64);
        v.im += __shfl_xor(v.im, off, 64);
    }
    return v;
}

// zeta slot of the interpolation partials: tripot[r][t][4] += sum over the
// near pairs (t, s) of gam[p] rho[r][tris[s]] (precorrected pulse integrals;
// t, s the grid's own triangle order, rho in the global numbering).  One
// wavefront per triangle.
__global__ void k_tri_near(int64_t ntg, const int64_t *__restrict__ pair_ptr, const int32_t *__restrict__ pair_s,
                           const int32_t *__restrict__ tris, const c128 *__restrict__ gam,
                           const c128 *__restrict__ rho, int64_t ldr, c128 *__restrict__ tripot) {
    const int lane = threadIdx.x & 63;
    const int64_t t = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    if (t >= ntg) return;
    rho += blockIdx.y * ldr;
    tripot += blockIdx.y * 5 * ntg;
    c128 acc;
    for (int64_t p = pair_ptr[t] + lane; p < pair_ptr[t + 1]; p += 64) acc += gam[p] * rho[tris[pair_s[p]]];
    acc = wsum64(acc);
    if (lane == 0) tripot[5 * t + 4] += acc;
}

void launch_tri_near(int64_t ntg, const int64_t *pair_ptr, const int32_t *pair_s, const int32_t *tris,
                     const c128 *gam, const c128 *rho, int64_t ldr, int nrhs, c128 *tripot, hipStream_t st) {
    if (ntg <= 0 || nrhs < 1) return;
    SIE_CHECK(nrhs <= 65535, SIE_EINVAL, "too many right-hand sides");
    hipLaunchKernelGGL(k_tri_near, dim3((unsigned)((ntg + 3) / 4), (unsigned)nrhs), dim3(256), 0, st, ntg, pair_ptr,
                       pair_s, tris, gam, rho, ldr, tripot);
    SIE_HIP(hipGetLastError());
}

// y[r][t] = sum_e sl[t][e] u[r][n_e] / k0 + j A_t sigma[r][t]
__global__ void k_continuity(int64_t nt, const int32_t *__restrict__ tri_rwg, const double *__restrict__ sl,
                             const double *__restrict__ area, double k0, const c128 *__restrict__ u, int64_t ldu,
                             const c128 *__restrict__ sg, int64_t lds, c128 *__restrict__ y, int64_t ldy) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nt) return;
    u += blockIdx.y * ldu;
    sg += blockIdx.y * lds;
    y += blockIdx.y * ldy;
    c128 acc;
    for (int e = 0; e < 3; ++e) acc += sl[3 * t + e] * u[tri_rwg[3 * t + e]];
    const c128 s = sg[t];
    y[t] = c128(acc.re / k0 - area[t] * s.im, acc.im / k0 + area[t] * s.re);
}

void launch_continuity(int64_t nt, const int32_t *tri_rwg, const double *sl, const double *area, double k0,
                       const c128 *u, int64_t ldu, const c128 *sg, int64_t lds, c128 *y, int64_t ldy, int nrhs,
                       hipStream_t st) {
    if (nt <= 0 || nrhs < 1) return;
    SIE_CHECK(nrhs <= 65535, SIE_EINVAL, "too many right-hand sides");
    hipLaunchKernelGGL(k_continuity, dim3((unsigned)((nt + 255) / 256), (unsigned)nrhs), dim3(256), 0, st, nt,
                       tri_rwg, sl, area, k0, u, ldu, sg, lds, y, ldy);
    SIE_HIP(hipGetLastError());
}

// Constraint preconditioner, before the Schur solve: with r = [r1 (E); r2 (T)]
// (stride ldr), b_t = (k0 r2_t - sum_e sl[t][e] r1[n_e] / ad[n_e]) / A_t, the
// right-hand side r2 / W - Dv ad^-1 r1 of S, stored at position iperm[t].
__global__ void k_cp_pre(int64_t nt, const int32_t *__restrict__ tri_rwg, const double *__restrict__ sl,
                         const double *__restrict__ area, double k0, const c128 *__restrict__ ad,
                         const int32_t *__restrict__ iperm, const c128 *__restrict__ r, int64_t ldr, int64_t E,
                         c128 *__restrict__ xnd) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nt) return;
    r += blockIdx.y * ldr;
    xnd += blockIdx.y * nt;
    c128 acc = k0 * r[E + t];
    for (int e = 0; e < 3; ++e) {
        const int32_t n = tri_rwg[3 * t + e];
        acc -= sl[3 * t + e] * cdiv(r[n], ad[n]);
    }
    xnd[iperm[t]] = (1.0 / area[t]) * acc;
}

// After the Schur solve (ys_t at position iperm[t]):
// y_u[n] = (r1[n] + sum_{t = T+, T-} sl[t][e] gself[t] ys_t / A_t) / ad[n],
// y_s[t] = ys_t.
__global__ void k_cp_post(int64_t E, int64_t nt, const int32_t *__restrict__ tpm, const int32_t *__restrict__ epm,
                          const double *__restrict__ sl, const double *__restrict__ area,
                          const c128 *__restrict__ gself, const c128 *__restrict__ ad,
                          const int32_t *__restrict__ iperm, const c128 *__restrict__ xnd,
                          const c128 *__restrict__ r, int64_t ldr, c128 *__restrict__ y, int64_t ldy) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= E + nt) return;
    r += blockIdx.y * ldr;
    y += blockIdx.y * ldy;
    xnd += blockIdx.y * nt;
    if (i < E) {
        c128 acc = r[i];
        for (int s = 0; s < 2; ++s) {
            const int32_t t = tpm[2 * i + s], e = epm[2 * i + s];
            acc += (sl[3 * (int64_t)t + e] / area[t]) * (gself[t] * xnd[iperm[t]]);
        }
        y[i] = cdiv(acc, ad[i]);
    } else {
        const int64_t t = i - E;
        y[i] = xnd[iperm[t]];
    }
}

void launch_cp_pre(int64_t nt, const int32_t *tri_rwg, const double *sl, const double *area, double k0, const c128 *ad,
                   const int32_t *iperm, const c128 *r, int64_t ldr, int64_t E, c128 *xnd, int nrhs, hipStream_t st) {
    if (nt <= 0 || nrhs < 1) return;
    SIE_CHECK(nrhs <= 65535, SIE_EINVAL, "too many right-hand sides");
    hipLaunchKernelGGL(k_cp_pre, dim3((unsigned)((nt + 255) / 256), (unsigned)nrhs), dim3(256), 0, st, nt, tri_rwg, sl,
                       area, k0, ad, iperm, r, ldr, E, xnd);
    SIE_HIP(hipGetLastError());
}

void launch_cp_post(int64_t E, int64_t nt, const int32_t *tpm, const int32_t *epm, const double *sl, const double *area,
                    const c128 *gself, const c128 *ad, const int32_t *iperm, const c128 *xnd, const c128 *r,
                    int64_t ldr, c128 *y, int64_t ldy, int nrhs, hipStream_t st) {
    if (E + nt <= 0 || nrhs < 1) return;
    SIE_CHECK(nrhs <= 65535, SIE_EINVAL, "too many right-hand sides");
    hipLaunchKernelGGL(k_cp_post, dim3((unsigned)((E + nt + 255) / 256), (unsigned)nrhs), dim3(256), 0, st, E, nt, tpm,
                       epm, sl, area, gself, ad, iperm, xnd, r, ldr, y, ldy);
    SIE_HIP(hipGetLastError());
}

}  // namespace sie
