// Kernels of the solve: plane-wave excitation, far field, and the batched
// block-Jacobi stand-in for the near-region preconditioner M_i = -j w eps_i L_i,NR
// (eq. nest2pc; the paper factorises M_i with a sparse LU, here diagonal
// blocks of spatially adjacent RWG functions are inverted in FP64).
#include "problem.h"
#include "solve_kernels.h"

namespace sie {

// e_m = int f_m . e0 exp(-j k0 khat . r) dS over the two triangles of m.
__global__ void k_excitation(int64_t E, const double *__restrict__ xyz, const int32_t *__restrict__ tri,
                             const int32_t *__restrict__ tpm, const int32_t *__restrict__ epm,
                             const double *__restrict__ len, const double *__restrict__ area,
                             const double *__restrict__ rule, int nq, double k0, double kx, double ky, double kz,
                             c128 ex, c128 ey, c128 ez, c128 *__restrict__ out) {
    int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= E) return;
    c128 acc;
    for (int s = 0; s < 2; ++s) {
        const int64_t t = tpm[2 * n + s];
        const int e = epm[2 * n + s];
        const double sg = s == 0 ? 1.0 : -1.0;
        const double A = area[t];
        const double c = sg * len[n] / (2.0 * A);
        double v[3][3];
        for (int k = 0; k < 3; ++k)
            for (int d = 0; d < 3; ++d) v[k][d] = xyz[3 * (int64_t)tri[3 * t + k] + d];
        for (int q = 0; q < nq; ++q) {
            double r[3];
            for (int d = 0; d < 3; ++d)
                r[d] = rule[4 * q] * v[0][d] + rule[4 * q + 1] * v[1][d] + rule[4 * q + 2] * v[2][d];
            const double ph = -k0 * (kx * r[0] + ky * r[1] + kz * r[2]);
            double sn, cs;
            sincos(ph, &sn, &cs);
            const c128 phase(cs, sn);
            const double w = rule[4 * q + 3] * A * c;
            const c128 fd = (r[0] - v[e][0]) * ex + (r[1] - v[e][1]) * ey + (r[2] - v[e][2]) * ez;
            acc += w * (fd * phase);
        }
    }
    out[n] = acc;
}

void launch_excitation(sie_problem *p, const double *rule, int nq, double k0, const double khat[3], const c128 e0[3],
                       c128 *out, hipStream_t st) {
    const int64_t E = p->mesh.nrwg;
    hipLaunchKernelGGL(k_excitation, dim3((unsigned)((E + 127) / 128)), dim3(128), 0, st, E, p->d_xyz.p, p->d_tri.p,
                       p->d_tpm.p, p->d_epm.p, p->d_len.p, p->d_area.p, rule, nq, k0, khat[0], khat[1], khat[2],
                       e0[0], e0[1], e0[2], out);
    SIE_HIP(hipGetLastError());
}

// Far-field amplitude for direction d (one block per direction):
// F = (-j k0 / 4 pi) [eta0 (N_u - rhat (rhat . N_u)) + rhat x N_v],
// N_x = int x(r') exp(j k0 rhat . r') dS'.
__global__ void k_farfield(int64_t T, const double *__restrict__ xyz, const int32_t *__restrict__ tri,
                           const int32_t *__restrict__ tri_rwg, const double *__restrict__ tri_sign,
                           const double *__restrict__ len, const double *__restrict__ area,
                           const double *__restrict__ rule, int nq, double k0, double eta0,
                           const double *__restrict__ rhat, const c128 *__restrict__ u, const c128 *__restrict__ v,
                           c128 *__restrict__ F) {
    __shared__ double red[12][256];
    const int d = blockIdx.x;
    const double rx = rhat[3 * d], ry = rhat[3 * d + 1], rz = rhat[3 * d + 2];
    c128 nu[3], nv[3];
    for (int64_t t = threadIdx.x; t < T; t += blockDim.x) {
        double vt[3][3];
        for (int k = 0; k < 3; ++k)
            for (int c = 0; c < 3; ++c) vt[k][c] = xyz[3 * (int64_t)tri[3 * t + k] + c];
        c128 cu[3], cv[3];
        double ce[3];
        for (int e = 0; e < 3; ++e) {
            const int n = tri_rwg[3 * t + e];
            ce[e] = tri_sign[3 * t + e] * len[n] / (2.0 * area[t]);
            cu[e] = u[n]; cv[e] = v[n];
        }
        for (int q = 0; q < nq; ++q) {
            double r[3];
            for (int c = 0; c < 3; ++c)
                r[c] = rule[4 * q] * vt[0][c] + rule[4 * q + 1] * vt[1][c] + rule[4 * q + 2] * vt[2][c];
            double sn, cs;
            sincos(k0 * (rx * r[0] + ry * r[1] + rz * r[2]), &sn, &cs);
            const c128 ph = (rule[4 * q + 3] * area[t]) * c128(cs, sn);
            for (int c = 0; c < 3; ++c) {
                c128 ju, jv;
                for (int e = 0; e < 3; ++e) {
                    const double f = ce[e] * (r[c] - vt[e][c]);
                    ju += f * cu[e];
                    jv += f * cv[e];
                }
                nu[c] += ph * ju;
                nv[c] += ph * jv;
            }
        }
    }
    for (int c = 0; c < 3; ++c) {
        red[2 * c][threadIdx.x] = nu[c].re; red[2 * c + 1][threadIdx.x] = nu[c].im;
        red[6 + 2 * c][threadIdx.x] = nv[c].re; red[7 + 2 * c][threadIdx.x] = nv[c].im;
    }
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 12; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        c128 Nu[3], Nv[3];
        for (int c = 0; c < 3; ++c) {
            Nu[c] = c128(red[2 * c][0], red[2 * c + 1][0]);
            Nv[c] = c128(red[6 + 2 * c][0], red[7 + 2 * c][0]);
        }
        const double rh[3] = {rx, ry, rz};
        const c128 rdot = rx * Nu[0] + ry * Nu[1] + rz * Nu[2];
        const c128 cr[3] = {ry * Nv[2] - rz * Nv[1], rz * Nv[0] - rx * Nv[2], rx * Nv[1] - ry * Nv[0]};
        const c128 pre(0.0, -k0 / (4.0 * 3.14159265358979323846));
        for (int c = 0; c < 3; ++c) F[3 * d + c] = pre * (eta0 * (Nu[c] - rh[c] * rdot) + cr[c]);
    }
}

void launch_farfield(sie_problem *p, const double *rule, int nq, double k0, double eta0, const double *rhat,
                     int64_t ndir, const c128 *u, const c128 *v, c128 *F, hipStream_t st) {
    if (ndir == 0) return;
    hipLaunchKernelGGL(k_farfield, dim3((unsigned)ndir), dim3(256), 0, st, p->mesh.nt(), p->d_xyz.p, p->d_tri.p,
                       p->d_tri_rwg.p, p->d_tri_sign.p, p->d_len.p, p->d_area.p, rule, nq, k0, eta0, rhat, u, v, F);
    SIE_HIP(hipGetLastError());
}

// ---------------------------------------------------------------- block Jacobi
// One workgroup per block of B RWG functions (perm: [nb][B], -1 = padding):
// gather the scaled direct near-region entries, invert by Gauss-Jordan with
// partial pivoting in LDS (FP64), store the inverse.
__global__ void k_bj_setup(int B, const int32_t *__restrict__ perm, int64_t rwg0, const int64_t *__restrict__ row_ptr,
                           const int32_t *__restrict__ cols, const c128 *__restrict__ vals, c128 scale,
                           c128 *__restrict__ inv64, c64 *__restrict__ inv32) {
    extern __shared__ unsigned char smem[];
    c128 *a = reinterpret_cast<c128 *>(smem);          // [B][2B]
    c128 *fcol = a + 2 * B * B;                         // [B]
    __shared__ int piv;
    const int b = blockIdx.x;
    const int W = 2 * B;
    const int32_t *pb = perm + (int64_t)b * B;
    for (int it = threadIdx.x; it < B * B; it += blockDim.x) {
        const int i = it / B, j = it - i * B;
        const int32_t r = pb[i], c = pb[j];
        c128 val;
        if (r < 0 || c < 0) {
            val = c128(i == j ? 1.0 : 0.0);
        } else {
            int64_t lo = row_ptr[r - rwg0], hi = row_ptr[r - rwg0 + 1];
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                const int32_t cm = cols[mid];
                if (cm == c) { val = scale * vals[mid]; break; }
                if (cm < c) lo = mid + 1; else hi = mid;
            }
        }
        a[i * W + j] = val;
        a[i * W + B + j] = c128(i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int k = 0; k < B; ++k) {
        if (threadIdx.x == 0) {
            int best = k;
            double bv = norm2(a[k * W + k]);
            for (int i = k + 1; i < B; ++i) {
                const double v = norm2(a[i * W + k]);
                if (v > bv) { bv = v; best = i; }
            }
            piv = best;
        }
        __syncthreads();
        const int pr = piv;
        if (pr != k)
            for (int j = threadIdx.x; j < W; j += blockDim.x) {
                const c128 t = a[k * W + j];
                a[k * W + j] = a[pr * W + j];
                a[pr * W + j] = t;
            }
        __syncthreads();
        const c128 pinv = cdiv(c128(1.0), a[k * W + k]);
        __syncthreads();
        for (int j = threadIdx.x; j < W; j += blockDim.x) a[k * W + j] = pinv * a[k * W + j];
        __syncthreads();
        for (int i = threadIdx.x; i < B; i += blockDim.x) fcol[i] = a[i * W + k];
        __syncthreads();
        for (int it = threadIdx.x; it < B * W; it += blockDim.x) {
            const int i = it / W, j = it - i * W;
            if (i != k) a[i * W + j] -= fcol[i] * a[k * W + j];
        }
        __syncthreads();
    }
    for (int it = threadIdx.x; it < B * B; it += blockDim.x) {
        const int i = it / B, j = it - i * B;
        const c128 v = a[i * W + B + j];
        inv64[(int64_t)b * B * B + it] = v;
        inv32[(int64_t)b * B * B + it] = c64((float)v.re, (float)v.im);
    }
}

void launch_bj_setup(int nb, int B, const int32_t *perm, int64_t rwg0, const int64_t *row_ptr, const int32_t *cols,
                     const c128 *vals, c128 scale, c128 *inv64, c64 *inv32, hipStream_t st) {
    if (!nb) return;
    const size_t sh = (2 * (size_t)B * B + B) * sizeof(c128);
    hipLaunchKernelGGL(k_bj_setup, dim3(nb), dim3(256), sh, st, B, perm, rwg0, row_ptr, cols, vals, scale, inv64,
                       inv32);
    SIE_HIP(hipGetLastError());
}

template <typename T>
__global__ void k_bj_apply(int B, const int32_t *__restrict__ perm, const cx<T> *__restrict__ inv,
                           const cx<T> *__restrict__ x, cx<T> *__restrict__ y) {
    extern __shared__ unsigned char smem[];
    cx<T> *xs = reinterpret_cast<cx<T> *>(smem);
    const int b = blockIdx.x;
    const int32_t *pb = perm + (int64_t)b * B;
    for (int j = threadIdx.x; j < B; j += blockDim.x) xs[j] = pb[j] >= 0 ? x[pb[j]] : cx<T>();
    __syncthreads();
    for (int i = threadIdx.x; i < B; i += blockDim.x) {
        if (pb[i] < 0) continue;
        const cx<T> *row = inv + ((int64_t)b * B + i) * B;
        cx<T> acc;
        for (int j = 0; j < B; ++j) acc += row[j] * xs[j];
        y[pb[i]] = acc;
    }
}

template <typename T>
void launch_bj_apply(int nb, int B, const int32_t *perm, const cx<T> *inv, const cx<T> *x, cx<T> *y, hipStream_t st) {
    if (!nb) return;
    hipLaunchKernelGGL(k_bj_apply<T>, dim3(nb), dim3(64), B * sizeof(cx<T>), st, B, perm, inv, x, y);
    SIE_HIP(hipGetLastError());
}

template void launch_bj_apply<float>(int, int, const int32_t *, const c64 *, const c64 *, c64 *, hipStream_t);
template void launch_bj_apply<double>(int, int, const int32_t *, const c128 *, const c128 *, c128 *, hipStream_t);

}  // namespace sie

namespace sie {

// ---------------------------------------------------------------- Schwarz clusters
// Restricted additive Schwarz form of the near-region preconditioner
// M_i = -j w eps_i L_i,NR (eq. nest2pc): the RWG functions are grouped into
// clusters of grid cells; cluster c owns its RWG functions and extends over
// the cells around it (ext).  M_i restricted to ext x ext is inverted, and the
// rows of the inverse that belong to the owned functions are kept:
//     y[own] = (M_ext^-1)[own, :] x[ext].
// Setup solves M_ext^T Y = E_own (E_own: unit columns at the owned
// positions) by Gauss-Jordan elimination with partial pivoting in FP64; the
// augmented matrix [M_ext^T | E_own] (n x (n + n_own), row-major) lives in a
// global workspace, one workgroup per cluster.

__global__ __launch_bounds__(512) void k_ras_gather(int c0, const int64_t *__restrict__ ext_off,
                                                    const int32_t *__restrict__ ext,
                                                    const int32_t *__restrict__ own_off,
                                                    const int32_t *__restrict__ own_pos,
                                                    const int64_t *__restrict__ ws_off,
                                                    const int32_t *__restrict__ cmed,
                                                    const RasSource *__restrict__ src, c128 *__restrict__ ws) {
    __shared__ int32_t xs[kRasMax];
    const int c = c0 + blockIdx.x;
    const RasSource s = src[cmed[c]];
    const int64_t rwg0 = s.rwg0;
    const int64_t *__restrict__ row_ptr = s.row_ptr;
    const int32_t *__restrict__ cols = s.cols;
    const c128 *__restrict__ vals = s.vals;
    const c128 scale = s.scale;
    const int64_t e0 = ext_off[c];
    const int n = (int)(ext_off[c + 1] - e0);
    const int o0 = own_off[c];
    const int no = own_off[c + 1] - o0;
    const int64_t W = n + no;
    c128 *B = ws + (ws_off[c] - ws_off[c0]);
    for (int i = threadIdx.x; i < n; i += blockDim.x) xs[i] = ext[e0 + i];
    for (int64_t t = threadIdx.x; t < (int64_t)n * W; t += blockDim.x) B[t] = c128();
    __syncthreads();
    for (int q = threadIdx.x; q < no; q += blockDim.x) B[(int64_t)own_pos[o0 + q] * W + n + q] = c128(1.0);
    // row i of M_ext (RWG xs[i]) is column i of B: one wave per row, lanes
    // over its near-field nonzeros, columns located in the sorted ext list
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int i = wv; i < n; i += nw) {
        const int64_t r = (int64_t)xs[i] - rwg0;
        const int64_t lo = row_ptr[r], hi = row_ptr[r + 1];
        for (int64_t t = lo + lane; t < hi; t += 64) {
            const int32_t col = cols[t];
            int a = 0, b = n;
            while (a < b) {
                const int mid = (a + b) >> 1;
                if (xs[mid] < col) a = mid + 1; else b = mid;
            }
            if (a < n && xs[a] == col) B[(int64_t)a * W + i] = scale * vals[t];
        }
    }
}

// Blocked Gauss-Jordan with partial pivoting.  Panels of bw pivot columns
// are factored in LDS: row swaps, the scaled pivot rows and, in place, the
// multiplier of every other row at each step.  Then the thread that owns a
// trailing column brings it up to date in one pass: the swaps in order, the
// bw scaled pivot rows R in registers, every other row minus its multipliers
// times R.  The subtractions per element come in the same order as pivot by
// pivot elimination, but the matrix streams once per panel instead of once
// per pivot.
constexpr int kPanelElems = 8192;   // n x bw complex128 panel: 128 KB of LDS
constexpr int kPanelMax = 16;

__global__ __launch_bounds__(512) void k_ras_invert(int c0, const int64_t *__restrict__ ext_off,
                                                   const int32_t *__restrict__ own_off,
                                                   const int64_t *__restrict__ ws_off,
                                                   const int64_t *__restrict__ m_off, c128 *__restrict__ ws,
                                                   c128 *__restrict__ m64, c64 *__restrict__ m32,
                                                   int *__restrict__ fail) {
    __shared__ __align__(16) double lds[2 * (kPanelElems + kPanelMax)];
    c128 *P = reinterpret_cast<c128 *>(lds);      // [n][bw] panel
    c128 *sinv = P + kPanelElems;                 // [bw] 1 / pivot
    __shared__ int swp[kPanelMax];
    __shared__ double rv[16];
    __shared__ int ri[16];
    const int c = c0 + blockIdx.x;
    const int n = (int)(ext_off[c + 1] - ext_off[c]);
    const int no = own_off[c + 1] - own_off[c];
    const int W = n + no;
    c128 *B = ws + (ws_off[c] - ws_off[c0]);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
    int bwmax = kPanelMax;                  // n <= kRasMax = 2048: width 2 always fits
    while (bwmax > 2 && n * bwmax > kPanelElems) bwmax >>= 1;
    for (int kb = 0; kb < n; kb += bwmax) {
        const int bw = min(bwmax, n - kb);
        for (int t = tid; t < n * bw; t += blockDim.x) {
            const int i = t / bw, jj = t - i * bw;
            P[t] = B[(int64_t)i * W + kb + jj];
        }
        __syncthreads();
        for (int jj = 0; jj < bw; ++jj) {
            const int k = kb + jj;
            // pivot: largest |P[i][jj]|, i >= k (lowest index among equals)
            double best = -1.0;
            int bi = n;
            for (int i = k + tid; i < n; i += blockDim.x) {
                const double v = norm2(P[i * bw + jj]);
                if (v > best) { best = v; bi = i; }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_down(best, off);
                const int oi = __shfl_down(bi, off);
                if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
            }
            if (lane == 0) { rv[wv] = best; ri[wv] = bi; }
            __syncthreads();
            if (tid == 0) {
                double bb = rv[0];
                int pp = ri[0];
                for (int w = 1; w < nw; ++w)
                    if (rv[w] > bb || (rv[w] == bb && ri[w] < pp)) { bb = rv[w]; pp = ri[w]; }
                swp[jj] = pp;
                if (!(bb > 0.0)) *fail = 1;
            }
            __syncthreads();
            const int pr = swp[jj];
            if (pr != k && tid < bw) {   // whole panel rows, multipliers included
                const c128 t = P[k * bw + tid];
                P[k * bw + tid] = P[pr * bw + tid];
                P[pr * bw + tid] = t;
            }
            __syncthreads();
            if (tid == 0) {
                const c128 d = P[k * bw + jj];
                sinv[jj] = norm2(d) > 0.0 ? cdiv(c128(1.0), d) : c128();
            }
            __syncthreads();
            if (tid > jj && tid < bw) P[k * bw + tid] = sinv[jj] * P[k * bw + tid];
            __syncthreads();
            // other rows, remaining panel columns; P[i][jj] keeps the multiplier
            const int rem = bw - jj - 1;
            if (rem > 0)
                for (int t = tid; t < n * rem; t += blockDim.x) {
                    const int i = t / rem, j2 = jj + 1 + (t - i * rem);
                    if (i != k) P[i * bw + j2] -= P[i * bw + jj] * P[k * bw + j2];
                }
            __syncthreads();
        }
        // trailing columns
        for (int j = kb + bw + tid; j < W; j += blockDim.x) {
            for (int jj = 0; jj < bw; ++jj) {
                const int pr = swp[jj];
                if (pr != kb + jj) {
                    const c128 t = B[(int64_t)(kb + jj) * W + j];
                    B[(int64_t)(kb + jj) * W + j] = B[(int64_t)pr * W + j];
                    B[(int64_t)pr * W + j] = t;
                }
            }
            c128 R[kPanelMax];
#pragma unroll
            for (int jj = 0; jj < kPanelMax; ++jj) {
                if (jj < bw) {
                    c128 x = B[(int64_t)(kb + jj) * W + j];
#pragma unroll
                    for (int q = 0; q < kPanelMax; ++q)
                        if (q < jj) x -= P[(kb + jj) * bw + q] * R[q];
                    R[jj] = sinv[jj] * x;
                }
            }
            for (int i = 0; i < n; ++i) {
                if (i >= kb && i < kb + bw) continue;
                c128 acc = B[(int64_t)i * W + j];
#pragma unroll
                for (int q = 0; q < kPanelMax; ++q)
                    if (q < bw) acc -= P[i * bw + q] * R[q];
                B[(int64_t)i * W + j] = acc;
            }
#pragma unroll
            for (int jj = 0; jj < kPanelMax; ++jj) {
                if (jj < bw) {
                    c128 x = R[jj];
#pragma unroll
                    for (int q = 0; q < kPanelMax; ++q)
                        if (q > jj && q < bw) x -= P[(kb + jj) * bw + q] * R[q];
                    B[(int64_t)(kb + jj) * W + j] = x;
                }
            }
        }
        __syncthreads();   // trailing columns complete before the next panel load
    }
    // Y = right block (n x no); row q of the kept inverse is column q of Y
    const int64_t mo = m_off[c];
    for (int64_t t = tid; t < (int64_t)no * n; t += blockDim.x) {
        const int q = (int)(t / n), j = (int)(t - (int64_t)q * n);
        const c128 v = B[(int64_t)j * W + n + q];
        m64[mo + t] = v;
        m32[mo + t] = c64((float)v.re, (float)v.im);
    }
}

void launch_ras_setup(int c0, int cnt, const int64_t *ext_off, const int32_t *ext, const int32_t *own_off,
                      const int32_t *own_pos, const int64_t *ws_off, const int64_t *m_off, const int32_t *cmed,
                      const RasSource *src, c128 *ws, c128 *m64, c64 *m32, int *fail, hipStream_t st) {
    if (cnt <= 0) return;
    hipLaunchKernelGGL(k_ras_gather, dim3(cnt), dim3(512), 0, st, c0, ext_off, ext, own_off, own_pos, ws_off, cmed,
                       src, ws);
    SIE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_ras_invert, dim3(cnt), dim3(512), 0, st, c0, ext_off, own_off, ws_off, m_off, ws, m64, m32,
                       fail);
    SIE_HIP(hipGetLastError());
}

// y[own] = M_own x[ext] for every cluster and every right-hand side: one
// workgroup per (cluster, kRasRows owned rows, right-hand side), x[ext]
// staged in LDS, one wave per owned row (lanes over the extended set).
constexpr int kRasRows = 16;

// active (optional, [nrhs][nobj]): the owned rows of a cluster whose object
// cobj[c] is inactive for the right-hand side are written zero.
template <typename T>
__global__ __launch_bounds__(256) void k_ras_apply(const int64_t *__restrict__ ext_off, const int32_t *__restrict__ ext,
                                                   const int32_t *__restrict__ own_off, const int32_t *__restrict__ own,
                                                   const int64_t *__restrict__ m_off, const cx<T> *__restrict__ M,
                                                   const cx<T> *__restrict__ x, cx<T> *__restrict__ y, int64_t ld,
                                                   const uint8_t *__restrict__ active, int nobj,
                                                   const int32_t *__restrict__ cobj) {
    __shared__ __align__(16) T lds[2 * kRasMax];
    cx<T> *xs = reinterpret_cast<cx<T> *>(lds);
    const int c = blockIdx.x;
    const int o0 = own_off[c];
    const int no = own_off[c + 1] - o0;
    const int q0 = blockIdx.y * kRasRows;
    if (q0 >= no) return;                      // uniform over the workgroup
    x += blockIdx.z * ld;
    y += blockIdx.z * ld;
    if (active && !active[(int64_t)blockIdx.z * nobj + cobj[c]]) {   // uniform over the workgroup
        const int q1 = min(no, q0 + kRasRows);
        for (int q = q0 + (int)threadIdx.x; q < q1; q += blockDim.x) y[own[o0 + q]] = cx<T>();
        return;
    }
    const int64_t e0 = ext_off[c];
    const int n = (int)(ext_off[c + 1] - e0);
    for (int i = threadIdx.x; i < n; i += blockDim.x) xs[i] = x[ext[e0 + i]];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const cx<T> *Mc = M + m_off[c];
    const int q1 = min(no, q0 + kRasRows);
    for (int q = q0 + wv; q < q1; q += nw) {
        const cx<T> *row = Mc + (int64_t)q * n;
        T re = 0, im = 0, re2 = 0, im2 = 0;
        int j = lane;
        for (; j + 64 < n; j += 128) {
            const cx<T> a = row[j], b = xs[j], a2 = row[j + 64], b2 = xs[j + 64];
            re += a.re * b.re - a.im * b.im;
            im += a.re * b.im + a.im * b.re;
            re2 += a2.re * b2.re - a2.im * b2.im;
            im2 += a2.re * b2.im + a2.im * b2.re;
        }
        if (j < n) {
            const cx<T> a = row[j], b = xs[j];
            re += a.re * b.re - a.im * b.im;
            im += a.re * b.im + a.im * b.re;
        }
        re += re2;
        im += im2;
        for (int off = 32; off > 0; off >>= 1) {
            re += __shfl_down(re, off);
            im += __shfl_down(im, off);
        }
        if (lane == 0) y[own[o0 + q]] = cx<T>(re, im);
    }
}

template <typename T>
void launch_ras_apply(int nc, int max_own, const int64_t *ext_off, const int32_t *ext, const int32_t *own_off,
                      const int32_t *own, const int64_t *m_off, const cx<T> *M, const cx<T> *x, cx<T> *y, int64_t ld,
                      int nrhs, hipStream_t st, const uint8_t *active, int nobj, const int32_t *cobj) {
    if (nc <= 0 || nrhs <= 0 || max_own <= 0) return;
    SIE_CHECK(nrhs <= 65535, SIE_EINVAL, "too many right-hand sides for one preconditioner launch");
    const dim3 grid((unsigned)nc, (unsigned)((max_own + kRasRows - 1) / kRasRows), (unsigned)nrhs);
    hipLaunchKernelGGL(k_ras_apply<T>, grid, dim3(256), 0, st, ext_off, ext, own_off, own, m_off, M, x, y, ld, active, nobj, cobj);
    SIE_HIP(hipGetLastError());
}

template void launch_ras_apply<float>(int, int, const int64_t *, const int32_t *, const int32_t *,
                                      const int32_t *, const int64_t *, const c64 *, const c64 *, c64 *, int64_t,
                                      int, hipStream_t, const uint8_t *, int, const int32_t *);
template void launch_ras_apply<double>(int, int, const int64_t *, const int32_t *, const int32_t *,
                                       const int32_t *, const int64_t *, const c128 *, const c128 *, c128 *,
                                       int64_t, int, hipStream_t, const uint8_t *, int, const int32_t *);

}  // namespace sie
