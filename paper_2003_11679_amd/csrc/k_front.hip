// Numeric multifrontal factorisation on the device (the ordering and the
// symbolic part are in sparse_lu.cpp): per front, in postorder on one
// stream, clear the front, place its original entries, add its children's
// update matrices, eliminate its own positions, and scatter the results
// into the factors' final arrays and the update-matrix stack.
//
// The dense partial elimination is right-looking and blocked by panels of
// kFrontPanel columns, no pivoting, FP64:
//   diagonal block   A11 = L11 U11                 (k_front_diag, in LDS)
//   column panel     L21 = A21 U11^-1              (k_tri_right)
//   row panel        U12 = L11^-1 A12              (k_tri_left, unit lower)
//   trailing block   A22 -= L21 U12                (k_gemm_sub)
// After the n own positions are eliminated, the inverses of the diagonal
// blocks L_NN (unit lower) and U_NN (upper) that the level-by-level solve
// applies are formed by blocked substitution on identity right-hand sides,
// with the same three kernels.
#include <algorithm>

#include "common.h"
#include "sparse_lu.h"

namespace sie {

constexpr int kFrontPanel = 32;

// LDS holds complex values as double2 (c128 has constructors).
__device__ inline c128 ld2(const double2 &v) { return c128(v.x, v.y); }
__device__ inline double2 st2(c128 v) { return make_double2(v.re, v.im); }

// LU without pivoting of the kb x kb block at (k0, k0), in place (unit lower
// multipliers below the diagonal).  A pivot that is zero or not finite sets
// *bad (the arithmetic goes on; the caller rejects the factors).
__global__ void __launch_bounds__(256) k_front_diag(c128 *__restrict__ F, int64_t ld, int k0, int kb, int *bad) {
    __shared__ double2 a[kFrontPanel][kFrontPanel + 1];
    const int t = threadIdx.x;
    for (int e = t; e < kb * kb; e += 256) a[e / kb][e % kb] = st2(F[(int64_t)(k0 + e / kb) * ld + k0 + e % kb]);
    __syncthreads();
    for (int k = 0; k < kb; ++k) {
        const c128 piv = ld2(a[k][k]);
        if (t == 0) {
            const double pa = sqrt(piv.re * piv.re + piv.im * piv.im);
            if (!(pa > 0.0) || !isfinite(pa)) *bad = 1;
        }
        const c128 ip = cdiv(c128(1.0), piv);
        __syncthreads();
        if (t > k && t < kb) a[t][k] = st2(ld2(a[t][k]) * ip);
        __syncthreads();
        const int w = kb - k - 1;
        for (int e = t; e < w * w; e += 256) {
            const int i = k + 1 + e / w, j = k + 1 + e % w;
            a[i][j] = st2(ld2(a[i][j]) - ld2(a[i][k]) * ld2(a[k][j]));
        }
        __syncthreads();
    }
    for (int e = t; e < kb * kb; e += 256) F[(int64_t)(k0 + e / kb) * ld + k0 + e % kb] = ld2(a[e / kb][e % kb]);
}

// Left solve on columns [c0, c1) of the kb rows at X (row stride ldx), in
// place, with the kb x kb triangle at T (row stride ldt):
//   UPPER = false:  X <- L^-1 X, L the unit lower triangle of T;
//   UPPER = true:   X <- U^-1 X, U the upper triangle of T (its diagonal).
// One thread per column; the triangle sits in LDS.
template <bool UPPER>
__global__ void __launch_bounds__(128)
    k_tri_left(const c128 *__restrict__ T, int64_t ldt, c128 *__restrict__ X, int64_t ldx, int kb, int c0, int c1) {
    __shared__ double2 tr[kFrontPanel][kFrontPanel + 1];
    for (int e = threadIdx.x; e < kb * kb; e += blockDim.x) tr[e / kb][e % kb] = st2(T[(int64_t)(e / kb) * ldt + e % kb]);
    __syncthreads();
    const int j = c0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= c1) return;
    c128 x[kFrontPanel];
#pragma unroll
    for (int i = 0; i < kFrontPanel; ++i)
        if (i < kb) x[i] = X[(int64_t)i * ldx + j];
    if (!UPPER) {
#pragma unroll
        for (int i = 1; i < kFrontPanel; ++i) {
            if (i < kb) {
                c128 s = x[i];
#pragma unroll
                for (int l = 0; l < i; ++l) s -= ld2(tr[i][l]) * x[l];
                x[i] = s;
            }
        }
    } else {
#pragma unroll
        for (int i = kFrontPanel - 1; i >= 0; --i) {
            if (i < kb) {
                c128 s = x[i];
#pragma unroll
                for (int l = i + 1; l < kFrontPanel; ++l)
                    if (l < kb) s -= ld2(tr[i][l]) * x[l];
                x[i] = cdiv(s, ld2(tr[i][i]));
            }
        }
    }
#pragma unroll
    for (int i = 0; i < kFrontPanel; ++i)
        if (i < kb) X[(int64_t)i * ldx + j] = x[i];
}

// Right solve X <- X U^-1 on rows [0, nrows) of the kb columns at X (row
// stride ldx), U the upper triangle of the kb x kb block at T.  One thread
// per row.
__global__ void __launch_bounds__(128)
    k_tri_right(const c128 *__restrict__ T, int64_t ldt, c128 *__restrict__ X, int64_t ldx, int kb, int nrows) {
    __shared__ double2 tr[kFrontPanel][kFrontPanel + 1];
    for (int e = threadIdx.x; e < kb * kb; e += blockDim.x) tr[e / kb][e % kb] = st2(T[(int64_t)(e / kb) * ldt + e % kb]);
    __syncthreads();
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    c128 *row = X + (int64_t)r * ldx;
    c128 x[kFrontPanel];
#pragma unroll
    for (int j = 0; j < kFrontPanel; ++j)
        if (j < kb) x[j] = row[j];
#pragma unroll
    for (int j = 0; j < kFrontPanel; ++j) {
        if (j < kb) {
            c128 s = x[j];
#pragma unroll
            for (int l = 0; l < j; ++l) s -= x[l] * ld2(tr[l][j]);
            x[j] = cdiv(s, ld2(tr[j][j]));
        }
    }
#pragma unroll
    for (int j = 0; j < kFrontPanel; ++j)
        if (j < kb) row[j] = x[j];
}

// C -= A B for C [M][N], A [M][K], B [K][N] (row strides ldc, lda, ldb).
// 64 x 64 tiles of C per workgroup of 256 threads (each a 4 x 4 strided
// sub-tile), K in slices of 16 staged through LDS.
constexpr int kGT = 64, kGK = 16;
__global__ void __launch_bounds__(256)
    k_gemm_sub(c128 *__restrict__ C, int64_t ldc, const c128 *__restrict__ A, int64_t lda,
               const c128 *__restrict__ B, int64_t ldb, int M, int N, int K) {
    __shared__ double2 as[kGT][kGK + 1];
    __shared__ double2 bs[kGK][kGT + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i0 = blockIdx.y * kGT, j0 = blockIdx.x * kGT;
    c128 acc[4][4];
    for (int k0 = 0; k0 < K; k0 += kGK) {
        for (int e = threadIdx.x; e < kGT * kGK; e += 256) {
            const int i = e / kGK, k = e % kGK;
            as[i][k] = st2((i0 + i < M && k0 + k < K) ? A[(int64_t)(i0 + i) * lda + k0 + k] : c128());
            const int kk = e / kGT, j = e % kGT;
            bs[kk][j] = st2((k0 + kk < K && j0 + j < N) ? B[(int64_t)(k0 + kk) * ldb + j0 + j] : c128());
        }
        __syncthreads();
#pragma unroll 4
        for (int k = 0; k < kGK; ++k) {
            c128 a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = ld2(as[ty + 16 * r][k]);
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = ld2(bs[k][tx + 16 * c]);
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = i0 + ty + 16 * r;
        if (i >= M) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int j = j0 + tx + 16 * c;
            if (j < N) C[(int64_t)i * ldc + j] -= acc[r][c];
        }
    }
}

// X <- identity, n x n.
__global__ void k_front_eye(c128 *__restrict__ X, int n) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    X[e] = (e / n == e % n) ? c128(1.0) : c128();
}

// F <- 0, cnt entries.
__global__ void k_front_zero(c128 *__restrict__ F, int64_t cnt) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < cnt) F[e] = c128();
}

// Original entries: every one has a front position of its own.
__global__ void k_front_place(c128 *__restrict__ F, int64_t m, const int32_t *__restrict__ arow,
                              const int32_t *__restrict__ acol, const int32_t *__restrict__ asrc, int64_t cnt,
                              const c128 *__restrict__ val) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < cnt) F[arow[e] * m + acol[e]] = val[asrc[e]];
}

// Extend-add of one child's update matrix (its boundary positions are
// distinct positions of F).
__global__ void k_front_extend(c128 *__restrict__ F, int64_t m, const c128 *__restrict__ upd, int bc,
                               const int32_t *__restrict__ map) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)bc * bc) return;
    const int a = (int)(e / bc), b = (int)(e % bc);
    F[map[a] * m + map[b]] += upd[e];
}

// L_BN rows and U_NB rows into the factors' CSR value arrays.
__global__ void k_front_extract(const c128 *__restrict__ F, int64_t m, int n, int nb, c128 *__restrict__ lval,
                                const int64_t *__restrict__ loff, c128 *__restrict__ uval,
                                const int64_t *__restrict__ urow) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t half = (int64_t)n * nb;
    if (e < half) {
        const int a = (int)(e / n), k = (int)(e % n);
        lval[loff[a] + k] = F[(n + a) * m + k];
    } else if (e < 2 * half) {
        const int64_t q = e - half;
        const int k = (int)(q / nb), b = (int)(q % nb);
        uval[urow[k] + b] = F[k * m + n + b];
    }
}

// The Schur complement on the boundary onto the update-matrix stack.
__global__ void k_front_push(const c128 *__restrict__ F, int64_t m, int n, int nb, c128 *__restrict__ upd) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)nb * nb) return;
    upd[e] = F[(n + e / nb) * m + n + e % nb];
}

namespace {

unsigned blocks_for(int64_t cnt) { return (unsigned)((cnt + 255) / 256); }

void tri_left(bool upper, const c128 *T, int64_t ldt, c128 *X, int64_t ldx, int kb, int c0, int c1, hipStream_t st) {
    if (c1 <= c0) return;
    const dim3 grid((unsigned)((c1 - c0 + 127) / 128));
    if (upper) hipLaunchKernelGGL(k_tri_left<true>, grid, dim3(128), 0, st, T, ldt, X, ldx, kb, c0, c1);
    else hipLaunchKernelGGL(k_tri_left<false>, grid, dim3(128), 0, st, T, ldt, X, ldx, kb, c0, c1);
    SIE_HIP(hipGetLastError());
}

void gemm_sub(c128 *C, int64_t ldc, const c128 *A, int64_t lda, const c128 *B, int64_t ldb, int M, int N, int K,
              hipStream_t st) {
    if (M <= 0 || N <= 0 || K <= 0) return;
    const dim3 grid((unsigned)((N + kGT - 1) / kGT), (unsigned)((M + kGT - 1) / kGT));
    hipLaunchKernelGGL(k_gemm_sub, grid, dim3(256), 0, st, C, ldc, A, lda, B, ldb, M, N, K);
    SIE_HIP(hipGetLastError());
}

}  // namespace

static void front_eliminate(c128 *F, int m, int n, c128 *linv, c128 *uinv, int *bad, hipStream_t st) {
    SIE_CHECK(m >= n && n > 0 && m <= 65535 * kGT, SIE_EINVAL, "front: bad size");
    const int64_t ld = m;
    for (int k0 = 0; k0 < n; k0 += kFrontPanel) {
        const int kb = std::min(kFrontPanel, n - k0), r0 = k0 + kb, rest = m - r0;
        hipLaunchKernelGGL(k_front_diag, dim3(1), dim3(256), 0, st, F, ld, k0, kb, bad);
        SIE_HIP(hipGetLastError());
        if (rest <= 0) continue;
        const c128 *T = F + (int64_t)k0 * ld + k0;
        hipLaunchKernelGGL(k_tri_right, dim3((unsigned)((rest + 127) / 128)), dim3(128), 0, st, T, ld,
                           F + (int64_t)r0 * ld + k0, ld, kb, rest);
        SIE_HIP(hipGetLastError());
        tri_left(false, T, ld, F + (int64_t)k0 * ld, ld, kb, r0, m, st);
        gemm_sub(F + (int64_t)r0 * ld + r0, ld, F + (int64_t)r0 * ld + k0, ld, F + (int64_t)k0 * ld + r0, ld, rest,
                 rest, kb, st);
    }
    const int64_t nn = (int64_t)n * n;
    const unsigned eg = (unsigned)((nn + 255) / 256);
    hipLaunchKernelGGL(k_front_eye, dim3(eg), dim3(256), 0, st, linv, n);
    hipLaunchKernelGGL(k_front_eye, dim3(eg), dim3(256), 0, st, uinv, n);
    SIE_HIP(hipGetLastError());
    // L_NN X = I, block rows top down: X_k = L_kk^-1 X_k on the columns left
    // of the block's end, then the rows below lose L_ik X_k
    for (int k0 = 0; k0 < n; k0 += kFrontPanel) {
        const int kb = std::min(kFrontPanel, n - k0), r0 = k0 + kb;
        tri_left(false, F + (int64_t)k0 * ld + k0, ld, linv + (int64_t)k0 * n, n, kb, 0, r0, st);
        gemm_sub(linv + (int64_t)r0 * n, n, F + (int64_t)r0 * ld + k0, ld, linv + (int64_t)k0 * n, n, n - r0, r0, kb,
                 st);
    }
    // U_NN X = I, block rows bottom up: X_k = U_kk^-1 X_k on the columns from
    // the block's start, then the rows above lose U_ik X_k
    for (int k0 = ((n - 1) / kFrontPanel) * kFrontPanel; k0 >= 0; k0 -= kFrontPanel) {
        const int kb = std::min(kFrontPanel, n - k0);
        tri_left(true, F + (int64_t)k0 * ld + k0, ld, uinv + (int64_t)k0 * n, n, kb, k0, n, st);
        gemm_sub(uinv + k0, n, F + k0, ld, uinv + (int64_t)k0 * n + k0, n, k0, n - k0, kb, st);
    }
}

void launch_front_step(const FrontStep &s, hipStream_t st) {
    const int m = s.m, n = s.n, nb = m - n;
    SIE_CHECK(m > 0 && n >= 0 && nb >= 0 && m <= 65535 * kGT, SIE_EINVAL, "front: bad size");
    SIE_CHECK(s.child_upd.size() == s.child_nb.size() && s.child_map.size() == s.child_nb.size(), SIE_EINVAL,
              "front: bad children");
    const int64_t mm = (int64_t)m * m;
    hipLaunchKernelGGL(k_front_zero, dim3(blocks_for(mm)), dim3(256), 0, st, s.F, mm);
    SIE_HIP(hipGetLastError());
    if (s.nasm > 0) {
        hipLaunchKernelGGL(k_front_place, dim3(blocks_for(s.nasm)), dim3(256), 0, st, s.F, (int64_t)m, s.arow,
                           s.acol, s.asrc, s.nasm, s.val);
        SIE_HIP(hipGetLastError());
    }
    for (size_t c = 0; c < s.child_nb.size(); ++c) {
        const int bc = s.child_nb[c];
        SIE_CHECK(bc > 0 && bc <= m, SIE_EINVAL, "front: bad child boundary");
        hipLaunchKernelGGL(k_front_extend, dim3(blocks_for((int64_t)bc * bc)), dim3(256), 0, st, s.F, (int64_t)m,
                           s.child_upd[c], bc, s.child_map[c]);
        SIE_HIP(hipGetLastError());
    }
    if (n > 0) {
        front_eliminate(s.F, m, n, s.linv, s.uinv, s.bad, st);
        if (nb > 0) {
            hipLaunchKernelGGL(k_front_extract, dim3(blocks_for(2 * (int64_t)n * nb)), dim3(256), 0, st, s.F,
                               (int64_t)m, n, nb, s.lval, s.loff, s.uval, s.urow);
            SIE_HIP(hipGetLastError());
        }
    }
    if (nb > 0) {
        hipLaunchKernelGGL(k_front_push, dim3(blocks_for((int64_t)nb * nb)), dim3(256), 0, st, s.F, (int64_t)m, n,
                           nb, s.upd);
        SIE_HIP(hipGetLastError());
    }
}

}  // namespace sie
