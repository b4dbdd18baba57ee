// Device application of the supernodal LU factors (see sparse_lu.cpp), one
// level of the dissection tree at a time.  The rows of a level first gather
// what the already solved supernodes contribute (descendants in the forward
// sweep, ancestors in the backward sweep) into a work vector, then the
// dense inverse of each supernode's diagonal block is applied to it.  Rows
// are spread over workgroups (a few rows each, one wavefront per row), so
// that the few large separators near the root still fill many compute
// units.  Supernodes of one level own disjoint positions and read only
// positions of other levels.
#include "common.h"
#include "sparse_lu.h"

namespace sie {

template <typename T>
__device__ inline cx<T> lu_wave_sum(cx<T> v) {
    for (int off = 32; off > 0; off >>= 1) {
        v.re += __shfl_xor(v.re, off, 64);
        v.im += __shfl_xor(v.im, off, 64);
    }
    return v;
}

// Gather: for row i of the block's supernode (one wavefront, lanes over the
// row's off-block entries), w[p0 + i] = x[p0 + i] - sum_j A[p0 + i][j] x[j],
// j in the levels solved before.  T: precision of the factors and vectors.
template <typename T>
__global__ void __launch_bounds__(64 * kLURowsPerBlock)
    k_lu_rows_gather(const int32_t *__restrict__ blk_sn, const int32_t *__restrict__ blk_row0,
                     const int32_t *__restrict__ sn_p0, const int32_t *__restrict__ sn_n,
                     const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ cols,
                     const cx<T> *__restrict__ vals, const cx<T> *__restrict__ x, cx<T> *__restrict__ w, int64_t n) {
    const int lane = threadIdx.x & 63;
    const int sn = blk_sn[blockIdx.x];
    const int i = blk_row0[blockIdx.x] + (threadIdx.x >> 6);
    if (i >= sn_n[sn]) return;   // uniform over the wavefront
    const int64_t p = sn_p0[sn] + i;
    const cx<T> *xr = x + (int64_t)blockIdx.y * n;
    cx<T> acc;
    // four entries per lane in flight (the same order of summation per lane)
    int64_t j = row_ptr[p] + lane;
    const int64_t e = row_ptr[p + 1];
    for (; j + 192 < e; j += 256) {
        const int32_t c0 = cols[j], c1 = cols[j + 64], c2 = cols[j + 128], c3 = cols[j + 192];
        const cx<T> v0 = vals[j], v1 = vals[j + 64], v2 = vals[j + 128], v3 = vals[j + 192];
        const cx<T> x0 = xr[c0], x1 = xr[c1], x2 = xr[c2], x3 = xr[c3];
        acc += v0 * x0;
        acc += v1 * x1;
        acc += v2 * x2;
        acc += v3 * x3;
    }
    for (; j < e; j += 64) acc += vals[j] * xr[cols[j]];
    acc = lu_wave_sum(acc);
    if (lane == 0) w[(int64_t)blockIdx.y * n + p] = xr[p] - acc;
}

// Dense step: x[p0 + i] = sum_k Dinv[i][k] w[p0 + k] over the triangle of the
// inverse (k <= i forward, k >= i backward), one wavefront per row, lanes
// over k (the row-major inverse read contiguously).
template <bool FWD, typename T>
__global__ void __launch_bounds__(64 * kLURowsPerBlock)
    k_lu_rows_dense(const int32_t *__restrict__ blk_sn, const int32_t *__restrict__ blk_row0,
                    const int32_t *__restrict__ sn_p0, const int32_t *__restrict__ sn_n,
                    const int64_t *__restrict__ inv_off, const cx<T> *__restrict__ inv,
                    const cx<T> *__restrict__ w, cx<T> *__restrict__ x, int64_t n) {
    const int lane = threadIdx.x & 63;
    const int sn = blk_sn[blockIdx.x];
    const int nn = sn_n[sn];
    const int i = blk_row0[blockIdx.x] + (threadIdx.x >> 6);
    if (i >= nn) return;   // uniform over the wavefront
    const int64_t p0 = sn_p0[sn];
    const cx<T> *row = inv + inv_off[sn] + (int64_t)i * nn;
    const cx<T> *wr = w + (int64_t)blockIdx.y * n + p0;
    const int k0 = FWD ? 0 : i, k1 = FWD ? i + 1 : nn;
    cx<T> acc;
    int k = k0 + lane;
    for (; k + 192 < k1; k += 256) {
        const cx<T> a0 = row[k], a1 = row[k + 64], a2 = row[k + 128], a3 = row[k + 192];
        const cx<T> b0 = wr[k], b1 = wr[k + 64], b2 = wr[k + 128], b3 = wr[k + 192];
        acc += a0 * b0;
        acc += a1 * b1;
        acc += a2 * b2;
        acc += a3 * b3;
    }
    for (; k < k1; k += 64) acc += row[k] * wr[k];
    acc = lu_wave_sum(acc);
    if (lane == 0) x[(int64_t)blockIdx.y * n + p0 + i] = acc;
}

template <typename T> struct LUArrays;
template <> struct LUArrays<double> {
    static const c128 *lval(const SparseLU &f) { return f.lval.p; }
    static const c128 *uval(const SparseLU &f) { return f.uval.p; }
    static const c128 *linv(const SparseLU &f) { return f.linv.p; }
    static const c128 *uinv(const SparseLU &f) { return f.uinv.p; }
    static c128 *work(const SparseLU &f) { return f.work.p; }
    static size_t work_n(const SparseLU &f) { return f.work.n; }
};
template <> struct LUArrays<float> {
    static const c64 *lval(const SparseLU &f) { return f.lval32.p; }
    static const c64 *uval(const SparseLU &f) { return f.uval32.p; }
    static const c64 *linv(const SparseLU &f) { return f.linv32.p; }
    static const c64 *uinv(const SparseLU &f) { return f.uinv32.p; }
    static c64 *work(const SparseLU &f) { return f.work32.p; }
    static size_t work_n(const SparseLU &f) { return f.work32.n; }
};

template <typename T>
void launch_lu_level(const SparseLU &f, int level, bool forward, int nrhs, cx<T> *x, hipStream_t st) {
    using A = LUArrays<T>;
    const int b = f.blk_ptr[level], e = f.blk_ptr[level + 1];
    if (e <= b || nrhs < 1) return;
    SIE_CHECK(nrhs <= 65535, SIE_EINVAL, "too many right-hand sides");
    SIE_CHECK(A::work_n(f) >= (size_t)nrhs * f.n, SIE_EINVAL, "sparse LU work buffer too small");
    const dim3 grid((unsigned)(e - b), (unsigned)nrhs), block(64 * kLURowsPerBlock);
    const int32_t *bs = f.blk_sn.p + b, *br = f.blk_row0.p + b;
    hipLaunchKernelGGL(k_lu_rows_gather<T>, grid, block, 0, st, bs, br, f.sn_p0.p, f.sn_n.p,
                       forward ? f.lrow_ptr.p : f.urow_ptr.p, forward ? f.lcol.p : f.ucol.p,
                       forward ? A::lval(f) : A::uval(f), x, A::work(f), f.n);
    SIE_HIP(hipGetLastError());
    if (forward)
        hipLaunchKernelGGL((k_lu_rows_dense<true, T>), grid, block, 0, st, bs, br, f.sn_p0.p, f.sn_n.p, f.inv_off.p,
                           A::linv(f), A::work(f), x, f.n);
    else
        hipLaunchKernelGGL((k_lu_rows_dense<false, T>), grid, block, 0, st, bs, br, f.sn_p0.p, f.sn_n.p,
                           f.inv_off.p, A::uinv(f), A::work(f), x, f.n);
    SIE_HIP(hipGetLastError());
}

template void launch_lu_level<double>(const SparseLU &, int, bool, int, c128 *, hipStream_t);
template void launch_lu_level<float>(const SparseLU &, int, bool, int, c64 *, hipStream_t);

__global__ void k_lu_narrow(const c128 *__restrict__ a, c64 *__restrict__ b, int64_t n) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) b[e] = c64((float)a[e].re, (float)a[e].im);
}

void lu_make_fp32(SparseLU &f, hipStream_t st) {
    auto narrow = [&](const DBuf<c128> &a, DBuf<c64> &b) {
        b.alloc(a.n);
        if (!a.n) return;
        hipLaunchKernelGGL(k_lu_narrow, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a.p, b.p,
                           (int64_t)a.n);
        SIE_HIP(hipGetLastError());
    };
    narrow(f.lval, f.lval32);
    narrow(f.uval, f.uval32);
    narrow(f.linv, f.linv32);
    narrow(f.uinv, f.uinv32);
    SIE_HIP(hipStreamSynchronize(st));
}

template <typename T>
__global__ void k_lu_gather(int64_t n, int64_t r0, int64_t E, const int32_t *__restrict__ iperm,
                            const cx<T> *__restrict__ x, cx<T> *__restrict__ xp) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    xp[blockIdx.y * n + iperm[j]] = x[blockIdx.y * E + r0 + j];
}

template <typename T>
__global__ void k_lu_scatter(int64_t n, int64_t r0, int64_t E, const int32_t *__restrict__ iperm,
                             const cx<T> *__restrict__ xp, cx<T> *__restrict__ y) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    y[blockIdx.y * E + r0 + j] = xp[blockIdx.y * n + iperm[j]];
}

template <typename T>
void launch_lu_gather(int64_t n, int64_t r0, int64_t E, int nrhs, const int32_t *iperm, const cx<T> *x, cx<T> *xp,
                      hipStream_t st) {
    if (n <= 0 || nrhs < 1) return;
    SIE_CHECK(nrhs <= 65535, SIE_EINVAL, "too many right-hand sides");
    hipLaunchKernelGGL(k_lu_gather<T>, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs), dim3(256), 0, st, n, r0, E,
                       iperm, x, xp);
    SIE_HIP(hipGetLastError());
}

template <typename T>
void launch_lu_scatter(int64_t n, int64_t r0, int64_t E, int nrhs, const int32_t *iperm, const cx<T> *xp, cx<T> *y,
                       hipStream_t st) {
    if (n <= 0 || nrhs < 1) return;
    SIE_CHECK(nrhs <= 65535, SIE_EINVAL, "too many right-hand sides");
    hipLaunchKernelGGL(k_lu_scatter<T>, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs), dim3(256), 0, st, n, r0,
                       E, iperm, xp, y);
    SIE_HIP(hipGetLastError());
}

template void launch_lu_gather<float>(int64_t, int64_t, int64_t, int, const int32_t *, const c64 *, c64 *,
                                      hipStream_t);
template void launch_lu_gather<double>(int64_t, int64_t, int64_t, int, const int32_t *, const c128 *, c128 *,
                                       hipStream_t);
template void launch_lu_scatter<float>(int64_t, int64_t, int64_t, int, const int32_t *, const c64 *, c64 *,
                                       hipStream_t);
template void launch_lu_scatter<double>(int64_t, int64_t, int64_t, int, const int32_t *, const c128 *, c128 *,
                                        hipStream_t);

}  // namespace sie
