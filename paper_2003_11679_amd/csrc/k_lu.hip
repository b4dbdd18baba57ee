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

__device__ inline c128 lu_wave_sum(c128 v) {
    for (int off = 32; off > 0; off >>= 1) {
        v.re += __shfl_xor(v.re, off, 64);
        v.im += __shfl_xor(v.im, off, 64);
    }
    return v;
}

// Gather: for row i of the block's supernode (one wavefront, lanes over the
// row's off-block entries), w[p0 + i] = x[p0 + i] - sum_j A[p0 + i][j] x[j],
// j in the levels solved before.
__global__ void __launch_bounds__(64 * kLURowsPerBlock)
    k_lu_rows_gather(const int32_t *__restrict__ blk_sn, const int32_t *__restrict__ blk_row0,
                     const int32_t *__restrict__ sn_p0, const int32_t *__restrict__ sn_n,
                     const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ cols,
                     const c128 *__restrict__ vals, const c128 *__restrict__ x, c128 *__restrict__ w, int64_t n) {
    const int lane = threadIdx.x & 63;
    const int sn = blk_sn[blockIdx.x];
    const int i = blk_row0[blockIdx.x] + (threadIdx.x >> 6);
    if (i >= sn_n[sn]) return;   // uniform over the wavefront
    const int64_t p = sn_p0[sn] + i;
    const c128 *xr = x + (int64_t)blockIdx.y * n;
    c128 acc;
    for (int64_t j = row_ptr[p] + lane; j < row_ptr[p + 1]; j += 64) acc += vals[j] * xr[cols[j]];
    acc = lu_wave_sum(acc);
    if (lane == 0) w[(int64_t)blockIdx.y * n + p] = xr[p] - acc;
}

// Dense step: x[p0 + i] = sum_k Dinv[i][k] w[p0 + k] over the triangle of the
// inverse (k <= i forward, k >= i backward), one wavefront per row, lanes
// over k (the row-major inverse read contiguously).
template <bool FWD>
__global__ void __launch_bounds__(64 * kLURowsPerBlock)
    k_lu_rows_dense(const int32_t *__restrict__ blk_sn, const int32_t *__restrict__ blk_row0,
                    const int32_t *__restrict__ sn_p0, const int32_t *__restrict__ sn_n,
                    const int64_t *__restrict__ inv_off, const c128 *__restrict__ inv,
                    const c128 *__restrict__ w, c128 *__restrict__ x, int64_t n) {
    const int lane = threadIdx.x & 63;
    const int sn = blk_sn[blockIdx.x];
    const int nn = sn_n[sn];
    const int i = blk_row0[blockIdx.x] + (threadIdx.x >> 6);
    if (i >= nn) return;   // uniform over the wavefront
    const int64_t p0 = sn_p0[sn];
    const c128 *row = inv + inv_off[sn] + (int64_t)i * nn;
    const c128 *wr = w + (int64_t)blockIdx.y * n + p0;
    const int k0 = FWD ? 0 : i, k1 = FWD ? i + 1 : nn;
    c128 acc;
    for (int k = k0 + lane; k < k1; k += 64) acc += row[k] * wr[k];
    acc = lu_wave_sum(acc);
    if (lane == 0) x[(int64_t)blockIdx.y * n + p0 + i] = acc;
}

void launch_lu_level(const SparseLU &f, int level, bool forward, int nrhs, c128 *x, hipStream_t st) {
    const int b = f.blk_ptr[level], e = f.blk_ptr[level + 1];
    if (e <= b || nrhs < 1) return;
    SIE_CHECK(nrhs <= 65535, SIE_EINVAL, "too many right-hand sides");
    SIE_CHECK(f.work.n >= (size_t)nrhs * f.n, SIE_EINVAL, "sparse LU work buffer too small");
    const dim3 grid((unsigned)(e - b), (unsigned)nrhs), block(64 * kLURowsPerBlock);
    const int32_t *bs = f.blk_sn.p + b, *br = f.blk_row0.p + b;
    hipLaunchKernelGGL(k_lu_rows_gather, grid, block, 0, st, bs, br, f.sn_p0.p, f.sn_n.p,
                       forward ? f.lrow_ptr.p : f.urow_ptr.p, forward ? f.lcol.p : f.ucol.p,
                       forward ? f.lval.p : f.uval.p, x, f.work.p, f.n);
    SIE_HIP(hipGetLastError());
    if (forward)
        hipLaunchKernelGGL(k_lu_rows_dense<true>, grid, block, 0, st, bs, br, f.sn_p0.p, f.sn_n.p, f.inv_off.p,
                           f.linv.p, f.work.p, x, f.n);
    else
        hipLaunchKernelGGL(k_lu_rows_dense<false>, grid, block, 0, st, bs, br, f.sn_p0.p, f.sn_n.p, f.inv_off.p,
                           f.uinv.p, f.work.p, x, f.n);
    SIE_HIP(hipGetLastError());
}


template <typename T>
__global__ void k_lu_gather(int64_t n, int64_t r0, int64_t E, const int32_t *__restrict__ iperm,
                            const cx<T> *__restrict__ x, c128 *__restrict__ xp) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    const cx<T> v = x[blockIdx.y * E + r0 + j];
    xp[blockIdx.y * n + iperm[j]] = c128((double)v.re, (double)v.im);
}

template <typename T>
__global__ void k_lu_scatter(int64_t n, int64_t r0, int64_t E, const int32_t *__restrict__ iperm,
                             const c128 *__restrict__ xp, cx<T> *__restrict__ y) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    const c128 v = xp[blockIdx.y * n + iperm[j]];
    y[blockIdx.y * E + r0 + j] = cx<T>((T)v.re, (T)v.im);
}

template <typename T>
void launch_lu_gather(int64_t n, int64_t r0, int64_t E, int nrhs, const int32_t *iperm, const cx<T> *x, c128 *xp,
                      hipStream_t st) {
    if (n <= 0 || nrhs < 1) return;
    SIE_CHECK(nrhs <= 65535, SIE_EINVAL, "too many right-hand sides");
    hipLaunchKernelGGL(k_lu_gather<T>, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs), dim3(256), 0, st, n, r0, E,
                       iperm, x, xp);
    SIE_HIP(hipGetLastError());
}

template <typename T>
void launch_lu_scatter(int64_t n, int64_t r0, int64_t E, int nrhs, const int32_t *iperm, const c128 *xp, cx<T> *y,
                       hipStream_t st) {
    if (n <= 0 || nrhs < 1) return;
    SIE_CHECK(nrhs <= 65535, SIE_EINVAL, "too many right-hand sides");
    hipLaunchKernelGGL(k_lu_scatter<T>, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs), dim3(256), 0, st, n, r0,
                       E, iperm, xp, y);
    SIE_HIP(hipGetLastError());
}

template void launch_lu_gather<float>(int64_t, int64_t, int64_t, int, const int32_t *, const c64 *, c128 *,
                                      hipStream_t);
template void launch_lu_gather<double>(int64_t, int64_t, int64_t, int, const int32_t *, const c128 *, c128 *,
                                       hipStream_t);
template void launch_lu_scatter<float>(int64_t, int64_t, int64_t, int, const int32_t *, const c128 *, c64 *,
                                       hipStream_t);
template void launch_lu_scatter<double>(int64_t, int64_t, int64_t, int, const int32_t *, const c128 *, c128 *,
                                        hipStream_t);

}  // namespace sie
