// Device application of the supernodal LU factors (see sparse_lu.cpp): one
// workgroup per supernode of a level.  Its rows first gather what the
// already solved supernodes contribute (descendants in the forward sweep,
// ancestors in the backward sweep), then the dense inverse of the
// supernode's diagonal block is applied.  Supernodes of one level own
// disjoint positions and read only positions of other levels.
#include "common.h"
#include "sparse_lu.h"

namespace sie {

template <bool FWD>
__global__ void __launch_bounds__(256) k_lu_level(const int32_t *__restrict__ lev_sn, const int32_t *__restrict__ sn_p0,
                                                  const int32_t *__restrict__ sn_n, const int64_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ cols, const c128 *__restrict__ vals,
                                                  const int64_t *__restrict__ inv_off, const c128 *__restrict__ inv,
                                                  c128 *x, int64_t n) {
    __shared__ double tsh[2 * kLUMaxSupernode];
    c128 *t = reinterpret_cast<c128 *>(tsh);
    const int sn = lev_sn[blockIdx.x];
    const int p0 = sn_p0[sn], nn = sn_n[sn];
    c128 *xr = x + (int64_t)blockIdx.y * n;
    for (int i = threadIdx.x; i < nn; i += blockDim.x) {
        c128 acc = xr[p0 + i];
        const int64_t b = row_ptr[p0 + i], e = row_ptr[p0 + i + 1];
        for (int64_t j = b; j < e; ++j) acc -= vals[j] * xr[cols[j]];
        t[i] = acc;
    }
    __syncthreads();
    const c128 *M = inv + inv_off[sn];
    for (int i = threadIdx.x; i < nn; i += blockDim.x) {
        c128 s;
        const c128 *row = M + (int64_t)i * nn;
        if (FWD) {
            for (int k = 0; k <= i; ++k) s += row[k] * t[k];
        } else {
            for (int k = i; k < nn; ++k) s += row[k] * t[k];
        }
        xr[p0 + i] = s;
    }
}

void launch_lu_level(const SparseLU &f, int level, bool forward, int nrhs, c128 *x, hipStream_t st) {
    const int b = f.lev_ptr[level], e = f.lev_ptr[level + 1];
    if (e <= b || nrhs < 1) return;
    SIE_CHECK(nrhs <= 65535, SIE_EINVAL, "too many right-hand sides");
    const dim3 grid((unsigned)(e - b), (unsigned)nrhs);
    if (forward)
        hipLaunchKernelGGL(k_lu_level<true>, grid, dim3(256), 0, st, f.lev_sn.p + b, f.sn_p0.p, f.sn_n.p,
                           f.lrow_ptr.p, f.lcol.p, f.lval.p, f.inv_off.p, f.linv.p, x, f.n);
    else
        hipLaunchKernelGGL(k_lu_level<false>, grid, dim3(256), 0, st, f.lev_sn.p + b, f.sn_p0.p, f.sn_n.p,
                           f.urow_ptr.p, f.ucol.p, f.uval.p, f.inv_off.p, f.uinv.p, x, f.n);
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
