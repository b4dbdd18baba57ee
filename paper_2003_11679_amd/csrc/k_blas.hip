// Vector kernels of the Krylov solvers: conversions, axpby, batched dot
// products with FP64 accumulation (Gram-Schmidt), basis updates.
#include "problem.h"

namespace sie {

template <typename Ti, typename To>
__global__ void k_convert(const cx<Ti> *__restrict__ in, cx<To> *__restrict__ out, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = cx<To>((To)in[i].re, (To)in[i].im);
}
template <typename Ti, typename To>
void launch_convert(const cx<Ti> *in, cx<To> *out, int64_t n, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL((k_convert<Ti, To>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
    SIE_HIP(hipGetLastError());
}

template <typename T>
__global__ void k_axpby(int64_t n, c128 a, const cx<T> *__restrict__ x, c128 b, cx<T> *__restrict__ y) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const cx<T> aa((T)a.re, (T)a.im), bb((T)b.re, (T)b.im);
    y[i] = aa * x[i] + bb * y[i];
}
template <typename T> void launch_axpby(int64_t n, c128 a, const cx<T> *x, c128 b, cx<T> *y, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_axpby<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, x, b, y);
    SIE_HIP(hipGetLastError());
}

template <typename T>
__global__ void k_scale_into(int64_t n, c128 a, const cx<T> *__restrict__ x, cx<T> *__restrict__ y) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = cx<T>((T)a.re, (T)a.im) * x[i];
}
template <typename T> void launch_scale_into(int64_t n, c128 a, const cx<T> *x, cx<T> *y, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scale_into<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, x, y);
    SIE_HIP(hipGetLastError());
}

// y = 0 (a fill kernel, so the call also works where memset nodes are unwanted)
template <typename T>
__global__ void k_zero(int64_t n, cx<T> *__restrict__ y) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = cx<T>();
}
template <typename T> void launch_zero(int64_t n, cx<T> *y, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, y);
    SIE_HIP(hipGetLastError());
}

// Batched dot products of ns systems stored [ns][n] inside every vector:
// h[s * hstride + j] = sum_i conj(V_j[s][i]) w[s][i], j < J, where V_j starts
// at V + j * ldv.  Partial sums per block (b, j, s), then a final reduction;
// FP64 accumulation.
template <typename T>
__global__ void k_dots_part(int64_t n, const cx<T> *__restrict__ V, int64_t ldv, const cx<T> *__restrict__ w,
                            c128 *__restrict__ part, int nb) {
    __shared__ double sre[256], sim[256];
    const int j = blockIdx.y, s = blockIdx.z, J = gridDim.y;
    const cx<T> *v = V + j * ldv + s * n;
    const cx<T> *ws = w + s * n;
    double re = 0, im = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double ar = v[i].re, ai = v[i].im, br = ws[i].re, bi = ws[i].im;
        re += ar * br + ai * bi;
        im += ar * bi - ai * br;
    }
    sre[threadIdx.x] = re; sim[threadIdx.x] = im;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) { sre[threadIdx.x] += sre[threadIdx.x + k]; sim[threadIdx.x] += sim[threadIdx.x + k]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[((int64_t)s * J + j) * nb + blockIdx.x] = c128(sre[0], sim[0]);
}

__global__ void k_dots_final(int J, const c128 *__restrict__ part, int nb, c128 *__restrict__ h, int hstride,
                             c128 *__restrict__ hmirror) {
    __shared__ double sre[256], sim[256];
    const int j = blockIdx.x, s = blockIdx.y;
    const c128 *ps = part + ((int64_t)s * J + j) * nb;
    double re = 0, im = 0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) { re += ps[b].re; im += ps[b].im; }
    sre[threadIdx.x] = re; sim[threadIdx.x] = im;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) { sre[threadIdx.x] += sre[threadIdx.x + k]; sim[threadIdx.x] += sim[threadIdx.x + k]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const c128 v(sre[0], sim[0]);
        h[(int64_t)s * hstride + j] = v;
        if (hmirror) hmirror[(int64_t)s * hstride + j] = v;
    }
}

// part holds ns * J * nb partial sums.
template <typename T>
void launch_dots_sys(int64_t n, int J, const cx<T> *V, int64_t ldv, int ns, const cx<T> *w, c128 *part, int nb,
                     c128 *h, int hstride, hipStream_t st, c128 *hmirror) {
    if (J <= 0 || ns <= 0) return;
    hipLaunchKernelGGL(k_dots_part<T>, dim3(nb, J, ns), dim3(256), 0, st, n, V, ldv, w, part, nb);
    SIE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_dots_final, dim3(J, ns), dim3(256), 0, st, J, part, nb, h, hstride, hmirror);
    SIE_HIP(hipGetLastError());
}

template <typename T>
void launch_dots(int64_t n, int J, const cx<T> *V, int64_t ldv, const cx<T> *w, c128 *part, int nb, c128 *h,
                 hipStream_t st) {
    launch_dots_sys<T>(n, J, V, ldv, 1, w, part, nb, h, J, st, nullptr);
}

// w[s] += SGN sum_j V_j[s] h[s * hstride + j].  A workgroup covers 64
// elements; its 4 waves take every fourth j (FP64 partial sums), and wave 0
// adds the 4 partials in a fixed order.
template <typename T, int SGN>
__global__ __launch_bounds__(256) void k_gemv(int64_t n, int J, const cx<T> *__restrict__ V, int64_t ldv,
                                              const c128 *__restrict__ h, int hstride, cx<T> *__restrict__ w) {
    __shared__ double pre[4][64], pim[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t i = blockIdx.x * (int64_t)64 + lane;
    const int s = blockIdx.y;
    V += s * n;
    h += (int64_t)s * hstride;
    w += s * n;
    double re = 0, im = 0;
    if (i < n)
        for (int j = wv; j < J; j += 4) {
            const cx<T> v = V[j * ldv + i];
            const c128 c = h[j];
            re += v.re * c.re - v.im * c.im;
            im += v.re * c.im + v.im * c.re;
        }
    pre[wv][lane] = re;
    pim[wv][lane] = im;
    __syncthreads();
    if (wv == 0 && i < n) {
        const double sr = ((pre[0][lane] + pre[1][lane]) + pre[2][lane]) + pre[3][lane];
        const double si = ((pim[0][lane] + pim[1][lane]) + pim[2][lane]) + pim[3][lane];
        w[i] = cx<T>((T)(w[i].re + SGN * sr), (T)(w[i].im + SGN * si));
    }
}
template <typename T>
void launch_gemv_sys(int64_t n, int J, const cx<T> *V, int64_t ldv, int ns, const c128 *h, int hstride, cx<T> *w,
                     bool add, hipStream_t st) {
    if (J <= 0 || n <= 0 || ns <= 0) return;
    const dim3 grid((unsigned)((n + 63) / 64), (unsigned)ns);
    if (add) hipLaunchKernelGGL((k_gemv<T, 1>), grid, dim3(256), 0, st, n, J, V, ldv, h, hstride, w);
    else hipLaunchKernelGGL((k_gemv<T, -1>), grid, dim3(256), 0, st, n, J, V, ldv, h, hstride, w);
    SIE_HIP(hipGetLastError());
}
template <typename T>
void launch_gemv_sub(int64_t n, int J, const cx<T> *V, int64_t ldv, const c128 *h, cx<T> *w, hipStream_t st) {
    launch_gemv_sys<T>(n, J, V, ldv, 1, h, J, w, false, st);
}
template <typename T>
void launch_gemv_add(int64_t n, int J, const cx<T> *V, int64_t ldv, const c128 *h, cx<T> *w, hipStream_t st) {
    launch_gemv_sys<T>(n, J, V, ldv, 1, h, J, w, true, st);
}

// y[s] = c[s] x[s] for ns systems [ns][n] (c on the device)
template <typename T>
__global__ void k_scale_sys(int64_t n, const c128 *__restrict__ c, const cx<T> *__restrict__ x, cx<T> *__restrict__ y) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = blockIdx.y;
    const cx<T> cc((T)c[s].re, (T)c[s].im);
    y[s * n + i] = cc * x[s * n + i];
}
template <typename T>
void launch_scale_sys(int64_t n, int ns, const c128 *c, const cx<T> *x, cx<T> *y, hipStream_t st) {
    if (n <= 0 || ns <= 0) return;
    hipLaunchKernelGGL(k_scale_sys<T>, dim3((unsigned)((n + 255) / 256), (unsigned)ns), dim3(256), 0, st, n, c, x, y);
    SIE_HIP(hipGetLastError());
}

// y[s] = c.v[s] x[s] with the coefficients passed by value (no copy to the
// device ahead of the launch)
template <typename T>
__global__ void k_scale_val(int64_t n, ScaleArg c, const cx<T> *__restrict__ x, cx<T> *__restrict__ y) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = blockIdx.y;
    const cx<T> cc((T)c.v[s].re, (T)c.v[s].im);
    y[s * n + i] = cc * x[s * n + i];
}
template <typename T>
void launch_scale_val(int64_t n, int ns, const ScaleArg &c, const cx<T> *x, cx<T> *y, hipStream_t st) {
    if (n <= 0 || ns <= 0) return;
    SIE_CHECK(ns <= kScaleArg, SIE_EINVAL, "too many systems for by-value coefficients");
    hipLaunchKernelGGL(k_scale_val<T>, dim3((unsigned)((n + 255) / 256), (unsigned)ns), dim3(256), 0, st, n, c, x, y);
    SIE_HIP(hipGetLastError());
}

// y[s] = x[s] / sqrt(Re d[s * dstride]) for a squared norm d on the device;
// zero where that norm is zero
template <typename T>
__global__ void k_scale_rnorm(int64_t n, const c128 *__restrict__ d, int dstride, const cx<T> *__restrict__ x,
                              cx<T> *__restrict__ y) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = blockIdx.y;
    const double q = d[(int64_t)s * dstride].re;
    const T c = q > 0.0 ? (T)(1.0 / sqrt(q)) : (T)0;
    const cx<T> v = x[s * n + i];
    y[s * n + i] = cx<T>(c * v.re, c * v.im);
}
template <typename T>
void launch_scale_rnorm(int64_t n, int ns, const c128 *d, int dstride, const cx<T> *x, cx<T> *y, hipStream_t st) {
    if (n <= 0 || ns <= 0) return;
    hipLaunchKernelGGL(k_scale_rnorm<T>, dim3((unsigned)((n + 255) / 256), (unsigned)ns), dim3(256), 0, st, n, d,
                       dstride, x, y);
    SIE_HIP(hipGetLastError());
}

template <typename T>
__global__ void k_diag_mul(int64_t n, const c128 *__restrict__ d, const cx<T> *__restrict__ x, cx<T> *__restrict__ y) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const cx<T> dd((T)d[i].re, (T)d[i].im);
    y[i] = dd * x[i];
}
template <typename T> void launch_diag_mul(int64_t n, const c128 *d, const cx<T> *x, cx<T> *y, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_diag_mul<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, d, x, y);
    SIE_HIP(hipGetLastError());
}

template void launch_convert<double, float>(const c128 *, c64 *, int64_t, hipStream_t);
template void launch_convert<float, double>(const c64 *, c128 *, int64_t, hipStream_t);
template void launch_convert<double, double>(const c128 *, c128 *, int64_t, hipStream_t);
#define SIE_INST_B(T)                                                                                          \
    template void launch_zero<T>(int64_t, cx<T> *, hipStream_t);                                               \
    template void launch_axpby<T>(int64_t, c128, const cx<T> *, c128, cx<T> *, hipStream_t);                  \
    template void launch_scale_into<T>(int64_t, c128, const cx<T> *, cx<T> *, hipStream_t);                   \
    template void launch_dots<T>(int64_t, int, const cx<T> *, int64_t, const cx<T> *, c128 *, int, c128 *,     \
                                 hipStream_t);                                                                \
    template void launch_gemv_sub<T>(int64_t, int, const cx<T> *, int64_t, const c128 *, cx<T> *, hipStream_t); \
    template void launch_gemv_add<T>(int64_t, int, const cx<T> *, int64_t, const c128 *, cx<T> *, hipStream_t); \
    template void launch_dots_sys<T>(int64_t, int, const cx<T> *, int64_t, int, const cx<T> *, c128 *, int, c128 *, \
                                     int, hipStream_t, c128 *);                                               \
    template void launch_gemv_sys<T>(int64_t, int, const cx<T> *, int64_t, int, const c128 *, int, cx<T> *, bool, \
                                     hipStream_t);                                                            \
    template void launch_scale_sys<T>(int64_t, int, const c128 *, const cx<T> *, cx<T> *, hipStream_t);       \
    template void launch_scale_val<T>(int64_t, int, const ScaleArg &, const cx<T> *, cx<T> *, hipStream_t);   \
    template void launch_scale_rnorm<T>(int64_t, int, const c128 *, int, const cx<T> *, cx<T> *, hipStream_t); \
    template void launch_diag_mul<T>(int64_t, const c128 *, const cx<T> *, cx<T> *, hipStream_t);
SIE_INST_B(float)
SIE_INST_B(double)

}  // namespace sie
