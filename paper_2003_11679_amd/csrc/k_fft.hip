// Zero-padded 3D FFT convolution on the live box of an AIM grid
// (Sec. III-D-1: grid potentials from grid sources through the Toeplitz
// convolution matrices G and G_grad, applied in the spectral domain).
//
// The 3D transform is done as five passes over HBM, each a batch of 1D
// transforms of power-of-two length along one axis, staged through LDS:
//   x forward   grid[F][nz][ny][nx]  -> A[F][nz][ny][mx]   (pad nx -> mx)
//   y forward   A                    -> B[F][nz][my][mx]   (pad ny -> my)
//   z fused     B (in place): forward z (pad nz -> mz), multiply by the
//               octant-folded spectrum, inverse z, keep nz
//   y inverse   B -> A  (keep ny)
//   x inverse   A -> out[F][nz][ny][nx] (keep nx)
// Zero padding is never stored: a pass reads only the live prefix of its
// lines and writes only what the next pass reads.
#include "common.h"
#include "kernels.h"

namespace sie {

template <typename T> __device__ inline void sincospi_t(T x, T *s, T *c);
template <> __device__ inline void sincospi_t<double>(double x, double *s, double *c) { sincospi(x, s, c); }
template <> __device__ inline void sincospi_t<float>(float x, float *s, float *c) { sincospif(x, s, c); }

// Radix-2 Stockham transform of `nl` lines of length L held in LDS (line-major,
// row pitch `pitch`).  Ping-pongs between a and b; returns the buffer holding
// the result.  sign = -1 forward, +1 inverse (unscaled).
template <typename T>
__device__ cx<T> *lds_fft(cx<T> *a, cx<T> *b, int L, int nl, int pitch, T sign) {
    const int half = L >> 1;
    const int total = nl * half;
    for (int p = 1; p < L; p <<= 1) {
        for (int it = threadIdx.x; it < total; it += blockDim.x) {
            const int line = it / half;
            const int i = it - line * half;
            const int k = i & (p - 1);
            cx<T> u0 = a[line * pitch + i];
            cx<T> u1 = a[line * pitch + i + half];
            T s, c;
            sincospi_t<T>(sign * T(k) / T(p), &s, &c);
            cx<T> w(c, s);
            u1 = w * u1;
            const int j = (i << 1) - k;
            b[line * pitch + j] = u0 + u1;
            b[line * pitch + j + p] = u0 - u1;
        }
        __syncthreads();
        cx<T> *t = a; a = b; b = t;
    }
    return a;
}

// Generic pass: lines of length L along an axis with element strides
// (s_in, s_out); the block handles `tx` lines.  Line (b, j) starts at
// in + b*bs_in + j*js_in.  j runs over [0, nj), b over gridDim.y * (tiles).
// contiguous: element stride 1 (x passes) -> threads walk along lines;
// otherwise lines are adjacent in memory (js = 1) -> threads walk across lines.
template <typename T>
__global__ void k_fft_pass(const cx<T> *__restrict__ in, cx<T> *__restrict__ out, int L, int n_in,
                           int n_out, long s_in, long s_out, long js_in, long js_out, long bs_in,
                           long bs_out, int nj, int tx, int contiguous, T sign) {
    extern __shared__ unsigned char smem_raw[];
    cx<T> *buf0 = reinterpret_cast<cx<T> *>(smem_raw);
    const int pitch = L + 1;
    cx<T> *buf1 = buf0 + tx * pitch;
    const int j0 = blockIdx.x * tx;
    const long b = blockIdx.y;
    const int nlines = min(tx, nj - j0);
    const cx<T> *src = in + b * bs_in + (long)j0 * js_in;
    cx<T> *dst = out + b * bs_out + (long)j0 * js_out;
    const int total = tx * L;
    for (int it = threadIdx.x; it < total; it += blockDim.x) {
        int line, pos;
        if (contiguous) { line = it / L; pos = it - line * L; }
        else { pos = it / tx; line = it - pos * tx; }
        cx<T> v;
        if (line < nlines && pos < n_in) v = src[(long)line * js_in + (long)pos * s_in];
        buf0[line * pitch + pos] = v;
    }
    __syncthreads();
    cx<T> *res = lds_fft<T>(buf0, buf1, L, tx, pitch, sign);
    const int totalo = tx * n_out;
    for (int it = threadIdx.x; it < totalo; it += blockDim.x) {
        int line, pos;
        if (contiguous) { line = it / n_out; pos = it - line * n_out; }
        else { pos = it / tx; line = it - pos * tx; }
        if (line < nlines) dst[(long)line * js_out + (long)pos * s_out] = res[line * pitch + pos];
    }
}

// Octant lookup of a spectrum that is even (kind 0) or odd along axis
// (kind - 1) (kinds 1..3 = dG/dx, dG/dy, dG/dz).
template <typename T>
__device__ inline cx<T> spec_at(const cx<T> *spec, long oct, int kind, int kx, int ky, int kz,
                                int mx, int my, int mz) {
    int fx = kx <= mx / 2 ? kx : mx - kx;
    int fy = ky <= my / 2 ? ky : my - ky;
    int fz = kz <= mz / 2 ? kz : mz - kz;
    cx<T> v = spec[(long)kind * oct + ((long)fz * (my / 2 + 1) + fy) * (mx / 2 + 1) + fx];
    bool neg = (kind == 1 && kx > mx / 2) || (kind == 2 && ky > my / 2) || (kind == 3 && kz > mz / 2);
    return neg ? -v : v;
}

// Fused z pass.  buf [F][nz][my][mx]; lines along z (stride my*mx), tiles of
// tx consecutive x.  mode 0: every field times G (scalar kernel).  mode 1:
// the three fields (J_x, J_y, J_z) are replaced by grad G x J:
//   psi_x = Gy Jz - Gz Jy,  psi_y = Gz Jx - Gx Jz,  psi_z = Gx Jy - Gy Jx.
template <typename T>
__global__ void k_fft_zpass(cx<T> *__restrict__ buf, const cx<T> *__restrict__ spec, int mx, int my,
                            int mz, int nz, int nf, int tx, int mode) {
    extern __shared__ unsigned char smem_raw[];
    const int nfb = mode == 1 ? 3 : 1;        // fields per block
    const int pitch = mz + 1;
    cx<T> *buf0 = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *buf1 = buf0 + nfb * tx * pitch;
    const int x0 = blockIdx.x * tx;
    const int ky = blockIdx.y;
    const int f0 = mode == 1 ? 0 : blockIdx.z;
    const int nlines = min(tx, mx - x0);
    const long plane = (long)my * mx;
    const long fstride = (long)nz * plane;
    const long oct = (long)(mx / 2 + 1) * (my / 2 + 1) * (mz / 2 + 1);
    const int nl = nfb * tx;                  // LDS lines: (field, x)
    for (int it = threadIdx.x; it < nl * mz; it += blockDim.x) {
        int pos = it / nl, l = it - pos * nl;
        int f = l / tx, xi = l - f * tx;
        cx<T> v;
        if (xi < nlines && pos < nz) v = buf[(long)(f0 + f) * fstride + pos * plane + (long)ky * mx + x0 + xi];
        buf0[l * pitch + pos] = v;
    }
    __syncthreads();
    cx<T> *res = lds_fft<T>(buf0, buf1, mz, nl, pitch, T(-1));
    cx<T> *oth = res == buf0 ? buf1 : buf0;
    // spectral product
    for (int it = threadIdx.x; it < tx * mz; it += blockDim.x) {
        int kz = it / tx, xi = it - kz * tx;
        int kx = x0 + xi;
        if (xi >= nlines) continue;
        if (mode == 0) {
            cx<T> g = spec_at<T>(spec, oct, 0, kx, ky, kz, mx, my, mz);
            res[xi * pitch + kz] = g * res[xi * pitch + kz];
        } else {
            cx<T> gx = spec_at<T>(spec, oct, 1, kx, ky, kz, mx, my, mz);
            cx<T> gy = spec_at<T>(spec, oct, 2, kx, ky, kz, mx, my, mz);
            cx<T> gz = spec_at<T>(spec, oct, 3, kx, ky, kz, mx, my, mz);
            cx<T> jx = res[(0 * tx + xi) * pitch + kz];
            cx<T> jy = res[(1 * tx + xi) * pitch + kz];
            cx<T> jz = res[(2 * tx + xi) * pitch + kz];
            res[(0 * tx + xi) * pitch + kz] = gy * jz - gz * jy;
            res[(1 * tx + xi) * pitch + kz] = gz * jx - gx * jz;
            res[(2 * tx + xi) * pitch + kz] = gx * jy - gy * jx;
        }
    }
    __syncthreads();
    res = lds_fft<T>(res, oth, mz, nl, pitch, T(1));
    for (int it = threadIdx.x; it < nl * nz; it += blockDim.x) {
        int pos = it / nl, l = it - pos * nl;
        int f = l / tx, xi = l - f * tx;
        if (xi < nlines) buf[(long)(f0 + f) * fstride + pos * plane + (long)ky * mx + x0 + xi] = res[l * pitch + pos];
    }
}

static int lines_per_block(int L, size_t elem, int nf_per_block) {
    // two LDS buffers of tx lines x (L + 1) elements within 64 KiB
    long cap = 65536 / (2 * (long)(L + 1) * elem * nf_per_block);
    int tx = 1;
    while (tx * 2 <= cap && tx * 2 <= 64) tx *= 2;
    return tx;
}

template <typename T>
static void pass(const cx<T> *in, cx<T> *out, int L, int n_in, int n_out, long s_in, long s_out,
                 long js_in, long js_out, long bs_in, long bs_out, int nj, long nb, bool contiguous,
                 T sign, hipStream_t st) {
    int tx = lines_per_block(L, sizeof(cx<T>), 1);
    if (contiguous) tx = std::min(tx, 16);
    dim3 grid((nj + tx - 1) / tx, (unsigned)nb);
    size_t sh = 2 * (size_t)tx * (L + 1) * sizeof(cx<T>);
    hipLaunchKernelGGL(k_fft_pass<T>, grid, dim3(256), sh, st, in, out, L, n_in, n_out, s_in, s_out,
                       js_in, js_out, bs_in, bs_out, nj, tx, contiguous ? 1 : 0, sign);
    SIE_HIP(hipGetLastError());
}

// out may alias in.  nf fields; mode 0 (G) or 1 (grad G x, nf == 3).
template <typename T>
void fft_convolve(const Grid &g, const cx<T> *spec, int nf, int mode, const cx<T> *in, cx<T> *out,
                  cx<T> *bufA, cx<T> *bufB, hipStream_t st) {
    const int nx = g.nl[0], ny = g.nl[1], nz = g.nl[2];
    const int mx = g.m[0], my = g.m[1], mz = g.m[2];
    SIE_CHECK(mode == 0 || nf == 3, SIE_EINVAL, "grad-G convolution needs 3 fields");
    SIE_CHECK(mx <= 1024 && my <= 1024 && mz <= 1024, SIE_EGRID, "FFT length above 1024");
    // x forward: lines (f, z, y) contiguous; batch b = f*nz + z, j = y
    pass<T>(in, bufA, mx, nx, mx, 1, 1, nx, mx, (long)ny * nx, (long)ny * mx, ny, (long)nf * nz, true,
            T(-1), st);
    // y forward: lines along y, j = x (adjacent), batch b = f*nz + z
    pass<T>(bufA, bufB, my, ny, my, mx, mx, 1, 1, (long)ny * mx, (long)my * mx, mx, (long)nf * nz, false,
            T(-1), st);
    // z fused
    {
        int nfb = mode == 1 ? 3 : 1;
        int tx = lines_per_block(mz, sizeof(cx<T>), nfb);
        dim3 grid((mx + tx - 1) / tx, my, mode == 1 ? 1 : nf);
        size_t sh = 2 * (size_t)nfb * tx * (mz + 1) * sizeof(cx<T>);
        hipLaunchKernelGGL(k_fft_zpass<T>, grid, dim3(256), sh, st, bufB, spec, mx, my, mz, nz, nf, tx, mode);
        SIE_HIP(hipGetLastError());
    }
    // y inverse: keep ny
    pass<T>(bufB, bufA, my, my, ny, mx, mx, 1, 1, (long)my * mx, (long)ny * mx, mx, (long)nf * nz, false,
            T(1), st);
    // x inverse: keep nx
    pass<T>(bufA, out, mx, mx, nx, 1, 1, mx, nx, (long)ny * mx, (long)ny * nx, ny, (long)nf * nz, true,
            T(1), st);
}

// Full (unpruned) forward 3D FFT of a [mz][my][mx] complex128 volume in place,
// using `tmp` of the same size (spectrum construction).
void fft3d_full_fwd(c128 *vol, c128 *tmp, int mx, int my, int mz, hipStream_t st) {
    pass<double>(vol, tmp, mx, mx, mx, 1, 1, mx, mx, (long)my * mx, (long)my * mx, my, mz, true, -1.0, st);
    pass<double>(tmp, vol, my, my, my, mx, mx, 1, 1, (long)my * mx, (long)my * mx, mx, mz, false, -1.0, st);
    // z: lines along z with stride my*mx; treat (y) as batch, j = x
    pass<double>(vol, tmp, mz, mz, mz, (long)my * mx, (long)my * mx, 1, 1, mx, mx, mx, my, false, -1.0, st);
    SIE_HIP(hipMemcpyAsync(vol, tmp, sizeof(c128) * (size_t)mx * my * mz, hipMemcpyDeviceToDevice, st));
}

template void fft_convolve<float>(const Grid &, const c64 *, int, int, const c64 *, c64 *, c64 *, c64 *, hipStream_t);
template void fft_convolve<double>(const Grid &, const c128 *, int, int, const c128 *, c128 *, c128 *, c128 *, hipStream_t);

}  // namespace sie
