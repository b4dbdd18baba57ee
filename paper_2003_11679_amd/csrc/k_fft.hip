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
//
// Inside a block a tile of lines sits in LDS and is transformed by
// radix-8 (then 4 or 2) Stockham stages whose butterflies run in
// registers.  The line length is a template parameter, so LDS offsets fold
// into instruction immediates; global addresses are a uniform base plus a
// per-thread 32-bit offset plus a uniform step per register slot.
#include "common.h"
#include "kernels.h"
#include "tune.h"

#include <algorithm>
#include <atomic>

namespace sie {

// LDS tiles store element j of a line at j + j/8: one pad slot every eight
// elements, so that the stride-R writes of the early Stockham stages fall
// on distinct banks.
__device__ __forceinline__ int padj(int j) { return j + (j >> 3); }

// padj(j0 + r * S) for a compile-time stride S: separable when S is a
// multiple of 8 (then the pad of the step is exact).
template <int S>
__device__ __forceinline__ int padj_step(int j0, int r) {
    if constexpr (S % 8 == 0) return padj(j0) + r * (S + S / 8);
    else return padj(j0 + r * S);
}

// LDS element access through float2 / double2, so that a complex value
// moves with one 64-bit (FP32) or 128-bit (FP64) LDS instruction.  LDS
// tiles hold whole elements at element-aligned offsets.
template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };
template <typename T>
__device__ __forceinline__ cx<T> lds_ld(const cx<T> *p) {
    const typename Vec2<T>::type v = *reinterpret_cast<const typename Vec2<T>::type *>(p);
    return cx<T>(v.x, v.y);
}
template <typename T>
__device__ __forceinline__ void lds_st(cx<T> *p, cx<T> a) {
    typename Vec2<T>::type v;
    v.x = a.re;
    v.y = a.im;
    *reinterpret_cast<typename Vec2<T>::type *>(p) = v;
}

// Half twiddle table exp(-2 pi i j / L), j < L/2, built per block in LDS
// (FP64 sincospi, rounded to T).  A stage reads only w^j1, w^2j1 and w^4j1
// with j1 < L/(2R), so every index stays below L/2.
__host__ __device__ constexpr int twiddle_len(int L) { return L >= 2 ? L / 2 : 1; }

template <typename T>
__device__ __forceinline__ void init_twiddles(cx<T> *tw, int L) {
    for (int j = threadIdx.x; j < twiddle_len(L); j += blockDim.x) {
        double sn, cs;
        sincospi(-2.0 * (double)j / (double)L, &sn, &cs);
        lds_st(tw + j, cx<T>((T)cs, (T)sn));
    }
}

// -i a (forward) or +i a (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cx<T> rot_mi(cx<T> a) {
    return INV ? cx<T>(-a.im, a.re) : cx<T>(a.im, -a.re);
}

// In-register DFTs of length 2, 4, 8; forward exp(-2 pi i rq/R), inverse +.
template <typename T>
__device__ __forceinline__ void dft2(cx<T> *u) {
    const cx<T> a = u[0], b = u[1];
    u[0] = a + b;
    u[1] = a - b;
}
template <typename T, bool INV>
__device__ __forceinline__ void dft4(cx<T> *u) {
    const cx<T> s02 = u[0] + u[2], d02 = u[0] - u[2], s13 = u[1] + u[3], d13 = u[1] - u[3];
    const cx<T> jd = rot_mi<T, INV>(d13);
    u[0] = s02 + s13;
    u[2] = s02 - s13;
    u[1] = d02 + jd;
    u[3] = d02 - jd;
}
template <typename T, bool INV>
__device__ __forceinline__ void dft8(cx<T> *u) {
    cx<T> e[4] = {u[0], u[2], u[4], u[6]}, o[4] = {u[1], u[3], u[5], u[7]};
    dft4<T, INV>(e);
    dft4<T, INV>(o);
    const T r2 = T(0.70710678118654752440);
    // w = exp(-+ 2 pi i / 8): w^1 = (1 -+ i)/sqrt2, w^2 = -+ i, w^3 = (-1 -+ i)/sqrt2
    const cx<T> o1 = r2 * (o[1] + rot_mi<T, INV>(o[1]));
    const cx<T> o2 = rot_mi<T, INV>(o[2]);
    const cx<T> o3 = r2 * (rot_mi<T, INV>(o[3]) - o[3]);
    u[0] = e[0] + o[0]; u[4] = e[0] - o[0];
    u[1] = e[1] + o1;   u[5] = e[1] - o1;
    u[2] = e[2] + o2;   u[6] = e[2] - o2;
    u[3] = e[3] + o3;   u[7] = e[3] - o3;
}
template <typename T, int R, bool INV>
__device__ __forceinline__ void dftR(cx<T> *u) {
    if constexpr (R == 2) dft2(u);
    else if constexpr (R == 4) dft4<T, INV>(u);
    else dft8<T, INV>(u);
}

// One radix-R Stockham stage over nl lines of length L = 2^LGL in LDS, in
// place: each thread stages NB = VPT/R butterflies in registers between two
// barriers (the block has NT threads and nl * L <= NT * VPT).  p = 2^LGP is
// the product of the earlier radices; butterfly i (k = i mod p) takes
// x[i + r L/R] times w^(r k L/(p R)) and writes its DFT_R outputs to
// ((i - k) R + k + r p).
// Slot b of thread t: when a line has at most NT butterflies, butterfly
// t mod (L/R) of line t / (L/R) + b NT/(L/R) (so the twiddles are the same
// for all b); otherwise butterfly t + (b mod BPL) NT of line b / BPL, with
// BPL = (L/R)/NT slots per line.
// ZIN (first stage only): inputs at L/2 and above are zero and not read.
// ZOUT (last stage only): outputs at L/2 and above are not written.
template <typename T, int R, int NT, int VPT, int LGL, int LGP, int PITCH, bool INV, bool ZIN, bool ZOUT>
__device__ __forceinline__ void fft_stage(cx<T> *buf, int nl, const cx<T> *tw) {
    constexpr int L = 1 << LGL;
    constexpr int LGR = R == 8 ? 3 : (R == 4 ? 2 : 1);
    constexpr int NB = VPT / R;
    static_assert(NB >= 1, "too few values per thread for this radix");
    constexpr int LGNBF = LGL - LGR;
    constexpr int NBF = 1 << LGNBF;
    constexpr bool WIDE = NBF > NT;
    constexpr int BPL = WIDE ? NBF / NT : 1;
    constexpr int DLINE = WIDE ? 0 : NT >> LGNBF;
    constexpr int P = 1 << LGP;
    constexpr int LGTWS = LGL - LGP - LGR;
    const int tid = threadIdx.x;
    auto bf_i = [&](int b) { return WIDE ? tid + (b % BPL) * NT : tid & (NBF - 1); };
    auto bf_line = [&](int b) { return WIDE ? b / BPL : (tid >> LGNBF) + b * DLINE; };

    // w^(r k L/(p R)), r = 1..R-1: powers 1, 2, 4 from the table, the
    // others as products of those
    auto twiddles = [&](int k, cx<T> *w) {
        const int j1 = k << LGTWS;
        w[1] = lds_ld(tw + j1);
        if constexpr (R >= 4) {
            w[2] = lds_ld(tw + 2 * j1);
            w[3] = w[1] * w[2];
        }
        if constexpr (R == 8) {
            w[4] = lds_ld(tw + 4 * j1);
            w[5] = w[1] * w[4];
            w[6] = w[2] * w[4];
            w[7] = w[3] * w[4];
        }
        if constexpr (INV) {
#pragma unroll
            for (int r = 1; r < R; ++r) w[r] = conj(w[r]);
        }
    };
    constexpr bool SHARED_TW = !WIDE || P <= NT;   // k independent of b
    cx<T> w[R];
    if constexpr (P > 1 && SHARED_TW) twiddles(bf_i(0) & (P - 1), w);

    cx<T> u[NB][R];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int i = bf_i(b), line = bf_line(b);
        if (line < nl) {
            const cx<T> *rd = buf + line * PITCH;
#pragma unroll
            for (int r = 0; r < R; ++r)
                u[b][r] = ZIN && r >= R / 2 ? cx<T>() : lds_ld(rd + padj_step<NBF>(i, r));
            if constexpr (P > 1) {
                cx<T> wb[R];
                if constexpr (!SHARED_TW) twiddles(i & (P - 1), wb);
#pragma unroll
                for (int r = 1; r < R; ++r) u[b][r] = (SHARED_TW ? w[r] : wb[r]) * u[b][r];
            }
            dftR<T, R, INV>(u[b]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int i = bf_i(b), line = bf_line(b);
        if (line < nl) {
            const int k = i & (P - 1);
            const int j = ((i - k) << LGR) + k;
            cx<T> *wr = buf + line * PITCH;
#pragma unroll
            for (int r = 0; r < (ZOUT ? R / 2 : R); ++r) {
                int o;
                if constexpr (P == 1 && R == 8) o = padj(j) + r;   // j = 8 i: no carry into j / 8
                else o = padj_step<P>(j, r);
                lds_st(wr + o, u[b][r]);
            }
        }
    }
    __syncthreads();
}

// Full transform of nl lines of length 2^LGL (lines PITCH apart), natural
// order in and out; radix 8 while at least three factors of two remain,
// then 4 or 2.  The stage sequence is fixed at compile time so that every
// stage's registers are allocated on their own.  ZIN: the upper half of
// every input line is zero (zero-padded forward transform); ZOUT: only the
// lower half of the output is used (pruned inverse transform).
template <typename T, int NT, int VPT, int LGL, int PITCH, bool INV, bool ZIN, bool ZOUT, int LGP = 0>
__device__ __forceinline__ void lds_fft(cx<T> *buf, int nl, const cx<T> *tw) {
    if constexpr (LGP < LGL) {
        constexpr int rem = LGL - LGP;
        constexpr int LGR = rem >= 3 ? 3 : rem;
        constexpr bool LAST = LGP + LGR == LGL;
        fft_stage<T, 1 << LGR, NT, VPT, LGL, LGP, PITCH, INV, ZIN && LGP == 0, ZOUT && LAST>(buf, nl, tw);
        lds_fft<T, NT, VPT, LGL, PITCH, INV, false, ZOUT, LGP + LGR>(buf, nl, tw);
    }
}

// Tile shape of a block: TX = 2^LGTX lines of length L = 2^LGL, PITCH
// elements apart, plus the half twiddle table.  TX is the largest power of
// two with TX * L <= NT * VPT, TX <= NT / 8 (so that the per-slot step along
// a line in the across-lines layouts is a multiple of 8 elements and keeps
// the LDS pad of that step exact) and the tile within kLdsBudget.  PITCH is
// the padded length rounded up so that the TX lines of one row segment fall
// on distinct bank slots of a kBankRow-byte LDS row.
constexpr long kLdsBudget = 80 * 1024;
constexpr int kBankRow = 128;

template <typename T, int NT, int VPT, int LGL>
struct Tile {
    static constexpr int L = 1 << LGL;
    static constexpr int ESZ = 2 * sizeof(T);
    static constexpr int E = kBankRow / ESZ;          // elements per bank row
    static constexpr int base_pitch(int tx) {
        const int b = L + L / 8, c = tx >= E ? 1 : E / tx;
        return b + ((c - b) % E + E) % E;
    }
    static constexpr int lines() {
        int tx = 1;
        while (2 * tx * L <= NT * VPT && 2 * tx <= NT / 8 &&
               (long)(2 * tx * base_pitch(2 * tx) + twiddle_len(L)) * ESZ <= kLdsBudget)
            tx *= 2;
        return tx;
    }
    static constexpr int TX = lines();
    static constexpr int LGTX = TX <= 1 ? 0 : (TX <= 2 ? 1 : (TX <= 4 ? 2 : (TX <= 8 ? 3 : (TX <= 16 ? 4 : (TX <= 32 ? 5 : 6)))));
    static constexpr int PITCH = base_pitch(TX);
    static constexpr size_t BYTES = (size_t)(TX * PITCH + twiddle_len(L)) * ESZ;
    static_assert((1 << LGTX) == TX, "tile lines must be a power of two <= 64");
    static_assert(TX * L <= NT * VPT, "tile larger than the block's register slots");
    static_assert(L <= NT * VPT, "line longer than the block's register slots");
};

// Fields the passes leave out: with active set, field fl of a launch (field
// f0 + fl of the convolution, slot (f0 + fl) / fps, object obj0 + slot) is
// skipped when its object is inactive; batches hold nzb lines per field.
// Nothing reads a skipped field's output (one right-hand side).
struct FieldMask {
    const uint8_t *active = nullptr;
    int obj0 = 0, fps = 1, nslot = 1;
    long f0 = 0, nzb = 1;
};
__device__ __forceinline__ bool field_off(const FieldMask &m, long fl) {
    return m.active && !m.active[m.obj0 + (int)(((m.f0 + fl) / m.fps) % m.nslot)];
}

// Generic pass: TX lines of length L = 2^LGL per block along one axis
// (tile shape Tile<T, NT, VPT, LGL>).  Line (b, j) starts at
// in + b*bs_in + j*js_in.
//   CONTIG: element stride 1 (x passes); threads walk along lines.
//   otherwise adjacent lines are adjacent in memory (stride 1 between
//   lines, s between elements) and threads walk across lines, so each row
//   segment of the tile is one coalesced access.
// Element q of thread t is (line0 + dline(q), pos0 + dpos(q)) with
// dline/dpos compile-time.  Zero padding beyond n_in; only n_out outputs
// written.  PRUNE: forward passes have n_in <= L/2, inverse passes
// n_out <= L/2 (zero-padded convolution), and the transforms skip the
// zero inputs / unused outputs.
template <typename T, int NT, int VPT, int LGL, bool CONTIG, bool INV, bool PRUNE, int MINW>
__global__ void __launch_bounds__(NT, MINW) k_fft_pass(const cx<T> *__restrict__ in, cx<T> *__restrict__ out,
                                                       int n_in, int n_out, int s_in, int s_out, int js_in,
                                                       int js_out, long bs_in, long bs_out, int nj, FieldMask fm) {
    if (field_off(fm, blockIdx.y / fm.nzb)) return;   // uniform over the block
    using TS = Tile<T, NT, VPT, LGL>;
    constexpr int L = 1 << LGL, PITCH = TS::PITCH, TX = TS::TX, LGTX = TS::LGTX;
    constexpr bool ZIN = PRUNE && !INV, ZOUT = PRUNE && INV;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T> *tw = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *buf = tw + twiddle_len(L);
    const int j0 = blockIdx.x * TX;
    const int nlines = min(TX, nj - j0);
    const cx<T> *src = in + (long)blockIdx.y * bs_in + (long)j0 * (CONTIG ? js_in : 1);
    cx<T> *dst = out + (long)blockIdx.y * bs_out + (long)j0 * (CONTIG ? js_out : 1);
    const int tid = threadIdx.x;
    const int line0 = CONTIG ? tid >> LGL : tid & (TX - 1);
    const int pos0 = CONTIG ? tid & (L - 1) : tid >> LGTX;
    auto dline = [&](int q) { return CONTIG ? (q * NT) >> LGL : 0; };
    auto dpos = [&](int q) { return CONTIG ? (q * NT) & (L - 1) : (q * NT) >> LGTX; };
    // LDS slots the transform reads: the whole tile, or its lower half
    // when the upper half of every line is known to be zero
    auto lds_in = [&](int q) {
        return CONTIG ? line0 + dline(q) < TX && (!ZIN || pos0 + dpos(q) < L / 2)
                      : pos0 + dpos(q) < (ZIN ? L / 2 : L);
    };
    auto lds_out = [&](int q) {
        return CONTIG ? line0 + dline(q) < TX && (!ZOUT || pos0 + dpos(q) < L / 2)
                      : pos0 + dpos(q) < (ZOUT ? L / 2 : L);
    };
    const int goff_in = CONTIG ? line0 * js_in + pos0 : line0 + pos0 * s_in;
    const int goff_out = CONTIG ? line0 * js_out + pos0 : line0 + pos0 * s_out;
    const int loff = line0 * PITCH + padj(pos0);   // dpos(q) is a multiple of 8

    cx<T> r[VPT];
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
        const int dl = dline(q), dp = dpos(q);
        if (line0 + dl < nlines && pos0 + dp < n_in)
            r[q] = src[goff_in + (CONTIG ? dl * js_in + dp : dp * s_in)];
        else
            r[q] = cx<T>();
    }
    init_twiddles(tw, L);
#pragma unroll
    for (int q = 0; q < VPT; ++q)
        if (lds_in(q)) lds_st(buf + loff + dline(q) * PITCH + dpos(q) + dpos(q) / 8, r[q]);
    __syncthreads();
    lds_fft<T, NT, VPT, LGL, PITCH, INV, ZIN, ZOUT>(buf, TX, tw);
    // gather the whole tile from LDS first, then issue the global stores
#pragma unroll
    for (int q = 0; q < VPT; ++q)
        if (lds_out(q)) r[q] = lds_ld(buf + loff + dline(q) * PITCH + dpos(q) + dpos(q) / 8);
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
        const int dl = dline(q), dp = dpos(q);
        if (line0 + dl < nlines && pos0 + dp < n_out) dst[goff_out + (CONTIG ? dl * js_out + dp : dp * s_out)] = r[q];
    }
}

// Fused z pass.  buf [F][nz][my][mx]; a block owns a tile of tx (Tile
// shape) consecutive x at one ky and runs its z lines (length mz = 2^LGL,
// nz <= mz/2 live) field by field through LDS: forward z (pruned input),
// spectral product, inverse z (pruned output, keep nz).
// Element q of thread t is (kz, xi) = (t / tx + q NT / tx, t mod tx).
//   MODE 0: each field times G; a block takes up to kZFields fields
//           (blockIdx.z chunk) of rows ky and my - ky (ky <= my/2), which
//           see the same G values, and reads those once into registers.
//   MODE 1: the fields (J_x, J_y, J_z) of triple blockIdx.z become grad G x J,
//           psi_x = Gy Jz - Gz Jy, psi_y = Gz Jx - Gx Jz, psi_z = Gx Jy - Gy Jx;
//           the transformed fields are held in registers until all three
//           are known.
// The spectrum is stored on its (mx/2+1)(my/2+1)(mz/2+1) octant: G is even
// along every axis, dG/dx_a odd along axis a (kinds 1..3).
constexpr int kZFields = 4;   // fields per G z-pass block

// Fields come in runs of fps consecutive fields that share one spectrum:
// run j (of this launch) uses spectrum (run0 + j) mod nspec, spec_stride
// elements apart.  MODE 0: block z index = (run, chunk of kZFields fields of
// the run); MODE 1: block z index = triple, fps a multiple of 3.
template <typename T, int NT, int VPT, int LGL, int MODE, int MINW>
__global__ void __launch_bounds__(NT, MINW) k_fft_zpass(cx<T> *__restrict__ buf, const cx<T> *__restrict__ spec,
                                                        int mx, int my, int nz, int fps, int run0, int nspec,
                                                        long spec_stride, FieldMask fm) {
    using TS = Tile<T, NT, VPT, LGL>;
    constexpr int mz = 1 << LGL, PITCH = TS::PITCH, tx = TS::TX, lgtx = TS::LGTX;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T> *tw = reinterpret_cast<cx<T> *>(smem_raw);
    cx<T> *lb = tw + twiddle_len(mz);
    const int x0 = blockIdx.x * tx;
    // MODE 0 pairs row ky with its mirror my - ky (same G values);
    // MODE 1 takes one row (dG/dy changes sign across the mirror)
    const int ky = blockIdx.y;
    const int nrows = MODE == 0 && ky > 0 && 2 * ky < my ? 2 : 1;
    const int nlines = min(tx, mx - x0);
    const int plane = my * mx;
    const long fstride = (long)nz * plane;
    const int tid = threadIdx.x;
    const int xi = tid & (tx - 1);
    const int pos0 = tid >> lgtx;
    auto dpos = [&](int q) { return (q * NT) >> lgtx; };
    const int goff = pos0 * plane + xi;
    const int loff = xi * PITCH + padj(pos0);
    auto row_base = [&](int row) { return buf + (long)(row == 0 ? ky : my - ky) * mx + x0; };
    // folded spectrum coordinates of this thread's elements
    const int kx = min(x0 + xi, mx - 1);
    const int fx = kx <= mx / 2 ? kx : mx - kx;
    const int fy = ky <= my / 2 ? ky : my - ky;
    const int sx = mx / 2 + 1, sxy = sx * (my / 2 + 1);
    const long oct = (long)sxy * (mz / 2 + 1);
    const int soff = fy * sx + fx;
    init_twiddles(tw, mz);

    auto load_field = [&](int f, int row) {
        const cx<T> *fb = row_base(row) + f * fstride;
        cx<T> r[VPT];
#pragma unroll
        for (int q = 0; q < VPT; ++q)
            r[q] = xi < nlines && pos0 + dpos(q) < nz ? fb[goff + dpos(q) * plane] : cx<T>();
        __syncthreads();                      // earlier readers of lb are done
#pragma unroll
        for (int q = 0; q < VPT; ++q)
            if (pos0 + dpos(q) < mz / 2) lds_st(lb + loff + dpos(q) + dpos(q) / 8, r[q]);
        __syncthreads();
    };
    auto store_field = [&](int f, int row) {
        cx<T> *fb = row_base(row) + f * fstride;
        cx<T> r[VPT];
#pragma unroll
        for (int q = 0; q < VPT; ++q)
            if (pos0 + dpos(q) < mz / 2) r[q] = lds_ld(lb + loff + dpos(q) + dpos(q) / 8);
#pragma unroll
        for (int q = 0; q < VPT; ++q)
            if (xi < nlines && pos0 + dpos(q) < nz) fb[goff + dpos(q) * plane] = r[q];
    };
    auto lds_q = [&](int q) { return lb + loff + dpos(q) + dpos(q) / 8; };
    // spectrum value of kind `kind` at element q (padding lanes clamp kx;
    // their products are never stored)
    auto spec_q = [&](int kind, int q) {
        const int kz = min(pos0 + dpos(q), mz - 1);
        const int fz = kz <= mz / 2 ? kz : mz - kz;
        const cx<T> v = spec[kind * oct + fz * sxy + soff];
        const bool neg = (kind == 1 && kx > mx / 2) || (kind == 2 && ky > my / 2) || (kind == 3 && kz > mz / 2);
        return neg ? -v : v;
    };

    if constexpr (MODE == 0) {
        const int cpr = (fps + kZFields - 1) / kZFields;   // chunks per run
        const int run = blockIdx.z / cpr, ch = blockIdx.z - run * cpr;
        if (field_off(fm, (long)run * fps)) return;          // uniform over the block
        spec += (long)((run0 + run) % nspec) * spec_stride;
        cx<T> g[VPT];
#pragma unroll
        for (int q = 0; q < VPT; ++q) g[q] = spec_q(0, q);
        const int fb = run * fps + ch * kZFields, nfb = min(kZFields, fps - ch * kZFields);
        for (int t = 0; t < nrows * nfb; ++t) {
            const int row = t / nfb, f = fb + t - row * nfb;
            load_field(f, row);
            lds_fft<T, NT, VPT, LGL, PITCH, false, true, false>(lb, tx, tw);
#pragma unroll
            for (int q = 0; q < VPT; ++q)
                if (pos0 + dpos(q) < mz) lds_st(lds_q(q), g[q] * lds_ld(lds_q(q)));
            __syncthreads();
            lds_fft<T, NT, VPT, LGL, PITCH, true, false, true>(lb, tx, tw);
            store_field(f, row);
        }
    } else {
        cx<T> J[3][VPT];
        const int f0 = 3 * blockIdx.z;            // the block's (J_x, J_y, J_z) triple
        if (field_off(fm, f0)) return;            // uniform over the block
        spec += (long)((run0 + f0 / fps) % nspec) * spec_stride;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            load_field(f0 + f, 0);
            lds_fft<T, NT, VPT, LGL, PITCH, false, true, false>(lb, tx, tw);
#pragma unroll
            for (int q = 0; q < VPT; ++q) J[f][q] = pos0 + dpos(q) < mz ? lds_ld(lds_q(q)) : cx<T>();
        }
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const cx<T> gx = spec_q(1, q), gy = spec_q(2, q), gz = spec_q(3, q);
            const cx<T> jx = J[0][q], jy = J[1][q], jz = J[2][q];
            J[0][q] = gy * jz - gz * jy;
            J[1][q] = gz * jx - gx * jz;
            J[2][q] = gx * jy - gy * jx;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            __syncthreads();                  // earlier readers of lb are done
#pragma unroll
            for (int q = 0; q < VPT; ++q)
                if (pos0 + dpos(q) < mz) lds_st(lds_q(q), J[c][q]);
            __syncthreads();
            lds_fft<T, NT, VPT, LGL, PITCH, true, false, true>(lb, tx, tw);
            store_field(f0 + c, 0);
        }
    }
}

// Block shapes (threads NT, values per thread VPT; a tile holds NT * VPT
// values).  Pass and G z-pass tiles hold up to 64 KiB of data (8192
// complex64 or 4096 complex128) with 512 threads, so that two blocks (four
// waves per SIMD, the launch-bounds minimum) share a CU within 128
// registers.  The grad-G z pass keeps three transformed fields in registers
// and runs 256 x 8, at two waves per SIMD in FP32 and one in FP64 (which
// would spill at two).
template <typename T> struct FftShape {
    static constexpr int nt = 512;
    static constexpr int vpt = sizeof(T) == 4 ? 16 : 8;
    static constexpr int minw = 4;
    static constexpr int z_nt = 256;
    static constexpr int z_vpt = sizeof(T) == 4 ? 16 : 8;
    static constexpr int z_minw = 4;
    static constexpr int grad_nt = 256;
    static constexpr int grad_vpt = 8;
    static constexpr int grad_minw = sizeof(T) == 4 ? 2 : 1;
};

// Tile shapes the launch-shape tuner chooses among for the strided y
// passes and the G z pass (threads, values per thread; the first is the
// built-in shape).  A shape only changes which thread runs which butterfly:
// every candidate computes the same values.
template <typename T> struct FftCands;
template <> struct FftCands<float> {
    static constexpr int ny = 3;
    static constexpr int y_nt[ny] = {512, 256, 256};
    static constexpr int y_vpt[ny] = {16, 16, 8};
    static constexpr int nz = 5;
    static constexpr int z_nt[nz] = {256, 512, 256, 128, 128};
    static constexpr int z_vpt[nz] = {16, 16, 8, 16, 8};
};
template <> struct FftCands<double> {
    static constexpr int ny = 2;
    static constexpr int y_nt[ny] = {512, 256};
    static constexpr int y_vpt[ny] = {8, 8};
    static constexpr int nz = 3;
    static constexpr int z_nt[nz] = {256, 512, 128};
    static constexpr int z_vpt[nz] = {8, 8, 8};
};
static_assert(FftCands<float>::y_nt[0] == FftShape<float>::nt && FftCands<float>::y_vpt[0] == FftShape<float>::vpt,
              "the first y candidate is the built-in shape");
static_assert(FftCands<double>::y_nt[0] == FftShape<double>::nt && FftCands<double>::y_vpt[0] == FftShape<double>::vpt,
              "the first y candidate is the built-in shape");
static_assert(FftCands<float>::z_nt[0] == FftShape<float>::z_nt && FftCands<float>::z_vpt[0] == FftShape<float>::z_vpt,
              "the first z candidate is the built-in shape");
static_assert(FftCands<double>::z_nt[0] == FftShape<double>::z_nt &&
                  FftCands<double>::z_vpt[0] == FftShape<double>::z_vpt,
              "the first z candidate is the built-in shape");

// Shortest and longest supported transform (2^3 .. 2^10).
constexpr int kMinLg = 3, kMaxLg = 10;

// Dynamic LDS available to one block on the current device.
static long lds_limit() {
    static std::atomic<long> cached[64];
    int dev = 0;
    SIE_HIP(hipGetDevice(&dev));
    SIE_CHECK(dev >= 0 && dev < 64, SIE_EINVAL, "device index out of range");
    long v = cached[dev].load();
    if (v == 0) {
        int lim = 0;
        SIE_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        v = lim;
        cached[dev].store(v);
    }
    return v;
}

static int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// 32-bit per-thread offsets: every element a block touches must lie within
// 2^31 elements of its uniform base.
static void check_span(long span) {
    SIE_CHECK(span >= 0 && span < (1L << 31), SIE_EGRID, "FFT pass spans more than 2^31 elements");
}

template <typename TS>
static void check_tile() {
    SIE_CHECK((long)TS::BYTES <= lds_limit(), SIE_EDEVICE, "FFT tile needs more LDS than the device offers");
}

template <typename T, int LGL, bool INV, bool PRUNE, int NT = FftShape<T>::nt, int V = FftShape<T>::vpt>
static void launch_pass(const cx<T> *in, cx<T> *out, int n_in, int n_out, long s_in, long s_out, long js_in,
                        long js_out, long bs_in, long bs_out, int nj, long nb, bool contiguous, hipStream_t st,
                        const FieldMask &fm) {
    constexpr int W = FftShape<T>::minw;
    using TS = Tile<T, NT, V, LGL>;
    constexpr int L = 1 << LGL;
    check_tile<TS>();
    SIE_CHECK(nb >= 1 && nb <= 65535, SIE_EGRID, "FFT batch above 65535 lines");
    SIE_CHECK(n_in >= 0 && n_in <= L && n_out >= 0 && n_out <= L, SIE_EINVAL, "FFT line extents exceed the length");
    if (PRUNE) SIE_CHECK(INV ? n_out <= L / 2 : n_in <= L / 2, SIE_EINVAL, "pruned FFT needs a half-length live line");
    dim3 grid((nj + TS::TX - 1) / TS::TX, (unsigned)nb);
    if constexpr (NT == FftShape<T>::nt && V == FftShape<T>::vpt) {
        if (contiguous) {
            SIE_CHECK(s_in == 1 && s_out == 1, SIE_EINVAL, "contiguous FFT pass needs unit element stride");
            check_span((long)TS::TX * std::max(js_in, js_out) + L);
            hipLaunchKernelGGL((k_fft_pass<T, NT, V, LGL, true, INV, PRUNE, W>), grid, dim3(NT), TS::BYTES, st, in,
                               out, n_in, n_out, 1, 1, (int)js_in, (int)js_out, bs_in, bs_out, nj, fm);
            SIE_HIP(hipGetLastError());
            return;
        }
    } else {
        SIE_CHECK(!contiguous, SIE_EINVAL, "contiguous FFT passes take the built-in shape");
    }
    {
        SIE_CHECK(js_in == 1 && js_out == 1, SIE_EINVAL, "strided FFT pass needs adjacent lines");
        check_span((long)L * std::max(s_in, s_out) + TS::TX);
        hipLaunchKernelGGL((k_fft_pass<T, NT, V, LGL, false, INV, PRUNE, W>), grid, dim3(NT), TS::BYTES, st, in,
                           out, n_in, n_out, (int)s_in, (int)s_out, 1, 1, bs_in, bs_out, nj, fm);
    }
    SIE_HIP(hipGetLastError());
}

// Strided pass with y candidate shape C (of FftCands<T>).
template <typename T, int LGL, bool INV, bool PRUNE, int C = 0>
static void launch_pass_shape(int shape, const cx<T> *in, cx<T> *out, int n_in, int n_out, long s_in, long s_out,
                              long js_in, long js_out, long bs_in, long bs_out, int nj, long nb, bool contiguous,
                              hipStream_t st, const FieldMask &fm) {
    if constexpr (C < FftCands<T>::ny) {
        if (shape == C)
            launch_pass<T, LGL, INV, PRUNE, FftCands<T>::y_nt[C], FftCands<T>::y_vpt[C]>(
                in, out, n_in, n_out, s_in, s_out, js_in, js_out, bs_in, bs_out, nj, nb, contiguous, st, fm);
        else
            launch_pass_shape<T, LGL, INV, PRUNE, C + 1>(shape, in, out, n_in, n_out, s_in, s_out, js_in, js_out,
                                                         bs_in, bs_out, nj, nb, contiguous, st, fm);
    } else {
        SIE_CHECK(false, SIE_EINVAL, "FFT pass shape out of range");
    }
}

template <typename T, bool INV, bool PRUNE, int LGL = kMinLg>
static void pass_lg(int lg, const cx<T> *in, cx<T> *out, int n_in, int n_out, long s_in, long s_out, long js_in,
                    long js_out, long bs_in, long bs_out, int nj, long nb, bool contiguous, hipStream_t st,
                    int shape = 0, const FieldMask &fm = FieldMask()) {
    if constexpr (LGL <= kMaxLg) {
        if (lg != LGL)
            pass_lg<T, INV, PRUNE, LGL + 1>(lg, in, out, n_in, n_out, s_in, s_out, js_in, js_out, bs_in, bs_out,
                                            nj, nb, contiguous, st, shape, fm);
        else if (contiguous || shape == 0)
            launch_pass<T, LGL, INV, PRUNE>(in, out, n_in, n_out, s_in, s_out, js_in, js_out, bs_in, bs_out, nj,
                                            nb, contiguous, st, fm);
        else
            launch_pass_shape<T, LGL, INV, PRUNE>(shape, in, out, n_in, n_out, s_in, s_out, js_in, js_out, bs_in,
                                                  bs_out, nj, nb, contiguous, st, fm);
    } else {
        SIE_CHECK(false, SIE_EGRID, "FFT length must be a power of two between 8 and 1024");
    }
}

// One pass of the zero-padded convolution (pruned: forward passes read a
// half-length live prefix, inverse passes keep one).
template <typename T>
static void pass(const cx<T> *in, cx<T> *out, int L, int n_in, int n_out, long s_in, long s_out, long js_in,
                 long js_out, long bs_in, long bs_out, int nj, long nb, bool contiguous, bool inv, hipStream_t st,
                 int shape = 0, const FieldMask &fm = FieldMask()) {
    SIE_CHECK((L & (L - 1)) == 0, SIE_EGRID, "FFT length must be a power of two");
    if (inv)
        pass_lg<T, true, true>(ilog2(L), in, out, n_in, n_out, s_in, s_out, js_in, js_out, bs_in, bs_out, nj, nb,
                               contiguous, st, shape, fm);
    else
        pass_lg<T, false, true>(ilog2(L), in, out, n_in, n_out, s_in, s_out, js_in, js_out, bs_in, bs_out, nj, nb,
                                contiguous, st, shape, fm);
}

// G z pass with z candidate shape C (of FftCands<T>).
template <typename T, int LGL, int C = 0>
static void launch_zpass0(int shape, cx<T> *bufB, const cx<T> *spec, int mx, int my, int nz, int fps, int run0,
                          int nspec, int nf, long spec_stride, hipStream_t st, const FieldMask &fm) {
    if constexpr (C < FftCands<T>::nz) {
        if (shape != C) {
            launch_zpass0<T, LGL, C + 1>(shape, bufB, spec, mx, my, nz, fps, run0, nspec, nf, spec_stride, st, fm);
            return;
        }
        constexpr int NT = FftCands<T>::z_nt[C], V = FftCands<T>::z_vpt[C], W = FftShape<T>::z_minw;
        using TS = Tile<T, NT, V, LGL>;
        check_tile<TS>();
        const int cpr = (fps + kZFields - 1) / kZFields;
        dim3 grid((mx + TS::TX - 1) / TS::TX, my / 2 + 1, (nf / fps) * cpr);
        hipLaunchKernelGGL((k_fft_zpass<T, NT, V, LGL, 0, W>), grid, dim3(NT), TS::BYTES, st, bufB, spec, mx, my, nz,
                           fps, run0, nspec, spec_stride, fm);
    } else {
        SIE_CHECK(false, SIE_EINVAL, "FFT z-pass shape out of range");
    }
}

template <typename T, int LGL = kMinLg>
static void zpass_lg(int lg, const GridView &g, const cx<T> *spec, long spec_stride, int fps, int run0, int nspec,
                     int nf, int mode, cx<T> *bufB, hipStream_t st, int shape = 0,
                     const FieldMask &fm = FieldMask()) {
    if constexpr (LGL <= kMaxLg) {
        if (lg != LGL) {
            zpass_lg<T, LGL + 1>(lg, g, spec, spec_stride, fps, run0, nspec, nf, mode, bufB, st, shape, fm);
            return;
        }
        SIE_CHECK(fps >= 1 && nf % fps == 0 && nspec >= 1, SIE_EINVAL, "fields must form whole spectrum runs");
        constexpr int mz = 1 << LGL;
        const int mx = g.m[0], my = g.m[1], nz = g.nl[2];
        check_span((long)nz * my * mx);
        SIE_CHECK(nz <= mz / 2, SIE_EGRID, "z live extent above half the FFT length");
        if (mode == 0) {
            launch_zpass0<T, LGL>(shape, bufB, spec, mx, my, nz, fps, run0, nspec, nf, spec_stride, st, fm);
        } else {
            constexpr int NT = FftShape<T>::grad_nt, V = FftShape<T>::grad_vpt, W = FftShape<T>::grad_minw;
            using TS = Tile<T, NT, V, LGL>;
            check_tile<TS>();
            SIE_CHECK(fps % 3 == 0, SIE_EINVAL, "grad-G spectrum runs must hold whole field triples");
            dim3 grid((mx + TS::TX - 1) / TS::TX, my, nf / 3);
            hipLaunchKernelGGL((k_fft_zpass<T, NT, V, LGL, 1, W>), grid, dim3(NT), TS::BYTES, st, bufB, spec, mx, my,
                               nz, fps, run0, nspec, spec_stride, fm);
        }
        SIE_HIP(hipGetLastError());
    } else {
        SIE_CHECK(false, SIE_EGRID, "FFT length must be a power of two between 8 and 1024");
    }
}

// One chunk of fields through the five passes (nf * nz <= 65535).
template <typename T>
static void convolve_chunk(const GridView &g, const cx<T> *spec, long spec_stride, int fps, int run0, int nspec,
                           int nf, int mode, const cx<T> *in, cx<T> *out, cx<T> *bufA, cx<T> *bufB, hipStream_t st,
                           const FieldMask &fm) {
    const int nx = g.nl[0], ny = g.nl[1], nz = g.nl[2];
    const int mx = g.m[0], my = g.m[1], mz = g.m[2];
    SIE_CHECK((mz & (mz - 1)) == 0, SIE_EGRID, "FFT length must be a power of two");
    // the timed candidates run without the field mask (whole passes)
    const FieldMask none;
    auto yfwd = [&](int shape, const FieldMask &m) {   // lines along y, j = x (adjacent), batch b = f*nz + z
        pass<T>(bufA, bufB, my, ny, my, mx, mx, 1, 1, (long)ny * mx, (long)my * mx, mx, (long)nf * nz, false, false,
                st, shape, m);
        return true;
    };
    auto zfused = [&](int shape, const FieldMask &m) {
        zpass_lg<T>(ilog2(mz), g, spec, spec_stride, fps, run0, nspec, nf, mode, bufB, st, shape, m);
        return true;
    };
    auto yinv = [&](int shape, const FieldMask &m) {   // keep ny
        pass<T>(bufB, bufA, my, my, ny, mx, mx, 1, 1, (long)my * mx, (long)ny * mx, mx, (long)nf * nz, false, true,
                st, shape, m);
        return true;
    };
    // tile shapes: on the first call for this shape the candidates run on
    // bufA / bufB before they hold anything (the passes below overwrite
    // both), so timing them disturbs no data
    int dev = 0;
    SIE_HIP(hipGetDevice(&dev));
    const int prec = (int)sizeof(T);
    const TuneKey kyf{dev, TUNE_FFT_YFWD, prec, {my, mx, ny, (int64_t)nf * nz, 0}};
    const TuneKey kyi{dev, TUNE_FFT_YINV, prec, {my, mx, ny, (int64_t)nf * nz, 0}};
    const TuneKey kz{dev, TUNE_FFT_Z, prec, {mz, mx, my, nz, (int64_t)nf * 65536 + fps}};
    const int syf = tune_pick(kyf, FftCands<T>::ny, [&](int c) { return yfwd(c, none); }, st);
    const int sz = mode == 0 ? tune_pick(kz, FftCands<T>::nz, [&](int c) { return zfused(c, none); }, st) : 0;
    const int syi = tune_pick(kyi, FftCands<T>::ny, [&](int c) { return yinv(c, none); }, st);
    // x forward: lines (f, z, y) contiguous; batch b = f*nz + z, j = y
    pass<T>(in, bufA, mx, nx, mx, 1, 1, nx, mx, (long)ny * nx, (long)ny * mx, ny, (long)nf * nz, true, false, st, 0,
            fm);
    yfwd(syf, fm);
    zfused(sz, fm);
    yinv(syi, fm);
    // x inverse: keep nx
    pass<T>(bufA, out, mx, mx, nx, 1, 1, mx, nx, (long)ny * mx, (long)ny * nx, ny, (long)nf * nz, true, true, st, 0,
            fm);
}

// out may alias in.  nf fields [nf][nl_z][nl_y][nl_x]: mode 0 each with G;
// mode 1 consecutive triples (J_x, J_y, J_z) to grad G x J (nf % 3 == 0).
// bufA / bufB hold nf fields of their pass layouts.
template <typename T>
void fft_convolve(const GridView &g, const cx<T> *spec, int64_t spec_stride, int fps, int nspec, int nf, int mode,
                  const cx<T> *in, cx<T> *out, cx<T> *bufA, cx<T> *bufB, hipStream_t st) {
    SIE_CHECK(nf >= 1 && (mode == 0 || nf % 3 == 0), SIE_EINVAL, "grad-G convolution needs field triples");
    const bool single = fps >= nf || nspec <= 1;      // one spectrum for every field
    SIE_CHECK(single || (fps >= 1 && nf % fps == 0 && (mode == 0 || fps % 3 == 0)), SIE_EINVAL,
              "fields must form whole spectrum runs");
    const int nx = g.nl[0], ny = g.nl[1], nz = g.nl[2];
    const int mx = g.m[0], my = g.m[1];
    const int unit = single ? (mode == 1 ? 3 : 1) : fps;   // chunks hold whole runs
    const int chunk = std::max(unit, (65535 / nz) / unit * unit);
    SIE_CHECK((long)chunk * nz <= 65535, SIE_EGRID, "live box too deep for one FFT batch");
    const long flive = (long)nx * ny * nz, fa = (long)nz * ny * mx, fb = (long)nz * my * mx;
    // fields of inactive objects (one right-hand side) are left out
    FieldMask fm;
    if (g.active) {
        fm.active = g.active;
        fm.obj0 = g.obj0;
        fm.fps = std::max(1, fps);
        fm.nslot = std::max(1, g.nslot);
        fm.nzb = nz;
    }
    for (int f0 = 0; f0 < nf; f0 += chunk) {
        const int c = std::min(chunk, nf - f0);
        fm.f0 = f0;
        convolve_chunk<T>(g, spec, (long)spec_stride, single ? c : fps, single ? 0 : f0 / fps, single ? 1 : nspec, c,
                          mode, in + f0 * flive, out + f0 * flive, bufA + f0 * fa, bufB + f0 * fb, st, fm);
    }
}

// Full (unpruned) forward 3D FFT of a [mz][my][mx] complex128 volume in place,
// using `tmp` of the same size (spectrum construction).
void fft3d_full_fwd(c128 *vol, c128 *tmp, int mx, int my, int mz, hipStream_t st) {
    auto full = [&](const c128 *in, c128 *out, int L, long s, long js, long bs, int nj, long nb, bool contiguous) {
        SIE_CHECK((L & (L - 1)) == 0, SIE_EGRID, "FFT length must be a power of two");
        pass_lg<double, false, false>(ilog2(L), in, out, L, L, s, s, js, js, bs, bs, nj, nb, contiguous, st);
    };
    full(vol, tmp, mx, 1, mx, (long)my * mx, my, mz, true);
    full(tmp, vol, my, mx, 1, (long)my * mx, mx, mz, false);
    // z: lines along z with stride my*mx; treat (y) as batch, j = x
    full(vol, tmp, mz, (long)my * mx, 1, mx, mx, my, false);
    SIE_HIP(hipMemcpyAsync(vol, tmp, sizeof(c128) * (size_t)mx * my * mz, hipMemcpyDeviceToDevice, st));
}

template void fft_convolve<float>(const GridView &, const c64 *, int64_t, int, int, int, int, const c64 *, c64 *,
                                  c64 *, c64 *, hipStream_t);
template void fft_convolve<double>(const GridView &, const c128 *, int64_t, int, int, int, int, const c128 *, c128 *,
                                   c128 *, c128 *, hipStream_t);

}  // namespace sie
