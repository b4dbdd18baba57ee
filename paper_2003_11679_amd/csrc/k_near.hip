// Near region of the AIM (Sec. III-D-1): triangle pairs whose stencil
// centres are within R cells (Chebyshev), their direct Galerkin integrals in
// FP64 (near entries "computed accurately with direct integration") minus the
// grid's own contribution (precorrection, eq. LinNRP / KinNRP), assembled per
// RWG pair into one CSR pattern; and the grid Green's function samples and
// spectra used by the convolution.
//
// Direct integrals of a pair (t, s), observation r on t, source r' on s:
//   S(r) = int_s G,  V(r) = int_s G r',  Gv(r) = int_s grad_r G
// with G = exp(-jkR)/(4 pi R) split into 1/(4 pi R), integrated in closed form
// (Wilton et al. 1984; Graglia 1993), plus a bounded remainder integrated by
// quadrature.  With f_e = c_e (r - p_e) on t and f_f = c_f (r' - p_f) on s and
// W the outer weights:
//   A[e][f]   = c_e c_f [sum W r.V - p_f . sum W S r - p_e . sum W V + p_e.p_f sum W S]
//   Phi[e][f] = 4 c_e c_f sum W S
//   K[e][f]   = c_e c_f [(p_f - p_e) . sum W (Gv x r) + (sum W Gv) . (p_f x p_e)]
// (the K inner integral reduces to Gv x (r - p_f) because grad_r G is parallel
// to r - r').
#include "common.h"
#include "kernels.h"

namespace sie {

// ----------------------------------------------------------------- near pairs
// Skin-depth cutoff (Sec. V): with dc > 0 a pair is kept only if its
// centroids are at most dc + rho_t + rho_s apart (rho: a triangle's bounding
// radius about its centroid), the squares compared without contraction so
// that the decision does not depend on fused rounding.
__device__ __forceinline__ bool within_cutoff(const NearCut &c, int64_t t, int64_t s) {
    if (!(c.dc > 0.0)) return true;
    const int64_t gt = c.tris[t], gs = c.tris[s];
    const double dx = __dsub_rn(c.centroid[3 * gt], c.centroid[3 * gs]);
    const double dy = __dsub_rn(c.centroid[3 * gt + 1], c.centroid[3 * gs + 1]);
    const double dz = __dsub_rn(c.centroid[3 * gt + 2], c.centroid[3 * gs + 2]);
    const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    const double lim = __dadd_rn(__dadd_rn(c.dc, c.rho[gt]), c.rho[gs]);
    return d2 <= __dmul_rn(lim, lim);
}

__global__ void k_near_count(const int32_t *__restrict__ centre, int64_t ntg, const int32_t *__restrict__ cell_ptr,
                             int lox, int loy, int loz, int nlx, int nly, int nlz, int R, NearCut cut,
                             int64_t *__restrict__ count) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= ntg) return;
    const int cx_ = centre[3 * t] - lox, cy = centre[3 * t + 1] - loy, cz = centre[3 * t + 2] - loz;
    const int x0 = max(cx_ - R, 0), x1 = min(cx_ + R, nlx - 1);
    int64_t n = 0;
    for (int z = max(cz - R, 0); z <= min(cz + R, nlz - 1); ++z)
        for (int y = max(cy - R, 0); y <= min(cy + R, nly - 1); ++y) {
            const int64_t base = ((int64_t)z * nly + y) * nlx;
            if (cut.dc > 0.0) {
                for (int32_t s = cell_ptr[base + x0]; s < cell_ptr[base + x1 + 1]; ++s) n += within_cutoff(cut, t, s);
            } else {
                n += cell_ptr[base + x1 + 1] - cell_ptr[base + x0];
            }
        }
    count[t] = n;
}

__global__ void k_near_emit(const int32_t *__restrict__ centre, int64_t ntg, const int32_t *__restrict__ cell_ptr,
                            int lox, int loy, int loz, int nlx, int nly, int nlz, int R, NearCut cut,
                            const int64_t *__restrict__ pair_ptr, int32_t *__restrict__ pair_s) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= ntg) return;
    const int cx_ = centre[3 * t] - lox, cy = centre[3 * t + 1] - loy, cz = centre[3 * t + 2] - loz;
    const int x0 = max(cx_ - R, 0), x1 = min(cx_ + R, nlx - 1);
    int64_t o = pair_ptr[t];
    for (int z = max(cz - R, 0); z <= min(cz + R, nlz - 1); ++z)
        for (int y = max(cy - R, 0); y <= min(cy + R, nly - 1); ++y) {
            const int64_t base = ((int64_t)z * nly + y) * nlx;
            for (int32_t s = cell_ptr[base + x0]; s < cell_ptr[base + x1 + 1]; ++s)
                if (within_cutoff(cut, t, s)) pair_s[o++] = s;
        }
}

void launch_near_count(const int32_t *centre, int64_t ntg, const int32_t *cell_ptr, const NearCut &cut,
                       const int lo[3], const int nl[3], int R, int64_t *count, hipStream_t st) {
    if (!ntg) return;
    hipLaunchKernelGGL(k_near_count, dim3((unsigned)((ntg + 255) / 256)), dim3(256), 0, st, centre, ntg, cell_ptr,
                       lo[0], lo[1], lo[2], nl[0], nl[1], nl[2], R, cut, count);
    SIE_HIP(hipGetLastError());
}

void launch_near_emit(const int32_t *centre, int64_t ntg, const int32_t *cell_ptr, const NearCut &cut,
                      const int lo[3], const int nl[3], int R, const int64_t *pair_ptr, int32_t *pair_s,
                      hipStream_t st) {
    if (!ntg) return;
    hipLaunchKernelGGL(k_near_emit, dim3((unsigned)((ntg + 255) / 256)), dim3(256), 0, st, centre, ntg, cell_ptr,
                       lo[0], lo[1], lo[2], nl[0], nl[1], nl[2], R, cut, pair_ptr, pair_s);
    SIE_HIP(hipGetLastError());
}

// ----------------------------------------------------------------- RWG pattern
// One block per RWG row: mark the columns of all near pairs of the row's two
// triangles in an LDS bitmap over the grid's RWG range, then count (pass 0)
// or write them in ascending order (pass 1).
__global__ void k_rwg_pattern(int64_t nrow, int64_t rwg0, int64_t nbits, const int32_t *__restrict__ rwg_loc,
                              const int64_t *__restrict__ pair_ptr, const int32_t *__restrict__ pair_s,
                              const int32_t *__restrict__ tris, const int32_t *__restrict__ tri_rwg,
                              int64_t *__restrict__ row_len, const int64_t *__restrict__ row_ptr,
                              int32_t *__restrict__ cols, int pass) {
    extern __shared__ unsigned int bits[];
    __shared__ int64_t part[256];
    const int64_t r = blockIdx.x;
    if (r >= nrow) return;
    const int nw = (int)((nbits + 31) / 32);
    for (int i = threadIdx.x; i < nw; i += blockDim.x) bits[i] = 0u;
    __syncthreads();
    for (int side = 0; side < 2; ++side) {
        const int64_t tl = rwg_loc[2 * r + side] >> 2;
        for (int64_t k = pair_ptr[tl] + threadIdx.x; k < pair_ptr[tl + 1]; k += blockDim.x) {
            const int64_t g = tris[pair_s[k]];
            for (int e = 0; e < 3; ++e) {
                const int64_t b = (int64_t)tri_rwg[3 * g + e] - rwg0;
                atomicOr(&bits[b >> 5], 1u << (b & 31));
            }
        }
    }
    __syncthreads();
    // each thread owns a contiguous chunk of words
    const int chunk = (nw + blockDim.x - 1) / blockDim.x;
    const int w0 = threadIdx.x * chunk, w1 = min(nw, w0 + chunk);
    int64_t mine = 0;
    for (int w = w0; w < w1; ++w) mine += __popc(bits[w]);
    part[threadIdx.x] = mine;
    __syncthreads();
    if (pass == 0) {
        if (threadIdx.x == 0) {
            int64_t s = 0;
            for (int i = 0; i < (int)blockDim.x; ++i) s += part[i];
            row_len[r] = s;
        }
        return;
    }
    // exclusive scan of part (small, serial per thread over predecessors)
    int64_t off = 0;
    for (int i = 0; i < (int)threadIdx.x; ++i) off += part[i];
    int64_t o = row_ptr[r] + off;
    for (int w = w0; w < w1; ++w) {
        unsigned int v = bits[w];
        while (v) {
            const int b = __ffs(v) - 1;
            v &= v - 1;
            cols[o++] = (int32_t)(rwg0 + (int64_t)w * 32 + b);
        }
    }
}

void launch_rwg_pattern(int64_t nrow, int64_t rwg0, int64_t nbits, const int32_t *rwg_loc, const int64_t *pair_ptr,
                         const int32_t *pair_s, const int32_t *tris, const int32_t *tri_rwg, int64_t *row_len,
                         const int64_t *row_ptr, int32_t *cols, int pass, hipStream_t st) {
    if (!nrow) return;
    const size_t sh = ((nbits + 31) / 32) * sizeof(unsigned int);
    SIE_CHECK(sh <= 96 * 1024, SIE_EINVAL, "RWG range of a grid too large for the pattern builder");
    hipLaunchKernelGGL(k_rwg_pattern, dim3((unsigned)nrow), dim3(256), sh, st, nrow, rwg0, nbits, rwg_loc, pair_ptr,
                       pair_s, tris, tri_rwg, row_len, row_ptr, cols, pass);
    SIE_HIP(hipGetLastError());
}

// ----------------------------------------------------------------- direct integrals
struct V3 { double x, y, z; };
__device__ inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
__device__ inline double len(V3 a) { return sqrt(dot(a, a)); }

struct CV3 { c128 x, y, z; };
__device__ inline CV3 cscale(c128 s, V3 a) { return {a.x * s, a.y * s, a.z * s}; }
__device__ inline void cadd(CV3 &a, CV3 b) { a.x += b.x; a.y += b.y; a.z += b.z; }
__device__ inline c128 cdot(V3 a, CV3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline CV3 ccross_cv(CV3 a, V3 b) {   // a x b
    return {b.z * a.y - b.y * a.z, b.x * a.z - b.z * a.x, b.y * a.x - b.x * a.y};
}

// ln((R+ + l+)/(R- + l-)) free of cancellation for any foot-point position.
__device__ inline double logratio(double lp, double lm, double Rp, double Rm, double R02) {
    if (lm >= 0.0) return log((Rp + lp) / (Rm + lm));
    if (lp <= 0.0) return log((Rm - lm) / (Rp - lp));
    return log((Rp + lp) * (Rm - lm)) - log(R02);
}

struct SrcTri {
    V3 v[3];
    V3 n;
    V3 lh[3], mh[3];
    double A, e01;
};

// Static potentials of source triangle st at r: I = int 1/R,
// Irho = int (rho' - rho)/R, gI = grad_r int 1/R; d snapped to 0 in-plane.
__device__ inline void static_potentials(const SrcTri &st, V3 r, double &I, V3 &Irho, V3 &gI, double &d) {
    d = dot(r - st.v[0], st.n);
    if (fabs(d) <= 1e-10 * st.e01) d = 0.0;
    const double ad = fabs(d);
    double sI = 0.0, sb = 0.0;
    Irho = {0, 0, 0};
    gI = {0, 0, 0};
    for (int i = 0; i < 3; ++i) {
        const V3 a = st.v[i], b = st.v[(i + 1) % 3];
        const V3 bm = b - r, am = a - r;
        const double lp = dot(bm, st.lh[i]), lm = dot(am, st.lh[i]), t = dot(am, st.mh[i]);
        const double Rp = len(bm), Rm = len(am);
        const double R02 = t * t + d * d;
        const bool online = R02 <= 1e-30 * (lp * lp + lm * lm + 1e-300);
        const double f = logratio(lp, lm, Rp, Rm, R02);
        double beta = 0.0;
        if (!online) {
            beta = atan2(t * lp, R02 + ad * Rp) - atan2(t * lm, R02 + ad * Rm);
            sI += t * f;
        }
        sb += beta;
        const double coef = (online ? 0.0 : R02 * f) + lp * Rp - lm * Rm;
        Irho = Irho + (0.5 * coef) * st.mh[i];
        gI = gI - f * st.mh[i];
    }
    I = sI - ad * sb;
    const double sg = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
    gI = gI - (sg * sb) * st.n;
}

__device__ inline c128 cexp_mjk(c128 k, double R) {   // exp(-j k R)
    const double mag = exp(k.im * R);
    double s, c;
    sincos(k.re * R, &s, &c);
    return {mag * c, -mag * s};
}

// ---------------------------------------------------------------- strong loss
// When the medium's field decays within a small fraction of a triangle
// (|Im k| l > 2 for the source triangle's longest edge l, |Im k| >= 0.38 |k|),
// the static extraction cancels to far below its parts and the remainder
// rule fails (distant pairs keep its quadrature error in place of an
// exponentially small value).  Every pair then integrates in polar coordinates
// about the projection rho0 of the observation point: the triangle is the
// signed sum of the triangles (rho0, edge), swept by the angle theta with
// direction u(theta), edge distance rho(theta), Re = sqrt(rho^2 + d^2):
//   S    = sum int dtheta [exp(-jk|d|) - exp(-jk Re)] / (4 pi jk)
//   V    = rho0 S + sum int dtheta u IV(rho),   IV = int_0^rho G rp^2 drp
//   Gv.n = sum int dtheta [d exp(-jk Re)/Re - sign(d) exp(-jk|d|)] / (4 pi)
//   Gv_t = -sum int dtheta u J(rho),  J = IT - (ln(rho + Re) - rho/Re - ln|d|)/(4 pi)
// with IT the radial integral of the gradient kernel's remainder
// [1 - (1 + jkR) exp(-jkR)] rp^2/(4 pi R^3).  In the plane (d = 0) the ln|d|
// term diverges and drops out: it is theta-independent and the signed sum of
// int u dtheta vanishes for in-plane points, which never lie on the
// triangle's boundary (off the plane they can: points of a face at right
// angles project onto the shared edge, so there it is kept).  The
// radial integrals use Gauss-Legendre on intervals graded in 1/|k| up to the
// cut 64/|k|, beyond which IV and J are constant and their angular integrals
// closed-form; the angle uses composite Gauss-Legendre, broken where rho
// crosses a radial breakpoint.
constexpr int kPolarNB = 14, kPolarNG = 8;
__constant__ double kPolarB[kPolarNB] = {0.25, 0.5, 1.0, 2.0, 3.0, 4.0, 6.0, 8.0, 12.0, 16.0, 24.0, 32.0, 48.0, 64.0};
constexpr double kPolarKL = 2.0, kPolarLoss = 0.38;

__device__ inline void polar_radial(c128 k, double d, double lo, double hi, const double *gx, const double *gw,
                                    c128 &IV, c128 &IT) {
    const double h = 0.5 * (hi - lo), c = 0.5 * (hi + lo);
    for (int g = 0; g < kPolarNG; ++g) {
        const double rp = c + h * gx[g];
        const double R = sqrt(rp * rp + d * d);
        const c128 e = cexp_mjk(k, R);
        const double w = h * gw[g] * rp * rp / (4.0 * M_PI * R);
        IV += w * e;
        const c128 opjkR(1.0 - k.im * R, k.re * R);          // 1 + j k R
        IT += (w / (R * R)) * (c128(1.0) - opjkR * e);
    }
}

__device__ void polar_potentials(const SrcTri &st, V3 r, c128 k, const double *gl, c128 &S, CV3 &V, CV3 &Gv) {
    const double *gx = gl, *gw = gl + kPolarNG;
    const double inv4pi = 1.0 / (4.0 * M_PI);
    double d = dot(r - st.v[0], st.n);
    if (fabs(d) <= 1e-10 * st.e01) d = 0.0;
    const double ad = fabs(d), sgd = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
    const V3 rho0 = r - d * st.n;
    const double u = 1.0 / hypot(k.re, k.im);
    double b[kPolarNB];
    c128 CV[kPolarNB], CT[kPolarNB];
    {
        c128 iv, it;
        double lo = 0.0;
        for (int j = 0; j < kPolarNB; ++j) {
            b[j] = kPolarB[j] * u;
            polar_radial(k, d, lo, b[j], gx, gw, iv, it);
            CV[j] = iv;
            CT[j] = it;
            lo = b[j];
        }
    }
    const double rc = b[kPolarNB - 1], Rc = sqrt(rc * rc + d * d);
    const c128 Vc = CV[kPolarNB - 1];
    const double gref = ad > 0.0 ? log(ad) : 0.0;
    const c128 Jc = CT[kPolarNB - 1] - c128(inv4pi * (log(rc + Rc) - rc / Rc - gref));
    const c128 ekd = cexp_mjk(k, ad);
    c128 sumS, sumN;
    CV3 UV = {}, UJ = {};
    double tot = 0.0;
    for (int i = 0; i < 3; ++i) {
        const V3 a = st.v[i], bb = st.v[(i + 1) % 3];
        const double ll = len(bb - a);
        const V3 lh = st.lh[i], mh = st.mh[i];
        const V3 am = a - rho0, bm = bb - rho0;
        const double t = dot(am, mh), sa = dot(am, lh), sb = dot(bm, lh);
        if (fabs(t) <= 1e-12 * ll) continue;
        const double at = fabs(t), sg = t > 0.0 ? 1.0 : -1.0;
        const double tha = atan(sa / at), thb = atan(sb / at);
        tot += sg * (thb - tha);
        double bp[2 * kPolarNB + 2];
        int nbp = 0;
        bp[nbp++] = tha;
        for (int j = 0; j < kPolarNB; ++j) {
            if (b[j] <= at) continue;
            const double ph = acos(at / b[j]);
            if (-ph > tha && -ph < thb) bp[nbp++] = -ph;
            if (ph > tha && ph < thb) bp[nbp++] = ph;
        }
        bp[nbp++] = thb;
        for (int x = 1; x < nbp; ++x)
            for (int y = x; y > 0 && bp[y - 1] > bp[y]; --y) {
                const double q = bp[y];
                bp[y] = bp[y - 1];
                bp[y - 1] = q;
            }
        for (int q = 0; q + 1 < nbp; ++q) {
            const double t1 = bp[q], t2 = bp[q + 1];
            const double h = 0.5 * (t2 - t1), c = 0.5 * (t2 + t1);
            if (h <= 0.0) continue;
            if (at / cos(c) >= rc) {
                const V3 U = sg * ((sg * (sin(t2) - sin(t1))) * mh - (cos(t2) - cos(t1)) * lh);
                cadd(UV, cscale(Vc, U));
                cadd(UJ, cscale(Jc, U));
                continue;
            }
            for (int g = 0; g < kPolarNG; ++g) {
                const double th = c + h * gx[g];
                const double wt = sg * h * gw[g];
                const double ct = cos(th), sn = sin(th);
                const double rho = at / ct, Re = sqrt(rho * rho + d * d);
                const V3 uh = (sg * ct) * mh + sn * lh;
                int j = -1;
                while (j + 1 < kPolarNB && b[j + 1] <= rho) ++j;
                c128 IV = j >= 0 ? CV[j] : c128(), IT = j >= 0 ? CT[j] : c128();
                polar_radial(k, d, j >= 0 ? b[j] : 0.0, rho, gx, gw, IV, IT);
                const c128 J = IT - c128(inv4pi * (log(rho + Re) - rho / Re - gref));
                const c128 eR = cexp_mjk(k, Re);
                sumS += wt * eR;
                sumN += (wt * d / Re) * eR;
                cadd(UV, cscale(wt * IV, uh));
                cadd(UJ, cscale(wt * J, uh));
            }
        }
    }
    const c128 ijk = cdiv(c128(1.0), c128(-k.im, k.re));   // 1/(j k)
    S = (tot * ekd - sumS) * inv4pi * ijk;
    const c128 nrm = inv4pi * (sumN - (sgd * tot) * ekd);
    const CV3 sr = cscale(S, rho0), nn = cscale(nrm, st.n);
    V = {sr.x + UV.x, sr.y + UV.y, sr.z + UV.z};
    Gv = {nn.x - UJ.x, nn.y - UJ.y, nn.z - UJ.z};
}

__device__ inline int rule_index_outer(int kind, int loc) {
    // 0 self, 1..3 edge(opp), 4..6 vertex(vtx), 7 close, 8 far
    if (kind == KIND_SELF) return 0;
    if (kind == KIND_EDGE) return 1 + loc;
    if (kind == KIND_VERTEX) return 4 + loc;
    return kind == KIND_CLOSE ? 7 : 8;
}
__device__ inline int rule_index_inner(int kind) {
    return kind <= KIND_VERTEX ? 9 : (kind == KIND_CLOSE ? 10 : 11);
}

// Classification of a pair: self / edge-adjacent / vertex-adjacent by shared
// vertices, else close (centroid distance < CLOSE_FACTOR x longest edge) or far.
// loc: local vertex of t opposite the shared edge (edge) or shared (vertex).
__device__ inline int classify(const NearFillArgs &a, int64_t tg, int64_t sg, int &loc) {
    int vt[3], vs[3];
    for (int i = 0; i < 3; ++i) { vt[i] = a.tri[3 * tg + i]; vs[i] = a.tri[3 * sg + i]; }
    int nshared = 0, shared_mask = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (vt[i] == vs[j]) { ++nshared; shared_mask |= 1 << i; }
    loc = 0;
    if (nshared == 3) return KIND_SELF;
    if (nshared == 2) { const int m = ~shared_mask & 7; loc = m == 1 ? 0 : (m == 2 ? 1 : 2); return KIND_EDGE; }
    if (nshared == 1) { loc = shared_mask == 1 ? 0 : (shared_mask == 2 ? 1 : 2); return KIND_VERTEX; }
    const V3 o = {a.centroid[3 * tg], a.centroid[3 * tg + 1], a.centroid[3 * tg + 2]};
    V3 pt[3], ps[3];
    for (int i = 0; i < 3; ++i) {
        pt[i] = V3{a.xyz[3 * (int64_t)vt[i]], a.xyz[3 * (int64_t)vt[i] + 1], a.xyz[3 * (int64_t)vt[i] + 2]} - o;
        ps[i] = V3{a.xyz[3 * (int64_t)vs[i]], a.xyz[3 * (int64_t)vs[i] + 1], a.xyz[3 * (int64_t)vs[i] + 2]} - o;
    }
    double hmax = 0.0;
    for (int i = 0; i < 3; ++i) {
        hmax = fmax(hmax, len(pt[(i + 1) % 3] - pt[(i + 2) % 3]));
        hmax = fmax(hmax, len(ps[(i + 1) % 3] - ps[(i + 2) % 3]));
    }
    const V3 cs = V3{a.centroid[3 * sg], a.centroid[3 * sg + 1], a.centroid[3 * sg + 2]} - o;
    return len(cs) < CLOSE_FACTOR * hmax ? KIND_CLOSE : KIND_FAR;
}

// Direct integrals of pair (tl, sl) minus its grid contribution; writes the
// L, K and direct-L 3x3 blocks of pair slot p.  The grid contribution reads
// the test-node sums of tl from a.ptab (k_precorr_table); gr: radial tables
// in LDS, gr[2 q] = G(h sqrt(q)), gr[2 q + 1] = -(1 + j k r) exp(-j k r)/(4 pi
// r^3) at r = h sqrt(q), q = |d|^2 (0 at q = 0).
// G > 1: G consecutive lanes (aligned, in one wavefront, all active) share
// the pair; lane sub of the group takes the outer points sub, sub + G, ...,
// the group's partial sums are added by butterfly exchanges, and lane 0
// finishes the pair alone.
__device__ inline void group_sum(c128 &v, int G) {
    for (int off = G >> 1; off > 0; off >>= 1) {
        v.re += __shfl_xor(v.re, off, 64);
        v.im += __shfl_xor(v.im, off, 64);
    }
}
__device__ inline void group_sum(CV3 &v, int G) {
    group_sum(v.x, G);
    group_sum(v.y, G);
    group_sum(v.z, G);
}

template <bool POLAR, int G = 1>
__device__ void fill_pair(const NearFillArgs &a, int64_t tl, int64_t sl, int64_t p, int kind, int loc,
                          const c128 *gr, int sub = 0) {
    const int64_t tg = a.tris[tl], sg = a.tris[sl];
    const V3 o = {a.centroid[3 * tg], a.centroid[3 * tg + 1], a.centroid[3 * tg + 2]};
    V3 pt[3], ps[3];
    for (int i = 0; i < 3; ++i) {
        const int64_t vt = a.tri[3 * tg + i], vs = a.tri[3 * sg + i];
        pt[i] = V3{a.xyz[3 * vt], a.xyz[3 * vt + 1], a.xyz[3 * vt + 2]} - o;
        ps[i] = V3{a.xyz[3 * vs], a.xyz[3 * vs + 1], a.xyz[3 * vs + 2]} - o;
    }
    // source triangle geometry
    SrcTri st;
    for (int i = 0; i < 3; ++i) st.v[i] = ps[i];
    {
        const V3 e1 = ps[1] - ps[0], e2 = ps[2] - ps[0];
        const V3 c = cross(e1, e2);
        const double nn = len(c);
        st.n = (1.0 / nn) * c;
        st.A = 0.5 * nn;
        st.e01 = len(e1);
        for (int i = 0; i < 3; ++i) {
            const V3 le = ps[(i + 1) % 3] - ps[i];
            st.lh[i] = (1.0 / len(le)) * le;
            st.mh[i] = cross(st.lh[i], st.n);
        }
    }
    const double At = 0.5 * len(cross(pt[1] - pt[0], pt[2] - pt[0]));
    const c128 k = a.k;
    const double inv4pi = 0.07957747154594767;   // 1/(4 pi)
    const int ro = rule_index_outer(kind, loc), ri = rule_index_inner(kind);
    const double *Ro = a.rules + 4 * a.rule_off[ro];
    const double *Ri = a.rules + 4 * a.rule_off[ri];
    const int no = a.rule_n[ro], ni = a.rule_n[ri];
    double lmax = 0.0;
    for (int i = 0; i < 3; ++i) lmax = fmax(lmax, len(ps[(i + 1) % 3] - ps[i]));
    const bool polar = POLAR && a.polar && fabs(k.im) * lmax > kPolarKL;

    c128 aRV, aS;
    CV3 aV = {}, aSR = {}, aGR = {}, aG = {};
    for (int qo = sub; qo < no; qo += G) {
        const V3 r = Ro[4 * qo] * pt[0] + Ro[4 * qo + 1] * pt[1] + Ro[4 * qo + 2] * pt[2];
        const double W = Ro[4 * qo + 3] * At;
        c128 S;
        CV3 V, Gv;
        if (polar) {
            polar_potentials(st, r, k, a.polar_gl, S, V, Gv);
        } else {
        double I0, d;
        V3 Irho, gI;
        static_potentials(st, r, I0, Irho, gI, d);
        const V3 rho = r - d * st.n;
        S = c128(I0 * inv4pi, 0.0);
        V = {c128((Irho.x + rho.x * I0) * inv4pi), c128((Irho.y + rho.y * I0) * inv4pi),
             c128((Irho.z + rho.z * I0) * inv4pi)};
        Gv = {c128(gI.x * inv4pi), c128(gI.y * inv4pi), c128(gI.z * inv4pi)};
        for (int qi = 0; qi < ni; ++qi) {
            const V3 rp = Ri[4 * qi] * ps[0] + Ri[4 * qi + 1] * ps[1] + Ri[4 * qi + 2] * ps[2];
            const double wA = Ri[4 * qi + 3] * st.A;
            const V3 df = r - rp;
            const double R = len(df);
            c128 rem, hg;
            if (R == 0.0) {
                rem = c128(k.im * inv4pi, -k.re * inv4pi);      // -j k /(4 pi)
            } else {
                const c128 ez = cexp_mjk(k, R);
                const c128 z(k.im * R, -k.re * R);               // z = -j k R
                rem = (inv4pi / R) * (ez - c128(1.0));
                const c128 one_mz(1.0 - z.re, -z.im);
                hg = (inv4pi / (R * R * R)) * (c128(1.0) - one_mz * ez);
            }
            S += wA * rem;
            cadd(V, cscale(wA * rem, rp));
            cadd(Gv, cscale(wA * hg, df));
        }
        }
        aRV += W * cdot(r, V);
        aS += W * S;
        cadd(aV, CV3{W * V.x, W * V.y, W * V.z});
        cadd(aSR, cscale(W * S, r));
        const CV3 gxr = ccross_cv(Gv, r);   // Gv x r
        cadd(aGR, CV3{W * gxr.x, W * gxr.y, W * gxr.z});
        cadd(aG, CV3{W * Gv.x, W * Gv.y, W * Gv.z});
    }
    if (G > 1) {
        group_sum(aRV, G);
        group_sum(aS, G);
        group_sum(aV, G);
        group_sum(aSR, G);
        group_sum(aGR, G);
        group_sum(aG, G);
        if (sub != 0) return;
    }

    // precorrection: grid contribution of the pair over the 27 x 27 stencil
    // node pairs, offsets d = (c_t + o_a) - (c_s + o_b); none for a medium
    // without grid part (its near values are the direct integrals)
    c128 S00, S11, C11;
    CV3 S10 = {}, S01 = {}, Vs = {}, Vt = {}, U = {};
    if (!a.no_grid) {
    const int dx0 = a.centre[3 * tl] - a.centre[3 * sl];
    const int dy0 = a.centre[3 * tl + 1] - a.centre[3 * sl + 1];
    const int dz0 = a.centre[3 * tl + 2] - a.centre[3 * sl + 2];
    // The sums over node pairs factor through the source node b: for each b
    // the test-node sums at offset e = (c_t - c_s) - o_b (from the row's
    // table) Gb0 = sum_a m0t G, Gb1 = sum_a m1t G, gb0 = sum_a m0t g and
    // gb1x = sum_a g x m1t, then
    //   S00 += m0s Gb0, S01 += m1s Gb0, S10 += m0s Gb1, S11 += m1s . Gb1,
    //   U += m0s gb0, Vs += gb0 x m1s, Vt -= m0s gb1x, C11 -= m1s . gb1x
    // (g . (m1s x m1t) = -m1s . (g x m1t)).
    const int W = a.tab_w, S = 2 * W + 1;
    const c128 *tt = a.ptab + (tl - a.tab_row0) * (int64_t)(S * S * S) * 10;
    const double *ms = a.mom + sl * 27 * 4;
    for (int ib = 0; ib < 27; ++ib) {
        const int bx = ib % 3 - 1, by = (ib / 3) % 3 - 1, bz = ib / 9 - 1;
        // near pairs lie within the near radius per axis, so |e| <= W; the
        // clamps only keep the read inside the table
        const int ex = min(max(dx0 - bx, -W), W), ey = min(max(dy0 - by, -W), W), ez = min(max(dz0 - bz, -W), W);
        const c128 *te = tt + ((int64_t)((ez + W) * S + (ey + W)) * S + (ex + W)) * 10;
        const c128 Gb0 = te[0];
        const CV3 Gb1 = {te[1], te[2], te[3]}, gb0 = {te[4], te[5], te[6]}, gb1x = {te[7], te[8], te[9]};
        const double m0s = ms[4 * ib];
        const V3 m1s = {ms[4 * ib + 1], ms[4 * ib + 2], ms[4 * ib + 3]};
        S00 += m0s * Gb0;
        cadd(S01, cscale(Gb0, m1s));
        cadd(S10, CV3{m0s * Gb1.x, m0s * Gb1.y, m0s * Gb1.z});
        S11 += cdot(m1s, Gb1);
        cadd(U, CV3{m0s * gb0.x, m0s * gb0.y, m0s * gb0.z});
        cadd(Vs, ccross_cv(gb0, m1s));
        cadd(Vt, CV3{-m0s * gb1x.x, -m0s * gb1x.y, -m0s * gb1x.z});
        C11 += -cdot(m1s, gb1x);
    }
    }
    const c128 ik2 = cdiv(c128(1.0), k * k);
    const double *ct = a.tri_coef + tl * 12;
    const double *cs = a.tri_coef + sl * 12;
    c128 *out = a.blocks + p * a.bstride;
    const bool aug = a.bstride > 27;
    for (int e = 0; e < 3; ++e) {
        const double ce = ct[4 * e];
        const V3 qe = {ct[4 * e + 1], ct[4 * e + 2], ct[4 * e + 3]};
        const V3 pe = pt[e];
        for (int f = 0; f < 3; ++f) {
            const double cf = cs[4 * f];
            const V3 qf = {cs[4 * f + 1], cs[4 * f + 2], cs[4 * f + 3]};
            const V3 pf = ps[f];
            const double cc = ce * cf;
            const c128 Ad = cc * (aRV - cdot(pf, aSR) - cdot(pe, aV) + dot(pe, pf) * aS);
            const c128 Pd = (4.0 * cc) * aS;
            const c128 Kd = cc * (cdot(pf - pe, aGR) + cdot(cross(pf, pe), aG));
            const c128 Ag = cc * (S11 - cdot(qf, S10) - cdot(qe, S01) + dot(qe, qf) * S00);
            const c128 Pg = (4.0 * cc) * S00;
            const c128 Kg = cc * (C11 - cdot(qe, Vs) - cdot(qf, Vt) + cdot(cross(qf, qe), U));
            out[e * 3 + f] = (Ad - Ag) - ik2 * (Pd - Pg);
            out[9 + e * 3 + f] = Kd - Kg;
            out[18 + e * 3 + f] = Ad - ik2 * Pd;     // direct (unprecorrected) L
            if (aug) {
                out[27 + e * 3 + f] = Ad - Ag;       // precorrected vector potential
                out[36 + e * 3 + f] = Ad;            // direct vector potential
            }
        }
    }
    if (aug) {
        a.gam[p] = aS - S00;                         // pulse integral minus its grid part
        if (tl == sl) a.gself[tg] = aS;
    }
}

// Radial Green's tables for |d|^2 = 0 .. nq-1 (grid offsets in cells).
__global__ void k_green_radial(c128 k, double h, int nq, c128 *gr) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    if (q == 0) { gr[0] = c128(); gr[1] = c128(); return; }
    const double r = h * sqrt((double)q);
    const double inv4pi = 0.07957747154594767;
    const c128 e = cexp_mjk(k, r);
    gr[2 * q] = (inv4pi / r) * e;
    const c128 onejkr(1.0 - k.im * r, k.re * r);
    gr[2 * q + 1] = (-inv4pi / (r * r * r)) * (onejkr * e);
}

__device__ inline void load_radial(const c128 *g, int nq, c128 *lds) {
    for (int i = threadIdx.x; i < 2 * nq; i += blockDim.x) lds[i] = g[i];
}

// kinds[p] = kind | loc << 4 of every pair of row triangle blockIdx.x.
__global__ void k_pair_kinds(NearFillArgs a, int64_t ntg, uint8_t *kinds) {
    const int64_t tl = blockIdx.x;
    if (tl >= ntg) return;
    const int64_t tg = a.tris[tl];
    for (int64_t p = a.pair_ptr[tl] + threadIdx.x; p < a.pair_ptr[tl + 1]; p += blockDim.x) {
        int loc;
        const int kind = classify(a, tg, a.tris[a.pair_s[p]], loc);
        kinds[p] = (uint8_t)(kind | (loc << 4));
    }
}

void launch_pair_kinds(const NearFillArgs &a, uint8_t *kinds, hipStream_t st) {
    if (a.ntg <= 0) return;
    hipLaunchKernelGGL(k_pair_kinds, dim3((unsigned)a.ntg), dim3(128), 0, st, a, a.ntg, kinds);
    SIE_HIP(hipGetLastError());
}

// Pass 0 counts, pass 1 appends, the non-far pairs of each kind (lists[kind]).
// One atomic per wave and kind: the lanes of a kind take consecutive slots
// after the wave's base (ballot and population count).
__global__ void k_near_classify(NearFillArgs a, int64_t ntg, int pass, unsigned long long *counts,
                                int64_t *lists0, int64_t *lists1, int64_t *lists2, int64_t *lists3) {
    const int64_t tl = blockIdx.x;
    if (tl >= ntg) return;
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t p0 = a.pair_ptr[tl], p1 = a.pair_ptr[tl + 1];
    for (int64_t base = p0; base < p1; base += blockDim.x) {   // same trip count for every lane
        const int64_t p = base + threadIdx.x;
        int kind = KIND_FAR, loc = 0;
        if (p < p1) {
            const int b = a.pkind[p];
            kind = b & 15;
            loc = b >> 4;
        }
        for (int kd = 0; kd < 4; ++kd) {
            const unsigned long long m = __ballot(kind == kd);
            if (!m) continue;
            const int leader = __ffsll((long long)m) - 1;
            unsigned long long off = 0;
            if (lane == leader) off = atomicAdd(&counts[kd], (unsigned long long)__popcll(m));
            off = __shfl(off, leader);
            if (pass == 1 && kind == kd) {
                int64_t *L = kd == 0 ? lists0 : (kd == 1 ? lists1 : (kd == 2 ? lists2 : lists3));
                L[off + __popcll(m & below)] = (p << 2) | loc;
            }
        }
    }
}

// Test-node sums of the precorrection (eq. LinNRP / KinNRP) for row triangle
// row0 + blockIdx.x and every offset e in [-W, W]^3 between its stencil centre
// and a source stencil node (W = near radius + 1): with G and g the Green's
// function and its gradient at the node offset e + o_a,
//   [0] sum_a m0t G, [1..3] sum_a G m1t, [4..6] sum_a m0t g, [7..9] sum_a g x m1t
// over the 27 test nodes a.  Every source triangle of the row with the same
// offset reuses them.
__global__ void __launch_bounds__(256) k_precorr_table(NearFillArgs a, int64_t row0, c128 *tab) {
    extern __shared__ unsigned char smem[];
    c128 *gr = reinterpret_cast<c128 *>(smem);
    double *mt = reinterpret_cast<double *>(gr + 2 * a.nq);
    const int64_t tl = row0 + blockIdx.x;
    load_radial(a.gradial, a.nq, gr);
    for (int i = threadIdx.x; i < 108; i += blockDim.x) mt[i] = a.mom[tl * 108 + i];
    __syncthreads();
    const int W = a.tab_w, S = 2 * W + 1, NT = S * S * S;
    const double h = a.h;
    for (int idx = threadIdx.x; idx < NT; idx += blockDim.x) {
        const int ex = idx % S - W, ey = (idx / S) % S - W, ez = idx / (S * S) - W;
        c128 Gb0;
        CV3 Gb1 = {}, gb0 = {}, gb1x = {};
        for (int ia = 0; ia < 27; ++ia) {
            const int ddx = ex + ia % 3 - 1, ddy = ey + (ia / 3) % 3 - 1, ddz = ez + ia / 9 - 1;
            const int q = ddx * ddx + ddy * ddy + ddz * ddz;
            const c128 G = gr[2 * q];
            const c128 sr = gr[2 * q + 1];
            const CV3 g = {(h * ddx) * sr, (h * ddy) * sr, (h * ddz) * sr};
            const double m0t = mt[4 * ia];
            const V3 m1t = {mt[4 * ia + 1], mt[4 * ia + 2], mt[4 * ia + 3]};
            Gb0 += m0t * G;
            cadd(Gb1, cscale(G, m1t));
            cadd(gb0, CV3{m0t * g.x, m0t * g.y, m0t * g.z});
            cadd(gb1x, ccross_cv(g, m1t));
        }
        c128 *o = tab + ((int64_t)blockIdx.x * NT + idx) * 10;
        o[0] = Gb0;
        o[1] = Gb1.x; o[2] = Gb1.y; o[3] = Gb1.z;
        o[4] = gb0.x; o[5] = gb0.y; o[6] = gb0.z;
        o[7] = gb1x.x; o[8] = gb1x.y; o[9] = gb1x.z;
    }
}

void launch_precorr_table(const NearFillArgs &a, int64_t row0, int64_t nrows, c128 *tab, hipStream_t st) {
    if (nrows <= 0) return;
    const size_t sh = 2 * (size_t)a.nq * sizeof(c128) + 108 * sizeof(double);
    hipLaunchKernelGGL(k_precorr_table, dim3((unsigned)nrows), dim3(256), sh, st, a, row0, tab);
    SIE_HIP(hipGetLastError());
}

// Far pairs: one workgroup per row triangle; the radial tables live in LDS.
// POLAR: the strong-loss scheme may apply (its code is left out otherwise,
// which frees registers and scratch for the common case).
template <bool POLAR>
__global__ void __launch_bounds__(128, POLAR ? 1 : 2) k_near_fill_far(NearFillArgs a, int64_t ntg) {
    extern __shared__ unsigned char smem[];
    c128 *gr = reinterpret_cast<c128 *>(smem);
    const int64_t tl = blockIdx.x;
    if (tl >= ntg) return;
    load_radial(a.gradial, a.nq, gr);
    __syncthreads();
    for (int64_t p = a.pair_ptr[tl] + threadIdx.x; p < a.pair_ptr[tl + 1]; p += blockDim.x) {
        const int64_t sl = a.pair_s[p];
        if ((a.pkind[p] & 15) != KIND_FAR) continue;
        fill_pair<POLAR>(a, tl, sl, p, KIND_FAR, 0, gr);
    }
}

// Listed (touching / close) pairs of one kind: G consecutive threads per
// pair (G = 1, 2, 4, 8 or 16).
template <bool POLAR, int G>
__global__ void __launch_bounds__(128, POLAR ? 1 : 2) k_near_fill_list(NearFillArgs a, int64_t ntg, const int64_t *list, int64_t n,
                                                        int kind) {
    extern __shared__ unsigned char smem[];
    c128 *gr = reinterpret_cast<c128 *>(smem);
    load_radial(a.gradial, a.nq, gr);
    __syncthreads();
    const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
    const int sub = (int)(threadIdx.x % G);
    if (i >= n) return;   // uniform over each group
    const int64_t e = list[i];
    const int64_t p = e >> 2;
    const int loc = (int)(e & 3);
    int64_t lo = 0, hi = ntg;   // row: pair_ptr[tl] <= p < pair_ptr[tl + 1]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (a.pair_ptr[mid] <= p) lo = mid; else hi = mid;
    }
    fill_pair<POLAR, G>(a, lo, a.pair_s[p], p, kind, loc, gr, sub);
}

template <bool POLAR, int G>
static void launch_fill_list(const NearFillArgs &a, int64_t ntg, const int64_t *list, int64_t n, int kind,
                             size_t sh, hipStream_t st) {
    const dim3 grid((unsigned)((n * G + 127) / 128));
    hipLaunchKernelGGL((k_near_fill_list<POLAR, G>), grid, dim3(128), sh, st, a, ntg, list, n, kind);
    SIE_HIP(hipGetLastError());
}

// Threads per listed pair: enough for about 64 K threads in the launch, at
// most 16 (the smallest outer rules have 25 points).
template <bool POLAR>
static void launch_fill_list(const NearFillArgs &a, int64_t ntg, const int64_t *list, int64_t n, int kind,
                             size_t sh, hipStream_t st) {
    int G = 1;
    while (G < 16 && n * G < 65536) G <<= 1;
    switch (G) {
        case 1: launch_fill_list<POLAR, 1>(a, ntg, list, n, kind, sh, st); break;
        case 2: launch_fill_list<POLAR, 2>(a, ntg, list, n, kind, sh, st); break;
        case 4: launch_fill_list<POLAR, 4>(a, ntg, list, n, kind, sh, st); break;
        case 8: launch_fill_list<POLAR, 8>(a, ntg, list, n, kind, sh, st); break;
        default: launch_fill_list<POLAR, 16>(a, ntg, list, n, kind, sh, st); break;
    }
}

void launch_green_radial(c128 k, double h, int nq, c128 *gr, hipStream_t st) {
    hipLaunchKernelGGL(k_green_radial, dim3((nq + 255) / 256), dim3(256), 0, st, k, h, nq, gr);
    SIE_HIP(hipGetLastError());
}

void launch_near_fill(const NearFillArgs &a, int64_t npairs, hipStream_t st) {
    if (!npairs) return;
    const int64_t ntg = a.ntg;
    const size_t sh_rad = 2 * (size_t)a.nq * sizeof(c128);
    // classify non-far pairs into per-kind lists
    DBuf<unsigned long long> counts(4);
    SIE_HIP(hipMemsetAsync(counts.p, 0, 4 * sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_near_classify, dim3((unsigned)ntg), dim3(128), 0, st, a, ntg, 0, counts.p, nullptr, nullptr,
                       nullptr, nullptr);
    SIE_HIP(hipGetLastError());
    std::vector<unsigned long long> cnt(4);
    SIE_HIP(hipMemcpyAsync(cnt.data(), counts.p, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    SIE_HIP(hipStreamSynchronize(st));
    DBuf<int64_t> lists[4];
    for (int kd = 0; kd < 4; ++kd) lists[kd].alloc(std::max<unsigned long long>(cnt[kd], 1));
    SIE_HIP(hipMemsetAsync(counts.p, 0, 4 * sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_near_classify, dim3((unsigned)ntg), dim3(128), 0, st, a, ntg, 1, counts.p, lists[0].p,
                       lists[1].p, lists[2].p, lists[3].p);
    SIE_HIP(hipGetLastError());
    // far pairs per row triangle
    if (a.polar) hipLaunchKernelGGL(k_near_fill_far<true>, dim3((unsigned)ntg), dim3(128), sh_rad, st, a, ntg);
    else hipLaunchKernelGGL(k_near_fill_far<false>, dim3((unsigned)ntg), dim3(128), sh_rad, st, a, ntg);
    SIE_HIP(hipGetLastError());
    for (int kd = 0; kd < 4; ++kd) {
        if (!cnt[kd]) continue;
        if (a.polar) launch_fill_list<true>(a, ntg, lists[kd].p, (int64_t)cnt[kd], kd, sh_rad, st);
        else launch_fill_list<false>(a, ntg, lists[kd].p, (int64_t)cnt[kd], kd, sh_rad, st);
    }
    SIE_HIP(hipStreamSynchronize(st));
}

// Deterministic CSR assembly: entry (m, n) sums the blocks of the (at most 4)
// near triangle pairs (T+-(m), T+-(n)).
// One workgroup per RWG row: the pair lists of its two triangles (this
// chunk's) are staged in LDS when they fit and searched there; a row whose
// triangles have no pairs in the chunk returns at once.
constexpr int kGatherLds = 4096;

__global__ __launch_bounds__(256) void k_near_gather(int64_t nrow, int64_t rwg0, const int64_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ cols, const int32_t *__restrict__ rwg_loc,
                                                     const int32_t *__restrict__ glob2loc, const int32_t *__restrict__ tpm,
                                                     const int32_t *__restrict__ epm, const int64_t *__restrict__ pair_ptr,
                                                     const int32_t *__restrict__ pair_s, const c128 *__restrict__ blocks,
                                                     int bstride, c128 *__restrict__ nL64, c128 *__restrict__ nK64,
                                                     c128 *__restrict__ nLd64, c128 *__restrict__ nA64,
                                                     c128 *__restrict__ adiag) {
    __shared__ int32_t ls[2][kGatherLds];
    const int64_t r = blockIdx.x;
    if (r >= nrow) return;
    int64_t b0[2], nn[2];
    int ea[2];
    for (int sa = 0; sa < 2; ++sa) {
        const int32_t lc = rwg_loc[2 * r + sa];
        const int64_t tl = lc >> 2;
        ea[sa] = lc & 3;
        b0[sa] = pair_ptr[tl];
        nn[sa] = pair_ptr[tl + 1] - b0[sa];
    }
    if (nn[0] == 0 && nn[1] == 0) return;   // uniform over the workgroup
    for (int sa = 0; sa < 2; ++sa)
        if (nn[sa] <= kGatherLds)
            for (int64_t i = threadIdx.x; i < nn[sa]; i += blockDim.x) ls[sa][i] = pair_s[b0[sa] + i];
    __syncthreads();
    for (int64_t j = row_ptr[r] + threadIdx.x; j < row_ptr[r + 1]; j += blockDim.x) {
        const int32_t n = cols[j];
        c128 L, K, Ld, A, Ad;
        for (int sa = 0; sa < 2; ++sa) {
            if (nn[sa] == 0) continue;
            const bool inl = nn[sa] <= kGatherLds;
            for (int sb = 0; sb < 2; ++sb) {
                const int32_t sl = glob2loc[tpm[2 * (int64_t)n + sb]];
                if (sl < 0) continue;
                const int eb = epm[2 * (int64_t)n + sb];
                int64_t lo = 0, hi = nn[sa], q = -1;
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    const int32_t v = inl ? ls[sa][mid] : pair_s[b0[sa] + mid];
                    if (v == sl) { q = b0[sa] + mid; break; }
                    if (v < sl) lo = mid + 1; else hi = mid;
                }
                if (q < 0) continue;
                const c128 *bq = blocks + q * bstride + ea[sa] * 3 + eb;
                L += bq[0];
                K += bq[9];
                Ld += bq[18];
                if (nA64) {
                    A += bq[27];
                    Ad += bq[36];
                }
            }
        }
        // row-triangle chunks are processed one after the other: accumulate
        nL64[j] += L;
        nK64[j] += K;
        nLd64[j] += Ld;
        if (nA64) {
            nA64[j] += A;
            if (n == rwg0 + r) adiag[r] += Ad;   // one column of the row is its diagonal
        }
    }
}

void launch_near_gather(int64_t nrow, int64_t rwg0, int64_t max_row, const int64_t *row_ptr, const int32_t *cols,
                         const int32_t *rwg_loc, const int32_t *glob2loc, const int32_t *tpm, const int32_t *epm,
                         const int64_t *pair_ptr, const int32_t *pair_s, const c128 *blocks, int bstride,
                         c128 *nL64, c128 *nK64, c128 *nLd64, c128 *nA64, c128 *adiag, hipStream_t st) {
    if (!nrow || !max_row) return;
    SIE_CHECK(nrow < (1LL << 31), SIE_EINVAL, "too many rows");
    SIE_CHECK(bstride == 27 || (bstride == 45 && nA64 && adiag), SIE_EINVAL, "bad pair block layout");
    hipLaunchKernelGGL(k_near_gather, dim3((unsigned)nrow), dim3(256), 0, st, nrow, rwg0, row_ptr, cols, rwg_loc,
                       glob2loc, tpm, epm, pair_ptr, pair_s, blocks, bstride, nL64, nK64, nLd64,
                       bstride == 45 ? nA64 : nullptr, adiag);
    SIE_HIP(hipGetLastError());
}

// ----------------------------------------------------------------- Green's function tables
__device__ inline void green_at(c128 k, double h, int dx, int dy, int dz, c128 out[4]) {
    const double rx = h * dx, ry = h * dy, rz = h * dz;
    const double r = sqrt(rx * rx + ry * ry + rz * rz);
    if (r == 0.0) { out[0] = out[1] = out[2] = out[3] = c128(); return; }
    const double inv4pi = 0.07957747154594767;
    const c128 e = cexp_mjk(k, r);
    out[0] = (inv4pi / r) * e;
    // grad_r G = r_vec * ( -(1 + j k r) exp(-j k r) / (4 pi r^3) )
    const c128 onejkr(1.0 - k.im * r, k.re * r);
    const c128 s = (-inv4pi / (r * r * r)) * (onejkr * e);
    out[1] = rx * s; out[2] = ry * s; out[3] = rz * s;
}

// Circulant embedding of G (kind 0) or dG/dx_(kind-1) on [mz][my][mx]:
// index i maps to offset i (i < nl) or i - m (i > m - nl); other indices 0.
__global__ void k_green_sample(c128 k, double h, int nlx, int nly, int nlz, int mx, int my, int mz, int kind,
                               c128 *vol) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)mx * my * mz) return;
    const int ix = (int)(i % mx), iy = (int)((i / mx) % my), iz = (int)(i / ((int64_t)mx * my));
    auto off = [](int idx, int nl, int m, bool &ok) {
        if (idx < nl) { ok = true; return idx; }
        if (idx > m - nl) { ok = true; return idx - m; }
        ok = false; return 0;
    };
    bool okx, oky, okz;
    const int dx = off(ix, nlx, mx, okx), dy = off(iy, nly, my, oky), dz = off(iz, nlz, mz, okz);
    c128 g[4];
    if (okx && oky && okz) green_at(k, h, dx, dy, dz, g);
    else g[0] = g[1] = g[2] = g[3] = c128();
    vol[i] = g[kind];
}

void launch_green_sample(c128 k, double h, const int nl[3], const int m[3], int kind, c128 *vol, hipStream_t st) {
    const int64_t n = (int64_t)m[0] * m[1] * m[2];
    hipLaunchKernelGGL(k_green_sample, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, k, h, nl[0], nl[1], nl[2],
                       m[0], m[1], m[2], kind, vol);
    SIE_HIP(hipGetLastError());
}

__global__ void k_fold_octant(const c128 *vol, int mx, int my, int mz, double scale, c128 *s64, c64 *s32) {
    const int ox = mx / 2 + 1, oy = my / 2 + 1, oz = mz / 2 + 1;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)ox * oy * oz) return;
    const int fx = (int)(i % ox), fy = (int)((i / ox) % oy), fz = (int)(i / ((int64_t)ox * oy));
    const c128 v = scale * vol[((int64_t)fz * my + fy) * mx + fx];
    s64[i] = v;
    s32[i] = c64((float)v.re, (float)v.im);
}

void launch_fold_octant(const c128 *vol, const int m[3], int kind, double scale, c128 *spec64, c64 *spec32,
                        hipStream_t st) {
    const int64_t oct = (int64_t)(m[0] / 2 + 1) * (m[1] / 2 + 1) * (m[2] / 2 + 1);
    hipLaunchKernelGGL(k_fold_octant, dim3((unsigned)((oct + 255) / 256)), dim3(256), 0, st, vol, m[0], m[1], m[2],
                       scale, spec64 + kind * oct, spec32 + kind * oct);
    SIE_HIP(hipGetLastError());
}

}  // namespace sie
