/* Oracle: Galerkin double integrals over triangle pairs (plain C, FP64).
 *
 * Test infrastructure only (see oracle/__init__.py).  Computes, for each pair
 * (t, s) of test and source triangles, the local 3x3 blocks (test edge e of t,
 * source edge f of s) of
 *
 *   A   = int_t int_s f_e . f_f G dS' dS
 *   Phi = int_t int_s (div f_e)(div f_f) G dS' dS
 *   K   = int_t f_e . int_s grad_r G(r - r') x f_f(r') dS' dS
 *
 * with G = exp(-j k R)/(4 pi R) (operators of Sec. III-A, eq. opL/opK/Grrpki).
 * The inner integral splits G into 1/(4 pi R), integrated in closed form
 * (Wilton et al. 1984, Graglia 1993), plus a bounded remainder integrated with
 * the caller's quadrature rule.  Using grad G x (r' - p) = grad G x (r - p)
 * (grad_r G is parallel to r - r'), the K inner integral needs only
 * int_s grad_r G dS'.
 */
#include <math.h>
#include <complex.h>
#include <string.h>

#define PI_ 3.14159265358979323846
#define JJ _Complex_I

typedef double complex cplx;

static void sub3(const double *a, const double *b, double *o) { o[0]=a[0]-b[0]; o[1]=a[1]-b[1]; o[2]=a[2]-b[2]; }
static double dot3(const double *a, const double *b) { return a[0]*b[0]+a[1]*b[1]+a[2]*b[2]; }
static void cross3(const double *a, const double *b, double *o) {
    o[0]=a[1]*b[2]-a[2]*b[1]; o[1]=a[2]*b[0]-a[0]*b[2]; o[2]=a[0]*b[1]-a[1]*b[0];
}
static double norm3(const double *a) { return sqrt(dot3(a, a)); }

/* ln((R+ + l+)/(R- + l-)) without cancellation for any foot-point position. */
static double log_ratio(double lp, double lm, double Rp, double Rm, double R02) {
    if (lm >= 0.0) return log((Rp + lp) / (Rm + lm));
    if (lp <= 0.0) return log((Rm - lm) / (Rp - lp));
    return log((Rp + lp) * (Rm - lm)) - log(R02);
}

/* Closed-form static potentials of triangle v at point r:
 * I = int 1/R, Irho = int (rho' - rho)/R, gI = grad_r int 1/R. */
static void static_pot(const double v[3][3], const double n[3], const double r[3],
                       double *Iout, double Irho[3], double gI[3]) {
    double tmp[3];
    sub3(r, v[0], tmp);
    double d = dot3(tmp, n);
    /* Points in the source plane up to rounding take the principal value
     * (sign(d) = 0); the +-1/2 jump terms are carried by the X operator. */
    double e01[3]; sub3(v[1], v[0], e01);
    if (fabs(d) <= 1e-10 * norm3(e01)) d = 0.0;
    double ad = fabs(d);
    double sI = 0.0, sb = 0.0;
    Irho[0] = Irho[1] = Irho[2] = 0.0;
    gI[0] = gI[1] = gI[2] = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double *a = v[i], *b = v[(i + 1) % 3];
        double le[3], lh[3], mh[3], am[3], bm[3];
        sub3(b, a, le);
        double ll = norm3(le);
        lh[0] = le[0]/ll; lh[1] = le[1]/ll; lh[2] = le[2]/ll;
        cross3(lh, n, mh);
        sub3(b, r, bm); sub3(a, r, am);
        double lp = dot3(bm, lh), lm = dot3(am, lh), t = dot3(am, mh);
        double Rp = norm3(bm), Rm = norm3(am);
        double R02 = t * t + d * d;
        int online = R02 <= 1e-30 * (lp * lp + lm * lm + 1e-300);
        double f = log_ratio(lp, lm, Rp, Rm, R02);
        double beta = 0.0;
        if (!online) beta = atan2(t * lp, R02 + ad * Rp) - atan2(t * lm, R02 + ad * Rm);
        if (!online) sI += t * f;
        sb += beta;
        double coef = (online ? 0.0 : R02 * f) + lp * Rp - lm * Rm;
        for (int c = 0; c < 3; ++c) {
            Irho[c] += 0.5 * coef * mh[c];
            gI[c] -= f * mh[c];
        }
    }
    *Iout = sI - ad * sb;
    double sg = (d > 0.0) ? 1.0 : ((d < 0.0) ? -1.0 : 0.0);
    for (int c = 0; c < 3; ++c) gI[c] -= sg * sb * n[c];
}

/* Exported for the oracle's own tests. */
void oracle_static_pot(const double *v9, const double *r, double *out7) {
    double v[3][3]; memcpy(v, v9, sizeof(v));
    double e1[3], e2[3], n[3];
    sub3(v[1], v[0], e1); sub3(v[2], v[0], e2); cross3(e1, e2, n);
    double nn = norm3(n); n[0] /= nn; n[1] /= nn; n[2] /= nn;
    static_pot(v, n, r, &out7[0], &out7[1], &out7[4]);
}

/* verts [T][3][3], area [T], sgn [T][3], len [T][3]
 * pairs tl[P], sl[P]; k = kr + j ki
 * outer rule (no, bo[no][3], wo[no]); inner rule (ni, bi[ni][3], wi[ni])
 * outputs (interleaved complex) A, Phi, K: [P][3][3][2] */
void oracle_pair_blocks(const double *verts, const double *area, const double *sgn,
                        const double *len, long long P, const long long *tl, const long long *sl,
                        double kr, double ki,
                        int no, const double *bo, const double *wo,
                        int ni, const double *bi, const double *wi,
                        double *Aout, double *Pout, double *Kout) {
    const cplx k = kr + JJ * ki;
    const double inv4pi = 1.0 / (4.0 * PI_);
    #pragma omp parallel for schedule(dynamic, 64)
    for (long long p = 0; p < P; ++p) {
        const long long t = tl[p], s = sl[p];
        double tv[3][3], sv[3][3];
        memcpy(tv, verts + 9 * t, sizeof(tv));
        memcpy(sv, verts + 9 * s, sizeof(sv));
        const double At = area[t], As = area[s];
        double ct[3], cs[3];
        for (int e = 0; e < 3; ++e) {
            ct[e] = sgn[3 * t + e] * len[3 * t + e] / (2.0 * At);
            cs[e] = sgn[3 * s + e] * len[3 * s + e] / (2.0 * As);
        }
        double e1[3], e2[3], ns[3];
        sub3(sv[1], sv[0], e1); sub3(sv[2], sv[0], e2); cross3(e1, e2, ns);
        double nn = norm3(ns); ns[0] /= nn; ns[1] /= nn; ns[2] /= nn;
        /* inner quadrature points */
        double ip[256][3];
        for (int q = 0; q < ni; ++q)
            for (int c = 0; c < 3; ++c)
                ip[q][c] = bi[3*q] * sv[0][c] + bi[3*q+1] * sv[1][c] + bi[3*q+2] * sv[2][c];
        cplx A[3][3] = {{0}}, Ph[3][3] = {{0}}, K[3][3] = {{0}};
        for (int qo = 0; qo < no; ++qo) {
            double r[3];
            for (int c = 0; c < 3; ++c)
                r[c] = bo[3*qo] * tv[0][c] + bo[3*qo+1] * tv[1][c] + bo[3*qo+2] * tv[2][c];
            const double W = wo[qo] * At;
            double I0, Irho[3], gI[3];
            static_pot(sv, ns, r, &I0, Irho, gI);
            double tmp[3]; sub3(r, sv[0], tmp);
            double d = dot3(tmp, ns);
            if (fabs(d) <= 1e-10 * norm3(e1)) d = 0.0;
            double rho[3] = { r[0] - d * ns[0], r[1] - d * ns[1], r[2] - d * ns[2] };
            cplx S = I0 * inv4pi;
            cplx V[3], Gv[3];
            for (int c = 0; c < 3; ++c) {
                V[c] = (Irho[c] + rho[c] * I0) * inv4pi;
                Gv[c] = gI[c] * inv4pi;
            }
            for (int qi = 0; qi < ni; ++qi) {
                double df[3]; sub3(r, ip[qi], df);
                double R = norm3(df);
                double wA = wi[qi] * As;
                cplx rem, hg;
                if (R == 0.0) {
                    rem = -JJ * k * inv4pi;      /* limit of (exp(-jkR) - 1)/(4 pi R) */
                    hg = 0.0;                   /* multiplied by r - r' = 0 */
                } else {
                    cplx z = -JJ * k * R;
                    cplx ez = cexp(z);
                    rem = (ez - 1.0) * inv4pi / R;
                    hg = (1.0 - (1.0 - z) * ez) * inv4pi / (R * R * R);
                }
                S += wA * rem;
                for (int c = 0; c < 3; ++c) {
                    V[c] += wA * rem * ip[qi][c];
                    Gv[c] += wA * hg * df[c];
                }
            }
            for (int e = 0; e < 3; ++e) {
                double fe[3];
                for (int c = 0; c < 3; ++c) fe[c] = ct[e] * (r[c] - tv[e][c]);
                for (int f = 0; f < 3; ++f) {
                    /* int_s G f_f = cs (V - p_f S) */
                    cplx va = 0.0, kk = 0.0;
                    double rp[3];
                    sub3(r, sv[f], rp);
                    cplx cr[3] = { Gv[1]*rp[2] - Gv[2]*rp[1], Gv[2]*rp[0] - Gv[0]*rp[2],
                                   Gv[0]*rp[1] - Gv[1]*rp[0] };
                    for (int c = 0; c < 3; ++c) {
                        va += fe[c] * (V[c] - sv[f][c] * S);
                        kk += fe[c] * cr[c];
                    }
                    A[e][f] += W * cs[f] * va;
                    K[e][f] += W * cs[f] * kk;
                    Ph[e][f] += W * (2.0 * ct[e]) * (2.0 * cs[f]) * S;
                }
            }
        }
        for (int e = 0; e < 3; ++e)
            for (int f = 0; f < 3; ++f) {
                long long o = ((p * 3 + e) * 3 + f) * 2;
                Aout[o] = creal(A[e][f]); Aout[o + 1] = cimag(A[e][f]);
                Pout[o] = creal(Ph[e][f]); Pout[o + 1] = cimag(Ph[e][f]);
                Kout[o] = creal(K[e][f]); Kout[o + 1] = cimag(K[e][f]);
            }
    }
}
