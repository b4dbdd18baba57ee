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
 *
 * Strongly lossy media (|Im k| l > 2 on the source triangle's longest edge l,
 * |Im k| >= 0.38 |k|) make G decay within a small fraction of a triangle; the
 * extracted static part and the quadrature of the remainder then cancel to a
 * result far below either, and the remainder rule fails (distant pairs keep
 * its quadrature error in place of an exponentially small value).  All pairs
 * there take polar_pot: polar coordinates around the projection of the
 * observation point, the radial integral of G in closed form, the radial
 * integrals of G r' and of the gradient remainder by Gauss-Legendre on
 * intervals graded in units of 1/|k| (cut at 64/|k|, with the closed-form
 * static tail of the gradient beyond), and composite Gauss-Legendre in the
 * angle, broken where the distance to the edge crosses a radial breakpoint.
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

/* Radial breakpoints of the strong-loss scheme in units of 1/|k|; the last
 * one is the cut. */
static const double POLAR_B[] = {0.25, 0.5, 1.0, 2.0, 3.0, 4.0, 6.0, 8.0, 12.0, 16.0, 24.0, 32.0, 48.0, 64.0};
#define POLAR_NB 14
#define POLAR_NG 8

/* Gauss-Legendre on [a, b] of the radial integrands at height d:
 * fV = exp(-jkR) rp^2 / (4 pi R)      (vector potential, r' - rho0 part)
 * fT = [1 - (1 + jkR) exp(-jkR)] rp^2 / (4 pi R^3)   (gradient remainder). */
static void radial_gl(cplx k, double d, double a, double b, const double *gx, const double *gw,
                      cplx *IV, cplx *IT) {
    const double h = 0.5 * (b - a), c = 0.5 * (b + a);
    for (int g = 0; g < POLAR_NG; ++g) {
        const double rp = c + h * gx[g];
        const double R = sqrt(rp * rp + d * d);
        const cplx e = cexp(-JJ * k * R);
        const double w = h * gw[g] * rp * rp / (4.0 * PI_ * R);
        *IV += w * e;
        *IT += w * (1.0 - (1.0 + JJ * k * R) * e) / (R * R);
    }
}

/* S = int G, V = int G r', Gv = int grad_r G over triangle v at r, for
 * strongly lossy media (see the header).  With rho0 the projection of r on
 * the plane, d the height, and the triangle split into the signed triangles
 * (rho0, edge) swept by the angle theta (direction u(theta), edge distance
 * rho(theta), Re = sqrt(rho^2 + d^2)):
 *   S   = sum int dtheta [exp(-jk|d|) - exp(-jk Re)] / (4 pi jk)
 *   V   = rho0 S + sum int dtheta u IV(rho),  IV = int_0^rho G rp^2 drp
 *   Gv.n = sum int dtheta [d exp(-jk Re)/Re - sign(d) exp(-jk|d|)] / (4 pi)
 *   Gv_t = -sum int dtheta u J(rho),  J = int_0^rho g rp^2 drp, g R^3 = -(1 + jkR) exp(-jkR)/(4 pi)
 * J splits into -(ln(rho + Re) - rho/Re - ln|d|)/(4 pi) plus the integral
 * IT of the remainder g + 1/(4 pi R^3).  In the plane (d = 0) the ln|d| term
 * diverges; it is theta-independent and drops out there, since the signed
 * sum of int u dtheta vanishes for in-plane points, which never lie on the
 * triangle's boundary (off the plane they may: points of a face at right
 * angles project onto the shared edge, so the term is kept).  Beyond the
 * cut IV and J are constant and their angular integrals are closed-form. */
static void polar_pot(const double v[3][3], const double n[3], const double r[3], cplx k,
                      const double *gx, const double *gw, cplx *S, cplx V[3], cplx Gv[3]) {
    const double inv4pi = 1.0 / (4.0 * PI_);
    double tmp[3];
    sub3(r, v[0], tmp);
    double d = dot3(tmp, n);
    double e01[3]; sub3(v[1], v[0], e01);
    if (fabs(d) <= 1e-10 * norm3(e01)) d = 0.0;
    const double ad = fabs(d), sgd = (d > 0.0) ? 1.0 : ((d < 0.0) ? -1.0 : 0.0);
    const double rho0[3] = { r[0] - d * n[0], r[1] - d * n[1], r[2] - d * n[2] };
    const double u = 1.0 / cabs(k);
    double b[POLAR_NB];
    cplx CV[POLAR_NB], CT[POLAR_NB];
    {
        cplx iv = 0.0, it = 0.0;
        double lo = 0.0;
        for (int j = 0; j < POLAR_NB; ++j) {
            b[j] = POLAR_B[j] * u;
            radial_gl(k, d, lo, b[j], gx, gw, &iv, &it);
            CV[j] = iv; CT[j] = it;
            lo = b[j];
        }
    }
    const double rc = b[POLAR_NB - 1], Rc = sqrt(rc * rc + d * d);
    const cplx Vc = CV[POLAR_NB - 1];
    const double gref = ad > 0.0 ? log(ad) : 0.0;
    const cplx Jc = CT[POLAR_NB - 1] - inv4pi * (log(rc + Rc) - rc / Rc - gref);
    const cplx ekd = cexp(-JJ * k * ad);
    cplx sumS = 0.0, sumN = 0.0, UV[3] = {0.0, 0.0, 0.0}, UJ[3] = {0.0, 0.0, 0.0};
    double tot = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double *a = v[i], *bb = v[(i + 1) % 3];
        double le[3], lh[3], mh[3], am[3], bm[3];
        sub3(bb, a, le);
        const double ll = norm3(le);
        lh[0] = le[0] / ll; lh[1] = le[1] / ll; lh[2] = le[2] / ll;
        cross3(lh, n, mh);
        sub3(a, rho0, am); sub3(bb, rho0, bm);
        const double t = dot3(am, mh), sa = dot3(am, lh), sb = dot3(bm, lh);
        if (fabs(t) <= 1e-12 * ll) continue;
        const double at = fabs(t), sg = t > 0.0 ? 1.0 : -1.0;
        const double tha = atan(sa / at), thb = atan(sb / at);
        tot += sg * (thb - tha);
        double bp[2 * POLAR_NB + 2];
        int nbp = 0;
        bp[nbp++] = tha;
        for (int j = 0; j < POLAR_NB; ++j) {
            if (b[j] <= at) continue;
            const double ph = acos(at / b[j]);
            if (-ph > tha && -ph < thb) bp[nbp++] = -ph;
            if (ph > tha && ph < thb) bp[nbp++] = ph;
        }
        bp[nbp++] = thb;
        for (int x = 1; x < nbp; ++x)          /* insertion sort */
            for (int y = x; y > 0 && bp[y - 1] > bp[y]; --y) { double q = bp[y]; bp[y] = bp[y - 1]; bp[y - 1] = q; }
        for (int q = 0; q + 1 < nbp; ++q) {
            const double t1 = bp[q], t2 = bp[q + 1];
            const double h = 0.5 * (t2 - t1), c = 0.5 * (t2 + t1);
            if (h <= 0.0) continue;
            if (at / cos(c) >= rc) {
                /* beyond the cut: sg int u dtheta times the constants */
                for (int m = 0; m < 3; ++m) {
                    const double U = sg * (sg * (sin(t2) - sin(t1)) * mh[m] - (cos(t2) - cos(t1)) * lh[m]);
                    UV[m] += U * Vc;
                    UJ[m] += U * Jc;
                }
                continue;
            }
            for (int g = 0; g < POLAR_NG; ++g) {
                const double th = c + h * gx[g];
                const double wt = sg * h * gw[g];
                const double ct = cos(th), st = sin(th);
                const double rho = at / ct, Re = sqrt(rho * rho + d * d);
                double uh[3];
                for (int m = 0; m < 3; ++m) uh[m] = sg * ct * mh[m] + st * lh[m];
                int j = -1;
                while (j + 1 < POLAR_NB && b[j + 1] <= rho) ++j;
                cplx IV = j >= 0 ? CV[j] : 0.0, IT = j >= 0 ? CT[j] : 0.0;
                radial_gl(k, d, j >= 0 ? b[j] : 0.0, rho, gx, gw, &IV, &IT);
                const cplx J = IT - inv4pi * (log(rho + Re) - rho / Re - gref);
                const cplx eR = cexp(-JJ * k * Re);
                sumS += wt * eR;
                sumN += wt * d * eR / Re;
                for (int m = 0; m < 3; ++m) {
                    UV[m] += wt * uh[m] * IV;
                    UJ[m] += wt * uh[m] * J;
                }
            }
        }
    }
    *S = (ekd * tot - sumS) * inv4pi / (JJ * k);
    const cplx nrm = inv4pi * (sumN - sgd * ekd * tot);
    for (int m = 0; m < 3; ++m) {
        V[m] = rho0[m] * (*S) + UV[m];
        Gv[m] = n[m] * nrm - UJ[m];
    }
}

/* Exported for the oracle's own tests. */
void oracle_static_pot(const double *v9, const double *r, double *out7) {
    double v[3][3]; memcpy(v, v9, sizeof(v));
    double e1[3], e2[3], n[3];
    sub3(v[1], v[0], e1); sub3(v[2], v[0], e2); cross3(e1, e2, n);
    double nn = norm3(n); n[0] /= nn; n[1] /= nn; n[2] /= nn;
    static_pot(v, n, r, &out7[0], &out7[1], &out7[4]);
}

/* Exported for the oracle's own tests: out14 = S, V[3], Gv[3] (re, im). */
void oracle_polar_pot(const double *v9, const double *r, double kr, double ki, const double *gx,
                      const double *gw, double *out14) {
    double v[3][3]; memcpy(v, v9, sizeof(v));
    double e1[3], e2[3], n[3];
    sub3(v[1], v[0], e1); sub3(v[2], v[0], e2); cross3(e1, e2, n);
    double nn = norm3(n); n[0] /= nn; n[1] /= nn; n[2] /= nn;
    cplx S, V[3], Gv[3];
    polar_pot(v, n, r, kr + JJ * ki, gx, gw, &S, V, Gv);
    out14[0] = creal(S); out14[1] = cimag(S);
    for (int m = 0; m < 3; ++m) {
        out14[2 + 2 * m] = creal(V[m]); out14[3 + 2 * m] = cimag(V[m]);
        out14[8 + 2 * m] = creal(Gv[m]); out14[9 + 2 * m] = cimag(Gv[m]);
    }
}

/* verts [T][3][3], area [T], sgn [T][3], len [T][3]
 * pairs tl[P], sl[P]; k = kr + j ki
 * outer rule (no, bo[no][3], wo[no]); inner rule (ni, bi[ni][3], wi[ni]);
 * polar != 0: the strong-loss inner scheme (polar_pot, Gauss-Legendre nodes
 * gx, weights gw on [-1, 1], POLAR_NG of each) instead of the inner rule
 * outputs (interleaved complex) A, Phi, K: [P][3][3][2] */
void oracle_pair_blocks(const double *verts, const double *area, const double *sgn,
                        const double *len, long long P, const long long *tl, const long long *sl,
                        double kr, double ki,
                        int no, const double *bo, const double *wo,
                        int ni, const double *bi, const double *wi,
                        int polar, const double *gx, const double *gw,
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
            cplx S, V[3], Gv[3];
            if (polar) {
                polar_pot(sv, ns, r, k, gx, gw, &S, V, Gv);
            } else {
            double I0, Irho[3], gI[3];
            static_pot(sv, ns, r, &I0, Irho, gI);
            double tmp[3]; sub3(r, sv[0], tmp);
            double d = dot3(tmp, ns);
            if (fabs(d) <= 1e-10 * norm3(e1)) d = 0.0;
            double rho[3] = { r[0] - d * ns[0], r[1] - d * ns[1], r[2] - d * ns[2] };
            S = I0 * inv4pi;
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
