// Triangle quadrature rules for the near-region direct integrals.
//
// Gauss-Legendre nodes on [0, 1] come from Newton iteration on the Legendre
// three-term recurrence.  The product rules built from them:
//   collapsed: x = u, y = v (1 - u) (smooth integrands);
//   corner:    collapsed at a vertex V with radius rho = u^2 and the angle
//              coordinate sigma = v^3 graded towards the side V -> E, which
//              turns the logarithmic singularities of the outer integrand of
//              touching pairs (at the shared vertex and along the shared edge)
//              into smooth functions of (u, v);
//   self:      six corner rules (vertex, edge midpoint, centroid);
//   edge:      two corner rules (shared vertex, shared-edge midpoint, opposite vertex);
//   vertex:    one corner rule at the shared vertex.
#include <cmath>

#include "common.h"

namespace sie {

void gauss_legendre01(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1; p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        // node on [-1, 1] is z; map to [0, 1] (ascending order)
        x[n - 1 - i] = 0.5 * (z + 1.0);
        w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);   // = 0.5 * 2/((1-z^2) P'^2)
    }
}

Rule rule_collapsed(int n) {
    std::vector<double> x, w;
    gauss_legendre01(n, x, w);
    Rule r;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double px = x[i], py = x[j] * (1.0 - x[i]);
            r.bary.insert(r.bary.end(), {1.0 - px - py, px, py});
            r.w.push_back(2.0 * w[i] * w[j] * (1.0 - x[i]));
        }
    return r;
}

static void corner(Rule &r, int n, const double V[3], const double Ev[3], const double F[3], double frac) {
    std::vector<double> x, w;
    gauss_legendre01(n, x, w);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double rho = x[i] * x[i];
            double sig = x[j] * x[j] * x[j];
            double jac = 2.0 * rho * (2.0 * x[i]) * (3.0 * x[j] * x[j]) * frac;
            for (int c = 0; c < 3; ++c)
                r.bary.push_back(V[c] + rho * ((1.0 - sig) * (Ev[c] - V[c]) + sig * (F[c] - V[c])));
            r.w.push_back(w[i] * w[j] * jac);
        }
}

static void unit(int i, double e[3]) { e[0] = e[1] = e[2] = 0.0; e[i] = 1.0; }

Rule rule_self(int n) {
    Rule r;
    const double g[3] = {1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0};
    for (int opp = 0; opp < 3; ++opp) {
        int a = (opp + 1) % 3, b = (opp + 2) % 3;
        double ea[3], eb[3], m[3];
        unit(a, ea); unit(b, eb);
        for (int c = 0; c < 3; ++c) m[c] = 0.5 * (ea[c] + eb[c]);
        corner(r, n, ea, m, g, 1.0 / 6.0);
        corner(r, n, eb, m, g, 1.0 / 6.0);
    }
    return r;
}

Rule rule_edge(int n, int opp) {
    Rule r;
    int a = (opp + 1) % 3, b = (opp + 2) % 3;
    double ea[3], eb[3], eo[3], m[3];
    unit(a, ea); unit(b, eb); unit(opp, eo);
    for (int c = 0; c < 3; ++c) m[c] = 0.5 * (ea[c] + eb[c]);
    corner(r, n, ea, m, eo, 0.5);
    corner(r, n, eb, m, eo, 0.5);
    return r;
}

Rule rule_vertex(int n, int vtx) {
    // collapsed at vtx with rho = u^2 and an ungraded angle coordinate
    Rule r;
    std::vector<double> x, w;
    gauss_legendre01(n, x, w);
    int a = (vtx + 1) % 3, b = (vtx + 2) % 3;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double rho = x[i] * x[i], s = x[j];
            double bc[3] = {0, 0, 0};
            bc[vtx] = 1.0 - rho; bc[a] = rho * (1.0 - s); bc[b] = rho * s;
            r.bary.insert(r.bary.end(), {bc[0], bc[1], bc[2]});
            r.w.push_back(w[i] * w[j] * 2.0 * rho * 2.0 * x[i]);
        }
    return r;
}

}  // namespace sie
