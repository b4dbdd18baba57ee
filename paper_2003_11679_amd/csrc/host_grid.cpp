// AIM grid parameters from the lossy-media error analysis (Sec. IV).
//
// With the loss factor s = sigma / (w eps) and k = k_r sqrt(1 - j s)
// (eq. kdefs), lengths normalised as theta = k_r d, the interpolation error
// of an order-n stencil is bounded (eq. LboundsD2) by
//   (theta_n - theta_0)^(n+1) / (n+1)! |D_n(theta_0, s)|,
// D_n being the (n+1)-th derivative of exp(-j a theta)/theta, a = sqrt(1 - j s)
// (eq. Ddef).  For one grid, lossy and lossless bounds differ by the factor
// |D_n(theta_0, s)| / |D_n(theta_0, 0)|, at most about 1.5 over all theta_0
// and s.  Hence the rule: spacing lambda_r / 20 with lambda_r = 2 pi / k_r,
// i.e. the wavelength of the medium without its losses.  Where stricter
// control is asked for, the spacing is refined by the (n+1)-th root of the
// worst factor over the far region (theta_0 from the near-region boundary
// outwards), which brings the lossy bound back to the lossless one.
#include <algorithm>
#include <cmath>
#include <complex>

#include "problem.h"

namespace sie {

namespace {

const double PI = 3.14159265358979323846;
const double C0 = 299792458.0;

double factorial(int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

double binom(int n, int k) { return factorial(n) / (factorial(k) * factorial(n - k)); }

// D_n(theta, s) of eq. Ddef: product-rule expansion of the (n+1)-th derivative
std::complex<double> d_n(int n, double theta, double s) {
    using C = std::complex<double>;
    const C a = std::sqrt(C(1.0, -s));
    const C mj(0.0, -1.0);
    C acc(0.0, 0.0);
    for (int l = 0; l <= n + 1; ++l) {
        const double sign = ((n + 1 - l) % 2) ? -1.0 : 1.0;
        acc += binom(n + 1, l) * sign * factorial(n + 1 - l) * std::pow(theta, -(double)(n - l + 2)) *
               std::pow(mj * a, (double)l);
    }
    return std::exp(mj * theta * a) * acc;
}

}  // namespace

double loss_ratio(int n, double theta0, double s) {
    return std::abs(d_n(n, theta0, s)) / std::abs(d_n(n, theta0, 0.0));
}

// Largest loss ratio for theta0 >= theta_min (geometric samples up to
// 200 theta_min, beyond which both bounds are negligible).
double worst_loss_ratio_beyond(int n, double theta_min, double s) {
    double worst = 0.0;
    const int K = 400;
    for (int i = 0; i <= K; ++i) {
        const double th = theta_min * std::pow(200.0, (double)i / K);
        worst = std::max(worst, loss_ratio(n, th, s));
    }
    return worst;
}

void choose_grid(double freq, double eps_r, double mu_r, double sigma, double extent, double mean_edge,
                 int near_radius, int strict, sie_grid_params *out) {
    *out = sie_grid_params{};
    SIE_CHECK(freq > 0 && eps_r > 0 && mu_r > 0 && sigma >= 0, SIE_EINVAL, "bad material or frequency");
    SIE_CHECK(extent > 0 && mean_edge > 0, SIE_EINVAL, "extent and mean edge must be positive");
    SIE_CHECK(near_radius >= 1 && near_radius <= 12, SIE_EINVAL, "near radius must be in [1, 12]");
    const int order = 2;
    const double w = 2.0 * PI * freq;
    const double kr = w * std::sqrt(eps_r * mu_r) / C0;
    const double lam_r = 2.0 * PI / kr;
    const double eps0 = 1.0 / (4e-7 * PI * C0 * C0);
    const double s = sigma / (w * eps0 * eps_r);
    double h = lam_r / 20.0;
    // far interactions start at the near-region boundary: theta_0 = k_r R h
    const double ratio = s > 0.0 ? worst_loss_ratio_beyond(order, kr * near_radius * h, s) : 1.0;
    if (strict && ratio > 1.0) h /= std::pow(ratio, 1.0 / (order + 1));
    // the stencil must span a triangle: no coarser than the mean edge
    h = std::min(h, mean_edge);
    long n = (long)std::ceil(extent / h) + 3;
    n = std::max(5L, std::min(n, 1024L));
    out->n = (int32_t)n;
    out->h = extent / (double)(n - 3);
    out->origin[0] = out->origin[1] = out->origin[2] = std::nan("");
    out->order = order;
    out->near_radius = near_radius;
    out->loss_ratio = ratio;
    out->lambda_r = lam_r;
}

}  // namespace sie
