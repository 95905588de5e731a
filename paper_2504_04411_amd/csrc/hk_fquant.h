// Critical value of the F-test (Sec. 3.2.2): the (1 - alpha) quantile of the F(d1, d2) distribution,
// evaluated in float64 on the host and on the device by the same routine (header-only so that the
// device code of every translation unit can inline it).
//
// Method (textbook, written from the definitions):
//   P(F > f) = I_y(d2/2, d1/2) with y = d2 / (d1 f + d2), I the regularised incomplete beta;
//   I_x(a, b) is evaluated by its hypergeometric series (DLMF 8.17.8), whose terms are positive;
//   log B(a, b) for a large argument uses a Stirling-series difference so that the two huge
//   log-gamma values never cancel (d2 reaches ~1e10 with millions of photons per iteration);
//   the quantile is the root of log P(F > f) = log alpha by Newton steps on a bisection bracket.
#pragma once
#include <math.h>

#include <hip/hip_runtime.h>

namespace hk {

// Correction term of the Stirling series: log Gamma(z) - [(z - 1/2) log z - z + log(2 pi) / 2].
__host__ __device__ inline double stirling_tail(double z)
{
    const double z2 = 1.0 / (z * z);
    return (1.0 / 12.0 - z2 * (1.0 / 360.0 - z2 * (1.0 / 1260.0 - z2 * (1.0 / 1680.0)))) / z;
}

// log Gamma(q) - log Gamma(q + p) for q >= 20 by the Stirling series of both terms (next term of the
// series is below 1e-15 there).
__host__ __device__ inline double lgamma_ratio_large(double q, double p)
{
    const double qp = q + p;
    const double d = -(q - 0.5) * log1p(p / q) - p * log(qp) + p;
    return d + stirling_tail(q) - stirling_tail(qp);
}

__host__ __device__ inline double log_beta(double a, double b)
{
    const double p = a < b ? a : b;
    const double q = a < b ? b : a;
    if (q < 20.0) return lgamma(p) + lgamma(q) - lgamma(p + q);
    return lgamma(p) + lgamma_ratio_large(q, p);
}

// Hypergeometric series of the CDF (DLMF 8.17.8):
//   I_x(a, b) = x^a (1 - x)^b / (a B(a, b)) * sum_n [(a + b)_n / (a + 1)_n] x^n.
// Every term is positive, so the sum has no cancellation even when b ~ 1e10 (where the continued
// fraction of the complement loses digits); it converges for x < 1 and needs about (a + b) x terms.
__host__ __device__ inline double ibeta_series(double a, double b, double x)
{
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 100000; ++n) {
        term *= (a + b + (n - 1)) * x / (a + n);
        sum += term;
        if (term < 1e-17 * sum && (a + b + n) * x < (a + n + 1)) break;
    }
    return sum;
}

// log of x^a y^b / B(a, b) with lx = log x, ly = log y.
__host__ __device__ inline double log_kernel(double a, double b, double lx, double ly)
{
    return a * lx + b * ly - log_beta(a, b);
}

// Upper tail P(F > f) = 1 - I_x(d1/2, d2/2), x = d1 f / (d1 f + d2); returns log P(F > f) and writes
// log pdf(f) = log(x^a y^b / B(a, b)) - log f.
__host__ __device__ inline double log_sf(double d1, double d2, double f, double *log_pdf)
{
    const double a = 0.5 * d1, b = 0.5 * d2;
    const double den = d1 * f + d2;
    const double x = d1 * f / den;
    const double y = d2 / den;                  // 1 - x without cancellation
    double lx, ly;
    if (x < 0.5) { lx = log(x); ly = log1p(-x); }   // keeps b log y accurate for huge b
    else { lx = log1p(-y); ly = log(y); }
    const double lk = log_kernel(a, b, lx, ly);
    *log_pdf = lk - log(f);
    const double cdf = exp(lk - log(a)) * ibeta_series(a, b, x);
    return log1p(-fmin(cdf, 1.0));
}

__host__ __device__ inline double f_quantile(double d1, double d2, double alpha)
{
    if (!(d1 > 0.0) || !(d2 > 0.0) || !(alpha > 0.0) || !(alpha < 1.0)) return NAN;
    const double target = log(alpha);
    double lpdf;
    double lo = 0.0, hi = 2.0;
    int guard = 0;
    while (log_sf(d1, d2, hi, &lpdf) > target && guard++ < 200) {
        lo = hi;
        hi *= 2.0;
    }
    double f = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        const double ls = log_sf(d1, d2, f, &lpdf);
        const double g = ls - target;           // decreasing in f
        if (g > 0.0) lo = f; else hi = f;
        // Newton on log P(F > f): d/df log sf = -pdf / sf
        double step = g * exp(ls - lpdf);
        double fn = f + step;
        if (!(fn > lo && fn < hi)) fn = 0.5 * (lo + hi);
        if (fabs(fn - f) <= 1e-15 * f || hi - lo <= 1e-15 * hi) { f = fn; break; }
        f = fn;
    }
    return f;
}

}  // namespace hk

