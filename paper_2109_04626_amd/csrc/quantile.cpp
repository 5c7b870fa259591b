// Threshold of the two-sided Fisher-z test, Phi^{-1}(1 - alpha/2)
// (Sec. 2.2.2).  Computed as the root x of the upper-tail equation
// Q(x) = erfc(x / sqrt 2) / 2 = alpha / 2: a starting value from the
// rational approximation of Abramowitz & Stegun 26.2.23 (error < 4.5e-4)
// refined by Halley steps on Q using the C library's erfc.
#include <cmath>

#include "fpc_internal.h"

namespace fpc {

double normal_quantile_upper(double alpha)
{
    if (!(alpha > 0.0 && alpha < 1.0)) return NAN;
    const double ptail = 0.5 * alpha;  // in (0, 0.5)
    const double t = std::sqrt(-2.0 * std::log(ptail));
    double x = t - (2.515517 + 0.802853 * t + 0.010328 * t * t) /
                       (1.0 + 1.432788 * t + 0.189269 * t * t + 0.001308 * t * t * t);
    const double inv_sqrt2 = 0.70710678118654752440;
    const double inv_sqrt_2pi = 0.39894228040143267794;
    for (int it = 0; it < 40; ++it) {
        const double q = 0.5 * std::erfc(x * inv_sqrt2);
        const double phi = inv_sqrt_2pi * std::exp(-0.5 * x * x);
        if (!(phi > 0.0)) break;
        // f(x) = Q(x) - ptail, f' = -phi, f'' = x phi  ->  Halley step
        const double f = q - ptail;
        const double d = f / phi;               // -f/f'
        const double step = d / (1.0 - 0.5 * x * d);
        x += step;
        if (std::fabs(step) <= 1e-16 * std::fabs(x)) break;
    }
    return x;
}

}  // namespace fpc

extern "C" double fpc_quantile(double alpha) { return fpc::normal_quantile_upper(alpha); }
