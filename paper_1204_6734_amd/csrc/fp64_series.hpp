// fp64_series.hpp — written by gen_fp64_series.py (same folder); do not edit.
//
// Coefficients, in increasing powers of the argument squared, of the
// polynomials of the FP64 Box-Muller transform: Taylor series economised by
// Chebyshev truncation (dropped coefficients sum to at most 2^-57) in exact
// rational arithmetic, rounded once to FP64.
#pragma once

namespace flb {

// sin r = r S(r^2), 0 <= r <= pi/4; truncation 3.15e-18
constexpr int kSinSeriesTerms = 7;
constexpr double kSinSeries[7] = {1.0, -0.16666666666666616, 0.008333333333320366, -0.00019841269828652788, 2.755731337717005e-06, -2.5050717083864503e-08, 1.5894742519179647e-10};

// cos r = C(r^2), 0 <= r <= pi/4; truncation 3.03e-20
constexpr int kCosSeriesTerms = 8;
constexpr double kCosSeries[8] = {1.0, -0.5, 0.04166666666666645, -0.00138888888888611, 2.480158728388366e-05, -2.755731309837908e-07, 2.0875582449261705e-09, -1.1353382776502543e-11};

// artanh z = z A(z^2), |z| <= 0.1716; truncation 1.15e-18
constexpr int kAtanhSeriesTerms = 8;
constexpr double kAtanhSeries[8] = {1.0, 0.33333333333333826, 0.19999999999649118, 0.14285714380754716, 0.11111098484742916, 0.09091818088351948, 0.07656206682675742, 0.07405430106491899};

}  // namespace flb
