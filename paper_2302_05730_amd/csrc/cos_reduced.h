// cos(x) for the oscillatory integrand, whose arguments (2 pi u_0 +
// sum a_i x_i) stay within a few hundred radians: the argument reduction of
// Cody and Waite (1980) by pi/2 in two fused multiply-adds, then the Taylor
// series of cos or sin on [-pi/4, pi/4] in Horner form.  Truncated after the
// x^16 (cos) and x^17 (sin) terms, the series are exact to better than 3e-18
// relative there.  The two roundings of the reduced argument and the
// evaluation bound the absolute error by about 3e-16 for |x| <= 2^20;
// beyond that the library's cos is called, out of line, so that its
// large-argument reduction does not weigh on the registers of the kernels
// that inline this function.  Usable on the host as well, so that it can be
// checked against the C library.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace mcubes {

__host__ __device__ __attribute__((noinline)) inline double cos_wide(double x) {
    return std::cos(x);
}

__host__ __device__ __forceinline__ double cos_reduced(double x) {
    constexpr double kTwoOverPi = 0.63661977236758134308;
    constexpr double kPiHalfHi = 1.5707963267948966192;      // fl(pi/2)
    constexpr double kPiHalfLo = 6.123233995736766036e-17;   // fl(pi/2 - fl(pi/2))
    constexpr double kMaxArg = 1048576.0;                    // 2^20
    if (std::fabs(x) > kMaxArg) return cos_wide(x);
    const double k = std::rint(x * kTwoOverPi);
    double r = std::fma(-k, kPiHalfHi, x);
    r = std::fma(-k, kPiHalfLo, r);
    const double s = r * r;
    // cos r = 1 + s (-1/2! + s (1/4! - ...)), sin r = r + r s (-1/3! + ...)
    double pc = 1.0 / 20922789888000.0;   // 1/16!
    pc = std::fma(pc, s, -1.0 / 87178291200.0);
    pc = std::fma(pc, s, 1.0 / 479001600.0);
    pc = std::fma(pc, s, -1.0 / 3628800.0);
    pc = std::fma(pc, s, 1.0 / 40320.0);
    pc = std::fma(pc, s, -1.0 / 720.0);
    pc = std::fma(pc, s, 1.0 / 24.0);
    pc = std::fma(pc, s, -0.5);
    const double c = std::fma(s, pc, 1.0);
    double ps = 1.0 / 355687428096000.0;  // 1/17!
    ps = std::fma(ps, s, -1.0 / 1307674368000.0);
    ps = std::fma(ps, s, 1.0 / 6227020800.0);
    ps = std::fma(ps, s, -1.0 / 39916800.0);
    ps = std::fma(ps, s, 1.0 / 362880.0);
    ps = std::fma(ps, s, -1.0 / 5040.0);
    ps = std::fma(ps, s, 1.0 / 120.0);
    ps = std::fma(ps, s, -1.0 / 6.0);
    const double sn = std::fma(r * s, ps, r);
    // x = k pi/2 + r: cos x = cos r, -sin r, -cos r, sin r for k mod 4 = 0..3
    const int q = (int)(int64_t)k & 3;
    const double v = (q & 1) ? sn : c;
    return ((q + 1) & 2) ? -v : v;
}

}  // namespace mcubes
