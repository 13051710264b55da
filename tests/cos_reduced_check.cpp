// Host check of cos_reduced (the oscillatory integrand's cosine) against the
// C library's cos: the largest absolute error over uniform arguments in
// [-300, 300], arguments next to multiples of pi/2, tiny arguments, the top
// of the fast range [2^19, 2^20] and, past 2^20, equality with the library.
#include <cmath>
#include <cstdio>
#include <random>

#include "cos_reduced.h"

int main() {
    std::mt19937_64 rng(12345);
    double worst = 0.0, worst_x = 0.0, worst_rel = 0.0;
    long n = 0;
    auto check = [&](double x) {
        const double a = mcubes::cos_reduced(x), b = std::cos(x);
        const double e = std::fabs(a - b);
        if (e > worst) {
            worst = e;
            worst_x = x;
        }
        if (std::fabs(b) >= 0.5) {
            const double rel = e / std::fabs(b);
            if (rel > worst_rel) worst_rel = rel;
        }
        ++n;
    };
    std::uniform_real_distribution<double> wide(-300.0, 300.0), unit(-1.0, 1.0);
    for (int i = 0; i < 2000000; ++i) check(wide(rng));
    for (int k = -200; k <= 200; ++k)
        for (int j = -50; j <= 50; ++j) check(k * 1.5707963267948966 + j * 1e-15);
    for (int i = 0; i < 100000; ++i) check(unit(rng) * 1e-8);
    std::uniform_real_distribution<double> top(524288.0, 1048576.0);
    for (int i = 0; i < 200000; ++i) check(top(rng));
    int beyond_bad = 0;
    std::uniform_real_distribution<double> far(1048577.0, 1e12);
    for (int i = 0; i < 20000; ++i) {
        const double x = far(rng);
        if (mcubes::cos_reduced(x) != std::cos(x) || mcubes::cos_reduced(-x) != std::cos(-x))
            ++beyond_bad;
    }
    const bool nan_ok = std::isnan(mcubes::cos_reduced(NAN)) &&
                        std::isnan(mcubes::cos_reduced(INFINITY));
    std::printf("points %ld max_abs_err %.3e at x=%.17g max_rel_err(|cos|>=0.5) %.3e "
                "beyond_2^20_mismatches %d nan_ok %d\n",
                n, worst, worst_x, worst_rel, beyond_bad, nan_ok ? 1 : 0);
    return (worst <= 4e-16 && worst_rel <= 6e-16 && beyond_bad == 0 && nan_ok) ? 0 : 1;
}
