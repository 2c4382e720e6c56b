// Host build of the library's FP64 exponential (csrc/qmc_exp.h) with the
// C library's fma, compared with the long-double exponential: prints the
// largest error in units in the last place over x in [lo, 0] and the count
// of arguments checked.
#define __host__
#define __device__
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "qmc_exp.h"

static double ulp_of(double y) {
    if (y == 0.0) return 4.9406564584124654e-324;
    return std::nextafter(y, INFINITY) - y;
}

int main(int argc, char **argv) {
    const double lo = argc > 1 ? std::atof(argv[1]) : -745.0;
    const long n = argc > 2 ? std::atol(argv[2]) : 2000000;
    double worst = 0.0, worst_x = 0.0;
    long checked = 0;
    auto fma3 = [](double a, double b, double c) { return std::fma(a, b, c); };
    for (long i = 0; i <= n; ++i) {
        double x = lo * (double)i / (double)n;
        for (int k = 0; k < 2; ++k) {  // the grid point and a neighbour off the grid
            const double xv = k == 0 ? x : std::nextafter(x, -INFINITY) * (1.0 + 1e-13);
            if (xv < lo || xv > 0.0) continue;
            const double got = exp_cody_waite(xv, fma3);
            const long double ref = expl((long double)xv);
            const double err = (double)(fabsl((long double)got - ref) / (long double)ulp_of((double)ref));
            if (err > worst) {
                worst = err;
                worst_x = xv;
            }
            ++checked;
        }
    }
    std::printf("%.6f %.17g %ld\n", worst, worst_x, checked);
    return 0;
}
