// exp(x) in FP64 for the orbitals' exponentials: Cody-Waite reduction
// x = n ln2 + r, |r| <= ln2 / 2 (ln2 split into a head with trailing zero
// bits, so n * head is exact, and a tail), the degree-13 Taylor polynomial
// of e^r (truncation below 5e-18 relative), and one scaling by 2^n that
// rounds once, so underflow to subnormals and zero needs no branch.  Within
// one ulp of the exact value for x <= 0 (checked on the host against a
// long-double exponential).  `fma3(a, b, c)` computes a * b + c with one
// rounding; the caller picks the instruction form.  The including file
// provides __host__ / __device__.
#pragma once

#include <math.h>

template <typename Fma3>
__host__ __device__ inline double exp_cody_waite(double x, Fma3 fma3) {
    const double n = __builtin_rint(x * 1.4426950408889634);
    double r = fma(-n, 6.93147180369123816490e-01, x);
    r = fma(-n, 1.90821492927058770002e-10, r);
    double p = fma3(r, 1.0 / 6227020800.0, 1.0 / 479001600.0);
    p = fma3(p, r, 1.0 / 39916800.0);
    p = fma3(p, r, 1.0 / 3628800.0);
    p = fma3(p, r, 1.0 / 362880.0);
    p = fma3(p, r, 1.0 / 40320.0);
    p = fma3(p, r, 1.0 / 5040.0);
    p = fma3(p, r, 1.0 / 720.0);
    p = fma3(p, r, 1.0 / 120.0);
    p = fma3(p, r, 1.0 / 24.0);
    p = fma3(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)n);
}
