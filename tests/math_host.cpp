// Host build of the kernels' FP64 elementary functions (mech_math.h), checked
// against long-double references: prints the worst error in ulps per
// function over seeded random arguments, and a few special values.
#define MECH_HD_INLINE static inline
#include "mech_math.h"

#include <stdio.h>
#include <stdlib.h>

static double ulps(double got, long double ref) {
    const double r = (double)ref;
    if (r == 0.0) return got == 0.0 ? 0.0 : INFINITY;
    const double u = nextafter(fabs(r), INFINITY) - fabs(r);
    return (double)(fabsl((long double)got - ref) / (long double)u);
}

int main(int argc, char **argv) {
    const long n = argc > 1 ? atol(argv[1]) : 1000000;
    srand48(20190505);
    double e_exp = 0, e_em1 = 0, e_log = 0, e_sin = 0, a_sin = 0;
    for (long i = 0; i < n; ++i) {
        const int c = (int)(i % 4);
        const double span = c == 0 ? 60.0 : c == 1 ? 1.0 : c == 2 ? 1e-3 : 700.0;
        const double x = (2.0 * drand48() - 1.0) * span;
        e_exp = fmax(e_exp, ulps(mech::exp_d(x), expl((long double)x)));
        e_em1 = fmax(e_em1, ulps(mech::expm1_d(x), expm1l((long double)x)));
        // ln over 1e-12 .. 1e12, log-uniform
        const double y = pow(10.0, (2.0 * drand48() - 1.0) * 12.0);
        e_log = fmax(e_log, ulps(mech::log_d(y), logl((long double)y)));
        // sin over |x| < 1e5 (the clamp waveform's phase stays far smaller)
        const double z = (2.0 * drand48() - 1.0) * (c == 0 ? 1.0 : c == 1 ? 100.0 : 1e5);
        const long double sref = sinl((long double)z);
        a_sin = fmax(a_sin, (double)fabsl((long double)mech::sin_d(z) - sref));
        if (fabsl(sref) > 1e-3L) e_sin = fmax(e_sin, ulps(mech::sin_d(z), sref));
    }
    printf("exp %.4f\nexpm1 %.4f\nlog %.4f\nsin %.4f\nsin_abs %.4g\n", e_exp, e_em1, e_log, e_sin, a_sin);
    printf("exp(-800) %.17g\nexp(800) %.17g\nexpm1(-800) %.17g\nexpm1(0) %.17g\nlog(1) %.17g\nlog(0) %.17g\n"
           "log(-1) %.17g\nsin(0) %.17g\nexp(nan) %.17g\n",
           mech::exp_d(-800.0), mech::exp_d(800.0), mech::expm1_d(-800.0), mech::expm1_d(0.0), mech::log_d(1.0),
           mech::log_d(0.0), mech::log_d(-1.0), mech::sin_d(0.0), mech::exp_d(NAN));
    return 0;
}
