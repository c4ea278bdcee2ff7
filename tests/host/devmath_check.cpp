// Host check of the library's branch-free sincos_cw and exp_cw (devmath.h, compiled here for
// the host by hipcc) against long-double sinl, cosl and expl on seeded samples.  Prints one
// line per sample range: the range, the number of points, and the largest error
//   sincos: absolute error of sin and of cos in units of 2^-52 (the spacing above 1),
//   exp:    relative error in units of 2^-52.
#include <cmath>
#include <cstdint>
#include <cstdio>

#include "devmath.h"

namespace {

struct Lcg {  // 64-bit linear congruential generator (Knuth's MMIX constants)
    uint64_t s;
    double uniform() {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        return (double)(s >> 11) * 0x1p-53;
    }
};

void check_sincos(const char *name, double lo, double hi, long count, uint64_t seed) {
    Lcg g{seed};
    double worst_s = 0.0, worst_c = 0.0;
    for (long i = 0; i < count; ++i) {
        const double x = lo + (hi - lo) * g.uniform();
        double s, c;
        bemrat::sincos_cw(x, s, c);
        const long double xl = x;
        worst_s = fmax(worst_s, (double)fabsl((long double)s - sinl(xl)));
        worst_c = fmax(worst_c, (double)fabsl((long double)c - cosl(xl)));
    }
    printf("sincos %s %ld %.3f %.3f\n", name, count, worst_s / 0x1p-52, worst_c / 0x1p-52);
}

void check_sincos_near(const char *name, double step, int kmax) {
    // points within a few ulps of multiples of pi/2, where the reduction is most delicate
    double worst_s = 0.0, worst_c = 0.0;
    long count = 0;
    for (int k = -kmax; k <= kmax; ++k) {
        const double base = k * step;
        double x = base;
        for (int u = 0; u < 8; ++u) {
            double s, c;
            bemrat::sincos_cw(x, s, c);
            const long double xl = x;
            worst_s = fmax(worst_s, (double)fabsl((long double)s - sinl(xl)));
            worst_c = fmax(worst_c, (double)fabsl((long double)c - cosl(xl)));
            x = nextafter(x, 1e300);
            ++count;
        }
    }
    printf("sincos %s %ld %.3f %.3f\n", name, count, worst_s / 0x1p-52, worst_c / 0x1p-52);
}

void check_exp(const char *name, double lo, double hi, long count, uint64_t seed) {
    Lcg g{seed};
    double worst = 0.0;
    for (long i = 0; i < count; ++i) {
        const double x = lo + (hi - lo) * g.uniform();
        const double e = bemrat::exp_cw(x);
        const long double r = expl((long double)x);
        worst = fmax(worst, (double)(fabsl((long double)e - r) / r));
    }
    printf("exp %s %ld %.3f\n", name, count, worst / 0x1p-52);
}

}  // namespace

int main() {
    check_sincos("kernel_range", -40.0, 40.0, 4000000, 1);
    check_sincos("full_range", -1e6, 1e6, 4000000, 2);
    check_sincos("small", -1e-3, 1e-3, 1000000, 3);
    check_sincos_near("near_half_pi_multiples", 1.5707963267948966, 20000);
    check_exp("kernel_range", -40.0, 40.0, 4000000, 4);
    check_exp("full_range", -708.0, 708.0, 4000000, 5);
    return 0;
}
