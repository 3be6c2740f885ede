// Host check of the FBP floor-threshold table: for several (c0, t0, dt, K),
// every threshold is the first FP64 squared distance whose sample index
// floor((sqrt(r2) / c0 - t0) / dt) reaches m (the double just below it does
// not), and for random squared distances, including ones that land exactly
// on a sample time, comparing r2 with the table gives that floor for every
// index in -1 .. K.  Prints "OK <checks>" or the first failure.
#include <cmath>
#include <cstdio>
#include <random>
#include "oat_fbp_floor.hpp"

using namespace oat;

static long kidx(double r2, double c0, double t0, double dt)
{
    return (long)std::floor((std::sqrt(r2) / c0 - t0) / dt);
}

int main()
{
    struct Case { double c0, t0, dt; int K; };
    const Case cases[] = {
        {1.5, 0.0, 0.05, 1024},     // 20 MHz, t0 = 0
        {1.54, 17.5, 0.05, 1022},   // the paper's simulation timing
        {1.5, -1.0, 0.1, 260},      // samples at negative times
        {1.0, 0.0, 0.125, 300},     // exact binary sample spacing
        {1.5, 3.0, 0.2, 3},         // the fewest samples
    };
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> U01(0.0, 1.0);
    long checks = 0;
    for (const Case &c : cases) {
        const std::vector<double> thr = fbp_floor_thresholds(c.c0, c.t0, c.dt, c.K);
        for (int m = -1; m <= c.K; ++m) {
            const double t = thr[(size_t)(m + 1)];
            if (!std::isfinite(t)) continue;
            if (kidx(t, c.c0, c.t0, c.dt) < m) {
                std::printf("FAIL threshold %d does not reach it (c0 %g t0 %g)\n", m, c.c0, c.t0);
                return 1;
            }
            if (t > 0.0 && kidx(std::nextafter(t, 0.0), c.c0, c.t0, c.dt) >= m) {
                std::printf("FAIL threshold %d is not the first (c0 %g t0 %g)\n", m, c.c0, c.t0);
                return 1;
            }
            if (m >= 0 && thr[(size_t)m] > t) {
                std::printf("FAIL thresholds decrease at %d\n", m);
                return 1;
            }
            ++checks;
        }
        const double rmax = c.c0 * (c.t0 + (c.K + 2) * c.dt);
        for (int i = 0; i < 200000; ++i) {
            double r2;
            if (i % 2 == 0) {
                const double r = rmax * U01(rng);
                r2 = r * r;
            } else {
                // a distance at a sample time, and its neighbouring doubles
                const double r = c.c0 * (c.t0 + (double)(long)(U01(rng) * c.K) * c.dt);
                r2 = r * r;
                const int s = (int)(U01(rng) * 5) - 2;
                for (int k = 0; k < std::abs(s); ++k) r2 = std::nextafter(r2, s > 0 ? 1e300 : 0.0);
                if (!(r2 >= 0.0)) continue;
            }
            const long k = kidx(r2, c.c0, c.t0, c.dt);
            for (long m = std::max(-1l, k - 1); m <= std::min((long)c.K, k + 2); ++m) {
                const bool by_table = r2 >= thr[(size_t)(m + 1)];
                if (by_table != (k >= m)) {
                    std::printf("FAIL r2 %.17g index %ld m %ld (c0 %g t0 %g)\n", r2, k, m, c.c0,
                                c.t0);
                    return 1;
                }
                ++checks;
            }
        }
    }
    std::printf("OK %ld\n", checks);
    return 0;
}
