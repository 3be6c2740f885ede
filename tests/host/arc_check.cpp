// Host check of the ring/brick arc enumeration of the G kernels: for random
// transducers, bricks and rings, every ring point whose exact (FP64)
// position lies in the brick's cell box (widened by 0.01 cell) must fall
// inside the arc returned by ring_arc, and shells/rings outside the
// candidate ranges must hold no such point.  Prints "OK <rings> <points>
// <waste>" or the first failure.
#define __host__
#define __device__
#define __forceinline__ inline
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include "oat_geom.hpp"

using namespace oat;

int main(int argc, char **argv)
{
    int trials = argc > 1 ? atoi(argv[1]) : 200;
    unsigned seed = argc > 2 ? (unsigned)atoi(argv[2]) : 1u;
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U01(0.0, 1.0);
    // atan2_approx (Abramowitz & Stegun 4.4.49 after octant reduction)
    // against the library atan2 over the whole circle and several radii.
    double atan_err = 0.0;
    for (int i = 0; i <= 400000; ++i) {
        const double a = -M_PI + 2.0 * M_PI * i / 400000.0;
        for (double rad : {1e-3, 1.0, 700.0}) {
            const float x = (float)(rad * cos(a)), y = (float)(rad * sin(a));
            double e = fabs((double)atan2_approx(y, x) - atan2((double)y, (double)x));
            if (e > M_PI) e = 2.0 * M_PI - e;   // the two ends of (-pi, pi]
            atan_err = fmax(atan_err, e);
        }
    }
    if (!(atan_err <= 1e-6)) {
        printf("FAIL atan2_approx error %.3e\n", atan_err);
        return 1;
    }
    long rings = 0, inside = 0, covered = 0;
    for (int t = 0; t < trials; ++t) {
        // transducer at distance 40..600 grid units, random direction
        double z = 2 * U01(rng) - 1, ph = 2 * M_PI * U01(rng);
        double dist = 40 + 560 * U01(rng);
        double r[3] = {dist * sqrt(1 - z * z) * cos(ph), dist * sqrt(1 - z * z) * sin(ph), dist * z};
        double d = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        double th = acos(r[2] / d), phs = atan2(r[1], r[0]);
        double e1[3] = {cos(th) * cos(phs), cos(th) * sin(phs), -sin(th)};
        double e2[3] = {sin(phs), -cos(phs), 0.0};
        double e3[3] = {-r[0] / d, -r[1] / d, -r[2] / d};
        float e1f[3], e2f[3];
        for (int a = 0; a < 3; ++a) { e1f[a] = (float)e1[a]; e2f[a] = (float)e2[a]; }
        // brick near the origin, size 1..21 cells
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = (int)floor((U01(rng) - 0.5) * 0.6 * dist);
            hi[a] = lo[a] + 1 + (int)(21 * U01(rng));
        }
        ArcUnit Uu;
        arc_unit_setup(Uu, lo, hi, r, e1f, e2f, e3, 0.02f);
        double rho_step = 0.3 + 3.0 * U01(rng);
        double dmin2 = 0, dmax2 = 0;
        for (int a = 0; a < 3; ++a) {
            double dl = lo[a] - r[a], dh = r[a] - hi[a];
            double dm = std::max(std::max(dl, dh), 0.0);
            dmin2 += dm * dm;
            double e = std::max(fabs(r[a] - lo[a]), fabs(r[a] - hi[a]));
            dmax2 += e * e;
        }
        for (int k = 0; k < 100000; ++k) {
            double rho = 0.5 * rho_step + k * rho_step;
            if (rho > sqrt(dmax2) + 1.0) break;
            if (rho < sqrt(dmin2) - 1.0) continue;
            double dth = 1.0 / rho;
            long nring = (long)ceil(M_PI / dth);
            for (long i = 0; i < nring; ++i) {
                double tlo = i * dth, thi = std::min((i + 1) * dth, M_PI), tt = 0.5 * (tlo + thi);
                int nj = (int)std::max(1.0, floor(2 * M_PI * rho * sin(tt) + 0.5));
                double rc = rho * cos(tt), rs = rho * sin(tt);
                double C[3];
                for (int a = 0; a < 3; ++a) C[a] = r[a] + rc * e3[a];
                // Rings whose circle stays farther than the box's half
                // diagonal (+1) from the box centre hold no box point.
                double v[3], hd2 = 0, v3 = 0, vv = 0;
                for (int a = 0; a < 3; ++a) {
                    v[a] = 0.5 * (lo[a] + hi[a]) - C[a];
                    hd2 += 0.25 * (hi[a] - lo[a]) * (hi[a] - lo[a]);
                    v3 += v[a] * e3[a];
                    vv += v[a] * v[a];
                }
                double vperp = sqrt(std::max(0.0, vv - v3 * v3));
                double md = sqrt(v3 * v3 + (vperp - rs) * (vperp - rs));
                if (md > sqrt(hd2) + 1.0) continue;
                float Cf[3] = {(float)C[0], (float)C[1], (float)C[2]};
                int jlo, cnt;
                ring_arc(Uu, Cf, (float)rs, (float)rc, nj, jlo, cnt);
                ++rings;
                for (int j = 0; j < nj; ++j) {
                    double phj = 2 * M_PI * j / nj, p[3];
                    bool in = true;
                    for (int a = 0; a < 3; ++a) {
                        p[a] = C[a] + rs * (cos(phj) * e1[a] + sin(phj) * e2[a]);
                        if (!(p[a] >= lo[a] - 0.01 && p[a] < hi[a] + 0.01)) in = false;
                    }
                    if (!in) continue;
                    ++inside;
                    int rel = ((j - jlo) % nj + nj) % nj;
                    if (rel >= cnt) {
                        printf("FAIL trial %d k %d i %ld j %d nj %d arc [%d,+%d) r %.3f pos %.4f %.4f %.4f box [%d,%d)x[%d,%d)x[%d,%d)\n",
                               t, k, i, j, nj, jlo, cnt, rs, p[0], p[1], p[2], lo[0], hi[0], lo[1], hi[1], lo[2], hi[2]);
                        return 1;
                    }
                }
                covered += cnt;
            }
        }
    }
    printf("OK %ld %ld %.4f\n", rings, inside, inside ? (double)covered / inside : 0.0);
    return 0;
}
