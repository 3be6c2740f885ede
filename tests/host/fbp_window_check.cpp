// Host check of FBP's staged sample windows over a workload geometry: for
// every voxel tile and every transducer, the sample index floor(kt) of every
// voxel of the tile (kt = (|r_n - r_q| / c0 - t0) / dt, the FP64 problem
// statement, which the kernel's floor decisions reproduce) lies in
// k_lo .. k_lo + win - 2, with k_lo and win formed as the kernel forms them
// (its FP32 tile-centre distance, here also perturbed by 2 ulp either way).
// The update reads samples floor(kt) and floor(kt) + 1 of the window.
//
// Input on stdin: nx ny nz dx x0 y0 z0 c0 dt t0 K Q, then Q lines x y z (mm).
// Prints "OK <pairs> <min low margin> <min high margin>" or the first
// failure.
// The header's functions are host-and-device functions; compiled here for
// the host only.
#define __host__
#define __device__
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <vector>

#include "oat_fbp_window.hpp"

using namespace oat;

int main()
{
    int nx, ny, nz, K, Q;
    double dx, x0, y0, z0, c0, dt, t0;
    if (std::scanf("%d %d %d %lf %lf %lf %lf %lf %lf %lf %d %d", &nx, &ny, &nz, &dx, &x0, &y0,
                   &z0, &c0, &dt, &t0, &K, &Q) != 12) {
        std::printf("FAIL bad header\n");
        return 1;
    }
    std::vector<double> r(3 * (size_t)Q);
    for (int q = 0; q < Q; ++q)
        if (std::scanf("%lf %lf %lf", &r[3 * q], &r[3 * q + 1], &r[3 * q + 2]) != 3) {
            std::printf("FAIL bad transducer %d\n", q);
            return 1;
        }
    const float sigma = (float)(dx / (c0 * dt)), tau = (float)(t0 / dt);
    const int win = fbp_window(sigma);
    const int n[3] = {nx, ny, nz};
    const double o[3] = {x0, y0, z0};
    const int T[3] = {FBP_TX, FBP_TY, FBP_TZ};
    // FP64 sample position of the node at grid point g (problem statement).
    auto kt64 = [&](const int g[3], const double *rq) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double w = o[a] + g[a] * dx - rq[a];
            s += w * w;
        }
        return (std::sqrt(s) / c0 - t0) / dt;
    };
    long pairs = 0;
    long lo_margin = 1L << 40, hi_margin = 1L << 40;
    const int nt[3] = {(nx + FBP_TX - 1) / FBP_TX, (ny + FBP_TY - 1) / FBP_TY,
                       (nz + FBP_TZ - 1) / FBP_TZ};
    for (int bz = 0; bz < nt[2]; ++bz)
        for (int by = 0; by < nt[1]; ++by)
            for (int bx = 0; bx < nt[0]; ++bx) {
                const int b[3] = {bx, by, bz};
                int lo[3], hi[3];
                float c[3];
                for (int a = 0; a < 3; ++a) {
                    lo[a] = b[a] * T[a];
                    hi[a] = std::min(lo[a] + T[a] - 1, n[a] - 1);
                    c[a] = (float)(b[a] * T[a]) + 0.5f * (float)(T[a] - 1);
                }
                for (int q = 0; q < Q; ++q) {
                    const double *rq = &r[3 * (size_t)q];
                    float uqf[3];
                    double uq[3];
                    for (int a = 0; a < 3; ++a) {
                        uq[a] = (rq[a] - o[a]) / dx;
                        uqf[a] = (float)uq[a];
                    }
                    const float vx = c[0] - uqf[0], vy = c[1] - uqf[1], vz = c[2] - uqf[2];
                    const float dc = sqrtf(vx * vx + vy * vy + vz * vz);
                    int k_min = 1 << 30, k_max = -(1 << 30);
                    float d = dc;
                    for (int u = 0; u < 2; ++u) d = nextafterf(d, 0.f);
                    for (int v = 0; v < 5; ++v) {
                        const int k = fbp_first_sample(d, sigma, tau);
                        k_min = std::min(k_min, k);
                        k_max = std::max(k_max, k);
                        d = nextafterf(d, INFINITY);
                    }
                    // nearest and farthest node of the tile (squared distance
                    // separates by axis)
                    int gn[3], gf[3];
                    for (int a = 0; a < 3; ++a) {
                        const double t = std::floor(uq[a] + 0.5);
                        gn[a] = (int)std::min<double>(std::max<double>(t, lo[a]), hi[a]);
                        gf[a] = std::fabs(uq[a] - lo[a]) > std::fabs(uq[a] - hi[a]) ? lo[a] : hi[a];
                    }
                    // a rounding unit of slack on either side of the FP64 kt
                    const double kn = kt64(gn, rq), kf = kt64(gf, rq);
                    const long fn = (long)std::floor(kn - 1e-9 * (std::fabs(kn) + 1.0));
                    const long ff = (long)std::floor(kf + 1e-9 * (std::fabs(kf) + 1.0));
                    const long lm = fn - k_max, hm = (win - 2) - (ff - k_min);
                    if (lm < 0 || hm < 0) {
                        std::printf("FAIL tile (%d,%d,%d) transducer %d: floor(kt) %ld .. %ld, "
                                    "k_lo %d .. %d, win %d\n", bx, by, bz, q, fn, ff, k_min,
                                    k_max, win);
                        return 1;
                    }
                    lo_margin = std::min(lo_margin, lm);
                    hi_margin = std::min(hi_margin, hm);
                    ++pairs;
                }
            }
    std::printf("OK %ld %ld %ld\n", pairs, lo_margin, hi_margin);
    return 0;
}
