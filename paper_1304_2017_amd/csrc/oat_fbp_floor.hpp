// Exact FP64 floor decisions of the FBP interpolation, Eq. (disfbp), by
// table (host only).
//
// The problem statement takes the sample index of node r_n and transducer r_q
// as k = floor(kt), kt = (|r_n - r_q| / c0 - t0) / dt, in FP64, with
// |r_n - r_q| = sqrt(r2) and r2 the FP64 squared distance.  Every step after
// r2 (square root, division by c0 > 0, subtraction of t0, division by
// dt > 0, floor) is correctly rounded and non-decreasing, so floor(kt) is a
// non-decreasing function of r2: floor(kt) >= m holds exactly for
// r2 >= thr(m), the smallest FP64 r2 with that property.  The FBP kernel
// computes kt in FP32 and, where that lands within its error bound of an
// integer m, compares its FP64 r2 with thr(m) instead of evaluating the
// square root and the two divisions.
#pragma once

#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

namespace oat {

inline double fbp_kt(double r2, double c0, double t0, double dt)
{
    return (std::sqrt(r2) / c0 - t0) / dt;
}

// thr[m + 1] for m = -1 .. K: the smallest FP64 r2 >= 0 with
// floor(fbp_kt(r2)) >= m, or +infinity when no finite r2 reaches m.  Below
// m = -1 and above m = K both candidate indices select only zero samples, so
// the decision there does not matter.
inline std::vector<double> fbp_floor_thresholds(double c0, double t0, double dt, int K)
{
    auto to_bits = [](double x) {
        uint64_t u;
        std::memcpy(&u, &x, sizeof u);
        return u;
    };
    auto from_bits = [](uint64_t u) {
        double x;
        std::memcpy(&x, &u, sizeof x);
        return x;
    };
    // Non-negative doubles are ordered like their bit patterns.
    auto reaches = [&](uint64_t u, int m) {
        return std::floor(fbp_kt(from_bits(u), c0, t0, dt)) >= (double)m;
    };
    const uint64_t top = to_bits(std::numeric_limits<double>::max());
    std::vector<double> thr((size_t)K + 2);
    for (int m = -1; m <= K; ++m) {
        double &t = thr[(size_t)(m + 1)];
        if (reaches(0, m)) {
            t = 0.0;
        } else if (!reaches(top, m)) {
            t = std::numeric_limits<double>::infinity();
        } else {
            uint64_t lo = 0, hi = top;   // reaches(lo) is false, reaches(hi) true
            while (hi - lo > 1) {
                const uint64_t mid = lo + (hi - lo) / 2;
                if (reaches(mid, m))
                    hi = mid;
                else
                    lo = mid;
            }
            t = from_bits(hi);
        }
    }
    return thr;
}

}  // namespace oat
