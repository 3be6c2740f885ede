// Geometry helpers of the brick-driven spherical Radon transform that are
// shared by host tests and the gfx950 kernels (__host__ __device__).
//
// The quadrature of G (Appendix: rings of arc length dx in theta, points of
// arc length ~dx in phi, on spheres rho_k = c0 t_k about each transducer)
// is enumerated per (image brick, transducer): for every ring that can reach
// the brick, an arc of ring indices j is found that contains every point of
// the ring lying inside the brick's cell box.  The arc is a superset; the
// exact ownership test is done per point on the point's own position.
#pragma once

#include <math.h>
#include <stdint.h>

#ifndef __HIP_DEVICE_COMPILE__
#include <algorithm>
#endif

namespace oat {

#define OAT_HD __host__ __device__ __forceinline__

constexpr float kPi = 3.14159265358979323846f;
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr float kInvTwoPi = 0.15915494309189533577f;

OAT_HD float fminf_(float a, float b) { return a < b ? a : b; }
OAT_HD float fmaxf_(float a, float b) { return a > b ? a : b; }

// Reciprocal and square root for the conservative range code (results carry
// margins): the hardware approximations on the GPU, libm on the host.
OAT_HD float rcp_approx(float x)
{
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

OAT_HD float sqrt_approx(float x)
{
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_sqrtf(x);
#else
    return sqrtf(x);
#endif
}

// arccos with absolute error below 1e-4 (Abramowitz & Stegun 4.4.45 form);
// used only for conservative ranges that carry margins of their own.
OAT_HD float acos_approx(float x)
{
    x = fminf_(1.0f, fmaxf_(-1.0f, x));
    float ax = fabsf(x);
    float p = 1.5707288f + ax * (-0.2121144f + ax * (0.0742610f - 0.0187293f * ax));
    float r = sqrt_approx(1.0f - ax) * p;
    return x >= 0.0f ? r : kPi - r;
}

// atan2 by octant reduction to atan on [0, 1], with the polynomial of
// Abramowitz & Stegun 4.4.49 (|error| <= 2e-8 rad on [0, 1]; in FP32, with
// the approximate reciprocal, a few 1e-7 rad); conservative-range use only.
OAT_HD float atan2_approx(float y, float x)
{
    float ax = fabsf(x), ay = fabsf(y);
    float mx = fmaxf_(ax, ay), mn = fminf_(ax, ay);
    float a = mx > 0.0f ? mn * rcp_approx(mx) : 0.0f;
    float s = a * a;
    float p = 0.0028662257f;
    p = p * s - 0.0161657367f;
    p = p * s + 0.0429096138f;
    p = p * s - 0.0752896400f;
    p = p * s + 0.1065626393f;
    p = p * s - 0.1420889944f;
    p = p * s + 0.1999355085f;
    p = p * s - 0.3333314528f;
    float r = (p * s) * a + a;
    if (ay > ax) r = 1.57079632679f - r;
    if (x < 0.0f) r = kPi - r;
    return y < 0.0f ? -r : r;
}

// cos/sin to about 1e-6 (hardware on the GPU, libm on the host); used only
// where the arc margins absorb the error.
OAT_HD void sincos_approx(float a, float &c, float &s)
{
#ifdef __HIP_DEVICE_COMPILE__
    c = __cosf(a);
    s = __sinf(a);
#else
    c = cosf(a);
    s = sinf(a);
#endif
}

// Per (brick, transducer) constants for the ring/box arc test.  All in grid
// units.  The box is the set of points whose cell floor(u) lies in
// [lo, hi) per axis, widened by a small margin.
struct ArcUnit {
    float lo[3], hi[3];  // widened box faces
    float nrm[3];        // |projection of axis a on the ring plane|
    float gam[3];        // azimuth (from the box-centre direction) of axis a in the ring plane
    float phic;          // azimuth of the box centre in the ring frame (from e1 toward e2)
    float V3;            // (box centre - transducer) . e3
    float rhov2, rhov;   // squared / plain distance of the box centre from the z^tr axis
    float h2;            // squared radius of the ball that holds the box (+margin)
};

// Fill the arc constants.  cb: box centre, uq: transducer (grid units,
// double), e1/e2/e3: local frame.
OAT_HD void arc_unit_setup(ArcUnit &U, const int lo[3], const int hi[3], const double uq[3],
                           const float e1[3], const float e2[3], const double e3[3],
                           float margin)
{
    double cb[3], V[3];
    double hd2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        U.lo[a] = (float)lo[a] - margin;
        U.hi[a] = (float)hi[a] + margin;
        cb[a] = 0.5 * ((double)lo[a] + (double)hi[a]);
        V[a] = cb[a] - uq[a];
        double e = 0.5 * (double)(hi[a] - lo[a]);
        hd2 += e * e;
    }
    float h = (float)sqrt(hd2) + 0.5f;
    U.h2 = h * h;
    float V1 = (float)(V[0] * e1[0] + V[1] * e1[1] + V[2] * e1[2]);
    float V2 = (float)(V[0] * e2[0] + V[1] * e2[1] + V[2] * e2[2]);
    U.V3 = (float)(V[0] * e3[0] + V[1] * e3[1] + V[2] * e3[2]);
    U.rhov2 = V1 * V1 + V2 * V2;
    U.rhov = sqrtf(U.rhov2);
    U.phic = atan2_approx(V2, V1);
    float c, s;
    sincos_approx(U.phic, c, s);
    for (int a = 0; a < 3; ++a) {
        float E1 = c * e1[a] + s * e2[a];
        float E2 = -s * e1[a] + c * e2[a];
        U.nrm[a] = sqrtf(E1 * E1 + E2 * E2);
        U.gam[a] = atan2_approx(E2, E1);
    }
}

// Conservative arc of ring indices holding every point of the ring that lies
// in the widened box.  Ring: centre C, radius r (grid units), axial offset
// rc = rho cos(theta_i) (grid units), nj points at phi_j = 2 pi j / nj in
// the ring frame.  Output: first index jlo in [0, nj) and count cnt in
// [0, nj]; the arc is jlo, jlo+1, ..., jlo+cnt-1 taken modulo nj.
OAT_HD void ring_arc(const ArcUnit &U, const float C[3], float r, float rc, int nj,
                     int &jlo, int &cnt)
{
    // Window of the ring inside the ball around the box: |p - cb|^2 =
    // rhov^2 + v3^2 + r^2 - 2 r rhov cos(psi), psi = phi - phic.  Written
    // without data-dependent branches (all lanes of a wave take one path).
    const float v3 = U.V3 - rc;
    const float num = U.rhov2 + v3 * v3 + r * r - U.h2;
    const float den = 2.0f * r * U.rhov;
    const bool tiny = den <= 1e-6f;
    const float kappa = tiny ? (num > 0.0f ? 2.0f : -2.0f) : num * rcp_approx(den);
    bool empty = kappa >= 1.0f;
    bool full = kappa <= 0.0f;
    const float psiw = acos_approx(kappa) + 2e-4f;
    float plo = -psiw, phi = psiw;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float m = r * U.nrm[a];
        const bool degen = m < 1e-4f;
        const float inv = rcp_approx(fmaxf_(m, 1e-4f));
        const float x1 = (U.lo[a] - C[a]) * inv;
        const float x2 = (U.hi[a] - C[a]) * inv;
        const bool out = degen ? (C[a] + m < U.lo[a] || C[a] - m > U.hi[a])
                               : (x1 > 1.0f || x2 < -1.0f);
        const bool nocon = degen || (x1 <= -1.0f && x2 >= 1.0f);
        const float A1 = acos_approx(x2);   // smaller angle
        const float A2 = acos_approx(x1);   // larger angle
        const float g = U.gam[a];
        float lo_a = 1e30f, hi_a = -1e30f;
        // allowed psi - g in [A1, A2] U [-A2, -A1] (mod 2 pi), clipped to the window
#pragma unroll
        for (int sh = -1; sh <= 1; ++sh) {
            const float off = g + (float)sh * kTwoPi;
            const float a0 = fmaxf_(off + A1 - 2e-4f, plo), b0 = fminf_(off + A2 + 2e-4f, phi);
            const bool k0 = a0 <= b0;
            lo_a = k0 ? fminf_(lo_a, a0) : lo_a;
            hi_a = k0 ? fmaxf_(hi_a, b0) : hi_a;
            const float a1 = fmaxf_(off - A2 - 2e-4f, plo), b1 = fminf_(off - A1 + 2e-4f, phi);
            const bool k1 = a1 <= b1;
            lo_a = k1 ? fminf_(lo_a, a1) : lo_a;
            hi_a = k1 ? fmaxf_(hi_a, b1) : hi_a;
        }
        empty = empty || out || (!nocon && lo_a > hi_a);
        plo = nocon ? plo : fmaxf_(plo, lo_a);
        phi = nocon ? phi : fminf_(phi, hi_a);
    }
    empty = empty || (!full && plo > phi);
    const float f = (float)nj * kInvTwoPi;
    const int j0 = (int)floorf((U.phic + plo) * f) - 1;
    const int j1 = (int)ceilf((U.phic + phi) * f) + 1;
    const int c = j1 - j0 + 1;
    int m = j0 % nj;
    m = m < 0 ? m + nj : m;
    const bool whole = full || c >= nj;
    jlo = (empty || whole) ? 0 : m;
    cnt = empty ? 0 : (whole ? nj : c);
}

// Points of a ring are split into fixed segments of L consecutive indices;
// every point is evaluated relative to its segment's reference index, so a
// point's position is a function of (transducer, shell, ring, j) only.
OAT_HD int seg_shift(int nj)
{
    // L = 2^shift is the largest power of two <= nj/8 (at least 1, at most 32),
    // so a segment spans at most pi/8 of the ring about its reference.
    int e = nj >> 3, sh = 0;
    while (sh < 5 && (2 << sh) <= e) ++sh;
    return sh;
}

// cos and sin of 2 pi x for x in [0, 1), about 1 ulp: quarter-turn reduction
// (exact) and Taylor polynomials on [-pi/4, pi/4].
OAT_HD void sincos_turns(float x, float &c, float &s)
{
    float t = x * 4.0f;
    float qf = rintf(t);
    float y = t - qf;
    int q = ((int)qf) & 3;
    float z = y * 1.57079632679489661923f;
    float z2 = z * z;
    float sp = fmaf(z2, fmaf(z2, fmaf(z2, fmaf(z2, 2.7557319e-6f, -1.9841270e-4f),
                                      8.3333333e-3f), -1.6666667e-1f), 1.0f) * z;
    float cp = fmaf(z2, fmaf(z2, fmaf(z2, fmaf(z2, fmaf(z2, -2.7557319e-7f, 2.4801587e-5f),
                                                -1.3888889e-3f), 4.1666667e-2f), -0.5f), 1.0f);
    // Quadrant q: (cp, sp) turned by q quarter turns (selects only).
    const bool odd = (q & 1) != 0, neg = (q & 2) != 0;
    const float cc = odd ? -sp : cp, ss = odd ? cp : sp;
    c = neg ? -cc : cc;
    s = neg ? -ss : ss;
}

// FP64 cos and sin of 2 pi x for x in [0, 1), to a few units in the last
// place: exact quarter-turn reduction, then Taylor series on [-pi/4, pi/4]
// through z^15 (sin) and z^16 (cos); the first omitted terms are below 5e-17.
OAT_HD void sincos_turns_d(double x, double &c, double &s)
{
    double t = x * 4.0;
    double qf = rint(t);
    double y = t - qf;
    int q = ((int)qf) & 3;
    double z = y * 1.5707963267948966;
    double z2 = z * z;
    double sp = fma(z2, -7.6471637318198165e-13, 1.6059043836821613e-10);
    sp = fma(z2, sp, -2.5052108385441720e-08);
    sp = fma(z2, sp, 2.7557319223985891e-06);
    sp = fma(z2, sp, -1.9841269841269841e-04);
    sp = fma(z2, sp, 8.3333333333333333e-03);
    sp = fma(z2, sp, -1.6666666666666667e-01);
    sp = fma(z2 * z, sp, z);
    double cp = fma(z2, 4.7794773323873853e-14, -1.1470745597729725e-11);
    cp = fma(z2, cp, 2.0876756987868099e-09);
    cp = fma(z2, cp, -2.7557319223985891e-07);
    cp = fma(z2, cp, 2.4801587301587302e-05);
    cp = fma(z2, cp, -1.3888888888888889e-03);
    cp = fma(z2, cp, 4.1666666666666667e-02);
    cp = fma(z2, cp, -0.5);
    cp = fma(z2, cp, 1.0);
    // Quadrant q: (cos, sin) = (cp, sp) turned by q quarter turns, i.e.
    // swapped with a sign for odd q, both negated for q >= 2 (selects only).
    const bool odd = (q & 1) != 0, neg = (q & 2) != 0;
    const double cc = odd ? -sp : cp, ss = odd ? cp : sp;
    c = neg ? -cc : cc;
    s = neg ? -ss : ss;
}

// A small rotation d (|d| <= pi/8): cm1 = cos d - 1, sn = sin d, each a
// polynomial in d^2 with its leading term exact and the other two fitted for
// the least maximum relative error on (0, pi/8] (2.9e-8 for sin, 7.6e-9 for
// cos - 1, in FP64; fit_small_rot.py derives the coefficients).
OAT_HD void small_rot(float d, float &cm1, float &sn)
{
    float d2 = d * d;
    sn = fmaf(d2, fmaf(d2, 0.008290755f, -0.16666463f), 1.0f) * d;
    cm1 = fmaf(d2, fmaf(d2, -0.0013835691f, 0.04166641f), -0.5f) * d2;
}

}  // namespace oat
