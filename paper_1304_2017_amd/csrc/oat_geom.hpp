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
    U.phic = atan2f(V2, V1);
    float c = cosf(U.phic), s = sinf(U.phic);
    for (int a = 0; a < 3; ++a) {
        float E1 = c * e1[a] + s * e2[a];
        float E2 = -s * e1[a] + c * e2[a];
        U.nrm[a] = sqrtf(E1 * E1 + E2 * E2);
        U.gam[a] = atan2f(E2, E1);
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
    jlo = 0;
    cnt = 0;
    // Window of the ring inside the ball around the box: |p - cb|^2 =
    // rhov^2 + v3^2 + r^2 - 2 r rhov cos(psi), psi = phi - phic.
    float v3 = U.V3 - rc;
    float num = U.rhov2 + v3 * v3 + r * r - U.h2;
    float den = 2.0f * r * U.rhov;
    float psiw;
    if (den <= 1e-6f) {
        if (num > 0.0f) return;       // every ring point is farther than h
        cnt = nj;                     // ring inside the ball: take it whole
        return;
    }
    float kappa = num * rcp_approx(den);
    if (kappa >= 1.0f) return;
    if (kappa <= 0.0f) { cnt = nj; return; }   // wide window: whole ring
    psiw = acos_approx(kappa) + 2e-4f;
    float plo = -psiw, phi = psiw;
    const float Ca[3] = {C[0], C[1], C[2]};
    for (int a = 0; a < 3; ++a) {
        float m = r * U.nrm[a];
        if (m < 1e-4f) {
            if (Ca[a] + m < U.lo[a] || Ca[a] - m > U.hi[a]) return;
            continue;
        }
        float inv = rcp_approx(m);
        float x1 = (U.lo[a] - Ca[a]) * inv;
        float x2 = (U.hi[a] - Ca[a]) * inv;
        if (x1 > 1.0f || x2 < -1.0f) return;
        if (x1 <= -1.0f && x2 >= 1.0f) continue;
        float A1 = acos_approx(x2);   // smaller angle
        float A2 = acos_approx(x1);   // larger angle
        float g = U.gam[a];
        float lo_a = 1e30f, hi_a = -1e30f;
        // allowed psi - g in [A1, A2] U [-A2, -A1] (mod 2 pi), clipped to the window
        for (int sh = -1; sh <= 1; ++sh) {
            float off = g + (float)sh * kTwoPi;
            float a0 = fmaxf_(off + A1 - 2e-4f, plo), b0 = fminf_(off + A2 + 2e-4f, phi);
            if (a0 <= b0) { lo_a = fminf_(lo_a, a0); hi_a = fmaxf_(hi_a, b0); }
            float a1 = fmaxf_(off - A2 - 2e-4f, plo), b1 = fminf_(off - A1 + 2e-4f, phi);
            if (a1 <= b1) { lo_a = fminf_(lo_a, a1); hi_a = fmaxf_(hi_a, b1); }
        }
        if (lo_a > hi_a) return;
        plo = fmaxf_(plo, lo_a);
        phi = fminf_(phi, hi_a);
        if (plo > phi) return;
    }
    float f = (float)nj * kInvTwoPi;
    int j0 = (int)floorf((U.phic + plo) * f) - 1;
    int j1 = (int)ceilf((U.phic + phi) * f) + 1;
    int c = j1 - j0 + 1;
    if (c >= nj) { cnt = nj; return; }
    int m = j0 % nj;
    if (m < 0) m += nj;
    jlo = m;
    cnt = c;
}

// Points of a ring are split into fixed segments of L consecutive indices;
// every point is evaluated relative to its segment's reference index, so a
// point's position is a function of (transducer, shell, ring, j) only.
OAT_HD int seg_len(int nj)
{
    int L = nj >> 3;
    return L < 1 ? 1 : (L > 32 ? 32 : L);
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
    float cc, ss;
    switch (q) {
        case 0: cc = cp; ss = sp; break;
        case 1: cc = -sp; ss = cp; break;
        case 2: cc = -cp; ss = -sp; break;
        default: cc = sp; ss = -cp; break;
    }
    c = cc;
    s = ss;
}

// Taylor parts of a small rotation d (|d| <= pi/8): cm1 = cos d - 1, sn = sin d.
OAT_HD void small_rot(float d, float &cm1, float &sn)
{
    float d2 = d * d;
    sn = fmaf(d2, fmaf(d2, fmaf(d2, -1.9841270e-4f, 8.3333333e-3f), -1.6666667e-1f), 1.0f) * d;
    cm1 = fmaf(d2, fmaf(d2, fmaf(d2, 2.4801587e-5f, -1.3888889e-3f), 4.1666667e-2f), -0.5f) * d2;
}

}  // namespace oat
