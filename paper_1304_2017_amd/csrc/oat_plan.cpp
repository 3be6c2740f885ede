// Host side of liboat: geometry validation, FP64 quadrature tables, device
// workspace and the C-ABI entry points declared in include/oat.h.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "oat.h"
#include "oat_internal.hpp"
#include "oat_fbp_floor.hpp"
#include "oat_geom.hpp"

using namespace oat;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int fail_hip(hipError_t e, const char *where)
{
    g_last_error = std::string(where) + ": " + hipGetErrorName(e) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? OAT_ERR_NOMEM : OAT_ERR_DEVICE;
}

// Transducer local frame (Appendix, Fig. geo(b)): z^tr from r_q to the origin.
void frame(const double *r, double e1[3], double e2[3], double e3[3], double *dist)
{
    double d = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    double th = std::acos(r[2] / d);
    double ph = std::atan2(r[1], r[0]);
    e3[0] = -r[0] / d;
    e3[1] = -r[1] / d;
    e3[2] = -r[2] / d;
    e1[0] = std::cos(th) * std::cos(ph);
    e1[1] = std::cos(th) * std::sin(ph);
    e1[2] = -std::sin(th);
    e2[0] = std::sin(ph);
    e2[1] = -std::cos(ph);
    e2[2] = 0.0;
    *dist = d;
}

bool is_fin(double v) { return std::isfinite(v); }

}  // namespace

struct oat_plan {
    int device = 0;
    int nx = 0, ny = 0, nz = 0, nq = 0, nt = 0;
    Problem P{};
    DetRec *d_det = nullptr;
    ShellRec *d_shell = nullptr;
    RingRec *d_ring = nullptr;
    float *d_part = nullptr;     // G windows [bricks][Q][window]
    int *d_klo = nullptr;        // [bricks][Q]
    float *d_gp = nullptr;       // D^T y  [Q][K]
    double *d_acc = nullptr;     // G^T brick node sums [bricks][BOX^3]
    float *d_rowmax = nullptr;   // [Q] max reachable |D^T y| per transducer
    float *d_adjr = nullptr;     // [bricks][windows] G^T calibration
    double *d_fbp_thr = nullptr; // [K + 2] FBP floor thresholds (Problem::fbp_thr)
    double2 *d_segref = nullptr; // segment reference azimuths (Problem::segref)
    double4 *d_sph_pts = nullptr; // transducer face nodes (Problem::sph_pts)
    std::vector<DetRec> det;      // host copy of the transducer records
    double ap_w = 0.0, ap_h = 0.0;   // face of oat_plan_set_aperture (0: point-like)
    int ap_m = 0;
    long long *d_tab_off = nullptr;   // arc table (see Problem)
    unsigned *d_tab_run = nullptr;
    unsigned *d_tab_arc = nullptr;
    double *d_eir_h = nullptr;        // EIR taps [eir_taps]
    double2 *d_eir_spec = nullptr;    // transform of the delayed EIR [eir_n]
    double2 *d_eir_tw = nullptr;      // FFT twiddles [eir_n / 2]
    double2 *d_eir_filt = nullptr;    // deconvolution filter of a call [eir_n]
    float *d_eirbuf = nullptr;        // D G img before H^e / H^e^T y before D^T  [Q][K]
    int eir_taps = 0, eir_n = 0;
    double2 *d_sph_part = nullptr;    // spherical-voxel workspace (chunk / slice sums)
    size_t sph_part_bytes = 0;
    long long *d_seg_off = nullptr;   // segment table (see Problem)
    unsigned *d_seg = nullptr;
    int64_t tab_bytes = 0, tab_entries = 0, tab_build_us = 0, calib_us = 0;
    int64_t seg_bytes = 0, seg_entries = 0, seg_build_us = 0;
    int max_nj = 0, max_rings = 0;
    float w_max = 0.f;
    int64_t n_rings = 0;
    int64_t ws_bytes = 0, table_bytes = 0;
};

namespace {

// Gauss-Legendre nodes x and weights w on [-1, 1] (m points): the roots of
// P_m by Newton's method from cos(pi (i + 3/4) / (m + 1/2)), P_m and P_m'
// from the three-term recurrence, w = 2 / ((1 - x^2) P_m'(x)^2).
void gauss_legendre(int m, double *x, double *w)
{
    for (int i = 0; i < m; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (m + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p1 = 1.0, p0 = 0.0;
            for (int j = 1; j <= m; ++j) {
                const double pm = p0;
                p0 = p1;
                p1 = ((2.0 * j - 1.0) * z * p0 - (j - 1.0) * pm) / j;
            }
            dp = m * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) <= 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Face nodes of every transducer (see Problem::sph_pts): with m = 0 the
// point r_q with weight 1; else the m x m Gauss-Legendre nodes of the
// width x height rectangle centred at r_q, its width along the frame's e1
// (polar direction) and height along e2, weights summing to 1.
std::vector<double4> face_nodes(const std::vector<DetRec> &det, double width, double height, int m)
{
    const int S = m > 0 ? m * m : 1;
    std::vector<double4> pts(det.size() * (size_t)S);
    std::vector<double> x(m > 0 ? m : 1), w(m > 0 ? m : 1);
    if (m > 0) gauss_legendre(m, x.data(), w.data());
    for (size_t q = 0; q < det.size(); ++q) {
        const DetRec &d = det[q];
        if (m == 0) {
            pts[q] = make_double4(d.r[0], d.r[1], d.r[2], 1.0);
            continue;
        }
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                const double a = 0.5 * width * x[i], b = 0.5 * height * x[j];
                pts[q * S + i * m + j] =
                    make_double4(d.r[0] + a * d.e1d[0] + b * d.e2d[0],
                                 d.r[1] + a * d.e1d[1] + b * d.e2d[1],
                                 d.r[2] + a * d.e1d[2] + b * d.e2d[2], 0.25 * w[i] * w[j]);
            }
    }
    return pts;
}

// Arc table of a plan (see Problem): the count pass, an exclusive prefix sum
// of the per-unit counts on the host, the fill pass.  budget < 0: up to 40%
// of the device memory free now.  A table that does not fit, or a geometry
// whose ring indices exceed 16 bits, leaves the plan without one (kernels
// then bound the arcs themselves); a failing launch fails the plan.
int build_arc_table(oat_plan *plan, int64_t budget)
{
    Problem &P = plan->P;
    if (plan->max_nj > 65535 || plan->max_rings > 65535) return OAT_OK;
    if (budget < 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return OAT_OK;
        budget = (int64_t)(0.4 * (double)fr);
    }
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t units = (int64_t)P.nbx * P.nby * P.nbz * P.nq;
    const size_t run_b = sizeof(unsigned) * (size_t)units * P.window;
    const size_t off_b = sizeof(long long) * (size_t)units;
    const size_t cnt_b = sizeof(int) * (size_t)units;
    if ((int64_t)(run_b + off_b + cnt_b) > budget) return OAT_OK;
    unsigned *run = nullptr;
    long long *off = nullptr;
    int *cnt = nullptr;
    unsigned *arc = nullptr;
    auto release = [&]() {
        if (run) (void)hipFree(run);
        if (off) (void)hipFree(off);
        if (cnt) (void)hipFree(cnt);
        if (arc) (void)hipFree(arc);
        run = nullptr;
        off = nullptr;
        cnt = nullptr;
        arc = nullptr;
    };
    if (hipMalloc((void **)&run, run_b) != hipSuccess || hipMalloc((void **)&off, off_b) != hipSuccess ||
        hipMalloc((void **)&cnt, cnt_b) != hipSuccess) {
        release();
        (void)hipGetLastError();
        return OAT_OK;
    }
    hipError_t e = hipMemset(run, 0, run_b);
    Problem Pc = P;
    Pc.tab_run = run;
    Pc.tab_cnt = cnt;
    if (e == hipSuccess) e = launch_arc_build(Pc, 0, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    std::vector<int> hcnt(units);
    if (e == hipSuccess) e = hipMemcpy(hcnt.data(), cnt, cnt_b, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        release();
        return fail_hip(e, "oat_plan_create: arc table count pass");
    }
    std::vector<long long> hoff(units);
    long long total = 0;
    for (int64_t u = 0; u < units; ++u) {
        hoff[u] = total;
        total += hcnt[u];
    }
    const size_t arc_b = sizeof(unsigned) * (size_t)(total > 0 ? total : 1);
    if ((int64_t)(run_b + off_b + arc_b) > budget || hipMalloc((void **)&arc, arc_b) != hipSuccess) {
        release();
        (void)hipGetLastError();
        return OAT_OK;
    }
    (void)hipFree(cnt);
    cnt = nullptr;
    e = hipMemcpy(off, hoff.data(), off_b, hipMemcpyHostToDevice);
    Pc.tab_cnt = nullptr;
    Pc.tab_off = off;
    Pc.tab_arc = arc;
    if (e == hipSuccess) e = launch_arc_build(Pc, 1, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        release();
        return fail_hip(e, "oat_plan_create: arc table fill pass");
    }
    plan->d_tab_run = run;
    plan->d_tab_off = off;
    plan->d_tab_arc = arc;
    P.tab_run = run;
    P.tab_off = off;
    P.tab_arc = arc;
    P.tab_cnt = nullptr;
    plan->tab_bytes = (int64_t)(run_b + off_b + arc_b);
    plan->tab_entries = total;
    plan->tab_build_us = (int64_t)std::chrono::duration_cast<std::chrono::microseconds>(
                             std::chrono::steady_clock::now() - t0).count();
    return OAT_OK;
}

// Segment table, built over the bounds walk (no arc table needed): a count
// pass (segments per unit and per point count, and a flag for segments that
// do not fit the compact entry), the host prefix sum, a fill pass that
// writes each unit's entries ordered by decreasing count.  Skipped (OAT_OK,
// no table) when it does not fit the budget (< 0: 40% of the device memory
// free now) or when a segment does not fit its entry; a failing launch fails
// the plan.
int build_seg_table(oat_plan *plan, int64_t budget)
{
    Problem &P = plan->P;
    if (plan->max_nj > 65535 || plan->max_rings > 65535) return OAT_OK;
    if (budget < 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return OAT_OK;
        budget = (int64_t)(0.4 * (double)fr);
    }
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t units = (int64_t)P.nbx * P.nby * P.nbz * P.nq;
    const size_t cnt_b = sizeof(int) * (size_t)units;
    const size_t hist_b = sizeof(int) * 32 * (size_t)units;
    const size_t off_b = sizeof(long long) * (size_t)(units + 1);
    if ((int64_t)(cnt_b + hist_b + off_b) > budget) return OAT_OK;
    int *cnt = nullptr, *hist = nullptr, *flag = nullptr;
    long long *off = nullptr;
    unsigned *seg = nullptr;
    auto release = [&]() {
        for (void *b : {(void *)cnt, (void *)hist, (void *)flag, (void *)off, (void *)seg})
            if (b) (void)hipFree(b);
        cnt = hist = flag = nullptr;
        off = nullptr;
        seg = nullptr;
    };
    if (hipMalloc((void **)&cnt, cnt_b) != hipSuccess ||
        hipMalloc((void **)&hist, hist_b) != hipSuccess ||
        hipMalloc((void **)&flag, sizeof(int)) != hipSuccess) {
        release();
        (void)hipGetLastError();
        return OAT_OK;
    }
    Problem Pc = P;
    Pc.seg_cnt = cnt;
    Pc.seg_hist = hist;
    Pc.seg_flag = flag;
    hipError_t e = hipMemset(flag, 0, sizeof(int));
    if (e == hipSuccess) e = launch_arc_build(Pc, 2, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    std::vector<int> hcnt(units);
    int hflag = 0;
    if (e == hipSuccess) e = hipMemcpy(hcnt.data(), cnt, cnt_b, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        release();
        return fail_hip(e, "oat_plan_create: segment table count pass");
    }
    if (hflag != 0) {   // a segment does not fit the compact entry
        release();
        return OAT_OK;
    }
    std::vector<long long> hoff(units + 1);
    long long total = 0;
    for (int64_t u = 0; u < units; ++u) {
        hoff[u] = total;
        total += hcnt[u];
    }
    hoff[units] = total;
    (void)hipFree(cnt);
    cnt = nullptr;
    const size_t seg_b = sizeof(unsigned) * (size_t)(total > 0 ? total : 1);
    if ((int64_t)(seg_b + hist_b + off_b) > budget || hipMalloc((void **)&off, off_b) != hipSuccess ||
        hipMalloc((void **)&seg, seg_b) != hipSuccess) {
        release();
        (void)hipGetLastError();
        return OAT_OK;
    }
    e = hipMemcpy(off, hoff.data(), off_b, hipMemcpyHostToDevice);
    Pc.seg_cnt = nullptr;
    Pc.seg_off = off;
    Pc.seg = seg;
    if (e == hipSuccess) e = launch_arc_build(Pc, 3, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        release();
        return fail_hip(e, "oat_plan_create: segment table fill pass");
    }
    (void)hipFree(hist);
    (void)hipFree(flag);
    hist = flag = nullptr;
    plan->d_seg_off = off;
    plan->d_seg = seg;
    P.seg_off = off;
    P.seg = seg;
    P.seg_cnt = nullptr;
    P.seg_hist = nullptr;
    P.seg_flag = nullptr;
    plan->seg_bytes = (int64_t)(seg_b + off_b);
    plan->seg_entries = total;
    plan->seg_build_us = (int64_t)std::chrono::duration_cast<std::chrono::microseconds>(
                             std::chrono::steady_clock::now() - t0).count();
    return OAT_OK;
}

}  // namespace

void oat::set_last_error(const char *msg) { g_last_error = msg ? msg : ""; }

extern "C" {

const char *oat_last_error(void) { return g_last_error.c_str(); }

void oat_plan_destroy(oat_plan *plan)
{
    if (!plan) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(plan->device);
    void *bufs[] = {plan->d_det, plan->d_shell, plan->d_ring, plan->d_part,
                    plan->d_klo, plan->d_gp, plan->d_acc, plan->d_rowmax, plan->d_adjr,
                    plan->d_tab_off, plan->d_tab_run, plan->d_tab_arc, plan->d_seg_off,
                    plan->d_seg, plan->d_eir_h, plan->d_eir_spec, plan->d_eir_tw,
                    plan->d_eir_filt, plan->d_eirbuf, plan->d_sph_part, plan->d_fbp_thr,
                    plan->d_segref, plan->d_sph_pts};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    (void)hipSetDevice(prev);
    delete plan;
}

int oat_plan_create(const oat_geometry *g, int device, oat_plan **out)
{
    return oat_plan_create_ex(g, device, nullptr, out);
}

int oat_plan_create_ex(const oat_geometry *g, int device, const oat_plan_options *opt,
                       oat_plan **out)
{
    g_last_error.clear();
    if (!g || !out) return fail(OAT_ERR_ARG, "oat_plan_create: null argument");
    const int64_t table_budget = opt ? opt->arc_table_bytes : -1;
    if (table_budget < -1) return fail(OAT_ERR_ARG, "arc_table_bytes must be >= -1");
    const int64_t seg_budget = opt ? opt->segment_table_bytes : -1;
    if (seg_budget < -1) return fail(OAT_ERR_ARG, "segment_table_bytes must be >= -1");
    *out = nullptr;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1)
        return fail(OAT_ERR_GEOMETRY, "grid sizes must be >= 1");
    if (!(g->dx > 0.0) || !is_fin(g->dx)) return fail(OAT_ERR_GEOMETRY, "dx must be > 0");
    if (!is_fin(g->x0) || !is_fin(g->y0) || !is_fin(g->z0))
        return fail(OAT_ERR_GEOMETRY, "grid origin must be finite");
    if (g->n_det < 1 || !g->det_xyz) return fail(OAT_ERR_ARG, "need n_det >= 1 and det_xyz");
    if (g->n_t < 3) return fail(OAT_ERR_GEOMETRY, "n_t must be >= 3");
    if (!(g->dt > 0.0) || !is_fin(g->dt)) return fail(OAT_ERR_GEOMETRY, "dt must be > 0");
    if (!is_fin(g->t0)) return fail(OAT_ERR_GEOMETRY, "t0 must be finite");
    if (!(g->c0 > 0.0) || !is_fin(g->c0)) return fail(OAT_ERR_GEOMETRY, "c0 must be > 0");
    if (!(g->gamma > 0.0) || !is_fin(g->gamma)) return fail(OAT_ERR_GEOMETRY, "gamma must be > 0");
    const int64_t N = (int64_t)g->nx * g->ny * g->nz;
    if (N >= (1ll << 31) || (int64_t)g->n_det * g->n_t >= (1ll << 31))
        return fail(OAT_ERR_GEOMETRY, "image or data larger than 2^31 elements");
    if (g->n_t > 4096)
        return fail(OAT_ERR_GEOMETRY, "n_t must be <= 4096");
    if (g->t0 + (g->n_t - 1) * g->dt <= 0.0)
        return fail(OAT_ERR_GEOMETRY, "all sample times are <= 0");

    const int Q = g->n_det, K = g->n_t;
    const double dx = g->dx;
    // Support radius: farthest corner of [x0-dx, x0+nx*dx] x ... (Sec. III.A).
    double lo[3] = {g->x0 - dx, g->y0 - dx, g->z0 - dx};
    double hi[3] = {g->x0 + g->nx * dx, g->y0 + g->ny * dx, g->z0 + g->nz * dx};
    double R2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double m = std::fmax(std::fabs(lo[a]), std::fabs(hi[a]));
        R2 += m * m;
    }
    const double R = std::sqrt(R2);

    std::vector<DetRec> det(Q);
    double dmin = 1e300, dmax = 0.0;
    for (int q = 0; q < Q; ++q) {
        const double *r = g->det_xyz + 3 * (size_t)q;
        if (!is_fin(r[0]) || !is_fin(r[1]) || !is_fin(r[2]))
            return fail(OAT_ERR_GEOMETRY, "transducer position not finite");
        double e1[3], e2[3], e3[3], d;
        frame(r, e1, e2, e3, &d);
        if (!(d > R)) {
            char buf[160];
            std::snprintf(buf, sizeof buf,
                          "transducer %d at distance %.6g mm lies inside the support sphere "
                          "(radius %.6g mm)", q, d, R);
            return fail(OAT_ERR_GEOMETRY, buf);
        }
        if (g->det_area && !(g->det_area[q] >= 0.0 && is_fin(g->det_area[q])))
            return fail(OAT_ERR_GEOMETRY, "patch areas must be finite and >= 0");
        dmin = std::fmin(dmin, d);
        dmax = std::fmax(dmax, d);
        DetRec &D = det[q];
        D.uq[0] = (r[0] - g->x0) / dx;
        D.uq[1] = (r[1] - g->y0) / dx;
        D.uq[2] = (r[2] - g->z0) / dx;
        for (int a = 0; a < 3; ++a) {
            D.e3[a] = e3[a];
            D.e1d[a] = e1[a];
            D.e2d[a] = e2[a];
            D.e1[a] = (float)e1[a];
            D.e2[a] = (float)e2[a];
            D.uqf[a] = (float)D.uq[a];
        }
        D.dist = (float)(d / dx);
        double area = g->det_area ? g->det_area[q] : 4.0 * M_PI * d * d / Q;
        D.fbp_w = (float)(area / d);
        D.pad = 0.f;
        D.r[0] = r[0];
        D.r[1] = r[1];
        D.r[2] = r[2];
        D.pad2 = 0.0;
    }

    // Quadrature tables in FP64 (Appendix; bands of arc length dx from the pole).
    std::vector<ShellRec> shell(K);
    std::vector<RingRec> ring;
    int max_nj = 0, max_rings = 0;
    float w_max = 0.f;
    for (int k = 0; k < K; ++k) {
        double rho = g->c0 * (g->t0 + k * g->dt);
        ShellRec &S = shell[k];
        S.ring_base = (int32_t)ring.size();
        S.n_rings = 0;
        S.rho = (float)(rho / dx);
        S.inv_rho = rho > 0.0 ? (float)(dx / rho) : 0.f;
        if (!(rho > 0.0) || rho < dmin - R || rho > dmax + R) continue;
        double dth = dx / rho;
        long nring = (long)std::ceil(M_PI / dth);
        if ((int64_t)ring.size() + nring >= (1ll << 31))
            return fail(OAT_ERR_GEOMETRY, "quadrature tables exceed 2^31 rings");
        S.n_rings = (int32_t)nring;
        if (nring > max_rings) max_rings = (int)nring;
        for (long i = 0; i < nring; ++i) {
            double tlo = i * dth;
            double thi = (i + 1) * dth;
            if (thi > M_PI) thi = M_PI;
            double th = 0.5 * (tlo + thi);
            double area = 2.0 * M_PI * rho * rho * (std::cos(tlo) - std::cos(thi));
            long nj = (long)std::floor(2.0 * M_PI * rho * std::sin(th) / dx + 0.5);
            if (nj < 1) nj = 1;
            RingRec rr;
            rr.rc = rho * std::cos(th) / dx;
            rr.rs = rho * std::sin(th) / dx;
            rr.rsf = (float)rr.rs;
            rr.nj = (int32_t)nj;
            rr.w = (float)(area / (double)nj);
            rr.delta = (float)(2.0 * M_PI / (double)nj);
            rr.lshift = seg_shift((int)nj);
            rr.sref = 0;   // set below, once every ring size is known
            if (nj > max_nj) max_nj = (int)nj;
            if (rr.w > w_max) w_max = rr.w;
            ring.push_back(rr);
        }
    }
    if (ring.empty()) ring.push_back(RingRec{0.0, 0.0, 0.f, 1, 0.f, 0.f, 0, 0});
    if (max_nj < 1) max_nj = 1;
    // Segment reference azimuths in FP64 per ring size: every segment of
    // every ring of nj points starts from (cos, sin) of 2 pi jref / nj, so
    // the kernels evaluate no FP64 sine.  The reduction to [0, 1/8] turn is
    // exact in integers; the octant's sine and cosine come from long double.
    std::vector<int32_t> sref_of(max_nj + 1, 0);
    std::vector<double2> segref;
    for (int nj = 1; nj <= max_nj; ++nj) {
        sref_of[nj] = (int32_t)segref.size();
        const int ls = seg_shift(nj), nseg = (nj + (1 << ls) - 1) >> ls;
        for (int sg = 0; sg < nseg; ++sg) {
            const int64_t j = seg_ref_index(sg, ls, nj);
            // 2 pi j / nj = (pi/4) (m + r) with m = floor(8 j / nj) and r in [0, 1)
            const int64_t m = (8 * j) / nj, rn = 8 * j - m * nj;   // r = rn / nj
            const long double qa = (long double)M_PI / 4.0L;
            // angle within the octant, measured from the octant's even edge
            const bool odd = (m & 1) != 0;
            const long double a = qa * (long double)(odd ? nj - rn : rn) / (long double)nj;
            long double c = std::cos(a), sn = std::sin(a);
            // octant m spans [m pi/4, (m+1) pi/4]; odd octants measure from
            // the upper edge, so reflect about the diagonal first
            long double cc = odd ? sn : c, ss = odd ? c : sn;
            // rotate by the quarter turns m / 2
            for (int t = 0; t < (int)(m / 2); ++t) {
                const long double tc = -ss;
                ss = cc;
                cc = tc;
            }
            segref.push_back(make_double2((double)cc, (double)ss));
        }
    }
    for (RingRec &rr : ring) rr.sref = sref_of[rr.nj];

    oat_plan *plan = new (std::nothrow) oat_plan();
    if (!plan) return fail(OAT_ERR_NOMEM, "host allocation failed");
    plan->device = device;
    plan->nx = g->nx;
    plan->ny = g->ny;
    plan->nz = g->nz;
    plan->nq = Q;
    plan->nt = K;
    plan->n_rings = (int64_t)ring.size();
    plan->max_nj = max_nj;
    plan->max_rings = max_rings;

    Problem &P = plan->P;
    P.nx = g->nx;
    P.ny = g->ny;
    P.nz = g->nz;
    P.nq = Q;
    P.nt = K;
    P.nbx = (g->nx + BRICK - 1) / BRICK;
    P.nby = (g->ny + BRICK - 1) / BRICK;
    P.nbz = (g->nz + BRICK - 1) / BRICK;
    P.rho0 = (float)(g->c0 * g->t0 / dx);
    P.rho_step = (float)(g->c0 * g->dt / dx);
    {
        // Widest shell range seen by a brick: the cell box spans BRICK+1 cells.
        double diag = std::sqrt(3.0) * (BRICK + 1) + 0.2;
        int w = (int)std::ceil(diag / (g->c0 * g->dt / dx)) + 3;
        if (w > K) w = K;
        if (w > WMAX) {
            delete plan;
            return fail(OAT_ERR_GEOMETRY, "c0*dt/dx too small: shell window exceeds the kernel limit");
        }
        P.window = w;
    }
    P.w_max = w_max;
    P.r_sup = (float)(R / dx);
    P.t0 = (float)g->t0;
    P.dt = (float)g->dt;
    P.d_coef = (float)(g->gamma / (4.0 * M_PI * g->c0 * g->c0) / (2.0 * g->dt));
    P.fbp_scale = (float)(-1.0 / (M_PI * g->gamma * g->c0 * g->dt));
    P.sigma = (float)(dx / (g->c0 * g->dt));
    P.inv_sigma = (float)(g->c0 * g->dt / dx);
    P.tau = (float)(g->t0 / g->dt);
    P.x0 = g->x0;
    P.y0 = g->y0;
    P.z0 = g->z0;
    P.dxd = dx;
    P.c0d = g->c0;
    P.t0d = g->t0;
    P.dtd = g->dt;
    P.gammad = g->gamma;

    const int nbricks = P.nbx * P.nby * P.nbz;

    int prev = 0;
    (void)hipGetDevice(&prev);
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) {
        delete plan;
        return fail_hip(e, "hipSetDevice");
    }
    {
        // Resolve this device's fixed scratch (oat_sph_backproject_noalloc)
        // while the device is current; later plans reuse the cached address.
        double *scr = nullptr;
        if ((e = sph_scratch_address(device, &scr)) != hipSuccess) {
            delete plan;
            (void)hipSetDevice(prev);
            return fail_hip(e, "oat_plan_create: hipGetSymbolAddress(scratch)");
        }
    }
    auto alloc = [&](void **p, size_t bytes, const char *what) -> hipError_t {
        hipError_t err = hipMalloc(p, bytes < 16 ? 16 : bytes);
        if (err != hipSuccess) g_last_error = std::string("hipMalloc ") + what;
        return err;
    };
    size_t det_b = sizeof(DetRec) * Q, sh_b = sizeof(ShellRec) * K,
           ring_b = sizeof(RingRec) * ring.size();
    size_t part_b = sizeof(float) * (size_t)nbricks * Q * P.window;
    size_t klo_b = sizeof(int) * (size_t)nbricks * Q;
    size_t gp_b = sizeof(float) * (size_t)Q * K;
    // G^T brick node sums, one set per slice of the transducer windows
    size_t acc_b = sizeof(double) * (size_t)adj_slices(nbricks, Q) * nbricks * BOX3;
    size_t rowmax_b = sizeof(float) * (size_t)Q;
    size_t adjr_b = sizeof(float) * (size_t)nbricks * adj_windows(Q);
    const std::vector<double> fbp_thr = fbp_floor_thresholds(g->c0, g->t0, g->dt, K);
    size_t thr_b = sizeof(double) * fbp_thr.size();
    size_t segref_b = sizeof(double2) * segref.size();
    const std::vector<double4> faces = face_nodes(det, 0.0, 0.0, 0);
    size_t faces_b = sizeof(double4) * faces.size();
    if ((e = alloc((void **)&plan->d_det, det_b, "det")) != hipSuccess ||
        (e = alloc((void **)&plan->d_shell, sh_b, "shell")) != hipSuccess ||
        (e = alloc((void **)&plan->d_ring, ring_b, "ring")) != hipSuccess ||
        (e = alloc((void **)&plan->d_part, part_b, "partials")) != hipSuccess ||
        (e = alloc((void **)&plan->d_klo, klo_b, "klo")) != hipSuccess ||
        (e = alloc((void **)&plan->d_gp, gp_b, "gp")) != hipSuccess ||
        (e = alloc((void **)&plan->d_acc, acc_b, "brick node sums")) != hipSuccess ||
        (e = alloc((void **)&plan->d_rowmax, rowmax_b, "gp row max")) != hipSuccess ||
        (e = alloc((void **)&plan->d_adjr, adjr_b, "G^T calibration")) != hipSuccess ||
        (e = alloc((void **)&plan->d_fbp_thr, thr_b, "FBP floor thresholds")) != hipSuccess ||
        (e = alloc((void **)&plan->d_segref, segref_b, "segment references")) != hipSuccess ||
        (e = alloc((void **)&plan->d_sph_pts, faces_b, "transducer faces")) != hipSuccess) {
        int code = fail_hip(e, "oat_plan_create: hipMalloc");
        oat_plan_destroy(plan);
        (void)hipSetDevice(prev);
        return code;
    }
    if ((e = hipMemcpy(plan->d_det, det.data(), det_b, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(plan->d_shell, shell.data(), sh_b, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(plan->d_ring, ring.data(), ring_b, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(plan->d_fbp_thr, fbp_thr.data(), thr_b, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(plan->d_segref, segref.data(), segref_b, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(plan->d_sph_pts, faces.data(), faces_b, hipMemcpyHostToDevice)) !=
            hipSuccess) {
        int code = fail_hip(e, "oat_plan_create: hipMemcpy");
        oat_plan_destroy(plan);
        (void)hipSetDevice(prev);
        return code;
    }
    P.det = plan->d_det;
    P.shell = plan->d_shell;
    P.ring = plan->d_ring;
    P.gp_rowmax = plan->d_rowmax;
    P.fbp_thr = plan->d_fbp_thr;
    P.segref = plan->d_segref;
    P.n_rings = (int)ring.size();
    P.n_segref = (int)segref.size();
    P.sph_pts = plan->d_sph_pts;
    P.sph_ns = 1;
    plan->det = det;
    P.adj_r = nullptr;
    P.tab_off = nullptr;
    P.tab_run = nullptr;
    P.tab_arc = nullptr;
    P.tab_cnt = nullptr;
    P.seg_off = nullptr;
    P.seg = nullptr;
    P.seg_cnt = nullptr;
    P.seg_hist = nullptr;
    P.seg_flag = nullptr;
    plan->ws_bytes = (int64_t)(part_b + klo_b + gp_b + acc_b + rowmax_b);
    plan->table_bytes = (int64_t)(det_b + sh_b + ring_b + adjr_b + thr_b + segref_b + faces_b);
    {
        // The segment table if it fits, else the arc table if that fits,
        // else neither (the kernels then bound the arcs themselves).
        int code = OAT_OK;
        if (seg_budget != 0) code = build_seg_table(plan, seg_budget);
        if (code == OAT_OK && !plan->d_seg && table_budget != 0)
            code = build_arc_table(plan, table_budget);
        if (code != OAT_OK) {
            oat_plan_destroy(plan);
            (void)hipSetDevice(prev);
            return code;
        }
    }
    {
        // G^T calibration: per (brick, transducer window) the largest node
        // sum of psi w, which bounds the fixed-point fields of every call.
        const auto t0 = std::chrono::steady_clock::now();
        e = launch_adj_calibrate(plan->P, plan->d_adjr, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            int code = fail_hip(e, "oat_plan_create: G^T calibration");
            oat_plan_destroy(plan);
            (void)hipSetDevice(prev);
            return code;
        }
        plan->P.adj_r = plan->d_adjr;
        plan->calib_us = (int64_t)std::chrono::duration_cast<std::chrono::microseconds>(
                             std::chrono::steady_clock::now() - t0).count();
    }
    (void)hipSetDevice(prev);
    *out = plan;
    return OAT_OK;
}

int oat_plan_stats(const oat_plan *plan, int64_t *stats, int n)
{
    if (!plan || !stats || n < 0) return fail(OAT_ERR_ARG, "oat_plan_stats: null argument");
    int64_t v[13] = {plan->n_rings, (int64_t)plan->P.nbx * plan->P.nby * plan->P.nbz, BRICK,
                     plan->P.window, plan->ws_bytes, plan->table_bytes, plan->tab_bytes,
                     plan->tab_entries, plan->tab_build_us, plan->calib_us, plan->seg_bytes,
                     plan->seg_entries, plan->seg_build_us};
    for (int i = 0; i < n && i < 13; ++i) stats[i] = v[i];
    return OAT_OK;
}

static int check_common(oat_plan *plan, const void *a, int adt, const void *b, int bdt,
                        uint32_t flags, uint32_t allowed, const char *who)
{
    if (!plan) return fail(OAT_ERR_ARG, std::string(who) + ": null plan");
    if (!a || !b) return fail(OAT_ERR_ARG, std::string(who) + ": null buffer");
    if (a == b) return fail(OAT_ERR_ARG, std::string(who) + ": input and output alias");
    if ((adt != OAT_F32 && adt != OAT_BF16) || (bdt != OAT_F32 && bdt != OAT_BF16))
        return fail(OAT_ERR_DTYPE, std::string(who) + ": unknown dtype");
    if (flags & ~allowed) return fail(OAT_ERR_ARG, std::string(who) + ": unknown flag");
    return OAT_OK;
}

static int with_device(oat_plan *plan, int &prev)
{
    (void)hipGetDevice(&prev);
    hipError_t e = hipSetDevice(plan->device);
    if (e != hipSuccess) return fail_hip(e, "hipSetDevice");
    return OAT_OK;
}

int oat_project(oat_plan *plan, const void *img, oat_dtype img_dtype, void *data,
                oat_dtype data_dtype, uint32_t flags, void *stream)
{
    int rc = check_common(plan, img, img_dtype, data, data_dtype, flags,
                          OAT_FLAG_SRT_ONLY | OAT_FLAG_DETERMINISTIC, "oat_project");
    if (rc) return rc;
    int prev;
    if ((rc = with_device(plan, prev))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const bool srt_only = (flags & OAT_FLAG_SRT_ONLY) != 0;
    const bool eir = plan->eir_taps > 0 && !srt_only;
    hipError_t e = launch_srt_fwd(plan->P, img, (int)img_dtype, plan->d_part, plan->d_klo, s);
    if (e == hipSuccess)
        e = launch_srt_reduce(plan->P, plan->d_part, plan->d_klo, eir ? plan->d_eirbuf : data,
                              eir ? 0 : (int)data_dtype, srt_only ? 0 : 1, s);
    if (e == hipSuccess && eir)
        e = launch_eir(plan->P, plan->d_eirbuf, 0, data, (int)data_dtype, plan->d_eir_h,
                       plan->eir_taps, 0, s);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) return fail_hip(e, "oat_project: launch");
    return OAT_OK;
}

int oat_backproject(oat_plan *plan, const void *data, oat_dtype data_dtype, void *img,
                    oat_dtype img_dtype, uint32_t flags, void *stream)
{
    int rc = check_common(plan, data, data_dtype, img, img_dtype, flags,
                          OAT_FLAG_SRT_ONLY | OAT_FLAG_DETERMINISTIC,
                          "oat_backproject");
    if (rc) return rc;
    int prev;
    if ((rc = with_device(plan, prev))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const bool srt_only = (flags & OAT_FLAG_SRT_ONLY) != 0;
    const bool eir = plan->eir_taps > 0 && !srt_only;
    hipError_t e = hipSuccess;
    if (eir)
        e = launch_eir(plan->P, data, (int)data_dtype, plan->d_eirbuf, 0, plan->d_eir_h,
                       plan->eir_taps, 1, s);
    if (e == hipSuccess)
        e = launch_diff_adj(plan->P, eir ? (const void *)plan->d_eirbuf : data,
                            eir ? 0 : (int)data_dtype, plan->d_gp, srt_only ? 0 : 1, s);
    if (e == hipSuccess)
        e = launch_srt_adj(plan->P, plan->d_gp, plan->d_acc, img, (int)img_dtype, s);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) return fail_hip(e, "oat_backproject: launch");
    return OAT_OK;
}

int oat_fbp(oat_plan *plan, const void *pres, oat_dtype pres_dtype, void *img, oat_dtype img_dtype,
            uint32_t flags, void *stream)
{
    int rc = check_common(plan, pres, pres_dtype, img, img_dtype, flags, OAT_FLAG_DETERMINISTIC,
                          "oat_fbp");
    if (rc) return rc;
    int prev;
    if ((rc = with_device(plan, prev))) return rc;
    hipError_t e = launch_fbp(plan->P, pres, (int)pres_dtype, img, (int)img_dtype,
                              (hipStream_t)stream);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) return fail_hip(e, "oat_fbp: launch");
    return OAT_OK;
}

int oat_plan_set_eir(oat_plan *plan, const double *h, int n_taps)
{
    if (!plan) return fail(OAT_ERR_ARG, "oat_plan_set_eir: null plan");
    if (n_taps < 0 || n_taps > plan->P.nt || (n_taps > 0 && !h))
        return fail(OAT_ERR_ARG, "oat_plan_set_eir: need 0 <= n_taps <= n_t and taps");
    for (int m = 0; m < n_taps; ++m)
        if (!std::isfinite(h[m])) return fail(OAT_ERR_ARG, "oat_plan_set_eir: taps must be finite");
    int prev;
    int rc = with_device(plan, prev);
    if (rc) return rc;
    if (n_taps == 0) {
        plan->eir_taps = 0;
        (void)hipSetDevice(prev);
        return OAT_OK;
    }
    const int K = plan->P.nt;
    int N = 1;
    while (N < 2 * K) N *= 2;
    hipError_t e = hipSuccess;
    if (!plan->d_eir_h) {
        auto al = [&](void **p, size_t b) {
            if (e == hipSuccess) e = hipMalloc(p, b);
        };
        al((void **)&plan->d_eir_h, sizeof(double) * (size_t)K);
        al((void **)&plan->d_eir_spec, sizeof(double2) * (size_t)N);
        al((void **)&plan->d_eir_tw, sizeof(double2) * (size_t)(N / 2));
        al((void **)&plan->d_eir_filt, sizeof(double2) * (size_t)N);
        al((void **)&plan->d_eirbuf, sizeof(float) * (size_t)plan->P.nq * K);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            (void)hipSetDevice(prev);
            return fail(OAT_ERR_NOMEM, "oat_plan_set_eir: hipMalloc");
        }
        plan->ws_bytes += (int64_t)(sizeof(float) * (size_t)plan->P.nq * K +
                                    sizeof(double2) * (size_t)(2 * N + N / 2));
        plan->table_bytes += (int64_t)(sizeof(double) * (size_t)K);
    }
    // The previous EIR may still be in use by calls queued on other streams.
    e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = hipMemcpy(plan->d_eir_h, h, sizeof(double) * (size_t)n_taps, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = launch_eir_spectrum(plan->d_eir_h, n_taps, N, plan->d_eir_spec, plan->d_eir_tw, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    (void)hipSetDevice(prev);
    if (e != hipSuccess) return fail_hip(e, "oat_plan_set_eir");
    plan->eir_taps = n_taps;
    plan->eir_n = N;
    return OAT_OK;
}

int oat_deconvolve(oat_plan *plan, const void *u, oat_dtype u_dtype, void *p, oat_dtype p_dtype,
                   double f_cut, uint32_t flags, void *stream)
{
    int rc = check_common(plan, u, u_dtype, p, p_dtype, flags, OAT_FLAG_DETERMINISTIC,
                          "oat_deconvolve");
    if (rc) return rc;
    if (plan->eir_taps == 0) return fail(OAT_ERR_ARG, "oat_deconvolve: the plan has no EIR");
    if (!(f_cut > 0.0) || !std::isfinite(f_cut))
        return fail(OAT_ERR_ARG, "oat_deconvolve: f_cut must be > 0");
    int prev;
    if ((rc = with_device(plan, prev))) return rc;
    hipError_t e = launch_deconvolve(plan->P, u, (int)u_dtype, p, (int)p_dtype, plan->d_eir_spec,
                                     plan->d_eir_tw, plan->d_eir_filt, plan->eir_n, f_cut,
                                     (hipStream_t)stream);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) return fail_hip(e, "oat_deconvolve: launch");
    return OAT_OK;
}

static int check_sph(oat_plan *plan, const void *a, const void *b, int img_dt, int n_f,
                     double f_min, double df, uint32_t flags, const char *who)
{
    if (!plan) return fail(OAT_ERR_ARG, std::string(who) + ": null plan");
    if (!a || !b) return fail(OAT_ERR_ARG, std::string(who) + ": null buffer");
    if (a == b) return fail(OAT_ERR_ARG, std::string(who) + ": input and output alias");
    if (img_dt != OAT_F32 && img_dt != OAT_BF16)
        return fail(OAT_ERR_DTYPE, std::string(who) + ": unknown dtype");
    if (flags & ~OAT_FLAG_DETERMINISTIC) return fail(OAT_ERR_ARG, std::string(who) + ": unknown flag");
    if (n_f < 1 || n_f > 4096 || !(f_min >= 0.0) || !std::isfinite(f_min) || !(df > 0.0) ||
        !std::isfinite(df))
        return fail(OAT_ERR_ARG, std::string(who) + ": need 1 <= n_f <= 4096, f_min >= 0, df > 0");
    return OAT_OK;
}

// The spherical-voxel workspace (forward chunk sums, adjoint slice sums),
// grown to `need` bytes; earlier calls may still use the old buffer, so a
// growth waits for the device first.  The device is current.
static int ensure_sph_workspace(oat_plan *plan, size_t need, const char *who)
{
    if (need <= plan->sph_part_bytes) return OAT_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess && plan->d_sph_part) e = hipFree(plan->d_sph_part);
    plan->d_sph_part = nullptr;
    plan->sph_part_bytes = 0;
    if (e == hipSuccess) e = hipMalloc((void **)&plan->d_sph_part, need);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(OAT_ERR_NOMEM, std::string(who) + ": hipMalloc");
    }
    plan->sph_part_bytes = need;
    return OAT_OK;
}

int oat_sph_project(oat_plan *plan, const void *img, oat_dtype img_dtype, void *u, int n_f,
                    double f_min, double df, uint32_t flags, void *stream)
{
    int rc = check_sph(plan, img, u, (int)img_dtype, n_f, f_min, df, flags, "oat_sph_project");
    if (rc) return rc;
    int prev;
    if ((rc = with_device(plan, prev))) return rc;
    if ((rc = ensure_sph_workspace(plan, sph_workspace_bytes(plan->P, n_f), "oat_sph_project"))) {
        (void)hipSetDevice(prev);
        return rc;
    }
    hipError_t e = launch_sph_project(plan->P, img, (int)img_dtype, (float2 *)u, n_f, f_min, df,
                                      plan->d_sph_part, (hipStream_t)stream);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) return fail_hip(e, "oat_sph_project: launch");
    return OAT_OK;
}

int oat_sph_backproject(oat_plan *plan, const void *u, int n_f, double f_min, double df,
                        void *img, oat_dtype img_dtype, uint32_t flags, void *stream)
{
    int rc = check_sph(plan, u, img, (int)img_dtype, n_f, f_min, df, flags, "oat_sph_backproject");
    if (rc) return rc;
    int prev;
    if ((rc = with_device(plan, prev))) return rc;
    if ((rc = ensure_sph_workspace(plan, sph_adj_workspace_bytes(plan->P),
                                   "oat_sph_backproject"))) {
        (void)hipSetDevice(prev);
        return rc;
    }
    hipError_t e = launch_sph_backproject(plan->P, (const float2 *)u, n_f, f_min, df, img,
                                          (int)img_dtype, (double *)plan->d_sph_part,
                                          (hipStream_t)stream);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) return fail_hip(e, "oat_sph_backproject: launch");
    return OAT_OK;
}

int oat_plan_set_aperture(oat_plan *plan, double width, double height, int m)
{
    if (!plan) return fail(OAT_ERR_ARG, "oat_plan_set_aperture: null plan");
    if (!(width >= 0.0) || !(height >= 0.0) || !std::isfinite(width) || !std::isfinite(height))
        return fail(OAT_ERR_ARG, "oat_plan_set_aperture: width and height must be finite and >= 0");
    const bool point = width == 0.0 && height == 0.0;
    if (!point && (width <= 0.0 || height <= 0.0 || m < 1 || m > OAT_APERTURE_MAX_ORDER))
        return fail(OAT_ERR_ARG, "oat_plan_set_aperture: need width, height > 0 and 1 <= m <= 8");
    const double R = std::sqrt(0.25 * (width * width + height * height));
    for (const DetRec &d : plan->det)
        if (!point && !(R < std::sqrt(d.r[0] * d.r[0] + d.r[1] * d.r[1] + d.r[2] * d.r[2]) -
                               (double)plan->P.r_sup * plan->P.dxd))
            return fail(OAT_ERR_GEOMETRY,
                        "oat_plan_set_aperture: a face reaches into the image support sphere");
    const int mm = point ? 0 : m;
    const std::vector<double4> faces = face_nodes(plan->det, width, height, mm);
    int prev;
    int rc = with_device(plan, prev);
    if (rc) return rc;
    // earlier calls may still read the old table
    hipError_t e = hipDeviceSynchronize();
    double4 *buf = nullptr;
    if (e == hipSuccess) e = hipMalloc((void **)&buf, sizeof(double4) * faces.size());
    if (e == hipSuccess)
        e = hipMemcpy(buf, faces.data(), sizeof(double4) * faces.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (buf) (void)hipFree(buf);
        (void)hipGetLastError();
        (void)hipSetDevice(prev);
        return fail_hip(e, "oat_plan_set_aperture");
    }
    (void)hipFree(plan->d_sph_pts);
    plan->table_bytes += (int64_t)(sizeof(double4) * faces.size()) -
                         (int64_t)(sizeof(double4) * plan->det.size() * (size_t)plan->P.sph_ns);
    plan->d_sph_pts = buf;
    plan->P.sph_pts = buf;
    plan->P.sph_ns = point ? 1 : m * m;
    plan->ap_w = point ? 0.0 : width;
    plan->ap_h = point ? 0.0 : height;
    plan->ap_m = mm;
    (void)hipSetDevice(prev);
    return OAT_OK;
}

int oat_sph_backproject_noalloc(oat_plan *plan, const void *u, int n_f, double f_min, double df,
                                void *img, oat_dtype img_dtype, uint32_t flags, void *stream)
{
    int rc = check_sph(plan, u, img, (int)img_dtype, n_f, f_min, df, flags,
                       "oat_sph_backproject_noalloc");
    if (rc) return rc;
    const size_t need = sph_adj_workspace_bytes(plan->P);
    if (need > SPH_SCRATCH_BYTES)
        return fail(OAT_ERR_ARG, "oat_sph_backproject_noalloc: the image needs " +
                                     std::to_string(need) + " bytes of scratch, more than the " +
                                     std::to_string(SPH_SCRATCH_BYTES) + " available");
    int prev;
    if ((rc = with_device(plan, prev))) return rc;
    double *scr = nullptr;
    hipError_t e = sph_scratch_address(plan->device, &scr);
    if (e == hipSuccess)
        e = launch_sph_backproject(plan->P, (const float2 *)u, n_f, f_min, df, img, (int)img_dtype,
                                   scr, (hipStream_t)stream);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) return fail_hip(e, "oat_sph_backproject_noalloc: launch");
    return OAT_OK;
}

}  // extern "C"
