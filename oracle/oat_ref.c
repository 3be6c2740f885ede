/*
 * Oracle for the interpolation-based 3-D optoacoustic imaging operators.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header or table with the HIP
 * path.
 *
 * Plain double-precision loops, written for a reader to check against the
 * paper (Wang et al., "Accelerating image reconstruction in three-dimensional
 * optoacoustic tomography on graphics processing units"):
 *
 *   G    discrete spherical Radon transform       Sec. II.B.1, Eq. (dis_srt),
 *                                                  Appendix Eqs. (srtlocal)-(srtdislocal)
 *   D    time derivative of g/t                   Eq. (g2p) and Eq. (dis_g2p)
 *   D^T, G^T  exact adjoints                      Sec. II.B.3 (adjoint operators)
 *   FBP  discretised spherical-surface FBP        Eq. (fbp), Eq. (linearint), Eq. (disfbp)
 *
 * Units: lengths in mm, times in us.  Image alpha[iz][iy][ix], node
 * (ix,iy,iz) at (x0+ix*dx, y0+iy*dx, z0+iz*dx).  Data [q][k], t_k = t0+k*dt.
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *  - quadrature bands of arc length dx anchored at the pole of the local
 *    frame, mid-band polar angle, N_j = max(1, round(2*pi*rho*sin(theta)/dx))
 *    evenly spaced azimuths, weight = exact band area / N_j;
 *  - local frame: e3 = -r_q/|r_q|, e1 = unit polar vector, e2 = -unit azimuth
 *    vector of r_q (right handed);
 *  - D uses s_k = g_k/t_k (0 where t_k <= 0) with zero padding at both ends;
 *  - FBP uses Eq. (disfbp) with a per-transducer patch area and 1/|r_q| in
 *    place of 1/R^s, and p = 0 outside [0, K).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    int nx, ny, nz;      /* nodes per axis */
    double dx;           /* node spacing Delta_s */
    double x0, y0, z0;   /* position of node (0,0,0) */
    int nq;              /* number of transducers Q */
    const double *rq;    /* Q x 3 transducer positions */
    const double *aq;    /* Q patch areas for FBP, or NULL for 4 pi |r_q|^2 / Q */
    int nt;              /* samples per transducer K */
    double dt, t0;       /* t_k = t0 + k dt */
    double c0;           /* speed of sound */
    double gamma;        /* Grueneisen coefficient beta c0^2 / Cp */
} ref_geom;

/* ------------------------------------------------------------------ */
/* Expansion functions: trilinear interpolation, Eq. (expfunI).        */
/* Psi(alpha; x) = sum_n alpha_n psi_n(x); nodes outside the grid are  */
/* zero, so Psi vanishes outside [x0-dx, x0+nx*dx) per axis.           */
/* ------------------------------------------------------------------ */
static double psi_sum(const ref_geom *G, const double *alpha,
                      double x, double y, double z)
{
    double ux = (x - G->x0) / G->dx;
    double uy = (y - G->y0) / G->dx;
    double uz = (z - G->z0) / G->dx;
    if (!(ux >= -1.0 && ux < G->nx && uy >= -1.0 && uy < G->ny &&
          uz >= -1.0 && uz < G->nz))
        return 0.0;
    double fx = floor(ux), fy = floor(uy), fz = floor(uz);
    int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    double tx = ux - fx, ty = uy - fy, tz = uz - fz;
    double s = 0.0;
    for (int c = 0; c < 8; ++c) {
        int jx = ix + (c & 1), jy = iy + ((c >> 1) & 1), jz = iz + ((c >> 2) & 1);
        if (jx < 0 || jx >= G->nx || jy < 0 || jy >= G->ny || jz < 0 || jz >= G->nz)
            continue;
        double w = ((c & 1) ? tx : 1.0 - tx) * (((c >> 1) & 1) ? ty : 1.0 - ty) *
                   (((c >> 2) & 1) ? tz : 1.0 - tz);
        s += w * alpha[((size_t)jz * G->ny + jy) * G->nx + jx];
    }
    return s;
}

/* Transpose of psi_sum: alpha_n += v * psi_n(x). */
static void psi_scatter(const ref_geom *G, double *alpha, double x, double y,
                        double z, double v)
{
    double ux = (x - G->x0) / G->dx;
    double uy = (y - G->y0) / G->dx;
    double uz = (z - G->z0) / G->dx;
    if (!(ux >= -1.0 && ux < G->nx && uy >= -1.0 && uy < G->ny &&
          uz >= -1.0 && uz < G->nz))
        return;
    double fx = floor(ux), fy = floor(uy), fz = floor(uz);
    int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    double tx = ux - fx, ty = uy - fy, tz = uz - fz;
    for (int c = 0; c < 8; ++c) {
        int jx = ix + (c & 1), jy = iy + ((c >> 1) & 1), jz = iz + ((c >> 2) & 1);
        if (jx < 0 || jx >= G->nx || jy < 0 || jy >= G->ny || jz < 0 || jz >= G->nz)
            continue;
        double w = ((c & 1) ? tx : 1.0 - tx) * (((c >> 1) & 1) ? ty : 1.0 - ty) *
                   (((c >> 2) & 1) ? tz : 1.0 - tz);
        alpha[((size_t)jz * G->ny + jy) * G->nx + jx] += w * v;
    }
}

/* Radius of the origin-centred sphere that holds the support of Psi:
 * the farthest corner of the box [x0-dx, x0+nx*dx] x ... (Sec. III.A,
 * "the cuboid was contained in another sphere of radius R"). */
double ref_support_radius(const ref_geom *G)
{
    double lo[3] = {G->x0 - G->dx, G->y0 - G->dx, G->z0 - G->dx};
    double hi[3] = {G->x0 + G->nx * G->dx, G->y0 + G->ny * G->dx,
                    G->z0 + G->nz * G->dx};
    double r2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double m = fmax(fabs(lo[a]), fabs(hi[a]));
        r2 += m * m;
    }
    return sqrt(r2);
}

/* Local frame of transducer q (Appendix, Fig. geo(b)): z^tr points from
 * the transducer to the origin. */
static void frame(const double *r, double e1[3], double e2[3], double e3[3],
                  double *dist)
{
    double d = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    double th = acos(r[2] / d);
    double ph = atan2(r[1], r[0]);
    e3[0] = -r[0] / d; e3[1] = -r[1] / d; e3[2] = -r[2] / d;
    e1[0] = cos(th) * cos(ph); e1[1] = cos(th) * sin(ph); e1[2] = -sin(th);
    e2[0] = sin(ph); e2[1] = -cos(ph); e2[2] = 0.0;
    *dist = d;
}

/* Visit every quadrature point of shell (q, k) whose band can touch the
 * support; call fn(point, weight).  Bands beyond theta_max hold points with
 * |x| >= R where Psi = 0, so leaving them out changes nothing. */
typedef void (*point_fn)(void *ctx, double x, double y, double z, double w);

static void shell_points(const ref_geom *G, int q, int k, double R,
                         point_fn fn, void *ctx)
{
    double rho = G->c0 * (G->t0 + k * G->dt);
    if (!(rho > 0.0)) return;
    double e1[3], e2[3], e3[3], d;
    frame(G->rq + 3 * (size_t)q, e1, e2, e3, &d);
    if (rho < d - R || rho > d + R) return;
    double cmax = (d * d + rho * rho - R * R) / (2.0 * rho * d);
    if (cmax > 1.0) cmax = 1.0;
    if (cmax < -1.0) cmax = -1.0;
    double thmax = acos(cmax);
    double dth = G->dx / rho;                 /* arc length dx in theta */
    long nring = (long)ceil(M_PI / dth);
    const double *r = G->rq + 3 * (size_t)q;
    for (long i = 0; i < nring; ++i) {
        double tlo = i * dth;
        if (tlo >= thmax) break;
        double thi = (i + 1) * dth;
        if (thi > M_PI) thi = M_PI;
        double th = 0.5 * (tlo + thi);
        double area = 2.0 * M_PI * rho * rho * (cos(tlo) - cos(thi));
        long nj = (long)floor(2.0 * M_PI * rho * sin(th) / G->dx + 0.5);
        if (nj < 1) nj = 1;
        double w = area / (double)nj;
        double st = sin(th), ct = cos(th);
        for (long j = 0; j < nj; ++j) {
            double ph = 2.0 * M_PI * (double)j / (double)nj;
            double a = rho * st * cos(ph), b = rho * st * sin(ph), c = rho * ct;
            double x = r[0] + a * e1[0] + b * e2[0] + c * e3[0];
            double y = r[1] + a * e1[1] + b * e2[1] + c * e3[1];
            double z = r[2] + a * e1[2] + b * e2[2] + c * e3[2];
            fn(ctx, x, y, z, w);
        }
    }
}

/* ---------------------------- G --------------------------------- */
typedef struct { const ref_geom *G; const double *alpha; double sum; } gather_ctx;

static void gather_point(void *vctx, double x, double y, double z, double w)
{
    gather_ctx *c = (gather_ctx *)vctx;
    c->sum += w * psi_sum(c->G, c->alpha, x, y, z);
}

/* g[q*K + k] = sum_i sum_j w_{k,i} Psi(alpha; x_{q,k,i,j})   Eq. (dis_srt).
 * qsel (length nsel) selects the rows computed; g is nsel x K. */
void ref_srt_rows(const ref_geom *G, const double *alpha, const int *qsel,
                  int nsel, double *g)
{
    double R = ref_support_radius(G);
    long total = (long)nsel * G->nt;
#pragma omp parallel for schedule(dynamic, 4)
    for (long idx = 0; idx < total; ++idx) {
        int s = (int)(idx / G->nt), k = (int)(idx % G->nt);
        gather_ctx c = {G, alpha, 0.0};
        shell_points(G, qsel[s], k, R, gather_point, &c);
        g[idx] = c.sum;
    }
}

void ref_srt(const ref_geom *G, const double *alpha, double *g)
{
    int *qs = (int *)malloc(sizeof(int) * (size_t)G->nq);
    for (int q = 0; q < G->nq; ++q) qs[q] = q;
    ref_srt_rows(G, alpha, qs, G->nq, g);
    free(qs);
}

/* ---------------------------- G^T ------------------------------- */
typedef struct { const ref_geom *G; double *alpha; double v; } scatter_ctx;

static void scatter_point(void *vctx, double x, double y, double z, double w)
{
    scatter_ctx *c = (scatter_ctx *)vctx;
    psi_scatter(c->G, c->alpha, x, y, z, w * c->v);
}

/* alpha'[n] = sum_{q,k} g'[q,k] sum_{i,j} w_{k,i} psi_n(x_{q,k,i,j})
 * (adjoint of G, Sec. II.B.3).  Only rows listed in qsel are used; gp is
 * nsel x K.  Each thread scatters into its own image, the images are then
 * summed in thread order. */
void ref_srt_adj_rows(const ref_geom *G, const double *gp, const int *qsel,
                      int nsel, double *alpha_out)
{
    double R = ref_support_radius(G);
    size_t N = (size_t)G->nx * G->ny * G->nz;
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double *acc = (double *)calloc((size_t)nthr * N, sizeof(double));
    long total = (long)nsel * G->nt;
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *mine = acc + (size_t)tid * N;
#pragma omp for schedule(dynamic, 4)
        for (long idx = 0; idx < total; ++idx) {
            double v = gp[idx];
            if (v == 0.0) continue;
            int s = (int)(idx / G->nt), k = (int)(idx % G->nt);
            scatter_ctx c = {G, mine, v};
            shell_points(G, qsel[s], k, R, scatter_point, &c);
        }
    }
    for (size_t n = 0; n < N; ++n) {
        double s = 0.0;
        for (int t = 0; t < nthr; ++t) s += acc[(size_t)t * N + n];
        alpha_out[n] = s;
    }
    free(acc);
}

void ref_srt_adj(const ref_geom *G, const double *gp, double *alpha_out)
{
    int *qs = (int *)malloc(sizeof(int) * (size_t)G->nq);
    for (int q = 0; q < G->nq; ++q) qs[q] = q;
    ref_srt_adj_rows(G, gp, qs, G->nq, alpha_out);
    free(qs);
}

/* ---------------------------- D and D^T ------------------------- */
/* p_k = Gamma/(4 pi c0^2) * (s_{k+1} - s_{k-1}) / (2 dt),  s_k = g_k / t_k.
 * Eq. (g2p) with beta/Cp = Gamma/c0^2, differenced as in Eq. (dis_g2p). */
void ref_diff(const ref_geom *G, int nrows, const double *g, double *p)
{
    double coef = G->gamma / (4.0 * M_PI * G->c0 * G->c0) / (2.0 * G->dt);
    int K = G->nt;
    double *s = (double *)malloc(sizeof(double) * (size_t)(K + 2));
    for (int r = 0; r < nrows; ++r) {
        const double *gr = g + (size_t)r * K;
        s[0] = 0.0;
        s[K + 1] = 0.0;
        for (int k = 0; k < K; ++k) {
            double t = G->t0 + k * G->dt;
            s[k + 1] = (t > 0.0) ? gr[k] / t : 0.0;
        }
        for (int k = 0; k < K; ++k) p[(size_t)r * K + k] = coef * (s[k + 2] - s[k]);
    }
    free(s);
}

/* g'_k = Gamma/(4 pi c0^2)/(2 dt) * (y_{k-1} - y_{k+1}) / t_k, zero where
 * t_k <= 0 and y_{-1} = y_K = 0: the transpose of ref_diff (Sec. II.B.3). */
void ref_diff_adj(const ref_geom *G, int nrows, const double *y, double *gp)
{
    double coef = G->gamma / (4.0 * M_PI * G->c0 * G->c0) / (2.0 * G->dt);
    int K = G->nt;
    for (int r = 0; r < nrows; ++r) {
        const double *yr = y + (size_t)r * K;
        for (int k = 0; k < K; ++k) {
            double t = G->t0 + k * G->dt;
            double ym = (k > 0) ? yr[k - 1] : 0.0;
            double yp = (k + 1 < K) ? yr[k + 1] : 0.0;
            gp[(size_t)r * K + k] = (t > 0.0) ? coef * (ym - yp) / t : 0.0;
        }
    }
}

/* ------------------------- H and H^T ---------------------------- */
void ref_project_rows(const ref_geom *G, const double *alpha, const int *qsel,
                      int nsel, double *p)
{
    double *g = (double *)malloc(sizeof(double) * (size_t)nsel * G->nt);
    ref_srt_rows(G, alpha, qsel, nsel, g);
    ref_diff(G, nsel, g, p);
    free(g);
}

void ref_backproject_rows(const ref_geom *G, const double *y, const int *qsel,
                          int nsel, double *alpha_out)
{
    double *gp = (double *)malloc(sizeof(double) * (size_t)nsel * G->nt);
    ref_diff_adj(G, nsel, y, gp);
    ref_srt_adj_rows(G, gp, qsel, nsel, alpha_out);
    free(gp);
}

/* ---------------------------- FBP ------------------------------- */
/* Eq. (disfbp): for each voxel n and transducer q,
 *   kt = (|r_n - r_q| / c0 - t0) / dt,  k = floor(kt),  tau = t0 / dt,
 *   term = a_q/|r_q| * { [(k+1+tau)/(kt+tau) - 1.5] p_k + [1.5 - (k+tau)/(kt+tau)] p_{k+1} }
 *   img_n = -1/(pi Gamma c0 dt) * sum_q term
 * Computes the voxels listed in vsel (flat indices), or all when vsel is NULL. */
void ref_fbp_voxels(const ref_geom *G, const double *p, const long *vsel,
                    long nsel, double *out)
{
    double tau = G->t0 / G->dt;
    double pref = -1.0 / (M_PI * G->gamma * G->c0 * G->dt);
    long n_all = (long)G->nx * G->ny * G->nz;
    long count = vsel ? nsel : n_all;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < count; ++s) {
        long n = vsel ? vsel[s] : s;
        int ix = (int)(n % G->nx);
        int iy = (int)((n / G->nx) % G->ny);
        int iz = (int)(n / ((long)G->nx * G->ny));
        double x = G->x0 + ix * G->dx, y = G->y0 + iy * G->dx, z = G->z0 + iz * G->dx;
        double sum = 0.0;
        for (int q = 0; q < G->nq; ++q) {
            const double *r = G->rq + 3 * (size_t)q;
            double rs = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
            double a = G->aq ? G->aq[q] : 4.0 * M_PI * rs * rs / G->nq;
            double ddx = x - r[0], ddy = y - r[1], ddz = z - r[2];
            double dist = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
            double kt = (dist / G->c0 - G->t0) / G->dt;
            double kf = floor(kt);
            long k = (long)kf;
            double clo = (kf + 1.0 + tau) / (kt + tau) - 1.5;
            double chi = 1.5 - (kf + tau) / (kt + tau);
            const double *pr = p + (size_t)q * G->nt;
            double pk = (k >= 0 && k < G->nt) ? pr[k] : 0.0;
            double pk1 = (k + 1 >= 0 && k + 1 < G->nt) ? pr[k + 1] : 0.0;
            sum += a / rs * (clo * pk + chi * pk1);
        }
        out[s] = pref * sum;
    }
}

void ref_fbp(const ref_geom *G, const double *p, double *img)
{
    ref_fbp_voxels(G, p, NULL, 0, img);
}

/* The quadrature points of one shell (q, k), in visiting order: up to cap
 * rows of (x, y, z, w) are written to out and the number of points visited is
 * returned (0 when the shell misses the support).  This is the enumeration G
 * and G^T use, exposed so that it can be checked on its own against the
 * Appendix's band construction. */
typedef struct { double *out; long cap, n; } list_ctx;
static void list_point(void *vctx, double x, double y, double z, double w)
{
    list_ctx *c = (list_ctx *)vctx;
    if (c->n < c->cap) {
        double *o = c->out + 4 * c->n;
        o[0] = x; o[1] = y; o[2] = z; o[3] = w;
    }
    c->n += 1;
}

long ref_shell_points(const ref_geom *G, int q, int k, double *out, long cap)
{
    list_ctx c = {out, cap, 0};
    shell_points(G, q, k, ref_support_radius(G), list_point, &c);
    return c.n;
}

/* Thread count of the following calls (timing only; results do not depend on it). */
void ref_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int ref_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
