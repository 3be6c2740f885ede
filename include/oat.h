/*
 * oat.h -- C ABI of the MI355X (gfx950) library for the interpolation-based
 * imaging operators of three-dimensional optoacoustic tomography.
 *
 * Operators (Wang, Huang, Kao, Chou, Oraevsky, Anastasio, "Accelerating image
 * reconstruction in three-dimensional optoacoustic tomography on graphics
 * processing units"):
 *
 *   oat_project      p = H alpha = H^e D G alpha   Sec. II.B.1: Eq. (dis_srt), Eq. (dis_g2p),
 *                                              then Eq. (EIR) if the plan has an EIR
 *                                              (point-like transducers otherwise: H^e = I)
 *   oat_backproject  alpha' = H^T y = G^T D^T H^e^T y   Sec. II.B.3, the exact adjoint
 *   oat_fbp          alpha_fbp from p          Sec. III.B, Eq. (disfbp)
 *   oat_deconvolve   p from measured u         Sec. IV.B: Fourier deconvolution of the
 *                                              EIR with a Hann window, before oat_fbp
 *   oat_sph_project  u~ = H_sph alpha          Sec. II.B.2: the spherical-voxel model,
 *   oat_sph_backproject  H_sph^T u~            Eq. (dis_sph) and Eq. (sphbwd), in the
 *                                              temporal-frequency domain
 *
 * Units: lengths in mm, times in microseconds.
 *
 * Image layout: C-contiguous [nz][ny][nx] (x fastest); node (ix,iy,iz) sits at
 * (x0 + ix*dx, y0 + iy*dx, z0 + iz*dx).  alpha_n is the value at node n
 * (Eq. (coeffint)); between nodes the image is the trilinear expansion of
 * Eq. (expfunI), zero outside the grid.
 *
 * Data layout: C-contiguous [n_det][n_t] (time fastest), sample k of
 * transducer q at t_k = t0 + k*dt; the flat index is q*n_t + k as in
 * Eq. (CDmodel).
 *
 * Discretisation of G (the Appendix, made definite):
 *  - each shell k is the sphere of radius rho_k = c0*t_k about r_q, described
 *    in a frame with z^tr = -r_q/|r_q| (pointing at the origin),
 *    x^tr = unit polar vector and y^tr = minus the unit azimuthal vector of r_q;
 *  - the polar angle is cut into bands of arc length dx starting at the pole,
 *    [i dtheta, min((i+1) dtheta, pi)] with dtheta = dx/rho_k; ring i sits at
 *    the mid-band angle and holds N_j = max(1, round(2 pi rho_k sin(theta_i)/dx))
 *    points at azimuths 2 pi j / N_j, each weighted by the band area / N_j;
 *  - g[q,k] = sum of weight * (trilinear image value) over these points.
 * D:  s_k = g_k/t_k (0 where t_k <= 0), p_k = Gamma/(4 pi c0^2) (s_{k+1}-s_{k-1})/(2 dt),
 *     with s_{-1} = s_{n_t} = 0 (Eq. (g2p) with beta/Cp = Gamma/c0^2).
 *
 * Buffers: every image/data pointer passed to oat_project, oat_backproject
 * and oat_fbp is a DEVICE pointer on the plan's device, owned by the caller,
 * C-contiguous, and must not overlap another argument.  Each call overwrites
 * its whole output (nothing accumulates across calls).
 *
 * Streams: calls are asynchronous on `stream` (a hipStream_t; NULL = the
 * default stream).  The caller synchronises before reading outputs.  A plan
 * holds one workspace: calls on the same plan must not overlap in time (use
 * one stream per plan, or one plan per stream).
 *
 * Errors: every function returns an oat_status; nothing aborts or throws
 * across the ABI.  Arguments are validated before anything is launched.
 * oat_last_error() returns a thread-local description of the last failure.
 */
#ifndef OAT_H
#define OAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OAT_OK = 0,
    OAT_ERR_ARG = -1,       /* null pointer, bad size, unknown flag */
    OAT_ERR_GEOMETRY = -2,  /* invalid or unsupported geometry (see oat_plan_create) */
    OAT_ERR_DTYPE = -3,     /* unknown oat_dtype */
    OAT_ERR_DEVICE = -4,    /* HIP runtime error; text in oat_last_error() */
    OAT_ERR_NOMEM = -5,     /* device or host allocation failed */
    OAT_ERR_INTERNAL = -6
} oat_status;

typedef enum {
    OAT_F32 = 0,            /* IEEE binary32 */
    OAT_BF16 = 1            /* bfloat16 storage; arithmetic is FP32 */
} oat_dtype;

/* Problem statement (Sec. II.B and Sec. III.A).  Host memory; copied by
 * oat_plan_create, so the caller may free it afterwards. */
typedef struct {
    int32_t nx, ny, nz;         /* nodes per axis, >= 1 */
    double dx;                  /* node spacing Delta_s (mm), > 0 */
    double x0, y0, z0;          /* position of node (0,0,0) (mm) */
    int32_t n_det;              /* number of transducers Q, >= 1 */
    const double *det_xyz;      /* Q x 3 transducer positions r_q (mm), host */
    const double *det_area;     /* Q patch areas a_q (mm^2) used by oat_fbp, host;
                                   NULL means 4 pi |r_q|^2 / Q */
    int32_t n_t;                /* samples per transducer K, 3 <= K <= 4096 */
    double dt;                  /* sampling interval (us), > 0 */
    double t0;                  /* time of sample 0 (us) */
    double c0;                  /* speed of sound (mm/us), > 0 */
    double gamma;               /* Grueneisen coefficient Gamma = beta c0^2 / Cp, > 0 */
} oat_geometry;

typedef struct oat_plan oat_plan;

/* Expose the G or G^T stage alone: oat_project returns g = G alpha and
 * oat_backproject returns G^T y (D and D^T are skipped). */
#define OAT_FLAG_SRT_ONLY 1u

/* Ask for bit-stable output (ordered reductions).  Every operator of this
 * library already gives bit-identical results for identical inputs (G's
 * shell sums are fixed-point integers on the segment-table path and FP64 sums
 * formed by one wave in program order on the others, and its brick partials
 * are summed in a fixed order; G^T adds exact fixed-point integers; FBP and
 * the EIR and deconvolution kernels have no atomics), so the flag is accepted
 * and changes nothing. */
#define OAT_FLAG_DETERMINISTIC 2u

/* Validate the geometry, build the quadrature tables in FP64 on the host,
 * upload them and allocate the workspace on `device`.
 * Returns OAT_ERR_GEOMETRY when a transducer lies inside the sphere that
 * holds the image support (radius R = largest corner norm of the box
 * [x0-dx, x0+nx*dx] x ...; Sec. III.A assumes the measurement surface lies
 * outside it), when t_k stays <= 0, or when sizes exceed 32-bit indexing.
 * On success *out owns device memory until oat_plan_destroy. */
int oat_plan_create(const oat_geometry *geom, int device, oat_plan **out);

/* Plan options for oat_plan_create_ex.  The kernels of oat_project and
 * oat_backproject enumerate, for every (image brick, transducer) pair, the
 * quadrature points of Eq. (dis_srt) whose trilinear cell lies in the brick.
 * A plan can record that enumeration once, in one of two tables; results
 * are the same on every path up to FP32 summation order in oat_project and
 * bit for bit in oat_backproject.
 *
 * segment_table_bytes: device memory the plan may spend on its segment
 * table: for every pair, the ring segments (runs of at most 32 consecutive
 * points) that hold the brick's points, 4 bytes each, ordered by point
 * count; about 20 GB for a 256^3 image at 2048 transducers and 1024
 * samples, 80 GB at 8192 transducers.  With it the kernels take one segment
 * per lane and skip every bound computation.  It is built on the device at
 * plan creation by two passes of the kernels' own bounds walk (each about as
 * costly as one oat_project without a table), and is not built when a
 * segment does not fit its 4-byte entry (more than 63 candidate rings per
 * shell or 256 segments per ring, far beyond the workloads above).
 *
 * arc_table_bytes: device memory the plan may spend on its arc table, built
 * only when the plan has no segment table: for every pair, the rings that
 * hold points of the brick and the exact index range of those points on
 * each ring, about 4 bytes per (brick, transducer, ring) triple (15 GB for
 * the 256^3 case above); the kernels then skip the per-ring bound
 * computations.  Without either table, or when the geometry has rings of
 * more than 65535 points or shells of more than 65535 rings, the kernels
 * bound the arcs themselves.
 *
 * Values of both fields:
 *   -1  automatic: build the table if it fits in 40% of the device memory
 *       free at that point of plan creation (the default of oat_plan_create);
 *    0  never build it;
 *  > 0  build it if it fits in this many bytes. */
typedef struct {
    int64_t arc_table_bytes;
    int64_t segment_table_bytes;
} oat_plan_options;

/* oat_plan_create with options (NULL = defaults: -1 and -1).  OAT_ERR_ARG
 * when arc_table_bytes or segment_table_bytes < -1. */
int oat_plan_create_ex(const oat_geometry *geom, int device, const oat_plan_options *opt,
                       oat_plan **out);

/* Frees the plan's tables and workspace.  NULL is accepted.  The caller
 * must make sure no call on the plan is still running. */
void oat_plan_destroy(oat_plan *plan);

/* data = H img  (n_det x n_t), or G img with OAT_FLAG_SRT_ONLY.
 * img: device [nz][ny][nx] of img_dtype; data: device [n_det][n_t] of
 * data_dtype.  G is accumulated in FP32 and D is applied before any BF16
 * rounding of the output. */
int oat_project(oat_plan *plan, const void *img, oat_dtype img_dtype, void *data,
                oat_dtype data_dtype, uint32_t flags, void *stream);

/* img = H^T data = G^T D^T data  (or G^T data with OAT_FLAG_SRT_ONLY).
 * data: device [n_det][n_t] of data_dtype; img: device [nz][ny][nx] of
 * img_dtype.  Uses exactly the quadrature points and weights of
 * oat_project, so <H x, y> = <x, H^T y> up to FP32 rounding. */
int oat_backproject(oat_plan *plan, const void *data, oat_dtype data_dtype, void *img,
                    oat_dtype img_dtype, uint32_t flags, void *stream);

/* Filtered backprojection, Eq. (disfbp) with the patch area a_q and 1/|r_q|
 * of each transducer:
 *   img_n = -1/(pi Gamma c0 dt) sum_q a_q/|r_q| { [(k+1+tau)/(kt+tau) - 1.5] p[q,k]
 *                                              + [1.5 - (k+tau)/(kt+tau)] p[q,k+1] }
 * with kt = (|r_n - r_q|/c0 - t0)/dt, k = floor(kt), tau = t0/dt and p = 0
 * outside [0, n_t).  pres: device [n_det][n_t]; img: device [nz][ny][nx]. */
int oat_fbp(oat_plan *plan, const void *pres, oat_dtype pres_dtype, void *img,
            oat_dtype img_dtype, uint32_t flags, void *stream);

/* Electrical impulse response of the transducers, Eq. (EIR):
 * [H^e p]_{q,k} = sum_{kappa=0}^{n_t-1} h[k-1-kappa] p_{q,kappa}, with h[m] = 0
 * outside [0, n_taps) (the printed index, a one-sample delay).  From then on
 * oat_project returns H^e D G alpha and oat_backproject G^T D^T H^e^T y, with
 * H^e^T from the adjoint formula of Sec. II.B.3 (OAT_FLAG_SRT_ONLY still
 * returns G and G^T alone).  h: host array of n_taps finite doubles,
 * h[m] = dt h^e(m dt), copied; 1 <= n_taps <= n_t.  n_taps = 0 removes the
 * EIR (h may be NULL).  Synchronous: waits for the device, so no call on the
 * plan may be in flight.  Sums are FP64, with one rounding to the output
 * type.  OAT_ERR_ARG on bad sizes or non-finite taps. */
int oat_plan_set_eir(oat_plan *plan, const double *h, int n_taps);

/* Fourier deconvolution of the plan's EIR with a Hann window (Sec. IV.B),
 * per transducer row: p~(f) = u~(f) W(f) / h~(f), where
 *   W(f) = (1 - cos(pi (f_cut - |f|) / f_cut)) / 2 for |f| <= f_cut, 0 beyond,
 *   h~   = the transform of the response of Eq. (EIR), one-sample delay included,
 * and bins where h~ = 0 give 0.  Each record is zero-padded to N = the power
 * of two >= 2 n_t, so the division undoes the linear (not circular)
 * convolution, and the first n_t samples of the inverse transform are
 * returned.  Transforms in FP64.  f_cut in cycles per time unit (MHz when
 * times are in microseconds), > 0.  u, p: device [n_det][n_t], may not
 * alias.  flags: 0 or OAT_FLAG_DETERMINISTIC.  Asynchronous on `stream`.
 * OAT_ERR_ARG when the plan has no EIR. */
int oat_deconvolve(oat_plan *plan, const void *u, oat_dtype u_dtype, void *p, oat_dtype p_dtype,
                   double f_cut, uint32_t flags, void *stream);

/* Spherical-voxel model (Sec. II.B.2), point-like transducers (the surface
 * integral over S_q divided by S_q is its value at r_q), ideal EIR:
 *   u~[q][l] = p0(f_l) sum_n alpha_n exp(-j 2 pi f_l d_qn / c0) / (2 pi d_qn),
 *   p0(f) = -j Gamma c0 / f [dx/(2 c0) cos(pi f dx / c0) - sin(pi f dx / c0) / (2 pi f)]
 *   (Eq. (p0f) with beta c0^3 / Cp = Gamma c0; p0(0) = 0), d_qn = |r_q - r_n|,
 * f_l = f_min + l df for l = 0 .. n_f - 1 (the listings' frequency grid).
 * alpha_n is the voxel's absorbed-energy density; r_n are the plan's nodes.
 * img: device [nz][ny][nx] (oat_dtype); u: device [n_det][n_f] complex FP32,
 * interleaved (re, im).  Every term is evaluated (a dense sum); phases and
 * sums are FP64; each run of frequencies starts from an FP32 exponential
 * (about 1 ulp) and steps it in FP64 (H_sph) or in FP32 (H_sph^T).
 * 1 <= n_f <= 4096, f_min >= 0, df > 0,
 * flags: 0 or OAT_FLAG_DETERMINISTIC.  The two calls share a workspace in
 * the plan and may allocate or grow it: oat_sph_project for a larger n_f,
 * oat_sph_backproject for an image of fewer than 512K voxels, whose
 * transducers it splits into slices of FP64 partial images (added in slice
 * order).  Results are deterministic. */
int oat_sph_project(oat_plan *plan, const void *img, oat_dtype img_dtype, void *u, int n_f,
                    double f_min, double df, uint32_t flags, void *stream);

/* Eq. (sphbwd): img[n] = Re sum_{q,l} u~[q][l] conj(p0(f_l)) exp(+j 2 pi f_l d_qn / c0) / (2 pi d_qn),
 * the adjoint of oat_sph_project over real images.  Same arguments.  With
 * finite faces (oat_plan_set_aperture) both calls use (1/S_q) h~_q below in
 * place of the point-like term. */
int oat_sph_backproject(oat_plan *plan, const void *u, int n_f, double f_min, double df,
                        void *img, oat_dtype img_dtype, uint32_t flags, void *stream);

/* Finite transducer faces for the spherical-voxel model (Sec. II.B.2): the
 * SIR h~_q(r_n, f) of Eq. (dis_sph) is the integral over the face S_q of
 * exp(-j 2 pi f |r^s - r_n| / c0) / (2 pi |r^s - r_n|), and the model uses
 * (1/S_q) h~_q.  Every face is a flat width x height rectangle (mm) centred
 * at r_q and normal to r_q, its width along the unit polar vector of r_q and
 * its height along minus the unit azimuthal vector (the frame of G); the
 * face average is the m x m Gauss-Legendre product rule, i.e. a weighted sum
 * of the point-like terms of m^2 nodes, so a call costs m^2 times a
 * point-like one.  width = height = 0 restores point-like transducers (m is
 * then ignored).  Affects oat_sph_project, oat_sph_backproject and
 * oat_sph_backproject_noalloc only; the interpolation model is
 * point-like.  Synchronous: waits for the device, so no call on the plan may
 * be in flight.  OAT_ERR_ARG for negative or non-finite sizes, one size 0
 * and not the other, or m outside 1 .. OAT_APERTURE_MAX_ORDER;
 * OAT_ERR_GEOMETRY when a face reaches into the sphere that holds the image
 * support. */
#define OAT_APERTURE_MAX_ORDER 8
int oat_plan_set_aperture(oat_plan *plan, double width, double height, int m);

/* oat_sph_backproject for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops and harnesses that forbid
 * hipMalloc.  Same arguments, operation and results (bit for bit) as
 * oat_sph_backproject, which may grow the plan's workspace; this variant
 * calls no hipMalloc, hipFree or allocating library routine and never waits
 * for the device.  Images of fewer than 512K voxels split the transducers
 * into slices whose FP64 partial images go to a fixed 8 MiB scratch array in
 * device memory, one per GPU (resolved at the first oat_plan_create on that
 * GPU and held until the process ends); every image this library accepts
 * needs at most 2 x 523776 x 8 bytes of it, and a larger need is rejected
 * with OAT_ERR_ARG.  Every slice value is written before it is read, so the
 * scratch needs no clearing.  All calls on one GPU share that scratch: calls
 * that overlap in time on one GPU (other streams, other plans, other
 * threads) race and give wrong results. */
int oat_sph_backproject_noalloc(oat_plan *plan, const void *u, int n_f, double f_min, double df,
                                void *img, oat_dtype img_dtype, uint32_t flags, void *stream);

/* Thread-local, NUL-terminated description of the last non-OK status
 * returned on this thread ("" if none).  Valid until the next call. */
const char *oat_last_error(void);

/* Work accounting of a plan (host values, filled at plan creation):
 * stats[0] = number of quadrature rings in the tables,
 * stats[1] = number of image bricks, stats[2] = brick edge (cells),
 * stats[3] = shell window per (brick, transducer),
 * stats[4] = bytes of device workspace, stats[5] = bytes of device tables,
 * stats[6] = bytes of the arc table (0: none built, which is the case
 * whenever the plan has a segment table), stats[7] = its ring entries,
 * stats[8] = its build time in microseconds,
 * stats[9] = time of the G^T calibration pass in microseconds (the plan runs
 * G^T's walk once with unit data to bound its fixed-point sums),
 * stats[10] = bytes of the segment table (0: none), stats[11] = its entries,
 * stats[12] = its build time in microseconds.
 * n = capacity of stats (at most 13 are written); returns OAT_OK. */
int oat_plan_stats(const oat_plan *plan, int64_t *stats, int n);

#ifdef __cplusplus
}
#endif

#endif /* OAT_H */
