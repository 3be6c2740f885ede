// Internal tables and launch interfaces shared by the host plan and the
// gfx950 kernels of liboat.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oat {

// Edge of an image brick in cells.  One workgroup owns one brick and keeps
// its (BRICK+2)^3 nodes in LDS.
constexpr int BRICK = 20;
constexpr int BOX = BRICK + 2;                // LDS nodes per axis
constexpr int BOX_SY = BOX + 2;               // LDS row pitch (dwords)
constexpr int BOX_SZ = BOX_SY * BOX + 38;     // LDS slice pitch (dwords); pitches chosen
                                              // to spread arcs of any direction over banks
constexpr int BOX_WORDS = BOX_SZ * BOX;
constexpr int BOX3 = BOX * BOX * BOX;          // dense box in HBM (G^T brick output)
constexpr int WAVES = 8;                      // waves per workgroup (srt kernels)
constexpr int WAVE = 64;
constexpr int WMAX = 256;                    // largest shell window per (brick, transducer)
// G^T takes the transducers in windows of ADJ_WINDOW, with one fixed-point
// scale and one flush of its LDS box per window.
constexpr int ADJ_WINDOW = 128;
// Spherical-voxel forward: voxel chunks summed separately, then in order.
constexpr int SPH_CHUNKS = 64;
__host__ __device__ inline int adj_windows(int nq) { return (nq + ADJ_WINDOW - 1) / ADJ_WINDOW; }

// Slices of a brick's work (G: transducers, G^T: transducer windows) as
// separate workgroups.  A kernel that runs one workgroup per CU runs its grid
// in rounds of 256 workgroups, and a partly empty last round leaves CUs idle:
// brick_slices takes the count (1..4, at least min_items items per slice)
// whose grid fills its last round best, a smaller count winning ties within
// 0.5%, and returns the number of non-empty slices of ceil(items / count)
// items.
inline int brick_slices(int nbricks, int items, int min_items)
{
    int best = 1;
    double best_eff = 0.0;
    for (int sl = 1; sl <= 4; ++sl) {
        if (sl > 1 && items / sl < min_items) break;
        const long long g = (long long)nbricks * sl;
        const double eff = (double)g / (double)(((g + 255) / 256) * 256);
        if (eff > best_eff + 0.005) {
            best = sl;
            best_eff = eff;
        }
    }
    const int per = (items + best - 1) / best;
    return (items + per - 1) / per;
}
// Slice counts for the kernels whose grids run in rounds of `round`
// workgroups: among 1..max_slices slices of at least min_items items, the
// count whose grid fills its rounds best, a larger count winning ties within
// 0.5% (shorter workgroups leave a shorter tail when the last ones finish).
inline int fill_slices(int nbricks, int items, int min_items, int max_slices, int round)
{
    int best = 1;
    double best_eff = 0.0;
    for (int c = 1; c <= max_slices; ++c) {
        if (c > 1 && items / c < min_items) break;
        const int per = (items + c - 1) / c, n = (items + per - 1) / per;
        const long long g = (long long)nbricks * n;
        const double eff = (double)g / (double)(((g + round - 1) / round) * round);
        if (eff >= best_eff - 0.005) {
            best = n;
            best_eff = eff > best_eff ? eff : best_eff;
        }
    }
    return best;
}
// G on the arc-table and bounds paths (one workgroup per CU): transducers
// per slice >= 64.
inline int fwd_slices(int nbricks, int nq) { return brick_slices(nbricks, nq, 64); }
// G on the segment table runs two workgroups per CU (rounds of 512): up to 8
// slices of at least 64 transducers.
inline int seg_fwd_slices(int nbricks, int nq) { return fill_slices(nbricks, nq, 64, 8, 512); }
// G^T (one workgroup per CU): up to 8 slices of at least 2 windows; each
// slice keeps its own FP64 brick sums ([slice][brick][BOX3]; the same slicing
// for every table mode).
inline int adj_slices(int nbricks, int nq) { return fill_slices(nbricks, adj_windows(nq), 2, 8, 256); }

// Per-transducer record (grid units: positions are (r - r_0)/dx).
struct alignas(16) DetRec {
    double uq[3];      // transducer position
    double e3[3];      // unit vector to the origin (z of the local frame)
    double e1d[3];     // x of the local frame
    double e2d[3];     // y of the local frame
    float e1[3];       // e1d rounded to FP32 (arc bounds)
    float e2[3];       // e2d rounded to FP32 (arc bounds)
    float dist;        // |r_q| / dx
    float fbp_w;       // a_q / |r_q|  (mm)
    float uqf[3];      // transducer position rounded to FP32
    float pad;
    double r[3];       // transducer position in mm
    double pad2;
};

// Per-shell record: shell k holds rings [ring_base, ring_base + n_rings).
struct alignas(16) ShellRec {
    int32_t ring_base;
    int32_t n_rings;
    float rho;         // rho_k / dx
    float inv_rho;     // dx / rho_k  (= band width in theta)
};

// Per-ring record (shell k, band i).
struct alignas(16) RingRec {
    double rc;         // rho cos(theta_i) / dx
    double rs;         // rho sin(theta_i) / dx
    float rsf;         // rs rounded to FP32 (arc bounds)
    int32_t nj;        // points on the ring
    float w;           // band area / nj  (mm^2)
    float delta;       // 2 pi / nj
    int32_t lshift;    // ring segments hold 2^lshift consecutive points
    int32_t sref;      // first entry of this ring size in Problem::segref
};

// Ring segments: segment s of a ring of nj points holds the indices
// s 2^lshift .. min((s+1) 2^lshift, nj) - 1; its reference index is the
// middle one (the lower of the two for an even count).
__host__ __device__ inline int seg_ref_index(int s, int lshift, int nj)
{
    const int sb = s << lshift;
    const int se = sb + (1 << lshift) < nj ? sb + (1 << lshift) : nj;
    return sb + ((se - sb - 1) >> 1);
}

// Compact segment-table entry (4 bytes; see Problem::seg).
constexpr int SEG_SHELL_BITS = 8, SEG_RING_BITS = 6, SEG_INDEX_BITS = 8;
constexpr int SEG_OFF_BITS = 5, SEG_CNT_BITS = 5;
static_assert(SEG_SHELL_BITS + SEG_RING_BITS + SEG_INDEX_BITS + SEG_OFF_BITS + SEG_CNT_BITS == 32,
              "one 32-bit word per segment");
__host__ __device__ inline unsigned seg_pack(int shell, int ring, int index, int off, int cnt)
{
    return (unsigned)shell | ((unsigned)ring << SEG_SHELL_BITS) |
           ((unsigned)index << (SEG_SHELL_BITS + SEG_RING_BITS)) |
           ((unsigned)off << (SEG_SHELL_BITS + SEG_RING_BITS + SEG_INDEX_BITS)) |
           ((unsigned)(cnt - 1) << (32 - SEG_CNT_BITS));
}

// Everything a kernel needs about the problem (passed by value).
struct Problem {
    int nx, ny, nz;
    int nq, nt;
    int nbx, nby, nbz;     // bricks per axis
    int window;            // shells per (brick, transducer) window
    float rho0, rho_step;  // rho_k/dx = rho0 + k * rho_step
    float t0, dt;
    float d_coef;          // Gamma / (4 pi c0^2) / (2 dt)
    float fbp_scale;       // -1 / (pi Gamma c0 dt)
    float sigma;           // dx / (c0 dt)
    float inv_sigma;       // c0 dt / dx
    float tau;             // t0 / dt
    // FP64 problem statement for FBP's floor decisions (same formula as the
    // problem statement: kt = (|r_n - r_q| / c0 - t0) / dt, r_n = r_0 + dx * n)
    double x0, y0, z0, dxd, c0d, t0d, dtd;
    double gammad;         // Gamma (spherical-voxel model)
    // [nt + 2]: entry m + 1 (m = -1 .. nt) is the smallest FP64 squared
    // distance (mm^2) at which that floor reaches m (see oat_fbp_floor.hpp)
    const double *fbp_thr;
    float w_max;           // largest ring weight
    float r_sup;           // radius of the image support sphere / dx
    float *gp_rowmax;      // [nq] max |g'| per transducer over reachable samples (D^T kernel)
    const float *adj_r;    // [bricks][adj_windows(nq)] G^T calibration: max node sum of psi w
    const DetRec *det;
    const ShellRec *shell;
    const RingRec *ring;
    // Arc table (null when the plan has none).  Unit u = brick * nq + q:
    // tab_run[u * window + s] = i0 | n << 16, the rings i0 .. i0+n-1 of shell
    // klo(u) + s that may hold points owned by the brick; their entries
    // tab_arc[tab_off[u] + (entries of the unit's earlier shells) + i - i0]
    // = jlo | jcnt << 16, the tight arc of the ring's owned points (jcnt = 0:
    // none).  tab_cnt[u] = entries of unit u (written by the count pass).
    const long long *tab_off;
    unsigned *tab_run;
    unsigned *tab_arc;
    int *tab_cnt;
    // segref[sref(nj) + s] = (cos, sin) in FP64 of the reference azimuth
    // 2 pi seg_ref_index(s) / nj of segment s of any ring of nj points.
    const double2 *segref;
    int n_rings, n_segref;  // entries of ring and segref (index clamps)
    // Spherical-voxel model: each transducer's face as sph_ns quadrature
    // nodes [nq][sph_ns], (x, y, z) in mm and the weight in w (the weights
    // of a transducer sum to 1); point-like transducers: one node r_q, 1.
    const double4 *sph_pts;
    int sph_ns;
    // Segment table (null when the plan has none): the segments of unit u
    // that hold points owned by the brick are entries seg_off[u] ..
    // seg_off[u+1]-1, one 32-bit word each (seg_pack): the shell offset
    // k - klo(u), the ring index relative to the first candidate ring of
    // that shell (shell_rings), the segment index, the first owned point's
    // offset in the segment and the count of points from it to the last
    // owned one.  A unit's entries are ordered by decreasing count (walk
    // order within a count), so a window of 64 has nearly equal counts.
    // Written by two passes of the bounds walk: seg_cnt[u] and
    // seg_hist[u * 32 + count - 1] (count pass), then the entries (fill
    // pass, from seg_off and seg_hist); seg_flag is set when a segment does
    // not fit the entry's fields (the plan then keeps no table).
    const long long *seg_off;
    unsigned *seg;
    int *seg_cnt;
    int *seg_hist;
    int *seg_flag;
};

// Sets the thread-local text returned by oat_last_error (defined with the
// plan's entry points).
void set_last_error(const char *msg);

// Launchers (defined in the .hip files); dtype: 0 = f32, 1 = bf16.
hipError_t launch_srt_fwd(const Problem &P, const void *img, int img_dtype, float *part,
                          int *klo, hipStream_t s);
// Table passes: mode 0 writes tab_run and tab_cnt (tab_run zeroed
// beforehand), 1 writes tab_arc (tab_off set); 2 writes seg_cnt and
// seg_hist and 3 writes seg (seg_off and seg_hist set), both over the
// bounds walk (no arc table needed).
hipError_t launch_arc_build(const Problem &P, int mode, hipStream_t s);
hipError_t launch_srt_reduce(const Problem &P, const float *part, const int *klo,
                             void *out, int out_dtype, int apply_d, hipStream_t s);
hipError_t launch_diff_adj(const Problem &P, const void *y, int y_dtype, float *gp,
                           int apply_dt, hipStream_t s);
hipError_t launch_srt_adj(const Problem &P, const float *gp, double *acc, void *img,
                          int img_dtype, hipStream_t s);
// Writes P.adj_r's values to r (the plan calls it once, with P.adj_r unset).
hipError_t launch_adj_calibrate(const Problem &P, float *r, hipStream_t s);
hipError_t launch_adj_gather(const Problem &P, const double *acc, void *img, int img_dtype,
                             hipStream_t s);
hipError_t launch_fbp(const Problem &P, const void *p, int p_dtype, void *img,
                      int img_dtype, hipStream_t s);
// EIR (oat_eir.hip): H^e (adjoint = 0) or its transpose on every data row;
// the transform of the delayed response on the N-point grid and the FFT
// twiddles; the Hann-window deconvolution (F is a workspace of N values).
hipError_t launch_eir(const Problem &P, const void *in, int in_dt, void *out, int out_dt,
                      const double *h, int taps, int adjoint, hipStream_t s);
hipError_t launch_eir_spectrum(const double *h, int taps, int N, double2 *Ht, double2 *tw,
                               hipStream_t s);
hipError_t launch_deconvolve(const Problem &P, const void *u, int u_dt, void *p, int p_dt,
                             const double2 *Ht, const double2 *tw, double2 *F, int N, double fc,
                             hipStream_t s);
// Spherical-voxel model (oat_sph.hip); part holds sph_workspace_bytes.
size_t sph_workspace_bytes(const Problem &P, int n_f);
hipError_t launch_sph_project(const Problem &P, const void *img, int img_dt, float2 *u, int n_f,
                              double f_min, double df, double2 *part, hipStream_t s);
// Adjoint: small images split the transducers into sph_adj_slices(P) slices
// whose FP64 partial images go to work (sph_adj_workspace_bytes; none for
// one slice).
int sph_adj_slices(const Problem &P);
size_t sph_adj_workspace_bytes(const Problem &P);
hipError_t launch_sph_backproject(const Problem &P, const float2 *u, int n_f, double f_min,
                                  double df, void *img, int img_dt, double *work, hipStream_t s);
// The adjoint's slice sums never exceed 2 x 523776 doubles: sph_adj_slices
// splits only images of fewer than 1024 workgroups of 512 voxels, and over
// every such voxel count N the product slices x N peaks at two slices of
// 523776 voxels.  So this fixed scratch holds them for every image.
constexpr size_t SPH_SCRATCH_BYTES = size_t(8) << 20;
// Device address of the fixed scratch on `device`, which must be current.
// Resolved by hipGetSymbolAddress on the first call for that device, cached
// afterwards (thread-safe).
hipError_t sph_scratch_address(int device, double **out);

}  // namespace oat
