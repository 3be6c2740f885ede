// Spherical-voxel imaging model on gfx950 (Sec. II.B.2): H_sph of
// Eq. (dis_sph) with p0 of Eq. (p0f), and its adjoint, Eq. (sphbwd), for
// point-like transducers (the surface integral over S_q divided by S_q is the
// value at r_q) and an ideal EIR:
//   u[q, l] = p0(f_l) sum_n alpha_n exp(-j 2 pi f_l d_qn / c0) / (2 pi d_qn),
//   f_l = f_min + l df,   d_qn = |r_q - r_n|.
// Every (transducer, frequency, voxel) term is evaluated: a dense sum, bound
// by the VALU.  Distances and phases are FP64 (a phase of hundreds of turns
// must keep ~1e-7 turn); the complex exponentials are an accurate sincos of
// the phase's fractional turn followed by short recurrences along l (an FP64
// rotation by an FP64 step in the forward kernel, FP32 Horner's rule in the
// adjoint); sums are FP64.
#include <mutex>
#include <vector>

#include "oat_dtype.hpp"
#include "oat_geom.hpp"
#include "oat_internal.hpp"

#pragma clang fp contract(off)

namespace oat {

namespace {

constexpr int SPH_THREADS = 256;
constexpr int SPH_FB = 32;       // frequencies per thread (forward)
constexpr int SPH_TILE = 256;    // voxels staged per LDS tile (forward)
constexpr int SPH_SHARE = 1024;  // (transducer, voxel) values shared per step (forward)
constexpr int SPH_ANCHOR = 16;   // frequencies per Horner block (adjoint)
constexpr int SPH_VQ = 4096;     // staged u p0* values per adjoint tile (32 KB: 4 groups per CU)
constexpr int SPH_NV = 2;        // consecutive voxels per adjoint thread

__device__ __forceinline__ double frac_turn(double x) { return x - floor(x); }

// Node n of the [nz][ny][nx] grid in FP64.
__device__ __forceinline__ void node_pos(const Problem &P, long long n, double &x, double &y,
                                         double &z)
{
    const long long ix = n % P.nx, iy = (n / P.nx) % P.ny, iz = n / ((long long)P.nx * P.ny);
    x = P.x0 + (double)ix * P.dxd;
    y = P.y0 + (double)iy * P.dxd;
    z = P.z0 + (double)iz * P.dxd;
}

// Partial sums of one voxel chunk.  Thread: transducer q = blockIdx.x * QB +
// t / LB, frequencies l0 = (t % LB) * SPH_FB ... + SPH_FB - 1.
// part[chunk][q][l] = sum over the chunk's voxels (FP64 complex, no p0).
__global__ void __launch_bounds__(SPH_THREADS)
sph_fwd_kernel(Problem P, const void *__restrict__ img, int img_dt, int n_f, double f_min,
               double df, int LB, long long chunk_len, double2 *__restrict__ part)
{
    static_assert(SPH_TILE == SPH_THREADS && SPH_THREADS % 64 == 0, "one voxel per thread per tile");
    __shared__ double sx[SPH_TILE], sy[SPH_TILE], sz[SPH_TILE];
    __shared__ float sa[SPH_TILE];
    __shared__ int wcnt[SPH_THREADS / 64];
    __shared__ double stau[SPH_SHARE], sw[SPH_SHARE];
    __shared__ double2 sstep[SPH_SHARE];
    const int QB = SPH_THREADS / LB;
    const int t = threadIdx.x;
    const int q = blockIdx.x * QB + t / LB;
    const int l0 = (t % LB) * SPH_FB;
    const bool active = (t / LB) < QB && q < P.nq && l0 < n_f;
    const long long N = (long long)P.nx * P.ny * P.nz;
    const long long n0 = (long long)blockIdx.y * chunk_len, n1 = min(N, n0 + chunk_len);
    const double inv_c0 = 1.0 / P.c0d;
    const double fa = f_min + df * (double)l0;   // first frequency of the thread
    double ar[SPH_FB], ai[SPH_FB];
#pragma unroll
    for (int i = 0; i < SPH_FB; ++i) ar[i] = ai[i] = 0.0;
    for (long long base = n0; base < n1; base += SPH_TILE) {
        // Stage the tile's non-zero voxels (their terms are the only
        // non-zero ones), compacted in voxel order: wave ballots give each
        // voxel its rank, so the sums keep the order of the voxels.
        __syncthreads();
        const long long n = base + t;
        const float a_n = n < n1 ? load_val(img, (size_t)n, img_dt) : 0.f;
        const bool keep = a_n != 0.f;
        const uint64_t bal = __ballot(keep);
        const int wv = t >> 6, ln = t & 63;
        if (ln == 0) wcnt[wv] = __popcll(bal);
        __syncthreads();
        int off = 0, cnt = 0;
#pragma unroll
        for (int w = 0; w < SPH_THREADS / 64; ++w) {
            const int c = wcnt[w];
            off += w < wv ? c : 0;
            cnt += c;
        }
        if (keep) {
            const int pos = off + __popcll(bal & ((1ull << ln) - 1ull));
            double x, y, z;
            node_pos(P, n, x, y, z);
            sx[pos] = x;
            sy[pos] = y;
            sz[pos] = z;
            sa[pos] = a_n;
        }
        // Per (transducer, voxel, face node) values shared by the
        // transducer's LB threads, formed once for SUB (voxel, node) items at
        // a time: tau = d/c0, the weight a w_node/(2 pi d) and the frequency
        // step exp(-j 2 pi df tau); items run voxel-major.
        const int NS = P.sph_ns;
        const int SUB = min(SPH_TILE * NS, SPH_SHARE / QB);
        for (int s0 = 0; s0 < cnt * NS; s0 += SUB) {
            const int m = min(SUB, cnt * NS - s0);
            __syncthreads();
            for (int idx = t; idx < QB * m; idx += SPH_THREADS) {
                // item (voxel jj, face node fs) of transducer qq
                const int ql = idx / m, it = s0 + idx % m;
                const int jj = it / NS, fs = it - jj * NS;
                const int qq = blockIdx.x * QB + ql;
                double tq = 0.0, wq = 0.0, cz = 1.0, szs = 0.0;
                if (qq < P.nq) {
                    const double4 fp = P.sph_pts[(size_t)qq * NS + fs];
                    const double vx = sx[jj] - fp.x, vy = sy[jj] - fp.y, vz = sz[jj] - fp.z;
                    const double dd = sqrt(fma(vz, vz, fma(vy, vy, vx * vx)));
                    tq = dd * inv_c0;
                    wq = (double)sa[jj] * fp.w / (6.283185307179586 * dd);
                    sincos_turns_d(frac_turn(df * tq), cz, szs);
                }
                stau[idx] = tq;
                sw[idx] = wq;
                sstep[idx] = make_double2(cz, -szs);   // exp(-j dtheta)
            }
            __syncthreads();
            if (!active) continue;
            const int row = (t / LB) * m;
            for (int jj = 0; jj < m; ++jj) {
                const double tau = stau[row + jj], w = sw[row + jj];
                const double2 zs = sstep[row + jj];
                float c, sn;
                sincos_turns((float)frac_turn(fa * tau), c, sn);
                // w exp(-j theta) = w (c, -sn), stepped by exp(-j dtheta) in
                // FP64 (as fast as FP32 here, and no conversions per term)
                double er = w * (double)c, ei = -(w * (double)sn);
                const double zr = zs.x, zi = zs.y;
#pragma unroll
                for (int i = 0; i < SPH_FB; ++i) {
                    ar[i] += er;
                    ai[i] += ei;
                    const double nr = fma(er, zr, -(ei * zi)), ni = fma(er, zi, ei * zr);
                    er = nr;
                    ei = ni;
                }
            }
        }
    }
    if (active) {
        double2 *dst = part + ((size_t)blockIdx.y * P.nq + q) * n_f;
        for (int i = 0; i < SPH_FB && l0 + i < n_f; ++i) dst[l0 + i] = make_double2(ar[i], ai[i]);
    }
}

// p0(f) of Eq. (p0f) with beta c0^3 / Cp = Gamma c0, ideal EIR; 0 at f = 0.
__device__ __forceinline__ double2 sph_p0(const Problem &P, double f)
{
    if (f == 0.0) return make_double2(0.0, 0.0);
    const double x = 3.141592653589793 * f * P.dxd / P.c0d;
    const double br = P.dxd / (2.0 * P.c0d) * cos(x) - sin(x) / (6.283185307179586 * f);
    return make_double2(0.0, -P.gammad * P.c0d / f * br);
}

// u[q][l] = p0(f_l) * sum over chunks (in chunk order) of part, as complex FP32.
__global__ void __launch_bounds__(SPH_THREADS)
sph_fwd_reduce_kernel(Problem P, const double2 *__restrict__ part, int nchunk, int n_f,
                      double f_min, double df, float2 *__restrict__ u)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)P.nq * n_f;
    if (i >= total) return;
    const int l = (int)(i % n_f);
    double sr = 0.0, si = 0.0;
    for (int c = 0; c < nchunk; ++c) {
        const double2 v = part[(size_t)c * total + i];
        sr += v.x;
        si += v.y;
    }
    const double2 p0 = sph_p0(P, f_min + df * (double)l);
    u[i] = make_float2((float)(p0.x * sr - p0.y * si), (float)(p0.x * si + p0.y * sr));
}

// SPH_NV consecutive voxels per thread:
//   out[n] = Re sum_q sum_l v[q,l] exp(+j 2 pi f_l d_qn / c0) / (2 pi d_qn),
//   v[q,l] = u[q,l] conj(p0(f_l)), staged per transducer in LDS.
// The frequencies are taken in blocks of SPH_ANCHOR.  Within a block,
// sum_i v[l0+i] z^i with z = exp(+j 2 pi df d/c0) is formed by Horner's rule
// in FP32 (S <- S z + v, four FMAs per term); the block's anchor
// A = exp(+j 2 pi f_l0 d/c0) comes from an FP64 recurrence (the first anchor
// and the block step are FP64 sin/cos of fractional turns), and Re(A S) is
// added in FP64.  One staged read serves the thread's voxels.
template <int IMG_DT>
__global__ void __launch_bounds__(SPH_THREADS)
sph_adj_kernel(Problem P, const float2 *__restrict__ u, int n_f, double f_min, double df,
               void *__restrict__ img, double *__restrict__ slice_sum, int q_per_slice)
{
    extern __shared__ float2 sv[];   // [qt][n_fp]: rows padded with zeros to whole blocks
    constexpr int NV = SPH_NV;
    const long long N = (long long)P.nx * P.ny * P.nz;
    const long long nb = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * NV;
    double x[NV], y[NV], z[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        x[v] = y[v] = z[v] = 0.0;
        if (nb + v < N) node_pos(P, nb + v, x[v], y[v], z[v]);
    }
    const double inv_c0 = 1.0 / P.c0d;
    const double dfa = df * SPH_ANCHOR;
    const int n_fp = (n_f + SPH_ANCHOR - 1) / SPH_ANCHOR * SPH_ANCHOR;
    const int qt = max(1, SPH_VQ / n_fp);   // transducers per LDS tile (32 KB)
    const int NS = P.sph_ns;                // face nodes per transducer
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    // Transducers of this slice (blockIdx.y); with one slice, all of them.
    const int qb = (int)blockIdx.y * q_per_slice, qe = min(P.nq, qb + q_per_slice);
    for (int q0 = qb; q0 < qe; q0 += qt) {
        const int nq = min(qt, qe - q0);
        __syncthreads();
        for (int k = threadIdx.x; k < nq * n_fp; k += blockDim.x) {
            const int jq = k / n_fp, l = k % n_fp;
            float2 val = make_float2(0.f, 0.f);   // zero terms pad the last block
            if (l < n_f) {
                const float2 w = u[(size_t)(q0 + jq) * n_f + l];
                const double2 p = sph_p0(P, f_min + df * (double)l);   // w * conj(p0)
                val = make_float2((float)(w.x * p.x + w.y * p.y), (float)(w.y * p.x - w.x * p.y));
            }
            sv[k] = val;
        }
        __syncthreads();
        if (nb >= N) continue;
        for (int jf = 0; jf < nq * NS; ++jf) {
            // transducer j, face node fs
            const int j = jf / NS, fs = jf - j * NS;
            const double4 fp = P.sph_pts[(size_t)(q0 + j) * NS + fs];
            float zr[NV], zi[NV];
            double ar[NV], ai[NV], gr[NV], gi[NV], rd[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double vx = x[v] - fp.x, vy = y[v] - fp.y, vz = z[v] - fp.z;
                const double dd = sqrt(fma(vz, vz, fma(vy, vy, vx * vx)));
                const double tau = dd * inv_c0;
                sincos_turns((float)frac_turn(df * tau), zr[v], zi[v]);
                sincos_turns_d(frac_turn(f_min * tau), ar[v], ai[v]);
                sincos_turns_d(frac_turn(dfa * tau), gr[v], gi[v]);
                rd[v] = fp.w / (6.283185307179586 * dd);
            }
            const float2 *vq = sv + j * n_fp;
            double part[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) part[v] = 0.0;
            for (int l0 = 0; l0 < n_fp; l0 += SPH_ANCHOR) {
                float sr[NV], si[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) sr[v] = si[v] = 0.f;
#pragma unroll
                for (int i = SPH_ANCHOR - 1; i >= 0; --i) {
                    const float2 w = vq[l0 + i];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const float nr = fmaf(sr[v], zr[v], fmaf(-si[v], zi[v], w.x));
                        const float ni = fmaf(sr[v], zi[v], fmaf(si[v], zr[v], w.y));
                        sr[v] = nr;
                        si[v] = ni;
                    }
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    part[v] = fma(ar[v], (double)sr[v], fma(-ai[v], (double)si[v], part[v]));
                    const double tr = ar[v] * gr[v] - ai[v] * gi[v];
                    ai[v] = ar[v] * gi[v] + ai[v] * gr[v];
                    ar[v] = tr;
                }
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] = fma(part[v], rd[v], acc[v]);
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (nb + v >= N) continue;
        if (slice_sum)
            slice_sum[(size_t)blockIdx.y * N + nb + v] = acc[v];
        else
            store_val(img, (size_t)(nb + v), IMG_DT, (float)acc[v]);
    }
}

// img[n] = sum over the slices, in slice order, of slice_sum[slice][n].
__global__ void __launch_bounds__(SPH_THREADS)
sph_adj_sum_kernel(const double *__restrict__ slice_sum, int slices, long long N,
                   void *__restrict__ img, int img_dt)
{
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double acc = 0.0;
    for (int sl = 0; sl < slices; ++sl) acc += slice_sum[(size_t)sl * N + n];
    store_val(img, (size_t)n, img_dt, (float)acc);
}

// Device scratch of oat_sph_backproject_noalloc: the adjoint's FP64 slice
// partial images.  Each GPU the library runs on holds its own copy until the
// process ends.  In host code this name is only a stand-in for the symbol:
// kernels and copies get the address that sph_scratch_address resolved.
static __device__ __align__(256) double scratch[SPH_SCRATCH_BYTES / sizeof(double)];

}  // namespace

hipError_t sph_scratch_address(int device, double **out)
{
    static std::mutex mu;
    static std::vector<double *> addr;   // per device ordinal; null until resolved
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0) return hipErrorInvalidDevice;
    if ((size_t)device >= addr.size()) addr.resize((size_t)device + 1, nullptr);
    if (!addr[(size_t)device]) {
        double *p = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[(size_t)device] = p;
    }
    *out = addr[(size_t)device];
    return hipSuccess;
}

size_t sph_workspace_bytes(const Problem &P, int n_f)
{
    return sizeof(double2) * (size_t)SPH_CHUNKS * P.nq * n_f;
}

hipError_t launch_sph_project(const Problem &P, const void *img, int img_dt, float2 *u, int n_f,
                              double f_min, double df, double2 *part, hipStream_t s)
{
    const long long N = (long long)P.nx * P.ny * P.nz;
    // n_f <= SPH_THREADS * SPH_FB (checked by the caller): a transducer's
    // frequency blocks fit one workgroup.
    const int LB = (n_f + SPH_FB - 1) / SPH_FB;
    const int QB = SPH_THREADS / LB;
    const long long chunk_len = (N + SPH_CHUNKS - 1) / SPH_CHUNKS;
    const int nchunk = (int)((N + chunk_len - 1) / chunk_len);
    dim3 grid((P.nq + QB - 1) / QB, nchunk);
    hipLaunchKernelGGL(sph_fwd_kernel, grid, dim3(SPH_THREADS), 0, s, P, img, img_dt, n_f, f_min,
                       df, LB, chunk_len, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long total = (long long)P.nq * n_f;
    hipLaunchKernelGGL(sph_fwd_reduce_kernel, dim3((unsigned)((total + SPH_THREADS - 1) / SPH_THREADS)),
                       dim3(SPH_THREADS), 0, s, P, part, nchunk, n_f, f_min, df, u);
    return hipGetLastError();
}

// Transducer slices of the adjoint: a grid of fewer than 1024 workgroups
// (a small image) takes the transducers in up to 4 slices along grid y, so
// the device holds more waves; their FP64 partial images are then added in
// slice order.
int sph_adj_slices(const Problem &P)
{
    const long long N = (long long)P.nx * P.ny * P.nz;
    const long long blocks = ((N + SPH_NV - 1) / SPH_NV + SPH_THREADS - 1) / SPH_THREADS;
    if (blocks >= 1024) return 1;
    long long sl = (1024 + blocks - 1) / blocks;
    if (sl > 4) sl = 4;
    if (sl > P.nq) sl = P.nq;
    return (int)sl;
}

size_t sph_adj_workspace_bytes(const Problem &P)
{
    const int S = sph_adj_slices(P);
    return S > 1 ? sizeof(double) * (size_t)S * P.nx * P.ny * P.nz : 0;
}

hipError_t launch_sph_backproject(const Problem &P, const float2 *u, int n_f, double f_min,
                                  double df, void *img, int img_dt, double *work, hipStream_t s)
{
    const long long N = (long long)P.nx * P.ny * P.nz;
    const int n_fp = (n_f + SPH_ANCHOR - 1) / SPH_ANCHOR * SPH_ANCHOR;
    const int qt = (SPH_VQ / n_fp) > 1 ? SPH_VQ / n_fp : 1;
    const size_t shm = sizeof(float2) * (size_t)qt * n_fp;
    const long long threads = (N + SPH_NV - 1) / SPH_NV;
    const int S = sph_adj_slices(P);
    if (S > 1 && !work) return hipErrorInvalidValue;
    const int qps = (P.nq + S - 1) / S;
    double *slice_sum = S > 1 ? work : nullptr;
    dim3 grid((unsigned)((threads + SPH_THREADS - 1) / SPH_THREADS), (unsigned)S);
    if (img_dt == 0)
        hipLaunchKernelGGL(sph_adj_kernel<0>, grid, dim3(SPH_THREADS), shm, s, P, u, n_f, f_min, df,
                           img, slice_sum, qps);
    else
        hipLaunchKernelGGL(sph_adj_kernel<1>, grid, dim3(SPH_THREADS), shm, s, P, u, n_f, f_min, df,
                           img, slice_sum, qps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || S == 1) return e;
    hipLaunchKernelGGL(sph_adj_sum_kernel, dim3((unsigned)((N + SPH_THREADS - 1) / SPH_THREADS)),
                       dim3(SPH_THREADS), 0, s, slice_sum, S, N, img, img_dt);
    return hipGetLastError();
}

}  // namespace oat
