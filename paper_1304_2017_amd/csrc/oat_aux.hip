// Data-side kernels on gfx950: the reduction of G's brick partials fused
// with D (Eq. (dis_g2p)), its transpose D^T (Sec. II.B.3), the gather of G^T's
// brick boxes into the image, and the voxel-driven filtered backprojection
// of Eq. (disfbp).
#include "oat_dtype.hpp"
#include "oat_internal.hpp"
#include "oat_fbp_window.hpp"

#pragma clang fp contract(off)

namespace oat {

namespace {

constexpr int RED_WAVES = 4;

// floor(x) as an integer in one instruction.
__device__ __forceinline__ int cvt_floor(float x)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

}  // namespace

// One workgroup per transducer: sum the (brick, transducer) windows of G in
// a fixed order (each wave keeps its own copy, the copies are added in wave
// order), then apply D on the whole trace.  Deterministic.
__global__ void __launch_bounds__(RED_WAVES *WAVE)
srt_reduce_kernel(Problem P, const float *__restrict__ part, const int *__restrict__ klo,
                  void *__restrict__ out, int out_dt, int apply_d)
{
    extern __shared__ float sg[];   // RED_WAVES * nt
    const int q = blockIdx.x;
    const int K = P.nt;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    for (int i = threadIdx.x; i < RED_WAVES * K; i += blockDim.x) sg[i] = 0.f;
    __syncthreads();
    const int nb = P.nbx * P.nby * P.nbz;
    float *mine = sg + wave * K;
    // Four of the wave's bricks per pass, all their loads issued before
    // the adds, which keep the brick order (the sums do not change).
    constexpr int U = 4, H = WMAX / WAVE;
    for (int b0 = wave; b0 < nb; b0 += U * RED_WAVES) {
        int kl[U];
        float v[U][H];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int b = b0 + u * RED_WAVES;
            kl[u] = K;
#pragma unroll
            for (int h = 0; h < H; ++h) v[u][h] = 0.f;
            if (b < nb) {
                const size_t row = (size_t)b * P.nq + q;
                kl[u] = klo[row];
                const float *src = part + row * P.window;
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    const int j = lane + h * WAVE;
                    if (j < P.window) v[u][h] = src[j];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const int j = lane + h * WAVE, k = kl[u] + j;
                if (j < P.window && k < K) mine[k] += v[u][h];
            }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        float s = sg[k];
        for (int w = 1; w < RED_WAVES; ++w) s += sg[w * K + k];
        sg[k] = s;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        float v;
        if (apply_d) {
            // s_k = g_k / t_k (0 where t_k <= 0); p_k = coef (s_{k+1} - s_{k-1})
            float sp = 0.f, sm = 0.f;
            if (k + 1 < K) {
                float t = fmaf((float)(k + 1), P.dt, P.t0);
                sp = t > 0.f ? sg[k + 1] / t : 0.f;
            }
            if (k - 1 >= 0) {
                float t = fmaf((float)(k - 1), P.dt, P.t0);
                sm = t > 0.f ? sg[k - 1] / t : 0.f;
            }
            v = P.d_coef * (sp - sm);
        } else {
            v = sg[k];
        }
        store_val(out, (size_t)q * K + k, out_dt, v);
    }
}

// g'[q,k] = coef (y_{k-1} - y_{k+1}) / t_k  (0 where t_k <= 0; y_{-1} = y_K = 0),
// or a plain FP32 copy of y when apply_dt == 0.  One workgroup per transducer
// q, which also writes P.gp_rowmax[q], the largest |g'| among its samples
// whose shell can reach the image support (G^T sets its fixed-point scales
// from these; the other samples meet no quadrature point).
__global__ void __launch_bounds__(256) diff_adj_kernel(Problem P, const void *__restrict__ y,
                                                       int y_dt, float *__restrict__ gp,
                                                       int apply_dt)
{
    __shared__ float wmax[4];
    const int q = blockIdx.x;
    const size_t row = (size_t)q * P.nt;
    const float dq = P.det[q].dist;
    float m = 0.f;
    for (int k = threadIdx.x; k < P.nt; k += blockDim.x) {
        const size_t i = row + k;
        float v;
        if (apply_dt) {
            float t = fmaf((float)k, P.dt, P.t0);
            float ym = k > 0 ? load_val(y, i - 1, y_dt) : 0.f;
            float yp = k + 1 < P.nt ? load_val(y, i + 1, y_dt) : 0.f;
            v = t > 0.f ? P.d_coef * (ym - yp) / t : 0.f;
        } else {
            v = load_val(y, i, y_dt);
        }
        gp[i] = v;
        const float rho = fmaf((float)k, P.rho_step, P.rho0);
        if (fabsf(rho - dq) <= P.r_sup + 2.f) m = fmaxf(m, fabsf(v));
    }
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        P.gp_rowmax[q] = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
}

// G^T output.  A brick's box holds the nodes of its cells, one node below
// its first owned node through its last owned node, so node c (per axis)
// receives the box of its owner brick c / BRICK and, when c is the last node
// of that brick, the box of the next brick, where c is box node 0.  Each box
// comes in `slices` parts (one per slice of the transducer windows).  The at
// most 8 x slices contributions are added in a fixed order: the result is
// deterministic.
template <int IMG_DT>
__global__ void __launch_bounds__(256)
adj_gather_kernel(Problem P, const double *__restrict__ acc, int slices, void *__restrict__ img)
{
    const int x = blockIdx.x * 64 + threadIdx.x % 64;
    const int y = blockIdx.y * 4 + threadIdx.x / 64;
    const int z = blockIdx.z;
    if (x >= P.nx || y >= P.ny) return;
    const int c[3] = {x, y, z};
    const int nb[3] = {P.nbx, P.nby, P.nbz};
    int bi[3][2], off[3][2], cnt[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int b0 = c[a] / BRICK, r = c[a] - b0 * BRICK;
        bi[a][0] = b0;
        off[a][0] = r + 1;
        bi[a][1] = b0 + 1;
        off[a][1] = 0;
        cnt[a] = (r == BRICK - 1 && b0 + 1 < nb[a]) ? 2 : 1;
    }
    const size_t slice_len = (size_t)P.nbx * P.nby * P.nbz * BOX3;
    double sum = 0.0;
    for (int iz = 0; iz < cnt[2]; ++iz)
        for (int iy = 0; iy < cnt[1]; ++iy)
            for (int ix = 0; ix < cnt[0]; ++ix) {
                const size_t b = ((size_t)bi[2][iz] * P.nby + bi[1][iy]) * P.nbx + bi[0][ix];
                const size_t i = b * BOX3 + (off[2][iz] * BOX + off[1][iy]) * BOX + off[0][ix];
                for (int sl = 0; sl < slices; ++sl) sum += acc[sl * slice_len + i];
            }
    store_val(img, ((size_t)z * P.ny + y) * P.nx + x, IMG_DT, (float)sum);
}

// FBP, Eq. (disfbp): a block takes a 16 x 16 x 8 tile of voxels, each thread
// a column of FBP_TZ = 8 voxels along z, and loops over the transducers in
// chunks; the transducer's data (position, weight, staged window) and the
// x/y part of the squared distance are loaded or formed once per column.
// For each chunk the samples a tile can touch, k in [k_lo, k_lo + win), are
// staged in LDS per transducer (zero outside [0, K)), so each update reads
// p_k and p_{k+1} with one LDS access.  k~ is formed in FP32; when its
// fractional part lies within the FP32 error bound of an integer, floor(k~)
// is decided exactly as the FP64 problem statement takes it (the plan's
// threshold table), because Eq. (disfbp) switches its forward difference at
// integer k~.
constexpr int FBP_LDS = 8192;   // floats of staged samples per chunk

template <int P_DT, int IMG_DT>
__global__ void __launch_bounds__(FBP_TX *FBP_TY)
fbp_kernel(Problem P, const void *__restrict__ pres, void *__restrict__ img, int win, int chunk)
{
    __shared__ float sp[FBP_LDS];
    __shared__ int2 sklo[FBP_LDS / 8];    // first staged sample, 1/2 - FP64-decision tolerance
    const int tx = threadIdx.x % FBP_TX, ty = threadIdx.x / FBP_TX;
    const int ix = blockIdx.x * FBP_TX + tx, iy = blockIdx.y * FBP_TY + ty;
    const int iz0 = blockIdx.z * FBP_TZ;
    const float fx = (float)ix, fy = (float)iy;
    float fz[FBP_TZ];
#pragma unroll
    for (int v = 0; v < FBP_TZ; ++v) fz[v] = (float)(iz0 + v);
    // tile centre and half-diagonal (grid units)
    const float cx = blockIdx.x * FBP_TX + 0.5f * (FBP_TX - 1), cy = blockIdx.y * FBP_TY + 0.5f * (FBP_TY - 1);
    const float cz = iz0 + 0.5f * (FBP_TZ - 1);
    const float hd = fbp_half_diag();
    const int K = P.nt;
    // With fr = kt - k and inv = 1/(kt + tau) = ri c0 dt / dx, the two
    // coefficients of Eq. (disfbp) are (1 - fr) inv - 1/2 and fr inv + 1/2,
    // so a transducer adds w inv (p_k + fr (p_{k+1} - p_k)) + w (p_{k+1} - p_k) / 2.
    // acc_a sums w ri (p_k + fr dp), acc_b sums w dp; the scale is applied once.
    float acc_a[FBP_TZ], acc_b[FBP_TZ];
#pragma unroll
    for (int v = 0; v < FBP_TZ; ++v) acc_a[v] = acc_b[v] = 0.f;
    for (int q0 = 0; q0 < P.nq; q0 += chunk) {
        const int nq = min(chunk, P.nq - q0);
        __syncthreads();
        for (int j = threadIdx.x; j < nq; j += blockDim.x) {
            const DetRec &d = P.det[q0 + j];
            const float vx = cx - d.uqf[0], vy = cy - d.uqf[1], vz = cz - d.uqf[2];
            const float dc = sqrtf(vx * vx + vy * vy + vz * vz);
            // |FP32 kt - kt| <= 5e-7 (kt + tau) + 1e-6 (transducer position
            // rounded to FP32, the difference, the squared norm, rsqrt to
            // 1 ulp, the product); the tolerance is twice that at the tile's
            // largest kt.
            const float tol = fmaf(1e-6f, (dc + hd + 1.f) * P.sigma, 1e-5f);
            sklo[j] = make_int2(fbp_first_sample(dc, P.sigma, P.tau), __float_as_int(0.5f - tol));
        }
        __syncthreads();
        for (int t = threadIdx.x; t < nq * win; t += blockDim.x) {
            const int j = t / win, i = t % win;
            const int k = sklo[j].x + i;
            float v = 0.f;
            if (k >= 0 && k < K) {
                const size_t idx = (size_t)(q0 + j) * K + k;
                v = P_DT == 0 ? ((const float *)pres)[idx]
                              : __uint_as_float(((unsigned)((const unsigned short *)pres)[idx]) << 16);
            }
            sp[t] = v;
        }
        __syncthreads();
        for (int j = 0; j < nq; ++j) {
            const DetRec &d = P.det[q0 + j];
            const float vx = fx - d.uqf[0], vy = fy - d.uqf[1];
            const float rxy = fmaf(vy, vy, vx * vx);
            const int2 sk = sklo[j];
            const float *row = sp + j * win;
#pragma unroll
            for (int v = 0; v < FBP_TZ; ++v) {
                const float vz = fz[v] - d.uqf[2];
                const float r2 = fmaf(vz, vz, rxy);
                // r2 is hundreds of cells squared: the hardware rsqrt (1 ulp)
                // needs no denormal scaling.
                const float ri = __builtin_amdgcn_rsqf(r2);
                const float kt = fmaf(r2 * ri, P.sigma, -P.tau);
                float fr = __builtin_amdgcn_fractf(kt);
                int ki = cvt_floor(kt);
                // Within the tolerance of an integer m, floor(kt) of the FP64
                // problem statement is m - 1 or m: decided by the FP64 squared
                // distance in physical units (no contraction here) against the
                // plan's threshold for m.  Outside m = -1 .. K both candidates
                // select zero samples.
                if (fabsf(fr - 0.5f) > __int_as_float(sk.y)) {
                    const int m = fr > 0.5f ? ki + 1 : ki;
                    if (m >= -1 && m <= K) {
                        const double x = P.x0 + ix * P.dxd, y = P.y0 + iy * P.dxd,
                                     z = P.z0 + (iz0 + v) * P.dxd;
                        const double wx = x - d.r[0], wy = y - d.r[1], wz = z - d.r[2];
                        const double r2d = wx * wx + wy * wy + wz * wz;
                        ki = r2d >= P.fbp_thr[m + 1] ? m : m - 1;
                        fr = kt - (float)ki;
                    }
                }
                // ki - sk.x lies in 0 .. win - 2 (the window spans the tile's
                // sample range with margins; tests/host/fbp_window_check.cpp
                // checks it over every workload geometry); the unsigned
                // minimum only keeps the reads inside the row.
                const unsigned li = min((unsigned)(ki - sk.x), (unsigned)(win - 2));
                const float p0 = row[li], dp = row[li + 1] - p0;
                acc_a[v] = fmaf(d.fbp_w * ri, fmaf(fr, dp, p0), acc_a[v]);
                acc_b[v] = fmaf(d.fbp_w, dp, acc_b[v]);
            }
        }
    }
    if (ix < P.nx && iy < P.ny) {
#pragma unroll
        for (int v = 0; v < FBP_TZ; ++v) {
            if (iz0 + v >= P.nz) break;
            const size_t n = ((size_t)(iz0 + v) * P.ny + iy) * P.nx + ix;
            const float val = P.fbp_scale * fmaf(P.inv_sigma, acc_a[v], 0.5f * acc_b[v]);
            if (IMG_DT == 0)
                ((float *)img)[n] = val;
            else
                ((unsigned short *)img)[n] = to_bf16(val);
        }
    }
}

hipError_t launch_srt_reduce(const Problem &P, const float *part, const int *klo, void *out,
                             int out_dtype, int apply_d, hipStream_t s)
{
    size_t shm = (size_t)RED_WAVES * P.nt * sizeof(float);
    hipLaunchKernelGGL(srt_reduce_kernel, dim3(P.nq), dim3(RED_WAVES * WAVE), shm, s, P, part, klo,
                       out, out_dtype, apply_d);
    return hipGetLastError();
}

hipError_t launch_diff_adj(const Problem &P, const void *y, int y_dtype, float *gp, int apply_dt,
                           hipStream_t s)
{
    hipLaunchKernelGGL(diff_adj_kernel, dim3(P.nq), dim3(256), 0, s, P, y, y_dtype, gp, apply_dt);
    return hipGetLastError();
}

hipError_t launch_adj_gather(const Problem &P, const double *acc, void *img, int img_dtype,
                             hipStream_t s)
{
    dim3 grid((P.nx + 63) / 64, (P.ny + 3) / 4, P.nz), block(256);
    const int sl = adj_slices(P.nbx * P.nby * P.nbz, P.nq);
    if (img_dtype == 0)
        hipLaunchKernelGGL(adj_gather_kernel<0>, grid, block, 0, s, P, acc, sl, img);
    else
        hipLaunchKernelGGL(adj_gather_kernel<1>, grid, block, 0, s, P, acc, sl, img);
    return hipGetLastError();
}

hipError_t launch_fbp(const Problem &P, const void *p, int p_dtype, void *img, int img_dtype,
                      hipStream_t s)
{
    // Samples a tile can touch per transducer: its diagonal in shells plus margins.
    const int win = fbp_window(P.sigma);
    int chunk = FBP_LDS / win;
    if (chunk > FBP_LDS / 8) chunk = FBP_LDS / 8;
    if (chunk < 1) return hipErrorInvalidValue;
    dim3 grid((P.nx + FBP_TX - 1) / FBP_TX, (P.ny + FBP_TY - 1) / FBP_TY, (P.nz + FBP_TZ - 1) / FBP_TZ);
    dim3 block(FBP_TX * FBP_TY);
    if (p_dtype == 0 && img_dtype == 0)
        hipLaunchKernelGGL((fbp_kernel<0, 0>), grid, block, 0, s, P, p, img, win, chunk);
    else if (p_dtype == 0)
        hipLaunchKernelGGL((fbp_kernel<0, 1>), grid, block, 0, s, P, p, img, win, chunk);
    else if (img_dtype == 0)
        hipLaunchKernelGGL((fbp_kernel<1, 0>), grid, block, 0, s, P, p, img, win, chunk);
    else
        hipLaunchKernelGGL((fbp_kernel<1, 1>), grid, block, 0, s, P, p, img, win, chunk);
    return hipGetLastError();
}

}  // namespace oat
