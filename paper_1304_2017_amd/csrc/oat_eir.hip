// Transducer electrical impulse response (EIR) on gfx950: the convolution
// H^e of Eq. (EIR) and its transpose (Sec. II.B.3), and the Hann-window
// Fourier deconvolution that compensates the EIR before FBP (Sec. IV.B).
//
// All three work per transducer row of the [n_det][n_t] data, one workgroup
// per row, in FP64 (sums, spectrum and FFT), with one rounding to the output
// type; the work is O(n_t * taps) and O(N log N) per row, small next to G.
#include "oat_dtype.hpp"
#include "oat_internal.hpp"

#pragma clang fp contract(off)

namespace oat {

namespace {

constexpr int EIR_THREADS = 256;

// ADJ = 0: out[k] = sum_m h[m] in[k - 1 - m]  (Eq. (EIR), h[m] = 0 outside [0, L));
// ADJ = 1: out[k] = sum_m h[m] in[k + 1 + m]  (its transpose, Sec. II.B.3).
// The row and the taps sit in LDS in FP64: (K + L) * 8 bytes <= 64 KB.
template <int ADJ>
__global__ void __launch_bounds__(EIR_THREADS)
eir_kernel(const void *__restrict__ in, int in_dt, void *__restrict__ out, int out_dt,
           const double *__restrict__ h, int L, int K)
{
    extern __shared__ double sm[];
    double *row = sm, *tap = sm + K;
    const size_t base = (size_t)blockIdx.x * K;
    for (int k = threadIdx.x; k < K; k += blockDim.x) row[k] = (double)load_val(in, base + k, in_dt);
    for (int m = threadIdx.x; m < L; m += blockDim.x) tap[m] = h[m];
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        double acc = 0.0;
        if (ADJ == 0) {
            const int mmax = min(L - 1, k - 1);
            for (int m = 0; m <= mmax; ++m) acc = fma(tap[m], row[k - 1 - m], acc);
        } else {
            const int mmax = min(L - 1, K - 2 - k);
            for (int m = 0; m <= mmax; ++m) acc = fma(tap[m], row[k + 1 + m], acc);
        }
        store_val(out, base + k, out_dt, (float)acc);
    }
}

// Transform of the delayed response on the N-point grid and the twiddles:
// Ht[n] = sum_m h[m] exp(-2 pi i n (m + 1) / N) by a direct FP64 sum (the
// exponent index is reduced mod N exactly), tw[n] = exp(-2 pi i n / N).
__global__ void __launch_bounds__(EIR_THREADS)
eir_spectrum_kernel(const double *__restrict__ h, int L, int N, double2 *__restrict__ Ht,
                    double2 *__restrict__ tw)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n < N) {
        double re = 0.0, im = 0.0;
        for (int m = 0; m < L; ++m) {
            const long long e = ((long long)n * (m + 1)) % N;
            double s, c;
            sincospi(2.0 * (double)e / (double)N, &s, &c);
            re = fma(h[m], c, re);
            im = fma(-h[m], s, im);
        }
        Ht[n] = make_double2(re, im);
    }
    if (n < N / 2) {
        double s, c;
        sincospi(2.0 * (double)n / (double)N, &s, &c);
        tw[n] = make_double2(c, -s);
    }
}

// Deconvolution filter of one call: F[n] = W(|f_n|) / Ht[n] with the FFT
// frequency f_n = n / (N dt) for n < N/2, (n - N) / (N dt) otherwise, the
// Hann window W(f) = (1 - cos(pi (fc - f) / fc)) / 2 for f <= fc, 0 beyond;
// 0 where Ht[n] = 0.
__global__ void __launch_bounds__(EIR_THREADS)
deconv_filter_kernel(const double2 *__restrict__ Ht, int N, double dt, double fc,
                     double2 *__restrict__ F)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const double f = fabs((double)(n < N / 2 ? n : n - N) / ((double)N * dt));
    const double w = f <= fc ? 0.5 * (1.0 - cospi((fc - f) / fc)) : 0.0;
    const double2 H = Ht[n];
    const double d = H.x * H.x + H.y * H.y;
    F[n] = (d > 0.0 && w != 0.0) ? make_double2(w * H.x / d, -w * H.y / d) : make_double2(0.0, 0.0);
}

// In-place radix-2 decimation in time on bit-reversed input (natural-order
// output); inverse with conjugate twiddles.  tw[t] = exp(-2 pi i t / N).
__device__ __forceinline__ void fft_stages(double2 *x, const double2 *__restrict__ tw, int N,
                                           int logN, bool inv)
{
    for (int s = 0; s < logN; ++s) {
        const int hs = 1 << s;
        for (int b = threadIdx.x; b < N / 2; b += blockDim.x) {
            const int pos = b & (hs - 1);
            const int i = ((b >> s) << (s + 1)) + pos, j = i + hs;
            double2 w = tw[pos << (logN - 1 - s)];
            if (inv) w.y = -w.y;
            const double2 a = x[i], c = x[j];
            const double tr = w.x * c.x - w.y * c.y, ti = w.x * c.y + w.y * c.x;
            x[i] = make_double2(a.x + tr, a.y + ti);
            x[j] = make_double2(a.x - tr, a.y - ti);
        }
        __syncthreads();
    }
}

// One row: zero-pad to N, transform, multiply by F, transform back, keep
// the first K samples (divided by N).
template <int NMAX>
__global__ void __launch_bounds__(EIR_THREADS)
deconv_kernel(const void *__restrict__ u, int u_dt, void *__restrict__ p, int p_dt,
              const double2 *__restrict__ F, const double2 *__restrict__ tw, int K, int N, int logN)
{
    __shared__ double2 x[NMAX];
    const size_t base = (size_t)blockIdx.x * K;
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const int r = (int)(__brev((unsigned)n) >> (32 - logN));
        x[r] = make_double2(n < K ? (double)load_val(u, base + n, u_dt) : 0.0, 0.0);
    }
    __syncthreads();
    fft_stages(x, tw, N, logN, false);
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const double2 a = x[n], f = F[n];
        x[n] = make_double2(a.x * f.x - a.y * f.y, a.x * f.y + a.y * f.x);
    }
    __syncthreads();
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const int r = (int)(__brev((unsigned)n) >> (32 - logN));
        if (n < r) {
            const double2 t = x[n];
            x[n] = x[r];
            x[r] = t;
        }
    }
    __syncthreads();
    fft_stages(x, tw, N, logN, true);
    const double inv_n = 1.0 / (double)N;
    for (int k = threadIdx.x; k < K; k += blockDim.x) store_val(p, base + k, p_dt, (float)(x[k].x * inv_n));
}

}  // namespace

hipError_t launch_eir(const Problem &P, const void *in, int in_dt, void *out, int out_dt,
                      const double *h, int taps, int adjoint, hipStream_t s)
{
    const size_t shm = sizeof(double) * (size_t)(P.nt + taps);
    if (adjoint)
        hipLaunchKernelGGL(eir_kernel<1>, dim3(P.nq), dim3(EIR_THREADS), shm, s, in, in_dt, out,
                           out_dt, h, taps, P.nt);
    else
        hipLaunchKernelGGL(eir_kernel<0>, dim3(P.nq), dim3(EIR_THREADS), shm, s, in, in_dt, out,
                           out_dt, h, taps, P.nt);
    return hipGetLastError();
}

hipError_t launch_eir_spectrum(const double *h, int taps, int N, double2 *Ht, double2 *tw,
                               hipStream_t s)
{
    hipLaunchKernelGGL(eir_spectrum_kernel, dim3((N + EIR_THREADS - 1) / EIR_THREADS),
                       dim3(EIR_THREADS), 0, s, h, taps, N, Ht, tw);
    return hipGetLastError();
}

hipError_t launch_deconvolve(const Problem &P, const void *u, int u_dt, void *p, int p_dt,
                             const double2 *Ht, const double2 *tw, double2 *F, int N, double fc,
                             hipStream_t s)
{
    int logN = 0;
    while ((1 << logN) < N) ++logN;
    hipLaunchKernelGGL(deconv_filter_kernel, dim3((N + EIR_THREADS - 1) / EIR_THREADS),
                       dim3(EIR_THREADS), 0, s, Ht, N, (double)P.dtd, fc, F);
    if (N <= 2048)
        hipLaunchKernelGGL(deconv_kernel<2048>, dim3(P.nq), dim3(EIR_THREADS), 0, s, u, u_dt, p,
                           p_dt, F, tw, P.nt, N, logN);
    else if (N <= 4096)
        hipLaunchKernelGGL(deconv_kernel<4096>, dim3(P.nq), dim3(EIR_THREADS), 0, s, u, u_dt, p,
                           p_dt, F, tw, P.nt, N, logN);
    else
        hipLaunchKernelGGL(deconv_kernel<8192>, dim3(P.nq), dim3(EIR_THREADS), 0, s, u, u_dt, p,
                           p_dt, F, tw, P.nt, N, logN);
    return hipGetLastError();
}

}  // namespace oat
