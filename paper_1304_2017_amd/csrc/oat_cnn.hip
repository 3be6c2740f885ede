// Small 3-D convolution network on gfx950: "same" 3x3x3 convolutions with
// 1 or 16 channels, their weight gradient, Adam and a mean-squared-error
// loss, behind the C ABI of include/oat_cnn.h.  Used as a learned
// preconditioner of the PLS reconstruction; activations stored in FP32 or
// BF16, all sums in FP32 (weights) or FP64 (loss).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "oat.h"
#include "oat_cnn.h"
#include "oat_internal.hpp"

namespace {

constexpr int TT = 8;               // output tile edge
constexpr int TI = TT + 2;          // input tile edge (one-voxel halo)
constexpr int TI3 = TI * TI * TI;   // 1000
constexpr int TT3 = TT * TT * TT;   // 512
constexpr int NT = 512;             // threads per workgroup

__device__ __forceinline__ float ldv(const void *p, size_t i, int dt)
{
    if (dt == 0) return ((const float *)p)[i];
    return __uint_as_float(((unsigned)((const unsigned short *)p)[i]) << 16);
}

__device__ __forceinline__ void stv(void *p, size_t i, int dt, float v)
{
    if (dt == 0) {
        ((float *)p)[i] = v;
    } else {
        unsigned u = __float_as_uint(v);
        u += 0x7fffu + ((u >> 16) & 1u);     // round to nearest even
        ((unsigned short *)p)[i] = (unsigned short)(u >> 16);
    }
}

// Input tile of CI channels with a one-voxel halo (zero outside the volume).
template <int CI>
__device__ __forceinline__ void load_tile(float (*xs)[TI3], const void *x, int xdt, int D, int H,
                                          int W, int x0, int y0, int z0)
{
    const size_t plane = (size_t)H * W, vol = plane * D;
    for (int i = threadIdx.x; i < CI * TI3; i += NT) {
        const int ci = i / TI3, r = i - ci * TI3;
        const int zz = r / (TI * TI), yy = (r / TI) % TI, xx = r % TI;
        const int gz = z0 - 1 + zz, gy = y0 - 1 + yy, gx = x0 - 1 + xx;
        float v = 0.f;
        if (gz >= 0 && gz < D && gy >= 0 && gy < H && gx >= 0 && gx < W)
            v = ldv(x, ci * vol + gz * plane + (size_t)gy * W + gx, xdt);
        xs[ci][r] = v;
    }
}

// Tile of the VALU forward: FX x FY x FZ = 512 output voxels.  With one
// input channel it is 64 x 4 x 2, so a wave's 64 consecutive voxels write
// whole cache lines of each of its output channels; 16 -> 1 takes 32 x 4 x 4
// (a halo tile of 78 KB of FP32 values), 16 -> 16 an 8^3 cube (the smallest
// halo: its cost is the 6912 products per voxel, not the stores).
template <int CI, int CO> struct FwdTile {
    static constexpr int FX = CI == 1 ? 64 : (CO == 1 ? 32 : 8);
    static constexpr int FY = CI == 1 ? 4 : (CO == 1 ? 4 : 8);
    static constexpr int FZ = CI == 1 ? 2 : (CO == 1 ? 4 : 8);
    static constexpr int HX = FX + 2, HY = FY + 2, HZ = FZ + 2, HALO = HX * HY * HZ;
};

// One output voxel per thread, all CO channels; FwdTile<CI, CO> voxels per workgroup.
template <int CI, int CO>
__global__ void __launch_bounds__(NT) conv_fwd_kernel(const void *__restrict__ x, int xdt, int D,
                                                      int H, int W, const float *__restrict__ wt,
                                                      const float *__restrict__ bias,
                                                      void *__restrict__ y, int ydt, int relu,
                                                      const void *__restrict__ mask)
{
    using T = FwdTile<CI, CO>;
    static_assert(T::FX * T::FY * T::FZ == NT, "one voxel per thread");
    __shared__ float xs[CI][T::HALO];
    __shared__ float ws[CI * 27][CO];       // [ci][tap][co]: a broadcast read per (ci, tap)
    const int x0 = blockIdx.x * T::FX, y0 = blockIdx.y * T::FY, z0 = blockIdx.z * T::FZ;
    const size_t plane = (size_t)H * W, vol = plane * D;
    if constexpr (CO != 1)
        for (int i = threadIdx.x; i < CI * 27 * CO; i += NT) {
            const int co = i % CO, r = i / CO, ci = r / 27, t = r % 27;
            ws[r][co] = wt[(co * CI + ci) * 27 + t];
        }
    // halo tile, zero outside the volume; consecutive threads take
    // consecutive x, so the loads of a row are coalesced
    for (int i = threadIdx.x; i < CI * T::HALO; i += NT) {
        const int ci = i / T::HALO, r = i - ci * T::HALO;
        const int zz = r / (T::HX * T::HY), yy = (r / T::HX) % T::HY, xx = r % T::HX;
        const int gz = z0 - 1 + zz, gy = y0 - 1 + yy, gx = x0 - 1 + xx;
        float v = 0.f;
        if (gz >= 0 && gz < D && gy >= 0 && gy < H && gx >= 0 && gx < W)
            v = ldv(x, ci * vol + gz * plane + (size_t)gy * W + gx, xdt);
        xs[ci][r] = v;
    }
    __syncthreads();
    const int lx = threadIdx.x % T::FX, ly = (threadIdx.x / T::FX) % T::FY,
              lz = threadIdx.x / (T::FX * T::FY);
    float acc[CO];
#pragma unroll
    for (int co = 0; co < CO; ++co) acc[co] = bias ? bias[co] : 0.f;
    if constexpr (CO == 1) {
        // One output channel: the weights are the same for every thread, so
        // a channel's 27 come through the scalar cache, and the LDS serves
        // only the voxel values.
        for (int ci = 0; ci < CI; ++ci) {
            const float *wc = wt + ci * 27;
#pragma unroll
            for (int t = 0; t < 27; ++t) {
                const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
                const float v = xs[ci][((lz + dz) * T::HY + ly + dy) * T::HX + lx + dx];
                acc[0] = fmaf(wc[t], v, acc[0]);
            }
        }
    } else {
        // Taps in rows of 3 along x: a row's weights are read when it runs
        // (a fully unrolled loop would hold all CI x 27 x CO weights in
        // registers).
        for (int ci = 0; ci < CI; ++ci) {
#pragma unroll 1
            for (int r = 0; r < 9; ++r) {
                const int dz = r / 3, dy = r % 3;
                const float *xr = &xs[ci][((lz + dz) * T::HY + ly + dy) * T::HX + lx];
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const float v = xr[dx];
                    const float *wr = ws[ci * 27 + r * 3 + dx];
#pragma unroll
                    for (int co = 0; co < CO; ++co) acc[co] = fmaf(wr[co], v, acc[co]);
                }
            }
        }
    }
    const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
    if (gx >= W || gy >= H || gz >= D) return;
    const size_t off = gz * plane + (size_t)gy * W + gx;
#pragma unroll
    for (int co = 0; co < CO; ++co) {
        float r = acc[co];
        if (relu) r = fmaxf(r, 0.f);
        if (mask && !(ldv(mask, co * vol + off, ydt) > 0.f)) r = 0.f;
        stv(y, co * vol + off, ydt, r);
    }
}

// Per-tile partial weight and bias gradients: part[tile][j], j = (co, ci, tap)
// for j < CO*CI*27 and co for the CO entries after them.
template <int CI, int CO>
__global__ void __launch_bounds__(NT) conv_bwd_w_kernel(const void *__restrict__ x, int xdt,
                                                        const void *__restrict__ dy, int dydt,
                                                        int D, int H, int W, float *__restrict__ part)
{
    __shared__ float xs[CI][TI3];
    __shared__ float gs[CO][TT3];
    const int x0 = blockIdx.x * TT, y0 = blockIdx.y * TT, z0 = blockIdx.z * TT;
    load_tile<CI>(xs, x, xdt, D, H, W, x0, y0, z0);
    const size_t plane = (size_t)H * W, vol = plane * D;
    for (int i = threadIdx.x; i < CO * TT3; i += NT) {
        const int co = i / TT3, v = i - co * TT3;
        const int gz = z0 + v / (TT * TT), gy = y0 + (v / TT) % TT, gx = x0 + v % TT;
        float g = 0.f;
        if (gz < D && gy < H && gx < W) g = ldv(dy, co * vol + gz * plane + (size_t)gy * W + gx, dydt);
        gs[co][v] = g;
    }
    __syncthreads();
    constexpr int NW = CO * CI * 27, NJ = NW + CO;
    const size_t tile = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    float *dst = part + tile * NJ;
    for (int j = threadIdx.x; j < NJ; j += NT) {
        float s = 0.f;
        if (j < NW) {
            const int co = j / (CI * 27), r = j % (CI * 27), ci = r / 27, t = r % 27;
            const int dz = t / 9, dyy = (t / 3) % 3, dx = t % 3;
            for (int v = 0; v < TT3; ++v) {
                const int lz = v / (TT * TT), ly = (v / TT) % TT, lx = v % TT;
                s = fmaf(gs[co][v], xs[ci][((lz + dz) * TI + ly + dyy) * TI + lx + dx], s);
            }
        } else {
            const int co = j - NW;
            for (int v = 0; v < TT3; ++v) s += gs[co][v];
        }
        dst[j] = s;
    }
}

// ---------------------------------------------------------------------------
// BF16 16 -> 16 channel layers on the matrix cores (v_mfma_f32_16x16x32_bf16,
// FP32 accumulation).  The convolution is an implicit GEMM per 8^3 tile:
//   forward  Y[voxel][co] = sum_k X[voxel][k] W[k][co],  k = (tap, ci),
//            27 taps (+ one zero tap) x 16 channels = 14 steps of K = 32;
//   weights  dW_tap[co][ci] = sum_v dY[co][v] X[ci][v + tap], K = the tile's
//            512 voxels = 16 steps of 32 (4 rows of 8 along x) per tap.
// MFMA operand layout (16x16x32): lane l holds row (A) or column (B) l % 16
// and the 8 consecutive k values 8 (l / 16) .. 8 (l / 16) + 7; the 16x16
// result holds column l % 16 and rows 4 (l / 16) .. 4 (l / 16) + 3.
// Weights are rounded to BF16 (round to nearest even) like the activations.
// ---------------------------------------------------------------------------
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float floatx4;
typedef __attribute__((ext_vector_type(4))) unsigned u32x4;

constexpr int MF_THREADS = 256;   // 4 waves
constexpr int MF_KSTEPS = 14;     // 28 taps in pairs

__device__ __forceinline__ unsigned bf16_bits(float v)
{
    unsigned u = __float_as_uint(v);
    u += 0x7fffu + ((u >> 16) & 1u);     // round to nearest even
    return u >> 16;
}

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// Offset (voxels of the 10^3 halo tile) of tap t = 9 dz + 3 dy + dx.
__host__ __device__ constexpr int tap_off(int t) { return ((t / 9) * TI + (t / 3) % 3) * TI + t % 3; }

// Forward (and data backward) of a 16 -> 16 layer on BF16 activations.  A
// workgroup owns an 8^3 output tile; each wave 128 of its voxels (8 row
// blocks of 16), all 16 output channels.
constexpr int MF_XS_BYTES = TI3 * 16 * 2;                  // halo tile, channel-last BF16
constexpr int MF_BF_BYTES = MF_KSTEPS * 64 * 16;           // B fragments
constexpr int MF_OS_BYTES = TT3 * 16 * 4;                  // output tile, FP32 [co][voxel]
constexpr int MF_SMEM = MF_XS_BYTES + MF_BF_BYTES > MF_OS_BYTES ? MF_XS_BYTES + MF_BF_BYTES
                                                                : MF_OS_BYTES;

__global__ void __launch_bounds__(MF_THREADS)
conv16_mfma_kernel(const unsigned short *__restrict__ x, int D, int H, int W,
                   const float *__restrict__ wt, const float *__restrict__ bias,
                   void *__restrict__ y, int ydt, int relu, const void *__restrict__ mask)
{
    // halo tile, channel-last: [z][y][x][ci], 32 bytes per voxel, then the B
    // fragments of the 14 steps, one 16-byte entry per lane: [step][lane];
    // after the products, the output tile [co][voxel] in FP32 over both
    __shared__ __attribute__((aligned(16))) unsigned char smem[MF_SMEM];
    unsigned short *xs = reinterpret_cast<unsigned short *>(smem);
    u32x4 *bfrag = reinterpret_cast<u32x4 *>(smem + MF_XS_BYTES);
    float *os = reinterpret_cast<float *>(smem);
    const int x0 = blockIdx.x * TT, y0 = blockIdx.y * TT, z0 = blockIdx.z * TT;
    const size_t plane = (size_t)H * W, vol = plane * D;
    // Weights: entry (s, lane) holds in word e the BF16 pair of channels
    // ci0 + 2e, ci0 + 2e + 1 of column co = lane % 16, tap 2 s + (lane / 16 >> 1),
    // ci0 = ((lane / 16) & 1) 8.
    for (int i = threadIdx.x; i < MF_KSTEPS * 64; i += MF_THREADS) {
        const int ln = i & 63, st = i >> 6;
        const int co = ln & 15, g = ln >> 4;
        const int tap = 2 * st + (g >> 1);
        u32x4 f;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int ci = (g & 1) * 8 + 2 * e;
            const float lo = tap < 27 ? wt[(co * 16 + ci) * 27 + tap] : 0.f;
            const float hi = tap < 27 ? wt[(co * 16 + ci + 1) * 27 + tap] : 0.f;
            f[e] = bf16_bits(lo) | (bf16_bits(hi) << 16);
        }
        bfrag[st * 64 + ln] = f;
    }
    // Halo rows (z, y), x0 - 1 .. x0 + 8, of a group of 8 channels: a
    // thread reads the group's 8 rows (the middle 8 voxels in one 16-byte
    // load when the row lies inside the volume and is 16-byte aligned, the
    // two ends and edge rows element by element) and writes each of the 10
    // voxels' 8 channels as one 16-byte word.
    const bool vec_ok = x0 + TT <= W && (W % 8) == 0 && ((uintptr_t)x % 16) == 0;
    for (int r = threadIdx.x; r < 2 * TI * TI; r += MF_THREADS) {
        const int cg = r / (TI * TI), zy = r - cg * TI * TI;
        const int zz = zy / TI, yy = zy - zz * TI;
        const int gz = z0 - 1 + zz, gy = y0 - 1 + yy;
        u32x4 w[TI];
#pragma unroll
        for (int k = 0; k < TI; ++k) w[k] = u32x4{0u, 0u, 0u, 0u};
        if (gz >= 0 && gz < D && gy >= 0 && gy < H) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const unsigned short *row =
                    x + (size_t)(cg * 8 + c) * vol + gz * plane + (size_t)gy * W;
                unsigned v[TI];
#pragma unroll
                for (int k = 0; k < TI; ++k) v[k] = 0u;
                if (vec_ok) {
                    const u32x4 mid = *reinterpret_cast<const u32x4 *>(row + x0);
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        v[1 + 2 * k] = mid[k] & 0xffffu;
                        v[2 + 2 * k] = mid[k] >> 16;
                    }
                    if (x0 > 0) v[0] = row[x0 - 1];
                    if (x0 + TT < W) v[TI - 1] = row[x0 + TT];
                } else {
#pragma unroll
                    for (int k = 0; k < TI; ++k) {
                        const int gx = x0 - 1 + k;
                        if (gx >= 0 && gx < W) v[k] = row[gx];
                    }
                }
#pragma unroll
                for (int k = 0; k < TI; ++k) w[k][c >> 1] |= v[k] << (16 * (c & 1));
            }
        }
#pragma unroll
        for (int k = 0; k < TI; ++k)
            *reinterpret_cast<u32x4 *>(xs + (zy * TI + k) * 16 + cg * 8) = w[k];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, g = lane >> 4;
    __syncthreads();
    bf16x8 bw[MF_KSTEPS];
#pragma unroll
    for (int s = 0; s < MF_KSTEPS; ++s) bw[s] = as_bf16x8(bfrag[s * 64 + lane]);
    floatx4 acc[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        // A row: voxel v of the tile; k = tap 2 s + (g >> 1), channels (g & 1) 8 ..
        const int v = wave * 128 + m * 16 + col;
        const int lx = v & 7, ly = (v >> 3) & 7, lz = v >> 6;
        const unsigned short *base = xs + ((lz * TI + ly) * TI + lx) * 16 + (g & 1) * 8;
        acc[m] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < MF_KSTEPS; ++s) {
            const int t0 = 2 * s, t1 = 2 * s + 1;
            const int tap = (g >> 1) ? t1 : t0;
            u32x4 av = {0u, 0u, 0u, 0u};
            if (tap < 27) av = *reinterpret_cast<const u32x4 *>(base + ((g >> 1) ? tap_off(t1 < 27 ? t1 : 0) : tap_off(t0)) * 16);
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(av), bw[s], acc[m], 0, 0, 0);
        }
    }
    // results: column co = col, rows (voxels) m 16 + 4 g + r, through LDS
    // [co][voxel] to rows of 8 voxels along x per (co, z, y)
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 8; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) os[col * TT3 + wave * 128 + m * 16 + 4 * g + r] = acc[m][r];
    __syncthreads();
    const bool row_ok = x0 + TT <= W && (W % 8) == 0 && ((uintptr_t)y % 32) == 0 &&
                        (!mask || ((uintptr_t)mask % 32) == 0);
    for (int rr = threadIdx.x; rr < 16 * TT * TT; rr += MF_THREADS) {
        const int co = rr / (TT * TT), zy = rr - co * TT * TT;
        const int lz = zy / TT, ly = zy - lz * TT;
        const int gz = z0 + lz, gy = y0 + ly;
        if (gz >= D || gy >= H) continue;
        const float bcol = bias ? bias[co] : 0.f;
        const float *src = os + co * TT3 + zy * TT;
        float o[TT];
#pragma unroll
        for (int k = 0; k < TT; ++k) {
            o[k] = src[k] + bcol;
            if (relu) o[k] = fmaxf(o[k], 0.f);
        }
        const size_t off = (size_t)co * vol + gz * plane + (size_t)gy * W + x0;
        if (row_ok) {
            if (mask) {
                float mv[TT];
                if (ydt == 0) {
                    const floatx4 a = *reinterpret_cast<const floatx4 *>((const float *)mask + off);
                    const floatx4 b = *reinterpret_cast<const floatx4 *>((const float *)mask + off + 4);
#pragma unroll
                    for (int k = 0; k < 4; ++k) mv[k] = a[k], mv[4 + k] = b[k];
                } else {
                    const u32x4 a = *reinterpret_cast<const u32x4 *>((const unsigned short *)mask + off);
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        mv[2 * k] = __uint_as_float(a[k] << 16);
                        mv[2 * k + 1] = __uint_as_float(a[k] & 0xffff0000u);
                    }
                }
#pragma unroll
                for (int k = 0; k < TT; ++k)
                    if (!(mv[k] > 0.f)) o[k] = 0.f;
            }
            if (ydt == 0) {
                float *dst = (float *)y + off;
                *reinterpret_cast<floatx4 *>(dst) = floatx4{o[0], o[1], o[2], o[3]};
                *reinterpret_cast<floatx4 *>(dst + 4) = floatx4{o[4], o[5], o[6], o[7]};
            } else {
                u32x4 b;
#pragma unroll
                for (int k = 0; k < 4; ++k) b[k] = bf16_bits(o[2 * k]) | (bf16_bits(o[2 * k + 1]) << 16);
                *reinterpret_cast<u32x4 *>((unsigned short *)y + off) = b;
            }
        } else {
#pragma unroll
            for (int k = 0; k < TT; ++k) {
                if (x0 + k >= W) break;
                float v = o[k];
                if (mask && !(ldv(mask, off + k, ydt) > 0.f)) v = 0.f;
                stv(y, off + k, ydt, v);
            }
        }
    }
}

// Per-tile partial weight and bias gradients of a 16 -> 16 layer on BF16
// activations (same part[tile][j] layout as conv_bwd_w_kernel).  Wave w
// takes taps w, w + 4, ...; dy and three x copies shifted by dx = 0, 1, 2
// (so every 8-voxel row starts on 16 bytes) are staged in LDS.
__global__ void __launch_bounds__(MF_THREADS)
conv16_wgrad_mfma_kernel(const unsigned short *__restrict__ x, const unsigned short *__restrict__ dy,
                         int D, int H, int W, float *__restrict__ part)
{
    __shared__ __attribute__((aligned(16))) unsigned short xs3[3][16][TI * TI][TT];  // [dx][ci][z y][x]
    __shared__ __attribute__((aligned(16))) unsigned short gs[16][TT3];             // [co][v]
    __shared__ float bsum[16][16];
    const int x0 = blockIdx.x * TT, y0 = blockIdx.y * TT, z0 = blockIdx.z * TT;
    const size_t plane = (size_t)H * W, vol = plane * D;
    // Rows (ci, z, y) of the halo, x0 - 1 .. x0 + 8; copy dx holds
    // x0 - 1 + dx .. x0 + 6 + dx.  The middle 8 come in one 16-byte load when
    // the row lies inside the volume and is 16-byte aligned.
    const bool vec_ok = x0 + TT <= W && (W % 8) == 0 && ((uintptr_t)x % 16) == 0;
    for (int r = threadIdx.x; r < 16 * TI * TI; r += MF_THREADS) {
        const int ci = r / (TI * TI), zy = r - ci * TI * TI;
        const int gz = z0 - 1 + zy / TI, gy = y0 - 1 + zy % TI;
        unsigned short v[TI];
#pragma unroll
        for (int k = 0; k < TI; ++k) v[k] = 0;
        if (gz >= 0 && gz < D && gy >= 0 && gy < H) {
            const unsigned short *row = x + ci * vol + gz * plane + (size_t)gy * W;
            if (vec_ok) {
                const u32x4 mid = *reinterpret_cast<const u32x4 *>(row + x0);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    v[1 + 2 * k] = (unsigned short)(mid[k] & 0xffffu);
                    v[2 + 2 * k] = (unsigned short)(mid[k] >> 16);
                }
                if (x0 > 0) v[0] = row[x0 - 1];
                if (x0 + TT < W) v[TI - 1] = row[x0 + TT];
            } else {
#pragma unroll
                for (int k = 0; k < TI; ++k) {
                    const int gx = x0 - 1 + k;
                    if (gx >= 0 && gx < W) v[k] = row[gx];
                }
            }
        }
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            u32x4 pk;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                pk[k] = (unsigned)v[dx + 2 * k] | ((unsigned)v[dx + 2 * k + 1] << 16);
            *reinterpret_cast<u32x4 *>(&xs3[dx][ci][zy][0]) = pk;
        }
    }
    // dy rows (co, z, y) of the tile, 8 voxels along x: one 16-byte load and
    // one 16-byte LDS word when the row lies inside the volume and is aligned
    const bool dvec_ok = x0 + TT <= W && (W % 8) == 0 && ((uintptr_t)dy % 16) == 0;
    for (int r = threadIdx.x; r < 16 * TT * TT; r += MF_THREADS) {
        const int co = r / (TT * TT), zy = r - co * TT * TT;
        const int gz = z0 + zy / TT, gy = y0 + zy % TT;
        u32x4 pk = {0u, 0u, 0u, 0u};
        if (gz < D && gy < H) {
            const unsigned short *row = dy + co * vol + gz * plane + (size_t)gy * W;
            if (dvec_ok) {
                pk = *reinterpret_cast<const u32x4 *>(row + x0);
            } else {
#pragma unroll
                for (int k = 0; k < TT; ++k)
                    if (x0 + k < W) pk[k >> 1] |= (unsigned)row[x0 + k] << (16 * (k & 1));
            }
        }
        *reinterpret_cast<u32x4 *>(&gs[co][zy * TT]) = pk;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, g = lane >> 4;
    constexpr int NW = 16 * 16 * 27;
    const size_t tile = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    float *dst = part + tile * (NW + 16);
    for (int tap = wave; tap < 27; tap += 4) {
        const int dz = tap / 9, dyy = (tap / 3) % 3, dx = tap % 3;
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
            // k = voxels of row R = 4 kk + g (8 along x) of the tile
            const int R = 4 * kk + g, lz = R >> 3, ly = R & 7;
            // A: row co = col, dy[co][R 8 .. R 8 + 7]
            const u32x4 av = *reinterpret_cast<const u32x4 *>(&gs[col][R * TT]);
            // B: column ci = col, x[ci][lz + dz][ly + dy][dx .. dx + 7]
            const u32x4 bv =
                *reinterpret_cast<const u32x4 *>(&xs3[dx][col][(lz + dz) * TI + ly + dyy][0]);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(av), as_bf16x8(bv), acc, 0, 0, 0);
        }
        // rows co = 4 g + r, column ci = col
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[((4 * g + r) * 16 + col) * 27 + tap] = acc[r];
    }
    // bias: 16 partial sums of 32 voxels per channel, added in a fixed order
    {
        const int co = threadIdx.x >> 4, pp = threadIdx.x & 15;
        float sacc = 0.f;
        for (int v = pp * 32; v < pp * 32 + 32; ++v)
            sacc += __uint_as_float((unsigned)gs[co][v] << 16);
        bsum[co][pp] = sacc;
    }
    __syncthreads();
    if (threadIdx.x < 16) {
        float sb = 0.f;
        for (int pp = 0; pp < 16; ++pp) sb += bsum[threadIdx.x][pp];
        dst[NW + threadIdx.x] = sb;
    }
}

// Partials per tile are summed in two fixed-order stages (deterministic):
// groups of SUM_GROUP consecutive tiles, then the groups.
constexpr int SUM_GROUP = 64;

__global__ void sum_tile_groups_kernel(const float *__restrict__ part, int ntiles, int nj,
                                       float *__restrict__ gsum)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nj) return;
    const int t0 = blockIdx.y * SUM_GROUP, t1 = min(ntiles, t0 + SUM_GROUP);
    float s = 0.f;
    for (int t = t0; t < t1; ++t) s += part[(size_t)t * nj + j];
    gsum[(size_t)blockIdx.y * nj + j] = s;
}

__global__ void sum_tiles_kernel(const float *__restrict__ gsum, int ngroups, int nj, int nw,
                                 float *__restrict__ dw, float *__restrict__ db)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nj) return;
    float s = 0.f;
    for (int t = 0; t < ngroups; ++t) s += gsum[(size_t)t * nj + j];
    if (j < nw)
        dw[j] = s;
    else if (db)
        db[j - nw] = s;
}

__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

constexpr int MSE_BLOCKS = 1024;

__global__ void mse_kernel(const void *__restrict__ y, int ydt, const void *__restrict__ t, int tdt,
                           int64_t n, void *__restrict__ dy, double *__restrict__ part)
{
    __shared__ double ws[4];
    double s = 0.0;
    const float k = 2.f / (float)n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float d = ldv(y, i, ydt) - ldv(t, i, tdt);
        s += (double)d * (double)d;
        stv(dy, i, ydt, k * d);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

__global__ void mse_sum_kernel(const double *__restrict__ part, int64_t n, float *__restrict__ loss)
{
    __shared__ double ws[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < MSE_BLOCKS; i += blockDim.x) s += part[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) loss[0] = (float)(((ws[0] + ws[1]) + (ws[2] + ws[3])) / (double)n);
}

int cnn_fail(int code, const char *msg)
{
    oat::set_last_error(msg);
    return code;
}

int launched(const char *who)
{
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) return OAT_OK;
    oat::set_last_error((std::string(who) + ": " + hipGetErrorName(e)).c_str());
    return OAT_ERR_DEVICE;
}

bool ch_ok(int c) { return c == 1 || c == 16; }
bool dt_ok(int d) { return d == OAT_F32 || d == OAT_BF16; }

dim3 tiles(int d, int h, int w) { return dim3((w + TT - 1) / TT, (h + TT - 1) / TT, (d + TT - 1) / TT); }

template <int CI, int CO> dim3 fwd_tiles(int d, int h, int w)
{
    using T = FwdTile<CI, CO>;
    return dim3((w + T::FX - 1) / T::FX, (h + T::FY - 1) / T::FY, (d + T::FZ - 1) / T::FZ);
}

}  // namespace

extern "C" {

int oat_conv3d_forward(const void *x, oat_dtype xdt, int c_in, int d, int h, int w,
                       const float *weight, const float *bias, int c_out, void *y, oat_dtype ydt,
                       int relu, const void *mask, void *stream)
{
    if (!x || !weight || !y) return cnn_fail(OAT_ERR_ARG, "oat_conv3d_forward: null pointer");
    if (!ch_ok(c_in) || !ch_ok(c_out)) return cnn_fail(OAT_ERR_ARG, "channels must be 1 or 16");
    if (d < 1 || h < 1 || w < 1) return cnn_fail(OAT_ERR_ARG, "volume sizes must be >= 1");
    if (!dt_ok(xdt) || !dt_ok(ydt)) return cnn_fail(OAT_ERR_DTYPE, "unknown dtype");
    if (x == y) return cnn_fail(OAT_ERR_ARG, "input and output alias");
    hipStream_t s = (hipStream_t)stream;
    dim3 g = tiles(d, h, w), b(NT);
#define FWD(CI, CO)                                                                                 \
    hipLaunchKernelGGL((conv_fwd_kernel<CI, CO>), (fwd_tiles<CI, CO>(d, h, w)), b, 0, s, x, (int)xdt, \
                       d, h, w, weight, bias, y, (int)ydt, relu, mask)
    if (c_in == 16 && c_out == 16 && xdt == OAT_BF16)
        hipLaunchKernelGGL(conv16_mfma_kernel, g, dim3(MF_THREADS), 0, s,
                           (const unsigned short *)x, d, h, w, weight, bias, y, (int)ydt, relu,
                           mask);
    else if (c_in == 1 && c_out == 16) FWD(1, 16);
    else if (c_in == 16 && c_out == 16) FWD(16, 16);
    else if (c_in == 16 && c_out == 1) FWD(16, 1);
    else FWD(1, 1);
#undef FWD
    return launched("oat_conv3d_forward");
}

size_t oat_conv3d_backward_weight_workspace(int c_in, int c_out, int d, int h, int w)
{
    if (!ch_ok(c_in) || !ch_ok(c_out) || d < 1 || h < 1 || w < 1) return 0;
    dim3 g = tiles(d, h, w);
    const size_t nt = (size_t)g.x * g.y * g.z, ng = (nt + SUM_GROUP - 1) / SUM_GROUP;
    return sizeof(float) * (nt + ng) * (size_t)(c_out * c_in * 27 + c_out);
}

int oat_conv3d_backward_weight(const void *x, oat_dtype xdt, const void *dy, oat_dtype dydt,
                               int c_in, int c_out, int d, int h, int w, float *dweight,
                               float *dbias, void *workspace, size_t workspace_bytes, void *stream)
{
    if (!x || !dy || !dweight || !workspace)
        return cnn_fail(OAT_ERR_ARG, "oat_conv3d_backward_weight: null pointer");
    if (!ch_ok(c_in) || !ch_ok(c_out)) return cnn_fail(OAT_ERR_ARG, "channels must be 1 or 16");
    if (d < 1 || h < 1 || w < 1) return cnn_fail(OAT_ERR_ARG, "volume sizes must be >= 1");
    if (!dt_ok(xdt) || !dt_ok(dydt)) return cnn_fail(OAT_ERR_DTYPE, "unknown dtype");
    if (workspace_bytes < oat_conv3d_backward_weight_workspace(c_in, c_out, d, h, w))
        return cnn_fail(OAT_ERR_ARG, "oat_conv3d_backward_weight: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    dim3 g = tiles(d, h, w), b(NT);
    float *part = (float *)workspace;
#define BWD(CI, CO)                                                                                \
    hipLaunchKernelGGL((conv_bwd_w_kernel<CI, CO>), g, b, 0, s, x, (int)xdt, dy, (int)dydt, d, h, w, \
                       part)
    if (c_in == 16 && c_out == 16 && xdt == OAT_BF16 && dydt == OAT_BF16)
        hipLaunchKernelGGL(conv16_wgrad_mfma_kernel, g, dim3(MF_THREADS), 0, s,
                           (const unsigned short *)x, (const unsigned short *)dy, d, h, w, part);
    else if (c_in == 1 && c_out == 16) BWD(1, 16);
    else if (c_in == 16 && c_out == 16) BWD(16, 16);
    else if (c_in == 16 && c_out == 1) BWD(16, 1);
    else BWD(1, 1);
#undef BWD
    int rc = launched("oat_conv3d_backward_weight");
    if (rc) return rc;
    const int nw = c_out * c_in * 27, nj = nw + c_out, ntiles = (int)(g.x * g.y * g.z);
    const int ngroups = (ntiles + SUM_GROUP - 1) / SUM_GROUP;
    float *gsum = part + (size_t)ntiles * nj;
    hipLaunchKernelGGL(sum_tile_groups_kernel, dim3((nj + 255) / 256, ngroups), dim3(256), 0, s,
                       part, ntiles, nj, gsum);
    rc = launched("oat_conv3d_backward_weight");
    if (rc) return rc;
    hipLaunchKernelGGL(sum_tiles_kernel, dim3((nj + 255) / 256), dim3(256), 0, s, gsum, ngroups, nj,
                       nw, dweight, dbias);
    return launched("oat_conv3d_backward_weight");
}

int oat_adam_step(float *param, const float *grad, float *m, float *v, int64_t n, float lr,
                  float beta1, float beta2, float eps, int step, void *stream)
{
    if (!param || !grad || !m || !v || n < 0 || step < 1)
        return cnn_fail(OAT_ERR_ARG, "oat_adam_step: bad argument");
    if (n == 0) return OAT_OK;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, step)));
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, param, grad, m,
                       v, n, lr, beta1, beta2, eps, c1, c2);
    return launched("oat_adam_step");
}

size_t oat_mse_workspace(void) { return sizeof(double) * MSE_BLOCKS; }

int oat_mse(const void *y, oat_dtype ydt, const void *target, oat_dtype tdt, int64_t n, float *loss,
            void *dy, void *workspace, void *stream)
{
    if (!y || !target || !loss || !dy || !workspace || n < 1)
        return cnn_fail(OAT_ERR_ARG, "oat_mse: bad argument");
    if (!dt_ok(ydt) || !dt_ok(tdt)) return cnn_fail(OAT_ERR_DTYPE, "unknown dtype");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(mse_kernel, dim3(MSE_BLOCKS), dim3(256), 0, s, y, (int)ydt, target, (int)tdt, n,
                       dy, (double *)workspace);
    int rc = launched("oat_mse");
    if (rc) return rc;
    hipLaunchKernelGGL(mse_sum_kernel, dim3(1), dim3(256), 0, s, (const double *)workspace, n, loss);
    return launched("oat_mse");
}

}  // extern "C"
