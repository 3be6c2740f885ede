// Brick-driven spherical Radon transform G and its exact adjoint G^T on
// gfx950 (CDNA4, wave64).
//
// G  (Eq. (dis_srt)): g[q,k] = sum_{i,j} w_{k,i} Psi(alpha; x_{q,k,i,j})
// G^T (adjoint, Sec. II.B.3): alpha'_n = sum_{q,k,i,j} w_{k,i} g'[q,k] psi_n(x_{q,k,i,j})
//
// The image is cut into bricks of BRICK^3 cells.  A workgroup owns one brick
// and keeps its (BRICK+2)^3 nodes in LDS: the image values for G, a 64-bit
// fixed-point accumulator for G^T.  Each wave takes one transducer at a time and
// enumerates exactly the quadrature points whose trilinear cell lies in the
// brick, in three wave-wide expansions:
//   shells k -> candidate rings (k, i) -> ring segments -> points.
// Every point's position is a deterministic function of (q, k, i, j) and
// the same code evaluates it in both kernels, so each point belongs to
// exactly one brick of G and the adjoint uses the identical point set.
#include <type_traits>

#include "oat_internal.hpp"
#include "oat_geom.hpp"

#pragma clang fp contract(off)

namespace oat {

namespace {

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int bperm_i(int src, int v)
{
    return __builtin_amdgcn_ds_bpermute(src << 2, v);
}

__device__ __forceinline__ float bperm_f(int src, float v)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

__device__ __forceinline__ double bperm_d(int src, double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xF, false);
}

// Exclusive prefix sum over the wave of non-negative values below 2^BITS,
// and the total; all 64 lanes must be active (every caller runs in
// wave-uniform control flow of full waves).  Inclusive sums within each row
// of 16 lanes by row shifts of 1, 2, 4 and 8 (a lane whose source lies
// outside the row adds 0), then the row totals carried across rows by the
// two row broadcasts.
template <int BITS>
__device__ __forceinline__ int excl_scan_wave(int v, int &total)
{
    static_assert(BITS <= 24, "the wave total must fit an int");
    int s = v;
    s += dpp_i<0x111, 0xF>(s);   // row_shr:1
    s += dpp_i<0x112, 0xF>(s);   // row_shr:2
    s += dpp_i<0x114, 0xF>(s);   // row_shr:4
    s += dpp_i<0x118, 0xF>(s);   // row_shr:8
    s += dpp_i<0x142, 0xA>(s);   // row_bcast:15 into rows 1 and 3
    s += dpp_i<0x143, 0xC>(s);   // row_bcast:31 into rows 2 and 3
    total = __builtin_amdgcn_readlane(s, 63);
    return s - v;
}

// Sum over the 64 lanes with DPP row operations (no LDS traffic); the result
// is returned to every lane through lane 63.
__device__ __forceinline__ float wave_sum_dpp(float v)
{
    v += dpp_f<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
    v += dpp_f<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
    v += dpp_f<0x141, 0xF>(v);   // row_half_mirror
    v += dpp_f<0x140, 0xF>(v);   // row_mirror: every lane holds its row sum
    v += dpp_f<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_f<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ uint64_t mask_below() { return (1ull << lane_id()) - 1ull; }

// floor(x) as an integer in one instruction (the compiler emits floor + convert).
__device__ __forceinline__ int cvt_floor(float x)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// One quadrature point as handed to the gather/scatter: owned by the brick,
// cell relative to the box, fractional position in the cell.
struct Pt {
    bool own;
    int cx, cy, cz;
    float fx, fy, fz;
};

// One level of wave-wide expansion: producer lanes hold counts, consumers
// walk the concatenation 64 items at a time.  Head bits mark where each
// producer's run starts; a ballot plus popcount turns them into a rank, and a
// rank -> (lane, offset) table gives the producer and the local index.
struct Level {
    unsigned *bits;
    int *prod;
    int total, base;
};

template <int BITS>
__device__ __forceinline__ void level_begin(Level &L, int cnt)
{
    int total;
    int excl = excl_scan_wave<BITS>(cnt, total);
    L.total = total;
    L.base = 0;
    int nw = (total + 31) >> 5;
    for (int w = lane_id(); w < nw; w += WAVE) L.bits[w] = 0u;
    uint64_t nz = __ballot(cnt > 0);
    int rank = __popcll(nz & mask_below());
    wave_sync();
    if (cnt > 0) {
        atomicOr(&L.bits[excl >> 5], 1u << (excl & 31));
        L.prod[rank] = lane_id() | (excl << 8);
    }
    wave_sync();
}

// Consumer side of a window starting at F (uniform control flow).
__device__ __forceinline__ bool level_item(Level &L, int F, int &src, int &local)
{
    int idx = F + lane_id();
    bool valid = idx < L.total;
    unsigned word = L.bits[(valid ? idx : 0) >> 5];
    bool head = valid && ((word >> (idx & 31)) & 1u);
    uint64_t hm = __ballot(head);
    int rank = L.base + __popcll(hm & (mask_below() | (1ull << lane_id()))) - 1;
    L.base += __popcll(hm);
    rank = min(max(rank, 0), WAVE - 1);
    int pe = L.prod[rank];
    src = valid ? (pe & 63) : 0;
    local = idx - (pe >> 8);
    return valid;
}

constexpr int CAP1 = 64;   // candidate rings per shell per pass (64 * 64 bits)
constexpr int CAP2 = 16;   // segments per ring per pass (64 * 16 bits)

// Per-wave LDS scratch of the point level: per-segment data handed to the
// points, and the level-3 head bitmap and producer table.
struct SegLds {
    float4 stage[64][3];
    unsigned bits3[64];
    int prod3[64];
};

// Per-wave LDS scratch of the full walk (shell and ring levels too).
struct WaveLds : SegLds {
    unsigned bits1[128];
    unsigned bits2[32];
    int prod1[64];
    int prod2[64];
};

// Cell box of brick b: cells lo .. hi-1 per axis.  The bricks partition the
// cells [-1, n) that can hold a quadrature point with a nonzero trilinear
// weight: brick i owns cells 20i-1 .. 20i+18, the last one up to n-1.  n0 ..
// n1-1 are the nodes the brick owns.
__device__ __forceinline__ void brick_box(const Problem &P, int b, int lo[3], int hi[3],
                                          int n0[3], int n1[3])
{
    int bx = b % P.nbx, by = (b / P.nbx) % P.nby, bz = b / (P.nbx * P.nby);
    const int bi[3] = {bx, by, bz};
    const int nb[3] = {P.nbx, P.nby, P.nbz};
    const int n[3] = {P.nx, P.ny, P.nz};
    for (int a = 0; a < 3; ++a) {
        n0[a] = bi[a] * BRICK;
        n1[a] = min(n0[a] + BRICK, n[a]);
        lo[a] = n0[a] - 1;
        hi[a] = (bi[a] == nb[a] - 1) ? n[a] : n1[a] - 1;
    }
}

// What walk_unit does with the points it enumerates.
enum WalkMode {
    WALK_POINTS = 0,    // call fn on every window of points (G, G^T)
    WALK_COUNT = 1,     // arc table, first pass: runs of rings with owned points
    WALK_FILL = 2,      // arc table, second pass: tight arc of every ring in a run
    WALK_SEGCOUNT = 3,  // segment table, first pass: segments per unit
    WALK_SEGFILL = 4    // segment table, second pass: the unit's segment entries
};

// Where the rings and arcs of a unit come from.
enum TableMode {
    TM_BOUNDS = 0,  // ball/slab bounds of the brick, computed per unit
    TM_ARC = 1,     // plan's arc table: tight arcs of the rings with owned points
    TM_SEG = 2      // plan's segment table: the unit's segments, in walk order
};

// Per-wave LDS of the arc-table passes: owned-index span (in arc order) per
// ring of the current level-1 window, owned-ring span per shell of the chunk.
struct BuildLds {
    int rmin[64], rmax[64];
    int smin[64], smax[64];
    int hist[32];    // segment passes: the unit's segments per point count
};

// Reference point of a ring segment.  cs = (cos, sin) in FP64 of the
// segment's reference azimuth (Problem::segref).  The point, formed in FP64,
// is split into an integer cell relative to the box (clamped; clamped
// offsets only occur for points far outside the box) and an FP32 fraction
// Pl; (xa, xb) = rs (cos, sin) are its in-plane coordinates.
__device__ __forceinline__ void seg_ref(const double uq[3], const double e3[3],
                                        const double e1d[3], const double e2d[3],
                                        const int lo[3], double rc, double rs, double2 cs,
                                        float Pl[3], int dc[3], float &xa, float &xb)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double pa = fma(rc, e3[a], uq[a]) + rs * fma(cs.x, e1d[a], cs.y * e2d[a]);
        const double ph = floor(pa);
        Pl[a] = (float)(pa - ph);
        dc[a] = min(max((int)ph - lo[a], -512), 511);
    }
    xa = (float)(rs * cs.x);
    xb = (float)(rs * cs.y);
}

// Point j of a segment, dj = j - jref, relative to the segment's reference
// point: ref + (cos d - 1) A + sin d B (seg_axes), d = dj 2 pi / nj
// (dd = 2 pi / nj).  The fraction stays within a few tens of cells, so
// positions carry a few 1e-6 cell of FP32 error, and every brick evaluates
// the same FP32 operations, so each point belongs to exactly one brick.
// own: its cell lies in the brick.
// In-plane axes of a segment: point j sits at ref + (cos d - 1) A + sin d B
// with A = xa e1 + xb e2 and B = xa e2 - xb e1.
struct SegAxes {
    float A[3], B[3];
};
__device__ __forceinline__ SegAxes seg_axes(float xa, float xb, const float e1[3],
                                            const float e2[3])
{
    SegAxes s;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s.A[a] = fmaf(xb, e2[a], xa * e1[a]);
        s.B[a] = fmaf(-xb, e1[a], xa * e2[a]);
    }
    return s;
}

__device__ __forceinline__ Pt seg_point(const float Pl[3], const int dc[3], const SegAxes &ax,
                                        float dd, float dj, const int lo[3], const int hi[3])
{
    float cm1, sn;
    small_rot(dj * dd, cm1, sn);
    const float ux = fmaf(sn, ax.B[0], fmaf(cm1, ax.A[0], Pl[0]));
    const float uy = fmaf(sn, ax.B[1], fmaf(cm1, ax.A[1], Pl[1]));
    const float uz = fmaf(sn, ax.B[2], fmaf(cm1, ax.A[2], Pl[2]));
    Pt t;
    t.cx = cvt_floor(ux) + dc[0];
    t.cy = cvt_floor(uy) + dc[1];
    t.cz = cvt_floor(uz) + dc[2];
    t.fx = __builtin_amdgcn_fractf(ux);
    t.fy = __builtin_amdgcn_fractf(uy);
    t.fz = __builtin_amdgcn_fractf(uz);
    t.own = (unsigned)t.cx < (unsigned)(hi[0] - lo[0]) &&
            (unsigned)t.cy < (unsigned)(hi[1] - lo[1]) &&
            (unsigned)t.cz < (unsigned)(hi[2] - lo[2]);
    return t;
}

// One window of up to 64 segments, one per lane (v2 = the lane holds one):
// ring (rc, rs, reference table offset sref, delta, nj, segment shift ls),
// shell k2, its weight w2 (w g' 2^s in G^T), points jb .. jb+npts-1 of
// segment jb >> ls.  Stages the segments' data and walks their points two
// per lane (level 3).  ub and rl are the arc-table passes' offset of jb in
// the ring's arc and the ring's level-1 lane.  The segment-table passes
// (unit, rrel = ring index relative to the shell's first candidate ring,
// scount = the unit's segments so far) record each segment's owned index
// range and count or write its compact entry.
template <int MODE, class Fn>
__device__ __forceinline__ void segment_points(const Problem &P, SegLds &W, BuildLds *B,
                                               const int lo[3], const int hi[3],
                                               const double uq[3], const double e3[3],
                                               const double e1d[3], const double e2d[3],
                                               const float e1[3], const float e2[3], bool v2,
                                               double rc2, double rs2, int sref2, float w2,
                                               float dl2, int nj2, int ls2, int k2, int jb,
                                               int npts, int ub, int rl, int klo, size_t unit,
                                               int rrel, long long &scount, Fn &&fn)
{
    constexpr bool SEGB = MODE == WALK_SEGCOUNT || MODE == WALK_SEGFILL;
    const int lane = lane_id();
    Level L3{W.bits3, W.prod3, 0, 0};
    const int sg = jb >> ls2;
    const int jref = seg_ref_index(sg, ls2, nj2);
    float Pl[3], xa, xb;
    int dc[3];
    seg_ref(uq, e3, e1d, e2d, lo, rc2, rs2, v2 ? P.segref[sref2 + sg] : make_double2(1.0, 0.0),
            Pl, dc, xa, xb);
    const int np = v2 ? npts : 0;
    // jb - jref in [-16, 16], npts <= 32, shell index < 4096 (n_t <= 4096)
    const int meta = (jb - jref + 64) | (np << 7) | (k2 << 13);
    // The segment-table passes key their owned ranges by the segment's lane.
    const int tag = SEGB ? (lane | (jb << 8)) : (rl | (ub << 8));
    // The segment's data goes to the wave's LDS stage, where the lanes of its
    // points read it (a broadcast read; cheaper than one bpermute per value
    // on this part).  The cell offsets are stored unpacked: the point level
    // reads them with the same three 16-byte reads.
    wave_sync();
    W.stage[lane][0] = make_float4(Pl[0], Pl[1], Pl[2], __int_as_float(meta));
    W.stage[lane][1] = make_float4(xa, xb, dl2, w2);
    W.stage[lane][2] = make_float4(__int_as_float(dc[0]), __int_as_float(dc[1]),
                                   __int_as_float(dc[2]), __int_as_float(tag));
    if (SEGB) {
        B->rmin[lane] = 0x7fffffff;
        B->rmax[lane] = -1;
    }
    // Level 3: each lane takes two consecutive points of a segment
    // (level_begin orders the stage writes before the reads).
    level_begin<5>(L3, (np + 1) >> 1);
    for (int F3 = 0; F3 < L3.total; F3 += WAVE) {
        int s3, pr;
        const bool v3 = level_item(L3, F3, s3, pr);
        const float4 r0 = W.stage[s3][0], r1 = W.stage[s3][1], r2 = W.stage[s3][2];
        const float p3[3] = {r0.x, r0.y, r0.z};
        const int mt = __float_as_int(r0.w);
        const float qa = r1.x, qb = r1.y, dd = r1.z, wv = r1.w;
        const int d3[3] = {__float_as_int(r2.x), __float_as_int(r2.y), __float_as_int(r2.z)};
        int rlp = 0, ur = 0;
        if (MODE != WALK_POINTS) {
            const int ru = __float_as_int(r2.w);
            rlp = ru & 255;
            ur = (ru >> 8) + 2 * pr;
        }
        const int npp = (mt >> 7) & 63, kk = mt >> 13;
        const int djA = (mt & 127) - 64 + 2 * pr;
        Pt pt[2];
        const SegAxes ax = seg_axes(qa, qb, e1, e2);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            pt[h] = seg_point(p3, d3, ax, dd, (float)(djA + h), lo, hi);
            pt[h].own = pt[h].own && v3 && 2 * pr + h < npp;
        }
        if (MODE == WALK_POINTS) {
            fn(pt[0], pt[1], wv, kk, klo);
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h)
                if (pt[h].own) {
                    atomicMin(&B->rmin[rlp], ur + h);
                    atomicMax(&B->rmax[rlp], ur + h);
                }
        }
    }
    if constexpr (SEGB) {
        // The segment's owned points span jmin .. jmax (a superset of them
        // when the brick cuts the segment twice; the kernels test each).
        wave_sync();
        const int jmin = B->rmin[lane], jmax = B->rmax[lane];
        const bool has = v2 && jmax >= 0;
        const int koff = k2 - klo, cnt = jmax - jmin + 1;
        const int off = jmin - (sg << ls2);
        if (has && (rrel < 0 || rrel >= (1 << SEG_RING_BITS) || koff < 0 ||
                    koff >= (1 << SEG_SHELL_BITS) || sg >= (1 << SEG_INDEX_BITS) || off < 0 ||
                    cnt > 32))
            atomicOr(P.seg_flag, 1);
        const uint64_t bal = __ballot(has);
        if (MODE == WALK_SEGCOUNT) {
            if (has) atomicAdd(&B->hist[cnt - 1], 1);
        } else {
            // Entries of equal count keep walk order: per count present in
            // this window, the lanes holding it take consecutive places
            // after the count's earlier entries (B->hist holds each count's
            // next place, counts in decreasing order).
            uint64_t pend = bal;
            while (pend) {
                const int first = __ffsll((long long)pend) - 1;
                const int c = __shfl(cnt, first);
                const uint64_t m = __ballot(has && cnt == c);
                const int base = B->hist[c - 1];
                if (has && cnt == c) {
                    const long long pos = P.seg_off[unit] + base + __popcll(m & mask_below());
                    // the count pass saw the same segments; the guard only
                    // keeps a mismatch inside the unit's range
                    if (pos < P.seg_off[unit + 1])
                        P.seg[pos] = seg_pack(koff, rrel, sg, off, cnt);
                }
                wave_sync();
                if (lane == first) B->hist[c - 1] = base + __popcll(m);
                wave_sync();
                pend &= ~m;
            }
        }
        scount += __popcll(bal);
        wave_sync();
    }
}

// Shells klo .. khi of the transducer at uq (grid units) that can reach the
// cell box [lo, hi) (at most the plan's window of them; klo > khi: none).
__device__ __forceinline__ void unit_shells(const Problem &P, const double uq[3], const int lo[3],
                                            const int hi[3], int &klo, int &khi)
{
    float dmin2 = 0.f, dmax2 = 0.f;
    for (int a = 0; a < 3; ++a) {
        float u = (float)uq[a];
        float dl = (float)lo[a] - u, dh = u - (float)hi[a];
        float dm = fmaxf(fmaxf(dl, dh), 0.f);
        dmin2 += dm * dm;
        float e = fmaxf(fabsf(u - (float)lo[a]), fabsf(u - (float)hi[a]));
        dmax2 += e * e;
    }
    float dmin = sqrtf(dmin2) - 0.1f, dmax = sqrtf(dmax2) + 0.1f;
    klo = max(0, (int)ceilf((dmin - P.rho0) / P.rho_step));
    khi = min(P.nt - 1, (int)floorf((dmax - P.rho0) / P.rho_step));
    khi = min(khi, klo + P.window - 1);
}

// Candidate rings i0 .. i0+cnt-1 of shell sh that can reach the ball that
// holds the box (D = distance of its centre from the transducer, thb = the
// centre's polar angle in the transducer frame, h2 = squared radius); a
// superset of the rings with points in the box.  cnt = 0: none.
__device__ __forceinline__ void shell_rings(const ShellRec &sh, float D, float thb, float h2,
                                            int &i0, int &cnt)
{
    i0 = 0;
    cnt = 0;
    if (sh.n_rings <= 0) return;
    const float rho = sh.rho;
    const float om = (h2 - (rho - D) * (rho - D)) * rcp_approx(2.f * rho * D);   // 1 - cos(delta)
    if (!(om > 0.f)) return;
    const float delta = om >= 2.f ? kPi : acos_approx(1.f - om);
    const float tlo = (thb - delta) * rho - 0.5f;
    const float thi = (thb + delta) * rho - 0.5f;
    const int a = max(0, (int)floorf(tlo) - 2);
    const int b = min(sh.n_rings - 1, (int)ceilf(thi) + 2);
    if (b >= a) {
        i0 = a;
        cnt = b - a + 1;
    }
}

// Walk all points of transducer q owned by the brick (unit = brick * nq + q).
// The rings and arcs come from the ball/slab bounds (TM_BOUNDS) or the
// plan's arc table (TM_ARC: tight arcs of exactly the rings that hold owned
// points); both give the same owned points (and so does walk_seg, the
// segment-table walk).  In WALK_POINTS mode fn is called per window of 64
// lanes with the lane's two consecutive points of one segment (Pt each),
// their weight, their shell index and the unit's first shell.  The
// segment-table passes (bounds walk) count or write the unit's segments.
template <bool ADJ, int TM, int MODE, class WL, class Fn>
__device__ __forceinline__ void walk_unit(const Problem &P, int q, size_t unit, const int lo[3],
                                          const int hi[3], WL &W, BuildLds *B,
                                          const float *gp, float gscale, float gscale2,
                                          int &klo_out, Fn &&fn)
{
    static_assert(TM != TM_SEG, "the segment table is walked by walk_seg");
    constexpr bool TAB = TM == TM_ARC;
    constexpr bool READ_RUNS = TAB || MODE == WALK_FILL;
    constexpr bool SEGB = MODE == WALK_SEGCOUNT || MODE == WALK_SEGFILL;
    const DetRec &d = P.det[q];
    const double uq[3] = {d.uq[0], d.uq[1], d.uq[2]};
    const double e3[3] = {d.e3[0], d.e3[1], d.e3[2]};
    const double e1d[3] = {d.e1d[0], d.e1d[1], d.e1d[2]};
    const double e2d[3] = {d.e2d[0], d.e2d[1], d.e2d[2]};
    const float e1[3] = {d.e1[0], d.e1[1], d.e1[2]};
    const float e2[3] = {d.e2[0], d.e2[1], d.e2[2]};

    int klo, khi;
    unit_shells(P, uq, lo, hi, klo, khi);
    klo_out = klo;
    const int lane = lane_id();

    if (SEGB) {
        // Per point count: the count pass tallies the unit's segments; the
        // fill pass starts each count's entries after those of all larger
        // counts.
        int h = 0;
        if (MODE == WALK_SEGFILL && lane < 32) h = P.seg_hist[unit * 32 + (31 - lane)];
        int tot;
        const int before = excl_scan_wave<24>(lane < 32 ? h : 0, tot);
        if (lane < 32) B->hist[31 - lane] = MODE == WALK_SEGFILL ? before : 0;
        wave_sync();
    }
    ArcUnit U;
    if (!TAB) arc_unit_setup(U, lo, hi, uq, e1, e2, e3, 0.02f);
    const float D = TAB ? 0.f : sqrtf(U.rhov2 + U.V3 * U.V3);
    const float thb = TAB ? 0.f : acos_approx(U.V3 * rcp_approx(D));
    const float h2 = U.h2;

    Level L1{W.bits1, W.prod1, 0, 0};
    Level L2{W.bits2, W.prod2, 0, 0};

    const long long ebase = READ_RUNS ? P.tab_off[unit] : 0ll;
    int run_base = 0;     // table entries of the earlier shell chunks
    int ucount = 0;       // WALK_COUNT: table entries of the unit (per shell lane)
    long long scount = 0; // segment passes: segments of the unit so far

    for (int kc = klo; kc <= khi; kc += WAVE) {
        // Level 1 producers: one shell per lane -> candidate ring range.
        int k = kc + lane;
        int cnt_all = 0, ilo_all = 0, rbase = 0;
        int r_i0 = 0, r_n = 0, r_ex = 0;   // run of table rings of this shell
        if (READ_RUNS) {
            if (k <= khi) {
                const unsigned run = P.tab_run[unit * P.window + (k - klo)];
                r_i0 = (int)(run & 0xffffu);
                r_n = (int)(run >> 16);
            }
            int tot;
            r_ex = excl_scan_wave<16>(r_n, tot) + run_base;
            run_base += tot;
        }
        if (TAB) {
            if (r_n > 0) {
                cnt_all = r_n;
                ilo_all = r_i0;
                rbase = P.shell[k].ring_base;
            }
        } else if (k <= khi) {
            const ShellRec sh = P.shell[k];
            shell_rings(sh, D, thb, h2, ilo_all, cnt_all);
            rbase = sh.ring_base;
        }
        if (MODE == WALK_COUNT) {
            B->smin[lane] = 0x7fffffff;
            B->smax[lane] = -1;
            wave_sync();
        }
        // Candidate rings are taken CAP1 per shell per pass so the head
        // bitmap never exceeds 64 * CAP1 bits.
        for (int pass1 = 0; __ballot(cnt_all - pass1 * CAP1 > 0) != 0ull; ++pass1) {
        const int cnt1 = min(max(cnt_all - pass1 * CAP1, 0), CAP1);
        const int ilo = ilo_all + pass1 * CAP1;
        level_begin<7>(L1, cnt1);
        for (int F1 = 0; F1 < L1.total; F1 += WAVE) {
            int s1, loc1;
            bool v1 = level_item(L1, F1, s1, loc1);
            int kr = bperm_i(s1, k);
            int ir = bperm_i(s1, ilo) + loc1;
            int rb = bperm_i(s1, rbase);
            // segment passes: ring index relative to the shell's first candidate
            const int rrel1 = SEGB ? ir - bperm_i(s1, ilo_all) : 0;
            const int run_i0 = READ_RUNS ? bperm_i(s1, r_i0) : 0;
            const int run_n = READ_RUNS ? bperm_i(s1, r_n) : 0;
            const int run_ex = READ_RUNS ? bperm_i(s1, r_ex) : 0;
            // Ring (kr, ir): arc of indices that holds every owned point.
            double rcd = 0.0, rsd = 0.0;
            float w = 0.f, dlt = 0.f;
            int nj = 1, jlo = 0, jcnt = 0, ls = 0, n1 = 0, items_all = 0, srf = 0;
            if (v1) {
                const RingRec rr = P.ring[rb + ir];
                rcd = rr.rc;
                rsd = rr.rs;
                srf = rr.sref;
                nj = rr.nj;
                w = rr.w;
                dlt = rr.delta;
                if (TAB) {
                    const unsigned e = P.tab_arc[ebase + run_ex + (ir - run_i0)];
                    jlo = (int)(e & 0xffffu);
                    jcnt = (int)(e >> 16);
                } else {
                    const float C[3] = {(float)fma(rr.rc, e3[0], uq[0]),
                                        (float)fma(rr.rc, e3[1], uq[1]),
                                        (float)fma(rr.rc, e3[2], uq[2])};
                    ring_arc(U, C, rr.rsf, (float)rr.rc, nj, jlo, jcnt);
                }
                ls = rr.lshift;
                if (jcnt > 0) {
                    int jend = jlo + jcnt;
                    if (jend <= nj) {
                        n1 = ((jend - 1) >> ls) - (jlo >> ls) + 1;
                        items_all = n1;
                    } else {
                        n1 = ((nj - 1) >> ls) - (jlo >> ls) + 1;
                        items_all = n1 + ((jend - nj - 1) >> ls) + 1;
                    }
                }
            }
            if (ADJ && v1 && items_all > 0)
                w = w * ((gp[(size_t)q * P.nt + kr] * gscale) * gscale2);
            if (MODE == WALK_COUNT || MODE == WALK_FILL) {
                B->rmin[lane] = 0x7fffffff;
                B->rmax[lane] = -1;
                wave_sync();
            }
            for (int pass2 = 0; __ballot(items_all - pass2 * CAP2 > 0) != 0ull; ++pass2) {
            const int nitems = min(max(items_all - pass2 * CAP2, 0), CAP2);
            level_begin<5>(L2, nitems);
            for (int F2 = 0; F2 < L2.total; F2 += WAVE) {
                int s2, m;
                bool v2 = level_item(L2, F2, s2, m);
                m += pass2 * CAP2;
                const int nj2 = bperm_i(s2, nj), jlo2 = bperm_i(s2, jlo), jc2 = bperm_i(s2, jcnt);
                const int ls2 = bperm_i(s2, ls), n12 = bperm_i(s2, n1), k2 = bperm_i(s2, kr);
                // Segment of this item and its index range.
                const bool wrap = m >= n12;
                const int s = wrap ? m - n12 : (jlo2 >> ls2) + m;
                const int sb = s << ls2, se = min(sb + (1 << ls2), nj2);
                const int jb = wrap ? sb : max(sb, jlo2);
                const int je = min(se, wrap ? jlo2 + jc2 - nj2 : jlo2 + jc2);
                const int npts = v2 ? max(je - jb, 0) : 0;
                const double rc2 = bperm_d(s2, rcd), rs2 = bperm_d(s2, rsd);
                const int sr2 = bperm_i(s2, srf);
                const float w2 = bperm_f(s2, w), dl2 = bperm_f(s2, dlt);
                const int rrel2 = SEGB ? bperm_i(s2, rrel1) : 0;
                const int ub = wrap ? jb + nj2 - jlo2 : jb - jlo2;   // offset of jb in the arc
                segment_points<MODE>(P, W, B, lo, hi, uq, e3, e1d, e2d, e1, e2, v2, rc2, rs2, sr2,
                                     w2, dl2, nj2, ls2, k2, jb, npts, ub, s2, klo, unit, rrel2,
                                     scount, fn);
            }
            }  // pass2
            if (MODE == WALK_COUNT || MODE == WALK_FILL) {
                wave_sync();
                const int umin = B->rmin[lane], umax = B->rmax[lane];
                const bool has = v1 && umax >= 0;
                if (MODE == WALK_COUNT) {
                    if (has) {
                        atomicMin(&B->smin[s1], ir);
                        atomicMax(&B->smax[s1], ir);
                    }
                } else if (v1 && ir >= run_i0 && ir < run_i0 + run_n) {
                    int jl = jlo + umin;
                    if (jl >= nj) jl -= nj;
                    P.tab_arc[ebase + run_ex + (ir - run_i0)] =
                        has ? ((unsigned)jl | ((unsigned)(umax - umin + 1) << 16)) : 0u;
                }
                wave_sync();
            }
        }
        }  // pass1
        if (MODE == WALK_COUNT) {
            wave_sync();
            if (k <= khi) {
                const int imin = B->smin[lane], imax = B->smax[lane];
                const bool any = imax >= 0;
                P.tab_run[unit * P.window + (k - klo)] =
                    any ? ((unsigned)imin | ((unsigned)(imax - imin + 1) << 16)) : 0u;
                ucount += any ? imax - imin + 1 : 0;
            }
            wave_sync();
        }
    }
    if (MODE == WALK_COUNT) {
        const float tot = wave_sum_dpp((float)ucount);
        if (lane == 0) P.tab_cnt[unit] = (int)tot;
    }
    if (MODE == WALK_SEGCOUNT) {
        if (lane == 0) P.seg_cnt[unit] = (int)scount;
        if (lane < 32) P.seg_hist[unit * 32 + lane] = B->hist[lane];
    }
}

// Per-wave LDS of the segment-table walk: the global index of each shell's
// first candidate ring for the current unit.
struct SegWave {
    int gbase[WMAX];
};

// Maximum over the 64 lanes (all active), returned to every lane.
__device__ __forceinline__ int wave_max_i(int v)
{
    v = max(v, dpp_i<0xB1, 0xF>(v));    // quad_perm [1,0,3,2]
    v = max(v, dpp_i<0x4E, 0xF>(v));    // quad_perm [2,3,0,1]
    v = max(v, dpp_i<0x141, 0xF>(v));   // row_half_mirror
    v = max(v, dpp_i<0x140, 0xF>(v));   // row_mirror: every lane holds its row maximum
    v = max(v, __builtin_amdgcn_readlane(v, 16));
    v = max(v, __builtin_amdgcn_readlane(v, 32));
    v = max(v, __builtin_amdgcn_readlane(v, 48));
    return __builtin_amdgcn_readfirstlane(v);
}

// Walk the points of transducer q owned by the brick from the plan's segment
// table: one segment per lane, 64 at a time, each lane taking its segment's
// points one after the other (a window's segments have nearly equal counts:
// the table orders a unit's segments by decreasing count).  The positions
// are those of walk_unit's point level (seg_ref, seg_point), so the owned
// point set is the same.  pfn(t, w) is called for every point of a segment
// with its weight (w g' in G^T), then sfn(np, so, w) once per window with
// the lane's segment count (0: none), shell offset and weight.
template <bool ADJ, class PFn, class SFn>
__device__ __forceinline__ void walk_seg(const Problem &P, int q, size_t unit, const int lo[3],
                                         const int hi[3], int *gbase, const float *gp,
                                         float gscale, float gscale2, int &klo_out, PFn &&pfn,
                                         SFn &&sfn)
{
    const DetRec &d = P.det[q];
    const double uq[3] = {d.uq[0], d.uq[1], d.uq[2]};
    const double e3[3] = {d.e3[0], d.e3[1], d.e3[2]};
    const double e1d[3] = {d.e1d[0], d.e1d[1], d.e1d[2]};
    const double e2d[3] = {d.e2d[0], d.e2d[1], d.e2d[2]};
    const float e1[3] = {d.e1[0], d.e1[1], d.e1[2]};
    const float e2[3] = {d.e2[0], d.e2[1], d.e2[2]};
    int klo, khi;
    unit_shells(P, uq, lo, hi, klo, khi);
    klo_out = klo;
    const int lane = lane_id();
    const long long s0 = P.seg_off[unit], s1 = P.seg_off[unit + 1];
    if (s0 >= s1) return;
    // Each shell's first candidate ring, as the bounds walk found it when
    // the table was built (the same FP32 operations).
    {
        ArcUnit U;
        arc_unit_setup(U, lo, hi, uq, e1, e2, e3, 0.02f);
        const float D = sqrtf(U.rhov2 + U.V3 * U.V3);
        const float thb = acos_approx(U.V3 * rcp_approx(D));
        for (int so = lane; so <= khi - klo; so += WAVE) {
            const ShellRec sh = P.shell[klo + so];
            int i0, cnt;
            shell_rings(sh, D, thb, U.h2, i0, cnt);
            gbase[so] = sh.ring_base + i0;
        }
        wave_sync();
    }
    // The next window's entries are loaded while this window runs.
    unsigned nxt = s0 + lane < s1 ? P.seg[s0 + lane] : 0u;
    for (long long c = s0; c < s1; c += WAVE) {
        const bool v = c + lane < s1;
        const unsigned ent = nxt;
        const long long en = c + WAVE + lane;
        nxt = en < s1 ? P.seg[en] : 0u;
        const int so = (int)(ent & ((1u << SEG_SHELL_BITS) - 1u));
        const int rrel = (int)((ent >> SEG_SHELL_BITS) & ((1u << SEG_RING_BITS) - 1u));
        const int sg = (int)((ent >> (SEG_SHELL_BITS + SEG_RING_BITS)) &
                             ((1u << SEG_INDEX_BITS) - 1u));
        const int off = (int)((ent >> (32 - SEG_CNT_BITS - SEG_OFF_BITS)) &
                              ((1u << SEG_OFF_BITS) - 1u));
        const int np = v ? (int)(ent >> (32 - SEG_CNT_BITS)) + 1 : 0;
        // (the clamps only keep a table that disagrees with the walk inside
        // the tables; they never bind for a table built by this plan)
        const RingRec rr = P.ring[v ? min(max(gbase[so] + rrel, 0), P.n_rings - 1) : 0];
        const int jref = seg_ref_index(sg, rr.lshift, rr.nj);
        const int dj0 = (sg << rr.lshift) + off - jref;   // first point, relative to jref
        float Pl[3], xa, xb;
        int dc[3];
        seg_ref(uq, e3, e1d, e2d, lo, rr.rc, rr.rs,
                v ? P.segref[min(rr.sref + sg, P.n_segref - 1)] : make_double2(1.0, 0.0), Pl,
                dc, xa, xb);
        float w = rr.w;
        if (ADJ && v) w = w * ((gp[(size_t)q * P.nt + klo + so] * gscale) * gscale2);
        const SegAxes ax = seg_axes(xa, xb, e1, e2);
        const int nmax = wave_max_i(np);
        // dj0 + t as an FP32 counter (exact: |dj| < 2^24), one add per point
        float fdj = (float)dj0;
        for (int t = 0; t < nmax; ++t, fdj += 1.f) {
            if (t < np) {
                const Pt pt = seg_point(Pl, dc, ax, rr.delta, fdj, lo, hi);
                if (pt.own) pfn(pt, w);
            }
        }
        sfn(np, so, w);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// G: partial sums per (brick, transducer) window.
// ---------------------------------------------------------------------------
constexpr int FWD_WAVES = 16;

template <int IMG_DT, int TM>
__global__ void __launch_bounds__(FWD_WAVES *WAVE) __attribute__((amdgpu_waves_per_eu(4, 4)))
srt_fwd_kernel(Problem P, const void *__restrict__ img, float *__restrict__ part,
               int *__restrict__ klo_out, int q_per_slice)
{
    static_assert(TM != TM_SEG, "the segment table has srt_fwd_seg_kernel");
    using WL = WaveLds;
    __shared__ float box[BOX_WORDS];
    __shared__ WL wl[FWD_WAVES];
    __shared__ double gwin[FWD_WAVES][WMAX];
    __shared__ int q_next;
    const int b = blockIdx.x;
    int lo[3], hi[3], n0[3], n1[3];
    brick_box(P, b, lo, hi, n0, n1);
    // Transducers of this workgroup's slice (blockIdx.y) of the brick's.
    const int qb = (int)blockIdx.y * q_per_slice, qe = min(P.nq, qb + q_per_slice);
    if (threadIdx.x == 0) q_next = qb;

    // Stage nodes lo .. lo+BOX-1 (zero outside the grid).
    for (int t = threadIdx.x; t < BOX * BOX * BOX; t += blockDim.x) {
        int x = t % BOX, y = (t / BOX) % BOX, z = t / (BOX * BOX);
        int gx = lo[0] + x, gy = lo[1] + y, gz = lo[2] + z;
        float v = 0.f;
        if (gx >= 0 && gx < P.nx && gy >= 0 && gy < P.ny && gz >= 0 && gz < P.nz) {
            size_t n = ((size_t)gz * P.ny + gy) * P.nx + gx;
            if (IMG_DT == 0)
                v = ((const float *)img)[n];
            else
                v = __uint_as_float(((unsigned)((const unsigned short *)img)[n]) << 16);
        }
        box[z * BOX_SZ + y * BOX_SY + x] = v;
    }
    __syncthreads();

    const int wave = threadIdx.x / WAVE;
    const int lane = lane_id();
    WL &W = wl[wave];
    double *gw = gwin[wave];
    // Each wave takes the slice's next transducer when it finishes one (an
    // LDS counter), so the waves end together whatever the units cost.
    for (;;) {
        int q = 0;
        if (lane == 0) q = atomicAdd(&q_next, 1);
        q = __builtin_amdgcn_readfirstlane(q);
        if (q >= qe) break;
        for (int j = lane; j < P.window; j += WAVE) gw[j] = 0.0;
        wave_sync();
        int klo = 0;
        // Each lane keeps a running FP32 sum for its current shell (a lane's
        // points arrive in shell order) and adds it to the wave's FP64 shell
        // window with the native LDS FP64 atomic when the shell changes.
        float racc = 0.f;
        int rk = -1, rbase = 0;
        auto interp = [&](const Pt &t) {
            const float *pb = box + __umul24((unsigned)t.cz, BOX_SZ) + __umul24((unsigned)t.cy, BOX_SY) + t.cx;
            const float *pz = pb + BOX_SZ;
            const float v000 = pb[0], v001 = pb[1], v010 = pb[BOX_SY], v011 = pb[BOX_SY + 1];
            const float v100 = pz[0], v101 = pz[1], v110 = pz[BOX_SY], v111 = pz[BOX_SY + 1];
            const float c00 = fmaf(t.fx, v001 - v000, v000), c01 = fmaf(t.fx, v011 - v010, v010);
            const float c10 = fmaf(t.fx, v101 - v100, v100), c11 = fmaf(t.fx, v111 - v110, v110);
            const float c0 = fmaf(t.fy, c01 - c00, c00), c1 = fmaf(t.fy, c11 - c10, c10);
            return fmaf(t.fz, c1 - c0, c0);
        };
        auto gather = [&](const Pt &a, const Pt &c, float wv, int kk, int kbase) {
            float sum = 0.f;
            if (a.own) sum = interp(a);
            if (c.own) sum += interp(c);
            if (a.own || c.own) {
                if (kk != rk) {
                    if (rk >= 0) atomicAdd(gw + (rk - rbase), (double)racc);
                    rk = kk;
                    rbase = kbase;
                    racc = 0.f;
                }
                racc = fmaf(sum, wv, racc);
            }
        };
        walk_unit<false, TM, WALK_POINTS>(P, q, (size_t)b * P.nq + q, lo, hi, W, nullptr,
                                           nullptr, 1.f, 1.f, klo, gather);
        if (rk >= 0) atomicAdd(gw + (rk - rbase), (double)racc);
        wave_sync();
        float *dst = part + ((size_t)b * P.nq + q) * P.window;
        for (int j = lane; j < P.window; j += WAVE) dst[j] = (float)gw[j];
        if (lane == 0) klo_out[(size_t)b * P.nq + q] = klo;
        wave_sync();
    }
}

// G on the segment table: one segment per lane (walk_seg), FWD_SEG_WAVES
// waves per workgroup and two workgroups per CU (at most 64 VGPRs, the LDS
// of two boxes).  Per wave, dynamic LDS holds the unit's first candidate
// ring per shell (window ints) and its fixed-point shell sums (window
// 64-bit integers).
constexpr int FWD_SEG_WAVES = 16;

template <int IMG_DT>
__global__ void __launch_bounds__(FWD_SEG_WAVES *WAVE) __attribute__((amdgpu_waves_per_eu(8, 8)))
srt_fwd_seg_kernel(Problem P, const void *__restrict__ img, float *__restrict__ part,
                   int *__restrict__ klo_out, int q_per_slice)
{
    constexpr int NW = FWD_SEG_WAVES;
    __shared__ float box[BOX_WORDS];
    __shared__ int q_next;
    __shared__ float wmax[NW];
    __shared__ int wbad[NW];
    __shared__ double fx_scale, fx_unscale;
    extern __shared__ double dyn_lds[];
    const int win = P.window;
    const int b = blockIdx.x;
    int lo[3], hi[3], n0[3], n1[3];
    brick_box(P, b, lo, hi, n0, n1);
    const int qb = (int)blockIdx.y * q_per_slice, qe = min(P.nq, qb + q_per_slice);
    if (threadIdx.x == 0) q_next = qb;
    // the box's largest |node| (and whether any node is not finite) sets
    // the fixed-point scale of the shell sums below
    float amax = 0.f;
    int abad = 0;
    auto node = [&](int x, int y, int z) {
        const int gx = lo[0] + x, gy = lo[1] + y, gz = lo[2] + z;
        float v = 0.f;
        if (gx >= 0 && gx < P.nx && gy >= 0 && gy < P.ny && gz >= 0 && gz < P.nz) {
            const size_t n = ((size_t)gz * P.ny + gy) * P.nx + gx;
            if (IMG_DT == 0)
                v = ((const float *)img)[n];
            else
                v = __uint_as_float(((unsigned)((const unsigned short *)img)[n]) << 16);
        }
        const float a = fabsf(v);
        abad |= !(a <= 3.4028235e38f);
        amax = fmaxf(amax, a);
        return v;
    };
    // FP32 images: one node per word.  BF16 images: word x holds the BF16
    // pair (node x, node x + 1), so a point's 8 corners are 4 words (2 reads).
    if constexpr (IMG_DT == 0) {
        for (int t = threadIdx.x; t < BOX * BOX * BOX; t += blockDim.x) {
            const int x = t % BOX, y = (t / BOX) % BOX, z = t / (BOX * BOX);
            box[z * BOX_SZ + y * BOX_SY + x] = node(x, y, z);
        }
    } else {
        unsigned *bw = reinterpret_cast<unsigned *>(box);
        for (int t = threadIdx.x; t < (BOX - 1) * BOX * BOX; t += blockDim.x) {
            const int x = t % (BOX - 1), y = (t / (BOX - 1)) % BOX, z = t / ((BOX - 1) * BOX);
            bw[z * BOX_SZ + y * BOX_SY + x] =
                (__float_as_uint(node(x, y, z)) >> 16) | (__float_as_uint(node(x + 1, y, z)) & 0xffff0000u);
        }
    }
    const int wave = threadIdx.x / WAVE;
    const int lane = lane_id();
    for (int o = 32; o > 0; o >>= 1) {
        amax = fmaxf(amax, __shfl_xor(amax, o));
        abad |= __shfl_xor(abad, o);
    }
    if (lane == 0) {
        wmax[wave] = amax;
        wbad[wave] = abad;
    }
    // Shell sums in 64-bit fixed point (order-independent, and the integer
    // LDS add is cheaper than the FP64 one).  A unit's shell holds at most
    // 2^19 points (63 rings x 256 segments x 32 points: the entry's fields),
    // each adding |psi-interpolated node| w <= M w_max, so with
    // M w_max < 2^e a scale of 2^(43 - e) keeps every sum below 2^62.  A box
    // with a non-finite node gives NaN sums.
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = 0.f;
        int bad = 0;
        for (int w = 0; w < NW; ++w) {
            m = fmaxf(m, wmax[w]);
            bad |= wbad[w];
        }
        int e = 0;
        frexp((double)m * (double)P.w_max, &e);
        if (!(m > 0.f)) e = 43;
        fx_scale = bad ? __longlong_as_double(0x7ff8000000000000ll) : ldexp(1.0, 43 - e);
        fx_unscale = bad ? fx_scale : ldexp(1.0, e - 43);
    }
    unsigned long long *gw = reinterpret_cast<unsigned long long *>(dyn_lds) + (size_t)wave * win;
    int *gbase = reinterpret_cast<int *>(dyn_lds + (size_t)NW * win) + wave * win;
    __syncthreads();
    // (uniform: kept in scalar registers)
    auto uniform = [](double x) {
        const long long b = __double_as_longlong(x);
        return __longlong_as_double(
            ((long long)__builtin_amdgcn_readfirstlane((int)(b >> 32)) << 32) |
            (unsigned)__builtin_amdgcn_readfirstlane((int)b));
    };
    const double fxs = uniform(fx_scale), fxi = uniform(fx_unscale);
    for (;;) {
        int q = 0;
        if (lane == 0) q = atomicAdd(&q_next, 1);
        q = __builtin_amdgcn_readfirstlane(q);
        if (q >= qe) break;
        for (int j = lane; j < win; j += WAVE) gw[j] = 0ull;
        wave_sync();
        int klo = 0;
        float racc = 0.f;
        // FP32 images: a point in the same cell as the lane's previous point
        // reuses its corners without reading LDS (BF16 images, with half the
        // reads, are faster without the test).
        unsigned prev = 0xffffffffu;
        float c8[8];   // loaded before any use: prev starts out unmatched
        auto point = [&](const Pt &t, float) {
            float v000, v001, v010, v011, v100, v101, v110, v111;
            const unsigned off = __umul24((unsigned)t.cz, BOX_SZ) +
                                 __umul24((unsigned)t.cy, BOX_SY) + t.cx;
            if constexpr (IMG_DT == 0) {
                if (off != prev) {
                    prev = off;
                    const float *pb = box + off;
                    const float *pz = pb + BOX_SZ;
                    c8[0] = pb[0], c8[1] = pb[1], c8[2] = pb[BOX_SY], c8[3] = pb[BOX_SY + 1];
                    c8[4] = pz[0], c8[5] = pz[1], c8[6] = pz[BOX_SY], c8[7] = pz[BOX_SY + 1];
                }
                v000 = c8[0], v001 = c8[1], v010 = c8[2], v011 = c8[3];
                v100 = c8[4], v101 = c8[5], v110 = c8[6], v111 = c8[7];
            } else {
                const unsigned *pb = reinterpret_cast<const unsigned *>(box) + off;
                const unsigned *pz = pb + BOX_SZ;
                const unsigned w00 = pb[0], w01 = pb[BOX_SY], w10 = pz[0], w11 = pz[BOX_SY];
                v000 = __uint_as_float(w00 << 16), v001 = __uint_as_float(w00 & 0xffff0000u);
                v010 = __uint_as_float(w01 << 16), v011 = __uint_as_float(w01 & 0xffff0000u);
                v100 = __uint_as_float(w10 << 16), v101 = __uint_as_float(w10 & 0xffff0000u);
                v110 = __uint_as_float(w11 << 16), v111 = __uint_as_float(w11 & 0xffff0000u);
            }
            const float c00 = fmaf(t.fx, v001 - v000, v000), c01 = fmaf(t.fx, v011 - v010, v010);
            const float c10 = fmaf(t.fx, v101 - v100, v100), c11 = fmaf(t.fx, v111 - v110, v110);
            const float c0 = fmaf(t.fy, c01 - c00, c00), c1 = fmaf(t.fy, c11 - c10, c10);
            racc += fmaf(t.fz, c1 - c0, c0);
        };
        // one segment (one shell) per lane: the weighted sum of its points,
        // racc w (exact in FP64) times the power-of-two scale, goes to the
        // shell's fixed-point entry.  The term is below 2^48 (at most 32
        // points), so adding 1.5 2^52 rounds it to an integer that the low
        // bits of the sum hold exactly, offset by the constant's bits.
        auto segment = [&](int np, int so, float wv) {
            if (np > 0) {
                const double t = fma((double)racc * (double)wv, fxs, 0x1.8p52);
                atomicAdd(gw + so, (unsigned long long)(__double_as_longlong(t) -
                                                        __double_as_longlong(0x1.8p52)));
            }
            racc = 0.f;
            prev = 0xffffffffu;
        };
        walk_seg<false>(P, q, (size_t)b * P.nq + q, lo, hi, gbase, nullptr, 1.f, 1.f, klo, point,
                        segment);
        wave_sync();
        float *dst = part + ((size_t)b * P.nq + q) * win;
        for (int j = lane; j < win; j += WAVE) {
            const long long sj = (long long)gw[j];
            dst[j] = (float)(fma((double)(int)(sj >> 32), 0x1p32, (double)(unsigned)sj) * fxi);
        }
        if (lane == 0) klo_out[(size_t)b * P.nq + q] = klo;
        wave_sync();
    }
}

// ---------------------------------------------------------------------------
// G^T: each brick takes the same cells (hence the same points) as in G and
// accumulates their trilinear weights w g' psi in an LDS box of fixed-point
// integers, 12 or 16 waves sharing the box.
//
// One 64-bit word per cell column holds two 32-bit fields: node x in the low
// half and node x + 1 in the high half, so a point adds its 8 corner weights
// with 4 ds_add_u64 (the x pair of each (y, z) corner in one atomic; the
// 64-bit integer add is the cheapest LDS atomic on this part, the FP32 one
// is microcoded).  A field value v is added as the signed 64-bit integer
// lo + hi 2^32; as long as the sums of both fields stay inside 32-bit signed
// range the word decodes exactly: lo = low 32 bits (signed), hi = (word - lo)
// >> 32 (arithmetic).
//
// The transducers are taken in windows of ADJ_WINDOW = 128 (the NW waves
// take a window's transducers one at a time from an LDS counter).  A window's
// weights are multiplied by S = 0.99 * 2^31 / (R G) and rounded to the nearest
// integer (v_cvt_rpi_i32_f32), where
//   R(brick, window) = max over box nodes of sum psi w over the window's
//                      points (measured once per plan, calibration mode), and
//   G(window)        = max |g'| of the window's transducers over the samples
//                      whose shell can reach the image support,
// so no field can leave 32-bit range.  After each window the fields are
// decoded, multiplied by 1/S and added into the brick's FP64 node
// accumulators in HBM (window order fixed: G^T is deterministic), and the box
// is cleared.  Each rounding error is at most half a unit, 2^-32 of R G: the
// precision of an FP32 sum of the window's terms, without its dependence on
// the order of the atomics.
//
// Calibration mode (once per plan): the same walk with g' = 1 on the
// per-node 64-bit box layout (8 atomics per point, each term below 2^30,
// sums far below 2^63), writing R(brick, window) rounded up.
//
// The box (its owned nodes and the one-node layer below them, which belongs
// to the neighbouring bricks) ends in HBM in FP64; adj_gather_kernel adds the
// overlapping layers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int cvt_rne(float x)
{
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));   // floor(x + 0.5)
    return r;
}

// Exponent s with bound * 2^s < 2^target (bound > 0, finite), as two normal
// FP32 factors 2^(s/2) 2^(s - s/2) (|s| <= 252) and the FP64 inverse.
__device__ __forceinline__ void window_scale(double bound, int target, float &g1, float &g2,
                                             double &unscale)
{
    int e = 0;
    (void)frexp(bound, &e);                   // bound < 2^e
    const int sh = (bound > 0.0 && bound <= 1e300) ? min(max(target - e, -252), 252) : 0;
    g1 = ldexpf(1.f, sh / 2);
    g2 = ldexpf(1.f, sh - sh / 2);
    unscale = ldexp(1.0, -sh);
}

// Scale 0.99 * 2^31 / bound (bound > 0, finite) as two FP32 factors and the
// FP64 inverse of their product: with it no sum of terms whose magnitudes
// add up to at most bound leaves 32-bit signed range (the 1% margin covers
// FP32 rounding of the terms and half a unit per rounded term).
__device__ __forceinline__ void field_scale(double bound, float &g1, float &g2, double &unscale)
{
    if (!(bound > 0.0 && bound <= 1e300)) {
        g1 = g2 = 1.f;
        unscale = 1.0;
        return;
    }
    int e = 0;
    const double m = frexp(bound, &e);        // bound = m 2^e, m in [0.5, 1)
    const int sh = min(max(31 - e, -250), 250);
    g1 = ldexpf(1.f, sh / 2);
    g2 = ldexpf((float)(0.99 / m), sh - sh / 2);
    unscale = 1.0 / ((double)g1 * (double)g2);
}

template <int TM, bool CALIB, int NW>
__global__ void __launch_bounds__(NW *WAVE) __attribute__((amdgpu_waves_per_eu(NW / 4, NW / 4)))
srt_adj_kernel(Problem P, const float *__restrict__ gp, double *__restrict__ acc,
               float *__restrict__ rcal, int win_per_slice)
{
    // The segment-table walk needs only the point level's LDS, which leaves
    // room for 16 waves beside the box.
    static_assert(NW <= 12 || TM == TM_SEG, "16 waves fit the LDS only on the segment path");
    using WL = typename std::conditional<TM == TM_SEG, SegWave, WaveLds>::type;
    __shared__ unsigned long long box[BOX_WORDS];
    __shared__ WL wl[NW];
    __shared__ unsigned long long wred[NW];
    __shared__ int q_next;
    __shared__ int qperm[ADJ_WINDOW];
    __shared__ long long qcost[ADJ_WINDOW];
    const int b = blockIdx.x;
    int lo[3], hi[3], n0[3], n1[3];
    brick_box(P, b, lo, hi, n0, n1);
    const int nwin = adj_windows(P.nq);
    const int wave = threadIdx.x / WAVE, lane = lane_id();
    // Order in which the waves take a window's transducers (wave 0 writes
    // it): with the segment table by decreasing segment count, so the
    // longest units start first and the waves reach the window's barrier
    // close together; otherwise in index order.
    auto order_window = [&](int wn) {
        const int qa = wn * ADJ_WINDOW, cnt = min(ADJ_WINDOW, P.nq - qa);
        if constexpr (TM == TM_SEG && !CALIB) {
            for (int i = lane; i < cnt; i += WAVE) {
                const size_t u = (size_t)b * P.nq + qa + i;
                qcost[i] = P.seg_off[u + 1] - P.seg_off[u];
            }
            wave_sync();
            for (int i = lane; i < cnt; i += WAVE) {
                const long long c = qcost[i];
                int rank = 0;
                for (int j = 0; j < cnt; ++j) {
                    const long long cj = qcost[j];
                    rank += (cj > c || (cj == c && j < i)) ? 1 : 0;
                }
                qperm[rank] = qa + i;
            }
        } else {
            for (int i = lane; i < cnt; i += WAVE) qperm[i] = qa + i;
        }
    };
    // Windows of this workgroup's slice (blockIdx.y); each slice has its own
    // FP64 brick sums.
    const int w0 = (int)blockIdx.y * win_per_slice, w1 = min(nwin, w0 + win_per_slice);
    for (int t = threadIdx.x; t < BOX_WORDS; t += blockDim.x) box[t] = 0ull;
    if (threadIdx.x == 0) q_next = 0;
    if (wave == 0) order_window(w0);
    __syncthreads();
    WL &W = wl[wave];
    for (int win = w0; win < w1; ++win) {
        const int q0 = win * ADJ_WINDOW;
        float g1, g2;
        double unscale;
        if (CALIB) {
            window_scale((double)P.w_max, 30, g1, g2, unscale);
        } else {
            float m = 0.f;
            for (int j = lane; j < ADJ_WINDOW && q0 + j < P.nq; j += WAVE)
                m = fmaxf(m, P.gp_rowmax[q0 + j]);
            for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
            field_scale((double)P.adj_r[(size_t)b * nwin + win] * (double)m, g1, g2, unscale);
        }
        // Each wave takes the window's next transducer (in qperm order) when
        // it finishes one (an LDS counter): the waves reach the flush
        // together whatever the units cost.  The LDS sums are exact
        // integers, so the order of the units does not change them.
        const int cntw = min(ADJ_WINDOW, P.nq - q0);
        for (;;) {
            int i = 0;
            if (lane == 0) i = atomicAdd(&q_next, 1);
            i = __builtin_amdgcn_readfirstlane(i);
            if (i >= cntw) break;
            const int q = qperm[i];
            int klo = 0;
            if (CALIB) {
                auto scatter1 = [&](const Pt &t, float wv) {
                    unsigned long long *pb = box + __umul24((unsigned)t.cz, BOX_SZ) +
                                             __umul24((unsigned)t.cy, BOX_SY) + t.cx;
                    unsigned long long *pz = pb + BOX_SZ;
                    const float gx = 1.f - t.fx, gy = 1.f - t.fy, gz = 1.f - t.fz;
                    const float w00 = gy * gz * wv, w01 = t.fy * gz * wv, w10 = gy * t.fz * wv,
                                w11 = t.fy * t.fz * wv;
                    auto add = [](unsigned long long *p, float v) {
                        atomicAdd(p, (unsigned long long)(long long)cvt_rne(v));
                    };
                    add(pb, gx * w00);
                    add(pb + 1, t.fx * w00);
                    add(pb + BOX_SY, gx * w01);
                    add(pb + BOX_SY + 1, t.fx * w01);
                    add(pz, gx * w10);
                    add(pz + 1, t.fx * w10);
                    add(pz + BOX_SY, gx * w11);
                    add(pz + BOX_SY + 1, t.fx * w11);
                };
                if constexpr (TM == TM_SEG) {
                    auto point = [&](const Pt &t, float wv) { scatter1(t, (wv * g1) * g2); };
                    auto segment = [](int, int, float) {};
                    walk_seg<false>(P, q, (size_t)b * P.nq + q, lo, hi, W.gbase, nullptr, 1.f,
                                    1.f, klo, point, segment);
                } else {
                    auto scatter = [&](const Pt &a, const Pt &c, float wv, int, int) {
                        if (a.own) scatter1(a, (wv * g1) * g2);
                        if (c.own) scatter1(c, (wv * g1) * g2);
                    };
                    walk_unit<false, TM, WALK_POINTS>(P, q, (size_t)b * P.nq + q, lo, hi, W,
                                                       nullptr, nullptr, 1.f, 1.f, klo, scatter);
                }
            } else {
                auto scatter1 = [&](const Pt &t, float wv) {
                    // word index, then bytes (one multiply-add fewer than
                    // scaling each term)
                    const unsigned wi = __umul24((unsigned)t.cz, BOX_SZ) +
                                        (__umul24((unsigned)t.cy, BOX_SY) + (unsigned)t.cx);
                    unsigned long long *pb = reinterpret_cast<unsigned long long *>(
                        reinterpret_cast<char *>(box) + (wi << 3));
                    unsigned long long *pz = pb + BOX_SZ;
                    // trilinear corner weights, (1 - f) v formed as v - f v
                    const float a = fmaf(-t.fz, wv, wv), c = t.fz * wv;
                    const float w00 = fmaf(-t.fy, a, a), w01 = t.fy * a, w10 = fmaf(-t.fy, c, c),
                                w11 = t.fy * c;
                    // fields (node x, node x + 1) of one word: the 64-bit
                    // integer l + h 2^32 (l sign-extended), formed with 32-bit
                    // operations: high word h + (l >> 31)
                    auto add2 = [&](unsigned long long *p, float wyz) {
                        const int l = cvt_rne(fmaf(-t.fx, wyz, wyz)), h = cvt_rne(t.fx * wyz);
                        const unsigned hw = (unsigned)h + (unsigned)(l >> 31);
                        atomicAdd(p, ((unsigned long long)hw << 32) | (unsigned)l);
                    };
                    add2(pb, w00);
                    add2(pb + BOX_SY, w01);
                    add2(pz, w10);
                    add2(pz + BOX_SY, w11);
                };
                if constexpr (TM == TM_SEG) {
                    auto point = [&](const Pt &t, float wv) { scatter1(t, wv); };
                    auto segment = [](int, int, float) {};
                    walk_seg<true>(P, q, (size_t)b * P.nq + q, lo, hi, W.gbase, gp, g1, g2, klo,
                                   point, segment);
                } else {
                    auto scatter = [&](const Pt &a, const Pt &c, float wv, int, int) {
                        if (a.own) scatter1(a, wv);
                        if (c.own) scatter1(c, wv);
                    };
                    walk_unit<true, TM, WALK_POINTS>(P, q, (size_t)b * P.nq + q, lo, hi, W,
                                                      nullptr, gp, g1, g2, klo, scatter);
                }
            }
        }
        __syncthreads();
        if (CALIB) {
            unsigned long long m = 0ull;
            for (int t = threadIdx.x; t < BOX_WORDS; t += blockDim.x) {
                const long long v = (long long)box[t];
                m = max(m, (unsigned long long)(v < 0 ? -v : v));
            }
            for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o));
            if (lane == 0) wred[wave] = m;
            __syncthreads();
            if (threadIdx.x == 0) {
                unsigned long long mm = 0ull;
                for (int w = 0; w < NW; ++w) mm = max(mm, wred[w]);
                // rounded up: (float) may round down, and each of the at most
                // 2^20 terms of a node lost at most half a unit
                const double r = ((double)mm + 1048576.0) * unscale;
                rcal[(size_t)b * nwin + win] = (float)r * (1.f + 1.f / 1024.f);
            }
        } else {
            double *dst =
                acc + ((size_t)blockIdx.y * (P.nbx * P.nby * P.nbz) + b) * BOX3;
            for (int t = threadIdx.x; t < BOX3; t += blockDim.x) {
                const int x = t % BOX, y = (t / BOX) % BOX, z = t / (BOX * BOX);
                const unsigned long long *row = box + z * BOX_SZ + y * BOX_SY;
                long long v = 0;
                if (x < BOX - 1) v += (long long)(int)(unsigned)row[x];
                if (x > 0) {
                    const long long wd = (long long)row[x - 1];
                    const long long l = (long long)(int)(unsigned)wd;
                    v += (wd - l) >> 32;
                }
                const double a = (double)v * unscale;
                dst[t] = win == w0 ? a : dst[t] + a;
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < BOX_WORDS; t += blockDim.x) box[t] = 0ull;
        if (threadIdx.x == 0) q_next = 0;
        if (wave == 0 && win + 1 < w1) order_window(win + 1);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Arc table, built once per plan in two passes over the same enumeration as
// G: WALK_COUNT records, per (brick, transducer, shell), the run of rings
// that hold owned points and the unit's entry count; after the host has
// turned the counts into offsets, WALK_FILL writes each ring's tight arc.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ void __launch_bounds__(WAVES *WAVE) __attribute__((amdgpu_waves_per_eu(4, 4)))
arc_build_kernel(Problem P)
{
    __shared__ WaveLds wl[WAVES];
    __shared__ BuildLds bl[WAVES];
    const int b = blockIdx.x;
    int lo[3], hi[3], n0[3], n1[3];
    brick_box(P, b, lo, hi, n0, n1);
    const int wave = threadIdx.x / WAVE;
    auto none = [](const Pt &, const Pt &, float, int, int) {};
    for (int q = wave; q < P.nq; q += WAVES) {
        int klo = 0;
        walk_unit<false, TM_BOUNDS, MODE>(P, q, (size_t)b * P.nq + q, lo, hi, wl[wave],
                                          &bl[wave], nullptr, 1.f, 1.f, klo, none);
    }
}

template <int TM>
static void fwd_launch(const Problem &P, const void *img, int img_dtype, float *part, int *klo,
                       hipStream_t s)
{
    const int nb = P.nbx * P.nby * P.nbz;
    const int sl = TM == TM_SEG ? seg_fwd_slices(nb, P.nq) : fwd_slices(nb, P.nq);
    const int qps = (P.nq + sl - 1) / sl;
    if constexpr (TM == TM_SEG) {
        dim3 grid(P.nbx * P.nby * P.nbz, sl), block(FWD_SEG_WAVES * WAVE);
        const size_t dyn = (size_t)FWD_SEG_WAVES * P.window * (sizeof(double) + sizeof(int));
        if (img_dtype == 0)
            hipLaunchKernelGGL(srt_fwd_seg_kernel<0>, grid, block, dyn, s, P, img, part, klo, qps);
        else
            hipLaunchKernelGGL(srt_fwd_seg_kernel<1>, grid, block, dyn, s, P, img, part, klo, qps);
    } else {
        dim3 grid(P.nbx * P.nby * P.nbz, sl), block(FWD_WAVES * WAVE);
        if (img_dtype == 0)
            hipLaunchKernelGGL((srt_fwd_kernel<0, TM>), grid, block, 0, s, P, img, part, klo, qps);
        else
            hipLaunchKernelGGL((srt_fwd_kernel<1, TM>), grid, block, 0, s, P, img, part, klo, qps);
    }
}

static int table_mode(const Problem &P)
{
    return P.seg != nullptr ? TM_SEG : (P.tab_arc != nullptr ? TM_ARC : TM_BOUNDS);
}

hipError_t launch_srt_fwd(const Problem &P, const void *img, int img_dtype, float *part, int *klo,
                          hipStream_t s)
{
    switch (table_mode(P)) {
    case TM_SEG: fwd_launch<TM_SEG>(P, img, img_dtype, part, klo, s); break;
    case TM_ARC: fwd_launch<TM_ARC>(P, img, img_dtype, part, klo, s); break;
    default: fwd_launch<TM_BOUNDS>(P, img, img_dtype, part, klo, s); break;
    }
    return hipGetLastError();
}

// 16 waves on the segment path, 12 otherwise; the calibration always takes
// 12 (its per-node box needs more registers), which does not change R: a
// window's node sums do not depend on how its transducers are split among
// the waves.
template <bool CALIB>
static void adj_launch(const Problem &P, const float *gp, double *acc, float *r, hipStream_t s)
{
    const int nb = P.nbx * P.nby * P.nbz, nwin = adj_windows(P.nq);
    const int sl = adj_slices(nb, P.nq), wps = (nwin + sl - 1) / sl;
    dim3 grid(nb, sl), b12(12 * WAVE), b16(16 * WAVE);
    switch (table_mode(P)) {
    case TM_SEG:
        if (CALIB)
            hipLaunchKernelGGL((srt_adj_kernel<TM_SEG, true, 12>), grid, b12, 0, s, P, gp, acc, r,
                               wps);
        else
            hipLaunchKernelGGL((srt_adj_kernel<TM_SEG, false, 16>), grid, b16, 0, s, P, gp, acc, r,
                               wps);
        break;
    case TM_ARC:
        hipLaunchKernelGGL((srt_adj_kernel<TM_ARC, CALIB, 12>), grid, b12, 0, s, P, gp, acc, r,
                           wps);
        break;
    default:
        hipLaunchKernelGGL((srt_adj_kernel<TM_BOUNDS, CALIB, 12>), grid, b12, 0, s, P, gp, acc, r,
                           wps);
        break;
    }
}

hipError_t launch_srt_adj(const Problem &P, const float *gp, double *acc, void *img,
                          int img_dtype, hipStream_t s)
{
    adj_launch<false>(P, gp, acc, nullptr, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_adj_gather(P, acc, img, img_dtype, s);
}

hipError_t launch_adj_calibrate(const Problem &P, float *r, hipStream_t s)
{
    adj_launch<true>(P, nullptr, nullptr, r, s);
    return hipGetLastError();
}

hipError_t launch_arc_build(const Problem &P, int mode, hipStream_t s)
{
    dim3 grid(P.nbx * P.nby * P.nbz), block(WAVES * WAVE);
    switch (mode) {
    case 0: hipLaunchKernelGGL(arc_build_kernel<WALK_COUNT>, grid, block, 0, s, P); break;
    case 1: hipLaunchKernelGGL(arc_build_kernel<WALK_FILL>, grid, block, 0, s, P); break;
    case 2: hipLaunchKernelGGL(arc_build_kernel<WALK_SEGCOUNT>, grid, block, 0, s, P); break;
    case 3: hipLaunchKernelGGL(arc_build_kernel<WALK_SEGFILL>, grid, block, 0, s, P); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace oat
