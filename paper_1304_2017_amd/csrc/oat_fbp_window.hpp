// FBP's staged sample windows (Eq. (disfbp)), shared by the kernel, its
// launcher and the host check of the window bounds.
//
// A block takes a tile of FBP_TX x FBP_TY x FBP_TZ voxels.  For each
// transducer it stages the samples k in [k_lo, k_lo + win) of the data row,
// where k_lo is taken at the tile centre's distance dc (grid units) minus the
// tile's half-diagonal hd.  Every voxel of the tile lies within hd of the
// centre, so its kt = |r_n - r_q| sigma - tau (sigma = dx / (c0 dt),
// tau = t0 / dt) satisfies (dc - hd) sigma - tau <= kt <= (dc + hd) sigma - tau.
// With the floor decided as in the problem statement and the update reading
// samples floor(kt) and floor(kt) + 1, the margins (2 below, and the window
// 2 hd sigma + 6 long) keep floor(kt) - k_lo in 0 .. win - 2.
#pragma once

#include <math.h>

namespace oat {

constexpr int FBP_TX = 16, FBP_TY = 16, FBP_TZ = 8;

// Half the tile's diagonal in grid units.
__host__ __device__ inline float fbp_half_diag()
{
    return 0.5f * sqrtf((float)((FBP_TX - 1) * (FBP_TX - 1) + (FBP_TY - 1) * (FBP_TY - 1) +
                                (FBP_TZ - 1) * (FBP_TZ - 1)));
}

// Staged samples per (tile, transducer).
__host__ __device__ inline int fbp_window(float sigma)
{
    return (int)ceilf(2.f * fbp_half_diag() * sigma) + 6;
}

// First staged sample for a tile whose centre lies dc grid units from the
// transducer.
__host__ __device__ inline int fbp_first_sample(float dc, float sigma, float tau)
{
    return (int)floorf(fmaf(dc - fbp_half_diag(), sigma, -tau)) - 2;
}

}  // namespace oat
