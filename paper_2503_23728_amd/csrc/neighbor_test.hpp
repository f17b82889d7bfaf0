// The neighbour membership test of a pair (shared by the neighbour-list
// kernels and the lane-per-centre kernels of small molecules, so both take
// the same decision bit for bit): float32 with one rounding per operation,
//   d  = x_w[j] - x_w[i]; d -= L rint(d invL)   (periodic beads)
//   r2 = (dx dx + dy dy) + dz dz;  a neighbour iff r2 < fl32(rc^2)
// on the wrapped positions (the raw ones without a box).
#pragma once

#include "device_common.hpp"

namespace pimd {

__device__ __forceinline__ bool within_cutoff(const float4 &pi, const float4 &pj, const BeadInfo &bi, float rc2)
{
#pragma clang fp contract(off)
    float dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
    if (bi.periodic) {
        const float sx = bi.L[0] * rintf(dx * bi.invL[0]);
        const float sy = bi.L[1] * rintf(dy * bi.invL[1]);
        const float sz = bi.L[2] * rintf(dz * bi.invL[2]);
        dx = dx - sx;
        dy = dy - sy;
        dz = dz - sz;
    }
    const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
    const float r2 = (xx + yy) + zz;
    return r2 < rc2;
}

}  // namespace pimd
