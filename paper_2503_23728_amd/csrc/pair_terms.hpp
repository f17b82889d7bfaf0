// Pair terms shared by the per-centre kernels of the energy model and of the
// direct-force head: the displacement of a neighbour pair and the cutoff
// function with its derivative.
#pragma once

#include "device_common.hpp"

namespace pimd {

constexpr float kLog2e = 1.4426950408889634f;

// exp2 on the hardware transcendental unit (about 1 ulp).  The pair terms
// take exp(-eta x^2) as exp2_hw(-eta kLog2e x^2): the float32 rounding of the
// argument already costs ~1e-7 |a| relative, and the library exp's range
// reduction (a dozen instructions per call, 16 calls per slot in the radial
// terms) buys no accuracy beyond that.
__device__ __forceinline__ float exp2_hw(float a) { return __builtin_amdgcn_exp2f(a); }

// Displacement d_ij = q_j - q_i (minimum image) of the unwrapped float32
// positions, formed in FP64 with the FP64 box and rounded once to float32, so
// it carries no rounding from wrapping large coordinates.  The neighbour set
// itself comes from the float32 test of the neighbour kernel; for |d| < rc <
// L/2 the minimum image is unique, so both choose the same image.
// r = r_f + r_lo without an FP64 square root or division: r_f is the float32
// square root of r^2 (rounded), and the residual e = r^2 - r_f^2 is exact in
// FP64 (r_f^2 has 48 significant bits and the two terms are within a factor 2
// of each other), so r = r_f + e/(2 r_f) up to e^2/(8 r_f^3) ~ 1e-14 r; r_lo
// is that correction in float32.  1/r is the float32 reciprocal of r_f after
// one Newton step on r_f + r_lo (as accurate as the rounded FP64 quotient in a
// float32 emulation).
__device__ __forceinline__ void displacement(const float4 &pi, const float4 &pj, const BeadInfo &bi, float3 &d,
                                             float &r, float &r_lo, float &inv_r)
{
    double dx = (double)pj.x - (double)pi.x, dy = (double)pj.y - (double)pi.y, dz = (double)pj.z - (double)pi.z;
    if (bi.periodic) {
        dx -= bi.L64[0] * rint(dx * bi.invL64[0]);
        dy -= bi.L64[1] * rint(dy * bi.invL64[1]);
        dz -= bi.L64[2] * rint(dz * bi.invL64[2]);
    }
    const double r2 = dx * dx + dy * dy + dz * dz;
    const float rf = __builtin_amdgcn_sqrtf((float)r2);
    const double e = fma(-(double)rf, (double)rf, r2);
    const float inv = __builtin_amdgcn_rcpf(rf);
    d = make_float3((float)dx, (float)dy, (float)dz);
    r = rf;
    r_lo = (float)e * (0.5f * inv);
    const float t = fmaf(-rf, inv, 1.0f) - r_lo * inv;
    inv_r = fmaf(inv, t, inv);
}

// Cutoff function and derivative from x = r/rc in [0, 1):
//   f_c = (cos(pi x) + 1)/2 = cos^2(pi x/2),  f_c' = -(pi/rc) sin(pi x/2) cos(pi x/2).
// sin and cos of pi u (u = x/2) come from their Taylor series on the reduced
// argument w = min(u, 1/2 - u) <= 1/4 (five and six terms: truncation below
// 3e-8); the reflection keeps both relative-accurate, so f_c has no
// cancellation near the cutoff.
__device__ __forceinline__ void cutoff_fn(float x, float pi_over_rc, float &fc, float &dfc)
{
    const float u = 0.5f * x;
    const float w = fminf(u, 0.5f - u);
    const float t = 3.14159265358979f * w;
    const float t2 = t * t;
    float ps = 2.7557319224e-06f;
    ps = fmaf(ps, t2, -1.9841269841e-04f);
    ps = fmaf(ps, t2, 8.3333333333e-03f);
    ps = fmaf(ps, t2, -1.6666666667e-01f);
    ps = fmaf(ps, t2, 1.0f);
    ps *= t;
    float pc = -2.7557319224e-07f;
    pc = fmaf(pc, t2, 2.4801587302e-05f);
    pc = fmaf(pc, t2, -1.3888888889e-03f);
    pc = fmaf(pc, t2, 4.1666666667e-02f);
    pc = fmaf(pc, t2, -0.5f);
    pc = fmaf(pc, t2, 1.0f);
    const bool big = u > 0.25f;
    const float sn = big ? pc : ps, cs = big ? ps : pc;
    fc = cs * cs;
    dfc = -pi_over_rc * sn * cs;
}

// Cutoff function of u = (r/rc)^2 in [0, 1], for the triplet terms, which
// have r^2 and no other use for r:
//   f_c = (cos(pi r/rc) + 1)/2 = c^2,  c(u) = cos(pi sqrt(u)/2),
//   d f_c/du = 2 c c',  (1/r) d f_c/dr = 2 (d f_c/du)/rc^2.
// c(u) = sum_n (-1)^n (pi^2/4)^n u^n/(2n)! is an entire function of u; its
// Taylor polynomials of degree 6 (c) and 5 (c') leave alternating remainders
// below 7e-9 and 5e-8 on [0, 1], under the ~1e-7 absolute rounding of the
// float32 sums.  No square root and no argument reduction.
__device__ __forceinline__ float cutoff_sq_c(float u)
{
    float c = 4.7108747788e-07f;
    c = fmaf(c, u, -2.5202042373e-05f);
    c = fmaf(c, u, 9.1926027484e-04f);
    c = fmaf(c, u, -2.0863480763e-02f);
    c = fmaf(c, u, 2.5366950790e-01f);
    c = fmaf(c, u, -1.2337005501e+00f);
    return fmaf(c, u, 1.0f);
}

__device__ __forceinline__ float cutoff_sq_fc(float u)
{
    const float c = cutoff_sq_c(u);
    return c * c;
}

__device__ __forceinline__ void cutoff_sq(float u, float &fc, float &dfc_du)
{
    const float c = cutoff_sq_c(u);
    float d = 2.8265248673e-06f;
    d = fmaf(d, u, -1.2601021187e-04f);
    d = fmaf(d, u, 3.6770410994e-03f);
    d = fmaf(d, u, -6.2590442290e-02f);
    d = fmaf(d, u, 5.0733901580e-01f);
    d = fmaf(d, u, -1.2337005501e+00f);
    fc = c * c;
    dfc_du = 2.0f * c * d;
}

}  // namespace pimd
