// Well-tempered metadynamics on bead collective variables (Sec. 2.5).
//
// Every bead carries its own hills; per force evaluation:
//   k_xrd_rows     (XRD CV only) one workgroup per 256-row tile of a bead:
//                  row sums f_i sum_j f_j sinc(Q R_ij) and gradients dS/dq_i,
//                  every ordered pair of the bead (the all-pairs sum of the
//                  Sec. 3.2 CV), j staged through LDS 256 rows at a time
//   k_metad_bias   one workgroup per bead: the CV (row sums reduced, or the
//                  distance terms), the bias and its slope from the bead's
//                  hills, the deposition of a new hill, the bias forces
//   k_metad_advance  one thread: the shared hill count after a deposition
//
// Arithmetic of the XRD sum is FP64 throughout (geometry, the phase x = Q R,
// its quarter-period reduction with Cody and Waite's two-part constant, sin
// and cos as Taylor polynomials on |t| <= pi/4, the sums): FP64 adds,
// multiplies and FMAs issue at the non-packed float32 rate on this chip, and a
// float32 phase of a pair 40 A apart carries ~4e-6 rad of rounding, which
// over ~1e4 partners moves S by more than 1e-7 of itself -- a large error
// against hill widths of a few hundredths of S.  Only the seed of 1/r is a
// float32 hardware reciprocal square root, refined by two Newton steps.
#include "device_common.hpp"

namespace pimd {
namespace {

constexpr int kXrdBlock = 256;

// sin and cos of t, |t| <= pi/4, in FP64 (Taylor series to t^17 and t^18:
// truncation below 2e-17).
__device__ __forceinline__ void sincos_reduced(double t, double &sn, double &cs)
{
    const double t2 = t * t;
    double ps = 1.0 / 355687428096000.0;            //  1/17!
    ps = fma(ps, t2, -1.0 / 1307674368000.0);       // -1/15!
    ps = fma(ps, t2, 1.0 / 6227020800.0);           //  1/13!
    ps = fma(ps, t2, -1.0 / 39916800.0);            // -1/11!
    ps = fma(ps, t2, 1.0 / 362880.0);               //  1/9!
    ps = fma(ps, t2, -1.0 / 5040.0);                // -1/7!
    ps = fma(ps, t2, 1.0 / 120.0);                  //  1/5!
    ps = fma(ps, t2, -1.0 / 6.0);                   // -1/3!
    sn = fma(ps * t2, t, t);
    double pc = -1.0 / 6402373705728000.0;          // -1/18!
    pc = fma(pc, t2, 1.0 / 20922789888000.0);       //  1/16!
    pc = fma(pc, t2, -1.0 / 87178291200.0);         // -1/14!
    pc = fma(pc, t2, 1.0 / 479001600.0);            //  1/12!
    pc = fma(pc, t2, -1.0 / 3628800.0);             // -1/10!
    pc = fma(pc, t2, 1.0 / 40320.0);                //  1/8!
    pc = fma(pc, t2, -1.0 / 720.0);                 // -1/6!
    pc = fma(pc, t2, 1.0 / 24.0);                   //  1/4!
    pc = fma(pc, t2, -0.5);
    cs = fma(pc, t2, 1.0);
}

// sin(x), cos(x) of x >= 0: x = n pi/2 + t with the two-part constant of
// Cody and Waite, then the quadrant n mod 4 permutes and signs (sin t, cos t).
__device__ __forceinline__ void sincos_phase(double x, double &sn, double &cs)
{
    constexpr double kTwoOverPi = 0.63661977236758134308;
    constexpr double kHalfPiHi = 1.5707963267948966;         // fl64(pi/2)
    constexpr double kHalfPiLo = 6.123233995736766e-17;      // pi/2 - fl64(pi/2)
    const double n = rint(x * kTwoOverPi);
    const double t = fma(-n, kHalfPiLo, fma(-n, kHalfPiHi, x));
    double ps, pc;
    sincos_reduced(t, ps, pc);
    const int k = (int)n;
    const bool swap = k & 1;
    const double s0 = swap ? pc : ps, c0 = swap ? ps : pc;
    sn = (k & 2) ? -s0 : s0;
    cs = ((k + 1) & 2) ? -c0 : c0;
}

// Positions of one staged partner: FP64 coordinates and its form factor.
struct Partner {
    double x, y, z, f;
};

template <bool PERIODIC>
__global__ __launch_bounds__(256) void k_xrd_rows(const float *__restrict__ q, const BeadInfo *__restrict__ beads,
                                                  const SysInfo *__restrict__ sys,
                                                  const int32_t *__restrict__ species_atom,
                                                  const int2 *__restrict__ tiles, MetadParams mp,
                                                  double *__restrict__ row_out, float *__restrict__ grad_out)
{
    __shared__ Partner part[kXrdBlock];
    const int2 tile = tiles[blockIdx.x];
    const BeadInfo bi = beads[tile.x];
    const int n = bi.n;
    const int atom0 = sys[bi.sys].atom0;
    const int li = tile.y + (int)threadIdx.x;
    const bool active = li < n;
    double xi = 0, yi = 0, zi = 0, fi = 0;
    if (active) {
        const int64_t r = (int64_t)bi.ba0 + li;
        xi = q[3 * r + 0];
        yi = q[3 * r + 1];
        zi = q[3 * r + 2];
        fi = mp.form_factor[species_atom[atom0 + li]];
    }
    const double Q = mp.q_scatter;
    const double invQ = 1.0 / Q;
    double S = 0, gx = 0, gy = 0, gz = 0;
    for (int j0 = 0; j0 < n; j0 += kXrdBlock) {
        __syncthreads();
        const int lj = j0 + (int)threadIdx.x;
        if (lj < n) {
            const int64_t r = (int64_t)bi.ba0 + lj;
            Partner pj;
            pj.x = q[3 * r + 0];
            pj.y = q[3 * r + 1];
            pj.z = q[3 * r + 2];
            pj.f = mp.form_factor[species_atom[atom0 + lj]];
            part[threadIdx.x] = pj;
        }
        __syncthreads();
        const int nj = min(kXrdBlock, n - j0);
        for (int jj = 0; jj < nj; ++jj) {
            const Partner pj = part[jj];
            double dx = xi - pj.x, dy = yi - pj.y, dz = zi - pj.z;
            if (PERIODIC && bi.periodic) {
                dx -= bi.L64[0] * rint(dx * bi.invL64[0]);
                dy -= bi.L64[1] * rint(dy * bi.invL64[1]);
                dz -= bi.L64[2] * rint(dz * bi.invL64[2]);
            }
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            // i = j (or coincident atoms): sinc(0) = 1 and no gradient; the
            // arithmetic below runs on r2 = 1 so it stays finite.
            const bool self = r2 == 0.0;
            const double r2s = self ? 1.0 : r2;
            // 1/r: float32 estimate (hardware reciprocal square root; r2 is a
            // normal number) and two Newton steps (relative error ~1e-16)
            double y = (double)__builtin_amdgcn_rsqf((float)r2s);
            y = y * fma(-0.5 * r2s, y * y, 1.5);
            y = y * fma(-0.5 * r2s, y * y, 1.5);
            const double x = Q * (r2s * y);
            double sn, cs;
            sincos_phase(x, sn, cs);
            const double f = pj.f;
            const double sc = self ? 1.0 : sn * (y * invQ);
            // dS/dq_i term: f_j Q sinc'(x) d/r with sinc'(x) = (cos x - sinc x)/x,
            // i.e. f_j (cos x - sinc x) d / r^2
            S = fma(f, sc, S);
            const double w = f * (cs - sc) * (y * y);
            gx = fma(w, dx, gx);
            gy = fma(w, dy, gy);
            gz = fma(w, dz, gz);
        }
    }
    if (active) {
        const int64_t r = (int64_t)bi.ba0 + li;
        row_out[r] = fi * S;
        const double c = 2.0 * fi / (double)n;
        grad_out[3 * r + 0] = (float)(c * gx);
        grad_out[3 * r + 1] = (float)(c * gy);
        grad_out[3 * r + 2] = (float)(c * gz);
    }
}

// Deterministic sum over the 256 threads of a workgroup (fixed tree).
__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum_f64(v);
    const int w = threadIdx.x / kWave;
    __syncthreads();
    if (lane_id() == 0)
        red[w] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

__device__ __forceinline__ void min_image(double &dx, double &dy, double &dz, const BeadInfo &bi)
{
    if (bi.periodic) {
        dx -= bi.L64[0] * rint(dx * bi.invL64[0]);
        dy -= bi.L64[1] * rint(dy * bi.invL64[1]);
        dz -= bi.L64[2] * rint(dz * bi.invL64[2]);
    }
}

__global__ __launch_bounds__(256) void k_metad_bias(const float *__restrict__ q, const BeadInfo *__restrict__ beads,
                                                    const double *__restrict__ xrd_row,
                                                    const float *__restrict__ xrd_grad,
                                                    const int32_t *__restrict__ cv_atoms,
                                                    const double *__restrict__ cv_coef,
                                                    const double *__restrict__ wt_scale, MetadParams mp,
                                                    double2 *__restrict__ hills,
                                                    const int32_t *__restrict__ n_hills_p,
                                                    const int64_t *__restrict__ step, int deposit,
                                                    double *__restrict__ cv_out, double *__restrict__ v_out,
                                                    float *__restrict__ F, int add, uint32_t *__restrict__ status)
{
    __shared__ double red[4];
    const int bead = blockIdx.x;
    const BeadInfo bi = beads[bead];
    const int n = bi.n;
    const int tid = threadIdx.x;
    // 1. the CV of the bead
    double part = 0.0;
    if (mp.cv == 2) {
        for (int i = tid; i < n; i += 256)
            part += xrd_row[(int64_t)bi.ba0 + i];
    } else if (tid < mp.n_terms) {
        const int64_t a = (int64_t)bi.ba0 + cv_atoms[2 * tid], b = (int64_t)bi.ba0 + cv_atoms[2 * tid + 1];
        double dx = (double)q[3 * a] - (double)q[3 * b], dy = (double)q[3 * a + 1] - (double)q[3 * b + 1],
               dz = (double)q[3 * a + 2] - (double)q[3 * b + 2];
        min_image(dx, dy, dz, bi);
        part = cv_coef[tid] * sqrt(dx * dx + dy * dy + dz * dz);
    }
    double s = block_sum(part, red);
    if (mp.cv == 2)
        s /= (double)n;
    // 2. bias and slope from the bead's hills
    const int nh = *n_hills_p;
    const double2 *hb = hills + (int64_t)bead * mp.max_hills;
    double v = 0.0, dv = 0.0;
    for (int h = tid; h < nh; h += 256) {
        const double2 c = hb[h];
        const double x = (s - c.x) * mp.inv_sigma;
        const double g = c.y * exp(-0.5 * x * x);
        v += g;
        dv -= g * x;
    }
    v = block_sum(v, red);
    dv = block_sum(dv, red) * mp.inv_sigma;
    if (tid == 0) {
        if (cv_out)
            cv_out[bead] = s;
        if (v_out)
            v_out[bead] = v;
        // 3. deposition after every stride-th completed step (step counts the
        //    steps completed before the one in progress)
        if (deposit && (*step + 1) % mp.stride == 0) {
            if (nh < mp.max_hills)
                hills[(int64_t)bead * mp.max_hills + nh] = make_double2(s, mp.height0 * exp(-v * wt_scale[bi.sys]));
            else
                atomicOr(status, kStatusHills);
        }
    }
    // 4. bias forces F = -dV/ds ds/dq on the bead's atoms
    if (!F)
        return;
    const int64_t r0 = bi.ba0;
    if (mp.cv == 2) {
        for (int i = tid; i < n; i += 256) {
            const int64_t r = r0 + i;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float fb = (float)(-dv * (double)xrd_grad[3 * r + c]);
                F[3 * r + c] = add ? F[3 * r + c] + fb : fb;
            }
        }
        return;
    }
    if (!add) {
        for (int i = tid; i < 3 * n; i += 256)
            F[3 * r0 + i] = 0.f;
    }
    __syncthreads();
    if (tid == 0) {
        // one thread walks the terms: several terms may share an atom
        for (int m = 0; m < mp.n_terms; ++m) {
            const int64_t a = r0 + cv_atoms[2 * m], b = r0 + cv_atoms[2 * m + 1];
            double d[3] = {(double)q[3 * a] - (double)q[3 * b], (double)q[3 * a + 1] - (double)q[3 * b + 1],
                           (double)q[3 * a + 2] - (double)q[3 * b + 2]};
            min_image(d[0], d[1], d[2], bi);
            const double k = -dv * cv_coef[m] / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            for (int c = 0; c < 3; ++c) {
                const float fa = (float)(k * d[c]);
                F[3 * a + c] += fa;
                F[3 * b + c] -= fa;
            }
        }
    }
}

__global__ void k_metad_advance(const int64_t *__restrict__ step, int stride, int max_hills,
                                int32_t *__restrict__ n_hills)
{
    if (threadIdx.x == 0 && blockIdx.x == 0 && (*step + 1) % stride == 0 && *n_hills < max_hills)
        *n_hills += 1;
}

// Quantum free energy on a grid (Sec. 2.5 reweighting), one thread per grid
// point: F^(k)(s) = -gamma_ratio V^(k)(s), gamma_ratio = gamma/(gamma-1),
// F(s) = -kT ln[(1/P) sum_k exp(-F^(k)/kT)], summed as a running
// log-sum-exp (m the smallest F^(k) so far, acc = sum_k exp(-(F^(k) - m)/kT)).
__global__ __launch_bounds__(256) void k_metad_fes(const double2 *__restrict__ hills,
                                                   const int32_t *__restrict__ n_hills_p, int max_hills,
                                                   int bead0, int P, double inv_sigma, double kT,
                                                   double gamma_ratio, const double *__restrict__ grid, int n_grid,
                                                   double *__restrict__ out)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_grid)
        return;
    const double s = grid[g];
    const int nh = *n_hills_p;
    double m = 0.0, acc = 0.0;
    for (int k = 0; k < P; ++k) {
        const double2 *hb = hills + (int64_t)(bead0 + k) * max_hills;
        double v = 0.0;
        for (int h = 0; h < nh; ++h) {
            const double x = (s - hb[h].x) * inv_sigma;
            v += hb[h].y * exp(-0.5 * x * x);
        }
        const double Fk = -gamma_ratio * v;
        if (k == 0) {
            m = Fk;
            acc = 1.0;
        } else if (Fk < m) {
            acc = acc * exp(-(m - Fk) / kT) + 1.0;
            m = Fk;
        } else {
            acc += exp(-(Fk - m) / kT);
        }
    }
    out[g] = m - kT * log(acc / P);
}

}  // namespace

void launch_metad(const float *q, const DevBuffers &d, const Sizes &z, const MetadParams &mp, int n_xrd_tiles,
                  float *F, int add, int deposit, double *cv_out, double *v_out, hipStream_t s)
{
    if (mp.cv == 2) {
        if (z.any_box)
            hipLaunchKernelGGL(k_xrd_rows<true>, dim3(n_xrd_tiles), dim3(256), 0, s, q, d.beads, d.sys,
                               d.species_atom, d.xrd_tiles, mp, d.xrd_row, d.xrd_grad);
        else
            hipLaunchKernelGGL(k_xrd_rows<false>, dim3(n_xrd_tiles), dim3(256), 0, s, q, d.beads, d.sys,
                               d.species_atom, d.xrd_tiles, mp, d.xrd_row, d.xrd_grad);
    }
    hipLaunchKernelGGL(k_metad_bias, dim3(z.n_beads_total), dim3(256), 0, s, q, d.beads, d.xrd_row, d.xrd_grad,
                       d.cv_atoms, d.cv_coef, d.wt_scale, mp, d.hills, d.n_hills, d.step, deposit, cv_out, v_out, F,
                       add, d.status);
}

void launch_metad_advance(const DevBuffers &d, const MetadParams &mp, hipStream_t s)
{
    hipLaunchKernelGGL(k_metad_advance, dim3(1), dim3(64), 0, s, d.step, mp.stride, mp.max_hills, d.n_hills);
}

void launch_metad_fes(const DevBuffers &d, const MetadParams &mp, int bead0, int P, double kT, double gamma_ratio,
                      const double *grid, int n_grid, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_metad_fes, dim3((n_grid + 255) / 256), dim3(256), 0, s, d.hills, d.n_hills, mp.max_hills,
                       bead0, P, mp.inv_sigma, kT, gamma_ratio, grid, n_grid, out);
}

}  // namespace pimd
