// Well-tempered metadynamics on bead collective variables (Sec. 2.5).
//
// Every bead carries its own hills; per force evaluation:
//   k_xrd_pairs    (XRD CV only) the all-pairs sum of the Sec. 3.2 CV, one
//                  workgroup per pair of row tiles of a bead, each pair of
//                  atoms evaluated once for both of its rows
//   k_xrd_reduce   row sums f_i sum_j f_j sinc(Q R_ij) and gradients dS/dq_i
//                  from the per-tile partials, in a fixed order
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

// One pair (i, j) of the XRD sum: sinc(Q r_ij) and base = (cos x - sinc x) / r^2
// (the gradient term of row i is f_j base d, of row j -f_i base d, with
// d = q_i - q_j; sinc'(x) Q / r = (cos x - sinc x) / r^2).  i = j (or
// coincident atoms): sinc = 1 and the arithmetic runs on r^2 = 1 so it stays
// finite (d = 0 carries no gradient).
template <bool PERIODIC>
__device__ __forceinline__ void xrd_pair(double xi, double yi, double zi, double xj, double yj, double zj,
                                         const BeadInfo &bi, double Q, double invQ, double &sc, double &base,
                                         double &dx, double &dy, double &dz)
{
    dx = xi - xj;
    dy = yi - yj;
    dz = zi - zj;
    if (PERIODIC && bi.periodic) {
        dx -= bi.L64[0] * rint(dx * bi.invL64[0]);
        dy -= bi.L64[1] * rint(dy * bi.invL64[1]);
        dz -= bi.L64[2] * rint(dz * bi.invL64[2]);
    }
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const bool self = r2 == 0.0;
    const double r2s = self ? 1.0 : r2;
    // 1/r: float32 estimate (hardware reciprocal square root; r2 is a normal
    // number) and two Newton steps (relative error ~1e-16)
    double y = (double)__builtin_amdgcn_rsqf((float)r2s);
    y = y * fma(-0.5 * r2s, y * y, 1.5);
    y = y * fma(-0.5 * r2s, y * y, 1.5);
    const double x = Q * (r2s * y);
    double sn, cs;
    sincos_phase(x, sn, cs);
    sc = self ? 1.0 : sn * (y * invQ);
    base = (cs - sc) * (y * y);
}

// Pair sum over tiles of T = 64 W rows: one workgroup per work item (bead,
// tiles I <= J).  I = J: every ordered pair of the tile, into the rows.
// I < J: every pair once; row i of tile I accumulates in registers, row j of
// tile J in LDS.  In phase ph, wave w owns the 64 columns of block
// (w + ph) mod W, and at step k lane l takes column (l + k) mod 64 of it, so
// no two lanes (or waves) touch one column accumulator at a time.  Each item
// writes one partial (sum_j f_j sinc, gradient sum) per row and partner tile:
// part[part0 + partner * n + row].
template <int W, bool PERIODIC>
__global__ __launch_bounds__(64 * W) void k_xrd_pairs(const float *__restrict__ q,
                                                      const BeadInfo *__restrict__ beads,
                                                      const SysInfo *__restrict__ sys,
                                                      const int32_t *__restrict__ species_atom,
                                                      const int4 *__restrict__ items, MetadParams mp,
                                                      double4 *__restrict__ part)
{
    constexpr int T = 64 * W;
    __shared__ double cx[T], cy[T], cz[T], cf[T];
    __shared__ double aS[T], ax[T], ay[T], az[T];
    const int4 it = items[blockIdx.x];
    const BeadInfo bi = beads[it.x];
    const int n = bi.n, I = it.y, J = it.z;
    const int64_t p0 = it.w;
    const int atom0 = sys[bi.sys].atom0;
    const int tid = threadIdx.x;
    const int li = I * T + tid, lj = J * T + tid;
    double xi = 0, yi = 0, zi = 0, fi = 0;
    if (li < n) {
        const int64_t r = (int64_t)bi.ba0 + li;
        xi = q[3 * r + 0];
        yi = q[3 * r + 1];
        zi = q[3 * r + 2];
        fi = mp.form_factor[species_atom[atom0 + li]];
    }
    {
        // rows past the end stage as f = 0 at the origin: their pairs add nothing
        double x = 0, y = 0, z = 0, f = 0;
        if (lj < n) {
            const int64_t r = (int64_t)bi.ba0 + lj;
            x = q[3 * r + 0];
            y = q[3 * r + 1];
            z = q[3 * r + 2];
            f = mp.form_factor[species_atom[atom0 + lj]];
        }
        cx[tid] = x;
        cy[tid] = y;
        cz[tid] = z;
        cf[tid] = f;
        aS[tid] = 0.0;
        ax[tid] = 0.0;
        ay[tid] = 0.0;
        az[tid] = 0.0;
    }
    __syncthreads();
    const double Q = mp.q_scatter, invQ = 1.0 / Q;
    double S = 0, gx = 0, gy = 0, gz = 0;
    double sc, base, dx, dy, dz;
    if (I == J) {
        for (int jj = 0; jj < T; ++jj) {
            const double fj = cf[jj];
            xrd_pair<PERIODIC>(xi, yi, zi, cx[jj], cy[jj], cz[jj], bi, Q, invQ, sc, base, dx, dy, dz);
            S = fma(fj, sc, S);
            const double wj = fj * base;
            gx = fma(wj, dx, gx);
            gy = fma(wj, dy, gy);
            gz = fma(wj, dz, gz);
        }
    } else {
        const int w = tid >> 6, lane = tid & 63;
        for (int ph = 0; ph < W; ++ph) {
            const int blk = ((w + ph) % W) * 64;
            for (int k = 0; k < 64; ++k) {
                const int jj = blk + ((lane + k) & 63);
                const double fj = cf[jj];
                xrd_pair<PERIODIC>(xi, yi, zi, cx[jj], cy[jj], cz[jj], bi, Q, invQ, sc, base, dx, dy, dz);
                S = fma(fj, sc, S);
                const double wj = fj * base;
                gx = fma(wj, dx, gx);
                gy = fma(wj, dy, gy);
                gz = fma(wj, dz, gz);
                const double wi = -fi * base;
                aS[jj] = fma(fi, sc, aS[jj]);
                ax[jj] = fma(wi, dx, ax[jj]);
                ay[jj] = fma(wi, dy, ay[jj]);
                az[jj] = fma(wi, dz, az[jj]);
                wave_sync();    // the next step's lanes read what this step wrote
            }
            __syncthreads();    // the next phase hands this block to another wave
        }
    }
    if (li < n)
        part[p0 + (int64_t)J * n + li] = make_double4(S, gx, gy, gz);
    if (I != J && lj < n)
        part[p0 + (int64_t)I * n + lj] = make_double4(aS[tid], ax[tid], ay[tid], az[tid]);
}

// Row totals in fixed partner order: row_out = f_i sum_j f_j sinc(Q r_ij),
// grad_out = dS/dq_i = (2 f_i / n) sum_j f_j base_ij d_ij.
__global__ __launch_bounds__(256) void k_xrd_reduce(const BeadInfo *__restrict__ beads,
                                                    const int32_t *__restrict__ bead_of_ba,
                                                    const SysInfo *__restrict__ sys,
                                                    const int32_t *__restrict__ species_atom,
                                                    const int32_t *__restrict__ part0, int T, MetadParams mp,
                                                    const double4 *__restrict__ part, double *__restrict__ row_out,
                                                    float *__restrict__ grad_out, int B)
{
    const int ba = blockIdx.x * blockDim.x + threadIdx.x;
    if (ba >= B)
        return;
    const int bead = bead_of_ba[ba];
    const BeadInfo bi = beads[bead];
    const int a = ba - bi.ba0, n = bi.n;
    const int nt = (n + T - 1) / T;
    const double4 *pp = part + part0[bead] + a;
    double S = 0, gx = 0, gy = 0, gz = 0;
    for (int p = 0; p < nt; ++p) {
        const double4 v = pp[(int64_t)p * n];
        S += v.x;
        gx += v.y;
        gy += v.z;
        gz += v.w;
    }
    const double f = mp.form_factor[species_atom[sys[bi.sys].atom0 + a]];
    row_out[ba] = f * S;
    const double c = 2.0 * f / (double)n;
    grad_out[3 * (int64_t)ba + 0] = (float)(c * gx);
    grad_out[3 * (int64_t)ba + 1] = (float)(c * gy);
    grad_out[3 * (int64_t)ba + 2] = (float)(c * gz);
}

// Deterministic sum over the NT threads of a workgroup (fixed tree; one wave:
// the butterfly alone).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum_f64(v);
    if (NT == kWave)
        return v;
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

template <int NT>
__global__ __launch_bounds__(NT) void k_metad_bias(const float *__restrict__ q, const BeadInfo *__restrict__ beads,
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
        for (int i = tid; i < n; i += NT)
            part += xrd_row[(int64_t)bi.ba0 + i];
    } else if (tid < mp.n_terms) {
        const int64_t a = (int64_t)bi.ba0 + cv_atoms[2 * tid], b = (int64_t)bi.ba0 + cv_atoms[2 * tid + 1];
        double dx = (double)q[3 * a] - (double)q[3 * b], dy = (double)q[3 * a + 1] - (double)q[3 * b + 1],
               dz = (double)q[3 * a + 2] - (double)q[3 * b + 2];
        min_image(dx, dy, dz, bi);
        part = cv_coef[tid] * sqrt(dx * dx + dy * dy + dz * dz);
    }
    double s = block_sum<NT>(part, red);
    if (mp.cv == 2)
        s /= (double)n;
    // 2. bias and slope from the bead's hills
    const int nh = *n_hills_p;
    const double2 *hb = hills + (int64_t)bead * mp.max_hills;
    double v = 0.0, dv = 0.0;
    for (int h = tid; h < nh; h += NT) {
        const double2 c = hb[h];
        const double x = (s - c.x) * mp.inv_sigma;
        const double g = c.y * exp(-0.5 * x * x);
        v += g;
        dv -= g * x;
    }
    v = block_sum<NT>(v, red);
    dv = block_sum<NT>(dv, red) * mp.inv_sigma;
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
        for (int i = tid; i < n; i += NT) {
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
        for (int i = tid; i < 3 * n; i += NT)
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
                                int32_t *__restrict__ n_hills, const uint32_t *__restrict__ status)
{
    // a latched fault means the step does not complete: its hill is not kept
    if (threadIdx.x == 0 && blockIdx.x == 0 && *status == 0u && (*step + 1) % stride == 0 && *n_hills < max_hills)
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

void launch_metad(const float *q, const DevBuffers &d, const Sizes &z, const MetadParams &mp, int n_xrd_items,
                  float *F, int add, int deposit, double *cv_out, double *v_out, hipStream_t s)
{
    if (mp.cv == 2) {
        const dim3 g(n_xrd_items);
        if (mp.xrd_tile == 256) {
            if (z.any_box)
                hipLaunchKernelGGL((k_xrd_pairs<4, true>), g, dim3(256), 0, s, q, d.beads, d.sys, d.species_atom,
                                   d.xrd_items, mp, d.xrd_part);
            else
                hipLaunchKernelGGL((k_xrd_pairs<4, false>), g, dim3(256), 0, s, q, d.beads, d.sys, d.species_atom,
                                   d.xrd_items, mp, d.xrd_part);
        } else {
            if (z.any_box)
                hipLaunchKernelGGL((k_xrd_pairs<1, true>), g, dim3(64), 0, s, q, d.beads, d.sys, d.species_atom,
                                   d.xrd_items, mp, d.xrd_part);
            else
                hipLaunchKernelGGL((k_xrd_pairs<1, false>), g, dim3(64), 0, s, q, d.beads, d.sys, d.species_atom,
                                   d.xrd_items, mp, d.xrd_part);
        }
        hipLaunchKernelGGL(k_xrd_reduce, dim3((z.B + 255) / 256), dim3(256), 0, s, d.beads, d.bead_of_ba, d.sys,
                           d.species_atom, d.xrd_part0, mp.xrd_tile, mp, d.xrd_part, d.xrd_row, d.xrd_grad, z.B);
    }
    // the XRD CV reduces a bead's rows with 256 threads; a distance CV (<= 64
    // terms) needs one wave per bead
    if (mp.cv == 2)
        hipLaunchKernelGGL(k_metad_bias<256>, dim3(z.n_beads_total), dim3(256), 0, s, q, d.beads, d.xrd_row,
                           d.xrd_grad, d.cv_atoms, d.cv_coef, d.wt_scale, mp, d.hills, d.n_hills, d.step, deposit,
                           cv_out, v_out, F, add, d.status);
    else
        hipLaunchKernelGGL(k_metad_bias<64>, dim3(z.n_beads_total), dim3(64), 0, s, q, d.beads, d.xrd_row,
                           d.xrd_grad, d.cv_atoms, d.cv_coef, d.wt_scale, mp, d.hills, d.n_hills, d.step, deposit,
                           cv_out, v_out, F, add, d.status);
}

void launch_metad_advance(const DevBuffers &d, const MetadParams &mp, hipStream_t s)
{
    hipLaunchKernelGGL(k_metad_advance, dim3(1), dim3(64), 0, s, d.step, mp.stride, mp.max_hills, d.n_hills, d.status);
}

void launch_metad_fes(const DevBuffers &d, const MetadParams &mp, int bead0, int P, double kT, double gamma_ratio,
                      const double *grid, int n_grid, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_metad_fes, dim3((n_grid + 255) / 256), dim3(256), 0, s, d.hills, d.n_hills, mp.max_hills,
                       bead0, P, mp.inv_sigma, kT, gamma_ratio, grid, n_grid, out);
}

}  // namespace pimd
