// Ring-polymer propagation in normal modes with the PILE-L thermostat
// (Sec. 2.1: normal-mode transformation of the ring polymer; Table S3:
// PILE-L), or PILE-G (a global thermostat on the centroid, below), split as
// O(dt/2) B(dt/2) A(dt) [forces] B(dt/2) O(dt/2).
//
// A workgroup owns `ncol` columns (atom, xyz) of one system and P threads per
// column.  The P bead values of each column are staged in LDS; thread k of a
// column forms normal mode k as the real discrete Fourier sum with twiddles
// cos(2 pi m/P), sin(2 pi m/P) (m = jk mod P) from a 2P-entry table in LDS
// and the normalisations 1/sqrt(P), sqrt(2/P), applies the O/B/A updates of
// that mode, and the inverse transform is the same sum over k for bead j.
// For P <= 128 the direct sum costs little arithmetic next to the loads, and
// the table keeps what each workgroup stages at 2P + 2 values instead of a
// P x P matrix.  The state is float32 in memory; the transforms, the
// O/B/A updates and their coefficients are FP64 in registers, because float32
// coefficients (C not orthogonal, cos^2 + sin^2 != 1 at the 1e-7 level) change
// the ring-polymer energy by a fixed amount every step, a drift that grows as
// dt shrinks.
//
//   O: p~_k <- c1_k p~_k + sqrt(m) sig_T c2_k xi,   (kinetic-energy change -> heat bath)
//   B: p~_k <- p~_k + dt/2 F~_k / MVV2E
//   A: k = 0: q~ += dt p~/m;  k > 0: exact rotation at w_k in (q~, p~/(m w_k)).
// Noise xi: Philox4x32-10, counter (row of (system, mode k, atom), half, step),
// unless the caller injected a buffer.
#include "device_common.hpp"

namespace pimd {

struct IntegArgs {
    float *q, *p;
    float *q_prev, *p_prev;   // the state at the start of the step in progress
    const uint32_t *status;   // device status word: nonzero freezes the integrator
    const float *F;
    const SysInfo *sys;
    const ModeInfo *modes;
    const IntegUnit *units;
    const double *cmat;
    const float *mass_atom;
    const int64_t *step;
    double *dke_part;
    const float *xi;     // injected noise [2][B][3] or null
    const double *svr;   // PILE-G: per-system factor of the centroid momenta for this half step, else null
    int B;
    float dt;
    uint32_t key0, key1;
};

__device__ __forceinline__ float noise_value(const IntegArgs &a, int half, int64_t row, int comp, int64_t step)
{
    if (a.xi)
        return a.xi[((int64_t)half * a.B + row) * 3 + comp];
    return thermostat_normal(a.key0, a.key1, step, half, row, comp);
}

__device__ double block_sum_double(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = blockDim.x >> 1; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o)
            red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    return red[0];
}

// Staging coordinates of one column (bead values v[0..P-1], index k = l - 1):
//   u_k = v_k - (k v_{k+1} + v_0) / (k + 1)  (k >= 1, v_P = v_0),  u_0 = v_0;
//   force on u_k:  k = 0: sum_j F_j;  k >= 1: (1/k) sum_{j=1..k} j F_j
//   (the chain rule through the inverse, written out);
//   inverse:  v_0 = u_0,  v_j = u_0 + j sum_{k=j..P-1} u_k / k  (j >= 1).
__device__ __forceinline__ double staging_u(const double *v, int k, int P)
{
    return k == 0 ? v[0] : v[k] - ((double)k * v[(k + 1) % P] + v[0]) / (double)(k + 1);
}

__device__ __forceinline__ double staging_force(const double *f, int k, int P)
{
    double a = 0.0;
    if (k == 0) {
        for (int j = 0; j < P; ++j)
            a += f[j];
        return a;
    }
    for (int j = 1; j <= k; ++j)
        a += (double)j * f[j];
    return a / (double)k;
}

__device__ __forceinline__ double staging_r(const double *u, int j, int P)
{
    if (j == 0)
        return u[0];
    double a = 0.0;
    for (int k = j; k < P; ++k)
        a += u[k] / (double)k;
    return u[0] + (double)j * a;
}

// Coordinates of the integrator: normal modes, staging, or primitive
// (Cartesian beads, springs as forces: -m w_P^2 (2 q_k - q_{k+1} - q_{k-1})).
enum { kNormalModes = 0, kStaging = 1, kPrimitive = 2 };

__device__ __forceinline__ double spring_force(const double *q, int k, int P, double m_w2)
{
    return P == 1 ? 0.0 : -m_w2 * kMvv2e * (2.0 * q[k] - q[(k + 1) % P] - q[(k + P - 1) % P]);
}

// LDS (doubles): tw[2P + 2] (cos, sin, 1/sqrt(P), sqrt(2/P)) | s0[256] | s1[256] | s2[256] | red[256]
// (staging and primitive leave tw unused: their transforms are closed forms.)
template <bool PRE, int XF>
__global__ __launch_bounds__(256) void k_integrate(IntegArgs a)
{
    constexpr bool STAGING = XF == kStaging, PRIMITIVE = XF == kPrimitive, NM = XF == kNormalModes;
    extern __shared__ double ism[];
    // Units of neighbouring columns share cache lines of q, p and F (a column
    // reads one float per bead row); workgroups go round-robin over the 8 XCDs,
    // each with its own L2, so the unit index is remapped to give every XCD a
    // contiguous run of units.
    const int ui = xcd_block(blockIdx.x, gridDim.x);
    const IntegUnit u = a.units[ui];
    const SysInfo S = a.sys[u.sys];
    const int P = S.P, N = S.N;
    double *tw = ism;
    double *s0 = tw + 2 * P + 2;
    double *s1 = s0 + 256;
    double *s2 = s1 + 256;
    double *red = s2 + 256;
    const int tid = threadIdx.x;
    const int cl = tid / P, kk = tid - cl * P;
    const bool valid = cl < u.ncol;
    const int col = u.col0 + cl;
    const int atom = col / 3, cc = col - 3 * (col / 3);
    const int64_t row = (int64_t)S.ba0 + (int64_t)kk * N + atom;   // bead kk (loads) = mode kk (noise)
    // A latched fault (neighbour overflow, non-finite value) freezes the state
    // at the last step that completed without one: the pre-force half does
    // nothing, the post-force half puts back the state the step started from.
    // The status word is only written by kernels of earlier stages, so every
    // thread of the launch reads the same value.
    if (*a.status != 0u) {
        if (!PRE && valid) {
            a.q[row * 3 + cc] = a.q_prev[row * 3 + cc];
            a.p[row * 3 + cc] = a.p_prev[row * 3 + cc];
        }
        return;
    }
    if (NM)
        for (int idx = tid; idx < 2 * P + 2; idx += 256)
            tw[idx] = a.cmat[S.cmat0 + idx];
    // normal-mode matrix C[j][k] = nrm_k * (k <= P/2 ? cos : sin)(2 pi (jk mod P)/P),
    // nrm_k = 1/sqrt(P) for k = 0 and P/2, sqrt(2/P) otherwise
    const int halfP = P / 2;
    const int64_t step = *a.step;
    double m = 1.0;
    if (valid) {
        m = (double)a.mass_atom[S.atom0 + atom];
        const float pv = a.p[row * 3 + cc];
        s0[tid] = (double)pv;
        s1[tid] = (double)a.F[row * 3 + cc];
        if (PRE || PRIMITIVE) {
            const float qv = a.q[row * 3 + cc];
            s2[tid] = (double)qv;
            if (PRE) {
                a.q_prev[row * 3 + cc] = qv;
                a.p_prev[row * 3 + cc] = pv;
            }
        }
    }
    __syncthreads();
    const double kick = 0.5 * (double)a.dt / kMvv2e;
    double dke = 0.0;
    double pt = 0.0, qt = 0.0;
    // Twiddles by rotation: (x, y) turns by the angle 2 pi kk / P per term,
    // whose cos and sin the table holds correctly rounded (exact at quarter
    // turns); the recurrence adds ~1e-16 per step, ~P 1e-16 in all, where a
    // table read per term and thread (each lane a different address) cost
    // more LDS bandwidth than the four FP64 operations of a turn.
    const double Cw = NM ? tw[kk] : 1.0, Sw = NM ? tw[P + kk] : 0.0;
    if (valid) {
        const double nrm = (kk == 0 || kk == halfP) ? tw[2 * P] : tw[2 * P + 1];
        // mode kk takes cos(j theta) (kk <= P/2) or sin(j theta) = cos(j theta - pi/2)
        const double x0 = kk > halfP ? 0.0 : 1.0, y0 = kk > halfP ? -1.0 : 0.0;
        const double *sp = s0 + cl * P, *sf = s1 + cl * P, *sq = s2 + cl * P;
        const ModeInfo M = a.modes[S.mode0 + kk];
        const double mk = m * M.mfac;                 // kinetic mass of mode kk
        const double sig = sqrt(mk) * (double)S.sig_T;
        if (PRE) {
            double Ft = 0.0;
            if (STAGING) {
                pt = sp[kk];                          // the state holds staging momenta
                Ft = staging_force(sf, kk, P);
                qt = staging_u(sq, kk, P);
            } else if (PRIMITIVE) {
                pt = sp[kk];
                Ft = sf[kk] + spring_force(sq, kk, P, m * M.w * M.w);
                qt = sq[kk];
            } else {
                double x = x0, y = y0;
                for (int j = 0; j < P; ++j) {
                    pt += x * sp[j];
                    Ft += x * sf[j];
                    qt += x * sq[j];
                    const double xn = x * Cw - y * Sw;
                    y = y * Cw + x * Sw;
                    x = xn;
                }
                pt *= nrm;
                Ft *= nrm;
                qt *= nrm;
            }
            // O(dt/2), half 0 (PILE-G: the centroid takes the global factor instead)
            const double xi = (double)noise_value(a, 0, row, cc, step);
            const double pn = (NM && a.svr && kk == 0) ? a.svr[u.sys] * pt : M.c1 * pt + sig * M.c2 * xi;
            dke = 0.5 * (pn * pn - pt * pt) / mk * kMvv2e;
            pt = pn + kick * Ft;  // B(dt/2)
            // A(dt)
            if (kk == 0 || PRIMITIVE) {
                qt += (double)a.dt * pt / mk;
            } else {
                const double mw = mk * M.w;
                const double qn = M.sw * pt / mw + M.cw * qt;
                const double pn2 = M.cw * pt - mw * M.sw * qt;
                qt = qn;
                pt = pn2;
            }
        } else {
            // B(dt/2), then O(dt/2) in modes
            if (STAGING) {
                pt = sp[kk] + kick * staging_force(sf, kk, P);
            } else if (PRIMITIVE) {
                pt = sp[kk] + kick * (sf[kk] + spring_force(sq, kk, P, m * M.w * M.w));
            } else {
                double x = x0, y = y0;
                for (int j = 0; j < P; ++j) {
                    pt += x * (sp[j] + kick * sf[j]);
                    const double xn = x * Cw - y * Sw;
                    y = y * Cw + x * Sw;
                    x = xn;
                }
                pt *= nrm;
            }
            const double xi = (double)noise_value(a, 1, row, cc, step);
            const double pn = (NM && a.svr && kk == 0) ? a.svr[u.sys] * pt : M.c1 * pt + sig * M.c2 * xi;
            dke = 0.5 * (pn * pn - pt * pt) / mk * kMvv2e;
            pt = pn;
        }
    }
    __syncthreads();
    if (valid) {
        s0[tid] = pt;
        if (PRE)
            s2[tid] = qt;
    }
    __syncthreads();
    if (valid) {
        const double *sp = s0 + cl * P, *sq = s2 + cl * P;
        double pj = 0.0, qj = 0.0;
        if (STAGING) {
            pj = pt;
            if (PRE)
                qj = staging_r(sq, kk, P);
        } else if (PRIMITIVE) {
            pj = pt;
            qj = qt;
        } else {
            // back to beads: x_j = sum_k C[j][k] x~_k, with j = kk: (x, y) =
            // (cos k phi, sin k phi), phi = 2 pi j / P; cos up to k = P/2, sin
            // above, normalisation 1/sqrt(P) at k = 0 and P/2, sqrt(2/P) between
            const double n0 = tw[2 * P], n1 = tw[2 * P + 1];
            double x = 1.0, y = 0.0;
            auto term = [&](double c, int k) {
                pj += c * sp[k];
                if (PRE)
                    qj += c * sq[k];
                const double xn = x * Cw - y * Sw;
                y = y * Cw + x * Sw;
                x = xn;
            };
            term(n0, 0);
            for (int k = 1; k < halfP; ++k)
                term(n1 * x, k);
            if (P > 1)
                term(n0 * x, halfP);
            for (int k = halfP + 1; k < P; ++k)
                term(n1 * y, k);
        }
        a.p[row * 3 + cc] = (float)pj;
        if (PRE)
            a.q[row * 3 + cc] = (float)qj;
    }
    const double tot = block_sum_double(dke, red);
    if (tid == 0)
        a.dke_part[2 * ui + (PRE ? 0 : 1)] = tot;
}

// PILE-G: the centroid mode of every system is thermostatted by one factor
// per half step, the stochastic velocity rescaling of Bussi, Donadio and
// Parrinello (J. Chem. Phys. 126, 014101 (2007), Appendix), while the other
// modes keep their Langevin friction.  With N_f = 3N, the centroid kinetic
// energy K (of p~_0 = sum_j p_j / sqrt(P), after the force kick in the second
// half), Kbar = N_f k_B T P / 2 and c = exp(-(dt/2)/tau0):
//   alpha^2 = c + (Kbar/(N_f K))(1 - c)(R_1^2 + S) + 2 R_1 sqrt(c (1 - c) Kbar/(N_f K)),
//   sign(alpha) = sign(R_1 + sqrt(c N_f K / ((1 - c) Kbar))),
// R_1 the centroid normal of (atom 0, x) and S the sum of squares of its other
// 3N - 1 normals, so the random numbers are those of the thermostat's own
// counters (or the injected buffer).
// k_centroid_terms: per integrator unit, one thread per column: K and sum xi^2
// of its columns, tree-summed in FP64 -> part[2 unit], part[2 unit + 1].
template <bool PRE>
__global__ __launch_bounds__(256) void k_centroid_terms(IntegArgs a, double *__restrict__ part)
{
    __shared__ double red[256];
    const IntegUnit u = a.units[blockIdx.x];
    const SysInfo S = a.sys[u.sys];
    const int tid = threadIdx.x;
    const int64_t step = *a.step;
    const double kick = 0.5 * (double)a.dt / kMvv2e;
    double ke = 0.0, x2 = 0.0;
    for (int cl = tid; cl < u.ncol; cl += 256) {
        const int col = u.col0 + cl;
        const int atom = col / 3, cc = col - 3 * atom;
        double sum = 0.0;
        for (int j = 0; j < S.P; ++j) {
            const int64_t r = (int64_t)S.ba0 + (int64_t)j * S.N + atom;
            sum += (double)a.p[r * 3 + cc];
            if (!PRE)
                sum += kick * (double)a.F[r * 3 + cc];
        }
        const double m = (double)a.mass_atom[S.atom0 + atom];
        ke += 0.5 * kMvv2e * sum * sum / ((double)S.P * m);
        const double xi = (double)noise_value(a, PRE ? 0 : 1, (int64_t)S.ba0 + atom, cc, step);
        x2 += xi * xi;
    }
    const double kt = block_sum_double(ke, red);
    __syncthreads();
    const double xt = block_sum_double(x2, red);
    if (tid == 0) {
        part[2 * blockIdx.x] = kt;
        part[2 * blockIdx.x + 1] = xt;
    }
}

// k_svr_alpha: one workgroup per system: its units' terms summed in a fixed
// order, then alpha (alpha = 1 when K = 0: no direction to rescale).
template <bool PRE>
__global__ __launch_bounds__(256) void k_svr_alpha(IntegArgs a, const double *__restrict__ part,
                                                   const double *__restrict__ kbar, double c, double *__restrict__ alpha)
{
    __shared__ double red[256];
    const SysInfo S = a.sys[blockIdx.x];
    double ke = 0.0, x2 = 0.0;
    for (int u = S.unit0 + threadIdx.x; u < S.unit0 + S.nunit; u += 256) {
        ke += part[2 * u];
        x2 += part[2 * u + 1];
    }
    const double K = block_sum_double(ke, red);
    __syncthreads();
    const double X = block_sum_double(x2, red);
    if (threadIdx.x == 0) {
        double f = 1.0;
        if (K > 0.0) {
            const double nf = 3.0 * (double)S.N;
            const double r1 = (double)noise_value(a, PRE ? 0 : 1, (int64_t)S.ba0, 0, *a.step);
            const double rest = X - r1 * r1;
            const double ratio = kbar[blockIdx.x] / (nf * K);
            const double a2 = c + ratio * (1.0 - c) * (r1 * r1 + rest) + 2.0 * r1 * sqrt(c * (1.0 - c) * ratio);
            f = sqrt(a2);
            if (r1 + sqrt(c / ((1.0 - c) * ratio)) < 0.0)
                f = -f;
        }
        alpha[blockIdx.x] = f;
    }
}

// heat_bath[s] -= (sum of O-step kinetic-energy changes of the step); step += 1.
// One workgroup per system; fixed-order tree sum in FP64.
// Nothing while a fault is latched (the step did not complete).
__global__ __launch_bounds__(256) void k_finish_step(const SysInfo *__restrict__ sys,
                                                     const double *__restrict__ dke_part, double *__restrict__ heat,
                                                     int64_t *__restrict__ step, const uint32_t *__restrict__ status)
{
    __shared__ double red[256];
    if (*status != 0u)
        return;
    const SysInfo S = sys[blockIdx.x];
    double d = 0.0;
    for (int u = S.unit0 + threadIdx.x; u < S.unit0 + S.nunit; u += 256)
        d += dke_part[2 * u] + dke_part[2 * u + 1];
    const double tot = block_sum_double(d, red);
    if (threadIdx.x == 0) {
        heat[blockIdx.x] -= tot;
        if (blockIdx.x == 0)
            step[0] += 1;
    }
}

// Estimator terms per column (atom, xyz) of every system:
// [0] m sum_k (q_{k+1} - q_k)^2, [1] sum_k (q_k - qbar) F_k, [2] sum_k p_k^2 / (m mfac_k)
__global__ __launch_bounds__(256) void k_estimator_terms(const float *__restrict__ q, const float *__restrict__ p,
                                                         const float *__restrict__ F, const SysInfo *__restrict__ sys,
                                                         const ModeInfo *__restrict__ modes,
                                                         const int32_t *__restrict__ col_sys,
                                                         const float *__restrict__ mass_atom,
                                                         float *__restrict__ out, int ncol)
{
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= ncol)
        return;
    const SysInfo S = sys[col_sys[col]];
    const int gatom = col / 3, cc = col - 3 * gatom;
    const int atom = gatom - S.atom0;
    const float m = mass_atom[gatom];
    float qbar = 0.0f;
    for (int k = 0; k < S.P; ++k)
        qbar += q[((int64_t)S.ba0 + (int64_t)k * S.N + atom) * 3 + cc];
    qbar /= (float)S.P;
    float spring = 0.0f, cv = 0.0f, ke = 0.0f;
    for (int k = 0; k < S.P; ++k) {
        const int64_t r = (int64_t)S.ba0 + (int64_t)k * S.N + atom;
        const int64_t rn = (int64_t)S.ba0 + (int64_t)((k + 1) % S.P) * S.N + atom;
        const float qk = q[r * 3 + cc];
        const float dq = q[rn * 3 + cc] - qk;
        spring += dq * dq;
        cv += (qk - qbar) * F[r * 3 + cc];
        const float pk = p[r * 3 + cc];
        ke += pk * pk / (float)modes[S.mode0 + k].mfac;   // kinetic mass of the slot's momentum
    }
    out[3 * (int64_t)col + 0] = m * spring;
    out[3 * (int64_t)col + 1] = cv;
    out[3 * (int64_t)col + 2] = ke / m;
}

// Isotropic harmonic well V = 1/2 m w^2 |q|^2 per atom (the oscillator of Sec. S1).
__global__ __launch_bounds__(256) void k_harmonic(const float *__restrict__ q, const BeadInfo *__restrict__ beads,
                                                  const int32_t *__restrict__ bead_of_ba,
                                                  const SysInfo *__restrict__ sys,
                                                  const float *__restrict__ mass_atom, float w2_mvv2e,
                                                  float *__restrict__ E_atom, float *__restrict__ F,
                                                  float *__restrict__ vir_atom, int B)
{
    const int ba = blockIdx.x * blockDim.x + threadIdx.x;
    if (ba >= B)
        return;
    const BeadInfo bi = beads[bead_of_ba[ba]];
    const float m = mass_atom[sys[bi.sys].atom0 + (ba - bi.ba0)];
    const float k = m * w2_mvv2e;
    const float x = q[3 * ba], y = q[3 * ba + 1], z = q[3 * ba + 2];
    E_atom[ba] = 0.5f * k * (x * x + y * y + z * z);
    const float f[3] = {-k * x, -k * y, -k * z};
    if (F) {
        F[3 * ba] = f[0];
        F[3 * ba + 1] = f[1];
        F[3 * ba + 2] = f[2];
    }
    const float r[3] = {x, y, z};
    for (int a2 = 0; a2 < 3; ++a2)
        for (int b2 = 0; b2 < 3; ++b2)
            vir_atom[9 * (int64_t)ba + 3 * a2 + b2] = r[a2] * f[b2];
}

__global__ void k_philox_words(uint32_t k0, uint32_t k1, int64_t step, int half, int64_t n, uint32_t *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n)
        return;
    const uint4 w = philox4x32_10(make_uint4((uint32_t)t, (uint32_t)half, (uint32_t)step,
                                             (uint32_t)((uint64_t)step >> 32)), k0, k1);
    out[4 * t + 0] = w.x;
    out[4 * t + 1] = w.y;
    out[4 * t + 2] = w.z;
    out[4 * t + 3] = w.w;
}

__global__ void k_check_finite(const float *a, int64_t n, uint32_t *status)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n && !isfinite(a[t]))
        atomicOr(status, kStatusNonFinite);
}

static IntegArgs integ_args(const DevBuffers &d, const Sizes &z, float dt, uint32_t k0, uint32_t k1, const float *xi)
{
    IntegArgs a;
    a.svr = d.svr_alpha;
    a.q = d.q;
    a.p = d.p;
    a.q_prev = d.q_prev;
    a.p_prev = d.p_prev;
    a.status = d.status;
    a.F = d.F;
    a.sys = d.sys;
    a.modes = d.modes;
    a.units = d.units;
    a.cmat = d.cmat;
    a.mass_atom = d.mass_atom;
    a.step = d.step;
    a.dke_part = d.dke_part;
    a.xi = xi;
    a.B = z.B;
    a.dt = dt;
    a.key0 = k0;
    a.key1 = k1;
    return a;
}

static size_t integ_lds(int max_P)
{
    return ((size_t)2 * max_P + 2 + 4 * 256) * sizeof(double);
}

size_t integrator_lds_bytes(int max_P) { return integ_lds(max_P); }

hipError_t configure_integrator_lds(int max_P)
{
    const int b = (int)integ_lds(max_P);
    hipError_t e = hipSuccess;
    for (const void *f : {(const void *)k_integrate<true, kNormalModes>, (const void *)k_integrate<false, kNormalModes>,
                          (const void *)k_integrate<true, kStaging>, (const void *)k_integrate<false, kStaging>,
                          (const void *)k_integrate<true, kPrimitive>, (const void *)k_integrate<false, kPrimitive>})
        if (e == hipSuccess)
            e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    return e;
}

template <bool PRE>
static void launch_integrate(const DevBuffers &d, const Sizes &z, float dt, uint32_t k0, uint32_t k1, const float *xi,
                             int max_P, int transform, double svr_c, hipStream_t s)
{
    const IntegArgs args = integ_args(d, z, dt, k0, k1, xi);
    const size_t lds = integ_lds(max_P);
    if (d.svr_alpha && transform == kNormalModes) {
        hipLaunchKernelGGL(k_centroid_terms<PRE>, dim3(z.n_units), dim3(256), 0, s, args, d.svr_part);
        hipLaunchKernelGGL(k_svr_alpha<PRE>, dim3(z.n_sys), dim3(256), 0, s, args, d.svr_part, d.svr_kbar, svr_c,
                           d.svr_alpha);
    }
    if (transform == kStaging)
        hipLaunchKernelGGL((k_integrate<PRE, kStaging>), dim3(z.n_units), dim3(256), lds, s, args);
    else if (transform == kPrimitive)
        hipLaunchKernelGGL((k_integrate<PRE, kPrimitive>), dim3(z.n_units), dim3(256), lds, s, args);
    else
        hipLaunchKernelGGL((k_integrate<PRE, kNormalModes>), dim3(z.n_units), dim3(256), lds, s, args);
}

void launch_integrate_pre(const DevBuffers &d, const Sizes &z, float dt, uint32_t k0, uint32_t k1, const float *xi,
                          int max_P, int transform, double svr_c, hipStream_t s)
{
    launch_integrate<true>(d, z, dt, k0, k1, xi, max_P, transform, svr_c, s);
}

void launch_integrate_post(const DevBuffers &d, const Sizes &z, float dt, uint32_t k0, uint32_t k1, const float *xi,
                           int max_P, int transform, double svr_c, hipStream_t s)
{
    launch_integrate<false>(d, z, dt, k0, k1, xi, max_P, transform, svr_c, s);
}

void launch_finish_step(const DevBuffers &d, const Sizes &z, hipStream_t s)
{
    hipLaunchKernelGGL(k_finish_step, dim3(z.n_sys), dim3(256), 0, s, d.sys, d.dke_part, d.heat, d.step, d.status);
}

void launch_estimator_terms(const DevBuffers &d, const Sizes &z, hipStream_t s)
{
    hipLaunchKernelGGL(k_estimator_terms, dim3((z.ncol + 255) / 256), dim3(256), 0, s, d.q, d.p, d.F, d.sys,
                       d.modes, d.col_sys, d.mass_atom, d.est_cols, z.ncol);
}

void launch_harmonic(const float *q, const DevBuffers &d, const Sizes &z, float w2_mvv2e, float *F, hipStream_t s)
{
    hipLaunchKernelGGL(k_harmonic, dim3((z.B + 255) / 256), dim3(256), 0, s, q, d.beads, d.bead_of_ba, d.sys,
                       d.mass_atom, w2_mvv2e, d.E_atom, F, d.vir_atom, z.B);
}

void launch_philox_words(uint32_t k0, uint32_t k1, int64_t step, int half, int64_t n, uint32_t *out, hipStream_t s)
{
    if (n <= 0)
        return;
    hipLaunchKernelGGL(k_philox_words, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, k0, k1, step, half, n,
                       out);
}

void launch_check_finite(const float *a, int64_t n, uint32_t *status, hipStream_t s)
{
    if (n <= 0)
        return;
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, n, status);
}

}  // namespace pimd
