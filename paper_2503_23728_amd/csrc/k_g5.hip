// G5 angular symmetry functions in O(K) per centre atom, and their adjoint.
//
//   G5[{e1,e2}, eta, zeta, lambda] = 2^(1-zeta) sum_{j<k, {Z_j,Z_k} = {e1,e2}}
//        (1 + lambda cos theta_jik)^zeta w_eta(r_ij) w_eta(r_ik),
//   w_eta(r) = exp(-eta r^2) f_c(r)
// (the G4 sum without the factors of r_jk; Behler-Parrinello descriptors,
// cited in the Introduction).  Without r_jk the double sum over neighbour
// pairs factorises.  With P_l the Legendre polynomials, (1 + lambda c)^zeta
// = sum_{l <= zeta} a_l^{zeta,lambda} P_l(c), and by the addition theorem
//   sum_{j in e1, k in e2} w_j w_k P_l(u_j . u_k) = sum_m c_m M_e1[lm] M_e2[lm],
//   M_e[lm] = sum_{j in e} w_j Y_lm(u_j),
// with real harmonics Y_lm(u) = q_l^m(z) (A_m, B_m)(x, y), A_m + i B_m =
// (x + i y)^m, q_l^m = sqrt((l-m)!/(l+m)!) times the associated Legendre
// function without its sin^m factor, c_0 = 1 and c_m = 2 for the cos and sin
// parts of m > 0.  For e1 = e2 the ordered double sum counts each pair twice
// and holds the j = k terms, so
//   G5 = 2^(1-zeta) sum_l a_l sum_m c_m (M_e[lm]^2 - R_e[lm]) / 2,  R_e[lm] = sum_{j in e} (w_j Y_lm(u_j))^2:
// subtracting the self terms harmonic by harmonic makes them cancel with the
// same roundings they entered with (subtracting the exact (1 + lambda)^zeta
// sum_j w_j^2 instead leaves a residue of the size of that sum).
// Per centre: 81 moments per (element, eta) instead of K^2/2 pair terms.
//
// Forward, one wave per centre, element by element: each lane takes one
// neighbour of a chunk of 64, evaluates its 81 harmonics by the upward
// recursion in l at fixed m and writes them to LDS; then each lane takes one
// harmonic and sums w_eta Y and (w_eta Y)^2 over the chunk's neighbours in
// FP64 (the features are differences of these sums: in FP32 they lose
// about 1e-5 of the features' scale).  The moments go to memory, rounded to
// float, for the adjoint.
//
// Adjoint: dE/dM_e[lm] = c_m sum_e' H_l(e, e') M_e'[lm] with
// H_l(e, e') = sum_{zeta,lambda} dE/dG[{e,e'}] 2^(1-zeta) a_l.  Each
// neighbour slot j then gets its vector dE/dd_ij from its own lane: the
// gradient of sum_eta w_eta(r) sum_lm g_lm Y_lm(d/r) with
// g_lm = dE/dM_e[lm] - c_m H_l(e, e) w_eta Y_lm(u_j) (the derivative of the R
// term), the harmonics differentiated as polynomials in (x, y, z) and
// projected on the plane normal to u.  No triplets, no atomics: every slot is
// written by one lane.
#include "device_common.hpp"
#include "pair_terms.hpp"

namespace pimd {

constexpr int kG5L = 8;                       // (1 +- cos)^zeta, zeta <= 8
constexpr int kG5Y = (kG5L + 1) * (kG5L + 1);  // real harmonics up to l = 8
constexpr int kG5Lm = (kG5L + 1) * (kG5L + 2) / 2;  // (l, m >= 0) pairs
constexpr int kChunk = 64;                     // neighbours per pass (one per lane)
constexpr int kRowStride = 68;                 // chunk buffer row: 64 slots + 4 (16-byte rows, banks spread)

// Harmonic index of (l, m, part): part 0 is the cos (m = 0: the only) part.
__host__ __device__ constexpr int g5_index(int l, int m, int part) { return l * l + (m == 0 ? 0 : 2 * m - 1 + part); }

// Walks the harmonics of the unit vector (x, y, z) in the order m = 0..8,
// l = m..8, calling f(l, m, q, dq, A_m, B_m, A_{m-1}, B_{m-1}) with q = q_l^m(z)
// and dq its z derivative.  Recursion at fixed m:
//   q_m^m = q_{m-1}^{m-1} sqrt((2m - 1)/(2m)),  q_{m+1}^m = sqrt(2m + 1) z q_m^m,
//   q_l^m = ((2l - 1) z q_{l-1}^m - sqrt((l-1)^2 - m^2) q_{l-2}^m) / sqrt(l^2 - m^2).
// The loops unroll completely, so every coefficient is a folded constant.
template <typename F>
__device__ __forceinline__ void for_each_harmonic(float x, float y, float z, F &&f)
{
    float A = 1.0f, Bs = 0.0f, Ap = 0.0f, Bp = 0.0f, qmm = 1.0f;
#pragma unroll
    for (int m = 0; m <= kG5L; ++m) {
        if (m > 0) {
            const float An = x * A - y * Bs, Bn = x * Bs + y * A;
            Ap = A;
            Bp = Bs;
            A = An;
            Bs = Bn;
            qmm *= (float)__builtin_sqrt((2.0 * m - 1.0) / (2.0 * m));
        }
        float q1 = 0.0f, q2 = 0.0f, d1 = 0.0f, d2 = 0.0f;
#pragma unroll
        for (int l = m; l <= kG5L; ++l) {
            float q, dq;
            if (l == m) {
                q = qmm;
                dq = 0.0f;
            } else if (l == m + 1) {
                const float c = (float)__builtin_sqrt(2.0 * m + 1.0);
                q = c * z * qmm;
                dq = c * qmm;
            } else {
                const float a = (float)((2.0 * l - 1.0) / __builtin_sqrt((double)(l * l - m * m)));
                const float b = (float)__builtin_sqrt((double)((l - 1) * (l - 1) - m * m) / (double)(l * l - m * m));
                q = fmaf(a * z, q1, -b * q2);
                dq = fmaf(a, fmaf(z, d1, q1), -b * d2);
            }
            q2 = q1;
            d2 = d1;
            q1 = q;
            d1 = dq;
            f(l, m, q, dq, A, Bs, Ap, Bp);
        }
    }
}

__device__ __forceinline__ int pair_of(int e1, int e2, int n_el)
{
    const int a = e1 < e2 ? e1 : e2, b = e1 < e2 ? e2 : e1;
    return a * n_el - a * (a - 1) / 2 + (b - a);
}

__device__ __forceinline__ void pair_elements(int pair, int n_el, int &e1, int &e2)
{
    e1 = 0;
    while (pair >= n_el - e1) {
        pair -= n_el - e1;
        ++e1;
    }
    e2 = e1 + pair;
}

// LDS bytes per wave of the forward kernel: the 64-row float chunk buffer,
// the chunk's w_eta as doubles, the FP64 moments of every element, the FP64
// power spectra and the feature row.
__host__ __device__ inline size_t g5_forward_wave_bytes(const DescParams &dp)
{
    const int n_pairs = dp.n_el * (dp.n_el + 1) / 2;
    const size_t b = (size_t)64 * kRowStride * 4 + (size_t)kChunk * 16 + (size_t)dp.n_el * dp.n_ang_eta * kG5Y * 8 +
                     (size_t)n_pairs * dp.n_ang_eta * 9 * 8 + (size_t)((dp.D + 3) & ~3) * 4;
    return (b + 15) & ~(size_t)15;
}

// Floats of LDS per wave of the adjoint: dE/dG, H and dE/dM (float2 per (l, m)).
__host__ __device__ inline size_t g5_adjoint_wave_floats(const DescParams &dp)
{
    const int n_pairs = dp.n_el * (dp.n_el + 1) / 2;
    const size_t h = ((size_t)n_pairs * dp.n_ang_eta * 9 + 3) & ~(size_t)3;
    return (size_t)((dp.D + 3) & ~3) + h + (size_t)dp.n_el * dp.n_ang_eta * 2 * kG5Lm;
}

// ---------------------------------------------------------------------------
// forward: xhat[i][D] and the moments mom[i][e][eta][kG5Mom] (float)
// ---------------------------------------------------------------------------
template <int NETA>
__global__ __launch_bounds__(256) void k_descriptors_g5(const float4 *__restrict__ posu,
                                                        const BeadInfo *__restrict__ beads,
                                                        const int32_t *__restrict__ bead_of_ba,
                                                        const int32_t *__restrict__ order,
                                                        const int32_t *__restrict__ nbr,
                                                        const int32_t *__restrict__ nbr_cnt,
                                                        const int32_t *__restrict__ nbr_grp,
                                                        const float *__restrict__ norm, DescParams dp,
                                                        float *__restrict__ xhat, float *__restrict__ mom, int B)
{
    extern __shared__ double ldsd[];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int n_pairs = dp.n_el * (dp.n_el + 1) / 2;
    char *base = reinterpret_cast<char *>(ldsd) + w * g5_forward_wave_bytes(dp);
    float *buf = reinterpret_cast<float *>(base);                         // [row][kRowStride]: row = harmonic, col = slot
    double2 *wt = reinterpret_cast<double2 *>(base + 64 * kRowStride * 4);  // [64] (w_0, w_1)
    double *Ms = reinterpret_cast<double *>(wt + kChunk);                 // [e][eta][81]
    double *Pw = Ms + dp.n_el * NETA * kG5Y;                              // [pair][eta][l]
    float *Gs = reinterpret_cast<float *>(Pw + n_pairs * NETA * (kG5L + 1));
    double *Rs = reinterpret_cast<double *>(buf);   // [eta][81] of the current element, once its chunks are done
    const int Frad = dp.n_el * dp.n_rad;
    const int s_rad = kG5Y - 64;                    // second-pass rows: harmonics 64..80, then radial
    const float inv_rc = 1.0f / dp.rc;

    // sums over the chunk's slots of row `lane`: M += w y, R += (w y)^2 in FP64
    // (slots past the chunk's end carry w = 0 and finite y), four slots per read
    auto accumulate = [&](int cnt, double (&M)[NETA], double (&R)[NETA], float &rsum) {
        const float *rowp = buf + lane * kRowStride;
#pragma unroll 2
        for (int s0 = 0; s0 < cnt; s0 += 4) {
            const float4 y4 = *reinterpret_cast<const float4 *>(rowp + s0);
            const float ys[4] = {y4.x, y4.y, y4.z, y4.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double2 ww = wt[s0 + k];
                const double y = (double)ys[k];
                const double a = ww.x * y;
                M[0] += a;
                R[0] = fma(a, a, R[0]);
                if (NETA > 1) {
                    const double c = ww.y * y;
                    M[NETA - 1] += c;
                    R[NETA - 1] = fma(c, c, R[NETA - 1]);
                }
                rsum += ys[k];
            }
        }
    };

    const CentreRange cr = centre_range(B);
    for (int ci = cr.begin; ci < cr.end; ++ci) {
        const int i = __builtin_amdgcn_readfirstlane(order ? order[ci] : ci);
        const BeadInfo bi = beads[bead_of_ba[i]];
        const float4 pi = posu[i];
        const int zi = __float_as_int(pi.w);
        const int32_t *row = nbr + (int64_t)i * dp.Kmax;
        int lo = 0;
        for (int e = 0; e < dp.n_el; ++e) {
            // the slots of element e: [lo, hi) (keys sorted by element)
            const int hi = lo + nbr_grp[(int64_t)i * kMaxElements + e];
            double M1[NETA], R1[NETA], M2[NETA], R2[NETA];
#pragma unroll
            for (int ie = 0; ie < NETA; ++ie)
                M1[ie] = R1[ie] = M2[ie] = R2[ie] = 0.0;
            float rac = 0.0f, unused = 0.0f;
            for (int c0 = lo; c0 < hi; c0 += kChunk) {
                const int n = c0 + lane, cnt = hi - c0 < kChunk ? hi - c0 : kChunk;
                float3 d = make_float3(0.0f, 0.0f, 1.0f);
                float r = 1.0f, r_lo = 0.0f, inv_r = 1.0f, fc = 0.0f, dfc = 0.0f;
                if (n < hi) {
                    displacement(pi, posu[row[n] & (int)kRowMask], bi, d, r, r_lo, inv_r);
                    cutoff_fn(r * inv_rc, dp.pi_over_rc, fc, dfc);
                }
                float wv[NETA];
#pragma unroll
                for (int ie = 0; ie < NETA; ++ie)
                    wv[ie] = expf(-dp.ang_eta[ie] * r * r) * fc;
                wt[lane] = make_double2((double)wv[0], (double)wv[NETA - 1]);
                // harmonics 0..63 straight to the buffer (row = harmonic, column = slot)
                float Yh[kG5Y - 64];
                float *col = buf + lane;
                for_each_harmonic(d.x * inv_r, d.y * inv_r, d.z * inv_r,
                                  [&](int l, int m, float q, float, float A, float Bs, float, float) {
                                      const int t0 = g5_index(l, m, 0), t1 = g5_index(l, m, 1);
                                      if (t0 < 64)
                                          col[t0 * kRowStride] = q * A;
                                      else
                                          Yh[t0 - 64] = q * A;
                                      if (m > 0) {
                                          if (t1 < 64)
                                              col[t1 * kRowStride] = q * Bs;
                                          else
                                              Yh[t1 - 64] = q * Bs;
                                      }
                                  });
                wave_sync();
                accumulate(cnt, M1, R1, unused);
                wave_sync();
                // pass 2: harmonics 64..80 and the radial functions of the element
#pragma unroll
                for (int t = 0; t < kG5Y - 64; ++t)
                    col[t * kRowStride] = Yh[t];
                for (int q = 0; q < dp.n_rad; ++q) {
                    // r - R_s from the two-float r and R_s (the steep Gaussians would
                    // turn the float rounding of r into 1e-6 relative errors)
                    const float x = (r - dp.rad_center[q]) + (r_lo - dp.rad_center_lo[q]);
                    col[(s_rad + q) * kRowStride] = expf(-dp.rad_eta[q] * x * x) * fc;
                }
                wave_sync();
                accumulate(cnt, M2, R2, rac);
                wave_sync();
            }
            // moments of element e; its own power spectrum without the j = k
            // terms, sum_m c_m (M^2 - R), so the diagonal cancels term by term
#pragma unroll
            for (int ie = 0; ie < NETA; ++ie) {
                double *me = Ms + (e * NETA + ie) * kG5Y;
                me[lane] = M1[ie];
                Rs[ie * kG5Y + lane] = R1[ie];
                if (lane < kG5Y - 64) {
                    me[64 + lane] = M2[ie];
                    Rs[ie * kG5Y + 64 + lane] = R2[ie];
                }
            }
            if (lane >= s_rad && lane < s_rad + dp.n_rad)
                Gs[e * dp.n_rad + (lane - s_rad)] = rac;
            wave_sync();
            if (lane < NETA * (kG5L + 1)) {
                const int ie = lane / (kG5L + 1), l = lane - ie * (kG5L + 1);
                const double *me = Ms + (e * NETA + ie) * kG5Y + l * l;
                const double *re = Rs + ie * kG5Y + l * l;
                double p = 0.0;
                for (int k = 1; k <= 2 * l; ++k)
                    p += me[k] * me[k] - re[k];
                Pw[(pair_of(e, e, dp.n_el) * NETA + ie) * (kG5L + 1) + l] = 2.0 * p + (me[0] * me[0] - re[0]);
            }
            wave_sync();
            lo = hi;
        }
        // power spectra of the mixed pairs, p = sum_m c_m M_e1 M_e2
        for (int t = lane; t < n_pairs * NETA * (kG5L + 1); t += kWave) {
            const int l = t % (kG5L + 1), pe = t / (kG5L + 1);
            const int ie = pe % NETA, pair = pe / NETA;
            int e1, e2;
            pair_elements(pair, dp.n_el, e1, e2);
            if (e1 == e2)
                continue;
            const double *m1 = Ms + (e1 * NETA + ie) * kG5Y + l * l, *m2 = Ms + (e2 * NETA + ie) * kG5Y + l * l;
            double p = 0.0;
            for (int k = 1; k <= 2 * l; ++k)
                p = fma(m1[k], m2[k], p);
            Pw[t] = fma(m1[0], m2[0], 2.0 * p);
        }
        wave_sync();
        // features (pair, eta, zeta, lambda) = sum_l 2^(1-zeta) a_l (+-1)^l p_l, halved for e1 = e2
        for (int f = lane; f < n_pairs * dp.n_ang; f += kWave) {
            const int pair = f / dp.n_ang, qf = f - pair * dp.n_ang;
            const int ie = qf >> 3, iz = (qf >> 1) & 3, il = qf & 1;
            const double *p = Pw + (pair * NETA + ie) * (kG5L + 1);
            double v = 0.0;
#pragma unroll
            for (int l = 0; l <= kG5L; ++l)
                v = fma((double)dp.g5_leg[iz][l] * ((il && (l & 1)) ? -1.0 : 1.0), p[l], v);
            int e1, e2;
            pair_elements(pair, dp.n_el, e1, e2);
            Gs[Frad + f] = (float)(e1 == e2 ? 0.5 * v : v);
        }
        float *mo = mom + (int64_t)i * dp.n_el * NETA * kG5Mom;
        for (int t = lane; t < dp.n_el * NETA * kG5Mom; t += kWave) {
            const int ee = t / kG5Mom, k = t - ee * kG5Mom;
            mo[t] = k < kG5Y ? (float)Ms[ee * kG5Y + k] : 0.0f;
        }
        wave_sync();
        const float *shift = norm + (int64_t)zi * 2 * dp.D;
        const float *inv_scale = shift + dp.D;
        for (int f = lane; f < dp.D; f += kWave)
            xhat[(int64_t)i * dp.D + f] = (Gs[f] - shift[f]) * inv_scale[f];
        wave_sync();
    }
}

// ---------------------------------------------------------------------------
// adjoint: v[i][slot] = dE/d d_{i, slot}; per-atom virial -sum d (x) v
// ---------------------------------------------------------------------------
template <int NETA>
__global__ __launch_bounds__(256) void k_adjoint_g5(const float4 *__restrict__ posu, const BeadInfo *__restrict__ beads,
                                                    const int32_t *__restrict__ bead_of_ba,
                                                    const int32_t *__restrict__ order, const int32_t *__restrict__ nbr,
                                                    const int32_t *__restrict__ nbr_cnt,
                                                    const float *__restrict__ dEdG, const float *__restrict__ mom,
                                                    const int32_t *__restrict__ fence, DescParams dp,
                                                    float4 *__restrict__ vslot, float4 *__restrict__ vrev,
                                                    float *__restrict__ vir_atom, uint32_t *__restrict__ status,
                                                    int B)
{
    extern __shared__ float lds[];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int n_pairs = dp.n_el * (dp.n_el + 1) / 2;
    float *gl = lds + w * g5_adjoint_wave_floats(dp);
    float *H = gl + ((dp.D + 3) & ~3);                                              // [pair][eta][l]
    float2 *gM = reinterpret_cast<float2 *>(H + ((n_pairs * NETA * 9 + 3) & ~3));   // [e][eta][(l, m)]
    const int Frad = dp.n_el * dp.n_rad;
    const float inv_rc = 1.0f / dp.rc;

    const CentreRange cr = centre_range(B);
    for (int ci = cr.begin; ci < cr.end; ++ci) {
        const int i = __builtin_amdgcn_readfirstlane(order ? order[ci] : ci);
        const BeadInfo bi = beads[bead_of_ba[i]];
        const float4 pi = posu[i];
        for (int f = lane; f < dp.D; f += kWave)
            gl[f] = dEdG[(int64_t)i * dp.D + f];
        wave_sync();
        // H_l(pair, eta) = sum_{zeta, lambda} dE/dG 2^(1-zeta) a_l (+-1)^l
        for (int t = lane; t < n_pairs * NETA * (kG5L + 1); t += kWave) {
            const int l = t % (kG5L + 1), pe = t / (kG5L + 1);
            const int ie = pe % NETA, pair = pe / NETA;
            const float *g = gl + Frad + pair * dp.n_ang + ie * 8;
            float h = 0.0f;
#pragma unroll
            for (int iz = 0; iz < 4; ++iz) {
                const float gz = (l & 1) ? g[2 * iz] - g[2 * iz + 1] : g[2 * iz] + g[2 * iz + 1];
                h = fmaf(dp.g5_leg[iz][l], gz, h);
            }
            H[t] = h;
        }
        wave_sync();
        // dE/dM_e[lm] = c_m sum_e' H_l(e, e') M_e'[lm], lane = harmonic
        const float *mo = mom + (int64_t)i * dp.n_el * NETA * kG5Mom;
        for (int t = lane; t < kG5Y; t += kWave) {
            int l = 0;
            while ((l + 1) * (l + 1) <= t)
                ++l;
            const int k = t - l * l, m = (k + 1) >> 1, part = k > 0 ? (k - 1) & 1 : 0;
            const float cm = m ? 2.0f : 1.0f;
            for (int e = 0; e < dp.n_el; ++e)
#pragma unroll
                for (int ie = 0; ie < NETA; ++ie) {
                    float g = 0.0f;
                    for (int e2 = 0; e2 < dp.n_el; ++e2)
                        g = fmaf(H[(pair_of(e, e2, dp.n_el) * NETA + ie) * (kG5L + 1) + l],
                                 mo[(e2 * NETA + ie) * kG5Mom + t], g);
                    float *dst = reinterpret_cast<float *>(gM + (e * NETA + ie) * kG5Lm + l * (l + 1) / 2 + m);
                    dst[part] = cm * g;
                    if (m == 0)
                        dst[1] = 0.0f;
                }
        }
        wave_sync();
        float W[16];
#pragma unroll
        for (int q = 0; q < 16; ++q)
            W[q] = 0.0f;
        const int K = nbr_cnt[i];
        const int32_t *row = nbr + (int64_t)i * dp.Kmax;
        const int key_i = (__float_as_int(pi.w) << kKeyShift) | i;
        bool missing = false;
        for (int n = lane; n < K; n += kWave) {
            const int key = row[n];
            const int e = key >> kKeyShift;
            float3 d;
            float r, r_lo, inv_r, fc, dfc;
            displacement(pi, posu[key & (int)kRowMask], bi, d, r, r_lo, inv_r);
            cutoff_fn(r * inv_rc, dp.pi_over_rc, fc, dfc);
            // radial functions: dE/dr
            float sr = 0.0f;
            for (int t = 0; t < dp.n_rad; ++t) {
                const float x = (r - dp.rad_center[t]) + (r_lo - dp.rad_center_lo[t]);
                const float eta = dp.rad_eta[t];
                sr += gl[e * dp.n_rad + t] * expf(-eta * x * x) * (-2.0f * eta * x * fc + dfc);
            }
            float wv[NETA], dw[NETA], Hs[NETA][kG5L + 1];
#pragma unroll
            for (int ie = 0; ie < NETA; ++ie) {
                const float ex = expf(-dp.ang_eta[ie] * r * r);
                wv[ie] = ex * fc;
                dw[ie] = ex * (-2.0f * dp.ang_eta[ie] * r * fc + dfc);
                const float *h = H + (pair_of(e, e, dp.n_el) * NETA + ie) * (kG5L + 1);
#pragma unroll
                for (int l = 0; l <= kG5L; ++l)
                    Hs[ie][l] = h[l];
            }
            const float ux = d.x * inv_r, uy = d.y * inv_r, uz = d.z * inv_r;
            // dE/d(w Y_lm) of this slot = dE/dM_e[lm] - c_m H_l(e, e) w Y_lm: the
            // moments include the slot itself, and the e = e' power spectrum
            // excludes j = k.  Per eta, Psi = sum of those times Y and its gradient in
            // (x, y, z), accumulated over l at fixed m (C, S: cos and sin parts;
            // z: the z derivative; T, Tz: the self terms sum_l H_l q^2, H_l q dq)
            float Psi[NETA], Gx[NETA], Gy[NETA], Gz[NETA], C[NETA], S[NETA], Cz[NETA], Sz[NETA], T[NETA], Tz[NETA];
#pragma unroll
            for (int ie = 0; ie < NETA; ++ie)
                Psi[ie] = Gx[ie] = Gy[ie] = Gz[ie] = C[ie] = S[ie] = Cz[ie] = Sz[ie] = T[ie] = Tz[ie] = 0.0f;
            const float2 *gme = gM + e * NETA * kG5Lm;
            for_each_harmonic(ux, uy, uz, [&](int l, int m, float q, float dq, float A, float Bs, float Ap, float Bp) {
#pragma unroll
                for (int ie = 0; ie < NETA; ++ie) {
                    const float2 g = gme[ie * kG5Lm + l * (l + 1) / 2 + m];
                    C[ie] = fmaf(g.x, q, C[ie]);
                    Cz[ie] = fmaf(g.x, dq, Cz[ie]);
                    if (m > 0) {
                        S[ie] = fmaf(g.y, q, S[ie]);
                        Sz[ie] = fmaf(g.y, dq, Sz[ie]);
                    }
                    const float hq = Hs[ie][l] * q;
                    T[ie] = fmaf(hq, q, T[ie]);
                    Tz[ie] = fmaf(hq, dq, Tz[ie]);
                }
                if (l == kG5L) {   // last l of this m: fold the m terms in
#pragma unroll
                    for (int ie = 0; ie < NETA; ++ie) {
                        const float cw = (m ? 2.0f : 1.0f) * wv[ie];
                        const float c = C[ie] - cw * T[ie] * A, sv = S[ie] - cw * T[ie] * Bs;
                        const float cz = Cz[ie] - cw * Tz[ie] * A, sz = Sz[ie] - cw * Tz[ie] * Bs;
                        Psi[ie] += c * A + sv * Bs;
                        Gz[ie] += cz * A + sz * Bs;
                        if (m > 0) {
                            Gx[ie] += (float)m * (c * Ap + sv * Bp);
                            Gy[ie] += (float)m * (sv * Ap - c * Bp);
                        }
                        C[ie] = S[ie] = Cz[ie] = Sz[ie] = T[ie] = Tz[ie] = 0.0f;
                    }
                }
            });
            float tx = 0.0f, ty = 0.0f, tz = 0.0f;
#pragma unroll
            for (int ie = 0; ie < NETA; ++ie) {
                sr = fmaf(dw[ie], Psi[ie], sr);
                tx = fmaf(wv[ie], Gx[ie], tx);
                ty = fmaf(wv[ie], Gy[ie], ty);
                tz = fmaf(wv[ie], Gz[ie], tz);
            }
            // dE/dd = sr u + (T - (u.T) u) / r
            const float ut = ux * tx + uy * ty + uz * tz;
            const float4 v = make_float4(sr * ux + (tx - ut * ux) * inv_r, sr * uy + (ty - ut * uy) * inv_r,
                                         sr * uz + (tz - ut * uz) * inv_r, 0.0f);
            store_slot_values(nbr, fence, dp.Kmax, i, key_i, n, v, vslot, vrev, missing);
            const float dd[3] = {d.x, d.y, d.z}, vv[3] = {v.x, v.y, v.z};
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    W[a * 3 + b] -= dd[a] * vv[b];
        }
        const float tot = transpose_reduce<16>(W);
        if ((lane & 3) == 0 && (lane >> 2) < 9)
            vir_atom[(int64_t)i * 9 + (lane >> 2)] = tot;
        const bool any_missing = __ballot(missing) != 0;
        if (lane == 0 && any_missing)
            atomicOr(status, kStatusOverflow);
        wave_sync();
    }
}

hipError_t configure_g5_lds(const DescParams &dp)
{
    const int f = (int)(4 * g5_forward_wave_bytes(dp));
    const int a = (int)(4 * sizeof(float) * g5_adjoint_wave_floats(dp));
    hipError_t e;
    if (dp.n_ang_eta == 2) {
        e = hipFuncSetAttribute((const void *)k_descriptors_g5<2>, hipFuncAttributeMaxDynamicSharedMemorySize, f);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_adjoint_g5<2>, hipFuncAttributeMaxDynamicSharedMemorySize, a);
    } else {
        e = hipFuncSetAttribute((const void *)k_descriptors_g5<1>, hipFuncAttributeMaxDynamicSharedMemorySize, f);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_adjoint_g5<1>, hipFuncAttributeMaxDynamicSharedMemorySize, a);
    }
    return e;
}

// The forward always runs one wave per workgroup: its 21.8 kB of LDS per wave
// (water) make bigger workgroups leave CUs idle (water 4096: 3.81 ms at one
// wave, 4.51 at two, 6.29 at four), whatever shape suits the other kernels.
void launch_descriptors_g5(const DevBuffers &d, const Sizes &z, const DescParams &dp, const Tuning &tn,
                           hipStream_t s)
{
    Tuning one = tn;
    one.centre_waves = 1;
    const int wpg = 1, grid = centre_grid(z.B, one);
    const size_t lds = wpg * g5_forward_wave_bytes(dp);
    if (dp.n_ang_eta == 2)
        hipLaunchKernelGGL(k_descriptors_g5<2>, dim3(grid), dim3(kWave * wpg), lds, s, d.posu4, d.beads,
                           d.bead_of_ba, centre_order(d, z), d.nbr, d.nbr_cnt, d.nbr_grp, d.norm, dp, d.xhat,
                           d.g5_mom, z.B);
    else
        hipLaunchKernelGGL(k_descriptors_g5<1>, dim3(grid), dim3(kWave * wpg), lds, s, d.posu4, d.beads,
                           d.bead_of_ba, centre_order(d, z), d.nbr, d.nbr_cnt, d.nbr_grp, d.norm, dp, d.xhat,
                           d.g5_mom, z.B);
}

void launch_adjoint_g5(const DevBuffers &d, const Sizes &z, const DescParams &dp, const Tuning &tn, hipStream_t s)
{
    const int wpg = tn.centre_waves, grid = centre_grid(z.B, tn);
    const size_t lds = wpg * sizeof(float) * g5_adjoint_wave_floats(dp);
    if (dp.n_ang_eta == 2)
        hipLaunchKernelGGL(k_adjoint_g5<2>, dim3(grid), dim3(kWave * wpg), lds, s, d.posu4, d.beads, d.bead_of_ba,
                           centre_order(d, z), d.nbr, d.nbr_cnt, d.dEdG, d.g5_mom, d.nbr_fence, dp, d.vslot,
                           tn.force_rows ? d.vrev : nullptr,
                           d.vir_atom, d.status, z.B);
    else
        hipLaunchKernelGGL(k_adjoint_g5<1>, dim3(grid), dim3(kWave * wpg), lds, s, d.posu4, d.beads, d.bead_of_ba,
                           centre_order(d, z), d.nbr, d.nbr_cnt, d.dEdG, d.g5_mom, d.nbr_fence, dp, d.vslot,
                           tn.force_rows ? d.vrev : nullptr,
                           d.vir_atom, d.status, z.B);
}

}  // namespace pimd
