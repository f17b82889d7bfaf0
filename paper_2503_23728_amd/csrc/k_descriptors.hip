// Behler-Parrinello symmetry functions (forward) and their adjoint
// (dE/d d_ij for every neighbour slot, with recomputation of the pair and
// triplet terms instead of storing dG/dr), and the atomic-free force
// assembly.  One wave per centre atom.
//
//   f_c(r) = (cos(pi r/rc) + 1)/2
//   G2[e,s] = sum_{j: Z_j = e} exp(-eta_s (r_ij - R_s)^2) f_c(r_ij)
//   G4[{e1,e2}, eta, zeta, lambda] = 2^(1-zeta) sum_{j<k} (1 + lambda cos)^zeta
//        exp(-eta (r_ij^2 + r_ik^2 + r_jk^2)) f_c(r_ij) f_c(r_ik) f_c(r_jk)
// (Behler-Parrinello descriptors, cited in the Introduction; forces from the
// energy by the chain rule, the energy-model route of Sec. 2.2.)
//
// The neighbour slots of a centre arrive grouped by element (keys sorted by
// (element, row)), so an element-pair block is either a rectangle n1 x n2
// (e1 < e2) or a triangle n1 (n1 - 1)/2 (e1 = e2) of slot pairs; the pairs of
// a block are flattened and dealt to the 64 lanes.  Per-neighbour terms
// (displacement, r, f_c, exp(-eta r^2) f_c and their r-derivatives) are staged
// once in LDS and shared by all triplets of the centre.
#include "device_common.hpp"

namespace pimd {

struct StagedA {  // per neighbour slot
    float4 d;     // dx, dy, dz, r
    float4 e;     // fc, E_0 = exp(-eta_0 r^2) fc, E_1, 1/r
};

// Displacement d_ij = q_j - q_i (minimum image) of the unwrapped float32
// positions, formed in FP64 with the FP64 box and rounded once to float32, so
// it carries no rounding from wrapping large coordinates.  The neighbour set
// itself comes from the float32 test of the neighbour kernel; for |d| < rc <
// L/2 the minimum image is unique, so both choose the same image.
__device__ __forceinline__ void displacement(const float4 &pi, const float4 &pj, const BeadInfo &bi, float3 &d,
                                             float &r, float &inv_r)
{
    double dx = (double)pj.x - (double)pi.x, dy = (double)pj.y - (double)pi.y, dz = (double)pj.z - (double)pi.z;
    if (bi.periodic) {
        dx -= bi.L64[0] * rint(dx * bi.invL64[0]);
        dy -= bi.L64[1] * rint(dy * bi.invL64[1]);
        dz -= bi.L64[2] * rint(dz * bi.invL64[2]);
    }
    const double r64 = sqrt(dx * dx + dy * dy + dz * dz);
    d = make_float3((float)dx, (float)dy, (float)dz);
    r = (float)r64;
    inv_r = (float)(1.0 / r64);
}

// Slot pair t of a block -> (a, b) slot offsets inside the two groups.
__device__ __forceinline__ void decode_pair(int t, bool tri, int n2, float inv_n2, int &a, int &b)
{
    if (tri) {
        // t = b (b - 1)/2 + a, 0 <= a < b
        int bb = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)t)) * 0.5f);
        if (bb * (bb - 1) / 2 > t)
            --bb;
        if ((bb + 1) * bb / 2 <= t)
            ++bb;
        b = bb;
        a = t - bb * (bb - 1) / 2;
    } else {
        int aa = (int)(((float)t + 0.5f) * inv_n2);
        int bb = t - aa * n2;
        if (bb < 0) {
            --aa;
            bb += n2;
        } else if (bb >= n2) {
            ++aa;
            bb -= n2;
        }
        a = aa;
        b = bb;
    }
}

// Walk over the slot pairs of one element-pair block.  Each lane owns one
// slot b of the "own" group for the whole block and pairs it with partner
// slot (b + s) mod n_par for a uniform shift s:
//   triangle (e1 = e2, n slots): s = 1 .. n/2, and for even n the shift n/2
//     only for b < n/2, so every unordered pair appears once;
//   rectangle (e1 < e2): own = the larger group, s = 0 .. n_par - 1.
// Lane work is balanced and the lane's own slot changes only between
// chunks of 64 slots, so its share of the gradient can stay in registers.
struct BlockWalk {
    bool tri;
    int n_own, n_par, o_own, o_par, s0, s1;
    __device__ BlockWalk(int e1, int e2, const int *gcnt, const int *goff)
    {
        tri = e1 == e2;
        if (tri) {
            n_own = n_par = gcnt[e1];
            o_own = o_par = goff[e1];
            s0 = 1;
            s1 = n_own / 2;
        } else {
            const bool swap = gcnt[e1] > gcnt[e2];
            const int eo = swap ? e1 : e2, ep = swap ? e2 : e1;
            n_own = gcnt[eo];
            n_par = gcnt[ep];
            o_own = goff[eo];
            o_par = goff[ep];
            s0 = 0;
            s1 = n_par - 1;
        }
    }
    __device__ bool active(bool own_ok, int b, int s) const
    {
        return own_ok && (!tri || 2 * s != n_own || b < s);
    }
};

// Stage the neighbour records of centre i; returns K.  Also fills grp_off.
template <int NETA, bool ADJ>
__device__ __forceinline__ int stage_neighbors(int i, const float4 &pi, const BeadInfo &bi, const int32_t *nbr,
                                               const int32_t *nbr_cnt, const float4 *posu, const DescParams &dp,
                                               StagedA *rec, float4 *recd)
{
    const int lane = lane_id();
    const int K = nbr_cnt[i];
    const int32_t *row = nbr + (int64_t)i * dp.Kmax;
    for (int n = lane; n < K; n += kWave) {
        const int j = row[n] & (int)kRowMask;
        const float4 pj = posu[j];
        float3 d;
        float r, inv_r;
        displacement(pi, pj, bi, d, r, inv_r);
        const float r2 = r * r;
        const float x = r * (1.0f / dp.rc);
        const float fc = 0.5f * cospif(x) + 0.5f;
        const float g0 = expf(-dp.ang_eta[0] * r2);
        const float g1 = NETA > 1 ? expf(-dp.ang_eta[1] * r2) : 0.0f;
        StagedA s;
        s.d = make_float4(d.x, d.y, d.z, r);
        s.e = make_float4(fc, g0 * fc, g1 * fc, inv_r);
        rec[n] = s;
        if (ADJ) {
            // dE_eta/dr = exp(-eta r^2) (-2 eta r fc + fc'),  fc' = -(pi/(2 rc)) sin(pi r/rc)
            const float dfc = -0.5f * dp.pi_over_rc * sinpif(x);
            recd[n] = make_float4(g0 * (-2.0f * dp.ang_eta[0] * r * fc + dfc),
                                  NETA > 1 ? g1 * (-2.0f * dp.ang_eta[1] * r * fc + dfc) : 0.0f, dfc, 0.0f);
        }
    }
    return K;
}

// ---------------------------------------------------------------------------
// forward: normalised descriptors xhat[i][D]
// ---------------------------------------------------------------------------
template <int NETA>
__global__ __launch_bounds__(256) void k_descriptors(const float4 *__restrict__ posu,
                                                     const BeadInfo *__restrict__ beads,
                                                     const int32_t *__restrict__ bead_of_ba,
                                                     const int32_t *__restrict__ nbr,
                                                     const int32_t *__restrict__ nbr_cnt,
                                                     const int32_t *__restrict__ nbr_grp,
                                                     const float *__restrict__ norm, DescParams dp,
                                                     float *__restrict__ xhat, int B)
{
    extern __shared__ float4 lds4[];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int Dcap = (dp.D + 3) & ~3;
    float4 *base = lds4 + w * (2 * dp.Kmax + Dcap / 4);
    StagedA *rec = reinterpret_cast<StagedA *>(base);
    float *Gs = reinterpret_cast<float *>(base + 2 * dp.Kmax);
    const int Frad = dp.n_el * dp.n_rad;

    for (int i = blockIdx.x * 4 + w; i < B; i += gridDim.x * 4) {
        const BeadInfo bi = beads[bead_of_ba[i]];
        const float4 pi = posu[i];
        const int zi = __float_as_int(pi.w);
        stage_neighbors<NETA, false>(i, pi, bi, nbr, nbr_cnt, posu, dp, rec, nullptr);
        int gcnt[kMaxElements], goff[kMaxElements];
        {
            int o = 0;
            for (int e = 0; e < kMaxElements; ++e) {
                gcnt[e] = e < dp.n_el ? nbr_grp[(int64_t)i * kMaxElements + e] : 0;
                goff[e] = o;
                o += gcnt[e];
            }
        }
        wave_sync();
        // radial: lane -> feature (e, s); the two half-waves split the group
        for (int f0 = 0; f0 < Frad; f0 += 32) {
            const int f = f0 + (lane & 31);
            float acc = 0.0f;
            if (f < Frad) {
                const int e = f / dp.n_rad, s = f - e * dp.n_rad;
                const int lo = goff[e], hi = goff[e] + gcnt[e];
                const int mid = (lo + hi) >> 1;
                const int a0 = (lane < 32) ? lo : mid, a1 = (lane < 32) ? mid : hi;
                const float Rs = dp.rad_center[s], eta = dp.rad_eta[s];
                for (int n = a0; n < a1; ++n) {
                    const float x = rec[n].d.w - Rs;
                    acc += expf(-eta * x * x) * rec[n].e.x;
                }
            }
            acc += __shfl_xor(acc, 32, kWave);
            if (lane < 32 && f < Frad)
                Gs[f] = acc;
        }
        // angular blocks
        int pair = 0;
        for (int e1 = 0; e1 < dp.n_el; ++e1)
            for (int e2 = e1; e2 < dp.n_el; ++e2, ++pair) {
                BlockWalk bw(e1, e2, gcnt, goff);
                float acc[8 * NETA];
#pragma unroll
                for (int q = 0; q < 8 * NETA; ++q)
                    acc[q] = 0.0f;
                for (int b0 = 0; b0 < bw.n_own; b0 += kWave) {
                    const int b = b0 + lane;
                    const bool own_ok = b < bw.n_own;
                    const StagedA A = rec[bw.o_own + (own_ok ? b : 0)];
                    const int bm = bw.tri ? b : ((own_ok && bw.n_par > 0) ? b % bw.n_par : 0);
                    for (int s = bw.s0; s <= bw.s1; ++s) {
                        if (!bw.active(own_ok, b, s))
                            continue;
                        int p = bm + s;
                        p -= p >= bw.n_par ? bw.n_par : 0;
                        const StagedA C = rec[bw.o_par + p];
                        const float jx = C.d.x - A.d.x, jy = C.d.y - A.d.y, jz = C.d.z - A.d.z;
                        const float r2jk = jx * jx + jy * jy + jz * jz;
                        if (r2jk < dp.rc2) {
                            const float rjk = sqrtf(r2jk);
                            const float fcjk = 0.5f * cospif(rjk * (1.0f / dp.rc)) + 0.5f;
                            const float cs = (A.d.x * C.d.x + A.d.y * C.d.y + A.d.z * C.d.z) * (A.e.w * C.e.w);
                            const float p1 = 1.0f + cs, m1 = 1.0f - cs;
                            const float p2 = p1 * p1, m2 = m1 * m1;
                            const float p4 = p2 * p2, m4 = m2 * m2;
                            const float p8 = p4 * p4, m8 = m4 * m4;
#pragma unroll
                            for (int ie = 0; ie < NETA; ++ie) {
                                const float Ea = ie == 0 ? A.e.y : A.e.z;
                                const float Eb = ie == 0 ? C.e.y : C.e.z;
                                const float R = Ea * Eb * expf(-dp.ang_eta[ie] * r2jk) * fcjk;
                                acc[ie * 8 + 0] += p1 * R;
                                acc[ie * 8 + 1] += m1 * R;
                                acc[ie * 8 + 2] += p2 * R;
                                acc[ie * 8 + 3] += m2 * R;
                                acc[ie * 8 + 4] += p4 * R;
                                acc[ie * 8 + 5] += m4 * R;
                                acc[ie * 8 + 6] += p8 * R;
                                acc[ie * 8 + 7] += m8 * R;
                            }
                        }
                    }
                }
                float mine = 0.0f;
#pragma unroll
                for (int q = 0; q < 8 * NETA; ++q) {
                    const float v = wave_sum(acc[q]);
                    if (lane == q)
                        mine = v;
                }
                if (lane < 8 * NETA) {
                    const int iz = (lane & 7) >> 1;
                    const float scale = iz == 0 ? 1.0f : (iz == 1 ? 0.5f : (iz == 2 ? 0.125f : 0.0078125f));
                    Gs[Frad + pair * dp.n_ang + lane] = mine * scale;
                }
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
__global__ __launch_bounds__(256) void k_adjoint(const float4 *__restrict__ posu, const BeadInfo *__restrict__ beads,
                                                 const int32_t *__restrict__ bead_of_ba,
                                                 const int32_t *__restrict__ nbr,
                                                 const int32_t *__restrict__ nbr_cnt,
                                                 const int32_t *__restrict__ nbr_grp,
                                                 const float *__restrict__ dEdG, DescParams dp,
                                                 float4 *__restrict__ vslot, float *__restrict__ vir_atom, int B)
{
    extern __shared__ float4 lds4[];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int Dcap = (dp.D + 3) & ~3;
    float4 *base = lds4 + w * (4 * dp.Kmax + Dcap / 4);
    StagedA *rec = reinterpret_cast<StagedA *>(base);
    float4 *recd = base + 2 * dp.Kmax;
    float4 *vacc = base + 3 * dp.Kmax;
    float *gl = reinterpret_cast<float *>(base + 4 * dp.Kmax);
    const int Frad = dp.n_el * dp.n_rad;

    for (int i = blockIdx.x * 4 + w; i < B; i += gridDim.x * 4) {
        const BeadInfo bi = beads[bead_of_ba[i]];
        const float4 pi = posu[i];
        const int K = stage_neighbors<NETA, true>(i, pi, bi, nbr, nbr_cnt, posu, dp, rec, recd);
        for (int f = lane; f < dp.D; f += kWave)
            gl[f] = dEdG[(int64_t)i * dp.D + f];
        int gcnt[kMaxElements], goff[kMaxElements];
        {
            int o = 0;
            for (int e = 0; e < kMaxElements; ++e) {
                gcnt[e] = e < dp.n_el ? nbr_grp[(int64_t)i * kMaxElements + e] : 0;
                goff[e] = o;
                o += gcnt[e];
            }
        }
        const int32_t *row = nbr + (int64_t)i * dp.Kmax;
        wave_sync();
        // radial part of every slot: sum_s g[e,s] dG2/dr * d/r
        for (int n = lane; n < K; n += kWave) {
            const int e = row[n] >> kKeyShift;
            const StagedA s = rec[n];
            const float r = s.d.w, fc = s.e.x, dfc = recd[n].z;
            float acc = 0.0f;
            for (int q = 0; q < dp.n_rad; ++q) {
                const float x = r - dp.rad_center[q];
                const float eta = dp.rad_eta[q];
                acc += gl[e * dp.n_rad + q] * expf(-eta * x * x) * (-2.0f * eta * x * fc + dfc);
            }
            const float c = acc * s.e.w;
            vacc[n] = make_float4(c * s.d.x, c * s.d.y, c * s.d.z, 0.0f);
        }
        wave_sync();
        int pair = 0;
        for (int e1 = 0; e1 < dp.n_el; ++e1)
            for (int e2 = e1; e2 < dp.n_el; ++e2, ++pair) {
                BlockWalk bw(e1, e2, gcnt, goff);
                // block coefficients with the 2^(1-zeta) factors folded in
                float gq[8 * NETA];
#pragma unroll
                for (int q = 0; q < 8 * NETA; ++q) {
                    const int iz = (q & 7) >> 1;
                    const float scale = iz == 0 ? 1.0f : (iz == 1 ? 0.5f : (iz == 2 ? 0.125f : 0.0078125f));
                    gq[q] = gl[Frad + pair * dp.n_ang + q] * scale;
                }
                for (int b0 = 0; b0 < bw.n_own; b0 += kWave) {
                    const int b = b0 + lane;
                    const bool own_ok = b < bw.n_own;
                    const int ia_slot = bw.o_own + (own_ok ? b : 0);
                    const StagedA A = rec[ia_slot];
                    const float4 dA = recd[ia_slot];
                    const int bm = bw.tri ? b : ((own_ok && bw.n_par > 0) ? b % bw.n_par : 0);
                    float vx = 0.0f, vy = 0.0f, vz = 0.0f;   // gradient on the lane's own slot
                    for (int s = bw.s0; s <= bw.s1; ++s) {
                        if (!bw.active(own_ok, b, s))
                            continue;
                        int p = bm + s;
                        p -= p >= bw.n_par ? bw.n_par : 0;
                        const int ic = bw.o_par + p;
                        const StagedA C = rec[ic];
                        const float jx = C.d.x - A.d.x, jy = C.d.y - A.d.y, jz = C.d.z - A.d.z;
                        const float r2jk = jx * jx + jy * jy + jz * jz;
                        if (!(r2jk < dp.rc2))
                            continue;
                        const float4 dC = recd[ic];
                        const float rjk = sqrtf(r2jk), inv_rjk = 1.0f / rjk;
                        const float x = rjk * (1.0f / dp.rc);
                        const float fcjk = 0.5f * cospif(x) + 0.5f;
                        const float dfcjk = -0.5f * dp.pi_over_rc * sinpif(x);
                        const float cs = (A.d.x * C.d.x + A.d.y * C.d.y + A.d.z * C.d.z) * (A.e.w * C.e.w);
                        const float p1 = 1.0f + cs, m1 = 1.0f - cs;
                        const float p2 = p1 * p1, m2 = m1 * m1;
                        const float p3 = p2 * p1, m3 = m2 * m1;
                        const float p4 = p2 * p2, m4 = m2 * m2;
                        const float p7 = p4 * p3, m7 = m4 * m3;
                        const float p8 = p4 * p4, m8 = m4 * m4;
                        float Pc = 0.0f, Pa = 0.0f, Pb = 0.0f, Pjk = 0.0f;
#pragma unroll
                        for (int ie = 0; ie < NETA; ++ie) {
                            const float *g = gq + ie * 8;
                            const float S = g[0] * p1 + g[1] * m1 + g[2] * p2 + g[3] * m2 + g[4] * p4 + g[5] * m4 +
                                            g[6] * p8 + g[7] * m8;
                            const float Sd = (g[0] - g[1]) + 2.0f * (g[2] * p1 - g[3] * m1) +
                                             4.0f * (g[4] * p3 - g[5] * m3) + 8.0f * (g[6] * p7 - g[7] * m7);
                            const float eta = dp.ang_eta[ie];
                            const float X = expf(-eta * r2jk);
                            const float Ea = ie == 0 ? A.e.y : A.e.z, Eb = ie == 0 ? C.e.y : C.e.z;
                            const float dEa = ie == 0 ? dA.x : dA.y, dEb = ie == 0 ? dC.x : dC.y;
                            const float Xf = X * fcjk;
                            const float EaEb = Ea * Eb;
                            Pc += Sd * EaEb * Xf;
                            Pa += S * dEa * Eb * Xf;
                            Pb += S * Ea * dEb * Xf;
                            Pjk += S * EaEb * X * (-2.0f * eta * rjk * fcjk + dfcjk);
                        }
                        const float ia = A.e.w, ib = C.e.w;
                        const float alpha_a = (Pa - Pc * cs * ia) * ia;
                        const float alpha_b = (Pb - Pc * cs * ib) * ib;
                        const float beta = Pc * ia * ib;
                        const float gam = Pjk * inv_rjk;
                        vx += alpha_a * A.d.x + beta * C.d.x - gam * jx;
                        vy += alpha_a * A.d.y + beta * C.d.y - gam * jy;
                        vz += alpha_a * A.d.z + beta * C.d.z - gam * jz;
                        // partner slots differ across lanes for triangles; for rectangles at most
                        // ceil(n_own / n_par) lanes share one
                        atomicAdd(&vacc[ic].x, alpha_b * C.d.x + beta * A.d.x + gam * jx);
                        atomicAdd(&vacc[ic].y, alpha_b * C.d.y + beta * A.d.y + gam * jy);
                        atomicAdd(&vacc[ic].z, alpha_b * C.d.z + beta * A.d.z + gam * jz);
                    }
                    if (own_ok) {
                        atomicAdd(&vacc[ia_slot].x, vx);
                        atomicAdd(&vacc[ia_slot].y, vy);
                        atomicAdd(&vacc[ia_slot].z, vz);
                    }
                }
            }
        wave_sync();
        float W[9];
#pragma unroll
        for (int q = 0; q < 9; ++q)
            W[q] = 0.0f;
        float4 *out = vslot + (int64_t)i * dp.Kmax;
        for (int n = lane; n < K; n += kWave) {
            const float4 v = vacc[n];
            out[n] = v;
            const float4 d = rec[n].d;
            const float dd[3] = {d.x, d.y, d.z}, vv[3] = {v.x, v.y, v.z};
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    W[a * 3 + b] -= dd[a] * vv[b];
        }
        float mine = 0.0f;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const float v = wave_sum(W[q]);
            if (lane == q)
                mine = v;
        }
        if (lane < 9)
            vir_atom[(int64_t)i * 9 + lane] = mine;
        wave_sync();
    }
}

// ---------------------------------------------------------------------------
// forces: F_i = sum_slots v[i][n] - sum_slots v[j][slot of i in j's list]
// (the list is symmetric, so the reverse slot is found by binary search of
// i's key in j's sorted list); no atomics, fixed summation order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_assemble_forces(const float4 *__restrict__ pos4,
                                                         const int32_t *__restrict__ nbr,
                                                         const int32_t *__restrict__ nbr_cnt,
                                                         const float4 *__restrict__ vslot, int Kmax,
                                                         float *__restrict__ F, uint32_t *__restrict__ status, int B)
{
    const int lane = lane_id(), w = threadIdx.x >> 6;
    for (int i = blockIdx.x * 4 + w; i < B; i += gridDim.x * 4) {
        const int K = nbr_cnt[i];
        const int key_i = (__float_as_int(pos4[i].w) << kKeyShift) | i;
        const int32_t *row = nbr + (int64_t)i * Kmax;
        double fx = 0.0, fy = 0.0, fz = 0.0;
        bool missing = false;
        for (int n = lane; n < K; n += kWave) {
            const float4 v = vslot[(int64_t)i * Kmax + n];
            const int j = row[n] & (int)kRowMask;
            const int32_t *rj = nbr + (int64_t)j * Kmax;
            int lo = 0, hi = nbr_cnt[j] - 1, m = -1;
            while (lo <= hi) {
                const int mid = (lo + hi) >> 1;
                const int kv = rj[mid];
                if (kv == key_i) {
                    m = mid;
                    break;
                }
                if (kv < key_i)
                    lo = mid + 1;
                else
                    hi = mid - 1;
            }
            fx += (double)v.x;
            fy += (double)v.y;
            fz += (double)v.z;
            if (m >= 0) {
                const float4 u = vslot[(int64_t)j * Kmax + m];
                fx -= (double)u.x;
                fy -= (double)u.y;
                fz -= (double)u.z;
            } else {
                missing = true;
            }
        }
        fx = wave_sum_f64(fx);
        fy = wave_sum_f64(fy);
        fz = wave_sum_f64(fz);
        const bool any_missing = __ballot(missing) != 0;
        if (lane == 0) {
            F[3 * (int64_t)i + 0] = (float)fx;
            F[3 * (int64_t)i + 1] = (float)fy;
            F[3 * (int64_t)i + 2] = (float)fz;
            if (any_missing)
                atomicOr(status, kStatusOverflow);
            if (!(isfinite(fx) && isfinite(fy) && isfinite(fz)))
                atomicOr(status, kStatusNonFinite);
        }
    }
}

// Per-bead energy and virial sums (one workgroup per bead, fixed tree order).
__global__ __launch_bounds__(256) void k_bead_sums(const BeadInfo *__restrict__ beads,
                                                   const float *__restrict__ E_atom,
                                                   const float *__restrict__ vir_atom, float *__restrict__ E_bead,
                                                   float *__restrict__ W_bead, int virial,
                                                   uint32_t *__restrict__ status)
{
    const BeadInfo bi = beads[blockIdx.x];
    __shared__ float red[10][256];
    float acc[10];
    for (int q = 0; q < 10; ++q)
        acc[q] = 0.0f;
    for (int t = threadIdx.x; t < bi.n; t += 256) {
        acc[0] += E_atom[bi.ba0 + t];
        if (virial)
            for (int q = 0; q < 9; ++q)
                acc[1 + q] += vir_atom[9 * (int64_t)(bi.ba0 + t) + q];
    }
    for (int q = 0; q < 10; ++q)
        red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o)
            for (int q = 0; q < 10; ++q)
                red[q][threadIdx.x] += red[q][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        E_bead[blockIdx.x] = red[0][0];
        if (!isfinite(red[0][0]))
            atomicOr(status, kStatusNonFinite);
    }
    if (virial && W_bead && threadIdx.x < 9)
        W_bead[9 * blockIdx.x + threadIdx.x] = red[1 + threadIdx.x][0];
}

// Work counter: neighbour pairs, j<k triplets, triplets with r_jk < rc.
__global__ __launch_bounds__(256) void k_work_counts(const float4 *__restrict__ posu,
                                                     const BeadInfo *__restrict__ beads,
                                                     const int32_t *__restrict__ bead_of_ba,
                                                     const int32_t *__restrict__ nbr,
                                                     const int32_t *__restrict__ nbr_cnt, DescParams dp,
                                                     unsigned long long *__restrict__ counts, int B)
{
    extern __shared__ float4 lds4[];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    StagedA *rec = reinterpret_cast<StagedA *>(lds4 + w * 2 * dp.Kmax);
    unsigned long long pairs = 0, trip = 0, trip_in = 0;
    for (int i = blockIdx.x * 4 + w; i < B; i += gridDim.x * 4) {
        const BeadInfo bi = beads[bead_of_ba[i]];
        const int K = stage_neighbors<1, false>(i, posu[i], bi, nbr, nbr_cnt, posu, dp, rec, nullptr);
        wave_sync();
        const int np = K * (K - 1) / 2;
        for (int t = lane; t < np; t += kWave) {
            int a, b;
            decode_pair(t, true, 0, 0.0f, a, b);
            const float jx = rec[b].d.x - rec[a].d.x, jy = rec[b].d.y - rec[a].d.y, jz = rec[b].d.z - rec[a].d.z;
            trip_in += (jx * jx + jy * jy + jz * jz) < dp.rc2 ? 1 : 0;
        }
        if (lane == 0) {
            pairs += K;
            trip += np;
        }
        wave_sync();
    }
    atomicAdd(&counts[0], pairs);
    atomicAdd(&counts[1], trip);
    atomicAdd(&counts[2], trip_in);
}

static size_t desc_lds(const DescParams &dp, int records)
{
    const int Dcap = (dp.D + 3) & ~3;
    return (size_t)4 * (records * dp.Kmax + Dcap / 4) * sizeof(float4);
}

size_t descriptor_lds_bytes(const DescParams &dp, bool adjoint) { return desc_lds(dp, adjoint ? 4 : 2); }

hipError_t configure_descriptor_lds(const DescParams &dp)
{
    const int f = (int)desc_lds(dp, 2), a = (int)desc_lds(dp, 4);
    hipError_t e = hipSuccess;
    if (dp.n_ang_eta == 2) {
        e = hipFuncSetAttribute((const void *)k_descriptors<2>, hipFuncAttributeMaxDynamicSharedMemorySize, f);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_adjoint<2>, hipFuncAttributeMaxDynamicSharedMemorySize, a);
    } else {
        e = hipFuncSetAttribute((const void *)k_descriptors<1>, hipFuncAttributeMaxDynamicSharedMemorySize, f);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_adjoint<1>, hipFuncAttributeMaxDynamicSharedMemorySize, a);
    }
    return e;
}

void launch_descriptors(const DevBuffers &d, const Sizes &z, const DescParams &dp, hipStream_t s)
{
    const int grid = (z.B + 3) / 4;
    const size_t lds = desc_lds(dp, 2);
    if (dp.n_ang_eta == 2)
        hipLaunchKernelGGL(k_descriptors<2>, dim3(grid), dim3(256), lds, s, d.posu4, d.beads, d.bead_of_ba, d.nbr,
                           d.nbr_cnt, d.nbr_grp, d.norm, dp, d.xhat, z.B);
    else
        hipLaunchKernelGGL(k_descriptors<1>, dim3(grid), dim3(256), lds, s, d.posu4, d.beads, d.bead_of_ba, d.nbr,
                           d.nbr_cnt, d.nbr_grp, d.norm, dp, d.xhat, z.B);
}

void launch_adjoint(const DevBuffers &d, const Sizes &z, const DescParams &dp, hipStream_t s)
{
    const int grid = (z.B + 3) / 4;
    const size_t lds = desc_lds(dp, 4);
    if (dp.n_ang_eta == 2)
        hipLaunchKernelGGL(k_adjoint<2>, dim3(grid), dim3(256), lds, s, d.posu4, d.beads, d.bead_of_ba, d.nbr,
                           d.nbr_cnt, d.nbr_grp, d.dEdG, dp, d.vslot, d.vir_atom, z.B);
    else
        hipLaunchKernelGGL(k_adjoint<1>, dim3(grid), dim3(256), lds, s, d.posu4, d.beads, d.bead_of_ba, d.nbr,
                           d.nbr_cnt, d.nbr_grp, d.dEdG, dp, d.vslot, d.vir_atom, z.B);
}

void launch_work_counts(const DevBuffers &d, const Sizes &z, const DescParams &dp, unsigned long long *counts,
                        hipStream_t s)
{
    const int grid = (z.B + 3) / 4 < 4096 ? (z.B + 3) / 4 : 4096;
    hipLaunchKernelGGL(k_work_counts, dim3(grid), dim3(256), (size_t)4 * 2 * dp.Kmax * sizeof(float4), s, d.posu4,
                       d.beads, d.bead_of_ba, d.nbr, d.nbr_cnt, dp, counts, z.B);
}

void launch_assemble_forces(const DevBuffers &d, const Sizes &z, float *F, hipStream_t s)
{
    const int grid = (z.B + 3) / 4;
    hipLaunchKernelGGL(k_assemble_forces, dim3(grid), dim3(256), 0, s, d.pos4, d.nbr, d.nbr_cnt, d.vslot, z.Kmax, F,
                       d.status, z.B);
}

void launch_bead_sums(const DevBuffers &d, const Sizes &z, float *E_bead, float *W_bead, bool virial, hipStream_t s)
{
    hipLaunchKernelGGL(k_bead_sums, dim3(z.n_beads_total), dim3(256), 0, s, d.beads, d.E_atom, d.vir_atom, E_bead,
                       W_bead, virial ? 1 : 0, d.status);
}

}  // namespace pimd
