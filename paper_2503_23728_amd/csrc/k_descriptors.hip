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
// once in LDS and shared by all triplets of the centre.  The forward keeps
// the slot pairs it finds within range (one 16-bit (j, k) slot pair per
// triplet, in processing order, with a count per element-pair block), and the
// adjoint walks that list instead of testing every slot pair again.
#include "device_common.hpp"
#include "pair_terms.hpp"

namespace pimd {

// Per-neighbour records staged in LDS, shared by all triplets of a centre.
// Three arrays of 16-byte entries (not one interleaved struct), so gathers by
// slot index spread over the LDS banks:
//   recD[n] = d_ij (x, y, z), 1/r_ij
//   recE[n] = E_0, E_1 (E_eta = exp(-eta r^2) f_c(r)), dE_0/dr, dE_1/dr
//   rr[n]   = r, f_c, f_c', r_lo   (pair terms; r + r_lo is r to ~FP64 accuracy)
struct Recs {
    float4 *D;
    float4 *E;
    float4 *rr;
};

// Stage the records of centre i (slot order = key order: grouped by element)
// and hand each slot's pair terms to per_slot(n, element, d, r, r_lo, inv_r,
// f_c, f_c') in the lane that computed them.  Returns K.
template <int NETA, bool ADJ, typename PerSlot>
__device__ __forceinline__ int stage_neighbors(int i, const float4 &pi, const BeadInfo &bi, const int32_t *nbr,
                                               const int32_t *nbr_cnt, const float4 *posu, const DescParams &dp,
                                               const Recs &rec, PerSlot &&per_slot)
{
    const int lane = lane_id();
    const int K = nbr_cnt[i];
    const int32_t *row = nbr + (int64_t)i * dp.Kmax;
    for (int n = lane; n < K; n += kWave) {
        const int key = row[n];
        const int j = key & (int)kRowMask;
        float3 d;
        float r, r_lo, inv_r;
        displacement(pi, posu[j], bi, d, r, r_lo, inv_r);
        const float r2 = r * r;
        float fc, dfc;
        cutoff_fn(r * (1.0f / dp.rc), dp.pi_over_rc, fc, dfc);
        const float g0 = exp2_hw(-dp.ang_eta[0] * kLog2e * r2);
        const float g1 = NETA > 1 ? exp2_hw(-dp.ang_eta[1] * kLog2e * r2) : 0.0f;
        rec.D[n] = make_float4(d.x, d.y, d.z, inv_r);
        // dE_eta/dr = exp(-eta r^2) (-2 eta r f_c + f_c')
        rec.E[n] = make_float4(g0 * fc, g1 * fc, ADJ ? g0 * (-2.0f * dp.ang_eta[0] * r * fc + dfc) : 0.0f,
                               (ADJ && NETA > 1) ? g1 * (-2.0f * dp.ang_eta[1] * r * fc + dfc) : 0.0f);
        per_slot(n, key >> kKeyShift, d, r, r_lo, inv_r, fc, dfc);
    }
    return K;
}

__device__ __forceinline__ void group_offsets(const int32_t *nbr_grp, int i, int n_el, int (&gcnt)[kMaxElements],
                                              int (&goff)[kMaxElements])
{
    int o = 0;
    for (int e = 0; e < kMaxElements; ++e) {
        gcnt[e] = e < n_el ? nbr_grp[(int64_t)i * kMaxElements + e] : 0;
        goff[e] = o;
        o += gcnt[e];
    }
}

// Slot pair t of the triangle of K slots (t = b(b-1)/2 + a, a < b); used by
// the work counter.
__device__ __forceinline__ void decode_triangle(int t, int &a, int &b)
{
    int bb = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)t)) * 0.5f);
    if (bb * (bb - 1) / 2 > t)
        --bb;
    if ((bb + 1) * bb / 2 <= t)
        ++bb;
    b = bb;
    a = t - bb * (bb - 1) / 2;
}

// Walk over the slot pairs of one element-pair block.  Each lane owns one
// slot b of the "own" group and pairs it with partner slot (b + s) mod n_par
// for a uniform shift s:
//   triangle (e1 = e2, n slots): s = 1 .. n/2, and for even n the shift n/2
//     only for b < n/2, so every unordered pair appears once;
//   rectangle (e1 < e2): own = the larger group, s = 0 .. n_par - 1.
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
};

constexpr int kQueue = 128;   // ring of in-range slot pairs per wave (< 64 waiting + one shift's 64)

// Phase 1 of a block: every lane tests its (own, partner) pairs with the
// cheap r_jk^2 < rc^2 test and appends the pairs in range to the wave's LDS
// ring; whenever 64 are waiting, `body` runs on the oldest 64 with one pair
// per lane (phase 2), so the costly triplet terms never run on idle lanes.
// Fewer than 64 wait before a shift appends at most 64, so the ring of 128
// never overwrites a pair that has not been taken.
template <typename Body>
__device__ __forceinline__ void for_each_triplet_in_range(const BlockWalk &bw, const float4 *recD, float rc2,
                                                          uint32_t *queue, Body &&body)
{
    if (bw.s1 < bw.s0)
        return;   // fewer than two slots in a triangle, or an empty partner group
    const int lane = lane_id();
    // the half shift of an even triangle pairs only the own slots b < s; it
    // runs after the loop so the loop itself tests no slot order
    const bool has_half = bw.tri && 2 * bw.s1 == bw.n_own;
    const int s_last = has_half ? bw.s1 - 1 : bw.s1;
    int qh = 0, qn = 0;   // ring head and pairs waiting (wave-uniform)
    for (int b0 = 0; b0 < bw.n_own; b0 += kWave) {
        const int b = b0 + lane;
        const bool own_ok = b < bw.n_own;
        const int bb = own_ok ? b : 0;
        const int ia = bw.o_own + bb;
        // lanes past the own group sit far away: their test fails by distance
        const float4 A = own_ok ? recD[ia] : make_float4(3e18f, 3e18f, 3e18f, 0.0f);
        const uint32_t key_a = (uint32_t)ia << 16;
        // partner slot ic = o_par + (b + s) mod n_par, advanced by one per
        // shift; its record is loaded one shift ahead, into the other of two
        // registers (the shifts run in pairs, so no register copy per shift)
        const int p_end = bw.o_par + bw.n_par;
        // the wrap target in a vector register (the select per shift then
        // needs no move); a lane shuffle yields a value the compiler keeps there
        const int o_par_v = __shfl(bw.o_par, lane, kWave);
        int ic_next = (bw.tri ? bb : bb % bw.n_par) + bw.s0;
        ic_next = bw.o_par + ic_next - (ic_next >= bw.n_par ? bw.n_par : 0);
        float4 Ca = recD[ic_next], Cb;
        auto test = [&](bool ok, const float4 &C, float4 &Cn) {
            const int ic = ic_next;
            ic_next = ic + 1 == p_end ? o_par_v : ic + 1;
            Cn = recD[ic_next];
            const float jx = C.x - A.x, jy = C.y - A.y, jz = C.z - A.z;
            // bitwise (not short-circuit) so the test stays branch-free
            const bool inr = ok & (jx * jx + jy * jy + jz * jz < rc2);
            const uint64_t m = __builtin_amdgcn_ballot_w64(inr);
            if (inr) {
                const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                queue[(qh + qn + (int)below) & (kQueue - 1)] = key_a | (uint32_t)ic;
            }
            qn = __builtin_amdgcn_readfirstlane(qn + (int)__popcll(m));   // uniform: a scalar branch below
            if (qn >= kWave) {
                wave_sync();
                const uint32_t q = queue[(qh + lane) & (kQueue - 1)];
                body(q >> 16, q & 0xFFFFu, true);
                wave_sync();
                qh = (qh + kWave) & (kQueue - 1);
                qn -= kWave;
            }
        };
        int s = bw.s0;
        for (; s + 1 <= s_last; s += 2) {
            test(true, Ca, Cb);
            test(true, Cb, Ca);
        }
        if (s <= s_last) {
            test(true, Ca, Cb);
            Ca = Cb;
        }
        if (has_half)
            test(b < bw.s1, Ca, Cb);
    }
    if (qn > 0) {
        wave_sync();
        const uint32_t q = lane < qn ? queue[(qh + lane) & (kQueue - 1)] : 0u;
        body(q >> 16, q & 0xFFFFu, lane < qn);
        wave_sync();
    }
}

// A wave-uniform float moved to a scalar register.  The builtin takes and
// returns int: the value passes through it as bits, not converted.
__device__ __forceinline__ float uniform_float(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}

__device__ __forceinline__ float block_scale(int q)
{
    const int iz = (q & 7) >> 1;   // 2^(1 - zeta) for zeta = 1, 2, 4, 8
    return iz == 0 ? 1.0f : (iz == 1 ? 0.5f : (iz == 2 ? 0.125f : 0.0078125f));
}

// exp(-eta x) for the small arguments of the triplet terms (eta x <= ~1):
// hardware exp2 of a pre-scaled argument, relative error about 1e-7 there.
__device__ __forceinline__ float exp_small(float neg_eta_log2e, float x)
{
    return __builtin_amdgcn_exp2f(neg_eta_log2e * x);
}

// Coefficients of the angular sums as polynomials in cos: per element-pair
// block and eta, a_0 .. a_8 of S and b_0 .. b_7 of dS/dcos (17 floats).
__host__ __device__ inline int adjoint_coef_count(const DescParams &dp)
{
    return dp.n_el * (dp.n_el + 1) / 2 * dp.n_ang_eta * 17;
}

// Binomial coefficient C(zeta, k) for zeta = 2^z (z < 4), k <= zeta: the rows
// packed 7 bits per entry into one 64-bit immediate each, so a lane with its
// own k reads it with a shift instead of a memory load.
__device__ __forceinline__ double binom_zeta(int z, int k)
{
    constexpr uint64_t rows[4] = {0x81ull, 0x4101ull, 0x10818201ull, 0x11071c467070401ull};
    return (double)(int)((rows[z] >> (7 * k)) & 127u);
}

// LDS per wave of the adjoint kernel: records D and E (16 B each per slot),
// the FP64 slot accumulators (24 B per slot), the dE/dG row, the reverse
// slots (2 B per slot) and the polynomial coefficients, rounded up to 16 bytes.  The pair terms of the radial part never leave registers.
__host__ __device__ inline size_t adjoint_wave_bytes(const DescParams &dp)
{
    const int Dcap = (dp.D + 3) & ~3;
    const size_t b = (size_t)58 * dp.Kmax + 4 * (size_t)Dcap + 4 * (size_t)adjoint_coef_count(dp);
    return (b + 15) & ~(size_t)15;
}

// ---------------------------------------------------------------------------
// forward: normalised descriptors xhat[i][D]
// ---------------------------------------------------------------------------
template <int NETA, bool POW4>
__global__ __launch_bounds__(256) void k_descriptors(const float4 *__restrict__ posu,
                                                     const BeadInfo *__restrict__ beads,
                                                     const int32_t *__restrict__ bead_of_ba,
                                                     const int32_t *__restrict__ order,
                                                     const int32_t *__restrict__ nbr,
                                                     const int32_t *__restrict__ nbr_cnt,
                                                     const int32_t *__restrict__ nbr_grp,
                                                     const float *__restrict__ norm, DescParams dp,
                                                     float *__restrict__ xhat, uint16_t *__restrict__ tri_pairs,
                                                     int32_t *__restrict__ tri_cnt, int B)
{
    extern __shared__ float4 lds4[];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int Dcap = (dp.D + 3) & ~3;
    float4 *base = lds4 + w * (3 * dp.Kmax + Dcap / 4 + kQueue / 4);
    const Recs rec{base, base + dp.Kmax, base + 2 * dp.Kmax};
    const float4 *rr = rec.rr;
    float *Gs = reinterpret_cast<float *>(base + 3 * dp.Kmax);
    uint32_t *queue = reinterpret_cast<uint32_t *>(base + 3 * dp.Kmax + Dcap / 4);
    const int Frad = dp.n_el * dp.n_rad;
    const float nel0 = -dp.ang_eta[0] * 1.4426950408889634f, nel1 = -dp.ang_eta[1] * 1.4426950408889634f;
    const float inv_rc2 = 1.0f / dp.rc2;

    const CentreRange cr = centre_range(B);
    for (int ci = cr.begin; ci < cr.end; ++ci) {
        // wave-uniform: the per-centre values below live in scalar registers
        const int i = __builtin_amdgcn_readfirstlane(order ? order[ci] : ci);
        const BeadInfo bi = beads[bead_of_ba[i]];
        const float4 pi = posu[i];
        const int zi = __float_as_int(pi.w);
        stage_neighbors<NETA, false>(i, pi, bi, nbr, nbr_cnt, posu, dp, rec,
                                     [&](int n, int, const float3 &, float r, float r_lo, float, float fc, float dfc) {
                                         rec.rr[n] = make_float4(r, fc, dfc, r_lo);
                                     });
        int gcnt[kMaxElements], goff[kMaxElements];
        group_offsets(nbr_grp, i, dp.n_el, gcnt, goff);
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
                const float Rs = dp.rad_center[s], Rs_lo = dp.rad_center_lo[s], eta = dp.rad_eta[s];
                for (int n = a0; n < a1; ++n) {
                    const float4 q = rr[n];
                    // r - R_s from the two-float r and R_s: the steep Gaussians
                    // (eta up to ~5/A^2) would turn the float rounding of r into
                    // 1e-6 relative errors
                    const float x = (q.x - Rs) + (q.w - Rs_lo);
                    acc += exp2_hw(-eta * kLog2e * x * x) * q.y;
                }
            }
            acc += __shfl_xor(acc, 32, kWave);
            if (lane < 32 && f < Frad)
                Gs[f] = acc;
        }
        // angular blocks; the in-range slot pairs are kept for the adjoint
        uint16_t *kept = tri_pairs + (int64_t)i * tri_capacity(dp.Kmax);
        int n_kept = 0;
        int pair = 0;
        for (int e1 = 0; e1 < dp.n_el; ++e1)
            for (int e2 = e1; e2 < dp.n_el; ++e2, ++pair) {
                const BlockWalk bw(e1, e2, gcnt, goff);
                const int kept0 = n_kept;
                float acc[8 * NETA];
#pragma unroll
                for (int q = 0; q < 8 * NETA; ++q)
                    acc[q] = 0.0f;
                for_each_triplet_in_range(bw, rec.D, dp.rc2, queue, [&](uint32_t ia, uint32_t ic, bool ok) {
                    // the pairs of a batch occupy its first lanes
                    if (ok)
                        kept[n_kept + lane] = (uint16_t)((ia << 8) | ic);
                    n_kept += __popcll(__ballot(ok));
                    if (!ok)
                        return;
                    const float4 Ad = rec.D[ia], Cd = rec.D[ic], Ae = rec.E[ia], Ce = rec.E[ic];
                    const float jx = Cd.x - Ad.x, jy = Cd.y - Ad.y, jz = Cd.z - Ad.z;
                    const float r2jk = jx * jx + jy * jy + jz * jz;
                    const float fcjk = cutoff_sq_fc(r2jk * inv_rc2);
                    const float cs = (Ad.x * Cd.x + Ad.y * Cd.y + Ad.z * Cd.z) * (Ad.w * Cd.w);
                    const float p1 = 1.0f + cs, m1 = 1.0f - cs;
                    const float p2 = p1 * p1, m2 = m1 * m1;
                    const float p4 = p2 * p2, m4 = m2 * m2;
                    const float p8 = p4 * p4, m8 = m4 * m4;
                    const float X0 = exp_small(nel0, r2jk);
                    float X1 = 0.0f;
                    if (NETA > 1) {
                        const float X0sq = X0 * X0;
                        X1 = POW4 ? X0sq * X0sq : exp_small(nel1, r2jk);
                    }
#pragma unroll
                    for (int ie = 0; ie < NETA; ++ie) {
                        const float Ea = ie == 0 ? Ae.x : Ae.y;
                        const float Eb = ie == 0 ? Ce.x : Ce.y;
                        const float R = Ea * Eb * (ie == 0 ? X0 : X1) * fcjk;
                        acc[ie * 8 + 0] += p1 * R;
                        acc[ie * 8 + 1] += m1 * R;
                        acc[ie * 8 + 2] += p2 * R;
                        acc[ie * 8 + 3] += m2 * R;
                        acc[ie * 8 + 4] += p4 * R;
                        acc[ie * 8 + 5] += m4 * R;
                        acc[ie * 8 + 6] += p8 * R;
                        acc[ie * 8 + 7] += m8 * R;
                    }
                });
                if (lane == 0)
                    tri_cnt[(int64_t)i * kMaxPairs + pair] = n_kept - kept0;
                // lane l ends with the total of feature l / (64 / (8 NETA))
                const float tot = transpose_reduce<8 * NETA>(acc);
                constexpr int group = 64 / (8 * NETA);
                if ((lane & (group - 1)) == 0) {
                    const int q = lane / group;
                    Gs[Frad + pair * dp.n_ang + q] = tot * block_scale(q);
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
// At most 96 VGPRs (five waves per SIMD; the LDS of two-wave workgroups
// admits five as well): 1-2 % faster than 101 VGPRs and four waves.
template <int NETA, bool POW4>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_adjoint(const float4 *__restrict__ posu, const BeadInfo *__restrict__ beads,
                                                 const int32_t *__restrict__ bead_of_ba, const int32_t *__restrict__ order,
                                                 const int32_t *__restrict__ nbr,
                                                 const int32_t *__restrict__ nbr_cnt,
                                                 const float *__restrict__ dEdG,
                                                 const uint16_t *__restrict__ tri_pairs,
                                                 const int32_t *__restrict__ tri_cnt,
                                                 const int32_t *__restrict__ fence, DescParams dp,
                                                 float4 *__restrict__ vslot, float4 *__restrict__ vrev,
                                                 float *__restrict__ vir_atom, uint32_t *__restrict__ status, int B)
{
    extern __shared__ float4 lds4[];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    char *base = reinterpret_cast<char *>(lds4) + w * adjoint_wave_bytes(dp);
    const Recs rec{reinterpret_cast<float4 *>(base), reinterpret_cast<float4 *>(base) + dp.Kmax, nullptr};
    // slot accumulators: FP64 (x, y, z) per slot, interleaved so that one
    // address and two immediate offsets reach a slot's three components; each
    // slot sums ~K mixed-sign triplet terms
    double *vacc = reinterpret_cast<double *>(base + 32 * dp.Kmax);
    float *gl = reinterpret_cast<float *>(base + 56 * dp.Kmax);
    // reverse slots: where atom j = nbr[i][n] keeps the pair (j, i)
    int16_t *rev = reinterpret_cast<int16_t *>(gl + ((dp.D + 3) & ~3));
    float *coef = reinterpret_cast<float *>(rev + dp.Kmax);   // Kmax is a multiple of 16
    const int Frad = dp.n_el * dp.n_rad;
    const float nel0 = -dp.ang_eta[0] * 1.4426950408889634f, nel1 = -dp.ang_eta[1] * 1.4426950408889634f;
    const float inv_rc2 = 1.0f / dp.rc2;

    const CentreRange cr = centre_range(B);
    for (int ci = cr.begin; ci < cr.end; ++ci) {
        // wave-uniform: the per-centre values below live in scalar registers
        const int i = __builtin_amdgcn_readfirstlane(order ? order[ci] : ci);
        const BeadInfo bi = beads[bead_of_ba[i]];
        const float4 pi = posu[i];
        for (int f = lane; f < dp.D; f += kWave)
            gl[f] = dEdG[(int64_t)i * dp.D + f];
        const int key_i = (__float_as_int(pi.w) << kKeyShift) | i;
        wave_sync();
        // staging, the reverse slots when the slot values are also stored
        // there (their loads overlap the triplet work of this centre), and
        // the radial part of every slot in the lane that
        // staged it: v = sum_s g[e,s] dG2/dr * d/r
        const int K = stage_neighbors<NETA, true>(
            i, pi, bi, nbr, nbr_cnt, posu, dp, rec,
            [&](int n, int e, const float3 &d, float r, float r_lo, float inv_r, float fc, float dfc) {
                if (vrev) {
                    const int j = nbr[(int64_t)i * dp.Kmax + n] & (int)kRowMask;
                    rev[n] = (int16_t)reverse_slot(nbr, fence, dp.Kmax, j, key_i);
                }
                float acc = 0.0f;
                for (int t = 0; t < dp.n_rad; ++t) {
                    const float4 rp = dp.rad_pack[t];
                    const float x = (r - rp.x) + (r_lo - rp.y);
                    acc += gl[e * dp.n_rad + t] * exp2_hw(rp.z * x * x) * (rp.w * x * fc + dfc);
                }
                const float c = acc * inv_r;
                vacc[3 * n] = (double)(c * d.x);
                vacc[3 * n + 1] = (double)(c * d.y);
                vacc[3 * n + 2] = (double)(c * d.z);
            });
        wave_sync();
        // S(c) = sum_{zeta, lambda} g 2^(1-zeta) (1 + lambda c)^zeta as a
        // polynomial in c of degree 8, S = sum_k a_k c^k with
        // a_k = sum_zeta C(zeta, k) 2^(1-zeta) (g_+ + (-1)^k g_-), and
        // dS/dc = sum_k b_k c^k, b_k = (k + 1) a_{k+1}: Horner's rule in the
        // triplet body replaces the powers of 1 +- c.  Every term of the
        // expansion is bounded by the size of the original terms
        // (sum_k C(zeta, k) 2^(1-zeta) = 2), so nothing cancels beyond what the
        // sum itself does.  One coefficient per lane, formed in FP64 and
        // rounded once, for every block of the centre.
        const int n_coef = adjoint_coef_count(dp);
        for (int t = lane; t < n_coef; t += kWave) {
            const int c = t % 17, pe = t / 17, ie = pe % NETA, blk = pe / NETA;
            const int k = c < 9 ? c : c - 8;   // a_c, or b_{c-9} = k a_k with k = c - 8
            double a = 0.0;
#pragma unroll
            for (int z = 0; z < 4; ++z) {
                if (k <= (1 << z)) {
                    const int q = 8 * ie + 2 * z;
                    const double gp = (double)gl[Frad + blk * dp.n_ang + q] * (double)block_scale(q);
                    const double gm = (double)gl[Frad + blk * dp.n_ang + q + 1] * (double)block_scale(q + 1);
                    a += binom_zeta(z, k) * (k & 1 ? gp - gm : gp + gm);
                }
            }
            coef[t] = (float)(c < 9 ? a : (double)k * a);
        }
        wave_sync();
        const uint16_t *kept = tri_pairs + (int64_t)i * tri_capacity(dp.Kmax);
        int pair = 0;
        for (int e1 = 0; e1 < dp.n_el; ++e1)
            for (int e2 = e1; e2 < dp.n_el; ++e2, ++pair) {
                const int n_pairs_block = tri_cnt[(int64_t)i * kMaxPairs + pair];
                // the block's polynomial coefficients in scalar registers, the
                // leading ones in vector registers: an FMA takes one scalar
                // operand, so the first Horner step then needs no move
                float ga[9 * NETA], gb[8 * NETA];
#pragma unroll
                for (int ie = 0; ie < NETA; ++ie) {
                    const float *cb = coef + (pair * NETA + ie) * 17;
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        ga[9 * ie + k] = uniform_float(cb[k]);
                    ga[9 * ie + 8] = cb[8];
#pragma unroll
                    for (int k = 0; k < 7; ++k)
                        gb[8 * ie + k] = uniform_float(cb[9 + k]);
                    gb[8 * ie + 7] = cb[16];
                }
                auto body = [&](uint32_t ia, uint32_t ic, bool ok) {
                    if (!ok)
                        return;
                    const float4 Ad = rec.D[ia], Cd = rec.D[ic], Ae = rec.E[ia], Ce = rec.E[ic];
                    const float jx = Cd.x - Ad.x, jy = Cd.y - Ad.y, jz = Cd.z - Ad.z;
                    const float r2jk = jx * jx + jy * jy + jz * jz;
                    // dfcjk = (1/r_jk) d f_c/d r_jk
                    float fcjk, dfcjk;
                    cutoff_sq(r2jk * inv_rc2, fcjk, dfcjk);
                    dfcjk *= 2.0f * inv_rc2;
                    const float iab = Ad.w * Cd.w;
                    const float cs = (Ad.x * Cd.x + Ad.y * Cd.y + Ad.z * Cd.z) * iab;
                    // per eta, with Y = exp(-eta r_jk^2) f_c(r_jk):
                    //   dE/dcos:  Sd Ea Eb Y;  dE/dr_ij: S dEa Eb Y;  dE/dr_ik: S Ea dEb Y
                    //   dE/dr_jk / r_jk: S Ea Eb exp(-eta r_jk^2) (f_c'/r_jk - 2 eta f_c)
                    float Pc = 0.0f, Pa = 0.0f, Pb = 0.0f, Pjk = 0.0f;
                    const float X0 = exp_small(nel0, r2jk);
                    float X1 = 0.0f;
                    if (NETA > 1) {
                        const float X0sq = X0 * X0;
                        X1 = POW4 ? X0sq * X0sq : exp_small(nel1, r2jk);
                    }
#pragma unroll
                    for (int ie = 0; ie < NETA; ++ie) {
                        const float *a = ga + 9 * ie, *b = gb + 8 * ie;
                        float S = a[8], Sd = b[7];
#pragma unroll
                        for (int k = 7; k >= 0; --k)
                            S = fmaf(S, cs, a[k]);
#pragma unroll
                        for (int k = 6; k >= 0; --k)
                            Sd = fmaf(Sd, cs, b[k]);
                        const float X = ie == 0 ? X0 : X1;
                        const float Ea = ie == 0 ? Ae.x : Ae.y, Eb = ie == 0 ? Ce.x : Ce.y;
                        const float dEa = ie == 0 ? Ae.z : Ae.w, dEb = ie == 0 ? Ce.z : Ce.w;
                        const float Y = X * fcjk;
                        const float SY = S * Y;
                        const float EaEb = Ea * Eb;
                        Pa = fmaf(dEa, Eb * SY, Pa);
                        Pb = fmaf(dEb, Ea * SY, Pb);
                        Pc = fmaf(Sd, EaEb * Y, Pc);
                        const float gjk = fmaf(-2.0f * dp.ang_eta[ie], fcjk, dfcjk);
                        Pjk = fmaf(S * EaEb, X * gjk, Pjk);
                    }
                    // dE/d d_ij = alpha_a d_ij + beta d_ik - gam d_jk and
                    // dE/d d_ik = alpha_b d_ik + beta d_ij + gam d_jk with
                    // d_jk = d_ik - d_ij, regrouped onto d_ij and d_ik
                    const float ia_ = Ad.w, ib_ = Cd.w;
                    const float Pcs = Pc * cs;
                    const float gam = Pjk;
                    const float ka = (Pa - Pcs * ia_) * ia_ + gam;
                    const float kc = (Pb - Pcs * ib_) * ib_ + gam;
                    const float kb = Pc * iab - gam;
                    double *va = vacc + 3 * ia, *vc = vacc + 3 * ic;
                    atomicAdd(va, (double)(ka * Ad.x + kb * Cd.x));
                    atomicAdd(va + 1, (double)(ka * Ad.y + kb * Cd.y));
                    atomicAdd(va + 2, (double)(ka * Ad.z + kb * Cd.z));
                    atomicAdd(vc, (double)(kc * Cd.x + kb * Ad.x));
                    atomicAdd(vc + 1, (double)(kc * Cd.y + kb * Ad.y));
                    atomicAdd(vc + 2, (double)(kc * Cd.z + kb * Ad.z));
                };
                // the block's in-range slot pairs as the forward found them, one
                // per lane; the next batch's pairs load while this one runs.
                // Every lane loads from a wave-uniform base: the loads past the
                // block's last pair (at most 127 entries, inside the centre's
                // capacity) are never used.
                const uint16_t *ahead = kept + kWave;
                uint32_t nxt = kept[lane];
                for (int t0 = 0; t0 < n_pairs_block; t0 += kWave) {
                    const uint32_t v = nxt;
                    nxt = ahead[lane];
                    ahead += kWave;
                    body(v >> 8, v & 0xFFu, t0 + lane < n_pairs_block);
                }
                kept += n_pairs_block;
            }
        wave_sync();
        float W[16];
#pragma unroll
        for (int q = 0; q < 16; ++q)
            W[q] = 0.0f;
        bool missing = false;
        for (int n = lane; n < K; n += kWave) {
            const float4 v = make_float4((float)vacc[3 * n], (float)vacc[3 * n + 1], (float)vacc[3 * n + 2], 0.0f);
            vslot[(int64_t)i * dp.Kmax + n] = v;
            if (vrev) {
                const int j = nbr[(int64_t)i * dp.Kmax + n] & (int)kRowMask;
                const int hit = rev[n];
                if (hit >= 0)
                    vrev[(int64_t)j * dp.Kmax + hit] = v;
                else
                    missing = true;
            }
            const float4 dn = rec.D[n];
            const float dd[3] = {dn.x, dn.y, dn.z}, vv[3] = {v.x, v.y, v.z};
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    W[a * 3 + b] -= dd[a] * vv[b];
        }
        // components 9..15 are padding; lane 4q holds the total of component q
        const float tot = transpose_reduce<16>(W);
        if ((lane & 3) == 0 && (lane >> 2) < 9)
            vir_atom[(int64_t)i * 9 + (lane >> 2)] = tot;
        const bool any_missing = __ballot(missing) != 0;
        if (lane == 0 && any_missing)
            atomicOr(status, kStatusOverflow);
        wave_sync();
    }
}

// ---------------------------------------------------------------------------
// forces: F_i = sum_slots v[i][n] - sum_slots v[j][slot of i in j's list].
// With ROWS the adjoint stored the second term at i's slot n, so both are
// contiguous rows of i; without, it is gathered from j's row through the
// reverse-slot search.  The same sums in the same order either way, no
// atomics.
// ---------------------------------------------------------------------------
template <bool ROWS>
__global__ __launch_bounds__(256) void k_assemble_forces(const float4 *__restrict__ pos4,
                                                         const int32_t *__restrict__ order,
                                                         const int32_t *__restrict__ nbr,
                                                         const int32_t *__restrict__ nbr_cnt,
                                                         const int32_t *__restrict__ fence,
                                                         const float4 *__restrict__ vslot,
                                                         const float4 *__restrict__ vrev, int Kmax,
                                                         float *__restrict__ F, uint32_t *__restrict__ status, int B)
{
    const int lane = lane_id();
    const CentreRange cr = centre_range(B);
    for (int ci = cr.begin; ci < cr.end; ++ci) {
        // wave-uniform: the per-centre values below live in scalar registers
        const int i = __builtin_amdgcn_readfirstlane(order ? order[ci] : ci);
        const int K = nbr_cnt[i];
        double fx = 0.0, fy = 0.0, fz = 0.0;
        bool missing = false;
        for (int n = lane; n < K; n += kWave) {
            const float4 v = vslot[(int64_t)i * Kmax + n];
            float4 u = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if constexpr (ROWS) {
                u = vrev[(int64_t)i * Kmax + n];
            } else {
                const int j = nbr[(int64_t)i * Kmax + n] & (int)kRowMask;
                const int hit = reverse_slot(nbr, fence, Kmax, j, (__float_as_int(pos4[i].w) << kKeyShift) | i);
                if (hit >= 0)
                    u = vslot[(int64_t)j * Kmax + hit];
                else
                    missing = true;
            }
            fx += (double)v.x;
            fy += (double)v.y;
            fz += (double)v.z;
            fx -= (double)u.x;
            fy -= (double)u.y;
            fz -= (double)u.z;
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

// The same sums when no bead has more than 64 atoms (batches of small
// molecules): one lane per bead, atoms added in row order in FP64, instead of
// a 256-thread workgroup holding a few atoms.
__global__ __launch_bounds__(256) void k_bead_sums_lanes(const BeadInfo *__restrict__ beads,
                                                         const float *__restrict__ E_atom,
                                                         const float *__restrict__ vir_atom, float *__restrict__ E_bead,
                                                         float *__restrict__ W_bead, int virial, int n_beads,
                                                         uint32_t *__restrict__ status)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_beads)
        return;
    const BeadInfo bi = beads[b];
    double e = 0.0, w[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int t = 0; t < bi.n; ++t) {
        e += (double)E_atom[bi.ba0 + t];
        if (virial)
#pragma unroll
            for (int q = 0; q < 9; ++q)
                w[q] += (double)vir_atom[9 * (int64_t)(bi.ba0 + t) + q];
    }
    E_bead[b] = (float)e;
    if (!isfinite(e))
        atomicOr(status, kStatusNonFinite);
    if (virial && W_bead)
#pragma unroll
        for (int q = 0; q < 9; ++q)
            W_bead[9 * (int64_t)b + q] = (float)w[q];
}

// Work counter: neighbour pairs, j<k triplets, triplets with r_jk < rc.
__global__ __launch_bounds__(256) void k_work_counts(const float4 *__restrict__ posu,
                                                     const BeadInfo *__restrict__ beads,
                                                     const int32_t *__restrict__ bead_of_ba,
                                                     const int32_t *__restrict__ nbr,
                                                     const int32_t *__restrict__ nbr_cnt, DescParams dp,
                                                     unsigned long long *__restrict__ counts, int B)
{
    const int32_t *order = nullptr;   // counts do not depend on the centre order
    extern __shared__ float4 lds4[];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    float4 *base = lds4 + w * 3 * dp.Kmax;
    const Recs rec{base, base + dp.Kmax, base + 2 * dp.Kmax};
    unsigned long long pairs = 0, trip = 0, trip_in = 0;
    const CentreRange cr = centre_range(B);
    for (int ci = cr.begin; ci < cr.end; ++ci) {
        // wave-uniform: the per-centre values below live in scalar registers
        const int i = __builtin_amdgcn_readfirstlane(order ? order[ci] : ci);
        const BeadInfo bi = beads[bead_of_ba[i]];
        const int K = stage_neighbors<1, false>(i, posu[i], bi, nbr, nbr_cnt, posu, dp, rec,
                                                [](int, int, const float3 &, float, float, float, float, float) {});
        wave_sync();
        const int np = K * (K - 1) / 2;
        for (int t = lane; t < np; t += kWave) {
            int a, b;
            decode_triangle(t, a, b);
            const float4 Da = rec.D[a], Db = rec.D[b];
            const float jx = Db.x - Da.x, jy = Db.y - Da.y, jz = Db.z - Da.z;
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

// LDS per wave of the forward kernel: records D, E and the pair terms (16 B
// each per slot), the feature row and the pair queue.
static size_t forward_wave_bytes(const DescParams &dp)
{
    const int Dcap = (dp.D + 3) & ~3;
    return (size_t)(3 * dp.Kmax + Dcap / 4 + kQueue / 4) * sizeof(float4);
}

size_t descriptor_lds_bytes(const DescParams &dp, bool adjoint)
{
    return 4 * (adjoint ? adjoint_wave_bytes(dp) : forward_wave_bytes(dp));
}

// the attribute is the largest workgroup's (four waves); smaller ones use less
hipError_t configure_descriptor_lds(const DescParams &dp)
{
    const int f = (int)descriptor_lds_bytes(dp, false), a = (int)descriptor_lds_bytes(dp, true);
    hipError_t e = hipSuccess;
    for (const void *fn : {(const void *)k_descriptors<1, false>, (const void *)k_descriptors<2, false>,
                           (const void *)k_descriptors<2, true>})
        if (e == hipSuccess)
            e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, f);
    for (const void *fn : {(const void *)k_adjoint<1, false>, (const void *)k_adjoint<2, false>,
                           (const void *)k_adjoint<2, true>})
        if (e == hipSuccess)
            e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, a);
    return e;
}

void launch_descriptors(const DevBuffers &d, const Sizes &z, const DescParams &dp, const Tuning &tn, hipStream_t s)
{
    const int wpg = tn.centre_waves, grid = centre_grid(z.B, tn);
    const size_t lds = wpg * forward_wave_bytes(dp);
    auto kern = dp.n_ang_eta == 1 ? k_descriptors<1, false>
                : (dp.eta_pow4 ? k_descriptors<2, true> : k_descriptors<2, false>);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWave * wpg), lds, s, d.posu4, d.beads, d.bead_of_ba, centre_order(d, z),
                       d.nbr, d.nbr_cnt, d.nbr_grp, d.norm, dp, d.xhat, d.tri_pairs, d.tri_cnt, z.B);
}

void launch_adjoint(const DevBuffers &d, const Sizes &z, const DescParams &dp, const Tuning &tn, hipStream_t s)
{
    const int wpg = tn.centre_waves, grid = centre_grid(z.B, tn);
    const size_t lds = wpg * adjoint_wave_bytes(dp);
    auto kern = dp.n_ang_eta == 1 ? k_adjoint<1, false> : (dp.eta_pow4 ? k_adjoint<2, true> : k_adjoint<2, false>);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWave * wpg), lds, s, d.posu4, d.beads, d.bead_of_ba, centre_order(d, z),
                       d.nbr, d.nbr_cnt, d.dEdG, d.tri_pairs, d.tri_cnt, d.nbr_fence, dp, d.vslot,
                       tn.force_rows ? d.vrev : nullptr, d.vir_atom, d.status, z.B);
}

void launch_work_counts(const DevBuffers &d, const Sizes &z, const DescParams &dp, unsigned long long *counts,
                        hipStream_t s)
{
    const int grid = (z.B + 3) / 4 < 4096 ? (z.B + 3) / 4 : 4096;
    hipLaunchKernelGGL(k_work_counts, dim3(grid), dim3(256), (size_t)4 * 3 * dp.Kmax * sizeof(float4), s, d.posu4,
                       d.beads, d.bead_of_ba, d.nbr, d.nbr_cnt, dp, counts, z.B);
}

void launch_assemble_forces(const DevBuffers &d, const Sizes &z, float *F, const Tuning &tn, hipStream_t s)
{
    if (tn.force_rows)
        hipLaunchKernelGGL(k_assemble_forces<true>, dim3(centre_grid(z.B, tn)), dim3(kWave * tn.centre_waves), 0, s,
                           d.pos4, centre_order(d, z), d.nbr, d.nbr_cnt, d.nbr_fence, d.vslot, d.vrev, z.Kmax, F,
                           d.status, z.B);
    else
        hipLaunchKernelGGL(k_assemble_forces<false>, dim3(centre_grid(z.B, tn)), dim3(kWave * tn.centre_waves), 0, s,
                           d.pos4, centre_order(d, z), d.nbr, d.nbr_cnt, d.nbr_fence, d.vslot, nullptr, z.Kmax, F,
                           d.status, z.B);
}

void launch_bead_sums(const DevBuffers &d, const Sizes &z, float *E_bead, float *W_bead, bool virial, hipStream_t s)
{
    if (z.max_bead_atoms <= kWave)
        hipLaunchKernelGGL(k_bead_sums_lanes, dim3((z.n_beads_total + 255) / 256), dim3(256), 0, s, d.beads, d.E_atom,
                           d.vir_atom, E_bead, W_bead, virial ? 1 : 0, z.n_beads_total, d.status);
    else
        hipLaunchKernelGGL(k_bead_sums, dim3(z.n_beads_total), dim3(256), 0, s, d.beads, d.E_atom, d.vir_atom, E_bead,
                           W_bead, virial ? 1 : 0, d.status);
}

}  // namespace pimd
