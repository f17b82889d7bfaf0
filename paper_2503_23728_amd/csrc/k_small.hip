// Lane-per-centre kernels for batches of small molecules (every system
// without a box and at most kSmAtoms atoms): the descriptors (with the
// neighbour lists) and the adjoint with the force assembly.  With one wave
// per centre, a 10-atom molecule (9 neighbours, 36 slot pairs) leaves most of
// the 64 lanes idle in every phase; here one wave takes whole beads -- as
// many as fit in 64 lanes -- and every lane is one centre atom that walks
// its own bead's atoms and atom pairs in a loop that is the same for all
// lanes (unrolled to a compile-time bound, so per-atom arrays are registers),
// and the force assembly reads the reverse slot values from the partner's
// lane.  Same definitions
// as the wave-per-centre kernels (Behler-Parrinello G2/G4, cited in the
// Introduction; forces by the chain rule, the energy-model route of Sec.
// 2.2); sums run in a different order.
//
// Per lane: the records of its neighbours (d_ij and 1/r_ij; E_eta = exp(-eta
// r^2) f_c and dE_eta/dr) and, in the adjoint, the FP64 slot accumulators in
// registers; the feature row (forward) and the dE/dG row (adjoint) in LDS
// columns [feature][64 lanes], so a wave's accesses are consecutive words.
#include "device_common.hpp"
#include "neighbor_test.hpp"
#include "pair_terms.hpp"

namespace pimd {

namespace {

// Element-pair block of {a, b}: blocks enumerated (0,0), (0,1), ..., (1,1), ...
__device__ __forceinline__ int pair_block(int a, int b, int n_el)
{
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return lo * n_el - lo * (lo - 1) / 2 + (hi - lo);
}

__device__ __forceinline__ float zeta_scale(int q)
{
    const int iz = (q & 7) >> 1;   // 2^(1 - zeta) for zeta = 1, 2, 4, 8
    return iz == 0 ? 1.0f : (iz == 1 ? 0.5f : (iz == 2 ? 0.125f : 0.0078125f));
}

struct SmLane {
    bool act;
    int row, i, N;
    BeadInfo bi;
    float4 pw, pu;
};

__device__ __forceinline__ SmLane sm_lane(const SmUnit &u, const float4 *pos4, const float4 *posu4,
                                          const BeadInfo *beads, const int32_t *bead_of_ba)
{
    SmLane L;
    const int lane = threadIdx.x;
    L.act = lane < u.nrows;
    L.row = u.row0 + (L.act ? lane : 0);
    L.bi = beads[bead_of_ba[L.row]];
    L.i = L.row - L.bi.ba0;
    L.N = L.bi.n;
    L.pw = pos4[L.row];
    L.pu = posu4[L.row];
    return L;
}

}  // namespace

// Forward: neighbour lists (keys (element << 27) | row, ascending, element
// groups, fence row) and normalised descriptors.  The loops over the bead's
// atoms run to the compile-time bound NMAX and are unrolled, so the
// per-neighbour records live in registers; the feature row is a column of
// LDS that each lane only ever touches itself.
template <int NETA, int NMAX>
__global__ __launch_bounds__(64) void k_sm_forward(const float4 *__restrict__ pos4, const float4 *__restrict__ posu4,
                                                   const BeadInfo *__restrict__ beads,
                                                   const int32_t *__restrict__ bead_of_ba,
                                                   const SmUnit *__restrict__ units, const float *__restrict__ norm,
                                                   DescParams dp, int32_t *__restrict__ nbr,
                                                   int32_t *__restrict__ nbr_cnt, int32_t *__restrict__ nbr_grp,
                                                   int32_t *__restrict__ fence, float *__restrict__ xhat)
{
    extern __shared__ float sm_f[];
    const int lane = threadIdx.x;
    float4 *sw = reinterpret_cast<float4 *>(sm_f);    // [64] wrapped positions of the unit's rows
    float4 *su = sw + kWave;                          // [64] unwrapped positions
    float *G = sm_f + 8 * kWave;                      // [D][64]
    const SmUnit u = units[blockIdx.x];
    const SmLane L = sm_lane(u, pos4, posu4, beads, bead_of_ba);
    const int Frad = dp.n_el * dp.n_rad;
    const float inv_rc = 1.0f / dp.rc, inv_rc2 = 1.0f / dp.rc2;
    sw[lane] = L.pw;
    su[lane] = L.pu;
    for (int f = 0; f < dp.D; ++f)
        G[f * kWave + lane] = 0.0f;
    wave_sync();
    const int lane0 = lane - L.i;   // lane of atom 0 of this bead
    // pass 1: membership, pair records, radial functions
    float4 rD[NMAX];
    float2 rE[NMAX];
    uint32_t inr = 0u, epack = 0u;
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        rD[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        rE[j] = make_float2(0.0f, 0.0f);
        if (!L.act || j >= L.N || j == L.i)
            continue;
        const float4 qw = sw[lane0 + j];
        if (!within_cutoff(L.pw, qw, L.bi, dp.rc2))
            continue;
        const int ej = __float_as_int(qw.w);
        inr |= 1u << j;
        epack |= (uint32_t)ej << (2 * j);
        float3 d;
        float r, r_lo, inv_r;
        displacement(L.pu, su[lane0 + j], L.bi, d, r, r_lo, inv_r);
        float fc, dfc;
        cutoff_fn(r * inv_rc, dp.pi_over_rc, fc, dfc);
        for (int s = 0; s < dp.n_rad; ++s) {
            const float x = (r - dp.rad_center[s]) + (r_lo - dp.rad_center_lo[s]);
            G[(ej * dp.n_rad + s) * kWave + lane] += exp2_hw(-dp.rad_eta[s] * kLog2e * x * x) * fc;
        }
        const float r2 = r * r;
        rD[j] = make_float4(d.x, d.y, d.z, inv_r);
        rE[j] = make_float2(exp2_hw(-dp.ang_eta[0] * kLog2e * r2) * fc,
                            NETA > 1 ? exp2_hw(-dp.ang_eta[1] * kLog2e * r2) * fc : 0.0f);
    }
    // neighbour list in key order: by element, then row
    if (L.act) {
        int32_t *out = nbr + (int64_t)L.row * dp.Kmax;
        int cnt = 0;
        for (int e = 0; e < dp.n_el; ++e) {
            int grp = 0;
#pragma unroll
            for (int j = 0; j < NMAX; ++j)
                if (((inr >> j) & 1u) && (int)((epack >> (2 * j)) & 3u) == e) {
                    out[cnt++] = (e << kKeyShift) | (L.bi.ba0 + j);
                    ++grp;
                }
            nbr_grp[(int64_t)L.row * kMaxElements + e] = grp;
        }
        nbr_cnt[L.row] = cnt;
        fence[(int64_t)L.row * kFence] = cnt;   // at most NMAX - 1 < 16 slots: no other fence entries
        for (int m = 1; m < kFence; ++m)
            fence[(int64_t)L.row * kFence + m] = 0x7FFFFFFF;
    }
    // pass 2: angular terms of every in-range pair (j < k) with r_jk < rc
    const float nel0 = -dp.ang_eta[0] * 1.4426950408889634f, nel1 = -dp.ang_eta[1] * 1.4426950408889634f;
#pragma unroll
    for (int j = 0; j + 1 < NMAX; ++j) {
#pragma unroll
        for (int k = j + 1; k < NMAX; ++k) {
            if (!((inr >> j) & (inr >> k) & 1u))
                continue;
            const float4 A = rD[j], C = rD[k];
            const float jx = C.x - A.x, jy = C.y - A.y, jz = C.z - A.z;
            const float r2jk = jx * jx + jy * jy + jz * jz;
            if (!(r2jk < dp.rc2))
                continue;
            const int ej = (int)((epack >> (2 * j)) & 3u), ek = (int)((epack >> (2 * k)) & 3u);
            float *gb = G + (Frad + pair_block(ej, ek, dp.n_el) * dp.n_ang) * kWave + lane;
            const float fcjk = cutoff_sq_fc(r2jk * inv_rc2);
            const float cs = (A.x * C.x + A.y * C.y + A.z * C.z) * (A.w * C.w);
            const float p1 = 1.0f + cs, m1 = 1.0f - cs;
            const float p2 = p1 * p1, m2 = m1 * m1;
            const float p4 = p2 * p2, m4 = m2 * m2;
            const float p8 = p4 * p4, m8 = m4 * m4;
#pragma unroll
            for (int ie = 0; ie < NETA; ++ie) {
                const float Ea = ie == 0 ? rE[j].x : rE[j].y, Eb = ie == 0 ? rE[k].x : rE[k].y;
                const float R = Ea * Eb * __builtin_amdgcn_exp2f((ie == 0 ? nel0 : nel1) * r2jk) * fcjk;
                float *g = gb + ie * 8 * kWave;
                g[0 * kWave] += p1 * R;
                g[1 * kWave] += m1 * R;
                g[2 * kWave] += p2 * R;
                g[3 * kWave] += m2 * R;
                g[4 * kWave] += p4 * R;
                g[5 * kWave] += m4 * R;
                g[6 * kWave] += p8 * R;
                g[7 * kWave] += m8 * R;
            }
        }
    }
    if (!L.act)
        return;
    wave_sync();
    const int zi = __float_as_int(L.pw.w);
    const float *shift = norm + (int64_t)zi * 2 * dp.D;
    const float *inv_scale = shift + dp.D;
    for (int f = 0; f < dp.D; ++f) {
        const float sc = f < Frad ? 1.0f : zeta_scale((f - Frad) % dp.n_ang);
        xhat[(int64_t)L.row * dp.D + f] = (G[f * kWave + lane] * sc - shift[f]) * inv_scale[f];
    }
}

// Adjoint with the force assembly: v_ij = dE_i/d d_ij accumulated per slot
// in FP64 registers (unrolled loops over the bead's atoms), then
//   F_i = sum_j v_ij - sum_j v_ji   (v_ji read from the lane of atom j
// through LDS, float32 values summed in FP64 as in the general assembly),
// the per-atom virial -sum_j d_ij (x) v_ij, and the slot values in list
// order (the debug slot buffer).  F may be null (virial only).
template <int NETA, int NMAX>
__global__ __launch_bounds__(64) void k_sm_adjoint(const float4 *__restrict__ pos4, const float4 *__restrict__ posu4,
                                                   const BeadInfo *__restrict__ beads,
                                                   const int32_t *__restrict__ bead_of_ba,
                                                   const SmUnit *__restrict__ units, const float *__restrict__ dEdG,
                                                   DescParams dp, float4 *__restrict__ vslot,
                                                   float *__restrict__ F, float *__restrict__ vir_atom)
{
    extern __shared__ float sm_f[];
    const int lane = threadIdx.x;
    float4 *sw = reinterpret_cast<float4 *>(sm_f);    // [64] wrapped positions of the unit's rows
    float4 *su = sw + kWave;                          // [64] unwrapped positions
    float *g = sm_f + 8 * kWave;                      // [D][64] dE/dG rows
    float *vx = g + dp.D * kWave;                     // [NMAX][3][64] slot values for the exchange
    const SmUnit u = units[blockIdx.x];
    const SmLane L = sm_lane(u, pos4, posu4, beads, bead_of_ba);
    const int Frad = dp.n_el * dp.n_rad;
    const float inv_rc = 1.0f / dp.rc, inv_rc2 = 1.0f / dp.rc2;
    sw[lane] = L.pw;
    su[lane] = L.pu;
    if (L.act)
        for (int f = 0; f < dp.D; ++f)
            g[f * kWave + lane] = dEdG[(int64_t)L.row * dp.D + f];
    wave_sync();
    const int lane0 = lane - L.i;   // lane of atom 0 of this bead
    // pass 1: records and the radial part of every slot
    float4 rD[NMAX], rE[NMAX];
    double v[NMAX][3];
    uint32_t inr = 0u, epack = 0u;
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        v[j][0] = v[j][1] = v[j][2] = 0.0;
        rD[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        rE[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (!L.act || j >= L.N || j == L.i)
            continue;
        const float4 qw = sw[lane0 + j];
        if (!within_cutoff(L.pw, qw, L.bi, dp.rc2))
            continue;
        const int ej = __float_as_int(qw.w);
        inr |= 1u << j;
        epack |= (uint32_t)ej << (2 * j);
        float3 d;
        float r, r_lo, inv_r;
        displacement(L.pu, su[lane0 + j], L.bi, d, r, r_lo, inv_r);
        float fc, dfc;
        cutoff_fn(r * inv_rc, dp.pi_over_rc, fc, dfc);
        float acc = 0.0f;
        for (int t = 0; t < dp.n_rad; ++t) {
            const float4 rp = dp.rad_pack[t];
            const float x = (r - rp.x) + (r_lo - rp.y);
            acc += g[(ej * dp.n_rad + t) * kWave + lane] * exp2_hw(rp.z * x * x) * (rp.w * x * fc + dfc);
        }
        const float c = acc * inv_r;
        v[j][0] = (double)(c * d.x);
        v[j][1] = (double)(c * d.y);
        v[j][2] = (double)(c * d.z);
        const float r2 = r * r;
        const float g0 = exp2_hw(-dp.ang_eta[0] * kLog2e * r2);
        const float g1 = NETA > 1 ? exp2_hw(-dp.ang_eta[1] * kLog2e * r2) : 0.0f;
        rD[j] = make_float4(d.x, d.y, d.z, inv_r);
        rE[j] = make_float4(g0 * fc, g1 * fc, g0 * (-2.0f * dp.ang_eta[0] * r * fc + dfc),
                            NETA > 1 ? g1 * (-2.0f * dp.ang_eta[1] * r * fc + dfc) : 0.0f);
    }
    // pass 2: triplets
    const float nel0 = -dp.ang_eta[0] * 1.4426950408889634f, nel1 = -dp.ang_eta[1] * 1.4426950408889634f;
#pragma unroll
    for (int j = 0; j + 1 < NMAX; ++j) {
#pragma unroll
        for (int k = j + 1; k < NMAX; ++k) {
            if (!((inr >> j) & (inr >> k) & 1u))
                continue;
            const float4 A = rD[j], C = rD[k], Ae = rE[j], Ce = rE[k];
            const float jx = C.x - A.x, jy = C.y - A.y, jz = C.z - A.z;
            const float r2jk = jx * jx + jy * jy + jz * jz;
            if (!(r2jk < dp.rc2))
                continue;
            const int ej = (int)((epack >> (2 * j)) & 3u), ek = (int)((epack >> (2 * k)) & 3u);
            const float *gb = g + (Frad + pair_block(ej, ek, dp.n_el) * dp.n_ang) * kWave + lane;
            // dfcjk = (1/r_jk) d f_c/d r_jk
            float fcjk, dfcjk;
            cutoff_sq(r2jk * inv_rc2, fcjk, dfcjk);
            dfcjk *= 2.0f * inv_rc2;
            const float iab = A.w * C.w;
            const float cs = (A.x * C.x + A.y * C.y + A.z * C.z) * iab;
            const float p1 = 1.0f + cs, m1 = 1.0f - cs;
            const float p2 = p1 * p1, m2 = m1 * m1;
            const float p3 = p2 * p1, m3 = m2 * m1;
            const float p4 = p2 * p2, m4 = m2 * m2;
            const float p7 = p4 * p3, m7 = m4 * m3;
            const float p8 = p4 * p4, m8 = m4 * m4;
            float Pc = 0.0f, Pa = 0.0f, Pb = 0.0f, Pjk = 0.0f;
#pragma unroll
            for (int ie = 0; ie < NETA; ++ie) {
                float gq[8];
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    gq[q] = gb[(ie * 8 + q) * kWave] * zeta_scale(q);
                const float S = gq[0] * p1 + gq[1] * m1 + gq[2] * p2 + gq[3] * m2 + gq[4] * p4 + gq[5] * m4 +
                                gq[6] * p8 + gq[7] * m8;
                const float Sd = (gq[0] - gq[1]) + 2.0f * gq[2] * p1 - 2.0f * gq[3] * m1 + 4.0f * gq[4] * p3 -
                                 4.0f * gq[5] * m3 + 8.0f * gq[6] * p7 - 8.0f * gq[7] * m7;
                const float X = __builtin_amdgcn_exp2f((ie == 0 ? nel0 : nel1) * r2jk);
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
            // dE/d d_ij = ka d_ij + kb d_ik,  dE/d d_ik = kc d_ik + kb d_ij
            const float ia_ = A.w, ib_ = C.w;
            const float Pcs = Pc * cs;
            const float gam = Pjk;
            const float ka = (Pa - Pcs * ia_) * ia_ + gam;
            const float kc = (Pb - Pcs * ib_) * ib_ + gam;
            const float kb = Pc * iab - gam;
            v[j][0] += (double)(ka * A.x + kb * C.x);
            v[j][1] += (double)(ka * A.y + kb * C.y);
            v[j][2] += (double)(ka * A.z + kb * C.z);
            v[k][0] += (double)(kc * C.x + kb * A.x);
            v[k][1] += (double)(kc * C.y + kb * A.y);
            v[k][2] += (double)(kc * C.z + kb * A.z);
        }
    }
    // slot values as float32 (what the general assembly sums), shared through LDS
    float vf[NMAX][3];
#pragma unroll
    for (int j = 0; j < NMAX; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            vf[j][c] = (float)v[j][c];
            vx[(j * 3 + c) * kWave + lane] = vf[j][c];
        }
    wave_sync();
    if (!L.act)
        return;
    // forces: own slot values minus the partners' values at this atom's slot
    double f[3] = {0.0, 0.0, 0.0}, W[9];
#pragma unroll
    for (int q = 0; q < 9; ++q)
        W[q] = 0.0;
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        if (j >= L.N || j == L.i)
            continue;
        const float *vji = vx + (L.i * 3) * kWave + lane0 + j;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            f[c] += (double)vf[j][c] - (double)vji[c * kWave];
        const double dd[3] = {(double)rD[j].x, (double)rD[j].y, (double)rD[j].z};
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = 0; q < 3; ++q)
                W[3 * p + q] -= dd[p] * (double)vf[j][q];
    }
    if (F) {
        F[3 * (int64_t)L.row + 0] = (float)f[0];
        F[3 * (int64_t)L.row + 1] = (float)f[1];
        F[3 * (int64_t)L.row + 2] = (float)f[2];
    }
#pragma unroll
    for (int q = 0; q < 9; ++q)
        vir_atom[9 * (int64_t)L.row + q] = (float)W[q];
    // slot values in list order (by element, then row)
    int n = 0;
    for (int e = 0; e < dp.n_el; ++e)
#pragma unroll
        for (int j = 0; j < NMAX; ++j)
            if (((inr >> j) & 1u) && (int)((epack >> (2 * j)) & 3u) == e)
                vslot[(int64_t)L.row * dp.Kmax + n++] = make_float4(vf[j][0], vf[j][1], vf[j][2], 0.0f);
}

size_t sm_forward_lds_bytes(const DescParams &dp) { return (size_t)(8 + dp.D) * kWave * sizeof(float); }

size_t sm_adjoint_lds_bytes(const DescParams &dp, int nmax)
{
    return (size_t)(8 + dp.D + 3 * nmax) * kWave * sizeof(float);
}

// the atom bound of the unrolled loops: 12 or 16
static int sm_bound(int nmax) { return nmax <= 12 ? 12 : 16; }

hipError_t configure_sm_lds(const DescParams &dp)
{
    const int f = (int)sm_forward_lds_bytes(dp), a = (int)sm_adjoint_lds_bytes(dp, kSmAtoms);
    hipError_t e = hipSuccess;
    for (const void *fn : {(const void *)k_sm_forward<1, 12>, (const void *)k_sm_forward<2, 12>,
                           (const void *)k_sm_forward<1, 16>, (const void *)k_sm_forward<2, 16>})
        if (e == hipSuccess)
            e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, f);
    for (const void *fn : {(const void *)k_sm_adjoint<1, 12>, (const void *)k_sm_adjoint<2, 12>,
                           (const void *)k_sm_adjoint<1, 16>, (const void *)k_sm_adjoint<2, 16>})
        if (e == hipSuccess)
            e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, a);
    return e;
}

void launch_sm_forward(const DevBuffers &d, const DescParams &dp, int n_units, int nmax, hipStream_t s)
{
    const size_t lds = sm_forward_lds_bytes(dp);
    const bool two = dp.n_ang_eta == 2, wide = sm_bound(nmax) == 16;
    auto kern = two ? (wide ? k_sm_forward<2, 16> : k_sm_forward<2, 12>)
                    : (wide ? k_sm_forward<1, 16> : k_sm_forward<1, 12>);
    hipLaunchKernelGGL(kern, dim3(n_units), dim3(kWave), lds, s, d.pos4, d.posu4, d.beads, d.bead_of_ba, d.sm_units,
                       d.norm, dp, d.nbr, d.nbr_cnt, d.nbr_grp, d.nbr_fence, d.xhat);
}

void launch_sm_adjoint(const DevBuffers &d, const DescParams &dp, int n_units, int nmax, float *F, hipStream_t s)
{
    const int bound = sm_bound(nmax);
    const size_t lds = sm_adjoint_lds_bytes(dp, bound);
    const bool two = dp.n_ang_eta == 2, wide = bound == 16;
    auto kern = two ? (wide ? k_sm_adjoint<2, 16> : k_sm_adjoint<2, 12>)
                    : (wide ? k_sm_adjoint<1, 16> : k_sm_adjoint<1, 12>);
    hipLaunchKernelGGL(kern, dim3(n_units), dim3(kWave), lds, s, d.pos4, d.posu4, d.beads, d.bead_of_ba, d.sm_units,
                       d.dEdG, dp, d.vslot, F, d.vir_atom);
}

}  // namespace pimd
