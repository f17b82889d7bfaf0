// Direct-force head in the graph-field-network form (Sec. 2.2): forces are
// read out per edge from edge representations that exchange messages with
// node representations, without differentiating an energy.
//
//   rho_s(r)   = exp(-eta_s (r - R_s)^2) f_c(r)
//   e_ij^(0)   = W_r rho(r_ij) + b[Z_i][Z_j],   n_i^(0) = a[Z_i]
//   m_i^(l)    = sum_j phi_msg^(l)(e_ij^(l))
//   n_i^(l+1)  = n_i^(l) + phi_node^(l)([n_i^(l); m_i^(l)])
//   e_ij^(l+1) = e_ij^(l) + phi_edge^(l)(n_i^(l) + n_j^(l))
//   F_i        = sum_j f_c(r_ij) d_ij / r_ij phi_f(e_ij^(L))
//
// One wave per centre, a lane per neighbour slot, in the centre order of the
// energy model's kernels.  Edge representations are never stored: a layer
// kernel rebuilds e_ij^(l) from the radial basis and the stored node states
// n^(0..l-1) (B x H floats each), and the readout kernel rebuilds e_ij^(L).
// The small per-edge MLPs run on the VALU with their weights as wave-uniform
// (scalar) operands.
#include "device_common.hpp"
#include "pair_terms.hpp"

namespace pimd {

__device__ __forceinline__ float tanh_stable(float a)
{
    const float e = expf(-2.0f * fabsf(a));
    return copysignf((1.0f - e) / (1.0f + e), a);
}

// y = W2 tanh(W1 x + b1) + b2, W1 [H][IN], W2 [H][H]
template <int H, int IN>
__device__ __forceinline__ void gfn_mlp(const GfnMlp &p, const float (&x)[IN], float (&y)[H])
{
    float h[H];
#pragma unroll
    for (int o = 0; o < H; ++o) {
        float a = p.b1[o];
#pragma unroll
        for (int k = 0; k < IN; ++k)
            a = fmaf(p.W1[o * IN + k], x[k], a);
        h[o] = tanh_stable(a);
    }
#pragma unroll
    for (int o = 0; o < H; ++o) {
        float a = p.b2[o];
#pragma unroll
        for (int k = 0; k < H; ++k)
            a = fmaf(p.W2[o * H + k], h[k], a);
        y[o] = a;
    }
}

template <int H>
__device__ __forceinline__ void load_node(const float *nodes, int64_t row, float (&n)[H])
{
    const float4 *src = reinterpret_cast<const float4 *>(nodes + row * H);
#pragma unroll
    for (int c = 0; c < H / 4; ++c) {
        const float4 v = src[c];
        n[4 * c] = v.x;
        n[4 * c + 1] = v.y;
        n[4 * c + 2] = v.z;
        n[4 * c + 3] = v.w;
    }
}

// e_ij^(l) of one edge: the radial basis and pair embedding, then the edge
// updates of layers 0 .. l-1 from the stored node states.
template <int H>
__device__ __forceinline__ void edge_state(const DescParams &dp, const GfnParams &gp, const float *nodes, int B,
                                           int l, int zi, int zj, int i, int j, float r, float r_lo, float fc,
                                           float (&e)[H])
{
    const float *pe = gp.pair_embed + ((int64_t)zi * dp.n_el + zj) * H;
#pragma unroll
    for (int h = 0; h < H; ++h)
        e[h] = pe[h];
    for (int s = 0; s < dp.n_rad; ++s) {
        // r - R_s from the two-float r and R_s, as in the radial symmetry functions
        const float x = (r - dp.rad_center[s]) + (r_lo - dp.rad_center_lo[s]);
        const float rho = expf(-dp.rad_eta[s] * x * x) * fc;
#pragma unroll
        for (int h = 0; h < H; ++h)
            e[h] = fmaf(gp.edge_in[h * dp.n_rad + s], rho, e[h]);
    }
    for (int lp = 0; lp < l; ++lp) {
        float ni[H], nj[H], x[H], u[H];
        load_node<H>(nodes + (int64_t)lp * B * H, i, ni);
        load_node<H>(nodes + (int64_t)lp * B * H, j, nj);
#pragma unroll
        for (int h = 0; h < H; ++h)
            x[h] = ni[h] + nj[h];
        gfn_mlp<H, H>(gp.edge[lp], x, u);
#pragma unroll
        for (int h = 0; h < H; ++h)
            e[h] += u[h];
    }
}

// Layer l: m_i = sum_j phi_msg(e_ij^(l)), n_i^(l+1) = n_i^(l) + phi_node([n_i^(l); m_i]).
template <int H>
__global__ __launch_bounds__(256) void k_gfn_layer(const float4 *__restrict__ posu, const BeadInfo *__restrict__ beads,
                                                   const int32_t *__restrict__ bead_of_ba,
                                                   const int32_t *__restrict__ order,
                                                   const int32_t *__restrict__ nbr,
                                                   const int32_t *__restrict__ nbr_cnt, DescParams dp, GfnParams gp,
                                                   float *__restrict__ nodes, int l, int B)
{
    const int lane = lane_id();
    const CentreRange cr = centre_range(B);
    for (int ci = cr.begin; ci < cr.end; ++ci) {
        const int i = __builtin_amdgcn_readfirstlane(order ? order[ci] : ci);
        const BeadInfo bi = beads[bead_of_ba[i]];
        const float4 pi = posu[i];
        const int zi = __float_as_int(pi.w);
        const int K = nbr_cnt[i];
        const int32_t *row = nbr + (int64_t)i * dp.Kmax;
        float macc[H];
#pragma unroll
        for (int h = 0; h < H; ++h)
            macc[h] = 0.0f;
        for (int n = lane; n < K; n += kWave) {
            const int key = row[n];
            const int j = key & (int)kRowMask, zj = key >> kKeyShift;
            float3 d;
            float r, r_lo, inv_r, fc, dfc;
            displacement(pi, posu[j], bi, d, r, r_lo, inv_r);
            cutoff_fn(r * (1.0f / dp.rc), dp.pi_over_rc, fc, dfc);
            float e[H], msg[H];
            edge_state<H>(dp, gp, nodes, B, l, zi, zj, i, j, r, r_lo, fc, e);
            gfn_mlp<H, H>(gp.msg[l], e, msg);
#pragma unroll
            for (int h = 0; h < H; ++h)
                macc[h] += msg[h];
        }
        float ni[H], x[2 * H], upd[H];
        load_node<H>(nodes + (int64_t)l * B * H, i, ni);
#pragma unroll
        for (int h = 0; h < H; ++h) {
            x[h] = ni[h];
            x[H + h] = wave_sum(macc[h]);
        }
        gfn_mlp<H, 2 * H>(gp.node[l], x, upd);
        if (lane == 0) {
            float4 *dst = reinterpret_cast<float4 *>(nodes + ((int64_t)(l + 1) * B + i) * H);
#pragma unroll
            for (int c = 0; c < H / 4; ++c)
                dst[c] = make_float4(x[4 * c] + upd[4 * c], x[4 * c + 1] + upd[4 * c + 1],
                                     x[4 * c + 2] + upd[4 * c + 2], x[4 * c + 3] + upd[4 * c + 3]);
        }
    }
}

// Readout: F_i = sum_j f_c(r_ij) d_ij / r_ij phi_f(e_ij^(L)), summed in FP64;
// the atomic energies and virials of the head are zero.
template <int H>
__global__ __launch_bounds__(256) void k_gfn_forces(const float4 *__restrict__ posu,
                                                    const BeadInfo *__restrict__ beads,
                                                    const int32_t *__restrict__ bead_of_ba,
                                                    const int32_t *__restrict__ order,
                                                    const int32_t *__restrict__ nbr,
                                                    const int32_t *__restrict__ nbr_cnt, DescParams dp,
                                                    GfnParams gp, const float *__restrict__ nodes,
                                                    float *__restrict__ F, float *__restrict__ E_atom,
                                                    float *__restrict__ vir_atom, int B)
{
    const int lane = lane_id();
    const CentreRange cr = centre_range(B);
    for (int ci = cr.begin; ci < cr.end; ++ci) {
        const int i = __builtin_amdgcn_readfirstlane(order ? order[ci] : ci);
        const BeadInfo bi = beads[bead_of_ba[i]];
        const float4 pi = posu[i];
        const int zi = __float_as_int(pi.w);
        const int K = nbr_cnt[i];
        const int32_t *row = nbr + (int64_t)i * dp.Kmax;
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int n = lane; n < K; n += kWave) {
            const int key = row[n];
            const int j = key & (int)kRowMask, zj = key >> kKeyShift;
            float3 d;
            float r, r_lo, inv_r, fc, dfc;
            displacement(pi, posu[j], bi, d, r, r_lo, inv_r);
            cutoff_fn(r * (1.0f / dp.rc), dp.pi_over_rc, fc, dfc);
            float e[H];
            edge_state<H>(dp, gp, nodes, B, gp.L, zi, zj, i, j, r, r_lo, fc, e);
            float s = gp.fb2;
#pragma unroll
            for (int o = 0; o < H; ++o) {
                float a = gp.fb1[o];
#pragma unroll
                for (int k = 0; k < H; ++k)
                    a = fmaf(gp.fW1[o * H + k], e[k], a);
                s = fmaf(gp.fw2[o], tanh_stable(a), s);
            }
            const float c = fc * s * inv_r;
            fx += (double)(c * d.x);
            fy += (double)(c * d.y);
            fz += (double)(c * d.z);
        }
        fx = wave_sum_f64(fx);
        fy = wave_sum_f64(fy);
        fz = wave_sum_f64(fz);
        if (lane == 0) {
            F[3 * (int64_t)i + 0] = (float)fx;
            F[3 * (int64_t)i + 1] = (float)fy;
            F[3 * (int64_t)i + 2] = (float)fz;
            E_atom[i] = 0.0f;
        }
        if (lane < 9)
            vir_atom[(int64_t)i * 9 + lane] = 0.0f;
    }
}

// ---------------------------------------------------------------------------
// The same head with the per-edge matrix products on MFMA
// (v_mfma_f32_16x16x16bf16_1k, FP32 accumulation; BF16 operands as a
// three-term hi/lo split or rounded once).  A centre's edges are taken 16 at
// a time as the columns of a tile; every per-edge vector is held in the MFMA
// layout, lane (lr = lane & 15, lg = lane >> 4) holding features
// 16 b + 4 lg .. 16 b + 4 lg + 3 of edge lr for each 16-row block b.  That is
// the layout of both a product's result and its B operand, so the two layers
// of each small MLP chain without moving data.  Weights arrive as bfloat16
// tiles already in A-operand order: tile (ob, kb) holds, per lane, the four
// k = 16 kb + 4 lg .. + 3 of row 16 ob + lr, hi parts then lo parts.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef short i16x8 __attribute__((ext_vector_type(8)));

template <int MODE>
__device__ __forceinline__ void split4(const f32x4 &v, i16x4 &hi, i16x4 &lo)
{
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const __bf16 h = (__bf16)v[q];
        hi[q] = __builtin_bit_cast(short, h);
        lo[q] = MODE == 1 ? __builtin_bit_cast(short, (__bf16)(v[q] - (float)h)) : (short)0;
    }
}

// acc + W[16 ob .. 16 ob + 15][all k] x B, the k-blocks of B given in parts.
template <int MODE, int KB>
__device__ __forceinline__ f32x4 mma_rows(const uint16_t *tiles, int ob, const i16x4 (&bh)[KB],
                                          const i16x4 (&bl)[KB], f32x4 acc)
{
    const int lane = lane_id();
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const i16x8 w = *reinterpret_cast<const i16x8 *>(tiles + ((int64_t)(ob * KB + kb) * kWave + lane) * 8);
        const i16x4 ah = {w[0], w[1], w[2], w[3]};
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh[kb], acc, 0, 0, 0);
        if (MODE == 1) {
            const i16x4 al = {w[4], w[5], w[6], w[7]};
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh[kb], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl[kb], acc, 0, 0, 0);
        }
    }
    return acc;
}

__device__ __forceinline__ f32x4 load4(const float *p)
{
    const float4 v = *reinterpret_cast<const float4 *>(p);
    return f32x4{v.x, v.y, v.z, v.w};
}

// y = W2 tanh(W1 x + b1) + b2 for the 16 edges of a tile (HB = H / 16).
template <int MODE, int HB>
__device__ __forceinline__ void mlp_tile(const uint16_t *t1, const float *b1, const uint16_t *t2, const float *b2,
                                         const f32x4 (&x)[HB], f32x4 (&y)[HB])
{
    const int lg = lane_id() >> 4;
    i16x4 xh[HB], xl[HB];
#pragma unroll
    for (int b = 0; b < HB; ++b)
        split4<MODE>(x[b], xh[b], xl[b]);
    f32x4 h[HB];
#pragma unroll
    for (int ob = 0; ob < HB; ++ob) {
        f32x4 a = mma_rows<MODE, HB>(t1, ob, xh, xl, load4(b1 + 16 * ob + 4 * lg));
#pragma unroll
        for (int q = 0; q < 4; ++q)
            a[q] = tanh_stable(a[q]);
        h[ob] = a;
    }
#pragma unroll
    for (int b = 0; b < HB; ++b)
        split4<MODE>(h[b], xh[b], xl[b]);
#pragma unroll
    for (int ob = 0; ob < HB; ++ob)
        y[ob] = mma_rows<MODE, HB>(t2, ob, xh, xl, load4(b2 + 16 * ob + 4 * lg));
}

// One edge of a tile per lane column: the pair terms (an edge past the
// centre's count gets f_c = 0 and a unit direction, so its column stays finite).
struct TileEdge {
    int j, zj;
    bool valid;
    float3 d;
    float r, r_lo, inv_r, fc;
};

__device__ __forceinline__ TileEdge tile_edge(const float4 &pi, const BeadInfo &bi, const float4 *posu,
                                              const int32_t *row, int K, int n, int i, const DescParams &dp)
{
    TileEdge te;
    te.valid = n < K;
    if (te.valid) {
        const int key = row[n];
        te.j = key & (int)kRowMask;
        te.zj = key >> kKeyShift;
        float dfc;
        displacement(pi, posu[te.j], bi, te.d, te.r, te.r_lo, te.inv_r);
        cutoff_fn(te.r * (1.0f / dp.rc), dp.pi_over_rc, te.fc, dfc);
    } else {
        te.j = i;
        te.zj = 0;
        te.d = make_float3(dp.rc, 0.0f, 0.0f);
        te.r = dp.rc;
        te.r_lo = 0.0f;
        te.inv_r = 1.0f / dp.rc;
        te.fc = 0.0f;
    }
    return te;
}

// e_ij^(l) of the tile's edges in the MFMA layout (RB = 16-blocks of the radial basis).
template <int MODE, int HB, int RB>
__device__ __forceinline__ void edge_state_tile(const DescParams &dp, const GfnParams &gp, const float *nodes, int B,
                                                int l, int zi, int i, const TileEdge &te, f32x4 (&e)[HB])
{
    constexpr int H = 16 * HB;
    const int lg = lane_id() >> 4;
    i16x4 rh[RB], rl[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        f32x4 rho;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int sidx = 16 * rb + 4 * lg + q;
            float v = 0.0f;
            if (sidx < dp.n_rad) {
                const float x = (te.r - dp.rad_center[sidx]) + (te.r_lo - dp.rad_center_lo[sidx]);
                v = expf(-dp.rad_eta[sidx] * x * x) * te.fc;
            }
            rho[q] = v;
        }
        split4<MODE>(rho, rh[rb], rl[rb]);
    }
    const float *pe = gp.pair_embed + ((int64_t)zi * dp.n_el + te.zj) * H;
#pragma unroll
    for (int ob = 0; ob < HB; ++ob)
        e[ob] = mma_rows<MODE, RB>(gp.t_in, ob, rh, rl, load4(pe + 16 * ob + 4 * lg));
    for (int lp = 0; lp < l; ++lp) {
        const float *nl = nodes + (int64_t)lp * B * H;
        f32x4 x[HB], u[HB];
#pragma unroll
        for (int b = 0; b < HB; ++b)
            x[b] = load4(nl + (int64_t)i * H + 16 * b + 4 * lg) + load4(nl + (int64_t)te.j * H + 16 * b + 4 * lg);
        mlp_tile<MODE, HB>(gp.t_edge1[lp], gp.edge[lp].b1, gp.t_edge2[lp], gp.edge[lp].b2, x, u);
#pragma unroll
        for (int b = 0; b < HB; ++b)
            e[b] += u[b];
    }
}

template <int MODE, int HB, int RB>
__global__ __launch_bounds__(256) void k_gfn_layer_mma(const float4 *__restrict__ posu,
                                                       const BeadInfo *__restrict__ beads,
                                                       const int32_t *__restrict__ bead_of_ba,
                                                       const int32_t *__restrict__ order,
                                                       const int32_t *__restrict__ nbr,
                                                       const int32_t *__restrict__ nbr_cnt, DescParams dp,
                                                       GfnParams gp, float *__restrict__ nodes, int l, int B)
{
    constexpr int H = 16 * HB;
    const int lane = lane_id(), lr = lane & 15, lg = lane >> 4;
    const CentreRange cr = centre_range(B);
    for (int ci = cr.begin; ci < cr.end; ++ci) {
        const int i = __builtin_amdgcn_readfirstlane(order ? order[ci] : ci);
        const BeadInfo bi = beads[bead_of_ba[i]];
        const float4 pi = posu[i];
        const int zi = __float_as_int(pi.w);
        const int K = nbr_cnt[i];
        const int32_t *row = nbr + (int64_t)i * dp.Kmax;
        f32x4 macc[HB];
#pragma unroll
        for (int b = 0; b < HB; ++b)
            macc[b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int t0 = 0; t0 < K; t0 += 16) {
            const TileEdge te = tile_edge(pi, bi, posu, row, K, t0 + lr, i, dp);
            f32x4 e[HB], msg[HB];
            edge_state_tile<MODE, HB, RB>(dp, gp, nodes, B, l, zi, i, te, e);
            mlp_tile<MODE, HB>(gp.t_msg1[l], gp.msg[l].b1, gp.t_msg2[l], gp.msg[l].b2, e, msg);
#pragma unroll
            for (int b = 0; b < HB; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    macc[b][q] += te.valid ? msg[b][q] : 0.0f;
        }
        // m_i: sum over the 16 edge columns, then every lane gathers all H features
        float x[2 * H];
        load_node<H>(nodes + (int64_t)l * B * H, i, *reinterpret_cast<float(*)[H]>(x));
#pragma unroll
        for (int b = 0; b < HB; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float v = row16_sum(macc[b][q]);
#pragma unroll
                for (int g = 0; g < 4; ++g)
                    x[H + 16 * b + 4 * g + q] = __shfl(v, 16 * g, kWave);
            }
        // node update n_i + W2 tanh(W1 [n_i; m_i] + b1) + b2 with lane o (mod H)
        // computing output o of each layer (the hidden values pass by shuffles)
        const int o = lane & (H - 1);
        const GfnMlp &nm = gp.node[l];
        float a = nm.b1[o];
#pragma unroll
        for (int k = 0; k < 2 * H; k += 4) {
            const float4 w = *reinterpret_cast<const float4 *>(nm.W1 + o * 2 * H + k);
            a = fmaf(w.x, x[k], a);
            a = fmaf(w.y, x[k + 1], a);
            a = fmaf(w.z, x[k + 2], a);
            a = fmaf(w.w, x[k + 3], a);
        }
        const float hid = tanh_stable(a);
        float y = nm.b2[o];
#pragma unroll
        for (int k = 0; k < H; k += 4) {
            const float4 w = *reinterpret_cast<const float4 *>(nm.W2 + o * H + k);
            y = fmaf(w.x, __shfl(hid, k, kWave), y);
            y = fmaf(w.y, __shfl(hid, k + 1, kWave), y);
            y = fmaf(w.z, __shfl(hid, k + 2, kWave), y);
            y = fmaf(w.w, __shfl(hid, k + 3, kWave), y);
        }
        float xo = x[0];
#pragma unroll
        for (int k = 1; k < H; ++k)
            xo = o == k ? x[k] : xo;
        if (lane < H)
            nodes[((int64_t)(l + 1) * B + i) * H + o] = xo + y;
        (void)lg;
    }
}

template <int MODE, int HB, int RB>
__global__ __launch_bounds__(256) void k_gfn_forces_mma(const float4 *__restrict__ posu,
                                                        const BeadInfo *__restrict__ beads,
                                                        const int32_t *__restrict__ bead_of_ba,
                                                        const int32_t *__restrict__ order,
                                                        const int32_t *__restrict__ nbr,
                                                        const int32_t *__restrict__ nbr_cnt, DescParams dp,
                                                        GfnParams gp, const float *__restrict__ nodes,
                                                        float *__restrict__ F, float *__restrict__ E_atom,
                                                        float *__restrict__ vir_atom, int B)
{
    const int lane = lane_id(), lr = lane & 15, lg = lane >> 4;
    const CentreRange cr = centre_range(B);
    for (int ci = cr.begin; ci < cr.end; ++ci) {
        const int i = __builtin_amdgcn_readfirstlane(order ? order[ci] : ci);
        const BeadInfo bi = beads[bead_of_ba[i]];
        const float4 pi = posu[i];
        const int zi = __float_as_int(pi.w);
        const int K = nbr_cnt[i];
        const int32_t *row = nbr + (int64_t)i * dp.Kmax;
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int t0 = 0; t0 < K; t0 += 16) {
            const TileEdge te = tile_edge(pi, bi, posu, row, K, t0 + lr, i, dp);
            f32x4 e[HB];
            edge_state_tile<MODE, HB, RB>(dp, gp, nodes, B, gp.L, zi, i, te, e);
            i16x4 eh[HB], el[HB];
#pragma unroll
            for (int b = 0; b < HB; ++b)
                split4<MODE>(e[b], eh[b], el[b]);
            float part = 0.0f;
#pragma unroll
            for (int ob = 0; ob < HB; ++ob) {
                const f32x4 a = mma_rows<MODE, HB>(gp.t_f1, ob, eh, el, load4(gp.fb1 + 16 * ob + 4 * lg));
                const f32x4 w = load4(gp.fw2 + 16 * ob + 4 * lg);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    part = fmaf(w[q], tanh_stable(a[q]), part);
            }
            // phi_f of edge lr: the four feature groups of the column
            part += __shfl_xor(part, 16, kWave);
            part += __shfl_xor(part, 32, kWave);
            const float sphi = part + gp.fb2;
            if (te.valid && lg == 0) {
                const float c = te.fc * sphi * te.inv_r;
                fx += (double)(c * te.d.x);
                fy += (double)(c * te.d.y);
                fz += (double)(c * te.d.z);
            }
        }
        fx = wave_sum_f64(fx);
        fy = wave_sum_f64(fy);
        fz = wave_sum_f64(fz);
        if (lane == 0) {
            F[3 * (int64_t)i + 0] = (float)fx;
            F[3 * (int64_t)i + 1] = (float)fy;
            F[3 * (int64_t)i + 2] = (float)fz;
            E_atom[i] = 0.0f;
        }
        if (lane < 9)
            vir_atom[(int64_t)i * 9 + lane] = 0.0f;
    }
}

// n^(0) = a[Z] for every row.
__global__ void k_gfn_embed(const float4 *__restrict__ posu, const float *__restrict__ node_embed, int H,
                            float *__restrict__ nodes, int B)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)B * H)
        return;
    const int64_t row = t / H;
    const int h = (int)(t - row * H);
    nodes[t] = node_embed[__float_as_int(posu[row].w) * H + h];
}

template <int HB, int RB>
static void gfn_layers_mma(const DevBuffers &d, const Sizes &z, const DescParams &dp, const GfnParams &gp, int grid,
                           int wpg, int l, hipStream_t s)
{
    if (gp.mode == 1)
        hipLaunchKernelGGL((k_gfn_layer_mma<1, HB, RB>), dim3(grid), dim3(kWave * wpg), 0, s, d.posu4, d.beads,
                           d.bead_of_ba, centre_order(d, z), d.nbr, d.nbr_cnt, dp, gp, d.gfn_nodes, l, z.B);
    else
        hipLaunchKernelGGL((k_gfn_layer_mma<2, HB, RB>), dim3(grid), dim3(kWave * wpg), 0, s, d.posu4, d.beads,
                           d.bead_of_ba, centre_order(d, z), d.nbr, d.nbr_cnt, dp, gp, d.gfn_nodes, l, z.B);
}

template <int HB, int RB>
static void gfn_forces_mma(const DevBuffers &d, const Sizes &z, const DescParams &dp, const GfnParams &gp, int grid,
                           int wpg, float *F, hipStream_t s)
{
    if (gp.mode == 1)
        hipLaunchKernelGGL((k_gfn_forces_mma<1, HB, RB>), dim3(grid), dim3(kWave * wpg), 0, s, d.posu4, d.beads,
                           d.bead_of_ba, centre_order(d, z), d.nbr, d.nbr_cnt, dp, gp, d.gfn_nodes, F, d.E_atom,
                           d.vir_atom, z.B);
    else
        hipLaunchKernelGGL((k_gfn_forces_mma<2, HB, RB>), dim3(grid), dim3(kWave * wpg), 0, s, d.posu4, d.beads,
                           d.bead_of_ba, centre_order(d, z), d.nbr, d.nbr_cnt, dp, gp, d.gfn_nodes, F, d.E_atom,
                           d.vir_atom, z.B);
}

void launch_gfn_layers(const DevBuffers &d, const Sizes &z, const DescParams &dp, const GfnParams &gp,
                       const Tuning &tn, hipStream_t s)
{
    const int wpg = tn.centre_waves, grid = centre_grid(z.B, tn);
    const int64_t n0 = (int64_t)z.B * gp.H;
    hipLaunchKernelGGL(k_gfn_embed, dim3((unsigned)((n0 + 255) / 256)), dim3(256), 0, s, d.posu4, gp.node_embed,
                       gp.H, d.gfn_nodes, z.B);
    const bool rb2 = dp.n_rad > 16;
    for (int l = 0; l < gp.L; ++l) {
        if (gp.mode != 0) {
            if (gp.H == 32)
                rb2 ? gfn_layers_mma<2, 2>(d, z, dp, gp, grid, wpg, l, s) : gfn_layers_mma<2, 1>(d, z, dp, gp, grid, wpg, l, s);
            else
                rb2 ? gfn_layers_mma<1, 2>(d, z, dp, gp, grid, wpg, l, s) : gfn_layers_mma<1, 1>(d, z, dp, gp, grid, wpg, l, s);
        } else if (gp.H == 32) {
            hipLaunchKernelGGL(k_gfn_layer<32>, dim3(grid), dim3(kWave * wpg), 0, s, d.posu4, d.beads, d.bead_of_ba,
                               centre_order(d, z), d.nbr, d.nbr_cnt, dp, gp, d.gfn_nodes, l, z.B);
        } else {
            hipLaunchKernelGGL(k_gfn_layer<16>, dim3(grid), dim3(kWave * wpg), 0, s, d.posu4, d.beads, d.bead_of_ba,
                               centre_order(d, z), d.nbr, d.nbr_cnt, dp, gp, d.gfn_nodes, l, z.B);
        }
    }
}

void launch_gfn_forces(const DevBuffers &d, const Sizes &z, const DescParams &dp, const GfnParams &gp,
                       const Tuning &tn, float *F, hipStream_t s)
{
    const int wpg = tn.centre_waves, grid = centre_grid(z.B, tn);
    const bool rb2 = dp.n_rad > 16;
    if (gp.mode != 0) {
        if (gp.H == 32)
            rb2 ? gfn_forces_mma<2, 2>(d, z, dp, gp, grid, wpg, F, s) : gfn_forces_mma<2, 1>(d, z, dp, gp, grid, wpg, F, s);
        else
            rb2 ? gfn_forces_mma<1, 2>(d, z, dp, gp, grid, wpg, F, s) : gfn_forces_mma<1, 1>(d, z, dp, gp, grid, wpg, F, s);
    } else if (gp.H == 32) {
        hipLaunchKernelGGL(k_gfn_forces<32>, dim3(grid), dim3(kWave * wpg), 0, s, d.posu4, d.beads, d.bead_of_ba,
                           centre_order(d, z), d.nbr, d.nbr_cnt, dp, gp, d.gfn_nodes, F, d.E_atom, d.vir_atom, z.B);
    } else {
        hipLaunchKernelGGL(k_gfn_forces<16>, dim3(grid), dim3(kWave * wpg), 0, s, d.posu4, d.beads, d.bead_of_ba,
                           centre_order(d, z), d.nbr, d.nbr_cnt, dp, gp, d.gfn_nodes, F, d.E_atom, d.vir_atom, z.B);
    }
}

}  // namespace pimd
