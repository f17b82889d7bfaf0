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

void launch_gfn_layers(const DevBuffers &d, const Sizes &z, const DescParams &dp, const GfnParams &gp,
                       const Tuning &tn, hipStream_t s)
{
    const int wpg = tn.centre_waves, grid = centre_grid(z.B, tn);
    const int64_t n0 = (int64_t)z.B * gp.H;
    hipLaunchKernelGGL(k_gfn_embed, dim3((unsigned)((n0 + 255) / 256)), dim3(256), 0, s, d.posu4, gp.node_embed,
                       gp.H, d.gfn_nodes, z.B);
    for (int l = 0; l < gp.L; ++l) {
        if (gp.H == 32)
            hipLaunchKernelGGL(k_gfn_layer<32>, dim3(grid), dim3(kWave * wpg), 0, s, d.posu4, d.beads, d.bead_of_ba,
                               centre_order(d, z), d.nbr, d.nbr_cnt, dp, gp, d.gfn_nodes, l, z.B);
        else
            hipLaunchKernelGGL(k_gfn_layer<16>, dim3(grid), dim3(kWave * wpg), 0, s, d.posu4, d.beads, d.bead_of_ba,
                               centre_order(d, z), d.nbr, d.nbr_cnt, dp, gp, d.gfn_nodes, l, z.B);
    }
}

void launch_gfn_forces(const DevBuffers &d, const Sizes &z, const DescParams &dp, const GfnParams &gp,
                       const Tuning &tn, float *F, hipStream_t s)
{
    const int wpg = tn.centre_waves, grid = centre_grid(z.B, tn);
    if (gp.H == 32)
        hipLaunchKernelGGL(k_gfn_forces<32>, dim3(grid), dim3(kWave * wpg), 0, s, d.posu4, d.beads, d.bead_of_ba,
                           centre_order(d, z), d.nbr, d.nbr_cnt, dp, gp, d.gfn_nodes, F, d.E_atom, d.vir_atom, z.B);
    else
        hipLaunchKernelGGL(k_gfn_forces<16>, dim3(grid), dim3(kWave * wpg), 0, s, d.posu4, d.beads, d.bead_of_ba,
                           centre_order(d, z), d.nbr, d.nbr_cnt, dp, gp, d.gfn_nodes, F, d.E_atom, d.vir_atom, z.B);
}

}  // namespace pimd
