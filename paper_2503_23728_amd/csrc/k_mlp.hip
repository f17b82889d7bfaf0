// Per-element MLP of the Behler-Parrinello potential on MFMA, fused:
// forward through the hidden tanh layers, the energy readout, and the input
// gradient dE/dx by the transposed chain, divided by the feature scale
// (dE/dG), for one tile of 16, 32 or 64 rows per workgroup.
//
//   h_l = tanh(W_l h_{l-1} + b_l),  E = w_o . h_L + b_o
//   g_L = w_o * (1 - h_L^2),  g_{l-1} = (W_l^T g_l) * (1 - h_{l-1}^2),  dE/dx = W_1^T g_1
//
// Each GEMM is rows x K times K x N with the 16x16 MFMA tiles of gfx950,
// accumulating in FP32 (in the FP32 mode with the block-wise compensated sum
// of gemm16_cols); the operand precision modes are listed below.
// Activations pass between layers through the workgroup's LDS tile;
// (1 - h^2) of every hidden layer stays in registers in the MFMA output
// layout, which is also the layout of the backward GEMM outputs.
// Weights are read from global memory (L2-resident, shared by all waves):
// W[out][in] serves the forward B operand and its transpose WT[in][out] the
// backward one, so each lane reads contiguous k.
#include "device_common.hpp"

namespace pimd {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef short i16x4 __attribute__((ext_vector_type(4)));

// Operand precision modes: 0 FP32 operands (v_mfma_f32_16x16x4f32, this
// kernel); 1 BF16 operands in a three-term split, with a = a_hi + a_lo and
// b = b_hi + b_lo (each part bfloat16), acc += a_hi b_hi + a_lo b_hi + a_hi b_lo
// (the dropped a_lo b_lo term is below 2^-16 of the product); 4 the same when
// every weight is a bfloat16 value (b_lo = 0): a_hi b + a_lo b; 2 BF16
// operands, one term (modes 1, 2 and 4: k_mlp_bf16); 3 FP64 (k_mlp_f64).
struct MlpCfg {
    static constexpr int S = 130;  // LDS row stride of the FP32 tile (floats)
};

__device__ __forceinline__ float bf16_value(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// acc[r][t] = A[16 r .. 16 r + 15][K] * B[K][16 ct ...] for the row blocks
// r < RT of the tile and the column tiles ct = w + 4t < nct, with
// B[k][n] = Bt[n][k] (row-major Bt[N][ldb]); A is the LDS tile.  Each B
// fragment read from memory feeds RT MFMAs.
// The k range is summed in blocks of 32 (eight MFMAs into a zeroed FP32
// accumulator); the block sums are added into a float-float pair (hi, lo)
// by Knuth's two-sum, so the rounding of a long FP32 running sum (which
// grows with K) is left out: a dot product's error is that of a 32-term FP32
// sum.  On the random-weight water and ice networks this cuts the MLP's
// share of the worst-atom force error about threefold (float32 emulation
// against the FP64 oracle), for three VALU operations per MFMA.
template <int RT>
__device__ __forceinline__ void gemm16_cols(const float *act, int K, const float *Bt, int ldb, int nct, int w,
                                            f32x4 (&acc)[RT][2])
{
    constexpr int S = MlpCfg::S;
    const int lane = lane_id();
    const int lr = lane & 15, lg = lane >> 4;
    f32x4 lo[RT][2];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            acc[r][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            lo[r][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    for (int kb = 0; kb < K; kb += 32) {
        const int ke = kb + 32 < K ? kb + 32 : K;
        f32x4 blk[RT][2];
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int t = 0; t < 2; ++t)
                blk[r][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int k0 = kb; k0 < ke; k0 += 4) {
            float a[RT];
#pragma unroll
            for (int r = 0; r < RT; ++r)
                a[r] = act[(16 * r + lr) * S + k0 + lg];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int ct = w + 4 * t;
                if (ct < nct) {
                    const float b = Bt[(ct * 16 + lr) * ldb + k0 + lg];
#pragma unroll
                    for (int r = 0; r < RT; ++r)
                        blk[r][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[r], b, blk[r][t], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float s0 = acc[r][t][q], b0 = blk[r][t][q];
                    const float sum = s0 + b0;
                    const float bv = sum - s0;
                    const float av = sum - bv;
                    lo[r][t][q] += (s0 - av) + (b0 - bv);
                    acc[r][t][q] = sum;
                }
    }
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc[r][t][q] += lo[r][t][q];
}

// One workgroup per tile of 16 RT rows (tiles of all elements in one
// launch); the four waves split the output columns of every GEMM (column
// tiles w and w+4) and run all RT row blocks of the tile, and the activations
// of the tile live in LDS between layers.  Row r's arithmetic is the same for
// every RT.
template <int RT>
__global__ __launch_bounds__(256) void k_mlp(const int32_t *__restrict__ rows, const MlpTile *__restrict__ tiles,
                                             const float *__restrict__ xhat, int D, int Dp, MlpNets nets,
                                             float *__restrict__ E_atom, float *__restrict__ dEdG)
{
    constexpr int S = MlpCfg::S;
    constexpr int MT = 16 * RT;
    __shared__ __attribute__((aligned(16))) float act[MT * S];
    __shared__ float epart[4][MT];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const MlpTile tile = tiles[blockIdx.x];
    const MlpNet &net = nets.net[tile.e];
    const int32_t *trows = rows + tile.row0;
    const int nrows = tile.nrows;

    for (int idx = threadIdx.x; idx < MT * Dp; idx += 256) {
        const int r = idx / Dp, c = idx - r * Dp;
        act[r * S + c] = (r < nrows && c < D) ? xhat[(int64_t)trows[r] * D + c] : 0.0f;
    }
    __syncthreads();

    f32x4 dsave[3][RT][2];
    f32x4 acc[RT][2];
    int K = Dp;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if (l < net.n_hidden) {
            const MlpLayer L = net.layer[l];
            gemm16_cols<RT>(act, K, L.W, L.in_pad, L.out / 16, w, acc);
            __syncthreads();
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int ct = w + 4 * t;
                if (ct < L.out / 16) {
                    const int col = ct * 16 + lr;
                    const float bias = L.b[col];
#pragma unroll
                    for (int r = 0; r < RT; ++r)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            // tanh and 1 - tanh^2 = sech^2 from e = exp(-2|z|): tanh = sign(z)(1 - e)/(1 + e),
                            // sech^2 = 4e/(1 + e)^2, free of the cancellation in 1 - h^2 for saturated units
                            const float z = acc[r][t][q] + bias;
                            const float e = expf(-2.0f * fabsf(z));
                            const float ope = 1.0f + e;
                            dsave[l][r][t][q] = 4.0f * e / (ope * ope);
                            act[(16 * r + lg * 4 + q) * S + col] = copysignf((1.0f - e) / ope, z);
                        }
                }
            }
            __syncthreads();
            K = L.out;
        }
    }
    // energy readout (FP32 on the VALU in every mode); waves hold column slices
    const int nlast = K / 16;
    float e_part[RT][4];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            e_part[r][q] = 0.0f;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int ct = w + 4 * t;
        if (ct < nlast) {
            const int col = ct * 16 + lr;
            const float wo = net.wo[col];
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    e_part[r][q] += act[(16 * r + lg * 4 + q) * S + col] * wo;
        }
    }
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            e_part[r][q] = row16_sum(e_part[r][q]);
    if (lr == 0)
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                epart[w][16 * r + lg * 4 + q] = e_part[r][q];
    __syncthreads();
    if (threadIdx.x < MT && (int)threadIdx.x < nrows)
        E_atom[trows[threadIdx.x]] = ((epart[0][threadIdx.x] + epart[1][threadIdx.x]) +
                                      (epart[2][threadIdx.x] + epart[3][threadIdx.x])) + net.bo;
    // g_L = w_o * (1 - h_L^2)
    const int nh = net.n_hidden;
#pragma unroll
    for (int l = 2; l >= 0; --l) {
        if (l == nh - 1) {
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int ct = w + 4 * t;
                if (ct < nlast) {
                    const int col = ct * 16 + lr;
                    const float wo = net.wo[col];
#pragma unroll
                    for (int r = 0; r < RT; ++r)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            act[(16 * r + lg * 4 + q) * S + col] = wo * dsave[l][r][t][q];
                }
            }
        }
    }
    __syncthreads();
    // g_{l-1} = (W_l^T g_l) * (1 - h_{l-1}^2)
#pragma unroll
    for (int l = 2; l >= 1; --l) {
        if (l < nh) {
            const MlpLayer L = net.layer[l];
            gemm16_cols<RT>(act, L.out, L.WT, L.out, L.in_pad / 16, w, acc);
            __syncthreads();
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int ct = w + 4 * t;
                if (ct < L.in_pad / 16) {
                    const int col = ct * 16 + lr;
#pragma unroll
                    for (int r = 0; r < RT; ++r)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            act[(16 * r + lg * 4 + q) * S + col] = acc[r][t][q] * dsave[l - 1][r][t][q];
                }
            }
            __syncthreads();
        }
    }
    // dE/dx = W_1^T g_1 and dE/dG = dE/dx / scale
    const MlpLayer L0 = net.layer[0];
    gemm16_cols<RT>(act, L0.out, L0.WT, L0.out, Dp / 16, w, acc);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int ct = w + 4 * t;
        if (ct < Dp / 16) {
            const int col = ct * 16 + lr;
            if (col < D) {
                const float is = net.inv_scale[col];
#pragma unroll
                for (int r = 0; r < RT; ++r)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int row = 16 * r + lg * 4 + q;
                        if (row < nrows)
                            dEdG[(int64_t)trows[row] * D + col] = acc[r][t][q] * is;
                    }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// BF16 operand modes (1: three-term split, 2: one term).  The activations of
// the tile are kept in LDS as bfloat16 parts (hi, and lo = bf16(v - hi) in
// the split mode), converted once when a layer's outputs are written instead
// of once per GEMM k-step in every wave; 32-deep k-steps use
// v_mfma_f32_16x16x32_bf16 (each lane holds eight consecutive k of its row or
// column), a 16-deep remainder v_mfma_f32_16x16x16bf16_1k.
typedef short i16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kBfStride = 136;   // LDS row stride of the bf16 tiles (elements): 272-byte rows

__device__ __forceinline__ f32x4 mfma_k32(const i16x8 &a, const i16x8 &b, const f32x4 &c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

// Nearest-even float -> bfloat16 (one v_cvt_pk_bf16_f32 on gfx950).
__device__ __forceinline__ uint16_t to_bf16(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }

// Modes 1 and 4 split the activations into hi and lo bfloat16 parts; mode 1
// splits the weights too, mode 4 takes weights that are bfloat16 values
// already (their lo parts are zero), so a product costs two MFMAs, not three.
template <int MODE>
constexpr bool split_act() { return MODE == 1 || MODE == 4; }

template <int MODE>
__device__ __forceinline__ void store_bf16(uint16_t *hi, uint16_t *lo, int idx, float v)
{
    const uint16_t h = to_bf16(v);
    hi[idx] = h;
    if (split_act<MODE>())
        lo[idx] = to_bf16(v - bf16_value(h));
}

// acc[r][t] = A[16 r .. 16 r + 15][K] * B[K][16 ct ...] (ct = w + NW t < nct),
// B[k][n] = Bt[n][k] with Bt row-major [N][ldb] in bfloat16 parts; NW waves
// share the (at most 8) column tiles of a layer, CT = 8 / NW each.
template <int MODE, int RT, int NW>
__device__ __forceinline__ void gemm_bf16(const uint16_t *ahi, const uint16_t *alo, int K, const uint16_t *Bh,
                                          const uint16_t *Bl, int ldb, int nct, int w, f32x4 (&acc)[RT][8 / NW])
{
    constexpr int SB = kBfStride;
    constexpr int CT = 8 / NW;
    const int lane = lane_id();
    const int lr = lane & 15, lg = lane >> 4;
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int t = 0; t < CT; ++t)
            acc[r][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // weight fragments of up to four 32-deep steps are loaded together, so
    // one latency of the (L2-resident) weights covers 4 RT MFMA groups
    int k0 = 0;
    for (; k0 + 32 <= K; k0 += 128) {
        const int nsteps = min(4, (K - k0) >> 5);
        i16x8 bh[CT][4], bl[CT][4];
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            const int ct = w + NW * t;
            if (ct < nct) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (u < nsteps) {
                        const int64_t o = (int64_t)(ct * 16 + lr) * ldb + k0 + 32 * u + 8 * lg;
                        bh[t][u] = *reinterpret_cast<const i16x8 *>(Bh + o);
                        if (MODE == 1)
                            bl[t][u] = *reinterpret_cast<const i16x8 *>(Bl + o);
                    }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (u < nsteps) {
                i16x8 ah[RT], al[RT];
#pragma unroll
                for (int r = 0; r < RT; ++r) {
                    const int o = (16 * r + lr) * SB + k0 + 32 * u + 8 * lg;
                    ah[r] = *reinterpret_cast<const i16x8 *>(ahi + o);
                    if (split_act<MODE>())
                        al[r] = *reinterpret_cast<const i16x8 *>(alo + o);
                }
#pragma unroll
                for (int t = 0; t < CT; ++t) {
                    const int ct = w + NW * t;
                    if (ct < nct) {
#pragma unroll
                        for (int r = 0; r < RT; ++r) {
                            acc[r][t] = mfma_k32(ah[r], bh[t][u], acc[r][t]);
                            if (split_act<MODE>())
                                acc[r][t] = mfma_k32(al[r], bh[t][u], acc[r][t]);
                            if (MODE == 1)
                                acc[r][t] = mfma_k32(ah[r], bl[t][u], acc[r][t]);
                        }
                    }
                }
            }
        }
    }
    k0 = K & ~31;
    if (k0 < K) {   // K is a multiple of 16: one 16-deep step remains
        i16x4 ah[RT], al[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            const int o = (16 * r + lr) * SB + k0 + 4 * lg;
            ah[r] = *reinterpret_cast<const i16x4 *>(ahi + o);
            if (split_act<MODE>())
                al[r] = *reinterpret_cast<const i16x4 *>(alo + o);
        }
#pragma unroll
        for (int t = 0; t < CT; ++t) {
            const int ct = w + NW * t;
            if (ct < nct) {
                const int64_t o = (int64_t)(ct * 16 + lr) * ldb + k0 + 4 * lg;
                const i16x4 bh = *reinterpret_cast<const i16x4 *>(Bh + o);
                i16x4 bl;
                if (MODE == 1)
                    bl = *reinterpret_cast<const i16x4 *>(Bl + o);
#pragma unroll
                for (int r = 0; r < RT; ++r) {
                    acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[r], bh, acc[r][t], 0, 0, 0);
                    if (split_act<MODE>())
                        acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[r], bh, acc[r][t], 0, 0, 0);
                    if (MODE == 1)
                        acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[r], bl, acc[r][t], 0, 0, 0);
                }
            }
        }
    }
}

// One workgroup per tile of 16 RT rows of one element, as k_mlp; the energy
// readout is taken from the last layer's FP32 tanh values in registers.
template <int MODE, int RT, int NW>
__global__ __launch_bounds__(64 * NW) void k_mlp_bf16(const int32_t *__restrict__ rows,
                                                  const MlpTile *__restrict__ tiles,
                                                  const float *__restrict__ xhat, int D, int Dp, MlpNets nets,
                                                  float *__restrict__ E_atom, float *__restrict__ dEdG)
{
    constexpr int SB = kBfStride;
    constexpr int MT = 16 * RT;
    __shared__ __attribute__((aligned(16))) uint16_t ahi[MT * SB];
    __shared__ __attribute__((aligned(16))) uint16_t alo[split_act<MODE>() ? MT * SB : 8];
    constexpr int CT = 8 / NW;
    __shared__ float epart[4][MT];
    // NW = 8: the second half of the waves hands its per-lane readout partials
    // to the first half, so the sums keep the order of the four-wave layout
    __shared__ float ehand[NW == 8 ? 4 * 64 * 4 * RT : 1];
    // the wave index is wave-uniform: column-tile tests become scalar branches
    const int lane = lane_id(), w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lr = lane & 15, lg = lane >> 4;
    const MlpTile tile = tiles[blockIdx.x];
    const MlpNet &net = nets.net[tile.e];
    const int32_t *trows = rows + tile.row0;
    const int nrows = tile.nrows;

    for (int idx = threadIdx.x; idx < MT * Dp; idx += 64 * NW) {
        const int r = idx / Dp, c = idx - r * Dp;
        store_bf16<MODE>(ahi, alo, r * SB + c, (r < nrows && c < D) ? xhat[(int64_t)trows[r] * D + c] : 0.0f);
    }
    __syncthreads();

    f32x4 dsave[3][RT][CT];
    f32x4 acc[RT][CT];
    float e_part[RT][4];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            e_part[r][q] = 0.0f;
    const int nh = net.n_hidden;
    int K = Dp;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if (l < nh) {
            const MlpLayer L = net.layer[l];
            gemm_bf16<MODE, RT, NW>(ahi, alo, K, L.Wb, L.Wb_lo, L.in_pad, L.out / 16, w, acc);
            __syncthreads();
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                const int ct = w + NW * t;
                if (ct < L.out / 16) {
                    const int col = ct * 16 + lr;
                    const float bias = L.b[col];
                    const float wo = l == nh - 1 ? net.wo[col] : 0.0f;
#pragma unroll
                    for (int r = 0; r < RT; ++r)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            // tanh and sech^2 from e = exp(-2|z|), as in k_mlp, with the
                            // hardware exp2 and reciprocal: their ~1e-7 relative errors are
                            // far below the 2^-16 resolution of the split operands
                            const float z = acc[r][t][q] + bias;
                            const float e = __builtin_amdgcn_exp2f(-2.8853900817779268f * fabsf(z));
                            const float rope = __builtin_amdgcn_rcpf(1.0f + e);
                            const float h = copysignf((1.0f - e) * rope, z);
                            dsave[l][r][t][q] = 4.0f * e * rope * rope;
                            store_bf16<MODE>(ahi, alo, (16 * r + lg * 4 + q) * SB + col, h);
                            if (l == nh - 1)
                                e_part[r][q] += h * wo;
                        }
                }
            }
            __syncthreads();
            K = L.out;
        }
    }
    // energy readout: the column slices of the four waves (tiles w and w + 4
    // of wave w, as one wave holds them when NW = 4)
    if (NW == 8) {
        if (w >= 4)
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    ehand[(((w - 4) * RT + r) * 4 + q) * 64 + lane] = e_part[r][q];
        __syncthreads();
        if (w < 4)
#pragma unroll
            for (int r = 0; r < RT; ++r)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    e_part[r][q] += ehand[((w * RT + r) * 4 + q) * 64 + lane];
    }
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            e_part[r][q] = row16_sum(e_part[r][q]);
    if (lr == 0 && w < 4)
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                epart[w][16 * r + lg * 4 + q] = e_part[r][q];
    // g_L = w_o * (1 - h_L^2)
    const int nlast = K / 16;
#pragma unroll
    for (int l = 2; l >= 0; --l) {
        if (l == nh - 1) {
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                const int ct = w + NW * t;
                if (ct < nlast) {
                    const int col = ct * 16 + lr;
                    const float wo = net.wo[col];
#pragma unroll
                    for (int r = 0; r < RT; ++r)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            store_bf16<MODE>(ahi, alo, (16 * r + lg * 4 + q) * SB + col, wo * dsave[l][r][t][q]);
                }
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < MT && (int)threadIdx.x < nrows)
        E_atom[trows[threadIdx.x]] = ((epart[0][threadIdx.x] + epart[1][threadIdx.x]) +
                                      (epart[2][threadIdx.x] + epart[3][threadIdx.x])) + net.bo;
    // g_{l-1} = (W_l^T g_l) * (1 - h_{l-1}^2)
#pragma unroll
    for (int l = 2; l >= 1; --l) {
        if (l < nh) {
            const MlpLayer L = net.layer[l];
            gemm_bf16<MODE, RT, NW>(ahi, alo, L.out, L.WTb, L.WTb_lo, L.out, L.in_pad / 16, w, acc);
            __syncthreads();
#pragma unroll
            for (int t = 0; t < CT; ++t) {
                const int ct = w + NW * t;
                if (ct < L.in_pad / 16) {
                    const int col = ct * 16 + lr;
#pragma unroll
                    for (int r = 0; r < RT; ++r)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            store_bf16<MODE>(ahi, alo, (16 * r + lg * 4 + q) * SB + col,
                                             acc[r][t][q] * dsave[l - 1][r][t][q]);
                }
            }
            __syncthreads();
        }
    }
    // dE/dx = W_1^T g_1 and dE/dG = dE/dx / scale
    const MlpLayer L0 = net.layer[0];
    gemm_bf16<MODE, RT, NW>(ahi, alo, L0.out, L0.WTb, L0.WTb_lo, L0.out, Dp / 16, w, acc);
#pragma unroll
    for (int t = 0; t < CT; ++t) {
        const int ct = w + NW * t;
        if (ct < Dp / 16) {
            const int col = ct * 16 + lr;
            if (col < D) {
                const float is = net.inv_scale[col];
#pragma unroll
                for (int r = 0; r < RT; ++r)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int row = 16 * r + lg * 4 + q;
                        if (row < nrows)
                            dEdG[(int64_t)trows[row] * D + col] = acc[r][t][q] * is;
                    }
            }
        }
    }
}

// FP64 variant (precision mode 3): the same chain with FP64 operands,
// activations and accumulation on v_mfma_f64_16x16x4f64, so the MLP adds no
// error visible next to the FP32 descriptors.  Its A and B operand layouts
// match the FP32 16x16x4 instruction; its output rows interleave by four
// (element q of lane (g, l) is row 4q + g, column l).
__device__ __forceinline__ void gemm16_cols_f64(const double *act, int K, const double *Bt, int ldb, int nct, int w,
                                                f64x4 (&acc)[2])
{
    constexpr int S = 130;
    const int lane = lane_id();
    const int lr = lane & 15, lg = lane >> 4;
    acc[0] = f64x4{0.0, 0.0, 0.0, 0.0};
    acc[1] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 4) {
        const double a = act[lr * S + k0 + lg];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int ct = w + 4 * t;
            if (ct < nct) {
                const double b = Bt[(ct * 16 + lr) * ldb + k0 + lg];
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_mlp_f64(const int32_t *__restrict__ rows, const MlpTile *__restrict__ tiles,
                                                 const float *__restrict__ xhat, int D, int Dp, MlpNets nets,
                                                 float *__restrict__ E_atom, float *__restrict__ dEdG)
{
    constexpr int S = 130;
    __shared__ double act[16 * S];
    __shared__ double epart[4][16];
    const int lane = lane_id(), w = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    // v_mfma_f64_16x16x4f64 returns element q of lane (lg, lr) as C[4 q + lg][lr]
    auto crow = [lg](int q) { return 4 * q + lg; };
    const MlpTile tile = tiles[blockIdx.x];
    const MlpNet &net = nets.net[tile.e];
    const int32_t *trows = rows + tile.row0;
    const int nrows = tile.nrows;
    for (int idx = threadIdx.x; idx < 16 * Dp; idx += 256) {
        const int r = idx / Dp, c = idx - r * Dp;
        act[r * S + c] = (r < nrows && c < D) ? (double)xhat[(int64_t)trows[r] * D + c] : 0.0;
    }
    __syncthreads();
    f64x4 dsave[3][2];
    f64x4 acc[2];
    int K = Dp;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if (l < net.n_hidden) {
            const MlpLayer L = net.layer[l];
            gemm16_cols_f64(act, K, L.W64, L.in_pad, L.out / 16, w, acc);
            __syncthreads();
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int ct = w + 4 * t;
                if (ct < L.out / 16) {
                    const int col = ct * 16 + lr;
                    const double bias = (double)L.b[col];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double z = acc[t][q] + bias;
                        const double e = exp(-2.0 * fabs(z));
                        const double ope = 1.0 + e;
                        dsave[l][t][q] = 4.0 * e / (ope * ope);
                        act[crow(q) * S + col] = copysign((1.0 - e) / ope, z);
                    }
                }
            }
            __syncthreads();
            K = L.out;
        }
    }
    const int nlast = K / 16;
    double e_part[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int ct = w + 4 * t;
        if (ct < nlast) {
            const int col = ct * 16 + lr;
            const double wo = (double)net.wo[col];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                e_part[q] += act[crow(q) * S + col] * wo;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int o = 8; o > 0; o >>= 1)
            e_part[q] += __shfl_xor(e_part[q], o, kWave);
    if (lr == 0)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            epart[w][crow(q)] = e_part[q];
    __syncthreads();
    if (threadIdx.x < 16 && (int)threadIdx.x < nrows)
        E_atom[trows[threadIdx.x]] = (float)(((epart[0][threadIdx.x] + epart[1][threadIdx.x]) +
                                              (epart[2][threadIdx.x] + epart[3][threadIdx.x])) + (double)net.bo);
    const int nh = net.n_hidden;
#pragma unroll
    for (int l = 2; l >= 0; --l) {
        if (l == nh - 1) {
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int ct = w + 4 * t;
                if (ct < nlast) {
                    const int col = ct * 16 + lr;
                    const double wo = (double)net.wo[col];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        act[crow(q) * S + col] = wo * dsave[l][t][q];
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int l = 2; l >= 1; --l) {
        if (l < nh) {
            const MlpLayer L = net.layer[l];
            gemm16_cols_f64(act, L.out, L.WT64, L.out, L.in_pad / 16, w, acc);
            __syncthreads();
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int ct = w + 4 * t;
                if (ct < L.in_pad / 16) {
                    const int col = ct * 16 + lr;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        act[crow(q) * S + col] = acc[t][q] * dsave[l - 1][t][q];
                }
            }
            __syncthreads();
        }
    }
    const MlpLayer L0 = net.layer[0];
    gemm16_cols_f64(act, L0.out, L0.WT64, L0.out, Dp / 16, w, acc);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int ct = w + 4 * t;
        if (ct < Dp / 16) {
            const int col = ct * 16 + lr;
            if (col < D) {
                const double is = (double)net.inv_scale[col];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = crow(q);
                    if (r < nrows)
                        dEdG[(int64_t)trows[r] * D + col] = (float)(acc[t][q] * is);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Register-chained BF16 MLP (modes 1, 2, 4): one wave per 16 rows of one
// element; activations never leave the registers and no wave waits for
// another.  Every GEMM is taken transposed, Y^T = W X^T: the weights are the
// A operand (its rows are output features) and the wave's 16 rows are the
// columns of the B operand.  The MFMA result of a 16-feature output tile
// leaves features 4g .. 4g+3 of row r in lane (r, g) (r = lane mod 16,
// g = lane / 16); two output tiles 2b and 2b+1 thus give lane (r, g) the eight
// features {32b + 4g + j, 32b + 16 + 4g + j : j < 4}, which is a B operand of
// a 32-deep k-step when the step's k index runs over the features in that
// order.  The weight fragments are packed on the host in the same order (one
// 16-byte fragment per lane per output tile and k-step), so the tanh outputs
// of a layer, split into bfloat16 parts in place, are the next layer's
// operand.  The backward chain is the same with W^T as the A operand, and
// (1 - h^2) of every layer stays in registers in the output layout.
// Fragments are read from global memory (a few hundred kB per element,
// L2-resident).  Limits: widths and D at most 128, D a multiple of 4.
constexpr int kChainTiles = 8;   // output tiles of 16 features
constexpr int kChainSteps = 4;   // 32-deep k-steps

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two floats as nearest-even bfloat16 values, the first in the low half.
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}

// Four values of one output tile into the k-step operand words: half 0 or 1
// of block b (elements 4 half .. 4 half + 3), hi parts and, when split, the
// bfloat16 remainders v - hi.
template <bool SPLIT>
__device__ __forceinline__ void chain_put(const f32x4 &v, int half, u32x4 &xh, u32x4 &xl)
{
    const uint32_t h0 = pack_bf16x2(v[0], v[1]), h1 = pack_bf16x2(v[2], v[3]);
    if (half == 0) {
        xh[0] = h0;
        xh[1] = h1;
    } else {
        xh[2] = h0;
        xh[3] = h1;
    }
    if (SPLIT) {
        const uint32_t l0 = pack_bf16x2(v[0] - __uint_as_float(h0 << 16), v[1] - __uint_as_float(h0 & 0xFFFF0000u));
        const uint32_t l1 = pack_bf16x2(v[2] - __uint_as_float(h1 << 16), v[3] - __uint_as_float(h1 & 0xFFFF0000u));
        if (half == 0) {
            xl[0] = l0;
            xl[1] = l1;
        } else {
            xl[2] = l0;
            xl[3] = l1;
        }
    }
}

__device__ __forceinline__ i16x8 as_op(const u32x4 &v) { return __builtin_bit_cast(i16x8, v); }


// acc[o] = sum over the KB k-steps of fragment (o, b) x operand b, o < OT.
// The fragments of step b + 1 are loaded while step b's MFMAs run (two
// buffers); scheduling barriers keep the compiler from hoisting further
// loads, which would hold every fragment of the layer in registers.
template <int MODE, int OT, int KB>
__device__ __forceinline__ void chain_load(const uint16_t *__restrict__ F, const uint16_t *__restrict__ Flo, int b,
                                           i16x8 (&fh)[OT], i16x8 (&fl)[OT])
{
    const int lane = lane_id();
#pragma unroll
    for (int o = 0; o < OT; ++o) {
        const int64_t at = ((int64_t)(o * KB + b) * 64 + lane) * 8;
        fh[o] = *reinterpret_cast<const i16x8 *>(F + at);
        if (MODE == 1)
            fl[o] = *reinterpret_cast<const i16x8 *>(Flo + at);
    }
}

template <int MODE, int OT, int KB>
__device__ __forceinline__ void chain_gemm(const uint16_t *__restrict__ F, const uint16_t *__restrict__ Flo,
                                           const u32x4 (&xh)[kChainSteps], const u32x4 (&xl)[kChainSteps],
                                           f32x4 (&acc)[kChainTiles])
{
#pragma unroll
    for (int o = 0; o < OT; ++o)
        acc[o] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // NB buffers: the loads run NB - 1 steps ahead of the MFMAs (a step of
    // OT x 2 MFMAs is shorter than an L2 round trip)
    constexpr int NB = MODE == 1 ? 2 : 3;
    i16x8 fh[NB][OT], fl[NB][OT];
#pragma unroll
    for (int b = 0; b < NB - 1; ++b)
        if (b < KB)
            chain_load<MODE, OT, KB>(F, Flo, b, fh[b], fl[b]);
#pragma unroll
    for (int b = 0; b < KB; ++b) {
        if (b + NB - 1 < KB)
            chain_load<MODE, OT, KB>(F, Flo, b + NB - 1, fh[(b + NB - 1) % NB], fl[(b + NB - 1) % NB]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int o = 0; o < OT; ++o) {
            const i16x8 a = fh[b % NB][o];
            acc[o] = mfma_k32(a, as_op(xh[b]), acc[o]);
            if (split_act<MODE>())
                acc[o] = mfma_k32(a, as_op(xl[b]), acc[o]);
            if (MODE == 1)
                acc[o] = mfma_k32(fl[b % NB][o], as_op(xh[b]), acc[o]);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Output tiles 0 .. OT-1 of acc (times s, when given) into the operand of the
// next GEMM: k-steps 0 .. (OT+1)/2 - 1, the half of an odd last step zeroed.
template <bool SPLIT, int OT>
__device__ __forceinline__ void chain_operand(const f32x4 (&v)[kChainTiles], u32x4 (&xh)[kChainSteps],
                                              u32x4 (&xl)[kChainSteps])
{
#pragma unroll
    for (int o = 0; o < OT; ++o)
        chain_put<SPLIT>(v[o], o & 1, xh[o >> 1], xl[o >> 1]);
    if (OT & 1)
        chain_put<SPLIT>(f32x4{0.0f, 0.0f, 0.0f, 0.0f}, 1, xh[OT >> 1], xl[OT >> 1]);
}

// One wave per 16 rows; the network shape is compile-time: D in KB0 32-deep
// steps, hidden widths H1, H2 and H3 (H3 = 0: two hidden layers).
// Two waves per SIMD where the registers allow it (the three-product mode,
// with both weight parts in flight, would spill).
template <int MODE, int KB0, int H1, int H2, int H3>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MODE == 1 ? 1 : 2))) void k_mlp_chain(const int32_t *__restrict__ rows,
                                                   const MlpTile *__restrict__ tiles,
                                                   const float *__restrict__ xhat, int D, MlpNets nets,
                                                   float *__restrict__ E_atom, float *__restrict__ dEdG)
{
    constexpr bool SPLIT = split_act<MODE>();
    constexpr int NH = H3 ? 3 : 2;
    constexpr int OT1 = H1 / 16, OT2 = H2 / 16, OT3 = H3 / 16;
    constexpr int OTL = NH == 3 ? OT3 : OT2;   // tiles of the last hidden layer
    constexpr int KB1 = (OT1 + 1) / 2, KB2 = (OT2 + 1) / 2, KB3 = (OT3 + 1) / 2;
    constexpr int OTD = KB0 * 2;               // tiles of dE/dx (features >= D are dropped)
    const int lane = lane_id(), w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = lane & 15, g = lane >> 4;
    const MlpTile tile = tiles[blockIdx.x];
    const int nrw = min(16, tile.nrows - 16 * w);   // rows of this wave
    if (nrw <= 0)
        return;
    const MlpNet &net = nets.net[tile.e];
    const bool row_ok = r < nrw;
    const int64_t row = row_ok ? (int64_t)rows[tile.row0 + 16 * w + r] : 0;

    u32x4 xh[kChainSteps], xl[kChainSteps];
    f32x4 acc[kChainTiles];   // GEMM results, overwritten in place by h, g and their products
    f32x4 ds1[kChainTiles], ds2[kChainTiles], ds3[kChainTiles];
    // input operand: features {32b + 4g + j, 32b + 16 + 4g + j} of the lane's row
#pragma unroll
    for (int b = 0; b < KB0; ++b)
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int f = 32 * b + 16 * half + 4 * g;
            f32x4 v = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            if (row_ok && f < D)
                v = *reinterpret_cast<const f32x4 *>(xhat + row * D + f);
            chain_put<SPLIT>(v, half, xh[b], xl[b]);
        }
    float e_part = 0.0f;
    // forward: h = tanh(W x + b), ds = 1 - h^2; the last layer's h feeds the readout
    auto layer = [&](const MlpLayer &L, auto OTc, f32x4 (&ds)[kChainTiles], bool last) {
        constexpr int OT = decltype(OTc)::value;
#pragma unroll
        for (int o = 0; o < OT; ++o) {
            const f32x4 bias = *reinterpret_cast<const f32x4 *>(L.b + 16 * o + 4 * g);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                // tanh and sech^2 from e = exp(-2|z|), as in k_mlp_bf16
                const float z = acc[o][j] + bias[j];
                const float e = __builtin_amdgcn_exp2f(-2.8853900817779268f * fabsf(z));
                const float rope = __builtin_amdgcn_rcpf(1.0f + e);
                acc[o][j] = copysignf((1.0f - e) * rope, z);
                ds[o][j] = 4.0f * e * rope * rope;
            }
            if (last) {
                const f32x4 wo = *reinterpret_cast<const f32x4 *>(net.wo + 16 * o + 4 * g);
                e_part += (acc[o][0] * wo[0] + acc[o][1] * wo[1]) + (acc[o][2] * wo[2] + acc[o][3] * wo[3]);
            }
        }
    };
    chain_gemm<MODE, OT1, KB0>(net.layer[0].Wc, net.layer[0].Wc_lo, xh, xl, acc);
    layer(net.layer[0], std::integral_constant<int, OT1>{}, ds1, false);
    chain_operand<SPLIT, OT1>(acc, xh, xl);
    chain_gemm<MODE, OT2, KB1>(net.layer[1].Wc, net.layer[1].Wc_lo, xh, xl, acc);
    layer(net.layer[1], std::integral_constant<int, OT2>{}, ds2, NH == 2);
    if constexpr (NH == 3) {
        chain_operand<SPLIT, OT2>(acc, xh, xl);
        chain_gemm<MODE, OT3, KB2>(net.layer[2].Wc, net.layer[2].Wc_lo, xh, xl, acc);
        layer(net.layer[2], std::integral_constant<int, OT3>{}, ds3, true);
    }
    // energy: the four lane groups of a row hold disjoint features
    e_part += __shfl_xor(e_part, 16);
    e_part += __shfl_xor(e_part, 32);
    if (g == 0 && row_ok)
        E_atom[row] = e_part + net.bo;
    // g_L = w_o (1 - h_L^2); g_{l-1} = (W_l^T g_l)(1 - h_{l-1}^2); dE/dx = W_1^T g_1
    const f32x4(&dsL)[kChainTiles] = NH == 3 ? ds3 : ds2;
#pragma unroll
    for (int o = 0; o < OTL; ++o) {
        const f32x4 wo = *reinterpret_cast<const f32x4 *>(net.wo + 16 * o + 4 * g);
        acc[o] = wo * dsL[o];
    }
    chain_operand<SPLIT, OTL>(acc, xh, xl);
    if constexpr (NH == 3) {
        chain_gemm<MODE, OT2, KB3>(net.layer[2].WTc, net.layer[2].WTc_lo, xh, xl, acc);
#pragma unroll
        for (int o = 0; o < OT2; ++o)
            acc[o] *= ds2[o];
        chain_operand<SPLIT, OT2>(acc, xh, xl);
    }
    chain_gemm<MODE, OT1, KB2>(net.layer[1].WTc, net.layer[1].WTc_lo, xh, xl, acc);
#pragma unroll
    for (int o = 0; o < OT1; ++o)
        acc[o] *= ds1[o];
    chain_operand<SPLIT, OT1>(acc, xh, xl);
    chain_gemm<MODE, OTD, KB1>(net.layer[0].WTc, net.layer[0].WTc_lo, xh, xl, acc);
    if (row_ok) {
#pragma unroll
        for (int o = 0; o < OTD; ++o) {
            const int f = 16 * o + 4 * g;
            if (f < D) {
                const f32x4 is = *reinterpret_cast<const f32x4 *>(net.inv_scale + f);
                *reinterpret_cast<f32x4 *>(dEdG + row * D + f) = acc[o] * is;
            }
        }
    }
}

// Network shapes with a chained kernel: (32-deep steps of D, hidden widths).
struct ChainShape {
    int kb0, h1, h2, h3;
};
constexpr ChainShape kChainShapes[] = {{3, 128, 128, 64}, {3, 64, 64, 0}};

bool mlp_chain_shape(int D, int n_hidden, const int *hidden)
{
    if (D % 4 != 0 || n_hidden < 2 || n_hidden > 3)
        return false;
    for (const ChainShape &c : kChainShapes)
        if ((D + 31) / 32 == c.kb0 && hidden[0] == c.h1 && hidden[1] == c.h2 &&
            (n_hidden == 3 ? hidden[2] == c.h3 : c.h3 == 0))
            return true;
    return false;
}

// Launches the instantiation of the nets' shape; false when there is none.
template <int MODE>
static bool launch_mlp_chain(const DevBuffers &d, const MlpNets &nets, int n_tiles, int D, int rows, hipStream_t s)
{
    const MlpNet &n = nets.net[0];
    if (!n.layer[0].Wc)
        return false;
    const int kb0 = (D + 31) / 32, h1 = n.layer[0].out, h2 = n.layer[1].out, h3 = n.n_hidden == 3 ? n.layer[2].out : 0;
    if (kb0 == 3 && h1 == 128 && h2 == 128 && h3 == 64)
        hipLaunchKernelGGL((k_mlp_chain<MODE, 3, 128, 128, 64>), dim3(n_tiles), dim3(4 * rows), 0, s, d.elem_rows,
                           d.mlp_tiles, d.xhat, D, nets, d.E_atom, d.dEdG);
    else if (kb0 == 3 && h1 == 64 && h2 == 64 && h3 == 0)
        hipLaunchKernelGGL((k_mlp_chain<MODE, 3, 64, 64, 0>), dim3(n_tiles), dim3(4 * rows), 0, s, d.elem_rows,
                           d.mlp_tiles, d.xhat, D, nets, d.E_atom, d.dEdG);
    else
        return false;
    return true;
}

static void launch_mlp_fp32(const DevBuffers &d, const MlpNets &nets, int n_tiles, int D, int Dp, int rows,
                            hipStream_t s)
{
    if (rows == 64)
        hipLaunchKernelGGL((k_mlp<4>), dim3(n_tiles), dim3(256), 0, s, d.elem_rows, d.mlp_tiles, d.xhat, D, Dp,
                           nets, d.E_atom, d.dEdG);
    else if (rows == 32)
        hipLaunchKernelGGL((k_mlp<2>), dim3(n_tiles), dim3(256), 0, s, d.elem_rows, d.mlp_tiles, d.xhat, D, Dp,
                           nets, d.E_atom, d.dEdG);
    else
        hipLaunchKernelGGL((k_mlp<1>), dim3(n_tiles), dim3(256), 0, s, d.elem_rows, d.mlp_tiles, d.xhat, D, Dp,
                           nets, d.E_atom, d.dEdG);
}

template <int MODE, int NW>
static void launch_mlp_bf16(const DevBuffers &d, const MlpNets &nets, int n_tiles, int D, int Dp, int rows,
                            hipStream_t s)
{
    if (rows == 64)
        hipLaunchKernelGGL((k_mlp_bf16<MODE, 4, NW>), dim3(n_tiles), dim3(64 * NW), 0, s, d.elem_rows, d.mlp_tiles,
                           d.xhat, D, Dp, nets, d.E_atom, d.dEdG);
    else if (rows == 32)
        hipLaunchKernelGGL((k_mlp_bf16<MODE, 2, NW>), dim3(n_tiles), dim3(64 * NW), 0, s, d.elem_rows, d.mlp_tiles,
                           d.xhat, D, Dp, nets, d.E_atom, d.dEdG);
    else
        hipLaunchKernelGGL((k_mlp_bf16<MODE, 1, NW>), dim3(n_tiles), dim3(64 * NW), 0, s, d.elem_rows, d.mlp_tiles,
                           d.xhat, D, Dp, nets, d.E_atom, d.dEdG);
}

void launch_mlp(const DevBuffers &d, const MlpNets &nets, int n_tiles, int D, int Dp, int mlp_mode, int rows,
                int waves, bool chain, hipStream_t s)
{
    if (n_tiles <= 0)
        return;
    if (chain && mlp_mode == 4 && launch_mlp_chain<4>(d, nets, n_tiles, D, rows, s))
        return;
    if (chain && mlp_mode == 1 && launch_mlp_chain<1>(d, nets, n_tiles, D, rows, s))
        return;
    if (chain && mlp_mode == 2 && launch_mlp_chain<2>(d, nets, n_tiles, D, rows, s))
        return;
    if (mlp_mode == 3)
        hipLaunchKernelGGL(k_mlp_f64, dim3(n_tiles), dim3(256), 0, s, d.elem_rows, d.mlp_tiles, d.xhat, D, Dp, nets,
                           d.E_atom, d.dEdG);
    else if (mlp_mode == 4 && waves == 8)
        launch_mlp_bf16<4, 8>(d, nets, n_tiles, D, Dp, rows, s);
    else if (mlp_mode == 4)
        launch_mlp_bf16<4, 4>(d, nets, n_tiles, D, Dp, rows, s);
    else if (mlp_mode == 1 && waves == 8)
        launch_mlp_bf16<1, 8>(d, nets, n_tiles, D, Dp, rows, s);
    else if (mlp_mode == 1)
        launch_mlp_bf16<1, 4>(d, nets, n_tiles, D, Dp, rows, s);
    else if (mlp_mode == 2 && waves == 8)
        launch_mlp_bf16<2, 8>(d, nets, n_tiles, D, Dp, rows, s);
    else if (mlp_mode == 2)
        launch_mlp_bf16<2, 4>(d, nets, n_tiles, D, Dp, rows, s);
    else
        launch_mlp_fp32(d, nets, n_tiles, D, Dp, rows, s);
}

}  // namespace pimd
