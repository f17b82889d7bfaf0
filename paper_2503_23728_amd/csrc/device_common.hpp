// Device helpers: wave-level synchronisation and reductions, bfloat16
// rounding, and the Philox4x32-10 generator of the thermostat noise.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pimd_internal.hpp"

namespace pimd {

// Orders the LDS accesses of one wave across lanes (lanes of a wave run in
// lock step; this stops the compiler from moving accesses across the point).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Butterfly sum over the 64 lanes; every lane gets the total.  The order of
// the additions is fixed, so the result is bitwise reproducible.
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, kWave);
    return v;
}

// Transposed reduction of N per-lane values (N a power of two, 2..64): each
// butterfly step exchanges half of the remaining values with the partner
// lane, so the total shuffle count is N - 1 + log2(64/N) instead of 6N.
// Afterwards lane l holds the wave total of value (l / (64/N)) and every lane
// of the same group of 64/N lanes holds the same total.  Fixed order: bitwise
// reproducible.
template <int N>
__device__ __forceinline__ float transpose_reduce(float (&v)[N])
{
    const int lane = lane_id();
#pragma unroll
    for (int half = N / 2, d = 32; half >= 1; half /= 2, d /= 2) {
        // bit select (not a ?: on two array elements, which the compiler may
        // turn into a dynamically indexed access and move the array to scratch)
        const uint32_t m = (lane & d) ? 0xFFFFFFFFu : 0u;
#pragma unroll
        for (int j = 0; j < half; ++j) {
            const uint32_t a = __float_as_uint(v[j]), b = __float_as_uint(v[j + half]);
            const float keep = __uint_as_float((a & ~m) | (b & m));
            const float send = __uint_as_float((b & ~m) | (a & m));
            v[j] = keep + __shfl_xor(send, d, kWave);
        }
    }
    float t = v[0];
#pragma unroll
    for (int d = 32 / N; d >= 1; d /= 2)
        t += __shfl_xor(t, d, kWave);
    return t;
}

// Sum over the 16 lanes that share lane / 16.
__device__ __forceinline__ float row16_sum(float v)
{
#pragma unroll
    for (int o = 8; o > 0; o >>= 1)
        v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ uint64_t lanes_below_mask()
{
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// float -> bfloat16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// products mixed with the other counter words and the round key; the key
// advances by the Weyl constants after each round.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = c.x * 0xD2511F53u, hi0 = __umulhi(c.x, 0xD2511F53u);
        const uint32_t lo1 = c.z * 0xCD9E8D57u, hi1 = __umulhi(c.z, 0xCD9E8D57u);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Thermostat normal for component comp (0, 1, 2) of counter row `row`:
// u = (x + 1/2) 2^-32; Box-Muller on (u0, u1) gives x and y, on (u2, u3) z.
__device__ __forceinline__ float thermostat_normal(uint32_t k0, uint32_t k1, int64_t step, int half,
                                                   int64_t row, int comp)
{
    const uint4 w = philox4x32_10(make_uint4((uint32_t)row, (uint32_t)half, (uint32_t)step,
                                             (uint32_t)((uint64_t)step >> 32)), k0, k1);
    const float scale = 2.3283064365386963e-10f;  // 2^-32
    const uint32_t xr = comp < 2 ? w.x : w.z;
    const uint32_t xa = comp < 2 ? w.y : w.w;
    const float ur = fmaf((float)xr, scale, 0.5f * scale);
    const float ua = fmaf((float)xa, scale, 0.5f * scale);
    const float r = sqrtf(-2.0f * logf(ur));
    float sn, cs;
    sincospif(2.0f * ua, &sn, &cs);
    return comp == 1 ? r * sn : r * cs;
}

// Centres of one wave in the per-centre kernels.  Workgroups are dispatched
// round-robin over the 8 XCDs of the chip, each with its own L2; the logical
// block index gives XCD x the contiguous block range it serves, and each wave
// takes a contiguous run of the centre order (cell order, so consecutive
// centres share their neighbourhoods).  A bijection of [0, G) for any G.
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_block(int b, int G)
{
    const int x = b % kXcds, k = b / kXcds, q = G / kXcds, r = G % kXcds;
    return x * q + (x < r ? x : r) + k;
}

struct CentreRange {
    int begin, end;
};

__device__ __forceinline__ CentreRange centre_range(int B)
{
    const int wpg = blockDim.x >> 6, w = threadIdx.x >> 6;
    const int nw = gridDim.x * wpg;
    const int v = xcd_block(blockIdx.x, gridDim.x) * wpg + w;
    const int per = (B + nw - 1) / nw;
    const int b0 = v * per;
    return CentreRange{b0 < B ? b0 : B, b0 + per < B ? b0 + per : B};
}

// Slot of key_i in atom j's sorted list, or -1 when it is not there.  The
// lists are symmetric, so this is where atom j keeps the pair (j, i): j's
// fence row (its count and every 16th key) picks the 16-key segment, the
// segment the slot; two dependent 64-byte reads instead of a binary search.
__device__ __forceinline__ int reverse_slot(const int32_t *__restrict__ nbr, const int32_t *__restrict__ fence,
                                            int Kmax, int j, int key_i)
{
    const int4 *fj = reinterpret_cast<const int4 *>(fence + (int64_t)j * kFence);
    int seg = 0, Kj = 0;
#pragma unroll
    for (int c = 0; c < kFence / 4; ++c) {
        const int4 f = fj[c];
        Kj = c == 0 ? f.x : Kj;
        seg += (c > 0 && f.x <= key_i) + (f.y <= key_i) + (f.z <= key_i) + (f.w <= key_i);
    }
    const int4 *sj = reinterpret_cast<const int4 *>(nbr + (int64_t)j * Kmax + 16 * seg);
    int m = 16 * seg, hit = -1;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int4 kv = 16 * seg + 4 * c < Kj ? sj[c] : make_int4(0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF, 0x7FFFFFFF);
        const int kk[4] = {kv.x, kv.y, kv.z, kv.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int pos = 16 * seg + 4 * c + e;
            const bool in = pos < Kj;
            m += (in && kk[e] < key_i) ? 1 : 0;
            hit = (in && kk[e] == key_i) ? pos : hit;
        }
    }
    return hit >= 0 && hit == m ? hit : -1;
}

// After the adjoint of centre i: v[i][n] goes to its own slot and, with
// vrev, to the slot that atom j = nbr[i][n] keeps for i, so that the force
// assembly reads both terms of every pair from atom i's own rows.  An
// asymmetric list (never built by the neighbour kernels) is reported as an
// overflow.
__device__ __forceinline__ void store_slot_values(const int32_t *__restrict__ nbr, const int32_t *__restrict__ fence,
                                                  int Kmax, int i, int key_i, int n, const float4 &v,
                                                  float4 *__restrict__ vslot, float4 *__restrict__ vrev,
                                                  bool &missing)
{
    vslot[(int64_t)i * Kmax + n] = v;
    if (!vrev)
        return;
    const int j = nbr[(int64_t)i * Kmax + n] & (int)kRowMask;
    const int hit = reverse_slot(nbr, fence, Kmax, j, key_i);
    if (hit >= 0)
        vrev[(int64_t)j * Kmax + hit] = v;
    else
        missing = true;
}

}  // namespace pimd
