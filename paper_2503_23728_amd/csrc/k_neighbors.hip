// Per-bead cell lists and neighbour lists (the molecular graph of Sec. 2.2
// with the cutoff of Tables S1/S2), periodic orthorhombic boxes.
//
// Membership is decided in float32 with one rounding per operation (no
// contraction into fused multiply-adds), so it is reproducible bit for bit:
//   x_w = x - L floor(x invL)            wrap into the box, invL = fl32(1/L)
//   d   = x_w[j] - x_w[i]; d -= L rint(d invL)
//   r2  = (dx dx + dy dy) + dz dz;  j is a neighbour iff j != i and r2 < fl32(rc^2)
// Non-periodic systems test every pair on the raw positions.
//
// Output per centre row i: nbr[i][0..cnt) holds keys (element << 27) | row,
// sorted ascending, i.e. grouped by element and ascending row within a
// group; nbr_grp[i][e] counts each element's group.
#include "device_common.hpp"

namespace pimd {

#pragma clang fp contract(off)

__device__ __forceinline__ float wrap_coord(float x, float L, float invL)
{
    const float t = x * invL;
    const float f = floorf(t);
    const float m = L * f;
    return x - m;
}

__device__ __forceinline__ int cell_of(float xw, float scale, int nc)
{
    int c = (int)(xw * scale);
    c = c < 0 ? 0 : c;
    return c >= nc ? nc - 1 : c;
}

__global__ __launch_bounds__(256) void k_wrap_bin(const float *__restrict__ q, const BeadInfo *__restrict__ beads,
                                                  const int32_t *__restrict__ bead_of_ba,
                                                  const int32_t *__restrict__ species_atom,
                                                  const SysInfo *__restrict__ sys, float4 *__restrict__ pos4,
                                                  float4 *__restrict__ posu4,
                                                  int32_t *__restrict__ cell_count, int32_t *__restrict__ atom_cell,
                                                  int32_t *__restrict__ atom_slot, int B)
{
    const int ba = blockIdx.x * blockDim.x + threadIdx.x;
    if (ba >= B)
        return;
    const BeadInfo bi = beads[bead_of_ba[ba]];
    const int local = (ba - bi.ba0);
    const int atom = sys[bi.sys].atom0 + local % bi.n;
    const int z = species_atom[atom];
    float x = q[3 * ba + 0], y = q[3 * ba + 1], w = q[3 * ba + 2];
    posu4[ba] = make_float4(x, y, w, __int_as_float(z));
    if (bi.periodic) {
        x = wrap_coord(x, bi.L[0], bi.invL[0]);
        y = wrap_coord(y, bi.L[1], bi.invL[1]);
        w = wrap_coord(w, bi.L[2], bi.invL[2]);
        const int cx = cell_of(x, bi.cell_scale[0], bi.nc[0]);
        const int cy = cell_of(y, bi.cell_scale[1], bi.nc[1]);
        const int cz = cell_of(w, bi.cell_scale[2], bi.nc[2]);
        const int c = bi.cell0 + (cx * bi.nc[1] + cy) * bi.nc[2] + cz;
        atom_cell[ba] = c;
        atom_slot[ba] = atomicAdd(&cell_count[c], 1);
    }
    pos4[ba] = make_float4(x, y, w, __int_as_float(z));
}

// Exclusive scan of the cell counts of one bead (one workgroup per bead).
__global__ __launch_bounds__(256) void k_cell_scan(const BeadInfo *__restrict__ beads,
                                                   const int32_t *__restrict__ cell_count,
                                                   int32_t *__restrict__ cell_start)
{
    const BeadInfo bi = beads[blockIdx.x];
    if (!bi.periodic)
        return;
    const int ncell = bi.nc[0] * bi.nc[1] * bi.nc[2];
    __shared__ int32_t part[256];
    __shared__ int32_t carry;
    if (threadIdx.x == 0)
        carry = 0;
    __syncthreads();
    for (int base = 0; base < ncell; base += 256) {
        const int c = base + threadIdx.x;
        const int v = c < ncell ? cell_count[bi.cell0 + c] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const int t = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
            __syncthreads();
            part[threadIdx.x] += t;
            __syncthreads();
        }
        if (c < ncell)
            cell_start[bi.cell0 + c] = carry + part[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 255)
            carry += part[255];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_cell_fill(const BeadInfo *__restrict__ beads,
                                                   const int32_t *__restrict__ bead_of_ba,
                                                   const int32_t *__restrict__ atom_cell,
                                                   const int32_t *__restrict__ atom_slot,
                                                   const int32_t *__restrict__ cell_start,
                                                   int32_t *__restrict__ cell_atoms, int B)
{
    const int ba = blockIdx.x * blockDim.x + threadIdx.x;
    if (ba >= B)
        return;
    const BeadInfo bi = beads[bead_of_ba[ba]];
    // rows of a bead in cell order (the centre order of the per-centre
    // kernels); a bead without a box keeps its own row order
    cell_atoms[bi.periodic ? bi.ba0 + cell_start[atom_cell[ba]] + atom_slot[ba] : ba] = ba;
}

// Keys buffered per wave: up to Kmax + 63 candidates (a pass may overshoot
// Kmax) and room for the sort's padding to a power of two.
__host__ __device__ inline int nl_buffer(int Kmax)
{
    int n = 1;
    while (n < Kmax)
        n <<= 1;
    return n > Kmax + kWave ? n : Kmax + kWave;
}

__device__ __forceinline__ bool within_cutoff(const float4 &pi, const float4 &pj, const BeadInfo &bi, float rc2)
{
    float dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
    if (bi.periodic) {
        const float sx = bi.L[0] * rintf(dx * bi.invL[0]);
        const float sy = bi.L[1] * rintf(dy * bi.invL[1]);
        const float sz = bi.L[2] * rintf(dz * bi.invL[2]);
        dx = dx - sx;
        dy = dy - sy;
        dz = dz - sz;
    }
    const float xx = dx * dx, yy = dy * dy, zz = dz * dz;
    const float r2 = (xx + yy) + zz;
    return r2 < rc2;
}

// One wave per centre row.  Candidates come from the (deduplicated) 27-cell
// stencil, or every atom of the bead when the system is not periodic;
// accepted keys are compacted into LDS and rank-sorted.
__global__ __launch_bounds__(256) void k_neighbors(const float4 *__restrict__ pos4,
                                                   const BeadInfo *__restrict__ beads,
                                                   const int32_t *__restrict__ bead_of_ba,
                                                   const int32_t *__restrict__ cell_count,
                                                   const int32_t *__restrict__ cell_start,
                                                   const int32_t *__restrict__ cell_atoms,
                                                   const int32_t *__restrict__ order, float rc2, int Kmax,
                                                   int n_el, int32_t *__restrict__ nbr, int32_t *__restrict__ nbr_cnt,
                                                   int32_t *__restrict__ nbr_grp, uint32_t *__restrict__ status, int B)
{
    extern __shared__ int32_t nl_lds[];
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    int32_t *buf = nl_lds + w * nl_buffer(Kmax);
    const uint64_t below = lanes_below_mask();
    const CentreRange cr = centre_range(B);
    for (int ci = cr.begin; ci < cr.end; ++ci) {
        // wave-uniform: the per-centre values below live in scalar registers
        const int i = __builtin_amdgcn_readfirstlane(order ? order[ci] : ci);
        const BeadInfo bi = beads[bead_of_ba[i]];
        const float4 pi = pos4[i];
        int count = 0;
        auto consider = [&](int j, bool valid) {
            bool acc = false;
            float4 pj;
            if (valid && j != i) {
                pj = pos4[j];
                acc = within_cutoff(pi, pj, bi, rc2);
            }
            const uint64_t m = __ballot(acc);
            const int pos = count + __popcll(m & below);
            if (acc && pos < Kmax) {
                const int z = __float_as_int(pj.w);
                buf[pos] = (z << kKeyShift) | j;
            }
            count += __popcll(m);
        };
        if (bi.periodic) {
            // the (deduplicated) stencil cells, one per lane: lane c < n_cells
            // holds cell c's first slot and its end in the flattened candidate
            // index space, so each pass tests 64 candidates of any cells
            const int cx = cell_of(pi.x, bi.cell_scale[0], bi.nc[0]);
            const int cy = cell_of(pi.y, bi.cell_scale[1], bi.nc[1]);
            const int cz = cell_of(pi.z, bi.cell_scale[2], bi.nc[2]);
            const int an0 = bi.nc[0] < 3 ? bi.nc[0] : 3, an1 = bi.nc[1] < 3 ? bi.nc[1] : 3;
            const int an2 = bi.nc[2] < 3 ? bi.nc[2] : 3;
            const int n_cells = an0 * an1 * an2;
            int first = 0, cnt = 0;
            if (lane < n_cells) {
                const int c = lane % an2, b = (lane / an2) % an1, a = lane / (an1 * an2);
                // axis offsets -1, 0, +1 (or every cell of an axis with fewer than 3)
                const int ux = bi.nc[0] < 3 ? a : (cx + bi.nc[0] - 1 + a) % bi.nc[0];
                const int uy = bi.nc[1] < 3 ? b : (cy + bi.nc[1] - 1 + b) % bi.nc[1];
                const int uz = bi.nc[2] < 3 ? c : (cz + bi.nc[2] - 1 + c) % bi.nc[2];
                const int cell = bi.cell0 + (ux * bi.nc[1] + uy) * bi.nc[2] + uz;
                first = cell_start[cell];
                cnt = cell_count[cell];
            }
            int end = cnt;   // inclusive prefix sum of the counts over the lanes
            for (int o = 1; o < kWave; o <<= 1) {
                const int t = __shfl_up(end, o, kWave);
                end += lane >= o ? t : 0;
            }
            const int total = __shfl(end, kWave - 1, kWave);
            const int base = first - (end - cnt);   // slot of candidate t in cell c: base_c + t
            for (int t0 = 0; t0 < total; t0 += kWave) {
                const int t = t0 + lane;
                const bool valid = t < total;
                int k = 0;   // the cell holding candidate t: number of cell ends <= t
                for (int c = 0; c < n_cells; ++c)
                    k += t >= __shfl(end, c, kWave) ? 1 : 0;
                const int bk = __shfl(base, k < n_cells ? k : 0, kWave);
                const int j = valid ? cell_atoms[bi.ba0 + bk + t] : 0;
                consider(j, valid);
            }
        } else {
            for (int t0 = 0; t0 < bi.n; t0 += kWave) {
                const int t = t0 + lane;
                consider(bi.ba0 + t, t < bi.n);
            }
        }
        wave_sync();
        if (count > Kmax && lane == 0)
            atomicOr(status, kStatusOverflow);
        const int K = count < Kmax ? count : Kmax;
        // bitonic sort of the K keys (distinct) in the wave's buffer, padded
        // with INT_MAX to a power of two; then the sorted keys go out
        // coalesced and the element groups are counted from them
        int n = 1;
        while (n < K)
            n <<= 1;
        for (int t = K + lane; t < n; t += kWave)
            buf[t] = 0x7FFFFFFF;
        wave_sync();
        for (int size = 2; size <= n; size <<= 1)
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int p = lane; p < (n >> 1); p += kWave) {
                    const int lo = ((p & ~(stride - 1)) << 1) | (p & (stride - 1)), hi = lo + stride;
                    const int a = buf[lo], b = buf[hi];
                    if ((a > b) == ((lo & size) == 0)) {
                        buf[lo] = b;
                        buf[hi] = a;
                    }
                }
                wave_sync();
            }
        int32_t *out = nbr + (int64_t)i * Kmax;
        int grp[kMaxElements] = {0, 0, 0, 0};
        for (int t0 = 0; t0 < K; t0 += kWave) {
            const int t = t0 + lane;
            const int v = t < K ? buf[t] : -1;
            if (t < K)
                out[t] = v;
#pragma unroll
            for (int e = 0; e < kMaxElements; ++e)
                grp[e] += __popcll(__ballot(t < K && (v >> kKeyShift) == e));
        }
        if (lane < n_el) {
            int c = grp[0];
#pragma unroll
            for (int e = 1; e < kMaxElements; ++e)
                c = lane == e ? grp[e] : c;
            nbr_grp[(int64_t)i * kMaxElements + lane] = c;
        }
        if (lane == 0)
            nbr_cnt[i] = K;
        wave_sync();
    }
}

__global__ void k_zero_i32(int32_t *p, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n)
        p[t] = 0;
}

void launch_zero_i32(int32_t *p, int64_t n, hipStream_t s)
{
    if (n <= 0)
        return;
    hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
}

void launch_wrap_bin(const float *q, const DevBuffers &d, const Sizes &z, hipStream_t s)
{
    hipLaunchKernelGGL(k_wrap_bin, dim3((z.B + 255) / 256), dim3(256), 0, s, q, d.beads, d.bead_of_ba,
                       d.species_atom, d.sys, d.pos4, d.posu4, d.cell_count, d.atom_cell, d.atom_slot, z.B);
}

void launch_cell_scan(const DevBuffers &d, const Sizes &z, hipStream_t s)
{
    hipLaunchKernelGGL(k_cell_scan, dim3(z.n_beads_total), dim3(256), 0, s, d.beads, d.cell_count, d.cell_start);
}

void launch_cell_fill(const DevBuffers &d, const Sizes &z, hipStream_t s)
{
    hipLaunchKernelGGL(k_cell_fill, dim3((z.B + 255) / 256), dim3(256), 0, s, d.beads, d.bead_of_ba, d.atom_cell,
                       d.atom_slot, d.cell_start, d.cell_atoms, z.B);
}

void launch_neighbors(const DevBuffers &d, const Sizes &z, float rc2, int n_el, const Tuning &tn, hipStream_t s)
{
    const int wpg = tn.centre_waves;
    const size_t lds = (size_t)wpg * nl_buffer(z.Kmax) * sizeof(int32_t);
    hipLaunchKernelGGL(k_neighbors, dim3(centre_grid(z.B, tn)), dim3(kWave * wpg), lds, s, d.pos4, d.beads,
                       d.bead_of_ba, d.cell_count, d.cell_start, d.cell_atoms, centre_order(d, z), rc2, z.Kmax, n_el,
                       d.nbr, d.nbr_cnt,
                       d.nbr_grp, d.status, z.B);
}

}  // namespace pimd
