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
#include "neighbor_test.hpp"

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
    const int b = n > Kmax + kWave ? n : Kmax + kWave;
    return (b + 3) & ~3;
}

// The (deduplicated) stencil of cell (cx, cy, cz), one cell per lane: lane
// c < n_cells holds cell c's first slot in the bead's cell-sorted atoms and
// the inclusive end of its candidates in a flat index space over all stencil
// cells (lanes past n_cells hold the total), so a pass tests 64 candidates
// drawn from any cells.
struct Stencil {
    int n_cells, end, base, total;   // candidate t of cell c sits at slot base_c + t
};

__device__ __forceinline__ Stencil stencil_of(const BeadInfo &bi, int cx, int cy, int cz,
                                              const int32_t *cell_start, const int32_t *cell_count)
{
    const int lane = lane_id();
    const int an0 = bi.nc[0] < 3 ? bi.nc[0] : 3, an1 = bi.nc[1] < 3 ? bi.nc[1] : 3;
    const int an2 = bi.nc[2] < 3 ? bi.nc[2] : 3;
    Stencil st;
    st.n_cells = an0 * an1 * an2;
    int first = 0, cnt = 0;
    if (lane < st.n_cells) {
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
    st.end = end;
    st.total = __shfl(end, kWave - 1, kWave);
    st.base = first - (end - cnt);
    return st;
}

// Slot (in the bead's cell-sorted atoms) of flat candidate t.
__device__ __forceinline__ int stencil_slot(const Stencil &st, int t)
{
    int k = 0;   // the cell holding candidate t: number of cell ends <= t
    for (int c = 0; c < st.n_cells; ++c)
        k += t >= __shfl(st.end, c, kWave) ? 1 : 0;
    return __shfl(st.base, k < st.n_cells ? k : 0, kWave) + t;
}

// Appends the accepted keys of one pass to the wave's buffer.
__device__ __forceinline__ void append_keys(bool acc, int key, int Kmax, int32_t *buf, int &count)
{
    const uint64_t m = __ballot(acc);
    const int pos = count + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    if (acc && pos < Kmax)
        buf[pos] = key;
    count += __popcll(m);
}

// Sorts the wave's `count` keys (distinct) and writes list, count and
// element groups of centre i: a bitonic network in the buffer, padded with
// INT_MAX to a power of two; the element groups are counted with ballots
// over the sorted keys.
__device__ __forceinline__ void finish_list(int32_t *buf, int count, int i, int Kmax, int n_el,
                                            int32_t *__restrict__ nbr, int32_t *__restrict__ nbr_cnt,
                                            int32_t *__restrict__ nbr_grp, int32_t *__restrict__ fence,
                                            uint32_t *__restrict__ status)
{
    const int lane = lane_id();
    wave_sync();
    if (count > Kmax && lane == 0)
        atomicOr(status, kStatusOverflow);
    const int K = count < Kmax ? count : Kmax;
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
    // fence row: the count, then every 16th key (INT_MAX past the end)
    if (lane < kFence)
        fence[(int64_t)i * kFence + lane] = lane == 0 ? K : (16 * lane < K ? buf[16 * lane] : 0x7FFFFFFF);
    wave_sync();
}

// One wave per centre row, candidates read from global memory: the stencil
// cells of a periodic bead, or every atom of a bead without a box.  With
// skip_periodic the periodic centres are left to k_neighbors_cells.
__global__ __launch_bounds__(256) void k_neighbors(const float4 *__restrict__ pos4,
                                                   const BeadInfo *__restrict__ beads,
                                                   const int32_t *__restrict__ bead_of_ba,
                                                   const int32_t *__restrict__ cell_count,
                                                   const int32_t *__restrict__ cell_start,
                                                   const int32_t *__restrict__ cell_atoms,
                                                   const int32_t *__restrict__ order, float rc2, int Kmax,
                                                   int n_el, int skip_periodic, int32_t *__restrict__ nbr,
                                                   int32_t *__restrict__ nbr_cnt, int32_t *__restrict__ nbr_grp,
                                                   int32_t *__restrict__ fence, uint32_t *__restrict__ status,
                                                   int B)
{
    extern __shared__ int32_t nl_lds[];
    const int lane = lane_id();
    const int w = threadIdx.x >> 6;
    int32_t *buf = nl_lds + w * nl_buffer(Kmax);
    const CentreRange cr = centre_range(B);
    for (int ci = cr.begin; ci < cr.end; ++ci) {
        // wave-uniform: the per-centre values below live in scalar registers
        const int i = __builtin_amdgcn_readfirstlane(order ? order[ci] : ci);
        const BeadInfo bi = beads[bead_of_ba[i]];
        if (bi.periodic && skip_periodic)
            continue;
        const float4 pi = pos4[i];
        int count = 0;
        auto consider = [&](int j, bool valid) {
            bool acc = false;
            float4 pj = pi;
            if (valid && j != i) {
                pj = pos4[j];
                acc = within_cutoff(pi, pj, bi, rc2);
            }
            append_keys(acc, (__float_as_int(pj.w) << kKeyShift) | j, Kmax, buf, count);
        };
        if (bi.periodic) {
            const Stencil st = stencil_of(bi, cell_of(pi.x, bi.cell_scale[0], bi.nc[0]),
                                          cell_of(pi.y, bi.cell_scale[1], bi.nc[1]),
                                          cell_of(pi.z, bi.cell_scale[2], bi.nc[2]), cell_start, cell_count);
            for (int t0 = 0; t0 < st.total; t0 += kWave) {
                const int t = t0 + lane;
                const bool valid = t < st.total;
                const int slot = stencil_slot(st, t);
                consider(valid ? cell_atoms[bi.ba0 + slot] : 0, valid);
            }
        } else {
            for (int t0 = 0; t0 < bi.n; t0 += kWave) {
                const int t = t0 + lane;
                consider(bi.ba0 + t, t < bi.n);
            }
        }
        finish_list(buf, count, i, Kmax, n_el, nbr, nbr_cnt, nbr_grp, fence, status);
    }
}

// One workgroup per cell of a periodic bead: the atoms of the cell's stencil
// are staged in LDS once (rows and positions) and every centre of the cell,
// a wave each, tests them from there instead of gathering them from global
// memory centre by centre.  A stencil with more than max_cand atoms is read
// from global memory as in k_neighbors.  The lists are the same.
__global__ __launch_bounds__(256) void k_neighbors_cells(const float4 *__restrict__ pos4,
                                                         const BeadInfo *__restrict__ beads,
                                                         const int32_t *__restrict__ cell_bead,
                                                         const int32_t *__restrict__ cell_count,
                                                         const int32_t *__restrict__ cell_start,
                                                         const int32_t *__restrict__ cell_atoms, float rc2,
                                                         int Kmax, int n_el, int max_cand,
                                                         int32_t *__restrict__ nbr, int32_t *__restrict__ nbr_cnt,
                                                         int32_t *__restrict__ nbr_grp, int32_t *__restrict__ fence,
                                                         uint32_t *__restrict__ status)
{
    extern __shared__ int32_t nl_lds[];
    const int lane = lane_id();
    const int w = threadIdx.x >> 6, wpg = blockDim.x >> 6;
    const int nlb = nl_buffer(Kmax);
    int32_t *buf = nl_lds + w * nlb;
    int32_t *crow = nl_lds + wpg * nlb;
    float4 *cpos = reinterpret_cast<float4 *>(crow + max_cand);   // max_cand and nlb are multiples of 4
    const int cell = xcd_block(blockIdx.x, gridDim.x);
    const BeadInfo bi = beads[cell_bead[cell]];
    const int home_n = cell_count[cell], home_first = cell_start[cell];
    if (home_n == 0)
        return;
    const int local = cell - bi.cell0;
    const int cz = local % bi.nc[2], cy = (local / bi.nc[2]) % bi.nc[1], cx = local / (bi.nc[1] * bi.nc[2]);
    const Stencil st = stencil_of(bi, cx, cy, cz, cell_start, cell_count);
    const bool staged = st.total <= max_cand;
    if (staged) {
        for (int t0 = 0; t0 < st.total; t0 += blockDim.x) {
            const int t = t0 + (int)threadIdx.x;
            const int slot = stencil_slot(st, t);
            if (t < st.total) {
                const int j = cell_atoms[bi.ba0 + slot];
                crow[t] = j;
                cpos[t] = pos4[j];
            }
        }
        __syncthreads();
    }
    for (int s = w; s < home_n; s += wpg) {
        const int i = __builtin_amdgcn_readfirstlane(cell_atoms[bi.ba0 + home_first + s]);
        const float4 pi = pos4[i];
        int count = 0;
        for (int t0 = 0; t0 < st.total; t0 += kWave) {
            const int t = t0 + lane;
            const bool valid = t < st.total;
            int j;
            float4 pj;
            if (staged) {
                j = valid ? crow[t] : i;
                pj = valid ? cpos[t] : pi;
            } else {
                const int slot = stencil_slot(st, t);
                j = valid ? cell_atoms[bi.ba0 + slot] : i;
                pj = pos4[j];
            }
            const bool acc = j != i && within_cutoff(pi, pj, bi, rc2);
            append_keys(acc, (__float_as_int(pj.w) << kKeyShift) | j, Kmax, buf, count);
        }
        finish_list(buf, count, i, Kmax, n_el, nbr, nbr_cnt, nbr_grp, fence, status);
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

// ---------------------------------------------------------------------------
// Shared neighbour lists with a skin: one list per atom of the ring-polymer
// centroids, with the cutoff widened by the skin, rebuilt only when some bead
// has left the sphere of half the skin around its atom's centroid of the
// last build; every bead's list is that list filtered with the float32
// decision above.  If every bead-atom q^k_i is within s/2 of c_i (the build
// centroid), a pair of bead k within R_c under the image shift n has
// |c_i - c_j - n L| < R_c + s, so the minimum-image centroid distance is below
// R_c + s too and the centroid list holds j; the filtered lists equal the
// per-bead search key for key (same decision, same (element, row) order).
// The guarantee needs the positions of the step itself within s/2 of the
// centroids of the list: when the rebuild finds a bead already farther
// than that from its fresh centroid (a ring spread wider than the skin), the
// step's filter tests every atom of the bead instead.
// flag[0]: rebuild request; flag[1]: this step's lists cannot be trusted.
// ---------------------------------------------------------------------------

// Wrap as k_wrap_bin (no cells) and flag a rebuild when a bead-atom's
// unwrapped position is more than half the skin from its build centroid.
__global__ __launch_bounds__(256) void k_wrap_skin(const float *__restrict__ q, const BeadInfo *__restrict__ beads,
                                                   const int32_t *__restrict__ bead_of_ba,
                                                   const int32_t *__restrict__ species_atom,
                                                   const SysInfo *__restrict__ sys, const double4 *__restrict__ c0,
                                                   double half_skin2, float4 *__restrict__ pos4,
                                                   float4 *__restrict__ posu4, int32_t *__restrict__ flag, int B)
{
    const int ba = blockIdx.x * blockDim.x + threadIdx.x;
    if (ba == 0)
        flag[1] = 0;
    if (ba >= B)
        return;
    const BeadInfo bi = beads[bead_of_ba[ba]];
    const int atom = sys[bi.sys].atom0 + (ba - bi.ba0);
    const int z = species_atom[atom];
    float x = q[3 * ba + 0], y = q[3 * ba + 1], w = q[3 * ba + 2];
    posu4[ba] = make_float4(x, y, w, __int_as_float(z));
    const double4 c = c0[atom];
    const double dx = (double)x - c.x, dy = (double)y - c.y, dz = (double)w - c.z;
    if (!(dx * dx + dy * dy + dz * dz <= half_skin2))   // also catches a non-finite position
        atomicOr(&flag[0], 1);
    x = wrap_coord(x, bi.L[0], bi.invL[0]);
    y = wrap_coord(y, bi.L[1], bi.invL[1]);
    w = wrap_coord(w, bi.L[2], bi.invL[2]);
    pos4[ba] = make_float4(x, y, w, __int_as_float(z));
}

// Rebuild, step 1 (only when flagged): centroid of every atom over its beads,
// and whether every bead is within s/2 of it.
__global__ __launch_bounds__(256) void k_skin_centroids(const float4 *__restrict__ posu4,
                                                        const SysInfo *__restrict__ sys,
                                                        const int32_t *__restrict__ sys_of_atom,
                                                        double half_skin2, int32_t *__restrict__ flag,
                                                        double4 *__restrict__ c0, int A)
{
    if (flag[0] == 0)
        return;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= A)
        return;
    const SysInfo S = sys[sys_of_atom[a]];
    const int local = a - S.atom0;
    double x = 0.0, y = 0.0, z = 0.0;
    for (int k = 0; k < S.P; ++k) {
        const float4 p = posu4[S.ba0 + k * S.N + local];
        x += p.x;
        y += p.y;
        z += p.z;
    }
    const double inv = 1.0 / S.P;
    x *= inv;
    y *= inv;
    z *= inv;
    c0[a] = make_double4(x, y, z, 0.0);
    for (int k = 0; k < S.P; ++k) {
        const float4 p = posu4[S.ba0 + k * S.N + local];
        const double dx = p.x - x, dy = p.y - y, dz = p.z - z;
        if (!(dx * dx + dy * dy + dz * dz <= half_skin2)) {
            atomicOr(&flag[1], 1);
            break;
        }
    }
}

// Rebuild, step 2 (only when flagged): one wave per atom, every atom of its
// system tested in FP64 (minimum image) against (R_c + s + 1e-3 A)^2, one pass
// per element so the keys (element << 27) | local atom come out sorted.
__global__ __launch_bounds__(256) void k_skin_lists(const double4 *__restrict__ c0, const SysInfo *__restrict__ sys,
                                                    const int32_t *__restrict__ sys_of_atom,
                                                    const int32_t *__restrict__ species_atom,
                                                    const BeadInfo *__restrict__ beads,
                                                    const int32_t *__restrict__ bead_of_ba, double reach2, int n_el,
                                                    int Kc, const int32_t *__restrict__ flag,
                                                    int32_t *__restrict__ keys, int32_t *__restrict__ cnt,
                                                    unsigned long long *__restrict__ builds,
                                                    uint32_t *__restrict__ status, int A)
{
    if (flag[0] == 0)
        return;
    const int lane = lane_id();
    const int a = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        atomicAdd(builds, 1ull);
    if (a >= A)
        return;
    const SysInfo S = sys[sys_of_atom[a]];
    const BeadInfo bi = beads[bead_of_ba[S.ba0]];
    const int il = a - S.atom0;
    const double4 ci = c0[a];
    int32_t *out = keys + (int64_t)a * Kc;
    int count = 0;
    for (int e = 0; e < n_el; ++e)
        for (int j0 = 0; j0 < S.N; j0 += kWave) {
            const int jl = j0 + lane;
            bool acc = false;
            if (jl < S.N && jl != il && species_atom[S.atom0 + jl] == e) {
                const double4 cj = c0[S.atom0 + jl];
                double dx = cj.x - ci.x, dy = cj.y - ci.y, dz = cj.z - ci.z;
                dx -= bi.L64[0] * rint(dx * bi.invL64[0]);
                dy -= bi.L64[1] * rint(dy * bi.invL64[1]);
                dz -= bi.L64[2] * rint(dz * bi.invL64[2]);
                acc = dx * dx + dy * dy + dz * dz < reach2;
            }
            const uint64_t m = __ballot(acc);
            const int pos = count + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            if (acc && pos < Kc)
                out[pos] = (e << kKeyShift) | jl;
            count += __popcll(m);
        }
    if (lane == 0) {
        cnt[a] = count < Kc ? count : Kc;
        if (count > Kc)
            atomicOr(status, kStatusOverflow);
    }
}

// Every step: one wave per bead-atom row, its atom's centroid list filtered
// with within_cutoff on the wrapped bead positions, written in order (the
// candidates are sorted, and row = first row of the bead + local atom keeps
// the order), with the element groups and the fence row of finish_list.
// When flag[1] is set, every atom of the bead is a candidate, element by
// element in row order (the same order).
__global__ __launch_bounds__(256) void k_skin_filter(const float4 *__restrict__ pos4,
                                                     const BeadInfo *__restrict__ beads,
                                                     const int32_t *__restrict__ bead_of_ba,
                                                     const SysInfo *__restrict__ sys,
                                                     const int32_t *__restrict__ keys,
                                                     const int32_t *__restrict__ cnt, int Kc, float rc2, int Kmax,
                                                     int n_el, int32_t *__restrict__ flag,
                                                     unsigned long long *__restrict__ full_scans,
                                                     int32_t *__restrict__ nbr, int32_t *__restrict__ nbr_cnt,
                                                     int32_t *__restrict__ nbr_grp, int32_t *__restrict__ fence,
                                                     uint32_t *__restrict__ status, int B)
{
    const int lane = lane_id();
    const bool scan_all = __builtin_amdgcn_readfirstlane(flag[1]) != 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        flag[0] = 0;   // this step's lists are built (the build kernels ran before)
        if (scan_all)
            atomicAdd(full_scans, 1ull);
    }
    const CentreRange cr = centre_range(B);
    for (int i = cr.begin; i < cr.end; ++i) {
        const BeadInfo bi = beads[bead_of_ba[i]];
        const int atom = sys[bi.sys].atom0 + (i - bi.ba0);
        const int n_cand = scan_all ? n_el * bi.n : cnt[atom];
        const int32_t *cand = keys + (int64_t)atom * Kc;
        const float4 pi = pos4[i];
        int32_t *out = nbr + (int64_t)i * Kmax;
        int count = 0;
        int grp[kMaxElements] = {0, 0, 0, 0};
        // list candidates: keys loaded two chunks ahead and positions one
        // chunk ahead, so a chunk's two dependent loads are in flight while
        // the chunks before it are tested
        // (only on the list path: a whole-bead scan has no list, and key 0 names
        // the bead's first row, so every prefetch stays inside the bead)
        const int n_list = scan_all ? 0 : n_cand;
        int c_next = lane < n_list ? cand[lane] : 0;
        int c_after = kWave + lane < n_list ? cand[kWave + lane] : 0;
        float4 p_next = pos4[bi.ba0 + (c_next & (int)kRowMask)];
        for (int t0 = 0; t0 < n_cand; t0 += kWave) {
            const int t = t0 + lane;
            int key = 0;
            bool acc = false;
            if (scan_all) {
                // candidate t: element t / n, row ba0 + t % n (passes per element keep the order)
                const int e = t / bi.n, j = bi.ba0 + (t - e * bi.n);
                if (t < n_cand && j != i) {
                    const float4 pj = pos4[j];
                    acc = __float_as_int(pj.w) == e && within_cutoff(pi, pj, bi, rc2);
                    key = (e << kKeyShift) | j;
                }
            } else {
                const int c = c_next;
                const float4 pj = p_next;
                c_next = c_after;
                c_after = t + 2 * kWave < n_list ? cand[t + 2 * kWave] : 0;
                p_next = pos4[bi.ba0 + (c_next & (int)kRowMask)];
                if (t < n_cand) {
                    const int j = bi.ba0 + (c & (int)kRowMask);
                    acc = within_cutoff(pi, pj, bi, rc2);
                    key = (c & ~(int)kRowMask) | j;
                }
            }
            const uint64_t m = __ballot(acc);
            const int pos = count + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            const bool keep = acc && pos < Kmax;
            if (keep) {
                out[pos] = key;
                if ((pos & 15) == 0 && pos > 0 && (pos >> 4) < kFence)
                    fence[(int64_t)i * kFence + (pos >> 4)] = key;
            }
#pragma unroll
            for (int e = 0; e < kMaxElements; ++e)
                grp[e] += __popcll(__ballot(keep && (key >> kKeyShift) == e));
            count += __popcll(m);
        }
        if (count > Kmax && lane == 0)
            atomicOr(status, kStatusOverflow);
        const int K = count < Kmax ? count : Kmax;
        if (lane < n_el) {
            int c = grp[0];
#pragma unroll
            for (int e = 1; e < kMaxElements; ++e)
                c = lane == e ? grp[e] : c;
            nbr_grp[(int64_t)i * kMaxElements + lane] = c;
        }
        if (lane == 0)
            nbr_cnt[i] = K;
        if (lane < kFence && (lane == 0 || 16 * lane >= K))
            fence[(int64_t)i * kFence + lane] = lane == 0 ? K : 0x7FFFFFFF;
    }
}

void launch_skin_neighbors(const float *q, const DevBuffers &d, const Sizes &z, const SkinParams &sp, float rc2,
                           int n_el, const Tuning &tn, hipStream_t s)
{
    hipLaunchKernelGGL(k_wrap_skin, dim3((z.B + 255) / 256), dim3(256), 0, s, q, d.beads, d.bead_of_ba,
                       d.species_atom, d.sys, d.skin_c0, sp.half_skin2, d.pos4, d.posu4, d.skin_flag, z.B);
    hipLaunchKernelGGL(k_skin_centroids, dim3((z.n_atoms_total + 255) / 256), dim3(256), 0, s, d.posu4, d.sys,
                       d.sys_of_atom, sp.half_skin2, d.skin_flag, d.skin_c0, z.n_atoms_total);
    hipLaunchKernelGGL(k_skin_lists, dim3((z.n_atoms_total + 3) / 4), dim3(256), 0, s, d.skin_c0, d.sys,
                       d.sys_of_atom, d.species_atom, d.beads, d.bead_of_ba, sp.reach2, n_el, sp.Kc, d.skin_flag,
                       d.skin_keys, d.skin_cnt, d.skin_builds, d.status, z.n_atoms_total);
    hipLaunchKernelGGL(k_skin_filter, dim3(centre_grid(z.B, tn)), dim3(kWave * tn.centre_waves), 0, s, d.pos4,
                       d.beads, d.bead_of_ba, d.sys, d.skin_keys, d.skin_cnt, sp.Kc, rc2, z.Kmax, n_el, d.skin_flag,
                       d.skin_builds + 1, d.nbr, d.nbr_cnt, d.nbr_grp, d.nbr_fence, d.status, z.B);
}

// Candidates staged per cell: up to kMaxCand stencil atoms (27 cells of ~30).
constexpr int kMaxCand = 1536;

size_t neighbors_cells_lds(int Kmax) { return (size_t)4 * nl_buffer(Kmax) * 4 + (size_t)kMaxCand * 20; }

hipError_t configure_neighbor_lds(int Kmax)
{
    return hipFuncSetAttribute((const void *)k_neighbors_cells, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)neighbors_cells_lds(Kmax));
}

void launch_neighbors(const DevBuffers &d, const Sizes &z, float rc2, int n_el, const Tuning &tn, hipStream_t s)
{
    const bool cells = z.any_periodic && tn.nl_cells;
    if (cells)
        hipLaunchKernelGGL(k_neighbors_cells, dim3(z.total_cells), dim3(256), neighbors_cells_lds(z.Kmax), s, d.pos4,
                           d.beads, d.cell_bead, d.cell_count, d.cell_start, d.cell_atoms, rc2, z.Kmax, n_el, kMaxCand,
                           d.nbr, d.nbr_cnt, d.nbr_grp, d.nbr_fence, d.status);
    if (!cells || z.any_open) {
        const int wpg = tn.centre_waves;
        const size_t lds = (size_t)wpg * nl_buffer(z.Kmax) * sizeof(int32_t);
        hipLaunchKernelGGL(k_neighbors, dim3(centre_grid(z.B, tn)), dim3(kWave * wpg), lds, s, d.pos4, d.beads,
                           d.bead_of_ba, d.cell_count, d.cell_start, d.cell_atoms, centre_order(d, z), rc2, z.Kmax,
                           n_el, cells ? 1 : 0, d.nbr, d.nbr_cnt, d.nbr_grp, d.nbr_fence, d.status, z.B);
    }
}

}  // namespace pimd
