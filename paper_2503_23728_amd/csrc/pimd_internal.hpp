// Internal types shared by the host runtime (pimd_api.cpp) and the HIP
// kernels.  Plain structs only; no STL in device-visible declarations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pimd {

constexpr int kWave = 64;
constexpr int kMaxElements = 4;
constexpr int kSmAtoms = 16;                   // lane-per-centre kernels: atoms per molecule, at most
constexpr int kMaxRad = 32;
constexpr int kMaxPairs = kMaxElements * (kMaxElements + 1) / 2;   // element-pair blocks
// slot pairs kept per centre by the descriptor forward for the adjoint: every
// unordered pair of Kmax slots (16 bits each: the two slot indices)
// Kept slot pairs per centre: all K(K-1)/2 pairs, and 256 entries that the
// adjoint's look-ahead loads may read past a block's last pair.
__host__ __device__ inline int64_t tri_capacity(int Kmax) { return (int64_t)Kmax * (Kmax - 1) / 2 + 256; }
constexpr int kG5Mom = 84;       // floats per (centre, element, eta) of the G5 moments: 81 and 3 of padding
constexpr int kMaxBeads = 128;
constexpr int kMaxNeighbors = 256;
constexpr int kKeyShift = 27;                 // neighbour key = (element << 27) | row
constexpr int kFence = 16;                    // fence row per list: count, then the keys at slots 16, 32, ...
constexpr uint32_t kRowMask = (1u << kKeyShift) - 1u;

// device status word bits
constexpr uint32_t kStatusOverflow = 1u;
constexpr uint32_t kStatusNonFinite = 2u;

// physical constants (CODATA 2018), library side
constexpr double kKB = 8.617333262e-5;        // eV / K
constexpr double kHbar = 0.6582119569;        // eV fs
constexpr double kMvv2e = 103.64269652680505; // eV per amu A^2 / fs^2

// One entry per global bead.
struct BeadInfo {
    int32_t sys;        // system index
    int32_t ba0;        // first row of the bead in the state layout
    int32_t n;          // atoms in the bead
    int32_t periodic;   // 1 if the system has a box
    float L[3];         // box lengths
    float invL[3];      // fl32(1 / L)
    float cell_scale[3];// cells per unit length (nc / L)
    int32_t nc[3];      // cells per axis
    int32_t cell0;      // first cell of this bead in the cell arrays
    int32_t pad;
    double L64[3];      // box lengths in FP64 (displacements of the descriptor kernels)
    double invL64[3];
};

// Descriptor grid and cutoff, passed by value to the descriptor kernels.
struct DescParams {
    int32_t n_el, n_rad, n_ang_eta, n_ang, D, Kmax;
    float rc, rc2, pi_over_rc, half_over_rc;  // half_over_rc = 1/(2 rc): cos(pi r/rc) = cos(2 pi (r half_over_rc))
    float rad_center[kMaxRad];     // R_s rounded to float ...
    float rad_center_lo[kMaxRad];  // ... and the remainder R_s - float(R_s)
    float rad_eta[kMaxRad];
    // per radial function, as the slot derivatives use it: R_s, its remainder,
    // the exponent factor -eta log2(e) (float product) and -2 eta; one
    // 16-byte scalar load per function
    float4 rad_pack[kMaxRad];
    float ang_eta[2];
    int32_t eta_pow4;              // 1: ang_eta[1] == 4 ang_eta[0] exactly, so exp(-eta_1 x) = exp(-eta_0 x)^4
    int32_t angular;               // 0: G4 angular functions, 1: G5
    float g5_leg[4][9];            // G5: 2^(1-zeta) a_l of (1 + c)^zeta = sum_l a_l P_l(c), zeta = 1, 2, 4, 8
};

// One layer of one element network on the device.
struct MlpLayer {
    const float *W;        // [out][in_pad]   forward B operand (B[k][n] = W[n][k])
    const float *WT;       // [in_pad][out]   backward B operand
    const uint16_t *Wb;    // bfloat16 copies of the two (nearest-even rounding) ...
    const uint16_t *WTb;
    const uint16_t *Wb_lo; // ... and of the rounding remainders W - bf16(W)
    const uint16_t *WTb_lo;
    const uint16_t *Wc, *Wc_lo;   // fragments of W and W^T for the register-chained BF16 kernel
    const uint16_t *WTc, *WTc_lo; // (hi and lo parts; null when the model exceeds its limits)
    const double *W64;     // FP64 copies of W and WT
    const double *WT64;
    const float *b;        // [out]
    int32_t in_pad, out;
};

struct MlpNet {
    MlpLayer layer[3];
    int32_t n_hidden;
    const float *wo;       // [out of last hidden]
    float bo;
    const float *inv_scale;// [D] 1 / feat_scale
    const float *shift;    // [D] feat_shift (used by the descriptor kernel)
};

struct MlpNets {
    MlpNet net[kMaxElements];
};

// Tile of up to 16, 32 or 64 rows of one element for the MLP kernel.
struct MlpTile {
    int32_t e, row0, nrows, pad;
};

// Integrator work unit: `ncol` columns (atom, xyz) of one system, P threads each.
// Work unit of the lane-per-centre kernels: whole beads of small molecules,
// rows row0 .. row0 + nrows - 1 (nrows <= 64), nmax atoms in the largest bead.
struct SmUnit {
    int32_t row0, nrows, nmax, pad;
};

struct IntegUnit {
    int32_t sys;
    int32_t col0;
    int32_t ncol;
    int32_t pad;
};

struct SysInfo {
    int32_t N, P, ba0, atom0;   // atoms, beads, first row, first atom (in species order)
    int32_t mode0;              // first entry of this system in the mode table
    int32_t cmat0;              // offset of this P's normal-mode twiddle table
    int32_t unit0, nunit;       // integrator units of this system
    float sig_T;                // sqrt(k_B T P / MVV2E): thermal momentum per sqrt(amu)
    float pad[3];
};

// Coefficients in FP64: a rotation whose float32 cos and sin miss
// cos^2 + sin^2 = 1 by ~1e-7 changes every mode's energy by that factor each
// step, a drift per step that does not shrink with dt.
struct ModeInfo {
    double c1, c2;      // O step: exp(-gamma dt/2), sqrt(1 - c1^2)
    double cw, sw;      // cos(w dt), sin(w dt)
    double w;           // mode frequency (1/fs)
    double mfac;        // kinetic mass / physical mass: 1 (normal modes, beads); staging: P, P l/(l-1) for l >= 2
    double pad[2];
};

// Direct-force head: one small MLP y = W2 tanh(W1 x + b1) + b2 and the whole head
// (pointers into the packed float32 weights in device memory).
struct GfnMlp {
    const float *W1, *b1, *W2, *b2;
};

struct GfnParams {
    const float *node_embed;   // [n_el][H]
    const float *pair_embed;   // [n_el][n_el][H]
    const float *edge_in;      // [H][n_rad]
    GfnMlp msg[3], node[3], edge[3];
    const float *fW1, *fb1, *fw2;
    float fb2;
    int32_t H, L;
    // MFMA path: 0 off (float32 vector ALU), 1 BF16 operands split hi + lo
    // (three products), 2 BF16 operands rounded once; bfloat16 weight tiles in
    // A-operand order (16 x 16 blocks, 64 lanes x (4 hi, 4 lo) each)
    int32_t mode;
    const uint16_t *t_in;                       // edge_in [H][n_rad]
    const uint16_t *t_msg1[3], *t_msg2[3];      // phi_msg W1, W2 per layer
    const uint16_t *t_edge1[3], *t_edge2[3];    // phi_edge W1, W2 per layer
    const uint16_t *t_f1;                       // readout W1
};

// Well-tempered metadynamics on bead CVs, passed by value to its kernels.
constexpr int kMaxCvTerms = 64;
constexpr uint32_t kStatusHills = 4u;        // a deposition found the hill store full

struct MetadParams {
    int32_t cv;              // 1 distances, 2 XRD
    int32_t n_terms;
    int32_t stride, max_hills;
    int32_t xrd_tile;        // rows per tile of the XRD pair sum: 64 or 256
    int32_t pad;
    double q_scatter;        // Q (1/A)
    double sigma, inv_sigma, height0;
    double form_factor[kMaxElements];
};

// Everything a step needs on the device, carved from the workspace.
struct DevBuffers {
    float *q, *p, *F, *E_bead;     // integrator state, forces of q, bead energies
    float *q_prev, *p_prev;        // the state at the start of the step in progress (restored on a fault)
    float *xi;                     // injected noise [2][B][3]
    float4 *pos4;                  // wrapped positions + species bits (neighbour search)
    float4 *posu4;                 // unwrapped positions + species bits (displacements)
    int32_t *atom_cell, *atom_slot;
    int32_t *cell_count, *cell_start, *cell_atoms;
    int32_t *cell_bead;            // bead of every cell (periodic beads)
    int32_t *nbr, *nbr_cnt, *nbr_grp;
    int32_t *nbr_fence;            // [B][kFence]: list count, then every 16th key (reverse-slot search)
    float *xhat, *dEdG, *E_atom;
    float *g5_mom;           // G5: per centre [element][eta][kG5Mom] moments, kept for the adjoint
    uint16_t *tri_pairs;     // G4: per centre the in-range slot pairs (j << 8 | k) found by the forward
    int32_t *tri_cnt;        // G4: per centre [kMaxPairs] pairs per element-pair block
    // shared neighbour lists with a skin (neighbor_skin_A > 0)
    int32_t *skin_keys;      // [atoms][Kc] (element << 27) | atom within its system, sorted
    int32_t *skin_cnt;       // [atoms]
    double4 *skin_c0;        // [atoms] centroid at the last build
    int32_t *skin_flag;      // [0] rebuild before this step's filter, [1] the step's lists cannot be trusted
    unsigned long long *skin_builds;   // [0] builds, [1] evaluations that scanned every atom of the bead
    int32_t *sys_of_atom;    // [atoms]
    float4 *vslot;                 // [B][Kmax] v[i][n] = dE/d d_(i, slot n)
    float4 *vrev;                  // [B][Kmax] v[j][slot of i in j's list], at i's slot n of j
    float *vir_atom, *W_bead;
    double *heat, *dke_part;       // heat bath per system; O-step energy changes per unit (2 halves)
    double *svr_part;              // PILE-G: per unit (centroid kinetic energy, sum of centroid normals^2)
    double *svr_alpha;             // PILE-G: per system factor of the centroid momenta (null: PILE-L)
    double *svr_kbar;              // PILE-G: per system N_f k_B T P / 2
    SmUnit *sm_units;              // lane-per-centre kernels: whole beads per wave
    int64_t *step;
    uint32_t *status;
    float *est_cols;               // estimator terms per column [ncol][3]
    // tables
    BeadInfo *beads;
    int32_t *bead_of_ba;
    int32_t *species_atom;         // [sum N]
    int32_t *elem_rows;            // rows grouped by element (MLP gather)
    MlpTile *mlp_tiles;            // row tiles over all elements
    float *mass_atom;              // [sum N]
    SysInfo *sys;
    ModeInfo *modes;
    IntegUnit *units;
    double *cmat;                  // normal modes per distinct P: cos, sin twiddles [P] each, 1/sqrt(P), sqrt(2/P)
    int32_t *col_sys;              // [ncol] system of each column
    float *mlp_f32;                // packed f32 weights (W, WT, b, wo per element)
    uint16_t *mlp_bf16;            // packed bf16 weights (W, WT per element)
    uint16_t *mlp_chain;           // MFMA fragments of W and W^T for the register-chained MLP (or null)
    double *mlp_f64;               // packed f64 weights (W, WT per element)
    float *norm;                   // [n_el][2][D] shift, 1/scale
    float *gfn_params;             // direct-force head: packed weights
    float *gfn_nodes;              // direct-force head: node states n^(0..L) [L+1][B][H]
    uint16_t *gfn_tiles;           // direct-force head: bfloat16 weight tiles of the MFMA path
    // metadynamics
    double2 *hills;                // [beads][max_hills] (center, height)
    int32_t *n_hills;              // hills deposited per bead (one counter: all beads deposit together)
    double *cv_bead, *vbias_bead;  // CV and bias energy of every bead at the last force evaluation
    double *cv_eval, *vbias_eval;  // the same for pimd_bias_forces
    double *xrd_row;               // [B] f_i sum_j f_j sinc(Q R_ij)
    float *xrd_grad;               // [B][3] dS/dq_i
    int4 *xrd_items;               // (bead, tile I, tile J >= I, first partial of the bead) of the pair sum
    int32_t *xrd_part0;            // [beads] first partial of every bead
    double4 *xrd_part;             // per bead [partner tile][row] (sum_j f_j sinc, gradient sum)
    int32_t *cv_atoms;             // [n_terms][2]
    double *cv_coef;               // [n_terms]
    double *wt_scale;              // [n_sys] 1 / (k_B T (gamma - 1)), 0 for gamma = infinity
};

// Launch shapes chosen by the tuner (results do not depend on them: every
// centre atom is still one wave, every MLP row the same MFMA chain).
struct Tuning {
    int32_t centre_waves;  // waves (centre atoms in flight) per workgroup of the per-centre kernels: 1, 2 or 4
    int32_t centre_grid;   // 0: one wave per centre; > 0: at most this many workgroups, waves stride over centres
    int32_t mlp_rows;      // rows per MLP workgroup tile: 16, 32 or 64
    int32_t nl_cells;      // periodic neighbour search per cell with the stencil in LDS (1) or per centre (0)
    int32_t mlp_waves;     // waves per BF16 MLP workgroup: 4 (two column tiles each) or 8 (one each)
    int32_t force_rows;    // 1: the adjoint also stores each slot value at the neighbour's reverse slot and the
                           // force assembly reads rows; 0: the assembly gathers through the reverse-slot search
    int32_t centre_lanes;  // 1: small molecules, one lane per centre (whole beads per wave); 0: one wave per centre
    int32_t mlp_chain;     // BF16 MLP: 1 activations kept in registers between layers (a wave per 16 rows),
                           // 0 activations staged in LDS (mlp_waves waves split the output columns)
};

// Workgroups of a per-centre launch over B centres.
inline int centre_grid(int B, const Tuning &tn)
{
    const int full = (B + tn.centre_waves - 1) / tn.centre_waves;
    return tn.centre_grid > 0 && tn.centre_grid < full ? tn.centre_grid : (full > 0 ? full : 1);
}

// ---------------------------------------------------------------- launchers
struct Sizes {
    int32_t n_sys, B, n_beads_total, n_atoms_total, ncol, total_cells, n_units, D, Kmax;
    int32_t any_periodic;   // some system has a box (cell lists)
    int32_t any_open;       // some system has none (all-pairs lists)
    int32_t any_box;        // some system has a box (minimum image of the metadynamics CVs)
    int32_t skin;           // shared centroid lists with a skin instead of per-bead cell lists
    int32_t max_bead_atoms; // atoms of the largest bead
};

struct SkinParams {
    double half_skin2;      // (skin / 2)^2: a bead-atom farther from its build centroid forces a rebuild
    double reach2;          // (cutoff + skin + 1e-3 A)^2 of the centroid lists
    int32_t Kc;             // slots per centroid list
};

// Order in which the per-centre kernels visit the rows: cell order within
// every bead (written by the cell fill) when any system has a box, else the
// row order itself (null).
inline const int32_t *centre_order(const DevBuffers &d, const Sizes &z)
{
    return z.any_periodic && !z.skin ? d.cell_atoms : nullptr;
}

void launch_zero_i32(int32_t *p, int64_t n, hipStream_t s);
void launch_wrap_bin(const float *q, const DevBuffers &d, const Sizes &z, hipStream_t s);
void launch_cell_scan(const DevBuffers &d, const Sizes &z, hipStream_t s);
void launch_cell_fill(const DevBuffers &d, const Sizes &z, hipStream_t s);
void launch_neighbors(const DevBuffers &d, const Sizes &z, float rc2, int n_el, const Tuning &tn, hipStream_t s);
void launch_descriptors(const DevBuffers &d, const Sizes &z, const DescParams &dp, const Tuning &tn, hipStream_t s);
// mlp_mode: 0 FP32 operands; 1 BF16 operands, three-term split; 2 BF16 operands, one term; 3 FP64;
// 4 BF16 split activations on bfloat16-valued weights
// rows: rows per tile of d.mlp_tiles (16, 32 or 64; mode 3 takes 16 only); waves: 4 or 8 (BF16 modes);
// chain: the register-chained kernel (modes 1, 2, 4; the nets' chain fragments must exist)
void launch_mlp(const DevBuffers &d, const MlpNets &nets, int n_tiles, int D, int Dp, int mlp_mode, int rows,
                int waves, bool chain, hipStream_t s);
// The register-chained kernel exists for this network shape (features, hidden widths).
bool mlp_chain_shape(int D, int n_hidden, const int *hidden);
void launch_adjoint(const DevBuffers &d, const Sizes &z, const DescParams &dp, const Tuning &tn, hipStream_t s);
void launch_gfn_layers(const DevBuffers &d, const Sizes &z, const DescParams &dp, const GfnParams &gp,
                       const Tuning &tn, hipStream_t s);
void launch_gfn_forces(const DevBuffers &d, const Sizes &z, const DescParams &dp, const GfnParams &gp,
                       const Tuning &tn, float *F, hipStream_t s);
void launch_assemble_forces(const DevBuffers &d, const Sizes &z, float *F, const Tuning &tn, hipStream_t s);
void launch_bead_sums(const DevBuffers &d, const Sizes &z, float *E_bead, float *W_bead, bool virial,
                      hipStream_t s);
void launch_harmonic(const float *q, const DevBuffers &d, const Sizes &z, float k_over_m,
                     float *F, hipStream_t s);
// transform: 0 normal modes, 1 staging (momenta state = staging momenta),
// 2 primitive (Cartesian beads, springs as forces); with d.svr_alpha set
// (PILE-G, normal modes) the centroid's global factor is formed first, with
// svr_c = exp(-(dt/2)/tau0)
void launch_integrate_pre(const DevBuffers &d, const Sizes &z, float dt, uint32_t key0, uint32_t key1,
                          const float *xi, int max_P, int transform, double svr_c, hipStream_t s);
void launch_integrate_post(const DevBuffers &d, const Sizes &z, float dt, uint32_t key0, uint32_t key1,
                           const float *xi, int max_P, int transform, double svr_c, hipStream_t s);
void launch_finish_step(const DevBuffers &d, const Sizes &z, hipStream_t s);
void launch_estimator_terms(const DevBuffers &d, const Sizes &z, hipStream_t s);
void launch_philox_words(uint32_t key0, uint32_t key1, int64_t step, int half, int64_t n, uint32_t *out,
                         hipStream_t s);
void launch_check_finite(const float *a, int64_t n, uint32_t *status, hipStream_t s);

// Metadynamics: CV rows (XRD), then per bead the CV, bias, optional
// deposition (deposit != 0: when the step that is completing is a multiple of
// the stride) and the bias forces (add != 0: F += bias force, else F = bias force).
void launch_metad(const float *q, const DevBuffers &d, const Sizes &z, const MetadParams &mp, int n_xrd_items,
                  float *F, int add, int deposit, double *cv_out, double *v_out, hipStream_t s);
void launch_metad_advance(const DevBuffers &d, const MetadParams &mp, hipStream_t s);
void launch_metad_fes(const DevBuffers &d, const MetadParams &mp, int bead0, int P, double kT, double gamma_ratio,
                      const double *grid, int n_grid, double *out, hipStream_t s);

void launch_work_counts(const DevBuffers &d, const Sizes &z, const DescParams &dp,
                        unsigned long long *counts, hipStream_t s);

// Raise the dynamic-LDS limit of kernels whose LDS grows with Kmax or P.
hipError_t configure_descriptor_lds(const DescParams &dp);
// lane-per-centre kernels of small molecules (k_small.hip): descriptors with
// the neighbour lists, then adjoint with the force assembly (F may be null)
hipError_t configure_sm_lds(const DescParams &dp);
void launch_sm_forward(const DevBuffers &d, const DescParams &dp, int n_units, int nmax, hipStream_t s);
void launch_sm_adjoint(const DevBuffers &d, const DescParams &dp, int n_units, int nmax, float *F, hipStream_t s);
// neighbour stage with shared centroid lists: wrap and drift check, rebuild when
// flagged (centroids, lists), per-bead filter into nbr / nbr_cnt / nbr_grp / fence
void launch_skin_neighbors(const float *q, const DevBuffers &d, const Sizes &z, const SkinParams &sp, float rc2,
                           int n_el, const Tuning &tn, hipStream_t s);
// G5 angular functions (dp.angular = 1): forward (xhat, g5_mom) and adjoint (vslot, vir_atom)
hipError_t configure_g5_lds(const DescParams &dp);
void launch_descriptors_g5(const DevBuffers &d, const Sizes &z, const DescParams &dp, const Tuning &tn,
                           hipStream_t s);
void launch_adjoint_g5(const DevBuffers &d, const Sizes &z, const DescParams &dp, const Tuning &tn, hipStream_t s);
hipError_t configure_integrator_lds(int max_P);
hipError_t configure_neighbor_lds(int Kmax);
size_t descriptor_lds_bytes(const DescParams &dp, bool adjoint);
size_t integrator_lds_bytes(int max_P);

}  // namespace pimd
