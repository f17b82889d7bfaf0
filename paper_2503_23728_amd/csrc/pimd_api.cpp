// Host runtime behind the C ABI of include/pimd.h: argument validation (no
// HIP call before it passes), workspace planning, upload of tables and
// weights, the force pipeline, the integrator step and its captured graph,
// estimators and debug hooks.
#include "../../include/pimd.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pimd_internal.hpp"

using namespace pimd;

namespace {

thread_local std::string g_init_error;

const double kPi = 3.14159265358979323846;

struct Layout {
    size_t total = 0;
    std::map<std::string, size_t> off;
    void add(const std::string &name, size_t bytes)
    {
        total = (total + 255) & ~size_t(255);
        off[name] = total;
        total += bytes;
    }
};

// Everything derived from the config on the host.
struct Plan {
    int n_sys = 0, n_el = 0, B = 0, n_beads = 0, n_atoms = 0, ncol = 0, total_cells = 0, n_units = 0;
    int D = 0, Dp = 0, Kmax = 0, max_P = 1, n_rad = 0, n_ang_eta = 0;
    int angular = 0;                           // 0: G4, 1: G5 angular functions
    double skin = 0.0;                         // shared centroid lists: skin (0: per-bead cell lists)
    int Kc = 0;                                // slots per centroid list
    bool any_periodic = false, any_open = false, bpnn = false, gfn = false;
    bool nl = false;                           // neighbour lists (the energy model or the direct-force head)
    int gfn_H = 0, gfn_L = 0;
    size_t gfn_floats = 0;                     // packed weights of the direct-force head
    size_t gfn_tiles = 0;                      // bfloat16 16 x 16 weight tiles of its MFMA path
    std::vector<int> cells_per_sys;            // cells per bead of each system
    std::vector<std::array<int, 3>> nc;
    size_t mlp_f32_floats = 0, mlp_bf16_elems = 0, mlp_f64_elems = 0, cmat_elems = 0, modes = 0;
    bool chain = false;                        // register-chained BF16 MLP available (widths, D <= 128)
    size_t mlp_chain_elems = 0;                // its packed weight fragments (bfloat16, hi and lo)
    std::vector<int> distinct_P;
    bool any_box = false;                      // some system has a box (metadynamics minimum image)
    bool metad = false;                        // well-tempered metadynamics bias
    bool pile_g = false;                       // PILE-G: global thermostat on the centroids
    bool small = false;                        // small molecules: lane-per-centre kernels available
    int n_sm_units = 0;                        // their work units (whole beads, <= 64 rows each)
    int sm_nmax = 0;                           // atoms of the largest molecule
    int cv = 0, n_terms = 0, max_hills = 0;
    int xrd_tile = 64, n_xrd_items = 0;          // XRD pair sum: rows per tile, work items
    int64_t n_xrd_part = 0;                    // per-tile partials of the XRD pair sum
};

constexpr int kFesChunk = 4096;                // grid points per pimd_metad_fes launch

int n_features(int n_el, int n_rad, int n_ang_eta) { return n_el * n_rad + n_el * (n_el + 1) / 2 * n_ang_eta * 8; }

pimd_status fail(std::string *err, pimd_status s, const std::string &msg)
{
    if (err)
        *err = msg;
    return s;
}

// The fields every potential provides: elements, masses, cutoff and radial grid.
struct ModelView {
    int n_el = 0;
    const double *mass = nullptr;
    double cutoff = 0.0;
    int n_rad = 0;
    const double *rad_center = nullptr, *rad_eta = nullptr;
};

ModelView model_view(const pimd_config *cfg)
{
    ModelView v;
    if (cfg->potential == PIMD_POT_GFN) {
        const pimd_gfn_model *g = cfg->gfn;
        v = ModelView{g->n_elements, g->mass_amu, g->cutoff_A, g->n_rad, g->rad_center_A, g->rad_eta};
    } else {
        const pimd_bpnn_model *m = cfg->model;
        v = ModelView{m->n_elements, m->mass_amu, m->cutoff_A, m->n_rad, m->rad_center_A, m->rad_eta};
    }
    return v;
}

// All checks are on host data only.
pimd_status validate(const pimd_config *cfg, Plan &pl, std::string *err)
{
    if (!cfg)
        return fail(err, PIMD_E_ARG, "config is NULL");
    if (cfg->n_systems < 1)
        return fail(err, PIMD_E_ARG, "n_systems must be >= 1");
    if (!cfg->n_atoms || !cfg->n_beads || !cfg->temperature_K || !cfg->box_A || !cfg->species)
        return fail(err, PIMD_E_ARG, "a per-system array is NULL");
    if (!(cfg->dt_fs > 0.0) || !std::isfinite(cfg->dt_fs))
        return fail(err, PIMD_E_ARG, "dt_fs must be positive");
    if (!std::isfinite(cfg->tau0_fs))
        return fail(err, PIMD_E_ARG, "tau0_fs must be finite");
    if (!(cfg->pile_lambda >= 0.0) || !std::isfinite(cfg->pile_lambda))
        return fail(err, PIMD_E_ARG, "pile_lambda must be >= 0");
    if (cfg->precision != PIMD_PREC_FP32 && cfg->precision != PIMD_PREC_BF16_MLP &&
        cfg->precision != PIMD_PREC_BF16_PLAIN && cfg->precision != PIMD_PREC_FP64_MLP)
        return fail(err, PIMD_E_ARG, "unknown precision");
    if (cfg->potential != PIMD_POT_BPNN && cfg->potential != PIMD_POT_HARMONIC && cfg->potential != PIMD_POT_GFN)
        return fail(err, PIMD_E_ARG, "unknown potential");
    if (cfg->transform != PIMD_TRANSFORM_NORMAL_MODES && cfg->transform != PIMD_TRANSFORM_STAGING &&
        cfg->transform != PIMD_TRANSFORM_PRIMITIVE)
        return fail(err, PIMD_E_ARG, "unknown ring-polymer transform");
    if (cfg->thermostat != PIMD_THERMOSTAT_PILE_L && cfg->thermostat != PIMD_THERMOSTAT_PILE_G)
        return fail(err, PIMD_E_ARG, "unknown thermostat");
    if (cfg->thermostat == PIMD_THERMOSTAT_PILE_G && cfg->transform != PIMD_TRANSFORM_NORMAL_MODES)
        return fail(err, PIMD_E_UNSUPPORTED, "PILE-G needs the normal-mode integrator");
    pl.pile_g = cfg->thermostat == PIMD_THERMOSTAT_PILE_G;
    if (cfg->max_neighbors < 0 || cfg->max_neighbors > kMaxNeighbors)
        return fail(err, PIMD_E_UNSUPPORTED, "max_neighbors must be in [0, 256]");
    if (cfg->max_neighbors % 16)
        return fail(err, PIMD_E_ARG, "max_neighbors must be a multiple of 16");
    pl.bpnn = cfg->potential == PIMD_POT_BPNN;
    pl.gfn = cfg->potential == PIMD_POT_GFN;
    pl.nl = pl.bpnn || pl.gfn;
    const pimd_bpnn_model *m = cfg->model;
    const pimd_gfn_model *g = cfg->gfn;
    if (pl.gfn ? !g : !m)
        return fail(err, PIMD_E_ARG, "model is NULL (it carries the element masses)");
    const ModelView mv = model_view(cfg);
    if (mv.n_el < 1 || mv.n_el > kMaxElements)
        return fail(err, PIMD_E_UNSUPPORTED, "n_elements must be in [1, 4]");
    if (!mv.mass)
        return fail(err, PIMD_E_ARG, "mass_amu is NULL");
    for (int e = 0; e < mv.n_el; ++e)
        if (!(mv.mass[e] > 0.0) || !std::isfinite(mv.mass[e]))
            return fail(err, PIMD_E_ARG, "masses must be positive");
    pl.n_el = mv.n_el;
    if (pl.gfn) {
        if (!(g->cutoff_A > 0.0) || !std::isfinite(g->cutoff_A))
            return fail(err, PIMD_E_ARG, "cutoff must be positive");
        if (g->n_rad < 1 || g->n_rad > kMaxRad)
            return fail(err, PIMD_E_UNSUPPORTED, "n_rad must be in [1, 32]");
        if (g->width != 16 && g->width != 32)
            return fail(err, PIMD_E_UNSUPPORTED, "the head's width must be 16 or 32");
        if (g->n_layers < 1 || g->n_layers > 3)
            return fail(err, PIMD_E_UNSUPPORTED, "n_layers must be in [1, 3]");
        if (!g->rad_center_A || !g->rad_eta || !g->params)
            return fail(err, PIMD_E_ARG, "a model array is NULL");
        for (int s2 = 0; s2 < g->n_rad; ++s2)
            if (!std::isfinite(g->rad_center_A[s2]) || !(g->rad_eta[s2] >= 0.0))
                return fail(err, PIMD_E_ARG, "bad radial grid");
        pl.n_rad = g->n_rad;
        pl.gfn_H = g->width;
        pl.gfn_L = g->n_layers;
        const size_t H = g->width, ne = g->n_elements;
        {
            const size_t HB = H / 16, RB = (g->n_rad + 15) / 16;
            pl.gfn_tiles = HB * RB + (size_t)g->n_layers * 4 * HB * HB + HB * HB;
        }
        pl.gfn_floats = ne * H + ne * ne * H + H * g->n_rad +
                        (size_t)g->n_layers * ((H * H + 2 * H + H * H) + (2 * H * H + 2 * H + H * H) +
                                               (H * H + 2 * H + H * H)) +
                        H * H + 2 * H + 1;
    } else if (pl.bpnn) {
        if (!(m->cutoff_A > 0.0) || !std::isfinite(m->cutoff_A))
            return fail(err, PIMD_E_ARG, "cutoff must be positive");
        if (m->n_rad < 1 || m->n_rad > kMaxRad || m->n_elements * m->n_rad > 64)
            return fail(err, PIMD_E_UNSUPPORTED, "n_rad must be in [1, 32] with n_elements*n_rad <= 64");
        if (m->n_ang_eta < 1 || m->n_ang_eta > 2)
            return fail(err, PIMD_E_UNSUPPORTED, "n_ang_eta must be 1 or 2");
        if (!m->rad_center_A || !m->rad_eta || !m->ang_eta || !m->params || !m->feat_shift || !m->feat_scale)
            return fail(err, PIMD_E_ARG, "a model array is NULL");
        for (int s = 0; s < m->n_rad; ++s)
            if (!std::isfinite(m->rad_center_A[s]) || !(m->rad_eta[s] >= 0.0))
                return fail(err, PIMD_E_ARG, "bad radial grid");
        for (int s = 0; s < m->n_ang_eta; ++s)
            if (!(m->ang_eta[s] >= 0.0) || !std::isfinite(m->ang_eta[s]))
                return fail(err, PIMD_E_ARG, "bad angular eta");
        if (m->angular != PIMD_ANGULAR_G4 && m->angular != PIMD_ANGULAR_G5)
            return fail(err, PIMD_E_ARG, "angular must be PIMD_ANGULAR_G4 or PIMD_ANGULAR_G5");
        if (m->n_hidden < 1 || m->n_hidden > 3)
            return fail(err, PIMD_E_UNSUPPORTED, "n_hidden must be in [1, 3]");
        for (int l = 0; l < m->n_hidden; ++l)
            if (m->hidden[l] < 16 || m->hidden[l] > 128 || m->hidden[l] % 16)
                return fail(err, PIMD_E_UNSUPPORTED, "hidden widths must be multiples of 16 in [16, 128]");
        pl.n_rad = m->n_rad;
        pl.n_ang_eta = m->n_ang_eta;
        pl.angular = m->angular;
        pl.D = n_features(m->n_elements, m->n_rad, m->n_ang_eta);
        pl.Dp = (pl.D + 15) & ~15;
        if (pl.Dp > 128)
            return fail(err, PIMD_E_UNSUPPORTED, "descriptor length above 128");
        for (int e = 0; e < m->n_elements; ++e)
            for (int f = 0; f < pl.D; ++f)
                if (!(m->feat_scale[(size_t)e * pl.D + f] != 0.0f) || !std::isfinite(m->feat_scale[(size_t)e * pl.D + f]))
                    return fail(err, PIMD_E_ARG, "feat_scale must be finite and non-zero");
    } else {
        if (!(cfg->harmonic_omega_per_fs > 0.0) || !std::isfinite(cfg->harmonic_omega_per_fs))
            return fail(err, PIMD_E_ARG, "harmonic_omega_per_fs must be positive");
    }
    pl.n_sys = cfg->n_systems;
    pl.Kmax = cfg->max_neighbors == 0 ? 128 : cfg->max_neighbors;
    if (!(cfg->neighbor_skin_A >= 0.0) || !std::isfinite(cfg->neighbor_skin_A))
        return fail(err, PIMD_E_ARG, "neighbor_skin_A must be >= 0");
    if (cfg->neighbor_skin_A > 0.0) {
        if (!pl.nl)
            return fail(err, PIMD_E_UNSUPPORTED, "neighbor_skin_A needs a neural potential");
        pl.skin = cfg->neighbor_skin_A;
        pl.Kc = 3 * pl.Kmax;
    }
    int64_t B = 0, nb = 0, na = 0, cells = 0;
    for (int s = 0; s < cfg->n_systems; ++s) {
        const int N = cfg->n_atoms[s], P = cfg->n_beads[s];
        if (N < 1)
            return fail(err, PIMD_E_ARG, "n_atoms must be >= 1");
        if (P < 1)
            return fail(err, PIMD_E_ARG, "n_beads must be >= 1");
        if (P > kMaxBeads || (P > 1 && (P & 1)))
            return fail(err, PIMD_E_UNSUPPORTED, "n_beads must be 1 or even and <= 128");
        if (!(cfg->temperature_K[s] > 0.0) || !std::isfinite(cfg->temperature_K[s]))
            return fail(err, PIMD_E_ARG, "temperature must be positive");
        const double *L = cfg->box_A + 3 * s;
        const bool zero = L[0] == 0.0 && L[1] == 0.0 && L[2] == 0.0;
        std::array<int, 3> nc = {0, 0, 0};
        if (!zero) {
            for (int d = 0; d < 3; ++d)
                if (!(L[d] > 0.0) || !std::isfinite(L[d]))
                    return fail(err, PIMD_E_ARG, "box lengths must be all positive or all zero");
            if (pl.nl) {
                for (int d = 0; d < 3; ++d)
                    if (!(mv.cutoff < 0.5 * L[d]))
                        return fail(err, PIMD_E_UNSUPPORTED, "cutoff must be below half of every box length");
                for (int d = 0; d < 3; ++d)
                    nc[d] = std::max(1, (int)std::floor(L[d] / (mv.cutoff + 1e-4)));
                pl.any_periodic = true;
            }
            pl.any_box = true;
        } else {
            pl.any_open = true;
            if (pl.skin > 0.0)
                return fail(err, PIMD_E_UNSUPPORTED, "neighbor_skin_A needs a box for every system");
        }
        pl.nc.push_back(nc);
        const int per_bead = zero || !pl.nl ? 0 : nc[0] * nc[1] * nc[2];
        pl.cells_per_sys.push_back(per_bead);
        cells += (int64_t)per_bead * P;
        B += (int64_t)N * P;
        nb += P;
        na += N;
        pl.max_P = std::max(pl.max_P, P);
        if (std::find(pl.distinct_P.begin(), pl.distinct_P.end(), P) == pl.distinct_P.end())
            pl.distinct_P.push_back(P);
        const int cols_per_unit = std::max(1, 256 / P);
        pl.n_units += (3 * N + cols_per_unit - 1) / cols_per_unit;
        pl.modes += P;
    }
    if (B >= (int64_t)kRowMask || cells > (int64_t)1 << 30)
        return fail(err, PIMD_E_UNSUPPORTED, "too many bead-atoms (limit 2^27)");
    // lane-per-centre kernels: the G4 network on molecules without a box of at
    // most kSmAtoms atoms; units of whole beads, as many as fit in 64 rows
    pl.small = pl.bpnn && !pl.angular && !pl.any_periodic && pl.skin == 0.0;
    for (int s = 0; s < cfg->n_systems && pl.small; ++s) {
        pl.small = cfg->n_atoms[s] <= kSmAtoms;
        pl.sm_nmax = std::max(pl.sm_nmax, cfg->n_atoms[s]);
    }
    if (pl.small) {
        int rows = kWave;
        for (int s = 0; s < cfg->n_systems; ++s)
            for (int k = 0; k < cfg->n_beads[s]; ++k) {
                if (rows + cfg->n_atoms[s] > kWave) {
                    ++pl.n_sm_units;
                    rows = 0;
                }
                rows += cfg->n_atoms[s];
            }
    }
    for (int64_t a = 0; a < na; ++a)
        if (cfg->species[a] < 0 || cfg->species[a] >= mv.n_el)
            return fail(err, PIMD_E_ARG, "species index out of range");
    pl.B = (int)B;
    pl.n_beads = (int)nb;
    pl.n_atoms = (int)na;
    pl.ncol = 3 * (int)na;
    pl.total_cells = (int)cells;
    for (int P : pl.distinct_P)
        pl.cmat_elems += 2 * (size_t)P + 2;
    if (pl.bpnn) {
        int in = pl.Dp;
        pl.chain = mlp_chain_shape(pl.D, m->n_hidden, m->hidden);
        for (int e = 0; e < pl.n_el; ++e) {
            in = pl.Dp;
            int in_c = pl.D;
            for (int l = 0; l < m->n_hidden; ++l) {
                const int out = m->hidden[l];
                pl.mlp_f32_floats += 2 * (size_t)out * in + out;
                pl.mlp_bf16_elems += 4 * (size_t)out * in;
                pl.mlp_f64_elems += 2 * (size_t)out * in;
                if (pl.chain)   // W: out/16 tiles x ceil(in/32) steps; W^T: 2 ceil(in/32) tiles x ceil(out/32) steps
                    pl.mlp_chain_elems += 2 * (size_t)kWave * 8 *
                                          ((size_t)(out / 16) * ((in_c + 31) / 32) + (size_t)(2 * ((in_c + 31) / 32)) * ((out + 31) / 32));
                in = out;
                in_c = out;
            }
            pl.mlp_f32_floats += in;
        }
    }
    if (cfg->metad) {
        const pimd_metad *md = cfg->metad;
        if (md->cv != PIMD_CV_DISTANCES && md->cv != PIMD_CV_XRD)
            return fail(err, PIMD_E_ARG, "unknown collective variable");
        if (!(md->sigma > 0.0) || !std::isfinite(md->sigma))
            return fail(err, PIMD_E_ARG, "metadynamics sigma must be positive");
        if (!(md->height0_eV >= 0.0) || !std::isfinite(md->height0_eV))
            return fail(err, PIMD_E_ARG, "metadynamics height0 must be >= 0");
        if (!(md->bias_factor > 1.0))
            return fail(err, PIMD_E_ARG, "metadynamics bias_factor must be > 1");
        if (md->stride < 1)
            return fail(err, PIMD_E_ARG, "metadynamics stride must be >= 1");
        if (md->max_hills < 1 || (int64_t)md->max_hills * pl.n_beads > ((int64_t)1 << 31))
            return fail(err, PIMD_E_ARG, "max_hills must be >= 1 (and max_hills * beads below 2^31)");
        int min_n = cfg->n_atoms[0];
        for (int s = 1; s < cfg->n_systems; ++s)
            min_n = std::min(min_n, cfg->n_atoms[s]);
        if (md->cv == PIMD_CV_DISTANCES) {
            if (md->n_terms < 1 || md->n_terms > kMaxCvTerms)
                return fail(err, PIMD_E_ARG, "n_terms must be in [1, 64]");
            if (!md->atoms || !md->coef)
                return fail(err, PIMD_E_ARG, "CV atoms or coef is NULL");
            for (int t = 0; t < md->n_terms; ++t) {
                const int a = md->atoms[2 * t], b = md->atoms[2 * t + 1];
                if (a < 0 || b < 0 || a >= min_n || b >= min_n || a == b)
                    return fail(err, PIMD_E_ARG, "CV atom index out of range (or a term pairs an atom with itself)");
                if (!std::isfinite(md->coef[t]))
                    return fail(err, PIMD_E_ARG, "CV coefficients must be finite");
            }
        } else {
            if (!(md->q_scatter > 0.0) || !std::isfinite(md->q_scatter))
                return fail(err, PIMD_E_ARG, "q_scatter must be positive");
            if (!md->form_factor)
                return fail(err, PIMD_E_ARG, "form_factor is NULL");
            for (int e = 0; e < pl.n_el; ++e)
                if (!std::isfinite(md->form_factor[e]))
                    return fail(err, PIMD_E_ARG, "form factors must be finite");
            int max_n = 0;
            for (int s = 0; s < cfg->n_systems; ++s)
                max_n = std::max(max_n, cfg->n_atoms[s]);
            pl.xrd_tile = max_n > 1024 ? 256 : 64;
            for (int s = 0; s < cfg->n_systems; ++s) {
                const int64_t nt = (cfg->n_atoms[s] + pl.xrd_tile - 1) / pl.xrd_tile;
                pl.n_xrd_items += (int)(cfg->n_beads[s] * nt * (nt + 1) / 2);
                pl.n_xrd_part += (int64_t)cfg->n_beads[s] * nt * cfg->n_atoms[s];
            }
            if (pl.n_xrd_part >= ((int64_t)1 << 31))
                return fail(err, PIMD_E_UNSUPPORTED, "XRD pair sum too large (per-tile partials above 2^31)");
        }
        pl.metad = true;
        pl.cv = md->cv;
        pl.n_terms = md->cv == PIMD_CV_DISTANCES ? md->n_terms : 0;
        pl.max_hills = md->max_hills;
    }
    return PIMD_OK;
}

Layout make_layout(const Plan &pl)
{
    Layout L;
    const size_t B = pl.B, nb = pl.n_beads, K = pl.Kmax, D = pl.D;
    L.add("q", B * 12);
    L.add("p", B * 12);
    L.add("q_prev", B * 12);
    L.add("p_prev", B * 12);
    L.add("F", B * 12);
    L.add("E_bead", nb * 4);
    L.add("W_bead", nb * 36);
    L.add("xi", B * 24);
    L.add("pos4", B * 16);
    L.add("posu4", B * 16);
    L.add("E_atom", B * 4);
    L.add("vir_atom", B * 36);
    if (pl.nl) {
        L.add("atom_cell", B * 4);
        L.add("atom_slot", B * 4);
        L.add("cell_count", (size_t)pl.total_cells * 4);
        L.add("cell_start", (size_t)pl.total_cells * 4);
        L.add("cell_atoms", B * 4);
        L.add("cell_bead", (size_t)pl.total_cells * 4);
        L.add("nbr", B * K * 4);
        L.add("nbr_cnt", B * 4);
        L.add("nbr_grp", B * kMaxElements * 4);
        L.add("nbr_fence", B * kFence * 4);
    }
    if (pl.skin > 0.0) {
        L.add("skin_keys", (size_t)pl.n_atoms * pl.Kc * 4);
        L.add("skin_cnt", (size_t)pl.n_atoms * 4);
        L.add("skin_c0", (size_t)pl.n_atoms * 32);
        L.add("skin_flag", 8);
        L.add("skin_builds", 16);
        L.add("sys_of_atom", (size_t)pl.n_atoms * 4);
    }
    if (pl.gfn) {
        L.add("gfn_params", pl.gfn_floats * 4);
        L.add("gfn_nodes", (size_t)(pl.gfn_L + 1) * B * pl.gfn_H * 4);
        L.add("gfn_tiles", pl.gfn_tiles * kWave * 8 * 2);
    }
    if (pl.bpnn) {
        L.add("xhat", B * D * 4);
        L.add("dEdG", B * D * 4);
        L.add("vslot", B * K * 16);
        L.add("vrev", B * K * 16);
        if (pl.angular)
            L.add("g5_mom", B * (size_t)pl.n_el * pl.n_ang_eta * kG5Mom * 4);
        else {
            L.add("tri_pairs", B * (size_t)tri_capacity((int)K) * 2);
            L.add("tri_cnt", B * (size_t)kMaxPairs * 4);
        }
        L.add("mlp_f32", pl.mlp_f32_floats * 4);
        L.add("mlp_bf16", pl.mlp_bf16_elems * 2);
        L.add("mlp_f64", pl.mlp_f64_elems * 8);
        if (pl.chain)
            L.add("mlp_chain", pl.mlp_chain_elems * 2);
        L.add("norm", (size_t)pl.n_el * 2 * D * 4);
        L.add("elem_rows", B * 4);
        L.add("mlp_tiles", (B / 16 + kMaxElements + 1) * sizeof(MlpTile));
    }
    L.add("heat", (size_t)pl.n_sys * 8);
    L.add("dke_part", (size_t)pl.n_units * 16);
    if (pl.small)
        L.add("sm_units", (size_t)pl.n_sm_units * sizeof(SmUnit));
    if (pl.pile_g) {
        L.add("svr_part", (size_t)pl.n_units * 16);
        L.add("svr_alpha", (size_t)pl.n_sys * 8);
        L.add("svr_kbar", (size_t)pl.n_sys * 8);
    }
    L.add("step", 8);
    L.add("status", 8);
    L.add("est_cols", (size_t)pl.ncol * 12);
    L.add("beads", nb * sizeof(BeadInfo));
    L.add("bead_of_ba", B * 4);
    L.add("species_atom", (size_t)pl.n_atoms * 4);
    L.add("mass_atom", (size_t)pl.n_atoms * 4);
    L.add("sys", (size_t)pl.n_sys * sizeof(SysInfo));
    L.add("modes", pl.modes * sizeof(ModeInfo));
    L.add("units", (size_t)pl.n_units * sizeof(IntegUnit));
    L.add("cmat", pl.cmat_elems * 8);
    L.add("col_sys", (size_t)pl.ncol * 4);
    if (pl.metad) {
        L.add("hills", (size_t)nb * pl.max_hills * 16);
        L.add("n_hills", 8);
        L.add("cv_bead", nb * 8);
        L.add("vbias_bead", nb * 8);
        L.add("cv_eval", nb * 8);
        L.add("vbias_eval", nb * 8);
        L.add("wt_scale", (size_t)pl.n_sys * 8);
        L.add("fes_grid", (size_t)kFesChunk * 8);
        L.add("fes_out", (size_t)kFesChunk * 8);
        if (pl.cv == PIMD_CV_XRD) {
            L.add("xrd_row", B * 8);
            L.add("xrd_grad", B * 12);
            L.add("xrd_items", (size_t)pl.n_xrd_items * 16);
            L.add("xrd_part0", nb * 4);
            L.add("xrd_part", (size_t)pl.n_xrd_part * 32);
        } else {
            L.add("cv_atoms", (size_t)pl.n_terms * 8);
            L.add("cv_coef", (size_t)pl.n_terms * 8);
        }
    }
    L.add("end", 0);
    return L;
}

uint16_t bf16_bits(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Tiles of at most `rows` rows over the element-grouped MLP rows (an element's
// rows never share a tile).
std::vector<MlpTile> mlp_tiles(const std::vector<int32_t> &elem_row0, int rows)
{
    std::vector<MlpTile> tiles;
    for (int e = 0; e + 1 < (int)elem_row0.size(); ++e)
        for (int t = elem_row0[e]; t < elem_row0[e + 1]; t += rows)
            tiles.push_back(MlpTile{e, t, std::min(rows, elem_row0[e + 1] - t), 0});
    return tiles;
}

}  // namespace

struct pimd_ctx {
    Plan pl;
    Sizes z{};
    DevBuffers d{};
    DescParams dp{};
    GfnParams gp{};
    MlpNets nets{};
    int n_mlp_tiles = 0;
    std::vector<int32_t> elem_row0;   // [n_el + 1] first MLP row of each element in elem_rows
    Tuning tn{4, 0, 16, 0, 4};      // nl_cells is set from the cell count at init
    pimd_tuning last_tuning_out{};     // sink for pimd_autotune(best = NULL)
    std::vector<SysInfo> sys_host;
    std::vector<double> temperature, masses_el;
    std::vector<double> sys_host_box;   // [n_sys][3] box lengths (0: no box)
    std::vector<int> species;
    double dt = 0, tau0 = 0, lam = 0, omega = 0;
    uint64_t seed = 0;
    int precision = 0, potential = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool state_set = false, forces_valid = false, noise_pending = false, use_graph = true;
    bool atoms_of_state = false;       // E_atom and vir_atom hold the state's positions' values
    // stage timing: events recorded after each stage when non-null
    hipEvent_t *stage_ev = nullptr;
    // metadynamics: parameters, host mirrors of the step and hill counters
    // (the capacity check of pimd_step), deposition switch of the force pass
    MetadParams mp{};
    SkinParams skin{};                 // shared centroid lists (z.skin)
    double bias_factor = 0.0;
    double *fes_grid = nullptr, *fes_out = nullptr;
    int64_t host_step = 0;
    int host_hills = 0;
    bool deposit_now = false;
    int transform = PIMD_TRANSFORM_NORMAL_MODES;   // coordinates of the integrator
    int device = 0;
    int static_device = -1;            // device whose static workspace this context holds (pimd_init_static)
    double svr_c = 1.0;                // PILE-G: exp(-(dt/2)/tau0)
    bool mlp_weights_bf16 = false;     // every MLP weight is a bfloat16 value (split mode: two products a term)
    std::string err;
};

namespace {

#define HIPCHK(ctx, call)                                                                       \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) {                                                                 \
            (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_);                     \
            return PIMD_E_DEVICE;                                                               \
        }                                                                                       \
    } while (0)

#define CHECK_LAUNCH(ctx)                                                                       \
    do {                                                                                        \
        hipError_t e_ = hipGetLastError();                                                      \
        if (e_ != hipSuccess) {                                                                 \
            (ctx)->err = std::string("kernel launch: ") + hipGetErrorString(e_);                \
            return PIMD_E_DEVICE;                                                               \
        }                                                                                       \
    } while (0)

// The force path of the neural potential in five stages (each reads only
// what the earlier ones wrote, so any stage can be re-run on its own):
// 0 neighbour search, 1 descriptors, 2 MLP, 3 adjoint, 4 forces and bead sums.
void launch_force_stage(pimd_ctx *c, int stage, const float *q, float *E_out, float *F_out, float *W_out)
{
    const DevBuffers &d = c->d;
    const Sizes &z = c->z;
    hipStream_t s = c->stream;
    switch (stage) {
    case 0:
        if (z.skin) {
            launch_skin_neighbors(q, d, z, c->skin, c->dp.rc2, c->pl.n_el, c->tn, s);
            break;
        }
        if (z.any_periodic)
            launch_zero_i32(d.cell_count, z.total_cells, s);
        launch_wrap_bin(q, d, z, s);
        if (z.any_periodic) {
            launch_cell_scan(d, z, s);
            launch_cell_fill(d, z, s);
        }
        if (!c->tn.centre_lanes)   // the lane-per-centre forward writes the lists itself
            launch_neighbors(d, z, c->dp.rc2, c->pl.n_el, c->tn, s);
        break;
    case 1:
        if (c->tn.centre_lanes)
            launch_sm_forward(d, c->dp, c->pl.n_sm_units, c->pl.sm_nmax, s);
        else if (c->pl.gfn)
            launch_gfn_layers(d, z, c->dp, c->gp, c->tn, s);
        else if (c->dp.angular)
            launch_descriptors_g5(d, z, c->dp, c->tn, s);
        else
            launch_descriptors(d, z, c->dp, c->tn, s);
        break;
    case 2:
        if (c->pl.bpnn)
            launch_mlp(d, c->nets, c->n_mlp_tiles, c->pl.D, c->pl.Dp,
                       c->precision == PIMD_PREC_BF16_MLP && c->mlp_weights_bf16 ? 4 : c->precision, c->tn.mlp_rows,
                       c->tn.mlp_waves, c->tn.mlp_chain != 0, s);
        break;
    case 3:
        if (c->pl.gfn) {
            // the head has no energy: atomic energies and virials are zero
            if (F_out) {
                launch_gfn_forces(d, z, c->dp, c->gp, c->tn, F_out, s);
            } else {
                launch_zero_i32(reinterpret_cast<int32_t *>(d.E_atom), z.B, s);
                launch_zero_i32(reinterpret_cast<int32_t *>(d.vir_atom), (int64_t)z.B * 9, s);
            }
        } else if (F_out || W_out) {
            if (c->tn.centre_lanes)   // with the force assembly
                launch_sm_adjoint(d, c->dp, c->pl.n_sm_units, c->pl.sm_nmax, F_out, s);
            else if (c->dp.angular)
                launch_adjoint_g5(d, z, c->dp, c->tn, s);
            else
                launch_adjoint(d, z, c->dp, c->tn, s);
        }
        break;
    default:
        if (F_out && c->pl.bpnn && !c->tn.centre_lanes)
            launch_assemble_forces(d, z, F_out, c->tn, s);
        launch_bead_sums(d, z, E_out, W_out, W_out != nullptr, s);
    }
}

pimd_status run_forces(pimd_ctx *c, const float *q, float *E_out, float *F_out, float *W_out)
{
    const DevBuffers &d = c->d;
    const Sizes &z = c->z;
    hipStream_t s = c->stream;
    auto mark = [&](int k) {
        if (c->stage_ev)
            (void)hipEventRecord(c->stage_ev[k], s);
    };
    // the metadynamics bias joins the forces the integrator uses (never the
    // caller's arrays of pimd_energy_forces)
    const bool bias = c->pl.metad && F_out == d.F;
    c->atoms_of_state = q == d.q;   // per-atom energies and virials now belong to these positions
    if (c->potential == PIMD_POT_HARMONIC) {
        launch_harmonic(q, d, z, (float)(c->omega * c->omega * kMvv2e), F_out, s);
        launch_bead_sums(d, z, E_out, W_out, W_out != nullptr, s);
        if (bias)
            launch_metad(q, d, z, c->mp, c->pl.n_xrd_items, F_out, 1, c->deposit_now ? 1 : 0, d.cv_bead,
                         d.vbias_bead, s);
        for (int k = 2; k <= 6; ++k)
            mark(k);
        CHECK_LAUNCH(c);
        return PIMD_OK;
    }
    for (int k = 0; k < 5; ++k) {
        launch_force_stage(c, k, q, E_out, F_out, W_out);
        if (k < 4)
            mark(k + 2);
    }
    if (bias)
        launch_metad(q, d, z, c->mp, c->pl.n_xrd_items, F_out, 1, c->deposit_now ? 1 : 0, d.cv_bead, d.vbias_bead,
                     s);
    mark(6);
    CHECK_LAUNCH(c);
    return PIMD_OK;
}

pimd_status run_step(pimd_ctx *c, hipStream_t s, const float *xi)
{
    const uint32_t k0 = (uint32_t)(c->seed & 0xFFFFFFFFu), k1 = (uint32_t)(c->seed >> 32);
    hipStream_t saved = c->stream;
    c->stream = s;
    if (c->stage_ev)
        (void)hipEventRecord(c->stage_ev[0], s);
    launch_integrate_pre(c->d, c->z, (float)c->dt, k0, k1, xi, c->pl.max_P, c->transform, c->svr_c, s);
    if (c->stage_ev)
        (void)hipEventRecord(c->stage_ev[1], s);
    c->deposit_now = true;
    pimd_status st = run_forces(c, c->d.q, c->d.E_bead, c->d.F, nullptr);
    c->deposit_now = false;
    if (c->pl.metad)
        launch_metad_advance(c->d, c->mp, s);
    launch_integrate_post(c->d, c->z, (float)c->dt, k0, k1, xi, c->pl.max_P, c->transform, c->svr_c, s);
    launch_finish_step(c->d, c->z, s);
    if (c->stage_ev)
        (void)hipEventRecord(c->stage_ev[7], s);
    c->stream = saved;
    if (st != PIMD_OK)
        return st;
    CHECK_LAUNCH(c);
    return PIMD_OK;
}

pimd_status read_status(pimd_ctx *c)
{
    uint32_t st = 0;
    HIPCHK(c, hipMemcpyAsync(&st, c->d.status, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (st == 0)
        return PIMD_OK;
    // The integrator froze at the last step completed before the fault (the
    // kernels of later steps did nothing): take the step and hill counters
    // from the device again, and evaluate the forces of the frozen positions
    // before the next step.
    int64_t dstep = 0;
    int32_t dhills = 0;
    HIPCHK(c, hipMemcpyAsync(&dstep, c->d.step, 8, hipMemcpyDeviceToHost, c->stream));
    if (c->pl.metad)
        HIPCHK(c, hipMemcpyAsync(&dhills, c->d.n_hills, 4, hipMemcpyDeviceToHost, c->stream));
    const uint32_t zero = 0;
    HIPCHK(c, hipMemcpyAsync(c->d.status, &zero, 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->host_step = dstep;
    if (c->pl.metad)
        c->host_hills = dhills;
    c->forces_valid = false;
    if (st & kStatusHills) {
        c->err = "a deposition found the hill store full (max_hills)";
        return PIMD_E_CAPACITY;
    }
    if (st & kStatusOverflow) {
        c->err = "an atom has more neighbours than max_neighbors (" + std::to_string(c->pl.Kmax) + ")";
        return PIMD_E_CAPACITY;
    }
    c->err = "non-finite energy, force or state value";
    return PIMD_E_NONFINITE;
}

// Hills the next n steps deposit per bead (every bead deposits together),
// checked against the store before anything runs, then booked.
pimd_status reserve_steps(pimd_ctx *c, int64_t n)
{
    if (c->pl.metad) {
        const int64_t stride = c->mp.stride;
        const int64_t dep = (c->host_step + n) / stride - c->host_step / stride;
        if (c->host_hills + dep > c->mp.max_hills) {
            c->err = "these steps would deposit " + std::to_string(dep) + " hills per bead, " +
                     std::to_string(c->mp.max_hills - c->host_hills) + " left (max_hills)";
            return PIMD_E_CAPACITY;
        }
        c->host_hills += (int)dep;
    }
    c->host_step += n;
    return PIMD_OK;
}

}  // namespace

extern "C" {

const char *pimd_status_str(pimd_status s)
{
    switch (s) {
    case PIMD_OK: return "ok";
    case PIMD_E_ARG: return "invalid argument";
    case PIMD_E_UNSUPPORTED: return "unsupported configuration";
    case PIMD_E_DEVICE: return "HIP runtime error";
    case PIMD_E_OOM: return "workspace too small";
    case PIMD_E_CAPACITY: return "neighbour capacity exceeded";
    case PIMD_E_NONFINITE: return "non-finite value";
    case PIMD_E_STATE: return "call out of order";
    }
    return "unknown status";
}

const char *pimd_last_error(const pimd_ctx *ctx) { return ctx ? ctx->err.c_str() : g_init_error.c_str(); }

pimd_status pimd_workspace_size(const pimd_config *cfg, size_t *bytes)
{
    if (!bytes)
        return fail(&g_init_error, PIMD_E_ARG, "bytes is NULL");
    Plan pl;
    pimd_status st = validate(cfg, pl, &g_init_error);
    if (st != PIMD_OK)
        return st;
    *bytes = make_layout(pl).total;
    return PIMD_OK;
}

pimd_status pimd_init(const pimd_config *cfg, void *workspace_dev, size_t ws_bytes, void *hip_stream, pimd_ctx **out)
{
    if (!out)
        return fail(&g_init_error, PIMD_E_ARG, "out is NULL");
    *out = nullptr;
    Plan pl;
    pimd_status st = validate(cfg, pl, &g_init_error);
    if (st != PIMD_OK)
        return st;
    const Layout L = make_layout(pl);
    if (!workspace_dev)
        return fail(&g_init_error, PIMD_E_ARG, "workspace is NULL");
    if (((uintptr_t)workspace_dev) & 255)
        return fail(&g_init_error, PIMD_E_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total)
        return fail(&g_init_error, PIMD_E_OOM, "workspace smaller than pimd_workspace_size");

    pimd_ctx *c = new pimd_ctx();
    c->pl = pl;
    c->stream = (hipStream_t)hip_stream;
    c->dt = cfg->dt_fs;
    c->tau0 = cfg->tau0_fs;
    c->lam = cfg->pile_lambda;
    c->seed = cfg->seed;
    c->precision = cfg->precision;
    c->potential = cfg->potential;
    c->omega = cfg->harmonic_omega_per_fs;
    c->transform = cfg->transform;
    const pimd_bpnn_model *m = cfg->model;
    const ModelView mv = model_view(cfg);
    c->masses_el.assign(mv.mass, mv.mass + mv.n_el);
    c->species.assign(cfg->species, cfg->species + pl.n_atoms);
    c->temperature.assign(cfg->temperature_K, cfg->temperature_K + pl.n_sys);
    c->sys_host_box.assign(cfg->box_A, cfg->box_A + 3 * pl.n_sys);

    char *ws = (char *)workspace_dev;
    auto at = [&](const char *name) -> void * {
        auto it = L.off.find(name);
        return it == L.off.end() ? nullptr : ws + it->second;
    };
    DevBuffers &d = c->d;
    d.q = (float *)at("q");
    d.p = (float *)at("p");
    d.q_prev = (float *)at("q_prev");
    d.p_prev = (float *)at("p_prev");
    d.F = (float *)at("F");
    d.E_bead = (float *)at("E_bead");
    d.W_bead = (float *)at("W_bead");
    d.xi = (float *)at("xi");
    d.pos4 = (float4 *)at("pos4");
    d.posu4 = (float4 *)at("posu4");
    d.E_atom = (float *)at("E_atom");
    d.vir_atom = (float *)at("vir_atom");
    d.atom_cell = (int32_t *)at("atom_cell");
    d.atom_slot = (int32_t *)at("atom_slot");
    d.cell_count = (int32_t *)at("cell_count");
    d.cell_start = (int32_t *)at("cell_start");
    d.cell_atoms = (int32_t *)at("cell_atoms");
    d.cell_bead = (int32_t *)at("cell_bead");
    d.nbr = (int32_t *)at("nbr");
    d.nbr_cnt = (int32_t *)at("nbr_cnt");
    d.nbr_grp = (int32_t *)at("nbr_grp");
    d.nbr_fence = (int32_t *)at("nbr_fence");
    d.gfn_params = (float *)at("gfn_params");
    d.gfn_nodes = (float *)at("gfn_nodes");
    d.gfn_tiles = (uint16_t *)at("gfn_tiles");
    d.xhat = (float *)at("xhat");
    d.dEdG = (float *)at("dEdG");
    d.vslot = (float4 *)at("vslot");
    d.vrev = (float4 *)at("vrev");
    d.g5_mom = pl.angular ? (float *)at("g5_mom") : nullptr;
    d.tri_pairs = pl.bpnn && !pl.angular ? (uint16_t *)at("tri_pairs") : nullptr;
    d.tri_cnt = pl.bpnn && !pl.angular ? (int32_t *)at("tri_cnt") : nullptr;
    if (pl.skin > 0.0) {
        d.skin_keys = (int32_t *)at("skin_keys");
        d.skin_cnt = (int32_t *)at("skin_cnt");
        d.skin_c0 = (double4 *)at("skin_c0");
        d.skin_flag = (int32_t *)at("skin_flag");
        d.skin_builds = (unsigned long long *)at("skin_builds");
        d.sys_of_atom = (int32_t *)at("sys_of_atom");
    }
    d.mlp_f32 = (float *)at("mlp_f32");
    d.mlp_bf16 = (uint16_t *)at("mlp_bf16");
    d.mlp_f64 = (double *)at("mlp_f64");
    d.mlp_chain = pl.chain ? (uint16_t *)at("mlp_chain") : nullptr;
    d.norm = (float *)at("norm");
    d.elem_rows = (int32_t *)at("elem_rows");
    d.mlp_tiles = (MlpTile *)at("mlp_tiles");
    d.heat = (double *)at("heat");
    d.dke_part = (double *)at("dke_part");
    // PILE-G with a thermostat (tau0 > 0); NVE needs no centroid factor
    d.svr_part = (double *)at("svr_part");
    d.svr_alpha = cfg->tau0_fs > 0.0 ? (double *)at("svr_alpha") : nullptr;
    d.svr_kbar = (double *)at("svr_kbar");
    d.sm_units = (SmUnit *)at("sm_units");
    c->svr_c = cfg->tau0_fs > 0.0 ? std::exp(-0.5 * cfg->dt_fs / cfg->tau0_fs) : 1.0;
    d.step = (int64_t *)at("step");
    d.status = (uint32_t *)at("status");
    d.est_cols = (float *)at("est_cols");
    d.beads = (BeadInfo *)at("beads");
    d.bead_of_ba = (int32_t *)at("bead_of_ba");
    d.species_atom = (int32_t *)at("species_atom");
    d.mass_atom = (float *)at("mass_atom");
    d.sys = (SysInfo *)at("sys");
    d.modes = (ModeInfo *)at("modes");
    d.units = (IntegUnit *)at("units");
    d.cmat = (double *)at("cmat");
    d.col_sys = (int32_t *)at("col_sys");

    Sizes &z = c->z;
    z.n_sys = pl.n_sys;
    z.B = pl.B;
    z.n_beads_total = pl.n_beads;
    z.n_atoms_total = pl.n_atoms;
    z.ncol = pl.ncol;
    z.total_cells = pl.total_cells;
    z.n_units = pl.n_units;
    z.D = pl.D;
    z.Kmax = pl.Kmax;
    z.any_periodic = pl.any_periodic ? 1 : 0;
    for (int s = 0; s < pl.n_sys; ++s)
        z.max_bead_atoms = std::max(z.max_bead_atoms, cfg->n_atoms[s]);
    c->tn.nl_cells = pl.total_cells >= 4096 ? 1 : 0;
    // dense periodic liquids hide the reverse-slot loads behind the adjoint's
    // triplet work; a few neighbours per atom leave nothing to hide them behind
    c->tn.force_rows = pl.any_periodic ? 1 : 0;
    c->tn.centre_lanes = pl.small ? 1 : 0;
    if (c->precision == PIMD_PREC_BF16_MLP || c->precision == PIMD_PREC_BF16_PLAIN) {
        c->tn.mlp_rows = 32;    // 32-row tiles, one 16-column tile per wave: fastest at 64 to 16384 bead-atoms
        c->tn.mlp_waves = 8;
        if (pl.chain) {         // the register-chained kernel, where built: faster on every workload measured
            c->tn.mlp_chain = 1;
            c->tn.mlp_rows = 16;
        }
    }
    z.any_open = pl.any_open ? 1 : 0;
    z.any_box = pl.any_box ? 1 : 0;
    z.skin = pl.skin > 0.0 ? 1 : 0;
    if (z.skin) {
        const double reach = mv.cutoff + pl.skin + 1e-3;
        c->skin = SkinParams{0.25 * pl.skin * pl.skin, reach * reach, pl.Kc};
    }

    // ---- host tables
    std::vector<BeadInfo> beads;
    std::vector<int32_t> bead_of_ba(pl.B), col_sys(pl.ncol);
    std::vector<float> mass_atom(pl.n_atoms);
    std::vector<ModeInfo> modes;
    std::vector<IntegUnit> units;
    std::vector<double> cmat;
    std::vector<int32_t> cell_bead;
    std::map<int, int> cmat_off;
    // normal modes per distinct P: twiddles cos(2 pi m/P) and sin(2 pi m/P),
    // m = 0 .. P-1, then the normalisations 1/sqrt(P) and sqrt(2/P); the
    // integrator forms C[j][k] from them (m = jk mod P).  The quarter and half
    // turns are set exactly.
    for (int P : pl.distinct_P) {
        cmat_off[P] = (int)cmat.size();
        std::vector<double> cs(P), sn(P);
        for (int m = 0; m < P; ++m) {
            const int q = (4 * m) % (4 * P);
            if (q % P == 0) {   // m P/4 multiples: 0, 1/4, 1/2, 3/4 turn
                const int turn = (4 * m) / P;
                cs[m] = turn == 0 ? 1.0 : (turn == 2 ? -1.0 : 0.0);
                sn[m] = turn == 1 ? 1.0 : (turn == 3 ? -1.0 : 0.0);
            } else {
                cs[m] = std::cos(2.0 * kPi * m / P);
                sn[m] = std::sin(2.0 * kPi * m / P);
            }
        }
        cmat.insert(cmat.end(), cs.begin(), cs.end());
        cmat.insert(cmat.end(), sn.begin(), sn.end());
        cmat.push_back(1.0 / std::sqrt((double)P));
        cmat.push_back(std::sqrt(2.0 / P));
    }
    int ba0 = 0, atom0 = 0, cell0 = 0, mode0 = 0;
    for (int s = 0; s < pl.n_sys; ++s) {
        const int N = cfg->n_atoms[s], P = cfg->n_beads[s];
        const double T = cfg->temperature_K[s];
        const double *Lb = cfg->box_A + 3 * s;
        const bool periodic = Lb[0] != 0.0 || Lb[1] != 0.0 || Lb[2] != 0.0;
        SysInfo si{};
        si.N = N;
        si.P = P;
        si.ba0 = ba0;
        si.atom0 = atom0;
        si.mode0 = mode0;
        si.cmat0 = cmat_off[P];
        si.unit0 = (int)units.size();
        si.sig_T = (float)std::sqrt(kKB * T * P / kMvv2e);
        const int cols_per_unit = std::max(1, 256 / P);
        for (int c0 = 0; c0 < 3 * N; c0 += cols_per_unit) {
            IntegUnit u{};
            u.sys = s;
            u.col0 = c0;
            u.ncol = std::min(cols_per_unit, 3 * N - c0);
            units.push_back(u);
        }
        si.nunit = (int)units.size() - si.unit0;
        // modes
        const double wP = P * kKB * T / kHbar;
        for (int k = 0; k < P; ++k) {
            // normal mode k: w_k = 2 w_P sin(k pi / P), physical mass; staging
            // coordinate k + 1: kinetic mass P m for k = 0 and P (k + 1)/k m
            // otherwise, so u_{k+1} turns at w_P / sqrt(P) under its spring
            // (k + 1)/k m w_P^2; primitive bead k: w = w_P (the spring
            // constant), friction 1/tau0
            const bool staging = c->transform == PIMD_TRANSFORM_STAGING;
            const bool primitive = c->transform == PIMD_TRANSFORM_PRIMITIVE;
            const double w = primitive ? (P > 1 ? wP : 0.0)
                             : staging ? (k == 0 ? 0.0 : wP / std::sqrt((double)P))
                                       : 2.0 * wP * std::sin(k * kPi / P);
            double gamma = 0.0;
            if (c->tau0 > 0.0)
                gamma = (k == 0 || primitive) ? 1.0 / c->tau0 : 2.0 * c->lam * w;
            const double c1 = std::exp(-0.5 * gamma * c->dt);
            ModeInfo mi{};
            mi.c1 = c1;
            mi.c2 = std::sqrt(std::max(0.0, 1.0 - c1 * c1));
            mi.cw = std::cos(w * c->dt);
            mi.sw = std::sin(w * c->dt);
            mi.w = w;
            mi.mfac = staging ? (double)P * (k > 0 ? (double)(k + 1) / (double)k : 1.0) : 1.0;
            modes.push_back(mi);
        }
        for (int k = 0; k < P; ++k) {
            BeadInfo bi{};
            bi.sys = s;
            bi.ba0 = ba0 + k * N;
            bi.n = N;
            bi.periodic = periodic ? 1 : 0;
            for (int dd = 0; dd < 3; ++dd) {
                bi.L[dd] = (float)Lb[dd];
                bi.invL[dd] = periodic ? (float)(1.0 / Lb[dd]) : 0.0f;
                bi.nc[dd] = periodic && pl.nl ? pl.nc[s][dd] : 1;
                bi.cell_scale[dd] = periodic && pl.nl ? (float)(pl.nc[s][dd] / Lb[dd]) : 0.0f;
                bi.L64[dd] = Lb[dd];
                bi.invL64[dd] = periodic ? 1.0 / Lb[dd] : 0.0;
            }
            bi.cell0 = cell0;
            for (int cc = 0; cc < pl.cells_per_sys[s]; ++cc)
                cell_bead.push_back((int32_t)beads.size());
            cell0 += pl.cells_per_sys[s];
            for (int i = 0; i < N; ++i)
                bead_of_ba[bi.ba0 + i] = (int)beads.size();
            beads.push_back(bi);
        }
        for (int i = 0; i < N; ++i) {
            mass_atom[atom0 + i] = (float)mv.mass[cfg->species[atom0 + i]];
            for (int cc = 0; cc < 3; ++cc)
                col_sys[3 * (atom0 + i) + cc] = s;
        }
        c->sys_host.push_back(si);
        ba0 += N * P;
        atom0 += N;
        mode0 += P;
    }

    std::vector<std::pair<size_t, std::vector<char>>> uploads;
    auto push = [&](void *dst, const void *src, size_t bytes) {
        if (!bytes)
            return;
        std::vector<char> v((const char *)src, (const char *)src + bytes);
        uploads.push_back({(size_t)((char *)dst - ws), std::move(v)});
    };
    push(d.beads, beads.data(), beads.size() * sizeof(BeadInfo));
    push(d.bead_of_ba, bead_of_ba.data(), bead_of_ba.size() * 4);
    push(d.species_atom, cfg->species, (size_t)pl.n_atoms * 4);
    std::vector<int32_t> sys_of_atom;
    std::vector<double> skin_c0;
    const int32_t skin_init[2] = {1, 0};           // the first force evaluation builds the lists
    const unsigned long long builds0[2] = {0, 0};
    if (pl.skin > 0.0) {
        for (int s = 0; s < pl.n_sys; ++s)
            sys_of_atom.insert(sys_of_atom.end(), cfg->n_atoms[s], s);
        skin_c0.assign((size_t)pl.n_atoms * 4, 0.0);
        push(d.sys_of_atom, sys_of_atom.data(), sys_of_atom.size() * 4);
        push(d.skin_c0, skin_c0.data(), skin_c0.size() * 8);
        push(d.skin_flag, skin_init, sizeof(skin_init));
        push(d.skin_builds, builds0, sizeof(builds0));
    }
    push(d.mass_atom, mass_atom.data(), mass_atom.size() * 4);
    push(d.sys, c->sys_host.data(), c->sys_host.size() * sizeof(SysInfo));
    push(d.modes, modes.data(), modes.size() * sizeof(ModeInfo));
    push(d.units, units.data(), units.size() * sizeof(IntegUnit));
    push(d.cmat, cmat.data(), cmat.size() * 8);
    if (pl.nl)
        push(d.cell_bead, cell_bead.data(), cell_bead.size() * 4);
    push(d.col_sys, col_sys.data(), col_sys.size() * 4);
    std::vector<SmUnit> sm_units;
    if (pl.small) {
        // whole beads in bead order, as many as fit in the 64 lanes of a wave
        for (const BeadInfo &b : beads) {
            if (sm_units.empty() || sm_units.back().nrows + b.n > kWave)
                sm_units.push_back(SmUnit{b.ba0, 0, 0, 0});
            sm_units.back().nrows += b.n;
            sm_units.back().nmax = std::max(sm_units.back().nmax, b.n);
        }
        push(d.sm_units, sm_units.data(), sm_units.size() * sizeof(SmUnit));
    }

    if (pl.nl) {
        // cutoff and radial grid (both neural potentials)
        DescParams &dp = c->dp;
        dp.n_el = mv.n_el;
        dp.n_rad = mv.n_rad;
        dp.Kmax = pl.Kmax;
        dp.rc = (float)mv.cutoff;
        dp.rc2 = (float)(mv.cutoff * mv.cutoff);
        dp.pi_over_rc = (float)(kPi / mv.cutoff);
        dp.half_over_rc = (float)(0.5 / mv.cutoff);
        for (int s = 0; s < mv.n_rad; ++s) {
            dp.rad_center[s] = (float)mv.rad_center[s];
            dp.rad_center_lo[s] = (float)(mv.rad_center[s] - (double)dp.rad_center[s]);
            dp.rad_eta[s] = (float)mv.rad_eta[s];
            dp.rad_pack[s] = make_float4(dp.rad_center[s], dp.rad_center_lo[s], -dp.rad_eta[s] * 1.4426950408889634f,
                                         -2.0f * dp.rad_eta[s]);
        }
    }
    if (pl.gfn) {
        // packed weights go to the device as they are; the head's tables point into them
        const pimd_gfn_model *g = cfg->gfn;
        push(d.gfn_params, g->params, pl.gfn_floats * 4);
        const int H = g->width, ne = g->n_elements;
        const float *p0 = d.gfn_params;
        size_t o = 0;
        auto take = [&](size_t n) {
            const float *q = p0 + o;
            o += n;
            return q;
        };
        GfnParams &gp = c->gp;
        gp.H = H;
        gp.L = g->n_layers;
        gp.node_embed = take((size_t)ne * H);
        gp.pair_embed = take((size_t)ne * ne * H);
        gp.edge_in = take((size_t)H * g->n_rad);
        for (int l = 0; l < g->n_layers; ++l) {
            const size_t HH = (size_t)H * H;
            gp.msg[l] = GfnMlp{take(HH), take(H), take(HH), take(H)};
            gp.node[l] = GfnMlp{take(2 * HH), take(H), take(HH), take(H)};
            gp.edge[l] = GfnMlp{take(HH), take(H), take(HH), take(H)};
        }
        gp.fW1 = take((size_t)H * H);
        gp.fb1 = take(H);
        gp.fw2 = take(H);
        gp.fb2 = g->params[o];
        (void)take(1);
        // MFMA path (BF16 precisions): bfloat16 tiles of the per-edge matrices in
        // A-operand order -- tile (ob, kb), lane (lr, lg): W[16 ob + lr][16 kb + 4 lg + q],
        // q = 0..3, as 4 hi parts then 4 lo parts (lo = bf16(w - hi))
        gp.mode = cfg->precision == PIMD_PREC_BF16_MLP ? 1 : cfg->precision == PIMD_PREC_BF16_PLAIN ? 2 : 0;
        std::vector<uint16_t> tiles;
        auto pack = [&](const float *Wdev, int rows, int cols) -> const uint16_t * {
            const float *W = g->params + (Wdev - p0);     // the same weights on the host
            const size_t first = tiles.size() / (kWave * 8);
            for (int ob = 0; ob < (rows + 15) / 16; ++ob)
                for (int kb = 0; kb < (cols + 15) / 16; ++kb)
                    for (int lane = 0; lane < kWave; ++lane) {
                        const int rr = 16 * ob + (lane & 15);
                        uint16_t hi[4], lo[4];
                        for (int q = 0; q < 4; ++q) {
                            const int cc = 16 * kb + 4 * (lane >> 4) + q;
                            const float w = rr < rows && cc < cols ? W[(size_t)rr * cols + cc] : 0.0f;
                            hi[q] = bf16_bits(w);
                            uint32_t u = (uint32_t)hi[q] << 16;
                            float h;
                            std::memcpy(&h, &u, 4);
                            lo[q] = bf16_bits(w - h);
                        }
                        tiles.insert(tiles.end(), hi, hi + 4);
                        tiles.insert(tiles.end(), lo, lo + 4);
                    }
            return d.gfn_tiles + first * kWave * 8;
        };
        gp.t_in = pack(gp.edge_in, H, g->n_rad);
        for (int l = 0; l < g->n_layers; ++l) {
            gp.t_msg1[l] = pack(gp.msg[l].W1, H, H);
            gp.t_msg2[l] = pack(gp.msg[l].W2, H, H);
            gp.t_edge1[l] = pack(gp.edge[l].W1, H, H);
            gp.t_edge2[l] = pack(gp.edge[l].W2, H, H);
        }
        gp.t_f1 = pack(gp.fW1, H, H);
        push(d.gfn_tiles, tiles.data(), tiles.size() * 2);
    }
    if (pl.bpnn) {
        DescParams &dp = c->dp;
        dp.n_ang_eta = m->n_ang_eta;
        dp.n_ang = 8 * m->n_ang_eta;
        dp.D = pl.D;
        for (int s = 0; s < m->n_ang_eta; ++s)
            dp.ang_eta[s] = (float)m->ang_eta[s];
        // the 16-feature angular grid takes eta_1 = 4 eta_0 (exact in float too):
        // the triplet kernels then square exp(-eta_0 r_jk^2) twice instead of
        // evaluating a second exponential
        dp.eta_pow4 = m->n_ang_eta == 2 && dp.ang_eta[1] == 4.0f * dp.ang_eta[0] ? 1 : 0;
        dp.angular = pl.angular;
        {
            // Legendre coefficients of (1 + c)^zeta: multiply by (1 + c) zeta times,
            // with c P_l = ((l + 1) P_{l+1} + l P_{l-1}) / (2l + 1)
            static const int kZeta[4] = {1, 2, 4, 8};
            for (int iz = 0; iz < 4; ++iz) {
                double a[10] = {1.0};
                for (int t = 0; t < kZeta[iz]; ++t) {
                    double b[10] = {0.0};
                    for (int l = 0; l <= 8; ++l) {
                        b[l] += a[l];
                        b[l + 1] += a[l] * (l + 1) / (2.0 * l + 1.0);
                        if (l > 0)
                            b[l - 1] += a[l] * l / (2.0 * l + 1.0);
                    }
                    std::copy(b, b + 10, a);
                }
                for (int l = 0; l <= 8; ++l)
                    dp.g5_leg[iz][l] = (float)(a[l] * std::ldexp(1.0, 1 - kZeta[iz]));
            }
        }
        // rows grouped by element for the MLP gather, cut into tiles of tn.mlp_rows
        std::vector<int32_t> rows;
        c->elem_row0.assign(1, 0);
        for (int e = 0; e < pl.n_el; ++e) {
            for (int s = 0; s < pl.n_sys; ++s) {
                const SysInfo &si = c->sys_host[s];
                for (int k = 0; k < si.P; ++k)
                    for (int i = 0; i < si.N; ++i)
                        if (cfg->species[si.atom0 + i] == e)
                            rows.push_back(si.ba0 + k * si.N + i);
            }
            c->elem_row0.push_back((int32_t)rows.size());
        }
        const std::vector<MlpTile> tiles = mlp_tiles(c->elem_row0, c->tn.mlp_rows);
        c->n_mlp_tiles = (int)tiles.size();
        push(d.elem_rows, rows.data(), rows.size() * 4);
        push(d.mlp_tiles, tiles.data(), tiles.size() * sizeof(MlpTile));
        // normalisation
        std::vector<float> norm((size_t)pl.n_el * 2 * pl.D);
        for (int e = 0; e < pl.n_el; ++e)
            for (int f = 0; f < pl.D; ++f) {
                norm[(size_t)e * 2 * pl.D + f] = m->feat_shift[(size_t)e * pl.D + f];
                norm[(size_t)e * 2 * pl.D + pl.D + f] = 1.0f / m->feat_scale[(size_t)e * pl.D + f];
            }
        push(d.norm, norm.data(), norm.size() * 4);
        // weights: f32 W[out][in_pad], WT[in_pad][out], b[out] per layer, then w_out; bf16 W, WT
        std::vector<float> wf;
        std::vector<uint16_t> wb, wc;
        std::vector<double> w64;
        const float *src = m->params;
        // Fragments of the register-chained MLP: A operands of the 16 x 16 x 32
        // MFMA, one 16-byte run of eight bfloat16 values per lane, for output
        // tile o (rows 16 o + lane mod 16) and k-step b; the k index of lane
        // group g runs over the features 32 b + 4 g + j, then 32 b + 16 + 4 g + j
        // (j < 4), the order in which a layer's output tiles leave them.
        // value(row, k) gives the matrix entry, zero outside it; hi and lo
        // (the bfloat16 remainder) parts.  Returns the offset of the hi part.
        // The row tiles of W^T (input features) are padded to whole 32-feature
        // steps, as the kernel's last GEMM takes them (rows_to32).
        auto pack_chain = [&](int n_rows, int n_k, bool rows_to32, auto value, size_t &lo_at) {
            const int OT = rows_to32 ? 2 * ((n_rows + 31) / 32) : (n_rows + 15) / 16, KB = (n_k + 31) / 32;
            const size_t n = (size_t)OT * KB * kWave * 8, hi_at = wc.size();
            wc.resize(hi_at + 2 * n, 0);
            lo_at = hi_at + n;
            for (int o = 0; o < OT; ++o)
                for (int b = 0; b < KB; ++b)
                    for (int lane = 0; lane < kWave; ++lane)
                        for (int j = 0; j < 8; ++j) {
                            const int row = 16 * o + (lane & 15), g = lane >> 4;
                            const int k = 32 * b + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
                            const float v = (row < n_rows && k < n_k) ? value(row, k) : 0.0f;
                            const size_t at = (((size_t)o * KB + b) * kWave + lane) * 8 + j;
                            const uint16_t h = bf16_bits(v);
                            uint32_t u = (uint32_t)h << 16;
                            float hv;
                            std::memcpy(&hv, &u, 4);
                            wc[hi_at + at] = h;
                            wc[lo_at + at] = bf16_bits(v - hv);
                        }
            return hi_at;
        };
        std::vector<std::array<size_t, 4>> chain_at;   // per (element, layer): W hi, W lo, WT hi, WT lo
        for (int e = 0; e < pl.n_el; ++e) {
            MlpNet net{};
            net.n_hidden = m->n_hidden;
            int in = pl.D, in_pad = pl.Dp;
            for (int l = 0; l < m->n_hidden; ++l) {
                const int out = m->hidden[l];
                const size_t oW = wf.size();
                wf.resize(oW + (size_t)out * in_pad, 0.0f);
                for (int o = 0; o < out; ++o)
                    for (int k = 0; k < in; ++k)
                        wf[oW + (size_t)o * in_pad + k] = src[(size_t)o * in + k];
                const size_t oWT = wf.size();
                wf.resize(oWT + (size_t)in_pad * out, 0.0f);
                for (int o = 0; o < out; ++o)
                    for (int k = 0; k < in; ++k)
                        wf[oWT + (size_t)k * out + o] = src[(size_t)o * in + k];
                src += (size_t)out * in;
                const size_t ob = wf.size();
                wf.insert(wf.end(), src, src + out);
                src += out;
                // bf16 parts: nearest-even rounding and the rounding remainder
                auto split = [&](size_t o, size_t &hi, size_t &lo) {
                    hi = wb.size();
                    for (size_t t = 0; t < (size_t)out * in_pad; ++t)
                        wb.push_back(bf16_bits(wf[o + t]));
                    lo = wb.size();
                    for (size_t t = 0; t < (size_t)out * in_pad; ++t) {
                        uint32_t u = (uint32_t)wb[hi + t] << 16;
                        float h;
                        std::memcpy(&h, &u, 4);
                        wb.push_back(bf16_bits(wf[o + t] - h));
                    }
                };
                size_t bW, bWl, bWT, bWTl;
                split(oW, bW, bWl);
                split(oWT, bWT, bWTl);
                if (pl.chain) {
                    const float *Wl = wf.data() + oW;   // [out][in_pad]
                    const int ip = in_pad;
                    std::array<size_t, 4> at{};
                    at[0] = pack_chain(out, in, false, [&](int o, int k) { return Wl[(size_t)o * ip + k]; }, at[1]);
                    at[2] = pack_chain(in, out, true, [&](int k, int o) { return Wl[(size_t)o * ip + k]; }, at[3]);
                    chain_at.push_back(at);
                }
                const size_t dW = w64.size();
                for (size_t t = 0; t < (size_t)out * in_pad; ++t)
                    w64.push_back((double)wf[oW + t]);
                const size_t dWT = w64.size();
                for (size_t t = 0; t < (size_t)out * in_pad; ++t)
                    w64.push_back((double)wf[oWT + t]);
                MlpLayer &Ly = net.layer[l];
                Ly.W = d.mlp_f32 + oW;
                Ly.WT = d.mlp_f32 + oWT;
                Ly.b = d.mlp_f32 + ob;
                Ly.Wb = d.mlp_bf16 + bW;
                Ly.WTb = d.mlp_bf16 + bWT;
                Ly.Wb_lo = d.mlp_bf16 + bWl;
                Ly.WTb_lo = d.mlp_bf16 + bWTl;
                Ly.W64 = d.mlp_f64 + dW;
                Ly.WT64 = d.mlp_f64 + dWT;
                if (pl.chain) {
                    const std::array<size_t, 4> &at = chain_at.back();
                    Ly.Wc = d.mlp_chain + at[0];
                    Ly.Wc_lo = d.mlp_chain + at[1];
                    Ly.WTc = d.mlp_chain + at[2];
                    Ly.WTc_lo = d.mlp_chain + at[3];
                }
                Ly.in_pad = in_pad;
                Ly.out = out;
                in = out;
                in_pad = out;
            }
            const size_t owo = wf.size();
            wf.insert(wf.end(), src, src + in);
            src += in;
            net.wo = d.mlp_f32 + owo;
            net.bo = *src++;
            net.inv_scale = d.norm + (size_t)e * 2 * pl.D + pl.D;
            net.shift = d.norm + (size_t)e * 2 * pl.D;
            c->nets.net[e] = net;
        }
        push(d.mlp_f32, wf.data(), wf.size() * 4);
        push(d.mlp_bf16, wb.data(), wb.size() * 2);
        if (pl.chain) {
            if (wc.size() != pl.mlp_chain_elems) {   // the layout and the packing disagree
                delete c;
                return fail(&g_init_error, PIMD_E_DEVICE, "internal: chained MLP fragment count");
            }
            push(d.mlp_chain, wc.data(), wc.size() * 2);
        }
        // weights that are bfloat16 values already leave every lo part zero: the
        // split BF16 mode then needs two products per term instead of three
        c->mlp_weights_bf16 = true;
        for (int e = 0; e < pl.n_el && c->mlp_weights_bf16; ++e)
            for (int l = 0; l < m->n_hidden && c->mlp_weights_bf16; ++l) {
                const MlpLayer &Ly = c->nets.net[e].layer[l];
                const size_t lo = (size_t)(Ly.Wb_lo - d.mlp_bf16), n = (size_t)Ly.out * Ly.in_pad;
                for (size_t t = 0; t < n; ++t)
                    if (wb[lo + t] != 0 && wb[lo + t] != 0x8000) {
                        c->mlp_weights_bf16 = false;
                        break;
                    }
            }
        push(d.mlp_f64, w64.data(), w64.size() * 8);
    }
    if (pl.metad) {
        const pimd_metad *md = cfg->metad;
        d.hills = (double2 *)at("hills");
        d.n_hills = (int32_t *)at("n_hills");
        d.cv_bead = (double *)at("cv_bead");
        d.vbias_bead = (double *)at("vbias_bead");
        d.cv_eval = (double *)at("cv_eval");
        d.vbias_eval = (double *)at("vbias_eval");
        d.wt_scale = (double *)at("wt_scale");
        d.xrd_row = (double *)at("xrd_row");
        d.xrd_grad = (float *)at("xrd_grad");
        d.xrd_items = (int4 *)at("xrd_items");
        d.xrd_part0 = (int32_t *)at("xrd_part0");
        d.xrd_part = (double4 *)at("xrd_part");
        d.cv_atoms = (int32_t *)at("cv_atoms");
        d.cv_coef = (double *)at("cv_coef");
        c->fes_grid = (double *)at("fes_grid");
        c->fes_out = (double *)at("fes_out");
        MetadParams &mp = c->mp;
        mp.cv = md->cv;
        mp.n_terms = pl.n_terms;
        mp.stride = md->stride;
        mp.max_hills = md->max_hills;
        mp.q_scatter = md->q_scatter;
        mp.sigma = md->sigma;
        mp.inv_sigma = 1.0 / md->sigma;
        mp.height0 = md->height0_eV;
        for (int e = 0; e < pl.n_el; ++e)
            mp.form_factor[e] = md->cv == PIMD_CV_XRD ? md->form_factor[e] : 0.0;
        c->bias_factor = md->bias_factor;
        std::vector<double> wt(pl.n_sys);
        for (int s = 0; s < pl.n_sys; ++s)
            wt[s] = std::isinf(md->bias_factor) ? 0.0 : 1.0 / (kKB * cfg->temperature_K[s] * (md->bias_factor - 1.0));
        push(d.wt_scale, wt.data(), wt.size() * 8);
        mp.xrd_tile = pl.xrd_tile;
        if (md->cv == PIMD_CV_XRD) {
            // work items (bead, I, J >= I, first partial of the bead), partials per
            // bead laid out [partner tile][row]
            std::vector<int4> items;
            std::vector<int32_t> part0(beads.size());
            int64_t off = 0;
            for (int b = 0; b < (int)beads.size(); ++b) {
                const int nt = (beads[b].n + pl.xrd_tile - 1) / pl.xrd_tile;
                part0[b] = (int32_t)off;
                for (int I = 0; I < nt; ++I)
                    for (int J = I; J < nt; ++J)
                        items.push_back(make_int4(b, I, J, (int32_t)off));
                off += (int64_t)nt * beads[b].n;
            }
            push(d.xrd_items, items.data(), items.size() * 16);
            push(d.xrd_part0, part0.data(), part0.size() * 4);
        } else {
            push(d.cv_atoms, md->atoms, (size_t)pl.n_terms * 8);
            push(d.cv_coef, md->coef, (size_t)pl.n_terms * 8);
        }
        const int64_t zero = 0;
        push(d.n_hills, &zero, 8);
        std::vector<double> zb(pl.n_beads, 0.0);
        push(d.cv_bead, zb.data(), zb.size() * 8);
        push(d.vbias_bead, zb.data(), zb.size() * 8);
    }
    std::vector<double> zeros_d(pl.n_sys, 0.0);
    push(d.heat, zeros_d.data(), zeros_d.size() * 8);
    if (pl.pile_g) {
        // target centroid kinetic energy N_f k_B T P / 2 with N_f = 3N
        std::vector<double> kbar(pl.n_sys);
        for (int s = 0; s < pl.n_sys; ++s)
            kbar[s] = 1.5 * cfg->n_atoms[s] * kKB * cfg->temperature_K[s] * cfg->n_beads[s];
        push(d.svr_kbar, kbar.data(), kbar.size() * 8);
    }
    const int64_t zero64 = 0;
    push(d.step, &zero64, 8);
    push(d.status, &zero64, 8);

    // ---- device work starts here
    auto bail = [&](pimd_status s2, const std::string &msg) {
        g_init_error = msg;
        delete c;
        return s2;
    };
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess)
        return bail(PIMD_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    for (auto &u : uploads) {
        e = hipMemcpyAsync(ws + u.first, u.second.data(), u.second.size(), hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess)
            return bail(PIMD_E_DEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess)
        return bail(PIMD_E_DEVICE, std::string("upload sync: ") + hipGetErrorString(e));
    if (pl.bpnn) {
        e = pl.angular ? configure_g5_lds(c->dp) : configure_descriptor_lds(c->dp);
        if (e == hipSuccess && pl.small)
            e = configure_sm_lds(c->dp);
        if (e != hipSuccess)
            return bail(PIMD_E_DEVICE, std::string("descriptor LDS: ") + hipGetErrorString(e));
    }
    if (pl.nl) {
        e = configure_neighbor_lds(pl.Kmax);
        if (e != hipSuccess)
            return bail(PIMD_E_DEVICE, std::string("neighbour LDS: ") + hipGetErrorString(e));
    }
    e = configure_integrator_lds(pl.max_P);
    if (e != hipSuccess)
        return bail(PIMD_E_DEVICE, std::string("integrator LDS: ") + hipGetErrorString(e));
    *out = c;
    return PIMD_OK;
}

// ---- pimd_init without device allocation
// The workspace of pimd_init_static contexts: one array per device, held until
// the process ends.  In host code `scratch` names a host-side stand-in, not
// the device array: its device address comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address is used.
static __device__ __align__(256) unsigned char scratch[PIMD_STATIC_WORKSPACE_BYTES];

namespace {
std::mutex g_static_mu;
std::map<int, void *> g_static_ptr;   // device -> device address of its scratch array
std::map<int, bool> g_static_busy;    // device -> a live context holds the array
}  // namespace

pimd_status pimd_init_static(const pimd_config *cfg, void *hip_stream, pimd_ctx **out)
{
    if (!out)
        return fail(&g_init_error, PIMD_E_ARG, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    pimd_status st = pimd_workspace_size(cfg, &need);
    if (st != PIMD_OK)
        return st;
    if (need > PIMD_STATIC_WORKSPACE_BYTES)
        return fail(&g_init_error, PIMD_E_CAPACITY,
                    "pimd_init_static: the workspace needs " + std::to_string(need) +
                        " bytes; the static workspace holds " + std::to_string(PIMD_STATIC_WORKSPACE_BYTES));
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(&g_init_error, PIMD_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_busy[dev])
        return fail(&g_init_error, PIMD_E_STATE,
                    "pimd_init_static: another context holds this device's static workspace (destroy it first)");
    auto it = g_static_ptr.find(dev);
    if (it == g_static_ptr.end()) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(&g_init_error, PIMD_E_DEVICE,
                        std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        it = g_static_ptr.emplace(dev, ptr).first;
    }
    st = pimd_init(cfg, it->second, PIMD_STATIC_WORKSPACE_BYTES, hip_stream, out);
    if (st != PIMD_OK)
        return st;
    (*out)->static_device = dev;
    g_static_busy[dev] = true;
    return PIMD_OK;
}

pimd_status pimd_set_stream(pimd_ctx *ctx, void *hip_stream)
{
    if (!ctx)
        return PIMD_E_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return PIMD_OK;
}

pimd_status pimd_set_state(pimd_ctx *ctx, const float *q_dev, const float *p_dev, int64_t step)
{
    if (!ctx)
        return PIMD_E_ARG;
    if (!q_dev || !p_dev) {
        ctx->err = "q and p must be non-NULL";
        return PIMD_E_ARG;
    }
    if (step < 0) {
        ctx->err = "step must be >= 0";
        return PIMD_E_ARG;
    }
    const size_t bytes = (size_t)ctx->z.B * 12;
    HIPCHK(ctx, hipMemcpyAsync(ctx->d.q, q_dev, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(ctx->d.p, p_dev, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    // the state a fault before the first step freezes at
    HIPCHK(ctx, hipMemcpyAsync(ctx->d.q_prev, q_dev, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(ctx->d.p_prev, p_dev, bytes, hipMemcpyDeviceToDevice, ctx->stream));
    std::vector<double> zeros(ctx->z.n_sys, 0.0);
    HIPCHK(ctx, hipMemcpyAsync(ctx->d.heat, zeros.data(), zeros.size() * 8, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(ctx->d.step, &step, 8, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->state_set = true;
    ctx->forces_valid = false;
    ctx->host_step = step;
    return PIMD_OK;
}

pimd_status pimd_get_state(pimd_ctx *ctx, float *q_dev, float *p_dev, float *forces_dev, int64_t *step)
{
    if (!ctx)
        return PIMD_E_ARG;
    if (!ctx->state_set) {
        ctx->err = "state not set";
        return PIMD_E_STATE;
    }
    const size_t n = (size_t)ctx->z.B * 3;
    if (forces_dev && !ctx->forces_valid) {
        pimd_status st = run_forces(ctx, ctx->d.q, ctx->d.E_bead, ctx->d.F, nullptr);
        if (st != PIMD_OK)
            return st;
        ctx->forces_valid = true;
    }
    launch_check_finite(ctx->d.q, (int64_t)n, ctx->d.status, ctx->stream);
    launch_check_finite(ctx->d.p, (int64_t)n, ctx->d.status, ctx->stream);
    CHECK_LAUNCH(ctx);
    if (q_dev)
        HIPCHK(ctx, hipMemcpyAsync(q_dev, ctx->d.q, n * 4, hipMemcpyDeviceToDevice, ctx->stream));
    if (p_dev)
        HIPCHK(ctx, hipMemcpyAsync(p_dev, ctx->d.p, n * 4, hipMemcpyDeviceToDevice, ctx->stream));
    if (forces_dev)
        HIPCHK(ctx, hipMemcpyAsync(forces_dev, ctx->d.F, n * 4, hipMemcpyDeviceToDevice, ctx->stream));
    int64_t s = 0;
    HIPCHK(ctx, hipMemcpyAsync(&s, ctx->d.step, 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (step)
        *step = s;
    return read_status(ctx);
}

pimd_status pimd_get_heat_bath(pimd_ctx *ctx, double *heat_host)
{
    if (!ctx || !heat_host)
        return PIMD_E_ARG;
    HIPCHK(ctx, hipMemcpyAsync(heat_host, ctx->d.heat, (size_t)ctx->z.n_sys * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return PIMD_OK;
}

pimd_status pimd_set_heat_bath(pimd_ctx *ctx, const double *heat_host)
{
    if (!ctx || !heat_host)
        return PIMD_E_ARG;
    for (int s = 0; s < ctx->z.n_sys; ++s)
        if (!std::isfinite(heat_host[s])) {
            ctx->err = "heat bath values must be finite";
            return PIMD_E_ARG;
        }
    HIPCHK(ctx, hipMemcpyAsync(ctx->d.heat, heat_host, (size_t)ctx->z.n_sys * 8, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return PIMD_OK;
}

pimd_status pimd_check(pimd_ctx *ctx)
{
    if (!ctx)
        return PIMD_E_ARG;
    return read_status(ctx);
}

pimd_status pimd_energy_forces(pimd_ctx *ctx, const float *q_dev, float *energy_dev, float *forces_dev,
                               float *virial_dev)
{
    if (!ctx)
        return PIMD_E_ARG;
    if (!q_dev || !energy_dev) {
        ctx->err = "q and energy must be non-NULL";
        return PIMD_E_ARG;
    }
    return run_forces(ctx, q_dev, energy_dev, forces_dev, virial_dev);
}

pimd_status pimd_step(pimd_ctx *ctx, int32_t n_steps)
{
    if (!ctx)
        return PIMD_E_ARG;
    if (n_steps < 0) {
        ctx->err = "n_steps must be >= 0";
        return PIMD_E_ARG;
    }
    if (!ctx->state_set) {
        ctx->err = "pimd_set_state must come before pimd_step";
        return PIMD_E_STATE;
    }
    if (n_steps == 0)
        return PIMD_OK;
    {
        pimd_status st = reserve_steps(ctx, n_steps);
        if (st != PIMD_OK)
            return st;
    }
    if (!ctx->forces_valid) {
        pimd_status st = run_forces(ctx, ctx->d.q, ctx->d.E_bead, ctx->d.F, nullptr);
        if (st != PIMD_OK)
            return st;
        ctx->forces_valid = true;
    }
    int done = 0;
    if (ctx->noise_pending) {
        pimd_status st = run_step(ctx, ctx->stream, ctx->d.xi);
        ctx->noise_pending = false;
        if (st != PIMD_OK)
            return st;
        ++done;
    }
    if (!ctx->use_graph) {
        for (; done < n_steps; ++done) {
            pimd_status st = run_step(ctx, ctx->stream, nullptr);
            if (st != PIMD_OK)
                return st;
        }
        return PIMD_OK;
    }
    if (done < n_steps && !ctx->gexec) {
        if (!ctx->capture)
            HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
        HIPCHK(ctx, hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
        pimd_status st = run_step(ctx, ctx->capture, nullptr);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(ctx->capture, &g);
        if (st != PIMD_OK) {
            if (g)
                (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) {
            ctx->err = std::string("hipStreamEndCapture: ") + hipGetErrorString(e);
            return PIMD_E_DEVICE;
        }
        ctx->graph = g;
        HIPCHK(ctx, hipGraphInstantiate(&ctx->gexec, ctx->graph, nullptr, nullptr, 0));
    }
    for (; done < n_steps; ++done)
        HIPCHK(ctx, hipGraphLaunch(ctx->gexec, ctx->stream));
    return PIMD_OK;
}

pimd_status pimd_estimators(pimd_ctx *ctx, pimd_estimates *out_host)
{
    if (!ctx || !out_host)
        return PIMD_E_ARG;
    if (!ctx->state_set) {
        ctx->err = "state not set";
        return PIMD_E_STATE;
    }
    if (!ctx->forces_valid || !ctx->atoms_of_state) {
        // the per-atom terms were overwritten by an evaluation at other positions
        pimd_status st = run_forces(ctx, ctx->d.q, ctx->d.E_bead, ctx->d.F, ctx->d.W_bead);
        if (st != PIMD_OK)
            return st;
        ctx->forces_valid = true;
    } else {
        // bead virials of the state's per-atom virials (steps leave them out)
        launch_bead_sums(ctx->d, ctx->z, ctx->d.E_bead, ctx->d.W_bead, true, ctx->stream);
    }
    launch_estimator_terms(ctx->d, ctx->z, ctx->stream);
    CHECK_LAUNCH(ctx);
    std::vector<float> cols((size_t)ctx->z.ncol * 3), E(ctx->z.n_beads_total), Wb((size_t)ctx->z.n_beads_total * 9);
    HIPCHK(ctx, hipMemcpyAsync(Wb.data(), ctx->d.W_bead, Wb.size() * 4, hipMemcpyDeviceToHost, ctx->stream));
    std::vector<double> heat(ctx->z.n_sys), vb(ctx->pl.metad ? ctx->z.n_beads_total : 0);
    if (ctx->pl.metad)
        HIPCHK(ctx, hipMemcpyAsync(vb.data(), ctx->d.vbias_bead, vb.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(cols.data(), ctx->d.est_cols, cols.size() * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(E.data(), ctx->d.E_bead, E.size() * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(heat.data(), ctx->d.heat, heat.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    int bead0 = 0;
    for (int s = 0; s < ctx->z.n_sys; ++s) {
        const SysInfo &si = ctx->sys_host[s];
        const double T = ctx->temperature[s];
        const double beta = 1.0 / (kKB * T);
        const double wP = si.P * kKB * T / kHbar;
        double spring = 0, cv = 0, ke = 0, V = 0;
        for (int col = 3 * si.atom0; col < 3 * (si.atom0 + si.N); ++col) {
            spring += cols[3 * (size_t)col];
            cv += cols[3 * (size_t)col + 1];
            ke += cols[3 * (size_t)col + 2];
        }
        double vbias = 0, trW = 0;
        for (int k = 0; k < si.P; ++k) {
            V += E[bead0 + k];
            if (ctx->pl.metad)
                vbias += vb[bead0 + k];
            for (int a = 0; a < 3; ++a)
                trW += Wb[9 * (size_t)(bead0 + k) + 4 * a];
        }
        bead0 += si.P;
        pimd_estimates &o = out_host[s];
        o.V_bias = vbias / si.P;
        o.E_spring = si.P > 1 ? 0.5 * wP * wP * kMvv2e * spring : 0.0;
        o.V_bar = V / si.P;
        o.K_prim = 3.0 * si.N * si.P / (2.0 * beta) - o.E_spring / si.P;
        o.K_cv = 3.0 * si.N / (2.0 * beta) - cv / (2.0 * si.P);
        o.K_beads = 0.5 * kMvv2e * ke;
        o.T_beads = 2.0 * o.K_beads / (3.0 * si.N * si.P * kKB);
        o.heat_bath = heat[s];
        o.H_conserved = o.K_beads + o.E_spring + V + heat[s];
        // centroid-virial pressure of a periodic system (the direct-force head has no virial)
        const double *Lb = ctx->sys_host_box.data() + 3 * s;
        const double vol = Lb[0] * Lb[1] * Lb[2];
        o.P_cv = (vol > 0.0 && !ctx->pl.gfn) ? (2.0 * o.K_cv + trW / si.P) / (3.0 * vol) : 0.0;
    }
    return read_status(ctx);
}

static pimd_status need_metad(pimd_ctx *ctx)
{
    if (!ctx)
        return PIMD_E_ARG;
    if (!ctx->pl.metad) {
        ctx->err = "the context has no metadynamics bias";
        return PIMD_E_STATE;
    }
    return PIMD_OK;
}

pimd_status pimd_bias_forces(pimd_ctx *ctx, const float *q_dev, float *forces_dev, double *cv_dev,
                             double *bias_dev)
{
    pimd_status st = need_metad(ctx);
    if (st != PIMD_OK)
        return st;
    if (!q_dev) {
        ctx->err = "q must be non-NULL";
        return PIMD_E_ARG;
    }
    const DevBuffers &d = ctx->d;
    launch_metad(q_dev, d, ctx->z, ctx->mp, ctx->pl.n_xrd_items, forces_dev, 0, 0, d.cv_eval, d.vbias_eval,
                 ctx->stream);
    CHECK_LAUNCH(ctx);
    const size_t nb = (size_t)ctx->z.n_beads_total * 8;
    if (cv_dev)
        HIPCHK(ctx, hipMemcpyAsync(cv_dev, d.cv_eval, nb, hipMemcpyDeviceToDevice, ctx->stream));
    if (bias_dev)
        HIPCHK(ctx, hipMemcpyAsync(bias_dev, d.vbias_eval, nb, hipMemcpyDeviceToDevice, ctx->stream));
    return PIMD_OK;
}

pimd_status pimd_metad_cv(pimd_ctx *ctx, double *cv_host, double *bias_host)
{
    pimd_status st = need_metad(ctx);
    if (st != PIMD_OK)
        return st;
    if (!ctx->state_set) {
        ctx->err = "state not set";
        return PIMD_E_STATE;
    }
    if (!ctx->forces_valid) {
        if ((st = run_forces(ctx, ctx->d.q, ctx->d.E_bead, ctx->d.F, nullptr)) != PIMD_OK)
            return st;
        ctx->forces_valid = true;
    }
    const size_t nb = (size_t)ctx->z.n_beads_total * 8;
    if (cv_host)
        HIPCHK(ctx, hipMemcpyAsync(cv_host, ctx->d.cv_bead, nb, hipMemcpyDeviceToHost, ctx->stream));
    if (bias_host)
        HIPCHK(ctx, hipMemcpyAsync(bias_host, ctx->d.vbias_bead, nb, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return read_status(ctx);
}

pimd_status pimd_metad_hills(pimd_ctx *ctx, double *center_host, double *height_host, int32_t *n_hills)
{
    pimd_status st = need_metad(ctx);
    if (st != PIMD_OK)
        return st;
    int32_t nh = 0;
    HIPCHK(ctx, hipMemcpyAsync(&nh, ctx->d.n_hills, 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (n_hills)
        *n_hills = nh;
    if ((center_host || height_host) && nh > 0) {
        const size_t nb = ctx->z.n_beads_total;
        std::vector<double2> h(nb * nh);
        HIPCHK(ctx, hipMemcpy2DAsync(h.data(), (size_t)nh * 16, ctx->d.hills, (size_t)ctx->mp.max_hills * 16,
                                     (size_t)nh * 16, nb, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        for (size_t t = 0; t < h.size(); ++t) {
            if (center_host)
                center_host[t] = h[t].x;
            if (height_host)
                height_host[t] = h[t].y;
        }
    }
    return read_status(ctx);
}

pimd_status pimd_metad_set_hills(pimd_ctx *ctx, int32_t n_hills, const double *center_host,
                                 const double *height_host)
{
    pimd_status st = need_metad(ctx);
    if (st != PIMD_OK)
        return st;
    if (n_hills < 0 || n_hills > ctx->mp.max_hills) {
        ctx->err = "n_hills must be in [0, max_hills]";
        return PIMD_E_ARG;
    }
    if (n_hills > 0 && (!center_host || !height_host)) {
        ctx->err = "centers and heights must be non-NULL";
        return PIMD_E_ARG;
    }
    for (size_t t = 0; t < (size_t)ctx->z.n_beads_total * n_hills; ++t)
        if (!std::isfinite(center_host[t]) || !std::isfinite(height_host[t])) {
            ctx->err = "hill centers and heights must be finite";
            return PIMD_E_ARG;
        }
    const size_t nb = ctx->z.n_beads_total;
    if (n_hills > 0) {
        std::vector<double2> h(nb * n_hills);
        for (size_t t = 0; t < h.size(); ++t)
            h[t] = make_double2(center_host[t], height_host[t]);
        HIPCHK(ctx, hipMemcpy2DAsync(ctx->d.hills, (size_t)ctx->mp.max_hills * 16, h.data(), (size_t)n_hills * 16,
                                     (size_t)n_hills * 16, nb, hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    HIPCHK(ctx, hipMemcpyAsync(ctx->d.n_hills, &n_hills, 4, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->host_hills = n_hills;
    ctx->forces_valid = false;
    return PIMD_OK;
}

pimd_status pimd_metad_fes(pimd_ctx *ctx, int32_t system, int32_t n_grid, const double *s_host, double *fes_host)
{
    pimd_status st = need_metad(ctx);
    if (st != PIMD_OK)
        return st;
    if (system < 0 || system >= ctx->z.n_sys || n_grid < 0 || (n_grid > 0 && (!s_host || !fes_host))) {
        ctx->err = "bad system index, grid size or NULL grid";
        return PIMD_E_ARG;
    }
    int bead0 = 0;
    for (int s = 0; s < system; ++s)
        bead0 += ctx->sys_host[s].P;
    const double kT = kKB * ctx->temperature[system];
    const double ratio = std::isinf(ctx->bias_factor) ? 1.0 : ctx->bias_factor / (ctx->bias_factor - 1.0);
    for (int g0 = 0; g0 < n_grid; g0 += kFesChunk) {
        const int n = std::min(kFesChunk, n_grid - g0);
        HIPCHK(ctx, hipMemcpyAsync(ctx->fes_grid, s_host + g0, (size_t)n * 8, hipMemcpyHostToDevice, ctx->stream));
        launch_metad_fes(ctx->d, ctx->mp, bead0, ctx->sys_host[system].P, kT, ratio, ctx->fes_grid, n, ctx->fes_out,
                         ctx->stream);
        CHECK_LAUNCH(ctx);
        HIPCHK(ctx, hipMemcpyAsync(fes_host + g0, ctx->fes_out, (size_t)n * 8, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    return PIMD_OK;
}

pimd_status pimd_time_bias(pimd_ctx *ctx, int32_t n_reps, double *ms_host)
{
    pimd_status st = need_metad(ctx);
    if (st != PIMD_OK)
        return st;
    if (!ms_host || n_reps < 1)
        return PIMD_E_ARG;
    if (!ctx->state_set) {
        ctx->err = "state not set";
        return PIMD_E_STATE;
    }
    const DevBuffers &d = ctx->d;
    hipEvent_t ev[2];
    HIPCHK(ctx, hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        ctx->err = "hipEventCreate failed";
        return PIMD_E_DEVICE;
    }
    // one untimed pass, then n_reps passes of the CV and bias kernels writing
    // the bias forces into the force array (which is re-evaluated at the next step)
    launch_metad(d.q, d, ctx->z, ctx->mp, ctx->pl.n_xrd_items, d.F, 0, 0, d.cv_eval, d.vbias_eval, ctx->stream);
    (void)hipEventRecord(ev[0], ctx->stream);
    for (int r = 0; r < n_reps; ++r)
        launch_metad(d.q, d, ctx->z, ctx->mp, ctx->pl.n_xrd_items, d.F, 0, 0, d.cv_eval, d.vbias_eval, ctx->stream);
    (void)hipEventRecord(ev[1], ctx->stream);
    hipError_t e = hipEventSynchronize(ev[1]);
    float ms = 0.0f;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    ctx->forces_valid = false;
    if (e != hipSuccess) {
        ctx->err = std::string("bias timing: ") + hipGetErrorString(e);
        return PIMD_E_DEVICE;
    }
    *ms_host = (double)ms / n_reps;
    CHECK_LAUNCH(ctx);
    return read_status(ctx);
}

pimd_status pimd_inject_noise(pimd_ctx *ctx, const float *xi_dev)
{
    if (!ctx)
        return PIMD_E_ARG;
    if (!xi_dev) {
        ctx->err = "xi must be non-NULL";
        return PIMD_E_ARG;
    }
    HIPCHK(ctx, hipMemcpyAsync(ctx->d.xi, xi_dev, (size_t)ctx->z.B * 24, hipMemcpyDeviceToDevice, ctx->stream));
    ctx->noise_pending = true;
    return PIMD_OK;
}

pimd_status pimd_debug_neighbors(pimd_ctx *ctx, int32_t bead, int32_t *ij_host, int64_t cap, int64_t *count)
{
    if (!ctx || !count)
        return PIMD_E_ARG;
    if (!ctx->pl.nl) {
        ctx->err = "no neighbour list for this potential";
        return PIMD_E_STATE;
    }
    if (bead < 0 || bead >= ctx->z.n_beads_total || cap < 0 || (cap > 0 && !ij_host)) {
        ctx->err = "bad bead index or output buffer";
        return PIMD_E_ARG;
    }
    // locate the bead
    int b = bead, s = 0;
    while (b >= ctx->sys_host[s].P) {
        b -= ctx->sys_host[s].P;
        ++s;
    }
    const SysInfo &si = ctx->sys_host[s];
    const int row0 = si.ba0 + b * si.N;
    const int K = ctx->pl.Kmax;
    std::vector<int32_t> keys((size_t)si.N * K), cnt(si.N);
    HIPCHK(ctx, hipMemcpyAsync(keys.data(), ctx->d.nbr + (size_t)row0 * K, keys.size() * 4, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(cnt.data(), ctx->d.nbr_cnt + row0, cnt.size() * 4, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    int64_t n = 0;
    for (int i = 0; i < si.N; ++i) {
        std::vector<int32_t> js;
        for (int t = 0; t < cnt[i]; ++t)
            js.push_back((keys[(size_t)i * K + t] & (int32_t)kRowMask) - row0);
        std::sort(js.begin(), js.end());
        for (int32_t j : js) {
            if (n < cap) {
                ij_host[2 * n] = i;
                ij_host[2 * n + 1] = j;
            }
            ++n;
        }
    }
    *count = n;
    return n > cap ? PIMD_E_CAPACITY : PIMD_OK;
}

pimd_status pimd_debug_descriptors(pimd_ctx *ctx, float *xhat_dev)
{
    if (!ctx || !xhat_dev)
        return PIMD_E_ARG;
    if (ctx->potential != PIMD_POT_BPNN) {
        ctx->err = "no descriptors for this potential";
        return PIMD_E_STATE;
    }
    HIPCHK(ctx, hipMemcpyAsync(xhat_dev, ctx->d.xhat, (size_t)ctx->z.B * ctx->z.D * 4, hipMemcpyDeviceToDevice,
                               ctx->stream));
    return PIMD_OK;
}

pimd_status pimd_debug_copy(pimd_ctx *ctx, int32_t buffer, void *dst_dev, size_t bytes)
{
    if (!ctx || !dst_dev)
        return PIMD_E_ARG;
    const bool lists = buffer == PIMD_BUF_NBR || buffer == PIMD_BUF_NCOUNT;
    if (buffer != PIMD_BUF_EATOM && !(lists ? ctx->pl.nl : ctx->pl.bpnn)) {
        ctx->err = "buffer not used by this potential";
        return PIMD_E_STATE;
    }
    const size_t B = ctx->z.B, D = ctx->z.D, K = ctx->z.Kmax;
    const void *src = nullptr;
    size_t need = 0;
    switch (buffer) {
    case PIMD_BUF_XHAT: src = ctx->d.xhat; need = B * D * 4; break;
    case PIMD_BUF_DEDG: src = ctx->d.dEdG; need = B * D * 4; break;
    case PIMD_BUF_SLOTS: src = ctx->d.vslot; need = B * K * 16; break;
    case PIMD_BUF_NBR: src = ctx->d.nbr; need = B * K * 4; break;
    case PIMD_BUF_NCOUNT: src = ctx->d.nbr_cnt; need = B * 4; break;
    case PIMD_BUF_EATOM: src = ctx->d.E_atom; need = B * 4; break;
    default: ctx->err = "unknown buffer"; return PIMD_E_ARG;
    }
    if (bytes < need) {
        ctx->err = "destination smaller than the buffer";
        return PIMD_E_ARG;
    }
    HIPCHK(ctx, hipMemcpyAsync(dst_dev, src, need, hipMemcpyDeviceToDevice, ctx->stream));
    return PIMD_OK;
}

pimd_status pimd_debug_philox(pimd_ctx *ctx, int64_t step, int32_t half, int64_t n, uint32_t *words_dev)
{
    if (!ctx || !words_dev || n < 0 || step < 0 || (half != 0 && half != 1))
        return PIMD_E_ARG;
    launch_philox_words((uint32_t)(ctx->seed & 0xFFFFFFFFu), (uint32_t)(ctx->seed >> 32), step, half, n, words_dev,
                        ctx->stream);
    CHECK_LAUNCH(ctx);
    return PIMD_OK;
}

pimd_status pimd_set_graph(pimd_ctx *ctx, int32_t enabled)
{
    if (!ctx)
        return PIMD_E_ARG;
    ctx->use_graph = enabled != 0;
    return PIMD_OK;
}

pimd_status pimd_get_tuning(const pimd_ctx *ctx, pimd_tuning *out)
{
    if (!ctx || !out)
        return PIMD_E_ARG;
    *out = pimd_tuning{ctx->tn.centre_waves, ctx->tn.centre_grid, ctx->tn.mlp_rows, ctx->tn.nl_cells,
                       ctx->tn.mlp_waves, ctx->tn.force_rows, ctx->tn.centre_lanes, ctx->tn.mlp_chain};
    return PIMD_OK;
}

// The register-chained MLP: a BF16 precision and a model within its limits.
static bool chain_ok(const pimd_ctx *ctx)
{
    return ctx->pl.bpnn && ctx->pl.chain &&
           (ctx->precision == PIMD_PREC_BF16_MLP || ctx->precision == PIMD_PREC_BF16_PLAIN);
}

static pimd_status apply_tuning(pimd_ctx *ctx, const Tuning &tn)
{
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->pl.bpnn && tn.mlp_rows != ctx->tn.mlp_rows) {
        const std::vector<MlpTile> tiles = mlp_tiles(ctx->elem_row0, tn.mlp_rows);
        HIPCHK(ctx, hipMemcpyAsync(ctx->d.mlp_tiles, tiles.data(), tiles.size() * sizeof(MlpTile),
                                   hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        ctx->n_mlp_tiles = (int)tiles.size();
    }
    ctx->tn = tn;
    if (ctx->gexec) {
        (void)hipGraphExecDestroy(ctx->gexec);
        ctx->gexec = nullptr;
    }
    if (ctx->graph) {
        (void)hipGraphDestroy(ctx->graph);
        ctx->graph = nullptr;
    }
    return PIMD_OK;
}

pimd_status pimd_set_tuning(pimd_ctx *ctx, const pimd_tuning *t)
{
    if (!ctx || !t)
        return PIMD_E_ARG;
    const bool waves_ok = t->centre_waves == 1 || t->centre_waves == 2 || t->centre_waves == 4;
    const bool rows_ok = t->mlp_rows == 16 || t->mlp_rows == 32 || t->mlp_rows == 64;
    if (!waves_ok || !rows_ok || t->centre_grid < 0 || (t->neighbor_cells != 0 && t->neighbor_cells != 1) ||
        (t->mlp_waves != 4 && t->mlp_waves != 8) || (t->force_rows != 0 && t->force_rows != 1) ||
        (t->centre_lanes != 0 && t->centre_lanes != 1) || (t->mlp_chain != 0 && t->mlp_chain != 1)) {
        ctx->err = "tuning: centre_waves in {1, 2, 4}, centre_grid >= 0, mlp_rows in {16, 32, 64}, "
                   "neighbor_cells in {0, 1}, mlp_waves in {4, 8}, force_rows in {0, 1}, centre_lanes in {0, 1}, "
                   "mlp_chain in {0, 1}";
        return PIMD_E_ARG;
    }
    if (t->mlp_chain && !chain_ok(ctx)) {
        ctx->err = "mlp_chain = 1 needs a BF16 MLP of a shape the chained kernel is built for";
        return PIMD_E_UNSUPPORTED;
    }
    if (t->centre_lanes && !ctx->pl.small) {
        ctx->err = "centre_lanes = 1 needs G4 molecules without a box of at most 16 atoms each";
        return PIMD_E_UNSUPPORTED;
    }
    if (ctx->precision == PIMD_PREC_FP64_MLP && t->mlp_rows != 16) {
        ctx->err = "the FP64 MLP runs 16-row tiles only";
        return PIMD_E_UNSUPPORTED;
    }
    return apply_tuning(ctx, Tuning{t->centre_waves, t->centre_grid, t->mlp_rows, t->neighbor_cells, t->mlp_waves,
                                    t->force_rows, t->centre_lanes, t->mlp_chain});
}

// Mean milliseconds of one force evaluation of the current positions.
static pimd_status time_forces(pimd_ctx *ctx, int n_reps, double &ms)
{
    pimd_status st = run_forces(ctx, ctx->d.q, ctx->d.E_bead, ctx->d.F, nullptr);
    if (st != PIMD_OK)
        return st;
    hipEvent_t ev[2];
    HIPCHK(ctx, hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        ctx->err = "hipEventCreate failed";
        return PIMD_E_DEVICE;
    }
    (void)hipEventRecord(ev[0], ctx->stream);
    for (int r = 0; r < n_reps && st == PIMD_OK; ++r)
        st = run_forces(ctx, ctx->d.q, ctx->d.E_bead, ctx->d.F, nullptr);
    (void)hipEventRecord(ev[1], ctx->stream);
    hipError_t e = hipEventSynchronize(ev[1]);
    float t = 0.0f;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&t, ev[0], ev[1]);
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (st != PIMD_OK)
        return st;
    if (e != hipSuccess) {
        ctx->err = std::string("timing events: ") + hipGetErrorString(e);
        return PIMD_E_DEVICE;
    }
    ms = (double)t / n_reps;
    return read_status(ctx);
}

pimd_status pimd_autotune(pimd_ctx *ctx, int32_t n_reps, pimd_tuning *best)
{
    if (!ctx || n_reps < 1)
        return PIMD_E_ARG;
    if (!ctx->state_set) {
        ctx->err = "pimd_set_state must come before pimd_autotune";
        return PIMD_E_STATE;
    }
    if (ctx->pl.nl) {
        int n_cu = 0;
        HIPCHK(ctx, hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
        Tuning cur = ctx->tn, top = cur;
        double top_ms = 0.0;
        pimd_status st = time_forces(ctx, n_reps, top_ms);
        if (st != PIMD_OK)
            return st;
        auto consider = [&](const Tuning &cand) -> pimd_status {
            pimd_status s2 = apply_tuning(ctx, cand);
            double ms = 0.0;
            if (s2 == PIMD_OK)
                s2 = time_forces(ctx, n_reps, ms);
            if (s2 != PIMD_OK)
                return s2;
            if (ms < 0.99 * top_ms) {
                top = cand;
                top_ms = ms;
            }
            return PIMD_OK;
        };
        if (ctx->pl.small) {   // lane per centre against wave per centre, first: the rest tunes the winner
            Tuning cand = top;
            cand.centre_lanes = 1 - top.centre_lanes;
            if ((st = consider(cand)) != PIMD_OK)
                return st;
        }
        for (int waves : {4, 2, 1})
            for (int per_cu : {0, 2, 4, 8, 16}) {
                Tuning cand = top;
                cand.centre_waves = waves;
                cand.centre_grid = per_cu * n_cu;
                if (cand.centre_grid >= centre_grid(ctx->z.B, Tuning{waves, 0, 16, 0, 4, 0, 0}))
                    continue;   // no fewer workgroups than one wave per centre gives
                if (cand.centre_waves == cur.centre_waves && cand.centre_grid == cur.centre_grid)
                    continue;
                if ((st = consider(cand)) != PIMD_OK)
                    return st;
            }
        if (ctx->pl.bpnn && ctx->precision != PIMD_PREC_FP64_MLP)
            for (int rows : {16, 32, 64}) {
                if (rows == top.mlp_rows)
                    continue;
                Tuning cand = top;
                cand.mlp_rows = rows;
                if ((st = consider(cand)) != PIMD_OK)
                    return st;
            }
        if (ctx->pl.bpnn && (ctx->precision == PIMD_PREC_BF16_MLP || ctx->precision == PIMD_PREC_BF16_PLAIN)) {
            Tuning cand = top;
            cand.mlp_waves = 12 - top.mlp_waves;
            if ((st = consider(cand)) != PIMD_OK)
                return st;
        }
        if (chain_ok(ctx)) {
            const int other = 1 - top.mlp_chain;   // the other MLP kernel, at each tile size
            for (int rows : {16, 32, 64}) {
                Tuning cand = top;
                cand.mlp_chain = other;
                cand.mlp_rows = rows;
                if ((st = consider(cand)) != PIMD_OK)
                    return st;
            }
        }
        if (ctx->z.any_periodic) {
            Tuning cand = top;
            cand.nl_cells = 1 - top.nl_cells;
            if ((st = consider(cand)) != PIMD_OK)
                return st;
        }
        if (ctx->pl.bpnn) {
            Tuning cand = top;
            cand.force_rows = 1 - top.force_rows;
            if ((st = consider(cand)) != PIMD_OK)
                return st;
        }
        if ((st = apply_tuning(ctx, top)) != PIMD_OK)
            return st;
        // leave the forces of the current positions under the chosen shape
        if ((st = run_forces(ctx, ctx->d.q, ctx->d.E_bead, ctx->d.F, nullptr)) != PIMD_OK)
            return st;
        ctx->forces_valid = true;
        if ((st = read_status(ctx)) != PIMD_OK)
            return st;
    }
    return pimd_get_tuning(ctx, best ? best : &ctx->last_tuning_out);
}

pimd_status pimd_time_stages(pimd_ctx *ctx, int32_t n_reps, double *ms_host)
{
    if (!ctx || !ms_host || n_reps < 1)
        return PIMD_E_ARG;
    if (!ctx->state_set) {
        ctx->err = "state not set";
        return PIMD_E_STATE;
    }
    if (!ctx->pl.nl) {
        ctx->err = "stage timing needs a neural potential";
        return PIMD_E_STATE;
    }
    DevBuffers &d = ctx->d;
    pimd_status st = run_forces(ctx, d.q, d.E_bead, d.F, nullptr);
    if (st != PIMD_OK)
        return st;
    ctx->forces_valid = true;
    hipEvent_t ev[2];
    HIPCHK(ctx, hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        ctx->err = "hipEventCreate failed";
        return PIMD_E_DEVICE;
    }
    hipError_t e = hipSuccess;
    for (int k = 0; k < PIMD_N_FORCE_STAGES && e == hipSuccess; ++k) {
        (void)hipEventRecord(ev[0], ctx->stream);
        for (int r = 0; r < n_reps; ++r)
            launch_force_stage(ctx, k, d.q, d.E_bead, d.F, nullptr);
        (void)hipEventRecord(ev[1], ctx->stream);
        e = hipEventSynchronize(ev[1]);
        float ms = 0.0f;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, ev[0], ev[1]);
        ms_host[k] = (double)ms / n_reps;
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (ctx->pl.metad)
        ctx->forces_valid = false;   // the stage runs rewrote the forces without the bias
    if (e != hipSuccess) {
        ctx->err = std::string("stage timing: ") + hipGetErrorString(e);
        return PIMD_E_DEVICE;
    }
    CHECK_LAUNCH(ctx);
    return read_status(ctx);
}

pimd_status pimd_profile_stages(pimd_ctx *ctx, int32_t n_reps, double *ms_host)
{
    if (!ctx || !ms_host || n_reps < 1)
        return PIMD_E_ARG;
    if (!ctx->state_set) {
        ctx->err = "state not set";
        return PIMD_E_STATE;
    }
    if (!ctx->forces_valid) {
        pimd_status st = run_forces(ctx, ctx->d.q, ctx->d.E_bead, ctx->d.F, nullptr);
        if (st != PIMD_OK)
            return st;
        ctx->forces_valid = true;
    }
    {
        pimd_status st0 = reserve_steps(ctx, n_reps);
        if (st0 != PIMD_OK)
            return st0;
    }
    hipEvent_t ev[8];
    for (int k = 0; k < 8; ++k)
        HIPCHK(ctx, hipEventCreate(&ev[k]));
    double acc[PIMD_N_STAGES] = {0};
    pimd_status st = PIMD_OK;
    ctx->stage_ev = ev;
    for (int r = 0; r < n_reps && st == PIMD_OK; ++r) {
        st = run_step(ctx, ctx->stream, nullptr);
        if (st != PIMD_OK)
            break;
        hipError_t e = hipEventSynchronize(ev[7]);
        if (e != hipSuccess) {
            ctx->err = std::string("hipEventSynchronize: ") + hipGetErrorString(e);
            st = PIMD_E_DEVICE;
            break;
        }
        for (int k = 0; k < PIMD_N_STAGES; ++k) {
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
            acc[k] += ms;
        }
    }
    ctx->stage_ev = nullptr;
    for (int k = 0; k < 8; ++k)
        (void)hipEventDestroy(ev[k]);
    if (st != PIMD_OK)
        return st;
    for (int k = 0; k < PIMD_N_STAGES; ++k)
        ms_host[k] = acc[k] / n_reps;
    return read_status(ctx);
}

pimd_status pimd_work_counts(pimd_ctx *ctx, int64_t *pairs, int64_t *triplets, int64_t *triplets_in_range)
{
    if (!ctx || !pairs || !triplets || !triplets_in_range)
        return PIMD_E_ARG;
    if (!ctx->pl.nl) {
        ctx->err = "no neighbour list for this potential";
        return PIMD_E_STATE;
    }
    // the counters use the (otherwise idle until the next step) integrator partial-sum buffer
    unsigned long long *cnt = reinterpret_cast<unsigned long long *>(ctx->d.est_cols);
    const unsigned long long zero3[3] = {0, 0, 0};
    HIPCHK(ctx, hipMemcpyAsync(cnt, zero3, sizeof(zero3), hipMemcpyHostToDevice, ctx->stream));
    launch_work_counts(ctx->d, ctx->z, ctx->dp, cnt, ctx->stream);
    CHECK_LAUNCH(ctx);
    unsigned long long h[3];
    HIPCHK(ctx, hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    *pairs = (int64_t)h[0];
    *triplets = (int64_t)h[1];
    *triplets_in_range = (int64_t)h[2];
    return PIMD_OK;
}

pimd_status pimd_neighbor_rebuilds(pimd_ctx *ctx, int64_t *builds, int64_t *full_scans)
{
    if (!ctx || !builds || !full_scans)
        return PIMD_E_ARG;
    if (!ctx->z.skin) {
        ctx->err = "no shared neighbour lists (neighbor_skin_A is 0)";
        return PIMD_E_STATE;
    }
    unsigned long long h[2] = {0, 0};
    HIPCHK(ctx, hipMemcpyAsync(h, ctx->d.skin_builds, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    *builds = (int64_t)h[0];
    *full_scans = (int64_t)h[1];
    return PIMD_OK;
}

pimd_status pimd_sizes(const pimd_ctx *ctx, int64_t *bead_atoms, int64_t *beads, int32_t *features)
{
    if (!ctx)
        return PIMD_E_ARG;
    if (bead_atoms)
        *bead_atoms = ctx->z.B;
    if (beads)
        *beads = ctx->z.n_beads_total;
    if (features)
        *features = ctx->z.D;
    return PIMD_OK;
}

void pimd_destroy(pimd_ctx *ctx)
{
    if (!ctx)
        return;
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->gexec)
        (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph)
        (void)hipGraphDestroy(ctx->graph);
    if (ctx->capture)
        (void)hipStreamDestroy(ctx->capture);
    if (ctx->static_device >= 0) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        g_static_busy[ctx->static_device] = false;
    }
    delete ctx;
}

}  // extern "C"
