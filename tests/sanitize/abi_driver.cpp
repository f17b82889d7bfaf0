// Host-side driver of the C-ABI validation and set-up code, built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host pass only.
// Every call returns before the first device operation (argument errors) or
// fails at it (no GPU where this runs), so everything it exercises is host
// code: argument checks, workspace layout, and pimd_init's table building
// (neighbour cells, normal-mode matrices, integrator units, MLP tiles and
// packed weights, metadynamics work items), which runs before the device is
// touched.  Exit status 0 when every call returned the status expected.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "pimd.h"

namespace {

int g_fail = 0;

void expect(const char *what, pimd_status got, pimd_status want)
{
    if (got != want) {
        std::printf("FAIL %s: status %d (%s), expected %d\n", what, (int)got, pimd_status_str(got), (int)want);
        ++g_fail;
    } else {
        std::printf("ok   %s: %s\n", what, pimd_status_str(got));
    }
}

struct Bpnn {
    std::vector<double> mass{1.008, 15.999}, rc, re, ae{0.005, 0.02};
    std::vector<float> params, shift, scale;
    pimd_bpnn_model m{};
    Bpnn(int angular)
    {
        const int n_el = 2, n_rad = 16, D = n_el * n_rad + 3 * 16;
        for (int s = 0; s < n_rad; ++s) {
            rc.push_back(0.8 + s * 4.7 / (n_rad - 1));
            re.push_back(1.0 / (2.0 * std::pow(4.7 / (n_rad - 1), 2)));
        }
        const int widths[5] = {D, 128, 128, 64, 1};
        for (int e = 0; e < n_el; ++e)
            for (int l = 0; l < 4; ++l)
                for (int k = 0; k < widths[l] * widths[l + 1] + widths[l + 1]; ++k)
                    params.push_back(0.01f * (float)((k * 7919 + l * 31 + e) % 101 - 50));
        shift.assign((size_t)n_el * D, 0.0f);
        scale.assign((size_t)n_el * D, 2.0f);
        m.n_elements = n_el;
        m.mass_amu = mass.data();
        m.cutoff_A = 6.0;
        m.n_rad = n_rad;
        m.rad_center_A = rc.data();
        m.rad_eta = re.data();
        m.n_ang_eta = 2;
        m.ang_eta = ae.data();
        m.n_hidden = 3;
        m.hidden[0] = 128;
        m.hidden[1] = 128;
        m.hidden[2] = 64;
        m.params = params.data();
        m.feat_shift = shift.data();
        m.feat_scale = scale.data();
        m.angular = angular;
    }
};

struct Gfn {
    std::vector<double> mass{1.008, 15.999}, rc, re;
    std::vector<float> params;
    pimd_gfn_model g{};
    Gfn()
    {
        const int n_el = 2, n_rad = 8, H = 16, L = 2;
        for (int s = 0; s < n_rad; ++s) {
            rc.push_back(0.8 + s * 0.6);
            re.push_back(1.4);
        }
        size_t n = (size_t)n_el * H + (size_t)n_el * n_el * H + (size_t)H * n_rad;
        const size_t mlp_hh = 2 * (size_t)H * H + 2 * H;
        n += L * (mlp_hh + (2 * (size_t)H * H + (size_t)H * H + 2 * H) + mlp_hh);
        n += (size_t)H * H + H + H + 1;
        for (size_t k = 0; k < n; ++k)
            params.push_back(0.02f * (float)((k * 104729) % 97 - 48));
        g.n_elements = n_el;
        g.mass_amu = mass.data();
        g.cutoff_A = 6.0;
        g.n_rad = n_rad;
        g.rad_center_A = rc.data();
        g.rad_eta = re.data();
        g.width = H;
        g.n_layers = L;
        g.params = params.data();
    }
};

// Two systems: 24 atoms in a 12.5 A box with 8 beads, and a 10-atom molecule
// without a box with 4 beads (or both periodic, for the shared lists).
struct Systems {
    std::vector<int32_t> n_atoms{24, 10}, n_beads{8, 4}, species;
    std::vector<double> T{300.0, 250.0}, box{12.5, 12.5, 12.5, 0.0, 0.0, 0.0};
    Systems(bool both_periodic)
    {
        if (both_periodic)
            box[3] = box[4] = box[5] = 13.0;
        for (int i = 0; i < 34; ++i)
            species.push_back(i % 3 == 0 ? 1 : 0);
    }
};

pimd_config base(const Systems &S)
{
    pimd_config c{};
    c.n_systems = 2;
    c.n_atoms = S.n_atoms.data();
    c.n_beads = S.n_beads.data();
    c.temperature_K = S.T.data();
    c.box_A = S.box.data();
    c.species = S.species.data();
    c.dt_fs = 0.25;
    c.tau0_fs = 100.0;
    c.pile_lambda = 1.0;
    c.seed = 4242;
    return c;
}

// workspace size, then pimd_init on a fake (never dereferenced) aligned
// workspace: the host tables are built and the first device call fails
void init_without_gpu(const char *what, const pimd_config &c)
{
    size_t bytes = 0;
    const pimd_status s = pimd_workspace_size(&c, &bytes);
    expect(what, s, PIMD_OK);
    if (s != PIMD_OK)
        return;
    pimd_ctx *ctx = nullptr;
    void *fake = reinterpret_cast<void *>((uintptr_t)1 << 40);
    const pimd_status st = pimd_init(&c, fake, bytes, nullptr, &ctx);
    if (st != PIMD_E_DEVICE && st != PIMD_OK) {
        std::printf("FAIL %s: pimd_init returned %s (%s)\n", what, pimd_status_str(st), pimd_last_error(nullptr));
        ++g_fail;
    }
    if (ctx)
        pimd_destroy(ctx);
}

}  // namespace

int main()
{
    Bpnn g4(0), g5(1);
    Gfn gfn;
    Systems mixed(false), boxed(true);
    for (int prec : {PIMD_PREC_FP32, PIMD_PREC_BF16_MLP, PIMD_PREC_BF16_PLAIN, PIMD_PREC_FP64_MLP}) {
        pimd_config c = base(mixed);
        c.model = &g4.m;
        c.precision = prec;
        init_without_gpu("bpnn G4", c);
    }
    {
        pimd_config c = base(mixed);
        c.model = &g5.m;
        init_without_gpu("bpnn G5", c);
        c.model = &g4.m;
        c.thermostat = PIMD_THERMOSTAT_PILE_G;
        init_without_gpu("bpnn PILE-G", c);
        c.thermostat = PIMD_THERMOSTAT_PILE_L;
        c.transform = PIMD_TRANSFORM_STAGING;
        init_without_gpu("bpnn staging", c);
        c.transform = PIMD_TRANSFORM_NORMAL_MODES;
        c.max_neighbors = 192;
        init_without_gpu("bpnn 192 slots", c);
    }
    {
        pimd_config c = base(boxed);
        c.model = &g4.m;
        c.neighbor_skin_A = 2.0;
        init_without_gpu("bpnn shared lists", c);
        c.potential = PIMD_POT_GFN;
        c.gfn = &gfn.g;
        c.neighbor_skin_A = 0.0;
        init_without_gpu("direct-force head", c);
        c.precision = PIMD_PREC_BF16_MLP;
        init_without_gpu("direct-force head, MFMA", c);
    }
    {
        pimd_config c = base(mixed);
        c.model = &g4.m;
        pimd_metad md{};
        const int32_t atoms[4] = {0, 1, 2, 3};
        const double coef[2] = {1.0, -1.0};
        md.cv = PIMD_CV_DISTANCES;
        md.n_terms = 2;
        md.atoms = atoms;
        md.coef = coef;
        md.sigma = 0.05;
        md.height0_eV = 0.01;
        md.bias_factor = 10.0;
        md.stride = 10;
        md.max_hills = 64;
        c.metad = &md;
        init_without_gpu("metadynamics, distances", c);
        pimd_metad x{};
        const double ff[2] = {0.5, 6.0};
        x.cv = PIMD_CV_XRD;
        x.q_scatter = 1.69;
        x.form_factor = ff;
        x.sigma = 0.05;
        x.height0_eV = 0.01;
        x.bias_factor = 60.0;
        x.stride = 200;
        x.max_hills = 16;
        c.metad = &x;
        init_without_gpu("metadynamics, XRD", c);
    }
    {
        pimd_config c = base(mixed);
        c.model = &g4.m;
        c.potential = PIMD_POT_HARMONIC;
        c.harmonic_omega_per_fs = 0.01;
        init_without_gpu("harmonic", c);
    }
    // argument errors, all caught before any HIP call
    size_t bytes = 0;
    expect("NULL config", pimd_workspace_size(nullptr, &bytes), PIMD_E_ARG);
    {
        pimd_config c = base(mixed);
        c.model = &g4.m;
        c.dt_fs = -1.0;
        expect("negative dt", pimd_workspace_size(&c, &bytes), PIMD_E_ARG);
        c.dt_fs = 0.25;
        std::vector<int32_t> odd{24, 3};
        c.n_beads = odd.data();
        expect("odd bead count", pimd_workspace_size(&c, &bytes), PIMD_E_UNSUPPORTED);
        c.n_beads = mixed.n_beads.data();
        c.max_neighbors = 17;
        expect("slots not a multiple of 16", pimd_workspace_size(&c, &bytes), PIMD_E_ARG);
        c.max_neighbors = 0;
        c.thermostat = 5;
        expect("unknown thermostat", pimd_workspace_size(&c, &bytes), PIMD_E_ARG);
        c.thermostat = PIMD_THERMOSTAT_PILE_G;
        c.transform = PIMD_TRANSFORM_PRIMITIVE;
        expect("PILE-G with primitive beads", pimd_workspace_size(&c, &bytes), PIMD_E_UNSUPPORTED);
        c.thermostat = PIMD_THERMOSTAT_PILE_L;
        c.transform = PIMD_TRANSFORM_NORMAL_MODES;
        std::vector<double> small{10.0, 10.0, 10.0, 0.0, 0.0, 0.0};
        c.box_A = small.data();
        expect("cutoff beyond half the box", pimd_workspace_size(&c, &bytes), PIMD_E_UNSUPPORTED);
        c.box_A = mixed.box.data();
        pimd_ctx *ctx = nullptr;
        expect("NULL workspace", pimd_init(&c, nullptr, 1 << 20, nullptr, &ctx), PIMD_E_ARG);
        expect("misaligned workspace",
               pimd_init(&c, reinterpret_cast<void *>(((uintptr_t)1 << 40) + 8), (size_t)1 << 30, nullptr, &ctx),
               PIMD_E_ARG);
        expect("workspace too small", pimd_init(&c, reinterpret_cast<void *>((uintptr_t)1 << 40), 256, nullptr, &ctx),
               PIMD_E_OOM);
        // 3072 bead-atoms with 256 slots each: ~200 MB of triplet lists
        std::vector<int32_t> many{128, 4};
        c.n_beads = many.data();
        c.max_neighbors = 256;
        expect("static workspace too small", pimd_init_static(&c, nullptr, &ctx), PIMD_E_CAPACITY);
    }
    expect("NULL context step", pimd_step(nullptr, 1), PIMD_E_ARG);
    std::printf("%s\n", g_fail ? "FAILED" : "ALL OK");
    return g_fail ? 1 : 0;
}
