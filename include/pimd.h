/*
 * pimd.h -- C ABI of the MI355X ring-polymer (path-integral) MD library.
 *
 * The calls follow the paper's statement of the problem (Sec. 2.1 and 2.3):
 * a system (coordinates, masses, periodic box) is wrapped with a potential
 * that returns energies and forces, a normal-mode PIMD integrator with a
 * Langevin thermostat advances it, and finite-P estimators are read back
 * (the estimator of Sec. 2.1; the virial kinetic energy of the bead test in
 * Sec. S3).  The potential is a Behler-Parrinello symmetry-function network
 * (the descriptor family named in the Introduction) whose forces come from a
 * hand-written adjoint of the energy (the energy-model route of Sec. 2.2), or
 * an isotropic harmonic well (the oscillator of Sec. S1).
 *
 * Units: Angstrom, fs, amu, eV; momenta in amu*A/fs.
 *
 * Layout of every per-bead-atom array ("state layout"): float32 [B][3] with
 * B = sum_s P_s N_s; system s occupies the rows off_s .. off_s + P_s N_s - 1
 * (off_s = sum_{t<s} P_t N_t), bead k of system s starts at off_s + k N_s and
 * lists its N_s atoms in input order.  Per-bead arrays have sum_s P_s rows,
 * system-major then bead.
 *
 * Memory and threads: pointers named *_dev are device pointers on the
 * device that was current at pimd_init; the caller owns them.  The library
 * owns no device memory: every internal buffer lives in the caller's
 * workspace (pimd_workspace_size bytes, 256-byte aligned), which must stay
 * valid until pimd_destroy.  All device work is enqueued on the stream given
 * to pimd_init (the caller's, e.g. torch's current stream) and runs
 * asynchronously unless a call says it synchronises.  A context is not
 * thread-safe; separate contexts are independent.
 *
 * Errors: every call returns a pimd_status and never aborts.  Arguments are
 * checked on the host before any HIP call, so argument errors need no GPU.
 * Faults found on the device (neighbour overflow, non-finite energy or
 * forces) are latched in a device status word and returned by the next
 * synchronising call; pimd_last_error gives a message.
 */
#ifndef PIMD_H
#define PIMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pimd_ctx pimd_ctx;

typedef enum {
    PIMD_OK = 0,
    PIMD_E_ARG = 1,          /* invalid argument (null pointer, bad size or value)       */
    PIMD_E_UNSUPPORTED = 2,  /* valid but outside what the library implements            */
    PIMD_E_DEVICE = 3,       /* a HIP runtime call failed                                  */
    PIMD_E_OOM = 4,          /* the workspace is smaller than pimd_workspace_size           */
    PIMD_E_CAPACITY = 5,     /* an atom had more than max_neighbors neighbours              */
    PIMD_E_NONFINITE = 6,    /* an energy, force or state value became NaN or infinite      */
    PIMD_E_STATE = 7         /* call out of order (e.g. pimd_step before pimd_set_state)    */
} pimd_status;

/* MLP GEMM operand precision (accumulation is FP32 except in FP64_MLP):
 *   FP32        FP32 operands;
 *   BF16_MLP    BF16 operands in a three-term split (a_hi b_hi + a_lo b_hi + a_hi b_lo,
 *               every part bfloat16), about FP32 accuracy;
 *   BF16_PLAIN  BF16 operands rounded once (one product per tile);
 *   FP64_MLP    FP64 operands, activations and accumulation (FP64 MFMA).
 * Descriptors, adjoint and integrator are FP32 in every mode. */
enum { PIMD_PREC_FP32 = 0, PIMD_PREC_BF16_MLP = 1, PIMD_PREC_BF16_PLAIN = 2, PIMD_PREC_FP64_MLP = 3 };
enum { PIMD_POT_BPNN = 0, PIMD_POT_HARMONIC = 1, PIMD_POT_GFN = 2 };
enum { PIMD_ANGULAR_G4 = 0, PIMD_ANGULAR_G5 = 1 };

/*
 * Behler-Parrinello model.  Symmetry functions of centre atom i with
 * neighbours N(i) = { j : |d_ij| < cutoff } (d_ij the minimum-image vector
 * q_j - q_i), f_c(r) = (cos(pi r / cutoff) + 1) / 2:
 *   radial   G[e*n_rad + s] = sum_{j, Z_j = e} exp(-rad_eta[s] (r_ij - rad_center[s])^2) f_c(r_ij)
 *   angular  G[n_el*n_rad + pair*n_ang + (ie*4 + iz)*2 + il]
 *            = 2^(1-zeta) sum_{j<k, {Z_j,Z_k} = pair} (1 + lambda cos theta_jik)^zeta
 *              exp(-ang_eta[ie] (r_ij^2 + r_ik^2 + r_jk^2)) f_c(r_ij) f_c(r_ik) f_c(r_jk)
 *   with zeta = {1,2,4,8}[iz], lambda = {+1,-1}[il], r_jk = |d_ik - d_ij|,
 *   pair = lexicographic index of (min(Z_j,Z_k), max(Z_j,Z_k)), n_ang = 8*n_ang_eta,
 *   D = n_el*n_rad + n_el*(n_el+1)/2 * n_ang features.
 * angular = PIMD_ANGULAR_G5 drops the two factors of r_jk from the angular
 *   sum (the G5 form): exp(-ang_eta[ie] (r_ij^2 + r_ik^2)) f_c(r_ij) f_c(r_ik),
 *   every pair of neighbours counting; same layout.  The library then sums it
 *   through 81 spherical-harmonic moments per (element, eta) of each centre,
 *   O(K) per atom instead of O(K^2).
 * Network per element e: x = (G - feat_shift[e]) / feat_scale[e];
 *   h_l = tanh(W_l h_{l-1} + b_l) for the n_hidden hidden layers, E_i = w_o . h + b_o.
 * params: for each element in order, for each layer (hidden layers, then the
 *   output layer with one output): W [out][in] row-major, then b [out]; float32.
 * All arrays are host pointers, copied during pimd_init.
 */
typedef struct {
    int32_t n_elements;          /* 1..4 */
    const double *mass_amu;      /* [n_elements] */
    double cutoff_A;             /* > 0; below half of every periodic box length */
    int32_t n_rad;               /* 1..32, n_elements*n_rad <= 64 */
    const double *rad_center_A;  /* [n_rad] */
    const double *rad_eta;       /* [n_rad] 1/A^2 */
    int32_t n_ang_eta;           /* 1 or 2 */
    const double *ang_eta;       /* [n_ang_eta] 1/A^2 */
    int32_t n_hidden;            /* 1..3 */
    int32_t hidden[3];           /* widths, multiples of 16, <= 128 */
    const float *params;         /* packed weights, see above */
    const float *feat_shift;     /* [n_elements][D] */
    const float *feat_scale;     /* [n_elements][D], non-zero */
    int32_t angular;             /* PIMD_ANGULAR_G4 (0) or PIMD_ANGULAR_G5 (1); PIMD_E_ARG otherwise */
} pimd_bpnn_model;

/*
 * Direct-force head in the form of the graph field network of Sec. 2.2:
 * forces are an edge property, read out from edge representations that
 * exchange messages with node representations; there is no energy (bead
 * energies and V_bar are reported as 0, the virial as 0).  Width H (16 or
 * 32), L = n_layers (1..3), tanh activations, phi(x) = W2 tanh(W1 x + b1) + b2:
 *   rho_s(r)   = exp(-rad_eta_s (r - rad_center_s)^2) f_c(r),  f_c = (cos(pi r/rc) + 1)/2
 *   n_i^(0)    = node_embed[Z_i]
 *   e_ij^(0)   = edge_in rho(r_ij) + pair_embed[Z_i][Z_j]          (pair_embed symmetric)
 *   m_i^(l)    = sum_{j in N(i)} phi_msg^(l)(e_ij^(l))
 *   n_i^(l+1)  = n_i^(l) + phi_node^(l)([n_i^(l); m_i^(l)])
 *   e_ij^(l+1) = e_ij^(l) + phi_edge^(l)(n_i^(l) + n_j^(l))
 *   F_i        = sum_{j in N(i)} f_c(r_ij) (q_j - q_i)/r_ij (w2 . tanh(W1 e_ij^(L) + b1) + b2)
 * params, float32 row-major, in this order: node_embed [n_el][H],
 * pair_embed [n_el][n_el][H], edge_in [H][n_rad]; per layer phi_msg (W1 [H][H],
 * b1 [H], W2 [H][H], b2 [H]), phi_node (W1 [H][2H], b1, W2 [H][H], b2), phi_edge
 * (W1 [H][H], b1, W2, b2); then the readout W1 [H][H], b1 [H], w2 [H], b2 [1].
 * The neighbour lists are those of the energy model (same cutoff rules).
 */
typedef struct {
    int32_t n_elements;          /* 1..4 */
    const double *mass_amu;      /* [n_elements] */
    double cutoff_A;             /* < half of every box length */
    int32_t n_rad;               /* 1..32 */
    const double *rad_center_A;  /* [n_rad] */
    const double *rad_eta;       /* [n_rad] 1/A^2 */
    int32_t width;               /* H: 16 or 32 */
    int32_t n_layers;            /* 1..3 */
    const float *params;         /* packed weights, see above */
} pimd_gfn_model;

/*
 * Well-tempered metadynamics on bead collective variables (Sec. 2.5; the CVs
 * of Sec. 3.1 and Sec. 3.2).  Every bead k of every system carries its own
 * bias, a sum of Gaussian hills deposited at that bead's own CV values:
 *   V^(k)(s) = sum_h height_h exp(-(s - center_h)^2 / (2 sigma^2)),
 * added to that bead's potential (bias force -dV^(k)/ds * ds/dq on the bead's
 * atoms, added to the forces the integrator uses; bead energies stay the
 * potential's).  After every `stride` completed steps each bead deposits a
 * hill at its current CV s^(k) with height
 *   height0 * exp(-V^(k)(s^(k)) / (k_B T (bias_factor - 1)))
 * (T the system's temperature, V^(k) before the new hill; the forces of that
 * step use the bias before the hill).  The free-energy surface of a system
 * is the path-integral reweighting over its beads (pimd_metad_fes).
 * Collective variables of one bead (the same definition for every system):
 *   PIMD_CV_DISTANCES  s = sum_m coef[m] |q_atoms[2m] - q_atoms[2m+1]|  (A;
 *                      minimum image in a box; atom indices within the bead,
 *                      below every system's atom count), e.g. the double
 *                      proton transfer coordinate of Sec. 3.1
 *   PIMD_CV_XRD        S = (1/N) sum_i sum_j f_i f_j sin(Q R_ij) / (Q R_ij),
 *                      over all ordered pairs including i = j (term 1),
 *                      R_ij the minimum-image distance in a box, f_i =
 *                      form_factor[element of i] (the X-ray intensity CV of
 *                      Sec. 3.2)
 * All arrays are host pointers, copied during pimd_init.
 */
enum { PIMD_CV_DISTANCES = 1, PIMD_CV_XRD = 2 };
typedef struct {
    int32_t cv;                  /* PIMD_CV_* */
    int32_t n_terms;             /* DISTANCES: 1..64 */
    const int32_t *atoms;        /* DISTANCES: [n_terms][2] */
    const double *coef;          /* DISTANCES: [n_terms] */
    double q_scatter;            /* XRD: Q > 0 (1/A) */
    const double *form_factor;   /* XRD: [n_elements] */
    double height0_eV;           /* >= 0 */
    double sigma;                /* > 0, CV units */
    double bias_factor;          /* > 1; infinity: every hill has height0 */
    int32_t stride;              /* >= 1 steps between depositions */
    int32_t max_hills;           /* >= 1 hills kept per bead; pimd_step refuses to pass it */
} pimd_metad;

/*
 * Ring polymers.  n_systems independent systems, each with its own atom
 * count, bead count (1 or even, <= 128), temperature and orthorhombic box.
 * Integrator: normal-mode PIMD with the PILE-L thermostat in the splitting
 * O(dt/2) B(dt/2) A(dt) [forces] B(dt/2) O(dt/2); the ring polymer is sampled
 * as exp(-beta H_P / P) with springs of frequency w_P = P k_B T / hbar on
 * physical masses; mode k has w_k = 2 w_P sin(k pi / P) (normal-mode matrix
 * columns: 1/sqrt(P); sqrt(2/P) cos(2 pi j k/P) for 0<k<P/2; (-1)^j/sqrt(P);
 * sqrt(2/P) sin(2 pi j k/P) for k>P/2).  Friction gamma_0 = 1/tau0,
 * gamma_k = 2 pile_lambda w_k; tau0_fs <= 0 switches the thermostat off (NVE).
 * Thermostat noise: Philox4x32-10 with key = seed, counter = (row index of
 * (system, mode, atom) in the state layout, half (0 before / 1 after the
 * force), step lo, step hi), words u = (x + 1/2) 2^-32, Box-Muller on
 * (u0,u1) -> x, y and (u2,u3) -> z.
 */
/* Ring-polymer coordinates of the integrator (Sec. 2.1 names both):
 *   NORMAL_MODES  as above; the state momenta are Cartesian bead momenta.
 *   STAGING       u_1 = r_1, u_l = r_l - ((l-1) r_{l+1} + r_1)/l (l = 2..P,
 *                 r_{P+1} = r_1); springs sum_{l>=2} 1/2 m_l' w_P^2 u_l^2 with
 *                 m_l' = l m/(l-1); kinetic masses P m for u_1 and P m_l' for
 *                 u_l (the staging masses of the V/P form, times P in this
 *                 bead-potential form), so every u_l (l >= 2) turns at
 *                 w_P/sqrt(P) in the exact A step; friction 1/tau0 on u_1 and
 *                 2 pile_lambda w_P/sqrt(P) on the others.  The state momenta
 *                 (pimd_set_state, pimd_get_state) are the staging momenta, row
 *                 of bead l - 1 holding the momentum of u_l; K_beads and
 *                 T_beads use the kinetic masses.
 *   PRIMITIVE     Cartesian beads (Sec. 2.3 "primitive PIMD"): the springs are
 *                 forces -m w_P^2 (2 q_k - q_{k+1} - q_{k-1}) added in both B
 *                 steps, A is a free drift, O a friction 1/tau0 on every bead
 *                 (velocity Verlet on H_P: keep 2 w_P dt well below 2). */
enum { PIMD_TRANSFORM_NORMAL_MODES = 0, PIMD_TRANSFORM_STAGING = 1, PIMD_TRANSFORM_PRIMITIVE = 2 };

/* Thermostat of the normal-mode integrator (the PILE family of Table S3):
 *   PILE_L  Langevin friction on every mode: gamma_0 = 1/tau0 on the centroid,
 *           gamma_k = 2 pile_lambda w_k on the others.
 *   PILE_G  the same on the non-centroid modes; the centroid of every system
 *           is rescaled as a whole, once per half step, by the stochastic
 *           velocity rescaling of Bussi, Donadio and Parrinello (J. Chem. Phys.
 *           126, 014101 (2007)) with time constant tau0 towards the canonical
 *           centroid kinetic energy 3N k_B T P / 2: with K the centroid kinetic
 *           energy and c = exp(-(dt/2)/tau0),
 *             alpha^2 = c + (Kbar/(3N K))(1 - c)(R_1^2 + S) + 2 R_1 sqrt(c (1 - c) Kbar/(3N K)),
 *             sign(alpha) = sign(R_1 + sqrt(3N K c / ((1 - c) Kbar))),
 *           R_1 the thermostat normal of (centroid mode, atom 0, x) and S the
 *           sum of squares of the system's other 3N - 1 centroid normals (the
 *           same Philox counters as PILE-L, or the injected noise).  Normal
 *           modes only (PIMD_E_UNSUPPORTED with staging or primitive). */
enum { PIMD_THERMOSTAT_PILE_L = 0, PIMD_THERMOSTAT_PILE_G = 1 };

typedef struct {
    int32_t n_systems;                 /* >= 1 */
    const int32_t *n_atoms;            /* [n_systems], >= 1 */
    const int32_t *n_beads;            /* [n_systems], 1 or even, <= 128 */
    const double *temperature_K;       /* [n_systems], > 0 */
    const double *box_A;               /* [n_systems][3]; (0,0,0) = non-periodic */
    const int32_t *species;            /* [sum n_atoms], 0 <= Z < n_elements */
    double dt_fs;                      /* > 0 */
    double tau0_fs;                    /* centroid friction time; <= 0 => NVE */
    double pile_lambda;                /* >= 0 */
    uint64_t seed;                     /* Philox key */
    int32_t precision;                 /* PIMD_PREC_* (MLP GEMM operand precision) */
    int32_t potential;                 /* PIMD_POT_* */
    const pimd_bpnn_model *model;      /* PIMD_POT_BPNN: the model; HARMONIC: masses only */
    double harmonic_omega_per_fs;      /* PIMD_POT_HARMONIC: V = sum 1/2 m w^2 |q|^2 */
    int32_t max_neighbors;             /* neighbour slots per atom: 0 => 128; a multiple of 16, <= 256 */
    const pimd_gfn_model *gfn;         /* PIMD_POT_GFN: the direct-force head; FP32 and FP64_MLP run its
                                          per-edge products on the float32 vector ALU, BF16_MLP and
                                          BF16_PLAIN on BF16 MFMA (split or single operands) */
    const pimd_metad *metad;           /* well-tempered metadynamics bias, or NULL for none */
    int32_t transform;                 /* PIMD_TRANSFORM_* (0: normal modes) */
    double neighbor_skin_A;            /* 0: every bead's neighbour list searched through cell lists each
                                          force evaluation; > 0: one list per atom of the ring-polymer
                                          centroids with the cutoff widened by this skin, 3 * max_neighbors
                                          slots, rebuilt when a bead-atom is more than half the skin from its
                                          atom's centroid of the last build, filtered per bead each
                                          evaluation (the same lists, key for key).  Needs a box for every
                                          system (PIMD_E_UNSUPPORTED otherwise); a full centroid list is
                                          PIMD_E_CAPACITY like a full bead list */
    int32_t thermostat;                /* PIMD_THERMOSTAT_* (0: PILE-L) */
} pimd_config;

/* Finite-P estimators of one system (Sec. 2.1; virial kinetic energy of
 * Sec. S3), eV except T_beads (K):
 *   V_bar  = sum_k V(q^k) / P
 *   E_spring = sum_k sum_i 1/2 m_i w_P^2 |q_i^{k+1} - q_i^k|^2
 *   K_prim = 3NP/(2 beta) - E_spring / P
 *   K_cv   = 3N/(2 beta) - 1/(2P) sum_k sum_i (q_i^k - qbar_i) . F_i^k
 *   K_beads = sum |p|^2 / (2m),  T_beads = 2 K_beads / (3 N P k_B)  (-> P T)
 *   heat_bath = -(sum of kinetic-energy changes made by every O step)
 *   H_conserved = K_beads + E_spring + sum_k V(q^k) + heat_bath
 *   P_cv   = (2 K_cv + (1/P) sum_k tr W^(k)) / (3 V)  (eV/A^3), the centroid-virial
 *            pressure of a system with a box of volume V: scaling the box and the
 *            centroids while every bead keeps its offset from its centroid
 *            leaves the springs unchanged, so P_cv V - N k_B T is minus the
 *            strain derivative of (1/P) sum_k V(q^k) (the NPT estimator of
 *            Sec. 2.1's bead averages); W^(k) the virial of bead k as in
 *            pimd_energy_forces.  0 without a box and with the direct-force head
 *            (no energy, no virial)
 * With a metadynamics bias the forces, and so K_cv, are those of the biased
 * ring (P_cv uses the unbiased virial); H_conserved leaves the (time-dependent)
 * bias out. */
typedef struct {
    double V_bar, K_prim, K_cv, E_spring, K_beads, T_beads, H_conserved, heat_bath;
    double V_bias;   /* sum_k V^(k)(s^(k)) / P, the metadynamics bias (0 without one) */
    double P_cv;     /* centroid-virial pressure, eV/A^3 */
} pimd_estimates;

/* Bytes of device workspace a context needs for cfg.  No GPU needed. */
pimd_status pimd_workspace_size(const pimd_config *cfg, size_t *bytes);

/* Validate cfg, carve the workspace and upload tables and weights: the
 * system (coordinates come with pimd_set_state), its potential and the
 * integrator settings, the parts the paper wraps together before running
 * (Sec. 2.3, Charts 1 and 2; ring polymer and normal modes of Sec. 2.1;
 * PILE-L of Table S3).
 * workspace_dev: device memory of ws_bytes (>= pimd_workspace_size), 256-byte
 * aligned, owned by the caller.  hip_stream: a hipStream_t (NULL = default).
 * On success *out holds a new context; the state must be set with
 * pimd_set_state before pimd_step. */
pimd_status pimd_init(const pimd_config *cfg, void *workspace_dev, size_t ws_bytes,
                      void *hip_stream, pimd_ctx **out);

/* Allocation-free pimd_init, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same as pimd_init, with the workspace taken from a static
 * device array of PIMD_STATIC_WORKSPACE_BYTES inside the library instead of
 * the caller's memory: each device the library runs on holds its own array
 * until the process ends.  The call allocates no device memory (no hipMalloc,
 * hipFree, stream or graph creation; the context itself is host memory, as
 * for pimd_init).
 * Errors: PIMD_E_CAPACITY (nothing set up) when pimd_workspace_size(cfg)
 * exceeds the array; PIMD_E_STATE while another context made by this call
 * lives on the current device -- one such context per device at a time, since
 * two would share the array (pimd_destroy releases it); PIMD_E_DEVICE when the
 * array's device address cannot be obtained.  The array keeps the last
 * context's contents: like pimd_init on uninitialised memory, this call writes
 * every table, counter and flag the kernels read before they read it. */
#define PIMD_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
pimd_status pimd_init_static(const pimd_config *cfg, void *hip_stream, pimd_ctx **out);

/* Replace the stream later calls enqueue on. */
pimd_status pimd_set_stream(pimd_ctx *ctx, void *hip_stream);

/* Copy positions and momenta (state layout, device) into the context and set
 * the step counter; forces are evaluated at the first pimd_step. */
pimd_status pimd_set_state(pimd_ctx *ctx, const float *q_dev, const float *p_dev, int64_t step);

/* Copy positions, momenta (state layout; either may be NULL) and optionally
 * the forces of the current positions (forces_dev, NULL to skip) out of the
 * context.  Synchronises; returns a latched device fault, if any. */
pimd_status pimd_get_state(pimd_ctx *ctx, float *q_dev, float *p_dev, float *forces_dev, int64_t *step);

/* Heat bath of every system (heat_host[n_systems], eV: minus the kinetic
 * energy the thermostat's O steps have added since pimd_set_state, the term
 * that makes H_conserved conserved).  pimd_set_state zeroes it; a checkpoint
 * carries it with pimd_get_heat_bath and puts it back with
 * pimd_set_heat_bath after pimd_set_state.  Both synchronise; set takes
 * finite values only (PIMD_E_ARG). */
pimd_status pimd_get_heat_bath(pimd_ctx *ctx, double *heat_host);
pimd_status pimd_set_heat_bath(pimd_ctx *ctx, const double *heat_host);

/* Synchronise the context stream and return a latched device fault, if any,
 * clearing it.  A fault latched during a step freezes the integrator: that
 * step and every later one enqueued before this call leave positions,
 * momenta, step counter, heat bath and hills as they were after the last step
 * that completed without a fault, so a caller can read that state back
 * (pimd_get_state), rebuild the context (e.g. with more max_neighbors) and
 * replay the lost steps.  The forces are evaluated again at the next step.
 * Every synchronising call that reports faults does the same. */
pimd_status pimd_check(pimd_ctx *ctx);

/* Potential energy of every bead at positions q_dev (state layout), with
 * forces as minus the gradient of the energy (the energy-model route of
 * Sec. 2.2, here a descriptor network of the family the Introduction
 * cites, differentiated by a hand-written adjoint) -- the bead potentials
 * V(r^(k)) of the effective Hamiltonian of Sec. 2.1:
 * energy_dev[sum P_s] (eV); forces_dev [B][3] = -dE/dq (eV/A) or NULL for
 * energy only; virial_dev [sum P_s][9] (row-major W_ab = -sum_i sum_j
 * d_ij,a dE_i/dd_ij,b, eV) or NULL.  The integrator state is not touched.
 * Asynchronous. */
pimd_status pimd_energy_forces(pimd_ctx *ctx, const float *q_dev, float *energy_dev,
                               float *forces_dev, float *virial_dev);

/* Advance every system by n_steps full integrator steps (one force
 * evaluation each): normal-mode (or staging, or primitive) ring-polymer
 * dynamics of Sec. 2.1 and Sec. 2.3 under the PILE-L thermostat of Table S3,
 * all beads of all systems in one batch.  After the first step the step is replayed as a captured
 * HIP graph.  With metadynamics, PIMD_E_CAPACITY (nothing run) when the
 * steps would deposit more than max_hills hills per bead.  Asynchronous. */
pimd_status pimd_step(pimd_ctx *ctx, int32_t n_steps);

/* Estimators of the current state for every system (out_host[n_systems]):
 * the finite-P bead averages of Sec. 2.1 and the virial kinetic energy used
 * for the bead-convergence check of Sec. S3 (definitions at pimd_estimates).
 * Synchronises; returns a latched device fault, if any. */
pimd_status pimd_estimators(pimd_ctx *ctx, pimd_estimates *out_host);

/* Metadynamics (pimd_config.metad non-NULL; else PIMD_E_STATE).
 *
 * pimd_bias_forces: CV (cv_dev[sum P_s], double), bias energy (bias_dev
 *   [sum P_s], double, eV) and bias forces (forces_dev [B][3] float32, eV/A,
 *   overwritten) of every bead at positions q_dev with the current hills;
 *   any output may be NULL.  No deposition, the state is not touched.
 *   Asynchronous.
 * pimd_metad_cv: CV and bias energy of every bead at the current state
 *   (cv_host, bias_host [sum P_s], either may be NULL), as the last force
 *   evaluation of the state saw them.  Synchronises.
 * pimd_metad_hills: hills deposited so far per bead (*n_hills of them):
 *   center_host, height_host [sum P_s][*n_hills] (either may be NULL to
 *   query the count).  Synchronises.
 * pimd_metad_set_hills: replaces every bead's hills (restart):
 *   center_host, height_host [sum P_s][n_hills], 0 <= n_hills <= max_hills.
 *   The forces of the state are re-evaluated at the next step.  Synchronises.
 * pimd_metad_fes: quantum free-energy surface of system `system` on a grid
 *   s_host[n_grid] (Sec. 2.5 reweighting): F^(k)(s) = -(gamma/(gamma-1)) V^(k)(s),
 *   F(s) = -k_B T ln[(1/P) sum_k exp(-F^(k)(s) / k_B T)] -> fes_host[n_grid]
 *   (eV).  Synchronises. */
pimd_status pimd_bias_forces(pimd_ctx *ctx, const float *q_dev, float *forces_dev, double *cv_dev,
                             double *bias_dev);
pimd_status pimd_metad_cv(pimd_ctx *ctx, double *cv_host, double *bias_host);
pimd_status pimd_metad_hills(pimd_ctx *ctx, double *center_host, double *height_host, int32_t *n_hills);
pimd_status pimd_metad_set_hills(pimd_ctx *ctx, int32_t n_hills, const double *center_host,
                                 const double *height_host);
pimd_status pimd_metad_fes(pimd_ctx *ctx, int32_t system, int32_t n_grid, const double *s_host,
                           double *fes_host);

/* Timing of the bias pass (CV kernels, bias, bias forces; no deposition) at
 * the current positions: n_reps passes back to back between two HIP events
 * on the context stream after one untimed pass; *ms_host = mean milliseconds
 * per pass.  The forces of the state are re-evaluated at the next step.
 * Synchronises. */
pimd_status pimd_time_bias(pimd_ctx *ctx, int32_t n_reps, double *ms_host);

/* Test hook: the next pimd_step uses xi_dev ([2][B][3] float32 normals:
 * half 0 then half 1, rows indexed like the Philox counter) instead of
 * Philox for its two O steps.  The buffer is copied at this call. */
pimd_status pimd_inject_noise(pimd_ctx *ctx, const float *xi_dev);

/* Debug: neighbour list of global bead `bead` from the last force
 * evaluation, as (i, j) pairs of atom indices within the bead, sorted by
 * (i, j): ij_host[2*cap].  Synchronises. */
pimd_status pimd_debug_neighbors(pimd_ctx *ctx, int32_t bead, int32_t *ij_host, int64_t cap,
                                 int64_t *count);

/* Debug: normalised descriptors of the last force evaluation, [B][D]
 * float32 (device).  BPNN only. */
pimd_status pimd_debug_descriptors(pimd_ctx *ctx, float *xhat_dev);

/* Debug: copy an internal buffer of the last force evaluation to dst_dev
 * (device memory of at least the buffer's size, else PIMD_E_ARG):
 *   PIMD_BUF_XHAT   [B][D] float32 normalised descriptors
 *   PIMD_BUF_DEDG   [B][D] float32 dE/dG
 *   PIMD_BUF_SLOTS  [B][max_neighbors][4] float32 slot vectors dE_i/d d_ij (xyz, 0)
 *   PIMD_BUF_NBR    [B][max_neighbors] int32 neighbour keys (element << 27 | row)
 *   PIMD_BUF_NCOUNT [B] int32 neighbour counts
 *   PIMD_BUF_EATOM  [B] float32 atomic energies */
enum { PIMD_BUF_XHAT = 0, PIMD_BUF_DEDG = 1, PIMD_BUF_SLOTS = 2, PIMD_BUF_NBR = 3, PIMD_BUF_NCOUNT = 4,
       PIMD_BUF_EATOM = 5 };
pimd_status pimd_debug_copy(pimd_ctx *ctx, int32_t buffer, void *dst_dev, size_t bytes);

/* Debug: Philox words of the thermostat for (step, half): words_dev[n][4]
 * uint32 for counter rows 0..n-1. */
pimd_status pimd_debug_philox(pimd_ctx *ctx, int64_t step, int32_t half, int64_t n, uint32_t *words_dev);

/* Launch mode of pimd_step: enabled = 1 (default) replays the step as a
 * captured HIP graph; 0 enqueues every kernel of every step one by one. */
pimd_status pimd_set_graph(pimd_ctx *ctx, int32_t enabled);

/* Launch shapes of the force kernels.  Many ring polymers and beads run as
 * one flat batch (the concurrent-trajectory parallelism of Sec. 2.3 and the
 * multi-trajectory point of Sec. 4); these fields only change how that batch
 * is cut into workgroups, never the results (centre_lanes and mlp_chain aside, below):
 * each centre atom is one wave and each MLP row runs the same MFMA chain
 * whatever the shape.
 *   centre_waves  waves (one centre atom each) per workgroup of the neighbour,
 *                 descriptor, adjoint and force-assembly kernels: 1, 2 or 4
 *                 (default 4)
 *   centre_grid   0 (default): one wave per centre atom; > 0: at most this
 *                 many workgroups, whose waves stride over the centres
 *   mlp_rows      rows per MLP workgroup tile: 16, 32 or 64 (default 16
 *                 with the chained BF16 MLP, 32 with the other BF16 MLP, else
 *                 16); PIMD_PREC_FP64_MLP takes 16 only
 *   neighbor_cells  periodic neighbour search: 0 = one wave per centre
 *                 gathering its stencil from global memory, 1 = one workgroup
 *                 per cell with the stencil staged in LDS once for all of the
 *                 cell's centres (default 1 from 4096 cells on, else 0)
 *   mlp_waves     waves per workgroup of the BF16 MLP: 4 (two 16-column
 *                 tiles of every layer each) or 8 (default; one each, so each
 *                 row tile's chain of MFMAs is half as long); the FP32 and
 *                 FP64 MLPs ignore it
 *   force_rows    energy network only: 1 = the adjoint also stores each
 *                 slot value v[i][n] at the slot where atom j = nbr[i][n]
 *                 keeps the pair, and the force assembly reads two contiguous
 *                 rows per atom (default with a box); 0 = the assembly looks
 *                 the reverse slot up itself (default without).  The forces
 *                 are bitwise the same
 *   centre_lanes  G4 energy network on molecules without a box of at most 16
 *                 atoms each (else 0 only, PIMD_E_UNSUPPORTED): 1 (default
 *                 there) = one lane per centre atom, each wave taking whole
 *                 beads (as many as fit in 64 lanes), the neighbour lists
 *                 written by the descriptor kernel and the forces assembled in
 *                 the adjoint from the partners' lanes; 0 = one wave per centre
 *                 as above.  The two differ in summation order only (results
 *                 agree to rounding, not bitwise); every other field leaves
 *                 the results of either bitwise unchanged
 *   mlp_chain     BF16 precisions and the network shapes the chained kernel
 *                 is built for (65 to 96 features, a multiple of 4, with
 *                 hidden widths 128-128-64 or 64-64; else 0 only,
 *                 PIMD_E_UNSUPPORTED): 1 (default there) = one wave per 16
 *                 MLP rows with the activations kept in registers between
 *                 layers (each GEMM taken transposed, weights as the MFMA A
 *                 operand in a packed order); 0 = activations staged in LDS,
 *                 mlp_waves waves splitting the output columns.  The two sum
 *                 the MFMA products in another order (results agree to
 *                 rounding, not bitwise); within each, every other field
 *                 leaves the results bitwise unchanged */
typedef struct {
    int32_t centre_waves;
    int32_t centre_grid;
    int32_t mlp_rows;
    int32_t neighbor_cells;
    int32_t mlp_waves;
    int32_t force_rows;
    int32_t centre_lanes;
    int32_t mlp_chain;
} pimd_tuning;

pimd_status pimd_get_tuning(const pimd_ctx *ctx, pimd_tuning *out);

/* Applies a launch shape (PIMD_E_ARG for a value outside the lists above,
 * PIMD_E_UNSUPPORTED for mlp_rows != 16 in FP64-MLP mode) and drops the
 * captured step graph, which the next pimd_step captures again.
 * Synchronises. */
pimd_status pimd_set_tuning(pimd_ctx *ctx, const pimd_tuning *t);

/* Autotuner: times the force evaluation of the current positions (n_reps
 * evaluations per candidate after one untimed one, HIP events on the context
 * stream) for every centre_waves x centre_grid candidate (centre_grid from 0
 * and 2, 4, 8, 16 workgroups per compute unit), then for every mlp_rows
 * candidate with the best centre shape, then for the other neighbor_cells
 * value (systems with a box), then for the other mlp_waves (BF16 MLP), then
 * for the other force_rows (energy network); applies
 * the fastest (a candidate
 * replaces the current best only when at least 1% faster) and writes it to
 * best (may be NULL).  The state does not advance; the forces left behind are
 * those of the current positions.  Needs pimd_set_state first
 * (PIMD_E_STATE); with the harmonic potential there is nothing to tune and
 * the current shape is returned.  Synchronises. */
pimd_status pimd_autotune(pimd_ctx *ctx, int32_t n_reps, pimd_tuning *best);

/* Stage timing: runs n_reps integrator steps with the kernels enqueued one
 * by one, records HIP events between the stages on the context stream and
 * writes the mean milliseconds per step of each stage to
 * ms_host[PIMD_N_STAGES] in this order: integrate (before the force),
 * neighbour search (wrap, cells, lists), descriptors, MLP, adjoint, force
 * assembly with bead sums, integrate (after the force) with the step
 * bookkeeping.  Advances the state by n_reps steps.  Synchronises. */
#define PIMD_N_STAGES 7
pimd_status pimd_profile_stages(pimd_ctx *ctx, int32_t n_reps, double *ms_host);

/* Kernel timing without launch gaps (neural potential only): for each force
 * stage in the order neighbour search (wrap, cells, lists), descriptors,
 * MLP, adjoint, force assembly with bead sums, enqueues the stage n_reps
 * times back to back between two HIP events on the context stream and writes
 * the mean milliseconds of one run to ms_host[PIMD_N_FORCE_STAGES].  Each
 * stage rereads what the stage before it wrote for the current positions,
 * so the state does not advance and the forces left behind are those of the
 * current positions.  PIMD_E_STATE before pimd_set_state or with the
 * harmonic potential.  Synchronises. */
#define PIMD_N_FORCE_STAGES 5
pimd_status pimd_time_stages(pimd_ctx *ctx, int32_t n_reps, double *ms_host);

/* Work of the last force evaluation (BPNN): neighbour pairs (i, j), j<k
 * neighbour pairs of every centre (triplets) and the triplets with
 * r_jk < cutoff.  Synchronises. */
pimd_status pimd_work_counts(pimd_ctx *ctx, int64_t *pairs, int64_t *triplets, int64_t *triplets_in_range);

/* Shared neighbour lists (neighbor_skin_A > 0): how many times the centroid
 * lists have been built since pimd_init (the first force evaluation builds
 * them), and how many force evaluations found a bead farther than half the
 * skin from its fresh centroid (a ring wider than the skin) and tested every
 * atom of the bead instead.  PIMD_E_STATE without a skin.  Synchronises. */
pimd_status pimd_neighbor_rebuilds(pimd_ctx *ctx, int64_t *builds, int64_t *full_scans);

/* Sizes of a configured context: total bead-atoms B, total beads, features D. */
pimd_status pimd_sizes(const pimd_ctx *ctx, int64_t *bead_atoms, int64_t *beads, int32_t *features);

const char *pimd_last_error(const pimd_ctx *ctx);  /* ctx may be NULL: last init error */
const char *pimd_status_str(pimd_status s);
void pimd_destroy(pimd_ctx *ctx);                   /* synchronises; NULL is a no-op */

#ifdef __cplusplus
}
#endif
#endif /* PIMD_H */
