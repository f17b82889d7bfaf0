/*
 * Oracle (test infrastructure, not product code): plain FP64 CPU evaluation
 * of Behler-Parrinello symmetry functions and of their gradient with respect
 * to the neighbour displacement vectors.
 *
 * The paper names descriptor networks of the Behler-Parrinello family as the
 * established MLFF route (Introduction); its own energy model gets forces by
 * differentiating the energy with respect to the coordinates (Sec. 2.2).  The
 * functions below are the textbook definitions written out, with one loop
 * per sum and no blocking or reordering:
 *
 *   f_c(r)  = 0.5 (cos(pi r / R_c) + 1)          for r < R_c, else 0
 *   G2[e,s] = sum_{j in N(i), Z_j = e} exp(-eta_s (r_ij - R_s)^2) f_c(r_ij)
 *   G4[{e1,e2},(eta,zeta,lambda)] = 2^(1-zeta) sum_{j<k in N(i), {Z_j,Z_k} = {e1,e2}}
 *        (1 + lambda cos theta_jik)^zeta exp(-eta (r_ij^2 + r_ik^2 + r_jk^2))
 *        f_c(r_ij) f_c(r_ik) f_c(r_jk)
 *   with d_ij the minimum-image vector q_j - q_i, cos theta = d_ij.d_ik/(r_ij r_ik),
 *   r_jk = |d_ik - d_ij|, each unordered triplet counted once (j < k in the
 *   neighbour list order).
 *
 * angular = 1 selects the G5 form of the angular functions instead: the same
 * sum without the factors that involve r_jk,
 *   G5[{e1,e2},(eta,zeta,lambda)] = 2^(1-zeta) sum_{j<k in N(i), {Z_j,Z_k} = {e1,e2}}
 *        (1 + lambda cos theta_jik)^zeta exp(-eta (r_ij^2 + r_ik^2)) f_c(r_ij) f_c(r_ik)
 * so every pair of neighbours counts, however far apart j and k are.
 *
 * Feature layout: radial index e*n_rad + s; angular index
 * n_el*n_rad + pair*n_ang + (i_eta*4 + i_zeta)*2 + i_lambda, with zeta in
 * {1,2,4,8}, lambda in {+1,-1}, pair = lexicographic index of (e1 <= e2).
 *
 * Neighbour lists come in CSR form (start[c]..start[c+1]) from the caller.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

static const int ZETA[4] = {1, 2, 4, 8};
static const double LAMBDA[2] = {1.0, -1.0};

static double cutoff_fn(double r, double rc)
{
    return r < rc ? 0.5 * (cos(M_PI * r / rc) + 1.0) : 0.0;
}

static double cutoff_deriv(double r, double rc)
{
    return r < rc ? -0.5 * (M_PI / rc) * sin(M_PI * r / rc) : 0.0;
}

static double ipow(double x, int n)
{
    double y = 1.0;
    for (int t = 0; t < n; ++t)
        y *= x;
    return y;
}

static void displacement(const double *q, int i, int j, const double *box, int periodic, double d[3])
{
    for (int c = 0; c < 3; ++c) {
        d[c] = q[3 * j + c] - q[3 * i + c];
        if (periodic)
            d[c] -= box[c] * nearbyint(d[c] / box[c]);
    }
}

static int pair_index(int a, int b, int n_el)
{
    int e1 = a < b ? a : b, e2 = a < b ? b : a;
    return e1 * n_el - e1 * (e1 - 1) / 2 + (e2 - e1);
}

static double norm3(const double d[3])
{
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

int oracle_n_features(int n_el, int n_rad, int n_ang_eta)
{
    return n_el * n_rad + (n_el * (n_el + 1) / 2) * n_ang_eta * 8;
}

/* G[c][D] for each centre c (atom centers[c]).  Also returns counts[c*2+0] =
 * number of j<k triplets and counts[c*2+1] = those with r_jk < R_c. */
void oracle_descriptors(int n_atoms, const double *q, const int32_t *species,
                        const double *box, int periodic,
                        int n_el, int n_rad, const double *rad_center, const double *rad_eta,
                        int n_ang_eta, const double *ang_eta, double rc,
                        int n_centers, const int32_t *centers,
                        const int64_t *nbr_start, const int32_t *nbr_idx,
                        double *G, int64_t *counts, int angular)
{
    (void)n_atoms;
    const int D = oracle_n_features(n_el, n_rad, n_ang_eta);
    const int n_ang = n_ang_eta * 8;
#pragma omp parallel for schedule(dynamic, 4)
    for (int c = 0; c < n_centers; ++c) {
        const int i = centers[c];
        double *g = G + (int64_t)c * D;
        memset(g, 0, sizeof(double) * D);
        const int32_t *nb = nbr_idx + nbr_start[c];
        const int K = (int)(nbr_start[c + 1] - nbr_start[c]);
        int64_t n_trip = 0, n_trip_in = 0;
        for (int a = 0; a < K; ++a) {
            const int j = nb[a];
            double d[3];
            displacement(q, i, j, box, periodic, d);
            const double r = norm3(d);
            const double f = cutoff_fn(r, rc);
            for (int s = 0; s < n_rad; ++s) {
                const double x = r - rad_center[s];
                g[species[j] * n_rad + s] += exp(-rad_eta[s] * x * x) * f;
            }
        }
        for (int a = 0; a < K; ++a) {
            const int j = nb[a];
            double dij[3];
            displacement(q, i, j, box, periodic, dij);
            const double rij = norm3(dij);
            for (int b = a + 1; b < K; ++b) {
                const int k = nb[b];
                double dik[3], djk[3];
                displacement(q, i, k, box, periodic, dik);
                for (int t = 0; t < 3; ++t)
                    djk[t] = dik[t] - dij[t];
                const double rik = norm3(dik), rjk = norm3(djk);
                ++n_trip;
                if (!angular && rjk >= rc)
                    continue;
                ++n_trip_in;
                const double cos_t = (dij[0] * dik[0] + dij[1] * dik[1] + dij[2] * dik[2]) / (rij * rik);
                const double fcs = angular ? cutoff_fn(rij, rc) * cutoff_fn(rik, rc)
                                           : cutoff_fn(rij, rc) * cutoff_fn(rik, rc) * cutoff_fn(rjk, rc);
                const double r2sum = angular ? rij * rij + rik * rik : rij * rij + rik * rik + rjk * rjk;
                const int base = n_el * n_rad + pair_index(species[j], species[k], n_el) * n_ang;
                for (int ie = 0; ie < n_ang_eta; ++ie) {
                    const double radial = exp(-ang_eta[ie] * r2sum) * fcs;
                    for (int iz = 0; iz < 4; ++iz)
                        for (int il = 0; il < 2; ++il) {
                            const double ang = pow(2.0, 1 - ZETA[iz]) * ipow(1.0 + LAMBDA[il] * cos_t, ZETA[iz]);
                            g[base + (ie * 4 + iz) * 2 + il] += ang * radial;
                        }
                }
            }
        }
        if (counts) {
            counts[2 * c] = n_trip;
            counts[2 * c + 1] = n_trip_in;
        }
    }
}

/* Vector-Jacobian product: given dEdG[c][D] = dE/dG for centre c, write
 * v[slot][3] = dE_c/d(d_{i,j}) for every neighbour slot of every centre
 * (same CSR layout as nbr_idx).  The caller turns slot vectors into forces
 * (dE/dq_j += v, dE/dq_i -= v) and the virial. */
void oracle_descriptor_vjp(int n_atoms, const double *q, const int32_t *species,
                           const double *box, int periodic,
                           int n_el, int n_rad, const double *rad_center, const double *rad_eta,
                           int n_ang_eta, const double *ang_eta, double rc,
                           int n_centers, const int32_t *centers,
                           const int64_t *nbr_start, const int32_t *nbr_idx,
                           const double *dEdG, double *v, int angular)
{
    (void)n_atoms;
    const int D = oracle_n_features(n_el, n_rad, n_ang_eta);
    const int n_ang = n_ang_eta * 8;
#pragma omp parallel for schedule(dynamic, 4)
    for (int c = 0; c < n_centers; ++c) {
        const int i = centers[c];
        const double *g = dEdG + (int64_t)c * D;
        const int32_t *nb = nbr_idx + nbr_start[c];
        double *vc = v + 3 * nbr_start[c];
        const int K = (int)(nbr_start[c + 1] - nbr_start[c]);
        memset(vc, 0, sizeof(double) * 3 * K);
        /* radial: G2 depends on r_ij only */
        for (int a = 0; a < K; ++a) {
            const int j = nb[a];
            double d[3];
            displacement(q, i, j, box, periodic, d);
            const double r = norm3(d);
            const double f = cutoff_fn(r, rc), df = cutoff_deriv(r, rc);
            double dEdr = 0.0;
            for (int s = 0; s < n_rad; ++s) {
                const double x = r - rad_center[s];
                const double e = exp(-rad_eta[s] * x * x);
                dEdr += g[species[j] * n_rad + s] * e * (-2.0 * rad_eta[s] * x * f + df);
            }
            for (int t = 0; t < 3; ++t)
                vc[3 * a + t] += dEdr * d[t] / r;
        }
        /* angular: each triplet depends on d_ij and d_ik */
        for (int a = 0; a < K; ++a) {
            const int j = nb[a];
            double A[3];
            displacement(q, i, j, box, periodic, A);
            const double rij = norm3(A);
            for (int b = a + 1; b < K; ++b) {
                const int k = nb[b];
                double B[3], C[3];
                displacement(q, i, k, box, periodic, B);
                for (int t = 0; t < 3; ++t)
                    C[t] = B[t] - A[t];
                const double rik = norm3(B), rjk = norm3(C);
                if (!angular && rjk >= rc)
                    continue;
                const double cos_t = (A[0] * B[0] + A[1] * B[1] + A[2] * B[2]) / (rij * rik);
                /* G5: the r_jk factor is 1 and its derivative 0 */
                const double fij = cutoff_fn(rij, rc), fik = cutoff_fn(rik, rc);
                const double fjk = angular ? 1.0 : cutoff_fn(rjk, rc);
                const double dfij = cutoff_deriv(rij, rc), dfik = cutoff_deriv(rik, rc);
                const double dfjk = angular ? 0.0 : cutoff_deriv(rjk, rc);
                const double eta_jk = angular ? 0.0 : 1.0;
                const int base = n_el * n_rad + pair_index(species[j], species[k], n_el) * n_ang;
                double S_c = 0.0, S_ij = 0.0, S_ik = 0.0, S_jk = 0.0;
                for (int ie = 0; ie < n_ang_eta; ++ie) {
                    const double eta = ang_eta[ie];
                    const double ex = exp(-eta * (rij * rij + rik * rik + eta_jk * rjk * rjk));
                    /* radial factor R = ex * fij * fik * fjk and its partials */
                    const double R = ex * fij * fik * fjk;
                    const double dR_dij = ex * fik * fjk * (-2.0 * eta * rij * fij + dfij);
                    const double dR_dik = ex * fij * fjk * (-2.0 * eta * rik * fik + dfik);
                    const double dR_djk = ex * fij * fik * (-2.0 * eta * eta_jk * rjk * fjk + dfjk);
                    for (int iz = 0; iz < 4; ++iz)
                        for (int il = 0; il < 2; ++il) {
                            const double w = g[base + (ie * 4 + iz) * 2 + il] * pow(2.0, 1 - ZETA[iz]);
                            const double base_t = 1.0 + LAMBDA[il] * cos_t;
                            const double T = ipow(base_t, ZETA[iz]);
                            const double dT = ZETA[iz] * LAMBDA[il] * ipow(base_t, ZETA[iz] - 1);
                            S_c += w * dT * R;
                            S_ij += w * T * dR_dij;
                            S_ik += w * T * dR_dik;
                            S_jk += w * T * dR_djk;
                        }
                }
                for (int t = 0; t < 3; ++t) {
                    const double dcos_dA = B[t] / (rij * rik) - cos_t * A[t] / (rij * rij);
                    const double dcos_dB = A[t] / (rij * rik) - cos_t * B[t] / (rik * rik);
                    vc[3 * a + t] += S_c * dcos_dA + S_ij * A[t] / rij - S_jk * C[t] / rjk;
                    vc[3 * b + t] += S_c * dcos_dB + S_ik * B[t] / rik + S_jk * C[t] / rjk;
                }
            }
        }
    }
}
