/* Driver of the oracle's C core built with AddressSanitizer and
 * UndefinedBehaviorSanitizer: descriptors and their vector-Jacobian product
 * of a small periodic water-like cluster and of an open molecule, for both
 * angular forms, with CSR neighbour lists built here by brute force.  Exit
 * status 0 when every output is finite and the sanitizers report nothing. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_n_features(int n_el, int n_rad, int n_ang_eta);
void oracle_descriptors(int n_atoms, const double *q, const int32_t *species, const double *box, int periodic,
                        int n_el, int n_rad, const double *rad_center, const double *rad_eta, int n_ang_eta,
                        const double *ang_eta, double rc, int n_centers, const int32_t *centers,
                        const int64_t *nbr_start, const int32_t *nbr_idx, double *G, int64_t *counts, int angular);
void oracle_descriptor_vjp(int n_atoms, const double *q, const int32_t *species, const double *box, int periodic,
                           int n_el, int n_rad, const double *rad_center, const double *rad_eta, int n_ang_eta,
                           const double *ang_eta, double rc, int n_centers, const int32_t *centers,
                           const int64_t *nbr_start, const int32_t *nbr_idx, const double *dEdG, double *v,
                           int angular);

static int run(int n, double L, int angular)
{
    const int n_el = 2, n_rad = 8, n_ang_eta = 2;
    const double rc = 6.0;
    double rad_center[8], rad_eta[8], ang_eta[2] = {0.005, 0.02};
    for (int s = 0; s < n_rad; ++s) {
        rad_center[s] = 0.8 + s * 0.7;
        rad_eta[s] = 1.0;
    }
    double box[3] = {L, L, L};
    const int periodic = L > 0.0;
    double *q = malloc(sizeof(double) * 3 * n);
    int32_t *species = malloc(sizeof(int32_t) * n), *centers = malloc(sizeof(int32_t) * n);
    unsigned s = 12345u;
    for (int i = 0; i < n; ++i) {
        for (int c = 0; c < 3; ++c) {
            s = s * 1103515245u + 12345u;
            q[3 * i + c] = (periodic ? L : 7.0) * (double)(s >> 8) / 16777216.0;
        }
        species[i] = i % 3 == 0 ? 1 : 0;
        centers[i] = i;
    }
    int64_t *start = malloc(sizeof(int64_t) * (n + 1));
    int32_t *idx = malloc(sizeof(int32_t) * n * n);
    int64_t m = 0;
    for (int i = 0; i < n; ++i) {
        start[i] = m;
        for (int j = 0; j < n; ++j) {
            if (j == i)
                continue;
            double r2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                double d = q[3 * j + c] - q[3 * i + c];
                if (periodic)
                    d -= L * rint(d / L);
                r2 += d * d;
            }
            if (r2 < rc * rc)
                idx[m++] = j;
        }
    }
    start[n] = m;
    const int D = oracle_n_features(n_el, n_rad, n_ang_eta);
    double *G = malloc(sizeof(double) * n * D), *g = malloc(sizeof(double) * n * D);
    int64_t *counts = malloc(sizeof(int64_t) * 2 * n);
    double *v = malloc(sizeof(double) * 3 * (m > 0 ? m : 1));
    oracle_descriptors(n, q, species, box, periodic, n_el, n_rad, rad_center, rad_eta, n_ang_eta, ang_eta, rc, n,
                       centers, start, idx, G, counts, angular);
    for (int k = 0; k < n * D; ++k)
        g[k] = 0.01 * (double)((k * 37) % 11 - 5);
    oracle_descriptor_vjp(n, q, species, box, periodic, n_el, n_rad, rad_center, rad_eta, n_ang_eta, ang_eta, rc,
                          n, centers, start, idx, g, v, angular);
    int bad = 0;
    for (int k = 0; k < n * D; ++k)
        bad += !isfinite(G[k]);
    for (int64_t k = 0; k < 3 * m; ++k)
        bad += !isfinite(v[k]);
    printf("n %d box %.1f angular %d: %lld slots, %d non-finite\n", n, L, angular, (long long)m, bad);
    free(q), free(species), free(centers), free(start), free(idx), free(G), free(g), free(counts), free(v);
    return bad;
}

int main(void)
{
    int bad = 0;
    for (int angular = 0; angular < 2; ++angular) {
        bad += run(24, 12.5, angular);
        bad += run(10, 0.0, angular);
    }
    printf("%s\n", bad ? "FAILED" : "ALL OK");
    return bad ? 1 : 0;
}
