/* Exercises every function of the oracle's C part on small seeded inputs, for an
 * AddressSanitizer + UndefinedBehaviorSanitizer build (test infrastructure, CPU only).
 * Exits 0 when every call ran; the sanitizers abort on the first finding. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_morton_keys(int64_t n, const double *x, const double *y, const double *z, double L,
                     uint64_t *key);
void orc_merge_thresholds(double L, double R_lc, double b, double theta, double *T2);
double orc_a_min(int64_t n, const double *x, const double *y, const double *z,
                 const double *gx, const double *gy, const double *gz, double L,
                 const double *xobs, double Rb);
int64_t orc_coarsen(int64_t n, const double *x, const double *y, const double *z,
                    const double *px, const double *py, const double *pz,
                    const uint32_t *mult, const uint32_t *id, const uint8_t *type, double L,
                    const double *xobs, double R_lc, double b, double theta, int k_min,
                    int crit, double alpha, double Gm0, const double *gx, const double *gy,
                    const double *gz, double *a_min_out, double *ox, double *oy, double *oz,
                    double *opx, double *opy, double *opz, uint32_t *omult, uint32_t *oid,
                    uint8_t *otype, int64_t *group_of, int64_t *n_merged_nodes);
double orc_g_soft(double r, double h);
double orc_split_S(double u);
void orc_short_range(int64_t n, const double *x, const double *y, const double *z,
                     const uint32_t *mult, double L, double m0, double eps0, double G,
                     double r_s, double r_cut, int64_t n_targets, const int64_t *targets,
                     double *gx, double *gy, double *gz);
void orc_cic_deposit(int64_t n, const double *x, const double *y, const double *z,
                     const uint32_t *mult, double L, int ng, double m0, double *rho);
void orc_cic_interp(int64_t n, const double *x, const double *y, const double *z, double L,
                    int ng, const double *mesh, double *out);

static uint64_t state = 20050528u;
static double uniform(void) {   /* xorshift64*: inputs only */
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (double)((state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

int main(void) {
    const int64_t n = 3000;
    const double L = 100.0;
    double *x = malloc(sizeof(double) * n), *y = malloc(sizeof(double) * n),
           *z = malloc(sizeof(double) * n), *px = malloc(sizeof(double) * n),
           *py = malloc(sizeof(double) * n), *pz = malloc(sizeof(double) * n),
           *gx = malloc(sizeof(double) * n), *gy = malloc(sizeof(double) * n),
           *gz = malloc(sizeof(double) * n);
    uint32_t *mult = malloc(sizeof(uint32_t) * n), *id = malloc(sizeof(uint32_t) * n);
    uint8_t *type = malloc(n);
    for (int64_t i = 0; i < n; ++i) {
        x[i] = L * uniform();
        y[i] = L * uniform();
        z[i] = (i % 7 == 0) ? 0.0 : L * uniform();   /* some on a face */
        px[i] = uniform() - 0.5;
        py[i] = uniform() - 0.5;
        pz[i] = uniform() - 0.5;
        gx[i] = gy[i] = gz[i] = 0.0;
        mult[i] = 1u + (uint32_t)(8.0 * uniform());
        id[i] = (uint32_t)(n - 1 - i);
        type[i] = 0;
    }
    uint64_t *key = malloc(sizeof(uint64_t) * n);
    orc_morton_keys(n, x, y, z, L, key);
    double T2[22];
    orc_merge_thresholds(L, 20.0, 5.0, 1.0, T2);
    const double xo[3] = {0.0, 0.0, 0.0};
    const double r_s = 1.25 * L / 32, r_cut = 4.5 * r_s;
    orc_short_range(n, x, y, z, mult, L, 1.0, 0.1, 43.0091, r_s, r_cut, 0, NULL, gx, gy, gz);
    int64_t t[5] = {0, 17, 1234, 2000, n - 1};
    double tg[3][5];
    orc_short_range(n, x, y, z, mult, L, 1.0, 0.1, 43.0091, r_s, r_cut, 5, t, tg[0], tg[1], tg[2]);
    double am = orc_a_min(n, x, y, z, gx, gy, gz, L, xo, 25.0);
    double *ox = malloc(sizeof(double) * n), *oy = malloc(sizeof(double) * n),
           *oz = malloc(sizeof(double) * n), *opx = malloc(sizeof(double) * n),
           *opy = malloc(sizeof(double) * n), *opz = malloc(sizeof(double) * n);
    uint32_t *om = malloc(sizeof(uint32_t) * n), *oi = malloc(sizeof(uint32_t) * n);
    uint8_t *ot = malloc(n);
    int64_t *grp = malloc(sizeof(int64_t) * n), nm = 0;
    double amin = 0.0;
    int64_t nout = orc_coarsen(n, x, y, z, px, py, pz, mult, id, type, L, xo, 20.0, 5.0, 1.0, 2,
                               0, 0.0, 0.0, NULL, NULL, NULL, &amin, ox, oy, oz, opx, opy, opz,
                               om, oi, ot, grp, &nm);
    int64_t nout2 = orc_coarsen(n, x, y, z, px, py, pz, mult, id, type, L, xo, 20.0, 5.0, 0.0, 2,
                                1, 0.3, 43.0091, gx, gy, gz, &amin, ox, oy, oz, opx, opy, opz,
                                om, oi, ot, grp, &nm);
    const int ng = 32;
    double *rho = malloc(sizeof(double) * ng * ng * ng), *out = malloc(sizeof(double) * n);
    orc_cic_deposit(n, x, y, z, mult, L, ng, 1.0, rho);
    orc_cic_interp(n, x, y, z, L, ng, rho, out);
    double s = orc_g_soft(0.05, 0.28) + orc_g_soft(0.2, 0.28) + orc_g_soft(1.0, 0.28) +
               orc_split_S(0.0) + orc_split_S(4.5);
    printf("oracle driver: keys %llu, a_min %g, coarsened %lld and %lld, checksum %g\n",
           (unsigned long long)key[n - 1], am, (long long)nout, (long long)nout2,
           s + out[0] + tg[0][0]);
    free(x); free(y); free(z); free(px); free(py); free(pz); free(gx); free(gy); free(gz);
    free(mult); free(id); free(type); free(key); free(ox); free(oy); free(oz); free(opx);
    free(opy); free(opz); free(om); free(oi); free(ot); free(grp); free(rho); free(out);
    return 0;
}
