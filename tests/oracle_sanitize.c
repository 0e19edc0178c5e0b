/* Host sanitizer driver for the CPU oracle (test infrastructure): compiles
 * the oracle's translation unit together with this driver under
 * AddressSanitizer and UndefinedBehaviorSanitizer and runs every entry point
 * on small clustered inputs with coincident particles, a few cell scales
 * and the predictor-corrector step.  Prints "ok" and a checksum. */
#include "../oracle/oracle.c"

#include <stdio.h>

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double urand(void)       /* SplitMix64 -> [0, 1) */
{
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1p-53;
}

int main(void)
{
    const int64_t ng = 700, nh = 300, n = ng + nh;
    double *x = malloc(n * sizeof(double)), *y = malloc(n * sizeof(double));
    double *z = malloc(n * sizeof(double)), *m = malloc(n * sizeof(double));
    double *vx = malloc(n * sizeof(double)), *vy = malloc(n * sizeof(double));
    double *vz = malloc(n * sizeof(double)), *e = malloc(ng * sizeof(double));
    double *h = malloc(ng * sizeof(double));
    for (int64_t i = 0; i < n; i++) {
        double r = pow(urand(), 2.0) * 3.0;
        double u = 2.0 * urand() - 1.0, ph = 6.283185307179586 * urand();
        double s = sqrt(1.0 - u * u);
        x[i] = r * s * cos(ph);
        y[i] = r * s * sin(ph);
        z[i] = r * u;
        m[i] = (0.5 + urand()) / (double)n;
        vx[i] = 0.1 * (urand() - 0.5);
        vy[i] = 0.1 * (urand() - 0.5);
        vz[i] = 0.1 * (urand() - 0.5);
        if (i < ng) {
            e[i] = 0.02 + 0.06 * urand();
            h[i] = 0.05 + 0.1 * r + 0.01 * urand();
        }
    }
    for (int k = 0; k < 12; k++) {        /* coincident gas particles */
        x[100 + k] = x[5];
        y[100 + k] = y[5];
        z[100 + k] = z[5];
    }
    double check = 0.0;
    for (int scale = -1; scale <= 1; scale++) {
        or_grid_t g;
        if (or_grid(ng, x, y, z, h, scale, &g) != 0) {
            printf("grid failed\n");
            return 1;
        }
        int32_t *key = malloc(ng * sizeof(int32_t)), *lev = malloc(ng * sizeof(int32_t));
        or_keys(ng, x, y, z, h, &g, key, lev);
        int32_t *count = malloc((size_t)g.M * sizeof(int32_t)), *perm = malloc(ng * sizeof(int32_t));
        int64_t *coff = malloc(((size_t)g.M + 1) * sizeof(int64_t));
        double *hmax = malloc((size_t)g.M * sizeof(double));
        or_count_sort(ng, g.M, key, h, count, coff, hmax, perm);
        check += (double)coff[g.M] + (double)perm[ng / 2];
        free(key); free(lev); free(count); free(perm); free(coff); free(hmax);
    }
    int64_t *off = malloc((ng + 1) * sizeof(int64_t));
    or_nbrs_brute(ng, x, y, z, h, off, NULL);
    int32_t *idx = malloc((size_t)(off[ng] > 0 ? off[ng] : 1) * sizeof(int32_t));
    or_nbrs_brute(ng, x, y, z, h, off, idx);
    /* rows again from all-pairs candidates, and one brute row */
    int64_t *cand_off = malloc((ng + 1) * sizeof(int64_t));
    int32_t *cand = malloc((size_t)ng * ng * sizeof(int32_t));
    int64_t w = 0;
    cand_off[0] = 0;
    for (int64_t i = 0; i < ng; i++) {
        for (int64_t j = 0; j < ng; j++)
            if (j != i) cand[w++] = (int32_t)j;
        cand_off[i + 1] = w;
    }
    int64_t *off2 = malloc((ng + 1) * sizeof(int64_t));
    or_nbrs_from_candidates(ng, x, y, z, h, cand_off, cand, off2, NULL);
    int32_t *idx2 = malloc((size_t)(off2[ng] > 0 ? off2[ng] : 1) * sizeof(int32_t));
    or_nbrs_from_candidates(ng, x, y, z, h, cand_off, cand, off2, idx2);
    int32_t row[256];
    int64_t rl = or_nbr_row_brute(ng, x, y, z, h, 5, row, 256);
    if (off2[ng] != off[ng] || rl != off[6] - off[5]) {
        printf("row mismatch\n");
        return 1;
    }
    or_grid_t g0;
    or_grid(ng, x, y, z, h, 0, &g0);
    int32_t *key = malloc(ng * sizeof(int32_t));
    or_keys(ng, x, y, z, h, &g0, key, NULL);
    int32_t *count = malloc((size_t)g0.M * sizeof(int32_t)), *perm = malloc(ng * sizeof(int32_t));
    int64_t *coff = malloc(((size_t)g0.M + 1) * sizeof(int64_t));
    double *hmax = malloc((size_t)g0.M * sizeof(double));
    or_count_sort(ng, g0.M, key, h, count, coff, hmax, perm);
    int64_t *soff = malloc((ng + 1) * sizeof(int64_t));
    soff[0] = 0;
    for (int64_t s = 0; s < ng; s++) soff[s + 1] = soff[s] + (off[perm[s] + 1] - off[perm[s]]);
    int32_t *sidx = malloc((size_t)(off[ng] > 0 ? off[ng] : 1) * sizeof(int32_t));
    or_rows_to_slots(ng, perm, off, idx, soff, sidx);

    double *rho = malloc(ng * sizeof(double)), *p = malloc(ng * sizeof(double));
    double *c = malloc(ng * sizeof(double));
    or_density(ng, x, y, z, m, h, off, idx, rho);
    or_eos(ng, 5.0 / 3.0, rho, e, p, c);
    double *ax = calloc(n, sizeof(double)), *ay = calloc(n, sizeof(double));
    double *az = calloc(n, sizeof(double)), *de = calloc(n, sizeof(double));
    or_sph_force(ng, x, y, z, vx, vy, vz, m, h, rho, e, 5.0 / 3.0, 1.0, 2.0, 0.1, off, idx,
                 ax, ay, az, de);
    int64_t *tgt = malloc(n * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) tgt[i] = i;
    double *gx = malloc(n * sizeof(double)), *gy = malloc(n * sizeof(double));
    double *gz = malloc(n * sizeof(double)), *pot = malloc(n * sizeof(double));
    or_gravity(n, x, y, z, m, 1.0, 0.01, n, tgt, gx, gy, gz, pot);
    for (int64_t i = 0; i < n; i++) {
        ax[i] += gx[i];
        ay[i] += gy[i];
        az[i] += gz[i];
    }
    double dt = or_cfl_dt(ng, x, y, z, vx, vy, vz, h, c, ax, ay, az, de, 0.5, 1.0, 2.0, 0.1, off, idx);
    double *vtx = malloc(n * sizeof(double)), *vty = malloc(n * sizeof(double));
    double *vtz = malloc(n * sizeof(double)), *et = malloc(ng * sizeof(double));
    or_predict(n, ng, 1e-3, x, y, z, vx, vy, vz, e, ax, ay, az, de, vtx, vty, vtz, et);
    or_correct(n, ng, 1e-3, vx, vy, vz, e, vtx, vty, vtz, et, ax, ay, az, de);
    double diag[10];
    or_diagnostics(n, ng, x, y, z, vx, vy, vz, m, e, pot, diag);
    or_update_h(ng, 1.25, m, rho, h);
    for (int k = 0; k < 10; k++) check += diag[k];
    check += rho[7] + ax[3] + de[11] + pot[n - 1] + (dt < 1e300 ? dt : 0.0) + h[9] + (double)sidx[0];
    printf("ok %.17g levels %d cells %lld pairs %lld\n", check, or_max_levels(),
           (long long)g0.M, (long long)off[ng]);
    free(x); free(y); free(z); free(m); free(vx); free(vy); free(vz); free(e); free(h);
    free(off); free(idx); free(cand_off); free(cand); free(off2); free(idx2);
    free(key); free(count); free(perm); free(coff); free(hmax); free(soff); free(sidx);
    free(rho); free(p); free(c); free(ax); free(ay); free(az); free(de); free(tgt);
    free(gx); free(gy); free(gz); free(pot); free(vtx); free(vty); free(vtz); free(et);
    return 0;
}
