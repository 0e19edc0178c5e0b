/*
 * oracle.c -- plain, slow, CPU FP64 reference of the SPH + direct-gravity
 * force evaluation of Khrapov & Khoperskov, "Smoothed-Particle Hydrodynamics
 * Models: Implementation Features on GPUs" (CCIS 793, 2017).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or constant with the HIP
 * library.
 *
 * Every function below follows one passage of the paper (cited by section and
 * equation) or, where the paper is silent, the reading written next to it.
 * Floating point is FP64 throughout, except the neighbour predicate, which is
 * defined in FP32 so that integer neighbour lists can be compared bit for bit.
 * Build with -O2 -fopenmp -ffp-contract=off and without fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846
#define OR_MAX_LEVELS 16

/* ------------------------------------------------------------------------ */
/* Smoothing kernels (Sec. 2.2)                                              */
/* ------------------------------------------------------------------------ */

/* Cubic spline of Eq. (SPH-Kernel): normalisation 1/(pi h^3), support 2h.
 * The two branches agree at xi = 1 and xi = 2, so no tie rule is needed. */
double or_W(double r, double h)
{
    double xi = r / h;
    double s = 1.0 / (OR_PI * h * h * h);
    if (xi <= 1.0)
        return s * (1.0 - 1.5 * xi * xi + 0.75 * xi * xi * xi);
    if (xi <= 2.0) {
        double t = 2.0 - xi;
        return s * 0.25 * t * t * t;
    }
    return 0.0;
}

/* Force kernel of Eq. (SPH-Kernel-p): 15/(64 pi h^3) (2 - xi)^3 on [0,2]. */
double or_Wp(double r, double h)
{
    double xi = r / h;
    if (xi >= 2.0)
        return 0.0;
    double t = 2.0 - xi;
    return 15.0 / (64.0 * OR_PI * h * h * h) * t * t * t;
}

/* dW_p/dxi obtained by differentiating Eq. (SPH-Kernel-p):
 * -45/(64 pi h^3) (2 - xi)^2.  (The limit printed after that equation
 * differs; the derivative of the printed kernel is taken as authoritative.) */
double or_dWp_dxi(double r, double h)
{
    double xi = r / h;
    if (xi >= 2.0)
        return 0.0;
    double t = 2.0 - xi;
    return -45.0 / (64.0 * OR_PI * h * h * h) * t * t;
}

/* ------------------------------------------------------------------------ */
/* Neighbour predicate                                                       */
/* ------------------------------------------------------------------------ */

/* j is an SPH neighbour of i when xi = |r_ij| / h_ij < 2 with
 * h_ij = (h_i + h_j)/2 (Sec. 2.2, after Eq. SPH-Kernel), i.e. |r_ij| < h_i+h_j.
 * To make integer neighbour lists reproducible bit for bit, the test is
 * carried out in FP32: each FP64 coordinate difference is rounded once to
 * FP32, r^2 = fma(dz,dz, fma(dy,dy, dx*dx)), cut = (float)h_i + (float)h_j,
 * and the pair qualifies iff r^2 < cut*cut.  The test is symmetric in i, j. */
int or_pred(double xi, double yi, double zi, double hi,
            double xj, double yj, double zj, double hj)
{
    float dx = (float)(xi - xj);
    float dy = (float)(yi - yj);
    float dz = (float)(zi - zj);
    float dxx = dx * dx;
    float r2 = fmaf(dz, dz, fmaf(dy, dy, dxx));
    float cut = (float)hi + (float)hj;
    float cut2 = cut * cut;
    return r2 < cut2;
}

/* ------------------------------------------------------------------------ */
/* Grid of cells (Sec. 3: M_x x M_y x M_z grid, CellSPH, hmaxCell)           */
/* ------------------------------------------------------------------------ */

/* The paper covers the domain with a grid of M cells and keeps per-cell
 * counts, inclusive prefix sums and the maximum smoothing length, but does
 * not give the cell size or the meaning of "hierarchical".  Reading used
 * here: a stack of uniform grids ("levels") whose cell sides are powers of
 * two, L_l = L_0 2^l, with L_0 the smallest power of two >= (2 + 2^-9) h_min;
 * a particle lives on the first level with L_l >= (2 + 2^-9) h_i.  Each
 * non-empty level spans the bounding box of its own particles, with origin
 * floor(min/L_l) L_l and M_d = floor((max - origin)/L_l) + 1 cells along d.
 * Cells are numbered level by level, then z, y, x (x fastest).  A cell-size
 * scale 2^s (s = cell_scale_log2 in {-1, 0, 1}, a tuning choice of the
 * search, not of the method) multiplies every cell side, L_l = L_0 2^(l+s),
 * while the level of each particle is still decided by L_0 2^l. */
typedef struct {
    double L0;
    int32_t nlev;                   /* levels 0..nlev-1 (some may be empty) */
    int32_t pad;
    double L[OR_MAX_LEVELS];
    double org[OR_MAX_LEVELS][3];
    int64_t dim[OR_MAX_LEVELS][3];
    int64_t base[OR_MAX_LEVELS];
    int64_t ncell[OR_MAX_LEVELS];
    int64_t npart[OR_MAX_LEVELS];
    double hmax[OR_MAX_LEVELS];
    int64_t M;
} or_grid_t;

static double or_pow2_ceil(double t)
{
    int e;
    double f = frexp(t, &e);        /* t = f 2^e, f in [0.5, 1) */
    if (f == 0.5)
        return t;
    return ldexp(1.0, e);
}

static int or_level_of(double h, double L0)
{
    double t = h * (2.0 + 0x1p-9);
    double L = L0;
    int l = 0;
    while (L < t) {
        L *= 2.0;
        l++;
        if (l >= OR_MAX_LEVELS)
            return -1;
    }
    return l;
}

/* Returns 0 on success, -1 if a level beyond OR_MAX_LEVELS is needed,
 * -2 if the cell count overflows 2^31-1, -3 on empty input. */
int or_grid(int64_t ng, const double *x, const double *y, const double *z,
            const double *h, int cell_scale_log2, or_grid_t *g)
{
    memset(g, 0, sizeof(*g));
    if (ng <= 0)
        return -3;
    double hmin = h[0];
    for (int64_t i = 1; i < ng; i++)
        if (h[i] < hmin)
            hmin = h[i];
    g->L0 = or_pow2_ceil(hmin * (2.0 + 0x1p-9));
    double lo[OR_MAX_LEVELS][3], hi[OR_MAX_LEVELS][3];
    for (int l = 0; l < OR_MAX_LEVELS; l++) {
        g->L[l] = ldexp(g->L0, l + cell_scale_log2);
        g->hmax[l] = 0.0;
        for (int d = 0; d < 3; d++) {
            lo[l][d] = INFINITY;
            hi[l][d] = -INFINITY;
        }
    }
    int maxl = 0;
    for (int64_t i = 0; i < ng; i++) {
        int l = or_level_of(h[i], g->L0);
        if (l < 0)
            return -1;
        if (l > maxl)
            maxl = l;
        double p[3] = {x[i], y[i], z[i]};
        for (int d = 0; d < 3; d++) {
            if (p[d] < lo[l][d]) lo[l][d] = p[d];
            if (p[d] > hi[l][d]) hi[l][d] = p[d];
        }
        if (h[i] > g->hmax[l])
            g->hmax[l] = h[i];
        g->npart[l]++;
    }
    g->nlev = maxl + 1;
    int64_t M = 0;
    for (int l = 0; l < g->nlev; l++) {
        g->base[l] = M;
        if (g->npart[l] == 0) {
            g->ncell[l] = 0;
            continue;
        }
        int64_t nc = 1;
        for (int d = 0; d < 3; d++) {
            double o = floor(lo[l][d] / g->L[l]) * g->L[l];
            g->org[l][d] = o;
            g->dim[l][d] = (int64_t)floor((hi[l][d] - o) / g->L[l]) + 1;
            nc *= g->dim[l][d];
            if (nc > INT32_MAX)
                return -2;
        }
        g->ncell[l] = nc;
        M += nc;
        if (M > INT32_MAX)
            return -2;
    }
    g->M = M;
    return 0;
}

/* Cell key of every particle (the role of indexPC[i].x in Sec. 3). */
void or_keys(int64_t ng, const double *x, const double *y, const double *z,
             const double *h, const or_grid_t *g, int32_t *key, int32_t *level)
{
    for (int64_t i = 0; i < ng; i++) {
        int l = or_level_of(h[i], g->L0);
        double p[3] = {x[i], y[i], z[i]};
        int64_t c[3];
        for (int d = 0; d < 3; d++) {
            int64_t v = (int64_t)floor((p[d] - g->org[l][d]) / g->L[l]);
            if (v < 0) v = 0;
            if (v > g->dim[l][d] - 1) v = g->dim[l][d] - 1;
            c[d] = v;
        }
        key[i] = (int32_t)(g->base[l] +
                           (c[2] * g->dim[l][1] + c[1]) * g->dim[l][0] + c[0]);
        if (level)
            level[i] = l;
    }
}

/* Counting sort by cell (Sec. 3, CellSPH / indexPC / hmaxCell): per-cell
 * count, exclusive offsets off[0..M] (off[k+1] is the paper's inclusive
 * CellSPH[k].y), per-cell maximum h (0 for an empty cell) and the slot ->
 * particle map.  Particles are placed in ascending id order, so the order
 * inside a cell is ascending id (the paper's atomic cursor leaves it
 * unspecified; a fixed order is chosen so that results are reproducible). */
void or_count_sort(int64_t ng, int64_t M, const int32_t *key, const double *h,
                   int32_t *count, int64_t *off, double *hmax, int32_t *perm)
{
    for (int64_t k = 0; k < M; k++) {
        count[k] = 0;
        hmax[k] = 0.0;
    }
    for (int64_t i = 0; i < ng; i++) {
        count[key[i]]++;
        if (h[i] > hmax[key[i]])
            hmax[key[i]] = h[i];
    }
    off[0] = 0;
    for (int64_t k = 0; k < M; k++)
        off[k + 1] = off[k] + count[k];
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(M > 0 ? M : 1));
    for (int64_t k = 0; k < M; k++)
        cur[k] = off[k];
    for (int64_t i = 0; i < ng; i++)
        perm[cur[key[i]]++] = (int32_t)i;
    free(cur);
}

/* ------------------------------------------------------------------------ */
/* Neighbour lists in particle-id space                                      */
/* ------------------------------------------------------------------------ */

/* Brute force over all pairs.  Count mode when idx == NULL (off[i+1]-off[i]
 * receives the row length, off[0] = 0 and off is made cumulative); fill mode
 * otherwise (rows ascending in j). */
void or_nbrs_brute(int64_t ng, const double *x, const double *y,
                   const double *z, const double *h, int64_t *off,
                   int32_t *idx)
{
    if (!idx) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < ng; i++) {
            int64_t c = 0;
            for (int64_t j = 0; j < ng; j++)
                if (j != i && or_pred(x[i], y[i], z[i], h[i], x[j], y[j], z[j], h[j]))
                    c++;
            off[i + 1] = c;
        }
        off[0] = 0;
        for (int64_t i = 0; i < ng; i++)
            off[i + 1] += off[i];
        return;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < ng; i++) {
        int64_t w = off[i];
        for (int64_t j = 0; j < ng; j++)
            if (j != i && or_pred(x[i], y[i], z[i], h[i], x[j], y[j], z[j], h[j]))
                idx[w++] = (int32_t)j;
    }
}

/* Brute-force row of a single particle i (used for sampled rows at sizes
 * where full brute force is too slow).  Returns the row length; writes at
 * most cap entries (ascending). */
int64_t or_nbr_row_brute(int64_t ng, const double *x, const double *y,
                         const double *z, const double *h, int64_t i,
                         int32_t *out, int64_t cap)
{
    int64_t c = 0;
    for (int64_t j = 0; j < ng; j++)
        if (j != i && or_pred(x[i], y[i], z[i], h[i], x[j], y[j], z[j], h[j])) {
            if (c < cap)
                out[c] = (int32_t)j;
            c++;
        }
    return c;
}

static int or_cmp_i32(const void *a, const void *b)
{
    int32_t u = *(const int32_t *)a, v = *(const int32_t *)b;
    return (u > v) - (u < v);
}

/* Exact rows from a candidate superset.  cand_off/cand_idx is any CSR in
 * which, for every true neighbour pair (i, j), j is listed under i or i is
 * listed under j (e.g. all j within 2 h_i (1 + 2^-10) of i: for a true pair
 * |r_ij| < h_i + h_j <= 2 max(h_i, h_j)).  The candidates are symmetrised,
 * de-duplicated, filtered by or_pred and written ascending.  Count mode when
 * idx == NULL, as in or_nbrs_brute. */
void or_nbrs_from_candidates(int64_t ng, const double *x, const double *y,
                             const double *z, const double *h,
                             const int64_t *cand_off, const int32_t *cand_idx,
                             int64_t *off, int32_t *idx)
{
    int64_t nc = cand_off[ng];
    int64_t *toff = (int64_t *)calloc((size_t)ng + 1, sizeof(int64_t));
    int32_t *tidx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
    for (int64_t e = 0; e < nc; e++)
        toff[cand_idx[e] + 1]++;
    for (int64_t i = 0; i < ng; i++)
        toff[i + 1] += toff[i];
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ng > 0 ? ng : 1));
    for (int64_t i = 0; i < ng; i++)
        cur[i] = toff[i];
    for (int64_t i = 0; i < ng; i++)
        for (int64_t e = cand_off[i]; e < cand_off[i + 1]; e++)
            tidx[cur[cand_idx[e]]++] = (int32_t)i;
    free(cur);
#pragma omp parallel
    {
        int64_t bufcap = 256;
        int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)bufcap);
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < ng; i++) {
            int64_t n = (cand_off[i + 1] - cand_off[i]) + (toff[i + 1] - toff[i]);
            if (n > bufcap) {
                bufcap = 2 * n;
                buf = (int32_t *)realloc(buf, sizeof(int32_t) * (size_t)bufcap);
            }
            int64_t b = 0;
            for (int64_t e = cand_off[i]; e < cand_off[i + 1]; e++)
                buf[b++] = cand_idx[e];
            for (int64_t e = toff[i]; e < toff[i + 1]; e++)
                buf[b++] = tidx[e];
            qsort(buf, (size_t)b, sizeof(int32_t), or_cmp_i32);
            int64_t c = 0, w = idx ? off[i] : 0;
            for (int64_t e = 0; e < b; e++) {
                int32_t j = buf[e];
                if (e > 0 && buf[e - 1] == j)
                    continue;
                if (j == i)
                    continue;
                if (!or_pred(x[i], y[i], z[i], h[i], x[j], y[j], z[j], h[j]))
                    continue;
                if (idx)
                    idx[w++] = j;
                c++;
            }
            if (!idx)
                off[i + 1] = c;
        }
        free(buf);
    }
    if (!idx) {
        off[0] = 0;
        for (int64_t i = 0; i < ng; i++)
            off[i + 1] += off[i];
    }
    free(toff);
    free(tidx);
}

/* Id-space rows -> slot-space rows: row(s) = sorted { slot(j) : j in nb(perm[s]) }.
 * soff must already hold the slot-space offsets (row lengths permuted). */
void or_rows_to_slots(int64_t ng, const int32_t *perm, const int64_t *off,
                      const int32_t *idx, const int64_t *soff, int32_t *sidx)
{
    int32_t *slot = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ng > 0 ? ng : 1));
    for (int64_t s = 0; s < ng; s++)
        slot[perm[s]] = (int32_t)s;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t s = 0; s < ng; s++) {
        int32_t i = perm[s];
        int64_t w = soff[s];
        for (int64_t e = off[i]; e < off[i + 1]; e++)
            sidx[w++] = slot[idx[e]];
        qsort(sidx + soff[s], (size_t)(soff[s + 1] - soff[s]), sizeof(int32_t), or_cmp_i32);
    }
    free(slot);
}

/* ------------------------------------------------------------------------ */
/* SPH sums (Sec. 2.2)                                                       */
/* ------------------------------------------------------------------------ */

/* Eq. (SPH-mass-density) with h_ij = (h_i + h_j)/2.  The sum runs over all
 * gas particles including j = i (the equation has no j != i), so the self
 * term m_i W(0, h_i) is included. */
void or_density(int64_t ng, const double *x, const double *y, const double *z,
                const double *m, const double *h, const int64_t *off,
                const int32_t *idx, double *rho)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ng; i++) {
        double s = m[i] * or_W(0.0, h[i]);
        for (int64_t e = off[i]; e < off[i + 1]; e++) {
            int32_t j = idx[e];
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            s += m[j] * or_W(r, 0.5 * (h[i] + h[j]));
        }
        rho[i] = s;
    }
}

/* Eq. (e_p_rho) solved for p, and the sound speed sqrt(gamma p / rho) used
 * in c_ij (Sec. 2.2, artificial viscosity). */
void or_eos(int64_t ng, double gamma, const double *rho, const double *e,
            double *p, double *c)
{
    for (int64_t i = 0; i < ng; i++) {
        p[i] = (gamma - 1.0) * rho[i] * e[i];
        c[i] = sqrt(gamma * p[i] / rho[i]);
    }
}

/* Eqs. (dv_dt-SPH) and (de_dt-SPH), hydrodynamic part only:
 *   a_i   = - sum_j m_j Pi_ij grad W_p(|r_ij|, h_ij)
 *   de_i  = 1/2 sum_j m_j Pi_ij (v_i - v_j) . grad W_p
 * grad W_p = dW_p/dxi * r_ij/|r_ij| / h_ij; a coincident pair (|r_ij| = 0)
 * contributes nothing.  Pi_ij = p_i/rho_i^2 + p_j/rho_j^2 + nu_ij with the
 * Monaghan-type viscosity nu_ij = mu_ij (beta mu_ij - alpha c_ij) / rho_ij,
 * mu_ij = h_ij r.v / (|r|^2 + eta h_ij^2) when r.v < 0 and 0 otherwise,
 * rho_ij and c_ij being arithmetic means. */
void or_sph_force(int64_t ng, const double *x, const double *y,
                  const double *z, const double *vx, const double *vy,
                  const double *vz, const double *m, const double *h,
                  const double *rho, const double *e, double gamma,
                  double alpha, double beta, double eta, const int64_t *off,
                  const int32_t *idx, double *ax, double *ay, double *az,
                  double *dedt)
{
    double *p = (double *)malloc(sizeof(double) * (size_t)(ng > 0 ? ng : 1));
    double *c = (double *)malloc(sizeof(double) * (size_t)(ng > 0 ? ng : 1));
    or_eos(ng, gamma, rho, e, p, c);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ng; i++) {
        double sx = 0, sy = 0, sz = 0, se = 0;
        for (int64_t k = off[i]; k < off[i + 1]; k++) {
            int32_t j = idx[k];
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0)
                continue;
            double r = sqrt(r2);
            double hij = 0.5 * (h[i] + h[j]);
            double dvx = vx[i] - vx[j], dvy = vy[i] - vy[j], dvz = vz[i] - vz[j];
            double rv = dx * dvx + dy * dvy + dz * dvz;
            double mu = 0.0;
            if (rv < 0.0)
                mu = hij * rv / (r2 + eta * hij * hij);
            double rhoij = 0.5 * (rho[i] + rho[j]);
            double cij = 0.5 * (c[i] + c[j]);
            double nu = mu * (beta * mu - alpha * cij) / rhoij;
            double Pi = p[i] / (rho[i] * rho[i]) + p[j] / (rho[j] * rho[j]) + nu;
            double g = or_dWp_dxi(r, hij) / (r * hij);   /* grad W_p = g * r_ij */
            double gx = g * dx, gy = g * dy, gz = g * dz;
            sx -= m[j] * Pi * gx;
            sy -= m[j] * Pi * gy;
            sz -= m[j] * Pi * gz;
            se += 0.5 * m[j] * Pi * (dvx * gx + dvy * gy + dvz * gz);
        }
        ax[i] = sx;
        ay[i] = sy;
        az[i] = sz;
        dedt[i] = se;
    }
    free(p);
    free(c);
}

/* ------------------------------------------------------------------------ */
/* Direct (Particle-Particle) gravity, Eq. (self-gravity)                    */
/* ------------------------------------------------------------------------ */

/* Neumaier's compensated summation, used so that the oracle's gravity sums
 * are exact to a few units of FP64 rounding, independent of order. */
typedef struct { double s, c; } or_sum;
static inline void or_add(or_sum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

/* f_ij = -G m_j (r_i - r_j) / (|r_i - r_j|^2 + eps^2)^{3/2}, summed over all
 * N particles j != i (the printed denominator |r_i - r_j + delta|^3 is read
 * as Plummer softening with length eps).  pot (optional) receives the
 * matching potential -G sum_{j != i} m_j / sqrt(|r_ij|^2 + eps^2).
 * Only the nt particles listed in tgt are evaluated; out[k] belongs to
 * particle tgt[k]. */
void or_gravity(int64_t n, const double *x, const double *y, const double *z,
                const double *m, double G, double eps, int64_t nt,
                const int64_t *tgt, double *ax, double *ay, double *az,
                double *pot)
{
    double e2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nt; k++) {
        int64_t i = tgt[k];
        or_sum sx = {0, 0}, sy = {0, 0}, sz = {0, 0}, sp = {0, 0};
        for (int64_t j = 0; j < n; j++) {
            if (j == i)
                continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double d2 = dx * dx + dy * dy + dz * dz + e2;
            double d = sqrt(d2);
            double f = G * m[j] / (d2 * d);
            or_add(&sx, -f * dx);
            or_add(&sy, -f * dy);
            or_add(&sz, -f * dz);
            or_add(&sp, -G * m[j] / d);
        }
        ax[k] = sx.s + sx.c;
        ay[k] = sy.s + sy.c;
        az[k] = sz.s + sz.c;
        if (pot)
            pot[k] = sp.s + sp.c;
    }
}

/* ------------------------------------------------------------------------ */
/* Predictor-corrector ("leapfrog") update, Eqs. (v-predictor)..(e-corrector)*/
/* ------------------------------------------------------------------------ */

/* Predictor: vt = v + dt Q, et = e + dt E, r <- r + dt/2 (vt + v).
 * Halo particles (index >= ng) carry no internal energy. */
void or_predict(int64_t n, int64_t ng, double dt, double *x, double *y,
                double *z, const double *vx, const double *vy,
                const double *vz, const double *e, const double *qx,
                const double *qy, const double *qz, const double *E,
                double *vtx, double *vty, double *vtz, double *et)
{
    for (int64_t i = 0; i < n; i++) {
        vtx[i] = vx[i] + dt * qx[i];
        vty[i] = vy[i] + dt * qy[i];
        vtz[i] = vz[i] + dt * qz[i];
        x[i] = x[i] + 0.5 * dt * (vtx[i] + vx[i]);
        y[i] = y[i] + 0.5 * dt * (vty[i] + vy[i]);
        z[i] = z[i] + 0.5 * dt * (vtz[i] + vz[i]);
    }
    for (int64_t i = 0; i < ng; i++)
        et[i] = e[i] + dt * E[i];
}

/* Corrector: v <- (v + vt)/2 + dt/2 Qt, e <- (e + et)/2 + dt/2 Et, where Qt,
 * Et are evaluated at the new positions with the predicted vt, et. */
void or_correct(int64_t n, int64_t ng, double dt, double *vx, double *vy,
                double *vz, double *e, const double *vtx, const double *vty,
                const double *vtz, const double *et, const double *qx,
                const double *qy, const double *qz, const double *E)
{
    for (int64_t i = 0; i < n; i++) {
        vx[i] = 0.5 * (vx[i] + vtx[i]) + 0.5 * dt * qx[i];
        vy[i] = 0.5 * (vy[i] + vty[i]) + 0.5 * dt * qy[i];
        vz[i] = 0.5 * (vz[i] + vtz[i]) + 0.5 * dt * qz[i];
    }
    for (int64_t i = 0; i < ng; i++)
        e[i] = 0.5 * (e[i] + et[i]) + 0.5 * dt * E[i];
}

/* ------------------------------------------------------------------------ */
/* Conserved quantities                                                      */
/* ------------------------------------------------------------------------ */

/* out[0] = E_kin = sum m v^2/2, out[1] = E_int = sum_gas m e,
 * out[2] = E_pot = 1/2 sum m phi, out[3] = total energy,
 * out[4..6] = momentum sum m v, out[7..9] = angular momentum sum m r x v.
 * pot may be NULL (then E_pot = 0). */
void or_diagnostics(int64_t n, int64_t ng, const double *x, const double *y,
                    const double *z, const double *vx, const double *vy,
                    const double *vz, const double *m, const double *e,
                    const double *pot, double *out)
{
    or_sum a[10];
    memset(a, 0, sizeof(a));
    for (int64_t i = 0; i < n; i++) {
        or_add(&a[0], 0.5 * m[i] * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]));
        if (i < ng)
            or_add(&a[1], m[i] * e[i]);
        if (pot)
            or_add(&a[2], 0.5 * m[i] * pot[i]);
        or_add(&a[4], m[i] * vx[i]);
        or_add(&a[5], m[i] * vy[i]);
        or_add(&a[6], m[i] * vz[i]);
        or_add(&a[7], m[i] * (y[i] * vz[i] - z[i] * vy[i]));
        or_add(&a[8], m[i] * (z[i] * vx[i] - x[i] * vz[i]));
        or_add(&a[9], m[i] * (x[i] * vy[i] - y[i] * vx[i]));
    }
    for (int k = 0; k < 10; k++)
        out[k] = a[k].s + a[k].c;
    out[3] = out[0] + out[1] + out[2];
}


/* ------------------------------------------------------------------------ */
/* Step control (Sec. 2.2)                                                   */
/* ------------------------------------------------------------------------ */

/* Eq. (dt-stability): dt = C min_i s_i / (cmax_i (1 + 1.2 alpha)
 *   + 1.2 beta mumax_i + sqrt(s_i (|Q_i| + |E_i|))), over gas particles with
 * at least one neighbour, where s_i = min_j |r_ij|, cmax_i = max_j c_ij,
 * c_ij = (c_i + c_j)/2 and mumax_i = max_j |mu_ij| (mu_ij as in the
 * viscosity; it is never positive, so its largest magnitude is taken).
 * Q_i is the total acceleration and E_i = de_i/dt.  The square-root term is
 * used as printed (its two parts carry different units).  Returns +inf when
 * no particle has a neighbour. */
double or_cfl_dt(int64_t ng, const double *x, const double *y, const double *z,
                 const double *vx, const double *vy, const double *vz, const double *h,
                 const double *c, const double *qx, const double *qy, const double *qz,
                 const double *E, double C, double alpha, double beta, double eta,
                 const int64_t *off, const int32_t *idx)
{
    double best = INFINITY;
    for (int64_t i = 0; i < ng; i++) {
        if (off[i + 1] == off[i])
            continue;
        double smin = INFINITY, cmax = 0.0, mumax = 0.0;
        for (int64_t k = off[i]; k < off[i + 1]; k++) {
            int32_t j = idx[k];
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            double r2 = dx * dx + dy * dy + dz * dz;
            double r = sqrt(r2);
            if (r < smin)
                smin = r;
            double cij = 0.5 * (c[i] + c[j]);
            if (cij > cmax)
                cmax = cij;
            double rv = dx * (vx[i] - vx[j]) + dy * (vy[i] - vy[j]) + dz * (vz[i] - vz[j]);
            if (rv < 0.0) {
                double hij = 0.5 * (h[i] + h[j]);
                double mu = fabs(hij * rv / (r2 + eta * hij * hij));
                if (mu > mumax)
                    mumax = mu;
            }
        }
        double q = sqrt(qx[i] * qx[i] + qy[i] * qy[i] + qz[i] * qz[i]);
        double den = cmax * (1.0 + 1.2 * alpha) + 1.2 * beta * mumax + sqrt(smin * (q + fabs(E[i])));
        double dt = den > 0.0 ? smin / den : INFINITY;
        if (dt < best)
            best = dt;
    }
    return C * best;
}

/* h_i = sigma (m_i / rho_i)^(1/3) (Sec. 2.2, after Eq. SPH-Kernel). */
void or_update_h(int64_t ng, double sigma, const double *m, const double *rho, double *h)
{
    for (int64_t i = 0; i < ng; i++)
        h[i] = sigma * cbrt(m[i] / rho[i]);
}

int or_max_levels(void) { return OR_MAX_LEVELS; }

/* Threads of the OpenMP loops (timing on one core or on all of them). */
#ifdef _OPENMP
#include <omp.h>
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int or_get_threads(void) { return omp_get_max_threads(); }
#else
void or_set_threads(int n) { (void)n; }
int or_get_threads(void) { return 1; }
#endif
size_t or_grid_size(void) { return sizeof(or_grid_t); }
