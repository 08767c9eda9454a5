/*
 * FP64 CPU oracle for the Dynamic-Zoom-Simulation (DZS) gravity step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the GPU path is
 * checked against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header or constant generator with the GPU library.
 *
 * Every routine is written for a reader holding the paper (Garaldi, Nori & Baldi,
 * "Dynamic Zoom Simulations", arXiv:2005.05328): it follows the definitions in the order
 * the paper states them, with no blocking, fusion or reordering beyond that.  Where the
 * paper is silent, the reading taken is stated at the routine.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (IEEE round-to-nearest FP64,
 * no contraction, so every rounding below is the one written).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define KEY_BITS 21                 /* bits per dimension of the Morton key */
#define KEY_SIDE 2097152.0          /* 2^21 */

/* ------------------------------------------------------------------------------------ */
/* Periodic helpers                                                                      */
/* ------------------------------------------------------------------------------------ */

/* Minimum image of one component of a separation, box side L: map d into [-L/2, L/2). */
static double min_image(double d, double L)
{
    if (d >= 0.5 * L)
        d -= L;
    else if (d < -0.5 * L)
        d += L;
    return d;
}

/* Wrap a coordinate into [0, L): x - L*floor(x/L), and a result equal to L becomes 0. */
static double wrap_coord(double x, double L)
{
    double q = floor(x / L);
    double w = x - L * q;
    if (w >= L)
        w = 0.0;
    return w;
}

/* ------------------------------------------------------------------------------------ */
/* Morton keys.  The paper's oct-tree (Sec. 2.1) splits the box into octants recursively; */
/* a particle's level-k node is the level-k cube containing it.  We name the cubes by      */
/* interleaved integer coordinates: i_d = min(floor(x_d * s), 2^21 - 1), s = fl(2^21/L),  */
/* key bit 3j+2 = bit j of i_x, bit 3j+1 = bit j of i_y, bit 3j = bit j of i_z.  The      */
/* level-k cube of a particle is then key >> 3(21-k).                                     */
/* ------------------------------------------------------------------------------------ */

static uint64_t cell_index(double v, double s)
{
    double t = floor(v * s);
    if (t < 0.0)
        t = 0.0;
    if (t > KEY_SIDE - 1.0)
        t = KEY_SIDE - 1.0;
    return (uint64_t)t;
}

static uint64_t interleave(uint64_t ix, uint64_t iy, uint64_t iz)
{
    uint64_t key = 0;
    for (int j = 0; j < KEY_BITS; ++j) {
        key |= ((ix >> j) & 1ull) << (3 * j + 2);
        key |= ((iy >> j) & 1ull) << (3 * j + 1);
        key |= ((iz >> j) & 1ull) << (3 * j);
    }
    return key;
}

void orc_morton_keys(int64_t n, const double *x, const double *y, const double *z, double L,
                     uint64_t *key)
{
    const double s = KEY_SIDE / L;
    for (int64_t i = 0; i < n; ++i)
        key[i] = interleave(cell_index(x[i], s), cell_index(y[i], s), cell_index(z[i], s));
}

/* ------------------------------------------------------------------------------------ */
/* DZS coarsening (Sec. 2.2 and 2.2.1, eqs. 1 and 3).                                     */
/*                                                                                       */
/* The walk starts at the root node.  A node that meets the merging criteria is replaced  */
/* by a single particle carrying its centre-of-mass properties; otherwise the walk visits */
/* each child.  The geometric criterion (eq. 1) is made node-centric and global by        */
/* replacing the particle-node distance with D_n = max(d_{n-obs} - R_lc - b, 0) (eq. 3),  */
/* d measured from the node's centre of mass to the observer.  A node merges when         */
/* l_n < theta * D_n, i.e. when the force criterion would *not* open it, and only if its  */
/* side does not exceed l_max (the background-resolution cap).                            */
/*                                                                                       */
/* Readings taken where the paper is silent:                                             */
/*  - distances use the periodic minimum image; the observer sits at x_obs;               */
/*  - the cap l_n <= l_max is the level bound k >= k_min (l_k = L / 2^k);                 */
/*  - l_k < theta*D_n with D_n > 0 is evaluated as |d|^2 > T_k^2, T_k = R_lc + b + l_k/theta;*/
/*  - a node needs at least two member particles to merge;                                 */
/*  - node sums run over members in ascending (Morton key, id) order, Neumaier-compensated;*/
/*  - the new particle: mult = sum of mult, x = centre of mass (wrapped into [0,L)),       */
/*    p = mass-weighted mean momentum (momentum conserved), id = smallest member id,       */
/*    type = 1.                                                                           */
/*                                                                                       */
/* Dynamical criterion (eq. 2 made node-centric with eq. 3, Sec. 2.2.1): the force walk   */
/* opens a node when G M_n l_n^2 / d^4 >= alpha |a_old|; DZS replaces d by D_n and |a_old| */
/* by the smallest previous acceleration among the particles inside the lightcone plus    */
/* buffer.  A node therefore merges when G M_n l_k^2 < alpha a_min D_n^4 with D_n > 0.    */
/* Readings: "inside" is sqrt(|d_i|^2) < R_lc + b on the minimum-image offset; a_min is   */
/* sqrt of the smallest g.g among those particles (+inf when none is inside, so every     */
/* node with D_n > 0 qualifies); D_n = sqrt(|d|^2) - (R_lc + b); the comparison is        */
/* evaluated as ((G m0) K) l_k^2 < (alpha a_min) ((D D)(D D)), l_k^2 = l_k l_k.            */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    double sum, comp;
} neumaier_t;

static void neumaier_add(neumaier_t *a, double v)
{
    double t = a->sum + v;
    if (fabs(a->sum) >= fabs(v))
        a->comp += (a->sum - t) + v;
    else
        a->comp += (v - t) + a->sum;
    a->sum = t;
}

static double neumaier_value(const neumaier_t *a) { return a->sum + a->comp; }

typedef struct {
    /* inputs */
    const double *x, *y, *z, *px, *py, *pz;
    const uint32_t *mult, *id;
    const uint8_t *type;
    const uint64_t *key;
    const int64_t *order; /* particle indices sorted by (key, id) */
    double L, xobs[3];
    double T2[KEY_BITS + 1];
    int k_min;
    /* dynamical criterion (crit == 1) */
    int crit;
    double Gm0, Rb, alpha_amin, lk2[KEY_BITS + 1];
    /* outputs */
    double *ox, *oy, *oz, *opx, *opy, *opz;
    uint32_t *omult, *oid;
    uint8_t *otype;
    int64_t *group_of;
    int64_t n_out, n_merged_nodes;
} coarsen_ctx;

static void emit_survivor(coarsen_ctx *c, int64_t i)
{
    int64_t o = c->n_out++;
    c->ox[o] = c->x[i];
    c->oy[o] = c->y[i];
    c->oz[o] = c->z[i];
    c->opx[o] = c->px[i];
    c->opy[o] = c->py[i];
    c->opz[o] = c->pz[i];
    c->omult[o] = c->mult[i];
    c->oid[o] = c->id[i];
    c->otype[o] = c->type[i];
    c->group_of[i] = o;
}

/* Try to merge the level-k node whose members are order[s..e).  Returns 1 if merged. */
static int try_merge(coarsen_ctx *c, int k, int64_t s, int64_t e)
{
    neumaier_t S[3] = {{0, 0}, {0, 0}, {0, 0}}, P[3] = {{0, 0}, {0, 0}, {0, 0}};
    uint64_t K = 0;
    uint32_t min_id = 0xffffffffu;
    for (int64_t r = s; r < e; ++r) {
        int64_t i = c->order[r];
        double m = (double)c->mult[i];
        K += c->mult[i];
        neumaier_add(&S[0], m * c->x[i]);
        neumaier_add(&S[1], m * c->y[i]);
        neumaier_add(&S[2], m * c->z[i]);
        neumaier_add(&P[0], m * c->px[i]);
        neumaier_add(&P[1], m * c->py[i]);
        neumaier_add(&P[2], m * c->pz[i]);
        if (c->id[i] < min_id)
            min_id = c->id[i];
    }
    double Kd = (double)K;
    double X[3], d[3];
    for (int a = 0; a < 3; ++a) {
        X[a] = wrap_coord(neumaier_value(&S[a]) / Kd, c->L);
        d[a] = min_image(X[a] - c->xobs[a], c->L);
    }
    double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (c->crit == 0) {
        if (!(d2 > c->T2[k]))
            return 0;
    } else {
        double D = sqrt(d2) - c->Rb;
        if (!(D > 0.0))
            return 0;
        double lhs = (c->Gm0 * Kd) * c->lk2[k];
        double rhs = c->alpha_amin * ((D * D) * (D * D));
        if (!(lhs < rhs))
            return 0;
    }
    int64_t o = c->n_out++;
    c->ox[o] = X[0];
    c->oy[o] = X[1];
    c->oz[o] = X[2];
    c->opx[o] = neumaier_value(&P[0]) / Kd;
    c->opy[o] = neumaier_value(&P[1]) / Kd;
    c->opz[o] = neumaier_value(&P[2]) / Kd;
    c->omult[o] = (uint32_t)K;
    c->oid[o] = min_id;
    c->otype[o] = 1;
    for (int64_t r = s; r < e; ++r)
        c->group_of[c->order[r]] = o;
    c->n_merged_nodes++;
    return 1;
}

/* Visit the level-k node with members order[s..e) (all share the level-k key prefix). */
static void visit(coarsen_ctx *c, int k, int64_t s, int64_t e)
{
    if (e - s == 1) { /* a single particle is a leaf of the tree: it survives */
        emit_survivor(c, c->order[s]);
        return;
    }
    if (k >= c->k_min && try_merge(c, k, s, e))
        return;
    if (k == KEY_BITS) { /* finest cell: cannot be split further */
        for (int64_t r = s; r < e; ++r)
            emit_survivor(c, c->order[r]);
        return;
    }
    /* open the node: children are the level-(k+1) cubes, contiguous in (key,id) order */
    const int shift = 3 * (KEY_BITS - (k + 1));
    int64_t r = s;
    while (r < e) {
        uint64_t digit = (c->key[c->order[r]] >> shift) & 7ull;
        int64_t q = r + 1;
        while (q < e && ((c->key[c->order[q]] >> shift) & 7ull) == digit)
            ++q;
        visit(c, k + 1, r, q);
        r = q;
    }
}

static const uint64_t *g_sort_key;
static const uint32_t *g_sort_id;

static int cmp_key_id(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    if (g_sort_key[a] != g_sort_key[b])
        return g_sort_key[a] < g_sort_key[b] ? -1 : 1;
    if (g_sort_id[a] != g_sort_id[b])
        return g_sort_id[a] < g_sort_id[b] ? -1 : 1;
    return 0;
}

/* Merge threshold per level: T_k^2 with T_k = (R_lc + b) + l_k / theta, l_k = L / 2^k.
 * Exposed so tests can read the exact values the oracle uses. */
void orc_merge_thresholds(double L, double R_lc, double b, double theta, double *T2 /* [22] */)
{
    for (int k = 0; k <= KEY_BITS; ++k) {
        double lk = ldexp(L, -k);
        double T = (R_lc + b) + lk / theta;
        T2[k] = T * T;
    }
}

/* The smallest previous acceleration among the particles inside the lightcone plus buffer
 * (the a_old replacement of Sec. 2.2.1): sqrt of min g.g over particles with
 * sqrt(|min-image(x_i - x_obs)|^2) < R_lc + b; +inf when there is none. */
double orc_a_min(int64_t n, const double *x, const double *y, const double *z,
                 const double *gx, const double *gy, const double *gz, double L,
                 const double *xobs, double Rb)
{
    double best = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double dx = min_image(x[i] - xobs[0], L);
        double dy = min_image(y[i] - xobs[1], L);
        double dz = min_image(z[i] - xobs[2], L);
        if (!(sqrt(dx * dx + dy * dy + dz * dz) < Rb))
            continue;
        double g2 = gx[i] * gx[i] + gy[i] * gy[i] + gz[i] * gz[i];
        if (g2 < best)
            best = g2;
    }
    return sqrt(best);
}

/* crit 0: geometric (theta).  crit 1: dynamical (alpha, with G m0 and the previous
 * accelerations gx, gy, gz); *a_min_out (optional) receives the a_min used. */
int64_t orc_coarsen(int64_t n, const double *x, const double *y, const double *z,
                    const double *px, const double *py, const double *pz,
                    const uint32_t *mult, const uint32_t *id, const uint8_t *type, double L,
                    const double *xobs, double R_lc, double b, double theta, int k_min,
                    int crit, double alpha, double Gm0, const double *gx, const double *gy,
                    const double *gz, double *a_min_out,
                    double *ox, double *oy, double *oz, double *opx, double *opy, double *opz,
                    uint32_t *omult, uint32_t *oid, uint8_t *otype, int64_t *group_of,
                    int64_t *n_merged_nodes)
{
    if (n <= 0) {
        *n_merged_nodes = 0;
        if (a_min_out)
            *a_min_out = INFINITY;
        return 0;
    }
    uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    orc_morton_keys(n, x, y, z, L, key);
    for (int64_t i = 0; i < n; ++i)
        order[i] = i;
    g_sort_key = key;
    g_sort_id = id;
    qsort(order, (size_t)n, sizeof(int64_t), cmp_key_id);

    coarsen_ctx c;
    memset(&c, 0, sizeof(c));
    c.x = x; c.y = y; c.z = z; c.px = px; c.py = py; c.pz = pz;
    c.mult = mult; c.id = id; c.type = type; c.key = key; c.order = order;
    c.L = L;
    c.xobs[0] = xobs[0]; c.xobs[1] = xobs[1]; c.xobs[2] = xobs[2];
    orc_merge_thresholds(L, R_lc, b, theta, c.T2);
    c.k_min = k_min;
    c.crit = crit;
    if (crit == 1) {
        c.Gm0 = Gm0;
        c.Rb = R_lc + b;
        for (int k = 0; k <= KEY_BITS; ++k) {
            double lk = ldexp(L, -k);
            c.lk2[k] = lk * lk;
        }
        double a_min = orc_a_min(n, x, y, z, gx, gy, gz, L, xobs, c.Rb);
        c.alpha_amin = alpha * a_min;
        if (a_min_out)
            *a_min_out = a_min;
    } else if (a_min_out) {
        *a_min_out = NAN;
    }
    c.ox = ox; c.oy = oy; c.oz = oz; c.opx = opx; c.opy = opy; c.opz = opz;
    c.omult = omult; c.oid = oid; c.otype = otype; c.group_of = group_of;
    visit(&c, 0, 0, n);
    free(key);
    free(order);
    *n_merged_nodes = c.n_merged_nodes;
    return c.n_out;
}

/* ------------------------------------------------------------------------------------ */
/* Short-range force, by direct summation (Sec. 2.1: the tree handles the short-range part */
/* of the TreePM split; its exact value is the sum over all pairs closer than the cutoff). */
/*                                                                                       */
/* g_i = -G sum_{j != i, r_ij < r_cut} m_j r_ij g_soft(r_ij, h_ij) S(r_ij / r_s)          */
/*   r_ij = minimum image of x_i - x_j; S(u) = erfc(u/2) + u/sqrt(pi) exp(-u^2/4) is the  */
/*   real-space complement of a Gaussian long-range filter exp(-k^2 r_s^2).               */
/*   Softening: cubic-spline kernel of support h = 2.8 eps; eps = eps0 mult^(1/3) (the    */
/*   paper's (M/M_init)^(1/3) rescaling, Sec. 2.2); mixed pairs take h_ij = max(h_i,h_j). */
/*   g_soft is the spline's enclosed-mass force divided by r: r^-3 for r >= h.            */
/* ------------------------------------------------------------------------------------ */

double orc_g_soft(double r, double h)
{
    if (r >= h)
        return 1.0 / (r * r * r);
    double u = r / h;
    double h3 = 1.0 / (h * h * h);
    if (u < 0.5)
        return h3 * (32.0 / 3.0 - 192.0 / 5.0 * u * u + 32.0 * u * u * u);
    return h3 * (64.0 / 3.0 - 48.0 * u + 192.0 / 5.0 * u * u - 32.0 / 3.0 * u * u * u -
                 1.0 / (15.0 * u * u * u));
}

double orc_split_S(double u)
{
    return erfc(0.5 * u) + u / sqrt(M_PI) * exp(-0.25 * u * u);
}

void orc_short_range(int64_t n, const double *x, const double *y, const double *z,
                     const uint32_t *mult, double L, double m0, double eps0, double G,
                     double r_s, double r_cut, int64_t n_targets, const int64_t *targets,
                     double *gx, double *gy, double *gz)
{
    /* cell list with cells no smaller than r_cut; it only narrows the candidate set, the
     * pair set summed is exactly {j != i : r_ij < r_cut}. */
    int nc = (int)floor(L / r_cut);
    if (nc < 3)
        nc = 1; /* fewer than 3 cells per side: one cell holds every candidate */
    if (nc > 256)
        nc = 256;
    const double cs = L / nc;
    int64_t ncell = (int64_t)nc * nc * nc;
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t c = 0; c < ncell; ++c)
        head[c] = -1;
    for (int64_t j = n - 1; j >= 0; --j) {
        int cx = (int)(x[j] / cs), cy = (int)(y[j] / cs), cz = (int)(z[j] / cs);
        if (cx >= nc) cx = nc - 1;
        if (cy >= nc) cy = nc - 1;
        if (cz >= nc) cz = nc - 1;
        int64_t c = ((int64_t)cx * nc + cy) * nc + cz;
        next[j] = head[c];
        head[c] = j;
    }
    const double rc2 = r_cut * r_cut;
    const int span = nc >= 3 ? 1 : 0;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t t = 0; t < n_targets; ++t) {
        int64_t i = targets ? targets[t] : t;
        double hi = 2.8 * eps0 * cbrt((double)mult[i]);
        double ax = 0, ay = 0, az = 0;
        int cx = (int)(x[i] / cs), cy = (int)(y[i] / cs), cz = (int)(z[i] / cs);
        if (cx >= nc) cx = nc - 1;
        if (cy >= nc) cy = nc - 1;
        if (cz >= nc) cz = nc - 1;
        for (int ox = -span; ox <= span; ++ox)
            for (int oy = -span; oy <= span; ++oy)
                for (int oz = -span; oz <= span; ++oz) {
                    int64_t c = ((int64_t)((cx + ox + nc) % nc) * nc + (cy + oy + nc) % nc) * nc +
                                (cz + oz + nc) % nc;
                    for (int64_t j = head[c]; j >= 0; j = next[j]) {
                        if (j == i)
                            continue;
                        double dx = min_image(x[i] - x[j], L);
                        double dy = min_image(y[i] - y[j], L);
                        double dz = min_image(z[i] - z[j], L);
                        double r2 = dx * dx + dy * dy + dz * dz;
                        if (!(r2 < rc2))
                            continue;
                        double r = sqrt(r2);
                        double hj = 2.8 * eps0 * cbrt((double)mult[j]);
                        double h = hi > hj ? hi : hj;
                        double f = G * m0 * (double)mult[j] * orc_g_soft(r, h) * orc_split_S(r / r_s);
                        ax -= f * dx;
                        ay -= f * dy;
                        az -= f * dz;
                    }
                }
        gx[t] = ax;
        gy[t] = ay;
        gz[t] = az;
    }
    free(head);
    free(next);
}

/* ------------------------------------------------------------------------------------ */
/* PM long-range force, mesh parts (Sec. 2.1: density on an auxiliary uniform grid,      */
/* Poisson equation solved in Fourier space).  Mesh points at j*Delta, Delta = L/N_g;     */
/* cloud-in-cell weights w1 = u - floor(u), w0 = 1 - w1 with u = x/Delta, indices mod N_g. */
/* Mesh layout: index (ix*N_g + iy)*N_g + iz.                                             */
/* ------------------------------------------------------------------------------------ */

static void cic_weights(double x, double L, int ng, int *i0, int *i1, double *w0, double *w1)
{
    double u = x / (L / ng);
    double f = floor(u);
    int i = (int)f;
    *w1 = u - f;
    *w0 = 1.0 - *w1;
    i %= ng;
    if (i < 0)
        i += ng;
    *i0 = i;
    *i1 = (i + 1) % ng;
}

/* rho_j = sum_i m_i W_ij / Delta^3 (mass density), sequential accumulation. */
void orc_cic_deposit(int64_t n, const double *x, const double *y, const double *z,
                     const uint32_t *mult, double L, int ng, double m0, double *rho)
{
    const int64_t ng3 = (int64_t)ng * ng * ng;
    const double delta = L / ng;
    const double inv_vol = 1.0 / (delta * delta * delta);
    memset(rho, 0, sizeof(double) * (size_t)ng3);
    for (int64_t p = 0; p < n; ++p) {
        int ix[2], iy[2], iz[2];
        double wx[2], wy[2], wz[2];
        cic_weights(x[p], L, ng, &ix[0], &ix[1], &wx[0], &wx[1]);
        cic_weights(y[p], L, ng, &iy[0], &iy[1], &wy[0], &wy[1]);
        cic_weights(z[p], L, ng, &iz[0], &iz[1], &wz[0], &wz[1]);
        double m = m0 * (double)mult[p];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c)
                    rho[((int64_t)ix[a] * ng + iy[b]) * ng + iz[c]] +=
                        m * wx[a] * wy[b] * wz[c] * inv_vol;
    }
}

/* out_i = sum_j W_ij mesh_j with the same cloud-in-cell weights. */
void orc_cic_interp(int64_t n, const double *x, const double *y, const double *z, double L, int ng,
                    const double *mesh, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        int ix[2], iy[2], iz[2];
        double wx[2], wy[2], wz[2];
        cic_weights(x[p], L, ng, &ix[0], &ix[1], &wx[0], &wx[1]);
        cic_weights(y[p], L, ng, &iy[0], &iy[1], &wy[0], &wy[1]);
        cic_weights(z[p], L, ng, &iz[0], &iz[1], &wz[0], &wz[1]);
        double s = 0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c)
                    s += wx[a] * wy[b] * wz[c] * mesh[((int64_t)ix[a] * ng + iy[b]) * ng + iz[c]];
        out[p] = s;
    }
}
