// Per-particle streaming kernels: kick, drift with the lightcone crossing test, Morton keys,
// and the gathers that apply a sort permutation to the structure-of-arrays state.
// All are HBM-bound: one thread per particle, coalesced loads and stores of each array.
#include "internal.h"

#define PT_THREADS 256

static inline uint32_t blocks_for(uint64_t n, uint32_t t) { return (uint32_t)((n + t - 1) / t); }

// ---------------------------------------------------------------------------------------
// kick: p <- p + g K (one rounded product, one rounded sum: no contraction)
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(PT_THREADS) void k_kick(uint64_t n, double *__restrict__ px,
                                                     double *__restrict__ py,
                                                     double *__restrict__ pz,
                                                     const double *__restrict__ gx,
                                                     const double *__restrict__ gy,
                                                     const double *__restrict__ gz, double K,
                                                     const double *__restrict__ Kp) {
    uint64_t i = (uint64_t)blockIdx.x * PT_THREADS + threadIdx.x;
    if (i >= n)
        return;
    if (Kp)
        K = *Kp;  // the step's factor from a device parameter block
    px[i] = px[i] + gx[i] * K;
    py[i] = py[i] + gy[i] * K;
    pz[i] = pz[i] + gz[i] * K;
}

dzs_status dzs_launch_kick(dzs_ctx *ctx, const dzs_particles *p, double K, hipStream_t s,
                           const double *K_dev) {
    if (p->n == 0)
        return DZS_OK;
    dzs_timed t(ctx, KC_KICK, s);
    hipLaunchKernelGGL(k_kick, dim3(blocks_for(p->n, PT_THREADS)), dim3(PT_THREADS), 0, s, p->n,
                       p->px, p->py, p->pz, (const double *)p->gx, (const double *)p->gy,
                       (const double *)p->gz, K, K_dev);
    return dzs_check_launch(ctx, "kick");
}

__global__ __launch_bounds__(PT_THREADS) void k_add3(uint64_t n, double *__restrict__ ax,
                                                     double *__restrict__ ay,
                                                     double *__restrict__ az,
                                                     const double *__restrict__ bx,
                                                     const double *__restrict__ by,
                                                     const double *__restrict__ bz, double s) {
    const uint64_t i = (uint64_t)blockIdx.x * PT_THREADS + threadIdx.x;
    if (i >= n)
        return;
    ax[i] = ax[i] + s * bx[i];
    ay[i] = ay[i] + s * by[i];
    az[i] = az[i] + s * bz[i];
}

dzs_status dzs_launch_add3(dzs_ctx *ctx, uint64_t n, double *ax, double *ay, double *az,
                           const double *bx, const double *by, const double *bz, double s,
                           hipStream_t st) {
    if (n == 0)
        return DZS_OK;
    hipLaunchKernelGGL(k_add3, dim3(blocks_for(n, PT_THREADS)), dim3(PT_THREADS), 0, st, n, ax,
                       ay, az, bx, by, bz, s);
    return dzs_check_launch(ctx, "add3");
}

// Largest |px| + |py| + |pz| times |D| (a bound on the drift's displacement) over the state:
// a block maximum, one atomic per block on the bits of the non-negative double.
__global__ __launch_bounds__(PT_THREADS) void k_drift_bound(uint64_t n,
                                                            const double *__restrict__ px,
                                                            const double *__restrict__ py,
                                                            const double *__restrict__ pz,
                                                            double D,
                                                            unsigned long long *step_max) {
    __shared__ double s_m[PT_THREADS / 64];
    const uint64_t i = (uint64_t)blockIdx.x * PT_THREADS + threadIdx.x;
    double v = 0.0;
    if (i < n)
        v = (fabs(px[i]) + fabs(py[i]) + fabs(pz[i])) * fabs(D);
    for (int o = 32; o >= 1; o >>= 1)
        v = fmax(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63u) == 0u)
        s_m[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = s_m[0];
        for (int w = 1; w < PT_THREADS / 64; ++w)
            m = fmax(m, s_m[w]);
        atomicMax(step_max, (unsigned long long)__double_as_longlong(m));
    }
}

// total += the step's bound; the step's slot back to zero
__global__ void k_drift_bound_acc(unsigned long long *step_max, double *total) {
    *total = *total + __longlong_as_double((long long)*step_max);
    *step_max = 0ull;
}

__global__ void k_drift_bound_reset(unsigned long long *step_max, double *total) {
    *step_max = 0ull;
    *total = 0.0;
}

dzs_status dzs_drift_bound_reset(dzs_ctx *ctx, hipStream_t s) {
    hipLaunchKernelGGL(k_drift_bound_reset, dim3(1), dim3(1), 0, s,
                       (unsigned long long *)(ctx->d_small + DZS_SMALL_DRIFT_STEP),
                       (double *)(ctx->d_small + DZS_SMALL_DRIFT_TOTAL));
    return dzs_check_launch(ctx, "drift_bound_reset");
}

dzs_status dzs_drift_bound_add(dzs_ctx *ctx, const dzs_particles *p, double D, hipStream_t s) {
    if (p->n == 0)
        return DZS_OK;
    unsigned long long *step = (unsigned long long *)(ctx->d_small + DZS_SMALL_DRIFT_STEP);
    hipLaunchKernelGGL(k_drift_bound, dim3(blocks_for(p->n, PT_THREADS)), dim3(PT_THREADS), 0, s,
                       p->n, (const double *)p->px, (const double *)p->py,
                       (const double *)p->pz, D, step);
    DZS_TRY(dzs_check_launch(ctx, "drift_bound"));
    hipLaunchKernelGGL(k_drift_bound_acc, dim3(1), dim3(1), 0, s, step,
                       (double *)(ctx->d_small + DZS_SMALL_DRIFT_TOTAL));
    return dzs_check_launch(ctx, "drift_bound_acc");
}

// box of particle i in a batch: the last b with first[b] <= i (first[] ascending, nb entries)
__device__ __forceinline__ uint32_t batch_box_of(const uint64_t *first, uint32_t nb, uint64_t i) {
    uint32_t lo = 0, hi = nb - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (first[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------------------
// drift + lightcone
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double cheb_eval(const double *c, int n, double t) {
    // Clenshaw recurrence for sum_k c_k T_k(t)
    double b1 = 0.0, b2 = 0.0;
    const double t2 = 2.0 * t;
    for (int k = n - 1; k >= 1; --k) {
        double b0 = fma(t2, b1, c[k] - b2);
        b2 = b1;
        b1 = b0;
    }
    return fma(t, b1, c[0] - b2);
}

// Crossing of the shrinking lightcone sphere: the root of
// F(t) = |d0 + p D(a0, a(t))|^2 - chi(a(t))^2 on t in [-1, 1], F(-1) < 0 <= F(1), by bisection
// to the last bit of t.  Returns t; *dc receives d0 + p D(a0, a(t)).
__device__ double lc_solve(const lc_args &A, double d0x, double d0y, double d0z, double px,
                           double py, double pz, double *dcx, double *dcy, double *dcz) {
    double lo = -1.0, hi = 1.0;
    for (int it = 0; it < 62; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi)
            break;
        double Dm = cheb_eval(A.cdrift, A.n_cheb, mid);
        double cm = cheb_eval(A.cchi, A.n_cheb, mid);
        double x = d0x + px * Dm, y = d0y + py * Dm, z = d0z + pz * Dm;
        double F = (x * x + y * y + z * z) - cm * cm;
        if (F < 0.0)
            lo = mid;
        else
            hi = mid;
    }
    double t = 0.5 * (lo + hi);
    double Dt = cheb_eval(A.cdrift, A.n_cheb, t);
    *dcx = d0x + px * Dt;
    *dcy = d0y + py * Dt;
    *dcz = d0z + pz * Dt;
    return t;
}

// PBLOCK: the drift and lightcone parameters come from a device block (*Ap) rather than the
// kernel arguments, so that a captured launch can be replayed for another step.
template <bool PBLOCK>
__global__ __launch_bounds__(PT_THREADS) void k_drift_lc(
    uint64_t n, double *__restrict__ x, double *__restrict__ y, double *__restrict__ z,
    const double *__restrict__ px, const double *__restrict__ py, const double *__restrict__ pz,
    const uint32_t *__restrict__ id, const uint32_t *__restrict__ mult, double L, lc_args A_arg,
    const lc_args *__restrict__ Ap, int do_lc, int do_drift, dzs_lc_record *__restrict__ rec, uint64_t rec_cap,
    unsigned long long *__restrict__ rec_count, uint32_t *__restrict__ overflow,
    const uint64_t *__restrict__ bfirst, const dzs_bbox *__restrict__ boxes, uint32_t nb) {
    uint64_t i = (uint64_t)blockIdx.x * PT_THREADS + threadIdx.x;
    if (i >= n)
        return;
    if (boxes)
        L = boxes[batch_box_of(bfirst, nb, i)].L;
    const lc_args &A = PBLOCK ? *Ap : A_arg;
    const double xi = x[i], yi = y[i], zi = z[i];
    const double pxi = px[i], pyi = py[i], pzi = pz[i];
    const double sx = pxi * A.D, sy = pyi * A.D, sz = pzi * A.D;
    const double nx = dzs_wrap(xi + sx, L), ny = dzs_wrap(yi + sy, L), nz = dzs_wrap(zi + sz, L);
    if (do_lc) {
        const double dx = dzs_min_image(xi - A.xo[0], L);
        const double dy = dzs_min_image(yi - A.xo[1], L);
        const double dz = dzs_min_image(zi - A.xo[2], L);
        const double f0 = (dx * dx + dy * dy + dz * dz) - A.chi2_0;
        // the end-of-drift test uses the offset the next drift starts from (the drifted,
        // wrapped position, minimum image): f1 here is f0 there, so a particle is emitted once
        const double ex = dzs_min_image(nx - A.xo[0], L);
        const double ey = dzs_min_image(ny - A.xo[1], L);
        const double ez = dzs_min_image(nz - A.xo[2], L);
        const double f1 = (ex * ex + ey * ey + ez * ez) - A.chi2_1;
        // one atomic per wave: the wave's emitters take consecutive slots
        const bool emit = f0 < 0.0 && f1 >= 0.0;
        const uint64_t m = __ballot(emit);
        if (m != 0ull) {
            const uint32_t lane = threadIdx.x & 63u;
            const uint32_t leader = (uint32_t)__ffsll((long long)m) - 1u;
            unsigned long long base = 0ull;
            if (lane == leader)
                base = atomicAdd(rec_count, (unsigned long long)__popcll(m));
            base = __shfl(base, (int)leader, 64);
            if (emit) {
                double cx, cy, cz;
                const double t = lc_solve(A, dx, dy, dz, pxi, pyi, pzi, &cx, &cy, &cz);
                const unsigned long long slot =
                    base + (unsigned long long)__popcll(m & ((1ull << lane) - 1ull));
                if (slot < rec_cap) {
                    dzs_lc_record r;
                    r.id = id[i];
                    r.mult = mult[i];
                    r.a_cross = A.a0 + 0.5 * (t + 1.0) * (A.a1 - A.a0);
                    r.d[0] = cx;
                    r.d[1] = cy;
                    r.d[2] = cz;
                    r.p[0] = pxi;
                    r.p[1] = pyi;
                    r.p[2] = pzi;
                    rec[slot] = r;
                } else {
                    *overflow = 1u;
                }
            }
        }
    }
    if (do_drift) {
        x[i] = nx;
        y[i] = ny;
        z[i] = nz;
    }
}

void dzs_make_lc_args(const dzs_lc_params *lc, lc_args *A) {
    memset(A, 0, sizeof(*A));
    for (int d = 0; d < 3; ++d)
        A->xo[d] = lc->x_obs[d];
    A->chi2_0 = lc->chi2_0;
    A->chi2_1 = lc->chi2_1;
    A->D = lc->D;
    A->a0 = lc->a0;
    A->a1 = lc->a1;
    A->n_cheb = lc->n_cheb;
    for (int k = 0; k < DZS_CHEB_MAX; ++k) {
        A->cchi[k] = lc->cheb_chi[k];
        A->cdrift[k] = lc->cheb_drift[k];
    }
}

dzs_status dzs_launch_drift_lc(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                               const dzs_lc_params *lc, dzs_lc_ring *ring, int do_lc,
                               int do_drift, hipStream_t s, bool batch, uint32_t nb,
                               const lc_args *A_dev) {
    if (p->n == 0)
        return DZS_OK;
    lc_args A;
    dzs_make_lc_args(lc, &A);
    dzs_lc_record *rec = nullptr;
    uint64_t cap = 0;
    unsigned long long *cnt = nullptr;
    uint32_t *ovf = nullptr;
    if (do_lc) {
        rec = ring->records;
        cap = ring->capacity;
        cnt = ring->count;
        ovf = ring->overflow;
    }
    dzs_timed t(ctx, KC_DRIFT_LC, s);
    if (A_dev)
        hipLaunchKernelGGL(k_drift_lc<true>, dim3(blocks_for(p->n, PT_THREADS)), dim3(PT_THREADS),
                           0, s, p->n, p->x, p->y, p->z, (const double *)p->px,
                           (const double *)p->py, (const double *)p->pz,
                           (const uint32_t *)p->id, (const uint32_t *)p->mult, box->L, A, A_dev,
                           do_lc, do_drift, rec, cap, cnt, ovf,
                           (const uint64_t *)ctx->batch_first, batch ? ctx->batch_box : nullptr,
                           nb);
    else
        hipLaunchKernelGGL(k_drift_lc<false>, dim3(blocks_for(p->n, PT_THREADS)),
                           dim3(PT_THREADS), 0, s, p->n, p->x, p->y, p->z,
                           (const double *)p->px, (const double *)p->py,
                           (const double *)p->pz, (const uint32_t *)p->id,
                           (const uint32_t *)p->mult, box->L, A, A_dev, do_lc, do_drift, rec,
                           cap, cnt, ovf, (const uint64_t *)ctx->batch_first,
                           batch ? ctx->batch_box : nullptr, nb);
    return dzs_check_launch(ctx, "drift_lc");
}

// ---------------------------------------------------------------------------------------
// Morton keys + identity index
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(PT_THREADS) void k_keys(uint64_t n, const double *__restrict__ x,
                                                     const double *__restrict__ y,
                                                     const double *__restrict__ z, double s,
                                                     uint64_t *__restrict__ key,
                                                     uint32_t *__restrict__ idx,
                                                     const uint64_t *__restrict__ bfirst,
                                                     const dzs_bbox *__restrict__ boxes,
                                                     uint32_t nb) {
    uint64_t i = (uint64_t)blockIdx.x * PT_THREADS + threadIdx.x;
    if (i >= n)
        return;
    if (boxes) {
        // a batch: the box in the top DZS_BATCH_LEVELS digits, 2^18 cells per side below
        const uint64_t b = batch_box_of(bfirst, nb, i);
        const double sb = DZS_BATCH_SIDE / boxes[b].L;
        auto cell = [&](double v) -> uint64_t {
            double t = floor(v * sb);
            t = t < 0.0 ? 0.0 : (t > DZS_BATCH_SIDE - 1.0 ? DZS_BATCH_SIDE - 1.0 : t);
            return (uint64_t)t;
        };
        key[i] = (b << DZS_BATCH_SHIFT) | (dzs_spread3(cell(x[i])) << 2) |
                 (dzs_spread3(cell(y[i])) << 1) | dzs_spread3(cell(z[i]));
    } else {
        key[i] = dzs_morton(x[i], y[i], z[i], s);
    }
    if (idx)
        idx[i] = (uint32_t)i;
}

dzs_status dzs_launch_keys(dzs_ctx *ctx, const double *x, const double *y, const double *z,
                           uint64_t n, double L, uint64_t *key, uint32_t *idx, hipStream_t s,
                           bool batch, uint32_t nb) {
    if (n == 0)
        return DZS_OK;
    const double scale = DZS_KEY_SIDE / L;
    dzs_timed t(ctx, KC_KEYS, s);
    hipLaunchKernelGGL(k_keys, dim3(blocks_for(n, PT_THREADS)), dim3(PT_THREADS), 0, s, n, x, y,
                       z, scale, key, idx, (const uint64_t *)ctx->batch_first,
                       batch ? ctx->batch_box : nullptr, nb);
    return dzs_check_launch(ctx, "keys");
}

// ---------------------------------------------------------------------------------------
// gathers / scatters through a permutation
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(PT_THREADS) void k_gather(uint64_t n, const T *__restrict__ src,
                                                       const uint32_t *__restrict__ perm,
                                                       T *__restrict__ dst) {
    uint64_t i = (uint64_t)blockIdx.x * PT_THREADS + threadIdx.x;
    if (i < n)
        dst[i] = src[perm[i]];
}

template <typename T>
__global__ __launch_bounds__(PT_THREADS) void k_copy(uint64_t n, const T *__restrict__ src,
                                                     T *__restrict__ dst) {
    uint64_t i = (uint64_t)blockIdx.x * PT_THREADS + threadIdx.x;
    if (i < n)
        dst[i] = src[i];
}

template <typename T>
static dzs_status permute_one(dzs_ctx *ctx, T *arr, const uint32_t *perm, uint64_t n,
                              hipStream_t s) {
    T *tmp = (T *)ctx->gather_tmp;
    uint32_t b = blocks_for(n, PT_THREADS);
    hipLaunchKernelGGL(k_gather<T>, dim3(b), dim3(PT_THREADS), 0, s, n, (const T *)arr, perm, tmp);
    DZS_TRY(dzs_check_launch(ctx, "gather"));
    hipLaunchKernelGGL(k_copy<T>, dim3(b), dim3(PT_THREADS), 0, s, n, (const T *)tmp, arr);
    return dzs_check_launch(ctx, "copy");
}

dzs_status dzs_permute_state(dzs_ctx *ctx, dzs_particles *p, const uint32_t *perm, int with_g,
                             hipStream_t s) {
    const uint64_t n = p->n;
    if (n == 0)
        return DZS_OK;
    dzs_timed t(ctx, KC_PERMUTE, s);
    double *f64[9] = {p->x, p->y, p->z, p->px, p->py, p->pz, p->gx, p->gy, p->gz};
    const int nf = with_g ? 9 : 6;
    for (int k = 0; k < nf; ++k)
        DZS_TRY(permute_one<double>(ctx, f64[k], perm, n, s));
    DZS_TRY(permute_one<uint32_t>(ctx, p->mult, perm, n, s));
    DZS_TRY(permute_one<uint32_t>(ctx, p->id, perm, n, s));
    DZS_TRY(permute_one<uint8_t>(ctx, p->type, perm, n, s));
    return DZS_OK;
}

// ---------------------------------------------------------------------------------------
// individual power-of-two time steps
// ---------------------------------------------------------------------------------------
// Bin of each particle for a global step of length Dl in ln a: the smallest b <= B with
// Dl 2^-b <= delta = sqrt(C eps / |g|), eps = eps0 mult^(1/3) (|g| = 0: bin 0).  With a
// limiter radius, the largest bin among particles inside the sphere is reduced (as bin + 1,
// 0 = nobody inside) into *cap.
__global__ __launch_bounds__(PT_THREADS) void k_hier_bins(
    uint64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const double *__restrict__ gx, const double *__restrict__ gy,
    const double *__restrict__ gz, const uint32_t *__restrict__ mult, double eps0, double C,
    double Dl, int B, double L, double xo0, double xo1, double xo2, double R_lim,
    uint8_t *__restrict__ bins, uint32_t *cap) {
    const uint64_t i = (uint64_t)blockIdx.x * PT_THREADS + threadIdx.x;
    uint32_t inside_bin = 0;
    if (i < n) {
        const double g2 = gx[i] * gx[i] + gy[i] * gy[i] + gz[i] * gz[i];
        const double gn = sqrt(g2);
        const double eps = eps0 * cbrt((double)mult[i]);
        const double delta = gn > 0.0 ? sqrt(C * eps / gn) : __builtin_inf();
        int b = 0;
        while (b < B && ldexp(Dl, -b) > delta)
            ++b;
        bins[i] = (uint8_t)b;
        if (cap) {
            const double dx = dzs_min_image(x[i] - xo0, L);
            const double dy = dzs_min_image(y[i] - xo1, L);
            const double dz = dzs_min_image(z[i] - xo2, L);
            if (sqrt(dx * dx + dy * dy + dz * dz) < R_lim)
                inside_bin = (uint32_t)b + 1u;
        }
    }
    if (cap) {
        for (int o = 32; o >= 1; o >>= 1)
            inside_bin = max(inside_bin, (uint32_t)__shfl_xor((int)inside_bin, o, 64));
        if ((threadIdx.x & 63u) == 0u && inside_bin > 0u)
            atomicMax(cap, inside_bin);
    }
}

__global__ __launch_bounds__(PT_THREADS) void k_hier_limit(
    uint64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, double L, double xo0, double xo1, double xo2, double R_lim,
    const uint32_t *__restrict__ cap, uint8_t *__restrict__ bins) {
    const uint64_t i = (uint64_t)blockIdx.x * PT_THREADS + threadIdx.x;
    if (i >= n || *cap == 0u)
        return;
    const double dx = dzs_min_image(x[i] - xo0, L);
    const double dy = dzs_min_image(y[i] - xo1, L);
    const double dz = dzs_min_image(z[i] - xo2, L);
    if (!(sqrt(dx * dx + dy * dy + dz * dz) < R_lim)) {
        const uint8_t c = (uint8_t)(*cap - 1u);
        if (bins[i] > c)
            bins[i] = c;
    }
}

__global__ __launch_bounds__(1) void k_hier_cap_clear(uint32_t *cap) { *cap = 0u; }

struct bin_factors {
    double K[DZS_HIER_MAX_BIN + 1];  // kick factor of each bin at this boundary (0: none)
};

// p += g K[bin] for the bins that kick at this boundary
__global__ __launch_bounds__(PT_THREADS) void k_kick_bins(
    uint64_t n, double *__restrict__ px, double *__restrict__ py, double *__restrict__ pz,
    const double *__restrict__ gx, const double *__restrict__ gy,
    const double *__restrict__ gz, const uint8_t *__restrict__ bins, bin_factors F) {
    const uint64_t i = (uint64_t)blockIdx.x * PT_THREADS + threadIdx.x;
    if (i >= n)
        return;
    const double K = F.K[bins[i]];
    if (K == 0.0)
        return;
    px[i] = px[i] + gx[i] * K;
    py[i] = py[i] + gy[i] * K;
    pz[i] = pz[i] + gz[i] * K;
}

dzs_status dzs_launch_hier_bins(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                                double C, double Dl, int B, const double *x_obs, double R_lim,
                                int limiter, uint8_t *bins, hipStream_t s) {
    if (p->n == 0)
        return DZS_OK;
    uint32_t *cap = limiter ? ctx->d_small + DZS_SMALL_HIER_CAP : nullptr;
    if (cap) {
        hipLaunchKernelGGL(k_hier_cap_clear, dim3(1), dim3(1), 0, s, cap);
        DZS_TRY(dzs_check_launch(ctx, "hier_cap_clear"));
    }
    const uint32_t b = blocks_for(p->n, PT_THREADS);
    hipLaunchKernelGGL(k_hier_bins, dim3(b), dim3(PT_THREADS), 0, s, p->n, (const double *)p->x,
                       (const double *)p->y, (const double *)p->z, (const double *)p->gx,
                       (const double *)p->gy, (const double *)p->gz, (const uint32_t *)p->mult,
                       box->eps0, C, Dl, B, box->L, x_obs[0], x_obs[1], x_obs[2], R_lim, bins,
                       cap);
    DZS_TRY(dzs_check_launch(ctx, "hier_bins"));
    if (cap) {
        hipLaunchKernelGGL(k_hier_limit, dim3(b), dim3(PT_THREADS), 0, s, p->n,
                           (const double *)p->x, (const double *)p->y, (const double *)p->z,
                           box->L, x_obs[0], x_obs[1], x_obs[2], R_lim, (const uint32_t *)cap,
                           bins);
        DZS_TRY(dzs_check_launch(ctx, "hier_limit"));
    }
    return DZS_OK;
}

dzs_status dzs_launch_kick_bins(dzs_ctx *ctx, const dzs_particles *p, const uint8_t *bins,
                                const double *K, hipStream_t s) {
    if (p->n == 0)
        return DZS_OK;
    bin_factors F;
    for (int b = 0; b <= DZS_HIER_MAX_BIN; ++b)
        F.K[b] = K[b];
    hipLaunchKernelGGL(k_kick_bins, dim3(blocks_for(p->n, PT_THREADS)), dim3(PT_THREADS), 0, s,
                       p->n, p->px, p->py, p->pz, (const double *)p->gx, (const double *)p->gy,
                       (const double *)p->gz, bins, F);
    return dzs_check_launch(ctx, "kick_bins");
}

dzs_status dzs_permute_u8(dzs_ctx *ctx, uint8_t *arr, const uint32_t *perm, uint64_t n,
                          hipStream_t s) {
    if (n == 0)
        return DZS_OK;
    return permute_one<uint8_t>(ctx, arr, perm, n, s);
}

// |g| of each particle (slot i takes particle perm[i] when perm is given), in FP32: the
// relative opening criterion's previous accelerations.
__global__ __launch_bounds__(PT_THREADS) void k_gnorm(uint64_t n, const double *__restrict__ gx,
                                                      const double *__restrict__ gy,
                                                      const double *__restrict__ gz,
                                                      const uint32_t *__restrict__ perm,
                                                      float *__restrict__ out) {
    const uint64_t i = (uint64_t)blockIdx.x * PT_THREADS + threadIdx.x;
    if (i >= n)
        return;
    const uint64_t j = perm ? perm[i] : i;
    out[i] = (float)sqrt(gx[j] * gx[j] + gy[j] * gy[j] + gz[j] * gz[j]);
}

dzs_status dzs_launch_gnorm(dzs_ctx *ctx, uint64_t n, const double *gx, const double *gy,
                            const double *gz, const uint32_t *perm, float *out, hipStream_t s) {
    if (n == 0)
        return DZS_OK;
    hipLaunchKernelGGL(k_gnorm, dim3(blocks_for(n, PT_THREADS)), dim3(PT_THREADS), 0, s, n, gx,
                       gy, gz, perm, out);
    return dzs_check_launch(ctx, "gnorm");
}

dzs_status dzs_permute_f32(dzs_ctx *ctx, float *arr, const uint32_t *perm, uint64_t n,
                           hipStream_t s) {
    if (n == 0)
        return DZS_OK;
    return permute_one<float>(ctx, arr, perm, n, s);
}

dzs_status dzs_gather_f64(dzs_ctx *ctx, const double *src, const uint32_t *perm, double *dst,
                          uint64_t n, hipStream_t s) {
    if (n == 0)
        return DZS_OK;
    hipLaunchKernelGGL(k_gather<double>, dim3(blocks_for(n, PT_THREADS)), dim3(PT_THREADS), 0, s,
                       n, src, perm, dst);
    return dzs_check_launch(ctx, "gather_f64");
}

dzs_status dzs_gather_u32(dzs_ctx *ctx, const uint32_t *src, const uint32_t *perm,
                          uint32_t *dst, uint64_t n, hipStream_t s) {
    if (n == 0)
        return DZS_OK;
    hipLaunchKernelGGL(k_gather<uint32_t>, dim3(blocks_for(n, PT_THREADS)), dim3(PT_THREADS), 0,
                       s, n, src, perm, dst);
    return dzs_check_launch(ctx, "gather_u32");
}

dzs_status dzs_gather_u8(dzs_ctx *ctx, const uint8_t *src, const uint32_t *perm, uint8_t *dst,
                         uint64_t n, hipStream_t s) {
    if (n == 0)
        return DZS_OK;
    hipLaunchKernelGGL(k_gather<uint8_t>, dim3(blocks_for(n, PT_THREADS)), dim3(PT_THREADS), 0,
                       s, n, src, perm, dst);
    return dzs_check_launch(ctx, "gather_u8");
}

// ---------------------------------------------------------------------------------------
// target flags of the walk
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(PT_THREADS) void k_fill_u8(uint64_t n, uint8_t *__restrict__ a,
                                                        uint8_t v) {
    const uint64_t i = (uint64_t)blockIdx.x * PT_THREADS + threadIdx.x;
    if (i < n)
        a[i] = v;
}

__global__ __launch_bounds__(PT_THREADS) void k_mark_targets(uint64_t nt,
                                                             const uint32_t *__restrict__ t,
                                                             uint64_t n, uint8_t *__restrict__ flags,
                                                             uint32_t *__restrict__ bad) {
    const uint64_t k = (uint64_t)blockIdx.x * PT_THREADS + threadIdx.x;
    if (k >= nt)
        return;
    const uint32_t i = t[k];
    if (i < n)
        flags[i] = 1u;
    else
        atomicOr(bad, 1u);
}

dzs_status dzs_mark_targets(dzs_ctx *ctx, const uint32_t *targets, uint64_t n_targets,
                            uint64_t n, uint8_t *flags, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u8, dim3(blocks_for(n, PT_THREADS)), dim3(PT_THREADS), 0, s, n,
                       flags, (uint8_t)0);
    DZS_TRY(dzs_check_launch(ctx, "fill_u8"));
    if (n_targets == 0)
        return DZS_OK;
    hipLaunchKernelGGL(k_mark_targets, dim3(blocks_for(n_targets, PT_THREADS)), dim3(PT_THREADS),
                       0, s, n_targets, targets, n, flags, ctx->bstate + DZS_BS_BADINPUT);
    return dzs_check_launch(ctx, "mark_targets");
}

__global__ __launch_bounds__(PT_THREADS) void k_hier_active(uint64_t n,
                                                            const uint8_t *__restrict__ bins,
                                                            uint32_t jn, uint32_t B,
                                                            uint8_t *__restrict__ active) {
    const uint64_t i = (uint64_t)blockIdx.x * PT_THREADS + threadIdx.x;
    if (i < n)
        active[i] = (jn & ((1u << (B - bins[i])) - 1u)) == 0u ? 1u : 0u;
}

__global__ void k_bin_hist_clear(uint32_t *counts) {
    for (int b = 0; b < 8; ++b)
        counts[b] = 0u;
}

__global__ __launch_bounds__(PT_THREADS) void k_bin_hist(uint64_t n,
                                                         const uint8_t *__restrict__ bins,
                                                         uint32_t *counts) {
    __shared__ uint32_t s_c[8];
    if (threadIdx.x < 8)
        s_c[threadIdx.x] = 0u;
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * PT_THREADS + threadIdx.x;
    if (i < n)
        atomicAdd(&s_c[bins[i] & 7u], 1u);
    __syncthreads();
    if (threadIdx.x < 8 && s_c[threadIdx.x])
        atomicAdd(&counts[threadIdx.x], s_c[threadIdx.x]);
}

dzs_status dzs_launch_bin_hist(dzs_ctx *ctx, uint64_t n, const uint8_t *bins, hipStream_t s) {
    uint32_t *counts = ctx->d_small + DZS_SMALL_BIN_COUNT;
    hipLaunchKernelGGL(k_bin_hist_clear, dim3(1), dim3(1), 0, s, counts);
    DZS_TRY(dzs_check_launch(ctx, "bin_hist_clear"));
    if (n == 0)
        return DZS_OK;
    hipLaunchKernelGGL(k_bin_hist, dim3(blocks_for(n, PT_THREADS)), dim3(PT_THREADS), 0, s, n,
                       bins, counts);
    return dzs_check_launch(ctx, "bin_hist");
}

dzs_status dzs_launch_hier_active(dzs_ctx *ctx, uint64_t n, const uint8_t *bins, uint32_t jn,
                                  uint32_t B, uint8_t *active, hipStream_t s) {
    if (n == 0)
        return DZS_OK;
    hipLaunchKernelGGL(k_hier_active, dim3(blocks_for(n, PT_THREADS)), dim3(PT_THREADS), 0, s, n,
                       bins, jn, B, active);
    return dzs_check_launch(ctx, "hier_active");
}
