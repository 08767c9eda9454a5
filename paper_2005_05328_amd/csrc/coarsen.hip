// DZS coarsening on the GPU (paper Sec. 2.2 and 2.2.1, eqs. 1 and 3).
//
// The paper walks the tree from the root and replaces every node that meets the merging
// criterion by one particle, without descending further.  Equivalently, every particle joins
// its shallowest qualifying ancestor.  On the GPU the levels are processed from k_min down
// to the finest: at level k the first particle of each level-k cube (a contiguous run of the
// (key, id)-sorted state) sums its cube's members in order — mult, mult*x and mult*p with
// Neumaier compensation — tests the criterion, and if it holds stamps the cube's members
// with its own index.  Particles stamped at a shallower level are skipped.  A compaction then
// writes survivors and one new particle per stamped cube, in sorted order.
//
// The node sums, the centre of mass, the minimum-image distance and the threshold comparison
// use the exact operation sequence of the definition (no contraction), so the grouping is
// bit-identical to any implementation that follows the same definition.
//
// Two criteria (Sec. 2.2.1): the geometric one (eq. 1 with eq. 3) compares |d|^2 with a
// per-level threshold; the dynamical one (eq. 2 with eq. 3) compares G m0 K l_k^2 with
// alpha a_min D^4, where a_min, the smallest previous acceleration inside the lightcone plus
// buffer, is reduced on the device beforehand (an order-independent minimum, so exact).
#include "internal.h"

#define DZ_THREADS 256
#define DZ_NONE 0xffffffffu

static inline uint32_t blocks_for(uint64_t n, uint32_t t) { return (uint32_t)((n + t - 1) / t); }

struct neumaier {
    double sum, comp;
};

__device__ __forceinline__ void nm_add(neumaier &a, double v) {
    const double t = a.sum + v;
    if (fabs(a.sum) >= fabs(v))
        a.comp += (a.sum - t) + v;
    else
        a.comp += (v - t) + a.sum;
    a.sum = t;
}

__device__ __forceinline__ double nm_value(const neumaier &a) { return a.sum + a.comp; }

struct dz_level_args {
    uint64_t n;
    int k, crit;
    double L, T2;
    double Gm0, lk2, Rb, alpha;       // dynamical criterion
    const unsigned long long *amin2;  // bits of min g.g inside the lightcone (device)
    double xo[3];
    const uint64_t *key;
    const double *x, *y, *z, *px, *py, *pz;
    const uint32_t *mult, *id;
    uint32_t *head;
    double *nx, *ny, *nz, *npx, *npy, *npz;
    uint32_t *nmult, *nid;
};

// Largest minimum-image |x - x_obs| along one axis over the cube [a, a + l), widened by a
// margin far above the rounding of the keys and of the centre of mass.
__device__ __forceinline__ double dz_axis_far(double a, double l, double xo, double L) {
    const double m = 1e-9 * L;
    const double u = a - m - xo, v = a + l + m - xo;
    // the farthest offset, L/2 (mod L), lies inside [u, v]
    if (ceil((u - 0.5 * L) / L) <= floor((v - 0.5 * L) / L))
        return 0.5 * L;
    const double wu = u - L * floor(u / L + 0.5), wv = v - L * floor(v / L + 0.5);
    return fmax(fabs(wu), fabs(wv));
}

__global__ __launch_bounds__(DZ_THREADS) void k_dz_level(dz_level_args A) {
    const uint64_t i = (uint64_t)blockIdx.x * DZ_THREADS + threadIdx.x;
    if (i >= A.n || A.head[i] != DZ_NONE)
        return;
    const int sh = 3 * (DZS_KEY_BITS - A.k);
    const uint64_t pk = A.key[i] >> sh;
    if (i > 0 && (A.key[i - 1] >> sh) == pk)
        return;  // not the first member of its level-k cube
    {
        // A cube whose every point is too close to merge is skipped before its members are
        // visited: this bound never excludes a cube the criterion would merge.
        const double l = ldexp(A.L, -A.k);
        const double fx = dz_axis_far((double)dzs_compact3(pk >> 2) * l, l, A.xo[0], A.L);
        const double fy = dz_axis_far((double)dzs_compact3(pk >> 1) * l, l, A.xo[1], A.L);
        const double fz = dz_axis_far((double)dzs_compact3(pk) * l, l, A.xo[2], A.L);
        const double far2 = fx * fx + fy * fy + fz * fz;
        if (A.crit == DZS_CRIT_GEOMETRIC) {
            if (far2 * (1.0 + 1e-12) <= A.T2)
                return;
        } else {
            const double Dmax = sqrt(far2) * (1.0 + 1e-12) - A.Rb;
            if (!(Dmax > 0.0))
                return;
            const double amin = sqrt(__longlong_as_double((long long)*A.amin2));
            const double D2 = Dmax * Dmax;
            if ((A.Gm0 * 2.0) * A.lk2 >= (A.alpha * amin) * (D2 * D2) * (1.0 + 1e-9))
                return;
        }
    }
    uint64_t e = i + 1;
    while (e < A.n && (A.key[e] >> sh) == pk)
        ++e;
    if (e - i < 2)
        return;
    neumaier S[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    neumaier P[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    uint64_t K = 0;
    uint32_t min_id = 0xffffffffu;
    for (uint64_t r = i; r < e; ++r) {
        const uint32_t mu = A.mult[r];
        const double m = (double)mu;
        K += mu;
        nm_add(S[0], m * A.x[r]);
        nm_add(S[1], m * A.y[r]);
        nm_add(S[2], m * A.z[r]);
        nm_add(P[0], m * A.px[r]);
        nm_add(P[1], m * A.py[r]);
        nm_add(P[2], m * A.pz[r]);
        const uint32_t idr = A.id[r];
        min_id = idr < min_id ? idr : min_id;
    }
    const double Kd = (double)K;
    const double X = dzs_wrap(nm_value(S[0]) / Kd, A.L);
    const double Y = dzs_wrap(nm_value(S[1]) / Kd, A.L);
    const double Z = dzs_wrap(nm_value(S[2]) / Kd, A.L);
    const double dx = dzs_min_image(X - A.xo[0], A.L);
    const double dy = dzs_min_image(Y - A.xo[1], A.L);
    const double dz = dzs_min_image(Z - A.xo[2], A.L);
    const double d2 = dx * dx + dy * dy + dz * dz;
    if (A.crit == DZS_CRIT_GEOMETRIC) {
        if (!(d2 > A.T2))
            return;
    } else {
        const double D = sqrt(d2) - A.Rb;
        if (!(D > 0.0))
            return;
        const double amin = sqrt(__longlong_as_double((long long)*A.amin2));
        const double lhs = (A.Gm0 * Kd) * A.lk2;
        const double rhs = (A.alpha * amin) * ((D * D) * (D * D));
        if (!(lhs < rhs))
            return;
    }
    for (uint64_t r = i; r < e; ++r)
        A.head[r] = (uint32_t)i;
    A.nx[i] = X;
    A.ny[i] = Y;
    A.nz[i] = Z;
    A.npx[i] = nm_value(P[0]) / Kd;
    A.npy[i] = nm_value(P[1]) / Kd;
    A.npz[i] = nm_value(P[2]) / Kd;
    A.nmult[i] = (uint32_t)K;
    A.nid[i] = min_id;
}

// The smallest g.g among particles strictly inside R_lc + b of the observer (minimum image);
// its bit pattern orders like the value because g.g >= 0, so blocks combine by an integer
// atomic minimum on a slot preset to +inf.
__global__ __launch_bounds__(1) void k_dz_amin_init(unsigned long long *out) {
    *out = 0x7ff0000000000000ull;
}

__global__ __launch_bounds__(DZ_THREADS) void k_dz_amin(uint64_t n, const double *__restrict__ x,
                                                       const double *__restrict__ y,
                                                       const double *__restrict__ z,
                                                       const double *__restrict__ gx,
                                                       const double *__restrict__ gy,
                                                       const double *__restrict__ gz, double L,
                                                       double xo0, double xo1, double xo2,
                                                       double Rb, unsigned long long *out) {
    __shared__ double red[DZ_THREADS];
    double best = __builtin_inf();
    const uint64_t stride = (uint64_t)gridDim.x * DZ_THREADS;
    for (uint64_t i = (uint64_t)blockIdx.x * DZ_THREADS + threadIdx.x; i < n; i += stride) {
        const double dx = dzs_min_image(x[i] - xo0, L);
        const double dy = dzs_min_image(y[i] - xo1, L);
        const double dz = dzs_min_image(z[i] - xo2, L);
        if (!(sqrt(dx * dx + dy * dy + dz * dz) < Rb))
            continue;
        const double g2 = gx[i] * gx[i] + gy[i] * gy[i] + gz[i] * gz[i];
        best = g2 < best ? g2 : best;
    }
    red[threadIdx.x] = best;
    __syncthreads();
    for (int h = DZ_THREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            const double o = red[threadIdx.x + h];
            red[threadIdx.x] = o < red[threadIdx.x] ? o : red[threadIdx.x];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        atomicMin(out, (unsigned long long)__double_as_longlong(red[0]));
}

dzs_status dzs_coarsen_amin(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                            const dzs_coarsen_params *prm, hipStream_t s) {
    unsigned long long *slot = (unsigned long long *)(ctx->d_small + DZS_SMALL_AMIN);
    hipLaunchKernelGGL(k_dz_amin_init, dim3(1), dim3(1), 0, s, slot);
    DZS_TRY(dzs_check_launch(ctx, "dz_amin_init"));
    if (p->n == 0)
        return DZS_OK;
    const uint64_t want = (p->n + DZ_THREADS - 1) / DZ_THREADS;
    const uint32_t blocks = (uint32_t)(want < 2048 ? want : 2048);
    hipLaunchKernelGGL(k_dz_amin, dim3(blocks), dim3(DZ_THREADS), 0, s, p->n,
                       (const double *)p->x, (const double *)p->y, (const double *)p->z,
                       (const double *)p->gx, (const double *)p->gy, (const double *)p->gz,
                       box->L, prm->x_obs[0], prm->x_obs[1], prm->x_obs[2], prm->R_lc + prm->b,
                       slot);
    return dzs_check_launch(ctx, "dz_amin");
}

// After a merge the state stays in key order (a merged particle takes its cube's first slot
// and its centre of mass lies in that cube), unless rounding put a centre of mass on the
// cube's far face: flag any descent.
__global__ __launch_bounds__(1) void k_dz_flag_clear(uint32_t *flag) { *flag = 0u; }

__global__ __launch_bounds__(DZ_THREADS) void k_dz_unsorted(uint64_t n, const uint64_t *key,
                                                           uint32_t *flag) {
    const uint64_t i = (uint64_t)blockIdx.x * DZ_THREADS + threadIdx.x;
    if (i + 1 < n && key[i] > key[i + 1])
        atomicOr(flag, 1u);
}

dzs_status dzs_coarsen_rekey(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                             bool *sorted, hipStream_t s) {
    *sorted = true;
    if (p->n < 2)
        return dzs_launch_keys(ctx, p->x, p->y, p->z, p->n, box->L, ctx->key, nullptr, s);
    DZS_TRY(dzs_launch_keys(ctx, p->x, p->y, p->z, p->n, box->L, ctx->key, nullptr, s));
    uint32_t *flag = ctx->d_small + DZS_SMALL_UNSORTED;
    hipLaunchKernelGGL(k_dz_flag_clear, dim3(1), dim3(1), 0, s, flag);
    DZS_TRY(dzs_check_launch(ctx, "dz_flag_clear"));
    hipLaunchKernelGGL(k_dz_unsorted, dim3(blocks_for(p->n, DZ_THREADS)), dim3(DZ_THREADS), 0, s,
                       p->n, (const uint64_t *)ctx->key, flag);
    DZS_TRY(dzs_check_launch(ctx, "dz_unsorted"));
    DZS_HIP(ctx, hipMemcpyAsync(ctx->h_small + DZS_SMALL_UNSORTED, flag, sizeof(uint32_t),
                                hipMemcpyDeviceToHost, s));
    DZS_HIP(ctx, hipStreamSynchronize(s));
    *sorted = ctx->h_small[DZS_SMALL_UNSORTED] == 0u;
    return DZS_OK;
}

__global__ __launch_bounds__(DZ_THREADS) void k_dz_init(uint64_t n, uint32_t *head) {
    const uint64_t i = (uint64_t)blockIdx.x * DZ_THREADS + threadIdx.x;
    if (i < n)
        head[i] = DZ_NONE;
}

// survivors and group heads emit one output particle each
__global__ __launch_bounds__(DZ_THREADS) void k_dz_flags(uint64_t n, const uint32_t *head,
                                                         uint32_t *flag) {
    const uint64_t i = (uint64_t)blockIdx.x * DZ_THREADS + threadIdx.x;
    if (i < n)
        flag[i] = (head[i] == DZ_NONE || head[i] == (uint32_t)i) ? 1u : 0u;
}

template <typename T>
__global__ __launch_bounds__(DZ_THREADS) void k_dz_emit(uint64_t n, const uint32_t *head,
                                                        const uint32_t *scan, const T *old_val,
                                                        const T *new_val, T *out) {
    const uint64_t i = (uint64_t)blockIdx.x * DZ_THREADS + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t h = head[i];
    if (h == DZ_NONE)
        out[scan[i]] = old_val[i];
    else if (h == (uint32_t)i)
        out[scan[i]] = new_val[i];
}

__global__ __launch_bounds__(DZ_THREADS) void k_dz_type(uint64_t n, const uint32_t *head,
                                                        const uint32_t *scan,
                                                        const uint8_t *old_type, uint8_t *out) {
    const uint64_t i = (uint64_t)blockIdx.x * DZ_THREADS + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t h = head[i];
    if (h == DZ_NONE)
        out[scan[i]] = old_type[i];
    else if (h == (uint32_t)i)
        out[scan[i]] = 1u;
}

__global__ __launch_bounds__(DZ_THREADS) void k_dz_groupmap(uint64_t n, const uint32_t *head,
                                                            const uint32_t *scan,
                                                            const uint32_t *perm,
                                                            uint32_t *group_of) {
    const uint64_t i = (uint64_t)blockIdx.x * DZ_THREADS + threadIdx.x;
    if (i >= n)
        return;
    const uint32_t h = head[i];
    group_of[perm[i]] = scan[h == DZ_NONE ? (uint32_t)i : h];
}

__global__ __launch_bounds__(DZ_THREADS) void k_dz_count_heads(uint64_t n, const uint32_t *head,
                                                               uint32_t *count) {
    const uint64_t i = (uint64_t)blockIdx.x * DZ_THREADS + threadIdx.x;
    const bool is_head = i < n && head[i] == (uint32_t)i;
    const uint64_t m = __ballot(is_head);
    if ((threadIdx.x & 63) == 0 && m)
        atomicAdd(count, (uint32_t)__popcll(m));
}

template <typename T>
__global__ __launch_bounds__(DZ_THREADS) void k_dz_copy(uint64_t n, const T *src, T *dst) {
    const uint64_t i = (uint64_t)blockIdx.x * DZ_THREADS + threadIdx.x;
    if (i < n)
        dst[i] = src[i];
}

template <typename T>
static dzs_status emit_field(dzs_ctx *ctx, uint64_t n, uint64_t n_new, T *arr, const T *new_val,
                             hipStream_t s) {
    T *tmp = (T *)ctx->gather_tmp;
    hipLaunchKernelGGL(k_dz_emit<T>, dim3(blocks_for(n, DZ_THREADS)), dim3(DZ_THREADS), 0, s, n,
                       (const uint32_t *)ctx->dz_head, (const uint32_t *)ctx->dz_scan,
                       (const T *)arr, new_val, tmp);
    DZS_TRY(dzs_check_launch(ctx, "dz_emit"));
    if (n_new > 0) {
        hipLaunchKernelGGL(k_dz_copy<T>, dim3(blocks_for(n_new, DZ_THREADS)), dim3(DZ_THREADS), 0,
                           s, n_new, (const T *)tmp, arr);
        DZS_TRY(dzs_check_launch(ctx, "dz_copy"));
    }
    return DZS_OK;
}

// State already sorted by (key, id) with ctx->key holding the sorted keys and ctx->dz_perm
// the entry index of each sorted slot.
dzs_status dzs_coarsen_sorted(dzs_ctx *ctx, const dzs_box *box, dzs_particles *p,
                              const dzs_coarsen_params *prm, uint32_t *group_of,
                              dzs_coarsen_report *report, hipStream_t s) {
    const uint64_t n = p->n;
    const bool dyn = prm->criterion == DZS_CRIT_DYNAMICAL;
    if (report) {
        report->n_before = n;
        report->n_after = n;
        report->n_groups = 0;
        report->a_min = dyn ? __builtin_inf() : __builtin_nan("");
    }
    if (n == 0)
        return DZS_OK;
    double T2[DZS_KEY_BITS + 1];
    dzs_merge_thresholds(box->L, prm->R_lc, prm->b, dyn ? 1.0 : prm->theta, T2);
    const uint64_t cap = ctx->cap_n;
    dz_level_args A;
    A.n = n;
    A.L = box->L;
    A.crit = dyn ? DZS_CRIT_DYNAMICAL : DZS_CRIT_GEOMETRIC;
    A.Gm0 = box->G * box->m0;
    A.Rb = prm->R_lc + prm->b;
    A.alpha = prm->alpha_dyn;
    A.amin2 = (const unsigned long long *)(ctx->d_small + DZS_SMALL_AMIN);
    for (int d = 0; d < 3; ++d)
        A.xo[d] = prm->x_obs[d];
    A.key = ctx->key;
    A.x = p->x; A.y = p->y; A.z = p->z; A.px = p->px; A.py = p->py; A.pz = p->pz;
    A.mult = p->mult;
    A.id = p->id;
    A.head = ctx->dz_head;
    A.nx = ctx->dz_new; A.ny = ctx->dz_new + cap; A.nz = ctx->dz_new + 2 * cap;
    A.npx = ctx->dz_new + 3 * cap; A.npy = ctx->dz_new + 4 * cap; A.npz = ctx->dz_new + 5 * cap;
    A.nmult = ctx->dz_newmult;
    A.nid = ctx->dz_newid;
    const uint32_t blocks = blocks_for(n, DZ_THREADS);
    {
        dzs_timed t(ctx, KC_DZS_LEVELS, s);
        hipLaunchKernelGGL(k_dz_init, dim3(blocks), dim3(DZ_THREADS), 0, s, n, ctx->dz_head);
        DZS_TRY(dzs_check_launch(ctx, "dz_init"));
        for (int k = prm->k_min; k <= DZS_KEY_BITS; ++k) {
            // geometric: no centre of mass lies beyond sqrt(3)/2 L (minimum image), so a level
            // whose threshold exceeds it cannot merge anything
            if (!dyn && T2[k] > 0.75 * box->L * box->L * (1.0 + 1e-9))
                continue;
            A.k = k;
            A.T2 = T2[k];
            const double lk = ldexp(box->L, -k);
            A.lk2 = lk * lk;
            hipLaunchKernelGGL(k_dz_level, dim3(blocks), dim3(DZ_THREADS), 0, s, A);
            DZS_TRY(dzs_check_launch(ctx, "dz_level"));
        }
    }
    uint64_t n_new, n_heads;
    {
        dzs_timed t(ctx, KC_DZS_COMPACT, s);
        hipLaunchKernelGGL(k_dz_flags, dim3(blocks), dim3(DZ_THREADS), 0, s, n,
                           (const uint32_t *)ctx->dz_head, ctx->dz_flag);
        DZS_TRY(dzs_check_launch(ctx, "dz_flags"));
        DZS_TRY(dzs_scan_u32(ctx, ctx->dz_flag, ctx->dz_scan, n, ctx->d_small + 8, s));
        DZS_HIP(ctx, hipMemsetAsync(ctx->d_small + 9, 0, sizeof(uint32_t), s));
        hipLaunchKernelGGL(k_dz_count_heads, dim3(blocks), dim3(DZ_THREADS), 0, s, n,
                           (const uint32_t *)ctx->dz_head, ctx->d_small + 9);
        DZS_TRY(dzs_check_launch(ctx, "dz_count_heads"));
        DZS_HIP(ctx, hipMemcpyAsync(ctx->h_small + 8, ctx->d_small + 8,
                                    (DZS_SMALL_AMIN + 2 - 8) * sizeof(uint32_t),
                                    hipMemcpyDeviceToHost, s));
        DZS_HIP(ctx, hipStreamSynchronize(s));
        n_new = ctx->h_small[8];
        n_heads = ctx->h_small[9];
        if (dyn && report) {
            unsigned long long bits;
            memcpy(&bits, ctx->h_small + DZS_SMALL_AMIN, sizeof(bits));
            double g2;
            memcpy(&g2, &bits, sizeof(g2));
            report->a_min = sqrt(g2);
        }
        if (group_of) {
            hipLaunchKernelGGL(k_dz_groupmap, dim3(blocks), dim3(DZ_THREADS), 0, s, n,
                               (const uint32_t *)ctx->dz_head, (const uint32_t *)ctx->dz_scan,
                               (const uint32_t *)ctx->dz_perm, group_of);
            DZS_TRY(dzs_check_launch(ctx, "dz_groupmap"));
        }
        if (n_new != n) {
            DZS_TRY(emit_field<double>(ctx, n, n_new, p->x, A.nx, s));
            DZS_TRY(emit_field<double>(ctx, n, n_new, p->y, A.ny, s));
            DZS_TRY(emit_field<double>(ctx, n, n_new, p->z, A.nz, s));
            DZS_TRY(emit_field<double>(ctx, n, n_new, p->px, A.npx, s));
            DZS_TRY(emit_field<double>(ctx, n, n_new, p->py, A.npy, s));
            DZS_TRY(emit_field<double>(ctx, n, n_new, p->pz, A.npz, s));
            DZS_TRY(emit_field<uint32_t>(ctx, n, n_new, p->mult, ctx->dz_newmult, s));
            DZS_TRY(emit_field<uint32_t>(ctx, n, n_new, p->id, ctx->dz_newid, s));
            uint8_t *tmp = (uint8_t *)ctx->gather_tmp;
            hipLaunchKernelGGL(k_dz_type, dim3(blocks), dim3(DZ_THREADS), 0, s, n,
                               (const uint32_t *)ctx->dz_head, (const uint32_t *)ctx->dz_scan,
                               (const uint8_t *)p->type, tmp);
            DZS_TRY(dzs_check_launch(ctx, "dz_type"));
            hipLaunchKernelGGL(k_dz_copy<uint8_t>, dim3(blocks_for(n_new, DZ_THREADS)),
                               dim3(DZ_THREADS), 0, s, n_new, (const uint8_t *)tmp, p->type);
            DZS_TRY(dzs_check_launch(ctx, "dz_copy_type"));
        }
    }
    if (report) {
        report->n_after = n_new;
        report->n_groups = n_heads;
    }
    p->n = n_new;
    return DZS_OK;
}
