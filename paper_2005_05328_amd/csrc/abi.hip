// The C ABI of libdzs: context lifetime, argument checks, orchestration of the step, and
// HIP-event timing of the kernel classes.
#include <math.h>
#include <stdarg.h>
#include <stdlib.h>

#include <vector>

#include "internal.h"

const char *const dzs_kclass_names[KC_COUNT] = {
    "kick",        "drift_lightcone", "morton_keys", "radix_sort",  "permute",
    "tree_build",  "tree_moments",    "tree_groups", "tree_walk",   "pm_deposit",
    "pm_fft_x",    "pm_fft_y",        "pm_fft_z_green", "pm_interp", "dzs_levels",
    "dzs_compact", "misc"};

dzs_status dzs_fail(dzs_ctx *ctx, dzs_status code, const char *fmt, ...) {
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

dzs_status dzs_check_launch(dzs_ctx *ctx, const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return dzs_fail(ctx, DZS_EHIP, "launch of %s failed: %s", what, hipGetErrorString(e));
    return DZS_OK;
}

// ---------------------------------------------------------------------------------------
// timing
// ---------------------------------------------------------------------------------------
static void drain_timers(dzs_ctx *ctx) {
    dzs_timer_pool *P = ctx->timers;
    if (!P)
        return;
    for (int i = 0; i < P->used; ++i) {
        float ms = 0.0f;
        if (hipEventSynchronize(P->stop[i]) == hipSuccess &&
            hipEventElapsedTime(&ms, P->start[i], P->stop[i]) == hipSuccess) {
            ctx->t_ms[P->cls[i]] += ms;
            ctx->t_calls[P->cls[i]] += 1;
        }
    }
    P->used = 0;
}

void dzs_time_begin(dzs_ctx *ctx, int cls, hipStream_t s, int *slot) {
    *slot = -1;
    if (!ctx->timing || !ctx->timers || !((ctx->timing_mask >> cls) & 1u))
        return;
    dzs_timer_pool *P = ctx->timers;
    if (P->used >= dzs_timer_pool::CAP)
        drain_timers(ctx);
    const int k = P->used++;
    P->cls[k] = cls;
    if (hipEventRecord(P->start[k], s) == hipSuccess)
        *slot = k;
    else
        P->used--;
}

void dzs_time_end(dzs_ctx *ctx, hipStream_t s, int slot) {
    if (slot < 0)
        return;
    (void)hipEventRecord(ctx->timers->stop[slot], s);
}

extern "C" dzs_status dzs_counters(dzs_ctx *ctx, int32_t reset, uint64_t *pair_interactions) {
    if (!ctx || !pair_interactions)
        return DZS_EINVAL;
    uint64_t v = 0;
    DZS_HIP(ctx, hipDeviceSynchronize());
    DZS_HIP(ctx, hipMemcpy(&v, ctx->walk_counter + 8, sizeof(uint64_t), hipMemcpyDeviceToHost));
    *pair_interactions = v;
    if (reset)
        DZS_HIP(ctx, hipMemset(ctx->walk_counter + 8, 0, sizeof(uint64_t)));
    return DZS_OK;
}

extern "C" int32_t dzs_timing(dzs_ctx *ctx, int32_t enable, int32_t reset, const char **names,
                              double *ms_avg, uint64_t *calls, int32_t cap) {
    if (!ctx)
        return 0;
    if (enable < 0) {  // names only
        int32_t w = 0;
        for (int c = 0; c < KC_COUNT && w < cap; ++c)
            if (names)
                names[w++] = dzs_kclass_names[c];
            else
                ++w;
        return w;
    }
    if (enable > 0 && !ctx->timers) {
        ctx->timers = new dzs_timer_pool();
        for (int i = 0; i < dzs_timer_pool::CAP; ++i) {
            (void)hipEventCreate(&ctx->timers->start[i]);
            (void)hipEventCreate(&ctx->timers->stop[i]);
        }
        ctx->timers->created = true;
    }
    drain_timers(ctx);
    int32_t w = 0;
    for (int c = 0; c < KC_COUNT && w < cap; ++c) {
        if (names)
            names[w] = dzs_kclass_names[c];
        if (ms_avg)
            ms_avg[w] = ctx->t_calls[c] ? ctx->t_ms[c] / (double)ctx->t_calls[c] : 0.0;
        if (calls)
            calls[w] = ctx->t_calls[c];
        ++w;
    }
    if (reset) {
        for (int c = 0; c < KC_COUNT; ++c) {
            ctx->t_ms[c] = 0.0;
            ctx->t_calls[c] = 0;
        }
    }
    ctx->timing = enable != 0;
    ctx->timing_mask = enable > 1 ? (uint32_t)enable >> 1 : 0xffffffffu;
    return w;
}

// ---------------------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------------------
template <typename T>
static dzs_status alloc(dzs_ctx *ctx, T **p, uint64_t count) {
    void *v = nullptr;
    uint64_t bytes = sizeof(T) * (count > 0 ? count : 1);
    hipError_t e = hipMalloc(&v, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return dzs_fail(ctx, DZS_ENOMEM, "hipMalloc of %llu bytes failed: %s",
                        (unsigned long long)bytes, hipGetErrorString(e));
    }
    *p = (T *)v;
    return DZS_OK;
}

static void release(dzs_ctx *ctx) {
    void *ptrs[] = {ctx->key, ctx->key_alt, ctx->idx, ctx->idx_alt, ctx->hist, ctx->hist_scan,
                    ctx->scan_tmp, ctx->sx, ctx->sy, ctx->sz, ctx->smult, ctx->aold,
                    ctx->hbins, ctx->active, ctx->gpm, ctx->grp_list, ctx->tg_flag,
                    ctx->tg_tscan, ctx->tg_gscan, ctx->tg_pos, ctx->arena, ctx->bstate, ctx->grp_first,
                    ctx->walk_stack, ctx->walk_counter, ctx->cell_node, ctx->cell_dl,
                    ctx->batch_box, ctx->batch_tab, ctx->batch_first, ctx->batch_members,
                    ctx->step_dev, ctx->fp32_meshes ? nullptr : (void *)ctx->mesh_q, ctx->mesh_c,
                    ctx->mesh_phi,
                    ctx->pm_tables, ctx->d_small};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
    if (ctx->pm_stream)
        (void)hipStreamDestroy(ctx->pm_stream);
    if (ctx->ev_fork)
        (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_pm)
        (void)hipEventDestroy(ctx->ev_pm);
    if (ctx->h_small)
        (void)hipHostFree(ctx->h_small);
    if (ctx->batch_box_h)
        (void)hipHostFree(ctx->batch_box_h);
    if (ctx->batch_first_h)
        (void)hipHostFree(ctx->batch_first_h);
    if (ctx->step_h)
        (void)hipHostFree(ctx->step_h);
    if (ctx->timers) {
        for (int i = 0; i < dzs_timer_pool::CAP; ++i) {
            (void)hipEventDestroy(ctx->timers->start[i]);
            (void)hipEventDestroy(ctx->timers->stop[i]);
        }
        delete ctx->timers;
    }
}

static dzs_status create(dzs_ctx *c, const dzs_capacity *cap) {
    const uint64_t n = cap->max_particles + 64;
    const uint64_t ng = cap->max_mesh_side;
    const uint64_t ng3 = ng * ng * ng;
    c->cap_n = n;
    c->cap_ng = (uint32_t)ng;
    DZS_TRY(alloc(c, &c->key, n));
    DZS_TRY(alloc(c, &c->key_alt, n));
    DZS_TRY(alloc(c, &c->idx, n));
    DZS_TRY(alloc(c, &c->idx_alt, n));
    c->hist_cap = dzs_sort_hist_words(n);
    DZS_TRY(alloc(c, &c->hist, c->hist_cap));
    DZS_TRY(alloc(c, &c->hist_scan, c->hist_cap));
    uint64_t scan_n = n > c->hist_cap ? n : c->hist_cap;
    c->scan_tmp_cap = dzs_scan_tmp_words(scan_n);
    DZS_TRY(alloc(c, &c->scan_tmp, c->scan_tmp_cap));
    // the permutation scratch shares the sort's ping-pong keys (free once a sort returns)
    c->gather_tmp = (double *)c->key_alt;
    // One arena holds, at different times, the tree (nodes, which live from the build to the
    // end of the walk, plus the build's frontier scratch and the group flags) and the DZS
    // coarsening buffers (used before the tree of the same step is built).  Nodes: at most
    // n/2 + 4096 (internal nodes hold more than one particle; the build flags an overflow).
    const uint64_t nn = n / 2 + 4096;
    c->cap_nodes = nn;
    uint64_t off_t = 0, off_d = 0;
    auto carve = [](uint64_t &off, uint64_t bytes) {
        const uint64_t at = off;
        off += (bytes + 255) & ~255ull;
        return at;
    };
    const uint64_t o_first = carve(off_t, 4 * nn), o_count = carve(off_t, 4 * nn),
                   o_child = carve(off_t, 4 * nn), o_nchild = carve(off_t, nn),
                   o_level = carve(off_t, nn), o_rec = carve(off_t, sizeof(dzs_node_rec) * nn),
                   o_fr = carve(off_t, 4 * nn), o_frn = carve(off_t, 4 * nn),
                   o_nc = carve(off_t, 4 * nn), o_ni = carve(off_t, 4 * nn),
                   o_co = carve(off_t, 4 * nn), o_io = carve(off_t, 4 * nn),
                   o_cb = carve(off_t, 36 * nn), o_gf = carve(off_t, 4 * n),
                   o_gs = carve(off_t, 4 * n);
    const uint64_t o_head = carve(off_d, 4 * n), o_flag = carve(off_d, 4 * n),
                   o_scan = carve(off_d, 4 * n), o_new = carve(off_d, 48 * n),
                   o_nmult = carve(off_d, 4 * n), o_nid = carve(off_d, 4 * n),
                   o_perm = carve(off_d, 4 * n);
    DZS_TRY(alloc(c, &c->arena, off_t > off_d ? off_t : off_d));
    c->arena_bytes = off_t > off_d ? off_t : off_d;
    char *A = c->arena;
    c->nd_first = (uint32_t *)(A + o_first);
    c->nd_count = (uint32_t *)(A + o_count);
    c->nd_child = (uint32_t *)(A + o_child);
    c->nd_nchild = (uint8_t *)(A + o_nchild);
    c->nd_level = (uint8_t *)(A + o_level);
    c->nd_rec = (dzs_node_rec *)(A + o_rec);
    c->frontier = (uint32_t *)(A + o_fr);
    c->frontier_next = (uint32_t *)(A + o_frn);
    c->fr_nchild = (uint32_t *)(A + o_nc);
    c->fr_ninternal = (uint32_t *)(A + o_ni);
    c->fr_child_off = (uint32_t *)(A + o_co);
    c->fr_int_off = (uint32_t *)(A + o_io);
    c->child_bounds = (uint32_t *)(A + o_cb);
    c->grp_flag = (uint32_t *)(A + o_gf);
    c->grp_scan = (uint32_t *)(A + o_gs);
    c->dz_head = (uint32_t *)(A + o_head);
    c->dz_flag = (uint32_t *)(A + o_flag);
    c->dz_scan = (uint32_t *)(A + o_scan);
    c->dz_new = (double *)(A + o_new);
    c->dz_newmult = (uint32_t *)(A + o_nmult);
    c->dz_newid = (uint32_t *)(A + o_nid);
    c->dz_perm = (uint32_t *)(A + o_perm);
    DZS_TRY(alloc(c, &c->bstate, 64));
    DZS_HIP(c, hipMemset(c->bstate, 0, 64 * sizeof(uint32_t)));
    DZS_TRY(alloc(c, &c->grp_first, n + 1));
    c->walk_stack_slots = 4096;
    c->walk_stack_depth = 8192;
    DZS_TRY(alloc(c, &c->walk_stack, c->walk_stack_slots * c->walk_stack_depth));
    DZS_TRY(alloc(c, &c->walk_counter, 64));
    DZS_HIP(c, hipMemset(c->walk_counter, 0, 64 * sizeof(uint32_t)));
    DZS_TRY(alloc(c, &c->cell_node, 1ull << (3 * DZS_CELL_K_MAX)));
    // the relative criterion's |g|, the time-step bins and the walk's target flags
    DZS_TRY(alloc(c, &c->aold, n));
    DZS_TRY(alloc(c, &c->hbins, n));
    DZS_TRY(alloc(c, &c->active, n));
    if (cap->flags & DZS_CAP_HIER_SPLIT) {
        DZS_TRY(alloc(c, &c->gpm, 3 * n));
        DZS_TRY(alloc(c, &c->grp_list, n));
        DZS_TRY(alloc(c, &c->tg_flag, n));
        DZS_TRY(alloc(c, &c->tg_tscan, n));
        DZS_TRY(alloc(c, &c->tg_gscan, n));
        DZS_TRY(alloc(c, &c->tg_pos, n + 1));
    }
    if (!(cap->flags & DZS_CAP_NO_COPIES)) {
        // tree_force's sorted copies of an input in any order
        DZS_TRY(alloc(c, &c->sx, n));
        DZS_TRY(alloc(c, &c->sy, n));
        DZS_TRY(alloc(c, &c->sz, n));
        DZS_TRY(alloc(c, &c->smult, n));
    }
    const uint32_t nbox = cap->max_boxes ? cap->max_boxes : DZS_BATCH_MAX;
    c->cap_boxes = nbox;
    DZS_TRY(alloc(c, &c->batch_box, nbox));
    DZS_TRY(alloc(c, &c->batch_first, nbox + 1));
    DZS_TRY(alloc(c, &c->batch_members, nbox));
    if (ng > 0) {
        // per box 2 ng (Green factors, k^2) and per distinct mesh side 2 ng (twiddles)
        c->batch_tab_cap = 4ull * nbox * ng;
        DZS_TRY(alloc(c, &c->batch_tab, c->batch_tab_cap));
    }
    DZS_TRY(alloc(c, &c->step_dev, 1));
    {
        void *hb = nullptr, *hf = nullptr, *hs = nullptr;
        DZS_HIP(c, hipHostMalloc(&hb, sizeof(dzs_bbox) * nbox, hipHostMallocDefault));
        c->batch_box_h = (dzs_bbox *)hb;
        DZS_HIP(c, hipHostMalloc(&hf, sizeof(uint64_t) * (nbox + 1), hipHostMallocDefault));
        c->batch_first_h = (uint64_t *)hf;
        DZS_HIP(c, hipHostMalloc(&hs, sizeof(dzs_step_block), hipHostMallocDefault));
        c->step_h = (dzs_step_block *)hs;
    }
    DZS_TRY(alloc(c, &c->cell_dl, 1ull << (3 * DZS_CELL_K_MAX)));
    if (ng > 0) {
        c->fp32_meshes = (cap->flags & DZS_CAP_FP32_MESHES) != 0;
        if (c->fp32_meshes) {
            // precision form only: 8-byte complex cells hold the 8-byte fixed-point deposit
            // in place (the first FFT pass reads a tile, then writes it), 4-byte potential
            char *m = nullptr;
            DZS_TRY(alloc(c, &m, 8 * ng3));
            c->mesh_c = (double2 *)m;
            c->mesh_q = (long long *)m;
            char *ph = nullptr;
            DZS_TRY(alloc(c, &ph, 4 * ng3));
            c->mesh_phi = (double *)ph;
        } else {
            DZS_TRY(alloc(c, &c->mesh_q, ng3));
            DZS_TRY(alloc(c, &c->mesh_c, ng3));
            DZS_TRY(alloc(c, &c->mesh_phi, ng3));
        }
        DZS_TRY(alloc(c, &c->pm_tables, 4 * ng));
    }
    DZS_TRY(alloc(c, &c->d_small, 64));
    void *h = nullptr;
    DZS_HIP(c, hipHostMalloc(&h, 64 * sizeof(uint32_t), hipHostMallocDefault));
    c->h_small = (uint32_t *)h;
    memset(c->h_small, 0, 64 * sizeof(uint32_t));
    return DZS_OK;
}

extern "C" dzs_status dzs_ctx_create(dzs_ctx **out, int32_t device, const dzs_capacity *cap) {
    if (!out || !cap || cap->max_particles == 0 || cap->max_particles > 0xfffff000ull ||
        cap->max_boxes > DZS_BATCH_MAX || cap->reserved != 0 ||
        (cap->flags & ~(DZS_CAP_FP32_MESHES | DZS_CAP_NO_COPIES | DZS_CAP_HIER_SPLIT)) != 0)
        return DZS_EINVAL;
    if (cap->max_mesh_side != 0 && (cap->max_mesh_side < 8 || cap->max_mesh_side > 1024))
        return DZS_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return DZS_EHIP;
    if (hipSetDevice(device) != hipSuccess)
        return DZS_EHIP;
    dzs_ctx *c = new dzs_ctx();
    c->device = device;
    dzs_status st = create(c, cap);
    if (st != DZS_OK) {
        release(c);
        delete c;
        return st;
    }
    *out = c;
    return DZS_OK;
}

extern "C" dzs_status dzs_ctx_destroy(dzs_ctx *ctx) {
    if (!ctx)
        return DZS_EINVAL;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    release(ctx);
    delete ctx;
    return DZS_OK;
}

extern "C" const char *dzs_last_error(const dzs_ctx *ctx) { return ctx ? ctx->err : "no context"; }

// ---------------------------------------------------------------------------------------
// argument checks
// ---------------------------------------------------------------------------------------
static dzs_status check_common(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p) {
    if (!ctx)
        return DZS_EINVAL;
    ctx->err[0] = 0;
    if (!box || !p)
        return dzs_fail(ctx, DZS_EINVAL, "null box or particle view");
    if (!(box->L > 0.0) || !(box->m0 > 0.0) || !(box->eps0 > 0.0) || !(box->G > 0.0))
        return dzs_fail(ctx, DZS_EINVAL, "box L, m0, eps0 and G must be positive");
    if (p->n > p->capacity)
        return dzs_fail(ctx, DZS_EINVAL, "n (%llu) exceeds the view's capacity (%llu)",
                        (unsigned long long)p->n, (unsigned long long)p->capacity);
    if (p->n + 64 > ctx->cap_n)
        return dzs_fail(ctx, DZS_ECAPACITY, "n (%llu) exceeds the context capacity (%llu)",
                        (unsigned long long)p->n, (unsigned long long)(ctx->cap_n - 64));
    if (p->n > 0 && (!p->x || !p->y || !p->z || !p->mult))
        return dzs_fail(ctx, DZS_EINVAL, "null position or multiplicity array");
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != ctx->device)
        DZS_HIP(ctx, hipSetDevice(ctx->device));
    return DZS_OK;
}

static dzs_status check_tree(dzs_ctx *ctx, const dzs_box *box, const dzs_tree_params *t,
                             dzs_tree_params *out) {
    if (!t)
        return dzs_fail(ctx, DZS_EINVAL, "null tree parameters");
    *out = *t;
    if (out->leaf_size == 0)
        out->leaf_size = 8;
    if (out->group_size == 0)
        out->group_size = 16;
    if (!(t->r_s > 0.0) || !(t->r_cut > 0.0) || !(t->r_cut < 0.5 * box->L) || !(t->theta >= 0.0))
        return dzs_fail(ctx, DZS_EINVAL, "tree: need r_s > 0, 0 < r_cut < L/2, theta >= 0");
    if (out->leaf_size < 1 || out->leaf_size > 64 || out->group_size < 1 ||
        out->group_size > 64 || (out->group_size & (out->group_size - 1)) != 0)
        return dzs_fail(ctx, DZS_EINVAL,
                        "tree: leaf_size must be in 1..64, group_size a power of two <= 64");
    if (t->r_cut > 5.0 * t->r_s)
        return dzs_fail(ctx, DZS_EINVAL, "tree: r_cut must not exceed 5 r_s");
    if (t->precision != DZS_FP64 && t->precision != DZS_FP32)
        return dzs_fail(ctx, DZS_EINVAL, "tree: precision must be DZS_FP64 or DZS_FP32");
    if (t->opening != DZS_OPEN_GEOMETRIC && t->opening != DZS_OPEN_RELATIVE)
        return dzs_fail(ctx, DZS_EINVAL, "tree: unknown opening criterion %d", t->opening);
    if (t->opening == DZS_OPEN_RELATIVE && !(t->alpha_open >= 0.0 && t->alpha_open < HUGE_VAL))
        return dzs_fail(ctx, DZS_EINVAL, "tree: the relative criterion needs a finite "
                        "alpha_open >= 0");
    return DZS_OK;
}

static dzs_status check_pm(dzs_ctx *ctx, const dzs_pm_params *m) {
    if (!m)
        return dzs_fail(ctx, DZS_EINVAL, "null PM parameters");
    if (!dzs_pm_mesh_ok(m->ng))
        return dzs_fail(ctx, DZS_EINVAL, "pm: mesh side %d must be an even 2^a 3^b in [8, 1024]", m->ng);
    if ((uint32_t)m->ng > ctx->cap_ng)
        return dzs_fail(ctx, DZS_ECAPACITY, "pm: mesh side %d exceeds the context's %u", m->ng,
                        ctx->cap_ng);
    if (!(m->r_s > 0.0))
        return dzs_fail(ctx, DZS_EINVAL, "pm: r_s must be positive");
    if (m->precision != DZS_FP64 && m->precision != DZS_FP32)
        return dzs_fail(ctx, DZS_EINVAL, "pm: precision must be DZS_FP64 or DZS_FP32");
    const int32_t dc = m->tile_chunk;
    if (dc != 0 && dc != -1 &&
        (dc < DZS_PM_CHUNK_MIN || dc > DZS_PM_CHUNK_MAX || (dc & (dc - 1)) != 0))
        return dzs_fail(ctx, DZS_EINVAL, "pm: tile_chunk %d must be 0, -1 or a power of two "
                        "in [%d, %d]", dc, DZS_PM_CHUNK_MIN, DZS_PM_CHUNK_MAX);
    if (m->precision == DZS_FP64 && ctx->fp32_meshes)
        return dzs_fail(ctx, DZS_EINVAL, "pm: the context holds meshes for the precision form "
                        "only (DZS_CAP_FP32_MESHES)");
    return DZS_OK;
}

static dzs_status check_coarsen(dzs_ctx *ctx, const dzs_coarsen_params *c) {
    if (!c)
        return dzs_fail(ctx, DZS_EINVAL, "null coarsening parameters");
    if (c->criterion != DZS_CRIT_GEOMETRIC && c->criterion != DZS_CRIT_DYNAMICAL)
        return dzs_fail(ctx, DZS_EINVAL, "coarsen: unknown criterion %d", c->criterion);
    if (c->criterion == DZS_CRIT_GEOMETRIC && !(c->theta > 0.0))
        return dzs_fail(ctx, DZS_EINVAL, "coarsen: the geometric criterion needs theta > 0");
    if (c->criterion == DZS_CRIT_DYNAMICAL && !(c->alpha_dyn >= 0.0 && c->alpha_dyn < HUGE_VAL))
        return dzs_fail(ctx, DZS_EINVAL, "coarsen: the dynamical criterion needs a finite "
                        "alpha_dyn >= 0");
    if (c->k_min < 1 || c->k_min > DZS_KEY_BITS || !(c->R_lc >= 0.0) || !(c->b >= 0.0))
        return dzs_fail(ctx, DZS_EINVAL, "coarsen: need 1 <= k_min <= 21, R_lc, b >= 0");
    return DZS_OK;
}

static dzs_status check_lc(dzs_ctx *ctx, const dzs_lc_params *lc, const dzs_lc_ring *ring) {
    if (!lc || !ring || !ring->records || !ring->count || !ring->overflow)
        return dzs_fail(ctx, DZS_EINVAL, "lightcone: null parameters or ring");
    if (lc->n_cheb < 1 || lc->n_cheb > DZS_CHEB_MAX || !(lc->a1 > lc->a0))
        return dzs_fail(ctx, DZS_EINVAL, "lightcone: need 1 <= n_cheb <= %d and a1 > a0",
                        DZS_CHEB_MAX);
    return DZS_OK;
}

// The second stream (default priority, non-blocking) and the events of kdk_step's overlap.
static dzs_status ensure_pm_stream(dzs_ctx *ctx) {
    if (ctx->pm_stream)
        return DZS_OK;
    DZS_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    DZS_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_pm, hipEventDisableTiming));
    DZS_HIP(ctx, hipStreamCreateWithFlags(&ctx->pm_stream, hipStreamNonBlocking));
    return DZS_OK;
}

// ---------------------------------------------------------------------------------------
// sorting the state
// ---------------------------------------------------------------------------------------
// tree_only: the order a tree build needs (keys ordered to level DZS_TREE_LEVELS, stable), not
// the full key order
static dzs_status sort_state(dzs_ctx *ctx, const dzs_box *box, dzs_particles *p, int ties_by_id,
                             int with_g, hipStream_t s, bool tree_only = false) {
    DZS_TRY(dzs_launch_keys(ctx, p->x, p->y, p->z, p->n, box->L, ctx->key, ctx->idx, s));
    DZS_TRY(dzs_radix_sort(ctx, p->n, s, tree_only ? DZS_TREE_FIRST_PASS : 0));
    if (ties_by_id)
        DZS_TRY(dzs_fix_ties(ctx, p->n, p->id, s));
    return dzs_permute_state(ctx, p, ctx->idx, with_g, s);
}

extern "C" dzs_status dzs_morton_keys(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                                      uint64_t *keys, void *stream) {
    DZS_TRY(check_common(ctx, box, p));
    if (!keys && p->n)
        return dzs_fail(ctx, DZS_EINVAL, "null keys");
    return dzs_launch_keys(ctx, p->x, p->y, p->z, p->n, box->L, keys, nullptr,
                           (hipStream_t)stream);
}

extern "C" dzs_status dzs_sort_state(dzs_ctx *ctx, const dzs_box *box, dzs_particles *p,
                                     int32_t ties_by_id, uint32_t *perm, void *stream) {
    DZS_TRY(check_common(ctx, box, p));
    if (p->n > 0 && (!p->px || !p->py || !p->pz || !p->id || !p->type || !p->gx || !p->gy ||
                     !p->gz))
        return dzs_fail(ctx, DZS_EINVAL, "null state array");
    hipStream_t s = (hipStream_t)stream;
    DZS_TRY(sort_state(ctx, box, p, ties_by_id, 1, s));
    if (perm && p->n)
        DZS_HIP(ctx, hipMemcpyAsync(perm, ctx->idx, sizeof(uint32_t) * p->n,
                                    hipMemcpyDeviceToDevice, s));
    return DZS_OK;
}

// ---------------------------------------------------------------------------------------
// the five calls
// ---------------------------------------------------------------------------------------
extern "C" dzs_status dzs_coarsen(dzs_ctx *ctx, const dzs_box *box, dzs_particles *inout,
                                  const dzs_coarsen_params *prm, uint32_t *group_of,
                                  dzs_coarsen_report *report, void *stream) {
    DZS_TRY(check_common(ctx, box, inout));
    DZS_TRY(check_coarsen(ctx, prm));
    if (inout->n > 0 && (!inout->px || !inout->py || !inout->pz || !inout->id || !inout->type))
        return dzs_fail(ctx, DZS_EINVAL, "null state array");
    const bool dyn = prm->criterion == DZS_CRIT_DYNAMICAL;
    if (dyn && inout->n > 0 && (!inout->gx || !inout->gy || !inout->gz))
        return dzs_fail(ctx, DZS_EINVAL, "coarsen: the dynamical criterion reads g (null)");
    hipStream_t s = (hipStream_t)stream;
    if (inout->n == 0) {
        if (report)
            *report = dzs_coarsen_report{0, 0, 0, dyn ? HUGE_VAL : NAN};
        return DZS_OK;
    }
    if (dyn)  // before the sort, which leaves g behind
        DZS_TRY(dzs_coarsen_amin(ctx, box, inout, prm, s));
    DZS_TRY(sort_state(ctx, box, inout, 1, 0, s));
    DZS_HIP(ctx, hipMemcpyAsync(ctx->dz_perm, ctx->idx, sizeof(uint32_t) * inout->n,
                                hipMemcpyDeviceToDevice, s));
    return dzs_coarsen_sorted(ctx, box, inout, prm, group_of, report, s);
}

extern "C" dzs_status pm_force(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                               const dzs_pm_params *prm, void *stream) {
    DZS_TRY(check_common(ctx, box, p));
    DZS_TRY(check_pm(ctx, prm));
    if (p->n > 0 && (!p->gx || !p->gy || !p->gz))
        return dzs_fail(ctx, DZS_EINVAL, "null acceleration array");
    return dzs_pm_run(ctx, box, p, prm, (hipStream_t)stream);
}

extern "C" dzs_status tree_force(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                                 const dzs_tree_params *prm, const uint32_t *targets,
                                 uint64_t n_targets, void *stream) {
    DZS_TRY(check_common(ctx, box, p));
    dzs_tree_params t;
    DZS_TRY(check_tree(ctx, box, prm, &t));
    if (p->n > 0 && (!p->gx || !p->gy || !p->gz))
        return dzs_fail(ctx, DZS_EINVAL, "null acceleration array");
    if (t.presorted != 0 && t.presorted != 1)
        return dzs_fail(ctx, DZS_EINVAL, "tree: presorted must be 0 or 1");
    if (!t.presorted && !ctx->sx)
        return dzs_fail(ctx, DZS_EINVAL, "tree: the context has no sorted copies "
                        "(DZS_CAP_NO_COPIES): pass particles in key order with presorted = 1");
    if (targets && n_targets > p->n)
        return dzs_fail(ctx, DZS_EINVAL, "tree: %llu targets for %llu particles",
                        (unsigned long long)n_targets, (unsigned long long)p->n);
    const uint64_t n = p->n;
    if (n == 0 || (targets && n_targets == 0))
        return DZS_OK;
    hipStream_t s = (hipStream_t)stream;
    const bool sorted_in = t.presorted != 0;
    const double *tx = p->x, *ty = p->y, *tz = p->z;
    const uint32_t *tm = p->mult;
    const uint32_t *perm = nullptr;  // tree slot -> entry index (none: the same)
    DZS_TRY(dzs_launch_keys(ctx, p->x, p->y, p->z, n, box->L, ctx->key, ctx->idx, s));
    if (sorted_in) {
        DZS_TRY(dzs_check_order(ctx, n, s));
    } else {
        DZS_TRY(dzs_radix_sort(ctx, n, s, DZS_TREE_FIRST_PASS));
        dzs_timed tm_(ctx, KC_PERMUTE, s);
        DZS_TRY(dzs_gather_f64(ctx, p->x, ctx->idx, ctx->sx, n, s));
        DZS_TRY(dzs_gather_f64(ctx, p->y, ctx->idx, ctx->sy, n, s));
        DZS_TRY(dzs_gather_f64(ctx, p->z, ctx->idx, ctx->sz, n, s));
        DZS_TRY(dzs_gather_u32(ctx, p->mult, ctx->idx, ctx->smult, n, s));
        tx = ctx->sx;
        ty = ctx->sy;
        tz = ctx->sz;
        tm = ctx->smult;
        perm = ctx->idx;
    }
    const uint8_t *active = nullptr;
    if (targets) {
        // the targets' flags in tree order (entry-order flags staged in the sort's free
        // ping-pong keys when the tree order differs)
        uint8_t *flags = sorted_in ? ctx->active : (uint8_t *)ctx->key_alt;
        DZS_TRY(dzs_mark_targets(ctx, targets, n_targets, n, flags, s));
        if (!sorted_in)
            DZS_TRY(dzs_gather_u8(ctx, flags, perm, ctx->active, n, s));
        active = ctx->active;
    }
    const float *aold = nullptr;
    if (t.opening == DZS_OPEN_RELATIVE) {
        // the targets' |g| on entry, in tree order
        DZS_TRY(dzs_launch_gnorm(ctx, n, p->gx, p->gy, p->gz, perm, ctx->aold, s));
        aold = ctx->aold;
    }
    DZS_TRY(dzs_tree_build(ctx, box, n, tx, ty, tz, tm, t.leaf_size, t.group_size, s));
    dzs_walk_io io;
    io.aold = aold;
    io.active = active;
    io.out_perm = perm;
    DZS_TRY(dzs_tree_walk(ctx, box, n, tx, ty, tz, tm, p->gx, p->gy, p->gz, &t, s, io));
    return dzs_latch_bad_input(ctx, s);
}

// ---------------------------------------------------------------------------------------
// PM force without any allocation: the meshes in a static device array of the library
// ---------------------------------------------------------------------------------------
#define NOALLOC_CELLS ((uint64_t)DZS_PM_NOALLOC_MAX_SIDE * DZS_PM_NOALLOC_MAX_SIDE * \
                       DZS_PM_NOALLOC_MAX_SIDE)
#define NOALLOC_DEVICES 64
// fixed-point density (8 B/cell), complex work mesh (16), potential (8), per-axis tables
static __device__ __align__(256) unsigned char
    scratch[32 * NOALLOC_CELLS + 4 * sizeof(double) * DZS_PM_NOALLOC_MAX_SIDE];

// Per device: a context shell whose meshes point into that device's copy of scratch.
struct noalloc_pm {
    bool ready = false;
    dzs_ctx shell;
    double host_tab[4 * DZS_PM_NOALLOC_MAX_SIDE];
};
static noalloc_pm g_noalloc[NOALLOC_DEVICES];

extern "C" dzs_status pm_force_noalloc(const dzs_box *box, const dzs_particles *p,
                                       const dzs_pm_params *prm, void *stream) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return DZS_EHIP;
    }
    if (dev < 0 || dev >= NOALLOC_DEVICES)
        return DZS_EINVAL;
    noalloc_pm &S = g_noalloc[dev];
    if (!S.ready) {
        // the device's own copy of the array: its address, looked up once with that device
        // current (the array's name is a host-side stand-in, not a device address)
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return DZS_EHIP;
        }
        char *base = (char *)ptr;
        dzs_ctx &c = S.shell;
        c.device = dev;
        c.cap_n = ~0ull >> 1;  // the PM keeps no per-particle scratch
        c.cap_ng = DZS_PM_NOALLOC_MAX_SIDE;
        c.mesh_q = (long long *)base;
        c.mesh_c = (double2 *)(base + 8 * NOALLOC_CELLS);
        c.mesh_phi = (double *)(base + 24 * NOALLOC_CELLS);
        c.pm_tables = (double *)(base + 32 * NOALLOC_CELLS);
        c.pm_host_tab = S.host_tab;
        S.ready = true;
    }
    dzs_ctx *ctx = &S.shell;
    DZS_TRY(check_common(ctx, box, p));
    DZS_TRY(check_pm(ctx, prm));
    if (p->n > 0 && (!p->gx || !p->gy || !p->gz))
        return dzs_fail(ctx, DZS_EINVAL, "null acceleration array");
    return dzs_pm_run(ctx, box, p, prm, (hipStream_t)stream);
}

extern "C" dzs_status lightcone_emit(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                                     const dzs_lc_params *prm, dzs_lc_ring *ring, void *stream) {
    DZS_TRY(check_common(ctx, box, p));
    DZS_TRY(check_lc(ctx, prm, ring));
    if (p->n > 0 && (!p->px || !p->py || !p->pz || !p->id))
        return dzs_fail(ctx, DZS_EINVAL, "null state array");
    return dzs_launch_drift_lc(ctx, box, p, prm, ring, 1, 0, (hipStream_t)stream);
}

extern "C" dzs_status kdk_step(dzs_ctx *ctx, const dzs_box *box, dzs_particles *st,
                               const dzs_step_params *prm, dzs_lc_ring *ring,
                               dzs_coarsen_report *report, void *stream) {
    DZS_TRY(check_common(ctx, box, st));
    if (!prm)
        return dzs_fail(ctx, DZS_EINVAL, "null step parameters");
    if (st->n > 0 && (!st->px || !st->py || !st->pz || !st->gx || !st->gy || !st->gz || !st->id ||
                      !st->type))
        return dzs_fail(ctx, DZS_EINVAL, "null state array");
    dzs_tree_params t;
    DZS_TRY(check_tree(ctx, box, &prm->tree, &t));
    DZS_TRY(check_pm(ctx, &prm->pm));
    if (prm->do_lightcone)
        DZS_TRY(check_lc(ctx, &prm->lc, ring));
    else if (!(prm->lc.D == prm->lc.D))
        return dzs_fail(ctx, DZS_EINVAL, "step: drift factor is NaN");
    if (prm->do_coarsen)
        DZS_TRY(check_coarsen(ctx, &prm->coarsen));
    hipStream_t s = (hipStream_t)stream;
    if (report)
        *report = dzs_coarsen_report{st->n, st->n, 0, NAN};

    // relative opening: the accelerations held on entry, carried through every reordering;
    // lost (geometric fallback) when the coarsening merges particles
    const bool relative = t.opening == DZS_OPEN_RELATIVE && st->n > 0;
    bool aold_ok = relative;
    if (relative)
        DZS_TRY(dzs_launch_gnorm(ctx, st->n, st->gx, st->gy, st->gz, nullptr, ctx->aold, s));
    DZS_TRY(dzs_launch_kick(ctx, st, prm->K1, s));
    DZS_TRY(dzs_launch_drift_lc(ctx, box, st, &prm->lc, ring, prm->do_lightcone, 1, s));
    const bool can_merge = prm->do_coarsen &&
                           prm->coarsen.R_lc + prm->coarsen.b < 0.5 * sqrt(3.0) * box->L;
    // the state in key order for the tree: after DZS it already is (the coarsening sorts by
    // (key, id) and a merged particle stays in its cube's slot); only new keys are needed,
    // with a full sort if rounding moved a centre of mass out of its cube
    bool in_order = false;
    if (can_merge && st->n > 0) {
        if (prm->coarsen.criterion == DZS_CRIT_DYNAMICAL)  // g is the previous force here
            DZS_TRY(dzs_coarsen_amin(ctx, box, st, &prm->coarsen, s));
        DZS_TRY(sort_state(ctx, box, st, 1, 0, s));
        if (aold_ok)
            DZS_TRY(dzs_permute_f32(ctx, ctx->aold, ctx->idx, st->n, s));
        DZS_HIP(ctx, hipMemcpyAsync(ctx->dz_perm, ctx->idx, sizeof(uint32_t) * st->n,
                                    hipMemcpyDeviceToDevice, s));
        const uint64_t n_in = st->n;
        DZS_TRY(dzs_coarsen_sorted(ctx, box, st, &prm->coarsen, nullptr, report, s));
        if (st->n == n_in) {
            in_order = true;  // nothing merged: the sort's keys still hold
        } else {
            aold_ok = false;
            DZS_TRY(dzs_coarsen_rekey(ctx, box, st, &in_order, s));
        }
    }
    if (st->n > 0) {
        if (!in_order) {
            DZS_TRY(sort_state(ctx, box, st, 0, 0, s, true));
            if (aold_ok)
                DZS_TRY(dzs_permute_f32(ctx, ctx->aold, ctx->idx, st->n, s));
        }
        // the mesh solve (deposit, FFTs) runs on the context's second stream while this one
        // builds the tree (many small launches and a few host read-backs that leave most of
        // the GPU idle); the walk starts after both, alone on the GPU (overlapping it with the
        // FFTs slowed the 512^3 walk by 7%)
        DZS_TRY(ensure_pm_stream(ctx));
        DZS_HIP(ctx, hipEventRecord(ctx->ev_fork, s));
        DZS_HIP(ctx, hipStreamWaitEvent(ctx->pm_stream, ctx->ev_fork, 0));
        dzs_pm_params pm = prm->pm;
        pm.accumulate = 0;
        DZS_TRY(dzs_pm_solve(ctx, box, st, &pm, ctx->pm_stream));
        DZS_HIP(ctx, hipEventRecord(ctx->ev_pm, ctx->pm_stream));
        DZS_TRY(dzs_tree_build(ctx, box, st->n, st->x, st->y, st->z, st->mult, t.leaf_size,
                               t.group_size, s));
        DZS_HIP(ctx, hipStreamWaitEvent(s, ctx->ev_pm, 0));
        DZS_TRY(dzs_pm_apply(ctx, box, st, &pm, s));
        t.accumulate = 1;
        dzs_walk_io io;
        io.aold = aold_ok ? ctx->aold : nullptr;
        DZS_TRY(dzs_tree_walk(ctx, box, st->n, st->x, st->y, st->z, st->mult, st->gx, st->gy,
                              st->gz, &t, s, io));
        DZS_TRY(dzs_launch_kick(ctx, st, prm->K2, s));
    }
    return DZS_OK;
}

// ---------------------------------------------------------------------------------------
// individual time steps
// ---------------------------------------------------------------------------------------
// The force of the targets that end a step at sub-step boundary jn (all when bins is null):
// key order, tree, PM for everyone, the walk for the active targets only.
static dzs_status hier_force(dzs_ctx *ctx, const dzs_box *box, dzs_particles *st,
                             const dzs_step_params *prm, const dzs_tree_params &t0,
                             const uint8_t *bins, uint32_t jn, uint32_t B, bool in_order,
                             hipStream_t s) {
    if (st->n == 0)
        return DZS_OK;
    if (!in_order) {
        DZS_TRY(sort_state(ctx, box, st, 0, 0, s, true));
        if (bins)
            DZS_TRY(dzs_permute_u8(ctx, ctx->hbins, ctx->idx, st->n, s));
    }
    dzs_tree_params t = t0;
    // the mesh solve overlaps the tree build, as in kdk_step
    DZS_TRY(ensure_pm_stream(ctx));
    DZS_HIP(ctx, hipEventRecord(ctx->ev_fork, s));
    DZS_HIP(ctx, hipStreamWaitEvent(ctx->pm_stream, ctx->ev_fork, 0));
    dzs_pm_params pm = prm->pm;
    pm.accumulate = 0;
    DZS_TRY(dzs_pm_solve(ctx, box, st, &pm, ctx->pm_stream));
    DZS_HIP(ctx, hipEventRecord(ctx->ev_pm, ctx->pm_stream));
    DZS_TRY(dzs_tree_build(ctx, box, st->n, st->x, st->y, st->z, st->mult, t.leaf_size,
                           t.group_size, s));
    DZS_HIP(ctx, hipStreamWaitEvent(s, ctx->ev_pm, 0));
    DZS_TRY(dzs_pm_apply(ctx, box, st, &pm, s));
    t.accumulate = 1;
    // the targets that end a step at this boundary (all when bins is null)
    dzs_walk_io io;
    if (bins) {
        DZS_TRY(dzs_launch_hier_active(ctx, st->n, bins, jn, B, ctx->active, s));
        io.active = ctx->active;
        if (ctx->grp_list && jn < (1u << B)) {
            // a part of the targets: walked in groups of consecutive active targets
            DZS_TRY(dzs_tree_active_targets(ctx, st->n, ctx->active, s));
            io.target_list = true;
        }
    }
    return dzs_tree_walk(ctx, box, st->n, st->x, st->y, st->z, st->mult, st->gx, st->gy, st->gz,
                         &t, s, io);
}

extern "C" dzs_status kdk_step_hier(dzs_ctx *ctx, const dzs_box *box, dzs_particles *st,
                                    const dzs_step_params *prm, const dzs_hier_params *hp,
                                    dzs_lc_ring *ring, dzs_coarsen_report *report,
                                    uint8_t *bins_out, void *stream) {
    DZS_TRY(check_common(ctx, box, st));
    if (!prm || !hp)
        return dzs_fail(ctx, DZS_EINVAL, "hier: null parameters");
    if (st->n > 0 && (!st->px || !st->py || !st->pz || !st->gx || !st->gy || !st->gz || !st->id ||
                      !st->type))
        return dzs_fail(ctx, DZS_EINVAL, "null state array");
    dzs_tree_params t;
    DZS_TRY(check_tree(ctx, box, &prm->tree, &t));
    if (t.opening != DZS_OPEN_GEOMETRIC)
        return dzs_fail(ctx, DZS_EINVAL, "hier: only the geometric opening criterion");
    DZS_TRY(check_pm(ctx, &prm->pm));
    if (prm->do_lightcone && (!ring || !ring->records || !ring->count || !ring->overflow))
        return dzs_fail(ctx, DZS_EINVAL, "hier: null lightcone ring");
    if (prm->do_coarsen)
        DZS_TRY(check_coarsen(ctx, &prm->coarsen));
    if (hp->pm_global != 0 && hp->pm_global != 1)
        return dzs_fail(ctx, DZS_EINVAL, "hier: pm_global must be 0 or 1");
    if (hp->reserved != 0)
        return dzs_fail(ctx, DZS_EINVAL, "hier: reserved must be 0");
    if (hp->pm_global && !ctx->gpm)
        return dzs_fail(ctx, DZS_EINVAL, "hier: pm_global needs a context created with "
                        "DZS_CAP_HIER_SPLIT");
    const int B = hp->max_bin;
    if (B < 0 || B > DZS_HIER_MAX_BIN || !(hp->eta > 0.0) || !(hp->a0 > 0.0) ||
        !(hp->a1 > hp->a0) || !(hp->a1 <= 1.0) || !(hp->omega_m > 0.0) ||
        !(hp->omega_m <= 1.0) || (hp->limiter && !(hp->R_lim >= 0.0)))
        return dzs_fail(ctx, DZS_EINVAL, "hier: need 0 <= max_bin <= %d, eta > 0, "
                        "0 < a0 < a1 <= 1, 0 < omega_m <= 1, R_lim >= 0", DZS_HIER_MAX_BIN);
    hipStream_t s = (hipStream_t)stream;
    if (report)
        *report = dzs_coarsen_report{st->n, st->n, 0, NAN};
    const int S = 1 << B;
    const double om = hp->omega_m, a0 = hp->a0, a1 = hp->a1;
    const double Dl = log(a1 / a0);
    // half-sub-step grid, uniform in ln a, ends exact
    std::vector<double> u(2 * S + 1);
    for (int k = 0; k <= 2 * S; ++k)
        u[k] = exp(log(a0) + Dl * k / (2 * S));
    u[0] = a0;
    u[2 * S] = a1;
    if (st->n > 0) {
        const double H = 100.0 * sqrt(om / (a0 * a0 * a0) + (1.0 - om));
        const double C = 2.0 * hp->eta * (a0 * a0 * a0) * (H * H);
        DZS_TRY(dzs_launch_hier_bins(ctx, box, st, C, Dl, B, prm->coarsen.x_obs, hp->R_lim,
                                     hp->limiter, ctx->hbins, s));
        if (bins_out)
            DZS_HIP(ctx, hipMemcpyAsync(bins_out, ctx->hbins, st->n, hipMemcpyDeviceToDevice, s));
    }
    // which bins hold particles: a sub-step boundary where none of them ends a step has no
    // target and is skipped
    bool populated[8] = {false};
    if (st->n > 0) {
        DZS_TRY(dzs_launch_bin_hist(ctx, st->n, ctx->hbins, s));
        DZS_HIP(ctx, hipMemcpyAsync(ctx->h_small + DZS_SMALL_BIN_COUNT,
                                    ctx->d_small + DZS_SMALL_BIN_COUNT, 8 * sizeof(uint32_t),
                                    hipMemcpyDeviceToHost, s));
        DZS_HIP(ctx, hipStreamSynchronize(s));
        for (int b = 0; b <= B; ++b)
            populated[b] = ctx->h_small[DZS_SMALL_BIN_COUNT + b] != 0u;
    }
    auto ends_here = [&](int jn) {
        for (int b = 0; b <= B; ++b)
            if (populated[b] && jn % (1 << (B - b)) == 0)
                return true;
        return false;
    };
    // the long-range force on the global step: state in key order and tree once, at a0; the
    // PM force at a0 (into gpm) opens the step with its half-kick and leaves g the short-range
    // part of the entry force
    const bool split = hp->pm_global != 0 && st->n > 0;
    dzs_particles pmv = *st;   // the state with gpm as its force
    if (split) {
        pmv.gx = ctx->gpm;
        pmv.gy = ctx->gpm + ctx->cap_n;
        pmv.gz = ctx->gpm + 2 * ctx->cap_n;
        DZS_TRY(sort_state(ctx, box, st, 0, 1, s, true));   // the entry force moves along
        DZS_TRY(dzs_permute_u8(ctx, ctx->hbins, ctx->idx, st->n, s));
        pmv.n = st->n;
        dzs_pm_params pm = prm->pm;
        pm.accumulate = 0;
        DZS_TRY(dzs_pm_solve(ctx, box, &pmv, &pm, s));
        DZS_TRY(dzs_pm_apply(ctx, box, &pmv, &pm, s));
        DZS_TRY(dzs_launch_add3(ctx, st->n, st->gx, st->gy, st->gz, pmv.gx, pmv.gy, pmv.gz, -1.0,
                                s));
        DZS_TRY(dzs_launch_kick(ctx, &pmv, dzs_kick_factor(a0, u[S], om), s));
        DZS_TRY(dzs_tree_build(ctx, box, st->n, st->x, st->y, st->z, st->mult, t.leaf_size,
                               t.group_size, s));
        DZS_TRY(dzs_drift_bound_reset(ctx, s));
    }
    for (int j = 0; j < S && st->n > 0; ++j) {
        double K[DZS_HIER_MAX_BIN + 1] = {0.0};
        for (int b = 0; b <= B; ++b) {
            const int L = 1 << (B - b);
            if (j % L == 0)
                K[b] = dzs_kick_factor(u[2 * j], u[2 * j + L], om);
        }
        DZS_TRY(dzs_launch_kick_bins(ctx, st, ctx->hbins, K, s));
        dzs_step_params sub = *prm;
        DZS_TRY(dzs_step_factors(u[2 * j], u[2 * j + 2], om, &sub));
        if (split)   // the kept tree's walk widens its start cells by the displacement bound
            DZS_TRY(dzs_drift_bound_add(ctx, st, sub.lc.D, s));
        DZS_TRY(dzs_launch_drift_lc(ctx, box, st, &sub.lc, ring, prm->do_lightcone, 1, s));
        const int jn = j + 1;
        if (!ends_here(jn)) {
            // no particle ends a step here: no force, no kick
        } else if (split) {
            // the short-range force of the targets that end a step here, on the kept tree
            DZS_TRY(dzs_tree_refresh(ctx, box, st->n, st->x, st->y, st->z, st->mult, s));
            DZS_TRY(dzs_launch_hier_active(ctx, st->n, ctx->hbins, (uint32_t)jn, (uint32_t)B,
                                           ctx->active, s));
            dzs_tree_params ts = t;
            ts.accumulate = 0;
            dzs_walk_io io;
            io.active = ctx->active;
            io.kept_tree = true;
            if (jn < S) {
                // a part of the targets: walked in groups of consecutive active targets
                DZS_TRY(dzs_tree_active_targets(ctx, st->n, ctx->active, s));
                io.target_list = true;
            }
            DZS_TRY(dzs_tree_walk(ctx, box, st->n, st->x, st->y, st->z, st->mult, st->gx,
                                  st->gy, st->gz, &ts, s, io));
        } else {
            DZS_TRY(hier_force(ctx, box, st, prm, t, ctx->hbins, (uint32_t)jn, (uint32_t)B,
                               false, s));
        }
        for (int b = 0; b <= B; ++b) {
            const int L = 1 << (B - b);
            K[b] = jn % L == 0 ? dzs_kick_factor(u[2 * jn - L], u[2 * jn], om) : 0.0;
        }
        DZS_TRY(dzs_launch_kick_bins(ctx, st, ctx->hbins, K, s));
    }
    if (split) {
        // the PM force at a1 closes the step; the state keeps g_PM + g_SR
        dzs_pm_params pm = prm->pm;
        pm.accumulate = 0;
        DZS_TRY(dzs_pm_solve(ctx, box, &pmv, &pm, s));
        DZS_TRY(dzs_pm_apply(ctx, box, &pmv, &pm, s));
        DZS_TRY(dzs_launch_kick(ctx, &pmv, dzs_kick_factor(u[S], a1, om), s));
        DZS_TRY(dzs_launch_add3(ctx, st->n, st->gx, st->gy, st->gz, pmv.gx, pmv.gy, pmv.gz, 1.0,
                                s));
    }
    // every particle is synchronised at a1: DZS, then a new force if anything merged
    const bool can_merge = prm->do_coarsen &&
                           prm->coarsen.R_lc + prm->coarsen.b < 0.5 * sqrt(3.0) * box->L;
    if (can_merge && st->n > 0) {
        if (prm->coarsen.criterion == DZS_CRIT_DYNAMICAL)
            DZS_TRY(dzs_coarsen_amin(ctx, box, st, &prm->coarsen, s));
        DZS_TRY(sort_state(ctx, box, st, 1, 1, s));
        DZS_HIP(ctx, hipMemcpyAsync(ctx->dz_perm, ctx->idx, sizeof(uint32_t) * st->n,
                                    hipMemcpyDeviceToDevice, s));
        const uint64_t n_in = st->n;
        DZS_TRY(dzs_coarsen_sorted(ctx, box, st, &prm->coarsen, nullptr, report, s));
        if (st->n != n_in && st->n > 0) {
            bool in_order = false;
            DZS_TRY(dzs_coarsen_rekey(ctx, box, st, &in_order, s));
            DZS_TRY(hier_force(ctx, box, st, prm, t, nullptr, 0u, 0u, in_order, s));
        }
    }
    // the sub-steps' tree capacities and stack depths
    return dzs_tree_check(ctx, s);
}

// ---------------------------------------------------------------------------------------
// batched step
// ---------------------------------------------------------------------------------------
extern "C" dzs_status kdk_step_batch(dzs_ctx *ctx, const dzs_batch *batch, dzs_particles *st,
                                     const dzs_step_params *prm, dzs_lc_ring *ring,
                                     void *stream) {
    if (!ctx)
        return DZS_EINVAL;
    ctx->err[0] = 0;
    if (!batch || !st || !prm || !batch->boxes || !batch->first || !batch->ng || !batch->r_s ||
        !batch->r_cut)
        return dzs_fail(ctx, DZS_EINVAL, "batch: null argument");
    const uint32_t nb = batch->n_boxes;
    if (nb < 1 || nb > DZS_BATCH_MAX)
        return dzs_fail(ctx, DZS_EINVAL, "batch: need 1 <= n_boxes <= %d", DZS_BATCH_MAX);
    if (nb > ctx->cap_boxes)
        return dzs_fail(ctx, DZS_ECAPACITY, "batch: %u boxes exceed the context's %u", nb,
                        ctx->cap_boxes);
    if (batch->first[0] != 0 || batch->first[nb] != st->n)
        return dzs_fail(ctx, DZS_EINVAL, "batch: first[0] must be 0 and first[n_boxes] = n");
    if (st->n > st->capacity || st->n > ctx->cap_n || st->n >= (1ull << 32))
        return dzs_fail(ctx, DZS_ECAPACITY, "batch: %llu particles exceed the capacity",
                        (unsigned long long)st->n);
    if (st->n > 0 && (!st->x || !st->y || !st->z || !st->px || !st->py || !st->pz || !st->gx ||
                      !st->gy || !st->gz || !st->mult || !st->id || !st->type))
        return dzs_fail(ctx, DZS_EINVAL, "batch: null state array");
    if (prm->do_coarsen)
        return dzs_fail(ctx, DZS_EINVAL, "batch: coarsening runs per box (dzs_coarsen), not in "
                        "the batched step");
    if (prm->tree.opening != DZS_OPEN_GEOMETRIC)
        return dzs_fail(ctx, DZS_EINVAL, "batch: only the geometric opening criterion");
    dzs_tree_params t, t_in = prm->tree;
    t_in.r_s = batch->r_s[0];
    t_in.r_cut = batch->r_cut[0];
    DZS_TRY(check_tree(ctx, &batch->boxes[0], &t_in, &t));
    if (prm->pm.precision != DZS_FP64 && prm->pm.precision != DZS_FP32)
        return dzs_fail(ctx, DZS_EINVAL, "batch: PM precision must be DZS_FP64 or DZS_FP32");
    if (prm->pm.precision == DZS_FP64 && ctx->fp32_meshes)
        return dzs_fail(ctx, DZS_EINVAL, "batch: the context holds meshes for the precision "
                        "form only (DZS_CAP_FP32_MESHES)");
    if (prm->do_lightcone)
        DZS_TRY(check_lc(ctx, &prm->lc, ring));
    const double ratio = batch->r_cut[0] / batch->r_s[0];
    std::vector<dzs_bbox> tb(nb);
    for (uint32_t b = 0; b < nb; ++b) {
        const dzs_box &bx = batch->boxes[b];
        const double rs = batch->r_s[b], rc = batch->r_cut[b];
        if (batch->first[b + 1] < batch->first[b])
            return dzs_fail(ctx, DZS_EINVAL, "batch: first[] must not decrease");
        if (!(bx.L > 0.0) || !(bx.m0 > 0.0) || !(bx.eps0 > 0.0) || bx.G != batch->boxes[0].G)
            return dzs_fail(ctx, DZS_EINVAL, "batch: box %u needs L, m0, eps0 > 0 and the same G "
                            "as box 0", b);
        if (!(rs > 0.0) || !(rc > 0.0) || !(rc < 0.5 * bx.L) || rc > 5.0 * rs ||
            fabs(rc / rs - ratio) > 1e-12 * ratio)
            return dzs_fail(ctx, DZS_EINVAL, "batch: box %u needs 0 < r_cut < L/2, r_cut <= 5 r_s "
                            "and the r_cut / r_s of box 0", b);
        dzs_bbox &h = tb[b];
        memset(&h, 0, sizeof(h));
        h.L = bx.L;
        h.halfL = 0.5 * bx.L;
        h.m0 = bx.m0;
        h.h0 = 2.8 * bx.eps0;
        h.G = bx.G;
        h.r_s = rs;
        h.r_cut = rc;
        h.rcut2 = rc * rc;
        h.rs_inv = 1.0 / rs;
        h.rs_inv2 = h.rs_inv * h.rs_inv;
        h.wide_limit = 0.5 * (h.halfL - rc);   // see the walk's minimum-image rule
        h.first = batch->first[b];
        h.count = batch->first[b + 1] - batch->first[b];
        h.ng = batch->ng[b];
        h.root = 0xffffffffu;
    }
    hipStream_t s = (hipStream_t)stream;
    // the box tables, particle offsets and mesh tables are uploaded when the batch changes;
    // a repeated batch (the steps of one run, or a captured step) reuses them without any
    // host synchronisation
    bool same = ctx->batch_ready && ctx->batch_nb == nb;
    for (uint32_t b = 0; same && b < nb; ++b) {
        const dzs_bbox &o = ctx->batch_box_h[b], &n = tb[b];
        same = o.L == n.L && o.m0 == n.m0 && o.h0 == n.h0 && o.G == n.G && o.r_s == n.r_s &&
               o.r_cut == n.r_cut && o.first == n.first && o.count == n.count && o.ng == n.ng;
    }
    if (!same) {
        ctx->batch_ready = false;
        DZS_HIP(ctx, hipStreamSynchronize(s));  // the staging buffers may be in use
        memcpy(ctx->batch_box_h, tb.data(), sizeof(dzs_bbox) * nb);
        DZS_TRY(dzs_pm_batch_prepare(ctx, nb, ctx->batch_box_h, s));
        for (uint32_t b = 0; b <= nb; ++b)
            ctx->batch_first_h[b] = batch->first[b];
        DZS_HIP(ctx, hipMemcpyAsync(ctx->batch_box, ctx->batch_box_h, sizeof(dzs_bbox) * nb,
                                    hipMemcpyHostToDevice, s));
        DZS_HIP(ctx, hipMemcpyAsync(ctx->batch_first, ctx->batch_first_h,
                                    sizeof(uint64_t) * (nb + 1), hipMemcpyHostToDevice, s));
        DZS_HIP(ctx, hipStreamSynchronize(s));
        ctx->batch_nb = nb;
        ctx->batch_ready = true;
    }
    // Eager calls pass this step's factors as kernel arguments.  Under graph capture they are
    // read from a device block that a captured copy fills, when the graph runs, from the
    // pinned staging (written here and by kdk_step_batch_stage between replays); eager calls
    // do not use the staging, whose copy could still be pending when the next call writes it.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    DZS_HIP(ctx, hipStreamIsCapturing(s, &cs));
    const bool captured = cs == hipStreamCaptureStatusActive;
    if (captured) {
        ctx->step_h->K1 = prm->K1;
        ctx->step_h->K2 = prm->K2;
        dzs_make_lc_args(&prm->lc, &ctx->step_h->lc);
        DZS_HIP(ctx, hipMemcpyAsync(ctx->step_dev, ctx->step_h, sizeof(dzs_step_block),
                                    hipMemcpyHostToDevice, s));
    }
    const double *K1_dev = captured ? &ctx->step_dev->K1 : nullptr;
    const double *K2_dev = captured ? &ctx->step_dev->K2 : nullptr;
    const lc_args *lc_dev = captured ? &ctx->step_dev->lc : nullptr;
    if (st->n == 0)
        return DZS_OK;

    DZS_TRY(dzs_launch_kick(ctx, st, prm->K1, s, K1_dev));
    DZS_TRY(dzs_launch_drift_lc(ctx, &batch->boxes[0], st, &prm->lc, ring, prm->do_lightcone, 1,
                                s, true, nb, lc_dev));
    // keys with the box on top, one sort for every box: each box stays in its range
    DZS_TRY(dzs_launch_keys(ctx, st->x, st->y, st->z, st->n, 1.0, ctx->key, ctx->idx, s, true,
                            nb));
    DZS_TRY(dzs_radix_sort(ctx, st->n, s, DZS_TREE_FIRST_PASS));
    DZS_TRY(dzs_permute_state(ctx, st, ctx->idx, 0, s));
    DZS_TRY(dzs_tree_build_ex(ctx, &batch->boxes[0], st->n, st->x, st->y, st->z, st->mult,
                              t.leaf_size, t.group_size, DZS_BATCH_LEVELS, ctx->batch_box, s));
    DZS_TRY(dzs_batch_roots(ctx, ctx->batch_box, s));
    DZS_TRY(dzs_pm_run_batch(ctx, st, prm->pm.precision, prm->pm.tile_chunk, ctx->batch_box,
                             batch->boxes[0].G, s));
    t.r_s = batch->r_s[0];
    t.r_cut = batch->r_cut[0];
    t.accumulate = 1;
    DZS_TRY(dzs_tree_walk_ex(ctx, &batch->boxes[0], st->n, st->x, st->y, st->z, st->mult, st->gx,
                             st->gy, st->gz, &t, ctx->batch_box, s));
    return dzs_launch_kick(ctx, st, prm->K2, s, K2_dev);
}

extern "C" dzs_status kdk_step_batch_stage(dzs_ctx *ctx, const dzs_step_params *prm) {
    if (!ctx)
        return DZS_EINVAL;
    ctx->err[0] = 0;
    if (!prm)
        return dzs_fail(ctx, DZS_EINVAL, "null step parameters");
    if (prm->lc.n_cheb < 1 || prm->lc.n_cheb > DZS_CHEB_MAX)
        return dzs_fail(ctx, DZS_EINVAL, "step: need 1 <= n_cheb <= %d", DZS_CHEB_MAX);
    ctx->step_h->K1 = prm->K1;
    ctx->step_h->K2 = prm->K2;
    dzs_make_lc_args(&prm->lc, &ctx->step_h->lc);
    return DZS_OK;
}

extern "C" dzs_status dzs_check(dzs_ctx *ctx, void *stream) {
    if (!ctx)
        return DZS_EINVAL;
    ctx->err[0] = 0;
    return dzs_tree_check(ctx, (hipStream_t)stream);
}
