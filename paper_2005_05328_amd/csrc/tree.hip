// Oct-tree on Morton-sorted particles and the wavefront-cooperative short-range walk.
//
// Build (paper Sec. 2.1: root = box, each node split into its 8 octants while it holds more
// than one particle; here a node stops splitting at `leaf_size` particles): level by level
// from the root.  A node's particles are a contiguous range of the sorted order and its
// children are the sub-ranges with equal next 3 key bits, found by binary search.  Nodes are
// stored level-major, children of a node contiguous and in Morton order.  Moments (mass,
// centre of mass, particle bounding box, largest softening) are accumulated bottom-up.
//
// Walk: one wave64 per target group (<= 64 Morton-contiguous particles inside one node,
// one target per lane).  The wave pops up to 64 nodes from its stack at a time; each lane
// classifies one node against the group's bounding box: skip (farther than r_cut),
// monopole (side < theta * distance of the node's centre of mass from the box), leaf, or
// open.  Opened nodes push their children; monopoles and leaf particles are appended,
// shifted to the periodic image nearest the group, to an interaction list staged in LDS.
// When the list fills, every lane sums its target's interactions with the whole list
// (LDS broadcast reads).
#include <type_traits>

#include "internal.h"

#define TB_THREADS 256
#define WALK_LIST 128
#define WALK_DEPTH 8192u
#define WALK_SLOTS_MAX 4096u

static inline uint32_t blocks_for(uint64_t n, uint32_t t) { return (uint32_t)((n + t - 1) / t); }

// ---------------------------------------------------------------------------------------
// build
// ---------------------------------------------------------------------------------------
// Build state in device memory (ctx->bstate): the counts of the level-synchronous build stay
// on the device, so the build needs no host synchronisation (and can be graph-captured).
#define BS_NF 0         // frontier nodes at the current level
#define BS_NODES 1      // nodes so far
#define BS_GROUPS 2     // target groups
#define BS_OVERFLOW DZS_BS_OVERFLOW  // sticky: the tree needed more than the node capacity
#define BS_CHILDREN 4   // scan totals of the current level
#define BS_INTERNAL 5
#define BS_LEVEL 8      // [BS_LEVEL + k]: first node of level k (k <= DZS_KEY_BITS + 1)

// An input flagged out of order (DZS_BS_BADINPUT) builds an empty root and nothing below it.
__global__ void k_tree_root(uint32_t n, uint32_t *nd_first, uint32_t *nd_count,
                            uint32_t *nd_child, uint8_t *nd_nchild, uint8_t *nd_level,
                            uint32_t *frontier,
                            uint32_t *bs, uint32_t leaf, int KB) {
    if (bs[DZS_BS_BADINPUT])
        n = 0;
    nd_first[0] = 0;
    nd_count[0] = n;
    nd_child[0] = 0;
    nd_nchild[0] = 0;
    nd_level[0] = 0;
    frontier[0] = 0;
    bs[BS_NF] = (n > leaf || (KB > 0 && n > 0)) ? 1u : 0u;
    bs[BS_NODES] = 1;
    bs[BS_GROUPS] = 0;
    bs[BS_LEVEL + 0] = 0;
    for (int k = 1; k <= DZS_KEY_BITS + 1; ++k)
        bs[BS_LEVEL + k] = 1;
}

// After the emit of level k: advance the node count and the frontier; a level that would
// exceed the node capacity stops the build (its nodes were not written) and flags it.
__global__ void k_tree_level(uint32_t *bs, int k, uint64_t cap) {
    const uint64_t nodes = (uint64_t)bs[BS_NODES] + bs[BS_CHILDREN];
    if (nodes > cap) {
        bs[BS_OVERFLOW] = 1u;
        bs[BS_NF] = 0;
    } else {
        bs[BS_NODES] = (uint32_t)nodes;
        bs[BS_NF] = bs[BS_INTERNAL];
    }
    for (int j = k + 2; j <= DZS_KEY_BITS + 1; ++j)
        bs[BS_LEVEL + j] = bs[BS_NODES];
}

// For each frontier node at level k: the 9 bounds of its 8 octant sub-ranges.  One wave per
// node (grid-stride over the frontier).  A node of at most 64 particles is read in one round;
// a larger one is searched for the 7 inner bounds at once: lanes 9 (d - 1) .. 9 (d - 1) + 8
// sample the bracket of "first index whose digit is >= d" at 9 points, which shrinks it about
// 9-fold per round (dependent loads: log_9 of the node size, not 7 log_2 of it).
__global__ __launch_bounds__(TB_THREADS) void k_tree_split(
    const uint32_t *__restrict__ frontier, const uint32_t *__restrict__ bs, int k,
    const uint64_t *__restrict__ key,
    const uint32_t *__restrict__ nd_first, const uint32_t *__restrict__ nd_count,
    uint32_t *__restrict__ bounds, uint32_t *__restrict__ nchild, uint32_t *__restrict__ ninternal,
    uint32_t leaf, int KB) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t waves = gridDim.x * (TB_THREADS / 64);
    const uint32_t nf = bs[BS_NF];
    const int shift = 3 * (DZS_KEY_BITS - (k + 1));
    const uint32_t g = lane / 9u, j = lane - 9u * g;  // search group (digit g + 1), sample
    for (uint32_t f = blockIdx.x * (TB_THREADS / 64) + (threadIdx.x >> 6); f < nf; f += waves) {
        const uint32_t node = frontier[f];
        const uint32_t s = nd_first[node], e = s + nd_count[node];
        uint32_t b = s;  // lane d in 1..7: first index in [s, e) whose digit is >= d
        if (e - s <= 64u) {
            const uint32_t i = s + lane;
            const uint32_t dig = i < e ? (uint32_t)(key[i] >> shift) & 7u : 8u;
            for (uint32_t d = 1; d < 8; ++d) {
                const uint64_t m = __ballot(dig < d);
                if (lane == d)
                    b = s + (uint32_t)__popcll(m);
            }
        } else {
            uint32_t lo = s, hi = e;  // the bound lies in [lo, hi]
            const uint32_t d = g + 1u;
            while (__ballot(g < 7u && lo < hi) != 0ull) {
                const uint32_t len = hi - lo;
                const uint32_t step = (len + 8u) / 9u;
                const uint32_t p = lo + j * step;
                // positions at or past hi count as "digit >= d" (the bracket's invariant)
                bool ge = true;
                if (g < 7u && lo < hi && p < hi)
                    ge = ((uint32_t)(key[p] >> shift) & 7u) >= d;
                const uint64_t m = __ballot(ge);
                if (g < 7u && lo < hi) {
                    const uint32_t gm = (uint32_t)(m >> (9u * g)) & 0x1ffu;
                    if (gm & 1u) {
                        hi = lo;  // the digit at lo is already >= d
                    } else if (gm == 0u) {
                        lo += 8u * step + 1u;  // every sample (all below hi) has digit < d
                    } else {
                        // between the last sample below d and the first at or above it
                        const uint32_t jj = (uint32_t)__builtin_ctz(gm);
                        const uint32_t nhi = lo + jj * step;
                        lo += (jj - 1u) * step + 1u;
                        hi = nhi < hi ? nhi : hi;
                    }
                }
            }
            const uint32_t src = (lane >= 1u && lane <= 7u) ? 9u * (lane - 1u) : 0u;
            const uint32_t got = __shfl(lo, (int)src, 64);
            if (lane >= 1u && lane <= 7u)
                b = got;
        }
        if (lane == 8u)
            b = e;
        // counts of the 8 children (lane d: bound d + 1 - bound d)
        const uint32_t bn = __shfl_down(b, 1, 64);
        const uint32_t c = lane < 8u ? bn - b : 0u;
        const bool child = lane < 8u && c > 0u;
        // nodes above level KB (the box digits of a batch) always split
        const bool internal = child && (c > leaf || k + 1 < KB) && k + 1 < DZS_TREE_LEVELS;
        const uint64_t mc = __ballot(child), mi = __ballot(internal);
        if (lane <= 8u)
            bounds[(uint64_t)f * 9 + lane] = b;
        if (lane == 0u) {
            nchild[f] = (uint32_t)__popcll(mc);
            ninternal[f] = (uint32_t)__popcll(mi);
        }
    }
}

__global__ __launch_bounds__(TB_THREADS) void k_tree_emit(
    const uint32_t *__restrict__ frontier, const uint32_t *__restrict__ bs, int k,
    const uint32_t *__restrict__ bounds, const uint32_t *__restrict__ child_off,
    const uint32_t *__restrict__ int_off, uint64_t cap, uint32_t *__restrict__ nd_first,
    uint32_t *__restrict__ nd_count, uint32_t *__restrict__ nd_child,
    uint8_t *__restrict__ nd_nchild, uint8_t *__restrict__ nd_level,
    uint32_t *__restrict__ frontier_next, uint32_t leaf, int KB) {
    uint32_t f = blockIdx.x * TB_THREADS + threadIdx.x;
    if (f >= bs[BS_NF])
        return;
    // the whole level is dropped when it does not fit (k_tree_level flags it)
    if ((uint64_t)bs[BS_NODES] + bs[BS_CHILDREN] > cap)
        return;
    const uint32_t node = frontier[f];
    uint32_t c = bs[BS_NODES] + child_off[f];
    uint32_t q = int_off[f];
    nd_child[node] = c;
    uint32_t nc = 0;
    for (int d = 0; d < 8; ++d) {
        uint32_t s = bounds[(uint64_t)f * 9 + d], e = bounds[(uint64_t)f * 9 + d + 1];
        if (e == s)
            continue;
        nd_first[c] = s;
        nd_count[c] = e - s;
        nd_child[c] = 0;
        nd_nchild[c] = 0;
        nd_level[c] = (uint8_t)(k + 1);
        if ((e - s > leaf || k + 1 < KB) && k + 1 < DZS_TREE_LEVELS)
            frontier_next[q++] = c;
        ++c;
        ++nc;
    }
    nd_nchild[node] = (uint8_t)nc;
}

// mult^(1/3), the softening factor of a particle of multiplicity mult (1 for an original
// particle without the library call: most particles)
__device__ __forceinline__ double mult_cbrt(uint32_t mult) {
    return mult == 1u ? 1.0 : cbrt((double)mult);
}

// Half extent of [mn, mx] about c, as an FP32 value rounded up: the box c +- h holds both ends.
__device__ __forceinline__ float half_up(double mn, double mx, double c) {
    return __double2float_ru(fmax(mx - c, c - mn));
}

// Moments of node v (mass, centre of mass, particle bounding box, largest softening): of its
// particles for a leaf, of its children (already complete) otherwise; written with the
// node's topology into its walk record.
__device__ __forceinline__ void node_moments(
    uint32_t v, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const uint32_t *__restrict__ mult, double m0, double h0,
    const uint32_t *__restrict__ nd_first, const uint32_t *__restrict__ nd_count,
    const uint32_t *__restrict__ nd_child, const uint8_t *__restrict__ nd_nchild,
    const uint8_t *__restrict__ nd_level, dzs_node_rec *__restrict__ rec,
    const uint64_t *__restrict__ key, const dzs_bbox *__restrict__ boxes, double L, int unwrap) {
    if (boxes && nd_nchild[v] == 0) {
        // a batch: the leaf's box (its key prefix) sets the mass unit and the softening
        const uint64_t b = key[nd_first[v]] >> DZS_BATCH_SHIFT;
        m0 = boxes[b].m0;
        h0 = boxes[b].h0;
    }
    double m = 0.0, sx = 0.0, sy = 0.0, sz = 0.0, hmax = 0.0;
    double mnx = 1e300, mny = 1e300, mnz = 1e300, mxx = -1e300, mxy = -1e300, mxz = -1e300;
    const uint32_t nc = nd_nchild[v];
    // kept tree: a member (child) more than half a box from the first one crossed a face of
    // the periodic box since the build; it is taken at the image next to the first one
    const double halfL = 0.5 * L;
    auto near = [&](double a, double a0) -> double {
        return a - a0 > halfL ? a - L : (a - a0 < -halfL ? a + L : a);
    };
    uint32_t crossed = 0u;
    if (nc == 0) {
        const uint32_t s = nd_first[v], e = s + nd_count[v];
        const double x0 = x[s], y0 = y[s], z0 = z[s];
        uint32_t mmax = 0;
        for (uint32_t j = s; j < e; ++j) {
            const uint32_t mu = mult[j];
            const double mj = m0 * (double)mu;
            double xj = x[j], yj = y[j], zj = z[j];
            if (unwrap) {
                const double ux = near(xj, x0), uy = near(yj, y0), uz = near(zj, z0);
                crossed |= (ux != xj || uy != yj || uz != zj) ? 1u : 0u;
                xj = ux;
                yj = uy;
                zj = uz;
            }
            m += mj;
            sx += mj * xj;
            sy += mj * yj;
            sz += mj * zj;
            mnx = fmin(mnx, xj); mny = fmin(mny, yj); mnz = fmin(mnz, zj);
            mxx = fmax(mxx, xj); mxy = fmax(mxy, yj); mxz = fmax(mxz, zj);
            mmax = mu > mmax ? mu : mmax;
        }
        hmax = h0 * mult_cbrt(mmax);  // the softening grows with the multiplicity
    } else {
        const uint32_t c0 = nd_child[v];
        const double x0 = rec[c0].cx, y0 = rec[c0].cy, z0 = rec[c0].cz;
        for (uint32_t c = c0; c < c0 + nc; ++c) {
            const dzs_node_rec &r = rec[c];
            const double mc = r.mass;
            double rcx = r.cx, rcy = r.cy, rcz = r.cz;
            double rmx = r.comx, rmy = r.comy, rmz = r.comz;
            if (unwrap) {
                // the child's box and centre of mass move together, by the box's shift
                const double dx = near(rcx, x0) - rcx, dy = near(rcy, y0) - rcy,
                             dz = near(rcz, z0) - rcz;
                rcx += dx; rcy += dy; rcz += dz;
                rmx += dx; rmy += dy; rmz += dz;
            }
            m += mc;
            sx += mc * rmx;
            sy += mc * rmy;
            sz += mc * rmz;
            mnx = fmin(mnx, rcx - (double)r.hx); mny = fmin(mny, rcy - (double)r.hy);
            mnz = fmin(mnz, rcz - (double)r.hz);
            mxx = fmax(mxx, rcx + (double)r.hx); mxy = fmax(mxy, rcy + (double)r.hy);
            mxz = fmax(mxz, rcz + (double)r.hz);
            hmax = fmax(hmax, r.hmax);
        }
    }
    dzs_node_rec out;
    out.cx = 0.5 * (mnx + mxx);
    out.cy = 0.5 * (mny + mxy);
    out.cz = 0.5 * (mnz + mxz);
    out.comx = sx / m;
    out.comy = sy / m;
    out.comz = sz / m;
    out.mass = m;
    out.hmax = hmax;
    out.hx = half_up(mnx, mxx, out.cx);
    out.hy = half_up(mny, mxy, out.cy);
    out.hz = half_up(mnz, mxz, out.cz);
    out.first = nd_first[v];
    out.count = nd_count[v];
    out.child = nd_child[v];
    out.nl = nc | ((uint32_t)nd_level[v] << 8);
    out.pad = crossed;
    rec[v] = out;
}

// Moments of the nodes of level k, [level_start[k], level_start[k+1]) read on the device;
// levels run bottom-up, so the children of every node are complete before it.
__global__ __launch_bounds__(TB_THREADS) void k_tree_moments(
    const uint32_t *__restrict__ bs, int k, const double *__restrict__ x,
    const double *__restrict__ y, const double *__restrict__ z, const uint32_t *__restrict__ mult,
    double m0, double h0, const uint32_t *__restrict__ nd_first,
    const uint32_t *__restrict__ nd_count, const uint32_t *__restrict__ nd_child,
    const uint8_t *__restrict__ nd_nchild, const uint8_t *__restrict__ nd_level,
    dzs_node_rec *rec, const uint64_t *__restrict__ key, const dzs_bbox *__restrict__ boxes,
    double L, int unwrap) {
    const uint32_t end = bs[BS_LEVEL + k + 1];
    for (uint32_t v = bs[BS_LEVEL + k] + blockIdx.x * TB_THREADS + threadIdx.x; v < end;
         v += gridDim.x * TB_THREADS)
        node_moments(v, x, y, z, mult, m0, h0, nd_first, nd_count, nd_child, nd_nchild, nd_level,
                     rec, key, boxes, L, unwrap);
}

// Target groups: each node with more than G particles packs its consecutive children that
// hold at most G particles into bins of at most G (greedy, Morton order); a bin starts a
// group.  Leaves with more than G particles (coincident particles at the finest level) are
// cut into chunks of G.
__global__ __launch_bounds__(TB_THREADS) void k_tree_groups(
    const uint32_t *__restrict__ bs, const uint32_t *__restrict__ nd_first,
    const uint32_t *__restrict__ nd_count,
    const uint32_t *__restrict__ nd_child, const uint8_t *__restrict__ nd_nchild, uint32_t G,
    uint32_t *__restrict__ flag, const uint8_t *__restrict__ nd_level, int KB) {
    uint32_t v = blockIdx.x * TB_THREADS + threadIdx.x;
    if (v >= bs[BS_NODES])
        return;
    const uint32_t cnt = nd_count[v];
    if (KB > 0) {
        // a batch: nothing above the box nodes (level KB) is a group, and the box nodes of at
        // most G particles are groups of their own
        const int lev = nd_level[v];
        if (lev + 1 < KB)
            return;
        if (lev + 1 == KB) {
            const uint32_t c0 = nd_child[v];
            for (uint32_t c = c0; c < c0 + nd_nchild[v]; ++c)
                if (nd_count[c] <= G)
                    flag[nd_first[c]] = 1u;
            return;
        }
    }
    if (v == 0 && cnt <= G) {
        flag[0] = 1u;
        return;
    }
    if (cnt <= G)
        return;
    const uint32_t nc = nd_nchild[v];
    if (nc == 0) {
        for (uint32_t j = nd_first[v]; j < nd_first[v] + cnt; j += G)
            flag[j] = 1u;
        return;
    }
    uint32_t bin = 0;
    const uint32_t c0 = nd_child[v];
    for (uint32_t c = c0; c < c0 + nc; ++c) {
        const uint32_t cc = nd_count[c];
        if (cc > G) {
            bin = 0;
        } else if (bin > 0 && bin + cc <= G) {
            bin += cc;
        } else {
            flag[nd_first[c]] = 1u;
            bin = cc;
        }
    }
}

__global__ __launch_bounds__(TB_THREADS) void k_group_compact(uint32_t n,
                                                              const uint32_t *__restrict__ flag,
                                                              const uint32_t *__restrict__ scan,
                                                              uint32_t *__restrict__ grp_first) {
    uint32_t i = blockIdx.x * TB_THREADS + threadIdx.x;
    if (i < n && flag[i])
        grp_first[scan[i]] = i;
    if (i == 0)
        grp_first[scan[n - 1] + flag[n - 1]] = n;
}

__global__ __launch_bounds__(TB_THREADS) void k_fill_u32(uint64_t n, uint32_t *a, uint32_t v);

// flag[i] = 1 for a flagged target
__global__ __launch_bounds__(TB_THREADS) void k_target_flag(uint32_t n,
                                                            const uint8_t *__restrict__ active,
                                                            uint32_t *__restrict__ flag) {
    const uint32_t i = blockIdx.x * TB_THREADS + threadIdx.x;
    if (i < n)
        flag[i] = active[i] != 0 ? 1u : 0u;
}

__global__ __launch_bounds__(TB_THREADS) void k_target_list(uint32_t n,
                                                            const uint32_t *__restrict__ flag,
                                                            const uint32_t *__restrict__ scan,
                                                            uint32_t *__restrict__ list) {
    const uint32_t i = blockIdx.x * TB_THREADS + threadIdx.x;
    if (i < n && flag[i])
        list[scan[i]] = i;
}

// The tree's groups that hold a flagged target start a group of the target list at their
// first slot (the group then holds its flagged targets only; a group without one is left out).
__global__ __launch_bounds__(TB_THREADS) void k_target_groups(
    uint32_t n, const uint32_t *__restrict__ n_groups, const uint32_t *__restrict__ grp_first,
    const uint8_t *__restrict__ active, uint32_t *__restrict__ flag) {
    const uint32_t g = blockIdx.x * TB_THREADS + threadIdx.x;
    if (g >= n || g >= *n_groups)
        return;
    uint32_t any = 0u;
    for (uint32_t j = grp_first[g]; j < grp_first[g + 1] && !any; ++j)
        any = active[j] != 0 ? 1u : 0u;
    if (any)
        flag[grp_first[g]] = 1u;
}

// pos[k] = the target-list position where group k starts; pos[count] = the number of targets
__global__ __launch_bounds__(TB_THREADS) void k_target_group_pos(
    uint32_t n, const uint32_t *__restrict__ gflag, const uint32_t *__restrict__ gscan,
    const uint32_t *__restrict__ tscan, const uint32_t *__restrict__ n_tgt,
    const uint32_t *__restrict__ n_grp, uint32_t *__restrict__ pos) {
    const uint32_t i = blockIdx.x * TB_THREADS + threadIdx.x;
    if (i < n && gflag[i])
        pos[gscan[i]] = tscan[i];
    if (i == 0)
        pos[*n_grp] = *n_tgt;
}

dzs_status dzs_tree_active_targets(dzs_ctx *ctx, uint64_t n64, const uint8_t *active,
                                   hipStream_t s) {
    const uint32_t n = (uint32_t)n64;
    if (!ctx->grp_list || !ctx->tree_built || n != ctx->tree_n)
        return dzs_fail(ctx, DZS_EINVAL, "active targets: no target list or no tree");
    uint32_t *n_tgt = ctx->d_small + DZS_SMALL_GROUP_LIST;
    uint32_t *n_grp = ctx->d_small + DZS_SMALL_GROUP_LIST + 1;
    // the target list
    hipLaunchKernelGGL(k_target_flag, dim3(blocks_for(n, TB_THREADS)), dim3(TB_THREADS), 0, s, n,
                       active, ctx->tg_flag);
    DZS_TRY(dzs_check_launch(ctx, "target_flag"));
    DZS_TRY(dzs_scan_u32(ctx, ctx->tg_flag, ctx->tg_tscan, n, n_tgt, s));
    hipLaunchKernelGGL(k_target_list, dim3(blocks_for(n, TB_THREADS)), dim3(TB_THREADS), 0, s, n,
                       (const uint32_t *)ctx->tg_flag, (const uint32_t *)ctx->tg_tscan,
                       ctx->grp_list);
    DZS_TRY(dzs_check_launch(ctx, "target_list"));
    // their groups (the tree's, less the unflagged targets): flags at group-start slots, then
    // the list positions where they start
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, TB_THREADS)), dim3(TB_THREADS), 0, s,
                       (uint64_t)n, ctx->tg_flag, 0u);
    DZS_TRY(dzs_check_launch(ctx, "target_group_clear"));
    hipLaunchKernelGGL(k_target_groups, dim3(blocks_for(n, TB_THREADS)), dim3(TB_THREADS), 0, s,
                       n, (const uint32_t *)(ctx->bstate + BS_GROUPS),
                       (const uint32_t *)ctx->grp_first, active, ctx->tg_flag);
    DZS_TRY(dzs_check_launch(ctx, "target_groups"));
    DZS_TRY(dzs_scan_u32(ctx, ctx->tg_flag, ctx->tg_gscan, n, n_grp, s));
    hipLaunchKernelGGL(k_target_group_pos, dim3(blocks_for(n, TB_THREADS)), dim3(TB_THREADS), 0,
                       s, n, (const uint32_t *)ctx->tg_flag, (const uint32_t *)ctx->tg_gscan,
                       (const uint32_t *)ctx->tg_tscan, (const uint32_t *)n_tgt,
                       (const uint32_t *)n_grp, ctx->tg_pos);
    return dzs_check_launch(ctx, "target_group_pos");
}

dzs_status dzs_tree_build(dzs_ctx *ctx, const dzs_box *box, uint64_t n64, const double *x,
                          const double *y, const double *z, const uint32_t *mult, int leaf_size,
                          int group_size, hipStream_t s) {
    return dzs_tree_build_ex(ctx, box, n64, x, y, z, mult, leaf_size, group_size, 0, nullptr, s);
}

__global__ __launch_bounds__(TB_THREADS) void k_fill_u32(uint64_t n, uint32_t *a, uint32_t v) {
    const uint64_t i = (uint64_t)blockIdx.x * TB_THREADS + threadIdx.x;
    if (i < n)
        a[i] = v;
}

// KB > 0: a batch whose keys carry the box in their top KB digits; the nodes above level KB
// always split, the box table supplies each leaf's mass unit and softening.
//
// Every level runs whether or not the tree is that deep (an empty frontier makes its kernels
// return at once): the counts stay on the device and nothing here waits for the host.  The
// launches of level k are sized for the largest frontier it can have: 8^k nodes, and below
// the forced levels the internal nodes of more than `leaf` particles, at most n / (leaf + 1).
// Moments of every level of the last built tree, bottom-up (levels 0 .. ctx->tree_deepest).
static dzs_status tree_moments(dzs_ctx *ctx, const dzs_box *box, uint32_t n, const double *x,
                               const double *y, const double *z, const uint32_t *mult,
                               const dzs_bbox *boxes, int unwrap, hipStream_t s) {
    dzs_timed t(ctx, KC_TREE_MOMENTS, s);
    for (int k = ctx->tree_deepest; k >= 0; --k) {
        // at most 8^k nodes on level k, and never more than the particles
        uint64_t ub = n;
        if (k < 8 && (1ull << (3 * k)) < ub)
            ub = 1ull << (3 * k);
        uint32_t nbk = blocks_for(ub, TB_THREADS);
        nbk = nbk < 8192u ? nbk : 8192u;   // grid-stride beyond
        hipLaunchKernelGGL(k_tree_moments, dim3(nbk), dim3(TB_THREADS), 0, s,
                           (const uint32_t *)ctx->bstate, k, x, y, z, mult, box->m0,
                           2.8 * box->eps0, ctx->nd_first, ctx->nd_count, ctx->nd_child,
                           ctx->nd_nchild, ctx->nd_level, ctx->nd_rec,
                           (const uint64_t *)ctx->key, boxes, box->L, unwrap);
        DZS_TRY(dzs_check_launch(ctx, "tree_moments"));
    }
    return DZS_OK;
}

dzs_status dzs_tree_refresh(dzs_ctx *ctx, const dzs_box *box, uint64_t n, const double *x,
                            const double *y, const double *z, const uint32_t *mult,
                            hipStream_t s) {
    if (!ctx->tree_built || n != ctx->tree_n)
        return dzs_fail(ctx, DZS_EINVAL, "tree refresh: no tree of %llu particles",
                        (unsigned long long)n);
    return tree_moments(ctx, box, (uint32_t)n, x, y, z, mult, nullptr, 1, s);
}

dzs_status dzs_tree_build_ex(dzs_ctx *ctx, const dzs_box *box, uint64_t n64, const double *x,
                             const double *y, const double *z, const uint32_t *mult,
                             int leaf_size, int group_size, int KB, const dzs_bbox *boxes,
                             hipStream_t s) {
    const uint32_t n = (uint32_t)n64;
    ctx->tree_built = false;
    if (n == 0)
        return DZS_OK;
    const uint32_t leaf = (uint32_t)leaf_size;
    const uint64_t cap = ctx->cap_nodes;
    uint32_t *bs = ctx->bstate;
    int deepest = 0;  // the deepest level the build may have created
    {
        dzs_timed t(ctx, KC_TREE_BUILD, s);
        hipLaunchKernelGGL(k_tree_root, dim3(1), dim3(1), 0, s, n, ctx->nd_first, ctx->nd_count,
                           ctx->nd_child, ctx->nd_nchild, ctx->nd_level, ctx->frontier, bs, leaf,
                           KB);
        DZS_TRY(dzs_check_launch(ctx, "tree_root"));
        uint32_t *fr = ctx->frontier, *fr_next = ctx->frontier_next;
        for (int k = 0; k < DZS_TREE_LEVELS; ++k) {
            deepest = k + 1;
            uint64_t ub = k <= KB ? n : n / (leaf + 1) + 1;
            if (k < 8 && (1ull << (3 * k)) < ub)
                ub = 1ull << (3 * k);
            // one wave per frontier node, grid-stride
            const uint64_t sb = (ub + TB_THREADS / 64 - 1) / (TB_THREADS / 64);
            hipLaunchKernelGGL(k_tree_split, dim3((uint32_t)(sb < 2048 ? sb : 2048)),
                               dim3(TB_THREADS), 0,
                               s, fr, (const uint32_t *)bs, k, ctx->key, ctx->nd_first,
                               ctx->nd_count, ctx->child_bounds, ctx->fr_nchild,
                               ctx->fr_ninternal, leaf, KB);
            DZS_TRY(dzs_check_launch(ctx, "tree_split"));
            DZS_TRY(dzs_scan2_u32_dev(ctx, ctx->fr_nchild, ctx->fr_child_off, ctx->fr_ninternal,
                                      ctx->fr_int_off, ub, bs + BS_NF, bs + BS_CHILDREN,
                                      bs + BS_INTERNAL, s));
            hipLaunchKernelGGL(k_tree_emit, dim3(blocks_for(ub, TB_THREADS)), dim3(TB_THREADS), 0,
                               s, fr, (const uint32_t *)bs, k, ctx->child_bounds,
                               ctx->fr_child_off, ctx->fr_int_off, cap, ctx->nd_first,
                               ctx->nd_count, ctx->nd_child, ctx->nd_nchild, ctx->nd_level,
                               fr_next, leaf, KB);
            DZS_TRY(dzs_check_launch(ctx, "tree_emit"));
            hipLaunchKernelGGL(k_tree_level, dim3(1), dim3(1), 0, s, bs, k, cap);
            DZS_TRY(dzs_check_launch(ctx, "tree_level"));
            uint32_t *tmp = fr;
            fr = fr_next;
            fr_next = tmp;
        }
    }
    ctx->tree_deepest = deepest;
    DZS_TRY(tree_moments(ctx, box, n, x, y, z, mult, boxes, 0, s));
    {
        dzs_timed t(ctx, KC_TREE_GROUPS, s);
        hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, TB_THREADS)), dim3(TB_THREADS), 0, s,
                           (uint64_t)n, ctx->grp_flag, 0u);
        DZS_TRY(dzs_check_launch(ctx, "group_clear"));
        hipLaunchKernelGGL(k_tree_groups, dim3(blocks_for(cap, TB_THREADS)), dim3(TB_THREADS), 0,
                           s, (const uint32_t *)bs, ctx->nd_first, ctx->nd_count, ctx->nd_child,
                           ctx->nd_nchild, (uint32_t)group_size, ctx->grp_flag, ctx->nd_level,
                           KB);
        DZS_TRY(dzs_check_launch(ctx, "tree_groups"));
        DZS_TRY(dzs_scan_u32(ctx, ctx->grp_flag, ctx->grp_scan, n, bs + BS_GROUPS, s));
        hipLaunchKernelGGL(k_group_compact, dim3(blocks_for(n, TB_THREADS)), dim3(TB_THREADS), 0, s,
                           n, ctx->grp_flag, ctx->grp_scan, ctx->grp_first);
        DZS_TRY(dzs_check_launch(ctx, "group_compact"));
    }
    ctx->tree_built = true;
    ctx->tree_n = n;
    return DZS_OK;
}

// The sticky overflow flags of the tree build (node capacity) and of the walk (stack depth),
// read back and cleared (synchronises the stream).
dzs_status dzs_tree_check(dzs_ctx *ctx, hipStream_t s) {
    DZS_HIP(ctx, hipMemcpyAsync(ctx->h_small + 8, ctx->bstate + BS_OVERFLOW, sizeof(uint32_t),
                                hipMemcpyDeviceToHost, s));
    DZS_HIP(ctx, hipMemcpyAsync(ctx->h_small + 9, ctx->walk_counter + 2, sizeof(uint32_t),
                                hipMemcpyDeviceToHost, s));
    DZS_HIP(ctx, hipMemcpyAsync(ctx->h_small + 11, ctx->bstate + DZS_BS_BADREPORT,
                                sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    DZS_HIP(ctx, hipStreamSynchronize(s));
    const uint32_t tree_over = ctx->h_small[8], walk_over = ctx->h_small[9];
    const uint32_t bad = ctx->h_small[11];
    if (tree_over || walk_over || bad) {
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, s, (uint64_t)1,
                           ctx->bstate + BS_OVERFLOW, 0u);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, s, (uint64_t)1,
                           ctx->walk_counter + 2, 0u);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, s, (uint64_t)1,
                           ctx->bstate + DZS_BS_BADREPORT, 0u);
        DZS_HIP(ctx, hipStreamSynchronize(s));
    }
    if (bad)
        return dzs_fail(ctx, DZS_EINVAL, "tree_force: particles out of key order under "
                        "presorted, or a target index out of range (nothing was computed)");
    if (tree_over)
        return dzs_fail(ctx, DZS_ECAPACITY, "tree needs more than %llu nodes",
                        (unsigned long long)ctx->cap_nodes);
    if (walk_over)
        return dzs_fail(ctx, DZS_ECAPACITY, "tree walk stack overflow (depth %llu)",
                        (unsigned long long)ctx->walk_stack_depth);
    return DZS_OK;
}

// presorted input: keys (ctx->key) must ascend to the tree's depth; a descent flags the input
__global__ __launch_bounds__(TB_THREADS) void k_check_order(uint64_t n,
                                                            const uint64_t *__restrict__ key,
                                                            uint32_t *__restrict__ bad) {
    const int shift = 3 * (DZS_KEY_BITS - DZS_TREE_LEVELS);
    for (uint64_t i = (uint64_t)blockIdx.x * TB_THREADS + threadIdx.x; i + 1 < n;
         i += (uint64_t)gridDim.x * TB_THREADS)
        if ((key[i] >> shift) > (key[i + 1] >> shift))
            atomicOr(bad, 1u);
}

__global__ void k_latch_bad(uint32_t *bs) {
    bs[DZS_BS_BADREPORT] |= bs[DZS_BS_BADINPUT];
    bs[DZS_BS_BADINPUT] = 0u;
}

dzs_status dzs_latch_bad_input(dzs_ctx *ctx, hipStream_t s) {
    hipLaunchKernelGGL(k_latch_bad, dim3(1), dim3(1), 0, s, ctx->bstate);
    return dzs_check_launch(ctx, "latch_bad");
}

dzs_status dzs_check_order(dzs_ctx *ctx, uint64_t n, hipStream_t s) {
    if (n < 2)
        return DZS_OK;
    uint64_t nb = (n + TB_THREADS - 1) / TB_THREADS;
    nb = nb < 8192 ? nb : 8192;
    hipLaunchKernelGGL(k_check_order, dim3((uint32_t)nb), dim3(TB_THREADS), 0, s, n,
                       (const uint64_t *)ctx->key, ctx->bstate + DZS_BS_BADINPUT);
    return dzs_check_launch(ctx, "check_order");
}

// ---------------------------------------------------------------------------------------
// walk + pair evaluation (FP64)
//
// Lane layout: a wave holds G = 64/P targets; lane = t + G*s serves target t and evaluates
// every P-th list entry starting at s, so a group of G targets is served by all 64 lanes and
// a smaller G wastes fewer evaluations on sources inside the group's cutoff region but
// outside the target's cutoff sphere.  The P partial sums of a target are added in a fixed
// order at the end (deterministic).
//
// Split factor: S(u) = erfc(u/2) + u/sqrt(pi) exp(-u^2/4) = 1 - u w q(w), w = u^2, where
// q(w) = (erf(u/2) - u/sqrt(pi) e^{-u^2/4}) / u^3 is an entire function of w.  The host fits q
// on [0, (r_cut/r_s)^2] by a Chebyshev series (from its Taylor series in long double) and
// passes the monomial coefficients in t = 2 w / w_max - 1; the kernel evaluates it by Horner.
// The fit is checked on the host to 1e-12 relative error in S.
// ---------------------------------------------------------------------------------------
#define WALK_QN 18  // split-factor polynomial coefficients (Horner, fully unrolled): worst
                    // relative error in S 1.3e-13 at r_cut = 4.5 r_s, 7e-12 at 5 r_s
// FP32: S(u) from a table of cubics, one per interval of u = r / r_s on [0, r_cut / r_s]:
// Hermite interpolation of S and dS/du at both ends of each interval (worst absolute error
// in S below 1e-7 at 64 intervals, FP32 coefficients included; checked on the host), plus
// an entry past the cutoff that extends the last one linearly (a pair within rounding of
// r_cut).  The table rides in the kernel arguments and each workgroup stages it in LDS.
#define WALK_TAB_N 64
// list region / cutoff sphere below which a group evaluates densely: in FP32 the one-pass loop
// wins even for wide groups (512^3 walk: 300 ms masked, 285 ms at 2.5, 282 ms at 3-4, 281 ms
// dense everywhere), in FP64 the masked loop wins everywhere (128^3 walk: 2.38 ms masked,
// 2.40 at 2.0, 2.81 dense everywhere)
#ifndef WALK_DENSE_E_F32
#define WALK_DENSE_E_F32 6.0
#endif
#ifndef WALK_DENSE_E_F64
#define WALK_DENSE_E_F64 0.0
#endif

struct walk_args {
    const uint32_t *grp_first;
    const uint32_t *n_groups;   // device: the build's group count
    const double *x, *y, *z;
    const uint32_t *mult;
    const dzs_node_rec *rec;  // the nodes as the walk reads them
    double L, halfL, rcut2, rcut, theta2, rs_inv, rs_inv2, G, m0, h0, t_scale;
    double *gx, *gy, *gz;
    int accumulate;
    int G_lanes;  // targets per wave (64 / phases)
    uint32_t *stack;
    uint32_t depth;
    uint32_t *counter;  // [0] next group, [1] overflow flag
    unsigned long long *pair_count;
    double q[WALK_QN];
    float4 stab[WALK_TAB_N + 1];  // FP32 form: the cubics of S(u), coefficients of f^0..f^3
    double stab_scale;            // intervals per unit of u (WALK_TAB_N r_s / r_cut)
    // start cells: the walk of a group begins at the level-K nodes (and shallower leaves) of
    // the cells that meet its bounding box grown by r_cut, instead of at the root
    const uint32_t *cell_node;  // [8^K] node covering each level-K cell (Morton order)
    const uint8_t *cell_dl;     // [8^K] K - level of that node
    int cell_K;                 // 0: start at the root
    // a batch: the box of a group is its first particle's key prefix
    const uint64_t *key;
    const dzs_bbox *boxes;
    // relative opening criterion: previous |g| per target (nullptr: geometric) and
    // alpha_open / G (the walk's masses and distances carry no G)
    const float *aold;
    double alpha_g;
    // only flagged targets get a force (nullptr: every target); the force of tree slot i
    // goes to entry out_perm[i] (nullptr: i)
    const uint8_t *active;
    const uint32_t *out_perm;
    const uint32_t *bad;  // tree_force input rejected on the device: the walk does nothing
    // a kept, refreshed tree: targets are taken at the image next to the group's first one,
    // and a leaf flagged for members across a face keeps them all with minimum-image pairs;
    // the start cells are widened by the bound on every particle's displacement since the
    // build (device), since a node's particles may have left its cell
    int kept;
    const double *cell_extra;
    // only these targets (nullptr: the tree's groups): tgt[] in slot order, group g holding
    // tgt[tpos[g] .. tpos[g + 1]), g < *n_tgrp
    const uint32_t *tgt;
    const uint32_t *tpos;
    const uint32_t *n_tgrp;
};

// Geometry and constants of the box a group lives in.
struct walk_geom {
    double L, halfL, rcut, rcut2, rs_inv, rs_inv2, Gc, m0, h0, wide;
    uint32_t root;
};

// ---------------------------------------------------------------------------------------
// batch: the node of each box (the level-KB node with the box's key prefix)
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(TB_THREADS) void k_batch_roots(const uint32_t *__restrict__ bs,
                                                            int KB,
                                                            const uint64_t *__restrict__ key,
                                                            const uint32_t *__restrict__ nd_first,
                                                            dzs_bbox *__restrict__ boxes) {
    const uint32_t v = bs[BS_LEVEL + KB] + blockIdx.x * TB_THREADS + threadIdx.x;
    if (v < bs[BS_LEVEL + KB + 1])
        boxes[key[nd_first[v]] >> DZS_BATCH_SHIFT].root = v;
}

dzs_status dzs_batch_roots(dzs_ctx *ctx, dzs_bbox *boxes, hipStream_t s) {
    const int KB = DZS_BATCH_LEVELS;
    hipLaunchKernelGGL(k_batch_roots, dim3(blocks_for(1u << (3 * KB), TB_THREADS)),
                       dim3(TB_THREADS), 0, s, (const uint32_t *)ctx->bstate, KB,
                       (const uint64_t *)ctx->key, ctx->nd_first, boxes);
    return dzs_check_launch(ctx, "batch_roots");
}

// ---------------------------------------------------------------------------------------
// start cells
// ---------------------------------------------------------------------------------------
#define CELL_EMPTY 0xffffffffu

__global__ __launch_bounds__(TB_THREADS) void k_cell_clear(uint64_t n, uint32_t *cell_node) {
    const uint64_t i = (uint64_t)blockIdx.x * TB_THREADS + threadIdx.x;
    if (i < n)
        cell_node[i] = CELL_EMPTY;
}

// Every node at level K, and every leaf above level K, claims the level-K cells of its cube:
// in Morton order these form the contiguous range [P 8^(K-l), (P+1) 8^(K-l)), P = the node's
// key prefix.  The claimed ranges are disjoint; cells no node claims hold no particle.
__global__ __launch_bounds__(TB_THREADS) void k_cell_fill(
    const uint32_t *__restrict__ bs, int K, const uint64_t *__restrict__ key,
    const uint32_t *__restrict__ nd_first, const uint8_t *__restrict__ nd_nchild,
    const uint8_t *__restrict__ nd_level, uint32_t *__restrict__ cell_node,
    uint8_t *__restrict__ cell_dl) {
    const uint32_t node = blockIdx.x * TB_THREADS + threadIdx.x;
    if (node >= bs[BS_LEVEL + K + 1])  // the nodes of levels 0..K
        return;
    const int l = nd_level[node];
    if (l > K || (l < K && nd_nchild[node] != 0))
        return;
    const uint64_t P = key[nd_first[node]] >> (3 * (DZS_KEY_BITS - l));
    const int dl = K - l;
    const uint64_t lo = P << (3 * dl), hi = (P + 1) << (3 * dl);
    for (uint64_t m = lo; m < hi; ++m) {
        cell_node[m] = node;
        cell_dl[m] = (uint8_t)dl;
    }
}

// Arithmetic of the pair loop in the precision T of the form: FP64 (plain) or FP32
// (precision form; coordinates relative to the group centre, so FP32 keeps ~1e-7 of r_cut).
__device__ __forceinline__ double wfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float wfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double wmax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float wmax(float a, float b) { return fmaxf(a, b); }
template <typename T> __device__ __forceinline__ T wmin_image(T d, T L) {
    if (d >= T(0.5) * L)
        d -= L;
    else if (d < T(-0.5) * L)
        d += L;
    return d;
}

// Cubic-spline softened 1/r^3 (enclosed-mass force / r), r < h.
template <typename T> __device__ __forceinline__ T gsoft_inner(T r, T h) {
    const T hinv = T(1.0) / h;
    const T u = r * hinv;
    const T h3 = hinv * hinv * hinv;
    if (u < T(0.5))
        return h3 * (T(32.0 / 3.0) + u * u * (T(32.0) * u - T(192.0 / 5.0)));
    return h3 * (T(64.0 / 3.0) - T(48.0) * u + T(192.0 / 5.0) * u * u - T(32.0 / 3.0) * u * u * u -
                 T(1.0) / (T(15.0) * u * u * u));
}

// One interaction-list entry in LDS: pm = position (shifted to the image nearest the group;
// in FP32 relative to the group centre) and mass; hh = (hm2, h): the entry's spline support h
// and hm2 = max(h^2, the largest h_i^2 of the group's targets), an upper bound of the pair's
// squared support that decides, with one comparison, whether the exact spline test is
// needed.  FP32: 32 bytes, one 16-byte read for pm and one 4-byte read for hm2.
template <typename T> struct vec4_of;
template <> struct vec4_of<float> { typedef float4 type; typedef float2 half; };
struct dvec4 { double x, y, z, w; };   // 8-byte aligned: a 48-byte FP64 entry
struct dvec2 { double x, y; };
template <> struct vec4_of<double> { typedef dvec4 type; typedef dvec2 half; };
template <typename T> struct src_entry {
    typename vec4_of<T>::type pm;
    typename vec4_of<T>::half hh;
};
template <typename T> struct src_list {
    src_entry<T> *e;
};

template <typename T> struct split_coef;
template <> struct split_coef<double> {
    static constexpr int N = WALK_QN;
    static __device__ __forceinline__ double at(const walk_args &A, int k) { return A.q[k]; }
};

// 1/sqrt: the FP32 form takes the hardware approximation (about 1 ulp; its inputs are far
// from the denormal range).  The plain form refines the hardware FP64 estimate y by one
// third-order Newton step, y (1 + e/2 + 3 e^2/8) with e = 1 - a y^2, which takes a relative
// error eps to about (5/16) eps^3; a is a positive, normal squared separation here, so the
// special-value handling of the library's rsqrt is not needed.
__device__ __forceinline__ double pair_rsqrt(double a) {
    const double y = __builtin_amdgcn_rsq(a);
    const double e = __builtin_fma(-a * y, y, 1.0);
    return __builtin_fma(y * e, __builtin_fma(e, 0.375, 0.5), y);
}
__device__ __forceinline__ float pair_rsqrt(float a) { return __builtin_amdgcn_rsqf(a); }
// The larger of two non-negative squared supports (no NaN canonicalisation needed).
__device__ __forceinline__ double pair_hmax(double a, double b) { return a > b ? a : b; }
__device__ __forceinline__ float pair_hmax(float a, float b) {
    return __uint_as_float(max(__float_as_uint(a), __float_as_uint(b)));
}

// Separation of a list entry from the target (minimum image for wide groups).
template <typename T, bool MINIMG, typename E>
__device__ __forceinline__ T pair_sep(const E &e, T xi, T yi, T zi, T L, T &dx, T &dy,
                                      T &dz) {
    dx = e.x - xi;
    dy = e.y - yi;
    dz = e.z - zi;
    if (MINIMG) {
        dx = wmin_image(dx, L);
        dy = wmin_image(dy, L);
        dz = wmin_image(dz, L);
    }
    return wfma(dx, dx, wfma(dy, dy, dz * dz));
}

// Pair force factor g (the force on the target is m r_ij g): g_soft(r) S(r/r_s) with
// S = 1 - u^3 q(u^2), u = r/r_s; outside the spline support g_soft = r^-3 and the product is
// r^-3 - r_s^-3 q, one fused operation.  (FP64; the FP32 form is pair_factor_tab.)
template <typename T>
__device__ __forceinline__ T pair_factor(const walk_args &A, T r2, T eh, T hm2, T hi, T hi2,
                                         T rs_inv2, T rs_inv3, T t_scale) {
    constexpr int QN = split_coef<T>::N;
    const T rinv = pair_rsqrt(r2);
    const T w = r2 * rs_inv2;
    const T t = wfma(w, t_scale, T(-1.0));
    T q = split_coef<T>::at(A, QN - 1);
#pragma unroll
    for (int c = QN - 2; c >= 0; --c)
        q = wfma(q, t, split_coef<T>::at(A, c));
    const T rq = rs_inv3 * q;
    T g = wfma(rinv * rinv, rinv, -rq);
    if (r2 < hm2 && r2 < pair_hmax(eh * eh, hi2)) {
        const T r = r2 * rinv;
        const T ks = gsoft_inner(r, wmax(eh, hi));
        g = ks - ks * (r2 * r) * rq;
    }
    return g;
}

// FP32 pair force factor g_soft(r) S(r/r_s) with S from the LDS table: x = u WALK_TAB_N /
// u_cut = r tscale, interval k = floor(x) (at most WALK_TAB_N, the entry past the cutoff), the
// cubic at f = x - k.  r2 = 0 (the target itself) gives a finite g: its separation is zero.
//
// x in [WALK_TAB_N, ...) (r at or past r_cut: only a pair within rounding of the cutoff is
// kept) takes the last entry at the fraction of x, a linear continuation from S(r_cut).
// r2 = 0 (the target itself) makes g NaN: the caller masks the pair out by r2 > 0.
__device__ __forceinline__ float pair_factor_tab(const float4 *__restrict__ tab, float r2,
                                                float hm2, const float *eh_ptr, float hi,
                                                float hi2, float tscale) {
    const float rinv = pair_rsqrt(r2);
    const float r = r2 * rinv;
    const float x = r * tscale;
    uint32_t k = (uint32_t)x;
    k = k < (uint32_t)WALK_TAB_N ? k : (uint32_t)WALK_TAB_N;
    const float f = __builtin_amdgcn_fractf(x);
    const float4 c = tab[k];
    const float S = __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(c.w, f, c.z), f, c.y), f, c.x);
    float g = (rinv * rinv) * (rinv * S);
    if (r2 < hm2) {  // rare: the exact spline test
        const float eh = *eh_ptr;
        if (r2 < pair_hmax(eh * eh, hi2))
            g = gsoft_inner(r, fmaxf(eh, hi)) * S;
    }
    return g;
}

template <typename T> struct pair_eval;
template <> struct pair_eval<double> {
    const walk_args *A;
    double rs_inv2, rs_inv3, t_scale;
    // hh: the entry's (hm2, h)
    __device__ __forceinline__ double operator()(double r2, const dvec2 *hh, double hi,
                                                 double hi2) const {
        const dvec2 v = *hh;
        return pair_factor<double>(*A, r2, v.y, v.x, hi, hi2, rs_inv2, rs_inv3, t_scale);
    }
};
template <> struct pair_eval<float> {
    const float4 *tab;
    float tscale;
    __device__ __forceinline__ float operator()(float r2, const float2 *hh, float hi,
                                                float hi2) const {
        return pair_factor_tab(tab, r2, hh->x, &hh->y, hi, hi2, tscale);
    }
};

// The lane's share of the list (entries s, s + P, s + 2P, ...) in two passes per block of 32
// of its entries: a cheap pass shifts one acceptance bit per entry (inside r_cut, not the
// target itself) into a 32-bit mask, first entry highest, then the lane evaluates only the
// marked pairs in ascending order.  A list culled against the group's box holds several
// times more entries than any one target's cutoff sphere; without the mask the whole wave
// would step through the force arithmetic for every entry some lane accepts.  The caller
// fills the P entries past the list with far-away sentinels, so the block bound is uniform.
template <typename T, bool MINIMG>
__device__ __forceinline__ void pair_loop(const pair_eval<T> &ev, const walk_geom &W,
                                          const src_list<T> src, uint32_t nlist, uint32_t s,
                                          uint32_t P, T xi, T yi, T zi, T hi, T hi2, T &ax,
                                          T &ay, T &az, uint32_t &n_pairs) {
    const T rcut2 = T(W.rcut2), L = T(W.L);
    // entries per lane: uniform, so the block loops run on the scalar unit
    const uint32_t n_max = (uint32_t)__builtin_amdgcn_readfirstlane((int)((nlist + P - 1) / P));
    for (uint32_t kb = 0; kb < n_max; kb += 32u) {
        const uint32_t blk = s + kb * P;
        const uint32_t kmax =
            (uint32_t)__builtin_amdgcn_readfirstlane((int)(n_max - kb < 32u ? n_max - kb : 32u));
        uint32_t mask = 0;
        for (uint32_t k = 0; k < kmax; ++k) {
            T dx, dy, dz;
            const T r2 = pair_sep<T, MINIMG>(src.e[blk + k * P].pm, xi, yi, zi, L, dx, dy, dz);
            mask = mask + mask + ((r2 < rcut2 && r2 > T(0.0)) ? 1u : 0u);
        }
        mask <<= 32u - kmax;
        n_pairs += (uint32_t)__popc(mask);
        while (mask) {
            const uint32_t k = (uint32_t)__builtin_clz(mask);
            mask ^= 0x80000000u >> k;
            const auto e = src.e[blk + k * P].pm;
            T dx, dy, dz;
            const T r2 = pair_sep<T, MINIMG>(e, xi, yi, zi, L, dx, dy, dz);
            const T f = e.w * ev(r2, &src.e[blk + k * P].hh, hi, hi2);
            ax = wfma(f, dx, ax);
            ay = wfma(f, dy, ay);
            az = wfma(f, dz, az);
        }
    }
}

// The lane's share of the list in one pass: every entry is evaluated and the pairs outside
// r_cut (and the target itself) are multiplied by zero.  All lanes of a phase read the same
// entry and every lane works on every iteration, so when most of the list lies inside most
// targets' cutoff spheres (a compact group) this costs less than the masked two-pass loop.
// 0 < r2 < rcut2: in FP32 one unsigned comparison of the bit patterns (r2 is a sum of
// squares: +0, positive, or +inf for the far sentinels), so the result is a single mask
__device__ __forceinline__ bool pair_inside(float r2, float rcut2) {
    return __float_as_uint(r2) - 1u < __float_as_uint(rcut2) - 1u;
}
__device__ __forceinline__ bool pair_inside(double r2, double rcut2) {
    return r2 < rcut2 && r2 > 0.0;
}

template <typename T, bool MINIMG>
__device__ __forceinline__ void pair_dense(const pair_eval<T> &ev, const walk_geom &W,
                                           const src_list<T> src, uint32_t nlist, uint32_t s,
                                           uint32_t P, T xi, T yi, T zi, T hi, T hi2, T &ax,
                                           T &ay, T &az, uint64_t act_mask, uint32_t &np_wave) {
    const T rcut2 = T(W.rcut2), L = T(W.L);
    const uint32_t n_max = (uint32_t)__builtin_amdgcn_readfirstlane((int)((nlist + P - 1) / P));
    uint32_t cnt = 0;   // wave-uniform, kept on the scalar unit
    for (uint32_t k = 0; k < n_max; ++k) {
        const src_entry<T> *q = src.e + s + k * P;
        const auto e = q->pm;
        T dx, dy, dz;
        const T r2 = pair_sep<T, MINIMG>(e, xi, yi, zi, L, dx, dy, dz);
        const bool in = pair_inside(r2, rcut2);
        // pairs of the flagged targets, counted on the scalar unit
        cnt = (uint32_t)__builtin_amdgcn_readfirstlane(
            (int)(cnt + (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(in) & act_mask)));
        const T g = ev(r2, &q->hh, hi, hi2);
        // the factor of a pair outside (or of the target itself: r = 0) is not used
        const T f = in ? e.w * g : T(0.0);
        ax = wfma(f, dx, ax);
        ay = wfma(f, dy, ay);
        az = wfma(f, dz, az);
    }
    np_wave += cnt;
}

// one wave per workgroup; the FP32 walk fits 4 waves per SIMD (128 VGPRs), the FP64 one 3
template <typename T, bool CELLS, bool BATCH>
__global__ __launch_bounds__(64, sizeof(T) == 4 ? 4 : 3) void k_tree_walk(walk_args A) {
    static_assert(!(CELLS && BATCH), "a batch walk starts at the box nodes");
    constexpr int KBL = BATCH ? DZS_BATCH_LEVELS : 0;  // tree levels above a box
    __shared__ src_entry<T> s_list[WALK_LIST + 64];
    const src_list<T> src{s_list};
    __shared__ uint32_t q_first[64];
    __shared__ uint32_t q_pref[65];
    __shared__ double q_org[3][64];   // a queued leaf's origin in the list frame (image shift)
    __shared__ uint32_t q_wide[64];
    __shared__ uint32_t q_mark[64];
    __shared__ uint32_t s_g;
    __shared__ float s_hbox[12];
    __shared__ float4 s_tab[sizeof(T) == 4 ? WALK_TAB_N + 1 : 1];

    const uint32_t lane = threadIdx.x;
    const uint32_t G = (uint32_t)A.G_lanes;
    const uint32_t P = 64u / G;
    const uint32_t tl = lane % G, ph = lane / G;
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint32_t *stk = A.stack + (uint64_t)blockIdx.x * A.depth;
    if (A.bad && *A.bad)
        return;
    if (sizeof(T) == 4) {
        for (uint32_t k = lane; k <= WALK_TAB_N; k += 64)
            s_tab[k] = A.stab[k];
        __syncthreads();
    }

    for (;;) {
        if (lane == 0)
            s_g = atomicAdd(&A.counter[0], 1u);
        __syncthreads();
        const uint32_t g = s_g;
        __syncthreads();
        uint32_t first, cnt;
        if (A.tgt) {
            if (g >= *A.n_tgrp)
                break;
            first = A.tpos[g];
            cnt = A.tpos[g + 1] - first;
            if (cnt == 0u)
                continue;   // a group start with no flagged target before the next one
        } else {
            if (g >= *A.n_groups)
                break;
            first = A.grp_first[g];
            cnt = A.grp_first[g + 1] - first;
        }
        // a source node and the group may be wide enough that the image nearest the group
        // centre is not every pair's nearest image: an entry kept for the group lies within
        // 2 (h_node + h_group) + r_cut of any of its targets per axis, which must not exceed
        // L/2; above W.wide (half-extent sum (L/2 - r_cut) / 2) the pair loop reduces each
        // separation to the minimum image
        walk_geom W;
        if (BATCH) {
            const dzs_bbox &bx = A.boxes[A.key[first] >> DZS_BATCH_SHIFT];
            W = walk_geom{bx.L,      bx.halfL,   bx.r_cut, bx.rcut2, bx.rs_inv, bx.rs_inv2,
                          bx.G,      bx.m0,      bx.h0,    bx.wide_limit, bx.root};
        } else {
            W = walk_geom{A.L,  A.halfL, A.rcut, A.rcut2, A.rs_inv, A.rs_inv2,
                          A.G,  A.m0,    A.h0,   0.5 * (A.halfL - A.rcut), 0u};
        }
        const bool valid = tl < cnt;
        const uint32_t i = A.tgt ? A.tgt[valid ? first + tl : first] : (valid ? first + tl : first);
        const bool active = valid && (!A.active || A.active[i] != 0);
        if (A.active && __ballot(active) == 0ull)
            continue;  // no target in this group
        double xi = A.x[i], yi = A.y[i], zi = A.z[i];
        if (A.kept) {
            const double x0 = __shfl(xi, 0, 64), y0 = __shfl(yi, 0, 64), z0 = __shfl(zi, 0, 64);
            xi = xi - x0 > W.halfL ? xi - W.L : (xi - x0 < -W.halfL ? xi + W.L : xi);
            yi = yi - y0 > W.halfL ? yi - W.L : (yi - y0 < -W.halfL ? yi + W.L : yi);
            zi = zi - z0 > W.halfL ? zi - W.L : (zi - z0 < -W.halfL ? zi + W.L : zi);
        }
        const double hi = W.h0 * mult_cbrt(A.mult[i]);
        // group bounding box
        double mnx = xi, mny = yi, mnz = zi, mxx = xi, mxy = yi, mxz = zi;
        for (int o = 32; o >= 1; o >>= 1) {
            mnx = fmin(mnx, __shfl_xor(mnx, o, 64));
            mny = fmin(mny, __shfl_xor(mny, o, 64));
            mnz = fmin(mnz, __shfl_xor(mnz, o, 64));
            mxx = fmax(mxx, __shfl_xor(mxx, o, 64));
            mxy = fmax(mxy, __shfl_xor(mxy, o, 64));
            mxz = fmax(mxz, __shfl_xor(mxz, o, 64));
        }
        const double gcx = 0.5 * (mnx + mxx), gcy = 0.5 * (mny + mxy), gcz = 0.5 * (mnz + mxz);
        const double ghx = 0.5 * (mxx - mnx), ghy = 0.5 * (mxy - mny), ghz = 0.5 * (mxz - mnz);
        const double ghmax = fmax(ghx, fmax(ghy, ghz));
        // the list is culled to the group's box grown by r_cut (Steiner: volume, surface,
        // edge and ball terms); when that region is at most WALK_DENSE_E_* times one cutoff
        // sphere, enough entries are inside enough targets' spheres to evaluate densely
        const double rc = W.rcut, pi = 3.14159265358979323846;
        const double v_ball = (4.0 / 3.0) * pi * rc * rc * rc;
        const double v_list = 8.0 * ghx * ghy * ghz + 8.0 * rc * (ghx * ghy + ghy * ghz + ghz * ghx) +
                              2.0 * pi * rc * rc * (ghx + ghy + ghz) + v_ball;
        const double dense_e = sizeof(T) == 4 ? WALK_DENSE_E_F32 : WALK_DENSE_E_F64;
        // (every lane holds the same group box: a wave-uniform choice)
        const bool dense = __builtin_amdgcn_readfirstlane(v_list <= dense_e * v_ball ? 1 : 0) != 0;
        // relative criterion: alpha / G times the smallest previous |g| of the group
        double alpha_a = 0.0;
        if (A.aold) {
            double a = valid ? (double)A.aold[i] : __builtin_inf();
            for (int o = 32; o >= 1; o >>= 1)
                a = fmin(a, __shfl_xor(a, o, 64));
            alpha_a = A.alpha_g * a;
        }
        // list coordinates: absolute in FP64, relative to the group centre in FP32
        const bool rel = sizeof(T) == 4;
        const double ox = rel ? gcx : 0.0, oy = rel ? gcy : 0.0, oz = rel ? gcz : 0.0;
        const T txi = T(xi - ox), tyi = T(yi - oy), tzi = T(zi - oz), thi = T(hi);
        const T thi2 = thi * thi;
        // the largest squared support among the group's targets (the bound stored as hm2)
        T hg2 = valid ? thi2 : T(0.0);
        for (int o = 32; o >= 1; o >>= 1)
            hg2 = wmax(hg2, (T)__shfl_xor(hg2, o, 64));
        const uint64_t act_mask = __ballot(active);
        const T m_unit = T(W.m0), h_unit = T(W.h0);
        const typename vec4_of<T>::half hh_unit = {wmax(h_unit * h_unit, hg2), h_unit};
        // A dense FP32 group is evaluated as two halves, A (its targets 0 .. G/2-1) and B
        // (G/2 .. G-1), compact in Morton order, each against the entries near its own box: at
        // every flush the list is reordered (stably) into the entries near A only, near both and
        // near B only, so that each half steps through a contiguous part of it with twice the
        // phases.  Entries farther than r_cut from both boxes are dropped.
        const uint32_t Gh = G >> 1;
        const uint32_t Ph = G >= 4u ? 64u / Gh : 1u;
        const bool halves = sizeof(T) == 4 && dense && G >= 4u;
        float rc_cls2 = 0.0f;
        if (sizeof(T) == 4 && halves) {
            const float inf = __builtin_inff();
            float b[6] = {valid ? float(txi) : inf, valid ? float(tyi) : inf,
                          valid ? float(tzi) : inf, valid ? float(txi) : -inf,
                          valid ? float(tyi) : -inf, valid ? float(tzi) : -inf};
            for (uint32_t o = 1; o < Gh; o <<= 1)
                for (int c = 0; c < 6; ++c) {
                    const float t = __shfl_xor(b[c], (int)o, 64);
                    b[c] = c < 3 ? fminf(b[c], t) : fmaxf(b[c], t);
                }
            // the halves' boxes (lo x, y, z, hi x, y, z in the group-centre frame) to LDS
            if (lane == 0u || lane == Gh)
                for (int c = 0; c < 6; ++c)
                    s_hbox[lane == 0u ? c : 6 + c] = b[c];
            // a few FP32 ulps of the largest coordinate above r_cut, so that the box test never
            // drops an entry the pair test would take
            const double rc_m = W.rcut * (1.0 + 1e-6) + 1e-6 * (W.rcut + 2.0 * ghmax);
            rc_cls2 = __double2float_ru(rc_m * rc_m);
        }

        pair_eval<T> ev;
        if constexpr (sizeof(T) == 4) {
            ev.tab = s_tab;
            ev.tscale = float(A.stab_scale * W.rs_inv);
        } else {
            ev.A = &A;
            ev.rs_inv2 = W.rs_inv2;
            ev.rs_inv3 = W.rs_inv * W.rs_inv2;
            ev.t_scale = A.t_scale;
        }
        T ax = T(0.0), ay = T(0.0), az = T(0.0);
        T bx = T(0.0), by = T(0.0), bz = T(0.0);   // half B's (ax, ay, az hold half A's)
        uint32_t nlist = 0;
        uint32_t n_pairs = 0;   // per lane (the masked loop)
        uint32_t np_wave = 0;   // the wave's (the dense loop)
        bool wide = false;

        auto flush = [&]() {
            if constexpr (sizeof(T) == 4) {
                if (halves) {
                    uint32_t nA = nlist, bB = 0u, nB = nlist, nt = nlist;
                    if (!wide) {
                        // lane l holds entries l and l + 64 (the list holds at most 128)
                        static_assert(WALK_LIST <= 128, "two list entries per lane");
                        float hbA[6], hbB[6];
                        for (int c = 0; c < 6; ++c) {
                            hbA[c] = s_hbox[c];
                            hbB[c] = s_hbox[6 + c];
                        }
                        float4 p0 = {0.0f, 0.0f, 0.0f, 0.0f}, p1 = p0;
                        float2 q0 = {0.0f, 0.0f}, q1 = q0;
                        uint32_t c0 = 0u, c1 = 0u;   // 1 near A only, 2 near both, 3 near B only
                        auto cls = [&](const float4 &p) -> uint32_t {
                            auto d2 = [&](const float *bx_) {
                                const float dx = fmaxf(fmaxf(bx_[0] - p.x, p.x - bx_[3]), 0.0f);
                                const float dy = fmaxf(fmaxf(bx_[1] - p.y, p.y - bx_[4]), 0.0f);
                                const float dz = fmaxf(fmaxf(bx_[2] - p.z, p.z - bx_[5]), 0.0f);
                                return __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
                            };
                            const bool a = d2(hbA) < rc_cls2, b = d2(hbB) < rc_cls2;
                            return a ? (b ? 2u : 1u) : (b ? 3u : 0u);
                        };
                        if (lane < nlist) {
                            p0 = src.e[lane].pm;
                            q0 = src.e[lane].hh;
                            c0 = cls(p0);
                        }
                        if (lane + 64u < nlist) {
                            p1 = src.e[lane + 64u].pm;
                            q1 = src.e[lane + 64u].hh;
                            c1 = cls(p1);
                        }
                        const uint64_t m01 = __ballot(c0 == 1u), m02 = __ballot(c0 == 2u),
                                       m03 = __ballot(c0 == 3u), m11 = __ballot(c1 == 1u),
                                       m12 = __ballot(c1 == 2u), m13 = __ballot(c1 == 3u);
                        const uint32_t n1 = (uint32_t)(__popcll(m01) + __popcll(m11));
                        const uint32_t n2 = (uint32_t)(__popcll(m02) + __popcll(m12));
                        const uint32_t n3 = (uint32_t)(__popcll(m03) + __popcll(m13));
                        // stable destinations: class base, then the entries of the class before
                        const uint32_t s0 =
                            c0 == 1u ? (uint32_t)__popcll(m01 & lt_mask)
                                     : (c0 == 2u ? n1 + (uint32_t)__popcll(m02 & lt_mask)
                                                 : n1 + n2 + (uint32_t)__popcll(m03 & lt_mask));
                        const uint32_t r11 = (uint32_t)(__popcll(m01) + __popcll(m11 & lt_mask));
                        const uint32_t r12 = (uint32_t)(__popcll(m02) + __popcll(m12 & lt_mask));
                        const uint32_t r13 = (uint32_t)(__popcll(m03) + __popcll(m13 & lt_mask));
                        const uint32_t s1 = c1 == 1u ? r11 : (c1 == 2u ? n1 + r12 : n1 + n2 + r13);
                        __syncthreads();   // every entry read before any is moved
                        if (c0 != 0u) {
                            src.e[s0].pm = p0;
                            src.e[s0].hh = q0;
                        }
                        if (c1 != 0u) {
                            src.e[s1].pm = p1;
                            src.e[s1].hh = q1;
                        }
                        nA = n1 + n2;
                        bB = n1;
                        nB = n2 + n3;
                        nt = n1 + n2 + n3;
                    }
                    if (lane < Ph) {  // sentinels: far outside every cutoff, in any image
                        src.e[nt + lane].pm = {T(1e30), T(1e30), T(1e30), T(0.0)};
                        src.e[nt + lane].hh = {T(0.0), T(0.0)};
                    }
                    __syncthreads();
                    const uint32_t sph = lane / Gh, t0 = lane % Gh;
                    {
                        const uint32_t ts = t0;   // main-layout lane of the target (half A)
                        const T xs = __shfl(txi, (int)ts, 64), ys = __shfl(tyi, (int)ts, 64),
                                zs = __shfl(tzi, (int)ts, 64), hs = __shfl(thi, (int)ts, 64);
                        const uint64_t am = __ballot(__shfl((int)active, (int)ts, 64) != 0);
                        if (wide)
                            pair_dense<T, true>(ev, W, src, nA, sph, Ph, xs, ys, zs, hs, hs * hs,
                                                ax, ay, az, am, np_wave);
                        else
                            pair_dense<T, false>(ev, W, src, nA, sph, Ph, xs, ys, zs, hs, hs * hs,
                                                 ax, ay, az, am, np_wave);
                    }
                    {
                        const uint32_t ts = Gh + t0;   // half B
                        const T xs = __shfl(txi, (int)ts, 64), ys = __shfl(tyi, (int)ts, 64),
                                zs = __shfl(tzi, (int)ts, 64), hs = __shfl(thi, (int)ts, 64);
                        const uint64_t am = __ballot(__shfl((int)active, (int)ts, 64) != 0);
                        const src_list<T> sB{src.e + bB};
                        if (wide)
                            pair_dense<T, true>(ev, W, sB, nB, sph, Ph, xs, ys, zs, hs, hs * hs,
                                                bx, by, bz, am, np_wave);
                        else
                            pair_dense<T, false>(ev, W, sB, nB, sph, Ph, xs, ys, zs, hs, hs * hs,
                                                 bx, by, bz, am, np_wave);
                    }
                    nlist = 0;
                    __syncthreads();
                    return;
                }
            }
            if (lane < P) {  // sentinels: far outside every cutoff, in any image
                src.e[nlist + lane].pm = {T(1e30), T(1e30), T(1e30), T(0.0)};
                src.e[nlist + lane].hh = {T(0.0), T(0.0)};
            }
            __syncthreads();
            if (dense) {
                if (wide)
                    pair_dense<T, true>(ev, W, src, nlist, ph, P, txi, tyi, tzi, thi, thi2, ax,
                                        ay, az, act_mask, np_wave);
                else
                    pair_dense<T, false>(ev, W, src, nlist, ph, P, txi, tyi, tzi, thi, thi2, ax,
                                         ay, az, act_mask, np_wave);
            } else if (wide) {
                pair_loop<T, true>(ev, W, src, nlist, ph, P, txi, tyi, tzi, thi, thi2, ax, ay,
                                   az, n_pairs);
            } else {
                pair_loop<T, false>(ev, W, src, nlist, ph, P, txi, tyi, tzi, thi, thi2, ax, ay,
                                    az, n_pairs);
            }
            nlist = 0;
            __syncthreads();
        };

        uint32_t sp = 0;
        bool overflow = false;
        if (!CELLS) {
            if (lane == 0)
                stk[0] = W.root;
            sp = 1;
        } else {
            // cells of level K met by the bounding box grown by r_cut (plus a margin far above
            // rounding, so that every particle in it is found in a listed cell), wrapped
            const int K = A.cell_K;
            const int side = 1 << K, kmask = side - 1;
            const double inv = (double)side / W.L,
                         margin = 1e-9 * W.L + (A.cell_extra ? *A.cell_extra : 0.0);
            const int lox = (int)floor((mnx - W.rcut - margin) * inv);
            const int loy = (int)floor((mny - W.rcut - margin) * inv);
            const int loz = (int)floor((mnz - W.rcut - margin) * inv);
            const int nx = min((int)floor((mxx + W.rcut + margin) * inv) - lox + 1, side);
            const int ny = min((int)floor((mxy + W.rcut + margin) * inv) - loy + 1, side);
            const int nz = min((int)floor((mxz + W.rcut + margin) * inv) - loz + 1, side);
            const uint32_t nyz = (uint32_t)(ny * nz), total = (uint32_t)nx * nyz;
            for (uint32_t c0 = 0; c0 < total; c0 += 64) {
                const uint32_t c = c0 + lane;
                uint32_t node = CELL_EMPTY;
                if (c < total) {
                    const uint32_t cxo = c / nyz, rem = c - cxo * nyz;
                    const uint32_t cyo = rem / (uint32_t)nz, czo = rem - cyo * (uint32_t)nz;
                    const int cx = lox + (int)cxo, cy = loy + (int)cyo, cz = loz + (int)czo;
                    const uint32_t wx = (uint32_t)(cx & kmask), wy = (uint32_t)(cy & kmask),
                                   wz = (uint32_t)(cz & kmask);
                    const uint32_t m = (uint32_t)((dzs_spread3(wx) << 2) | (dzs_spread3(wy) << 1) |
                                                  dzs_spread3(wz));
                    node = A.cell_node[m];
                    const int dl = A.cell_dl[m];
                    if (node != CELL_EMPTY && dl > 0) {
                        // a leaf above level K covers 2^dl cells per axis: only the first
                        // listed cell inside its cube (per axis, in listing order) pushes it
                        const int span = 1 << dl;
                        auto first = [&](int lo, uint32_t w) -> int {
                            const int n0 = (int)w & ~(span - 1);
                            const int wlo = lo & kmask;
                            return ((wlo - n0) & kmask) < span ? lo : lo + ((n0 - wlo) & kmask);
                        };
                        if (cx != first(lox, wx) || cy != first(loy, wy) || cz != first(loz, wz))
                            node = CELL_EMPTY;
                    }
                }
                const uint32_t put = node != CELL_EMPTY ? 1u : 0u;
                const uint32_t incl = dzs_wave_scan_add_full(put);
                const uint32_t tot = dzs_wave_last(incl);
                if (sp + tot > A.depth) {
                    overflow = true;
                    break;
                }
                if (put)
                    stk[sp + incl - 1] = node;
                sp += tot;
            }
        }
        __threadfence_block();
        while (sp > 0 && !overflow) {
            const uint32_t take = sp < 64 ? sp : 64;
            sp -= take;
            const bool has = lane < take;
            const uint32_t node = has ? stk[sp + lane] : 0u;
            // classify: 0 skip, 1 leaf, 2 monopole, 3 open
            int act = 0;
            double shx = 0.0, shy = 0.0, shz = 0.0;
            uint32_t ncount = 0, nchild = 0, child = 0, nfirst = 0;
            double comx = 0.0, comy = 0.0, comz = 0.0, nmass = 0.0, nhmax = 0.0;
            bool node_wide = false;
            if (has) {
                // the node's record: one address, the fields read where they are needed
                const dzs_node_rec &nd = A.rec[node];
                comx = nd.comx;
                comy = nd.comy;
                comz = nd.comz;
                const uint32_t nl = nd.nl;
                const int nlev = (int)(nl >> 8);
                nchild = nl & 0xffu;
                ncount = nd.count;
                nfirst = nd.first;
                child = nd.child;
                double dcx = nd.cx - gcx, dcy = nd.cy - gcy, dcz = nd.cz - gcz;
                shx = dcx > W.halfL ? -W.L : (dcx < -W.halfL ? W.L : 0.0);
                shy = dcy > W.halfL ? -W.L : (dcy < -W.halfL ? W.L : 0.0);
                shz = dcz > W.halfL ? -W.L : (dcz < -W.halfL ? W.L : 0.0);
                dcx += shx; dcy += shy; dcz += shz;
                const double nhx = nd.hx, nhy = nd.hy, nhz = nd.hz;
                const double gx_ = fmax(0.0, fabs(dcx) - nhx - ghx);
                const double gy_ = fmax(0.0, fabs(dcy) - nhy - ghy);
                const double gz_ = fmax(0.0, fabs(dcz) - nhz - ghz);
                const double dist2 = gx_ * gx_ + gy_ * gy_ + gz_ * gz_;
                node_wide = fmax(nhx, fmax(nhy, nhz)) + ghmax > W.wide || nd.pad != 0u;
                if (dist2 >= W.rcut2) {
                    act = 0;
                } else if (nchild == 0) {
                    act = 1;
                } else {
                    act = 3;
                    if (A.theta2 > 0.0 || A.aold) {
                        const double cx = comx + shx - gcx;
                        const double cy = comy + shy - gcy;
                        const double cz = comz + shz - gcz;
                        const double ex = fmax(0.0, fabs(cx) - ghx);
                        const double ey = fmax(0.0, fabs(cy) - ghy);
                        const double ez = fmax(0.0, fabs(cz) - ghz);
                        const double d2 = ex * ex + ey * ey + ez * ez;
                        const double side = ldexp(W.L, -(nlev - KBL));
                        if (A.aold) {
                            // G M l^2 < alpha a_min d^4
                            if (nd.mass * (side * side) < alpha_a * (d2 * d2))
                                act = 2;
                        } else if (side * side < A.theta2 * d2) {
                            act = 2;
                        }
                        if (act == 2) {
                            nmass = nd.mass;
                            nhmax = nd.hmax;
                        }
                    }
                }
            }
            if (__ballot((act == 1 || act == 2) && node_wide) != 0ull)
                wide = true;
            // ---- pushes
            const uint32_t npush = act == 3 ? nchild : 0u;
            const uint32_t pincl = dzs_wave_scan_add_full(npush);
            const uint32_t ptot = dzs_wave_last(pincl);
            if (sp + ptot > A.depth) {
                overflow = true;
                break;
            }
            for (uint32_t j = 0; j < npush; ++j)
                stk[sp + pincl - npush + j] = child + j;
            sp += ptot;
            __threadfence_block();
            // ---- monopoles
            const uint64_t mono = __ballot(act == 2);
            const uint32_t nmono = (uint32_t)__popcll(mono);
            if (nmono > 0) {
                if (nlist + nmono > WALK_LIST)
                    flush();
                if (act == 2) {
                    const uint32_t slot = nlist + (uint32_t)__popcll(mono & lt_mask);
                    src.e[slot].pm = {T(comx + shx - ox), T(comy + shy - oy),
                                      T(comz + shz - oz), T(nmass)};
                    const T hn = T(nhmax);
                    src.e[slot].hh = {wmax(hn * hn, hg2), hn};
                }
                nlist += nmono;
            }
            // ---- leaves: queue, then stream their particles into the list, keeping only the
            //      particles within r_cut of the group's bounding box
            const uint64_t lmask = __ballot(act == 1);
            const uint32_t nq = (uint32_t)__popcll(lmask);
            if (nq > 0) {
                const uint32_t lc = act == 1 ? ncount : 0u;
                const uint32_t lincl = dzs_wave_scan_add_full(lc);
                const uint32_t Ptot = dzs_wave_last(lincl);
                __syncthreads();
                if (act == 1) {
                    const uint32_t q = (uint32_t)__popcll(lmask & lt_mask);
                    q_first[q] = nfirst;
                    q_pref[q] = lincl - lc;
                    q_org[0][q] = ox - shx;
                    q_org[1][q] = oy - shy;
                    q_org[2][q] = oz - shz;
                    q_wide[q] = node_wide ? 1u : 0u;
                }
                if (lane == 0)
                    q_pref[nq] = Ptot;
                __syncthreads();
                // candidate f of a pass belongs to the last leaf starting at or before it: each
                // leaf marks its start in the pass's window, a wave max-scan spreads the marks
                // (the leaf of the window's first slot carries over from the pass before)
                const uint32_t lstart = lincl - lc;
                const uint32_t lq = (uint32_t)__popcll(lmask & lt_mask);
                uint32_t carry = 0;
                for (uint32_t done = 0; done < Ptot; done += 64) {
                    // room for every candidate of the pass: no candidate is held across a flush
                    if (nlist + min(Ptot - done, 64u) > WALK_LIST)
                        flush();
                    const uint32_t f = done + lane;
                    q_mark[lane] = 0u;
                    __syncthreads();
                    if (act == 1 && lstart >= done && lstart - done < 64u)
                        q_mark[lstart - done] = lq + 1u;
                    __syncthreads();
                    uint32_t v = q_mark[lane];
                    if (lane == 0)
                        v = v > carry + 1u ? v : carry + 1u;
                    v = dzs_wave_scan_max_full(v);
                    const uint32_t lo = v - 1u;
                    carry = dzs_wave_last(lo);
                    bool keep = false;
                    double ex_ = 0.0, ey_ = 0.0, ez_ = 0.0;
                    uint32_t mj = 0;
                    if (f < Ptot) {
                        const uint32_t j = q_first[lo] + (f - q_pref[lo]);
                        // the particle in the list frame: its nearest image, less the group
                        // centre in FP32 (then the offset from the centre is the coordinate)
                        ex_ = A.x[j] - q_org[0][lo];
                        ey_ = A.y[j] - q_org[1][lo];
                        ez_ = A.z[j] - q_org[2][lo];
                        mj = A.mult[j];
                        const double cx = fmax(0.0, fabs(rel ? ex_ : ex_ - gcx) - ghx);
                        const double cy = fmax(0.0, fabs(rel ? ey_ : ey_ - gcy) - ghy);
                        const double cz = fmax(0.0, fabs(rel ? ez_ : ez_ - gcz) - ghz);
                        keep = q_wide[lo] != 0u || cx * cx + cy * cy + cz * cz < W.rcut2;
                    }
                    const uint64_t kmask = __ballot(keep);
                    const uint32_t nk = (uint32_t)__popcll(kmask);
                    if (nk > 0) {
                        if (keep) {
                            const uint32_t slot = nlist + (uint32_t)__popcll(kmask & lt_mask);
                            // an original particle (multiplicity 1) takes the group's constants
                            T mj_mass = m_unit;
                            typename vec4_of<T>::half mj_hh = hh_unit;
                            if (mj != 1u) {
                                mj_mass = T(W.m0 * (double)mj);
                                const T hj = T(W.h0 * mult_cbrt(mj));
                                mj_hh = {wmax(hj * hj, hg2), hj};
                            }
                            src.e[slot].pm = {T(ex_), T(ey_), T(ez_), mj_mass};
                            src.e[slot].hh = mj_hh;
                        }
                        nlist += nk;
                    }
                }
                __syncthreads();
            }
        }
        if (overflow) {
            if (lane == 0)
                atomicOr(&A.counter[2], 1u);   // sticky until checked
        }
        flush();
        if (halves) {
            // fixed-order sums of the Ph partial accelerations of each half's targets, then each
            // target's sum moved to its lane (tl) of the group layout
            for (uint32_t o = Gh; o < 64; o <<= 1) {
                ax += __shfl_xor(ax, o, 64);
                ay += __shfl_xor(ay, o, 64);
                az += __shfl_xor(az, o, 64);
                bx += __shfl_xor(bx, o, 64);
                by += __shfl_xor(by, o, 64);
                bz += __shfl_xor(bz, o, 64);
            }
            const int sl = (int)(tl % Gh);
            const T ax2 = __shfl(ax, sl, 64), ay2 = __shfl(ay, sl, 64), az2 = __shfl(az, sl, 64);
            const T bx2 = __shfl(bx, sl, 64), by2 = __shfl(by, sl, 64), bz2 = __shfl(bz, sl, 64);
            const bool inA = tl < Gh;
            ax = inA ? ax2 : bx2;
            ay = inA ? ay2 : by2;
            az = inA ? az2 : bz2;
        } else {
            // fixed-order sum of the P partial accelerations of each target
            for (uint32_t o = G; o < 64; o <<= 1) {
                ax += __shfl_xor(ax, o, 64);
                ay += __shfl_xor(ay, o, 64);
                az += __shfl_xor(az, o, 64);
            }
        }
        {
            uint64_t cnt_pairs = active ? n_pairs : 0u;
            for (int o = 32; o >= 1; o >>= 1)
                cnt_pairs += __shfl_xor(cnt_pairs, o, 64);
            if (lane == 0)
                atomicAdd(A.pair_count, (unsigned long long)(cnt_pairs + np_wave));
        }
        if (active && ph == 0) {
            const double gxv = W.Gc * (double)ax, gyv = W.Gc * (double)ay, gzv = W.Gc * (double)az;
            const uint32_t o = A.out_perm ? A.out_perm[i] : i;
            if (A.accumulate) {
                A.gx[o] += gxv;
                A.gy[o] += gyv;
                A.gz[o] += gzv;
            } else {
                A.gx[o] = gxv;
                A.gy[o] = gyv;
                A.gz[o] = gzv;
            }
        }
    }
}

// ---- host: the split-factor polynomial ------------------------------------------------
namespace {

// q(w) = (erf(u/2) - u/sqrt(pi) exp(-u^2/4)) / u^3 from its Taylor series:
// q(w) = (1/sqrt(pi)) sum_{n>=1} (-1)^(n+1) 2n w^(n-1) / ((2n+1) 4^n n!)
long double q_taylor(long double w) {
    const long double inv_sqrt_pi = 0.564189583547756286948079451560772586L;
    long double term = 1.0L;  // w^(n-1) / (4^n n!) * 4, starts at n = 1 as 1/4 * 4 ... kept as ratio
    long double sum = 0.0L;
    long double pw = 1.0L;     // w^(n-1)
    long double fac = 1.0L;    // 4^n n!
    for (int n = 1; n < 200; ++n) {
        fac *= 4.0L * n;
        term = (n % 2 ? 1.0L : -1.0L) * 2.0L * n * pw / ((2.0L * n + 1.0L) * fac);
        sum += term;
        if (n > 4 && fabsl(term) < 1e-24L * fabsl(sum))
            break;
        pw *= w;
    }
    return sum * inv_sqrt_pi;
}

// Chebyshev fit of q on [0, wmax] with n coefficients, converted to monomials in t.
void fit_q(long double wmax, int n, long double *mono) {
    const long double pi = 3.14159265358979323846264338327950288L;
    long double f[WALK_QN], c[WALK_QN];
    for (int j = 0; j < n; ++j) {
        long double t = cosl(pi * (j + 0.5L) / n);
        f[j] = q_taylor(0.5L * (t + 1.0L) * wmax);
    }
    for (int k = 0; k < n; ++k) {
        long double s = 0.0L;
        for (int j = 0; j < n; ++j)
            s += f[j] * cosl(pi * k * (j + 0.5L) / n);
        c[k] = s * (k == 0 ? 1.0L : 2.0L) / n;
    }
    // T_k as monomial vectors: T_0 = 1, T_1 = t, T_{k+1} = 2 t T_k - T_{k-1}
    long double Tm[WALK_QN], T0[WALK_QN], T1[WALK_QN];
    for (int i = 0; i < n; ++i)
        mono[i] = T0[i] = T1[i] = 0.0L;
    T0[0] = 1.0L;
    T1[1 < n ? 1 : 0] += (n > 1) ? 1.0L : 0.0L;
    for (int i = 0; i < n; ++i)
        mono[i] += c[0] * T0[i];
    if (n > 1)
        for (int i = 0; i < n; ++i)
            mono[i] += c[1] * T1[i];
    for (int k = 2; k < n; ++k) {
        for (int i = 0; i < n; ++i)
            Tm[i] = -T0[i] + (i > 0 ? 2.0L * T1[i - 1] : 0.0L);
        for (int i = 0; i < n; ++i) {
            mono[i] += c[k] * Tm[i];
            T0[i] = T1[i];
            T1[i] = Tm[i];
        }
    }
}

}  // namespace

// The WALK_QN-coefficient fit and its worst relative error in S on [0, wmax].
static double split_poly(double wmax, double *q) {
    long double mono[WALK_QN];
    fit_q(wmax, WALK_QN, mono);
    long double worst = 0.0L;
    for (int k = 0; k <= 800; ++k) {
        long double w = wmax * k / 800.0L;
        long double t = 2.0L * w / wmax - 1.0L;
        long double qa = 0.0L;
        for (int i = WALK_QN - 1; i >= 0; --i)
            qa = qa * t + mono[i];
        long double qe = q_taylor(w);
        long double u = sqrtl(w);
        long double S = 1.0L - u * w * qe;
        long double err = fabsl(u * w * (qa - qe)) / fabsl(S);
        worst = err > worst ? err : worst;
    }
    for (int i = 0; i < WALK_QN; ++i)
        q[i] = (double)mono[i];
    return (double)worst;
}

// The FP32 table of S(u) on [0, ucut] (WALK_TAB_N intervals): on interval j, with
// h = ucut / WALK_TAB_N and f in [0, 1], the cubic Hermite interpolant of S and h dS/du at
// both ends, in powers of f; entry WALK_TAB_N continues the last interval's end linearly.
// Returns the worst absolute error in S (FP32 coefficients, exact long double evaluation).
static double split_table_f32(double ucut, float4 *tab) {
    const long double pi = 3.14159265358979323846264338327950288L;
    auto S = [&](long double u) {
        return erfcl(0.5L * u) + u / sqrtl(pi) * expl(-0.25L * u * u);
    };
    auto dS = [&](long double u) { return -u * u / (2.0L * sqrtl(pi)) * expl(-0.25L * u * u); };
    const long double h = (long double)ucut / WALK_TAB_N;
    for (int j = 0; j <= WALK_TAB_N; ++j) {
        const long double u0 = h * j, u1 = h * (j + 1);
        const long double s0 = S(u0), d0 = h * dS(u0);
        if (j == WALK_TAB_N) {
            tab[j] = make_float4((float)s0, (float)d0, 0.0f, 0.0f);
            break;
        }
        const long double s1 = S(u1), d1 = h * dS(u1);
        tab[j] = make_float4((float)s0, (float)d0, (float)(3.0L * (s1 - s0) - 2.0L * d0 - d1),
                             (float)(2.0L * (s0 - s1) + d0 + d1));
    }
    long double worst = 0.0L;
    for (int j = 0; j < WALK_TAB_N; ++j)
        for (int k = 0; k <= 16; ++k) {
            const long double f = k / 16.0L;
            const float4 c = tab[j];
            const long double v = (long double)c.x +
                                  f * ((long double)c.y + f * ((long double)c.z + f * c.w));
            const long double e = fabsl(v - S(h * (j + f)));
            worst = e > worst ? e : worst;
        }
    return (double)worst;
}

dzs_status dzs_tree_walk(dzs_ctx *ctx, const dzs_box *box, uint64_t n, const double *x,
                         const double *y, const double *z, const uint32_t *mult, double *gx,
                         double *gy, double *gz, const dzs_tree_params *prm, hipStream_t s,
                         const dzs_walk_io &io) {
    return dzs_tree_walk_ex(ctx, box, n, x, y, z, mult, gx, gy, gz, prm, nullptr, s, io);
}

// boxes != nullptr: a batch (device table of the boxes; the keys in ctx->key carry the box);
// every box must share r_cut / r_s, the ratio the split-factor polynomial is fitted for.
dzs_status dzs_tree_walk_ex(dzs_ctx *ctx, const dzs_box *box, uint64_t n, const double *x,
                            const double *y, const double *z, const uint32_t *mult, double *gx,
                            double *gy, double *gz, const dzs_tree_params *prm,
                            const dzs_bbox *boxes, hipStream_t s, const dzs_walk_io &io) {
    if (n == 0 || !ctx->tree_built)
        return DZS_OK;
    const float *aold = io.aold;
    const bool relative = prm->opening == DZS_OPEN_RELATIVE && aold && !boxes;
    walk_args A;
    memset(&A, 0, sizeof(A));
    A.grp_first = ctx->grp_first;
    A.n_groups = ctx->bstate + BS_GROUPS;
    A.x = x; A.y = y; A.z = z; A.mult = mult;
    A.rec = ctx->nd_rec;
    A.L = box->L;
    A.halfL = 0.5 * box->L;
    A.rcut = prm->r_cut;
    A.rcut2 = prm->r_cut * prm->r_cut;
    A.theta2 = prm->theta * prm->theta;
    A.rs_inv = 1.0 / prm->r_s;
    A.rs_inv2 = A.rs_inv * A.rs_inv;
    A.G = box->G;
    A.m0 = box->m0;
    A.h0 = 2.8 * box->eps0;
    A.gx = gx; A.gy = gy; A.gz = gz;
    A.accumulate = prm->accumulate;
    A.G_lanes = prm->group_size;
    A.aold = relative ? aold : nullptr;
    A.active = boxes ? nullptr : io.active;
    A.out_perm = boxes ? nullptr : io.out_perm;
    A.bad = ctx->bstate + DZS_BS_BADINPUT;
    A.kept = (io.kept_tree && !boxes) ? 1 : 0;
    A.cell_extra = A.kept ? (const double *)(ctx->d_small + DZS_SMALL_DRIFT_TOTAL) : nullptr;
    if (io.target_list && !boxes && ctx->grp_list) {
        A.tgt = ctx->grp_list;
        A.tpos = ctx->tg_pos;
        A.n_tgrp = ctx->d_small + DZS_SMALL_GROUP_LIST + 1;
    }
    A.alpha_g = relative ? prm->alpha_open / box->G : 0.0;
    const double wmax = (prm->r_cut / prm->r_s) * (prm->r_cut / prm->r_s);
    if (ctx->q_wmax != wmax) {
        ctx->q_err = split_poly(wmax, ctx->q_coef);
        ctx->qf_err = split_table_f32(sqrt(wmax), ctx->stab);
        ctx->q_wmax = wmax;
    }
    const bool fp32 = prm->precision == DZS_FP32;
    if (!(ctx->q_err < 1e-10) || (fp32 && !(ctx->qf_err < 2e-7)))
        return dzs_fail(ctx, DZS_EINVAL, "tree: split-factor fit error %.2e / %.2e (FP32) for "
                        "r_cut/r_s = %.3f", ctx->q_err, ctx->qf_err, sqrt(wmax));
    for (int k = 0; k < WALK_QN; ++k)
        A.q[k] = ctx->q_coef[k];
    for (int k = 0; k <= WALK_TAB_N; ++k)
        A.stab[k] = ctx->stab[k];
    A.stab_scale = WALK_TAB_N * prm->r_s / prm->r_cut;
    A.t_scale = 2.0 / wmax;
    A.stack = ctx->walk_stack;
    A.depth = (uint32_t)ctx->walk_stack_depth;
    A.counter = ctx->walk_counter;
    A.pair_count = (unsigned long long *)(ctx->walk_counter + 8);
    // start level K: the deepest level whose cells are at least r_cut wide, at most
    // DZS_CELL_K_MAX.  Every node above level K is opened: eq. 1 could accept some of them
    // (a group's box can lie up to r_cut + sqrt(3) l from the centre of mass of a node of
    // side l, farther than l / theta), so the walk is at least as accurate as eq. 1 alone
    A.key = (const uint64_t *)ctx->key;
    A.boxes = boxes;
    int K = 0;
    if ((prm->theta <= 1.0 || relative) && !boxes)
        while (K < DZS_CELL_K_MAX && ldexp(box->L, -(K + 1)) >= prm->r_cut)
            ++K;
    A.cell_K = K;
    A.cell_node = ctx->cell_node;
    A.cell_dl = ctx->cell_dl;
    if (K > 0) {
        dzs_timed t(ctx, KC_TREE_BUILD, s);
        const uint64_t n_cells = 1ull << (3 * K);
        hipLaunchKernelGGL(k_cell_clear, dim3(blocks_for(n_cells, TB_THREADS)), dim3(TB_THREADS),
                           0, s, n_cells, ctx->cell_node);
        DZS_TRY(dzs_check_launch(ctx, "cell_clear"));
        // at most (8^(K+1) - 1) / 7 nodes sit on levels 0..K
        uint64_t n_top = ((1ull << (3 * (K + 1))) - 1) / 7;
        n_top = n_top < ctx->cap_nodes ? n_top : ctx->cap_nodes;
        hipLaunchKernelGGL(k_cell_fill, dim3(blocks_for(n_top, TB_THREADS)), dim3(TB_THREADS), 0,
                           s, (const uint32_t *)ctx->bstate, K, (const uint64_t *)ctx->key,
                           ctx->nd_first, ctx->nd_nchild, ctx->nd_level, ctx->cell_node,
                           ctx->cell_dl);
        DZS_TRY(dzs_check_launch(ctx, "cell_fill"));
    }
    // persistent waves: each takes groups until the counter passes the device group count
    uint32_t slots = (uint32_t)ctx->walk_stack_slots;
    if (n < slots)
        slots = (uint32_t)n;   // there are at most n groups
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(TB_THREADS), 0, s, (uint64_t)1, ctx->walk_counter,
                       0u);
    DZS_TRY(dzs_check_launch(ctx, "walk_counter_clear"));
    {
        dzs_timed t(ctx, KC_TREE_WALK, s);
        if (boxes && fp32)
            hipLaunchKernelGGL((k_tree_walk<float, false, true>), dim3(slots), dim3(64), 0, s, A);
        else if (boxes)
            hipLaunchKernelGGL((k_tree_walk<double, false, true>), dim3(slots), dim3(64), 0, s, A);
        else if (fp32 && K > 0)
            hipLaunchKernelGGL((k_tree_walk<float, true, false>), dim3(slots), dim3(64), 0, s, A);
        else if (fp32)
            hipLaunchKernelGGL((k_tree_walk<float, false, false>), dim3(slots), dim3(64), 0, s, A);
        else if (K > 0)
            hipLaunchKernelGGL((k_tree_walk<double, true, false>), dim3(slots), dim3(64), 0, s, A);
        else
            hipLaunchKernelGGL((k_tree_walk<double, false, false>), dim3(slots), dim3(64), 0, s, A);
        DZS_TRY(dzs_check_launch(ctx, "tree_walk"));
    }
    return DZS_OK;  // overflows stay on the device until dzs_check
}

static_assert(sizeof(((dzs_ctx *)nullptr)->stab) == sizeof(float4) * (WALK_TAB_N + 1),
              "the context's table of S(u) holds WALK_TAB_N + 1 cubics");
