// Internal declarations of libdzs: the context, error handling, launch timing and the
// launchers each translation unit provides.  Device code for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "../../include/dzs.h"

#define DZS_KEY_BITS 21
// deepest level of the force tree: the sort before a tree build orders the keys to this level
// only (bits 16..62), the build stops there (a level-15 node of more than leaf_size
// particles stays a leaf)
#define DZS_TREE_LEVELS 15
#define DZS_TREE_FIRST_PASS 2  // radix passes of 8 bits skipped by that sort
#define DZS_CELL_K_MAX 7  // deepest level of the walk start cells (8^7 cells, 10 MB)
#define DZS_KEY_SIDE 2097152.0

// ---------------------------------------------------------------------------------------
// kernel classes timed by dzs_timing
// ---------------------------------------------------------------------------------------
enum dzs_kclass {
    KC_KICK = 0,
    KC_DRIFT_LC,
    KC_KEYS,
    KC_SORT,
    KC_PERMUTE,
    KC_TREE_BUILD,
    KC_TREE_MOMENTS,
    KC_TREE_GROUPS,
    KC_TREE_WALK,
    KC_PM_DEPOSIT,
    KC_PM_FFT_X,
    KC_PM_FFT_Y,
    KC_PM_FFT_Z_GREEN,
    KC_PM_INTERP,
    KC_DZS_LEVELS,
    KC_DZS_COMPACT,
    KC_MISC,
    KC_COUNT
};

extern const char *const dzs_kclass_names[KC_COUNT];

struct dzs_timer_pool {
    static const int CAP = 8192;
    hipEvent_t start[CAP], stop[CAP];
    int cls[CAP];
    int used = 0;
    bool created = false;
};

// A batched step (many independent boxes in one particle array): box b's particles carry
// Morton keys prefixed by b in their top DZS_BATCH_LEVELS octal digits, so one sort keeps each
// box contiguous and one tree holds every box below the node of its prefix.
#define DZS_BATCH_LEVELS 3                       // 8^3 = 512 boxes at most
#define DZS_BATCH_SHIFT (3 * (DZS_KEY_BITS - DZS_BATCH_LEVELS))  // 54: box id = key >> 54
#define DZS_BATCH_SIDE 262144.0                  // 2^18 cells per side below the box digits

// drift and lightcone parameters of one drift (kernel argument or device block)
struct lc_args {
    double xo[3];
    double chi2_0, chi2_1, D, a0, a1;
    int n_cheb;
    double cchi[DZS_CHEB_MAX];
    double cdrift[DZS_CHEB_MAX];
};

// the factors of one batched step, in a device block (and its pinned host staging): a
// captured step reads them when it runs
struct dzs_step_block {
    double K1, K2;
    lc_args lc;
};

// per-box parameters of a batched step, in device memory
struct dzs_bbox {
    double L, halfL;
    double m0, h0, G;                 // mass unit, spline support of mult 1, gravity
    double r_s, r_cut, rcut2, rs_inv, rs_inv2, wide_limit;
    double delta, q_scale;            // PM mesh spacing, fixed-point deposit scale
    uint64_t first, count;            // particle range of the box
    uint64_t mesh_off;                // first cell of the box's mesh in the mesh arrays
    uint64_t tab_off;                 // first entry of its Green's function tables
    int32_t ng;
    uint32_t root;                    // tree node of the box (its key prefix)
};

// One tree node as the walk reads it, 96 bytes (six 16-byte loads, one cache line for most
// nodes): the particles' bounding box as a centre (FP64) and half extents (FP32 rounded up,
// so the box still holds every particle), the centre of mass, mass and largest softening
// support (FP64), and the topology (first particle, count, first child, children and level).
struct alignas(16) dzs_node_rec {
    double cx, cy, cz;
    double comx, comy, comz;
    double mass, hmax;
    float hx, hy, hz;
    uint32_t first;
    uint32_t count, child, nl;  // nl = nchild | level << 8
    uint32_t pad;
};
static_assert(sizeof(dzs_node_rec) == 96, "node record layout");

struct dzs_ctx {
    int device = 0;
    uint64_t cap_n = 0;
    uint32_t cap_ng = 0;
    char err[512] = {0};

    // ---- sort / permutation scratch
    uint64_t *key = nullptr, *key_alt = nullptr;
    uint32_t *idx = nullptr, *idx_alt = nullptr;
    uint32_t *hist = nullptr, *hist_scan = nullptr;  // radix histograms (256 * tiles)
    uint64_t hist_cap = 0;
    uint32_t *scan_tmp = nullptr;  // partial sums for the multi-level scan
    uint64_t scan_tmp_cap = 0;
    void *gather_tmp = nullptr;  // one array of max_particles doubles for in-place permutes

    // ---- sorted copies used by tree_force on an input in any order (none with
    //      DZS_CAP_NO_COPIES)
    double *sx = nullptr, *sy = nullptr, *sz = nullptr;
    uint32_t *smult = nullptr;
    float *aold = nullptr;     // |g| on entry, for the relative opening criterion
    uint8_t *hbins = nullptr;  // bins of the individual time steps
    uint8_t *active = nullptr; // the walk's target flags (tree order)
    uint32_t cap_boxes = 0;    // batch tables sized for this many boxes

    // ---- octree (structure of arrays)
    uint64_t cap_nodes = 0;
    uint32_t *nd_first = nullptr, *nd_count = nullptr, *nd_child = nullptr;
    uint8_t *nd_nchild = nullptr, *nd_level = nullptr;
    struct dzs_node_rec *nd_rec = nullptr;  // moments and topology as the walk reads them
    int tree_deepest = 0;                    // deepest level the last build may have made
    double *gpm = nullptr;  // [3 cap] the PM force of the split individual step (capacity flag)
    uint32_t *grp_list = nullptr;  // [cap] slots of the active targets (same capacity flag)
    uint32_t *tg_flag = nullptr, *tg_tscan = nullptr, *tg_gscan = nullptr, *tg_pos = nullptr;
    uint32_t *frontier = nullptr, *frontier_next = nullptr;
    uint32_t *fr_nchild = nullptr, *fr_ninternal = nullptr, *fr_child_off = nullptr,
             *fr_int_off = nullptr;
    uint32_t *child_bounds = nullptr;  // 9 per frontier node
    uint32_t *grp_flag = nullptr, *grp_scan = nullptr, *grp_first = nullptr;
    uint32_t *walk_stack = nullptr;
    uint64_t walk_stack_slots = 0, walk_stack_depth = 0;
    uint32_t *walk_counter = nullptr;  // [0] work counter, [1] overflow flag, [8..9] pair count
    double q_coef[32] = {0};           // split-factor polynomial (see tree.hip)
    double q_wmax = -1.0;
    double q_err = 1.0;
    float4 stab[65];                   // the precision form's table of S(u) (tree.hip)
    dzs_bbox *batch_box = nullptr;     // batched step: per-box table [DZS_BATCH_MAX]
    dzs_bbox *batch_box_h = nullptr;   // pinned host staging of the same
    double *batch_tab = nullptr;       // Green's function tables of every box
    uint64_t batch_tab_cap = 0;
    uint64_t *batch_first = nullptr;   // [DZS_BATCH_MAX + 1] particle offsets of the boxes
    uint32_t *batch_members = nullptr; // [DZS_BATCH_MAX] boxes grouped by mesh side
    std::vector<int> batch_sides;      // distinct mesh sides of the prepared batch
    std::vector<size_t> batch_tw_off;  // their twiddle tables in batch_tab
    std::vector<uint32_t> batch_cls_first;  // their member ranges in batch_members
    uint64_t batch_cells = 0;          // mesh cells of all boxes
    bool batch_ready = false;          // batch tables match batch_box_h
    uint32_t batch_nb = 0;
    uint64_t *batch_first_h = nullptr; // pinned staging of the particle offsets
    dzs_step_block *step_dev = nullptr, *step_h = nullptr;
    uint32_t *cell_node = nullptr;     // walk start cells: [8^DZS_CELL_K_MAX] node ids
    uint8_t *cell_dl = nullptr;        // and the level offset of each
    double qf_err = 1.0;
    uint32_t *bstate = nullptr;        // tree build state on the device (counts, level starts,
                                       // the sticky error flags dzs_check reports)
    bool tree_built = false;           // a tree for tree_n particles is in the node arrays
    uint32_t tree_n = 0;
    char *arena = nullptr;             // tree and coarsening buffers (shared, see create())
    uint64_t arena_bytes = 0;
    bool fp32_meshes = false;          // meshes sized for the precision form only

    // ---- PM mesh
    long long *mesh_q = nullptr;  // fixed-point density accumulator, ng^3
    double2 *mesh_c = nullptr;    // complex work mesh, ng^3
    double *mesh_phi = nullptr;   // real potential, ng^3
    double *pm_tables = nullptr;  // per-axis tables (twiddles, Green factors)
    double *pm_host_tab = nullptr;  // host staging of those tables (null: a temporary)
    int pm_tab_ng = 0;
    double pm_tab_L = 0.0, pm_tab_rs = 0.0;

    // ---- DZS
    uint32_t *dz_head = nullptr;     // group head (sorted index) or 0xffffffff
    uint32_t *dz_flag = nullptr, *dz_scan = nullptr;
    double *dz_new = nullptr;        // 6 * cap: merged x,y,z,px,py,pz at the head slot
    uint32_t *dz_newmult = nullptr, *dz_newid = nullptr;
    uint32_t *dz_perm = nullptr;     // entry index of each sorted slot

    // ---- small device / host scalars
    uint32_t *d_small = nullptr;  // 64 words of device scratch (DZS_SMALL_* slots)
    uint32_t *h_small = nullptr;  // 64 words of pinned host memory

    // ---- timing
    bool timing = false;
    uint32_t timing_mask = 0xffffffffu;  // bit c: class c is timed
    dzs_timer_pool *timers = nullptr;
    // second stream (default priority) for the mesh solve that overlaps the tree build and
    // walk of kdk_step, and its fork / join events; created at first use
    hipStream_t pm_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_pm = nullptr;
    double t_ms[KC_COUNT] = {0};
    uint64_t t_calls[KC_COUNT] = {0};
};

// ---------------------------------------------------------------------------------------
// error handling
// ---------------------------------------------------------------------------------------
dzs_status dzs_fail(dzs_ctx *ctx, dzs_status code, const char *fmt, ...);

#define DZS_HIP(ctx, call)                                                                 \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return dzs_fail((ctx), DZS_EHIP, "%s failed: %s (%s:%d)", #call,               \
                            hipGetErrorString(e_), __FILE__, __LINE__);                    \
    } while (0)

#define DZS_TRY(expr)                                                                      \
    do {                                                                                   \
        dzs_status s_ = (expr);                                                            \
        if (s_ != DZS_OK)                                                                  \
            return s_;                                                                     \
    } while (0)

// launch timing: record an event pair around the launches between begin and end
void dzs_time_begin(dzs_ctx *ctx, int cls, hipStream_t s, int *slot);
void dzs_time_end(dzs_ctx *ctx, hipStream_t s, int slot);
dzs_status dzs_check_launch(dzs_ctx *ctx, const char *what);

struct dzs_timed {
    dzs_ctx *ctx;
    hipStream_t s;
    int slot;
    dzs_timed(dzs_ctx *c, int cls, hipStream_t st) : ctx(c), s(st), slot(-1) {
        dzs_time_begin(c, cls, st, &slot);
    }
    ~dzs_timed() { dzs_time_end(ctx, s, slot); }
};

// ---------------------------------------------------------------------------------------
// device helpers shared by the kernels of this library
// ---------------------------------------------------------------------------------------

// minimum image of one separation component: into [-L/2, L/2)
__device__ __forceinline__ double dzs_min_image(double d, double L) {
    if (d >= 0.5 * L)
        d -= L;
    else if (d < -0.5 * L)
        d += L;
    return d;
}

// x - L floor(x/L); a result equal to L becomes 0
__device__ __forceinline__ double dzs_wrap(double x, double L) {
    double q = floor(x / L);
    double w = x - L * q;
    if (w >= L)
        w = 0.0;
    return w;
}

// spread the low 21 bits of v to every third bit
__device__ __forceinline__ uint64_t dzs_spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// gather every third bit of v (from bit 0) into the low 21 bits: the inverse of dzs_spread3
__device__ __forceinline__ uint64_t dzs_compact3(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v | (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v | (v >> 4)) & 0x100f00f00f00f00full;
    v = (v | (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v | (v >> 16)) & 0x1f00000000ffffull;
    v = (v | (v >> 32)) & 0x1fffffull;
    return v;
}

__device__ __forceinline__ uint64_t dzs_cell(double v, double s) {
    double t = floor(v * s);
    t = t < 0.0 ? 0.0 : t;
    t = t > DZS_KEY_SIDE - 1.0 ? DZS_KEY_SIDE - 1.0 : t;
    return (uint64_t)t;
}

__device__ __forceinline__ uint64_t dzs_morton(double x, double y, double z, double s) {
    return (dzs_spread3(dzs_cell(x, s)) << 2) | (dzs_spread3(dzs_cell(y, s)) << 1) |
           dzs_spread3(dzs_cell(z, s));
}

// wave64 helpers
__device__ __forceinline__ uint32_t dzs_lane() { return __lane_id(); }

__device__ __forceinline__ uint32_t dzs_wave_incl_scan(uint32_t v) {
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d, 64);
        if (lane >= (uint32_t)d)
            v += t;
    }
    return v;
}

// Inclusive scans over the 64 lanes by DPP (no LDS round trips): a Hillis-Steele scan inside
// each row of 16 lanes by row shifts of 1, 2, 4 and 8 (a lane whose source lies before its row
// takes 0), then the last lane of row 0 broadcast into row 1 and of row 2 into row 3, then the
// last lane of row 1 into rows 2 and 3.  Every lane of the wave must be active.
#define DZS_DPP_ROW_SHR(n) (0x110 + (n))
#define DZS_DPP_ROW_BCAST15 0x142
#define DZS_DPP_ROW_BCAST31 0x143
__device__ __forceinline__ uint32_t dzs_wave_scan_add_full(uint32_t v) {
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, DZS_DPP_ROW_SHR(1), 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DZS_DPP_ROW_SHR(2), 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DZS_DPP_ROW_SHR(4), 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DZS_DPP_ROW_SHR(8), 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DZS_DPP_ROW_BCAST15, 0xa, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DZS_DPP_ROW_BCAST31, 0xc, 0xf, false);
    return (uint32_t)x;
}
__device__ __forceinline__ uint32_t dzs_wave_scan_max_full(uint32_t v) {
    uint32_t x = v;
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DZS_DPP_ROW_SHR(1), 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DZS_DPP_ROW_SHR(2), 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DZS_DPP_ROW_SHR(4), 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DZS_DPP_ROW_SHR(8), 0xf, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DZS_DPP_ROW_BCAST15, 0xa, 0xf, false));
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, DZS_DPP_ROW_BCAST31, 0xc, 0xf, false));
    return x;
}
// the value of lane 63, uniform over the wave
__device__ __forceinline__ uint32_t dzs_wave_last(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// ---------------------------------------------------------------------------------------
// launchers (defined in the .hip files)
// ---------------------------------------------------------------------------------------

// scan.hip / sort.hip
uint64_t dzs_scan_tmp_words(uint64_t n);
dzs_status dzs_scan_u32(dzs_ctx *ctx, const uint32_t *in, uint32_t *out, uint64_t n,
                        uint32_t *total_dev, hipStream_t s);
// the same over min(n_max, *n_dev) elements, the count read on the device
dzs_status dzs_scan_u32_dev(dzs_ctx *ctx, const uint32_t *in, uint32_t *out, uint64_t n_max,
                            const uint32_t *n_dev, uint32_t *total_dev, hipStream_t s);
dzs_status dzs_scan2_u32_dev(dzs_ctx *ctx, const uint32_t *in0, uint32_t *out0,
                             const uint32_t *in1, uint32_t *out1, uint64_t n_max,
                             const uint32_t *n_dev, uint32_t *total0, uint32_t *total1,
                             hipStream_t s);
uint64_t dzs_sort_hist_words(uint64_t n);
dzs_status dzs_radix_sort(dzs_ctx *ctx, uint64_t n, hipStream_t s,
                          int first_pass = 0);  // ctx->key/idx in+out; an even first_pass
dzs_status dzs_fix_ties(dzs_ctx *ctx, uint64_t n, const uint32_t *id, hipStream_t s);

// particles.hip
dzs_status dzs_launch_kick(dzs_ctx *ctx, const dzs_particles *p, double K, hipStream_t s,
                           const double *K_dev = nullptr);
void dzs_make_lc_args(const dzs_lc_params *lc, lc_args *A);
// batch = true: the box of each particle (its L) from ctx->batch_first / ctx->batch_box (nb boxes)
dzs_status dzs_launch_drift_lc(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                               const dzs_lc_params *lc, dzs_lc_ring *ring, int do_lc,
                               int do_drift, hipStream_t s, bool batch = false, uint32_t nb = 0,
                               const lc_args *A_dev = nullptr);
dzs_status dzs_launch_keys(dzs_ctx *ctx, const double *x, const double *y, const double *z,
                           uint64_t n, double L, uint64_t *key, uint32_t *idx, hipStream_t s,
                           bool batch = false, uint32_t nb = 0);
dzs_status dzs_permute_state(dzs_ctx *ctx, dzs_particles *p, const uint32_t *perm,
                             int with_g, hipStream_t s);
dzs_status dzs_gather_f64(dzs_ctx *ctx, const double *src, const uint32_t *perm, double *dst,
                          uint64_t n, hipStream_t s);
dzs_status dzs_launch_gnorm(dzs_ctx *ctx, uint64_t n, const double *gx, const double *gy,
                            const double *gz, const uint32_t *perm, float *out, hipStream_t s);
dzs_status dzs_permute_f32(dzs_ctx *ctx, float *arr, const uint32_t *perm, uint64_t n,
                           hipStream_t s);
dzs_status dzs_permute_u8(dzs_ctx *ctx, uint8_t *arr, const uint32_t *perm, uint64_t n,
                          hipStream_t s);
// individual time steps: bins of the global step (C = 2 eta a0^3 H(a0)^2, Dl = ln(a1/a0)),
// the limiter when asked, and kicks by bin
dzs_status dzs_launch_hier_bins(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                                double C, double Dl, int B, const double *x_obs, double R_lim,
                                int limiter, uint8_t *bins, hipStream_t s);
dzs_status dzs_launch_kick_bins(dzs_ctx *ctx, const dzs_particles *p, const uint8_t *bins,
                                const double *K, hipStream_t s);
// the targets that end a step at sub-step boundary jn: active[i] = (jn mod 2^(B - bin_i)) == 0
dzs_status dzs_launch_hier_active(dzs_ctx *ctx, uint64_t n, const uint8_t *bins, uint32_t jn,
                                  uint32_t B, uint8_t *active, hipStream_t s);
// flags[i] = 1 for the listed targets, 0 elsewhere (n entries); an index >= n sets
// DZS_BS_BADINPUT
dzs_status dzs_mark_targets(dzs_ctx *ctx, const uint32_t *targets, uint64_t n_targets,
                            uint64_t n, uint8_t *flags, hipStream_t s);
dzs_status dzs_gather_u8(dzs_ctx *ctx, const uint8_t *src, const uint32_t *perm, uint8_t *dst,
                         uint64_t n, hipStream_t s);
// host cosmology (cosmo.cpp): K(a0, a1) = int da / (a^2 H)
double dzs_kick_factor(double a0, double a1, double omega_m);
dzs_status dzs_gather_u32(dzs_ctx *ctx, const uint32_t *src, const uint32_t *perm,
                          uint32_t *dst, uint64_t n, hipStream_t s);

// tree.hip
// Tree build state words (ctx->bstate) that dzs_check reads: sticky error flags.
#define DZS_BS_OVERFLOW 3   // the tree needed more than the node capacity
#define DZS_BS_BADINPUT 40  // tree_force: an input out of key order under presorted, or a
                            // target index out of range (the build and walk of that call
                            // then do nothing); cleared at the end of the call into
#define DZS_BS_BADREPORT 41 // the sticky copy dzs_check reports
// end of a tree_force call: DZS_BS_BADREPORT |= DZS_BS_BADINPUT, DZS_BS_BADINPUT = 0
dzs_status dzs_latch_bad_input(dzs_ctx *ctx, hipStream_t s);
// What a walk reads and writes besides the tree and the positions: aold (the relative
// criterion's |g| on entry, tree order; null = geometric), active (per tree slot, nonzero =
// a target; null = every particle) and out_perm (tree slot -> index of g written; null = the
// slot itself).
struct dzs_walk_io {
    const float *aold = nullptr;
    const uint8_t *active = nullptr;
    const uint32_t *out_perm = nullptr;
    // a tree kept from an earlier build and refreshed (dzs_tree_refresh): the walk starts at
    // the root and unwraps targets and leaf members that crossed a face of the box
    bool kept_tree = false;
    // walk only the targets listed by dzs_tree_active_targets, in its groups
    bool target_list = false;
};
// Recompute the moments and bounding boxes of the last built tree from positions that moved
// since (same particles in the same slots), bottom-up, unwrapping members that crossed a
// face of the periodic box; a leaf with such a member is flagged in its record (pad bit 0).
dzs_status dzs_tree_refresh(dzs_ctx *ctx, const dzs_box *box, uint64_t n, const double *x,
                            const double *y, const double *z, const uint32_t *mult,
                            hipStream_t s);
// a[i] += s b[i] for the three components (exact for s = +-1)
dzs_status dzs_launch_add3(dzs_ctx *ctx, uint64_t n, double *ax, double *ay, double *az,
                           const double *bx, const double *by, const double *bz, double s,
                           hipStream_t st);
dzs_status dzs_tree_build(dzs_ctx *ctx, const dzs_box *box, uint64_t n, const double *x,
                          const double *y, const double *z, const uint32_t *mult,
                          int leaf_size, int group_size, hipStream_t s);
dzs_status dzs_tree_build_ex(dzs_ctx *ctx, const dzs_box *box, uint64_t n, const double *x,
                             const double *y, const double *z, const uint32_t *mult,
                             int leaf_size, int group_size, int KB, const dzs_bbox *boxes,
                             hipStream_t s);
// io.aold null makes a relative-criterion call use the geometric one.
dzs_status dzs_tree_walk(dzs_ctx *ctx, const dzs_box *box, uint64_t n, const double *x,
                         const double *y, const double *z, const uint32_t *mult, double *gx,
                         double *gy, double *gz, const dzs_tree_params *prm, hipStream_t s,
                         const dzs_walk_io &io = dzs_walk_io());
// tree_force, presorted: flag (DZS_BS_BADINPUT) keys in ctx->key out of order to the tree's
// depth
dzs_status dzs_check_order(dzs_ctx *ctx, uint64_t n, hipStream_t s);

dzs_status dzs_batch_roots(dzs_ctx *ctx, dzs_bbox *boxes, hipStream_t s);
dzs_status dzs_tree_check(dzs_ctx *ctx, hipStream_t s);
dzs_status dzs_tree_walk_ex(dzs_ctx *ctx, const dzs_box *box, uint64_t n, const double *x,
                            const double *y, const double *z, const uint32_t *mult, double *gx,
                            double *gy, double *gz, const dzs_tree_params *prm,
                            const dzs_bbox *boxes, hipStream_t s,
                            const dzs_walk_io &io = dzs_walk_io());

// pm.hip
bool dzs_pm_mesh_ok(int ng);
dzs_status dzs_pm_solve(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                        const dzs_pm_params *prm, hipStream_t s);
dzs_status dzs_pm_apply(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                        const dzs_pm_params *prm, hipStream_t s);
dzs_status dzs_pm_run(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                      const dzs_pm_params *prm, hipStream_t s);
dzs_status dzs_pm_batch_prepare(dzs_ctx *ctx, uint32_t nb, dzs_bbox *hb, hipStream_t s);
dzs_status dzs_pm_run_batch(dzs_ctx *ctx, const dzs_particles *p, int precision,
                            int32_t tile_chunk, const dzs_bbox *db, double G, hipStream_t s);

// coarsen.hip
// d_small word slots: 8 the coarsening survivor count, 9 its head count, 16..17 the bits of
// the dynamical criterion's min g.g (8-byte aligned).
#define DZS_SMALL_AMIN 16
// d_small word 20: set when the keys of a coarsened state are out of order
#define DZS_SMALL_UNSORTED 20
// d_small word 24: largest bin + 1 inside the limiter sphere (0: nobody inside)
#define DZS_SMALL_HIER_CAP 24
// d_small words 26..27: the bits of the current sub-step's largest drift bound; 28..29: the
// bound on any particle's displacement since the kept tree was built (a double)
#define DZS_SMALL_DRIFT_STEP 26
#define DZS_SMALL_DRIFT_TOTAL 28
// d_small word 30: the number of targets in ctx->grp_list, 31: the number of their groups;
// 32..39: particles per time-step bin
#define DZS_SMALL_GROUP_LIST 30
#define DZS_SMALL_BIN_COUNT 32
// Particles per bin (bins 0..7) into d_small[DZS_SMALL_BIN_COUNT ..].
dzs_status dzs_launch_bin_hist(dzs_ctx *ctx, uint64_t n, const uint8_t *bins, hipStream_t s);
// The slots of the targets flagged in `active`, ascending, in ctx->grp_list (their number in
// d_small[DZS_SMALL_GROUP_LIST]), grouped as the last built tree groups them, groups without
// a flagged target left out (start positions in ctx->tg_pos, their number in the next word),
// for the walk to take instead of every tree group.
dzs_status dzs_tree_active_targets(dzs_ctx *ctx, uint64_t n, const uint8_t *active,
                                   hipStream_t s);
// The kept tree's displacement bound: reset (at the build), add a drift's
// max_i (|px| + |py| + |pz|) |D| (before it), both on the device.
dzs_status dzs_drift_bound_reset(dzs_ctx *ctx, hipStream_t s);
dzs_status dzs_drift_bound_add(dzs_ctx *ctx, const dzs_particles *p, double D, hipStream_t s);
// Reduce the dynamical criterion's a_min^2 over the state (before any reordering that leaves
// g behind) into d_small[DZS_SMALL_AMIN].
dzs_status dzs_coarsen_amin(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                            const dzs_coarsen_params *prm, hipStream_t s);
// Keys of the coarsened state into ctx->key and whether they are still ascending
// (synchronises the stream).
dzs_status dzs_coarsen_rekey(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                             bool *sorted, hipStream_t s);
dzs_status dzs_coarsen_sorted(dzs_ctx *ctx, const dzs_box *box, dzs_particles *p,
                              const dzs_coarsen_params *prm, uint32_t *group_of,
                              dzs_coarsen_report *report, hipStream_t s);

// cosmo.cpp (host)
void dzs_merge_thresholds(double L, double R_lc, double b, double theta, double *T2);
