// Exclusive prefix scan (u32) and stable LSD radix sort of (u64 Morton key, u32 index)
// pairs for gfx950.
//
// Sort: 8 passes of 8-bit digits (the sort before a tree build skips the lowest two: the tree
// reads the keys' order to level 15 only).  Per pass: (1) each 256-thread block counts the digits of
// its 4096-key tile in LDS; (2) one exclusive scan over the digit-major table gives every
// (digit, tile) its global start; (3) each block ranks its tile stably — each wave ranks its
// own quarter of the tile by wave-level digit matching through eight ballots, then the waves'
// digit counts become offsets — stages the tile in LDS in local digit order, and writes it out
// so that consecutive lanes write consecutive addresses of the same digit run.
#include "internal.h"

#define SCAN_THREADS 256
#define SCAN_ITEMS 16
#define SCAN_TILE (SCAN_THREADS * SCAN_ITEMS)

#define SORT_THREADS 256
#define SORT_ITEMS 16
#define SORT_TILE (SORT_THREADS * SORT_ITEMS)

// ---------------------------------------------------------------------------------------
// block-wide exclusive scan of one value per thread (256 threads = 4 wave64)
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t block_excl_scan_256(uint32_t v, uint32_t *s_wave,
                                                       uint32_t *total) {
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t incl = dzs_wave_incl_scan(v);
    if (lane == 63)
        s_wave[wave] = incl;
    __syncthreads();
    uint32_t off = 0;
    for (uint32_t w = 0; w < wave; ++w)
        off += s_wave[w];
    uint32_t tot = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    __syncthreads();
    if (total)
        *total = tot;
    return off + incl - v;
}

// n_dev (optional): the element count is min(n, *n_dev), read on the device, so that a
// launch sized for an upper bound needs no host copy of the count.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const uint32_t *__restrict__ in,
                                                              uint64_t n,
                                                              uint32_t *__restrict__ part,
                                                              const uint32_t *__restrict__ n_dev) {
    __shared__ uint32_t s_wave[4];
    if (n_dev && *n_dev < n)
        n = *n_dev;
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    uint32_t sum = 0;
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        uint64_t e = base + (uint64_t)r * SCAN_THREADS + threadIdx.x;
        if (e < n)
            sum += in[e];
    }
    uint32_t tot;
    block_excl_scan_256(sum, s_wave, &tot);
    if (threadIdx.x == 0)
        part[blockIdx.x] = tot;
}

// Offset of tile b from the unscanned tile sums part[0..b) (b <= SCAN_TILE), summed by the
// block; every thread returns it.
__device__ __forceinline__ uint32_t tile_offset(const uint32_t *__restrict__ part, uint32_t b,
                                                uint32_t *s_wave) {
    uint32_t sum = 0;
    for (uint32_t i = threadIdx.x; i < b; i += SCAN_THREADS)
        sum += part[i];
    uint32_t tot;
    block_excl_scan_256(sum, s_wave, &tot);
    return tot;
}

// scan one tile (blocked: thread t owns items t*16 .. t*16+15), adding the tile offset: the
// scanned tile sums offs[b], or the unscanned tile sums part[0..b) (two-launch scan), or 0
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tile(const uint32_t *__restrict__ in,
                                                            uint32_t *__restrict__ out,
                                                            uint64_t n,
                                                            const uint32_t *__restrict__ offs,
                                                            const uint32_t *__restrict__ part,
                                                            uint32_t *__restrict__ total,
                                                            const uint32_t *__restrict__ n_dev) {
    __shared__ uint32_t s_wave[4];
    if (n_dev && *n_dev < n)
        n = *n_dev;
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t sum = 0;
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        uint64_t e = base + r;
        v[r] = e < n ? in[e] : 0u;
        sum += v[r];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan_256(sum, s_wave, &tot);
    if (offs)
        run += offs[blockIdx.x];
    else if (part)
        run += tile_offset(part, blockIdx.x, s_wave);
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        uint64_t e = base + r;
        if (e < n)
            out[e] = run;
        run += v[r];
    }
    if (total && threadIdx.x == SCAN_THREADS - 1 && blockIdx.x == gridDim.x - 1)
        *total = run;
}

// Two independent scans of the same length in one pass (the tree build's child and
// internal-node counts): tile sums of in0 to part[b], of in1 to part[nb + b].
__global__ __launch_bounds__(SCAN_THREADS) void k_scan2_reduce(const uint32_t *__restrict__ in0,
                                                               const uint32_t *__restrict__ in1,
                                                               uint64_t n,
                                                               uint32_t *__restrict__ part,
                                                               const uint32_t *__restrict__ n_dev) {
    __shared__ uint32_t s_wave[4];
    if (n_dev && *n_dev < n)
        n = *n_dev;
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    uint32_t s0 = 0, s1 = 0;
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        uint64_t e = base + (uint64_t)r * SCAN_THREADS + threadIdx.x;
        if (e < n) {
            s0 += in0[e];
            s1 += in1[e];
        }
    }
    uint32_t t0, t1;
    block_excl_scan_256(s0, s_wave, &t0);
    block_excl_scan_256(s1, s_wave, &t1);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = t0;
        part[gridDim.x + blockIdx.x] = t1;
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan2_tile(
    const uint32_t *__restrict__ in0, uint32_t *__restrict__ out0,
    const uint32_t *__restrict__ in1, uint32_t *__restrict__ out1, uint64_t n,
    const uint32_t *__restrict__ part, uint32_t *__restrict__ total0,
    uint32_t *__restrict__ total1, const uint32_t *__restrict__ n_dev) {
    __shared__ uint32_t s_wave[4];
    if (n_dev && *n_dev < n)
        n = *n_dev;
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v0[SCAN_ITEMS], v1[SCAN_ITEMS];
    uint32_t s0 = 0, s1 = 0;
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        uint64_t e = base + r;
        v0[r] = e < n ? in0[e] : 0u;
        v1[r] = e < n ? in1[e] : 0u;
        s0 += v0[r];
        s1 += v1[r];
    }
    uint32_t t;
    uint32_t run0 = block_excl_scan_256(s0, s_wave, &t);
    uint32_t run1 = block_excl_scan_256(s1, s_wave, &t);
    if (part) {
        run0 += tile_offset(part, blockIdx.x, s_wave);
        run1 += tile_offset(part + gridDim.x, blockIdx.x, s_wave);
    }
#pragma unroll
    for (int r = 0; r < SCAN_ITEMS; ++r) {
        uint64_t e = base + r;
        if (e < n) {
            out0[e] = run0;
            out1[e] = run1;
        }
        run0 += v0[r];
        run1 += v1[r];
    }
    if (threadIdx.x == SCAN_THREADS - 1 && blockIdx.x == gridDim.x - 1) {
        *total0 = run0;
        *total1 = run1;
    }
}

uint64_t dzs_scan_tmp_words(uint64_t n) {
    uint64_t words = 0;
    while (n > SCAN_TILE) {
        uint64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
        words += 2 * nb;
        n = nb;
    }
    return words + 64;
}

// One tile: one launch.  Up to SCAN_TILE tiles: tile sums, then the tiles, each adding the
// sum of the tile sums before it (two launches).  More: the tile sums are scanned recursively.
static dzs_status scan_rec(dzs_ctx *ctx, const uint32_t *in, uint32_t *out, uint64_t n,
                           uint32_t *total_dev, uint32_t *tmp, const uint32_t *n_dev,
                           hipStream_t s) {
    uint64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb <= 1) {
        hipLaunchKernelGGL(k_scan_tile, dim3(1), dim3(SCAN_THREADS), 0, s, in, out, n,
                           (const uint32_t *)nullptr, (const uint32_t *)nullptr, total_dev, n_dev);
        return dzs_check_launch(ctx, "scan_tile");
    }
    // tiles past the device count sum to zero, so the partial sums need no count of their own
    uint32_t *part = tmp, *part_scan = tmp + nb;
    hipLaunchKernelGGL(k_scan_reduce, dim3((uint32_t)nb), dim3(SCAN_THREADS), 0, s, in, n, part,
                       n_dev);
    DZS_TRY(dzs_check_launch(ctx, "scan_reduce"));
    if (nb <= SCAN_TILE) {
        hipLaunchKernelGGL(k_scan_tile, dim3((uint32_t)nb), dim3(SCAN_THREADS), 0, s, in, out, n,
                           (const uint32_t *)nullptr, (const uint32_t *)part, total_dev, n_dev);
        return dzs_check_launch(ctx, "scan_tile");
    }
    DZS_TRY(scan_rec(ctx, part, part_scan, nb, nullptr, tmp + 2 * nb, nullptr, s));
    hipLaunchKernelGGL(k_scan_tile, dim3((uint32_t)nb), dim3(SCAN_THREADS), 0, s, in, out, n,
                       (const uint32_t *)part_scan, (const uint32_t *)nullptr, total_dev, n_dev);
    return dzs_check_launch(ctx, "scan_tile");
}

dzs_status dzs_scan_u32(dzs_ctx *ctx, const uint32_t *in, uint32_t *out, uint64_t n,
                        uint32_t *total_dev, hipStream_t s) {
    if (n == 0) {
        if (total_dev)
            DZS_HIP(ctx, hipMemsetAsync(total_dev, 0, sizeof(uint32_t), s));
        return DZS_OK;
    }
    if (dzs_scan_tmp_words(n) > ctx->scan_tmp_cap)
        return dzs_fail(ctx, DZS_ECAPACITY, "scan of %llu elements exceeds scratch",
                        (unsigned long long)n);
    return scan_rec(ctx, in, out, n, total_dev, ctx->scan_tmp, nullptr, s);
}

dzs_status dzs_scan_u32_dev(dzs_ctx *ctx, const uint32_t *in, uint32_t *out, uint64_t n_max,
                            const uint32_t *n_dev, uint32_t *total_dev, hipStream_t s) {
    if (n_max == 0)
        n_max = 1;
    if (dzs_scan_tmp_words(n_max) > ctx->scan_tmp_cap)
        return dzs_fail(ctx, DZS_ECAPACITY, "scan of %llu elements exceeds scratch",
                        (unsigned long long)n_max);
    return scan_rec(ctx, in, out, n_max, total_dev, ctx->scan_tmp, n_dev, s);
}

// Two exclusive scans of n_max (count on the device) elements with one pair of launches when
// they span at most SCAN_TILE tiles; otherwise one scan after the other.
dzs_status dzs_scan2_u32_dev(dzs_ctx *ctx, const uint32_t *in0, uint32_t *out0,
                             const uint32_t *in1, uint32_t *out1, uint64_t n_max,
                             const uint32_t *n_dev, uint32_t *total0, uint32_t *total1,
                             hipStream_t s) {
    if (n_max == 0)
        n_max = 1;
    const uint64_t nb = (n_max + SCAN_TILE - 1) / SCAN_TILE;
    if (nb > SCAN_TILE) {
        DZS_TRY(dzs_scan_u32_dev(ctx, in0, out0, n_max, n_dev, total0, s));
        return dzs_scan_u32_dev(ctx, in1, out1, n_max, n_dev, total1, s);
    }
    if (dzs_scan_tmp_words(n_max) > ctx->scan_tmp_cap)
        return dzs_fail(ctx, DZS_ECAPACITY, "scan of %llu elements exceeds scratch",
                        (unsigned long long)n_max);
    uint32_t *part = nullptr;
    if (nb > 1) {
        part = ctx->scan_tmp;  // 2 nb words
        hipLaunchKernelGGL(k_scan2_reduce, dim3((uint32_t)nb), dim3(SCAN_THREADS), 0, s, in0, in1,
                           n_max, part, n_dev);
        DZS_TRY(dzs_check_launch(ctx, "scan2_reduce"));
    }
    hipLaunchKernelGGL(k_scan2_tile, dim3((uint32_t)nb), dim3(SCAN_THREADS), 0, s, in0, out0, in1,
                       out1, n_max, (const uint32_t *)part, total0, total1, n_dev);
    return dzs_check_launch(ctx, "scan2_tile");
}

// ---------------------------------------------------------------------------------------
// radix sort
// ---------------------------------------------------------------------------------------
uint64_t dzs_sort_hist_words(uint64_t n) {
    uint64_t tiles = (n + SORT_TILE - 1) / SORT_TILE;
    if (tiles == 0)
        tiles = 1;
    return 256 * tiles;
}

__global__ __launch_bounds__(SORT_THREADS) void k_radix_hist(const uint64_t *__restrict__ key,
                                                             uint64_t n, int shift,
                                                             uint32_t *__restrict__ hist,
                                                             uint32_t tiles) {
    __shared__ uint32_t s_h[256];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * SORT_TILE;
    for (int r = 0; r < SORT_ITEMS; ++r) {
        uint64_t e = base + (uint64_t)r * SORT_THREADS + threadIdx.x;
        if (e < n)
            atomicAdd(&s_h[(uint32_t)(key[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * tiles + blockIdx.x] = s_h[threadIdx.x];
}

// The scanned histogram from digit-major ([256][tiles], the order of the global scan) to
// tile-major ([tiles][256]), so that a scatter tile reads its 256 start offsets as one
// contiguous kilobyte: 64 tiles per workgroup through an LDS block (rows padded by one word).
__global__ __launch_bounds__(SORT_THREADS) void k_hist_tile_major(const uint32_t *__restrict__ in,
                                                                  uint32_t *__restrict__ out,
                                                                  uint32_t tiles) {
    static_assert(SORT_THREADS == 256, "one thread per digit");
    __shared__ uint32_t s_t[256][65];
    const uint32_t t0 = blockIdx.x * 64u;
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    for (uint32_t d = w; d < 256u; d += SORT_THREADS / 64) {
        const uint32_t t = t0 + lane;
        s_t[d][lane] = t < tiles ? in[(uint64_t)d * tiles + t] : 0u;
    }
    __syncthreads();
    for (uint32_t r = 0; r < 64u && t0 + r < tiles; ++r)
        out[(uint64_t)(t0 + r) * 256u + threadIdx.x] = s_t[threadIdx.x][r];
}

// Each wave ranks its own contiguous quarter of the tile (16 rounds of 64 keys, in input
// order) against running per-wave digit counts in LDS, with no block barrier between rounds:
// lanes holding the same digit are found with eight ballots, the lowest of them advances the
// wave's count.  Then the waves' counts become offsets (wave 0's keys of a digit first), the
// tile is staged in LDS in local digit order, and written out so that consecutive lanes write
// consecutive addresses of the same digit run.  Equal digits keep their input order.
__global__ __launch_bounds__(SORT_THREADS) void k_radix_scatter(
    const uint64_t *__restrict__ key_in, const uint32_t *__restrict__ idx_in,
    uint64_t *__restrict__ key_out, uint32_t *__restrict__ idx_out, uint64_t n, int shift,
    const uint32_t *__restrict__ gstart) {
    constexpr int WAVES = SORT_THREADS / 64;
    constexpr int ROUNDS = SORT_ITEMS;  // rounds of 64 keys per wave: 4 waves x 16 x 64 = tile
    __shared__ uint64_t s_key[SORT_TILE];
    __shared__ uint32_t s_idx[SORT_TILE];
    __shared__ uint32_t s_lstart[256], s_gstart[256];
    __shared__ uint32_t s_wcnt[WAVES][256];
    __shared__ uint32_t s_wave[4];

    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t base = (uint64_t)blockIdx.x * SORT_TILE;
    const uint32_t cnt = (uint32_t)((n - base) < SORT_TILE ? (n - base) : SORT_TILE);
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));

    // the tile's global start of each digit (tile-major scanned histogram)
    s_gstart[tid] = gstart[(uint64_t)blockIdx.x * 256u + tid];
    for (int w = 0; w < WAVES; ++w)
        s_wcnt[w][tid] = 0;
    __syncthreads();

    uint64_t k[ROUNDS];
    uint32_t id[ROUNDS], pos[ROUNDS];
    const uint32_t q0 = wave * (ROUNDS * 64);
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const uint32_t local = q0 + (uint32_t)r * 64u + lane;
        const bool valid = local < cnt;
        k[r] = valid ? key_in[base + local] : 0ull;
        id[r] = valid ? idx_in[base + local] : 0u;
        const uint32_t d = (uint32_t)(k[r] >> shift) & 255u;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bal = __ballot(((d >> bit) & 1u) != 0u);
            m &= ((d >> bit) & 1u) ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(m & lt_mask);
        // every lane reads the wave's count before the lowest lane of the digit advances it
        // (LDS operations of one wave complete in order)
        const uint32_t prev = s_wcnt[wave][d];
        pos[r] = prev + rank;
        if (valid && rank == 0)
            s_wcnt[wave][d] = prev + (uint32_t)__popcll(m);
    }
    __syncthreads();
    {
        // the tile's count of digit tid (the waves' counts), its start inside the tile, and
        // the offsets of each wave's run of it
        uint32_t c = 0;
        for (int w = 0; w < WAVES; ++w)
            c += s_wcnt[w][tid];
        const uint32_t ls = block_excl_scan_256(c, s_wave, nullptr);
        s_lstart[tid] = ls;
        uint32_t run = ls;
        for (int w = 0; w < WAVES; ++w) {
            const uint32_t t = s_wcnt[w][tid];
            s_wcnt[w][tid] = run;
            run += t;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const uint32_t local = q0 + (uint32_t)r * 64u + lane;
        if (local < cnt) {
            const uint32_t d = (uint32_t)(k[r] >> shift) & 255u;
            const uint32_t lp = s_wcnt[wave][d] + pos[r];
            s_key[lp] = k[r];
            s_idx[lp] = id[r];
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < cnt; i += SORT_THREADS) {
        const uint64_t kk = s_key[i];
        const uint32_t d = (uint32_t)(kk >> shift) & 255u;
        const uint64_t gp = (uint64_t)s_gstart[d] + (i - s_lstart[d]);
        key_out[gp] = kk;
        idx_out[gp] = s_idx[i];
    }
}

dzs_status dzs_radix_sort(dzs_ctx *ctx, uint64_t n, hipStream_t s, int first_pass) {
    if (n <= 1)
        return DZS_OK;
    if (n > 0xffffffffull)
        return dzs_fail(ctx, DZS_EINVAL, "radix sort: n exceeds 2^32-1");
    if (first_pass < 0 || first_pass > 6 || (first_pass & 1))
        return dzs_fail(ctx, DZS_EINVAL, "radix sort: first pass %d", first_pass);
    const uint32_t tiles = (uint32_t)((n + SORT_TILE - 1) / SORT_TILE);
    const uint64_t words = 256ull * tiles;
    if (words > ctx->hist_cap)
        return dzs_fail(ctx, DZS_ECAPACITY, "radix sort histogram exceeds scratch");
    dzs_timed t(ctx, KC_SORT, s);
    uint64_t *kin = ctx->key, *kout = ctx->key_alt;
    uint32_t *iin = ctx->idx, *iout = ctx->idx_alt;
    for (int pass = first_pass; pass < 8; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_radix_hist, dim3(tiles), dim3(SORT_THREADS), 0, s, kin, n, shift,
                           ctx->hist, tiles);
        DZS_TRY(dzs_check_launch(ctx, "radix_hist"));
        DZS_TRY(dzs_scan_u32(ctx, ctx->hist, ctx->hist_scan, words, nullptr, s));
        // the counts are no longer needed: their buffer takes the tile-major starts
        hipLaunchKernelGGL(k_hist_tile_major, dim3((tiles + 63u) / 64u), dim3(SORT_THREADS), 0,
                           s, (const uint32_t *)ctx->hist_scan, ctx->hist, tiles);
        DZS_TRY(dzs_check_launch(ctx, "radix_hist_tile_major"));
        hipLaunchKernelGGL(k_radix_scatter, dim3(tiles), dim3(SORT_THREADS), 0, s, kin, iin,
                           kout, iout, n, shift, (const uint32_t *)ctx->hist);
        DZS_TRY(dzs_check_launch(ctx, "radix_scatter"));
        uint64_t *tk = kin; kin = kout; kout = tk;
        uint32_t *ti = iin; iin = iout; iout = ti;
    }
    // an even number of passes: the result is back in ctx->key / ctx->idx
    return DZS_OK;
}

// Equal keys keep their input order (the sort is stable); where a canonical order is
// needed, runs of equal keys are re-ordered by ascending particle id (runs are short).
__global__ void k_fix_ties(const uint64_t *__restrict__ key, uint32_t *__restrict__ idx,
                           const uint32_t *__restrict__ id, uint64_t n) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i + 1 >= n)
        return;
    if (key[i] != key[i + 1] || (i > 0 && key[i - 1] == key[i]))
        return;
    uint64_t e = i + 1;
    while (e < n && key[e] == key[i])
        ++e;
    for (uint64_t a = i + 1; a < e; ++a) {
        uint32_t v = idx[a];
        uint32_t vid = id[v];
        uint64_t b = a;
        while (b > i && id[idx[b - 1]] > vid) {
            idx[b] = idx[b - 1];
            --b;
        }
        idx[b] = v;
    }
}

dzs_status dzs_fix_ties(dzs_ctx *ctx, uint64_t n, const uint32_t *id, hipStream_t s) {
    if (n <= 1)
        return DZS_OK;
    dzs_timed t(ctx, KC_SORT, s);
    uint32_t blocks = (uint32_t)((n + 255) / 256);
    hipLaunchKernelGGL(k_fix_ties, dim3(blocks), dim3(256), 0, s, ctx->key, ctx->idx, id, n);
    return dzs_check_launch(ctx, "fix_ties");
}
