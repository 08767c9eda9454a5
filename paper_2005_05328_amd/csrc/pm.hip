// Particle-mesh long-range force (paper Sec. 2.1: density on a uniform grid, Poisson
// equation in Fourier space, Gaussian split kernel).
//
//   deposit     cloud-in-cell, deterministic: each contribution mult * w_x w_y w_z is rounded
//               to 32.32 fixed point and added with 64-bit integer atomics, so the mesh does
//               not depend on the order the GPU adds in
//   FFT         3-D complex transform as three passes of 1-D line transforms, each line held
//               in LDS (mixed radix 4/2/3 Stockham, autosorting, twiddles from a host table);
//               the x pass reads the fixed-point mesh directly, the z pass multiplies by the
//               Green's function and transforms back in the same kernel, the last inverse x
//               pass writes the real potential
//   Green       -4 pi G exp(-k^2 r_s^2) / (k^2 W(k)^2) / N_g^3, separable per-axis tables
//   gradient +  the 4-point difference of the potential at the 8 cloud-in-cell corners of each
//   interp      particle, weighted with the same cloud-in-cell weights (one kernel)
//
// Mesh layout: index (ix * N_g + iy) * N_g + iz.  Mesh points at j * Delta, Delta = L / N_g.
#include <limits.h>
#include <math.h>
#include <vector>

#include "internal.h"

#define PM_THREADS 256
#define FFT_THREADS 256
#define FFT_ELEMS 2048       // complex elements per workgroup tile (32 KB in FP64)
#define FFT_MAX_STAGES 12
#define FFT_MAX_SLOTS 4
#define DEP_FRAC 4294967296.0  // 2^32: fixed-point scale of the deposit
#define DEP_TILE 4096          // mesh points of the LDS deposit tile (32 KB of 64-bit sums)
#define INTERP_TILE_BYTES 32768  // LDS interpolation tile (8192 FP32 / 4096 FP64 values)
#define PM_PIECE_MIN 128       // smallest piece of a chunk that still tries an LDS tile

static inline uint32_t blocks_for(uint64_t n, uint32_t t) { return (uint32_t)((n + t - 1) / t); }

struct fft_plan {
    int n;                       // line length
    int n_stages;
    int radix[FFT_MAX_STAGES];
};

// A batch of boxes, each with its own mesh at its own offset of the mesh arrays.  Deposit and
// interpolation find a particle's box from its key prefix; the FFT kernels of one mesh-size
// class run blocks_per_mesh blocks for each member box.  boxes == nullptr: a single box.
struct pm_batch {
    const dzs_bbox *boxes;
    const uint32_t *members;
    int blocks_per_mesh;
    const uint64_t *key;
};

// ---------------------------------------------------------------------------------------
// LDS line FFT
// ---------------------------------------------------------------------------------------
// C is double2 (plain form) or float2 (precision form); R its component type.
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }

template <int R, bool INV, typename C>
__device__ __forceinline__ void dft_small(C *v) {
    typedef decltype(v[0].x) Rt;
    if (R == 2) {
        C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if (R == 4) {
        C a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
        C c = cadd(v[1], v[3]), t = csub(v[1], v[3]);
        // forward: t * (-i) = (t.y, -t.x); inverse: t * (+i) = (-t.y, t.x)
        C d = INV ? C{-t.y, t.x} : C{t.y, -t.x};
        v[0] = cadd(a, c);
        v[1] = cadd(b, d);
        v[2] = csub(a, c);
        v[3] = csub(b, d);
    } else {  // R == 3
        const Rt s3 = Rt(0.86602540378443865);  // sqrt(3)/2
        C t = cadd(v[1], v[2]), s = csub(v[1], v[2]);
        C m = C{v[0].x - Rt(0.5) * t.x, v[0].y - Rt(0.5) * t.y};
        // forward: X1 = m - i s3 s, X2 = m + i s3 s ; inverse swaps the sign of i
        C is = INV ? C{-s3 * s.y, s3 * s.x} : C{s3 * s.y, -s3 * s.x};
        v[0] = cadd(v[0], t);
        v[1] = cadd(m, is);
        v[2] = csub(m, is);
    }
}

// One Stockham stage over TL lines held in LDS.  Element e of line l lives at
// buf[e * se + l * sl].  All loads of the stage complete before any store (barrier), so the
// stage runs in place.
template <int R, bool INV, typename C>
__device__ void fft_stage(C *buf, const C *tw, int n, int TL, int se, int sl, int Ns) {
    const int nb = n / R;
    const int total = TL * nb;
    const int step = n / (Ns * R);
    C v[FFT_MAX_SLOTS][R];
#pragma unroll
    for (int q = 0; q < FFT_MAX_SLOTS; ++q) {
        const int b = threadIdx.x + q * FFT_THREADS;
        if (b < total) {
            int l, j;
            if (sl == 1) {
                l = b % TL;
                j = b / TL;
            } else {
                j = b % nb;
                l = b / nb;
            }
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[q][r] = buf[(j + r * nb) * se + l * sl];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < FFT_MAX_SLOTS; ++q) {
        const int b = threadIdx.x + q * FFT_THREADS;
        if (b < total) {
            int l, j;
            if (sl == 1) {
                l = b % TL;
                j = b / TL;
            } else {
                j = b % nb;
                l = b / nb;
            }
            const int k = j % Ns;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                C w = tw[r * k * step];
                if (INV)
                    w.y = -w.y;
                v[q][r] = cmul(v[q][r], w);
            }
            dft_small<R, INV>(v[q]);
            const int idxD = (j / Ns) * Ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r)
                buf[(idxD + r * Ns) * se + l * sl] = v[q][r];
        }
    }
    __syncthreads();
}

template <bool INV, typename C>
__device__ void fft_lines(C *buf, const C *tw, const fft_plan &P, int TL, int se, int sl) {
    int Ns = 1;
    for (int s = 0; s < P.n_stages; ++s) {
        const int R = P.radix[s];
        if (R == 4)
            fft_stage<4, INV>(buf, tw, P.n, TL, se, sl, Ns);
        else if (R == 2)
            fft_stage<2, INV>(buf, tw, P.n, TL, se, sl, Ns);
        else
            fft_stage<3, INV>(buf, tw, P.n, TL, se, sl, Ns);
        Ns *= R;
    }
}

// twiddles e^{-2 pi i m / n} from the FP64 host table, rounded to the form's precision
template <typename C>
__device__ __forceinline__ void load_twiddles(C *s_tw, const double2 *tw, int n) {
    typedef decltype(s_tw[0].x) Rt;
    for (int i = threadIdx.x; i < n; i += FFT_THREADS)
        s_tw[i] = C{Rt(tw[i].x), Rt(tw[i].y)};
}

// ---------------------------------------------------------------------------------------
// deposit
// ---------------------------------------------------------------------------------------
// Unwrapped cloud-in-cell base index floor(x / Delta) of one axis and the weights of the
// base point and the next one (x times the reciprocal of Delta: a loop over particles of one
// mesh computes the reciprocal once).
__device__ __forceinline__ int cic_base(double x, double delta, double &w0, double &w1) {
    const double u = x * (1.0 / delta);
    const double f = floor(u);
    w1 = u - f;
    w0 = 1.0 - w1;
    return (int)f;
}

__device__ __forceinline__ int wrap_index(int i, int ng) {
    i %= ng;
    return i < 0 ? i + ng : i;
}

// The same for an index within one period of the mesh, -ng <= i < 2 ng, by compares instead
// of a division: a stencil point i0 + d (|d| <= 3 < ng), or a tile point (the base indices of
// positions in [0, L) lie in [0, ng], a tile reaches at most ng + 2 points past its lowest and
// starts at most 2 before it; meshes have at least 8 points per side).
__device__ __forceinline__ int wrap_near(int i, int ng) {
    return i < 0 ? i + ng : (i >= ng ? i - ng : i);
}

__device__ __forceinline__ void cic_axis(double x, double delta, int ng, int &i0, int &i1,
                                         double &w0, double &w1) {
    const int i = wrap_index(cic_base(x, delta, w0, w1), ng);
    i0 = i;
    i1 = i + 1 == ng ? 0 : i + 1;
}

// One corner's contribution in 32.32 fixed point (the same expression on every path, so the
// integer sums, and with them the mesh, do not depend on which path adds them).
__device__ __forceinline__ unsigned long long dep_fixed(double m, double wx, double wy, double wz) {
    return (unsigned long long)llrint(m * wx * wy * wz);
}

// Direct deposit: eight 64-bit atomic adds per particle into the mesh.
__device__ __forceinline__ void dep_direct(const double *__restrict__ x, const double *__restrict__ y,
                                           const double *__restrict__ z,
                                           const uint32_t *__restrict__ mult, uint64_t p,
                                           double delta, int ng, unsigned long long *q) {
    int ix[2], iy[2], iz[2];
    double wx[2], wy[2], wz[2];
    cic_axis(x[p], delta, ng, ix[0], ix[1], wx[0], wx[1]);
    cic_axis(y[p], delta, ng, iy[0], iy[1], wy[0], wy[1]);
    cic_axis(z[p], delta, ng, iz[0], iz[1], wz[0], wz[1]);
    const double m = (double)mult[p] * DEP_FRAC;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const unsigned long long iv = dep_fixed(m, wx[a], wy[b], wz[c]);
                if (iv)
                    atomicAdd(&q[((uint64_t)ix[a] * ng + iy[b]) * ng + iz[c]], iv);
            }
}

__global__ __launch_bounds__(PM_THREADS) void k_pm_deposit(uint64_t n, const double *__restrict__ x,
                                                           const double *__restrict__ y,
                                                           const double *__restrict__ z,
                                                           const uint32_t *__restrict__ mult,
                                                           double delta, int ng,
                                                           unsigned long long *__restrict__ q,
                                                           pm_batch B) {
    uint64_t p = (uint64_t)blockIdx.x * PM_THREADS + threadIdx.x;
    if (p >= n)
        return;
    if (B.boxes) {
        const dzs_bbox &bx = B.boxes[B.key[p] >> DZS_BATCH_SHIFT];
        delta = bx.delta;
        ng = bx.ng;
        q += bx.mesh_off;
    }
    dep_direct(x, y, z, mult, p, delta, ng, q);
}

// Bounding box of the cloud-in-cell base indices of particles [p0, p1) (unwrapped) and the
// range of their boxes (batch), reduced over the workgroup: every thread returns the same
// values.  s_red: PM_THREADS / 64 rows of 8 ints of LDS.
__device__ __forceinline__ void chunk_bounds(uint64_t p0, uint64_t p1, const double *__restrict__ x,
                                             const double *__restrict__ y,
                                             const double *__restrict__ z, double delta,
                                             const pm_batch &B, int (*s_red)[8], int &lo0,
                                             int &lo1, int &lo2, int &hi0, int &hi1, int &hi2,
                                             int &blo, int &bhi) {
    const uint32_t tid = threadIdx.x;
    lo0 = lo1 = lo2 = blo = INT_MAX;
    hi0 = hi1 = hi2 = bhi = INT_MIN;
    for (uint64_t p = p0 + tid; p < p1; p += PM_THREADS) {
        double d = delta;
        if (B.boxes) {
            const int b = (int)(B.key[p] >> DZS_BATCH_SHIFT);
            d = B.boxes[b].delta;
            blo = min(blo, b);
            bhi = max(bhi, b);
        }
        double w0, w1;
        const int i = cic_base(x[p], d, w0, w1), j = cic_base(y[p], d, w0, w1),
                  k = cic_base(z[p], d, w0, w1);
        lo0 = min(lo0, i); hi0 = max(hi0, i);
        lo1 = min(lo1, j); hi1 = max(hi1, j);
        lo2 = min(lo2, k); hi2 = max(hi2, k);
    }
    for (int o = 32; o >= 1; o >>= 1) {
        lo0 = min(lo0, __shfl_xor(lo0, o, 64)); hi0 = max(hi0, __shfl_xor(hi0, o, 64));
        lo1 = min(lo1, __shfl_xor(lo1, o, 64)); hi1 = max(hi1, __shfl_xor(hi1, o, 64));
        lo2 = min(lo2, __shfl_xor(lo2, o, 64)); hi2 = max(hi2, __shfl_xor(hi2, o, 64));
        blo = min(blo, __shfl_xor(blo, o, 64)); bhi = max(bhi, __shfl_xor(bhi, o, 64));
    }
    if ((tid & 63u) == 0u) {
        int *r = s_red[tid >> 6];
        r[0] = lo0; r[1] = lo1; r[2] = lo2; r[3] = hi0; r[4] = hi1; r[5] = hi2;
        r[6] = blo; r[7] = bhi;
    }
    __syncthreads();
    for (int w = 0; w < PM_THREADS / 64; ++w) {
        const int *r = s_red[w];
        lo0 = min(lo0, r[0]); lo1 = min(lo1, r[1]); lo2 = min(lo2, r[2]);
        hi0 = max(hi0, r[3]); hi1 = max(hi1, r[4]); hi2 = max(hi2, r[5]);
        blo = min(blo, r[6]); bhi = max(bhi, r[7]);
    }
}

// LDS-binned deposit.  A workgroup takes `chunk` consecutive particles (in key order they
// fill a compact region) in pieces: a piece finds the box of mesh points its clouds touch
// (unwrapped indices, so a region across the periodic boundary stays compact) and, when it
// holds at most DEP_TILE points and the particles share one box of a batch, sums their
// contributions into an LDS tile with 64-bit LDS atomics, then adds each non-zero tile point
// to the mesh (wrapped) with one global atomic.  A piece whose box is too large is halved (a
// sparse region) down to PM_PIECE_MIN particles, below which it adds directly.  The mesh is
// the same integer sum either way.
// The coordinates (a, b, e) of tile point c = (a tey + b) tez + e, advanced by a fixed stride
// with carries instead of two integer divisions per point.
struct tile_walk {
    uint32_t a, b, e, da, db, de, tey, tez;
    __device__ __forceinline__ tile_walk(uint32_t c0, uint32_t stride, uint32_t tey_,
                                         uint32_t tez_)
        : tey(tey_), tez(tez_) {
        const uint32_t pyz = tey * tez;
        a = c0 / pyz;
        const uint32_t r = c0 - a * pyz;
        b = r / tez;
        e = r - b * tez;
        da = stride / pyz;
        const uint32_t q = stride - da * pyz;
        db = q / tez;
        de = q - db * tez;
    }
    __device__ __forceinline__ void next() {
        e += de;
        b += db;
        a += da;
        if (e >= tez) {
            e -= tez;
            ++b;
        }
        if (b >= tey) {
            b -= tey;
            ++a;
        }
    }
};

__global__ __launch_bounds__(PM_THREADS) void k_pm_deposit_tiled(
    uint64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const uint32_t *__restrict__ mult, double delta, int ng,
    unsigned long long *__restrict__ q, pm_batch B, uint32_t chunk) {
    __shared__ unsigned long long s_tile[DEP_TILE];
    __shared__ int s_red[PM_THREADS / 64][8];
    const uint64_t c0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t c1 = c0 + chunk < n ? c0 + chunk : n;
    const uint32_t tid = threadIdx.x;
    uint64_t p0 = c0;
    uint32_t piece = chunk;
    while (p0 < c1) {
        const uint64_t p1 = p0 + piece < c1 ? p0 + piece : c1;
        int lo0, lo1, lo2, hi0, hi1, hi2, blo, bhi;
        chunk_bounds(p0, p1, x, y, z, delta, B, s_red, lo0, lo1, lo2, hi0, hi1, hi2, blo, bhi);
        // points spanned per axis (base .. base + 1); every thread holds the same values, so
        // the choices below are uniform over the workgroup
        const int64_t ex = (int64_t)hi0 - lo0 + 2, ey = (int64_t)hi1 - lo1 + 2,
                      ez = (int64_t)hi2 - lo2 + 2;
        const bool fits = (!B.boxes || blo == bhi) && ex <= DEP_TILE && ey <= DEP_TILE &&
                          ez <= DEP_TILE && ex * ey * ez <= DEP_TILE;
        __syncthreads();   // s_red is read by every thread before the next piece writes it
        if (!fits && piece > PM_PIECE_MIN) {
            piece >>= 1;
            continue;
        }
        if (!fits) {
            for (uint64_t p = p0 + tid; p < p1; p += PM_THREADS) {
                double d = delta;
                int g = ng;
                unsigned long long *qq = q;
                if (B.boxes) {
                    const dzs_bbox &bx = B.boxes[B.key[p] >> DZS_BATCH_SHIFT];
                    d = bx.delta;
                    g = bx.ng;
                    qq = q + bx.mesh_off;
                }
                dep_direct(x, y, z, mult, p, d, g, qq);
            }
            p0 = p1;
            continue;
        }
        double dl = delta;
        int gn = ng;
        unsigned long long *qb = q;
        if (B.boxes) {
            const dzs_bbox &bx = B.boxes[blo];
            dl = bx.delta;
            gn = bx.ng;
            qb = q + bx.mesh_off;
        }
        const uint32_t tey = (uint32_t)ey, tez = (uint32_t)ez;
        const uint32_t cells = (uint32_t)(ex * ey * ez);
        for (uint32_t c = tid; c < cells; c += PM_THREADS)
            s_tile[c] = 0ull;
        __syncthreads();
        for (uint64_t p = p0 + tid; p < p1; p += PM_THREADS) {
            double wx[2], wy[2], wz[2];
            const uint32_t i = (uint32_t)(cic_base(x[p], dl, wx[0], wx[1]) - lo0);
            const uint32_t j = (uint32_t)(cic_base(y[p], dl, wy[0], wy[1]) - lo1);
            const uint32_t k = (uint32_t)(cic_base(z[p], dl, wz[0], wz[1]) - lo2);
            const double m = (double)mult[p] * DEP_FRAC;
#pragma unroll
            for (uint32_t a = 0; a < 2; ++a)
#pragma unroll
                for (uint32_t b = 0; b < 2; ++b)
#pragma unroll
                    for (uint32_t c = 0; c < 2; ++c) {
                        const unsigned long long iv = dep_fixed(m, wx[a], wy[b], wz[c]);
                        if (iv)
                            atomicAdd(&s_tile[((i + a) * tey + (j + b)) * tez + (k + c)], iv);
                    }
        }
        __syncthreads();
        tile_walk w(tid, PM_THREADS, tey, tez);
        for (uint32_t c = tid; c < cells; c += PM_THREADS, w.next()) {
            const unsigned long long v = s_tile[c];
            if (!v)
                continue;
            const int ix = wrap_near(lo0 + (int)w.a, gn), iy = wrap_near(lo1 + (int)w.b, gn),
                      iz = wrap_near(lo2 + (int)w.e, gn);
            atomicAdd(&qb[((uint64_t)ix * gn + iy) * gn + iz], v);
        }
        __syncthreads();   // the tile is read before the next piece clears it
        p0 = p1;
    }
}

// ---------------------------------------------------------------------------------------
// x passes, real <-> half spectrum.  The density and the potential are real, so only the
// planes k_x = 0 .. N_g/2 of the transform are kept (the others are their conjugates): the
// y and z passes run on N_g/2 + 1 planes.  A tile is 2 CL consecutive iz values for a fixed
// iy; lines iz0 + t and iz0 + t + CL travel as the real and imaginary parts of one complex
// line of length N_g, and their spectra are separated (forward) or combined (inverse) with
// the conjugate symmetry of a real line's transform.  The complex mesh keeps the layout
// (k_x N_g + iy) N_g + iz.
// ---------------------------------------------------------------------------------------
template <typename C>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_x_r2c(const unsigned long long *q, C *c,
                                                           const double2 *__restrict__ tw,
                                                           fft_plan P, int CL, double q_scale,
                                                           pm_batch B) {
    // q and c may be the same memory (meshes for the precision form only): the tile writes
    // only cells it has read, after all of its loads
    typedef decltype(C::x) Rt;
    __shared__ C s_buf[FFT_ELEMS];
    __shared__ C s_tw[1024];
    const int n = P.n;
    const int TZ = 2 * CL;
    const int tiles_z = n / TZ;
    uint32_t blk = blockIdx.x;
    if (B.boxes) {
        const dzs_bbox &bx = B.boxes[B.members[blk / (uint32_t)B.blocks_per_mesh]];
        blk %= (uint32_t)B.blocks_per_mesh;
        q += bx.mesh_off;
        c += bx.mesh_off;
        q_scale = bx.q_scale;
    }
    const int iy = blk / tiles_z;
    const int iz0 = (blk % tiles_z) * TZ;
    const uint64_t sx = (uint64_t)n * n;
    const uint64_t base = (uint64_t)iy * n + iz0;
    load_twiddles(s_tw, tw, n);
    for (int e = threadIdx.x; e < n * CL; e += FFT_THREADS) {
        const int t = e % CL, a = e / CL;
        const uint64_t gi = base + (uint64_t)a * sx + t;
        s_buf[a * CL + t] = C{Rt((double)(long long)q[gi] * q_scale),
                              Rt((double)(long long)q[gi + CL] * q_scale)};
    }
    __syncthreads();
    fft_lines<false>(s_buf, s_tw, P, CL, CL, 1);
    // Z = A + i B with A, B the spectra of the two real lines: A[k] = (Z[k] + conj Z[n-k]) / 2,
    // B[k] = (Z[k] - conj Z[n-k]) / 2i
    const int nh = n / 2 + 1;
    for (int e = threadIdx.x; e < nh * CL; e += FFT_THREADS) {
        const int t = e % CL, k = e / CL;
        const C z = s_buf[k * CL + t];
        const C w = s_buf[(k == 0 ? 0 : n - k) * CL + t];
        const uint64_t gi = base + (uint64_t)k * sx + t;
        c[gi] = C{Rt(0.5) * (z.x + w.x), Rt(0.5) * (z.y - w.y)};
        c[gi + CL] = C{Rt(0.5) * (z.y + w.y), Rt(-0.5) * (z.x - w.x)};
    }
}

template <typename C>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_x_c2r(const C *__restrict__ c,
                                                           decltype(C::x) *__restrict__ phi,
                                                           const double2 *__restrict__ tw,
                                                           fft_plan P, int CL, pm_batch B) {
    typedef decltype(C::x) Rt;
    __shared__ C s_buf[FFT_ELEMS];
    __shared__ C s_tw[1024];
    const int n = P.n;
    const int TZ = 2 * CL;
    const int tiles_z = n / TZ;
    uint32_t blk = blockIdx.x;
    if (B.boxes) {
        const dzs_bbox &bx = B.boxes[B.members[blk / (uint32_t)B.blocks_per_mesh]];
        blk %= (uint32_t)B.blocks_per_mesh;
        c += bx.mesh_off;
        phi += bx.mesh_off;
    }
    const int iy = blk / tiles_z;
    const int iz0 = (blk % tiles_z) * TZ;
    const uint64_t sx = (uint64_t)n * n;
    const uint64_t base = (uint64_t)iy * n + iz0;
    load_twiddles(s_tw, tw, n);
    // Z[k] = A[k] + i B[k], Z[n-k] = conj A[k] + i conj B[k]; the k_x = 0 and N_g/2 values of
    // a real line's spectrum are real (their imaginary rounding is dropped, as the real part
    // of a full inverse transform drops it)
    const int nh = n / 2 + 1;
    for (int e = threadIdx.x; e < nh * CL; e += FFT_THREADS) {
        const int t = e % CL, k = e / CL;
        const uint64_t gi = base + (uint64_t)k * sx + t;
        C a = c[gi], b = c[gi + CL];
        const bool edge = k == 0 || 2 * k == n;
        if (edge)
            a.y = b.y = Rt(0.0);
        s_buf[k * CL + t] = C{a.x - b.y, a.y + b.x};
        if (!edge)
            s_buf[(n - k) * CL + t] = C{a.x + b.y, b.x - a.y};
    }
    __syncthreads();
    fft_lines<true>(s_buf, s_tw, P, CL, CL, 1);
    for (int e = threadIdx.x; e < n * CL; e += FFT_THREADS) {
        const int t = e % CL, a = e / CL;
        const uint64_t gi = base + (uint64_t)a * sx + t;
        const C z = s_buf[a * CL + t];
        phi[gi] = z.x;
        phi[gi + CL] = z.y;
    }
}

// ---------------------------------------------------------------------------------------
// y passes: a tile is TZ consecutive iz values x all N_g values of iy, for a fixed k_x plane.
// ---------------------------------------------------------------------------------------
template <bool INV, typename C>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_y(C *__restrict__ c,
                                                       const double2 *__restrict__ tw,
                                                       fft_plan P, int TZ, pm_batch B) {
    __shared__ C s_buf[FFT_ELEMS];
    __shared__ C s_tw[1024];
    const int n = P.n;
    const int tiles_z = n / TZ;
    uint32_t blk = blockIdx.x;
    if (B.boxes) {
        const dzs_bbox &bx = B.boxes[B.members[blk / (uint32_t)B.blocks_per_mesh]];
        blk %= (uint32_t)B.blocks_per_mesh;
        c += bx.mesh_off;
    }
    const int ix = blk / tiles_z;
    const int iz0 = (blk % tiles_z) * TZ;
    const uint64_t base = (uint64_t)ix * n * n + iz0;
    load_twiddles(s_tw, tw, n);
    const int total = n * TZ;
    for (int e = threadIdx.x; e < total; e += FFT_THREADS) {
        const int t = e % TZ, a = e / TZ;
        s_buf[a * TZ + t] = c[base + (uint64_t)a * n + t];
    }
    __syncthreads();
    fft_lines<INV>(s_buf, s_tw, P, TZ, TZ, 1);
    for (int e = threadIdx.x; e < total; e += FFT_THREADS) {
        const int t = e % TZ, a = e / TZ;
        c[base + (uint64_t)a * n + t] = s_buf[a * TZ + t];
    }
}

// z pass: TL whole contiguous lines (fixed k_x plane, consecutive iy): forward FFT, Green's
// function, inverse FFT.
template <typename C>
__global__ __launch_bounds__(FFT_THREADS) void k_fft_z_green(C *__restrict__ c,
                                                              const double2 *__restrict__ tw,
                                                              const double *__restrict__ gt,
                                                              const double *__restrict__ k2t,
                                                              fft_plan P, int TL, double gconst,
                                                              pm_batch B) {
    typedef decltype(C::x) Rt;
    __shared__ C s_buf[FFT_ELEMS];
    __shared__ C s_tw[1024];
    const int n = P.n;
    const int tiles_y = n / TL;
    uint32_t blk = blockIdx.x;
    if (B.boxes) {
        const dzs_bbox &bx = B.boxes[B.members[blk / (uint32_t)B.blocks_per_mesh]];
        blk %= (uint32_t)B.blocks_per_mesh;
        c += bx.mesh_off;
        gt += bx.tab_off;
        k2t += bx.tab_off + (uint64_t)n;
    }
    const int ix = blk / tiles_y;
    const int iy0 = (blk % tiles_y) * TL;
    const uint64_t base = ((uint64_t)ix * n + iy0) * n;
    load_twiddles(s_tw, tw, n);
    const int total = n * TL;
    for (int e = threadIdx.x; e < total; e += FFT_THREADS)
        s_buf[e] = c[base + e];
    __syncthreads();
    fft_lines<false>(s_buf, s_tw, P, TL, 1, n);
    for (int e = threadIdx.x; e < total; e += FFT_THREADS) {
        const int iz = e % n, l = e / n;
        const int iy = iy0 + l;
        const double k2 = k2t[ix] + k2t[iy] + k2t[iz];
        double gk = 0.0;
        if (k2 > 0.0)
            gk = gconst * gt[ix] * gt[iy] * gt[iz] / k2;
        const Rt g = Rt(gk);
        C v = s_buf[e];
        s_buf[e] = C{v.x * g, v.y * g};
    }
    __syncthreads();
    fft_lines<true>(s_buf, s_tw, P, TL, 1, n);
    for (int e = threadIdx.x; e < total; e += FFT_THREADS)
        c[base + e] = s_buf[e];
}

// ---------------------------------------------------------------------------------------
// gradient + interpolation
// ---------------------------------------------------------------------------------------
// The 4-point difference of the potential at the 8 cloud-in-cell points of one particle,
// weighted with the cloud-in-cell weights.  at(a, b, c) returns the potential at index offsets
// from the particle's base point (a, b, c in [-2, 3]); both paths below run this same
// arithmetic, so they give the same bits.
template <typename Rt, typename At>
__device__ __forceinline__ void cic_gradient(const At &at, const double *wx, const double *wy,
                                             const double *wz, Rt &sx, Rt &sy, Rt &sz) {
    const Rt c1 = Rt(2.0 / 3.0), c2 = Rt(1.0 / 12.0);
    sx = sy = sz = Rt(0.0);
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) {
                const Rt w = Rt(wx[a] * wy[b] * wz[c]);
                const Rt dxp = c1 * (at(a + 1, b, c) - at(a - 1, b, c)) -
                               c2 * (at(a + 2, b, c) - at(a - 2, b, c));
                const Rt dyp = c1 * (at(a, b + 1, c) - at(a, b - 1, c)) -
                               c2 * (at(a, b + 2, c) - at(a, b - 2, c));
                const Rt dzp = c1 * (at(a, b, c + 1) - at(a, b, c - 1)) -
                               c2 * (at(a, b, c + 2) - at(a, b, c - 2));
                sx += w * dxp;
                sy += w * dyp;
                sz += w * dzp;
            }
}

template <typename Rt>
__device__ __forceinline__ void interp_store(uint64_t p, double delta, Rt sx, Rt sy, Rt sz,
                                             double *__restrict__ gx, double *__restrict__ gy,
                                             double *__restrict__ gz, int accumulate) {
    const double s = -1.0 / delta;
    if (accumulate) {
        gx[p] += s * (double)sx;
        gy[p] += s * (double)sy;
        gz[p] += s * (double)sz;
    } else {
        gx[p] = s * (double)sx;
        gy[p] = s * (double)sy;
        gz[p] = s * (double)sz;
    }
}

// Direct: the potential read from the mesh (wrapped indices).
template <typename Rt>
__device__ __forceinline__ void interp_direct(const double *__restrict__ x,
                                              const double *__restrict__ y,
                                              const double *__restrict__ z,
                                              const Rt *__restrict__ phi, uint64_t p, double delta,
                                              int ng, double *__restrict__ gx,
                                              double *__restrict__ gy, double *__restrict__ gz,
                                              int accumulate) {
    double wx[2], wy[2], wz[2];
    const int i = wrap_index(cic_base(x[p], delta, wx[0], wx[1]), ng);
    const int j = wrap_index(cic_base(y[p], delta, wy[0], wy[1]), ng);
    const int k = wrap_index(cic_base(z[p], delta, wz[0], wz[1]), ng);
    const uint64_t N = (uint64_t)ng;
    auto at = [&](int a, int b, int c) -> Rt {
        return phi[((uint64_t)wrap_near(i + a, ng) * N + wrap_near(j + b, ng)) * N +
                   wrap_near(k + c, ng)];
    };
    Rt sx, sy, sz;
    cic_gradient<Rt>(at, wx, wy, wz, sx, sy, sz);
    interp_store<Rt>(p, delta, sx, sy, sz, gx, gy, gz, accumulate);
}

template <typename Rt>
__global__ __launch_bounds__(PM_THREADS) void k_pm_interp(
    uint64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const Rt *__restrict__ phi, double delta, int ng,
    double *__restrict__ gx, double *__restrict__ gy, double *__restrict__ gz, int accumulate,
    pm_batch B) {
    uint64_t p = (uint64_t)blockIdx.x * PM_THREADS + threadIdx.x;
    if (p >= n)
        return;
    if (B.boxes) {
        const dzs_bbox &bx = B.boxes[B.key[p] >> DZS_BATCH_SHIFT];
        delta = bx.delta;
        ng = bx.ng;
        phi += bx.mesh_off;
    }
    interp_direct<Rt>(x, y, z, phi, p, delta, ng, gx, gy, gz, accumulate);
}

// LDS-staged: a workgroup takes `chunk` consecutive particles in pieces; a piece loads once
// the block of potential values its stencils read (base - 2 .. base + 3 on each axis,
// wrapped) into a 32 KB LDS tile when they fit and the piece lies in one box of a batch, and
// evaluates every particle from LDS.  A piece whose block is too large is halved down to
// PM_PIECE_MIN particles, below which each particle reads the mesh directly (the same values
// and arithmetic: the result does not depend on the path).
template <typename Rt>
__global__ __launch_bounds__(PM_THREADS) void k_pm_interp_tiled(
    uint64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const Rt *__restrict__ phi, double delta, int ng,
    double *__restrict__ gx, double *__restrict__ gy, double *__restrict__ gz, int accumulate,
    pm_batch B, uint32_t chunk) {
    constexpr uint32_t TILE = INTERP_TILE_BYTES / sizeof(Rt);
    __shared__ Rt s_phi[TILE];
    __shared__ int s_red[PM_THREADS / 64][8];
    const uint64_t c0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t c1 = c0 + chunk < n ? c0 + chunk : n;
    const uint32_t tid = threadIdx.x;
    uint64_t p0 = c0;
    uint32_t piece = chunk;
    while (p0 < c1) {
        const uint64_t p1 = p0 + piece < c1 ? p0 + piece : c1;
        int lo0, lo1, lo2, hi0, hi1, hi2, blo, bhi;
        chunk_bounds(p0, p1, x, y, z, delta, B, s_red, lo0, lo1, lo2, hi0, hi1, hi2, blo, bhi);
        const int64_t ex = (int64_t)hi0 - lo0 + 6, ey = (int64_t)hi1 - lo1 + 6,
                      ez = (int64_t)hi2 - lo2 + 6;
        const bool fits = (!B.boxes || blo == bhi) && ex <= TILE && ey <= TILE && ez <= TILE &&
                          ex * ey * ez <= TILE;
        __syncthreads();   // s_red is read by every thread before the next piece writes it
        if (!fits && piece > PM_PIECE_MIN) {
            piece >>= 1;
            continue;
        }
        if (!fits) {
            for (uint64_t p = p0 + tid; p < p1; p += PM_THREADS) {
                double d = delta;
                int g = ng;
                const Rt *ph = phi;
                if (B.boxes) {
                    const dzs_bbox &bx = B.boxes[B.key[p] >> DZS_BATCH_SHIFT];
                    d = bx.delta;
                    g = bx.ng;
                    ph = phi + bx.mesh_off;
                }
                interp_direct<Rt>(x, y, z, ph, p, d, g, gx, gy, gz, accumulate);
            }
            p0 = p1;
            continue;
        }
        double dl = delta;
        int gn = ng;
        const Rt *pb = phi;
        if (B.boxes) {
            const dzs_bbox &bx = B.boxes[blo];
            dl = bx.delta;
            gn = bx.ng;
            pb = phi + bx.mesh_off;
        }
        const uint32_t tey = (uint32_t)ey, tez = (uint32_t)ez;
        const uint32_t cells = (uint32_t)(ex * ey * ez);
        const uint64_t N = (uint64_t)gn;
        tile_walk w(tid, PM_THREADS, tey, tez);
        for (uint32_t c = tid; c < cells; c += PM_THREADS, w.next()) {
            const int ix = wrap_near(lo0 - 2 + (int)w.a, gn),
                      iy = wrap_near(lo1 - 2 + (int)w.b, gn),
                      iz = wrap_near(lo2 - 2 + (int)w.e, gn);
            s_phi[c] = pb[((uint64_t)ix * N + iy) * N + iz];
        }
        __syncthreads();
        for (uint64_t p = p0 + tid; p < p1; p += PM_THREADS) {
            double wx[2], wy[2], wz[2];
            // tile coordinates of the base point (the tile starts at lo - 2)
            const int i = cic_base(x[p], dl, wx[0], wx[1]) - lo0 + 2;
            const int j = cic_base(y[p], dl, wy[0], wy[1]) - lo1 + 2;
            const int k = cic_base(z[p], dl, wz[0], wz[1]) - lo2 + 2;
            auto at = [&](int a, int b, int c) -> Rt {
                return s_phi[((uint32_t)(i + a) * tey + (uint32_t)(j + b)) * tez +
                             (uint32_t)(k + c)];
            };
            Rt sx, sy, sz;
            cic_gradient<Rt>(at, wx, wy, wz, sx, sy, sz);
            interp_store<Rt>(p, dl, sx, sy, sz, gx, gy, gz, accumulate);
        }
        __syncthreads();   // the tile is read before the next piece loads it
        p0 = p1;
    }
}

// ---------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------
static bool make_plan(int n, fft_plan *P) {
    P->n = n;
    P->n_stages = 0;
    int m = n;
    while (m % 4 == 0 && P->n_stages < FFT_MAX_STAGES) {
        P->radix[P->n_stages++] = 4;
        m /= 4;
    }
    while (m % 2 == 0 && P->n_stages < FFT_MAX_STAGES) {
        P->radix[P->n_stages++] = 2;
        m /= 2;
    }
    while (m % 3 == 0 && P->n_stages < FFT_MAX_STAGES) {
        P->radix[P->n_stages++] = 3;
        m /= 3;
    }
    return m == 1;
}

// largest power of two t <= cap with t * ng <= FFT_ELEMS and t dividing ng
static int tile_lines(int ng, int cap) {
    int t = 1;
    while (2 * t <= cap && 2 * t * ng <= FFT_ELEMS && ng % (2 * t) == 0)
        t *= 2;
    return t;
}

// complex lines per x tile: each carries two real lines, so 2 CL must divide N_g
static int pair_lines(int ng) {
    int t = 1;
    while (2 * t <= 16 && 2 * t * ng <= FFT_ELEMS && ng % (4 * t) == 0)
        t *= 2;
    return t;
}

// even 2^a 3^b sides (the x passes pair real lines and keep N_g/2 + 1 planes)
bool dzs_pm_mesh_ok(int ng) {
    fft_plan P;
    return ng >= 8 && ng <= 1024 && ng % 2 == 0 && make_plan(ng, &P);
}

// tables at ctx->pm_tables: [0, 2n) twiddles (double2), [2n, 3n) gt, [3n, 4n) k^2
static dzs_status upload_tables(dzs_ctx *ctx, int ng, double L, double r_s, hipStream_t s) {
    // staged in the context's host table when it has one (the allocation-free entry point),
    // else in a temporary
    std::vector<double> tmp(ctx->pm_host_tab ? 0 : 4 * (size_t)ng);
    double *h = ctx->pm_host_tab ? ctx->pm_host_tab : tmp.data();
    const long double pi = 3.14159265358979323846264338327950288L;
    for (int m = 0; m < ng; ++m) {
        long double ang = -2.0L * pi * m / ng;
        h[2 * m] = (double)cosl(ang);
        h[2 * m + 1] = (double)sinl(ang);
    }
    const double delta = L / ng;
    for (int m = 0; m < ng; ++m) {
        const int nn = m < ng / 2 ? m : m - ng;  // frequency index in [-ng/2, ng/2)
        const long double k = 2.0L * pi * nn / L;
        long double hh = 0.5L * k * delta;
        long double sinc = hh == 0.0L ? 1.0L : sinl(hh) / hh;
        long double w2 = sinc * sinc * sinc * sinc;  // W^2 per axis: sinc^4
        h[2 * ng + m] = (double)(expl(-k * k * (long double)r_s * r_s) / w2);
        h[3 * ng + m] = (double)(k * k);
    }
    DZS_HIP(ctx, hipMemcpyAsync(ctx->pm_tables, h, sizeof(double) * 4 * (size_t)ng,
                                hipMemcpyHostToDevice, s));
    DZS_HIP(ctx, hipStreamSynchronize(s));
    return DZS_OK;
}

// The Poisson solve (x, y passes forward, z pass with the Green's function, y, x passes
// inverse) over n_meshes meshes of side P.n, in the complex type C of the form.
template <typename C>
static dzs_status pm_solve(dzs_ctx *ctx, const fft_plan &P, const double2 *tw, const double *gt,
                           const double *k2t, double q_scale, double gconst, uint32_t n_meshes,
                           pm_batch B, hipStream_t s) {
    typedef decltype(C::x) Rt;
    const int ng = P.n;
    const int nkx = ng / 2 + 1;                  // k_x planes kept
    const int CL = pair_lines(ng);               // complex lines per x tile (2 CL real lines)
    const int TZ = tile_lines(ng, 16);           // lines per y tile
    const int TL = tile_lines(ng, FFT_ELEMS);    // lines per z tile
    const uint32_t x_per = (uint32_t)((uint64_t)ng * (ng / (2 * CL)));
    const uint32_t y_per = (uint32_t)((uint64_t)nkx * (ng / TZ));
    const uint32_t z_per = (uint32_t)((uint64_t)nkx * (ng / TL));
    const unsigned long long *mq = (const unsigned long long *)ctx->mesh_q;
    C *mc = (C *)ctx->mesh_c;
    Rt *phi = (Rt *)ctx->mesh_phi;
    pm_batch Bx = B, By = B, Bz = B;
    Bx.blocks_per_mesh = (int)x_per;
    By.blocks_per_mesh = (int)y_per;
    Bz.blocks_per_mesh = (int)z_per;
    const dim3 gx(x_per * n_meshes), gy(y_per * n_meshes), gz(z_per * n_meshes);
    {
        dzs_timed t(ctx, KC_PM_FFT_X, s);
        hipLaunchKernelGGL(k_fft_x_r2c<C>, gx, dim3(FFT_THREADS), 0, s, mq, mc, tw, P, CL,
                           q_scale, Bx);
        DZS_TRY(dzs_check_launch(ctx, "fft_x_fwd"));
    }
    {
        dzs_timed t(ctx, KC_PM_FFT_Y, s);
        hipLaunchKernelGGL((k_fft_y<false, C>), gy, dim3(FFT_THREADS), 0, s, mc, tw, P, TZ, By);
        DZS_TRY(dzs_check_launch(ctx, "fft_y_fwd"));
    }
    {
        dzs_timed t(ctx, KC_PM_FFT_Z_GREEN, s);
        hipLaunchKernelGGL(k_fft_z_green<C>, gz, dim3(FFT_THREADS), 0, s, mc, tw, gt, k2t, P, TL,
                           gconst, Bz);
        DZS_TRY(dzs_check_launch(ctx, "fft_z_green"));
    }
    {
        dzs_timed t(ctx, KC_PM_FFT_Y, s);
        hipLaunchKernelGGL((k_fft_y<true, C>), gy, dim3(FFT_THREADS), 0, s, mc, tw, P, TZ, By);
        DZS_TRY(dzs_check_launch(ctx, "fft_y_inv"));
    }
    {
        dzs_timed t(ctx, KC_PM_FFT_X, s);
        hipLaunchKernelGGL(k_fft_x_c2r<C>, gx, dim3(FFT_THREADS), 0, s, mc, phi, tw, P, CL, Bx);
        DZS_TRY(dzs_check_launch(ctx, "fft_x_inv"));
    }
    return DZS_OK;
}

// Tiles only when the particles are at least half as many as the mesh points: on a finer
// mesh a chunk's stencils rarely fit the tile and the direct reads are faster.
template <typename Rt>
static dzs_status pm_interp(dzs_ctx *ctx, const dzs_particles *p, int accumulate, double delta,
                            int ng, pm_batch B, int32_t chunk, uint64_t cells, hipStream_t s) {
    if (p->n == 0)
        return DZS_OK;
    dzs_timed t(ctx, KC_PM_INTERP, s);
    if (chunk == 0)
        chunk = DZS_PM_CHUNK_DEFAULT;
    if (2 * p->n < cells)
        chunk = -1;
    if (chunk < 0) {
        hipLaunchKernelGGL(k_pm_interp<Rt>, dim3(blocks_for(p->n, PM_THREADS)), dim3(PM_THREADS),
                           0, s, p->n, (const double *)p->x, (const double *)p->y,
                           (const double *)p->z, (const Rt *)ctx->mesh_phi, delta, ng, p->gx,
                           p->gy, p->gz, accumulate, B);
    } else {
        hipLaunchKernelGGL(k_pm_interp_tiled<Rt>, dim3(blocks_for(p->n, (uint32_t)chunk)),
                           dim3(PM_THREADS), 0, s, p->n, (const double *)p->x,
                           (const double *)p->y, (const double *)p->z, (const Rt *)ctx->mesh_phi,
                           delta, ng, p->gx, p->gy, p->gz, accumulate, B, (uint32_t)chunk);
    }
    return dzs_check_launch(ctx, "pm_interp");
}

// zero fill by a kernel (a memset node in a captured graph is avoided)
__global__ __launch_bounds__(PM_THREADS) void k_zero_u64(uint64_t n, unsigned long long *a) {
    for (uint64_t i = (uint64_t)blockIdx.x * PM_THREADS + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * PM_THREADS)
        a[i] = 0ull;
}

// chunk: particles per LDS tile (a power of two in [DZS_PM_CHUNK_MIN, _MAX]), 0 for the
// default, -1 for the direct deposit.
static dzs_status pm_deposit(dzs_ctx *ctx, const dzs_particles *p, uint64_t cells, double delta,
                             int ng, pm_batch B, int32_t chunk, hipStream_t s) {
    dzs_timed t(ctx, KC_PM_DEPOSIT, s);
    const uint64_t zb = (cells + PM_THREADS - 1) / PM_THREADS;
    hipLaunchKernelGGL(k_zero_u64, dim3((uint32_t)(zb < 65536 ? zb : 65536)), dim3(PM_THREADS), 0,
                       s, cells, (unsigned long long *)ctx->mesh_q);
    DZS_TRY(dzs_check_launch(ctx, "mesh_clear"));
    if (p->n == 0)
        return DZS_OK;
    if (chunk == 0)
        chunk = DZS_PM_CHUNK_DEFAULT;
    if (chunk < 0) {
        hipLaunchKernelGGL(k_pm_deposit, dim3(blocks_for(p->n, PM_THREADS)), dim3(PM_THREADS), 0, s,
                           p->n, (const double *)p->x, (const double *)p->y, (const double *)p->z,
                           (const uint32_t *)p->mult, delta, ng, (unsigned long long *)ctx->mesh_q,
                           B);
    } else {
        hipLaunchKernelGGL(k_pm_deposit_tiled, dim3(blocks_for(p->n, (uint32_t)chunk)),
                           dim3(PM_THREADS), 0, s, p->n, (const double *)p->x,
                           (const double *)p->y, (const double *)p->z, (const uint32_t *)p->mult,
                           delta, ng, (unsigned long long *)ctx->mesh_q, B, (uint32_t)chunk);
    }
    return dzs_check_launch(ctx, "pm_deposit");
}

// The potential on the mesh (deposit, forward FFT, Green's function, inverse FFT).
dzs_status dzs_pm_solve(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                        const dzs_pm_params *prm, hipStream_t s) {
    const int ng = prm->ng;
    fft_plan P;
    if (!dzs_pm_mesh_ok(ng) || !make_plan(ng, &P))
        return dzs_fail(ctx, DZS_EINVAL, "pm_force: mesh side %d is not an even 2^a 3^b", ng);
    const uint64_t ng3 = (uint64_t)ng * ng * ng;
    const double delta = box->L / ng;
    if (ctx->pm_tab_ng != ng || ctx->pm_tab_L != box->L || ctx->pm_tab_rs != prm->r_s) {
        DZS_TRY(upload_tables(ctx, ng, box->L, prm->r_s, s));
        ctx->pm_tab_ng = ng;
        ctx->pm_tab_L = box->L;
        ctx->pm_tab_rs = prm->r_s;
    }
    const double2 *tw = (const double2 *)ctx->pm_tables;
    const double *gt = ctx->pm_tables + 2 * ng;
    const double *k2t = ctx->pm_tables + 3 * ng;
    const pm_batch none{nullptr, nullptr, 0, nullptr};
    DZS_TRY(pm_deposit(ctx, p, ng3, delta, ng, none, prm->tile_chunk, s));
    const double q_scale = box->m0 / (DEP_FRAC * delta * delta * delta);
    const double gconst = -4.0 * 3.14159265358979323846 * box->G / (double)ng3;
    if (prm->precision == DZS_FP32)
        return pm_solve<float2>(ctx, P, tw, gt, k2t, q_scale, gconst, 1, none, s);
    return pm_solve<double2>(ctx, P, tw, gt, k2t, q_scale, gconst, 1, none, s);
}

// The long-range force at the particles from the potential dzs_pm_solve left on the mesh
// (same box, particles and parameters).
dzs_status dzs_pm_apply(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                        const dzs_pm_params *prm, hipStream_t s) {
    const int ng = prm->ng;
    const uint64_t ng3 = (uint64_t)ng * ng * ng;
    const double delta = box->L / ng;
    const pm_batch none{nullptr, nullptr, 0, nullptr};
    if (prm->precision == DZS_FP32)
        return pm_interp<float>(ctx, p, prm->accumulate, delta, ng, none, prm->tile_chunk, ng3,
                                s);
    return pm_interp<double>(ctx, p, prm->accumulate, delta, ng, none, prm->tile_chunk, ng3, s);
}

dzs_status dzs_pm_run(dzs_ctx *ctx, const dzs_box *box, const dzs_particles *p,
                      const dzs_pm_params *prm, hipStream_t s) {
    DZS_TRY(dzs_pm_solve(ctx, box, p, prm, s));
    return dzs_pm_apply(ctx, box, p, prm, s);
}

// A batch: every box's mesh at its offset of the mesh arrays.  dzs_pm_batch_prepare fills
// each box's mesh offset, spacing, deposit scale and table offset in the host table hb[] and
// uploads the twiddle and Green's function tables of every box and mesh size; the caller
// uploads hb[] to the device table.  Boxes of one mesh size share each FFT launch.
dzs_status dzs_pm_batch_prepare(dzs_ctx *ctx, uint32_t nb, dzs_bbox *hb, hipStream_t s) {
    ctx->batch_sides.clear();
    uint64_t cells = 0;
    for (uint32_t b = 0; b < nb; ++b) {
        if (!dzs_pm_mesh_ok(hb[b].ng))
            return dzs_fail(ctx, DZS_EINVAL, "batch: box %u mesh side %d is not an even 2^a 3^b "
                            "in [8, 1024]", b, hb[b].ng);
        hb[b].mesh_off = cells;
        cells += (uint64_t)hb[b].ng * hb[b].ng * hb[b].ng;
        bool seen = false;
        for (int v : ctx->batch_sides)
            seen |= v == hb[b].ng;
        if (!seen)
            ctx->batch_sides.push_back(hb[b].ng);
    }
    const uint64_t cap_cells = (uint64_t)ctx->cap_ng * ctx->cap_ng * ctx->cap_ng;
    if (cells > cap_cells)
        return dzs_fail(ctx, DZS_ECAPACITY, "batch: meshes need %llu cells, the context holds %llu",
                        (unsigned long long)cells, (unsigned long long)cap_cells);
    ctx->batch_cells = cells;
    // tables: per box [Green factor (ng), k^2 (ng)], then per mesh side twiddles (2 ng)
    std::vector<double> tab;
    const long double pi = 3.14159265358979323846264338327950288L;
    for (uint32_t b = 0; b < nb; ++b) {
        const int ng = hb[b].ng;
        const double L = hb[b].L, delta = L / ng;
        hb[b].delta = delta;
        hb[b].q_scale = hb[b].m0 / (DEP_FRAC * delta * delta * delta);
        hb[b].tab_off = tab.size();
        tab.resize(tab.size() + 2 * (size_t)ng);
        double *gt = tab.data() + hb[b].tab_off, *k2 = gt + ng;
        for (int m = 0; m < ng; ++m) {
            const int nn = m < ng / 2 ? m : m - ng;
            const long double k = 2.0L * pi * nn / L;
            const long double hh = 0.5L * k * delta;
            const long double sinc = hh == 0.0L ? 1.0L : sinl(hh) / hh;
            const long double w2 = sinc * sinc * sinc * sinc;
            gt[m] = (double)(expl(-k * k * (long double)hb[b].r_s * hb[b].r_s) / w2);
            k2[m] = (double)(k * k);
        }
    }
    ctx->batch_tw_off.clear();
    ctx->batch_cls_first.clear();
    std::vector<uint32_t> members;
    for (int ng : ctx->batch_sides) {
        ctx->batch_tw_off.push_back(tab.size());
        tab.resize(tab.size() + 2 * (size_t)ng);
        for (int m = 0; m < ng; ++m) {
            const long double ang = -2.0L * pi * m / ng;
            tab[ctx->batch_tw_off.back() + 2 * m] = (double)cosl(ang);
            tab[ctx->batch_tw_off.back() + 2 * m + 1] = (double)sinl(ang);
        }
        ctx->batch_cls_first.push_back((uint32_t)members.size());
        for (uint32_t b = 0; b < nb; ++b)
            if (hb[b].ng == ng)
                members.push_back(b);
    }
    ctx->batch_cls_first.push_back((uint32_t)members.size());
    // per box 2 ng and per distinct side 2 ng doubles: within the 4 max_boxes max_mesh_side
    // the context holds
    if (tab.size() > ctx->batch_tab_cap)
        return dzs_fail(ctx, DZS_ECAPACITY, "batch: tables of %llu doubles exceed the context's "
                        "%llu", (unsigned long long)tab.size(),
                        (unsigned long long)ctx->batch_tab_cap);
    DZS_HIP(ctx, hipMemcpyAsync(ctx->batch_tab, tab.data(), sizeof(double) * tab.size(),
                                hipMemcpyHostToDevice, s));
    DZS_HIP(ctx, hipMemcpyAsync(ctx->batch_members, members.data(),
                                sizeof(uint32_t) * members.size(), hipMemcpyHostToDevice, s));
    // the staging vectors die here: wait for the copies
    DZS_HIP(ctx, hipStreamSynchronize(s));
    return DZS_OK;
}

// The long-range force of every box of a prepared batch into g (g = g_long); db is the device
// box table and ctx->key the sorted keys (box in the top digits) of the particles.
dzs_status dzs_pm_run_batch(dzs_ctx *ctx, const dzs_particles *p, int precision,
                            int32_t tile_chunk, const dzs_bbox *db, double G, hipStream_t s) {
    const pm_batch all{db, nullptr, 0, (const uint64_t *)ctx->key};
    DZS_TRY(pm_deposit(ctx, p, ctx->batch_cells, 0.0, 0, all, tile_chunk, s));
    for (size_t c = 0; c < ctx->batch_sides.size(); ++c) {
        const int ng = ctx->batch_sides[c];
        fft_plan P;
        make_plan(ng, &P);
        const uint32_t nm = ctx->batch_cls_first[c + 1] - ctx->batch_cls_first[c];
        const pm_batch B{db, ctx->batch_members + ctx->batch_cls_first[c], 0,
                         (const uint64_t *)ctx->key};
        const double2 *tw = (const double2 *)(ctx->batch_tab + ctx->batch_tw_off[c]);
        const double gconst = -4.0 * 3.14159265358979323846 * G / ((double)ng * ng * ng);
        if (precision == DZS_FP32)
            DZS_TRY(pm_solve<float2>(ctx, P, tw, ctx->batch_tab, ctx->batch_tab, 0.0, gconst, nm,
                                     B, s));
        else
            DZS_TRY(pm_solve<double2>(ctx, P, tw, ctx->batch_tab, ctx->batch_tab, 0.0, gconst, nm,
                                      B, s));
    }
    if (precision == DZS_FP32)
        return pm_interp<float>(ctx, p, 0, 0.0, 0, all, tile_chunk, ctx->batch_cells, s);
    return pm_interp<double>(ctx, p, 0, 0.0, 0, all, tile_chunk, ctx->batch_cells, s);
}
