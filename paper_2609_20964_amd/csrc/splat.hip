// Point-side kernels: binning, the 27-cell normal splat fused with the
// divergence (Warp-Geo Sec. 2.3, Eq. 22-26), its transpose (Sec. 2.5, Eq. 39)
// and the iso-value (Sec. 2.4) with its reverse.
//
// The normal field V (Eq. 23) is never stored: each point adds its share of
// b = -h^2 D_h V straight into b.  With face values F = (V_i + V_{i+1})/2 on
// interior faces and 0 on the outer faces, a point whose weights cover the
// 3x3x3 block around its cell touches the 81 cells of that block widened by
// one along each axis.  Points are binned into 8^3-cell tiles; a workgroup
// accumulates one tile's points in LDS and adds the window to b once.
#include <cmath>
#include <type_traits>

#include "kernels.h"

namespace wg {

namespace {

// Per-axis data of one point: central cell k, fractional offset f in [0,1),
// factors 1/2 (1 - |D|/2) of Eq. 25 for the offsets -1, 0, +1 (0 outside the
// grid) and their x-derivatives -sign(D)/(4h); in FP32 or (WG_FP64) FP64.
template <class T>
struct AxisW {
    int k;
    T f;
    T a[3];
    T da[3];
};

template <class T>
__device__ __forceinline__ bool bin_axis(float x, double lo, double h, int n, AxisW<T> &w, T inv4h) {
    double t = ((double)x - lo) / h;
    if (!(t >= 0.0 && t < (double)n)) return false;    // also rejects NaN
    int k = (int)floor(t);
    if (k >= n) return false;
    w.k = k;
    w.f = (T)(t - (double)k);
    for (int d = -1; d <= 1; ++d) {
        T D = w.f - T(0.5) - (T)d;
        bool in = (k + d >= 0) && (k + d < n);
        w.a[d + 1] = in ? T(0.5) * (T(1) - fabs(D) * T(0.5)) : T(0);
        T sg = D > T(0) ? T(1) : (D < T(0) ? T(-1) : T(0));
        w.da[d + 1] = in ? -sg * inv4h : T(0);
    }
    return true;
}

template <class T>
__device__ __forceinline__ T raw_w(const AxisW<T> &X, const AxisW<T> &Y, const AxisW<T> &Z, int dx, int dy, int dz) {
    if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1) return T(0);
    if (dx == 0 && dy == 0 && dz == 0) return T(0.5);
    return X.a[dx + 1] * Y.a[dy + 1] * Z.a[dz + 1];
}

__device__ __forceinline__ bool in_range(int k, int o, int n) { return k + o >= 0 && k + o < n; }

}  // namespace

// Contributions of one point to b: calls emit(cx, cy, cz, value) for every
// cell k + (cx, cy, cz) of the 81-cell support (|c| <= 2, at most one |c| = 2)
// inside the grid.  value = -(h/2) h^-3 / S * sum_xi n_xi (face terms).
// |value| <= 3.75 h^-2 max_k |n_k|: |h^-2 / (2 S)| <= h^-2 (S >= 1/2), and each
// face term pairs two raw weights summing to at most 0.625.
// AXES: the three axis terms separately, emit(cx, cy, cz, vx, vy, vz) (the
// exact-quadrature right-hand side filters each with the mass across its axis).
template <bool AXES = false, class T, class Emit>
__device__ __forceinline__ void point_divergence(const AxisW<T> &X, const AxisW<T> &Y, const AxisW<T> &Z, T n0, T n1,
                                                 T n2, const GridF &g, Emit &&emit) {
    const T Sx = X.a[0] + X.a[1] + X.a[2], Sy = Y.a[0] + Y.a[1] + Y.a[2], Sz = Z.a[0] + Z.a[1] + Z.a[2];
    const T S = Sx * Sy * Sz - X.a[1] * Y.a[1] * Z.a[1] + T(0.5);     // Eq. 24 normaliser
    const T coef = T(-0.5) * (T)g.h * (T)(1.0 / (g.h * g.h * g.h)) / S;
#pragma unroll
    for (int cz = -2; cz <= 2; ++cz)
#pragma unroll
        for (int cy = -2; cy <= 2; ++cy)
#pragma unroll
            for (int cx = -2; cx <= 2; ++cx) {
                if ((cx == -2 || cx == 2) + (cy == -2 || cy == 2) + (cz == -2 || cz == 2) > 1) continue;
                if (!in_range(X.k, cx, g.d.nx) || !in_range(Y.k, cy, g.d.ny) || !in_range(Z.k, cz, g.d.nz))
                    continue;
                const T r0 = raw_w(X, Y, Z, cx, cy, cz);
                // one sum (in this order) or one per axis
                T acc[3] = {T(0), T(0), T(0)};
                T &ax = acc[0], &ay = acc[AXES ? 1 : 0], &az = acc[AXES ? 2 : 0];
                if (in_range(X.k, cx + 1, g.d.nx)) ax += n0 * (r0 + raw_w(X, Y, Z, cx + 1, cy, cz));
                if (in_range(X.k, cx - 1, g.d.nx)) ax -= n0 * (raw_w(X, Y, Z, cx - 1, cy, cz) + r0);
                if (in_range(Y.k, cy + 1, g.d.ny)) ay += n1 * (r0 + raw_w(X, Y, Z, cx, cy + 1, cz));
                if (in_range(Y.k, cy - 1, g.d.ny)) ay -= n1 * (raw_w(X, Y, Z, cx, cy - 1, cz) + r0);
                if (in_range(Z.k, cz + 1, g.d.nz)) az += n2 * (r0 + raw_w(X, Y, Z, cx, cy, cz + 1));
                if (in_range(Z.k, cz - 1, g.d.nz)) az -= n2 * (raw_w(X, Y, Z, cx, cy, cz - 1) + r0);
                if constexpr (AXES) {
                    if (acc[0] != T(0) || acc[1] != T(0) || acc[2] != T(0))
                        emit(cx, cy, cz, coef * acc[0], coef * acc[1], coef * acc[2]);
                } else if (acc[0] != T(0)) {
                    emit(cx, cy, cz, coef * acc[0]);
                }
            }
}

// F1: central cell of each point (FP64 floor), copies of the points into the
// handle, the linear cell key, and a histogram of points per kTile^3 tile.
// rank[i] is the point's slot inside its tile.  A point outside the grid sets
// *err and gets key -1, tile -1.
__global__ __launch_bounds__(256) void k_bin_points(const float *__restrict__ xyz, const float *__restrict__ nrm,
                                                     int npts, GridF g, TileDims td, int32_t *__restrict__ keys,
                                                     float *__restrict__ xyz_c, float *__restrict__ nrm_c,
                                                     int32_t *__restrict__ tile_of, uint32_t *__restrict__ rank,
                                                     uint32_t *__restrict__ tile_cnt, int *err,
                                                     uint32_t *nmax_bits) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    const float x0 = xyz[3 * i], x1 = xyz[3 * i + 1], x2 = xyz[3 * i + 2];
    xyz_c[3 * i] = x0; xyz_c[3 * i + 1] = x1; xyz_c[3 * i + 2] = x2;
    nrm_c[3 * i] = nrm[3 * i]; nrm_c[3 * i + 1] = nrm[3 * i + 1]; nrm_c[3 * i + 2] = nrm[3 * i + 2];
    if (nmax_bits) {
        // largest |normal component| as float bits (NaN and Inf order above every finite value)
        uint32_t m = max(max(__float_as_uint(fabsf(nrm[3 * i])), __float_as_uint(fabsf(nrm[3 * i + 1]))),
                         __float_as_uint(fabsf(nrm[3 * i + 2])));
        atomicMax(nmax_bits, m);
    }
    AxisW<float> X, Y, Z;
    if (!bin_axis(x0, g.lo[0], g.h, g.d.nx, X, 0.f) || !bin_axis(x1, g.lo[1], g.h, g.d.ny, Y, 0.f) ||
        !bin_axis(x2, g.lo[2], g.h, g.d.nz, Z, 0.f)) {
        keys[i] = -1;
        tile_of[i] = -1;
        atomicOr(err, 1);
        return;
    }
    keys[i] = X.k + g.d.nx * (Y.k + g.d.ny * Z.k);
    const int t = X.k / kTile + td.tx * (Y.k / kTile + td.ty * (Z.k / kTile));
    tile_of[i] = t;
    rank[i] = atomicAdd(tile_cnt + t, 1u);
}

// Points ordered by tile: perm[tile_off[t] + rank[i]] = i.
__global__ __launch_bounds__(256) void k_tile_scatter(const int32_t *__restrict__ tile_of,
                                                       const uint32_t *__restrict__ rank,
                                                       const uint32_t *__restrict__ tile_off, int npts,
                                                       uint32_t *__restrict__ perm) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    const int t = tile_of[i];
    if (t >= 0) perm[tile_off[t] + rank[i]] = (uint32_t)i;
}

// Chunks of at most kChunk points of one tile: chunk counts per tile ...
__global__ __launch_bounds__(256) void k_chunk_counts(const uint32_t *__restrict__ tile_cnt, uint32_t ntiles,
                                                       uint32_t *__restrict__ ch_cnt) {
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ntiles) ch_cnt[t] = (tile_cnt[t] + kChunk - 1) / kChunk;
}

// ... and the tile of every chunk.
__global__ __launch_bounds__(256) void k_chunk_tiles(const uint32_t *__restrict__ ch_cnt,
                                                      const uint32_t *__restrict__ ch_off, uint32_t ntiles,
                                                      uint32_t *__restrict__ chunk_tile) {
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    for (uint32_t c = 0; c < ch_cnt[t]; ++c) chunk_tile[ch_off[t] + c] = t;
}

// F2 + F3: a workgroup takes chunks (at most kChunk points of one tile); the
// points add their divergence contributions into a (kTile + 4)^3 window in
// LDS (the support reaches two cells out), then each touched cell of the
// window gets one atomic add into the global sums.  The grid strides over the
// chunks; their count is read on the device.  Modes:
//   kSplatF32:   FP32 contributions, FP32 atomics into b (b zero on entry);
//   kSplatFixed: FP32 contributions rounded to 64-bit fixed point (unit
//                fix->inv), integer atomics into acc (zero on entry);
//   kSplatFixed64: the same with FP64 weights and contributions;
//   kSplatExact: the exact-quadrature right-hand side (Eq. 26 integrated
//                exactly), b = sum_xi M_perp,xi b_xi, where b_xi is the
//                kSplatF32 sum's xi term and M_perp,xi applies the 1-D mass
//                m = (1, 4, 1)/6 (indices clamped to the grid) along the two
//                other axes.  The three terms go to three LDS windows; after
//                the chunk's points, each cell of the window widened by one
//                (the mass reaches one cell further) gathers its filtered sum
//                and adds it to b (FP32 atomics, b zero on entry).
// Integer sums do not depend on the order the adds arrive in, so the fixed
// point modes give the same acc however threads and workgroups interleave.
template <int Mode>
__global__ __launch_bounds__(256) void k_splat_chunks(const uint32_t *__restrict__ perm,
                                                       const uint32_t *__restrict__ tile_off,
                                                       const uint32_t *__restrict__ tile_cnt,
                                                       const uint32_t *__restrict__ ch_off,
                                                       const uint32_t *__restrict__ chunk_tile,
                                                       const uint32_t *__restrict__ n_chunks,
                                                       const float *__restrict__ xyz_c, const float *__restrict__ nrm_c,
                                                       GridF g, TileDims td, float *__restrict__ b,
                                                       unsigned long long *__restrict__ acc, const FixedScale *fix) {
    constexpr bool kFloat = Mode == kSplatF32 || Mode == kSplatExact;
    using T = typename std::conditional<Mode == kSplatFixed64, double, float>::type;
    using W = typename std::conditional<kFloat, float, unsigned long long>::type;
    constexpr int WN = kTile + 4, W3 = WN * WN * WN;
    constexpr int NW = Mode == kSplatExact ? 3 : 1;
    __shared__ W win[NW * W3];
    const uint32_t total = n_chunks[0];
    const double scale = kFloat ? 0.0 : fix->scale;
    for (uint32_t ch = blockIdx.x; ch < total; ch += gridDim.x) {
        const uint32_t tile = chunk_tile[ch];
        const uint32_t c = ch - ch_off[tile];
        const uint32_t p0 = c * kChunk, p1 = min(p0 + kChunk, tile_cnt[tile]);
        for (int l = threadIdx.x; l < NW * W3; l += blockDim.x) win[l] = W(0);
        __syncthreads();
        const int T0x = (int)(tile % td.tx) * kTile, T0y = (int)((tile / td.tx) % td.ty) * kTile,
                  T0z = (int)(tile / (td.tx * td.ty)) * kTile;
        const uint32_t off = tile_off[tile];
        for (uint32_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
            const uint32_t i = perm[off + p];
            AxisW<T> X, Y, Z;
            bin_axis(xyz_c[3 * i], g.lo[0], g.h, g.d.nx, X, T(0));
            bin_axis(xyz_c[3 * i + 1], g.lo[1], g.h, g.d.ny, Y, T(0));
            bin_axis(xyz_c[3 * i + 2], g.lo[2], g.h, g.d.nz, Z, T(0));
            const int lx = X.k - T0x + 2, ly = Y.k - T0y + 2, lz = Z.k - T0z + 2;
            if constexpr (Mode == kSplatExact) {
                point_divergence<true>(X, Y, Z, nrm_c[3 * i], nrm_c[3 * i + 1], nrm_c[3 * i + 2], g,
                                       [&](int cx, int cy, int cz, float vx, float vy, float vz) {
                                           float *dst = win + (lx + cx) + WN * ((ly + cy) + WN * (lz + cz));
                                           atomicAdd(dst, vx);
                                           atomicAdd(dst + W3, vy);
                                           atomicAdd(dst + 2 * W3, vz);
                                       });
            } else {
                point_divergence(X, Y, Z, (T)nrm_c[3 * i], (T)nrm_c[3 * i + 1], (T)nrm_c[3 * i + 2], g,
                                 [&](int cx, int cy, int cz, T v) {
                                     W *dst = win + (lx + cx) + WN * ((ly + cy) + WN * (lz + cz));
                                     if constexpr (Mode == kSplatF32) atomicAdd(dst, v);
                                     else atomicAdd(dst, (unsigned long long)__double2ll_rn((double)v * scale));
                                 });
            }
        }
        __syncthreads();
        if constexpr (Mode == kSplatExact) {
            // output cells T0 - 3 .. T0 + kTile + 2 per axis; window coordinate
            // of a grid cell: g - T0 + 2, valid in [0, WN)
            constexpr int WO = kTile + 6;
            const float mw[3] = {1.f / 6.f, 2.f / 3.f, 1.f / 6.f};
            for (int l = threadIdx.x; l < WO * WO * WO; l += blockDim.x) {
                const int gx = T0x - 3 + l % WO, gy = T0y - 3 + (l / WO) % WO, gz = T0z - 3 + l / (WO * WO);
                if (gx < 0 || gx >= g.d.nx || gy < 0 || gy >= g.d.ny || gz < 0 || gz >= g.d.nz) continue;
                // window coordinates of the clamped neighbours (-1: outside the window)
                int wx[3], wy[3], wz[3];
                for (int a = 0; a < 3; ++a) {
                    const int ux = min(max(gx + a - 1, 0), g.d.nx - 1) - T0x + 2;
                    const int uy = min(max(gy + a - 1, 0), g.d.ny - 1) - T0y + 2;
                    const int uz = min(max(gz + a - 1, 0), g.d.nz - 1) - T0z + 2;
                    wx[a] = (ux >= 0 && ux < WN) ? ux : -1;
                    wy[a] = (uy >= 0 && uy < WN) ? uy : -1;
                    wz[a] = (uz >= 0 && uz < WN) ? uz * WN * WN : -1;
                }
                float v = 0.f;
                for (int a = 0; a < 3; ++a)
                    for (int e = 0; e < 3; ++e) {
                        const float w = mw[a] * mw[e];
                        if (wx[1] >= 0 && wy[a] >= 0 && wz[e] >= 0) v += w * win[wx[1] + WN * wy[a] + wz[e]];
                        if (wy[1] >= 0 && wx[a] >= 0 && wz[e] >= 0) v += w * win[W3 + wx[a] + WN * wy[1] + wz[e]];
                        if (wz[1] >= 0 && wx[a] >= 0 && wy[e] >= 0)
                            v += w * win[2 * W3 + wx[a] + WN * wy[e] + wz[1]];
                    }
                if (v != 0.f) unsafeAtomicAdd(b + (size_t)gx + (size_t)g.d.nx * (gy + (size_t)g.d.ny * gz), v);
            }
            __syncthreads();
            continue;
        }
        for (int l = threadIdx.x; l < WN * WN * WN; l += blockDim.x) {
            const W v = win[l];
            if (v == W(0)) continue;
            const int gx = T0x - 2 + l % WN, gy = T0y - 2 + (l / WN) % WN, gz = T0z - 2 + l / (WN * WN);
            // contributions only ever target cells inside the grid
            const size_t o = (size_t)gx + (size_t)g.d.nx * (gy + (size_t)g.d.ny * gz);
            if constexpr (Mode == kSplatF32) unsafeAtomicAdd(b + o, v);
            else atomicAdd(acc + o, v);
        }
        __syncthreads();
    }
}

template __global__ void k_splat_chunks<kSplatF32>(const uint32_t *, const uint32_t *, const uint32_t *,
                                                   const uint32_t *, const uint32_t *, const uint32_t *, const float *,
                                                   const float *, GridF, TileDims, float *, unsigned long long *,
                                                   const FixedScale *);
template __global__ void k_splat_chunks<kSplatFixed>(const uint32_t *, const uint32_t *, const uint32_t *,
                                                     const uint32_t *, const uint32_t *, const uint32_t *,
                                                     const float *, const float *, GridF, TileDims, float *,
                                                     unsigned long long *, const FixedScale *);
template __global__ void k_splat_chunks<kSplatExact>(const uint32_t *, const uint32_t *, const uint32_t *,
                                                     const uint32_t *, const uint32_t *, const uint32_t *,
                                                     const float *, const float *, GridF, TileDims, float *,
                                                     unsigned long long *, const FixedScale *);
template __global__ void k_splat_chunks<kSplatFixed64>(const uint32_t *, const uint32_t *, const uint32_t *,
                                                       const uint32_t *, const uint32_t *, const uint32_t *,
                                                       const float *, const float *, GridF, TileDims, float *,
                                                       unsigned long long *, const FixedScale *);

// The fixed-point unit of the deterministic splat: 2^-e with e the largest
// exponent for which npts * 3.75 h^-2 max|n_k| (a bound on any cell's sum, see
// point_divergence) stays below 2^61 in units.  A non-finite normal sets bit 2
// of *err and leaves the scale 0.
__global__ void k_fixed_scale(const uint32_t *nmax_bits, int npts, double h, FixedScale *fix, int *err) {
    const uint32_t bits = *nmax_bits;
    if (bits >= 0x7f800000u) {
        atomicOr(err, 4);
        fix->scale = fix->inv = 0.0;
        return;
    }
    const double bound = (double)npts * 3.75 * (double)__uint_as_float(bits) / (h * h);
    int e = 0;
    if (bound > 0.0) e = 61 - (int)ceil(log2(bound));
    fix->scale = ldexp(1.0, e);
    fix->inv = ldexp(1.0, -e);
}

// b = acc * unit, as float or (in place over acc) as double.
template <class T>
__global__ __launch_bounds__(256) void k_fixed_to_b(const long long *acc, const FixedScale *fix, size_t n, T *b) {
    const double inv = fix->inv;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = (T)((double)acc[i] * inv);
}
template __global__ void k_fixed_to_b<float>(const long long *, const FixedScale *, size_t, float *);
template __global__ void k_fixed_to_b<double>(const long long *, const FixedScale *, size_t, double *);

// Bounding box of a cloud: per axis the minimum and maximum coordinate, as
// order-preserving unsigned keys (a float's bits with the sign bit flipped for
// non-negative values and all bits flipped for negative ones), so that
// unsigned atomics take exact minima and maxima in any order.  box[0..2] min,
// box[3..5] max; box is set to (0xffffffff x 3, 0 x 3) before the launch.
__device__ __forceinline__ uint32_t order_key(float v) {
    const uint32_t b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__global__ __launch_bounds__(256) void k_bbox(const float *__restrict__ xyz, int npts, uint32_t *box, int *err) {
    uint32_t mn[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, mx[3] = {0u, 0u, 0u};
    bool bad = false;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += gridDim.x * blockDim.x)
        for (int a = 0; a < 3; ++a) {
            const float v = xyz[3 * i + a];
            bad |= !isfinite(v);
            const uint32_t k = order_key(v);
            mn[a] = min(mn[a], k);
            mx[a] = max(mx[a], k);
        }
    for (int a = 0; a < 3; ++a)
        for (int o = 32; o > 0; o >>= 1) {
            mn[a] = min(mn[a], (uint32_t)__shfl_xor((int)mn[a], o, 64));
            mx[a] = max(mx[a], (uint32_t)__shfl_xor((int)mx[a], o, 64));
        }
    // the workgroup's wavefronts meet in LDS; one set of global atomics per workgroup
    __shared__ uint32_t wmn[3], wmx[3];
    __shared__ int wbad;
    if (threadIdx.x < 3) {
        wmn[threadIdx.x] = 0xffffffffu;
        wmx[threadIdx.x] = 0u;
    }
    if (threadIdx.x == 0) wbad = 0;
    __syncthreads();
    if (__ballot(bad) != 0 && threadIdx.x % 64 == 0) atomicOr(&wbad, 1);
    if (threadIdx.x % 64 == 0)
        for (int a = 0; a < 3; ++a) {
            atomicMin(&wmn[a], mn[a]);
            atomicMax(&wmx[a], mx[a]);
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (wbad) atomicOr(err, 1);
        for (int a = 0; a < 3; ++a) {
            atomicMin(box + a, wmn[a]);
            atomicMax(box + 3 + a, wmx[a]);
        }
    }
}

namespace {

// Trilinear stencil of a cell-centred field at a world point: base cell and
// weights along each axis, u = (x - lo)/h - 1/2 clamped to [0, n-1].
struct Tri1 {
    int i0;
    double t;
    bool clamped;
};
__device__ __forceinline__ Tri1 tri_axis(float x, double lo, double h, int n) {
    double u = ((double)x - lo) / h - 0.5;
    Tri1 r;
    r.clamped = !(u >= 0.0 && u <= (double)(n - 1));
    u = fmin(fmax(u, 0.0), (double)(n - 1));
    int i0 = (int)floor(u);
    if (i0 > n - 2) i0 = n - 2;
    r.i0 = i0;
    r.t = u - (double)i0;
    return r;
}

}  // namespace

// chi_h at point i, interpolated trilinearly (the indicator values near the
// samples that the iso-value is taken from, Sec. 2.4)
__device__ __forceinline__ double iso_point(const float *__restrict__ xyz, int i, const GridF &g,
                                            const double *__restrict__ chi) {
    Tri1 X = tri_axis(xyz[3 * i], g.lo[0], g.h, g.d.nx);
    Tri1 Y = tri_axis(xyz[3 * i + 1], g.lo[1], g.h, g.d.ny);
    Tri1 Z = tri_axis(xyz[3 * i + 2], g.lo[2], g.h, g.d.nz);
    const size_t sy = g.d.nx, sz = (size_t)g.d.nx * g.d.ny;
    const double *c = chi + X.i0 + sy * Y.i0 + sz * Z.i0;
    double v = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? X.t : 1.0 - X.t) * (dy ? Y.t : 1.0 - Y.t) * (dz ? Z.t : 1.0 - Z.t);
                v += w * c[dx + sy * dy + sz * dz];
            }
    return v;
}

// Iso-value partial sums: sum_i chi_h(x_i) with chi in FP64 (Sec. 2.4).
__global__ __launch_bounds__(256) void k_iso_partial(const float *__restrict__ xyz, int npts, GridF g,
                                                      const double *__restrict__ chi, double *partials) {
    double acc[1] = {0.0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += gridDim.x * blockDim.x)
        acc[0] += iso_point(xyz, i, g, chi);
    __shared__ double lds[4][1];
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
}

// The same mean independent of the points' order (deterministic requests):
// the largest |chi_h| at a point (atomicMax on the bits of a non-negative
// double, which order like integers) fixes a unit 2^-e with npts * max < 2^61
// units; each point's value rounded to that unit is summed with 64-bit
// integer atomics, which associate.  w[0]: the bits of the largest value,
// w[1]: the sum (both zero on entry).
__device__ __forceinline__ int iso_unit_exp(unsigned long long maxbits, int npts) {
    const double bound = __longlong_as_double((long long)maxbits) * (double)npts;
    return bound > 0.0 ? 61 - (int)ceil(log2(bound)) : 0;
}

__global__ __launch_bounds__(256) void k_iso_absmax(const float *__restrict__ xyz, int npts, GridF g,
                                                     const double *__restrict__ chi, unsigned long long *w) {
    unsigned long long m = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += gridDim.x * blockDim.x) {
        const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(iso_point(xyz, i, g, chi)));
        m = b > m ? b : m;
    }
    if (m) atomicMax(w, m);
}

__global__ __launch_bounds__(256) void k_iso_fixed(const float *__restrict__ xyz, int npts, GridF g,
                                                    const double *__restrict__ chi, unsigned long long *w) {
    const int e = iso_unit_exp(w[0], npts);
    long long acc = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += gridDim.x * blockDim.x)
        acc += __double2ll_rn(ldexp(iso_point(xyz, i, g, chi), e));
    if (acc) atomicAdd(w + 1, (unsigned long long)acc);
}

__global__ void k_iso_fixed_finalize(const unsigned long long *w, int npts, double *out) {
    out[0] = ldexp((double)(long long)w[1], -iso_unit_exp(w[0], npts)) / (double)npts;
}

// c = (sum of partials) / N  (minus nothing: the caller subtracts the field mean)
__global__ void k_iso_finalize(const double *partials, int nb, int npts, double *out) {
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < nb; i += blockDim.x) v[0] += partials[i];
    __shared__ double lds[4][1];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) out[0] = v[0] / (double)npts;
}

// Reverse of the iso-value into the field: g_chi += (g_c / N) * trilinear weights.
__global__ __launch_bounds__(256) void k_iso_T(const float *__restrict__ xyz, int npts, GridF g,
                                                const double *g_c, float *__restrict__ g_chi) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    const float s = (float)(g_c[0] / (double)npts);
    if (s == 0.f) return;
    Tri1 X = tri_axis(xyz[3 * i], g.lo[0], g.h, g.d.nx);
    Tri1 Y = tri_axis(xyz[3 * i + 1], g.lo[1], g.h, g.d.ny);
    Tri1 Z = tri_axis(xyz[3 * i + 2], g.lo[2], g.h, g.d.nz);
    const size_t sy = g.d.nx, sz = (size_t)g.d.nx * g.d.ny;
    float *c = g_chi + X.i0 + sy * Y.i0 + sz * Z.i0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                float w = (float)((dx ? X.t : 1.0 - X.t) * (dy ? Y.t : 1.0 - Y.t) * (dz ? Z.t : 1.0 - Z.t));
                unsafeAtomicAdd(c + dx + sy * dy + sz * dz, s * w);
            }
}

// Transpose of the exact-quadrature right-hand side at every cell:
// g_V_xi = h (g^T along xi, m across) lambda, with g the 1-D face-average
// divergence (g^T u at p: (u[p+1] - u[p-1]) / 2, indices clamped to the grid)
// and m = (1, 4, 1)/6 with clamped indices; FP64 sums, stored FP32 in the
// three fields gv.p[xi].
__global__ __launch_bounds__(256) void k_grad27_T(const double *__restrict__ lam, Dims d, double h, Planes3 gv) {
    const size_t N = d.count();
    const size_t sy = (size_t)d.nx, sz = (size_t)d.nx * d.ny;
    const double mw[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(c % sy), j = (int)((c / sy) % d.ny), k = (int)(c / sz);
        size_t ox[3], oy[3], oz[3];
        for (int a = 0; a < 3; ++a) {
            ox[a] = (size_t)min(max(i + a - 1, 0), d.nx - 1);
            oy[a] = (size_t)min(max(j + a - 1, 0), d.ny - 1) * sy;
            oz[a] = (size_t)min(max(k + a - 1, 0), d.nz - 1) * sz;
        }
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int e = 0; e < 3; ++e) {
                const double w = mw[a] * mw[e];
                gx += w * (lam[ox[2] + oy[a] + oz[e]] - lam[ox[0] + oy[a] + oz[e]]);
                gy += w * (lam[ox[a] + oy[2] + oz[e]] - lam[ox[a] + oy[0] + oz[e]]);
                gz += w * (lam[ox[a] + oy[e] + oz[2]] - lam[ox[a] + oy[e] + oz[0]]);
            }
        gv.p[0][c] = (float)(0.5 * h * gx);
        gv.p[1][c] = (float)(0.5 * h * gy);
        gv.p[2][c] = (float)(0.5 * h * gz);
    }
}

// B5 + B6 (+ the point term of the iso-value reverse).  With lambda the
// adjoint solution, g_V = -h^2 D_h^T lambda is formed on the fly at each of
// the 27 stencil cells (EXACT: read from the fields k_grad27_T wrote), then
//   g_n_i = h^-3 sum_o alpha_o g_V,o,
//   g_x_i = h^-3 sum_o (d alpha_o / d x_i) (n_i . g_V,o) + (g_c / N) grad chi_h(x_i).
// The central cell of each point is the one recorded by the forward pass.
template <bool EXACT>
__global__ __launch_bounds__(256) void k_splat_T(const float *__restrict__ xyz, const float *__restrict__ nrm,
                                                  const int32_t *__restrict__ keys, int npts, GridF g,
                                                  const double *__restrict__ lam, Planes3 gvp,
                                                  const double *__restrict__ chi, const double *g_c,
                                                  float *__restrict__ gxyz, float *__restrict__ gnrm) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    const float xv[3] = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
    const float nv[3] = {nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2]};
    const int key = keys[i];
    const int kk[3] = {key % g.d.nx, (key / g.d.nx) % g.d.ny, key / (g.d.nx * g.d.ny)};
    const int nn[3] = {g.d.nx, g.d.ny, g.d.nz};
    const float inv4h = (float)(0.25 / g.h);
    AxisW<float> W[3];
    for (int a = 0; a < 3; ++a) {
        double t = ((double)xv[a] - g.lo[a]) / g.h;
        W[a].k = kk[a];
        W[a].f = (float)(t - (double)kk[a]);
        for (int d = -1; d <= 1; ++d) {
            float D = W[a].f - 0.5f - (float)d;
            bool in = in_range(kk[a], d, nn[a]);
            W[a].a[d + 1] = in ? 0.5f * (1.f - fabsf(D) * 0.5f) : 0.f;
            float sg = D > 0.f ? 1.f : (D < 0.f ? -1.f : 0.f);
            W[a].da[d + 1] = in ? -sg * inv4h : 0.f;
        }
    }
    const AxisW<float> &X = W[0], &Y = W[1], &Z = W[2];
    const float Sx = X.a[0] + X.a[1] + X.a[2], Sy = Y.a[0] + Y.a[1] + Y.a[2], Sz = Z.a[0] + Z.a[1] + Z.a[2];
    const float S = Sx * Sy * Sz - X.a[1] * Y.a[1] * Z.a[1] + 0.5f;
    const float dSx = (X.da[0] + X.da[1] + X.da[2]) * Sy * Sz - X.da[1] * Y.a[1] * Z.a[1];
    const float dSy = Sx * (Y.da[0] + Y.da[1] + Y.da[2]) * Sz - X.a[1] * Y.da[1] * Z.a[1];
    const float dSz = Sx * Sy * (Z.da[0] + Z.da[1] + Z.da[2]) - X.a[1] * Y.a[1] * Z.da[1];
    const size_t sy = (size_t)g.d.nx, sz = (size_t)g.d.nx * g.d.ny;
    const size_t c0 = (size_t)X.k + sy * Y.k + sz * Z.k;
    const double half_h = 0.5 * g.h;
    float gn[3] = {0.f, 0.f, 0.f};
    float sum_rs = 0.f, sum_drs[3] = {0.f, 0.f, 0.f};
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!in_range(X.k, dx, g.d.nx) || !in_range(Y.k, dy, g.d.ny) || !in_range(Z.k, dz, g.d.nz)) continue;
                const size_t o = c0 + (ptrdiff_t)dx + (ptrdiff_t)dy * (ptrdiff_t)sy + (ptrdiff_t)dz * (ptrdiff_t)sz;
                float gv[3];
                if constexpr (EXACT) {
                    for (int a = 0; a < 3; ++a) gv[a] = gvp.p[a][o];
                } else {
                    const double lo_ = lam[o];
                    const int off[3] = {dx, dy, dz};
                    const size_t st[3] = {1, sy, sz};
                    for (int a = 0; a < 3; ++a) {
                        double acc = 0.0;
                        if (in_range(kk[a], off[a] - 1, nn[a])) acc += lam[o - st[a]] - lo_;
                        if (in_range(kk[a], off[a] + 1, nn[a])) acc += lo_ - lam[o + st[a]];
                        gv[a] = (float)(-half_h * acc);
                    }
                }
                const bool centre = dx == 0 && dy == 0 && dz == 0;
                const float ax = X.a[dx + 1], ay = Y.a[dy + 1], az = Z.a[dz + 1];
                const float raw = centre ? 0.5f : ax * ay * az;
                const float s_o = nv[0] * gv[0] + nv[1] * gv[1] + nv[2] * gv[2];
                for (int a = 0; a < 3; ++a) gn[a] += raw * gv[a];
                sum_rs += raw * s_o;
                if (!centre) {
                    sum_drs[0] += X.da[dx + 1] * ay * az * s_o;
                    sum_drs[1] += ax * Y.da[dy + 1] * az * s_o;
                    sum_drs[2] += ax * ay * Z.da[dz + 1] * s_o;
                }
            }
    const float hm3 = (float)(1.0 / (g.h * g.h * g.h));
    const float invS = 1.f / S;
    const float dS[3] = {dSx, dSy, dSz};
    float gx[3];
    for (int a = 0; a < 3; ++a) {
        gnrm[3 * i + a] = hm3 * gn[a] * invS;
        gx[a] = hm3 * (sum_drs[a] * invS - dS[a] * invS * invS * sum_rs);
    }
    // iso-value: c = mean chi_h(x_i)  ->  g_x += (g_c / N) grad chi_h
    const double sc = g_c[0] / (double)npts;
    if (sc != 0.0) {
        Tri1 T[3];
        for (int a = 0; a < 3; ++a) T[a] = tri_axis(xv[a], g.lo[a], g.h, nn[a]);
        const double *c = chi + T[0].i0 + sy * T[1].i0 + sz * T[2].i0;
        double grad[3] = {0, 0, 0};
        for (int ez = 0; ez < 2; ++ez)
            for (int ey = 0; ey < 2; ++ey)
                for (int ex = 0; ex < 2; ++ex) {
                    double v = c[ex + sy * ey + sz * ez];
                    double fx = ex ? T[0].t : 1.0 - T[0].t, fy = ey ? T[1].t : 1.0 - T[1].t,
                           fz = ez ? T[2].t : 1.0 - T[2].t;
                    double gx_ = (ex ? 1.0 : -1.0) * fy * fz, gy_ = fx * (ey ? 1.0 : -1.0) * fz,
                           gz_ = fx * fy * (ez ? 1.0 : -1.0);
                    grad[0] += gx_ * v;
                    grad[1] += gy_ * v;
                    grad[2] += gz_ * v;
                }
        for (int a = 0; a < 3; ++a)
            if (!T[a].clamped) gx[a] += (float)(sc * grad[a] / g.h);
    }
    for (int a = 0; a < 3; ++a) gxyz[3 * i + a] = gx[a];
}

template __global__ void k_splat_T<false>(const float *, const float *, const int32_t *, int, GridF, const double *,
                                          Planes3, const double *, const double *, float *, float *);
template __global__ void k_splat_T<true>(const float *, const float *, const int32_t *, int, GridF, const double *,
                                         Planes3, const double *, const double *, float *, float *);

}  // namespace wg
