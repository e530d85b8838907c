// Normal estimation and orientation (Warp-Geo Sec. 2.1-2.2): the steps before
// the Poisson path, for clouds that come without oriented normals.
//
// Both run over a uniform point grid: the points sorted by cell (a counting
// sort), so that the cells of one x row are one contiguous range of the
// sorted array.  A search visits, for each (y, z) cell row that a query ball
// reaches, one range of points; threads take the points in sorted order, so
// the threads of a wavefront search the same rows and their loads coincide.
//
// Decisions that turn a floating-point comparison into an integer (is a point
// within R, is a probe within r_d, the nearest spacing) compare FP32 squared
// distances, products and sums rounded one by one and summed x, y, z in that
// order, with no contraction: the same arithmetic as the host-side statement
// of the method, so the neighbour sets, detection arrays and flips are the
// same bit for bit.  Everything after a neighbour set is formed is FP64.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>

#include "kernels.h"
#include "scan.h"

namespace wg {

namespace {

__device__ __forceinline__ float d2f(float ax, float ay, float az, float bx, float by, float bz) {
#pragma clang fp contract(off)
    const float dx = bx - ax, dy = by - ay, dz = bz - az;
    float s = dx * dx;
    s = s + dy * dy;
    s = s + dz * dz;
    return s;
}

// Points sorted by cell; w of each float4 holds the point's index (bits).
struct PGrid {
    float lo[3];
    float inv_cs;
    int n[3];
    const uint32_t *start;   // [cells + 1]
    const float4 *pts;
};

__device__ __forceinline__ int cell_of(const PGrid &g, int a, float v) {
    const int c = (int)floorf((v - g.lo[a]) * g.inv_cs);
    return min(max(c, 0), g.n[a] - 1);
}

// Calls f(q) for every point q of the cells within `reach` of (x, y, z)
// (reach slightly above the decision radius, so every point the exact test
// accepts lies in a visited cell); f returns true to stop.
template <class F>
__device__ __forceinline__ bool for_near(const PGrid &g, float x, float y, float z, float reach, F &&f) {
    const int x0 = cell_of(g, 0, x - reach), x1 = cell_of(g, 0, x + reach);
    const int y0 = cell_of(g, 1, y - reach), y1 = cell_of(g, 1, y + reach);
    const int z0 = cell_of(g, 2, z - reach), z1 = cell_of(g, 2, z + reach);
    for (int cz = z0; cz <= z1; ++cz)
        for (int cy = y0; cy <= y1; ++cy) {
            const size_t row = (size_t)g.n[0] * (cy + (size_t)g.n[1] * cz);
            const uint32_t b = g.start[row + x0], e = g.start[row + x1 + 1];
            for (uint32_t j = b; j < e; ++j)
                if (f(g.pts[j])) return true;
        }
    return false;
}

// ---- point grid -------------------------------------------------------------

__global__ __launch_bounds__(256) void k_pg_count(const float *__restrict__ xyz, int npts, PGrid g,
                                                   uint32_t *__restrict__ cell, uint32_t *__restrict__ rank,
                                                   uint32_t *__restrict__ cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    const int cx = cell_of(g, 0, xyz[3 * i]), cy = cell_of(g, 1, xyz[3 * i + 1]), cz = cell_of(g, 2, xyz[3 * i + 2]);
    const uint32_t c = (uint32_t)cx + (uint32_t)g.n[0] * ((uint32_t)cy + (uint32_t)g.n[1] * (uint32_t)cz);
    cell[i] = c;
    rank[i] = atomicAdd(cnt + c, 1u);
}

__global__ __launch_bounds__(256) void k_pg_scatter(const float *__restrict__ xyz, int npts,
                                                     const uint32_t *__restrict__ cell,
                                                     const uint32_t *__restrict__ rank,
                                                     const uint32_t *__restrict__ start, float4 *__restrict__ pts) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    pts[start[cell[i]] + rank[i]] = make_float4(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], __int_as_float(i));
}

__global__ void k_set_word(uint32_t *p, uint32_t v) { *p = v; }

// *bad = 1 if any of the n values is NaN or infinite
__global__ __launch_bounds__(256) void k_any_nonfinite(const float *__restrict__ v, size_t n, int *bad) {
    bool b = false;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b |= !isfinite(v[i]);
    if (__ballot(b) != 0 && threadIdx.x % 64 == 0) atomicOr(bad, 1);
}

// chunks of at most `per` points of one cell: their count per cell, then the
// cell of every chunk
__global__ __launch_bounds__(256) void k_cell_chunks(const uint32_t *__restrict__ cnt, uint32_t cells, uint32_t per,
                                                      uint32_t *__restrict__ ch_cnt) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < cells) ch_cnt[c] = (cnt[c] + per - 1) / per;
}
__global__ __launch_bounds__(256) void k_chunk_cells(const uint32_t *__restrict__ ch_cnt,
                                                      const uint32_t *__restrict__ ch_off, uint32_t cells,
                                                      uint32_t *__restrict__ chunk_cell) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    for (uint32_t k = 0; k < ch_cnt[c]; ++k) chunk_cell[ch_off[c] + k] = c;
}

// ---- D-PCA (Sec. 2.1) ---------------------------------------------------------

// Eigenvector of the smallest eigenvalue of the symmetric 3x3 matrix
// a = (xx, xy, xz, yy, yz, zz), by the cyclic Jacobi method (plane rotations
// annihilating each off-diagonal entry in turn until they vanish), FP64.
__device__ void min_eigvec3(const double a[6], double v[3]) {
    double A[3][3] = {{a[0], a[1], a[2]}, {a[1], a[3], a[4]}, {a[2], a[4], a[5]}};
    double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int sweep = 0; sweep < 24; ++sweep) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (!(off > 1e-34 * dia) || off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                const double apq = A[p][q];
                if (apq == 0.0) continue;
                const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
                const double t = fabs(theta) > 1e150 ? 0.5 / theta
                                                     : (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 3; ++k) {   // A <- A J (columns p, q)
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {   // A <- J^T A (rows p, q)
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {   // V <- V J
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
    int m = 0;
    if (A[1][1] < A[m][m]) m = 1;
    if (A[2][2] < A[m][m]) m = 2;
    const double nn = sqrt(V[0][m] * V[0][m] + V[1][m] * V[1][m] + V[2][m] * V[2][m]);
    for (int k = 0; k < 3; ++k) v[k] = V[k][m] / nn;
}

// D-PCA of every point.  Neighbours: FP32 squared distance
// <= R^2 (Eq. 1).  Weights 1/(d + eps) (Eq. 2) in FP32 from the root of that
// same squared distance (hardware root and reciprocal, 1 ulp each; relative
// error ~2e-7, which moves a normal by about
// 1e-7 over the relative gap of the two smallest eigenvalues); the weighted
// first and second moments of the offsets q - p accumulate in FP64 and give
// the centroid (Eq. 3) and the covariance about it (Eq. 4),
// C = S2/W - m m^T with m = S1/W.
//
// A workgroup of four wavefronts takes a chunk of at most 64 points of one
// cell (so they share one search box; lane l of every wavefront holds point
// l) and streams the candidates of that box through LDS in tiles of 256: one
// coalesced load per tile, then wavefront w tests candidates 64w..64w+63 of
// the tile against its lane's point (a broadcast LDS read per candidate).
// The four partial sums of each point are added in LDS at the end.
constexpr int kDpcaChunk = 64;
constexpr int kDpcaWaves = 4;

__global__ __launch_bounds__(kDpcaChunk * kDpcaWaves) void k_dpca(PGrid g, const uint32_t *__restrict__ chunk_cell,
                                                                   const uint32_t *__restrict__ ch_off, float R2,
                                                                   float reach, float eps, float *__restrict__ nrm) {
    constexpr int NT = kDpcaChunk * kDpcaWaves;
    __shared__ float4 tile[NT];
    __shared__ double part[kDpcaWaves - 1][10][kDpcaChunk];
    const int lane = threadIdx.x % kDpcaChunk, wv = threadIdx.x / kDpcaChunk;
    const uint32_t ch = blockIdx.x;
    const uint32_t c = chunk_cell[ch];
    const uint32_t first = g.start[c] + (ch - ch_off[c]) * kDpcaChunk, last = g.start[c + 1];
    const uint32_t me = first + lane;
    const bool live = me < last;
    const float4 p = g.pts[live ? me : first];
    // the cell's search box: the cells within reach of any point of the cell
    const int cx = (int)(c % (uint32_t)g.n[0]), cy = (int)((c / (uint32_t)g.n[0]) % (uint32_t)g.n[1]),
              cz = (int)(c / ((uint32_t)g.n[0] * (uint32_t)g.n[1]));
    const float cs = 1.0f / g.inv_cs;
    const float lx = g.lo[0] + cx * cs, ly = g.lo[1] + cy * cs, lz = g.lo[2] + cz * cs;
    const int x0 = min(cell_of(g, 0, lx - reach), cx), x1 = max(cell_of(g, 0, lx + cs + reach), cx);
    const int y0 = min(cell_of(g, 1, ly - reach), cy), y1 = max(cell_of(g, 1, ly + cs + reach), cy);
    const int z0 = min(cell_of(g, 2, lz - reach), cz), z1 = max(cell_of(g, 2, lz + cs + reach), cz);
    const double px = p.x, py = p.y, pz = p.z;
    double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};   // W, S1 (3), S2 (6)
    for (int bz = z0; bz <= z1; ++bz)
        for (int by = y0; by <= y1; ++by) {
            const size_t row = (size_t)g.n[0] * (by + (size_t)g.n[1] * bz);
            const uint32_t b = g.start[row + x0], e = g.start[row + x1 + 1];
            for (uint32_t j0 = b; j0 < e; j0 += NT) {
                const uint32_t cnt = min((uint32_t)NT, e - j0);
                __syncthreads();
                if (threadIdx.x < cnt) tile[threadIdx.x] = g.pts[j0 + threadIdx.x];
                __syncthreads();
                const uint32_t k0 = (uint32_t)wv * kDpcaChunk, k1 = min(k0 + kDpcaChunk, cnt);
#pragma unroll 4
                for (uint32_t k = k0; k < k1; ++k) {
                    const float4 q = tile[k];
                    const float d2 = d2f(p.x, p.y, p.z, q.x, q.y, q.z);
                    if (d2 <= R2) {
                        // hardware root and reciprocal (1 ulp): the weight's error stays ~1e-7 relative
                        const double w = (double)__builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(d2) + eps);
                        const double dx = (double)q.x - px, dy = (double)q.y - py, dz = (double)q.z - pz;
                        const double wx = w * dx, wy = w * dy, wz = w * dz;
                        acc[0] += w;
                        acc[1] += wx;
                        acc[2] += wy;
                        acc[3] += wz;
                        acc[4] += wx * dx;
                        acc[5] += wx * dy;
                        acc[6] += wx * dz;
                        acc[7] += wy * dy;
                        acc[8] += wy * dz;
                        acc[9] += wz * dz;
                    }
                }
            }
        }
    if (wv > 0)
        for (int k = 0; k < 10; ++k) part[wv - 1][k][lane] = acc[k];
    __syncthreads();
    if (wv > 0 || !live) return;
    for (int w = 0; w < kDpcaWaves - 1; ++w)
        for (int k = 0; k < 10; ++k) acc[k] += part[w][k][lane];
    const double W = acc[0];
    const double m[3] = {acc[1] / W, acc[2] / W, acc[3] / W};
    const double C[6] = {acc[4] / W - m[0] * m[0], acc[5] / W - m[0] * m[1], acc[6] / W - m[0] * m[2],
                         acc[7] / W - m[1] * m[1], acc[8] / W - m[1] * m[2], acc[9] / W - m[2] * m[2]};
    double v[3];
    min_eigvec3(C, v);
    const int i = __float_as_int(p.w);
    nrm[3 * i] = (float)v[0];
    nrm[3 * i + 1] = (float)v[1];
    nrm[3 * i + 2] = (float)v[2];
}

// ---- orientation (Sec. 2.2) -----------------------------------------------------

// max over points of the FP32 squared distance to the nearest other point
// (Eq. 13 before the root), as float bits (non-negative floats order as
// unsigned integers).  Rings of cells around the point's cell, until the
// nearest point found is nearer than any point outside the searched cube can
// be (every point outside is at least ring x cell size away).
__global__ __launch_bounds__(256) void k_nn_spacing(PGrid g, float cs, float slack, int npts, uint32_t *d2max_bits) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npts) return;
    const float4 p = g.pts[t];
    const int self = __float_as_int(p.w);
    const int c[3] = {cell_of(g, 0, p.x), cell_of(g, 1, p.y), cell_of(g, 2, p.z)};
    const int maxn = max(g.n[0], max(g.n[1], g.n[2]));
    float best = INFINITY;
    for (int r = 1;; ++r) {
        const int z0 = max(c[2] - r, 0), z1 = min(c[2] + r, g.n[2] - 1);
        const int y0 = max(c[1] - r, 0), y1 = min(c[1] + r, g.n[1] - 1);
        const int x0 = max(c[0] - r, 0), x1 = min(c[0] + r, g.n[0] - 1);
        for (int cz = z0; cz <= z1; ++cz)
            for (int cy = y0; cy <= y1; ++cy) {
                const size_t row = (size_t)g.n[0] * (cy + (size_t)g.n[1] * cz);
                const bool shell = r == 1 || abs(cz - c[2]) == r || abs(cy - c[1]) == r;
                // the shell of this ring: whole rows on its y and z faces, the two end cells elsewhere
                for (int part = 0; part < (shell ? 1 : 2); ++part) {
                    int a = x0, b = x1;
                    if (!shell) {
                        a = b = part == 0 ? c[0] - r : c[0] + r;
                        if (a < 0 || a >= g.n[0]) continue;
                    }
                    for (uint32_t j = g.start[row + a], e = g.start[row + b + 1]; j < e; ++j) {
                        const float4 q = g.pts[j];
                        if (__float_as_int(q.w) == self) continue;
                        best = fminf(best, d2f(p.x, p.y, p.z, q.x, q.y, q.z));
                    }
                }
            }
        const float reach = (float)r * cs - slack;   // every point outside the cube is farther than this
        if ((reach > 0.0f && best < reach * reach) || r >= maxn) break;
    }
    if (best < INFINITY) atomicMax(d2max_bits, __float_as_uint(best));
}

struct RayParams {
    float rd2, ds, reach;
    int M, n_tol, refine;
    float box_lo[3], box_hi[3];   // the cloud's box widened by reach: no detection outside
    const uint32_t *near;         // bit per cell: some point within reach of the cell's range
};

// Bit c of `near`: some point lies in a cell within one cell of c on every
// axis.  The grid's cell size exceeds the detection reach, so a probe within
// reach of a point lies within one cell of it: a probe whose cell has no bit
// detects nothing.  Built as occupancy bits (one atomic per point), then
// dilated by one cell (one thread per cell, 64 cells per wavefront, the bits
// gathered by a ballot).
__global__ __launch_bounds__(256) void k_mark_occ(const float *__restrict__ xyz, int npts, PGrid g,
                                                   uint32_t *occ) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    const uint32_t c = (uint32_t)cell_of(g, 0, xyz[3 * i]) +
                       (uint32_t)g.n[0] * ((uint32_t)cell_of(g, 1, xyz[3 * i + 1]) +
                                           (uint32_t)g.n[1] * (uint32_t)cell_of(g, 2, xyz[3 * i + 2]));
    atomicOr(occ + (c >> 5), 1u << (c & 31));
}

__global__ __launch_bounds__(256) void k_dilate(const uint32_t *__restrict__ occ, PGrid g, uint32_t cells,
                                                 uint32_t *__restrict__ near) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;   // 64 consecutive cells per wavefront
    bool any = false;
    if (c < cells) {
        const int cx = (int)(c % (uint32_t)g.n[0]), cy = (int)((c / (uint32_t)g.n[0]) % (uint32_t)g.n[1]),
                  cz = (int)(c / ((uint32_t)g.n[0] * (uint32_t)g.n[1]));
        for (int z = max(cz - 1, 0); z <= min(cz + 1, g.n[2] - 1) && !any; ++z)
            for (int y = max(cy - 1, 0); y <= min(cy + 1, g.n[1] - 1) && !any; ++y)
                for (int x = max(cx - 1, 0); x <= min(cx + 1, g.n[0] - 1); ++x) {
                    const uint32_t d = (uint32_t)x + (uint32_t)g.n[0] * ((uint32_t)y + (uint32_t)g.n[1] * (uint32_t)z);
                    if ((occ[d >> 5] >> (d & 31)) & 1u) {
                        any = true;
                        break;
                    }
                }
    }
    const unsigned long long m = __ballot(any);
    const uint32_t base = c - (threadIdx.x % 64);   // first cell of this wavefront, a multiple of 64
    if (threadIdx.x % 64 == 0) {
        const uint32_t words = (cells + 31) / 32;
        if ((base >> 5) < words) near[base >> 5] = (uint32_t)m;
        if ((base >> 5) + 1 < words) near[(base >> 5) + 1] = (uint32_t)(m >> 32);
    }
}

// Detection array of one ray (Eq. 8-9) reduced on the fly to (N_i, N_one)
// (Eq. 10-11 and the initial-one count).  Probe y_m = x + (m ds) s, FP32,
// one rounding per product and sum.
__device__ __forceinline__ void cast_ray(const PGrid &g, const RayParams &rp, float x, float y, float z, float sx,
                                         float sy, float sz, int &N, int &n_one) {
#pragma clang fp contract(off)
    int prev = 1, n_all = 0, ones = 0;
    bool first = true;
    for (int m = 0; m <= rp.M; ++m) {
        const float t = (float)m * rp.ds;
        const float px = x + t * sx, py = y + t * sy, pz = z + t * sz;
        int d = 0;
        if (px >= rp.box_lo[0] && px <= rp.box_hi[0] && py >= rp.box_lo[1] && py <= rp.box_hi[1] &&
            pz >= rp.box_lo[2] && pz <= rp.box_hi[2]) {
            const uint32_t c = (uint32_t)cell_of(g, 0, px) +
                               (uint32_t)g.n[0] * ((uint32_t)cell_of(g, 1, py) + (uint32_t)g.n[1] * (uint32_t)cell_of(g, 2, pz));
            if ((rp.near[c >> 5] >> (c & 31)) & 1u)
                d = for_near(g, px, py, pz, rp.reach, [&](const float4 &q) {
                    return d2f(px, py, pz, q.x, q.y, q.z) <= rp.rd2;
                }) ? 1 : 0;
        }
        if (m > 0 && d == 0 && prev == 1) ++n_all;
        if (first) {
            if (d) ++ones;
            else first = false;
        }
        prev = d;
    }
    N = n_all - 1;
    n_one = ones;
}

// Two lanes per point (adjacent, so one shuffle pairs them): the even lane
// casts the ray along +n, the odd one along -n; then the even lane takes the
// flips of Sec. 2.2: iteration 0 flips an odd N_i; a normal whose ray (along
// the normal after iteration 0) starts with more than n_tol detecting probes
// is flipped (iteration 1) and flipped back if the flipped direction shows
// more crossings than the other (iteration 2).
__global__ __launch_bounds__(256) void k_orient(PGrid g, RayParams rp, const float *__restrict__ xyz, int npts,
                                                 float *__restrict__ nrm, int32_t *__restrict__ counts,
                                                 uint32_t *n_flipped) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = tid >> 1, dir = tid & 1;
    const bool live = i < npts;
    const int ii = live ? i : npts - 1;   // lanes past the end pair up on the last point
    const float x = xyz[3 * ii], y = xyz[3 * ii + 1], z = xyz[3 * ii + 2];
    const float nx = nrm[3 * ii], ny = nrm[3 * ii + 1], nz = nrm[3 * ii + 2];
    int N, N1;
    if (dir == 0) cast_ray(g, rp, x, y, z, nx, ny, nz, N, N1);
    else cast_ray(g, rp, x, y, z, -nx, -ny, -nz, N, N1);
    const int No = __shfl_xor(N, 1, 64), N1o = __shfl_xor(N1, 1, 64);
    if (!live || dir != 0) return;
    const int Np = N, N1p = N1, Nm = No, N1m = N1o;
    int s = (Np % 2 != 0) ? -1 : 1;   // iteration 0
    if (rp.refine) {
        const int N0 = s > 0 ? Np : Nm, Nc1 = s > 0 ? N1p : N1m, Nopp = s > 0 ? Nm : Np;
        if (Nc1 > rp.n_tol) {
            s = -s;                         // iteration 1: N_i != 0 or N_one > N_tol holds
            if (Nopp > N0) s = -s;          // iteration 2: the flipped direction crosses more
        }
    }
    if (counts) {
        counts[4 * i] = Np;
        counts[4 * i + 1] = N1p;
        counts[4 * i + 2] = Nm;
        counts[4 * i + 3] = N1m;
    }
    if (s < 0) {
        nrm[3 * i] = -nx;
        nrm[3 * i + 1] = -ny;
        nrm[3 * i + 2] = -nz;
        atomicAdd(n_flipped, 1u);
    }
}

// ---- host side -----------------------------------------------------------------

// Stream-ordered device buffers of one call, freed on the stream at the end.
class Scratch {
  public:
    explicit Scratch(hipStream_t s) : s_(s) {}
    ~Scratch() {
        for (void *p : bufs_) (void)hipFreeAsync(p, s_);
    }
    template <class T> T *take(size_t n) {
        void *p = nullptr;
        WG_HIP(hipMallocAsync(&p, (n ? n : 1) * sizeof(T), s_));
        bufs_.push_back(p);
        return static_cast<T *>(p);
    }

  private:
    hipStream_t s_;
    std::vector<void *> bufs_;
};

float key_to_float(uint32_t k) {
    const uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    float v;
    std::memcpy(&v, &b, 4);
    return v;
}

struct Box {
    float lo[3], hi[3];
    // search reach for a decision radius r: r widened by 0.1% and by a few
    // FP32 ulps of the largest coordinate, so that rounding in cell
    // boundaries and squared distances never hides a point the exact test
    // would accept
    double reach(double r) const {
        double m = 0.0;
        for (int a = 0; a < 3; ++a) m = std::max(m, std::max(std::fabs((double)lo[a]), std::fabs((double)hi[a])));
        return r * 1.001 + 1e-6 * m;
    }
};

// Bounding box of the cloud (exact, from order-preserving keys); a
// non-finite coordinate is an error.
Box cloud_box(const float *xyz, int npts, Scratch &sc, hipStream_t st) {
    uint32_t *dbox = sc.take<uint32_t>(6);
    int *derr = sc.take<int>(1);
    const uint32_t init[6] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0u, 0u, 0u};
    WG_HIP(hipMemcpyAsync(dbox, init, sizeof(init), hipMemcpyHostToDevice, st));
    WG_HIP(hipMemsetAsync(derr, 0, sizeof(int), st));
    k_bbox<<<std::min<unsigned>(cdiv(npts, 256), 256u), 256, 0, st>>>(xyz, npts, dbox, derr);
    WG_LAUNCH_CHECK();
    uint32_t hb[6];
    int herr = 0;
    WG_HIP(hipMemcpyAsync(hb, dbox, sizeof(hb), hipMemcpyDeviceToHost, st));
    WG_HIP(hipMemcpyAsync(&herr, derr, sizeof(int), hipMemcpyDeviceToHost, st));
    WG_HIP(hipStreamSynchronize(st));
    require(herr == 0, WG_EINVAL, "a point coordinate is NaN or infinite");
    Box b;
    for (int a = 0; a < 3; ++a) {
        b.lo[a] = key_to_float(hb[a]);
        b.hi[a] = key_to_float(hb[3 + a]);
    }
    return b;
}

constexpr double kMaxCells = double(1 << 25);

// Sort the points into cells of size >= cs over the box (enlarged if the grid
// would exceed kMaxCells); returns the grid and the cell size used.
PGrid build_grid(const float *xyz, int npts, const Box &b, double cs, Scratch &sc, hipStream_t st, double &cs_used,
                 const uint32_t **counts = nullptr) {
    double ext[3];
    for (int a = 0; a < 3; ++a) ext[a] = (double)b.hi[a] - (double)b.lo[a];
    int n[3];
    for (;;) {
        double total = 1.0;
        for (int a = 0; a < 3; ++a) {
            n[a] = (int)std::floor(ext[a] / cs) + 1;
            total *= n[a];
        }
        if (total <= kMaxCells) break;
        cs *= std::cbrt(total / kMaxCells) * 1.01;
    }
    cs_used = cs;
    PGrid g;
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = b.lo[a];
        g.n[a] = n[a];
    }
    g.inv_cs = (float)(1.0 / cs);
    const uint32_t cells = (uint32_t)((size_t)n[0] * n[1] * n[2]);
    uint32_t *cnt = sc.take<uint32_t>(cells);
    uint32_t *start = sc.take<uint32_t>((size_t)cells + 1);
    uint32_t *act = sc.take<uint32_t>(cells);
    const uint32_t nblk = cdiv(cells, scan::kScanBlock);
    uint32_t *blk = sc.take<uint32_t>(2 * (size_t)nblk);
    uint32_t *tot = sc.take<uint32_t>(2);
    uint32_t *cell = sc.take<uint32_t>(npts);
    uint32_t *rank = sc.take<uint32_t>(npts);
    float4 *pts = sc.take<float4>(npts);
    WG_HIP(hipMemsetAsync(cnt, 0, cells * sizeof(uint32_t), st));
    g.start = start;
    g.pts = pts;
    k_pg_count<<<cdiv(npts, 256), 256, 0, st>>>(xyz, npts, g, cell, rank, cnt);
    scan::k_scan_partial<<<nblk, 256, 0, st>>>(cnt, cells, blk);
    scan::k_scan_top<<<1, 256, 0, st>>>(blk, nblk, tot);
    scan::k_scan_final<<<nblk, 256, 0, st>>>(cnt, cells, blk, start, act);
    k_set_word<<<1, 1, 0, st>>>(start + cells, (uint32_t)npts);
    k_pg_scatter<<<cdiv(npts, 256), 256, 0, st>>>(xyz, npts, cell, rank, start, pts);
    WG_LAUNCH_CHECK();
    if (counts) *counts = cnt;
    return g;
}

int dpca(const float *xyz, int npts, double R, double eps, float *nrm, hipStream_t st) {
    require(npts >= 1, WG_EINVAL, "n_points must be >= 1");
    require(xyz && nrm, WG_EINVAL, "null pointer");
    require(R > 0 && std::isfinite(R), WG_EINVAL, "radius must be positive");
    if (!(eps > 0)) eps = 1e-6 * R;
    Scratch sc(st);
    const Box b = cloud_box(xyz, npts, sc, st);
    double cs = 0.0;
    const uint32_t *cnt = nullptr;
    const PGrid g = build_grid(xyz, npts, b, 0.5 * R, sc, st, cs, &cnt);
    // chunks of at most kDpcaChunk points of one cell
    const uint32_t cells = (uint32_t)((size_t)g.n[0] * g.n[1] * g.n[2]);
    uint32_t *ch_cnt = sc.take<uint32_t>(cells), *ch_off = sc.take<uint32_t>(cells), *act = sc.take<uint32_t>(cells);
    const uint32_t nblk = cdiv(cells, scan::kScanBlock);
    uint32_t *blk = sc.take<uint32_t>(2 * (size_t)nblk), *tot = sc.take<uint32_t>(2);
    k_cell_chunks<<<cdiv(cells, 256), 256, 0, st>>>(cnt, cells, kDpcaChunk, ch_cnt);
    scan::k_scan_partial<<<nblk, 256, 0, st>>>(ch_cnt, cells, blk);
    scan::k_scan_top<<<1, 256, 0, st>>>(blk, nblk, tot);
    scan::k_scan_final<<<nblk, 256, 0, st>>>(ch_cnt, cells, blk, ch_off, act);
    WG_LAUNCH_CHECK();
    uint32_t nch = 0;
    WG_HIP(hipMemcpyAsync(&nch, tot, sizeof(nch), hipMemcpyDeviceToHost, st));
    WG_HIP(hipStreamSynchronize(st));
    uint32_t *chunk_cell = sc.take<uint32_t>(nch);
    k_chunk_cells<<<cdiv(cells, 256), 256, 0, st>>>(ch_cnt, ch_off, cells, chunk_cell);
    const float R2 = (float)(R * R);
    k_dpca<<<nch, kDpcaChunk * kDpcaWaves, 0, st>>>(g, chunk_cell, ch_off, R2, (float)b.reach(R), (float)eps, nrm);
    WG_LAUNCH_CHECK();
    WG_HIP(hipStreamSynchronize(st));
    return WG_OK;
}

int orient(const float *xyz, int npts, float *nrm, const wg_orient_opts &o, int32_t *counts, wg_orient_info *info,
           hipStream_t st) {
    require(npts >= 2, WG_EINVAL, "n_points must be >= 2 (the detection radius needs a nearest neighbour)");
    require(xyz && nrm, WG_EINVAL, "null pointer");
    require(o.gamma_r >= 1.0 && std::isfinite(o.gamma_r), WG_EINVAL, "gamma_r must be >= 1 (Eq. 14)");
    require(o.n_tol >= 0, WG_EINVAL, "n_tol must be >= 0");
    require(o.refine == 0 || o.refine == 1, WG_EINVAL, "refine must be 0 or 1");
    Scratch sc(st);
    const Box b = cloud_box(xyz, npts, sc, st);
    {
        int *dbad = sc.take<int>(1), hbad = 0;
        WG_HIP(hipMemsetAsync(dbad, 0, sizeof(int), st));
        k_any_nonfinite<<<std::min<unsigned>(cdiv(3 * (size_t)npts, 256), 256u), 256, 0, st>>>(nrm, 3 * (size_t)npts,
                                                                                             dbad);
        WG_LAUNCH_CHECK();
        WG_HIP(hipMemcpyAsync(&hbad, dbad, sizeof(int), hipMemcpyDeviceToHost, st));
        WG_HIP(hipStreamSynchronize(st));
        require(hbad == 0, WG_ENUMERIC, "a normal is NaN or infinite");
    }
    // nearest spacing on a grid of about two surface spacings per cell (the
    // box's surface area over the point count), rings widen it where sparse
    double ext[3], area = 0.0, diag2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        ext[a] = (double)b.hi[a] - (double)b.lo[a];
        diag2 += ext[a] * ext[a];
    }
    area = 2.0 * (ext[0] * ext[1] + ext[1] * ext[2] + ext[2] * ext[0]);
    double cs_nn = area > 0 ? 2.0 * std::sqrt(area / npts) : std::sqrt(diag2) / std::cbrt((double)npts);
    if (!(cs_nn > 0)) cs_nn = 1.0;   // every point coincides: one cell
    double cs_used = 0.0;
    const PGrid gn = build_grid(xyz, npts, b, cs_nn, sc, st, cs_used);
    uint32_t *dmax = sc.take<uint32_t>(1);
    WG_HIP(hipMemsetAsync(dmax, 0, sizeof(uint32_t), st));
    k_nn_spacing<<<cdiv(npts, 256), 256, 0, st>>>(gn, (float)cs_used, (float)(b.reach(cs_used) - cs_used), npts,
                                                  dmax);
    WG_LAUNCH_CHECK();
    uint32_t bits = 0;
    WG_HIP(hipMemcpyAsync(&bits, dmax, sizeof(bits), hipMemcpyDeviceToHost, st));
    WG_HIP(hipStreamSynchronize(st));
    float d2max;
    std::memcpy(&d2max, &bits, 4);
    require(d2max > 0.0f, WG_EINVAL, "every point has a coincident twin: the detection radius (Eq. 13) is 0");
    // Eq. 13-14 and the probe spacing, in FP64 from the FP32 maximum
    const double rd0 = 0.5 * std::sqrt((double)d2max), rd = o.gamma_r * rd0, ds = 0.75 * rd;
    const double Md = std::ceil((std::sqrt(diag2) + rd) / ds) + 1.0;
    require(Md <= 1e5, WG_EINVAL,
            "more than 1e5 probes per ray: the detection radius is too small for the cloud's extent");
    RayParams rp;
    rp.rd2 = (float)(rd * rd);
    rp.ds = (float)ds;
    rp.reach = (float)b.reach(rd);
    rp.M = (int)Md;
    rp.n_tol = o.n_tol;
    rp.refine = o.refine;
    // cells a little larger than the reach, so that a probe within reach of a point is within one cell of it
    const PGrid go = build_grid(xyz, npts, b, (double)rp.reach * 1.0001, sc, st, cs_used);
    const uint32_t cells = (uint32_t)((size_t)go.n[0] * go.n[1] * go.n[2]);
    const size_t words = ((size_t)cells + 31) / 32;
    uint32_t *occ = sc.take<uint32_t>(words), *near = sc.take<uint32_t>(words);
    WG_HIP(hipMemsetAsync(occ, 0, words * sizeof(uint32_t), st));
    k_mark_occ<<<cdiv(npts, 256), 256, 0, st>>>(xyz, npts, go, occ);
    k_dilate<<<cdiv(cells, 256), 256, 0, st>>>(occ, go, cells, near);
    WG_LAUNCH_CHECK();
    rp.near = near;
    for (int a = 0; a < 3; ++a) {
        rp.box_lo[a] = (float)((double)b.lo[a] - 2.0 * (double)rp.reach);
        rp.box_hi[a] = (float)((double)b.hi[a] + 2.0 * (double)rp.reach);
    }
    uint32_t *nflip = sc.take<uint32_t>(1);
    WG_HIP(hipMemsetAsync(nflip, 0, sizeof(uint32_t), st));
    k_orient<<<cdiv(2 * (size_t)npts, 256), 256, 0, st>>>(go, rp, xyz, npts, nrm, counts, nflip);
    WG_LAUNCH_CHECK();
    uint32_t hflip = 0;
    WG_HIP(hipMemcpyAsync(&hflip, nflip, sizeof(hflip), hipMemcpyDeviceToHost, st));
    WG_HIP(hipStreamSynchronize(st));
    if (info) {
        info->spacing2 = (double)d2max;
        info->rd0 = rd0;
        info->rd = rd;
        info->ds = ds;
        info->n_probes = rp.M;
        info->n_flipped = (int)hflip;
    }
    return WG_OK;
}

template <class F>
int guarded(F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        set_error(e.what());
        return e.code;
    } catch (const std::exception &e) {
        set_error(e.what());
        return WG_EDEVICE;
    } catch (...) {
        set_error("unknown failure");
        return WG_EDEVICE;
    }
}

}  // namespace

}  // namespace wg

extern "C" int wg_dpca_normals(const float *d_xyz, int n_points, double radius, double eps, float *d_nrm_out,
                               void *hip_stream) {
    return wg::guarded([&] { return wg::dpca(d_xyz, n_points, radius, eps, d_nrm_out, (hipStream_t)hip_stream); });
}

extern "C" int wg_orient_normals(const float *d_xyz, int n_points, float *d_nrm, const wg_orient_opts *opts,
                                 int32_t *d_counts, wg_orient_info *info, void *hip_stream) {
    return wg::guarded([&] {
        wg::require(opts != nullptr, WG_EINVAL, "null options");
        return wg::orient(d_xyz, n_points, d_nrm, *opts, d_counts, info, (hipStream_t)hip_stream);
    });
}
