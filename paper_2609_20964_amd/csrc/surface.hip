// Surface extraction, exact signed distance on every grid node, sampling and
// their reverses.  See surface.h for the data layout.
#include <cmath>

#include "mc_table.inc"
#include "prof.h"
#include "surface.h"

namespace wg {

namespace {

constexpr int kBrick = 4;                   // cubes per brick edge (64 = one wavefront)
constexpr int kMaxLevels = 12;
constexpr int kStack = 64;

struct LevelInfo {
    uint32_t off[kMaxLevels];
    uint32_t cnt[kMaxLevels];
    int L;
};

__device__ __forceinline__ uint32_t compact3(uint32_t m) {
    m &= 0x09249249u;
    m = (m ^ (m >> 2)) & 0x030c30c3u;
    m = (m ^ (m >> 4)) & 0x0300f00fu;
    m = (m ^ (m >> 8)) & 0xff0000ffu;
    m = (m ^ (m >> 16)) & 0x000003ffu;
    return m;
}

// Corner bit b = dx + 2 dy + 4 dz.  Edge e: lower corner b0, upper corner b1, axis.
__device__ __forceinline__ void edge_ends(int e, int &b0, int &b1, int &axis) {
    int r = e & 3;
    axis = e >> 2;
    if (axis == 0) b0 = 2 * (r & 1) + 4 * (r >> 1);
    else if (axis == 1) b0 = (r & 1) + 4 * (r >> 1);
    else b0 = (r & 1) + 2 * (r >> 1);
    b1 = b0 + (1 << axis);
}

__device__ __forceinline__ int cube_case(const double *chi, size_t c, size_t sy, size_t sz, double iso) {
    int cs = 0;
    for (int b = 0; b < 8; ++b) {
        size_t o = c + (b & 1) + sy * ((b >> 1) & 1) + sz * (b >> 2);
        cs |= (chi[o] < iso) << b;
    }
    return cs;
}

struct BrickPos {
    int i, j, k;      // cube
    bool ok;
};

__device__ __forceinline__ BrickPos brick_lane(uint32_t m, int lane, const int nb[3], const Dims &d) {
    int bx = compact3(m), by = compact3(m >> 1), bz = compact3(m >> 2);
    BrickPos p;
    p.i = bx * kBrick + (lane & 3);
    p.j = by * kBrick + ((lane >> 2) & 3);
    p.k = bz * kBrick + (lane >> 4);
    p.ok = bx < nb[0] && by < nb[1] && bz < nb[2] && p.i < d.nx - 1 && p.j < d.ny - 1 && p.k < d.nz - 1;
    return p;
}

struct NB {
    int v[3];
};

__global__ __launch_bounds__(256) void k_mc_count(const double *__restrict__ chi, const double *iso, Dims d, NB nb,
                                                   uint32_t nbricks, uint32_t *__restrict__ cnt) {
    const int lane = threadIdx.x % 64;
    const uint32_t m = blockIdx.x * 4 + threadIdx.x / 64;
    if (m >= nbricks) return;   // whole wavefront
    const double c = iso[0];
    BrickPos p = brick_lane(m, lane, nb.v, d);
    int nt = 0;
    if (p.ok) {
        const size_t sy = d.nx, sz = (size_t)d.nx * d.ny;
        nt = WG_MC_NTRI[cube_case(chi, p.i + sy * p.j + sz * p.k, sy, sz, c)];
    }
    for (int o = 32; o > 0; o >>= 1) nt += __shfl_xor(nt, o, 64);
    if (lane == 0) cnt[m] = nt;
}

// Exclusive block scan of (count, nonzero-flag) pairs over 256 threads.
__device__ __forceinline__ void block_scan2(uint32_t a, uint32_t f, uint32_t &ea, uint32_t &ef, uint32_t &ta,
                                            uint32_t &tf) {
    __shared__ uint32_t wa[4], wf[4];
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    uint32_t xa = a, xf = f;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t ya = __shfl_up(xa, o, 64), yf = __shfl_up(xf, o, 64);
        if (lane >= o) {
            xa += ya;
            xf += yf;
        }
    }
    if (lane == 63) {
        wa[w] = xa;
        wf[w] = xf;
    }
    __syncthreads();
    uint32_t pa = 0, pf = 0;
    for (int k = 0; k < w; ++k) {
        pa += wa[k];
        pf += wf[k];
    }
    ta = wa[0] + wa[1] + wa[2] + wa[3];
    tf = wf[0] + wf[1] + wf[2] + wf[3];
    ea = pa + xa - a;
    ef = pf + xf - f;
    __syncthreads();
}

constexpr int kScanPer = 4;      // entries per thread
constexpr int kScanBlock = 256 * kScanPer;

__global__ __launch_bounds__(256) void k_scan_partial(const uint32_t *cnt, uint32_t n, uint32_t *blk) {
    uint32_t a = 0, f = 0;
    for (int q = 0; q < kScanPer; ++q) {
        uint32_t idx = blockIdx.x * kScanBlock + threadIdx.x * kScanPer + q;
        if (idx < n) {
            a += cnt[idx];
            f += cnt[idx] != 0;
        }
    }
    uint32_t ea, ef, ta, tf;
    block_scan2(a, f, ea, ef, ta, tf);
    if (threadIdx.x == 0) {
        blk[2 * blockIdx.x] = ta;
        blk[2 * blockIdx.x + 1] = tf;
    }
}

__global__ __launch_bounds__(256) void k_scan_top(uint32_t *blk, uint32_t nblk, SurfaceCounts *out) {
    uint32_t carry_a = 0, carry_f = 0;
    for (uint32_t base = 0; base < nblk; base += 256) {
        uint32_t idx = base + threadIdx.x;
        uint32_t a = idx < nblk ? blk[2 * idx] : 0, f = idx < nblk ? blk[2 * idx + 1] : 0;
        uint32_t ea, ef, ta, tf;
        block_scan2(a, f, ea, ef, ta, tf);
        if (idx < nblk) {
            blk[2 * idx] = carry_a + ea;
            blk[2 * idx + 1] = carry_f + ef;
        }
        carry_a += ta;
        carry_f += tf;
    }
    if (threadIdx.x == 0) {
        out->n_tris = carry_a;
        out->n_active = carry_f;
    }
}

__global__ __launch_bounds__(256) void k_scan_final(const uint32_t *cnt, uint32_t n, const uint32_t *blk,
                                                     uint32_t *off, uint32_t *active) {
    uint32_t v[kScanPer];
    uint32_t a = 0, f = 0;
    for (int q = 0; q < kScanPer; ++q) {
        uint32_t idx = blockIdx.x * kScanBlock + threadIdx.x * kScanPer + q;
        v[q] = idx < n ? cnt[idx] : 0;
        a += v[q];
        f += v[q] != 0;
    }
    uint32_t ea, ef, ta, tf;
    block_scan2(a, f, ea, ef, ta, tf);
    uint32_t oa = blk[2 * blockIdx.x] + ea, of = blk[2 * blockIdx.x + 1] + ef;
    for (int q = 0; q < kScanPer; ++q) {
        uint32_t idx = blockIdx.x * kScanBlock + threadIdx.x * kScanPer + q;
        if (idx < n) {
            off[idx] = oa;
            if (v[q]) active[of++] = idx;
            oa += v[q];
        }
    }
}

// One wavefront per non-empty brick: triangles of its cubes (vertices by
// Eq. 28 with eta in FP64) and the brick's bounding box (hierarchy leaf).
__global__ __launch_bounds__(256) void k_mc_emit(const double *__restrict__ chi, const double *iso, Dims d, NB nb,
                                                  const uint32_t *__restrict__ active, uint32_t n_active,
                                                  const uint32_t *__restrict__ off, float4 *__restrict__ tri,
                                                  int2 *__restrict__ info, float4 *__restrict__ box) {
    const int lane = threadIdx.x % 64;
    const uint32_t idx = blockIdx.x * 4 + threadIdx.x / 64;
    if (idx >= n_active) return;   // whole wavefront
    const double c = iso[0];
    const uint32_t m = active[idx];
    BrickPos p = brick_lane(m, lane, nb.v, d);
    const size_t sy = d.nx, sz = (size_t)d.nx * d.ny;
    const size_t cell = p.ok ? p.i + sy * p.j + sz * p.k : 0;
    int cs = 0, nt = 0;
    if (p.ok) {
        cs = cube_case(chi, cell, sy, sz, c);
        nt = WG_MC_NTRI[cs];
    }
    int pre = nt;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(pre, o, 64);
        if (lane >= o) pre += y;
    }
    pre -= nt;
    const uint32_t base = off[m] + pre;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int t = 0; t < nt; ++t) {
        int packed = 0;
        for (int q = 0; q < 3; ++q) {
            int e = WG_MC_TRI[cs][3 * t + q];
            packed |= e << (4 * q);
            int b0, b1, ax;
            edge_ends(e, b0, b1, ax);
            double x1 = chi[cell + (b0 & 1) + sy * ((b0 >> 1) & 1) + sz * (b0 >> 2)];
            double x2 = chi[cell + (b1 & 1) + sy * ((b1 >> 1) & 1) + sz * (b1 >> 2)];
            double eta = (c - x1) / (x2 - x1);
            double pos[3] = {(double)(p.i + (b0 & 1)), (double)(p.j + ((b0 >> 1) & 1)), (double)(p.k + (b0 >> 2))};
            pos[ax] += eta;
            float4 v = make_float4((float)pos[0], (float)pos[1], (float)pos[2], 0.f);
            tri[3 * (size_t)(base + t) + q] = v;
            lo[0] = fminf(lo[0], v.x); lo[1] = fminf(lo[1], v.y); lo[2] = fminf(lo[2], v.z);
            hi[0] = fmaxf(hi[0], v.x); hi[1] = fmaxf(hi[1], v.y); hi[2] = fmaxf(hi[2], v.z);
        }
        info[base + t] = make_int2((int)cell, packed);
    }
    for (int o = 32; o > 0; o >>= 1)
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], o, 64));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o, 64));
        }
    if (lane == 0) {
        box[2 * (size_t)idx] = make_float4(lo[0], lo[1], lo[2], 0.f);
        box[2 * (size_t)idx + 1] = make_float4(hi[0], hi[1], hi[2], 0.f);
    }
}

__global__ __launch_bounds__(256) void k_box_level(const float4 *__restrict__ child, uint32_t nchild,
                                                    float4 *__restrict__ parent, uint32_t nparent) {
    uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nparent) return;
    float4 lo = make_float4(INFINITY, INFINITY, INFINITY, 0.f), hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.f);
    uint32_t c1 = min(8 * j + 8, nchild);
    for (uint32_t c = 8 * j; c < c1; ++c) {
        float4 a = child[2 * (size_t)c], b = child[2 * (size_t)c + 1];
        lo.x = fminf(lo.x, a.x); lo.y = fminf(lo.y, a.y); lo.z = fminf(lo.z, a.z);
        hi.x = fmaxf(hi.x, b.x); hi.y = fmaxf(hi.y, b.y); hi.z = fmaxf(hi.z, b.z);
    }
    parent[2 * (size_t)j] = lo;
    parent[2 * (size_t)j + 1] = hi;
}

__device__ __forceinline__ float box_d2(float px, float py, float pz, float4 lo, float4 hi) {
    float dx = fmaxf(fmaxf(lo.x - px, 0.f), px - hi.x);
    float dy = fmaxf(fmaxf(lo.y - py, 0.f), py - hi.y);
    float dz = fmaxf(fmaxf(lo.z - pz, 0.f), pz - hi.z);
    return dx * dx + dy * dy + dz * dz;
}

__device__ __forceinline__ float seg_d2(float3 p, float3 a, float3 b, float &t) {
    float3 ab = make_float3(b.x - a.x, b.y - a.y, b.z - a.z);
    float3 ap = make_float3(p.x - a.x, p.y - a.y, p.z - a.z);
    float l2 = ab.x * ab.x + ab.y * ab.y + ab.z * ab.z;
    t = l2 > 0.f ? (ap.x * ab.x + ap.y * ab.y + ap.z * ab.z) / l2 : 0.f;
    t = fminf(fmaxf(t, 0.f), 1.f);
    float ex = ap.x - t * ab.x, ey = ap.y - t * ab.y, ez = ap.z - t * ab.z;
    return ex * ex + ey * ey + ez * ez;
}

// Closest point of triangle (a,b,c) to p by Voronoi-region classification
// (Ericson, Real-Time Collision Detection, 2005, Sec. 5.1.5), with guards
// for zero-length edges and zero-area triangles.  Returns the squared
// distance; (v, w) are the barycentric weights of b and c at the closest point.
__device__ float tri_d2(float3 p, float3 a, float3 b, float3 c, float &v, float &w) {
    float3 ab = make_float3(b.x - a.x, b.y - a.y, b.z - a.z);
    float3 ac = make_float3(c.x - a.x, c.y - a.y, c.z - a.z);
    float3 ap = make_float3(p.x - a.x, p.y - a.y, p.z - a.z);
    float d1 = ab.x * ap.x + ab.y * ap.y + ab.z * ap.z;
    float d2 = ac.x * ap.x + ac.y * ap.y + ac.z * ap.z;
    float3 bp = make_float3(p.x - b.x, p.y - b.y, p.z - b.z);
    float d3 = ab.x * bp.x + ab.y * bp.y + ab.z * bp.z;
    float d4 = ac.x * bp.x + ac.y * bp.y + ac.z * bp.z;
    float3 cp = make_float3(p.x - c.x, p.y - c.y, p.z - c.z);
    float d5 = ab.x * cp.x + ab.y * cp.y + ab.z * cp.z;
    float d6 = ac.x * cp.x + ac.y * cp.y + ac.z * cp.z;
    float vc = d1 * d4 - d3 * d2;
    float vb = d5 * d2 - d1 * d6;
    float va = d3 * d6 - d5 * d4;
    if (d1 <= 0.f && d2 <= 0.f) { v = 0.f; w = 0.f; }
    else if (d3 >= 0.f && d4 <= d3) { v = 1.f; w = 0.f; }
    else if (vc <= 0.f && d1 >= 0.f && d3 <= 0.f) {
        float den = d1 - d3;
        v = den > 0.f ? d1 / den : 0.f;
        w = 0.f;
    } else if (d6 >= 0.f && d5 <= d6) { v = 0.f; w = 1.f; }
    else if (vb <= 0.f && d2 >= 0.f && d6 <= 0.f) {
        float den = d2 - d6;
        v = 0.f;
        w = den > 0.f ? d2 / den : 0.f;
    } else if (va <= 0.f && (d4 - d3) >= 0.f && (d5 - d6) >= 0.f) {
        float den = (d4 - d3) + (d5 - d6);
        w = den > 0.f ? (d4 - d3) / den : 0.f;
        v = 1.f - w;
    } else {
        float sum = va + vb + vc;
        if (sum > 0.f) {
            v = vb / sum;
            w = vc / sum;
        } else {
            // zero area: nearest of the three edges
            float t0, t1, t2;
            float e0 = seg_d2(p, a, b, t0), e1 = seg_d2(p, b, c, t1), e2 = seg_d2(p, c, a, t2);
            if (e0 <= e1 && e0 <= e2) { v = t0; w = 0.f; }
            else if (e1 <= e2) { v = 1.f - t1; w = t1; }
            else { v = 0.f; w = 1.f - t2; }
        }
    }
    float qx = a.x + v * ab.x + w * ac.x - p.x;
    float qy = a.y + v * ab.y + w * ac.y - p.y;
    float qz = a.z + v * ab.z + w * ac.z - p.z;
    return qx * qx + qy * qy + qz * qz;
}

__device__ __forceinline__ float3 f3(float4 v) { return make_float3(v.x, v.y, v.z); }

__device__ __forceinline__ int cdiv_dev(int n) { return (n + 3) / 4; }

// Exact unsigned distance from every node of a 4x4x4 tile (one wavefront) to
// the mesh, by a wavefront-cooperative walk of the box hierarchy; sign from
// chi >= c (outside positive); phi = sign * distance * h.
__global__ __launch_bounds__(256) void k_sdf(const double *__restrict__ chi, const double *iso, Dims d, double h,
                                              const float4 *__restrict__ box, LevelInfo lev,
                                              const uint32_t *__restrict__ active, const uint32_t *__restrict__ off,
                                              const uint32_t *__restrict__ cnt, const float4 *__restrict__ tri,
                                              uint32_t n_tris, float *__restrict__ phi, int32_t *__restrict__ argmin,
                                              int *err) {
    __shared__ uint32_t stk[4][kStack];
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    const int tx = cdiv_dev(d.nx), ty = cdiv_dev(d.ny), tz = cdiv_dev(d.nz);
    const uint32_t tile = blockIdx.x * 4 + w;
    if (tile >= (uint32_t)(tx * ty * tz)) return;   // whole wavefront
    const int bx = tile % tx, by = (tile / tx) % ty, bz = tile / (tx * ty);
    const int gi = bx * 4 + (lane & 3), gj = by * 4 + ((lane >> 2) & 3), gk = bz * 4 + (lane >> 4);
    const bool valid = gi < d.nx && gj < d.ny && gk < d.nz;
    const int i = min(gi, d.nx - 1), j = min(gj, d.ny - 1), k = min(gk, d.nz - 1);
    const float px = (float)i, py = (float)j, pz = (float)k;
    const float cx = bx * 4 + 1.5f, cy = by * 4 + 1.5f, cz = bz * 4 + 1.5f;
    float best = INFINITY;
    int arg = -1;
    if (n_tris > 0) {
        int sp = 0;
        stk[w][0] = (uint32_t)(lev.L - 1) << 24;
        sp = 1;
        while (sp > 0) {
            --sp;
            const uint32_t ent = __builtin_amdgcn_readfirstlane(stk[w][sp]);
            const int level = ent >> 24;
            const uint32_t idx = ent & 0xffffffu;
            const size_t bi = lev.off[level] + idx;
            const float4 blo = box[2 * bi], bhi = box[2 * bi + 1];
            if (__ballot(box_d2(px, py, pz, blo, bhi) < best) == 0) continue;
            if (level == 0) {
                const uint32_t m = active[idx];
                const uint32_t t0 = off[m], t1 = t0 + cnt[m];
                const float3 p = make_float3(px, py, pz);
                for (uint32_t t = t0; t < t1; ++t) {
                    float v_, w_;
                    float dd = tri_d2(p, f3(tri[3 * (size_t)t]), f3(tri[3 * (size_t)t + 1]), f3(tri[3 * (size_t)t + 2]),
                                      v_, w_);
                    if (dd < best) {
                        best = dd;
                        arg = (int)t;
                    }
                }
            } else {
                const uint32_t c0 = idx * 8;
                const uint32_t nch = min(8u, lev.cnt[level - 1] - c0);
                const uint32_t coff = lev.off[level - 1];
                float key[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    key[q] = -1.f;
                    if ((uint32_t)q < nch) {
                        const size_t ci = coff + c0 + q;
                        const float4 lo = box[2 * ci], hi = box[2 * ci + 1];
                        if (__ballot(box_d2(px, py, pz, lo, hi) < best) != 0) key[q] = box_d2(cx, cy, cz, lo, hi);
                    }
                }
                if (sp + 8 > kStack) {
                    atomicOr(err, 2);
                    continue;
                }
                // push farthest first so the nearest child is popped next
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    int qb = -1;
                    float kb = -0.5f;
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (key[q] > kb) {
                            kb = key[q];
                            qb = q;
                        }
                    if (qb < 0) break;
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (q == qb) key[q] = -1.f;
                    stk[w][sp] = ((uint32_t)(level - 1) << 24) | (c0 + qb);
                    ++sp;
                }
            }
        }
    }
    if (valid) {
        const size_t o = (size_t)i + (size_t)d.nx * (j + (size_t)d.ny * k);
        const float s = chi[o] >= iso[0] ? 1.f : -1.f;
        phi[o] = s * sqrtf(best) * (float)h;
        argmin[o] = arg;
    }
}

// Reverse of phi through the distance (envelope theorem on Eq. 33) and the
// Marching Cubes vertices (Eq. 28): g_chi at the two ends of each vertex's
// edge, g_c in FP64.
__global__ __launch_bounds__(256) void k_sdf_T(const float *__restrict__ gphi, const double *__restrict__ chi,
                                                const double *iso, Dims d, double h, const int32_t *__restrict__ argmin,
                                                const float4 *__restrict__ tri, const int2 *__restrict__ info,
                                                float *__restrict__ g_chi, double *g_c) {
    const size_t n = d.count();
    const size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double gc = 0.0;
    const float g = o < n ? gphi[o] : 0.f;
    const int t = o < n ? argmin[o] : -1;
    if (g != 0.f && t >= 0) {
        const double c = iso[0];
        const int i = o % d.nx, j = (o / d.nx) % d.ny, k = o / ((size_t)d.nx * d.ny);
        const float3 p = make_float3((float)i, (float)j, (float)k);
        const float3 A = f3(tri[3 * (size_t)t]), B = f3(tri[3 * (size_t)t + 1]), C = f3(tri[3 * (size_t)t + 2]);
        float v, w;
        tri_d2(p, A, B, C, v, w);
        float q[3] = {A.x + v * (B.x - A.x) + w * (C.x - A.x), A.y + v * (B.y - A.y) + w * (C.y - A.y),
                      A.z + v * (B.z - A.z) + w * (C.z - A.z)};
        float u[3] = {p.x - q[0], p.y - q[1], p.z - q[2]};
        float dist = sqrtf(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        if (dist > 0.f) {
            const float sgn = chi[o] >= c ? 1.f : -1.f;
            const float gd = sgn * (float)h * g;       // dL / d(distance in grid units)
            const float beta[3] = {1.f - v - w, v, w};
            const int2 inf = info[t];
            const size_t sy = d.nx, sz = (size_t)d.nx * d.ny;
            for (int vq = 0; vq < 3; ++vq) {
                int e = (inf.y >> (4 * vq)) & 15, b0, b1, ax;
                edge_ends(e, b0, b1, ax);
                const float geta = -beta[vq] * (u[ax] / dist) * gd;
                const size_t c1 = (size_t)inf.x + (b0 & 1) + sy * ((b0 >> 1) & 1) + sz * (b0 >> 2);
                const size_t c2 = (size_t)inf.x + (b1 & 1) + sy * ((b1 >> 1) & 1) + sz * (b1 >> 2);
                const double x1 = chi[c1], x2 = chi[c2], D = x2 - x1;
                unsafeAtomicAdd(g_chi + c1, (float)((double)geta * (c - x2) / (D * D)));
                unsafeAtomicAdd(g_chi + c2, (float)(-(double)geta * (c - x1) / (D * D)));
                gc += (double)geta / D;
            }
        }
    }
    gc = wave_sum(gc);
    if (threadIdx.x % 64 == 0 && gc != 0.0) unsafeAtomicAdd(g_c, gc);
}

// Trilinear stencil along one axis for a query (clamped to the node box).
struct Q1 {
    int i0;
    float t;
    bool clamped;
};
__device__ __forceinline__ Q1 q_axis(float x, double lo, double h, int n) {
    double u = ((double)x - lo) / h - 0.5;
    Q1 r;
    r.clamped = !(u >= 0.0 && u <= (double)(n - 1));
    u = fmin(fmax(u, 0.0), (double)(n - 1));
    int i0 = (int)floor(u);
    if (i0 > n - 2) i0 = n - 2;
    r.i0 = i0;
    r.t = (float)(u - (double)i0);
    return r;
}

// Grid gradient of phi at node (i,j,k): central differences, one-sided on the boundary.
__device__ __forceinline__ void node_grad(const float *phi, const Dims &d, int i, int j, int k, float hinv,
                                          float g[3]) {
    const size_t sy = d.nx, sz = (size_t)d.nx * d.ny;
    const size_t o = i + sy * j + sz * k;
    const int c[3] = {i, j, k};
    const int n[3] = {d.nx, d.ny, d.nz};
    const size_t st[3] = {1, sy, sz};
    for (int a = 0; a < 3; ++a) {
        const int up = c[a] + 1 < n[a] ? 1 : 0, dn = c[a] > 0 ? 1 : 0;
        g[a] = (phi[o + up * st[a]] - phi[o - dn * st[a]]) * hinv / (float)(up + dn);
    }
}

__global__ __launch_bounds__(256) void k_sample(GridF g, const float *__restrict__ phi, const float *__restrict__ q,
                                                 int nq, float *__restrict__ out_phi, float *__restrict__ out_nrm) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    Q1 X = q_axis(q[3 * i], g.lo[0], g.h, g.d.nx), Y = q_axis(q[3 * i + 1], g.lo[1], g.h, g.d.ny),
       Z = q_axis(q[3 * i + 2], g.lo[2], g.h, g.d.nz);
    const size_t sy = g.d.nx, sz = (size_t)g.d.nx * g.d.ny;
    const float hinv = (float)(1.0 / g.h);
    float val = 0.f, G[3] = {0.f, 0.f, 0.f};
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const float wgt = (dx ? X.t : 1.f - X.t) * (dy ? Y.t : 1.f - Y.t) * (dz ? Z.t : 1.f - Z.t);
                const int ci = X.i0 + dx, cj = Y.i0 + dy, ck = Z.i0 + dz;
                val += wgt * phi[ci + sy * cj + sz * ck];
                if (out_nrm) {
                    float gc[3];
                    node_grad(phi, g.d, ci, cj, ck, hinv, gc);
                    for (int a = 0; a < 3; ++a) G[a] += wgt * gc[a];
                }
            }
    out_phi[i] = val;
    if (out_nrm) {
        float nn = sqrtf(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
        float inv = nn > 0.f ? 1.f / nn : 0.f;
        for (int a = 0; a < 3; ++a) out_nrm[3 * i + a] = G[a] * inv;
    }
}

// Reverse of k_sample: scatters dL/dphi(q) and dL/dn(q) onto the node field
// (atomics) and writes dL/dq.
__global__ __launch_bounds__(256) void k_sample_T(GridF g, const float *__restrict__ phi, const float *__restrict__ q,
                                                   int nq, const float *__restrict__ gphi_q,
                                                   const float *__restrict__ gnrm_q, float *__restrict__ gphi,
                                                   float *__restrict__ gq) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    Q1 T[3] = {q_axis(q[3 * i], g.lo[0], g.h, g.d.nx), q_axis(q[3 * i + 1], g.lo[1], g.h, g.d.ny),
               q_axis(q[3 * i + 2], g.lo[2], g.h, g.d.nz)};
    const size_t sy = g.d.nx, sz = (size_t)g.d.nx * g.d.ny;
    const size_t st[3] = {1, sy, sz};
    const int n[3] = {g.d.nx, g.d.ny, g.d.nz};
    const float hinv = (float)(1.0 / g.h);
    const float gv = gphi_q[i];
    // forward quantities needed by the normal path
    float G[3] = {0.f, 0.f, 0.f}, gG[3] = {0.f, 0.f, 0.f};
    float gcn[8][3];
    const bool want_n = gnrm_q != nullptr;
    for (int cidx = 0; cidx < 8; ++cidx) {
        const int dx = cidx & 1, dy = (cidx >> 1) & 1, dz = cidx >> 2;
        const float wgt = (dx ? T[0].t : 1.f - T[0].t) * (dy ? T[1].t : 1.f - T[1].t) * (dz ? T[2].t : 1.f - T[2].t);
        if (want_n) {
            node_grad(phi, g.d, T[0].i0 + dx, T[1].i0 + dy, T[2].i0 + dz, hinv, gcn[cidx]);
            for (int a = 0; a < 3; ++a) G[a] += wgt * gcn[cidx][a];
        }
    }
    if (want_n) {
        const float nn = sqrtf(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
        if (nn > 0.f) {
            const float nh[3] = {G[0] / nn, G[1] / nn, G[2] / nn};
            const float gn[3] = {gnrm_q[3 * i], gnrm_q[3 * i + 1], gnrm_q[3 * i + 2]};
            const float dotn = nh[0] * gn[0] + nh[1] * gn[1] + nh[2] * gn[2];
            for (int a = 0; a < 3; ++a) gG[a] = (gn[a] - nh[a] * dotn) / nn;
        }
    }
    float gqv[3] = {0.f, 0.f, 0.f};
    for (int cidx = 0; cidx < 8; ++cidx) {
        const int dd[3] = {cidx & 1, (cidx >> 1) & 1, cidx >> 2};
        float f[3], df[3];
        for (int a = 0; a < 3; ++a) {
            f[a] = dd[a] ? T[a].t : 1.f - T[a].t;
            df[a] = T[a].clamped ? 0.f : (dd[a] ? hinv : -hinv);
        }
        const float wgt = f[0] * f[1] * f[2];
        const int c[3] = {T[0].i0 + dd[0], T[1].i0 + dd[1], T[2].i0 + dd[2]};
        const size_t o = c[0] + sy * c[1] + sz * c[2];
        const float phic = phi[o];
        float s = phic * gv;
        if (want_n) s += gcn[cidx][0] * gG[0] + gcn[cidx][1] * gG[1] + gcn[cidx][2] * gG[2];
        gqv[0] += df[0] * f[1] * f[2] * s;
        gqv[1] += f[0] * df[1] * f[2] * s;
        gqv[2] += f[0] * f[1] * df[2] * s;
        if (gv != 0.f) unsafeAtomicAdd(gphi + o, wgt * gv);
        if (want_n) {
            for (int a = 0; a < 3; ++a) {
                const float gg = wgt * gG[a];
                if (gg == 0.f) continue;
                const int up = c[a] + 1 < n[a] ? 1 : 0, dn = c[a] > 0 ? 1 : 0;
                const float sc = gg * hinv / (float)(up + dn);
                unsafeAtomicAdd(gphi + o + up * st[a], sc);
                unsafeAtomicAdd(gphi + o - dn * st[a], -sc);
            }
        }
    }
    if (gq)
        for (int a = 0; a < 3; ++a) gq[3 * i + a] = gqv[a];
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static void brick_geometry(const Dims &d, int nb[3], int &bits, size_t &pad) {
    nb[0] = (int)cdiv(d.nx - 1, kBrick);
    nb[1] = (int)cdiv(d.ny - 1, kBrick);
    nb[2] = (int)cdiv(d.nz - 1, kBrick);
    int mx = nb[0] > nb[1] ? nb[0] : nb[1];
    mx = mx > nb[2] ? mx : nb[2];
    bits = 0;
    while ((1 << bits) < mx) ++bits;
    pad = (size_t)1 << (3 * bits);
}

void Surface::plan(Arena &a, const Dims &d) {
    int nb[3], bits;
    size_t pad;
    brick_geometry(d, nb, bits, pad);
    for (int k = 0; k < 3; ++k) a.reserve(pad * sizeof(uint32_t));   // counts, offsets, active
    a.reserve(2 * (size_t)cdiv(pad, kScanBlock) * sizeof(uint32_t));
    a.reserve(sizeof(SurfaceCounts));
}

void Surface::bind(Arena &a, const Dims &d, hipStream_t s) {
    st_ = s;
    d_ = d;
    brick_geometry(d, nb_, mbits_, nbricks_pad_);
    require(mbits_ <= 10, WG_EINVAL, "grid too large for the brick index");
    cnt_b_ = a.take<uint32_t>(nbricks_pad_);
    off_b_ = a.take<uint32_t>(nbricks_pad_);
    active_ = a.take<uint32_t>(nbricks_pad_);
    blk_ = a.take<uint32_t>(2 * (size_t)cdiv(nbricks_pad_, kScanBlock));
    dcnt_ = a.take<SurfaceCounts>(1);
    WG_HIP(hipHostMalloc((void **)&hcnt_, sizeof(SurfaceCounts), hipHostMallocDefault));
    // a first guess at the triangle capacity: ~4 per cube over a few slices
    size_t face = (size_t)d.nx * d.ny;
    if ((size_t)d.ny * d.nz > face) face = (size_t)d.ny * d.nz;
    if ((size_t)d.nx * d.nz > face) face = (size_t)d.nx * d.nz;
    ensure_capacity((uint32_t)(4 * face), (uint32_t)(face / 4 + 16));
}

Surface::~Surface() {
    if (tri_) (void)hipFree(tri_);
    if (info_) (void)hipFree(info_);
    if (box_) (void)hipFree(box_);
    if (hcnt_) (void)hipHostFree(hcnt_);
}

void Surface::ensure_capacity(uint32_t tris, uint32_t active) {
    if (tris > cap_) {
        if (tri_) WG_HIP(hipFree(tri_));
        if (info_) WG_HIP(hipFree(info_));
        tri_ = nullptr;
        info_ = nullptr;
        size_t c = (size_t)tris + tris / 4 + 64;
        WG_HIP(hipMalloc(&tri_, c * 3 * sizeof(float4)));
        WG_HIP(hipMalloc(&info_, c * sizeof(int2)));
        cap_ = c;
    }
    // boxes of every level: at most active * 8/7 + levels
    size_t need = (size_t)active + active / 7 + kMaxLevels + 1;
    if (need > box_cap_) {
        if (box_) WG_HIP(hipFree(box_));
        box_ = nullptr;
        size_t c = need + need / 4 + 64;
        WG_HIP(hipMalloc(&box_, c * 2 * sizeof(float4)));
        box_cap_ = c;
    }
}

uint32_t Surface::extract(const double *chi, const double *c) {
    NB nb{{nb_[0], nb_[1], nb_[2]}};
    const uint32_t nbr = (uint32_t)nbricks_pad_;
    prof::Scope ps(WG_PROF_MC, st_, 8.0 * (double)d_.count());
    k_mc_count<<<cdiv(nbr, 4), 256, 0, st_>>>(chi, c, d_, nb, nbr, cnt_b_);
    WG_LAUNCH_CHECK();
    const uint32_t nblk = cdiv(nbr, kScanBlock);
    k_scan_partial<<<nblk, 256, 0, st_>>>(cnt_b_, nbr, blk_);
    k_scan_top<<<1, 256, 0, st_>>>(blk_, nblk, dcnt_);
    k_scan_final<<<nblk, 256, 0, st_>>>(cnt_b_, nbr, blk_, off_b_, active_);
    WG_LAUNCH_CHECK();
    WG_HIP(hipMemcpyAsync(hcnt_, dcnt_, sizeof(SurfaceCounts), hipMemcpyDeviceToHost, st_));
    WG_HIP(hipStreamSynchronize(st_));
    cnt_ = *hcnt_;
    levels_ = 0;
    level_off_.clear();
    level_cnt_.clear();
    if (cnt_.n_tris == 0) return 0;
    ensure_capacity(cnt_.n_tris, cnt_.n_active);
    k_mc_emit<<<cdiv(cnt_.n_active, 4), 256, 0, st_>>>(chi, c, d_, nb, active_, cnt_.n_active, off_b_, tri_, info_,
                                                       box_);
    WG_LAUNCH_CHECK();
    uint32_t n = cnt_.n_active, off = 0;
    level_off_.push_back(0);
    level_cnt_.push_back(n);
    while (n > 1) {
        uint32_t m = (n + 7) / 8;
        uint32_t noff = off + n;
        k_box_level<<<cdiv(m, 256), 256, 0, st_>>>(box_ + 2 * (size_t)off, n, box_ + 2 * (size_t)noff, m);
        WG_LAUNCH_CHECK();
        off = noff;
        n = m;
        level_off_.push_back(off);
        level_cnt_.push_back(n);
    }
    levels_ = (int)level_off_.size();
    require(levels_ <= kMaxLevels, WG_EINVAL, "surface hierarchy too deep");
    return cnt_.n_tris;
}

void Surface::sdf(const double *chi, const double *c, double h, float *phi, int32_t *argmin, int *err) {
    LevelInfo lev{};
    lev.L = levels_;
    for (int l = 0; l < levels_; ++l) {
        lev.off[l] = level_off_[l];
        lev.cnt[l] = level_cnt_[l];
    }
    const uint32_t tiles = cdiv(d_.nx, 4) * cdiv(d_.ny, 4) * cdiv(d_.nz, 4);
    prof::Scope ps(WG_PROF_SDF, st_, (double)d_.count());
    k_sdf<<<cdiv(tiles, 4), 256, 0, st_>>>(chi, c, d_, h, box_, lev, active_, off_b_, cnt_b_, tri_, cnt_.n_tris, phi,
                                           argmin, err);
    WG_LAUNCH_CHECK();
}

void Surface::sdf_T(const float *gphi, const double *chi, const double *c, const int32_t *argmin, double h,
                    float *g_chi, double *g_c) {
    if (cnt_.n_tris == 0) return;
    k_sdf_T<<<cdiv(d_.count(), 256), 256, 0, st_>>>(gphi, chi, c, d_, h, argmin, tri_, info_, g_chi, g_c);
    WG_LAUNCH_CHECK();
}

void launch_sample(const GridF &g, const float *phi, const float *q, int nq, float *out_phi, float *out_nrm,
                   hipStream_t s) {
    if (nq <= 0) return;
    prof::Scope ps(WG_PROF_SAMPLE, s, 28.0 * (double)nq);
    k_sample<<<cdiv(nq, 256), 256, 0, s>>>(g, phi, q, nq, out_phi, out_nrm);
    WG_LAUNCH_CHECK();
}

void launch_sample_T(const GridF &g, const float *phi, const float *q, int nq, const float *gphi_q,
                     const float *gnrm_q, float *gphi, float *gq, hipStream_t s) {
    if (nq <= 0) return;
    k_sample_T<<<cdiv(nq, 256), 256, 0, s>>>(g, phi, q, nq, gphi_q, gnrm_q, gphi, gq);
    WG_LAUNCH_CHECK();
}

}  // namespace wg
