// Surface extraction, exact signed distance on every grid node, sampling and
// their reverses.  See surface.h for the data layout.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "mc_table.inc"
#include "scan.h"
#include "prof.h"
#include "surface.h"

namespace wg {

namespace {

constexpr int kBrick = 4;                   // cubes per brick edge (64 = one wavefront)
constexpr int kMaxLevels = 12;
// Traversal stack of the distance walk (per wavefront).  A pop of an internal
// node at depth l (root 0) finds at most 7 unvisited siblings of it and of each
// ancestor below the root on the stack (7 l entries) and pushes at most 8
// children; internal nodes sit at depths up to kMaxLevels - 2, which extract()
// enforces.  So the stack never holds more than 7 (kMaxLevels - 2) + 8 entries.
constexpr int kStack = 7 * (kMaxLevels - 2) + 8;
constexpr uint32_t kLeaf = 4;               // triangles per hierarchy leaf
constexpr int kNode = 4;                    // float4 per hierarchy node
constexpr int kTri = 4;                     // float4 per triangle record
// packed node word: (count - 1) << 27 | first index (first triangle of a
// leaf, absolute index of the first child node otherwise), bit 30 set on an
// internal node whose children are leaves
constexpr uint32_t kKidsLeaves = 1u << 30;
constexpr uint32_t kLeafEntry = 1u << 31;   // traversal stack entry: the node is a leaf
// The distance walk's tiles are split into kWalkParts z slabs, one work queue
// each; workgroup b starts on slab b % kWalkParts (the XCD it runs on, as
// workgroups are dealt to the 8 XCDs in turn), so each XCD's L2 holds the part
// of the hierarchy near its slab, and moves on to the other slabs' queues when
// its own is empty.
constexpr int kWalkParts = 8;
// Tiles of the walk: a wavefront of 4 x 4 x 4 lanes, each with kWalkKZ nodes
// along z (4 x 4 x 16 nodes) on grids of kSeedMinNodes or more, one node
// (4 x 4 x 4) on smaller ones.  A small grid has few tiles per wavefront
// (8192 at 128^3 against 7168 resident wavefronts), so its walk lasts about
// as long as its slowest tile, and smaller tiles shorten that: 128^3 torus
// 3.33 -> 1.96 ms; 64^3 and 128^3 serving requests -49% and -32% (4 x 4 x 8:
// 2.41 ms, -32%, -23%).
constexpr int kWalkLX = 4, kWalkLY = 4, kWalkLZ = 4, kWalkKZ = 4, kWalkKZSmall = 1;
// Work units a wavefront adds to its tile's cost per stack pop, per internal
// node expanded and per leaf expanded (in proportion to their vector
// instruction counts); the next walk takes each slab's tiles in decreasing
// order of these costs.
constexpr uint32_t kCostPop = 1, kCostInner = 50, kCostLeaf = 75;
constexpr int kCostBuckets = 64;   // two per octave of cost
// Seeds of the walk: the exact nearest triangle of every node of a lattice of
// stride kSeedStride (nodes 0, 8, 16, ... per axis, 32768 at 256^3).  Each
// node's bound starts at its distance to the seed of the lattice node nearest
// to it, which prunes from the first box on.
constexpr int kSeedStride = 8;   // 16 measured 0.8% slower per pipelined step
constexpr int kSeedStack = 64;
// A seed search stops after this many stack entries with the nearest triangle
// found so far (any triangle bounds the distance; the walk stays exact).  The
// search is latency-bound, one lane per lattice node, so its length is the
// pass's time.  Beside the walk, 160, 320 and 1000 measured alike (320 best
// for plain steps, whose next step waits for the search).
constexpr int kSeedPops = 320;
// Run before the walk (a cold walk, which waits for it), a shorter search
// pays: ten cold 256^3 serving shapes walked in 110.5-110.9 ms in total at
// 160 entries, 113.4-113.6 at 320, 113.0 at 80.
constexpr int kSeedPopsFirst = 160;
// Seeds arrive 1-1.5 ms into a walk whatever the grid; they pay only where
// the walk takes several (256^3: 6.8 -> 6.3 ms), so smaller grids walk unseeded.
constexpr size_t kSeedMinNodes = (size_t)1 << 23;
inline int walk_kz(const Dims &d) { return d.count() >= kSeedMinNodes ? kWalkKZ : kWalkKZSmall; }
inline uint32_t walk_tiles(const Dims &d) {
    return cdiv(d.nx, kWalkLX) * cdiv(d.ny, kWalkLY) * cdiv(d.nz, kWalkLZ * walk_kz(d));
}
// A walk with no related walk before it (a new handle, or a cloud unrelated to
// the last) on a grid of kCoopMaxNodes nodes or more orders its tiles by an
// estimate taken from the node sides: the costliest tiles lie deep inside a
// body, where many triangles are at nearly the same distance.  A tile with no
// outside node gets its depth in steps of 4 cells (a tile across x and y;
// 16-cell tiles count four along z) to the nearest tile that has one, by
// kDepthPasses relaxation passes over the tile grid; deeper tiles tie.  Every
// other tile ranks below them by its count of inside nodes.
constexpr int kDepthPasses = 12;
static_assert(kDepthPasses % 2 == 0, "the last pass writes the first buffer");
constexpr uint32_t kTileFull = 0x80000000u;   // flag: no outside node; low 16 bits: depth
constexpr uint32_t kDepthCap = 13;
struct SeedDims {
    int x, y, z;
};
inline SeedDims seed_dims(const Dims &d) {
    return {(int)cdiv(d.nx, kSeedStride), (int)cdiv(d.ny, kSeedStride), (int)cdiv(d.nz, kSeedStride)};
}


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
    // Morton order inside the brick too, so the triangle list is in Morton order of cubes
    p.i = bx * kBrick + (int)compact3((uint32_t)lane);
    p.j = by * kBrick + (int)compact3((uint32_t)lane >> 1);
    p.k = bz * kBrick + (int)compact3((uint32_t)lane >> 2);
    p.ok = bx < nb[0] && by < nb[1] && bz < nb[2] && p.i < d.nx - 1 && p.j < d.ny - 1 && p.k < d.nz - 1;
    return p;
}

struct NB {
    int v[3];
};

// Triangles per brick, from the node sides (k_sign_bits runs first: a corner
// is inside, chi < c, where its side bit is clear).  A wavefront takes a brick
// at a time (grid-stride over bricks): lanes 0..24 each read one row of the
// brick's 5 x 5 x 5 corner nodes (5 consecutive bits), and each lane gathers
// its cube's four rows from them by shuffles.  Reading chi at eight corners
// per lane instead made the kernel bound by cache-line requests.
__global__ __launch_bounds__(256) void k_mc_count(const uint32_t *__restrict__ side, Dims d, NB nb,
                                                   uint32_t nbricks, uint32_t *__restrict__ cnt) {
    constexpr int E = kBrick + 1;
    __shared__ unsigned char ntri[256];   // triangles per cube case
    ntri[threadIdx.x] = WG_MC_NTRI[threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x % 64;
    const size_t n_words = ((size_t)d.count() + 31) / 32;
    // the lane's cube inside a brick (Morton order, as in brick_lane)
    const int dx = (int)compact3((uint32_t)lane), dy = (int)compact3((uint32_t)lane >> 1),
              dz = (int)compact3((uint32_t)lane >> 2);
    const int r0 = dy + E * dz;   // its four corner rows: r0, r0 + 1, r0 + E, r0 + E + 1
    for (uint32_t m = blockIdx.x * 4 + threadIdx.x / 64; m < nbricks; m += gridDim.x * 4) {
        const int bx = (int)compact3(m), by = (int)compact3(m >> 1), bz = (int)compact3(m >> 2);
        uint32_t row = 0;   // bit x: side of node (4 bx + x, row's y, row's z); rows past the grid are clamped
        if (lane < E * E && bx < nb.v[0] && by < nb.v[1] && bz < nb.v[2]) {
            const int gj = min(by * kBrick + lane % E, d.ny - 1), gk = min(bz * kBrick + lane / E, d.nz - 1);
            const size_t o = (size_t)bx * kBrick + (size_t)d.nx * ((size_t)gj + (size_t)d.ny * gk);
            const size_t w = o >> 5;
            const int sh = (int)(o & 31);
            uint64_t v = side[w];
            if (sh + E > 32 && w + 1 < n_words) v |= (uint64_t)side[w + 1] << 32;
            row = (uint32_t)(v >> sh) & ((1u << E) - 1u);
        }
        const uint32_t q00 = __shfl(row, r0, 64), q10 = __shfl(row, r0 + 1, 64);
        const uint32_t q01 = __shfl(row, r0 + E, 64), q11 = __shfl(row, r0 + E + 1, 64);
        const int i = bx * kBrick + dx, j = by * kBrick + dy, k = bz * kBrick + dz;
        const bool ok = bx < nb.v[0] && by < nb.v[1] && bz < nb.v[2] && i < d.nx - 1 && j < d.ny - 1 && k < d.nz - 1;
        int nt = 0;
        if (ok) {
            // corner b = dx' + 2 dy' + 4 dz' is inside where its side bit is clear
            const uint32_t q[4] = {q00, q10, q01, q11};
            int cs = 0;
            for (int b = 0; b < 8; ++b) cs |= (int)(((q[b >> 1] >> (dx + (b & 1))) & 1u) ^ 1u) << b;
            nt = ntri[cs];
        }
        // nt <= 5 (three bits): the wavefront's sum from three ballots
        const uint32_t sum = (uint32_t)__popcll(__ballot(nt & 1)) + 2u * (uint32_t)__popcll(__ballot(nt & 2)) +
                             4u * (uint32_t)__popcll(__ballot(nt & 4));
        if (lane == 0) cnt[m] = sum;
    }
}

// One wavefront per non-empty brick: the triangles of its cubes, vertices by
// Eq. 28 with eta in FP64.  Each triangle is stored ready for the distance
// test: A = (a, |ab|^2), B = (ab, ab.ac), C = (ac, |ac|^2) with ab = b - a,
// ac = c - a in grid units.
__global__ __launch_bounds__(256) void k_mc_emit(const double *__restrict__ chi, const double *iso, Dims d, NB nb,
                                                  const uint32_t *__restrict__ active, uint32_t n_active,
                                                  const uint32_t *__restrict__ off, float4 *__restrict__ tri,
                                                  int2 *__restrict__ info) {
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
    for (int t = 0; t < nt; ++t) {
        int packed = 0;
        double V[3][3];
        for (int q = 0; q < 3; ++q) {
            int e = WG_MC_TRI[cs][3 * t + q];
            packed |= e << (4 * q);
            int b0, b1, ax;
            edge_ends(e, b0, b1, ax);
            double x1 = chi[cell + (b0 & 1) + sy * ((b0 >> 1) & 1) + sz * (b0 >> 2)];
            double x2 = chi[cell + (b1 & 1) + sy * ((b1 >> 1) & 1) + sz * (b1 >> 2)];
            double eta = (c - x1) / (x2 - x1);
            V[q][0] = (double)(p.i + (b0 & 1));
            V[q][1] = (double)(p.j + ((b0 >> 1) & 1));
            V[q][2] = (double)(p.k + (b0 >> 2));
            V[q][ax] += eta;
        }
        float a[3], ab[3], ac[3];
        for (int k = 0; k < 3; ++k) {
            a[k] = (float)V[0][k];
            ab[k] = (float)(V[1][k] - V[0][k]);
            ac[k] = (float)(V[2][k] - V[0][k]);
        }
        {
            // A zero-area triangle (a vertex on a cube corner: chi = c there) is
            // a segment or a point.  Store it as (P, Q, P), P and Q its two
            // vertices farthest apart: with ac = 0 the walk's Voronoi tests
            // give the exact nearest point of PQ (see tri_d2).  The mesh export
            // and the reverse pass rebuild the vertices from chi and the edge
            // ids, so they still see the three Marching Cubes vertices.
            const double cx = (double)ab[1] * ac[2] - (double)ab[2] * ac[1];
            const double cy = (double)ab[2] * ac[0] - (double)ab[0] * ac[2];
            const double cz = (double)ab[0] * ac[1] - (double)ab[1] * ac[0];
            if (cx * cx + cy * cy + cz * cz == 0.0) {
                double l2[3] = {0, 0, 0};   // |ab|^2, |ac|^2, |bc|^2
                for (int k = 0; k < 3; ++k) {
                    l2[0] += (double)ab[k] * ab[k];
                    l2[1] += (double)ac[k] * ac[k];
                    l2[2] += ((double)ac[k] - ab[k]) * ((double)ac[k] - ab[k]);
                }
                for (int k = 0; k < 3; ++k) {
                    if (l2[2] > l2[0] && l2[2] > l2[1]) {   // b -> c
                        a[k] = (float)V[1][k];
                        ab[k] = (float)(V[2][k] - V[1][k]);
                    } else if (l2[1] > l2[0]) {               // a -> c
                        ab[k] = ac[k];
                    }
                    ac[k] = 0.f;
                }
            }
        }
        double aa = 0, bc = 0, cc = 0, ee = 0;
        for (int k = 0; k < 3; ++k) {
            aa += (double)ab[k] * ab[k];
            bc += (double)ab[k] * ac[k];
            cc += (double)ac[k] * ac[k];
            const double e = (double)ac[k] - ab[k];
            ee += e * e;
        }
        const double nx = (double)ab[1] * ac[2] - (double)ab[2] * ac[1];
        const double ny = (double)ab[2] * ac[0] - (double)ab[0] * ac[2];
        const double nz = (double)ab[0] * ac[1] - (double)ab[1] * ac[0];
        const double det = nx * nx + ny * ny + nz * nz;   // |ab x ac|^2 = aa cc - bc^2
        const size_t o = kTri * (size_t)(base + t);
        tri[o] = make_float4(a[0], a[1], a[2], (float)aa);
        tri[o + 1] = make_float4(ab[0], ab[1], ab[2], (float)bc);
        tri[o + 2] = make_float4(ac[0], ac[1], ac[2], (float)cc);
        // a reciprocal that does not fit a finite float marks the length (or area) as zero
        auto rcp = [](double x) { return x > 0 && 1.0 / x < 3.0e38 ? (float)(1.0 / x) : 0.f; };
        tri[o + 3] = make_float4(rcp(aa), rcp(cc), rcp(ee), rcp(det));
        info[base + t] = make_int2((int)cell, packed);
    }
}

// Hierarchy nodes take kNode float4 each.  A leaf (kLeaf consecutive
// triangles) is an oriented box:
//   [0] = (centre, e_u), [1] = (u, e_v), [2] = (v, e_n), [3] = (n, word),
// with (u, v, n) orthonormal, n along the area-weighted normal of its
// triangles, e_* the half extents; where the normals cancel the axes are the
// coordinate axes.  An internal node (up to 8 consecutive children) is an
// axis-aligned box: [0] = (lo, word), [1] = (hi, 0).  Over curved patches of
// many triangles the axis-aligned box is the tighter (and cheaper) bound; over
// a few triangles of one patch the oriented box is.  Extents carry a small
// relative margin so a bound never exceeds the true distance.
__device__ __forceinline__ void frame_from_normal(float nx, float ny, float nz, float *u, float *v, float *n) {
    const float L = sqrtf(nx * nx + ny * ny + nz * nz);
    if (!(L > 1e-12f)) {
        u[0] = 1; u[1] = 0; u[2] = 0; v[0] = 0; v[1] = 1; v[2] = 0; n[0] = 0; n[1] = 0; n[2] = 1;
        return;
    }
    n[0] = nx / L; n[1] = ny / L; n[2] = nz / L;
    // u = normalize(n x e_k), e_k the coordinate axis least aligned with n
    const float ax = fabsf(n[0]), ay = fabsf(n[1]), az = fabsf(n[2]);
    float e[3] = {0, 0, 0};
    e[(ax <= ay && ax <= az) ? 0 : (ay <= az ? 1 : 2)] = 1.f;
    float ux = n[1] * e[2] - n[2] * e[1], uy = n[2] * e[0] - n[0] * e[2], uz = n[0] * e[1] - n[1] * e[0];
    const float lu = sqrtf(ux * ux + uy * uy + uz * uz);
    u[0] = ux / lu; u[1] = uy / lu; u[2] = uz / lu;
    v[0] = n[1] * u[2] - n[2] * u[1]; v[1] = n[2] * u[0] - n[0] * u[2]; v[2] = n[0] * u[1] - n[1] * u[0];
}

__device__ __forceinline__ float box_margin(float m) { return 1e-5f * (1.f + fabsf(m)); }

// Leaves: one thread per group of kLeaf consecutive triangles.  Also writes
// the leaf's axis-aligned box to aabb[2 g], aabb[2 g + 1] for the parents.
__global__ __launch_bounds__(256) void k_leaf_nodes(const float4 *__restrict__ tri, uint32_t n_tris,
                                                     float4 *__restrict__ nodes, float4 *__restrict__ aabb,
                                                     uint32_t n_leaves) {
    uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_leaves) return;
    const uint32_t t0 = g * kLeaf, t1 = min(t0 + kLeaf, n_tris);
    float ns[3] = {0.f, 0.f, 0.f};
    for (uint32_t t = t0; t < t1; ++t) {
        const float4 B = tri[kTri * (size_t)t + 1], C = tri[kTri * (size_t)t + 2];
        ns[0] += B.y * C.z - B.z * C.y;
        ns[1] += B.z * C.x - B.x * C.z;
        ns[2] += B.x * C.y - B.y * C.x;
    }
    float u[3], v[3], n[3];
    frame_from_normal(ns[0], ns[1], ns[2], u, v, n);
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    float alo[3] = {INFINITY, INFINITY, INFINITY}, ahi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t t = t0; t < t1; ++t) {
        const float4 A = tri[kTri * (size_t)t], B = tri[kTri * (size_t)t + 1], C = tri[kTri * (size_t)t + 2];
        const float P[3][3] = {{A.x, A.y, A.z}, {A.x + B.x, A.y + B.y, A.z + B.z}, {A.x + C.x, A.y + C.y, A.z + C.z}};
        for (int q = 0; q < 3; ++q) {
            const float pu = P[q][0] * u[0] + P[q][1] * u[1] + P[q][2] * u[2];
            const float pv = P[q][0] * v[0] + P[q][1] * v[1] + P[q][2] * v[2];
            const float pn = P[q][0] * n[0] + P[q][1] * n[1] + P[q][2] * n[2];
            lo[0] = fminf(lo[0], pu); hi[0] = fmaxf(hi[0], pu);
            lo[1] = fminf(lo[1], pv); hi[1] = fmaxf(hi[1], pv);
            lo[2] = fminf(lo[2], pn); hi[2] = fmaxf(hi[2], pn);
            for (int k = 0; k < 3; ++k) {
                alo[k] = fminf(alo[k], P[q][k]);
                ahi[k] = fmaxf(ahi[k], P[q][k]);
            }
        }
    }
    float c[3], e[3];
    for (int k = 0; k < 3; ++k) {
        const float m = 0.5f * (lo[k] + hi[k]);
        e[k] = 0.5f * (hi[k] - lo[k]) + box_margin(m);
        c[k] = m;
    }
    float4 *nd = nodes + (size_t)kNode * g;
    nd[0] = make_float4(c[0] * u[0] + c[1] * v[0] + c[2] * n[0], c[0] * u[1] + c[1] * v[1] + c[2] * n[1],
                        c[0] * u[2] + c[1] * v[2] + c[2] * n[2], e[0]);
    nd[1] = make_float4(u[0], u[1], u[2], e[1]);
    nd[2] = make_float4(v[0], v[1], v[2], e[2]);
    nd[3] = make_float4(n[0], n[1], n[2], __uint_as_float(((t1 - t0 - 1) << 27) | t0));
    for (int k = 0; k < 3; ++k) {
        alo[k] -= box_margin(alo[k]);
        ahi[k] += box_margin(ahi[k]);
    }
    aabb[2 * (size_t)g] = make_float4(alo[0], alo[1], alo[2], 0.f);
    aabb[2 * (size_t)g + 1] = make_float4(ahi[0], ahi[1], ahi[2], 0.f);
}

// Parents: one thread per parent; its box is the union of its (up to 8)
// children's axis-aligned boxes.  child_first: absolute index of the child
// level's first node; aabb holds every level's boxes at absolute indices.
__global__ __launch_bounds__(256) void k_parent_nodes(float4 *__restrict__ nodes, float4 *__restrict__ aabb,
                                                       uint32_t child_first, uint32_t nchild, uint32_t parent_first,
                                                       uint32_t nparent, uint32_t kids_leaves) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nparent) return;
    const uint32_t c0 = child_first + 8 * j, cnt = min(8u, nchild - 8 * j);
    float4 lo = aabb[2 * (size_t)c0], hi = aabb[2 * (size_t)c0 + 1];
    for (uint32_t q = 1; q < cnt; ++q) {
        const float4 a = aabb[2 * (size_t)(c0 + q)], b = aabb[2 * (size_t)(c0 + q) + 1];
        lo.x = fminf(lo.x, a.x); lo.y = fminf(lo.y, a.y); lo.z = fminf(lo.z, a.z);
        hi.x = fmaxf(hi.x, b.x); hi.y = fmaxf(hi.y, b.y); hi.z = fmaxf(hi.z, b.z);
    }
    const uint32_t p = parent_first + j;
    aabb[2 * (size_t)p] = lo;
    aabb[2 * (size_t)p + 1] = hi;
    float4 *nd = nodes + (size_t)kNode * p;
    nd[0] = make_float4(lo.x, lo.y, lo.z, __uint_as_float(kids_leaves | ((cnt - 1) << 27) | c0));
    nd[1] = make_float4(hi.x, hi.y, hi.z, 0.f);
}

// Mesh export: the three Marching Cubes vertices of each triangle (Eq. 28),
// rebuilt in FP64 from chi and the triangle's cube and edge ids as k_mc_emit
// formed them, as float[9] (the walk's records can hold a zero-area triangle
// as a segment).
__global__ __launch_bounds__(256) void k_export_tris(const double *__restrict__ chi, const double *iso, Dims d,
                                                      const int2 *__restrict__ info, uint32_t n, float *__restrict__ out) {
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double c = iso[0];
    const size_t sy = d.nx, sz = (size_t)d.nx * d.ny;
    const int2 inf = info[t];
    const int ci = inf.x % d.nx, cj = (inf.x / d.nx) % d.ny, ck = inf.x / (int)sz;
    float *o = out + 9 * (size_t)t;
    for (int q = 0; q < 3; ++q) {
        int b0, b1, ax;
        edge_ends((inf.y >> (4 * q)) & 15, b0, b1, ax);
        const double x1 = chi[(size_t)inf.x + (b0 & 1) + sy * ((b0 >> 1) & 1) + sz * (b0 >> 2)];
        const double x2 = chi[(size_t)inf.x + (b1 & 1) + sy * ((b1 >> 1) & 1) + sz * (b1 >> 2)];
        double v[3] = {(double)(ci + (b0 & 1)), (double)(cj + ((b0 >> 1) & 1)), (double)(ck + (b0 >> 2))};
        v[ax] += (c - x1) / (x2 - x1);
        for (int k = 0; k < 3; ++k) o[3 * q + k] = (float)v[k];
    }
}

// Closest point of a triangle to p by Voronoi-region classification (Ericson,
// Real-Time Collision Detection, 2005, Sec. 5.1.5), on the stored record
// A = (a, |ab|^2), B = (ab, ab.ac), C = (ac, |ac|^2),
// R = (1/|ab|^2, 1/|ac|^2, 1/|bc|^2, 1/|ab x ac|^2) (0 where the length is 0).
// With ap = p - a, every dot product of that method follows from d1 = ab.ap
// and d2 = ac.ap, and each of its divisions is by one of the four constants in
// R, so a region costs one or two multiplications.  The regions are tested in
// the method's order (vertices, edges, face interior); neighbouring nodes of a
// wavefront mostly share a region, so the branches rarely diverge.  A
// zero-area triangle is stored as the segment (P, Q, P) (see k_mc_emit): with
// ac = 0, d2 = d4 = d6 = 0 and vc = 0 exactly, so the vertex tests and the ab
// edge test alone decide it, and they give the exact nearest point of PQ.
// Returns the squared distance; (v, w) are the barycentric weights of b and c
// at the closest point.
__device__ __forceinline__ float tri_d2(float px, float py, float pz, float4 A, float4 B, float4 C, float4 R,
                                        float &v, float &w) {
    const float apx = px - A.x, apy = py - A.y, apz = pz - A.z;
    const float d1 = B.x * apx + B.y * apy + B.z * apz;
    const float d2 = C.x * apx + C.y * apy + C.z * apz;
    const float d3 = d1 - A.w, d4 = d2 - B.w;   // against p - b
    const float d5 = d1 - B.w, d6 = d2 - C.w;   // against p - c
    const float vc = d1 * d4 - d3 * d2;
    const float vb = d5 * d2 - d1 * d6;
    const float va = d3 * d6 - d5 * d4;
    if (d1 <= 0.f && d2 <= 0.f) { v = 0.f; w = 0.f; }
    else if (d3 >= 0.f && d4 <= d3) { v = 1.f; w = 0.f; }
    else if (vc <= 0.f && d1 >= 0.f && d3 <= 0.f) { v = d1 * R.x; w = 0.f; }
    else if (d6 >= 0.f && d5 <= d6) { v = 0.f; w = 1.f; }
    else if (vb <= 0.f && d2 >= 0.f && d6 <= 0.f) { v = 0.f; w = d2 * R.y; }
    else if (va <= 0.f && (d4 - d3) >= 0.f && (d5 - d6) >= 0.f) { w = (d4 - d3) * R.z; v = 1.f - w; }
    else { v = vb * R.w; w = vc * R.w; }
    const float qx = apx - v * B.x - w * C.x;
    const float qy = apy - v * B.y - w * C.y;
    const float qz = apz - v * B.z - w * C.z;
    return qx * qx + qy * qy + qz * qz;
}

// Descending compare-exchange of two wave-uniform keys.
__device__ __forceinline__ void cx_desc(uint32_t &a, uint32_t &b) {
    const uint32_t hi = a > b ? a : b, lo = a > b ? b : a;
    a = hi;
    b = lo;
}

// Squared distance bounds of a box for a lane's kTZ nodes (same x, y; z in
// pz): `need` is set if any of them is below that node's best; returns the
// bound of the first node.  Oriented box record (N0..N3) and axis-aligned
// box record (lo in A0, hi in A1).
template <int kTZ>
__device__ __forceinline__ float obb_bound(float4 N0, float4 N1, float4 N2, float4 N3, float px, float py,
                                           const float (&pz)[kTZ], const float (&best)[kTZ], bool &need) {
    const float rx = px - N0.x, ry = py - N0.y;
    const float bu = N1.x * rx + N1.y * ry - N1.z * N0.z, bv = N2.x * rx + N2.y * ry - N2.z * N0.z,
                bn = N3.x * rx + N3.y * ry - N3.z * N0.z;
    float d0 = 0.f;
#pragma unroll
    for (int k = 0; k < kTZ; ++k) {
        const float du = fmaxf(fabsf(bu + N1.z * pz[k]) - N0.w, 0.f);
        const float dv = fmaxf(fabsf(bv + N2.z * pz[k]) - N1.w, 0.f);
        const float dn = fmaxf(fabsf(bn + N3.z * pz[k]) - N2.w, 0.f);
        const float dd = du * du + dv * dv + dn * dn;
        need |= dd < best[k];
        if (k == 0) d0 = dd;
    }
    return d0;
}

// The same oriented-box bound, as a mask: bit k set if node k of the lane is
// below its best.
template <int kTZ>
__device__ __forceinline__ uint32_t obb_layers(float4 N0, float4 N1, float4 N2, float4 N3, float px, float py,
                                               const float (&pz)[kTZ], const float (&best)[kTZ]) {
    const float rx = px - N0.x, ry = py - N0.y;
    const float bu = N1.x * rx + N1.y * ry - N1.z * N0.z, bv = N2.x * rx + N2.y * ry - N2.z * N0.z,
                bn = N3.x * rx + N3.y * ry - N3.z * N0.z;
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < kTZ; ++k) {
        const float du = fmaxf(fabsf(bu + N1.z * pz[k]) - N0.w, 0.f);
        const float dv = fmaxf(fabsf(bv + N2.z * pz[k]) - N1.w, 0.f);
        const float dn = fmaxf(fabsf(bn + N3.z * pz[k]) - N2.w, 0.f);
        if (du * du + dv * dv + dn * dn < best[k]) m |= 1u << k;
    }
    return m;
}

template <int kTZ>
__device__ __forceinline__ float aabb_bound(float4 A0, float4 A1, float px, float py, const float (&pz)[kTZ],
                                            const float (&best)[kTZ], bool &need) {
    const float dx = fmaxf(fmaxf(A0.x - px, px - A1.x), 0.f);
    const float dy = fmaxf(fmaxf(A0.y - py, py - A1.y), 0.f);
    const float dxy = dx * dx + dy * dy;
    float d0 = 0.f;
#pragma unroll
    for (int k = 0; k < kTZ; ++k) {
        const float dz = fmaxf(fmaxf(A0.z - pz[k], pz[k] - A1.z), 0.f);
        const float dd = dz * dz + dxy;
        need |= dd < best[k];
        if (k == 0) d0 = dd;
    }
    return d0;
}

// Squared distance from p to an axis-aligned box (lo, hi in .xyz).
__device__ __forceinline__ float box_d2(float4 lo, float4 hi, float px, float py, float pz) {
    const float dx = fmaxf(fmaxf(lo.x - px, px - hi.x), 0.f);
    const float dy = fmaxf(fmaxf(lo.y - py, py - hi.y), 0.f);
    const float dz = fmaxf(fmaxf(lo.z - pz, pz - hi.z), 0.f);
    return dx * dx + dy * dy + dz * dz;
}

// Levels of the hierarchy as the seed search indexes them: node `local` of
// level l (0 = leaves) is nodes[off[l] + local]; its children are the nodes
// 8 local .. 8 local + 7 of level l - 1 (fewer at the end of a level), and
// leaf L holds triangles kLeaf L .. kLeaf L + kLeaf - 1.
struct SeedLevels {
    uint32_t off[kMaxLevels], cnt[kMaxLevels];
    int levels;
};

// Nearest triangle of each seed-lattice node: one node per lane, each lane
// with its own nearest-first traversal (few nodes, so divergence costs
// little), for at most max_pops stack entries.  A stack entry carries the
// level, the index and the box bound it was pushed with, so a pop that the
// bound rules out touches no memory and every other pop takes one round trip
// (a leaf's triangles, or a node's child boxes).  A stack that would overflow
// drops the children.  Either way the seed is a triangle, only perhaps not
// the nearest: seeds only bound.
__global__ __launch_bounds__(64) void k_sdf_seed(Dims d, SeedDims nc, SeedLevels lv, const float4 *__restrict__ nodes,
                                                  const float4 *__restrict__ leaf_aabb, const float4 *__restrict__ tri,
                                                  uint32_t n_tris, int32_t *__restrict__ seed, int max_pops) {
    __shared__ uint32_t stk[kSeedStack][64];
    __shared__ float stb[kSeedStack][64];
    const int lane = threadIdx.x;
    const int id = blockIdx.x * 64 + lane;
    if (id >= nc.x * nc.y * nc.z) return;
    const float px = (float)min((id % nc.x) * kSeedStride, d.nx - 1);
    const float py = (float)min(((id / nc.x) % nc.y) * kSeedStride, d.ny - 1);
    const float pz = (float)min((id / (nc.x * nc.y)) * kSeedStride, d.nz - 1);
    float best = INFINITY;
    int arg = -1;
    int sp = 0;
    stk[0][lane] = (uint32_t)(lv.levels - 1) << 27;   // the root, local index 0
    stb[0][lane] = 0.f;
    sp = 1;
    for (int pops = 0; sp > 0 && pops < max_pops; ++pops) {
        --sp;
        const uint32_t ent = stk[sp][lane];
        if (stb[sp][lane] >= best) continue;
        const int l = (int)(ent >> 27);
        const uint32_t loc = ent & 0x07ffffffu;
        if (l == 0) {
            const uint32_t t1 = min(loc * kLeaf + kLeaf, n_tris);
            for (uint32_t t = loc * kLeaf; t < t1; ++t) {
                const float4 *tr = tri + kTri * (size_t)t;
                float v_, w_;
                const float dd = tri_d2(px, py, pz, tr[0], tr[1], tr[2], tr[3], v_, w_);
                if (dd < best) {
                    best = dd;
                    arg = (int)t;
                }
            }
            continue;
        }
        const uint32_t c0 = 8 * loc, cc = min(8u, lv.cnt[l - 1] - c0);
        // key: bit 31 = to be visited, then the child's bound (a non-negative
        // float, ordered like its bits; clearing its low 3 bits keeps it a
        // lower bound) with the child's index in the low 3 bits
        uint32_t key[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            key[q] = 0u;
            if ((uint32_t)q < cc) {
                const float4 *cb = l == 1 ? leaf_aabb + 2 * (size_t)(c0 + q)
                                          : nodes + (size_t)kNode * (lv.off[l - 1] + c0 + q);
                const float b = box_d2(cb[0], cb[1], px, py, pz);
                if (b < best) key[q] = 0x80000000u | (__float_as_uint(b) & 0x7ffffff8u) | (uint32_t)q;
            }
        }
        if (sp + 8 > kSeedStack) continue;
        cx_desc(key[0], key[2]); cx_desc(key[1], key[3]); cx_desc(key[4], key[6]); cx_desc(key[5], key[7]);
        cx_desc(key[0], key[4]); cx_desc(key[1], key[5]); cx_desc(key[2], key[6]); cx_desc(key[3], key[7]);
        cx_desc(key[0], key[1]); cx_desc(key[2], key[3]); cx_desc(key[4], key[5]); cx_desc(key[6], key[7]);
        cx_desc(key[2], key[4]); cx_desc(key[3], key[5]);
        cx_desc(key[1], key[4]); cx_desc(key[3], key[6]);
        cx_desc(key[1], key[2]); cx_desc(key[3], key[4]); cx_desc(key[5], key[6]);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (key[r] != 0u) {
                stk[sp][lane] = ((uint32_t)(l - 1) << 27) | (c0 + (key[r] & 7u));
                stb[sp][lane] = __uint_as_float(key[r] & 0x7ffffff8u);
                ++sp;
            }
        }
    }
    __hip_atomic_store(seed + id, arg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Side of every node: bit (o & 31) of word o >> 5 is set where chi >= c
// (outside, Eq. 31: the mesh separates exactly the nodes with chi >= c from
// the others).  One node per lane; a wavefront writes two words.
__global__ __launch_bounds__(256) void k_sign_bits(const double *__restrict__ chi, const double *iso, size_t n,
                                                    uint32_t *__restrict__ sign) {
    const double c = iso[0];
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    // grid-stride in whole wavefronts (stride is a multiple of 64)
    for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o - threadIdx.x % 64 < n; o += stride) {
        const size_t base = o - threadIdx.x % 64;
        const uint64_t bits = __ballot(o < n && chi[o] >= c);
        if (threadIdx.x % 64 == 0) {
            sign[base >> 5] = (uint32_t)bits;
            if (base + 32 < n) sign[(base >> 5) + 1] = (uint32_t)(bits >> 32);
        }
    }
}

// Tile = LX x LY x (LZ * kTZ) nodes: lane (x, y, z) of an LX x LY x LZ block
// owns the kTZ nodes z, z + LZ, ... of its column.
template <int LX, int LY, int LZ, int kTZ>
__global__ __launch_bounds__(256, 8) void k_sdf(const uint32_t *__restrict__ sign, Dims d, double h,
                                              const float4 *__restrict__ nodes, const float4 *__restrict__ leaf_aabb,
                                              uint32_t root,
                                              const float4 *__restrict__ tri, uint32_t n_tris,
                                              float *__restrict__ phi, int32_t *__restrict__ argmin, int *err,
                                              uint32_t *next_tile, const uint32_t *__restrict__ order,
                                              uint32_t *__restrict__ tile_cost, const int32_t *__restrict__ seed,
                                              SeedDims snc, unsigned long long *__restrict__ counts) {
    static_assert(LX * LY * LZ == 64, "one node column per lane");
    __shared__ uint32_t stk[4][kStack];
    // test counts of this wavefront (wave-uniform; a box test applies to its
    // 64 kTZ nodes, a triangle test to one layer of 64), added to counts[] at
    // exit when profiling
    uint32_t n_tri = 0, n_aabb = 0, n_obb = 0, n_tiles = 0, n_seed = 0;
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    constexpr int TZ = LZ * kTZ;
    const int tx = (d.nx + LX - 1) / LX, ty = (d.ny + LY - 1) / LY, tz = (d.nz + TZ - 1) / TZ;
    const uint32_t n_tiles_all = (uint32_t)(tx * ty * tz);
    // persistent: each wavefront takes the next tile of its slab's queue, then
    // of the following slabs', until every queue is empty (each queue is left
    // once it runs dry, so every wavefront exits after at most kWalkParts
    // failed takes)
    int part = (int)(blockIdx.x % kWalkParts), visited = 0;
    for (;;) {
        const uint32_t t0 = (uint32_t)((uint64_t)n_tiles_all * part / kWalkParts);
        const uint32_t t1 = (uint32_t)((uint64_t)n_tiles_all * (part + 1) / kWalkParts);
        uint32_t slot = 0;
        if (lane == 0) slot = t0 + atomicAdd(next_tile + part, 1u);
        slot = __builtin_amdgcn_readfirstlane(slot);
        if (slot >= t1) {   // whole wavefront: this queue is empty
            if (++visited == kWalkParts) break;
            part = (part + 1) % kWalkParts;
            continue;
        }
        // longest tiles (by the previous walk's costs) first, so that the
        // queues end on short ones
        const uint32_t tile = order ? __builtin_amdgcn_readfirstlane(order[slot]) : slot;
        uint32_t work = 0;
        const int bx = tile % tx, by = (tile / tx) % ty, bz = tile / (tx * ty);
        const int gi = bx * LX + lane % LX, gj = by * LY + (lane / LX) % LY, gk0 = bz * TZ + lane / (LX * LY);
        const int i = min(gi, d.nx - 1), j = min(gj, d.ny - 1);
        const float px = (float)i, py = (float)j;
        float pz[kTZ], best[kTZ];
        int arg[kTZ];
#pragma unroll
        for (int k = 0; k < kTZ; ++k) {
            pz[k] = (float)min(gk0 + LZ * k, d.nz - 1);
            best[k] = INFINITY;
            arg[k] = -1;
        }
        if (seed) {
            // start from the distance to the seed of the nearest lattice node
            // (being searched beside this walk: any triangle index bounds)
            const int sa = min((i + kSeedStride / 2) / kSeedStride, snc.x - 1);
            const int sb = min((j + kSeedStride / 2) / kSeedStride, snc.y - 1);
#pragma unroll
            for (int k = 0; k < kTZ; ++k) {
                const int sc = min((min(gk0 + LZ * k, d.nz - 1) + kSeedStride / 2) / kSeedStride, snc.z - 1);
                const int t = __hip_atomic_load(seed + sa + snc.x * (sb + snc.y * sc), __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
                if (t >= 0 && (uint32_t)t < n_tris) {
                    const float4 *tr = tri + kTri * (size_t)t;
                    float v_, w_;
                    best[k] = tri_d2(px, py, pz[k], tr[0], tr[1], tr[2], tr[3], v_, w_);
                    arg[k] = t;
                }
                if (counts) n_seed += (uint32_t)__popcll(__ballot(t >= 0 && (uint32_t)t < n_tris));
            }
        }
        if (n_tris > 0) {
            int sp = 1;
            stk[w][0] = root;
            while (sp > 0) {
                --sp;
                work += kCostPop;
                const uint32_t ent = __builtin_amdgcn_readfirstlane(stk[w][sp]);
                const float4 *nd = nodes + (size_t)kNode * (ent & ~kLeafEntry);
                if (ent & kLeafEntry) {
                    // leaf: recheck its oriented box against the current bests,
                    // then its triangles for the layers of the tile (node k of
                    // every lane: LX x LY x LZ nodes) that some node still
                    // needs; a node whose bound rules the box out cannot gain
                    // from its triangles, so skipping the others is exact
                    const float4 N0 = nd[0], N1 = nd[1], N2 = nd[2], N3 = nd[3];
                    const uint32_t lane_layers = obb_layers<kTZ>(N0, N1, N2, N3, px, py, pz, best);
                    ++n_obb;
                    uint32_t layers = 0;   // wave-uniform
#pragma unroll
                    for (int k = 0; k < kTZ; ++k)
                        if (__ballot((lane_layers >> k) & 1u) != 0) layers |= 1u << k;
                    if (layers == 0) continue;
                    work += kCostLeaf;
                    const uint32_t word = __float_as_uint(N3.w);
                    const uint32_t first = word & 0x07ffffffu, cnt = ((word >> 27) & 7u) + 1;
                    n_tri += cnt * (uint32_t)__popc(layers);
                    for (uint32_t t = first; t < first + cnt; ++t) {
                        const float4 *tr = tri + kTri * (size_t)t;
                        const float4 A = tr[0], B = tr[1], C = tr[2], R = tr[3];
#pragma unroll
                        for (int k = 0; k < kTZ; ++k) {
                            if (!(layers & (1u << k))) continue;
                            float v_, w_;
                            const float dd = tri_d2(px, py, pz[k], A, B, C, R, v_, w_);
                            if (dd < best[k]) {
                                best[k] = dd;
                                arg[k] = (int)t;
                            }
                        }
                    }
                    continue;
                }
                // internal node: recheck its axis-aligned box, then order its children
                const float4 A0 = nd[0], A1 = nd[1];
                {
                    bool need = false;
                    aabb_bound<kTZ>(A0, A1, px, py, pz, best, need);
                    ++n_aabb;
                    if (__ballot(need) == 0) continue;
                }
                work += kCostInner;
                n_aabb += 8;   // the eight child boxes (clamped to the last child)
                const uint32_t word = __float_as_uint(A0.w);
                const uint32_t first = word & 0x07ffffffu, cnt = ((word >> 27) & 7u) + 1;
                const bool kids_leaves = (word & kKidsLeaves) != 0;
                // sort key of a child: bit 31 = to be visited, then the bound of
                // lane 0's first node (a non-negative float, so its bits order
                // like integers) with the child's index in the low 3 bits
                uint32_t key[8];
                if (kids_leaves) {
                    // leaves: their axis-aligned boxes first (cheaper, looser), the
                    // oriented box only for the leaves some lane still needs
                    uint32_t pass = 0;
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        // always a valid leaf (clamped), so all eight loads can be issued together
                        const float4 *ab = leaf_aabb + 2 * (size_t)(first + min((uint32_t)q, cnt - 1));
                        bool vis = false;
                        aabb_bound<kTZ>(ab[0], ab[1], px, py, pz, best, vis);
                        if ((uint32_t)q < cnt && __ballot(vis) != 0) pass |= 1u << q;
                    }
                    n_obb += (uint32_t)__popc(pass);
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        key[q] = 0u;
                        if (pass & (1u << q)) {
                            const float4 *cd = nodes + (size_t)kNode * (first + q);
                            const float4 C0 = cd[0], C1 = cd[1], C2 = cd[2], C3 = cd[3];
                            bool vis = false;
                            const float d0 = obb_bound<kTZ>(C0, C1, C2, C3, px, py, pz, best, vis);
                            const uint32_t kb = __builtin_amdgcn_readfirstlane(__float_as_uint(d0));
                            if (__ballot(vis) != 0) key[q] = 0x80000000u | (kb & 0x7ffffff8u) | q;
                        }
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const float4 *cd = nodes + (size_t)kNode * (first + min((uint32_t)q, cnt - 1));
                        const float4 C0 = cd[0], C1 = cd[1];
                        bool vis = false;
                        const float d0 = aabb_bound<kTZ>(C0, C1, px, py, pz, best, vis);
                        const uint32_t kb = __builtin_amdgcn_readfirstlane(__float_as_uint(d0));
                        key[q] = ((uint32_t)q < cnt && __ballot(vis) != 0) ? (0x80000000u | (kb & 0x7ffffff8u) | q)
                                                                             : 0u;
                    }
                }
                if (sp + 8 > kStack) {   // cannot happen (see kStack); kept as a guard
                    atomicOr(err, 2);
                    continue;
                }
                // 19-comparator sorting network, descending: the farthest child is
                // pushed first so the nearest is popped next
                cx_desc(key[0], key[2]); cx_desc(key[1], key[3]); cx_desc(key[4], key[6]); cx_desc(key[5], key[7]);
                cx_desc(key[0], key[4]); cx_desc(key[1], key[5]); cx_desc(key[2], key[6]); cx_desc(key[3], key[7]);
                cx_desc(key[0], key[1]); cx_desc(key[2], key[3]); cx_desc(key[4], key[5]); cx_desc(key[6], key[7]);
                cx_desc(key[2], key[4]); cx_desc(key[3], key[5]);
                cx_desc(key[1], key[4]); cx_desc(key[3], key[6]);
                cx_desc(key[1], key[2]); cx_desc(key[3], key[4]); cx_desc(key[5], key[6]);
                const uint32_t flag = kids_leaves ? kLeafEntry : 0u;
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    if (key[r] == 0u) break;
                    stk[w][sp] = (first + (key[r] & 7u)) | flag;
                    ++sp;
                }
            }
        }
        if (lane == 0 && tile < n_tiles_all) tile_cost[tile] = work;
        ++n_tiles;
        if (gi < d.nx && gj < d.ny) {
#pragma unroll
            for (int k = 0; k < kTZ; ++k) {
                if (gk0 + LZ * k >= d.nz) break;
                const size_t o = (size_t)i + (size_t)d.nx * (j + (size_t)d.ny * (gk0 + LZ * k));
                const float s = ((sign[o >> 5] >> (o & 31)) & 1u) ? 1.f : -1.f;
                phi[o] = s * sqrtf(best[k]) * (float)h;
                argmin[o] = arg[k];
            }
        }
    }
    if (counts && lane == 0) {
        constexpr unsigned long long kNodes = 64ull * kTZ;
        atomicAdd(counts + 0, 64ull * n_tri + n_seed);
        atomicAdd(counts + 1, kNodes * n_aabb);
        atomicAdd(counts + 2, kNodes * n_obb);
        atomicAdd(counts + 3, kNodes * n_tiles);
    }
}

// Small grids (below kCoopMaxNodes nodes): the four wavefronts of a workgroup
// share one 4x4x4 tile.  Such a grid's walk lasts about as long as its
// slowest tile (a tile deep inside a body, where many triangles lie at nearly
// the same distance), and splitting each tile's hierarchy four ways shortens
// that: 64^3 serving requests walked in 0.41 ms instead of 0.91.  The split
// costs work (each wavefront descends its own part before the others' finds
// prune it), so where tiles outnumber the resident wavefronts it is slower:
// 128^3, 2.64 ms instead of 2.19 (one wavefront per tile, plain order).
//
// Wavefront w walks the nodes w, w + 4, ... of one level of the hierarchy
// (`first`, `n_start` entries, leaves if `leaf_start`); lane l of every
// wavefront stands for node l of the tile.  The nodes' bests meet in LDS as
// (squared distance bits << 32 | triangle) words under atomicMin, so each
// wavefront prunes with the others' finds.  A lane takes a triangle whose
// word is below its best word, and opens every box whose bound is at most
// its best distance (not only below it), so a tie between triangles goes to
// the smallest index whatever the timing.  The start level has at most 120
// nodes (the highest level with 16 or more), so a wavefront starts with at
// most 30 entries on its stack.
constexpr int kCoopStart = 16;
constexpr size_t kCoopMaxNodes = (size_t)1 << 20;
constexpr int kStackCoop = 32 + kStack;
__global__ __launch_bounds__(256, 8) void k_sdf_coop(const uint32_t *__restrict__ sign, Dims d, double h,
                                                   const float4 *__restrict__ nodes,
                                                   const float4 *__restrict__ leaf_aabb, uint32_t first,
                                                   uint32_t n_start, bool leaf_start, const float4 *__restrict__ tri,
                                                   uint32_t n_tris, float *__restrict__ phi,
                                                   int32_t *__restrict__ argmin, int *err, uint32_t *next_tile,
                                                   const uint32_t *__restrict__ order,
                                                   uint32_t *__restrict__ tile_cost,
                                                   unsigned long long *__restrict__ counts) {
    constexpr int LX = kWalkLX, LY = kWalkLY, LZ = kWalkLZ;
    static_assert(LX * LY * LZ == 64, "one node per lane");
    constexpr unsigned long long kNone = 0x7f800000ull << 32 | 0xffffffffull;   // +inf, no triangle
    __shared__ uint32_t stk[4][kStackCoop];
    __shared__ unsigned long long sbest[64];
    __shared__ uint32_t s_slot, s_work;
    uint32_t n_tri = 0, n_aabb = 0, n_obb = 0, n_tiles = 0;
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    const int tx = (d.nx + LX - 1) / LX, ty = (d.ny + LY - 1) / LY, tz = (d.nz + LZ - 1) / LZ;
    const uint32_t n_tiles_all = (uint32_t)(tx * ty * tz);
    int part = (int)(blockIdx.x % kWalkParts), visited = 0;
    for (;;) {
        const uint32_t t0 = (uint32_t)((uint64_t)n_tiles_all * part / kWalkParts);
        const uint32_t t1 = (uint32_t)((uint64_t)n_tiles_all * (part + 1) / kWalkParts);
        __syncthreads();   // every wavefront has read the last slot and the last tile's bests
        if (threadIdx.x == 0) {
            s_slot = t0 + atomicAdd(next_tile + part, 1u);
            s_work = 0;
        }
        if (w == 0) sbest[lane] = kNone;
        __syncthreads();
        const uint32_t slot = __builtin_amdgcn_readfirstlane(s_slot);
        if (slot >= t1) {   // whole workgroup: this queue is empty
            if (++visited == kWalkParts) break;
            part = (part + 1) % kWalkParts;
            continue;
        }
        const uint32_t tile = order ? __builtin_amdgcn_readfirstlane(order[slot]) : slot;
        uint32_t work = 0;
        const int bx = tile % tx, by = (tile / tx) % ty, bz = tile / (tx * ty);
        const int gi = bx * LX + lane % LX, gj = by * LY + (lane / LX) % LY, gk = bz * LZ + lane / (LX * LY);
        const int i = min(gi, d.nx - 1), j = min(gj, d.ny - 1), k = min(gk, d.nz - 1);
        const float px = (float)i, py = (float)j;
        const float pz[1] = {(float)k};
        unsigned long long cur = kNone;   // this lane's best word
        float best[1];                    // the pruning bound: just above cur's distance
        int sp = 0;
        for (uint32_t e = (uint32_t)w; e < n_start; e += 4) stk[w][sp++] = (first + e) | (leaf_start ? kLeafEntry : 0u);
        while (sp > 0) {
            --sp;
            work += kCostPop;
            // the others' finds bound this node too
            cur = min(cur, sbest[lane]);
            {
                const uint32_t db = (uint32_t)(cur >> 32);
                best[0] = db < 0x7f800000u ? __uint_as_float(db + 1u) : INFINITY;
            }
            const uint32_t ent = __builtin_amdgcn_readfirstlane(stk[w][sp]);
            const float4 *nd = nodes + (size_t)kNode * (ent & ~kLeafEntry);
            if (ent & kLeafEntry) {
                const float4 N0 = nd[0], N1 = nd[1], N2 = nd[2], N3 = nd[3];
                ++n_obb;
                if (__ballot(obb_layers<1>(N0, N1, N2, N3, px, py, pz, best) != 0u) == 0) continue;
                work += kCostLeaf;
                const uint32_t word = __float_as_uint(N3.w);
                const uint32_t t_first = word & 0x07ffffffu, cnt = ((word >> 27) & 7u) + 1;
                n_tri += cnt;
                bool found = false;
                for (uint32_t t = t_first; t < t_first + cnt; ++t) {
                    const float4 *tr = tri + kTri * (size_t)t;
                    float v_, w_;
                    const float dd = tri_d2(px, py, pz[0], tr[0], tr[1], tr[2], tr[3], v_, w_);
                    const unsigned long long cand = (unsigned long long)__float_as_uint(dd) << 32 | t;
                    if (cand < cur) {
                        cur = cand;
                        found = true;
                    }
                }
                if (found) atomicMin(sbest + lane, cur);
                continue;
            }
            const float4 A0 = nd[0], A1 = nd[1];
            {
                bool need = false;
                aabb_bound<1>(A0, A1, px, py, pz, best, need);
                ++n_aabb;
                if (__ballot(need) == 0) continue;
            }
            work += kCostInner;
            n_aabb += 8;
            const uint32_t word = __float_as_uint(A0.w);
            const uint32_t c_first = word & 0x07ffffffu, cnt = ((word >> 27) & 7u) + 1;
            const bool kids_leaves = (word & kKidsLeaves) != 0;
            uint32_t key[8];
            if (kids_leaves) {
                uint32_t pass = 0;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const float4 *ab = leaf_aabb + 2 * (size_t)(c_first + min((uint32_t)q, cnt - 1));
                    bool vis = false;
                    aabb_bound<1>(ab[0], ab[1], px, py, pz, best, vis);
                    if ((uint32_t)q < cnt && __ballot(vis) != 0) pass |= 1u << q;
                }
                n_obb += (uint32_t)__popc(pass);
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    key[q] = 0u;
                    if (pass & (1u << q)) {
                        const float4 *cd = nodes + (size_t)kNode * (c_first + q);
                        const float4 C0 = cd[0], C1 = cd[1], C2 = cd[2], C3 = cd[3];
                        bool vis = false;
                        const float d0 = obb_bound<1>(C0, C1, C2, C3, px, py, pz, best, vis);
                        const uint32_t kb = __builtin_amdgcn_readfirstlane(__float_as_uint(d0));
                        if (__ballot(vis) != 0) key[q] = 0x80000000u | (kb & 0x7ffffff8u) | q;
                    }
                }
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const float4 *cd = nodes + (size_t)kNode * (c_first + min((uint32_t)q, cnt - 1));
                    const float4 C0 = cd[0], C1 = cd[1];
                    bool vis = false;
                    const float d0 = aabb_bound<1>(C0, C1, px, py, pz, best, vis);
                    const uint32_t kb = __builtin_amdgcn_readfirstlane(__float_as_uint(d0));
                    key[q] = ((uint32_t)q < cnt && __ballot(vis) != 0) ? (0x80000000u | (kb & 0x7ffffff8u) | q) : 0u;
                }
            }
            if (sp + 8 > kStackCoop) {   // cannot happen (see kStackCoop); kept as a guard
                atomicOr(err, 2);
                continue;
            }
            cx_desc(key[0], key[2]); cx_desc(key[1], key[3]); cx_desc(key[4], key[6]); cx_desc(key[5], key[7]);
            cx_desc(key[0], key[4]); cx_desc(key[1], key[5]); cx_desc(key[2], key[6]); cx_desc(key[3], key[7]);
            cx_desc(key[0], key[1]); cx_desc(key[2], key[3]); cx_desc(key[4], key[5]); cx_desc(key[6], key[7]);
            cx_desc(key[2], key[4]); cx_desc(key[3], key[5]);
            cx_desc(key[1], key[4]); cx_desc(key[3], key[6]);
            cx_desc(key[1], key[2]); cx_desc(key[3], key[4]); cx_desc(key[5], key[6]);
            const uint32_t flag = kids_leaves ? kLeafEntry : 0u;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                if (key[r] == 0u) break;
                stk[w][sp] = (c_first + (key[r] & 7u)) | flag;
                ++sp;
            }
        }
        if (lane == 0) atomicAdd(&s_work, work);
        __syncthreads();   // every wavefront's finds are in sbest
        if (w == 0) {
            if (lane == 0 && tile < n_tiles_all) tile_cost[tile] = s_work;
            ++n_tiles;
            if (gi < d.nx && gj < d.ny && gk < d.nz) {
                const unsigned long long b = sbest[lane];
                const size_t o = (size_t)i + (size_t)d.nx * (j + (size_t)d.ny * k);
                const float s = ((sign[o >> 5] >> (o & 31)) & 1u) ? 1.f : -1.f;
                phi[o] = s * sqrtf(__uint_as_float((uint32_t)(b >> 32))) * (float)h;
                argmin[o] = (int32_t)(uint32_t)b;
            }
        }
    }
    if (counts && lane == 0) {
        atomicAdd(counts + 0, 64ull * n_tri);
        atomicAdd(counts + 1, 64ull * n_aabb);
        atomicAdd(counts + 2, 64ull * n_obb);
        atomicAdd(counts + 3, 64ull * n_tiles);
    }
}

// One workgroup per slab: the slab's tiles in decreasing order of the costs
// the previous walk recorded (a counting sort on two buckets per octave; the
// order inside a bucket is arbitrary, and no result depends on it).
__device__ __forceinline__ int cost_bucket(uint32_t c) {
    if (c == 0) return 0;
    const int e = 31 - __clz(c);
    return 2 * e + (e > 0 ? (int)((c >> (e - 1)) & 1u) : 0);
}

__global__ __launch_bounds__(256) void k_walk_order(const uint32_t *__restrict__ cost, uint32_t n_tiles,
                                                     uint32_t *__restrict__ order) {
    __shared__ uint32_t pos[kCostBuckets];
    const uint32_t p = blockIdx.x;
    const uint32_t t0 = (uint32_t)((uint64_t)n_tiles * p / kWalkParts);
    const uint32_t t1 = (uint32_t)((uint64_t)n_tiles * (p + 1) / kWalkParts);
    if (threadIdx.x < kCostBuckets) pos[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) atomicAdd(&pos[cost_bucket(cost[t])], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {   // exclusive offsets, the costliest bucket first
        uint32_t s = t0;
        for (int b = kCostBuckets - 1; b >= 0; --b) {
            const uint32_t c = pos[b];
            pos[b] = s;
            s += c;
        }
    }
    __syncthreads();
    for (uint32_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) order[atomicAdd(&pos[cost_bucket(cost[t])], 1u)] = t;
}

// One wavefront per tile, lanes as in the walk: kTileFull with an unknown
// depth if no node of the tile is outside, else its count of inside nodes.
template <int KZ>
__global__ __launch_bounds__(256) void k_tile_sides(const uint32_t *__restrict__ side, Dims d,
                                                     uint32_t *__restrict__ out) {
    constexpr int LX = kWalkLX, LY = kWalkLY, LZ = kWalkLZ, TZ = LZ * KZ;
    const int lane = threadIdx.x % 64;
    const int tx = (d.nx + LX - 1) / LX, ty = (d.ny + LY - 1) / LY, tz = (d.nz + TZ - 1) / TZ;
    const uint32_t tile = blockIdx.x * 4 + threadIdx.x / 64;
    if (tile >= (uint32_t)(tx * ty * tz)) return;   // uniform per wavefront
    const int bx = tile % tx, by = (tile / tx) % ty, bz = tile / (tx * ty);
    const int gi = bx * LX + lane % LX, gj = by * LY + (lane / LX) % LY, gk0 = bz * TZ + lane / (LX * LY);
    uint32_t inside = 0, outside = 0;
#pragma unroll
    for (int k = 0; k < KZ; ++k) {
        const int gk = gk0 + LZ * k;
        bool in = false, out_ = false;
        if (gi < d.nx && gj < d.ny && gk < d.nz) {
            const size_t o = (size_t)gi + (size_t)d.nx * (gj + (size_t)d.ny * gk);
            out_ = ((side[o >> 5] >> (o & 31)) & 1u) != 0u;
            in = !out_;
        }
        inside += (uint32_t)__popcll(__ballot(in));
        outside += (uint32_t)__popcll(__ballot(out_));
    }
    if (lane == 0) out[tile] = outside == 0 ? (kTileFull | 0xffffu) : inside;
}

// One relaxation pass of the depths (one thread per tile); tiles beyond the
// grid count as outside.  last: write the sort keys instead, 512 << depth for
// tiles with no outside node (above any inside count), the count otherwise.
template <int KZ>
__global__ __launch_bounds__(256) void k_tile_depth(const uint32_t *__restrict__ in, Dims d, uint32_t *__restrict__ out,
                                                     bool last) {
    const int tx = (d.nx + kWalkLX - 1) / kWalkLX, ty = (d.ny + kWalkLY - 1) / kWalkLY,
              tz = (d.nz + kWalkLZ * KZ - 1) / (kWalkLZ * KZ);
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (uint32_t)(tx * ty * tz)) return;
    uint32_t v = in[t];
    if (v & kTileFull) {
        const int bx = t % tx, by = (t / tx) % ty, bz = t / (tx * ty);
        auto dep = [&](int x, int y, int z) -> uint32_t {
            if (x < 0 || y < 0 || z < 0 || x >= tx || y >= ty || z >= tz) return 0u;
            const uint32_t u = in[(size_t)x + (size_t)tx * (y + (size_t)ty * z)];
            return (u & kTileFull) ? (u & 0xffffu) : 0u;
        };
        uint32_t m = v & 0xffffu;
        m = min(m, dep(bx - 1, by, bz) + 1u);
        m = min(m, dep(bx + 1, by, bz) + 1u);
        m = min(m, dep(bx, by - 1, bz) + 1u);
        m = min(m, dep(bx, by + 1, bz) + 1u);
        m = min(m, dep(bx, by, bz - 1) + (uint32_t)KZ);   // a tile is KZ times as tall as wide
        m = min(m, dep(bx, by, bz + 1) + (uint32_t)KZ);
        v = kTileFull | m;
    }
    if (last) v = (v & kTileFull) ? (512u << min(v & 0xffffu, kDepthCap)) : v;
    out[t] = v;
}

// Closest point to the origin on the triangle (a, b, c) in FP64, by the same
// Voronoi-region method as tri_d2 (Ericson 2005, Sec. 5.1.5) with its
// divisions; a zero-area triangle takes the nearest point of its three edges.
// Returns the barycentric weights (v, w) of b and c.
__device__ void closest_on_tri64(const double (&a)[3], const double (&b)[3], const double (&c)[3], double &v,
                                 double &w) {
    double ab[3], ac[3], ap[3], bp[3], cp[3];
    for (int k = 0; k < 3; ++k) {
        ab[k] = b[k] - a[k];
        ac[k] = c[k] - a[k];
        ap[k] = -a[k];
        bp[k] = -b[k];
        cp[k] = -c[k];
    }
    auto dot = [](const double *x, const double *y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; };
    const double cr[3] = {ab[1] * ac[2] - ab[2] * ac[1], ab[2] * ac[0] - ab[0] * ac[2], ab[0] * ac[1] - ab[1] * ac[0]};
    if (dot(cr, cr) == 0.0) {
        // segment or point: nearest of the edges ab, ac, bc
        double best = INFINITY;
        const double *P[3] = {a, a, b}, *Q[3] = {b, c, c};
        for (int e = 0; e < 3; ++e) {
            double pq[3], pp[3];
            for (int k = 0; k < 3; ++k) {
                pq[k] = Q[e][k] - P[e][k];
                pp[k] = -P[e][k];
            }
            const double l2 = dot(pq, pq);
            const double t = l2 > 0 ? fmin(fmax(dot(pp, pq) / l2, 0.0), 1.0) : 0.0;
            double dd = 0;
            for (int k = 0; k < 3; ++k) dd += (pp[k] - t * pq[k]) * (pp[k] - t * pq[k]);
            if (dd < best) {
                best = dd;
                v = e == 0 ? t : e == 1 ? 0.0 : 1.0 - t;
                w = e == 0 ? 0.0 : t;
            }
        }
        return;
    }
    const double d1 = dot(ab, ap), d2 = dot(ac, ap);
    if (d1 <= 0 && d2 <= 0) { v = 0; w = 0; return; }
    const double d3 = dot(ab, bp), d4 = dot(ac, bp);
    if (d3 >= 0 && d4 <= d3) { v = 1; w = 0; return; }
    const double vc = d1 * d4 - d3 * d2;
    if (vc <= 0 && d1 >= 0 && d3 <= 0) { v = d1 / (d1 - d3); w = 0; return; }
    const double d5 = dot(ab, cp), d6 = dot(ac, cp);
    if (d6 >= 0 && d5 <= d6) { v = 0; w = 1; return; }
    const double vb = d5 * d2 - d1 * d6;
    if (vb <= 0 && d2 >= 0 && d6 <= 0) { v = 0; w = d2 / (d2 - d6); return; }
    const double va = d3 * d6 - d5 * d4;
    if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0) {
        w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        v = 1 - w;
        return;
    }
    const double den = 1.0 / (va + vb + vc);
    v = vb * den;
    w = vc * den;
}

// B2: reverse of the distance through the Marching Cubes vertices.  With p*
// the closest point of the node's nearest triangle (recorded by the walk) and
// beta its barycentric weights, d dist / d v_k = -beta_k (p - p*) / dist; a
// vertex on the edge chi1 -> chi2 along axis a sits at eta = (c - chi1) /
// (chi2 - chi1), so d eta / d chi1 = (c - chi2) / D^2, d eta / d chi2 =
// -(c - chi1) / D^2 and d eta / d c = 1 / D (D = chi2 - chi1).  The vertices
// are rebuilt here in FP64 from chi and the triangle's edge ids, relative to
// the node, as Marching Cubes formed them: the FP32 records the walk reads
// carry absolute grid coordinates (a rounding of up to ~1e-5 cells at 256
// cells per axis), too coarse for the direction (p - p*) / dist at nodes a
// small fraction of a cell from the surface.
__global__ __launch_bounds__(256) void k_sdf_T(const float *__restrict__ gphi, const double *__restrict__ chi,
                                                const double *iso, Dims d, double h, const int32_t *__restrict__ argmin,
                                                const int2 *__restrict__ info, float *__restrict__ g_chi,
                                                double *g_c) {
    const size_t n = d.count();
    const size_t sy = d.nx, sz = (size_t)d.nx * d.ny;
    double gc = 0.0;
    // grid-stride over nodes; the wavefront sums g_c once at the end
    for (size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x; o < n; o += (size_t)gridDim.x * blockDim.x) {
        const float g = gphi[o];
        const int t = argmin[o];
        if (g == 0.f || t < 0) continue;
        const double c = iso[0];
        const int i = o % d.nx, j = (o / d.nx) % d.ny, k = o / sz;
        const int2 inf = info[t];
        const int ci = inf.x % d.nx, cj = (inf.x / d.nx) % d.ny, ck = inf.x / (int)sz;
        double V[3][3], Dq[3];
        size_t C1[3], C2[3];
        int AX[3];
        for (int vq = 0; vq < 3; ++vq) {
            int b0, b1, ax;
            edge_ends((inf.y >> (4 * vq)) & 15, b0, b1, ax);
            C1[vq] = (size_t)inf.x + (b0 & 1) + sy * ((b0 >> 1) & 1) + sz * (b0 >> 2);
            C2[vq] = (size_t)inf.x + (b1 & 1) + sy * ((b1 >> 1) & 1) + sz * (b1 >> 2);
            const double x1 = chi[C1[vq]], x2 = chi[C2[vq]];
            Dq[vq] = x2 - x1;
            AX[vq] = ax;
            V[vq][0] = (double)(ci + (b0 & 1) - i);
            V[vq][1] = (double)(cj + ((b0 >> 1) & 1) - j);
            V[vq][2] = (double)(ck + (b0 >> 2) - k);
            V[vq][ax] += (c - x1) / Dq[vq];
        }
        double v, w;
        closest_on_tri64(V[0], V[1], V[2], v, w);
        const double beta[3] = {1.0 - v - w, v, w};
        // p - p* (p at the origin)
        double u[3], dist = 0.0;
        for (int a = 0; a < 3; ++a) {
            u[a] = -(beta[0] * V[0][a] + beta[1] * V[1][a] + beta[2] * V[2][a]);
            dist += u[a] * u[a];
        }
        dist = sqrt(dist);
        if (!(dist > 0.0)) continue;
        const double sgn = chi[o] >= c ? 1.0 : -1.0;
        const double gd = sgn * h * (double)g;   // dL / d(distance in grid units)
        for (int vq = 0; vq < 3; ++vq) {
            const double geta = -beta[vq] * (u[AX[vq]] / dist) * gd;
            const double x1 = chi[C1[vq]], x2 = chi[C2[vq]], D = Dq[vq];
            unsafeAtomicAdd(g_chi + C1[vq], (float)(geta * (c - x2) / (D * D)));
            unsafeAtomicAdd(g_chi + C2[vq], (float)(-geta * (c - x1) / (D * D)));
            gc += geta / D;
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
    a.reserve(2 * (size_t)cdiv(pad, scan::kScanBlock) * sizeof(uint32_t));
    a.reserve(sizeof(SurfaceCounts));
    a.reserve(cdiv(d.count(), 32) * sizeof(uint32_t));   // node sides
    a.reserve(kWalkParts * sizeof(uint32_t));             // tile counters of the walk
    a.reserve((size_t)walk_tiles(d) * sizeof(uint32_t));   // tile costs of the walk
    a.reserve((size_t)walk_tiles(d) * sizeof(uint32_t));   // tile order of the walk
    const SeedDims sd = seed_dims(d);
    a.reserve((size_t)sd.x * sd.y * sd.z * sizeof(int32_t));   // seeds of the walk
}

void Surface::bind(Arena &a, const Dims &d, hipStream_t s) {
    st_ = s;
    d_ = d;
    brick_geometry(d, nb_, mbits_, nbricks_pad_);
    require(mbits_ <= 10, WG_EINVAL, "grid too large for the brick index");
    cnt_b_ = a.take<uint32_t>(nbricks_pad_);
    off_b_ = a.take<uint32_t>(nbricks_pad_);
    active_ = a.take<uint32_t>(nbricks_pad_);
    blk_ = a.take<uint32_t>(2 * (size_t)cdiv(nbricks_pad_, scan::kScanBlock));
    dcnt_ = a.take<SurfaceCounts>(1);
    sign_ = a.take<uint32_t>(cdiv(d.count(), 32));
    next_tile_ = a.take<uint32_t>(kWalkParts);
    tile_cost_ = a.take<uint32_t>(walk_tiles(d));
    walk_order_ = a.take<uint32_t>(walk_tiles(d));
    {
        const SeedDims sd = seed_dims(d);
        const size_t ns = (size_t)sd.x * sd.y * sd.z;
        seed_ = a.take<int32_t>(ns);
        WG_HIP(hipMemsetAsync(seed_, 0xff, ns * sizeof(int32_t), s));   // -1: no seed before the first search
    }
    have_order_ = false;
    // The persistent walk stays below full residency: its workgroups only
    // retire when the tile queues are empty, and work on the other streams
    // needs free slots meanwhile.  Alone it leaves one workgroup slot per
    // compute unit (the splat, reductions, host read-backs and the seed
    // search fit there).  Beside the next step's solve (pipelined steps) it
    // leaves four, so that one fused V-cycle workgroup (two wavefronts per SIMD
    // of up to 128 VGPRs) fits too: the walk is slower, but the solve no
    // longer waits for it (256^3: 8.2 ms per step against 8.55 with one; two or
    // three free slots are slower than one, five or six much slower; the post
    // pass squeezed to 96 VGPRs to fit beside a five-slot walk spills).
    int dev = 0, cus = 0, per_cu = 0;
    WG_HIP(hipGetDevice(&dev));
    WG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    WG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sdf<4, 4, 4, 4>, 256, 0));
    const unsigned ncu = (unsigned)(cus > 0 ? cus : 256);
    sdf_blocks_full_ = ncu * (unsigned)(per_cu > 1 ? per_cu - 1 : 1);
    sdf_blocks_beside_ = ncu * (unsigned)(per_cu > 4 ? per_cu - 4 : 1);
    hcnt_.alloc();
    ensure_capacity(initial_tris(d));
}

void Surface::set_persistent(bool on) { persistent_ = on; }

Surface::~Surface() {
    if (seed_st_) (void)hipStreamSynchronize(seed_st_);
    if (ev_pre_) (void)hipEventDestroy(ev_pre_);
    if (ev_seed_) (void)hipEventDestroy(ev_seed_);
    if (seed_st_) (void)hipStreamDestroy(seed_st_);
    if (tri_) (void)hipFree(tri_);
    if (info_) (void)hipFree(info_);
    if (box_) (void)hipFree(box_);
    if (aabb_) (void)hipFree(aabb_);
    for (void *p : retired_) (void)hipFree(p);
}

namespace {
// triangle capacity for t triangles (with slack) and hierarchy nodes over them
size_t tri_cap_for(size_t t) { return t + t / 4 + 64; }
size_t box_cap_for(size_t t) {
    const size_t leaves = (t + kLeaf - 1) / kLeaf;
    const size_t need = leaves + leaves / 7 + kMaxLevels + 1;
    return need + need / 4 + 64;
}
}  // namespace

uint32_t Surface::initial_tris(const Dims &d) {
    size_t face = (size_t)d.nx * d.ny;
    if ((size_t)d.ny * d.nz > face) face = (size_t)d.ny * d.nz;
    if ((size_t)d.nx * d.nz > face) face = (size_t)d.nx * d.nz;
    return (uint32_t)(4 * face);
}

size_t Surface::initial_bytes(const Dims &d) {
    const size_t t = initial_tris(d);
    return buf_bytes(tri_cap_for(t), box_cap_for(t));
}

void Surface::ensure_capacity(uint32_t tris) {
    const bool grow_tris = tris > cap_;
    const size_t tcap = grow_tris ? tri_cap_for(tris) : cap_;
    const size_t leaves = ((size_t)tris + kLeaf - 1) / kLeaf;
    const bool grow_boxes = leaves + leaves / 7 + kMaxLevels + 1 > box_cap_;
    const size_t bcap = grow_boxes ? box_cap_for(tris) : box_cap_;
    if (!grow_tris && !grow_boxes) return;
    // a handle's first buffers are part of its footprint; growth is extra
    const size_t extra = buf_bytes(grow_tris ? tcap : 0, grow_boxes ? bcap : 0);
    if (grow_hook_ && (cap_ > 0 || box_cap_ > 0)) grow_hook_(extra);
    auto retire = [&](void *&p, size_t bytes) {
        if (p) {
            retired_.push_back(p);
            retired_bytes_ += bytes;
        }
        p = nullptr;
    };
    if (grow_tris) {
        retire(reinterpret_cast<void *&>(tri_), cap_ * kTri * sizeof(float4));
        retire(reinterpret_cast<void *&>(info_), cap_ * sizeof(int2));
        WG_HIP(hipMalloc(&tri_, tcap * kTri * sizeof(float4)));
        WG_HIP(hipMalloc(&info_, tcap * sizeof(int2)));
        cap_ = tcap;
    }
    if (grow_boxes) {
        retire(reinterpret_cast<void *&>(box_), box_cap_ * kNode * sizeof(float4));
        retire(reinterpret_cast<void *&>(aabb_), box_cap_ * 2 * sizeof(float4));
        WG_HIP(hipMalloc(&box_, bcap * kNode * sizeof(float4)));
        WG_HIP(hipMalloc(&aabb_, bcap * 2 * sizeof(float4)));
        box_cap_ = bcap;
    }
}

uint32_t Surface::extract(const double *chi, const double *c) {
    NB nb{{nb_[0], nb_[1], nb_[2]}};
    const uint32_t nbr = (uint32_t)nbricks_pad_;
    prof::Scope ps(WG_PROF_MC, st_, 8.0 * (double)d_.count());
    // node sides first: the brick counts read them, and so does the distance walk
    const size_t nodes = d_.count();
    k_sign_bits<<<std::min(cdiv(nodes, 256), 8192u), 256, 0, st_>>>(chi, c, nodes, sign_);
    k_mc_count<<<std::min(cdiv(nbr, 4), 16384u), 256, 0, st_>>>(sign_, d_, nb, nbr, cnt_b_);
    WG_LAUNCH_CHECK();
    const uint32_t nblk = cdiv(nbr, scan::kScanBlock);
    scan::k_scan_partial<<<nblk, 256, 0, st_>>>(cnt_b_, nbr, blk_);
    scan::k_scan_top<<<1, 256, 0, st_>>>(blk_, nblk, reinterpret_cast<uint32_t *>(dcnt_));
    scan::k_scan_final<<<nblk, 256, 0, st_>>>(cnt_b_, nbr, blk_, off_b_, active_);
    WG_LAUNCH_CHECK();
    hcnt_.fetch(dcnt_, st_);
    cnt_ = hcnt_.wait();
    levels_ = 0;
    level_off_.clear();
    level_cnt_.clear();
    if (cnt_.n_tris == 0) return 0;
    ensure_capacity(cnt_.n_tris);
    k_mc_emit<<<cdiv(cnt_.n_active, 4), 256, 0, st_>>>(chi, c, d_, nb, active_, cnt_.n_active, off_b_, tri_, info_);
    WG_LAUNCH_CHECK();
    uint32_t n = cdiv(cnt_.n_tris, kLeaf), off = 0;
    k_leaf_nodes<<<cdiv(n, 256), 256, 0, st_>>>(tri_, cnt_.n_tris, box_, aabb_, n);
    WG_LAUNCH_CHECK();
    level_off_.push_back(0);
    level_cnt_.push_back(n);
    while (n > 1) {
        const uint32_t m = (n + 7) / 8;
        const uint32_t noff = off + n;
        k_parent_nodes<<<cdiv(m, 256), 256, 0, st_>>>(box_, aabb_, off, n, noff, m,
                                                       level_off_.size() == 1 ? kKidsLeaves : 0u);
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

template <int LX, int LY, int LZ, int KZ>
static void launch_sdf(const Dims &d, const uint32_t *sign, double h, const float4 *nodes,
                       const float4 *leaf_aabb, uint32_t root, const float4 *tri, uint32_t n_tris, float *phi,
                       int32_t *argmin, int *err, uint32_t *next_tile, const uint32_t *order, uint32_t *tile_cost,
                       const int32_t *seed, unsigned blocks, hipStream_t s) {
    const uint32_t tiles = cdiv(d.nx, LX) * cdiv(d.ny, LY) * cdiv(d.nz, LZ * KZ);
    if (blocks > cdiv(tiles, 4)) blocks = cdiv(tiles, 4);
    WG_HIP(hipMemsetAsync(next_tile, 0, kWalkParts * sizeof(uint32_t), s));
    prof::Scope ps(WG_PROF_SDF, s, (double)d.count());   // the walk alone
    k_sdf<LX, LY, LZ, KZ><<<blocks, 256, 0, s>>>(sign, d, h, nodes, leaf_aabb, root, tri, n_tris, phi, argmin, err,
                                                 next_tile, order, tile_cost, seed, seed_dims(d),
                                                 prof::walk_counters());
    WG_LAUNCH_CHECK();
}

static void launch_sdf_coop(const Dims &d, const uint32_t *sign, double h, const float4 *nodes,
                            const float4 *leaf_aabb, uint32_t first, uint32_t n_start, bool leaf_start,
                            const float4 *tri, uint32_t n_tris, float *phi, int32_t *argmin, int *err,
                            uint32_t *next_tile, const uint32_t *order, uint32_t *tile_cost, unsigned blocks,
                            hipStream_t s) {
    const uint32_t tiles = cdiv(d.nx, kWalkLX) * cdiv(d.ny, kWalkLY) * cdiv(d.nz, kWalkLZ);
    if (blocks > tiles) blocks = tiles;   // a workgroup per tile at a time
    WG_HIP(hipMemsetAsync(next_tile, 0, kWalkParts * sizeof(uint32_t), s));
    prof::Scope ps(WG_PROF_SDF, s, (double)d.count());   // the walk alone
    k_sdf_coop<<<blocks, 256, 0, s>>>(sign, d, h, nodes, leaf_aabb, first, n_start, leaf_start, tri, n_tris, phi,
                                      argmin, err, next_tile, order, tile_cost, prof::walk_counters());
    WG_LAUNCH_CHECK();
}

void Surface::sdf(double h, float *phi, int32_t *argmin, int *err, hipStream_t s, bool beside, bool related) {
    const unsigned blocks = !persistent_ ? ~0u : beside ? sdf_blocks_beside_ : sdf_blocks_full_;
    // Tile order: the last walk's costs when that walk was of a related
    // surface; from kCoopMaxNodes nodes up otherwise the estimate from the
    // node sides (the walk_order_ buffer holds the alternate relaxation passes).
    const bool cold = d_.count() >= kCoopMaxNodes && (!related || !have_order_);
    if (cold) {
        const uint32_t nt = walk_tiles(d_);
        const bool tall = walk_kz(d_) == kWalkKZ;
        if (tall) k_tile_sides<kWalkKZ><<<cdiv(nt, 4), 256, 0, s>>>(sign_, d_, tile_cost_);
        else k_tile_sides<kWalkKZSmall><<<cdiv(nt, 4), 256, 0, s>>>(sign_, d_, tile_cost_);
        for (int p = 0; p < kDepthPasses; ++p) {
            const bool even = p % 2 == 0;
            uint32_t *src = even ? tile_cost_ : walk_order_, *dst = even ? walk_order_ : tile_cost_;
            if (tall) k_tile_depth<kWalkKZ><<<cdiv(nt, 256), 256, 0, s>>>(src, d_, dst, p == kDepthPasses - 1);
            else k_tile_depth<kWalkKZSmall><<<cdiv(nt, 256), 256, 0, s>>>(src, d_, dst, p == kDepthPasses - 1);
        }
        k_walk_order<<<kWalkParts, 256, 0, s>>>(tile_cost_, nt, walk_order_);
        WG_LAUNCH_CHECK();
        have_order_ = true;
    }
    // a one-level hierarchy is a single leaf
    const uint32_t root = levels_ > 1 ? level_off_[levels_ - 1] : kLeafEntry;
    // Seeds: after a related walk, searched on a stream of their own beside
    // the walk; the walk reads each seed when it starts the tile that needs
    // it, so early tiles see the previous walk's seed.  After an unrelated
    // surface (cold) those would bound nothing useful, so the search runs
    // first, on the walk's stream.  The walk takes an index below n_tris as a
    // triangle, which bounds whichever triangle it is, and ignores others (-1
    // on a new handle).
    const bool seeded = cnt_.n_tris > 0 && d_.count() >= kSeedMinNodes;
    if (seeded) {
        if (!seed_st_) {
            WG_HIP(hipStreamCreateWithFlags(&seed_st_, hipStreamNonBlocking));
            WG_HIP(hipEventCreateWithFlags(&ev_pre_, hipEventDisableTiming));
            WG_HIP(hipEventCreateWithFlags(&ev_seed_, hipEventDisableTiming));
        }
        SeedLevels lv{};
        lv.levels = levels_;
        for (int l = 0; l < levels_; ++l) {
            lv.off[l] = level_off_[l];
            lv.cnt[l] = level_cnt_[l];
        }
        const SeedDims snc = seed_dims(d_);
        const unsigned ns = (unsigned)(snc.x * snc.y * snc.z);
        hipStream_t ss = cold ? s : seed_st_;
        if (!cold) {
            WG_HIP(hipEventRecord(ev_pre_, s));
            WG_HIP(hipStreamWaitEvent(seed_st_, ev_pre_, 0));
        }
        k_sdf_seed<<<cdiv(ns, 64), 64, 0, ss>>>(d_, snc, lv, box_, aabb_, tri_, cnt_.n_tris, seed_,
                                                cold ? kSeedPopsFirst : kSeedPops);
        WG_LAUNCH_CHECK();
        WG_HIP(hipEventRecord(ev_seed_, ss));
    }
    // a wavefront takes 4x4x4 columns of 4 nodes along z (a 4x4x16 tile) on a
    // large grid, 4x4x4 nodes on a mid-sized one; on a small one a workgroup's
    // four wavefronts share 4x4x4 nodes
    const uint32_t *order = have_order_ ? walk_order_ : nullptr;
    if (walk_kz(d_) == kWalkKZ) {
        launch_sdf<kWalkLX, kWalkLY, kWalkLZ, kWalkKZ>(d_, sign_, h, box_, aabb_, root, tri_, cnt_.n_tris, phi, argmin,
                                                      err, next_tile_, order, tile_cost_, seeded ? seed_ : nullptr,
                                                      blocks, s);
    } else if (d_.count() >= kCoopMaxNodes) {   // no seeds below kSeedMinNodes
        launch_sdf<kWalkLX, kWalkLY, kWalkLZ, kWalkKZSmall>(d_, sign_, h, box_, aabb_, root, tri_, cnt_.n_tris, phi,
                                                           argmin, err, next_tile_, order, tile_cost_, nullptr,
                                                           blocks, s);
    } else {
        // start level: the highest one with kCoopStart nodes or more (else the leaves)
        int l0 = 0;
        for (int l = levels_ - 1; l > 0; --l)
            if (level_cnt_[l] >= (uint32_t)kCoopStart) {
                l0 = l;
                break;
            }
        const uint32_t n_start = cnt_.n_tris > 0 ? level_cnt_[l0] : 0u;
        const uint32_t first = cnt_.n_tris > 0 ? level_off_[l0] : 0u;
        require(n_start <= 4u * (kStackCoop - kStack), WG_EINVAL, "distance walk: start level too wide");
        launch_sdf_coop(d_, sign_, h, box_, aabb_, first, n_start, l0 == 0, tri_, cnt_.n_tris, phi, argmin, err,
                        next_tile_, order, tile_cost_, blocks, s);
    }
    // the seed search reads the hierarchy the next extraction rewrites: order
    // the walk's stream (which the next extraction waits for) after it
    if (seeded) WG_HIP(hipStreamWaitEvent(s, ev_seed_, 0));
    // the next walk's order, from this walk's costs (off the critical path of
    // a pipelined step: it runs beside the next step's solve)
    k_walk_order<<<kWalkParts, 256, 0, s>>>(tile_cost_, walk_tiles(d_), walk_order_);
    WG_LAUNCH_CHECK();
    have_order_ = true;   // ordered by the costs of the walk just launched
}

void Surface::sdf_T(const float *gphi, const double *chi, const double *c, const int32_t *argmin, double h,
                    float *g_chi, double *g_c) {
    if (cnt_.n_tris == 0) return;
    k_sdf_T<<<std::min(cdiv(d_.count(), 256), 8192u), 256, 0, st_>>>(gphi, chi, c, d_, h, argmin, info_, g_chi, g_c);
    WG_LAUNCH_CHECK();
}

void Surface::export_tris(const double *chi, const double *c, float *out, uint32_t n) {
    if (n == 0) return;
    k_export_tris<<<cdiv(n, 256), 256, 0, st_>>>(chi, c, d_, info_, n, out);
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
