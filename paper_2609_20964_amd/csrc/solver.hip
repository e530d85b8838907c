// Matrix-free multigrid-preconditioned CG for the grid Poisson problem.
//
// The single-operator sweeps (the CG direction update with A, the FP64
// residual) are 2.5-D: a wavefront takes rows of float4 columns and marches
// z planes, keeping the z-1, z, z+1 values in registers and reading x/y
// neighbours through the caches; x is the fastest (coalesced) axis.  Each
// V-cycle level is two fused passes that stage haloed tiles in LDS (see
// k_vc_pre / k_vc_post).  Blocks are remapped so that each XCD sweeps one
// contiguous slab.
// Every reduction is two-stage and deterministic: one FP64 partial per block
// (fixed block order), summed by a single-block finalize kernel.
#include <atomic>
#include <cmath>

#include "prof.h"
#include "solver.h"

namespace wg {

namespace {

constexpr int TX = 64, TY = 4, ZC = 16;
constexpr int kRedBlocks = 2048;     // grid of the pointwise reductions
constexpr int kMaxRed = 5;
constexpr float kOmega = 6.0f / 7.0f;   // weighted-Jacobi factor of the sweeps on an odd-sized coarsest level
constexpr int kCoarseTarget = 32;       // coarsen until every extent is <= this (or odd)
// Exact coarsest solve when every extent is <= kDirectAxis; a grid whose every
// extent is that small is solved on one level, the exact solve being the whole
// preconditioner (64^3 serving requests: about one inner iteration per
// refinement instead of three to four V-cycled ones).
constexpr int kDirectAxis = 64;

// An inner PCG enqueues its next iteration before the host has seen whether
// the current one stopped it; once a finalize has set the flag, the kernels of
// that iteration return at once (skip: null outside an inner solve).
__device__ __forceinline__ bool skipped(const int *skip) { return skip != nullptr && *skip != 0; }

struct Tiles {
    unsigned gx, gy, gz;
    __host__ __device__ unsigned count() const { return gx * gy * gz; }
};
Tiles tiles_of(const Dims &d) { return {cdiv(d.nx, TX), cdiv(d.ny, TY), cdiv(d.nz, ZC)}; }

// Generic 7-point sweep.  Op::load(idx) yields the stencil input at a linear
// index; Op::apply(idx, centre, neighbour_sum, diag, acc) consumes one cell.
// Scalars an operator reads from device memory once per workgroup (none by default).
template <class Op> __device__ __forceinline__ void fetch_scalars(Op &) {}

template <class Op>
__global__ __launch_bounds__(256) void k_stencil(Op op, Dims d, Tiles t, double *partials, const int *skip) {
    using T = typename Op::T;
    if (skipped(skip)) return;
    fetch_scalars(op);
    const unsigned nb = t.count();
    const unsigned lb = xcd_logical_block(blockIdx.x, nb);
    const unsigned bx = lb % t.gx, by = (lb / t.gx) % t.gy, bz = lb / (t.gx * t.gy);
    const int i = bx * TX + threadIdx.x % TX;
    const int j = by * TY + threadIdx.x / TX;
    const int z0 = bz * ZC;
    double acc[Op::NRED > 0 ? Op::NRED : 1];
    for (int k = 0; k < (Op::NRED > 0 ? Op::NRED : 1); ++k) acc[k] = 0.0;
    if (i < d.nx && j < d.ny) {
        const size_t plane = (size_t)d.nx * d.ny;
        const size_t base = (size_t)i + (size_t)d.nx * j;
        const int z1 = min(z0 + ZC, d.nz);
        const bool xm = i > 0, xp = i + 1 < d.nx, ym = j > 0, yp = j + 1 < d.ny;
        const int nb_xy = (!xm) + (!xp) + (!ym) + (!yp);
        T cm = z0 > 0 ? op.load(base + (size_t)(z0 - 1) * plane) : T(0);
        T cc = op.load(base + (size_t)z0 * plane);
        for (int k = z0; k < z1; ++k) {
            const size_t idx = base + (size_t)k * plane;
            const bool zp = k + 1 < d.nz;
            T cp = zp ? op.load(idx + plane) : T(0);
            T s = T(0);
            if (xm) s += op.load(idx - 1);
            if (xp) s += op.load(idx + 1);
            if (ym) s += op.load(idx - d.nx);
            if (yp) s += op.load(idx + d.nx);
            if (k > 0) s += cm;
            s += cp;
            const int nbf = nb_xy + (k == 0) + (!zp);
            const T diag = T(6 + d.bc_sign * nbf);
            op.apply(idx, cc, s, diag, acc);
            cm = cc;
            cc = cp;
        }
    }
    if constexpr (Op::NRED > 0) {
        __shared__ double lds[4][Op::NRED];
        block_sum<Op::NRED>(acc, lds);
        if (threadIdx.x == 0)
            for (int k = 0; k < Op::NRED; ++k) partials[(size_t)k * nb + lb] = acc[k];
    }
}

// Four consecutive x cells per lane (x extent divisible by 4).  A wavefront
// covers R rows x L float4 columns (L = min(64, nx/4), R = 64/L) and marches
// ZC planes in z; x neighbours inside the wavefront come from lane shuffles,
// the two ends of a row segment load theirs.  One 16-byte load per field and
// plane per lane keeps the sweep at streaming bandwidth.
template <class T>
struct V4 {
    T v[4];
};

template <class T>
__device__ __forceinline__ V4<T> ld4(const T *p) {
    V4<T> r;
    if constexpr (sizeof(T) == 4) {
        const float4 q = *reinterpret_cast<const float4 *>(p);
        r.v[0] = q.x; r.v[1] = q.y; r.v[2] = q.z; r.v[3] = q.w;
    } else {
        const double2 a = *reinterpret_cast<const double2 *>(p), b = *reinterpret_cast<const double2 *>(p + 2);
        r.v[0] = a.x; r.v[1] = a.y; r.v[2] = b.x; r.v[3] = b.y;
    }
    return r;
}
__device__ __forceinline__ void st4(float *p, const V4<float> &r) {
    *reinterpret_cast<float4 *>(p) = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
}

struct Waves4 {
    unsigned L, R, S, G, gz, zlen;   // lanes per row segment, rows per wave, segments per row,
                                     // row groups, z chunks, planes per chunk
    __host__ __device__ unsigned tasks() const { return S * G * gz; }
};
// z-march length: as long as possible (fewer halo planes) while keeping at
// least kTasks wavefront tasks; `even` keeps chunk starts even.
constexpr unsigned kTasks = 4096;
inline void set_zlen(Waves4 &w, int nz, bool even = false) {
    unsigned cols = w.S * w.G;
    unsigned z = (unsigned)(((size_t)nz * cols) / kTasks);
    z = z < 1 ? 1 : (z > (unsigned)ZC ? (unsigned)ZC : z);
    if (even) z = z < 2 ? 2 : (z & ~1u);
    w.zlen = z;
    w.gz = cdiv(nz, z);
}
inline Waves4 waves4_of(const Dims &d, bool even = false) {
    Waves4 w;
    const unsigned W4 = (unsigned)d.nx / 4;
    w.L = W4 < 64 ? W4 : 64;
    w.R = 64 / w.L;
    w.S = (W4 + w.L - 1) / w.L;
    w.G = ((unsigned)d.ny + w.R - 1) / w.R;
    set_zlen(w, d.nz, even);
    return w;
}

template <class Op>
__global__ __launch_bounds__(256) void k_stencil4(Op op, Dims d, Waves4 wv, double *partials, const int *skip) {
    using T = typename Op::T;
    if (skipped(skip)) return;
    fetch_scalars(op);
    const unsigned nb = gridDim.x;
    const unsigned lb = xcd_logical_block(blockIdx.x, nb);
    const unsigned task = lb * 4 + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    double acc[Op::NRED > 0 ? Op::NRED : 1];
    for (int k = 0; k < (Op::NRED > 0 ? Op::NRED : 1); ++k) acc[k] = 0.0;
    const unsigned W4 = (unsigned)d.nx / 4;
    const unsigned seg = task % wv.S, grp = (task / wv.S) % wv.G, zc = task / (wv.S * wv.G);
    const unsigned sl = lane % wv.L, rr = lane / wv.L;
    const unsigned x4 = seg * wv.L + sl;
    const int j = (int)(grp * wv.R + rr);
    const bool valid = task < wv.tasks() && rr < wv.R && x4 < W4 && j < d.ny;
    const int z0 = (int)(zc * wv.zlen);
    if (task < wv.tasks()) {
        const int i = 4 * (int)(valid ? x4 : 0);
        const int jj = valid ? j : 0;
        const size_t plane = (size_t)d.nx * d.ny;
        const size_t base = (size_t)i + (size_t)d.nx * jj;
        const int z1 = min(z0 + (int)wv.zlen, d.nz);
        const bool ym = jj > 0, yp = jj + 1 < d.ny;
        const bool xl = i > 0, xr = i + 4 < d.nx;                 // neighbours exist
        const bool shl = sl > 0, shr = sl + 1 < wv.L && x4 + 1 < W4; // ... and sit in the next lane
        const int nb_y = (!ym) + (!yp);
        // rows j-1 (a) and j+1 (b) of a plane are fetched with its row j, one
        // plane ahead of their use, when the neighbouring wavefronts fetch them
        // as their own rows
        V4<T> cm, cc, a, b;
        for (int q = 0; q < 4; ++q) cm.v[q] = cc.v[q] = a.v[q] = b.v[q] = T(0);
        if (valid && z0 > 0) cm = op.load4(base + (size_t)(z0 - 1) * plane);
        if (valid) cc = op.load4(base + (size_t)z0 * plane);
        if (valid && ym) a = op.load4(base + (size_t)z0 * plane - d.nx);
        if (valid && yp) b = op.load4(base + (size_t)z0 * plane + d.nx);
        for (int k = z0; k < z1; ++k) {
            const size_t idx = base + (size_t)k * plane;
            const bool zp = k + 1 < d.nz;
            V4<T> cp, ap, bp;
            for (int q = 0; q < 4; ++q) cp.v[q] = ap.v[q] = bp.v[q] = T(0);
            if (valid && zp) cp = op.load4(idx + plane);
            if (valid && zp && ym) ap = op.load4(idx + plane - d.nx);
            if (valid && zp && yp) bp = op.load4(idx + plane + d.nx);
            T left = __shfl_up(cc.v[3], 1, 64), right = __shfl_down(cc.v[0], 1, 64);
            if (!shl) left = (valid && xl) ? op.load1(idx - 1) : T(0);
            if (!shr) right = (valid && xr) ? op.load1(idx + 4) : T(0);
            if (!xl) left = T(0);
            if (!xr) right = T(0);
            if (valid) {
                const int nbc = nb_y + (k == 0) + (!zp);
                V4<T> s, dg;
                for (int q = 0; q < 4; ++q) {
                    s.v[q] = a.v[q] + b.v[q] + cm.v[q] + cp.v[q];
                    dg.v[q] = T(6 + d.bc_sign * nbc);
                }
                s.v[0] += left + cc.v[1];
                s.v[1] += cc.v[0] + cc.v[2];
                s.v[2] += cc.v[1] + cc.v[3];
                s.v[3] += cc.v[2] + right;
                if (!xl) dg.v[0] += T(d.bc_sign);
                if (!xr) dg.v[3] += T(d.bc_sign);
                op.apply4(idx, cc, s, dg, acc);
            }
            cm = cc;
            cc = cp;
            a = ap;
            b = bp;
        }
    }
    if constexpr (Op::NRED > 0) {
        __shared__ double lds[4][Op::NRED];
        block_sum<Op::NRED>(acc, lds);
        if (threadIdx.x == 0)
            for (int k = 0; k < Op::NRED; ++k) partials[(size_t)k * nb + lb] = acc[k];
    }
}

// 27-point sweep of the exact-quadrature stiffness (Eq. 21 integrated exactly
// for trilinear tents mirrored across the outer faces):
//   A = k (x) m (x) m + m (x) k (x) m + m (x) m (x) k,
// with m = (1, 4, 1)/6 and k = (-1, 2, -1) along each axis and indices clamped
// to the grid (Neumann only).  A wavefront holds 64 consecutive x cells of one
// row (x neighbours by lane shuffles, the row ends load theirs), a workgroup
// four rows, and each marches ZC planes in z.  Per plane it forms the in-plane
// filters Q = m_x m_y u and P = (k_x m_y + m_x k_y) u and keeps three planes;
// plane z's output is sum_dz m(dz) P(z + dz) + k(dz) Q(z + dz), z + dz clamped.
// Op::applyA(idx, centre, A u, acc) consumes one cell.
template <class Op>
__global__ __launch_bounds__(256) void k_stencil27(Op op, Dims d, Tiles t, double *partials, const int *skip) {
    using T = typename Op::T;
    if (skipped(skip)) return;
    fetch_scalars(op);
    const unsigned nb = t.count();
    const unsigned lb = xcd_logical_block(blockIdx.x, nb);
    const unsigned bx = lb % t.gx, by = (lb / t.gx) % t.gy, bz = lb / (t.gx * t.gy);
    const int lane = threadIdx.x % TX;
    const int i = bx * TX + lane;
    const int j = by * TY + threadIdx.x / TX;   // one row per wavefront
    const int z0 = bz * ZC;
    double acc[Op::NRED > 0 ? Op::NRED : 1];
    for (int k = 0; k < (Op::NRED > 0 ? Op::NRED : 1); ++k) acc[k] = 0.0;
    if (j < d.ny) {   // uniform over the wavefront
        const size_t plane = (size_t)d.nx * d.ny;
        const int ic = min(i, d.nx - 1);   // lanes past the row end shadow its last cell
        const size_t rows[3] = {(size_t)max(j - 1, 0) * d.nx, (size_t)j * d.nx, (size_t)min(j + 1, d.ny - 1) * d.nx};
        const T sixth = T(1) / T(6);
        // in-plane filters of plane z: P, Q and the centre value
        auto filt = [&](int z, T &P, T &Q, T &C) {
            T mx[3], kx[3];
            for (int r = 0; r < 3; ++r) {
                const size_t base = (size_t)z * plane + rows[r];
                const T c = op.load(base + ic);
                T l = __shfl_up(c, 1, 64), rr = __shfl_down(c, 1, 64);
                if (lane == 0) l = op.load(base + max(ic - 1, 0));
                if (lane == TX - 1 || i + 1 >= d.nx) rr = i + 1 < d.nx ? op.load(base + i + 1) : c;
                mx[r] = (l + T(4) * c + rr) * sixth;
                kx[r] = T(2) * c - l - rr;
                if (r == 1) C = c;
            }
            Q = (mx[0] + T(4) * mx[1] + mx[2]) * sixth;
            P = (kx[0] + T(4) * kx[1] + kx[2]) * sixth + (T(2) * mx[1] - mx[0] - mx[2]);
        };
        const int z1 = min(z0 + ZC, d.nz);
        T Pm, Qm, Cm, Pc, Qc, Cc;
        filt(max(z0 - 1, 0), Pm, Qm, Cm);
        filt(z0, Pc, Qc, Cc);
        for (int k = z0; k < z1; ++k) {
            T Pp, Qp, Cp;
            filt(min(k + 1, d.nz - 1), Pp, Qp, Cp);
            const T au = (Pm + T(4) * Pc + Pp) * sixth + (T(2) * Qc - Qm - Qp);
            if (i < d.nx) op.applyA(rows[1] + (size_t)i + (size_t)k * plane, Cc, au, acc);
            Pm = Pc; Qm = Qc; Cm = Cc;
            Pc = Pp; Qc = Qp; Cc = Cp;
        }
    }
    if constexpr (Op::NRED > 0) {
        __shared__ double lds[4][Op::NRED];
        block_sum<Op::NRED>(acc, lds);
        if (threadIdx.x == 0)
            for (int k = 0; k < Op::NRED; ++k) partials[(size_t)k * nb + lb] = acc[k];
    }
}

// The same 27-point sweep with four consecutive x cells per lane (x extent
// divisible by 4), in the wavefront layout of k_stencil4: a lane loads one
// 16-byte vector per row and plane, the x neighbours inside it are its own,
// those of the two ends come from the next lanes (or a load at a row
// segment's end).  Op::applyA4(idx, centres, A u, acc) consumes four cells.
template <class Op>
__global__ __launch_bounds__(256) void k_stencil27x4(Op op, Dims d, Waves4 wv, double *partials, const int *skip) {
    using T = typename Op::T;
    if (skipped(skip)) return;
    fetch_scalars(op);
    const unsigned nb = gridDim.x;
    const unsigned lb = xcd_logical_block(blockIdx.x, nb);
    const unsigned task = lb * 4 + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    double acc[Op::NRED > 0 ? Op::NRED : 1];
    for (int k = 0; k < (Op::NRED > 0 ? Op::NRED : 1); ++k) acc[k] = 0.0;
    const unsigned W4 = (unsigned)d.nx / 4;
    const unsigned seg = task % wv.S, grp = (task / wv.S) % wv.G, zc = task / (wv.S * wv.G);
    const unsigned sl = lane % wv.L, rr = lane / wv.L;
    const unsigned x4 = seg * wv.L + sl;
    const int j = (int)(grp * wv.R + rr);
    const bool valid = task < wv.tasks() && rr < wv.R && x4 < W4 && j < d.ny;
    if (task < wv.tasks()) {   // uniform over the wavefront
        const int i = 4 * (int)(valid ? x4 : 0);
        const int jj = valid ? j : 0;
        const size_t plane = (size_t)d.nx * d.ny;
        const size_t rows[3] = {(size_t)max(jj - 1, 0) * d.nx, (size_t)jj * d.nx,
                                (size_t)min(jj + 1, d.ny - 1) * d.nx};
        const bool xl = i > 0, xr = i + 4 < d.nx;                    // neighbours exist
        const bool shl = sl > 0, shr = sl + 1 < wv.L && x4 + 1 < W4;  // ... and sit in the next lane
        const T sixth = T(1) / T(6);
        auto filt = [&](int z, V4<T> &P, V4<T> &Q, V4<T> &C) {
            V4<T> mx[3], kx[3];
            for (int r = 0; r < 3; ++r) {
                const size_t base = (size_t)z * plane + rows[r] + i;
                V4<T> c;
                if (valid) c = op.load4(base);
                else for (int q = 0; q < 4; ++q) c.v[q] = T(0);
                T left = __shfl_up(c.v[3], 1, 64), right = __shfl_down(c.v[0], 1, 64);
                if (!shl) left = (valid && xl) ? op.load1(base - 1) : c.v[0];
                if (!shr) right = (valid && xr) ? op.load1(base + 4) : c.v[3];
                if (!xl) left = c.v[0];    // clamped: the mirror image of the first cell
                if (!xr) right = c.v[3];
                for (int q = 0; q < 4; ++q) {
                    const T l = q == 0 ? left : c.v[q - 1], rt = q == 3 ? right : c.v[q + 1];
                    mx[r].v[q] = (l + T(4) * c.v[q] + rt) * sixth;
                    kx[r].v[q] = T(2) * c.v[q] - l - rt;
                }
                if (r == 1) C = c;
            }
            for (int q = 0; q < 4; ++q) {
                Q.v[q] = (mx[0].v[q] + T(4) * mx[1].v[q] + mx[2].v[q]) * sixth;
                P.v[q] = (kx[0].v[q] + T(4) * kx[1].v[q] + kx[2].v[q]) * sixth +
                         (T(2) * mx[1].v[q] - mx[0].v[q] - mx[2].v[q]);
            }
        };
        const int z0 = (int)(zc * wv.zlen);
        const int z1 = min(z0 + (int)wv.zlen, d.nz);
        V4<T> Pm, Qm, Cm, Pc, Qc, Cc;
        filt(max(z0 - 1, 0), Pm, Qm, Cm);
        filt(z0, Pc, Qc, Cc);
        for (int k = z0; k < z1; ++k) {
            V4<T> Pp, Qp, Cp, au;
            filt(min(k + 1, d.nz - 1), Pp, Qp, Cp);
            for (int q = 0; q < 4; ++q)
                au.v[q] = (Pm.v[q] + T(4) * Pc.v[q] + Pp.v[q]) * sixth + (T(2) * Qc.v[q] - Qm.v[q] - Qp.v[q]);
            if (valid) op.applyA4(rows[1] + (size_t)i + (size_t)k * plane, Cc, au, acc);
            Pm = Pc; Qm = Qc; Cm = Cc;
            Pc = Pp; Qc = Qp; Cc = Cp;
        }
    }
    if constexpr (Op::NRED > 0) {
        __shared__ double lds[4][Op::NRED];
        block_sum<Op::NRED>(acc, lds);
        if (threadIdx.x == 0)
            for (int k = 0; k < Op::NRED; ++k) partials[(size_t)k * nb + lb] = acc[k];
    }
}

// r = (b - mb) - A x in FP64 (r stored FP32); sums of r, r^2, x, b - mb,
// (b - mb)^2.  mb is the mean of b for zero-flux boundaries (the compatibility
// projection of the right-hand side), 0 otherwise.
template <class TB>
struct OpResid64 {
    using T = double;
    static constexpr int NRED = 5;
    const double *x;
    const TB *b;   // the right-hand side, FP32 or FP64
    float *r;
    const SolveScalars *sc;   // mean of b formed on the device (Neumann), or null (no shift)
    double mb;
    __device__ double load(size_t i) const { return x[i]; }
    __device__ double load1(size_t i) const { return x[i]; }
    __device__ V4<double> load4(size_t i) const { return ld4(x + i); }
    __device__ void apply(size_t i, double c, double s, double diag, double *acc) const {
        double bv = (double)b[i] - mb;
        double rv = bv - (diag * c - s);
        r[i] = (float)rv;
        acc[0] += rv;
        acc[1] += rv * rv;
        acc[2] += c;
        acc[3] += bv;
        acc[4] += bv * bv;
    }
    __device__ void apply4(size_t i, const V4<double> &c, const V4<double> &s, const V4<double> &dg,
                           double *acc) const {
        const V4<TB> bb = ld4(b + i);
        V4<float> out;
        for (int q = 0; q < 4; ++q) {
            const double bv = (double)bb.v[q] - mb;
            const double rv = bv - (dg.v[q] * c.v[q] - s.v[q]);
            out.v[q] = (float)rv;
            acc[0] += rv;
            acc[1] += rv * rv;
            acc[2] += c.v[q];
            acc[3] += bv;
            acc[4] += bv * bv;
        }
        st4(r + i, out);
    }
    __device__ void applyA(size_t i, double c, double au, double *acc) const {
        const double bv = (double)b[i] - mb;
        const double rv = bv - au;
        r[i] = (float)rv;
        acc[0] += rv;
        acc[1] += rv * rv;
        acc[2] += c;
        acc[3] += bv;
        acc[4] += bv * bv;
    }
    __device__ void applyA4(size_t i, const V4<double> &c, const V4<double> &au, double *acc) const {
        const V4<TB> bb = ld4(b + i);
        V4<float> out;
        for (int q = 0; q < 4; ++q) {
            const double bv = (double)bb.v[q] - mb;
            const double rv = bv - au.v[q];
            out.v[q] = (float)rv;
            acc[0] += rv;
            acc[1] += rv * rv;
            acc[2] += c.v[q];
            acc[3] += bv;
            acc[4] += bv * bv;
        }
        st4(r + i, out);
    }
};

// First weighted-Jacobi sweep from a zero guess: x = w rhs / diag.
struct OpSmoothFirst {
    using T = float;
    static constexpr int NRED = 0;
    const float *rhs;
    float *out;
    float w;
    __device__ float load(size_t) const { return 0.f; }
    __device__ float load1(size_t) const { return 0.f; }
    __device__ V4<float> load4(size_t) const { return V4<float>{{0.f, 0.f, 0.f, 0.f}}; }
    __device__ void apply(size_t i, float, float, float diag, double *) const { out[i] = w * rhs[i] / diag; }
    __device__ void apply4(size_t i, const V4<float> &, const V4<float> &, const V4<float> &dg, double *) const {
        const V4<float> r = ld4(rhs + i);
        V4<float> o;
        for (int q = 0; q < 4; ++q) o.v[q] = w * r.v[q] / dg.v[q];
        st4(out + i, o);
    }
};

// Smoothing: a degree-2 Chebyshev polynomial in A/6 on [kChebLo, 2] (the
// spectrum of A/6 lies in [0, 2]: the rows of A sum to at most 12), applied as
// two Richardson sweeps x <- x + w_k (rhs - A x) with w_k = 1 / (6 lambda_k),
// lambda_k the polynomial's roots.  The factor |s(lambda)| stays below 1 on
// (0, 2] and below 1/T_2((2 + lo) / (2 - lo)) on [lo, 2]; both sweeps are
// polynomials in the same matrix, so pre- and post-smoothing commute and the
// V-cycle is a symmetric preconditioner.  From a zero guess the first sweep is
// pointwise, x1 = wa rhs, so the two pre-smoothing sweeps are one pass over
// rhs: x2 = x1 + wb (rhs - A x1), a 7-point stencil of rhs.
constexpr double kChebLo = 0.25;
constexpr double kChebL1 = (2.0 + kChebLo) / 2 - (2.0 - kChebLo) / 2 * 0.70710678118654752;
constexpr double kChebL2 = (2.0 + kChebLo) / 2 + (2.0 - kChebLo) / 2 * 0.70710678118654752;
constexpr float kChebWa = (float)(1.0 / (6.0 * kChebL1));
constexpr float kChebWb = (float)(1.0 / (6.0 * kChebL2));

// Weighted-Jacobi sweep x_out = x + w (rhs - A x) / diag (only on an
// odd-sized coarsest level, where no exact solve applies).
struct OpSmooth {
    using T = float;
    static constexpr int NRED = 0;
    const float *x, *rhs;
    float *out;
    float w;
    __device__ float load(size_t i) const { return x[i]; }
    __device__ float load1(size_t i) const { return x[i]; }
    __device__ V4<float> load4(size_t i) const { return ld4(x + i); }
    __device__ void apply(size_t i, float c, float s, float diag, double *) const {
        out[i] = c + w * (rhs[i] - (diag * c - s)) / diag;
    }
    __device__ void apply4(size_t i, const V4<float> &c, const V4<float> &s, const V4<float> &dg, double *) const {
        const V4<float> r = ld4(rhs + i);
        V4<float> o;
        for (int q = 0; q < 4; ++q) o.v[q] = c.v[q] + w * (r.v[q] - (dg.v[q] * c.v[q] - s.v[q])) / dg.v[q];
        st4(out + i, o);
    }
};

// CG direction update fused with the operator: p = z + beta p_old (computed
// on the fly for the neighbours too), q = A p, sum p.q.
template <bool FIRST>
struct OpPMatvec {
    using T = float;
    static constexpr int NRED = 1;
    const float *z, *pold;
    float *pnew, *q;
    const SolveScalars *sc;   // beta, formed on the device by the last finalize
    float beta;
    __device__ float load(size_t i) const {
        if constexpr (FIRST) return z[i];
        else return z[i] + beta * pold[i];
    }
    __device__ float load1(size_t i) const { return load(i); }
    __device__ V4<float> load4(size_t i) const {
        V4<float> r = ld4(z + i);
        if constexpr (!FIRST) {
            const V4<float> p = ld4(pold + i);
            for (int k = 0; k < 4; ++k) r.v[k] += beta * p.v[k];
        }
        return r;
    }
    __device__ void apply(size_t i, float c, float s, float diag, double *acc) const {
        float qv = diag * c - s;
        pnew[i] = c;
        q[i] = qv;
        acc[0] += (double)c * (double)qv;
    }
    __device__ void apply4(size_t i, const V4<float> &c, const V4<float> &s, const V4<float> &dg, double *acc) const {
        V4<float> qq;
        for (int k = 0; k < 4; ++k) {
            qq.v[k] = dg.v[k] * c.v[k] - s.v[k];
            acc[0] += (double)c.v[k] * (double)qq.v[k];
        }
        st4(pnew + i, c);
        st4(q + i, qq);
    }
    __device__ void applyA(size_t i, float c, float au, double *acc) const {
        pnew[i] = c;
        q[i] = au;
        acc[0] += (double)c * (double)au;
    }
    __device__ void applyA4(size_t i, const V4<float> &c, const V4<float> &au, double *acc) const {
        for (int k = 0; k < 4; ++k) acc[0] += (double)c.v[k] * (double)au.v[k];
        st4(pnew + i, c);
        st4(q + i, au);
    }
};

// Exact quadrature: the 7-point V-cycle M7 is wrapped between two Jacobi
// steps on the 27-point operator A, z = M r with
//   z1 = w r,  z2 = z1 + M7 (r - A z1),  z = z2 + w (r - A z2),
// i.e. I - M A = (I - w A)(I - M7 A)(I - w A): symmetric, and M >= w I, so
// positive definite.  On the cosine modes A lies in (0, 4) and A / A7 in
// [1/9, 1]; M7 alone leaves the modes high in all three axes at A / A7 ~ 1/9,
// which the steps with w = 3/8 (the inverse of A's diagonal 8/3) damp by
// (1 - w A)^2 <= 1/4.
constexpr float kJacobi27 = 0.375f;

// first step: out = r - w A r
struct OpJacobi27a {
    using T = float;
    static constexpr int NRED = 0;
    const float *r;
    float *out;
    float w;
    __device__ float load(size_t i) const { return r[i]; }
    __device__ float load1(size_t i) const { return r[i]; }
    __device__ V4<float> load4(size_t i) const { return ld4(r + i); }
    __device__ void applyA(size_t i, float c, float au, double *) const { out[i] = c - w * au; }
    __device__ void applyA4(size_t i, const V4<float> &c, const V4<float> &au, double *) const {
        V4<float> o;
        for (int k = 0; k < 4; ++k) o.v[k] = c.v[k] - w * au.v[k];
        st4(out + i, o);
    }
};

// last step, with u = w r + y (y = M7 applied to the first step's output):
// z = u + w (r - A u), and the sum r.z
struct OpJacobi27b {
    using T = float;
    static constexpr int NRED = 1;
    const float *r, *y;
    float *z;
    float w;
    __device__ float load(size_t i) const { return w * r[i] + y[i]; }
    __device__ float load1(size_t i) const { return load(i); }
    __device__ V4<float> load4(size_t i) const {
        const V4<float> a = ld4(r + i), b = ld4(y + i);
        V4<float> o;
        for (int k = 0; k < 4; ++k) o.v[k] = w * a.v[k] + b.v[k];
        return o;
    }
    __device__ void applyA(size_t i, float c, float au, double *acc) const {
        const float ri = r[i];
        const float zz = c + w * (ri - au);
        z[i] = zz;
        acc[0] += (double)ri * (double)zz;
    }
    __device__ void applyA4(size_t i, const V4<float> &c, const V4<float> &au, double *acc) const {
        const V4<float> rr = ld4(r + i);
        V4<float> o;
        for (int k = 0; k < 4; ++k) {
            o.v[k] = c.v[k] + w * (rr.v[k] - au.v[k]);
            acc[0] += (double)rr.v[k] * (double)o.v[k];
        }
        st4(z + i, o);
    }
};

__device__ __forceinline__ void fetch_scalars(OpPMatvec<false> &op) { op.beta = (float)op.sc->beta; }
template <class TB>
__device__ __forceinline__ void fetch_scalars(OpResid64<TB> &op) { op.mb = op.sc ? op.sc->mean_b : 0.0; }

template <bool FIRST>
__global__ __launch_bounds__(256) void k_cg_update(float *__restrict__ x, float *__restrict__ r,
                                                    const float *__restrict__ p, const float *__restrict__ q,
                                                    const SolveScalars *sc, size_t n, double *partials) {
    if (sc->done) return;
    const float a = (float)sc->alpha;
    double acc[1] = {0.0};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float pi = p[i];
        if constexpr (FIRST) x[i] = a * pi;
        else x[i] += a * pi;
        float rv = r[i] - a * q[i];
        r[i] = rv;
        acc[0] += (double)rv * (double)rv;
    }
    __shared__ double lds[4][1];
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
}

template <class TB>
__global__ __launch_bounds__(256) void k_sum(const TB *__restrict__ x, size_t n, double *partials) {
    double acc[1] = {0.0};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        acc[0] += (double)x[i];
    __shared__ double lds[4][1];
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
}

__global__ void k_axpy64(double *x, const float *e, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] += (double)e[i];
}

__global__ void k_shift64(double *x, double by, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] -= by;
}

// zero n 32-bit words (a kernel rather than a memset node, so the clear is an
// ordinary kernel wherever the launch ends up)
__global__ void k_zero_words(uint32_t *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void k_fill64(double *x, double v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        x[i] = v;
}

// 1-D weight of fine cell f = 2C - 1 + t (t = 0..3) in the trilinear
// prolongation column of coarse cell C; boundary ghosts mirror with sign s.
__device__ __forceinline__ float restrict_w(int t, int C, int nc, int s) {
    switch (t) {
        case 0: return C >= 1 ? 0.25f : 0.f;
        case 1: return 0.75f + (C == 0 ? 0.25f * s : 0.f);
        case 2: return 0.75f + (C == nc - 1 ? 0.25f * s : 0.f);
        default: return C + 1 < nc ? 0.25f : 0.f;
    }
}

// 1-D trilinear prolongation weights of fine cell f: coarse cells a = f / 2
// (3/4) and its neighbour b on f's side (1/4); past a boundary the missing
// neighbour mirrors onto a with sign s.
struct Prolong1 {
    int a, b;
    float wa, wb;
};
__device__ __forceinline__ Prolong1 prolong_w(int f, int nc, int s) {
    Prolong1 r;
    r.a = f >> 1;
    r.b = (f & 1) ? r.a + 1 : r.a - 1;
    r.wa = 0.75f;
    r.wb = 0.25f;
    if (r.b < 0 || r.b >= nc) {
        r.wa = 0.75f + 0.25f * s;
        r.wb = 0.f;
        r.b = r.a;
    }
    return r;
}

// ---------------------------------------------------------------------------
// Fused V-cycle kernels.  Each level of the V-cycle is two passes over the
// fine field instead of six:
//   pre:  x = S rhs (both Chebyshev sweeps from a zero guess), r = rhs - A x,
//         coarse rhs = 1/2 P^T r;
//   post: x <- x + P e (e: the coarse correction), then the two Chebyshev
//         sweeps in reverse order, and at the finest level the sum rhs . x.
// A workgroup takes a tile of up to kVTX x kVTY fine (x, y) columns plus a
// halo (3 cells for pre: r is needed one cell beyond the tile for the
// restriction, x two, rhs three; 2 for post) and marches a chunk of z planes.
// Each thread owns fixed columns of the haloed tile and keeps their z
// neighbours in registers; the in-plane neighbours of the plane being worked
// on come through LDS.  Values outside the grid are 0, which is what the
// boundary rows of A assume (their diagonal carries the missing faces).
// Halo cells are recomputed by every tile that needs them; each output is
// written by its owner tile only.
constexpr int kVB = 512;                  // threads per workgroup
constexpr int kVTX = 64, kVTY = 16;       // largest fine tile
constexpr int kPreH = 3, kPostH = 2;
// the four corner cells of a haloed tile feed no 7-point stencil: no slot holds them
constexpr int kPreCols = (kVTX + 2 * kPreH) * (kVTY + 2 * kPreH) - 4;
constexpr int kPostCols = (kVTX + 2 * kPostH) * (kVTY + 2 * kPostH) - 4;
constexpr int kPreCPT = (kPreCols + kVB - 1) / kVB;
constexpr int kPostCPT = (kPostCols + kVB - 1) / kVB;

struct VTile {
    int tx, ty, zc;   // fine tile extents (even) and fine planes per chunk (even)
    int gx, gy, gz;   // tiles per axis
    __host__ __device__ unsigned count() const { return (unsigned)gx * (unsigned)gy * (unsigned)gz; }
};

// tiles of a level with a coarser level below it (every extent even)
VTile vtile_of(const Dims &d) {
    VTile t;
    t.tx = d.nx < kVTX ? d.nx : kVTX;
    t.ty = d.ny < kVTY ? d.ny : kVTY;
    t.gx = (int)cdiv(d.nx, t.tx);
    t.gy = (int)cdiv(d.ny, t.ty);
    // longest chunk (fewest recomputed halo planes, at most 32) that still gives >= 512 workgroups
    for (t.zc = 32;; t.zc /= 2) {
        t.gz = (int)cdiv(d.nz, t.zc);
        if (t.zc == 2 || (size_t)t.gx * t.gy * t.gz >= 512) break;
    }
    return t;
}

// One owned column of the haloed tile.  Slots past the tile's columns (the
// last thread rows) and columns off the grid compute with in = 0, so every
// value they produce is 0 and no lane branches.
struct VCol {
    int c;       // index in the tile
    unsigned off;   // i + nx j (0 off the grid: a valid address, masked at use)
    float in;    // 1 on the grid, else 0
    float dxy;   // 6 + bc_sign * (missing x/y faces)
    bool own;    // an output cell of this tile
};

__device__ __forceinline__ VCol vcol(int k, int W, int Ht, int H, int X0, int Y0, int tx, int ty, const Dims &d,
                                      int &i, int &j) {
    // slot k -> tile cell c, skipping cells 0, W-1, (Ht-1) W and Ht W - 1
    int c = k + 1;
    c += c >= W - 1;
    c += c >= (Ht - 1) * W;
    c += c >= Ht * W - 1;
    VCol r;
    r.c = c;
    r.off = 0;
    r.in = 0.f;
    r.dxy = 6.f;
    r.own = false;
    const int u = c % W, v = c / W;
    i = X0 - H + u;
    j = Y0 - H + v;
    if (v < Ht && i >= 0 && i < d.nx && j >= 0 && j < d.ny) {
        r.off = (unsigned)(i + d.nx * j);
        r.in = 1.f;
        r.dxy = (float)(6 + d.bc_sign * ((i == 0) + (i == d.nx - 1) + (j == 0) + (j == d.ny - 1)));
        r.own = u >= H && u < H + tx && v >= H && v < H + ty;
    } else {
        i = j = 0;
    }
    return r;
}

// The LDS planes carry a pad of one tile row plus one on each side, so the
// four in-plane neighbours of every slot are plain offsets; a value that
// reads past the tile (or a pad) is never used.
__device__ __forceinline__ float vnbr(const float *s, int c, int W) {
    return (s[c - 1] + s[c + 1]) + (s[c - W] + s[c + W]);
}

// z-face part of the diagonal on plane z (uniform)
__device__ __forceinline__ float vdz(int z, const Dims &d) {
    return (float)(d.bc_sign * ((z == 0) + (z == d.nz - 1)));
}

// LDS planes: the tile's cells at [pad, pad + slots + 4), a pad of one tile
// row plus a few cells on each side, so the four in-plane neighbours of every
// slot are plain offsets.  Pads and the four corner cells are zeroed once.
constexpr int kPrePad = kVTX + 2 * kPreH + 4, kPreLds = 2 * kPrePad + kPreCPT * kVB + 4;
constexpr int kPostPad = kVTX + 2 * kPostH + 4, kPostLds = 2 * kPostPad + kPostCPT * kVB + 4;

template <int N, int PAD>
__device__ __forceinline__ void zero_pads(float *s, int W, int Ht) {
    for (int k = threadIdx.x; k < PAD; k += kVB) {
        s[k] = 0.f;
        s[N - 1 - k] = 0.f;
    }
    if (threadIdx.x == 0) {
        s[PAD] = 0.f;
        s[PAD + W - 1] = 0.f;
        s[PAD + (Ht - 1) * W] = 0.f;
        s[PAD + Ht * W - 1] = 0.f;
    }
}

// pre: xo = x2 of the pre-smoothing from a zero guess, crhs = 1/2 P^T (rhs - A xo).
__global__ __launch_bounds__(kVB, 4) void k_vc_pre(const float *__restrict__ rhs, float *__restrict__ xo,
                                                 float *__restrict__ crhs, Dims df, Dims dc, VTile vt, float wa,
                                                 float wb, const int *skip) {
    constexpr int H = kPreH, CPT = kPreCPT;
    if (skipped(skip)) return;
    __shared__ float sR[2][kPreLds];
    __shared__ float sX[2][kPreLds];
    __shared__ __align__(16) float sr[2][kPreLds];   // read as float2 by the restriction
    const unsigned lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int bx = (int)(lb % (unsigned)vt.gx), by = (int)((lb / (unsigned)vt.gx) % (unsigned)vt.gy),
              bz = (int)(lb / ((unsigned)vt.gx * (unsigned)vt.gy));
    const int X0 = bx * vt.tx, Y0 = by * vt.ty;
    const int W = vt.tx + 2 * H, Ht = vt.ty + 2 * H;
    zero_pads<kPreLds, kPrePad>(sR[0], W, Ht);
    zero_pads<kPreLds, kPrePad>(sR[1], W, Ht);
    zero_pads<kPreLds, kPrePad>(sX[0], W, Ht);
    zero_pads<kPreLds, kPrePad>(sX[1], W, Ht);
    zero_pads<kPreLds, kPrePad>(sr[0], W, Ht);
    zero_pads<kPreLds, kPrePad>(sr[1], W, Ht);
    const int K0 = bz * (vt.zc / 2), K1 = min(K0 + vt.zc / 2, dc.nz);
    const size_t plane = (size_t)df.nx * df.ny;
    VCol col[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        int i, j;
        col[q] = vcol((int)threadIdx.x + kVB * q, W, Ht, H, X0, Y0, vt.tx, vt.ty, df, i, j);
        col[q].c += kPrePad;
    }
    // rhs is fetched four planes ahead into four buffers that the unrolled
    // loop below uses in turn (the kernel's few workgroups per compute unit
    // need that many fetches in flight).  Fetches are unconditional (a plane
    // outside [0, nz) is fetched clamped and scaled by 0), so a buffer keeps
    // its registers across iterations and no fetch is waited for early.
    const int s0 = 2 * K0 - 3, s1 = 2 * K1 + 2;   // s0 odd
    auto load = [&](int s, float(&buf)[CPT], float &sc) {
        sc = (s >= 0 && s < df.nz) ? 1.f : 0.f;
        const float *rp = rhs + (size_t)min(max(s, 0), df.nz - 1) * plane;
#pragma unroll
        for (int q = 0; q < CPT; ++q) buf[q] = rp[col[q].off];
    };
    float bA[CPT], bB[CPT], bC[CPT], bD[CPT], sa, sb, sc, sd;
    load(s0, bA, sa);
    load(s0 + 1, bB, sb);
    load(s0 + 2, bC, sc);
    load(s0 + 3, bD, sd);
    // coarse cell of this thread in the restriction (x fastest)
    const int ctx = vt.tx / 2, cty = vt.ty / 2;
    const int ca = (int)threadIdx.x % ctx, cb = (int)threadIdx.x / ctx;
    const int I = X0 / 2 + ca, J = Y0 / 2 + cb;
    const bool cown = cb < cty && I < dc.nx && J < dc.ny;
    const int ms = -dc.bc_sign;   // mirror sign: +1 Neumann, -1 Dirichlet
    float wx[4], wy[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        wx[t] = cown ? restrict_w(t, I, dc.nx, ms) : 0.f;
        wy[t] = cown ? restrict_w(t, J, dc.ny, ms) : 0.f;
    }
    // fine cells 2I-1 .. 2I+2 sit at tile columns 2 ca + 2 .. 2 ca + 5 (H = 3)
    const int rbase = kPrePad + W * (2 * cb + 2) + 2 * ca + 2;
    float z0 = 0.f, z1 = 0.f, z2 = 0.f, z3 = 0.f;   // x/y-restricted r of fine planes t-3 .. t
    // z rings: rhs on planes s-2, s-1, s; x on planes s-3, s-2, s-1
    float h0[CPT], h1[CPT], h2[CPT], x0[CPT], x1[CPT], x2[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) h0[q] = h1[q] = h2[q] = x0[q] = x1[q] = x2[q] = 0.f;
    // One z step (par = s & 1, a constant at every call), with one barrier:
    // every LDS plane it reads was written in the previous step, and every
    // plane it writes was last read in the previous step.
    //   rhs(s) -> sR[s];  x(s-1) from sR[s-1] -> sX[s-1];
    //   r(s-2) from sX[s-2] -> sr[s-2];  restriction of r(s-3) from sr[s-3].
    auto step = [&](int s, int par, float(&buf)[CPT], float &bsc) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            h0[q] = h1[q];
            h1[q] = h2[q];
            h2[q] = buf[q] * (col[q].in * bsc);
        }
        load(s + 4, buf, bsc);
        {
            float *R = sR[par];
#pragma unroll
            for (int q = 0; q < CPT; ++q) R[col[q].c] = h2[q];
        }
        // pre-smoothed x on plane p = s - 1: x1 = wa rhs, x2 = x1 + wb (rhs - A x1)
        const int p = s - 1;
        {
            const bool pin = p >= 0 && p < df.nz;
            const float pm = pin ? 1.f : 0.f, dzp = vdz(p, df);
            const float *Rp = sR[par ^ 1];
            float *X = sX[par ^ 1];
            float *xop = xo + (size_t)(pin ? p : 0) * plane;
            const bool pout = p >= 2 * K0 && p < 2 * K1;
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                const float nb = vnbr(Rp, col[q].c, W) + (h0[q] + h2[q]);
                const float c = h1[q];
                const float v = (wa * c + wb * (c - wa * ((col[q].dxy + dzp) * c - nb))) * (col[q].in * pm);
                if (pout && col[q].own) xop[col[q].off] = v;
                x0[q] = x1[q];
                x1[q] = x2[q];
                x2[q] = v;
                X[col[q].c] = v;
            }
        }
        // residual on plane t = s - 2
        const int t = s - 2;
        if (t >= 2 * K0 - 1) {
            const float tm = (t >= 0 && t < df.nz) ? 1.f : 0.f, dzt = vdz(t, df);
            const float *Xt = sX[par];
            float *r = sr[par];
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                const float nb = vnbr(Xt, col[q].c, W) + (x0[q] + x2[q]);
                r[col[q].c] = (h0[q] - ((col[q].dxy + dzt) * x1[q] - nb)) * (col[q].in * tm);
            }
        }
        // residual of plane t - 1, restricted in x and y
        const int tr = s - 3;
        if (tr >= 2 * K0 - 1 && cown) {
            const float *r = sr[par ^ 1] + rbase;
            float acc = 0.f;
#pragma unroll
            // rbase and W are even: each row's four cells are two 8-byte reads
            for (int ty = 0; ty < 4; ++ty) {
                const float2 *row = reinterpret_cast<const float2 *>(r + W * ty);
                const float2 a = row[0], b = row[1];
                acc += wy[ty] * (wx[0] * a.x + wx[1] * a.y + wx[2] * b.x + wx[3] * b.y);
            }
            z0 = z1;
            z1 = z2;
            z2 = z3;
            z3 = acc;
            if (tr >= 2 * K0 + 2 && !(tr & 1)) {   // tr = 2K + 2: fine planes 2K-1 .. 2K+2 are in
                const int K = tr / 2 - 1;
                crhs[(size_t)I + (size_t)dc.nx * ((size_t)J + (size_t)dc.ny * K)] =
                    0.5f * (restrict_w(0, K, dc.nz, ms) * z0 + restrict_w(1, K, dc.nz, ms) * z1 +
                            restrict_w(2, K, dc.nz, ms) * z2 + restrict_w(3, K, dc.nz, ms) * z3);
            }
        }
    };
    // the last restricted plane, 2 K1, is restricted at step 2 K1 + 3 = s1 + 1
    for (int s = s0; s <= s1 + 1; s += 4) {
        step(s, 1, bA, sa);
        if (s + 1 > s1 + 1) break;
        step(s + 1, 0, bB, sb);
        if (s + 2 > s1 + 1) break;
        step(s + 2, 1, bC, sc);
        if (s + 3 > s1 + 1) break;
        step(s + 3, 0, bD, sd);
    }
}

// post: u = x + P e, v = u + wb (rhs - A u), xo = v + wa (rhs - A v); DOT adds
// rhs . xo to the block's partial.
template <bool DOT>
__global__ __launch_bounds__(kVB, 4) void k_vc_post(const float *__restrict__ x, const float *__restrict__ rhs,
                                                     const float *__restrict__ e, float *__restrict__ xo, Dims df,
                                                     Dims dc, VTile vt, float wb, float wa, double *partials,
                                                     const int *skip) {
    constexpr int H = kPostH, CPT = kPostCPT;
    if (skipped(skip)) return;
    __shared__ float sU[2][kPostLds];
    __shared__ float sV[2][kPostLds];
    __shared__ float sQ[3][kPostLds];   // x/y-interpolated coarse planes, by coarse index mod 3
    const unsigned lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int bx = (int)(lb % (unsigned)vt.gx), by = (int)((lb / (unsigned)vt.gx) % (unsigned)vt.gy),
              bz = (int)(lb / ((unsigned)vt.gx * (unsigned)vt.gy));
    const int X0 = bx * vt.tx, Y0 = by * vt.ty;
    const int W = vt.tx + 2 * H, Ht = vt.ty + 2 * H;
    zero_pads<kPostLds, kPostPad>(sU[0], W, Ht);
    zero_pads<kPostLds, kPostPad>(sU[1], W, Ht);
    zero_pads<kPostLds, kPostPad>(sV[0], W, Ht);
    zero_pads<kPostLds, kPostPad>(sV[1], W, Ht);
    const int k0 = bz * vt.zc, k1 = min(k0 + vt.zc, df.nz);
    const size_t plane = (size_t)df.nx * df.ny, cplane = (size_t)dc.nx * dc.ny;
    const int ms = -dc.bc_sign;
    VCol col[CPT];
    unsigned ij[CPT];   // i | j << 16 of the column (0 off the grid)
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        int i, j;
        col[q] = vcol((int)threadIdx.x + kVB * q, W, Ht, H, X0, Y0, vt.tx, vt.ty, df, i, j);
        col[q].c += kPostPad;
        ij[q] = (unsigned)i | ((unsigned)j << 16);
    }
    // The x/y-interpolated coarse plane m at each column goes to sQ[m % 3]:
    // its four coarse values are fetched two steps before they are mixed.
    // Each thread reads back only its own columns, so no barrier is needed.
    // Off the coarse grid the plane is 0 (its weight is 0 too); the fetch is
    // then clamped and scaled by cscale = 0.
    float c0[CPT], c1[CPT], c2[CPT], c3[CPT];
    float cscale = 0.f;
    auto qfetch = [&](int m) {
        cscale = (m >= 0 && m < dc.nz) ? 1.f : 0.f;
        const float *em = e + (size_t)min(max(m, 0), dc.nz - 1) * cplane;
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const Prolong1 px = prolong_w((int)(ij[q] & 0xffffu), dc.nx, ms);
            const Prolong1 py = prolong_w((int)(ij[q] >> 16), dc.ny, ms);
            const unsigned ra = (unsigned)(dc.nx * py.a), rb = (unsigned)(dc.nx * py.b);
            c0[q] = em[ra + (unsigned)px.a];
            c1[q] = em[ra + (unsigned)px.b];
            c2[q] = em[rb + (unsigned)px.a];
            c3[q] = em[rb + (unsigned)px.b];
        }
    };
    auto qstore = [&](int m) {   // m: the plane of the last qfetch
        float *Q = sQ[(m + 3) % 3];
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const Prolong1 px = prolong_w((int)(ij[q] & 0xffffu), dc.nx, ms);
            const Prolong1 py = prolong_w((int)(ij[q] >> 16), dc.ny, ms);
            Q[col[q].c] = cscale * (py.wa * (px.wa * c0[q] + px.wb * c1[q]) + py.wb * (px.wa * c2[q] + px.wb * c3[q]));
        }
    };
    // x is used at the step that takes its plane, so it is fetched two steps
    // ahead (a two-plane queue); rhs of plane s is first used at step s + 1,
    // so it is fetched at step s.  The fetches are unconditional (the buffers
    // keep their registers across the loop).  A plane outside [0, nz) is
    // fetched clamped: every value computed from it there is masked to 0, and
    // rhs enters only the planes' own (in-range) updates.
    auto load = [&](const float *f, int s, float(&buf)[CPT]) {
        const float *fp = f + (size_t)min(max(s, 0), df.nz - 1) * plane;
#pragma unroll
        for (int q = 0; q < CPT; ++q) buf[q] = fp[col[q].off];
    };
    const int s0 = k0 - 2, s1 = k1 + 1;   // k0 even: s0 even, s0 >> 1 >= -1
    qfetch((s0 >> 1) - 1);
    qstore((s0 >> 1) - 1);
    qfetch(s0 >> 1);
    qstore(s0 >> 1);
    qfetch((s0 >> 1) + 1);
    float xA[CPT], xB[CPT], hN[CPT];
    load(x, s0, xA);
    load(x, s0 + 1, xB);
    double acc[1] = {0.0};
    // z rings: u on planes s-2 .. s, v on s-3 .. s-1, rhs on s-2 .. s-1 (and s in flight)
    float u0[CPT], u1[CPT], u2[CPT], v0[CPT], v1[CPT], v2[CPT], h0[CPT], h1[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) u0[q] = u1[q] = u2[q] = v0[q] = v1[q] = v2[q] = h0[q] = h1[q] = hN[q] = 0.f;
    // One z step (par = s & 1) with one barrier: every LDS plane it reads was
    // written in the previous step, and every plane it writes was last read in
    // the previous step.  sQ is read back only by the thread that wrote it.
    //   u(s) -> sU[s];  v(s-1) from sU[s-1] -> sV[s-1];  xo(s-2) from sV[s-2].
    auto step = [&](int s, int par) {
        __syncthreads();
        const int K = s >> 1;
        if (!par) {
            // planes K-1 and K are in sQ; K+1 (first needed at s+1) arrived: mix it, fetch K+2
            qstore(K + 1);
            qfetch(K + 2);
        }
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            h0[q] = h1[q];
            h1[q] = hN[q];
        }
        load(rhs, s, hN);
        // u on plane s; z prolongation: plane s takes coarse K (3/4) and K-1 (even s) or K+1 (odd s)
        {
            const int N = par ? K + 1 : K - 1;
            const bool nin = N >= 0 && N < dc.nz;
            const float wK = nin ? 0.75f : 0.75f + 0.25f * ms, wN = nin ? 0.25f : 0.f;
            const float sm = (s >= 0 && s < df.nz) ? 1.f : 0.f;
            const float *QK = sQ[(K + 3) % 3], *QN = sQ[(N + 3) % 3];
            float *U = sU[par];
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                const float uv = (xA[q] + wK * QK[col[q].c] + wN * QN[col[q].c]) * (col[q].in * sm);
                u0[q] = u1[q];
                u1[q] = u2[q];
                u2[q] = uv;
                U[col[q].c] = uv;
                xA[q] = xB[q];
            }
            load(x, s + 2, xB);
        }
        const int p = s - 1;
        if (p >= k0 - 1) {
            const float pm = (p >= 0 && p < df.nz) ? 1.f : 0.f, dzp = vdz(p, df);
            const float *Up = sU[par ^ 1];
            float *V = sV[par ^ 1];
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                const float nb = vnbr(Up, col[q].c, W) + (u0[q] + u2[q]);
                const float vv = (u1[q] + wb * (h1[q] - ((col[q].dxy + dzp) * u1[q] - nb))) * (col[q].in * pm);
                v0[q] = v1[q];
                v1[q] = v2[q];
                v2[q] = vv;
                V[col[q].c] = vv;
            }
        }
        const int t = s - 2;
        if (t >= k0) {   // t < k1 holds: s <= k1 + 1
            const float dzt = vdz(t, df);
            const float *Vt = sV[par];
            float *xop = xo + (size_t)t * plane;
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                const float nb = vnbr(Vt, col[q].c, W) + (v0[q] + v2[q]);
                const float w = v1[q] + wa * (h0[q] - ((col[q].dxy + dzt) * v1[q] - nb));
                if (col[q].own) {
                    xop[col[q].off] = w;
                    if constexpr (DOT) acc[0] += (double)h0[q] * (double)w;
                }
            }
        }
    };
    for (int s = s0; s <= s1; ++s) step(s, s & 1);
    if constexpr (DOT) {
        __shared__ double lds[kVB / 64][1];
        block_sum<1>(acc, lds);
        if (threadIdx.x == 0) partials[lb] = acc[0];
    }
}

// out = rhs . x summed per block (the r.z of a single-level hierarchy).
__global__ __launch_bounds__(256) void k_dot(const float *__restrict__ a, const float *__restrict__ b, size_t n,
                                              double *partials, const int *skip) {
    if (skipped(skip)) return;
    double acc[1] = {0.0};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        acc[0] += (double)a[i] * (double)b[i];
    __shared__ double lds[4][1];
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
}

// Exact solve on the coarsest level (every extent <= kDirectAxis) by the
// separable eigenbasis of the 7-point operator: transform along x, y, z with
// the orthonormal 1-D bases, divide by lambda_x + lambda_y + lambda_z (the
// constant mode is dropped), transform back.  Three small kernels: the x and
// y transforms of one z plane per workgroup, then the z transform, division
// and inverse z transform of one y row of coefficients per workgroup, then
// the inverse y and x transforms per z plane.  Each workgroup stages its
// N x N slice (N = 32 or 64) and the bases in LDS (the bases stored so that a
// wavefront's lanes read consecutive or identical entries) and computes N / 8
// or N / 4 outputs per thread.  E = [phi_x (cx*cx), phi_y (cy*cy),
// phi_z (cz*cz), lam_x, lam_y, lam_z], phi_a[m * n_a + i] = mode m at cell i.
// N: the slice edge, 32 or 64 (every extent of the level at most N).  At
// N = 32 a wavefront spans two rows of a slice, so rows are padded; at N = 64
// a wavefront is one row group and every slice access is a run of consecutive
// entries or one broadcast entry, so the four 64 x 64 arrays go unpadded
// (64 KiB of LDS per workgroup).
template <int N> struct Eig {
    static_assert(N == 32 || N == 64, "slice edge");
    static constexpr int G = 256 / N;          // row groups of a 256-thread workgroup
    static constexpr int P = N == 32 ? 1 : 0;  // row padding
};

// FWD: c[k][my][mx] = sum_j sum_i phi_y[my][j] phi_x[mx][i] f[k][j][i] for z plane k = blockIdx.x;
// inverse: f[k][j][i] = sum_my sum_mx phi_y[my][j] phi_x[mx][i] c[k][my][mx].
template <int N, bool FWD>
__global__ __launch_bounds__(256) void k_eig_plane(const float *__restrict__ src, float *__restrict__ dst,
                                                   const float *__restrict__ E, int cx, int cy, const int *skip) {
    if (skipped(skip)) return;
    constexpr int G = Eig<N>::G, P = Eig<N>::P;
    __shared__ float T[N][N + P];
    __shared__ float U[N][N + P];
    // forward: Px[i][m] = phi_x[m][i]; inverse: Px[m][i] = phi_x[m][i] (lanes run along i either way)
    __shared__ float Px[N][N + P];
    __shared__ float Py[N][N + P];   // Py[j][m] = phi_y[m][j]
    const size_t plane = (size_t)cx * cy, k = blockIdx.x;
    const float *ex = E, *ey = E + cx * cx;
    for (int o = threadIdx.x; o < N * N; o += blockDim.x) {
        const int r = o / N, c = o % N;
        Px[r][c] = (r < cx && c < cx) ? (FWD ? ex[c * cx + r] : ex[r * cx + c]) : 0.f;
        Py[r][c] = (r < cy && c < cy) ? ey[c * cy + r] : 0.f;
        T[r][c] = (r < cy && c < cx) ? src[k * plane + (size_t)r * cx + c] : 0.f;
    }
    __syncthreads();
    const int a = threadIdx.x % N, g = threadIdx.x / N;   // lane in a row, G row groups
    if (FWD) {
        for (int j = g; j < N; j += G) {   // along x: U[j][m] = sum_i phi_x[m][i] T[j][i]
            float acc = 0.f;
#pragma unroll 8
            for (int i = 0; i < N; ++i) acc += Px[i][a] * T[j][i];
            U[j][a] = acc;
        }
        __syncthreads();
        for (int my = g; my < N; my += G) {   // along y: T[my][m] = sum_j phi_y[my][j] U[j][m]
            float acc = 0.f;
#pragma unroll 8
            for (int j = 0; j < N; ++j) acc += Py[j][my] * U[j][a];
            T[my][a] = acc;
        }
    } else {
        for (int j = g; j < N; j += G) {   // along y: U[j][m] = sum_my phi_y[my][j] T[my][m]
            float acc = 0.f;
#pragma unroll 8
            for (int my = 0; my < N; ++my) acc += Py[j][my] * T[my][a];
            U[j][a] = acc;
        }
        __syncthreads();
        for (int j = g; j < N; j += G) {   // along x: T[j][i] = sum_m phi_x[m][i] U[j][m]
            float acc = 0.f;
#pragma unroll 8
            for (int m = 0; m < N; ++m) acc += Px[m][a] * U[j][m];
            T[j][a] = acc;
        }
    }
    __syncthreads();
    for (int o = threadIdx.x; o < N * N; o += blockDim.x) {
        const int r = o / N, c = o % N;
        if (r < cy && c < cx) dst[k * plane + (size_t)r * cx + c] = T[r][c];
    }
}

// In place on the coefficients of y mode my = blockIdx.x: transform along z,
// divide by the eigenvalue (0 for the constant mode), transform back.
template <int N>
__global__ __launch_bounds__(256) void k_eig_z(float *__restrict__ buf, const float *__restrict__ E, int cx, int cy,
                                               int cz, const int *skip) {
    if (skipped(skip)) return;
    constexpr int G = Eig<N>::G, P = Eig<N>::P;
    __shared__ float V[N][N + P];
    __shared__ float Wz[N][N + P];
    __shared__ float Pz[N][N + P];   // Pz[k][n] = phi_z[n][k]
    __shared__ float lx[N], lz[N];
    const size_t plane = (size_t)cx * cy, my = blockIdx.x;
    const float *ez = E + cx * cx + cy * cy, *lam = ez + cz * cz;
    for (int o = threadIdx.x; o < N * N; o += blockDim.x) {
        const int r = o / N, c = o % N;
        Pz[r][c] = (r < cz && c < cz) ? ez[c * cz + r] : 0.f;
        V[r][c] = (r < cz && c < cx) ? buf[(size_t)r * plane + my * cx + c] : 0.f;
    }
    if (threadIdx.x < N) {
        lx[threadIdx.x] = threadIdx.x < cx ? lam[threadIdx.x] : 0.f;
        lz[threadIdx.x] = threadIdx.x < cz ? lam[cx + cy + threadIdx.x] : 0.f;
    }
    __syncthreads();
    const float ly = lam[cx + my];
    const int a = threadIdx.x % N, g = threadIdx.x / N;
    for (int n = g; n < N; n += G) {   // along z and divide: W[n][m] = sum_k phi_z[n][k] V[k][m] / lambda
        float acc = 0.f;
#pragma unroll 8
        for (int k = 0; k < N; ++k) acc += Pz[k][n] * V[k][a];
        const float l = lx[a] + ly + lz[n];
        Wz[n][a] = (a < cx && n < cz && l > 1e-12f) ? acc / l : 0.f;
    }
    __syncthreads();
    for (int k = g; k < cz; k += G) {   // back along z: V[k][m] = sum_n phi_z[n][k] W[n][m]
        float acc = 0.f;
#pragma unroll 8
        for (int n = 0; n < N; ++n) acc += Pz[k][n] * Wz[n][a];
        if (a < cx) buf[(size_t)k * plane + my * cx + a] = acc;
    }
}

enum { FIN_RESID = 0, FIN_RZ = 1, FIN_PQ = 2, FIN_RR = 3, FIN_BSUM = 4 };

// Final stage of a two-stage reduction: sums the per-block partials in a
// fixed order and updates the solver scalars.  The refinement's finalizes
// (FIN_RESID, FIN_BSUM) copy the scalars to the host-mapped record and store
// seq after them.  An inner iteration's FIN_RR decides on the device whether
// the inner solve stops (r.r at the target, r.r not halved in four iterations,
// or a breakdown) and stores the status word (see PublishedScalars); FIN_PQ,
// FIN_RZ and FIN_RR return at once once it has stopped.
__global__ __launch_bounds__(256) void k_finalize(const double *partials, unsigned nb, int mode, int flag,
                                                   SolveScalars *sc, double ncells, PublishedScalars *mirror,
                                                   unsigned seq) {
    if ((mode == FIN_PQ || mode == FIN_RR || (mode == FIN_RZ && !flag)) && sc->done) return;
    const int nred = mode == FIN_RESID ? 5 : 1;
    double v[5] = {0, 0, 0, 0, 0};
    for (int k = 0; k < nred; ++k) {
        double a = 0.0;
        for (unsigned i = threadIdx.x; i < nb; i += blockDim.x) a += partials[(size_t)k * nb + i];
        v[k] = a;
    }
    __shared__ double lds[4][5];
    block_sum<5>(v, lds);
    if (threadIdx.x != 0) return;
    bool bad = false;
    for (int k = 0; k < nred; ++k) bad |= !isfinite(v[k]);
    if (bad) sc->bad |= 1;
    switch (mode) {
        case FIN_RESID: {
            sc->res_sum = v[0];
            sc->res_sq = v[1];
            sc->x_sum = v[2];
            sc->b_sum = v[3];
            sc->b_sq = v[4];
            if (flag) {   // Neumann: project out the mean
                double m = v[0] / ncells;
                sc->mean_r = m;
                sc->res_norm2 = fmax(v[1] - ncells * m * m, 0.0);
                double mb = v[3] / ncells;
                sc->b_norm2 = fmax(v[4] - ncells * mb * mb, 0.0);
            } else {
                sc->mean_r = 0.0;
                sc->res_norm2 = v[1];
                sc->b_norm2 = v[4];
            }
            break;
        }
        case FIN_RZ:
            sc->rz = v[0];
            sc->beta = flag ? 0.0 : (sc->rz_old != 0.0 ? v[0] / sc->rz_old : 0.0);
            sc->rz_old = v[0];
            return;
        case FIN_PQ:
            sc->pq = v[0];
            sc->alpha = (v[0] > 0.0 && isfinite(v[0])) ? sc->rz / v[0] : 0.0;
            if (!(v[0] > 0.0)) sc->bad |= 2;
            return;
        case FIN_RR: {
            const double rr = v[0];
            sc->rr = rr;
            sc->iters += 1;
            int done = 0;
            if (sc->bad || !isfinite(rr)) done = 1;
            else if (rr <= sc->stop_rr) done = 1;
            else if (rr < 0.5 * sc->best) { sc->best = rr; sc->stall = 0; }
            else if (++sc->stall >= 4) done = 1;
            sc->done = done;
            const unsigned long long st = ((unsigned long long)seq << 32) | ((unsigned long long)sc->iters << 2) |
                                          ((unsigned long long)(sc->bad & 1) << 1) | (unsigned long long)done;
            __threadfence_system();
            __hip_atomic_store(&mirror->status, st, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            return;
        }
        case FIN_BSUM:
            sc->b_sum = v[0];
            sc->mean_b = v[0] / ncells;
            break;
    }
    mirror->s = *sc;
    // the host reads the scalars once it sees seq: make them visible first
    __threadfence_system();
    __hip_atomic_store(&mirror->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Start of an inner PCG: clears the stop flag and sets the target r.r from
// the refinement residual's r.r (rr0 = res_norm2).
__global__ void k_pcg_begin(SolveScalars *sc, double tol2) {
    sc->done = 0;
    sc->iters = 0;
    sc->stall = 0;
    sc->bad &= ~2;
    sc->best = sc->res_norm2;
    sc->stop_rr = tol2 * sc->res_norm2;
}

// Orthonormal 1-D eigenbases and eigenvalues of the 7-point operator on the
// coarsest level, laid out for the eigen-solve kernels: phi_x [nx][nx],
// phi_y [ny][ny], phi_z [nz][nz] (mode-major), then lambda_x, lambda_y,
// lambda_z.  Mode m of an axis of n cells: Neumann k = m, cos(pi k (i + 1/2) / n)
// scaled by sqrt((k == 0 ? 1 : 2) / n); Dirichlet k = m + 1, sin(...) scaled by
// sqrt((k == n ? 1 : 2) / n); lambda = 4 sin^2(pi k / (2 n)).  Formed in FP64
// on the device, one entry per thread, so binding a solver copies nothing from
// the host.
__global__ void k_coarse_basis(float *__restrict__ E, int nx, int ny, int nz, int bc) {
    const int n[3] = {nx, ny, nz};
    const int nphi = nx * nx + ny * ny + nz * nz, total = nphi + nx + ny + nz;
    for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < total; o += gridDim.x * blockDim.x) {
        int r = o, a = 0;
        if (o < nphi) {
            while (r >= n[a] * n[a]) r -= n[a] * n[a], ++a;
            const int m = r / n[a], i = r % n[a];
            const int k = bc == WG_BC_NEUMANN ? m : m + 1;
            const double nrm = bc == WG_BC_NEUMANN ? sqrt((k == 0 ? 1.0 : 2.0) / n[a])
                                                   : sqrt((k == n[a] ? 1.0 : 2.0) / n[a]);
            const double t = M_PI * k * (i + 0.5) / n[a];
            E[o] = (float)(nrm * (bc == WG_BC_NEUMANN ? cos(t) : sin(t)));
        } else {
            r -= nphi;
            while (r >= n[a]) r -= n[a], ++a;
            const int k = bc == WG_BC_NEUMANN ? r : r + 1;
            const double sn = sin(M_PI * k / (2.0 * n[a]));
            E[o] = (float)(4.0 * sn * sn);
        }
    }
}

size_t basis_floats(const Dims &c) {
    return (size_t)c.nx * c.nx + (size_t)c.ny * c.ny + (size_t)c.nz * c.nz + c.nx + c.ny + c.nz;
}

// The multigrid hierarchy: one level when every extent is <= kDirectAxis (the
// exact solve alone preconditions), else halve every extent while all are
// even and >= 4 and one exceeds kCoarseTarget.  Returns the level count.
int level_dims(int nx, int ny, int nz, Dims (&out)[Solver::kMaxLevels]) {
    Dims d{nx, ny, nz, -1};
    int n = 0;
    out[n++] = d;
    if (nx <= kDirectAxis && ny <= kDirectAxis && nz <= kDirectAxis) return n;
    while (d.nx % 2 == 0 && d.ny % 2 == 0 && d.nz % 2 == 0 && d.nx >= 4 && d.ny >= 4 && d.nz >= 4 &&
           (d.nx > kCoarseTarget || d.ny > kCoarseTarget || d.nz > kCoarseTarget) && n < Solver::kMaxLevels) {
        d = Dims{d.nx / 2, d.ny / 2, d.nz / 2, -1};
        out[n++] = d;
    }
    return n;
}

// blocks of the sweep kernel that runs on grid d (its reductions write one partial per block)
unsigned sweep_blocks(const Dims &d) {
    return d.nx % 4 == 0 ? cdiv(waves4_of(d).tasks(), 4) : tiles_of(d).count();
}

// ... and of the 27-point sweep
unsigned sweep27_blocks(const Dims &d) {
    return d.nx % 4 == 0 ? cdiv(waves4_of(d).tasks(), 4) : tiles_of(d).count();
}

// blocks of the finest post-smoothing pass (0 for a single-level hierarchy)
unsigned post_blocks(const Dims *dims, int nl) { return nl > 1 ? vtile_of(dims[0]).count() : 0u; }

size_t partial_slots(const Dims *dims, int nl) {
    size_t nb = sweep_blocks(dims[0]);
    if (sweep27_blocks(dims[0]) > nb) nb = sweep27_blocks(dims[0]);
    const size_t pb = post_blocks(dims, nl);
    if (pb > nb) nb = pb;
    return (nb > (size_t)kRedBlocks ? nb : (size_t)kRedBlocks) * kMaxRed;
}

unsigned red_blocks(size_t n) {
    size_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < (size_t)kRedBlocks ? (b ? b : 1) : kRedBlocks);
}

}  // namespace

void Solver::plan(Arena &a, int nx, int ny, int nz) {
    Dims dims[kMaxLevels];
    const int nl = level_dims(nx, ny, nz, dims);
    size_t N = dims[0].count();
    // fine level: r, z, z2, e, p0, p1, q
    for (int k = 0; k < 7; ++k) a.reserve(N * sizeof(float));
    for (int l = 1; l < nl; ++l)
        for (int k = 0; k < 3; ++k) a.reserve(dims[l].count() * sizeof(float));
    a.reserve(partial_slots(dims, nl) * sizeof(double));
    a.reserve(sizeof(SolveScalars));
    a.reserve(sizeof(PublishedScalars));
    const Dims &c = dims[nl - 1];
    if (c.nx <= kDirectAxis && c.ny <= kDirectAxis && c.nz <= kDirectAxis)
        for (int bc = 0; bc < 2; ++bc) a.reserve(basis_floats(c) * sizeof(float));
}

void Solver::bind(Arena &a, int nx, int ny, int nz, hipStream_t s, bool mapped) {
    st_ = s;
    Dims dims[kMaxLevels];
    nlv_ = level_dims(nx, ny, nz, dims);
    size_t N = dims[0].count();
    Level &f = lv_[0];
    f.d = dims[0];
    f.rhs = a.take<float>(N);   // the CG residual r
    f.x = a.take<float>(N);     // z = M r
    f.x2 = a.take<float>(N);
    e_ = a.take<float>(N);
    p_[0] = a.take<float>(N);
    p_[1] = a.take<float>(N);
    q_ = a.take<float>(N);
    for (int l = 1; l < nlv_; ++l) {
        Level &L = lv_[l];
        L.d = dims[l];
        size_t n = dims[l].count();
        L.rhs = a.take<float>(n);
        L.x = a.take<float>(n);
        L.x2 = a.take<float>(n);
    }
    partials_ = a.take<double>(partial_slots(dims, nlv_));
    post_blocks_ = post_blocks(dims, nlv_);
    dsc_ = a.take<SolveScalars>(1);
    PublishedScalars *dev_rec = a.take<PublishedScalars>(1);
    mapped_ = mapped;
    if (mapped) {
        WG_HIP(hipHostMalloc((void **)&pub_, sizeof(PublishedScalars), hipHostMallocMapped | hipHostMallocCoherent));
        WG_HIP(hipHostGetDevicePointer((void **)&pub_dev_, pub_, 0));
        pub_->seq = seq_;
        pub_->status = 0;
        hsc_ = &pub_->s;
    } else {
        pub_dev_ = dev_rec;
        hsc_ = &host_pub_.s;
    }
    const Dims &c = dims[nlv_ - 1];
    coarse_direct_ = c.nx <= kDirectAxis && c.ny <= kDirectAxis && c.nz <= kDirectAxis;
    eig64_ = c.nx > 32 || c.ny > 32 || c.nz > 32;
    if (coarse_direct_) {
        const size_t nf = basis_floats(c);
        for (int bc = 0; bc < 2; ++bc) {
            coarseM_[bc] = a.take<float>(nf);
            k_coarse_basis<<<cdiv(nf, 256), 256, 0, st_>>>(coarseM_[bc], c.nx, c.ny, c.nz, bc);
            WG_LAUNCH_CHECK();
        }
    }
}

Solver::~Solver() {
    if (pub_) (void)hipHostFree(pub_);
}

void Solver::finalize(int mode, unsigned nb, int flag) {
    // FIN_RR publishes a status word with a sequence number of its own
    const unsigned seq = mode == FIN_RR ? ++sseq_ : (mode == FIN_RESID || mode == FIN_BSUM ? ++seq_ : 0u);
    k_finalize<<<1, 256, 0, st_>>>(partials_, nb, mode, flag, dsc_, (double)lv_[0].d.count(), pub_dev_, seq);
    WG_LAUNCH_CHECK();
}

// Wait until the last refinement finalize has published its scalars.
void Solver::read_scalars() {
    if (mapped_) {
        wait_published(&pub_->seq, seq_, st_);
    } else {
        WG_HIP(hipMemcpyAsync(&host_pub_, pub_dev_, sizeof(PublishedScalars), hipMemcpyDeviceToHost, st_));
        WG_HIP(hipStreamSynchronize(st_));
    }
}

// Wait until the status word carries sequence number `want` or a later one
// (a later iteration's word also tells whether the solve has stopped) and
// return it.
unsigned long long Solver::wait_status(unsigned want) {
    if (!mapped_) {
        WG_HIP(hipMemcpyAsync(&host_pub_, pub_dev_, sizeof(PublishedScalars), hipMemcpyDeviceToHost, st_));
        WG_HIP(hipStreamSynchronize(st_));
        return host_pub_.status;
    }
    for (unsigned k = 1;; ++k) {
        const unsigned long long st = __atomic_load_n(&pub_->status, __ATOMIC_ACQUIRE);
        if ((int)((unsigned)(st >> 32) - want) >= 0) return st;
        if ((k & 255) == 0) {
            const hipError_t e = hipStreamQuery(st_);
            if (e == hipSuccess) {
                const unsigned long long s2 = __atomic_load_n(&pub_->status, __ATOMIC_ACQUIRE);
                if ((int)((unsigned)(s2 >> 32) - want) >= 0) return s2;
                throw Error(WG_EDEVICE, "the solver's status never arrived");
            }
            if (e != hipErrorNotReady) hip_check(e, "hipStreamQuery", __FILE__, __LINE__);
        }
    }
}

// kind / bytes_per_cell: optional timing bracket (WG_PROF_*) and the sweep's
// algorithmic bytes per cell; skip: see skipped().
template <class Op>
static void launch_stencil(const Op &op, const Dims &d, double *partials, hipStream_t s, int kind = -1,
                           double bytes_per_cell = 0.0, const int *skip = nullptr) {
    prof::Scope ps(kind, s, bytes_per_cell * (double)d.count());
    if (d.nx % 4 == 0) {
        const Waves4 wv = waves4_of(d);
        k_stencil4<Op><<<cdiv(wv.tasks(), 4), 256, 0, s>>>(op, d, wv, partials, skip);
    } else {
        const Tiles t = tiles_of(d);
        k_stencil<Op><<<t.count(), TX * TY, 0, s>>>(op, d, t, partials, skip);
    }
    WG_LAUNCH_CHECK();
}

// The fine-level operator: the 7-point sweep, or (exact quadrature) the 27-point one.
template <class Op>
void Solver::sweep(const Op &op, int kind, double bytes_per_cell, const int *skip) {
    if (exact_) sweep27(op, kind, bytes_per_cell, skip);
    else launch_stencil(op, lv_[0].d, partials_, st_, kind, bytes_per_cell, skip);
}

template <class Op>
void Solver::sweep27(const Op &op, int kind, double bytes_per_cell, const int *skip) {
    const Dims &d = lv_[0].d;
    prof::Scope ps(kind, st_, bytes_per_cell * (double)d.count());
    if (d.nx % 4 == 0) {
        const Waves4 wv = waves4_of(d);
        k_stencil27x4<Op><<<cdiv(wv.tasks(), 4), 256, 0, st_>>>(op, d, wv, partials_, skip);
    } else {
        const Tiles t = tiles_of(d);
        k_stencil27<Op><<<t.count(), TX * TY, 0, st_>>>(op, d, t, partials_, skip);
    }
    WG_LAUNCH_CHECK();
}

unsigned Solver::sweep_partials() const { return exact_ ? sweep27_blocks(lv_[0].d) : sweep_blocks(lv_[0].d); }

void Solver::vcycle(int l) {
    Level &L = lv_[l];
    L.d.bc_sign = bc_sign_;
    const int last = nlv_ - 1;
    if (l == last) {
        if (coarse_direct_) {
            const float *E = coarseM_[bc_sign_ > 0 ? 1 : 0];
            if (eig64_) {
                k_eig_plane<64, true><<<L.d.nz, 256, 0, st_>>>(L.rhs, L.x2, E, L.d.nx, L.d.ny, skip_);
                k_eig_z<64><<<L.d.ny, 256, 0, st_>>>(L.x2, E, L.d.nx, L.d.ny, L.d.nz, skip_);
                k_eig_plane<64, false><<<L.d.nz, 256, 0, st_>>>(L.x2, L.x, E, L.d.nx, L.d.ny, skip_);
            } else {
                k_eig_plane<32, true><<<L.d.nz, 256, 0, st_>>>(L.rhs, L.x2, E, L.d.nx, L.d.ny, skip_);
                k_eig_z<32><<<L.d.ny, 256, 0, st_>>>(L.x2, E, L.d.nx, L.d.ny, L.d.nz, skip_);
                k_eig_plane<32, false><<<L.d.nz, 256, 0, st_>>>(L.x2, L.x, E, L.d.nx, L.d.ny, skip_);
            }
            WG_LAUNCH_CHECK();
        } else {
            // no direct solve possible (odd extents): a fixed, even number of sweeps
            launch_stencil(OpSmoothFirst{L.rhs, L.x2, kOmega}, L.d, nullptr, st_, -1, 0.0, skip_);
            for (int k = 0; k < 15; ++k) {
                launch_stencil(OpSmooth{L.x2, L.rhs, L.x, kOmega}, L.d, nullptr, st_, -1, 0.0, skip_);
                launch_stencil(OpSmooth{L.x, L.rhs, L.x2, kOmega}, L.d, nullptr, st_, -1, 0.0, skip_);
            }
            launch_stencil(OpSmooth{L.x2, L.rhs, L.x, kOmega}, L.d, nullptr, st_, -1, 0.0, skip_);
        }
        return;
    }
    Level &C = lv_[l + 1];
    C.d.bc_sign = bc_sign_;
    const int ks = l == 0 ? pk(WG_PROF_SMOOTH) : -1, kt = l == 0 ? pk(WG_PROF_TRANSFER) : -1;
    const VTile vt = vtile_of(L.d);
    {
        // rhs read, x written; 1/8 of a cell's bytes for the coarse rhs
        prof::Scope ps(ks, st_, 8.0 * (double)L.d.count() + 4.0 * (double)C.d.count());
        k_vc_pre<<<vt.count(), kVB, 0, st_>>>(L.rhs, L.x, C.rhs, L.d, C.d, vt, kChebWa, kChebWb, skip_);
        WG_LAUNCH_CHECK();
    }
    vcycle(l + 1);
    {
        // x and rhs read, the result written, the coarse correction read
        prof::Scope ps(kt, st_, 12.0 * (double)L.d.count() + 4.0 * (double)C.d.count());
        if (l == 0)   // + r.z
            k_vc_post<true><<<vt.count(), kVB, 0, st_>>>(L.x, L.rhs, C.x, L.x2, L.d, C.d, vt, kChebWb, kChebWa,
                                                           partials_, skip_);
        else
            k_vc_post<false><<<vt.count(), kVB, 0, st_>>>(L.x, L.rhs, C.x, L.x2, L.d, C.d, vt, kChebWb, kChebWa,
                                                            nullptr, skip_);
        WG_LAUNCH_CHECK();
        std::swap(L.x, L.x2);
    }
}

// z = M r with r.z summed into partials_ (rz_blocks() of them).
void Solver::precond() {
    if (exact_) {
        // M7 between two Jacobi steps on the 27-point operator; q_ (free
        // until the next direction's matvec) takes the first step's output
        Level &F = lv_[0];
        float *r = F.rhs;
        sweep27(OpJacobi27a{r, q_, kJacobi27}, pk(WG_PROF_SMOOTH), 8.0, skip_);
        F.rhs = q_;
        vcycle(0);
        F.rhs = r;
        sweep27(OpJacobi27b{r, F.x, F.x2, kJacobi27}, pk(WG_PROF_SMOOTH), 12.0, skip_);
        std::swap(F.x, F.x2);
        return;
    }
    vcycle(0);
    if (nlv_ == 1) {
        // the coarsest solve alone forms no sum: one more pass
        Level &F = lv_[0];
        const size_t N = F.d.count();
        k_dot<<<red_blocks(N), kBlock, 0, st_>>>(F.rhs, F.x, N, partials_, skip_);
        WG_LAUNCH_CHECK();
    }
}

unsigned Solver::rz_blocks() const {
    if (exact_) return sweep27_blocks(lv_[0].d);
    return nlv_ > 1 ? post_blocks_ : red_blocks(lv_[0].d.count());
}

void Solver::mg_apply(const float *r, float *z, int bc) {
    require(bc == WG_BC_NEUMANN || bc == WG_BC_DIRICHLET, WG_EINVAL, "unknown boundary condition");
    bc_sign_ = bc == WG_BC_NEUMANN ? -1 : +1;
    for (int l = 0; l < nlv_; ++l) lv_[l].d.bc_sign = bc_sign_;
    Level &F = lv_[0];
    const size_t N = F.d.count();
    WG_HIP(hipMemcpyAsync(F.rhs, r, N * sizeof(float), hipMemcpyDeviceToDevice, st_));
    vcycle(0);
    WG_HIP(hipMemcpyAsync(z, F.x, N * sizeof(float), hipMemcpyDeviceToDevice, st_));
}

// Iteration `it` of the inner PCG: for it > 0 first z = M r and beta (the
// step after the last r.r test), then the direction with q = A p and alpha,
// the update of the correction and of r, and the r.r finalize that decides
// on the device whether to stop.  Every kernel returns at once once stopped.
void Solver::pcg_iteration(int it, int &cur) {
    Level &F = lv_[0];
    const size_t N = F.d.count();
    if (it > 0) {
        precond();   // z for the next direction
        finalize(FIN_RZ, rz_blocks(), 0);   // beta = rz / rz_old
        cur ^= 1;
    }
    if (it == 0)
        sweep(OpPMatvec<true>{F.x, nullptr, p_[cur], q_, nullptr, 0.f}, pk(WG_PROF_SWEEP), 12.0, skip_);
    else   // beta = rz / rz_old, formed by the last finalize, read on the device
        sweep(OpPMatvec<false>{F.x, p_[cur ^ 1], p_[cur], q_, dsc_, 0.f}, pk(WG_PROF_SWEEP), 16.0, skip_);
    finalize(FIN_PQ, sweep_partials(), 0);
    const unsigned rb = red_blocks(N);
    {
        prof::Scope ps(pk(WG_PROF_CGUPDATE), st_, (it == 0 ? 20.0 : 24.0) * (double)N);
        if (it == 0)
            k_cg_update<true><<<rb, kBlock, 0, st_>>>(e_, F.rhs, p_[cur], q_, dsc_, N, partials_);
        else
            k_cg_update<false><<<rb, kBlock, 0, st_>>>(e_, F.rhs, p_[cur], q_, dsc_, N, partials_);
        WG_LAUNCH_CHECK();
    }
    finalize(FIN_RR, rb, 0);
}

// Inner PCG on A e = r (r in the finest level's rhs) from e = 0, to r.r <=
// tol^2 r0.r0 or max_it iterations.  The host keeps one iteration enqueued
// beyond the one whose status it waits for, so the device does not idle
// through a host round trip; the iteration after the stopping one returns
// at once in every kernel.  Returns the iterations taken.
int Solver::pcg(double tol, int max_it, bool &non_finite) {
    non_finite = false;
    k_pcg_begin<<<1, 1, 0, st_>>>(dsc_, tol * tol);
    WG_LAUNCH_CHECK();
    skip_ = &dsc_->done;
    // z = M r, rz = r.z ; the first finalize must not form beta
    precond();
    finalize(FIN_RZ, rz_blocks(), 1);
    int cur = 0, enq = 0, checked = 0, iters = 0;
    unsigned seq_of[2] = {0, 0};
    // timing records of each iteration are grouped, so that those of an
    // iteration that returned at once can be dropped
    static std::atomic<unsigned long long> next_group{1};
    unsigned long long group_of[2] = {0, 0};
    auto push = [&] {
        group_of[enq % 2] = instrument_ ? next_group.fetch_add(1) : 0ull;
        prof::set_group(group_of[enq % 2]);
        pcg_iteration(enq, cur);
        prof::set_group(0);
        seq_of[enq % 2] = sseq_;
        ++enq;
    };
    push();
    for (;;) {
        if (enq < max_it) push();
        const unsigned long long st = wait_status(seq_of[checked % 2]);
        ++checked;
        iters = (int)((st >> 2) & 0x3fffffffu);
        if (st & 3u) {
            non_finite = (st & 2u) != 0;
            break;
        }
        if (checked == enq) break;   // the budget is spent
    }
    if (enq > iters) prof::drop_group(group_of[(enq - 1) % 2]);   // enqueued after the stop: did nothing
    skip_ = nullptr;
    return iters;
}

SolveResult Solver::solve(const float *b, double *x, int bc, const wg_solve_opts &o) { return solve_impl(b, x, bc, o); }
SolveResult Solver::solve(const double *b, double *x, int bc, const wg_solve_opts &o) { return solve_impl(b, x, bc, o); }

template <class TB>
SolveResult Solver::solve_impl(const TB *b, double *x, int bc, const wg_solve_opts &o) {
    require(bc == WG_BC_NEUMANN || bc == WG_BC_DIRICHLET, WG_EINVAL, "unknown boundary condition");
    require(o.quadrature == WG_VERTEX_QUADRATURE || o.quadrature == WG_EXACT_QUADRATURE, WG_EINVAL,
            "unknown quadrature");
    require(o.quadrature == WG_VERTEX_QUADRATURE || bc == WG_BC_NEUMANN, WG_EINVAL,
            "exact quadrature is defined for zero-flux boundaries only");
    exact_ = o.quadrature == WG_EXACT_QUADRATURE;
    bc_sign_ = bc == WG_BC_NEUMANN ? -1 : +1;
    for (int l = 0; l < nlv_; ++l) lv_[l].d.bc_sign = bc_sign_;
    Level &F = lv_[0];
    const size_t N = F.d.count();
    const unsigned tb = sweep_partials();
    const unsigned gb = red_blocks(N);
    SolveResult res;
    static_assert(sizeof(SolveScalars) % 4 == 0, "scalars are whole words");
    k_zero_words<<<1, 64, 0, st_>>>(reinterpret_cast<uint32_t *>(dsc_), sizeof(SolveScalars) / 4);
    WG_LAUNCH_CHECK();
    if (!o.warm_start) {
        k_fill64<<<gb, kBlock, 0, st_>>>(x, 0.0, N);
        WG_LAUNCH_CHECK();
    }
    // Neumann: the residual kernel subtracts the mean of b, formed on the device
    const SolveScalars *mean_src = nullptr;
    if (bc == WG_BC_NEUMANN) {
        k_sum<TB><<<gb, kBlock, 0, st_>>>(b, N, partials_);
        WG_LAUNCH_CHECK();
        finalize(FIN_BSUM, gb, 0);
        mean_src = dsc_;
    }
    const double tol = o.rel_tol > 0 ? o.rel_tol : 1e-6;
    const int max_iters = o.max_iters > 0 ? o.max_iters : 500;
    double bnorm = -1.0;
    for (;;) {
        sweep(OpResid64<TB>{x, b, F.rhs, mean_src, 0.0}, pk(WG_PROF_RESID64), 12.0 + sizeof(TB), nullptr);
        finalize(FIN_RESID, tb, bc == WG_BC_NEUMANN);
        read_scalars();
        ++res.refinements;
        if (hsc_->bad) {
            res.status = WG_ENUMERIC;
            res.rel_res = NAN;
            return res;
        }
        if (bnorm < 0) bnorm = std::sqrt(hsc_->b_norm2);
        const double rnorm = std::sqrt(hsc_->res_norm2);
        res.x_mean = hsc_->x_sum / (double)N;
        if (bnorm == 0.0) {
            res.rel_res = 0.0;
            if (rnorm == 0.0) break;
            // b vanishes: the solution is x = 0
            k_fill64<<<gb, kBlock, 0, st_>>>(x, 0.0, N);
            WG_LAUNCH_CHECK();
            res.x_mean = 0.0;
            break;
        }
        res.rel_res = rnorm / bnorm;
        if (res.rel_res <= tol) break;
        if (res.iters >= max_iters || res.refinements > 40) {
            res.status = WG_ENOTCONV;
            break;
        }
        double inner = 0.5 * tol / res.rel_res;
        // FP32 vectors reach about 1e-7 relative: aim no lower than 1e-6 per inner solve
        if (inner < 1e-6) inner = 1e-6;
        if (inner > 0.5) inner = 0.5;
        int budget = max_iters - res.iters;
        if (budget > 60) budget = 60;
        bool non_finite = false;
        res.iters += pcg(inner, budget, non_finite);
        if (non_finite) {
            res.status = WG_ENUMERIC;
            res.rel_res = NAN;
            return res;
        }
        k_axpy64<<<gb, kBlock, 0, st_>>>(x, e_, N);
        WG_LAUNCH_CHECK();
    }
    return res;
}

void Solver::shift(double *x, double by) {
    const size_t N = lv_[0].d.count();
    k_shift64<<<red_blocks(N), kBlock, 0, st_>>>(x, by, N);
    WG_LAUNCH_CHECK();
}

}  // namespace wg
