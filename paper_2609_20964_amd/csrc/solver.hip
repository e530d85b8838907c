// Matrix-free multigrid-preconditioned CG for the grid Poisson problem.
//
// Hot kernels are 2.5-D sweeps: a 64 x 4 workgroup tile of (x, y) columns
// marches ZC planes in z, keeping the z-1, z, z+1 values in registers and
// reading x/y neighbours through the caches; x is the fastest (coalesced)
// axis.  Blocks are remapped so that each XCD sweeps one contiguous slab.
// Every reduction is two-stage and deterministic: one FP64 partial per block
// (fixed block order), summed by a single-block finalize kernel.
#include <cmath>

#include "prof.h"
#include "solver.h"

namespace wg {

namespace {

constexpr int TX = 64, TY = 4, ZC = 16;
constexpr int kRedBlocks = 2048;     // grid of the pointwise reductions
constexpr int kMaxRed = 5;
constexpr float kOmega = 6.0f / 7.0f;   // weighted-Jacobi factor of the sweeps on an odd-sized coarsest level
constexpr int kCoarseTarget = 16;       // coarsen until every extent is <= this (or odd)
constexpr int kCoarseAxis = 16;         // exact coarsest solve when every extent is <= this

struct Tiles {
    unsigned gx, gy, gz;
    __host__ __device__ unsigned count() const { return gx * gy * gz; }
};
Tiles tiles_of(const Dims &d) { return {cdiv(d.nx, TX), cdiv(d.ny, TY), cdiv(d.nz, ZC)}; }

// Generic 7-point sweep.  Op::load(idx) yields the stencil input at a linear
// index; Op::apply(idx, centre, neighbour_sum, diag, acc) consumes one cell.
template <class Op>
__global__ __launch_bounds__(256) void k_stencil(Op op, Dims d, Tiles t, double *partials) {
    using T = typename Op::T;
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
__global__ __launch_bounds__(256) void k_stencil4(Op op, Dims d, Waves4 wv, double *partials) {
    using T = typename Op::T;
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
        V4<T> cm, cc;
        for (int q = 0; q < 4; ++q) cm.v[q] = T(0);
        if (valid && z0 > 0) cm = op.load4(base + (size_t)(z0 - 1) * plane);
        if (valid) cc = op.load4(base + (size_t)z0 * plane);
        else for (int q = 0; q < 4; ++q) cc.v[q] = T(0);
        for (int k = z0; k < z1; ++k) {
            const size_t idx = base + (size_t)k * plane;
            const bool zp = k + 1 < d.nz;
            V4<T> cp, a, b;
            for (int q = 0; q < 4; ++q) cp.v[q] = a.v[q] = b.v[q] = T(0);
            if (valid && zp) cp = op.load4(idx + plane);
            if (valid && ym) a = op.load4(idx - d.nx);
            if (valid && yp) b = op.load4(idx + d.nx);
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
struct OpResid64 {
    using T = double;
    static constexpr int NRED = 5;
    const double *x;
    const float *b;
    float *r;
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
        const V4<float> bb = ld4(b + i);
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

struct OpSmooth2 {
    using T = float;
    static constexpr int NRED = 0;
    const float *rhs;
    float *out;
    float wa, wb;
    __device__ float load(size_t i) const { return rhs[i]; }
    __device__ float load1(size_t i) const { return rhs[i]; }
    __device__ V4<float> load4(size_t i) const { return ld4(rhs + i); }
    __device__ void apply(size_t i, float c, float s, float diag, double *) const {
        out[i] = wa * c + wb * (c - wa * (diag * c - s));
    }
    __device__ void apply4(size_t i, const V4<float> &c, const V4<float> &s, const V4<float> &dg, double *) const {
        V4<float> o;
        for (int q = 0; q < 4; ++q) o.v[q] = wa * c.v[q] + wb * (c.v[q] - wa * (dg.v[q] * c.v[q] - s.v[q]));
        st4(out + i, o);
    }
};

// Weighted-Jacobi sweep x_out = x + w (rhs - A x) / diag; DOT adds rhs . x_out.
template <bool DOT>
struct OpSmooth {
    using T = float;
    static constexpr int NRED = DOT ? 1 : 0;
    const float *x, *rhs;
    float *out;
    float w;
    __device__ float load(size_t i) const { return x[i]; }
    __device__ float load1(size_t i) const { return x[i]; }
    __device__ V4<float> load4(size_t i) const { return ld4(x + i); }
    __device__ void apply(size_t i, float c, float s, float diag, double *acc) const {
        float rv = rhs[i];
        float v = c + w * (rv - (diag * c - s)) / diag;
        out[i] = v;
        if constexpr (DOT) acc[0] += (double)rv * (double)v;
    }
    __device__ void apply4(size_t i, const V4<float> &c, const V4<float> &s, const V4<float> &dg, double *acc) const {
        const V4<float> r = ld4(rhs + i);
        V4<float> o;
        for (int q = 0; q < 4; ++q) {
            o.v[q] = c.v[q] + w * (r.v[q] - (dg.v[q] * c.v[q] - s.v[q])) / dg.v[q];
            if constexpr (DOT) acc[0] += (double)r.v[q] * (double)o.v[q];
        }
        st4(out + i, o);
    }
};

// Post-smoothing sweep with the constant diagonal: x_out = x + wd (rhs - A x);
// DOT adds rhs . x_out.
template <bool DOT>
struct OpSmoothC {
    using T = float;
    static constexpr int NRED = DOT ? 1 : 0;
    const float *x, *rhs;
    float *out;
    float wd;
    __device__ float load(size_t i) const { return x[i]; }
    __device__ float load1(size_t i) const { return x[i]; }
    __device__ V4<float> load4(size_t i) const { return ld4(x + i); }
    __device__ void apply(size_t i, float c, float s, float diag, double *acc) const {
        float rv = rhs[i];
        float v = c + wd * (rv - (diag * c - s));
        out[i] = v;
        if constexpr (DOT) acc[0] += (double)rv * (double)v;
    }
    __device__ void apply4(size_t i, const V4<float> &c, const V4<float> &s, const V4<float> &dg, double *acc) const {
        const V4<float> r = ld4(rhs + i);
        V4<float> o;
        for (int q = 0; q < 4; ++q) {
            o.v[q] = c.v[q] + wd * (r.v[q] - (dg.v[q] * c.v[q] - s.v[q]));
            if constexpr (DOT) acc[0] += (double)r.v[q] * (double)o.v[q];
        }
        st4(out + i, o);
    }
};

// out = rhs - A x.
struct OpResid {
    using T = float;
    static constexpr int NRED = 0;
    const float *x, *rhs;
    float *out;
    __device__ float load(size_t i) const { return x[i]; }
    __device__ float load1(size_t i) const { return x[i]; }
    __device__ V4<float> load4(size_t i) const { return ld4(x + i); }
    __device__ void apply(size_t i, float c, float s, float diag, double *) const {
        out[i] = rhs[i] - (diag * c - s);
    }
    __device__ void apply4(size_t i, const V4<float> &c, const V4<float> &s, const V4<float> &dg, double *) const {
        const V4<float> r = ld4(rhs + i);
        V4<float> o;
        for (int q = 0; q < 4; ++q) o.v[q] = r.v[q] - (dg.v[q] * c.v[q] - s.v[q]);
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
};

template <bool FIRST>
__global__ __launch_bounds__(256) void k_cg_update(float *__restrict__ x, float *__restrict__ r,
                                                    const float *__restrict__ p, const float *__restrict__ q,
                                                    const SolveScalars *sc, size_t n, double *partials) {
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

__global__ __launch_bounds__(256) void k_sum(const float *__restrict__ x, size_t n, double *partials) {
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

// coarse = 1/2 P^T fine (P = cell-centred trilinear prolongation).
__global__ __launch_bounds__(256) void k_restrict(const float *__restrict__ fine, Dims df,
                                                   float *__restrict__ coarse, Dims dc) {
    size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= dc.count()) return;
    int I = idx % dc.nx, J = (idx / dc.nx) % dc.ny, K = idx / ((size_t)dc.nx * dc.ny);
    const int s = -dc.bc_sign;    // mirror sign: +1 Neumann, -1 Dirichlet
    float acc = 0.f;
    for (int tz = 0; tz < 4; ++tz) {
        float wz = restrict_w(tz, K, dc.nz, s);
        if (wz == 0.f) continue;
        int fk = 2 * K - 1 + tz;
        for (int ty = 0; ty < 4; ++ty) {
            float wy = restrict_w(ty, J, dc.ny, s);
            if (wy == 0.f) continue;
            int fj = 2 * J - 1 + ty;
            const float *row = fine + ((size_t)fk * df.ny + fj) * df.nx;
            float ax = 0.f;
            for (int tx = 0; tx < 4; ++tx) {
                float wx = restrict_w(tx, I, dc.nx, s);
                if (wx != 0.f) ax += wx * row[2 * I - 1 + tx];
            }
            acc += wz * wy * ax;
        }
    }
    coarse[idx] = 0.5f * acc;
}

__device__ __forceinline__ void prolong_1d(int f, int nc, int s, int &I, int &J, float &wI, float &wJ) {
    I = f >> 1;
    J = (f & 1) ? I + 1 : I - 1;
    wI = 0.75f;
    wJ = 0.25f;
    if (J < 0 || J >= nc) {
        wI += 0.25f * s;
        wJ = 0.f;
        J = I;
    }
}

// fine += P coarse.
__global__ __launch_bounds__(256) void k_prolong_add(const float *__restrict__ coarse, Dims dc,
                                                      float *__restrict__ fine, Dims df) {
    size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= df.count()) return;
    int i = idx % df.nx, j = (idx / df.nx) % df.ny, k = idx / ((size_t)df.nx * df.ny);
    const int s = -dc.bc_sign;
    int I[2], Jy[2], K[2];
    float wx[2], wy[2], wz[2];
    prolong_1d(i, dc.nx, s, I[0], I[1], wx[0], wx[1]);
    prolong_1d(j, dc.ny, s, Jy[0], Jy[1], wy[0], wy[1]);
    prolong_1d(k, dc.nz, s, K[0], K[1], wz[0], wz[1]);
    float acc = 0.f;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a)
                acc += wz[c] * wy[b] * wx[a] * coarse[((size_t)K[c] * dc.ny + Jy[b]) * dc.nx + I[a]];
    fine[idx] += acc;
}

// Vector transfers (fine x extent divisible by 4).  Lane layout as in
// k_stencil4: a wavefront covers R rows x L float4 columns of the fine grid;
// one fine float4 covers two coarse cells in x.

// coarse = 1/2 P^T fine: a wavefront takes R coarse rows J (fine rows
// 2J-1 .. 2J+2) and marches over coarse planes K.
__global__ __launch_bounds__(256) void k_restrict4(const float *__restrict__ fine, Dims df, float *__restrict__ coarse,
                                                   Dims dc, Waves4 wv) {
    const unsigned task = blockIdx.x * 4 + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    if (task >= wv.tasks()) return;   // whole wavefront
    const int s = -dc.bc_sign;
    const unsigned W4 = (unsigned)df.nx / 4;
    const unsigned seg = task % wv.S, grp = (task / wv.S) % wv.G, zc = task / (wv.S * wv.G);
    const unsigned sl = lane % wv.L, rr = lane / wv.L;
    const unsigned t = seg * wv.L + sl;                  // fine float4 column = coarse pair (2t, 2t+1)
    const int J = (int)(grp * wv.R + rr);
    const bool valid = rr < wv.R && t < W4 && J < dc.ny;
    const bool shl = sl > 0, shr = sl + 1 < wv.L && t + 1 < W4;
    const int I0 = 2 * (int)t, I1 = I0 + 1;
    // x weights of the 6 fine cells 4t-1 .. 4t+4 for coarse I0 and I1
    const float a0 = restrict_w(0, I0, dc.nx, s), a1 = restrict_w(1, I0, dc.nx, s), a2 = restrict_w(2, I0, dc.nx, s),
                a3 = restrict_w(3, I0, dc.nx, s);
    const float b0 = restrict_w(0, I1, dc.nx, s), b1 = restrict_w(1, I1, dc.nx, s), b2 = restrict_w(2, I1, dc.nx, s),
                b3 = restrict_w(3, I1, dc.nx, s);
    const int K0 = (int)(zc * wv.zlen), K1 = min(K0 + (int)wv.zlen, dc.nz);
    const size_t fplane = (size_t)df.nx * df.ny;
    // y-reduced, x-restricted value pair of fine plane p
    auto yx = [&](int p, float &v0, float &v1) {
        v0 = v1 = 0.f;
        for (int ty = 0; ty < 4; ++ty) {
            const int fj = 2 * J - 1 + ty;
            const float wy = valid ? restrict_w(ty, J, dc.ny, s) : 0.f;
            float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
            const bool inrow = valid && wy != 0.f && p >= 0 && p < df.nz;
            const size_t o = inrow ? (size_t)4 * t + (size_t)df.nx * fj + fplane * p : 0;
            if (inrow) q = *reinterpret_cast<const float4 *>(fine + o);
            float left = __shfl_up(q.w, 1, 64), right = __shfl_down(q.x, 1, 64);
            if (!shl) left = (inrow && t > 0) ? fine[o - 1] : 0.f;
            if (!shr) right = (inrow && t + 1 < W4) ? fine[o + 4] : 0.f;
            const float x0 = a0 * left + a1 * q.x + a2 * q.y + a3 * q.z;
            const float x1 = b0 * q.y + b1 * q.z + b2 * q.w + b3 * right;
            v0 += wy * x0;
            v1 += wy * x1;
        }
    };
    // rolling y-reduced planes 2K-1 .. 2K+2
    float m0, m1, c0, c1;           // planes 2K-1, 2K
    yx(2 * K0 - 1, m0, m1);
    yx(2 * K0, c0, c1);
    for (int K = K0; K < K1; ++K) {
        float p0, p1, q0, q1;       // planes 2K+1, 2K+2
        yx(2 * K + 1, p0, p1);
        yx(2 * K + 2, q0, q1);
        const float w0 = restrict_w(0, K, dc.nz, s), w1 = restrict_w(1, K, dc.nz, s),
                    w2 = restrict_w(2, K, dc.nz, s), w3 = restrict_w(3, K, dc.nz, s);
        if (valid) {
            const float r0 = 0.5f * (w0 * m0 + w1 * c0 + w2 * p0 + w3 * q0);
            const float r1 = 0.5f * (w0 * m1 + w1 * c1 + w2 * p1 + w3 * q1);
            *reinterpret_cast<float2 *>(coarse + (size_t)I0 + (size_t)dc.nx * (J + (size_t)dc.ny * K)) =
                make_float2(r0, r1);
        }
        m0 = p0; m1 = p1; c0 = q0; c1 = q1;
    }
}

// fine += P coarse: a wavefront takes R fine rows j and marches over fine
// planes in pairs (2K, 2K+1), which share coarse planes K-1 .. K+1.
__global__ __launch_bounds__(256) void k_prolong4(const float *__restrict__ coarse, Dims dc, float *__restrict__ fine,
                                                  Dims df, Waves4 wv) {
    const unsigned task = blockIdx.x * 4 + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    if (task >= wv.tasks()) return;   // whole wavefront
    const int s = -dc.bc_sign;
    const unsigned W4 = (unsigned)df.nx / 4;
    const unsigned seg = task % wv.S, grp = (task / wv.S) % wv.G, zc = task / (wv.S * wv.G);
    const unsigned sl = lane % wv.L, rr = lane / wv.L;
    const unsigned t = seg * wv.L + sl;
    const int j = (int)(grp * wv.R + rr);
    const bool valid = rr < wv.R && t < W4 && j < df.ny;
    const bool shl = sl > 0, shr = sl + 1 < wv.L && t + 1 < W4;
    // y: coarse rows and weights
    int Jy[2];
    float wy[2];
    prolong_1d(valid ? j : 0, dc.ny, s, Jy[0], Jy[1], wy[0], wy[1]);
    const bool lb = 2 * (int)t - 1 >= 0, rb = 2 * (int)t + 2 < dc.nx;   // coarse x neighbours exist
    // x-interpolated fine quad from coarse row (J, K)
    auto xrow = [&](int J, int K, float4 &o) {
        float2 c = make_float2(0.f, 0.f);
        const size_t base = (size_t)dc.nx * (J + (size_t)dc.ny * K);
        if (valid) c = *reinterpret_cast<const float2 *>(coarse + base + 2 * t);
        float l = __shfl_up(c.y, 1, 64), r = __shfl_down(c.x, 1, 64);
        if (!shl) l = (valid && lb) ? coarse[base + 2 * t - 1] : 0.f;
        if (!shr) r = (valid && rb) ? coarse[base + 2 * t + 2] : 0.f;
        o.x = lb ? 0.75f * c.x + 0.25f * l : (0.75f + 0.25f * s) * c.x;
        o.y = 0.75f * c.x + 0.25f * c.y;
        o.z = 0.75f * c.y + 0.25f * c.x;
        o.w = rb ? 0.75f * c.y + 0.25f * r : (0.75f + 0.25f * s) * c.y;
    };
    auto yrow = [&](int K, float4 &o) {   // y-combined quad at coarse plane K for fine row j
        float4 a, b;
        xrow(Jy[0], K, a);
        xrow(Jy[1], K, b);
        o = make_float4(wy[0] * a.x + wy[1] * b.x, wy[0] * a.y + wy[1] * b.y, wy[0] * a.z + wy[1] * b.z,
                        wy[0] * a.w + wy[1] * b.w);
    };
    const int k0 = (int)(zc * wv.zlen), k1 = min(k0 + (int)wv.zlen, df.nz);   // zlen even: k0 even
    const size_t fplane = (size_t)df.nx * df.ny;
    for (int k = k0; k < k1; k += 2) {
        const int K = k >> 1;
        float4 cm, cc, cp;
        yrow(K > 0 ? K - 1 : K, cm);
        yrow(K, cc);
        yrow(K + 1 < dc.nz ? K + 1 : K, cp);
        for (int h = 0; h < 2 && k + h < k1; ++h) {
            // fine plane k+h: even -> (K, K-1), odd -> (K, K+1); mirror at the ends
            const bool odd = h == 1;
            const bool inb = odd ? (K + 1 < dc.nz) : (K > 0);
            const float wK = inb ? 0.75f : 0.75f + 0.25f * s, wN = inb ? 0.25f : 0.f;
            const float4 &N = odd ? cp : cm;
            if (valid) {
                float4 *f = reinterpret_cast<float4 *>(fine + (size_t)4 * t + (size_t)df.nx * j + fplane * (k + h));
                float4 v = *f;
                v.x += wK * cc.x + wN * N.x;
                v.y += wK * cc.y + wN * N.y;
                v.z += wK * cc.z + wN * N.z;
                v.w += wK * cc.w + wN * N.w;
                *f = v;
            }
        }
    }
}

// Exact solve on the coarsest level (every extent <= kCoarseAxis = 16) by the
// separable eigenbasis of the 7-point operator: transform along x, y, z with
// the orthonormal 1-D bases, divide by lambda_x + lambda_y + lambda_z (the
// constant mode is dropped), transform back.  One workgroup of 16 x 16
// threads; the field sits in LDS as [k][j][i] (row length padded to 17 so the
// strided line reads are free of bank conflicts), each thread transforms whole
// lines held in registers, and the bases sit in LDS zero-padded to 16 x 16
// (every lane reads the same entry: a broadcast).  E = [phi_x (cx*cx),
// phi_y (cy*cy), phi_z (cz*cz), lam_x, lam_y, lam_z], phi_a[m * n_a + i] =
// mode m at cell i.
constexpr int kEigPad = kCoarseAxis + 1;
constexpr int kEigB = kCoarseAxis * kCoarseAxis;

// out[m] = sum_i P[m][i] in[i] (FWD) or sum_i P[i][m] in[i] (inverse), P padded 16 x 16
template <bool FWD>
__device__ __forceinline__ void eig_line(const float *P, const float (&in)[kCoarseAxis], float (&out)[kCoarseAxis]) {
#pragma unroll
    for (int m = 0; m < kCoarseAxis; ++m) out[m] = 0.f;
#pragma unroll
    for (int i = 0; i < kCoarseAxis; ++i) {
#pragma unroll
        for (int m = 0; m < kCoarseAxis; ++m) out[m] += P[FWD ? m * kCoarseAxis + i : i * kCoarseAxis + m] * in[i];
    }
}

__global__ __launch_bounds__(256) void k_coarse_eig(const float *__restrict__ rhs, float *__restrict__ x,
                                                     const float *__restrict__ E, int cx, int cy, int cz) {
    __shared__ float L[kCoarseAxis * kCoarseAxis * kEigPad];
    __shared__ float Pm[3 * kEigB + 3 * kCoarseAxis];
    const int n = cx * cy * cz;
    const int ext[3] = {cx, cy, cz};
    {
        const float *src = E;
        for (int a = 0; a < 3; ++a) {
            const int na = ext[a];
            for (int o = threadIdx.x; o < kEigB; o += blockDim.x) {
                const int m = o / kCoarseAxis, i = o % kCoarseAxis;
                Pm[a * kEigB + o] = (m < na && i < na) ? src[m * na + i] : 0.f;
            }
            src += na * na;
        }
        for (int a = 0; a < 3; ++a) {
            const int na = ext[a];
            for (int o = threadIdx.x; o < kCoarseAxis; o += blockDim.x) Pm[3 * kEigB + a * kCoarseAxis + o] = o < na ? src[o] : 0.f;
            src += na;
        }
    }
    const float *Px = Pm, *Py = Pm + kEigB, *Pz = Pm + 2 * kEigB;
    const float *Lx = Pm + 3 * kEigB, *Ly = Lx + kCoarseAxis, *Lz = Ly + kCoarseAxis;
    auto at = [](int i, int j, int k) { return i + kEigPad * (j + kCoarseAxis * k); };
    for (int o = threadIdx.x; o < kCoarseAxis * kCoarseAxis * kEigPad; o += blockDim.x) L[o] = 0.f;
    __syncthreads();
    for (int o = threadIdx.x; o < n; o += blockDim.x) {
        const int i = o % cx, j = (o / cx) % cy, k = o / (cx * cy);
        L[at(i, j, k)] = rhs[o];
    }
    __syncthreads();
    const int u = threadIdx.x % kCoarseAxis, v = threadIdx.x / kCoarseAxis;
    float in[kCoarseAxis], out[kCoarseAxis];
    // forward x: line (j, k) = (u, v)
    for (int i = 0; i < kCoarseAxis; ++i) in[i] = L[at(i, u, v)];
    eig_line<true>(Px, in, out);
    for (int i = 0; i < kCoarseAxis; ++i) L[at(i, u, v)] = out[i];
    __syncthreads();
    // forward y: line (i, k) = (u, v)
    for (int j = 0; j < kCoarseAxis; ++j) in[j] = L[at(u, j, v)];
    eig_line<true>(Py, in, out);
    for (int j = 0; j < kCoarseAxis; ++j) L[at(u, j, v)] = out[j];
    __syncthreads();
    // forward z, divide by the eigenvalue (0 for the constant mode and the padding), inverse z: line (i, j)
    for (int k = 0; k < kCoarseAxis; ++k) in[k] = L[at(u, v, k)];
    eig_line<true>(Pz, in, out);
    for (int k = 0; k < kCoarseAxis; ++k) {
        const float lam = Lx[u] + Ly[v] + Lz[k];
        in[k] = (u < cx && v < cy && k < cz && lam > 1e-12f) ? out[k] / lam : 0.f;
    }
    eig_line<false>(Pz, in, out);
    for (int k = 0; k < kCoarseAxis; ++k) L[at(u, v, k)] = out[k];
    __syncthreads();
    // inverse y
    for (int j = 0; j < kCoarseAxis; ++j) in[j] = L[at(u, j, v)];
    eig_line<false>(Py, in, out);
    for (int j = 0; j < kCoarseAxis; ++j) L[at(u, j, v)] = out[j];
    __syncthreads();
    // inverse x
    for (int i = 0; i < kCoarseAxis; ++i) in[i] = L[at(i, u, v)];
    eig_line<false>(Px, in, out);
    for (int i = 0; i < kCoarseAxis; ++i) L[at(i, u, v)] = out[i];
    __syncthreads();
    for (int o = threadIdx.x; o < n; o += blockDim.x) {
        const int i = o % cx, j = (o / cx) % cy, k = o / (cx * cy);
        x[o] = L[at(i, j, k)];
    }
}

enum { FIN_RESID = 0, FIN_RZ = 1, FIN_PQ = 2, FIN_RR = 3, FIN_BSUM = 4 };

// Final stage of a two-stage reduction: sums the per-block partials in a
// fixed order, updates the solver scalars and copies them to `mirror`, a
// host-mapped buffer the host reads after synchronising the stream.
__global__ __launch_bounds__(256) void k_finalize(const double *partials, unsigned nb, int mode, int flag,
                                                   SolveScalars *sc, double ncells, SolveScalars *mirror) {
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
    if (bad) sc->bad = 1;
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
            break;
        case FIN_PQ:
            sc->pq = v[0];
            sc->alpha = (v[0] > 0.0 && isfinite(v[0])) ? sc->rz / v[0] : 0.0;
            if (!(v[0] > 0.0)) sc->bad |= 2;
            break;
        case FIN_RR:
            sc->rr = v[0];
            break;
        case FIN_BSUM:
            sc->b_sum = v[0];
            break;
    }
    *mirror = *sc;
}

// Orthonormal 1-D eigenbasis of the 7-point operator along one axis.
void basis_1d(int n, int bc, std::vector<double> &phi, std::vector<double> &lam) {
    phi.assign((size_t)n * n, 0.0);
    lam.assign(n, 0.0);
    for (int m = 0; m < n; ++m) {
        int k = bc == WG_BC_NEUMANN ? m : m + 1;
        double nrm = bc == WG_BC_NEUMANN ? std::sqrt((k == 0 ? 1.0 : 2.0) / n)
                                         : std::sqrt((k == n ? 1.0 : 2.0) / n);
        lam[m] = 4.0 * std::pow(std::sin(M_PI * k / (2.0 * n)), 2);
        for (int i = 0; i < n; ++i) {
            double a = M_PI * k * (i + 0.5) / n;
            phi[(size_t)m * n + i] = nrm * (bc == WG_BC_NEUMANN ? std::cos(a) : std::sin(a));
        }
    }
}

// 1-D eigenbases and eigenvalues of the coarsest level, laid out for k_coarse_eig.
std::vector<float> coarse_basis(const Dims &d, int bc) {
    std::vector<float> out;
    std::vector<double> phi[3], lam[3];
    const int n[3] = {d.nx, d.ny, d.nz};
    for (int a = 0; a < 3; ++a) basis_1d(n[a], bc, phi[a], lam[a]);
    for (int a = 0; a < 3; ++a) out.insert(out.end(), phi[a].begin(), phi[a].end());
    for (int a = 0; a < 3; ++a) out.insert(out.end(), lam[a].begin(), lam[a].end());
    return out;
}

std::vector<Dims> level_dims(int nx, int ny, int nz) {
    std::vector<Dims> out;
    Dims d{nx, ny, nz, -1};
    out.push_back(d);
    while (d.nx % 2 == 0 && d.ny % 2 == 0 && d.nz % 2 == 0 && d.nx >= 4 && d.ny >= 4 && d.nz >= 4 &&
           (d.nx > kCoarseTarget || d.ny > kCoarseTarget || d.nz > kCoarseTarget)) {
        d = Dims{d.nx / 2, d.ny / 2, d.nz / 2, -1};
        out.push_back(d);
    }
    return out;
}

// blocks of the sweep kernel that runs on grid d (its reductions write one partial per block)
unsigned sweep_blocks(const Dims &d) {
    return d.nx % 4 == 0 ? cdiv(waves4_of(d).tasks(), 4) : tiles_of(d).count();
}

size_t partial_slots(const Dims &fine) {
    size_t nb = sweep_blocks(fine);
    return (nb > (size_t)kRedBlocks ? nb : (size_t)kRedBlocks) * kMaxRed;
}

unsigned red_blocks(size_t n) {
    size_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < (size_t)kRedBlocks ? (b ? b : 1) : kRedBlocks);
}

}  // namespace

void Solver::plan(Arena &a, int nx, int ny, int nz) {
    auto dims = level_dims(nx, ny, nz);
    size_t N = dims[0].count();
    // fine level: r, z, z2, t0, e, p0, p1, q
    for (int k = 0; k < 8; ++k) a.reserve(N * sizeof(float));
    for (size_t l = 1; l < dims.size(); ++l)
        for (int k = 0; k < 4; ++k) a.reserve(dims[l].count() * sizeof(float));
    a.reserve(partial_slots(dims[0]) * sizeof(double));
    a.reserve(sizeof(SolveScalars));
    const Dims &c = dims.back();
    if (c.nx <= kCoarseAxis && c.ny <= kCoarseAxis && c.nz <= kCoarseAxis)
        for (int bc = 0; bc < 2; ++bc)
            a.reserve((size_t)(c.nx * c.nx + c.ny * c.ny + c.nz * c.nz + c.nx + c.ny + c.nz) * sizeof(float));
}

void Solver::bind(Arena &a, int nx, int ny, int nz, hipStream_t s) {
    st_ = s;
    auto dims = level_dims(nx, ny, nz);
    size_t N = dims[0].count();
    lv_.resize(dims.size());
    Level &f = lv_[0];
    f.d = dims[0];
    f.rhs = a.take<float>(N);   // the CG residual r
    f.x = a.take<float>(N);     // z = M r
    f.x2 = a.take<float>(N);
    f.tmp = a.take<float>(N);
    e_ = a.take<float>(N);
    p_[0] = a.take<float>(N);
    p_[1] = a.take<float>(N);
    q_ = a.take<float>(N);
    for (size_t l = 1; l < dims.size(); ++l) {
        Level &L = lv_[l];
        L.d = dims[l];
        size_t n = dims[l].count();
        L.rhs = a.take<float>(n);
        L.x = a.take<float>(n);
        L.x2 = a.take<float>(n);
        L.tmp = a.take<float>(n);
    }
    partials_ = a.take<double>(partial_slots(dims[0]));
    dsc_ = a.take<SolveScalars>(1);
    WG_HIP(hipHostMalloc((void **)&hsc_, sizeof(SolveScalars), hipHostMallocMapped | hipHostMallocCoherent));
    WG_HIP(hipHostGetDevicePointer((void **)&hsc_dev_, hsc_, 0));
    const Dims &c = dims.back();
    coarse_direct_ = c.nx <= kCoarseAxis && c.ny <= kCoarseAxis && c.nz <= kCoarseAxis;
    if (coarse_direct_) {
        for (int bc = 0; bc < 2; ++bc) {
            auto E = coarse_basis(c, bc);
            coarseM_[bc] = a.take<float>(E.size());
            WG_HIP(hipMemcpy(coarseM_[bc], E.data(), E.size() * sizeof(float), hipMemcpyHostToDevice));
        }
    }
}

Solver::~Solver() {
    if (hsc_) (void)hipHostFree(hsc_);
}

void Solver::finalize(int mode, unsigned nb, int flag) {
    k_finalize<<<1, 256, 0, st_>>>(partials_, nb, mode, flag, dsc_, (double)lv_[0].d.count(), hsc_dev_);
    WG_LAUNCH_CHECK();
}

void Solver::read_scalars() {
    // the last finalize wrote the host-mapped copy
    WG_HIP(hipStreamSynchronize(st_));
}

// kind / bytes_per_cell: optional timing bracket (WG_PROF_*) and the sweep's
// algorithmic bytes per cell.
template <class Op>
static void launch_stencil(const Op &op, const Dims &d, double *partials, hipStream_t s, int kind = -1,
                           double bytes_per_cell = 0.0) {
    prof::Scope ps(kind, s, bytes_per_cell * (double)d.count());
    if (d.nx % 4 == 0) {
        const Waves4 wv = waves4_of(d);
        k_stencil4<Op><<<cdiv(wv.tasks(), 4), 256, 0, s>>>(op, d, wv, partials);
    } else {
        const Tiles t = tiles_of(d);
        k_stencil<Op><<<t.count(), TX * TY, 0, s>>>(op, d, t, partials);
    }
    WG_LAUNCH_CHECK();
}

void Solver::vcycle(int l) {
    Level &L = lv_[l];
    L.d.bc_sign = bc_sign_;
    const int last = (int)lv_.size() - 1;
    if (l == last) {
        if (coarse_direct_) {
            k_coarse_eig<<<1, kCoarseAxis * kCoarseAxis, 0, st_>>>(L.rhs, L.x, coarseM_[bc_sign_ > 0 ? 1 : 0], L.d.nx, L.d.ny, L.d.nz);
            WG_LAUNCH_CHECK();
        } else {
            // no direct solve possible (odd extents): a fixed, even number of sweeps
            launch_stencil(OpSmoothFirst{L.rhs, L.x2, kOmega}, L.d, nullptr, st_);
            for (int k = 0; k < 15; ++k) {
                launch_stencil(OpSmooth<false>{L.x2, L.rhs, L.x, kOmega}, L.d, nullptr, st_);
                launch_stencil(OpSmooth<false>{L.x, L.rhs, L.x2, kOmega}, L.d, nullptr, st_);
            }
            launch_stencil(OpSmooth<false>{L.x2, L.rhs, L.x, kOmega}, L.d, nullptr, st_);
        }
        return;
    }
    Level &C = lv_[l + 1];
    C.d.bc_sign = bc_sign_;
    const int ks = l == 0 ? WG_PROF_SMOOTH : -1, kt = l == 0 ? WG_PROF_TRANSFER : -1;
    launch_stencil(OpSmooth2{L.rhs, L.x, kChebWa, kChebWb}, L.d, nullptr, st_, ks, 8.0);
    launch_stencil(OpResid{L.x, L.rhs, L.tmp}, L.d, nullptr, st_, ks, 12.0);
    {
        prof::Scope ps(kt, st_, 4.0 * (double)(L.d.count() + C.d.count()));
        if (L.d.nx % 4 == 0) {
            Waves4 wv = waves4_of(L.d);
            wv.G = ((unsigned)C.d.ny + wv.R - 1) / wv.R;   // rows of the coarse grid
            set_zlen(wv, C.d.nz);
            k_restrict4<<<cdiv(wv.tasks(), 4), 256, 0, st_>>>(L.tmp, L.d, C.rhs, C.d, wv);
        } else {
            k_restrict<<<cdiv(C.d.count(), 256), 256, 0, st_>>>(L.tmp, L.d, C.rhs, C.d);
        }
        WG_LAUNCH_CHECK();
    }
    vcycle(l + 1);
    {
        prof::Scope ps(kt, st_, 8.0 * (double)L.d.count() + 4.0 * (double)C.d.count());
        if (L.d.nx % 4 == 0) {
            const Waves4 wv = waves4_of(L.d, true);
            k_prolong4<<<cdiv(wv.tasks(), 4), 256, 0, st_>>>(C.x, C.d, L.x, L.d, wv);
        } else {
            k_prolong_add<<<cdiv(L.d.count(), 256), 256, 0, st_>>>(C.x, C.d, L.x, L.d);
        }
        WG_LAUNCH_CHECK();
    }
    launch_stencil(OpSmoothC<false>{L.x, L.rhs, L.x2, kChebWb}, L.d, nullptr, st_, ks, 12.0);
    if (l == 0) {
        launch_stencil(OpSmoothC<true>{L.x2, L.rhs, L.x, kChebWa}, L.d, partials_, st_, ks, 12.0);   // + r.z
    } else {
        launch_stencil(OpSmoothC<false>{L.x2, L.rhs, L.x, kChebWa}, L.d, nullptr, st_);
    }
}

int Solver::pcg(double tol, int max_it, double rr0) {
    Level &F = lv_[0];
    const size_t N = F.d.count();
    const unsigned tb = sweep_blocks(F.d);
    const unsigned rb = red_blocks(N);
    // z = M r, rz = r.z ; the first finalize must not form beta
    vcycle(0);
    finalize(FIN_RZ, tb, 1);
    int cur = 0, it = 0;
    double best = rr0;
    int stall = 0;
    for (; it < max_it; ++it) {
        if (it == 0)
            launch_stencil(OpPMatvec<true>{F.x, nullptr, p_[cur], q_, 0.f}, F.d, partials_, st_, WG_PROF_SWEEP,
                           12.0);
        else {
            // beta is read on the host-visible copy after the last finalize
            launch_stencil(OpPMatvec<false>{F.x, p_[cur ^ 1], p_[cur], q_, (float)hsc_->beta}, F.d, partials_, st_,
                           WG_PROF_SWEEP, 16.0);
        }
        finalize(FIN_PQ, tb, 0);
        {
            prof::Scope ps(WG_PROF_CGUPDATE, st_, (it == 0 ? 20.0 : 24.0) * (double)N);
            if (it == 0)
                k_cg_update<true><<<rb, kBlock, 0, st_>>>(e_, F.rhs, p_[cur], q_, dsc_, N, partials_);
            else
                k_cg_update<false><<<rb, kBlock, 0, st_>>>(e_, F.rhs, p_[cur], q_, dsc_, N, partials_);
            WG_LAUNCH_CHECK();
        }
        finalize(FIN_RR, rb, 0);
        vcycle(0);   // z for the next direction
        finalize(FIN_RZ, tb, 0);   // beta = rz / rz_old
        read_scalars();
        const double rr = hsc_->rr;
        if (hsc_->bad || !std::isfinite(rr)) { ++it; break; }
        if (rr <= tol * tol * rr0) { ++it; break; }
        if (rr < 0.5 * best) { best = rr; stall = 0; }
        else if (++stall >= 4) { ++it; break; }
        cur ^= 1;
    }
    return it;
}

SolveResult Solver::solve(const float *b, double *x, int bc, const wg_solve_opts &o) {
    require(bc == WG_BC_NEUMANN || bc == WG_BC_DIRICHLET, WG_EINVAL, "unknown boundary condition");
    bc_sign_ = bc == WG_BC_NEUMANN ? -1 : +1;
    for (auto &L : lv_) L.d.bc_sign = bc_sign_;
    Level &F = lv_[0];
    const size_t N = F.d.count();
    const unsigned tb = sweep_blocks(F.d);
    const unsigned gb = red_blocks(N);
    SolveResult res;
    WG_HIP(hipMemsetAsync(dsc_, 0, sizeof(SolveScalars), st_));
    if (!o.warm_start) {
        k_fill64<<<gb, kBlock, 0, st_>>>(x, 0.0, N);
        WG_LAUNCH_CHECK();
    }
    double mb = 0.0;
    if (bc == WG_BC_NEUMANN) {
        k_sum<<<gb, kBlock, 0, st_>>>(b, N, partials_);
        WG_LAUNCH_CHECK();
        finalize(FIN_BSUM, gb, 0);
        read_scalars();
        mb = hsc_->b_sum / (double)N;
    }
    const double tol = o.rel_tol > 0 ? o.rel_tol : 1e-6;
    const int max_iters = o.max_iters > 0 ? o.max_iters : 500;
    double bnorm = -1.0;
    for (;;) {
        launch_stencil(OpResid64{x, b, F.rhs, mb}, F.d, partials_, st_, WG_PROF_RESID64, 16.0);
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
        res.iters += pcg(inner, budget, hsc_->res_norm2);
        if (hsc_->bad & 1) {
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
