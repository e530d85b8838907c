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

constexpr int TX = 64, TY = 4, ZC = 8;
constexpr int kRedBlocks = 2048;     // grid of the pointwise reductions
constexpr int kMaxRed = 5;
constexpr float kOmega = 6.0f / 7.0f;   // weighted-Jacobi smoothing factor
constexpr int kCoarseMax = 512;         // dense coarse solve up to this many cells

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

// r = b - A x in FP64 (r stored FP32); sums of r, r^2, x, b, b^2.
struct OpResid64 {
    using T = double;
    static constexpr int NRED = 5;
    const double *x;
    const float *b;
    float *r;
    __device__ double load(size_t i) const { return x[i]; }
    __device__ void apply(size_t i, double c, double s, double diag, double *acc) const {
        double bv = (double)b[i];
        double rv = bv - (diag * c - s);
        r[i] = (float)rv;
        acc[0] += rv;
        acc[1] += rv * rv;
        acc[2] += c;
        acc[3] += bv;
        acc[4] += bv * bv;
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
    __device__ void apply(size_t i, float, float, float diag, double *) const { out[i] = w * rhs[i] / diag; }
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
    __device__ void apply(size_t i, float c, float s, float diag, double *acc) const {
        float rv = rhs[i];
        float v = c + w * (rv - (diag * c - s)) / diag;
        out[i] = v;
        if constexpr (DOT) acc[0] += (double)rv * (double)v;
    }
};

// out = rhs - A x.
struct OpResid {
    using T = float;
    static constexpr int NRED = 0;
    const float *x, *rhs;
    float *out;
    __device__ float load(size_t i) const { return x[i]; }
    __device__ void apply(size_t i, float c, float s, float diag, double *) const {
        out[i] = rhs[i] - (diag * c - s);
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
    __device__ void apply(size_t i, float c, float s, float diag, double *acc) const {
        float qv = diag * c - s;
        pnew[i] = c;
        q[i] = qv;
        acc[0] += (double)c * (double)qv;
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

__global__ void k_sub_mean(float *r, const SolveScalars *sc, size_t n) {
    const float m = (float)sc->mean_r;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        r[i] -= m;
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

// x = M rhs with the dense pseudo-inverse of the coarsest operator.
__global__ __launch_bounds__(256) void k_coarse_direct(const float *__restrict__ rhs, float *__restrict__ x,
                                                        const float *__restrict__ M, int n) {
    __shared__ float r[kCoarseMax];
    for (int i = threadIdx.x; i < n; i += blockDim.x) r[i] = rhs[i];
    __syncthreads();
    for (int row = threadIdx.x; row < n; row += blockDim.x) {
        const float *m = M + (size_t)row * n;
        float acc = 0.f;
        for (int j = 0; j < n; ++j) acc += m[j] * r[j];
        x[row] = acc;
    }
}

enum { FIN_RESID = 0, FIN_RZ = 1, FIN_PQ = 2, FIN_RR = 3 };

__global__ __launch_bounds__(256) void k_finalize(const double *partials, unsigned nb, int mode, int flag,
                                                   SolveScalars *sc, double ncells) {
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
    }
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

// Dense pseudo-inverse of A on a small grid from the separable eigenbasis.
std::vector<float> coarse_pinv(const Dims &d, int bc) {
    std::vector<double> px, py, pz, lx, ly, lz;
    basis_1d(d.nx, bc, px, lx);
    basis_1d(d.ny, bc, py, ly);
    basis_1d(d.nz, bc, pz, lz);
    const int N = (int)d.count();
    std::vector<double> M((size_t)N * N, 0.0), v(N);
    for (int c = 0; c < d.nz; ++c)
        for (int b = 0; b < d.ny; ++b)
            for (int a = 0; a < d.nx; ++a) {
                double lam = lx[a] + ly[b] + lz[c];
                if (lam < 1e-12) continue;
                for (int k = 0; k < d.nz; ++k)
                    for (int j = 0; j < d.ny; ++j)
                        for (int i = 0; i < d.nx; ++i)
                            v[(k * d.ny + j) * d.nx + i] =
                                px[(size_t)a * d.nx + i] * py[(size_t)b * d.ny + j] * pz[(size_t)c * d.nz + k];
                for (int r = 0; r < N; ++r) {
                    double vr = v[r] / lam;
                    double *row = &M[(size_t)r * N];
                    for (int s = 0; s < N; ++s) row[s] += vr * v[s];
                }
            }
    return std::vector<float>(M.begin(), M.end());
}

std::vector<Dims> level_dims(int nx, int ny, int nz) {
    std::vector<Dims> out;
    Dims d{nx, ny, nz, -1};
    out.push_back(d);
    while (d.nx % 2 == 0 && d.ny % 2 == 0 && d.nz % 2 == 0 && d.nx >= 4 && d.ny >= 4 && d.nz >= 4 &&
           d.count() > 64) {
        d = Dims{d.nx / 2, d.ny / 2, d.nz / 2, -1};
        out.push_back(d);
    }
    return out;
}

size_t partial_slots(const Dims &fine) {
    size_t nb = tiles_of(fine).count();
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
    if (c.count() <= (size_t)kCoarseMax)
        for (int bc = 0; bc < 2; ++bc) a.reserve(c.count() * c.count() * sizeof(float));
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
    WG_HIP(hipHostMalloc((void **)&hsc_, sizeof(SolveScalars), hipHostMallocDefault));
    const Dims &c = dims.back();
    coarse_direct_ = c.count() <= (size_t)kCoarseMax;
    if (coarse_direct_) {
        for (int bc = 0; bc < 2; ++bc) {
            coarseM_[bc] = a.take<float>(c.count() * c.count());
            auto M = coarse_pinv(c, bc);
            WG_HIP(hipMemcpy(coarseM_[bc], M.data(), M.size() * sizeof(float), hipMemcpyHostToDevice));
        }
    }
}

Solver::~Solver() {
    if (hsc_) (void)hipHostFree(hsc_);
}

void Solver::finalize(int mode, unsigned nb, int flag) {
    k_finalize<<<1, 256, 0, st_>>>(partials_, nb, mode, flag, dsc_, (double)lv_[0].d.count());
    WG_LAUNCH_CHECK();
}

void Solver::read_scalars() {
    WG_HIP(hipMemcpyAsync(hsc_, dsc_, sizeof(SolveScalars), hipMemcpyDeviceToHost, st_));
    WG_HIP(hipStreamSynchronize(st_));
}

// kind / bytes_per_cell: optional timing bracket (WG_PROF_*) and the sweep's
// algorithmic bytes per cell.
template <class Op>
static void launch_stencil(const Op &op, const Dims &d, double *partials, hipStream_t s, int kind = -1,
                           double bytes_per_cell = 0.0) {
    Tiles t = tiles_of(d);
    prof::Scope ps(kind, s, bytes_per_cell * (double)d.count());
    k_stencil<Op><<<t.count(), TX * TY, 0, s>>>(op, d, t, partials);
    WG_LAUNCH_CHECK();
}

void Solver::vcycle(int l) {
    Level &L = lv_[l];
    L.d.bc_sign = bc_sign_;
    const int last = (int)lv_.size() - 1;
    if (l == last) {
        if (coarse_direct_) {
            k_coarse_direct<<<1, 256, 0, st_>>>(L.rhs, L.x, coarseM_[bc_sign_ > 0 ? 1 : 0], (int)L.d.count());
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
    launch_stencil(OpSmoothFirst{L.rhs, L.x2, kOmega}, L.d, nullptr, st_, ks, 8.0);
    launch_stencil(OpSmooth<false>{L.x2, L.rhs, L.x, kOmega}, L.d, nullptr, st_, ks, 12.0);
    launch_stencil(OpResid{L.x, L.rhs, L.tmp}, L.d, nullptr, st_, ks, 12.0);
    {
        prof::Scope ps(kt, st_, 4.0 * (double)(L.d.count() + C.d.count()));
        k_restrict<<<cdiv(C.d.count(), 256), 256, 0, st_>>>(L.tmp, L.d, C.rhs, C.d);
        WG_LAUNCH_CHECK();
    }
    vcycle(l + 1);
    {
        prof::Scope ps(kt, st_, 8.0 * (double)L.d.count() + 4.0 * (double)C.d.count());
        k_prolong_add<<<cdiv(L.d.count(), 256), 256, 0, st_>>>(C.x, C.d, L.x, L.d);
        WG_LAUNCH_CHECK();
    }
    launch_stencil(OpSmooth<false>{L.x, L.rhs, L.x2, kOmega}, L.d, nullptr, st_, ks, 12.0);
    if (l == 0) {
        launch_stencil(OpSmooth<true>{L.x2, L.rhs, L.x, kOmega}, L.d, partials_, st_, ks, 12.0);   // + r.z
    } else {
        launch_stencil(OpSmooth<false>{L.x2, L.rhs, L.x, kOmega}, L.d, nullptr, st_);
    }
}

int Solver::pcg(double tol, int max_it, double rr0) {
    Level &F = lv_[0];
    const size_t N = F.d.count();
    const unsigned tb = tiles_of(F.d).count();
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
    const unsigned tb = tiles_of(F.d).count();
    const unsigned gb = red_blocks(N);
    SolveResult res;
    WG_HIP(hipMemsetAsync(dsc_, 0, sizeof(SolveScalars), st_));
    if (!o.warm_start) {
        k_fill64<<<gb, kBlock, 0, st_>>>(x, 0.0, N);
        WG_LAUNCH_CHECK();
    }
    const double tol = o.rel_tol > 0 ? o.rel_tol : 1e-6;
    const int max_iters = o.max_iters > 0 ? o.max_iters : 500;
    double bnorm = -1.0;
    for (;;) {
        launch_stencil(OpResid64{x, b, F.rhs}, F.d, partials_, st_, WG_PROF_RESID64, 16.0);
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
        if (bc == WG_BC_NEUMANN) {
            k_sub_mean<<<gb, kBlock, 0, st_>>>(F.rhs, dsc_, N);
            WG_LAUNCH_CHECK();
        }
        double inner = 0.5 * tol / res.rel_res;
        if (inner < 1e-3) inner = 1e-3;
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
