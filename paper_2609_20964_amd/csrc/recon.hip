// Reconstruction handle: resident device state and the forward / reverse
// drivers behind the C ABI (include/wgeo.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "prof.h"
#include "recon.h"
#include "scan.h"

namespace wg {

__global__ __launch_bounds__(kWave) void k_mirror_words(const uint32_t *src, uint32_t *dst, int n, unsigned *seq_dst,
                                                          unsigned seq) {
    for (int i = threadIdx.x; i < n; i += kWave) dst[i] = src[i];
    // one wavefront: the fence orders every lane's stores before seq
    __threadfence_system();
    if (threadIdx.x == 0) __hip_atomic_store(seq_dst, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

namespace {

constexpr int kIsoBlocks = 512;

__global__ void k_copy_shift(const double *x, double by, double *out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = x[i] - by;
}

__global__ void k_shift_scalar(const double *in, double by, double *out) { out[0] = in[0] - by; }
__global__ void k_set_scalar(double *out, double v) { out[0] = v; }

struct Timer {
    hipEvent_t ev[9];
    hipStream_t s;
    explicit Timer(hipStream_t st) : s(st) {
        // timing only: no system-scope fence (no cache writeback at the marker)
        for (auto &e : ev) WG_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    }
    ~Timer() {
        for (auto &e : ev) (void)hipEventDestroy(e);
    }
    void mark(int k) { WG_HIP(hipEventRecord(ev[k], s)); }
    float between(int a, int b) {
        float ms = 0.f;
        WG_HIP(hipEventElapsedTime(&ms, ev[a], ev[b]));
        return ms;
    }
};

}  // namespace

size_t Recon::footprint(const wg_grid &g, int max_points) {
    Arena a;
    plan(a, g, max_points);
    return a.planned() + Surface::initial_bytes(Dims{g.n[0], g.n[1], g.n[2], -1});
}

void Recon::plan(Arena &a, const wg_grid &g, int max_points) {
    const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
    Dims d{g.n[0], g.n[1], g.n[2], -1};
    a.reserve(N * sizeof(float));        // b
    a.reserve(N * sizeof(double));       // chi
    a.reserve(N * sizeof(float));        // phi
    a.reserve(N * sizeof(int32_t));      // argmin
    a.reserve(N * sizeof(float));        // g_phi (reverse)
    a.reserve(N * sizeof(float));        // g_chi (reverse)
    a.reserve(N * sizeof(double));       // lambda (reverse)
    a.reserve((size_t)max_points * 3 * sizeof(float));       // points
    a.reserve((size_t)max_points * 3 * sizeof(float));       // normals
    a.reserve((size_t)max_points * sizeof(int32_t));          // keys
    a.reserve((size_t)max_points * sizeof(int32_t));          // tile of each point
    a.reserve((size_t)max_points * sizeof(uint32_t));         // rank inside the tile
    a.reserve((size_t)max_points * sizeof(uint32_t));         // points ordered by tile
    const size_t nt = (size_t)tile_dims(d).count();
    for (int k = 0; k < 6; ++k) a.reserve(nt * sizeof(uint32_t));   // tile and chunk counts, offsets, lists
    for (int k = 0; k < 2; ++k) {
        a.reserve(2 * (size_t)cdiv(nt, scan::kScanBlock) * sizeof(uint32_t));
        a.reserve(2 * sizeof(uint32_t));
    }
    a.reserve((nt + (size_t)max_points / kChunk + 1) * sizeof(uint32_t));   // tile of each chunk
    a.reserve(kIsoBlocks * sizeof(double));
    a.reserve(8 * sizeof(double) + 4 * sizeof(int));   // scalars (c, c_shifted, g_c), then error flags
    a.reserve(sizeof(FixedScale));                       // fixed-point unit of the deterministic splat
    a.reserve(sizeof(uint32_t));                         // largest |normal component| (float bits)
    Solver::plan(a, d.nx, d.ny, d.nz);
    Surface::plan(a, d);
}

Recon::Recon(const wg_grid &g, int max_points, hipStream_t s) : grid_(g), max_points_(max_points), st_(s) {
    require(g.n[0] >= 4 && g.n[1] >= 4 && g.n[2] >= 4, WG_EINVAL, "each grid extent must be >= 4");
    require(g.h > 0 && std::isfinite(g.h), WG_EINVAL, "grid spacing must be positive");
    require(max_points >= 0, WG_EINVAL, "max_points must be >= 0");
    require((double)g.n[0] * g.n[1] * g.n[2] < 2.0e9, WG_EINVAL, "grid too large for 32-bit cell indices");
    d_ = Dims{g.n[0], g.n[1], g.n[2], -1};
    gf_.d = d_;
    for (int a = 0; a < 3; ++a) gf_.lo[a] = g.lo[a];
    gf_.h = g.h;
    plan(arena_, g, max_points);
    arena_.allocate();
    const size_t N = d_.count();
    b_ = arena_.take<float>(N);
    chi_ = arena_.take<double>(N);
    phi_ = arena_.take<float>(N);
    argmin_ = arena_.take<int32_t>(N);
    gphi_ = arena_.take<float>(N);
    gchi_ = arena_.take<float>(N);
    lam_ = arena_.take<double>(N);
    xyz_ = arena_.take<float>((size_t)max_points * 3);
    nrm_ = arena_.take<float>((size_t)max_points * 3);
    keys_ = arena_.take<int32_t>((size_t)max_points);
    tile_of_ = arena_.take<int32_t>((size_t)max_points);
    rank_ = arena_.take<uint32_t>((size_t)max_points);
    perm_ = arena_.take<uint32_t>((size_t)max_points);
    td_ = tile_dims(d_);
    const size_t nt = (size_t)td_.count();
    tile_cnt_ = arena_.take<uint32_t>(nt);
    tile_off_ = arena_.take<uint32_t>(nt);
    tile_act_ = arena_.take<uint32_t>(nt);
    ch_cnt_ = arena_.take<uint32_t>(nt);
    ch_off_ = arena_.take<uint32_t>(nt);
    ch_act_ = arena_.take<uint32_t>(nt);
    tile_blk_ = arena_.take<uint32_t>(2 * (size_t)cdiv(nt, scan::kScanBlock));
    tile_tot_ = arena_.take<uint32_t>(2);
    ch_blk_ = arena_.take<uint32_t>(2 * (size_t)cdiv(nt, scan::kScanBlock));
    ch_tot_ = arena_.take<uint32_t>(2);
    chunk_tile_ = arena_.take<uint32_t>(nt + (size_t)max_points / kChunk + 1);
    iso_part_ = arena_.take<double>(kIsoBlocks);
    scal_ = arena_.take<double>(10);
    err_ = reinterpret_cast<int *>(scal_ + 8);
    fix_ = arena_.take<FixedScale>(1);
    nmax_ = arena_.take<uint32_t>(1);
    solver_.bind(arena_, d_.nx, d_.ny, d_.nz, st_);
    surf_.bind(arena_, d_, st_);
    hm_.alloc();
    WG_HIP(hipMemsetAsync(chi_, 0, N * sizeof(double), st_));
    WG_HIP(hipMemsetAsync(err_, 0, 4 * sizeof(int), st_));
    WG_HIP(hipStreamSynchronize(st_));
}

Recon::~Recon() {
    if (sdf_st_) (void)hipStreamSynchronize(sdf_st_);
    if (ev_mc_) (void)hipEventDestroy(ev_mc_);
    if (ev_sdf_) (void)hipEventDestroy(ev_sdf_);
    if (ev_tail_) (void)hipEventDestroy(ev_tail_);
    if (sdf_st_) (void)hipStreamDestroy(sdf_st_);
}

void check_opts(const wg_solve_opts &o) {
    require(o.precision == WG_FP32_FP64REDUCE || o.precision == WG_FP64, WG_EINVAL, "unknown precision");
    require(o.deterministic == 0 || o.deterministic == 1, WG_EINVAL, "deterministic must be 0 or 1");
    require(o.quadrature == WG_VERTEX_QUADRATURE || o.quadrature == WG_EXACT_QUADRATURE, WG_EINVAL,
            "unknown quadrature");
    require(o.quadrature == WG_VERTEX_QUADRATURE || (o.precision == WG_FP32_FP64REDUCE && o.deterministic == 0),
            WG_EINVAL, "exact quadrature runs with the FP32 splat only (no WG_FP64, not deterministic)");
}

// The handle stream waits (on the device) for the last distance walk.
void Recon::wait_sdf() {
    if (sdf_pending_) {
        WG_HIP(hipStreamWaitEvent(st_, ev_sdf_, 0));
        sdf_pending_ = false;
    }
}

void Recon::join() {
    wait_sdf();
    if (tail_pending_) {
        WG_HIP(hipStreamWaitEvent(st_, ev_tail_, 0));
        tail_pending_ = false;
    }
}

void Recon::finish() {
    join();
    hm_.fetch(scal_, st_);
    const Mirror &m = hm_.wait();
    if (m.err[1] & 2) {
        // reported here; the next forward must not report it again
        WG_HIP(hipMemsetAsync(err_ + 1, 0, sizeof(int), st_));
        throw Error(WG_EDEVICE, "distance traversal stack overflow (last step)");
    }
}

size_t Recon::bytes_resident() const { return arena_.planned() + surf_.bytes(); }

// err_[0]: splat flags (bit 0: a point outside the grid); err_[1]: distance
// walk flags (bit 1: stack overflow), read only once that walk is known to be
// complete on the handle stream.
void Recon::check_err(const char *what) {
    hm_.fetch(scal_, st_);
    const Mirror &m = hm_.wait();
    if (m.err[0] & 1) throw Error(WG_EINVAL, std::string(what) + ": a point lies outside the grid");
    if (m.err[0] & 4) throw Error(WG_ENUMERIC, std::string(what) + ": a normal is NaN or infinite");
    if (!sdf_pending_ && (m.err[1] & 2)) throw Error(WG_EDEVICE, "distance traversal stack overflow");
}

int Recon::forward(const float *xyz, const float *nrm, int npts, const wg_solve_opts &o, wg_stats *st,
                   bool pipelined) {
    require(npts >= 0 && npts <= max_points_, WG_EINVAL, "n_points outside [0, max_points]");
    require(npts == 0 || (xyz && nrm), WG_EINVAL, "null point or normal pointer");
    check_opts(o);
    have_forward_ = false;
    const size_t N = d_.count();
    // WG_FP64 and deterministic splats sum in 64-bit fixed point, in the
    // lambda buffer (the reverse pass's; free during a forward)
    const bool fp64 = o.precision == WG_FP64, fixed = fp64 || o.deterministic;
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(lam_);
    Timer tm(st_);
    tm.mark(0);
    if (fixed) {
        WG_HIP(hipMemsetAsync(acc, 0, N * sizeof(unsigned long long), st_));
        WG_HIP(hipMemsetAsync(nmax_, 0, sizeof(uint32_t), st_));
    } else {
        WG_HIP(hipMemsetAsync(b_, 0, N * sizeof(float), st_));
    }
    WG_HIP(hipMemsetAsync(err_, 0, sizeof(int), st_));
    if (npts > 0) {
        // per point: 24 B read, 24 B copied, 4 B key, tile bookkeeping, 81 contributions to b
        prof::Scope ps(WG_PROF_SPLAT, st_, 376.0 * npts);
        const uint32_t nt = (uint32_t)td_.count();
        WG_HIP(hipMemsetAsync(tile_cnt_, 0, nt * sizeof(uint32_t), st_));
        k_bin_points<<<cdiv(npts, 256), 256, 0, st_>>>(xyz, nrm, npts, gf_, td_, keys_, xyz_, nrm_, tile_of_, rank_,
                                                      tile_cnt_, err_, fixed ? nmax_ : nullptr);
        const uint32_t nblk = cdiv(nt, scan::kScanBlock);
        scan::k_scan_partial<<<nblk, 256, 0, st_>>>(tile_cnt_, nt, tile_blk_);
        scan::k_scan_top<<<1, 256, 0, st_>>>(tile_blk_, nblk, tile_tot_);
        scan::k_scan_final<<<nblk, 256, 0, st_>>>(tile_cnt_, nt, tile_blk_, tile_off_, tile_act_);
        k_tile_scatter<<<cdiv(npts, 256), 256, 0, st_>>>(tile_of_, rank_, tile_off_, npts, perm_);
        k_chunk_counts<<<cdiv(nt, 256), 256, 0, st_>>>(tile_cnt_, nt, ch_cnt_);
        scan::k_scan_partial<<<nblk, 256, 0, st_>>>(ch_cnt_, nt, ch_blk_);
        scan::k_scan_top<<<1, 256, 0, st_>>>(ch_blk_, nblk, ch_tot_);
        scan::k_scan_final<<<nblk, 256, 0, st_>>>(ch_cnt_, nt, ch_blk_, ch_off_, ch_act_);
        k_chunk_tiles<<<cdiv(nt, 256), 256, 0, st_>>>(ch_cnt_, ch_off_, nt, chunk_tile_);
        const unsigned grid = std::min<unsigned>(2048u, nt + cdiv(npts, kChunk));
        if (o.quadrature == WG_EXACT_QUADRATURE) {
            k_splat_chunks<kSplatExact><<<grid, 256, 0, st_>>>(perm_, tile_off_, tile_cnt_, ch_off_, chunk_tile_,
                                                               ch_tot_, xyz_, nrm_, gf_, td_, b_, nullptr, nullptr);
        } else if (!fixed) {
            k_splat_chunks<kSplatF32><<<grid, 256, 0, st_>>>(perm_, tile_off_, tile_cnt_, ch_off_, chunk_tile_,
                                                             ch_tot_, xyz_, nrm_, gf_, td_, b_, nullptr, nullptr);
        } else {
            k_fixed_scale<<<1, 1, 0, st_>>>(nmax_, npts, grid_.h, fix_, err_);
            if (fp64)
                k_splat_chunks<kSplatFixed64><<<grid, 256, 0, st_>>>(perm_, tile_off_, tile_cnt_, ch_off_,
                                                                     chunk_tile_, ch_tot_, xyz_, nrm_, gf_, td_,
                                                                     nullptr, acc, fix_);
            else
                k_splat_chunks<kSplatFixed><<<grid, 256, 0, st_>>>(perm_, tile_off_, tile_cnt_, ch_off_,
                                                                   chunk_tile_, ch_tot_, xyz_, nrm_, gf_, td_, nullptr,
                                                                   acc, fix_);
        }
        WG_LAUNCH_CHECK();
    } else if (fixed) {
        k_fixed_scale<<<1, 1, 0, st_>>>(nmax_, 0, grid_.h, fix_, err_);
        WG_LAUNCH_CHECK();
    }
    if (fixed) {
        // b = sums * unit: FP32 always (the exported right-hand side), FP64 in place for WG_FP64
        const unsigned gb = std::min<unsigned>(cdiv(N, 256), 4096u);
        const long long *sums = reinterpret_cast<const long long *>(acc);
        k_fixed_to_b<float><<<gb, 256, 0, st_>>>(sums, fix_, N, b_);
        if (fp64) k_fixed_to_b<double><<<gb, 256, 0, st_>>>(sums, fix_, N, lam_);
        WG_LAUNCH_CHECK();
    }
    check_err("splat");
    tm.mark(1);
    n_points_ = npts;
    SolveResult sr = fp64 ? solver_.solve(lam_, chi_, WG_BC_NEUMANN, o) : solver_.solve(b_, chi_, WG_BC_NEUMANN, o);
    if (sr.status == WG_ENUMERIC) throw Error(WG_ENUMERIC, "non-finite value in the Poisson solve");
    chi_mean_ = sr.x_mean;
    tm.mark(2);
    // iso-value c = mean of chi_h at the points (0 without points); summed in
    // fixed point, whatever the points' order, where the splat was
    if (npts > 0) {
        unsigned nb = cdiv(npts, 256);
        if (nb > (unsigned)kIsoBlocks) nb = kIsoBlocks;
        if (fixed) {
            auto *w = reinterpret_cast<unsigned long long *>(iso_part_);
            WG_HIP(hipMemsetAsync(w, 0, 2 * sizeof(unsigned long long), st_));
            k_iso_absmax<<<nb, 256, 0, st_>>>(xyz_, npts, gf_, chi_, w);
            k_iso_fixed<<<nb, 256, 0, st_>>>(xyz_, npts, gf_, chi_, w);
            k_iso_fixed_finalize<<<1, 1, 0, st_>>>(w, npts, scal_);
        } else {
            k_iso_partial<<<nb, 256, 0, st_>>>(xyz_, npts, gf_, chi_, iso_part_);
            k_iso_finalize<<<1, 256, 0, st_>>>(iso_part_, nb, npts, scal_);
        }
    } else {
        WG_HIP(hipMemsetAsync(scal_, 0, sizeof(double), st_));
        k_shift_scalar<<<1, 1, 0, st_>>>(scal_, -chi_mean_, scal_);
    }
    WG_LAUNCH_CHECK();
    tm.mark(3);
    extract_surface();
    tm.mark(4);
    walk(pipelined, o.warm_start != 0);
    tm.mark(5);
    if (!pipelined) check_err("sdf");
    WG_HIP(hipEventSynchronize(tm.ev[5]));   // the timing events (a pipelined walk runs on the second stream)
    have_forward_ = true;
    field_only_ = false;
    quad_ = o.quadrature;
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->iters = sr.iters;
        st->refinements = sr.refinements;
        st->rel_res = sr.rel_res;
        st->iso_c = iso_c_ - chi_mean_;
        st->chi_mean = chi_mean_;
        st->n_tris = surf_.n_tris();
        st->status = sr.status;
        for (int k = 0; k < 5; ++k) st->ms[k] = tm.between(k, k + 1);
        if (pipelined) st->ms[4] = 0.f;   // the walk is still running
        st->bytes_resident = bytes_resident();
    }
    return sr.status;
}

// Marching Cubes of {chi_ = scal_[0]} (F6) once the previous walk is done.
void Recon::extract_surface() {
    // the previous distance walk (and pipelined sampling) reads the triangle
    // records, the hierarchy, the node sides and phi that follow: wait for it
    join();
    hm_.fetch(scal_, st_);        // c and the previous walk's flags
    surf_.extract(chi_, scal_);   // waits for the triangle count
    {
        const Mirror &m = hm_.wait();
        if (m.err[1] & 2) throw Error(WG_EDEVICE, "distance traversal stack overflow (previous forward)");
        iso_c_ = m.scal[0];
    }
    WG_HIP(hipMemsetAsync(err_ + 1, 0, sizeof(int), st_));
}

// The distance walk (F7) to the extracted surface, on the second stream when
// pipelined.
void Recon::walk(bool pipelined, bool related) {
    if (pipelined) {
        // distance walk on the second stream (created on first use): it reads
        // neither chi nor anything the next splat and solve write, so it may
        // overlap them
        if (!sdf_st_) {
            WG_HIP(hipStreamCreateWithFlags(&sdf_st_, hipStreamNonBlocking));
            WG_HIP(hipEventCreateWithFlags(&ev_mc_, hipEventDisableTiming));
            WG_HIP(hipEventCreateWithFlags(&ev_sdf_, hipEventDisableTiming));
            WG_HIP(hipEventCreateWithFlags(&ev_tail_, hipEventDisableTiming));
        }
        WG_HIP(hipEventRecord(ev_mc_, st_));
        WG_HIP(hipStreamWaitEvent(sdf_st_, ev_mc_, 0));
        surf_.sdf(grid_.h, phi_, argmin_, err_ + 1, sdf_st_, true, related);
        WG_HIP(hipEventRecord(ev_sdf_, sdf_st_));
        sdf_pending_ = true;
    } else {
        surf_.sdf(grid_.h, phi_, argmin_, err_ + 1, st_, false, related);
    }
}

int Recon::sdf_from_field(const double *chi, double c, wg_stats *st) {
    require(chi != nullptr, WG_EINVAL, "null field");
    require(std::isfinite(c), WG_EINVAL, "iso-value must be finite");
    have_forward_ = false;
    join();
    const size_t N = d_.count();
    Timer tm(st_);
    tm.mark(0);
    WG_HIP(hipMemcpyAsync(chi_, chi, N * sizeof(double), hipMemcpyDeviceToDevice, st_));
    k_set_scalar<<<1, 1, 0, st_>>>(scal_, c);
    WG_LAUNCH_CHECK();
    chi_mean_ = 0.0;
    n_points_ = 0;
    tm.mark(1);
    extract_surface();
    tm.mark(2);
    walk(false, false);
    tm.mark(3);
    check_err("sdf");
    WG_HIP(hipEventSynchronize(tm.ev[3]));
    have_forward_ = true;
    field_only_ = true;
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->iso_c = c;
        st->n_tris = surf_.n_tris();
        st->ms[3] = tm.between(1, 2);
        st->ms[4] = tm.between(2, 3);
        st->bytes_resident = bytes_resident();
    }
    return WG_OK;
}

int Recon::sample(const float *q, int nq, float *phi, float *nrm, bool pipelined) {
    require(have_forward_, WG_ESTATE, "sample before a successful forward");
    require(nq >= 0 && (nq == 0 || (q && phi)), WG_EINVAL, "bad query arguments");
    if (pipelined && sdf_st_) {
        // behind the walk on the second stream; q was ready on the handle stream
        // when the walk's start event was recorded after it
        launch_sample(gf_, phi_, q, nq, phi, nrm, sdf_st_);
        WG_HIP(hipEventRecord(ev_tail_, sdf_st_));
        tail_pending_ = true;
    } else {
        join();
        launch_sample(gf_, phi_, q, nq, phi, nrm, st_);
    }
    return WG_OK;
}

int Recon::backward(const float *q, int nq, const float *gphi_q, const float *gnrm_q, float *gxyz, float *gnrm_pts,
                    float *gq, const wg_solve_opts &o, wg_stats *st) {
    require(have_forward_, WG_ESTATE, "backward before a successful forward");
    require(!field_only_, WG_ESTATE, "backward after wg_sdf_from_field (no point cloud to differentiate)");
    require(nq >= 0 && (nq == 0 || (q && gphi_q)), WG_EINVAL, "bad query arguments");
    require(n_points_ == 0 || (gxyz && gnrm_pts), WG_EINVAL, "null point-gradient outputs");
    wg_solve_opts ao = o;
    ao.warm_start = 0;
    ao.quadrature = quad_;
    check_opts(ao);
    const size_t N = d_.count();
    join();
    Timer tm(st_);
    tm.mark(0);
    WG_HIP(hipMemsetAsync(gphi_, 0, N * sizeof(float), st_));
    WG_HIP(hipMemsetAsync(gchi_, 0, N * sizeof(float), st_));
    WG_HIP(hipMemsetAsync(scal_ + 2, 0, sizeof(double), st_));   // g_c
    // B1: transposed sampling
    launch_sample_T(gf_, phi_, q, nq, gphi_q, gnrm_q, gphi_, gq, st_);
    // B2: distance and vertex reverse -> g_chi, g_c
    surf_.sdf_T(gphi_, chi_, scal_, argmin_, grid_.h, gchi_, scal_ + 2);
    // B3: iso-value reverse into the field
    if (n_points_ > 0) {
        k_iso_T<<<cdiv(n_points_, 256), 256, 0, st_>>>(xyz_, n_points_, gf_, scal_ + 2, gchi_);
        WG_LAUNCH_CHECK();
    }
    tm.mark(1);
    // B4: adjoint solve A lambda = P g_chi (A symmetric), from zero
    SolveResult sr = solver_.solve(gchi_, lam_, WG_BC_NEUMANN, ao);
    if (sr.status == WG_ENUMERIC) throw Error(WG_ENUMERIC, "non-finite value in the adjoint solve");
    // B5 + B6: transposed divergence and splat, plus the iso-value point term
    if (n_points_ > 0 && quad_ == WG_EXACT_QUADRATURE) {
        // g_V by axis on the whole grid, in three solver vectors that are free after the solve
        const Planes3 gv{{solver_.spare(0), solver_.spare(1), solver_.spare(2)}};
        k_grad27_T<<<std::min<unsigned>(cdiv(N, 256), 8192u), 256, 0, st_>>>(lam_, d_, grid_.h, gv);
        k_splat_T<true><<<cdiv(n_points_, 256), 256, 0, st_>>>(xyz_, nrm_, keys_, n_points_, gf_, lam_, gv, chi_,
                                                               scal_ + 2, gxyz, gnrm_pts);
        WG_LAUNCH_CHECK();
    } else if (n_points_ > 0) {
        k_splat_T<false><<<cdiv(n_points_, 256), 256, 0, st_>>>(xyz_, nrm_, keys_, n_points_, gf_, lam_, Planes3{},
                                                                chi_, scal_ + 2, gxyz, gnrm_pts);
        WG_LAUNCH_CHECK();
    }
    tm.mark(2);
    WG_HIP(hipStreamSynchronize(st_));
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->iters = sr.iters;
        st->refinements = sr.refinements;
        st->rel_res = sr.rel_res;
        st->iso_c = iso_c_ - chi_mean_;
        st->chi_mean = chi_mean_;
        st->n_tris = surf_.n_tris();
        st->status = sr.status;
        st->ms[6] = tm.between(0, 1);
        st->ms[7] = tm.between(1, 2);
        st->bytes_resident = bytes_resident();
    }
    return sr.status;
}

int Recon::poisson(const float *b, double *x, int bc, const wg_solve_opts &o, wg_stats *st) {
    require(b && x, WG_EINVAL, "null pointer");
    check_opts(o);
    Timer tm(st_);
    tm.mark(0);
    SolveResult sr = solver_.solve(b, x, bc, o);
    if (sr.status == WG_ENUMERIC) throw Error(WG_ENUMERIC, "non-finite value in the Poisson solve");
    if (bc == WG_BC_NEUMANN && sr.x_mean != 0.0) solver_.shift(x, sr.x_mean);
    tm.mark(1);
    WG_HIP(hipStreamSynchronize(st_));
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->iters = sr.iters;
        st->refinements = sr.refinements;
        st->rel_res = sr.rel_res;
        st->status = sr.status;
        st->ms[1] = tm.between(0, 1);
        st->bytes_resident = bytes_resident();
    }
    return sr.status;
}

int Recon::mg_apply(const float *r, float *z, int bc) {
    require(r && z, WG_EINVAL, "null pointer");
    solver_.mg_apply(r, z, bc);
    return WG_OK;
}

int Recon::get_fields(float *b, double *chi, float *phi, int32_t *keys) {
    require(have_forward_, WG_ESTATE, "no forward result");
    join();
    const size_t N = d_.count();
    if (b) WG_HIP(hipMemcpyAsync(b, b_, N * sizeof(float), hipMemcpyDeviceToDevice, st_));
    if (chi) {
        k_copy_shift<<<cdiv(N, 256) < 4096 ? cdiv(N, 256) : 4096, 256, 0, st_>>>(chi_, chi_mean_, chi, N);
        WG_LAUNCH_CHECK();
    }
    if (phi) WG_HIP(hipMemcpyAsync(phi, phi_, N * sizeof(float), hipMemcpyDeviceToDevice, st_));
    if (keys && n_points_ > 0)
        WG_HIP(hipMemcpyAsync(keys, keys_, (size_t)n_points_ * sizeof(int32_t), hipMemcpyDeviceToDevice, st_));
    return WG_OK;
}

int Recon::get_mesh(float *tris, int32_t *info, int64_t max_tris, int64_t *n_tris) {
    require(have_forward_, WG_ESTATE, "no forward result");
    join();
    const int64_t T = surf_.n_tris();
    if (n_tris) *n_tris = T;
    const int64_t m = T < max_tris ? T : max_tris;
    if (m > 0 && tris) surf_.export_tris(chi_, scal_, tris, (uint32_t)m);
    if (m > 0 && info)
        WG_HIP(hipMemcpyAsync(info, surf_.tri_info(), (size_t)m * sizeof(int2), hipMemcpyDeviceToDevice, st_));
    return WG_OK;
}

// ---------------------------------------------------------------------------
// grids over a cloud's bounding box
// ---------------------------------------------------------------------------

// Sec. 2.3 takes the domain as the cloud's bounding box on a uniform grid
// whose density d (Table 1) sets the cell count along each axis; read as d
// cells per unit length (h = 1/d).  The box is widened by `pad` cells on each
// side (the splat reaches two cells past a point's cell) and each extent is
// rounded up to a multiple of q = 2^L, L the fewest halvings that bring the
// largest extent to at most 32, and to at least 2q, so that the solver's
// multigrid hierarchy coarsens to an exactly solved level; the box is centred.
void grid_from_bbox(const double lo[3], const double hi[3], double density, int pad, wg_grid &g) {
    require(std::isfinite(density) && density > 0.0, WG_EINVAL, "grid density must be positive");
    require(pad >= 0 && pad <= 1024, WG_EINVAL, "pad outside [0, 1024] cells");
    const double h = 1.0 / density;
    double need[3];
    double most = 0.0;
    for (int a = 0; a < 3; ++a) {
        require(std::isfinite(lo[a]) && std::isfinite(hi[a]) && hi[a] >= lo[a], WG_EINVAL, "empty or non-finite box");
        need[a] = std::ceil((hi[a] - lo[a]) / h) + 2.0 * pad;
        if (need[a] < 1.0) need[a] = 1.0;
        most = std::max(most, need[a]);
    }
    int L = 0;
    while (most / std::ldexp(1.0, L) > 32.0) ++L;
    const double q = std::ldexp(1.0, L);
    double cells = 1.0;
    for (int a = 0; a < 3; ++a) {
        const double n = std::max(std::ceil(need[a] / q), 2.0) * q;
        require(n <= 1 << 20, WG_EINVAL, "grid extent above 2^20 cells");
        g.n[a] = (int)n;
        cells *= n;
        g.lo[a] = 0.5 * (lo[a] + hi[a]) - 0.5 * n * h;
    }
    require(cells < 2.0e9, WG_EINVAL, "grid too large for 32-bit cell indices");
    g.h = h;
}

void grid_from_cloud(const float *xyz, int npts, double density, int pad, wg_grid &g, hipStream_t s) {
    require(npts > 0 && xyz != nullptr, WG_EINVAL, "an empty cloud has no bounding box");
    // a small device record and its host copy (set-up, not a hot path)
    uint32_t *dev = nullptr;
    WG_HIP(hipMalloc(&dev, 8 * sizeof(uint32_t)));
    uint32_t host[8] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0u, 0u, 0u, 0u, 0u};
    try {
        WG_HIP(hipMemcpyAsync(dev, host, sizeof(host), hipMemcpyHostToDevice, s));
        const unsigned blocks = std::min<unsigned>(cdiv(npts, 256), 256u);
        k_bbox<<<blocks, 256, 0, s>>>(xyz, npts, dev, reinterpret_cast<int *>(dev + 6));
        WG_LAUNCH_CHECK();
        WG_HIP(hipMemcpyAsync(host, dev, sizeof(host), hipMemcpyDeviceToHost, s));
        WG_HIP(hipStreamSynchronize(s));
    } catch (...) {
        (void)hipFree(dev);
        throw;
    }
    WG_HIP(hipFree(dev));
    require(host[6] == 0, WG_EINVAL, "a point coordinate is NaN or infinite");
    auto value = [](uint32_t k) {
        const uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
        float f;
        std::memcpy(&f, &b, 4);
        return (double)f;
    };
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = value(host[a]);
        hi[a] = value(host[3 + a]);
    }
    grid_from_bbox(lo, hi, density, pad, g);
}

// ---------------------------------------------------------------------------
// error channel
// ---------------------------------------------------------------------------

static thread_local std::string g_last_error;

void set_error(const std::string &m) { g_last_error = m; }
const char *last_error() { return g_last_error.c_str(); }

}  // namespace wg

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

struct wg_recon {
    wg::Recon *impl;
    hipStream_t stream;
};

template <class F>
static int guarded(F &&f) {
    try {
        return f();
    } catch (const wg::Error &e) {
        wg::set_error(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        wg::set_error("host allocation failed");
        return WG_ENOMEM;
    } catch (const std::exception &e) {
        wg::set_error(e.what());
        return WG_EDEVICE;
    } catch (...) {
        wg::set_error("unknown failure");
        return WG_EDEVICE;
    }
}

extern "C" {

const char *wg_last_error(void) { return wg::last_error(); }

size_t wg_recon_footprint(const wg_grid *grid, int max_points) {
    if (!grid) return 0;
    return wg::Recon::footprint(*grid, max_points);
}

int wg_recon_create(wg_recon **out, const wg_grid *grid, int max_points, void *hip_stream) {
    return guarded([&] {
        wg::require(out && grid, WG_EINVAL, "null argument");
        *out = nullptr;
        auto *r = new wg_recon{nullptr, (hipStream_t)hip_stream};
        try {
            r->impl = new wg::Recon(*grid, max_points, (hipStream_t)hip_stream);
        } catch (...) {
            delete r;
            throw;
        }
        *out = r;
        return WG_OK;
    });
}

void wg_recon_destroy(wg_recon *r) {
    if (!r) return;
    if (r->stream) (void)hipStreamSynchronize(r->stream);
    else (void)hipDeviceSynchronize();
    delete r->impl;
    delete r;
}

void *wg_recon_stream(wg_recon *r) { return r ? (void *)r->stream : nullptr; }

int wg_recon_forward(wg_recon *r, const float *d_xyz, const float *d_nrm, int n_points, const wg_solve_opts *opts,
                     wg_stats *stats) {
    return guarded([&] {
        wg::require(r && opts, WG_EINVAL, "null argument");
        return r->impl->forward(d_xyz, d_nrm, n_points, *opts, stats);
    });
}

int wg_sample_sdf_normals(wg_recon *r, const float *d_q, int n_q, float *d_phi, float *d_nrm_out) {
    return guarded([&] {
        wg::require(r, WG_EINVAL, "null handle");
        return r->impl->sample(d_q, n_q, d_phi, d_nrm_out);
    });
}

int wg_recon_step(wg_recon *r, const float *d_xyz, const float *d_nrm, int n_points, const float *d_q, int n_q,
                  float *d_phi, float *d_nrm_out, const wg_solve_opts *opts, wg_stats *stats) {
    return guarded([&] {
        wg::require(r && opts, WG_EINVAL, "null argument");
        wg::require(n_q >= 0 && (n_q == 0 || (d_q && d_phi)), WG_EINVAL, "bad query arguments");
        const int rc = r->impl->forward(d_xyz, d_nrm, n_points, *opts, stats, true);
        r->impl->sample(d_q, n_q, d_phi, d_nrm_out, true);
        return rc;
    });
}

int wg_recon_wait(wg_recon *r) {
    return guarded([&] {
        wg::require(r, WG_EINVAL, "null handle");
        r->impl->finish();
        return WG_OK;
    });
}

int wg_recon_backward(wg_recon *r, const float *d_q, int n_q, const float *d_gphi, const float *d_gnrm,
                      float *d_gxyz, float *d_gnrm_pts, float *d_gq, const wg_solve_opts *opts, wg_stats *stats) {
    return guarded([&] {
        wg::require(r && opts, WG_EINVAL, "null argument");
        return r->impl->backward(d_q, n_q, d_gphi, d_gnrm, d_gxyz, d_gnrm_pts, d_gq, *opts, stats);
    });
}

int wg_poisson_solve(wg_recon *r, const float *d_b, double *d_x, int bc, const wg_solve_opts *opts,
                     wg_stats *stats) {
    return guarded([&] {
        wg::require(r && opts, WG_EINVAL, "null argument");
        wg::require(bc == WG_BC_NEUMANN || bc == WG_BC_DIRICHLET, WG_EINVAL, "unknown boundary condition");
        return r->impl->poisson(d_b, d_x, bc, *opts, stats);
    });
}

int wg_mg_apply(wg_recon *r, const float *d_r, float *d_z, int bc) {
    return guarded([&] {
        wg::require(r, WG_EINVAL, "null handle");
        wg::require(bc == WG_BC_NEUMANN || bc == WG_BC_DIRICHLET, WG_EINVAL, "unknown boundary condition");
        return r->impl->mg_apply(d_r, d_z, bc);
    });
}

int wg_sdf_from_field(wg_recon *r, const double *d_chi, double c, wg_stats *stats) {
    return guarded([&] {
        wg::require(r, WG_EINVAL, "null handle");
        return r->impl->sdf_from_field(d_chi, c, stats);
    });
}

int wg_grid_from_bbox(const double lo[3], const double hi[3], double density, int pad_cells, wg_grid *out) {
    return guarded([&] {
        wg::require(lo && hi && out, WG_EINVAL, "null argument");
        wg::grid_from_bbox(lo, hi, density, pad_cells, *out);
        return WG_OK;
    });
}

int wg_grid_from_cloud(const float *d_xyz, int n_points, double density, int pad_cells, wg_grid *out,
                       void *hip_stream) {
    return guarded([&] {
        wg::require(out != nullptr, WG_EINVAL, "null argument");
        wg::grid_from_cloud(d_xyz, n_points, density, pad_cells, *out, (hipStream_t)hip_stream);
        return WG_OK;
    });
}

int wg_get_fields(wg_recon *r, float *d_b, double *d_chi, float *d_phi, int32_t *d_keys) {
    return guarded([&] {
        wg::require(r, WG_EINVAL, "null handle");
        return r->impl->get_fields(d_b, d_chi, d_phi, d_keys);
    });
}

int wg_get_mesh(wg_recon *r, float *d_tris, int32_t *d_info, int64_t max_tris, int64_t *n_tris) {
    return guarded([&] {
        wg::require(r, WG_EINVAL, "null handle");
        return r->impl->get_mesh(d_tris, d_info, max_tris, n_tris);
    });
}

}  // extern "C"
