// wg_poisson_solve_noalloc: the standalone Poisson solve of wg_poisson_solve
// (Eq. 20-21 operator, multigrid-preconditioned CG with FP64 refinement) for
// callers that cannot allocate device memory.  Every work buffer of the solver
// (CG vectors, multigrid levels, reduction partials, scalars, the coarsest
// level's eigenbases) is carved from `scratch`, a fixed device array of this
// library; the caller passes only the right-hand side, the solution and a
// stream.  The solve runs the same kernels in the same launch configuration as
// wg_poisson_solve, so both give the same result.
//
// Each GPU holds its own copy of `scratch` at its own address, looked up once
// per device with hipGetSymbolAddress (the array's name in host code is only a
// host-side stand-in).  Calls on one device share that copy: a per-device lock
// serialises them, and each call returns once its solve is complete, so the
// array keeps the last call's contents.  Work that another thread enqueues with
// the same copy outside this entry point would race; there is none.
#include <chrono>
#include <cstring>
#include <mutex>

#include "solver.h"

namespace wg {

namespace {

constexpr size_t kScratchBytes = size_t(10) << 20;   // 10 MiB: every grid of up to 64^3 cells
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_init_mu;
void *g_scratch[kMaxDevices];        // device address of scratch, per device (null: not looked up yet)
std::mutex g_dev_mu[kMaxDevices];    // serialises the calls on one device

// Bytes of scratch a solve on grid g needs (host arithmetic only).
size_t scratch_need(const wg_grid &g) {
    Arena a;
    Solver::plan(a, g.n[0], g.n[1], g.n[2]);
    return a.planned();
}

// Device address of this device's scratch; the device must be current.
void *scratch_of(int dev) {
    std::lock_guard<std::mutex> lk(g_init_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        WG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        require(p != nullptr && ((uintptr_t)p & 255u) == 0, WG_EDEVICE, "scratch array has no usable device address");
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

}  // namespace

static int poisson_noalloc(const wg_grid *grid, const float *d_b, double *d_x, int bc, const wg_solve_opts *opts,
                           wg_stats *stats, hipStream_t st) {
    require(grid && opts, WG_EINVAL, "null argument");
    const wg_grid &g = *grid;
    require(g.n[0] >= 4 && g.n[1] >= 4 && g.n[2] >= 4, WG_EINVAL, "each grid extent must be >= 4");
    require((double)g.n[0] * g.n[1] * g.n[2] < 2.0e9, WG_EINVAL, "grid too large for 32-bit cell indices");
    require(bc == WG_BC_NEUMANN || bc == WG_BC_DIRICHLET, WG_EINVAL, "unknown boundary condition");
    require(opts->precision == WG_FP32_FP64REDUCE || opts->precision == WG_FP64, WG_EINVAL, "unknown precision");
    require(opts->deterministic == 0 || opts->deterministic == 1, WG_EINVAL, "deterministic must be 0 or 1");
    const size_t need = scratch_need(g);
    require(need <= kScratchBytes, WG_EINVAL,
            "grid " + std::to_string(g.n[0]) + "x" + std::to_string(g.n[1]) + "x" + std::to_string(g.n[2]) +
                " needs " + std::to_string(need) + " bytes of solver scratch, above the " +
                std::to_string(kScratchBytes) + "-byte maximum of the no-allocation solve");
    require(d_b && d_x, WG_EINVAL, "null pointer");
    int dev = 0;
    WG_HIP(hipGetDevice(&dev));
    require(dev >= 0 && dev < kMaxDevices, WG_EDEVICE, "device index beyond the library's table");
    void *base = scratch_of(dev);
    std::lock_guard<std::mutex> lk(g_dev_mu[dev]);
    const auto t0 = std::chrono::steady_clock::now();
    Arena a;
    a.adopt(base, kScratchBytes);
    Solver s;
    s.set_instrumented(false);   // timing brackets create events
    s.bind(a, g.n[0], g.n[1], g.n[2], st, /*mapped=*/false);
    SolveResult sr = s.solve(d_b, d_x, bc, *opts);
    if (sr.status == WG_ENUMERIC) throw Error(WG_ENUMERIC, "non-finite value in the Poisson solve");
    if (bc == WG_BC_NEUMANN && sr.x_mean != 0.0) s.shift(d_x, sr.x_mean);
    WG_HIP(hipStreamSynchronize(st));
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->iters = sr.iters;
        stats->refinements = sr.refinements;
        stats->rel_res = sr.rel_res;
        stats->status = sr.status;
        stats->ms[1] = (float)std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        stats->bytes_resident = 0;
    }
    return sr.status;
}

}  // namespace wg

extern "C" int wg_poisson_solve_noalloc(const wg_grid *grid, const float *d_b, double *d_x, int bc,
                                        const wg_solve_opts *opts, wg_stats *stats, void *hip_stream) {
    try {
        return wg::poisson_noalloc(grid, d_b, d_x, bc, opts, stats, (hipStream_t)hip_stream);
    } catch (const wg::Error &e) {
        wg::set_error(e.what());
        return e.code;
    } catch (const std::exception &e) {
        wg::set_error(e.what());
        return WG_EDEVICE;
    } catch (...) {
        wg::set_error("unknown failure");
        return WG_EDEVICE;
    }
}
