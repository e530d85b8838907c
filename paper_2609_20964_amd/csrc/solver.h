// Matrix-free Poisson solver on a cell-centred grid (internal).
//
// Solves A x = b for the 7-point operator of Warp-Geo Eq. (20)-(21) under
// vertex quadrature, A = -h^2 L_h: (A x)_i = sum over the cell's interior
// faces of (x_i - x_j); zero-flux (Neumann, Eq. 19) boundaries, or the
// cell-centred Dirichlet test mode (ghost = -x, diagonal 6 + #boundary faces).
// With exact quadrature (zero-flux only) the fine-level operator is the
// 27-point Q1 stiffness of the same equations; the preconditioner is the
// 7-point V-cycle between two Jacobi steps on the 27-point operator.
//
// Precision scheme: the solution lives in FP64; each refinement step forms the
// FP64 residual r = P(b - A x) (P: mean removal for Neumann), solves A e = r
// approximately with FP32-vector multigrid-preconditioned CG whose inner
// products accumulate in FP64, and adds e to x in FP64.
#pragma once

#include "common.h"

namespace wg {

struct SolveScalars {
    double rz, rz_old, pq, alpha, beta, rr;
    double res_sum, res_sq, x_sum, b_sum, b_sq;
    double mean_r, res_norm2, b_norm2;
    double mean_b;   // mean of the right-hand side (Neumann)
    // inner PCG, decided on the device after each iteration's r.r
    double stop_rr;  // stop at r.r <= stop_rr (tol^2 times the starting r.r)
    double best;     // smallest r.r of the stall test so far
    int stall;       // iterations since r.r last halved
    int iters;       // iterations taken by this inner solve
    int done;        // the inner solve has stopped: its kernels return at once
    int bad;         // bit 0: a non-finite sum; bit 1: p.Ap <= 0
};

// Host-mapped copies of the scalars.  A finalize of the refinement stores the
// whole record, then seq, and the host waits for the value it expects.  Each
// inner iteration's r.r finalize stores one 64-bit status word instead (read
// whole, so never torn while a later iteration's finalize writes it):
// (its own sequence number << 32) | iters << 2 | (non-finite) << 1 | done.
struct PublishedScalars {
    SolveScalars s;
    unsigned seq;
    unsigned pad;
    unsigned long long status;
};

struct SolveResult {
    int iters = 0, refinements = 0, status = WG_OK;
    double rel_res = 0.0, x_mean = 0.0;
};

class Solver {
  public:
    static void plan(Arena &a, int nx, int ny, int nz);
    // Carve the solver's buffers from a (planned by plan()).  mapped: publish
    // the scalars the host reads through host-mapped pinned memory (allocated
    // here); otherwise through a device record inside the arena that the host
    // copies back, so that binding allocates nothing.
    void bind(Arena &a, int nx, int ny, int nz, hipStream_t s, bool mapped = true);
    ~Solver();
    // Timing brackets (wg_profile_*) around the solver's launches; on by default.
    void set_instrumented(bool on) { instrument_ = on; }

    // Solve A x = b (x: FP64, initial guess if opts.warm_start).  The mean of
    // the Neumann solution is reported in x_mean, not removed from x.
    SolveResult solve(const float *b, double *x, int bc, const wg_solve_opts &o);
    // the same with an FP64 right-hand side (WG_FP64)
    SolveResult solve(const double *b, double *x, int bc, const wg_solve_opts &o);

    // x -= mean (FP64), used where a zero-mean field is promised.
    void shift(double *x, double by);

    // Three fine-level FP32 vectors (the CG directions and A p) that hold
    // nothing between solves; callers may use them as scratch there.
    float *spare(int k) const { return k == 0 ? p_[0] : (k == 1 ? p_[1] : q_); }

    // z = M r: one V-cycle of the preconditioner with boundary condition bc
    // (r, z: FP32 on the device, on the solver's stream).
    void mg_apply(const float *r, float *z, int bc);

    // most levels a hierarchy can have (each halves every extent)
    static constexpr int kMaxLevels = 24;

  private:
    struct Level {
        Dims d;
        float *rhs, *x, *x2;
    };
    int pk(int kind) const { return instrument_ ? kind : -1; }
    template <class TB> SolveResult solve_impl(const TB *b, double *x, int bc, const wg_solve_opts &o);
    void vcycle(int l);
    void precond();
    unsigned rz_blocks() const;
    int pcg(double tol, int max_it, bool &non_finite);
    void pcg_iteration(int it, int &cur);
    void finalize(int mode, unsigned nb, int flag);
    template <class Op> void sweep(const Op &op, int kind, double bytes_per_cell, const int *skip);
    template <class Op> void sweep27(const Op &op, int kind, double bytes_per_cell, const int *skip);
    unsigned sweep_partials() const;
    void read_scalars();
    unsigned long long wait_status(unsigned want);

    hipStream_t st_ = nullptr;
    Level lv_[kMaxLevels] = {};
    int nlv_ = 0;
    float *e_ = nullptr, *p_[2] = {nullptr, nullptr}, *q_ = nullptr;
    double *partials_ = nullptr;
    SolveScalars *dsc_ = nullptr;
    PublishedScalars *pub_ = nullptr, *pub_dev_ = nullptr;   // host-mapped copy (host / device address)
    PublishedScalars host_pub_{};   // without mapped memory: the host's copy of *pub_dev_
    bool mapped_ = true, instrument_ = true;
    const SolveScalars *hsc_ = nullptr;                       // &pub_->s or &host_pub_.s
    unsigned seq_ = 0;                                        // sequence number of the last finalize
    unsigned sseq_ = 0;                                       // ... of the last status word
    const int *skip_ = nullptr;   // &dsc_->done while an inner PCG runs, else null
    float *coarseM_[2] = {nullptr, nullptr};   // [bc] 1-D eigenbases of the coarsest level
    int coarse_direct_ = 0;
    bool eig64_ = false;   // the exact solve's slices are 64 x 64 (an extent above 32)
    unsigned post_blocks_ = 0;   // workgroups of the finest post-smoothing pass (partials of r.z)
    int bc_sign_ = -1;
    bool exact_ = false;   // fine-level operator: the 27-point exact-quadrature stiffness
};

}  // namespace wg
