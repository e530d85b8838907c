/*
 * wgeo.h -- C ABI of the MI355X grid-Poisson SDF library (libwgeo.so).
 *
 * The library reconstructs a signed distance field and surface normals on a
 * uniform 3-D grid from an oriented point cloud, following Warp-Geo
 * (arXiv 2609.20964):
 *
 *   splat the point normals to the 27 cells around each point (Sec. 2.3,
 *   Eq. 23-25) -> divergence b (Eq. 22, 26) -> Poisson solve A chi = b with
 *   zero-flux boundaries (Eq. 19-21) -> iso-value c (Sec. 2.4) -> Marching
 *   Cubes surface (Eq. 27-28) -> exact distance to that surface with the
 *   inside/outside sign on every grid node (Eq. 29-34) -> trilinear sampling of
 *   the SDF and of its grid gradient (normals, Sec. 2.4 after Eq. 32).
 *
 * The reverse pass follows Sec. 2.5 (Eq. 35-39): one adjoint solve with A^T
 * (= A), no stored solver iterates.
 *
 * Conventions
 *   - Grid: n[0] x n[1] x n[2] cubic cells of edge h starting at lo; unknowns
 *     at cell centres lo + (i + 1/2) h.  Grid scalars are [n2][n1][n0]
 *     (x fastest).  Each n[d] >= 4.
 *   - Points, normals and queries are float32 [count][3] (x, y, z).
 *   - Every d_* pointer is DEVICE memory owned by the caller.  The library
 *     never frees it and never allocates user-visible outputs.
 *   - Calls enqueue work on the handle's HIP stream.  The host waits only for
 *     small results: the splat's error flags, the solver's convergence
 *     scalars, the triangle count after surface extraction, and at the end
 *     of wg_recon_forward / wg_recon_step / wg_recon_backward for the call's
 *     statistics (a forward's distance walk included; a pipelined step's walk
 *     not).  Outputs are ready once the stream reaches them (synchronise the
 *     stream before reading them on the host).
 *   - Return codes: WG_OK (0), WG_PENDING (> 0, wg_poll only) or a negative
 *     WG_E* value; wg_last_error() gives this thread's last message.  No C++
 *     exception crosses the ABI.
 *   - A handle is not thread-safe: one caller thread at a time.
 */
#ifndef WGEO_H
#define WGEO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    WG_OK = 0,
    WG_PENDING = 1,     /* wg_poll: request admitted or queued, not finished     */
    WG_EINVAL = -1,     /* bad pointer, size, option, or a point outside the grid */
    WG_ENOMEM = -2,     /* device allocation failed / footprint above the budget  */
    WG_ENOTCONV = -3,   /* non-fatal: outputs written, stats.rel_res says how far */
    WG_ENUMERIC = -4,   /* NaN or Inf met in a reduction                           */
    WG_EDEVICE = -5,    /* HIP runtime error                                       */
    WG_ESTATE = -6      /* call order (backward without forward, unknown ticket)  */
};

enum { WG_BC_NEUMANN = 0, WG_BC_DIRICHLET = 1 };

/* wg_solve_opts.quadrature: how the Galerkin integrals of Eq. 21 and 26 are taken */
enum {
    WG_VERTEX_QUADRATURE = 0, /* at the grid vertices: the 7-point operator (diagonal =
                                 interior neighbours, off-diagonal -1) and b = -h^2 D_h V
                                 with face-averaged fluxes                          */
    WG_EXACT_QUADRATURE = 1   /* exactly, for the trilinear tents mirrored across the
                                 outer faces: the 27-point Q1 stiffness {8/3, 0, -1/6,
                                 -1/12} (indices clamped at the faces) and b = h sum_xi
                                 (g along xi, m across) V_xi with the 1-D mass m =
                                 (1/6, 2/3, 1/6); the solver keeps the 7-point
                                 multigrid as preconditioner.  FP32 splat only.      */
};

/* wg_solve_opts.precision */
enum {
    WG_FP32_FP64REDUCE = 0, /* splat weights and sums in FP32 (FP32 atomics); stencil
                               sweeps FP32 with FP64 inner products; the solution
                               refined in FP64                                    */
    WG_FP64 = 1             /* the right-hand side b in FP64: splat weights and the
                               divergence in FP64, summed exactly in 64-bit fixed
                               point (so also deterministic); FP64 residuals and
                               solution as above                                  */
};

typedef struct {
    int n[3];           /* cells per axis (x, y, z), each >= 4                    */
    double lo[3];       /* world position of the grid's lower corner              */
    double h;           /* cell edge                                               */
} wg_grid;

typedef struct {
    double rel_tol;     /* stop at ||P b - A chi||_2 <= rel_tol ||P b||_2 (FP64)  */
    int max_iters;      /* cap on inner preconditioned-CG iterations, all refinements */
    int warm_start;     /* 1: start from the handle's last solution; also marks the
                           cloud as close to the last one, so the distance walk
                           reuses the last walk's tile costs and seeds.  0: an
                           unrelated cloud; on grids of 2^23 nodes or more the
                           walk orders its tiles by their depth inside the new
                           surface and searches its seeds first.  No result
                           depends on this beyond the solver's start.          */
    int precision;      /* WG_FP32_FP64REDUCE (0) or WG_FP64 (1)                   */
    int deterministic;  /* 1: the splat sums each cell's contributions in 64-bit
                           fixed point (integer adds, in any order), so b -- and
                           with it chi, the surface and phi -- is the same bit for
                           bit however points, threads and concurrent requests
                           interleave.  The fixed-point unit is 2^-e with e the
                           largest exponent for which npts * 3.75 h^-2 max|n_k|
                           fits below 2^61 (a bound on any cell's sum).  The
                           iso-value's mean over the points is summed the same
                           way (unit from the largest |chi_h| at a point).
                           Forward pass only: the reverse pass still scatters
                           with FP32 atomics.  0: FP32 atomics (WG_FP64
                           implies 1).                                         */
    int quadrature;     /* WG_VERTEX_QUADRATURE (0) or WG_EXACT_QUADRATURE (1)     */
} wg_solve_opts;

typedef struct {
    int iters;              /* inner PCG iterations (all refinement steps)        */
    int refinements;        /* FP64 residual evaluations                           */
    double rel_res;         /* final FP64 relative residual                        */
    double iso_c;           /* iso-value c, for the zero-mean field chi            */
    double chi_mean;        /* mean removed from the stored FP64 solution          */
    int64_t n_tris;         /* Marching Cubes triangles                            */
    int status;             /* WG_OK or WG_ENOTCONV                                */
    float ms[8];            /* 0 splat, 1 solve, 2 iso, 3 surface, 4 sdf, 5 sample,
                               6 reverse-sampling/surface adjoint, 7 adjoint solve+splat */
    size_t bytes_resident;  /* device bytes held by the handle                     */
} wg_stats;

typedef struct wg_recon wg_recon;
typedef struct wg_server wg_server;

/* ---------------------------------------------------------------------------
 * Reconstruction handle
 * ------------------------------------------------------------------------- */

/* Allocate the resident state for one uniform grid of n[0] x n[1] x n[2]
 * cubic cells of edge h from lo (Sec. 2.3: the domain discretised by l x m x n
 * cells of size h, one unknown per cell, Eq. 16-17) and up to max_points
 * points (splat buffers, FP64 solution, solver and multigrid vectors, SDF
 * grid, surface buffers).  hip_stream: a hipStream_t (NULL = default stream),
 * on which every call on the handle enqueues its work.  The caller owns *out
 * and frees it with wg_recon_destroy.  Returns WG_EINVAL for n[d] < 4, h <= 0
 * or more than 2^31 cells, WG_ENOMEM if allocation fails. */
int wg_recon_create(wg_recon **out, const wg_grid *grid, int max_points, void *hip_stream);

/* A grid over a bounding box (Sec. 2.3: the domain is the point cloud's
 * bounding box, discretised uniformly; Table 1's grid density d sets the
 * cells per axis, read here as d cells per unit length, h = 1/d).  lo, hi:
 * the box corners (hi >= lo per axis).  The box is widened by pad_cells cells
 * on each side (the 27-cell splat reaches two cells past a point's cell, so
 * use pad_cells >= 3 for a cloud in the box) and each extent rounded up to a
 * multiple of 2^L, L the fewest halvings that bring the largest extent to 32
 * or less, and to at least 2^(L+1) cells, so that the solver's multigrid
 * hierarchy reaches an exactly solved coarsest level; the box sits at the
 * centre.  Host arithmetic only; WG_EINVAL for density <= 0, a bad box or a
 * grid above 2^31 cells. */
int wg_grid_from_bbox(const double lo[3], const double hi[3], double density, int pad_cells, wg_grid *out);

/* wg_grid_from_bbox over the bounding box of n_points device points d_xyz
 * ([n_points][3] float32), taken on the device (exact minima and maxima) on
 * hip_stream.  Synchronises the stream (and allocates a small record); for
 * set-up, not per step.  WG_EINVAL for an empty cloud or a non-finite
 * coordinate. */
int wg_grid_from_cloud(const float *d_xyz, int n_points, double density, int pad_cells, wg_grid *out,
                       void *hip_stream);

/* Footprint (bytes) that wg_recon_create would allocate. */
size_t wg_recon_footprint(const wg_grid *grid, int max_points);

/* Forward reconstruction (Sec. 2.3-2.4): bins the points, splats their normals,
 * forms b, solves A chi = b to opts->rel_tol with FP32 sweeps, FP64 reductions
 * and FP64 residual refinement, takes the iso-value, extracts the surface and
 * writes the signed distance to every grid node.  d_xyz, d_nrm: [n_points][3]
 * float32 (copied into the handle).  A point whose cell
 * floor((x - lo)/h) (FP64) falls outside the grid gives WG_EINVAL.
 * Returns WG_ENOTCONV (results written) if max_iters stopped the solve. */
int wg_recon_forward(wg_recon *r, const float *d_xyz, const float *d_nrm, int n_points,
                     const wg_solve_opts *opts, wg_stats *stats);

/* Sample the last forward's SDF at n_q query points and the surface normal
 * there (Sec. 2.4: phi is a grid field, Eq. 34, whose normal is
 * grad(phi)/|grad(phi)| as after Eq. 32): phi(q) trilinear in the node values,
 * the normal from grid central differences (one-sided on boundary cells)
 * interpolated trilinearly and normalised (0 where the gradient vanishes).
 * d_q: [n_q][3] float32 (read); d_phi: [n_q] and d_nrm_out: [n_q][3] or NULL
 * (written); all caller-owned device memory.  Queries outside the grid's
 * cell-centre box are clamped to it.  WG_ESTATE before a forward,
 * WG_EINVAL for n_q < 0 or a null pointer with n_q > 0.  Enqueued on the
 * handle's stream (after the last pipelined walk); does not block. */
int wg_sample_sdf_normals(wg_recon *r, const float *d_q, int n_q, float *d_phi, float *d_nrm_out);

/* Forward reconstruction followed by sampling at d_q, pipelined with the next
 * call on the same handle (a moving-boundary loop, Sec. 3.2).  Computes what
 * wg_recon_forward then wg_sample_sdf_normals compute, but returns once the
 * surface is extracted: the distance walk and the sampling of this call run
 * on the handle's second stream while the next wg_recon_step bins, splats and
 * solves (the walk reads neither the field nor the point buffers that step
 * overwrites).  d_phi / d_nrm_out of a call are complete once a later
 * wg_recon_wait(r) has been reached on the handle's stream (or the device has
 * been synchronised); every other call on r orders itself after them.  d_q
 * must stay valid until then.  Errors and statistics are those of
 * wg_recon_forward; stats->ms[4] (the walk) is reported as 0. */
int wg_recon_step(wg_recon *r, const float *d_xyz, const float *d_nrm, int n_points,
                  const float *d_q, int n_q, float *d_phi, float *d_nrm_out,
                  const wg_solve_opts *opts, wg_stats *stats);

/* Orders the handle's stream after all work r has left running on its second
 * stream (the last wg_recon_step's walk and sampling), then blocks the host
 * until that work is complete.  Returns WG_EDEVICE if the last walk failed
 * (its d_phi / d_nrm_out are then not valid). */
int wg_recon_wait(wg_recon *r);

/* Reverse pass (Sec. 2.5, Eq. 35-39) of the last forward + sampling at d_q:
 * given dL/dphi(q) (d_gphi, [n_q]) and optionally dL/dn(q) (d_gnrm, [n_q][3]
 * or NULL), writes dL/dx (d_gxyz, [n_points][3]) and dL/dn_i (d_gnrm_pts,
 * [n_points][3]) for the points of the last forward, and dL/dq (d_gq,
 * [n_q][3], or NULL).  Runs one adjoint Poisson solve with opts; the
 * quadrature is the last forward's whatever opts->quadrature says (the
 * reverse pass differentiates the system that forward solved).
 * Gradients hold almost everywhere: the central cell of each point is kept
 * fixed, Marching Cubes cases and nearest triangles are those of the forward.
 * WG_ESTATE if no forward has run on r. */
int wg_recon_backward(wg_recon *r, const float *d_q, int n_q, const float *d_gphi,
                      const float *d_gnrm, float *d_gxyz, float *d_gnrm_pts, float *d_gq,
                      const wg_solve_opts *opts, wg_stats *stats);

/* Standalone Poisson solve on r's grid (Eq. 20-21): A x = b with bc
 * WG_BC_NEUMANN (zero flux; b is projected to zero mean and x returned with
 * zero mean) or WG_BC_DIRICHLET (cell-centred ghost = -x; test mode).
 * opts->quadrature picks the operator (exact: WG_BC_NEUMANN only, else
 * WG_EINVAL).  d_b: [N] float32; d_x: [N] float64, used as the initial guess when
 * opts->warm_start is set, overwritten with the solution. */
int wg_poisson_solve(wg_recon *r, const float *d_b, double *d_x, int bc,
                     const wg_solve_opts *opts, wg_stats *stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of wg_poisson_solve on `grid`, with no handle and no allocation.  Every work
 * buffer comes from a fixed 10 MiB device array inside the library (one copy
 * per GPU, held until the process ends), which holds the solver state of any
 * grid of up to 64^3 cells; a grid needing more gives WG_EINVAL before any
 * device work.  d_b, d_x, bc, opts and the result are as for wg_poisson_solve
 * (same kernels, same launch configuration).  Work runs on hip_stream (a
 * hipStream_t, NULL = default stream); the call returns once the solve is
 * complete (it blocks the host).  Calls on one GPU share its array and are
 * serialised by the library; the array keeps the last call's contents.
 * stats->ms[1] is the call's wall time; bytes_resident is 0. */
int wg_poisson_solve_noalloc(const wg_grid *grid, const float *d_b, double *d_x, int bc,
                             const wg_solve_opts *opts, wg_stats *stats, void *hip_stream);

/* One application z = M r of the multigrid preconditioner that the Poisson
 * solves (Eq. 20-21 operator, Sec. 2.5's iterative solve) use on r's grid:
 * a V-cycle with cell-centred trilinear prolongation P, restriction P^T / 2,
 * degree-2 Chebyshev smoothing before and after the coarse correction and an
 * exact solve on the coarsest level (32 or 64 cells per axis at most; a grid
 * whose every extent is at most 64 is that level alone, M = A^-1 up to FP32
 * rounding, the constant mode dropped under zero flux).  M is symmetric and
 * linear.  d_r, d_z:
 * float32 [N] on the device (distinct; d_r is not modified); bc as for
 * wg_poisson_solve.  Runs on the handle's stream without blocking the host;
 * shares the solver's work buffers with forward/backward/poisson calls on r,
 * which the stream orders. */
int wg_mg_apply(wg_recon *r, const float *d_r, float *d_z, int bc);

/* Signed-distance reinitialisation of a given implicit field (Sec. 2.4,
 * Eq. 27-34): the Marching Cubes surface {chi = c} on the dual lattice of r's
 * grid, then the exact signed distance to it at every grid node (positive
 * where chi >= c), as wg_recon_forward computes them after its solve.  d_chi:
 * float64 [N] on the device (copied into the handle); c: the iso-value.
 * Afterwards wg_sample_sdf_normals, wg_get_fields (chi as given) and
 * wg_get_mesh see this surface; wg_recon_backward returns WG_ESTATE (there is
 * no point cloud to differentiate).  stats: iso_c = c, n_tris, ms[3] (surface)
 * and ms[4] (distance).  Host-synchronising like wg_recon_forward. */
int wg_sdf_from_field(wg_recon *r, const double *d_chi, double c, wg_stats *stats);

/* Copies of resident fields from the last forward into caller-owned device
 * buffers: d_b float32 [N] (the right-hand side b of Eq. 20, as Eq. 26 forms
 * it), d_chi float64 [N] (the coefficients a of Eq. 16, zero mean), d_phi
 * float32 [N] (the signed distance of Eq. 34 at the cell centres), d_keys
 * int32 [n_points] (each point's central cell of the 27-cell stencil of
 * Eq. 24-25, linear index i + n0 (j + n1 k)).  Any pointer may be NULL.
 * WG_ESTATE before a forward.  Enqueued on the handle's stream. */
int wg_get_fields(wg_recon *r, float *d_b, double *d_chi, float *d_phi, int32_t *d_keys);

/* Copy of the last forward's triangles: d_tris float32 [n_tris][9] (three
 * vertices in grid units, cell centre (i,j,k) at (i,j,k)), d_info int32
 * [n_tris][2] (dual-cube linear index, 3 local edge ids packed 4 bits each).
 * max_tris bounds the copy; *n_tris receives the total. */
int wg_get_mesh(wg_recon *r, float *d_tris, int32_t *d_info, int64_t max_tris, int64_t *n_tris);

void wg_recon_destroy(wg_recon *r);

/* Device pointer of the handle's HIP stream (hipStream_t). */
void *wg_recon_stream(wg_recon *r);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of reconstructions of uneven sizes
 * ------------------------------------------------------------------------- */

typedef struct {
    wg_grid grid;
    const float *d_xyz;     /* [n_points][3] device; copied at submit            */
    const float *d_nrm;     /* [n_points][3] device; copied at submit            */
    int n_points;
    const float *d_q;       /* [n_q][3] device; copied at submit                 */
    int n_q;
    const float *d_gphi;    /* [n_q] dL/dphi(q) (copied), or NULL: no reverse pass */
    wg_solve_opts opts;
    /* caller-owned device outputs, written before wg_poll reports WG_OK */
    float *d_phi;           /* [n_q]                                             */
    float *d_nrm_out;       /* [n_q][3] or NULL                                  */
    float *d_gxyz;          /* [n_points][3], used iff d_gphi != NULL            */
    float *d_gnrm_pts;      /* [n_points][3], used iff d_gphi != NULL            */
    const float *d_gnrm;    /* [n_q][3] dL/dn(q) (copied), or NULL; needs d_gphi  */
    float *d_gq;            /* [n_q][3] dL/dq output, or NULL; needs d_gphi       */
} wg_request;

typedef struct {
    int status;             /* WG_OK / WG_ENOTCONV / error of this request       */
    wg_stats stats;
    double t_submit;        /* seconds on the server's monotonic clock            */
    double t_start;         /* admitted to a slot                                 */
    double t_done;          /* outputs complete on the device                     */
} wg_result;

/* Start a server on `device` with at most max_inflight concurrent requests,
 * each on its own stream, and a device-memory budget for resident handles.
 * Requests start in arrival order, except that requests whose grid has 2^21
 * cells or more (128^3 and 256^3, say: each one's distance walk alone holds
 * every compute unit) take turns:
 * while one holds the turn, a free slot takes the first smaller request
 * queued.  A turn lasts to the end of the request, or, when another such
 * request was queued as it started and it has no reverse pass (d_gphi null),
 * until its distance walk is enqueued (the
 * next one's splat and solve then run beside the walk; that request's
 * stats.ms[4] is reported as 0). */
int wg_server_create(wg_server **out, size_t hbm_budget_bytes, int max_inflight, int device);

/* Queue a request (inputs are copied before return); *ticket identifies it.
 * WG_ENOMEM if the request alone exceeds the budget. */
int wg_submit(wg_server *s, const wg_request *req, uint64_t *ticket);

/* WG_PENDING while the request runs; otherwise its final status with *out
 * filled, after which the ticket is released.  WG_ESTATE for unknown tickets. */
int wg_poll(wg_server *s, uint64_t ticket, wg_result *out);

/* Seconds on the server's clock (same origin as wg_result times). */
double wg_server_now(wg_server *s);

/* Waits for all queued requests, then stops the worker threads. */
void wg_server_destroy(wg_server *s);

/* ---------------------------------------------------------------------------
 * Kernel timing (instrumentation, off by default)
 * ------------------------------------------------------------------------- */

/* Kernel kinds: the fused splat + divergence; the finest-level PCG direction
 * update fused with the 7-point operator; the finest-level V-cycle pass
 * before the coarse correction (pre-smoothing, residual and restriction in one
 * kernel); the FP64 residual of the refinement; the finest-level pass after
 * it (prolongation and post-smoothing in one kernel); the CG vector update;
 * Marching Cubes (count, scan, emit, boxes); the distance walk; query
 * sampling.  "units" accumulate the algorithmic bytes each launch
 * must move (the bytes per cell, point or query of that kernel times the
 * cells, points or queries it processes), except for the distance walk, whose
 * units are grid nodes. */
enum {
    WG_PROF_SPLAT = 0,
    WG_PROF_SWEEP = 1,
    WG_PROF_SMOOTH = 2,
    WG_PROF_RESID64 = 3,
    WG_PROF_TRANSFER = 4,
    WG_PROF_CGUPDATE = 5,
    WG_PROF_MC = 6,
    WG_PROF_SDF = 7,
    WG_PROF_SAMPLE = 8,
    WG_PROF_KINDS = 9
};

/* Enable timing for the kinds whose bit (1 << kind) is set (0 disables).
 * Each timed launch is bracketed by two HIP events on its own stream. */
void wg_profile_enable(unsigned kinds_mask);

/* Totals since the last reset for one kind: summed launch durations (ms),
 * launch count and processed units.  Waits for the pending events. */
int wg_profile_read(int kind, double *total_ms, int64_t *launches, double *units);

void wg_profile_reset(void);

/* Work of the distance walk (Eq. 33's minimum over triangles, taken by a
 * hierarchy walk), counted on the device while WG_PROF_SDF is enabled, summed
 * over launches since the last wg_profile_reset: out[0] node-triangle distance
 * tests, out[1] node-box bound tests against axis-aligned boxes, out[2]
 * against oriented boxes, out[3] node slots walked (tiles x nodes per tile).
 * A wavefront tests every visited triangle and box for each of its nodes.
 * Synchronises the device. */
int wg_profile_walk_counts(uint64_t out[4]);

/* Streaming device copy of `bytes` (a multiple of 16, both pointers 16-byte
 * aligned) from d_src to d_dst on hip_stream: the bandwidth reference that
 * the library's HBM fractions are compared with (instrumentation).  Enqueues
 * and returns; WG_EINVAL for misaligned or null arguments. */
int wg_stream_copy(void *d_dst, const void *d_src, size_t bytes, void *hip_stream);

/* ---- Unoriented clouds: normals and their orientation (Sec. 2.1-2.2) ----- */

/* Unoriented normals by distance-weighted PCA (Sec. 2.1, Eq. 1-6).  For each
 * point x_i: the neighbours within `radius` (Eq. 1; x_i itself included;
 * membership decided on the FP32 squared distance, summed x, y, z, against
 * radius^2 rounded to FP32), weights 1/(|x_j - x_i| + eps) (Eq. 2), the
 * weighted centroid (Eq. 3) and covariance about it (Eq. 4) in FP64; the
 * normal is the unit eigenvector of the smallest eigenvalue (Eq. 5-6).
 * d_xyz [n_points][3] float32 (device); d_nrm_out [n_points][3] float32
 * (device; sign arbitrary, undefined where the two smallest eigenvalues
 * coincide, as for a point without neighbours).  eps <= 0 selects
 * 1e-6 radius.  Allocates its work buffers on the stream and frees them;
 * blocks until done.  WG_EINVAL for n_points < 1, radius <= 0 or a
 * non-finite coordinate. */
int wg_dpca_normals(const float *d_xyz, int n_points, double radius, double eps, float *d_nrm_out,
                    void *hip_stream);

typedef struct {
    double gamma_r; /* detection-radius expansion factor (Eq. 14; Table 1: 2.5), >= 1 */
    int n_tol;      /* initial-one threshold of the refinement (Table 1: 2) */
    int refine;     /* 1: the refinement iterations of Sec. 2.2; 0: plain parity (Eq. 12) */
} wg_orient_opts;

typedef struct {
    double spacing2;  /* max_i min_{j != i} of the FP32 squared distance */
    double rd0, rd;   /* Eq. 13 and Eq. 14 */
    double ds;        /* probe spacing, 0.75 rd */
    int n_probes;     /* M: probes m = 0..M per ray, ceil((box diagonal + rd) / ds) + 1 */
    int n_flipped;    /* normals whose sign this call changed */
} wg_orient_info;

/* Outward orientation by point-cloud ray casting (Sec. 2.2, Eq. 7-14).  Rays
 * from each point along +n and -n, probes y_m = x + m ds n (FP32), detection
 * d_m = [some point within rd of y_m] (FP32 squared distances against rd^2
 * rounded to FP32), N = (1 -> 0 transitions) - 1 and N_one = the leading
 * detecting probes.  Iteration 0 flips an odd N; with refine, a normal whose
 * initial block is longer than n_tol probes is flipped (iteration 1) and
 * flipped back if that direction crosses more often than the other
 * (iteration 2).  d_nrm [n_points][3] float32, flipped in place (signs only);
 * d_counts NULL or [n_points][4] int32 (N, N_one along the input +n, then
 * along -n); info NULL or filled.  Allocates its work buffers on the stream
 * and frees them; blocks until done.  WG_ENUMERIC for a NaN or infinite
 * normal; WG_EINVAL for n_points < 2, gamma_r < 1,
 * a non-finite coordinate, or a cloud whose points all have coincident twins
 * (rd = 0) or one whose rays would need more than 1e5 probes. */
int wg_orient_normals(const float *d_xyz, int n_points, float *d_nrm, const wg_orient_opts *opts,
                      int32_t *d_counts, wg_orient_info *info, void *hip_stream);

/* Thread-local message of the last failing call on this thread. */
const char *wg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* WGEO_H */
