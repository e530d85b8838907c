// Reconstruction handle (internal): owns the resident device state of one
// grid and drives the forward and reverse passes.
#pragma once

#include "kernels.h"
#include "solver.h"
#include "surface.h"

namespace wg {

// Validates precision / deterministic (WG_EINVAL otherwise).
void check_opts(const wg_solve_opts &o);

class Recon {
  public:
    Recon(const wg_grid &g, int max_points, hipStream_t s);
    ~Recon();
    static size_t footprint(const wg_grid &g, int max_points);

    // pipelined: leave the distance walk running on the second stream (it
    // overlaps the splat and solve of the next forward); otherwise the handle
    // stream waits for it before returning.
    int forward(const float *xyz, const float *nrm, int npts, const wg_solve_opts &o, wg_stats *st,
                bool pipelined = false);
    // pipelined: sample on the second stream right behind the distance walk.
    int sample(const float *q, int nq, float *phi, float *nrm, bool pipelined = false);
    // Order the handle stream after everything enqueued on the second stream.
    void join();
    // join(), then wait on the host for the last walk and check its flags.
    void finish();
    // distance walk as a persistent kernel (default) or one workgroup per 4 tiles
    void set_persistent(bool on) { surf_.set_persistent(on); }
    // Called with the extra device bytes before the surface buffers grow past
    // the handle's footprint (a larger mesh than any before); may throw.
    void set_grow_hook(std::function<void(size_t)> f) { surf_.set_grow_hook(std::move(f)); }
    int backward(const float *q, int nq, const float *gphi_q, const float *gnrm_q, float *gxyz, float *gnrm_pts,
                 float *gq, const wg_solve_opts &o, wg_stats *st);
    int poisson(const float *b, double *x, int bc, const wg_solve_opts &o, wg_stats *st);
    // Surface and signed distance of a given FP64 field at iso-value c.
    int sdf_from_field(const double *chi, double c, wg_stats *st);
    int mg_apply(const float *r, float *z, int bc);
    int get_fields(float *b, double *chi, float *phi, int32_t *keys);
    int get_mesh(float *tris, int32_t *info, int64_t max_tris, int64_t *n_tris);

    size_t bytes_resident() const;
    const wg_grid &grid() const { return grid_; }
    int max_points() const { return max_points_; }
    hipStream_t stream() const { return st_; }

  private:
    static void plan(Arena &a, const wg_grid &g, int max_points);
    void check_err(const char *what);
    void extract_surface();
    void walk(bool pipelined, bool related);
    void wait_sdf();

    wg_grid grid_;
    int max_points_;
    hipStream_t st_;
    Dims d_{};
    GridF gf_{};
    Arena arena_;
    Solver solver_;
    Surface surf_;
    float *b_ = nullptr, *phi_ = nullptr, *gphi_ = nullptr, *gchi_ = nullptr;
    double *chi_ = nullptr, *lam_ = nullptr, *iso_part_ = nullptr, *scal_ = nullptr;
    int32_t *argmin_ = nullptr, *keys_ = nullptr, *tile_of_ = nullptr;
    uint32_t *rank_ = nullptr, *perm_ = nullptr, *tile_cnt_ = nullptr, *tile_off_ = nullptr, *tile_act_ = nullptr;
    uint32_t *tile_blk_ = nullptr, *tile_tot_ = nullptr, *ch_cnt_ = nullptr, *ch_off_ = nullptr, *ch_act_ = nullptr;
    uint32_t *ch_blk_ = nullptr, *ch_tot_ = nullptr, *chunk_tile_ = nullptr;
    TileDims td_{};
    float *xyz_ = nullptr, *nrm_ = nullptr;
    // scal_[0..7] (c, c shifted, g_c) and err_[0..3] are one device block,
    // mirrored whole into hm_
    int *err_ = nullptr;
    FixedScale *fix_ = nullptr;   // fixed-point unit of the deterministic splat
    uint32_t *nmax_ = nullptr;    // largest |normal component| (float bits)
    struct Mirror {
        double scal[8];
        int err[4];
    };
    HostMapped<Mirror> hm_;
    int n_points_ = 0;
    bool have_forward_ = false;
    bool field_only_ = false;   // the last surface came from wg_sdf_from_field (no cloud)
    int quad_ = WG_VERTEX_QUADRATURE;   // quadrature of the last forward's system
    // second stream: the distance walk (and pipelined sampling)
    hipStream_t sdf_st_ = nullptr;
    hipEvent_t ev_mc_ = nullptr, ev_sdf_ = nullptr, ev_tail_ = nullptr;
    bool sdf_pending_ = false;   // ev_sdf_ recorded and not yet waited for on st_
    bool tail_pending_ = false;  // work after ev_sdf_ on sdf_st_ (pipelined sampling)
    double chi_mean_ = 0.0, iso_c_ = 0.0;
};


}  // namespace wg
