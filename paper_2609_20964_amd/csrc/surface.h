// Surface extraction, signed distance and sampling on the device (internal).
//
// Marching Cubes (Warp-Geo Eq. 27-28) runs on the dual lattice whose cube
// corners are the cell centres.  Cubes are grouped into 4x4x4 bricks (one
// wavefront each); bricks, and the cubes inside a brick, are visited in Morton
// order, so the triangle list is Morton ordered.  Groups of 4 consecutive
// triangles are the leaves of an 8-ary hierarchy built bottom-up over that
// order: oriented boxes (thin along the patch normal) at the leaves,
// axis-aligned boxes above.  The signed distance (Eq. 29-34) of every grid
// node is the exact minimum over all triangles: one wavefront per 4x4x16 node
// tile (4x4x4 on grids below 2^23 nodes) walks the hierarchy together, pruning
// a box only when it is farther than every lane's current best, so the result
// equals the brute-force minimum.
#pragma once

#include <functional>

#include "kernels.h"

namespace wg {

struct SurfaceCounts {
    uint32_t n_tris;
    uint32_t n_active;    // non-empty bricks
};

class Surface {
  public:
    static void plan(Arena &a, const Dims &d);
    // Bytes of the triangle and hierarchy buffers a handle starts with (a
    // part of its footprint): room for about 4 triangles per cell of the
    // grid's largest face.
    static size_t initial_bytes(const Dims &d);
    static uint32_t initial_tris(const Dims &d);
    void bind(Arena &a, const Dims &d, hipStream_t s);
    ~Surface();
    // Called with the extra bytes before the triangle or hierarchy buffers
    // grow past what they hold; it may throw (WG_ENOMEM) to refuse.
    void set_grow_hook(std::function<void(size_t)> f) { grow_hook_ = std::move(f); }

    // Side of every node (chi >= c: outside) and the mesh of {chi = *c} (c on
    // the device).  Host-synchronising: returns the triangle count.  The
    // distance walk reads the node sides, not chi.
    uint32_t extract(const double *chi, const double *c);
    // phi and the nearest-triangle index on every node, on stream s (after
    // extract has completed there).  beside: the next step's solve will run
    // meanwhile (a persistent walk then leaves it room).  related: the surface
    // is close to the last one walked (a warm-started step), so that walk's
    // tile costs order this one; otherwise, on large grids, the depth of each
    // tile inside the surface does.  No result depends on the order.
    void sdf(double h, float *phi, int32_t *argmin, int *err, hipStream_t s, bool beside, bool related);
    // reverse of sdf through the vertices: g_chi, g_c (+=)
    void sdf_T(const float *gphi, const double *chi, const double *c, const int32_t *argmin, double h,
               float *g_chi, double *g_c);

    uint32_t n_tris() const { return cnt_.n_tris; }
    // first n triangles as float[9] (vertices in grid units), rebuilt from the
    // field chi and iso-value *c the mesh was extracted from
    void export_tris(const double *chi, const double *c, float *out, uint32_t n);
    // persistent = true (default): the distance walk runs as many workgroups
    // as fit on the device at once, less a few free slots for the other
    // streams' work, each taking tiles from a queue (no tail).
    // false: one workgroup per 4 tiles, so the walks of concurrent handles
    // interleave workgroup by workgroup.
    void set_persistent(bool on);
    const float4 *tris() const { return tri_; }
    const int2 *tri_info() const { return info_; }
    size_t bytes() const { return buf_bytes(cap_, box_cap_) + retired_bytes_; }

  private:
    static size_t buf_bytes(size_t tri_cap, size_t box_cap) {
        return tri_cap * (4 * sizeof(float4) + sizeof(int2)) + box_cap * 6 * sizeof(float4);
    }
    void ensure_capacity(uint32_t tris);

    hipStream_t st_ = nullptr;
    Dims d_{};
    int nb_[3] = {0, 0, 0};        // bricks per axis
    int mbits_ = 0;                // Morton bits per axis
    size_t nbricks_pad_ = 0;       // (2^mbits)^3
    uint32_t *cnt_b_ = nullptr, *off_b_ = nullptr, *active_ = nullptr, *blk_ = nullptr;
    SurfaceCounts *dcnt_ = nullptr;
    HostMapped<SurfaceCounts> hcnt_;
    uint32_t *sign_ = nullptr;     // [ceil(N / 32)] node sides
    uint32_t *next_tile_ = nullptr;   // per-slab work counters of the distance walk
    uint32_t *tile_cost_ = nullptr;   // work per tile recorded by the last walk
    uint32_t *walk_order_ = nullptr;  // tiles of each slab, costliest first
    int32_t *seed_ = nullptr;         // nearest triangle of each seed-lattice node
    bool have_order_ = false;
    hipStream_t seed_st_ = nullptr;   // the seed search, beside the walk
    hipEvent_t ev_pre_ = nullptr, ev_seed_ = nullptr;
    bool persistent_ = true;
    unsigned sdf_blocks_full_ = 0, sdf_blocks_beside_ = 0;   // persistent workgroups: alone, beside a solve
    SurfaceCounts cnt_{};
    // growable
    float4 *tri_ = nullptr;        // [cap][4] records (a,|ab|^2) (ab,ab.ac) (ac,|ac|^2) (reciprocals)
    int2 *info_ = nullptr;         // [cap]
    float4 *box_ = nullptr;        // [box_cap][4] oriented-box nodes of every hierarchy level
    float4 *aabb_ = nullptr;       // [box_cap][2] axis-aligned box of every node (the walk reads the leaves')
    size_t cap_ = 0, box_cap_ = 0;
    // Buffers outgrown by a larger surface.  They are freed with the handle,
    // not when outgrown: hipFree waits for the whole device, which would stall
    // every other stream's work (other requests of a server) mid-forward.
    std::vector<void *> retired_;
    size_t retired_bytes_ = 0;
    std::function<void(size_t)> grow_hook_;
    std::vector<uint32_t> level_off_, level_cnt_;
    int levels_ = 0;
};

// Sampling (F8) and its reverse (B1); phi is the node SDF.
void launch_sample(const GridF &g, const float *phi, const float *q, int nq, float *out_phi, float *out_nrm,
                   hipStream_t s);
void launch_sample_T(const GridF &g, const float *phi, const float *q, int nq, const float *gphi_q,
                     const float *gnrm_q, float *gphi, float *gq, hipStream_t s);

}  // namespace wg
