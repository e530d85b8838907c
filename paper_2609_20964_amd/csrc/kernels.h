// Kernel declarations shared between the HIP translation units (internal).
#pragma once

#include "common.h"

namespace wg {

// Grid geometry handed to point- and query-side kernels.
struct GridF {
    Dims d;
    double lo[3];
    double h;
};

// Points are binned into kTile^3-cell tiles for the splat.
constexpr int kTile = 8;
constexpr uint32_t kChunk = 256;   // points per splat workgroup pass
struct TileDims {
    int tx, ty, tz;
    __host__ __device__ int count() const { return tx * ty * tz; }
};
inline TileDims tile_dims(const Dims &d) {
    return {(d.nx + kTile - 1) / kTile, (d.ny + kTile - 1) / kTile, (d.nz + kTile - 1) / kTile};
}

// ---- recon.hip -------------------------------------------------------------
// Copies n 32-bit words into host-mapped memory, then stores seq to *seq_dst.
// One wavefront: it fits beside a resident persistent kernel, where the
// runtime's copy kernels (several wavefronts per SIMD) wait until that
// kernel's workgroups retire.
__global__ void k_mirror_words(const uint32_t *src, uint32_t *dst, int n, unsigned *seq_dst, unsigned seq);

// Host-mapped, coherent pinned memory for a small device record the host reads:
// fetch() enqueues the copy, wait() returns once it has landed.
template <class T> class HostMapped {
  public:
    HostMapped() = default;
    HostMapped(const HostMapped &) = delete;
    HostMapped &operator=(const HostMapped &) = delete;
    ~HostMapped() {
        if (host_) (void)hipHostFree(host_);
    }
    void alloc() {
        WG_HIP(hipHostMalloc((void **)&host_, sizeof(Rec), hipHostMallocMapped | hipHostMallocCoherent));
        WG_HIP(hipHostGetDevicePointer((void **)&dev_, host_, 0));
        host_->seq = seq_;
    }
    void fetch(const void *src, hipStream_t s) {
        static_assert(sizeof(T) % 4 == 0, "mirrored records are whole 32-bit words");
        k_mirror_words<<<1, kWave, 0, s>>>(static_cast<const uint32_t *>(src), reinterpret_cast<uint32_t *>(&dev_->v),
                                          (int)(sizeof(T) / 4), &dev_->seq, ++seq_);
        WG_LAUNCH_CHECK();
        s_ = s;
    }
    // the record of the last fetch()
    const T &wait() const {
        wait_published(&host_->seq, seq_, s_);
        return host_->v;
    }

  private:
    struct Rec {
        T v;
        unsigned seq;
    };
    Rec *host_ = nullptr, *dev_ = nullptr;
    unsigned seq_ = 0;
    hipStream_t s_ = nullptr;
};

// ---- splat.hip -------------------------------------------------------------
// Fixed-point unit of the deterministic splat: value = sum * inv, scale = 1 / inv.
struct FixedScale {
    double scale, inv;
};
enum { kSplatF32 = 0, kSplatFixed = 1, kSplatFixed64 = 2, kSplatExact = 3 };

__global__ void k_bin_points(const float *xyz, const float *nrm, int npts, GridF g, TileDims td, int32_t *keys,
                             float *xyz_c, float *nrm_c, int32_t *tile_of, uint32_t *rank, uint32_t *tile_cnt,
                             int *err, uint32_t *nmax_bits);
__global__ void k_tile_scatter(const int32_t *tile_of, const uint32_t *rank, const uint32_t *tile_off, int npts,
                               uint32_t *perm);
__global__ void k_chunk_counts(const uint32_t *tile_cnt, uint32_t ntiles, uint32_t *ch_cnt);
__global__ void k_chunk_tiles(const uint32_t *ch_cnt, const uint32_t *ch_off, uint32_t ntiles, uint32_t *chunk_tile);
template <int Mode>
__global__ void k_splat_chunks(const uint32_t *perm, const uint32_t *tile_off, const uint32_t *tile_cnt,
                               const uint32_t *ch_off, const uint32_t *chunk_tile, const uint32_t *n_chunks,
                               const float *xyz_c, const float *nrm_c, GridF g, TileDims td, float *b,
                               unsigned long long *acc, const FixedScale *fix);
__global__ void k_bbox(const float *xyz, int npts, uint32_t *box, int *err);
__global__ void k_fixed_scale(const uint32_t *nmax_bits, int npts, double h, FixedScale *fix, int *err);
template <class T>
__global__ void k_fixed_to_b(const long long *acc, const FixedScale *fix, size_t n, T *b);
__global__ void k_iso_partial(const float *xyz, int npts, GridF g, const double *chi, double *partials);
__global__ void k_iso_finalize(const double *partials, int nb, int npts, double *out);
__global__ void k_iso_absmax(const float *xyz, int npts, GridF g, const double *chi, unsigned long long *w);
__global__ void k_iso_fixed(const float *xyz, int npts, GridF g, const double *chi, unsigned long long *w);
__global__ void k_iso_fixed_finalize(const unsigned long long *w, int npts, double *out);
__global__ void k_iso_T(const float *xyz, int npts, GridF g, const double *g_c, float *g_chi);
// three cell fields (the exact-quadrature g_V by axis)
struct Planes3 {
    float *p[3];
};
template <bool EXACT>
__global__ void k_splat_T(const float *xyz, const float *nrm, const int32_t *keys, int npts, GridF g,
                          const double *lam, Planes3 gvp, const double *chi, const double *g_c, float *gxyz,
                          float *gnrm);
__global__ void k_grad27_T(const double *lam, Dims d, double h, Planes3 gv);

}  // namespace wg
