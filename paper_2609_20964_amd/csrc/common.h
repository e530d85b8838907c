// Internal helpers shared by the HIP sources of libwgeo.so (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "wgeo.h"

namespace wg {

// Errors inside the library are C++ exceptions carrying a WG_E* code; the ABI
// layer turns them into a return code and the thread-local message.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

inline void hip_check(hipError_t e, const char *what, const char *file, int line) {
    if (e != hipSuccess) {
        int code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? WG_ENOMEM : WG_EDEVICE;
        throw Error(code, std::string(what) + ": " + hipGetErrorString(e) + " (" + file + ":" +
                              std::to_string(line) + ")");
    }
}
#define WG_HIP(x) ::wg::hip_check((x), #x, __FILE__, __LINE__)
#define WG_LAUNCH_CHECK() ::wg::hip_check(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

inline void require(bool ok, int code, const std::string &msg) {
    if (!ok) throw Error(code, msg);
}

// Thread-local message of the last failing ABI call (wg_last_error).
void set_error(const std::string &m);
const char *last_error();

// Wait until a kernel on stream s has stored `want` into the host-mapped word
// *seq (after the data it publishes).  Polling returns as soon as the store
// lands, without a stream synchronisation's completion round trip; the stream
// is queried now and then so that an error, or a stream that drained without
// publishing, ends the wait.
inline void wait_published(const unsigned *seq, unsigned want, hipStream_t s) {
    for (unsigned k = 1;; ++k) {
        if (__atomic_load_n(seq, __ATOMIC_ACQUIRE) == want) return;
        if ((k & 255) == 0) {
            const hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) {
                if (__atomic_load_n(seq, __ATOMIC_ACQUIRE) == want) return;
                throw Error(WG_EDEVICE, "a published result never arrived");
            }
            if (e != hipErrorNotReady) hip_check(e, "hipStreamQuery", __FILE__, __LINE__);
        }
    }
}

constexpr int kBlock = 256;   // threads per workgroup for 1-D kernels
constexpr int kWave = 64;

// Grid extents handed to kernels.  bc_sign is -1 for zero-flux (Neumann)
// boundaries and +1 for the cell-centred Dirichlet test mode: a cell with nb
// boundary faces has diagonal 6 + bc_sign * nb in the 7-point operator.
struct Dims {
    int nx, ny, nz;
    int bc_sign;
    __host__ __device__ size_t count() const { return (size_t)nx * ny * nz; }
};

// One device allocation carved into 256-byte aligned sub-buffers.
class Arena {
  public:
    void reserve(size_t bytes) { plan_ += (bytes + 255) & ~size_t(255); }
    size_t planned() const { return plan_; }
    void allocate() {
        if (plan_ && !base_) WG_HIP(hipMalloc(&base_, plan_));
        used_ = 0;
    }
    // Carve from caller-owned device memory (256-byte aligned, `bytes` long)
    // instead of allocating; release() then frees nothing.
    void adopt(void *base, size_t bytes) {
        base_ = base;
        plan_ = bytes;
        used_ = 0;
        owned_ = false;
    }
    template <class T> T *take(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
        require(used_ + bytes <= plan_, WG_EDEVICE, "arena overflow");
        T *p = reinterpret_cast<T *>(static_cast<char *>(base_) + used_);
        used_ += bytes;
        return p;
    }
    void release() {
        if (base_ && owned_) (void)hipFree(base_);
        base_ = nullptr;
        plan_ = used_ = 0;
        owned_ = true;
    }
    ~Arena() { release(); }

  private:
    void *base_ = nullptr;
    size_t plan_ = 0, used_ = 0;
    bool owned_ = true;
};

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

// Blocks are dealt round-robin to the 8 XCDs (block b runs on XCD b % 8).
// Remap so each XCD gets one contiguous run of logical tiles: neighbouring
// tiles then share halo rows in the same L2.
__device__ __forceinline__ unsigned xcd_logical_block(unsigned b, unsigned nblocks) {
    const unsigned nx = 8;
    unsigned per = nblocks / nx, rem = nblocks % nx;
    unsigned x = b % nx, slot = b / nx;
    // XCD x owns logical blocks [start(x), start(x) + per + (x < rem))
    unsigned start = x * per + (x < rem ? x : rem);
    return start + slot;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_sumf(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Deterministic block sum of NV doubles; thread 0 gets the totals.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*lds)[NV]) {
    int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    int lane = tid % 64;
    int wid = tid / 64;
    int nwaves = (blockDim.x * blockDim.y * blockDim.z + 63) / 64;
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
        for (int k = 0; k < NV; ++k) lds[wid][k] = v[k];
    __syncthreads();
    if (wid == 0) {
        for (int k = 0; k < NV; ++k) {
            double t = lane < nwaves ? lds[lane][k] : 0.0;
            v[k] = wave_sum(t);
        }
    }
}

inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace wg
