// Exclusive scan of per-item counts with compaction of the non-zero items
// (internal).  k_scan_partial -> k_scan_top -> k_scan_final turn counts[n]
// into exclusive offsets[n] and the increasing list of items with a non-zero
// count; totals = {sum of counts, number of non-zero items}.  Each block
// handles kScanBlock items; k_scan_top is a single block looping over the
// block sums, so any n works.
#pragma once

#include "common.h"

namespace wg {
namespace scan {
namespace {

// Exclusive block scan of (count, nonzero-flag) pairs over 256 threads.
__device__ __forceinline__ void block_scan2(uint32_t a, uint32_t f, uint32_t &ea, uint32_t &ef, uint32_t &ta,
                                            uint32_t &tf) {
    __shared__ uint32_t wa[4], wf[4];
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    uint32_t xa = a, xf = f;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t ya = __shfl_up(xa, o, 64), yf = __shfl_up(xf, o, 64);
        if (lane >= o) {
            xa += ya;
            xf += yf;
        }
    }
    if (lane == 63) {
        wa[w] = xa;
        wf[w] = xf;
    }
    __syncthreads();
    uint32_t pa = 0, pf = 0;
    for (int k = 0; k < w; ++k) {
        pa += wa[k];
        pf += wf[k];
    }
    ta = wa[0] + wa[1] + wa[2] + wa[3];
    tf = wf[0] + wf[1] + wf[2] + wf[3];
    ea = pa + xa - a;
    ef = pf + xf - f;
    __syncthreads();
}

constexpr int kScanPer = 4;      // entries per thread
constexpr int kScanBlock = 256 * kScanPer;

__global__ __launch_bounds__(256) void k_scan_partial(const uint32_t *cnt, uint32_t n, uint32_t *blk) {
    uint32_t a = 0, f = 0;
    for (int q = 0; q < kScanPer; ++q) {
        uint32_t idx = blockIdx.x * kScanBlock + threadIdx.x * kScanPer + q;
        if (idx < n) {
            a += cnt[idx];
            f += cnt[idx] != 0;
        }
    }
    uint32_t ea, ef, ta, tf;
    block_scan2(a, f, ea, ef, ta, tf);
    if (threadIdx.x == 0) {
        blk[2 * blockIdx.x] = ta;
        blk[2 * blockIdx.x + 1] = tf;
    }
}

__global__ __launch_bounds__(256) void k_scan_top(uint32_t *blk, uint32_t nblk, uint32_t *totals) {
    uint32_t carry_a = 0, carry_f = 0;
    for (uint32_t base = 0; base < nblk; base += 256) {
        uint32_t idx = base + threadIdx.x;
        uint32_t a = idx < nblk ? blk[2 * idx] : 0, f = idx < nblk ? blk[2 * idx + 1] : 0;
        uint32_t ea, ef, ta, tf;
        block_scan2(a, f, ea, ef, ta, tf);
        if (idx < nblk) {
            blk[2 * idx] = carry_a + ea;
            blk[2 * idx + 1] = carry_f + ef;
        }
        carry_a += ta;
        carry_f += tf;
    }
    if (threadIdx.x == 0) {
        totals[0] = carry_a;
        totals[1] = carry_f;
    }
}

__global__ __launch_bounds__(256) void k_scan_final(const uint32_t *cnt, uint32_t n, const uint32_t *blk,
                                                     uint32_t *off, uint32_t *active) {
    uint32_t v[kScanPer];
    uint32_t a = 0, f = 0;
    for (int q = 0; q < kScanPer; ++q) {
        uint32_t idx = blockIdx.x * kScanBlock + threadIdx.x * kScanPer + q;
        v[q] = idx < n ? cnt[idx] : 0;
        a += v[q];
        f += v[q] != 0;
    }
    uint32_t ea, ef, ta, tf;
    block_scan2(a, f, ea, ef, ta, tf);
    uint32_t oa = blk[2 * blockIdx.x] + ea, of = blk[2 * blockIdx.x + 1] + ef;
    for (int q = 0; q < kScanPer; ++q) {
        uint32_t idx = blockIdx.x * kScanBlock + threadIdx.x * kScanPer + q;
        if (idx < n) {
            off[idx] = oa;
            if (v[q]) active[of++] = idx;
            oa += v[q];
        }
    }
}

}  // namespace
}  // namespace scan
}  // namespace wg
