// Exclusive prefix sum of u32 arrays (reduce, scan the block totals, scan
// down).  Used for the radix-sort digit offsets and the group numbering.
#include "bh_internal.h"
#include "wave.h"

namespace bh {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

int64_t scan_part_len(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

// exclusive scan of one value per thread across a 256-thread block
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t *total, uint32_t *lds /*[4]*/) {
    uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v, lane);
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / 64; ++k) {
        uint32_t t = lds[k];
        if ((uint32_t)k < w) off += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t *__restrict__ in,
                                                              uint32_t n,
                                                              uint32_t *__restrict__ part) {
    __shared__ uint32_t lds[4];
    uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        uint64_t i = base + (uint64_t)k * kScanThreads + threadIdx.x;
        if (i < n) s += in[i];
    }
    s = wave_sum(s);
    if (lane_id() == 0) lds[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = lds[0] + lds[1] + lds[2] + lds[3];
}

__global__ __launch_bounds__(kScanThreads) void k_scan_top(uint32_t *part, uint32_t nb) {
    __shared__ uint32_t lds[4];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += kScanTile) {
        uint32_t v[kScanItems], s = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            uint32_t i = base + threadIdx.x * kScanItems + k;
            v[k] = i < nb ? part[i] : 0u;
            s += v[k];
        }
        uint32_t tot;
        uint32_t off = block_excl_scan(s, &tot, lds) + carry;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            uint32_t i = base + threadIdx.x * kScanItems + k;
            if (i < nb) part[i] = off;
            off += v[k];
        }
        carry += tot;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t *in, uint32_t *out,
                                                            uint32_t n,
                                                            const uint32_t *__restrict__ part) {
    __shared__ uint32_t lds[4];
    __shared__ uint32_t tile[kScanTile];
    uint64_t base = (uint64_t)blockIdx.x * kScanTile;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        uint64_t i = base + (uint64_t)k * kScanThreads + threadIdx.x;
        tile[k * kScanThreads + threadIdx.x] = i < n ? in[i] : 0u;
    }
    __syncthreads();
    uint32_t v[kScanItems], s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = tile[threadIdx.x * kScanItems + k];
        s += v[k];
    }
    uint32_t tot;
    uint32_t off = block_excl_scan(s, &tot, lds) + part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        tile[threadIdx.x * kScanItems + k] = off;
        off += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        uint64_t i = base + (uint64_t)k * kScanThreads + threadIdx.x;
        if (i < n) out[i] = tile[k * kScanThreads + threadIdx.x];
    }
}

void launch_exclusive_scan(const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *part,
                           hipStream_t st) {
    if (n == 0) return;
    uint32_t nb = cdiv(n, kScanTile);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, st, in, n, part);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, st, part, nb);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kScanThreads), 0, st, in, out, n,
                       (const uint32_t *)part);
}

}  // namespace bh
