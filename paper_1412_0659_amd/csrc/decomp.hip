// Cut of the sorted particles into p domains of equal tree-walk work
// (Sec. III.B.1: the cuts balance the floating-point operations of the walk
// kernel, with no domain more than a cap above the average particle count).
//
// The cost of a particle is 23 npp + 65 npc of its group's last walk (the
// operation counts of Sec. VI.A), the same for every particle of a group.
// With S_i the cost of sorted slots [0, i) and W = S_n, cut j is the first
// slot i with S_i p >= W j; since S is non-decreasing, that is the number of
// slots with S_i p < W j.  Three launches:
//   * k_cut_prefix (one workgroup): S at every group start (FP-free, 64-bit);
//   * k_cut_search (one thread per cut): the last group starting below the
//     target, then the slot inside it by one integer division;
//   * k_cut_clamp (one workgroup): the cap, applied in cut order because
//     each bound depends on the previous clamped cut.
// Products S p and W j are formed in 128 bits.
#include "bh_internal.h"

namespace bh {

constexpr int kCutThreads = 1024;
constexpr int kClampTile = 4096;

__device__ __forceinline__ uint64_t group_weight(const uint32_t *npp, const uint32_t *npc,
                                                 uint32_t g) {
    return 23ull * (uint64_t)npp[g] + 65ull * (uint64_t)npc[g];
}

// S[g] = cost of the particles of groups [0, g), S[ng] = W.  Thread t sums a
// contiguous run of groups; the runs are scanned in LDS; each thread then
// writes the prefix of every group of its run.
__global__ __launch_bounds__(kCutThreads) void k_cut_prefix(const uint32_t *__restrict__ gbeg,
                                                            const uint32_t *__restrict__ npp,
                                                            const uint32_t *__restrict__ npc,
                                                            const uint32_t *__restrict__ ngp,
                                                            uint64_t *__restrict__ S) {
    __shared__ uint64_t run[kCutThreads];
    const uint32_t ng = *ngp;
    const uint32_t per = (ng + kCutThreads - 1) / kCutThreads;
    const uint32_t g0 = min(ng, threadIdx.x * per), g1 = min(ng, g0 + per);
    uint64_t sum = 0;
    for (uint32_t g = g0; g < g1; ++g)
        sum += (uint64_t)(gbeg[g + 1] - gbeg[g]) * group_weight(npp, npc, g);
    run[threadIdx.x] = sum;
    __syncthreads();
    for (uint32_t d = 1; d < (uint32_t)kCutThreads; d <<= 1) {  // inclusive scan
        const uint64_t v = threadIdx.x >= d ? run[threadIdx.x - d] : 0ull;
        __syncthreads();
        run[threadIdx.x] += v;
        __syncthreads();
    }
    uint64_t acc = run[threadIdx.x] - sum;
    for (uint32_t g = g0; g < g1; ++g) {
        S[g] = acc;
        acc += (uint64_t)(gbeg[g + 1] - gbeg[g]) * group_weight(npp, npc, g);
    }
    if (threadIdx.x == 0) S[ng] = run[kCutThreads - 1];
}

// cuts[j] for j in [1, p): the number of sorted slots i with S_i p < W j.
__global__ __launch_bounds__(256) void k_cut_search(const uint64_t *__restrict__ S,
                                                    const uint32_t *__restrict__ gbeg,
                                                    const uint32_t *__restrict__ npp,
                                                    const uint32_t *__restrict__ npc,
                                                    const uint32_t *__restrict__ ngp, int32_t p,
                                                    int64_t *__restrict__ cuts) {
    const uint32_t j = blockIdx.x * 256u + threadIdx.x + 1u;
    if (j >= (uint32_t)p) return;
    const uint32_t ng = *ngp;
    typedef unsigned __int128 u128;
    const u128 target = (u128)S[ng] * j;
    // k = number of groups g with S[g] p < target (a prefix: S is non-decreasing)
    uint32_t lo = 0, hi = ng;
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if ((u128)S[mid] * (uint32_t)p < target) lo = mid + 1;
        else hi = mid;
    }
    int64_t cut = 0;
    if (lo > 0) {
        const uint32_t g = lo - 1;
        const uint32_t b = gbeg[g], cnt = gbeg[g + 1] - b;
        const uint64_t w = group_weight(npp, npc, g);
        // slots b + t, t < cnt, have S = S[g] + t w; count those with S p < target
        uint64_t add = cnt;
        if (w != 0) {
            const u128 gap = target - (u128)S[g] * (uint32_t)p;  // > 0
            const u128 step = (u128)w * (uint32_t)p;
            const u128 t = (gap + step - 1) / step;
            if (t < (u128)cnt) add = (uint64_t)t;
        }
        cut = (int64_t)b + (int64_t)add;
    }
    cuts[j] = cut;
}

// cuts[j] clamped to [max(cuts[j-1], n - (p - j) C), min(cuts[j-1] + C, n)],
// in order (C >= 1); a tile of cuts is staged in LDS and thread 0 runs the
// recurrence.
__global__ __launch_bounds__(kCutThreads) void k_cut_clamp(int64_t *cuts, int32_t p, int64_t n,
                                                           int64_t C) {
    __shared__ int64_t buf[kClampTile];
    int64_t prev = 0;  // the clamped cut before the tile (thread 0 only)
    for (int64_t base = 1; base < p; base += kClampTile) {
        const int64_t m = min((int64_t)kClampTile, (int64_t)p - base);
        for (int64_t t = threadIdx.x; t < m; t += kCutThreads) buf[t] = cuts[base + t];
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int64_t t = 0; t < m; ++t) {
                const int64_t rest = (int64_t)p - (base + t);  // domains after this cut
                // n - rest C, or a value <= prev where that is negative (no overflow)
                const int64_t lo = max(prev, rest <= n / C ? n - rest * C : (int64_t)0);
                const int64_t hi = min(prev + C, n);
                prev = min(max(buf[t], lo), hi);
                buf[t] = prev;
            }
        }
        __syncthreads();
        for (int64_t t = threadIdx.x; t < m; t += kCutThreads) cuts[base + t] = buf[t];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cuts[0] = 0;
        cuts[p] = n;
    }
}

void launch_cut(bh_ctx *c, int32_t p, int64_t C, uint64_t *S, int64_t *cuts, hipStream_t st) {
    const Groups &g = c->groups;
    hipLaunchKernelGGL(k_cut_prefix, dim3(1), dim3(kCutThreads), 0, st,
                       (const uint32_t *)g.begin, (const uint32_t *)g.npp,
                       (const uint32_t *)g.npc, (const uint32_t *)g.count_dev, S);
    if (p > 1)
        hipLaunchKernelGGL(k_cut_search, dim3((uint32_t)((p - 1 + 255) / 256)), dim3(256), 0, st,
                           (const uint64_t *)S, (const uint32_t *)g.begin,
                           (const uint32_t *)g.npp, (const uint32_t *)g.npc,
                           (const uint32_t *)g.count_dev, p, cuts);
    hipLaunchKernelGGL(k_cut_clamp, dim3(1), dim3(kCutThreads), 0, st, cuts, p, (int64_t)c->n, C);
}

}  // namespace bh
