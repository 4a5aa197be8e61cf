// Octree construction from sorted Morton keys, level by level (Sec. I.A:
// octants are split until a cell holds at most nleaf particles; Table II
// "Tree-construction"), and the target groups of the walk.
//
// Cells are numbered breadth first: the cells of level l, in key order,
// then those of level l + 1.  A cell (l, P) with more than nleaf particles
// and l < 21 gets one child per non-empty 3-bit digit d, found by binary
// search for the key bound (8 P + d) << 3 (20 - l) inside the cell's range.
// Each level takes three launches over a fixed grid that reads the level's
// cell range from device memory (count children / scan block totals / write
// children), so the build never waits on the host.  On the top levels the
// searches are replaced by a table: for every key prefix q of level
// kTableLevel, lbt[q] is the first sorted slot whose key is >= q shifted to a
// full key (a lower bound over all keys, so inside a cell it is exactly the
// bound the search would find); one launch of 8^kTableLevel independent
// searches fills it per build.
#include "bh_internal.h"
#include "wave.h"

namespace bh {

constexpr int kBuildThreads = 256;
constexpr uint32_t kFewCells = 16384;  // levels with fewer cells are latency bound

__device__ __forceinline__ uint32_t key_lower_bound(const uint64_t *__restrict__ k, uint32_t lo,
                                                    uint32_t hi, uint64_t v) {
    while (lo < hi) {
        uint32_t mid = lo + ((hi - lo) >> 1);
        if (k[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// digit boundaries of the children of cell c (level l): bnd[0] = begin,
// bnd[8] = end; child d holds [bnd[d], bnd[d+1]).  On a level of few cells
// (latency bound: the top of the tree) a large range runs the seven
// searches in lock step over the whole range, so their loads overlap
// instead of waiting on each other; otherwise the searches are chained,
// each starting at the previous bound (fewer loads).
__device__ __forceinline__ void child_bounds(const uint64_t *__restrict__ key,
                                             const uint32_t *__restrict__ lbt, uint64_t P,
                                             uint32_t b, uint32_t e, int l, bool few,
                                             uint32_t bnd[9]) {
    uint32_t shift = 3u * (kKeyBits - 1 - l);
    bnd[0] = b;
    bnd[8] = e;
    if (l < kTableLevel) {  // children on a level <= kTableLevel: look the bounds up
        const uint32_t up = 3u * (uint32_t)(kTableLevel - 1 - l);
#pragma unroll
        for (uint32_t d = 1; d < 8; ++d) bnd[d] = lbt[((P << 3) | d) << up];
        return;
    }
    if (few && e - b >= 256u) {
        uint32_t base[8];
#pragma unroll
        for (uint32_t d = 1; d < 8; ++d) base[d] = b;
        uint32_t len = e - b;
        while (len > 1u) {
            const uint32_t half = len >> 1;
#pragma unroll
            for (uint32_t d = 1; d < 8; ++d)
                base[d] = key[base[d] + half] < (((P << 3) | d) << shift) ? base[d] + half
                                                                          : base[d];
            len -= half;
        }
#pragma unroll
        for (uint32_t d = 1; d < 8; ++d)
            bnd[d] = base[d] + (key[base[d]] < (((P << 3) | d) << shift) ? 1u : 0u);
        return;
    }
#pragma unroll
    for (uint32_t d = 1; d < 8; ++d)
        bnd[d] = key_lower_bound(key, bnd[d - 1], e, ((P << 3) | d) << shift);
}

__global__ void k_build_init(Cells c, uint32_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c.prefix[0] = 0;
        c.level[0] = 0;
        c.begin[0] = 0;
        c.count[0] = n;
        c.child0[0] = kNone;
        c.nchild[0] = 0;
        c.parent[0] = kNone;
    }
    if (blockIdx.x == 0 && threadIdx.x < kLsSize) c.ls[threadIdx.x] = threadIdx.x == 0 ? 0u : 1u;
}

__device__ __forceinline__ void level_chunk(const Cells &c, int l, uint32_t &cs, uint32_t &ce) {
    uint32_t first = c.ls[l], last = c.ls[l + 1];
    uint32_t chunk = (last - first + gridDim.x - 1) / gridDim.x;
    cs = first + blockIdx.x * chunk;
    ce = min(last, cs + chunk);
    if (cs > ce) cs = ce;
}

__global__ __launch_bounds__(kBuildThreads) void k_build_count(Cells c,
                                                               const uint64_t *__restrict__ key,
                                                               int l, uint32_t nleaf,
                                                               uint32_t nmax) {
    __shared__ uint32_t lds[4];
    uint32_t cs, ce;
    level_chunk(c, l, cs, ce);
    const uint32_t first = c.ls[l];
    const bool few = c.ls[l + 1] - first < kFewCells;
    uint32_t sum = 0;
    for (uint32_t i = cs + threadIdx.x; i < ce; i += kBuildThreads) {
        uint32_t nch = 0;
        uint32_t cnt = c.count[i];
        if (cnt > nleaf) {
            uint32_t bnd[9];
            uint32_t b = c.begin[i];
            child_bounds(key, c.lbt, c.prefix[i], b, b + cnt, l, few, bnd);
#pragma unroll
            for (int d = 0; d < 8; ++d) nch += bnd[d + 1] > bnd[d];
            // kept for the write pass (a level holds at most nmax cells)
            if (i - first < nmax) {
                uint4 *cb = reinterpret_cast<uint4 *>(c.cbnd + 8 * (size_t)(i - first));
                cb[0] = make_uint4(bnd[1], bnd[2], bnd[3], bnd[4]);
                cb[1] = make_uint4(bnd[5], bnd[6], bnd[7], bnd[8]);
            }
        }
        c.nchild[i] = nch;
        sum += nch;
    }
    sum = wave_sum(sum);
    if (lane_id() == 0) lds[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) c.part[blockIdx.x] = lds[0] + lds[1] + lds[2] + lds[3];
}

// exclusive scan of the kBuildGrid block totals; sets the end of level l + 1
__global__ __launch_bounds__(kBuildThreads) void k_build_scan(Cells c, int l, uint32_t cap,
                                                              uint32_t *status) {
    __shared__ uint32_t lds[4];
    constexpr int per = kBuildGrid / kBuildThreads;
    uint32_t v[per], s = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        v[k] = c.part[threadIdx.x * per + k];
        s += v[k];
    }
    uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(s, lane);
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (uint32_t k = 0; k < 4; ++k) {
        if (k < w) off += lds[k];
        tot += lds[k];
    }
    off += inc - s;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        c.part[threadIdx.x * per + k] = off;
        off += v[k];
    }
    if (threadIdx.x == 0) {
        uint32_t end = c.ls[l + 1] + tot;
        if (end > cap) {
            atomicOr(status, kStOverflow);
            end = cap;
        }
        c.ls[l + 2] = end;
    }
}

__global__ __launch_bounds__(kBuildThreads) void k_build_write(Cells c,
                                                               const uint64_t *__restrict__ key,
                                                               int l, uint32_t cap,
                                                               uint32_t nmax) {
    __shared__ uint32_t lds[4];
    uint32_t cs, ce;
    level_chunk(c, l, cs, ce);
    const uint32_t first = c.ls[l];
    const bool few = c.ls[l + 1] - first < kFewCells;
    uint32_t carry = c.ls[l + 1] + c.part[blockIdx.x];
    uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    for (uint32_t base = cs; base < ce; base += kBuildThreads) {
        uint32_t i = base + threadIdx.x;
        uint32_t v = i < ce ? c.nchild[i] : 0u;
        uint32_t inc = wave_incl_scan(v, lane);
        if (lane == 63) lds[w] = inc;
        __syncthreads();
        uint32_t off = 0, tot = 0;
        for (uint32_t k = 0; k < 4; ++k) {
            if (k < w) off += lds[k];
            tot += lds[k];
        }
        __syncthreads();
        if (v > 0) {
            uint32_t ch = carry + off + inc - v;
            c.child0[i] = ch;
            uint32_t b = c.begin[i];
            uint64_t P = c.prefix[i];
            uint32_t bnd[9];
            if (i - first < nmax) {  // the bounds the count pass found
                const uint4 *cb = reinterpret_cast<const uint4 *>(c.cbnd + 8 * (size_t)(i - first));
                const uint4 u = cb[0], w = cb[1];
                bnd[0] = b;
                bnd[1] = u.x; bnd[2] = u.y; bnd[3] = u.z; bnd[4] = u.w;
                bnd[5] = w.x; bnd[6] = w.y; bnd[7] = w.z; bnd[8] = w.w;
            } else {
                child_bounds(key, c.lbt, P, b, b + c.count[i], l, few, bnd);
            }
            for (uint32_t d = 0; d < 8; ++d) {
                if (bnd[d + 1] > bnd[d]) {
                    if (ch < cap) {
                        c.prefix[ch] = (P << 3) | d;
                        c.level[ch] = (uint32_t)(l + 1);
                        c.begin[ch] = bnd[d];
                        c.count[ch] = bnd[d + 1] - bnd[d];
                        c.child0[ch] = kNone;
                        c.nchild[ch] = 0;
                        c.parent[ch] = i;
                    }
                    ++ch;
                }
            }
        } else if (i < ce) {
            c.child0[i] = kNone;
        }
        carry += tot;
    }
}

// lbt[q] for q in [0, 8^kTableLevel]: the first of the n sorted keys that is
// >= q << 3 (21 - kTableLevel); lbt[8^kTableLevel] = n
__global__ __launch_bounds__(256) void k_lb_table(const uint64_t *__restrict__ key, uint32_t n,
                                                  uint32_t *__restrict__ lbt) {
    constexpr uint32_t kQ = 1u << (3 * kTableLevel);
    const uint32_t q = blockIdx.x * 256u + threadIdx.x;
    if (q > kQ) return;
    lbt[q] = q == kQ ? n
                     : key_lower_bound(key, 0u, n, (uint64_t)q << (3 * (kKeyBits - kTableLevel)));
}

// Levels l0 .. 20 in one workgroup: the deep end of the tree, where a level
// holds few cells (or none) and three launches per level would cost more
// than the work.  Per level: each round of 1024 cells finds its children's
// bounds, a block scan numbers the children in cell order, and the children
// are written, exactly as the three grid kernels would.  Any level size is
// handled (only more slowly), so the split between grid and tail levels
// affects the time, never the tree.  Then publishes the level starts and the
// build's number to the host (pinned memory, tagged before and after).
constexpr int kTailThreads = 1024;

__global__ __launch_bounds__(kTailThreads) void k_build_tail(Cells c,
                                                             const uint64_t *__restrict__ key,
                                                             int l0, uint32_t nleaf, uint32_t cap,
                                                             uint32_t *status,
                                                             volatile uint32_t *hint,
                                                             uint32_t gen) {
    __shared__ uint32_t wtot[kTailThreads / 64];
    const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
    uint32_t first = 0, last = 0;
    if (l0 < kLevels - 1) {
        first = c.ls[l0];
        last = c.ls[l0 + 1];
    }
    for (int l = l0; l < kLevels - 1; ++l) {
        const bool few = last - first < kFewCells;
        uint32_t next = last;  // the next level is built at [last, next)
        for (uint32_t base = first; base < last; base += kTailThreads) {
            const uint32_t i = base + threadIdx.x;
            uint32_t bnd[9];
            uint32_t nch = 0, b = 0;
            uint64_t P = 0;
            if (i < last) {
                const uint32_t cnt = c.count[i];
                if (cnt > nleaf) {
                    b = c.begin[i];
                    P = c.prefix[i];
                    child_bounds(key, c.lbt, P, b, b + cnt, l, few, bnd);
#pragma unroll
                    for (int d = 0; d < 8; ++d) nch += bnd[d + 1] > bnd[d];
                }
                c.nchild[i] = nch;
            }
            const uint32_t inc = wave_incl_scan(nch, lane);
            if (lane == 63) wtot[w] = inc;
            __syncthreads();
            uint32_t off = 0, tot = 0;
            for (uint32_t k = 0; k < (uint32_t)(kTailThreads / 64); ++k) {
                if (k < w) off += wtot[k];
                tot += wtot[k];
            }
            __syncthreads();
            if (i < last) {
                if (nch > 0) {
                    uint32_t ch = next + off + inc - nch;
                    c.child0[i] = ch;
                    for (uint32_t d = 0; d < 8; ++d) {
                        if (bnd[d + 1] > bnd[d]) {
                            if (ch < cap) {
                                c.prefix[ch] = (P << 3) | d;
                                c.level[ch] = (uint32_t)(l + 1);
                                c.begin[ch] = bnd[d];
                                c.count[ch] = bnd[d + 1] - bnd[d];
                                c.child0[ch] = kNone;
                                c.nchild[ch] = 0;
                                c.parent[ch] = i;
                            }
                            ++ch;
                        }
                    }
                } else {
                    c.child0[i] = kNone;
                }
            }
            next += tot;
        }
        if (next > cap) {
            if (threadIdx.x == 0) atomicOr(status, kStOverflow);
            next = cap;
        }
        if (threadIdx.x == 0) c.ls[l + 2] = next;
        __syncthreads();  // the new level's cells are read by the whole block next
        first = last;
        last = next;
    }
    __syncthreads();
    if (threadIdx.x == 0 && hint) {
        hint[0] = gen;
        __threadfence_system();
        for (int k = 0; k < kLevels + 1; ++k) hint[2 + k] = c.ls[k];
        __threadfence_system();
        hint[1] = gen;
    }
}

// Levels 0 .. grid_levels - 1 are split by the grid kernels, the rest by
// k_build_tail.
void launch_build(bh_ctx *ctx, uint32_t n, hipStream_t st, int grid_levels) {
    Cells &c = ctx->cells;
    constexpr uint32_t kQ = 1u << (3 * kTableLevel);
    hipLaunchKernelGGL(k_lb_table, dim3((kQ + 1 + 255) / 256), dim3(256), 0, st,
                       (const uint64_t *)ctx->sort.key[0], n, c.lbt);
    hipLaunchKernelGGL(k_build_init, dim3(1), dim3(64), 0, st, c, n);
    uint32_t cap = (uint32_t)ctx->cap_cells;
    const int L = grid_levels < 0 ? 0 : (grid_levels > kLevels - 1 ? kLevels - 1 : grid_levels);
    for (int l = 0; l < L; ++l) {
        hipLaunchKernelGGL(k_build_count, dim3(kBuildGrid), dim3(kBuildThreads), 0, st, c,
                           (const uint64_t *)ctx->sort.key[0], l, (uint32_t)ctx->p.nleaf,
                           (uint32_t)ctx->nmax);
        hipLaunchKernelGGL(k_build_scan, dim3(1), dim3(kBuildThreads), 0, st, c, l, cap,
                           ctx->status);
        hipLaunchKernelGGL(k_build_write, dim3(kBuildGrid), dim3(kBuildThreads), 0, st, c,
                           (const uint64_t *)ctx->sort.key[0], l, cap, (uint32_t)ctx->nmax);
    }
    hipLaunchKernelGGL(k_build_tail, dim3(1), dim3(kTailThreads), 0, st, c,
                       (const uint64_t *)ctx->sort.key[0], L, (uint32_t)ctx->p.nleaf, cap,
                       ctx->status, (volatile uint32_t *)ctx->hint_dev, ctx->build_gen);
}

// ---- groups -----------------------------------------------------------------
//
// A cell is a group iff (count <= ncrit or it is a leaf) and (it is the root
// or its parent holds more than ncrit).  Groups partition the sorted
// particles; a group cell larger than ncrit (a level-21 leaf of coincident
// keys) is cut into chunks of ncrit.  Group numbers follow key order: flag
// each group's first particle, scan the flags.

__global__ __launch_bounds__(256) void k_group_flags(Cells c, uint32_t ncrit, uint32_t *flag,
                                                     uint32_t *gpar) {
    uint32_t nc = c.ls[kLevels];
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nc; i += gridDim.x * 256) {
        uint32_t cnt = c.count[i];
        bool small = cnt <= ncrit || c.nchild[i] == 0;
        bool top = i == 0 || c.count[c.parent[i]] > ncrit;
        if (small && top) {
            uint32_t b = c.begin[i];
            for (uint32_t s = 0; s < cnt; s += ncrit) {
                flag[b + s] = 1u;
                if (gpar) gpar[b + s] = i == 0 ? kNone : c.parent[i];
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_group_fill(const uint32_t *__restrict__ flag,
                                                    const uint32_t *__restrict__ scan, uint32_t n,
                                                    uint32_t *gbeg, uint32_t *ngroups) {
    uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    if (flag[i]) gbeg[scan[i]] = i;
    if (i == n - 1) {
        uint32_t ng = scan[i] + flag[i];
        *ngroups = ng;
        gbeg[ng] = n;
    }
}

// Paired target sets (bh_params.pair_groups = cap, off by default): groups
// 2k and 2k + 1 that are siblings (group cells with one parent; gpar holds
// it at each group's first particle) and hold at most cap particles together
// become one target set, walked once against the box of their union, by
// clearing the start flag of group 2k + 1.
__global__ __launch_bounds__(256) void k_pair_flags(const uint32_t *__restrict__ gbeg,
                                                    const uint32_t *__restrict__ ngroups,
                                                    const uint32_t *__restrict__ gpar,
                                                    uint32_t cap, uint32_t *flag) {
    const uint32_t ng = *ngroups;
    for (uint32_t j = 2 * (blockIdx.x * 256 + threadIdx.x) + 1; j < ng;
         j += 2 * gridDim.x * 256) {
        const uint32_t a = gbeg[j - 1], b = gbeg[j];
        if (gbeg[j + 1] - a <= cap && gpar[a] == gpar[b] && gpar[a] != kNone) flag[b] = 0u;
    }
}

void launch_groups(bh_ctx *ctx, uint32_t n, hipStream_t st) {
    Groups &g = ctx->groups;
    launch_fill_u32(g.flag, 0u, n, st);
    // paired target sets: each group's parent cell is kept in npp until the walk
    uint32_t *gpar = ctx->pair_groups ? g.npp : nullptr;
    hipLaunchKernelGGL(k_group_flags, dim3(kGrid), dim3(256), 0, st, ctx->cells,
                       (uint32_t)ctx->p.ncrit, g.flag, gpar);
    launch_exclusive_scan(g.flag, g.scan, n, ctx->sort.scan_part, st);
    hipLaunchKernelGGL(k_group_fill, dim3(cdiv(n, 256)), dim3(256), 0, st,
                       (const uint32_t *)g.flag, (const uint32_t *)g.scan, n, g.begin,
                       g.count_dev);
    if (ctx->pair_groups) {
        hipLaunchKernelGGL(k_pair_flags, dim3(kGrid), dim3(256), 0, st,
                           (const uint32_t *)g.begin, (const uint32_t *)g.count_dev,
                           (const uint32_t *)gpar, ctx->pair_groups, g.flag);
        launch_exclusive_scan(g.flag, g.scan, n, ctx->sort.scan_part, st);
        hipLaunchKernelGGL(k_group_fill, dim3(cdiv(n, 256)), dim3(256), 0, st,
                           (const uint32_t *)g.flag, (const uint32_t *)g.scan, n, g.begin,
                           g.count_dev);
    }
}

}  // namespace bh
