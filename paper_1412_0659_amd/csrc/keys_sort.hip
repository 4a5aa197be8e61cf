// Bounding box, Morton keys, LSD radix sort of (key, index) and the gather of
// the particle state into key order (Sec. III.B.1: keys computed from the
// bounding box; Table II "Sorting SFC").
//
// Keys: 21 bits per axis, x the high bit of each 3-bit digit,
//   q = min(trunc(fl32(fl32(x - lo) * scale)), 2^21 - 1),
//   scale = fl32(2^21 / side) with the division in FP64,
// built with contraction off so the FP32 quantisation is exactly the one
// written above.
#include "bh_internal.h"
#include "wave.h"

namespace bh {

constexpr int kBoxThreads = 256;
constexpr int kBoxBlocks = 1024;

__global__ __launch_bounds__(kBoxThreads) void k_bbox_partial(const float *__restrict__ x,
                                                              const float *__restrict__ y,
                                                              const float *__restrict__ z,
                                                              uint32_t n, float *part,
                                                              uint32_t *status) {
    __shared__ float lds[4][6];
    float lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY;
    float hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY;
    bool bad = false;
    for (uint32_t i = blockIdx.x * kBoxThreads + threadIdx.x; i < n;
         i += gridDim.x * kBoxThreads) {
        float a = x[i], b = y[i], c = z[i];
        bad |= !(isfinite(a) && isfinite(b) && isfinite(c));
        lo0 = fminf(lo0, a); hi0 = fmaxf(hi0, a);
        lo1 = fminf(lo1, b); hi1 = fmaxf(hi1, b);
        lo2 = fminf(lo2, c); hi2 = fmaxf(hi2, c);
    }
    if (bad) atomicOr(status, kStNonFinite);
    lo0 = wave_min(lo0); lo1 = wave_min(lo1); lo2 = wave_min(lo2);
    hi0 = wave_max(hi0); hi1 = wave_max(hi1); hi2 = wave_max(hi2);
    uint32_t w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        lds[w][0] = lo0; lds[w][1] = lo1; lds[w][2] = lo2;
        lds[w][3] = hi0; lds[w][4] = hi1; lds[w][5] = hi2;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        float v = lds[0][threadIdx.x];
        for (int k = 1; k < 4; ++k)
            v = threadIdx.x < 3 ? fminf(v, lds[k][threadIdx.x]) : fmaxf(v, lds[k][threadIdx.x]);
        part[blockIdx.x * 6 + threadIdx.x] = v;
    }
}

// Reduce the block partials.  fixed == 0: the cube of side = largest
// extent at the minimum corner.  fixed == 1: the caller's box (flo, fside),
// and kStOutside is latched when on some axis a particle lies below flo or
// has fl32(x - flo) > fside (the difference the keys quantise).
__global__ __launch_bounds__(64) void k_bbox_final(const float *__restrict__ part, uint32_t nb,
                                                   float *box, int fixed, float flo0, float flo1,
                                                   float flo2, float fside, uint32_t *status) {
    float lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY;
    float hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY;
    for (uint32_t b = threadIdx.x; b < nb; b += 64) {
        lo0 = fminf(lo0, part[6 * b + 0]); lo1 = fminf(lo1, part[6 * b + 1]);
        lo2 = fminf(lo2, part[6 * b + 2]); hi0 = fmaxf(hi0, part[6 * b + 3]);
        hi1 = fmaxf(hi1, part[6 * b + 4]); hi2 = fmaxf(hi2, part[6 * b + 5]);
    }
    lo0 = wave_min(lo0); lo1 = wave_min(lo1); lo2 = wave_min(lo2);
    hi0 = wave_max(hi0); hi1 = wave_max(hi1); hi2 = wave_max(hi2);
    if (threadIdx.x == 0) {
        if (fixed) {
            bool out = lo0 < flo0 || lo1 < flo1 || lo2 < flo2 || hi0 - flo0 > fside ||
                       hi1 - flo1 > fside || hi2 - flo2 > fside;
            if (out) atomicOr(status, kStOutside);
            box[0] = flo0; box[1] = flo1; box[2] = flo2;
            box[3] = fside;
            box[4] = (float)(2097152.0 / (double)fside);
            return;
        }
        float side = 0.f, e;
        e = hi0 - lo0; if (e > side) side = e;
        e = hi1 - lo1; if (e > side) side = e;
        e = hi2 - lo2; if (e > side) side = e;
        if (side == 0.f) side = 1.f;
        box[0] = lo0; box[1] = lo1; box[2] = lo2;
        box[3] = side;
        box[4] = (float)(2097152.0 / (double)side);
    }
}

void launch_bbox(bh_ctx *c, const State &s, uint32_t n, hipStream_t st) {
    uint32_t nb = cdiv(n, kBoxThreads * 8);
    if (nb > kBoxBlocks) nb = kBoxBlocks;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(kBoxThreads), 0, st, s.x, s.y, s.z, n,
                       c->box_part, c->status);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, st, (const float *)c->box_part, nb,
                       c->box, c->fixed_box ? 1 : 0, c->box_lo[0], c->box_lo[1], c->box_lo[2],
                       c->box_side, c->status);
}

// 21 bits -> every third bit of a 63-bit word
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint32_t quantise(float v, float lo, float scale) {
    float t = v - lo;
    float u = t * scale;
    if (!(u > 0.f)) return 0u;  // below a caller-given box: the first cell
    uint32_t q = (uint32_t)u;
    return q > 0x1fffffu ? 0x1fffffu : q;
}

// 63-bit keys: the quantised coordinates interleaved (Morton), or their
// Peano-Hilbert transposed index interleaved the same way
template <bool kPH>
__global__ __launch_bounds__(256) void k_keys(const float *__restrict__ x,
                                              const float *__restrict__ y,
                                              const float *__restrict__ z, uint32_t n,
                                              const float *__restrict__ box,
                                              uint64_t *__restrict__ key,
                                              uint32_t *__restrict__ idx) {
    uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float lo0 = box[0], lo1 = box[1], lo2 = box[2], scale = box[4];
    uint32_t X[3] = {quantise(x[i], lo0, scale), quantise(y[i], lo1, scale),
                     quantise(z[i], lo2, scale)};
    if (kPH) ph_encode(X, kKeyBits);
    key[i] = (spread3(X[0]) << 2) | (spread3(X[1]) << 1) | spread3(X[2]);
    idx[i] = i;
}

void launch_keys(bh_ctx *c, const State &s, uint32_t n, hipStream_t st) {
    if (c->p.curve == 1)
        hipLaunchKernelGGL(k_keys<true>, dim3(cdiv(n, 256)), dim3(256), 0, st, s.x, s.y, s.z, n,
                           (const float *)c->box, c->sort.key[0], c->sort.idx[0]);
    else
        hipLaunchKernelGGL(k_keys<false>, dim3(cdiv(n, 256)), dim3(256), 0, st, s.x, s.y, s.z,
                           n, (const float *)c->box, c->sort.key[0], c->sort.idx[0]);
}

// ---- LSD radix sort, 8 bits per pass -------------------------------------
//
// A tile is 8192 keys handled by 1024 threads (16 waves x 8 rounds x 64
// lanes); wave w owns the contiguous keys [512 w, 512 w + 512) of the tile,
// in rounds of 64 consecutive keys, so (wave, round, lane) order is input
// order and the ranking below is stable.  Pass structure: per-tile digit
// counts -> one exclusive scan over (digit, tile) -> stable scatter.  A tile
// of 8192 keys gives digit runs of 32 keys on average, so the scatter writes
// mostly whole cache lines (the tile and its reorder buffer, 112 KB of LDS,
// fit one workgroup of gfx950).

constexpr int kSortThreads = 1024;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortThreads * kSortRounds;

int64_t sort_counts_len(int64_t nmax) { return 256 * ((nmax + kSortTile - 1) / kSortTile) + 1; }

__global__ __launch_bounds__(kSortThreads) void k_sort_count(const uint64_t *__restrict__ key,
                                                             uint32_t n, uint32_t shift,
                                                             uint32_t ntiles,
                                                             uint32_t *__restrict__ counts) {
    __shared__ uint32_t hist[256];
    if (threadIdx.x < 256) hist[threadIdx.x] = 0;
    __syncthreads();
    uint32_t w = threadIdx.x >> 6, lane = lane_id();
    uint64_t base = (uint64_t)blockIdx.x * kSortTile + w * 512 + lane;
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        uint64_t i = base + r * 64;
        if (i < n) atomicAdd(&hist[(uint32_t)(key[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 256) counts[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = hist[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(
    const uint64_t *__restrict__ key_in, const uint32_t *__restrict__ idx_in, uint32_t n,
    uint32_t shift, uint32_t ntiles, const uint32_t *__restrict__ offsets,
    uint64_t *__restrict__ key_out, uint32_t *__restrict__ idx_out) {
    __shared__ uint32_t cnt[kSortWaves][256];
    uint32_t w = threadIdx.x >> 6, lane = lane_id();
    for (int k = 0; k < kSortWaves * 256; k += kSortThreads)
        (&cnt[0][0])[k + threadIdx.x] = 0;
    __syncthreads();
    uint64_t base = (uint64_t)blockIdx.x * kSortTile + w * 512 + lane;
    uint64_t kk[kSortRounds];
    uint32_t vv[kSortRounds], dd[kSortRounds], rk[kSortRounds];
    uint64_t lt = mask_lt(lane);
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        uint64_t i = base + r * 64;
        bool valid = i < n;
        uint64_t k = valid ? key_in[i] : 0ull;
        uint32_t v = valid ? idx_in[i] : 0u;
        uint32_t d = (uint32_t)(k >> shift) & 255u;
        // lanes of this round holding the same digit
        uint64_t peers = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t m = ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t before = __popcll(peers & lt);
        uint32_t run = valid ? cnt[w][d] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (valid && before == 0) cnt[w][d] = run + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        kk[r] = k;
        vv[r] = v;
        dd[r] = valid ? d : 256u;
        rk[r] = run + before;
    }
    __syncthreads();
    // the tile reordered by digit in LDS: digit d starts at lo[d] (an
    // exclusive scan of the tile's digit counts), wave w's keys of digit d
    // after those of the waves before it; then written out in LDS order,
    // so that consecutive threads store consecutive keys of one digit run
    // (whole cache lines) instead of one key per run
    __shared__ uint64_t skey[kSortTile];
    __shared__ uint32_t sidx[kSortTile];
    __shared__ uint32_t wsum[4];
    __shared__ int32_t delta[256];
    uint32_t tot = 0, lo = 0;
    if (threadIdx.x < 256) {  // waves 0..3: one digit per thread
        const uint32_t d = threadIdx.x;
#pragma unroll
        for (int k = 0; k < kSortWaves; ++k) tot += cnt[k][d];
        const uint32_t inc = wave_incl_scan(tot, lane);
        if (lane == 63) wsum[w] = inc;
        lo = inc - tot;
    }
    __syncthreads();
    if (threadIdx.x < 256) {
        const uint32_t d = threadIdx.x;
        for (uint32_t k = 0; k < w; ++k) lo += wsum[k];
        const uint32_t g = offsets[(uint64_t)d * ntiles + blockIdx.x];
        delta[d] = (int32_t)(g - lo);
        uint32_t run = lo;
#pragma unroll
        for (int k = 0; k < kSortWaves; ++k) {
            const uint32_t c = cnt[k][d];
            cnt[k][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        if (dd[r] < 256u) {
            const uint32_t lp = cnt[w][dd[r]] + rk[r];
            skey[lp] = kk[r];
            sidx[lp] = vv[r];
        }
    }
    __syncthreads();
    const uint64_t t0 = (uint64_t)blockIdx.x * kSortTile;
    const uint32_t valid = n - t0 < (uint64_t)kSortTile ? (uint32_t)(n - t0) : (uint32_t)kSortTile;
    for (uint32_t t = threadIdx.x; t < valid; t += kSortThreads) {
        const uint64_t k = skey[t];
        const uint32_t pos = (uint32_t)(delta[(uint32_t)(k >> shift) & 255u] + (int32_t)t);
        key_out[pos] = k;
        idx_out[pos] = sidx[t];
    }
}

void launch_radix_sort(bh_ctx *c, uint32_t n, hipStream_t st) {
    uint32_t ntiles = cdiv(n, kSortTile);
    uint32_t len = 256u * ntiles;
    int src = 0;
    for (uint32_t pass = 0; pass < 8; ++pass) {
        uint32_t shift = 8 * pass;
        hipLaunchKernelGGL(k_sort_count, dim3(ntiles), dim3(kSortThreads), 0, st,
                           (const uint64_t *)c->sort.key[src], n, shift, ntiles, c->sort.counts);
        launch_exclusive_scan(c->sort.counts, c->sort.counts, len, c->sort.scan_part, st);
        hipLaunchKernelGGL(k_sort_scatter, dim3(ntiles), dim3(kSortThreads), 0, st,
                           (const uint64_t *)c->sort.key[src], (const uint32_t *)c->sort.idx[src],
                           n, shift, ntiles, (const uint32_t *)c->sort.counts,
                           c->sort.key[src ^ 1], c->sort.idx[src ^ 1]);
        src ^= 1;
    }
    // 8 passes: the result is back in buffer 0
}

// ---- gather the state into sorted order ------------------------------------

__global__ __launch_bounds__(256) void k_gather(const uint32_t *__restrict__ idx, uint32_t n,
                                                State a, State b, float4 *__restrict__ xyzm) {
    uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    uint32_t s = idx[i];
    float px = a.x[s], py = a.y[s], pz = a.z[s], pm = a.m[s];
    b.x[i] = px;
    b.y[i] = py;
    b.z[i] = pz;
    b.m[i] = pm;
    xyzm[i] = make_float4(px, py, pz, pm);
    b.vx[i] = a.vx[s];
    b.vy[i] = a.vy[s];
    b.vz[i] = a.vz[s];
    b.cid[i] = a.cid[s];
    if (a.x64) {
        b.x64[i] = a.x64[s];
        b.y64[i] = a.y64[s];
        b.z64[i] = a.z64[s];
    }
}

void launch_gather(bh_ctx *c, uint32_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_gather, dim3(cdiv(n, 256)), dim3(256), 0, st,
                       (const uint32_t *)c->sort.idx[0], n, c->st[c->cur], c->st[c->cur ^ 1],
                       c->xyzm);
    c->cur ^= 1;
}

}  // namespace bh
