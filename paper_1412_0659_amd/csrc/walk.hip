// Group-wise tree walk fused with the force evaluation (Sec. III.A: walk
// and force in one kernel, interaction lists kept on chip and evaluated on
// the fly; Sec. I.A: opening angle theta; Sec. VI.A Eq. (1)-(2); Table II
// "Compute gravity").
//
// One 64-lane wavefront walks the tree for one target group:
//   * a stack of sibling ranges (first << 3 | count - 1); each pass pops up
//     to 64 cells, one per lane.  Children of opened cells are pushed with
//     shallower ranges below deeper ones, so the stack holds at most 64
//     ranges per level (1408).  Its top 256 entries live in an LDS ring; the
//     rest spill to a per-wave area in device memory in blocks of 64 (any
//     ring of at least 128 entries works: a spill happens only when more
//     than ring - 64 entries are resident, a refill only when fewer than 64);
//   * each lane applies the opening test: distance d from the cell's centre
//     of mass to the group's box, accept the cell whole iff
//     d^2 >= (l / theta + delta)^2 (FP32, no contraction);
//   * accepted cells and the particles of opened leaves are compacted
//     (ballot + mbcnt) into two LDS index lists; no source data is read
//     during the traversal;
//   * a full list is evaluated in chunks of 64 sources: each lane loads one
//     source record into LDS (the next chunk's loads are issued before the
//     current chunk is evaluated), then lane = (target, slice) evaluates the
//     chunk, slice s taking entries s, s + r, ...  A group of g targets uses
//     one phase with r = floor(64 / g) slices, or two phases (most targets
//     with ceil(64 / g) slices, the remaining few with many), whichever
//     needs fewer rounds; the slices are summed at the end.
// Groups are taken from eight contiguous ranges (one per XCD, blockIdx % 8)
// through atomic counters, so neighbouring groups share an L2; every wave
// leaves once all ranges are exhausted.
#include "bh_internal.h"
#include "wave.h"

namespace bh {

constexpr int kRing = 256;        // LDS window of the range stack (a.ring <= kRing)
constexpr int kPcCap = 256;       // particle-cell index list
constexpr int kPcFlush = kPcCap - 64;
constexpr int kPpCap = 512;       // particle-particle index list
constexpr int kChunk = 64;        // sources staged per evaluation round
constexpr int kNull = kChunk;     // staging slot of the null source

struct WalkArgs {
    const float4 *xyzm;                  // sorted positions + mass
    const float4 *wA;                    // com, r_open^2
    const uint2 *wN;                     // (first, n | leaf bit)
    const float4 *P0, *P1, *P2;          // particle-cell records
    const uint32_t *gbeg, *ngroups;
    uint32_t *work, *spill;
    float4 *acc, *gbox;
    uint32_t *npp, *npc, *status;
    float eps2;
    uint32_t ring;  // ring entries in use: kRing, or 128 to exercise the spill path
};

__device__ __forceinline__ float rsq(float v) { return __builtin_amdgcn_rsqf(v); }

// One particle-cell term, Eq. (1)-(2) with r^2 -> r^2 + eps^2.
// A = (com x, y, z, M); B = (-3 Qxx, -3 Qyy, -3 Qzz, -3 Qxy);
// C = (-3 Qxz, -3 Qyz, tr Q / 2, -3 tr Q / 2).  With q = -3 Q d:
//   phi += -M/r + (tr/2)/r^3 + (1/2) d.q / r^5
//   a   += d [M/r^3 - (3/2) tr/r^5 - (5/2) d.q / r^7] + q / r^5
__device__ __forceinline__ void pc_term(const float4 &T, const float4 &A, const float4 &B,
                                        const float4 &C, float eps2, float4 &acc) {
    float dx = A.x - T.x, dy = A.y - T.y, dz = A.z - T.z;
    float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
    float ri = rsq(r2);
    float ri2 = ri * ri;
    float mr = A.w * ri;
    float ri3 = ri * ri2;
    float ri5 = ri3 * ri2;
    float qx = fmaf(B.x, dx, fmaf(B.w, dy, C.x * dz));
    float qy = fmaf(B.w, dx, fmaf(B.y, dy, C.y * dz));
    float qz = fmaf(C.x, dx, fmaf(C.y, dy, B.z * dz));
    float dq = fmaf(dx, qx, fmaf(dy, qy, dz * qz));
    float a5 = dq * ri5;
    acc.w = acc.w - mr;
    acc.w = fmaf(C.z, ri3, acc.w);
    acc.w = fmaf(0.5f, a5, acc.w);
    float u = fmaf(-2.5f, a5, mr);
    float s = fmaf(C.w, ri5, u * ri2);
    acc.x = fmaf(s, dx, fmaf(qx, ri5, acc.x));
    acc.y = fmaf(s, dy, fmaf(qy, ri5, acc.y));
    acc.z = fmaf(s, dz, fmaf(qz, ri5, acc.z));
}

// One particle-particle term (a point mass P.w at P.xyz).
template <bool kEps0>
__device__ __forceinline__ void pp_term(const float4 &T, const float4 &P, float eps2,
                                        float4 &acc) {
    float dx = P.x - T.x, dy = P.y - T.y, dz = P.z - T.z;
    float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
    float ri = rsq(r2);
    if (kEps0) ri = r2 > 0.f ? ri : 0.f;
    float mr = P.w * ri;
    float mr3 = mr * (ri * ri);
    acc.w = acc.w - mr;
    acc.x = fmaf(mr3, dx, acc.x);
    acc.y = fmaf(mr3, dy, acc.y);
    acc.z = fmaf(mr3, dz, acc.z);
}

struct WalkLds {
    float4 stage[3][kChunk + 1];  // source records of one chunk + the null source
    uint32_t ring[kRing];
    uint32_t pcidx[kPcCap];
    uint32_t ppidx[kPpCap];
    uint32_t offs[64], firsts[64], starts[64];
};

// Target roles of a lane in one evaluation phase: T targets, r slices;
// lanes >= T * r are idle (they repeat slice 0 and are ignored).
struct Phase {
    uint32_t T, r, slice;
    bool act;
    float4 tgt;
    float4 acc;
};

// Evaluate n (<= 64) staged sources for one phase; entries past n read the
// null source (far away, zero mass) so every round is uniform.
template <bool kIsPc, bool kEps0>
__device__ __forceinline__ void eval_chunk(Phase &ph, uint32_t n, const WalkLds &L, float eps2) {
    const uint32_t r = ph.r;
    const uint32_t full = n / r, rem = n - full * r;
    uint32_t k = ph.slice;
    for (uint32_t j = 0; j < full; ++j, k += r) {
        if (kIsPc) pc_term(ph.tgt, L.stage[0][k], L.stage[1][k], L.stage[2][k], eps2, ph.acc);
        else pp_term<kEps0>(ph.tgt, L.stage[0][k], eps2, ph.acc);
    }
    if (rem) {
        const uint32_t kk = ph.slice < rem ? k : (uint32_t)kNull;
        if (kIsPc) pc_term(ph.tgt, L.stage[0][kk], L.stage[1][kk], L.stage[2][kk], eps2, ph.acc);
        else pp_term<kEps0>(ph.tgt, L.stage[0][kk], eps2, ph.acc);
    }
}

template <bool kEps0>
__device__ void walk_group(const WalkArgs &a, uint32_t g, uint32_t lane, WalkLds &L,
                           uint32_t *spill) {
    const uint32_t gb = a.gbeg[g];
    const uint32_t gn = a.gbeg[g + 1] - gb;  // 1..64 by construction
    if (gn == 0u || gn > 64u) {
        if (lane == 0) atomicOr(a.status, kStOverflow);
        return;
    }

    // ---- group box
    const bool own = lane < gn;
    const float4 me = a.xyzm[gb + (own ? lane : 0u)];
    float gcx, gcy, gcz, ghx, ghy, ghz;
    {
        float mn = wave_min(own ? me.x : INFINITY), mx = wave_max(own ? me.x : -INFINITY);
        gcx = (mn + mx) * 0.5f; ghx = (mx - mn) * 0.5f;
        mn = wave_min(own ? me.y : INFINITY); mx = wave_max(own ? me.y : -INFINITY);
        gcy = (mn + mx) * 0.5f; ghy = (mx - mn) * 0.5f;
        mn = wave_min(own ? me.z : INFINITY); mx = wave_max(own ? me.z : -INFINITY);
        gcz = (mn + mx) * 0.5f; ghz = (mx - mn) * 0.5f;
    }
    if (lane == 0) {
        a.gbox[2 * (size_t)g] = make_float4(gcx, gcy, gcz, 0.f);
        a.gbox[2 * (size_t)g + 1] = make_float4(ghx, ghy, ghz, 0.f);
    }

    // ---- lane roles: one or two phases, whichever needs fewer rounds
    Phase p1, p2;
    {
        const uint32_t rs = 64u / gn;
        const uint32_t cost1 = (64u + rs - 1u) / rs;
        const uint32_t ra = (64u + gn - 1u) / gn, Ta = 64u / ra, Tb = gn - Ta;
        const uint32_t rb = Tb ? 64u / Tb : 0u;
        const uint32_t cost2 = (64u + ra - 1u) / ra + (Tb ? (64u + rb - 1u) / rb : 0u);
        if (Tb && cost2 < cost1) {
            p1.T = Ta; p1.r = ra; p2.T = Tb; p2.r = rb;
        } else {
            p1.T = gn; p1.r = rs; p2.T = 0; p2.r = 0;
        }
        p1.act = lane < p1.T * p1.r;
        p1.slice = p1.act ? lane / p1.T : 0u;
        p1.tgt = a.xyzm[gb + (p1.act ? lane % p1.T : 0u)];
        p1.acc = make_float4(0.f, 0.f, 0.f, 0.f);
        p2.act = p2.T && lane < p2.T * p2.r;
        p2.slice = p2.act ? lane / p2.T : 0u;
        p2.tgt = a.xyzm[gb + (p2.act ? p1.T + lane % p2.T : 0u)];
        p2.acc = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const bool two = p2.T != 0u;

    uint32_t cnt_pc = 0, cnt_pp = 0, pc_n = 0, pp_n = 0;
    uint32_t sp = 1, lo = 0;  // stack positions [lo, sp) are in the LDS ring
    const uint32_t rmask = a.ring - 1u;
    if (lane == 0) {
        L.ring[0] = 0u;  // the root: first cell 0, one cell
        L.stage[0][kNull] = make_float4(1e30f, 1e30f, 1e30f, 0.f);
        L.stage[1][kNull] = make_float4(0.f, 0.f, 0.f, 0.f);
        L.stage[2][kNull] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();

    // evaluate the particle-cell list: stage 64 records at a time, loading
    // the next chunk while the current one is evaluated
    auto flush_pc = [&](uint32_t n) {
        if (n == 0) return;
        float4 r0, r1, r2;
        {
            const uint32_t c = L.pcidx[lane < n ? lane : 0u];
            r0 = a.P0[c]; r1 = a.P1[c]; r2 = a.P2[c];
        }
        for (uint32_t base = 0; base < n; base += kChunk) {
            const uint32_t m = n - base < (uint32_t)kChunk ? n - base : (uint32_t)kChunk;
            __syncthreads();
            L.stage[0][lane] = r0; L.stage[1][lane] = r1; L.stage[2][lane] = r2;
            __syncthreads();
            if (base + kChunk < n) {
                const uint32_t q = base + kChunk + lane;
                const uint32_t c = L.pcidx[q < n ? q : base + kChunk];
                r0 = a.P0[c]; r1 = a.P1[c]; r2 = a.P2[c];
            }
            eval_chunk<true, kEps0>(p1, m, L, a.eps2);
            if (two) eval_chunk<true, kEps0>(p2, m, L, a.eps2);
        }
        __syncthreads();
    };
    auto flush_pp = [&](uint32_t n) {
        if (n == 0) return;
        float4 r0 = a.xyzm[L.ppidx[lane < n ? lane : 0u]];
        for (uint32_t base = 0; base < n; base += kChunk) {
            const uint32_t m = n - base < (uint32_t)kChunk ? n - base : (uint32_t)kChunk;
            __syncthreads();
            L.stage[0][lane] = r0;
            __syncthreads();
            if (base + kChunk < n) {
                const uint32_t q = base + kChunk + lane;
                r0 = a.xyzm[L.ppidx[q < n ? q : base + kChunk]];
            }
            eval_chunk<false, kEps0>(p1, m, L, a.eps2);
            if (two) eval_chunk<false, kEps0>(p2, m, L, a.eps2);
        }
        __syncthreads();
    };

    while (sp > 0) {
        // ---- refill the ring from the spill area when the top range is not resident
        const uint32_t avail = sp < 64u ? sp : 64u;
        if (sp - avail < lo) {
            lo -= 64u;
            L.ring[(lo + lane) & rmask] = spill[lo + lane];
            __syncthreads();
        }
        // ---- pop up to 64 cells from the top ranges
        uint32_t e = 0, ne = 0;
        if (lane < avail) {
            e = L.ring[(sp - 1 - lane) & rmask];
            ne = (e & 7u) + 1u;
        }
        const uint32_t incl = wave_incl_scan(ne, lane);
        const uint32_t excl = incl - ne;
        const uint32_t nfull = (uint32_t)__popcll(ballot(lane < avail && incl <= 64u));
        const uint32_t tall = shfl(incl, (int)avail - 1);
        const uint32_t total = tall < 64u ? tall : 64u;
        L.starts[lane] = 0u;
        __syncthreads();
        if (lane < avail && excl < 64u) L.starts[excl] = 1u;
        __syncthreads();
        const uint64_t smask = ballot(L.starts[lane] != 0u);
        const bool have = lane < total;
        const uint32_t j = (uint32_t)__popcll(smask & mask_le(lane)) - 1u;
        const uint32_t ej = shfl(e, (int)j), xj = shfl(excl, (int)j);
        const uint32_t cell = (ej >> 3) + (lane - xj);
        const uint32_t sp_new = sp - nfull;
        if (nfull < avail && lane == nfull && excl < 64u) {
            const uint32_t taken = 64u - excl;  // the rest of this range stays on top
            L.ring[(sp_new - 1) & rmask] = (((e >> 3) + taken) << 3) | (ne - taken - 1u);
        }

        // ---- opening test
        float4 A = make_float4(0.f, 0.f, 0.f, 0.f);
        uint2 N = make_uint2(0u, 0u);
        if (have) {
            A = a.wA[cell];
            N = a.wN[cell];
        }
        const float dxm = fmaxf(fabsf(A.x - gcx) - ghx, 0.f);
        const float dym = fmaxf(fabsf(A.y - gcy) - ghy, 0.f);
        const float dzm = fmaxf(fabsf(A.z - gcz) - ghz, 0.f);
        float d2 = dxm * dxm + dym * dym;
        d2 = d2 + dzm * dzm;
        const bool accept = have && d2 >= A.w;
        const bool isleaf = (N.y & kLeafBit) != 0u;
        const bool openleaf = have && !accept && isleaf;
        const bool openint = have && !accept && !isleaf;

        // ---- accepted cells -> particle-cell index list
        const uint64_t am = ballot(accept);
        if (accept) L.pcidx[pc_n + count_below(am)] = cell;
        const uint32_t nacc = (uint32_t)__popcll(am);
        pc_n += nacc;
        cnt_pc += nacc;

        // ---- opened internal cells -> their children ranges, shallowest lowest
        const uint64_t om = ballot(openint);
        const uint32_t npush = (uint32_t)__popcll(om);
        if (sp_new + npush > (uint32_t)kStackMax) {  // cannot happen: 64 ranges per level
            if (lane == 0) atomicOr(a.status, kStOverflow);
            break;
        }
        if (sp_new + npush > lo + a.ring) {
            // spill the 64 lowest resident entries (all below sp_new)
            __syncthreads();
            spill[lo + lane] = L.ring[(lo + lane) & rmask];
            lo += 64u;
            __syncthreads();
        }
        if (openint) {
            const uint32_t above = lane == 63u ? 0u : (uint32_t)__popcll(om >> (lane + 1u));
            L.ring[(sp_new + above) & rmask] = (N.x << 3) | (N.y - 1u);
        }
        sp = sp_new + npush;

        // ---- particles of opened leaves -> particle-particle index list
        const uint32_t lc = openleaf ? (N.y & ~kLeafBit) : 0u;
        const uint32_t lincl = wave_incl_scan(lc, lane);
        const uint32_t P = shfl(lincl, 63);
        if (P > 0u) {
            L.offs[lane] = lincl - lc;
            L.firsts[lane] = N.x;
            __syncthreads();
            cnt_pp += P;
            for (uint32_t base = 0; base < P;) {
                if (pp_n == (uint32_t)kPpCap) {
                    flush_pp(pp_n);
                    pp_n = 0;
                }
                const uint32_t room = (uint32_t)kPpCap - pp_n;
                const uint32_t take = room < P - base ? room : P - base;
                for (uint32_t q = lane; q < take; q += 64u) {
                    const uint32_t f = base + q;
                    uint32_t s = 0;
#pragma unroll
                    for (uint32_t step = 32; step > 0; step >>= 1)
                        if (L.offs[s + step] <= f) s += step;
                    L.ppidx[pp_n + q] = L.firsts[s] + (f - L.offs[s]);
                }
                pp_n += take;
                base += take;
                __syncthreads();
            }
        }
        __syncthreads();
        if (pc_n > (uint32_t)kPcFlush) {
            flush_pc(pc_n);
            pc_n = 0;
        }
    }
    __syncthreads();
    flush_pc(pc_n);
    flush_pp(pp_n);

    // ---- sum the slices of each target (staging area reused)
    float4 res = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    L.stage[0][lane] = p1.acc;
    __syncthreads();
    if (lane < p1.T)
        for (uint32_t k = 0; k < p1.r; ++k) {
            const float4 o = L.stage[0][lane + k * p1.T];
            res.x += o.x; res.y += o.y; res.z += o.z; res.w += o.w;
        }
    if (two) {
        __syncthreads();
        L.stage[0][lane] = p2.acc;
        __syncthreads();
        if (lane >= p1.T && lane < gn)
            for (uint32_t k = 0; k < p2.r; ++k) {
                const float4 o = L.stage[0][lane - p1.T + k * p2.T];
                res.x += o.x; res.y += o.y; res.z += o.z; res.w += o.w;
            }
    }
    if (own) {
        // the self pair was evaluated with r^2 = eps^2; take its potential out
        if (!kEps0) res.w += me.w * rsq(a.eps2);
        a.acc[gb + lane] = res;
    }
    if (lane == 0) {
        a.npp[g] = cnt_pp;
        a.npc[g] = cnt_pc;
    }
    __syncthreads();
}

template <bool kEps0>
__global__ __launch_bounds__(64) void k_walk(WalkArgs a) {
    __shared__ WalkLds L;
    const uint32_t lane = threadIdx.x;
    const uint32_t ng = *a.ngroups;
    uint32_t *spill = a.spill + (size_t)blockIdx.x * kStackMax;
    for (uint32_t k = 0; k < 8; ++k) {
        const uint32_t part = (blockIdx.x + k) & 7u;
        const uint32_t r0 = (uint32_t)(((uint64_t)ng * part) >> 3);
        const uint32_t r1 = (uint32_t)(((uint64_t)ng * (part + 1)) >> 3);
        for (;;) {
            uint32_t t = 0;
            if (lane == 0) t = atomicAdd(&a.work[part], 1u);
            t = uniform(t);
            if (t >= r1 - r0) break;
            walk_group<kEps0>(a, r0 + t, lane, L, spill);
        }
    }
}

__global__ void k_reset_work(uint32_t *work) {
    if (threadIdx.x < 8) work[threadIdx.x] = 0u;
}

int walk_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_walk<false>, 64, 0) != hipSuccess ||
        nb < 1)
        nb = 4;
    return nb;
}

void launch_walk(bh_ctx *c, float eps, hipStream_t st) {
    WalkArgs a;
    a.xyzm = c->xyzm;
    a.wA = c->cells.wA; a.wN = c->cells.wN;
    a.P0 = c->cells.P0; a.P1 = c->cells.P1; a.P2 = c->cells.P2;
    a.gbeg = c->groups.begin; a.ngroups = c->groups.count_dev;
    a.work = c->work; a.spill = c->spill;
    a.acc = c->acc; a.gbox = c->groups.box;
    a.npp = c->groups.npp; a.npc = c->groups.npc; a.status = c->status;
    a.eps2 = eps * eps;
    a.ring = c->walk_small_stack ? 128u : (uint32_t)kRing;
    hipLaunchKernelGGL(k_reset_work, dim3(1), dim3(64), 0, st, c->work);
    (void)hipEventRecord(c->ev[4], st);
    c->ev_rec[4] = true;
    if (eps == 0.f)
        hipLaunchKernelGGL(k_walk<true>, dim3(c->walk_grid), dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL(k_walk<false>, dim3(c->walk_grid), dim3(64), 0, st, a);
    (void)hipEventRecord(c->ev[5], st);
    c->ev_rec[5] = true;
}

}  // namespace bh
