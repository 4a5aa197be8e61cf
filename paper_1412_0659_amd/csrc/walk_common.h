// The group-wise tree traversal shared by the force walk and its adjoint
// (Sec. III.A: one walk per group of targets; Sec. I.A: a cell is used whole
// when it passes the opening test with angle theta, otherwise it is opened).
//
// One 64-lane wavefront walks the tree for one target group:
//   * a stack of sibling ranges (first << 3 | count - 1); each pass pops up
//     to 128 cells, two per lane, from the top 64 ranges.  Children of
//     opened cells are pushed with shallower ranges below deeper ones, so
//     the stack holds at most 128 ranges per level (kStackMax).  Its top
//     entries live in an LDS ring of kRing entries, of which at most `ring`
//     (256, or 192 to exercise the spill path) are resident; the rest spill
//     to a per-wave area in device memory in blocks of 64 (a spill happens
//     only when a push would exceed `ring` resident entries, a refill only
//     when fewer than 64 are resident);
//   * each lane applies the opening test: distance d from the cell's centre
//     of mass to the group's box, accept the cell whole iff
//     d^2 >= (l / theta + delta)^2 (FP32, no contraction);
//   * accepted cells and the particles of opened leaves are compacted
//     (ballot + mbcnt) into two LDS index lists; no source data is read
//     during the traversal.  The caller's flush functions evaluate a list
//     when it fills, and once more at the end.
// Groups are taken from eight contiguous ranges (one per XCD, blockIdx % 8)
// through atomic counters, so neighbouring groups share an L2; every wave
// leaves once all ranges are exhausted.
#pragma once

#include "bh_internal.h"
#include "wave.h"

namespace bh {

constexpr int kRing = 256;   // LDS window of the range stack (TreeView::ring <= kRing)
constexpr int kPcCap = 752;  // particle-cell index list
constexpr int kPcFlush = kPcCap - 128;  // a pass appends at most 128 cells
constexpr int kPpCap = 512;  // particle-particle index list
constexpr int kChunk = 64;   // sources staged per evaluation round
constexpr int kNull = kChunk;  // staging slot of the null source

struct TravLds {
    uint32_t ring[kRing];
    uint32_t pcidx[kPcCap];
    uint32_t ppidx[kPpCap];
    uint32_t firsts[128];
    union {                   // a pass uses starts while popping, offs afterwards
        uint32_t offs[128];   // first list position of each opened leaf's particles
        uint8_t starts[128];  // 1 where a popped range begins
    };
};

struct TreeView {
    const float4 *wA;   // com, r_open^2
    const uint2 *wN;    // (first, n | leaf bit)
    uint32_t ring;      // resident stack entries allowed: kRing, or 192 to exercise the spill path
    uint32_t *status;
};

struct GroupBox {
    float cx, cy, cz, hx, hy, hz;
};

// Tight FP32 box of the gn targets (lane < gn holds one): centre (min+max)/2,
// half size (max-min)/2.
__device__ __forceinline__ GroupBox group_box(const float4 &me, bool own) {
    GroupBox b;
    float mn = wave_min(own ? me.x : INFINITY), mx = wave_max(own ? me.x : -INFINITY);
    b.cx = (mn + mx) * 0.5f; b.hx = (mx - mn) * 0.5f;
    mn = wave_min(own ? me.y : INFINITY); mx = wave_max(own ? me.y : -INFINITY);
    b.cy = (mn + mx) * 0.5f; b.hy = (mx - mn) * 0.5f;
    mn = wave_min(own ? me.z : INFINITY); mx = wave_max(own ? me.z : -INFINITY);
    b.cz = (mn + mx) * 0.5f; b.hz = (mx - mn) * 0.5f;
    return b;
}

// Split the group's gn targets over the 64 lanes: one phase with
// r = floor(64 / gn) slices, or two phases (Ta targets with ceil(64 / gn)
// slices, the remaining Tb with floor(64 / Tb)) when that needs fewer rounds.
__device__ __forceinline__ void plan_phases(uint32_t gn, uint32_t &T1, uint32_t &r1,
                                            uint32_t &T2, uint32_t &r2) {
    const uint32_t rs = 64u / gn;
    const uint32_t cost1 = (64u + rs - 1u) / rs;
    const uint32_t ra = (64u + gn - 1u) / gn, Ta = 64u / ra, Tb = gn - Ta;
    const uint32_t rb = Tb ? 64u / Tb : 0u;
    const uint32_t cost2 = (64u + ra - 1u) / ra + (Tb ? (64u + rb - 1u) / rb : 0u);
    if (Tb && cost2 < cost1) {
        T1 = Ta; r1 = ra; T2 = Tb; r2 = rb;
    } else {
        T1 = gn; r1 = rs; T2 = 0; r2 = 0;
    }
}

// Squared distance from a cell's centre of mass to the group's box (FP32,
// no contraction): the left side of the opening test.
__device__ __forceinline__ float box_d2(const float4 &A, const GroupBox &b) {
    const float dxm = fmaxf(fabsf(A.x - b.cx) - b.hx, 0.f);
    const float dym = fmaxf(fabsf(A.y - b.cy) - b.hy, 0.f);
    const float dzm = fmaxf(fabsf(A.z - b.cz) - b.hz, 0.f);
    float d2 = dxm * dxm + dym * dym;
    d2 = d2 + dzm * dzm;
    return d2;
}

// Walk the tree for one group.  flush_pc(n) / flush_pp(n) evaluate the first
// n entries of L.pcidx / L.ppidx (called with n > 0, all lanes, after a
// barrier); both lists are empty when traverse returns.  Counts: accepted
// cells and particles of opened leaves.  kLeafCells: L.ppidx lists the
// opened leaf cells themselves instead of their particles (and the second
// count is of those leaves).
//
// A pass pops up to 128 cells from the top 64 ranges: lane l takes cells l
// (slot a) and 64 + l (slot b) of their concatenation, so the pop, the scan
// and the barriers are shared by two opening tests and two cell loads are in
// flight per lane.  Pop order is slot a's cells, then slot b's; every list
// and the pushed children keep that order.
template <bool kLeafCells = false, class FlushPc, class FlushPp>
__device__ __forceinline__ void traverse(const TreeView &tv, const GroupBox &b, uint32_t lane,
                                         TravLds &L, uint32_t *spill, uint32_t &cnt_pc,
                                         uint32_t &cnt_pp, FlushPc &&flush_pc,
                                         FlushPp &&flush_pp) {
    constexpr uint32_t rmask = (uint32_t)kRing - 1u;
    uint32_t pc_n = 0, pp_n = 0;
    uint32_t sp = 1, lo = 0;  // stack positions [lo, sp) are in the LDS ring
    cnt_pc = 0;
    cnt_pp = 0;
    if (lane == 0) L.ring[0] = 0u;  // the root: first cell 0, one cell
    __syncthreads();

    while (sp > 0) {
        // ---- refill the ring from the spill area when the top range is not resident
        const uint32_t avail = sp < 64u ? sp : 64u;
        if (sp - avail < lo) {
            lo -= 64u;
            L.ring[(lo + lane) & rmask] = spill[lo + lane];
            __syncthreads();
        }
        // ---- pop up to 128 cells from the top ranges (range lane = stack top - lane)
        uint32_t e = 0, ne = 0;
        if (lane < avail) {
            e = L.ring[(sp - 1 - lane) & rmask];
            ne = (e & 7u) + 1u;
        }
        const uint32_t incl = wave_incl_scan(ne, lane);
        const uint32_t excl = incl - ne;
        const uint32_t nfull = (uint32_t)__popcll(ballot(lane < avail && incl <= 128u));
        const uint32_t tall = read_lane(incl, avail - 1u);
        const uint32_t total = tall < 128u ? tall : 128u;
        L.starts[lane] = 0u;
        L.starts[64u + lane] = 0u;
        __syncthreads();
        if (lane < avail && excl < 128u) L.starts[excl] = 1u;
        __syncthreads();
        const uint64_t sa = ballot(L.starts[lane] != 0u);
        const uint64_t sb = ballot(L.starts[64u + lane] != 0u);
        // range of each slot's cell (cell 0 starts range 0: both indices are in 0..63)
        const uint32_t ja = (uint32_t)__popcll(sa & mask_le(lane)) - 1u;
        const uint32_t jb = (uint32_t)__popcll(sa) + (uint32_t)__popcll(sb & mask_le(lane)) - 1u;
        const uint32_t cell_a = (shfl(e, (int)ja) >> 3) + (lane - shfl(excl, (int)ja));
        const uint32_t cell_b = (shfl(e, (int)jb) >> 3) + (64u + lane - shfl(excl, (int)jb));
        const bool have_a = lane < total, have_b = 64u + lane < total;
        const uint32_t sp_new = sp - nfull;
        if (nfull < avail && lane == nfull && excl < 128u) {
            const uint32_t taken = 128u - excl;  // the rest of this range stays on top
            L.ring[(sp_new - 1) & rmask] = (((e >> 3) + taken) << 3) | (ne - taken - 1u);
        }

        // ---- opening test
        float4 Aa = make_float4(0.f, 0.f, 0.f, 0.f), Ab = Aa;
        uint2 Na = make_uint2(0u, 0u), Nb = Na;
        if (have_a) {
            Aa = tv.wA[cell_a];
            Na = tv.wN[cell_a];
        }
        if (have_b) {
            Ab = tv.wA[cell_b];
            Nb = tv.wN[cell_b];
        }
        const bool acc_a = have_a && box_d2(Aa, b) >= Aa.w;
        const bool acc_b = have_b && box_d2(Ab, b) >= Ab.w;
        const bool leaf_a = have_a && !acc_a && (Na.y & kLeafBit) != 0u;
        const bool leaf_b = have_b && !acc_b && (Nb.y & kLeafBit) != 0u;
        const bool open_a = have_a && !acc_a && (Na.y & kLeafBit) == 0u;
        const bool open_b = have_b && !acc_b && (Nb.y & kLeafBit) == 0u;

        // ---- accepted cells -> particle-cell index list
        const uint64_t ama = ballot(acc_a), amb = ballot(acc_b);
        const uint32_t na = (uint32_t)__popcll(ama);
        if (acc_a) L.pcidx[pc_n + count_below(ama)] = cell_a;
        if (acc_b) L.pcidx[pc_n + na + count_below(amb)] = cell_b;
        const uint32_t nacc = na + (uint32_t)__popcll(amb);
        pc_n += nacc;
        cnt_pc += nacc;

        // ---- opened internal cells -> their children ranges; the first popped
        // cell's children end on top, so deeper ranges stay above shallower ones
        const uint64_t oma = ballot(open_a), omb = ballot(open_b);
        const uint32_t nob = (uint32_t)__popcll(omb);
        const uint32_t npush = (uint32_t)__popcll(oma) + nob;
        if (sp_new + npush > (uint32_t)kStackMax) {  // cannot happen: 128 ranges per level
            if (lane == 0) atomicOr(tv.status, kStOverflow);
            break;
        }
        while (sp_new + npush > lo + tv.ring) {
            // spill the 64 lowest resident entries (all below sp_new when ring >= 192)
            __syncthreads();
            spill[lo + lane] = L.ring[(lo + lane) & rmask];
            lo += 64u;
            __syncthreads();
        }
        if (open_a) {
            const uint32_t above = lane == 63u ? 0u : (uint32_t)__popcll(oma >> (lane + 1u));
            L.ring[(sp_new + nob + above) & rmask] = (Na.x << 3) | (Na.y - 1u);
        }
        if (open_b) {
            const uint32_t above = lane == 63u ? 0u : (uint32_t)__popcll(omb >> (lane + 1u));
            L.ring[(sp_new + above) & rmask] = (Nb.x << 3) | (Nb.y - 1u);
        }
        sp = sp_new + npush;

        // ---- opened leaves -> their cells (kLeafCells)
        if constexpr (kLeafCells) {
            if (pp_n + 128u > (uint32_t)kPpCap) {
                __syncthreads();
                flush_pp(pp_n);
                pp_n = 0;
            }
            const uint64_t la = ballot(leaf_a), lb = ballot(leaf_b);
            const uint32_t nla = (uint32_t)__popcll(la);
            if (leaf_a) L.ppidx[pp_n + count_below(la)] = cell_a;
            if (leaf_b) L.ppidx[pp_n + nla + count_below(lb)] = cell_b;
            const uint32_t nl = nla + (uint32_t)__popcll(lb);
            pp_n += nl;
            cnt_pp += nl;
        }
        // ---- particles of opened leaves -> particle-particle index list.  Lane
        // l's leaves are entries 2l (slot a) and 2l + 1 (slot b) of the offset
        // table; a leaf holds at least one particle, so no opened leaf means
        // nothing to scan.
        const bool pa = !kLeafCells && leaf_a, pb = !kLeafCells && leaf_b;
        if (ballot(pa || pb) != 0ull) {
            const uint32_t ca = pa ? (Na.y & ~kLeafBit) : 0u;
            const uint32_t lc = ca + (pb ? (Nb.y & ~kLeafBit) : 0u);
            const uint32_t lincl = wave_incl_scan(lc, lane);
            const uint32_t P = read_lane(lincl, 63u);
            const uint32_t o = lincl - lc;
            L.offs[2u * lane] = o;
            L.offs[2u * lane + 1u] = o + ca;
            L.firsts[2u * lane] = Na.x;
            L.firsts[2u * lane + 1u] = Nb.x;
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
                    for (uint32_t step = 64; step > 0; step >>= 1)
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
    if (pc_n) flush_pc(pc_n);
    if (pp_n) flush_pp(pp_n);
    __syncthreads();
}

// Persistent group loop: groups come from eight contiguous ranges through
// the atomic counters work[0..7]; fn(g) handles group g.
template <class Fn>
__device__ __forceinline__ void for_each_group(uint32_t ng, uint32_t *work, uint32_t lane,
                                               Fn &&fn) {
    for (uint32_t k = 0; k < 8; ++k) {
        const uint32_t part = (blockIdx.x + k) & 7u;
        const uint32_t r0 = (uint32_t)(((uint64_t)ng * part) >> 3);
        const uint32_t r1 = (uint32_t)(((uint64_t)ng * (part + 1)) >> 3);
        for (;;) {
            uint32_t t = 0;
            if (lane == 0) t = atomicAdd(&work[part], 1u);
            t = uniform(t);
            if (t >= r1 - r0) break;
            fn(r0 + t);
        }
    }
}

}  // namespace bh
