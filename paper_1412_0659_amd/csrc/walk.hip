// Group-wise tree walk fused with the force evaluation (Sec. III.A: walk
// and force in one kernel, interaction lists kept on chip and evaluated on
// the fly; Sec. I.A: opening angle theta; Sec. VI.A Eq. (1)-(2); Table II
// "Compute gravity").
//
// One 64-lane wavefront walks the tree for one target group:
//   * the stack holds ranges of sibling cells (first << 3 | count - 1); each
//     pass pops up to 64 cells, one per lane;
//   * each lane applies the opening test: distance d from the cell's centre
//     of mass to the group's box, accept the cell whole iff
//     d^2 >= (l / theta + delta)^2 (FP32, no contraction);
//   * accepted cells are compacted (ballot + mbcnt) into an LDS
//     particle-cell list, particles of opened leaves into an LDS
//     particle-particle list, children of opened internal cells are pushed
//     back as ranges, shallower ranges below deeper ones so that the stack
//     holds at most 64 ranges per level;
//   * a list is evaluated when it fills: lane = (target t, slice s) with
//     r = floor(64 / group size) slices, slice s taking list entries
//     s, s + r, ...; the slices are summed at the end, so small groups still
//     keep most lanes busy.
// Groups are taken from eight contiguous ranges (one per XCD, blockIdx % 8)
// through atomic counters, so neighbouring groups share an L2; every wave
// leaves once all ranges are exhausted.
#include "bh_internal.h"
#include "wave.h"

namespace bh {

constexpr int kPcCap = 192;
constexpr int kPcFlush = kPcCap - 64;
constexpr int kPpCap = 256;
constexpr int kPpFlush = kPpCap - 64;
constexpr int kStack = 1408;  // 21 levels below the root x 64 ranges + root

struct WalkArgs {
    const float *x, *y, *z, *m;
    const float4 *wA, *wM, *wQ;
    const uint2 *wN;
    const uint32_t *gbeg, *ngroups;
    uint32_t *work;
    float4 *acc, *gbox;
    uint32_t *npp, *npc, *status;
    float eps2;
};

__device__ __forceinline__ float rsq(float v) { return __builtin_amdgcn_rsqf(v); }

// A = (com x, y, z, M), B = (Qxx, Qyy, Qzz, Qxy), C = (Qxz, Qyz, tr/2, -3 tr/2)
__device__ __forceinline__ void pc_term(float xi, float yi, float zi, float4 A, float4 B, float4 C,
                                        float eps2, float &ax, float &ay, float &az, float &ph) {
    float dx = A.x - xi, dy = A.y - yi, dz = A.z - zi;
    float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
    float ri = rsq(r2);
    float ri2 = ri * ri;
    float mr = A.w * ri;
    float ri3 = ri * ri2;
    float ri5 = ri3 * ri2;
    float qx = fmaf(B.x, dx, fmaf(B.w, dy, C.x * dz));
    float qy = fmaf(B.w, dx, fmaf(B.y, dy, C.y * dz));
    float qz = fmaf(C.x, dx, fmaf(C.y, dy, B.z * dz));
    float dqd = fmaf(dx, qx, fmaf(dy, qy, dz * qz));
    float a5 = dqd * ri5;
    ph = ph - mr;
    ph = fmaf(C.z, ri3, ph);
    ph = fmaf(-1.5f, a5, ph);
    float s = fmaf(C.w, ri5, mr * ri2);
    s = fmaf(7.5f * a5, ri2, s);
    float t = -3.0f * ri5;
    ax = fmaf(s, dx, fmaf(t, qx, ax));
    ay = fmaf(s, dy, fmaf(t, qy, ay));
    az = fmaf(s, dz, fmaf(t, qz, az));
}

template <bool kEps0>
__device__ __forceinline__ void pp_term(float xi, float yi, float zi, float4 P, float eps2,
                                        float &ax, float &ay, float &az, float &ph) {
    float dx = P.x - xi, dy = P.y - yi, dz = P.z - zi;
    float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
    float ri = rsq(r2);
    if (kEps0) ri = r2 > 0.f ? ri : 0.f;
    float mr = P.w * ri;
    float mr3 = mr * (ri * ri);
    ph = ph - mr;
    ax = fmaf(mr3, dx, ax);
    ay = fmaf(mr3, dy, ay);
    az = fmaf(mr3, dz, az);
}

struct WalkLds {
    float4 pcA[kPcCap], pcB[kPcCap], pcC[kPcCap];
    float4 pp[kPpCap];
    uint32_t stk[kStack];
    uint32_t offs[64], firsts[64], starts[64];
};

template <bool kEps0>
__device__ void walk_group(const WalkArgs &a, uint32_t g, uint32_t lane, WalkLds &L) {
    const uint32_t gb = a.gbeg[g];
    const uint32_t gn = a.gbeg[g + 1] - gb;  // 1..64 by construction
    if (gn == 0u || gn > 64u) {
        if (lane == 0) atomicOr(a.status, kStOverflow);
        return;
    }
    const uint32_t r = 64u / gn;
    const uint32_t tgt = lane % gn;
    const uint32_t slice = lane / gn;
    const bool act = slice < r;
    const float xi = a.x[gb + tgt], yi = a.y[gb + tgt], zi = a.z[gb + tgt];
    const bool own = lane < gn;

    float gcx, gcy, gcz, ghx, ghy, ghz;
    {
        float mn = wave_min(own ? xi : INFINITY), mx = wave_max(own ? xi : -INFINITY);
        gcx = (mn + mx) * 0.5f; ghx = (mx - mn) * 0.5f;
        mn = wave_min(own ? yi : INFINITY); mx = wave_max(own ? yi : -INFINITY);
        gcy = (mn + mx) * 0.5f; ghy = (mx - mn) * 0.5f;
        mn = wave_min(own ? zi : INFINITY); mx = wave_max(own ? zi : -INFINITY);
        gcz = (mn + mx) * 0.5f; ghz = (mx - mn) * 0.5f;
    }
    if (lane == 0) {
        a.gbox[2 * (size_t)g] = make_float4(gcx, gcy, gcz, 0.f);
        a.gbox[2 * (size_t)g + 1] = make_float4(ghx, ghy, ghz, 0.f);
    }

    float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
    uint32_t cnt_pc = 0, cnt_pp = 0, pc_n = 0, pp_n = 0;
    uint32_t sp = 1;
    if (lane == 0) L.stk[0] = 0u;  // the root: first cell 0, one cell
    __syncthreads();

    auto flush_pc = [&](uint32_t n) {
        if (act)
            for (uint32_t k = slice; k < n; k += r)
                pc_term(xi, yi, zi, L.pcA[k], L.pcB[k], L.pcC[k], a.eps2, ax, ay, az, ph);
    };
    auto flush_pp = [&](uint32_t n) {
        if (act)
            for (uint32_t k = slice; k < n; k += r)
                pp_term<kEps0>(xi, yi, zi, L.pp[k], a.eps2, ax, ay, az, ph);
    };

    while (sp > 0) {
        // ---- pop up to 64 cells from the top ranges
        const uint32_t avail = sp < 64u ? sp : 64u;
        uint32_t e = 0, ne = 0;
        if (lane < avail) {
            e = L.stk[sp - 1 - lane];
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
            L.stk[sp_new - 1] = (((e >> 3) + taken) << 3) | (ne - taken - 1u);
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

        // ---- accepted cells -> particle-cell list
        const uint64_t am = ballot(accept);
        if (accept) {
            const uint32_t slot = pc_n + count_below(am);
            const float4 M4 = a.wM[cell], Q4 = a.wQ[cell];
            L.pcA[slot] = make_float4(A.x, A.y, A.z, M4.x);
            L.pcB[slot] = make_float4(M4.y, M4.z, M4.w, Q4.x);
            L.pcC[slot] = make_float4(Q4.y, Q4.z, Q4.w, -3.0f * Q4.w);
        }
        const uint32_t nacc = (uint32_t)__popcll(am);
        pc_n += nacc;
        cnt_pc += nacc;

        // ---- opened internal cells -> their children ranges, shallowest lowest
        const uint64_t om = ballot(openint);
        if (openint) {
            const uint32_t above = lane == 63u ? 0u : (uint32_t)__popcll(om >> (lane + 1u));
            const uint32_t pos = sp_new + above;
            if (pos < (uint32_t)kStack) L.stk[pos] = (N.x << 3) | (N.y - 1u);
        }
        sp = sp_new + (uint32_t)__popcll(om);
        if (sp > (uint32_t)kStack) {
            if (lane == 0) atomicOr(a.status, kStOverflow);
            sp = 0;
        }

        // ---- particles of opened leaves -> particle-particle list
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
                    __syncthreads();
                }
                const uint32_t room = (uint32_t)kPpCap - pp_n;
                const uint32_t take = room < P - base ? room : P - base;
                for (uint32_t q = lane; q < take; q += 64u) {
                    const uint32_t f = base + q;
                    uint32_t lo = 0;
#pragma unroll
                    for (uint32_t step = 32; step > 0; step >>= 1)
                        if (L.offs[lo + step] <= f) lo += step;
                    const uint32_t pi = L.firsts[lo] + (f - L.offs[lo]);
                    L.pp[pp_n + q] = make_float4(a.x[pi], a.y[pi], a.z[pi], a.m[pi]);
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
            __syncthreads();
        }
        if (pp_n > (uint32_t)kPpFlush) {
            flush_pp(pp_n);
            pp_n = 0;
            __syncthreads();
        }
    }
    __syncthreads();
    flush_pc(pc_n);
    flush_pp(pp_n);

    // ---- sum the slices of each target
    __syncthreads();
    L.pp[lane] = make_float4(ax, ay, az, ph);
    __syncthreads();
    if (own) {
        float4 s = L.pp[lane];
        for (uint32_t k = 1; k < r; ++k) {
            const float4 o = L.pp[lane + k * gn];
            s.x += o.x;
            s.y += o.y;
            s.z += o.z;
            s.w += o.w;
        }
        // the self pair was evaluated with r^2 = eps^2; take its potential out
        if (!kEps0) s.w += a.m[gb + lane] * rsq(a.eps2);
        a.acc[gb + lane] = s;
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
    for (uint32_t k = 0; k < 8; ++k) {
        const uint32_t part = (blockIdx.x + k) & 7u;
        const uint32_t r0 = (uint32_t)(((uint64_t)ng * part) >> 3);
        const uint32_t r1 = (uint32_t)(((uint64_t)ng * (part + 1)) >> 3);
        for (;;) {
            uint32_t t = 0;
            if (lane == 0) t = atomicAdd(&a.work[part], 1u);
            t = uniform(t);
            if (t >= r1 - r0) break;
            walk_group<kEps0>(a, r0 + t, lane, L);
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
    const State &s = c->st[c->cur];
    WalkArgs a;
    a.x = s.x; a.y = s.y; a.z = s.z; a.m = s.m;
    a.wA = c->cells.wA; a.wM = c->cells.wM; a.wQ = c->cells.wQ; a.wN = c->cells.wN;
    a.gbeg = c->groups.begin; a.ngroups = c->groups.count_dev;
    a.work = c->work;
    a.acc = c->acc; a.gbox = c->groups.box;
    a.npp = c->groups.npp; a.npc = c->groups.npc; a.status = c->status;
    a.eps2 = eps * eps;
    hipLaunchKernelGGL(k_reset_work, dim3(1), dim3(64), 0, st, c->work);
    hipEventRecord(c->ev[4], st);
    c->ev_rec[4] = true;
    if (eps == 0.f)
        hipLaunchKernelGGL(k_walk<true>, dim3(c->walk_grid), dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL(k_walk<false>, dim3(c->walk_grid), dim3(64), 0, st, a);
    hipEventRecord(c->ev[5], st);
    c->ev_rec[5] = true;
}

}  // namespace bh
