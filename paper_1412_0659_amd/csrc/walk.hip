// Group-wise tree walk fused with the force evaluation (Sec. III.A: walk
// and force in one kernel, interaction lists kept on chip and evaluated on
// the fly; Sec. I.A: opening angle theta; Sec. VI.A Eq. (1)-(2); Table II
// "Compute gravity").
//
// The traversal (range stack, opening test, index lists, group scheduling)
// is in walk_common.h.  This file evaluates the lists: a full list is
// evaluated in chunks of 64 sources; each lane loads one source record into
// LDS (the next chunk's loads are issued before the current chunk is
// evaluated), then lane = (target, slice) evaluates the chunk, slice s
// taking entries s, s + r, ...; the slices are summed at the end.
#include "walk_common.h"

namespace bh {

struct WalkArgs {
    const float4 *xyzm;                  // targets: sorted positions + mass
    const float4 *sxyzm;                 // particle sources of the walked tree (= xyzm
                                         // unless the tree is another context's)
    const float4 *wA;                    // com, r_open^2
    const uint2 *wN;                     // (first, n | leaf bit)
    const float4 *P0, *P1, *P2;          // particle-cell records
    const uint32_t *gbeg, *ngroups;
    uint32_t *work, *spill;
    float4 *acc, *gbox;
    uint32_t *npp, *npc, *status;
    float eps2;
    uint32_t ring;  // resident stack entries allowed: kRing, or 192 to exercise the spill path
    uint32_t remote;  // 1: the walked tree is another domain's (no self pair)
    uint32_t accum;   // 1: add to acc, npp, npc instead of overwriting them
};

__device__ __forceinline__ float rsq(float v) { return __builtin_amdgcn_rsqf(v); }

// One particle-cell term, Eq. (1)-(2) with r^2 -> r^2 + eps^2.
// A = (com x, y, z, M); B = (-3 Qxx, -3 Qyy, -3 Qzz, -3 Qxy);
// C = (-3 Qxz, -3 Qyz, tr Q / 2, -3 tr Q / 2).  With q = -3 Q d and
// w = d.q / r^2, in nested form (33 VALU operations and one rsq):
//   phi += -M/r + (tr/2)/r^3 + (1/2) d.q / r^5 = [-M + (tr/2 + w/2) / r^2] / r
//   a   += d [M/r^3 - (3/2) tr/r^5 - (5/2) d.q / r^7] + q / r^5
//        = (q + h d) / r^5,  h = M r^2 - 3 tr/2 - 5 w/2
__device__ __forceinline__ void pc_term(const float4 &T, const float4 &A, const float4 &B,
                                        const float4 &C, float eps2, float4 &acc) {
    float dx = A.x - T.x, dy = A.y - T.y, dz = A.z - T.z;
    float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
    float ri = rsq(r2);
    float ri2 = ri * ri;
    float ri5 = (ri2 * ri2) * ri;
    float qx = fmaf(B.x, dx, fmaf(B.w, dy, C.x * dz));
    float qy = fmaf(B.w, dx, fmaf(B.y, dy, C.y * dz));
    float qz = fmaf(C.x, dx, fmaf(C.y, dy, B.z * dz));
    float dq = fmaf(dx, qx, fmaf(dy, qy, dz * qz));
    float w = dq * ri2;
    float p = fmaf(fmaf(0.5f, w, C.z), ri2, -A.w);
    acc.w = fmaf(p, ri, acc.w);
    float h = fmaf(A.w, r2, fmaf(-2.5f, w, C.w));
    acc.x = fmaf(ri5, fmaf(h, dx, qx), acc.x);
    acc.y = fmaf(ri5, fmaf(h, dy, qy), acc.y);
    acc.z = fmaf(ri5, fmaf(h, dz, qz), acc.z);
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

// ---- FP16 far field --------------------------------------------------------
//
// Particle-cell terms in packed FP16 with FP32 accumulation.  Each (group,
// cell) pair is rescaled by a power of two s so that every quantity in FP16
// is of order one: with L = |com - gc|_inf + |gh|_inf (gc, gh: group box)
// and s = 2^-e, 2^(e-1) <= L < 2^e,
//   d^ = (com - x_i) s = (com - gc) s - rho (x_i - gc) s_g,  rho = s / s_g,
//   Q^ = Q s^2 / M,  eps^2 -> eps^2 s^2,
//   a   = (M s^2) [d^ (r^-3 - 3/2 tr Q^ r^-5 + 15/2 d^Q^d^ r^-7) - 3 Q^ d^ r^-5]
//   phi = (M s)   [-r^-1 + 1/2 tr Q^ r^-3 - 3/2 d^Q^d^ r^-5]      (r = |d^|)
// where s_g = 2^-e_g scales the group (|x_i - gc| s_g < 1).  Both factors
// M s^2 and M s stay in FP32.  |d^| <= 2 sqrt(3); a pair whose box distance d
// has d s < 1/4 (a cell close to a wide group) would push r^-5 out of FP16
// range, so it is evaluated in FP32 instead.  Particle-particle terms are
// always FP32.
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ h2 hfma(h2 a, h2 b, h2 c) { return __builtin_elementwise_fma(a, b, c); }
__device__ __forceinline__ h2 hsplat(float v) {
    const _Float16 h = (_Float16)v;
    return h2{h, h};
}
__device__ __forceinline__ h2 as_h2(uint32_t u) { return __builtin_bit_cast(h2, u); }

// Pair record of cells (2p, 2p+1) of a chunk: 13 FP16x2 fields (low half =
// cell 2p), then the FP32 factors M s^2 and M s of both cells; 20 dwords so
// that it is read with four 16-byte loads and one 4-byte load.
enum { kDx, kDy, kDz, kRho, kE2, kBxx, kByy, kBzz, kBxy, kBxz, kByz, kHtr, kCtr, kH };
constexpr int kFa = kH, kFphi = kH + 2, kRec = 20;
constexpr int kNullPair = kChunk / 2;

struct Far16Lds {
    uint32_t rec[kChunk / 2 + 1][kRec];
};

struct WalkLds {
    float4 stage[3][kChunk + 1];  // source records of one chunk + the null source
    TravLds T;
};

// Target roles of a lane in one evaluation phase: T targets, r slices;
// lanes >= T * r are idle (they repeat slice 0 and are ignored).
struct Phase {
    uint32_t T, r, slice;
    bool act;
    float4 tgt;
    float4 acc;
    h2 ti[3];  // FP16 far field: (x_i - gc) s_g, both halves equal
};

// One pair of particle-cell terms in FP16 (cells 2p and 2p+1 of the chunk).
__device__ __forceinline__ void pc16_pair(const h2 ti[3], const Far16Lds &S, uint32_t p,
                                          float4 &acc) {
    const uint4 *R = reinterpret_cast<const uint4 *>(S.rec[p]);
    const uint4 q0 = R[0], q1 = R[1], q2 = R[2], q3 = R[3];
    const float fphi1 = __builtin_bit_cast(float, S.rec[p][kFphi + 1]);
    const h2 rho = as_h2(q0.w);
    const h2 dx = hfma(-rho, ti[0], as_h2(q0.x));
    const h2 dy = hfma(-rho, ti[1], as_h2(q0.y));
    const h2 dz = hfma(-rho, ti[2], as_h2(q0.z));
    const h2 r2 = hfma(dx, dx, hfma(dy, dy, hfma(dz, dz, as_h2(q1.x))));
    h2 ri;
    ri.x = __builtin_amdgcn_rsqh(r2.x);
    ri.y = __builtin_amdgcn_rsqh(r2.y);
    const h2 ri2 = ri * ri, ri3 = ri * ri2, ri5 = ri3 * ri2;
    const h2 bxx = as_h2(q1.y), byy = as_h2(q1.z), bzz = as_h2(q1.w);
    const h2 bxy = as_h2(q2.x), bxz = as_h2(q2.y), byz = as_h2(q2.z);
    const h2 qx = hfma(bxx, dx, hfma(bxy, dy, bxz * dz));
    const h2 qy = hfma(bxy, dx, hfma(byy, dy, byz * dz));
    const h2 qz = hfma(bxz, dx, hfma(byz, dy, bzz * dz));
    const h2 dq = hfma(dx, qx, hfma(dy, qy, dz * qz));
    const h2 a5 = dq * ri5;
    h2 ph = hfma(as_h2(q2.w), ri3, -ri);
    ph = hfma(hsplat(0.5f), a5, ph);
    const h2 u = hfma(hsplat(-2.5f), a5, ri);
    const h2 s = hfma(as_h2(q3.x), ri5, u * ri2);
    const h2 ax = hfma(s, dx, qx * ri5), ay = hfma(s, dy, qy * ri5), az = hfma(s, dz, qz * ri5);
    const float fa0 = __builtin_bit_cast(float, q3.y), fa1 = __builtin_bit_cast(float, q3.z);
    const float fphi0 = __builtin_bit_cast(float, q3.w);
    acc.x = fmaf((float)ax.x, fa0, acc.x);
    acc.x = fmaf((float)ax.y, fa1, acc.x);
    acc.y = fmaf((float)ay.x, fa0, acc.y);
    acc.y = fmaf((float)ay.y, fa1, acc.y);
    acc.z = fmaf((float)az.x, fa0, acc.z);
    acc.z = fmaf((float)az.y, fa1, acc.z);
    acc.w = fmaf((float)ph.x, fphi0, acc.w);
    acc.w = fmaf((float)ph.y, fphi1, acc.w);
}

// Evaluate n staged pairs for one phase (null pair past the end).
__device__ __forceinline__ void eval16_chunk(Phase &ph, uint32_t n, const Far16Lds &S) {
    const uint32_t r = ph.r;
    const uint32_t full = n / r, rem = n - full * r;
    uint32_t k = ph.slice;
    for (uint32_t j = 0; j < full; ++j, k += r) pc16_pair(ph.ti, S, k, ph.acc);
    if (rem) pc16_pair(ph.ti, S, ph.slice < rem ? k : (uint32_t)kNullPair, ph.acc);
}

// Write the FP16 half-record of cell k of the chunk (a far cell, or a hole
// that contributes nothing when !valid).  s = 2^-e scales the (group, cell)
// pair, eg the group; Q^ = Q s^2 / M uses an approximate 1/M (the FP16
// rounding dominates its error).
__device__ __forceinline__ void stage16(Far16Lds &S, uint32_t k, bool valid, const float4 &A,
                                        const float4 &B, const float4 &C, float cx, float cy,
                                        float cz, int e, int eg, float eps2) {
    float v[kH], fa = 0.f, fp = 0.f;
#pragma unroll
    for (int f = 0; f < kH; ++f) v[f] = 0.f;
    v[kDx] = 1.f;
    if (valid) {
        const float s = ldexpf(1.f, -e);
        const float k2 = s * s * __builtin_amdgcn_rcpf(A.w);
        v[kDx] = cx * s; v[kDy] = cy * s; v[kDz] = cz * s;
        v[kRho] = ldexpf(1.f, min(eg - e, 14));
        v[kE2] = fminf(eps2 * s * s, 6.0e4f);
        v[kBxx] = B.x * k2; v[kByy] = B.y * k2; v[kBzz] = B.z * k2;
        v[kBxy] = B.w * k2; v[kBxz] = C.x * k2; v[kByz] = C.y * k2;
        v[kHtr] = C.z * k2; v[kCtr] = C.w * k2;
        fa = A.w * s * s;
        fp = A.w * s;
    }
    uint32_t *rec = S.rec[k >> 1];
    _Float16 *h = reinterpret_cast<_Float16 *>(rec) + (k & 1u);
#pragma unroll
    for (int f = 0; f < kH; ++f) h[2 * f] = (_Float16)v[f];
    rec[kFa + (k & 1u)] = __builtin_bit_cast(uint32_t, fa);
    rec[kFphi + (k & 1u)] = __builtin_bit_cast(uint32_t, fp);
}

// Evaluate n (<= 64) staged sources for one phase; entries past n read the
// null source (far away, zero mass) so every round is uniform.
template <bool kIsPc, bool kEps0>
__device__ __forceinline__ void eval_chunk(Phase &ph, uint32_t n, const WalkLds &L, float eps2) {
    const uint32_t r = ph.r;
    const uint32_t full = n / r, rem = n - full * r;
    uint32_t j = 0;
    {
        // one induction variable: the lane's source record in stage[0]
        // (stage[1], stage[2] follow at fixed offsets)
        const float4 *src = &L.stage[0][ph.slice];
        constexpr uint32_t kRow = kChunk + 1;
        for (; j + 1u < full; j += 2u, src += 2u * r) {  // two sources per trip
            if (kIsPc) {
                pc_term(ph.tgt, src[0], src[kRow], src[2 * kRow], eps2, ph.acc);
                pc_term(ph.tgt, src[r], src[r + kRow], src[r + 2 * kRow], eps2, ph.acc);
            } else {
                pp_term<kEps0>(ph.tgt, src[0], eps2, ph.acc);
                pp_term<kEps0>(ph.tgt, src[r], eps2, ph.acc);
            }
        }
    }
    uint32_t k = ph.slice + j * r;
    if (j < full) {
        if (kIsPc) pc_term(ph.tgt, L.stage[0][k], L.stage[1][k], L.stage[2][k], eps2, ph.acc);
        else pp_term<kEps0>(ph.tgt, L.stage[0][k], eps2, ph.acc);
        k += r;
    }
    if (rem) {
        const uint32_t kk = ph.slice < rem ? k : (uint32_t)kNull;
        if (kIsPc) pc_term(ph.tgt, L.stage[0][kk], L.stage[1][kk], L.stage[2][kk], eps2, ph.acc);
        else pp_term<kEps0>(ph.tgt, L.stage[0][kk], eps2, ph.acc);
    }
}

template <bool kEps0, bool kF16>
__device__ void walk_group(const WalkArgs &a, uint32_t g, uint32_t lane, WalkLds &L,
                           Far16Lds &S, uint32_t *spill) {
    const uint32_t gb = a.gbeg[g];
    const uint32_t gn = a.gbeg[g + 1] - gb;  // 1..64 by construction
    if (gn == 0u || gn > 64u) {
        if (lane == 0) atomicOr(a.status, kStOverflow);
        return;
    }

    // ---- group box
    const bool own = lane < gn;
    const float4 me = a.xyzm[gb + (own ? lane : 0u)];
    const GroupBox b = group_box(me, own);
    if (lane == 0) {
        a.gbox[2 * (size_t)g] = make_float4(b.cx, b.cy, b.cz, 0.f);
        a.gbox[2 * (size_t)g + 1] = make_float4(b.hx, b.hy, b.hz, 0.f);
    }

    // ---- lane roles: one or two phases, whichever needs fewer rounds
    Phase p1, p2;
    plan_phases(gn, p1.T, p1.r, p2.T, p2.r);
    p1.act = lane < p1.T * p1.r;
    p1.slice = p1.act ? lane / p1.T : 0u;
    p1.tgt = a.xyzm[gb + (p1.act ? lane % p1.T : 0u)];
    p1.acc = make_float4(0.f, 0.f, 0.f, 0.f);
    p2.act = p2.T && lane < p2.T * p2.r;
    p2.slice = p2.act ? lane / p2.T : 0u;
    p2.tgt = a.xyzm[gb + (p2.act ? p1.T + lane % p2.T : 0u)];
    p2.acc = make_float4(0.f, 0.f, 0.f, 0.f);
    const bool two = p2.T != 0u;

    // FP16 far field: group scale s_g = 2^-eg with |x_i - gc| s_g < 1
    const float ghmax = fmaxf(fmaxf(b.hx, b.hy), b.hz);
    const int eg = ghmax > 0.f ? max(__builtin_amdgcn_frexp_expf(ghmax), -100) : -100;
    if (kF16) {
        const float sg = ldexpf(1.f, -eg);
        p1.ti[0] = hsplat((p1.tgt.x - b.cx) * sg);
        p1.ti[1] = hsplat((p1.tgt.y - b.cy) * sg);
        p1.ti[2] = hsplat((p1.tgt.z - b.cz) * sg);
        p2.ti[0] = hsplat((p2.tgt.x - b.cx) * sg);
        p2.ti[1] = hsplat((p2.tgt.y - b.cy) * sg);
        p2.ti[2] = hsplat((p2.tgt.z - b.cz) * sg);
    }

    // the null source of the FP32 staging area (rewritten by every flush: in
    // the FP16 walk the pair records share that area): massless and far
    // enough that 1/r^5 underflows to zero while r^2 stays finite, so every
    // product in its terms is an exact zero (M r^2 = 0 * inf would be NaN)
    auto put_null = [&]() {
        if (lane == 0) {
            L.stage[0][kNull] = make_float4(1e18f, 1e18f, 1e18f, 0.f);
            L.stage[1][kNull] = make_float4(0.f, 0.f, 0.f, 0.f);
            L.stage[2][kNull] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };

    // evaluate the particle-cell list: stage 64 records at a time, loading
    // the next chunk while the current one is evaluated
    auto flush_pc32 = [&](uint32_t n) {
        put_null();
        float4 r0, r1, r2;
        {
            const uint32_t c = L.T.pcidx[lane < n ? lane : 0u];
            r0 = a.P0[c]; r1 = a.P1[c]; r2 = a.P2[c];
        }
        for (uint32_t base = 0; base < n; base += kChunk) {
            const uint32_t m = n - base < (uint32_t)kChunk ? n - base : (uint32_t)kChunk;
            __syncthreads();
            L.stage[0][lane] = r0; L.stage[1][lane] = r1; L.stage[2][lane] = r2;
            __syncthreads();
            if (base + kChunk < n) {
                const uint32_t q = base + kChunk + lane;
                const uint32_t c = L.T.pcidx[q < n ? q : base + kChunk];
                r0 = a.P0[c]; r1 = a.P1[c]; r2 = a.P2[c];
            }
            eval_chunk<true, kEps0>(p1, m, L, a.eps2);
            if (two) eval_chunk<true, kEps0>(p2, m, L, a.eps2);
        }
        __syncthreads();
    };
    // FP16 far field: each chunk is staged as FP16 pair records; cells too
    // close to the group for FP16 leave a hole and their indices are moved
    // to the front of the list (positions already consumed), to be
    // evaluated in FP32, in full chunks, after the far cells
    auto flush_pc16 = [&](uint32_t n) {
        if (lane < 2) {  // the null pair
            const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
            stage16(S, kChunk + lane, false, z4, z4, z4, 0.f, 0.f, 0.f, 0, 0, 0.f);
        }
        float4 r0, r1, r2;
        {
            const uint32_t c = L.T.pcidx[lane < n ? lane : 0u];
            r0 = a.P0[c]; r1 = a.P1[c]; r2 = a.P2[c];
        }
        uint32_t nnear = 0;
        for (uint32_t base = 0; base < n; base += kChunk) {
            const uint32_t m = n - base < (uint32_t)kChunk ? n - base : (uint32_t)kChunk;
            const bool valid = lane < m;
            const uint32_t cidx = L.T.pcidx[base + (valid ? lane : 0u)];
            const float cx = r0.x - b.cx, cy = r0.y - b.cy, cz = r0.z - b.cz;
            const float Lc = fmaxf(fmaxf(fabsf(cx), fabsf(cy)), fabsf(cz)) + ghmax;
            const int e = __builtin_amdgcn_frexp_expf(Lc);
            const float bx = fmaxf(fabsf(cx) - b.hx, 0.f), by = fmaxf(fabsf(cy) - b.hy, 0.f),
                        bz = fmaxf(fabsf(cz) - b.hz, 0.f);
            // near: box distance d with d s < 1/4, i.e. d^2 < 2^(2e - 4)
            const float d2 = fmaf(bx, bx, fmaf(by, by, bz * bz));
            const bool near = valid && !(d2 >= ldexpf(1.f, 2 * e - 4));
            __syncthreads();
            stage16(S, lane, valid && !near, r0, r1, r2, cx, cy, cz, e, eg, a.eps2);
            const uint64_t nm = ballot(near);
            if (near) L.T.pcidx[nnear + count_below(nm)] = cidx;
            nnear += (uint32_t)__popcll(nm);
            __syncthreads();
            if (base + kChunk < n) {
                const uint32_t q = base + kChunk + lane;
                const uint32_t c = L.T.pcidx[q < n ? q : base + kChunk];
                r0 = a.P0[c]; r1 = a.P1[c]; r2 = a.P2[c];
            }
            const uint32_t np = (m + 1u) >> 1;
            eval16_chunk(p1, np, S);
            if (two) eval16_chunk(p2, np, S);
        }
        __syncthreads();
        if (nnear) flush_pc32(nnear);
    };
    auto flush_pc = [&](uint32_t n) {
        if (kF16) flush_pc16(n);
        else flush_pc32(n);
    };
    auto flush_pp = [&](uint32_t n) {
        put_null();
        float4 r0 = a.sxyzm[L.T.ppidx[lane < n ? lane : 0u]];
        for (uint32_t base = 0; base < n; base += kChunk) {
            const uint32_t m = n - base < (uint32_t)kChunk ? n - base : (uint32_t)kChunk;
            __syncthreads();
            L.stage[0][lane] = r0;
            __syncthreads();
            if (base + kChunk < n) {
                const uint32_t q = base + kChunk + lane;
                r0 = a.sxyzm[L.T.ppidx[q < n ? q : base + kChunk]];
            }
            eval_chunk<false, kEps0>(p1, m, L, a.eps2);
            if (two) eval_chunk<false, kEps0>(p2, m, L, a.eps2);
        }
        __syncthreads();
    };

    uint32_t cnt_pc, cnt_pp;
    const TreeView tv{a.wA, a.wN, a.ring, a.status};
    traverse(tv, b, lane, L.T, spill, cnt_pc, cnt_pp, flush_pc, flush_pp);

    // ---- sum the slices of each target (staging area reused)
    float4 res = make_float4(0.f, 0.f, 0.f, 0.f);
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
        if (!kEps0 && !a.remote) res.w += me.w * rsq(a.eps2);
        if (a.accum) {
            const float4 o = a.acc[gb + lane];
            res.x = o.x + res.x; res.y = o.y + res.y; res.z = o.z + res.z; res.w = o.w + res.w;
        }
        a.acc[gb + lane] = res;
    }
    if (lane == 0) {
        a.npp[g] = (a.accum ? a.npp[g] : 0u) + cnt_pp;
        a.npc[g] = (a.accum ? a.npc[g] : 0u) + cnt_pc;
    }
    __syncthreads();
}

template <bool kEps0, bool kF16>
__device__ __forceinline__ void walk_loop(const WalkArgs &a, WalkLds &L, Far16Lds &S) {
    const uint32_t lane = threadIdx.x;
    uint32_t *spill = a.spill + (size_t)blockIdx.x * kStackMax;
    for_each_group(*a.ngroups, a.work, lane,
                   [&](uint32_t g) { walk_group<kEps0, kF16>(a, g, lane, L, S, spill); });
}

template <bool kEps0, bool kF16>
__global__ __launch_bounds__(64) void k_walk(WalkArgs a) {
    __shared__ WalkLds L;
    // the FP16 pair records share the FP32 staging area: a flush uses one
    // or the other, and each flush rewrites its null source
    static_assert(sizeof(Far16Lds) <= sizeof(L.stage), "pair records exceed the staging area");
    walk_loop<kEps0, kF16>(a, L, *reinterpret_cast<Far16Lds *>(&L.stage[0][0]));
}

__global__ void k_reset_work(uint32_t *work) {
    if (threadIdx.x < 8) work[threadIdx.x] = 0u;
}

int walk_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_walk<false, false>, 64, 0) != hipSuccess ||
        nb < 1)
        nb = 4;
    return nb;
}

void launch_walk_view(bh_ctx *c, const SrcView &v, float eps, bool remote, bool accum,
                      hipStream_t st) {
    WalkArgs a;
    a.xyzm = c->xyzm;
    a.sxyzm = v.xyzm;
    a.wA = v.wA; a.wN = v.wN;
    a.P0 = v.P0; a.P1 = v.P1; a.P2 = v.P2;
    a.gbeg = c->groups.begin; a.ngroups = c->groups.count_dev;
    a.work = c->work; a.spill = c->spill;
    a.acc = c->acc; a.gbox = c->groups.box;
    a.npp = c->groups.npp; a.npc = c->groups.npc; a.status = c->status;
    a.eps2 = eps * eps;
    a.ring = c->walk_small_stack ? 192u : (uint32_t)kRing;
    a.remote = remote ? 1u : 0u;
    a.accum = accum ? 1u : 0u;
    hipLaunchKernelGGL(k_reset_work, dim3(1), dim3(64), 0, st, c->work);
    const bool own = !remote && !accum;  // the timed walk of the context's own tree
    if (own) record_event(c, 4, st);
    const bool f16 = c->p.far_fp16 != 0;
    if (eps == 0.f && f16)
        hipLaunchKernelGGL((k_walk<true, true>), dim3(c->walk_grid), dim3(64), 0, st, a);
    else if (eps == 0.f)
        hipLaunchKernelGGL((k_walk<true, false>), dim3(c->walk_grid), dim3(64), 0, st, a);
    else if (f16)
        hipLaunchKernelGGL((k_walk<false, true>), dim3(c->walk_grid), dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL((k_walk<false, false>), dim3(c->walk_grid), dim3(64), 0, st, a);
    if (own) record_event(c, 5, st);
}

SrcView own_view(const bh_ctx *c) {
    SrcView v;
    v.wA = c->cells.wA; v.wN = c->cells.wN;
    v.P0 = c->cells.P0; v.P1 = c->cells.P1; v.P2 = c->cells.P2;
    v.xyzm = c->xyzm;
    return v;
}

void launch_walk(bh_ctx *c, float eps, hipStream_t st) {
    launch_walk_view(c, own_view(c), eps, false, false, st);
}

}  // namespace bh
