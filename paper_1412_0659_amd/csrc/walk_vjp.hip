// Adjoint of the tree force with the walk's decisions held fixed: given a
// cotangent u_i of every acceleration a_i, accumulate u^T da/dx and
// u^T da/dm.  The force is Sec. VI.A Eq. (2) (with r^2 -> r^2 + eps^2) over
// the interaction lists of the walk; cells enter through their moments
// (Sec. I.A, Eq. (1)), so the adjoint has three parts:
//   * targets:  d a_i / d x_i = -sum J  (J = dF/dd, d = source - x_i);
//   * sources:  particle j gets +J^T u_i and d F/d m_j . u_i; cell c gets
//               dL/dcom += J^T u_i, dL/dM += dF/dM . u_i, dL/dQ += dF/dQ . u_i;
//   * moments:  each particle k receives, from every cell holding it, with
//               s = x_k - com:  dcom/dx_k = m_k / M, dQ/dx_k = m_k (e s^T + s e^T),
//               dM/dm_k = 1, dcom/dm_k = s / M, dQ/dm_k = s s^T (the centre of
//               mass dependence of Q cancels because sum m s = 0).
// The walk (walk_common.h) is repeated exactly, so the lists are those of the
// force evaluation.  Particle-cell chunks: lane = cell, looping over the
// group's targets; each pair's J^T u is added to the cell's adjoint and, summed
// over the lanes with DPP, subtracted from the target's.  Particle-particle
// chunks: pass A (lane = target, slice) accumulates the target terms in
// registers, pass B (lane = source) loops over the targets for the source
// terms.  Source terms reach FP64 accumulators with one atomic per source
// and group.  The self pair (zero separation by construction) contributes
// nothing.
//
// The accumulators are field-major (cell adjoint q of cell c at q * cap + c),
// so the lanes of one atomic instruction, neighbouring cells or the
// particles of one leaf, share a few cache lines; and they come in kXcd
// copies, one per XCD: a wave adds into the copy of the XCD it runs on (read
// from the hardware XCC id), so no cache line is updated from two XCDs.  The
// cells of the top levels are accepted by far more groups than deeper ones
// (a few cache lines of them take a quarter of all the atomics), so the first
// kHotCells cells get kHotCopies copies, kHotCopies / kXcd per XCD chosen by
// the workgroup.  The copies are summed after the walk.
#include "walk_common.h"

namespace bh {

constexpr uint32_t kXcd = 8;

// XCD (XCC) that runs the calling wave.
__device__ __forceinline__ uint32_t xcc_id() {
    uint32_t v;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
    return v & (kXcd - 1u);
}

// FP64 add executed in the L2 of the calling XCD (no return value).
__device__ __forceinline__ void add_l2(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

struct VjpArgs {
    const float4 *xyzm;   // sorted positions + mass
    const float4 *u;      // sorted cotangents of the accelerations
    const float4 *wA;
    const uint2 *wN;
    const float4 *P0, *P1, *P2;
    const uint32_t *gbeg, *ngroups;
    uint32_t *work, *spill, *status;
    uint32_t ring;
    // copy 0 of kXcd accumulators; copy k at + k * lstride / gstride.  Field
    // major: cell adjoint q of cell c at lcell[q * cap + c], particle
    // adjoint q of particle j at gsrc[q * nmax + j], so that the lanes of one
    // atomic instruction (neighbouring cells or particles) share cache lines
    double *lcell, *gsrc;
    uint64_t lstride, gstride, cap, nmax;
    // kHotCopies copies of the first kHotCells cells' adjoints, copy k at
    // lhot + k * kHotCopy, field q of cell c at + q * kHotField + c
    double *lhot;
    float eps2;
};

__device__ __forceinline__ float rsqv(float v) { return __builtin_amdgcn_rsqf(v); }

// Adjoint of one particle-cell term (records as in the force walk:
// A = (com, M), B = -3 (Qxx, Qyy, Qzz, Qxy), C = (-3 Qxz, -3 Qyz, tr/2, -3 tr/2)).
// Returns w = J^T u and adds the cell-side terms to running sums.  With
// B = -3 Q, ctr = -3 tr / 2, ud = u.d:
//   w = u [M r^-3 + ctr r^-5 - 5/2 dBd r^-7]
//     + d [-3 M ud r^-5 - 5 ctr ud r^-7 - 5 uBd r^-7 + 35/2 dBd ud r^-9]
//     + Bu r^-5 - 5 ud Bd r^-7
// dF/dM . u = ud r^-3 (added to sM).  dF/dQ . u for the six stored entries:
// with v = r^-5 u - 5/2 ud r^-7 d,
//   diagonal  -3 v_a d_a - 3/2 ud r^-5,   off-diagonal  -3 (v_a d_b + v_b d_a);
// sQ collects the v-terms unscaled (diagonal v_a d_a, off-diagonal
// v_a d_b + v_b d_a) and st the ud r^-5, so that the factors -3 and -3/2 are
// applied once per sum (pc_adj_finish).
__device__ __forceinline__ void pc_adj(const float4 &T, const float4 &U, const float4 &A,
                                       const float4 &B, const float4 &C, float eps2, float &wx,
                                       float &wy, float &wz, float &sM, float *sQ, float &st) {
    const float dx = A.x - T.x, dy = A.y - T.y, dz = A.z - T.z;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
    const float ri = rsqv(r2);
    const float ri2 = ri * ri, ri3 = ri * ri2, ri5 = ri3 * ri2, ri7 = ri5 * ri2;
    const float ud = fmaf(U.x, dx, fmaf(U.y, dy, U.z * dz));
    const float bdx = fmaf(B.x, dx, fmaf(B.w, dy, C.x * dz));
    const float bdy = fmaf(B.w, dx, fmaf(B.y, dy, C.y * dz));
    const float bdz = fmaf(C.x, dx, fmaf(C.y, dy, B.z * dz));
    const float bux = fmaf(B.x, U.x, fmaf(B.w, U.y, C.x * U.z));
    const float buy = fmaf(B.w, U.x, fmaf(B.y, U.y, C.y * U.z));
    const float buz = fmaf(C.x, U.x, fmaf(C.y, U.y, B.z * U.z));
    const float q2 = fmaf(dx, bdx, fmaf(dy, bdy, dz * bdz)) * ri2;  // dBd / r^2
    const float uBd = fmaf(U.x, bdx, fmaf(U.y, bdy, U.z * bdz));
    const float M = A.w, ctr = C.w;
    const float cu = fmaf(fmaf(-2.5f, q2, ctr), ri5, M * ri3);
    const float udr7 = ud * ri7;
    const float cd =
        fmaf(ud, fmaf(-3.f * M, ri5, fmaf(17.5f, q2, -5.f * ctr) * ri7), -5.f * uBd * ri7);
    const float cb = -5.f * udr7;
    wx = fmaf(cu, U.x, fmaf(cd, dx, fmaf(bux, ri5, cb * bdx)));
    wy = fmaf(cu, U.y, fmaf(cd, dy, fmaf(buy, ri5, cb * bdy)));
    wz = fmaf(cu, U.z, fmaf(cd, dz, fmaf(buz, ri5, cb * bdz)));
    sM = fmaf(ud, ri3, sM);
    st = fmaf(ud, ri5, st);
    const float h = -2.5f * udr7;
    const float vx = fmaf(h, dx, ri5 * U.x), vy = fmaf(h, dy, ri5 * U.y),
                vz = fmaf(h, dz, ri5 * U.z);
    sQ[0] = fmaf(vx, dx, sQ[0]);
    sQ[1] = fmaf(vy, dy, sQ[1]);
    sQ[2] = fmaf(vz, dz, sQ[2]);
    sQ[3] = fmaf(vx, dy, fmaf(vy, dx, sQ[3]));
    sQ[4] = fmaf(vx, dz, fmaf(vz, dx, sQ[4]));
    sQ[5] = fmaf(vy, dz, fmaf(vz, dy, sQ[5]));
}

// dL/dQ of the six stored entries from the sums of pc_adj.
__device__ __forceinline__ void pc_adj_finish(float *sQ, float st) {
    const float t = -1.5f * st;
    sQ[0] = fmaf(-3.f, sQ[0], t);
    sQ[1] = fmaf(-3.f, sQ[1], t);
    sQ[2] = fmaf(-3.f, sQ[2], t);
    sQ[3] *= -3.f;
    sQ[4] *= -3.f;
    sQ[5] *= -3.f;
}

// Adjoint of one particle-particle term: F = m d r^-3, J = m (I r^-3 - 3 d d^T r^-5).
template <bool kEps0>
__device__ __forceinline__ void pp_adj(const float4 &T, const float4 &U, const float4 &P,
                                       float eps2, float &wx, float &wy, float &wz, float &gm) {
    const float dx = P.x - T.x, dy = P.y - T.y, dz = P.z - T.z;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
    float ri = rsqv(r2);
    if (kEps0) ri = r2 > 0.f ? ri : 0.f;
    const float ri2 = ri * ri, ri3 = ri * ri2, ri5 = ri3 * ri2;
    const float ud = fmaf(U.x, dx, fmaf(U.y, dy, U.z * dz));
    const float c1 = P.w * ri3, c2 = -3.f * P.w * ud * ri5;
    wx = fmaf(c1, U.x, c2 * dx);
    wy = fmaf(c1, U.y, c2 * dy);
    wz = fmaf(c1, U.z, c2 * dz);
    gm = ud * ri3;
}

// Sum of v over the 64 lanes, returned uniform: DPP inclusive scan (row
// shifts, then row broadcasts), lane 63's value read into a scalar.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_add(float s) {
    return s + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(s), kCtrl, kRowMask,
                                                          0xf, false));
}
__device__ __forceinline__ float wave_total(float v) {
    v = dpp_add<0x111, 0xf>(v);  // row_shr:1
    v = dpp_add<0x112, 0xf>(v);  // row_shr:2
    v = dpp_add<0x114, 0xf>(v);  // row_shr:4
    v = dpp_add<0x118, 0xf>(v);  // row_shr:8
    v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 -> rows 1, 3
    v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 -> rows 2, 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

struct VjpLds {
    float4 stage[1][kChunk + 1];  // particle sources of one chunk + the null source
    uint32_t sidx[kChunk + 1];    // particle index of staged particle sources
    float4 tp[64], tu[64];        // the group's targets: position + mass, cotangent
    uint32_t tidx[64];
    TravLds T;
};

struct VPhase {
    uint32_t T, r, slice, tidx;
    bool act;
    float4 tgt, u;
    float gx, gy, gz;
};

// Target terms of one staged chunk of particle sources for one phase.
template <bool kEps0>
__device__ __forceinline__ void vjp_targets(VPhase &ph, uint32_t n, const VjpLds &L, float eps2) {
    const uint32_t r = ph.r;
    const uint32_t rounds = (n + r - 1u) / r;
    uint32_t k = ph.slice;
    for (uint32_t j = 0; j < rounds; ++j, k += r) {
        const uint32_t kk = k < n ? k : (uint32_t)kNull;
        float wx, wy, wz, gm;
        pp_adj<kEps0>(ph.tgt, ph.u, L.stage[0][kk], eps2, wx, wy, wz, gm);
        if (L.sidx[kk] == ph.tidx) wx = wy = wz = 0.f;
        ph.gx -= wx;
        ph.gy -= wy;
        ph.gz -= wz;
    }
}

template <bool kEps0>
__device__ void vjp_group(const VjpArgs &a, uint32_t g, uint32_t lane, VjpLds &L,
                          uint32_t *spill) {
    const uint32_t gb = a.gbeg[g];
    const uint32_t gn = a.gbeg[g + 1] - gb;
    if (gn == 0u || gn > 64u) {
        if (lane == 0) atomicOr(a.status, kStOverflow);
        return;
    }
    const uint32_t xcd = xcc_id();
    double *const lcx = a.lcell + xcd * a.lstride;
    double *const gsx = a.gsrc + xcd * a.gstride;
    const uint32_t hk = xcd + kXcd * ((blockIdx.x / kXcd) % (kHotCopies / kXcd));
    double *const lhx = a.lhot + hk * kHotCopy;
    const bool own = lane < gn;
    const uint32_t ti = gb + (own ? lane : 0u);
    const float4 me = a.xyzm[ti];
    const GroupBox b = group_box(me, own);
    L.tp[lane] = own ? me : make_float4(1e30f, 1e30f, 1e30f, 0.f);
    L.tu[lane] = own ? a.u[ti] : make_float4(0.f, 0.f, 0.f, 0.f);
    L.tidx[lane] = own ? ti : kNone;
    if (lane == 0) {
        L.stage[0][kNull] = make_float4(1e30f, 1e30f, 1e30f, 0.f);
        L.sidx[kNull] = kNone;
    }

    VPhase p1, p2;
    plan_phases(gn, p1.T, p1.r, p2.T, p2.r);
    p1.act = lane < p1.T * p1.r;
    p1.slice = p1.act ? lane / p1.T : 0u;
    p1.tidx = gb + (p1.act ? lane % p1.T : 0u);
    p1.tgt = a.xyzm[p1.tidx];
    p1.u = a.u[p1.tidx];
    p1.gx = p1.gy = p1.gz = 0.f;
    p2.act = p2.T && lane < p2.T * p2.r;
    p2.slice = p2.act ? lane / p2.T : 0u;
    p2.tidx = gb + (p2.act ? p1.T + lane % p2.T : 0u);
    p2.tgt = a.xyzm[p2.tidx];
    p2.u = a.u[p2.tidx];
    p2.gx = p2.gy = p2.gz = 0.f;
    const bool two = p2.T != 0u;

    // particle-cell lists: lane = cell (a null cell, zero mass and moments, far
    // away, on lanes past the list), looping over the group's targets; each
    // pair's J^T u serves both sides: summed over targets into the cell's
    // adjoint, and over the lanes (a DPP sum) into the target's
    float gtx = 0.f, gty = 0.f, gtz = 0.f;  // target side of lane t's target
    auto flush_pc = [&](uint32_t n) {
        for (uint32_t base = 0; base < n; base += kChunk) {
            const uint32_t m = n - base < (uint32_t)kChunk ? n - base : (uint32_t)kChunk;
            const bool valid = lane < m;
            const uint32_t c = L.T.pcidx[base + (valid ? lane : 0u)];
            float4 r0 = make_float4(1e18f, 1e18f, 1e18f, 0.f), r1 = make_float4(0.f, 0.f, 0.f, 0.f),
                   r2 = r1;
            if (valid) {
                r0 = a.P0[c];
                r1 = a.P1[c];
                r2 = a.P2[c];
            }
            float sw[3] = {0.f, 0.f, 0.f}, sM = 0.f, st = 0.f;
            float sQ[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            for (uint32_t t = 0; t < gn; ++t) {
                float wx, wy, wz;
                pc_adj(L.tp[t], L.tu[t], r0, r1, r2, a.eps2, wx, wy, wz, sM, sQ, st);
                sw[0] += wx; sw[1] += wy; sw[2] += wz;
                const float tx = wave_total(wx), ty = wave_total(wy), tz = wave_total(wz);
                if (lane == t) {
                    gtx -= tx;
                    gty -= ty;
                    gtz -= tz;
                }
            }
            pc_adj_finish(sQ, st);
            if (valid) {
                const bool hot = c < kHotCells;
                double *lc = hot ? lhx + c : lcx + c;
                const uint64_t fs = hot ? kHotField : a.cap;
                add_l2(lc, (double)sM);
                add_l2(lc + fs, (double)sw[0]);
                add_l2(lc + 2 * fs, (double)sw[1]);
                add_l2(lc + 3 * fs, (double)sw[2]);
#pragma unroll
                for (int q = 0; q < 6; ++q) add_l2(lc + (4 + q) * fs, (double)sQ[q]);
            }
        }
        __syncthreads();
    };
    auto flush_pp = [&](uint32_t n) {
        for (uint32_t base = 0; base < n; base += kChunk) {
            const uint32_t m = n - base < (uint32_t)kChunk ? n - base : (uint32_t)kChunk;
            const bool valid = lane < m;
            const uint32_t j = L.T.ppidx[base + (valid ? lane : 0u)];
            const float4 P = a.xyzm[j];
            __syncthreads();
            L.stage[0][lane] = P;
            L.sidx[lane] = valid ? j : kNone;
            __syncthreads();
            vjp_targets<kEps0>(p1, m, L, a.eps2);
            if (two) vjp_targets<kEps0>(p2, m, L, a.eps2);
            float sx = 0.f, sy = 0.f, sz = 0.f, sm = 0.f;
            for (uint32_t t = 0; t < gn; ++t) {
                float wx, wy, wz, gm;
                pp_adj<kEps0>(L.tp[t], L.tu[t], P, a.eps2, wx, wy, wz, gm);
                if (L.tidx[t] != j) {
                    sx += wx; sy += wy; sz += wz; sm += gm;
                }
            }
            if (valid) {
                double *gs = gsx + j;
                add_l2(gs, (double)sx);
                add_l2(gs + a.nmax, (double)sy);
                add_l2(gs + 2 * a.nmax, (double)sz);
                add_l2(gs + 3 * a.nmax, (double)sm);
            }
        }
        __syncthreads();
    };

    uint32_t cnt_pc, cnt_pp;
    const TreeView tv{a.wA, a.wN, a.ring, a.status};
    traverse(tv, b, lane, L.T, spill, cnt_pc, cnt_pp, flush_pc, flush_pp);

    // ---- sum the slices of each target and add the target terms
    float rx = 0.f, ry = 0.f, rz = 0.f;
    L.stage[0][lane] = make_float4(p1.gx, p1.gy, p1.gz, 0.f);
    __syncthreads();
    if (lane < p1.T)
        for (uint32_t k = 0; k < p1.r; ++k) {
            const float4 o = L.stage[0][lane + k * p1.T];
            rx += o.x; ry += o.y; rz += o.z;
        }
    if (two) {
        __syncthreads();
        L.stage[0][lane] = make_float4(p2.gx, p2.gy, p2.gz, 0.f);
        __syncthreads();
        if (lane >= p1.T && lane < gn)
            for (uint32_t k = 0; k < p2.r; ++k) {
                const float4 o = L.stage[0][lane - p1.T + k * p2.T];
                rx += o.x; ry += o.y; rz += o.z;
            }
    }
    if (own) {
        double *gs = gsx + ti;
        add_l2(gs, (double)rx + (double)gtx);
        add_l2(gs + a.nmax, (double)ry + (double)gty);
        add_l2(gs + 2 * a.nmax, (double)rz + (double)gtz);
    }
    __syncthreads();
}

template <bool kEps0>
__global__ __launch_bounds__(64) void k_walk_vjp(VjpArgs a) {
    __shared__ VjpLds L;
    const uint32_t lane = threadIdx.x;
    uint32_t *spill = a.spill + (size_t)blockIdx.x * kStackMax;
    for_each_group(*a.ngroups, a.work, lane,
                   [&](uint32_t g) { vjp_group<kEps0>(a, g, lane, L, spill); });
}

// ---- moments part, combination and unsorting --------------------------------

__global__ __launch_bounds__(256) void k_leafof(Cells c, uint32_t *leafof) {
    const uint32_t nc = c.ls[kLevels];
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nc; i += gridDim.x * 256) {
        if (c.nchild[i] != 0) continue;
        const uint32_t b = c.begin[i], e = b + c.count[i];
        for (uint32_t j = b; j < e; ++j) leafof[j] = i;
    }
}

__global__ __launch_bounds__(256) void k_usort(const float *__restrict__ u,
                                               const uint32_t *__restrict__ cid, uint32_t n,
                                               float4 *__restrict__ us) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const size_t p = cid[i];
    us[i] = make_float4(u[3 * p], u[3 * p + 1], u[3 * p + 2], 0.f);
}

// Zero `copies` copies (copy k at k * stride) of F fields of cnt entries each
// (field q at q * fs; cnt = the cell count of the current tree when ls is
// given, at most `lim`).
__global__ __launch_bounds__(256) void k_zero_xcd(double *p, uint64_t cnt, uint32_t F,
                                                  uint64_t fs, uint64_t stride, uint32_t copies,
                                                  const uint32_t *ls, uint64_t lim) {
    if (ls) cnt = ls[kLevels] < lim ? ls[kLevels] : lim;
    const uint64_t total = cnt * F;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * 256) {
        const uint64_t q = i / cnt, e = i - q * cnt;
        for (uint32_t k = 0; k < copies; ++k) p[q * fs + e + k * stride] = 0.0;
    }
}


// Fold the kXcd copies (same layout as k_zero_xcd) into copy 0.
__global__ __launch_bounds__(256) void k_fold_xcd(double *p, uint64_t cnt, uint32_t F,
                                                  uint64_t fs, uint64_t stride,
                                                  const uint32_t *ls) {
    if (ls) cnt = ls[kLevels];
    const uint64_t total = cnt * F;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * 256) {
        const uint64_t q = i / cnt, e = i - q * cnt, o = q * fs + e;
        double v = p[o];
#pragma unroll
        for (uint32_t k = 1; k < kXcd; ++k) v += p[o + k * stride];
        p[o] = v;
    }
}

// Add the kHotCopies copies of the first kHotCells cells' adjoints (copy k at
// k * kHotCopy, field q at q * kHotField) to copy 0 of the cell accumulators
// (field q of cell c at q * cap + c).
__global__ __launch_bounds__(256) void k_fold_hot(const double *__restrict__ hot, double *lcell,
                                                  uint64_t cap, const uint32_t *ls) {
    const uint32_t nc = ls[kLevels] < kHotCells ? ls[kLevels] : kHotCells;
    const uint32_t total = nc * 10u;
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < total; i += gridDim.x * 256) {
        const uint32_t q = i / nc, e = i - q * nc;
        const double *h = hot + q * kHotField + e;
        double v = 0.0;
        for (uint32_t k = 0; k < kHotCopies; ++k) v += h[k * kHotCopy];
        lcell[q * cap + e] += v;
    }
}


// Each particle adds the adjoints of the cells holding it (its leaf and the
// leaf's ancestors), then the total is scaled and added to the caller-order
// outputs.
__global__ __launch_bounds__(256) void k_moments_vjp(Cells c, const float4 *__restrict__ xyzm,
                                                     const uint32_t *__restrict__ leafof,
                                                     const uint32_t *__restrict__ cid,
                                                     const double *__restrict__ lcell,
                                                     const double *__restrict__ gsrc,
                                                     uint64_t cap, uint64_t nmax, uint32_t n,
                                                     float coef, float *g_pos, float *g_mass) {
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const float4 p = xyzm[k];
    const double xk = p.x, yk = p.y, zk = p.z, mk = p.w;
    double gx = gsrc[k], gy = gsrc[k + nmax], gz = gsrc[k + 2 * nmax], gm = gsrc[k + 3 * nmax];
    for (uint32_t cc = leafof[k]; cc != kNone; cc = c.parent[cc]) {
        const double *l = lcell + cc;
        const double lM = l[0], lx = l[cap], ly = l[2 * cap], lz = l[3 * cap];
        const double qxx = l[4 * cap], qyy = l[5 * cap], qzz = l[6 * cap], qxy = l[7 * cap],
                     qxz = l[8 * cap], qyz = l[9 * cap];
        const double M = c.M[cc];
        const double sx = xk - c.S[3 * (size_t)cc] / M, sy = yk - c.S[3 * (size_t)cc + 1] / M,
                     sz = zk - c.S[3 * (size_t)cc + 2] / M;
        const double Lx = 2.0 * qxx * sx + qxy * sy + qxz * sz;
        const double Ly = qxy * sx + 2.0 * qyy * sy + qyz * sz;
        const double Lz = qxz * sx + qyz * sy + 2.0 * qzz * sz;
        const double f = mk / M;
        gx += f * lx + mk * Lx;
        gy += f * ly + mk * Ly;
        gz += f * lz + mk * Lz;
        const double sLs = qxx * sx * sx + qyy * sy * sy + qzz * sz * sz + qxy * sx * sy +
                           qxz * sx * sz + qyz * sy * sz;
        gm += lM + (lx * sx + ly * sy + lz * sz) / M + sLs;
    }
    const size_t o = cid[k];
    if (g_pos) {
        g_pos[3 * o] += (float)(coef * gx);
        g_pos[3 * o + 1] += (float)(coef * gy);
        g_pos[3 * o + 2] += (float)(coef * gz);
    }
    if (g_mass) g_mass[o] += (float)(coef * gm);
}

__global__ void k_reset_work_vjp(uint32_t *work) {
    if (threadIdx.x < 8) work[threadIdx.x] = 0u;
}

void launch_walk_vjp(bh_ctx *c, float eps, const float *u, float coef, float *g_pos,
                     float *g_mass, hipStream_t st) {
    const uint32_t n = (uint32_t)c->n;
    const uint32_t nb = cdiv(n, 256);
    const uint32_t grid = nb < 4096u ? (nb ? nb : 1u) : 4096u;
    const uint64_t cap = (uint64_t)c->cap_cells, nmax = (uint64_t)c->nmax;
    const uint64_t lstride = 10ull * cap, gstride = 4ull * nmax;
    const uint32_t *ls = c->cells.ls;
    hipLaunchKernelGGL(k_zero_xcd, dim3(2048), dim3(256), 0, st, c->lcell, (uint64_t)0, 10u, cap,
                       lstride, kXcd, ls, cap);
    hipLaunchKernelGGL(k_zero_xcd, dim3(grid), dim3(256), 0, st, c->gsrc, (uint64_t)n, 4u, nmax,
                       gstride, kXcd, (const uint32_t *)nullptr, (uint64_t)n);
    hipLaunchKernelGGL(k_zero_xcd, dim3(640), dim3(256), 0, st, c->lhot, (uint64_t)0, 10u,
                       kHotField, kHotCopy, kHotCopies, ls, (uint64_t)kHotCells);
    hipLaunchKernelGGL(k_leafof, dim3(kGrid * 2), dim3(256), 0, st, c->cells, c->leafof);
    hipLaunchKernelGGL(k_usort, dim3(nb), dim3(256), 0, st, u,
                       (const uint32_t *)c->st[c->cur].cid, n, c->usort);
    VjpArgs a;
    a.xyzm = c->xyzm; a.u = c->usort;
    a.wA = c->cells.wA; a.wN = c->cells.wN;
    a.P0 = c->cells.P0; a.P1 = c->cells.P1; a.P2 = c->cells.P2;
    a.gbeg = c->groups.begin; a.ngroups = c->groups.count_dev;
    a.work = c->work; a.spill = c->spill; a.status = c->status;
    a.ring = c->walk_small_stack ? 192u : (uint32_t)kRing;
    a.lcell = c->lcell; a.gsrc = c->gsrc; a.lhot = c->lhot;
    a.lstride = lstride; a.gstride = gstride;
    a.cap = cap; a.nmax = nmax;
    a.eps2 = eps * eps;
    hipLaunchKernelGGL(k_reset_work_vjp, dim3(1), dim3(64), 0, st, c->work);
    record_event(c, 8, st);
    if (eps == 0.f)
        hipLaunchKernelGGL(k_walk_vjp<true>, dim3(c->walk_grid), dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL(k_walk_vjp<false>, dim3(c->walk_grid), dim3(64), 0, st, a);
    record_event(c, 9, st);
    hipLaunchKernelGGL(k_fold_xcd, dim3(2048), dim3(256), 0, st, c->lcell, (uint64_t)0, 10u, cap,
                       lstride, ls);
    hipLaunchKernelGGL(k_fold_hot, dim3(640), dim3(256), 0, st, (const double *)c->lhot, c->lcell,
                       cap, ls);
    hipLaunchKernelGGL(k_fold_xcd, dim3(grid), dim3(256), 0, st, c->gsrc, (uint64_t)n, 4u, nmax,
                       gstride, (const uint32_t *)nullptr);
    hipLaunchKernelGGL(k_moments_vjp, dim3(nb), dim3(256), 0, st, c->cells,
                       (const float4 *)c->xyzm, (const uint32_t *)c->leafof,
                       (const uint32_t *)c->st[c->cur].cid, (const double *)c->lcell,
                       (const double *)c->gsrc, cap, nmax, n, coef, g_pos, g_mass);
}

// y += a x over n [3]-vectors (the drift's transpose in the adjoint step)
__global__ __launch_bounds__(256) void k_axpy3(const float *__restrict__ x, float *y, float a,
                                               uint32_t n3) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < n3) y[i] = fmaf(a, x[i], y[i]);
}

void launch_axpy3(const float *x, float *y, float a, uint32_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_axpy3, dim3(cdiv(3ull * n, 256)), dim3(256), 0, st, x, y, a, 3u * n);
}

}  // namespace bh
