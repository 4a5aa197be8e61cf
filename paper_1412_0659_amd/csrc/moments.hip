// Upward pass: mass, centre of mass and quadrupole of every cell in FP64
// (Sec. I.A: multipole moments computed once the tree is built; Sec. VI.A
// Eq. (1): the quadrupole is the 3x3 second moment of the cell's mass about
// its centre of mass; Table II "Tree-properties").
//
//   leaf:   M = sum m, S = sum m x, com = S / M, Q = sum m s s^T, s = x - com
//   parent: M = sum M_c, S = sum S_c, com = S / M,
//           Q = sum (Q_c + M_c d d^T), d = com_c - com   (parallel axis)
//
// Each cell is one thread summing in a fixed order (a leaf over its
// particles in sorted order, a parent over its children in child order),
// with contraction off, so the result does not depend on the launch.  Level
// by level from the deepest, leaves and parents of a level in one pass that
// also writes the cell's walk records.  The FP64 record of a cell is M, S
// and Q (80 bytes, read once more by its parent); com = S / M is recomputed
// where needed.  The walk reads FP32 copies: com and the opening radius
// r_open = l / theta + |com - geometric centre| (l = cell size) for the
// opening test, and (com, M, -3 Q, tr Q / 2, -3 tr Q / 2) for the
// particle-cell terms.
#include "bh_internal.h"

namespace bh {

// Leaves of at most kStage particles are read once into registers (the loads
// issue together instead of one trip at a time) and summed from there; larger
// leaves (nleaf > kStage) and the leaves of the single-workgroup tail read
// their particles twice.  The sums run in the same order either way.
constexpr uint32_t kStage = 16;

struct MomArgs {
    Cells c;
    const float *x, *y, *z, *m;
    const float4 *xyzm;  // the same particles as (x, y, z, m) records, one load each
    const float *box;  // lo xyz, side
    int curve;
};

struct Mom {
    double M, s0, s1, s2, q0, q1, q2, q3, q4, q5;
};

template <bool kStaged>
__device__ __forceinline__ void leaf_sums(const MomArgs &a, uint32_t b, uint32_t cnt, Mom &r,
                                          double &c0, double &c1, double &c2) {
    const uint32_t e = b + cnt;
    double mm = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
    double q0 = 0, q1 = 0, q2 = 0, q3 = 0, q4 = 0, q5 = 0;
    if (kStaged && cnt <= kStage) {
        float px[kStage], py[kStage], pz[kStage], pm[kStage];
#pragma unroll
        for (uint32_t k = 0; k < kStage; ++k) {
            const float4 p = a.xyzm[k < cnt ? b + k : b];
            px[k] = p.x; py[k] = p.y; pz[k] = p.z; pm[k] = p.w;
        }
#pragma unroll
        for (uint32_t k = 0; k < kStage; ++k) {
            if (k < cnt) {
                const double mj = pm[k];
                mm = mm + mj;
                s0 = s0 + mj * (double)px[k];
                s1 = s1 + mj * (double)py[k];
                s2 = s2 + mj * (double)pz[k];
            }
        }
        c0 = s0 / mm; c1 = s1 / mm; c2 = s2 / mm;
#pragma unroll
        for (uint32_t k = 0; k < kStage; ++k) {
            if (k < cnt) {
                const double mj = pm[k];
                const double d0 = (double)px[k] - c0, d1 = (double)py[k] - c1,
                             d2 = (double)pz[k] - c2;
                q0 = q0 + (mj * d0) * d0;
                q1 = q1 + (mj * d1) * d1;
                q2 = q2 + (mj * d2) * d2;
                q3 = q3 + (mj * d0) * d1;
                q4 = q4 + (mj * d0) * d2;
                q5 = q5 + (mj * d1) * d2;
            }
        }
    } else {
        for (uint32_t j = b; j < e; ++j) {
            double mj = a.m[j];
            mm = mm + mj;
            s0 = s0 + mj * (double)a.x[j];
            s1 = s1 + mj * (double)a.y[j];
            s2 = s2 + mj * (double)a.z[j];
        }
        c0 = s0 / mm; c1 = s1 / mm; c2 = s2 / mm;
        for (uint32_t j = b; j < e; ++j) {
            double mj = a.m[j];
            double d0 = (double)a.x[j] - c0, d1 = (double)a.y[j] - c1, d2 = (double)a.z[j] - c2;
            q0 = q0 + (mj * d0) * d0;
            q1 = q1 + (mj * d1) * d1;
            q2 = q2 + (mj * d2) * d2;
            q3 = q3 + (mj * d0) * d1;
            q4 = q4 + (mj * d0) * d2;
            q5 = q5 + (mj * d1) * d2;
        }
    }
    r = Mom{mm, s0, s1, s2, q0, q1, q2, q3, q4, q5};
}

// A parent reads the mass, first and second moments (and with kStaged the
// quadrupoles) of its (at most eight) children at once, then sums them in
// child order; a child's centre of mass is its S / M, the same division that
// made it.
template <bool kStaged>
__device__ __forceinline__ void parent_sums(const Cells &c, uint32_t k0, uint32_t nch, Mom &r,
                                            double &c0, double &c1, double &c2) {
    double cm[8], cs0[8], cs1[8], cs2[8];
    double2 cq[8][3];  // the six quadrupole entries as three 16-byte loads
    const double2 *Q2 = reinterpret_cast<const double2 *>(c.Q);  // 16-byte aligned
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) {
        const uint32_t j = k0 + (k < nch ? k : 0u);
        cm[k] = c.M[j]; cs0[k] = c.S[3 * j]; cs1[k] = c.S[3 * j + 1]; cs2[k] = c.S[3 * j + 2];
        if (kStaged) {
            cq[k][0] = Q2[3 * (size_t)j]; cq[k][1] = Q2[3 * (size_t)j + 1];
            cq[k][2] = Q2[3 * (size_t)j + 2];
        }
    }
    double mm = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) {
        if (k < nch) {
            mm = mm + cm[k];
            s0 = s0 + cs0[k];
            s1 = s1 + cs1[k];
            s2 = s2 + cs2[k];
        }
    }
    c0 = s0 / mm; c1 = s1 / mm; c2 = s2 / mm;
    double q0 = 0, q1 = 0, q2 = 0, q3 = 0, q4 = 0, q5 = 0;
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) {
        if (k < nch) {
            const double mk = cm[k];
            const double d0 = cs0[k] / mk - c0, d1 = cs1[k] / mk - c1, d2 = cs2[k] / mk - c2;
            const size_t j = k0 + k;
            const double2 qa = kStaged ? cq[k][0] : Q2[3 * j], qb = kStaged ? cq[k][1] : Q2[3 * j + 1],
                          qc = kStaged ? cq[k][2] : Q2[3 * j + 2];
            q0 = q0 + (qa.x + (mk * d0) * d0);
            q1 = q1 + (qa.y + (mk * d1) * d1);
            q2 = q2 + (qb.x + (mk * d2) * d2);
            q3 = q3 + (qb.y + (mk * d0) * d1);
            q4 = q4 + (qc.x + (mk * d0) * d2);
            q5 = q5 + (qc.y + (mk * d1) * d2);
        }
    }
    r = Mom{mm, s0, s1, s2, q0, q1, q2, q3, q4, q5};
}

// every third bit of v (bits 0, 3, 6, ...) gathered into the low 21 bits
__device__ __forceinline__ uint32_t every_third_bit(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10C30C30C30C30C3ull;
    v = (v ^ (v >> 4)) & 0x100F00F00F00F00Full;
    v = (v ^ (v >> 8)) & 0x001F0000FF0000FFull;
    v = (v ^ (v >> 16)) & 0x001F00000000FFFFull;
    v = (v ^ (v >> 32)) & 0x00000000001FFFFFull;
    return (uint32_t)v;
}

// corner coordinates of a cell from its key prefix (x the high bit of each
// 3-bit digit, the first digit the most significant); lev only bounds the
// prefix, whose higher bits are zero
__device__ __forceinline__ void cell_coords(uint64_t prefix, uint32_t lev, uint32_t p[3]) {
    (void)lev;
    p[0] = every_third_bit(prefix >> 2);
    p[1] = every_third_bit(prefix >> 1);
    p[2] = every_third_bit(prefix);
}

// Cell i of level lev: its FP64 moments (M, S, Q; the centre of mass is
// S / M wherever it is needed) and its walk records.  kStaged: small leaves
// through registers (more VGPRs).
template <bool kStaged>
__device__ __forceinline__ void cell_pass(const MomArgs &a, uint32_t i, uint32_t lev) {
    const Cells &c = a.c;
    // the cell's topology in one round of loads (every field is defined for
    // every cell; child0 is only used by parents, begin and count by leaves)
    const uint32_t nch = c.nchild[i], b0 = c.begin[i], n0 = c.count[i], k0 = c.child0[i];
    const uint64_t prefix = c.prefix[i];
    Mom r;
    double c0, c1, c2;
    uint32_t first, cnt;
    if (nch == 0) {
        first = b0;
        cnt = n0;
        leaf_sums<kStaged>(a, first, cnt, r, c0, c1, c2);
    } else {
        first = k0;
        cnt = nch;
        parent_sums<kStaged>(c, first, nch, r, c0, c1, c2);
    }
    c.M[i] = r.M;
    c.S[3 * i] = r.s0; c.S[3 * i + 1] = r.s1; c.S[3 * i + 2] = r.s2;
    double2 *q = reinterpret_cast<double2 *>(c.Q) + 3 * (size_t)i;
    q[0] = make_double2(r.q0, r.q1);
    q[1] = make_double2(r.q2, r.q3);
    q[2] = make_double2(r.q4, r.q5);

    // walk records: com (FP32), opening-radius terms, particle-cell record
    const double lo0 = a.box[0], lo1 = a.box[1], lo2 = a.box[2], side = a.box[3];
    uint32_t p[3];
    cell_coords(prefix, lev, p);          // the digits, deinterleaved
    if (a.curve == 1) ph_decode(p, (int)lev);  // Peano-Hilbert prefix -> octant
    const double lc = side * (1.0 / (double)(1u << lev));
    const double e0 = c0 - (lo0 + ((double)p[0] + 0.5) * lc);
    const double e1 = c1 - (lo1 + ((double)p[1] + 0.5) * lc);
    const double e2 = c2 - (lo2 + ((double)p[2] + 0.5) * lc);
    const double dl = __dsqrt_rn((e0 * e0 + e1 * e1) + e2 * e2);
    const double tr = (r.q0 + r.q1) + r.q2;
    c.wA[i] = make_float4((float)c0, (float)c1, (float)c2, 0.f);
    c.P0[i] = make_float4((float)c0, (float)c1, (float)c2, (float)r.M);
    c.P1[i] = make_float4((float)(-3.0 * r.q0), (float)(-3.0 * r.q1), (float)(-3.0 * r.q2),
                          (float)(-3.0 * r.q3));
    c.P2[i] = make_float4((float)(-3.0 * r.q4), (float)(-3.0 * r.q5), (float)(0.5 * tr),
                          (float)(-1.5 * tr));
    c.wN[i] = nch ? make_uint2(first, cnt) : make_uint2(first, cnt | kLeafBit);
    c.size[i] = make_float2((float)lc, (float)dl);
}

__global__ __launch_bounds__(256) void k_moments_level(MomArgs a, int l) {
    const uint32_t first = a.c.ls[l], last = a.c.ls[l + 1];
    for (uint32_t i = first + blockIdx.x * 256 + threadIdx.x; i < last; i += gridDim.x * 256)
        cell_pass<true>(a, i, (uint32_t)l);
}

// Levels l0 down to l1 in one workgroup (the deep end of the tree, few or no
// cells), the same per-cell sums as k_moments_level (leaves read twice).
__global__ __launch_bounds__(1024) void k_moments_tail(MomArgs a, int l0, int l1) {
    for (int l = l0; l >= l1; --l) {
        const uint32_t first = a.c.ls[l], last = a.c.ls[l + 1];
        for (uint32_t i = first + threadIdx.x; i < last; i += 1024)
            cell_pass<false>(a, i, (uint32_t)l);
        __syncthreads();  // the next level up reads these cells
    }
}

// One pass per level from the deepest (leaves from their particles, parents
// from their children, each cell's walk records as soon as its moments are
// known): the levels above grid_levels by one grid launch each, levels 21
// down to grid_levels by k_moments_tail (level 21 by a grid launch too when
// grid_levels is 21: no recent tree said the deep levels are sparse).
void launch_moments(bh_ctx *ctx, hipStream_t st, int grid_levels) {
    const State &s = ctx->st[ctx->cur];
    MomArgs a;
    a.c = ctx->cells;
    a.x = s.x; a.y = s.y; a.z = s.z; a.m = s.m;
    a.xyzm = ctx->xyzm;
    a.box = ctx->box;
    a.curve = (int)ctx->p.curve;
    const int L = grid_levels < 0 ? 0 : (grid_levels > kLevels - 1 ? kLevels - 1 : grid_levels);
    if (L < kLevels - 1)
        hipLaunchKernelGGL(k_moments_tail, dim3(1), dim3(1024), 0, st, a, kLevels - 1, L);
    else
        hipLaunchKernelGGL(k_moments_level, dim3(kGrid), dim3(256), 0, st, a, kLevels - 1);
    for (int l = L - 1; l >= 0; --l)
        hipLaunchKernelGGL(k_moments_level, dim3(kGrid), dim3(256), 0, st, a, l);
}

// com = S / M of every cell (FP64), for export
__global__ __launch_bounds__(256) void k_com(Cells c) {
    const uint32_t nc = c.ls[kLevels];
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nc; i += gridDim.x * 256) {
        const double mm = c.M[i];
        c.com[3 * i] = c.S[3 * i] / mm;
        c.com[3 * i + 1] = c.S[3 * i + 1] / mm;
        c.com[3 * i + 2] = c.S[3 * i + 2] / mm;
    }
}

void launch_com(bh_ctx *ctx, hipStream_t st) {
    hipLaunchKernelGGL(k_com, dim3(kGrid * 2), dim3(256), 0, st, ctx->cells);
}

// r_open^2 = (fl32(l / theta) + delta)^2 in FP32, stored in wA.w
__global__ __launch_bounds__(256) void k_walk_prep(Cells c, float theta) {
    uint32_t nc = c.ls[kLevels];
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nc; i += gridDim.x * 256) {
        float2 sz = c.size[i];
        float r = sz.x / theta + sz.y;
        c.wA[i].w = r * r;
    }
}

void launch_walk_prep(bh_ctx *ctx, float theta, hipStream_t st) {
    hipLaunchKernelGGL(k_walk_prep, dim3(kGrid * 2), dim3(256), 0, st, ctx->cells, theta);
}

}  // namespace bh
