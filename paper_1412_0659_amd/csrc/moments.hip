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
// with contraction off, so the result does not depend on the launch.  Leaves
// first, then internal cells level by level from the deepest.  The walk
// reads FP32 copies: com and the opening radius
// r_open = l / theta + |com - geometric centre| (l = cell size) for the
// opening test, and (com, M, -3 Q, tr Q / 2, -3 tr Q / 2) for the
// particle-cell terms.
#include "bh_internal.h"

namespace bh {

// Leaves of at most kStage particles are read once into registers (the loads
// issue together instead of one trip at a time) and summed from there; larger
// leaves (nleaf > kStage, or the deepest level) read their particles twice.
// The sums run in the same order either way.
constexpr uint32_t kStage = 16;

__global__ __launch_bounds__(256) void k_moments_leaf(Cells c, const float *__restrict__ x,
                                                      const float *__restrict__ y,
                                                      const float *__restrict__ z,
                                                      const float *__restrict__ m) {
    uint32_t nc = c.ls[kLevels];
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nc; i += gridDim.x * 256) {
        if (c.nchild[i] != 0) continue;
        const uint32_t b = c.begin[i], cnt = c.count[i], e = b + cnt;
        double mm = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
        double q0 = 0, q1 = 0, q2 = 0, q3 = 0, q4 = 0, q5 = 0;
        double c0, c1, c2;
        if (cnt <= kStage) {
            float px[kStage], py[kStage], pz[kStage], pm[kStage];
#pragma unroll
            for (uint32_t k = 0; k < kStage; ++k) {
                const uint32_t j = k < cnt ? b + k : b;
                px[k] = x[j]; py[k] = y[j]; pz[k] = z[j]; pm[k] = m[j];
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
                double mj = m[j];
                mm = mm + mj;
                s0 = s0 + mj * (double)x[j];
                s1 = s1 + mj * (double)y[j];
                s2 = s2 + mj * (double)z[j];
            }
            c0 = s0 / mm; c1 = s1 / mm; c2 = s2 / mm;
            for (uint32_t j = b; j < e; ++j) {
                double mj = m[j];
                double d0 = (double)x[j] - c0, d1 = (double)y[j] - c1, d2 = (double)z[j] - c2;
                q0 = q0 + (mj * d0) * d0;
                q1 = q1 + (mj * d1) * d1;
                q2 = q2 + (mj * d2) * d2;
                q3 = q3 + (mj * d0) * d1;
                q4 = q4 + (mj * d0) * d2;
                q5 = q5 + (mj * d1) * d2;
            }
        }
        c.M[i] = mm;
        c.S[3 * i] = s0; c.S[3 * i + 1] = s1; c.S[3 * i + 2] = s2;
        c.com[3 * i] = c0; c.com[3 * i + 1] = c1; c.com[3 * i + 2] = c2;
        double *q = c.Q + 6 * (size_t)i;
        q[0] = q0; q[1] = q1; q[2] = q2; q[3] = q3; q[4] = q4; q[5] = q5;
    }
}

// A parent reads the mass and first moments of its (at most eight) children
// at once, then sums them in child order.
__device__ __forceinline__ void up_cell(const Cells &c, uint32_t i) {
    const uint32_t nch = c.nchild[i];
    if (nch == 0) return;
    const uint32_t k0 = c.child0[i];
    double cm[8], cs0[8], cs1[8], cs2[8];
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) {
        const uint32_t j = k0 + (k < nch ? k : 0u);
        cm[k] = c.M[j]; cs0[k] = c.S[3 * j]; cs1[k] = c.S[3 * j + 1]; cs2[k] = c.S[3 * j + 2];
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
    double c0 = s0 / mm, c1 = s1 / mm, c2 = s2 / mm;
    double q0 = 0, q1 = 0, q2 = 0, q3 = 0, q4 = 0, q5 = 0;
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) {
        if (k < nch) {
            const uint32_t j = k0 + k;
            const double mk = cm[k];
            double d0 = c.com[3 * j] - c0, d1 = c.com[3 * j + 1] - c1, d2 = c.com[3 * j + 2] - c2;
            const double *qk = c.Q + 6 * (size_t)j;
            q0 = q0 + (qk[0] + (mk * d0) * d0);
            q1 = q1 + (qk[1] + (mk * d1) * d1);
            q2 = q2 + (qk[2] + (mk * d2) * d2);
            q3 = q3 + (qk[3] + (mk * d0) * d1);
            q4 = q4 + (qk[4] + (mk * d0) * d2);
            q5 = q5 + (qk[5] + (mk * d1) * d2);
        }
    }
    c.M[i] = mm;
    c.S[3 * i] = s0; c.S[3 * i + 1] = s1; c.S[3 * i + 2] = s2;
    c.com[3 * i] = c0; c.com[3 * i + 1] = c1; c.com[3 * i + 2] = c2;
    double *q = c.Q + 6 * (size_t)i;
    q[0] = q0; q[1] = q1; q[2] = q2; q[3] = q3; q[4] = q4; q[5] = q5;
}

__global__ __launch_bounds__(256) void k_moments_up(Cells c, int l) {
    uint32_t first = c.ls[l], last = c.ls[l + 1];
    for (uint32_t i = first + blockIdx.x * 256 + threadIdx.x; i < last; i += gridDim.x * 256)
        up_cell(c, i);
}

// Levels 20 down to l1 in one workgroup (the deep end of the tree, few or no
// internal cells), the same per-cell sums as k_moments_up.
__global__ __launch_bounds__(1024) void k_moments_tail(Cells c, int l1) {
    for (int l = kLevels - 2; l >= l1; --l) {
        const uint32_t first = c.ls[l], last = c.ls[l + 1];
        for (uint32_t i = first + threadIdx.x; i < last; i += 1024) up_cell(c, i);
        __syncthreads();  // the next level up reads these cells
    }
}

// corner coordinates of a cell from its key prefix (x the high bit of each digit)
__device__ __forceinline__ void cell_coords(uint64_t prefix, uint32_t lev, uint32_t p[3]) {
    uint32_t a = 0, b = 0, d = 0;
    for (int s = (int)lev - 1; s >= 0; --s) {
        uint32_t dig = (uint32_t)(prefix >> (3 * s)) & 7u;
        a = (a << 1) | (dig >> 2);
        b = (b << 1) | ((dig >> 1) & 1u);
        d = (d << 1) | (dig & 1u);
    }
    p[0] = a; p[1] = b; p[2] = d;
}

__global__ __launch_bounds__(256) void k_moments_final(Cells c, const float *__restrict__ box,
                                                       int curve) {
    uint32_t nc = c.ls[kLevels];
    double lo0 = box[0], lo1 = box[1], lo2 = box[2], side = box[3];
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nc; i += gridDim.x * 256) {
        uint32_t lev = c.level[i];
        uint32_t p[3];
        cell_coords(c.prefix[i], lev, p);     // the digits, deinterleaved
        if (curve == 1) ph_decode(p, (int)lev);  // Peano-Hilbert prefix -> octant
        double lc = side * (1.0 / (double)(1u << lev));
        double c0 = c.com[3 * i], c1 = c.com[3 * i + 1], c2 = c.com[3 * i + 2];
        double e0 = c0 - (lo0 + ((double)p[0] + 0.5) * lc);
        double e1 = c1 - (lo1 + ((double)p[1] + 0.5) * lc);
        double e2 = c2 - (lo2 + ((double)p[2] + 0.5) * lc);
        double dl = __dsqrt_rn((e0 * e0 + e1 * e1) + e2 * e2);
        const double *q = c.Q + 6 * (size_t)i;
        double tr = (q[0] + q[1]) + q[2];
        c.wA[i] = make_float4((float)c0, (float)c1, (float)c2, 0.f);
        c.P0[i] = make_float4((float)c0, (float)c1, (float)c2, (float)c.M[i]);
        c.P1[i] = make_float4((float)(-3.0 * q[0]), (float)(-3.0 * q[1]), (float)(-3.0 * q[2]),
                              (float)(-3.0 * q[3]));
        c.P2[i] = make_float4((float)(-3.0 * q[4]), (float)(-3.0 * q[5]), (float)(0.5 * tr),
                              (float)(-1.5 * tr));
        uint32_t nch = c.nchild[i];
        c.wN[i] = nch ? make_uint2(c.child0[i], nch) : make_uint2(c.begin[i], c.count[i] | kLeafBit);
        c.size[i] = make_float2((float)lc, (float)dl);
    }
}

// Internal cells of levels grid_levels .. 20 by k_moments_tail, the levels
// above by one grid launch each.
void launch_moments(bh_ctx *ctx, hipStream_t st, int grid_levels) {
    const State &s = ctx->st[ctx->cur];
    Cells &c = ctx->cells;
    hipLaunchKernelGGL(k_moments_leaf, dim3(kGrid * 2), dim3(256), 0, st, c,
                       (const float *)s.x, (const float *)s.y, (const float *)s.z,
                       (const float *)s.m);
    const int L = grid_levels < 0 ? 0 : (grid_levels > kLevels - 1 ? kLevels - 1 : grid_levels);
    if (L < kLevels - 1) hipLaunchKernelGGL(k_moments_tail, dim3(1), dim3(1024), 0, st, c, L);
    for (int l = L - 1; l >= 0; --l)
        hipLaunchKernelGGL(k_moments_up, dim3(kGrid), dim3(256), 0, st, c, l);
    hipLaunchKernelGGL(k_moments_final, dim3(kGrid * 2), dim3(256), 0, st, c,
                       (const float *)ctx->box, (int)ctx->p.curve);
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
