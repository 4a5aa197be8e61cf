// Particle state in and out of the sorted layout, the leapfrog kicks and
// drift (Sec. III.B.2: second-order leap-frog after the forces), and the
// interaction totals of a walk (Sec. VI.A: flops = 23 per particle-particle
// and 65 per particle-cell interaction, counted during execution).
#include "bh_internal.h"
#include "wave.h"

namespace bh {

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, uint32_t v, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * 256)
        p[i] = v;
}

void launch_fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t st) {
    uint32_t nb = cdiv(n, 256);
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_fill_u32, dim3(nb), dim3(256), 0, st, p, v, n);
}

// caller [n][3] positions / velocities and [n] masses -> state (caller order)
__global__ __launch_bounds__(256) void k_ingest(const float *__restrict__ pos,
                                                const float *__restrict__ vel,
                                                const float *__restrict__ mass, uint32_t n,
                                                State s, uint32_t *status) {
    uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float px = pos[3 * (size_t)i], py = pos[3 * (size_t)i + 1], pz = pos[3 * (size_t)i + 2];
    s.x[i] = px;
    s.y[i] = py;
    s.z[i] = pz;
    if (s.x64) {
        s.x64[i] = px;
        s.y64[i] = py;
        s.z64[i] = pz;
    }
    float mi = mass[i];
    s.m[i] = mi;
    if (!(mi > 0.f) || !isfinite(mi)) atomicOr(status, kStMass);
    if (vel) {
        float a = vel[3 * (size_t)i], b = vel[3 * (size_t)i + 1], c = vel[3 * (size_t)i + 2];
        if (!(isfinite(a) && isfinite(b) && isfinite(c))) atomicOr(status, kStNonFinite);
        s.vx[i] = a;
        s.vy[i] = b;
        s.vz[i] = c;
    } else {
        s.vx[i] = 0.f;
        s.vy[i] = 0.f;
        s.vz[i] = 0.f;
    }
    s.cid[i] = i;
}

void launch_ingest(bh_ctx *c, const float *pos, const float *vel, const float *mass, uint32_t n,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_ingest, dim3(cdiv(n, 256)), dim3(256), 0, st, pos, vel, mass, n,
                       c->st[c->cur], c->status);
}

// v += a h
__global__ __launch_bounds__(256) void k_kick(State s, const float4 *__restrict__ acc, uint32_t n,
                                              float h) {
    uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float4 a = acc[i];
    s.vx[i] = fmaf(a.x, h, s.vx[i]);
    s.vy[i] = fmaf(a.y, h, s.vy[i]);
    s.vz[i] = fmaf(a.z, h, s.vz[i]);
}

// v += a h; x += v dt.  With an FP64 master copy the drift is done in FP64
// and the FP32 positions the tree is built from are its rounding.
__global__ __launch_bounds__(256) void k_kick_drift(State s, const float4 *__restrict__ acc,
                                                    uint32_t n, float h, float dt) {
    uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float4 a = acc[i];
    float vx = fmaf(a.x, h, s.vx[i]), vy = fmaf(a.y, h, s.vy[i]), vz = fmaf(a.z, h, s.vz[i]);
    s.vx[i] = vx;
    s.vy[i] = vy;
    s.vz[i] = vz;
    if (s.x64) {
        const double d = dt;
        const double x = fma((double)vx, d, s.x64[i]), y = fma((double)vy, d, s.y64[i]),
                     z = fma((double)vz, d, s.z64[i]);
        s.x64[i] = x;
        s.y64[i] = y;
        s.z64[i] = z;
        s.x[i] = (float)x;
        s.y[i] = (float)y;
        s.z[i] = (float)z;
    } else {
        s.x[i] = fmaf(vx, dt, s.x[i]);
        s.y[i] = fmaf(vy, dt, s.y[i]);
        s.z[i] = fmaf(vz, dt, s.z[i]);
    }
}

void launch_kick(bh_ctx *c, float h, uint32_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_kick, dim3(cdiv(n, 256)), dim3(256), 0, st, c->st[c->cur],
                       (const float4 *)c->acc, n, h);
}

void launch_kick_drift(bh_ctx *c, float h, float dt, uint32_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_kick_drift, dim3(cdiv(n, 256)), dim3(256), 0, st, c->st[c->cur],
                       (const float4 *)c->acc, n, h, dt);
}

// sorted acceleration + potential -> caller order (rows: output row of each
// caller index, or null for the identity)
__global__ __launch_bounds__(256) void k_unsort(const float4 *__restrict__ acc,
                                                const uint32_t *__restrict__ cid, uint32_t n,
                                                const uint32_t *__restrict__ rows,
                                                float *__restrict__ out_acc,
                                                float *__restrict__ out_pot) {
    uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float4 a = acc[i];
    uint32_t p = cid[i];
    if (rows) p = rows[p];
    if (out_acc) {
        out_acc[3 * (size_t)p] = a.x;
        out_acc[3 * (size_t)p + 1] = a.y;
        out_acc[3 * (size_t)p + 2] = a.z;
    }
    if (out_pot) out_pot[p] = a.w;
}

// sorted acceleration + potential added to caller-order outputs
__global__ __launch_bounds__(256) void k_unsort_add(const float4 *__restrict__ acc,
                                                    const uint32_t *__restrict__ cid, uint32_t n,
                                                    float *__restrict__ out_acc,
                                                    float *__restrict__ out_pot) {
    uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float4 a = acc[i];
    uint32_t p = cid[i];
    if (out_acc) {
        out_acc[3 * (size_t)p] += a.x;
        out_acc[3 * (size_t)p + 1] += a.y;
        out_acc[3 * (size_t)p + 2] += a.z;
    }
    if (out_pot) out_pot[p] += a.w;
}

void launch_unsort_add(bh_ctx *c, float *acc, float *pot, uint32_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_unsort_add, dim3(cdiv(n, 256)), dim3(256), 0, st,
                       (const float4 *)c->acc, (const uint32_t *)c->st[c->cur].cid, n, acc, pot);
}

void launch_unsort(bh_ctx *c, float *acc, float *pot, uint32_t n, hipStream_t st,
                   const uint32_t *rows) {
    hipLaunchKernelGGL(k_unsort, dim3(cdiv(n, 256)), dim3(256), 0, st, (const float4 *)c->acc,
                       (const uint32_t *)c->st[c->cur].cid, n, rows, acc, pot);
}

__global__ __launch_bounds__(256) void k_state_out(State s, uint32_t n, float *__restrict__ pos,
                                                   float *__restrict__ vel) {
    uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    uint32_t p = s.cid[i];
    if (pos) {
        pos[3 * (size_t)p] = s.x[i];
        pos[3 * (size_t)p + 1] = s.y[i];
        pos[3 * (size_t)p + 2] = s.z[i];
    }
    if (vel) {
        vel[3 * (size_t)p] = s.vx[i];
        vel[3 * (size_t)p + 1] = s.vy[i];
        vel[3 * (size_t)p + 2] = s.vz[i];
    }
}

void launch_state_out(bh_ctx *c, float *pos, float *vel, uint32_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_state_out, dim3(cdiv(n, 256)), dim3(256), 0, st, c->st[c->cur], n, pos,
                       vel);
}

// sorted slots [lo, lo + cnt) -> packed outputs in sorted order: the
// particles of one domain of the curve
__global__ __launch_bounds__(256) void k_range_out(State s, uint32_t lo, uint32_t cnt,
                                                   float *__restrict__ pos,
                                                   float *__restrict__ vel,
                                                   float *__restrict__ mass,
                                                   uint32_t *__restrict__ ids) {
    uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= cnt) return;
    uint32_t i = lo + k;
    if (pos) {
        pos[3 * (size_t)k] = s.x[i];
        pos[3 * (size_t)k + 1] = s.y[i];
        pos[3 * (size_t)k + 2] = s.z[i];
    }
    if (vel) {
        vel[3 * (size_t)k] = s.vx[i];
        vel[3 * (size_t)k + 1] = s.vy[i];
        vel[3 * (size_t)k + 2] = s.vz[i];
    }
    if (mass) mass[k] = s.m[i];
    if (ids) ids[k] = s.cid[i];
}

void launch_range_out(bh_ctx *c, uint32_t lo, uint32_t cnt, float *pos, float *vel, float *mass,
                      uint32_t *ids, hipStream_t st) {
    hipLaunchKernelGGL(k_range_out, dim3(cdiv(cnt, 256)), dim3(256), 0, st, c->st[c->cur], lo,
                       cnt, pos, vel, mass, ids);
}

// Conserved quantities of the state, FP64: total mass, kinetic energy,
// potential energy 1/2 sum m phi (phi of the last force evaluation, which
// excludes the self pair), momentum and angular momentum about the origin
// (positions as held: the FP64 master copy when kept).  Each block writes
// its partial sums; one wave folds them in block order, so the result does
// not depend on scheduling.
__global__ __launch_bounds__(256) void k_diag_partial(State s, const float4 *__restrict__ acc,
                                                      uint32_t n, double *part) {
    double v[kDiagN];
#pragma unroll
    for (int k = 0; k < kDiagN; ++k) v[k] = 0.0;
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const double m = s.m[i];
        const double x = s.x64 ? s.x64[i] : (double)s.x[i];
        const double y = s.x64 ? s.y64[i] : (double)s.y[i];
        const double z = s.x64 ? s.z64[i] : (double)s.z[i];
        const double vx = s.vx[i], vy = s.vy[i], vz = s.vz[i];
        v[0] += m;
        v[1] += 0.5 * m * (vx * vx + vy * vy + vz * vz);
        v[2] += 0.5 * m * (double)acc[i].w;
        v[3] += m * vx;
        v[4] += m * vy;
        v[5] += m * vz;
        v[6] += m * (y * vz - z * vy);
        v[7] += m * (z * vx - x * vz);
        v[8] += m * (x * vy - y * vx);
    }
    __shared__ double lds[4][kDiagN];
#pragma unroll
    for (int k = 0; k < kDiagN; ++k) {
        double t = v[k];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) t += __shfl_xor(t, d, 64);
        if (lane_id() == 0) lds[threadIdx.x >> 6][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < kDiagN)
        part[(size_t)blockIdx.x * kDiagN + threadIdx.x] =
            ((lds[0][threadIdx.x] + lds[1][threadIdx.x]) + lds[2][threadIdx.x]) + lds[3][threadIdx.x];
}

__global__ void k_diag_final(const double *__restrict__ part, uint32_t nb, double *out) {
    const uint32_t k = threadIdx.x;
    if (k >= (uint32_t)kDiagN) return;
    double t = 0.0;
    for (uint32_t b = 0; b < nb; ++b) t += part[(size_t)b * kDiagN + k];
    out[k] = t;
}

void launch_diagnostics(bh_ctx *c, hipStream_t st) {
    const uint32_t n = (uint32_t)c->n;
    uint32_t nb = cdiv(n, 256);
    if (nb > (uint32_t)kDiagBlocks) nb = kDiagBlocks;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_diag_partial, dim3(nb), dim3(256), 0, st, c->st[c->cur],
                       (const float4 *)c->acc, n, c->diag);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, st, (const double *)c->diag, nb,
                       c->diag + (size_t)kDiagBlocks * kDiagN);
}

// sum over groups of npp * size and npc * size (integers: order-free)
__global__ __launch_bounds__(256) void k_totals(const uint32_t *__restrict__ gbeg,
                                                const uint32_t *__restrict__ ngroups,
                                                const uint32_t *__restrict__ npp,
                                                const uint32_t *__restrict__ npc,
                                                unsigned long long *tot) {
    uint32_t ng = *ngroups;
    unsigned long long spp = 0, spc = 0;
    for (uint32_t g = blockIdx.x * 256 + threadIdx.x; g < ng; g += gridDim.x * 256) {
        unsigned long long sz = gbeg[g + 1] - gbeg[g];
        spp += sz * npp[g];
        spc += sz * npc[g];
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        spp += __shfl_xor(spp, d, 64);
        spc += __shfl_xor(spc, d, 64);
    }
    // one pair of atomics per block: the counters are shared by every block
    __shared__ unsigned long long part[4][2];
    const uint32_t w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        part[w][0] = spp;
        part[w][1] = spc;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        unsigned long long v = part[0][threadIdx.x] + part[1][threadIdx.x] +
                               part[2][threadIdx.x] + part[3][threadIdx.x];
        atomicAdd(&tot[threadIdx.x], v);
    }
}

// number of leaf cells of the tree into tot[2]
__global__ __launch_bounds__(256) void k_count_leaves(Cells c, unsigned long long *tot) {
    const uint32_t nc = c.ls[kLevels];
    unsigned long long k = 0;
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < nc; i += gridDim.x * 256)
        k += c.nchild[i] == 0u;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) k += __shfl_xor(k, d, 64);
    if (lane_id() == 0) atomicAdd(&tot[2], k);
}

__global__ void k_zero_leaves(unsigned long long *tot) {
    if (threadIdx.x == 0) tot[2] = 0ull;
}

void launch_count_leaves(bh_ctx *c, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_leaves, dim3(1), dim3(64), 0, st, c->totals);
    hipLaunchKernelGGL(k_count_leaves, dim3(512), dim3(256), 0, st, c->cells, c->totals);
}

__global__ void k_zero_totals(unsigned long long *tot) {
    if (threadIdx.x < 2) tot[threadIdx.x] = 0ull;
}

void launch_totals(bh_ctx *c, uint32_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_totals, dim3(1), dim3(64), 0, st, c->totals);
    uint32_t nb = cdiv(n, 256 * 64);
    if (nb > 256) nb = 256;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_totals, dim3(nb), dim3(256), 0, st, (const uint32_t *)c->groups.begin,
                       (const uint32_t *)c->groups.count_dev, (const uint32_t *)c->groups.npp,
                       (const uint32_t *)c->groups.npc, c->totals);
}

}  // namespace bh
