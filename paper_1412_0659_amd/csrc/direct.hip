// FP64 direct summation at chosen target particles over every particle of
// the current state: the theta -> 0 limit of the tree force (Sec. I.A), with
// Plummer softening, and the reference the error of the tree forces is
// stated against.  Positions are the FP32 values the tree is built from,
// widened exactly; every product and sum is FP64.  The self pair is skipped
// (no force, no potential); a zero-separation pair without softening has no
// finite term and is skipped too.
//
// Work split: a block of 256 lanes takes 256 targets and one span of the
// sources, staged through LDS 256 at a time; the spans of one target are
// summed with FP64 atomics, so the order of the partial sums (and the last
// bits of the result) may vary between runs.
#include "bh_internal.h"

namespace bh {

__global__ __launch_bounds__(256) void k_inverse(const uint32_t *__restrict__ cid, uint32_t n,
                                                 uint32_t *__restrict__ inv) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) inv[cid[i]] = i;
}

__global__ __launch_bounds__(256) void k_direct(const float4 *__restrict__ xyzm,
                                                const uint32_t *__restrict__ inv,
                                                const int64_t *__restrict__ tgt, uint32_t nt,
                                                uint32_t n, uint32_t span, double eps2,
                                                double *acc, double *pot,
                                                uint32_t *status) {
    __shared__ float4 src[256];
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    bool act = k < nt;
    uint32_t self = kNone;
    double tx = 0.0, ty = 0.0, tz = 0.0;
    if (act) {
        const int64_t t = tgt[k];
        if (t < 0 || t >= (int64_t)n) {
            if (blockIdx.y == 0) atomicOr(status, kStIndex);
            act = false;  // still takes part in the block's barriers
        } else {
            self = inv[t];
            const float4 p = xyzm[self];
            tx = p.x;
            ty = p.y;
            tz = p.z;
        }
    }
    const uint32_t j0 = blockIdx.y * span;
    const uint32_t j1 = j0 + span < n ? j0 + span : n;
    double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
    for (uint32_t base = j0; base < j1; base += 256) {
        const uint32_t j = base + threadIdx.x;
        __syncthreads();
        src[threadIdx.x] = j < j1 ? xyzm[j] : make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
        const uint32_t m = j1 - base < 256u ? j1 - base : 256u;
        if (!act) continue;
        for (uint32_t q = 0; q < m; ++q) {
            if (base + q == self) continue;
            const float4 s = src[q];
            const double dx = (double)s.x - tx, dy = (double)s.y - ty, dz = (double)s.z - tz;
            const double r2 = dx * dx + dy * dy + dz * dz + eps2;
            if (r2 == 0.0) continue;
            const double ri = 1.0 / sqrt(r2);
            const double mri = (double)s.w * ri;
            const double mri3 = mri * ri * ri;
            ax += mri3 * dx;
            ay += mri3 * dy;
            az += mri3 * dz;
            ph -= mri;
        }
    }
    if (act) {
        atomicAdd(acc + 3 * (size_t)k, ax);
        atomicAdd(acc + 3 * (size_t)k + 1, ay);
        atomicAdd(acc + 3 * (size_t)k + 2, az);
        atomicAdd(pot + k, ph);
    }
}

__global__ __launch_bounds__(256) void k_zero_f64(double *p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * 256)
        p[i] = 0.0;
}

void launch_direct(bh_ctx *c, const int64_t *tgt, uint32_t nt, float eps, double *acc,
                   double *pot, hipStream_t st) {
    const uint32_t n = (uint32_t)c->n;
    hipLaunchKernelGGL(k_inverse, dim3(cdiv(n, 256)), dim3(256), 0, st,
                       (const uint32_t *)c->st[c->cur].cid, n, c->inv);
    hipLaunchKernelGGL(k_zero_f64, dim3(cdiv(3ull * nt, 256)), dim3(256), 0, st, acc,
                       3ull * nt);
    hipLaunchKernelGGL(k_zero_f64, dim3(cdiv(nt, 256)), dim3(256), 0, st, pot, (uint64_t)nt);
    // enough blocks to fill the chip several times over; spans of >= 4096 sources
    const uint32_t tb = cdiv(nt, 256);
    uint32_t ns = cdiv(8192, tb);
    const uint32_t max_ns = cdiv(n, 4096);
    ns = ns < 1u ? 1u : (ns > max_ns ? max_ns : ns);
    const uint32_t span = cdiv(cdiv(n, ns), 256) * 256;
    ns = cdiv(n, span);
    const double e = (double)eps;
    hipLaunchKernelGGL(k_direct, dim3(tb, ns), dim3(256), 0, st, (const float4 *)c->xyzm,
                       (const uint32_t *)c->inv, tgt, nt, n, span, e * e, acc, pot, c->status);
}

}  // namespace bh
