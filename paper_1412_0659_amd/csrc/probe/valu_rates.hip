// Issue rate of single VALU instruction kinds on the current GPU: every lane
// runs 8 independent chains of one instruction kind for kIt trips; the grid
// holds enough waves to fill every SIMD.  Prints one JSON line with the
// wave64 instructions per cycle per SIMD at the nominal 2.4 GHz clock
// (0.25 = one wave64 instruction every 4 cycles).
//
// The kinds compared are those of the walk's particle-cell term: FP32 FMA
// with all operands in VGPRs, FP32 FMA reading an SGPR, packed FP16 FMA,
// mixed FP16/FP32 FMA (the FP16 far field's FP32 accumulation), the
// reciprocal square roots, and single encodings of FMA, multiply and add.
// Measurement only; not part of the library.
#include <hip/hip_runtime.h>

#include <cstdio>

typedef _Float16 h2 __attribute__((ext_vector_type(2)));
constexpr int kIt = 4096;

__global__ __launch_bounds__(256) void k_f32_vgpr(float *out, float a, float b) {
    float x[8], y[8];
    for (int i = 0; i < 8; ++i) {
        x[i] = threadIdx.x * 1e-3f + i;
        y[i] = a + i * 1e-4f * threadIdx.x;
    }
    for (int it = 0; it < kIt; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = fmaf(y[i], y[(i + 3) & 7], x[i]);
    float s = 0.f;
    for (int i = 0; i < 8; ++i) s += x[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_f32_sgpr(float *out, float a, float b) {
    float x[8];
    for (int i = 0; i < 8; ++i) x[i] = threadIdx.x * 1e-3f + i;
    for (int it = 0; it < kIt; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = fmaf(x[i], a, b);
    float s = 0.f;
    for (int i = 0; i < 8; ++i) s += x[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_pk_f16(float *out, float a, float b) {
    h2 x[8], y[8];
    for (int i = 0; i < 8; ++i) {
        x[i] = h2{(_Float16)(threadIdx.x * 1e-3f), (_Float16)i};
        y[i] = h2{(_Float16)(a + i * 1e-4f * threadIdx.x), (_Float16)b};
    }
    for (int it = 0; it < kIt; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = __builtin_elementwise_fma(x[i], y[i], y[(i + 1) & 7]);
    float s = 0.f;
    for (int i = 0; i < 8; ++i) s += (float)x[i].x + (float)x[i].y;
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_mix(float *out, float a, float b) {
    float x[8];
    const h2 hv = {(_Float16)a, (_Float16)b};
    const float bv = b + threadIdx.x * 1e-6f;
    for (int i = 0; i < 8; ++i) x[i] = threadIdx.x * 1e-3f + i;
    for (int it = 0; it < kIt; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i)
            asm volatile("v_fma_mix_f32 %0, %1, %2, %0 op_sel_hi:[1,0,0]" : "+v"(x[i]) : "v"(hv), "v"(bv));
    float s = 0.f;
    for (int i = 0; i < 8; ++i) s += x[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_rsq_f32(float *out, float a, float b) {
    float x[8];
    for (int i = 0; i < 8; ++i) x[i] = threadIdx.x * 1e-3f + i + 1.f;
    for (int it = 0; it < kIt; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = __builtin_amdgcn_rsqf(x[i]);
    float s = 0.f;
    for (int i = 0; i < 8; ++i) s += x[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_rsq_f16(float *out, float a, float b) {
    _Float16 x[8];
    for (int i = 0; i < 8; ++i) x[i] = (_Float16)(threadIdx.x * 1e-3f + i + 1.f);
    for (int it = 0; it < kIt; ++it)
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = __builtin_amdgcn_rsqh(x[i]);
    float s = 0.f;
    for (int i = 0; i < 8; ++i) s += (float)x[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

// One instruction form per kernel, written out so the encoding is fixed:
// VOP2 (4 bytes) against VOP3 (8 bytes), and the operand kinds of VOP2
// (an SGPR, an inline constant, a 32-bit literal) that the walk's terms use.
#define ASM_KERNEL(NAME, INSTR, ...)                                               \
    __global__ __launch_bounds__(256) void NAME(float *out, float a, float b) {   \
        float x[8], y[8];                                                        \
        for (int i = 0; i < 8; ++i) {                                            \
            x[i] = threadIdx.x * 1e-3f + i;                                      \
            y[i] = a + i * 1e-4f * threadIdx.x;                                  \
        }                                                                        \
        for (int it = 0; it < kIt; ++it)                                         \
            _Pragma("unroll") for (int i = 0; i < 8; ++i)                        \
                asm volatile(INSTR : "+v"(x[i]) : __VA_ARGS__);                  \
        float s = 0.f;                                                           \
        for (int i = 0; i < 8; ++i) s += x[i];                                   \
        out[blockIdx.x * 256 + threadIdx.x] = s;                                 \
    }

ASM_KERNEL(k_fmac_vop2, "v_fmac_f32_e32 %0, %1, %2", "v"(y[i]), "v"(y[(i + 3) & 7]))
ASM_KERNEL(k_fma_vop3, "v_fma_f32 %0, %1, %2, %0", "v"(y[i]), "v"(y[(i + 3) & 7]))
ASM_KERNEL(k_fma_vop3_neg, "v_fma_f32 %0, %1, %2, -%0", "v"(y[i]), "v"(y[(i + 3) & 7]))
ASM_KERNEL(k_fmac_vop2_sgpr, "v_fmac_f32_e32 %0, %1, %2", "s"(a), "v"(y[i]))
ASM_KERNEL(k_fmac_vop2_inline, "v_fmac_f32_e32 %0, 0.5, %1", "v"(y[i]))
ASM_KERNEL(k_fmac_vop2_literal, "v_fmac_f32_e32 %0, 0x3f7fbe77, %1", "v"(y[i]))
ASM_KERNEL(k_mul_vop2, "v_mul_f32_e32 %0, %1, %0", "v"(y[i]))
ASM_KERNEL(k_add_u32_vop2_sgpr, "v_add_u32_e32 %0, %1, %0", "s"(a))

typedef void (*Kern)(float *, float, float);

static double rate(Kern k, float *d, int nb) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
    for (int r = 0; r < 40; ++r)  // bring the clocks up
        hipLaunchKernelGGL(k, dim3(nb), dim3(256), 0, 0, d, 0.999f, 0.001f);
    (void)hipEventRecord(e0, 0);
    for (int r = 0; r < 5; ++r) hipLaunchKernelGGL(k, dim3(nb), dim3(256), 0, 0, d, 0.999f, 0.001f);
    (void)hipEventRecord(e1, 0);
    if (hipEventSynchronize(e1) != hipSuccess) return -1.0;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0);
    const double winstr = nb * 4.0 * 5.0 * 8.0 * kIt;  // waves x launches x chains x trips
    return winstr / (ms * 1e-3) / (4.0 * cus) / 2.4e9;
}

int main() {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess ||
        cus <= 0)
        return 1;
    const int nb = cus * 32;  // 128 waves per CU
    float *d = nullptr;
    if (hipMalloc(&d, (size_t)nb * 256 * sizeof(float)) != hipSuccess) return 1;
    const struct {
        const char *name;
        Kern k;
    } ks[] = {{"fma_f32_vgpr", k_f32_vgpr}, {"fma_f32_sgpr", k_f32_sgpr}, {"pk_fma_f16", k_pk_f16},
              {"fma_mix_f32", k_mix},      {"rsq_f32", k_rsq_f32},      {"rsq_f16", k_rsq_f16},
              {"fmac_vop2", k_fmac_vop2},  {"fma_vop3", k_fma_vop3},    {"fma_vop3_neg", k_fma_vop3_neg},
              {"fmac_vop2_sgpr", k_fmac_vop2_sgpr}, {"fmac_vop2_inline", k_fmac_vop2_inline},
              {"fmac_vop2_literal", k_fmac_vop2_literal}, {"mul_vop2", k_mul_vop2},
              {"add_u32_vop2_sgpr", k_add_u32_vop2_sgpr}};
    printf("{\"unit\": \"wave64 instructions per cycle per SIMD at 2.4 GHz\", \"cus\": %d", cus);
    for (const auto &e : ks) printf(", \"%s\": %.3f", e.name, rate(e.k, d, nb));
    printf("}\n");
    (void)hipFree(d);
    return 0;
}
