// Cloud-in-cell surface density on a polar (R, phi) grid and its adjoint:
// the observable of the differentiation workload (the face-on surface
// density of the disk, as the paper shows for its Milky Way run, Sec. IV).
//
// Cell centres R_i = r_min + (i + 1/2) dR, phi_j = (j + 1/2) dphi; a particle
// at (R, phi) with u = (R - r_min)/dR - 1/2 and v = phi/dphi - 1/2 spreads its
// mass bilinearly over the four cells around (u, v) (phi periodic, cells
// outside [0, n_r) dropped); particles with R outside [r_min, r_max) are
// dropped, so d(phi)/dx ~ 1/R stays bounded; density = mass /
// (dphi (R_{i+1}^2 - R_i^2) / 2).
#include "bh_internal.h"

namespace bh {

struct CicGeom {
    float rmin, rmax, dr, dphi;
    int nr, nphi;
};

__device__ __forceinline__ void cic_coords(float x, float y, const CicGeom &g, float &R, int &i0,
                                           int &j0, float &fu, float &fv) {
    R = sqrtf(x * x + y * y);
    float phi = atan2f(y, x);
    if (phi < 0.f) phi += 6.28318530717958647692f;
    const float u = (R - g.rmin) / g.dr - 0.5f;
    const float v = phi / g.dphi - 0.5f;
    const float fi = floorf(u), fj = floorf(v);
    i0 = (int)fi;
    j0 = (int)fj;
    fu = u - fi;
    fv = v - fj;
}

__device__ __forceinline__ float cic_area(int i, const CicGeom &g) {
    const float r0 = g.rmin + i * g.dr, r1 = r0 + g.dr;
    return 0.5f * g.dphi * (r1 * r1 - r0 * r0);
}

__global__ __launch_bounds__(256) void k_cic_deposit(const float *__restrict__ pos,
                                                     const float *__restrict__ mass,
                                                     const uint8_t *__restrict__ sel, uint32_t n,
                                                     CicGeom g, double *acc) {
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n || (sel && !sel[k])) return;
    float R, fu, fv;
    int i0, j0;
    cic_coords(pos[3 * (size_t)k], pos[3 * (size_t)k + 1], g, R, i0, j0, fu, fv);
    if (!(R >= g.rmin && R < g.rmax)) return;
    const float m = mass[k];
    for (int a = 0; a < 2; ++a) {
        const int i = i0 + a;
        if (i < 0 || i >= g.nr) continue;
        const float wu = a ? fu : 1.f - fu;
        for (int b = 0; b < 2; ++b) {
            int j = j0 + b;
            j = j < 0 ? j + g.nphi : (j >= g.nphi ? j - g.nphi : j);
            const float wv = b ? fv : 1.f - fv;
            atomicAdd(acc + (size_t)i * g.nphi + j, (double)(m * wu * wv));
        }
    }
}

__global__ __launch_bounds__(256) void k_cic_finish(const double *__restrict__ acc, CicGeom g,
                                                    float *density) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= g.nr * g.nphi) return;
    density[b] = (float)(acc[b] / (double)cic_area(b / g.nphi, g));
}

__global__ __launch_bounds__(256) void k_cic_vjp(const float *__restrict__ pos,
                                                 const float *__restrict__ mass,
                                                 const uint8_t *__restrict__ sel, uint32_t n,
                                                 CicGeom g, const float *__restrict__ gden,
                                                 float *g_pos, float *g_mass) {
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n || (sel && !sel[k])) return;
    const float x = pos[3 * (size_t)k], y = pos[3 * (size_t)k + 1];
    float R, fu, fv;
    int i0, j0;
    cic_coords(x, y, g, R, i0, j0, fu, fv);
    if (!(R >= g.rmin && R < g.rmax)) return;
    const float m = mass[k];
    float dfu = 0.f, dfv = 0.f, dm = 0.f;  // dL/dfu, dL/dfv, dL/dm
    for (int a = 0; a < 2; ++a) {
        const int i = i0 + a;
        if (i < 0 || i >= g.nr) continue;
        const float wu = a ? fu : 1.f - fu, su = a ? 1.f : -1.f;
        const float ia = 1.f / cic_area(i, g);
        for (int b = 0; b < 2; ++b) {
            int j = j0 + b;
            j = j < 0 ? j + g.nphi : (j >= g.nphi ? j - g.nphi : j);
            const float wv = b ? fv : 1.f - fv, sv = b ? 1.f : -1.f;
            const float gb = gden[(size_t)i * g.nphi + j] * ia;
            dm += gb * wu * wv;
            dfu += gb * m * su * wv;
            dfv += gb * m * wu * sv;
        }
    }
    // u = (R - rmin)/dR - 1/2, v = phi/dphi - 1/2; dR/dx = x/R, dphi/dx = -y/R^2
    const float du = dfu / g.dr, dv = dfv / g.dphi;
    const float iR = 1.f / R;
    if (g_pos) {
        g_pos[3 * (size_t)k] += du * x * iR - dv * y * iR * iR;
        g_pos[3 * (size_t)k + 1] += du * y * iR + dv * x * iR * iR;
    }
    if (g_mass) g_mass[k] += dm;
}

void launch_cic(const float *pos, const float *mass, const uint8_t *sel, uint32_t n, float rmin,
                float rmax, int nr, int nphi, double *scratch, float *density, hipStream_t st) {
    const CicGeom g{rmin, rmax, (rmax - rmin) / nr, 6.28318530717958647692f / nphi, nr, nphi};
    const uint32_t nb = (uint32_t)nr * (uint32_t)nphi;
    launch_fill_u32(reinterpret_cast<uint32_t *>(scratch), 0u, 2ull * nb, st);
    if (n) hipLaunchKernelGGL(k_cic_deposit, dim3(cdiv(n, 256)), dim3(256), 0, st, pos, mass, sel, n, g, scratch);
    hipLaunchKernelGGL(k_cic_finish, dim3(cdiv(nb, 256)), dim3(256), 0, st,
                       (const double *)scratch, g, density);
}

void launch_cic_vjp(const float *pos, const float *mass, const uint8_t *sel, uint32_t n,
                    float rmin, float rmax, int nr, int nphi, const float *gden, float *g_pos,
                    float *g_mass, hipStream_t st) {
    const CicGeom g{rmin, rmax, (rmax - rmin) / nr, 6.28318530717958647692f / nphi, nr, nphi};
    if (n) hipLaunchKernelGGL(k_cic_vjp, dim3(cdiv(n, 256)), dim3(256), 0, st, pos, mass, sel, n, g, gden, g_pos, g_mass);
}

}  // namespace bh
