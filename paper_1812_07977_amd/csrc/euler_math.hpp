// euler_math.hpp -- per-cell and per-face FP64 arithmetic of the Euler step
// for gfx950: primitive recovery, minmod-limited reconstruction, HLL flux and
// the signal rate of the CFL condition.  All functions are forced inline and
// use explicit fma() where a fused operation is wanted; the library is built
// with -ffp-contract=off so the compiler never fuses anything else, which
// keeps every face flux bit-identical wherever in a kernel it is evaluated.
#pragma once

#include <hip/hip_runtime.h>

namespace gs {

constexpr int NV = 5;  // fields: rho, m_x, m_y, m_z, E  /  rho, v_x, v_y, v_z, p

// Physical constants of one mesh, passed by value to every kernel.
struct Phys {
    double gamma;    // ratio of specific heats
    double gm1;      // gamma - 1
    double inv_gm1;  // 1 / (gamma - 1)
    double inv_h[3]; // 1 / cell width along x, y, z
    double cfl;      // Courant number
};

// 1/a for a > 0 normal: the hardware estimate r (relative error below
// 2^-24) refined by one third-order step r (1 + e + e^2), e = 1 - a r, which
// cubes the error, leaving only the final rounding.
__device__ __forceinline__ double recip(double a)
{
    double r = __builtin_amdgcn_rcp(a);
    double e = __builtin_fma(-a, r, 1.0);
    return __builtin_fma(r, __builtin_fma(e, e, e), r);
}

// 1/sqrt(x) for x > 0 normal: the hardware estimate y (relative error below
// 2^-24) refined by one third-order step y (1 + e/2 + 3e^2/8),
// e = 1 - x y^2.
__device__ __forceinline__ double rsqrt(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double e = __builtin_fma(-(x * y), y, 1.0);
    double q = e * __builtin_fma(e, 0.375, 0.5);
    return __builtin_fma(y, q, y);
}

// Sound speed sqrt(gamma p / rho), written as (gamma p) / sqrt(gamma p rho)
// so that it needs one reciprocal square root and no division.
__device__ __forceinline__ double sound_speed(double rho, double p, const Phys& k)
{
    double a = k.gamma * p;
    return a * rsqrt(a * rho);
}

// minmod(a, b): the median of (a, b, 0), i.e. the argument of smaller
// magnitude when both share a strict sign, otherwise 0.
__device__ __forceinline__ double minmod(double a, double b)
{
    double lo = __builtin_fmin(a, b);
    double hi = __builtin_fmax(a, b);
    return __builtin_fmax(lo, __builtin_fmin(hi, 0.0));
}

// Conserved -> primitive.  Returns false for a non-physical cell: rho or p
// not positive, or not finite.
__device__ __forceinline__ bool cons_to_prim(const double u[NV], double w[NV], const Phys& k)
{
    double ir = recip(u[0]);
    double vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
    double kin = 0.5 * ((u[1] * vx + u[2] * vy) + u[3] * vz);
    w[0] = u[0];
    w[1] = vx;
    w[2] = vy;
    w[3] = vz;
    w[4] = k.gm1 * (u[4] - kin);
    return (u[0] > 0.0) & (w[4] > 0.0) & (u[0] < __builtin_inf()) & (w[4] < __builtin_inf());
}

// Signal rate of the CFL condition, sum_d (|v_d| + c) / h_d.
__device__ __forceinline__ double signal_rate(const double w[NV], const Phys& k)
{
    double c = sound_speed(w[0], w[4], k);
    double r = (__builtin_fabs(w[1]) + c) * k.inv_h[0];
    r = r + (__builtin_fabs(w[2]) + c) * k.inv_h[1];
    return r + (__builtin_fabs(w[3]) + c) * k.inv_h[2];
}

// HLL flux through a face with normal along axis AX (0, 1, 2) between the
// primitive face states L and R, with Davis estimates S_L = min(u_L - c_L,
// u_R - c_R), S_R = max(u_L + c_L, u_R + c_R).  The branch form
// (F_L if S_L >= 0, F_R if S_R <= 0, else the HLL average) is evaluated as
// the single expression with S_L clamped to <= 0 and S_R to >= 0, which is
// the same function.
template <int AX>
__device__ __forceinline__ void hll_flux(const double L[NV], const double R[NV], const Phys& k,
                                         double F[NV])
{
    constexpr int N = 1 + AX;  // index of the normal velocity / momentum
    // conserved face states
    double mL1 = L[0] * L[1], mL2 = L[0] * L[2], mL3 = L[0] * L[3];
    double mR1 = R[0] * R[1], mR2 = R[0] * R[2], mR3 = R[0] * R[3];
    double v2L = __builtin_fma(L[3], L[3], __builtin_fma(L[2], L[2], L[1] * L[1]));
    double v2R = __builtin_fma(R[3], R[3], __builtin_fma(R[2], R[2], R[1] * R[1]));
    double EL = __builtin_fma(L[4], k.inv_gm1, (0.5 * L[0]) * v2L);
    double ER = __builtin_fma(R[4], k.inv_gm1, (0.5 * R[0]) * v2R);
    const double uL[NV] = {L[0], mL1, mL2, mL3, EL};
    const double uR[NV] = {R[0], mR1, mR2, mR3, ER};
    // physical fluxes
    double unL = L[N], unR = R[N];
    double fL[NV] = {uL[N], mL1 * unL, mL2 * unL, mL3 * unL, (EL + L[4]) * unL};
    double fR[NV] = {uR[N], mR1 * unR, mR2 * unR, mR3 * unR, (ER + R[4]) * unR};
    fL[N] = __builtin_fma(uL[N], unL, L[4]);
    fR[N] = __builtin_fma(uR[N], unR, R[4]);
    // signal speeds
    double cL = sound_speed(L[0], L[4], k);
    double cR = sound_speed(R[0], R[4], k);
    double sl = __builtin_fmin(__builtin_fmin(unL - cL, unR - cR), 0.0);
    double sr = __builtin_fmax(__builtin_fmax(unL + cL, unR + cR), 0.0);
    double inv = recip(sr - sl);
    double wl = sr * inv, wr = -sl * inv, wd = sl * wl;
#pragma unroll
    for (int v = 0; v < NV; ++v)
        F[v] = __builtin_fma(wl, fL[v], __builtin_fma(wr, fR[v], wd * (uR[v] - uL[v])));
}

// Flux through the face between cells b and c along axis AX, from the
// primitives of four consecutive cells a, b, c, d: one-sided differences,
// minmod slopes of b and c, face states b + sigma_b/2 and c - sigma_c/2.
template <int AX>
__device__ __forceinline__ void face_flux(const double a[NV], const double b[NV], const double c[NV],
                                          const double d[NV], const Phys& k, double F[NV])
{
    double L[NV], R[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double d0 = b[v] - a[v], d1 = c[v] - b[v], d2 = d[v] - c[v];
        L[v] = __builtin_fma(0.5, minmod(d0, d1), b[v]);
        R[v] = __builtin_fma(-0.5, minmod(d1, d2), c[v]);
    }
    hll_flux<AX>(L, R, k, F);
}

}  // namespace gs
