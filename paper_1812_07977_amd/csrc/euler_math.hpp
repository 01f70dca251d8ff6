// euler_math.hpp -- per-cell and per-face arithmetic of the Euler step for
// gfx950: primitive recovery, minmod-limited reconstruction, HLL flux and the
// signal rate of the CFL condition, for FP64 and FP32 states.  All functions
// are forced inline and use explicit fused multiply-adds where a fused
// operation is wanted; the library is built with -ffp-contract=off so the
// compiler never fuses anything else, which keeps every face flux
// bit-identical wherever in a kernel it is evaluated.
#pragma once

#include <hip/hip_runtime.h>

namespace gs {

constexpr int NV = 5;  // fields: rho, m_x, m_y, m_z, E  /  rho, v_x, v_y, v_z, p

// Physical constants of one mesh in the arithmetic type R, passed by value.
template <typename R>
struct PhysT {
    R gamma;     // ratio of specific heats
    R gm1;       // gamma - 1
    R inv_gm1;   // 1 / (gamma - 1)
    R inv_h[3];  // 1 / cell width along x, y, z
    R cfl;       // Courant number
};
using Phys = PhysT<double>;

// ---------------------------------------------------------------------------
// Scalar primitives per type
// ---------------------------------------------------------------------------

__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double minR(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float minR(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double maxR(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float maxR(float a, float b) { return __builtin_fmaxf(a, b); }

// 1/a for a > 0 normal.  FP64: the hardware estimate r (relative error below
// 2^-24) refined by one third-order step r (1 + e + e^2), e = 1 - a r, which
// cubes the error, leaving only the final rounding.  FP32: the hardware
// reciprocal, accurate to 1 ulp.
__device__ __forceinline__ double recip(double a)
{
    double r = __builtin_amdgcn_rcp(a);
    double e = __builtin_fma(-a, r, 1.0);
    return __builtin_fma(r, __builtin_fma(e, e, e), r);
}
__device__ __forceinline__ float recip(float a) { return __builtin_amdgcn_rcpf(a); }

// 1/sqrt(x) for x > 0 normal.  FP64: the hardware estimate y (relative error
// below 2^-24) refined by one third-order step y (1 + e/2 + 3e^2/8),
// e = 1 - x y^2.  FP32: the hardware estimate, accurate to 1 ulp.
__device__ __forceinline__ double rsqrt(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double e = __builtin_fma(-(x * y), y, 1.0);
    double q = e * __builtin_fma(e, 0.375, 0.5);
    return __builtin_fma(y, q, y);
}
__device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }

// Sound speed sqrt(gamma p / rho), written as (gamma p) / sqrt(gamma p rho)
// so that it needs one reciprocal square root and no division.
template <typename R>
__device__ __forceinline__ R sound_speed(R rho, R p, const PhysT<R>& k)
{
    R a = k.gamma * p;
    return a * rsqrt(a * rho);
}

// minmod(a, b): the median of (a, b, 0), i.e. the argument of smaller
// magnitude when both share a strict sign, otherwise 0.
template <typename R>
__device__ __forceinline__ R minmod(R a, R b)
{
    R lo = minR(a, b);
    R hi = maxR(a, b);
    return maxR(lo, minR(hi, R(0)));
}

// Conserved -> primitive in FP64.  Returns false for a non-physical cell:
// rho or p not positive, or not finite.
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

// Conserved -> primitive of an FP32 state: the cell is promoted to FP64 so
// that the pressure, a difference of total and kinetic energy, keeps its
// relative accuracy; the primitives are then rounded to FP32.
__device__ __forceinline__ bool cons_to_prim(const float u[NV], float w[NV], const Phys& k)
{
    double ud[NV], wd[NV];
#pragma unroll
    for (int f = 0; f < NV; ++f) ud[f] = u[f];
    bool ok = cons_to_prim(ud, wd, k);
#pragma unroll
    for (int f = 0; f < NV; ++f) w[f] = (float)wd[f];
    return ok;
}

// Signal rate of the CFL condition, sum_d (|v_d| + c) / h_d, in FP64.
__device__ __forceinline__ double signal_rate(const double w[NV], const Phys& k)
{
    double c = sound_speed(w[0], w[4], k);
    double r = (__builtin_fabs(w[1]) + c) * k.inv_h[0];
    r = r + (__builtin_fabs(w[2]) + c) * k.inv_h[1];
    return r + (__builtin_fabs(w[3]) + c) * k.inv_h[2];
}

// Signal rate of a conserved cell of either type, recovered in FP64.
template <typename T>
__device__ __forceinline__ bool cell_rate(const T u[NV], const Phys& k, double& rate)
{
    double ud[NV], wd[NV];
#pragma unroll
    for (int f = 0; f < NV; ++f) ud[f] = (double)u[f];
    bool ok = cons_to_prim(ud, wd, k);
    rate = signal_rate(wd, k);
    return ok;
}

// HLL flux through a face with normal along axis AX (0, 1, 2) between the
// primitive face states L and R, with Davis estimates S_L = min(u_L - c_L,
// u_R - c_R), S_R = max(u_L + c_L, u_R + c_R).  The branch form
// (F_L if S_L >= 0, F_R if S_R <= 0, else the HLL average) is evaluated as
// the single expression with S_L clamped to <= 0 and S_R to >= 0, which is
// the same function.
//
// The average is regrouped by side.  With w_L = S_R/(S_R - S_L),
// w_R = -S_L/(S_R - S_L) and w_d = S_L S_R/(S_R - S_L), the flux is
// w_L F_L + w_R F_R + w_d (U_R - U_L).  Every component of a physical flux
// is the conserved component times the normal velocity, plus a pressure term
// in the normal momentum and energy components, so each side contributes its
// conserved state times a_L = w_L u_L - w_d (a_R = w_R u_R + w_d) plus
// pressure terms; density times a_s (b_s) then carries the mass component
// and, times a velocity, every momentum component.  The conserved momenta
// and the physical fluxes are never formed.
//
// |v|^2 is summed as the normal component onto (first tangential^2 + second
// tangential^2), with the tangential components in the order (y, z), (x, z),
// (x, y) for AX = 0, 1, 2.  A face along x evaluated as AX = 1 with the x and
// y velocity slots exchanged therefore performs exactly the operations of
// the AX = 0 evaluation, every other step being per component.
template <int AX, typename R>
__device__ __forceinline__ void hll_flux(const R L[NV], const R Rs[NV], const PhysT<R>& k, R F[NV])
{
    constexpr int N = 1 + AX;                // index of the normal velocity / momentum
    constexpr int T1 = (AX == 0) ? 2 : 1;    // tangential components
    constexpr int T2 = (AX == 2) ? 2 : 3;
    const R half = R(0.5);
    // total energies of the face states
    R v2L = fmaR(L[N], L[N], fmaR(L[T2], L[T2], L[T1] * L[T1]));
    R v2R = fmaR(Rs[N], Rs[N], fmaR(Rs[T2], Rs[T2], Rs[T1] * Rs[T1]));
    R EL = fmaR(L[4], k.inv_gm1, (half * L[0]) * v2L);
    R ER = fmaR(Rs[4], k.inv_gm1, (half * Rs[0]) * v2R);
    // signal speeds and weights
    R unL = L[N], unR = Rs[N];
    R cL = sound_speed(L[0], L[4], k);
    R cR = sound_speed(Rs[0], Rs[4], k);
    R sl = minR(minR(unL - cL, unR - cR), R(0));
    R sr = maxR(maxR(unL + cL, unR + cR), R(0));
    R inv = recip(sr - sl);
    R wl = sr * inv, wr = -sl * inv, wd = sl * wl;
    // per-side factors
    R wlu = wl * unL, wru = wr * unR;
    R aL = wlu - wd, aR = wru + wd;
    R bL = L[0] * aL, bR = Rs[0] * aR;
    F[0] = bL + bR;
    F[T1] = fmaR(L[T1], bL, Rs[T1] * bR);
    F[T2] = fmaR(L[T2], bL, Rs[T2] * bR);
    F[N] = fmaR(L[N], bL, fmaR(Rs[N], bR, fmaR(wl, L[4], wr * Rs[4])));
    F[4] = fmaR(EL, aL, fmaR(ER, aR, fmaR(wlu, L[4], wru * Rs[4])));
}

// Flux through the face between cells b and c along axis AX, from the
// primitives of four consecutive cells a, b, c, d: one-sided differences,
// minmod slopes of b and c, face states b + sigma_b/2 and c - sigma_c/2.
// Both slopes involve the middle difference d1, and the median of (x, d1, 0)
// is x clamped to [min(d1, 0), max(d1, 0)], so the two slopes share those
// bounds: six min/max per field instead of eight, the same values (each
// form returns one of its arguments or zero).
template <int AX, typename R>
__device__ __forceinline__ void face_flux(const R a[NV], const R b[NV], const R c[NV], const R d[NV],
                                          const PhysT<R>& k, R F[NV])
{
    R L[NV], Rs[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        R d0 = b[v] - a[v], d1 = c[v] - b[v], d2 = d[v] - c[v];
        R lo = minR(d1, R(0)), hi = maxR(d1, R(0));
        L[v] = fmaR(R(0.5), minR(maxR(d0, lo), hi), b[v]);     // minmod(d0, d1)
        Rs[v] = fmaR(R(-0.5), minR(maxR(d2, lo), hi), c[v]);   // minmod(d1, d2)
    }
    hll_flux<AX>(L, Rs, k, F);
}

}  // namespace gs
