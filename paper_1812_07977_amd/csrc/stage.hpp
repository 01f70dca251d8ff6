// stage.hpp -- device code shared by the single-problem path (gs_fluid.hip)
// and the batched form (gs_batch.hip): mesh geometry and tiling, the device
// words of a problem, the fused substep body of one (tile, z-chunk) item, and
// the reduction and small state kernels.  The two sources are compiled with
// their own scheduling flags; each gets its own copy of these kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "euler_math.hpp"
#include "gs_fluid.h"

namespace gs {

// Mesh geometry and tiling, passed by value.
struct Geom {
    int nx, ny, nz;
    int periodic;
    int pitch;          // distance between rows (>= nx)
    int plane;          // pitch * ny: distance between planes
    long long field;    // pitch * ny * nz: distance between fields
    int ntx, nty;       // tiles along x, y
    int kz, nchunk;     // planes per chunk, chunks along z
    int band;           // tiles per XCD band (0: plain block order)
};

// Device-resident words of a handle.  rate[] and t[] are ping-pong pairs
// indexed by the step parity: step s reads slot s&1 and prepares slot
// (s+1)&1, so no kernel ever reads a word another kernel of the same step
// writes.  rate holds the IEEE bits of a non-negative double, so an unsigned
// max is a floating-point max.
struct DevState {
    unsigned long long rate[2];
    double t[2];
    unsigned long long rate_dt;  // result slot of the dt reduction
    unsigned int flags;          // bit 0: a non-physical cell was read
    unsigned int pad;
    double tot[NV];              // conserved totals of the last totals pass
};

__device__ __forceinline__ int map_index(int i, int n, int periodic)
{
    if (periodic) {
        int r = i % n;
        return r < 0 ? r + n : r;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Workgroup -> (tile x, tile y, chunk).  Workgroups are dispatched to the 8
// XCDs round-robin; with band > 0 the n-th workgroup an XCD receives works on
// chunk n / band of that XCD's band of tiles, so at any moment the XCDs hold
// adjacent bands of the same z-chunk.
__device__ __forceinline__ void block_tile(const Geom& g, int& tx0, int& ty0, int& kc)
{
    int b = blockIdx.x;
    int tile, chunk;
    if (g.band > 0) {
        int xcd = b & 7, n = b >> 3;
        chunk = n / g.band;
        tile = xcd * g.band + (n - chunk * g.band);
    } else {
        int ntile = g.ntx * g.nty;
        chunk = b / ntile;
        tile = b - chunk * ntile;
    }
    int ty = tile / g.ntx;
    tx0 = tile - ty * g.ntx;
    ty0 = ty;
    kc = chunk;
}

// FP64 cell access goes through buffer resources: the plane of one field is
// a buffer whose base address stays in scalar registers and a lane adds only
// its 32-bit byte offset, so a load or store costs no per-lane 64-bit
// address arithmetic (5% of the FP64 loop's VALU instructions, 0.4% of the
// step's time).  The FP32 form keeps global addressing, which measured
// faster for it (its batched form 2% so).  A buffer resource covers at most
// 2^32 - 1 bytes, so a field plane must end below byte 2^32 (the create
// calls accept planes of fewer than 2^29 cells).  NT: the non-temporal hint.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* p)
{
    // raw buffer, no stride, range 2^32 - 1 bytes; the fourth descriptor
    // word's data format field must be non-zero for loads to return data
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, 0xFFFFFFFF, 0x00020000);
}

// cell off (an index within the plane) of the field plane that starts at p
template <typename T, bool NT>
__device__ __forceinline__ T load_cell(const T* p, int off)
{
    if constexpr (sizeof(T) == 8) {
        const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(plane_rsrc(p), (unsigned)off * 8u, 0, NT ? 2 : 0);
        return __builtin_bit_cast(T, v);
    } else {
        if constexpr (NT) return __builtin_nontemporal_load(p + off);
        else return p[off];
    }
}

template <typename T, bool NT>
__device__ __forceinline__ void store_cell(T v, T* p, int off)
{
    if constexpr (sizeof(T) == 8) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), plane_rsrc(p), (unsigned)off * 8u,
                                              0, NT ? 2 : 0);
    } else {
        if constexpr (NT) __builtin_nontemporal_store(v, p + off);
        else p[off] = v;
    }
}

// the five fields of cell off of a plane: base is the plane of field 0,
// field the distance between fields
template <typename T>
__device__ __forceinline__ void load5(const T* __restrict__ base, long long field, int off, T u[NV])
{
#pragma unroll
    for (int f = 0; f < NV; ++f) u[f] = load_cell<T, false>(base + f * field, off);
}

// On large meshes the streams that a substep reads or writes exactly once
// (U(n) and its compensation in the combine, the outputs) carry the
// non-temporal hint, so that they do not push the stage input, whose lines
// neighbouring tiles share as halo, out of the caches: measured 2-5% faster
// steps from 192^3 up, 5-10% slower at 128^3 and below, where the state
// stays in the 256 MB last-level cache between the substeps.
template <typename T>
__device__ __forceinline__ void load5_nt(const T* __restrict__ base, long long field, int off, T u[NV])
{
#pragma unroll
    for (int f = 0; f < NV; ++f) u[f] = load_cell<T, true>(base + f * field, off);
}

// Fused RK2 substep on states of type T (double: the FP64 form; float: the
// FP32 form).  STAGE 1: Uout = Uin + dU(Uin); the FP32 form also stores the
// increment dU(Uin) itself into D0.  STAGE 2, FP64: Uout = 0.5 ((Un + Uin) +
// dU(Uin)); FP32: the same value written as U(n) plus the increment
// 0.5 (D0 + dU(Uin)), summed with Kahan compensation, Cn holding the
// compensation of Un (read and rewritten).  Storing D0 keeps the first
// substep's increment exact: U(1) - U(n) would have lost whatever part of it
// falls below the rounding of U(1).  Uout may alias Un (each cell's Un and Cn
// are read only by the thread that writes them).  DEVDT:
// dt = cfl / max rate (slot parity), clipped to t_end; else dt = dt_host.
// RATE: accumulate the max signal rate of Uout into rate[parity ^ 1].
// Primitive recovery and signal rates run in FP64 for both forms (kd); the
// reconstruction and flux arithmetic runs in T (kt).
// Waves per SIMD of the stage kernels: three for both forms (the FP64 body
// fits 168 VGPRs without spills; with two, the SIMD idles while its waves
// wait on LDS and memory), except FP64 32 x 8 tiles, whose LDS (57 KiB per
// workgroup) admits two workgroups per CU.
template <typename T, int TY>
struct StageOcc {
    static constexpr int waves = (sizeof(T) == 8 && TY == 8) ? 2 : 3;
};

// FP64 constants for the FP64 parts: the FP64 form's own constants, or the
// separate FP64 set of the FP32 form.
__device__ __forceinline__ const Phys& phys64(const Phys& kt, const Phys&) { return kt; }
__device__ __forceinline__ const Phys& phys64(const PhysT<float>&, const Phys& kd) { return kd; }

// The work of one (tile, z-chunk) item of a substep: tile (tix, tiy),
// chunk kc of mesh g, time step dt.  Sets bad if a non-physical cell was
// read and raises rmax to the largest signal rate written (RATE).  All
// threads of the workgroup call it together (it synchronises on LDS); tid
// is the caller's thread index in the workgroup.
template <typename T, int TX, int TY, int STAGE, bool RATE, bool NTH, bool EARLY_UN = true,
          bool FULL = false>
__device__ __forceinline__ void stage_tile(const T* __restrict__ Uin, const T* Un, T* Uout, T* Cn,
                                           T* D0, const Geom& g, const PhysT<T>& kt, const Phys& K,
                                           int tix, int tiy, int kc, double dt, bool& bad,
                                           double& rmax, int tid)
{
    constexpr int NT = TX * TY;
    constexpr int WX = TX + 4, WY = TY + 4;
    constexpr bool KAHAN = (STAGE == 2) && (sizeof(T) == 4);   // FP32 stage 2
    constexpr bool KEEPD = (STAGE == 1) && (sizeof(T) == 4);   // FP32 stage 1
    static_assert(4 * (TX + TY) <= NT, "one halo cell per thread at most");
    static_assert(TX + TY <= NT, "one edge face per thread at most");
    __shared__ T Ws[NV][WY][WX];     // primitives of the plane, +2 halo
    __shared__ T Fx[NV][TY][TX + 1]; // x-face fluxes, face i-1/2 at [i]
    __shared__ T Fy[NV][TY + 1][TX]; // y-face fluxes, face j-1/2 at [j]
    constexpr int NH = 4 * (TX + TY);     // halo cells of one plane
    __shared__ T Hr[3][NV][NH];      // halo ring: raw states of 3 planes

    const int tx = tid % TX, ty = tid / TX;
    const int x0 = tix * TX, y0 = tiy * TY;
    const int z0 = kc * g.kz;
    const int z1 = min(z0 + g.kz, g.nz);

    // own column (ghost columns of ragged tiles map to valid cells).  FULL:
    // the caller guarantees whole tiles (nx and ny multiples of TX and TY),
    // so no lane is inactive and the combine and stores take no branch;
    // with the branch, the compiler's wait counting merges its two paths
    // conservatively and waits for the plane's stores to complete at the
    // end of every plane
    const int i = x0 + tx, j = y0 + ty;
    const bool active = FULL || ((i < g.nx) & (j < g.ny));
    const int own = map_index(j, g.ny, g.periodic) * g.pitch + map_index(i, g.nx, g.periodic);

    // halo role: 4 cells per tile row (x) and per tile column (y).  Halo
    // thread h loads its cell of plane z+3 in the iteration of plane z, at
    // the same time as the neighbouring tiles load that plane as their own
    // columns, so the shared cache lines are fetched from HBM once; the raw
    // values wait in the thread's own slots of the LDS ring Hr until the
    // plane is staged (no other thread touches those slots).
    int hxl = 0, hyl = 0, hoff = 0;
    bool halo = false;
    if (tid < 4 * TY) {
        int q = tid & 3;
        hyl = tid >> 2;
        hxl = q < 2 ? q - 2 : TX + q - 2;
        halo = true;
    } else if (tid < 4 * TY + 4 * TX) {
        int h = tid - 4 * TY;
        int q = h / TX;
        hxl = h - q * TX;
        hyl = q < 2 ? q - 2 : TY + q - 2;
        halo = true;
    }
    if (halo)
        hoff = map_index(y0 + hyl, g.ny, g.periodic) * g.pitch + map_index(x0 + hxl, g.nx, g.periodic);

    // edge-face role: the last TX + TY threads compute the faces on the far
    // edges of the tile, y-faces above row TY-1 (e < TX) and x-faces right of
    // column TX-1.  Both are evaluated as y-faces: for an x-face the two
    // tangential velocity components are exchanged through the LDS addressing
    // (and exchanged back on the way out); hll_flux orders its one
    // cross-component sum so that this performs the very operations of an
    // x-face evaluation, giving bit-identical fluxes.
    const int e = tid - (NT - (TX + TY));
    constexpr int PLW = WY * WX;               // one field of Ws
    constexpr int PFX = TY * (TX + 1), PFY = (TY + 1) * TX;
    int e_base = 0, e_step = 0, e_v1 = PLW, e_v2 = 2 * PLW;
    T* e_out = nullptr;
    int e_f1 = PFY, e_f2 = 2 * PFY, e_fs = PFY;
    if (e >= 0 && e < TX) {
        e_base = TY * WX + e + 2;
        e_step = WX;
        e_out = &Fy[0][TY][e];
    } else if (e >= TX) {
        const int r = e - TX;
        e_base = (r + 2) * WX + TX;
        e_step = 1;
        e_v1 = 2 * PLW;
        e_v2 = PLW;
        e_out = &Fx[0][r][TX];
        e_f1 = 2 * PFX;
        e_f2 = PFX;
        e_fs = PFX;
    }

    const T dtT = (T)dt;
    const T sx = -dtT * kt.inv_h[0], sy = -dtT * kt.inv_h[1], sz = -dtT * kt.inv_h[2];

    const long long F = g.field;
    // FP64: the plane index is the same in every lane, and readfirstlane
    // keeps it, and the plane's address, in scalar registers for the buffer
    // resources
    auto plane_ptr = [&](const T* base, int z) {
        int zm = map_index(z, g.nz, g.periodic);
        if constexpr (sizeof(T) == 8) zm = __builtin_amdgcn_readfirstlane(zm);
        return base + (long long)zm * g.plane;
    };

    // ---- prologue: planes z0-2 .. z0+2 of the own column, halo of z0 ----
    T Uk[NV], Uk1[NV], Uk2[NV], Hk[NV];
    const int hslot = halo ? tid : 0;
    T Wk[NV], Wk1[NV], WLz[NV], Fm[NV];
    {
        T Um2[NV], Um1[NV], Wm2[NV], Wm1[NV];
        load5(plane_ptr(Uin, z0 - 2), F, own, Um2);
        load5(plane_ptr(Uin, z0 - 1), F, own, Um1);
        load5(plane_ptr(Uin, z0), F, own, Uk);
        load5(plane_ptr(Uin, z0 + 1), F, own, Uk1);
        load5(plane_ptr(Uin, z0 + 2), F, own, Uk2);
        if (halo) {
            // ring: planes z0, z0+1 stored, z0+2 held in registers
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                T h[NV];
                load5(plane_ptr(Uin, z0 + q), F, hoff, h);
#pragma unroll
                for (int v = 0; v < NV; ++v) Hr[(z0 + q) % 3][v][hslot] = h[v];
            }
            load5(plane_ptr(Uin, z0 + 2), F, hoff, Hk);
        }
        bad |= !cons_to_prim(Um2, Wm2, K);
        bad |= !cons_to_prim(Um1, Wm1, K);
        bad |= !cons_to_prim(Uk, Wk, K);
        bad |= !cons_to_prim(Uk1, Wk1, K);
        face_flux<2>(Wm2, Wm1, Wk, Wk1, kt, Fm);  // face z0 - 1/2
#pragma unroll
        for (int v = 0; v < NV; ++v)
            WLz[v] = fmaR(T(0.5), minmod(Wk[v] - Wm1[v], Wk1[v] - Wk[v]), Wk[v]);
    }

    // every load of the prologue complete before the plane loop: otherwise
    // the compiler's wait counting, which merges the loop's entry with its
    // back edge, takes the queue's plane z+2 as possibly in flight at every
    // plane and waits after the second barrier for the plane z+3 loads
    // issued at the top of the same plane (FP32 substep 1 1.5% faster with
    // this wait; FP64 unchanged)
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0); expcnt, lgkmcnt not waited

    for (int z = z0; z < z1; ++z) {
        // prefetch plane z+3 of the own column at the top of the plane, so
        // that it has the whole plane to arrive before the queue rotation
        // at its end consumes it (measured 1% faster than issuing it after
        // the in-plane faces, still three waves per SIMD)
        T Uk3[NV];
        load5(plane_ptr(Uin, z + 3), F, own, Uk3);
        // stage the plane's primitives in LDS
#pragma unroll
        for (int v = 0; v < NV; ++v) Ws[v][ty + 2][tx + 2] = Wk[v];
        if (halo) {
            T w[NV];
            T h[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                Hr[(z + 2) % 3][v][hslot] = Hk[v];   // plane z+2, loaded last iteration
                h[v] = Hr[z % 3][v][hslot];           // plane z
            }
            cons_to_prim(h, w, K);
#pragma unroll
            for (int v = 0; v < NV; ++v) Ws[v][hyl + 2][hxl + 2] = w[v];
        }
        __syncthreads();

        // in-plane faces: x-face left of the own cell, y-face below it
        {
            T a[NV], b[NV], c[NV], d[NV], f[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                a[v] = Ws[v][ty + 2][tx];
                b[v] = Ws[v][ty + 2][tx + 1];
                c[v] = Ws[v][ty + 2][tx + 2];
                d[v] = Ws[v][ty + 2][tx + 3];
            }
            face_flux<0>(a, b, c, d, kt, f);
#pragma unroll
            for (int v = 0; v < NV; ++v) Fx[v][ty][tx] = f[v];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                a[v] = Ws[v][ty][tx + 2];
                b[v] = Ws[v][ty + 1][tx + 2];
                d[v] = Ws[v][ty + 3][tx + 2];
            }
            face_flux<1>(a, b, c, d, kt, f);
#pragma unroll
            for (int v = 0; v < NV; ++v) Fy[v][ty][tx] = f[v];
        }
        // faces on the far edges of the tile (one evaluation per lane)
        if (e >= 0) {
            const T* ws = &Ws[0][0][0];
            const int off[NV] = {0, e_v1, e_v2, 3 * PLW, 4 * PLW};
            T a[NV], b[NV], c[NV], d[NV], f[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const T* p = ws + off[v] + e_base;
                a[v] = p[0];
                b[v] = p[e_step];
                c[v] = p[2 * e_step];
                d[v] = p[3 * e_step];
            }
            face_flux<1>(a, b, c, d, kt, f);
            e_out[0] = f[0];
            e_out[e_f1] = f[1];
            e_out[e_f2] = f[2];
            e_out[3 * e_fs] = f[3];
            e_out[4 * e_fs] = f[4];
        }
        // the halo of plane z+3 and, in the FP64 second substep, U(n) of
        // this plane, issued before the barrier rather than after it, so that
        // they are in flight while the workgroup waits there (2% faster steps
        // in both forms).  U(n) of the FP32 form and its compensation and
        // first increment stay after the barrier (issued before it, they made
        // the FP32 batched form 3% slower), and so does U(n) with EARLY_UN
        // false: in the batched kernels, whose item loop leaves no registers
        // for it, and in the FULL kernels, which measured 1% faster so
        if (halo) load5(plane_ptr(Uin, z + 3), F, hoff, Hk);
        constexpr bool UN_EARLY = STAGE == 2 && sizeof(T) == 8 && EARLY_UN;
        T Uo[NV], Co[NV], Do[NV];
        if (UN_EARLY) {
            if (NTH) load5_nt(Un + (long long)z * g.plane, F, own, Uo);
            else load5(Un + (long long)z * g.plane, F, own, Uo);
        }
        __syncthreads();

        // otherwise U(n) (FP32: with its compensation and the first
        // increment) of this plane here, for the combine below (loading them
        // a whole plane ahead would keep more registers live than the three
        // waves per SIMD allow)
        if (STAGE == 2 && !UN_EARLY) {
            if (NTH) load5_nt(Un + (long long)z * g.plane, F, own, Uo);
            else load5(Un + (long long)z * g.plane, F, own, Uo);
        }
        if (KAHAN) {
            if (NTH) {
                load5_nt(Cn + (long long)z * g.plane, F, own, Co);
                load5_nt(D0 + (long long)z * g.plane, F, own, Do);
            } else {
                load5(Cn + (long long)z * g.plane, F, own, Co);
                load5(D0 + (long long)z * g.plane, F, own, Do);
            }
        }

        // z-face above the own cell, from the register queue
        T Fp[NV], W2[NV];
        {
            T R[NV];
            bad |= !cons_to_prim(Uk2, W2, K);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const T w0 = Ws[v][ty + 2][tx + 2];
                T s1 = minmod(Wk1[v] - w0, W2[v] - Wk1[v]);
                R[v] = fmaR(T(-0.5), s1, Wk1[v]);
                Wk[v] = fmaR(T(0.5), s1, Wk1[v]);  // left state of face z+3/2
            }
            hll_flux<2>(WLz, R, kt, Fp);
        }

        // divergence, RK combine, store
        {
            T out[NV], aux[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                T du = (Fx[v][ty][tx + 1] - Fx[v][ty][tx]) * sx;
                du = fmaR(Fy[v][ty + 1][tx] - Fy[v][ty][tx], sy, du);
                du = fmaR(Fp[v] - Fm[v], sz, du);
                if (STAGE == 1) {
                    out[v] = Uk[v] + du;
                    aux[v] = du;
                } else if (!KAHAN) {
                    out[v] = T(0.5) * ((Uo[v] + Uk[v]) + du);
                } else {
                    // U(n+1) = U(n) + inc, inc = 0.5 (dU(U(n)) + dU(U(1))),
                    // summed with Kahan compensation: the represented value
                    // is head - compensation
                    T inc = T(0.5) * (Do[v] + du);
                    T y = inc - Co[v];
                    T s = Uo[v] + y;
                    aux[v] = (s - Uo[v]) - y;
                    out[v] = s;
                }
            }
            if (active) {
                T* po = Uout + (long long)z * g.plane;
#pragma unroll
                for (int v = 0; v < NV; ++v) store_cell<T, NTH>(out[v], po + v * F, own);
                if (KAHAN || KEEPD) {
                    T* pa = (KAHAN ? Cn : D0) + (long long)z * g.plane;
#pragma unroll
                    for (int v = 0; v < NV; ++v) store_cell<T, NTH>(aux[v], pa + v * F, own);
                }
            }
            if (RATE && active) {
                double r;
                cell_rate(out, K, r);
                rmax = __builtin_fmax(rmax, r);
            }
        }

        // rotate the queue: Wk holds the new left z-face state until here
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            WLz[v] = Wk[v];
            Wk[v] = Wk1[v];
            Wk1[v] = W2[v];
            Uk[v] = Uk1[v];
            Uk1[v] = Uk2[v];
            Uk2[v] = Uk3[v];
            Fm[v] = Fp[v];
        }
    }

}

namespace {

// Max signal rate over all cells of U (first pass: one partial per block) and
// the non-physical flag.  For the FP32 form U is the head of the state.
constexpr int RED_THREADS = 256;
constexpr int RED_BLOCKS = 1024;

template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
rate_partial_kernel(const T* __restrict__ U, long long ncell, Phys k,
                    double* __restrict__ partial, DevState* __restrict__ st)
{
    __shared__ double red[RED_THREADS / 64];
    double rmax = 0.0;
    bool bad = false;
    for (long long c = (long long)blockIdx.x * RED_THREADS + threadIdx.x; c < ncell;
         c += (long long)gridDim.x * RED_THREADS) {
        T u[NV];
#pragma unroll
        for (int f = 0; f < NV; ++f) u[f] = U[f * ncell + c];
        double r;
        bad |= !cell_rate(u, k, r);
        rmax = __builtin_fmax(rmax, r);
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&st->flags, 1u);
    for (int off = 32; off > 0; off >>= 1) rmax = __builtin_fmax(rmax, __shfl_xor(rmax, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < RED_THREADS / 64; ++w) m = __builtin_fmax(m, red[w]);
        partial[blockIdx.x] = m;
    }
}

// Second pass: max of the partials into *dst (as IEEE bits).
__global__ void __launch_bounds__(RED_THREADS)
rate_final_kernel(const double* __restrict__ partial, int n, unsigned long long* dst)
{
    __shared__ double red[RED_THREADS / 64];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += RED_THREADS) m = __builtin_fmax(m, partial[i]);
    for (int off = 32; off > 0; off >>= 1) m = __builtin_fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < RED_THREADS / 64; ++w) m = __builtin_fmax(m, red[w]);
        m = __builtin_fmax(red[0], m);
        *dst = (unsigned long long)__double_as_longlong(m);
    }
}

// Small state writes, as kernels so that the host never records a memset.
__global__ void init_state_kernel(DevState* st)
{
    st->rate[0] = st->rate[1] = 0ull;
    st->t[0] = st->t[1] = 0.0;
    st->rate_dt = 0ull;
    st->flags = 0u;
    st->pad = 0u;
    for (int f = 0; f < NV; ++f) st->tot[f] = 0.0;
}

__global__ void clear_flags_kernel(DevState* st) { st->flags = 0u; }

}  // namespace

// Host-side sizes shared by both sources.
inline size_t elem_size(int dtype) { return dtype == GS_F32 ? sizeof(float) : sizeof(double); }

// Substep workspace: U(1); the FP32 form also keeps the first increment.
inline long long state_work_bytes(long long ncell, int dtype)
{
    return ncell * NV * (long long)elem_size(dtype) * (dtype == GS_F32 ? 2 : 1);
}

}  // namespace gs
