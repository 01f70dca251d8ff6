// gs_fluid.hip -- gfx950 kernels and C ABI of libgs_fluid.so.
//
// One RK2 step is two launches of one fused stage kernel (the paper's
// Differences -> Reconstruction -> Fluxes -> Update plus the RK combine of
// Algorithm 1, each substep a single pass), plus a max-reduction for the
// time step, which the device-dt path fuses into the second substep.
//
// Stage kernel design (2.5D march):
//   * A workgroup of TX*TY threads owns a TX x TY column tile of the mesh and
//     marches through KZ consecutive z-planes.  Thread (tx, ty) owns cell
//     column (x0+tx, y0+ty).
//   * Along z every thread keeps its own column's stencil in registers: the
//     raw conserved states of planes k, k+1, k+2 (the last one prefetched one
//     iteration ahead), the left face state of face k+1/2 and the z-flux of
//     face k-1/2.  Every z-face flux is computed once.
//   * In the plane, primitives of the tile plus a two-cell halo (a cross: the
//     stencil never reads corners) are staged in LDS.  Thread (tx, ty)
//     computes the x-face to its left and the y-face below it; one wave
//     computes the TX + TY faces on the far edges, so every in-plane face is
//     also computed once.  Face fluxes go to LDS, and the divergence reads the
//     two faces of each cell back.
//   * Ghost cells are virtual: every index outside the mesh is mapped to the
//     proper cell it copies (outflow) or wraps to (periodic) before loading,
//     so arrays hold proper cells only and GhostExchange costs no pass.
//   * HBM traffic per stage is one read of the stage input, one write of the
//     output and, in the second stage, one read of U(n); halo re-reads are
//     served by L2 when neighbouring tiles run on the same XCD, for which the
//     workgroup -> tile map gives each XCD a contiguous band of tile rows and
//     walks all XCDs through the same z-chunk at the same time.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "euler_math.hpp"
#include "gs_fluid.h"

namespace gs {

// Mesh geometry and tiling, passed by value.
struct Geom {
    int nx, ny, nz;
    int periodic;
    int plane;          // nx * ny
    long long field;    // nx * ny * nz: distance between fields
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

template <typename T>
__device__ __forceinline__ void load5(const T* __restrict__ base, long long field, int off, T u[NV])
{
#pragma unroll
    for (int f = 0; f < NV; ++f) u[f] = base[f * field + off];
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
    for (int f = 0; f < NV; ++f) u[f] = __builtin_nontemporal_load(base + f * field + off);
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
#ifndef GS_STAGE_WAVES_PER_EU
#define GS_STAGE_WAVES_PER_EU 2
#endif
#ifndef GS_STAGE_WAVES_PER_EU_F32
#define GS_STAGE_WAVES_PER_EU_F32 3
#endif

template <typename T>
struct StageOcc {
    static constexpr int waves = sizeof(T) == 8 ? GS_STAGE_WAVES_PER_EU : GS_STAGE_WAVES_PER_EU_F32;
};

// FP64 constants for the FP64 parts: the FP64 form's own constants, or the
// separate FP64 set of the FP32 form.
__device__ __forceinline__ const Phys& phys64(const Phys& kt, const Phys&) { return kt; }
__device__ __forceinline__ const Phys& phys64(const PhysT<float>&, const Phys& kd) { return kd; }

// The work of one (tile, z-chunk) item of a substep: tile (tix, tiy),
// chunk kc of mesh g, time step dt.  Sets bad if a non-physical cell was
// read and raises rmax to the largest signal rate written (RATE).  All
// threads of the workgroup call it together (it synchronises on LDS).
template <typename T, int TX, int TY, int STAGE, bool RATE, bool NTH>
__device__ __forceinline__ void stage_tile(const T* __restrict__ Uin, const T* Un, T* Uout, T* Cn,
                                           T* D0, const Geom& g, const PhysT<T>& kt, const Phys& K,
                                           int tix, int tiy, int kc, double dt, bool& bad,
                                           double& rmax)
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

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int x0 = tix * TX, y0 = tiy * TY;
    const int z0 = kc * g.kz;
    const int z1 = min(z0 + g.kz, g.nz);

    // own column (ghost columns of ragged tiles map to valid cells)
    const int i = x0 + tx, j = y0 + ty;
    const bool active = (i < g.nx) & (j < g.ny);
    const int own = map_index(j, g.ny, g.periodic) * g.nx + map_index(i, g.nx, g.periodic);

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
        hoff = map_index(y0 + hyl, g.ny, g.periodic) * g.nx + map_index(x0 + hxl, g.nx, g.periodic);

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

    const long long F = g.field;
    auto plane_ptr = [&](const T* base, int z) {
        return base + (long long)map_index(z, g.nz, g.periodic) * g.plane;
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


    for (int z = z0; z < z1; ++z) {
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
        __syncthreads();

        // prefetch plane z+3 of the own column and of the halo; in stage 2
        // load U(n) (FP32: with its compensation and the first increment)
        // of this plane for the combine below.  Loading these one plane
        // ahead instead would keep 10-15 more registers live and cost the
        // FP64 second substep its third wave per SIMD.
        T Uk3[NV], Uo[NV], Co[NV], Do[NV];
        load5(plane_ptr(Uin, z + 3), F, own, Uk3);
        if (halo) load5(plane_ptr(Uin, z + 3), F, hoff, Hk);
        if (STAGE == 2) {
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
                T acc = (Fx[v][ty][tx + 1] - Fx[v][ty][tx]) * kt.inv_h[0];
                acc = acc + (Fy[v][ty + 1][tx] - Fy[v][ty][tx]) * kt.inv_h[1];
                acc = acc + (Fp[v] - Fm[v]) * kt.inv_h[2];
                T du = -dtT * acc;
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
                T* po = Uout + (long long)z * g.plane + own;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    if (NTH) __builtin_nontemporal_store(out[v], po + v * F);
                    else po[v * F] = out[v];
                }
                if (KAHAN || KEEPD) {
                    T* pa = (KAHAN ? Cn : D0) + (long long)z * g.plane + own;
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        if (NTH) __builtin_nontemporal_store(aux[v], pa + v * F);
                        else pa[v * F] = aux[v];
                    }
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

template <typename T, int TX, int TY, int STAGE, bool DEVDT, bool RATE, bool NTH>
__global__ void __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(StageOcc<T>::waves)))
stage_kernel(const T* __restrict__ Uin, const T* Un, T* Uout, T* Cn, T* D0, Geom g, PhysT<T> kt,
             Phys kd, DevState* __restrict__ st, int parity, double dt_host, double t_end,
             double* __restrict__ dt_log, int step)
{
    const Phys& K = phys64(kt, kd);
    const int tid = threadIdx.x;
    int tix, tiy, kc;
    block_tile(g, tix, tiy, kc);
    // time step
    double dt = dt_host;
    const double t_now = st->t[parity];
    if (DEVDT) {
        double rate = __longlong_as_double((long long)st->rate[parity]);
        dt = K.cfl / rate;
        if (t_end > 0.0) {
            if (!(t_now < t_end)) dt = 0.0;
            else if (t_now + dt > t_end) dt = t_end - t_now;
        }
    }
    if (STAGE == 1 && blockIdx.x == 0 && tid == 0) {
        st->t[parity ^ 1] = t_now + dt;
        st->rate[parity ^ 1] = 0ull;
        if (dt_log) dt_log[step] = dt;
    }

    bool bad = false;
    double rmax = 0.0;
    stage_tile<T, TX, TY, STAGE, RATE, NTH>(Uin, Un, Uout, Cn, D0, g, kt, K, tix, tiy, kc, dt, bad,
                                            rmax);

    // epilogue: flags and the max signal rate, one atomic per wavefront
    if (__any(bad) && (tid & 63) == 0) atomicOr(&st->flags, 1u);
    if (RATE) {
        for (int off = 32; off > 0; off >>= 1) rmax = __builtin_fmax(rmax, __shfl_xor(rmax, off));
        if ((tid & 63) == 0)
            atomicMax(&st->rate[parity ^ 1], (unsigned long long)__double_as_longlong(rmax));
    }
}

// ---------------------------------------------------------------------------
// Batched form: many independent problems in one launch per substep
// ---------------------------------------------------------------------------

// One problem of a batch as the batched kernels see it.
struct BatchInst {
    Geom g;              // mesh and tiling (band unused)
    Phys kd;             // FP64 constants, with this problem's cell widths
    PhysT<float> kf;     // the same rounded to FP32
    void* U;             // caller state (FP32 form: head, then compensation)
    void* U1;            // workspace: U(1) (FP32 form: then dU(U(n)))
    DevState* st;        // this problem's device words
    int item0;           // first work item (tile, z-chunk) of this problem
    int items;
};

__device__ __forceinline__ const Phys& batch_phys(const BatchInst& I, const Phys*) { return I.kd; }
__device__ __forceinline__ const PhysT<float>& batch_phys(const BatchInst& I, const PhysT<float>*)
{
    return I.kf;
}

// Work-item dispenser of the batched launches: one counter per XCD share of
// the items and a count of finished workgroups, each in its own 128-byte
// line.  The last workgroup of a launch to finish zeroes them all, so every
// launch starts from zero without a memset (graph replays included).
constexpr int SCHED_STRIDE = 32;
constexpr int SCHED_WORDS = 9 * SCHED_STRIDE;

// Substep STAGE of every problem of a batch with its own device time step.
// Persistent: a grid sized to the resident workgroups walks the work items
// (all tiles and z-chunks of all problems, problem by problem).  Items are
// split into eight contiguous shares, one per XCD; workgroup b runs on XCD
// b % 8 and draws the next item of its XCD's share from that share's
// counter, so neighbouring tiles of a problem meet in one L2 and cheap and
// dear items (ragged tiles, short last chunks) even out over the
// workgroups.  Once its own share is drawn out it draws from the other
// XCDs' shares in turn.  Each item is exactly the work of one workgroup of
// stage_kernel, whichever workgroup runs it, so a problem advanced in a
// batch and alone with the same tile shape and chunk give bit-identical
// results.
template <typename T, int TX, int TY, int STAGE, bool RATE>
__global__ void __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(StageOcc<T>::waves)))
batch_stage_kernel(const BatchInst* __restrict__ insts, int count, int total, int parity,
                   double t_end, unsigned int* __restrict__ sched)
{
    __shared__ int s_item;
    const int tid = threadIdx.x;
    const int xcd = blockIdx.x & 7;
    int tried = 0;  // shares found empty so far (thread 0 only)
    for (;;) {
        if (tid == 0) {
            int next = -1;
            while (tried < 8) {
                const int s = (xcd + tried) & 7;
                const long long beg = (long long)total * s / 8, end = (long long)total * (s + 1) / 8;
                const unsigned int k = atomicAdd(&sched[s * SCHED_STRIDE], 1u);
                if (beg + k < end) {
                    next = (int)(beg + k);
                    break;
                }
                ++tried;
            }
            s_item = next;
        }
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);  // the same in every lane
        if (item < 0) break;
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (insts[mid].item0 <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
        const BatchInst& I = insts[lo];
        const Geom g = I.g;
        const int local = item - I.item0;
        const int ntile = g.ntx * g.nty;
        const int kc = local / ntile, tile = local - kc * ntile;
        const int tiy = tile / g.ntx, tix = tile - tiy * g.ntx;
        DevState* st = I.st;
        const Phys& K = I.kd;
        const PhysT<T>& kt = batch_phys(I, (const PhysT<T>*)nullptr);

        const double rate = __longlong_as_double((long long)st->rate[parity]);
        const double t_now = st->t[parity];
        double dt = K.cfl / rate;
        if (t_end > 0.0) {
            if (!(t_now < t_end)) dt = 0.0;
            else if (t_now + dt > t_end) dt = t_end - t_now;
        }
        if (STAGE == 1 && local == 0 && tid == 0) {
            st->t[parity ^ 1] = t_now + dt;
            st->rate[parity ^ 1] = 0ull;
        }
        T* U = (T*)I.U;
        T* U1 = (T*)I.U1;
        T* C = (sizeof(T) == 4) ? U + NV * g.field : nullptr;
        T* D0 = (sizeof(T) == 4) ? U1 + NV * g.field : nullptr;
        bool bad = false;
        double rmax = 0.0;
        if (STAGE == 1)
            stage_tile<T, TX, TY, 1, false, false>(U, U, U1, nullptr, D0, g, kt, K, tix, tiy, kc, dt,
                                                   bad, rmax);
        else
            stage_tile<T, TX, TY, 2, RATE, false>(U1, U, U, C, D0, g, kt, K, tix, tiy, kc, dt, bad,
                                                  rmax);
        if (__any(bad) && (tid & 63) == 0) atomicOr(&st->flags, 1u);
        if (RATE) {
            for (int off = 32; off > 0; off >>= 1) rmax = __builtin_fmax(rmax, __shfl_xor(rmax, off));
            if ((tid & 63) == 0)
                atomicMax(&st->rate[parity ^ 1], (unsigned long long)__double_as_longlong(rmax));
        }
        __syncthreads();  // the next item reuses the LDS and s_item
    }
    // Every draw of this workgroup has returned before its finish is
    // counted; the last to finish has seen every other's, so no draw of this
    // launch is still in flight when it zeroes the words.
    if (tid == 0) {
        __threadfence();
        if (atomicAdd(&sched[8 * SCHED_STRIDE], 1u) == gridDim.x - 1) {
            for (int s = 0; s < 9; ++s) atomicExch(&sched[s * SCHED_STRIDE], 0u);
        }
    }
}

__global__ void clear_words_kernel(unsigned int* __restrict__ w, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) w[i] = 0u;
}

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

// Conserved totals in FP64: a running (sum, error) pair per field, the error
// collected by the exact TwoSum transformation (Knuth), so each total is
// the rounded exact sum up to second-order terms.  The partition of cells
// over threads and the combining tree are fixed, so the result is
// deterministic.  For the FP32 form each cell's value is head - compensation,
// exact in FP64.
__device__ __forceinline__ void two_sum_add(double& s, double& c, double x)
{
    double t = s + x;
    double bp = t - s;
    c += (s - (t - bp)) + (x - bp);
    s = t;
}

__device__ __forceinline__ void pair_add(double& s, double& c, double s2, double c2)
{
    two_sum_add(s, c, s2);
    c += c2;
}

template <typename T>
__global__ void __launch_bounds__(RED_THREADS)
totals_partial_kernel(const T* __restrict__ U, const T* __restrict__ C, long long ncell,
                      double* __restrict__ partial)
{
    __shared__ double red[2 * NV][RED_THREADS / 64];
    double s[NV], c[NV];
#pragma unroll
    for (int f = 0; f < NV; ++f) s[f] = c[f] = 0.0;
    for (long long i = (long long)blockIdx.x * RED_THREADS + threadIdx.x; i < ncell;
         i += (long long)gridDim.x * RED_THREADS) {
#pragma unroll
        for (int f = 0; f < NV; ++f) {
            double x = (double)U[f * ncell + i];
            if (C) x -= (double)C[f * ncell + i];
            two_sum_add(s[f], c[f], x);
        }
    }
#pragma unroll
    for (int f = 0; f < NV; ++f) {
        for (int off = 32; off > 0; off >>= 1) {
            double s2 = __shfl_xor(s[f], off), c2 = __shfl_xor(c[f], off);
            pair_add(s[f], c[f], s2, c2);
        }
        if ((threadIdx.x & 63) == 0) {
            red[2 * f][threadIdx.x >> 6] = s[f];
            red[2 * f + 1][threadIdx.x >> 6] = c[f];
        }
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int f = threadIdx.x;
        double S = red[2 * f][0], Cc = red[2 * f + 1][0];
        for (int w = 1; w < RED_THREADS / 64; ++w) pair_add(S, Cc, red[2 * f][w], red[2 * f + 1][w]);
        partial[(long long)blockIdx.x * 2 * NV + 2 * f] = S;
        partial[(long long)blockIdx.x * 2 * NV + 2 * f + 1] = Cc;
    }
}

// Second pass: one wave per field combines the partial pairs of all blocks
// in a fixed order and stores sum + error into tot[f].
__global__ void __launch_bounds__(64 * NV)
totals_final_kernel(const double* __restrict__ partial, int n, DevState* __restrict__ st)
{
    const int f = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double s = 0.0, c = 0.0;
    for (int b = lane; b < n; b += 64) pair_add(s, c, partial[2 * NV * b + 2 * f], partial[2 * NV * b + 2 * f + 1]);
    for (int off = 32; off > 0; off >>= 1) {
        double s2 = __shfl_xor(s, off), c2 = __shfl_xor(c, off);
        pair_add(s, c, s2, c2);
    }
    if (lane == 0) st->tot[f] = s + c;
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

__global__ void set_time_kernel(DevState* st, int parity, double t) { st->t[parity] = t; }

__global__ void clear_flags_kernel(DevState* st) { st->flags = 0u; }

}  // namespace gs

// ===========================================================================
// Host side
// ===========================================================================

using namespace gs;

namespace {

thread_local std::string g_create_error;

enum { K_STAGE1 = 0, K_STAGE2 = 1, K_RATE = 2, K_COUNT = 3 };

}  // namespace

struct gs_fluid {
    int nx, ny, nz;
    double h[3];
    double gamma, cfl;
    int bc;
    int dtype;             // GS_F64 or GS_F32
    size_t esize;          // bytes per state element
    int device;
    hipStream_t stream;
    void* U1;              // first-substep result (workspace)
    double* partial;       // reduction partials
    DevState* st;          // device words
    DevState* host_st;     // pinned host mirror for waiting calls
    int parity;
    int tile_y, chunk_z;   // launch shape (0 = default)
    std::string err;
    bool profile;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used[K_COUNT];
};

namespace {

int fail(gs_fluid* h, int code, const std::string& msg)
{
    if (h)
        h->err = msg;
    else
        g_create_error = msg;
    return code;
}

int hip_fail(gs_fluid* h, hipError_t e, const char* what)
{
    return fail(h, GS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

Phys make_phys(const gs_fluid* h)
{
    Phys k;
    k.gamma = h->gamma;
    k.gm1 = h->gamma - 1.0;
    k.inv_gm1 = 1.0 / (h->gamma - 1.0);
    for (int d = 0; d < 3; ++d) k.inv_h[d] = 1.0 / h->h[d];
    k.cfl = h->cfl;
    return k;
}

// The FP64 constants rounded to FP32 for the FP32 form's flux arithmetic.
PhysT<float> make_phys32(const gs_fluid* h)
{
    const Phys d = make_phys(h);
    PhysT<float> k;
    k.gamma = (float)d.gamma;
    k.gm1 = (float)d.gm1;
    k.inv_gm1 = (float)d.inv_gm1;
    for (int a = 0; a < 3; ++a) k.inv_h[a] = (float)d.inv_h[a];
    k.cfl = (float)d.cfl;
    return k;
}

template <typename T>
PhysT<T> phys_t(const gs_fluid* h);
template <>
PhysT<double> phys_t<double>(const gs_fluid* h) { return make_phys(h); }
template <>
PhysT<float> phys_t<float>(const gs_fluid* h) { return make_phys32(h); }

struct Launch {
    Geom g;
    int tx, ty;
    int blocks;
};

Launch make_launch(const gs_fluid* h)
{
    Launch L;
    // default tile rows span one 128-byte cache line per field: 16 doubles
    // or 32 floats
    L.ty = (h->tile_y != 0) ? h->tile_y : (h->dtype == GS_F32 ? 8 : 16);
    L.tx = 256 / L.ty;
    Geom& g = L.g;
    g.nx = h->nx;
    g.ny = h->ny;
    g.nz = h->nz;
    g.periodic = (h->bc == GS_BC_PERIODIC);
    g.plane = h->nx * h->ny;
    g.field = (long long)h->nx * h->ny * h->nz;
    g.ntx = (h->nx + L.tx - 1) / L.tx;
    g.nty = (h->ny + L.ty - 1) / L.ty;
    const int ntile = g.ntx * g.nty;
    int kz = h->chunk_z;
    if (kz <= 0) {
        // aim for at least 2048 workgroups (several per CU slot) with chunks
        // of 8 to 64 planes: shorter chunks keep the workgroups that share
        // halo lines closer together in z (fewer L2 misses), longer ones
        // waste less on the 4 planes each chunk re-reads.  FP32: 4096
        // workgroups and at most 32 planes (its substeps are shorter and its
        // second substep is bound by HBM: 24 to 32 planes measured 2-5%
        // faster than 64 at 512^3; for FP64 16 to 64 planes are within 1%)
        const bool f32 = h->dtype == GS_F32;
        const long long want_wg = f32 ? 4096 : 2048;
        long long want_chunks = (want_wg + ntile - 1) / ntile;
        kz = (int)((h->nz + want_chunks - 1) / want_chunks);
        const int kmax = f32 ? 32 : 64;
        if (kz > kmax) kz = kmax;
        if (kz < 8) kz = 8;
    }
    if (kz > h->nz) kz = h->nz;
    g.kz = kz;
    g.nchunk = (h->nz + kz - 1) / kz;
    g.band = (ntile % 8 == 0) ? ntile / 8 : 0;
    L.blocks = ntile * g.nchunk;
    return L;
}

hipEvent_t take_event(gs_fluid* h)
{
    if (!h->ev_pool.empty()) {
        hipEvent_t e = h->ev_pool.back();
        h->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records a start event if profiling; returns it (or null).
hipEvent_t prof_begin(gs_fluid* h)
{
    if (!h->profile) return nullptr;
    hipEvent_t e = take_event(h);
    if (e) (void)hipEventRecord(e, h->stream);
    return e;
}

void prof_end(gs_fluid* h, int kernel, hipEvent_t start)
{
    if (!h->profile || !start) return;
    hipEvent_t e = take_event(h);
    if (!e) return;
    (void)hipEventRecord(e, h->stream);
    h->ev_used[kernel].push_back({start, e});
}

// One substep launch.  FP32 form: C is the compensation of Un (stage 2) and
// D the first substep's increment (written by stage 1, read by stage 2);
// FP64 form: both null.
template <typename T, int TX, int TY>
hipError_t launch_stage_t(gs_fluid* h, const Launch& L, int stage, bool devdt, bool rate,
                          const T* Uin, const T* Un, T* Uout, T* C, T* D, double dt_host,
                          double t_end, double* dt_log, int step)
{
    const PhysT<T> kt = phys_t<T>(h);
    const Phys kd = make_phys(h);
    dim3 grid(L.blocks), block(TX * TY);
    // non-temporal hints on meshes whose state does not stay in the
    // last-level cache between the substeps
    const bool nth = (double)NV * L.g.field * sizeof(T) >= 128.0 * 1024 * 1024;
#define GS_LAUNCH(S_, D_, R_)                                                                     \
    do {                                                                                          \
        if (nth)                                                                                  \
            hipLaunchKernelGGL((stage_kernel<T, TX, TY, S_, D_, R_, true>), grid, block, 0,       \
                               h->stream, Uin, Un, Uout, C, D, L.g, kt, kd, h->st, h->parity,     \
                               dt_host, t_end, dt_log, step);                                     \
        else                                                                                      \
            hipLaunchKernelGGL((stage_kernel<T, TX, TY, S_, D_, R_, false>), grid, block, 0,      \
                               h->stream, Uin, Un, Uout, C, D, L.g, kt, kd, h->st, h->parity,     \
                               dt_host, t_end, dt_log, step);                                     \
    } while (0)
    if (stage == 1) {
        if (devdt) GS_LAUNCH(1, true, false);
        else GS_LAUNCH(1, false, false);
    } else {
        if (devdt) {
            if (rate) GS_LAUNCH(2, true, true);
            else GS_LAUNCH(2, true, false);
        } else {
            if (rate) GS_LAUNCH(2, false, true);
            else GS_LAUNCH(2, false, false);
        }
    }
#undef GS_LAUNCH
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stage(gs_fluid* h, int stage, bool devdt, bool rate, const T* Uin, const T* Un,
                        T* Uout, T* C, T* D, double dt_host, double t_end, double* dt_log,
                        int step)
{
    Launch L = make_launch(h);
    hipEvent_t ev = prof_begin(h);
    hipError_t e;
    if (L.ty == 8)
        e = launch_stage_t<T, 32, 8>(h, L, stage, devdt, rate, Uin, Un, Uout, C, D, dt_host,
                                     t_end, dt_log, step);
    else
        e = launch_stage_t<T, 16, 16>(h, L, stage, devdt, rate, Uin, Un, Uout, C, D, dt_host,
                                      t_end, dt_log, step);
    prof_end(h, stage == 1 ? K_STAGE1 : K_STAGE2, ev);
    return e;
}

int reduction_blocks(const gs_fluid* h)
{
    const long long ncell = (long long)h->nx * h->ny * h->nz;
    long long want = (ncell + RED_THREADS - 1) / RED_THREADS;
    return (int)(want < RED_BLOCKS ? want : RED_BLOCKS);
}

hipError_t launch_rate(gs_fluid* h, const void* U, unsigned long long* dst)
{
    const long long ncell = (long long)h->nx * h->ny * h->nz;
    const int blocks = reduction_blocks(h);
    hipEvent_t ev = prof_begin(h);
    if (h->dtype == GS_F32)
        hipLaunchKernelGGL(rate_partial_kernel<float>, dim3(blocks), dim3(RED_THREADS), 0,
                           h->stream, (const float*)U, ncell, make_phys(h), h->partial, h->st);
    else
        hipLaunchKernelGGL(rate_partial_kernel<double>, dim3(blocks), dim3(RED_THREADS), 0,
                           h->stream, (const double*)U, ncell, make_phys(h), h->partial, h->st);
    hipLaunchKernelGGL(rate_final_kernel, dim3(1), dim3(RED_THREADS), 0, h->stream, h->partial,
                       blocks, dst);
    prof_end(h, K_RATE, ev);
    return hipGetLastError();
}

hipError_t launch_totals(gs_fluid* h, const void* U)
{
    const long long ncell = (long long)h->nx * h->ny * h->nz;
    const int blocks = reduction_blocks(h);
    if (h->dtype == GS_F32) {
        const float* u = (const float*)U;
        hipLaunchKernelGGL(totals_partial_kernel<float>, dim3(blocks), dim3(RED_THREADS), 0,
                           h->stream, u, u + NV * ncell, ncell, h->partial);
    } else {
        hipLaunchKernelGGL(totals_partial_kernel<double>, dim3(blocks), dim3(RED_THREADS), 0,
                           h->stream, (const double*)U, (const double*)nullptr, ncell, h->partial);
    }
    hipLaunchKernelGGL(totals_final_kernel, dim3(1), dim3(64 * NV), 0, h->stream, h->partial,
                       blocks, h->st);
    return hipGetLastError();
}

// Waits for the stream and copies the device words to the pinned mirror;
// reports (once) a pending non-physical flag.
int sync_state(gs_fluid* h)
{
    hipError_t e = hipMemcpyAsync(h->host_st, h->st, sizeof(DevState), hipMemcpyDeviceToHost,
                                  h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "hipMemcpyAsync");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
    if (h->host_st->flags) {
        hipLaunchKernelGGL(clear_flags_kernel, dim3(1), dim3(1), 0, h->stream, h->st);
        return fail(h, GS_ERR_NONPHYSICAL,
                    "non-physical state (rho or p not positive, or not finite) was read");
    }
    return GS_OK;
}

bool aligned_to(const void* p, size_t a) { return ((uintptr_t)p & (a - 1)) == 0; }
bool aligned8(const void* p) { return aligned_to(p, 8); }

// Device address of a word of the handle's DevState.
unsigned long long* rate_slot(gs_fluid* h, int which)
{
    char* base = (char*)h->st;
    if (which < 0) return (unsigned long long*)(base + offsetof(DevState, rate_dt));
    return (unsigned long long*)(base + offsetof(DevState, rate) + which * sizeof(unsigned long long));
}

size_t elem_size(int dtype) { return dtype == GS_F32 ? sizeof(float) : sizeof(double); }

// Substep workspace: U(1); the FP32 form also keeps the first increment.
long long state_work_bytes(long long ncell, int dtype)
{
    return ncell * NV * (long long)elem_size(dtype) * (dtype == GS_F32 ? 2 : 1);
}

// Checks the state pointer of a call: present and aligned to the element.
int check_state(gs_fluid* h, const void* U)
{
    if (!U || !aligned_to(U, h->esize))
        return fail(h, GS_ERR_ARG, "U is NULL or not aligned to its element size");
    return GS_OK;
}

// Work arrays of one step: the compensation half of the caller's FP32 state,
// and the first substep's increment (second half of the FP32 workspace).
template <typename T>
struct StepArrays {
    T* u1;
    T* comp;
    T* d0;
};

template <typename T>
StepArrays<T> step_arrays(gs_fluid* h, T* u)
{
    const long long ncell = (long long)h->nx * h->ny * h->nz;
    StepArrays<T> a;
    a.u1 = (T*)h->U1;
    a.comp = (sizeof(T) == 4) ? u + NV * ncell : nullptr;
    a.d0 = (sizeof(T) == 4) ? a.u1 + NV * ncell : nullptr;
    return a;
}

template <typename T>
hipError_t step_t(gs_fluid* h, T* u, double dt)
{
    StepArrays<T> a = step_arrays(h, u);
    hipError_t e = launch_stage<T>(h, 1, false, false, u, u, a.u1, nullptr, a.d0, dt, 0.0,
                                   nullptr, 0);
    if (e == hipSuccess)
        e = launch_stage<T>(h, 2, false, false, a.u1, u, u, a.comp, a.d0, dt, 0.0, nullptr, 0);
    return e;
}

template <typename T>
hipError_t advance_t(gs_fluid* h, T* u, int nsteps, double t_end, double* dt_log)
{
    StepArrays<T> a = step_arrays(h, u);
    hipError_t e = launch_rate(h, u, rate_slot(h, h->parity));
    for (int s = 0; s < nsteps && e == hipSuccess; ++s) {
        e = launch_stage<T>(h, 1, true, false, u, u, a.u1, nullptr, a.d0, 0.0, t_end, dt_log, s);
        if (e == hipSuccess)
            e = launch_stage<T>(h, 2, true, true, a.u1, u, u, a.comp, a.d0, 0.0, t_end, dt_log, s);
        h->parity ^= 1;
    }
    return e;
}

}  // namespace

extern "C" {

long long gs_fluid_workspace_bytes(int nx, int ny, int nz, int dtype)
{
    if (nx < 1 || ny < 1 || nz < 1 || (dtype != GS_F64 && dtype != GS_F32)) return -1;
    long long ncell = (long long)nx * ny * nz;
    return state_work_bytes(ncell, dtype) + RED_BLOCKS * 2 * NV * (long long)sizeof(double) +
           (long long)sizeof(DevState);
}

int gs_fluid_create(int nx, int ny, int nz, double dx, double dy, double dz, double gamma,
                    double cfl, int bc, int dtype, void* stream, gs_fluid** out)
{
    g_create_error.clear();
    if (!out) return fail(nullptr, GS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return fail(nullptr, GS_ERR_ARG, "mesh sizes must be >= 1");
    if ((long long)nx * ny > (1LL << 30) ||
        (long long)nx * ny * nz * NV > (1LL << 40))
        return fail(nullptr, GS_ERR_ARG, "mesh too large");
    if (!finite_pos(dx) || !finite_pos(dy) || !finite_pos(dz))
        return fail(nullptr, GS_ERR_ARG, "cell widths must be finite and > 0");
    if (!std::isfinite(gamma) || !(gamma > 1.0))
        return fail(nullptr, GS_ERR_ARG, "gamma must be finite and > 1");
    if (!std::isfinite(cfl) || !(cfl > 0.0) || cfl > 1.0)
        return fail(nullptr, GS_ERR_ARG, "cfl must be in (0, 1]");
    if (bc != GS_BC_OUTFLOW && bc != GS_BC_PERIODIC)
        return fail(nullptr, GS_ERR_ARG, "unknown boundary kind");
    if (dtype != GS_F64 && dtype != GS_F32)
        return fail(nullptr, GS_ERR_ARG, "unknown dtype (GS_F64 or GS_F32)");

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, GS_ERR_HIP,
                    std::string("built for gfx950, device is ") + prop.gcnArchName);

    gs_fluid* h = new gs_fluid();
    h->nx = nx;
    h->ny = ny;
    h->nz = nz;
    h->h[0] = dx;
    h->h[1] = dy;
    h->h[2] = dz;
    h->gamma = gamma;
    h->cfl = cfl;
    h->bc = bc;
    h->dtype = dtype;
    h->esize = elem_size(dtype);
    h->device = dev;
    h->stream = (hipStream_t)stream;
    h->U1 = nullptr;
    h->partial = nullptr;
    h->st = nullptr;
    h->host_st = nullptr;
    h->parity = 0;
    h->tile_y = 0;
    h->chunk_z = 0;
    h->profile = false;

    const size_t state_bytes = (size_t)state_work_bytes((long long)nx * ny * nz, dtype);
    if ((e = hipMalloc(&h->U1, state_bytes)) != hipSuccess ||
        (e = hipMalloc((void**)&h->partial, RED_BLOCKS * 2 * NV * sizeof(double))) != hipSuccess ||
        (e = hipMalloc((void**)&h->st, sizeof(DevState))) != hipSuccess ||
        (e = hipHostMalloc((void**)&h->host_st, sizeof(DevState), hipHostMallocDefault)) !=
            hipSuccess) {
        int r = hip_fail(nullptr, e, "allocation");
        gs_fluid_destroy(h);
        return r;
    }
    hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(1), 0, h->stream, h->st);
    if ((e = hipGetLastError()) != hipSuccess) {
        int r = hip_fail(nullptr, e, "init kernel");
        gs_fluid_destroy(h);
        return r;
    }
    *out = h;
    return GS_OK;
}

int gs_fluid_dt(gs_fluid* h, const void* U, double* dt_out)
{
    if (!h) return fail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (check_state(h, U) != GS_OK) return GS_ERR_ARG;
    if (!dt_out) return fail(h, GS_ERR_ARG, "dt_out is NULL");
    hipError_t e = launch_rate(h, U, rate_slot(h, -1));
    if (e != hipSuccess) return hip_fail(h, e, "dt reduction launch");
    int r = sync_state(h);
    if (r != GS_OK) return r;
    double rate = __builtin_bit_cast(double, h->host_st->rate_dt);
    if (!(rate > 0.0) || !std::isfinite(rate))
        return fail(h, GS_ERR_NONPHYSICAL, "signal rate is not positive and finite");
    *dt_out = h->cfl / rate;
    return GS_OK;
}

int gs_fluid_step(gs_fluid* h, void* U, double dt)
{
    if (!h) return fail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (check_state(h, U) != GS_OK) return GS_ERR_ARG;
    if (!finite_pos(dt)) return fail(h, GS_ERR_ARG, "dt must be finite and > 0");
    hipError_t e = (h->dtype == GS_F32) ? step_t(h, (float*)U, dt) : step_t(h, (double*)U, dt);
    if (e != hipSuccess) return hip_fail(h, e, "stage launch");
    h->parity ^= 1;
    return GS_OK;
}

int gs_fluid_advance(gs_fluid* h, void* U, int nsteps, double t_end, double* dt_log)
{
    if (!h) return fail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (check_state(h, U) != GS_OK) return GS_ERR_ARG;
    if (nsteps < 0) return fail(h, GS_ERR_ARG, "nsteps must be >= 0");
    if (!std::isfinite(t_end) || t_end < 0.0) return fail(h, GS_ERR_ARG, "t_end must be finite and >= 0");
    if (dt_log && !aligned8(dt_log)) return fail(h, GS_ERR_ARG, "dt_log not 8-byte aligned");
    if (nsteps == 0) return GS_OK;
    hipError_t e = (h->dtype == GS_F32) ? advance_t(h, (float*)U, nsteps, t_end, dt_log)
                                        : advance_t(h, (double*)U, nsteps, t_end, dt_log);
    if (e != hipSuccess) return hip_fail(h, e, "advance launch");
    return GS_OK;
}

int gs_fluid_totals(gs_fluid* h, const void* U, double* totals)
{
    if (!h) return fail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (check_state(h, U) != GS_OK) return GS_ERR_ARG;
    if (!totals) return fail(h, GS_ERR_ARG, "totals is NULL");
    hipError_t e = launch_totals(h, U);
    if (e != hipSuccess) return hip_fail(h, e, "totals launch");
    int r = sync_state(h);
    for (int f = 0; f < NV; ++f) totals[f] = h->host_st->tot[f];
    return r;
}

int gs_fluid_sync(gs_fluid* h)
{
    if (!h) return fail(nullptr, GS_ERR_ARG, "handle is NULL");
    return sync_state(h);
}

int gs_fluid_get_time(gs_fluid* h, double* t_out)
{
    if (!h) return fail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (!t_out) return fail(h, GS_ERR_ARG, "t_out is NULL");
    int r = sync_state(h);
    *t_out = h->host_st->t[h->parity];
    return r;
}

int gs_fluid_set_time(gs_fluid* h, double t)
{
    if (!h) return fail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (!std::isfinite(t)) return fail(h, GS_ERR_ARG, "t must be finite");
    hipLaunchKernelGGL(set_time_kernel, dim3(1), dim3(1), 0, h->stream, h->st, h->parity, t);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GS_OK : hip_fail(h, e, "set_time");
}

int gs_fluid_set_stream(gs_fluid* h, void* stream)
{
    if (!h) return fail(nullptr, GS_ERR_ARG, "handle is NULL");
    h->stream = (hipStream_t)stream;
    return GS_OK;
}

int gs_fluid_set_launch(gs_fluid* h, int tile_y, int chunk_z)
{
    if (!h) return fail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (tile_y != 0 && tile_y != 8 && tile_y != 16)
        return fail(h, GS_ERR_ARG, "tile_y must be 0, 8 or 16");
    if (chunk_z < 0) return fail(h, GS_ERR_ARG, "chunk_z must be >= 0");
    h->tile_y = tile_y;
    h->chunk_z = chunk_z;
    return GS_OK;
}

int gs_fluid_profile(gs_fluid* h, int enable)
{
    if (!h) return fail(nullptr, GS_ERR_ARG, "handle is NULL");
    h->profile = enable != 0;
    return GS_OK;
}

int gs_fluid_kernel_ms(gs_fluid* h, int kernel, double* total_ms, int* launches)
{
    if (!h) return fail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (kernel < 0 || kernel >= K_COUNT) return fail(h, GS_ERR_ARG, "kernel must be 0, 1 or 2");
    if (!total_ms || !launches) return fail(h, GS_ERR_ARG, "output pointer is NULL");
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
    double sum = 0.0;
    int n = 0;
    for (auto& pr : h->ev_used[kernel]) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
            sum += ms;
            ++n;
        }
        h->ev_pool.push_back(pr.first);
        h->ev_pool.push_back(pr.second);
    }
    h->ev_used[kernel].clear();
    *total_ms = sum;
    *launches = n;
    return GS_OK;
}

void gs_fluid_destroy(gs_fluid* h)
{
    if (!h) return;
    for (auto& v : h->ev_used)
        for (auto& pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    if (h->U1) (void)hipFree(h->U1);
    if (h->partial) (void)hipFree(h->partial);
    if (h->st) (void)hipFree(h->st);
    if (h->host_st) (void)hipHostFree(h->host_st);
    delete h;
}

const char* gs_fluid_last_error(const gs_fluid* h)
{
    return h ? h->err.c_str() : g_create_error.c_str();
}

}  // extern "C"

// ===========================================================================
// Batched form: host side
// ===========================================================================

#include "gs_batch.h"

#include <array>
#include <fstream>
#include <sstream>

namespace {

thread_local std::string g_batch_create_error;

}  // namespace

struct gs_batch {
    int count;
    int dtype;
    size_t esize;
    int bc;
    double gamma, cfl;
    std::vector<std::array<int, 3>> dims;
    std::vector<void*> states;
    void* pool;                 // workspaces of all problems
    std::vector<size_t> pool_off;
    DevState* st;               // count blocks of device words
    DevState* tune_st;          // device words for autotuning runs
    DevState* host_st;          // pinned mirror of st
    double* partial;            // reduction partials, RED_BLOCKS per problem
    BatchInst* insts_dev;       // device table for the live states
    BatchInst* tune_dev;        // device table for scratch states
    unsigned int* sched;        // work-item dispenser (SCHED_WORDS words)
    int total_items;
    int tile_y, chunk_z;
    int grid[2];                // persistent grid of substep 1 and 2
    hipStream_t user_stream, stream;
    hipEvent_t ev_in, ev_out;
    hipGraphExec_t exec[2];
    bool graphs_valid;
    double graph_t_end;
    int parity;
    std::string err;
};

namespace {

int bfail(gs_batch* h, int code, const std::string& msg)
{
    if (h)
        h->err = msg;
    else
        g_batch_create_error = msg;
    return code;
}

int bhip(gs_batch* h, hipError_t e, const char* what)
{
    return bfail(h, GS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int batch_tile_y(const gs_batch* h) { return h->tile_y ? h->tile_y : (h->dtype == GS_F32 ? 8 : 16); }

// FP64 constants of problem i: cell width 1/max(n), inverted as the
// single-problem path inverts its widths, so both take identical steps
Phys batch_phys64(const gs_batch* h, int i)
{
    const double hw = 1.0 / std::max(h->dims[i][0], std::max(h->dims[i][1], h->dims[i][2]));
    Phys k;
    k.gamma = h->gamma;
    k.gm1 = h->gamma - 1.0;
    k.inv_gm1 = 1.0 / (h->gamma - 1.0);
    for (int d = 0; d < 3; ++d) k.inv_h[d] = 1.0 / hw;
    k.cfl = h->cfl;
    return k;
}

// Per-problem geometry, constants and item ranges for the current launch
// shape, with states `states` and device words `st`.
std::vector<BatchInst> batch_table(const gs_batch* h, const std::vector<void*>& states, DevState* st,
                                   int* total)
{
    const int ty = batch_tile_y(h), tx = 256 / ty;
    std::vector<BatchInst> v(h->count);
    int item = 0;
    for (int i = 0; i < h->count; ++i) {
        BatchInst& I = v[i];
        std::memset((void*)&I, 0, sizeof(I));
        const int nx = h->dims[i][0], ny = h->dims[i][1], nz = h->dims[i][2];
        Geom& g = I.g;
        g.nx = nx;
        g.ny = ny;
        g.nz = nz;
        g.periodic = h->bc == GS_BC_PERIODIC;
        g.plane = nx * ny;
        g.field = (long long)nx * ny * nz;
        g.ntx = (nx + tx - 1) / tx;
        g.nty = (ny + ty - 1) / ty;
        const int ntile = g.ntx * g.nty;
        int kz = h->chunk_z;
        if (kz <= 0) {
            // a few hundred items per problem at most sizes: chunks of 8 to
            // 64 planes, aiming at 64 items
            long long want = (64 + ntile - 1) / ntile;
            kz = (int)((nz + want - 1) / want);
            if (kz > 64) kz = 64;
            if (kz < 8) kz = 8;
        }
        if (kz > nz) kz = nz;
        g.kz = kz;
        g.nchunk = (nz + kz - 1) / kz;
        g.band = 0;
        I.kd = batch_phys64(h, i);
        const Phys& k = I.kd;
        I.kf.gamma = (float)k.gamma;
        I.kf.gm1 = (float)k.gm1;
        I.kf.inv_gm1 = (float)k.inv_gm1;
        for (int d = 0; d < 3; ++d) I.kf.inv_h[d] = (float)k.inv_h[d];
        I.kf.cfl = (float)k.cfl;
        I.U = states[i];
        I.U1 = (char*)h->pool + h->pool_off[i];
        I.st = st + i;
        I.item0 = item;
        I.items = ntile * g.nchunk;
        item += I.items;
    }
    *total = item;
    return v;
}

template <typename T, int TX, int TY>
hipError_t batch_launch_t(gs_batch* h, const BatchInst* table, int total, int parity, double t_end)
{
    hipLaunchKernelGGL((batch_stage_kernel<T, TX, TY, 1, false>), dim3(h->grid[0]), dim3(TX * TY), 0,
                       h->stream, table, h->count, total, parity, t_end, h->sched);
    hipLaunchKernelGGL((batch_stage_kernel<T, TX, TY, 2, true>), dim3(h->grid[1]), dim3(TX * TY), 0,
                       h->stream, table, h->count, total, parity, t_end, h->sched);
    return hipGetLastError();
}

// one step of every problem: the two substep launches
hipError_t batch_step(gs_batch* h, const BatchInst* table, int total, int parity, double t_end)
{
    const bool f32 = h->dtype == GS_F32;
    if (batch_tile_y(h) == 8)
        return f32 ? batch_launch_t<float, 32, 8>(h, table, total, parity, t_end)
                   : batch_launch_t<double, 32, 8>(h, table, total, parity, t_end);
    return f32 ? batch_launch_t<float, 16, 16>(h, table, total, parity, t_end)
               : batch_launch_t<double, 16, 16>(h, table, total, parity, t_end);
}

template <typename T, int TX, int TY, int STAGE, bool RATE>
int resident_blocks(int cus)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_stage_kernel<T, TX, TY, STAGE, RATE>,
                                                     TX * TY, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return per_cu * cus;
}

// persistent grids: the resident workgroups, a multiple of 8 (one share per
// XCD), at most the item count rounded up to 8
void batch_grids(gs_batch* h)
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    }
    int r1, r2;
    const bool f32 = h->dtype == GS_F32;
    if (batch_tile_y(h) == 8) {
        r1 = f32 ? resident_blocks<float, 32, 8, 1, false>(cus) : resident_blocks<double, 32, 8, 1, false>(cus);
        r2 = f32 ? resident_blocks<float, 32, 8, 2, true>(cus) : resident_blocks<double, 32, 8, 2, true>(cus);
    } else {
        r1 = f32 ? resident_blocks<float, 16, 16, 1, false>(cus) : resident_blocks<double, 16, 16, 1, false>(cus);
        r2 = f32 ? resident_blocks<float, 16, 16, 2, true>(cus) : resident_blocks<double, 16, 16, 2, true>(cus);
    }
    const int cap = ((h->total_items + 7) / 8) * 8;
    h->grid[0] = std::max(8, std::min(cap, (r1 / 8) * 8));
    h->grid[1] = std::max(8, std::min(cap, (r2 / 8) * 8));
}

void drop_graphs(gs_batch* h)
{
    for (int p = 0; p < 2; ++p)
        if (h->exec[p]) {
            (void)hipGraphExecDestroy(h->exec[p]);
            h->exec[p] = nullptr;
        }
    h->graphs_valid = false;
}

int rebuild_table(gs_batch* h)
{
    int total = 0;
    std::vector<BatchInst> t = batch_table(h, h->states, h->st, &total);
    hipError_t e = hipMemcpy(h->insts_dev, t.data(), sizeof(BatchInst) * h->count, hipMemcpyHostToDevice);
    if (e != hipSuccess) return bhip(h, e, "batch table upload");
    h->total_items = total;
    batch_grids(h);
    drop_graphs(h);
    return GS_OK;
}

// reduction of every problem's signal rate into its slot `parity`
hipError_t batch_rates(gs_batch* h, const std::vector<void*>& states, DevState* st, int parity)
{
    for (int i = 0; i < h->count; ++i) {
        const long long ncell = (long long)h->dims[i][0] * h->dims[i][1] * h->dims[i][2];
        long long want = (ncell + RED_THREADS - 1) / RED_THREADS;
        const int blocks = (int)(want < RED_BLOCKS ? want : RED_BLOCKS);
        const Phys k = batch_phys64(h, i);
        double* part = h->partial + (size_t)i * RED_BLOCKS;
        if (h->dtype == GS_F32)
            hipLaunchKernelGGL(rate_partial_kernel<float>, dim3(blocks), dim3(RED_THREADS), 0, h->stream,
                               (const float*)states[i], ncell, k, part, st + i);
        else
            hipLaunchKernelGGL(rate_partial_kernel<double>, dim3(blocks), dim3(RED_THREADS), 0, h->stream,
                               (const double*)states[i], ncell, k, part, st + i);
        char* base = (char*)(st + i);
        hipLaunchKernelGGL(rate_final_kernel, dim3(1), dim3(RED_THREADS), 0, h->stream, part, blocks,
                           (unsigned long long*)(base + offsetof(DevState, rate) +
                                                 parity * sizeof(unsigned long long)));
    }
    return hipGetLastError();
}

hipError_t capture_graphs(gs_batch* h, double t_end)
{
    drop_graphs(h);
    for (int p = 0; p < 2; ++p) {
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        hipError_t el = batch_step(h, h->insts_dev, h->total_items, p, t_end);
        e = hipStreamEndCapture(h->stream, &g);
        if (el != hipSuccess) return el;
        if (e != hipSuccess) return e;
        e = hipGraphInstantiate(&h->exec[p], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return e;
    }
    h->graphs_valid = true;
    h->graph_t_end = t_end;
    return hipSuccess;
}

uint64_t fnv1a(const std::string& s)
{
    uint64_t x = 1469598103934665603ull;
    for (unsigned char c : s) {
        x ^= c;
        x *= 1099511628211ull;
    }
    return x;
}

std::string batch_key(const gs_batch* h)
{
    std::ostringstream o;
    o.precision(17);
    o << "dtype " << h->dtype << " bc " << h->bc << " gamma " << h->gamma << " cfl " << h->cfl << " n "
      << h->count;
    for (auto& d : h->dims) o << " " << d[0] << "x" << d[1] << "x" << d[2];
    std::ostringstream k;
    k << std::hex << fnv1a(o.str());
    return k.str();
}

}  // namespace

extern "C" {

int gs_batch_create(int count, const int* dims, double gamma, double cfl, int bc, int dtype,
                    void* const* states, void* stream, gs_batch** out)
{
    g_batch_create_error.clear();
    if (!out) return bfail(nullptr, GS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (count < 1 || count > (1 << 16)) return bfail(nullptr, GS_ERR_ARG, "count must be in [1, 65536]");
    if (!dims || !states) return bfail(nullptr, GS_ERR_ARG, "dims or states is NULL");
    long long cells = 0;
    for (int i = 0; i < count; ++i) {
        const int nx = dims[3 * i], ny = dims[3 * i + 1], nz = dims[3 * i + 2];
        if (nx < 1 || ny < 1 || nz < 1) return bfail(nullptr, GS_ERR_ARG, "mesh sizes must be >= 1");
        if ((long long)nx * ny > (1LL << 30)) return bfail(nullptr, GS_ERR_ARG, "mesh too large");
        if (!states[i] || ((uintptr_t)states[i] & 15u))
            return bfail(nullptr, GS_ERR_ARG, "a state pointer is NULL or not 16-byte aligned");
        cells += (long long)nx * ny * nz;
    }
    if (cells > (1LL << 34)) return bfail(nullptr, GS_ERR_ARG, "batch too large");
    if (!std::isfinite(gamma) || !(gamma > 1.0)) return bfail(nullptr, GS_ERR_ARG, "gamma must be > 1");
    if (!std::isfinite(cfl) || !(cfl > 0.0) || cfl > 1.0) return bfail(nullptr, GS_ERR_ARG, "cfl must be in (0, 1]");
    if (bc != GS_BC_OUTFLOW && bc != GS_BC_PERIODIC) return bfail(nullptr, GS_ERR_ARG, "unknown boundary kind");
    if (dtype != GS_F64 && dtype != GS_F32) return bfail(nullptr, GS_ERR_ARG, "unknown dtype");

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return bhip(nullptr, e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return bhip(nullptr, e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return bfail(nullptr, GS_ERR_HIP, std::string("built for gfx950, device is ") + prop.gcnArchName);

    gs_batch* h = new gs_batch();
    h->count = count;
    h->dtype = dtype;
    h->esize = elem_size(dtype);
    h->bc = bc;
    h->gamma = gamma;
    h->cfl = cfl;
    h->dims.resize(count);
    h->states.assign(states, states + count);
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        h->dims[i] = {dims[3 * i], dims[3 * i + 1], dims[3 * i + 2]};
        h->pool_off.push_back(off);
        const long long ncell = (long long)dims[3 * i] * dims[3 * i + 1] * dims[3 * i + 2];
        off += ((size_t)state_work_bytes(ncell, dtype) + 255) / 256 * 256;
    }
    h->user_stream = (hipStream_t)stream;
    h->exec[0] = h->exec[1] = nullptr;
    if ((e = hipMalloc(&h->pool, off)) != hipSuccess ||
        (e = hipMalloc((void**)&h->st, sizeof(DevState) * count)) != hipSuccess ||
        (e = hipMalloc((void**)&h->tune_st, sizeof(DevState) * count)) != hipSuccess ||
        (e = hipMalloc((void**)&h->partial, sizeof(double) * RED_BLOCKS * count)) != hipSuccess ||
        (e = hipMalloc((void**)&h->insts_dev, sizeof(BatchInst) * count)) != hipSuccess ||
        (e = hipMalloc((void**)&h->tune_dev, sizeof(BatchInst) * count)) != hipSuccess ||
        (e = hipMalloc((void**)&h->sched, sizeof(unsigned int) * SCHED_WORDS)) != hipSuccess ||
        (e = hipHostMalloc((void**)&h->host_st, sizeof(DevState) * count, hipHostMallocDefault)) !=
            hipSuccess ||
        (e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming)) != hipSuccess) {
        int r = bhip(nullptr, e, "batch allocation");
        gs_batch_destroy(h);
        return r;
    }
    for (int i = 0; i < count; ++i) {
        hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(1), 0, h->stream, h->st + i);
        hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(1), 0, h->stream, h->tune_st + i);
    }
    hipLaunchKernelGGL(clear_words_kernel, dim3(1), dim3(256), 0, h->stream, h->sched, SCHED_WORDS);
    if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(h->stream)) != hipSuccess) {
        int r = bhip(nullptr, e, "batch init");
        gs_batch_destroy(h);
        return r;
    }
    if (rebuild_table(h) != GS_OK) {
        int r = bfail(nullptr, GS_ERR_HIP, h->err);
        gs_batch_destroy(h);
        return r;
    }
    *out = h;
    return GS_OK;
}

int gs_batch_set_launch(gs_batch* h, int tile_y, int chunk_z)
{
    if (!h) return bfail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (tile_y != 0 && tile_y != 8 && tile_y != 16) return bfail(h, GS_ERR_ARG, "tile_y must be 0, 8 or 16");
    if (chunk_z < 0) return bfail(h, GS_ERR_ARG, "chunk_z must be >= 0");
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return bhip(h, e, "hipStreamSynchronize");
    h->tile_y = tile_y;
    h->chunk_z = chunk_z;
    return rebuild_table(h);
}

int gs_batch_advance(gs_batch* h, int nsteps, double t_end, int use_graph)
{
    if (!h) return bfail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (nsteps < 0) return bfail(h, GS_ERR_ARG, "nsteps must be >= 0");
    if (!std::isfinite(t_end) || t_end < 0.0) return bfail(h, GS_ERR_ARG, "t_end must be finite and >= 0");
    if (nsteps == 0) return GS_OK;
    hipError_t e = hipEventRecord(h->ev_in, h->user_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(h->stream, h->ev_in, 0);
    if (e == hipSuccess) e = batch_rates(h, h->states, h->st, h->parity);
    if (e == hipSuccess && use_graph && (!h->graphs_valid || h->graph_t_end != t_end))
        e = capture_graphs(h, t_end);
    for (int s = 0; s < nsteps && e == hipSuccess; ++s) {
        if (use_graph)
            e = hipGraphLaunch(h->exec[h->parity], h->stream);
        else
            e = batch_step(h, h->insts_dev, h->total_items, h->parity, t_end);
        h->parity ^= 1;
    }
    if (e == hipSuccess) e = hipEventRecord(h->ev_out, h->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(h->user_stream, h->ev_out, 0);
    return e == hipSuccess ? GS_OK : bhip(h, e, "batch advance");
}

int gs_batch_times(gs_batch* h, double* times)
{
    if (!h) return bfail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (!times) return bfail(h, GS_ERR_ARG, "times is NULL");
    hipError_t e = hipMemcpyAsync(h->host_st, h->st, sizeof(DevState) * h->count, hipMemcpyDeviceToHost,
                                  h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return bhip(h, e, "batch times");
    bool bad = false;
    for (int i = 0; i < h->count; ++i) {
        times[i] = h->host_st[i].t[h->parity];
        bad |= h->host_st[i].flags != 0;
    }
    if (bad) {
        for (int i = 0; i < h->count; ++i)
            hipLaunchKernelGGL(clear_flags_kernel, dim3(1), dim3(1), 0, h->stream, h->st + i);
        return bfail(h, GS_ERR_NONPHYSICAL, "non-physical state (rho or p not positive, or not finite) was read");
    }
    return GS_OK;
}

int gs_batch_sync(gs_batch* h)
{
    if (!h) return bfail(nullptr, GS_ERR_ARG, "handle is NULL");
    std::vector<double> t(h->count);
    return gs_batch_times(h, t.data());
}

int gs_batch_autotune(gs_batch* h, const char* cache_path, int* tile_y, int* chunk_z, int* from_cache)
{
    if (!h) return bfail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (!tile_y || !chunk_z || !from_cache) return bfail(h, GS_ERR_ARG, "output is NULL");
    const std::string key = batch_key(h);
    *from_cache = 0;
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k;
            int ty = 0, kz = -1;
            if ((ls >> k >> ty >> kz) && k == key && (ty == 8 || ty == 16) && kz >= 0) {
                int r = gs_batch_set_launch(h, ty, kz);
                if (r != GS_OK) return r;
                *tile_y = ty;
                *chunk_z = kz;
                *from_cache = 1;
                return GS_OK;
            }
        }
    }
    // scratch copies of every state, and the tuning device words
    hipError_t e = hipStreamSynchronize(h->user_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return bhip(h, e, "autotune sync");
    std::vector<void*> scratch(h->count, nullptr);
    auto free_scratch = [&] {
        for (void* p : scratch)
            if (p) (void)hipFree(p);
    };
    for (int i = 0; i < h->count; ++i) {
        const long long ncell = (long long)h->dims[i][0] * h->dims[i][1] * h->dims[i][2];
        const size_t bytes = (size_t)ncell * NV * h->esize * (h->dtype == GS_F32 ? 2 : 1);
        if ((e = hipMalloc(&scratch[i], bytes)) != hipSuccess ||
            (e = hipMemcpyAsync(scratch[i], h->states[i], bytes, hipMemcpyDeviceToDevice, h->stream)) !=
                hipSuccess) {
            free_scratch();
            return bhip(h, e, "autotune scratch");
        }
    }
    const int tiles[2] = {16, 8};
    const int chunks[3] = {16, 32, 64};
    const int saved_ty = h->tile_y, saved_kz = h->chunk_z;
    double best = 1e300;
    int best_ty = batch_tile_y(h), best_kz = h->chunk_z;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    for (int ty : tiles)
        for (int kz : chunks) {
            h->tile_y = ty;
            h->chunk_z = kz;
            int total = 0;
            std::vector<BatchInst> t = batch_table(h, scratch, h->tune_st, &total);
            e = hipMemcpy(h->tune_dev, t.data(), sizeof(BatchInst) * h->count, hipMemcpyHostToDevice);
            if (e != hipSuccess) break;
            h->total_items = total;
            batch_grids(h);
            int par = 0;
            e = batch_rates(h, scratch, h->tune_st, par);
            if (e == hipSuccess) e = batch_step(h, h->tune_dev, total, par, 0.0);  // warm-up
            par ^= 1;
            if (e == hipSuccess) e = hipEventRecord(a, h->stream);
            for (int s = 0; s < 3 && e == hipSuccess; ++s, par ^= 1)
                e = batch_step(h, h->tune_dev, total, par, 0.0);
            if (e == hipSuccess) e = hipEventRecord(b, h->stream);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            if (e != hipSuccess) break;
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, a, b);
            if (ms < best) {
                best = ms;
                best_ty = ty;
                best_kz = kz;
            }
        }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipStreamSynchronize(h->stream);
    free_scratch();
    // the tuning runs may have flagged scratch states; clear their words
    for (int i = 0; i < h->count; ++i)
        hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(1), 0, h->stream, h->tune_st + i);
    if (e != hipSuccess) {
        h->tile_y = saved_ty;
        h->chunk_z = saved_kz;
        rebuild_table(h);
        return bhip(h, e, "autotune run");
    }
    int r = gs_batch_set_launch(h, best_ty, best_kz);
    if (r != GS_OK) return r;
    *tile_y = best_ty;
    *chunk_z = best_kz;
    if (cache_path) {
        std::ofstream o(cache_path, std::ios::app);
        o << key << " " << best_ty << " " << best_kz << " " << best / 3.0 << "\n";
    }
    return GS_OK;
}

void gs_batch_destroy(gs_batch* h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    drop_graphs(h);
    if (h->pool) (void)hipFree(h->pool);
    if (h->st) (void)hipFree(h->st);
    if (h->tune_st) (void)hipFree(h->tune_st);
    if (h->partial) (void)hipFree(h->partial);
    if (h->insts_dev) (void)hipFree(h->insts_dev);
    if (h->tune_dev) (void)hipFree(h->tune_dev);
    if (h->sched) (void)hipFree(h->sched);
    if (h->host_st) (void)hipHostFree(h->host_st);
    if (h->ev_in) (void)hipEventDestroy(h->ev_in);
    if (h->ev_out) (void)hipEventDestroy(h->ev_out);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

const char* gs_batch_last_error(const gs_batch* h)
{
    return h ? h->err.c_str() : g_batch_create_error.c_str();
}

}  // extern "C"
