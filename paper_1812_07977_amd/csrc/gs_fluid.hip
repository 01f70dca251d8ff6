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
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "gs_fluid.h"
#include "stage.hpp"

namespace gs {

template <typename T, int TX, int TY, int STAGE, bool DEVDT, bool RATE, bool NTH, bool FULL>
__global__ void __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(StageOcc<T, TY>::waves)))
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
    // U(n) of the FP64 second substep: issued before the plane's second
    // barrier in the kernels for ragged tiles, after it in the FULL kernels
    // (each measured faster where it is used: 2% and 1%)
    stage_tile<T, TX, TY, STAGE, RATE, NTH, !FULL, FULL>(Uin, Un, Uout, Cn, D0, g, kt, K, tix, tiy,
                                                         kc, dt, bad, rmax, tid);

    // epilogue: flags and the max signal rate, one atomic per wavefront
    if (__any(bad) && (tid & 63) == 0) atomicOr(&st->flags, 1u);
    if (RATE) {
        for (int off = 32; off > 0; off >>= 1) rmax = __builtin_fmax(rmax, __shfl_xor(rmax, off));
        if ((tid & 63) == 0)
            atomicMax(&st->rate[parity ^ 1], (unsigned long long)__double_as_longlong(rmax));
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

__global__ void set_time_kernel(DevState* st, int parity, double t) { st->t[parity] = t; }

// HBM streaming probe: c = a (one read per write) or c = a + b (two reads
// per write), the read:write mixes of the two substeps, over n doubles as
// 16-byte vectors.  Each thread moves PROBE_UNROLL vectors, 256 apart, all
// loads issued before the first store.  NTS: non-temporal stores.
constexpr int PROBE_THREADS = 256;
constexpr int PROBE_UNROLL = 4;
typedef double probe_d2 __attribute__((ext_vector_type(2)));

template <bool TWO, bool NTS>
__global__ void __launch_bounds__(PROBE_THREADS)
stream_probe_kernel(const probe_d2* __restrict__ a, const probe_d2* __restrict__ b,
                    probe_d2* __restrict__ c, long long n2)
{
    const long long base = (long long)blockIdx.x * PROBE_THREADS * PROBE_UNROLL + threadIdx.x;
    probe_d2 va[PROBE_UNROLL], vb[PROBE_UNROLL];
#pragma unroll
    for (int u = 0; u < PROBE_UNROLL; ++u) {
        const long long i = base + (long long)u * PROBE_THREADS;
        if (i < n2) {
            va[u] = a[i];
            if (TWO) vb[u] = b[i];
        }
    }
#pragma unroll
    for (int u = 0; u < PROBE_UNROLL; ++u) {
        const long long i = base + (long long)u * PROBE_THREADS;
        if (i < n2) {
            probe_d2 r = va[u];
            if (TWO) r = r + vb[u];
            if (NTS) __builtin_nontemporal_store(r, c + i);
            else c[i] = r;
        }
    }
}

// Workspace of the allocation-free advance (gs_fluid_advance_noalloc): the
// first-substep state (and the FP32 form's first increment), the reduction
// partials and the device words of one solve, in one file-scope array that
// every GPU the library runs on holds until the process ends.  Host code
// reaches it only through the address hipGetSymbolAddress returns on each
// device.
constexpr size_t NOALLOC_STATE_BYTES = size_t(96) << 20;
constexpr size_t NOALLOC_PARTIAL_BYTES = size_t(RED_BLOCKS) * 2 * NV * sizeof(double);
constexpr size_t NOALLOC_WORDS_BYTES = (sizeof(DevState) + 255) / 256 * 256;
constexpr size_t NOALLOC_BYTES = NOALLOC_STATE_BYTES + NOALLOC_PARTIAL_BYTES + NOALLOC_WORDS_BYTES;
__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// Copies the device time and the non-physical flag of a solve to caller
// memory (either pointer may be null).
__global__ void report_kernel(const DevState* st, int parity, double* t_out, unsigned int* flags_out)
{
    if (t_out) *t_out = st->t[parity];
    if (flags_out) *flags_out = st->flags;
}

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
    int cus;               // compute units of the device (0: unknown)
    std::string err;
    bool profile;
    bool rate_ready;       // rate[parity] holds the max signal rate of the
                           // state the last step or advance wrote
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
    g.pitch = h->nx;
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
        // FP64: chunks of at most 48 planes, their number rounded up, by at
        // most half again, so that the work items are a whole multiple of
        // the workgroups resident at once (three per CU with 16 x 16 tiles,
        // two with 32 x 8): no partly filled last generation, and shorter
        // chunks keep neighbouring tiles closer in z.  At 512^3: 12 chunks
        // of 43 planes, 0.8% faster steps than 8 of 64 (9 of 57: 0.3%; 16 of
        // 32: 0.3%), results unchanged (a cell's arithmetic does not depend
        // on the chunking)
        if (!f32 && h->cus > 0) {
            const int resident = h->cus * (L.ty == 8 ? 2 : 3);
            const int klim = kz < 48 ? kz : 48;
            int c = (h->nz + klim - 1) / klim;
            const int m = resident / std::gcd(ntile, resident);
            const int cr = (c + m - 1) / m * m;
            if (2 * cr <= 3 * c && (h->nz + cr - 1) / cr >= 8) c = cr;
            kz = (h->nz + c - 1) / c;
        }
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
    // whole tiles: every lane of every tile owns a cell of the mesh, and the
    // FULL kernels apply (bitwise identical; at 512^3 the FP64 step 1.2%
    // faster, the FP32 step 1%)
    const bool full = h->nx % TX == 0 && h->ny % TY == 0;
#define GS_LAUNCH1(S_, D_, R_, N_, W_)                                                            \
    hipLaunchKernelGGL((stage_kernel<T, TX, TY, S_, D_, R_, N_, W_>), grid, block, 0, h->stream,  \
                       Uin, Un, Uout, C, D, L.g, kt, kd, h->st, h->parity, dt_host, t_end,        \
                       dt_log, step)
#define GS_LAUNCH(S_, D_, R_)                                                                     \
    do {                                                                                          \
        if (nth) {                                                                                \
            if (full) GS_LAUNCH1(S_, D_, R_, true, true);                                         \
            else GS_LAUNCH1(S_, D_, R_, true, false);                                             \
        } else {                                                                                  \
            if (full) GS_LAUNCH1(S_, D_, R_, false, true);                                        \
            else GS_LAUNCH1(S_, D_, R_, false, false);                                            \
        }                                                                                         \
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
#undef GS_LAUNCH1
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

// One step of size dt; rate: the second substep also accumulates the max
// signal rate of U(n+1) into the next parity's slot.
template <typename T>
hipError_t step_t(gs_fluid* h, T* u, double dt, bool rate)
{
    StepArrays<T> a = step_arrays(h, u);
    hipError_t e = launch_stage<T>(h, 1, false, false, u, u, a.u1, nullptr, a.d0, dt, 0.0,
                                   nullptr, 0);
    if (e == hipSuccess)
        e = launch_stage<T>(h, 2, false, rate, a.u1, u, u, a.comp, a.d0, dt, 0.0, nullptr, 0);
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

namespace {

// Argument checks shared by gs_fluid_create and gs_fluid_advance_noalloc;
// no HIP call.
int check_problem(int nx, int ny, int nz, double dx, double dy, double dz, double gamma,
                  double cfl, int bc, int dtype)
{
    if (nx < 1 || ny < 1 || nz < 1) return fail(nullptr, GS_ERR_ARG, "mesh sizes must be >= 1");
    // a plane of fewer than 2^29 cells: the FP64 kernels address a field
    // plane through a buffer resource, whose range is at most 2^32 - 1 bytes,
    // so the last cell must end below byte 2^32
    if ((long long)nx * ny >= (1LL << 29) ||
        (long long)nx * ny * nz * NV > (1LL << 40))
        return fail(nullptr, GS_ERR_ARG, "mesh too large (nx*ny below 2^29 cells)");
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
    return GS_OK;
}

// The current device, checked to be a gfx950.
int current_gfx950(int* dev)
{
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, *dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, GS_ERR_HIP,
                    std::string("built for gfx950, device is ") + prop.gcnArchName);
    return GS_OK;
}

// Handle fields of a problem; no allocation, no HIP call.
void init_handle(gs_fluid* h, int nx, int ny, int nz, double dx, double dy, double dz,
                 double gamma, double cfl, int bc, int dtype, int dev, void* stream)
{
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
    h->rate_ready = false;
    // for the default z-chunk length; without it the default ignores the
    // resident workgroup count
    if (hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        h->cus = 0;
        (void)hipGetLastError();
    }
}

// Device address of the allocation-free workspace on each device, looked up
// once per device with that device current.
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[NOALLOC_MAX_DEVICES];

int scratch_address(unsigned char** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(nullptr, GS_ERR_HIP, "device index beyond the allocation-free table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        int r = current_gfx950(&dev);
        if (r != GS_OK) return r;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(nullptr, GS_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch[dev] = (unsigned char*)p;
    }
    *out = g_scratch[dev];
    return GS_OK;
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
    int r0 = check_problem(nx, ny, nz, dx, dy, dz, gamma, cfl, bc, dtype);
    if (r0 != GS_OK) return r0;

    int dev = 0;
    r0 = current_gfx950(&dev);
    if (r0 != GS_OK) return r0;
    hipError_t e;

    gs_fluid* h = new gs_fluid();
    init_handle(h, nx, ny, nz, dx, dy, dz, gamma, cfl, bc, dtype, dev, stream);

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

int gs_fluid_dt_last(gs_fluid* h, double* dt_out)
{
    if (!h) return fail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (!dt_out) return fail(h, GS_ERR_ARG, "dt_out is NULL");
    if (!h->rate_ready)
        return fail(h, GS_ERR_STATE, "the last state written was not written by gs_fluid_advance "
                                     "or gs_fluid_step_dt (or the time was set since)");
    int r = sync_state(h);
    if (r != GS_OK) return r;
    double rate = __builtin_bit_cast(double, h->host_st->rate[h->parity]);
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
    hipError_t e = (h->dtype == GS_F32) ? step_t(h, (float*)U, dt, false)
                                        : step_t(h, (double*)U, dt, false);
    h->parity ^= 1;
    h->rate_ready = false;
    if (e != hipSuccess) return hip_fail(h, e, "stage launch");
    return GS_OK;
}

int gs_fluid_step_dt(gs_fluid* h, void* U, double dt, double* dt_next)
{
    if (!h) return fail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (check_state(h, U) != GS_OK) return GS_ERR_ARG;
    if (!finite_pos(dt)) return fail(h, GS_ERR_ARG, "dt must be finite and > 0");
    if (!dt_next) return fail(h, GS_ERR_ARG, "dt_next is NULL");
    hipError_t e = (h->dtype == GS_F32) ? step_t(h, (float*)U, dt, true)
                                        : step_t(h, (double*)U, dt, true);
    h->parity ^= 1;
    h->rate_ready = (e == hipSuccess);
    if (e != hipSuccess) return hip_fail(h, e, "stage launch");
    return gs_fluid_dt_last(h, dt_next);
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
    h->rate_ready = (e == hipSuccess);
    if (e != hipSuccess) return hip_fail(h, e, "advance launch");
    return GS_OK;
}

int gs_fluid_advance_noalloc(int nx, int ny, int nz, double dx, double dy, double dz,
                             double gamma, double cfl, int bc, int dtype, void* U, int nsteps,
                             double t0, double t_end, double* dt_log, double* t_out,
                             unsigned int* flags_out, void* stream)
{
    g_create_error.clear();
    int r = check_problem(nx, ny, nz, dx, dy, dz, gamma, cfl, bc, dtype);
    if (r != GS_OK) return r;
    const long long ncell = (long long)nx * ny * nz;
    if (state_work_bytes(ncell, dtype) > (long long)NOALLOC_STATE_BYTES)
        return fail(nullptr, GS_ERR_ARG,
                    "mesh too large for the allocation-free entry point (its workspace holds "
                    "96 MiB: 2,516,582 cells)");
    if (!U || !aligned_to(U, elem_size(dtype)))
        return fail(nullptr, GS_ERR_ARG, "U is NULL or not aligned to its element size");
    if (nsteps < 0) return fail(nullptr, GS_ERR_ARG, "nsteps must be >= 0");
    if (!std::isfinite(t0)) return fail(nullptr, GS_ERR_ARG, "t0 must be finite");
    if (!std::isfinite(t_end) || t_end < 0.0)
        return fail(nullptr, GS_ERR_ARG, "t_end must be finite and >= 0");
    if ((dt_log && !aligned8(dt_log)) || (t_out && !aligned8(t_out)) ||
        (flags_out && !aligned_to(flags_out, 4)))
        return fail(nullptr, GS_ERR_ARG, "dt_log, t_out or flags_out misaligned");

    unsigned char* ws = nullptr;
    r = scratch_address(&ws);
    if (r != GS_OK) return r;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");

    // a handle on the stack whose workspace is the device array
    gs_fluid h;
    init_handle(&h, nx, ny, nz, dx, dy, dz, gamma, cfl, bc, dtype, dev, stream);
    h.U1 = ws;
    h.partial = (double*)(ws + NOALLOC_STATE_BYTES);
    h.st = (DevState*)(ws + NOALLOC_STATE_BYTES + NOALLOC_PARTIAL_BYTES);
    hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(1), 0, h.stream, h.st);
    hipLaunchKernelGGL(set_time_kernel, dim3(1), dim3(1), 0, h.stream, h.st, 0, t0);
    e = hipGetLastError();
    if (e == hipSuccess)
        e = (dtype == GS_F32) ? advance_t(&h, (float*)U, nsteps, t_end, dt_log)
                              : advance_t(&h, (double*)U, nsteps, t_end, dt_log);
    if (e == hipSuccess && (t_out || flags_out)) {
        hipLaunchKernelGGL(report_kernel, dim3(1), dim3(1), 0, h.stream, h.st, h.parity, t_out,
                           flags_out);
        e = hipGetLastError();
    }
    return e == hipSuccess ? GS_OK : hip_fail(nullptr, e, "allocation-free advance launch");
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
    h->rate_ready = false;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GS_OK : hip_fail(h, e, "set_time");
}

int gs_fluid_set_stream(gs_fluid* h, void* stream)
{
    if (!h) return fail(nullptr, GS_ERR_ARG, "handle is NULL");
    hipStream_t ns = (hipStream_t)stream;
    if (ns != h->stream) {
        // work queued on the old stream still uses the handle's workspace and
        // device words: the new stream waits for it before any later call
        hipEvent_t ev = nullptr;
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(ev, h->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(ns, ev, 0);
        if (ev) (void)hipEventDestroy(ev);
        if (e != hipSuccess) return hip_fail(h, e, "set_stream ordering");
    }
    h->stream = ns;
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

int gs_fluid_stream_probe(const double* a, const double* b, double* c, long long n, int flags,
                          void* stream)
{
    g_create_error.clear();
    if (!a || !c) return fail(nullptr, GS_ERR_ARG, "a or c is NULL");
    if (!aligned_to(a, 16) || !aligned_to(c, 16) || (b && !aligned_to(b, 16)))
        return fail(nullptr, GS_ERR_ARG, "a, b and c must be 16-byte aligned");
    if (n <= 0 || (n & 1)) return fail(nullptr, GS_ERR_ARG, "n must be even and > 0");
    if (flags & ~1) return fail(nullptr, GS_ERR_ARG, "unknown flags");
    const long long n2 = n / 2;
    const long long per = (long long)PROBE_THREADS * PROBE_UNROLL;
    const long long blocks = (n2 + per - 1) / per;
    if (blocks > 0x7fffffffLL) return fail(nullptr, GS_ERR_ARG, "n too large");
    hipStream_t st = (hipStream_t)stream;
    const probe_d2* A = (const probe_d2*)a;
    const probe_d2* B = (const probe_d2*)b;
    probe_d2* C = (probe_d2*)c;
    const bool nts = flags & 1;
    dim3 grid((unsigned)blocks), block(PROBE_THREADS);
    if (b) {
        if (nts) hipLaunchKernelGGL((stream_probe_kernel<true, true>), grid, block, 0, st, A, B, C, n2);
        else hipLaunchKernelGGL((stream_probe_kernel<true, false>), grid, block, 0, st, A, B, C, n2);
    } else {
        if (nts) hipLaunchKernelGGL((stream_probe_kernel<false, true>), grid, block, 0, st, A, B, C, n2);
        else hipLaunchKernelGGL((stream_probe_kernel<false, false>), grid, block, 0, st, A, B, C, n2);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GS_OK : hip_fail(nullptr, e, "stream probe launch");
}

const char* gs_fluid_last_error(const gs_fluid* h)
{
    return h ? h->err.c_str() : g_create_error.c_str();
}

}  // extern "C"
