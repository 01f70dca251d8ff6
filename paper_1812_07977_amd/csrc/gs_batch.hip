// gs_batch.hip -- the batched form of libgs_fluid.so (include/gs_batch.h):
// many independent problems of different mesh sizes, each with its own CFL
// time step, advanced by one persistent launch per substep over the work
// items of all of them.  Each item runs the same per-tile substep body
// (stage.hpp) as the single-problem stage kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "gs_batch.h"
#include "gs_fluid.h"
#include "stage.hpp"

namespace gs {

// ---------------------------------------------------------------------------
// Batched form: many independent problems in one launch per substep
// ---------------------------------------------------------------------------

// One problem of a batch as the batched kernels see it.
struct BatchInst {
    Geom g;              // mesh and tiling (band unused)
    Phys kd;             // FP64 constants, with this problem's cell widths
    PhysT<float> kf;     // the same rounded to FP32
    void* U;             // the state the steps advance: the batch's row-padded
                         // working copy, or the caller's state where rows are
                         // not padded (FP32 form: head, then compensation)
    void* U1;            // workspace: U(1) (FP32 form: then dU(U(n))), padded
    void* Uc;            // the caller's state, rows of nx cells
    DevState* st;        // this problem's device words
    int item0;           // first work item (tile, z-chunk) of this problem
    int items;
};

__device__ __forceinline__ const Phys& batch_phys(const BatchInst& I, const Phys*) { return I.kd; }
__device__ __forceinline__ const PhysT<float>& batch_phys(const BatchInst& I, const PhysT<float>*)
{
    return I.kf;
}

// A device address held in the table, as a pointer to global memory: loads
// and stores through it are then global, not flat, instructions (a flat
// access also counts against the LDS wait counter, so every LDS wait of the
// substep body would wait for the plane loads in flight as well).
template <typename P>
__device__ __forceinline__ P* global_ptr(const void* p)
{
    typedef __attribute__((address_space(1))) P* GP;
    return (P*)(GP)(uintptr_t)p;
}

// Waves per SIMD of the batched kernels: three (at most 168 VGPRs), except
// FP64 32 x 8 tiles, whose LDS (57 KiB per workgroup) admits two workgroups
// per CU.  Under the compiler's default scheduler the FP64 16 x 16 body
// fits the three-wave budget without spills (under the iterative ILP
// scheduler the item loop took about 210 VGPRs).
template <typename T, int TY>
struct BatchOcc {
    static constexpr int waves = (sizeof(T) == 8 && TY == 8) ? 2 : 3;
};

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
__global__ void __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(BatchOcc<T, TY>::waves)))
batch_stage_kernel(const BatchInst* __restrict__ insts, int count, int total, int parity,
                   double t_end, unsigned int* __restrict__ sched)
{
    __shared__ int s_item, s_tried;  // next item; shares found empty so far
    const int tid = threadIdx.x;
    const int xcd = blockIdx.x & 7;
    if (tid == 0) s_tried = 0;
    for (;;) {
        if (tid == 0) {
            int next = -1, tried = s_tried;
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
            s_tried = tried;
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
        DevState* st = global_ptr<DevState>(I.st);
        const Phys& K = I.kd;
        const PhysT<T>& kt = batch_phys(I, (const PhysT<T>*)nullptr);

        const double rate = __longlong_as_double((long long)st->rate[parity]);
        const double t_now = st->t[parity];
        double dt = K.cfl / rate;
        if (t_end > 0.0) {
            if (!(t_now < t_end)) dt = 0.0;
            else if (t_now + dt > t_end) dt = t_end - t_now;
        }
        {
            // dt is the same in every lane; held in scalar registers it
            // leaves the vector registers to the body (two fewer)
            const unsigned long long b = (unsigned long long)__double_as_longlong(dt);
            const unsigned int lo32 = __builtin_amdgcn_readfirstlane((unsigned int)b);
            const unsigned int hi32 = __builtin_amdgcn_readfirstlane((unsigned int)(b >> 32));
            dt = __longlong_as_double((long long)(((unsigned long long)hi32 << 32) | lo32));
        }
        if (STAGE == 1 && local == 0 && tid == 0) {
            st->t[parity ^ 1] = t_now + dt;
            st->rate[parity ^ 1] = 0ull;
        }
        T* U = global_ptr<T>(I.U);
        T* U1 = global_ptr<T>(I.U1);
        T* C = (sizeof(T) == 4) ? U + NV * g.field : nullptr;
        T* D0 = (sizeof(T) == 4) ? U1 + NV * g.field : nullptr;
        bool bad = false;
        double rmax = 0.0;
        // the thread index, opaque to the compiler on every item, so that the
        // per-thread offsets the body derives from it are computed per item
        // instead of being hoisted out of the item loop and held in registers
        // across it
        int ltid = tid;
        asm volatile("" : "+v"(ltid));
        // FP64: the streams touched once carry the non-temporal hint (2%
        // faster over the 64-problem batch); FP32: no hint (with it the
        // FP32 batch ran 35% slower)
        constexpr bool NTH = sizeof(T) == 8;
        if (STAGE == 1)
            stage_tile<T, TX, TY, 1, false, NTH>(U, U, U1, nullptr, D0, g, kt, K, tix, tiy, kc, dt,
                                                 bad, rmax, ltid);
        else
            stage_tile<T, TX, TY, 2, RATE, NTH, false>(U1, U, U, C, D0, g, kt, K, tix, tiy, kc, dt, bad,
                                                       rmax, ltid);
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

// Copies every problem's state between the caller's layout (rows of nx
// cells) and the batch's padded one (rows of g.pitch cells, each row
// starting on a 128-byte line): IN copies caller -> padded, else padded ->
// caller.  arrays = fields of a state (5; the FP32 form's pair 10).
// Workgroup (p, s) takes planes s, s + gridDim.y, ... of problem p (a plane
// is one field at one z), one wave per row; the padding cells are never
// read by the stage kernels.
template <typename T, bool IN>
__global__ void __launch_bounds__(256)
copy_rows_kernel(const BatchInst* __restrict__ insts, int arrays)
{
    const BatchInst& I = insts[blockIdx.x];
    if (I.U == I.Uc) return;  // steps run on the caller's state itself
    const int nx = I.g.nx, ny = I.g.ny, nz = I.g.nz;
    T* pad = global_ptr<T>(I.U);
    T* den = global_ptr<T>(I.Uc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int pl = blockIdx.y; pl < arrays * nz; pl += gridDim.y) {
        const int a = pl / nz, k = pl - a * nz;
        T* d = den + ((long long)a * nz + k) * ny * nx;
        T* q = pad + (long long)a * I.g.field + (long long)k * I.g.plane;
        for (int j = wave; j < ny; j += 4) {
            for (int i = lane; i < nx; i += 64) {
                if (IN) q[(long long)j * I.g.pitch + i] = d[(long long)j * nx + i];
                else d[(long long)j * nx + i] = q[(long long)j * I.g.pitch + i];
            }
        }
    }
}

}  // namespace gs

// ===========================================================================
// Host side
// ===========================================================================

using namespace gs;

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
    void* pool;                 // workspaces and padded states of all problems
    std::vector<size_t> pool_off;   // workspace U(1) of problem i
    std::vector<void*> padded;      // working copy of problem i's state with
                                    // padded rows (null: rows not padded)
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
// Row pitch of the batch's arrays.  FP64: rows padded to whole 128-byte
// lines (16 doubles), so that every 16-wide tile row is one line (the
// 64-problem batch measured 3% faster, copies included); FP32: the caller's
// rows as they are (padding its pairs measured 6% slower).
int batch_pitch(const gs_batch* h, int nx)
{
    if (h->dtype == GS_F32) return nx;
    const int per_line = 128 / (int)h->esize;
    return (nx + per_line - 1) / per_line * per_line;
}

// Elements of one padded array of problem i.
long long padded_field(const gs_batch* h, int i)
{
    return (long long)batch_pitch(h, h->dims[i][0]) * h->dims[i][1] * h->dims[i][2];
}

// Fields in a state (the FP32 form's pair: head and compensation) and in a
// workspace (FP32: U(1) and the first increment).
int state_arrays(const gs_batch* h) { return h->dtype == GS_F32 ? 2 * NV : NV; }

std::vector<BatchInst> batch_table(const gs_batch* h, const std::vector<void*>& states,
                                   const std::vector<void*>& padded, DevState* st, int* total)
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
        g.pitch = batch_pitch(h, nx);
        g.plane = g.pitch * ny;
        g.field = (long long)g.pitch * ny * nz;
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
        I.U = padded[i] ? padded[i] : states[i];
        I.U1 = (char*)h->pool + h->pool_off[i];
        I.Uc = states[i];
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

// caller states <-> padded copies of every problem of `table`
hipError_t batch_copy(gs_batch* h, const BatchInst* table, bool in)
{
    const dim3 grid(h->count, 64), block(256);
    const int arrays = state_arrays(h);
    if (h->dtype == GS_F32) {
        if (in) hipLaunchKernelGGL((copy_rows_kernel<float, true>), grid, block, 0, h->stream, table, arrays);
        else hipLaunchKernelGGL((copy_rows_kernel<float, false>), grid, block, 0, h->stream, table, arrays);
    } else {
        if (in) hipLaunchKernelGGL((copy_rows_kernel<double, true>), grid, block, 0, h->stream, table, arrays);
        else hipLaunchKernelGGL((copy_rows_kernel<double, false>), grid, block, 0, h->stream, table, arrays);
    }
    return hipGetLastError();
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
    std::vector<BatchInst> t = batch_table(h, h->states, h->padded, h->st, &total);
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
        // a plane of fewer than 2^29 cells, rows padded to 16 included: the
        // FP64 kernels address a field plane through a buffer resource, whose
        // range is at most 2^32 - 1 bytes
        if ((long long)(nx + 15) * ny >= (1LL << 29))
            return bfail(nullptr, GS_ERR_ARG, "mesh too large ((nx+15)*ny below 2^29 cells)");
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
    std::vector<size_t> pad_off(count);
    for (int i = 0; i < count; ++i) {
        h->dims[i] = {dims[3 * i], dims[3 * i + 1], dims[3 * i + 2]};
        // workspace and, where the rows are padded, a working copy of the
        // state: state_arrays arrays each
        const size_t bytes = (size_t)state_arrays(h) * padded_field(h, i) * h->esize;
        h->pool_off.push_back(off);
        off += (bytes + 255) / 256 * 256;
        pad_off[i] = off;
        if (batch_pitch(h, dims[3 * i]) != dims[3 * i]) off += (bytes + 255) / 256 * 256;
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
    for (int i = 0; i < count; ++i)
        h->padded.push_back(batch_pitch(h, h->dims[i][0]) != h->dims[i][0] ? (char*)h->pool + pad_off[i]
                                                                          : nullptr);
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
    if (e == hipSuccess) e = batch_copy(h, h->insts_dev, true);
    if (e == hipSuccess && use_graph && (!h->graphs_valid || h->graph_t_end != t_end))
        e = capture_graphs(h, t_end);
    for (int s = 0; s < nsteps && e == hipSuccess; ++s) {
        if (use_graph)
            e = hipGraphLaunch(h->exec[h->parity], h->stream);
        else
            e = batch_step(h, h->insts_dev, h->total_items, h->parity, t_end);
        h->parity ^= 1;
    }
    if (e == hipSuccess) e = batch_copy(h, h->insts_dev, false);
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
    // padded scratch copies of the states, filled below through the table
    for (int i = 0; i < h->count; ++i) {
        const size_t bytes = (size_t)state_arrays(h) * padded_field(h, i) * h->esize;
        if ((e = hipMalloc(&scratch[i], bytes)) != hipSuccess) {
            free_scratch();
            return bhip(h, e, "autotune scratch");
        }
    }
    bool filled = false;
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
            std::vector<BatchInst> t = batch_table(h, h->states, scratch, h->tune_st, &total);
            e = hipMemcpy(h->tune_dev, t.data(), sizeof(BatchInst) * h->count, hipMemcpyHostToDevice);
            if (e != hipSuccess) break;
            if (!filled) {
                e = batch_copy(h, h->tune_dev, true);
                if (e != hipSuccess) break;
                filled = true;
            }
            h->total_items = total;
            batch_grids(h);
            int par = 0;
            // time steps of the caller's states (unchanged by the tuning)
            e = batch_rates(h, h->states, h->tune_st, par);
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
