// gs_cnn.hip -- gfx950 kernels and C ABI of the learned-correction form: a
// 5 -> 32 -> 32 -> 5 network of 3x3x3 convolutions on BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation), its training, and the
// correction of an FP32 coarse state with a device-side fallback.
//
// Layouts.
//   * CL (channels-last) BF16 activations: act[v * C + c], v = (z ny + y) nx
//     + x, C = 8 (the 5 input fields padded with zeros) or 32.  One MFMA
//     operand fragment of 8 channels of one cell is one 16-byte load.
//   * RV (row-blocked, channel-major within a row) BF16 copies for the
//     weight gradient: element (c, v) of a C-channel array, v = row nx + x
//     with row = z ny + y, at (row C + c) nx + x; for a layer input three
//     copies shifted by dx = -1, 0, +1 along x (the boundary map applied
//     while copying), so that every operand fragment of 8 consecutive cells
//     along x is one aligned 16-byte load, and the channels a wave reads
//     together lie within a few kilobytes (a mesh-wide channel-major layout
//     put them megabytes apart, one page each).
//   * Weights in fragment order: for K-block kb and N-block nb, lane l holds
//     the 8 values of the 16x16x32 B operand it feeds: 64 lanes x 16 bytes.
//
// Matrix-core lane layout of v_mfma_f32_16x16x32_bf16 (checked on the
// device): lane l holds A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j]
// [l % 16], j = 0..7, and receives D[4 (l / 16) + i][l % 16], i = 0..3.
//
// Forward convolution as an implicit GEMM: M = cells (16 consecutive x of a
// row per M-block), N = output channels, K = 27 taps x input channels (one
// tap of 32 channels, or four taps of 8, per 32-wide K-block).  The input
// gradient of a convolution on a periodic mesh is the convolution of the
// output gradient with mirrored taps and transposed channels, so the same
// kernel runs the backward pass, with the ReLU mask fused into its epilogue.
// Its input tile and halo are staged in LDS once per plane.  The weight
// gradient is a GEMM over cells (K = cells): M = input channels, N = output
// channels, for all 27 taps per workgroup over its share of the mesh rows;
// one partial sum per workgroup and tap, reduced in a fixed order by a
// second kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "euler_math.hpp"
#include "gs_cnn.h"
#include "gs_fluid.h"

namespace gsc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int NF = 5;       // conserved fields
constexpr int HID = 32;     // hidden channels
constexpr int TAPS = 27;
constexpr int THREADS = 256;

// parameter layout (floats)
constexpr int W1_N = HID * NF * TAPS, B1_N = HID;
constexpr int W2_N = HID * HID * TAPS, B2_N = HID;
constexpr int W3_N = NF * HID * TAPS, B3_N = NF;
constexpr int W1_OFF = 0, B1_OFF = W1_OFF + W1_N;
constexpr int W2_OFF = B1_OFF + B1_N, B2_OFF = W2_OFF + W2_N;
constexpr int W3_OFF = B2_OFF + B2_N, B3_OFF = W3_OFF + W3_N;
constexpr int P_N = B3_OFF + B3_N;

// BF16 <-> FP32, round to nearest even (inputs are finite)
__device__ __forceinline__ u16 f2bf(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}
__device__ __forceinline__ float bf2f(u16 b) { return __uint_as_float((unsigned)b << 16); }

// compensated accumulation (Knuth's TwoSum): s + c tracks the exact sum
// of the added values to about one FP64 rounding of the total
__device__ __forceinline__ void two_sum_add(double& s, double& c, double x)
{
    double t = s + x, bp = t - s;
    c += (s - (t - bp)) + (x - bp);
    s = t;
}

__device__ __forceinline__ int wrap_or_clamp(int i, int n, int periodic)
{
    if (periodic) {
        int r = i % n;
        return r < 0 ? r + n : r;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

__device__ __forceinline__ f32x4 mfma(u32x4 a, u32x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// two FP32 values -> packed BF16 pair (low = a), round to nearest even
// (v_cvt_pk_bf16_f32; the same result as f2bf for finite values)
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned pack_bf16(float a, float b)
{
    return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2{a, b}), bf16x2));
}

// value of lane (l ^ 1) / (l ^ 2) of the same quad (DPP quad permutations)
__device__ __forceinline__ float quad_xor1(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ float quad_xor2(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
}

// 4 x 4 transpose within each quad of lanes: lane q of the quad holds
// v[i] = M[i][q] on entry and v[j] = M[q][j] on return.  Two exchange
// stages, with lane q ^ 1 (entries whose index differs from q in bit 0),
// then with lane q ^ 2 (bit 1).
__device__ __forceinline__ void quad_transpose(float (&v)[4], int q)
{
    const bool b0 = (q & 1) != 0, b1 = (q & 2) != 0;
    float r0 = quad_xor1(b0 ? v[0] : v[1]), r1 = quad_xor1(b0 ? v[2] : v[3]);
    const float u0 = b0 ? r0 : v[0], u1 = b0 ? v[1] : r0;
    const float u2 = b0 ? r1 : v[2], u3 = b0 ? v[3] : r1;
    r0 = quad_xor2(b1 ? u0 : u2);
    r1 = quad_xor2(b1 ? u1 : u3);
    v[0] = b1 ? r0 : u0;
    v[1] = b1 ? r1 : u1;
    v[2] = b1 ? u2 : r0;
    v[3] = b1 ? u3 : r1;
}

// ---------------------------------------------------------------------------
// weight packing
// ---------------------------------------------------------------------------

// Fragment-ordered BF16 weights of one convolution from the FP32 master
// array W[cout][cin][27].  CINP = 32: K-block kb = tap kb, k = input
// channel; CINP = 8: K-block kb = taps 4kb .. 4kb+3 (lane group), k = input
// channel (< 8).  MIRROR: the backward (input-gradient) convolution, whose
// input channels are the forward's outputs, output channels the forward's
// inputs, and tap t the forward's tap 26 - t.  Entries outside the logical
// sizes are zero.
__global__ void pack_weights_kernel(const float* __restrict__ W, int cin, int cout, int cinp,
                                    int nb_count, int kb_count, int mirror, u16* __restrict__ out)
{
    const int total = kb_count * nb_count * 64 * 8;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int j = e & 7, l = (e >> 3) & 63, frag = e >> 9;
        const int nb = frag % nb_count, kb = frag / nb_count;
        int tap, ci;
        if (cinp == 32) {
            tap = kb;
            ci = 8 * (l >> 4) + j;
        } else {
            tap = 4 * kb + (l >> 4);
            ci = j;
        }
        const int co = 16 * nb + (l & 15);
        float w = 0.0f;
        if (tap < TAPS) {
            // forward view: out channel co, in channel ci, tap
            // mirror view: out channel co = forward input, in channel ci =
            // forward output, tap mirrored
            const int fo = mirror ? ci : co, fi = mirror ? co : ci;
            const int ft = mirror ? TAPS - 1 - tap : tap;
            if (fo < cout && fi < cin) w = W[(fo * cin + fi) * TAPS + ft];
        }
        out[e] = f2bf(w);
    }
}

// ---------------------------------------------------------------------------
// convolution (forward, and input gradient with mirrored weights)
// ---------------------------------------------------------------------------

enum { EPI_RELU_BF16 = 0, EPI_F32_SOA = 1, EPI_MASK_BF16 = 2 };

struct ConvGeom {
    int nx, ny, nz;
    int periodic;
    int ntx, nty;   // 16 x 16 tiles
    int kz;         // planes per work item
    int items;      // work items: tiles x z-chunks
};

// LDS staging of the convolution input: the 16 x 16 output tile plus a
// one-cell halo (18 x 18 cells) per plane, in a ring of four plane slots:
// planes z-1, z, z+1 are read while plane z+2 is written into the fourth,
// so one barrier per plane suffices.  Within a plane, 16-byte chunk c
// (channels 8c .. 8c+7) of halo cell k sits at slot c CP + k: the 16 lanes
// of a quarter-wave read 16 consecutive cells of one chunk, 256 contiguous
// bytes, which the gfx950 LDS serves without bank conflicts (a cell-major
// layout with an 80-byte cell stride measured two cycles per read instead of
// one).  CP = 336 (a multiple of 16 slots) for four chunks.  The boundary
// map is applied once, while staging.
constexpr int HT = 18;
constexpr int RING = 4;
constexpr int CONV_ROWS = 2;                       // tile rows per wave
constexpr int CONV_THREADS = 64 * 16 / CONV_ROWS;  // 8 waves: two per SIMD

template <int CINP>
struct Stage {
    static constexpr int CH = CINP / 8;                  // 16-byte chunks per cell
    static constexpr int CP = (CINP == 32) ? 336 : HT * HT;  // slots per chunk plane
    static constexpr int PLANE = CH * CP;                // slots per plane
    static constexpr int CHUNKS = HT * HT * CH;
    static constexpr int LOADS = (CHUNKS + CONV_THREADS - 1) / CONV_THREADS;
};

// halo index i in [-1, n + 15] -> mesh index.  Positions past n feed only
// outputs outside the mesh (ragged tiles), so any valid index serves.
__device__ __forceinline__ int halo_map(int i, int n, int periodic)
{
    if (i > n) i = n;
    if (periodic) return i < 0 ? i + n : (i >= n ? i - n : i);
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

template <int CINP>
__device__ __forceinline__ void stage_fetch(const u16* __restrict__ X, const ConvGeom& g, int x0,
                                            int y0, int p, u32x4 (&r)[Stage<CINP>::LOADS])
{
    using S = Stage<CINP>;
    const int zs = halo_map(p, g.nz, g.periodic);
#pragma unroll
    for (int k = 0; k < S::LOADS; ++k) {
        const int e = threadIdx.x + k * CONV_THREADS;
        if (e < S::CHUNKS) {
            const int cell = e / S::CH, c = e % S::CH;
            const int hy = cell / HT, hx = cell - hy * HT;
            const int ys = halo_map(y0 - 1 + hy, g.ny, g.periodic);
            const int xs = halo_map(x0 - 1 + hx, g.nx, g.periodic);
            const long long v = ((long long)zs * g.ny + ys) * g.nx + xs;
            r[k] = *(const u32x4*)(X + v * CINP + 8 * c);
        }
    }
}

template <int CINP>
__device__ __forceinline__ void stage_store(u32x4* __restrict__ plane,
                                            const u32x4 (&r)[Stage<CINP>::LOADS])
{
    using S = Stage<CINP>;
#pragma unroll
    for (int k = 0; k < S::LOADS; ++k) {
        const int e = threadIdx.x + k * CONV_THREADS;
        if (e < S::CHUNKS) {
            const int cell = e / S::CH, c = e % S::CH;
            plane[c * S::CP + cell] = r[k];
        }
    }
}

// ---------------------------------------------------------------------------
// state of the correction, and its reductions
// ---------------------------------------------------------------------------

struct CorrState {
    double mean[NF];      // channel means of y
    double moved[NF];     // total represented change per field
    double mag[NF];       // sum of |change| per field
    unsigned int bad;     // a corrected cell is non-physical
    int applied, fallbacks;
    int ok;               // decision of the last correction
};

// The mean of each field from n per-block partials partial[b * NF + f]: one
// wave per field (wave w of the calling workgroup takes fields w, w + waves,
// ...), TwoSum over the partials lane-strided, then a fixed shuffle tree.
// Also clears the check's accumulators.
__device__ __forceinline__ void mean_body(const double* __restrict__ partial, int n, long long ncell,
                                          CorrState* __restrict__ cs)
{
    const int lane = threadIdx.x & 63;
    for (int f = threadIdx.x >> 6; f < NF; f += blockDim.x >> 6) {
        double S = 0.0, C = 0.0;
        for (int b = lane; b < n; b += 64) two_sum_add(S, C, partial[b * NF + f]);
        for (int off = 32; off > 0; off >>= 1) {
            double s2 = __shfl_xor(S, off), c2 = __shfl_xor(C, off);
            two_sum_add(S, C, s2);
            C += c2;
        }
        if (lane == 0) {
            cs->mean[f] = (S + C) / (double)ncell;
            cs->moved[f] = 0.0;
            cs->mag[f] = 0.0;
        }
    }
    if (threadIdx.x == 0) cs->bad = 0u;
}

// Decision from n per-block partials of the check (moved, magnitude per
// field): accept unless a candidate cell is non-physical or some |total
// change| exceeds 1e-5 of the change's magnitude plus 1e-30 (also false for
// NaN).  Wave w of the calling workgroup takes fields w, w + waves, ...,
// and sums their partials in a fixed order; every thread of the workgroup
// must call it.
__device__ __forceinline__ void decide_body(const double* __restrict__ partial, int n,
                                            CorrState* __restrict__ cs)
{
    __shared__ int okf[NF];
    const int lane = threadIdx.x & 63;
    for (int f = threadIdx.x >> 6; f < NF; f += blockDim.x >> 6) {
        double moved = 0.0, mag = 0.0;
        for (int b = lane; b < n; b += 64) {
            moved += partial[b * 2 * NF + 2 * f];
            mag += partial[b * 2 * NF + 2 * f + 1];
        }
        for (int off = 32; off > 0; off >>= 1) {
            moved += __shfl_xor(moved, off);
            mag += __shfl_xor(mag, off);
        }
        if (lane == 0) {
            cs->moved[f] = moved;
            cs->mag[f] = mag;
            okf[f] = (fabs(moved) <= 1e-5 * mag + 1e-30) ? 1 : 0;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        bool ok = cs->bad == 0u;
        for (int g = 0; g < NF; ++g) ok = ok && okf[g];
        cs->ok = ok ? 1 : 0;
        if (ok)
            cs->applied += 1;
        else
            cs->fallbacks += 1;
    }
}

// Where the last convolution of a correction sums its outputs for the mean
// removal (mode 0); part == nullptr in every other launch.
struct MeanSums {
    double* part;     // [workgroup][NF] sums of the stored outputs
    double clip;      // > 0: values are clamped to [-clip, clip] before summing
};

// X: CL input with CINP channels.  Wp: fragment-packed weights.  Output per
// EPI: RELU_BF16 -> CL BF16 [v][16 NB] of max(acc + bias, 0); F32_SOA ->
// FP32 [co][v] for co < cout_valid, acc + bias; MASK_BF16 -> CL BF16 of acc
// where mask (CL BF16, same shape) is positive, else 0.
//
// Persistent: workgroup b takes work items b, b + grid, ...; an item is one
// 16 x 16 tile over kz consecutive planes.  Eight waves (two per SIMD, so
// one's products overlap the other's stores and waits) share the ring; in
// general wave w computes rows 2w, 2w+1 of the tile (two M-blocks of 16
// cells) for all NB N-blocks, reading its operand fragments from LDS one
// group ahead of the products that use them: for 32 input channels a group
// is the three taps (dz, 0..2, dx), whose A fragments are four rows (the
// same rows shifted by dy); for 8 input channels a group is one K-block of
// four taps.  The forward hidden layer (32 -> 32) instead gives wave w rows
// 4 (w % 4) .. 4 (w % 4) + 3 and N-block w / 4, with that block's weights
// in registers (six A fragments per group, no B reads); the last layer
// (one N-block) keeps its weights in registers too.  The next plane of the ring
// is fetched into registers before the products of the current plane and
// written to LDS after them.
template <int CINP, int NB, int EPI>
__global__ void __launch_bounds__(CONV_THREADS)
conv_kernel(const u16* __restrict__ X, const u16* __restrict__ Wp, const float* __restrict__ bias,
            void* __restrict__ out, const u16* __restrict__ mask, ConvGeom g, int cout_valid,
            MeanSums ms_out)
{
    using S = Stage<CINP>;
    constexpr int KB = (CINP == 32) ? TAPS : 7;
    constexpr int COUT = 16 * NB;
    // one N-block of 32-channel inputs (the last layer): each lane keeps its
    // 27 weight fragments in registers, so the products read only their A
    // fragments from LDS; otherwise the fragments are staged in LDS
    // Two N-blocks of 32-channel inputs (the hidden layer): the eight waves
    // split the tile as four groups of four rows times the two N-blocks, and
    // each lane keeps the 27 weight fragments of its N-block in registers,
    // so each product group reads six A fragments and no B fragment from LDS
    // (against ten reads per twelve products with two rows and both N-blocks
    // per wave).
    constexpr bool SPLIT = CINP == 32 && NB == 2 && EPI == EPI_RELU_BF16;
    constexpr bool WREG = CINP == 32 && (NB == 1 || SPLIT);
    constexpr int NBW = SPLIT ? 1 : NB;  // N-blocks per wave
    const int nb0 = SPLIT ? (int)(threadIdx.x >> 8) : 0;  // the wave's first N-block
    __shared__ u32x4 Wl[WREG ? 1 : KB * NB * 64];
    __shared__ u32x4 In[RING * S::PLANE];
    u32x4 wr[WREG ? TAPS : 1];
    if constexpr (WREG) {
#pragma unroll
        for (int t = 0; t < TAPS; ++t) wr[t] = ((const u32x4*)Wp)[(t * NB + nb0) * 64 + (threadIdx.x & 63)];
    } else {
        for (int i = threadIdx.x; i < KB * NB * 64; i += CONV_THREADS) Wl[i] = ((const u32x4*)Wp)[i];
    }

    constexpr int RW = SPLIT ? 4 : CONV_ROWS;  // tile rows per wave
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int rowg = SPLIT ? (wave & 3) : wave;  // the wave's rows: RW rowg ..
    static_assert((SPLIT ? 4 : CONV_THREADS / 64) * RW == 16, "the waves cover the 16 tile rows");
    const int xl = l & 15, grp = l >> 4;
    const int ntile = g.ntx * g.nty;
    const long long ncell = (long long)g.nx * g.ny * g.nz;
    // per-lane LDS slot of its A fragment for halo offset (0, 0): row RW wave
    // (+ r + dy), column xl (+ dx), chunk grp
    const int lane_off = (RW * rowg) * HT + xl + ((CINP == 32) ? grp * S::CP : 0);
    // CINP = 8: K-block kb covers taps 4 kb .. 4 kb + 3, one per lane group
    int kb_plane[KB], kb_off[KB];
    if (CINP != 32) {
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            int tap = 4 * kb + grp;
            if (tap >= TAPS) tap = 13;  // padding taps carry zero weights
            kb_plane[kb] = tap / 9;
            kb_off[kb] = ((tap / 3) % 3) * HT + tap % 3;
        }
    }
    float bv[NBW];
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) bv[nb] = (EPI == EPI_MASK_BF16) ? 0.0f : bias[16 * (nb0 + nb) + xl];
    double msum = 0.0, mcomp = 0.0;  // F32_SOA with ms_out: this lane's sum of channel xl

    for (int item = blockIdx.x; item < g.items; item += gridDim.x) {
        const int tile = item % ntile, chunk = item / ntile;
        const int x0 = (tile % g.ntx) * 16, y0 = (tile / g.ntx) * 16;
        const int z0 = chunk * g.kz, z1 = min(z0 + g.kz, g.nz);
        // planes z0-1 .. z0+1 in one round trip; plane z0+2 stays in flight
        u32x4 pa[S::LOADS], pb[S::LOADS], pc[S::LOADS];
        stage_fetch<CINP>(X, g, x0, y0, z0 - 1, pa);
        stage_fetch<CINP>(X, g, x0, y0, z0, pb);
        stage_fetch<CINP>(X, g, x0, y0, z0 + 1, pc);
        stage_store<CINP>(In, pa);
        stage_store<CINP>(In + S::PLANE, pb);
        stage_store<CINP>(In + 2 * S::PLANE, pc);
        if (z0 + 1 < z1) stage_fetch<CINP>(X, g, x0, y0, z0 + 2, pa);
        __syncthreads();
        int sb = 0;  // ring slot of plane z-1; z, z+1 follow, the fourth is free
        // one output plane; cur holds plane z+2 (fetched one plane earlier),
        // nxt receives plane z+3, so each fetch has two planes of products
        // to arrive
        auto plane = [&](const int z, u32x4(&cur)[S::LOADS], u32x4(&nxt)[S::LOADS]) {
            if (z + 2 < z1) stage_fetch<CINP>(X, g, x0, y0, z + 3, nxt);
            // after the quad transpose of the epilogue, lane (grp, xl) holds
            // channels 16 nb + cq .. + 3 of cell x0 + 4 grp + q of each row
            const int q = xl & 3, cq = xl & ~3;
            uint2 mk[RW][NBW];
            if (EPI == EPI_MASK_BF16) {
                const int x = min(x0 + 4 * grp + q, g.nx - 1);
#pragma unroll
                for (int r = 0; r < RW; ++r) {
                    const int y = min(y0 + RW * rowg + r, g.ny - 1);
                    const long long v = ((long long)z * g.ny + y) * g.nx + x;
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        mk[r][nb] = *(const uint2*)(mask + v * COUT + 16 * nb + cq);
                }
            }
            const u32x4* pl[3] = {In + sb * S::PLANE, In + ((sb + 1) & 3) * S::PLANE,
                                  In + ((sb + 2) & 3) * S::PLANE};

            f32x4 acc[RW][NBW];
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int nb = 0; nb < NBW; ++nb) acc[r][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
            if constexpr (SPLIT) {
                // group q = (dz, dx): rows 0 .. RW+1 of A; the B fragments of
                // taps (dz, 0..2, dx) are in registers.  One buffer of A
                // fragments, its reads scheduled by the compiler (the other
                // wave of the SIMD covers their latency)
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    const int dz = q / 3, dx = q % 3;
                    const u32x4* src = pl[dz] + lane_off + dx;
                    u32x4 fa[RW + 2];
#pragma unroll
                    for (int j = 0; j < RW + 2; ++j) fa[j] = src[j * HT];
#pragma unroll
                    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                        for (int r = 0; r < RW; ++r)
                            acc[r][0] = mfma(fa[r + dy], wr[(dz * 9 + dy * 3 + dx) % (WREG ? TAPS : 1)], acc[r][0]);
                }
            } else if (CINP == 32) {
                // group q = (dz, dx): rows 0 .. RW+1 of A, B of taps (dz, 0..2, dx)
                u32x4 fa[2][RW + 2], fb[2][3][NB];
#pragma unroll
                for (int q = 0; q <= 9; ++q) {
                    if (q < 9) {
                        const int dz = q / 3, dx = q % 3, cur = q & 1;
                        const u32x4* src = pl[dz] + lane_off + dx;
#pragma unroll
                        for (int j = 0; j < RW + 2; ++j) fa[cur][j] = src[j * HT];
                        if constexpr (!WREG) {
#pragma unroll
                            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                                for (int nb = 0; nb < NB; ++nb)
                                    fb[cur][dy][nb] = Wl[((dz * 9 + dy * 3 + dx) * NB + nb) * 64 + l];
                        }
                    }
                    if (q > 0) {
                        const int prv = (q - 1) & 1;
                        const int pz = (q - 1) / 3, px = (q - 1) % 3;
#pragma unroll
                        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                            for (int nb = 0; nb < NBW; ++nb) {
                                const u32x4 b = WREG ? wr[(pz * 9 + dy * 3 + px) % (WREG ? TAPS : 1)]
                                                     : fb[prv][dy][nb];
#pragma unroll
                                for (int r = 0; r < RW; ++r) acc[r][nb] = mfma(fa[prv][r + dy], b, acc[r][nb]);
                            }
                    }
                    if (q > 0 && q < 9) {
                        // issue the next group's reads first, then this group's products
                        __builtin_amdgcn_sched_group_barrier(0x100, RW + 2 + (WREG ? 0 : 3 * NB), 0);
                        __builtin_amdgcn_sched_group_barrier(0x008, 3 * RW * NBW, 0);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            } else {
                u32x4 fa[2][RW], fb[2][NB];
#pragma unroll
                for (int kb = 0; kb <= KB; ++kb) {
                    if (kb < KB) {
                        const int cur = kb & 1, dzi = kb_plane[kb];
                        const u32x4* src =
                            (dzi == 0 ? pl[0] : (dzi == 1 ? pl[1] : pl[2])) + lane_off + kb_off[kb];
#pragma unroll
                        for (int r = 0; r < RW; ++r) fa[cur][r] = src[r * HT];
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb) fb[cur][nb] = Wl[(kb * NB + nb) * 64 + l];
                    }
                    if (kb > 0) {
                        const int prv = (kb - 1) & 1;
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                            for (int r = 0; r < RW; ++r) acc[r][nb] = mfma(fa[prv][r], fb[prv][nb], acc[r][nb]);
                    }
                    if (kb > 0 && kb < KB) {
                        __builtin_amdgcn_sched_group_barrier(0x100, RW + NB, 0);
                        __builtin_amdgcn_sched_group_barrier(0x008, RW * NB, 0);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            if (z + 1 < z1) stage_store<CINP>(In + ((sb + 3) & 3) * S::PLANE, cur);

            // epilogue: lane holds D[4 grp + i][xl]: cell x0 + 4 grp + i,
            // channel 16 nb + xl
            if (EPI == EPI_F32_SOA) {
                // four consecutive cells of channel xl: one 16-byte store
                // when they are all inside the mesh and aligned
                const int xa = x0 + 4 * grp;
                const bool vec = (g.nx & 3) == 0 && xa + 3 < g.nx;
                double pl_sum = 0.0;  // this plane's stored values of channel xl
#pragma unroll
                for (int r = 0; r < RW; ++r) {
                    const int y = y0 + RW * rowg + r;
                    if (y >= g.ny || xl >= cout_valid) continue;
                    float* o = (float*)out + xl * ncell + ((long long)z * g.ny + y) * g.nx + xa;
                    const float b0 = bv[0];
                    if (vec) {
                        *(f32x4*)o = f32x4{acc[r][0][0] + b0, acc[r][0][1] + b0, acc[r][0][2] + b0,
                                           acc[r][0][3] + b0};
                    } else {
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            if (xa + i < g.nx) o[i] = acc[r][0][i] + b0;
                    }
                    if (ms_out.part) {
                        // the correction's mean removal: the stored values,
                        // clipped as the correction clips them
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            double q = (double)(acc[r][0][i] + b0);
                            if (ms_out.clip > 0.0) q = fmin(fmax(q, -ms_out.clip), ms_out.clip);
                            pl_sum += (xa + i < g.nx) ? q : 0.0;
                        }
                    }
                }
                if (ms_out.part) two_sum_add(msum, mcomp, pl_sum);
            } else {
                const int x = x0 + 4 * grp + q;
#pragma unroll
                for (int r = 0; r < RW; ++r) {
                    const int y = y0 + RW * rowg + r;
                    const long long v = ((long long)z * g.ny + y) * g.nx + x;
#pragma unroll
                    for (int nb = 0; nb < NBW; ++nb) {
                        float t[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            t[i] = (EPI == EPI_RELU_BF16) ? fmaxf(acc[r][nb][i] + bv[nb], 0.0f)
                                                          : acc[r][nb][i];
                        quad_transpose(t, q);
                        uint2 w;
                        w.x = pack_bf16(t[0], t[1]);
                        w.y = pack_bf16(t[2], t[3]);
                        if (EPI == EPI_MASK_BF16) {
                            // keep a gradient where its mask entry is positive
                            const uint2 m = mk[r][nb];
                            const unsigned lo0 = (m.x & 0x7FFFu) ? 0xFFFFu : 0u;
                            const unsigned hi0 = (m.x & 0x7FFF0000u) ? 0xFFFF0000u : 0u;
                            const unsigned lo1 = (m.y & 0x7FFFu) ? 0xFFFFu : 0u;
                            const unsigned hi1 = (m.y & 0x7FFF0000u) ? 0xFFFF0000u : 0u;
                            w.x &= lo0 | hi0;
                            w.y &= lo1 | hi1;
                        }
                        if (x < g.nx && y < g.ny) *(uint2*)((u16*)out + v * COUT + 16 * (nb0 + nb) + cq) = w;
                    }
                }
            }
            __syncthreads();  // plane z+2 is in the ring; plane z-1's slot is free
            sb = (sb + 1) & 3;
        };
        for (int z = z0; z < z1; z += 2) {
            plane(z, pa, pb);
            if (z + 1 < z1) plane(z + 1, pb, pa);
        }
    }
    if constexpr (EPI == EPI_F32_SOA) {
        if (ms_out.part) {
            // per-workgroup sums of the NF channels (cout_valid = NF): lanes
            // xl, xl + 16, xl + 32, xl + 48 of a wave, then the waves in
            // order
            __shared__ double wsum[CONV_THREADS / 64][16][2];
            for (int off = 16; off < 64; off <<= 1) {
                const double s2 = __shfl_xor(msum, off), c2 = __shfl_xor(mcomp, off);
                two_sum_add(msum, mcomp, s2);
                mcomp += c2;
            }
            if (l < 16) {
                wsum[wave][l][0] = msum;
                wsum[wave][l][1] = mcomp;
            }
            __syncthreads();
            if (threadIdx.x < NF) {
                double S = 0.0, C = 0.0;
                for (int w = 0; w < CONV_THREADS / 64; ++w) {
                    two_sum_add(S, C, wsum[w][threadIdx.x][0]);
                    C += wsum[w][threadIdx.x][1];
                }
                ms_out.part[blockIdx.x * NF + threadIdx.x] = S + C;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient
// ---------------------------------------------------------------------------

// CL [v][C] -> RV copies out[s] of C16 channels (channels >= C are zero),
// copy s shifted by s - (ns == 3 ? 1 : 0) along x.  One thread per 8
// consecutive cells of a row (nx a multiple of 8, C of 8): it loads the 10
// cells x0-1 .. x0+8 as 16-byte chunks of 8 channels and writes each channel
// of each copy as one 16-byte store of 8 cells.
__global__ void to_vm_kernel(const u16* __restrict__ in, int C, int C16, int ns, int nx, int ny,
                             int nz, int periodic, u16* __restrict__ out)
{
    const long long ncell = (long long)nx * ny * nz;
    const int nx8 = nx / 8;
    const long long units = ncell / 8;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < units;
         e += (long long)gridDim.x * blockDim.x) {
        const long long row = e / nx8;
        const int x0 = (int)(e - row * nx8) * 8;
        const u16* src = in + row * nx * C;
        for (int c8 = 0; c8 < C16 / 8; ++c8) {
            // cells x0-1 .. x0+8: 8 channels each as 4 words
            unsigned w[10][4];
#pragma unroll
            for (int i = 0; i < 10; ++i) {
                const int xs = wrap_or_clamp(x0 - 1 + i, nx, periodic);
                u32x4 t = u32x4{0u, 0u, 0u, 0u};
                if (8 * c8 < C) t = *(const u32x4*)(src + (long long)xs * C + 8 * c8);
#pragma unroll
                for (int q = 0; q < 4; ++q) w[i][q] = t[q];
            }
            for (int s = 0; s < ns; ++s) {
                const int sh = s - (ns == 3 ? 1 : 0);  // copy s holds cell x + sh at x
                u16* o = out + (long long)s * C16 * ncell + (row * C16 + 8 * c8) * nx + x0;
#pragma unroll
                for (int ch = 0; ch < 8; ++ch) {
                    const int q = ch >> 1, hi = ch & 1;
                    u32x4 v;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        // cells 2k, 2k+1 of the window start at index 1 + sh
                        const unsigned a = w[1 + sh + 2 * k][q], b = w[2 + sh + 2 * k][q];
                        const unsigned lo = hi ? (a >> 16) : (a & 0xFFFFu);
                        const unsigned hb = hi ? (b & 0xFFFF0000u) : (b << 16);
                        v[k] = lo | hb;
                    }
                    *(u32x4*)(o + (long long)ch * nx) = v;
                }
            }
        }
    }
}

// Partial weight gradients.  Xs: RV input copies [3] of MB 16 channels
// (shifted by dx = -1, 0, +1); dA: RV output gradient of NB 16 channels.  Workgroup b sums over
// its share of the mesh rows (z, y), for all 27 taps: wave w of its nine
// handles the taps (dz, dy) = (w / 3 - 1, w % 3 - 1) with dx = -1, 0, +1, so
// that each operand row is fetched from memory about once and the nine waves
// reuse it through the caches (per tap, a walk over the whole mesh re-read
// all operands 27 times).  Each (tap, workgroup) writes one partial
// [MB 16][NB 16]; a second kernel sums them in a fixed order.
constexpr int WG_WAVES = 9;

template <int MB, int NB>
__global__ void __launch_bounds__(64 * WG_WAVES)
wgrad_kernel(const u16* __restrict__ Xs, const u16* __restrict__ dA, float* __restrict__ partial,
             int nx, int ny, int nz, int periodic)
{
    constexpr int CI16 = 16 * MB, CO16 = 16 * NB;
    // the walk over rows is the same for all lanes of a wave: keep it in
    // scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int l = threadIdx.x & 63;
    const int xl = l & 15, grp = l >> 4;
    const int dz = wave / 3 - 1, dy = wave % 3 - 1;
    const long long ncell = (long long)nx * ny * nz;
    const int nxb = nx / 32;
    const long long rows = (long long)nz * ny;
    const long long parts = gridDim.x, me = blockIdx.x;
    const long long r0 = rows * me / parts, r1 = rows * (me + 1) / parts;

    f32x4 acc[3][MB][NB];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int n = 0; n < NB; ++n) acc[d][m][n] = f32x4{0.f, 0.f, 0.f, 0.f};

    // per-lane channel rows of the operands: A = input copy shifted by dx =
    // d - 1, B = output gradient; fragment of 8 cells at x offset 8 grp
    const u16* pa[3][MB];
    const u16* pb[NB];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int m = 0; m < MB; ++m)
            pa[d][m] = Xs + (long long)d * CI16 * ncell + (16 * m + xl) * nx + 8 * grp;
#pragma unroll
    for (int n = 0; n < NB; ++n) pb[n] = dA + (16 * n + xl) * nx + 8 * grp;

    // K steps of 32 cells along each row
    int z = (int)(r0 / ny), y = (int)(r0 % ny);
    for (long long r = r0; r < r1; ++r) {
        const int zi = z + dz, yi = y + dy;
        const int zs = periodic ? (zi < 0 ? zi + nz : (zi >= nz ? zi - nz : zi)) : min(max(zi, 0), nz - 1);
        const int ys = periodic ? (yi < 0 ? yi + ny : (yi >= ny ? yi - ny : yi)) : min(max(yi, 0), ny - 1);
        const long long vin = ((long long)zs * ny + ys) * CI16 * nx;
        const long long vout = r * CO16 * nx;
        // two K steps in flight: all their loads, then their products
        for (int xb = 0; xb < nxb; xb += 2) {
            constexpr int S2 = 2;
            u32x4 a[S2][3][MB], b[S2][NB];
#pragma unroll
            for (int k = 0; k < S2; ++k) {
                const int xo = 32 * min(xb + k, nxb - 1);
#pragma unroll
                for (int d = 0; d < 3; ++d)
#pragma unroll
                    for (int m = 0; m < MB; ++m) a[k][d][m] = *(const u32x4*)(pa[d][m] + vin + xo);
#pragma unroll
                for (int n = 0; n < NB; ++n) b[k][n] = *(const u32x4*)(pb[n] + vout + xo);
            }
            // a step past the row end multiplies zeros (its loads repeat the
            // last block), which leaves the sums unchanged
            const bool ok = xb + 1 < nxb;
#pragma unroll
            for (int n = 0; n < NB; ++n) b[1][n] = ok ? b[1][n] : u32x4{0u, 0u, 0u, 0u};
#pragma unroll
            for (int k = 0; k < S2; ++k)
#pragma unroll
                for (int d = 0; d < 3; ++d)
#pragma unroll
                    for (int m = 0; m < MB; ++m)
#pragma unroll
                        for (int n = 0; n < NB; ++n)
                            acc[d][m][n] = mfma(a[k][d][m], b[k][n], acc[d][m][n]);
        }
        ++y;
        if (y == ny) {
            y = 0;
            ++z;
        }
    }
    // D[4 grp + i][xl] of block (m, n): input channel 16 m + 4 grp + i,
    // output channel 16 n + xl
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int tap = (dz + 1) * 9 + (dy + 1) * 3 + d;
        float* p = partial + ((long long)tap * parts + me) * CI16 * CO16;
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int n = 0; n < NB; ++n)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    p[(16 * m + 4 * grp + i) * CO16 + 16 * n + xl] = acc[d][m][n][i];
    }
}

// Gradient of the master weights W[cout][cin][27]: sum of the partials of
// every workgroup in a fixed order.  A workgroup sums 32 entries (ci, co) of
// one tap, e = (t ci16 + ci) co16 + co, so consecutive threads read
// consecutive partial entries: each of its 8 thread rows adds one eighth of
// the partials in order, then the eight sums are added in order.
constexpr int RED_SPLIT = 8;

__global__ void __launch_bounds__(THREADS)
wgrad_reduce_kernel(const float* __restrict__ partial, int parts, int ci16, int co16, int cin,
                    int cout, float* __restrict__ gW)
{
    constexpr int EPB = THREADS / RED_SPLIT;  // entries per workgroup
    __shared__ float sums[RED_SPLIT][EPB];
    const int total = TAPS * ci16 * co16;
    const int le = threadIdx.x % EPB, q = threadIdx.x / EPB;
    const int e = blockIdx.x * EPB + le;
    float s = 0.0f;
    if (e < total) {
        const int tap = e / (co16 * ci16), rem = e - tap * co16 * ci16;
        const float* p = partial + (long long)tap * parts * ci16 * co16 + rem;
        const int k0 = parts * q / RED_SPLIT, k1 = parts * (q + 1) / RED_SPLIT;
        for (int k = k0; k < k1; ++k) s += p[(long long)k * ci16 * co16];
    }
    sums[q][le] = s;
    __syncthreads();
    if (q == 0 && e < total) {
        float t = sums[0][le];
#pragma unroll
        for (int r = 1; r < RED_SPLIT; ++r) t += sums[r][le];
        const int co = e % co16, ci = (e / co16) % ci16, tap = e / (co16 * ci16);
        if (co < cout && ci < cin) gW[(co * cin + ci) * TAPS + tap] = t;
    }
}

// Bias gradient: sums over cells of the RV BF16 output gradient dA (C
// channels); workgroup (c, j) sums the j-th of BIAS_CHUNKS shares of channel
// c, then one thread per channel adds the shares in order.
constexpr int BIAS_CHUNKS = 64;

__global__ void __launch_bounds__(THREADS)
bias_partial_kernel(const u16* __restrict__ dA, long long ncell, int C, int nx,
                    float* __restrict__ part)
{
    __shared__ float red[THREADS];
    const int c = blockIdx.x / BIAS_CHUNKS, j = blockIdx.x % BIAS_CHUNKS;
    const long long beg = ncell * j / BIAS_CHUNKS, end = ncell * (j + 1) / BIAS_CHUNKS;
    float s = 0.0f;
    for (long long v = beg + threadIdx.x; v < end; v += THREADS) {
        const int row = (int)(v / nx), x = (int)(v - (long long)row * nx);
        s += bf2f(dA[((long long)row * C + c) * nx + x]);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = THREADS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void bias_final_kernel(const float* __restrict__ part, int C, float* __restrict__ gb)
{
    const int c = threadIdx.x;
    if (c >= C) return;
    float s = 0.0f;
    for (int j = 0; j < BIAS_CHUNKS; ++j) s += part[c * BIAS_CHUNKS + j];
    gb[c] = s;
}

// ---------------------------------------------------------------------------
// input packing, targets, loss, optimizer
// ---------------------------------------------------------------------------

// Inputs and correction scales.  mode 0: inputs are the conserved fields,
// corrections are tau (y - mean y).  mode 1 (scale-aware): inputs are
// (log rho, v_x, v_y, v_z, log p) and the correction of field f is
// tau_f (S_f y_f - mean(S_f y_f)) with local scales S = (rho, rho c, rho c,
// rho c, E) of the cell; both normalised per input by mu, sigma.
struct Norm {
    float mu[NF], inv_sigma[NF];
    double tau[NF], inv_tau[NF];
    double gamma;
    double clip;  // > 0: the applied output is clamped to [-clip, clip]
    int mode;
};

// primitives of a cell in FP64 (no positivity guard: callers clamp logs
// and square roots)
__device__ __forceinline__ void cell_prims(const double u[NF], double gamma, double& rho,
                                           double v[3], double& p)
{
    rho = u[0];
    const double ir = 1.0 / rho;
    v[0] = u[1] * ir;
    v[1] = u[2] * ir;
    v[2] = u[3] * ir;
    p = (gamma - 1.0) * (u[4] - 0.5 * ((u[1] * v[0] + u[2] * v[1]) + u[3] * v[2]));
}

// local correction scales S of a cell (mode 1), from its FP64 values
__device__ __forceinline__ void cell_scales(const double u[NF], double gamma, double S[NF])
{
    double rho, v[3], p;
    cell_prims(u, gamma, rho, v, p);
    const double rc = sqrt(fmax(gamma * p * rho, 1e-300));
    S[0] = rho;
    S[1] = S[2] = S[3] = rc;
    S[4] = u[4];
}

// head of an FP32 pair -> CL BF16 [v][8] of (feature - mu) / sigma,
// channels 5..7 = 0
__global__ void pack_input_kernel(const float* __restrict__ U, long long ncell, Norm nm,
                                  u16* __restrict__ X)
{
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < ncell;
         v += (long long)gridDim.x * blockDim.x) {
        float feat[NF];
        if (nm.mode == 1) {
            double u[NF], rho, vel[3], p;
            for (int f = 0; f < NF; ++f) u[f] = (double)U[f * ncell + v];
            cell_prims(u, nm.gamma, rho, vel, p);
            feat[0] = (float)log(fmax(rho, 1e-300));
            feat[1] = (float)vel[0];
            feat[2] = (float)vel[1];
            feat[3] = (float)vel[2];
            feat[4] = (float)log(fmax(p, 1e-300));
        } else {
            for (int f = 0; f < NF; ++f) feat[f] = U[f * ncell + v];
        }
        u16 x[8];
#pragma unroll
        for (int f = 0; f < NF; ++f) x[f] = f2bf((feat[f] - nm.mu[f]) * nm.inv_sigma[f]);
        x[5] = x[6] = x[7] = 0;
        u32x4 w;
        w[0] = x[0] | ((unsigned)x[1] << 16);
        w[1] = x[2] | ((unsigned)x[3] << 16);
        w[2] = x[4] | ((unsigned)x[5] << 16);
        w[3] = x[6] | ((unsigned)x[7] << 16);
        *(u32x4*)(X + v * 8) = w;
    }
}

// mean of the 2x2x2 fine cells over coarse cell (x, y, z), field f, FP64
__device__ __forceinline__ double restrict_cell(const double* __restrict__ fine, int f, int x,
                                                int y, int z, int nx, int ny, int nz)
{
    const long long fx = 2LL * nx, fy = 2LL * ny, fz = 2LL * nz;
    const double* p = fine + (long long)f * fx * fy * fz;
    double s = 0.0;
    for (int k = 0; k < 2; ++k)
        for (int j = 0; j < 2; ++j)
            for (int i = 0; i < 2; ++i) s += p[((2LL * z + k) * fy + 2 * y + j) * fx + 2 * x + i];
    return s * 0.125;
}

// mode 0: U = R(fine) as an FP32 pair; mode 1: target = (R(fine) - (head -
// comp)) / tau
__global__ void restrict_kernel(const double* __restrict__ fine, int nx, int ny, int nz, int mode,
                                float* __restrict__ U, float* __restrict__ target, Norm nm)
{
    const long long ncell = (long long)nx * ny * nz;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < ncell;
         v += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((long long)nx * ny));
        for (int f = 0; f < NF; ++f) {
            const double r = restrict_cell(fine, f, x, y, z, nx, ny, nz);
            if (mode == 0) {
                const float head = (float)r;
                U[f * ncell + v] = head;
                U[(NF + f) * ncell + v] = (float)((double)head - r);
            } else {
                double u[NF], S[NF];
                for (int g = 0; g < NF; ++g)
                    u[g] = (double)U[g * ncell + v] - (double)U[(NF + g) * ncell + v];
                if (nm.mode == 1) cell_scales(u, nm.gamma, S);
                const double scale = nm.mode == 1 ? nm.tau[f] * S[f] : nm.tau[f];
                target[f * ncell + v] = (float)((r - u[f]) / scale);
            }
        }
    }
}

// MSE loss partials (FP64, one per workgroup) and the output gradient
// 2 (y - t) / N as BF16, CL [v][8] (channels 5..7 zero) and RV (16 channels)
// (channels 5..15 zero)
__global__ void __launch_bounds__(THREADS)
loss_kernel(const float* __restrict__ y, const float* __restrict__ t, long long ncell, int nx,
            double* __restrict__ partial, u16* __restrict__ dCL, u16* __restrict__ dVM)
{
    __shared__ double red[THREADS];
    const float scale = (float)(2.0 / (double)(ncell * NF));
    double s = 0.0;
    for (long long v = (long long)blockIdx.x * THREADS + threadIdx.x; v < ncell;
         v += (long long)gridDim.x * THREADS) {
        u16 d[8];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const float e = y[f * ncell + v] - t[f * ncell + v];
            s += (double)e * (double)e;
            d[f] = f2bf(scale * e);
        }
        d[5] = d[6] = d[7] = 0;
        // RV copy of 16 channels (5 used)
        const int row = (int)(v / nx), x = (int)(v - (long long)row * nx);
        u16* o = dVM + (long long)row * 16 * nx + x;
        for (int f = 0; f < 16; ++f) o[(long long)f * nx] = f < NF ? d[f] : (u16)0;
        u32x4 w;
        w[0] = d[0] | ((unsigned)d[1] << 16);
        w[1] = d[2] | ((unsigned)d[3] << 16);
        w[2] = d[4] | ((unsigned)d[5] << 16);
        w[3] = d[6] | ((unsigned)d[7] << 16);
        *(u32x4*)(dCL + v * 8) = w;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = THREADS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Adam (Kingma and Ba, Algorithm 1); c1 = 1 / (1 - beta1^t), c2 = 1 / (1 -
// beta2^t)
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v2, int n, float lr, float c1, float c2)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v2[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v2[i] = vi;
        p[i] = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    }
}

// ---------------------------------------------------------------------------
// correction with fallback
// ---------------------------------------------------------------------------

// the per-field quantity whose mean the correction removes: y (mode 0) or
// S y (mode 1), S from the head of U; from the cell's values of both
__device__ __forceinline__ void scaled_from(const float head[NF], const float yv[NF], const Norm& nm,
                                            double out[NF])
{
    double S[NF] = {1.0, 1.0, 1.0, 1.0, 1.0};
    if (nm.mode == 1) {
        double u[NF];
        for (int f = 0; f < NF; ++f) u[f] = (double)head[f];
        cell_scales(u, nm.gamma, S);
    }
    for (int f = 0; f < NF; ++f) {
        double yy = (double)yv[f];
        if (nm.clip > 0.0) yy = fmin(fmax(yy, -nm.clip), nm.clip);
        out[f] = S[f] * yy;
    }
}

// the same, loading cell v of U's head and of y (all loads issued first)
__device__ __forceinline__ void scaled_output(const float* __restrict__ U, const float* __restrict__ y,
                                              long long ncell, long long v, const Norm& nm,
                                              double out[NF])
{
    float head[NF] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f}, yv[NF];
    for (int f = 0; f < NF; ++f) yv[f] = y[f * ncell + v];
    if (nm.mode == 1)
        for (int f = 0; f < NF; ++f) head[f] = U[f * ncell + v];
    scaled_from(head, yv, nm, out);
}

__global__ void __launch_bounds__(THREADS)
mean_partial_kernel(const float* __restrict__ U, const float* __restrict__ y, long long ncell,
                    Norm nm, double* __restrict__ partial)
{
    __shared__ double rs[NF][THREADS / 64], rc[NF][THREADS / 64];
    double s[NF], c[NF];
    for (int f = 0; f < NF; ++f) s[f] = c[f] = 0.0;
    for (long long v = (long long)blockIdx.x * THREADS + threadIdx.x; v < ncell;
         v += (long long)gridDim.x * THREADS) {
        double q[NF];
        scaled_output(U, y, ncell, v, nm, q);
        for (int f = 0; f < NF; ++f) two_sum_add(s[f], c[f], q[f]);
    }
    for (int f = 0; f < NF; ++f) {
        for (int off = 32; off > 0; off >>= 1) {
            double s2 = __shfl_xor(s[f], off), c2 = __shfl_xor(c[f], off);
            two_sum_add(s[f], c[f], s2);
            c[f] += c2;
        }
        if ((threadIdx.x & 63) == 0) {
            rs[f][threadIdx.x >> 6] = s[f];
            rc[f][threadIdx.x >> 6] = c[f];
        }
    }
    __syncthreads();
    if (threadIdx.x < NF) {
        const int f = threadIdx.x;
        double S = 0.0, C = 0.0;
        for (int w = 0; w < THREADS / 64; ++w) {
            two_sum_add(S, C, rs[f][w]);
            C += rc[f][w];
        }
        partial[blockIdx.x * NF + f] = S + C;
    }
}

// the mean of y (or S y) from n block partials, as its own one-workgroup
// launch (five waves)
__global__ void __launch_bounds__(64 * NF)
mean_final_kernel(const double* __restrict__ partial, int n, long long ncell,
                  CorrState* __restrict__ cs)
{
    mean_body(partial, n, ncell, cs);
}

// The corrected pair of one cell and field: delta = tau (q - mean) rounded
// to FP32 and Kahan-added into (head, comp).  The check and the commit both
// call it, so the committed values are the checked ones, bit for bit.
__device__ __forceinline__ void candidate(float head, float comp, double q, double tau, double mean,
                                          float& s, float& c2)
{
    const float d = (float)(tau * (q - mean));
    const float yy = d - comp;
    s = head + yy;
    c2 = (s - head) - yy;
}

// Check of the candidate corrected pair, without storing it: positivity of
// every candidate cell (FP64 primitive recovery) and per-block sums of the
// represented change and of its magnitude.
__global__ void __launch_bounds__(THREADS)
check_kernel(const float* __restrict__ U, const float* __restrict__ y, long long ncell, Norm nm,
             gs::Phys k, const CorrState* csr, double* __restrict__ partial, CorrState* cs)
{
    __shared__ double red[2 * NF][THREADS];
    double moved[NF], mag[NF], mean[NF];
    for (int f = 0; f < NF; ++f) {
        moved[f] = mag[f] = 0.0;
        mean[f] = csr->mean[f];
    }
    bool bad = false;
    for (long long v = (long long)blockIdx.x * THREADS + threadIdx.x; v < ncell;
         v += (long long)gridDim.x * THREADS) {
        double u[NF], w[NF], q[NF];
        float head[NF], comp[NF], yv[NF];
        for (int f = 0; f < NF; ++f) {
            head[f] = U[f * ncell + v];
            comp[f] = U[(NF + f) * ncell + v];
            yv[f] = y[f * ncell + v];
        }
        scaled_from(head, yv, nm, q);
        for (int f = 0; f < NF; ++f) {
            float s, c2;
            candidate(head[f], comp[f], q[f], nm.tau[f], mean[f], s, c2);
            const double change = ((double)s - (double)c2) - ((double)head[f] - (double)comp[f]);
            moved[f] += change;
            mag[f] += fabs(change);
            u[f] = (double)s - (double)c2;
        }
        bad |= !gs::cons_to_prim(u, w, k);
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&cs->bad, 1u);
    for (int f = 0; f < NF; ++f) {
        red[2 * f][threadIdx.x] = moved[f];
        red[2 * f + 1][threadIdx.x] = mag[f];
    }
    __syncthreads();
    for (int w = THREADS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int q = 0; q < 2 * NF; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 2 * NF) partial[blockIdx.x * 2 * NF + threadIdx.x] = red[threadIdx.x][0];
}

// the decision from n block partials of check_kernel (five waves)
__global__ void __launch_bounds__(64 * NF)
decide_kernel(const double* __restrict__ partial, int n, CorrState* __restrict__ cs)
{
    decide_body(partial, n, cs);
}

// If the decision accepted the candidate, write it into U in place: each
// thread recomputes the candidate of its own cells (the same arithmetic as
// check_kernel) from U and y before overwriting them.
__global__ void __launch_bounds__(THREADS)
commit_kernel(float* __restrict__ U, const float* __restrict__ y, long long ncell, Norm nm,
              const CorrState* __restrict__ cs)
{
    if (!cs->ok) return;
    double mean[NF];
    for (int f = 0; f < NF; ++f) mean[f] = cs->mean[f];
    for (long long v = (long long)blockIdx.x * THREADS + threadIdx.x; v < ncell;
         v += (long long)gridDim.x * THREADS) {
        double q[NF];
        float head[NF], comp[NF], yv[NF];
        for (int f = 0; f < NF; ++f) {
            head[f] = U[f * ncell + v];
            comp[f] = U[(NF + f) * ncell + v];
            yv[f] = y[f * ncell + v];
        }
        scaled_from(head, yv, nm, q);
        float s[NF], c2[NF];
        for (int f = 0; f < NF; ++f) candidate(head[f], comp[f], q[f], nm.tau[f], mean[f], s[f], c2[f]);
        for (int f = 0; f < NF; ++f) {
            U[f * ncell + v] = s[f];
            U[(NF + f) * ncell + v] = c2[f];
        }
    }
}

__global__ void init_corr_kernel(CorrState* cs)
{
    for (int f = 0; f < NF; ++f) cs->mean[f] = cs->moved[f] = cs->mag[f] = 0.0;
    cs->bad = 0u;
    cs->applied = cs->fallbacks = 0;
    cs->ok = 0;
}

__global__ void zero_floats_kernel(float* p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.0f;
}

}  // namespace gsc

// ===========================================================================
// Host side
// ===========================================================================

using namespace gsc;

namespace {

thread_local std::string g_cnn_create_error;

constexpr int RED_BLOCKS = 512;
constexpr int WG_PARTS = 512;  // workgroups (partial sums per tap) of the weight gradient

}  // namespace

struct gs_cnn {
    int nx, ny, nz, bc;
    double gamma;
    hipStream_t stream;
    std::string err;
    long long ncell;
    Norm norm;
    int step;  // Adam step count
    // parameters, gradients, moments (FP32)
    float *P, *G, *M, *V;
    // packed weights: forward l1, l2, l3; backward (mirrored) l2, l3
    u16 *wf1, *wf2, *wf3, *wb2, *wb3;
    // activations (CL): input x (8), h1, h2 (32); output y, FP32 SoA
    u16 *x, *h1, *h2;
    float* y;
    // training: gradients dY (CL 8, RV 16), dA2, dA1 (CL 32, RV 32), RV
    // shifted copies of x (16 ch), h1, h2 (32 ch)
    u16 *dY, *dYv, *dA2, *dA2v, *dA1, *dA1v, *xs, *h1s, *h2s;
    float* wpart;   // weight-gradient partials
    float* bpart;   // bias-gradient partials
    double* red;    // reduction partials
    double* host_red;
    CorrState* cs;
    CorrState* host_cs;
};

namespace {

int cfail(gs_cnn* h, int code, const std::string& msg)
{
    if (h)
        h->err = msg;
    else
        g_cnn_create_error = msg;
    return code;
}

int chip(gs_cnn* h, hipError_t e, const char* what)
{
    return cfail(h, GS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

int grid_for(long long n, int per = THREADS, int cap = 4096)
{
    long long b = (n + per - 1) / per;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

ConvGeom conv_geom(const gs_cnn* h)
{
    ConvGeom g;
    g.nx = h->nx;
    g.ny = h->ny;
    g.nz = h->nz;
    g.periodic = h->bc == GS_BC_PERIODIC;
    g.ntx = (h->nx + 15) / 16;
    g.nty = (h->ny + 15) / 16;
    const int ntile = g.ntx * g.nty;
    // about 1024 work items (a few per resident workgroup), each as many
    // planes as that allows: longer chunks stage fewer halo planes
    long long want = (1024 + ntile - 1) / ntile;
    int kz = (int)((h->nz + want - 1) / want);
    g.kz = kz < 1 ? 1 : kz;
    g.items = ntile * ((g.nz + g.kz - 1) / g.kz);
    return g;
}

// persistent grid of a convolution kernel: its resident workgroups, at most
// one per work item
template <int CINP, int NB, int EPI>
int conv_grid(const ConvGeom& g)
{
    static int resident = 0;
    if (resident == 0) {
        int dev = 0, per_cu = 0, cus = 256;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            cus = p.multiProcessorCount;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, conv_kernel<CINP, NB, EPI>,
                                                         CONV_THREADS, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        resident = per_cu * cus;
    }
    return std::min(resident, g.items);
}

template <int CINP, int NB, int EPI>
void launch_conv(gs_cnn* h, const ConvGeom& g, const u16* X, const u16* Wp, const float* bias, void* out,
                 const u16* mask, int cout_valid, MeanSums ms = MeanSums{})
{
    hipLaunchKernelGGL((conv_kernel<CINP, NB, EPI>), dim3(conv_grid<CINP, NB, EPI>(g)), dim3(CONV_THREADS), 0,
                       h->stream, X, Wp, bias, out, mask, g, cout_valid, ms);
}

hipError_t pack_all(gs_cnn* h)
{
    const int blocks = 64;
    hipLaunchKernelGGL(pack_weights_kernel, dim3(blocks), dim3(THREADS), 0, h->stream, h->P + W1_OFF,
                       NF, HID, 8, 2, 7, 0, h->wf1);
    hipLaunchKernelGGL(pack_weights_kernel, dim3(blocks), dim3(THREADS), 0, h->stream, h->P + W2_OFF,
                       HID, HID, 32, 2, TAPS, 0, h->wf2);
    hipLaunchKernelGGL(pack_weights_kernel, dim3(blocks), dim3(THREADS), 0, h->stream, h->P + W3_OFF,
                       HID, NF, 32, 1, TAPS, 0, h->wf3);
    // mirrored: layer 2 (in 32 -> out 32), layer 3 (in: 5 gradient channels
    // padded to 8 -> out 32)
    hipLaunchKernelGGL(pack_weights_kernel, dim3(blocks), dim3(THREADS), 0, h->stream, h->P + W2_OFF,
                       HID, HID, 32, 2, TAPS, 1, h->wb2);
    hipLaunchKernelGGL(pack_weights_kernel, dim3(blocks), dim3(THREADS), 0, h->stream, h->P + W3_OFF,
                       HID, NF, 8, 2, 7, 1, h->wb3);
    return hipGetLastError();
}

// forward pass from the head of U; keeps x, h1, h2; writes y (and, with
// ms.part, the sums of y for the correction's mean removal)
hipError_t forward(gs_cnn* h, const float* U, MeanSums ms = MeanSums{})
{
    const ConvGeom g = conv_geom(h);
    hipLaunchKernelGGL(pack_input_kernel, dim3(grid_for(h->ncell)), dim3(THREADS), 0, h->stream, U,
                       h->ncell, h->norm, h->x);
    launch_conv<8, 2, EPI_RELU_BF16>(h, g, h->x, h->wf1, h->P + B1_OFF, h->h1, nullptr, HID);
    launch_conv<32, 2, EPI_RELU_BF16>(h, g, h->h1, h->wf2, h->P + B2_OFF, h->h2, nullptr, HID);
    launch_conv<32, 1, EPI_F32_SOA>(h, g, h->h2, h->wf3, h->P + B3_OFF, h->y, nullptr, NF, ms);
    return hipGetLastError();
}

// bias gradients of the first C of the Cs channels of an RV array
void bias_grad(gs_cnn* h, const u16* dAv, int C, int Cs, float* gb)
{
    hipLaunchKernelGGL(bias_partial_kernel, dim3(C * BIAS_CHUNKS), dim3(THREADS), 0, h->stream, dAv,
                       h->ncell, Cs, h->nx, h->bpart);
    hipLaunchKernelGGL(bias_final_kernel, dim3(1), dim3(64), 0, h->stream, h->bpart, C, gb);
}

// loss and all parameter gradients into G (after forward); loss partials in
// red[0 .. RED_BLOCKS)
hipError_t backward(gs_cnn* h, const float* target)
{
    const ConvGeom g = conv_geom(h);
    const long long n = h->ncell;
    hipLaunchKernelGGL(loss_kernel, dim3(RED_BLOCKS), dim3(THREADS), 0, h->stream, h->y, target, n, h->nx,
                       h->red, h->dY, h->dYv);
    // layer 3: dW3 from h2 and dY; dH2 = conv(dY, mirrored W3) masked by h2
    hipLaunchKernelGGL(to_vm_kernel, dim3(grid_for(n / 8)), dim3(THREADS), 0, h->stream, h->h2, HID,
                       HID, 3, h->nx, h->ny, h->nz, 1, h->h2s);
    const int parts = WG_PARTS;
    const int rgrid = TAPS * 32 * 32 / (THREADS / RED_SPLIT);  // 32 entries per workgroup
    hipLaunchKernelGGL((wgrad_kernel<2, 1>), dim3(WG_PARTS), dim3(64 * WG_WAVES), 0, h->stream,
                       h->h2s, h->dYv, h->wpart, h->nx, h->ny, h->nz, 1);
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(rgrid), dim3(THREADS), 0, h->stream,
                       h->wpart, parts, 32, 16, HID, NF, h->G + W3_OFF);
    bias_grad(h, h->dYv, NF, 16, h->G + B3_OFF);
    launch_conv<8, 2, EPI_MASK_BF16>(h, g, h->dY, h->wb3, nullptr, h->dA2, h->h2, HID);
    // layer 2
    hipLaunchKernelGGL(to_vm_kernel, dim3(grid_for(n / 8)), dim3(THREADS), 0, h->stream, h->dA2, HID, HID,
                       1, h->nx, h->ny, h->nz, 1, h->dA2v);
    hipLaunchKernelGGL(to_vm_kernel, dim3(grid_for(n / 8)), dim3(THREADS), 0, h->stream, h->h1, HID,
                       HID, 3, h->nx, h->ny, h->nz, 1, h->h1s);
    hipLaunchKernelGGL((wgrad_kernel<2, 2>), dim3(WG_PARTS), dim3(64 * WG_WAVES), 0, h->stream,
                       h->h1s, h->dA2v, h->wpart, h->nx, h->ny, h->nz, 1);
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(rgrid), dim3(THREADS), 0, h->stream,
                       h->wpart, parts, 32, 32, HID, HID, h->G + W2_OFF);
    bias_grad(h, h->dA2v, HID, HID, h->G + B2_OFF);
    launch_conv<32, 2, EPI_MASK_BF16>(h, g, h->dA2, h->wb2, nullptr, h->dA1, h->h1, HID);
    // layer 1
    hipLaunchKernelGGL(to_vm_kernel, dim3(grid_for(n / 8)), dim3(THREADS), 0, h->stream, h->dA1, HID, HID,
                       1, h->nx, h->ny, h->nz, 1, h->dA1v);
    hipLaunchKernelGGL(to_vm_kernel, dim3(grid_for(n / 8)), dim3(THREADS), 0, h->stream, h->x, 8, 16,
                       3, h->nx, h->ny, h->nz, 1, h->xs);
    hipLaunchKernelGGL((wgrad_kernel<1, 2>), dim3(WG_PARTS), dim3(64 * WG_WAVES), 0, h->stream,
                       h->xs, h->dA1v, h->wpart, h->nx, h->ny, h->nz, 1);
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(rgrid), dim3(THREADS), 0, h->stream,
                       h->wpart, parts, 16, 32, NF, HID, h->G + W1_OFF);
    bias_grad(h, h->dA1v, HID, HID, h->G + B1_OFF);
    return hipGetLastError();
}

int read_loss(gs_cnn* h, double* loss)
{
    hipError_t e = hipMemcpyAsync(h->host_red, h->red, RED_BLOCKS * sizeof(double),
                                  hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return chip(h, e, "loss read-back");
    double s = 0.0;
    for (int b = 0; b < RED_BLOCKS; ++b) s += h->host_red[b];
    *loss = s / (double)(h->ncell * NF);
    return GS_OK;
}

int check_train(gs_cnn* h, const void* U, const void* target)
{
    if (!U || !target || !aligned16(U) || !aligned16(target))
        return cfail(h, GS_ERR_ARG, "U or target is NULL or not 16-byte aligned");
    if (h->bc != GS_BC_PERIODIC)
        return cfail(h, GS_ERR_ARG, "training needs periodic boundaries");
    if (h->nx % 32 != 0) return cfail(h, GS_ERR_ARG, "training needs nx to be a multiple of 32");
    return GS_OK;
}

}  // namespace

extern "C" {

int gs_cnn_param_count(void) { return P_N; }

int gs_cnn_create(int nx, int ny, int nz, int bc, double gamma, void* stream, gs_cnn** out)
{
    g_cnn_create_error.clear();
    if (!out) return cfail(nullptr, GS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return cfail(nullptr, GS_ERR_ARG, "mesh sizes must be >= 1");
    if ((long long)nx * ny * nz > (1LL << 28)) return cfail(nullptr, GS_ERR_ARG, "mesh too large");
    if (bc != GS_BC_OUTFLOW && bc != GS_BC_PERIODIC)
        return cfail(nullptr, GS_ERR_ARG, "unknown boundary kind");
    if (!std::isfinite(gamma) || !(gamma > 1.0)) return cfail(nullptr, GS_ERR_ARG, "gamma must be > 1");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return chip(nullptr, e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return chip(nullptr, e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return cfail(nullptr, GS_ERR_HIP, std::string("built for gfx950, device is ") + prop.gcnArchName);

    gs_cnn* h = new gs_cnn();
    std::memset((void*)&h->norm, 0, sizeof(Norm));
    h->nx = nx;
    h->ny = ny;
    h->nz = nz;
    h->bc = bc;
    h->gamma = gamma;
    h->stream = (hipStream_t)stream;
    h->ncell = (long long)nx * ny * nz;
    h->step = 0;
    h->norm.gamma = gamma;
    h->norm.clip = 0.0;
    h->norm.mode = 0;
    for (int f = 0; f < NF; ++f) {
        h->norm.mu[f] = 0.0f;
        h->norm.inv_sigma[f] = 1.0f;
        h->norm.tau[f] = 1.0;
        h->norm.inv_tau[f] = 1.0;
    }
    const long long n = h->ncell;
    struct Alloc {
        void** p;
        size_t bytes;
    } allocs[] = {
        {(void**)&h->P, P_N * 4}, {(void**)&h->G, P_N * 4}, {(void**)&h->M, P_N * 4},
        {(void**)&h->V, P_N * 4},
        {(void**)&h->wf1, 7 * 2 * 1024}, {(void**)&h->wf2, TAPS * 2 * 1024},
        {(void**)&h->wf3, TAPS * 1 * 1024}, {(void**)&h->wb2, TAPS * 2 * 1024},
        {(void**)&h->wb3, 7 * 2 * 1024},
        {(void**)&h->x, (size_t)n * 8 * 2}, {(void**)&h->h1, (size_t)n * 32 * 2},
        {(void**)&h->h2, (size_t)n * 32 * 2}, {(void**)&h->y, (size_t)n * NF * 4},
        {(void**)&h->dY, (size_t)n * 8 * 2}, {(void**)&h->dYv, (size_t)n * 16 * 2},
        {(void**)&h->dA2, (size_t)n * 32 * 2}, {(void**)&h->dA2v, (size_t)n * 32 * 2},
        {(void**)&h->dA1, (size_t)n * 32 * 2}, {(void**)&h->dA1v, (size_t)n * 32 * 2},
        {(void**)&h->xs, (size_t)n * 3 * 16 * 2}, {(void**)&h->h1s, (size_t)n * 3 * 32 * 2},
        {(void**)&h->h2s, (size_t)n * 3 * 32 * 2},
        {(void**)&h->wpart, (size_t)TAPS * WG_PARTS * 32 * 32 * 4},
        {(void**)&h->bpart, (size_t)32 * BIAS_CHUNKS * 4},
        {(void**)&h->red, RED_BLOCKS * 2 * NF * 8},
        {(void**)&h->cs, sizeof(CorrState)},
    };
    for (auto& a : allocs) *a.p = nullptr;
    h->host_red = nullptr;
    h->host_cs = nullptr;
    for (auto& a : allocs) {
        if ((e = hipMalloc(a.p, a.bytes)) != hipSuccess) {
            int r = chip(nullptr, e, "allocation");
            gs_cnn_destroy(h);
            return r;
        }
    }
    if ((e = hipHostMalloc((void**)&h->host_red, RED_BLOCKS * 2 * NF * 8, hipHostMallocDefault)) !=
            hipSuccess ||
        (e = hipHostMalloc((void**)&h->host_cs, sizeof(CorrState), hipHostMallocDefault)) != hipSuccess) {
        int r = chip(nullptr, e, "pinned allocation");
        gs_cnn_destroy(h);
        return r;
    }
    hipLaunchKernelGGL(zero_floats_kernel, dim3(64), dim3(THREADS), 0, h->stream, h->P, P_N);
    hipLaunchKernelGGL(zero_floats_kernel, dim3(64), dim3(THREADS), 0, h->stream, h->M, P_N);
    hipLaunchKernelGGL(zero_floats_kernel, dim3(64), dim3(THREADS), 0, h->stream, h->V, P_N);
    hipLaunchKernelGGL(init_corr_kernel, dim3(1), dim3(1), 0, h->stream, h->cs);
    e = pack_all(h);
    if (e != hipSuccess) {
        int r = chip(nullptr, e, "init kernels");
        gs_cnn_destroy(h);
        return r;
    }
    *out = h;
    return GS_OK;
}

int gs_cnn_set_params(gs_cnn* h, const float* host_params)
{
    if (!h) return cfail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (!host_params) return cfail(h, GS_ERR_ARG, "params is NULL");
    hipError_t e = hipMemcpyAsync(h->P, host_params, P_N * 4, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return chip(h, e, "parameter upload");
    hipLaunchKernelGGL(zero_floats_kernel, dim3(64), dim3(THREADS), 0, h->stream, h->M, P_N);
    hipLaunchKernelGGL(zero_floats_kernel, dim3(64), dim3(THREADS), 0, h->stream, h->V, P_N);
    h->step = 0;
    e = pack_all(h);
    return e == hipSuccess ? GS_OK : chip(h, e, "pack");
}

int gs_cnn_get_params(gs_cnn* h, float* host_params)
{
    if (!h) return cfail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (!host_params) return cfail(h, GS_ERR_ARG, "params is NULL");
    hipError_t e = hipMemcpyAsync(host_params, h->P, P_N * 4, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return e == hipSuccess ? GS_OK : chip(h, e, "parameter download");
}

int gs_cnn_set_norm(gs_cnn* h, const double* mu, const double* sigma, const double* tau)
{
    if (!h) return cfail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (!mu || !sigma || !tau) return cfail(h, GS_ERR_ARG, "NULL array");
    for (int f = 0; f < NF; ++f) {
        if (!std::isfinite(mu[f]) || !(sigma[f] > 0.0) || !std::isfinite(sigma[f]) || !(tau[f] > 0.0) ||
            !std::isfinite(tau[f]))
            return cfail(h, GS_ERR_ARG, "mu must be finite, sigma and tau finite and > 0");
    }
    for (int f = 0; f < NF; ++f) {
        h->norm.mu[f] = (float)mu[f];
        h->norm.inv_sigma[f] = (float)(1.0 / sigma[f]);
        h->norm.tau[f] = tau[f];
        h->norm.inv_tau[f] = 1.0 / tau[f];
    }
    return GS_OK;
}

int gs_cnn_set_features(gs_cnn* h, int mode, double clip)
{
    if (!h) return cfail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (mode != 0 && mode != 1) return cfail(h, GS_ERR_ARG, "mode must be 0 or 1");
    if (!std::isfinite(clip) || clip < 0.0) return cfail(h, GS_ERR_ARG, "clip must be finite and >= 0");
    h->norm.mode = mode;
    h->norm.clip = clip;
    return GS_OK;
}

int gs_cnn_forward(gs_cnn* h, const void* U, float* y)
{
    if (!h) return cfail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (!U || !y || !aligned16(U) || !aligned16(y))
        return cfail(h, GS_ERR_ARG, "U or y is NULL or not 16-byte aligned");
    hipError_t e = forward(h, (const float*)U);
    if (e == hipSuccess)
        e = hipMemcpyAsync(y, h->y, (size_t)h->ncell * NF * 4, hipMemcpyDeviceToDevice, h->stream);
    return e == hipSuccess ? GS_OK : chip(h, e, "forward");
}

int gs_cnn_restrict(gs_cnn* h, const double* fine, void* U)
{
    if (!h) return cfail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (!fine || !U || !aligned16(fine) || !aligned16(U))
        return cfail(h, GS_ERR_ARG, "fine or U is NULL or not 16-byte aligned");
    hipLaunchKernelGGL(restrict_kernel, dim3(grid_for(h->ncell)), dim3(THREADS), 0, h->stream, fine,
                       h->nx, h->ny, h->nz, 0, (float*)U, (float*)nullptr, h->norm);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GS_OK : chip(h, e, "restrict");
}

int gs_cnn_make_target(gs_cnn* h, const double* fine, const void* U, float* target)
{
    if (!h) return cfail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (!fine || !U || !target || !aligned16(fine) || !aligned16(U) || !aligned16(target))
        return cfail(h, GS_ERR_ARG, "NULL or misaligned pointer");
    hipLaunchKernelGGL(restrict_kernel, dim3(grid_for(h->ncell)), dim3(THREADS), 0, h->stream, fine,
                       h->nx, h->ny, h->nz, 1, (float*)U, target, h->norm);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GS_OK : chip(h, e, "target");
}

int gs_cnn_gradients(gs_cnn* h, const void* U, const float* target, float* host_grads, double* loss)
{
    if (!h) return cfail(nullptr, GS_ERR_ARG, "handle is NULL");
    int r = check_train(h, U, target);
    if (r != GS_OK) return r;
    if (!host_grads || !loss) return cfail(h, GS_ERR_ARG, "output is NULL");
    hipError_t e = forward(h, (const float*)U);
    if (e == hipSuccess) e = backward(h, target);
    if (e != hipSuccess) return chip(h, e, "gradients");
    r = read_loss(h, loss);
    if (r != GS_OK) return r;
    e = hipMemcpy(host_grads, h->G, P_N * 4, hipMemcpyDeviceToHost);
    return e == hipSuccess ? GS_OK : chip(h, e, "gradient download");
}

int gs_cnn_train_step(gs_cnn* h, const void* U, const float* target, float lr, double* loss)
{
    if (!h) return cfail(nullptr, GS_ERR_ARG, "handle is NULL");
    int r = check_train(h, U, target);
    if (r != GS_OK) return r;
    if (!std::isfinite(lr) || !(lr > 0.0f)) return cfail(h, GS_ERR_ARG, "lr must be finite and > 0");
    hipError_t e = forward(h, (const float*)U);
    if (e == hipSuccess) e = backward(h, target);
    if (e != hipSuccess) return chip(h, e, "train step");
    if (loss) {
        r = read_loss(h, loss);
        if (r != GS_OK) return r;
    }
    h->step += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, h->step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, h->step)));
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(P_N)), dim3(THREADS), 0, h->stream, h->P, h->G,
                       h->M, h->V, P_N, lr, c1, c2);
    e = pack_all(h);
    return e == hipSuccess ? GS_OK : chip(h, e, "adam");
}

int gs_cnn_correct(gs_cnn* h, void* U)
{
    if (!h) return cfail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (!U || !aligned16(U)) return cfail(h, GS_ERR_ARG, "U is NULL or not 16-byte aligned");
    const long long n = h->ncell;
    // mode 0: the last convolution also sums its outputs per workgroup (no
    // separate pass over y)
    const int g3 = conv_grid<32, 1, EPI_F32_SOA>(conv_geom(h));
    const bool fused_mean = h->norm.mode == 0 && g3 <= 2 * RED_BLOCKS;
    MeanSums ms{};
    if (fused_mean) {
        ms.part = h->red;
        ms.clip = h->norm.clip;
    }
    hipError_t e = forward(h, (const float*)U, ms);
    if (e != hipSuccess) return chip(h, e, "correct: forward");
    gs::Phys k;
    k.gamma = h->gamma;
    k.gm1 = h->gamma - 1.0;
    k.inv_gm1 = 1.0 / (h->gamma - 1.0);
    for (int d = 0; d < 3; ++d) k.inv_h[d] = 1.0;
    k.cfl = 1.0;
    if (!fused_mean)
        hipLaunchKernelGGL(mean_partial_kernel, dim3(RED_BLOCKS), dim3(THREADS), 0, h->stream,
                           (const float*)U, h->y, n, h->norm, h->red);
    hipLaunchKernelGGL(mean_final_kernel, dim3(1), dim3(64 * NF), 0, h->stream, h->red,
                       fused_mean ? g3 : RED_BLOCKS, n, h->cs);
    hipLaunchKernelGGL(check_kernel, dim3(RED_BLOCKS), dim3(THREADS), 0, h->stream, (const float*)U,
                       h->y, n, h->norm, k, h->cs, h->red, h->cs);
    hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(64 * NF), 0, h->stream, h->red, RED_BLOCKS, h->cs);
    hipLaunchKernelGGL(commit_kernel, dim3(grid_for(n)), dim3(THREADS), 0, h->stream, (float*)U, h->y, n,
                       h->norm, h->cs);
    e = hipGetLastError();
    return e == hipSuccess ? GS_OK : chip(h, e, "correct");
}

int gs_cnn_counts(gs_cnn* h, int* applied, int* fallbacks)
{
    if (!h) return cfail(nullptr, GS_ERR_ARG, "handle is NULL");
    if (!applied || !fallbacks) return cfail(h, GS_ERR_ARG, "output is NULL");
    hipError_t e = hipMemcpyAsync(h->host_cs, h->cs, sizeof(CorrState), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return chip(h, e, "counts");
    *applied = h->host_cs->applied;
    *fallbacks = h->host_cs->fallbacks;
    return GS_OK;
}

int gs_cnn_set_stream(gs_cnn* h, void* stream)
{
    if (!h) return cfail(nullptr, GS_ERR_ARG, "handle is NULL");
    hipStream_t ns = (hipStream_t)stream;
    if (ns != h->stream) {
        // kernels queued on the old stream still use the handle's buffers:
        // the new stream waits for them before any later call
        hipEvent_t ev = nullptr;
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(ev, h->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(ns, ev, 0);
        if (ev) (void)hipEventDestroy(ev);
        if (e != hipSuccess)
            return cfail(h, GS_ERR_HIP, std::string("set_stream ordering: ") + hipGetErrorString(e));
    }
    h->stream = ns;
    return GS_OK;
}

void gs_cnn_destroy(gs_cnn* h)
{
    if (!h) return;
    void* ps[] = {h->P, h->G, h->M, h->V, h->wf1, h->wf2, h->wf3, h->wb2, h->wb3, h->x, h->h1,
                  h->h2, h->y, h->dY, h->dYv, h->dA2, h->dA2v, h->dA1, h->dA1v, h->xs, h->h1s,
                  h->h2s, h->wpart, h->bpart, h->red, h->cs};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    if (h->host_red) (void)hipHostFree(h->host_red);
    if (h->host_cs) (void)hipHostFree(h->host_cs);
    delete h;
}

const char* gs_cnn_last_error(const gs_cnn* h)
{
    return h ? h->err.c_str() : g_cnn_create_error.c_str();
}

}  // extern "C"
