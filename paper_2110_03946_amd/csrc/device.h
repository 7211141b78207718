// Helpers shared by the HIP kernels of multilevel ORAS inpainting (gfx950,
// wave64): DPP lane shifts and fixed-order wave and workgroup sums, mask-bit
// selection, bfloat16 conversion, plane access through 32-bit byte offsets,
// the bilinear prolongation mix, the job lookup of batched launches, the
// column-walk geometry, and the host-side launch helpers. Everything here has
// internal linkage: each translation unit that includes it holds its own copy.
//
// All reductions run in a fixed order, so results are bitwise reproducible.
#pragma once

#include <algorithm>
#include <cstdint>

#include <hip/hip_ext.h>

#include "access.h"
#include "internal.h"

namespace ddi {
namespace {

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------

// GCN DPP controls: wave_shr:1 moves data one lane up (lane i receives lane
// i - 1), wave_shl:1 one lane down; row_shr:n shifts inside 16-lane rows.
// With bound_ctrl set, lanes whose source does not exist receive 0.
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, true));
}

// Value held by lane i - 1 (0 in lane 0).
__device__ __forceinline__ float from_left(float x) { return dpp<kDppWaveShr1>(x); }
// Value held by lane i + 1 (0 in lane 63).
__device__ __forceinline__ float from_right(float x) { return dpp<kDppWaveShl1>(x); }

__device__ __forceinline__ float readlane(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// Sum over the 64 lanes, returned uniformly (fixed order).
__device__ __forceinline__ float wave_sum(float x) {
    x += dpp<0x111>(x);  // row_shr:1
    x += dpp<0x112>(x);  // row_shr:2
    x += dpp<0x114>(x);  // row_shr:4
    x += dpp<0x118>(x);  // row_shr:8 -> lane 15 of each row holds the row sum
    return (readlane(x, 15) + readlane(x, 31)) + (readlane(x, 47) + readlane(x, 63));
}

__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// q where bit `bit` of `bits` is set, +0 elsewhere: a sign-extended bit
// field (v_bfe_i32) ANDed with q. Branch-free, and opaque enough that the
// compiler does not turn it into per-row lane masks held in scalar registers.
__device__ __forceinline__ float mask_keep(uint32_t bits, int bit, float q) {
    const int sel = __builtin_amdgcn_sbfe((int)bits, bit, 1);
    return __int_as_float(__float_as_int(q) & sel);
}

// bfloat16 storage of the correction equation: widen by a 16-bit shift,
// narrow with round-to-nearest-even (inputs are finite).
__device__ __forceinline__ float bf16_to_f(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }
__device__ __forceinline__ uint16_t f_to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// The same selection with the bit field extract written out: the compiler
// otherwise turns a one-bit v_bfe_i32 into and + compare + select (three
// instructions for two).
__device__ __forceinline__ float mask_bfe(uint32_t bits, int bit, float q) {
    int sel;
    asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(sel) : "v"(bits), "s"(bit));
    return __int_as_float(__float_as_int(q) & sel);
}

// Byte masks: byte k of a word is 0xff where row 4 j + k of the column is
// unknown (bit 4 j + k of the 32-bit mask word), 0 elsewhere.
__device__ __forceinline__ uint32_t mask_bytes(uint32_t bits, int j) {
    const uint32_t nib = (bits >> (4 * j)) & 0xfu;
    return ((nib * 0x00204081u) & 0x01010101u) * 0xffu;
}

// q where byte K of the byte mask m is 0xff, +0 where it is 0: one AND whose
// first operand is that byte sign-extended to 32 bits (an SDWA operand
// select), so a masked row costs one instruction instead of an extract and
// an AND.
template <int K>
__device__ __forceinline__ float mask_byte(uint32_t m, float q) {
    uint32_t out;
    asm("v_and_b32_sdwa %0, sext(%1), %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_%3 src1_sel:DWORD"
        : "=v"(out)
        : "v"(m), "v"(__float_as_uint(q)), "i"(K));
    return __uint_as_float(out);
}
// The same with the byte index as an argument; in unrolled loops it is a
// constant and the switch folds away.
__device__ __forceinline__ float mask_byte(uint32_t m, int k, float q) {
    switch (k & 3) {
        case 0: return mask_byte<0>(m, q);
        case 1: return mask_byte<1>(m, q);
        case 2: return mask_byte<2>(m, q);
        default: return mask_byte<3>(m, q);
    }
}

// Mask of one block column, built from the bits of the unknown pixels.
// Float storage (1 = unknown) for short columns; the bits themselves for
// 64-row columns, where registers are scarce.
template <int RPW, bool BITS>
struct ColMask;

template <int RPW>
struct ColMask<RPW, false> {
    float m[RPW];
    __device__ __forceinline__ void load(uint32_t lo, uint32_t hi) {
#pragma unroll
        for (int y = 0; y < RPW; ++y)
            m[y] = (((y < 32 ? lo : hi) >> (y & 31)) & 1u) ? 1.f : 0.f;
    }
    __device__ __forceinline__ float apply(int y, float q) const { return q * m[y]; }
    __device__ __forceinline__ void refresh() {}
};

template <int RPW>
struct ColMask<RPW, true> {
    uint32_t b[2];
    __device__ __forceinline__ void load(uint32_t lo, uint32_t hi) { b[0] = lo; b[1] = hi; }
    __device__ __forceinline__ float apply(int y, float q) const {
        return mask_keep(b[y >> 5], y & 31, q);
    }
    // Re-define the words once per CG step so that the 64 per-row bit
    // extracts stay inside the loop instead of occupying 64 registers.
    __device__ __forceinline__ void refresh() { asm volatile("" : "+v"(b[0]), "+v"(b[1])); }
};

// Element i of a plane through a 32-bit byte offset: a uniform base plus an
// unsigned 32-bit offset maps onto one global load with a scalar base
// (element offsets are below 2^30, so the byte offset fits).
template <class T>
__device__ __forceinline__ T at32(const T* base, uint32_t i) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ void put32(T* base, uint32_t i, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (uint32_t)sizeof(T)) = v;
}

// Bilinear prolongation (Sec. 4, read as cell-centred interpolation for the
// coarse-to-fine step): fine pixel y sits at coarse
// coordinate y/2 - 1/4, so along each axis it mixes the coarse sample y >> 1
// with weight 3/4 and that sample's neighbour on the fine pixel's side with
// weight 1/4, the neighbour index clamped to the coarse grid (where both
// weights fall on one sample, which the mix returns exactly). Columns first,
// then rows. Each mix is one rounding of the exact weighted sum of two
// float32 values: the 1/4 product is exact and the 3/4 one is fused.
__device__ __forceinline__ float pro_mix(float near, float far) {
    return __builtin_fmaf(0.75f, near, 0.25f * far);
}

// Index of the job whose workgroup range holds logical workgroup lb (jobs
// sorted by wg0, jobs[0].wg0 == 0).
template <class Job>
__device__ __forceinline__ int find_job(const Job* __restrict__ jobs, int njobs, int lb) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].wg0 <= lb) lo = mid; else hi = mid - 1;
    }
    return lo;
}

constexpr int kTpb = 256;

// Fixed-order block reduction of NV doubles per thread into out[0..NV):
// wave sums, then thread 0 adds the kTpb / 64 wave results in order.
template <int NV>
__device__ void block_reduce(double (&val)[NV], double* out) {
    __shared__ double sm[kTpb / 64][NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) val[j] = wave_sum_d(val[j]);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) sm[threadIdx.x >> 6][j] = val[j];
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < kTpb / 64; ++i) s += sm[i][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// Threads of the one-workgroup reductions (stop test, CG scalars).
constexpr int kDecideTpb = 1024;

// ---------------------------------------------------------------------------
// Column-walking stencil kernels. A workgroup is kWalkWaves waves side by
// side, each covering 64 consecutive columns of a band of kWalkRows rows;
// every lane walks down its column and keeps the rows above and below in
// registers, so each value is loaded once. Horizontal neighbours come from
// the neighbouring lanes (DPP); the columns just left and right of a wave
// come from one extra load per row in lanes 0 and 63. A missing neighbour
// at the image border takes the pixel's own value, so its difference is
// 0: the reflecting boundary. One float64 partial per workgroup and
// channel, in a fixed order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ Walk walk_geom(int h, int w) {
    return walk_at(h, w, blockIdx.x, blockIdx.y, threadIdx.x);
}

// Sum of acc over the workgroup into partial[wg][ch] (fixed order).
__device__ __forceinline__ void walk_partial(double acc, double* __restrict__ partial,
                                             int channels) {
    acc = wave_sum_d(acc);
    __shared__ double sm[kWalkWaves];
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < kWalkWaves; ++j) t += sm[j];
        partial[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * channels + blockIdx.z] = t;
    }
}

}  // namespace

// ---- host-side launch helpers ----

// A launch, or with timing events (ev0, ev1 non-null) a launch whose
// dispatch packet records the kernel's own start and end in them (no
// dispatch gap inside the bracket).
template <class K, class... Args>
static hipError_t launch_timed(K kernel, dim3 grid, dim3 block, hipStream_t s, hipEvent_t ev0,
                               hipEvent_t ev1, Args... args) {
    if (ev0 && ev1)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, ev0, ev1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
    return hipGetLastError();
}

static int grid1d(int64_t n) { return (int)((n + kTpb - 1) / kTpb); }

static bool aligned(const void* p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

static dim3 walk_grid(int h, int w, int channels) {
    return dim3(walk_groups_x(w), walk_groups_y(h), channels);
}

}  // namespace ddi
