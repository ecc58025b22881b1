// Shared device helpers and internal declarations of libsrw (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/srw.h"

#define SRW_WAVE 64
#ifndef SRW_CHUNK_WALKS
#define SRW_CHUNK_WALKS 256
#endif
// Walks of one row a wave takes from the walk queue at a time (the last chunk of a row
// may hold fewer): SRW_WAVE for the rows walked first (the lowest ranks, whose walks
// are the longest, so that they spread over many waves), CHUNK_WALKS for the others
// (fewer queue claims per wave).
constexpr uint32_t CHUNK_WALKS = SRW_CHUNK_WALKS;

// Status propagation for HIP runtime calls inside the C-ABI.
#define SRW_HIP(call)                                 \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return srw::hip_fail(e_, #call); \
    } while (0)

namespace srw {

// Records "what: <HIP error name>" as the calling thread's last error; returns
// SRW_E_NOMEM for allocation failures, SRW_E_HIP otherwise.
int hip_fail(hipError_t e, const char* what);
// Small pinned host block of this thread (32 int64), allocated on first use and kept
// until the process ends; nullptr if the allocation failed.  Slots: [0, 8) the build,
// [8, 12) the solvers, [16] the adaptive budget rounds.
int64_t* host_scratch();
void set_last_error(const char* msg);
// Ticks of the device's constant-rate wall clock (wall_clock64) in `seconds`, for the
// current device; the time limit of the triangular solves' waits.
int64_t wait_ticks(double seconds);
const char* get_last_error();

// Ground and step-limit markers in walk records / end-node lists.
constexpr uint32_t END_GROUND = 0xFFFFFFFFu;
constexpr uint32_t END_LIMIT = 0xFFFFFFFEu;

// walks_per_row of an internal build that runs no walks: every row keeps only its
// deterministic part (the IC(0) build lays out its pattern this way).
constexpr int32_t NO_WALKS = -1;

// |e_k| <= EXCESS_EPS * A_kk is zero excess (no path to ground).
constexpr double EXCESS_EPS = 1e-12;

// Flags packed into the high bits of a node descriptor's degree word.
constexpr uint32_t DESC_GROUNDED = 0x80000000u;
constexpr uint32_t DESC_DEG_MASK = 0x00FFFFFFu;

// ---------------------------------------------------------------- Philox4x64-10
// Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11): ten rounds of
// two 64x64->128-bit products with the Weyl key schedule.
struct u64x4 {
    uint64_t x0, x1, x2, x3;
};

__device__ __forceinline__ u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return {c0, c1, c2, c3};
}

constexpr uint64_t STREAM_WALK = 0;
constexpr uint64_t STREAM_ORDER = 1;

// ------------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const int l = __lane_id();
    return l ? (~0ull >> (64 - l)) : 0ull;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Lane 0's value as a wave-uniform (scalar) value.  v_readlane reads the lane whatever
// the execution mask, and the scalar result lets the compiler keep every branch on
// it uniform -- a broadcast through a shuffle would not, and the structurizer may then
// place the shuffle where lane 0's register no longer holds the value.
__device__ __forceinline__ uint64_t lane0_u64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 0);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 0);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t readfirstlane(uint32_t v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ uint64_t readfirstlane64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// floor((c / d) * 2^32) clamped to [0, 2^32 - 1]; the scale is exact, only the
// division rounds (IEEE, correctly rounded).
__device__ __forceinline__ uint32_t threshold32(double c, double d)
{
    const double x = (c / d) * 4294967296.0;
    if (x >= 4294967295.0) return 0xFFFFFFFFu;
    if (x <= 0.0) return 0u;
    return (uint32_t)x;
}

// ------------------------------------------------------------- device algorithms
// (implemented in scan_sort.hip)
// Exclusive prefix sum of n int64 values (in may alias out).  tmp: scan_tmp_bytes(n).
size_t scan_tmp_bytes(int64_t n);
hipError_t exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, void* tmp,
                              hipStream_t s);
// Same over int32 inputs widened to int64 outputs.
hipError_t exclusive_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, void* tmp,
                                     hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the keys.
// Buffers: keys/vals in, keys_alt/vals_alt scratch of the same size; the sorted
// result ends up in the buffers returned through *keys_out / *vals_out.
size_t radix_tmp_bytes(int64_t n);
hipError_t radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                          int64_t n, int bits, void* tmp, uint64_t** keys_out,
                          uint32_t** vals_out, hipStream_t s);
hipError_t radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                          int64_t n, int bits, void* tmp, uint32_t** keys_out,
                          uint32_t** vals_out, hipStream_t s);

inline int grid_for(int64_t n, int block)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 0x7FFFFFFF) g = 0x7FFFFFFF;
    return (int)g;
}

}  // namespace srw
