// Device-wide exclusive scan and stable LSD radix sort (wave64, gfx950).
//
// Scan: tiles of 256 threads x 8 items; tile sums are scanned recursively.
// Radix sort: 8-bit digits; each wave owns a tile of 64 x RADIX_ITEMS consecutive
// items, counts its digits in LDS, and after a digit-major scan of the per-tile
// counts scatters its items in index order, ranking equal digits inside a group
// of 64 with eight ballots -- so every pass is stable.
#include "common.hpp"

namespace srw {

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int64_t SCAN_TILE = (int64_t)SCAN_BLOCK * SCAN_ITEMS;

// Block-wide exclusive scan of one int64 per thread; returns the block total.
__device__ int64_t block_exclusive(int64_t v, int64_t* out_excl, int64_t* lds_waves)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform (scalar)
    int64_t incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) lds_waves[wave] = incl;
    __syncthreads();
    int64_t wave_base = 0, total = 0;
    for (int w = 0; w < SCAN_BLOCK / 64; ++w) {
        if (w < wave) wave_base += lds_waves[w];
        total += lds_waves[w];
    }
    __syncthreads();
    *out_excl = wave_base + incl - v;
    return total;
}

template <typename In>
__global__ __launch_bounds__(SCAN_BLOCK) void scan_tile_sums(const In* in, int64_t n,
                                                             int64_t* sums)
{
    __shared__ int64_t lds[SCAN_BLOCK / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < n) s += (int64_t)in[base + i];
    int64_t excl;
    const int64_t total = block_exclusive(s, &excl, lds);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

template <typename In>
__global__ __launch_bounds__(SCAN_BLOCK) void scan_tile_apply(const In* in, int64_t* out,
                                                              int64_t n, const int64_t* offs)
{
    __shared__ int64_t lds[SCAN_BLOCK / 64];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = (base + i < n) ? (int64_t)in[base + i] : 0;
        s += v[i];
    }
    int64_t excl;
    block_exclusive(s, &excl, lds);
    int64_t run = excl + (offs ? offs[blockIdx.x] : 0);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
}

int64_t ntiles(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }

template <typename In>
hipError_t scan_impl(const In* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t t = ntiles(n);
    if (t == 1) {
        scan_tile_apply<In><<<1, SCAN_BLOCK, 0, s>>>(in, out, n, nullptr);
        return hipGetLastError();
    }
    int64_t* sums = tmp;
    int64_t* rest = tmp + t;
    scan_tile_sums<In><<<(unsigned)t, SCAN_BLOCK, 0, s>>>(in, n, sums);
    hipError_t e = scan_impl<int64_t>(sums, sums, t, rest, s);
    if (e != hipSuccess) return e;
    scan_tile_apply<In><<<(unsigned)t, SCAN_BLOCK, 0, s>>>(in, out, n, sums);
    return hipGetLastError();
}

}  // namespace

size_t scan_tmp_bytes(int64_t n)
{
    size_t total = 0;
    while (n > SCAN_TILE) {
        n = ntiles(n);
        total += (size_t)n;
    }
    return (total + 1) * sizeof(int64_t);
}

hipError_t exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, void* tmp, hipStream_t s)
{
    return scan_impl<int64_t>(in, out, n, (int64_t*)tmp, s);
}

hipError_t exclusive_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, void* tmp,
                                     hipStream_t s)
{
    return scan_impl<int32_t>(in, out, n, (int64_t*)tmp, s);
}

// ------------------------------------------------------------------- radix sort
namespace {

constexpr int RADIX_BLOCK = 256;  // 4 waves, each an independent tile
constexpr int RADIX_ITEMS = 32;
constexpr int64_t RADIX_TILE = 64 * RADIX_ITEMS;

template <typename K>
__global__ __launch_bounds__(RADIX_BLOCK) void radix_hist(const K* keys, int64_t n, int shift,
                                                          int64_t ntile, int32_t* hist)
{
    __shared__ int32_t cnt[RADIX_BLOCK / 64][256];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform (scalar)
    for (int d = lane; d < 256; d += 64) cnt[wave][d] = 0;
    __syncthreads();
    const int64_t tile = (int64_t)blockIdx.x * (RADIX_BLOCK / 64) + wave;
    if (tile < ntile) {
        const int64_t base = tile * RADIX_TILE;
        for (int j = 0; j < RADIX_ITEMS; ++j) {
            const int64_t i = base + (int64_t)j * 64 + lane;
            if (i < n) atomicAdd(&cnt[wave][(uint32_t)(keys[i] >> shift) & 255u], 1);
        }
    }
    __syncthreads();
    if (tile < ntile)
        for (int d = lane; d < 256; d += 64) hist[(int64_t)d * ntile + tile] = cnt[wave][d];
}

template <typename K>
__global__ __launch_bounds__(RADIX_BLOCK) void radix_scatter(const K* keys, const uint32_t* vals,
                                                             K* keys_out, uint32_t* vals_out,
                                                             int64_t n, int shift, int64_t ntile,
                                                             const int64_t* offs)
{
    __shared__ int64_t off[RADIX_BLOCK / 64][256];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform (scalar)
    const int64_t tile = (int64_t)blockIdx.x * (RADIX_BLOCK / 64) + wave;
    if (tile >= ntile) return;  // whole wave leaves; no block barrier below
    for (int d = lane; d < 256; d += 64) off[wave][d] = offs[(int64_t)d * ntile + tile];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const int64_t base = tile * RADIX_TILE;
    const uint64_t lt = lanemask_lt();
    for (int j = 0; j < RADIX_ITEMS; ++j) {
        const int64_t i = base + (int64_t)j * 64 + lane;
        const bool valid = i < n;
        K key = valid ? keys[i] : K(0);
        uint32_t val = valid ? vals[i] : 0u;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bb = ballot(((d >> b) & 1u) != 0);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        const int64_t rank = __popcll(peers & lt);
        int64_t dst = 0;
        if (valid) dst = off[wave][d] + rank;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // the highest lane of each peer group advances its digit's offset
        if (valid && (peers >> lane) == 1ull) off[wave][d] = dst + 1;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (valid) {
            keys_out[dst] = key;
            vals_out[dst] = val;
        }
    }
}

template <typename K>
hipError_t radix_impl(K* keys, uint32_t* vals, K* keys_alt, uint32_t* vals_alt, int64_t n,
                      int bits, void* tmp, K** keys_out, uint32_t** vals_out, hipStream_t s)
{
    *keys_out = keys;
    *vals_out = vals;
    if (n <= 1) return hipSuccess;
    const int64_t nt = (n + RADIX_TILE - 1) / RADIX_TILE;
    const int64_t nh = nt * 256;
    int32_t* hist = (int32_t*)tmp;
    int64_t* offs = (int64_t*)((char*)tmp + ((nh * sizeof(int32_t) + 255) & ~(size_t)255));
    void* scan_tmp = (char*)offs + ((nh * sizeof(int64_t) + 255) & ~(size_t)255);
    const unsigned grid = (unsigned)((nt + RADIX_BLOCK / 64 - 1) / (RADIX_BLOCK / 64));
    K *ka = keys, *kb = keys_alt;
    uint32_t *va = vals, *vb = vals_alt;
    for (int shift = 0; shift < bits; shift += 8) {
        radix_hist<K><<<grid, RADIX_BLOCK, 0, s>>>(ka, n, shift, nt, hist);
        hipError_t e = exclusive_scan_i32_to_i64(hist, offs, nh, scan_tmp, s);
        if (e != hipSuccess) return e;
        radix_scatter<K><<<grid, RADIX_BLOCK, 0, s>>>(ka, va, kb, vb, n, shift, nt, offs);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        K* tk = ka; ka = kb; kb = tk;
        uint32_t* tv = va; va = vb; vb = tv;
    }
    *keys_out = ka;
    *vals_out = va;
    return hipSuccess;
}

}  // namespace

size_t radix_tmp_bytes(int64_t n)
{
    const int64_t nt = (n + RADIX_TILE - 1) / RADIX_TILE;
    const int64_t nh = nt * 256;
    return ((nh * sizeof(int32_t) + 255) & ~(size_t)255) +
           ((nh * sizeof(int64_t) + 255) & ~(size_t)255) + scan_tmp_bytes(nh) + 256;
}

hipError_t radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                          int64_t n, int bits, void* tmp, uint64_t** keys_out,
                          uint32_t** vals_out, hipStream_t s)
{
    return radix_impl<uint64_t>(keys, vals, keys_alt, vals_alt, n, bits, tmp, keys_out, vals_out, s);
}

hipError_t radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                          int64_t n, int bits, void* tmp, uint32_t** keys_out,
                          uint32_t** vals_out, hipStream_t s)
{
    return radix_impl<uint32_t>(keys, vals, keys_alt, vals_alt, n, bits, tmp, keys_out, vals_out, s);
}

}  // namespace srw
