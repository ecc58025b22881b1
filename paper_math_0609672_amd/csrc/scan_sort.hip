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

// block_exclusive for the radix sort's block (same size as the scan's)
__device__ int64_t block_exclusive_radix(int64_t v, int64_t* out_excl, int64_t* lds_waves)
{
    return block_exclusive(v, out_excl, lds_waves);
}

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

constexpr int RADIX_BLOCK = 256;  // one tile of RADIX_ITEMS items per thread
constexpr int RADIX_ITEMS = 16;
constexpr int64_t RADIX_TILE = (int64_t)RADIX_BLOCK * RADIX_ITEMS;

// Digit counts of each tile; item j*256 + t of the tile is thread t's j-th item.
template <typename K>
__global__ __launch_bounds__(RADIX_BLOCK) void radix_hist(const K* keys, int64_t n, int shift,
                                                          int64_t ntile, int32_t* hist)
{
    __shared__ int32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * RADIX_TILE;
#pragma unroll
    for (int j = 0; j < RADIX_ITEMS; ++j) {
        const int64_t i = base + (int64_t)j * RADIX_BLOCK + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(uint32_t)(keys[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntile + tile] = cnt[threadIdx.x];
}

// One tile per block: every item's rank among the tile's items of its digit (index
// order: j, then thread), then the tile sorted by digit in LDS, then written out in
// LDS order, so each digit's items of the tile leave as one contiguous run.  Stable.
template <typename K>
__global__ __launch_bounds__(RADIX_BLOCK) void radix_scatter(const K* keys, const uint32_t* vals,
                                                             K* keys_out, uint32_t* vals_out,
                                                             int64_t n, int shift, int64_t ntile,
                                                             const int64_t* offs)
{
    __shared__ K skey[RADIX_TILE];
    __shared__ uint32_t sval[RADIX_TILE];
    __shared__ int64_t goff[256];              // the tile's first output index per digit
    __shared__ int32_t run[256];               // items of the digit placed so far
    __shared__ int32_t wcnt[RADIX_BLOCK / 64][256];
    __shared__ int64_t lds_waves[RADIX_BLOCK / 64];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * RADIX_TILE;
    goff[t] = offs[(int64_t)t * ntile + tile];
    run[t] = 0;
#pragma unroll
    for (int w = 0; w < RADIX_BLOCK / 64; ++w) wcnt[w][t] = 0;
    K key[RADIX_ITEMS];
    uint32_t val[RADIX_ITEMS];
    int32_t pos[RADIX_ITEMS];
#pragma unroll
    for (int j = 0; j < RADIX_ITEMS; ++j) {
        const int64_t i = base + (int64_t)j * RADIX_BLOCK + t;
        key[j] = i < n ? keys[i] : K(0);
        val[j] = i < n ? vals[i] : 0u;
    }
    __syncthreads();
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int j = 0; j < RADIX_ITEMS; ++j) {
        const bool valid = base + (int64_t)j * RADIX_BLOCK + t < n;
        const uint32_t d = (uint32_t)(key[j] >> shift) & 255u;
        uint64_t peers = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bb = ballot(((d >> b) & 1u) != 0);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        // the highest lane of each group of equal digits records the group's size
        if (valid && (peers >> lane) == 1ull) wcnt[wave][d] = __popcll(peers);
        __syncthreads();
        int32_t before = run[d];
        for (int w = 0; w < wave; ++w) before += wcnt[w][d];
        pos[j] = valid ? before + (int32_t)__popcll(peers & lt) : -1;
        __syncthreads();
        int32_t add = 0;
#pragma unroll
        for (int w = 0; w < RADIX_BLOCK / 64; ++w) {
            add += wcnt[w][t];
            wcnt[w][t] = 0;
        }
        run[t] += add;
        __syncthreads();
    }
    // tile-local start of each digit
    int64_t start;
    const int64_t count = block_exclusive_radix(run[t], &start, lds_waves);
    (void)count;
    __syncthreads();
    run[t] = (int32_t)start;  // reused: the digit's first LDS position
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RADIX_ITEMS; ++j) {
        if (pos[j] >= 0) {
            const uint32_t d = (uint32_t)(key[j] >> shift) & 255u;
            const int p = run[d] + pos[j];
            skey[p] = key[j];
            sval[p] = val[j];
        }
    }
    __syncthreads();
    const int64_t m = n - base < RADIX_TILE ? n - base : RADIX_TILE;
    for (int p = t; p < m; p += RADIX_BLOCK) {
        const K k = skey[p];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        const int64_t dst = goff[d] + (p - run[d]);
        keys_out[dst] = k;
        vals_out[dst] = sval[p];
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
    const unsigned grid = (unsigned)nt;  // one tile per block
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
