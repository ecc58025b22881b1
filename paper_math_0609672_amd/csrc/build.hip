// Preconditioning phase of the hybrid solver (Algorithm 1, "Precondition") on gfx950.
//
//   validate      R-matrix check (Section 1) and a path to ground in every connected
//                 component (Section 2.1), one thread per row + union-find hooking
//   rank          random ordering (Section 5.4): Philox keys, stable radix sort
//   table         the walk game of Section 2.1 as 32-bit cumulative thresholds
//   walk          one lane = one walk; lanes take new walks from a chunk queue as
//                 theirs end; homes = lower rank or ground (Section 2.2.1); first
//                 step among higher-ranked neighbours (Section 5.2)
//   tally         one wave per row: LDS bitonic sort + run-length of end nodes
//                 (H'_{k,i}), wave sums of stays (J'_k) -- no global atomics
//   factor        eqs. newy, newz, d and the drop (Sections 3.3, 4, 5.2), FP64
//   plan          Y^T by a stable radix sort of the entries on (column, source rank);
//                 the rows of Y and Y^T relabelled by solve slot (rank or level order)
#include <algorithm>
#include <cstdio>
#include <cmath>
#include <cstring>

#include "factor.hpp"

namespace srw {

namespace {

constexpr int BLOCK = 256;

enum : int { ERR_ARG = 1, ERR_NOT_R = 2, ERR_SINGULAR = 4, ERR_LIMIT = 8, ERR_STACK = 16, ERR_WAIT = 32 };

// ------------------------------------------------------------------- validation
__global__ void k_check_structure(int64_t n, int64_t nnz, const int64_t* __restrict__ rowptr,
                                  const int32_t* __restrict__ col, int* err)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0 && (rowptr[0] != 0 || rowptr[n] != nnz)) atomicOr(err, ERR_ARG);
    if (k >= n) return;
    const int64_t r0 = rowptr[k], r1 = rowptr[k + 1];
    if (r0 < 0 || r1 < r0 || r1 > nnz || r1 - r0 - 1 > (int64_t)DESC_DEG_MASK) {
        atomicOr(err, ERR_ARG);
        return;
    }
    int ndiag = 0;
    int32_t prev = -1;
    for (int64_t p = r0; p < r1; ++p) {
        const int32_t j = col[p];
        if (j < 0 || j >= n || j <= prev) {
            atomicOr(err, ERR_ARG);
            return;
        }
        prev = j;
        ndiag += (j == k);
    }
    if (ndiag != 1) atomicOr(err, ERR_ARG);
}

// Needs a valid structure.  diag[k] = A_kk, grounded[k] = (e_k > eps a_k) with the
// excess summed in CSR order.
// values: positive diagonal, negative off-diagonal entries, row dominance; the
// mirrored entry must exist, with the same value unless `sym_values` is 0 (the game
// of an asymmetric A, Section 7.1)
__global__ void k_check_values(int64_t n, const int64_t* __restrict__ rowptr,
                               const int32_t* __restrict__ col, const double* __restrict__ val,
                               int sym_values, uint8_t* __restrict__ grounded, int* err)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t r0 = rowptr[k], r1 = rowptr[k + 1];
    double a = 0.0;
    for (int64_t p = r0; p < r1; ++p)
        if (col[p] == k) a = val[p];
    int bad = 0;
    if (!(a > 0.0)) bad = 1;
    double sum_w = 0.0;
    for (int64_t p = r0; p < r1 && !bad; ++p) {
        const int32_t j = col[p];
        if (j == k) continue;
        const double v = val[p];
        if (!(v < 0.0)) {
            bad = 1;
            break;
        }
        sum_w = sum_w + (-v);
        int64_t lo = rowptr[j], hi = rowptr[j + 1] - 1, found = -1;
        while (lo <= hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            const int32_t c = col[mid];
            if (c == (int32_t)k) {
                found = mid;
                break;
            }
            if (c < (int32_t)k) lo = mid + 1;
            else hi = mid - 1;
        }
        if (found < 0 || (sym_values && val[found] != v)) bad = 1;
    }
    if (!bad) {
        const double e = a - sum_w;
        if (e < -EXCESS_EPS * a) bad = 1;
        grounded[k] = (e > EXCESS_EPS * a) ? 1 : 0;
    } else {
        grounded[k] = 0;
    }
    if (bad) atomicOr(err, ERR_NOT_R);
}

// Plain loads: a label read here may be older than one another thread has just set
// (labels only decrease and label[x] <= x holds at every moment, so the walk up still
// ends at a root).  A stale root can only hook a node that is no longer a root, which
// at worst splits a tree along an edge the next pass hooks again; the loop ends after
// a pass in which no thread hooked, and in that pass nothing changed, so every thread
// read the settled labels.
__device__ __forceinline__ int32_t cc_root(const int32_t* label, int32_t x)
{
    for (;;) {
        const int32_t y = label[x];
        if (y == x) return x;
        x = y;
    }
}

__global__ void k_cc_init(int64_t n, int32_t* label)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) label[v] = (int32_t)v;
}

// Hooks the larger of two different roots under the smaller; labels only decrease,
// so the forest stays acyclic and find terminates.
__global__ void k_cc_hook(int64_t n, const int64_t* __restrict__ rowptr,
                          const int32_t* __restrict__ col, int32_t* label, int* changed)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int any = 0;
    int32_t ru = -1;
    for (int64_t p = rowptr[u]; p < rowptr[u + 1]; ++p) {
        const int32_t v = col[p];
        if (v <= u) continue;  // each undirected edge once
        if (ru < 0) ru = cc_root(label, (int32_t)u);
        const int32_t rv = cc_root(label, v);
        if (ru != rv) {
            atomicMin(&label[ru > rv ? ru : rv], ru < rv ? ru : rv);
            ru = ru < rv ? ru : rv;  // u's tree now hangs below the smaller root
            any = 1;
        }
    }
    if (any) atomicOr(changed, 1);
}

__global__ void k_cc_compress(int64_t n, int32_t* label)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) label[v] = cc_root(label, (int32_t)v);
}

__global__ void k_cc_ground(int64_t n, const int32_t* __restrict__ label,
                            const uint8_t* __restrict__ grounded, uint8_t* comp)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n && grounded[v]) comp[label[v]] = 1;
}

__global__ void k_cc_check(int64_t n, const int32_t* __restrict__ label,
                           const uint8_t* __restrict__ comp, int* err)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n && label[v] == (int32_t)v && !comp[v]) atomicOr(err, ERR_SINGULAR);
}

// -------------------------------------------------------------------- ordering
__global__ void k_rank_keys(int64_t n, uint64_t seed, uint64_t* keys, uint32_t* vals)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const u64x4 b = philox4x64_10(0, 0, (uint64_t)v, STREAM_ORDER, seed, 0);
    keys[v] = b.x0;
    vals[v] = (uint32_t)v;
}

__global__ void k_rank_scatter(int64_t n, const uint32_t* __restrict__ sorted, int32_t* rank,
                               int32_t* by_rank)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t v = sorted[p];
    by_rank[p] = (int32_t)v;
    rank[v] = (int32_t)p;
}

// natural ordering: rank = node id
__global__ void k_rank_natural(int64_t n, int32_t* rank, int32_t* by_rank)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    rank[v] = (int32_t)v;
    by_rank[v] = (int32_t)v;
}

__global__ void k_rank_given(int64_t n, const int32_t* __restrict__ given, int32_t* rank,
                             int32_t* by_rank, int32_t* seen, int* err)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t r = given[v];
    if (r < 0 || r >= n || atomicAdd(&seen[r], 1) != 0) {
        atomicOr(err, ERR_ARG);
        return;
    }
    rank[v] = r;
    by_rank[r] = (int32_t)v;
}

// ------------------------------------------------------------- walk schedule
// Work is cut into chunks of up to 64 walks of one row.  Chunks come in NSEG
// segments: segment 0 holds the rows ranked below `long_rank` (their walks meet few
// homes and run longest) in rank order, so they start first; segments 1..8 split the
// remaining rows by node id into eight slabs, one per XCD, so the walks in flight on
// one XCD share a compact part of the graph and of that XCD's L2.
constexpr int NSLAB = 8;
constexpr uint32_t REUSE_STACK = 64;  // walk reuse: stack entries per lane
// Default waves per CU of the walk kernel.  A walk step is one dependent record load,
// so the longest walks run at the memory latency the other walks cause: on a 3D grid
// (128^3, 256 walks per row) 8 waves per CU finish the walks in 165 ms, 12 in 179 ms
// (an earlier build: 8 in 175 ms, 24 in 205 ms, 4 in 283 ms).
constexpr int WALK_WAVES_PER_CU = 8;
constexpr int NSEG = NSLAB + 1;

__global__ void k_flag_long(int64_t n, int64_t long_rank, const int32_t* __restrict__ by_rank,
                            const int32_t* __restrict__ budget, int32_t* flag)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < long_rank) flag[p] = budget[by_rank[p]] > 0 ? 1 : 0;
}

__global__ void k_flag_slab(int64_t n, int64_t long_rank, const int32_t* __restrict__ rank,
                            const int32_t* __restrict__ budget, int32_t* flag)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) flag[v] = (budget[v] > 0 && rank[v] >= long_rank) ? 1 : 0;
}

// order[pos] = row, chunks[pos] = its number of chunks of cs walks
__global__ void k_compact(int64_t count, const int32_t* __restrict__ rows_or_null,
                          const int32_t* __restrict__ flag, const int64_t* __restrict__ pos,
                          int64_t base, const int32_t* __restrict__ budget, int32_t* order,
                          int32_t* chunks, int32_t cs)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count || !flag[i]) return;
    const int32_t v = rows_or_null ? rows_or_null[i] : (int32_t)i;
    order[base + pos[i]] = v;
    chunks[base + pos[i]] = (budget[v] + cs - 1) / cs;
}

// flag[i] = 1 for the rows whose budget lies in (lo, hi]
__global__ void k_budget_class(int64_t n, const int32_t* __restrict__ budget, int32_t lo,
                               int32_t hi, int32_t* __restrict__ flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = budget[i] > lo && budget[i] <= hi;
}

// the flagged rows, in row order, at their exclusive-scan positions
__global__ void k_scatter_rows(int64_t n, const int32_t* __restrict__ flag,
                               const int64_t* __restrict__ pos, int32_t* __restrict__ rows)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) rows[pos[i]] = (int32_t)i;
}

__global__ void k_read_last(const int64_t* scan, const int32_t* last_in, int64_t n, int64_t* out)
{
    out[0] = n > 0 ? scan[n - 1] + (int64_t)last_in[n - 1] : 0;
}

// bounds[0..NSEG]: first chunk of each segment (bounds[NSEG] = all chunks)
__global__ void k_seg_bounds(int64_t n, int64_t nlong, int64_t nslab_rows,
                             const int64_t* __restrict__ pos_slab,
                             const int64_t* __restrict__ chunk_off, int64_t* bounds)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    bounds[0] = 0;
    for (int x = 0; x < NSLAB; ++x) {
        const int64_t node = (int64_t)x * n / NSLAB;
        const int64_t opos = nlong + (node < n ? pos_slab[node] : nslab_rows);
        bounds[1 + x] = chunk_off[opos];
    }
    bounds[NSEG] = chunk_off[nlong + nslab_rows];
}

// ----------------------------------------------------------------------- walks
#include "walk.hpp"

// ----------------------------------------------------------- stopping rule
// Section 5.1: the first M >= min_walks whose walk lengths (walks 0 .. M-1 of the
// row, in walk order) satisfy delta * mean * sqrt(M) / sigma > z (sigma the sample
// standard deviation; sigma = 0 passes); 0 if none of the row's walks does, -1 for a
// row without walks.  One wave per row: exact integer prefix sums of the lengths and
// their squares, the test in float64 in the oracle's operation order.
__global__ __launch_bounds__(64) void k_length_rule(int64_t n, const int32_t* __restrict__ budget,
                                                    const int64_t* __restrict__ rec_off,
                                                    const uint32_t* __restrict__ rec_len,
                                                    double delta, double z, int32_t min_walks,
                                                    int32_t* __restrict__ found)
{
    const int lane = threadIdx.x;
    for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
    const int32_t m = budget[k];
    if (m == 0) {
        if (lane == 0) found[k] = -1;
        continue;
    }
    const int64_t base = rec_off[k];
    uint64_t s1 = 0, s2 = 0;  // sums over the walks before this chunk
    int32_t hit = 0;
    for (int32_t c0 = 0; c0 < m && hit == 0; c0 += 64) {
        const int32_t w = c0 + lane;
        const uint64_t len = w < m ? (uint64_t)rec_len[base + w] : 0;
        uint64_t p1 = len, p2 = len * len;  // inclusive prefix sums within the chunk
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint64_t a = __shfl_up(p1, off, 64), b = __shfl_up(p2, off, 64);
            if (lane >= off) {
                p1 += a;
                p2 += b;
            }
        }
        bool ok = false;
        const int32_t M = w + 1;
        if (w < m && M >= min_walks) {
            const uint64_t S1 = s1 + p1, S2 = s2 + p2;
            const double mean = (double)S1 / (double)M;
            const double var = ((double)S2 - (double)M * mean * mean) / (double)(M - 1);
            ok = !(var > 0.0) || delta * mean * sqrt((double)M) / sqrt(var) > z;
        }
        const uint64_t mask = ballot(ok);
        if (mask) hit = c0 + __ffsll((long long)mask);  // lowest satisfying walk count
        s1 += __shfl(p1, 63, 64);
        s2 += __shfl(p2, 63, 64);
    }
    if (lane == 0) found[k] = hit;
    }
}

// --------------------------------------------------------------------- tallies
// One wave per row, rows in a grid-stride loop over `rows` (all rows when null).  LDS:
// P sort keys + P run heads, P a power of two >= every listed row's budget; a row sorts
// only the smallest power of two (at least 64) that holds its own walks.  Launched with
// one workgroup per row: on a 3D grid (2.1M rows, 256 walks each) that takes 6.8 ms, a
// chip-sized grid looping over rows 8.5 ms.
__global__ __launch_bounds__(64) void k_tally(int64_t n, const int32_t* __restrict__ rows,
                                              const int32_t* __restrict__ budget,
                                              const int64_t* __restrict__ rec_off,
                                              const uint32_t* rec_end,
                                              const uint32_t* rec_vis,
                                              const uint32_t* __restrict__ rec_len, int P,
                                              uint64_t* __restrict__ J, uint32_t* __restrict__ G,
                                              uint64_t* __restrict__ steps,
                                              uint64_t* __restrict__ vsq,
                                              int32_t* __restrict__ hlen, uint32_t* h_end,
                                              uint32_t* h_cnt)
{
    extern __shared__ uint32_t lds[];
    uint32_t* key = lds;
    uint32_t* head = lds + P;
    const int lane = threadIdx.x;
    for (int64_t kk = blockIdx.x; kk < n; kk += gridDim.x) {
    const int64_t k = rows ? rows[kk] : kk;
    const int m = budget[k];
    if (m > P) continue;  // not this launch's row (the caller checks that none is left)
    if (m == 0) {  // exact row: no walks
        if (lane == 0) {
            J[k] = 0;
            G[k] = 0;
            steps[k] = 0;
            vsq[k] = 0;
            hlen[k] = 0;
        }
        continue;
    }
    const int64_t base = rec_off[k];
    int Pk = 64;
    while (Pk < m) Pk <<= 1;
    uint64_t jv = 0, sl = 0, vq = 0;
    uint32_t g = 0;
    for (int i = lane; i < Pk; i += 64) {
        uint32_t e = END_GROUND;
        if (i < m) {
            e = rec_end[base + i];
            const uint64_t v = rec_vis[base + i];
            jv += v;
            vq += v * v;
            sl += rec_len[base + i];
            g += (e == END_GROUND);
        }
        key[i] = e;
    }
    jv = wave_sum(jv);
    vq = wave_sum(vq);
    sl = wave_sum(sl);
    g = wave_sum(g);
    __syncthreads();
    // bitonic sort, ascending (ground markers sort last)
    for (int size = 2; size <= Pk; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = lane; i < (Pk >> 1); i += 64) {
                // stride is a power of two: pair i's lower index without a division
                const int lo = ((i & ~(stride - 1)) << 1) | (i & (stride - 1));
                const int hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const uint32_t x = key[lo], y = key[hi];
                if ((x > y) == asc) {
                    key[lo] = y;
                    key[hi] = x;
                }
            }
            __syncthreads();
        }
    }
    // run heads over the m - g walks that ended at a node
    const int nb = m - (int)g;
    const uint64_t lt = lanemask_lt();
    int run = 0;
    for (int i0 = 0; i0 < nb; i0 += 64) {
        const int i = i0 + lane;
        const bool h = i < nb && (i == 0 || key[i] != key[i - 1]);
        const uint64_t mask = ballot(h);
        if (h) head[run + __popcll(mask & lt)] = (uint32_t)i;
        run += __popcll(mask);
    }
    __syncthreads();
    for (int j = lane; j < run; j += 64) {
        h_end[base + j] = key[head[j]];
        h_cnt[base + j] = (j + 1 < run ? head[j + 1] : (uint32_t)nb) - head[j];
    }
    if (lane == 0) {
        J[k] = jv;
        G[k] = g;
        steps[k] = sl;
        vsq[k] = vq;
        hlen[k] = run;
    }
    __syncthreads();  // the next row reuses the LDS
    }
}

// The same tallies for budgets up to 2048 walks, without sorting every end node: the
// ends go into an LDS hash table (linear probing, counts by atomic add) of twice the
// smallest power of two >= the row's budget slots, at least 128; the distinct ends
// (about C/N of them) are compacted in slot order and only those are sorted, as
// (node << 32 | count).  The H list is then the same as k_tally's.  One workgroup per
// entry of `rows` (per row when null); rows whose budget exceeds P are left to another
// launch.  LDS: 2P keys + 2P counts (u32) + P pairs (u64).
__global__ __launch_bounds__(64) void k_tally_hash(int64_t n, const int32_t* __restrict__ rows,
                                                   const int32_t* __restrict__ budget,
                                                   const int64_t* __restrict__ rec_off,
                                                   const uint32_t* rec_end,
                                                   const uint32_t* rec_vis,
                                                   const uint32_t* __restrict__ rec_len, int P,
                                                   uint64_t* __restrict__ J,
                                                   uint32_t* __restrict__ G,
                                                   uint64_t* __restrict__ steps,
                                                   uint64_t* __restrict__ vsq,
                                                   int32_t* __restrict__ hlen, uint32_t* h_end,
                                                   uint32_t* h_cnt)
{
    extern __shared__ __align__(16) uint64_t lds64[];
    uint64_t* cp = lds64;                      // [P] compacted (node << 32 | count)
    uint32_t* tk = (uint32_t*)(lds64 + P);     // [2P] keys, END_GROUND = empty
    uint32_t* tc = tk + 2 * P;                 // [2P] counts
    if ((int64_t)blockIdx.x >= n) return;
    const int64_t k = rows ? rows[blockIdx.x] : blockIdx.x;
    const int m = budget[k];
    const int64_t base = rec_off[k];
    // both scalar loads leave before the branch on m (one round trip, not two)
    asm volatile("" ::"s"(base));
    const int lane = threadIdx.x;
    if (m > P) return;  // not this launch's row (the caller checks that none is left)
    int HS = 128;  // table slots, a power of two >= 2m
    while (HS < 2 * m) HS <<= 1;
    if (m == 0) {  // exact row: no walks
        if (lane == 0) {
            J[k] = 0;
            G[k] = 0;
            steps[k] = 0;
            vsq[k] = 0;
            hlen[k] = 0;
        }
        return;
    }
    int hbits = 0;
    while ((1 << hbits) < HS) ++hbits;
    // the row's first 256 walks are loaded before the table is cleared, in one round
    // trip rather than one per 64 walks
    constexpr int U = 4;
    uint32_t re[U], rv[U], rl[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t q = base + min(u * 64 + lane, m - 1);  // in the row; unused past m
        re[u] = rec_end[q];
        rv[u] = rec_vis[q];
        rl[u] = rec_len[q];
    }
    __shared__ uint32_t used[64];  // the first 64 slots taken, in the order taken
    __shared__ int nused;
    for (int i = lane; i < HS / 4; i += 64) {  // HS >= 128: whole 16-byte groups
        ((uint4*)tk)[i] = make_uint4(END_GROUND, END_GROUND, END_GROUND, END_GROUND);
        ((uint4*)tc)[i] = make_uint4(0u, 0u, 0u, 0u);
    }
    if (lane == 0) nused = 0;
    __syncthreads();
    uint64_t jv = 0, sl = 0, vq = 0;
    uint32_t g = 0;
    for (int i0 = 0; i0 < m; i0 += U * 64) {
        if (i0 > 0) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t q = base + min(i0 + u * 64 + lane, m - 1);
                re[u] = rec_end[q];
                rv[u] = rec_vis[q];
                rl[u] = rec_len[q];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (i0 + u * 64 + lane >= m) continue;
            const uint32_t e = re[u];
            const uint64_t v = rv[u];
            jv += v;
            vq += v * v;
            sl += rl[u];
            if (e == END_GROUND) {
                ++g;
                continue;
            }
            uint32_t h = (e * 0x9E3779B1u) >> (32 - hbits);
            for (;;) {  // at most m of the HS >= 2m slots are taken: an empty one is reached
                const uint32_t prev = atomicCAS(&tk[h], END_GROUND, e);
                if (prev == END_GROUND) {
                    const int at = atomicAdd(&nused, 1);
                    if (at < 64) used[at] = h;
                }
                if (prev == END_GROUND || prev == e) {
                    atomicAdd(&tc[h], 1u);
                    break;
                }
                h = (h + 1) & (uint32_t)(HS - 1);
            }
        }
    }
    jv = wave_sum(jv);
    vq = wave_sum(vq);
    sl = wave_sum(sl);
    g = wave_sum(g);
    __syncthreads();
    const int DU = nused;  // distinct ends
    if (DU <= 64) {
        // at most one distinct end per lane: its place in ascending order is the number
        // of smaller ends (the ends are distinct), counted over the lanes
        const uint32_t h = lane < DU ? used[lane] : 0u;
        const uint32_t key = lane < DU ? tk[h] : END_GROUND;
        const uint32_t cnt = lane < DU ? tc[h] : 0u;
        int below = 0;
        for (int j = 0; j < DU; ++j)  // j is wave-uniform: lane reads, no LDS
            below += (uint32_t)__builtin_amdgcn_readlane((int)key, j) < key;
        if (lane < DU) {
            h_end[base + below] = key;
            h_cnt[base + below] = cnt;
        }
        if (lane == 0) {
            J[k] = jv;
            G[k] = g;
            steps[k] = sl;
            vsq[k] = vq;
            hlen[k] = DU;
        }
        return;
    }
    const uint64_t lt = lanemask_lt();
    int D = 0;
    for (int i0 = 0; i0 < HS; i0 += 64) {
        const int i = i0 + lane;
        const uint32_t key = tk[i];
        const bool ok = key != END_GROUND;
        const uint64_t mask = ballot(ok);
        if (ok) cp[D + __popcll(mask & lt)] = ((uint64_t)key << 32) | tc[i];
        D += __popcll(mask);
    }
    int D2 = 1;
    while (D2 < D) D2 <<= 1;
    for (int i = D + lane; i < D2; i += 64) cp[i] = ~0ull;
    __syncthreads();
    // bitonic sort of the D2 pairs, ascending
    for (int size = 2; size <= D2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = lane; i < (D2 >> 1); i += 64) {
                const int lo = ((i & ~(stride - 1)) << 1) | (i & (stride - 1));
                const int hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const uint64_t x = cp[lo], y = cp[hi];
                if ((x > y) == asc) {
                    cp[lo] = y;
                    cp[hi] = x;
                }
            }
            __syncthreads();
        }
    }
    for (int j = lane; j < D; j += 64) {
        const uint64_t x = cp[j];
        h_end[base + j] = (uint32_t)(x >> 32);
        h_cnt[base + j] = (uint32_t)x;
    }
    if (lane == 0) {
        J[k] = jv;
        G[k] = g;
        steps[k] = sl;
        vsq[k] = vq;
        hlen[k] = D;
    }
}

// ------------------------------------------------------- tallies, walk reuse
// With walk reuse every counted walk is a record {start node << 32 | end node, stays,
// steps}; the records are sorted by key, so a row's records are contiguous with
// ascending end node (ground last).
__global__ void k_iota_u32(int64_t n, uint32_t* x)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = (uint32_t)i;
}

// beg[k] = first of the m sorted keys whose bits from `shift` up are >= k (k = 0..n;
// beg[n] = m when every key is below n << shift), by binary search
__global__ void k_row_begin(int64_t n, const uint64_t* __restrict__ key, int64_t m,
                            int64_t* __restrict__ beg, int shift = 32, uint64_t mask = ~0ull)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > n) return;
    const uint64_t want = (uint64_t)k << shift;
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if ((key[mid] & mask) < want) lo = mid + 1;
        else hi = mid;
    }
    beg[k] = lo;
}

__global__ void k_row_count(int64_t n, const int64_t* __restrict__ beg, int32_t* __restrict__ cnt)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) cnt[k] = (int32_t)(beg[k + 1] - beg[k]);
}

// One wave per row (grid-stride over rows) over its sorted records: the sums of k_tally and the H list
// (distinct end nodes, ascending, with counts) written from beg[k] on.  A run of equal
// end nodes starts at a head; the count of a run is the distance from its head to
// the next head (or to the first ground record).
__global__ __launch_bounds__(64) void k_tally_sorted(
    int64_t n, const int64_t* __restrict__ beg, const uint64_t* __restrict__ key,
    const uint32_t* __restrict__ idx, const uint2* __restrict__ vl, uint64_t* __restrict__ J,
    uint32_t* __restrict__ G, uint64_t* __restrict__ steps, uint64_t* __restrict__ vsq,
    int32_t* __restrict__ hlen, uint32_t* __restrict__ h_end, uint32_t* __restrict__ h_cnt)
{
    const int lane = threadIdx.x;
    const uint64_t lt = lanemask_lt();
    for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
    const int64_t b = beg[k], e = beg[k + 1];
    uint64_t jv = 0, sl = 0, vq = 0;
    uint32_t g = 0;
    int run = 0;             // runs so far
    int last_head = -1;      // offset of the last head so far
    uint32_t prev_end = 0;   // end node of the record before this chunk
    for (int64_t i0 = b; i0 < e; i0 += 64) {
        const int64_t i = i0 + lane;
        const bool in = i < e;
        uint32_t en = END_GROUND;
        if (in) {
            en = (uint32_t)key[i];
            const uint2 x = vl[idx[i]];
            jv += x.x;
            vq += (uint64_t)x.x * x.x;
            sl += x.y;
            g += (en == END_GROUND);
        }
        uint32_t pe = (uint32_t)__shfl_up((int)en, 1);
        if (lane == 0) pe = prev_end;
        const bool head = in && en != END_GROUND && (i == b || en != pe);
        const uint64_t mask = ballot(head);
        // offset of the nearest head at or below each lane (inclusive running max)
        int hv = head ? (int)(i - b) : -1;
        for (int d = 1; d < 64; d <<= 1) {
            const int o = __shfl_up(hv, d);
            if (lane >= d) hv = max(hv, o);
        }
        int below = __shfl_up(hv, 1);
        if (lane == 0) below = -1;
        below = max(below, last_head);
        if (head) {
            const int r = run + (int)__popcll(mask & lt);
            h_end[b + r] = en;
            if (r > 0) h_cnt[b + r - 1] = (uint32_t)((int)(i - b) - below);
        }
        run += (int)__popcll(mask);
        last_head = max(last_head, __shfl(hv, 63));
        prev_end = (uint32_t)__shfl((int)en, 63);
    }
    jv = wave_sum(jv);
    vq = wave_sum(vq);
    sl = wave_sum(sl);
    g = wave_sum(g);
    if (lane == 0) {
        const int nb = (int)(e - b) - (int)g;
        if (run > 0) h_cnt[b + run - 1] = (uint32_t)(nb - last_head);
        J[k] = jv;
        G[k] = g;
        steps[k] = sl;
        vsq[k] = vq;
        hlen[k] = run;
    }
    }
}

// ---------------------------------------------------------------------- factor
// Row k: merge of the lower-ranked neighbours (CSR order) and the end nodes of
// its walks (ascending), evaluated in FP64 exactly as written, no contraction:
//   Y_ki = -((w_ki / a) + (tau * (H / M))),  D_k = a / (1 + tau * ((J / M) - 1)).
template <typename T, bool FILL>
__global__ void k_factor(int64_t n, const int64_t* __restrict__ rowptr,
                         const int32_t* __restrict__ col, const double* __restrict__ val,
                         const int32_t* __restrict__ rank, const double* __restrict__ tau,
                         const int32_t* __restrict__ budget, const uint64_t* __restrict__ J,
                         const int64_t* __restrict__ h_off, const int32_t* __restrict__ hlen,
                         const uint32_t* __restrict__ h_end, const uint32_t* __restrict__ h_cnt,
                         double drop_tol, int32_t plain, int32_t* __restrict__ ynnz,
                         const int64_t* __restrict__ yptr, int32_t* __restrict__ ycol,
                         T* __restrict__ yval, T* __restrict__ dout)
{
#pragma clang fp contract(off)
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t r0 = rowptr[k], r1 = rowptr[k + 1];
    const int32_t rk = rank[k];
    double a = 0.0;
    for (int64_t p = r0; p < r1; ++p)
        if (col[p] == k) a = val[p];
    const double tk = tau[k];
    const uint32_t M = (uint32_t)budget[k];
    const int32_t H = M ? hlen[k] : 0;
    const int64_t hb = M ? h_off[k] : 0;
    int64_t p = r0;
    int32_t h = 0;
    int64_t kept = 0;
    const int64_t out0 = FILL ? yptr[k] : 0;
    if (plain) {
        // eq. yzdetail: Y_ki = -H'_ki / M' for every end node i; eq. d: D = M' a / J'
        for (; h < H; ++h) {
            const double y = -((double)h_cnt[hb + h] / (double)M);
            if (!(fabs(y) < drop_tol)) {
                if (FILL) {
                    ycol[out0 + kept] = (int32_t)h_end[hb + h];
                    yval[out0 + kept] = (T)y;
                }
                ++kept;
            }
        }
        if (FILL) dout[k] = (T)(((double)M * a) / (double)J[k]);
        if (ynnz) ynnz[k] = (int32_t)kept;
        return;
    }
    for (;;) {
        while (p < r1 && (col[p] == k || rank[col[p]] > rk)) ++p;
        const uint32_t ci = p < r1 ? (uint32_t)col[p] : 0xFFFFFFFFu;
        const uint32_t ch = h < H ? h_end[hb + h] : 0xFFFFFFFFu;
        if (ci == 0xFFFFFFFFu && ch == 0xFFFFFFFFu) break;
        const uint32_t i = ci < ch ? ci : ch;
        double w = 0.0;
        uint32_t cnt = 0;
        if (ci == i) {
            w = -val[p];
            ++p;
        }
        if (ch == i) {
            cnt = h_cnt[hb + h];
            ++h;
        }
        const double hfrac = M > 0 ? (double)cnt / (double)M : 0.0;
        const double y = -((w / a) + (tk * hfrac));
        if (!(fabs(y) < drop_tol)) {
            if (FILL) {
                ycol[out0 + kept] = (int32_t)i;
                yval[out0 + kept] = (T)y;
            }
            ++kept;
        }
    }
    if (FILL) {
        double dk = a;
        if (M > 0) {
            const double mbar = (double)J[k] / (double)M;
            dk = a / (1.0 + tk * (mbar - 1.0));
        }
        dout[k] = (T)dk;
    }
    if (ynnz) ynnz[k] = (int32_t)kept;
}

// Room for row k of Y before the drop: its neighbours other than itself (the
// lower-ranked ones are a subset) plus the distinct end nodes of its walks.
__global__ void k_factor_caps(int64_t n, const int64_t* __restrict__ rowptr,
                              const int32_t* __restrict__ budget, const int32_t* __restrict__ hlen,
                              int32_t* __restrict__ cap)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    cap[k] = (int32_t)(rowptr[k + 1] - rowptr[k] - 1) + (budget[k] ? hlen[k] : 0);
}

// The rows written at their padded offsets, packed into the factor's CSR; sixteen
// lanes per row.
template <typename T>
__global__ void k_pack_rows(int64_t n, const int64_t* __restrict__ pad_off,
                            const int64_t* __restrict__ yptr, const int32_t* __restrict__ ynnz,
                            const int32_t* __restrict__ pcol, const T* __restrict__ pval,
                            int32_t* __restrict__ ycol, T* __restrict__ yval)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = t >> 4;
    if (k >= n) return;
    const int64_t a = pad_off[k], b = yptr[k];
    for (int32_t j = (int32_t)(t & 15); j < ynnz[k]; j += 16) {
        ycol[b + j] = pcol[a + j];
        yval[b + j] = pval[a + j];
    }
}

// ------------------------------------------------------------------- transpose
// Entries of Y for the rows of Y^T, listed row by row in descending rank of the source
// row k, with key (position of k in that list) << 32 | column i.  A stable sort on the
// column alone then orders each row of Y^T by the rank of k descending -- the order in
// which the backward substitution finishes the w_k it needs, so a long Y^T row meets
// its last-ready values at its end.
// lens[r] = length of the row of rank n-1-r.
__global__ void k_desc_lens(int64_t n, const int32_t* __restrict__ by_rank,
                            const int64_t* __restrict__ yptr, int32_t* __restrict__ lens)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int32_t k = by_rank[n - 1 - r];
    lens[r] = (int32_t)(yptr[k + 1] - yptr[k]);
}

// Sixteen lanes per row (rows of Y hold about twenty entries), entries strided by 16.
// The column field is the column's node, or its rank when col_rank is given (the rows
// of Y^T then come out in rank order, the solve slots of a rank-ordered plan).
__global__ void k_entry_keys(int64_t n, const int32_t* __restrict__ by_rank,
                             const int64_t* __restrict__ yptr, const int32_t* __restrict__ ycol,
                             const int32_t* __restrict__ col_rank,
                             const int64_t* __restrict__ doff, uint32_t* idx, uint64_t* key)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = t >> 4;
    if (r >= n) return;
    const int32_t k = by_rank[n - 1 - r];
    const int64_t b = yptr[k], e = yptr[k + 1], o = doff[r] - b;
    for (int64_t q = b + (t & 15); q < e; q += 16) {
        idx[o + q] = (uint32_t)q;
        const int32_t c = col_rank ? col_rank[ycol[q]] : ycol[q];
        key[o + q] = ((uint64_t)r << 32) | (uint32_t)c;
    }
}

// The source row of a sorted entry comes back from its key's position field through
// the rank-ordered node list (a small, cached table) rather than a gather by entry.
template <typename T>
__global__ void k_transpose_fill(int64_t nnz, int64_t n, const uint64_t* __restrict__ sorted_key,
                                 const uint32_t* __restrict__ sorted_idx,
                                 const int32_t* __restrict__ by_rank, const T* __restrict__ yval,
                                 int32_t* __restrict__ ytcol, T* __restrict__ ytval)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nnz) return;
    const int64_t r = (int64_t)(sorted_key[j] >> 32);
    ytcol[j] = by_rank[n - 1 - r];
    ytval[j] = yval[sorted_idx[j]];
}

// The same for a rank-ordered plan, sorted on the column's rank: the entries land in
// the rows of Y^T by slot, the source row's slot (its rank) being n - 1 minus the
// key's position field.
template <typename T>
__global__ void k_transpose_fill_slots(int64_t nnz, int64_t n,
                                       const uint64_t* __restrict__ sorted_key,
                                       const uint32_t* __restrict__ sorted_idx,
                                       const T* __restrict__ yval, int32_t* __restrict__ bcol,
                                       T* __restrict__ bval)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nnz) return;
    bcol[j] = (int32_t)(n - 1 - (int64_t)(sorted_key[j] >> 32));
    bval[j] = yval[sorted_idx[j]];
}

__global__ void k_set_last(int64_t* ptr, int64_t n, int64_t v) { ptr[n] = v; }

// ------------------------------------------------------------------- solve plan
__global__ void k_copy_i32(int64_t n, const int32_t* __restrict__ a, int32_t* __restrict__ b)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ void k_invert(int64_t n, const int32_t* __restrict__ slot_node, int32_t* node_slot)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) node_slot[slot_node[s]] = (int32_t)s;
}

__global__ void k_slot_lens(int64_t n, const int32_t* __restrict__ slot_node,
                            const int64_t* __restrict__ ptr, int32_t* __restrict__ lens)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) {
        const int32_t k = slot_node[s];
        lens[s] = (int32_t)(ptr[k + 1] - ptr[k]);
    }
}

// Row of node slot_node[s] copied to slot s, entries in their order, columns as slots;
// one wave per slot.
template <typename T>
__global__ void k_permute_rows(int64_t n, const int32_t* __restrict__ slot_node,
                               const int32_t* __restrict__ node_slot,
                               const int64_t* __restrict__ sptr, const int32_t* __restrict__ scol,
                               const T* __restrict__ sval, const int64_t* __restrict__ dptr,
                               int32_t* __restrict__ dcol, T* __restrict__ dval)
{
    // sixteen lanes per slot (rows hold about twenty entries), one slot per group
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t s = t >> 4;
    if (s >= n) return;
    const int32_t k = slot_node[s];
    const int64_t a = sptr[k], len = sptr[k + 1] - a, o = dptr[s];
    for (int64_t j = t & 15; j < len; j += 16) {
        dcol[o + j] = node_slot[scol[a + j]];
        dval[o + j] = sval[a + j];
    }
}

template <typename T>
__global__ void k_gather_slots(int64_t n, const int32_t* __restrict__ slot_node,
                               const T* __restrict__ src, T* __restrict__ dst)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) dst[s] = src[slot_node[s]];
}

// The largest head h <= hmax (h = hmax or a multiple of 64) with h * fptr[h] <= cost:
// fptr, the rank-ordered plan's row starts, grows with h, and so does the product.
__global__ void k_head_bound(const int64_t* __restrict__ fptr, int64_t hmax, int64_t cost,
                             int64_t* out)
{
    if (hmax * fptr[hmax] <= cost) {
        *out = hmax;
        return;
    }
    int64_t lo = 0, hi = hmax / 64;  // in units of 64 rows: lo fits, hi does not
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (64 * mid * fptr[64 * mid] <= cost) lo = mid;
        else hi = mid;
    }
    *out = 64 * lo;
}

// (level, node) pairs of a rank-ordered plan, listed by slot, so a stable sort on the
// level keeps rank order inside each level.  The first h slots (the dense head) take
// key 0 and the others level + 1: the head stays first, in rank order.
__global__ void k_level_keys(int64_t n, int64_t h, const int32_t* __restrict__ slot_node,
                             const int32_t* __restrict__ lev, uint32_t* key, uint32_t* val)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    key[s] = s < h ? 0u : (uint32_t)lev[s] + 1u;
    val[s] = (uint32_t)slot_node[s];
}

// ptr[k] = the first position of the sorted keys (head 0, level + 1 past it) holding
// a key >= k, for k = 0 .. kmax + 1; every key up to kmax occurs
__global__ void k_key_ptr(int64_t n, const uint32_t* __restrict__ key, uint32_t kmax,
                          int64_t* __restrict__ ptr)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const uint32_t lo = i == 0 ? 0u : key[i - 1] + 1u;
    const uint32_t hi = i == n ? kmax + 1u : min(key[i], kmax + 1u);
    for (uint32_t k = lo; k <= hi; ++k) ptr[k] = i;
}

__global__ void k_sum_u64(int64_t n, const uint64_t* __restrict__ x, unsigned long long* out)
{
    uint64_t s = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        s += x[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(out, (unsigned long long)s);
}

// Grid of the one-wave-per-row kernels that loop over rows: 32 single-wave workgroups
// per CU, at least one and at most one per row.
unsigned row_grid(int64_t n)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        cus = 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)cus * 32));
}

// ------------------------------------------------------------------------ IC(0)
// Zero fill-in incomplete Cholesky, the ICCG preconditioner the paper compares with
// (Section 6, Tables 1-2), in the factor's form A ~ Y^T D Y: nodes are eliminated in
// decreasing rank and every update outside A's pattern is discarded, so row k of Y
// keeps exactly its lower-ranked neighbours (the pattern the build has laid out):
//   D_k  = A_kk - sum_{j in Up(k)} (D_j Y_jk) Y_jk
//   Y_ki = (A_ki - sum_{j in Up(k), j ~ i} (D_j Y_jk) Y_ji) / D_k
// Up(k) = the higher-ranked neighbours of k, in the CSR order of row k.
// One lane per row.  A wave claims the next 64 positions of the decreasing-rank order
// (one atomic per claim) and its lanes wait for their rows' higher-ranked neighbours:
// D of a row is published last (release), filled beforehand with a signalling-NaN
// pattern, and is the row's ready flag.  Claims are handed out in order, so the
// highest-ranked unfinished row always belongs to a running wave and has all its
// dependencies done: the factorization progresses whatever the grid's residency.
constexpr unsigned long long IC0_PENDING = 0x7FF4DEADBEEF5A5Aull;

__global__ void k_fill_u64(int64_t n, unsigned long long* x, unsigned long long v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

__device__ __forceinline__ double ic0_entry(const int64_t* __restrict__ yptr,
                                            const int32_t* __restrict__ ycol, const double* yval,
                                            int64_t j, int32_t c)
{
    for (int64_t q = yptr[j]; q < yptr[j + 1]; ++q)
        if (ycol[q] == c) return yval[q];
    return 0.0;
}

__global__ __launch_bounds__(BLOCK) void k_ic0(int64_t n, const int64_t* __restrict__ rowptr,
                                               const int32_t* __restrict__ col,
                                               const double* __restrict__ val,
                                               const int32_t* __restrict__ rank,
                                               const int32_t* __restrict__ by_rank,
                                               const int64_t* __restrict__ yptr,
                                               const int32_t* __restrict__ ycol, double* yval,
                                               double* d, unsigned long long* claim, int* err,
                                               int64_t ticks)
{
    const int lane = threadIdx.x & 63;
    unsigned long long* dbits = (unsigned long long*)d;
    for (;;) {
        const uint64_t base = lane0_u64(atomicAdd(claim, lane == 0 ? 64ull : 0ull));
        if (base >= (uint64_t)n) break;
        const int64_t pos = (int64_t)base + lane;
        bool done = pos >= n;
        const int32_t k = done ? 0 : by_rank[n - 1 - pos];
        const int64_t r0 = done ? 0 : rowptr[k], r1 = done ? 0 : rowptr[k + 1];
        const int32_t rk = done ? 0 : rank[k];
        const int64_t t0 = wall_clock64();
        uint32_t spins = 0;
        while (ballot(!done) != 0) {
            if (!done) {
                bool ready = true;
                for (int64_t p = r0; p < r1 && ready; ++p) {
                    const int32_t j = col[p];
                    if (j != k && rank[j] > rk)
                        ready = __hip_atomic_load(dbits + j, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT) != IC0_PENDING;
                }
                if (ready) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    double a = 0.0;
                    for (int64_t p = r0; p < r1; ++p)
                        if (col[p] == k) a = val[p];
                    double dk = a;
                    for (int64_t p = r0; p < r1; ++p) {
                        const int32_t j = col[p];
                        if (j == k || rank[j] < rk) continue;
                        const double yjk = ic0_entry(yptr, ycol, yval, j, k);
                        dk = dk - (d[j] * yjk) * yjk;
                    }
                    if (!(dk > 0.0)) atomicOr(err, ERR_NOT_R);
                    int64_t q = yptr[k];
                    for (int64_t p = r0; p < r1; ++p) {
                        const int32_t i = col[p];
                        if (i == k || rank[i] > rk) continue;
                        double sv = val[p];
                        for (int64_t p2 = r0; p2 < r1; ++p2) {
                            const int32_t j = col[p2];
                            if (j == k || rank[j] < rk) continue;
                            const double yji = ic0_entry(yptr, ycol, yval, j, i);
                            if (yji == 0.0) continue;
                            const double yjk = ic0_entry(yptr, ycol, yval, j, k);
                            sv = sv - (d[j] * yjk) * yji;
                        }
                        yval[q++] = sv / dk;
                    }
                    __hip_atomic_store(dbits + k, __builtin_bit_cast(unsigned long long, dk),
                                       __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    done = true;
                }
            }
            // a guard against a defect: give up after the time limit (the rows left
            // publish a quiet NaN so that the other waves drain)
            if ((++spins & 255u) == 0 && wall_clock64() - t0 > ticks) {
                if (!done) {
                    atomicOr(err, ERR_WAIT);
                    __hip_atomic_store(dbits + k, 0x7FF8000000000000ull, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    done = true;
                }
            }
        }
    }
}

int map_err(int e)
{
    if (e & ERR_ARG) return SRW_E_ARG;
    if (e & ERR_NOT_R) return SRW_E_NOT_RMATRIX;
    if (e & ERR_SINGULAR) return SRW_E_SINGULAR;
    if (e & ERR_LIMIT) return SRW_E_WALK_LIMIT;
    if (e & ERR_STACK) {
        set_last_error("walk reuse: a walk's stack of open walks grew past its capacity");
        return SRW_E_WALK_LIMIT;
    }
    if (e & ERR_WAIT) {
        set_last_error("IC(0): a row gave up waiting for a higher-ranked row");
        return SRW_E_HIP;
    }
    return SRW_OK;
}

}  // namespace

namespace {
thread_local char last_error[256] = "";
}

int64_t* host_scratch()
{
    thread_local int64_t* p = nullptr;
    if (!p && hipHostMalloc((void**)&p, 32 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess)
        p = nullptr;
    return p;
}

void set_last_error(const char* msg)
{
    std::snprintf(last_error, sizeof(last_error), "%s", msg ? msg : "");
}

const char* get_last_error() { return last_error; }

__global__ void k_rule_round(int64_t n, const int32_t* __restrict__ found, int32_t* __restrict__ target,
                             int32_t* __restrict__ walks, int32_t max_walks, int* __restrict__ open)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || walks[k] >= 0) return;  // decided before this round
    const int32_t f = found[k];
    if (f < 0) walks[k] = 0;                       // exact row: no walks
    else if (f > 0) walks[k] = f;                  // the rule is met after f walks
    else if (target[k] >= max_walks) walks[k] = max_walks;
    else {
        target[k] = min(2 * target[k], max_walks);
        atomicAdd(open, 1);
    }
}

__global__ void k_rule_budgets(int64_t n, const int32_t* __restrict__ walks,
                               const int32_t* __restrict__ target, int32_t* __restrict__ budget)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) budget[k] = walks[k] >= 0 ? 1 : target[k];  // decided rows: one cheap walk
}

__global__ void k_fill_i32v(int64_t n, int32_t* x, int32_t v)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) x[k] = v;
}

int adaptive_impl(const srw_csr* A, uint64_t seed, const srw_options* opt_in, double delta,
                  double z, int32_t min_walks, int32_t max_walks, int32_t* walks, hipStream_t s)
{
    const int64_t n = A->n;
    if (n == 0) return SRW_OK;
    int32_t *target = nullptr, *budget = nullptr, *found = nullptr;
    int* open = nullptr;
    int* host_open = nullptr;
    hipError_t e = hipMallocAsync((void**)&target, 3 * n * sizeof(int32_t) + 256, s);
    if (e != hipSuccess) return hip_fail(e, "adaptive budgets: workspace");
    budget = target + n;
    found = budget + n;
    open = (int*)(found + n);
    host_open = (int*)(host_scratch() ? host_scratch() + 16 : nullptr);
    if (!host_open) e = hipErrorOutOfMemory;
    const int g = grid_for(n, BLOCK);
    int status = SRW_OK;
    if (e == hipSuccess) {
        k_fill_i32v<<<g, BLOCK, 0, s>>>(n, target, min_walks);
        k_fill_i32v<<<g, BLOCK, 0, s>>>(n, walks, -1);
        e = hipGetLastError();
    }
    srw_options opt = *opt_in;
    opt.walks = budget;
    opt.keep = 0;
    opt.profile = 0;
    opt.reuse = 0;
    while (e == hipSuccess && status == SRW_OK) {
        k_rule_budgets<<<g, BLOCK, 0, s>>>(n, walks, target, budget);
        LengthRule rule{delta, z, min_walks, found};
        srw_factor* none = nullptr;
        status = build_factor_impl(A, 1, 0.0, seed, &opt, &none, s, nullptr, &rule);
        if (status != SRW_OK) break;
        k_fill_i32v<<<1, 1, 0, s>>>(1, (int32_t*)open, 0);
        k_rule_round<<<g, BLOCK, 0, s>>>(n, found, target, walks, max_walks, open);
        e = hipMemcpyAsync(host_open, open, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess || *host_open == 0) break;
    }
    (void)hipFreeAsync(target, s);
    (void)hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "adaptive budgets");
    return status;
}

void retain_pool_memory()
{
    static bool done[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64 || done[dev]) return;
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess && pool) {
        uint64_t keep_all = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep_all);
    }
    done[dev] = true;
}

int hip_fail(hipError_t e, const char* what)
{
    std::snprintf(last_error, sizeof(last_error), "%s: %s", what ? what : "HIP call",
                  hipGetErrorName(e));
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SRW_E_NOMEM;
    return SRW_E_HIP;
}

void free_factor(srw_factor* F)
{
    if (!F) return;
    free_factor(F->tgame);
    for (void* p : F->allocations) (void)hipFree(p);
    if (!F->pool_allocations.empty()) {
        // back to the pool once the device is idle (the caller guarantees no work on F
        // is pending; the synchronization is what hipFree would have done)
        (void)hipDeviceSynchronize();
        for (void* p : F->pool_allocations) (void)hipFreeAsync(p, nullptr);
        (void)hipStreamSynchronize(nullptr);
    }
    if (F->host_scalars) (void)hipHostFree(F->host_scalars);
    delete F;
}

// Random ordering alone (Section 5.4): rank of every node, as the build computes it.
int ordering_impl(int64_t n, uint64_t seed, int32_t* rank, hipStream_t s)
{
    if (n <= 0) return SRW_OK;
    const size_t nn = (size_t)n;
    auto align = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t bytes = 2 * align(nn * sizeof(uint64_t)) + 3 * align(nn * sizeof(uint32_t)) +
                         radix_tmp_bytes(n);
    char* ws = nullptr;
    SRW_HIP(hipMallocAsync((void**)&ws, bytes, s));
    char* p = ws;
    uint64_t* keys = (uint64_t*)p; p += align(nn * sizeof(uint64_t));
    uint64_t* keys2 = (uint64_t*)p; p += align(nn * sizeof(uint64_t));
    uint32_t* vals = (uint32_t*)p; p += align(nn * sizeof(uint32_t));
    uint32_t* vals2 = (uint32_t*)p; p += align(nn * sizeof(uint32_t));
    int32_t* by_rank = (int32_t*)p; p += align(nn * sizeof(int32_t));
    void* rt = p;
    const int g = grid_for(n, BLOCK);
    k_rank_keys<<<g, BLOCK, 0, s>>>(n, seed, keys, vals);
    uint64_t* ko;
    uint32_t* vo;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = radix_sort_u64(keys, vals, keys2, vals2, n, 64, rt, &ko, &vo, s);
    if (e == hipSuccess) {
        k_rank_scatter<<<g, BLOCK, 0, s>>>(n, vo, rank, by_rank);
        e = hipGetLastError();
    }
    (void)hipFreeAsync(ws, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    SRW_HIP(e);
    return SRW_OK;
}

int build_factor_impl(const srw_csr* A, int32_t walks_per_row, double drop_tol, uint64_t seed,
                      const srw_options* opt_in, srw_factor** out, hipStream_t s,
                      const BatchKeys* batch, const LengthRule* rule, bool asym, bool ic0)
{
    srw_options opt;
    srw_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (opt.max_steps == 0) opt.max_steps = 1ull << 22;
    if (opt.refill_period == 0) opt.refill_period = 8;
    // walk reuse: one instance of the walk kernel (refill period 8); its records
    // replace the per-walk records, which it cannot export; not for batches or
    // walks-only builds
    const bool reuse = opt.reuse != 0;
    if (reuse && (opt.refill_period != 8 || opt.keep >= 2 || batch || rule)) return SRW_E_ARG;
    // IC(0): no walks and no drop; the walk build lays out the pattern (every row's
    // lower-ranked neighbours), then k_ic0 fills in the values, FP64 only
    if (ic0) {
        if (reuse || batch || rule || asym || opt.factor_precision != SRW_FP64) return SRW_E_ARG;
        walks_per_row = NO_WALKS;
        drop_tol = 0.0;
        opt.one_step_exact = 1;
    }
    // the plain estimator of eqs. yzdetail and d: every row walks from its own record
    const bool plain = opt.one_step_exact == 0;
    if (plain && (reuse || batch || rule || asym)) return SRW_E_ARG;
    const int64_t n = A->n, nnz = A->nnz;
    const int64_t nnz_off = nnz - n;

    srw_factor* F = new srw_factor();
    F->reuse = reuse ? 1 : 0;
    F->n = n;
    F->nnz_a = nnz;
    F->precision = opt.factor_precision;
    F->keep = opt.keep;
    Arena keep;  // blocks that end up owned by F
    Arena tmp;   // build temporaries, from the stream-ordered pool
    retain_pool_memory();
    tmp.pooled = true;
    tmp.stream = s;
    keep.pooled = true;  // the factor's blocks too: repeated builds reuse pooled memory
    keep.stream = s;
    // shared chunks sized to the matrix: a few n-length arrays each
    keep.chunk = std::max<size_t>((size_t)1 << 20, ((size_t)std::max<int64_t>(n, 1) * 32 + 255) & ~(size_t)255);
    tmp.chunk = 4 * keep.chunk;
    // arrays only exports need: owned by F with keep >= 1, build temporaries otherwise
    Arena& xk = opt.keep >= 1 ? keep : tmp;
    int64_t* pinned = nullptr;
    int status = SRW_OK;
    const bool fp32 = opt.factor_precision == SRW_FP32;
    const size_t vbytes = fp32 ? sizeof(float) : sizeof(double);

#define FAIL(code)           \
    do {                     \
        status = (code);     \
        goto done;           \
    } while (0)
#define CHECK_HIP(call)                                  \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) FAIL(hip_fail(e_, #call)); \
    } while (0)
#define ALLOC(arena, T, cnt) (arena).alloc<T>(cnt)

    hipEvent_t ev[SRW_NUM_PHASES + 1] = {};
    const bool prof = opt.profile != 0;
    auto mark = [&](int i) {
        if (prof) (void)hipEventRecord(ev[i], s);
    };
    if (prof)
        for (auto& e : ev)
            if (hipEventCreate(&e) != hipSuccess) e = nullptr;
    {
        pinned = host_scratch();
        if (!pinned) FAIL(SRW_E_NOMEM);
        const int g = grid_for(n, BLOCK);
        int* err = ALLOC(tmp, int, 1);
        int* changed = ALLOC(tmp, int, 1);
        uint8_t* grounded = ALLOC(xk, uint8_t, n);
        int32_t* label = ALLOC(tmp, int32_t, n);
        uint8_t* comp = ALLOC(tmp, uint8_t, n);
        F->rank = ALLOC(keep, int32_t, n);
        F->by_rank = ALLOC(keep, int32_t, n);
        F->yptr = ALLOC(keep, int64_t, n + 1);
        if (!err || !changed || !grounded || !label || !comp || !F->rank || !F->by_rank ||
            !F->yptr)
            FAIL(SRW_E_NOMEM);
        F->grounded = grounded;

        // ---- 1. validation
        mark(0);
        CHECK_HIP(hipMemsetAsync(err, 0, sizeof(int), s));
        k_check_structure<<<g, BLOCK, 0, s>>>(n, nnz, A->rowptr, A->col, err);
        CHECK_HIP(hipGetLastError());
        int herr = 0;
        CHECK_HIP(hipMemcpyAsync(&pinned[0], err, sizeof(int), hipMemcpyDeviceToHost, s));
        CHECK_HIP(hipStreamSynchronize(s));
        std::memcpy(&herr, &pinned[0], sizeof(int));
        if (herr) FAIL(map_err(herr));
        if (nnz_off >= (int64_t)0xFFFFFFFFll) FAIL(SRW_E_ARG);
        k_check_values<<<g, BLOCK, 0, s>>>(n, A->rowptr, A->col, A->val, asym ? 0 : 1, grounded,
                                           err);
        k_cc_init<<<g, BLOCK, 0, s>>>(n, label);
        for (int it = 0; it < 64 * 64; ++it) {
            CHECK_HIP(hipMemsetAsync(changed, 0, sizeof(int), s));
            k_cc_hook<<<g, BLOCK, 0, s>>>(n, A->rowptr, A->col, label, changed);
            k_cc_compress<<<g, BLOCK, 0, s>>>(n, label);
            CHECK_HIP(hipMemcpyAsync(&pinned[1], changed, sizeof(int), hipMemcpyDeviceToHost, s));
            CHECK_HIP(hipStreamSynchronize(s));
            int ch = 0;
            std::memcpy(&ch, &pinned[1], sizeof(int));
            if (!ch) break;
        }
        CHECK_HIP(hipMemsetAsync(comp, 0, n, s));
        k_cc_ground<<<g, BLOCK, 0, s>>>(n, label, grounded, comp);
        k_cc_check<<<g, BLOCK, 0, s>>>(n, label, comp, err);
        CHECK_HIP(hipGetLastError());

        // ---- 2. ordering
        mark(1);
        if (opt.ordering == SRW_ORDER_GIVEN) {
            if (!opt.rank) FAIL(SRW_E_ARG);
            int32_t* seen = ALLOC(tmp, int32_t, n);
            if (!seen) FAIL(SRW_E_NOMEM);
            CHECK_HIP(hipMemsetAsync(seen, 0, n * sizeof(int32_t), s));
            k_rank_given<<<g, BLOCK, 0, s>>>(n, opt.rank, F->rank, F->by_rank, seen, err);
        } else if (opt.ordering == SRW_ORDER_NATURAL) {
            k_rank_natural<<<g, BLOCK, 0, s>>>(n, F->rank, F->by_rank);
        } else {
            uint64_t* keys = ALLOC(tmp, uint64_t, n);
            uint64_t* keys2 = ALLOC(tmp, uint64_t, n);
            uint32_t* vals = ALLOC(tmp, uint32_t, n);
            uint32_t* vals2 = ALLOC(tmp, uint32_t, n);
            void* rt = ALLOC(tmp, char, radix_tmp_bytes(n));
            if (!keys || !keys2 || !vals || !vals2 || !rt) FAIL(SRW_E_NOMEM);
            k_rank_keys<<<g, BLOCK, 0, s>>>(n, seed, keys, vals);
            uint64_t* ko;
            uint32_t* vo;
            CHECK_HIP(radix_sort_u64(keys, vals, keys2, vals2, n, 64, rt, &ko, &vo, s));
            k_rank_scatter<<<g, BLOCK, 0, s>>>(n, vo, F->rank, F->by_rank);
        }
        CHECK_HIP(hipGetLastError());
        CHECK_HIP(hipMemcpyAsync(&pinned[0], err, sizeof(int), hipMemcpyDeviceToHost, s));
        CHECK_HIP(hipStreamSynchronize(s));
        std::memcpy(&herr, &pinned[0], sizeof(int));
        if (herr) FAIL(map_err(herr));

        // ---- 3. transition table and walk budgets
        // walk records: line offsets from an exclusive scan of the lines per node
        int32_t* nlines = ALLOC(tmp, int32_t, n);
        int64_t* rline = ALLOC(tmp, int64_t, n);
        uint8_t* kbv = ALLOC(tmp, uint8_t, n);
        int64_t* ltot = ALLOC(tmp, int64_t, 1);
        void* lst = ALLOC(tmp, char, scan_tmp_bytes(n));
        if (!nlines || !rline || !kbv || !ltot || !lst) FAIL(SRW_E_NOMEM);
        // bucket lines for the wide nodes where they fit, unless the main lines would
        // pass 2^LINE_KB_SHIFT (then the plain layout)
        int32_t bucketing = 1;
        int64_t n_lines = 0;
        int32_t* anyb = ALLOC(tmp, int32_t, 1);
        if (!anyb) FAIL(SRW_E_NOMEM);
        for (;;) {
            CHECK_HIP(hipMemsetAsync(anyb, 0, sizeof(int32_t), s));
            k_rec_lines<<<g, BLOCK, 0, s>>>(n, A->rowptr, A->col, A->val, bucketing, nlines, kbv,
                                            anyb);
            CHECK_HIP(exclusive_scan_i32_to_i64(nlines, rline, n, lst, s));
            k_read_last<<<1, 1, 0, s>>>(rline, nlines, n, ltot);
            CHECK_HIP(hipMemcpyAsync(&pinned[0], ltot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            CHECK_HIP(hipMemcpyAsync(&pinned[1], anyb, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            CHECK_HIP(hipStreamSynchronize(s));
            n_lines = pinned[0];
            int32_t any = 0;
            std::memcpy(&any, &pinned[1], sizeof(int32_t));
            if (!bucketing || n_lines <= (int64_t)LINE_MASK) {
                bucketing = bucketing && any;  // the walk kernel decodes line words only then
                break;
            }
            bucketing = 0;
        }
        if (2 * n_lines >= (int64_t)UINT32_MAX) FAIL(SRW_E_ARG);  // line indices are 32-bit
        // walk records, then start records of the same shape
        uint4* recs = ALLOC(tmp, uint4, 2 * n_lines * 4);
        uint2* ent = opt.keep >= 1 ? ALLOC(keep, uint2, nnz_off) : nullptr;  // export only
        uint32_t* mthr = ALLOC(xk, uint32_t, nnz_off);
        double* tau = ALLOC(xk, double, n);
        int32_t* budget = ALLOC(xk, int32_t, n);
        int32_t* maxb = ALLOC(tmp, int32_t, 1);
        if (!recs || (opt.keep >= 1 && !ent) || !mthr || !tau || !budget || !maxb)
            FAIL(SRW_E_NOMEM);
        F->ent = ent;
        F->mthr = mthr;
        F->tau = tau;
        F->budget = budget;
        mark(2);
        CHECK_HIP(hipMemsetAsync(maxb, 0, sizeof(int32_t), s));
        k_table<<<g, BLOCK, 0, s>>>(n, A->rowptr, A->col, A->val, F->rank, grounded, walks_per_row,
                                    opt.walks, plain ? 1 : 0, rline, kbv, bucketing, n_lines,
                                    (uint32_t*)recs, ent,
                                    mthr, tau, budget, maxb);
        CHECK_HIP(hipGetLastError());

        // record offsets (node order) and the segmented chunk list
        int64_t* rec_off = ALLOC(xk, int64_t, n);
        int32_t* flag = ALLOC(tmp, int32_t, n);
        int32_t* flag2 = ALLOC(tmp, int32_t, n);
        int64_t* pos = ALLOC(tmp, int64_t, n);
        int64_t* pos2 = ALLOC(tmp, int64_t, n);
        int32_t* order = ALLOC(tmp, int32_t, n);
        int32_t* chunks = ALLOC(tmp, int32_t, n + 1);
        int64_t* chunk_off = ALLOC(tmp, int64_t, n + 1);
        int64_t* tot = ALLOC(tmp, int64_t, 8);
        int64_t* bounds = ALLOC(tmp, int64_t, NSEG + 1);
        void* st = ALLOC(tmp, char, scan_tmp_bytes(n + 1));
        if (!rec_off || !flag || !flag2 || !pos || !pos2 || !order || !chunks || !chunk_off ||
            !tot || !bounds || !st)
            FAIL(SRW_E_NOMEM);
        F->rec_off = rec_off;
        mark(3);
        // schedule 0: every walking row in the rank-ordered segment
        const int64_t long_rank = opt.schedule == 1 ? std::max<int64_t>(1, n / 256) : n;
        CHECK_HIP(exclusive_scan_i32_to_i64(budget, rec_off, n, st, s));
        k_read_last<<<1, 1, 0, s>>>(rec_off, budget, n, tot + 0);
        k_flag_long<<<grid_for(long_rank, BLOCK), BLOCK, 0, s>>>(n, long_rank, F->by_rank, budget, flag);
        CHECK_HIP(exclusive_scan_i32_to_i64(flag, pos, long_rank, st, s));
        k_read_last<<<1, 1, 0, s>>>(pos, flag, long_rank, tot + 1);
        k_flag_slab<<<g, BLOCK, 0, s>>>(n, long_rank, F->rank, budget, flag2);
        CHECK_HIP(exclusive_scan_i32_to_i64(flag2, pos2, n, st, s));
        k_read_last<<<1, 1, 0, s>>>(pos2, flag2, n, tot + 2);
        CHECK_HIP(hipMemcpyAsync(&pinned[0], tot, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        CHECK_HIP(hipMemcpyAsync(&pinned[3], maxb, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        CHECK_HIP(hipStreamSynchronize(s));
        const int64_t total_walks = pinned[0];
        const int64_t nlong = pinned[1];
        const int64_t nslab_rows = pinned[2];
        const int64_t norder = nlong + nslab_rows;
        int32_t max_budget = 0;
        std::memcpy(&max_budget, &pinned[3], sizeof(int32_t));
        // a chunk descriptor packs the first walk of a chunk into 16 bits and the tally
        // holds a row's ends in LDS: per-row budgets above 8192 are refused here, before
        // any walk runs
        if (max_budget > 8192) {
            set_last_error("srw_build_factor: a per-row walk budget exceeds 8192");
            FAIL(SRW_E_ARG);
        }
        k_compact<<<grid_for(long_rank, BLOCK), BLOCK, 0, s>>>(long_rank, F->by_rank, flag, pos, 0,
                                                               budget, order, chunks, SRW_WAVE);
        k_compact<<<g, BLOCK, 0, s>>>(n, nullptr, flag2, pos2, nlong, budget, order, chunks,
                                      (int32_t)CHUNK_WALKS);
        CHECK_HIP(exclusive_scan_i32_to_i64(chunks, chunk_off, norder, st, s));
        k_read_last<<<1, 1, 0, s>>>(chunk_off, chunks, norder, tot + 3);
        CHECK_HIP(hipMemcpyAsync(&pinned[4], tot + 3, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        CHECK_HIP(hipStreamSynchronize(s));
        const int64_t n_chunks = pinned[4];
        F->walks_total = total_walks;
        ChunkDesc* cdesc = ALLOC(tmp, ChunkDesc, n_chunks);
        if (!cdesc) FAIL(SRW_E_NOMEM);
        k_set_last<<<1, 1, 0, s>>>(chunk_off, norder, n_chunks);
        // a walk's first step reads the row's start record (higher-ranked neighbours
        // only), or for the plain estimator the row's own record
        k_chunks<<<grid_for(norder, BLOCK), BLOCK, 0, s>>>(
            norder, nlong, order, chunk_off, budget, rline, kbv, plain ? 0 : n_lines, F->rank, rec_off,
            seed,
            batch ? batch->node_mat : nullptr, batch ? batch->mat_off : nullptr,
            batch ? batch->mat_seed : nullptr, cdesc);
        k_seg_bounds<<<1, 1, 0, s>>>(n, nlong, nslab_rows, pos2, chunk_off, bounds);
        CHECK_HIP(hipGetLastError());

        // ---- 4. walks
        // per-walk records (not with walk reuse, whose records are the counted walks)
        uint32_t* rec_end = nullptr;
        uint32_t* rec_vis = nullptr;
        uint32_t* rec_len = nullptr;
        if (!reuse) {
            rec_end = ALLOC((opt.keep >= 2 ? keep : tmp), uint32_t, total_walks);
            rec_vis = ALLOC((opt.keep >= 2 ? keep : tmp), uint32_t, total_walks);
            rec_len = ALLOC((opt.keep >= 2 ? keep : tmp), uint32_t, total_walks);
            if (!rec_end || !rec_vis || !rec_len) FAIL(SRW_E_NOMEM);
        }
        // segment queues, degree sum, then (walk reuse) record count and step sum
        unsigned long long* queue = ALLOC(tmp, unsigned long long, NSEG + 3);
        if (!queue) FAIL(SRW_E_NOMEM);
        CHECK_HIP(hipMemsetAsync(queue, 0, (NSEG + 3) * sizeof(unsigned long long), s));
        uint64_t* out_key = nullptr;
        uint2* out_vl = nullptr;
        int64_t n_slots = 0;  // walk reuse: record slots taken (records and unused slots)
        if (opt.keep >= 2) {
            F->rec_end = rec_end;
            F->rec_vis = rec_vis;
            F->rec_len = rec_len;
        }
        mark(4);
        if (n_chunks > 0) {
            WalkArgs wa{};
            wa.recs = recs;
            wa.lds_lines = (uint32_t)(2 * n_lines);
            wa.chunks = cdesc;
            wa.bounds = bounds;
            wa.max_steps = opt.max_steps;
            wa.rec_end = rec_end;
            wa.rec_vis = rec_vis;
            wa.rec_len = rec_len;
            wa.queue = queue;
            // several slab chunks per claim, about 4 CHUNK_WALKS walks (the walks do not
            // depend on which wave runs them)
            wa.slab_claim = (uint32_t)std::min<int64_t>(
                16, std::max<int64_t>(1, 4 * (int64_t)CHUNK_WALKS / std::max<int32_t>(1, max_budget)));
            wa.deg_sum = queue + NSEG;
            wa.err = err;
            int dev = 0, cus = 0;
            CHECK_HIP(hipGetDevice(&dev));
            CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            void (*kern)(WalkArgs) = nullptr;
            // a table that fits in one workgroup's LDS is staged there (the default
            // refill period only)
            int lds_max = 0;
            CHECK_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
            const size_t table_bytes = (size_t)(2 * n_lines) * 64;
            const bool lds_table = !reuse && opt.refill_period == 8 && table_bytes <= (size_t)lds_max;
            size_t dyn_lds = 0;
            if (lds_table) {
                kern = bucketing ? k_walk_lds<true> : k_walk_lds<false>;
                dyn_lds = table_bytes;
                F->walk_lds = 1;
                CHECK_HIP(hipFuncSetAttribute((const void*)kern,
                                              hipFuncAttributeMaxDynamicSharedMemorySize,
                                              (int)dyn_lds));
            } else if (reuse) {
                kern = bucketing ? k_walk_reuse<true> : k_walk_reuse<false>;
            } else if (bucketing) {
                switch (opt.refill_period) {
                    case 2: kern = k_walk<2, true>; break;
                    case 4: kern = k_walk<4, true>; break;
                    case 8: kern = k_walk<8, true>; break;
                    default: kern = k_walk<1, true>; break;
                }
            } else {
                switch (opt.refill_period) {
                    case 2: kern = k_walk<2, false>; break;
                    case 4: kern = k_walk<4, false>; break;
                    case 8: kern = k_walk<8, false>; break;
                    default: kern = k_walk<1, false>; break;
                }
            }
            // persistent grid of walk_waves waves per CU (at most what fits)
            int per_cu = 0;
            CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, BLOCK, dyn_lds));
            const int want = (opt.walk_waves > 0 ? opt.walk_waves : WALK_WAVES_PER_CU) / (BLOCK / 64);
            int64_t blocks = (int64_t)cus * std::max(1, std::min(per_cu, want));
            F->walk_waves = std::max(1, std::min(per_cu, want)) * (BLOCK / 64);
            blocks = std::min<int64_t>(blocks, (n_chunks + BLOCK / 64 - 1) / (BLOCK / 64));
            if (blocks < 1) blocks = 1;
            if (!reuse) {
                hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(BLOCK), dyn_lds, s, wa);
                CHECK_HIP(hipGetLastError());
            } else {
                wa.stack_depth = REUSE_STACK;
                wa.stack = ALLOC(tmp, uint4, blocks * BLOCK * REUSE_STACK);
                wa.nrec = queue + NSEG + 1;
                wa.steps_sum = queue + NSEG + 2;
                if (!wa.stack) FAIL(SRW_E_NOMEM);
                // record buffers sized by a first guess; if the walks take more slots,
                // they run again (same draws, same records) into larger buffers
                const int64_t slack = 2 * blocks * (BLOCK / 64) * (int64_t)REUSE_CHUNK;
                int64_t cap = 12 * total_walks + slack;
                for (int pass = 0;; ++pass) {
                    out_key = ALLOC(tmp, uint64_t, cap);
                    out_vl = ALLOC(tmp, uint2, cap);
                    if (!out_key || !out_vl) FAIL(SRW_E_NOMEM);
                    wa.out_key = out_key;
                    wa.out_vl = out_vl;
                    wa.out_cap = (unsigned long long)cap;
                    if (pass > 0)
                        CHECK_HIP(hipMemsetAsync(queue, 0, (NSEG + 3) * sizeof(unsigned long long), s));
                    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(BLOCK), 0, s, wa);
                    CHECK_HIP(hipGetLastError());
                    CHECK_HIP(hipMemcpyAsync(&pinned[6], queue + NSEG + 1, 2 * sizeof(int64_t),
                                             hipMemcpyDeviceToHost, s));
                    CHECK_HIP(hipMemcpyAsync(&pinned[0], err, sizeof(int), hipMemcpyDeviceToHost, s));
                    CHECK_HIP(hipStreamSynchronize(s));
                    std::memcpy(&herr, &pinned[0], sizeof(int));
                    if (herr) FAIL(map_err(herr));
                    n_slots = pinned[6];
                    if (n_slots <= cap) break;
                    if (pass >= 2) {
                        set_last_error("walk reuse: record slots kept outgrowing their buffer");
                        FAIL(SRW_E_HIP);
                    }
                    cap = n_slots + slack;
                }
                if (n_slots >= (int64_t)UINT32_MAX) FAIL(SRW_E_ARG);  // slot indices are 32-bit
                F->steps_total = pinned[7];
            }
        }
        mark(5);
        CHECK_HIP(hipMemcpyAsync(&pinned[5], queue + NSEG, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        CHECK_HIP(hipMemcpyAsync(&pinned[0], err, sizeof(int), hipMemcpyDeviceToHost, s));
        CHECK_HIP(hipStreamSynchronize(s));
        std::memcpy(&herr, &pinned[0], sizeof(int));
        if (herr) FAIL(map_err(herr));
        F->deg_sum = pinned[5];
        if (rule) {  // walks only: the stopping rule's verdict per row, no factor
            k_length_rule<<<row_grid(n), 64, 0, s>>>(
                n, budget, rec_off, rec_len, rule->delta, rule->z, rule->min_walks, rule->found);
            CHECK_HIP(hipGetLastError());
            CHECK_HIP(hipStreamSynchronize(s));
            status = SRW_WALKS_ONLY;
            goto done;
        }

        // ---- 5. tallies
        uint64_t* tJ = ALLOC(xk, uint64_t, n);
        uint32_t* tG = ALLOC(xk, uint32_t, n);
        uint64_t* tsteps = ALLOC(xk, uint64_t, n);
        uint64_t* tvsq = ALLOC(xk, uint64_t, n);
        int32_t* hlen = ALLOC(xk, int32_t, n);
        // the H lists overwrite the records of their own row in place unless the
        // records or the lists outlive the build
        uint32_t* h_end = rec_end;
        uint32_t* h_cnt = rec_vis;
        int64_t* h_off = rec_off;
        int64_t tallied = total_walks;
        uint64_t* ko = out_key;
        uint32_t* vo = nullptr;
        if (reuse) {
            // sort the record slots by (start node, end node), unused slots last; the
            // first slot of every row, and so the number of records, by binary search
            h_off = ALLOC(xk, int64_t, n + 1);
            uint64_t* key2 = ALLOC(tmp, uint64_t, n_slots);
            uint32_t* idx = ALLOC(tmp, uint32_t, n_slots);
            uint32_t* idx2 = ALLOC(tmp, uint32_t, n_slots);
            void* rt = ALLOC(tmp, char, radix_tmp_bytes(n_slots));
            if (!h_off || !key2 || !idx || !idx2 || !rt) FAIL(SRW_E_NOMEM);
            int rbits = 1;  // 2^rbits > n: a record's key stays below an unused slot's
            while (rbits < 31 && ((int64_t)1 << rbits) <= n) ++rbits;
            vo = idx;
            if (n_slots > 0) {
                k_iota_u32<<<grid_for(n_slots, BLOCK), BLOCK, 0, s>>>(n_slots, idx);
                CHECK_HIP(radix_sort_u64(out_key, idx, key2, idx2, n_slots, 32 + rbits, rt, &ko,
                                         &vo, s));
            }
            k_row_begin<<<grid_for(n + 1, BLOCK), BLOCK, 0, s>>>(n, ko, n_slots, h_off);
            CHECK_HIP(hipMemcpyAsync(&pinned[0], h_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            CHECK_HIP(hipStreamSynchronize(s));
            tallied = pinned[0];
        }
        if (opt.keep >= 1 || reuse) {
            h_end = ALLOC((opt.keep >= 1 ? keep : tmp), uint32_t, tallied);
            h_cnt = ALLOC((opt.keep >= 1 ? keep : tmp), uint32_t, tallied);
        }
        if (!tJ || !tG || !tsteps || !tvsq || !hlen || !h_end || !h_cnt) FAIL(SRW_E_NOMEM);
        F->h_off = h_off;
        F->tallied_total = tallied;
        F->tJ = tJ;
        F->tG = tG;
        F->tsteps = tsteps;
        F->tvsq = tvsq;
        F->hlen = hlen;
        F->h_end = h_end;
        F->h_cnt = h_cnt;
        if (reuse) {
            // one wave per row over its sorted records; the walks per row become the
            // counted walks
            k_row_count<<<g, BLOCK, 0, s>>>(n, h_off, budget);
            k_tally_sorted<<<row_grid(n), 64, 0, s>>>(
                n, h_off, ko, vo, out_vl, tJ, tG, tsteps, tvsq, hlen, h_end, h_cnt);
            CHECK_HIP(hipGetLastError());
        } else if (max_budget > 0) {
            int P = 64;
            while (P < max_budget) P <<= 1;
            // Budget classes, each launched with the LDS of its largest budget so that
            // rows with few walks keep a CU's occupancy: up to 256 walks (every row,
            // those above skip), up to 2048 and up to 8192 (hash table, then sort),
            // the last two over compacted row lists.
            const int P0 = std::min(P, 256);
            const size_t lds0 = (size_t)P0 * sizeof(uint64_t) + (size_t)(4 * P0) * sizeof(uint32_t);
            k_tally_hash<<<(unsigned)n, 64, lds0, s>>>(n, nullptr, budget, rec_off, rec_end, rec_vis,
                                                      rec_len, P0, tJ, tG, tsteps, tvsq, hlen,
                                                      h_end, h_cnt);
            CHECK_HIP(hipGetLastError());
            if (P > 256) {
                int32_t* cflag = ALLOC(tmp, int32_t, n);
                int64_t* cpos = ALLOC(tmp, int64_t, n);
                int32_t* crows = ALLOC(tmp, int32_t, n);
                void* cst = ALLOC(tmp, char, scan_tmp_bytes(n));
                if (!cflag || !cpos || !crows || !cst) FAIL(SRW_E_NOMEM);
                const int classes[2][2] = {{256, 2048}, {2048, 8192}};
                for (const auto& c : classes) {
                    if (P <= c[0]) break;
                    k_budget_class<<<g, BLOCK, 0, s>>>(n, budget, c[0], c[1], cflag);
                    CHECK_HIP(exclusive_scan_i32_to_i64(cflag, cpos, n, cst, s));
                    k_scatter_rows<<<g, BLOCK, 0, s>>>(n, cflag, cpos, crows);
                    k_read_last<<<1, 1, 0, s>>>(cpos, cflag, n, tot + 3);
                    CHECK_HIP(hipMemcpyAsync(&pinned[4], tot + 3, sizeof(int64_t),
                                             hipMemcpyDeviceToHost, s));
                    CHECK_HIP(hipStreamSynchronize(s));
                    const int64_t nc = pinned[4];
                    if (nc == 0) continue;
                    const int Pc = std::min(P, c[1]);
                    if (c[1] <= 2048) {
                        const size_t lds = (size_t)Pc * sizeof(uint64_t) +
                                           (size_t)(4 * Pc) * sizeof(uint32_t);
                        k_tally_hash<<<(unsigned)nc, 64, lds, s>>>(
                            nc, crows, budget, rec_off, rec_end, rec_vis, rec_len, Pc, tJ, tG,
                            tsteps, tvsq, hlen, h_end, h_cnt);
                    } else {
                        const size_t lds = (size_t)(2 * Pc) * sizeof(uint32_t);
                        if (lds > 64 * 1024) FAIL(SRW_E_ARG);  // budgets above 8192 walks per row
                        k_tally<<<(unsigned)nc, 64, lds, s>>>(nc, crows, budget, rec_off, rec_end,
                                                             rec_vis, rec_len, Pc, tJ, tG, tsteps,
                                                             tvsq, hlen, h_end, h_cnt);
                    }
                    CHECK_HIP(hipGetLastError());
                }
            }
        } else {
            CHECK_HIP(hipMemsetAsync(tJ, 0, n * sizeof(uint64_t), s));
            CHECK_HIP(hipMemsetAsync(tG, 0, n * sizeof(uint32_t), s));
            CHECK_HIP(hipMemsetAsync(tsteps, 0, n * sizeof(uint64_t), s));
            CHECK_HIP(hipMemsetAsync(tvsq, 0, n * sizeof(uint64_t), s));
            CHECK_HIP(hipMemsetAsync(hlen, 0, n * sizeof(int32_t), s));
        }
        {
            unsigned long long* ssum = (unsigned long long*)(tot + 3);
            CHECK_HIP(hipMemsetAsync(ssum, 0, sizeof(int64_t), s));
            k_sum_u64<<<std::min(grid_for(n, BLOCK), 2048), BLOCK, 0, s>>>(n, tsteps, ssum);
            CHECK_HIP(hipMemcpyAsync(&pinned[4], ssum, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        }

        // ---- 6. factor: one pass writes every row at an offset padded to an upper
        // bound of its length (and the row's length), then the rows are packed
        int32_t* ynnz = ALLOC(tmp, int32_t, n);
        int32_t* pcap = ALLOC(tmp, int32_t, n);
        int64_t* pad_off = ALLOC(tmp, int64_t, n + 1);
        if (!ynnz || !pcap || !pad_off) FAIL(SRW_E_NOMEM);
        mark(6);
        k_factor_caps<<<g, BLOCK, 0, s>>>(n, A->rowptr, budget, hlen, pcap);
        CHECK_HIP(exclusive_scan_i32_to_i64(pcap, pad_off, n, st, s));
        k_read_last<<<1, 1, 0, s>>>(pad_off, pcap, n, tot + 2);
        CHECK_HIP(hipMemcpyAsync(&pinned[2], tot + 2, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        CHECK_HIP(hipStreamSynchronize(s));
        const int64_t cap_total = pinned[2];
        F->d = ALLOC(keep, char, n * vbytes);
        int32_t* pcol = ALLOC(tmp, int32_t, std::max<int64_t>(cap_total, 1));
        void* pval = ALLOC(tmp, char, std::max<int64_t>(cap_total, 1) * vbytes);
        if (!F->d || !pcol || !pval) FAIL(SRW_E_NOMEM);
        if (fp32)
            k_factor<float, true><<<g, BLOCK, 0, s>>>(n, A->rowptr, A->col, A->val, F->rank, tau,
                                                     budget, tJ, h_off, hlen, h_end, h_cnt,
                                                     drop_tol, plain ? 1 : 0, ynnz, pad_off, pcol,
                                                     (float*)pval, (float*)F->d);
        else
            k_factor<double, true><<<g, BLOCK, 0, s>>>(n, A->rowptr, A->col, A->val, F->rank, tau,
                                                      budget, tJ, h_off, hlen, h_end, h_cnt,
                                                      drop_tol, plain ? 1 : 0, ynnz, pad_off, pcol,
                                                      (double*)pval, (double*)F->d);
        CHECK_HIP(exclusive_scan_i32_to_i64(ynnz, F->yptr, n, st, s));
        k_read_last<<<1, 1, 0, s>>>(F->yptr, ynnz, n, tot + 0);
        CHECK_HIP(hipMemcpyAsync(&pinned[0], tot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        CHECK_HIP(hipStreamSynchronize(s));
        const int64_t nnz_y = pinned[0];
        if (!reuse) F->steps_total = pinned[4];
        F->nnz_y = nnz_y;
        if (nnz_y >= (int64_t)0xFFFFFFFFll) FAIL(SRW_E_ARG);
        k_set_last<<<1, 1, 0, s>>>(F->yptr, n, nnz_y);
        F->ycol = ALLOC(keep, int32_t, nnz_y);
        F->yval = ALLOC(keep, char, nnz_y * vbytes);
        if (!F->ycol || !F->yval) FAIL(SRW_E_NOMEM);
        if (fp32)
            k_pack_rows<float><<<grid_for(16 * n, BLOCK), BLOCK, 0, s>>>(
                n, pad_off, F->yptr, ynnz, pcol, (const float*)pval, F->ycol, (float*)F->yval);
        else
            k_pack_rows<double><<<grid_for(16 * n, BLOCK), BLOCK, 0, s>>>(
                n, pad_off, F->yptr, ynnz, pcol, (const double*)pval, F->ycol, (double*)F->yval);
        CHECK_HIP(hipGetLastError());

        if (ic0 && n > 0) {
            unsigned long long* claim = (unsigned long long*)ALLOC(tmp, int64_t, 1);
            if (!claim) FAIL(SRW_E_NOMEM);
            CHECK_HIP(hipMemsetAsync(err, 0, sizeof(int), s));
            CHECK_HIP(hipMemsetAsync(claim, 0, sizeof(int64_t), s));
            k_fill_u64<<<std::min(g, 2048), BLOCK, 0, s>>>(n, (unsigned long long*)F->d, IC0_PENDING);
            int dev = 0, cus = 0;
            CHECK_HIP(hipGetDevice(&dev));
            CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            const int64_t claims = (n + 63) / 64;
            const int blocks = (int)std::max<int64_t>(
                1, std::min<int64_t>((int64_t)cus * 8, (claims + BLOCK / 64 - 1) / (BLOCK / 64)));
            k_ic0<<<blocks, BLOCK, 0, s>>>(n, A->rowptr, A->col, A->val, F->rank, F->by_rank,
                                           F->yptr, F->ycol, (double*)F->yval, (double*)F->d,
                                           claim, err, wait_ticks(10.0));
            CHECK_HIP(hipGetLastError());
            CHECK_HIP(hipMemcpyAsync(&pinned[0], err, sizeof(int), hipMemcpyDeviceToHost, s));
            CHECK_HIP(hipStreamSynchronize(s));
            std::memcpy(&herr, &pinned[0], sizeof(int));
            if (herr) FAIL(map_err(herr));
        }

        // ---- 7. Y^T by a stable sort of the entries on their column, then the plan.
        // A rank-ordered plan (no level sort) sorts on the column's rank and fills its
        // rows of Y^T by slot straight from the sorted entries; the level order sorts
        // on the column's node, and the rows are relabelled once the slots are known.
        mark(7);
        const bool bt_direct = opt.solve_order != 1;
        int64_t* ytptr = nullptr;
        int32_t* ytcol = nullptr;
        void* ytval = nullptr;
        if (!bt_direct) {
            ytptr = ALLOC(tmp, int64_t, n + 1);
            ytcol = ALLOC(tmp, int32_t, nnz_y);
            ytval = ALLOC(tmp, char, nnz_y * vbytes);
            if (!ytptr || !ytcol || !ytval) FAIL(SRW_E_NOMEM);
        }
        uint64_t* yt_key = nullptr;  // sorted (listing position << 32 | column field)
        uint32_t* yt_idx = nullptr;  // and the entry each came from
        {
            uint32_t* idx = ALLOC(tmp, uint32_t, nnz_y);
            uint32_t* idx2 = ALLOC(tmp, uint32_t, nnz_y);
            uint64_t* key = ALLOC(tmp, uint64_t, nnz_y);
            uint64_t* key2 = ALLOC(tmp, uint64_t, nnz_y);
            void* rt = ALLOC(tmp, char, radix_tmp_bytes(nnz_y));
            if (!idx || !idx2 || !key || !key2 || !rt) FAIL(SRW_E_NOMEM);
            int rbits = 1;
            while (rbits < 31 && ((int64_t)1 << rbits) < n) ++rbits;
            int32_t* dlen = ALLOC(tmp, int32_t, n);
            int64_t* doff = ALLOC(tmp, int64_t, n + 1);
            if (!dlen || !doff) FAIL(SRW_E_NOMEM);
            k_desc_lens<<<g, BLOCK, 0, s>>>(n, F->by_rank, F->yptr, dlen);
            CHECK_HIP(exclusive_scan_i32_to_i64(dlen, doff, n, st, s));
            k_entry_keys<<<grid_for(16 * n, BLOCK), BLOCK, 0, s>>>(
                n, F->by_rank, F->yptr, F->ycol, bt_direct ? F->rank : nullptr, doff, idx, key);
            uint64_t* ko;
            uint32_t* vo;
            // stable on the column bits only: the listing order supplies the rank order
            CHECK_HIP(radix_sort_u64(key, idx, key2, idx2, nnz_y, rbits, rt, &ko, &vo, s));
            yt_key = ko;
            yt_idx = vo;
            if (!bt_direct) {
                // rows of Y^T: where each column's run of sorted keys begins
                k_row_begin<<<grid_for(n + 1, BLOCK), BLOCK, 0, s>>>(n, ko, nnz_y, ytptr, 0,
                                                                     (1ull << 32) - 1ull);
                if (fp32)
                    k_transpose_fill<float><<<grid_for(nnz_y, BLOCK), BLOCK, 0, s>>>(
                        nnz_y, n, ko, vo, F->by_rank, (const float*)F->yval, ytcol,
                        (float*)ytval);
                else
                    k_transpose_fill<double><<<grid_for(nnz_y, BLOCK), BLOCK, 0, s>>>(
                        nnz_y, n, ko, vo, F->by_rank, (const double*)F->yval, ytcol,
                        (double*)ytval);
            }
            CHECK_HIP(hipGetLastError());
        }

        // the solves' dense head (single builds): the lowest-ranked rows
        int64_t head =
            (batch || asym || rule || opt.head_rows < 0)
                ? 0
                : std::min<int64_t>(n, head_rows_fit(opt.head_rows == 0 ? HEAD_DEFAULT
                                                                        : (int64_t)opt.head_rows));
        // solve plan: rows of Y and Y^T by slot, starting from the rank order
        F->slot_node = ALLOC(keep, int32_t, n);
        F->node_slot = ALLOC(keep, int32_t, n);
        F->fptr = ALLOC(keep, int64_t, n + 1);
        F->fcol = ALLOC(keep, int32_t, nnz_y);
        F->fval = ALLOC(keep, char, nnz_y * vbytes);
        F->bptr = ALLOC(keep, int64_t, n + 1);
        F->bcol = ALLOC(keep, int32_t, nnz_y);
        F->bval = ALLOC(keep, char, nnz_y * vbytes);
        F->dslot = ALLOC(keep, char, n * vbytes);
        int32_t* lens = ALLOC(tmp, int32_t, n);
        if (!F->slot_node || !F->node_slot || !F->fptr || !F->fcol || !F->fval || !F->bptr ||
            !F->bcol || !F->bval || !F->dslot || !lens)
            FAIL(SRW_E_NOMEM);
        auto relabel = [&](const int64_t* sptr, const int32_t* scol, const void* sval,
                           int64_t* dptr, int32_t* dcol, void* dval) -> hipError_t {
            k_slot_lens<<<g, BLOCK, 0, s>>>(n, F->slot_node, sptr, lens);
            hipError_t e = exclusive_scan_i32_to_i64(lens, dptr, n, st, s);
            if (e != hipSuccess) return e;
            k_set_last<<<1, 1, 0, s>>>(dptr, n, nnz_y);
            const unsigned pg = (unsigned)grid_for(16 * n, BLOCK);
            if (fp32)
                k_permute_rows<float><<<pg, BLOCK, 0, s>>>(n, F->slot_node, F->node_slot, sptr,
                                                           scol, (const float*)sval, dptr, dcol,
                                                           (float*)dval);
            else
                k_permute_rows<double><<<pg, BLOCK, 0, s>>>(n, F->slot_node, F->node_slot, sptr,
                                                            scol, (const double*)sval, dptr, dcol,
                                                            (double*)dval);
            return hipGetLastError();
        };
        if (n > 0) {
            k_copy_i32<<<g, BLOCK, 0, s>>>(n, F->by_rank, F->slot_node);
            k_copy_i32<<<g, BLOCK, 0, s>>>(n, F->rank, F->node_slot);
            CHECK_HIP(relabel(F->yptr, F->ycol, F->yval, F->fptr, F->fcol, F->fval));
            if (head > 0) {
                // the head's inverse costs about head x (its entries) / 4 entry reads:
                // keep that within HEAD_COST (long rows, e.g. from large per-row
                // budgets, shorten the head)
                int64_t* hb = ALLOC(tmp, int64_t, 1);
                if (!hb) FAIL(SRW_E_NOMEM);
                k_head_bound<<<1, 1, 0, s>>>(F->fptr, head, HEAD_COST, hb);
                CHECK_HIP(hipMemcpyAsync(&pinned[0], hb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
                CHECK_HIP(hipStreamSynchronize(s));
                head = pinned[0];
            }
        } else {
            CHECK_HIP(hipMemsetAsync(F->fptr, 0, sizeof(int64_t), s));
            CHECK_HIP(hipMemsetAsync(F->bptr, 0, sizeof(int64_t), s));
        }
        // level order: slots by (dependency level, rank)
        if (opt.solve_order == 1 && n > 0) {  // 2 (automatic) is the rank order here
            int32_t* lev = ALLOC(tmp, int32_t, n);
            uint32_t* lkey = ALLOC(tmp, uint32_t, n);
            uint32_t* lkey2 = ALLOC(tmp, uint32_t, n);
            uint32_t* lval = ALLOC(tmp, uint32_t, n);
            uint32_t* lval2 = ALLOC(tmp, uint32_t, n);
            void* rt = ALLOC(tmp, char, radix_tmp_bytes(n));
            if (!lev || !lkey || !lkey2 || !lval || !lval2 || !rt) FAIL(SRW_E_NOMEM);
            int32_t depth = 0;
            status = dag_levels(F, lev, &depth, s, batch ? batch->level_order : nullptr);
            if (status) goto done;
            F->depth = depth;
            k_level_keys<<<g, BLOCK, 0, s>>>(n, head, F->slot_node, lev, lkey, lval);
            int bits = 8;
            while (bits < 32 && ((int64_t)1 << bits) <= (int64_t)depth + 1) bits += 8;
            uint32_t* ko;
            uint32_t* vo;
            CHECK_HIP(radix_sort_u32(lkey, lval, lkey2, lval2, n, bits, rt, &ko, &vo, s));
            // the levels' slot ranges, for level-by-level substitutions
            int64_t* kptr = ALLOC(tmp, int64_t, (size_t)depth + 2);
            if (!kptr) FAIL(SRW_E_NOMEM);
            k_key_ptr<<<grid_for(n + 1, BLOCK), BLOCK, 0, s>>>(n, ko, (uint32_t)depth, kptr);
            F->level_ptr.assign((size_t)depth + 1, 0);
            CHECK_HIP(hipMemcpyAsync(F->level_ptr.data(), kptr + 1, ((size_t)depth + 1) * sizeof(int64_t),
                                     hipMemcpyDeviceToHost, s));
            k_copy_i32<<<g, BLOCK, 0, s>>>(n, (const int32_t*)vo, F->slot_node);
            k_invert<<<g, BLOCK, 0, s>>>(n, F->slot_node, F->node_slot);
            CHECK_HIP(relabel(F->yptr, F->ycol, F->yval, F->fptr, F->fcol, F->fval));
        }
        if (n > 0) {
            if (bt_direct) {
                // slots are ranks: the sorted entries are already the rows of Y^T by slot
                k_row_begin<<<grid_for(n + 1, BLOCK), BLOCK, 0, s>>>(n, yt_key, nnz_y, F->bptr, 0,
                                                                     (1ull << 32) - 1ull);
                if (fp32)
                    k_transpose_fill_slots<float><<<grid_for(nnz_y, BLOCK), BLOCK, 0, s>>>(
                        nnz_y, n, yt_key, yt_idx, (const float*)F->yval, F->bcol,
                        (float*)F->bval);
                else
                    k_transpose_fill_slots<double><<<grid_for(nnz_y, BLOCK), BLOCK, 0, s>>>(
                        nnz_y, n, yt_key, yt_idx, (const double*)F->yval, F->bcol,
                        (double*)F->bval);
            } else {
                CHECK_HIP(relabel(ytptr, ytcol, ytval, F->bptr, F->bcol, F->bval));
            }
            if (fp32)
                k_gather_slots<float><<<g, BLOCK, 0, s>>>(n, F->slot_node, (const float*)F->d,
                                                          (float*)F->dslot);
            else
                k_gather_slots<double><<<g, BLOCK, 0, s>>>(n, F->slot_node, (const double*)F->d,
                                                           (double*)F->dslot);
            CHECK_HIP(hipGetLastError());
        }
        if (head > 0) {
            const size_t hb = (size_t)(head * (head + 1) / 2) * vbytes;
            F->head = head;
            F->hx = ALLOC(keep, char, hb);
            F->hxt = ALLOC(keep, char, hb);
            int* herr = ALLOC(tmp, int, 1);
            if (!F->hx || !F->hxt || !herr) FAIL(SRW_E_NOMEM);
            CHECK_HIP(head_inverse_launch(F, herr, s));
            CHECK_HIP(hipMemcpyAsync(&pinned[0], herr, sizeof(int), hipMemcpyDeviceToHost, s));
            CHECK_HIP(hipStreamSynchronize(s));
            int he = 0;
            std::memcpy(&he, &pinned[0], sizeof(int));
            if (he) {
                set_last_error("the dense head's inverse gave up waiting");
                FAIL(SRW_E_HIP);
            }
        }
        mark(8);
        CHECK_HIP(hipStreamSynchronize(s));
        if (prof) {
            for (int i = 0; i < SRW_NUM_PHASES; ++i) {
                float ms = -1.0f;
                if (ev[i] && ev[i + 1] && hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess)
                    F->phase_ms[i] = ms;
            }
        }
        if (keep.last != hipSuccess || tmp.last != hipSuccess) FAIL(SRW_E_NOMEM);
    }

done:
#undef FAIL
#undef CHECK_HIP
#undef ALLOC
    if (status == SRW_OK) {
        (void)hipStreamSynchronize(s);
    } else {
        (void)hipStreamSynchronize(s);
    }
    tmp.release();
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (status != SRW_OK) {
        keep.release();
        delete F;
        return status == SRW_WALKS_ONLY ? SRW_OK : status;
    }
    if (opt.keep < 1) {
        // what only export needs lived in the build temporaries
        F->ent = nullptr; F->mthr = nullptr; F->tau = nullptr; F->grounded = nullptr;
        F->budget = nullptr; F->rec_off = nullptr; F->h_off = nullptr; F->tJ = nullptr;
        F->tG = nullptr;
        F->tsteps = nullptr; F->tvsq = nullptr; F->hlen = nullptr;
        F->h_end = nullptr; F->h_cnt = nullptr;
    }
    F->pool_allocations = std::move(keep.blocks);
    *out = F;
    return SRW_OK;
}

}  // namespace srw
