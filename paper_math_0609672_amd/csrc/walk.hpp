// Walk records and the walk kernel (Sections 2.1, 2.2.1 and 5.2).  Included by
// build.hip inside its anonymous namespace, after BLOCK and the schedule constants
// (NSLAB, NSEG) are defined.
#pragma once

// ----------------------------------------------------------------------- table
// Walk record of node v: 64-byte lines starting at line rline[v].  32-bit words of the
// first line: [0] rank, [1] degree | grounded flag, [2] node id, [3] the line of the
// record of the neighbour taken when the draw passes every threshold (the last one).
// Every off-diagonal entry m (CSR order) is a pair: the threshold floor(2^32 c_m / a_v)
// and the line of the neighbour's record.  Unused words of a record's lines are 0.
//   degree <= 6: the pairs sit in words 4 + 2m, 5 + 2m of the first line.  The record
//     is one line, so a walk step is one dependent 64-byte load: the next node's
//     record, whose header holds the rank for the home test and the node id to record
//     where the walk ends.
//   degree > 6: the pairs fill the following lines, eight per line (entry m at word
//     16 + 2m of the record); words 4 .. 15 of the first line hold the last threshold
//     of each of the first twelve of those lines.  Thresholds grow with m, so the
//     first line whose last threshold exceeds the draw holds the chosen entry: a step
//     loads that one line.
// Start record of v: the same layout, from line n_lines + rline[v], for the first step
// of v's walks, which moves to a higher-ranked neighbour only (the exact one-step part
// of Section 5.2): the thresholds are floor(2^32 cm_m / sum of the higher-ranked
// weights) over the cumulative higher-ranked weight cm_m, word 3 is the last
// higher-ranked neighbour's line and the grounded flag is clear.  The first step is
// then the same select-and-load as every other step.
//
// Bucket lines.  A node of degree 7..BUCKET_MAX_DEG whose draw range [0, 2^32) splits
// into B = 2^kb equal parts (kb = 3..6) that each meet at most six entries' threshold
// intervals also gets B bucket lines, placed before its first line: bucket line b
// holds the record's header and, in words 4..15 as in a narrow record, the entries
// (entry order, zero-width ones left out) whose intervals meet [b 2^(32-kb),
// (b+1) 2^(32-kb)).  The chosen entry of a draw in that range is among them, so the
// selection is the narrow one.  A walk that moves to such a node holds its next draw
// already (the walk kernel makes each block of eight draws one step ahead) and loads
// the bucket line of that draw: one dependent load per step instead of two.  The line
// words of entries (and word 3) carry the target's kb in their top bits when the
// records are bucketed (all main lines below 2^LINE_KB_SHIFT).  The first line and the
// continuation lines stay: a walk of the plain estimator starts from its row's own
// record.
constexpr int REC_WORDS = 16;
constexpr uint32_t LINE_KB_SHIFT = 27;
constexpr uint32_t LINE_MASK = (1u << LINE_KB_SHIFT) - 1u;
constexpr int64_t BUCKET_MAX_DEG = 64;
constexpr uint32_t DESC_INLINE = 0x40000000u;  // the line's pairs are in words 4..15

// Most entries (of nonzero width) that meet one of the 2^kb draw ranges of node v.
__device__ uint32_t bucket_load(int64_t v, int64_t r0, int64_t r1, const int32_t* __restrict__ col,
                                const double* __restrict__ val, double a, uint32_t kb)
{
    const uint32_t sh = 32u - kb;
    uint32_t prev = 0u, cur = 0u, cnt = 0u, mx = 0u;
    double c = 0.0;
    for (int64_t p = r0; p < r1; ++p) {
        if (col[p] == v) continue;
        c = c + (-val[p]);
        const uint32_t thr = threshold32(c, a);
        if (thr > prev) {  // the entry's draws: [prev, thr)
            const uint32_t bl = prev >> sh, bh = (thr - 1u) >> sh;
            if (bl != cur) {
                mx = max(mx, cnt);
                cur = bl;
                cnt = 0u;
            }
            ++cnt;
            if (bh != bl) {
                mx = max(mx, cnt);
                cur = bh;
                cnt = 1u;
            }
        }
        prev = thr;
    }
    return max(mx, cnt);
}

// Lines per record and the bucket exponent kb of every node (0: no bucket lines);
// *any_bucket |= 1 if some node has bucket lines.
__global__ void k_rec_lines(int64_t n, const int64_t* __restrict__ rowptr,
                            const int32_t* __restrict__ col, const double* __restrict__ val,
                            int32_t bucketing, int32_t* __restrict__ lines, uint8_t* __restrict__ kbv,
                            int32_t* any_bucket)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int64_t r0 = rowptr[v], r1 = rowptr[v + 1];
    const int64_t deg = r1 - r0 - 1;
    uint32_t kb = 0u;
    if (bucketing && deg > 6 && deg <= BUCKET_MAX_DEG) {
        double a = 0.0;
        for (int64_t p = r0; p < r1; ++p)
            if (col[p] == v) a = val[p];
        for (uint32_t k = 3u; k <= 6u && kb == 0u; ++k)
            if (bucket_load(v, r0, r1, col, val, a, k) <= 6u) kb = k;
    }
    kbv[v] = (uint8_t)kb;
    if (kb) atomicOr(any_bucket, 1);
    lines[v] = (int32_t)((kb ? (1 << kb) : 0) + (deg <= 6 ? 1 : 1 + (deg + 7) / 8));
}

// a wide record's summary words: the last threshold of each of its first twelve
// continuation lines
__device__ __forceinline__ void wide_summary(uint32_t* rec, uint32_t m)
{
    const uint32_t L = (m + 7) / 8;
    for (uint32_t l = 1; l <= 12; ++l) {
        const uint32_t last = (l * 8 < m ? l * 8 : m) - 1;  // last entry of line l
        rec[3 + l] = l <= L ? rec[16 + 2 * last] : 0u;
    }
}

// the line word of an entry that moves to node j: its first record line, with its
// bucket exponent in the top bits when the records are bucketed
__device__ __forceinline__ uint32_t line_word(const int64_t* __restrict__ rline,
                                              const uint8_t* __restrict__ kbv, int32_t bucketing,
                                              int32_t j)
{
    return (uint32_t)rline[j] | (bucketing ? (uint32_t)kbv[j] << LINE_KB_SHIFT : 0u);
}

__global__ void k_table(int64_t n, const int64_t* __restrict__ rowptr,
                        const int32_t* __restrict__ col, const double* __restrict__ val,
                        const int32_t* __restrict__ rank, const uint8_t* __restrict__ grounded,
                        int32_t walks_per_row, const int32_t* __restrict__ budget_in,
                        int32_t plain, const int64_t* __restrict__ rline,
                        const uint8_t* __restrict__ kbv, int32_t bucketing, int64_t n_lines,
                        uint32_t* __restrict__ recs, uint2* __restrict__ ent,
                        uint32_t* __restrict__ mthr, double* __restrict__ tau,
                        int32_t* __restrict__ budget, int32_t* max_budget)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int64_t r0 = rowptr[v], r1 = rowptr[v + 1];
    const int32_t rv = rank[v];
    double a = 0.0, motel = 0.0;
    for (int64_t p = r0; p < r1; ++p) {
        const int32_t j = col[p];
        if (j == v) a = val[p];
        else if (rank[j] > rv) motel = motel + (-val[p]);
    }
    const int64_t start = r0 - v;
    const uint32_t kb = kbv[v];
    const int64_t first = rline[v] + (kb ? (1 << kb) : 0);  // the first line, after the buckets
    uint32_t* rec = recs + (size_t)first * REC_WORDS;
    uint32_t* srec = recs + (size_t)(n_lines + first) * REC_WORDS;
    const uint32_t deg = (uint32_t)(r1 - r0 - 1);
    const bool wide = deg > 6;
    double c = 0.0, cm = 0.0;
    uint32_t m = 0, last_line = 0, last_motel_line = 0;
    for (int64_t p = r0; p < r1; ++p) {
        const int32_t j = col[p];
        if (j == v) continue;
        const double w = -val[p];
        c = c + w;
        const uint32_t line = line_word(rline, kbv, bucketing, j);
        if (rank[j] > rv) {
            cm = cm + w;
            last_motel_line = line;
        }
        const uint32_t thr = threshold32(c, a);
        const uint32_t mt = motel > 0.0 ? threshold32(cm, motel) : 0u;
        const uint32_t slot = wide ? 16 + 2 * m : 4 + 2 * m;
        rec[slot] = thr;
        rec[slot + 1] = line;
        srec[slot] = mt;
        srec[slot + 1] = line;
        if (ent) ent[start + m] = make_uint2((uint32_t)j, thr);
        mthr[start + m] = mt;
        last_line = line;
        ++m;
    }
    const uint32_t flags = grounded[v] ? DESC_GROUNDED : 0u;
    const uint32_t inl = wide ? 0u : DESC_INLINE;
    rec[0] = (uint32_t)rv;
    rec[1] = m | flags | inl;
    rec[2] = (uint32_t)v;
    rec[3] = last_line;
    srec[0] = (uint32_t)rv;
    srec[1] = m | inl;
    srec[2] = (uint32_t)v;
    srec[3] = last_motel_line;
    if (kb) {
        // bucket lines: the header, then the entries meeting each draw range in order
        const uint32_t B = 1u << kb, sh = 32u - kb;
        uint32_t* bl0 = recs + (size_t)rline[v] * REC_WORDS;
        for (uint32_t b = 0; b < B; ++b) {
            uint32_t* L = bl0 + (size_t)b * REC_WORDS;
            L[0] = (uint32_t)rv;
            L[1] = m | flags | DESC_INLINE;
            L[2] = (uint32_t)v;
            L[3] = last_line;
            for (int q = 4; q < REC_WORDS; ++q) L[q] = 0u;
        }
        uint32_t prev = 0u, cur = 0u, slot = 0u;
        double cc = 0.0;
        for (int64_t p = r0; p < r1; ++p) {
            const int32_t j = col[p];
            if (j == v) continue;
            cc = cc + (-val[p]);
            const uint32_t thr = threshold32(cc, a);
            if (thr > prev) {
                const uint32_t lw = line_word(rline, kbv, bucketing, j);
                for (uint32_t b = prev >> sh; b <= ((thr - 1u) >> sh); ++b) {
                    if (b != cur) {
                        cur = b;
                        slot = 0u;
                    }
                    uint32_t* L = bl0 + (size_t)b * REC_WORDS;
                    L[4 + 2 * slot] = thr;
                    L[5 + 2 * slot] = lw;
                    ++slot;
                }
            }
            prev = thr;
        }
    }
    if (wide) {
        wide_summary(rec, m);
        wide_summary(srec, m);
        for (uint32_t q = 16 + 2 * m; q % REC_WORDS != 0; ++q) {
            rec[q] = 0u;
            srec[q] = 0u;
        }
    } else {
        for (uint32_t q = 4 + 2 * m; q < REC_WORDS; ++q) {
            rec[q] = 0u;
            srec[q] = 0u;
        }
    }
    tau[v] = motel / a;
    int32_t b = 0;
    // walking rows: those with a higher-ranked neighbour (the others are exact), or
    // every row for the plain estimator
    if ((motel > 0.0 || plain) && walks_per_row != NO_WALKS) {
        b = budget_in ? budget_in[v] : walks_per_row;
        if (b < 1) b = 1;
        atomicMax(max_budget, b);
    }
    budget[v] = b;
}

// ----------------------------------------------------------------------- walks
// Chunk: up to 64 walks of one row, everything a wave needs to start them.
struct ChunkDesc {
    uint32_t key;     // Philox key word of the row: its node id (in a batch, its id
                      // within its own matrix)
    uint32_t walks;   // first walk | count << 16
    uint32_t sline;   // the row's start record line
    uint32_t rank;    // the row's rank
    uint64_t rec;     // result index of the row's walk 0
    uint64_t seed;    // the seed of the row's matrix
};
static_assert(sizeof(ChunkDesc) == 32, "chunk descriptors are 32 bytes");

// chunk descriptors of the rows in schedule order: consecutive walks of a row, SRW_WAVE
// per chunk for the first nlong rows, CHUNK_WALKS for the others; a walk starts from
// the first line of the start record (sline_base: the start records) or, with
// sline_base 0, of the row's own record
__global__ void k_chunks(int64_t norder, int64_t nlong, const int32_t* __restrict__ order,
                         const int64_t* __restrict__ chunk_off, const int32_t* __restrict__ budget,
                         const int64_t* __restrict__ rline, const uint8_t* __restrict__ kbv,
                         int64_t sline_base,
                         const int32_t* __restrict__ rank, const int64_t* __restrict__ rec_off,
                         uint64_t seed, const int32_t* __restrict__ node_mat,
                         const int64_t* __restrict__ mat_off, const uint64_t* __restrict__ mat_seed,
                         ChunkDesc* __restrict__ cdesc)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= norder) return;
    const int32_t v = order[j];
    const int32_t b = budget[v];
    ChunkDesc d;
    d.key = (uint32_t)v;
    d.seed = seed;
    if (node_mat) {
        const int32_t mi = node_mat[v];
        d.key = (uint32_t)(v - mat_off[mi]);
        d.seed = mat_seed[mi];
    }
    d.sline = (uint32_t)(sline_base + rline[v] + (kbv[v] ? (1 << kbv[v]) : 0));
    d.rank = (uint32_t)rank[v];
    d.rec = (uint64_t)rec_off[v];
    for (int64_t c = chunk_off[j]; c < chunk_off[j + 1]; ++c) {
        const uint32_t cs = j < nlong ? (uint32_t)SRW_WAVE : CHUNK_WALKS;
        const uint32_t w0 = (uint32_t)(c - chunk_off[j]) * cs;
        const uint32_t cnt = min(cs, (uint32_t)b - w0);
        d.walks = w0 | (cnt << 16);
        cdesc[c] = d;
    }
}

struct WalkArgs {
    const uint4* recs;         // walk and start records, 4 x 16 bytes per line
    uint32_t lds_lines;        // lines of recs (k_walk_lds copies them all to LDS)
    const ChunkDesc* chunks;
    const int64_t* bounds;     // NSEG + 1 segment starts
    uint64_t max_steps;
    uint32_t* rec_end;
    uint32_t* rec_vis;
    uint32_t* rec_len;
    unsigned long long* queue;
    uint32_t slab_claim;       // chunks a wave claims at once from a slab queue (>= 1)
    unsigned long long* deg_sum;
    int* err;
    // walk reuse: per-lane stacks of stack_depth entries {rank, node, position,
    // stays}; counted walks go to out_key (start node << 32 | end node, END_GROUND for
    // ground) and out_vl (stays, steps).  A wave takes slots in blocks of REUSE_CHUNK
    // from *nrec and fills the slots it leaves unused with the key ~0 (sorts last);
    // slots at or beyond out_cap are only counted.  *steps_sum collects the simulated
    // steps.
    uint4* stack;
    uint32_t stack_depth;
    uint64_t* out_key;
    uint2* out_vl;
    unsigned long long* nrec;
    unsigned long long out_cap;
    unsigned long long* steps_sum;
};

constexpr uint32_t REUSE_CHUNK = 4096;

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src)
{
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v)
{
    for (int d = 32; d > 0; d >>= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, d);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), d);
        const uint64_t o = ((uint64_t)hi << 32) | lo;
        v = o > v ? o : v;
    }
    return v;
}

// Emission of counted walks by the lanes currently executing (walk reuse).  The wave's
// slot block [*next, *end) is the same in every lane that runs this; a lane with
// `em` set writes one record.
__device__ __forceinline__ void emit_walks(const WalkArgs& a, bool em, uint32_t row, uint32_t end,
                                           uint32_t stays, uint32_t steps, uint64_t& next,
                                           uint64_t& bend)
{
    const int lane = __lane_id();
    const uint64_t lt = lanemask_lt();
    const uint64_t act = ballot(true);
    const uint64_t m = ballot(em);
    if (m == 0) return;
    const uint32_t cnt = (uint32_t)__popcll(m);
    if (next + cnt > bend) {
        // the rest of the block stays unused: mark it, then take a new block
        const uint32_t na = (uint32_t)__popcll(act), me = (uint32_t)__popcll(act & lt);
        for (uint64_t q = next + me; q < bend; q += na)
            if (q < a.out_cap) a.out_key[q] = ~0ull;
        const int leader = __ffsll((long long)act) - 1;
        unsigned long long c = 0;
        if (lane == leader) c = atomicAdd(a.nrec, (unsigned long long)REUSE_CHUNK);
        c = shfl_u64(c, leader);
        next = c;
        bend = c + REUSE_CHUNK;
    }
    if (em) {
        const uint64_t slot = next + (uint64_t)__popcll(m & lt);
        if (slot < a.out_cap) {
            a.out_key[slot] = ((uint64_t)row << 32) | end;
            a.out_vl[slot] = make_uint2(stays, steps);
        }
    }
    next += cnt;
}

// Persistent walk kernel.  Every wave owns up to 64 walks at a time, one per lane.
// Every R steps the idle lanes of a wave take the next walks of the current chunk;
// an exhausted chunk is replaced by the next one from the segment queues: the
// long-walk segment first, then the wave's own slab (by the XCD its workgroup runs
// on), then the other slabs in turn.  A lane's draws come from the Philox block of its
// (row, walk, step div 8), generated when step mod 8 = 0.  A lane holds the first
// line of its current record in registers (at the start of a walk, the row's start
// record); a step selects the entry from it (a wide record loads one more line),
// then loads the next node's record line: one dependent 64-byte load per step.
//
// REUSE (Section 5.3, Algorithm "reuse"): a lane also keeps the two stacks of the
// algorithm for its walk, as one stack of entries {rank, node, position, stays} whose
// top lives in registers and the rest in the lane's own region of a.stack.  The start
// is position 1 and the node reached by step t is position t + 2.  A node ranked
// below the top pops it, and a popped entry pushed more than one position earlier is
// a walk of at least two steps from its node: it is emitted as a record.  A node
// ranked above the top is pushed, one equal to it is a stay.  The walk ends exactly
// when the stack empties; the walk itself is the bottom entry's record.
#ifndef SRW_WALK_WAVES
#define SRW_WALK_WAVES 4  // waves per SIMD the register budget is cut for (the grid runs 2)
#endif
// recs: the records (a.recs, or the workgroup's copy of them in LDS)
template <int R, bool REUSE, bool BUCKETS>
__device__ __forceinline__ void walk_body(const WalkArgs& a, const uint4* recs)
{
    const int lane = __lane_id();
    const uint64_t lt = lanemask_lt();
    // wave-uniform chunk state
    ChunkDesc cd{};
    uint32_t c_next = 0, c_end = 0;
    uint64_t c_cur = 0, c_lim = 0;  // the chunk held and the end of the range claimed
    bool done = false;
    const int home = 1 + (int)(blockIdx.x % NSLAB);
    int seg = 0, tried = 0;
    // per-lane walk state
    bool active = false;
    uint32_t key = 0, w = 0, visits = 0, rank_k = 0;
    uint32_t cline = 0;                        // current record's first line
    uint4 r0 = make_uint4(0, 0, 0, 0), r1 = r0, r2 = r0, r3 = r0;  // its words
    uint64_t t = 0, rec = 0, degsum = 0, seedw = 0;
    uint32_t q0 = 0, q1 = 0, q2 = 0, q3 = 0, q4 = 0, q5 = 0, q6 = 0, q7 = 0;
    // REUSE: stack top, depth below it, the lane's stack region, simulated steps
    uint32_t top_rank = 0, top_node = 0, top_pos = 0, top_vis = 0, depth = 0;
    uint4* const my_stack =
        REUSE ? a.stack + ((size_t)blockIdx.x * BLOCK + threadIdx.x) * a.stack_depth : nullptr;
    uint64_t steps_acc = 0;
    uint64_t blk_next = 0, blk_end = 0;  // the wave's block of record slots
    // LOCK: a finished walk's result waits one iteration and is stored just after the
    // next record load is issued.  Stored at once, the wave had to wait for the stores
    // to complete before that load could reuse their registers: a store round trip
    // in front of nearly every step.
    bool pend = false;
    uint64_t pend_rec = 0;
    uint32_t pend_end = 0, pend_vis = 0, pend_len = 0;

    for (uint32_t iter = 0;; ++iter) {
        if ((iter % R) == 0 && !done) {
            uint64_t idle = ballot(!active);
            while (idle != 0) {
                if (c_next >= c_end) {
                    // next chunk: long segment, then home slab, then the other slabs
                    // the next chunk of the range already claimed, else a new claim:
                    // one chunk from the long segment, slab_claim from a slab
                    bool got = c_cur + 1 < c_lim;
                    unsigned long long cidx = got ? ++c_cur : 0ull;
                    while (!done && !got) {
                        const int sq = seg == 0 ? 0 : 1 + (home - 1 + tried) % NSLAB;
                        const unsigned long long size =
                            (unsigned long long)(a.bounds[sq + 1] - a.bounds[sq]);
                        const unsigned long long k = sq == 0 ? 1ull : (unsigned long long)a.slab_claim;
                        const unsigned long long c =
                            lane0_u64(atomicAdd(&a.queue[sq], lane == 0 ? k : 0ull));
                        if (c < size) {
                            got = true;
                            cidx = (unsigned long long)a.bounds[sq] + c;
                            c_cur = cidx;
                            c_lim = (unsigned long long)a.bounds[sq] + (c + k < size ? c + k : size);
                        } else if (seg == 0) {
                            seg = 1;
                        } else if (++tried >= NSLAB) {
                            done = true;
                        }
                    }
                    if (done) break;
                    cd = a.chunks[cidx];
                    c_next = cd.walks & 0xFFFFu;
                    c_end = c_next + (cd.walks >> 16);
                }
                const uint32_t avail = c_end - c_next;
                const uint32_t pos = (uint32_t)__popcll(idle & lt);
                const bool take = ((idle >> lane) & 1ull) && pos < avail;
                if (take) {
                    key = cd.key;
                    w = c_next + pos;
                    t = 0;
                    visits = 1;
                    active = true;
                    rank_k = cd.rank;
                    seedw = cd.seed;
                    rec = cd.rec + w;
                    cline = cd.sline;
                    if constexpr (REUSE) {
                        top_rank = cd.rank;
                        top_node = cd.key;
                        top_pos = 1;
                        top_vis = 1;
                        depth = 0;
                    }
                    const uint4* lp = recs + (size_t)cline * 4;
                    r0 = lp[0];
                    r1 = lp[1];
                    r2 = lp[2];
                    r3 = lp[3];
                }
                const uint64_t taken = ballot(take);
                c_next += (uint32_t)__popcll(taken);
                idle &= ~taken;
            }
        }
        if (ballot(active) == 0) {
            if (done) break;
            continue;
        }
        // LOCK (refill period 8, no reuse): every lane runs the step; an idle lane takes
        // no entry and loads line 0 (any record line will do), and keeps no result.
        // Active lanes started their walks at multiples of 8 iterations, so t and the
        // iteration count agree mod 8 and the random block refresh is wave-uniform.
        constexpr bool LOCK = !REUSE && R == 8;
        if (LOCK || active) {  // structured: the lanes rejoin before the next refill's ballots
        // draws: step t's is the word t mod 8 of the Philox block t div 8.  With bucket
        // lines a walk needs its next draw during a step, so the next block is made at
        // the block's last step and the first block when the walk starts.
        const uint32_t phase = LOCK ? (iter & 7u) : (uint32_t)(t & 7);
        if (phase == 0 && (!BUCKETS || t == 0)) {
            const u64x4 b = philox4x64_10(t >> 3, w, key, STREAM_WALK, seedw, 0);
            q0 = (uint32_t)b.x0; q1 = (uint32_t)(b.x0 >> 32);
            q2 = (uint32_t)b.x1; q3 = (uint32_t)(b.x1 >> 32);
            q4 = (uint32_t)b.x2; q5 = (uint32_t)(b.x2 >> 32);
            q6 = (uint32_t)b.x3; q7 = (uint32_t)(b.x3 >> 32);
        }
        const uint32_t u = q0;
        q0 = q1; q1 = q2; q2 = q3; q3 = q4; q4 = q5; q5 = q6; q6 = q7;
        if constexpr (BUCKETS) {
            if (phase == 7) {  // q0 becomes the next step's draw
                const u64x4 b = philox4x64_10((t + 1) >> 3, w, key, STREAM_WALK, seedw, 0);
                q0 = (uint32_t)b.x0; q1 = (uint32_t)(b.x0 >> 32);
                q2 = (uint32_t)b.x1; q3 = (uint32_t)(b.x1 >> 32);
                q4 = (uint32_t)b.x2; q5 = (uint32_t)(b.x2 >> 32);
                q6 = (uint32_t)b.x3; q7 = (uint32_t)(b.x3 >> 32);
            }
        }

        const uint32_t deg = (!LOCK || active) ? (r0.y & DESC_DEG_MASK) : 0u;
        degsum += deg;
        // an idle lane takes the in-line path: it loads nothing more
        const bool inl = (LOCK && !active) || (r0.y & DESC_INLINE) != 0u;
        // The next node is the first entry m with u < threshold_m; the words of the
        // line held (a narrow record, a bucket line, or a wide record's first line)
        // are in registers.
        const uint32_t e[16] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w,
                                r2.x, r2.y, r2.z, r2.w, r3.x, r3.y, r3.z, r3.w};
        uint32_t next_line = 0;
        bool found = false;
        if (inl) {
            // entries 0..5 in words 4..15, scanned from the top with selects (the
            // lowest hit is taken last): no branches.  Unused entries are zero words,
            // and no u is below a zero threshold.
#pragma unroll
            for (int m = 5; m >= 0; --m) {
                const bool hit = u < e[4 + 2 * m];
                next_line = hit ? e[5 + 2 * m] : next_line;
                found = found || hit;
            }
        } else {
            // the first of the (up to twelve) summarised lines whose last threshold
            // exceeds u holds the entry; beyond twelve lines, scan on from line 13
            const uint32_t L = (deg + 7) / 8;
            uint32_t lh = 0;
#pragma unroll
            for (int i = 11; i >= 0; --i) {  // summaries past the last line are zero
                const bool h = u < e[4 + i];
                lh = h ? (uint32_t)(i + 1) : lh;
            }
            for (uint32_t l = lh ? lh : (L > 12 ? 13u : 0u); l != 0 && l <= L && !found; ++l) {
                const uint4* lp = recs + ((size_t)(cline + l) * 4);
                const uint4 x0 = lp[0], x1 = lp[1], x2 = lp[2], x3 = lp[3];
                const uint32_t f[16] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w,
                                        x2.x, x2.y, x2.z, x2.w, x3.x, x3.y, x3.z, x3.w};
                uint32_t nl = 0;
                bool hit_any = false;
#pragma unroll
                for (int i = 7; i >= 0; --i) {  // entries past the last are zero words
                    const bool hit = u < f[2 * i];
                    nl = hit ? f[2 * i + 1] : nl;
                    hit_any = hit_any || hit;
                }
                next_line = hit_any ? nl : next_line;
                found = hit_any;
            }
        }
        // past every threshold: to ground if v is grounded, else (rounding) to the
        // last neighbour; the grounded lane still loads that neighbour's line, which
        // keeps the load below unconditional
        const bool to_ground = !found && (r0.y & DESC_GROUNDED) != 0;
        if (!found) next_line = e[3];
        if constexpr (BUCKETS) {
            // the line word: a bucketed target's bucket line for the next draw (q0),
            // else its first line
            const uint32_t kb = next_line >> LINE_KB_SHIFT;
            const uint32_t base = next_line & LINE_MASK;
            next_line = kb == 0u ? base : base + (q0 >> (32u - kb));
        }
        if (LOCK && !active) next_line = 0;
        const uint4* lp = recs + (size_t)next_line * 4;
        r0 = lp[0];
        r1 = lp[1];
        r2 = lp[2];
        r3 = lp[3];
        cline = next_line;
        if (LOCK && pend) {  // the previous iteration's finished walk, behind this load
            a.rec_end[pend_rec] = pend_end;
            a.rec_vis[pend_rec] = pend_vis;
            a.rec_len[pend_rec] = pend_len;
            pend = false;
        }
        // home: a node ranked below the row (the first step only reaches higher ranks)
        bool fin = to_ground || r0.x < rank_k;
        uint32_t endv = to_ground ? END_GROUND : r0.z;
        visits += (!fin && r0.x == rank_k);
        if constexpr (REUSE) {
            const uint32_t l = (uint32_t)t + 2;  // position of the node just reached
            bool below = to_ground || r0.x < top_rank;
            bool empty = false;
            while (below) {
                emit_walks(a, l > top_pos + 1, top_node, endv, top_vis, l - top_pos, blk_next,
                           blk_end);
                if (depth == 0) {
                    empty = true;
                    break;
                }
                --depth;
                const uint4 e = my_stack[depth];
                top_rank = e.x;
                top_node = e.y;
                top_pos = e.z;
                top_vis = e.w;
                below = to_ground || r0.x < top_rank;
            }
            if (!empty) {
                if (r0.x > top_rank) {
                    if (depth == a.stack_depth) {
                        atomicOr(a.err, ERR_STACK);
                        fin = true;
                    } else {
                        my_stack[depth] = make_uint4(top_rank, top_node, top_pos, top_vis);
                        ++depth;
                        top_rank = r0.x;
                        top_node = r0.z;
                        top_pos = l;
                        top_vis = 1;
                    }
                } else {
                    ++top_vis;
                }
            }
        }
        ++t;
        if (LOCK && !active) fin = false;  // an idle lane keeps nothing
        if (!fin && active && t >= a.max_steps) {
            fin = true;
            endv = END_LIMIT;
            atomicOr(a.err, ERR_LIMIT);
        }
        if (fin) {
            if constexpr (REUSE) {
                steps_acc += t;
            } else if constexpr (LOCK) {
                pend = true;
                pend_rec = rec;
                pend_end = endv;
                pend_vis = visits;
                pend_len = (uint32_t)t;
            } else {
                a.rec_end[rec] = endv;
                a.rec_vis[rec] = visits;
                a.rec_len[rec] = (uint32_t)t;
            }
            active = false;
        }
        }  // active
        if constexpr (REUSE) {  // lanes that emitted moved the block on: agree again
            blk_next = wave_max_u64(blk_next);
            blk_end = wave_max_u64(blk_end);
        }
    }
    if constexpr (REUSE) {
        for (uint64_t q = blk_next + lane; q < blk_end; q += 64)
            if (q < a.out_cap) a.out_key[q] = ~0ull;
    }
    if (pend) {  // LOCK: the last finished walk of the lane
        a.rec_end[pend_rec] = pend_end;
        a.rec_vis[pend_rec] = pend_vis;
        a.rec_len[pend_rec] = pend_len;
    }
    degsum = wave_sum(degsum);
    if (lane == 0 && degsum) atomicAdd(a.deg_sum, (unsigned long long)degsum);
    if constexpr (REUSE) {
        steps_acc = wave_sum(steps_acc);
        if (lane == 0 && steps_acc) atomicAdd(a.steps_sum, (unsigned long long)steps_acc);
    }
}

// BUCKETS: some records have bucket lines (line words carry bucket exponents)
template <int R, bool BUCKETS>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(SRW_WALK_WAVES))) void k_walk(WalkArgs a)
{
    walk_body<R, false, BUCKETS>(a, a.recs);
}

// The same walks with the records staged in LDS: for a table of at most the LDS a
// workgroup can hold (a.lds_lines lines of 64 bytes, walk and start records), every
// workgroup first copies it, and each step then reads LDS instead of the caches.
template <bool BUCKETS>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(SRW_WALK_WAVES))) void k_walk_lds(WalkArgs a)
{
    extern __shared__ uint4 table[];
    const int64_t words = (int64_t)a.lds_lines * 4;
    for (int64_t i = threadIdx.x; i < words; i += BLOCK) table[i] = a.recs[i];
    __syncthreads();
    walk_body<8, false, BUCKETS>(a, table);
}

// walk reuse keeps the stack top in registers as well: a larger register budget
template <bool BUCKETS>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_walk_reuse(WalkArgs a)
{
    walk_body<8, true, BUCKETS>(a, a.recs);
}
