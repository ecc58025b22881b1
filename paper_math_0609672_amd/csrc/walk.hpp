// Walk records and the walk kernel (Sections 2.1, 2.2.1 and 5.2).  Included by
// build.hip inside its anonymous namespace, after BLOCK and the schedule constants
// (NSLAB, NSEG) are defined.
#pragma once

// ----------------------------------------------------------------------- table
// Walk record of node v: 64-byte lines starting at line rline[v].  32-bit words:
// [0] rank, [1] degree | grounded flag, [2] node id, [3] zero, then for off-diagonal
// entry m (CSR order) a threshold floor(2^32 c_m / a_v) and the line of the
// neighbour's record: words 4 + 2m, 5 + 2m for m < 6 in the first line, and eight
// pairs per further line.  A node of degree <= 6 fits one line, so a walk step is one
// dependent 64-byte load: the next node's record, whose header holds the rank for the
// home test and the node id to record where the walk ends.
// Start descriptor (read once per walk): x = record line, y = first off-diagonal
// entry (index into the first-step thresholds), z = rank, w = degree | grounded; the
// index of the last higher-ranked neighbour goes to lastm[v].
constexpr int REC_WORDS = 16;

__global__ void k_rec_lines(int64_t n, const int64_t* __restrict__ rowptr, int32_t* lines)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) lines[v] = (int32_t)((rowptr[v + 1] - rowptr[v] - 1 + 9) / 8);
}

__global__ void k_table(int64_t n, const int64_t* __restrict__ rowptr,
                        const int32_t* __restrict__ col, const double* __restrict__ val,
                        const int32_t* __restrict__ rank, const uint8_t* __restrict__ grounded,
                        int32_t walks_per_row, const int32_t* __restrict__ budget_in,
                        const int64_t* __restrict__ rline, uint32_t* __restrict__ recs,
                        uint2* __restrict__ ent, uint32_t* __restrict__ mthr,
                        uint4* __restrict__ desc, uint32_t* __restrict__ lastm,
                        double* __restrict__ tau, int32_t* __restrict__ budget,
                        int32_t* max_budget)
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
    uint32_t* rec = recs + (size_t)rline[v] * REC_WORDS;
    double c = 0.0, cm = 0.0;
    uint32_t m = 0, last_motel = 0;
    for (int64_t p = r0; p < r1; ++p) {
        const int32_t j = col[p];
        if (j == v) continue;
        const double w = -val[p];
        c = c + w;
        const bool is_motel = rank[j] > rv;
        if (is_motel) {
            cm = cm + w;
            last_motel = m;
        }
        const uint32_t thr = threshold32(c, a);
        const uint32_t slot = m < 6 ? 4 + 2 * m : 16 + 2 * (m - 6);
        rec[slot] = thr;
        rec[slot + 1] = (uint32_t)rline[j];
        if (ent) ent[start + m] = make_uint2((uint32_t)j, thr);
        mthr[start + m] = motel > 0.0 ? threshold32(cm, motel) : 0u;
        ++m;
    }
    const uint32_t flags = grounded[v] ? DESC_GROUNDED : 0u;
    rec[0] = (uint32_t)rv;
    rec[1] = m | flags;
    rec[2] = (uint32_t)v;
    rec[3] = 0;
    desc[v] = make_uint4((uint32_t)rline[v], (uint32_t)start, (uint32_t)rv, m | flags);
    lastm[v] = last_motel;
    tau[v] = motel / a;
    int32_t b = 0;
    if (motel > 0.0) {
        b = budget_in ? budget_in[v] : walks_per_row;
        if (b < 1) b = 1;
        atomicMax(max_budget, b);
    }
    budget[v] = b;
}

// ----------------------------------------------------------------------- walks
struct WalkArgs {
    const uint4* desc;
    const uint32_t* lastm;
    const uint4* recs;         // walk records, 4 x 16 bytes per line
    const uint32_t* mthr;
    const uint2* chunks;       // chunk descriptors
    const int64_t* bounds;     // NSEG + 1 segment starts
    const int64_t* rec_off;
    uint64_t seed;
    // batched build: matrix of every node, first node of every matrix and its seed;
    // a walk's draws are keyed by its start node's id within its matrix and that seed
    const int32_t* node_mat;
    const int64_t* mat_off;
    const uint64_t* mat_seed;
    uint64_t max_steps;
    uint32_t* rec_end;
    uint32_t* rec_vis;
    uint32_t* rec_len;
    unsigned long long* queue;
    unsigned long long* deg_sum;
    int* err;
};

// Persistent walk kernel.  Every wave owns up to 64 walks at a time, one per lane.
// Every R steps the idle lanes of a wave take the next walks of the current chunk
// (up to 64 walks of one row); an exhausted chunk is replaced by the next one from
// the segment queues: the long-walk segment first, then the wave's own slab (by the
// XCD its workgroup runs on), then the other slabs in turn.  A lane's draws come from
// the Philox block of its (row, walk, step div 8), generated when step mod 8 = 0.
#ifndef SRW_WALK_WAVES
#define SRW_WALK_WAVES 6  // waves per SIMD the register budget is cut for
#endif
template <int R, bool BATCH>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(SRW_WALK_WAVES))) void k_walk(WalkArgs a)
{
    const int lane = __lane_id();
    const uint64_t lt = lanemask_lt();
    // wave-uniform chunk state
    uint32_t c_row = 0, c_next = 0, c_end = 0;
    bool done = false;
    const int home = 1 + (int)(blockIdx.x % NSLAB);
    int seg = 0, tried = 0;
    // per-lane walk state
    bool active = false;
    uint32_t k = 0, w = 0, visits = 0, rank_k = 0, last_motel = 0;
    uint32_t kline = 0, kstart = 0, kdeg = 0;  // start node: record line, entries, degree
    uint32_t cline = 0;                        // current node's record line
    uint4 r0 = make_uint4(0, 0, 0, 0), r1 = r0, r2 = r0, r3 = r0;  // its first line
    uint64_t t = 0, rec = 0, degsum = 0;
    uint32_t kkey = 0;       // BATCH: start node id within its matrix
    uint64_t seedw = 0;      // BATCH: its matrix's seed
    uint32_t q0 = 0, q1 = 0, q2 = 0, q3 = 0, q4 = 0, q5 = 0, q6 = 0, q7 = 0;

    for (uint32_t iter = 0;; ++iter) {
        if ((iter % R) == 0 && !done) {
            uint64_t idle = ballot(!active);
            while (idle != 0) {
                if (c_next >= c_end) {
                    // next chunk: long segment, then home slab, then the other slabs
                    bool got = false;
                    unsigned long long cidx = 0;
                    while (!done && !got) {
                        const int sq = seg == 0 ? 0 : 1 + (home - 1 + tried) % NSLAB;
                        const unsigned long long size =
                            (unsigned long long)(a.bounds[sq + 1] - a.bounds[sq]);
                        const unsigned long long c =
                            lane0_u64(atomicAdd(&a.queue[sq], lane == 0 ? 1ull : 0ull));
                        if (c < size) {
                            got = true;
                            cidx = (unsigned long long)a.bounds[sq] + c;
                        } else if (seg == 0) {
                            seg = 1;
                        } else if (++tried >= NSLAB) {
                            done = true;
                        }
                    }
                    if (done) break;
                    const uint2 cd = a.chunks[cidx];
                    c_row = cd.x;
                    c_next = cd.y & 0xFFFFu;
                    c_end = c_next + (cd.y >> 16);
                }
                const uint32_t avail = c_end - c_next;
                const uint32_t pos = (uint32_t)__popcll(idle & lt);
                const bool take = ((idle >> lane) & 1ull) && pos < avail;
                if (take) {
                    k = c_row;
                    w = c_next + pos;
                    t = 0;
                    visits = 1;
                    active = true;
                    const uint4 dk = a.desc[k];
                    kline = dk.x;
                    kstart = dk.y;
                    rank_k = dk.z;
                    kdeg = dk.w & DESC_DEG_MASK;
                    last_motel = a.lastm[k];
                    rec = (uint64_t)a.rec_off[k] + w;
                    if constexpr (BATCH) {
                        const int32_t mi = a.node_mat[k];
                        kkey = k - (uint32_t)a.mat_off[mi];
                        seedw = a.mat_seed[mi];
                    }
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
        if (active) {  // structured: the lanes rejoin before the next refill's ballots
        if ((t & 7) == 0) {
            const u64x4 b = BATCH ? philox4x64_10(t >> 3, w, kkey, STREAM_WALK, seedw, 0)
                                  : philox4x64_10(t >> 3, w, k, STREAM_WALK, a.seed, 0);
            q0 = (uint32_t)b.x0; q1 = (uint32_t)(b.x0 >> 32);
            q2 = (uint32_t)b.x1; q3 = (uint32_t)(b.x1 >> 32);
            q4 = (uint32_t)b.x2; q5 = (uint32_t)(b.x2 >> 32);
            q6 = (uint32_t)b.x3; q7 = (uint32_t)(b.x3 >> 32);
        }
        const uint32_t u = q0;
        q0 = q1; q1 = q2; q2 = q3; q3 = q4; q4 = q5; q5 = q6; q6 = q7;

        uint32_t next_line = 0;
        bool to_ground = false;
        if (t == 0) {
            // first step: among higher-ranked neighbours of k (exact one-step part)
            degsum += kdeg;
            uint32_t sel = last_motel;
            for (uint32_t m = 0; m < kdeg; ++m)
                if (u < a.mthr[kstart + m]) {
                    sel = m;
                    break;
                }
            const uint32_t* kr = (const uint32_t*)a.recs + (size_t)kline * REC_WORDS;
            next_line = kr[sel < 6 ? 5 + 2 * sel : 17 + 2 * (sel - 6)];
        } else {
            const uint32_t deg = r0.y & DESC_DEG_MASK;
            degsum += deg;
            // The next node is the first entry m with u < threshold_m.  Entries 0..5
            // sit in the first line (words 4..15), held in registers; they are
            // scanned from the top with selects (the lowest hit is taken last), so
            // the scan has no branches.
            const uint32_t e[16] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w,
                                    r2.x, r2.y, r2.z, r2.w, r3.x, r3.y, r3.z, r3.w};
            uint32_t lastn = e[5];
#pragma unroll
            for (int m = 1; m < 6; ++m) lastn = (uint32_t)m < deg ? e[5 + 2 * m] : lastn;
            bool found = false;
#pragma unroll
            for (int m = 5; m >= 0; --m) {
                const bool hit = (uint32_t)m < deg && u < e[4 + 2 * m];
                next_line = hit ? e[5 + 2 * m] : next_line;
                found = found || hit;
            }
            // further lines of a node of degree > 6: 8 entries per line
            for (uint32_t m0 = 6, l = 1; !found && m0 < deg; m0 += 8, ++l) {
                const uint4* lp = a.recs + ((size_t)(cline + l) * 4);
                const uint4 x0 = lp[0], x1 = lp[1], x2 = lp[2], x3 = lp[3];
                const uint32_t f[16] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w,
                                        x2.x, x2.y, x2.z, x2.w, x3.x, x3.y, x3.z, x3.w};
                uint32_t nl = 0;
                bool hit_any = false;
#pragma unroll
                for (int i = 7; i >= 0; --i) {
                    const bool hit = m0 + i < deg && u < f[2 * i];
                    nl = hit ? f[2 * i + 1] : nl;
                    hit_any = hit_any || hit;
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) lastn = m0 + i < deg ? f[2 * i + 1] : lastn;
                next_line = hit_any ? nl : next_line;
                found = hit_any;
            }
            if (!found) {
                if (r0.y & DESC_GROUNDED) to_ground = true;
                else next_line = lastn;
            }
        }
        bool fin = false;
        uint32_t endv = 0;
        if (to_ground) {
            fin = true;
            endv = END_GROUND;
        } else {
            const uint4* lp = a.recs + (size_t)next_line * 4;
            const uint4 n0 = lp[0], n1 = lp[1], n2 = lp[2], n3 = lp[3];
            const uint32_t rank_next = n0.x;
            if (t > 0 && rank_next < rank_k) {
                fin = true;
                endv = n0.z;
            } else {
                visits += (rank_next == rank_k);
                cline = next_line;
                r0 = n0;
                r1 = n1;
                r2 = n2;
                r3 = n3;
            }
        }
        ++t;
        if (!fin && t >= a.max_steps) {
            fin = true;
            endv = END_LIMIT;
            atomicOr(a.err, ERR_LIMIT);
        }
        if (fin) {
            a.rec_end[rec] = endv;
            a.rec_vis[rec] = visits;
            a.rec_len[rec] = (uint32_t)t;
            active = false;
        }
        }  // active
    }
    degsum = wave_sum(degsum);
    if (lane == 0 && degsum) atomicAdd(a.deg_sum, (unsigned long long)degsum);
}
