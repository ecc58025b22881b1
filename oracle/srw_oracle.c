/*
 * srw_oracle.c -- plain, slow, FP64 CPU oracle of the random-walk incomplete
 * LDL^T preconditioner and its PCG solve, after H. Qian and S. S. Sapatnekar,
 * "Stochastic Preconditioning for Iterative Linear Equation Solvers" (SIAM).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code with the GPU library.
 *
 * Every step follows the paper in its own order and notation, one row and one
 * walk at a time, with no blocking or reordering:
 *   - the walk game of an R-matrix: transition probability -A_kj/A_kk, a path to
 *     ground with probability (sum_j A_kj)/A_kk (Section 2.1, eq. map);
 *   - "creating homes": walks from node k end at any node processed before k or at
 *     ground (Section 2.2.1); the processing order is a random ordering
 *     (Section 5.4);
 *   - tallies M_k, H_{k,i} and J_{k,k} (Section 3.1) collected with the exact
 *     one-step treatment: the first step is drawn among the not-yet-processed
 *     neighbours only (Section 5.2);
 *   - optionally, walk reuse: every walk also feeds the walks that Algorithm "reuse"
 *     extracts from it to the tallies of their start nodes (Section 5.3);
 *   - factor entries by eqs. newy and newz, the diagonal by eq. d (Sections 3.3 and
 *     5.2), then the optional drop of small entries (Section 4, footnote);
 *   - the hybrid solver: PCG with the preconditioner (L D L^T)^{-1} (Algorithm 1),
 *     stopped on ||b - Ax||_2 < tol ||b||_2 (Section 6);
 *   - asymmetric A (Section 7.1): the games of A and of A^T with one ordering give the
 *     LDU of rev(A) (eqs. y2, y3, d), the preconditioner of BiCGSTAB.
 *
 * Readings where the paper is silent (random-number generator, its key layout,
 * the uniform-to-neighbour map, ties, zero excess) are the library's documented
 * ones and are restated at each function.
 *
 * Parity status: every function here is pinned by a test against numpy's Philox,
 * dense elimination, closed forms or textbook solvers (see tests/test_oracle_*.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SRWO_OK 0
#define SRWO_NOT_CONVERGED 1
#define SRWO_E_ARG (-1)
#define SRWO_E_NOT_RMATRIX (-2)
#define SRWO_E_SINGULAR (-3)
#define SRWO_E_NOMEM (-5)

/* |e_k| <= EPS_EXCESS * A_kk counts as zero excess (no path to ground). */
static const double EPS_EXCESS = 1e-12;

/* ------------------------------------------------------------------------- */
/* Philox4x64-10 counter-based generator (Salmon, Moraes, Dror and Shaw,     */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).                   */
/* ------------------------------------------------------------------------- */
void srwo_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        unsigned __int128 p0 = (unsigned __int128)M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Stream identifiers in counter word 3. */
#define STREAM_WALK 0ULL
#define STREAM_ORDER 1ULL

/* The t-th 32-bit draw of walk w from row k: word (t mod 8) of the Philox block
 * with key (seed, 0) and counter (t div 8, w, k, STREAM_WALK); the low half of each
 * 64-bit output word comes first. */
uint32_t srwo_draw(uint64_t seed, int64_t k, int64_t w, uint64_t t)
{
    uint64_t ctr[4] = {t / 8, (uint64_t)w, (uint64_t)k, STREAM_WALK};
    uint64_t key[2] = {seed, 0};
    uint64_t out[4];
    srwo_philox4x64_10(ctr, key, out);
    uint64_t word = out[(t % 8) / 2];
    return (t % 2 == 0) ? (uint32_t)word : (uint32_t)(word >> 32);
}

/* ------------------------------------------------------------------------- */
/* Random ordering (Section 5.4: "random ordering is used").                */
/* ------------------------------------------------------------------------- */
typedef struct {
    uint64_t key;
    int64_t id;
} keyed_node;

static int cmp_keyed(const void* pa, const void* pb)
{
    const keyed_node* a = (const keyed_node*)pa;
    const keyed_node* b = (const keyed_node*)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->id != b->id) return a->id < b->id ? -1 : 1;
    return 0;
}

/* rank[v] = 0-based position of v when the nodes are sorted by (key_v, v), where
 * key_v is the first 64-bit word of Philox block (key (seed,0), counter
 * (0, 0, v, STREAM_ORDER)).  A lower rank is processed earlier, i.e. is a home for
 * the walks of every higher-ranked node. */
int srwo_rank(int64_t n, uint64_t seed, int32_t* rank)
{
    if (n < 0) return SRWO_E_ARG;
    keyed_node* nodes = (keyed_node*)malloc(sizeof(keyed_node) * (size_t)(n ? n : 1));
    if (!nodes) return SRWO_E_NOMEM;
    for (int64_t v = 0; v < n; v++) {
        uint64_t ctr[4] = {0, 0, (uint64_t)v, STREAM_ORDER};
        uint64_t key[2] = {seed, 0};
        uint64_t out[4];
        srwo_philox4x64_10(ctr, key, out);
        nodes[v].key = out[0];
        nodes[v].id = v;
    }
    qsort(nodes, (size_t)n, sizeof(keyed_node), cmp_keyed);
    for (int64_t p = 0; p < n; p++) rank[nodes[p].id] = (int32_t)p;
    free(nodes);
    return SRWO_OK;
}

/* ------------------------------------------------------------------------- */
/* R-matrix check (Section 1 definition; game construction of Section 2.1). */
/* ------------------------------------------------------------------------- */
static int64_t uf_find(int64_t* parent, int64_t v)
{
    while (parent[v] != v) {
        parent[v] = parent[parent[v]];
        v = parent[v];
    }
    return v;
}

/* Returns SRWO_OK, SRWO_E_ARG (malformed CSR), SRWO_E_NOT_RMATRIX (a non-positive
 * diagonal, a stored off-diagonal entry that is not negative, asymmetry, or a
 * negative excess e_k = A_kk - sum_j |A_kj| < -EPS_EXCESS*A_kk), or SRWO_E_SINGULAR
 * (a connected component without any node of positive excess: the game on it never
 * ends and A is singular). */
int srwo_validate(int64_t n, const int64_t* rowptr, const int32_t* col, const double* val)
{
    if (n < 0 || rowptr[0] != 0) return SRWO_E_ARG;
    /* structure first: monotone row pointers, sorted in-range columns, one diagonal */
    for (int64_t k = 0; k < n; k++) {
        if (rowptr[k + 1] < rowptr[k]) return SRWO_E_ARG;
        int ndiag = 0;
        for (int64_t p = rowptr[k]; p < rowptr[k + 1]; p++) {
            int32_t j = col[p];
            if (j < 0 || j >= n) return SRWO_E_ARG;
            if (p > rowptr[k] && col[p - 1] >= j) return SRWO_E_ARG;
            if (j == k) ndiag++;
        }
        if (ndiag != 1) return SRWO_E_ARG;
    }
    for (int64_t k = 0; k < n; k++) {
        double a = 0.0, sum_w = 0.0;
        for (int64_t p = rowptr[k]; p < rowptr[k + 1]; p++)
            if (col[p] == k) a = val[p];
        if (!(a > 0.0)) return SRWO_E_NOT_RMATRIX;
        for (int64_t p = rowptr[k]; p < rowptr[k + 1]; p++) {
            int32_t j = col[p];
            if (j == k) continue;
            if (!(val[p] < 0.0)) return SRWO_E_NOT_RMATRIX;
            sum_w = sum_w + (-val[p]);
            /* symmetry: A_jk must be stored with the same value */
            int64_t lo = rowptr[j], hi = rowptr[j + 1] - 1, found = -1;
            while (lo <= hi) {
                int64_t mid = lo + (hi - lo) / 2;
                if (col[mid] == k) { found = mid; break; }
                if (col[mid] < k) lo = mid + 1; else hi = mid - 1;
            }
            if (found < 0 || val[found] != val[p]) return SRWO_E_NOT_RMATRIX;
        }
        double e = a - sum_w;
        if (e < -EPS_EXCESS * a) return SRWO_E_NOT_RMATRIX;
    }
    /* every connected component needs a path to ground */
    int64_t* parent = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    unsigned char* grounded = (unsigned char*)calloc((size_t)(n ? n : 1), 1);
    if (!parent || !grounded) { free(parent); free(grounded); return SRWO_E_NOMEM; }
    for (int64_t v = 0; v < n; v++) parent[v] = v;
    for (int64_t k = 0; k < n; k++)
        for (int64_t p = rowptr[k]; p < rowptr[k + 1]; p++) {
            int64_t ra = uf_find(parent, k), rb = uf_find(parent, col[p]);
            if (ra != rb) parent[ra > rb ? ra : rb] = ra < rb ? ra : rb;
        }
    for (int64_t k = 0; k < n; k++) {
        double a = 0.0, sum_w = 0.0;
        for (int64_t p = rowptr[k]; p < rowptr[k + 1]; p++) {
            if (col[p] == k) a = val[p]; else sum_w = sum_w + (-val[p]);
        }
        if (a - sum_w > EPS_EXCESS * a) grounded[uf_find(parent, k)] = 1;
    }
    int status = SRWO_OK;
    for (int64_t v = 0; v < n; v++)
        if (uf_find(parent, v) == v && !grounded[v]) status = SRWO_E_SINGULAR;
    free(parent);
    free(grounded);
    return status;
}

/* ------------------------------------------------------------------------- */
/* The game of Section 2.1 as integer thresholds.                            */
/* ------------------------------------------------------------------------- */

/* floor((c / d) * 2^32), clamped to [0, 2^32 - 1].  Scaling by 2^32 is exact, so
 * only the division rounds. */
static uint32_t threshold(double c, double d)
{
    double x = (c / d) * 4294967296.0;
    if (x >= 4294967295.0) return 0xFFFFFFFFu;
    if (x <= 0.0) return 0u;
    return (uint32_t)floor(x);
}

/* Transition table of every row v, over its off-diagonal entries in CSR column
 * order m = 0..deg-1 (off-diagonal entry index q = rowptr[v] - v + m):
 *   nbr[q]      neighbour j_m;
 *   thr[q]      floor(2^32 * c_m / a_v), c_m = w_1 + ... + w_m summed in order,
 *               w = -A_vj: a draw u selects the first m with u < thr[q]; if there is
 *               none the walk goes to ground when v is grounded, else to j_deg;
 *   mthr[q]     the same over the motel neighbours of v only (rank[j] > rank[v]),
 *               normalised by S_v = their total weight; zero width elsewhere;
 *               if no entry qualifies the last motel is taken;
 *   tau[v]      S_v / a_v, the probability that the first step reaches a motel
 *               (the factor (sum_{j>k} A_kj)/A_kk of eqs. newy and newz, negated);
 *   grounded[v] e_v = a_v - c_deg > EPS_EXCESS * a_v;
 *   diag[v]     a_v. */
int srwo_table(int64_t n, const int64_t* rowptr, const int32_t* col, const double* val,
               const int32_t* rank, int32_t* nbr, uint32_t* thr, uint32_t* mthr,
               double* tau, unsigned char* grounded, double* diag)
{
    for (int64_t v = 0; v < n; v++) {
        double a = 0.0;
        for (int64_t p = rowptr[v]; p < rowptr[v + 1]; p++)
            if (col[p] == v) a = val[p];
        double motel_mass = 0.0;
        for (int64_t p = rowptr[v]; p < rowptr[v + 1]; p++)
            if (col[p] != v && rank[col[p]] > rank[v]) motel_mass = motel_mass + (-val[p]);
        int64_t q = rowptr[v] - v;
        double c = 0.0, cm = 0.0;
        for (int64_t p = rowptr[v]; p < rowptr[v + 1]; p++) {
            int32_t j = col[p];
            if (j == v) continue;
            double w = -val[p];
            c = c + w;
            if (rank[j] > rank[v]) cm = cm + w;
            nbr[q] = j;
            thr[q] = threshold(c, a);
            mthr[q] = motel_mass > 0.0 ? threshold(cm, motel_mass) : 0u;
            q++;
        }
        double e = a - c;
        grounded[v] = (e > EPS_EXCESS * a) ? 1 : 0;
        tau[v] = motel_mass / a;
        diag[v] = a;
    }
    return SRWO_OK;
}

/* ------------------------------------------------------------------------- */
/* Walks with rank homes and the exact one-step treatment (Sections 2.2.1,  */
/* 5.2).                                                                     */
/* ------------------------------------------------------------------------- */

/* Simulates walk w of row k (tau[k] > 0).  Step t = 0 moves from k to a motel
 * neighbour (first-step rule); each later step moves from the current node by the
 * full rule.  The walk ends when it steps to ground (end = -1) or to a node of lower
 * rank than k (end = that node).  visits counts the walker's stays at k, the start
 * included; length is the number of steps taken. */
void srwo_walk(int64_t n, const int64_t* rowptr, const int32_t* nbr, const uint32_t* thr,
               const uint32_t* mthr, const unsigned char* grounded, const int32_t* rank,
               uint64_t seed, int64_t k, int64_t w,
               int32_t* end_out, uint32_t* visits_out, uint32_t* length_out)
{
    (void)n;
    /* first step: among motel neighbours of k */
    int64_t base = rowptr[k] - k;
    int64_t deg = rowptr[k + 1] - rowptr[k] - 1;
    uint32_t u = srwo_draw(seed, k, w, 0);
    int64_t chosen = -1, last_motel = -1;
    for (int64_t m = 0; m < deg; m++) {
        if (rank[nbr[base + m]] > rank[k]) last_motel = m;
        if (chosen < 0 && u < mthr[base + m]) chosen = m;
    }
    if (chosen < 0) chosen = last_motel;
    int64_t cur = nbr[base + chosen];
    uint32_t visits = 1;
    for (uint64_t t = 1;; t++) {
        u = srwo_draw(seed, k, w, t);
        base = rowptr[cur] - cur;
        deg = rowptr[cur + 1] - rowptr[cur] - 1;
        int64_t next = -2;
        for (int64_t m = 0; m < deg; m++)
            if (u < thr[base + m]) { next = nbr[base + m]; break; }
        if (next == -2) next = grounded[cur] ? -1 : nbr[base + deg - 1];
        if (next == -1) {
            *end_out = -1; *visits_out = visits; *length_out = (uint32_t)(t + 1);
            return;
        }
        if (rank[next] < rank[k]) {
            *end_out = (int32_t)next; *visits_out = visits; *length_out = (uint32_t)(t + 1);
            return;
        }
        if (next == k) visits++;
        cur = next;
    }
}

/* Runs the walks of a list of rows.  For list entry r (row rows[r]) walks
 * w = 0..budget[r]-1 are simulated when tau[row] > 0 (rows with tau = 0 are exact
 * and run none); their records go to [rec_off[r], rec_off[r] + budget[r]) of the
 * output arrays. */
int srwo_walk_rows(int64_t n, const int64_t* rowptr, const int32_t* nbr, const uint32_t* thr,
                   const uint32_t* mthr, const double* tau, const unsigned char* grounded,
                   const int32_t* rank, uint64_t seed, int64_t nrows, const int64_t* rows,
                   const int32_t* budget, const int64_t* rec_off,
                   int32_t* end, uint32_t* visits, uint32_t* length)
{
    for (int64_t r = 0; r < nrows; r++) {
        int64_t k = rows[r];
        if (k < 0 || k >= n) return SRWO_E_ARG;
        if (!(tau[k] > 0.0)) continue;
        for (int64_t w = 0; w < budget[r]; w++)
            srwo_walk(n, rowptr, nbr, thr, mthr, grounded, rank, seed, k, w,
                      &end[rec_off[r] + w], &visits[rec_off[r] + w], &length[rec_off[r] + w]);
    }
    return SRWO_OK;
}

/* ------------------------------------------------------------------------- */
/* Walk reuse (Section 5.3, Algorithm "reuse").                              */
/* ------------------------------------------------------------------------- */

/* One walk counted in the tallies: its start node (the row it belongs to), end node
 * (-1 = ground), stays at the start (start included) and number of steps. */
typedef struct {
    int32_t row, end;
    uint32_t visits, length;
} srwo_rec;

typedef struct {
    srwo_rec* r;
    int64_t n, cap;
} srwo_recs;

static int recs_push(srwo_recs* o, int32_t row, int32_t end, uint32_t visits, uint32_t length)
{
    if (o->n == o->cap) {
        int64_t c = o->cap ? 2 * o->cap : 64;
        srwo_rec* q = (srwo_rec*)realloc(o->r, sizeof(srwo_rec) * (size_t)c);
        if (!q) return SRWO_E_NOMEM;
        o->r = q;
        o->cap = c;
    }
    o->r[o->n].row = row;
    o->r[o->n].end = end;
    o->r[o->n].visits = visits;
    o->r[o->n].length = length;
    o->n++;
    return SRWO_OK;
}

/* The two stacks of the algorithm: stack1 holds node keys (position in the
 * ordering; ground is below every node), stack2 the positions l at which they were
 * pushed (the start is position 1).  `node` and `visits` ride along with each entry:
 * the node id (for the records) and the stays at that node while it is the top (the
 * J_{k',k'} increments of the algorithm, start included). */
typedef struct {
    int64_t* key;
    int64_t* pos;
    int32_t* node;
    uint32_t* visits;
    int64_t top, cap;  /* top = number of entries */
} srwo_stacks;

static int stacks_push(srwo_stacks* s, int64_t key, int64_t pos, int32_t node)
{
    if (s->top == s->cap) {
        int64_t c = s->cap ? 2 * s->cap : 16;
        int64_t* k = (int64_t*)realloc(s->key, sizeof(int64_t) * (size_t)c);
        if (!k) return SRWO_E_NOMEM;
        s->key = k;
        int64_t* p = (int64_t*)realloc(s->pos, sizeof(int64_t) * (size_t)c);
        if (!p) return SRWO_E_NOMEM;
        s->pos = p;
        int32_t* nd = (int32_t*)realloc(s->node, sizeof(int32_t) * (size_t)c);
        if (!nd) return SRWO_E_NOMEM;
        s->node = nd;
        uint32_t* v = (uint32_t*)realloc(s->visits, sizeof(uint32_t) * (size_t)c);
        if (!v) return SRWO_E_NOMEM;
        s->visits = v;
        s->cap = c;
    }
    s->key[s->top] = key;
    s->pos[s->top] = pos;
    s->node[s->top] = node;
    s->visits[s->top] = 1;
    s->top++;
    return SRWO_OK;
}

static void stacks_free(srwo_stacks* s)
{
    free(s->key);
    free(s->pos);
    free(s->node);
    free(s->visits);
}

/* Position l of the walk holds node `node` with key `key`.  While key is below the
 * top of stack1, the top is popped; if the top was pushed more than one position
 * before l, the segment from it to l is a legal walk of at least two steps: M, H
 * and J of its start node take it (one record).  Then key is pushed if it is above
 * the new top, else (equal) it is a stay at the top's node.  Returns the number of
 * entries left (0 once the walk has dropped below its start). */
static int reuse_position(srwo_stacks* s, int64_t l, int64_t key, int32_t node, srwo_recs* out,
                          int* err)
{
    while (s->top > 0 && key < s->key[s->top - 1]) {
        const int64_t t = s->top - 1;
        if (l > s->pos[t] + 1) {
            int e = recs_push(out, s->node[t], node, s->visits[t], (uint32_t)(l - s->pos[t]));
            if (e) *err = e;
        }
        s->top--;
    }
    if (s->top == 0) return 0;
    if (key > s->key[s->top - 1]) {
        int e = stacks_push(s, key, l, node);
        if (e) *err = e;
    } else {
        s->visits[s->top - 1]++;
    }
    return (int)s->top;
}

/* Algorithm "reuse" on a given legal sequence: positions 1..len hold nodes node[i]
 * with keys key[i] (i = 0..len-1; ground as key -1, node -1).  Writes the records of
 * every walk the algorithm counts, in the order it counts them, to rows/ends/visits/
 * lengths (capacity cap) and returns their number, or a negative status. */
int64_t srwo_reuse_sequence(int64_t len, const int64_t* key, const int32_t* node, int64_t cap,
                            int32_t* rows, int32_t* ends, uint32_t* visits, uint32_t* lengths)
{
    if (len < 1) return 0;
    srwo_stacks st = {0};
    srwo_recs out = {0};
    int err = stacks_push(&st, key[0], 1, node[0]);
    for (int64_t i = 1; i < len && !err; i++)
        if (reuse_position(&st, i + 1, key[i], node[i], &out, &err) == 0) break;
    stacks_free(&st);
    if (err) {
        free(out.r);
        return err;
    }
    int64_t n = out.n;
    if (n > cap) n = cap;
    for (int64_t i = 0; i < n; i++) {
        rows[i] = out.r[i].row;
        ends[i] = out.r[i].end;
        visits[i] = out.r[i].visits;
        lengths[i] = out.r[i].length;
    }
    n = out.n;
    free(out.r);
    return n;
}

/* Walk w of row k as in srwo_walk, fed position by position (the start is position
 * 1, the node reached by step t is position t + 2) to the two stacks, with the rank
 * as key: the walk itself and every walk extracted from it go to `out`. */
static int srwo_walk_reuse(const int64_t* rowptr, const int32_t* nbr, const uint32_t* thr,
                           const uint32_t* mthr, const unsigned char* grounded,
                           const int32_t* rank, uint64_t seed, int64_t k, int64_t w,
                           srwo_stacks* st, srwo_recs* out)
{
    int err = SRWO_OK;
    st->top = 0;
    err = stacks_push(st, rank[k], 1, (int32_t)k);
    if (err) return err;
    /* first step: among motel neighbours of k (always a higher rank) */
    int64_t base = rowptr[k] - k;
    int64_t deg = rowptr[k + 1] - rowptr[k] - 1;
    uint32_t u = srwo_draw(seed, k, w, 0);
    int64_t chosen = -1, last_motel = -1;
    for (int64_t m = 0; m < deg; m++) {
        if (rank[nbr[base + m]] > rank[k]) last_motel = m;
        if (chosen < 0 && u < mthr[base + m]) chosen = m;
    }
    if (chosen < 0) chosen = last_motel;
    int64_t cur = nbr[base + chosen];
    reuse_position(st, 2, rank[cur], (int32_t)cur, out, &err);
    for (uint64_t t = 1; !err; t++) {
        u = srwo_draw(seed, k, w, t);
        base = rowptr[cur] - cur;
        deg = rowptr[cur + 1] - rowptr[cur] - 1;
        int64_t next = -2;
        for (int64_t m = 0; m < deg; m++)
            if (u < thr[base + m]) { next = nbr[base + m]; break; }
        if (next == -2) next = grounded[cur] ? -1 : nbr[base + deg - 1];
        const int64_t key = next < 0 ? -1 : rank[next];
        if (reuse_position(st, (int64_t)t + 2, key, (int32_t)next, out, &err) == 0) break;
        cur = next;
    }
    return err;
}

/* The walks of a list of rows (as srwo_walk_rows) with walk reuse: returns the
 * number of records (each walk simulated plus each walk extracted from one) and
 * hands the record array to the caller through *recs (free with srwo_free), or a
 * negative status. */
int64_t srwo_walk_rows_reuse(int64_t n, const int64_t* rowptr, const int32_t* nbr,
                             const uint32_t* thr, const uint32_t* mthr, const double* tau,
                             const unsigned char* grounded, const int32_t* rank, uint64_t seed,
                             int64_t nrows, const int64_t* rows, const int32_t* budget,
                             int32_t** rec_rows, int32_t** rec_ends, uint32_t** rec_visits,
                             uint32_t** rec_lengths)
{
    srwo_stacks st = {0};
    srwo_recs out = {0};
    int err = SRWO_OK;
    for (int64_t r = 0; r < nrows && !err; r++) {
        int64_t k = rows[r];
        if (k < 0 || k >= n) { err = SRWO_E_ARG; break; }
        if (!(tau[k] > 0.0)) continue;
        for (int64_t w = 0; w < budget[r] && !err; w++)
            err = srwo_walk_reuse(rowptr, nbr, thr, mthr, grounded, rank, seed, k, w, &st, &out);
    }
    stacks_free(&st);
    if (err) {
        free(out.r);
        return err;
    }
    const int64_t m = out.n;
    const size_t cnt = (size_t)(m > 0 ? m : 1);
    int32_t* a = (int32_t*)malloc(sizeof(int32_t) * cnt);
    int32_t* b = (int32_t*)malloc(sizeof(int32_t) * cnt);
    uint32_t* c = (uint32_t*)malloc(sizeof(uint32_t) * cnt);
    uint32_t* d = (uint32_t*)malloc(sizeof(uint32_t) * cnt);
    if (!a || !b || !c || !d) {
        free(a); free(b); free(c); free(d); free(out.r);
        return SRWO_E_NOMEM;
    }
    for (int64_t i = 0; i < m; i++) {
        a[i] = out.r[i].row;
        b[i] = out.r[i].end;
        c[i] = out.r[i].visits;
        d[i] = out.r[i].length;
    }
    free(out.r);
    *rec_rows = a;
    *rec_ends = b;
    *rec_visits = c;
    *rec_lengths = d;
    return m;
}

void srwo_free(void* p) { free(p); }

/* ------------------------------------------------------------------------- */
/* Tallies (Section 3.1, reduced journey record of Section 3.1/3.3).         */
/* ------------------------------------------------------------------------- */
static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* For list entry r with m = count[r] walk records starting at rec_off[r]:
 *   walks[r]  = M'  (number of simulated walks, all of length >= 2),
 *   J[r]      = sum of visits (J_{k,k} restricted to those walks),
 *   G[r]      = number of walks that ended at ground,
 *   steps[r]  = total steps, visits_sq[r] = sum of visits^2,
 *   H list    = distinct end nodes (ascending id) with their counts H'_{k,i},
 *               written at [rec_off[r], rec_off[r] + hlen[r]). */
int srwo_tally_rows(int64_t nrows, const int32_t* count, const int64_t* rec_off,
                    const int32_t* end, const uint32_t* visits, const uint32_t* length,
                    uint32_t* walks, uint64_t* J, uint32_t* G, uint64_t* steps,
                    uint64_t* visits_sq, int32_t* hlen, int32_t* h_end, uint32_t* h_cnt)
{
    int32_t* buf = NULL;
    int64_t cap = 0;
    for (int64_t r = 0; r < nrows; r++) {
        int64_t m = count[r], off = rec_off[r];
        if (m > cap) {
            free(buf);
            buf = (int32_t*)malloc(sizeof(int32_t) * (size_t)m);
            if (!buf) return SRWO_E_NOMEM;
            cap = m;
        }
        uint64_t jsum = 0, ssum = 0, vsq = 0;
        uint32_t g = 0;
        int64_t nb = 0;
        for (int64_t i = 0; i < m; i++) {
            jsum += visits[off + i];
            ssum += length[off + i];
            vsq += (uint64_t)visits[off + i] * (uint64_t)visits[off + i];
            if (end[off + i] < 0) g++; else buf[nb++] = end[off + i];
        }
        qsort(buf, (size_t)nb, sizeof(int32_t), cmp_i32);
        int64_t h = 0;
        for (int64_t i = 0; i < nb; i++) {
            if (i > 0 && buf[i] == buf[i - 1]) {
                h_cnt[off + h - 1]++;
            } else {
                h_end[off + h] = buf[i];
                h_cnt[off + h] = 1;
                h++;
            }
        }
        walks[r] = (uint32_t)m; J[r] = jsum; G[r] = g; steps[r] = ssum; visits_sq[r] = vsq;
        hlen[r] = (int32_t)h;
    }
    free(buf);
    return SRWO_OK;
}

/* ------------------------------------------------------------------------- */
/* Factor entries (eqs. newy, newz, d) and the drop (Section 4 footnote).    */
/* ------------------------------------------------------------------------- */

/* Row k of the factor from its tallies.  With a = A_kk, w_ki = -A_ki, tau = tau[k],
 * M = walks, H = H'_{k,i}, J = J'_k (walks of length >= 2 only):
 *   eq. newy:  Y_ki = A_ki/A_kk + (sum_{j motel} A_kj / A_kk) * H/M
 *                   = -( w_ki/a + tau * (H/M) ),
 *              for i a lower-ranked neighbour or an end node (first term 0 when i is
 *              not a neighbour, second 0 when no walk ended at i);
 *   eqs. newz and d:  D_k = 1/Z_kk = a / (1 + tau * (J/M - 1)).
 * Rows with tau = 0 have no walks: Y_ki = -w_ki/a and D_k = a (exact, Section 5.2).
 * Entries with |Y_ki| < drop_tol are dropped.  Entries come out in ascending column
 * id.  With out_col == NULL only the number of kept entries is returned in *nnz. */
void srwo_factor_row(int64_t k, const int64_t* rowptr, const int32_t* col, const double* val,
                     const int32_t* rank, double tau, uint32_t walks, uint64_t J,
                     int32_t hlen, const int32_t* h_end, const uint32_t* h_cnt,
                     double drop_tol, int32_t* out_col, double* out_val, int64_t* nnz,
                     double* d_out)
{
    double a = 0.0;
    for (int64_t p = rowptr[k]; p < rowptr[k + 1]; p++)
        if (col[p] == k) a = val[p];
    int64_t p = rowptr[k], pe = rowptr[k + 1];
    int32_t h = 0;
    int64_t kept = 0;
    while (1) {
        /* next lower-ranked neighbour */
        while (p < pe && (col[p] == k || rank[col[p]] > rank[k])) p++;
        int32_t ci = p < pe ? col[p] : INT32_MAX;
        int32_t ch = h < hlen ? h_end[h] : INT32_MAX;
        if (ci == INT32_MAX && ch == INT32_MAX) break;
        int32_t i = ci < ch ? ci : ch;
        double w = 0.0;
        uint32_t cnt = 0;
        if (ci == i) { w = -val[p]; p++; }
        if (ch == i) { cnt = h_cnt[h]; h++; }
        double hfrac = walks > 0 ? (double)cnt / (double)walks : 0.0;
        double y = -((w / a) + (tau * hfrac));
        if (!(fabs(y) < drop_tol)) {
            if (out_col) { out_col[kept] = i; out_val[kept] = y; }
            kept++;
        }
    }
    *nnz = kept;
    if (walks > 0) {
        double mbar = (double)J / (double)walks;
        *d_out = a / (1.0 + tau * (mbar - 1.0));
    } else {
        *d_out = a;
    }
}

/* The whole factor, row by row with srwo_factor_row.  Tallies are indexed by node
 * (walks[k] = 0 for rows without walks); the H list of row k sits at
 * [h_off[k], h_off[k] + hlen[k]).  First call with ycol == NULL fills yptr (n+1
 * row pointers); second call with the arrays sized yptr[n] fills ycol, yval and d. */
int srwo_factor(int64_t n, const int64_t* rowptr, const int32_t* col, const double* val,
                const int32_t* rank, const double* tau, const uint32_t* walks,
                const uint64_t* J, const int64_t* h_off, const int32_t* hlen,
                const int32_t* h_end, const uint32_t* h_cnt, double drop_tol,
                int64_t* yptr, int32_t* ycol, double* yval, double* d)
{
    if (!ycol) yptr[0] = 0;
    for (int64_t k = 0; k < n; k++) {
        int64_t nnz = 0;
        double dk = 0.0;
        srwo_factor_row(k, rowptr, col, val, rank, tau[k], walks[k], J[k], hlen[k],
                        h_end + h_off[k], h_cnt + h_off[k], drop_tol,
                        ycol ? ycol + yptr[k] : NULL, ycol ? yval + yptr[k] : NULL,
                        &nnz, &dk);
        if (!ycol) yptr[k + 1] = yptr[k] + nnz;
        else d[k] = dk;
    }
    return SRWO_OK;
}

/* ------------------------------------------------------------------------- */
/* Applying the preconditioner and PCG (Algorithm 1, Section 6).             */
/* ------------------------------------------------------------------------- */

/* z = (Y^T D Y)^{-1} r where Y (unit diagonal implicit, strictly lower in rank) is
 * given by rows: Y^T w = r by backward substitution in decreasing rank, v = w / D,
 * Y z = v by forward substitution in increasing rank.  In the paper's reversed
 * indexing this is (L D L^T)^{-1} with L = rev(Y)^T (eqs. y and d).  `by_rank[p]` is
 * the node of rank p; `work` holds n doubles. */
void srwo_apply(int64_t n, const int64_t* yptr, const int32_t* ycol, const double* yval,
                const double* d, const int32_t* by_rank, const double* r, double* z,
                double* work)
{
    double* w = work;
    for (int64_t v = 0; v < n; v++) w[v] = r[v];
    /* Y^T w = r: once w_k is final (all higher-ranked rows done), remove its
     * contribution Y_ki w_k from every lower-ranked i of row k. */
    for (int64_t p = n - 1; p >= 0; p--) {
        int64_t k = by_rank[p];
        for (int64_t q = yptr[k]; q < yptr[k + 1]; q++) w[ycol[q]] = w[ycol[q]] - yval[q] * w[k];
    }
    for (int64_t v = 0; v < n; v++) z[v] = w[v] / d[v];
    for (int64_t p = 0; p < n; p++) {
        int64_t k = by_rank[p];
        double s = z[k];
        for (int64_t q = yptr[k]; q < yptr[k + 1]; q++) s = s - yval[q] * z[ycol[q]];
        z[k] = s;
    }
}

static double dot(int64_t n, const double* a, const double* b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s = s + a[i] * b[i];
    return s;
}

static void spmv(int64_t n, const int64_t* rowptr, const int32_t* col, const double* val,
                 const double* x, double* y)
{
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) s = s + val[p] * x[col[p]];
        y[i] = s;
    }
}

/* Preconditioned conjugate gradient (Barrett et al., Templates, Alg. PCG) from
 * x0 = 0 with M^{-1} = srwo_apply (or the identity when yptr == NULL).  Stops when
 * the recurrence residual satisfies ||r|| <= tol ||b||; the true residual b - Ax is
 * then recomputed and, if it fails the test, PCG restarts from it.  *iters counts
 * products with A inside the iteration; *rel_res is ||b - Ax|| / ||b|| (0 for b = 0).
 * Returns SRWO_OK or SRWO_NOT_CONVERGED (x = last iterate). */
int srwo_pcg(int64_t n, const int64_t* rowptr, const int32_t* col, const double* val,
             const int64_t* yptr, const int32_t* ycol, const double* yval, const double* d,
             const int32_t* by_rank, const double* b, double tol, int32_t max_iter,
             double* x, int32_t* iters, double* rel_res)
{
    double* r = (double*)malloc(sizeof(double) * (size_t)(n ? n : 1) * 5);
    if (!r) return SRWO_E_NOMEM;
    double *z = r + n, *p = r + 2 * n, *q = r + 3 * n, *work = r + 4 * n;
    for (int64_t i = 0; i < n; i++) { x[i] = 0.0; r[i] = b[i]; }
    double bnorm = sqrt(dot(n, b, b));
    int32_t it = 0;
    int status = SRWO_NOT_CONVERGED;
    if (bnorm == 0.0) {
        *iters = 0; *rel_res = 0.0; free(r);
        return SRWO_OK;
    }
#define APPLY(src, dst)                                                          \
    do {                                                                         \
        if (yptr) srwo_apply(n, yptr, ycol, yval, d, by_rank, src, dst, work);   \
        else for (int64_t i_ = 0; i_ < n; i_++) dst[i_] = src[i_];               \
    } while (0)
    APPLY(r, z);
    for (int64_t i = 0; i < n; i++) p[i] = z[i];
    double rho = dot(n, r, z);
    while (it < max_iter) {
        spmv(n, rowptr, col, val, p, q);
        it++;
        double alpha = rho / dot(n, p, q);
        for (int64_t i = 0; i < n; i++) {
            x[i] = x[i] + alpha * p[i];
            r[i] = r[i] - alpha * q[i];
        }
        if (sqrt(dot(n, r, r)) <= tol * bnorm) {
            spmv(n, rowptr, col, val, x, q);
            for (int64_t i = 0; i < n; i++) r[i] = b[i] - q[i];
            if (sqrt(dot(n, r, r)) <= tol * bnorm) {
                status = SRWO_OK;
                break;
            }
            /* restart from the true residual */
            APPLY(r, z);
            for (int64_t i = 0; i < n; i++) p[i] = z[i];
            rho = dot(n, r, z);
            continue;
        }
        APPLY(r, z);
        double rho_new = dot(n, r, z);
        double beta = rho_new / rho;
        rho = rho_new;
        for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
    }
#undef APPLY
    spmv(n, rowptr, col, val, x, q);
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - q[i];
    *rel_res = sqrt(dot(n, r, r)) / bnorm;
    *iters = it;
    free(r);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Asymmetric matrices: two games, LDU of rev(A) (Section 7.1).              */
/* ------------------------------------------------------------------------- */

/* Asymmetric R-matrix check for the two-game construction: the CSR structure as in
 * srwo_validate; a positive diagonal and strictly negative off-diagonal entries; the
 * pattern symmetric (A_jk stored exactly when A_kj is; the values may differ); the
 * off-diagonal row sums and column sums both at most the diagonal (the game of A and
 * the game of A^T are both defined, Section 2.1); and in every connected component a
 * node with positive row excess and a node with positive column excess (a path to
 * ground in both games). */
int srwo_validate_asym(int64_t n, const int64_t* rowptr, const int32_t* col, const double* val)
{
    if (n < 0 || rowptr[0] != 0) return SRWO_E_ARG;
    for (int64_t k = 0; k < n; k++) {
        if (rowptr[k + 1] < rowptr[k]) return SRWO_E_ARG;
        int ndiag = 0;
        for (int64_t p = rowptr[k]; p < rowptr[k + 1]; p++) {
            int32_t j = col[p];
            if (j < 0 || j >= n) return SRWO_E_ARG;
            if (p > rowptr[k] && col[p - 1] >= j) return SRWO_E_ARG;
            if (j == k) ndiag++;
        }
        if (ndiag != 1) return SRWO_E_ARG;
    }
    double* colsum = (double*)calloc((size_t)(n ? n : 1), sizeof(double));
    double* diag = (double*)calloc((size_t)(n ? n : 1), sizeof(double));
    if (!colsum || !diag) { free(colsum); free(diag); return SRWO_E_NOMEM; }
    int status = SRWO_OK;
    for (int64_t k = 0; k < n && status == SRWO_OK; k++) {
        double a = 0.0, sum_w = 0.0;
        for (int64_t p = rowptr[k]; p < rowptr[k + 1]; p++)
            if (col[p] == k) a = val[p];
        if (!(a > 0.0)) { status = SRWO_E_NOT_RMATRIX; break; }
        diag[k] = a;
        for (int64_t p = rowptr[k]; p < rowptr[k + 1]; p++) {
            int32_t j = col[p];
            if (j == k) continue;
            if (!(val[p] < 0.0)) { status = SRWO_E_NOT_RMATRIX; break; }
            sum_w = sum_w + (-val[p]);
            /* structural symmetry */
            int64_t lo = rowptr[j], hi = rowptr[j + 1] - 1, found = -1;
            while (lo <= hi) {
                int64_t mid = lo + (hi - lo) / 2;
                if (col[mid] == k) { found = mid; break; }
                if (col[mid] < k) lo = mid + 1; else hi = mid - 1;
            }
            if (found < 0) { status = SRWO_E_NOT_RMATRIX; break; }
        }
        if (status == SRWO_OK && a - sum_w < -EPS_EXCESS * a) status = SRWO_E_NOT_RMATRIX;
    }
    if (status == SRWO_OK) {
        for (int64_t k = 0; k < n; k++)
            for (int64_t p = rowptr[k]; p < rowptr[k + 1]; p++)
                if (col[p] != k) colsum[col[p]] = colsum[col[p]] + (-val[p]);
        for (int64_t k = 0; k < n; k++)
            if (diag[k] - colsum[k] < -EPS_EXCESS * diag[k]) { status = SRWO_E_NOT_RMATRIX; break; }
    }
    if (status != SRWO_OK) { free(colsum); free(diag); return status; }
    int64_t* parent = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    unsigned char* gr = (unsigned char*)calloc((size_t)(n ? n : 1), 1);
    unsigned char* gc = (unsigned char*)calloc((size_t)(n ? n : 1), 1);
    if (!parent || !gr || !gc) {
        free(parent); free(gr); free(gc); free(colsum); free(diag);
        return SRWO_E_NOMEM;
    }
    for (int64_t v = 0; v < n; v++) parent[v] = v;
    for (int64_t k = 0; k < n; k++)
        for (int64_t p = rowptr[k]; p < rowptr[k + 1]; p++) {
            int64_t ra = uf_find(parent, k), rb = uf_find(parent, col[p]);
            if (ra != rb) parent[ra > rb ? ra : rb] = ra < rb ? ra : rb;
        }
    for (int64_t k = 0; k < n; k++) {
        double sum_w = 0.0;
        for (int64_t p = rowptr[k]; p < rowptr[k + 1]; p++)
            if (col[p] != k) sum_w = sum_w + (-val[p]);
        if (diag[k] - sum_w > EPS_EXCESS * diag[k]) gr[uf_find(parent, k)] = 1;
        if (diag[k] - colsum[k] > EPS_EXCESS * diag[k]) gc[uf_find(parent, k)] = 1;
    }
    for (int64_t v = 0; v < n; v++)
        if (uf_find(parent, v) == v && (!gr[v] || !gc[v])) status = SRWO_E_SINGULAR;
    free(parent); free(gr); free(gc); free(colsum); free(diag);
    return status;
}

/* z = (Y_T^T D Y_A)^{-1} r: the preconditioner of an asymmetric A from the factor of
 * the game of A (Y_A, D; eqs. y2 and d) and the factor of the game of A^T (Y_T;
 * eq. y3), both strictly lower in rank.  In rank order Y_A is the unit lower factor
 * of the reversed LDU of eq. y2 and Y_T^T the unit upper factor of eq. y3.  The solve
 * with Y_T^T runs first (ranks descending), then D, then the solve with Y_A. */
void srwo_apply_ldu(int64_t n, const int64_t* yptr, const int32_t* ycol, const double* yval,
                    const double* d, const int64_t* tptr, const int32_t* tcol,
                    const double* tval, const int32_t* by_rank, const double* r, double* z,
                    double* work)
{
    double* w = work;
    for (int64_t v = 0; v < n; v++) w[v] = r[v];
    for (int64_t p = n - 1; p >= 0; p--) {
        int64_t k = by_rank[p];
        for (int64_t q = tptr[k]; q < tptr[k + 1]; q++) w[tcol[q]] = w[tcol[q]] - tval[q] * w[k];
    }
    for (int64_t v = 0; v < n; v++) z[v] = w[v] / d[v];
    for (int64_t p = 0; p < n; p++) {
        int64_t k = by_rank[p];
        double s = z[k];
        for (int64_t q = yptr[k]; q < yptr[k + 1]; q++) s = s - yval[q] * z[ycol[q]];
        z[k] = s;
    }
}

/* Preconditioned BiCGSTAB (Barrett et al., Templates, Section 2.3.8, preconditioned
 * BiCGSTAB) from x0 = 0 with r~ = r0 and M^{-1} = srwo_apply_ldu (the identity when
 * yptr == NULL).  Each iteration: rho = r~.r; p = r (first) or r + beta (p - omega v)
 * with beta = (rho / rho_prev)(alpha / omega); p^ = M^{-1} p; v = A p^; alpha =
 * rho / r~.v; s = r - alpha v; if ||s|| <= tol ||b||, x += alpha p^ and the iteration
 * ends there; else s^ = M^{-1} s, t = A s^, omega = t.s / t.t, x += alpha p^ + omega s^,
 * r = s - omega t, test ||r|| <= tol ||b||.  A passed test is confirmed on the true
 * residual b - Ax; if it fails, the method restarts from it (r~ = r).  rho = 0,
 * r~.v = 0, t.t = 0 or omega = 0 is a breakdown: SRWO_NOT_CONVERGED with the current
 * x.  *iters counts iterations (a half iteration that meets the test counts as one). */
int srwo_bicgstab(int64_t n, const int64_t* rowptr, const int32_t* col, const double* val,
                  const int64_t* yptr, const int32_t* ycol, const double* yval, const double* d,
                  const int64_t* tptr, const int32_t* tcol, const double* tval,
                  const int32_t* by_rank, const double* b, double tol, int32_t max_iter,
                  double* x, int32_t* iters, double* rel_res)
{
    double* r = (double*)malloc(sizeof(double) * (size_t)(n ? n : 1) * 10);
    if (!r) return SRWO_E_NOMEM;
    double *rt = r + n, *p = r + 2 * n, *v = r + 3 * n, *ph = r + 4 * n, *s = r + 5 * n;
    double *sh = r + 6 * n, *t = r + 7 * n, *q = r + 8 * n, *work = r + 9 * n;
    for (int64_t i = 0; i < n; i++) { x[i] = 0.0; r[i] = b[i]; rt[i] = b[i]; }
    double bnorm = sqrt(dot(n, b, b));
    int32_t it = 0;
    int status = SRWO_NOT_CONVERGED;
    if (bnorm == 0.0) {
        *iters = 0; *rel_res = 0.0; free(r);
        return SRWO_OK;
    }
#define APPLY(src, dst)                                                                    \
    do {                                                                                   \
        if (yptr) srwo_apply_ldu(n, yptr, ycol, yval, d, tptr, tcol, tval, by_rank, src, dst, \
                                 work);                                                    \
        else for (int64_t i_ = 0; i_ < n; i_++) dst[i_] = src[i_];                         \
    } while (0)
    int first = 1;
    double rho_prev = 0.0, alpha = 0.0, omega = 0.0;
    while (it < max_iter) {
        double rho = dot(n, rt, r);
        if (rho == 0.0) break;
        if (first) {
            for (int64_t i = 0; i < n; i++) p[i] = r[i];
            first = 0;
        } else {
            double beta = (rho / rho_prev) * (alpha / omega);
            for (int64_t i = 0; i < n; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        }
        APPLY(p, ph);
        spmv(n, rowptr, col, val, ph, v);
        it++;
        double rtv = dot(n, rt, v);
        if (rtv == 0.0) break;
        alpha = rho / rtv;
        for (int64_t i = 0; i < n; i++) s[i] = r[i] - alpha * v[i];
        int converged = 0;
        if (sqrt(dot(n, s, s)) <= tol * bnorm) {
            for (int64_t i = 0; i < n; i++) x[i] = x[i] + alpha * ph[i];
            converged = 1;
        } else {
            APPLY(s, sh);
            spmv(n, rowptr, col, val, sh, t);
            double tt = dot(n, t, t);
            if (tt == 0.0) break;
            omega = dot(n, t, s) / tt;
            for (int64_t i = 0; i < n; i++) {
                x[i] = x[i] + alpha * ph[i] + omega * sh[i];
                r[i] = s[i] - omega * t[i];
            }
            rho_prev = rho;
            if (sqrt(dot(n, r, r)) <= tol * bnorm) converged = 1;
            else if (omega == 0.0) break;
        }
        if (converged) {
            spmv(n, rowptr, col, val, x, q);
            for (int64_t i = 0; i < n; i++) r[i] = b[i] - q[i];
            if (sqrt(dot(n, r, r)) <= tol * bnorm) {
                status = SRWO_OK;
                break;
            }
            /* restart from the true residual */
            for (int64_t i = 0; i < n; i++) rt[i] = r[i];
            first = 1;
        }
    }
#undef APPLY
    spmv(n, rowptr, col, val, x, q);
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - q[i];
    *rel_res = sqrt(dot(n, r, r)) / bnorm;
    *iters = it;
    free(r);
    return status;
}

/* ------------------------------------------------------------------------- */
/* IC(0): the incomplete Cholesky comparison preconditioner of Section 6     */
/* (the ICCG columns of Tables 1-2), in the factor's form A ~ Y^T D Y.       */
/* ------------------------------------------------------------------------- */

/* Y_{j,c} of a factor row stored in ascending column id, or 0 if absent. */
static double row_entry(const int64_t* yptr, const int32_t* ycol, const double* yval,
                        int64_t j, int32_t c)
{
    for (int64_t q = yptr[j]; q < yptr[j + 1]; q++)
        if (ycol[q] == c) return yval[q];
    return 0.0;
}

/* Zero fill-in incomplete Cholesky of an R-matrix in the factor's form: nodes are
 * eliminated one at a time in decreasing rank, and the update of every remaining
 * entry outside the pattern of A is discarded.  Row k of Y keeps exactly the
 * lower-ranked neighbours of k:
 *     D_k  = A_kk - sum_{j in Up(k)} (D_j Y_jk) Y_jk
 *     Y_ki = (A_ki - sum_{j in Up(k), j adjacent to i} (D_j Y_jk) Y_ji) / D_k
 * with Up(k) the higher-ranked neighbours of k, taken in the CSR order of row k.
 * First call with ycol == NULL fills yptr (entries in ascending column id); the
 * second fills ycol, yval and d.  by_rank[p] is the node of rank p.  Returns
 * SRWO_E_NOT_RMATRIX if a pivot is not positive. */
int srwo_ic0(int64_t n, const int64_t* rowptr, const int32_t* col, const double* val,
             const int32_t* rank, const int32_t* by_rank, int64_t* yptr, int32_t* ycol,
             double* yval, double* d)
{
    if (!ycol) {
        yptr[0] = 0;
        for (int64_t k = 0; k < n; k++) {
            int64_t m = 0;
            for (int64_t p = rowptr[k]; p < rowptr[k + 1]; p++)
                if (col[p] != k && rank[col[p]] < rank[k]) m++;
            yptr[k + 1] = yptr[k] + m;
        }
        return SRWO_OK;
    }
    for (int64_t pos = n - 1; pos >= 0; pos--) {
        int64_t k = by_rank[pos];
        double a = 0.0;
        for (int64_t p = rowptr[k]; p < rowptr[k + 1]; p++)
            if (col[p] == k) a = val[p];
        double dk = a;
        for (int64_t p = rowptr[k]; p < rowptr[k + 1]; p++) {
            int32_t j = col[p];
            if (j == k || rank[j] < rank[k]) continue;
            double yjk = row_entry(yptr, ycol, yval, j, (int32_t)k);
            dk = dk - (d[j] * yjk) * yjk;
        }
        if (!(dk > 0.0)) return SRWO_E_NOT_RMATRIX;
        d[k] = dk;
        int64_t q = yptr[k];
        for (int64_t p = rowptr[k]; p < rowptr[k + 1]; p++) {
            int32_t i = col[p];
            if (i == k || rank[i] > rank[k]) continue;
            double s = val[p];
            for (int64_t p2 = rowptr[k]; p2 < rowptr[k + 1]; p2++) {
                int32_t j = col[p2];
                if (j == k || rank[j] < rank[k]) continue;
                double yji = row_entry(yptr, ycol, yval, j, i);
                if (yji == 0.0) continue;
                double yjk = row_entry(yptr, ycol, yval, j, (int32_t)k);
                s = s - (d[j] * yjk) * yji;
            }
            ycol[q] = i;
            yval[q] = s / dk;
            q++;
        }
    }
    return SRWO_OK;
}

/* ------------------------------------------------------------------------- */
/* The plain estimator: eq. yzdetail with eq. d, without the exact one-step  */
/* treatment of Section 5.2 (a test mode: both must reach the same limit).   */
/* ------------------------------------------------------------------------- */

/* Walk w of row k by the full game of Section 2.1 from its first step on: every step,
 * the first included, leaves the current node by its thresholds (ground when the row
 * is grounded and u passes every threshold); the walk ends at ground or at the first
 * node ranked below k, after one step if the first step already gets there.  Draw t
 * (t = 0 for the first step) is srwo_draw(seed, k, w, t).  visits counts the stays at
 * k, the start included; length is the number of steps. */
void srwo_walk_plain(int64_t n, const int64_t* rowptr, const int32_t* nbr, const uint32_t* thr,
                     const unsigned char* grounded, const int32_t* rank, uint64_t seed,
                     int64_t k, int64_t w, int32_t* end_out, uint32_t* visits_out,
                     uint32_t* length_out)
{
    (void)n;
    int64_t cur = k;
    uint32_t visits = 1;
    for (uint64_t t = 0;; t++) {
        uint32_t u = srwo_draw(seed, k, w, t);
        int64_t base = rowptr[cur] - cur;
        int64_t deg = rowptr[cur + 1] - rowptr[cur] - 1;
        int64_t next = -2;
        for (int64_t m = 0; m < deg; m++)
            if (u < thr[base + m]) { next = nbr[base + m]; break; }
        if (next == -2) next = grounded[cur] ? -1 : nbr[base + deg - 1];
        if (next == -1) {
            *end_out = -1; *visits_out = visits; *length_out = (uint32_t)(t + 1);
            return;
        }
        if (rank[next] < rank[k]) {
            *end_out = (int32_t)next; *visits_out = visits; *length_out = (uint32_t)(t + 1);
            return;
        }
        if (next == k) visits++;
        cur = next;
    }
}

/* srwo_walk_rows for the plain estimator: every listed row runs budget[r] walks. */
int srwo_walk_rows_plain(int64_t n, const int64_t* rowptr, const int32_t* nbr,
                         const uint32_t* thr, const unsigned char* grounded, const int32_t* rank,
                         uint64_t seed, int64_t nrows, const int64_t* rows, const int32_t* budget,
                         const int64_t* rec_off, int32_t* end, uint32_t* visits, uint32_t* length)
{
    for (int64_t r = 0; r < nrows; r++) {
        int64_t k = rows[r];
        if (k < 0 || k >= n) return SRWO_E_ARG;
        for (int64_t w = 0; w < budget[r]; w++)
            srwo_walk_plain(n, rowptr, nbr, thr, grounded, rank, seed, k, w,
                            &end[rec_off[r] + w], &visits[rec_off[r] + w], &length[rec_off[r] + w]);
    }
    return SRWO_OK;
}

/* Factor rows of the plain estimator from the tallies of its walks (M = walks[k] > 0
 * for every row): eq. yzdetail gives Y_ki = -H'_{k,i} / M for every end node i, and
 * eq. d gives D_k = M A_kk / J'_k (J' counts the start).  Entries with
 * |Y_ki| < drop_tol are dropped; ascending column id.  Two calls as srwo_factor. */
int srwo_factor_plain(int64_t n, const int64_t* rowptr, const int32_t* col, const double* val,
                      const uint32_t* walks, const uint64_t* J, const int64_t* h_off,
                      const int32_t* hlen, const int32_t* h_end, const uint32_t* h_cnt,
                      double drop_tol, int64_t* yptr, int32_t* ycol, double* yval, double* d)
{
    if (!ycol) yptr[0] = 0;
    for (int64_t k = 0; k < n; k++) {
        double a = 0.0;
        for (int64_t p = rowptr[k]; p < rowptr[k + 1]; p++)
            if (col[p] == k) a = val[p];
        uint32_t M = walks[k];
        if (M == 0) return SRWO_E_ARG;
        int64_t kept = 0;
        for (int32_t h = 0; h < hlen[k]; h++) {
            double y = -((double)h_cnt[h_off[k] + h] / (double)M);
            if (!(fabs(y) < drop_tol)) {
                if (ycol) {
                    ycol[yptr[k] + kept] = h_end[h_off[k] + h];
                    yval[yptr[k] + kept] = y;
                }
                kept++;
            }
        }
        if (!ycol) yptr[k + 1] = yptr[k] + kept;
        else d[k] = ((double)M * a) / (double)J[k];
    }
    return SRWO_OK;
}
