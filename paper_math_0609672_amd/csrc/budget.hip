// Learned walk budgets (an extension; the paper fixes walks per row by a stopping rule on
// walk lengths, Section 5.1): per-row graph features, per-walk variance labels from a
// pilot factor's tallies, and an 8 -> 64 -> 64 -> 1 ReLU network run and trained on the
// GPU with bfloat16 MFMA operands and fp32 accumulation.
//
// Network layout (one fp32 array of SRW_MLP_PARAMS): W1 [8][64], b1 [64], W2 [64][64],
// b2 [64], W3 [64], b3.  The network is evaluated transposed -- hidden units along the
// MFMA rows, 16 matrix rows (graph rows) along its columns -- so that the output
// registers of one layer are already the B operand of the next:
//   v_mfma_f32_16x16x16_bf16: A lane l holds A[l%16][4(l/16)+j], B lane l holds
//   B[4(l/16)+j][l%16], D lane l holds D[4(l/16)+j][l%16], j = 0..3.
// Rounding points (mirrored by the oracle): the standardized inputs, the weights and the
// hidden activations are rounded to bfloat16 (nearest, ties to even) before each
// product; in the backward pass the pre-activation gradients dZ2 and dZ1 are rounded
// the same way.  Every sum is fp32; reductions run in a fixed order.
#include <cmath>

#include "factor.hpp"

namespace srw {

namespace {

constexpr int BLOCK = 256;
constexpr int NF = 8;
constexpr int NH = 64;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + NF * NH;
constexpr int OFF_W2 = OFF_B1 + NH;
constexpr int OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH;
constexpr int OFF_B3 = OFF_W3 + NH;
constexpr int NPARAM = OFF_B3 + 1;  // 4801
constexpr int PART = NPARAM + 1;    // a wave's partial: gradient + loss
static_assert(NPARAM == SRW_MLP_PARAMS, "parameter layout");

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // nearest, ties to even (finite inputs)
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h)
{
    return __uint_as_float((uint32_t)h << 16);
}
__device__ __forceinline__ float round_bf16(float f) { return from_bf16(to_bf16(f)); }

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d)
{
    bf16x4 v;
    v[0] = (short)to_bf16(a);
    v[1] = (short)to_bf16(b);
    v[2] = (short)to_bf16(c);
    v[3] = (short)to_bf16(d);
    return v;
}

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------- features
// e_k / a_k of every node.
__global__ void k_excess_ratio(int64_t n, const int64_t* __restrict__ rowptr,
                               const int32_t* __restrict__ col, const double* __restrict__ val,
                               double* __restrict__ ratio)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double a = 0.0, s = 0.0;
    for (int64_t q = rowptr[k]; q < rowptr[k + 1]; ++q) {
        if (col[q] == k) a = val[q];
        else s = s + (-val[q]);
    }
    ratio[k] = (a - s) / a;
}

// The eight features of a row (float64 arithmetic, stored as float32), in order:
// degree, log a_k, e_k / a_k, tau_k, fraction of neighbours ranked above k,
// log(max w / min w), log(n / (rank_k + 1)), mean of e_j / a_j over neighbours j.
__global__ void k_features(int64_t n, const int64_t* __restrict__ rowptr,
                           const int32_t* __restrict__ col, const double* __restrict__ val,
                           const int32_t* __restrict__ rank, const double* __restrict__ ratio,
                           float* __restrict__ feat)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int32_t rk = rank[k];
    double a = 0.0, motel = 0.0, wmin = 0.0, wmax = 0.0, rsum = 0.0;
    int deg = 0, higher = 0;
    for (int64_t q = rowptr[k]; q < rowptr[k + 1]; ++q) {
        const int32_t j = col[q];
        if (j == k) {
            a = val[q];
            continue;
        }
        const double w = -val[q];
        if (deg == 0 || w < wmin) wmin = w;
        if (deg == 0 || w > wmax) wmax = w;
        ++deg;
        if (rank[j] > rk) {
            ++higher;
            motel = motel + w;
        }
        rsum = rsum + ratio[j];
    }
    float* f = feat + k * NF;
    f[0] = (float)deg;
    f[1] = (float)log(a);
    f[2] = (float)ratio[k];
    f[3] = (float)(motel / a);
    f[4] = deg ? (float)((double)higher / (double)deg) : 0.0f;
    f[5] = deg ? (float)log(wmax / wmin) : 0.0f;
    f[6] = (float)log((double)n / ((double)rk + 1.0));
    f[7] = deg ? (float)(rsum / (double)deg) : 0.0f;
}

// --------------------------------------------------------------------- labels
// Per-walk variance of row k from its tallies: tau^2 sum_i p_i (1 - p_i) plus
// (tau / (1 + tau (m - 1)))^2 s^2 (m, s^2: mean and sample variance of the stays);
// per_step: divided by the row's mean walk length (steps per walk).  NaN for a row
// without walks.  One wave per row over its H list.
__global__ __launch_bounds__(64) void k_labels(int64_t n, const double* __restrict__ tau,
                                               const int32_t* __restrict__ walks,
                                               const uint64_t* __restrict__ J,
                                               const uint64_t* __restrict__ vsq,
                                               const uint64_t* __restrict__ steps, int per_step,
                                               const int64_t* __restrict__ h_off,
                                               const int32_t* __restrict__ hlen,
                                               const uint32_t* __restrict__ h_cnt,
                                               double* __restrict__ label)
{
    const int64_t k = blockIdx.x;
    const int lane = threadIdx.x;
    const int32_t m = walks[k];
    if (m == 0) {
        if (lane == 0) label[k] = NAN;
        return;
    }
    const double M = (double)m;
    double py = 0.0;
    const int64_t a = h_off[k];
    for (int i = lane; i < hlen[k]; i += 64) {
        const double p = (double)h_cnt[a + i] / M;
        py += p * (1.0 - p);
    }
    py = wave_sum(py);
    if (lane == 0) {
        const double mean = (double)J[k] / M;
        double s2 = m > 1 ? ((double)vsq[k] - M * mean * mean) / (M - 1.0) : 0.0;
        if (s2 < 0.0) s2 = 0.0;
        const double t = tau[k];
        const double c = t / (1.0 + t * (mean - 1.0));
        double v = t * t * py + c * c * s2;
        if (per_step) v = v / ((double)steps[k] / M);
        label[k] = v;
    }
}

// ------------------------------------------------------------------------ MLP
// Operands of a block's waves, built once per block in LDS from the fp32 weights:
//   a1[mb]      layer 1, A = W1^T block mb (k >= 8 zero)
//   a2[mb][kb]  layer 2, A = W2^T block (mb, kb)
//   a3[mb][kb]  backward dZ1 = W2 dZ2, A = W2 block (mb, kb)
struct MlpShared {
    bf16x4 a1[4][64];
    bf16x4 a2[16][64];
    bf16x4 a3[16][64];
    float b1[NH], b2[NH], w3[NH];  // w3 rounded to bfloat16
    float b3;
};

__device__ void load_shared(const float* __restrict__ P, MlpShared& sh)
{
    for (int t = threadIdx.x; t < 4 * 64; t += blockDim.x) {
        const int mb = t / 64, l = t % 64, g = l / 16, c = l % 16;
        float v[4];
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * g + j;
            v[j] = k < NF ? P[OFF_W1 + k * NH + 16 * mb + c] : 0.0f;
        }
        sh.a1[mb][l] = pack4(v[0], v[1], v[2], v[3]);
    }
    for (int t = threadIdx.x; t < 16 * 64; t += blockDim.x) {
        const int blk = t / 64, l = t % 64, mb = blk / 4, kb = blk % 4, g = l / 16, c = l % 16;
        float v[4], u[4];
        for (int j = 0; j < 4; ++j) {
            v[j] = P[OFF_W2 + (16 * kb + 4 * g + j) * NH + 16 * mb + c];  // W2^T[16mb+c][16kb+4g+j]
            u[j] = P[OFF_W2 + (16 * mb + c) * NH + 16 * kb + 4 * g + j];  // W2[16mb+c][16kb+4g+j]
        }
        sh.a2[blk][l] = pack4(v[0], v[1], v[2], v[3]);
        sh.a3[blk][l] = pack4(u[0], u[1], u[2], u[3]);
    }
    for (int t = threadIdx.x; t < NH; t += blockDim.x) {
        sh.b1[t] = P[OFF_B1 + t];
        sh.b2[t] = P[OFF_B2 + t];
        sh.w3[t] = round_bf16(P[OFF_W3 + t]);
    }
    if (threadIdx.x == 0) sh.b3 = P[OFF_B3];
    __syncthreads();
}

// Forward pass of one 16-row tile in the wave.  Outputs (per lane l, hidden unit
// h = 16 mb + 4 (l/16) + j, tile row l % 16): z1, z2 (fp32 pre-activations), h1b
// (bfloat16 B operands of layer 2), h2 (bfloat16-rounded activations) and y of the
// lane's row.  xs: the lane's standardized, rounded inputs (features 4(l/16)+j).
struct Tile {
    f32x4 z1[4], z2[4];
    bf16x4 h1b[4];
    float h2[4][4];
    float xs[4];
    float y;
};

__device__ __forceinline__ void tile_forward(const MlpShared& sh, const float* __restrict__ feat,
                                             const float* __restrict__ musd, int64_t row,
                                             bool valid, Tile& T)
{
    const int l = threadIdx.x & 63, g = l / 16;
    for (int j = 0; j < 4; ++j) {
        const int f = 4 * g + j;
        float x = 0.0f;
        if (valid && f < NF) x = round_bf16((feat[row * NF + f] - musd[f]) / musd[NF + f]);
        T.xs[j] = x;
    }
    const bf16x4 b1op = pack4(T.xs[0], T.xs[1], T.xs[2], T.xs[3]);
    for (int mb = 0; mb < 4; ++mb) {
        T.z1[mb] = mfma(sh.a1[mb][l], b1op, f32x4{0.0f, 0.0f, 0.0f, 0.0f});
        float h[4];
        for (int j = 0; j < 4; ++j) {
            T.z1[mb][j] = T.z1[mb][j] + sh.b1[16 * mb + 4 * g + j];
            h[j] = T.z1[mb][j] > 0.0f ? T.z1[mb][j] : 0.0f;
        }
        T.h1b[mb] = pack4(h[0], h[1], h[2], h[3]);
    }
    float part = 0.0f;
    for (int mb = 0; mb < 4; ++mb) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int kb = 0; kb < 4; ++kb) acc = mfma(sh.a2[4 * mb + kb][l], T.h1b[kb], acc);
        for (int j = 0; j < 4; ++j) {
            const int h = 16 * mb + 4 * g + j;
            T.z2[mb][j] = acc[j] + sh.b2[h];
            const float a = T.z2[mb][j] > 0.0f ? round_bf16(T.z2[mb][j]) : 0.0f;
            T.h2[mb][j] = a;
            part = part + a * sh.w3[h];
        }
    }
    // the four lane groups hold the same row's partial sums over disjoint units
    part = part + __shfl_xor(part, 16, 64);
    part = part + __shfl_xor(part, 32, 64);
    T.y = part + sh.b3;
}

__global__ __launch_bounds__(BLOCK) void k_mlp_forward(const float* __restrict__ P,
                                                       const float* __restrict__ musd,
                                                       const float* __restrict__ feat, int64_t n,
                                                       float* __restrict__ out)
{
    __shared__ MlpShared sh;
    load_shared(P, sh);
    const int l = threadIdx.x & 63;
    const int64_t ntile = (n + 15) / 16;
    const int64_t nw = (int64_t)gridDim.x * (BLOCK / 64);
    const int64_t w0 = (int64_t)blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    for (int64_t t = w0; t < ntile; t += nw) {
        const int64_t row = t * 16 + (l % 16);
        const bool valid = row < n;
        Tile T;
        tile_forward(sh, feat, musd, row, valid, T);
        if (l < 16 && valid) out[row] = T.y;
    }
}

// Gradient of mean((y - t)^2) over `n_total` rows, for the `n` rows given: each wave
// accumulates its tiles and writes one partial (gradient in parameter layout, then
// the sum of squared errors) to part[wave].
struct WaveLds {
    unsigned short h1[16][NH];   // tile row, hidden 1
    unsigned short dz2[16][NH];  // tile row, hidden 2
    unsigned short x[16][16];    // tile row, feature (8 used)
    unsigned short dz1[16][NH];
};

__global__ __launch_bounds__(BLOCK) void k_mlp_grad(const float* __restrict__ P,
                                                    const float* __restrict__ musd,
                                                    const float* __restrict__ feat,
                                                    const float* __restrict__ target,
                                                    const int32_t* __restrict__ rows,
                                                    int64_t n_rows, int64_t n, float inv_total,
                                                    float* __restrict__ part)
{
    __shared__ MlpShared sh;
    __shared__ WaveLds wl[BLOCK / 64];
    load_shared(P, sh);
    const int l = threadIdx.x & 63, g = l / 16, c = l % 16;
    const int wv = threadIdx.x >> 6;
    WaveLds& L = wl[wv];
    const int64_t ntile = (n + 15) / 16;
    const int64_t nw = (int64_t)gridDim.x * (BLOCK / 64);
    const int64_t w0 = (int64_t)blockIdx.x * (BLOCK / 64) + wv;

    f32x4 gw2[16], gw1[4];
    for (int i = 0; i < 16; ++i) gw2[i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int i = 0; i < 4; ++i) gw1[i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float gw3[4][4] = {}, gb2[4][4] = {}, gb1[4][4] = {};
    float gb3 = 0.0f, sse = 0.0f;

    for (int64_t t = w0; t < ntile; t += nw) {
        const int64_t i = t * 16 + c;
        // the i-th row given: rows[i] of the arrays, or row i without a list (the caller
        // has checked the list; a row outside the arrays would count as absent)
        const int64_t r = i < n ? (rows ? (int64_t)rows[i] : i) : -1;
        const bool valid = r >= 0 && r < n_rows;
        const int64_t row = valid ? r : 0;
        Tile T;
        tile_forward(sh, feat, musd, row, valid, T);
        const float err = valid ? T.y - target[row] : 0.0f;
        const float dy = 2.0f * err * inv_total;
        if (g == 0) {
            sse = sse + err * err;
            gb3 = gb3 + dy;
        }
        // dZ2 = dy W3 (Z2 > 0), rounded; W3 and b2 gradients
        float dz2[4][4];
        for (int mb = 0; mb < 4; ++mb)
            for (int j = 0; j < 4; ++j) {
                const int h = 16 * mb + 4 * g + j;
                gw3[mb][j] = gw3[mb][j] + dy * T.h2[mb][j];
                dz2[mb][j] = T.z2[mb][j] > 0.0f ? round_bf16(dy * sh.w3[h]) : 0.0f;
                gb2[mb][j] = gb2[mb][j] + dz2[mb][j];
            }
        // dZ1 = (W2 dZ2) (Z1 > 0), rounded
        bf16x4 dz2b[4];
        for (int kb = 0; kb < 4; ++kb) dz2b[kb] = pack4(dz2[kb][0], dz2[kb][1], dz2[kb][2], dz2[kb][3]);
        float dz1[4][4];
        for (int mb = 0; mb < 4; ++mb) {
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int kb = 0; kb < 4; ++kb) acc = mfma(sh.a3[4 * mb + kb][l], dz2b[kb], acc);
            for (int j = 0; j < 4; ++j) {
                dz1[mb][j] = T.z1[mb][j] > 0.0f ? round_bf16(acc[j]) : 0.0f;
                gb1[mb][j] = gb1[mb][j] + dz1[mb][j];
            }
        }
        // stage the tile row-major for the weight-gradient products (sum over rows)
        for (int mb = 0; mb < 4; ++mb)
            for (int j = 0; j < 4; ++j) {
                const int h = 16 * mb + 4 * g + j;
                L.h1[c][h] = (unsigned short)T.h1b[mb][j];
                L.dz2[c][h] = to_bf16(dz2[mb][j]);
                L.dz1[c][h] = to_bf16(dz1[mb][j]);
            }
        for (int j = 0; j < 4; ++j) L.x[c][4 * g + j] = to_bf16(T.xs[j]);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // dW2[k][h] += sum_rows H1[row][k] dZ2[row][h]: A = H1^T (k x rows), B = dZ2
        bf16x4 bz2[4], bz1[4];
        for (int nb = 0; nb < 4; ++nb) {
            bf16x4 b, b1;
            for (int j = 0; j < 4; ++j) {
                b[j] = (short)L.dz2[4 * g + j][16 * nb + c];
                b1[j] = (short)L.dz1[4 * g + j][16 * nb + c];
            }
            bz2[nb] = b;
            bz1[nb] = b1;
        }
        for (int mb = 0; mb < 4; ++mb) {
            bf16x4 a;
            for (int j = 0; j < 4; ++j) a[j] = (short)L.h1[4 * g + j][16 * mb + c];
            for (int nb = 0; nb < 4; ++nb) gw2[4 * mb + nb] = mfma(a, bz2[nb], gw2[4 * mb + nb]);
        }
        // dW1[f][k] += sum_rows Xs[row][f] dZ1[row][k]: A = Xs^T (features x rows)
        {
            bf16x4 a;
            for (int j = 0; j < 4; ++j) a[j] = (short)(c < NF ? L.x[4 * g + j][c] : 0);
            for (int nb = 0; nb < 4; ++nb) gw1[nb] = mfma(a, bz1[nb], gw1[nb]);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    if (w0 >= ntile) return;  // whole wave: no tile, no partial
    float* out = part + w0 * PART;
    // dW2 block (mb, nb): lane holds rows k = 16mb + 4g + j, column h = 16nb + c
    for (int mb = 0; mb < 4; ++mb)
        for (int nb = 0; nb < 4; ++nb)
            for (int j = 0; j < 4; ++j)
                out[OFF_W2 + (16 * mb + 4 * g + j) * NH + 16 * nb + c] = gw2[4 * mb + nb][j];
    for (int nb = 0; nb < 4; ++nb)
        for (int j = 0; j < 4; ++j)
            if (4 * g + j < NF) out[OFF_W1 + (4 * g + j) * NH + 16 * nb + c] = gw1[nb][j];
    // per-unit sums over the 16 rows held by the lanes of one group
    for (int mb = 0; mb < 4; ++mb)
        for (int j = 0; j < 4; ++j) {
            float a = gw3[mb][j], b = gb2[mb][j], d = gb1[mb][j];
            for (int off = 1; off < 16; off <<= 1) {
                a = a + __shfl_xor(a, off, 64);
                b = b + __shfl_xor(b, off, 64);
                d = d + __shfl_xor(d, off, 64);
            }
            if (c == 0) {
                const int h = 16 * mb + 4 * g + j;
                out[OFF_W3 + h] = a;
                out[OFF_B2 + h] = b;
                out[OFF_B1 + h] = d;
            }
        }
    for (int off = 1; off < 16; off <<= 1) {
        gb3 = gb3 + __shfl_xor(gb3, off, 64);
        sse = sse + __shfl_xor(sse, off, 64);
    }
    if (l == 0) {
        out[OFF_B3] = gb3;
        out[NPARAM] = sse;
    }
}

// Sum of the wave partials in wave order; then (adam != 0) one Adam step on the fp32
// parameters.  grad (if not null) receives the summed gradient, loss the mean squared
// error.
__global__ void k_mlp_reduce(const float* __restrict__ part, int64_t nparts, float inv_total,
                             float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                             int adam, int32_t step, float lr, float beta1, float beta2, float eps,
                             float* __restrict__ grad, float* __restrict__ loss)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > NPARAM) return;
    float s = 0.0f;
    for (int64_t w = 0; w < nparts; ++w) s = s + part[w * PART + i];
    if (i == NPARAM) {
        if (loss) *loss = s * inv_total;
        return;
    }
    if (grad) grad[i] = s;
    if (!adam) return;
    const float mi = beta1 * m[i] + (1.0f - beta1) * s;
    const float vi = beta2 * v[i] + (1.0f - beta2) * s * s;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.0f - powf(beta1, (float)step));
    const float vh = vi / (1.0f - powf(beta2, (float)step));
    P[i] = P[i] - lr * mh / (sqrtf(vh) + eps);
}

// walks = clamp(ceil(exp(pred) / eps), lo, hi)
__global__ void k_budgets(int64_t n, const float* __restrict__ pred, double eps, int32_t lo,
                          int32_t hi, int32_t* __restrict__ walks)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double m = ceil(exp((double)pred[k]) / eps);
    if (!(m >= (double)lo)) m = lo;  // NaN goes to lo
    if (m > (double)hi) m = hi;
    walks[k] = (int32_t)m;
}

int mlp_grid(int64_t n)
{
    const int64_t tiles = (n + 15) / 16;
    int64_t blocks = (tiles + BLOCK / 64 - 1) / (BLOCK / 64);
    return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, 256));
}

}  // namespace

int features_impl(const srw_csr* A, const int32_t* rank, float* feat, hipStream_t s)
{
    const int64_t n = A->n;
    if (n == 0) return SRW_OK;
    double* ratio = nullptr;
    SRW_HIP(hipMallocAsync((void**)&ratio, n * sizeof(double), s));
    const int g = grid_for(n, BLOCK);
    k_excess_ratio<<<g, BLOCK, 0, s>>>(n, A->rowptr, A->col, A->val, ratio);
    k_features<<<g, BLOCK, 0, s>>>(n, A->rowptr, A->col, A->val, rank, ratio, feat);
    hipError_t e = hipGetLastError();
    (void)hipFreeAsync(ratio, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    SRW_HIP(e);
    return SRW_OK;
}

// Per-row walk statistics from the tallies (Section 3.1 counts): the sample variance of
// the stays at the start, (sum v^2 - J'^2 / M') / (M' - 1), and the mean walk length
// steps / M'.  NaN where a row has too few walks (M' < 2 for the variance, M' = 0 for
// the mean).
__global__ void k_walk_stats(int64_t n, const int32_t* __restrict__ budget,
                             const uint64_t* __restrict__ J, const uint64_t* __restrict__ vsq,
                             const uint64_t* __restrict__ steps, double* __restrict__ var,
                             double* __restrict__ mean_len)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double M = (double)budget[k];
    if (var) {
        const double j = (double)J[k];
        var[k] = budget[k] >= 2 ? ((double)vsq[k] - (j * j) / M) / (M - 1.0) : __builtin_nan("");
    }
    if (mean_len) mean_len[k] = budget[k] >= 1 ? (double)steps[k] / M : __builtin_nan("");
}

int walk_stats_impl(const srw_factor* F, double* var, double* mean_len, hipStream_t s)
{
    if (F->n == 0) return SRW_OK;
    k_walk_stats<<<grid_for(F->n, BLOCK), BLOCK, 0, s>>>(F->n, F->budget, F->tJ, F->tvsq, F->tsteps,
                                                       var, mean_len);
    SRW_HIP(hipGetLastError());
    SRW_HIP(hipStreamSynchronize(s));
    return SRW_OK;
}

int labels_impl(const srw_factor* F, int per_step, double* label, hipStream_t s)
{
    if (F->n == 0) return SRW_OK;
    k_labels<<<(unsigned)F->n, 64, 0, s>>>(F->n, F->tau, F->budget, F->tJ, F->tvsq, F->tsteps,
                                           per_step, F->h_off, F->hlen, F->h_cnt, label);
    SRW_HIP(hipGetLastError());
    SRW_HIP(hipStreamSynchronize(s));
    return SRW_OK;
}

int mlp_forward_impl(const float* P, const float* musd, const float* feat, int64_t n, float* out,
                     hipStream_t s)
{
    if (n == 0) return SRW_OK;
    k_mlp_forward<<<mlp_grid(n), BLOCK, 0, s>>>(P, musd, feat, n, out);
    SRW_HIP(hipGetLastError());
    return SRW_OK;
}

// *bad = 1 if a listed row lies outside [0, n_rows)
__global__ void k_check_rows(int64_t n, const int32_t* __restrict__ rows, int64_t n_rows, int* bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && (rows[i] < 0 || (int64_t)rows[i] >= n_rows)) *bad = 1;
}

int mlp_train_impl(float* P, float* m, float* v, int32_t step, float lr, const float* musd,
                   const float* feat, const float* target, const int32_t* rows, int64_t n_rows,
                   int64_t n, float* grad, float* loss, hipStream_t s)
{
    if (n == 0) return SRW_OK;
    if (rows) {  // the list is checked before any training work is queued
        int* bad = nullptr;
        int hbad = 0;
        SRW_HIP(hipMallocAsync((void**)&bad, sizeof(int), s));
        hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), s);
        if (e == hipSuccess) {
            k_check_rows<<<grid_for(n, BLOCK), BLOCK, 0, s>>>(n, rows, n_rows, bad);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipFreeAsync(bad, s);
        SRW_HIP(e);
        if (hbad) return SRW_E_ARG;
    } else {
        n_rows = n;
    }
    const int grid = mlp_grid(n);
    const int64_t nparts = std::min<int64_t>((int64_t)grid * (BLOCK / 64), (n + 15) / 16);
    float* part = nullptr;
    SRW_HIP(hipMallocAsync((void**)&part, nparts * PART * sizeof(float), s));
    const float inv = 1.0f / (float)n;
    k_mlp_grad<<<grid, BLOCK, 0, s>>>(P, musd, feat, target, rows, n_rows, n, inv, part);
    k_mlp_reduce<<<(NPARAM + 1 + 255) / 256, 256, 0, s>>>(part, nparts, inv, P, m, v, m != nullptr,
                                                          step, lr, 0.9f, 0.999f, 1e-8f, grad,
                                                          loss);
    hipError_t e = hipGetLastError();
    (void)hipFreeAsync(part, s);
    SRW_HIP(e);
    return SRW_OK;
}

// ------------------------------------------------ training set from the labels
// A row enters the training set when its label is finite and positive; its target is
// log(label), halved for the per-step (Neyman) rule: budgets then follow sqrt(label).
__global__ void k_target_flags(int64_t n, const double* __restrict__ label, int32_t* __restrict__ flag)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double l = label[k];
    flag[k] = (l > 0.0 && l < __builtin_inf()) ? 1 : 0;  // false for NaN
}

// Kept rows in row order: features copied, target written at the row's position.
__global__ void k_target_scatter(int64_t n, const double* __restrict__ label,
                                 const float* __restrict__ feat, const int32_t* __restrict__ flag,
                                 const int64_t* __restrict__ pos, int half,
                                 float* __restrict__ x_out, float* __restrict__ y_out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || !flag[k]) return;
    const int64_t j = pos[k];
    const double t = log(label[k]);
    y_out[j] = (float)(half ? 0.5 * t : t);
    for (int f = 0; f < NF; ++f) x_out[j * NF + f] = feat[k * NF + f];
}

// Per-feature sums over a fixed block of rows per workgroup, in float64: pass 0 the
// values, pass 1 the squared deviations from mean (written by pass 0's finish).  Each
// workgroup writes NF partials; one workgroup adds them in workgroup order.
constexpr int STD_BLOCKS = 256;

// Column NF of the sums is the target (pass 0 only; 0 without targets).
constexpr int NS = NF + 1;

__global__ __launch_bounds__(BLOCK) void k_feat_partials(int64_t n, const float* __restrict__ feat,
                                                         const float* __restrict__ target,
                                                         const double* __restrict__ mean,
                                                         double* __restrict__ part)
{
    __shared__ double red[BLOCK / 64][NS];
    double acc[NS];
    for (int f = 0; f < NS; ++f) acc[f] = 0.0;
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = std::min<int64_t>(n, r0 + per);
    for (int64_t r = r0 + threadIdx.x; r < r1; r += BLOCK) {
        for (int f = 0; f < NF; ++f) {
            const double x = (double)feat[r * NF + f];
            acc[f] += mean ? (x - mean[f]) * (x - mean[f]) : x;
        }
        if (!mean && target) acc[NF] += (double)target[r];
    }
    for (int f = 0; f < NS; ++f) acc[f] = wave_sum(acc[f]);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int f = 0; f < NS; ++f) red[w][f] = acc[f];
    __syncthreads();
    if (threadIdx.x < NS) {
        double t = 0.0;
        for (int i = 0; i < BLOCK / 64; ++i) t += red[i][threadIdx.x];
        part[(int64_t)blockIdx.x * NS + threadIdx.x] = t;
    }
}

// pass 0: mean = sum / n (and the target mean).  pass 1: sd = sqrt(ss / (n - 1)), at
// least 1e-6 (1 for a single row); mu_sd (float32) = mean then sd.
__global__ void k_feat_finish(int64_t n, int nparts, const double* __restrict__ part,
                              double* __restrict__ mean, int pass, float* __restrict__ mu_sd,
                              float* __restrict__ target_mean)
{
    const int f = threadIdx.x;
    if (f >= NS) return;
    double t = 0.0;
    for (int i = 0; i < nparts; ++i) t += part[(int64_t)i * NS + f];
    if (pass == 0) {
        if (f == NF) {
            if (target_mean) *target_mean = (float)(t / (double)n);
            return;
        }
        mean[f] = t / (double)n;
        mu_sd[f] = (float)mean[f];
        return;
    }
    if (f == NF) return;
    const double sd = n >= 2 ? sqrt(t / (double)(n - 1)) : 1.0;
    mu_sd[NF + f] = (float)(sd > 1e-6 ? sd : 1e-6);
}

int budget_targets_impl(const double* label, const float* feat, int64_t n, int half, float* x_out,
                        float* y_out, int64_t* count, hipStream_t s)
{
    *count = 0;
    if (n == 0) return SRW_OK;
    const size_t tb = scan_tmp_bytes(n);
    char* ws = nullptr;
    const size_t o_pos = ((size_t)n * 4 + 255) & ~(size_t)255;
    const size_t o_tmp = o_pos + (((size_t)(n + 1) * 8 + 255) & ~(size_t)255);
    SRW_HIP(hipMallocAsync((void**)&ws, o_tmp + tb + 256, s));
    int32_t* flag = (int32_t*)ws;
    int64_t* pos = (int64_t*)(ws + o_pos);
    const unsigned g = (unsigned)grid_for(n, BLOCK);
    k_target_flags<<<g, BLOCK, 0, s>>>(n, label, flag);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = exclusive_scan_i32_to_i64(flag, pos, n, ws + o_tmp, s);
    if (e == hipSuccess) {
        k_target_scatter<<<g, BLOCK, 0, s>>>(n, label, feat, flag, pos, half, x_out, y_out);
        e = hipGetLastError();
    }
    int64_t last[1] = {0};
    int32_t lastf[1] = {0};
    if (e == hipSuccess) e = hipMemcpyAsync(last, pos + n - 1, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(lastf, flag + n - 1, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFreeAsync(ws, s);
    SRW_HIP(e);
    *count = last[0] + lastf[0];
    return SRW_OK;
}

int mlp_standardize_impl(const float* feat, const float* target, int64_t n, float* mu_sd,
                         float* target_mean, hipStream_t s)
{
    double* ws = nullptr;
    SRW_HIP(hipMallocAsync((void**)&ws, (STD_BLOCKS * NS + NF) * sizeof(double), s));
    double* mean = ws + STD_BLOCKS * NS;
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(STD_BLOCKS, (n + BLOCK - 1) / BLOCK));
    for (int pass = 0; pass < 2; ++pass) {
        k_feat_partials<<<nb, BLOCK, 0, s>>>(n, feat, target, pass ? mean : nullptr, ws);
        k_feat_finish<<<1, 64, 0, s>>>(n, nb, ws, mean, pass, mu_sd, target_mean);
    }
    hipError_t e = hipGetLastError();
    (void)hipFreeAsync(ws, s);
    SRW_HIP(e);
    return SRW_OK;
}

int budgets_impl(const float* pred, int64_t n, double eps, int32_t lo, int32_t hi, int32_t* walks,
                 hipStream_t s)
{
    if (n == 0) return SRW_OK;
    k_budgets<<<grid_for(n, BLOCK), BLOCK, 0, s>>>(n, pred, eps, lo, hi, walks);
    SRW_HIP(hipGetLastError());
    return SRW_OK;
}

}  // namespace srw
