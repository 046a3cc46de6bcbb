// Surrogate network on gfx950: BF16 matrix-core products with FP32
// accumulation for the forward and backward passes; the loss, its gradient
// (kept in BF16 for the products), the bias gradients and Adam in FP32.
// C-ABI in include/alelb_mlp.h.
//
// Every product is one kernel, k_gemm: a 256-thread workgroup (4 waves)
// computes a 64 x 64 tile of C = A B; each wave owns a 32 x 32 quarter and
// issues four v_mfma_f32_16x16x32_bf16 per 32-deep step of K.  The operands
// pass through LDS tiles KS deep in K (zeros outside the matrices); the next
// tiles' global loads are in flight while the matrix cores work on the
// current ones.  A and B are addressed through (row, column) strides, so the
// transposed operands of the backward pass need no copies: they are read as
// 8 x 8 blocks and transposed in registers.  The epilogue fuses bias + tanh
// (hidden layers), bias (output layer), or the tanh derivative together with
// the column sums the bias gradient needs; or it is a plain store.  A weight-
// gradient launch may carry one extra column of workgroups that turns those
// column sums into the bias gradient.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "alelb.h"
#include "alelb_impl.h"
#include "alelb_mlp.h"

namespace {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int TM = 64, TN = 64;  // output tile per workgroup (4 waves, 32 x 32 each)
constexpr int KSTEP = 32;        // K per MFMA
// K per LDS fill (32, 64 or 128: a tile's fill takes KS threads, eight 16-byte vectors
// each), for the products with a short K (forward, errors) and for the split
// batch-long ones (weight gradients); 32, 64 and 128 deep measured 0.875,
// 0.721 and 0.622 ms per training step at batch 65536
constexpr int KS_TALL = 128;
constexpr int KS_LONG = 128;
constexpr int GEMM_THREADS = 256;
constexpr int LDS_PAD = 8;       // row padding of the LDS tiles (bf16 elements)
constexpr int MAX_SPLIT = 64;    // K splits of the batch-long products
constexpr int ROW_CHUNK = TM;    // batch rows per bias-gradient and loss partial sum
// up to this many row chunks the weight-gradient product's launch also forms
// the bias gradients; beyond it the split sum's launch does (its per-column
// tree keeps thousands of chunks parallel)
constexpr int FUSED_BIAS_CHUNKS = 64;

enum Epilogue : int { EPI_STORE = 0, EPI_BIAS_TANH = 1, EPI_BIAS = 2, EPI_DTANH = 3 };

struct GemmArgs {
    const bf16 *A;
    long a_r, a_c;     // A(m, k) = A[m a_r + k a_c]
    const bf16 *B;
    long b_r, b_c;     // B(k, n) = B[k b_r + n b_c]
    int M, N, K;
    float *Cf;         // FP32 output C[m ldc + n] (may be null for EPI_BIAS_TANH / EPI_BIAS with Cb only)
    long ldc;
    bf16 *Cb;          // BF16 copy of the output (may be null)
    long ldcb;
    const float *bias; // [N] (EPI_BIAS_TANH, EPI_BIAS)
    const float *H;    // [M][ldh] activations whose tanh derivative scales the product (EPI_DTANH)
    long ldh;
    int kchunk;        // K per split (a multiple of the fill depth; >= K without split)
    float *part;       // split partials [splits][M][N] (split launches)
    float *colsum;     // EPI_DTANH: column sums of each 64-row tile of the result [row tiles][N] (or null)
    int a_read, b_read;  // rows of A (m) and columns of B (n) that may be read: >= M, N (0: M, N)
    // optional bias-gradient job run by one extra column of workgroups:
    // db[m] = sum over chunks c of bsrc[c][m], m < M (the weight gradients' rows)
    const float *bsrc;
    float *bdst;
    int bchunks;
    int bmode;  // 1: an extra column of the product's workgroups; 2: the split sum's launch
    int a_vec, b_vec;  // 1: the operand's tiles go through registers as 16-byte vectors
};

// h: the activation H(m, n) for EPI_DTANH (loaded by the caller)
template <int EPI>
__device__ __forceinline__ float epilogue(const GemmArgs &g, int m, int n, float v, float h = 0.0f)
{
    if (EPI == EPI_BIAS_TANH) v = tanhf(v + g.bias[n]);
    if (EPI == EPI_BIAS) v = v + g.bias[n];
    if (EPI == EPI_DTANH) v = v * (1.0f - h * h);
    if (g.Cf) g.Cf[long(m) * g.ldc + n] = v;
    if (g.Cb) g.Cb[long(m) * g.ldcb + n] = bf16(v);
    return v;
}

// How one operand's KS x 64 tile of the K range [k0, k0 + KS) is filled: X(r, k) =
// P[r sr + k sk] for rows [r0, r0 + 64), zero where k >= k_hi.  Rows up to
// nread may be read (a row beyond the matrix only feeds outputs that are not
// stored); KS threads fill the tile.  With 16-byte aligned runs and whole
// 8-element runs in range (`vec`) the tile goes through registers (v), eight
// 16-byte vectors per thread, loaded one step ahead:
//   k-fast operand (unit stride along k): 64 rows x KS/8 chunks of 8 k; lanes
//     take consecutive chunks of a row, so a wave reads whole row segments
//     and eight consecutive lanes store to distinct LDS banks;
//   transposed operand (unit stride along r): KS blocks of 8 k x 8 rows; a
//     lane loads its block's 8 k-rows and transposes the block in registers
//     into 8 rows of 8 consecutive k.
// Vectors outside the matrix read its first element instead and are zeroed.
// Other shapes are read element by element straight into LDS.
template <int KS, bool KFAST>
struct OperandTile {
    static_assert(KS % 32 == 0 && KS <= 128, "two waves fill a tile, in steps of one MFMA's K");
    const bf16 *P;
    long sr, sk;
    int r0, nread, k_hi, t;
    bool vec;
    int k0 = 0;

    __device__ __forceinline__ void load(bf16x8 (&v)[8], int k)
    {
        k0 = k;
        if (!vec || t >= KS) return;
        const bf16x8 zero = {};
        if constexpr (KFAST) {
            const int r = r0 + t / (KS / 8), kc = k0 + 8 * (t % (KS / 8));
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const bool ok = r + 8 * c < nread && kc < k_hi;
                const bf16x8 x = *reinterpret_cast<const bf16x8 *>(ok ? P + long(r + 8 * c) * sr + kc : P);
                v[c] = ok ? x : zero;
            }
        } else {
            const int kb = k0 + 8 * (t % (KS / 8)), r = r0 + 8 * (t / (KS / 8));
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const bool ok = r < nread && kb + e < k_hi;
                const bf16x8 x = *reinterpret_cast<const bf16x8 *>(ok ? P + long(kb + e) * sk + r : P);
                v[e] = ok ? x : zero;
            }
        }
    }

    // into S[64][KS + LDS_PAD], k-contiguous rows
    __device__ __forceinline__ void store(const bf16x8 (&v)[8], bf16 (*S)[KS + LDS_PAD]) const
    {
        if (t >= KS) return;
        if (!vec) {
#pragma unroll 8
            for (int x = t; x < 64 * KS; x += KS) {
                const int r = x / KS, k = x - KS * r;
                const bool ok = r0 + r < nread && k0 + k < k_hi;
                S[r][k] = ok ? P[long(r0 + r) * sr + long(k0 + k) * sk] : bf16(0.0f);
            }
            return;
        }
        if constexpr (KFAST) {
#pragma unroll
            for (int c = 0; c < 8; ++c)
                *reinterpret_cast<bf16x8 *>(&S[8 * c + t / (KS / 8)][8 * (t % (KS / 8))]) = v[c];
        } else {
            const int kb = t % (KS / 8), mb = t / (KS / 8);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                bf16x8 w;
#pragma unroll
                for (int k = 0; k < 8; ++k) w[k] = v[k][e];
                *reinterpret_cast<bf16x8 *>(&S[8 * mb + e][8 * kb]) = w;
            }
        }
    }
};

// C = A B over K range [k_lo, k_hi) of split blockIdx.z.  LDS holds both
// operands k-contiguous (sA[m][k], sB[n][k]), so each lane reads its MFMA
// operands as one 16-byte vector.  Waves 0-1 fill A, waves 2-3 fill B; AKF /
// BKF select the k-fast fill (unit stride along k), else the transposed one.
template <int EPI, bool SPLIT, int KS, bool AKF, bool BKF>
__global__ __launch_bounds__(GEMM_THREADS) void k_gemm(GemmArgs g)
{
    __shared__ bf16 sA[TM][KS + LDS_PAD];
    __shared__ bf16 sB[TN][KS + LDS_PAD];
    __shared__ float csum[2][32];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave >> 1, wc = wave & 1;
    const int row0 = blockIdx.y * TM, col0 = blockIdx.x * TN;
    if (g.bdst && g.bmode == 1 && blockIdx.x == gridDim.x - 1) {
        // the bias-gradient job: rows [row0, row0 + 64) of db, in a fixed
        // order (thread (c, q) adds chunks q, q + 4, ... of column c, then
        // the four partial sums in q order)
        if (blockIdx.z == 0) {
            const int c = tid & 63, q = tid >> 6, m = row0 + c;
            float sum = 0.0f;
            if (m < g.M)
#pragma unroll 4
                for (int ch = q; ch < g.bchunks; ch += 4) sum += g.bsrc[long(ch) * g.M + m];
            float (*bs)[64] = reinterpret_cast<float (*)[64]>(&sA[0][0]);  // the operand tiles are unused here
            bs[q][c] = sum;
            __syncthreads();
            if (q == 0 && m < g.M) g.bdst[m] = ((bs[0][c] + bs[1][c]) + bs[2][c]) + bs[3][c];
        }
        return;
    }
    const int k_lo = blockIdx.z * g.kchunk, k_hi = min(g.K, k_lo + g.kchunk);
    const bool fill_a = wave < 2;
    const int t = tid & 127;
    // A(m, k) = A[m a_r + k a_c]; B is filled as its transpose B'(n, k) = B[n b_c + k b_r]
    OperandTile<KS, AKF> opa{g.A, g.a_r, g.a_c, row0, g.a_read, k_hi, t, bool(g.a_vec)};
    OperandTile<KS, BKF> opb{g.B, g.b_c, g.b_r, col0, g.b_read, k_hi, t, bool(g.b_vec)};
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // EPI_DTANH: the activations of this lane's outputs, loaded before the K
    // loop so that their latency overlaps it
    float hv[2][2][4];
    if (EPI == EPI_DTANH && !SPLIT) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int n = col0 + 32 * wc + 16 * j + (lane & 15);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int m = row0 + 32 * wr + 16 * i + 4 * (lane >> 4) + q;
                    hv[i][j][q] = m < g.M && n < g.N ? g.H[long(m) * g.ldh + n] : 0.0f;
                }
            }
    }
    bf16x8 v[8];  // the register tile of whichever operand this wave fills
    if (k_lo < k_hi) {
        if (fill_a)
            opa.load(v, k_lo);
        else
            opb.load(v, k_lo);
    }
    for (int k0 = k_lo; k0 < k_hi; k0 += KS) {
        if (fill_a)
            opa.store(v, sA);
        else
            opb.store(v, sB);
        __syncthreads();
        if (k0 + KS < k_hi) {
            if (fill_a)
                opa.load(v, k0 + KS);
            else
                opb.load(v, k0 + KS);
        }
        // operands of v_mfma_f32_16x16x32_bf16: lane l holds A(row l%16, k 8(l/16)..+7)
        // and B(k 8(l/16)..+7, column l%16)
        const int r = lane & 15, kq = 8 * (lane >> 4);
        const int nsub = min(KS / KSTEP, (k_hi - k0 + KSTEP - 1) / KSTEP);
#pragma unroll 1
        for (int s = 0; s < nsub; ++s) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = *reinterpret_cast<const bf16x8 *>(&sA[32 * wr + 16 * i + r][KSTEP * s + kq]);
                b[i] = *reinterpret_cast<const bf16x8 *>(&sB[32 * wc + 16 * i + r][KSTEP * s + kq]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // result: lane l holds C(row 4(l/16) + q, column l%16) of each 16 x 16 block, q = 0..3
    float cs[2] = {0.0f, 0.0f};
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = col0 + 32 * wc + 16 * j + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = row0 + 32 * wr + 16 * i + 4 * (lane >> 4) + q;
                if (m >= g.M || n >= g.N) continue;
                if (SPLIT)
                    g.part[(long(blockIdx.z) * g.M + m) * g.N + n] = acc[i][j][q];
                else
                    cs[j] += epilogue<EPI>(g, m, n, acc[i][j][q], EPI == EPI_DTANH ? hv[i][j][q] : 0.0f);
            }
        }
    if (EPI == EPI_DTANH && !SPLIT && g.colsum) {
        // column sums of the tile in a fixed order: each lane's 8 rows, the
        // four lanes of a column, then the two waves of a column half
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            cs[j] += __shfl_xor(cs[j], 16);
            cs[j] += __shfl_xor(cs[j], 32);
        }
        if (wr == 1 && lane < 16) {
            csum[wc][lane] = cs[0];
            csum[wc][16 + lane] = cs[1];
        }
        __syncthreads();
        if (wr == 0 && lane < 16)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int n = col0 + 32 * wc + 16 * j + lane;
                if (n < g.N) g.colsum[long(blockIdx.y) * g.N + n] = cs[j] + csum[wc][16 * j + lane];
            }
    }
}

// db[n] = sum over the batch of dz[b][n] from the column sums of its chunks
// of ROW_CHUNK rows: one workgroup per column adds the chunks, strided over
// its threads, and reduces them as a tree (a fixed order)
__device__ __forceinline__ void bias_column(const float *part, int chunks, int n_out, int n, float *db)
{
    __shared__ float red[256];
    float s = 0.0f;
    for (int c = threadIdx.x; c < chunks; c += 256) s += part[long(c) * n_out + n];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[n] = red[0];
}

__global__ __launch_bounds__(256) void k_bias_sum(const float *part, int chunks, int n_out, float *db)
{
    bias_column(part, chunks, n_out, blockIdx.x, db);
}

// sum of the split partials in split order, then the epilogue
// (with a bias job in mode 2, workgroups beyond the sum's own each form one
// bias entry, as k_bias_sum does)
template <int EPI>
__global__ __launch_bounds__(256) void k_split_sum(GemmArgs g, int splits)
{
    const long mn = long(g.M) * g.N;
    if (g.bdst && g.bmode == 2) {
        const long own = (mn + 255) / 256;
        if (blockIdx.x >= own) {
            bias_column(g.bsrc, g.bchunks, g.M, int(blockIdx.x - own), g.bdst);
            return;
        }
    }
    const long j = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= mn) return;
    // eight loads in flight, then their sum in split order
    float v = 0.0f;
    for (int z0 = 0; z0 < splits; z0 += 8) {
        float t[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = z0 + e < splits ? g.part[(z0 + e) * mn + j] : 0.0f;
#pragma unroll
        for (int e = 0; e < 8; ++e) v += t[e];
    }
    (void)epilogue<EPI>(g, int(j / g.N), int(j % g.N), v);
}

inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

template <int EPI, bool SPLIT, int KS>
void launch_gemm(const GemmArgs &g, dim3 grid, hipStream_t st)
{
    const dim3 block(GEMM_THREADS);
    const bool akf = g.a_c == 1, bkf = g.b_r == 1;
    if (akf && bkf) hipLaunchKernelGGL((k_gemm<EPI, SPLIT, KS, true, true>), grid, block, 0, st, g);
    else if (akf) hipLaunchKernelGGL((k_gemm<EPI, SPLIT, KS, true, false>), grid, block, 0, st, g);
    else if (bkf) hipLaunchKernelGGL((k_gemm<EPI, SPLIT, KS, false, true>), grid, block, 0, st, g);
    else hipLaunchKernelGGL((k_gemm<EPI, SPLIT, KS, false, false>), grid, block, 0, st, g);
}

// one product; products with a long K (the batch) and few output tiles are
// split along K into `ws` (MAX_SPLIT x M x N floats) and summed in order
hipError_t gemm(int epi, GemmArgs g, hipStream_t st, float *ws = nullptr)
{
    // Operand tiles go through registers when runs of 8 along the unit-stride
    // dimension are 16-byte aligned (base and other stride multiples of 8
    // elements) and lie wholly inside or outside the readable range.
    if (g.a_read < g.M) g.a_read = g.M;
    if (g.b_read < g.N) g.b_read = g.N;
    g.a_vec = aligned16(g.A) && ((g.a_c == 1 && g.a_r % 8 == 0 && g.K % 8 == 0) ||
                                 (g.a_c != 1 && g.a_r == 1 && g.a_c % 8 == 0 && g.a_read % 8 == 0));
    g.b_vec = aligned16(g.B) && ((g.b_r == 1 && g.b_c % 8 == 0 && g.K % 8 == 0) ||
                                 (g.b_r != 1 && g.b_c == 1 && g.b_r % 8 == 0 && g.b_read % 8 == 0));
    const int tiles = ((g.N + TN - 1) / TN) * ((g.M + TM - 1) / TM);
    int splits = 1;
    if (ws) {
        while (splits < MAX_SPLIT && tiles * splits < 1024 && g.K / (splits * 2) >= 4 * KS_LONG) splits *= 2;
    }
    if (splits > 1) {
        g.kchunk = ((g.K / splits + KS_LONG - 1) / KS_LONG) * KS_LONG;
        splits = (g.K + g.kchunk - 1) / g.kchunk;
        const dim3 grid((g.N + TN - 1) / TN + (g.bdst && g.bmode == 1 ? 1 : 0), (g.M + TM - 1) / TM, splits);
        g.part = ws;
        launch_gemm<EPI_STORE, true, KS_LONG>(g, grid, st);
        const unsigned nb = unsigned((long(g.M) * g.N + 255) / 256) + (g.bdst && g.bmode == 2 ? g.M : 0);
        switch (epi) {
        case EPI_STORE: hipLaunchKernelGGL(k_split_sum<EPI_STORE>, dim3(nb), dim3(256), 0, st, g, splits); break;
        case EPI_BIAS_TANH: hipLaunchKernelGGL(k_split_sum<EPI_BIAS_TANH>, dim3(nb), dim3(256), 0, st, g, splits); break;
        case EPI_BIAS: hipLaunchKernelGGL(k_split_sum<EPI_BIAS>, dim3(nb), dim3(256), 0, st, g, splits); break;
        default: return hipErrorInvalidValue;  // the column sums of EPI_DTANH need whole tiles
        }
        return hipGetLastError();
    }
    g.kchunk = ((g.K + KS_TALL - 1) / KS_TALL) * KS_TALL;
    const dim3 grid((g.N + TN - 1) / TN + (g.bdst && g.bmode == 1 ? 1 : 0), (g.M + TM - 1) / TM, 1);
    if (g.bdst && g.bmode == 2) {
        // no split sum to ride in: the bias job runs on its own
        hipLaunchKernelGGL(k_bias_sum, dim3(g.M), dim3(256), 0, st, g.bsrc, g.bchunks, g.M, g.bdst);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    switch (epi) {
    case EPI_STORE: launch_gemm<EPI_STORE, false, KS_TALL>(g, grid, st); break;
    case EPI_BIAS_TANH: launch_gemm<EPI_BIAS_TANH, false, KS_TALL>(g, grid, st); break;
    case EPI_BIAS: launch_gemm<EPI_BIAS, false, KS_TALL>(g, grid, st); break;
    default: launch_gemm<EPI_DTANH, false, KS_TALL>(g, grid, st); break;
    }
    return hipGetLastError();
}

// input rows [batch][n_in] FP32 -> BF16 [batch][ld] (columns beyond n_in: zero)
__global__ void k_input_bf16(const float *x, int batch, int n_in, bf16 *xb, int ld)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= batch * ld) return;
    const int b = j / ld, c = j - ld * b;
    xb[j] = bf16(c < n_in ? x[b * n_in + c] : 0.0f);
}

// dL/dy of the mean squared error (BF16, the operand of the backward
// products), with two partial sums per chunk of ROW_CHUNK rows: of (y - t)^2
// per workgroup (FP64, thread sums then a tree), and of dL/dy per column
// (FP32, the output layer's bias gradient).  Grid: (column groups of 256, row chunks).
__global__ __launch_bounds__(256) void k_mse_grad(const float *y, const float *t, int batch, int n_y, float scale,
                                                  bf16 *dyb, double *partial, float *colsum)
{
    __shared__ double red[256];
    const int n = blockIdx.x * 256 + threadIdx.x;
    const int b0 = blockIdx.y * ROW_CHUNK, b1 = min(batch, b0 + ROW_CHUNK);
    double s = 0.0;
    if (n < n_y) {
        float cs = 0.0f;
#pragma unroll 8
        for (int b = b0; b < b1; ++b) {
            const long j = long(b) * n_y + n;
            const float d = y[j] - t[j];
            s += double(d) * double(d);
            const float gj = scale * d;
            dyb[j] = bf16(gj);
            cs += gj;
        }
        colsum[long(blockIdx.y) * n_y + n] = cs;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// the loss from k_mse_grad's block partials, in a fixed order: thread t adds
// partials t, t + 256, ... in turn, the 256 sums reduce as a tree, and the
// total is divided by the element count (one workgroup of 256 threads)
__global__ __launch_bounds__(256) void k_loss_sum(const double *partial, int nb, double n, double *out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += partial[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] / n;
}

// layers' places in the packed parameters, for the BF16 weight copies
constexpr int MAX_LAYERS = 16;
struct LayerMap {
    long off[MAX_LAYERS + 1];  // first parameter of layer l (W_l then b_l); off[L] = total
    int n_in[MAX_LAYERS], n_out[MAX_LAYERS], ld[MAX_LAYERS];
    bf16 *Wb[MAX_LAYERS];
    int L;
};

// Adam on FP32 master parameters; the new weights also go to their BF16 copies
// With lout, workgroup 0 first forms the step's loss from k_mse_grad's nb
// partials, as k_loss_sum does (same order), into *lout.
__global__ __launch_bounds__(256) void k_adam(float *p, const float *g, float *m1, float *m2, int n, float lr,
                                              float b1, float b2, float eps, float c1, float c2, LayerMap lm,
                                              const double *partial, int nb, double count, double *lout)
{
    if (lout && blockIdx.x == 0) {
        __shared__ double red[256];
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += 256) s += partial[b];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) *lout = red[0] / count;
    }
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float gj = g[j];
    const float a = b1 * m1[j] + (1.0f - b1) * gj;
    const float v = b2 * m2[j] + (1.0f - b2) * gj * gj;
    m1[j] = a;
    m2[j] = v;
    const float pj = p[j] - lr * (a / c1) / (sqrtf(v / c2) + eps);
    p[j] = pj;
    int l = 0;
    while (l + 1 < lm.L && j >= lm.off[l + 1]) ++l;
    const long w = j - lm.off[l];
    if (w < long(lm.n_out[l]) * lm.n_in[l]) {
        const int r = int(w / lm.n_in[l]), c = int(w - long(r) * lm.n_in[l]);
        lm.Wb[l][long(r) * lm.ld[l] + c] = bf16(pj);
    }
}

// BF16 copy of W [n_out][n_in] with rows padded to ld columns of zeros
__global__ void k_weights_bf16(const float *W, int n_out, int n_in, bf16 *Wb, int ld)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_out * ld) return;
    const int r = j / ld, c = j - ld * r;
    Wb[j] = bf16(c < n_in ? W[r * n_in + c] : 0.0f);
}

inline unsigned blocks(long n, int t = 256) { return unsigned((n + t - 1) / t); }
inline int pad32(int n) { return (n + 31) & ~31; }

}  // namespace

using alelb::report_error;

#define HIP_OK(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return report_error(e_ == hipErrorOutOfMemory ? ALE_LB_ENOMEM : ALE_LB_EDEVICE, "%s: %s", #expr, \
                                hipGetErrorString(e_));                                                \
    } while (0)

constexpr int LOSS_CHUNK = 1024;  // ale_mlp_train_steps: steps between loss copies to the host

struct ale_mlp {
    std::vector<int> w;        // widths
    std::vector<int> ld;       // padded widths (multiples of 32), BF16 row lengths
    std::vector<long> poff;    // offset of layer l's W in the packed parameters; b follows W
    long np = 0;               // number of parameters
    int L = 0, max_batch = 0;
    long steps = 0;
    hipStream_t st = nullptr;
    std::vector<void *> bufs;
    float *p = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;  // [np]
    std::vector<bf16 *> Wb;    // [L] BF16 W_l [w_{l+1}][ld_l]
    std::vector<float *> Hf;   // [L+1] FP32 activations [max_batch][w_l] (Hf[0] unused)
    std::vector<bf16 *> Hb;    // [L+1] BF16 activations [max_batch][ld_l]
    bf16 *dzb = nullptr, *dzb2 = nullptr;   // back-propagated errors [max_batch][max width]
    float *xin = nullptr, *tin = nullptr;   // staged host batches
    double *partial = nullptr;  // loss partial sums [row chunks][column groups]
    double *dloss = nullptr;  // per-step losses of ale_mlp_train_steps [LOSS_CHUNK]
    float *bpart = nullptr;   // bias-gradient column sums [row chunks][max width]
    float *ws = nullptr;      // split-K partials of the weight gradients [MAX_SPLIT][max width]^2

    template <typename T>
    T *alloc(size_t n, int *status)
    {
        void *q = nullptr;
        const hipError_t e = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
        if (e != hipSuccess) {
            *status = report_error(e == hipErrorOutOfMemory ? ALE_LB_ENOMEM : ALE_LB_EDEVICE, "hipMalloc: %s",
                                   hipGetErrorString(e));
            return nullptr;
        }
        bufs.push_back(q);
        return static_cast<T *>(q);
    }
    ~ale_mlp()
    {
        for (void *q : bufs) (void)hipFree(q);
    }
};

namespace {

int refresh_bf16_weights(ale_mlp *h)
{
    for (int l = 0; l < h->L; ++l) {
        const int n_out = h->w[l + 1], n_in = h->w[l];
        hipLaunchKernelGGL(k_weights_bf16, dim3(blocks(long(n_out) * h->ld[l])), dim3(256), 0, h->st,
                           h->p + h->poff[l], n_out, n_in, h->Wb[l], h->ld[l]);
    }
    HIP_OK(hipGetLastError());
    return ALE_LB_OK;
}

// forward pass of `batch` rows already in Hb[0]; leaves the output in Hf[L]
int forward(ale_mlp *h, int batch)
{
    for (int l = 0; l < h->L; ++l) {
        const int n_out = h->w[l + 1];
        const bool last = l == h->L - 1;
        GemmArgs a{};
        a.A = h->Hb[l];
        a.a_r = h->ld[l];
        a.a_c = 1;
        a.B = h->Wb[l];  // B(k, n) = W[n][k]
        a.b_r = 1;
        a.b_c = h->ld[l];
        a.M = batch;
        a.N = n_out;
        a.K = h->ld[l];
        a.Cf = h->Hf[l + 1];
        a.ldc = n_out;
        a.Cb = last ? nullptr : h->Hb[l + 1];
        a.ldcb = h->ld[l + 1];
        a.bias = h->p + h->poff[l] + long(n_out) * h->w[l];
        HIP_OK(gemm(last ? EPI_BIAS : EPI_BIAS_TANH, a, h->st));
    }
    return ALE_LB_OK;
}

// loss gradient and back-propagation for targets in tin; gradients into h->g
int backward(ale_mlp *h, int batch, const float *t, double *loss, double *dloss = nullptr)
{
    const int L = h->L, n_y = h->w[L];
    const long ny = long(batch) * n_y;
    const int chunks = (batch + ROW_CHUNK - 1) / ROW_CHUNK;
    const dim3 lgrid(blocks(n_y), chunks);
    const int nb = int(lgrid.x * lgrid.y);
    hipLaunchKernelGGL(k_mse_grad, lgrid, dim3(256), 0, h->st, h->Hf[L], t, batch, n_y, 2.0f / float(ny), h->dzb,
                       h->partial, h->bpart);
    HIP_OK(hipGetLastError());
    bf16 *dzb = h->dzb, *dzb_next = h->dzb2;
    for (int l = L - 1; l >= 0; --l) {
        const int n_out = h->w[l + 1], n_in = h->w[l];
        // dW_l [n_out][n_in] = dZ^T X (A(m, k) = dZ[k][m], B(k, n) = X[k][n]); its
        // launches also form db_l from the column sums of dZ_l's row chunks
        // (h->bpart): in the product's extra column for few chunks, else in the
        // split sum's launch
        GemmArgs a{};
        a.A = dzb;
        a.a_r = 1;
        a.a_c = n_out;
        a.B = h->Hb[l];
        a.b_r = h->ld[l];
        a.b_c = 1;
        a.M = n_out;
        a.N = n_in;
        a.b_read = h->ld[l];  // BF16 activations are padded with zeros to ld columns
        a.K = batch;
        a.Cf = h->g + h->poff[l];
        a.ldc = n_in;
        a.bsrc = h->bpart;
        a.bdst = h->g + h->poff[l] + long(n_out) * n_in;
        a.bchunks = chunks;
        a.bmode = chunks <= FUSED_BIAS_CHUNKS ? 1 : 2;
        HIP_OK(gemm(EPI_STORE, a, h->st, h->ws));
        if (l == 0) break;
        // dZ_{l-1} [batch][n_in] = (dZ_l W_l) * (1 - H_l^2), with its column sums per row chunk:
        // A = dZ [batch][n_out], B(k, n) = W[k][n]
        GemmArgs b{};
        b.A = dzb;
        b.a_r = n_out;
        b.a_c = 1;
        b.B = h->Wb[l];
        b.b_r = h->ld[l];
        b.b_c = 1;
        b.M = batch;
        b.N = n_in;
        b.b_read = h->ld[l];  // BF16 weights are padded with zeros to ld columns
        b.K = n_out;
        b.Cb = dzb_next;
        b.ldcb = n_in;
        b.H = h->Hf[l];
        b.ldh = n_in;
        b.colsum = h->bpart;
        HIP_OK(gemm(EPI_DTANH, b, h->st));
        std::swap(dzb, dzb_next);
    }
    // the loss goes to the device slot dloss, or through slot 0 to the host
    if (dloss || loss) {
        double *slot = dloss ? dloss : h->dloss;
        hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(256), 0, h->st, h->partial, nb, double(ny), slot);
        HIP_OK(hipGetLastError());
        if (loss) {
            HIP_OK(hipMemcpyAsync(loss, slot, sizeof(double), hipMemcpyDeviceToHost, h->st));
            HIP_OK(hipStreamSynchronize(h->st));
        }
    }
    return ALE_LB_OK;
}

// stage a batch: x into Hb[0] (BF16, padded), t (if any) into tin; returns the device target pointer
int stage(ale_mlp *h, const float *x, const float *t, int batch, int on_device, const float **td)
{
    if (batch < 1 || batch > h->max_batch)
        return report_error(ALE_LB_EINVAL, "batch %d outside 1..%d", batch, h->max_batch);
    const float *xd = x;
    if (!on_device) {
        HIP_OK(hipMemcpyAsync(h->xin, x, sizeof(float) * batch * h->w[0], hipMemcpyHostToDevice, h->st));
        xd = h->xin;
    }
    hipLaunchKernelGGL(k_input_bf16, dim3(blocks(long(batch) * h->ld[0])), dim3(256), 0, h->st, xd, batch, h->w[0],
                       h->Hb[0], h->ld[0]);
    HIP_OK(hipGetLastError());
    if (t && td) {
        *td = t;
        if (!on_device) {
            HIP_OK(hipMemcpyAsync(h->tin, t, sizeof(float) * batch * h->w[h->L], hipMemcpyHostToDevice, h->st));
            *td = h->tin;
        }
    }
    return ALE_LB_OK;
}

bool adam_args_ok(float lr, float beta1, float beta2, float eps)
{
    return lr > 0.0f && beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f;
}

// one Adam step (Kingma & Ba) on the gradients in h->g; also refreshes the BF16
// weights, and with lout puts the loss of the step's `batch` rows there
int adam(ale_mlp *h, float lr, float beta1, float beta2, float eps, int batch = 0, double *lout = nullptr)
{
    h->steps += 1;
    const float c1 = 1.0f - std::pow(beta1, float(h->steps)), c2 = 1.0f - std::pow(beta2, float(h->steps));
    LayerMap lm{};
    lm.L = h->L;
    for (int l = 0; l < h->L; ++l) {
        lm.off[l] = h->poff[l];
        lm.n_in[l] = h->w[l];
        lm.n_out[l] = h->w[l + 1];
        lm.ld[l] = h->ld[l];
        lm.Wb[l] = h->Wb[l];
    }
    lm.off[h->L] = h->np;
    const int n_y = h->w[h->L];
    const int nb = int(blocks(n_y)) * ((batch + ROW_CHUNK - 1) / ROW_CHUNK);
    hipLaunchKernelGGL(k_adam, dim3(blocks(h->np)), dim3(256), 0, h->st, h->p, h->g, h->m1, h->m2, int(h->np), lr,
                       beta1, beta2, eps, c1, c2, lm, h->partial, nb, double(long(batch) * n_y), lout);
    HIP_OK(hipGetLastError());
    return ALE_LB_OK;
}

}  // namespace

extern "C" {

int ale_mlp_create(const int32_t *widths, int32_t n_widths, int32_t max_batch, void *stream, ale_mlp_t **out)
{
    if (!widths || !out || n_widths < 2 || n_widths > MAX_LAYERS + 1 || max_batch < 1)
        return report_error(ALE_LB_EINVAL, "bad network shape");
    // batch row tiles run along the grids' y dimension
    if (max_batch > 65535 * ROW_CHUNK)
        return report_error(ALE_LB_EINVAL, "max_batch %d above %d", max_batch, 65535 * ROW_CHUNK);
    for (int l = 0; l < n_widths; ++l)
        if (widths[l] < 1 || widths[l] > 4096) return report_error(ALE_LB_EINVAL, "layer width %d outside 1..4096", widths[l]);
    *out = nullptr;
    ale_mlp *h = new ale_mlp();
    h->w.assign(widths, widths + n_widths);
    h->L = n_widths - 1;
    h->max_batch = max_batch;
    h->st = static_cast<hipStream_t>(stream);
    int wmax = 0;
    for (int l = 0; l < n_widths; ++l) {
        h->ld.push_back(pad32(widths[l]));
        wmax = std::max(wmax, pad32(widths[l]));
    }
    for (int l = 0; l < h->L; ++l) {
        h->poff.push_back(h->np);
        h->np += long(widths[l + 1]) * (widths[l] + 1);
    }
    int st = ALE_LB_OK;
    h->p = h->alloc<float>(h->np, &st);
    h->g = h->alloc<float>(h->np, &st);
    h->m1 = h->alloc<float>(h->np, &st);
    h->m2 = h->alloc<float>(h->np, &st);
    for (int l = 0; l < h->L && !st; ++l) h->Wb.push_back(h->alloc<bf16>(size_t(widths[l + 1]) * h->ld[l], &st));
    for (int l = 0; l <= h->L && !st; ++l) {
        h->Hf.push_back(l ? h->alloc<float>(size_t(max_batch) * widths[l], &st) : nullptr);
        h->Hb.push_back(h->alloc<bf16>(size_t(max_batch) * h->ld[l], &st));
    }
    h->dzb = h->alloc<bf16>(size_t(max_batch) * wmax, &st);
    h->dzb2 = h->alloc<bf16>(size_t(max_batch) * wmax, &st);
    h->xin = h->alloc<float>(size_t(max_batch) * widths[0], &st);
    h->tin = h->alloc<float>(size_t(max_batch) * widths[h->L], &st);
    const size_t chunks = size_t(max_batch + ROW_CHUNK - 1) / ROW_CHUNK;
    h->bpart = h->alloc<float>(chunks * wmax, &st);
    h->ws = h->alloc<float>(size_t(MAX_SPLIT) * wmax * wmax, &st);
    h->partial = h->alloc<double>(chunks * blocks(widths[h->L]), &st);
    h->dloss = h->alloc<double>(LOSS_CHUNK, &st);
    if (st) {
        delete h;
        return st;
    }
    // parameters, moments, activations and padding start at zero
    hipError_t e = hipSuccess;
    for (float *q : {h->p, h->g, h->m1, h->m2})
        if (e == hipSuccess) e = hipMemsetAsync(q, 0, sizeof(float) * h->np, h->st);
    for (int l = 0; l <= h->L && e == hipSuccess; ++l)
        e = hipMemsetAsync(h->Hb[l], 0, sizeof(bf16) * size_t(max_batch) * h->ld[l], h->st);
    for (int l = 0; l < h->L && e == hipSuccess; ++l)
        e = hipMemsetAsync(h->Wb[l], 0, sizeof(bf16) * size_t(widths[l + 1]) * h->ld[l], h->st);
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    if (e != hipSuccess) {
        delete h;
        return report_error(ALE_LB_EDEVICE, "network set-up: %s", hipGetErrorString(e));
    }
    *out = h;
    return ALE_LB_OK;
}

void ale_mlp_destroy(ale_mlp_t *h)
{
    if (h) {
        (void)hipStreamSynchronize(h->st);
        delete h;
    }
}

int ale_mlp_info(ale_mlp_t *h, int64_t *out, int32_t n)
{
    if (!h || !out) return report_error(ALE_LB_EINVAL, "null argument");
    const int64_t v[2] = {h->np, h->steps};
    for (int k = 0; k < n && k < 2; ++k) out[k] = v[k];
    return ALE_LB_OK;
}

int ale_mlp_set_params(ale_mlp_t *h, const float *params, int64_t n)
{
    if (!h || !params || n != h->np) return report_error(ALE_LB_EINVAL, "expected %ld parameters", h ? h->np : 0L);
    HIP_OK(hipMemcpyAsync(h->p, params, sizeof(float) * n, hipMemcpyHostToDevice, h->st));
    HIP_OK(hipMemsetAsync(h->m1, 0, sizeof(float) * n, h->st));
    HIP_OK(hipMemsetAsync(h->m2, 0, sizeof(float) * n, h->st));
    h->steps = 0;
    const int st = refresh_bf16_weights(h);
    if (st) return st;
    HIP_OK(hipStreamSynchronize(h->st));
    return ALE_LB_OK;
}

int ale_mlp_get_params(ale_mlp_t *h, float *params, int64_t n)
{
    if (!h || !params || n != h->np) return report_error(ALE_LB_EINVAL, "expected %ld parameters", h ? h->np : 0L);
    HIP_OK(hipMemcpyAsync(params, h->p, sizeof(float) * n, hipMemcpyDeviceToHost, h->st));
    HIP_OK(hipStreamSynchronize(h->st));
    return ALE_LB_OK;
}

int ale_mlp_forward(ale_mlp_t *h, const float *x, int32_t batch, float *y, int32_t on_device)
{
    if (!h || !x || !y) return report_error(ALE_LB_EINVAL, "null argument");
    int st = stage(h, x, nullptr, batch, on_device, nullptr);
    if (!st) st = forward(h, batch);
    if (st) return st;
    const size_t bytes = sizeof(float) * size_t(batch) * h->w[h->L];
    HIP_OK(hipMemcpyAsync(y, h->Hf[h->L], bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->st));
    HIP_OK(hipStreamSynchronize(h->st));
    return ALE_LB_OK;
}

int ale_mlp_gradients(ale_mlp_t *h, const float *x, const float *t, int32_t batch, float *grads, double *loss,
                      int32_t on_device)
{
    if (!h || !x || !t || !grads) return report_error(ALE_LB_EINVAL, "null argument");
    const float *td = nullptr;
    int st = stage(h, x, t, batch, on_device, &td);
    if (!st) st = forward(h, batch);
    if (!st) st = backward(h, batch, td, loss);
    if (st) return st;
    HIP_OK(hipMemcpyAsync(grads, h->g, sizeof(float) * h->np, hipMemcpyDeviceToHost, h->st));
    HIP_OK(hipStreamSynchronize(h->st));
    return ALE_LB_OK;
}

int ale_mlp_train_step(ale_mlp_t *h, const float *x, const float *t, int32_t batch, float lr, float beta1,
                       float beta2, float eps, double *loss, int32_t on_device)
{
    if (!h || !x || !t) return report_error(ALE_LB_EINVAL, "null argument");
    if (!adam_args_ok(lr, beta1, beta2, eps)) return report_error(ALE_LB_EINVAL, "bad Adam hyper-parameters");
    const float *td = nullptr;
    int st = stage(h, x, t, batch, on_device, &td);
    if (!st) st = forward(h, batch);
    if (!st) st = backward(h, batch, td, nullptr);
    if (!st) st = adam(h, lr, beta1, beta2, eps, batch, loss ? h->dloss : nullptr);
    if (st) return st;
    if (loss) HIP_OK(hipMemcpyAsync(loss, h->dloss, sizeof(double), hipMemcpyDeviceToHost, h->st));
    HIP_OK(hipStreamSynchronize(h->st));
    return ALE_LB_OK;
}

int ale_mlp_train_steps(ale_mlp_t *h, const float *x, const float *t, int32_t batch, int32_t n, const float *lr,
                        float beta1, float beta2, float eps, double *losses, int32_t on_device)
{
    if (!h || !x || !t || !lr) return report_error(ALE_LB_EINVAL, "null argument");
    if (n < 1) return report_error(ALE_LB_EINVAL, "step count %d < 1", n);
    for (int k = 0; k < n; ++k)
        if (!adam_args_ok(lr[k], beta1, beta2, eps))
            return report_error(ALE_LB_EINVAL, "bad Adam hyper-parameters (step %d)", k);
    const float *td = nullptr;
    int st = stage(h, x, t, batch, on_device, &td);
    if (st) return st;
    for (int k0 = 0; k0 < n; k0 += LOSS_CHUNK) {
        const int kn = std::min(n - k0, LOSS_CHUNK);
        for (int k = 0; k < kn; ++k) {
            st = forward(h, batch);
            if (!st) st = backward(h, batch, td, nullptr);
            if (!st) st = adam(h, lr[k0 + k], beta1, beta2, eps, batch, h->dloss + k);
            if (st) return st;
        }
        if (losses)
            HIP_OK(hipMemcpyAsync(losses + k0, h->dloss, sizeof(double) * kn, hipMemcpyDeviceToHost, h->st));
        HIP_OK(hipStreamSynchronize(h->st));
    }
    return ALE_LB_OK;
}

int ale_mlp_gemm_bf16(const uint16_t *A, const uint16_t *B, float *C, int32_t M, int32_t N, int32_t K)
{
    if (!A || !B || !C || M < 1 || N < 1 || K < 1) return report_error(ALE_LB_EINVAL, "bad product shape");
    GemmArgs g{};
    g.A = reinterpret_cast<const bf16 *>(A);
    g.a_r = K;
    g.a_c = 1;
    g.B = reinterpret_cast<const bf16 *>(B);
    g.b_r = N;
    g.b_c = 1;
    g.M = M;
    g.N = N;
    g.K = K;
    g.Cf = C;
    g.ldc = N;
    HIP_OK(gemm(EPI_STORE, g, nullptr));
    HIP_OK(hipStreamSynchronize(nullptr));
    return ALE_LB_OK;
}

}  // extern "C"
