// MLP surrogate of the generators: parameters -> graph statistics.
//
// d_in -> width -> ... -> width -> d_out, `hidden` SiLU layers, the output
// layer linear.  Master parameters are float32; every GEMM reads its weights
// and its input activations rounded to bfloat16 (round to nearest even) and
// accumulates in float32 on the matrix cores (v_mfma_f32_16x16x32_bf16).
// Biases, pre-activations, activations and every gradient stay float32.
// Rounding points:
//   forward   Xb_0 = bf16(x); Z_l = Xb_l Wb_l^T + b_l; Xb_{l+1} = bf16(SiLU(Z_l))
//   backward  dZb_l = bf16(dZ_l); dW_l = dZb_l^T Xb_l; db_l = sum_b dZ_l;
//             dH_{l-1} = dZb_l Wb_l; dZ_{l-1} = dH_{l-1} * SiLU'(Z_{l-1})
// with Wb_l = bf16(W_l).  Parameter layout: for each layer, W (out x in,
// row-major) then b (out).
#include <math.h>
#include <string.h>

#include <algorithm>

#include "common.hpp"

namespace sfg {
namespace {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

constexpr int kTile = 64;   // block tile (M and N)
constexpr int kKStep = 32;  // K per MFMA step
constexpr int kPad = 8;     // LDS row padding (bf16 elements)

// float -> bfloat16, round to nearest even (NaN stays NaN): the conversion
// instruction of the matrix-core generation (v_cvt_pk_bf16_f32, which rounds
// in the wave's rounding mode, nearest even by default).
__device__ __forceinline__ bf16 f2bf(float f) { return (bf16)f; }
__device__ __forceinline__ float bf2f(bf16 h) {
    const uint16_t b = __builtin_bit_cast(uint16_t, h);
    return __uint_as_float((uint32_t)b << 16);
}

// Stage rows [r0, r0 + 64) x k in [k0, k0 + 32) of an operand into an LDS
// tile t[row][k] (bf16, 16-byte rows chunks).  KMAJ: element (row, k) is
// X[row * ld + k] (k contiguous); else X[k * ld + row] (rows contiguous).
// Each of the 256 threads moves one 8-element vector when the vector lies
// inside the operand and the layout allows 16-byte loads (vec); elements
// outside [0, R) x [k0, ke) read as zero.
template <bool KMAJ>
__device__ __forceinline__ void stage_tile(const bf16 *__restrict__ X, int ld, int R, int r0, int k0, int ke, bool vec,
                                           bf16 (*t)[kKStep + kPad]) {
    const int tid = threadIdx.x;
    const bf16 zero = f2bf(0.f);
    if (KMAJ) {
        const int r = tid / 4, k8 = (tid % 4) * 8;
        const int gr = r0 + r, gk = k0 + k8;
        bf16x8 v;
        if (vec && gr < R && gk + 8 <= ke) {
            v = *reinterpret_cast<const bf16x8 *>(X + (size_t)gr * ld + gk);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = (gr < R && gk + e < ke) ? X[(size_t)gr * ld + gk + e] : zero;
        }
        *reinterpret_cast<bf16x8 *>(&t[r][k8]) = v;
    } else {
        const int k = tid / 8, r8 = (tid % 8) * 8;
        const int gk = k0 + k, gr = r0 + r8;
        bf16x8 v;
        if (vec && gk < ke && gr + 8 <= R) {
            v = *reinterpret_cast<const bf16x8 *>(X + (size_t)gk * ld + gr);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = (gk < ke && gr + e < R) ? X[(size_t)gk * ld + gr + e] : zero;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) t[r8 + e][k] = v[e];
    }
}

// C[M][N] (+)= sum_k A(m, k) B(k, n) over k in [k_begin, k_end), with
// A(m, k) = TA ? A[k * lda + m] : A[m * lda + k] and
// B(k, n) = TB ? B[n * ldb + k] : B[k * ldb + n]; bf16 in, fp32 out.
// Block: 256 threads, a 64 x 64 tile; wave w owns rows 32 (w / 2) .. +32 and
// columns 32 (w % 2) .. +32 as 2 x 2 MFMA 16 x 16 tiles.  Split-K: blockIdx.z
// selects a K range and a partial output C + z * M * N.  veca / vecb: the
// operand allows 16-byte loads (8-element aligned base and leading dimension).
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_bf16(const bf16 *__restrict__ A, int lda, const bf16 *__restrict__ B,
                                                 int ldb, float *__restrict__ C, int M, int N, int K, int ksplit,
                                                 int veca, int vecb) {
    __shared__ __align__(16) bf16 sA[kTile][kKStep + kPad];  // [m][k]
    __shared__ __align__(16) bf16 sB[kTile][kKStep + kPad];  // [n][k]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
    const int kper = ((K + ksplit - 1) / ksplit + kKStep - 1) / kKStep * kKStep;
    const int kb = blockIdx.z * kper, ke = std::min(K, kb + kper);
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += kKStep) {
        stage_tile<!TA>(A, lda, M, m0, k0, ke, veca != 0, sA);
        stage_tile<TB>(B, ldb, N, n0, k0, ke, vecb != 0, sB);
        __syncthreads();
        // 16x16x32 operands: lane l holds row/col (l % 16), k = 8 (l / 16) .. +7.
        const int r = lane % 16, kq = 8 * (lane / 16);
        bf16x8 fa[2], fb[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) fa[i] = *reinterpret_cast<const bf16x8 *>(&sA[32 * (w / 2) + 16 * i + r][kq]);
#pragma unroll
        for (int j = 0; j < 2; ++j) fb[j] = *reinterpret_cast<const bf16x8 *>(&sB[32 * (w % 2) + 16 * j + r][kq]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // Result: lane l holds rows 4 (l / 16) .. +3 and column l % 16 of each tile.
    float *Cz = C + (size_t)blockIdx.z * M * N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gm = m0 + 32 * (w / 2) + 16 * i + 4 * (lane / 16) + e;
                const int gn = n0 + 32 * (w % 2) + 16 * j + lane % 16;
                if (gm < M && gn < N) Cz[(size_t)gm * N + gn] = acc[i][j][e];
            }
}

// 1 / (1 + e^-z) with the hardware exponential (2^x of z log2 e) and
// reciprocal: relative error a few float32 ulps, far below the bf16 rounding
// applied to every activation; saturates to exactly 0 and 1.
__device__ __forceinline__ float sigmoidf_(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

// bf16 copy of every weight matrix of the parameter vector.
__global__ void round_weights(const float *p, bf16 *wb, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        wb[i] = f2bf(p[i]);
}

__global__ void round_input(const float *x, bf16 *xb, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        xb[i] = f2bf(x[i]);
}

// Z = acc + b (stored), then SiLU -> bf16 next input (hidden) or Y (output).
__global__ void bias_act(const float *acc, const float *b, float *Z, bf16 *Xnext, float *Y, int rows, int cols) {
    const uint64_t n = (uint64_t)rows * cols;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const float z = acc[i] + b[i % cols];
        if (Z) Z[i] = z;
        if (Xnext) Xnext[i] = f2bf(z * sigmoidf_(z));
        if (Y) Y[i] = z;
    }
}

// dZ = dH * SiLU'(Z) (or dZ = dY for the output layer when Z is null);
// writes the fp32 dZ and its bf16 copy.
__global__ void act_grad(const float *dH, const float *Z, float *dZ, bf16 *dZb, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        float g = dH[i];
        if (Z) {
            const float z = Z[i], s = sigmoidf_(z);
            g *= s * (1.0f + z * (1.0f - s));
        }
        dZ[i] = g;
        dZb[i] = f2bf(g);
    }
}

// Column sums db[c] = sum_r dZ[r][c] in a fixed order, in two passes so that
// no thread walks the whole batch: pass 1 sums row chunk blockIdx.y of 64
// columns (four row lanes per column, interleaved rows, combined in lane
// order) into part[chunk][c]; pass 2 sums the chunks the same way.
constexpr int kColChunks = 64;

__device__ __forceinline__ void col_sum_lanes(const float *v, int rows, int cols, int r0, int r1, float *out) {
    __shared__ float s[4][64];
    const int cl = threadIdx.x % 64, q = threadIdx.x / 64;
    const int c = blockIdx.x * 64 + cl;
    float acc = 0.f;
    if (c < cols)
        for (int r = r0 + q; r < r1; r += 4) acc += v[(size_t)r * cols + c];
    s[q][cl] = acc;
    __syncthreads();
    if (q == 0 && c < cols) *out = ((s[0][cl] + s[1][cl]) + s[2][cl]) + s[3][cl];
}

__global__ __launch_bounds__(256) void col_sums_chunks(const float *dZ, int rows, int cols, int chunk_rows,
                                                       float *part) {
    const int r0 = blockIdx.y * chunk_rows, r1 = min(rows, r0 + chunk_rows);
    const int c = blockIdx.x * 64 + threadIdx.x % 64;
    float tmp;
    col_sum_lanes(dZ, r1, cols, r0, r1, &tmp);
    if (threadIdx.x < 64 && c < cols) part[(size_t)blockIdx.y * cols + c] = tmp;
}

__global__ __launch_bounds__(256) void col_sums_total(const float *part, int chunks, int cols, float *db) {
    const int c = blockIdx.x * 64 + threadIdx.x % 64;
    float tmp;
    col_sum_lanes(part, chunks, cols, 0, chunks, &tmp);
    if (threadIdx.x < 64 && c < cols) db[c] = tmp;
}

// out[i] = sum over the split-K partials, in split order.
__global__ void reduce_splits(const float *part, int splits, uint64_t n, float *out) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        float acc = 0.f;
        for (int z = 0; z < splits; ++z) acc += part[(uint64_t)z * n + i];
        out[i] = acc;
    }
}

// Weighted squared error: loss = sum_{b,j} w_j mask_bj (y_bj - t_bj)^2 / B,
// dy = 2 w_j mask_bj (y_bj - t_bj) / B.  Per-row partial losses, then a
// single-block sum in row order.
__global__ void mse_grad(const float *y, const float *t, const float *mask, const float *cw, int B, int D, float *dy,
                         float *row_loss) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float acc = 0.f;
    for (int j = 0; j < D; ++j) {
        const size_t i = (size_t)b * D + j;
        const float wgt = (cw ? cw[j] : 1.f) * (mask ? mask[i] : 1.f);
        const float d = y[i] - t[i];
        dy[i] = wgt == 0.f ? 0.f : 2.f * wgt * d / (float)B;
        acc += wgt == 0.f ? 0.f : wgt * d * d;
    }
    row_loss[b] = acc / (float)B;
}

__global__ void sum_rows(const float *v, int n, float *out) {
    __shared__ float s[256];
    float acc = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) acc += v[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

__global__ void adam_kernel(uint64_t n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// Device-driven Adam: one thread advances the step counter, then every
// element reads the step and the learning rate from memory.
__global__ void adam_tick(uint32_t *step) { *step += 1; }

__global__ void adam_kernel_dev(uint64_t n, float *p, const float *g, float *m, float *v, const float *lr_p,
                                float b1, float b2, float eps, const uint32_t *step_p) {
    const float t = (float)*step_p, lr = *lr_p;
    const float c1 = 1.f - powf(b1, t), c2 = 1.f - powf(b2, t);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}


// ----------------------------------------------------------------------------- fused training step
// One training step in four launches.  mlp_round writes the bf16 weights,
// row-major and transposed.  mlp_rows runs, for a block of 64 rows, the
// forward pass, the loss gradient and the whole backward chain of activation
// gradients -- all of it row-local -- on the matrix cores, keeping the
// current layer's bf16 operand in LDS; it leaves the bf16 layer inputs, the
// bf16 gradients dZb and per-block column sums of dZ.  mlp_wgrad computes
// every weight-gradient tile over a 256-row slice of the batch (dW = dZb^T
// Xb) into per-slice partials; mlp_update sums the partials and the
// per-block bias sums in a fixed order, applies Adam and sums the loss.  The
// rounding points are those of mlp_forward / mlp_backward.
//
// The saved activations are feature-major, [feature][Bp], with the feature
// count padded to a multiple of 16 and the batch to Bp, a multiple of 64:
// a lane's four consecutive rows of one feature (the matrix-core output
// layout) are one vector store, the weight-gradient operands (contiguous in
// the batch) are direct fragment loads, and every element of the padding is
// written by every step -- zero in Xb and dZb for rows beyond the batch and
// features beyond the layer, so that they add exact zeros to dW.
constexpr int kFR = 64;       // rows per block of mlp_rows
constexpr int kFMax = 256;    // widest layer the fused step takes
constexpr int kFMaxL = 8;     // deepest network the fused step takes
constexpr int kWSlice = 256;  // batch rows per weight-gradient partial
constexpr int kRW = 8;        // waves per block of mlp_rows
constexpr int kCT = 2;        // column tiles per wave of mlp_rows

struct TrainArgs {
    int L, B, Bp;          // Bp: the batch rounded up to kFR
    int dims[kFMaxL + 1];  // dims[0] = d_in, dims[l + 1] = outputs of layer l
    size_t w_off[kFMaxL], b_off[kFMaxL];
    float *params;
    // bf16 weights of layer l, zero-padded: wb + wp_off[l] is [pad16(out)][pad32(in)],
    // wbt + wtp_off[l] is [pad16(in)][pad32(out)] (W transposed)
    const bf16 *wb, *wbt;
    size_t wp_off[kFMaxL], wtp_off[kFMaxL];
    const float *x, *target, *mask, *cw;
    const int64_t *rows;  // batch row r is row rows[r] of x, target and mask (null: row r)
    bf16 *xb[kFMaxL];     // [pad16(dims[l])][Bp] layer inputs
    float *z[kFMaxL];     // [pad16(dims[l + 1])][Bp] pre-activations (hidden layers)
    bf16 *dzb[kFMaxL];    // [pad16(dims[l + 1])][Bp]
    float *dbp[kFMaxL];   // [blocks][dims[l + 1]] column sums of dZ per block
    float *lossp;         // [blocks]
    uint32_t *step;       // advanced by block 0 of mlp_rows
};

__host__ __device__ __forceinline__ int round16(int x) { return (x + 15) & ~15; }
__device__ __forceinline__ int round32(int x) { return (x + 31) & ~31; }

typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;

// The zero-padded bf16 weight copies wb and wbt of every layer.
__global__ void mlp_round(TrainArgs a) {
    for (int l = 0; l < a.L; ++l) {
        const int in = a.dims[l], out = a.dims[l + 1];
        const int ki = round32(in), ko = round32(out), n1 = round16(out) * ki, n2 = round16(in) * ko;
        const float *W = a.params + a.w_off[l];
        bf16 *wb = const_cast<bf16 *>(a.wb) + a.wp_off[l], *wbt = const_cast<bf16 *>(a.wbt) + a.wtp_off[l];
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n1 + n2; i += gridDim.x * blockDim.x) {
            if (i < n1) {
                const int n = i / ki, k = i % ki;
                wb[i] = f2bf(n < out && k < in ? W[n * in + k] : 0.f);
            } else {
                const int k = (i - n1) / ko, n = (i - n1) % ko;
                wbt[i - n1] = f2bf(n < out && k < in ? W[n * in + k] : 0.f);
            }
        }
    }
}

// C (64 rows x N) = A (64 x K, bf16 in LDS, row stride kFMax + 8) * M^T with
// M [pad16(N)][K] the zero-padded bf16 weights (K a multiple of 32).  Wave w
// of the kRW waves takes the column tiles w and w + kRW (N <= 256).  All of
// the wave's M fragments for the layer (K <= 256: at most 8 k-steps) are
// loaded before the first product, so a layer costs one round trip to L2
// instead of one per k-step.
__device__ __forceinline__ void rows_gemm(const bf16 (*sA)[kFMax + 8], int K, const bf16 *M, int N,
                                          floatx4 (&acc)[4][kCT]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane % 16, kq = 8 * (lane / 16);
    const int ntiles = (N + 15) / 16;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < kCT; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    bf16x8 fb[kFMax / kKStep][kCT];
#pragma unroll
    for (int st = 0; st < kFMax / kKStep; ++st)
#pragma unroll
        for (int j = 0; j < kCT; ++j) {
            const int ct = w + kRW * j;
            if (st * kKStep < K && ct < ntiles)
                fb[st][j] = *reinterpret_cast<const bf16x8 *>(M + (size_t)(16 * ct + r) * K + st * kKStep + kq);
        }
#pragma unroll
    for (int st = 0; st < kFMax / kKStep; ++st) {
        if (st * kKStep >= K) break;
        bf16x8 fa[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) fa[i] = *reinterpret_cast<const bf16x8 *>(&sA[16 * i + r][st * kKStep + kq]);
#pragma unroll
        for (int j = 0; j < kCT; ++j)
            if (w + kRW * j < ntiles)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[st][j], acc[i][j], 0, 0, 0);
    }
}

// Column sums over the block's 64 rows of v (a lane's 4 x 4 values per
// column tile), in a fixed order, written to out[c].
__device__ __forceinline__ void block_col_sums(const float (&v)[4][kCT][4], int N, float *out) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int ntiles = (N + 15) / 16;
#pragma unroll
    for (int j = 0; j < kCT; ++j) {
        const int ct = w + kRW * j;
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) s += v[i][j][e];
        s += __shfl_xor(s, 16, 64);
        s += __shfl_xor(s, 32, 64);
        const int c = 16 * ct + lane % 16;
        if (ct < ntiles && lane < 16 && c < N) out[c] = s;
    }
}

// Lane layout of the 64 x 16 output tile (i, column tile ct) of rows_gemm:
// column c = 16 ct + lane % 16, rows 16 i + 4 (lane / 16) + e, e = 0..3.
// Each epilogue issues its global loads before any of its global stores (a
// load issued after a store waits for that store's completion too), and
// branches only on wave-uniform tile indices.
__global__ __launch_bounds__(64 * kRW) void mlp_rows(TrainArgs a) {
    __shared__ __align__(16) bf16 sA[kFR][kFMax + 8];
    __shared__ int64_t s_src[kFR];  // data row of each batch row (-1 beyond the batch)
    __shared__ float s_loss[kRW];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int r0 = blockIdx.x * kFR, Bp = a.Bp;
    const int L = a.L;
    const int rq = 4 * (lane / 16), cl = lane % 16;
    const bf16 bz = f2bf(0.f);
    if (blockIdx.x == 0 && tid == 0) *a.step += 1;
    if (tid < kFR) s_src[tid] = r0 + tid < a.B ? (a.rows ? a.rows[r0 + tid] : (int64_t)(r0 + tid)) : -1;
    __syncthreads();
    // Xb_0 = bf16(x), zero beyond d_in (up to the padded K) and beyond the batch.
    {
        const int din = a.dims[0], K = round32(din), n = kFR * K, P = round16(din);
        for (int i0 = 0; i0 < n; i0 += 64 * kRW * 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + 64 * kRW * u + tid, c = i / kFR, r = i % kFR;
                v[u] = (i < n && c < din && s_src[r] >= 0) ? a.x[(size_t)s_src[r] * din + c] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + 64 * kRW * u + tid, c = i / kFR, r = i % kFR;
                if (i >= n) continue;
                const bf16 xb = f2bf(v[u]);
                sA[r][c] = xb;
                if (c < P) a.xb[0][(size_t)c * Bp + r0 + r] = xb;
            }
        }
    }
    __syncthreads();
    floatx4 acc[4][kCT];
    float keep[4][kCT][4];  // fp32 dZ of this lane's outputs (loss / activation gradients)
    float lsum = 0.f;
    // ---------------- forward: Z = Xb Wb^T + b
    for (int l = 0; l < L; ++l) {
        const int in = a.dims[l], out = a.dims[l + 1];
        const bool last = l == L - 1;
        const int npad = round32(out), ntiles = (out + 15) / 16;
        float bj[kCT], cwj[kCT];
#pragma unroll
        for (int j = 0; j < kCT; ++j) {
            const int c = 16 * (w + kRW * j) + cl;
            bj[j] = c < out ? a.params[a.b_off[l] + c] : 0.f;
            cwj[j] = (last && c < out && a.cw) ? a.cw[c] : 1.f;
        }
        rows_gemm(sA, round32(in), a.wb + a.wp_off[l], out, acc);
        __syncthreads();  // every wave is done reading sA
        if (!last) {
#pragma unroll
            for (int j = 0; j < kCT; ++j) {
                const int ct = w + kRW * j, c = 16 * ct + cl;
                if (16 * ct >= npad) continue;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    floatx4 zv;
                    bf16x4 xv;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int r = 16 * i + rq + e;
                        const float z = acc[i][j][e] + bj[j];
                        const bf16 xn = (c < out && r0 + r < a.B) ? f2bf(z * sigmoidf_(z)) : bz;
                        sA[r][c] = xn;
                        zv[e] = z;
                        xv[e] = xn;
                    }
                    if (ct < ntiles) {
                        const size_t gi = (size_t)c * Bp + r0 + 16 * i + rq;
                        *reinterpret_cast<floatx4 *>(a.z[l] + gi) = zv;
                        *reinterpret_cast<bf16x4 *>(a.xb[l + 1] + gi) = xv;
                    }
                }
            }
        } else {
            // loss gradient dy = 2 w_c m (y - t) / B and the rows' loss terms;
            // the targets and mask entries of a column tile, then its stores.
#pragma unroll
            for (int j = 0; j < kCT; ++j) {
                const int ct = w + kRW * j, c = 16 * ct + cl;
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int e = 0; e < 4; ++e) keep[i][j][e] = 0.f;
                if (16 * ct >= npad) continue;
                float tg[4][4], mk[4][4];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int64_t src = s_src[16 * i + rq + e];
                        const bool ok = c < out && src >= 0;
                        const size_t si = ok ? (size_t)src * out + c : 0;
                        tg[i][e] = a.target[si];
                        mk[i][e] = a.mask ? a.mask[si] : 1.f;
                    }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    bf16x4 gv;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int r = 16 * i + rq + e;
                        const bool ok = c < out && r0 + r < a.B;
                        const float wgt = cwj[j] * mk[i][e];
                        const float d = (acc[i][j][e] + bj[j]) - tg[i][e];
                        const float dy = (ok && wgt != 0.f) ? 2.f * wgt * d / (float)a.B : 0.f;
                        lsum += (ok && wgt != 0.f) ? wgt * d * d : 0.f;
                        keep[i][j][e] = dy;
                        const bf16 g = f2bf(dy);
                        sA[r][c] = g;
                        gv[e] = g;
                    }
                    if (ct < ntiles)
                        *reinterpret_cast<bf16x4 *>(a.dzb[l] + (size_t)c * Bp + r0 + 16 * i + rq) = gv;
                }
            }
        }
        __syncthreads();
    }
    // the loss of the block's rows (fixed order: lanes, then waves)
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    if (lane == 0) s_loss[w] = lsum;
    // ---------------- backward: dZ_{l-1} = (dZb_l Wb_l) * SiLU'(Z_{l-1})
    block_col_sums(keep, a.dims[L], a.dbp[L - 1] + (size_t)blockIdx.x * a.dims[L]);
    for (int l = L - 1; l >= 1; --l) {
        const int out = a.dims[l + 1], in = a.dims[l];
        const int npad = round32(in), ntiles = (in + 15) / 16;
        // dH (64 x in) = dZb (64 x out) Wb (out x in): M = Wb^T
        rows_gemm(sA, round32(out), a.wbt + a.wtp_off[l], in, acc);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kCT; ++j) {
            const int ct = w + kRW * j, c = 16 * ct + cl;
            floatx4 zv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                zv[i] = floatx4{0.f, 0.f, 0.f, 0.f};
                if (ct < ntiles) zv[i] = *reinterpret_cast<const floatx4 *>(a.z[l - 1] + (size_t)c * Bp + r0 + 16 * i + rq);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                bf16x4 gv;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = 16 * i + rq + e;
                    const float zz = zv[i][e], s = sigmoidf_(zz);
                    const float g = (c < in && r0 + r < a.B) ? acc[i][j][e] * (s * (1.0f + zz * (1.0f - s))) : 0.f;
                    keep[i][j][e] = g;
                    const bf16 gb = f2bf(g);
                    if (16 * ct < npad) sA[r][c] = gb;
                    gv[e] = gb;
                }
                if (ct < ntiles) *reinterpret_cast<bf16x4 *>(a.dzb[l - 1] + (size_t)c * Bp + r0 + 16 * i + rq) = gv;
            }
        }
        block_col_sums(keep, in, a.dbp[l - 1] + (size_t)blockIdx.x * in);
        __syncthreads();
    }
    if (tid == 0) {
        float t = 0.f;
        for (int q = 0; q < kRW; ++q) t += s_loss[q];
        a.lossp[blockIdx.x] = t;
    }
}

// Weight-gradient tile (64 x 64) of one layer over one slice of up to 256
// batch rows: part[slice][w_off + j * in + i] = sum over the slice's rows r
// of dZb[j][r] Xb[i][r] (both feature-major: the matrix-core fragments are
// 16-byte loads, all of a slice's issued before the first product).
// Workgroup b: tile b / slices (layers in order, each row-major in 64 x 64
// tiles), slice b % slices.
struct WgradArgs {
    TrainArgs t;
    int slices;
    size_t nparams;
    float *part;  // [slices][nparams]
};

__global__ __launch_bounds__(256) void mlp_wgrad(WgradArgs a) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int slice = (int)blockIdx.x % a.slices;
    int l = 0, rem = (int)blockIdx.x / a.slices;
    for (; l < a.t.L; ++l) {
        const int mt = (a.t.dims[l + 1] + kTile - 1) / kTile, nt = (a.t.dims[l] + kTile - 1) / kTile;
        if (rem < mt * nt) break;
        rem -= mt * nt;
    }
    const int out = a.t.dims[l + 1], in = a.t.dims[l], Bp = a.t.Bp;
    const int ntl = (in + kTile - 1) / kTile;
    const int m0 = (rem / ntl) * kTile, n0 = (rem % ntl) * kTile;
    const int kb = slice * kWSlice, steps = (std::min(Bp, kb + kWSlice) - kb) / kKStep;
    const int r = lane % 16, kq = 8 * (lane / 16);
    const int mp = round16(out), np = round16(in);
    const bf16 *A = a.t.dzb[l], *Bm = a.t.xb[l];
    bf16x8 fa[kWSlice / kKStep][2], fb[kWSlice / kKStep][2];
#pragma unroll
    for (int st = 0; st < kWSlice / kKStep; ++st)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int gm = m0 + 32 * (w / 2) + 16 * i + r, gn = n0 + 32 * (w % 2) + 16 * i + r;
            const size_t k = (size_t)kb + st * kKStep + kq;
            fa[st][i] = bf16x8{};
            fb[st][i] = bf16x8{};
            if (st < steps && gm < mp) fa[st][i] = *reinterpret_cast<const bf16x8 *>(A + (size_t)gm * Bp + k);
            if (st < steps && gn < np) fb[st][i] = *reinterpret_cast<const bf16x8 *>(Bm + (size_t)gn * Bp + k);
        }
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int st = 0; st < kWSlice / kKStep; ++st)
        if (st < steps)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[st][i], fb[st][j], acc[i][j], 0, 0, 0);
    float *P = a.part + (size_t)slice * a.nparams + a.t.w_off[l];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gm = m0 + 32 * (w / 2) + 16 * i + 4 * (lane / 16) + e;
                const int gn = n0 + 32 * (w % 2) + 16 * j + lane % 16;
                if (gm < out && gn < in) P[(size_t)gm * in + gn] = acc[i][j][e];
            }
}

// Every parameter: its gradient (weight: the slice partials in slice order;
// bias: the per-block sums in block order), Adam, and the loss.
struct UpdateArgs {
    TrainArgs t;
    int slices, blocks;
    size_t nparams;
    const float *part;
    float *m, *v, *grad;
    const float *lr;
    float b1, b2, eps;
    float *loss;
};

// Sum of v[0], v[stride], ..., v[(n - 1) stride] in index order, 16 loads in
// flight at a time.
__device__ __forceinline__ float ordered_sum(const float *v, int n, size_t stride) {
    float g = 0.f;
    for (int z0 = 0; z0 < n; z0 += 16) {
        float t[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) t[u] = z0 + u < n ? v[(size_t)(z0 + u) * stride] : 0.f;
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (z0 + u < n) g += t[u];
    }
    return g;
}

__global__ void mlp_update(UpdateArgs a) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.loss = ordered_sum(a.t.lossp, a.blocks, 1) / (float)a.t.B;
    const float t = (float)*a.t.step, lr = *a.lr;
    const float c1 = 1.f - powf(a.b1, t), c2 = 1.f - powf(a.b2, t);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.nparams;
         i += (uint64_t)gridDim.x * blockDim.x) {
        int l = 0;
        while (l + 1 < a.t.L && i >= a.t.w_off[l + 1]) ++l;
        const float g = i < a.t.b_off[l]
                            ? ordered_sum(a.part + i, a.slices, a.nparams)
                            : ordered_sum(a.t.dbp[l] + (i - a.t.b_off[l]), a.blocks, (size_t)a.t.dims[l + 1]);
        const float mi = a.b1 * a.m[i] + (1.f - a.b1) * g;
        const float vi = a.b2 * a.v[i] + (1.f - a.b2) * g * g;
        a.m[i] = mi;
        a.v[i] = vi;
        a.t.params[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + a.eps);
        if (a.grad) a.grad[i] = g;
    }
}

// ----------------------------------------------------------------------------- host
struct Layer {
    int in, out;
    size_t w_off, b_off;  // in the parameter vector (floats)
};

struct Net {
    int L = 0;  // linear layers
    Layer layer[16];
    size_t nparams = 0;
    int maxw = 0;
};

bool make_net(const sfg_mlp_shape *s, Net &net) {
    if (!s || s->d_in == 0 || s->width == 0 || s->d_out == 0 || s->hidden == 0 || s->hidden > 14) return false;
    if (s->d_in > 4096 || s->width > 4096 || s->d_out > 4096) return false;
    net.L = (int)s->hidden + 1;
    size_t off = 0;
    for (int l = 0; l < net.L; ++l) {
        const int in = l == 0 ? (int)s->d_in : (int)s->width;
        const int out = l == net.L - 1 ? (int)s->d_out : (int)s->width;
        net.layer[l] = Layer{in, out, off, off + (size_t)in * out};
        off += (size_t)in * out + out;
        net.maxw = std::max({net.maxw, in, out});
    }
    net.nparams = off;
    return true;
}

constexpr int kSplits = 8;  // split-K of the weight gradients (reduction over the batch)

struct Ws {
    bf16 *wb;       // bf16 copy of the whole parameter vector (weights used)
    bf16 *xb[16];   // layer inputs (bf16)
    float *z[16];   // pre-activations
    float *acc;     // GEMM output scratch [B][maxw]
    float *dz, *dh; // [B][maxw]
    bf16 *dzb;      // [B][maxw]
    float *part;    // split-K partials [kSplits][maxw][maxw], then column-sum chunks [kColChunks][maxw]
    float *rowloss; // [B]
    size_t total;
};

Ws carve(const Net &net, uint32_t B, void *base) {
    Ws w;
    memset(&w, 0, sizeof(w));
    Carver c(base);
    w.wb = c.take<bf16>(net.nparams);
    for (int l = 0; l < net.L; ++l) w.xb[l] = c.take<bf16>((size_t)B * net.layer[l].in);
    for (int l = 0; l < net.L; ++l) w.z[l] = c.take<float>((size_t)B * net.layer[l].out);
    w.acc = c.take<float>((size_t)B * net.maxw);
    w.dz = c.take<float>((size_t)B * net.maxw);
    w.dh = c.take<float>((size_t)B * net.maxw);
    w.dzb = c.take<bf16>((size_t)B * net.maxw);
    w.part = c.take<float>(std::max((size_t)kSplits * net.maxw * net.maxw, (size_t)kColChunks * net.maxw));
    w.rowloss = c.take<float>(std::max<uint32_t>(B, 1));
    w.total = c.used;
    return w;
}

int grid_n(uint64_t n) { return (int)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 4096)); }

bool vec_ok(const bf16 *p, int ld) { return ((uintptr_t)p % 16) == 0 && ld % 8 == 0; }

template <bool TA, bool TB>
void gemm(const bf16 *A, int lda, const bf16 *B, int ldb, float *C, int M, int N, int K, int splits, hipStream_t s) {
    dim3 g((N + kTile - 1) / kTile, (M + kTile - 1) / kTile, splits);
    ProfScope _ps("mlp_gemm", s);
    gemm_bf16<TA, TB><<<g, 256, 0, s>>>(A, lda, B, ldb, C, M, N, K, splits, vec_ok(A, lda) ? 1 : 0,
                                        vec_ok(B, ldb) ? 1 : 0);
}

}  // namespace
}  // namespace sfg

using namespace sfg;

extern "C" size_t mlp_param_count(const sfg_mlp_shape *shape) {
    Net net;
    return make_net(shape, net) ? net.nparams : 0;
}

extern "C" size_t mlp_workspace_bytes(const sfg_mlp_shape *shape, uint32_t batch) {
    Net net;
    if (!make_net(shape, net)) return 0;
    return carve(net, batch, nullptr).total;
}

extern "C" int mlp_forward(const sfg_mlp_shape *shape, uint32_t batch, const float *params, const float *x, float *y,
                           void *workspace, size_t workspace_bytes, void *stream) {
    Net net;
    if (!make_net(shape, net)) return fail(SFG_EINVAL, "mlp_forward: bad shape");
    if (batch == 0 || batch > (1u << 24)) return fail(SFG_EINVAL, "mlp_forward: batch must be in [1, 2^24]");
    if (!params || !x || !y || !workspace) return fail(SFG_EINVAL, "mlp_forward: NULL buffer");
    Ws w = carve(net, batch, workspace);
    if (workspace_bytes < w.total) return fail(SFG_ENOSPACE, "mlp_forward: workspace too small (%zu < %zu)", workspace_bytes, w.total);
    hipStream_t s = as_stream(stream);
    { ProfScope _ps("mlp_elementwise", s); round_weights<<<grid_n(net.nparams), 256, 0, s>>>(params, w.wb, net.nparams); }
    { ProfScope _ps("mlp_elementwise", s); round_input<<<grid_n((uint64_t)batch * net.layer[0].in), 256, 0, s>>>(x, w.xb[0], (uint64_t)batch * net.layer[0].in); }
    for (int l = 0; l < net.L; ++l) {
        const Layer &ly = net.layer[l];
        // acc[B][out] = Xb[B][in] * Wb[out][in]^T
        gemm<false, true>(w.xb[l], ly.in, w.wb + ly.w_off, ly.in, w.acc, (int)batch, ly.out, ly.in, 1, s);
        const bool last = l == net.L - 1;
        ProfScope _ps("mlp_elementwise", s);
        bias_act<<<grid_n((uint64_t)batch * ly.out), 256, 0, s>>>(w.acc, params + ly.b_off, w.z[l],
                                                                   last ? nullptr : w.xb[l + 1], last ? y : nullptr,
                                                                   (int)batch, ly.out);
    }
    return check_launch("mlp_forward");
}

extern "C" int mlp_backward(const sfg_mlp_shape *shape, uint32_t batch, const float *params, const float *dy,
                            float *grad, float *dx, void *workspace, size_t workspace_bytes, void *stream) {
    Net net;
    if (!make_net(shape, net)) return fail(SFG_EINVAL, "mlp_backward: bad shape");
    if (batch == 0 || batch > (1u << 24)) return fail(SFG_EINVAL, "mlp_backward: batch must be in [1, 2^24]");
    if (!params || !dy || !workspace || (!grad && !dx)) return fail(SFG_EINVAL, "mlp_backward: NULL buffer");
    Ws w = carve(net, batch, workspace);
    if (workspace_bytes < w.total) return fail(SFG_ENOSPACE, "mlp_backward: workspace too small");
    hipStream_t s = as_stream(stream);
    const int B = (int)batch;
    for (int l = net.L - 1; l >= 0; --l) {
        const Layer &ly = net.layer[l];
        const uint64_t n = (uint64_t)B * ly.out;
        {
            ProfScope _ps("mlp_elementwise", s);
            // output layer: dZ = dy; hidden: dZ = dH * SiLU'(Z)
            act_grad<<<grid_n(n), 256, 0, s>>>(l == net.L - 1 ? dy : w.dh, l == net.L - 1 ? nullptr : w.z[l], w.dz,
                                                w.dzb, n);
        }
        if (grad) {
            // dW[out][in] = dZb^T [out][B] * Xb [B][in]  (split over the batch)
            gemm<true, false>(w.dzb, ly.out, w.xb[l], ly.in, w.part, ly.out, ly.in, B, kSplits, s);
            ProfScope _ps("mlp_elementwise", s);
            reduce_splits<<<grid_n((uint64_t)ly.out * ly.in), 256, 0, s>>>(w.part, kSplits, (uint64_t)ly.out * ly.in,
                                                                            grad + ly.w_off);
            // (the split-K partials are consumed above, so part is free again)
            const int chunk_rows = (B + kColChunks - 1) / kColChunks, chunks = (B + chunk_rows - 1) / chunk_rows;
            col_sums_chunks<<<dim3((ly.out + 63) / 64, chunks), 256, 0, s>>>(w.dz, B, ly.out, chunk_rows, w.part);
            col_sums_total<<<(ly.out + 63) / 64, 256, 0, s>>>(w.part, chunks, ly.out, grad + ly.b_off);
        }
        if (l > 0 || dx) {
            // dH[B][in] = dZb [B][out] * Wb [out][in]
            float *target = (l > 0) ? w.dh : dx;
            gemm<false, false>(w.dzb, ly.out, w.wb + ly.w_off, ly.in, target, B, ly.in, ly.out, 1, s);
        }
    }
    return check_launch("mlp_backward");
}

extern "C" int mlp_mse_grad(uint32_t batch, uint32_t d_out, const float *y, const float *target, const float *mask,
                            const float *col_weight, float *dy, float *loss, void *workspace, size_t workspace_bytes,
                            void *stream) {
    if (batch == 0 || d_out == 0) return fail(SFG_EINVAL, "mlp_mse_grad: empty batch");
    if (!y || !target || !dy || !loss || !workspace) return fail(SFG_EINVAL, "mlp_mse_grad: NULL buffer");
    if (workspace_bytes < (size_t)batch * 4) return fail(SFG_ENOSPACE, "mlp_mse_grad: workspace too small");
    hipStream_t s = as_stream(stream);
    float *rows = static_cast<float *>(workspace);
    ProfScope _ps("mlp_elementwise", s);
    mse_grad<<<(batch + 255) / 256, 256, 0, s>>>(y, target, mask, col_weight, (int)batch, (int)d_out, dy, rows);
    sum_rows<<<1, 256, 0, s>>>(rows, (int)batch, loss);
    return check_launch("mlp_mse_grad");
}

extern "C" int adam_step(uint64_t count, float *params, const float *grad, float *m, float *v, float lr, float beta1,
                         float beta2, float eps, uint32_t step, void *stream) {
    if (!params || !grad || !m || !v) return fail(SFG_EINVAL, "adam_step: NULL buffer");
    if (step == 0) return fail(SFG_EINVAL, "adam_step: step counts from 1");
    hipStream_t s = as_stream(stream);
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    ProfScope _ps("mlp_adam", s);
    adam_kernel<<<grid_n(count), 256, 0, s>>>(count, params, grad, m, v, lr, beta1, beta2, eps, c1, c2);
    return check_launch("adam_step");
}

extern "C" int adam_step_device(uint64_t count, float *params, const float *grad, float *m, float *v, const float *lr,
                                float beta1, float beta2, float eps, uint32_t *step, void *stream) {
    if (!params || !grad || !m || !v || !lr || !step) return fail(SFG_EINVAL, "adam_step_device: NULL buffer");
    hipStream_t s = as_stream(stream);
    ProfScope _ps("mlp_adam", s);
    adam_tick<<<1, 1, 0, s>>>(step);
    adam_kernel_dev<<<grid_n(count), 256, 0, s>>>(count, params, grad, m, v, lr, beta1, beta2, eps, step);
    return check_launch("adam_step_device");
}

// ----------------------------------------------------------------------------- fused training step (host)
namespace sfg {
namespace {

struct TrainWs {
    TrainArgs t;
    int blocks, slices;
    float *part;
    size_t total;
};

bool fused_ok(const Net &net) {
    if (net.L > kFMaxL) return false;
    for (int l = 0; l < net.L; ++l)
        if (net.layer[l].in > kFMax || net.layer[l].out > kFMax) return false;
    return true;
}

TrainWs carve_train(const Net &net, uint32_t B, void *base) {
    TrainWs w;
    memset(&w, 0, sizeof(w));
    Carver c(base);
    w.blocks = (int)((B + kFR - 1) / kFR);
    const int Bp = w.blocks * kFR;
    w.slices = (Bp + kWSlice - 1) / kWSlice;
    w.t.L = net.L;
    w.t.B = (int)B;
    w.t.Bp = Bp;
    w.t.dims[0] = net.layer[0].in;
    size_t wp = 0, wtp = 0;
    for (int l = 0; l < net.L; ++l) {
        const size_t in = net.layer[l].in, out = net.layer[l].out;
        w.t.wp_off[l] = wp;
        w.t.wtp_off[l] = wtp;
        wp += round16(out) * ((in + 31) & ~(size_t)31);
        wtp += round16(in) * ((out + 31) & ~(size_t)31);
    }
    w.t.wb = c.take<bf16>(wp);
    w.t.wbt = c.take<bf16>(wtp);
    for (int l = 0; l < net.L; ++l) {
        const size_t pin = round16(net.layer[l].in), pout = round16(net.layer[l].out);
        w.t.dims[l + 1] = net.layer[l].out;
        w.t.w_off[l] = net.layer[l].w_off;
        w.t.b_off[l] = net.layer[l].b_off;
        w.t.xb[l] = c.take<bf16>(pin * Bp);
        w.t.z[l] = l + 1 < net.L ? c.take<float>(pout * Bp) : nullptr;
        w.t.dzb[l] = c.take<bf16>(pout * Bp);
        w.t.dbp[l] = c.take<float>((size_t)w.blocks * net.layer[l].out);
    }
    w.t.lossp = c.take<float>(w.blocks);
    w.part = c.take<float>((size_t)w.slices * net.nparams);
    w.total = c.used;
    return w;
}

}  // namespace
}  // namespace sfg

extern "C" size_t mlp_train_workspace_bytes(const sfg_mlp_shape *shape, uint32_t batch) {
    Net net;
    if (!make_net(shape, net) || !fused_ok(net) || batch == 0) return 0;
    return carve_train(net, batch, nullptr).total;
}

extern "C" int mlp_train_step(const sfg_mlp_shape *shape, uint32_t batch, float *params, const float *x,
                              const float *target, const float *mask, const float *col_weight, const int64_t *rows,
                              float *m, float *v,
                              const float *lr, float beta1, float beta2, float eps, uint32_t *step, float *loss,
                              float *grad, void *workspace, size_t workspace_bytes, void *stream) {
    Net net;
    if (!make_net(shape, net)) return fail(SFG_EINVAL, "mlp_train_step: bad shape");
    if (!fused_ok(net)) return fail(SFG_EINVAL, "mlp_train_step: layers wider than 256 or more than 8 layers");
    if (batch == 0 || batch > (1u << 24)) return fail(SFG_EINVAL, "mlp_train_step: batch must be in [1, 2^24]");
    if (!params || !x || !target || !m || !v || !lr || !step || !loss || !workspace)
        return fail(SFG_EINVAL, "mlp_train_step: NULL buffer");
    TrainWs w = carve_train(net, batch, workspace);
    if (workspace_bytes < w.total)
        return fail(SFG_ENOSPACE, "mlp_train_step: workspace too small (%zu < %zu)", workspace_bytes, w.total);
    w.t.params = params;
    w.t.x = x;
    w.t.target = target;
    w.t.mask = mask;
    w.t.cw = col_weight;
    w.t.rows = rows;
    w.t.step = step;
    hipStream_t s = as_stream(stream);
    int ntiles = 0;
    for (int l = 0; l < net.L; ++l)
        ntiles += ((net.layer[l].out + kTile - 1) / kTile) * ((net.layer[l].in + kTile - 1) / kTile);
    { ProfScope _ps("mlp_round", s); mlp_round<<<grid_n(2 * net.nparams), 256, 0, s>>>(w.t); }
    { ProfScope _ps("mlp_rows", s); mlp_rows<<<w.blocks, 64 * kRW, 0, s>>>(w.t); }
    WgradArgs wa{w.t, w.slices, net.nparams, w.part};
    { ProfScope _ps("mlp_wgrad", s); mlp_wgrad<<<ntiles * w.slices, 256, 0, s>>>(wa); }
    UpdateArgs ua;
    memset(&ua, 0, sizeof(ua));
    ua.t = w.t;
    ua.slices = w.slices;
    ua.blocks = w.blocks;
    ua.nparams = net.nparams;
    ua.part = w.part;
    ua.m = m;
    ua.v = v;
    ua.grad = grad;
    ua.lr = lr;
    ua.b1 = beta1;
    ua.b2 = beta2;
    ua.eps = eps;
    ua.loss = loss;
    { ProfScope _ps("mlp_update", s); mlp_update<<<grid_n(net.nparams), 256, 0, s>>>(ua); }
    return check_launch("mlp_train_step");
}
