// esc_mlp.hip -- the learned cardinality estimator of the gate: an MLP
// 64 -> 256 -> 256 -> 256 -> 1 (ReLU) trained and run on the GPU with
// bfloat16 MFMA operands (v_mfma_f32_32x32x16_bf16) and float32 accumulation.
//
// The paper replaces estimates from synopses by exact counts (Section 2);
// the estimator here only decides which predicates need that exact count,
// and exact counts computed by the scan are its training labels.
//
// Rounding points (identical in the CPU oracle): every GEMM operand is
// bfloat16 (round to nearest even): the features, the weights, the hidden
// activations handed to the next layer and the back-propagated deltas;
// bias adds, ReLU, the head and all reductions are float32.  The ReLU
// derivative is taken from the rounded activation (> 0).
//
// Memory (all caller-owned): the state holds the float32 master weights,
// the Adam moments, the step counters and bfloat16 copies of the weights
// packed in MFMA B-operand fragment order (each wave's fragment of a
// 32-column tile and a 16-deep k step is one contiguous 1 KiB block, read
// with one 16-byte load per lane); for the backward products W2 and W3 are
// also packed transposed.  The training workspace holds the transposed
// activations and deltas of one batch and per-block partial sums.
//
// Kernels (a block is 8 waves; wave w owns output columns 32w .. 32w+31 of
// every 256-wide layer):
//   forward_kernel<MT>: 32*MT rows per block; all four layers in one launch,
//     activations in LDS between layers, weights straight from L2;
//   train_rows_kernel: 32 rows per block; gathers the minibatch, runs the
//     forward, the head with the Huber-loss derivative and the two backward
//     products, keeps every activation and delta in LDS, stores them
//     transposed (feature-major) for the weight gradients, and writes
//     per-block column sums (bias gradients), head-gradient and loss
//     partials;
//   weight_grad_kernel<ADAM>: one 32x32 tile of a weight gradient per wave
//     (a product over the batch rows), with Adam applied in the epilogue
//     (master weights, moments and both bf16 packings refreshed); one extra
//     block sums the partials over blocks in a fixed order for the biases,
//     W4, b4 and the loss.
// A training step is these two kernels plus a one-thread step advance,
// captured once per call into a hipGraph and replayed.  Every reduction has
// a fixed order, so training is deterministic run to run.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "esc_host.h"
#include "esc_runtime.h"

namespace esc {

constexpr int kIn = 64, kHid = 256;
constexpr int kMaxBatch = 4096;
constexpr float kHuber = 0.5f;   // Huber loss threshold on ln(selectivity) errors

// flat parameter layout (float32): W1, b1, W2, b2, W3, b3, W4, b4
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kIn * kHid;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid * kHid;
constexpr int kOffW4 = kOffB3 + kHid;
constexpr int kOffB4 = kOffW4 + kHid;
constexpr int kNParams = kOffB4 + 1;
static_assert(kNParams == ESC_MLP_NPARAMS, "parameter count");

// bf16 packings (element offsets): forward W1..W3, transposed W2 and W3, W4
constexpr int kPkF1 = 0;
constexpr int kPkF2 = kPkF1 + kIn * kHid;
constexpr int kPkF3 = kPkF2 + kHid * kHid;
constexpr int kPkB2 = kPkF3 + kHid * kHid;
constexpr int kPkB3 = kPkB2 + kHid * kHid;
constexpr int kPkW4 = kPkB3 + kHid * kHid;
constexpr int kNPack = kPkW4 + kHid;

constexpr size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// state layout (bytes)
constexpr size_t kStP = 0;
constexpr size_t kStM = up256(kStP + (size_t)kNParams * 4);
constexpr size_t kStV = up256(kStM + (size_t)kNParams * 4);
constexpr size_t kStSteps = up256(kStV + (size_t)kNParams * 4);   // int64 [0] Adam steps, [1] step of this call
constexpr size_t kStHyper = kStSteps + 64;                          // lr, b1, b2, eps
constexpr size_t kStPack = up256(kStHyper + 64);
constexpr size_t kStateBytes = up256(kStPack + (size_t)kNPack * 2);

// per-block partial sums of the training rows kernel (floats)
constexpr int kPartColsum = 0;               // [3][256] column sums of the layer deltas (bias gradients)
constexpr int kPartW4 = 3 * kHid;            // [256] head weight gradient
constexpr int kPartB4 = kPartW4 + kHid;      // head bias gradient
constexpr int kPartLoss = kPartB4 + 1;       // sum of the rows' losses
constexpr int kPartStride = kPartLoss + 7;   // 1032 floats per block

typedef uint16_t bf16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__host__ __device__ __forceinline__ float bf2f(bf16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

__host__ __device__ __forceinline__ bf16_t f2bf(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40);   // quiet NaN
    return (bf16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Element offset of B(k, n) of a K x N matrix in fragment order: fragment
// (n/32, k/16) is 64 lanes x 8 values, lane = 32 (k/8 % 2) + n % 32, value
// k % 8 (the B operand of v_mfma_f32_32x32x16_bf16).
__host__ __device__ __forceinline__ int frag_off(int k, int n, int K)
{
    return ((((n >> 5) * (K >> 4) + (k >> 4)) * 64 + ((k >> 3) & 1) * 32 + (n & 31)) << 3) + (k & 7);
}

struct Hyper {
    float lr, b1, b2, eps;
};

struct State {
    float *p, *m, *v;
    long long *steps;
    Hyper *hyper;
    bf16_t *pk;
};

struct TrainWs {
    bf16_t *aT[3];   // layer inputs, transposed: [fan_in][bp]
    bf16_t *gT[3];   // rounded deltas of layers 1..3, transposed: [256][bp]
    float *part;     // [blocks][kPartStride]
};

constexpr int kBlock = 512;   // 8 waves
constexpr int kWaves = kBlock / 64;
constexpr int LDA = kHid + 8;   // LDS row stride (bf16) of 256-wide activations: +16 bytes
constexpr int LDX = kIn + 8;

size_t train_ws_bytes(int batch, TrainWs *ws, char *base)
{
    const size_t bp = (size_t)((batch + 31) / 32 * 32);
    const size_t nb = bp / 32;
    size_t off = 0;
    const size_t sizes[6] = {kIn * bp * 2, kHid * bp * 2, kHid * bp * 2, kHid * bp * 2, kHid * bp * 2, kHid * bp * 2};
    char *ptr[6];
    for (int i = 0; i < 6; i++) {
        ptr[i] = base ? base + off : nullptr;
        off = up256(off + sizes[i]);
    }
    if (ws) {
        for (int i = 0; i < 3; i++) ws->aT[i] = (bf16_t *)ptr[i];
        for (int i = 0; i < 3; i++) ws->gT[i] = (bf16_t *)ptr[3 + i];
        ws->part = base ? (float *)(base + off) : nullptr;
    }
    off = up256(off + nb * kPartStride * 4);
    return off;
}

// ------------------------------------------------------------------ device helpers

__device__ __forceinline__ int lane_of() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_of() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// acc[mt] = A(rows 32 mt .. 32 mt + 31, 0..K) * B(0..K, columns 32 nt ..),
// A in LDS (bf16, row stride lda), B packed in fragment order in global
// memory (all of this wave's fragments are loaded before the products).
template <int MT, int K>
__device__ __forceinline__ void mma_layer(const bf16_t *As, int lda, const bf16_t *Bpk, int nt, f32x16 (&acc)[MT])
{
    constexpr int KS = K / 16;
    const int lane = lane_of();
    const u16x8 *src = (const u16x8 *)Bpk + (size_t)nt * KS * 64 + lane;
    u16x8 b[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ks++) b[ks] = src[ks * 64];
#pragma unroll
    for (int mt = 0; mt < MT; mt++)
#pragma unroll
        for (int i = 0; i < 16; i++) acc[mt][i] = 0.0f;
#pragma unroll
    for (int ks = 0; ks < KS; ks++) {
#pragma unroll
        for (int mt = 0; mt < MT; mt++) {
            const u16x8 a = *(const u16x8 *)&As[(32 * mt + (lane & 31)) * lda + 16 * ks + 8 * (lane >> 5)];
            acc[mt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                              __builtin_bit_cast(bf16x8, b[ks]), acc[mt], 0, 0, 0);
        }
    }
}

// accumulator element e of a lane: row 8 (e/4) + 4 (lane/32) + e%4, column lane%32
__device__ __forceinline__ int acc_row(int e) { return 8 * (e >> 2) + 4 * (lane_of() >> 5) + (e & 3); }

// H[m][n] = bf16(relu(acc + bias[n])) for the wave's column tile
template <int MT>
__device__ __forceinline__ void store_relu(const f32x16 (&acc)[MT], int nt, const float *bias, bf16_t *Hs)
{
    const int n = 32 * nt + (lane_of() & 31);
    const float bn = bias[n];
#pragma unroll
    for (int mt = 0; mt < MT; mt++)
#pragma unroll
        for (int e = 0; e < 16; e++) {
            const float z = acc[mt][e] + bn;
            Hs[(32 * mt + acc_row(e)) * LDA + n] = f2bf(z > 0.0f ? z : 0.0f);
        }
}

// dz = acc masked by (activation > 0); G[m][n] = bf16(dz); colsum[n] = sum of
// dz over the 32 rows (fixed order)
__device__ __forceinline__ void store_masked(const f32x16 &acc, int nt, const bf16_t *Mask, bf16_t *Gs,
                                             float *colsum)
{
    const int lane = lane_of();
    const int n = 32 * nt + (lane & 31);
    float s = 0.0f;
#pragma unroll
    for (int e = 0; e < 16; e++) {
        const int m = acc_row(e);
        const float dz = bf2f(Mask[m * LDA + n]) > 0.0f ? acc[e] : 0.0f;
        s += dz;
        Gs[m * LDA + n] = f2bf(dz);
    }
    s += __shfl_xor(s, 32, 64);
    if (lane < 32) colsum[n] = s;
}

__device__ __forceinline__ float wave_reduce(float s)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}

// y of row m: a3[m] . bf16(W4) + b4 (whole wave; result in every lane)
__device__ __forceinline__ float head_row(const bf16_t *A3, int m, const bf16_t *w4b, float b4)
{
    const int lane = lane_of();
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int k = lane + 64 * j;
        s += bf2f(A3[m * LDA + k]) * bf2f(w4b[k]);
    }
    return wave_reduce(s) + b4;
}

// T[f][col0 + r] = S[r][f] for r < 32, f < nf: each thread moves 8 rows of
// one feature as one 16-byte store
__device__ __forceinline__ void store_transposed(const bf16_t *S, int lds, int nf, bf16_t *T, size_t ldt, int col0)
{
    for (int it = threadIdx.x; it < nf * 4; it += kBlock) {
        const int f = it >> 2, r0 = (it & 3) * 8;
        u16x8 v;
#pragma unroll
        for (int j = 0; j < 8; j++) v[j] = S[(r0 + j) * lds + f];
        *(u16x8 *)&T[(size_t)f * ldt + col0 + r0] = v;
    }
}

// ------------------------------------------------------------------ inference

// yhat for rows [32 MT blockIdx.x, +32 MT) of X (n x 64 float32)
template <int MT>
__global__ __launch_bounds__(kBlock) void forward_kernel(const float *__restrict__ X, int64_t n,
                                                         const float *__restrict__ p, const bf16_t *__restrict__ pk,
                                                         float *__restrict__ yhat)
{
    constexpr int R = 32 * MT;
    __shared__ __attribute__((aligned(16))) bf16_t xs[R * LDX];
    __shared__ __attribute__((aligned(16))) bf16_t h0[R * LDA];
    __shared__ __attribute__((aligned(16))) bf16_t h1[R * LDA];
    const int64_t row0 = (int64_t)blockIdx.x * R;
    for (int i = threadIdx.x; i < R * kIn; i += kBlock) {
        const int m = i >> 6, k = i & 63;
        xs[m * LDX + k] = row0 + m < n ? f2bf(X[(row0 + m) * kIn + k]) : (bf16_t)0;
    }
    __syncthreads();
    const int w = wave_of();
    f32x16 acc[MT];
    mma_layer<MT, kIn>(xs, LDX, pk + kPkF1, w, acc);
    store_relu<MT>(acc, w, p + kOffB1, h0);
    __syncthreads();
    mma_layer<MT, kHid>(h0, LDA, pk + kPkF2, w, acc);
    store_relu<MT>(acc, w, p + kOffB2, h1);
    __syncthreads();
    mma_layer<MT, kHid>(h1, LDA, pk + kPkF3, w, acc);
    store_relu<MT>(acc, w, p + kOffB3, h0);
    __syncthreads();
    const float b4 = p[kOffB4];
    for (int m = w; m < R; m += kWaves) {
        const float y = head_row(h0, m, pk + kPkW4, b4);
        if (lane_of() == 0 && row0 + m < n) yhat[row0 + m] = y;
    }
}

// ------------------------------------------------------------------ training

// Forward and backward of rows [32 blockIdx.x, +32) of one minibatch of
// `batch` rows: row r is sample order[steps[1] * batch + r] (or r).
__global__ __launch_bounds__(kBlock) void train_rows_kernel(const float *__restrict__ X, const float *__restrict__ Y,
                                                            const int32_t *__restrict__ order, int batch,
                                                            const State st, const TrainWs ws)
{
    constexpr int R = 32;
    __shared__ __attribute__((aligned(16))) bf16_t xs[R * LDX];
    __shared__ __attribute__((aligned(16))) bf16_t a1[R * LDA];
    __shared__ __attribute__((aligned(16))) bf16_t a2[R * LDA];
    __shared__ __attribute__((aligned(16))) bf16_t a3[R * LDA];
    __shared__ __attribute__((aligned(16))) bf16_t g3[R * LDA];
    __shared__ __attribute__((aligned(16))) bf16_t g2[R * LDA];
    __shared__ __attribute__((aligned(16))) bf16_t g1[R * LDA];
    __shared__ float tgt[R], dys[R], lss[R];
    const int bp = (batch + 31) / 32 * 32;
    const int row0 = blockIdx.x * R;
    const long long base = order ? st.steps[1] * (long long)batch : 0;
    for (int i = threadIdx.x; i < R * kIn; i += kBlock) {
        const int m = i >> 6, k = i & 63;
        const int r = row0 + m;
        bf16_t v = 0;
        if (r < batch) {
            const long long src = order ? order[base + r] : r;
            v = f2bf(X[src * kIn + k]);
            if (k == 0) tgt[m] = Y[src];
        } else if (k == 0) {
            tgt[m] = 0.0f;
        }
        xs[m * LDX + k] = v;
    }
    __syncthreads();
    const float *p = st.p;
    const bf16_t *pk = st.pk;
    float *part = ws.part + (size_t)blockIdx.x * kPartStride;
    const int w = wave_of();
    f32x16 acc[1];
    mma_layer<1, kIn>(xs, LDX, pk + kPkF1, w, acc);
    store_relu<1>(acc, w, p + kOffB1, a1);
    __syncthreads();
    mma_layer<1, kHid>(a1, LDA, pk + kPkF2, w, acc);
    store_relu<1>(acc, w, p + kOffB2, a2);
    __syncthreads();
    mma_layer<1, kHid>(a2, LDA, pk + kPkF3, w, acc);
    store_relu<1>(acc, w, p + kOffB3, a3);
    __syncthreads();
    // head: dL/dy = clamp(y - t, -h, h) / batch for the Huber loss
    const float b4 = p[kOffB4];
    for (int m = w; m < R; m += kWaves) {
        const float y = head_row(a3, m, pk + kPkW4, b4);
        if (lane_of() == 0) {
            const bool ok = row0 + m < batch;
            const float e = y - tgt[m];
            const float ae = fabsf(e);
            dys[m] = ok ? fminf(fmaxf(e, -kHuber), kHuber) / (float)batch : 0.0f;
            lss[m] = ok ? (ae <= kHuber ? 0.5f * e * e : kHuber * (ae - 0.5f * kHuber)) : 0.0f;
        }
    }
    __syncthreads();
    // delta of layer 3 (masked by a3 > 0), its column sums, the head gradients
    if (threadIdx.x < kHid) {
        const int k = threadIdx.x;
        const float w4 = bf2f(pk[kPkW4 + k]);
        float cs = 0.0f, gw = 0.0f;
        for (int m = 0; m < R; m++) {
            const float a = bf2f(a3[m * LDA + k]);
            const float d = dys[m];
            const float dz = a > 0.0f ? d * w4 : 0.0f;
            cs += dz;
            gw += a * d;
            g3[m * LDA + k] = f2bf(dz);
        }
        part[kPartColsum + 2 * kHid + k] = cs;
        part[kPartW4 + k] = gw;
        if (k == 0) {
            float sd = 0.0f, sl = 0.0f;
            for (int m = 0; m < R; m++) {
                sd += dys[m];
                sl += lss[m];
            }
            part[kPartB4] = sd;
            part[kPartLoss] = sl;
        }
    }
    __syncthreads();
    // delta of layer 2 = (g3 W3^T) masked by a2 > 0
    mma_layer<1, kHid>(g3, LDA, pk + kPkB3, w, acc);
    store_masked(acc[0], w, a2, g2, part + kPartColsum + kHid);
    __syncthreads();
    // delta of layer 1 = (g2 W2^T) masked by a1 > 0
    mma_layer<1, kHid>(g2, LDA, pk + kPkB2, w, acc);
    store_masked(acc[0], w, a1, g1, part + kPartColsum);
    __syncthreads();
    store_transposed(xs, LDX, kIn, ws.aT[0], bp, row0);
    store_transposed(a1, LDA, kHid, ws.aT[1], bp, row0);
    store_transposed(a2, LDA, kHid, ws.aT[2], bp, row0);
    store_transposed(g1, LDA, kHid, ws.gT[0], bp, row0);
    store_transposed(g2, LDA, kHid, ws.gT[1], bp, row0);
    store_transposed(g3, LDA, kHid, ws.gT[2], bp, row0);
}

// Adam on one float32 master parameter; returns the new value
__device__ __forceinline__ float adam(const State &st, int i, float g, const Hyper &h, float c1, float c2)
{
    const float mi = h.b1 * st.m[i] + (1.0f - h.b1) * g;
    const float vi = h.b2 * st.v[i] + (1.0f - h.b2) * g * g;
    st.m[i] = mi;
    st.v[i] = vi;
    const float pi = st.p[i] - h.lr * (mi / c1) / (sqrtf(vi / c2) + h.eps);
    st.p[i] = pi;
    return pi;
}

constexpr int kGradTiles = (kIn / 32) * 8 + 2 * 8 * 8;   // 32x32 tiles of gW1, gW2, gW3: 144
constexpr int kGradWaves = 4;
constexpr int kGradTileBlocks = kGradTiles / kGradWaves;   // 36; one more block for biases, W4, b4, loss
static_assert(kGradTiles % kGradWaves == 0, "whole blocks of tiles");

// Weight gradients of one minibatch from the transposed activations and
// deltas (gW_l[i][j] = sum over rows of a_{l-1}[r][i] g_l[r][j]), then Adam
// (ADAM) or the gradient written flat into grads (!ADAM).
template <bool ADAM>
__global__ __launch_bounds__(kGradWaves * 64) void weight_grad_kernel(int batch, const State st, const TrainWs ws,
                                                                      float *__restrict__ grads,
                                                                      float *__restrict__ loss_out)
{
    const int bp = (batch + 31) / 32 * 32;
    Hyper h{};
    float c1 = 1.0f, c2 = 1.0f;
    if (ADAM) {
        h = *st.hyper;
        const float t = (float)(st.steps[0] + 1);
        c1 = 1.0f - powf(h.b1, t);
        c2 = 1.0f - powf(h.b2, t);
    }
    const int lane = lane_of();
    if (blockIdx.x < kGradTileBlocks) {
        int tile = blockIdx.x * kGradWaves + wave_of();
        int layer, mt, nt, fan_in;
        if (tile < 16) {
            layer = 0; fan_in = kIn;
        } else {
            tile -= 16;
            layer = 1 + tile / 64;
            tile %= 64;
            fan_in = kHid;
        }
        mt = tile >> 3;
        nt = tile & 7;
        const bf16_t *AT = ws.aT[layer] + (size_t)(32 * mt + (lane & 31)) * bp + 8 * (lane >> 5);
        const bf16_t *GT = ws.gT[layer] + (size_t)(32 * nt + (lane & 31)) * bp + 8 * (lane >> 5);
        f32x16 acc;
#pragma unroll
        for (int i = 0; i < 16; i++) acc[i] = 0.0f;
        const int ksteps = bp / 16;
        int ks = 0;
        for (; ks + 4 <= ksteps; ks += 4) {
            u16x8 a[4], b[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                a[j] = *(const u16x8 *)(AT + 16 * (ks + j));
                b[j] = *(const u16x8 *)(GT + 16 * (ks + j));
            }
#pragma unroll
            for (int j = 0; j < 4; j++)
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[j]),
                                                              __builtin_bit_cast(bf16x8, b[j]), acc, 0, 0, 0);
        }
        for (; ks < ksteps; ks++) {
            const u16x8 a = *(const u16x8 *)(AT + 16 * ks);
            const u16x8 b = *(const u16x8 *)(GT + 16 * ks);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                          acc, 0, 0, 0);
        }
        const int offW = layer == 0 ? kOffW1 : layer == 1 ? kOffW2 : kOffW3;
        const int pkF = layer == 0 ? kPkF1 : layer == 1 ? kPkF2 : kPkF3;
        const int pkB = layer == 1 ? kPkB2 : kPkB3;
        const int j = 32 * nt + (lane & 31);
#pragma unroll
        for (int e = 0; e < 16; e++) {
            const int i = 32 * mt + acc_row(e);
            const int idx = offW + i * kHid + j;
            if (ADAM) {
                const bf16_t wb = f2bf(adam(st, idx, acc[e], h, c1, c2));
                st.pk[pkF + frag_off(i, j, fan_in)] = wb;
                if (layer > 0) st.pk[pkB + frag_off(j, i, kHid)] = wb;
            } else {
                grads[idx] = acc[e];
            }
        }
        return;
    }
    // biases, W4 and b4 from the per-block partials (summed in block order)
    const int nb = bp / 32;
    for (int k = threadIdx.x; k < kHid; k += blockDim.x) {
        const int offB[3] = {kOffB1, kOffB2, kOffB3};
        for (int l = 0; l < 3; l++) {
            float s = 0.0f;
            for (int b = 0; b < nb; b++) s += ws.part[(size_t)b * kPartStride + kPartColsum + l * kHid + k];
            if (ADAM) adam(st, offB[l] + k, s, h, c1, c2);
            else grads[offB[l] + k] = s;
        }
        float s = 0.0f;
        for (int b = 0; b < nb; b++) s += ws.part[(size_t)b * kPartStride + kPartW4 + k];
        if (ADAM) st.pk[kPkW4 + k] = f2bf(adam(st, kOffW4 + k, s, h, c1, c2));
        else grads[kOffW4 + k] = s;
    }
    if (threadIdx.x == 0) {
        float sd = 0.0f, sl = 0.0f;
        for (int b = 0; b < nb; b++) {
            sd += ws.part[(size_t)b * kPartStride + kPartB4];
            sl += ws.part[(size_t)b * kPartStride + kPartLoss];
        }
        if (ADAM) adam(st, kOffB4, sd, h, c1, c2);
        else grads[kOffB4] = sd;
        if (loss_out) loss_out[ADAM ? st.steps[1] : 0] = sl / (float)batch;
    }
}

__global__ void advance_kernel(long long *steps)
{
    steps[0] += 1;
    steps[1] += 1;
}

__global__ void begin_call_kernel(long long *steps, Hyper *hyper, float lr)
{
    steps[1] = 0;
    *hyper = Hyper{lr, 0.9f, 0.999f, 1e-8f};
}

// bf16 packings of the weights from the float32 master copy
__global__ void pack_kernel(const float *__restrict__ p, bf16_t *__restrict__ pk)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kIn * kHid) {
        pk[kPkF1 + frag_off(i / kHid, i % kHid, kIn)] = f2bf(p[kOffW1 + i]);
    } else if (i < kIn * kHid + 2 * kHid * kHid) {
        const int l = (i - kIn * kHid) / (kHid * kHid);
        const int q = (i - kIn * kHid) % (kHid * kHid);
        const int r = q / kHid, c = q % kHid;
        const bf16_t wb = f2bf(p[(l == 0 ? kOffW2 : kOffW3) + q]);
        pk[(l == 0 ? kPkF2 : kPkF3) + frag_off(r, c, kHid)] = wb;
        pk[(l == 0 ? kPkB2 : kPkB3) + frag_off(c, r, kHid)] = wb;
    } else if (i < kIn * kHid + 2 * kHid * kHid + kHid) {
        const int k = i - kIn * kHid - 2 * kHid * kHid;
        pk[kPkW4 + k] = f2bf(p[kOffW4 + k]);
    }
}

}  // namespace esc

using namespace esc;

struct esc_mlp {
    int device = 0;
    char *state = nullptr;   // caller-owned, kStateBytes
    State st{};
    hipStream_t cap = nullptr;   // private stream for graph capture and state transfers
};

namespace {

int hipchk(hipError_t e, const char *what) { return e == hipSuccess ? ESC_OK : hip_fail(e, what); }

int check_mlp(const esc_mlp *m)
{
    if (!m) return fail(ESC_ERR_INVALID, "null mlp handle");
    return set_device(m->device);
}

int check_ws(const void *ws, size_t bytes, int batch)
{
    if (!ws || ((uintptr_t)ws & 255)) return fail(ESC_ERR_ALIGN, "workspace must be non-null and 256-byte aligned");
    const size_t need = train_ws_bytes(batch, nullptr, nullptr);
    if (bytes < need) return fail(ESC_ERR_OOM, "workspace of %zu bytes, %zu needed for %d rows", bytes, need, batch);
    return ESC_OK;
}

// 64-bit FNV-1a over a byte range (checkpoint integrity)
uint64_t fnv1a(const void *data, size_t n, uint64_t h)
{
    const unsigned char *b = (const unsigned char *)data;
    for (size_t i = 0; i < n; i++) {
        h ^= b[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

constexpr char kMagic[8] = {'E', 'S', 'C', 'M', 'L', 'P', '0', '1'};
constexpr uint32_t kFileVersion = 1;

struct FileHeader {
    char magic[8];
    uint32_t version;
    uint32_t nparams;
    int64_t step;
    uint64_t checksum;   // FNV-1a of params, m and v
};

}  // namespace

extern "C" {

size_t esc_mlp_state_bytes(void) { return kStateBytes; }

size_t esc_mlp_workspace_bytes(int batch)
{
    if (batch < 1 || batch > kMaxBatch) return 0;
    return train_ws_bytes(batch, nullptr, nullptr);
}

int esc_mlp_create(esc_ctx *ctx, void *dev_state, size_t state_bytes, esc_mlp **out)
{
    if (!ctx || !out) return fail(ESC_ERR_INVALID, "null argument");
    if (!dev_state || ((uintptr_t)dev_state & 255)) return fail(ESC_ERR_ALIGN, "state must be 256-byte aligned");
    if (state_bytes < kStateBytes) return fail(ESC_ERR_OOM, "state of %zu bytes, %zu needed", state_bytes, kStateBytes);
    if (int rc0 = set_device(ctx->device)) return rc0;
    esc_mlp *m = new (std::nothrow) esc_mlp;
    if (!m) return fail(ESC_ERR_OOM, "out of host memory");
    m->device = ctx->device;
    m->state = (char *)dev_state;
    m->st = State{(float *)(m->state + kStP), (float *)(m->state + kStM), (float *)(m->state + kStV),
                  (long long *)(m->state + kStSteps), (Hyper *)(m->state + kStHyper), (bf16_t *)(m->state + kStPack)};
    hipError_t e = hipStreamCreateWithFlags(&m->cap, hipStreamNonBlocking);
    if (e != hipSuccess) { delete m; return hip_fail(e, "stream"); }
    std::vector<float> z(kNParams, 0.0f);
    int rc = esc_mlp_set_params(m, z.data());
    if (rc) { esc_mlp_destroy(m); return rc; }
    *out = m;
    return ESC_OK;
}

int esc_mlp_destroy(esc_mlp *m)
{
    if (!m) return ESC_OK;
    (void)set_device(m->device);
    if (m->cap) (void)hipStreamDestroy(m->cap);
    delete m;
    return ESC_OK;
}

int esc_mlp_set_state(esc_mlp *m, const float *params, const float *adam_m, const float *adam_v, int64_t step)
{
    int rc = check_mlp(m);
    if (rc) return rc;
    if (!params || step < 0) return fail(ESC_ERR_INVALID, "null parameters or negative step");
    hipStream_t s = m->cap;
    if ((rc = hipchk(hipMemcpyAsync(m->st.p, params, kNParams * 4, hipMemcpyHostToDevice, s), "upload"))) return rc;
    if (adam_m) rc = hipchk(hipMemcpyAsync(m->st.m, adam_m, kNParams * 4, hipMemcpyHostToDevice, s), "upload");
    else rc = hipchk(hipMemsetAsync(m->st.m, 0, kNParams * 4, s), "memset");
    if (rc) return rc;
    if (adam_v) rc = hipchk(hipMemcpyAsync(m->st.v, adam_v, kNParams * 4, hipMemcpyHostToDevice, s), "upload");
    else rc = hipchk(hipMemsetAsync(m->st.v, 0, kNParams * 4, s), "memset");
    if (rc) return rc;
    const long long steps[2] = {(long long)step, 0};
    if ((rc = hipchk(hipMemcpyAsync(m->st.steps, steps, sizeof steps, hipMemcpyHostToDevice, s), "upload"))) return rc;
    constexpr int kPackItems = kIn * kHid + 2 * kHid * kHid + kHid;
    hipLaunchKernelGGL(pack_kernel, dim3((kPackItems + 255) / 256), dim3(256), 0, s, m->st.p, m->st.pk);
    return hipchk(hipStreamSynchronize(s), "sync");
}

int esc_mlp_set_params(esc_mlp *m, const float *host_params)
{
    return esc_mlp_set_state(m, host_params, nullptr, nullptr, 0);
}

int esc_mlp_get_state(esc_mlp *m, float *params, float *adam_m, float *adam_v, int64_t *step)
{
    int rc = check_mlp(m);
    if (rc) return rc;
    hipStream_t s = m->cap;
    if (params && (rc = hipchk(hipMemcpyAsync(params, m->st.p, kNParams * 4, hipMemcpyDeviceToHost, s), "download")))
        return rc;
    if (adam_m && (rc = hipchk(hipMemcpyAsync(adam_m, m->st.m, kNParams * 4, hipMemcpyDeviceToHost, s), "download")))
        return rc;
    if (adam_v && (rc = hipchk(hipMemcpyAsync(adam_v, m->st.v, kNParams * 4, hipMemcpyDeviceToHost, s), "download")))
        return rc;
    long long steps[2] = {0, 0};
    if ((rc = hipchk(hipMemcpyAsync(steps, m->st.steps, sizeof steps, hipMemcpyDeviceToHost, s), "download")))
        return rc;
    if ((rc = hipchk(hipStreamSynchronize(s), "sync"))) return rc;
    if (step) *step = steps[0];
    return ESC_OK;
}

int esc_mlp_get_params(esc_mlp *m, float *host_params)
{
    if (!host_params) return fail(ESC_ERR_INVALID, "null output");
    return esc_mlp_get_state(m, host_params, nullptr, nullptr, nullptr);
}

int esc_mlp_save(esc_mlp *m, const char *path)
{
    if (!path) return fail(ESC_ERR_INVALID, "null path");
    std::vector<float> buf(3 * (size_t)kNParams);
    int64_t step = 0;
    int rc = esc_mlp_get_state(m, buf.data(), buf.data() + kNParams, buf.data() + 2 * kNParams, &step);
    if (rc) return rc;
    FileHeader h{};
    memcpy(h.magic, kMagic, 8);
    h.version = kFileVersion;
    h.nparams = kNParams;
    h.step = step;
    h.checksum = fnv1a(buf.data(), buf.size() * 4, 0xcbf29ce484222325ull);
    FILE *f = fopen(path, "wb");
    if (!f) return fail(ESC_ERR_INVALID, "cannot open %s for writing", path);
    const bool ok = fwrite(&h, sizeof h, 1, f) == 1 && fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    const bool closed = fclose(f) == 0;
    if (!ok || !closed) return fail(ESC_ERR_INVALID, "writing %s failed", path);
    return ESC_OK;
}

int esc_mlp_load(esc_mlp *m, const char *path)
{
    if (!path) return fail(ESC_ERR_INVALID, "null path");
    int rc = check_mlp(m);
    if (rc) return rc;
    FILE *f = fopen(path, "rb");
    if (!f) return fail(ESC_ERR_INVALID, "cannot open %s", path);
    FileHeader h{};
    std::vector<float> buf(3 * (size_t)kNParams);
    const bool ok = fread(&h, sizeof h, 1, f) == 1 && fread(buf.data(), 4, buf.size(), f) == buf.size();
    char extra;
    const bool at_end = fread(&extra, 1, 1, f) == 0;
    fclose(f);
    if (!ok || !at_end) return fail(ESC_ERR_INVALID, "%s: wrong size for an estimator checkpoint", path);
    if (memcmp(h.magic, kMagic, 8) != 0) return fail(ESC_ERR_INVALID, "%s: not an estimator checkpoint", path);
    if (h.version != kFileVersion || h.nparams != (uint32_t)kNParams)
        return fail(ESC_ERR_INVALID, "%s: version %u with %u parameters, expected %u with %d", path, h.version,
                    h.nparams, kFileVersion, kNParams);
    if (h.step < 0) return fail(ESC_ERR_INVALID, "%s: negative step count", path);
    if (fnv1a(buf.data(), buf.size() * 4, 0xcbf29ce484222325ull) != h.checksum)
        return fail(ESC_ERR_INVALID, "%s: checksum mismatch", path);
    return esc_mlp_set_state(m, buf.data(), buf.data() + kNParams, buf.data() + 2 * kNParams, h.step);
}

int esc_mlp_predict(esc_mlp *m, const float *dev_x, int64_t n, float *dev_yhat, void *stream)
{
    int rc = check_mlp(m);
    if (rc) return rc;
    if (n < 0 || (n > 0 && (!dev_x || !dev_yhat))) return fail(ESC_ERR_INVALID, "bad arguments");
    if (n == 0) return ESC_OK;
    hipStream_t s = (hipStream_t)stream;
    const int64_t blocks = (n + 31) / 32;
    hipLaunchKernelGGL(forward_kernel<1>, dim3((unsigned)blocks), dim3(kBlock), 0, s, dev_x, n, m->st.p, m->st.pk,
                       dev_yhat);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ESC_OK : hip_fail(e, "predict launch");
}

int esc_mlp_gradients(esc_mlp *m, const float *dev_x, const float *dev_y, int64_t n, float *dev_grads,
                      void *dev_ws, size_t ws_bytes, void *stream)
{
    int rc = check_mlp(m);
    if (rc) return rc;
    if (n < 1 || n > kMaxBatch || !dev_x || !dev_y || !dev_grads)
        return fail(ESC_ERR_INVALID, "need 1 <= n <= %d and non-null buffers", kMaxBatch);
    if ((rc = check_ws(dev_ws, ws_bytes, (int)n))) return rc;
    hipStream_t s = (hipStream_t)stream;
    TrainWs ws;
    train_ws_bytes((int)n, &ws, (char *)dev_ws);
    const int nb = (int)((n + 31) / 32);
    hipLaunchKernelGGL(train_rows_kernel, dim3(nb), dim3(kBlock), 0, s, dev_x, dev_y, nullptr, (int)n, m->st, ws);
    hipLaunchKernelGGL(weight_grad_kernel<false>, dim3(kGradTileBlocks + 1), dim3(kGradWaves * 64), 0, s, (int)n,
                       m->st, ws, dev_grads, nullptr);
    return hipchk(hipStreamSynchronize(s), "sync");
}

int esc_mlp_train(esc_mlp *m, const float *dev_x, const float *dev_y, const int32_t *dev_order, int64_t steps,
                  int batch, float lr, void *dev_ws, size_t ws_bytes, void *stream, float *dev_loss)
{
    int rc = check_mlp(m);
    if (rc) return rc;
    if (steps < 0 || batch < 1 || batch > kMaxBatch || !dev_x || !dev_y || !dev_order || !(lr > 0.0f))
        return fail(ESC_ERR_INVALID, "bad training arguments");
    if ((rc = check_ws(dev_ws, ws_bytes, batch))) return rc;
    if (steps == 0) return ESC_OK;
    hipStream_t s = (hipStream_t)stream;
    TrainWs ws;
    train_ws_bytes(batch, &ws, (char *)dev_ws);
    hipLaunchKernelGGL(begin_call_kernel, dim3(1), dim3(1), 0, s, m->st.steps, m->st.hyper, lr);
    // one training step, captured once for this call and replayed `steps` times
    hipStream_t c = m->cap;
    if ((rc = hipchk(hipStreamBeginCapture(c, hipStreamCaptureModeThreadLocal), "begin capture"))) return rc;
    const int nb = (batch + 31) / 32;
    hipLaunchKernelGGL(train_rows_kernel, dim3(nb), dim3(kBlock), 0, c, dev_x, dev_y, dev_order, batch, m->st, ws);
    hipLaunchKernelGGL(weight_grad_kernel<true>, dim3(kGradTileBlocks + 1), dim3(kGradWaves * 64), 0, c, batch,
                       m->st, ws, nullptr, dev_loss);
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(1), 0, c, m->st.steps);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(c, &graph);
    if (e != hipSuccess) return hip_fail(e, "end capture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "instantiate");
    for (int64_t i = 0; i < steps && e == hipSuccess; i++) e = hipGraphLaunch(exec, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipGraphExecDestroy(exec);
    return e == hipSuccess ? ESC_OK : hip_fail(e, "training");
}

}  // extern "C"
