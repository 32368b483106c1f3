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
// Kernels: one generic LDS-staged bf16 GEMM (64x64 block tile, four waves of
// 32x32, K in steps of 32) with three epilogues (bias+ReLU -> bf16; masked
// delta -> float32 + bf16; plain float32), a per-row head kernel, column
// reductions and an Adam kernel that also refreshes the bf16 weight copies.
// A training step is 15 launches captured once per batch size into a
// hipGraph; the step counter, learning rate and sample order live in device
// memory so the same graph replays for every step.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <map>
#include <new>
#include <vector>

#include "esc_host.h"
#include "esc_runtime.h"

namespace esc {

constexpr int kIn = 64, kHid = 256;
constexpr int kMaxRows = 4096;   // rows per forward / gradient pass
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
// bf16 weight copies, same offsets for W1..W4 (biases unused)
constexpr int kNBf = kOffB4;

typedef uint16_t bf16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16_t f2bf(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40);   // quiet NaN
    return (bf16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// ------------------------------------------------------------------ GEMM

enum { EPI_F32 = 0, EPI_BIAS_RELU = 1, EPI_MASKED = 2 };

struct GemmArgs {
    int M, N, K;
    const bf16_t *A; long sam, sak;    // A(m,k) = A[m*sam + k*sak]
    const bf16_t *B; long sbk, sbn;    // B(k,n) = B[k*sbk + n*sbn]
    float *C; long scm;                // float32 out, row-major, ld scm
    const float *bias;                 // EPI_BIAS_RELU
    bf16_t *H; long shm;               // bf16 out, row-major, ld shm
    const bf16_t *mask; long smm;      // EPI_MASKED: derivative mask (activation > 0)
};

constexpr int GBM = 64, GBN = 64, GBK = 32, GLD = GBK + 8;   // LDS rows padded by 8 bf16

template <int EPI>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(const GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) bf16_t As[GBM][GLD];
    __shared__ __attribute__((aligned(16))) bf16_t Bs[GBN][GLD];   // transposed: Bs[n][k]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; i++) acc[i] = 0.0f;
    // each thread stages 8 elements of A and 8 of B per K step
    const int ar = tid >> 2, ak = (tid & 3) * 8;   // A: row, k-chunk
    const int bk = tid >> 3, bn = (tid & 7) * 8;   // B: k, n-chunk
    for (int k0 = 0; k0 < g.K; k0 += GBK) {
        {
            const int m = m0 + ar;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const int k = k0 + ak + j;
                As[ar][ak + j] = (m < g.M && k < g.K) ? g.A[m * g.sam + k * g.sak] : (bf16_t)0;
            }
            const int k = k0 + bk;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const int n = n0 + bn + j;
                Bs[bn + j][bk] = (k < g.K && n < g.N) ? g.B[k * g.sbk + n * g.sbn] : (bf16_t)0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GBK; kk += 16) {
            const int kl = kk + 8 * (lane >> 5);
            const u16x8 a = *(const u16x8 *)&As[wm + (lane & 31)][kl];
            const u16x8 b = *(const u16x8 *)&Bs[wn + (lane & 31)][kl];
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                          __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // accumulator element i of lane l holds (row 8*(i/4) + 4*(l/32) + i%4, col l%32)
    const int n = n0 + wn + (lane & 31);
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const int m = m0 + wm + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        if (m >= g.M || n >= g.N) continue;
        const float v = acc[i];
        if (EPI == EPI_F32) {
            g.C[(long)m * g.scm + n] = v;
        } else if (EPI == EPI_BIAS_RELU) {
            const float z = v + g.bias[n];
            g.H[(long)m * g.shm + n] = f2bf(z > 0.0f ? z : 0.0f);
        } else {
            const float dz = bf2f(g.mask[(long)m * g.smm + n]) > 0.0f ? v : 0.0f;
            g.C[(long)m * g.scm + n] = dz;
            g.H[(long)m * g.shm + n] = f2bf(dz);
        }
    }
}

template <int EPI>
static void gemm(const GemmArgs &g, hipStream_t s)
{
    dim3 grid((g.N + GBN - 1) / GBN, (g.M + GBM - 1) / GBM);
    hipLaunchKernelGGL(gemm_bf16_kernel<EPI>, grid, dim3(256), 0, s, g);
}

// ------------------------------------------------------------------ small kernels

// a0[r][k] = bf16(X[idx(r)][k]) with idx(r) = order[step*rows + r] (or r);
// tgt[r] = Y[idx(r)]
__global__ void gather_round_kernel(const float *X, const float *Y, const int32_t *order, const long long *step,
                                    int rows, bf16_t *a0, float *tgt)
{
    const int r = blockIdx.x;
    if (r >= rows) return;
    const long long base = (order && step) ? *step * rows : 0;
    const long long src = order ? order[base + r] : r;
    for (int k = threadIdx.x; k < kIn; k += blockDim.x) a0[r * kIn + k] = f2bf(X[src * kIn + k]);
    if (threadIdx.x == 0 && tgt && Y) tgt[r] = Y[src];
}

// One wave per row: y = a3 . bf16(W4) + b4; with targets, also the start of
// the backward pass for the Huber loss of e = y - t (e^2 / 2 for |e| <= kHuber,
// kHuber (|e| - kHuber / 2) beyond): dy = clamp(e, -kHuber, kHuber) / rows,
// dz3 = dy * bf16(W4) * (a3 > 0).
__global__ void head_kernel(const bf16_t *a3, const bf16_t *w4b, const float *b4, int rows, float *yhat,
                            const float *tgt, float *dy, float *rloss, float *dz3, bf16_t *g3)
{
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (r >= rows) return;
    float s = 0.0f;
    float w[4], a[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int k = lane + 64 * j;
        w[j] = bf2f(w4b[k]);
        a[j] = bf2f(a3[r * kHid + k]);
        s += a[j] * w[j];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    const float y = s + b4[0];
    if (lane == 0 && yhat) yhat[r] = y;
    if (!tgt) return;
    const float e = y - tgt[r];
    const float ae = fabsf(e);
    const float d = fminf(fmaxf(e, -kHuber), kHuber) / (float)rows;
    if (lane == 0) {
        dy[r] = d;
        rloss[r] = ae <= kHuber ? 0.5f * e * e : kHuber * (ae - 0.5f * kHuber);
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int k = lane + 64 * j;
        const float z = a[j] > 0.0f ? d * w[j] : 0.0f;
        dz3[r * kHid + k] = z;
        g3[r * kHid + k] = f2bf(z);
    }
}

// Column sums over rows, fixed order: out[n] = sum_r src[r][n] (+ weighted
// variant out[n] = sum_r wgt[r] * bf(a)[r][n]).  One thread per column.
__global__ void colsum_kernel(const float *src, int rows, int cols, float *out)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= cols) return;
    float s = 0.0f;
    for (int r = 0; r < rows; r++) s += src[(long)r * cols + n];
    out[n] = s;
}

// gW4[k] = sum_r a3[r][k] dy[r]; gb4 = sum_r dy[r]; loss = sum_r rloss[r] / rows
__global__ void head_reduce_kernel(const bf16_t *a3, const float *dy, const float *rloss, int rows, float *gw4,
                                   float *gb4, float *loss_buf, const long long *step)
{
    const int k = threadIdx.x;
    float s = 0.0f;
    for (int r = 0; r < rows; r++) s += bf2f(a3[r * kHid + k]) * dy[r];
    gw4[k] = s;
    if (k == 0) {
        float d = 0.0f, q = 0.0f;
        for (int r = 0; r < rows; r++) { d += dy[r]; q += rloss[r]; }
        gb4[0] = d;
        if (loss_buf) loss_buf[step ? *step : 0] = q / (float)rows;
    }
}

struct Hyper {
    float lr, b1, b2, eps;
};

// Adam on the float32 master weights; t = *step + 1; refreshes the bf16
// copies of the weights.
__global__ void adam_kernel(float *p, const float *g, float *m, float *v, bf16_t *wb, const Hyper *h,
                            const long long *step)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNParams) return;
    const float b1 = h->b1, b2 = h->b2;
    const float t = (float)(*step + 1);
    const float c1 = 1.0f - powf(b1, t), c2 = 1.0f - powf(b2, t);
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - h->lr * (mi / c1) / (sqrtf(vi / c2) + h->eps);
    p[i] = pi;
    if (i < kNBf) wb[i] = f2bf(pi);
}

__global__ void step_advance_kernel(long long *step) { *step += 1; }

__global__ void to_bf16_kernel(const float *p, bf16_t *wb, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = f2bf(p[i]);
}

}  // namespace esc

using namespace esc;

struct esc_mlp {
    esc_ctx *ctx = nullptr;
    int device = 0;                                                  // destruction never touches ctx
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;   // kNParams each
    bf16_t *wb = nullptr;                                            // kNBf
    bf16_t *a0 = nullptr, *a1 = nullptr, *a2 = nullptr, *a3 = nullptr;
    bf16_t *gd[2] = {nullptr, nullptr};                              // bf16 deltas (ping-pong)
    float *dz = nullptr, *tgt = nullptr, *dy = nullptr, *sq = nullptr;
    Hyper *hyper = nullptr;
    long long *steps = nullptr;   // [0] global Adam step, [1] step within the current train call
    float *loss = nullptr;
    int64_t loss_cap = 0;
    hipStream_t cap = nullptr;
};

namespace {

int hipchk(hipError_t e, const char *what) { return e == hipSuccess ? ESC_OK : hip_fail(e, what); }

__global__ void reset_local_step_kernel(long long *steps) { steps[1] = 0; }

__global__ void advance_kernel(long long *steps)
{
    steps[0] += 1;
    steps[1] += 1;
}

// forward of `rows` rows already in m->a0 (bf16); fills a1..a3 and yhat; with
// targets (m->tgt) the head also starts the backward pass
void forward(esc_mlp *m, int rows, float *yhat, hipStream_t s, bool with_targets)
{
    GemmArgs g{};
    g.M = rows;
    g.N = kHid;
    g.K = kIn;
    g.A = m->a0; g.sam = kIn; g.sak = 1;
    g.B = m->wb + kOffW1; g.sbk = kHid; g.sbn = 1;
    g.bias = m->p + kOffB1;
    g.H = m->a1; g.shm = kHid;
    gemm<EPI_BIAS_RELU>(g, s);
    g.K = kHid;
    g.A = m->a1; g.sam = kHid;
    g.B = m->wb + kOffW2;
    g.bias = m->p + kOffB2;
    g.H = m->a2;
    gemm<EPI_BIAS_RELU>(g, s);
    g.A = m->a2;
    g.B = m->wb + kOffW3;
    g.bias = m->p + kOffB3;
    g.H = m->a3;
    gemm<EPI_BIAS_RELU>(g, s);
    const int rpb = 4;   // rows (waves) per block
    hipLaunchKernelGGL(head_kernel, dim3((rows + rpb - 1) / rpb), dim3(64 * rpb), 0, s, m->a3, m->wb + kOffW4,
                       m->p + kOffB4, rows, yhat, with_targets ? m->tgt : nullptr, m->dy, m->sq, m->dz, m->gd[0]);
}

// backward of the last forward with targets: gradients into m->g
void backward(esc_mlp *m, int rows, hipStream_t s, float *loss_buf, const long long *lstep)
{
    float *G = m->g;
    hipLaunchKernelGGL(head_reduce_kernel, dim3(1), dim3(kHid), 0, s, m->a3, m->dy, m->sq, rows, G + kOffW4,
                       G + kOffB4, loss_buf, lstep);
    hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(kHid), 0, s, m->dz, rows, kHid, G + kOffB3);
    const bf16_t *acts[3] = {m->a0, m->a1, m->a2};
    const int fan_in[3] = {kIn, kHid, kHid};
    const int offW[3] = {kOffW1, kOffW2, kOffW3};
    const int offB[3] = {kOffB1, kOffB2, kOffB3};
    int cur = 0;   // m->gd[cur] holds the bf16 delta of layer l's output
    for (int l = 2; l >= 0; l--) {
        // gW_l = act_l^T * delta_l  (reduction over the rows)
        GemmArgs w{};
        w.M = fan_in[l]; w.N = kHid; w.K = rows;
        w.A = acts[l]; w.sam = 1; w.sak = fan_in[l];      // A(i, r) = act[r][i]
        w.B = m->gd[cur]; w.sbk = kHid; w.sbn = 1;        // B(r, n) = delta[r][n]
        w.C = G + offW[l]; w.scm = kHid;
        gemm<EPI_F32>(w, s);
        if (l == 0) break;
        // delta_{l-1} = (delta_l * W_l^T) masked by act_l > 0
        GemmArgs d{};
        d.M = rows; d.N = kHid; d.K = kHid;
        d.A = m->gd[cur]; d.sam = kHid; d.sak = 1;        // delta[r][j]
        d.B = m->wb + offW[l]; d.sbk = 1; d.sbn = kHid;   // B(j, i) = W_l[i][j]
        d.C = m->dz; d.scm = kHid;
        d.H = m->gd[cur ^ 1]; d.shm = kHid;
        d.mask = acts[l]; d.smm = kHid;
        gemm<EPI_MASKED>(d, s);
        hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(kHid), 0, s, m->dz, rows, kHid, G + offB[l - 1]);
        cur ^= 1;
    }
}

void free_mlp(esc_mlp *m)
{
    void *ptrs[] = {m->p, m->g, m->m, m->v, m->wb, m->a0, m->a1, m->a2, m->a3, m->gd[0], m->gd[1],
                    m->dz, m->tgt, m->dy, m->sq, m->hyper, m->steps, m->loss};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    if (m->cap) (void)hipStreamDestroy(m->cap);
    delete m;
}

int check_mlp(const esc_mlp *m)
{
    if (!m) return fail(ESC_ERR_INVALID, "null mlp handle");
    return set_device(m->device);
}

}  // namespace

extern "C" {

int esc_mlp_create(esc_ctx *ctx, esc_mlp **out)
{
    if (!ctx || !out) return fail(ESC_ERR_INVALID, "null argument");
    if (int rc0 = set_device(ctx->device)) return rc0;
    esc_mlp *m = new (std::nothrow) esc_mlp;
    if (!m) return fail(ESC_ERR_OOM, "out of host memory");
    m->ctx = ctx;
    m->device = ctx->device;
    struct { void **p; size_t bytes; } allocs[] = {
        {(void **)&m->p, kNParams * 4}, {(void **)&m->g, kNParams * 4}, {(void **)&m->m, kNParams * 4},
        {(void **)&m->v, kNParams * 4}, {(void **)&m->wb, kNBf * 2}, {(void **)&m->a0, kMaxRows * kIn * 2},
        {(void **)&m->a1, kMaxRows * kHid * 2}, {(void **)&m->a2, kMaxRows * kHid * 2},
        {(void **)&m->a3, kMaxRows * kHid * 2}, {(void **)&m->gd[0], kMaxRows * kHid * 2},
        {(void **)&m->gd[1], kMaxRows * kHid * 2}, {(void **)&m->dz, kMaxRows * kHid * 4},
        {(void **)&m->tgt, kMaxRows * 4}, {(void **)&m->dy, kMaxRows * 4}, {(void **)&m->sq, kMaxRows * 4},
        {(void **)&m->hyper, sizeof(Hyper)}, {(void **)&m->steps, 2 * sizeof(long long)}};
    for (auto &a : allocs) {
        hipError_t e = hipMalloc(a.p, a.bytes);
        if (e != hipSuccess) { free_mlp(m); return fail(ESC_ERR_OOM, "hipMalloc: %s", hipGetErrorString(e)); }
    }
    hipError_t e = hipStreamCreateWithFlags(&m->cap, hipStreamNonBlocking);
    if (e != hipSuccess) { free_mlp(m); return hip_fail(e, "stream"); }
    // zero parameters until set
    std::vector<float> z(kNParams, 0.0f);
    int rc = esc_mlp_set_params(m, z.data());
    if (rc) { free_mlp(m); return rc; }
    *out = m;
    return ESC_OK;
}

int esc_mlp_destroy(esc_mlp *m)
{
    if (!m) return ESC_OK;
    (void)set_device(m->device);
    free_mlp(m);
    return ESC_OK;
}

int esc_mlp_set_params(esc_mlp *m, const float *host_params)
{
    int rc = check_mlp(m);
    if (rc) return rc;
    if (!host_params) return fail(ESC_ERR_INVALID, "null parameters");
    hipStream_t s = m->cap;
    if ((rc = hipchk(hipMemcpyAsync(m->p, host_params, kNParams * 4, hipMemcpyHostToDevice, s), "upload"))) return rc;
    if ((rc = hipchk(hipMemsetAsync(m->m, 0, kNParams * 4, s), "memset"))) return rc;
    if ((rc = hipchk(hipMemsetAsync(m->v, 0, kNParams * 4, s), "memset"))) return rc;
    if ((rc = hipchk(hipMemsetAsync(m->steps, 0, 2 * sizeof(long long), s), "memset"))) return rc;
    hipLaunchKernelGGL(to_bf16_kernel, dim3((kNBf + 255) / 256), dim3(256), 0, s, m->p, m->wb, kNBf);
    return hipchk(hipStreamSynchronize(s), "sync");
}

int esc_mlp_get_params(esc_mlp *m, float *host_params)
{
    int rc = check_mlp(m);
    if (rc) return rc;
    if (!host_params) return fail(ESC_ERR_INVALID, "null output");
    if ((rc = hipchk(hipMemcpyAsync(host_params, m->p, kNParams * 4, hipMemcpyDeviceToHost, m->cap), "download")))
        return rc;
    return hipchk(hipStreamSynchronize(m->cap), "sync");
}

int esc_mlp_predict(esc_mlp *m, const float *dev_x, int64_t n, float *dev_yhat, void *stream)
{
    int rc = check_mlp(m);
    if (rc) return rc;
    if (n < 0 || (n > 0 && (!dev_x || !dev_yhat))) return fail(ESC_ERR_INVALID, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    for (int64_t r0 = 0; r0 < n; r0 += kMaxRows) {
        const int rows = (int)std::min<int64_t>(kMaxRows, n - r0);
        hipLaunchKernelGGL(gather_round_kernel, dim3(rows), dim3(64), 0, s, dev_x + r0 * kIn, nullptr, nullptr,
                           nullptr, rows, m->a0, nullptr);
        forward(m, rows, dev_yhat + r0, s, false);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ESC_OK : hip_fail(e, "predict launch");
}

int esc_mlp_gradients(esc_mlp *m, const float *dev_x, const float *dev_y, int64_t n, float *dev_grads,
                      void *stream)
{
    int rc = check_mlp(m);
    if (rc) return rc;
    if (n < 1 || n > kMaxRows || !dev_x || !dev_y || !dev_grads)
        return fail(ESC_ERR_INVALID, "need 1 <= n <= %d and non-null buffers", kMaxRows);
    hipStream_t s = (hipStream_t)stream;
    const int rows = (int)n;
    hipLaunchKernelGGL(gather_round_kernel, dim3(rows), dim3(64), 0, s, dev_x, dev_y, nullptr, nullptr, rows, m->a0,
                       m->tgt);
    forward(m, rows, nullptr, s, true);
    backward(m, rows, s, nullptr, nullptr);
    if ((rc = hipchk(hipMemcpyAsync(dev_grads, m->g, kNParams * 4, hipMemcpyDeviceToDevice, s), "copy grads")))
        return rc;
    return hipchk(hipStreamSynchronize(s), "sync");
}

int esc_mlp_train(esc_mlp *m, const float *dev_x, const float *dev_y, const int32_t *dev_order, int64_t steps,
                  int batch, float lr, void *stream, float *host_loss)
{
    int rc = check_mlp(m);
    if (rc) return rc;
    if (steps < 0 || batch < 1 || batch > kMaxRows || !dev_x || !dev_y || !dev_order || !(lr > 0.0f))
        return fail(ESC_ERR_INVALID, "bad training arguments");
    if (steps == 0) return ESC_OK;
    hipStream_t s = (hipStream_t)stream;
    if (host_loss && steps > m->loss_cap) {
        if (m->loss) (void)hipFree(m->loss);
        m->loss = nullptr;
        m->loss_cap = 0;
        hipError_t e = hipMalloc((void **)&m->loss, steps * sizeof(float));
        if (e != hipSuccess) return fail(ESC_ERR_OOM, "loss buffer: %s", hipGetErrorString(e));
        m->loss_cap = steps;
    }
    Hyper h{lr, 0.9f, 0.999f, 1e-8f};
    if ((rc = hipchk(hipMemcpyAsync(m->hyper, &h, sizeof h, hipMemcpyHostToDevice, s), "hyper"))) return rc;
    hipLaunchKernelGGL(reset_local_step_kernel, dim3(1), dim3(1), 0, s, m->steps);
    // one training step, captured once for this call and replayed `steps` times
    hipStream_t c = m->cap;
    if ((rc = hipchk(hipStreamBeginCapture(c, hipStreamCaptureModeThreadLocal), "begin capture"))) return rc;
    hipLaunchKernelGGL(gather_round_kernel, dim3(batch), dim3(64), 0, c, dev_x, dev_y, dev_order, m->steps + 1,
                       batch, m->a0, m->tgt);
    forward(m, batch, nullptr, c, true);
    backward(m, batch, c, host_loss ? m->loss : nullptr, m->steps + 1);
    hipLaunchKernelGGL(adam_kernel, dim3((kNParams + 255) / 256), dim3(256), 0, c, m->p, m->g, m->m, m->v, m->wb,
                       m->hyper, m->steps);
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(1), 0, c, m->steps);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(c, &graph);
    if (e != hipSuccess) return hip_fail(e, "end capture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "instantiate");
    for (int64_t i = 0; i < steps && e == hipSuccess; i++) e = hipGraphLaunch(exec, s);
    if (e == hipSuccess && host_loss)
        e = hipMemcpyAsync(host_loss, m->loss, steps * sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipGraphExecDestroy(exec);
    return e == hipSuccess ? ESC_OK : hip_fail(e, "training");
}

}  // extern "C"
