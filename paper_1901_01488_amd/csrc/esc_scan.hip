// esc_scan.hip -- gfx950 kernels and host entry points of the plain ESC scan:
// the COUNT(*) selectivity sub-query (Section 2) and its materialization as
// a temporary table in row order (Section 2, Section 2.1).
//
// Data layout: every column is a contiguous array of nrows 4-byte values
// (int32, date32 or float32), 16-byte aligned.  A block of 256 threads owns
// tiles of 256*RPT rows; in chunk j of a tile, thread t loads the 16 bytes of
// rows [base + (j*256 + t)*4, +4) of every column the predicate reads, so
// every load instruction of a wave is one fully coalesced 1 KiB request.
// The predicate program (esc_program.h) then runs with wave-uniform control:
// each test produces one 64-bit lane mask per row slot (a v_cmp result, i.e.
// a ballot), clauses combine masks on the scalar unit and the count is a
// scalar popcount.  Nothing per row is stored.
//
// Materialization is a single-pass, order-preserving stream compaction:
// tiles are claimed in increasing order from an atomic counter, each tile's
// row count becomes its aggregate, and a wave-parallel decoupled look-back
// over the predecessors' (flag, value) words -- one 64-bit atomic word each --
// yields the tile's exclusive prefix; each selected row is then written at
// prefix + its rank inside the tile (mbcnt over the lane masks).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <mutex>
#include <new>
#include <type_traits>

#include "esc_host.h"
#include "esc_kernels.h"

namespace esc {

// ------------------------------------------------------------------ device helpers

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float as_f(uint32_t u) { return __uint_as_float(u); }

template <int K, int C = 0, typename F>
__device__ __forceinline__ void for_slot(int s, F &&f)
{
    if constexpr (C < K) {
        if (s == C) f(std::integral_constant<int, C>{});
        else for_slot<K, C + 1>(s, f);
    }
}

// Lane masks of one test, folded straight into the clause state: MODE 0 ORs
// into the open clause cm, MODE 1 (a one-leaf clause) ANDs into acc.
template <int MODE, int RPT, typename T>
__device__ __forceinline__ void fold(uint64_t (&acc)[RPT], uint64_t (&cm)[RPT], T &&test)
{
#pragma unroll
    for (int r = 0; r < RPT; r++) {
        const uint64_t m = __ballot(test(r));
        if (MODE == 0) cm[r] |= m;
        else acc[r] &= m;
    }
}

template <int MODE, int RPT>
__device__ __forceinline__ void run_test(const Insn &I, const uint32_t *kpool, const uint32_t (&x)[RPT],
                                         uint64_t (&acc)[RPT], uint64_t (&cm)[RPT])
{
    switch (I.op) {
    case T_RANGE_I32: {
        const uint32_t lo = (uint32_t)I.a, span = (uint32_t)I.b;
        fold<MODE>(acc, cm, [&](int r) { return x[r] - lo <= span; });
        break;
    }
    case T_RANGE_F32: {
        const float lo = as_f((uint32_t)I.a), hi = as_f((uint32_t)I.b);
        fold<MODE>(acc, cm, [&](int r) { const float f = as_f(x[r]); return lo <= f && f <= hi; });
        break;
    }
    case T_BITSET: {
        const uint32_t lo = (uint32_t)I.a;
        const uint64_t bits = (uint64_t)(uint32_t)I.b | ((uint64_t)(uint32_t)I.c << 32);
        fold<MODE>(acc, cm, [&](int r) {
            const uint32_t d = x[r] - lo;
            return d < 64u && ((bits >> (d & 63u)) & 1ull);
        });
        break;
    }
    case T_IN_I32:
    case T_IN_F32: {
        // OR over the set members per row, then fold once
        uint64_t m[RPT];
#pragma unroll
        for (int r = 0; r < RPT; r++) m[r] = 0;
        const bool fl = I.op == T_IN_F32;
        for (int k = 0; k < I.b; k++) {
            const uint32_t kv = kpool[I.a + k];
            if (fl) {
                const float kf = as_f(kv);
#pragma unroll
                for (int r = 0; r < RPT; r++) m[r] |= __ballot(as_f(x[r]) == kf);
            } else {
#pragma unroll
                for (int r = 0; r < RPT; r++) m[r] |= __ballot(x[r] == kv);
            }
        }
#pragma unroll
        for (int r = 0; r < RPT; r++) {
            if (MODE == 0) cm[r] |= m[r];
            else acc[r] &= m[r];
        }
        break;
    }
    default:
        if (MODE == 1) {
#pragma unroll
            for (int r = 0; r < RPT; r++) acc[r] = 0;
        }
    }
}

template <int K, int RPT, int KK = (K > 0 ? K : 1)>
__device__ __forceinline__ void run_udf(const Insn &I, const uint32_t (&v)[KK][RPT], uint32_t (&u)[RPT])
{
    uint32_t o[RPT];
    if (I.flags & F_CONST) {
#pragma unroll
        for (int r = 0; r < RPT; r++) o[r] = (uint32_t)I.a;
    } else {
        for_slot<K>(I.src, [&](auto C) {
#pragma unroll
            for (int r = 0; r < RPT; r++) o[r] = v[C][r];
        });
    }
    switch (I.op) {
    case U_LOAD:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] = o[r];
        break;
    case U_ADD:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] += o[r];
        break;
    case U_SUB:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] -= o[r];
        break;
    case U_MUL:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] *= o[r];
        break;
    case U_MOD: {
        const int32_t m = I.a;   // > 0, checked by the compiler
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] = (uint32_t)((int32_t)u[r] % m);
        break;
    }
    case U_AND:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] &= o[r];
        break;
    case U_OR:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] |= o[r];
        break;
    case U_XOR:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] ^= o[r];
        break;
    case U_SHL:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] <<= (uint32_t)I.a;
        break;
    case U_SHR:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] = (uint32_t)((int32_t)u[r] >> I.a);
        break;
    }
}

// Runs the program on the loaded slots; acc[r] enters as the mask of valid
// rows and leaves as the mask of qualifying rows.
template <int K, int RPT, int KK = (K > 0 ? K : 1)>
__device__ __forceinline__ void run_program(const Program &P, const uint32_t (&v)[KK][RPT], uint64_t (&acc)[RPT])
{
    uint64_t cm[RPT];
    uint32_t u[RPT];
#pragma unroll
    for (int r = 0; r < RPT; r++) { cm[r] = 0; u[r] = 0; }
    const int n = P.ninsn;
    for (int i = 0; i < n; i++) {
        const Insn I = P.insn[i];
        if (I.op >= U_LOAD) {
            run_udf<K, RPT>(I, v, u);
            continue;
        }
        const bool single = I.flags & F_SINGLE;
        if (I.flags & F_SRC_UDF) {
            if (single) run_test<1, RPT>(I, P.kpool, u, acc, cm);
            else run_test<0, RPT>(I, P.kpool, u, acc, cm);
        } else if (single) {
            for_slot<K>(I.src, [&](auto C) { run_test<1, RPT>(I, P.kpool, v[C], acc, cm); });
        } else {
            for_slot<K>(I.src, [&](auto C) { run_test<0, RPT>(I, P.kpool, v[C], acc, cm); });
        }
        if (!single && (I.flags & F_END_CLAUSE)) {
#pragma unroll
            for (int r = 0; r < RPT; r++) { acc[r] &= cm[r]; cm[r] = 0; }
        }
    }
}

// Row of slot r for this thread: base + (j*256 + tid)*4 + e with r = 4j + e.
__device__ __forceinline__ int64_t row_of(int64_t base, int r)
{
    return base + ((int64_t)(r >> 2) * kScanBlock + threadIdx.x) * 4 + (r & 3);
}

template <int K, int RPT, int KK = (K > 0 ? K : 1)>
__device__ __forceinline__ void load_tile(const ColPtrs &cp, int64_t base, int64_t n, uint32_t (&v)[KK][RPT],
                                          uint64_t (&acc)[RPT])
{
    constexpr int TILE = kScanBlock * RPT;
    if (base + TILE <= n) {
#pragma unroll
        for (int j = 0; j < RPT / 4; j++) {
            const int64_t idx = base + ((int64_t)j * kScanBlock + threadIdx.x) * 4;
#pragma unroll
            for (int c = 0; c < K; c++) {
                const u32x4 q = __builtin_nontemporal_load((const u32x4 *)(cp.p[c] + idx));
                v[c][4 * j + 0] = q.x;
                v[c][4 * j + 1] = q.y;
                v[c][4 * j + 2] = q.z;
                v[c][4 * j + 3] = q.w;
            }
        }
#pragma unroll
        for (int r = 0; r < RPT; r++) acc[r] = ~0ull;
    } else {
#pragma unroll
        for (int r = 0; r < RPT; r++) {
            const int64_t row = row_of(base, r);
            const bool ok = row < n;
#pragma unroll
            for (int c = 0; c < K; c++) v[c][r] = ok ? cp.p[c][row] : 0u;
            acc[r] = __ballot(ok);
        }
    }
}

// ------------------------------------------------------------------ count

template <int K, int RPT>
__global__ __launch_bounds__(kScanBlock) void count_kernel(const Program P, const ColPtrs cp, int64_t n,
                                                           WsHeader *ws, unsigned long long *out)
{
    constexpr int TILE = kScanBlock * RPT;
    const int64_t ntiles = (n + TILE - 1) / TILE;
    uint32_t cnt = 0;   // wave-uniform
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        uint32_t v[K > 0 ? K : 1][RPT];
        uint64_t acc[RPT];
        load_tile<K, RPT>(cp, t * TILE, n, v, acc);
        run_program<K, RPT>(P, v, acc);
#pragma unroll
        for (int r = 0; r < RPT; r++) cnt += (uint32_t)__popcll(acc[r]);
    }
    __shared__ uint32_t s_cnt[kScanBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) s_cnt[wave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = 0;
        for (int w = 0; w < kScanBlock / 64; w++) b += s_cnt[w];
        if (b) atomicAdd(&ws->total, b);
        __threadfence();
        const unsigned tk = atomicAdd(&ws->ticket, 1u);
        if (tk == gridDim.x - 1) {
            // last block: every other block's add is visible; publish and reset
            __threadfence();
            const unsigned long long tot = atomicAdd(&ws->total, 0ull);
            *out = tot;
            atomicExch(&ws->total, 0ull);
            atomicExch(&ws->ticket, 0u);
        }
    }
}

// ------------------------------------------------------------------ materialize

constexpr unsigned long long kFlagAgg = 1ull << 62;
constexpr unsigned long long kFlagPrefix = 2ull << 62;
constexpr unsigned long long kValMask = (1ull << 62) - 1;
constexpr unsigned kSpinLimit = 1u << 24;

__device__ __forceinline__ unsigned long long ld_status(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_status(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Executed by one full wave.  Publishes the tile's aggregate, walks back over
// up to 64 predecessors at a time until one with an inclusive prefix is
// found, publishes the tile's own inclusive prefix and returns the exclusive
// one.  Every wait is bounded: after kSpinLimit polls the error flag is set
// and the walk gives up, so the grid always drains.
__device__ unsigned long long lookback(unsigned long long *status, int tile, unsigned long long agg, WsHeader *ws)
{
    const int lane = threadIdx.x & 63;
    if (tile == 0) {
        if (lane == 0) st_status(&status[0], kFlagPrefix | agg);
        return 0;
    }
    if (lane == 0) st_status(&status[tile], kFlagAgg | agg);
    unsigned long long excl = 0;
    int base = tile - 1;
    unsigned spins = 0;
    for (;;) {
        const int idx = base - lane;
        const unsigned long long s = idx >= 0 ? ld_status(&status[idx]) : kFlagPrefix;
        const unsigned flag = (unsigned)(s >> 62);
        const unsigned long long pm = __ballot(flag == 2);
        const unsigned long long inv = __ballot(flag == 0);
        const unsigned long long upto = pm ? (((pm & (~pm + 1)) << 1) - 1) : ~0ull;
        if (inv & upto) {
            if (++spins > kSpinLimit) {
                if (lane == 0) atomicOr(&ws->error, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        excl += wave_sum64(((upto >> lane) & 1ull) ? (s & kValMask) : 0ull);
        if (pm) break;
        base -= 64;
    }
    if (lane == 0) st_status(&status[tile], kFlagPrefix | (excl + agg));
    return excl;
}

template <int K, int RPT>
__global__ __launch_bounds__(kScanBlock) void materialize_kernel(const Program P, const ColPtrs cp, int64_t n,
                                                                 int ntiles, const ProjArgs pa, int32_t *rowids,
                                                                 unsigned long long cap, WsHeader *ws,
                                                                 unsigned long long *status)
{
    constexpr int TILE = kScanBlock * RPT;
    constexpr int NW = kScanBlock / 64;
    constexpr int NJ = RPT / 4;
    __shared__ int s_tile;
    __shared__ uint32_t s_wcnt[NJ][NW];
    __shared__ unsigned long long s_excl;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    constexpr int KK = K > 0 ? K : 1;
    for (;;) {
        if (threadIdx.x == 0) s_tile = (int)atomicAdd(&ws->tile_ctr, 1u);
        __syncthreads();
        const int tile = s_tile;
        if (tile >= ntiles) break;
        const int64_t base = (int64_t)tile * TILE;
        uint32_t v[KK][RPT];
        uint64_t acc[RPT];
        load_tile<K, RPT>(cp, base, n, v, acc);
        run_program<K, RPT>(P, v, acc);
#pragma unroll
        for (int j = 0; j < NJ; j++) {
            const uint32_t c = (uint32_t)(__popcll(acc[4 * j]) + __popcll(acc[4 * j + 1]) +
                                          __popcll(acc[4 * j + 2]) + __popcll(acc[4 * j + 3]));
            if (lane == 0) s_wcnt[j][wave] = c;
        }
        __syncthreads();
        // offset of (chunk j, this wave) inside the tile: chunk-major, then wave
        uint32_t off[NJ];
        uint32_t total = 0;
#pragma unroll
        for (int j = 0; j < NJ; j++)
#pragma unroll
            for (int w = 0; w < NW; w++) {
                if (w == wave) off[j] = total;
                total += s_wcnt[j][w];
            }
        if (wave == 0) {
            const unsigned long long ex = lookback(status, tile, total, ws);
            if (lane == 0) {
                s_excl = ex;
                if (tile == ntiles - 1) ws->result = ex + total;
            }
        }
        __syncthreads();
        const unsigned long long excl = s_excl;
        // rank of each selected row of this lane: lanes below first, then e
        unsigned long long pos[RPT];
        bool sel[RPT];
#pragma unroll
        for (int j = 0; j < NJ; j++) {
            unsigned long long p = excl + off[j];
#pragma unroll
            for (int e = 0; e < 4; e++) p += (unsigned long long)__popcll(acc[4 * j + e] & lt);
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const bool b = (acc[4 * j + e] >> lane) & 1ull;
                pos[4 * j + e] = p;
                sel[4 * j + e] = b && p < cap;
                p += b ? 1 : 0;
            }
        }
        if (rowids) {
#pragma unroll
            for (int r = 0; r < RPT; r++)
                if (sel[r]) rowids[pos[r]] = (int32_t)row_of(base, r);
        }
        for (int q = 0; q < pa.nproj; q++) {
            uint32_t *dst = pa.dst[q];
            const int slot = pa.slot[q];
            if (slot >= 0) {
                for_slot<KK>(slot, [&](auto C) {
#pragma unroll
                    for (int r = 0; r < RPT; r++)
                        if (sel[r]) dst[pos[r]] = v[C][r];
                });
            } else {
                const uint32_t *src = pa.src[q];
#pragma unroll
                for (int r = 0; r < RPT; r++)
                    if (sel[r]) dst[pos[r]] = src[row_of(base, r)];
            }
        }
        __syncthreads();   // s_tile, s_wcnt and s_excl are rewritten next round
    }
}

__global__ void zero_kernel(unsigned long long *p, int64_t nwords)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nwords; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// ------------------------------------------------------------------ dispatch tables

template <int K, int RPT>
struct ScanKernels {
    static constexpr CountFn count = count_kernel<K, RPT>;
    static constexpr MatFn mat = materialize_kernel<K, RPT>;
};

template <int RPT, int... Ks>
constexpr CountFn count_table_impl(int k, std::integer_sequence<int, Ks...>)
{
    CountFn t[] = {ScanKernels<Ks, RPT>::count...};
    return t[k];
}

CountFn count_fn(int k, int rpt)
{
    using S = std::make_integer_sequence<int, kMaxSlots + 1>;
    if (rpt == 4) return count_table_impl<4>(k, S{});
    return count_table_impl<8>(k, S{});
}

template <int RPT, int... Ks>
constexpr MatFn mat_table_impl(int k, std::integer_sequence<int, Ks...>)
{
    MatFn t[] = {ScanKernels<Ks, RPT>::mat...};
    return t[k];
}

MatFn mat_fn(int k, int rpt)
{
    using S = std::make_integer_sequence<int, kMaxSlots + 1>;
    if (rpt == 4) return mat_table_impl<4>(k, S{});
    return mat_table_impl<8>(k, S{});
}

void launch_zero(unsigned long long *p, int64_t nwords, hipStream_t s)
{
    if (nwords <= 0) return;
    int64_t blocks = (nwords + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, nwords);
}

}  // namespace esc
