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

#include "esc_device.h"
#include "esc_host.h"
#include "esc_kernels.h"

namespace esc {

// ------------------------------------------------------------------ count

// Grid-stride over tiles with a two-deep register pipeline: the loads of
// the block's next tile are in flight while the current one is evaluated.
template <int K, int RPT>
__global__ __launch_bounds__(kScanBlock) void count_kernel(const Program P, const ColPtrs cp, int64_t n,
                                                           WsHeader *ws, unsigned long long *out)
{
    constexpr int TILE = kScanBlock * RPT;
    constexpr int KK = K > 0 ? K : 1;
    const int64_t ntiles = (n + TILE - 1) / TILE;
    const int64_t step = gridDim.x;
    uint32_t cnt = 0;   // wave-uniform
    uint32_t va[KK][RPT], vb[KK][RPT];
    int64_t t = blockIdx.x;
    if (t < ntiles) load_vals<K, RPT>(cp, t * TILE, n, va);
    while (t < ntiles) {
        const int64_t t1 = t + step;
        if (t1 < ntiles) load_vals<K, RPT>(cp, t1 * TILE, n, vb);
        cnt += eval_count<K, RPT>(P, va, t * TILE, n);
        if (t1 >= ntiles) break;
        const int64_t t2 = t1 + step;
        if (t2 < ntiles) load_vals<K, RPT>(cp, t2 * TILE, n, va);
        cnt += eval_count<K, RPT>(P, vb, t1 * TILE, n);
        t = t2;
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

// Evaluates one loaded tile, obtains its exclusive prefix by look-back and
// writes its qualifying rows.  Called by the whole block.
template <int K, int RPT, int KK = (K > 0 ? K : 1)>
__device__ __forceinline__ void compact_tile(const Program &P, const uint32_t (&v)[KK][RPT], int tile, int ntiles,
                                             int64_t n, const ProjArgs &pa, int32_t *rowids,
                                             unsigned long long cap, WsHeader *ws, unsigned long long *status,
                                             uint32_t (*s_wcnt)[kScanBlock / 64], unsigned long long *s_excl)
{
    constexpr int TILE = kScanBlock * RPT;
    constexpr int NW = kScanBlock / 64;
    constexpr int NJ = RPT / 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)tile * TILE;
    uint64_t acc[RPT];
    valid_masks<RPT>(base, n, acc);
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
            *s_excl = ex;
            if (tile == ntiles - 1) ws->result = ex + total;
        }
    }
    __syncthreads();
    const unsigned long long excl = *s_excl;
    if (total == 0) return;
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
            const bool bit = (acc[4 * j + e] >> lane) & 1ull;
            pos[4 * j + e] = p;
            sel[4 * j + e] = bit && p < cap;
            p += bit ? 1 : 0;
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
}

// Persistent blocks claim tiles in increasing order from an atomic counter.
// The next tile is claimed and its loads issued before the current tile is
// evaluated, so memory stays busy during the look-back wait.
template <int K, int RPT>
__global__ __launch_bounds__(kScanBlock) void materialize_kernel(const Program P, const ColPtrs cp, int64_t n,
                                                                 int ntiles, const ProjArgs pa, int32_t *rowids,
                                                                 unsigned long long cap, WsHeader *ws,
                                                                 unsigned long long *status)
{
    constexpr int TILE = kScanBlock * RPT;
    constexpr int NW = kScanBlock / 64;
    constexpr int NJ = RPT / 4;
    constexpr int KK = K > 0 ? K : 1;
    __shared__ int s_tile[2];
    __shared__ uint32_t s_wcnt[NJ][NW];
    __shared__ unsigned long long s_excl;
    uint32_t va[KK][RPT], vb[KK][RPT];
    if (threadIdx.x == 0) s_tile[0] = (int)atomicAdd(&ws->tile_ctr, 1u);
    __syncthreads();
    int t = s_tile[0];
    if (t < ntiles) load_vals<K, RPT>(cp, (int64_t)t * TILE, n, va);
    while (t < ntiles) {
        if (threadIdx.x == 0) s_tile[1] = (int)atomicAdd(&ws->tile_ctr, 1u);
        __syncthreads();
        const int t1 = s_tile[1];
        if (t1 < ntiles) load_vals<K, RPT>(cp, (int64_t)t1 * TILE, n, vb);
        compact_tile<K, RPT>(P, va, t, ntiles, n, pa, rowids, cap, ws, status, s_wcnt, &s_excl);
        if (t1 >= ntiles) break;
        __syncthreads();   // s_tile, s_wcnt and s_excl are rewritten below
        if (threadIdx.x == 0) s_tile[0] = (int)atomicAdd(&ws->tile_ctr, 1u);
        __syncthreads();
        const int t2 = s_tile[0];
        if (t2 < ntiles) load_vals<K, RPT>(cp, (int64_t)t2 * TILE, n, va);
        compact_tile<K, RPT>(P, vb, t1, ntiles, n, pa, rowids, cap, ws, status, s_wcnt, &s_excl);
        __syncthreads();
        t = t2;
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
