// esc_join.hip -- gfx950 hash join over the outputs of exact selectivity
// computation: build hash tables on (filtered) build relations, then count
// the rows of the star join of the probe relation with them in one pass.
//
// Section 2.2 joins a probe relation (the largest) with build relations,
// hash tables being built on the build side, and pushes selections down
// only there; the build inputs are then the temporary tables of Section 2.1.
// A hash table is an open-addressing array of 2^m 8-byte slots, at least
// two per key, with linear probing; a slot holds (payload << 32 | key), the
// payload being the build row's index, and all-ones marks an empty slot
// (payloads are below 2^31, so no filled slot is all ones).  Several rows
// may share a key: each takes its own slot, and a lookup counts the slots
// holding its key up to the first empty one.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "esc_device.h"
#include "esc_runtime.h"

namespace esc {

constexpr unsigned long long kEmpty = ~0ull;
constexpr int kJoinMaxTables = 4;
constexpr int kProbeRPT = 16;

struct HashRef {
    const unsigned long long *slots[kJoinMaxTables];
    uint32_t mask[kJoinMaxTables];
    int32_t shift[kJoinMaxTables];   // 32 - log2(slots)
};

// Fibonacci hashing: the top m bits of key * 2^32 / golden ratio
__device__ __forceinline__ uint32_t slot_of(int32_t key, int shift)
{
    return ((uint32_t)key * 0x9E3779B1u) >> shift;
}

__global__ void fill_empty_kernel(unsigned long long *slots, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        slots[i] = kEmpty;
}

// One thread per build row (grid-stride).  At least half the slots stay
// empty, so every probe sequence ends within `mask + 1` steps.
__global__ void build_kernel(const int32_t *__restrict__ keys, int64_t n, unsigned long long *slots, uint32_t mask,
                             int shift)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t key = keys[i];
        const unsigned long long v = ((unsigned long long)(uint32_t)i << 32) | (uint32_t)key;
        uint32_t s = slot_of(key, shift);
        for (uint32_t step = 0; step <= mask; step++) {
            if (atomicCAS(&slots[s], kEmpty, v) == kEmpty) break;
            s = (s + 1u) & mask;
        }
    }
}

// slots holding `key`, up to the first empty slot of its probe sequence
__device__ __forceinline__ uint32_t matches(const unsigned long long *__restrict__ slots, uint32_t mask, int shift,
                                            int32_t key)
{
    uint32_t s = slot_of(key, shift), c = 0;
    for (uint32_t step = 0; step <= mask; step++) {
        const unsigned long long v = slots[s];
        if (v == kEmpty) break;
        c += (uint32_t)((uint32_t)v == (uint32_t)key);
        s = (s + 1u) & mask;
    }
    return c;
}

// Star-join count: sum over probe rows of the product over build sides of
// the matching build rows.  The probe's key columns are read as in the
// scans (wave tiles of 64 * 16 rows, 16-byte coalesced loads); per-block
// sums go to one 64-bit atomic.
template <int K>
__global__ __launch_bounds__(kScanBlock) void probe_count_kernel(const ColPtrs cp, int64_t n, const HashRef h,
                                                                 unsigned long long *out)
{
    constexpr int RPT = kProbeRPT;
    constexpr int TILE = kWave * RPT;
    constexpr int NW = kScanBlock / kWave;
    const int64_t ntiles = (n + TILE - 1) / TILE;
    const int64_t step = (int64_t)gridDim.x * NW;
    unsigned long long acc = 0;   // per lane
    for (int64_t t = (int64_t)blockIdx.x * NW + wave_id(); t < ntiles; t += step) {
        uint32_t v[K][RPT];
        load_vals<K, RPT>(cp, t * TILE, n, v);
        const uint32_t valid = valid_bits<RPT>(t * TILE, n);
#pragma unroll
        for (int r = 0; r < RPT; r++) {
            if (!((valid >> r) & 1u)) continue;
            unsigned long long prod = 1;
#pragma unroll
            for (int j = 0; j < K; j++) {
                if (prod == 0) break;
                prod *= matches(h.slots[j], h.mask[j], h.shift[j], (int32_t)v[j][r]);
            }
            acc += prod;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    __shared__ unsigned long long s_acc[NW];
    if (lane_id() == 0) s_acc[wave_id()] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = 0;
        for (int w = 0; w < NW; w++) b += s_acc[w];
        if (b) atomicAdd(out, b);
    }
}

// capacity (slots) of a table of `bytes`; 0 if the size is not 256 + 8 * 2^m, m in [6, 31]
int64_t table_slots(size_t bytes)
{
    if (bytes < 256 + 8 * 64) return 0;
    const size_t s = (bytes - 256) / 8;
    if ((s & (s - 1)) != 0 || s > (1ull << 31)) return 0;
    return (int64_t)s;
}

int log2_exact(int64_t s)
{
    int m = 0;
    while ((1ll << m) < s) m++;
    return m;
}

}  // namespace esc

using namespace esc;

extern "C" {

int esc_hash_table_bytes(int64_t nkeys, size_t *bytes)
{
    if (!bytes || nkeys < 0) return fail(ESC_ERR_INVALID, "null argument or nkeys < 0");
    if (nkeys > (1ll << 30)) return fail(ESC_ERR_UNSUPPORTED, "more than 2^30 keys");
    int64_t s = 64;
    while (s < 2 * nkeys) s *= 2;
    *bytes = 256 + 8 * (size_t)s;
    return ESC_OK;
}

int esc_hash_build(esc_ctx *ctx, const int32_t *dev_keys, int64_t nkeys, void *dev_table, size_t table_bytes,
                   void *stream)
{
    if (!ctx || !dev_table || (nkeys > 0 && !dev_keys) || nkeys < 0) return fail(ESC_ERR_INVALID, "null argument");
    const int64_t slots = table_slots(table_bytes);
    if (slots == 0) return fail(ESC_ERR_INVALID, "table_bytes %zu is not a size from esc_hash_table_bytes", table_bytes);
    if (2 * nkeys > slots) return fail(ESC_ERR_INVALID, "%lld keys need %lld slots or more, the table has %lld",
                                      (long long)nkeys, (long long)(2 * nkeys), (long long)slots);
    int rc = set_device(ctx->device);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *sl = (unsigned long long *)((char *)dev_table + 256);
    const int grid = ctx->num_cus * 8;
    hipLaunchKernelGGL(fill_empty_kernel, dim3(grid), dim3(256), 0, s, sl, slots);
    if (nkeys > 0) {
        const int m = log2_exact(slots);
        hipLaunchKernelGGL(build_kernel, dim3(grid), dim3(256), 0, s, dev_keys, nkeys, sl, (uint32_t)(slots - 1),
                           32 - m);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ESC_OK : hip_fail(e, "hash build launch");
}

int esc_join_count(esc_ctx *ctx, const esc_table *probe, const int32_t *key_cols, void *const *dev_tables,
                   const size_t *table_bytes, int ntables, void *dev_ws, size_t ws_bytes, void *stream,
                   uint64_t *out_count)
{
    if (!ctx || !probe || !key_cols || !dev_tables || !table_bytes || !out_count)
        return fail(ESC_ERR_INVALID, "null argument");
    if (!dev_ws || ((uintptr_t)dev_ws & 255)) return fail(ESC_ERR_ALIGN, "workspace must be non-null and 256-byte aligned");
    if (ws_bytes < sizeof(WsHeader)) return fail(ESC_ERR_OOM, "workspace of %zu bytes, %zu needed", ws_bytes, sizeof(WsHeader));
    if (ntables < 1 || ntables > kJoinMaxTables)
        return fail(ESC_ERR_INVALID, "ntables %d outside [1, %d]", ntables, kJoinMaxTables);
    if (!probe->has_data()) return fail(ESC_ERR_INVALID, "probe table has no device columns");
    HashRef h{};
    ColPtrs cp{};
    cp.nt = ctx->nt;
    for (int j = 0; j < ntables; j++) {
        const int c = key_cols[j];
        if (c < 0 || c >= (int)probe->dtypes.size()) return fail(ESC_ERR_INVALID, "key column %d out of range", c);
        if (probe->dtypes[c] == ESC_FLOAT32) return fail(ESC_ERR_TYPE, "key column %d is float32", c);
        const int64_t slots = table_slots(table_bytes[j]);
        if (slots == 0 || !dev_tables[j]) return fail(ESC_ERR_INVALID, "hash table %d: bad pointer or size", j);
        h.slots[j] = (const unsigned long long *)((const char *)dev_tables[j] + 256);
        h.mask[j] = (uint32_t)(slots - 1);
        h.shift[j] = 32 - log2_exact(slots);
        cp.p[j] = (const uint32_t *)probe->cols[c];
    }
    int rc = set_device(ctx->device);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *d_out = &((WsHeader *)dev_ws)->result;
    hipError_t e;
    launch_zero(d_out, 1, s);
    const int64_t n = probe->nrows;
    if (n > 0) {
        // lookups are latency-bound random reads: as many waves as fit
        typedef void (*ProbeFn)(const ColPtrs, int64_t, const HashRef, unsigned long long *);
        const ProbeFn fns[] = {probe_count_kernel<1>, probe_count_kernel<2>, probe_count_kernel<3>,
                               probe_count_kernel<4>};
        const ProbeFn fn = fns[ntables - 1];
        constexpr int TILE = kWave * kProbeRPT;
        const int64_t blocks_needed = ((n + TILE - 1) / TILE + 3) / 4;
        int64_t grid = (int64_t)ctx->num_cus * occupancy((const void *)fn, kScanBlock, 0);
        if (grid > blocks_needed) grid = blocks_needed;
        hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(kScanBlock), 0, s, cp, n, h, d_out);
    }
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "join probe launch");
    if ((e = hipMemcpyAsync(ctx->pinned, d_out, 8, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    *out_count = ctx->pinned[0];
    return ESC_OK;
}

}  // extern "C"
