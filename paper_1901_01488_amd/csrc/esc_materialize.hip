// esc_materialize.hip -- gfx950 kernels that materialize a selection as a
// temporary table in row order (Section 2, Section 2.1): order-preserving
// stream compaction in passes with no inter-block waiting, after the count
// pass of esc_count.hip stored per-tile counts and lane masks:
//   1. one block scans the tile counts into row-order output offsets;
//   2. the write pass reads the masks instead of the predicate's columns,
//      ranks the qualifying rows of each 256-row chunk with ballot masks,
//      compacts row ids and projected values in LDS and writes them as
//      contiguous runs at offset + rank.
// When the count pass was the caller's own preceding esc_count on the same
// workspace, table and predicate (count, decide, then materialize),
// materialization never reads the predicate's columns again.  A
// single-pass compaction with decoupled look-back serves a materialization
// with no count before it when asked for.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <type_traits>
#include <utility>

#include "esc_device.h"
#include "esc_host.h"
#include "esc_kernels.h"

namespace esc {

// ------------------------------------------------------------------ scan

// Exclusive scan of m per-tile counts into offsets[0..m]; offsets[m] is the
// total, also stored in ws->result.  One block of 1024 threads walks the
// counts in rounds of 16384: each thread takes 16 consecutive counts (four
// 16-byte loads, coalesced across the block), the thread totals are scanned
// with wave shuffles and a 16-entry LDS pass, and a carry links the rounds.
__global__ __launch_bounds__(1024) void scan_kernel(const uint32_t *counts, int64_t m, uint32_t *offsets,
                                                    WsHeader *ws, unsigned long long *total)
{
    constexpr int PER = 16, NT = 1024, NWV = NT / 64;
    __shared__ uint32_t s_wave[NWV];
    __shared__ uint32_t s_carry;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if (t == 0) s_carry = 0;
    __syncthreads();
    for (int64_t r0 = 0; r0 < m; r0 += (int64_t)PER * NT) {
        const int64_t i0 = r0 + (int64_t)t * PER;
        uint32_t c[PER];
        if (i0 + PER <= m) {
#pragma unroll
            for (int q = 0; q < PER / 4; q++) {
                const u32x4 v = *(const u32x4 *)(counts + i0 + 4 * q);
                c[4 * q] = v.x; c[4 * q + 1] = v.y; c[4 * q + 2] = v.z; c[4 * q + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < PER; q++) c[q] = i0 + q < m ? counts[i0 + q] : 0u;
        }
        uint32_t sum = 0;
#pragma unroll
        for (int q = 0; q < PER; q++) sum += c[q];
        // inclusive scan of the thread sums inside the wave
        uint32_t inc = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t x = __shfl_up(inc, o, 64);
            if (lane >= o) inc += x;
        }
        if (lane == 63) s_wave[wave] = inc;
        __syncthreads();
        uint32_t before = s_carry;
        for (int w = 0; w < wave; w++) before += s_wave[w];
        uint32_t run = before + inc - sum;   // exclusive prefix of this thread's first count
        uint32_t o16[PER];
#pragma unroll
        for (int q = 0; q < PER; q++) { o16[q] = run; run += c[q]; }
        if (i0 + PER <= m) {
#pragma unroll
            for (int q = 0; q < PER / 4; q++) {
                u32x4 v;
                v.x = o16[4 * q]; v.y = o16[4 * q + 1]; v.z = o16[4 * q + 2]; v.w = o16[4 * q + 3];
                *(u32x4 *)(offsets + i0 + 4 * q) = v;
            }
        } else {
#pragma unroll
            for (int q = 0; q < PER; q++)
                if (i0 + q < m) offsets[i0 + q] = o16[q];
        }
        __syncthreads();   // every thread has read s_wave and s_carry
        if (t == NT - 1) s_carry = run;
        __syncthreads();
    }
    if (t == 0) {
        offsets[m] = s_carry;
        ws->result = s_carry;
        if (total) *total = s_carry;
    }
}

// ------------------------------------------------------------------ write

// Stages up to 256 values of the current chunk in the wave's LDS buffer at
// their compacted slots, then writes the first `avail` of them to dst with
// consecutive lanes on consecutive words (coalesced).
template <typename V>
__device__ __forceinline__ void stage_and_flush(uint32_t *buf, uint32_t nib, const uint32_t (&slot)[4], V &&val,
                                                uint32_t *dst, uint32_t avail)
{
#pragma unroll
    for (int e = 0; e < 4; e++)
        if ((nib >> e) & 1u) buf[slot[e]] = val(e);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t i = lane_id(); i < avail; i += kWave) dst[i] = buf[i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Writes the qualifying rows of one wave tile (lane masks `bits`, rows from
// `base`) at output positions p onwards, in row order, at most up to `cap`.
// Chunk j of the tile (256 rows) is compacted in LDS (rank of a row = lanes
// below, from ballot masks, then e) and each output column is written as one
// contiguous run.  proj(q, j, e, r0) gives projected column q's value at row
// r0 + e of chunk j.
template <int RPT, typename Proj>
__device__ __forceinline__ void write_tile(uint32_t bits, int64_t base, unsigned long long p, const ProjArgs &pa,
                                           int32_t *rowids, unsigned long long cap, uint32_t *buf, Proj &&proj)
{
    constexpr int NJ = RPT / 4;
    const int lane = lane_id();
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const uint32_t nib = (bits >> (4 * j)) & 0xfu;
        uint32_t pre = 0, tot = 0;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            // set bits of the ballot in the lanes below this one (mbcnt: no
            // 64-bit shift by a per-lane amount)
            const uint64_t b = __ballot((nib >> e) & 1u);
            pre = __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, pre));
            tot += (uint32_t)__popcll(b);
        }
        if (tot == 0) continue;
        if (p >= cap) break;
        const uint32_t avail = (uint32_t)(p + tot <= cap ? tot : cap - p);
        uint32_t slot[4];
        uint32_t k = pre;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            slot[e] = k;
            k += (nib >> e) & 1u;
        }
        const int64_t r0 = base + (int64_t)j * (4 * kWave) + lane * 4;   // row of e = 0
        if (rowids)
            stage_and_flush(buf, nib, slot, [&](int e) { return (uint32_t)(r0 + e); }, (uint32_t *)rowids + p, avail);
        for (int q = 0; q < pa.nproj; q++) proj(q, j, r0, nib, slot, pa.dst[q] + p, avail);
        p += tot;
    }
}

// write_tile for a dense tile (every row exists, at least dense_min
// qualifying): the ranks of all NJ chunks are taken first, then for each
// projected column the loads of all NJ chunks are issued before any is
// staged, so that a wave keeps NJ 16-byte loads per lane in flight instead
// of one.  Output, order and cap handling are those of write_tile.
template <int RPT>
__device__ __forceinline__ void write_dense_tile(uint32_t bits, int64_t base, unsigned long long p0,
                                                 const ProjArgs &pa, int32_t *rowids, unsigned long long cap,
                                                 uint32_t *buf)
{
    constexpr int NJ = RPT / 4;
    const int lane = lane_id();
    uint32_t pre[NJ], tot[NJ];
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const uint32_t nib = (bits >> (4 * j)) & 0xfu;
        uint32_t pr = 0, t = 0;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const uint64_t b = __ballot((nib >> e) & 1u);
            pr = __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, pr));
            t += (uint32_t)__popcll(b);
        }
        pre[j] = pr;
        tot[j] = (uint32_t)__builtin_amdgcn_readfirstlane((int)t);
    }
    // stages chunk j's values (val(e) for e = 0..3 of this lane) at output p
    auto put = [&](int j, unsigned long long p, uint32_t *dst_base, auto &&val) {
        const uint32_t nib = (bits >> (4 * j)) & 0xfu;
        const uint32_t avail = (uint32_t)(p + tot[j] <= cap ? tot[j] : cap - p);
        uint32_t slot[4];
        uint32_t k = pre[j];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            slot[e] = k;
            k += (nib >> e) & 1u;
        }
        stage_and_flush(buf, nib, slot, val, dst_base + p, avail);
    };
    if (rowids) {
        unsigned long long p = p0;
#pragma unroll
        for (int j = 0; j < NJ; j++) {
            if (tot[j] == 0) continue;
            if (p >= cap) break;
            const int64_t r0 = base + (int64_t)j * (4 * kWave) + lane * 4;
            put(j, p, (uint32_t *)rowids, [&](int e) { return (uint32_t)(r0 + e); });
            p += tot[j];
        }
    }
    for (int q = 0; q < pa.nproj; q++) {
        const uint32_t *src = pa.src[q] + base + lane * 4;
        u32x4 x[NJ];
#pragma unroll
        for (int j = 0; j < NJ; j++) {
            // a lane loads its four rows only if one of them qualifies: the
            // memory system then fetches only the sectors that hold
            // qualifying rows, and a skipped lane's values are never staged
            x[j] = u32x4{0u, 0u, 0u, 0u};
            if ((bits >> (4 * j)) & 0xfu) x[j] = __builtin_nontemporal_load((const u32x4 *)(src + j * (4 * kWave)));
        }
        unsigned long long p = p0;
#pragma unroll
        for (int j = 0; j < NJ; j++) {
            if (tot[j] == 0) continue;
            if (p >= cap) break;
            put(j, p, pa.dst[q], [&](int e) { return x[j][e]; });
            p += tot[j];
        }
    }
}

// Writes the qualifying rows of every wave tile at offsets[t] onwards, in row
// order, from the lane masks of the count pass.  A projected column is read
// with the tile's coalesced 16-byte loads when the tile has at least
// dense_min qualifying rows, else gathered row by row.
template <int RPT>
__global__ __launch_bounds__(kScanBlock) void write_kernel(const uint32_t *tile_bits, const uint32_t *offsets,
                                                           int64_t n, const ProjArgs pa, int32_t *rowids,
                                                           unsigned long long cap, uint32_t dense_min)
{
    constexpr int TILE = kWave * RPT;
    constexpr int NW = kScanBlock / kWave;
    __shared__ uint32_t s_buf[NW][4 * kWave];
    uint32_t *buf = s_buf[wave_id()];
    const int64_t ntiles = (n + TILE - 1) / TILE;
    const int64_t step = (int64_t)gridDim.x * NW;
    for (int64_t t = (int64_t)blockIdx.x * NW + wave_id(); t < ntiles; t += step) {
        const uint32_t o0 = offsets[t], o1 = offsets[t + 1];
        if (o0 == o1 || o0 >= cap) continue;   // wave-uniform
        const int64_t base = t * TILE;
        const bool dense = base + TILE <= n && o1 - o0 >= dense_min;
        const uint32_t bits = tile_bits[t * kWave + lane_id()];
        if (dense) {
            write_dense_tile<RPT>(bits, base, o0, pa, rowids, cap, buf);
            continue;
        }
        write_tile<RPT>(bits, base, o0, pa, rowids, cap, buf,
                        [&](int q, int, int64_t r0, uint32_t nib, const uint32_t(&slot)[4], uint32_t *dst,
                            uint32_t avail) {
                            const uint32_t *src = pa.src[q];
                            if (dense) {
                                const u32x4 x = __builtin_nontemporal_load((const u32x4 *)(src + r0));
                                stage_and_flush(buf, nib, slot, [&](int e) { return x[e]; }, dst, avail);
                            } else {
                                stage_and_flush(buf, nib, slot, [&](int e) { return src[r0 + e]; }, dst, avail);
                            }
                        });
    }
}

// ------------------------------------------------------------------ single-pass compaction

// Status word of a wave tile in the single-pass compaction: flag in the top
// two bits (0 not yet published, 1 the tile's own count, 2 the inclusive
// prefix of all tiles up to it), the value in the low 62 bits.
constexpr unsigned long long kStAggregate = 1ull << 62, kStInclusive = 2ull << 62;
constexpr unsigned long long kStValue = (1ull << 62) - 1ull;

// Count and materialization in one pass (a materialization with no count
// before it): waves take wave tiles in increasing order from a counter,
// evaluate the predicate, publish the tile's count, and find the rows
// before the tile by looking back over the predecessors' status words (a
// predecessor that has published its inclusive prefix ends the walk; one
// that has published only its count adds it and the walk continues).  Every
// predecessor was taken by a running wave before this tile, so every wait
// ends.  The qualifying rows are then written at that offset exactly as the
// write pass does, taking the projected values of predicate columns from
// registers.  status (ntiles words) and ctr must be zero at launch.
template <int K, int RPT, bool UDF>
__global__ __launch_bounds__(kScanBlock) void compact_kernel(const Program P, const ColPtrs cp, int64_t n,
                                                             unsigned long long *status, unsigned int *ctr,
                                                             const ProjArgs pa, const ProjSlots ps, int32_t *rowids,
                                                             unsigned long long cap, uint32_t dense_min,
                                                             unsigned long long *total)
{
    constexpr int TILE = kWave * RPT;
    constexpr int KK = K > 0 ? K : 1;
    constexpr int NW = kScanBlock / kWave;
    __shared__ uint32_t s_buf[NW][4 * kWave];
    uint32_t *buf = s_buf[wave_id()];
    const int64_t ntiles = (n + TILE - 1) / TILE;
    const SlotTabs<kMaxTables> tabs = load_tables<kMaxTables>(P);
    for (;;) {
        uint32_t got = 0;
        if (lane_id() == 0) got = atomicAdd(ctr, 1u);
        const int64_t t = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)got);
        if (t >= ntiles) break;
        const int64_t base = t * TILE;
        uint32_t v[KK][RPT];
        load_vals<K, RPT>(cp, base, n, v);
        const uint32_t bits = run_program<K, RPT, UDF, kMaxTables>(P, v, valid_bits<RPT>(base, n), tabs);
        const unsigned long long c = wave_sum((uint32_t)__popc(bits));
        unsigned long long before = 0;
        if (t > 0) {
            __hip_atomic_store(&status[t], kStAggregate | c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int64_t j = t - 1;;) {
                // every lane reads the same word; its first lane's copy
                // makes the walk wave-uniform
                const unsigned long long w =
                    __hip_atomic_load(&status[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t wlo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)w);
                const uint32_t whi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(w >> 32));
                const unsigned long long wu = ((unsigned long long)whi << 32) | wlo;
                if ((wu >> 62) == 0ull) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                before += wu & kStValue;
                if ((wu >> 62) == 2ull) break;
                j--;
            }
        }
        __hip_atomic_store(&status[t], kStInclusive | (before + c), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (t == ntiles - 1 && lane_id() == 0) *total = before + c;
        if (c == 0 || before >= cap) continue;
        const bool dense = base + TILE <= n && c >= dense_min;
        write_tile<RPT>(bits, base, before, pa, rowids, cap, buf,
                        [&](int q, int j, int64_t r0, uint32_t nib, const uint32_t(&slot)[4], uint32_t *dst,
                            uint32_t avail) {
                            const int s = ps.slot[q];
                            bool done = false;
                            for_slot<K>(s, [&](auto C) {
                                stage_and_flush(buf, nib, slot, [&](int e) { return v[C][4 * j + e]; }, dst, avail);
                                done = true;
                            });
                            if (done) return;
                            const uint32_t *src = pa.src[q];
                            if (dense) {
                                const u32x4 x = __builtin_nontemporal_load((const u32x4 *)(src + r0));
                                stage_and_flush(buf, nib, slot, [&](int e) { return x[e]; }, dst, avail);
                            } else {
                                stage_and_flush(buf, nib, slot, [&](int e) { return src[r0 + e]; }, dst, avail);
                            }
                        });
    }
}

__global__ void zero_kernel(unsigned long long *p, int64_t nwords)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nwords; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// ------------------------------------------------------------------ dispatch tables

template <bool UDF, int... Ks>
constexpr CompactFn compact_table_impl(int k, std::integer_sequence<int, Ks...>)
{
    CompactFn t[] = {compact_kernel<Ks, kCompactRPT, UDF>...};
    return t[k];
}

CompactFn compact_fn(int nslots, bool udf)
{
    using S = std::make_integer_sequence<int, kMaxSlots + 1>;
    return udf ? compact_table_impl<true>(nslots, S{}) : compact_table_impl<false>(nslots, S{});
}

WriteFn write_fn(int rpt)
{
    return rpt == 8 ? write_kernel<8> : rpt == 16 ? write_kernel<16> : write_kernel<32>;
}

void launch_zero(unsigned long long *p, int64_t nwords, hipStream_t s)
{
    if (nwords <= 0) return;
    int64_t blocks = (nwords + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, nwords);
}

void launch_scan(const uint32_t *counts, int64_t m, uint32_t *offsets, WsHeader *ws, unsigned long long *total,
                 hipStream_t s)
{
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, counts, m, offsets, ws, total);
}

}  // namespace esc
