// esc_scan.hip -- gfx950 kernels of the plain ESC scan: the COUNT(*)
// selectivity sub-query (Section 2) and its materialization as a temporary
// table in row order (Section 2, Section 2.1).
//
// Data layout: every column is a contiguous array of nrows 4-byte values
// (int32, date32 or float32), 16-byte aligned.  The unit of work is a wave
// tile of 64*RPT consecutive rows (esc_device.h): its columns are read with
// coalesced 16-byte loads, the predicate program runs on registers with
// wave-uniform control, and the qualifying rows come out as per-lane bit
// masks.  Waves are independent; nothing per row is stored by a count.
//
// Materialization is order-preserving stream compaction in two passes and
// no inter-block waiting:
//   1. the count pass (the selectivity sub-query itself) also stores, per
//      wave tile, its qualifying-row count and every lane's truth mask
//      (1/32 of the bytes of one 4-byte column);
//   2. one block scans the tile counts into row-order output offsets;
//   3. the write pass reads the masks instead of the predicate's columns,
//      ranks the qualifying rows of each 256-row chunk with ballot masks,
//      compacts row ids and projected values in LDS and writes them as
//      contiguous runs at offset + rank.
// When the count pass was the caller's own preceding esc_count on the same
// workspace, table and predicate (count, decide, then materialize),
// materialization never reads the predicate's columns again.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <type_traits>
#include <utility>

#include "esc_device.h"
#include "esc_host.h"
#include "esc_kernels.h"

namespace esc {

// ------------------------------------------------------------------ count

// Grid-stride over wave tiles.  When to.counts is not null, every wave tile's
// count and lane masks are stored there.  UDF = false for programs without
// udf instructions.
template <int K, int RPT, bool UDF>
__global__ __launch_bounds__(kScanBlock) void count_kernel(const Program P, const ColPtrs cp, int64_t n,
                                                           WsHeader *ws, unsigned long long *out, const TileOut to)
{
    constexpr int TILE = kWave * RPT;
    constexpr int KK = K > 0 ? K : 1;
    constexpr int NW = kScanBlock / kWave;
    const int64_t ntiles = (n + TILE - 1) / TILE;
    const int64_t step = (int64_t)gridDim.x * NW;
    const int64_t first = (int64_t)blockIdx.x * NW + wave_id();
    // the workspace already holds this count's tiles: nothing to do (the
    // stamp is read from a previous launch's write, the same for every block)
    if (to.expect != 0ull && ws->stamp == to.expect) return;
    const SlotTabs<kMaxTables> tabs = load_tables<kMaxTables>(P);
    uint32_t cnt = 0;   // per lane
    for (int64_t t = first; t < ntiles; t += step) {
        uint32_t v[KK][RPT];
        load_vals<K, RPT>(cp, t * TILE, n, v);
        const uint32_t bits = run_program<K, RPT, UDF, kMaxTables>(P, v, valid_bits<RPT>(t * TILE, n), tabs);
        const uint32_t c = (uint32_t)__popc(bits);
        if (to.counts) {
            const uint32_t w = wave_sum(c);
            if (lane_id() == 0) to.counts[t] = w;
            to.bits[t * kWave + lane_id()] = bits;
        }
        cnt += c;
    }
    cnt = wave_sum(cnt);
    __shared__ uint32_t s_cnt[NW];
    const int wave = wave_id();
    if (lane_id() == 0) s_cnt[wave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = 0;
        for (int w = 0; w < NW; w++) b += s_cnt[w];
        // One 64-bit word carries both the running row count (low
        // kTotalBits bits) and the number of blocks done (high bits), so
        // each block's contribution is one atomic read-modify-write of one
        // location.  All such RMWs are totally ordered and each reads the
        // value left by the previous ones, so the block whose RMW returns
        // gridDim.x - 1 blocks done has read the sum of every other block:
        // exact without fences and without any order between two
        // addresses.  That block publishes the total and resets the word,
        // so the next launch on the workspace starts from zero.
        const unsigned long long old = atomicAdd(&ws->total, (1ull << kTotalBits) | b);
        if ((old >> kTotalBits) == gridDim.x - 1u) {
            *out = (old & ((1ull << kTotalBits) - 1ull)) + b;
            atomicExch(&ws->total, 0ull);
            if (to.counts) ws->stamp = to.stamp;
        }
    }
}

// ------------------------------------------------------------------ conjuncts

// Split selectivities: every conjunct program runs on each loaded wave tile;
// a running AND of their masks gives the prefix conjunctions.  Per-wave sums
// go to LDS, then one u64 atomic per counter per block.  out[i] = rows of
// conjunct i, out[kMaxConj + i] = rows of conjuncts 0..i.
template <int K, int RPT, bool UDF>
__global__ __launch_bounds__(kScanBlock) void conj_kernel(const Program *__restrict__ progs, int nconj,
                                                          const ColPtrs cp, int64_t n, unsigned long long *out)
{
    constexpr int TILE = kWave * RPT;
    constexpr int KK = K > 0 ? K : 1;
    constexpr int NW = kScanBlock / kWave;
    __shared__ uint32_t s_acc[NW][2 * kMaxConj];
    const int wave = wave_id();
    for (int i = threadIdx.x; i < NW * 2 * kMaxConj; i += kScanBlock) (&s_acc[0][0])[i] = 0;
    __syncthreads();
    const int64_t ntiles = (n + TILE - 1) / TILE;
    const int64_t step = (int64_t)gridDim.x * NW;
    for (int64_t t = (int64_t)blockIdx.x * NW + wave; t < ntiles; t += step) {
        uint32_t v[KK][RPT];
        load_vals<K, RPT>(cp, t * TILE, n, v);
        const uint32_t valid = valid_bits<RPT>(t * TILE, n);
        uint32_t prefix = valid;
        for (int i = 0; i < nconj; i++) {
            const uint32_t m = run_program<K, RPT, UDF>(progs[i], v, valid);
            prefix &= m;
            const uint32_t c1 = wave_sum((uint32_t)__popc(m));
            const uint32_t c2 = wave_sum((uint32_t)__popc(prefix));
            if (lane_id() == 0) {
                s_acc[wave][i] += c1;
                s_acc[wave][kMaxConj + i] += c2;
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * kMaxConj; i += kScanBlock) {
        if ((i % kMaxConj) >= nconj) continue;
        unsigned long long c = 0;
#pragma unroll
        for (int w = 0; w < NW; w++) c += s_acc[w][i];
        if (c) atomicAdd(&out[i], c);
    }
}

// ------------------------------------------------------------------ scan

// Exclusive scan of m per-tile counts into offsets[0..m]; offsets[m] is the
// total, also stored in ws->result.  One block of 1024 threads walks the
// counts in rounds of 16384: each thread takes 16 consecutive counts (four
// 16-byte loads, coalesced across the block), the thread totals are scanned
// with wave shuffles and a 16-entry LDS pass, and a carry links the rounds.
__global__ __launch_bounds__(1024) void scan_kernel(const uint32_t *counts, int64_t m, uint32_t *offsets,
                                                    WsHeader *ws)
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
        for (int j = 0; j < NJ; j++) x[j] = __builtin_nontemporal_load((const u32x4 *)(src + j * (4 * kWave)));
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

template <int RPT, bool UDF, int... Ks>
constexpr CountFn count_table_impl(int k, std::integer_sequence<int, Ks...>)
{
    CountFn t[] = {count_kernel<Ks, RPT, UDF>...};
    return t[k];
}

// variant 0: 16 rows per lane; variant 1: 32 rows per lane for programs of
// up to four column slots, 16 above (32 rows of five or more columns no
// longer fit the register file); variant 2: 8 rows per lane; variant 3 (the
// default): variant 1 when the count stores its tiles for a
// materialization, else 32 rows per lane for one or two columns, 16 for
// more, and twice the blocks for one column.  Measured on the 60M-row star
// table: plain counts 6.05 TB/s back to back against 5.9 for variant 1
// (one-column counts 5.2 against 4.8), while counts that store tiles keep
// variant 1 (with 16 rows per lane they store twice the mask bytes and the
// offset scan has twice the tiles: 154 against 145 us per count).
int count_rpt(int variant, int k, int ninsn, bool tiles)
{
    if (variant == 2) return 8;
    if (variant == 3 && !tiles) return k <= 2 ? 32 : 16;
    // plain counts of three or more columns: 16 rows per lane when the
    // program is one test per column; longer programs are interpreted once
    // per wave tile and keep 32 rows per lane to spread that over more rows
    if (variant == 4 && !tiles) return k <= 2 || ninsn > k ? 32 : 16;
    return variant == 0 || k > 4 ? 16 : 32;
}

// blocks of four waves per CU; one-column counts run two to keep enough
// loads in flight (variant 3: plain counts only; variant 4: also counts
// that store tiles)
int count_bpc(int variant, int k, int bpc, bool tiles)
{
    if (k > 1 || variant < 3 || (tiles && variant == 3)) return bpc;
    return 2 * bpc;
}

CountFn count_fn(int k, int ninsn, int variant, bool udf, bool tiles)
{
    using S = std::make_integer_sequence<int, kMaxSlots + 1>;
    switch (count_rpt(variant, k, ninsn, tiles)) {
    case 8: return udf ? count_table_impl<8, true>(k, S{}) : count_table_impl<8, false>(k, S{});
    case 16: return udf ? count_table_impl<16, true>(k, S{}) : count_table_impl<16, false>(k, S{});
    default: return udf ? count_table_impl<32, true>(k, S{}) : count_table_impl<32, false>(k, S{});
    }
}

template <bool UDF, int... Ks>
constexpr ConjFn conj_table_impl(int k, std::integer_sequence<int, Ks...>)
{
    ConjFn t[] = {conj_kernel<Ks, 16, UDF>...};
    return t[k];
}

ConjFn conj_fn(int nslots, bool udf)
{
    using S = std::make_integer_sequence<int, kMaxSlots + 1>;
    return udf ? conj_table_impl<true>(nslots, S{}) : conj_table_impl<false>(nslots, S{});
}

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

void launch_scan(const uint32_t *counts, int64_t m, uint32_t *offsets, WsHeader *ws, hipStream_t s)
{
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, counts, m, offsets, ws);
}

}  // namespace esc
