// esc_count.hip -- gfx950 kernels of the COUNT(*) selectivity sub-query
// (Section 2) and of the per-conjunct counts of split selectivity.
//
// Data layout: every column is a contiguous array of nrows 4-byte values
// (int32, date32 or float32), 16-byte aligned.  The unit of work is a wave
// tile of 64*RPT consecutive rows (esc_device.h): its columns are read with
// coalesced 16-byte loads, the predicate program runs on registers with
// wave-uniform control, and the qualifying rows come out as per-lane bit
// masks.  Waves are independent; nothing per row is stored by a plain
// count.  A count that precedes a materialization also stores, per wave
// tile, its qualifying-row count and every lane's truth mask (1/32 of the
// bytes of one 4-byte column), which the write pass (esc_materialize.hip)
// reads instead of the predicate's columns.
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

// A wave's tile records wait in LDS (masks) and in a register (counts, one
// tile per lane) and go out kTileBuf tiles at a time: a global store inside
// the tile loop would make the next tile's loads wait for its
// acknowledgement (stores and loads share one counter of outstanding
// memory operations), and with one wave per SIMD nothing hides that wait.
__device__ __forceinline__ void flush_tiles(const TileOut &to, const uint32_t *buf, uint32_t tcnt, int64_t t0,
                                            int64_t step, int nbuf)
{
    for (int j = 0; j < nbuf; j++) to.bits[(t0 + j * step) * kWave + lane_id()] = buf[j * kWave + lane_id()];
    if (lane_id() < nbuf) to.counts[t0 + lane_id() * step] = tcnt;
}

// Grid-stride over wave tiles.  With TILES, every wave tile's count and lane
// masks are stored in to.counts and to.bits (the launch then gives the block
// kTileBufBytes of dynamic LDS); a plain count carries none of that code.
// UDF = false for programs without udf instructions.
template <int K, int RPT, bool UDF, bool TILES>
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
    if (TILES && to.expect != 0ull && ws->stamp == to.expect) return;
    const SlotTabs<kMaxTables> tabs = load_tables<kMaxTables>(P);
    extern __shared__ uint32_t s_tbuf[];   // [NW][kTileBuf][kWave] lane masks
    const int wave = wave_id();
    uint32_t *buf = s_tbuf + wave * (kTileBuf * kWave);
    uint32_t tcnt = 0;   // lane j: count of the j-th buffered tile
    int nbuf = 0;
    int64_t t0 = first;  // the first buffered tile; the others follow at step
    uint32_t cnt = 0;    // per lane
    for (int64_t t = first; t < ntiles; t += step) {
        uint32_t v[KK][RPT];
        load_vals<K, RPT>(cp, t * TILE, n, v);
        const uint32_t bits = run_program<K, RPT, UDF, kMaxTables>(P, v, valid_bits<RPT>(t * TILE, n), tabs);
        const uint32_t c = (uint32_t)__popc(bits);
        if constexpr (TILES) {
            const uint32_t w = wave_sum(c);
            tcnt = lane_id() == nbuf ? w : tcnt;
            buf[nbuf * kWave + lane_id()] = bits;   // each lane reads back only its own words
            if (++nbuf == kTileBuf) {
                flush_tiles(to, buf, tcnt, t0, step, nbuf);
                nbuf = 0;
                t0 = t + step;
            }
        }
        cnt += c;
    }
    if (TILES && nbuf) flush_tiles(to, buf, tcnt, t0, step, nbuf);
    cnt = wave_sum(cnt);
    __shared__ uint32_t s_cnt[NW];
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
            if (TILES) ws->stamp = to.stamp;
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

// ------------------------------------------------------------------ dispatch tables

template <int RPT, bool UDF, bool TILES, int... Ks>
constexpr CountFn count_table_impl(int k, std::integer_sequence<int, Ks...>)
{
    CountFn t[] = {count_kernel<Ks, RPT, UDF, TILES>...};
    return t[k];
}

// Rows per lane of a count (ESC_COUNT_VARIANT selects a variant, for
// comparisons).  variant 0: 16; variant 1: 32 for programs of up to four
// column slots, 16 above; variant 2: 8 for plain counts (variant 1 for
// counts that store tiles); variant 3: variant 1 when the count stores its
// tiles for a materialization, else 32 for one or two columns and 16 for
// more, with twice the blocks for one column; variant 4 (the default):
// plain counts as variant 3 except that programs longer than one test per
// column keep 32, and counts that store tiles run 32 up to six columns.
// Measured on the 60M-row star table: plain counts 6.05 TB/s back to back
// with variant 3 against 5.9 for variant 1 (one-column counts 5.2 against
// 4.8); counts that store tiles with 16 rows per lane store twice the mask
// bytes and give the offset scan twice the tiles (154 against 145 us per
// count).
int count_rpt(int variant, int k, int ninsn, bool tiles)
{
    if (variant == 2 && !tiles) return 8;
    if (variant == 3 && !tiles) return k <= 2 ? 32 : 16;
    // plain counts of three or more columns: 16 rows per lane when the
    // program is one test per column; longer programs are interpreted once
    // per wave tile and keep 32 rows per lane to spread that over more rows
    if (variant == 4 && !tiles) return k <= 2 || ninsn > k ? 32 : 16;
    // counts that store tiles (variant 4): 32 rows per lane up to six
    // columns (at one wave per SIMD their values fit in registers: 280 and
    // 316 VGPRs for five and six), so the offset scan and the write pass
    // handle half the tiles
    return variant == 0 || k > (tiles && variant == 4 ? 6 : 4) ? 16 : 32;
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
    // counts that store tiles run 16 or 32 rows per lane (count_rpt)
    if (tiles) {
        if (count_rpt(variant, k, ninsn, true) == 16)
            return udf ? count_table_impl<16, true, true>(k, S{}) : count_table_impl<16, false, true>(k, S{});
        return udf ? count_table_impl<32, true, true>(k, S{}) : count_table_impl<32, false, true>(k, S{});
    }
    switch (count_rpt(variant, k, ninsn, false)) {
    case 8: return udf ? count_table_impl<8, true, false>(k, S{}) : count_table_impl<8, false, false>(k, S{});
    case 16: return udf ? count_table_impl<16, true, false>(k, S{}) : count_table_impl<16, false, false>(k, S{});
    default: return udf ? count_table_impl<32, true, false>(k, S{}) : count_table_impl<32, false, false>(k, S{});
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

}  // namespace esc
