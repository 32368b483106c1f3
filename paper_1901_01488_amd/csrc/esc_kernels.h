// esc_kernels.h -- launch-side declarations shared by the HIP sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "esc.h"
#include "esc_program.h"

namespace esc {

constexpr int kScanBlock = 256;
constexpr int kMaxConj = ESC_MAX_CONJ;

// device pointers of the loaded column slots
struct ColPtrs {
    const uint32_t *p[kMaxSlots];
    int32_t nt;   // 1: streaming (non-temporal) loads
};

// projected columns of a materialization (source column, output array)
struct ProjArgs {
    int32_t nproj;
    const uint32_t *src[ESC_MAX_PROJ];
    uint32_t *dst[ESC_MAX_PROJ];
};

// for each projected column, the predicate slot that holds it, or -1
struct ProjSlots {
    int32_t slot[ESC_MAX_PROJ];
};

// Per-wave-tile results of a count pass, kept for a materialization:
// counts[t] = qualifying rows of wave tile t; bits[64 t + l] = lane l's
// truth mask of tile t (bit r = row slot r).
// A count that stores tiles writes `stamp` into the workspace header.  With
// `expect` != 0 the launch first compares the header's stamp with it: when
// they are equal the tiles of this table and predicate are already in the
// workspace and every block returns at once.
// wave tiles whose records a tile-storing count holds in LDS before storing
// them, and the dynamic LDS its launch gives a block for that
constexpr int kTileBuf = 32;
constexpr int kTileBufBytes = (kScanBlock / 64) * kTileBuf * 64 * 4;
static_assert(kTileBuf <= 64, "one tile count per lane");

struct TileOut {
    uint32_t *counts;
    uint32_t *bits;
    unsigned long long stamp;
    unsigned long long expect;
};

// The count's running word: rows in bits 0..kTotalBits-1, blocks done above
// (a table has fewer than 2^31 rows, a grid fewer than 2^24 blocks).
constexpr int kTotalBits = 40;

// first 64 bytes of a scan workspace; per-wave-tile counts and output offsets follow
struct WsHeader {
    unsigned long long total;    // count: blocks done << kTotalBits | rows so far (reset by the last block)
    unsigned long long stamp;    // which count stored the tiles that follow (0: none)
    unsigned long long result;   // the count of the last call
    unsigned long long pad1[5];
};
static_assert(sizeof(WsHeader) == 64, "workspace header is 64 bytes");

typedef void (*CountFn)(const Program, const ColPtrs, int64_t, WsHeader *, unsigned long long *, const TileOut);
typedef void (*WriteFn)(const uint32_t *, const uint32_t *, int64_t, const ProjArgs, int32_t *, unsigned long long,
                        uint32_t);

CountFn count_fn(int nslots, int ninsn, int variant, bool udf, bool tiles);
constexpr int kCompactRPT = 16;   // rows per lane of the single-pass compaction
typedef void (*CompactFn)(const Program, const ColPtrs, int64_t, unsigned long long *, unsigned int *,
                          const ProjArgs, const ProjSlots, int32_t *, unsigned long long, uint32_t,
                          unsigned long long *);
CompactFn compact_fn(int nslots, bool udf);
int count_rpt(int variant, int nslots, int ninsn, bool tiles);
int count_bpc(int variant, int nslots, int bpc, bool tiles);
WriteFn write_fn(int rpt);
typedef void (*ConjFn)(const Program *, int, const ColPtrs, int64_t, unsigned long long *);
ConjFn conj_fn(int nslots, bool udf);
void launch_zero(unsigned long long *p, int64_t nwords, hipStream_t s);
// offsets of m tile counts in row order; the total goes to ws->result and,
// when total is not null, to *total
void launch_scan(const uint32_t *counts, int64_t m, uint32_t *offsets, WsHeader *ws, unsigned long long *total,
                 hipStream_t s);

}  // namespace esc
