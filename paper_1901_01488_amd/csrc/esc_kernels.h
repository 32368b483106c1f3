// esc_kernels.h -- launch-side declarations shared by the HIP sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "esc.h"
#include "esc_program.h"

namespace esc {

constexpr int kScanBlock = 256;

// device pointers of the loaded column slots
struct ColPtrs {
    const uint32_t *p[kMaxSlots];
};

// projected columns of a materialization: slot >= 0 when the column is
// already in registers, else it is gathered from src
struct ProjArgs {
    int32_t nproj;
    int32_t slot[ESC_MAX_PROJ];
    const uint32_t *src[ESC_MAX_PROJ];
    uint32_t *dst[ESC_MAX_PROJ];
};

// first 64 bytes of a scan workspace; tile status words follow
struct WsHeader {
    unsigned long long total;    // count: running sum (reset by the last block)
    unsigned int ticket;         // count: blocks done (reset by the last block)
    unsigned int error;          // materialize: a bounded wait expired
    unsigned long long result;   // the count of the last call
    unsigned int tile_ctr;       // materialize: next tile to claim
    unsigned int pad0;
    unsigned long long pad1[4];
};
static_assert(sizeof(WsHeader) == 64, "workspace header is 64 bytes");

typedef void (*CountFn)(const Program, const ColPtrs, int64_t, WsHeader *, unsigned long long *);
typedef void (*MatFn)(const Program, const ColPtrs, int64_t, int, const ProjArgs, int32_t *, unsigned long long,
                      WsHeader *, unsigned long long *);

CountFn count_fn(int nslots, int rpt);
MatFn mat_fn(int nslots, int rpt);
void launch_zero(unsigned long long *p, int64_t nwords, hipStream_t s);

}  // namespace esc
