// esc_runtime.h -- the context object and helpers shared by the HIP host code.
#pragma once
#include <hip/hip_runtime.h>

#include "esc_host.h"
#include "esc_kernels.h"

struct esc_ctx {
    int device = 0;
    int num_cus = 0;
    unsigned long long *pinned = nullptr;   // 4 KiB of pinned host memory for read-backs
    unsigned long long *pinned_dev = nullptr;   // the same memory as the device addresses it
    int count_variant = 4;                  // count kernel shape (see count_rpt / count_bpc)
    int nt = 1;                             // streaming loads in the scans
    int bpc = 1;                            // count-kernel blocks per CU (0: occupancy)
    int mat_bpc = 0;                        // materialize blocks per CU (0: occupancy)
    int dense_shift = 7;                    // projections of a tile read whole when >= tile rows >> shift qualify
    int cold_compact = 0;                   // a materialization without a count first: single pass (1) or count, scan, write (0)
    void *scratch = nullptr;                // this device's static scratch (esc_materialize_noalloc)
    hipEvent_t slot_event[ESC_COUNT_SLOTS] = {};   // esc_count_begin / esc_count_end
    bool slot_pending[ESC_COUNT_SLOTS] = {};
};

// words of the pinned block: [0, kSlotWord) read-backs of the blocking calls,
// then one word per esc_count_begin slot
constexpr int kSlotWord = 256;
static_assert(kSlotWord + ESC_COUNT_SLOTS <= 512, "the slots fit the 4 KiB pinned block");

namespace esc {

int hip_fail(hipError_t e, const char *what);
// Makes `device` current; on failure clears HIP's sticky error and reports it.
int set_device(int device);
int occupancy(const void *fn, int block, int dyn_lds);
ColPtrs slot_ptrs(const esc_table *t, const Program &P, int nt);

}  // namespace esc
