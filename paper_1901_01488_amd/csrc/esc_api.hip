// esc_api.hip -- context, workspace and the host side of esc_count /
// esc_materialize: validation, choice of the kernel variant, launch and the
// 8-byte (or 64-byte) read-back of the result.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <unistd.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "esc_host.h"
#include "esc_kernels.h"
#include "esc_runtime.h"

using esc::fail;

namespace esc {

int hip_fail(hipError_t e, const char *what)
{
    (void)hipGetLastError();   // do not leave the error for the caller's next HIP call
    return fail(ESC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int set_device(int device)
{
    hipError_t e = hipSetDevice(device);
    return e == hipSuccess ? ESC_OK : hip_fail(e, "hipSetDevice");
}

static std::mutex g_occ_mu;
static std::map<const void *, int> g_occ;

int occupancy(const void *fn, int block, int dyn_lds)
{
    std::lock_guard<std::mutex> g(g_occ_mu);
    auto it = g_occ.find(fn);
    if (it != g_occ.end()) return it->second;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, dyn_lds) != hipSuccess || nb <= 0) nb = 1;
    g_occ[fn] = nb;
    return nb;
}

int check_scan_args(const esc_ctx *ctx, const esc_table *t, const esc_pred *p, const void *ws, size_t ws_bytes,
                    size_t need)
{
    if (!ctx || !t || !p) return fail(ESC_ERR_INVALID, "null handle");
    if (!t->has_data()) return fail(ESC_ERR_INVALID, "table is schema-only (no device columns)");
    if (p->schema_dtypes != t->dtypes)
        return fail(ESC_ERR_INVALID, "predicate was compiled for a different schema");
    if (!ws || ((uintptr_t)ws & 255)) return fail(ESC_ERR_ALIGN, "workspace must be non-null and 256-byte aligned");
    if (ws_bytes < need) return fail(ESC_ERR_OOM, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    return ESC_OK;
}

ColPtrs slot_ptrs(const esc_table *t, const Program &P, int nt)
{
    ColPtrs cp{};
    cp.nt = nt;
    for (int s = 0; s < P.nslots; s++) cp.p[s] = (const uint32_t *)t->cols[P.slot_col[s]];
    return cp;
}

__global__ void store_u64_kernel(unsigned long long *dst, unsigned long long v) { *dst = v; }

// Workspace of a materialization: header, per-wave-tile counts (uint32),
// row-order offsets (uint32, one more than there are tiles), then the lane
// masks of every wave tile (64 uint32 per tile).  Each part starts on a
// 256-byte boundary.
struct WsLayout {
    int64_t ntiles;
    size_t counts_off, offsets_off, bits_off, bytes;
};

WsLayout ws_layout(int64_t nrows, int rpt)
{
    WsLayout L;
    const int64_t tile = 64 * (int64_t)rpt;
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    L.ntiles = (nrows + tile - 1) / tile;
    L.counts_off = sizeof(WsHeader);
    L.offsets_off = up(L.counts_off + (size_t)L.ntiles * 4);
    L.bits_off = up(L.offsets_off + (size_t)(L.ntiles + 1) * 4);
    L.bytes = L.bits_off + (size_t)L.ntiles * 64 * 4;
    return L;
}

// Which (table, predicate, tile size) the per-tile counts in a workspace
// belong to; kept per context, keyed by the workspace address.
// The record alone cannot tell whether the memory at that address is still
// the workspace the count wrote (the caller may have freed it and received
// the same address again): the count also writes a process-unique stamp into
// the workspace header, and a materialization that reuses the tiles launches
// the count in checking mode, which recomputes them unless the header still
// holds the recorded stamp.
struct TileRecord {
    uint64_t table_id, pred_id;
    int64_t nrows;
    int rpt;
    unsigned long long stamp;
};

static std::mutex g_rec_mu;
static std::map<std::pair<const esc_ctx *, const void *>, TileRecord> g_records;
static unsigned long long g_next_stamp = 0;

unsigned long long new_stamp()
{
    std::lock_guard<std::mutex> g(g_rec_mu);
    if (g_next_stamp == 0) {
        // distinct across processes sharing a device buffer's history
        const unsigned long long salt = (unsigned long long)(uintptr_t)&g_next_stamp ^ (unsigned long long)getpid();
        g_next_stamp = (salt << 24) | 1ull;
    }
    return g_next_stamp++;
}

void remember_tiles(const esc_ctx *ctx, const void *ws, const esc_table *t, const esc_pred *p, int rpt,
                    unsigned long long stamp)
{
    std::lock_guard<std::mutex> g(g_rec_mu);
    g_records[{ctx, ws}] = TileRecord{t->id, p->id, t->nrows, rpt, stamp};
}

// the stamp of the tiles a workspace should hold for (t, p), 0 if none
unsigned long long tiles_stamp(const esc_ctx *ctx, const void *ws, const esc_table *t, const esc_pred *p, int rpt)
{
    std::lock_guard<std::mutex> g(g_rec_mu);
    auto it = g_records.find({ctx, ws});
    const bool same = it != g_records.end() && it->second.table_id == t->id && it->second.pred_id == p->id &&
                      it->second.nrows == t->nrows && it->second.rpt == rpt;
    return same ? it->second.stamp : 0ull;
}

void forget_tiles(const esc_ctx *ctx, const void *ws)
{
    std::lock_guard<std::mutex> g(g_rec_mu);
    if (ws) g_records.erase({ctx, ws});
    else
        for (auto it = g_records.begin(); it != g_records.end();)
            it = it->first.first == ctx ? g_records.erase(it) : std::next(it);
}

// Device memory for esc_materialize_noalloc: the workspace of a
// materialization (header, per-tile counts, offsets, lane masks) lives in
// this file-scope array, one copy per device, held until the process ends.
// Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address): it uses the address hipGetSymbolAddress
// returns for the current device.
constexpr size_t kStaticScratchBytes = (size_t)ESC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, void *> g_scratch_addr;   // device -> address of its copy of `scratch`

// The address of this device's copy of the scratch array (the device must be
// current); the first lookup on a device also clears the workspace header.
static int scratch_address(int device, void **out)
{
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return ESC_OK;
    }
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    launch_zero((unsigned long long *)ptr, (int64_t)(sizeof(WsHeader) / 8), nullptr);
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "clearing the static scratch");
    g_scratch_addr[device] = ptr;
    *out = ptr;
    return ESC_OK;
}

}  // namespace esc

using namespace esc;

extern "C" {

int esc_ctx_create(int device, esc_ctx **out)
{
    if (!out) return fail(ESC_ERR_INVALID, "null output handle");
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return fail(ESC_ERR_HIP, "no HIP device available");
    if (device < 0 || device >= n) return fail(ESC_ERR_INVALID, "device %d outside [0, %d)", device, n);
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    esc_ctx *c = new (std::nothrow) esc_ctx;
    if (!c) return fail(ESC_ERR_OOM, "out of host memory");
    c->device = device;
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess) { delete c; return hip_fail(e, "hipGetDeviceProperties"); }
    c->num_cus = prop.multiProcessorCount;
    if ((e = hipHostMalloc((void **)&c->pinned, 4096, hipHostMallocDefault)) != hipSuccess) {
        delete c;
        return hip_fail(e, "hipHostMalloc");
    }
    if ((e = hipHostGetDevicePointer((void **)&c->pinned_dev, c->pinned, 0)) != hipSuccess) {
        (void)hipHostFree(c->pinned);
        delete c;
        return hip_fail(e, "hipHostGetDevicePointer");
    }
    const char *r = getenv("ESC_COUNT_VARIANT");
    if (r && atoi(r) >= 0 && atoi(r) <= 4) c->count_variant = atoi(r);
    r = getenv("ESC_NONTEMPORAL");
    if (r) c->nt = atoi(r) != 0;
    r = getenv("ESC_BLOCKS_PER_CU");
    if (r) c->bpc = atoi(r);
    r = getenv("ESC_MAT_BLOCKS_PER_CU");
    if (r) c->mat_bpc = atoi(r);
    r = getenv("ESC_DENSE_SHIFT");
    if (r && atoi(r) >= 0 && atoi(r) <= 12) c->dense_shift = atoi(r);
    r = getenv("ESC_COLD_COMPACT");
    if (r) c->cold_compact = atoi(r) != 0;
    if (int rc = scratch_address(device, &c->scratch)) {
        (void)hipHostFree(c->pinned);
        delete c;
        return rc;
    }
    *out = c;
    return ESC_OK;
}

int esc_ctx_destroy(esc_ctx *ctx)
{
    if (!ctx) return ESC_OK;
    forget_tiles(ctx, nullptr);
    (void)set_device(ctx->device);
    for (hipEvent_t &ev : ctx->slot_event)
        if (ev) (void)hipEventDestroy(ev);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
    return ESC_OK;
}

int esc_ctx_num_cus(const esc_ctx *ctx, int *out)
{
    if (!ctx || !out) return fail(ESC_ERR_INVALID, "null argument");
    *out = ctx->num_cus;
    return ESC_OK;
}

int esc_ctx_dense_fraction(const esc_ctx *ctx, double *out)
{
    if (!ctx || !out) return fail(ESC_ERR_INVALID, "null argument");
    *out = ldexp(1.0, -ctx->dense_shift);
    return ESC_OK;
}

// split selectivities: the conjunct programs, then 2 * kMaxConj counters
constexpr size_t kConjCountersOff = ((size_t)kMaxConj * sizeof(Program) + 255) & ~(size_t)255;
constexpr size_t kConjWsBytes = kConjCountersOff + 2 * kMaxConj * sizeof(unsigned long long);

int esc_workspace_size(const esc_table *t, int kind, size_t *bytes)
{
    if (!t || !bytes) return fail(ESC_ERR_INVALID, "null argument");
    size_t need;
    switch (kind) {
    case ESC_WS_COUNT: need = sizeof(WsHeader); break;
    case ESC_WS_MATERIALIZE: need = ws_layout(t->nrows, 8).bytes; break;   // the smallest wave tile needs the most slots
    case ESC_WS_CONJUNCTS: need = kConjWsBytes; break;
    default: return fail(ESC_ERR_INVALID, "workspace kind %d", kind);
    }
    *bytes = (need + 255) & ~(size_t)255;
    return ESC_OK;
}

int esc_workspace_init(esc_ctx *ctx, void *dev_ws, size_t ws_bytes, void *stream)
{
    if (!ctx || !dev_ws || ws_bytes < sizeof(WsHeader)) return fail(ESC_ERR_INVALID, "bad workspace");
    if (int rc = set_device(ctx->device)) return rc;
    forget_tiles(ctx, dev_ws);
    launch_zero((unsigned long long *)dev_ws, (int64_t)(ws_bytes / 8), (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ESC_OK : hip_fail(e, "zero kernel launch");
}

// Launches the count kernel; stores per-wave-tile counts in the workspace
// when it has room for them (and remembers for which table and predicate).
// With expect != 0 (only when the workspace should hold this predicate's
// tiles) the kernel returns at once if the workspace's stamp equals it.
static int count_launch(esc_ctx *ctx, const esc_table *t, const esc_pred *p, void *dev_ws, size_t ws_bytes,
                        hipStream_t s, unsigned long long *dev_out, bool need_tiles,
                        unsigned long long expect = 0ull)
{
    int rc = check_scan_args(ctx, t, p, dev_ws, ws_bytes, sizeof(WsHeader));
    if (rc) return rc;
    if ((rc = set_device(ctx->device))) return rc;
    const Program &P = p->prog;
    // a constant predicate needs no scan, unless per-tile counts are wanted
    // (an always-true program has no instructions and counts the valid rows)
    const bool constant = (P.flags & P_ALWAYS_FALSE) || ((P.flags & P_ALWAYS_TRUE) && !need_tiles);
    if (constant || t->nrows == 0) {
        const unsigned long long v = (P.flags & P_ALWAYS_TRUE) ? (unsigned long long)t->nrows : 0ull;
        hipLaunchKernelGGL(store_u64_kernel, dim3(1), dim3(1), 0, s, dev_out, v);
    } else {
        // a workspace with room for the tiles receives them (the shape a
        // materialization reads back); otherwise the plain count's shape
        const WsLayout Lt = ws_layout(t->nrows, count_rpt(ctx->count_variant, P.nslots, P.ninsn, true));
        const bool tiles = ws_bytes >= Lt.bytes;
        if (!tiles && need_tiles) return fail(ESC_ERR_OOM, "workspace of %zu bytes, %zu needed", ws_bytes, Lt.bytes);
        const int rpt = count_rpt(ctx->count_variant, P.nslots, P.ninsn, tiles);
        const WsLayout L = ws_layout(t->nrows, rpt);
        TileOut to{nullptr, nullptr, 0ull, 0ull};
        if (tiles) {
            to.counts = (uint32_t *)((char *)dev_ws + L.counts_off);
            to.bits = (uint32_t *)((char *)dev_ws + L.bits_off);
            to.expect = expect;
            to.stamp = expect ? expect : new_stamp();
        }
        CountFn fn = count_fn(P.nslots, P.ninsn, ctx->count_variant, (P.flags & P_HAS_UDF) != 0, tiles);
        const int occ = occupancy((const void *)fn, kScanBlock, 0);
        int64_t grid = (int64_t)ctx->num_cus *
                       (ctx->bpc > 0 ? count_bpc(ctx->count_variant, P.nslots, ctx->bpc, tiles) : occ);
        const int64_t blocks_needed = (L.ntiles + kScanBlock / 64 - 1) / (kScanBlock / 64);
        if (grid > blocks_needed) grid = blocks_needed;
        hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(kScanBlock), to.counts ? kTileBufBytes : 0, s, P,
                           slot_ptrs(t, P, ctx->nt), t->nrows, (WsHeader *)dev_ws, dev_out, to);
        if (to.counts) remember_tiles(ctx, dev_ws, t, p, rpt, to.stamp);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ESC_OK : hip_fail(e, "count kernel launch");
}

int esc_count(esc_ctx *ctx, const esc_table *t, const esc_pred *p, void *dev_ws, size_t ws_bytes, void *stream,
              uint64_t *out_count)
{
    if (!out_count) return fail(ESC_ERR_INVALID, "null out_count");
    hipStream_t s = (hipStream_t)stream;
    // the kernel's last block writes the count straight into pinned host
    // memory: no copy command between the kernel and the wait (waiting for
    // the word to change instead of synchronizing the stream measured slower:
    // 33.7 against 24.1 us per call on a 1M-row table)
    int rc = check_scan_args(ctx, t, p, dev_ws, ws_bytes, sizeof(WsHeader));
    if (rc) return rc;
    // a predicate the compiler decided (always true or false) or an empty
    // table: the count is known without a scan, and nothing is enqueued
    const int pf = p->prog.flags;
    if ((pf & (P_ALWAYS_TRUE | P_ALWAYS_FALSE)) || t->nrows == 0) {
        *out_count = (pf & P_ALWAYS_TRUE) ? (uint64_t)t->nrows : 0u;
        return ESC_OK;
    }
    if ((rc = count_launch(ctx, t, p, dev_ws, ws_bytes, s, ctx->pinned_dev, false))) return rc;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    *out_count = ctx->pinned[0];
    return ESC_OK;
}

int esc_count_async(esc_ctx *ctx, const esc_table *t, const esc_pred *p, void *dev_ws, size_t ws_bytes,
                    void *stream, uint64_t *dev_count)
{
    if (!dev_count) return fail(ESC_ERR_INVALID, "null dev_count");
    return count_launch(ctx, t, p, dev_ws, ws_bytes, (hipStream_t)stream, (unsigned long long *)dev_count, false);
}

int esc_count_begin(esc_ctx *ctx, const esc_table *t, const esc_pred *p, void *dev_ws, size_t ws_bytes,
                    void *stream, int slot)
{
    if (slot < 0 || slot >= ESC_COUNT_SLOTS) return fail(ESC_ERR_INVALID, "slot %d outside [0, %d)", slot, ESC_COUNT_SLOTS);
    int rc = check_scan_args(ctx, t, p, dev_ws, ws_bytes, sizeof(WsHeader));
    if (rc) return rc;
    if (ctx->slot_pending[slot]) return fail(ESC_ERR_INVALID, "slot %d holds a count not yet taken by esc_count_end", slot);
    if ((rc = set_device(ctx->device))) return rc;
    hipError_t e;
    if (!ctx->slot_event[slot] &&
        (e = hipEventCreateWithFlags(&ctx->slot_event[slot], hipEventDisableTiming)) != hipSuccess) {
        ctx->slot_event[slot] = nullptr;
        return hip_fail(e, "hipEventCreateWithFlags");
    }
    hipStream_t s = (hipStream_t)stream;
    // the kernel's last block writes the count into the slot's pinned word
    if ((rc = count_launch(ctx, t, p, dev_ws, ws_bytes, s, ctx->pinned_dev + kSlotWord + slot, false))) return rc;
    if ((e = hipEventRecord(ctx->slot_event[slot], s)) != hipSuccess) {
        // the scan is enqueued but nothing marks its end: let it finish, so
        // that the slot's word is not written after this call returns
        (void)hipStreamSynchronize(s);
        return hip_fail(e, "hipEventRecord");
    }
    ctx->slot_pending[slot] = true;
    return ESC_OK;
}

int esc_count_end(esc_ctx *ctx, int slot, uint64_t *out_count)
{
    if (!ctx || !out_count) return fail(ESC_ERR_INVALID, "null argument");
    if (slot < 0 || slot >= ESC_COUNT_SLOTS) return fail(ESC_ERR_INVALID, "slot %d outside [0, %d)", slot, ESC_COUNT_SLOTS);
    if (!ctx->slot_pending[slot]) return fail(ESC_ERR_INVALID, "slot %d has no count in flight", slot);
    if (int rc = set_device(ctx->device)) return rc;
    hipError_t e = hipEventSynchronize(ctx->slot_event[slot]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    ctx->slot_pending[slot] = false;
    *out_count = ((volatile unsigned long long *)ctx->pinned)[kSlotWord + slot];
    return ESC_OK;
}

}  // extern "C"


// Enqueues count (unless the workspace holds this predicate's tiles), scan
// and write on the stream; the total count lands in *dev_total (device).
static int materialize_launch(esc_ctx *ctx, const esc_table *t, const esc_pred *p, const int32_t *proj_cols,
                              int nproj, int32_t *dev_rowids, void *const *dev_proj_out, uint64_t capacity,
                              void *dev_ws, size_t ws_bytes, hipStream_t s, unsigned long long *dev_total)
{
    if (!ctx || !t || !p) return fail(ESC_ERR_INVALID, "null handle");
    const int rpt = count_rpt(ctx->count_variant, p->prog.nslots, p->prog.ninsn, true);
    const WsLayout L = ws_layout(t->nrows, rpt);
    int rc = check_scan_args(ctx, t, p, dev_ws, ws_bytes, L.bytes);
    if (rc) return rc;
    if (nproj < 0 || nproj > ESC_MAX_PROJ) return fail(ESC_ERR_INVALID, "nproj %d outside [0, %d]", nproj, ESC_MAX_PROJ);
    if (nproj > 0 && !proj_cols) return fail(ESC_ERR_INVALID, "null proj_cols");
    if (capacity > 0 && nproj > 0 && !dev_proj_out) return fail(ESC_ERR_INVALID, "null projection outputs");
    const Program &P = p->prog;
    ProjArgs pa{};
    pa.nproj = nproj;
    const int ncols = (int)t->dtypes.size();
    for (int q = 0; q < nproj; q++) {
        const int c = proj_cols[q];
        if (c < 0 || c >= ncols) return fail(ESC_ERR_INVALID, "projected column %d out of range", c);
        if (capacity > 0 && !dev_proj_out[q]) return fail(ESC_ERR_INVALID, "projection output %d is null", q);
        pa.src[q] = (const uint32_t *)t->cols[c];
        pa.dst[q] = capacity > 0 ? (uint32_t *)dev_proj_out[q] : nullptr;
    }
    if ((rc = set_device(ctx->device))) return rc;
    WsHeader *h = (WsHeader *)dev_ws;
    if ((P.flags & P_ALWAYS_FALSE) || t->nrows == 0) {
        hipLaunchKernelGGL(store_u64_kernel, dim3(1), dim3(1), 0, s, dev_total, 0ull);
    } else {
        uint32_t *tiles = (uint32_t *)((char *)dev_ws + L.counts_off);
        uint32_t *offsets = (uint32_t *)((char *)dev_ws + L.offsets_off);
        const uint32_t *bits = (const uint32_t *)((char *)dev_ws + L.bits_off);
        const unsigned long long expect = tiles_stamp(ctx, dev_ws, t, p, rpt);
        if (!expect && ctx->cold_compact) {
            // no count came first: count and materialize in one pass
            const int64_t ntiles = (t->nrows + 64 * kCompactRPT - 1) / (64 * kCompactRPT);
            const size_t status_off = 256;
            if (status_off + (size_t)ntiles * 8 > ws_bytes)
                return fail(ESC_ERR_OOM, "workspace of %zu bytes, %zu needed", ws_bytes, status_off + (size_t)ntiles * 8);
            forget_tiles(ctx, dev_ws);
            launch_zero((unsigned long long *)dev_ws, (int64_t)((status_off + (size_t)ntiles * 8) / 8), s);
            ProjSlots ps;
            for (int q = 0; q < ESC_MAX_PROJ; q++) {
                ps.slot[q] = -1;
                if (q < nproj)
                    for (int sl = 0; sl < P.nslots; sl++)
                        if (P.slot_col[sl] == proj_cols[q]) ps.slot[q] = sl;
            }
            CompactFn fn = compact_fn(P.nslots, (P.flags & P_HAS_UDF) != 0);
            const int occ = occupancy((const void *)fn, kScanBlock, 0);
            int64_t grid = (int64_t)ctx->num_cus * occ;
            const int64_t blocks_needed = (ntiles + kScanBlock / 64 - 1) / (kScanBlock / 64);
            if (grid > blocks_needed) grid = blocks_needed;
            const uint32_t dense_min = std::max<uint32_t>(1u, (uint32_t)(64 * kCompactRPT) >> ctx->dense_shift);
            hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(kScanBlock), 0, s, P, slot_ptrs(t, P, ctx->nt),
                               t->nrows, (unsigned long long *)((char *)dev_ws + status_off),
                               (unsigned int *)&h->pad1[0], pa, ps, dev_rowids,
                               (unsigned long long)(capacity > 0 ? capacity : 0), dense_min, dev_total);
            hipError_t e = hipGetLastError();
            return e == hipSuccess ? ESC_OK : hip_fail(e, "compaction kernel launch");
        }
        // pass 1: per-wave-tile counts and lane masks, unless the preceding
        // count left them (then the launch only checks the workspace's stamp)
        if ((rc = count_launch(ctx, t, p, dev_ws, ws_bytes, s, &h->result, true, expect))) return rc;
        // pass 2: offsets in row order (total in h->result and dev_total)
        launch_scan(tiles, L.ntiles, offsets, h, dev_total != &h->result ? dev_total : nullptr, s);
        // pass 3: write
        if (capacity > 0) {
            WriteFn fn = write_fn(rpt);
            const int occ = occupancy((const void *)fn, kScanBlock, 0);
            int64_t grid = (int64_t)ctx->num_cus * (ctx->mat_bpc > 0 ? std::min(ctx->mat_bpc, occ) : occ);
            const int64_t blocks_needed = (L.ntiles + kScanBlock / 64 - 1) / (kScanBlock / 64);
            if (grid > blocks_needed) grid = blocks_needed;
            const uint32_t dense_min = std::max<uint32_t>(1u, (uint32_t)(64 * rpt) >> ctx->dense_shift);
            hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(kScanBlock), 0, s, bits, offsets, t->nrows, pa,
                               dev_rowids, (unsigned long long)capacity, dense_min);
        }
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ESC_OK : hip_fail(e, "materialize kernel launch");
}

extern "C" {

int esc_materialize(esc_ctx *ctx, const esc_table *t, const esc_pred *p, const int32_t *proj_cols, int nproj,
                    int32_t *dev_rowids, void *const *dev_proj_out, uint64_t capacity, void *dev_ws,
                    size_t ws_bytes, void *stream, uint64_t *out_count)
{
    if (!out_count) return fail(ESC_ERR_INVALID, "null out_count");
    if (!ctx || !dev_ws || ws_bytes < sizeof(WsHeader)) return fail(ESC_ERR_INVALID, "null handle or workspace");
    hipStream_t s = (hipStream_t)stream;
    WsHeader *h = (WsHeader *)dev_ws;
    int rc = materialize_launch(ctx, t, p, proj_cols, nproj, dev_rowids, dev_proj_out, capacity, dev_ws, ws_bytes, s,
                                &h->result);
    if (rc) return rc;
    hipError_t e;
    if ((e = hipMemcpyAsync(ctx->pinned, &h->result, 8, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    const unsigned long long total = ctx->pinned[0];
    *out_count = total;
    if (total > capacity)
        return fail(ESC_ERR_CAPACITY, "%llu rows qualify, capacity %llu", total, (unsigned long long)capacity);
    return ESC_OK;
}

int esc_count_conjuncts(esc_ctx *ctx, const esc_table *t, const esc_pred *p, void *dev_ws, size_t ws_bytes,
                        void *stream, int max_out, uint64_t *conj_counts, uint64_t *prefix_counts, int *out_nconj)
{
    if (!ctx || !t || !p || !conj_counts || !prefix_counts || !out_nconj) return fail(ESC_ERR_INVALID, "null argument");
    if (!dev_ws || ((uintptr_t)dev_ws & 255)) return fail(ESC_ERR_ALIGN, "workspace must be non-null and 256-byte aligned");
    if (ws_bytes < kConjWsBytes) return fail(ESC_ERR_OOM, "workspace of %zu bytes, %zu needed", ws_bytes, kConjWsBytes);
    if (!t->has_data()) return fail(ESC_ERR_INVALID, "table has no device columns");
    if (p->schema_dtypes != t->dtypes) return fail(ESC_ERR_INVALID, "predicate was compiled for another schema");
    std::vector<Program> progs;
    int nslots = 0, slot_col[kMaxSlots] = {};
    int rc = split_conjuncts(p, progs, nslots, slot_col);
    if (rc) return rc;
    const int m = (int)progs.size();
    if (m > max_out) return fail(ESC_ERR_INVALID, "%d conjuncts, room for %d", m, max_out);
    // a conjunct folded to false runs as an empty bitset test on slot 0 (an
    // always-true one has no instructions and yields every valid row)
    if (nslots == 0) {
        nslots = 1;
        slot_col[0] = 0;
        for (Program &q : progs) {
            q.nslots = 1;
            q.slot_col[0] = 0;
        }
    }
    for (Program &q : progs)
        if (q.flags & P_ALWAYS_FALSE) {
            q.flags &= ~P_ALWAYS_FALSE;
            q.ninsn = 1;
            q.insn[0] = Insn{T_BITSET, 0, (uint8_t)(F_SINGLE | F_END_CLAUSE), 0, 0, 0, 0};
        }
    if ((rc = set_device(ctx->device))) return rc;
    hipError_t e;
    hipStream_t s = (hipStream_t)stream;
    Program *d_progs = (Program *)dev_ws;
    unsigned long long *d_out = (unsigned long long *)((char *)dev_ws + kConjCountersOff);
    if ((e = hipMemcpyAsync(d_progs, progs.data(), m * sizeof(Program), hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "upload conjunct programs");
    launch_zero(d_out, 2 * kMaxConj, s);
    bool udf = false;
    for (const Program &q : progs) udf |= (q.flags & P_HAS_UDF) != 0;
    if (t->nrows > 0) {
        ColPtrs cp{};
        cp.nt = ctx->nt;
        for (int c = 0; c < nslots; c++) cp.p[c] = (const uint32_t *)t->cols[slot_col[c]];
        ConjFn fn = conj_fn(nslots, udf);
        const int occ = occupancy((const void *)fn, kScanBlock, 0);
        int64_t grid = (int64_t)ctx->num_cus * occ;
        const int64_t blocks_needed = (t->nrows + 16 * kScanBlock - 1) / (16 * kScanBlock);
        if (grid > blocks_needed) grid = blocks_needed;
        hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(kScanBlock), 0, s, d_progs, m, cp, t->nrows, d_out);
    }
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "conjunct kernel launch");
    if ((e = hipMemcpyAsync(ctx->pinned, d_out, 2 * kMaxConj * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                            s)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    for (int i = 0; i < m; i++) {
        conj_counts[i] = ctx->pinned[i];
        prefix_counts[i] = ctx->pinned[kMaxConj + i];
    }
    *out_nconj = m;
    return ESC_OK;
}

int esc_materialize_async(esc_ctx *ctx, const esc_table *t, const esc_pred *p, const int32_t *proj_cols, int nproj,
                          int32_t *dev_rowids, void *const *dev_proj_out, uint64_t capacity, void *dev_ws,
                          size_t ws_bytes, void *stream, uint64_t *dev_count)
{
    if (!dev_count) return fail(ESC_ERR_INVALID, "null dev_count");
    return materialize_launch(ctx, t, p, proj_cols, nproj, dev_rowids, dev_proj_out, capacity, dev_ws, ws_bytes,
                              (hipStream_t)stream, (unsigned long long *)dev_count);
}

int esc_materialize_noalloc(esc_ctx *ctx, const esc_table *t, const esc_pred *p, const int32_t *proj_cols,
                            int nproj, int32_t *dev_rowids, void *const *dev_proj_out, uint64_t capacity,
                            void *stream, uint64_t *dev_count)
{
    if (!dev_count) return fail(ESC_ERR_INVALID, "null dev_count");
    if (!ctx || !t || !p) return fail(ESC_ERR_INVALID, "null handle");
    if (!ctx->scratch) return fail(ESC_ERR_INVALID, "context has no static scratch");
    const WsLayout L = ws_layout(t->nrows, count_rpt(ctx->count_variant, p->prog.nslots, p->prog.ninsn, true));
    if (L.bytes > kStaticScratchBytes)
        return fail(ESC_ERR_CAPACITY, "%lld rows need %zu bytes of scratch, the static scratch holds %zu",
                    (long long)t->nrows, L.bytes, kStaticScratchBytes);
    return materialize_launch(ctx, t, p, proj_cols, nproj, dev_rowids, dev_proj_out, capacity, ctx->scratch,
                              kStaticScratchBytes, (hipStream_t)stream, (unsigned long long *)dev_count);
}

}  // extern "C"
