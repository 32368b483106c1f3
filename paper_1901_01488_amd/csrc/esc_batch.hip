// esc_batch.hip -- batched exact selectivity computation: many COUNT(*)
// sub-queries over several tables in one persistent kernel, launched from a
// hipGraph.
//
// Section 2 runs one selectivity sub-query for every table that carries a
// selection.  Here all of them run at once: the predicates of a table are
// packed into groups whose column union fits the register slots; a group's
// rows are cut into chunks, and the (group, chunk) work items sit in a list
// ordered by decreasing cost.  Each block of the persistent grid pops items
// from an atomic counter, loads every column of the group once per tile and
// runs every member predicate on the registers.  Per-wave counts accumulate
// in LDS and reach the global u64 counters with one atomic per predicate per
// item.  Counts are exact and independent of the order of the additions.
//
// The launch (zero counters -> persistent kernel -> copy of the counts to
// pinned host memory) is captured once into a hipGraph; a count is one
// graph launch and one stream synchronisation.  Block shape, rows per thread,
// group size and chunk length are chosen by timing candidate plans on the
// actual tables (an autotuner with an in-process cache and an optional file).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "esc_device.h"
#include "esc_host.h"
#include "esc_kernels.h"
#include "esc_runtime.h"

namespace esc {

constexpr int kMaxGroup = 1024;   // predicates evaluated per pass over a chunk

struct BatchGroup {
    const uint32_t *cols[kMaxSlots];
    int32_t K;
    int32_t npred;
    int32_t pbegin;   // first program / predicate id of the group
    int32_t pad;
};

struct BatchItem {
    int32_t group;
    int32_t r0, r1;
    int32_t pad;
};

// Column pointers of a group come out of device memory, so the compiler
// cannot tell that they point to global memory and would emit flat loads
// (which also hold back every scalar-memory wait of the interpreter); the
// casts make them global loads.
typedef const uint32_t __attribute__((address_space(1))) gu32;
typedef const u32x4 __attribute__((address_space(1))) gu32x4;

// The columns of a full wave tile of the group starting at row `base`.
template <int K, int RPT>
__device__ __forceinline__ void load_tile(const BatchGroup &g, int64_t base, uint32_t (&v)[K][RPT])
{
#pragma unroll
    for (int j = 0; j < RPT / 4; j++) {
        const int64_t idx = base + (int64_t)j * (4 * kWave) + lane_id() * 4;
#pragma unroll
        for (int c = 0; c < K; c++) {
            const u32x4 q = __builtin_nontemporal_load((gu32x4 *)((gu32 *)g.cols[c] + idx));
            v[c][4 * j + 0] = q.x;
            v[c][4 * j + 1] = q.y;
            v[c][4 * j + 2] = q.z;
            v[c][4 * j + 3] = q.w;
        }
    }
}

// Every predicate of the group on one tile; counts into s_cnt.
template <int K, int RPT, bool UDF>
__device__ __forceinline__ void run_tile(const Program *gp, int npred, const uint32_t (&v)[K][RPT], uint32_t valid,
                                         uint32_t (*s_cnt)[kScanBlock / 64], int wave)
{
    for (int i = 0; i < npred; i++) {
        const uint32_t c = wave_sum((uint32_t)__popc(run_program<K, RPT, UDF, 0, true>(gp[i], v, valid)));
        if (lane_id() == 0) s_cnt[i][wave] += c;
    }
}

// The waves of a block walk the item's full wave tiles independently; each
// tile is loaded once and every predicate of the group runs on it.  The
// rows after the last full tile (fewer than one tile) are taken in tiles of
// four rows per lane, with bounds checks: kept apart, their code does not
// add to the registers of the main loop.
template <int K, int RPT, bool UDF>
__device__ __forceinline__ void run_group(const BatchGroup &g, const BatchItem &it, const Program *__restrict__ progs,
                                          uint32_t (*s_cnt)[kScanBlock / 64])
{
    constexpr int TILE = kWave * RPT;
    constexpr int NW = kScanBlock / kWave;
    const int wave = wave_id();
    const int npred = g.npred;
    const Program *gp = progs + g.pbegin;
    const int64_t full_end = it.r0 + (it.r1 - it.r0) / TILE * TILE;
    for (int64_t base = it.r0 + (int64_t)wave * TILE; base < full_end; base += (int64_t)NW * TILE) {
        uint32_t v[K][RPT];
        load_tile<K, RPT>(g, base, v);
        run_tile<K, RPT, UDF>(gp, npred, v, all_rows<RPT>(), s_cnt, wave);
    }
    constexpr int T4 = kWave * 4;
    for (int64_t base = full_end + (int64_t)wave * T4; base < it.r1; base += (int64_t)NW * T4) {
        const uint32_t rem = (uint32_t)(it.r1 - base);   // < TILE: 32-bit offsets
        const uint32_t off = (uint32_t)lane_id() * 4u;
        uint32_t v[K][4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
#pragma unroll
            for (int c = 0; c < K; c++) v[c][r] = off + r < rem ? ((gu32 *)g.cols[c] + base)[off + r] : 0u;
        }
        const uint32_t valid = (off < rem ? 1u : 0u) | (off + 1 < rem ? 2u : 0u) | (off + 2 < rem ? 4u : 0u) |
                               (off + 3 < rem ? 8u : 0u);
        run_tile<K, 4, UDF>(gp, npred, v, valid, s_cnt, wave);
    }
}

// One persistent kernel per (rows per lane, udf support, column slots KM):
// a group's K <= KM columns are dispatched to a body compiled for K, so the
// kernel's registers (and the waves a SIMD holds) follow from KM.
template <int RPT, bool UDF, int KM>
__global__ __launch_bounds__(kScanBlock) void batch_kernel(const BatchGroup *__restrict__ groups,
                                                           const BatchItem *__restrict__ items,
                                                           const Program *__restrict__ progs,
                                                           const int32_t *__restrict__ pred_ids,
                                                           unsigned long long *counts, unsigned int *queue)
{
    constexpr int NW = kScanBlock / 64;
    __shared__ uint32_t s_cnt[kMaxGroup][NW];
    __shared__ int s_item;
    const int nitems = (int)queue[1];   // written by the host with the plan
    for (int i = threadIdx.x; i < kMaxGroup * NW; i += kScanBlock) (&s_cnt[0][0])[i] = 0;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= nitems) break;
        const BatchItem it = items[item];
        const BatchGroup &g = groups[it.group];
        switch (g.K) {
        case 1: run_group<1, RPT, UDF>(g, it, progs, s_cnt); break;
        case 2: run_group<2, RPT, UDF>(g, it, progs, s_cnt); break;
        case 3: run_group<3, RPT, UDF>(g, it, progs, s_cnt); break;
        case 4: run_group<4, RPT, UDF>(g, it, progs, s_cnt); break;
        default:
            if constexpr (KM >= 6) {
                switch (g.K) {
                case 5: run_group<5, RPT, UDF>(g, it, progs, s_cnt); break;
                case 6: run_group<6, RPT, UDF>(g, it, progs, s_cnt); break;
                default:
                    if constexpr (KM >= 8) {
                        if (g.K == 7) run_group<7, RPT, UDF>(g, it, progs, s_cnt);
                        else run_group<8, RPT, UDF>(g, it, progs, s_cnt);
                    }
                    break;
                }
            }
            break;
        }        __syncthreads();
        for (int i = threadIdx.x; i < g.npred; i += kScanBlock) {
            unsigned long long s = 0;
#pragma unroll
            for (int w = 0; w < NW; w++) {
                s += s_cnt[i][w];
                s_cnt[i][w] = 0;
            }
            if (s) atomicAdd(&counts[pred_ids[g.pbegin + i]], s);
        }
        __syncthreads();
    }
}

typedef void (*BatchFn)(const BatchGroup *, const BatchItem *, const Program *, const int32_t *,
                        unsigned long long *, unsigned int *);

template <int KM>
static BatchFn batch_fn_km(int rpt, bool udf)
{
    if (rpt == 16) return udf ? batch_kernel<16, true, KM> : batch_kernel<16, false, KM>;
    return udf ? batch_kernel<8, true, KM> : batch_kernel<8, false, KM>;
}

static BatchFn batch_fn(int rpt, bool udf, int km)
{
    return km <= 4 ? batch_fn_km<4>(rpt, udf) : km <= 6 ? batch_fn_km<6>(rpt, udf) : batch_fn_km<8>(rpt, udf);
}

__global__ void batch_zero_kernel(unsigned long long *counts, int n, unsigned int *queue)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) counts[i] = 0ull;
    if (blockIdx.x == 0 && threadIdx.x == 0) *queue = 0u;
}

}  // namespace esc

using namespace esc;

struct TableInfo {
    int64_t nrows;
    std::vector<int32_t> dtypes;
    std::vector<const void *> cols;
};

struct Plan {
    std::vector<BatchGroup> groups;
    std::vector<BatchItem> items;
    std::vector<Program> progs;
    std::vector<int32_t> pred_ids;
};

struct esc_batch {
    esc_ctx *ctx = nullptr;
    int device = 0;                      // kept so that destruction never touches ctx
    std::vector<TableInfo> tables;
    std::vector<int32_t> pred_table;
    std::vector<Program> src;            // compiled programs as given
    std::vector<int> constant;           // 0: scanned; 1: always true; -1: always false or empty table
    esc_batch_opts opts{};
    int nkernel = 0;                     // predicates evaluated by the kernel
    // device state: fixed regions of the caller's workspace
    BatchGroup *d_groups = nullptr;
    BatchItem *d_items = nullptr;
    Program *d_progs = nullptr;
    int32_t *d_pred_ids = nullptr;
    unsigned long long *d_counts = nullptr;
    unsigned int *d_queue = nullptr;     // [0] next item, [1] number of items
    size_t cap_counts = 0;               // predicates the regions hold (the counters the graph zeroes and copies)
    size_t cap_items = 0;                // work items the item region holds
    const void *graph_fn = nullptr;      // kernel the captured graph launches
    unsigned long long *h_counts = nullptr;   // pinned host memory, cap_counts entries
    int nitems = 0;
    int grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap_stream = nullptr;
};

namespace {

int hipchk(hipError_t e, const char *what) { return e == hipSuccess ? ESC_OK : hip_fail(e, what); }

int tile_rows(int rpt) { return kScanBlock * rpt; }

// Remaps the slots of program P (its own slot order) onto the group's slots.
Program remap(const Program &P, const int *gslot_of_col, int K, const int *gcols)
{
    Program Q = P;
    for (int i = 0; i < P.ninsn; i++) {
        Insn &I = Q.insn[i];
        const bool udf_op = I.op >= U_LOAD;
        const bool reads_col = udf_op ? !(I.flags & F_CONST) : !(I.flags & F_SRC_UDF);
        if (reads_col) I.src = (uint8_t)gslot_of_col[P.slot_col[I.src]];
    }
    Q.nslots = K;
    for (int s = 0; s < kMaxSlots; s++) Q.slot_col[s] = s < K ? gcols[s] : 0;
    return Q;
}

// Column slots of the kernel a batch uses: the smallest of 4, 6 and 8 that
// holds max_cols and every scanned predicate's columns.
int slot_limit(const esc_batch *b, const esc_batch_opts &o)
{
    int need = std::max(1, (int)o.max_cols);
    for (size_t p = 0; p < b->src.size(); p++)
        if (b->constant[p] == 0) need = std::max(need, (int)b->src[p].nslots);
    return need <= 4 ? 4 : need <= 6 ? 6 : 8;
}

// chunk_rows == 0 sizes the chunks so that the plan has about eight items
// per block of the persistent grid (load balance at the end of the launch),
// but no fewer than 8 block tiles per item (the per-item cost of the atomic
// pop and of publishing the group's counts stays small).
int64_t chunk_rows_for(const esc_batch *b, const esc_batch_opts &o, int gmax, int grid)
{
    const int tile = tile_rows(o.rows_per_thread);
    int64_t chunk = o.chunk_rows;
    if (chunk <= 0) {
        int64_t rows = 0;
        for (size_t t = 0; t < b->tables.size(); t++) {
            int64_t np = 0;
            for (size_t p = 0; p < b->pred_table.size(); p++) np += b->pred_table[p] == (int)t && b->constant[p] == 0;
            rows += b->tables[t].nrows * ((np + gmax - 1) / gmax);   // a lower bound on the groups of the table
        }
        chunk = std::max<int64_t>(rows / (8 * (int64_t)std::max(grid, 1)), 8 * (int64_t)tile);
        chunk = std::min<int64_t>(chunk, 1 << 21);
    }
    return (chunk + tile - 1) / tile * tile;
}

int build_plan(const esc_batch *b, const esc_batch_opts &o, int grid, Plan &plan)
{
    plan = Plan{};
    const int gmax = o.group > 0 ? std::min(o.group, kMaxGroup) : kMaxGroup;
    const int kmax = slot_limit(b, o);
    const int64_t chunk = chunk_rows_for(b, o, gmax, grid);
    struct Cost { int64_t cost; BatchItem it; };
    std::vector<Cost> items;
    for (size_t t = 0; t < b->tables.size(); t++) {
        const TableInfo &T = b->tables[t];
        std::vector<int> members;
        for (size_t p = 0; p < b->pred_table.size(); p++)
            if (b->pred_table[p] == (int)t && b->constant[p] == 0) members.push_back((int)p);
        size_t i = 0;
        while (i < members.size()) {
            int gslot[64];
            for (int c = 0; c < 64; c++) gslot[c] = -1;
            int gcols[kMaxSlots];
            int K = 0;
            std::vector<int> mem;
            while (i < members.size() && (int)mem.size() < gmax) {
                const Program &P = b->src[members[i]];
                int add = 0;
                for (int s = 0; s < P.nslots; s++) add += gslot[P.slot_col[s]] < 0;
                if (K + add > kmax) break;
                for (int s = 0; s < P.nslots; s++)
                    if (gslot[P.slot_col[s]] < 0) { gslot[P.slot_col[s]] = K; gcols[K++] = P.slot_col[s]; }
                mem.push_back(members[i]);
                i++;
            }
            BatchGroup g{};
            g.K = K > 0 ? K : 1;
            if (K == 0) gcols[0] = 0;
            for (int s = 0; s < g.K; s++) g.cols[s] = (const uint32_t *)T.cols[gcols[s]];
            g.npred = (int)mem.size();
            g.pbegin = (int)plan.progs.size();
            for (int p : mem) {
                plan.progs.push_back(remap(b->src[p], gslot, g.K, gcols));
                plan.pred_ids.push_back(p);
            }
            const int gid = (int)plan.groups.size();
            plan.groups.push_back(g);
            for (int64_t r0 = 0; r0 < T.nrows; r0 += chunk) {
                const int64_t r1 = std::min<int64_t>(T.nrows, r0 + chunk);
                BatchItem it{gid, (int32_t)r0, (int32_t)r1, 0};
                items.push_back({(r1 - r0) * (int64_t)mem.size() * (K + 1), it});
            }
        }
    }
    std::stable_sort(items.begin(), items.end(), [](const Cost &a, const Cost &c) { return a.cost > c.cost; });
    for (auto &c : items) plan.items.push_back(c.it);
    return ESC_OK;
}

// Regions of a batch workspace for pcap predicates and icap work items.
struct BatchLayout {
    size_t queue, counts, ids, progs, groups, items, bytes;
};

BatchLayout batch_layout(size_t pcap, size_t icap)
{
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    BatchLayout L;
    L.queue = 0;
    L.counts = 256;
    L.ids = up(L.counts + pcap * sizeof(unsigned long long));
    L.progs = up(L.ids + pcap * sizeof(int32_t));
    L.groups = up(L.progs + pcap * sizeof(Program));
    L.items = up(L.groups + pcap * sizeof(BatchGroup));
    L.bytes = up(L.items + icap * sizeof(BatchItem));
    return L;
}

// Options as a batch uses them: rows per thread 8 or 16, block of 256.
esc_batch_opts normalized(const esc_batch_opts *opts)
{
    esc_batch_opts o{};
    if (opts) o = *opts;
    if (o.rows_per_thread != 16) o.rows_per_thread = 8;
    o.block = kScanBlock;
    if (o.max_cols != 4 && o.max_cols != 6 && o.max_cols != 8) o.max_cols = 0;
    if (o.group < 0) o.group = 0;
    if (o.chunk_rows < 0) o.chunk_rows = 0;
    if (o.blocks_per_cu < 0) o.blocks_per_cu = 0;
    return o;
}

void destroy_graph(esc_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Uploads a plan; captures zero -> kernel -> copy into a graph unless the
// graph of an earlier plan still fits (same buffers, kernel shape and counter
// capacity): the item count lives in device memory, so a new plan of the
// same shape costs a few small copies and no capture.
// The kernel a batch launches: rows per thread, and udf support when any
// scanned predicate has a udf.
BatchFn batch_kernel_for(const esc_batch *b, const esc_batch_opts &o)
{
    bool udf = false;
    for (size_t p = 0; p < b->src.size(); p++) udf |= b->constant[p] == 0 && (b->src[p].flags & P_HAS_UDF) != 0;
    return batch_fn(o.rows_per_thread, udf, slot_limit(b, o));
}

// Persistent grid of a launch: blocks per CU as asked, at most what fits
// (idle blocks exit at once).
int plan_grid(const esc_batch *b, const esc_batch_opts &o)
{
    const int occ = occupancy((const void *)batch_kernel_for(b, o), kScanBlock, 0);
    const int bpc = o.blocks_per_cu > 0 ? std::min(o.blocks_per_cu, occ) : occ;
    return std::max(1, b->ctx->num_cus * bpc);
}

std::string tune_key(const esc_batch *b);
bool cached_tune(const std::string &key, esc_batch_opts *out);

// The configurations a batch with these options may install: the options
// themselves, or with autotuning every candidate the tuner times (rows per
// thread x group size x chunk length) and a choice cached for these tables
// and predicates.
std::vector<esc_batch_opts> tuner_candidates(const esc_batch *b)
{
    std::vector<esc_batch_opts> out;
    const int rpts[] = {16, 8};
    const int groups[] = {0, 16, 8};
    const int chunks[] = {0, 1 << 17, 1 << 20};   // 0: sized to the grid
    esc_batch_opts least{};
    const int kmin = slot_limit(b, least);
    for (int km : {kmin, 8}) {
        for (int rpt : rpts)
            for (int grp : groups)
                for (int ch : chunks) {
                    esc_batch_opts c{};
                    c.block = kScanBlock;
                    c.rows_per_thread = rpt;
                    c.group = grp;
                    c.chunk_rows = ch;
                    c.max_cols = km;
                    out.push_back(c);
                }
        if (kmin == 8) break;
    }
    return out;
}

std::vector<esc_batch_opts> candidates(const esc_batch *b, const esc_batch_opts &o)
{
    if (!o.autotune) return {o};
    std::vector<esc_batch_opts> out = tuner_candidates(b);
    esc_batch_opts cached{};
    if (cached_tune(tune_key(b), &cached)) out.push_back(cached);
    return out;
}

int install(esc_batch *b, const esc_batch_opts &o)
{
    BatchFn fn = batch_kernel_for(b, o);
    const int grid = plan_grid(b, o);
    Plan plan;
    int rc = build_plan(b, o, grid, plan);
    if (rc) return rc;
    if (plan.items.size() > b->cap_items)
        return fail(ESC_ERR_OOM, "the plan has %zu work items, the workspace holds %zu", plan.items.size(),
                    b->cap_items);
    hipStream_t s = b->cap_stream;
    const unsigned int nitems = (unsigned int)plan.items.size();
    if ((rc = hipchk(hipMemcpyAsync(b->d_groups, plan.groups.data(), plan.groups.size() * sizeof(BatchGroup),
                                    hipMemcpyHostToDevice, s), "upload groups"))) return rc;
    if ((rc = hipchk(hipMemcpyAsync(b->d_items, plan.items.data(), plan.items.size() * sizeof(BatchItem),
                                    hipMemcpyHostToDevice, s), "upload items"))) return rc;
    if ((rc = hipchk(hipMemcpyAsync(b->d_progs, plan.progs.data(), plan.progs.size() * sizeof(Program),
                                    hipMemcpyHostToDevice, s), "upload programs"))) return rc;
    if ((rc = hipchk(hipMemcpyAsync(b->d_pred_ids, plan.pred_ids.data(), plan.pred_ids.size() * sizeof(int32_t),
                                    hipMemcpyHostToDevice, s), "upload ids"))) return rc;
    if ((rc = hipchk(hipMemcpyAsync(b->d_queue + 1, &nitems, sizeof nitems, hipMemcpyHostToDevice, s),
                     "upload item count"))) return rc;
    if ((rc = hipchk(hipStreamSynchronize(s), "upload sync"))) return rc;
    b->nitems = (int)nitems;
    b->opts = o;
    b->opts.blocks_per_cu = grid / std::max(1, b->ctx->num_cus);
    b->opts.max_cols = slot_limit(b, o);
    // the graph bakes in the workspace regions (fixed for the batch's
    // lifetime), the counter capacity and the kernel
    const bool reuse = b->exec && grid == b->grid && b->graph_fn == (const void *)fn;
    if (reuse) return ESC_OK;
    destroy_graph(b);
    b->grid = grid;
    const int cap = (int)b->cap_counts;
    if ((rc = hipchk(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture"))) return rc;
    hipLaunchKernelGGL(batch_zero_kernel, dim3(std::max(1, std::min(64, (cap + 255) / 256))), dim3(256), 0, s,
                       b->d_counts, cap, b->d_queue);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kScanBlock), 0, s, b->d_groups, b->d_items, b->d_progs, b->d_pred_ids,
                       b->d_counts, b->d_queue);
    (void)hipMemcpyAsync(b->h_counts, b->d_counts, cap * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (e != hipSuccess) return hip_fail(e, "end capture");
    b->graph = g;
    if ((e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0)) != hipSuccess) return hip_fail(e, "instantiate");
    b->graph_fn = (const void *)fn;
    return ESC_OK;
}

int run(esc_batch *b, hipStream_t s, uint64_t *out)
{
    hipError_t e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (out) {
        for (size_t p = 0; p < b->pred_table.size(); p++) {
            if (b->constant[p] == 1) out[p] = (uint64_t)b->tables[b->pred_table[p]].nrows;
            else if (b->constant[p] == -1) out[p] = 0;
            else out[p] = b->h_counts[p];
        }
    }
    return ESC_OK;
}

std::mutex g_tune_mu;
std::map<std::string, esc_batch_opts> g_tune_cache;

std::string tune_key(const esc_batch *b)
{
    std::string k = "cus=" + std::to_string(b->ctx->num_cus);
    for (size_t t = 0; t < b->tables.size(); t++) {
        int np = 0, ni = 0;
        for (size_t p = 0; p < b->pred_table.size(); p++)
            if (b->pred_table[p] == (int)t) { np++; ni += b->src[p].ninsn; }
        k += ";" + std::to_string(b->tables[t].nrows) + "x" + std::to_string(b->tables[t].dtypes.size()) + ":" +
             std::to_string(np) + "/" + std::to_string(ni);
    }
    return k;
}

// Whether cached options are ones a batch would accept as they are.
bool acceptable(const esc_batch_opts &o)
{
    return o.block == kScanBlock && (o.rows_per_thread == 8 || o.rows_per_thread == 16) && o.group >= 0 &&
           o.chunk_rows >= 0 && o.blocks_per_cu >= 0 &&
           (o.max_cols == 0 || o.max_cols == 4 || o.max_cols == 6 || o.max_cols == 8);
}

// Reads "key block rpt group chunk bpc [max_cols]" lines into the
// in-process cache; lines that do not parse or hold options a batch would
// not accept are skipped.  Needs g_tune_mu.
int read_tune_file(const char *path, int *accepted, int *rejected)
{
    FILE *f = fopen(path, "r");
    if (!f) return fail(ESC_ERR_INVALID, "cannot open %s", path);
    int ok = 0, bad = 0;
    char line[8192];
    while (fgets(line, sizeof line, f)) {
        char key[4096];
        esc_batch_opts o{};
        char extra[2];
        const int n = sscanf(line, "%4095s %d %d %d %d %d %d %1s", key, &o.block, &o.rows_per_thread, &o.group,
                             &o.chunk_rows, &o.blocks_per_cu, &o.max_cols, extra);
        if (n <= 0) continue;   // blank line
        if ((n == 6 || n == 7) && acceptable(o)) {
            g_tune_cache[key] = o;
            ok++;
        } else {
            bad++;
        }
    }
    fclose(f);
    if (accepted) *accepted = ok;
    if (rejected) *rejected = bad;
    return ESC_OK;
}

void load_tune_file()
{
    static bool done = false;
    if (done) return;
    done = true;
    const char *path = getenv("ESC_AUTOTUNE_CACHE");
    if (path) (void)read_tune_file(path, nullptr, nullptr);
    clear_error();
}

void save_tune(const std::string &key, const esc_batch_opts &o)
{
    const char *path = getenv("ESC_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d %d %d %d\n", key.c_str(), o.block, o.rows_per_thread, o.group, o.chunk_rows,
            o.blocks_per_cu, o.max_cols);
    fclose(f);
}

bool cached_tune(const std::string &key, esc_batch_opts *out)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    load_tune_file();
    auto it = g_tune_cache.find(key);
    if (it == g_tune_cache.end()) return false;
    *out = it->second;
    return true;
}

// Times candidate plans on the batch's own tables and keeps the fastest;
// every candidate's counts must agree (a free consistency check).
int autotune(esc_batch *b, hipStream_t s)
{
    const std::string key = tune_key(b);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        load_tune_file();
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) return install(b, it->second);
    }
    const int npreds = (int)b->pred_table.size();
    std::vector<uint64_t> ref(npreds), got(npreds);
    bool have_ref = false;
    float best = 1e30f;
    esc_batch_opts bo{};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(ESC_ERR_HIP, "hipEventCreate failed");
    int rc = ESC_OK;
    for (const esc_batch_opts &o : tuner_candidates(b)) {
                if ((rc = install(b, o))) goto done;
                if ((rc = run(b, s, got.data()))) goto done;
                if (!have_ref) { ref = got; have_ref = true; }
                else if (ref != got) { rc = fail(ESC_ERR_HIP, "autotune: candidate plans disagree on a count"); goto done; }
                float tmin = 1e30f;
                for (int rep = 0; rep < 3; rep++) {
                    (void)hipEventRecord(e0, s);
                    (void)hipGraphLaunch(b->exec, s);
                    (void)hipEventRecord(e1, s);
                    (void)hipEventSynchronize(e1);
                    float ms = 0;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    tmin = std::min(tmin, ms);
                }
                if (tmin < best) { best = tmin; bo = b->opts; }
            }
    rc = install(b, bo);
    if (!rc) {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune_cache[key] = b->opts;
        save_tune(key, b->opts);
    }
done:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int set_preds(esc_batch *b, const esc_pred *const *preds, int npreds)
{
    b->src.resize(npreds);
    b->constant.assign(npreds, 0);
    for (int p = 0; p < npreds; p++) {
        if (!preds[p]) return fail(ESC_ERR_INVALID, "predicate %d is null", p);
        const TableInfo &T = b->tables[b->pred_table[p]];
        if (preds[p]->schema_dtypes != T.dtypes)
            return fail(ESC_ERR_INVALID, "predicate %d was compiled for another schema than table %d", p, b->pred_table[p]);
        b->src[p] = preds[p]->prog;
        const int fl = preds[p]->prog.flags;
        if (T.nrows == 0 || (fl & P_ALWAYS_FALSE)) b->constant[p] = -1;
        else if (fl & P_ALWAYS_TRUE) b->constant[p] = 1;
    }
    return ESC_OK;
}

void free_batch(esc_batch *b)
{
    destroy_graph(b);
    if (b->h_counts) (void)hipHostFree(b->h_counts);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
}

}  // namespace

extern "C" {

int esc_batch_workspace_size(esc_ctx *ctx, const esc_table *const *tables, int ntables,
                             const esc_pred *const *preds, const int32_t *pred_table, int npreds,
                             const esc_batch_opts *opts, size_t *bytes)
{
    if (!ctx || !tables || !preds || !pred_table || !bytes) return fail(ESC_ERR_INVALID, "null argument");
    if (ntables <= 0 || npreds <= 0) return fail(ESC_ERR_INVALID, "empty batch");
    esc_batch tmp;   // host side only: the plans of these predicates
    tmp.ctx = ctx;
    for (int t = 0; t < ntables; t++) {
        if (!tables[t]) return fail(ESC_ERR_INVALID, "table %d is null", t);
        tmp.tables.push_back({tables[t]->nrows, tables[t]->dtypes, tables[t]->cols});
    }
    for (int p = 0; p < npreds; p++)
        if (pred_table[p] < 0 || pred_table[p] >= ntables) return fail(ESC_ERR_INVALID, "pred_table[%d] out of range", p);
    tmp.pred_table.assign(pred_table, pred_table + npreds);
    int rc = set_preds(&tmp, preds, npreds);
    if (rc) return rc;
    const esc_batch_opts o = normalized(opts);
    size_t items = 0;
    for (const esc_batch_opts &c : candidates(&tmp, o)) {
        Plan plan;
        if ((rc = build_plan(&tmp, c, plan_grid(&tmp, c), plan))) return rc;
        items = std::max(items, plan.items.size());
    }
    *bytes = batch_layout((size_t)std::max(npreds, o.max_preds), items).bytes;
    return ESC_OK;
}

int esc_batch_tune_cache_load(const char *path, int *accepted, int *rejected)
{
    if (!path) return fail(ESC_ERR_INVALID, "null path");
    std::lock_guard<std::mutex> g(g_tune_mu);
    return read_tune_file(path, accepted, rejected);
}

int esc_batch_create(esc_ctx *ctx, const esc_table *const *tables, int ntables, const esc_pred *const *preds,
                     const int32_t *pred_table, int npreds, const esc_batch_opts *opts, void *dev_ws,
                     size_t ws_bytes, void *stream, esc_batch **out)
{
    if (!ctx || !tables || !preds || !pred_table || !out) return fail(ESC_ERR_INVALID, "null argument");
    if (ntables <= 0 || npreds <= 0) return fail(ESC_ERR_INVALID, "empty batch");
    if (!dev_ws || ((uintptr_t)dev_ws & 255)) return fail(ESC_ERR_ALIGN, "workspace must be non-null and 256-byte aligned");
    const esc_batch_opts o = normalized(opts);
    size_t need = 0;
    int rc = esc_batch_workspace_size(ctx, tables, ntables, preds, pred_table, npreds, &o, &need);
    if (rc) return rc;
    if (ws_bytes < need) return fail(ESC_ERR_OOM, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    esc_batch *b = new (std::nothrow) esc_batch;
    if (!b) return fail(ESC_ERR_OOM, "out of host memory");
    b->ctx = ctx;
    b->device = ctx->device;
    if (int rc0 = set_device(ctx->device)) { delete b; return rc0; }
    for (int t = 0; t < ntables; t++) {
        if (!tables[t] || !tables[t]->has_data()) { free_batch(b); return fail(ESC_ERR_INVALID, "table %d has no device columns", t); }
        b->tables.push_back({tables[t]->nrows, tables[t]->dtypes, tables[t]->cols});
    }
    b->pred_table.assign(pred_table, pred_table + npreds);
    for (int p = 0; p < npreds; p++)
        if (pred_table[p] < 0 || pred_table[p] >= ntables) { free_batch(b); return fail(ESC_ERR_INVALID, "pred_table[%d] out of range", p); }
    if ((rc = set_preds(b, preds, npreds))) { free_batch(b); return rc; }
    // fixed regions of the workspace: counters and programs for pcap
    // predicates, the rest of it for work items
    const size_t pcap = (size_t)std::max(npreds, o.max_preds);
    const BatchLayout L0 = batch_layout(pcap, 0);
    char *base = (char *)dev_ws;
    b->d_queue = (unsigned int *)(base + L0.queue);
    b->d_counts = (unsigned long long *)(base + L0.counts);
    b->d_pred_ids = (int32_t *)(base + L0.ids);
    b->d_progs = (Program *)(base + L0.progs);
    b->d_groups = (BatchGroup *)(base + L0.groups);
    b->d_items = (BatchItem *)(base + L0.items);
    b->cap_counts = pcap;
    b->cap_items = (ws_bytes - L0.items) / sizeof(BatchItem);
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess) { free_batch(b); return hip_fail(e, "stream"); }
    if ((e = hipHostMalloc((void **)&b->h_counts, pcap * sizeof(unsigned long long), hipHostMallocDefault)) != hipSuccess) {
        b->h_counts = nullptr;
        free_batch(b);
        return fail(ESC_ERR_OOM, "pinned host counters: %s", hipGetErrorString(e));
    }
    if (o.autotune) rc = autotune(b, (hipStream_t)stream);
    else rc = install(b, o);
    if (rc) { free_batch(b); return rc; }
    *out = b;
    return ESC_OK;
}

int esc_batch_update(esc_batch *b, const esc_pred *const *preds, const int32_t *pred_table, int npreds,
                     void *stream)
{
    (void)stream;
    if (!b || !preds || npreds <= 0) return fail(ESC_ERR_INVALID, "null argument or empty batch");
    if (!pred_table && npreds != (int)b->pred_table.size())
        return fail(ESC_ERR_INVALID, "a different number of predicates needs pred_table");
    if (int rc0 = set_device(b->device)) return rc0;
    if ((size_t)npreds > b->cap_counts)
        return fail(ESC_ERR_OOM, "%d predicates, the batch was created for at most %zu", npreds, b->cap_counts);
    if (pred_table) {
        for (int p = 0; p < npreds; p++)
            if (pred_table[p] < 0 || pred_table[p] >= (int)b->tables.size())
                return fail(ESC_ERR_INVALID, "pred_table[%d] out of range", p);
        b->pred_table.assign(pred_table, pred_table + npreds);
    }
    int rc = set_preds(b, preds, npreds);
    if (rc) return rc;
    return install(b, b->opts);
}

int esc_batch_count(esc_batch *b, void *stream, uint64_t *out_counts)
{
    if (!b || !out_counts) return fail(ESC_ERR_INVALID, "null argument");
    if (int rc = set_device(b->device)) return rc;
    return run(b, (hipStream_t)stream, out_counts);
}

int esc_batch_get_opts(const esc_batch *b, esc_batch_opts *out)
{
    if (!b || !out) return fail(ESC_ERR_INVALID, "null argument");
    *out = b->opts;
    return ESC_OK;
}

int esc_batch_destroy(esc_batch *b)
{
    if (!b) return ESC_OK;
    (void)set_device(b->device);
    free_batch(b);
    return ESC_OK;
}

}  // extern "C"
