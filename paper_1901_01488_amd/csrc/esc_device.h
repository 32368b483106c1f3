// esc_device.h -- device-side evaluation of a compiled predicate program on
// a tile of rows held in registers (shared by the plain and batched scans).
//
// Tile layout: each wave owns a contiguous "wave tile" of 64*RPT rows; row
// slot r = 4*j + e of lane l is row base + j*256 + l*4 + e, so the j-th
// 16-byte load of the 64 lanes is one coalesced 1 KiB request, and the rows
// of a wave tile in row order are (j, lane, e).  Waves never wait for each
// other: a scan is a grid-stride loop over wave tiles.
//
// Truth values are per-lane bit masks: bit r of a lane's mask is the value
// for its row slot r.  A test costs three vector ops per row slot (compare
// and shift-in), clause logic costs one op per test for all RPT rows, and
// the scalar unit is left to the wave-uniform interpretation of the program.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "esc_kernels.h"
#include "esc_program.h"

namespace esc {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float as_f(uint32_t u) { return __uint_as_float(u); }

template <int K, int C = 0, typename F>
__device__ __forceinline__ void for_slot(int s, F &&f)
{
    if constexpr (C < K) {
        if (s == C) f(std::integral_constant<int, C>{});
        else for_slot<K, C + 1>(s, f);
    }
}

// for_slot as one switch (the compiler makes it a tree of about log2(K)
// branches instead of a chain of up to K).
template <int K, typename F>
__device__ __forceinline__ void switch_slot(int s, F &&f)
{
    switch (s) {
    case 0: if constexpr (K > 0) f(std::integral_constant<int, 0>{}); break;
    case 1: if constexpr (K > 1) f(std::integral_constant<int, 1>{}); break;
    case 2: if constexpr (K > 2) f(std::integral_constant<int, 2>{}); break;
    case 3: if constexpr (K > 3) f(std::integral_constant<int, 3>{}); break;
    case 4: if constexpr (K > 4) f(std::integral_constant<int, 4>{}); break;
    case 5: if constexpr (K > 5) f(std::integral_constant<int, 5>{}); break;
    case 6: if constexpr (K > 6) f(std::integral_constant<int, 6>{}); break;
    default: if constexpr (K > 7) f(std::integral_constant<int, 7>{}); break;
    }
    static_assert(K <= 8, "eight slots at most");
}

// Per-lane mask of a row test: bit r = test(r).
template <int RPT, typename T>
__device__ __forceinline__ uint32_t bits_of(T &&test)
{
    static_assert(RPT <= 32 && RPT % 2 == 0, "masks are 32-bit, rows come in pairs");
    // each row selects its own bit (one select per row), two rows are merged
    // into the mask by one three-input OR
    uint32_t m = 0;
#pragma unroll
    for (int r = 0; r < RPT; r += 2) m |= (test(r) ? 1u << r : 0u) | (test(r + 1) ? 1u << (r + 1) : 0u);
    return m;
}

template <int RPT>
__device__ __forceinline__ uint32_t all_rows()
{
    return RPT == 32 ? 0xffffffffu : ((1u << RPT) - 1u);
}

// Slot tables of a program held in registers, one entry per lane: NT =
// kMaxTables for kernels that run one program throughout (loaded once,
// before the first tile), NT = 0 for kernels that switch programs (each
// slot-table test then reads its table from the constant pool).  Named
// fields rather than an array: a runtime-indexed array would be moved to
// LDS by the compiler.
template <int NT>
struct SlotTabs {
    uint32_t e0 = 0, e1 = 0, e2 = 0, e3 = 0;
    static_assert(NT == 0 || NT == 4, "four slot tables per program");
};

template <int NT>
__device__ __forceinline__ SlotTabs<NT> load_tables(const Program &P)
{
    SlotTabs<NT> t;
    if constexpr (NT > 0) {
        const uint32_t *k = P.kpool + (threadIdx.x & 63u);
        const int nt = P.ntables;
        if (nt > 0) t.e0 = k[0];
        if (nt > 1) t.e1 = k[kSlotTable];
        if (nt > 2) t.e2 = k[2 * kSlotTable];
        if (nt > 3) t.e3 = k[3 * kSlotTable];
    }
    return t;
}

template <int RPT, int NT>
__device__ __forceinline__ uint32_t run_test(const Insn &I, const uint32_t *kpool, const SlotTabs<NT> &tabs,
                                             const uint32_t (&x)[RPT])
{
    switch (I.op) {
    case T_RANGE_I32: {
        const uint32_t lo = (uint32_t)I.a, span = (uint32_t)I.b;
        return bits_of<RPT>([&](int r) { return x[r] - lo <= span; });
    }
    case T_RANGE_F32: {
        const float lo = as_f((uint32_t)I.a), hi = as_f((uint32_t)I.b);
        return bits_of<RPT>([&](int r) { const float f = as_f(x[r]); return lo <= f && f <= hi; });
    }
    case T_BITSET: {
        // two 32-bit words rather than one 64-bit shift per row
        const uint32_t lo = (uint32_t)I.a, w0 = (uint32_t)I.b, w1 = (uint32_t)I.c;
        return bits_of<RPT>([&](int r) {
            const uint32_t d = x[r] - lo;
            const uint32_t w = d < 32u ? w0 : w1;
            return d < 64u && ((w >> (d & 31u)) & 1u);
        });
    }
    case T_IN_I32: {
        uint32_t m = 0;
        for (int k = 0; k < I.b; k++) {
            const uint32_t kv = kpool[I.a + k];
            m |= bits_of<RPT>([&](int r) { return x[r] == kv; });
        }
        return m;
    }
    case T_IN_F32: {
        uint32_t m = 0;
        for (int k = 0; k < I.b; k++) {
            const float kf = as_f(kpool[I.a + k]);
            m |= bits_of<RPT>([&](int r) { return as_f(x[r]) == kf; });
        }
        return m;
    }
    case T_IN_BITMAP: {
        // word d >> 5 of the bitmap comes from lane d >> 5 (byte address
        // (d >> 3) & 0xfc; rows with d >= 2048 read some word and fail the
        // range test)
        uint32_t entry;
        if constexpr (NT > 0) {
            entry = I.c == 0 ? tabs.e0 : I.c == 1 ? tabs.e1 : I.c == 2 ? tabs.e2 : tabs.e3;
        } else {
            entry = kpool[I.a + (threadIdx.x & 63u)];
        }
        const uint32_t lo = (uint32_t)I.b;
        if constexpr (NT > 0) {
            // kernels with the tables in registers run one wave per SIMD,
            // where nothing hides a read's latency: every row's cross-lane
            // read is issued before any is used, so the latencies overlap
            // (the batched kernel's other waves hide them, and it keeps
            // the registers this takes)
            uint32_t w[RPT];
#pragma unroll
            for (int r = 0; r < RPT; r++)
                w[r] = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(((x[r] - lo) >> 3) & 0xfcu), (int)entry);
            return bits_of<RPT>([&](int r) {
                const uint32_t d = x[r] - lo;
                return d < 2048u && ((w[r] >> (d & 31u)) & 1u);
            });
        }
        return bits_of<RPT>([&](int r) {
            const uint32_t d = x[r] - lo;
            const uint32_t w = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((d >> 3) & 0xfcu), (int)entry);
            return d < 2048u && ((w >> (d & 31u)) & 1u);
        });
    }
    case T_IN_HASH: {
        // Lane l holds table entry l; each row reads the entry of its slot
        // from that lane (the permute takes byte addresses, so the slot
        // field is cut out at bits 2..7).  Needs all 64 lanes active.
        uint32_t entry;
        if constexpr (NT > 0) {
            entry = I.c == 0 ? tabs.e0 : I.c == 1 ? tabs.e1 : I.c == 2 ? tabs.e2 : tabs.e3;
        } else {
            entry = kpool[I.a + (threadIdx.x & 63u)];
        }
        const uint32_t h = (uint32_t)I.b;
        auto lookup = [&](auto &&addr) {
            if constexpr (NT > 0) {
                uint32_t w[RPT];   // all reads in flight before the compares, as above
#pragma unroll
                for (int r = 0; r < RPT; r++) w[r] = (uint32_t)__builtin_amdgcn_ds_bpermute((int)addr(x[r]), (int)entry);
                return bits_of<RPT>([&](int r) { return w[r] == x[r]; });
            } else {
                return bits_of<RPT>(
                    [&](int r) { return (uint32_t)__builtin_amdgcn_ds_bpermute((int)addr(x[r]), (int)entry) == x[r]; });
            }
        };
        // byte address of the slot: a rotation's bits 2..7, or the top six
        // bits of the product with an odd multiplier
        if (h < 32u) return lookup([&](uint32_t v) { return __builtin_rotateright32(v, h) & 0xfcu; });
        return lookup([&](uint32_t v) { return ((v * h) >> 24) & 0xfcu; });
    }
    }
    return 0u;
}

template <int K, int RPT, int KK = (K > 0 ? K : 1)>
__device__ __forceinline__ void run_udf(const Insn &I, const uint32_t (&v)[KK][RPT], uint32_t (&u)[RPT])
{
    uint32_t o[RPT];
    if (I.flags & F_CONST) {
#pragma unroll
        for (int r = 0; r < RPT; r++) o[r] = (uint32_t)I.a;
    } else {
        for_slot<K>(I.src, [&](auto C) {
#pragma unroll
            for (int r = 0; r < RPT; r++) o[r] = v[C][r];
        });
    }
    switch (I.op) {
    case U_LOAD:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] = o[r];
        break;
    case U_ADD:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] += o[r];
        break;
    case U_SUB:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] -= o[r];
        break;
    case U_MUL:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] *= o[r];
        break;
    case U_MOD: {
        const int32_t m = I.a;   // > 0, checked by the compiler
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] = (uint32_t)((int32_t)u[r] % m);
        break;
    }
    case U_AND:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] &= o[r];
        break;
    case U_OR:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] |= o[r];
        break;
    case U_XOR:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] ^= o[r];
        break;
    case U_SHL:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] <<= (uint32_t)I.a;
        break;
    case U_SHR:
#pragma unroll
        for (int r = 0; r < RPT; r++) u[r] = (uint32_t)((int32_t)u[r] >> I.a);
        break;
    }
}

template <int K, int RPT, bool UDF, int NT, int KK = (K > 0 ? K : 1)>
__device__ __forceinline__ uint32_t run_program_tree(const Program &P, const uint32_t (&v)[KK][RPT], uint32_t valid,
                                                     const SlotTabs<NT> &tabs)
{
    uint32_t acc = valid, cm = 0;
    uint32_t u[UDF ? RPT : 1];
#pragma unroll
    for (int r = 0; r < (UDF ? RPT : 1); r++) u[r] = 0;
    const int n = P.ninsn;
    for (int i = 0; i < n; i++) {
        const Insn I = P.insn[i];
        uint32_t m = 0;
        bool on_udf = false;
        if constexpr (UDF) {
            if (I.op >= U_LOAD) {
                run_udf<K, RPT>(I, v, u);
                continue;
            }
            if (I.flags & F_SRC_UDF) {
                m = run_test<RPT, NT>(I, P.kpool, tabs, u);
                on_udf = true;
            }
        }
        if (!on_udf) {
            if (I.op == T_RANGE_I32) {
                const uint32_t lo = (uint32_t)I.a, span = (uint32_t)I.b;
                switch_slot<K>(I.src, [&](auto C) { m = bits_of<RPT>([&](int r) { return v[C][r] - lo <= span; }); });
            } else {
                switch_slot<K>(I.src, [&](auto C) { m = run_test<RPT, NT>(I, P.kpool, tabs, v[C]); });
            }
        }
        if (I.flags & F_SINGLE) {
            acc &= m;
        } else {
            cm |= m;
            if (I.flags & F_END_CLAUSE) { acc &= cm; cm = 0; }
        }
    }
    return acc;
}

// Runs the program on the loaded slots: returns valid & P(row) per row slot.
// UDF = false is the variant for programs without udf instructions (it does
// not reserve registers for the udf accumulator).  TREE = true dispatches
// on the slot with a switch and tests for the common int range first (the
// batched kernel, whose wave streams are dominated by the interpreter's
// scalar branches).
template <int K, int RPT, bool UDF = true, int NT = 0, bool TREE = false, int KK = (K > 0 ? K : 1)>
__device__ __forceinline__ uint32_t run_program(const Program &P, const uint32_t (&v)[KK][RPT], uint32_t valid,
                                                const SlotTabs<NT> &tabs = SlotTabs<NT>{})
{
    if constexpr (TREE) return run_program_tree<K, RPT, UDF, NT>(P, v, valid, tabs);
    uint32_t acc = valid, cm = 0;
    uint32_t u[UDF ? RPT : 1];
#pragma unroll
    for (int r = 0; r < (UDF ? RPT : 1); r++) u[r] = 0;
    const int n = P.ninsn;
    for (int i = 0; i < n; i++) {
        const Insn I = P.insn[i];
        uint32_t m = 0;
        if constexpr (UDF) {
            if (I.op >= U_LOAD) {
                run_udf<K, RPT>(I, v, u);
                continue;
            }
            if (I.flags & F_SRC_UDF) m = run_test<RPT, NT>(I, P.kpool, tabs, u);
            else for_slot<K>(I.src, [&](auto C) { m = run_test<RPT, NT>(I, P.kpool, tabs, v[C]); });
        } else {
            for_slot<K>(I.src, [&](auto C) { m = run_test<RPT, NT>(I, P.kpool, tabs, v[C]); });
        }
        if (I.flags & F_SINGLE) {
            acc &= m;
        } else {
            cm |= m;
            if (I.flags & F_END_CLAUSE) { acc &= cm; cm = 0; }
        }
    }
    return acc;
}

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Index of the wave in its block, as a wave-uniform (scalar) value: loops
// over wave tiles then run on the scalar unit instead of under exec masks.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Row of slot r of this lane in the wave tile starting at `base`.
__device__ __forceinline__ int64_t row_of(int64_t base, int r)
{
    return base + (int64_t)(r >> 2) * (4 * kWave) + lane_id() * 4 + (r & 3);
}

// Loads the K slot columns of the wave tile starting at row `base`; rows at
// or beyond n (only in the last tile) read as 0 and are masked by valid_bits.
template <int K, int RPT, int KK = (K > 0 ? K : 1)>
__device__ __forceinline__ void load_vals(const ColPtrs &cp, int64_t base, int64_t n, uint32_t (&v)[KK][RPT])
{
    constexpr int TILE = kWave * RPT;
    if (base + TILE <= n) {
#pragma unroll
        for (int j = 0; j < RPT / 4; j++) {
            const int64_t idx = base + (int64_t)j * (4 * kWave) + lane_id() * 4;
#pragma unroll
            for (int c = 0; c < K; c++) {
                const u32x4 *src = (const u32x4 *)(cp.p[c] + idx);
                const u32x4 q = cp.nt ? __builtin_nontemporal_load(src) : *src;
                v[c][4 * j + 0] = q.x;
                v[c][4 * j + 1] = q.y;
                v[c][4 * j + 2] = q.z;
                v[c][4 * j + 3] = q.w;
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < RPT; r++) {
            const int64_t row = row_of(base, r);
            const bool ok = row < n;
#pragma unroll
            for (int c = 0; c < K; c++) v[c][r] = ok ? cp.p[c][row] : 0u;
        }
    }
}

// Bits of the row slots of this lane that exist (all but in the last tile).
template <int RPT>
__device__ __forceinline__ uint32_t valid_bits(int64_t base, int64_t n)
{
    constexpr int TILE = kWave * RPT;
    if (base + TILE <= n) return all_rows<RPT>();
    return bits_of<RPT>([&](int r) { return row_of(base, r) < n; });
}

// Sum of a per-lane value over the wave.
// Sum of x over the 64 lanes of the wave, returned wave-uniform.  Two quad
// permutations and two rotations by 4 and 8 lanes within each row of 16
// (DPP operand modifiers: register moves, no LDS round trips) leave every
// lane with its row's sum; the four row sums are read from lanes 0, 16, 32
// and 48.  All 64 lanes must be active (every caller runs it under
// wave-uniform control flow).
__device__ __forceinline__ uint32_t wave_sum(uint32_t x)
{
    constexpr int kQuadSwapPairs = 0xB1;   // quad_perm [1, 0, 3, 2]
    constexpr int kQuadSwapHalves = 0x4E;  // quad_perm [2, 3, 0, 1]
    constexpr int kRowRor4 = 0x124, kRowRor8 = 0x128;
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kQuadSwapPairs, 0xF, 0xF, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kQuadSwapHalves, 0xF, 0xF, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kRowRor4, 0xF, 0xF, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kRowRor8, 0xF, 0xF, false);
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 0) + (uint32_t)__builtin_amdgcn_readlane((int)x, 16) +
           (uint32_t)__builtin_amdgcn_readlane((int)x, 32) + (uint32_t)__builtin_amdgcn_readlane((int)x, 48);
}

}  // namespace esc
