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

// Per-lane mask of a row test: bit r = test(r).
template <int RPT, typename T>
__device__ __forceinline__ uint32_t bits_of(T &&test)
{
    static_assert(RPT <= 32, "masks are 32-bit");
    uint32_t m = 0;
#pragma unroll
    for (int r = RPT - 1; r >= 0; r--) m = m + m + (test(r) ? 1u : 0u);
    return m;
}

template <int RPT>
__device__ __forceinline__ uint32_t all_rows()
{
    return RPT == 32 ? 0xffffffffu : ((1u << RPT) - 1u);
}

// Row-bit accumulation with add-with-carry (gfx950 VOP3 forms, carries in
// scalar register pairs).  A compare or subtraction writes one carry per row
// and an add-with-carry consumes it; four rows are interleaved so that every
// carry is read three instructions after the one that wrote it (the
// hardware requires two between a vector write of a scalar register and its
// use as a carry-in).  No vcc, no select, no wait states.

// m = 16 m + 8 [d3 > s] + 4 [d2 > s] + 2 [d1 > s] + [d0 > s] (unsigned), the
// borrows of s - d: bit set where a row lies outside the range.
__device__ __forceinline__ uint32_t shift_in_outside4(uint32_t m, uint32_t s, uint32_t d3, uint32_t d2, uint32_t d1,
                                                      uint32_t d0)
{
    uint32_t t0, t1, t2, t3;
    uint64_t c0, c1, c2, c3, co;
    asm("v_sub_co_u32_e64 %[t3], %[c3], %[s], %[d3]\n\t"
        "v_sub_co_u32_e64 %[t2], %[c2], %[s], %[d2]\n\t"
        "v_sub_co_u32_e64 %[t1], %[c1], %[s], %[d1]\n\t"
        "v_sub_co_u32_e64 %[t0], %[c0], %[s], %[d0]\n\t"
        "v_addc_co_u32_e64 %[m], %[co], %[m], %[m], %[c3]\n\t"
        "v_addc_co_u32_e64 %[m], %[co], %[m], %[m], %[c2]\n\t"
        "v_addc_co_u32_e64 %[m], %[co], %[m], %[m], %[c1]\n\t"
        "v_addc_co_u32_e64 %[m], %[co], %[m], %[m], %[c0]"
        : [m] "+v"(m), [t0] "=&v"(t0), [t1] "=&v"(t1), [t2] "=&v"(t2), [t3] "=&v"(t3), [c0] "=&s"(c0),
          [c1] "=&s"(c1), [c2] "=&s"(c2), [c3] "=&s"(c3), [co] "=&s"(co)
        : [s] "s"(s), [d0] "v"(d0), [d1] "v"(d1), [d2] "v"(d2), [d3] "v"(d3));
    return m;
}

// a_i += [x_i == k] for four rows (integer or float equality).
template <bool F32>
__device__ __forceinline__ void count_eq4(uint32_t &a0, uint32_t &a1, uint32_t &a2, uint32_t &a3, uint32_t k,
                                          uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3)
{
    uint64_t c0, c1, c2, c3, co;
    if constexpr (F32)
        asm("v_cmp_eq_f32_e64 %[c0], %[k], %[x0]\n\t"
            "v_cmp_eq_f32_e64 %[c1], %[k], %[x1]\n\t"
            "v_cmp_eq_f32_e64 %[c2], %[k], %[x2]\n\t"
            "v_cmp_eq_f32_e64 %[c3], %[k], %[x3]\n\t"
            "v_addc_co_u32_e64 %[a0], %[co], 0, %[a0], %[c0]\n\t"
            "v_addc_co_u32_e64 %[a1], %[co], 0, %[a1], %[c1]\n\t"
            "v_addc_co_u32_e64 %[a2], %[co], 0, %[a2], %[c2]\n\t"
            "v_addc_co_u32_e64 %[a3], %[co], 0, %[a3], %[c3]"
            : [a0] "+v"(a0), [a1] "+v"(a1), [a2] "+v"(a2), [a3] "+v"(a3), [c0] "=&s"(c0), [c1] "=&s"(c1),
              [c2] "=&s"(c2), [c3] "=&s"(c3), [co] "=&s"(co)
            : [k] "s"(k), [x0] "v"(x0), [x1] "v"(x1), [x2] "v"(x2), [x3] "v"(x3));
    else
        asm("v_cmp_eq_u32_e64 %[c0], %[k], %[x0]\n\t"
            "v_cmp_eq_u32_e64 %[c1], %[k], %[x1]\n\t"
            "v_cmp_eq_u32_e64 %[c2], %[k], %[x2]\n\t"
            "v_cmp_eq_u32_e64 %[c3], %[k], %[x3]\n\t"
            "v_addc_co_u32_e64 %[a0], %[co], 0, %[a0], %[c0]\n\t"
            "v_addc_co_u32_e64 %[a1], %[co], 0, %[a1], %[c1]\n\t"
            "v_addc_co_u32_e64 %[a2], %[co], 0, %[a2], %[c2]\n\t"
            "v_addc_co_u32_e64 %[a3], %[co], 0, %[a3], %[c3]"
            : [a0] "+v"(a0), [a1] "+v"(a1), [a2] "+v"(a2), [a3] "+v"(a3), [c0] "=&s"(c0), [c1] "=&s"(c1),
              [c2] "=&s"(c2), [c3] "=&s"(c3), [co] "=&s"(co)
            : [k] "s"(k), [x0] "v"(x0), [x1] "v"(x1), [x2] "v"(x2), [x3] "v"(x3));
}

// Set membership: per row the number of equal constants (duplicates in the
// list only raise it), then one bit per row.
template <int RPT, bool F32>
__device__ __forceinline__ uint32_t in_test(const Insn &I, const uint32_t *kpool, const uint32_t (&x)[RPT])
{
    uint32_t a[RPT];
#pragma unroll
    for (int r = 0; r < RPT; r++) a[r] = 0;
    for (int k = 0; k < I.b; k++) {
        const uint32_t kv = kpool[I.a + k];
#pragma unroll
        for (int g = 0; g < RPT; g += 4)
            count_eq4<F32>(a[g], a[g + 1], a[g + 2], a[g + 3], kv, x[g], x[g + 1], x[g + 2], x[g + 3]);
    }
    return bits_of<RPT>([&](int r) { return a[r] != 0u; });
}

template <int RPT>
__device__ __forceinline__ uint32_t run_test(const Insn &I, const uint32_t *kpool, const uint32_t (&x)[RPT])
{
    switch (I.op) {
    case T_RANGE_I32: {
        const uint32_t lo = (uint32_t)I.a, span = (uint32_t)I.b;
        static_assert(RPT % 4 == 0, "rows per lane come in fours");
        uint32_t outside = 0;
#pragma unroll
        for (int g = RPT - 4; g >= 0; g -= 4)
            outside = shift_in_outside4(outside, span, x[g + 3] - lo, x[g + 2] - lo, x[g + 1] - lo, x[g] - lo);
        return ~outside & all_rows<RPT>();
    }
    case T_RANGE_F32: {
        const float lo = as_f((uint32_t)I.a), hi = as_f((uint32_t)I.b);
        return bits_of<RPT>([&](int r) { const float f = as_f(x[r]); return lo <= f && f <= hi; });
    }
    case T_BITSET: {
        const uint32_t lo = (uint32_t)I.a;
        const uint64_t bits = (uint64_t)(uint32_t)I.b | ((uint64_t)(uint32_t)I.c << 32);
        return bits_of<RPT>([&](int r) {
            const uint32_t d = x[r] - lo;
            return d < 64u && ((bits >> (d & 63u)) & 1ull);
        });
    }
    case T_IN_I32:
        return in_test<RPT, false>(I, kpool, x);
    case T_IN_F32:
        return in_test<RPT, true>(I, kpool, x);
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

// Runs the program on the loaded slots: returns valid & P(row) per row slot.
// UDF = false is the variant for programs without udf instructions (it does
// not reserve registers for the udf accumulator).
template <int K, int RPT, bool UDF = true, int KK = (K > 0 ? K : 1)>
__device__ __forceinline__ uint32_t run_program(const Program &P, const uint32_t (&v)[KK][RPT], uint32_t valid)
{
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
            if (I.flags & F_SRC_UDF) m = run_test<RPT>(I, P.kpool, u);
            else for_slot<K>(I.src, [&](auto C) { m = run_test<RPT>(I, P.kpool, v[C]); });
        } else {
            for_slot<K>(I.src, [&](auto C) { m = run_test<RPT>(I, P.kpool, v[C]); });
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
__device__ __forceinline__ uint32_t wave_sum(uint32_t x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

}  // namespace esc
