// esc_device.h -- device-side evaluation of a compiled predicate program on
// a tile of rows held in registers (shared by the plain and batched scans).
//
// Tile layout: a block of kScanBlock threads covers kScanBlock*RPT rows; row
// slot r = 4*j + e of thread t is row base + (j*kScanBlock + t)*4 + e, so the
// j-th 16-byte load of every lane of a wave forms one coalesced 1 KiB request.
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

// Lane masks of one test, folded straight into the clause state: MODE 0 ORs
// into the open clause cm, MODE 1 (a one-leaf clause) ANDs into acc.
template <int MODE, int RPT, typename T>
__device__ __forceinline__ void fold(uint64_t (&acc)[RPT], uint64_t (&cm)[RPT], T &&test)
{
#pragma unroll
    for (int r = 0; r < RPT; r++) {
        const uint64_t m = __ballot(test(r));
        if (MODE == 0) cm[r] |= m;
        else acc[r] &= m;
    }
}

template <int MODE, int RPT>
__device__ __forceinline__ void run_test(const Insn &I, const uint32_t *kpool, const uint32_t (&x)[RPT],
                                         uint64_t (&acc)[RPT], uint64_t (&cm)[RPT])
{
    switch (I.op) {
    case T_RANGE_I32: {
        const uint32_t lo = (uint32_t)I.a, span = (uint32_t)I.b;
        fold<MODE>(acc, cm, [&](int r) { return x[r] - lo <= span; });
        break;
    }
    case T_RANGE_F32: {
        const float lo = as_f((uint32_t)I.a), hi = as_f((uint32_t)I.b);
        fold<MODE>(acc, cm, [&](int r) { const float f = as_f(x[r]); return lo <= f && f <= hi; });
        break;
    }
    case T_BITSET: {
        const uint32_t lo = (uint32_t)I.a;
        const uint64_t bits = (uint64_t)(uint32_t)I.b | ((uint64_t)(uint32_t)I.c << 32);
        fold<MODE>(acc, cm, [&](int r) {
            const uint32_t d = x[r] - lo;
            return d < 64u && ((bits >> (d & 63u)) & 1ull);
        });
        break;
    }
    case T_IN_I32:
    case T_IN_F32: {
        // OR over the set members into cm; a one-leaf clause (MODE 1) finds
        // cm empty on entry, uses it as scratch and leaves it empty
        const bool fl = I.op == T_IN_F32;
        for (int k = 0; k < I.b; k++) {
            const uint32_t kv = kpool[I.a + k];
            if (fl) {
                const float kf = as_f(kv);
#pragma unroll
                for (int r = 0; r < RPT; r++) cm[r] |= __ballot(as_f(x[r]) == kf);
            } else {
#pragma unroll
                for (int r = 0; r < RPT; r++) cm[r] |= __ballot(x[r] == kv);
            }
        }
        if (MODE == 1) {
#pragma unroll
            for (int r = 0; r < RPT; r++) { acc[r] &= cm[r]; cm[r] = 0; }
        }
        break;
    }
    default:
        if (MODE == 1) {
#pragma unroll
            for (int r = 0; r < RPT; r++) acc[r] = 0;
        }
    }
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

// Runs the program on the loaded slots; acc[r] enters as the mask of valid
// rows and leaves as the mask of qualifying rows.
template <int K, int RPT, int KK = (K > 0 ? K : 1)>
__device__ __forceinline__ void run_program(const Program &P, const uint32_t (&v)[KK][RPT], uint64_t (&acc)[RPT])
{
    uint64_t cm[RPT];
    uint32_t u[RPT];
#pragma unroll
    for (int r = 0; r < RPT; r++) { cm[r] = 0; u[r] = 0; }
    const int n = P.ninsn;
    for (int i = 0; i < n; i++) {
        const Insn I = P.insn[i];
        if (I.op >= U_LOAD) {
            run_udf<K, RPT>(I, v, u);
            continue;
        }
        const bool single = I.flags & F_SINGLE;
        if (I.flags & F_SRC_UDF) {
            if (single) run_test<1, RPT>(I, P.kpool, u, acc, cm);
            else run_test<0, RPT>(I, P.kpool, u, acc, cm);
        } else if (single) {
            for_slot<K>(I.src, [&](auto C) { run_test<1, RPT>(I, P.kpool, v[C], acc, cm); });
        } else {
            for_slot<K>(I.src, [&](auto C) { run_test<0, RPT>(I, P.kpool, v[C], acc, cm); });
        }
        if (!single && (I.flags & F_END_CLAUSE)) {
#pragma unroll
            for (int r = 0; r < RPT; r++) { acc[r] &= cm[r]; cm[r] = 0; }
        }
    }
}

// Row of slot r for this thread: base + (j*256 + tid)*4 + e with r = 4j + e.
__device__ __forceinline__ int64_t row_of(int64_t base, int r)
{
    return base + ((int64_t)(r >> 2) * kScanBlock + threadIdx.x) * 4 + (r & 3);
}

// Loads the K slot columns of the tile starting at row `base`; rows at or
// beyond n (only in the last tile) read as 0 and are masked by valid_masks.
template <int K, int RPT, int KK = (K > 0 ? K : 1)>
__device__ __forceinline__ void load_vals(const ColPtrs &cp, int64_t base, int64_t n, uint32_t (&v)[KK][RPT])
{
    constexpr int TILE = kScanBlock * RPT;
    if (base + TILE <= n) {
#pragma unroll
        for (int j = 0; j < RPT / 4; j++) {
            const int64_t idx = base + ((int64_t)j * kScanBlock + threadIdx.x) * 4;
#pragma unroll
            for (int c = 0; c < K; c++) {
                const u32x4 q = __builtin_nontemporal_load((const u32x4 *)(cp.p[c] + idx));
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

// Lane masks of the rows of the tile that exist (all ones except in the last tile).
template <int RPT>
__device__ __forceinline__ void valid_masks(int64_t base, int64_t n, uint64_t (&acc)[RPT])
{
    constexpr int TILE = kScanBlock * RPT;
    const bool full = base + TILE <= n;
#pragma unroll
    for (int r = 0; r < RPT; r++) acc[r] = full ? ~0ull : __ballot(row_of(base, r) < n);
}

// Qualifying rows of a loaded tile, as the count of set lane-mask bits.
template <int K, int RPT, int KK = (K > 0 ? K : 1)>
__device__ __forceinline__ uint32_t eval_count(const Program &P, const uint32_t (&v)[KK][RPT], int64_t base,
                                               int64_t n)
{
    uint64_t acc[RPT];
    valid_masks<RPT>(base, n, acc);
    run_program<K, RPT>(P, v, acc);
    uint32_t c = 0;
#pragma unroll
    for (int r = 0; r < RPT; r++) c += (uint32_t)__popcll(acc[r]);
    return c;
}

}  // namespace esc
