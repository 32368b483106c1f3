// esc_program.h -- the compiled, wave-uniform form of a selection predicate,
// shared by the host compiler and the gfx950 kernels.
//
// A predicate becomes an AND of OR-clauses over leaf tests.  The program is
// a flat instruction list executed identically by every lane (every branch
// depends only on the instruction, so it stays scalar): a test instruction
// turns the values of one column slot (or of the udf accumulator) into a
// 64-bit lane mask per row slot and ORs it into the open clause; a test
// flagged END_CLAUSE closes the clause by AND-ing it into the result.  udf
// instructions update a per-row int32 accumulator.  Columns are loaded
// once per tile into "slots" before the program runs.
#pragma once
#include <stdint.h>

namespace esc {

constexpr int kMaxSlots = 8;     // distinct columns per predicate
constexpr int kMaxInsns = 64;
constexpr int kMaxKpool = 256;   // IN constants per predicate
constexpr int kSlotTable = 64;   // entries of a slot table (one per lane)
constexpr int kMaxTables = kMaxKpool / kSlotTable;

enum Op : uint8_t {
    // tests (read slot `src`, or the udf accumulator when F_SRC_UDF)
    T_RANGE_I32 = 0,   // (uint32)(x - a) <= (uint32)b        a = lo, b = hi - lo
    T_RANGE_F32 = 1,   // fa <= x && x <= fb                  a, b = float bits
    T_IN_I32 = 2,      // x == kpool[a + i] for some i < b
    T_IN_F32 = 3,      // float ==, same layout
    T_BITSET = 4,      // d = (uint32)(x - a); d < 64 && bit d of (uint64)c<<32 | (uint32)b
    T_IN_HASH = 5,     // kpool[a + h(x)] == x bitwise, h(x) = (rotr(x, b) >> 2) & 63 for
                       // b < 32, else (x * b) >> 26 (b an odd multiplier >= 2^31): a
                       // 64-entry slot table whose keys occupy distinct slots (float
                       // lists hold both zeros and no NaN, so bit equality is float
                       // equality); table c of the program, a = 64 * c
    T_IN_BITMAP = 6,   // d = (uint32)(x - b); d < 2048 && bit (d & 31) of kpool[a + (d >> 5)]:
                       // a 64-word bitmap of int keys; table c, a = 64 * c
    // udf accumulator updates: operand = slot `src`, or constant a (F_CONST)
    U_LOAD = 16, U_ADD, U_SUB, U_MUL, U_MOD, U_AND, U_OR, U_XOR, U_SHL, U_SHR,
};

enum Flags : uint8_t {
    F_END_CLAUSE = 1,  // test closes its clause
    F_SRC_UDF = 2,     // test reads the udf accumulator
    F_CONST = 4,       // udf operand is the constant a
    F_SINGLE = 8,      // test is a whole clause by itself (AND straight into the result)
};

struct Insn {
    uint8_t op, src, flags, pad;
    int32_t a, b, c;
};
static_assert(sizeof(Insn) == 16, "Insn is 16 bytes");

enum ProgFlags : int32_t { P_ALWAYS_TRUE = 1, P_ALWAYS_FALSE = 2, P_HAS_UDF = 4 };

struct Program {
    int32_t ninsn;
    int32_t nslots;
    int32_t nk;
    int32_t flags;
    int32_t nclauses;
    int32_t ntables;   // slot tables, at kpool[0 .. 64 * ntables)
    int32_t pad[2];
    int32_t slot_col[kMaxSlots];   // table column of each slot
    Insn insn[kMaxInsns];
    uint32_t kpool[kMaxKpool];
};

}  // namespace esc
