// esc_compile.cpp -- error reporting, table descriptors and the predicate
// compiler (host only; needs no GPU).
//
// The compiler turns the pre-order esc_node tree of a selection (the
// predicate language of the paper's example selection, Section 1) into the
// wave-uniform esc::Program run by the scan kernels:
//   1. parse and validate the tree, type-check constants against columns;
//   2. normalise every leaf into one device test (int range, float range,
//      64-value bitmap, or a set), folding leaves whose value does not
//      depend on the row (always true / always false); sets of three or
//      more keys become slot tables when a 6-bit field of the value
//      separates the keys, else 2048-bit bitmaps when the int keys span
//      less than 2048 (one cross-lane read per row instead of one compare
//      per key);
//   3. convert to an AND of OR-clauses by distributing OR over AND -- exact
//      because the language has no negation;
//   4. give each referenced column a register slot and emit instructions.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <atomic>
#include <new>
#include <set>
#include <vector>

#include "esc_host.h"

namespace esc {

static thread_local char g_err[1024];

int fail(int status, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return status;
}

void clear_error() { g_err[0] = 0; }

uint64_t next_handle_id()
{
    static std::atomic<uint64_t> next{1};
    return next.fetch_add(1);
}

const char *last_error() { return g_err; }

namespace {

constexpr int kMaxNodes = 4096;
constexpr int kMaxDepth = 64;
constexpr int kMaxRawIn = 4096;

enum LeafKind { L_TRUE, L_FALSE, L_TEST };

struct Leaf {
    LeafKind kind = L_TEST;
    Insn test{};                 // op, a, b, c; src = table column (col leaves)
    bool udf = false;
    std::vector<Insn> uops;      // src = table column for column operands
    std::vector<uint32_t> kvals; // IN constants
};

using Clause = std::vector<int>;   // indices into leaves, sorted, unique
using Cnf = std::vector<Clause>;   // empty = TRUE; contains {} = FALSE

struct Ctx {
    const esc_table *schema;
    const esc_node *nodes;
    int nnodes;
    const esc_const *consts;
    int nconsts;
    const esc_udf_insn *udf;
    int nudf;
    std::vector<Leaf> leaves;
};

uint32_t fbits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
float bitsf(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

// the float just below x (x not NaN, not -inf), over IEEE-754 binary32
uint32_t next_down(float x)
{
    if (x == 0.0f) return 0x80000001u;
    uint32_t b = fbits(x);
    return (b >> 31) ? b + 1 : b - 1;
}

// the float just above x (x not NaN, not +inf)
uint32_t next_up(float x)
{
    if (x == 0.0f) return 0x00000001u;
    uint32_t b = fbits(x);
    return (b >> 31) ? b - 1 : b + 1;
}

int int_range(int64_t lo, int64_t hi, Leaf &L)
{
    if (lo > hi) { L.kind = L_FALSE; return ESC_OK; }
    if (lo <= INT32_MIN && hi >= INT32_MAX) { L.kind = L_TRUE; return ESC_OK; }
    L.kind = L_TEST;
    L.test.op = T_RANGE_I32;
    L.test.a = (int32_t)lo;
    L.test.b = (int32_t)(uint32_t)((uint32_t)(int32_t)hi - (uint32_t)(int32_t)lo);
    return ESC_OK;
}

int int_set(std::vector<int32_t> v, Leaf &L)
{
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    int64_t lo = v.front(), hi = v.back();
    if (hi - lo + 1 == (int64_t)v.size()) return int_range(lo, hi, L);
    L.kind = L_TEST;
    if (hi - lo < 64) {
        uint64_t bits = 0;
        for (int32_t x : v) bits |= 1ull << (uint64_t)((int64_t)x - lo);
        L.test.op = T_BITSET;
        L.test.a = (int32_t)lo;
        L.test.b = (int32_t)(uint32_t)bits;
        L.test.c = (int32_t)(uint32_t)(bits >> 32);
        return ESC_OK;
    }
    if ((int)v.size() > ESC_MAX_IN)
        return fail(ESC_ERR_UNSUPPORTED, "IN-list has %zu distinct constants (max %d)", v.size(), ESC_MAX_IN);
    L.test.op = T_IN_I32;
    for (int32_t x : v) L.kvals.push_back((uint32_t)x);
    return ESC_OK;
}

// ---- slot tables for IN-lists (op T_IN_HASH)

// Slot of key k under hash h: for h < 32, bits [h+2, h+8) of k taken
// cyclically (k rotated right by h); for an odd multiplier h >= 2^31, the
// top six bits of the 32-bit product k * h (multiplicative hashing).
int slot_of_key(uint32_t k, uint32_t h)
{
    if (h >= 32u) return (int)((k * h) >> 26);
    const uint32_t rot = h ? (k >> h) | (k << (32 - h)) : k;
    return (int)((rot >> 2) & 63u);
}

// The i-th candidate multiplier: odd (a bijection on 32-bit keys) with the
// top bit set (so that it cannot be read as a rotation).
uint32_t slot_multiplier(int i)
{
    return (0x9E3779B1u * (uint32_t)(2 * i + 1)) | 0x80000001u;
}

// The bit patterns a slot table must hold: the constants, plus -0.0 beside
// +0.0 for a float list (float equality treats the zeros as one value;
// NaN constants were already dropped).
std::vector<uint32_t> slot_keys(const Leaf &L)
{
    std::vector<uint32_t> keys = L.kvals;
    if (L.test.op == T_IN_F32)
        for (uint32_t k : L.kvals)
            if (k == 0u) keys.push_back(0x80000000u);
    return keys;
}

// Whether hash h puts every key in a slot of its own.
bool separates(const std::vector<uint32_t> &keys, uint32_t h)
{
    uint64_t used = 0;
    for (uint32_t k : keys) {
        const uint64_t bit = 1ull << slot_of_key(k, h);
        if (used & bit) return false;
        used |= bit;
    }
    return true;
}

// First rotation whose slots separate the keys, or -1.
int64_t slot_rotation(const std::vector<uint32_t> &keys)
{
    if (keys.empty() || keys.size() > (size_t)kSlotTable) return -1;
    for (uint32_t r = 0; r < 32; r++)
        if (separates(keys, r)) return r;
    return -1;
}

// First of kSlotMultipliers multipliers whose slots separate the keys, or -1
// (for keys that differ only in bits no 6-bit window holds together).  The
// product is a quarter-rate integer multiply per row, so lists of fewer than
// kMultiplierMin keys stay compare lists.
constexpr int kSlotMultipliers = 64;
constexpr int kMultiplierMin = 8;
int64_t slot_multiplier_for(const std::vector<uint32_t> &keys)
{
    if (keys.size() < (size_t)kMultiplierMin || keys.size() > (size_t)kSlotTable) return -1;
    for (int i = 0; i < kSlotMultipliers; i++)
        if (separates(keys, slot_multiplier(i))) return slot_multiplier(i);
    return -1;
}

// Whether conjuncts on one column are intersected at compile time
// (ESC_SIMPLIFY=0 turns it off, for comparisons).
bool simplify_enabled()
{
    const char *e = getenv("ESC_SIMPLIFY");
    return !(e && atoi(e) == 0);
}

// Smallest IN-list compiled to a slot table (ESC_IN_HASH_MIN; 0 = never).
// A list of n keys costs n compare-and-pack steps per row; a table lookup
// costs about two such steps plus one cross-lane read.
int in_hash_min()
{
    const char *e = getenv("ESC_IN_HASH_MIN");
    if (!e || !*e) return 3;
    return atoi(e);
}

// an int32 comparison (EQ/LT/GT/BETWEEN/IN) with constants ks
int int_test(int op, const std::vector<int32_t> &ks, Leaf &L)
{
    switch (op) {
    case ESC_EQ: return int_range(ks[0], ks[0], L);
    case ESC_LT: return int_range(INT32_MIN, (int64_t)ks[0] - 1, L);
    case ESC_GT: return int_range((int64_t)ks[0] + 1, INT32_MAX, L);
    case ESC_BETWEEN: return int_range(ks[0], ks[1], L);
    case ESC_IN: return int_set(ks, L);
    }
    return fail(ESC_ERR_INVALID, "bad comparison op %d", op);
}

int float_range(float lo, float hi, Leaf &L)
{
    if (isnan(lo) || isnan(hi) || lo > hi) { L.kind = L_FALSE; return ESC_OK; }
    L.kind = L_TEST;
    L.test.op = T_RANGE_F32;
    L.test.a = (int32_t)fbits(lo);
    L.test.b = (int32_t)fbits(hi);
    return ESC_OK;
}

int float_test(int op, const std::vector<float> &ks, Leaf &L)
{
    const float inf = INFINITY;
    switch (op) {
    case ESC_EQ: return float_range(ks[0], ks[0], L);
    case ESC_LT:
        if (isnan(ks[0]) || ks[0] == -inf) { L.kind = L_FALSE; return ESC_OK; }
        return float_range(-inf, bitsf(next_down(ks[0])), L);
    case ESC_GT:
        if (isnan(ks[0]) || ks[0] == inf) { L.kind = L_FALSE; return ESC_OK; }
        return float_range(bitsf(next_up(ks[0])), inf, L);
    case ESC_BETWEEN: return float_range(ks[0], ks[1], L);
    case ESC_IN: {
        std::vector<float> v;
        for (float k : ks) {
            if (isnan(k)) continue;
            float c = (k == 0.0f) ? 0.0f : k;   // -0 and +0 are the same member
            bool seen = false;
            for (float x : v) seen = seen || fbits(x) == fbits(c);
            if (!seen) v.push_back(c);
        }
        if (v.empty()) { L.kind = L_FALSE; return ESC_OK; }
        if (v.size() == 1) return float_range(v[0], v[0], L);
        if ((int)v.size() > ESC_MAX_IN)
            return fail(ESC_ERR_UNSUPPORTED, "IN-list has %zu distinct constants (max %d)", v.size(), ESC_MAX_IN);
        L.kind = L_TEST;
        L.test.op = T_IN_F32;
        for (float x : v) L.kvals.push_back(fbits(x));
        return ESC_OK;
    }
    }
    return fail(ESC_ERR_INVALID, "bad comparison op %d", op);
}

// gather the constants of a comparison node; `want` = required dtype
int gather_consts(Ctx &C, const esc_node &n, int op, int want, std::vector<uint32_t> &out)
{
    auto get = [&](int idx, uint32_t &v) -> int {
        if (idx < 0 || idx >= C.nconsts) return fail(ESC_ERR_INVALID, "constant index %d out of range", idx);
        if (C.consts[idx].dtype != want)
            return fail(ESC_ERR_TYPE, "constant %d has dtype %d, column needs %d", idx, C.consts[idx].dtype, want);
        v = C.consts[idx].v.bits;
        return ESC_OK;
    };
    uint32_t v;
    int rc;
    switch (op) {
    case ESC_EQ: case ESC_LT: case ESC_GT:
        if ((rc = get(n.k0, v))) return rc;
        out.push_back(v);
        return ESC_OK;
    case ESC_BETWEEN:
        if ((rc = get(n.k0, v))) return rc;
        out.push_back(v);
        if ((rc = get(n.k1, v))) return rc;
        out.push_back(v);
        return ESC_OK;
    case ESC_IN:
        if (n.k1 <= 0) return fail(ESC_ERR_INVALID, "empty IN-list");
        if (n.k1 > kMaxRawIn) return fail(ESC_ERR_UNSUPPORTED, "IN-list longer than %d", kMaxRawIn);
        if (n.k0 < 0 || (int64_t)n.k0 + n.k1 > C.nconsts) return fail(ESC_ERR_INVALID, "IN-list constants out of range");
        for (int i = 0; i < n.k1; i++) {
            if ((rc = get(n.k0 + i, v))) return rc;
            out.push_back(v);
        }
        return ESC_OK;
    }
    return fail(ESC_ERR_INVALID, "comparison op %d is not EQ/LT/GT/BETWEEN/IN", op);
}

int is_int_dtype(int d) { return d == ESC_INT32 || d == ESC_DATE32; }

int lower_udf(Ctx &C, const esc_node &n, Leaf &L)
{
    if (n.u1 <= 0 || n.u0 < 0 || (int64_t)n.u0 + n.u1 > C.nudf)
        return fail(ESC_ERR_INVALID, "udf program range [%d, +%d) out of range", n.u0, n.u1);
    const int ncols = (int)C.schema->dtypes.size();
    for (int i = 0; i < n.u1; i++) {
        const esc_udf_insn &u = C.udf[n.u0 + i];
        if ((i == 0) != (u.op == ESC_U_LOAD))
            return fail(ESC_ERR_INVALID, "udf must start with LOAD and use it only first");
        if (u.op < ESC_U_LOAD || u.op > ESC_U_SHR) return fail(ESC_ERR_INVALID, "bad udf op %d", u.op);
        Insn in{};
        in.op = (uint8_t)(U_LOAD + u.op);
        if (u.src == ESC_U_COL) {
            if (u.arg < 0 || u.arg >= ncols) return fail(ESC_ERR_INVALID, "udf column %d out of range", u.arg);
            if (!is_int_dtype(C.schema->dtypes[u.arg]))
                return fail(ESC_ERR_TYPE, "udf reads float32 column %d", u.arg);
            if (u.op == ESC_U_MOD || u.op == ESC_U_SHL || u.op == ESC_U_SHR)
                return fail(ESC_ERR_INVALID, "udf mod/shift needs a constant operand");
            in.src = (uint8_t)u.arg;   // table column for now; mapped to a slot later
        } else if (u.src == ESC_U_CONST) {
            if (u.op == ESC_U_MOD && u.arg <= 0) return fail(ESC_ERR_INVALID, "udf modulus %d is not positive", u.arg);
            if ((u.op == ESC_U_SHL || u.op == ESC_U_SHR) && (u.arg < 0 || u.arg > 31))
                return fail(ESC_ERR_INVALID, "udf shift %d outside [0,31]", u.arg);
            in.flags = F_CONST;
            in.a = u.arg;
        } else {
            return fail(ESC_ERR_INVALID, "bad udf operand kind %d", u.src);
        }
        L.uops.push_back(in);
    }
    std::vector<uint32_t> raw;
    int rc = gather_consts(C, n, n.cmp, ESC_INT32, raw);
    if (rc) return rc;
    std::vector<int32_t> ks(raw.begin(), raw.end());
    if ((rc = int_test(n.cmp, ks, L))) return rc;
    L.udf = true;
    L.test.flags |= F_SRC_UDF;
    return ESC_OK;
}

int lower_leaf(Ctx &C, const esc_node &n, Leaf &L)
{
    if (n.op == ESC_UDF) return lower_udf(C, n, L);
    const int ncols = (int)C.schema->dtypes.size();
    if (n.col < 0 || n.col >= ncols) return fail(ESC_ERR_INVALID, "column %d out of range", n.col);
    int dt = C.schema->dtypes[n.col];
    std::vector<uint32_t> raw;
    int rc = gather_consts(C, n, n.op, dt, raw);
    if (rc) return rc;
    if (dt == ESC_FLOAT32) {
        std::vector<float> ks;
        for (uint32_t b : raw) ks.push_back(bitsf(b));
        rc = float_test(n.op, ks, L);
    } else {
        std::vector<int32_t> ks(raw.begin(), raw.end());
        rc = int_test(n.op, ks, L);
    }
    if (rc) return rc;
    L.test.src = (uint8_t)n.col;
    return ESC_OK;
}

Clause merge(const Clause &a, const Clause &b)
{
    Clause c(a);
    c.insert(c.end(), b.begin(), b.end());
    std::sort(c.begin(), c.end());
    c.erase(std::unique(c.begin(), c.end()), c.end());
    return c;
}

// recursive descent over the pre-order array; returns the CNF of the subtree
int to_cnf(Ctx &C, int &pos, int depth, Cnf &out)
{
    if (depth > kMaxDepth) return fail(ESC_ERR_UNSUPPORTED, "predicate nested deeper than %d", kMaxDepth);
    if (pos >= C.nnodes) return fail(ESC_ERR_INVALID, "node array ends inside a subtree");
    const esc_node &n = C.nodes[pos++];
    if (n.op == ESC_AND || n.op == ESC_OR) {
        if (n.nchild <= 0) return fail(ESC_ERR_INVALID, "AND/OR node with %d children", n.nchild);
        for (int i = 0; i < n.nchild; i++) {
            Cnf k;
            int rc = to_cnf(C, pos, depth + 1, k);
            if (rc) return rc;
            if (i == 0) { out.swap(k); continue; }
            if (n.op == ESC_AND) {
                out.insert(out.end(), k.begin(), k.end());
            } else {
                if (out.size() * k.size() > (size_t)ESC_MAX_CLAUSES * 4)
                    return fail(ESC_ERR_UNSUPPORTED, "OR distributes into more than %d clauses", ESC_MAX_CLAUSES);
                Cnf prod;
                for (auto &a : out)
                    for (auto &b : k) prod.push_back(merge(a, b));
                out.swap(prod);
            }
            if (out.size() > (size_t)ESC_MAX_CLAUSES * 4)
                return fail(ESC_ERR_UNSUPPORTED, "predicate has more than %d clauses", ESC_MAX_CLAUSES);
        }
        return ESC_OK;
    }
    if (n.op < ESC_EQ || n.op > ESC_UDF) return fail(ESC_ERR_INVALID, "bad node op %d", n.op);
    if (n.nchild != 0) return fail(ESC_ERR_INVALID, "leaf node with children");
    Leaf L;
    int rc = lower_leaf(C, n, L);
    if (rc) return rc;
    if (L.kind == L_TRUE) { out.clear(); return ESC_OK; }
    if (L.kind == L_FALSE) { out.assign(1, Clause{}); return ESC_OK; }
    C.leaves.push_back(L);
    out.assign(1, Clause{(int)C.leaves.size() - 1});
    return ESC_OK;
}

// ---- conjunct simplification
//
// The value set a non-udf leaf accepts on its column: an int or float
// interval, or a finite set of ints or floats (float sets hold no NaN and
// one zero, +0).
struct ValSet {
    bool fl = false, set = false;
    int64_t lo = INT32_MIN, hi = INT32_MAX;   // int interval
    float flo = -INFINITY, fhi = INFINITY;    // float interval (compared as floats: -0 == +0)
    std::vector<int64_t> iv;                  // int set, sorted, unique
    std::vector<float> fv;                    // float set
};

bool value_set(const Leaf &L, ValSet &V)
{
    if (L.udf || L.kind != L_TEST) return false;
    const Insn &t = L.test;
    V = ValSet{};
    switch (t.op) {
    case T_RANGE_I32: V.lo = t.a; V.hi = (int64_t)t.a + (uint32_t)t.b; return true;
    case T_BITSET: {
        const uint64_t bits = ((uint64_t)(uint32_t)t.c << 32) | (uint32_t)t.b;
        V.set = true;
        for (int i = 0; i < 64; i++)
            if ((bits >> i) & 1u) V.iv.push_back((int64_t)t.a + i);
        return true;
    }
    case T_IN_I32:
        V.set = true;
        for (uint32_t k : L.kvals) V.iv.push_back((int32_t)k);
        std::sort(V.iv.begin(), V.iv.end());
        return true;
    case T_RANGE_F32: V.fl = true; V.flo = bitsf((uint32_t)t.a); V.fhi = bitsf((uint32_t)t.b); return true;
    case T_IN_F32:
        V.fl = V.set = true;
        for (uint32_t k : L.kvals) V.fv.push_back(bitsf(k));
        return true;
    }
    return false;
}

bool contains(const ValSet &V, int64_t x) { return V.set ? std::binary_search(V.iv.begin(), V.iv.end(), x) : V.lo <= x && x <= V.hi; }
bool contains(const ValSet &V, float x)
{
    if (!V.set) return V.flo <= x && x <= V.fhi;
    for (float y : V.fv)
        if (y == x) return true;
    return false;
}

// a ∩ b (same column, same kind of values)
ValSet intersect(const ValSet &a, const ValSet &b)
{
    ValSet r;
    r.fl = a.fl;
    if (!a.set && !b.set) {
        r.lo = std::max(a.lo, b.lo);
        r.hi = std::min(a.hi, b.hi);
        r.flo = std::max(a.flo, b.flo);
        r.fhi = std::min(a.fhi, b.fhi);
        return r;
    }
    const ValSet &s = a.set ? a : b, &o = a.set ? b : a;
    r.set = true;
    if (r.fl) {
        for (float x : s.fv)
            if (contains(o, x)) r.fv.push_back(x);
    } else {
        for (int64_t x : s.iv)
            if (contains(o, x)) r.iv.push_back(x);
    }
    return r;
}

bool empty(const ValSet &V)
{
    if (V.set) return V.fl ? V.fv.empty() : V.iv.empty();
    return V.fl ? !(V.flo <= V.fhi) : V.lo > V.hi;
}

// every value a accepts is accepted by b
bool subset(const ValSet &a, const ValSet &b)
{
    if (a.set) {
        if (a.fl) {
            for (float x : a.fv)
                if (!contains(b, x)) return false;
        } else {
            for (int64_t x : a.iv)
                if (!contains(b, x)) return false;
        }
        return true;
    }
    if (b.set) return false;   // an interval inside a finite set: not checked
    return a.fl ? (b.flo <= a.flo && a.fhi <= b.fhi) : (b.lo <= a.lo && a.hi <= b.hi);
}

// a leaf testing V on column col (kind L_FALSE when V is empty)
int leaf_of(const ValSet &V, int col, Leaf &L)
{
    L = Leaf{};
    int rc;
    if (V.fl) {
        rc = V.set ? float_test(ESC_IN, V.fv, L) : float_range(V.flo, V.fhi, L);
    } else if (V.set) {
        if (V.iv.empty()) { L.kind = L_FALSE; return ESC_OK; }
        rc = int_set(std::vector<int32_t>(V.iv.begin(), V.iv.end()), L);
    } else {
        rc = int_range(V.lo, V.hi, L);
    }
    L.test.src = (uint8_t)col;
    return rc;
}

// Within the AND of the CNF, the single-leaf clauses on one column are
// replaced by one leaf testing their intersection (empty: the predicate is
// false); then each multi-leaf clause loses the leaves that no value
// allowed on their column can satisfy, and is dropped when one of its
// leaves holds for every such value.  Exact: every step keeps the set of
// rows the conjunction accepts.
int simplify_units(Ctx &C, Cnf &cnf)
{
    std::map<int, ValSet> unit;          // column -> allowed values
    std::map<int, std::vector<int>> members;
    for (auto &c : cnf) {
        if (c.size() != 1) continue;
        ValSet V;
        if (!value_set(C.leaves[c[0]], V)) continue;
        const int col = C.leaves[c[0]].test.src;
        auto it = unit.find(col);
        unit[col] = it == unit.end() ? V : intersect(it->second, V);
        members[col].push_back(c[0]);
    }
    Cnf out;
    for (auto &[col, V] : unit) {
        if (empty(V)) { cnf.assign(1, Clause{}); return ESC_OK; }
        if (members[col].size() == 1) { out.push_back(Clause{members[col][0]}); continue; }
        Leaf L;
        int rc = leaf_of(V, col, L);
        if (rc) return rc;
        if (L.kind == L_FALSE) { cnf.assign(1, Clause{}); return ESC_OK; }
        if (L.kind == L_TRUE) continue;
        C.leaves.push_back(L);
        out.push_back(Clause{(int)C.leaves.size() - 1});
    }
    for (auto &c : cnf) {
        if (c.size() == 1) {
            ValSet V;
            if (value_set(C.leaves[c[0]], V)) continue;   // folded above
            out.push_back(c);
            continue;
        }
        Clause kept;
        bool holds = false;
        for (int li : c) {
            ValSet V;
            if (!value_set(C.leaves[li], V)) { kept.push_back(li); continue; }
            auto it = unit.find(C.leaves[li].test.src);
            if (it == unit.end()) { kept.push_back(li); continue; }
            if (empty(intersect(it->second, V))) continue;   // never true here
            if (subset(it->second, V)) { holds = true; break; }
            kept.push_back(li);
        }
        if (holds) continue;
        if (kept.empty()) { cnf.assign(1, Clause{}); return ESC_OK; }
        out.push_back(kept);
    }
    std::sort(out.begin(), out.end());
    out.erase(std::unique(out.begin(), out.end()), out.end());
    cnf.swap(out);
    return ESC_OK;
}

}  // namespace

int compile(const esc_table *schema, const esc_node *nodes, int nnodes, const esc_const *consts,
            int nconsts, const esc_udf_insn *udf, int nudf, esc_pred *p)
{
    if (!schema || !nodes || nnodes <= 0) return fail(ESC_ERR_INVALID, "null schema or empty node array");
    if (nnodes > kMaxNodes) return fail(ESC_ERR_UNSUPPORTED, "more than %d nodes", kMaxNodes);
    if (nconsts < 0 || (nconsts > 0 && !consts)) return fail(ESC_ERR_INVALID, "bad constant array");
    if (nudf < 0 || (nudf > 0 && !udf)) return fail(ESC_ERR_INVALID, "bad udf array");
    Ctx C{schema, nodes, nnodes, consts, nconsts, udf, nudf, {}};
    Cnf cnf;
    int pos = 0;
    int rc = to_cnf(C, pos, 0, cnf);
    if (rc) return rc;
    if (pos != nnodes) return fail(ESC_ERR_INVALID, "%d trailing nodes after the root's subtree", nnodes - pos);

    // drop duplicate clauses; an empty clause makes the whole predicate false
    std::sort(cnf.begin(), cnf.end());
    cnf.erase(std::unique(cnf.begin(), cnf.end()), cnf.end());
    Program &P = p->prog;
    memset(&P, 0, sizeof P);
    p->nhashed = 0;
    bool is_false = false;
    for (auto &c : cnf) is_false = is_false || c.empty();
    if (!is_false && simplify_enabled()) {
        if ((rc = simplify_units(C, cnf))) return rc;
        for (auto &c : cnf) is_false = is_false || c.empty();
    }
    if (is_false) { P.flags = P_ALWAYS_FALSE; return ESC_OK; }
    if (cnf.empty()) { P.flags = P_ALWAYS_TRUE; return ESC_OK; }
    if (cnf.size() > (size_t)ESC_MAX_CLAUSES)
        return fail(ESC_ERR_UNSUPPORTED, "predicate has %zu clauses (max %d)", cnf.size(), ESC_MAX_CLAUSES);

    // slots: the distinct columns read, in order of first use
    int slot_of[64];
    std::vector<int> col_of_slot;
    for (int i = 0; i < 64; i++) slot_of[i] = -1;
    auto use = [&](int col) -> int {
        if (col >= 64) return fail(ESC_ERR_UNSUPPORTED, "column %d beyond 64", col);
        if (slot_of[col] < 0) {
            if ((int)col_of_slot.size() == kMaxSlots)
                return fail(ESC_ERR_UNSUPPORTED, "predicate reads more than %d columns", kMaxSlots);
            slot_of[col] = (int)col_of_slot.size();
            col_of_slot.push_back(col);
        }
        return ESC_OK;
    };
    for (auto &c : cnf)
        for (int li : c) {
            const Leaf &L = C.leaves[li];
            if (L.udf) {
                for (auto &u : L.uops)
                    if (!(u.flags & F_CONST) && (rc = use(u.src))) return rc;
            } else if ((rc = use(L.test.src))) {
                return rc;
            }
        }

    // IN-lists: each distinct leaf stores its constants once.  Lists of at
    // least in_hash_min() keys become 64-entry slot tables when a slot field
    // separates their keys, largest lists first, as long as all IN-lists
    // still fit the constant pool.
    std::vector<int> in_leaves;
    {
        std::vector<char> seen(C.leaves.size(), 0);
        for (auto &c : cnf)
            for (int li : c) {
                const Insn &t = C.leaves[li].test;
                if ((t.op == T_IN_I32 || t.op == T_IN_F32) && !seen[li]) {
                    seen[li] = 1;
                    in_leaves.push_back(li);
                }
            }
    }
    int need = 0;
    for (int li : in_leaves) need += (int)C.leaves[li].kvals.size();
    if (need > kMaxKpool) return fail(ESC_ERR_UNSUPPORTED, "predicate has more than %d IN constants", kMaxKpool);
    std::vector<int64_t> hash_of(C.leaves.size(), -1);
    std::vector<int> table_of(C.leaves.size(), -1);
    std::vector<int32_t> bitmap_lo(C.leaves.size(), 0);
    int ntables = 0;
    {
        const int hmin = in_hash_min();
        std::vector<int> order = in_leaves;
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return C.leaves[x].kvals.size() > C.leaves[y].kvals.size(); });
        for (int li : order) {
            const Leaf &L = C.leaves[li];
            const int n = (int)L.kvals.size();
            if (hmin <= 0 || n < hmin || need + (kSlotTable - n) > kMaxKpool) continue;
            const std::vector<uint32_t> keys = slot_keys(L);
            const bool bitmap_fits =
                L.test.op == T_IN_I32 && (int64_t)(int32_t)L.kvals.back() - (int32_t)L.kvals.front() < 32 * kSlotTable;
            // a rotation (two ops per row), else a bitmap, else a multiplier
            int64_t h = slot_rotation(keys);
            if (h < 0 && !bitmap_fits) h = slot_multiplier_for(keys);
            uint32_t *tab = P.kpool + kSlotTable * ntables;
            if (h >= 0) {
                // every entry holds some key, so an entry equal to x means x is a key
                hash_of[li] = h;
                for (int e = 0; e < kSlotTable; e++) tab[e] = keys[0];
                for (uint32_t k : keys) tab[slot_of_key(k, (uint32_t)h)] = k;
            } else if (bitmap_fits) {
                // int keys within 2048 of the smallest: a bitmap, 32 bits per entry
                bitmap_lo[li] = (int32_t)L.kvals.front();
                for (int e = 0; e < kSlotTable; e++) tab[e] = 0u;
                for (uint32_t k : L.kvals) {
                    const uint32_t d = k - (uint32_t)bitmap_lo[li];
                    tab[d >> 5] |= 1u << (d & 31u);
                }
            } else {
                continue;
            }
            table_of[li] = ntables;
            ntables++;
            need += kSlotTable - n;
        }
    }
    P.ntables = ntables;
    p->nhashed = ntables;

    // emit
    int ni = 0, nk = kSlotTable * ntables;
    std::vector<int> kpool_at(C.leaves.size(), -1);
    auto emit = [&](Insn in) -> int {
        if (ni == kMaxInsns) return fail(ESC_ERR_UNSUPPORTED, "predicate needs more than %d instructions", kMaxInsns);
        P.insn[ni++] = in;
        return ESC_OK;
    };
    for (auto &c : cnf) {
        for (size_t j = 0; j < c.size(); j++) {
            const int li = c[j];
            const Leaf &L = C.leaves[li];
            if (L.udf) P.flags |= P_HAS_UDF;
            if (L.udf)
                for (Insn u : L.uops) {
                    if (!(u.flags & F_CONST)) u.src = (uint8_t)slot_of[u.src];
                    if ((rc = emit(u))) return rc;
                }
            Insn t = L.test;
            if (!L.udf) t.src = (uint8_t)slot_of[t.src];
            if (table_of[li] >= 0) {
                t.op = hash_of[li] >= 0 ? T_IN_HASH : T_IN_BITMAP;
                t.a = kSlotTable * table_of[li];
                t.b = hash_of[li] >= 0 ? (int32_t)(uint32_t)hash_of[li] : bitmap_lo[li];
                t.c = table_of[li];
            } else if (t.op == T_IN_I32 || t.op == T_IN_F32) {
                if (kpool_at[li] < 0) {
                    kpool_at[li] = nk;
                    for (uint32_t k : L.kvals) P.kpool[nk++] = k;
                }
                t.a = kpool_at[li];
                t.b = (int32_t)L.kvals.size();
            }
            if (j + 1 == c.size()) t.flags |= F_END_CLAUSE;
            if (c.size() == 1) t.flags |= F_SINGLE;
            if ((rc = emit(t))) return rc;
        }
    }
    P.ninsn = ni;
    P.nk = nk;
    P.nslots = (int32_t)col_of_slot.size();
    P.nclauses = (int32_t)cnf.size();
    for (size_t s = 0; s < col_of_slot.size(); s++) {
        P.slot_col[s] = col_of_slot[s];
        p->col_mask |= 1ull << col_of_slot[s];
    }
    return ESC_OK;
}

// Number of nodes of the pre-order subtree starting at pos (0 on a malformed
// array; the tree was validated when the predicate was compiled).
static int subtree_size(const std::vector<esc_node> &nodes, int pos)
{
    if (pos >= (int)nodes.size()) return 0;
    const esc_node &n = nodes[pos];
    int size = 1;
    if (n.op == ESC_AND || n.op == ESC_OR)
        for (int i = 0; i < n.nchild; i++) {
            const int k = subtree_size(nodes, pos + size);
            if (k == 0) return 0;
            size += k;
        }
    return size;
}

int split_conjuncts(const esc_pred *p, std::vector<Program> &out, int &nslots, int *slot_col)
{
    out.clear();
    esc_table schema;
    schema.dtypes = p->schema_dtypes;
    std::vector<std::pair<int, int>> parts;   // [start, size) of each top-level conjunct
    const esc_node &root = p->nodes[0];
    if (root.op == ESC_AND) {
        int pos = 1;
        for (int i = 0; i < root.nchild; i++) {
            const int k = subtree_size(p->nodes, pos);
            if (k == 0) return fail(ESC_ERR_INVALID, "malformed node array");
            parts.push_back({pos, k});
            pos += k;
        }
    } else {
        parts.push_back({0, (int)p->nodes.size()});
    }
    if ((int)parts.size() > ESC_MAX_CONJ)
        return fail(ESC_ERR_UNSUPPORTED, "%zu conjuncts (max %d)", parts.size(), ESC_MAX_CONJ);
    // compile each conjunct, then map its slots onto the union of columns
    int slot_of[64];
    for (int c = 0; c < 64; c++) slot_of[c] = -1;
    nslots = 0;
    for (auto &pt : parts) {
        esc_pred q;
        int rc = compile(&schema, p->nodes.data() + pt.first, pt.second, p->consts.data(), (int)p->consts.size(),
                         p->udf.data(), (int)p->udf.size(), &q);
        if (rc) return rc;
        for (int s = 0; s < q.prog.nslots; s++) {
            const int c = q.prog.slot_col[s];
            if (slot_of[c] < 0) {
                if (nslots == kMaxSlots)
                    return fail(ESC_ERR_UNSUPPORTED, "conjuncts read more than %d columns", kMaxSlots);
                slot_of[c] = nslots;
                slot_col[nslots++] = c;
            }
        }
        out.push_back(q.prog);
    }
    for (Program &Q : out) {
        const Program P = Q;
        for (int i = 0; i < P.ninsn; i++) {
            Insn &I = Q.insn[i];
            const bool udf_op = I.op >= U_LOAD;
            const bool reads_col = udf_op ? !(I.flags & F_CONST) : !(I.flags & F_SRC_UDF);
            if (reads_col) I.src = (uint8_t)slot_of[P.slot_col[I.src]];
        }
        Q.nslots = nslots;
        for (int s = 0; s < kMaxSlots; s++) Q.slot_col[s] = s < nslots ? slot_col[s] : 0;
    }
    return ESC_OK;
}

}  // namespace esc

// ---------------------------------------------------------------- C ABI

extern "C" {

const char *esc_last_error(void) { return esc::last_error(); }
int esc_abi_version(void) { return ESC_ABI_VERSION; }

int esc_table_create(int64_t nrows, int ncols, const int32_t *dtypes, const void *const *dev_cols,
                     esc_table **out)
{
    using esc::fail;
    if (!out || !dtypes) return fail(ESC_ERR_INVALID, "null argument");
    if (nrows < 0 || nrows > INT32_MAX) return fail(ESC_ERR_INVALID, "nrows %lld outside [0, 2^31-1]", (long long)nrows);
    if (ncols < 1 || ncols > 64) return fail(ESC_ERR_INVALID, "ncols %d outside [1, 64]", ncols);
    for (int c = 0; c < ncols; c++)
        if (dtypes[c] != ESC_INT32 && dtypes[c] != ESC_DATE32 && dtypes[c] != ESC_FLOAT32)
            return fail(ESC_ERR_INVALID, "column %d has unknown dtype %d", c, dtypes[c]);
    if (dev_cols)
        for (int c = 0; c < ncols; c++) {
            if (!dev_cols[c] && nrows > 0) return fail(ESC_ERR_INVALID, "column %d pointer is null", c);
            if (((uintptr_t)dev_cols[c]) & 15) return fail(ESC_ERR_ALIGN, "column %d is not 16-byte aligned", c);
        }
    esc_table *t = new (std::nothrow) esc_table;
    if (!t) return fail(ESC_ERR_OOM, "out of host memory");
    t->id = esc::next_handle_id();
    t->nrows = nrows;
    t->dtypes.assign(dtypes, dtypes + ncols);
    if (dev_cols) t->cols.assign(dev_cols, dev_cols + ncols);
    *out = t;
    return ESC_OK;
}

int esc_table_destroy(esc_table *t)
{
    delete t;
    return ESC_OK;
}

int esc_compile_predicate(const esc_table *schema, const esc_node *nodes, int nnodes, const esc_const *consts,
                          int nconsts, const esc_udf_insn *udf, int nudf, esc_pred **out)
{
    if (!out) return esc::fail(ESC_ERR_INVALID, "null output handle");
    esc_pred *p = new (std::nothrow) esc_pred;
    if (!p) return esc::fail(ESC_ERR_OOM, "out of host memory");
    int rc = esc::compile(schema, nodes, nnodes, consts, nconsts, udf, nudf, p);
    if (rc) { delete p; return rc; }
    p->id = esc::next_handle_id();
    p->ncols_schema = (int)schema->dtypes.size();
    p->schema_dtypes = schema->dtypes;
    p->nodes.assign(nodes, nodes + nnodes);
    if (nconsts) p->consts.assign(consts, consts + nconsts);
    if (nudf) p->udf.assign(udf, udf + nudf);
    *out = p;
    return ESC_OK;
}

int esc_pred_destroy(esc_pred *p)
{
    delete p;
    return ESC_OK;
}

int esc_pred_get_info(const esc_pred *p, esc_pred_info *out)
{
    if (!p || !out) return esc::fail(ESC_ERR_INVALID, "null argument");
    out->nclauses = p->prog.nclauses;
    out->ninsns = p->prog.ninsn;
    out->ncols = p->prog.nslots;
    out->constant = (p->prog.flags & esc::P_ALWAYS_TRUE) ? 1 : (p->prog.flags & esc::P_ALWAYS_FALSE) ? -1 : 0;
    out->col_mask = p->col_mask;
    out->nhashed = p->nhashed;
    out->pad = 0;
    return ESC_OK;
}

}  // extern "C"
