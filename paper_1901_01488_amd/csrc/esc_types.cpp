// esc_types.cpp -- TEXT and DECIMAL predicate columns (host only; needs no
// GPU).
//
// Section 3 (Table 3) measures predicates on TEXT and DECIMAL(15,2)
// columns beside INTEGER ones.  Both are stored here as 4-byte columns so
// that the scans keep their coalesced 16-byte loads and exact int32 tests:
//  - TEXT: dictionary codes.  A dictionary holds distinct byte strings in
//    byte-wise order; a column stores each value's rank (its code).  A
//    comparison of the strings is then a comparison of the codes, and a
//    prefix match is a code interval, so every string predicate becomes an
//    int32 range or set on the codes.
//  - DECIMAL(p, s): the value times 10^s as int32 (|value| * 10^s < 2^31).
//    A decimal literal is parsed exactly and a comparison with it becomes an
//    int32 bound (rounded in the direction that keeps the set of qualifying
//    values the same).
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "esc_host.h"

using esc::fail;

struct esc_dict {
    std::vector<std::string> s;   // distinct, byte-wise ascending; code = index
};

namespace {

bool less_bytes(const std::string &a, const std::string &b)
{
    return std::lexicographical_compare(a.begin(), a.end(), b.begin(), b.end(),
                                        [](char x, char y) { return (unsigned char)x < (unsigned char)y; });
}

// first code whose string is >= v (upper = false) or > v (upper = true)
int32_t bound(const esc_dict *d, const std::string &v, bool upper)
{
    auto it = upper ? std::upper_bound(d->s.begin(), d->s.end(), v, less_bytes)
                    : std::lower_bound(d->s.begin(), d->s.end(), v, less_bytes);
    return (int32_t)(it - d->s.begin());
}

// parse [+-]digits[.digits]; returns false on anything else
bool parse_decimal(const char *lit, bool &neg, std::string &ip, std::string &fp)
{
    neg = false;
    ip.clear();
    fp.clear();
    const char *c = lit;
    if (*c == '+' || *c == '-') neg = *c++ == '-';
    while (*c >= '0' && *c <= '9') ip += *c++;
    if (*c == '.') {
        c++;
        while (*c >= '0' && *c <= '9') fp += *c++;
    }
    return *c == 0 && (!ip.empty() || !fp.empty());
}

}  // namespace

extern "C" {

int esc_dict_create(const char *const *strings, int n, esc_dict **out)
{
    if (!out || n < 0 || (n > 0 && !strings)) return fail(ESC_ERR_INVALID, "null argument");
    esc_dict *d = new esc_dict;
    d->s.reserve((size_t)n);
    for (int i = 0; i < n; i++) {
        if (!strings[i]) { delete d; return fail(ESC_ERR_INVALID, "string %d is null", i); }
        d->s.emplace_back(strings[i]);
    }
    std::sort(d->s.begin(), d->s.end(), less_bytes);
    if (std::adjacent_find(d->s.begin(), d->s.end()) != d->s.end()) {
        delete d;
        return fail(ESC_ERR_INVALID, "dictionary strings must be distinct");
    }
    *out = d;
    return ESC_OK;
}

int esc_dict_destroy(esc_dict *d)
{
    delete d;
    return ESC_OK;
}

int esc_dict_size(const esc_dict *d, int *n)
{
    if (!d || !n) return fail(ESC_ERR_INVALID, "null argument");
    *n = (int)d->s.size();
    return ESC_OK;
}

int esc_dict_code(const esc_dict *d, const char *s, int32_t *code)
{
    if (!d || !s || !code) return fail(ESC_ERR_INVALID, "null argument");
    const std::string v(s);
    const int32_t i = bound(d, v, false);
    *code = (i < (int32_t)d->s.size() && d->s[(size_t)i] == v) ? i : -1;
    return ESC_OK;
}

int esc_dict_string(const esc_dict *d, int32_t code, const char **s)
{
    if (!d || !s) return fail(ESC_ERR_INVALID, "null argument");
    if (code < 0 || code >= (int32_t)d->s.size()) return fail(ESC_ERR_INVALID, "code %d out of range", code);
    *s = d->s[(size_t)code].c_str();
    return ESC_OK;
}

int esc_dict_range(const esc_dict *d, int op, const char *s, const char *s2, int32_t *lo, int32_t *hi)
{
    if (!d || !s || !lo || !hi || (op == ESC_BETWEEN && !s2)) return fail(ESC_ERR_INVALID, "null argument");
    const std::string v(s);
    const int32_t n = (int32_t)d->s.size();
    switch (op) {
    case ESC_EQ: *lo = bound(d, v, false); *hi = bound(d, v, true) - 1; break;
    case ESC_LT: *lo = 0; *hi = bound(d, v, false) - 1; break;
    case ESC_GT: *lo = bound(d, v, true); *hi = n - 1; break;
    case ESC_BETWEEN: *lo = bound(d, v, false); *hi = bound(d, std::string(s2), true) - 1; break;
    case ESC_DICT_PREFIX: {
        // the strings starting with v follow each other from the first >= v
        const auto first = d->s.begin() + bound(d, v, false);
        const auto end = std::partition_point(first, d->s.end(), [&](const std::string &x) {
            return x.compare(0, v.size(), v) == 0;
        });
        *lo = (int32_t)(first - d->s.begin());
        *hi = (int32_t)(end - d->s.begin()) - 1;
        break;
    }
    default: return fail(ESC_ERR_INVALID, "op %d is not a string comparison", op);
    }
    if (*lo > *hi) { *lo = 0; *hi = -1; }
    return ESC_OK;
}

int esc_decimal_bound(const char *literal, int scale, int op, int64_t *bound_out, int *empty)
{
    if (!literal || !bound_out || !empty) return fail(ESC_ERR_INVALID, "null argument");
    if (scale < 0 || scale > 9) return fail(ESC_ERR_INVALID, "scale %d outside [0, 9]", scale);
    bool neg;
    std::string ip, fp;
    if (!parse_decimal(literal, neg, ip, fp)) return fail(ESC_ERR_INVALID, "'%s' is not a decimal literal", literal);
    // |literal| * 10^scale = q + r, q an integer, r in [0, 1) (exact: r > 0 iff a dropped digit is nonzero)
    std::string digits = ip + fp.substr(0, std::min<size_t>(fp.size(), (size_t)scale));
    digits.append((size_t)scale - std::min<size_t>(fp.size(), (size_t)scale), '0');
    bool frac = false;
    for (size_t i = (size_t)scale; i < fp.size(); i++) frac = frac || fp[i] != '0';
    size_t k = 0;
    while (k + 1 < digits.size() && digits[k] == '0') k++;
    digits = digits.substr(k);
    int64_t q = 0;
    if (digits.size() > 18) {   // saturate: treated as 10^18 + 1/2, exact for every |x| < 10^18
        q = 1000000000000000000LL;
        frac = true;
    } else {
        for (char c : digits) q = q * 10 + (c - '0');
    }
    // the literal times 10^scale lies in [lo, hi] = [v, v] (exact) or (floor, floor + 1)
    int64_t fl, ce;
    if (!neg) { fl = q; ce = frac ? q + 1 : q; }
    else { fl = frac ? -q - 1 : -q; ce = -q; }
    *empty = 0;
    switch (op) {
    case ESC_EQ:   // x = c: only if c is a multiple of 10^-scale
        if (frac) *empty = 1;
        *bound_out = fl;
        break;
    case ESC_LT: *bound_out = ce - 1; break;   // x < c  <=> x <= ceil(c) - 1
    case ESC_GT: *bound_out = fl + 1; break;   // x > c  <=> x >= floor(c) + 1
    default: return fail(ESC_ERR_INVALID, "op %d: use ESC_EQ, ESC_LT (largest x) or ESC_GT (smallest x)", op);
    }
    return ESC_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ typed predicates
//
// Lowering rewrites every leaf on a TEXT or DECIMAL column into leaves on its
// int32 storage, in pre-order, keeping every other node as it is:
//  - TEXT: =, <, >, BETWEEN and a prefix are each one code interval (a
//    BETWEEN leaf, or an always-false leaf when no code qualifies); IN is
//    the set of codes of the listed strings that are in the dictionary;
//  - DECIMAL stored in int32: a literal becomes the exact bound that keeps
//    the same qualifying values (x < c <=> x <= the largest stored value
//    below c, ...), clamped to int32; IN keeps the literals that equal a
//    storable value;
//  - DECIMAL stored in int64 as two word columns H (high 32 bits, signed)
//    and L (low 32 bits with the sign bit flipped, so that signed order on L
//    is unsigned order on the low word): the values' order is the
//    lexicographic order of (H, L), and lo <= x <= hi becomes
//    H in [lo_H, hi_H] and (H > lo_H or L >= lo_L) and (H < hi_H or L <= hi_L)
//    (H = h and L in [lo_L, hi_L] when both bounds share their high word);
//    IN groups its values by high word: H in {h...} and, per h,
//    (H < h or H > h or L in lows(h)).
namespace {

struct Lowering {
    const esc_col_type *types = nullptr;
    int ncols = 0;
    const esc_const *consts = nullptr;
    int nconsts = 0;
    const char *const *lits = nullptr;
    int nlits = 0;
    std::vector<esc_node> nodes;
    std::vector<esc_const> out_consts;

    int add_const(int32_t v)
    {
        esc_const c{};
        c.dtype = ESC_INT32;
        c.v.i = v;
        out_consts.push_back(c);
        return (int)out_consts.size() - 1;
    }
    void leaf(int op, int col, int32_t a, int32_t b = 0)
    {
        esc_node n{};
        n.op = op;
        n.col = col;
        n.k0 = add_const(a);
        if (op == ESC_BETWEEN) n.k1 = add_const(b);
        nodes.push_back(n);
    }
    void in_leaf(int col, const std::vector<int32_t> &vals)
    {
        esc_node n{};
        n.op = ESC_IN;
        n.col = col;
        n.k0 = (int)out_consts.size();
        n.k1 = (int)vals.size();
        for (int32_t v : vals) add_const(v);
        nodes.push_back(n);
    }
    void never(int col) { leaf(ESC_LT, col, INT32_MIN); }   // folds to false
    void open(int op, int nchild)
    {
        esc_node n{};
        n.op = op;
        n.nchild = nchild;
        nodes.push_back(n);
    }
    // lo <= x <= hi on an int32 column (int64 bounds, clamped)
    void range32(int col, int64_t lo, int64_t hi)
    {
        lo = std::max<int64_t>(lo, INT32_MIN);
        hi = std::min<int64_t>(hi, INT32_MAX);
        if (lo > hi) never(col);
        else leaf(ESC_BETWEEN, col, (int32_t)lo, (int32_t)hi);
    }
    static void words(int64_t v, int32_t &h, int32_t &l)
    {
        h = (int32_t)(v >> 32);
        l = (int32_t)(((uint32_t)((uint64_t)v & 0xffffffffu)) ^ 0x80000000u);
    }
    // lo <= x <= hi on the word columns (H, L); has_lo / has_hi: bounded ends
    void range64(int H, int L, bool has_lo, int64_t lo, bool has_hi, int64_t hi)
    {
        if (has_lo && has_hi && lo > hi) { never(H); return; }
        int32_t lh = 0, ll = 0, hh = 0, hl = 0;
        if (has_lo) words(lo, lh, ll);
        if (has_hi) words(hi, hh, hl);
        if (has_lo && has_hi && lh == hh) {
            open(ESC_AND, 2);
            leaf(ESC_EQ, H, lh);
            leaf(ESC_BETWEEN, L, ll, hl);
            return;
        }
        const int parts = 1 + (has_lo ? 1 : 0) + (has_hi ? 1 : 0);
        if (parts > 1) open(ESC_AND, parts);
        leaf(ESC_BETWEEN, H, has_lo ? lh : INT32_MIN, has_hi ? hh : INT32_MAX);
        if (has_lo) {   // H > lh or L >= ll
            open(ESC_OR, 2);
            leaf(ESC_GT, H, lh);
            leaf(ESC_BETWEEN, L, ll, INT32_MAX);
        }
        if (has_hi) {   // H < hh or L <= hl
            open(ESC_OR, 2);
            leaf(ESC_LT, H, hh);
            leaf(ESC_BETWEEN, L, INT32_MIN, hl);
        }
    }

    int literal(const esc_node &n, int k, const char **out)
    {
        if (k < 0 || k >= nlits || !lits[k]) return fail(ESC_ERR_INVALID, "literal index %d out of range", k);
        *out = lits[k];
        return ESC_OK;
    }
    int dec(const char *lit, int scale, int op, int64_t *b, int *empty)
    {
        return esc_decimal_bound(lit, scale, op, b, empty);
    }

    int text_leaf(const esc_node &n, const esc_dict *d)
    {
        const char *a = nullptr, *b = nullptr;
        int32_t lo = 0, hi = -1;
        int rc;
        switch (n.op) {
        case ESC_IN: {
            std::vector<int32_t> codes;
            for (int i = 0; i < n.k1; i++) {
                if ((rc = literal(n, n.k0 + i, &a))) return rc;
                if ((rc = esc_dict_range(d, ESC_EQ, a, nullptr, &lo, &hi))) return rc;
                if (lo <= hi) codes.push_back(lo);
            }
            std::sort(codes.begin(), codes.end());
            codes.erase(std::unique(codes.begin(), codes.end()), codes.end());
            if (codes.empty()) never(n.col);
            else in_leaf(n.col, codes);
            return ESC_OK;
        }
        case ESC_BETWEEN:
            if ((rc = literal(n, n.k0, &a)) || (rc = literal(n, n.k1, &b))) return rc;
            if ((rc = esc_dict_range(d, ESC_BETWEEN, a, b, &lo, &hi))) return rc;
            break;
        case ESC_EQ: case ESC_LT: case ESC_GT: case ESC_PREFIX:
            if ((rc = literal(n, n.k0, &a))) return rc;
            if ((rc = esc_dict_range(d, n.op == ESC_PREFIX ? (int)ESC_DICT_PREFIX : n.op, a, nullptr, &lo, &hi)))
                return rc;
            break;
        default: return fail(ESC_ERR_INVALID, "op %d is not a TEXT comparison", n.op);
        }
        range32(n.col, lo, hi);
        return ESC_OK;
    }

    // the stored-value interval [lo, hi] of a DECIMAL comparison (has_*:
    // bounded); *none: nothing qualifies
    int dec_interval(const esc_node &n, int scale, bool &has_lo, int64_t &lo, bool &has_hi, int64_t &hi, bool &none)
    {
        const char *a = nullptr, *b = nullptr;
        int empty = 0, rc;
        has_lo = has_hi = none = false;
        switch (n.op) {
        case ESC_EQ:
            if ((rc = literal(n, n.k0, &a)) || (rc = dec(a, scale, ESC_EQ, &lo, &empty))) return rc;
            hi = lo;
            has_lo = has_hi = true;
            none = empty != 0;
            return ESC_OK;
        case ESC_LT:
            if ((rc = literal(n, n.k0, &a)) || (rc = dec(a, scale, ESC_LT, &hi, &empty))) return rc;
            has_hi = true;
            return ESC_OK;
        case ESC_GT:
            if ((rc = literal(n, n.k0, &a)) || (rc = dec(a, scale, ESC_GT, &lo, &empty))) return rc;
            has_lo = true;
            return ESC_OK;
        case ESC_BETWEEN:   // a <= x <= b: above the largest value below a, below the smallest above b
            if ((rc = literal(n, n.k0, &a)) || (rc = literal(n, n.k1, &b))) return rc;
            if ((rc = dec(a, scale, ESC_LT, &lo, &empty)) || (rc = dec(b, scale, ESC_GT, &hi, &empty))) return rc;
            lo += 1;
            hi -= 1;
            has_lo = has_hi = true;
            return ESC_OK;
        default: return fail(ESC_ERR_INVALID, "op %d is not a DECIMAL comparison", n.op);
        }
    }

    int in_values(const esc_node &n, int scale, std::vector<int64_t> &vals)
    {
        for (int i = 0; i < n.k1; i++) {
            const char *a = nullptr;
            int64_t v = 0;
            int empty = 0, rc;
            if ((rc = literal(n, n.k0 + i, &a)) || (rc = dec(a, scale, ESC_EQ, &v, &empty))) return rc;
            if (!empty) vals.push_back(v);
        }
        std::sort(vals.begin(), vals.end());
        vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
        return ESC_OK;
    }

    int decimal_leaf(const esc_node &n, int scale)
    {
        if (n.op == ESC_IN) {
            std::vector<int64_t> vals;
            int rc = in_values(n, scale, vals);
            if (rc) return rc;
            std::vector<int32_t> v32;
            for (int64_t v : vals)
                if (v >= INT32_MIN && v <= INT32_MAX) v32.push_back((int32_t)v);
            if (v32.empty()) never(n.col);
            else in_leaf(n.col, v32);
            return ESC_OK;
        }
        bool hl, hh, none;
        int64_t lo = 0, hi = 0;
        int rc = dec_interval(n, scale, hl, lo, hh, hi, none);
        if (rc) return rc;
        if (none) never(n.col);
        else range32(n.col, hl ? lo : INT32_MIN, hh ? hi : INT32_MAX);
        return ESC_OK;
    }

    int decimal64_leaf(const esc_node &n, int scale, int L)
    {
        const int H = n.col;
        if (n.op == ESC_IN) {
            std::vector<int64_t> vals;
            int rc = in_values(n, scale, vals);
            if (rc) return rc;
            if (vals.empty()) { never(H); return ESC_OK; }
            std::vector<std::pair<int32_t, std::vector<int32_t>>> groups;   // by high word, ascending
            for (int64_t v : vals) {
                int32_t h, l;
                words(v, h, l);
                if (groups.empty() || groups.back().first != h) groups.push_back({h, {}});
                groups.back().second.push_back(l);
            }
            open(ESC_AND, 1 + (int)groups.size());
            std::vector<int32_t> highs;
            for (auto &g : groups) highs.push_back(g.first);
            in_leaf(H, highs);
            for (auto &g : groups) {
                std::sort(g.second.begin(), g.second.end());
                if (groups.size() == 1) {
                    in_leaf(L, g.second);
                } else {
                    open(ESC_OR, 3);
                    leaf(ESC_LT, H, g.first);
                    leaf(ESC_GT, H, g.first);
                    in_leaf(L, g.second);
                }
            }
            return ESC_OK;
        }
        bool hl, hh, none;
        int64_t lo = 0, hi = 0;
        int rc = dec_interval(n, scale, hl, lo, hh, hi, none);
        if (rc) return rc;
        if (none) never(H);
        else range64(H, L, hl, lo, hh, hi);
        return ESC_OK;
    }

    // lowers the subtree at in[*pos], advancing *pos past it
    int walk(const esc_node *in, int nnodes, int *pos, int depth)
    {
        if (*pos >= nnodes) return fail(ESC_ERR_INVALID, "node array ends inside a subtree");
        if (depth > 64) return fail(ESC_ERR_INVALID, "predicate nested deeper than 64");
        const esc_node n = in[(*pos)++];
        if (n.op == ESC_AND || n.op == ESC_OR) {
            if (n.nchild < 1) return fail(ESC_ERR_INVALID, "AND/OR without children");
            nodes.push_back(n);
            for (int c = 0; c < n.nchild; c++)
                if (int rc = walk(in, nnodes, pos, depth + 1)) return rc;
            return ESC_OK;
        }
        if (n.op == ESC_UDF) {   // constants copied, the program indices kept
            esc_node m = n;
            const int cnt = n.cmp == ESC_IN ? n.k1 : n.cmp == ESC_BETWEEN ? 2 : 1;
            const int first = n.k0;
            m.k0 = (int)out_consts.size();
            for (int i = 0; i < cnt; i++) {
                const int k = n.cmp == ESC_BETWEEN ? (i == 0 ? n.k0 : n.k1) : first + i;
                if (k < 0 || k >= nconsts) return fail(ESC_ERR_INVALID, "constant index %d out of range", k);
                out_consts.push_back(consts[k]);
            }
            if (n.cmp == ESC_BETWEEN) m.k1 = m.k0 + 1;
            nodes.push_back(m);
            return ESC_OK;
        }
        if (n.col < 0 || n.col >= ncols) return fail(ESC_ERR_INVALID, "column %d out of range", n.col);
        const esc_col_type T = types ? types[n.col] : esc_col_type{};
        switch (T.kind) {
        case ESC_COL_PLAIN: {
            if (n.op == ESC_PREFIX) return fail(ESC_ERR_TYPE, "prefix match on column %d, which is not TEXT", n.col);
            esc_node m = n;
            const int cnt = n.op == ESC_IN ? n.k1 : n.op == ESC_BETWEEN ? 2 : 1;
            m.k0 = (int)out_consts.size();
            for (int i = 0; i < cnt; i++) {
                const int k = n.op == ESC_BETWEEN ? (i == 0 ? n.k0 : n.k1) : n.k0 + i;
                if (k < 0 || k >= nconsts) return fail(ESC_ERR_INVALID, "constant index %d out of range", k);
                out_consts.push_back(consts[k]);
            }
            if (n.op == ESC_BETWEEN) m.k1 = m.k0 + 1;
            nodes.push_back(m);
            return ESC_OK;
        }
        case ESC_COL_TEXT:
            if (!T.dict) return fail(ESC_ERR_INVALID, "TEXT column %d has no dictionary", n.col);
            return text_leaf(n, T.dict);
        case ESC_COL_DECIMAL:
        case ESC_COL_DECIMAL64:
            if (n.op == ESC_PREFIX) return fail(ESC_ERR_TYPE, "prefix match on DECIMAL column %d", n.col);
            if (T.kind == ESC_COL_DECIMAL) return decimal_leaf(n, T.scale);
            if (T.low_col < 0 || T.low_col >= ncols || T.low_col == n.col)
                return fail(ESC_ERR_INVALID, "DECIMAL64 column %d: low-word column %d", n.col, T.low_col);
            return decimal64_leaf(n, T.scale, T.low_col);
        default: return fail(ESC_ERR_INVALID, "column %d: kind %d", n.col, T.kind);
        }
    }
};

}  // namespace

extern "C" {

int esc_lower_typed(const esc_table *schema, const esc_col_type *coltypes, const esc_node *nodes, int nnodes,
                    const esc_const *consts, int nconsts, const char *const *literals, int nliterals,
                    esc_node *out_nodes, int max_nodes, int *out_nnodes, esc_const *out_consts, int max_consts,
                    int *out_nconsts)
{
    if (!schema || !nodes || nnodes < 1 || !out_nnodes || !out_nconsts || (nconsts > 0 && !consts) ||
        (nliterals > 0 && !literals))
        return fail(ESC_ERR_INVALID, "null argument");
    Lowering lw;
    lw.types = coltypes;
    lw.ncols = (int)schema->dtypes.size();
    lw.consts = consts;
    lw.nconsts = nconsts;
    lw.lits = literals;
    lw.nlits = nliterals;
    for (int c = 0; coltypes && c < lw.ncols; c++)
        if (coltypes[c].kind != ESC_COL_PLAIN && schema->dtypes[(size_t)c] != ESC_INT32)
            return fail(ESC_ERR_TYPE, "typed column %d must be stored as int32", c);
    int pos = 0;
    int rc = lw.walk(nodes, nnodes, &pos, 0);
    if (rc) return rc;
    if (pos != nnodes) return fail(ESC_ERR_INVALID, "%d nodes after the end of the tree", nnodes - pos);
    *out_nnodes = (int)lw.nodes.size();
    *out_nconsts = (int)lw.out_consts.size();
    if (lw.nodes.size() > (size_t)max_nodes || lw.out_consts.size() > (size_t)max_consts || !out_nodes ||
        (!out_consts && !lw.out_consts.empty()))
        return fail(ESC_ERR_CAPACITY, "the lowered predicate has %zu nodes and %zu constants", lw.nodes.size(),
                    lw.out_consts.size());
    std::copy(lw.nodes.begin(), lw.nodes.end(), out_nodes);
    std::copy(lw.out_consts.begin(), lw.out_consts.end(), out_consts);
    return ESC_OK;
}

int esc_decimal64_words(const int64_t *values, int64_t n, int32_t *high, int32_t *low)
{
    if (n < 0 || (n > 0 && (!values || !high || !low))) return fail(ESC_ERR_INVALID, "null argument");
    for (int64_t i = 0; i < n; i++) {
        high[i] = (int32_t)(values[i] >> 32);
        low[i] = (int32_t)(((uint32_t)((uint64_t)values[i] & 0xffffffffu)) ^ 0x80000000u);
    }
    return ESC_OK;
}

}  // extern "C"
