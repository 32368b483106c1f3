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
