// esc_features.cpp -- host-side featurization of compiled predicates for the
// learned estimator, and the gate that decides which predicates are sent to
// exact evaluation (host only; needs no GPU).
//
// The paper computes every selectivity exactly (Section 2) and uses it for
// two plan decisions: pushing a selection down with materialization only
// when it is selective enough, controlled by a maximum selectivity threshold
// and a minimum table size (Section 2.1), and the join order of the build
// relations, smallest first (Section 2.2).  The gate keeps the exact count
// for exactly those predicates whose estimate is close enough to a decision
// boundary that the estimator's error could flip the decision.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "esc_host.h"

using esc::fail;

namespace {

constexpr int kNF = 64;     // features per predicate
constexpr int kNCF = 6;     // columns described
constexpr int kPerCol = 10;
constexpr double kMinSel = 1e-9;               // floor of a column's selectivity estimate
constexpr double kLnMinSel = 20.72326583694641;   // -ln(kMinSel)

// Smoothed empirical CDF of one column from its catalog minimum, maximum and
// a row sample.  Knots at the distinct sampled values u_j with left / right
// limits L_j = (#{s < u_j} + 1/2) / m and R_j = (#{s <= u_j} - 1/2) / m
// (continuous at values sampled once, a jump of (count - 1) / m at values
// sampled more often), linear between knots, 0 at the minimum, 1 at the
// maximum.  Integer columns put value k in the cell [k - 1/2, k + 1/2].
struct Cdf {
    std::vector<double> u, L, R;
    bool integer = false;

    void build(const std::vector<double> &sample_in, double lo, double hi, bool is_int)
    {
        integer = is_int;
        std::vector<double> s;
        for (double v : sample_in)
            if (!isnan(v) && v >= lo && v <= hi) s.push_back(v);
        std::sort(s.begin(), s.end());
        const double m = (double)s.size();
        u.clear(); L.clear(); R.clear();
        for (size_t i = 0; i < s.size();) {
            size_t j = i;
            while (j < s.size() && s[j] == s[i]) j++;
            u.push_back(s[i]);
            L.push_back(((double)i + 0.5) / m);
            R.push_back(((double)j - 0.5) / m);
            i = j;
        }
        if (u.empty() || lo < u.front()) {
            u.insert(u.begin(), lo); L.insert(L.begin(), 0.0); R.insert(R.begin(), 0.0);
        } else {
            L.front() = 0.0;
        }
        if (hi > u.back()) {
            u.push_back(hi); L.push_back(1.0); R.push_back(1.0);
        } else {
            R.back() = 1.0;
        }
    }

    double g(double v, bool le) const
    {
        if (v < u.front()) return 0.0;
        if (v > u.back()) return 1.0;
        const size_t i = (size_t)(std::lower_bound(u.begin(), u.end(), v) - u.begin());
        if (u[i] == v) return le ? R[i] : L[i];
        const double t = (v - u[i - 1]) / (u[i] - u[i - 1]);
        return R[i - 1] + t * (L[i] - R[i - 1]);
    }

    // fraction of rows below v (le = false) or at most v (le = true)
    double at(double v, bool le) const
    {
        if (isnan(v)) return 0.0;
        if (integer) return g(le ? v + 0.5 : v - 0.5, le);
        return g(v, le);
    }
};

struct Walk {
    const esc_pred *p;
    const Cdf *cdf;   // kNCF columns
    double *f;        // kNF values, rounded to float32 by the caller
    int n_or = 0, n_leaves = 0, has_udf = 0;
    bool present[kNCF] = {};
};

// index just past the subtree rooted at node i
int skip(const esc_pred *p, int i)
{
    const esc_node &n = p->nodes[i];
    int j = i + 1;
    if (n.op == ESC_AND || n.op == ESC_OR)
        for (int k = 0; k < n.nchild; k++) j = skip(p, j);
    return j;
}

double value(const esc_pred *p, int col, esc_value v)
{
    return p->schema_dtypes[col] == ESC_FLOAT32 ? (double)v.f : (double)v.i;
}

bool is_col_leaf(int op) { return op >= ESC_EQ && op <= ESC_IN; }

// distinct non-NaN constants of an IN leaf, ascending
std::vector<double> in_values(const Walk &W, const esc_node &n)
{
    std::vector<double> v;
    for (int i = 0; i < n.k1; i++) {
        const double x = value(W.p, n.col, W.p->consts[n.k0 + i].v);
        if (!isnan(x)) v.push_back(x);
    }
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    return v;
}

// [fraction below the leaf's range, fraction at most its top]
void interval(const Walk &W, const esc_node &n, double &lo, double &hi)
{
    const Cdf &F = W.cdf[n.col];
    auto k = [&](int idx) { return value(W.p, n.col, W.p->consts[idx].v); };
    switch (n.op) {
    case ESC_EQ: lo = F.at(k(n.k0), false); hi = F.at(k(n.k0), true); return;
    case ESC_LT: lo = 0.0; hi = F.at(k(n.k0), false); return;
    case ESC_GT: lo = F.at(k(n.k0), true); hi = 1.0; return;
    case ESC_BETWEEN: lo = F.at(k(n.k0), false); hi = F.at(k(n.k1), true); return;
    default: {
        const std::vector<double> v = in_values(W, n);
        if (v.empty()) { lo = hi = 0.0; return; }
        lo = F.at(v.front(), false);
        hi = F.at(v.back(), true);
    }
    }
}

// estimated fraction of rows equal to one of the IN constants
double in_mass(const Walk &W, const esc_node &n)
{
    double m = 0.0;
    for (double x : in_values(W, n)) m += W.cdf[n.col].at(x, true) - W.cdf[n.col].at(x, false);
    return m;
}

// op flags, IN sizes and masses, OR marks (or_mark = ordinal / 4 of the
// conjunct holding the OR, 0 outside ORs)
void flags(Walk &W, int i, double or_mark)
{
    const esc_node &n = W.p->nodes[i];
    if (n.op == ESC_AND || n.op == ESC_OR) {
        if (n.op == ESC_OR) W.n_or++;
        int j = i + 1;
        for (int k = 0; k < n.nchild; k++) {
            flags(W, j, or_mark);
            j = skip(W.p, j);
        }
        return;
    }
    W.n_leaves++;
    if (n.op == ESC_UDF) { W.has_udf = 1; return; }
    if (n.col >= kNCF) return;
    double *c = W.f + kPerCol * n.col;
    W.present[n.col] = true;
    if (n.op == ESC_IN) {
        c[7] += in_mass(W, n);
        c[8] += (double)n.k1 / 16.0;
    } else {
        c[3 + (n.op - ESC_EQ)] = 1.0;   // is_eq, is_lt, is_gt, is_between
    }
    c[9] = std::max(c[9], or_mark);
}

bool contains_or(const esc_pred *p, int i)
{
    const esc_node &n = p->nodes[i];
    if (n.op == ESC_OR) return true;
    if (n.op != ESC_AND) return false;
    int j = i + 1;
    for (int k = 0; k < n.nchild; k++) {
        if (contains_or(p, j)) return true;
        j = skip(p, j);
    }
    return false;
}

void clamp_col(Walk &W, int col, double lo, double hi)
{
    double *c = W.f + kPerCol * col;
    c[1] = std::max(c[1], lo);
    c[2] = std::min(c[2], hi);
}

void featurize_one(Walk &W)
{
    for (int i = 0; i < kNF; i++) W.f[i] = 0.0;
    for (int c = 0; c < kNCF; c++) W.f[kPerCol * c + 2] = 1.0;
    std::vector<int> conj;
    const esc_node &root = W.p->nodes[0];
    if (root.op == ESC_AND) {
        int j = 1;
        for (int k = 0; k < root.nchild; k++) { conj.push_back(j); j = skip(W.p, j); }
    } else {
        conj.push_back(0);
    }
    int nth_or = 0;
    bool plain[kNCF] = {};
    for (int q : conj) {
        const bool has_or = contains_or(W.p, q);
        if (has_or) nth_or++;
        flags(W, q, has_or ? (double)nth_or / 4.0 : 0.0);
        const esc_node &n = W.p->nodes[q];
        if (is_col_leaf(n.op) && n.col < kNCF) plain[n.col] = true;
    }
    for (int q : conj) {
        const esc_node &n = W.p->nodes[q];
        if (is_col_leaf(n.op)) {
            if (n.col >= kNCF) continue;
            double lo, hi;
            interval(W, n, lo, hi);
            clamp_col(W, n.col, lo, hi);
            continue;
        }
        if (n.op != ESC_OR) continue;
        std::vector<int> kids;
        int j = q + 1;
        bool leaves = true;
        for (int k = 0; k < n.nchild; k++) {
            kids.push_back(j);
            leaves = leaves && is_col_leaf(W.p->nodes[j].op);
            j = skip(W.p, j);
        }
        if (!leaves) continue;
        // hull of the OR's leaves per column; one column: it bounds that
        // column; several: each bounds its column unless a plain conjunct does
        std::vector<int> cols;
        for (int kdx : kids) {
            const int col = W.p->nodes[kdx].col;
            if (std::find(cols.begin(), cols.end(), col) == cols.end()) cols.push_back(col);
        }
        for (int col : cols) {
            if (col >= kNCF || (cols.size() > 1 && plain[col])) continue;
            double lo = 2.0, hi = -1.0;
            for (int kdx : kids) {
                if (W.p->nodes[kdx].col != col) continue;
                double a, b;
                interval(W, W.p->nodes[kdx], a, b);
                lo = std::min(lo, a);
                hi = std::max(hi, b);
            }
            clamp_col(W, col, lo, hi);
        }
    }
    for (int c = 0; c < kNCF; c++) {
        double *v = W.f + kPerCol * c;
        if (!W.present[c]) continue;
        double est = std::max(v[2] - v[1], 0.0);
        if (v[8] > 0.0 && v[7] > 0.0) est = std::min(est, v[7]);
        v[0] = std::min((0.0 - log(std::max(est, kMinSel))) / kLnMinSel, 1.0);   // +0 when est = 1
    }
    W.f[60] = (double)conj.size() / 6.0;
    W.f[61] = (double)W.n_or / 6.0;
    W.f[62] = (double)W.has_udf;
    W.f[63] = (double)W.n_leaves / 16.0;
}

double log_sel(float yhat, int64_t n)
{
    return std::min(std::max((double)yhat, -log((double)n)), 0.0);
}

}  // namespace

extern "C" {

}  // extern "C"

// The column CDFs of a table's catalog, built once and reused by every
// featurization (building them sorts each column's sample).
struct esc_catalog {
    std::vector<int32_t> dtypes;
    Cdf cdf[kNCF];
};

extern "C" {

int esc_catalog_create(const esc_table *schema, const esc_value *col_min, const esc_value *col_max,
                       const esc_value *col_sample, int sample_size, esc_catalog **out)
{
    if (!schema || !col_min || !col_max || !out) return fail(ESC_ERR_INVALID, "null argument");
    if (sample_size < 0 || (sample_size > 0 && !col_sample)) return fail(ESC_ERR_INVALID, "bad column sample");
    esc_catalog *cat = new esc_catalog;
    cat->dtypes = schema->dtypes;
    const int nc = std::min((int)schema->dtypes.size(), kNCF);
    for (int c = 0; c < nc; c++) {
        const bool fl = schema->dtypes[c] == ESC_FLOAT32;
        auto val = [&](esc_value v) { return fl ? (double)v.f : (double)v.i; };
        std::vector<double> smp((size_t)sample_size);
        for (int i = 0; i < sample_size; i++) smp[i] = val(col_sample[(size_t)c * sample_size + i]);
        const double lo = val(col_min[c]), hi = val(col_max[c]);
        if (isnan(lo) || isnan(hi) || lo > hi) {
            delete cat;
            return fail(ESC_ERR_INVALID, "column %d: catalog minimum / maximum not ordered", c);
        }
        cat->cdf[c].build(smp, lo, hi, !fl);
    }
    *out = cat;
    return ESC_OK;
}

int esc_catalog_destroy(esc_catalog *cat)
{
    delete cat;
    return ESC_OK;
}

int esc_featurize_catalog(const esc_catalog *cat, const esc_pred *const *preds, int npreds, float *host_out)
{
    if (!cat || (npreds > 0 && (!preds || !host_out)) || npreds < 0) return fail(ESC_ERR_INVALID, "null argument");
    double f[kNF];
    for (int i = 0; i < npreds; i++) {
        if (!preds[i]) return fail(ESC_ERR_INVALID, "predicate %d is null", i);
        if (preds[i]->schema_dtypes != cat->dtypes)
            return fail(ESC_ERR_INVALID, "predicate %d was compiled for another schema", i);
        Walk W{preds[i], cat->cdf, f};
        featurize_one(W);
        for (int k = 0; k < kNF; k++) host_out[(size_t)i * kNF + k] = (float)f[k];
    }
    return ESC_OK;
}

int esc_featurize(const esc_table *schema, const esc_value *col_min, const esc_value *col_max,
                  const esc_value *col_sample, int sample_size, const esc_pred *const *preds, int npreds,
                  float *host_out)
{
    if (!schema || !col_min || !col_max || (npreds > 0 && (!preds || !host_out)) || npreds < 0)
        return fail(ESC_ERR_INVALID, "null argument");
    esc_catalog *cat = nullptr;
    int rc = esc_catalog_create(schema, col_min, col_max, col_sample, sample_size, &cat);
    if (rc) return rc;
    rc = esc_featurize_catalog(cat, preds, npreds, host_out);
    esc_catalog_destroy(cat);
    return rc;
}

int esc_gate_pushdown(const float *yhat, const int64_t *nrows, int n, double tau, double beta, int64_t min_rows,
                      uint8_t *route)
{
    if (n < 0 || (n > 0 && (!yhat || !nrows || !route))) return fail(ESC_ERR_INVALID, "null argument");
    if (!(tau > 0.0 && tau <= 1.0) || !(beta >= 1.0)) return fail(ESC_ERR_INVALID, "need 0 < tau <= 1 and beta >= 1");
    const double lo = log(tau) - log(beta), hi = log(tau) + log(beta);
    for (int i = 0; i < n; i++) {
        if (nrows[i] < 1) return fail(ESC_ERR_INVALID, "nrows[%d] < 1", i);
        const double s = log_sel(yhat[i], nrows[i]);
        route[i] = (uint8_t)(nrows[i] >= min_rows && lo <= s && s <= hi);
    }
    return ESC_OK;
}

int esc_gate_join_pair(float yhat_r, int64_t n_r, float yhat_s, int64_t n_s, double beta, uint8_t *route)
{
    return esc_gate_join_pairs(&yhat_r, n_r, &yhat_s, n_s, 1, beta, 0.0, route);
}

int esc_gate_join_pairs(const float *yhat_r, int64_t n_r, const float *yhat_s, int64_t n_s, int n, double beta,
                        double tie_sel, uint8_t *route)
{
    if (n < 0 || (n > 0 && (!yhat_r || !yhat_s || !route))) return fail(ESC_ERR_INVALID, "null argument");
    if (n_r < 1 || n_s < 1 || !(beta >= 1.0) || !(tie_sel >= 0.0 && tie_sel <= 1.0))
        return fail(ESC_ERR_INVALID, "need n_r, n_s >= 1, beta >= 1 and 0 <= tie_sel <= 1");
    const double lb = log(beta);
    const double lt = tie_sel > 0.0 ? log(tie_sel) : -HUGE_VAL;
    for (int i = 0; i < n; i++) {
        const double sr = log_sel(yhat_r[i], n_r), ss = log_sel(yhat_s[i], n_s);
        const double d = (sr + log((double)n_r)) - (ss + log((double)n_s));
        // both orders cost the same when neither filtered relation can keep
        // more than tie_sel of its rows, even at the top of the error band
        const bool tie = sr + lb <= lt && ss + lb <= lt;
        route[i] = (uint8_t)(!tie && -2.0 * lb <= d && d <= 2.0 * lb);
    }
    return ESC_OK;
}

}  // extern "C"
