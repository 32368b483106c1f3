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

struct Walk {
    const esc_pred *p;
    const esc_value *cmin, *cmax;
    float *f;
    int n_or = 0, n_leaves = 0, has_udf = 0;
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

float as_float(const esc_pred *p, int col, esc_value v)
{
    return p->schema_dtypes[col] == ESC_FLOAT32 ? v.f : (float)v.i;
}

// (v - min) / (max - min) in float32, clamped to [0, 1]; 0 for NaN or an empty span
float norm(const Walk &W, int col, esc_value v)
{
    const float x = as_float(W.p, col, v);
    const float lo = as_float(W.p, col, W.cmin[col]);
    const float hi = as_float(W.p, col, W.cmax[col]);
    if (isnan(x)) return 0.0f;
    const float span = hi - lo;
    if (span == 0.0f || isnan(span)) return 0.0f;
    const float q = (x - lo) / span;
    return std::min(std::max(q, 0.0f), 1.0f);
}

bool is_col_leaf(int op) { return op >= ESC_EQ && op <= ESC_IN; }

bool less_in(const esc_pred *p, int col, esc_value a, esc_value b)
{
    return p->schema_dtypes[col] == ESC_FLOAT32 ? a.f < b.f : a.i < b.i;
}

void interval(const Walk &W, const esc_node &n, float &lo, float &hi)
{
    const esc_const *k = W.p->consts.data();
    switch (n.op) {
    case ESC_EQ: lo = hi = norm(W, n.col, k[n.k0].v); return;
    case ESC_LT: lo = 0.0f; hi = norm(W, n.col, k[n.k0].v); return;
    case ESC_GT: lo = norm(W, n.col, k[n.k0].v); hi = 1.0f; return;
    case ESC_BETWEEN: lo = norm(W, n.col, k[n.k0].v); hi = norm(W, n.col, k[n.k1].v); return;
    default: {
        esc_value mn = k[n.k0].v, mx = k[n.k0].v;
        for (int i = 1; i < n.k1; i++) {
            if (less_in(W.p, n.col, k[n.k0 + i].v, mn)) mn = k[n.k0 + i].v;
            if (less_in(W.p, n.col, mx, k[n.k0 + i].v)) mx = k[n.k0 + i].v;
        }
        lo = norm(W, n.col, mn);
        hi = norm(W, n.col, mx);
    }
    }
}

void flags(Walk &W, int i, bool under_or)
{
    const esc_node &n = W.p->nodes[i];
    if (n.op == ESC_AND || n.op == ESC_OR) {
        if (n.op == ESC_OR) W.n_or++;
        int j = i + 1;
        for (int k = 0; k < n.nchild; k++) {
            flags(W, j, under_or || n.op == ESC_OR);
            j = skip(W.p, j);
        }
        return;
    }
    W.n_leaves++;
    if (n.op == ESC_UDF) { W.has_udf = 1; return; }
    if (n.col >= kNCF) return;
    float *c = W.f + kPerCol * n.col;
    c[0] = 1.0f;
    c[3 + (n.op - ESC_EQ)] = 1.0f;   // is_eq, is_lt, is_gt, is_between, is_in
    if (n.op == ESC_IN) c[8] = c[8] + (float)n.k1 / 16.0f;
    if (under_or) c[9] = 1.0f;
}

void clamp_col(Walk &W, int col, float lo, float hi)
{
    if (col >= kNCF) return;
    float *c = W.f + kPerCol * col;
    c[1] = std::max(c[1], lo);
    c[2] = std::min(c[2], hi);
}

void featurize_one(Walk &W)
{
    for (int i = 0; i < kNF; i++) W.f[i] = 0.0f;
    for (int c = 0; c < kNCF; c++) W.f[kPerCol * c + 2] = 1.0f;
    flags(W, 0, false);
    std::vector<int> conj;
    const esc_node &root = W.p->nodes[0];
    if (root.op == ESC_AND) {
        int j = 1;
        for (int k = 0; k < root.nchild; k++) { conj.push_back(j); j = skip(W.p, j); }
    } else {
        conj.push_back(0);
    }
    for (int q : conj) {
        const esc_node &n = W.p->nodes[q];
        if (is_col_leaf(n.op)) {
            float lo, hi;
            interval(W, n, lo, hi);
            clamp_col(W, n.col, lo, hi);
        } else if (n.op == ESC_OR) {
            bool same = true;
            int col = -1;
            int j = q + 1;
            std::vector<int> kids;
            for (int k = 0; k < n.nchild; k++) { kids.push_back(j); j = skip(W.p, j); }
            for (int kdx : kids) {
                const esc_node &m = W.p->nodes[kdx];
                if (!is_col_leaf(m.op)) { same = false; break; }
                if (col < 0) col = m.col;
                same = same && m.col == col;
            }
            if (!same) continue;
            float lo = 2.0f, hi = -1.0f;
            for (int kdx : kids) {
                float a, b;
                interval(W, W.p->nodes[kdx], a, b);
                lo = std::min(lo, a);
                hi = std::max(hi, b);
            }
            clamp_col(W, col, lo, hi);
        }
    }
    W.f[60] = (float)conj.size() / 6.0f;
    W.f[61] = (float)W.n_or / 6.0f;
    W.f[62] = (float)W.has_udf;
    W.f[63] = (float)W.n_leaves / 16.0f;
}

double log_sel(float yhat, int64_t n)
{
    return std::min(std::max((double)yhat, -log((double)n)), 0.0);
}

}  // namespace

extern "C" {

int esc_featurize(const esc_table *schema, const esc_value *col_min, const esc_value *col_max,
                  const esc_pred *const *preds, int npreds, float *host_out)
{
    if (!schema || !col_min || !col_max || (npreds > 0 && (!preds || !host_out)) || npreds < 0)
        return fail(ESC_ERR_INVALID, "null argument");
    for (int i = 0; i < npreds; i++) {
        if (!preds[i]) return fail(ESC_ERR_INVALID, "predicate %d is null", i);
        if (preds[i]->schema_dtypes != schema->dtypes)
            return fail(ESC_ERR_INVALID, "predicate %d was compiled for another schema", i);
        Walk W{preds[i], col_min, col_max, host_out + (size_t)i * kNF};
        featurize_one(W);
    }
    return ESC_OK;
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
    if (!route || n_r < 1 || n_s < 1 || !(beta >= 1.0)) return fail(ESC_ERR_INVALID, "bad argument");
    const double d = (log_sel(yhat_r, n_r) + log((double)n_r)) - (log_sel(yhat_s, n_s) + log((double)n_s));
    *route = (uint8_t)(-2.0 * log(beta) <= d && d <= 2.0 * log(beta));
    return ESC_OK;
}

}  // extern "C"
