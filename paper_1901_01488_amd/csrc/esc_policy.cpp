// esc_policy.cpp -- the materialization policy of a pushed-down selection
// (host only; needs no GPU).
//
// Section 2.1 keeps a selection's output as a temporary table only when
// enough rows are pruned and the table is large, with both limits set by
// the DBA.  Here the decision compares two costs in seconds from a model
// whose rates are measured on the device (the calibration times the
// library's own count, materialization and temporary-table scans), and the
// DBA's two parameters become the model's break-even points.  The
// materialization cost has two regimes, as the write pass has: below the
// dense fraction the projected values of the qualifying rows are gathered
// one by one, above it the projected columns are read whole.
#include <math.h>

#include "esc_host.h"

using esc::fail;

namespace {

bool model_ok(const esc_cost_model *m)
{
    if (!m) return false;
    const double v[] = {m->scan_bytes_per_s, m->fixed_s, m->sparse_row_s, m->dense_fraction,
                        m->dense_bytes_per_s, m->dense_row_s, m->tmp_bytes_per_s};
    for (double x : v)
        if (!isfinite(x)) return false;
    return m->scan_bytes_per_s > 0.0 && m->dense_bytes_per_s > 0.0 && m->tmp_bytes_per_s > 0.0 &&
           m->fixed_s >= 0.0 && m->sparse_row_s >= 0.0 && m->dense_row_s >= 0.0 && m->dense_fraction >= 0.0 &&
           m->dense_fraction <= 1.0;
}

bool shape_ok(int scan_cols, int proj_cols, int reuses)
{
    return scan_cols >= 1 && proj_cols >= 0 && reuses >= 1;
}

double t_scan(const esc_cost_model *m, double nrows, int k, int r)
{
    return (double)r * nrows * (4.0 * (double)k) / m->scan_bytes_per_s;
}

// seconds to read the temporary table's rows r times
double tmp_per_row(const esc_cost_model *m, int p, int r)
{
    return (double)r * (4.0 * (double)(1 + p)) / m->tmp_bytes_per_s;
}

// the dense regime's cost of reading the projected columns whole
double dense_cols(const esc_cost_model *m, double nrows, int p)
{
    return nrows * (4.0 * (double)p) / m->dense_bytes_per_s;
}

double t_mat(const esc_cost_model *m, double nrows, double count, int p, int r)
{
    const bool dense = count > 0.0 && count / nrows >= m->dense_fraction;   // nothing is read for no rows
    const double write = dense ? dense_cols(m, nrows, p) + count * m->dense_row_s : count * m->sparse_row_s;
    return m->fixed_s + write + count * tmp_per_row(m, p, r);
}

}  // namespace

extern "C" {

int esc_policy_keep(const esc_cost_model *m, const int64_t *nrows, const uint64_t *count, int n, int scan_cols,
                    int proj_cols, int reuses, uint8_t *keep, double *saving_s)
{
    if (!model_ok(m)) return fail(ESC_ERR_INVALID, "cost model: rates must be positive, costs non-negative, "
                                                   "dense_fraction in [0, 1]");
    if (n < 0 || (n > 0 && (!nrows || !count || !keep))) return fail(ESC_ERR_INVALID, "null argument");
    if (!shape_ok(scan_cols, proj_cols, reuses))
        return fail(ESC_ERR_INVALID, "need scan_cols >= 1, proj_cols >= 0, reuses >= 1");
    for (int i = 0; i < n; i++) {
        if (nrows[i] < 0 || count[i] > (uint64_t)nrows[i])
            return fail(ESC_ERR_INVALID, "selection %d: count %llu outside [0, nrows]", i,
                        (unsigned long long)count[i]);
    }
    for (int i = 0; i < n; i++) {
        const double s = t_scan(m, (double)nrows[i], scan_cols, reuses);
        const double c = t_mat(m, (double)nrows[i], (double)count[i], proj_cols, reuses);
        keep[i] = (uint8_t)(c < s);
        if (saving_s) saving_s[i] = s - c;
    }
    return ESC_OK;
}

int esc_policy_thresholds(const esc_cost_model *m, int64_t nrows, int scan_cols, int proj_cols, int reuses,
                          double *tau, double *min_rows)
{
    if (!model_ok(m)) return fail(ESC_ERR_INVALID, "cost model: rates must be positive, costs non-negative, "
                                                   "dense_fraction in [0, 1]");
    if (!tau || !min_rows || nrows < 0) return fail(ESC_ERR_INVALID, "null argument or nrows < 0");
    if (!shape_ok(scan_cols, proj_cols, reuses))
        return fail(ESC_ERR_INVALID, "need scan_cols >= 1, proj_cols >= 0, reuses >= 1");
    const double nr = (double)nrows;
    const double room = t_scan(m, nr, scan_cols, reuses) - m->fixed_s;
    const double tmp = tmp_per_row(m, proj_cols, reuses);
    double t = 0.0;
    if (nrows > 0 && room > 0.0) {
        // gather regime: T_mat - T_scan crosses 0 at s1
        const double per_sparse = m->sparse_row_s + tmp;
        const double s1 = per_sparse > 0.0 ? room / per_sparse / nr : 2.0;
        if (s1 < m->dense_fraction) {
            t = s1;
        } else {
            // keeping pays through the whole gather regime; dense regime crossing
            const double per_dense = m->dense_row_s + tmp;
            const double room_d = room - dense_cols(m, nr, proj_cols);
            const double s2 = per_dense > 0.0 ? room_d / per_dense / nr : (room_d > 0.0 ? 2.0 : -1.0);
            t = s2 < m->dense_fraction ? m->dense_fraction : s2;
        }
    }
    *tau = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    *min_rows = m->fixed_s * m->scan_bytes_per_s / ((double)reuses * (4.0 * (double)scan_cols));
    return ESC_OK;
}

}  // extern "C"
