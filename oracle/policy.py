"""CPU oracle of the materialization policy.

TEST INFRASTRUCTURE ONLY: used by tests, never by the product path.

Section 2.1 materializes a pushed-down selection only when it prunes
enough rows (the call overhead and the extra memory reads and writes must
be won back) and only on large tables; the paper leaves both limits to the
DBA.  The policy compares two times in seconds for a selection of c rows out
of N (s = c / N), p projected columns, k columns re-read, r later uses:

  re-reading the table at every use:
      T_scan = r * N * 4k / scan_bytes_per_s
  writing the temporary table once, then reading it at every use:
      T_mat  = fixed_s + W(c) + r * c * 4 (1 + p) / tmp_bytes_per_s
      W(c)   = c * sparse_row_s                                  if c = 0 or s < dense_fraction
               N * 4p / dense_bytes_per_s + c * dense_row_s       otherwise

(W mirrors the write pass: projected values are gathered row by row until
the projected columns are read whole).  Keep when T_mat < T_scan.  The DBA's
parameters become break-even points: tau = the selectivity below which
keeping pays (the crossing in the gathering regime if it comes before
dense_fraction, else dense_fraction if keeping no longer pays once the
columns are read whole, else the crossing in that regime; within [0, 1]),
and min_rows = the table size at which T_scan = fixed_s.  Arithmetic is
float64, left to right.
"""
from __future__ import annotations


def t_scan(m, n, k, r):
    return float(r) * float(n) * (4.0 * float(k)) / m["scan_bytes_per_s"]


def t_mat(m, n, c, p, r):
    n, c = float(n), float(c)
    if c > 0.0 and c / n >= m["dense_fraction"]:
        w = n * (4.0 * float(p)) / m["dense_bytes_per_s"] + c * m["dense_row_s"]
    else:
        w = c * m["sparse_row_s"]
    return m["fixed_s"] + w + c * (float(r) * (4.0 * float(1 + p)) / m["tmp_bytes_per_s"])


def keep(m, n, c, k, p, r):
    """(keep, saving_s) for one selection."""
    s = t_scan(m, n, k, r)
    cost = t_mat(m, n, c, p, r)
    return cost < s, s - cost


def thresholds(m, n, k, p, r):
    """(tau, min_rows)."""
    room = t_scan(m, n, k, r) - m["fixed_s"]
    tmp = float(r) * (4.0 * float(1 + p)) / m["tmp_bytes_per_s"]
    tau = 0.0
    if n > 0 and room > 0.0:
        per_sparse = m["sparse_row_s"] + tmp
        s1 = room / per_sparse / float(n) if per_sparse > 0.0 else 2.0
        if s1 < m["dense_fraction"]:
            tau = s1
        else:
            per_dense = m["dense_row_s"] + tmp
            room_d = room - float(n) * (4.0 * float(p)) / m["dense_bytes_per_s"]
            if per_dense > 0.0:
                s2 = room_d / per_dense / float(n)
            else:
                s2 = 2.0 if room_d > 0.0 else -1.0
            tau = m["dense_fraction"] if s2 < m["dense_fraction"] else s2
    tau = min(max(tau, 0.0), 1.0)
    min_rows = m["fixed_s"] * m["scan_bytes_per_s"] / (float(r) * (4.0 * float(k)))
    return tau, min_rows
