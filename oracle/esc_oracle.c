/*
 * esc_oracle.c -- plain, single-threaded CPU oracle for exact selectivity
 * computation (ESC).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or table with the GPU path.
 *
 * What it computes (Section 2, "Exact Selectivity Computation"): the exact
 * cardinality of a selection sigma_P(R), i.e. the value of
 *     SELECT COUNT(*) FROM R WHERE P
 * and, for the pushed-down projection of Section 2 / Section 2.1, the rows of
 *     SELECT <projected columns> FROM R WHERE P
 * kept in row order as a temporary table.  Both are written out here as their
 * plain definitions: one pass over the rows 0..N-1, evaluating P recursively
 * on each row.  No blocking, no reordering, no short-cut beyond what C's &&
 * and || already do (every leaf is total, so skipping is unobservable).
 *
 * Predicate language (Section 1, the example selection over R.B, R.C, R.D):
 * equality, range (BETWEEN, inclusive at both ends), OR, AND, IN-lists and a
 * deterministic integer user-defined function compared with a constant.
 * The oracle reads its own textual S-expression form:
 *
 *   P := (and P P ...) | (or P P ...)
 *      | (eq c K) | (lt c K) | (gt c K) | (between c K K) | (in c K K ...)
 *      | (udf E T)
 *   T := (eq K) | (lt K) | (gt K) | (between K K) | (in K K ...)
 *   E := (col c) | (const K) | (add E E) | (sub E E) | (mul E E) | (mod E E)
 *      | (band E E) | (bor E E) | (bxor E E) | (shl E E) | (shr E E)
 *
 * c is a 0-based column index.  K is a decimal int32 for int32/date32
 * columns (and for every udf constant) and "fx" + 8 hex digits (the IEEE-754
 * bit pattern) for float32 columns.
 *
 * Semantics (readings of points the paper leaves open):
 *  - no NULLs; every value participates;
 *  - BETWEEN a b  is  a <= v && v <= b  (empty when a > b);
 *  - float32 comparisons are the IEEE ordered ones: NaN matches nothing,
 *    -0.0 == +0.0, denormals compare exactly (no flush to zero);
 *  - udf arithmetic is int32 two's-complement with wrap-around, computed in
 *    uint32_t; mod is the truncated remainder (sign of the dividend) and
 *    needs a positive divisor; shift amounts must lie in [0,31]; shr is the
 *    arithmetic (sign-propagating) shift; float columns may not feed a udf.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#include <ctype.h>

enum { DT_INT32 = 0, DT_DATE32 = 1, DT_FLOAT32 = 2 };

enum {
    N_AND, N_OR, N_EQ, N_LT, N_GT, N_BETWEEN, N_IN, N_UDF,
    X_COL, X_CONST, X_ADD, X_SUB, X_MUL, X_MOD, X_BAND, X_BOR, X_BXOR, X_SHL, X_SHR
};

typedef struct onode {
    int kind;
    int col;              /* leaf column, or X_COL column */
    int nkid;
    struct onode **kid;   /* AND/OR children; UDF: kid[0]=expr, kid[1]=test; binary exprs: 2 */
    int nk;
    uint32_t *k;          /* constants as raw 32-bit patterns */
    int test;             /* UDF test node kind (N_EQ..N_IN), stored in kid[1]->kind */
} onode;

static char g_err[512];

static void set_err(const char *msg, const char *at)
{
    snprintf(g_err, sizeof g_err, "%s%s%.40s", msg, at ? " near: " : "", at ? at : "");
}

const char *oracle_error(void) { return g_err; }

/* ------------------------------------------------------------------ parse */

typedef struct {
    const char *s;
    int ncols;
    const int32_t *dtypes;
    int fail;
} parser;

static void skip_ws(parser *p) { while (*p->s && isspace((unsigned char)*p->s)) p->s++; }

static int expect(parser *p, char c)
{
    skip_ws(p);
    if (*p->s != c) { set_err(c == '(' ? "expected '('" : "expected ')'", p->s); p->fail = 1; return 0; }
    p->s++;
    return 1;
}

static int peek_close(parser *p) { skip_ws(p); return *p->s == ')'; }

static int read_word(parser *p, char *buf, int cap)
{
    skip_ws(p);
    int n = 0;
    while (*p->s && !isspace((unsigned char)*p->s) && *p->s != '(' && *p->s != ')') {
        if (n + 1 >= cap) { set_err("token too long", p->s); p->fail = 1; return 0; }
        buf[n++] = *p->s++;
    }
    buf[n] = 0;
    if (n == 0) { set_err("expected a token", p->s); p->fail = 1; return 0; }
    return 1;
}

static int read_int(parser *p, int64_t lo, int64_t hi, int64_t *out)
{
    char buf[64];
    if (!read_word(p, buf, sizeof buf)) return 0;
    char *end = NULL;
    long long v = strtoll(buf, &end, 10);
    if (*end != 0 || v < lo || v > hi) { set_err("bad integer", buf); p->fail = 1; return 0; }
    *out = v;
    return 1;
}

/* a constant in the dtype of column col (col < 0: int32, as in a udf) */
static int read_const(parser *p, int col, uint32_t *out)
{
    char buf[64];
    if (!read_word(p, buf, sizeof buf)) return 0;
    int is_float = col >= 0 && p->dtypes[col] == DT_FLOAT32;
    if (is_float) {
        if (buf[0] != 'f' || buf[1] != 'x' || strlen(buf) != 10) {
            set_err("float32 column needs an fx<8 hex> constant", buf); p->fail = 1; return 0;
        }
        char *end = NULL;
        unsigned long v = strtoul(buf + 2, &end, 16);
        if (*end != 0) { set_err("bad hex constant", buf); p->fail = 1; return 0; }
        *out = (uint32_t)v;
        return 1;
    }
    if (buf[0] == 'f') { set_err("int column needs a decimal constant", buf); p->fail = 1; return 0; }
    char *end = NULL;
    long long v = strtoll(buf, &end, 10);
    if (*end != 0 || v < INT32_MIN || v > INT32_MAX) { set_err("bad int32 constant", buf); p->fail = 1; return 0; }
    *out = (uint32_t)(int32_t)v;
    return 1;
}

static onode *new_node(int kind)
{
    onode *n = (onode *)calloc(1, sizeof *n);
    n->kind = kind;
    n->col = -1;
    return n;
}

static void free_node(onode *n)
{
    if (!n) return;
    for (int i = 0; i < n->nkid; i++) free_node(n->kid[i]);
    free(n->kid);
    free(n->k);
    free(n);
}

static void add_kid(onode *n, onode *k)
{
    n->kid = (onode **)realloc(n->kid, sizeof(onode *) * (size_t)(n->nkid + 1));
    n->kid[n->nkid++] = k;
}

static void add_k(onode *n, uint32_t v)
{
    n->k = (uint32_t *)realloc(n->k, sizeof(uint32_t) * (size_t)(n->nk + 1));
    n->k[n->nk++] = v;
}

static int kind_of(const char *w)
{
    static const char *names[] = { "and", "or", "eq", "lt", "gt", "between", "in", "udf",
                                   "col", "const", "add", "sub", "mul", "mod", "band", "bor",
                                   "bxor", "shl", "shr" };
    for (int i = 0; i < (int)(sizeof names / sizeof names[0]); i++)
        if (strcmp(w, names[i]) == 0) return i;
    return -1;
}

/* constants of a comparison: how many follow the operator */
static int read_cmp_consts(parser *p, onode *n, int col)
{
    uint32_t v;
    switch (n->kind) {
    case N_EQ: case N_LT: case N_GT:
        if (!read_const(p, col, &v)) return 0;
        add_k(n, v);
        return 1;
    case N_BETWEEN:
        for (int i = 0; i < 2; i++) { if (!read_const(p, col, &v)) return 0; add_k(n, v); }
        return 1;
    case N_IN:
        while (!peek_close(p)) {
            if (!read_const(p, col, &v)) return 0;
            add_k(n, v);
        }
        if (n->nk == 0) { set_err("empty IN list", p->s); p->fail = 1; return 0; }
        return 1;
    }
    return 0;
}

static onode *parse_expr(parser *p)
{
    char w[32];
    if (!expect(p, '(')) return NULL;
    if (!read_word(p, w, sizeof w)) return NULL;
    int kind = kind_of(w);
    if (kind < X_COL) { set_err("not a udf expression", w); p->fail = 1; return NULL; }
    onode *n = new_node(kind);
    if (kind == X_COL) {
        int64_t c;
        if (!read_int(p, 0, p->ncols - 1, &c)) { free_node(n); return NULL; }
        if (p->dtypes[c] == DT_FLOAT32) { set_err("float32 column inside a udf", w); p->fail = 1; free_node(n); return NULL; }
        n->col = (int)c;
    } else if (kind == X_CONST) {
        uint32_t v;
        if (!read_const(p, -1, &v)) { free_node(n); return NULL; }
        add_k(n, v);
    } else {
        for (int i = 0; i < 2; i++) {
            onode *k = parse_expr(p);
            if (!k) { free_node(n); return NULL; }
            add_kid(n, k);
        }
    }
    if (!expect(p, ')')) { free_node(n); return NULL; }
    return n;
}

static onode *parse_pred(parser *p)
{
    char w[32];
    if (!expect(p, '(')) return NULL;
    if (!read_word(p, w, sizeof w)) return NULL;
    int kind = kind_of(w);
    if (kind < 0 || kind > N_UDF) { set_err("unknown predicate operator", w); p->fail = 1; return NULL; }
    onode *n = new_node(kind);
    if (kind == N_AND || kind == N_OR) {
        while (!peek_close(p)) {
            onode *k = parse_pred(p);
            if (!k) { free_node(n); return NULL; }
            add_kid(n, k);
        }
        if (n->nkid == 0) { set_err("empty and/or", p->s); p->fail = 1; free_node(n); return NULL; }
    } else if (kind == N_UDF) {
        onode *e = parse_expr(p);
        if (!e) { free_node(n); return NULL; }
        add_kid(n, e);
        if (!expect(p, '(')) { free_node(n); return NULL; }
        if (!read_word(p, w, sizeof w)) { free_node(n); return NULL; }
        int tk = kind_of(w);
        if (tk < N_EQ || tk > N_IN) { set_err("bad udf comparison", w); p->fail = 1; free_node(n); return NULL; }
        onode *t = new_node(tk);
        add_kid(n, t);
        if (!read_cmp_consts(p, t, -1) || !expect(p, ')')) { free_node(n); return NULL; }
        n->test = tk;
    } else {
        int64_t c;
        if (!read_int(p, 0, p->ncols - 1, &c)) { free_node(n); return NULL; }
        n->col = (int)c;
        if (!read_cmp_consts(p, n, n->col)) { free_node(n); return NULL; }
    }
    if (!expect(p, ')')) { free_node(n); return NULL; }
    return n;
}

static onode *parse_all(const char *text, int ncols, const int32_t *dtypes)
{
    for (int c = 0; c < ncols; c++)
        if (dtypes[c] != DT_INT32 && dtypes[c] != DT_DATE32 && dtypes[c] != DT_FLOAT32) {
            set_err("unknown column dtype", NULL);
            return NULL;
        }
    parser p = { text, ncols, dtypes, 0 };
    onode *root = parse_pred(&p);
    if (!root) return NULL;
    skip_ws(&p);
    if (*p.s) { set_err("trailing text", p.s); free_node(root); return NULL; }
    return root;
}

/* --------------------------------------------------------------- evaluate */

typedef struct {
    int64_t n;
    const int32_t *dtypes;
    const void *const *cols;
    int fail;  /* run-time udf error: modulus <= 0 or shift out of range */
} table;

static float as_f32(uint32_t bits) { float f; memcpy(&f, &bits, 4); return f; }

static uint32_t cell(const table *t, int c, int64_t i) { return ((const uint32_t *)t->cols[c])[i]; }

/* the comparison of an int32 value against the node's constants */
static int cmp_int(int kind, int32_t v, const uint32_t *k, int nk)
{
    switch (kind) {
    case N_EQ: return v == (int32_t)k[0];
    case N_LT: return v < (int32_t)k[0];
    case N_GT: return v > (int32_t)k[0];
    case N_BETWEEN: return (int32_t)k[0] <= v && v <= (int32_t)k[1];
    case N_IN:
        for (int j = 0; j < nk; j++) if (v == (int32_t)k[j]) return 1;
        return 0;
    }
    return 0;
}

static int cmp_f32(int kind, float v, const uint32_t *k, int nk)
{
    switch (kind) {
    case N_EQ: return v == as_f32(k[0]);
    case N_LT: return v < as_f32(k[0]);
    case N_GT: return v > as_f32(k[0]);
    case N_BETWEEN: return as_f32(k[0]) <= v && v <= as_f32(k[1]);
    case N_IN:
        for (int j = 0; j < nk; j++) if (v == as_f32(k[j])) return 1;
        return 0;
    }
    return 0;
}

static uint32_t eval_expr(table *t, const onode *e, int64_t i)
{
    switch (e->kind) {
    case X_COL: return cell(t, e->col, i);
    case X_CONST: return e->k[0];
    }
    uint32_t a = eval_expr(t, e->kid[0], i);
    uint32_t b = eval_expr(t, e->kid[1], i);
    switch (e->kind) {
    case X_ADD: return a + b;
    case X_SUB: return a - b;
    case X_MUL: return a * b;
    case X_BAND: return a & b;
    case X_BOR: return a | b;
    case X_BXOR: return a ^ b;
    case X_MOD:
        if ((int32_t)b <= 0) { t->fail = 1; return 0; }
        return (uint32_t)((int32_t)a % (int32_t)b);
    case X_SHL:
        if (b > 31u) { t->fail = 1; return 0; }
        return a << b;
    case X_SHR:
        if (b > 31u) { t->fail = 1; return 0; }
        /* arithmetic shift written without relying on implementation-defined >> */
        if ((int32_t)a >= 0) return a >> b;
        return ~((~a) >> b);
    }
    t->fail = 1;
    return 0;
}

static int eval_pred(table *t, const onode *p, int64_t i)
{
    switch (p->kind) {
    case N_AND:
        for (int j = 0; j < p->nkid; j++) if (!eval_pred(t, p->kid[j], i)) return 0;
        return 1;
    case N_OR:
        for (int j = 0; j < p->nkid; j++) if (eval_pred(t, p->kid[j], i)) return 1;
        return 0;
    case N_UDF: {
        int32_t v = (int32_t)eval_expr(t, p->kid[0], i);
        return cmp_int(p->test, v, p->kid[1]->k, p->kid[1]->nk);
    }
    default:
        if (t->dtypes[p->col] == DT_FLOAT32)
            return cmp_f32(p->kind, as_f32(cell(t, p->col, i)), p->k, p->nk);
        return cmp_int(p->kind, (int32_t)cell(t, p->col, i), p->k, p->nk);
    }
}

/* ------------------------------------------------------------------- API */

/* Per-row truth values: mask[i] = P(row i) for i in [0, n).  Returns 0 or -1. */
int oracle_eval_rows(int64_t n, int ncols, const int32_t *dtypes, const void *const *cols,
                     const char *pred, uint8_t *mask)
{
    if (n < 0 || ncols <= 0 || !dtypes || !pred) { set_err("bad arguments", NULL); return -1; }
    onode *root = parse_all(pred, ncols, dtypes);
    if (!root) return -1;
    table t = { n, dtypes, cols, 0 };
    for (int64_t i = 0; i < n; i++) mask[i] = (uint8_t)eval_pred(&t, root, i);
    free_node(root);
    if (t.fail) { set_err("udf: modulus <= 0 or shift outside [0,31]", NULL); return -1; }
    return 0;
}

/* COUNT(*) of the selection: #{ i in [0,n) : P(row i) }.  Returns 0 or -1. */
int oracle_count(int64_t n, int ncols, const int32_t *dtypes, const void *const *cols,
                 const char *pred, uint64_t *out_count)
{
    if (n < 0 || ncols <= 0 || !dtypes || !pred || !out_count) { set_err("bad arguments", NULL); return -1; }
    onode *root = parse_all(pred, ncols, dtypes);
    if (!root) return -1;
    table t = { n, dtypes, cols, 0 };
    uint64_t c = 0;
    for (int64_t i = 0; i < n; i++) c += (uint64_t)eval_pred(&t, root, i);
    free_node(root);
    if (t.fail) { set_err("udf: modulus <= 0 or shift outside [0,31]", NULL); return -1; }
    *out_count = c;
    return 0;
}

/* The selection with its pushed-down projection, kept in row order:
 * rowids[r] = r-th qualifying row index (ascending), proj_out[j][r] =
 * column proj[j] at that row, bit for bit.  At most `capacity` rows are
 * written; *out_count always receives the full count.  Returns 0, -1 on
 * error, or 1 when the count exceeds capacity. */
int oracle_materialize(int64_t n, int ncols, const int32_t *dtypes, const void *const *cols,
                       const char *pred, int nproj, const int32_t *proj, int32_t *rowids,
                       void *const *proj_out, uint64_t capacity, uint64_t *out_count)
{
    if (n < 0 || ncols <= 0 || !dtypes || !pred || !out_count || nproj < 0) { set_err("bad arguments", NULL); return -1; }
    for (int j = 0; j < nproj; j++)
        if (proj[j] < 0 || proj[j] >= ncols) { set_err("projected column out of range", NULL); return -1; }
    onode *root = parse_all(pred, ncols, dtypes);
    if (!root) return -1;
    table t = { n, dtypes, cols, 0 };
    uint64_t c = 0;
    for (int64_t i = 0; i < n; i++) {
        if (!eval_pred(&t, root, i)) continue;
        if (c < capacity) {
            rowids[c] = (int32_t)i;
            for (int j = 0; j < nproj; j++)
                ((uint32_t *)proj_out[j])[c] = cell(&t, proj[j], i);
        }
        c++;
    }
    free_node(root);
    if (t.fail) { set_err("udf: modulus <= 0 or shift outside [0,31]", NULL); return -1; }
    *out_count = c;
    return c > capacity ? 1 : 0;
}

/* Syntax and type check only (no data).  Returns 0 or -1. */
int oracle_check(int ncols, const int32_t *dtypes, const char *pred)
{
    onode *root = parse_all(pred, ncols, dtypes);
    if (!root) return -1;
    free_node(root);
    return 0;
}
