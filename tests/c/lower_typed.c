/* A C caller of libesc lowers a Table 3 predicate on a 64-bit DECIMAL(15,2)
 * column (value * 100 in int64, held as the word columns H and L) and a TEXT
 * prefix, then compiles the result: host only, no Python anywhere.
 * Exit status 0 when every check holds; prints the first failure. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "esc.h"

#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            printf("check failed at line %d: %s (%s)\n", __LINE__, #cond, \
                   esc_last_error());                                      \
            return 1;                                                      \
        }                                                                  \
    } while (0)

static int leaf_is(const esc_node *n, const esc_const *c, int op, int col, int32_t a, int32_t b)
{
    if (n->op != op || n->col != col || c[n->k0].dtype != ESC_INT32 || c[n->k0].v.i != a) return 0;
    return op != ESC_BETWEEN || c[n->k1].v.i == b;
}

int main(void)
{
    /* columns: 0 TEXT codes, 1 H, 2 L */
    const int32_t dtypes[3] = {ESC_INT32, ESC_INT32, ESC_INT32};
    esc_table *schema = NULL;
    CHECK(esc_table_create(0, 3, dtypes, NULL, &schema) == ESC_OK);
    const char *words[4] = {"brass", "brown", "copper", "bronze"};
    esc_dict *d = NULL;
    CHECK(esc_dict_create(words, 4, &d) == ESC_OK);
    esc_col_type types[3];
    memset(types, 0, sizeof types);
    types[0].kind = ESC_COL_TEXT;
    types[0].dict = d;
    types[1].kind = ESC_COL_DECIMAL64;
    types[1].scale = 2;
    types[1].low_col = 2;

    /* price BETWEEN 1.00 AND 42949672.96 (stored 100 .. 2^32) AND name LIKE 'br%' */
    esc_node in[3];
    memset(in, 0, sizeof in);
    in[0].op = ESC_AND;
    in[0].nchild = 2;
    in[1].op = ESC_BETWEEN;
    in[1].col = 1;
    in[1].k0 = 0;
    in[1].k1 = 1;
    in[2].op = ESC_PREFIX;
    in[2].col = 0;
    in[2].k0 = 2;
    const char *lits[3] = {"1.00", "42949672.96", "br"};
    esc_node out[32];
    esc_const consts[32];
    int nn = 0, nc = 0;
    CHECK(esc_lower_typed(schema, types, in, 3, NULL, 0, lits, 3, out, 32, &nn, consts, 32, &nc) == ESC_OK);

    /* 100 = (H 0, L 100 ^ 2^31), 2^32 = (H 1, L 0 ^ 2^31):
     * AND[ AND[ H in [0,1], OR[H > 0, L >= lo_L], OR[H < 1, L <= hi_L] ], code in [0, 2] ] */
    const int32_t lo_l = (int32_t)(100u ^ 0x80000000u), hi_l = (int32_t)0x80000000u;
    CHECK(nn == 10);
    CHECK(out[0].op == ESC_AND && out[0].nchild == 2);
    CHECK(out[1].op == ESC_AND && out[1].nchild == 3);
    CHECK(leaf_is(&out[2], consts, ESC_BETWEEN, 1, 0, 1));
    CHECK(out[3].op == ESC_OR && out[3].nchild == 2);
    CHECK(leaf_is(&out[4], consts, ESC_GT, 1, 0, 0));
    CHECK(leaf_is(&out[5], consts, ESC_BETWEEN, 2, lo_l, INT32_MAX));
    CHECK(out[6].op == ESC_OR && out[6].nchild == 2);
    CHECK(leaf_is(&out[7], consts, ESC_LT, 1, 1, 0));
    CHECK(leaf_is(&out[8], consts, ESC_BETWEEN, 2, INT32_MIN, hi_l));
    /* sorted: brass, bronze, brown, copper: 'br%' = codes 0 .. 2 */
    CHECK(leaf_is(&out[9], consts, ESC_BETWEEN, 0, 0, 2));

    /* the lowered tree compiles into a device program */
    esc_pred *p = NULL;
    CHECK(esc_compile_predicate(schema, out, nn, consts, nc, NULL, 0, &p) == ESC_OK);
    esc_pred_info info;
    CHECK(esc_pred_get_info(p, &info) == ESC_OK);
    CHECK(info.constant == 0 && info.col_mask == 7u);

    /* word columns of a few int64 values */
    const int64_t v[3] = {100, 4294967296LL, -1};
    int32_t h[3], l[3];
    CHECK(esc_decimal64_words(v, 3, h, l) == ESC_OK);
    CHECK(h[0] == 0 && l[0] == lo_l && h[1] == 1 && l[1] == hi_l && h[2] == -1 && l[2] == INT32_MAX);

    esc_pred_destroy(p);
    esc_dict_destroy(d);
    esc_table_destroy(schema);
    printf("ok\n");
    return 0;
}
