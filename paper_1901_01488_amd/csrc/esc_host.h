// esc_host.h -- host-side objects behind the opaque handles of esc.h.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "esc.h"
#include "esc_program.h"

struct esc_table {
    uint64_t id = 0;   // unique per table handle (never reused)
    int64_t nrows = 0;
    std::vector<int32_t> dtypes;
    std::vector<const void *> cols;   // empty for a schema-only table
    bool has_data() const { return !cols.empty(); }
};

struct esc_pred {
    uint64_t id = 0;   // unique per predicate handle (never reused)
    esc::Program prog{};
    int ncols_schema = 0;
    std::vector<int32_t> schema_dtypes;
    // the source tree, kept for featurization
    std::vector<esc_node> nodes;
    std::vector<esc_const> consts;
    std::vector<esc_udf_insn> udf;
    uint64_t col_mask = 0;
    int nhashed = 0;   // IN-lists compiled to slot tables
};

namespace esc {

// thread-local error message; returns `status` so callers can `return fail(...)`
int fail(int status, const char *fmt, ...);
uint64_t next_handle_id();
void clear_error();

// host compiler (no HIP): fills p->prog from the tree
int compile(const esc_table *schema, const esc_node *nodes, int nnodes,
            const esc_const *consts, int nconsts, const esc_udf_insn *udf, int nudf,
            esc_pred *p);

// The top-level conjuncts of p (the children of a root AND; p itself
// otherwise), each compiled on its own, with their column slots mapped onto
// one common slot order (nslots, slot_col).
int split_conjuncts(const esc_pred *p, std::vector<Program> &out, int &nslots, int *slot_col);

}  // namespace esc
