/*
 * esc.h -- C ABI of the MI355X (gfx950) exact selectivity computation library.
 *
 * Exact selectivity computation (ESC; Section 2, "Exact Selectivity
 * Computation") replaces a cardinality estimate by the exact answer of the
 * sub-query  SELECT COUNT(*) FROM R WHERE P  run at optimisation time, and
 * optionally keeps the qualifying rows, restricted to the pushed-down
 * projection, as a temporary table in GPU memory for reuse by the plan
 * (Section 2 and Section 2.1, "Selection Materialization").
 *
 * Conventions for every call:
 *  - every function returns an esc_status; out-parameters are written only
 *    on ESC_OK (the one exception, ESC_ERR_CAPACITY, is documented at
 *    esc_materialize); a message for the last failure of the calling thread
 *    is available from esc_last_error();
 *  - no C++ exception crosses this boundary and nothing aborts;
 *  - "device pointer" means memory of the GPU the context was created on
 *    (hipMalloc'd or a torch CUDA tensor); the caller owns every device
 *    buffer passed in (columns, outputs, workspaces) and keeps it alive for
 *    the duration of the call (of the batch, for batched handles); the
 *    library never frees them;
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *  - handles are created and destroyed by the library; a handle may be used
 *    from one thread at a time.
 */
#ifndef ESC_H
#define ESC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ESC_ABI_VERSION 8

/* Column types.  DATE32 is int32 days since 1970-01-01, compared as int32. */
typedef enum { ESC_INT32 = 0, ESC_DATE32 = 1, ESC_FLOAT32 = 2 } esc_dtype;

typedef enum {
    ESC_OK = 0,
    ESC_ERR_INVALID = -1,      /* malformed tree, bad index, null handle, bad size */
    ESC_ERR_TYPE = -2,         /* constant dtype differs from its column, float in a udf */
    ESC_ERR_CAPACITY = -3,     /* materialized rows exceed the output capacity */
    ESC_ERR_ALIGN = -4,        /* a device column is not 16-byte aligned */
    ESC_ERR_HIP = -5,          /* a HIP runtime call failed (message has the HIP error) */
    ESC_ERR_OOM = -6,          /* host or device allocation failed, or workspace too small */
    ESC_ERR_UNSUPPORTED = -7,  /* valid but beyond the compiled limits (see ESC_MAX_*) */
    ESC_ERR_TIMEOUT = -8       /* reserved: a bounded device wait expired */
} esc_status;

/* Limits of one compiled predicate. */
#define ESC_MAX_COLUMNS_PER_PRED 8   /* distinct columns referenced */
#define ESC_MAX_INSNS 64             /* device instructions after normalisation */
#define ESC_MAX_CONSTS 256           /* IN-list constants after de-duplication */
#define ESC_MAX_IN 64                /* constants in one IN-list */
#define ESC_MAX_CLAUSES 32           /* conjuncts after conversion to AND-of-ORs */
#define ESC_MAX_PROJ 8               /* projected columns of one materialization */
#define ESC_MAX_CONJ 32              /* top-level conjuncts split by esc_count_conjuncts */

/* ------------------------------------------------------------------ predicates
 *
 * The predicate language of the paper's example selection (Section 1):
 * equality, ranges, BETWEEN, OR-ed alternatives and a deterministic integer
 * user-defined function compared with a constant, combined with AND / OR;
 * plus IN-lists.  A predicate is an array of esc_node in pre-order: an
 * AND/OR node is followed by its `nchild` direct children (each with its own
 * subtree), a leaf has no children.
 *
 * Semantics:
 *  EQ  v == k      LT  v < k      GT  v > k      BETWEEN  k0 <= v && v <= k1
 *  IN  v equals some listed constant (duplicates allowed, list non-empty)
 *  int32/date32 compare as int32; float32 uses IEEE ordered comparisons
 *  (NaN matches nothing, -0.0 == +0.0, denormals compare exactly).
 *  UDF: an int32 expression over int32/date32 columns and constants,
 *  evaluated with two's-complement wrap-around, then compared like a leaf
 *  (op `cmp`, int32 constants).  No NULLs: every row participates.
 */
typedef enum {
    ESC_AND = 0, ESC_OR = 1, ESC_EQ = 2, ESC_LT = 3, ESC_GT = 4,
    ESC_BETWEEN = 5, ESC_IN = 6, ESC_UDF = 7
} esc_op;

typedef union { int32_t i; float f; uint32_t bits; } esc_value;

/* A typed constant: `dtype` must equal the dtype of the column it is
 * compared with (ESC_INT32 for udf comparisons and udf operands). */
typedef struct { int32_t dtype; esc_value v; } esc_const;

typedef struct {
    int32_t op;      /* esc_op */
    int32_t col;     /* EQ..IN: 0-based column index; otherwise ignored */
    int32_t nchild;  /* AND/OR: number of direct children (>= 1); otherwise 0 */
    int32_t cmp;     /* UDF: ESC_EQ..ESC_IN, the comparison of the udf value */
    int32_t k0, k1;  /* constants (indices into `consts`): EQ/LT/GT consts[k0];
                        BETWEEN lo = consts[k0], hi = consts[k1];
                        IN consts[k0 .. k0 + k1) (k1 = list length);
                        UDF: the same, according to `cmp` */
    int32_t u0, u1;  /* UDF: program udf[u0 .. u0 + u1) */
} esc_node;

/* udf program: an accumulator machine.  The first instruction is ESC_U_LOAD;
 * each later one sets acc = acc <op> operand.  The operand is a column
 * (src = ESC_U_COL, arg = column index, int32/date32 only) or an int32
 * constant (src = ESC_U_CONST, arg = value).  MOD is the truncated
 * remainder (sign of the dividend) by a positive constant; SHL / SHR shift
 * by a constant in [0, 31], SHR arithmetic.  Left-deep expressions such as
 * (31*B + D) mod 97 map onto it directly. */
typedef enum {
    ESC_U_LOAD = 0, ESC_U_ADD = 1, ESC_U_SUB = 2, ESC_U_MUL = 3, ESC_U_MOD = 4,
    ESC_U_AND = 5, ESC_U_OR = 6, ESC_U_XOR = 7, ESC_U_SHL = 8, ESC_U_SHR = 9
} esc_udf_op;
typedef enum { ESC_U_COL = 0, ESC_U_CONST = 1 } esc_udf_src;
typedef struct { int32_t op, src, arg; } esc_udf_insn;

typedef struct esc_ctx esc_ctx;
typedef struct esc_table esc_table;
typedef struct esc_pred esc_pred;
typedef struct esc_batch esc_batch;
typedef struct esc_mlp esc_mlp;

/* Message of the calling thread's last failure ("" if none).  The pointer
 * stays valid until the thread's next failing call. */
const char *esc_last_error(void);
int esc_abi_version(void);

/* ------------------------------------------------------------------ context */

/* Binds HIP device `device`, reads its properties and allocates a small
 * pinned host buffer for results.  ESC_ERR_HIP when the device is absent.
 * Kernel-shape settings are read from the environment here, once per
 * context (all optional; the defaults are the measured best on MI355X):
 *   ESC_COUNT_VARIANT 0..4   count kernel rows per lane and blocks per CU
 *                            (4: by column count, program length and use);
 *   ESC_BLOCKS_PER_CU n      count grid = n blocks per CU (default: occupancy);
 *   ESC_MAT_BLOCKS_PER_CU n  same for the materialization's write pass;
 *   ESC_NONTEMPORAL 0|1      non-temporal column loads;
 *   ESC_DENSE_SHIFT 0..12    write-pass dense threshold 2^-shift (default 7).
 * Outside the context: ESC_IN_HASH_MIN (compiler: smallest IN-list given a
 * slot table or bitmap, default 3, 0 = never) and ESC_AUTOTUNE_CACHE (a file
 * that keeps batched autotuning results between processes). */
int esc_ctx_create(int device, esc_ctx **out);
int esc_ctx_destroy(esc_ctx *ctx);
/* Number of compute units of the context's device. */
int esc_ctx_num_cus(const esc_ctx *ctx, int *out);
/* Fraction of a wave tile's rows that must qualify for the materialization
 * to read the tile's projected columns whole rather than gather them
 * (1/128 unless ESC_DENSE_SHIFT sets another power of two). */
int esc_ctx_dense_fraction(const esc_ctx *ctx, double *out);

/* ------------------------------------------------------------------ tables
 *
 * A column-wise in-memory table (Section 2: column-wise in-memory databases
 * read only the columns a query needs).  `dev_cols[c]` is a device pointer
 * to nrows 4-byte values of dtype dtypes[c], 16-byte aligned (else
 * ESC_ERR_ALIGN).  dev_cols == NULL creates a schema-only table: it can
 * compile and featurize predicates but not be scanned.  The table borrows
 * the column pointers.  0 <= nrows <= 2^31 - 1 (row ids are int32),
 * 1 <= ncols <= 64. */
int esc_table_create(int64_t nrows, int ncols, const int32_t *dtypes,
                     const void *const *dev_cols, esc_table **out);
int esc_table_destroy(esc_table *t);

/* ------------------------------------------------------------------ compile
 *
 * Validates and type-checks the tree against `schema`, converts it to an
 * AND of OR-clauses (distributing OR over AND; exact, since the language
 * has no negation), folds leaves that are constant (e.g. LT INT32_MIN, a
 * NaN bound, an empty BETWEEN), normalises each leaf to a range, bitmap or
 * set test and emits a wave-uniform device program.  Host only: works
 * without a GPU.  Errors: ESC_ERR_INVALID (structure, indices, empty IN,
 * udf modulus <= 0, shift outside [0,31], udf not starting with LOAD),
 * ESC_ERR_TYPE (constant dtype mismatch, float32 column in a udf),
 * ESC_ERR_UNSUPPORTED (more than the ESC_MAX_* limits). */
int esc_compile_predicate(const esc_table *schema, const esc_node *nodes, int nnodes,
                          const esc_const *consts, int nconsts,
                          const esc_udf_insn *udf, int nudf, esc_pred **out);
int esc_pred_destroy(esc_pred *p);

typedef struct {
    int32_t nclauses;     /* conjuncts after normalisation */
    int32_t ninsns;       /* device instructions */
    int32_t ncols;        /* distinct columns read by a scan */
    int32_t constant;     /* 0: data-dependent; 1: always true; -1: always false */
    uint64_t col_mask;    /* bit c set when column c is read (c < 64) */
    int32_t nhashed;      /* IN-lists tested by one table lookup (64-slot key
                             table or 2048-bit bitmap) instead of one compare
                             per constant */
    int32_t pad;
} esc_pred_info;
int esc_pred_get_info(const esc_pred *p, esc_pred_info *out);

/* ------------------------------------------------------------------ scans
 *
 * Workspace: device memory of at least esc_workspace_size() bytes, 256-byte
 * aligned, zero-filled before its first use (esc_workspace_init does that);
 * every successful call leaves it ready for the next call.  Calls that may
 * overlap in time (different streams) need distinct workspaces.  A workspace
 * sized for materialization (materialize = 1; about nrows/4 bytes) also
 * receives, from every esc_count, the qualifying-row count of each tile of
 * rows and the per-row truth values as bit masks.  kind: ESC_WS_COUNT
 * (esc_count, esc_join_count: 256 bytes), ESC_WS_MATERIALIZE
 * (esc_materialize; also serves esc_count), ESC_WS_CONJUNCTS
 * (esc_count_conjuncts: the conjunct programs and counters). */
#define ESC_WS_COUNT 0
#define ESC_WS_MATERIALIZE 1
#define ESC_WS_CONJUNCTS 2
int esc_workspace_size(const esc_table *t, int kind, size_t *bytes);
int esc_workspace_init(esc_ctx *ctx, void *dev_ws, size_t ws_bytes, void *stream);

/* Exact COUNT(*) of the selection (Section 2: the selectivity sub-query
 * with a temporary COUNT aggregate).  Blocks until the count is on the
 * host.  A predicate the compiler decided (always true or always false,
 * e.g. contradictory conjuncts on one column) or an empty table is
 * answered on the host without any GPU work.  With a materialization-sized workspace the per-tile counts and
 * truth masks are left in it for a following esc_materialize of the same
 * predicate. */
int esc_count(esc_ctx *ctx, const esc_table *t, const esc_pred *p,
              void *dev_ws, size_t ws_bytes, void *stream, uint64_t *out_count);

/* Same scan, asynchronous: the count is written to device memory
 * `dev_count` (8 bytes) in stream order; nothing waits. */
int esc_count_async(esc_ctx *ctx, const esc_table *t, const esc_pred *p,
                    void *dev_ws, size_t ws_bytes, void *stream, uint64_t *dev_count);

/* The count split in two calls, so that a caller can enqueue more work
 * (say, the next selection's count) before waiting for this result, and
 * the GPU does not idle while the host decides.  esc_count_begin enqueues
 * the scan of esc_count on the stream; its last block writes the count
 * into a pinned host word of the context, slot `slot` (0 <= slot <
 * ESC_COUNT_SLOTS), and an event is recorded behind it.  esc_count_end
 * waits for that event only (not for work enqueued later) and returns the
 * count.  A slot holds one count at a time: beginning on a slot whose
 * count was not taken gives ESC_ERR_INVALID, as does ending a slot with no
 * count in flight.  Tiles for a following esc_materialize are left as by
 * esc_count.  Errors as esc_count. */
#define ESC_COUNT_SLOTS 64
int esc_count_begin(esc_ctx *ctx, const esc_table *t, const esc_pred *p,
                    void *dev_ws, size_t ws_bytes, void *stream, int slot);
int esc_count_end(esc_ctx *ctx, int slot, uint64_t *out_count);

/* The selection together with its pushed-down projection (Section 2) kept
 * as a temporary table (Section 2.1): dev_rowids[r] is the r-th qualifying
 * row in ascending row order, dev_proj_out[j][r] the value of column
 * proj_cols[j] at that row, bit for bit.  Outputs are caller-owned device
 * buffers of `capacity` elements (rowids int32, projections 4 bytes).
 * Blocks until the count is on the host.  When the count exceeds
 * `capacity`, the first `capacity` rows are written, *out_count receives the
 * full count and ESC_ERR_CAPACITY is returned.  0 <= nproj <= ESC_MAX_PROJ;
 * dev_rowids may be NULL when only projections are wanted.
 * When the last scan on this workspace (an esc_count or esc_materialize)
 * was of the same table handle and predicate handle (the ESC flow: count,
 * decide, materialize),
 * its per-tile counts and truth masks are reused and the predicate's columns
 * are not read again, only the projected ones.  The count writes a
 * process-unique stamp into the workspace and the reuse happens only if the
 * workspace still holds it (checked on the device), so memory that was
 * freed and handed out again at the same address is counted afresh.  The
 * reuse assumes that neither the table's contents nor the rest of the
 * workspace were written in between (call esc_workspace_init after changing
 * them).  Otherwise the call counts first.  Needs a workspace of
 * esc_workspace_size(t, 1, ...) bytes. */
int esc_materialize(esc_ctx *ctx, const esc_table *t, const esc_pred *p,
                    const int32_t *proj_cols, int nproj, int32_t *dev_rowids,
                    void *const *dev_proj_out, uint64_t capacity,
                    void *dev_ws, size_t ws_bytes, void *stream, uint64_t *out_count);

/* Same materialization, asynchronous: everything is enqueued on `stream` and
 * nothing waits.  The full count is written to device memory `dev_count`
 * (8 bytes) in stream order; when it exceeds `capacity` only the first
 * `capacity` rows were written (the caller compares after synchronizing).
 * Argument checks and the workspace rules are those of esc_materialize. */
int esc_materialize_async(esc_ctx *ctx, const esc_table *t, const esc_pred *p,
                          const int32_t *proj_cols, int nproj, int32_t *dev_rowids,
                          void *const *dev_proj_out, uint64_t capacity,
                          void *dev_ws, size_t ws_bytes, void *stream, uint64_t *dev_count);

/* Allocation-free materialization, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same computation and outputs as
 * esc_materialize_async, with the workspace taken from a static device
 * array of ESC_NOALLOC_SCRATCH_BYTES bytes that the library holds on each
 * device it runs on until the process ends (its address is looked up once
 * per device by esc_ctx_create).  No device memory is allocated or freed by
 * this call.  Tables whose materialization workspace exceeds the array
 * (more than 65,074,176 rows for predicates that read five or more
 * columns, 130,148,352 otherwise) are rejected with ESC_ERR_CAPACITY and
 * nothing is enqueued.  Every call on a device shares that device's array:
 * calls that may overlap in time on one device (different streams, several
 * host threads, several contexts) race and must be serialized by the
 * caller.  A call counts first unless the array still holds this table's and
 * predicate's tiles from this context's previous call (checked on the
 * device by a stamp, as in esc_materialize). */
#define ESC_NOALLOC_SCRATCH_BYTES (16u << 20)
int esc_materialize_noalloc(esc_ctx *ctx, const esc_table *t, const esc_pred *p,
                            const int32_t *proj_cols, int nproj, int32_t *dev_rowids,
                            void *const *dev_proj_out, uint64_t capacity,
                            void *stream, uint64_t *dev_count);

/* Split selectivities of a conjunction, from one scan: for a predicate
 * whose root is AND with m children (any other predicate: m = 1),
 * conj_counts[i] = rows that satisfy child i alone and prefix_counts[i] =
 * rows that satisfy children 0..i together, so prefix_counts[m-1] is the
 * predicate's count.  Children are compiled separately (constant folding
 * applies per child); together they read at most 8 columns.  m <=
 * ESC_MAX_CONJ and m <= max_out, else ESC_ERR_UNSUPPORTED / ESC_ERR_INVALID;
 * *out_nconj = m.  Needs a workspace of esc_workspace_size(t,
 * ESC_WS_CONJUNCTS) bytes (256-byte aligned, any contents); blocks until the
 * counts are on the host. */
int esc_count_conjuncts(esc_ctx *ctx, const esc_table *t, const esc_pred *p, void *dev_ws, size_t ws_bytes,
                        void *stream, int max_out, uint64_t *conj_counts, uint64_t *prefix_counts,
                        int *out_nconj);

/* ------------------------------------------------------------------ batched
 *
 * Section 2 runs one selectivity sub-query for every table that carries a
 * selection; this runs many such sub-queries at once.  One persistent kernel
 * reads each table's columns once per predicate group and counts every
 * predicate of the group; the whole launch is captured in a hipGraph.
 * The batch keeps the tables' column pointers; its device memory (work
 * list, programs, counters) is a caller-owned workspace of at least
 * esc_batch_workspace_size() bytes, 256-byte aligned, that must outlive the
 * batch (any contents; the batch never frees it). */
typedef struct {
    int32_t autotune;        /* 1: time candidate configurations at create */
    int32_t block;           /* threads per block (256 or 512); 0 = default */
    int32_t rows_per_thread; /* 8 or 16; other values = 8 */
    int32_t group;           /* predicates evaluated per pass over a chunk; 0 = all of the table's */
    int32_t chunk_rows;      /* rows per work item; 0 = about 8 items per block of the grid */
    int32_t blocks_per_cu;   /* persistent blocks per compute unit; 0 = default */
    int32_t max_preds;       /* predicates the batch may hold after esc_batch_update; 0 = npreds */
    int32_t max_cols;        /* distinct columns a predicate group loads per tile: 4, 6 or 8 (fewer
                                register slots let more waves share a SIMD); 0 = the smallest that
                                holds every predicate; other values = 0.  Autotuning tries that
                                smallest and 8 */
} esc_batch_opts;

/* Workspace bytes of a batch of these predicates over these tables: room
 * for max(npreds, opts->max_preds) predicates and for the work list of every
 * plan the options (or the autotuner's candidates, and a choice cached for
 * these tables and predicates) can build.  A later esc_batch_update whose
 * plan needs a longer work list gets ESC_ERR_OOM.  opts may be NULL
 * (defaults).  Host only (plans are built, nothing is launched). */
int esc_batch_workspace_size(esc_ctx *ctx, const esc_table *const *tables, int ntables,
                             const esc_pred *const *preds, const int32_t *pred_table, int npreds,
                             const esc_batch_opts *opts, size_t *bytes);
int esc_batch_create(esc_ctx *ctx, const esc_table *const *tables, int ntables,
                     const esc_pred *const *preds, const int32_t *pred_table, int npreds,
                     const esc_batch_opts *opts, void *dev_ws, size_t ws_bytes, void *stream,
                     esc_batch **out);
/* Loads autotuner choices from a file written by earlier runs (the file that
 * the ESC_AUTOTUNE_CACHE environment variable names is loaded the same way
 * at the first autotuned esc_batch_create).  One entry per line: a key and
 * five or six integers (block, rows per thread, group, chunk rows, blocks
 * per CU, and max_cols, 0 when absent); entries whose values a batch would
 * not accept (block other than 256, rows per thread other than 8 or 16,
 * negative group, chunk rows or blocks per CU, max_cols other than 0, 4, 6
 * or 8) are skipped.  *accepted / *rejected (either may be NULL) count the
 * lines kept and skipped.  Host only.  Errors: ESC_ERR_INVALID (null path or
 * unreadable file). */
int esc_batch_tune_cache_load(const char *path, int *accepted, int *rejected);
/* New predicates over the same tables: pred_table gives the owner of each
 * (NULL keeps the previous owners, then npreds must not change).  The work
 * list is rebuilt; the captured graph is reused whenever its kernel and
 * grid are unchanged, so a new predicate set costs a few host-to-device
 * copies.  More predicates than the batch was created for, or a plan whose
 * work list does not fit the workspace, give ESC_ERR_OOM. */
int esc_batch_update(esc_batch *b, const esc_pred *const *preds, const int32_t *pred_table, int npreds,
                     void *stream);
/* Launches the graph and waits; out_counts[i] = exact count of preds[i]. */
int esc_batch_count(esc_batch *b, void *stream, uint64_t *out_counts);
/* The configuration in use (after tuning). */
int esc_batch_get_opts(const esc_batch *b, esc_batch_opts *out);
int esc_batch_destroy(esc_batch *b);

/* ------------------------------------------------------------------ learned gate
 *
 * Featurization of predicates into 64 float32 values: for each column c < 6
 *   [lsel, lo, hi, is_eq, is_lt, is_gt, is_between, in_mass, in_size/16, in_or]
 * then [n_conj/6, n_or/6, has_udf, n_leaves/16].  Bounds are fractions of
 * rows under a smoothed empirical CDF of the column, built from its catalog
 * minimum and maximum (col_min / col_max) and a row sample: col_sample holds
 * sample_size values per column for columns 0 .. min(ncols, 6) - 1, in the
 * column's dtype, any order (sample_size 0: no sample, the CDF is linear
 * between minimum and maximum).  lo / hi: the range the conjunction leaves
 * to the column (a cross-column OR bounds each of its columns that no plain
 * conjunct bounds); lsel = -ln(max(est, 1e-9)) / -ln(1e-9), est = hi - lo
 * (or the IN mass when smaller); in_mass: the CDF mass of the IN constants;
 * in_or: ordinal / 4 of the conjunct holding the OR (0 outside ORs).  Host
 * only.  Errors: ESC_ERR_INVALID (null arguments, negative sample_size,
 * minimum above maximum, a predicate compiled for another schema). */
int esc_featurize(const esc_table *schema, const esc_value *col_min, const esc_value *col_max,
                  const esc_value *col_sample, int sample_size, const esc_pred *const *preds, int npreds,
                  float *host_out);
/* The same featurization with the catalog's column CDFs built once
 * (esc_catalog_create takes the arguments esc_featurize takes for the
 * catalog, with the same errors); the features are identical bit for bit. */
typedef struct esc_catalog esc_catalog;
int esc_catalog_create(const esc_table *schema, const esc_value *col_min, const esc_value *col_max,
                       const esc_value *col_sample, int sample_size, esc_catalog **out);
int esc_catalog_destroy(esc_catalog *cat);
int esc_featurize_catalog(const esc_catalog *cat, const esc_pred *const *preds, int npreds, float *host_out);

/* MLP 64 -> 256 -> 256 -> 256 -> 1 (ReLU) predicting ln(selectivity).
 * bfloat16 MFMA operands, float32 accumulation, float32 master weights and
 * Adam state on the device.  Parameters are exchanged as one float32 array
 * in the order W1[64][256], b1[256], W2[256][256], b2[256], W3[256][256],
 * b3[256], W4[256], b4[1] (ESC_MLP_NPARAMS values, weights [fan_in][fan_out]).
 *
 * Memory is the caller's: the state (esc_mlp_state_bytes(), 256-byte
 * aligned device memory that must outlive the handle) holds the master
 * weights, the Adam moments and step count, and bfloat16 copies of the
 * weights; a training workspace (esc_mlp_workspace_bytes(batch), 256-byte
 * aligned) holds one minibatch's activations and deltas.  Inference needs no
 * workspace.  The library allocates no device memory here.  Calls on one
 * handle must not overlap in time. */
#define ESC_MLP_NPARAMS 148481
size_t esc_mlp_state_bytes(void);
/* 0 when batch is outside [1, 4096] */
size_t esc_mlp_workspace_bytes(int batch);
/* The estimator starts with all parameters zero. */
int esc_mlp_create(esc_ctx *ctx, void *dev_state, size_t state_bytes, esc_mlp **out);
int esc_mlp_destroy(esc_mlp *m);   /* the state memory stays the caller's */
int esc_mlp_set_params(esc_mlp *m, const float *host_params);   /* also resets Adam (moments and step) */
int esc_mlp_get_params(esc_mlp *m, float *host_params);
/* The whole training state: parameters, Adam first and second moments
 * (ESC_MLP_NPARAMS floats each, parameter order) and the number of Adam
 * steps taken.  get: any output may be NULL.  set: NULL moments mean zero. */
int esc_mlp_get_state(esc_mlp *m, float *host_params, float *host_adam_m, float *host_adam_v,
                      int64_t *steps);
int esc_mlp_set_state(esc_mlp *m, const float *host_params, const float *host_adam_m,
                      const float *host_adam_v, int64_t steps);
/* Checkpoint of the whole training state to a file: a header (8-byte magic
 * "ESCMLP01", uint32 version 1, uint32 parameter count, int64 Adam steps,
 * uint64 FNV-1a hash of the three arrays), then parameters, first and second
 * moments as float32 in host byte order.  Training resumed from a checkpoint
 * continues exactly as without the interruption.  esc_mlp_load rejects a
 * file of another size, magic, version or parameter count, or whose hash
 * does not match (ESC_ERR_INVALID; the estimator is then unchanged). */
int esc_mlp_save(esc_mlp *m, const char *path);
int esc_mlp_load(esc_mlp *m, const char *path);
/* yhat[i] for n rows of dev_x (n x 64 float32, device) into dev_yhat. */
int esc_mlp_predict(esc_mlp *m, const float *dev_x, int64_t n, float *dev_yhat, void *stream);
/* Training loss: mean over rows of the Huber loss of e = yhat - y with
 * threshold 1/2 (e^2 / 2 for |e| <= 1/2, (|e| - 1/4) / 2 beyond): squared
 * for small ln-selectivity errors, linear for large ones.
 * esc_mlp_gradients: its gradient over the n rows (1 <= n <= 4096), written
 * as a flat float32 array in the parameter order into dev_grads (device);
 * needs a workspace of esc_mlp_workspace_bytes(n).  Blocks until done. */
int esc_mlp_gradients(esc_mlp *m, const float *dev_x, const float *dev_y, int64_t n,
                      float *dev_grads, void *dev_ws, size_t ws_bytes, void *stream);
/* Minibatch Adam: `steps` steps; step s uses rows dev_order[s*batch ..
 * (s+1)*batch) of (dev_x, dev_y); batch in [1, 4096]; a workspace of
 * esc_mlp_workspace_bytes(batch).  dev_loss, if not NULL, is device memory
 * of `steps` floats that receives the mean loss of each step.  Adam betas
 * 0.9 / 0.999, eps 1e-8; the Adam step count continues across calls.
 * Deterministic: the same inputs give bit-identical weights.  Blocks until
 * done. */
int esc_mlp_train(esc_mlp *m, const float *dev_x, const float *dev_y, const int32_t *dev_order,
                  int64_t steps, int batch, float lr, void *dev_ws, size_t ws_bytes, void *stream,
                  float *dev_loss);

/* Gate (Section 2.1 and 2.2 read as plan-flip tests): route[i] = 1 when the
 * predicted selectivity s = clamp(exp(yhat[i]), 1/n, 1) of a table with
 * n = nrows[i] >= min_rows lies in [tau/beta, tau*beta], i.e. the push-down
 * decision "selectivity below tau" could flip within the estimator's error
 * factor beta (> 1). */
int esc_gate_pushdown(const float *yhat, const int64_t *nrows, int n, double tau, double beta,
                      int64_t min_rows, uint8_t *route);
/* route = 1 when the predicted filtered sizes of two build relations are
 * within a factor beta^2 of each other, so their join order could flip. */
int esc_gate_join_pair(float yhat_r, int64_t n_r, float yhat_s, int64_t n_s, double beta,
                       uint8_t *route);
/* esc_gate_join_pair for n queries (yhat_r[i], yhat_s[i] over build
 * relations of n_r and n_s rows), with ties: when both predicted
 * selectivities, raised by the error factor beta, are at most tie_sel, the
 * two join orders differ by at most tie_sel of the probe relation's rows
 * in the second hash lookup (Section 2.2 joins on the probed input, so the
 * first join passes sel * |P| rows on), and route[i] = 0 whatever the
 * order.  tie_sel = 0 disables ties.  Errors: ESC_ERR_INVALID (null
 * pointers with n > 0, n_r or n_s < 1, beta < 1, tie_sel outside [0, 1]). */
int esc_gate_join_pairs(const float *yhat_r, int64_t n_r, const float *yhat_s, int64_t n_s, int n,
                        double beta, double tie_sel, uint8_t *route);

/* ------------------------------------------------------------------ TEXT and DECIMAL columns
 *
 * Section 3 (Table 3) evaluates predicates on TEXT and DECIMAL(15,2)
 * columns beside INTEGER ones.  Both are stored as 4-byte columns, so the
 * scans keep their coalesced loads and exact int32 tests, and their
 * predicates are written on the stored values (dtype ESC_INT32):
 *  - TEXT is dictionary-coded: a column holds each value's code, its rank
 *    in the dictionary's byte-wise order, so string comparisons are code
 *    comparisons and a prefix is a code interval;
 *  - DECIMAL(p, s) holds value * 10^s as int32 (|value| * 10^s < 2^31), and
 *    a decimal literal becomes an exact int32 bound. */
typedef struct esc_dict esc_dict;
enum { ESC_DICT_PREFIX = 100 };   /* esc_dict_range: strings starting with s */

/* A dictionary of n distinct strings (any order; the dictionary sorts them
 * byte-wise).  Errors: ESC_ERR_INVALID (null pointers, duplicates). */
int esc_dict_create(const char *const *strings, int n, esc_dict **out);
int esc_dict_destroy(esc_dict *d);
int esc_dict_size(const esc_dict *d, int *n);
/* *code = rank of s, or -1 when s is not in the dictionary. */
int esc_dict_code(const esc_dict *d, const char *s, int32_t *code);
/* The string of a code (owned by the dictionary). */
int esc_dict_string(const esc_dict *d, int32_t code, const char **s);
/* Codes [*lo, *hi] of the strings x with: x = s (ESC_EQ), x < s (ESC_LT),
 * x > s (ESC_GT), s <= x <= s2 (ESC_BETWEEN), x starts with s
 * (ESC_DICT_PREFIX); byte-wise comparison.  None: *lo = 0, *hi = -1. */
int esc_dict_range(const esc_dict *d, int op, const char *s, const char *s2, int32_t *lo, int32_t *hi);
/* For a decimal literal c ([+-]digits[.digits]) and scale s: ESC_EQ: the
 * stored value equal to c (*empty = 1 when c has more than s nonzero
 * decimals, so nothing equals it); ESC_LT: the largest stored value below c;
 * ESC_GT: the smallest stored value above c.  Exact, no floating point.
 * A literal of 10^18 or more in stored units (literal * 10^s) saturates to
 * +-(10^18 + 1/2), which gives the same bounds for every stored value below
 * 10^18 in magnitude (all int32 values).
 * Errors: ESC_ERR_INVALID (bad literal, scale outside [0, 9]). */
int esc_decimal_bound(const char *literal, int scale, int op, int64_t *bound, int *empty);

/* Typed predicates: a predicate tree as for esc_compile_predicate whose
 * leaves on TEXT or DECIMAL columns compare with literals (strings) instead
 * of esc_const values; esc_lower_typed rewrites it into an ordinary tree on
 * the int32 storage (to pass to esc_compile_predicate with the same udf
 * program).  coltypes has one entry per schema column (NULL: all plain):
 *  - ESC_COL_TEXT (dict): the column holds dictionary codes; leaves EQ, LT,
 *    GT (literals[k0]), BETWEEN (literals[k0], literals[k1]), IN
 *    (literals[k0 .. k0 + k1)) and ESC_PREFIX (strings starting with
 *    literals[k0]), compared byte-wise;
 *  - ESC_COL_DECIMAL (scale): the column holds value * 10^scale in int32;
 *    leaves EQ, LT, GT, BETWEEN, IN with decimal literals
 *    ([+-]digits[.digits], any number of digits), compared exactly;
 *  - ESC_COL_DECIMAL64 (scale, low_col): value * 10^scale in int64 held as
 *    two word columns: this column the high 32 bits (signed), low_col the
 *    low 32 bits with the sign bit flipped (esc_decimal64_words); the same
 *    leaves, lowered to tests on both columns.
 * Leaves on plain columns and UDF leaves keep their esc_const constants.
 * The output consts are int32 (typed leaves) or copies of the input ones.
 * Errors: ESC_ERR_INVALID (indices, bad literal, missing dictionary),
 * ESC_ERR_TYPE (a prefix on a non-TEXT column, a typed column not stored as
 * int32), ESC_ERR_CAPACITY (output arrays too small: *out_nnodes and
 * *out_nconsts give the sizes needed).  Host only. */
typedef enum { ESC_COL_PLAIN = 0, ESC_COL_TEXT = 1, ESC_COL_DECIMAL = 2, ESC_COL_DECIMAL64 = 3 } esc_col_kind;
enum { ESC_PREFIX = 8 };   /* typed leaf op: TEXT prefix match */
typedef struct {
    int32_t kind;           /* esc_col_kind */
    int32_t scale;          /* DECIMAL, DECIMAL64: digits after the point, 0..9 */
    int32_t low_col;        /* DECIMAL64: column of the low words */
    int32_t pad;
    const esc_dict *dict;   /* TEXT */
} esc_col_type;
int esc_lower_typed(const esc_table *schema, const esc_col_type *coltypes, const esc_node *nodes, int nnodes,
                    const esc_const *consts, int nconsts, const char *const *literals, int nliterals,
                    esc_node *out_nodes, int max_nodes, int *out_nnodes, esc_const *out_consts, int max_consts,
                    int *out_nconsts);
/* The word columns of int64 values (host arrays): high[i] = values[i] >> 32,
 * low[i] = (low 32 bits) XOR 0x80000000 as int32, so that the order of the
 * values is the lexicographic order of (high, low) as int32 pairs. */
int esc_decimal64_words(const int64_t *values, int64_t n, int32_t *high, int32_t *low);

/* ------------------------------------------------------------------ hash join
 *
 * Section 2.2: a left-deep plan probes the largest relation and builds hash
 * tables on the others, whose pushed-down selections (Section 2.1) leave
 * them as temporary tables.  A hash table lives in caller-owned device
 * memory of esc_hash_table_bytes(nkeys) bytes: open addressing with linear
 * probing over a power of two of 8-byte slots, at least two per key and at
 * least 64; several rows may share a key.  The table keeps each key with
 * the index of its build row. */
int esc_hash_table_bytes(int64_t nkeys, size_t *bytes);
/* Clears the table and inserts dev_keys[0 .. nkeys) (device int32), enqueued
 * on `stream`.  Errors: ESC_ERR_INVALID (null pointers, nkeys < 0, a size not
 * from esc_hash_table_bytes, fewer than 2 * nkeys slots), ESC_ERR_UNSUPPORTED
 * (more than 2^30 keys). */
int esc_hash_build(esc_ctx *ctx, const int32_t *dev_keys, int64_t nkeys, void *dev_table, size_t table_bytes,
                   void *stream);
/* Rows of the star join of `probe` with ntables (1..4) build sides: the sum
 * over probe rows i of the product over j of the number of build rows of
 * table j whose key equals probe column key_cols[j] at row i (int32 or
 * date32 columns).  Waits for the result.  The product of one row must fit
 * in 64 bits.  The count is reduced in a workspace of at least
 * esc_workspace_size(probe, ESC_WS_COUNT, ...) bytes (256-byte aligned, any
 * contents).  Errors: ESC_ERR_INVALID, ESC_ERR_TYPE (a float32 key column),
 * ESC_ERR_ALIGN / ESC_ERR_OOM (workspace). */
int esc_join_count(esc_ctx *ctx, const esc_table *probe, const int32_t *key_cols, void *const *dev_tables,
                   const size_t *table_bytes, int ntables, void *dev_ws, size_t ws_bytes, void *stream,
                   uint64_t *out_count);

/* ------------------------------------------------------------------ materialization policy
 *
 * Section 2.1: materializing a pushed-down selection pays only when enough
 * rows are pruned (the call overhead and the extra memory traffic must be
 * won back) and only on tables large enough; the paper leaves the minimum
 * table size and the maximum selectivity to the DBA and names adaptive
 * choices as future work.  Here both follow from a cost model whose
 * parameters are measured on the device.  For a selection of count rows
 * out of nrows, s = count / nrows, p projected columns, k distinct columns
 * read by a re-read of the table and r later uses:
 *   without the temporary table, every use re-reads the table:
 *     T_scan = r * nrows * 4k / scan_bytes_per_s
 *   with it (the materialization gathers projected values while
 *   s < dense_fraction and reads the projected columns whole above):
 *     T_mat  = fixed_s + count * sparse_row_s          (count = 0 or s < dense_fraction)
 *            = fixed_s + nrows * 4p / dense_bytes_per_s + count * dense_row_s   (otherwise)
 *            + r * count * 4 (1 + p) / tmp_bytes_per_s     (reading row ids and values)
 * Keep (materialize) when T_mat < T_scan.  Every expression is evaluated
 * left to right in double precision. */
typedef struct {
    double scan_bytes_per_s;   /* streaming read rate of a selection scan */
    double fixed_s;            /* materialization cost per call (launches, offsets) */
    double sparse_row_s;       /* per qualifying row while projected values are gathered */
    double dense_fraction;     /* selectivity from which projected columns are read whole */
    double dense_bytes_per_s;  /* read rate of whole projected columns */
    double dense_row_s;        /* per qualifying row when columns are read whole */
    double tmp_bytes_per_s;    /* read rate of a temporary table */
} esc_cost_model;

/* keep[i] = 1 when materializing selection i is cheaper; saving_s[i] (may
 * be NULL) = T_scan - T_mat.  scan_cols (k), proj_cols (p) and reuses (r)
 * apply to all n selections.  Errors: ESC_ERR_INVALID (null pointers, n < 0,
 * nrows[i] < 0, count[i] > nrows[i], a rate not positive, a cost negative,
 * dense_fraction outside [0, 1], scan_cols < 1, proj_cols < 0, reuses < 1). */
int esc_policy_keep(const esc_cost_model *m, const int64_t *nrows, const uint64_t *count, int n, int scan_cols,
                    int proj_cols, int reuses, uint8_t *keep, double *saving_s);
/* The two DBA parameters of Section 2.1 implied by the model for a table
 * shape: *tau = the selectivity up to which materializing pays (keep holds
 * for every s < tau, in [0, 1]) and *min_rows = the smallest table on which
 * materializing even an empty result pays (T_scan > fixed_s). */
int esc_policy_thresholds(const esc_cost_model *m, int64_t nrows, int scan_cols, int proj_cols, int reuses,
                          double *tau, double *min_rows);

#ifdef __cplusplus
}
#endif
#endif /* ESC_H */
