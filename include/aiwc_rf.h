/*
 * aiwc_rf.h -- C ABI of the MI355X (gfx950) random-forest performance model.
 *
 * The model is the one of Sec. III-B of "OpenCL Performance Prediction using
 * Architecture-Independent Features" (Johnston & Milthorpe, 2018): a random-forest
 * regression that maps the AIWC feature vector of an OpenCL kernel (Table I) plus
 * the device it runs on (Table II) to its execution time, with the three ranger
 * parameters num.trees, mtry and min.node.size.  The calls follow the problem as
 * the paper states it (Abstract; Sec. I; Sec. VI): features and a device id in,
 * a predicted execution time out; fitting happens once, querying is cheap.
 *
 * Conventions shared by every call:
 *   - Return value: AIWC_RF_OK (0) or a negative AIWC_RF_E* code.  The message of
 *     the last failure on the calling thread is returned by aiwc_rf_last_error().
 *     No C++ exception crosses this boundary.
 *   - Array arguments are DEVICE pointers (hipMalloc'ed or any device tensor's
 *     storage) unless the argument name ends in _host.  Device arrays must live on
 *     the current HIP device.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Work
 *     is enqueued on it; a call returns once its results are complete unless the
 *     call says otherwise.
 *   - Handles are opaque, owned by the library and released with the matching
 *     *_free call.  Outputs are caller-allocated.  A fitted forest is immutable, so
 *     predictions from several threads and streams may run concurrently.
 *
 * Numerical contract (identical, bit for bit, to the separate CPU oracle):
 *   - the response y (log10 seconds) is carried as int64 fixed point
 *     y_fp = rint(y * 2^16); |y| <= 64 is required;
 *   - node sums of weight N, response S and squared response Q are exact integers;
 *   - a split maximises S_L^2/N_L + S_R^2/N_R (variance reduction) evaluated in
 *     IEEE binary64 without contraction; ties keep the lowest (column, bin);
 *   - a leaf holds its mean as q = round-half-away(S * 2^16 / N) (units 2^-32);
 *     the prediction is (sum of q over trees) * 2^-32 / num.trees, one rounding.
 */
#ifndef AIWC_RF_H
#define AIWC_RF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define AIWC_RF_OK 0
#define AIWC_RF_EINVAL (-1) /* bad argument: null pointer, size or parameter out of range, NaN feature */
#define AIWC_RF_ERANGE (-2) /* response non-finite or |y| > 64, or an internal capacity limit hit */
#define AIWC_RF_ENOMEM (-3) /* device or host allocation failed, or a memory budget would be exceeded */
#define AIWC_RF_EHIP (-4)   /* a HIP runtime call failed; the message carries HIP's error string */
#define AIWC_RF_ESTATE (-5) /* handle used in a state that does not allow the call */

/* Limits.  Rows: the fixed-point budget keeps |S| <= 2^40 and Q <= 2^62 exact. */
#define AIWC_RF_MAX_ROWS (1 << 18)
#define AIWC_RF_LEAF 255 /* column value that marks a leaf in node words and exported node arrays */
#define AIWC_RF_MAX_COLS 255 /* code columns (features + device): column ids stay below AIWC_RF_LEAF */
#define AIWC_RF_MAX_FEATURES (AIWC_RF_MAX_COLS - 1)
#define AIWC_RF_MAX_BINS 256
#define AIWC_RF_MAX_TREES (1 << 14)

typedef struct aiwc_rf_binner aiwc_rf_binner; /* per-column thresholds and bin counts */
typedef struct aiwc_rf_forest aiwc_rf_forest; /* one or many fitted forests, device resident */

/* The three model parameters of Sec. III-B (num.trees, mtry, min.node.size), the
 * bootstrap switch and the seed of the Philox4x64-10 streams that draw the
 * bootstrap sample (counter (block, 0, 0, tree)) and each node's mtry candidate
 * columns (counter (block, 1, node, tree)), key (seed, 0). */
typedef struct {
  int32_t num_trees;     /* 1 .. AIWC_RF_MAX_TREES */
  int32_t mtry;          /* 1 .. number of code columns (features + device) */
  int32_t min_node_size; /* >= 1; a node whose bootstrap weight is <= this is a leaf */
  int32_t bootstrap;     /* 1: each tree draws n rows with replacement; 0: each row once */
  uint64_t seed;
} aiwc_rf_params;

/* ------------------------------------------------------------------------------
 * Binning.  Turns the AIWC feature matrix (Table I metrics; the paper uses 34 of
 * them, Sec. III-B) and the device id (Table II) into uint8 codes.
 *
 * X:         n x p float32, row-major (device).
 * device_id: n int32 in [0, n_devices) (device).
 * codes:     n x (p + 1) uint8, row-major, output (device); column p = device id.
 * *binner:   NULL on entry -> thresholds are fitted on these rows and a new binner
 *            is returned in *binner; non-NULL -> its thresholds are applied.
 * Thresholds per feature column: if the column has at most max_bins distinct
 * values, every distinct value but the largest (lossless); otherwise the order
 * statistics s[floor(k n / max_bins) - 1], k = 1 .. max_bins - 1, of the sorted
 * column, repeats and values not below the column maximum dropped.  code(x) = the
 * number of thresholds strictly below x (-0.0 is treated as +0.0).
 * Errors: EINVAL for null pointers, n outside [1, AIWC_RF_MAX_ROWS], p outside
 * [1, 254], n_devices outside [1, 256], max_bins outside [2, 256], a NaN feature or
 * a device id out of range; EINVAL also if an applied binner has another p.
 * Synchronous. */
int aiwc_rf_bin(const float* X, const int32_t* device_id, int64_t n, int32_t p, int32_t n_devices,
                int32_t max_bins, aiwc_rf_binner** binner, uint8_t* codes, void* stream);

/* A binner that only carries bin counts (n_bins_host[n_cols], each in [1, 256];
 * n_cols in [1, AIWC_RF_MAX_COLS]), for fitting code matrices that were binned
 * elsewhere.  It cannot bin features. */
int aiwc_rf_binner_from_counts(const int32_t* n_bins_host, int32_t n_cols, aiwc_rf_binner** binner);

/* Copy out p, n_devices, the bin count of each of the p + 1 columns and the
 * thresholds (p x 255 float32, column j's list first, unused slots 0).  Any output
 * pointer may be NULL.  thresholds_host must be NULL for a counts-only binner. */
int aiwc_rf_binner_export_host(const aiwc_rf_binner* binner, int32_t* p_host, int32_t* n_devices_host,
                               int32_t* n_bins_host, float* thresholds_host);
/* Releases the binner.  Work enqueued on other streams that still reads its bin
 * counts must be complete (synchronize those streams first). */
void aiwc_rf_binner_free(aiwc_rf_binner* binner);

/* ------------------------------------------------------------------------------
 * Fitting (Sec. III-B, and the tuning grids of Sec. III-B/III-C).
 *
 * codes:        n x n_cols uint8 row-major (device); every code < the binner's
 *               bin count of its column.
 * y_log10:      n float64 (device): log10 execution time of each row.
 * params_host:  n_forests parameter sets.
 * n_forests==1: one forest on the rows selected below.
 * n_forests >1: a grid; forest k trains on params_host[k] and on the rows whose
 *               fold differs from heldout_fold_host[k].
 * fold_id:      n int8 (device) fold of each row, -1 = always trained on; may be
 *               NULL when no heldout_fold_host entry is >= 0.
 * heldout_fold_host: n_forests ints (host) or NULL (= all -1 = train on all rows).
 * flags:        AIWC_RF_FIT_* below.
 * *forest:      receives a new forest handle.
 * Each forest's tree t grows from the Philox streams keyed by (seed, t), so a tree
 * depends only on its training rows, its parameters and (seed, t).
 * Errors: EINVAL for bad sizes/parameters/codes, ERANGE for a response outside
 * [-64, 64] or non-finite, ENOMEM when the node pool or scratch cannot be
 * allocated.  Synchronous unless AIWC_RF_FIT_ASYNC is given. */
#define AIWC_RF_FIT_FUSED 0u /* grid: every tree of every forest in one persistent launch, captured in a hipGraph */
#define AIWC_RF_FIT_PLAIN 1u /* grid: one launch sequence per forest (same results) */
#define AIWC_RF_FIT_ASYNC 2u /* return after enqueueing; aiwc_rf_forest_wait() reports the status */
#define AIWC_RF_FIT_TUNE 4u  /* pick the workgroup shape by timing the candidates on an evenly
                                strided sample of this call's trees (up to 64 per CU): workgroup
                                size, wide limit, waves per SIMD and columns per large-node task;
                                the choice is cached per problem shape (and in the file named by
                                AIWC_RF_TUNE_CACHE, if set); results never depend on it.
                                Without it the shape follows the problem size; the environment
                                variables AIWC_RF_GROW_BLOCK (192, 256, 512 or 1024 threads),
                                AIWC_RF_HUGE_MIN (rows above which a node is searched by the
                                whole workgroup), AIWC_RF_GROW_OCC (4, 5 or 6 waves per SIMD),
                                AIWC_RF_GROW_WG_PER_CU and AIWC_RF_BIG_COLS (1 to 4 columns per
                                large-node task) override it, again without changing results;
                                AIWC_RF_WIDE_SUMS=1 makes the small-node searches always add
                                64-bit sums (otherwise only when a bootstrap weight exceeds
                                255), also without changing results */
int aiwc_rf_fit(const uint8_t* codes, int64_t n, int32_t n_cols, const aiwc_rf_binner* binner,
                const double* y_log10, const int8_t* fold_id, const aiwc_rf_params* params_host,
                const int32_t* heldout_fold_host, int32_t n_forests, uint32_t flags, aiwc_rf_forest** forest,
                void* stream);

/* A grid whose forests train on unions of row groups (Sec. III-C: Algorithm 1
 * omits one kernel per model, Algorithm 2 trains on a random subset of the
 * kernels and tests on the rest).  group_id: n int8 (device), the group (e.g.
 * the kernel) of each row in [0, 63], or -1 for rows every forest trains on.
 * train_mask_host: n_forests uint64 (host); forest k trains on the rows whose
 * group has its bit set in train_mask_host[k], and holds out the other grouped
 * rows (see aiwc_rf_heldout_error).  The other arguments, the results and the
 * errors are those of aiwc_rf_fit (EINVAL also for a group id outside [-1, 63]
 * and for a mask that selects no row). */
int aiwc_rf_fit_groups(const uint8_t* codes, int64_t n, int32_t n_cols, const aiwc_rf_binner* binner,
                       const double* y_log10, const int8_t* group_id, const uint64_t* train_mask_host,
                       const aiwc_rf_params* params_host, int32_t n_forests, uint32_t flags, aiwc_rf_forest** forest,
                       void* stream);

/* Wait for an ASYNC fit and return its status (OK, ERANGE, EINVAL). */
int aiwc_rf_forest_wait(const aiwc_rf_forest* forest);

/* Number of forests, code columns and trees of forest forest_index. */
int aiwc_rf_forest_info(const aiwc_rf_forest* forest, int32_t forest_index, int32_t* n_forests_host,
                        int32_t* n_cols_host, int32_t* num_trees_host, int64_t* total_nodes_host);

/* Work statistics of a fit, for throughput accounting.  work_host[5] receives,
 * summed over the trees of forest forest_index: the in-bag rows of every node whose
 * split was searched, the number of such nodes, the in-bag rows of every node that
 * split (rows moved to children), (max over trees) the number of levels grown, and
 * the rows added to LDS histogram bins (in-bag rows x mtry of every searched node
 * above 32 rows: one LDS atomic add each).  The counts are of the work done: in a
 * fused fit, trees that differ only in min.node.size are grown once down to the
 * level where they part (task groups, see aiwc_rf_launch_info), and the shared
 * levels count for the group's tree with the smallest min.node.size.
 * grow_ms_host receives the device time of the call's tree-growing launch(es),
 * from events recorded on the fit stream around them (for a grid: the whole call).
 * Either output may be NULL.  Waits for an ASYNC fit. */
int aiwc_rf_forest_stats(const aiwc_rf_forest* forest, int32_t forest_index, int64_t* work_host, float* grow_ms_host);

/* The launch shape a fit used (the same for every forest of a grid).  Shapes never
 * change results; this reports which one ran, for tests and profiles. */
typedef struct {
  int32_t block;          /* threads per workgroup of the grow kernel */
  int32_t waves_per_simd; /* occupancy the grow kernel was compiled for */
  int32_t wide_limit;     /* nodes with more in-bag rows are searched by the whole workgroup */
  int32_t big_cols;       /* candidate columns per large-node task */
  int32_t grid;           /* workgroups of the (largest) persistent grow launch */
  int32_t wide_phase;     /* 1 when the kernel with the workgroup-wide phase ran */
  int32_t graph;          /* 1 when the fit ran as one executable-graph launch (fused grid) */
  int32_t graph_reused;   /* 1 when that graph was built by an earlier fit of the same shape */
  int32_t tuned;          /* 1 when the shape came from the autotuner (timed now or cached) */
  int32_t task_groups;    /* work items of the grow launch(es): a fused fit grows tree t of the
                             forests that differ only in min.node.size (up to 8 of them) as one
                             group, sharing the levels above the first one holding a node that is
                             a leaf for some of them only; otherwise every tree is its own item */
} aiwc_rf_launch_info;
int aiwc_rf_forest_launch(const aiwc_rf_forest* forest, aiwc_rf_launch_info* info_host);

/* Node counts of trees [tree_begin, tree_end) of a forest (n_nodes_host[tree_end - tree_begin]). */
int aiwc_rf_forest_tree_sizes(const aiwc_rf_forest* forest, int32_t forest_index, int32_t tree_begin,
                              int32_t tree_end, int64_t* n_nodes_host);

/* Node arrays of trees [tree_begin, tree_end), concatenated in tree order, each tree
 * in breadth-first node order (root = 0; the children of a split node are left and
 * left + 1).  col: split column or AIWC_RF_LEAF; bin: rows with code <= bin go
 * left; left: child id within the tree (-1 for leaves); q: leaf value in units of
 * 2^-32 (0 for split nodes); N: bootstrap weight of the node.  Arrays hold the sum
 * of the node counts; any may be NULL. */
int aiwc_rf_forest_export_host(const aiwc_rf_forest* forest, int32_t forest_index, int32_t tree_begin,
                               int32_t tree_end, uint8_t* col_host, uint8_t* bin_host, int32_t* left_host,
                               int64_t* q_host, int32_t* N_host);
/* Releases the forest.  Waits for the fit's own stream to finish the fit; work the
 * caller enqueued on other streams that still reads the forest (predictions,
 * scoring) must be complete first.  No other stream is waited for. */
void aiwc_rf_forest_free(aiwc_rf_forest* forest);

/* ------------------------------------------------------------------------------
 * Prediction (the query of Sec. I and Sec. VI: AIWC features + device -> time).
 *
 * codes:       n x n_cols uint8 row-major (device), binned with the fit's binner.
 * y_log10_out: n float64 (device): predicted log10 execution time.
 * Asynchronous on `stream`: the output is ready when the stream reaches it.
 * Errors: EINVAL for a bad forest_index, n < 0 or null pointers. */
int aiwc_rf_predict(const aiwc_rf_forest* forest, int32_t forest_index, const uint8_t* codes, int64_t n,
                    double* y_log10_out, void* stream);

/* aiwc_rf_predict for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and results as aiwc_rf_predict; the per-row int64 sums live
 * in a fixed device array of 2^20 entries (8 MiB) that each GPU the library runs
 * on holds until the process ends, so n <= 2^20 (EINVAL above), and nothing is
 * allocated or freed.  The forest must live on the current device (EINVAL
 * otherwise).  Every call on one GPU shares that array, so calls that overlap in
 * time on one GPU (other threads, or other streams not ordered with this one)
 * race and may return wrong sums: serialise them.  The array is cleared by the
 * call's own kernels where needed. */
int aiwc_rf_predict_noalloc(const aiwc_rf_forest* forest, int32_t forest_index, const uint8_t* codes, int64_t n,
                            double* y_log10_out, void* stream);

/* Exact partial sums: sum_out[i] = sum over trees [tree_begin, tree_end) of the
 * leaf value reached by row i (int64, units 2^-32).  Sums of disjoint tree ranges
 * add up exactly, so a forest split across devices recombines bit for bit. */
int aiwc_rf_predict_sum(const aiwc_rf_forest* forest, int32_t forest_index, int32_t tree_begin,
                        int32_t tree_end, const uint8_t* codes, int64_t n, int64_t* sum_out, void* stream);

/* Out-of-bag error (Sec. III-B: the objective the parameter search minimises;
 * Sec. III-C).  For forests [forest_begin, forest_end) of a fit, every training
 * row is predicted by the trees whose bootstrap sample left it out.  Outputs, any
 * of which may be NULL: oob_sum_out / oob_count_out (device; one entry per
 * training row of each forest in turn, rows in the order of the forest's training
 * list) get the exact int64 sum of those trees' leaf values (units 2^-32) and
 * their number; mse_host / mae_host / rows_host (forest_end - forest_begin
 * entries) get the mean squared and mean absolute difference between
 * (sum * 2^-32) / count and y over the rows with count > 0, and that number of
 * rows (0 when no tree left a row out, e.g. without bootstrap).  codes and
 * y_log10 must be the arrays the forest was fitted on.  Synchronous. */
int aiwc_rf_oob_error(const aiwc_rf_forest* forest, int32_t forest_begin, int32_t forest_end, const uint8_t* codes,
                      const double* y_log10, int64_t* oob_sum_out, int32_t* oob_count_out, double* mse_host,
                      double* mae_host, int64_t* rows_host, void* stream);

/* Held-out error (Sec. III-C: the error of a model on the kernels it was not
 * trained on; with aiwc_rf_fit it is the cross-validation error of a fold).  The
 * held-out rows of a forest are, ascending: for aiwc_rf_fit, the rows of its
 * held-out fold (none for -1); for aiwc_rf_fit_groups, the grouped rows outside
 * its mask.  Every held-out row is predicted by all of the forest's trees, as by
 * aiwc_rf_predict.  Outputs, any of which may be NULL: pred_sum_out (device, one
 * int64 per held-out row of each forest in turn) gets the exact leaf-value sum
 * (units 2^-32); mse_host / mae_host / rows_host (forest_end - forest_begin
 * entries) get the mean squared and mean absolute difference between the
 * prediction and y over the held-out rows, and their number (0 when a forest
 * holds out nothing, with mse = mae = 0).  codes and y_log10 must be the arrays
 * the forest was fitted on.  Synchronous. */
int aiwc_rf_heldout_error(const aiwc_rf_forest* forest, int32_t forest_begin, int32_t forest_end,
                          const uint8_t* codes, const double* y_log10, int64_t* pred_sum_out, double* mse_host,
                          double* mae_host, int64_t* rows_host, void* stream);

/* The held-out rows of forest forest_index: *n_host receives their number and,
 * unless rows_out_host is NULL, rows_out_host (host, *n_host entries) the row
 * indices, ascending. */
int aiwc_rf_heldout_rows(const aiwc_rf_forest* forest, int32_t forest_index, int32_t* rows_out_host, int32_t* n_host);

/* ------------------------------------------------------------------------------
 * Parameter search by simulated annealing (Sec. III-B: num.trees, mtry and
 * min.node.size are chosen by an annealing search that minimises the
 * out-of-bag error, from a starting location).
 *
 * The state is the parameter triple (num.trees, mtry, min.node.size), each in
 * [lower, upper].  The objective of a triple is the out-of-bag MSE of the forest
 * grown with it on all n rows (bootstrap, seed cfg->seed), summed on the host in
 * row order from the exact out-of-bag sums and counts, so that the whole search
 * is reproducible bit for bit.  The start is evaluated first.  At level l
 * (temperature T_l = t0 * cooling^l) `proposals` triples are drawn around the
 * state the level starts from: proposal j of level l takes block (0, 2, l, j)
 * of the Philox4x64-10 stream keyed (seed, 0); word c (c = 0, 1, 2) moves
 * coordinate c by floor(word * (2h_c + 1) / 2^64) - h_c, with half-width h_c =
 * max(1, floor(step_frac * (upper_c - lower_c))), clamped to the bounds; word
 * 3 gives u = (word >> 11) * 2^-53.  All proposals of a level are fitted
 * together as one grid and scored; then, in proposal order, a proposal whose
 * objective is not above the current one's, or whose u < exp(-(f' - f) / T_l),
 * becomes the current state.  The best triple over every evaluation (the first
 * on ties) is returned.
 */
typedef struct {
  int32_t lower[3];   /* bounds of num.trees, mtry, min.node.size (inclusive) */
  int32_t upper[3];
  int32_t start[3];   /* starting location */
  int32_t levels;     /* temperature levels */
  int32_t proposals;  /* proposals per level, fitted together */
  double t0;          /* initial temperature, in units of the objective */
  double cooling;     /* T_{l+1} = cooling * T_l */
  double step_frac;   /* proposal half-width as a fraction of each range */
  uint64_t seed;      /* forest seed and annealing stream key */
} aiwc_rf_sa_config;

/* One evaluation of the search: level (-1 for the start), proposal index, the
 * triple, its objective and out-of-bag row count, whether it was accepted, and
 * the current triple after the decision. */
typedef struct {
  int32_t level;
  int32_t index;
  int32_t params[3];
  int32_t accepted;
  int32_t current[3];
  int64_t oob_rows;
  double objective;
} aiwc_rf_sa_step;

/* Run the search on n rows of codes (device, n x n_cols, the binner's codes) and
 * y_log10 (device).  best_params_host (3 ints) and best_objective_host receive
 * the best triple and its objective; trace_host (1 + levels * proposals
 * entries, or NULL) every evaluation in order.  Errors: EINVAL for bounds with
 * lower > upper, a start outside them, mtry bounds outside [1, n_cols], levels
 * or proposals < 1, non-finite or negative t0, cooling or step_frac; the errors
 * of aiwc_rf_fit.  Synchronous. */
int aiwc_rf_tune_sa(const uint8_t* codes, int64_t n, int32_t n_cols, const aiwc_rf_binner* binner,
                    const double* y_log10, const aiwc_rf_sa_config* cfg, int32_t* best_params_host,
                    double* best_objective_host, aiwc_rf_sa_step* trace_host, void* stream);

/* Device selection (Sec. VI: the model is to tell a scheduler on which device a
 * kernel runs fastest).  feature_codes holds m kernels' AIWC feature codes only,
 * m x (n_cols - 1) uint8 row-major (device); every device id 0 .. D-1 (D = the
 * bin count of the device column, the last code column) is appended to each of
 * them and predicted.  times_out (m x D float64, device, or NULL) receives the
 * predicted log10 times, best_out (m int32, device) the device with the smallest
 * prediction, the lowest id on ties.  Asynchronous on `stream`. */
int aiwc_rf_select_device(const aiwc_rf_forest* forest, int32_t forest_index, const uint8_t* feature_codes,
                          int64_t m, double* times_out, int32_t* best_out, void* stream);

/* How well predicted times rank each kernel's devices: the criterion of Sec. VI,
 * where the model is useful to a scheduler when, for any pair of devices, it
 * names the one on which the kernel runs faster.
 *
 * times, truth: m x n_devices float64 row-major (device): predicted and measured
 *   (or, for synthetic frames, noiseless) log10 times of each kernel on each
 *   device, e.g. times_out of aiwc_rf_select_device.
 * For kernel k and devices i < j the prediction chooses i when times[k,i] <=
 * times[k,j] (the lowest id on a tie, like aiwc_rf_select_device) and j
 * otherwise; the choice is right when the chosen device's truth is strictly the
 * smaller.  Pairs with equal truth have no wrong choice and are not counted.
 * Outputs (device, m int32 each, any may be NULL): correct_out (pairs chosen
 * right), counted_out (pairs counted), hit_out (1 when the predicted fastest
 * device, the smallest prediction with the lowest id on ties, has the smallest
 * truth).  Only comparisons: exact.  Asynchronous on `stream`.
 * Errors: EINVAL for m < 0, n_devices outside [1, 256] or null inputs. */
int aiwc_rf_rank_accuracy(const double* times, const double* truth, int64_t m, int32_t n_devices,
                          int32_t* correct_out, int32_t* counted_out, int32_t* hit_out, void* stream);

/* ------------------------------------------------------------------------------
 * Serving (the scheduler-facing use of Sec. VI): a resident forest answers a
 * stream of prediction requests of different sizes.  Requests are packed into
 * batches as they arrive (continuous batching) and run on several streams, so that
 * copies and kernels of different batches overlap.  Each answer equals what
 * aiwc_rf_predict returns for the same rows alone.
 *
 * Memory admission: at creation the server allocates one device arena and one
 * pinned host arena that together hold at most memory_budget_bytes, cut into row
 * slots (a row costs 2 * n_cols + 24 bytes: n_cols + 16 on the device for its
 * codes, sum and answer, n_cols + 8 pinned for its staged codes and answer).  A
 * batch takes one contiguous range of slots and returns it when it completes;
 * requests that arrive while no range is large enough wait, in arrival order,
 * until running batches free their slots.  No allocation happens per request.
 *
 * create:  forest/forest_index to serve; memory_budget_bytes (see above);
 *          max_batch_rows caps one batch; n_streams in [1, 8].  EINVAL for bad
 *          arguments or a budget below one row, ESTATE if the fit failed, ENOMEM
 *          if the arenas cannot be allocated.
 * submit:  codes_host is n x n_cols uint8, out_host receives n float64; both stay
 *          owned by the caller and must stay valid until the request completes.
 *          Never blocks; returns the request's ticket.  ENOMEM if n rows alone
 *          exceed the arenas or max_batch_rows; ESTATE once the server failed.
 * poll:    copies up to max_tickets completed tickets (completion order) and their
 *          latency in seconds (submit -> results in out_host); *n_done receives the
 *          count.  EHIP (after copying) if a batch failed on the device.
 * drain:   blocks until every submitted request has completed (EHIP on failure).
 * stats:   rows served, batches launched, peak bytes of the arena slots in use,
 *          and how many times the oldest waiting request had to wait for slots.
 * Every failure sets aiwc_rf_last_error(). */
typedef struct aiwc_rf_server aiwc_rf_server;
int aiwc_rf_server_create(const aiwc_rf_forest* forest, int32_t forest_index, int64_t memory_budget_bytes,
                          int32_t max_batch_rows, int32_t n_streams, aiwc_rf_server** server);
int aiwc_rf_server_submit(aiwc_rf_server* server, const uint8_t* codes_host, int64_t n, double* out_host,
                          int64_t* ticket_host);
int aiwc_rf_server_poll(aiwc_rf_server* server, int64_t* tickets_host, double* latency_s_host,
                        int32_t max_tickets, int32_t* n_done_host);
int aiwc_rf_server_drain(aiwc_rf_server* server);
int aiwc_rf_server_stats(const aiwc_rf_server* server, int64_t* rows_host, int64_t* batches_host,
                         int64_t* peak_bytes_host, int64_t* memory_waits_host);
void aiwc_rf_server_free(aiwc_rf_server* server);

/* Message of the last failure on this thread ("" if none). */
const char* aiwc_rf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif
