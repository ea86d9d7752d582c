/*
 * CPU oracle of the random-forest performance model: TEST INFRASTRUCTURE ONLY.
 *
 * This is the plain, slow reference that the HIP library is checked against.  It
 * shares no code, header, table or constant with the library, and only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 *
 * The model is the one of Sec. III-B: a random-forest regression (Breiman's random
 * forest as implemented by ranger, with the three parameters num.trees, mtry and
 * min.node.size) of kernel execution time on the AIWC features of Table I plus the
 * device on which the kernel ran.  The paper fixes the model family and its
 * parameters but not the arithmetic; the readings taken here (binning, fixed point,
 * RNG, split rule, tie-break, leaf rounding) are listed at each function and are
 * the same readings the library implements.
 *
 * All functions return 0 on success or a negative ORACLE_E* code.
 */
#ifndef ORACLE_RF_H
#define ORACLE_RF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORACLE_OK = 0,
  ORACLE_EINVAL = -1,
  ORACLE_ERANGE = -2,
  ORACLE_ENOMEM = -3
};

typedef struct {
  int32_t num_trees;      /* num.trees (Sec. III-B) */
  int32_t mtry;           /* mtry: candidate columns drawn per node (Sec. III-B) */
  int32_t min_node_size;  /* min.node.size: a node with weight <= this is a leaf */
  int32_t bootstrap;      /* 1: n draws with replacement per tree; 0: every row once */
  uint64_t seed;          /* Philox key word 0 */
} oracle_rf_params;

/* One Philox4x64-10 block (Salmon et al., SC'11): out = philox(ctr, key). */
void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Quantile binning of a feature matrix.  X is n x p row-major float32, dev[n] the
 * device id in [0, n_devices).  Writes thresholds[p * 255] (column j's list at
 * thresholds + 255*j, unused slots 0), n_bins[p + 1] (the device column last) and
 * codes[n * (p + 1)] row-major, column p = device id. */
int oracle_rf_bin(const float* X, const int32_t* dev, int64_t n, int32_t p, int32_t n_devices,
                  int32_t max_bins, float* thresholds, int32_t* n_bins, uint8_t* codes);

/* Apply previously fitted thresholds to new rows (prediction-time binning). */
int oracle_rf_bin_apply(const float* X, const int32_t* dev, int64_t n, int32_t p, int32_t n_devices,
                        const float* thresholds, const int32_t* n_bins, uint8_t* codes);

/* y_fp = rint(y * 2^16) for finite |y| <= 64. */
int oracle_rf_y_fixed(const double* y, int64_t n, int64_t* y_fp);

/* Grow trees [tree_begin, tree_end) of one forest.  The training set is rows
 * train_rows[0 .. n_train) of the code matrix (NULL: rows 0 .. n_train).  Tree t
 * writes its nodes in breadth-first order to slot (t - tree_begin) of the output
 * arrays, each slot holding `capacity` nodes, and its node count to n_nodes.
 * Node arrays: col (255 = leaf), bin, left child id (-1 for a leaf; right = left+1),
 * q (leaf value, mean response times 2^32, 0 for internal nodes) and N (the summed
 * bootstrap weight of the node).  n_threads <= 0 means all OpenMP threads. */
int oracle_rf_fit(const uint8_t* codes, int64_t n, int32_t n_cols, const int32_t* n_bins,
                  const double* y, const int64_t* train_rows, int64_t n_train,
                  const oracle_rf_params* prm, int32_t tree_begin, int32_t tree_end,
                  int64_t capacity, uint8_t* col, uint8_t* bin, int32_t* left, int64_t* q,
                  int32_t* N, int64_t* n_nodes, int32_t n_threads);

/* Sum of leaf values P[i] = sum over trees of q(leaf reached by row i), and the
 * prediction yhat[i] = (P[i] * 2^-32) / n_trees.  Trees are given as `n_trees`
 * slots of `capacity` nodes each (the layout oracle_rf_fit writes).  Either output
 * may be NULL. */
int oracle_rf_predict(const uint8_t* codes, int64_t m, int32_t n_cols, int32_t n_trees,
                      int64_t capacity, const uint8_t* col, const uint8_t* bin, const int32_t* left,
                      const int64_t* q, int64_t* P, double* yhat);

/* Out-of-bag error of trees 0 .. n_trees-1 of a forest (slots as oracle_rf_fit
 * writes them, grown with the same training rows and parameters).  For training
 * row i: P[i] = sum of q over the trees whose bootstrap sample did not draw it,
 * cnt[i] = their number.  Over the rows with cnt > 0, in row order: mse = mean of
 * ((P * 2^-32) / cnt - y)^2, mae = mean of the absolute difference, m = rows. */
int oracle_rf_oob(const uint8_t* codes, int32_t n_cols, const double* y, const int64_t* train_rows, int64_t n_train,
                  const oracle_rf_params* prm, int32_t n_trees, int64_t capacity, const uint8_t* col,
                  const uint8_t* bin, const int32_t* left, const int64_t* q, int64_t* P, int32_t* cnt, double* mse,
                  double* mae, int64_t* m);

#ifdef __cplusplus
}
#endif

#endif
