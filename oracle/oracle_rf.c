/*
 * CPU oracle of the random-forest performance model: TEST INFRASTRUCTURE ONLY.
 *
 * Plain C, written for a reader to check against the method by eye: no blocking,
 * no fusion, no reordering.  Build with -O2 -ffp-contract=off -fno-fast-math so
 * that every floating-point operation below is one IEEE-754 binary64 operation,
 * rounded to nearest, in the order written.
 *
 * What the paper fixes (Sec. III-B): a random-forest regression of execution time
 * on the AIWC features plus the device, with num.trees trees, mtry columns tried
 * per node and min.node.size as the minimal node size; prediction is the forest
 * mean (Breiman's random forest, reference [22]).  Everything else below is a
 * reading of a point the paper leaves open, stated where it is used:
 *
 *   R1 response: log10 seconds, carried as int64 fixed point y_fp = rint(y * 2^16);
 *   R2 features: quantile binning to at most 256 codes per column (lossless when a
 *      column has no more distinct values than bins); device id is its own column;
 *   R3 RNG: Philox4x64-10 with key (seed, 0) and counter (block, tag, node, tree);
 *   R4 bootstrap: n draws with replacement per tree; multiplicity = weight;
 *   R5 split rule: variance reduction, i.e. maximise S_L^2/N_L + S_R^2/N_R over
 *      candidate (column, bin) pairs, scanned column-ascending then bin-ascending,
 *      keeping the first strictly greater score; split only if the best score
 *      exceeds S^2/N;
 *   R6 stopping: a node is a leaf if its weight N <= min.node.size, if it is pure
 *      (N*Q == S^2), or if no candidate split exists;
 *   R7 leaf value q = round-half-away(S * 2^16 / N) in units of 2^-32; the forest
 *      prediction is (sum of q over trees) * 2^-32 / num.trees.
 */
#include "oracle_rf.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define MAX_ROWS (1 << 18) /* fixed-point budget: |S| <= 2^40, Q <= 2^62 */
#define LEAF_COL 255
/* column ids must stay below the leaf marker: at most 255 code columns (254 features + device) */
#define MAX_COLS 255

/* ---------------------------------------------------------------------------
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11).  Each round multiplies counter words 0 and 2 by the two
 * round multipliers, and the key is bumped by the two Weyl increments between
 * rounds.
 * ------------------------------------------------------------------------- */
static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ULL; /* golden ratio */
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73BULL; /* sqrt(3) - 1 */

void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; round++) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * c0;
    unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* Draw j of the stream (seed, tag, node, tree): word j mod 4 of block j / 4. */
static uint64_t philox_draw(uint64_t seed, uint64_t tag, uint64_t node, uint64_t tree, uint64_t j) {
  uint64_t ctr[4] = {j / 4, tag, node, tree};
  uint64_t key[2] = {seed, 0};
  uint64_t out[4];
  oracle_philox4x64_10(ctr, key, out);
  return out[j % 4];
}

/* Integer in [0, m): floor(r * m / 2^64). */
static uint64_t scale_draw(uint64_t r, uint64_t m) {
  return (uint64_t)(((unsigned __int128)r * m) >> 64);
}

enum { TAG_BOOTSTRAP = 0, TAG_MTRY = 1 };

/* ---------------------------------------------------------------------------
 * Binning (reading R2).
 * ------------------------------------------------------------------------- */
static int cmp_float(const void* a, const void* b) {
  float x = *(const float*)a, y = *(const float*)b;
  return (x > y) - (x < y);
}

static int check_bin_args(const float* X, const int32_t* dev, int64_t n, int32_t p, int32_t n_devices) {
  if (!X || !dev || n < 1 || n > MAX_ROWS || p < 1 || p > MAX_COLS - 1 || n_devices < 1 || n_devices > 256)
    return ORACLE_EINVAL;
  for (int64_t i = 0; i < n; i++) {
    if (dev[i] < 0 || dev[i] >= n_devices) return ORACLE_EINVAL;
    for (int32_t j = 0; j < p; j++)
      if (isnan(X[i * p + j])) return ORACLE_EINVAL;
  }
  return ORACLE_OK;
}

/* code(x) = number of thresholds strictly below x, so bin k is (t_k, t_{k+1}]. */
static uint8_t code_of(float x, const float* t, int32_t n_t) {
  int32_t c = 0;
  for (int32_t k = 0; k < n_t; k++)
    if (t[k] < x) c++;
  return (uint8_t)c;
}

int oracle_rf_bin(const float* X, const int32_t* dev, int64_t n, int32_t p, int32_t n_devices,
                  int32_t max_bins, float* thresholds, int32_t* n_bins, uint8_t* codes) {
  int rc = check_bin_args(X, dev, n, p, n_devices);
  if (rc) return rc;
  if (max_bins < 2 || max_bins > 256 || !thresholds || !n_bins || !codes) return ORACLE_EINVAL;
  float* s = (float*)malloc(sizeof(float) * (size_t)n);
  if (!s) return ORACLE_ENOMEM;
  memset(thresholds, 0, sizeof(float) * 255 * (size_t)p);
  for (int32_t j = 0; j < p; j++) {
    /* canonical -0.0 -> +0.0, then sort ascending */
    for (int64_t i = 0; i < n; i++) {
      float x = X[i * p + j];
      s[i] = (x == 0.0f) ? 0.0f : x;
    }
    qsort(s, (size_t)n, sizeof(float), cmp_float);
    int64_t m = 1; /* number of distinct values */
    for (int64_t i = 1; i < n; i++)
      if (s[i] != s[i - 1]) m++;
    float vmax = s[n - 1];
    float* t = thresholds + 255 * (size_t)j;
    int32_t n_t = 0;
    if (m <= max_bins) {
      /* lossless: thresholds are every distinct value but the largest */
      for (int64_t i = 0; i < n; i++)
        if ((i == 0 || s[i] != s[i - 1]) && s[i] != vmax) t[n_t++] = s[i];
    } else {
      /* quantiles t_k = s[floor(k n / B) - 1], k = 1..B-1, strictly increasing, below the max */
      for (int32_t k = 1; k < max_bins; k++) {
        int64_t idx = ((int64_t)k * n) / max_bins - 1;
        float v = s[idx];
        if (v < vmax && (n_t == 0 || v > t[n_t - 1])) t[n_t++] = v;
      }
    }
    n_bins[j] = n_t + 1;
  }
  n_bins[p] = n_devices;
  free(s);
  return oracle_rf_bin_apply(X, dev, n, p, n_devices, thresholds, n_bins, codes);
}

int oracle_rf_bin_apply(const float* X, const int32_t* dev, int64_t n, int32_t p, int32_t n_devices,
                        const float* thresholds, const int32_t* n_bins, uint8_t* codes) {
  int rc = check_bin_args(X, dev, n, p, n_devices);
  if (rc) return rc;
  if (!thresholds || !n_bins || !codes) return ORACLE_EINVAL;
  for (int64_t i = 0; i < n; i++) {
    for (int32_t j = 0; j < p; j++)
      codes[i * (p + 1) + j] = code_of(X[i * p + j], thresholds + 255 * (size_t)j, n_bins[j] - 1);
    codes[i * (p + 1) + p] = (uint8_t)dev[i];
  }
  return ORACLE_OK;
}

/* ---------------------------------------------------------------------------
 * Fixed point (reading R1).
 * ------------------------------------------------------------------------- */
int oracle_rf_y_fixed(const double* y, int64_t n, int64_t* y_fp) {
  for (int64_t i = 0; i < n; i++) {
    if (!isfinite(y[i]) || fabs(y[i]) > 64.0) return ORACLE_ERANGE;
    y_fp[i] = (int64_t)rint(y[i] * 65536.0);
  }
  return ORACLE_OK;
}

/* ---------------------------------------------------------------------------
 * One tree (readings R3-R7), grown in breadth-first order: node ids are handed
 * out in the order nodes split, the left child first, and nodes are visited in
 * id order.
 * ------------------------------------------------------------------------- */
typedef struct {
  int64_t* a;
  int64_t len, cap;
} vec64;

static int vec_push(vec64* v, int64_t x) {
  if (v->len == v->cap) {
    int64_t cap = v->cap ? 2 * v->cap : 1024;
    int64_t* a = (int64_t*)realloc(v->a, sizeof(int64_t) * (size_t)cap);
    if (!a) return ORACLE_ENOMEM;
    v->a = a;
    v->cap = cap;
  }
  v->a[v->len++] = x;
  return ORACLE_OK;
}

static int grow_tree(const uint8_t* codes, int32_t C, const int32_t* n_bins, const int64_t* y_fp,
                     const int64_t* train_rows, int64_t n_train, const oracle_rf_params* prm, int32_t tree,
                     int64_t capacity, uint8_t* col, uint8_t* bin, int32_t* left, int64_t* q, int32_t* N_out,
                     int64_t* n_nodes_out) {
  int rc = ORACLE_OK;
  int64_t* w = (int64_t*)calloc((size_t)n_train, sizeof(int64_t));
  int64_t* seg_start = (int64_t*)malloc(sizeof(int64_t) * (size_t)capacity);
  int64_t* seg_len = (int64_t*)malloc(sizeof(int64_t) * (size_t)capacity);
  int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)C);
  int32_t* cand = (int32_t*)malloc(sizeof(int32_t) * (size_t)C);
  int64_t* hN = (int64_t*)malloc(sizeof(int64_t) * 256);
  int64_t* hS = (int64_t*)malloc(sizeof(int64_t) * 256);
  vec64 pool = {0, 0, 0};
  if (!w || !seg_start || !seg_len || !perm || !cand || !hN || !hS) {
    rc = ORACLE_ENOMEM;
    goto done;
  }

  /* R4: bootstrap multiplicities of the n_train training rows */
  if (prm->bootstrap) {
    for (int64_t j = 0; j < n_train; j++) {
      uint64_t r = philox_draw(prm->seed, TAG_BOOTSTRAP, 0, (uint64_t)tree, (uint64_t)j);
      w[scale_draw(r, (uint64_t)n_train)] += 1;
    }
  } else {
    for (int64_t i = 0; i < n_train; i++) w[i] = 1;
  }
  /* the root holds every in-bag row, ascending; pool entries are local row indices */
  for (int64_t i = 0; i < n_train; i++)
    if (w[i] > 0 && (rc = vec_push(&pool, i))) goto done;
  seg_start[0] = 0;
  seg_len[0] = pool.len;
  int64_t n_nodes = 1;

  for (int64_t node = 0; node < n_nodes; node++) {
    const int64_t start = seg_start[node], len = seg_len[node];
    /* node statistics: N = sum w, S = sum w*y_fp, Q = sum w*y_fp^2 */
    int64_t N = 0, S = 0, Q = 0;
    for (int64_t k = 0; k < len; k++) {
      int64_t i = pool.a[start + k];
      N += w[i];
      S += w[i] * y_fp[i];
      Q += w[i] * y_fp[i] * y_fp[i];
    }
    N_out[node] = (int32_t)N;

    int split = 0;
    int32_t best_c = -1, best_b = -1;
    if (N > prm->min_node_size && (__int128)N * Q != (__int128)S * S) {
      /* R3: mtry distinct columns by a partial Fisher-Yates shuffle, then ascending */
      for (int32_t c = 0; c < C; c++) perm[c] = c;
      for (int32_t k = 0; k < prm->mtry; k++) {
        uint64_t r = philox_draw(prm->seed, TAG_MTRY, (uint64_t)node, (uint64_t)tree, (uint64_t)k);
        int32_t j = k + (int32_t)scale_draw(r, (uint64_t)(C - k));
        int32_t tmp = perm[k];
        perm[k] = perm[j];
        perm[j] = tmp;
      }
      for (int32_t k = 0; k < prm->mtry; k++) {
        int32_t x = perm[k], m = k;
        while (m > 0 && cand[m - 1] > x) {
          cand[m] = cand[m - 1];
          m--;
        }
        cand[m] = x;
      }

      /* R5: dense scan of every (column, bin), first strictly greater score wins */
      double best = 0.0;
      int found = 0;
      for (int32_t k = 0; k < prm->mtry; k++) {
        const int32_t c = cand[k], B = n_bins[c];
        for (int32_t b = 0; b < B; b++) hN[b] = hS[b] = 0;
        for (int64_t e = 0; e < len; e++) {
          int64_t i = pool.a[start + e];
          int64_t row = train_rows ? train_rows[i] : i;
          uint8_t code = codes[row * C + c];
          hN[code] += w[i];
          hS[code] += w[i] * y_fp[i];
        }
        int64_t NL = 0, SL = 0;
        for (int32_t b = 0; b + 1 < B; b++) {
          NL += hN[b];
          SL += hS[b];
          int64_t NR = N - NL, SR = S - SL;
          if (NL == 0 || NR == 0) continue;
          double dSL = (double)SL, dSR = (double)SR;
          double score = dSL * dSL / (double)NL + dSR * dSR / (double)NR;
          if (!found || score > best) {
            best = score;
            best_c = c;
            best_b = b;
            found = 1;
          }
        }
      }
      double dS = (double)S;
      double parent = dS * dS / (double)N;
      split = found && (best - parent > 0.0);
    }

    if (split) {
      if (n_nodes + 2 > capacity) {
        rc = ORACLE_ERANGE;
        goto done;
      }
      const int64_t l = n_nodes, r = n_nodes + 1;
      col[node] = (uint8_t)best_c;
      bin[node] = (uint8_t)best_b;
      left[node] = (int32_t)l;
      q[node] = 0;
      /* rows with code <= bin go left, order preserved */
      seg_start[l] = pool.len;
      for (int64_t e = 0; e < len; e++) {
        int64_t i = pool.a[start + e];
        int64_t row = train_rows ? train_rows[i] : i;
        if (codes[row * C + best_c] <= best_b && (rc = vec_push(&pool, i))) goto done;
      }
      seg_len[l] = pool.len - seg_start[l];
      seg_start[r] = pool.len;
      for (int64_t e = 0; e < len; e++) {
        int64_t i = pool.a[start + e];
        int64_t row = train_rows ? train_rows[i] : i;
        if (codes[row * C + best_c] > best_b && (rc = vec_push(&pool, i))) goto done;
      }
      seg_len[r] = pool.len - seg_start[r];
      n_nodes += 2;
    } else {
      /* R7: q = sign(S) * floor((|S| * 2^17 + N) / (2 N)) = S * 2^16 / N rounded half away */
      int64_t a = S < 0 ? -S : S;
      int64_t mag = (a * 131072 + N) / (2 * N);
      col[node] = LEAF_COL;
      bin[node] = 0;
      left[node] = -1;
      q[node] = S < 0 ? -mag : mag;
    }
  }
  *n_nodes_out = n_nodes;

done:
  free(w);
  free(seg_start);
  free(seg_len);
  free(perm);
  free(cand);
  free(hN);
  free(hS);
  free(pool.a);
  return rc;
}

int oracle_rf_fit(const uint8_t* codes, int64_t n, int32_t n_cols, const int32_t* n_bins,
                  const double* y, const int64_t* train_rows, int64_t n_train,
                  const oracle_rf_params* prm, int32_t tree_begin, int32_t tree_end,
                  int64_t capacity, uint8_t* col, uint8_t* bin, int32_t* left, int64_t* q,
                  int32_t* N, int64_t* n_nodes, int32_t n_threads) {
  if (!codes || !n_bins || !y || !prm || !col || !bin || !left || !q || !N || !n_nodes) return ORACLE_EINVAL;
  if (n < 1 || n > MAX_ROWS || n_cols < 1 || n_cols > MAX_COLS || n_train < 1 || n_train > n) return ORACLE_EINVAL;
  if (prm->num_trees < 1 || prm->num_trees > (1 << 14) || prm->mtry < 1 || prm->mtry > n_cols ||
      prm->min_node_size < 1 || tree_begin < 0 || tree_end > prm->num_trees || tree_begin >= tree_end)
    return ORACLE_EINVAL;
  for (int32_t c = 0; c < n_cols; c++)
    if (n_bins[c] < 1 || n_bins[c] > 256) return ORACLE_EINVAL;
  if (capacity < 2 * n_train - 1) return ORACLE_EINVAL;
  for (int64_t i = 0; i < n * n_cols; i++)
    if (codes[i] >= n_bins[i % n_cols]) return ORACLE_EINVAL;
  if (train_rows)
    for (int64_t i = 0; i < n_train; i++)
      if (train_rows[i] < 0 || train_rows[i] >= n) return ORACLE_EINVAL;

  /* the responses of the training rows, in fixed point */
  int64_t* y_fp = (int64_t*)malloc(sizeof(int64_t) * (size_t)n_train);
  if (!y_fp) return ORACLE_ENOMEM;
  for (int64_t i = 0; i < n_train; i++) {
    double v = y[train_rows ? train_rows[i] : i];
    int rc = oracle_rf_y_fixed(&v, 1, &y_fp[i]);
    if (rc) {
      free(y_fp);
      return rc;
    }
  }

  int status = ORACLE_OK;
#ifdef _OPENMP
  int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
  for (int32_t t = tree_begin; t < tree_end; t++) {
    int64_t slot = (int64_t)(t - tree_begin) * capacity;
    int rc = grow_tree(codes, n_cols, n_bins, y_fp, train_rows, n_train, prm, t, capacity, col + slot,
                       bin + slot, left + slot, q + slot, N + slot, &n_nodes[t - tree_begin]);
    if (rc) {
#ifdef _OPENMP
#pragma omp critical
#endif
      status = rc;
    }
  }
  (void)n_threads;
  free(y_fp);
  return status;
}

int oracle_rf_predict(const uint8_t* codes, int64_t m, int32_t n_cols, int32_t n_trees,
                      int64_t capacity, const uint8_t* col, const uint8_t* bin, const int32_t* left,
                      const int64_t* q, int64_t* P, double* yhat) {
  if (!codes || m < 0 || n_cols < 1 || n_trees < 1 || n_trees > (1 << 14) || !col || !bin || !left || !q)
    return ORACLE_EINVAL;
  for (int64_t i = 0; i < m; i++) {
    int64_t sum = 0;
    for (int32_t t = 0; t < n_trees; t++) {
      const int64_t base = (int64_t)t * capacity;
      int64_t node = 0;
      while (col[base + node] != LEAF_COL) {
        uint8_t c = col[base + node];
        if (c >= n_cols) return ORACLE_EINVAL;
        node = codes[i * n_cols + c] <= bin[base + node] ? left[base + node] : left[base + node] + 1;
      }
      sum += q[base + node];
    }
    if (P) P[i] = sum;
    if (yhat) yhat[i] = ((double)sum * 0x1p-32) / (double)n_trees;
  }
  return ORACLE_OK;
}

/* ---------------------------------------------------------------------------
 * Out-of-bag error (the tuning objective of Sec. III-B): each training row is
 * predicted only by the trees whose bootstrap sample (reading R4) left it out.
 * ------------------------------------------------------------------------- */
int oracle_rf_oob(const uint8_t* codes, int32_t n_cols, const double* y, const int64_t* train_rows, int64_t n_train,
                  const oracle_rf_params* prm, int32_t n_trees, int64_t capacity, const uint8_t* col,
                  const uint8_t* bin, const int32_t* left, const int64_t* q, int64_t* P, int32_t* cnt, double* mse,
                  double* mae, int64_t* m) {
  if (!codes || !y || !prm || !col || !bin || !left || !q || !P || !cnt || n_train < 1 || n_trees < 1)
    return ORACLE_EINVAL;
  int64_t* w = (int64_t*)malloc(sizeof(int64_t) * (size_t)n_train);
  if (!w) return ORACLE_ENOMEM;
  for (int64_t i = 0; i < n_train; i++) {
    P[i] = 0;
    cnt[i] = 0;
  }
  for (int32_t t = 0; t < n_trees; t++) {
    for (int64_t i = 0; i < n_train; i++) w[i] = prm->bootstrap ? 0 : 1;
    if (prm->bootstrap)
      for (int64_t j = 0; j < n_train; j++)
        w[scale_draw(philox_draw(prm->seed, TAG_BOOTSTRAP, 0, (uint64_t)t, (uint64_t)j), (uint64_t)n_train)] += 1;
    const int64_t base = (int64_t)t * capacity;
    for (int64_t i = 0; i < n_train; i++) {
      if (w[i] != 0) continue;
      const int64_t row = train_rows ? train_rows[i] : i;
      int64_t node = 0;
      while (col[base + node] != LEAF_COL)
        node = codes[row * n_cols + col[base + node]] <= bin[base + node] ? left[base + node]
                                                                          : left[base + node] + 1;
      P[i] += q[base + node];
      cnt[i] += 1;
    }
  }
  double sq = 0.0, ab = 0.0;
  int64_t rows = 0;
  for (int64_t i = 0; i < n_train; i++) {
    if (cnt[i] == 0) continue;
    const int64_t row = train_rows ? train_rows[i] : i;
    double e = ((double)P[i] * 0x1p-32) / (double)cnt[i] - y[row];
    sq += e * e;
    ab += fabs(e);
    rows++;
  }
  *mse = rows ? sq / (double)rows : 0.0;
  *mae = rows ? ab / (double)rows : 0.0;
  *m = rows;
  free(w);
  return ORACLE_OK;
}
