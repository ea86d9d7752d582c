// Parameter search by simulated annealing over batched fits (Sec. III-B: the
// paper tunes num.trees, mtry and min.node.size by annealing on the out-of-bag
// error).  Every temperature level fits its proposals as one fused grid and
// scores them with the device's out-of-bag sums; the objective of each forest
// is then summed on the host in row order from those exact integers, so the
// search path does not depend on any reduction order.
#include <algorithm>
#include <array>
#include <cmath>
#include <memory>
#include <vector>

#include "internal.h"

namespace aiwc {
namespace {

// One Philox4x64-10 block (Salmon et al., SC'11) on the host: the generator of
// the device streams, here for the annealing stream (tag 2).
void philox_block(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1, uint64_t out[4]) {
  const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
  const uint64_t w0 = 0x9E3779B97F4A7C15ull, w1 = 0xBB67AE8584CAA73Bull;
  for (int r = 0; r < 10; ++r) {
    const unsigned __int128 p0 = (unsigned __int128)m0 * c0;
    const unsigned __int128 p1 = (unsigned __int128)m1 * c2;
    const uint64_t n0 = (uint64_t)(p1 >> 64) ^ c1 ^ k0;
    const uint64_t n2 = (uint64_t)(p0 >> 64) ^ c3 ^ k1;
    c1 = (uint64_t)p1;
    c3 = (uint64_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += w0;
    k1 += w1;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

constexpr uint64_t kTagAnneal = 2;

void check_rc(int rc) {
  if (rc != AIWC_RF_OK) fail(rc, aiwc_rf_last_error());
}

struct Eval {
  double f;
  int64_t rows;
};

// Out-of-bag MSE of the forests grown with each triple, on all rows.
std::vector<Eval> evaluate(const uint8_t* codes, int64_t n, int32_t n_cols, const aiwc_rf_binner* binner,
                           const double* y_dev, const std::vector<double>& y_host,
                           const std::vector<std::array<int32_t, 3>>& triples, uint64_t seed, hipStream_t s) {
  const int32_t K = (int32_t)triples.size();
  std::vector<aiwc_rf_params> prm((size_t)K);
  for (int32_t k = 0; k < K; ++k) prm[k] = aiwc_rf_params{triples[k][0], triples[k][1], triples[k][2], 1, seed};
  aiwc_rf_forest* raw = nullptr;
  check_rc(aiwc_rf_fit(codes, n, n_cols, binner, y_dev, nullptr, prm.data(), nullptr, K, AIWC_RF_FIT_TUNE, &raw, s));
  std::unique_ptr<aiwc_rf_forest, void (*)(aiwc_rf_forest*)> forest(raw, aiwc_rf_forest_free);
  DevBuf<int64_t> sums((size_t)K * n, s);
  DevBuf<int32_t> counts((size_t)K * n, s);
  check_rc(aiwc_rf_oob_error(forest.get(), 0, K, codes, y_dev, sums.p, counts.p, nullptr, nullptr, nullptr, s));
  std::vector<int64_t> P((size_t)K * n);
  std::vector<int32_t> C((size_t)K * n);
  AIWC_HIP(hipMemcpyAsync(P.data(), sums.p, sizeof(int64_t) * P.size(), hipMemcpyDeviceToHost, s));
  AIWC_HIP(hipMemcpyAsync(C.data(), counts.p, sizeof(int32_t) * C.size(), hipMemcpyDeviceToHost, s));
  AIWC_HIP(hipStreamSynchronize(s));
  std::vector<Eval> out((size_t)K);
  for (int32_t k = 0; k < K; ++k) {
    double sq = 0.0;
    int64_t rows = 0;
    for (int64_t i = 0; i < n; ++i) {
      const int32_t c = C[(size_t)k * n + i];
      if (c == 0) continue;
      const double e = ((double)P[(size_t)k * n + i] * 0x1p-32) / (double)c - y_host[i];
      sq += e * e;
      ++rows;
    }
    out[k] = Eval{rows ? sq / (double)rows : 0.0, rows};
  }
  return out;
}

}  // namespace

void anneal(const uint8_t* codes, int64_t n, int32_t n_cols, const aiwc_rf_binner* binner, const double* y_dev,
            const aiwc_rf_sa_config& cfg, int32_t* best_params, double* best_objective, aiwc_rf_sa_step* trace,
            hipStream_t s) {
  for (int c = 0; c < 3; ++c) {
    if (cfg.lower[c] > cfg.upper[c] || cfg.start[c] < cfg.lower[c] || cfg.start[c] > cfg.upper[c])
      fail(AIWC_RF_EINVAL, "annealing bounds must satisfy lower <= start <= upper");
  }
  if (cfg.lower[0] < 1 || cfg.upper[0] > AIWC_RF_MAX_TREES) fail(AIWC_RF_EINVAL, "num.trees bounds out of range");
  if (cfg.lower[1] < 1 || cfg.upper[1] > n_cols) fail(AIWC_RF_EINVAL, "mtry bounds must lie in [1, n_cols]");
  if (cfg.lower[2] < 1) fail(AIWC_RF_EINVAL, "min.node.size bounds must be >= 1");
  if (cfg.levels < 1 || cfg.proposals < 1) fail(AIWC_RF_EINVAL, "levels and proposals must be >= 1");
  if (!std::isfinite(cfg.t0) || cfg.t0 < 0.0 || !std::isfinite(cfg.cooling) || cfg.cooling < 0.0 ||
      !std::isfinite(cfg.step_frac) || cfg.step_frac < 0.0)
    fail(AIWC_RF_EINVAL, "t0, cooling and step_frac must be finite and >= 0");
  std::vector<double> y_host((size_t)n);
  AIWC_HIP(hipMemcpyAsync(y_host.data(), y_dev, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  AIWC_HIP(hipStreamSynchronize(s));

  int32_t half[3];
  for (int c = 0; c < 3; ++c)
    half[c] = std::max<int32_t>(1, (int32_t)std::floor(cfg.step_frac * (double)(cfg.upper[c] - cfg.lower[c])));

  std::array<int32_t, 3> cur{cfg.start[0], cfg.start[1], cfg.start[2]};
  const Eval e0 = evaluate(codes, n, n_cols, binner, y_dev, y_host, {cur}, cfg.seed, s)[0];
  double f_cur = e0.f;
  std::array<int32_t, 3> best = cur;
  double f_best = f_cur;
  int64_t t = 0;
  auto record = [&](int32_t level, int32_t index, const std::array<int32_t, 3>& p, const Eval& e, bool acc) {
    if (!trace) return;
    aiwc_rf_sa_step& st = trace[t];
    st.level = level;
    st.index = index;
    for (int c = 0; c < 3; ++c) {
      st.params[c] = p[c];
      st.current[c] = cur[c];
    }
    st.accepted = acc ? 1 : 0;
    st.oob_rows = e.rows;
    st.objective = e.f;
  };
  record(-1, 0, cur, e0, true);
  ++t;
  double T = cfg.t0;
  for (int32_t l = 0; l < cfg.levels; ++l) {
    const std::array<int32_t, 3> base = cur;
    std::vector<std::array<int32_t, 3>> props((size_t)cfg.proposals);
    std::vector<double> u((size_t)cfg.proposals);
    for (int32_t j = 0; j < cfg.proposals; ++j) {
      uint64_t w[4];
      philox_block(0, kTagAnneal, (uint64_t)l, (uint64_t)j, cfg.seed, 0, w);
      for (int c = 0; c < 3; ++c) {
        const uint64_t width = 2 * (uint64_t)half[c] + 1;
        const int64_t step = (int64_t)(uint64_t)(((unsigned __int128)w[c] * width) >> 64) - half[c];
        props[j][c] = (int32_t)std::min<int64_t>(cfg.upper[c], std::max<int64_t>(cfg.lower[c], base[c] + step));
      }
      u[j] = (double)(w[3] >> 11) * 0x1p-53;
    }
    const std::vector<Eval> ev = evaluate(codes, n, n_cols, binner, y_dev, y_host, props, cfg.seed, s);
    for (int32_t j = 0; j < cfg.proposals; ++j) {
      const double d = ev[j].f - f_cur;
      const bool acc = d <= 0.0 || u[j] < std::exp(-d / T);
      if (acc) {
        cur = props[j];
        f_cur = ev[j].f;
      }
      if (ev[j].f < f_best) {
        f_best = ev[j].f;
        best = props[j];
      }
      record(l, j, props[j], ev[j], acc);
      ++t;
    }
    T *= cfg.cooling;
  }
  for (int c = 0; c < 3; ++c) best_params[c] = best[c];
  *best_objective = f_best;
}

}  // namespace aiwc
