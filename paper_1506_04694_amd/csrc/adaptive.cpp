// Choosing the number of levels and samples of the MLMC estimator (host side).
//
// Section 3.2: the mean square error eq. (3.7) is split evenly between the
// variance sum_l V_l / N_l and the squared bias; the N_l minimise the cost
// sum_l N_l C_l for the variance part eps^2 / 2, which by a Lagrange multiplier
// gives N_l proportional to sqrt(V_l / C_l).  The complexity theorem's rates
// (M1)-(M3) are fitted as log2 slopes over the levels l >= 1, and the bias of
// the finest level is the geometric tail |E[Y_L]| / (2^alpha - 1) of the
// differences beyond it (h halves from level to level).
//
// The driver only calls the public entry points (level runs on the device),
// so a level's samples and results are exactly those of mlmc_level_run.
#include <chrono>
#include <cmath>
#include <vector>

#include "../../include/mlmc_darcy.h"

namespace mlmc {
mlmc_status set_error(mlmc_ctx* ctx, mlmc_status code, const char* msg);
}

namespace {

double mean_of(const mlmc_level_sums& s) { return s.sum_y / (double)s.n; }

double var_of(const mlmc_level_sums& s) {
  const double n = (double)s.n, mean = s.sum_y / n;
  return (s.sum_y2 - n * mean * mean) / (n - 1.0);
}

// Least squares slope of y against x.
double slope(const std::vector<double>& x, const std::vector<double>& y) {
  const size_t n = x.size();
  double sx = 0, sy = 0;
  for (size_t q = 0; q < n; ++q) {
    sx += x[q];
    sy += y[q];
  }
  const double mx = sx / n, my = sy / n;
  double sxy = 0, sxx = 0;
  for (size_t q = 0; q < n; ++q) {
    sxy += (x[q] - mx) * (y[q] - my);
    sxx += (x[q] - mx) * (x[q] - mx);
  }
  return sxy / sxx;
}

}  // namespace

extern "C" {

mlmc_status mlmc_optimal_samples(const double* var, const double* cost, int n_levels, double eps,
                                 int64_t* n_out) {
  if (!var || !cost || !n_out || n_levels < 1 || !(eps > 0.0)) return MLMC_EINVAL;
  double total = 0.0;
  for (int l = 0; l < n_levels; ++l) {
    if (!(var[l] >= 0.0) || !(cost[l] > 0.0) || !std::isfinite(var[l]) || !std::isfinite(cost[l]))
      return MLMC_EINVAL;
    total += std::sqrt(var[l] * cost[l]);
  }
  for (int l = 0; l < n_levels; ++l) {
    const double n = std::ceil(2.0 / (eps * eps) * std::sqrt(var[l] / cost[l]) * total);
    n_out[l] = n > 9.0e18 ? (int64_t)9e18 : (int64_t)n;
  }
  return MLMC_OK;
}

mlmc_status mlmc_rates(const mlmc_level_sums* sums, const double* cost, const int* m,
                       int n_levels, double* alpha, double* beta, double* gamma) {
  if (!sums || !cost || !m || !alpha || !beta || !gamma || n_levels < 3) return MLMC_EINVAL;
  std::vector<double> lh, la, lb, lc;
  for (int l = 1; l < n_levels; ++l) {
    if (sums[l].n < 2 || m[l] < 1 || !(cost[l] > 0.0)) return MLMC_EINVAL;
    lh.push_back(std::log2(1.0 / (double)m[l]));
    la.push_back(std::log2(std::fabs(mean_of(sums[l]))));
    lb.push_back(std::log2(var_of(sums[l])));
    lc.push_back(std::log2(cost[l]));
  }
  *alpha = slope(lh, la);
  *beta = slope(lh, lb);
  *gamma = -slope(lh, lc);
  return MLMC_OK;
}

mlmc_status mlmc_adaptive_opts_default(mlmc_adaptive_opts* o) {
  if (!o) return MLMC_EINVAL;
  o->eps = 1e-2;
  o->alpha = 0.0;
  o->n_initial = 64;
  o->min_levels = 3;
  o->cgv = 0;
  o->reserved = 0;
  o->max_samples = (int64_t)1 << 24;
  return MLMC_OK;
}

mlmc_status mlmc_adaptive(mlmc_ctx* ctx, const mlmc_model* model, int max_levels,
                          const int* m_levels, const int* n_ce, const mlmc_adaptive_opts* opts,
                          const mlmc_solver_opts* solver, mlmc_adaptive_result* out) {
  using mlmc::set_error;
  if (!ctx) return MLMC_EINVAL;
  if (!model || !m_levels || !opts || !solver || !out)
    return set_error(ctx, MLMC_EINVAL, "NULL argument to mlmc_adaptive");
  if (max_levels < 2 || max_levels > MLMC_MAX_LEVELS)
    return set_error(ctx, MLMC_EINVAL, "max_levels must be in [2, MLMC_MAX_LEVELS]");
  if (!(opts->eps > 0.0) || opts->n_initial < 2 || opts->min_levels < 2 ||
      opts->min_levels > max_levels || opts->max_samples < opts->n_initial || opts->alpha < 0.0)
    return set_error(ctx, MLMC_EINVAL, "bad mlmc_adaptive_opts");
  for (int l = 1; l < max_levels; ++l)
    if (m_levels[l] != 2 * m_levels[l - 1])
      return set_error(ctx, MLMC_EINVAL, "m_levels must double from level to level");

  *out = mlmc_adaptive_result{};
  const double eps = opts->eps;
  int L = opts->min_levels - 1;
  std::vector<int64_t> dn(max_levels, 0), big_n(max_levels, 0);
  std::vector<double> seconds(max_levels, 0.0), var(max_levels, 0.0), cost(max_levels, 0.0);
  std::vector<double> big_t(max_levels, 0.0);
  for (int l = 0; l <= L; ++l) dn[l] = opts->n_initial;
  double alpha = opts->alpha;
  for (int round = 0; round < 1000; ++round) {
    // the missing samples of every level, each call a block of new sample numbers
    for (int l = 0; l <= L; ++l) {
      int64_t todo = dn[l];
      // at most 2^26 fine cells per call (about 0.5 GB per FP64 field)
      const double cells = std::pow((double)m_levels[l], (double)model->dim);
      const int64_t cap = std::max<int64_t>(1, (int64_t)((double)(1 << 26) / cells));
      while (todo > 0) {
        const int chunk = (int)std::min<int64_t>(todo, std::min<int64_t>(cap, (int64_t)1 << 20));
        mlmc_model mdl = *model;
        if (n_ce) mdl.n_ce = n_ce[l];
        const auto t0 = std::chrono::steady_clock::now();
        const mlmc_status st =
            mlmc_level_run(ctx, &mdl, l, m_levels[l], (uint64_t)out->n[l], chunk, opts->cgv,
                           solver, &out->sums[l], nullptr, nullptr, nullptr);
        const double t =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        seconds[l] += t;
        if (st != MLMC_OK) return st;
        if (chunk >= big_n[l]) {
          big_n[l] = chunk;
          big_t[l] = t;
        }
        out->n[l] += chunk;
        todo -= chunk;
      }
      dn[l] = 0;
    }
    // a level run has a fixed per-call part (launches, synchronisation), so the
    // cost of one more sample is taken from the largest call of the level
    for (int l = 0; l <= L; ++l) {
      var[l] = var_of(out->sums[l]);
      cost[l] = big_t[l] / (double)big_n[l];
    }
    std::vector<int64_t> nopt(L + 1);
    const mlmc_status st = mlmc_optimal_samples(var.data(), cost.data(), L + 1, eps, nopt.data());
    if (st != MLMC_OK) return set_error(ctx, st, "non-finite level variance or cost");
    // at most 4x the samples per round: variance and cost are measured again at
    // the larger size before more samples are committed
    bool more = false;
    for (int l = 0; l <= L; ++l) {
      const int64_t want = std::min(std::min(nopt[l], opts->max_samples), 4 * out->n[l]);
      dn[l] = want > out->n[l] ? want - out->n[l] : 0;
      more = more || dn[l] > 0;
    }
    if (more) continue;
    // the variance part is met: bias of the finest level
    if (opts->alpha <= 0.0) {
      alpha = 0.5;
      if (L >= 2) {
        double a = 0, b = 0, g = 0;
        std::vector<int> mm(m_levels, m_levels + L + 1);
        if (mlmc_rates(out->sums, cost.data(), mm.data(), L + 1, &a, &b, &g) == MLMC_OK &&
            std::isfinite(a))
          alpha = std::max(0.5, a);
      }
    }
    const double bias = std::fabs(mean_of(out->sums[L])) / (std::pow(2.0, alpha) - 1.0);
    out->bias = bias;
    if (bias <= eps / std::sqrt(2.0)) {
      out->converged = 1;
      break;
    }
    if (L + 1 >= max_levels) break;
    ++L;
    dn[L] = opts->n_initial;
  }
  out->n_levels = L + 1;
  out->alpha = alpha;
  out->beta = out->gamma = std::nan("");
  if (L >= 2) {
    double a = 0, b = 0, g = 0;
    std::vector<int> mm(m_levels, m_levels + L + 1);
    if (mlmc_rates(out->sums, cost.data(), mm.data(), L + 1, &a, &b, &g) == MLMC_OK) {
      out->beta = b;
      out->gamma = g;
    }
  }
  double est = 0.0, v = 0.0, secs = 0.0;
  for (int l = 0; l <= L; ++l) {
    out->mean_y[l] = mean_of(out->sums[l]);
    out->var_y[l] = var_of(out->sums[l]);
    out->cost[l] = cost[l];
    est += out->mean_y[l];
    v += out->var_y[l] / (double)out->n[l];
    secs += seconds[l];
  }
  out->estimate = est;
  out->variance = v;
  out->seconds = secs;
  return MLMC_OK;
}

}  // extern "C"
