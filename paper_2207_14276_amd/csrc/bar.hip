// Bennett acceptance ratio (BAR) free-energy estimate between two states,
// with optional reweighting of the samples to a target potential: host code
// only (section "Accelerating Hybrid Simulations: an Alternative Reweighting
// Strategy" and the supplementary section on reweighted BAR: snapshots of a
// cheap reference ensemble U are re-evaluated with the network's energies,
// energy only, and reweighted to the hybrid potential U').
//
// Reduced units throughout (energies times beta).  State 0 samples carry
// u_i = beta (U_1 - U_0); state 1 samples carry v_j = beta (U_0 - U_1); with
// log weights lw (reweighting from the sampled to the target ensemble:
// lw = -beta (U'_s - U_s) of the sample's state s), averages are the weighted
// means <g>' = sum w g / sum w.  For any constant c the identity
//   Z_1 / Z_0 = e^{-c} <f(u - c)>'_0 / <f(v + c)>'_1,   f(x) = 1 / (1 + e^x),
// holds (Bennett's weight function 1 / (e^{-beta U_0} + e^{-beta (U_1 - C)})),
// so delta = beta (F_1 - F_0) = c - ln(<f(u - c)>'_0 / <f(v + c)>'_1).  The
// variance-minimizing c is delta + ln(n_1 / n_0) (effective sample sizes
// (sum w)^2 / sum w^2 when weighted), i.e. the root of
//   h(c) = ln <f(u - c)>'_0 - ln <f(v + c)>'_1 - ln(n_1 / n_0),
// which increases monotonically in c; it is bracketed and bisected in
// float64 with log-sum-exp sums.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/nnp.h"
#include "internal.h"

namespace nnp {
namespace {

// log f(x) = -log(1 + e^x), stable for large |x|
double log_fermi(double x) { return -(std::max(x, 0.0) + std::log1p(std::exp(-std::fabs(x)))); }

double logsumexp(const std::vector<double> &a) {
  double m = -INFINITY;
  for (double v : a) m = std::max(m, v);
  if (!std::isfinite(m)) return m;
  double s = 0.0;
  for (double v : a) s += std::exp(v - m);
  return m + std::log(s);
}

struct Side {
  const double *x;   // u (state 0) or v (state 1)
  const double *lw;  // log weights or null
  int64_t n;
  double sign;       // -1 for state 0 (f(u - c)), +1 for state 1 (f(v + c))
  double log_wsum;   // log sum w
  double n_eff;      // (sum w)^2 / sum w^2
};

// ln <f(x + sign c)>'
double log_mean_f(const Side &s, double c) {
  std::vector<double> t((size_t)s.n);
  for (int64_t k = 0; k < s.n; ++k) t[(size_t)k] = (s.lw ? s.lw[k] : 0.0) + log_fermi(s.x[k] + s.sign * c);
  return logsumexp(t) - s.log_wsum;
}

// <f^2>' / <f>'^2 - 1 at c, for the asymptotic variance
double rel_var_f(const Side &s, double c) {
  std::vector<double> t1((size_t)s.n), t2((size_t)s.n);
  for (int64_t k = 0; k < s.n; ++k) {
    const double lw = s.lw ? s.lw[k] : 0.0, lf = log_fermi(s.x[k] + s.sign * c);
    t1[(size_t)k] = lw + lf;
    t2[(size_t)k] = lw + 2.0 * lf;
  }
  const double l1 = logsumexp(t1) - s.log_wsum, l2 = logsumexp(t2) - s.log_wsum;
  return std::exp(l2 - 2.0 * l1) - 1.0;
}

void init_side(Side &s) {
  std::vector<double> lw((size_t)s.n), lw2((size_t)s.n);
  for (int64_t k = 0; k < s.n; ++k) {
    lw[(size_t)k] = s.lw ? s.lw[k] : 0.0;
    lw2[(size_t)k] = 2.0 * lw[(size_t)k];
  }
  s.log_wsum = logsumexp(lw);
  s.n_eff = std::exp(2.0 * s.log_wsum - logsumexp(lw2));
}

}  // namespace
}  // namespace nnp

using namespace nnp;

extern "C" int nnp_bar(int64_t n0, const double *u, const double *lw0, int64_t n1, const double *v,
                       const double *lw1, double *delta, double *sigma) {
  if (n0 < 1 || n1 < 1) return fail(NNP_EINVAL, "BAR needs at least one sample of each state");
  if (!u || !v || !delta) return fail(NNP_EINVAL, "null BAR input or output");
  for (int64_t k = 0; k < n0; ++k)
    if (!std::isfinite(u[k]) || (lw0 && !std::isfinite(lw0[k])))
      return fail(NNP_EINVAL, "BAR: non-finite value in state 0 samples");
  for (int64_t k = 0; k < n1; ++k)
    if (!std::isfinite(v[k]) || (lw1 && !std::isfinite(lw1[k])))
      return fail(NNP_EINVAL, "BAR: non-finite value in state 1 samples");
  Side s0{u, lw0, n0, -1.0, 0.0, 0.0}, s1{v, lw1, n1, +1.0, 0.0, 0.0};
  init_side(s0);
  init_side(s1);
  const double M = std::log(s1.n_eff / s0.n_eff);
  auto h = [&](double c) { return log_mean_f(s0, c) - log_mean_f(s1, c) - M; };
  // bracket the root around the mean of the two one-sided exponential
  // averages' midpoint, doubling the step until h changes sign
  double lo = 0.0;
  {
    double mu = 0.0, mv = 0.0;
    for (int64_t k = 0; k < n0; ++k) mu += u[k];
    for (int64_t k = 0; k < n1; ++k) mv += v[k];
    lo = 0.5 * (mu / (double)n0 - mv / (double)n1);
  }
  double hi = lo, step = 1.0;
  double hlo = h(lo), hhi = hlo;
  if (hlo == 0.0) hi = lo;
  else if (hlo < 0.0) {
    while (hhi < 0.0) {
      hi = lo + step;
      hhi = h(hi);
      if (hhi < 0.0) { lo = hi; hlo = hhi; }
      step *= 2.0;
      if (step > 1e12) return fail(NNP_EINVAL, "BAR: no overlap between the two states' samples");
    }
  } else {
    hi = lo;
    hhi = hlo;
    while (hlo > 0.0) {
      lo = hi - step;
      hlo = h(lo);
      if (hlo > 0.0) { hi = lo; hhi = hlo; }
      step *= 2.0;
      if (step > 1e12) return fail(NNP_EINVAL, "BAR: no overlap between the two states' samples");
    }
  }
  for (int it = 0; it < 200 && hi - lo > 1e-13 * std::max(1.0, std::fabs(lo)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (h(mid) < 0.0) lo = mid; else hi = mid;
  }
  const double c = 0.5 * (lo + hi);
  *delta = c - M;
  if (sigma) {
    const double var = rel_var_f(s0, c) / s0.n_eff + rel_var_f(s1, c) / s1.n_eff;
    *sigma = std::sqrt(std::max(var, 0.0));
  }
  return NNP_OK;
}
