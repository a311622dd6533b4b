// host_stats.cpp -- steady-state estimate from per-unit hit counters (host,
// double precision).  A unit is one trajectory, or one batch of a single long
// trajectory (batch means).  The paper estimates steady-state probabilities
// with the two-state Markov chain approach of Raftery and Lewis (Sections 1
// and 4.2); its published figures are reported beside the confidence interval.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <limits>

#include "internal.h"

namespace {

pbn_status fail(pbn_status code, const char* msg) {
  pbn::set_error(msg);
  return code;
}

// Standard normal quantile: bisection on the CDF 0.5 erfc(-x / sqrt 2), then
// two Newton steps (the density is known in closed form).
double normal_quantile(double p) {
  double lo = -40.0, hi = 40.0;
  for (int it = 0; it < 200 && hi - lo > 1e-12; ++it) {
    const double mid = 0.5 * (lo + hi);
    (0.5 * std::erfc(-mid / std::sqrt(2.0)) < p ? lo : hi) = mid;
  }
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 2; ++it) {
    const double f = 0.5 * std::erfc(-x / std::sqrt(2.0)) - p;
    x -= f / (std::exp(-0.5 * x * x) / std::sqrt(2.0 * M_PI));
  }
  return x;
}

// Regularised incomplete beta I_x(a, b): the standard continued fraction of the
// incomplete beta function, evaluated with the modified Lentz method (Lentz 1976;
// Thompson and Barnett 1986), as numerical-methods texts lay it out.
double betacf(double a, double b, double x) {
  const double tiny = 1e-300, eps = 1e-16;
  double c = 1.0, d = 1.0 - (a + b) * x / (a + 1.0);
  if (std::fabs(d) < tiny) d = tiny;
  d = 1.0 / d;
  double h = d;
  for (int m = 1; m <= 500; ++m) {
    const double m2 = 2.0 * m;
    double aa = m * (b - m) * x / ((a - 1.0 + m2) * (a + m2));
    d = 1.0 + aa * d;
    if (std::fabs(d) < tiny) d = tiny;
    c = 1.0 + aa / c;
    if (std::fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    h *= d * c;
    aa = -(a + m) * (a + b + m) * x / ((a + m2) * (a + 1.0 + m2));
    d = 1.0 + aa * d;
    if (std::fabs(d) < tiny) d = tiny;
    c = 1.0 + aa / c;
    if (std::fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double del = d * c;
    h *= del;
    if (std::fabs(del - 1.0) < eps) break;
  }
  return h;
}

// x and its complement xc = 1 - x are passed separately: callers compute the
// complement without cancellation.
double inc_beta(double a, double b, double x, double xc) {
  if (x <= 0) return 0;
  if (xc <= 0) return 1;
  const double lbt = std::lgamma(a + b) - std::lgamma(a) - std::lgamma(b) + a * std::log(x) + b * std::log(xc);
  if (x < (a + 1) / (a + b + 2)) return std::exp(lbt) * betacf(a, b, x) / a;
  return 1.0 - std::exp(lbt) * betacf(b, a, xc) / b;
}

// Student t CDF with nu degrees of freedom: 1 - I_x(nu/2, 1/2) / 2 for t >= 0,
// x = nu / (nu + t^2).  Near t = 0 the central mass I_xc(1/2, nu/2) is used
// directly so that small quantiles keep their relative precision.
double t_cdf(double t, double nu) {
  const double t2 = t * t;
  const double x = nu / (nu + t2), xc = t2 / (nu + t2);
  if (xc < 0.5) {
    const double central = inc_beta(0.5, nu / 2, xc, x);   // P(|T| <= |t|)
    return t >= 0 ? 0.5 + 0.5 * central : 0.5 - 0.5 * central;
  }
  const double tail = 0.5 * inc_beta(nu / 2, 0.5, x, xc);
  return t >= 0 ? 1 - tail : tail;
}

// Student t quantile: bisection on the CDF (monotone), to 1e-14 relative.
double t_quantile(double p, double nu) {
  if (nu > 1e7) return normal_quantile(p);
  double lo = -1.0, hi = 1.0;
  while (t_cdf(lo, nu) > p) lo *= 2;
  while (t_cdf(hi, nu) < p) hi *= 2;
  for (int it = 0; it < 400 && hi - lo > 1e-15 * std::fmax(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    (t_cdf(mid, nu) < p ? lo : hi) = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace

extern "C" double pbn_t_quantile(double p, double nu) { return t_quantile(p, nu); }
extern "C" double pbn_normal_quantile(double p) { return normal_quantile(p); }

extern "C" pbn_status pbn_estimate(const uint64_t* counts, uint32_t units, uint64_t steps_per_unit, double conf,
                                   double precision, pbn_estimate_out* out) {
  pbn::clear_error();
  if (!counts || !out || units == 0 || steps_per_unit == 0) return fail(PBN_EINVAL, "bad argument");
  if (!(conf > 0 && conf < 1)) return fail(PBN_EINVAL, "confidence must be in (0, 1)");
  const double T = double(steps_per_unit);
  double sum = 0, n01 = 0, n10 = 0;
  for (uint32_t u = 0; u < units; ++u) {
    sum += double(counts[3 * size_t(u)]);
    n01 += double(counts[3 * size_t(u) + 1]);
    n10 += double(counts[3 * size_t(u) + 2]);
  }
  const double mean = sum / (units * T);
  double ss = 0;
  for (uint32_t u = 0; u < units; ++u) {
    const double m = double(counts[3 * size_t(u)]) / T - mean;
    ss += m * m;
  }
  out->p_hat = mean;
  out->units = units;
  out->reserved = 0;
  out->half_width = std::numeric_limits<double>::quiet_NaN();
  if (units >= 2) {
    const double sd = std::sqrt(ss / (units - 1));
    out->half_width = t_quantile(0.5 + conf / 2, double(units - 1)) * sd / std::sqrt(double(units));
  }
  // two-state chain of the hit indicator: visits of state 1 = hits, of state 0 = the rest
  const double v1 = sum, v0 = units * T - sum;
  const double alpha = v0 > 0 ? n01 / v0 : 0.0, beta = v1 > 0 ? n10 / v1 : 0.0;
  out->alpha = alpha;
  out->beta = beta;
  out->n_required = std::numeric_limits<double>::infinity();
  out->burn_in = std::numeric_limits<double>::infinity();
  if (alpha + beta > 0 && precision > 0) {
    const double z = normal_quantile(0.5 + conf / 2);
    out->n_required = alpha * beta * (2 - alpha - beta) / std::pow(alpha + beta, 3) * (z / precision) * (z / precision);
    const double lam = std::fabs(1 - alpha - beta);
    // lam = 0 (independent) or 1 (alpha = beta = 1, a deterministic alternation):
    // the logarithm is -inf or 0; one step of burn-in
    out->burn_in = lam == 0 || lam == 1 ? 1.0 : std::log(1e-3 * (alpha + beta) / std::fmax(alpha, beta)) / std::log(lam);
  }
  return PBN_OK;
}

// ---------------------------------------------------------------------------
// Raftery and Lewis (1992), single chain, on a recorded hit-indicator sequence
// (bit t of the words = z_t).  Thinning k: the smallest k whose k-thinned
// sequence z_0, z_k, z_2k, ... prefers a first-order to a second-order Markov
// chain: BIC = G^2 - 2 log(L - 2) < 0, G^2 the likelihood-ratio statistic of
// the two models (two degrees of freedom), L the thinned length.  alpha and
// beta are estimated on the k-thinned sequence; burn-in = m* k and required
// sample size = N* k original steps (m*, N* as in pbn_estimate).

namespace {

inline uint32_t bit_at(const uint32_t* w, uint64_t t) { return (w[t >> 5] >> (t & 31u)) & 1u; }

double g2_second_vs_first(const uint64_t n[2][2][2]) {
  double g2 = 0.0;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const double nij = double(n[i][j][0] + n[i][j][1]);
      for (int l = 0; l < 2; ++l) {
        const double nijl = double(n[i][j][l]);
        if (nijl == 0) continue;
        const double njl = double(n[0][j][l] + n[1][j][l]);
        const double nj = double(n[0][j][0] + n[0][j][1] + n[1][j][0] + n[1][j][1]);
        g2 += 2.0 * nijl * std::log((nijl / nij) / (njl / nj));
      }
    }
  return g2;
}

}  // namespace

extern "C" pbn_status pbn_rl_diagnose(const uint32_t* bits, uint64_t nbits, double precision, double conf,
                                      double eps, uint32_t kmax, pbn_rl_out* out) {
  pbn::clear_error();
  if (!bits || !out || nbits < 3 || kmax < 1) return fail(PBN_EINVAL, "bad argument");
  if (!(conf > 0 && conf < 1) || !(precision > 0) || !(eps > 0)) return fail(PBN_EINVAL, "bad precision/confidence");
  uint32_t k = kmax;
  double g2 = std::numeric_limits<double>::quiet_NaN(), bic = g2;
  for (uint32_t kk = 1; kk <= kmax; ++kk) {
    const uint64_t L = (nbits + kk - 1) / kk;   // thinned length
    if (L < 3) break;
    uint64_t n[2][2][2] = {};
    uint32_t a = bit_at(bits, 0), b = bit_at(bits, kk);
    for (uint64_t s = 2; s < L; ++s) {
      const uint32_t c = bit_at(bits, s * kk);
      ++n[a][b][c];
      a = b;
      b = c;
    }
    g2 = g2_second_vs_first(n);
    bic = g2 - 2.0 * std::log(double(L - 2));
    if (bic < 0) {
      k = kk;
      break;
    }
  }
  const uint64_t L = (nbits + k - 1) / k;
  uint64_t n01 = 0, n10 = 0, n0 = 0, n1 = 0;
  for (uint64_t s = 0; s + 1 < L; ++s) {
    const uint32_t a = bit_at(bits, s * k), b = bit_at(bits, (s + 1) * k);
    if (a == 0) {
      ++n0;
      n01 += b;
    } else {
      ++n1;
      n10 += 1u - b;
    }
  }
  const double alpha = n0 ? double(n01) / double(n0) : 0.0, beta = n1 ? double(n10) / double(n1) : 0.0;
  out->k = k;
  out->reserved = 0;
  out->g2 = g2;
  out->bic = bic;
  out->alpha = alpha;
  out->beta = beta;
  out->n_required = std::numeric_limits<double>::infinity();
  out->burn_in = std::numeric_limits<double>::infinity();
  out->p_hat = std::numeric_limits<double>::quiet_NaN();
  out->steps = nbits;
  if (alpha + beta > 0) {
    const double z = normal_quantile(0.5 + conf / 2);
    const double nstar = alpha * beta * (2 - alpha - beta) / std::pow(alpha + beta, 3) * (z / precision) * (z / precision);
    const double lam = std::fabs(1 - alpha - beta);
    const double mstar = lam == 0 || lam == 1 ? 1.0 : std::log(eps * (alpha + beta) / std::fmax(alpha, beta)) / std::log(lam);
    out->n_required = nstar * k;
    out->burn_in = mstar * k;
    const uint64_t first = uint64_t(std::ceil(out->burn_in));
    if (first < nbits) {
      uint64_t ones = 0;
      for (uint64_t t = first; t < nbits; ++t) ones += bit_at(bits, t);
      out->p_hat = double(ones) / double(nbits - first);
    }
  }
  return PBN_OK;
}

// ------------------------------------------------------------------ Skart
// The Skart stopping rule (Tafazzoli, Steiger and Wilson, 2011), the second
// steady-state procedure the paper's authors name beside the two-state Markov
// chain approach (Section 1), on a recorded 0/1 sequence.  Batch sums are
// counted from the packed bits; every mean of batch means is the number of ones
// it covers over the number of observations, so equal batch means deviate by
// exactly zero.

namespace {

constexpr uint32_t kSkK0 = 1280, kSkKmax = 1024, kSkKmin = 30, kSkDmax = 10;
constexpr double kSkSkew = 4.0, kSkAlpha = 0.20;

// ones among bits [a, b)
uint64_t ones_in(const uint32_t* w, uint64_t a, uint64_t b) {
  uint64_t c = 0;
  while (a < b && (a & 31u)) c += bit_at(w, a++);
  for (; a + 32 <= b; a += 32) c += uint64_t(__builtin_popcount(w[a >> 5]));
  while (a < b) c += bit_at(w, a++);
  return c;
}

// Moments of the batch means c_j / m of the sums listed in `c` (n of them).
struct BatchStats {
  bool constant;
  double mean, ss, s3, sdiff2, slag;
};

BatchStats batch_stats(const std::vector<uint64_t>& c, uint64_t m) {
  BatchStats r{true, 0.0, 0.0, 0.0, 0.0, 0.0};
  const size_t n = c.size();
  uint64_t total = 0;
  for (size_t j = 0; j < n; ++j) {
    total += c[j];
    if (c[j] != c[0]) r.constant = false;
  }
  const double dm = double(m);
  r.mean = double(total) / (double(n) * dm);
  if (r.constant) return r;
  double prev = 0.0;
  for (size_t j = 0; j < n; ++j) {
    const double y = double(c[j]) / dm, dev = y - r.mean;
    r.ss += dev * dev;
    r.s3 += dev * dev * dev;
    if (j) {
      const double yp = double(c[j - 1]) / dm;
      r.sdiff2 += (y - yp) * (y - yp);
      r.slag += prev * dev;
    }
    prev = dev;
  }
  return r;
}

double sample_skewness(const BatchStats& s, size_t k) {
  if (k < 3 || s.constant) return 0.0;
  const double kk = double(k), m2 = s.ss / kk, g1 = (s.s3 / kk) / std::pow(m2, 1.5);
  return g1 * std::sqrt(kk * (kk - 1.0)) / (kk - 2.0);
}

double willink(double zeta, double beta) {
  if (beta == 0.0) return zeta;
  const double u = 6.0 * beta * (zeta - beta);
  const double root = u > -1.0 ? std::expm1(std::log1p(u) / 3.0) : std::cbrt(1.0 + u) - 1.0;
  return root / (2.0 * beta);
}

std::vector<uint64_t> sums_of(const uint32_t* bits, uint64_t start, uint64_t k, uint64_t m) {
  std::vector<uint64_t> c(k);
  for (uint64_t j = 0; j < k; ++j) c[j] = ones_in(bits, start + j * m, start + (j + 1) * m);
  return c;
}

}  // namespace

extern "C" pbn_status pbn_skart_analyze(const uint32_t* bits, uint64_t nbits, double precision, double conf,
                                        pbn_skart_out* out) {
  pbn::clear_error();
  if (!out || (nbits && !bits)) return fail(PBN_EINVAL, "null argument");
  if (!(conf > 0 && conf < 1) || !(precision > 0)) return fail(PBN_EINVAL, "bad precision/confidence");
  const double nan = std::numeric_limits<double>::quiet_NaN();
  *out = pbn_skart_out{};
  out->p_hat = out->lower = out->upper = out->half_width = nan;
  out->skewness = out->lag1 = out->ar_factor = nan;
  out->steps = nbits;
  auto need = [&](uint64_t n) {
    out->n_required = n;
    return PBN_OK;
  };
  // batch size until the last 80 % of the batch means are nearly symmetric
  uint64_t m = 1, k = kSkK0;
  out->stage = 1;
  for (;;) {
    out->batch_size = m;
    out->batch_count = uint32_t(k);
    if (k * m > nbits) return need(k * m);
    const std::vector<uint64_t> all = sums_of(bits, 0, k, m);
    const std::vector<uint64_t> tail(all.begin() + (k - uint64_t(0.8 * double(k))), all.end());
    if (std::fabs(sample_skewness(batch_stats(tail, m), tail.size())) <= kSkSkew) break;
    m *= 2;
  }
  // randomness test of batch means spaced by d batches; the spacer fixes the warm-up
  out->stage = 2;
  uint32_t b = 0, d = 0;
  for (;;) {
    out->batch_size = m;
    out->batch_count = uint32_t(k);
    out->failures = b;
    if (k * m > nbits) return need(k * m);
    const std::vector<uint64_t> all = sums_of(bits, 0, k, m);
    const double alpha = kSkAlpha * std::exp(-0.184 * double(b) * double(b));
    const double zc = normal_quantile(1.0 - alpha / 2.0);
    bool pass = false;
    for (d = 0; d <= kSkDmax && !pass; ++d) {
      std::vector<uint64_t> sp;
      for (uint64_t j = d; j < k; j += d + 1) sp.push_back(all[j]);
      const size_t kk = sp.size();
      if (kk < 3) continue;
      const BatchStats s = batch_stats(sp, m);
      const double c = s.constant ? 0.0 : 1.0 - s.sdiff2 / (2.0 * s.ss);
      const double sd = std::sqrt((double(kk) - 2.0) / (double(kk) * double(kk) - 1.0));
      if (std::fabs(c) <= zc * sd) pass = true;
    }
    if (pass) {
      --d;
      break;
    }
    ++b;
    m = uint64_t(std::ceil(std::sqrt(2.0) * double(m)));
    k = std::max<uint64_t>(uint64_t(std::ceil(0.9 * double(k))), kSkKmin);
  }
  const uint64_t w = uint64_t(d) * m;
  out->spacer = d;
  out->warmup = w;
  // interval on the post-warm-up observations, enlarged until precise enough
  out->stage = 3;
  uint64_t kc = std::min<uint64_t>(k - d, kSkKmax);
  uint64_t mc = (k * m - w) / kc;
  for (;;) {
    out->ci_batches = uint32_t(kc);
    out->ci_batch_size = mc;
    const uint64_t n = w + kc * mc;
    if (n > nbits) return need(n);
    const std::vector<uint64_t> c = sums_of(bits, w, kc, mc);
    const BatchStats s = batch_stats(c, mc);
    const double kk = double(kc);
    const double var = s.constant ? 0.0 : s.ss / (kk - 1.0);
    const double skew = sample_skewness(s, kc);
    const double phi = std::fmin(s.constant ? 0.0 : s.slag / s.ss, 0.99);
    const double a = std::fmax(1.0, (1.0 + phi) / (1.0 - phi));
    const double beta = skew / (6.0 * std::sqrt(kk));
    const double se = std::sqrt(a * var / kk);
    const double tq = t_quantile(0.5 + conf / 2.0, kk - 1.0);
    const double lo = s.mean - willink(tq, beta) * se, hi = s.mean - willink(-tq, beta) * se;
    out->p_hat = s.mean;
    out->lower = lo;
    out->upper = hi;
    out->half_width = std::fmax(s.mean - lo, hi - s.mean);
    out->skewness = skew;
    out->lag1 = phi;
    out->ar_factor = a;
    if (var > 0.0 && out->half_width <= precision) {
      out->done = 1;
      return need(n);
    }
    const double f = var > 0.0 ? (out->half_width / precision) * (out->half_width / precision) : 2.0;
    const double grow = f * kk;
    mc = uint64_t(std::ceil(double(mc) * std::fmax(1.0, grow / double(kSkKmax))));
    kc = std::min<uint64_t>(uint64_t(std::ceil(grow)), kSkKmax);
  }
}
