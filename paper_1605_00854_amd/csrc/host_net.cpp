// host_net.cpp -- network validation and integer quantisation (host, once per
// network).  The PBN model is Section 2.1 of the paper; the integer tables are
// this library's random-number contract (see pbn.h).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>

#include "internal.h"

namespace pbn {
static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }
const char* last_error() { return g_last_error.c_str(); }
}  // namespace pbn

static pbn_status fail(pbn_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  pbn::set_error(buf);
  return code;
}

extern "C" const char* pbn_last_error(void) { return pbn::last_error(); }

// Q[h] = floor(v_h * 2^64), v_0 = 1, v_h = v_{h-1} * (1 - p): the probability that
// h consecutive nodes are all unperturbed, as a 64-bit threshold.
static void quantise_perturbation(pbn_net& g) {
  g.Q.assign(g.n + 1, 0);
  const double q = 1.0 - g.p;
  double v = 1.0;
  for (uint32_t h = 1; h <= g.n; ++h) {
    v = v * q;
    g.Q[h] = static_cast<uint64_t>(std::floor(std::ldexp(v, 64)));
  }
}

// CUM[m] = min(2^32, floor(S_m * 2^32 + 1/2)), S_m the left-to-right double
// partial sum of the selection probabilities.  A 32-bit uniform never reaches
// 2^32, so a predictor after a partial sum of 1 (probability 0) is never chosen.
static void quantise_selection(pbn_net& g) {
  g.cum.assign(3 * size_t(g.n), kCumNever);
  for (uint32_t i = 0; i < g.n; ++i) {
    double s = 0.0;
    const uint32_t l = g.nfn(i);
    for (uint32_t m = 0; m + 1 < l; ++m) {
      s = s + g.sel[g.fn_off[i] + m];
      const double v = std::floor(std::ldexp(s, 32) + 0.5);
      g.cum[3 * size_t(i) + m] = v >= 4294967296.0 ? kCumNever : static_cast<uint64_t>(v);
    }
  }
  g.rank.assign(g.n, -1);
  g.n_multi = 0;
  for (uint32_t i = 0; i < g.n; ++i)
    if (g.nfn(i) >= 2) g.rank[i] = int32_t(g.n_multi++);
}

extern "C" pbn_status pbn_net_create(const pbn_desc* d, pbn_net** out) {
  pbn::clear_error();
  if (!d || !out) return fail(PBN_EINVAL, "null argument");
  *out = nullptr;
  if (d->n == 0) return fail(PBN_EINVAL, "n must be >= 1");
  if (d->n > PBN_MAX_NODES) return fail(PBN_ELIMIT, "n = %u exceeds %u", d->n, PBN_MAX_NODES);
  if (!(d->p > 0.0 && d->p < 1.0) || !(1.0 - d->p < 1.0))
    return fail(PBN_EINVAL, "perturbation rate p must satisfy 0 < p < 1 and 1 - p < 1");
  if (!d->fn_off || !d->sel_prob || !d->par_off || !d->tt_off || !d->tt)
    return fail(PBN_EINVAL, "null array in network description");
  const uint32_t n = d->n;
  if (d->fn_off[0] != 0) return fail(PBN_EINVAL, "fn_off[0] must be 0");
  for (uint32_t i = 0; i < n; ++i) {
    if (d->fn_off[i + 1] <= d->fn_off[i]) return fail(PBN_EINVAL, "node %u has no predictor", i);
    if (d->fn_off[i + 1] - d->fn_off[i] > PBN_MAX_PREDICTORS)
      return fail(PBN_ELIMIT, "node %u has more than %d predictors", i, PBN_MAX_PREDICTORS);
  }
  const uint32_t nf = d->fn_off[n];
  if (d->par_off[0] != 0 || d->tt_off[0] != 0)
    return fail(PBN_EINVAL, "par_off[0] and tt_off[0] must be 0");
  for (uint32_t f = 0; f < nf; ++f) {
    if (d->par_off[f + 1] < d->par_off[f]) return fail(PBN_EINVAL, "par_off not monotone at %u", f);
    const uint32_t k = d->par_off[f + 1] - d->par_off[f];
    if (k > PBN_MAX_FN_PARENTS)
      return fail(PBN_ELIMIT, "predictor %u has %u parents (max %d)", f, k, PBN_MAX_FN_PARENTS);
    const uint32_t words = k <= 6 ? 1u : (1u << k) / 64u;
    if (d->tt_off[f + 1] < d->tt_off[f] || d->tt_off[f + 1] - d->tt_off[f] != words)
      return fail(PBN_EINVAL, "predictor %u: truth table must have %u words", f, words);
    for (uint32_t j = d->par_off[f]; j < d->par_off[f + 1]; ++j)
      if (!d->parents || d->parents[j] >= n)
        return fail(PBN_EINVAL, "predictor %u: parent id out of range", f);
    if (k < 6) {
      const uint64_t used = (1ull << (1u << k)) - 1ull;
      if (d->tt[d->tt_off[f]] & ~used)
        return fail(PBN_EINVAL, "predictor %u: truth-table bits above 2^%u must be zero", f, k);
    }
  }
  for (uint32_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (uint32_t f = d->fn_off[i]; f < d->fn_off[i + 1]; ++f) {
      const double c = d->sel_prob[f];
      if (!std::isfinite(c) || c < 0.0) return fail(PBN_EINVAL, "node %u: bad selection probability", i);
      s += c;
    }
    if (std::fabs(s - 1.0) > 1e-9) return fail(PBN_EINVAL, "node %u: selection probabilities sum to %.17g", i, s);
  }
  try {
    auto* g = new pbn_net;
    g->n = n;
    g->p = d->p;
    g->fn_off.assign(d->fn_off, d->fn_off + n + 1);
    g->sel.assign(d->sel_prob, d->sel_prob + nf);
    g->par_off.assign(d->par_off, d->par_off + nf + 1);
    g->parents.assign(d->parents ? d->parents : d->par_off, (d->parents ? d->parents : d->par_off) + d->par_off[nf]);
    g->tt_off.assign(d->tt_off, d->tt_off + nf + 1);
    g->tt.assign(d->tt, d->tt + d->tt_off[nf]);
    quantise_perturbation(*g);
    quantise_selection(*g);
    *out = g;
    return PBN_OK;
  } catch (const std::bad_alloc&) {
    return fail(PBN_ENOMEM, "out of host memory");
  }
}

extern "C" pbn_status pbn_net_destroy(pbn_net* g) {
  delete g;
  return PBN_OK;
}

extern "C" pbn_status pbn_net_tables(const pbn_net* g, uint64_t* q, uint64_t* cum, int32_t* rank) {
  pbn::clear_error();
  if (!g) return fail(PBN_EINVAL, "null network");
  if (q)
    for (uint32_t h = 0; h <= g->n; ++h) q[h] = g->Q[h];
  if (cum)
    for (size_t i = 0; i < g->cum.size(); ++i) cum[i] = g->cum[i];
  if (rank)
    for (uint32_t i = 0; i < g->n; ++i) rank[i] = g->rank[i];
  return PBN_OK;
}
