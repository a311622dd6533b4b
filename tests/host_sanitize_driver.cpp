// host_sanitize_driver.cpp -- drives every host-side entry point of the C ABI
// (network validation, preparation with every option, plan queries and
// export, targets, estimators, the two-state diagnosis) on seeded random
// networks and on invalid inputs.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py; no device code.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "pbn.h"

namespace {

int g_failures = 0;
constexpr uint32_t kRemoved = 0xFFFFFFFFu;   // pbn_plan_node_pos of a node the reduction removed
#define CHECK(x)                                                          \
  do {                                                                    \
    if (!(x)) {                                                           \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #x, __LINE__); \
      ++g_failures;                                                       \
    }                                                                     \
  } while (0)

struct Rng {  // xorshift64*
  uint64_t s;
  uint64_t next() {
    s ^= s >> 12;
    s ^= s << 25;
    s ^= s >> 27;
    return s * 0x2545F4914F6CDD1Dull;
  }
  uint32_t below(uint32_t n) { return uint32_t(next() % n); }
  double unit() { return double(next() >> 11) * (1.0 / 9007199254740992.0); }
};

struct Desc {
  uint32_t n = 0;
  double p = 0.01;
  std::vector<uint32_t> fn_off, par_off, parents, tt_off;
  std::vector<double> sel;
  std::vector<uint64_t> tt;
  pbn_desc view() const {
    return pbn_desc{n, p, fn_off.data(), sel.data(), par_off.data(), parents.data(), tt_off.data(), tt.data()};
  }
};

Desc random_desc(Rng& r, uint32_t n, uint32_t lmax, uint32_t kmax) {
  Desc d;
  d.n = n;
  d.p = 1e-4 + 0.05 * r.unit();
  d.fn_off.push_back(0);
  d.par_off.push_back(0);
  d.tt_off.push_back(0);
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t l = 1 + r.below(lmax);
    double sum = 0.0;
    std::vector<double> w(l);
    for (auto& x : w) sum += (x = 0.05 + r.unit());
    for (uint32_t j = 0; j < l; ++j) {
      d.sel.push_back(w[j] / sum);
      const uint32_t k = std::min(n, r.below(kmax + 1));
      std::vector<uint32_t> ps;
      while (ps.size() < k) {
        const uint32_t q = r.below(n);
        bool dup = false;
        for (uint32_t x : ps) dup |= x == q;
        if (!dup) ps.push_back(q);
      }
      d.parents.insert(d.parents.end(), ps.begin(), ps.end());
      d.par_off.push_back(uint32_t(d.parents.size()));
      const uint32_t words = ((1u << k) + 63) / 64;
      for (uint32_t t = 0; t < words; ++t) {
        uint64_t v = r.next();
        if ((1u << k) < 64) v &= (1ull << (1u << k)) - 1ull;
        d.tt.push_back(v);
      }
      d.tt_off.push_back(uint32_t(d.tt.size()));
    }
    d.fn_off.push_back(uint32_t(d.sel.size()));
  }
  return d;
}

void exercise_plan(pbn_net* net, const Desc& d, Rng& r, const pbn_plan_opts& o) {
  std::vector<uint32_t> interest;
  for (uint32_t k = 0, m = 1 + r.below(3); k < m; ++k) interest.push_back(r.below(d.n));
  pbn_plan* plan = nullptr;
  const pbn_status st = pbn_plan_build(net, interest.data(), uint32_t(interest.size()), &o, &plan);
  if (st != PBN_OK) {
    CHECK(st == PBN_ELIMIT || st == PBN_ELDS);
    CHECK(plan == nullptr);
    CHECK(pbn_last_error()[0] != '\0');
    return;
  }
  pbn_plan_info info{};
  CHECK(pbn_plan_info_get(plan, &info) == PBN_OK);
  CHECK(info.n == d.n && info.n_kept >= 1 && info.n_kept <= d.n);
  std::vector<uint32_t> pos(d.n), slot(d.n), is_table(info.n_slots);
  CHECK(pbn_plan_node_pos(plan, pos.data()) == PBN_OK);
  CHECK(pbn_plan_slots(plan, slot.data(), is_table.data()) == PBN_OK);
  for (uint32_t v : interest) CHECK(pos[v] != kRemoved);
  for (auto fn : {pbn_plan_alg4_groups, pbn_plan_single_groups}) {
    uint32_t nm = 0, ng = 0;
    CHECK(fn(plan, nullptr, &nm, nullptr, &ng) == PBN_OK);
    std::vector<uint32_t> mem(nm + 1), off(ng + 1);
    CHECK(fn(plan, mem.data(), &nm, off.data(), &ng) == PBN_OK);
    CHECK(off[ng] == nm);
  }
  size_t bytes = 0;
  CHECK(pbn_plan_export(plan, nullptr, &bytes) == PBN_OK);
  std::vector<uint8_t> blob(bytes);
  size_t small = bytes / 2;
  CHECK(pbn_plan_export(plan, blob.data(), &small) == PBN_EINVAL);
  CHECK(pbn_plan_export(plan, blob.data(), &bytes) == PBN_OK);
  CHECK(bytes == info.blob_bytes);
  // targets: a pair on a kept node builds, one on a removed node is refused
  pbn_targets tg{};
  uint32_t node = interest[0], val = 1, tof = 0;
  CHECK(pbn_targets_build(plan, &node, &val, &tof, 1, 1, &tg) == PBN_OK);
  for (uint32_t v = 0; v < d.n; ++v)
    if (pos[v] == kRemoved) {
      node = v;
      CHECK(pbn_targets_build(plan, &node, &val, &tof, 1, 1, &tg) == PBN_EINVAL);
      break;
    }
  CHECK(pbn_plan_destroy(plan) == PBN_OK);
}

void exercise_invalid(Rng& r) {
  Desc d = random_desc(r, 6, 3, 3);
  pbn_net* net = nullptr;
  pbn_desc v = d.view();
  v.n = 0;
  CHECK(pbn_net_create(&v, &net) != PBN_OK);
  v = d.view();
  v.p = 1.5;
  CHECK(pbn_net_create(&v, &net) != PBN_OK);
  Desc bad = d;
  bad.parents[0] = 99;
  v = bad.view();
  CHECK(pbn_net_create(&v, &net) != PBN_OK);
  bad = d;
  bad.sel[0] += 0.25;
  v = bad.view();
  CHECK(pbn_net_create(&v, &net) != PBN_OK);
  CHECK(pbn_net_create(nullptr, &net) != PBN_OK);
  v = d.view();
  CHECK(pbn_net_create(&v, &net) == PBN_OK);
  pbn_plan_opts o;
  pbn_plan_opts_default(&o);
  pbn_plan* plan = nullptr;
  uint32_t interest = 0, out_of_range = 6;
  pbn_plan_opts b = o;
  b.reduce = 3;
  CHECK(pbn_plan_build(net, &interest, 1, &b, &plan) == PBN_EINVAL);
  b = o;
  b.sampling = 2;
  CHECK(pbn_plan_build(net, &interest, 1, &b, &plan) == PBN_EINVAL);
  b = o;
  b.max_group_nodes = 0;
  CHECK(pbn_plan_build(net, &interest, 1, &b, &plan) == PBN_EINVAL);
  CHECK(pbn_plan_build(net, &out_of_range, 1, &o, &plan) == PBN_EINVAL);
  CHECK(pbn_plan_build(nullptr, &interest, 1, &o, &plan) == PBN_EINVAL);
  CHECK(plan == nullptr);
  CHECK(pbn_net_destroy(net) == PBN_OK);
}

void exercise_stats(Rng& r) {
  for (int rep = 0; rep < 50; ++rep) {
    const uint32_t units = 1 + r.below(40);
    const uint64_t steps = 1 + r.below(10000);
    std::vector<uint64_t> counts(3 * units);
    for (uint32_t u = 0; u < units; ++u) {
      const uint64_t h = r.below(uint32_t(steps + 1));
      counts[3 * u] = h;
      counts[3 * u + 1] = r.below(uint32_t(std::min<uint64_t>(h, steps - h) + 1));
      counts[3 * u + 2] = counts[3 * u + 1];
    }
    pbn_estimate_out e{};
    const pbn_status st = pbn_estimate(counts.data(), units, steps, 0.95, 0.01, &e);
    CHECK(st == PBN_OK);
    if (st == PBN_OK) CHECK(e.p_hat >= 0.0 && e.p_hat <= 1.0);
    const uint64_t nbits = 3 + r.below(6000);
    std::vector<uint32_t> bits((nbits + 31) / 32);
    const double q = r.unit();
    for (uint64_t b = 0; b < nbits; ++b)
      if (r.unit() < q) bits[b / 32] |= 1u << (b % 32);
    pbn_rl_out o{};
    const pbn_status s2 = pbn_rl_diagnose(bits.data(), nbits, 0.01, 0.95, 1e-3, 100, &o);
    CHECK(s2 == PBN_OK || s2 == PBN_EINVAL || s2 == PBN_ERANGE);
    pbn_skart_out so{};
    CHECK(pbn_skart_analyze(bits.data(), nbits, 0.001 + 0.1 * r.unit(), 0.95, &so) == PBN_OK);
    CHECK(so.done ? so.n_required <= nbits : so.n_required > nbits);
    CHECK(pbn_skart_analyze(bits.data(), nbits, 0.0, 0.95, &so) == PBN_EINVAL);
    std::vector<uint64_t> w(1 + r.below(12));
    for (auto& x : w) x = 2 + r.below(1000);
    uint32_t m = 0;
    CHECK(pbn_eq2_lower_bound(w.data(), uint32_t(w.size()), 1 + r.below(1u << 20), &m) == PBN_OK);
    CHECK(std::isfinite(pbn_t_quantile(0.975, 1.0 + r.below(100))));
    CHECK(std::isfinite(pbn_normal_quantile(0.001 + 0.998 * r.unit())));
  }
  uint64_t c[3] = {1, 0, 0};
  pbn_estimate_out e{};
  CHECK(pbn_estimate(c, 0, 10, 0.95, 0.01, &e) != PBN_OK);
  CHECK(pbn_estimate(nullptr, 1, 10, 0.95, 0.01, &e) != PBN_OK);
}

}  // namespace

int main() {
  Rng r{0x9E3779B97F4A7C15ull};
  for (int rep = 0; rep < 24; ++rep) {
    const uint32_t n = 2 + r.below(rep < 20 ? 150 : 900);
    const Desc d = random_desc(r, n, 1 + r.below(4), 1 + r.below(7));
    pbn_net* net = nullptr;
    const pbn_desc v = d.view();
    if (pbn_net_create(&v, &net) != PBN_OK) {
      std::fprintf(stderr, "network %d rejected: %s\n", rep, pbn_last_error());
      ++g_failures;
      continue;
    }
    std::vector<uint64_t> q(n + 1);
    std::vector<uint64_t> cum(3 * size_t(n));
    std::vector<int32_t> rank(n);
    CHECK(pbn_net_tables(net, q.data(), cum.data(), rank.data()) == PBN_OK);
    for (uint32_t reduce = 0; reduce <= 2; ++reduce)
      for (uint32_t group = 0; group <= 1; ++group)
        for (uint32_t sampling = 0; sampling <= 1; ++sampling) {
          pbn_plan_opts o;
          pbn_plan_opts_default(&o);
          o.reduce = reduce;
          o.group = group;
          o.sampling = sampling;
          o.weight_mode = r.below(2);
          o.lds_budget_bytes = r.below(2) ? 65536 : 0;
          o.max_parent_bits = 4 + r.below(9);
          o.max_group_nodes = 1 + r.below(4);
          o.theta = 1 + r.below(1u << 20);
          exercise_plan(net, d, r, o);
        }
    CHECK(pbn_net_destroy(net) == PBN_OK);
  }
  exercise_invalid(r);
  exercise_stats(r);
  std::printf("host driver: %d failures\n", g_failures);
  return g_failures ? 1 : 0;
}
