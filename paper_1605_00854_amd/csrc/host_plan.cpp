// host_plan.cpp -- Preparation of Algorithm 5 on the host: leaf-node reduction
// (Section 3.1, Definition 1), node grouping (Section 3.3: Equation 2,
// Algorithm 3, Algorithm 4, grouping of single-predictor nodes by shared
// parents), combined predictor tables, and the device blob of the step kernel.
//
// Readings where the text is silent:
//  * a self-edge makes a node its own child (self-looped nodes are never leaves);
//  * Algorithm 4 starts at m = the Eq. 2 bound, stops at the first m whose
//    weight sum is <= theta, and never exceeds one group per item;
//  * Algorithm 3 sorts by weight descending, node id ascending; empty groups
//    weigh 0; ties go to the lowest group index; products saturate at 2^62;
//  * single-predictor nodes, in node-id order, join the group sharing the most
//    parents among groups within the node/parent caps (ties: smaller union,
//    lower index), else open a new group;
//  * a combined function's index takes the first member as its most
//    significant digit; member k's output is bit k of a table entry.
// Device adaptations: groups are capped at PBN_MAX_GROUP_NODES members and
// max_parent_bits / max_table_entries; a group of Algorithm 4 that exceeds a cap
// sheds its heaviest member into a single-node slot until it fits.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.h"

namespace {

constexpr uint64_t kSat = 1ull << 62;

pbn_status fail(pbn_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  pbn::set_error(buf);
  return code;
}

uint64_t sat_mul(uint64_t a, uint64_t b) {
  if (a == 0 || b == 0) return 0;
  if (a >= kSat || b >= kSat) return kSat;
  unsigned __int128 r = (unsigned __int128)a * b;
  return r >= kSat ? kSat : uint64_t(r);
}

size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// distinct parents of node i over all of its predictors, ascending
std::vector<uint32_t> node_parents(const pbn_net& g, uint32_t i) {
  std::vector<uint32_t> u;
  for (uint32_t f = g.fn_off[i]; f < g.fn_off[i + 1]; ++f)
    for (uint32_t k = g.par_off[f]; k < g.par_off[f + 1]; ++k) u.push_back(g.parents[k]);
  std::sort(u.begin(), u.end());
  u.erase(std::unique(u.begin(), u.end()), u.end());
  return u;
}

std::vector<uint32_t> union_of(const std::vector<std::vector<uint32_t>>& P, const std::vector<uint32_t>& members) {
  std::vector<uint32_t> u;
  for (uint32_t v : members) u.insert(u.end(), P[v].begin(), P[v].end());
  std::sort(u.begin(), u.end());
  u.erase(std::unique(u.begin(), u.end()), u.end());
  return u;
}

// Walker's alias method by Vose's construction (Section 2.2): column i of a
// uniformly drawn column is kept with probability keep[i], else it yields
// alias[i].  Stacks in ascending index order, popped from the back; the keep
// probability is stored as the 32-bit threshold floor(keep 2^32) (at most
// 2^32 - 1) that a drawn 32-bit coin must stay below.
void vose_table(const std::vector<double>& probs, std::vector<uint32_t>& thr, std::vector<uint32_t>& alias) {
  const size_t L = probs.size();
  std::vector<double> scaled(L), keep(L, 0.0);
  alias.assign(L, 0);
  std::vector<uint32_t> small, large;
  for (size_t i = 0; i < L; ++i) {
    scaled[i] = probs[i] * double(L);
    (scaled[i] < 1.0 ? small : large).push_back(uint32_t(i));
  }
  while (!small.empty() && !large.empty()) {
    const uint32_t sm = small.back(), lg = large.back();
    small.pop_back();
    large.pop_back();
    keep[sm] = scaled[sm];
    alias[sm] = lg;
    scaled[lg] = scaled[lg] + scaled[sm] - 1.0;
    (scaled[lg] < 1.0 ? small : large).push_back(lg);
  }
  for (uint32_t i : large) keep[i] = 1.0, alias[i] = i;
  for (uint32_t i : small) keep[i] = 1.0, alias[i] = i;
  thr.resize(L);
  for (size_t i = 0; i < L; ++i) {
    const double x = std::floor(keep[i] * 4294967296.0);
    thr[i] = x >= 4294967295.0 ? 0xFFFFFFFFu : uint32_t(x);
  }
}

// Definition 1: iterated removal of nodes that are not of interest and have no
// remaining children.  Returns removed[v].
std::vector<uint8_t> leaf_nodes(const pbn_net& g, const std::vector<uint8_t>& interest,
                                const std::vector<std::vector<uint32_t>>& P) {
  const uint32_t n = g.n;
  std::vector<uint32_t> nchild(n, 0);
  for (uint32_t v = 0; v < n; ++v)
    for (uint32_t p : P[v]) ++nchild[p];
  std::vector<uint8_t> removed(n, 0);
  std::vector<uint32_t> stack;
  for (uint32_t v = 0; v < n; ++v)
    if (!interest[v] && nchild[v] == 0) stack.push_back(v);
  while (!stack.empty()) {
    const uint32_t v = stack.back();
    stack.pop_back();
    if (removed[v]) continue;
    removed[v] = 1;
    for (uint32_t p : P[v])
      if (--nchild[p] == 0 && !interest[p] && !removed[p]) stack.push_back(p);
  }
  return removed;
}

// Every node from which no node of interest is reachable (the complement of
// the interest nodes' ancestors): Section 3.1's argument for removing leaves
// applied to whole unreachable regions, cycles included.
std::vector<uint8_t> cone_removed(const pbn_net& g, const std::vector<uint8_t>& interest,
                                  const std::vector<std::vector<uint32_t>>& P) {
  const uint32_t n = g.n;
  std::vector<uint8_t> keep(n, 0);
  std::vector<uint32_t> stack;
  for (uint32_t v = 0; v < n; ++v)
    if (interest[v]) {
      keep[v] = 1;
      stack.push_back(v);
    }
  while (!stack.empty()) {
    const uint32_t v = stack.back();
    stack.pop_back();
    for (uint32_t p : P[v])
      if (!keep[p]) {
        keep[p] = 1;
        stack.push_back(p);
      }
  }
  std::vector<uint8_t> removed(n, 0);
  for (uint32_t v = 0; v < n; ++v) removed[v] = keep[v] ? 0 : 1;
  return removed;
}

// Algorithm 3 (greedy multi-way partition on products).
std::vector<std::vector<uint32_t>> find_partitions(std::vector<std::pair<uint32_t, uint64_t>> items, uint32_t m) {
  std::stable_sort(items.begin(), items.end(), [](const auto& a, const auto& b) {
    if (a.second != b.second) return a.second > b.second;
    return a.first < b.first;
  });
  std::vector<std::vector<uint32_t>> groups(m);
  std::vector<uint64_t> prod(m, 0);   // empty group weighs 0
  for (const auto& it : items) {
    uint32_t best = 0;
    for (uint32_t k = 1; k < m; ++k)
      if (prod[k] < prod[best]) best = k;
    prod[best] = groups[best].empty() ? it.second : sat_mul(prod[best], it.second);
    groups[best].push_back(it.first);
  }
  return groups;
}

// Algorithm 4 on the multi-predictor nodes.  Every weight is >= 2, so merging
// two groups never lowers the weight sum (a b >= a + b): when the singletons
// already exceed theta no m < k can succeed and the loop would end at m = k.
std::vector<std::vector<uint32_t>> partition_multi(const std::vector<std::pair<uint32_t, uint64_t>>& items,
                                                   uint64_t theta) {
  if (items.empty()) return {};
  std::vector<uint64_t> w;
  uint64_t singles = 0;
  uint32_t max_id = 0;
  for (const auto& it : items) {
    w.push_back(it.second);
    singles = std::min(kSat, singles + it.second);
    max_id = std::max(max_id, it.first);
  }
  const uint32_t k = uint32_t(items.size());
  if (singles > theta) return find_partitions(items, k);
  std::vector<uint64_t> weight_of(size_t(max_id) + 1, 0);
  for (const auto& it : items) weight_of[it.first] = it.second;
  const uint32_t m0 = pbn::eq2_lower_bound(w, theta);
  uint32_t m = m0 == 0 ? k : std::min(std::max(1u, m0), k);
  for (;;) {
    auto groups = find_partitions(items, m);
    uint64_t total = 0;
    for (const auto& gr : groups) {
      uint64_t pr = 1;
      for (uint32_t v : gr) pr = sat_mul(pr, weight_of[v]);
      total = std::min(kSat, total + pr);
    }
    if (total <= theta || m >= k) return groups;
    ++m;
  }
}

// Grouping of single-predictor nodes by shared parents.
std::vector<std::vector<uint32_t>> group_single(const std::vector<uint32_t>& nodes,
                                                const std::vector<std::vector<uint32_t>>& P,
                                                uint32_t max_nodes, uint32_t max_bits) {
  std::vector<std::vector<uint32_t>> groups, unions;
  for (uint32_t v : nodes) {
    const auto& pv = P[v];
    int best = -1;
    size_t best_shared = 0, best_union = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      if (groups[gi].size() >= max_nodes) continue;
      std::vector<uint32_t> u;
      std::set_union(unions[gi].begin(), unions[gi].end(), pv.begin(), pv.end(), std::back_inserter(u));
      if (u.size() > max_bits) continue;
      const size_t shared = unions[gi].size() + pv.size() - u.size();
      if (best < 0 || shared > best_shared || (shared == best_shared && u.size() < best_union)) {
        best = int(gi);
        best_shared = shared;
        best_union = u.size();
      }
    }
    if (best < 0) {
      groups.push_back({v});
      unions.push_back(pv);
    } else {
      groups[best].push_back(v);
      std::vector<uint32_t> u;
      std::set_union(unions[best].begin(), unions[best].end(), pv.begin(), pv.end(), std::back_inserter(u));
      unions[best] = u;
    }
  }
  return groups;
}

std::atomic<uint32_t> g_plan_counter{1};

// Steps per Philox fill: the f <= 32 with f * njobs <= rounds * 64 whose calls
// use the largest share of their rounds of 64 lanes (ties: the larger f, fewer
// fills); 1 when a step needs more than 64 calls.  Plans of at most two lane
// passes (small states) take up to PBN_FILL_ROUNDS rounds; larger plans one,
// since their ring shares LDS with two large state buffers per wave.
uint32_t fill_steps_for(uint32_t njobs, uint32_t npass) {
  if (njobs > PBN_WAVE) return 1;
  const uint32_t rounds = npass <= 2 ? PBN_FILL_ROUNDS : 1;
  uint32_t best = 1;
  double best_use = 0.0;
  for (uint32_t f = 1; f <= 32 && f * njobs <= rounds * PBN_WAVE; ++f) {
    const uint32_t calls = f * njobs, rounds = (calls + PBN_WAVE - 1) / PBN_WAVE;
    const double use = double(calls) / double(rounds * PBN_WAVE);
    if (use >= best_use - 1e-12) {
      best = f;
      best_use = use;
    }
  }
  return best;
}

struct Slot {
  std::vector<uint32_t> members;   // original node ids
  bool table = false;
  std::vector<uint32_t> uni;       // TABLE: union parents (ascending)
  uint32_t cost_key = 0;
};

}  // namespace

namespace pbn {
// Smallest m >= 1 with m * W^(1/m) <= theta, W = prod w, compared in logs as
// log W + m log m <= m log theta (equality accepted within 1e-12 relative).
uint32_t eq2_lower_bound(const std::vector<uint64_t>& w, uint64_t theta) {
  if (w.empty()) return 0;
  long double L = 0.0L;
  for (uint64_t x : w) L += std::log((long double)x);
  const long double lt = std::log((long double)theta);
  for (uint64_t m = 1;; ++m) {
    const long double lhs = L + (long double)m * std::log((long double)m);
    const long double rhs = (long double)m * lt;
    if (lhs <= rhs + 1e-12L * (std::fabs(rhs) + 1.0L)) return uint32_t(m);
    if ((long double)m >= L + 1.0L) return 0;     // past the minimum: failures are final
    if (m > 0xFFFFFFF0ull) return 0;
  }
}
}  // namespace pbn

extern "C" void pbn_plan_opts_default(pbn_plan_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->reduce = 1;
  o->group = 1;
  o->weight_mode = 1;
  o->lds_budget_bytes = 65536;
  o->theta = 65536;
  o->max_table_entries = 4096;
  o->max_parent_bits = 12;
  o->max_group_nodes = 4;
}

extern "C" pbn_status pbn_eq2_lower_bound(const uint64_t* weights, uint32_t count, uint64_t theta, uint32_t* m_out) {
  pbn::clear_error();
  if (!m_out || (count && !weights) || theta == 0) return fail(PBN_EINVAL, "bad argument");
  std::vector<uint64_t> w(weights, weights + count);
  for (uint64_t x : w)
    if (x == 0) return fail(PBN_EINVAL, "weights must be positive");
  *m_out = pbn::eq2_lower_bound(w, theta);
  return PBN_OK;
}

static pbn_status build_plan(const pbn_net& g, const std::vector<uint8_t>& interest, const pbn_plan_opts& o,
                             pbn_plan& plan) {
  const uint32_t n = g.n;
  std::vector<std::vector<uint32_t>> P(n);
  for (uint32_t i = 0; i < n; ++i) P[i] = node_parents(g, i);

  // ---- Step 1: leaf-node reduction (Definition 1)
  std::vector<uint8_t> removed(n, 0);
  if (o.reduce == 1) removed = leaf_nodes(g, interest, P);
  if (o.reduce == 2) removed = cone_removed(g, interest, P);
  std::vector<uint32_t> kept;
  for (uint32_t i = 0; i < n; ++i)
    if (!removed[i]) kept.push_back(i);

  auto max_phi = [&](uint32_t v) {
    uint32_t m = 0;
    for (uint32_t f = g.fn_off[v]; f < g.fn_off[v + 1]; ++f) m = std::max(m, g.nparents(f));
    return m;
  };
  auto table_entries = [&](const std::vector<uint32_t>& members) {
    uint64_t e = 1;
    for (uint32_t v : members) e = sat_mul(e, g.nfn(v));
    const size_t nu = union_of(P, members).size();
    return nu >= 62 ? kSat : sat_mul(e, 1ull << nu);
  };
  auto fits = [&](const std::vector<uint32_t>& members) {
    if (members.size() > o.max_group_nodes) return false;
    if (union_of(P, members).size() > o.max_parent_bits) return false;
    return table_entries(members) <= o.max_table_entries;
  };

  // ---- Step 3: node grouping (Section 3.3)
  std::vector<Slot> slots;
  plan.alg4_groups.clear();
  plan.single_groups.clear();
  if (o.group) {
    std::vector<std::pair<uint32_t, uint64_t>> S;
    std::vector<uint32_t> S1;
    for (uint32_t v : kept) {
      if (g.nfn(v) >= 2) {
        uint64_t w = g.nfn(v);
        if (o.weight_mode == 1) w = P[v].size() >= 62 ? kSat : sat_mul(w, 1ull << P[v].size());
        S.emplace_back(v, w);
      } else {
        S1.push_back(v);
      }
    }
    plan.alg4_groups = partition_multi(S, o.theta);
    uint32_t bits_cap = o.max_parent_bits;
    while (bits_cap > 0 && (1ull << bits_cap) > o.max_table_entries) --bits_cap;
    plan.single_groups = group_single(S1, P, o.max_group_nodes, bits_cap);
    // device caps: shed the heaviest member until the group fits
    for (auto gr : plan.alg4_groups) {
      while (gr.size() > 1 && !fits(gr)) {
        slots.push_back(Slot{{gr.front()}});
        gr.erase(gr.begin());
      }
      slots.push_back(Slot{gr});
    }
    for (const auto& gr : plan.single_groups) slots.push_back(Slot{gr});
  } else {
    for (uint32_t v : kept) slots.push_back(Slot{{v}});
  }

  // slot modes: groups use a combined table; single nodes use their predictor
  // directly unless a predictor reads more than 7 parents (128-bit inline table)
  for (auto& s : slots) {
    s.table = s.members.size() > 1 || max_phi(s.members[0]) > 7;
    if (s.table) {
      s.uni = union_of(P, s.members);
      if (s.uni.size() > PBN_MAX_GROUP_PARENTS || table_entries(s.members) > std::max<uint64_t>(o.max_table_entries, 1))
        return fail(PBN_ELIMIT, "node %u needs a table of %llu entries (max_table_entries %u)", s.members[0],
                    (unsigned long long)table_entries(s.members), o.max_table_entries);
    }
  }
  // order: table slots first (by union size, descending), then FN slots:
  // multi-predictor nodes by selection rank (neighbouring lanes then read
  // neighbouring words of a step's drawn numbers), then one-predictor nodes
  // by parent count, descending
  std::stable_sort(slots.begin(), slots.end(), [&](const Slot& a, const Slot& b) {
    if (a.table != b.table) return a.table;
    if (!a.table) {
      const bool ma = g.nfn(a.members[0]) > 1, mb = g.nfn(b.members[0]) > 1;
      if (ma != mb) return ma;
      if (ma) return g.rank[a.members[0]] < g.rank[b.members[0]];
      return max_phi(a.members[0]) > max_phi(b.members[0]);
    }
    return a.uni.size() > b.uni.size();
  });

  const uint32_t ns = uint32_t(slots.size());
  if (ns == 0) return fail(PBN_EINVAL, "plan has no nodes");
  const uint32_t npass = (ns + PBN_WAVE - 1) / PBN_WAVE;
  // state bytes: table slot s (s < n_table) owns the word at 4 s (member k at
  // byte k); FN slot s owns one byte at 4 n_table + (s - n_table); then the
  // zero word read by unused parent entries; then one byte per padded lane of
  // the last pass (written with zeros, never read).  Every byte a lookup reads
  // lies below zero_pos + 4, so small states use distinct LDS banks.
  const uint32_t ntab = uint32_t(std::count_if(slots.begin(), slots.end(), [](const Slot& s) { return s.table; }));
  const uint32_t fn_pos0 = 4 * ntab;
  const uint32_t fn_end = fn_pos0 + (ns - ntab);
  // packed-bit layout (state_bits): pass p owns a segment of 256 bits when it
  // holds a table slot (lane L's member k at 4 L + k), else 64 (lane L at L);
  // the zero word follows the last segment.  Padded lanes own their segment
  // bits and write zeros there.
  const bool bits = o.state_bits != 0;
  std::vector<uint32_t> seg(npass + 1, 0);
  for (uint32_t p = 0; p < npass; ++p) {
    const bool tab = 64 * p < ns && slots[64 * p].table;   // table slots come first
    seg[p + 1] = seg[p] + (tab ? 256u : 64u);
  }
  auto seg_table = [&](uint32_t p) { return seg[p + 1] - seg[p] == 256u; };
  const uint32_t zero_pos = bits ? seg[npass] : (fn_end + 3) & ~3u;
  const uint32_t pad_pos0 = zero_pos + 4;
  const uint32_t state_words = bits ? zero_pos / 32 + 1 : (pad_pos0 + (npass * PBN_WAVE - ns) + 31) / 32;
  if (32ull * state_words > 65535) return fail(PBN_ELDS, "too many slots (%u) for 16-bit state positions", ns);
  auto slot_pos = [&](uint32_t s, uint32_t k) {
    if (bits) return seg[s / 64] + (seg_table(s / 64) ? 4 * (s % 64) + k : s % 64);
    return s < ntab ? 4 * s + k : fn_pos0 + (s - ntab);
  };

  plan.node_pos.assign(n, PBN_NONE);
  plan.node_slot.assign(n, PBN_NONE);
  plan.slot_is_table.assign(ns, 0);
  for (uint32_t s = 0; s < ns; ++s) {
    plan.slot_is_table[s] = slots[s].table;
    for (uint32_t k = 0; k < slots[s].members.size(); ++k) {
      plan.node_pos[slots[s].members[k]] = slot_pos(s, k);
      plan.node_slot[slots[s].members[k]] = s;
    }
  }

  // ---- SEL jobs: rank blocks that hold a kept multi-predictor node
  std::vector<uint32_t> blocks;
  for (uint32_t v : kept)
    if (g.rank[v] >= 0) blocks.push_back(uint32_t(g.rank[v]) >> 2);
  std::sort(blocks.begin(), blocks.end());
  blocks.erase(std::unique(blocks.begin(), blocks.end()), blocks.end());
  const uint32_t njobs = 1 + uint32_t(blocks.size());
  auto draw_off = [&](uint32_t v) {
    const uint32_t r = uint32_t(g.rank[v]);
    const uint32_t bi = uint32_t(std::lower_bound(blocks.begin(), blocks.end(), r >> 2) - blocks.begin());
    return (1 + bi) * 16 + (r & 3) * 4;
  };

  // ---- alias sampling (Algorithms 1, 2 and 5's per-group draws): selecting
  // slots numbered by their smallest member id; their draw words follow the
  // leaf word, an unused word and the 2 g pattern words
  const bool alias_mode = o.sampling == 1;
  const uint32_t nk = uint32_t(kept.size());
  const uint32_t ag = (nk + 15) / 16, ak = (nk + ag - 1) / ag, akp = nk - ak * (ag - 1);
  std::vector<uint32_t> sel_index(ns, PBN_NONE), sel_L(ns, 0);
  uint32_t n_sel = 0;
  size_t alias_bytes = 0;
  if (alias_mode) {
    std::vector<std::pair<uint32_t, uint32_t>> order;   // (smallest member id, slot)
    for (uint32_t s = 0; s < ns; ++s) {
      uint64_t L = 1;
      bool multi = false;
      for (uint32_t v : slots[s].members)
        if (g.nfn(v) > 1) multi = true, L *= g.nfn(v);
      if (!multi) continue;
      if (L > (1u << 20)) return fail(PBN_ELIMIT, "slot %u draws among %llu combined functions", s, (unsigned long long)L);
      sel_L[s] = uint32_t(L);
      order.emplace_back(*std::min_element(slots[s].members.begin(), slots[s].members.end()), s);
      alias_bytes += align16(16 + 8 * size_t(L));
    }
    std::sort(order.begin(), order.end());
    for (const auto& it : order) sel_index[it.second] = n_sel++;
  }

  // ---- image layout
  // FN records: 16 bytes when every FN slot reads at most 5 parents (one
  // 16-byte unit: 5 positions and a 32-entry table), else 32 bytes (two units:
  // 7 positions, then a 128-entry table).  An image that goes to LDS puts the
  // units in 128-byte rows (one row spans all LDS banks): slot s always uses
  // the unit at 16 (s mod 8) of its rows, so the 8 lanes a 16-byte read serves
  // at once never share a bank; a group of 8 slots takes units x (largest l
  // among its FN slots) rows, predictor j of slot s sits 128 units j bytes
  // after predictor 0, a record's second unit 128 bytes after its first.  An
  // image read from global memory packs records densely instead (fewer cache
  // lines): predictor j at 16 units j, second unit at +16; there a plan of
  // two-unit records gives two units only to the slots whose predictors read
  // more than 5 parents (fn_var), the others keep one (a slot record's parent
  // count tells the kernel which).
  const size_t slot_bytes = size_t(npass) * PBN_WAVE * 16;
  size_t nchoice = 0, tab_bytes = 0;
  uint32_t fn_phi = 0;
  // a table slot without multi-predictor members and with at most 5 union
  // bits carries its union positions in its slot record: no union list
  auto inline_table = [&](const Slot& s) {
    if (s.uni.size() > 5) return false;
    for (uint32_t v : s.members)
      if (g.nfn(v) > 1) return false;
    return true;
  };
  for (const auto& s : slots) {
    for (uint32_t v : s.members)
      if (g.nfn(v) > 1) ++nchoice;
    if (s.table) {
      tab_bytes += align16((inline_table(s) ? 0 : 32) + size_t(table_entries(s.members)));
    } else {
      fn_phi = std::max(fn_phi, max_phi(s.members[0]));
    }
  }
  ++nchoice;  // the default choice record of one-predictor FN slots and padded lanes
  const uint32_t units = fn_phi <= 5 ? 1u : 2u;
  const uint32_t ngroups = npass * PBN_WAVE / 8;
  std::vector<uint32_t> row0(ngroups, 0);
  uint32_t rows = units;   // the dummy records (all 8 units) come first
  for (uint32_t gi = 0; gi < ngroups; ++gi) {
    uint32_t lmax = 0;
    for (uint32_t s = 8 * gi; s < std::min(ns, 8 * gi + 8); ++s)
      if (!slots[s].table) lmax = std::max(lmax, g.nfn(slots[s].members[0]));
    row0[gi] = rows;
    rows += units * lmax;
  }
  const size_t choice_base = slot_bytes;
  const size_t fn_base = (choice_base + 16 * nchoice + 127) & ~size_t(127);
  // the perturbation chain's tables follow: Q[0..n] and orig -> position
  const size_t chain_bytes = 16 + 8 * size_t(n + 1) + 16 + 4 * size_t(n);
  const size_t swz_bytes = fn_base + 128 * size_t(rows) + tab_bytes + alias_bytes + chain_bytes;
  const bool swz = swz_bytes <= o.lds_budget_bytes;
  const bool fn_var = !swz && units == 2;
  auto slot_units = [&](size_t s) -> uint32_t { return fn_var ? (max_phi(slots[s].members[0]) > 5 ? 2u : 1u) : units; };
  size_t packed_fn = 16 * size_t(units);   // the dummy record, then every FN slot's records
  for (size_t s = 0; s < ns; ++s)
    if (!slots[s].table) packed_fn += 16 * size_t(slot_units(s)) * g.nfn(slots[s].members[0]);
  const size_t tab_base = fn_base + (swz ? 128 * size_t(rows) : packed_fn);
  const size_t alias_base = tab_base + tab_bytes;
  const size_t q_img = align16(alias_base + alias_bytes);
  const size_t o2p_img = align16(q_img + 8 * size_t(n + 1));
  const size_t image_bytes = align16(o2p_img + 4 * size_t(n));
  if (image_bytes > 0xFFFFFFF0ull) return fail(PBN_ELDS, "plan image too large");
  const uint32_t jstride = swz ? 128 * units : 16 * units, hoff = swz ? 128 : 16;
  std::vector<size_t> rec0(ns, 0);   // dense layout: record of predictor 0
  for (size_t s = 0, cur = fn_base + 16 * units; s < ns; ++s)
    if (!slots[s].table) {
      rec0[s] = cur;
      cur += 16 * size_t(slot_units(s)) * g.nfn(slots[s].members[0]);
    }
  auto fn_rec = [&](uint32_t s, uint32_t j) {
    return swz ? fn_base + 128 * size_t(row0[s / 8] + j * units) + 16 * (s % 8) : rec0[s] + 16 * size_t(slot_units(s)) * j;
  };
  auto dummy_of = [&](size_t s) { return swz ? fn_base + 16 * (s % 8) : fn_base; };

  std::vector<uint8_t> img(image_bytes, 0);
  auto put32 = [&](size_t off, uint32_t v) { std::memcpy(&img[off], &v, 4); };
  auto put16 = [&](size_t off, uint16_t v) { std::memcpy(&img[off], &v, 2); };
  // dummy FN records first (one per unit position of a row): every parent is
  // the zero position, truth table 0
  const size_t dummy_fn = fn_base;
  for (uint32_t q = 0; q < (swz ? 8u : 1u); ++q)
    for (uint32_t b = 0; b < (units == 1 || fn_var ? 6u : 8u); ++b) put16(dummy_fn + 16 * q + 2 * b, uint16_t(zero_pos));
  // default choice record first: ring offset 0, l = 1, no thresholds (selects predictor 0)
  const size_t default_choice = choice_base;
  put32(default_choice, 1u << 24);
  for (int m = 0; m < 3; ++m) put32(default_choice + 4 + 4 * m, 0xFFFFFFFFu);
  for (size_t s = ns; s < size_t(npass) * PBN_WAVE; ++s) {
    put32(s * 16 + 4, uint32_t(dummy_of(s)));
    put32(s * 16 + 8, uint32_t(default_choice));
    put32(s * 16 + 12, uint32_t(bits ? slot_pos(uint32_t(s), 0) : pad_pos0 + (s - ns)));
  }
  size_t choice_cur = choice_base + 16, tab_cur = tab_base;
  std::vector<pbn_pass_info> passes(npass, pbn_pass_info{0, 0, 0, 0});
  uint32_t max_fn_parents = 0, max_union = 0, multi_groups = 0;
  // LDS words read so far by each gather instruction (union bit k) of each
  // pass, per bank (32 banks of 4 bytes): a table slot's union bits are
  // ordered so that its lanes' parent bytes fall on banks the pass's other
  // lanes leave free, gather by gather (lanes reading one word share it)
  constexpr uint32_t kBanks = 32;
  std::vector<std::vector<std::vector<uint32_t>>> bank_words(
      size_t(npass) * PBN_MAX_GROUP_PARENTS, std::vector<std::vector<uint32_t>>(kBanks));
  auto bank_cost = [&](const std::vector<std::vector<uint32_t>>& bw, uint32_t word) -> size_t {
    const auto& b = bw[word % kBanks];
    return std::find(b.begin(), b.end(), word) != b.end() ? 0 : b.size();
  };
  for (uint32_t s = 0; s < ns; ++s) {
    const Slot& sl = slots[s];
    const size_t rec = size_t(s) * 16;
    pbn_pass_info& pi = passes[s / PBN_WAVE];
    uint32_t nmulti = 0;
    const size_t first_choice = choice_cur;
    for (uint32_t v : sl.members) {
      if (g.nfn(v) < 2) continue;
      ++nmulti;
      // the record's l counts the predictors a 32-bit word can reach: those
      // after a threshold of 2^32 (probability 0) are left out, so the
      // kernel's clamp to l - 1 and its never-reached thresholds exclude them
      uint32_t reach = 1;
      while (reach < g.nfn(v) && g.cum[3 * size_t(v) + reach - 1] < kCumNever) ++reach;
      put32(choice_cur + 0, draw_off(v) | (reach << 24));
      for (int m = 0; m < 3; ++m) {
        const uint64_t c = g.cum[3 * size_t(v) + m];
        put32(choice_cur + 4 + 4 * m, c < kCumNever ? uint32_t(c) : 0xFFFFFFFFu);
      }
      choice_cur += 16;
    }
    if (nmulti >= 2) ++multi_groups;
    uint32_t info = PBN_SLOT_VALID | uint32_t(sl.members.size() - 1) | (nmulti << 3);
    uint32_t y = 0, w = 0;
    uint32_t z = nmulti ? uint32_t(first_choice) : sl.table ? 0u : uint32_t(default_choice);
    if (!sl.table) {
      const uint32_t v = sl.members[0];
      const uint32_t pm = max_phi(v);
      info |= pm << 6;
      y = uint32_t(fn_rec(s, 0));
      w = slot_pos(s, 0);   // the slot's state position
      for (uint32_t f = g.fn_off[v]; f < g.fn_off[v + 1]; ++f) {
        const size_t r = fn_rec(s, f - g.fn_off[v]);
        const uint32_t k = g.nparents(f);
        const uint32_t su = slot_units(s);
        const uint32_t npos = su == 1 ? 6u : 8u;   // position slots (unused: the zero position)
        for (uint32_t b = 0; b < npos; ++b)
          put16(r + 2 * b, uint16_t(b < k ? plan.node_pos[g.parents[g.par_off[f] + b]] : zero_pos));
        const size_t tt = su == 1 ? r + 12 : r + hoff;   // truth table: bit x = f(x)
        const uint32_t ebits = 1u << k;
        for (uint32_t x = 0; x < ebits && x < 128; ++x)
          if (g.eval(f, x)) img[tt + (x >> 3)] |= uint8_t(1u << (x & 7));
      }
      pi.flags |= PBN_PASS_FN;
      pi.pmax = std::max(pi.pmax, pm);
      max_fn_parents = std::max(max_fn_parents, pm);
    } else {
      const uint32_t nu = uint32_t(sl.uni.size());
      info |= PBN_SLOT_TABLE | (nu << 6);
      const bool inl = inline_table(sl);
      const size_t list_bytes = inl ? 0 : 32;   // union list before the table (none for inline slots)
      y = uint32_t(tab_cur);
      // table index bit b reads union parent sl.uni[ord[b]] (inv: the reverse)
      std::vector<uint32_t> ord(nu), inv(nu);
      for (uint32_t b = 0; b < nu; ++b) ord[b] = b;
      if (!bits) {
        std::vector<bool> taken(nu, false);
        for (uint32_t b = 0; b < nu; ++b) {
          auto& bw = bank_words[size_t(s / PBN_WAVE) * PBN_MAX_GROUP_PARENTS + b];
          uint32_t best = nu;
          size_t best_cost = 0;
          for (uint32_t i = 0; i < nu; ++i) {
            if (taken[i]) continue;
            const size_t c = bank_cost(bw, plan.node_pos[sl.uni[i]] / 4);
            if (best == nu || c < best_cost) best = i, best_cost = c;
          }
          taken[best] = true;
          ord[b] = best;
          const uint32_t word = plan.node_pos[sl.uni[best]] / 4;
          auto& bank = bw[word % kBanks];
          if (std::find(bank.begin(), bank.end(), word) == bank.end()) bank.push_back(word);
        }
      }
      for (uint32_t b = 0; b < nu; ++b) inv[ord[b]] = b;
      auto upos = [&](uint32_t b) { return b < nu ? plan.node_pos[sl.uni[ord[b]]] : zero_pos; };
      if (!inl)
        for (uint32_t b = 0; b < 16; ++b) put16(tab_cur + 2 * b, uint16_t(upos(b)));
      // mixed radix: member k's digit weight = product of l over later members
      std::vector<uint32_t> radix(sl.members.size(), 1);
      for (int k = int(sl.members.size()) - 2; k >= 0; --k) radix[k] = radix[k + 1] * g.nfn(sl.members[k + 1]);
      uint32_t mi = 0;
      for (uint32_t k = 0; k < sl.members.size(); ++k)
        if (g.nfn(sl.members[k]) > 1) w |= (radix[k] & 0xFFu) << (8 * mi++);
      // combined table by direct evaluation of every member predictor
      uint32_t ncomb = 1;
      for (uint32_t v : sl.members) ncomb *= g.nfn(v);
      std::vector<std::vector<uint32_t>> map;   // per member predictor: parent -> union bit
      const size_t tbl = tab_cur + list_bytes;
      std::vector<uint32_t> digits(sl.members.size());
      for (uint32_t c = 0; c < ncomb; ++c) {
        uint32_t rest = c;
        for (int k = int(sl.members.size()) - 1; k >= 0; --k) {
          digits[k] = rest % g.nfn(sl.members[k]);
          rest /= g.nfn(sl.members[k]);
        }
        for (uint32_t x = 0; x < (1u << nu); ++x) {
          uint32_t out = 0;
          for (uint32_t k = 0; k < sl.members.size(); ++k) {
            const uint32_t f = g.fn_off[sl.members[k]] + digits[k];
            uint32_t idx = 0;
            for (uint32_t b = 0; b < g.nparents(f); ++b) {
              const uint32_t par = g.parents[g.par_off[f] + b];
              const uint32_t ub = uint32_t(std::lower_bound(sl.uni.begin(), sl.uni.end(), par) - sl.uni.begin());
              idx |= ((x >> inv[ub]) & 1u) << b;
            }
            out |= g.eval(f, idx) << k;
          }
          img[tbl + (size_t(c) << nu) + x] = uint8_t(out);
        }
      }
      if (inl) {
        // the union positions in the record itself (no union-list read)
        info |= PBN_SLOT_INLINE | (upos(4) << 11);
        z = upos(0) | (upos(1) << 16);
        w = upos(2) | (upos(3) << 16);
      }
      tab_cur += align16(list_bytes + (size_t(ncomb) << nu));
      pi.flags |= PBN_PASS_TABLE;
      pi.umax = std::max(pi.umax, nu);
      pi.mmax = std::max(pi.mmax, nmulti);
      max_union = std::max(max_union, nu);
    }
    if (nmulti) pi.flags |= PBN_PASS_MULTI;
    put32(rec + 0, info);
    put32(rec + 4, y);
    put32(rec + 8, z);
    put32(rec + 12, w);
  }
  if (alias_mode) {
    // alias records {draw byte offset, L, s, 0} + L x {threshold, alias}; the
    // outcome is the combined index over the multi-predictor members, first
    // member most significant (single-predictor members only have digit 0)
    size_t cur = alias_base;
    for (uint32_t s = 0; s < ns; ++s) {
      if (sel_index[s] == PBN_NONE) continue;
      const uint32_t L = sel_L[s];
      std::vector<uint32_t> mem;
      for (uint32_t v : slots[s].members)
        if (g.nfn(v) > 1) mem.push_back(v);
      std::vector<double> probs(L);
      std::vector<uint32_t> digits(mem.size());
      for (uint32_t c = 0; c < L; ++c) {
        uint32_t rest = c;
        for (int k = int(mem.size()) - 1; k >= 0; --k) {
          digits[k] = rest % g.nfn(mem[k]);
          rest /= g.nfn(mem[k]);
        }
        double q = 1.0;
        for (size_t k = 0; k < mem.size(); ++k) q = q * g.sel[g.fn_off[mem[k]] + digits[k]];
        probs[c] = q;
      }
      std::vector<uint32_t> thr, al;
      vose_table(probs, thr, al);
      put32(cur + 0, 4u * (2u + 2u * ag + sel_index[s]));
      put32(cur + 4, L);
      put32(cur + 8, sel_index[s]);
      for (uint32_t c = 0; c < L; ++c) {
        put32(cur + 16 + 8 * size_t(c), thr[c]);
        put32(cur + 20 + 8 * size_t(c), al[c]);
      }
      put32(size_t(s) * 16 + 8, uint32_t(cur));
      cur += align16(16 + 8 * size_t(L));
    }
  }

  // ---- blob
  const size_t hdr = align16(sizeof(pbn_plan_header));
  const size_t pass_off = hdr;
  const size_t q_off = align16(pass_off + sizeof(pbn_pass_info) * npass);
  const size_t o2p_off = align16(q_off + 8 * size_t(n + 1));
  const size_t p2o_off = align16(o2p_off + 4 * size_t(n));
  const size_t blk_off = align16(p2o_off + 4 * size_t(32 * state_words));
  const size_t pert_off = align16(blk_off + 4 * blocks.size() + 4);
  const size_t pert_bytes = alias_mode ? 8 * (size_t(1) << ak) : 0;
  const size_t kpos_off = align16(pert_off + pert_bytes);
  const size_t image_off = align16(kpos_off + (alias_mode ? 4 * size_t(nk) : 0));
  const size_t total = align16(image_off + image_bytes);
  if (total > 0xFFFFFFF0ull) return fail(PBN_ELDS, "plan blob too large");
  plan.blob.assign(total, 0);
  pbn_plan_header h{};
  h.magic = PBN_PLAN_MAGIC;
  h.version = 1;
  h.blob_bytes = uint32_t(total);
  h.plan_id = plan.plan_id = g_plan_counter.fetch_add(1);
  h.n = n;
  h.n_kept = uint32_t(kept.size());
  h.n_slots = ns;
  h.n_passes = npass;
  h.state_dwords = 8 * state_words;
  h.state_words = state_words;
  h.n_table = ntab;
  h.fn_base = fn_pos0;
  h.n_jobs = njobs;
  h.fill_steps = fill_steps_for(njobs, npass);
  h.image_bytes = uint32_t(image_bytes);
  h.image_off = uint32_t(image_off);
  h.q_off = uint32_t(q_off);
  h.o2p_off = uint32_t(o2p_off);
  h.p2o_off = uint32_t(p2o_off);
  h.blk_off = uint32_t(blk_off);
  h.pass_off = uint32_t(pass_off);
  h.zero_pos = zero_pos;
  h.max_pmax = max_fn_parents;
  h.image_in_lds = image_bytes <= o.lds_budget_bytes ? 1u : 0u;
  h.has_table = max_union > 0 || std::any_of(slots.begin(), slots.end(), [](const Slot& s) { return s.table; });
  h.dummy_fn = uint32_t(dummy_fn);
  h.fn_units = units;
  h.fn_var = fn_var ? 1u : 0u;
  h.state_bits = bits ? 1u : 0u;
  h.fn_jshift = uint32_t(__builtin_ctz(jstride));
  h.fn_hoff = hoff;
  h.q_img = uint32_t(q_img);
  h.o2p_img = uint32_t(o2p_img);
  if (alias_mode) {
    const uint32_t nw = 2 + 2 * ag + n_sel;
    h.sampling = 1;
    h.n_jobs = (nw + 3) / 4;
    h.fill_steps = fill_steps_for(h.n_jobs, npass);
    h.pert_off = uint32_t(pert_off);
    h.kpos_off = uint32_t(kpos_off);
    h.alias_k = ak;
    h.alias_g = ag;
    h.alias_kp = akp;
    h.n_sel = n_sel;
    // Algorithm 1: t = (1 - p)^l for the l removed nodes, a left-to-right
    // product; a leaf is perturbed when the drawn word exceeds ceil(t 2^32) - 1
    const uint32_t nl = n - nk;
    double t = 1.0;
    for (uint32_t i = 0; i < nl; ++i) t = t * (1.0 - g.p);
    const double c = std::ceil(t * 4294967296.0) - 1.0;
    h.leaf_thr = nl == 0 ? 0xFFFFFFFFu : c <= 0.0 ? 0u : c >= 4294967295.0 ? 0xFFFFFFFFu : uint32_t(c);
    // Algorithm 2's table over the 2^k patterns of one group: pattern c has
    // probability prod_b (p if bit b of c is set else 1 - p), left to right
    const uint32_t L = 1u << ak;
    std::vector<double> probs(L);
    const double q = 1.0 - g.p;
    for (uint32_t c2 = 0; c2 < L; ++c2) {
      double v = 1.0;
      for (uint32_t b = 0; b < ak; ++b) v = v * (((c2 >> b) & 1u) ? g.p : q);
      probs[c2] = v;
    }
    std::vector<uint32_t> thr, al;
    vose_table(probs, thr, al);
    for (uint32_t c2 = 0; c2 < L; ++c2) {
      std::memcpy(&plan.blob[pert_off + 8 * size_t(c2)], &thr[c2], 4);
      std::memcpy(&plan.blob[pert_off + 8 * size_t(c2) + 4], &al[c2], 4);
    }
    for (uint32_t i = 0; i < nk; ++i) std::memcpy(&plan.blob[kpos_off + 4 * size_t(i)], &plan.node_pos[kept[i]], 4);
  }
  std::memcpy(&plan.blob[0], &h, sizeof h);
  std::memcpy(&plan.blob[pass_off], passes.data(), sizeof(pbn_pass_info) * npass);
  std::memcpy(&plan.blob[q_off], g.Q.data(), 8 * size_t(n + 1));
  std::memcpy(&plan.blob[o2p_off], plan.node_pos.data(), 4 * size_t(n));
  std::vector<uint32_t> p2o(32 * size_t(state_words), PBN_NONE);
  for (uint32_t v = 0; v < n; ++v)
    if (plan.node_pos[v] != PBN_NONE) p2o[plan.node_pos[v]] = v;
  std::memcpy(&plan.blob[p2o_off], p2o.data(), 4 * p2o.size());
  if (!blocks.empty()) std::memcpy(&plan.blob[blk_off], blocks.data(), 4 * blocks.size());
  std::memcpy(&img[q_img], g.Q.data(), 8 * size_t(n + 1));
  std::memcpy(&img[o2p_img], plan.node_pos.data(), 4 * size_t(n));
  std::memcpy(&plan.blob[image_off], img.data(), image_bytes);

  plan.state_dwords = h.state_dwords;
  plan.fill_steps = h.fill_steps;
  plan.n_jobs = h.n_jobs;
  plan.sampling = h.sampling;
  plan.has_table = h.has_table;
  pbn_plan_info& in = plan.info;
  std::memset(&in, 0, sizeof in);
  in.n = n;
  in.n_kept = h.n_kept;
  in.n_slots = ns;
  in.n_table_slots = uint32_t(std::count_if(slots.begin(), slots.end(), [](const Slot& s) { return s.table; }));
  in.n_passes = npass;
  in.state_words = h.state_words;
  in.state_bytes = 32 * state_words;
  in.n_jobs = h.n_jobs;
  in.image_bytes = uint32_t(image_bytes);
  in.table_bytes = uint32_t(tab_bytes);
  in.image_in_lds = h.image_in_lds;
  in.blob_bytes = uint32_t(total);
  in.max_fn_parents = max_fn_parents;
  in.max_union_bits = max_union;
  in.n_multi_groups = multi_groups;
  return PBN_OK;
}

extern "C" pbn_status pbn_plan_build(const pbn_net* g, const uint32_t* interest, uint32_t n_interest,
                                     const pbn_plan_opts* opts, pbn_plan** out) {
  pbn::clear_error();
  if (!g || !out || (n_interest && !interest)) return fail(PBN_EINVAL, "null argument");
  *out = nullptr;
  pbn_plan_opts o;
  if (opts)
    o = *opts;
  else
    pbn_plan_opts_default(&o);
  if (o.reduce > 2) return fail(PBN_EINVAL, "reduce must be 0, 1 or 2");
  if (o.sampling > 1) return fail(PBN_EINVAL, "sampling must be 0 (keyed) or 1 (alias)");
  if (o.state_bits > 1) return fail(PBN_EINVAL, "state_bits must be 0 or 1");
  if (o.state_bits && o.sampling) return fail(PBN_EINVAL, "the packed-bit state layout takes keyed draws only");
  if (o.max_group_nodes < 1 || o.max_group_nodes > PBN_MAX_GROUP_NODES)
    return fail(PBN_EINVAL, "max_group_nodes must be 1..%d", PBN_MAX_GROUP_NODES);
  if (o.max_parent_bits > PBN_MAX_GROUP_PARENTS)
    return fail(PBN_EINVAL, "max_parent_bits must be <= %d", PBN_MAX_GROUP_PARENTS);
  if (o.theta == 0 || o.weight_mode > 1) return fail(PBN_EINVAL, "bad theta or weight_mode");
  std::vector<uint8_t> is_int(g->n, 0);
  for (uint32_t k = 0; k < n_interest; ++k) {
    if (interest[k] >= g->n) return fail(PBN_EINVAL, "interest node %u out of range", interest[k]);
    is_int[interest[k]] = 1;
  }
  try {
    auto* plan = new pbn_plan;
    const pbn_status st = build_plan(*g, is_int, o, *plan);
    if (st != PBN_OK) {
      delete plan;
      return st;
    }
    *out = plan;
    return PBN_OK;
  } catch (const std::bad_alloc&) {
    return fail(PBN_ENOMEM, "out of host memory");
  }
}

extern "C" pbn_status pbn_plan_destroy(pbn_plan* plan) {
  delete plan;
  return PBN_OK;
}

extern "C" pbn_status pbn_plan_info_get(const pbn_plan* plan, pbn_plan_info* info) {
  pbn::clear_error();
  if (!plan || !info) return fail(PBN_EINVAL, "null argument");
  *info = plan->info;
  return PBN_OK;
}

extern "C" pbn_status pbn_plan_node_pos(const pbn_plan* plan, uint32_t* pos) {
  pbn::clear_error();
  if (!plan || !pos) return fail(PBN_EINVAL, "null argument");
  std::copy(plan->node_pos.begin(), plan->node_pos.end(), pos);
  return PBN_OK;
}

extern "C" pbn_status pbn_plan_slots(const pbn_plan* plan, uint32_t* slot, uint32_t* is_table) {
  pbn::clear_error();
  if (!plan) return fail(PBN_EINVAL, "null argument");
  if (slot) std::copy(plan->node_slot.begin(), plan->node_slot.end(), slot);
  if (is_table) std::copy(plan->slot_is_table.begin(), plan->slot_is_table.end(), is_table);
  return PBN_OK;
}

static pbn_status export_groups(const std::vector<std::vector<uint32_t>>& groups, uint32_t* members,
                                uint32_t* n_members, uint32_t* offsets, uint32_t* n_groups) {
  uint32_t total = 0;
  for (const auto& gr : groups) total += uint32_t(gr.size());
  if (n_members) *n_members = total;
  if (n_groups) *n_groups = uint32_t(groups.size());
  if (members || offsets) {
    uint32_t k = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      if (offsets) offsets[gi] = k;
      for (uint32_t v : groups[gi]) {
        if (members) members[k] = v;
        ++k;
      }
    }
    if (offsets) offsets[groups.size()] = k;
  }
  return PBN_OK;
}

extern "C" pbn_status pbn_plan_alg4_groups(const pbn_plan* plan, uint32_t* members, uint32_t* n_members,
                                           uint32_t* offsets, uint32_t* n_groups) {
  pbn::clear_error();
  if (!plan) return fail(PBN_EINVAL, "null argument");
  return export_groups(plan->alg4_groups, members, n_members, offsets, n_groups);
}

extern "C" pbn_status pbn_plan_single_groups(const pbn_plan* plan, uint32_t* members, uint32_t* n_members,
                                             uint32_t* offsets, uint32_t* n_groups) {
  pbn::clear_error();
  if (!plan) return fail(PBN_EINVAL, "null argument");
  return export_groups(plan->single_groups, members, n_members, offsets, n_groups);
}

extern "C" pbn_status pbn_plan_export(const pbn_plan* plan, void* host_buf, size_t* bytes) {
  pbn::clear_error();
  if (!plan || !bytes) return fail(PBN_EINVAL, "null argument");
  if (!host_buf) {
    *bytes = plan->blob.size();
    return PBN_OK;
  }
  if (*bytes < plan->blob.size()) return fail(PBN_EINVAL, "buffer too small (%zu < %zu)", *bytes, plan->blob.size());
  std::memcpy(host_buf, plan->blob.data(), plan->blob.size());
  *bytes = plan->blob.size();
  return PBN_OK;
}

extern "C" pbn_status pbn_targets_build(const pbn_plan* plan, const uint32_t* node, const uint32_t* value,
                                        const uint32_t* target_of, uint32_t npairs, uint32_t ntargets,
                                        pbn_targets* out) {
  pbn::clear_error();
  if (!plan || !out || (npairs && (!node || !value || !target_of))) return fail(PBN_EINVAL, "null argument");
  if (ntargets == 0 || ntargets > 64) return fail(PBN_EINVAL, "ntargets must be 1..64");
  if (npairs > PBN_MAX_PAIRS) return fail(PBN_EINVAL, "npairs must be <= %d", PBN_MAX_PAIRS);
  std::memset(out, 0, sizeof *out);
  out->ntargets = ntargets;
  out->npairs = npairs;
  for (uint32_t k = 0; k < npairs; ++k) {
    if (node[k] >= plan->node_pos.size()) return fail(PBN_EINVAL, "pair %u: node out of range", k);
    if (plan->node_pos[node[k]] == PBN_NONE)
      return fail(PBN_EINVAL, "pair %u: node %u was removed as a leaf (list it as of interest)", k, node[k]);
    if (value[k] > 1) return fail(PBN_EINVAL, "pair %u: value must be 0 or 1", k);
    if (target_of[k] >= ntargets) return fail(PBN_EINVAL, "pair %u: target index out of range", k);
    out->pos[k] = plan->node_pos[node[k]];
    out->val[k] = value[k];
    out->mask[target_of[k]] |= 1ull << k;
  }
  for (uint32_t t = 0; t < ntargets; ++t)
    if (!out->mask[t]) return fail(PBN_EINVAL, "target %u has no pair", t);
  return PBN_OK;
}
