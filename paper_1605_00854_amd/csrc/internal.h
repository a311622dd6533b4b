// internal.h -- host-side objects behind the C ABI.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pbn.h"
#include "plan_format.h"

constexpr uint64_t kCumNever = 1ull << 32;   // a selection threshold no 32-bit uniform reaches

struct pbn_net {
  uint32_t n = 0;
  double p = 0.0;
  std::vector<uint32_t> fn_off, par_off, parents, tt_off;
  std::vector<double> sel;
  std::vector<uint64_t> tt;
  // random-number contract tables (quantised once at creation)
  std::vector<uint64_t> Q;      // Q[0..n], Q[0] unused (0)
  std::vector<uint64_t> cum;    // 3 per node, at most 2^32 (never reached); unused 2^32
  std::vector<int32_t> rank;    // rank among multi-predictor nodes, -1 otherwise
  uint32_t n_multi = 0;

  uint32_t nfn(uint32_t i) const { return fn_off[i + 1] - fn_off[i]; }
  uint32_t nparents(uint32_t f) const { return par_off[f + 1] - par_off[f]; }
  // output of predictor f for truth-table index x
  uint32_t eval(uint32_t f, uint32_t x) const {
    return uint32_t((tt[tt_off[f] + (x >> 6)] >> (x & 63)) & 1u);
  }
};

struct pbn_plan {
  pbn_plan_info info{};
  std::vector<uint8_t> blob;
  std::vector<uint32_t> node_pos;     // bit position per original node, or PBN_NONE
  std::vector<uint32_t> node_slot;    // slot per original node, or PBN_NONE
  std::vector<uint32_t> slot_is_table;
  std::vector<std::vector<uint32_t>> alg4_groups, single_groups;
  uint32_t plan_id = 0;
  uint32_t state_dwords = 0;
  uint32_t fill_steps = 1;
  uint32_t n_jobs = 1;
  uint32_t has_table = 0;
  uint32_t sampling = 0;     // 1: alias sampling (draw contract of the plan format)
};

namespace pbn {
void set_error(const std::string& msg);
void clear_error();
// Equation 2 lower bound (0 when no m satisfies it).
uint32_t eq2_lower_bound(const std::vector<uint64_t>& w, uint64_t theta);
}  // namespace pbn
