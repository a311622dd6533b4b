// device.hip -- HIP kernels for gfx950 and their C-ABI launchers.
//
// Step kernel (Algorithm 5's ParallelSimulation, Eq. 1 semantics): one
// wavefront advances one trajectory.  Per step:
//   * Philox calls of the step (one PERT call plus one SEL call per rank block
//     holding a kept multi-predictor node) are spread over the 64 lanes; when a
//     step needs <= 32 calls, one fill computes several future steps at once.
//     Results go to a per-wave ring in LDS.
//   * The first PERT word decides, wave-uniformly, whether any of the n
//     original nodes is perturbed (u >= Q[n]).  If so, the skip chain walks
//     the perturbed nodes (ballot counting over Q, radix 64), flips the kept
//     ones in place, and no predictor is applied (Eq. 1, Algorithm 5).  Leaf
//     perturbations only make the step perturbation-only (Algorithm 1's role).
//   * Otherwise each lane evaluates its slot(s): an FN slot selects its
//     predictor from its SEL word and integer thresholds and looks up the
//     predictor's truth table over its parents; a TABLE slot combines the
//     choices of its multi-predictor members into the combined-function index
//     and reads one byte of the group's combined table (Section 3.3).  Results
//     are written to the other state buffer (synchronous update).
//   * Target hits: lanes holding target pairs compare the new state, a ballot
//     collects mismatches, lane t counts hits of target t.
// The state of a trajectory lives in LDS as one byte per node value (a 32-bit
// word per table slot, a byte per FN slot); plan records and tables are staged
// in LDS when they fit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <string>
#include <vector>

#include "internal.h"

namespace {

constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;

// Three-input XOR in one VALU instruction: gfx950's three-input bitwise op
// with truth table 0x96 (a ^ b ^ c), through the compiler's builtin (plain
// a ^ b ^ k compiles to two XORs).  The key operand is wave-uniform.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t k) {
  return __builtin_amdgcn_bitop3_b32(a, b, k, 0x96);
}

// Philox4x32-10 (Salmon et al., SC'11): counter (c0..c3), key (k0, k1).  Each
// round multiplies words 0 and 2 by fixed constants (one full-rate
// v_mad_u64_u32 each gives both halves) and mixes the high halves with words
// 1 and 3 and the round key.
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t p0 = uint64_t(kM0) * c0;
    const uint64_t p1 = uint64_t(kM1) * c2;
    const uint32_t n0 = xor3(uint32_t(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3(uint32_t(p0 >> 32), c3, k1);
    c1 = uint32_t(p1);
    c3 = uint32_t(p0);
    c0 = n0;
    c2 = n2;
  }
  return make_uint4(c0, c1, c2, c3);
}

// Order LDS traffic between lanes of one wavefront.  The LDS executes the
// instructions of one wave in issue order, so a read issued after a write of
// the same wave observes it; only the compiler must be kept from reordering
// (no hardware wait is needed).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_wave_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ uint32_t uniform(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// Reads of a plan image.  G: the image is global memory reached through a
// pointer loaded at run time (a batch's work item), read through a pointer of
// the global address space so that the loads are global, not flat, loads
// (flat loads would also wait on outstanding LDS traffic).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
#define PBN_GLOBAL_AS __attribute__((address_space(1)))
template <bool G>
__device__ __forceinline__ uint4 img_u4(const uint8_t* p) {
  if constexpr (G) {
    const u32x4 v = *(const PBN_GLOBAL_AS u32x4*)(p);
    return make_uint4(v.x, v.y, v.z, v.w);
  } else {
    return *reinterpret_cast<const uint4*>(p);
  }
}
template <bool G>
__device__ __forceinline__ uint32_t img_u32(const uint8_t* p) {
  if constexpr (G)
    return *(const PBN_GLOBAL_AS uint32_t*)(p);
  else
    return *reinterpret_cast<const uint32_t*>(p);
}
template <bool G>
__device__ __forceinline__ unsigned long long blob_u64(const unsigned long long* p) {
  if constexpr (G)
    return *(const PBN_GLOBAL_AS unsigned long long*)(p);
  else
    return *p;
}
template <bool G>
__device__ __forceinline__ uint32_t blob_u32(const uint32_t* p) {
  if constexpr (G)
    return *(const PBN_GLOBAL_AS uint32_t*)(p);
  else
    return *p;
}
template <bool G>
__device__ __forceinline__ uint2 img_u2(const uint8_t* p) {
  if constexpr (G) {
    const u32x2 v = *(const PBN_GLOBAL_AS u32x2*)(p);
    return make_uint2(v.x, v.y);
  } else {
    return *reinterpret_cast<const uint2*>(p);
  }
}
template <bool G>
__device__ __forceinline__ uint32_t img_u8(const uint8_t* p) {
  if constexpr (G)
    return *(const PBN_GLOBAL_AS uint8_t*)(p);
  else
    return *p;
}
__device__ __forceinline__ unsigned long long uniform64(unsigned long long x) {
  return (static_cast<unsigned long long>(uniform(uint32_t(x >> 32))) << 32) | uniform(uint32_t(x));
}
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  return reinterpret_cast<T*>(uniform64(reinterpret_cast<unsigned long long>(p)));
}

// (b ^ want) & care: the compiler forms the three-input bitwise instruction
// itself (b is usually a ballot just written by a vector compare; written out
// here, the compiler also inserts the wait that such a read needs).
__device__ __forceinline__ uint32_t masked_xor(uint32_t b, uint32_t care, uint32_t want) {
  return (b ^ want) & care;
}

// (a << sh) | b: one shift-or instruction.  A gather passes sh = 1 from a
// launch argument: with a constant shift the compiler re-associates the chain
// of shift-ors into a tree of separate shifts and three-input ors (more
// instructions per parent bit); with a run-time amount it keeps the chain.
__device__ __forceinline__ uint32_t shl_or(uint32_t a, uint32_t b, uint32_t sh) { return (a << sh) | b; }

// High word of w + c for a 64-bit c = 2^64 - t: 0 when w >= t, all ones when
// w < t (t <= 2^32).  One 64-bit add (gfx950's shift-add on 64-bit operands).
__device__ __forceinline__ uint32_t borrow_hi(uint32_t w, unsigned long long c) {
  return uint32_t((static_cast<unsigned long long>(w) + c) >> 32);
}

struct SimParams {
  const uint8_t* blob;
  uint32_t* state;
  unsigned long long* counts;
  unsigned long long seed;
  uint32_t traj0, ntraj, step0, nsteps, count_from;
  uint32_t wpb;
  uint32_t wave_bytes;   // LDS bytes per wave: state buffer(s) + ring
  uint32_t record_traj;  // trajectories 0 .. record_traj-1 record target 0's indicator bits
  uint32_t record_words; // words per recording trajectory
  uint32_t gshift;       // 1: the gather step's shift, passed at run time (see shl_or)
  uint32_t* record;      // [record_traj][record_words] or null
  uint32_t tpw;          // trajectories per wavefront (k_simulate_multi)
  uint32_t mfill;        // steps per Philox fill (k_simulate_multi)
  pbn_targets tg;
};

template <int PM, int UM>
struct Shape {
  static constexpr int PW = (PM + 1) / 2;                    // parent-position words of an FN record
  static constexpr int TTW = PM <= 5 ? 1 : 4;                // truth-table words of an FN record
  static constexpr int UW = UM > 0 ? UM / 2 : 1;             // union-position words of a TABLE slot
  static constexpr int XW = PW > UW ? PW : UW;               // position words held per slot
};

// The part of an FN record a lookup needs: parent positions and truth table.
template <int PW, int TTW>
struct FnRec {
  uint32_t pw[PW];
  uint32_t tt[TTW];
};

// Per-lane data of one slot, either cached in registers for the whole launch
// (plans of at most NREG lane passes) or reloaded from the image every pass.
template <int XW, int TTW>
struct SlotRegs {
  uint32_t info;                    // slot-record info word (PBN_SLOT_*)
  uint32_t base;                    // FN: record of predictor 0; TABLE: union-parent list
  uint32_t choice, radix;           // TABLE: first choice record, mixed-radix weights
  uint32_t draw, thr0, thr1, thr2;  // FN: its choice record (ring offset | l << 24, thresholds)
  uint32_t spos;                    // state byte written by the slot
  uint32_t pw[XW];                  // TABLE: union parents; one-predictor FN: its parents
  uint32_t tt[TTW];                 // one-predictor FN: its truth table
};

template <int K>
__device__ __forceinline__ uint32_t gather(const uint8_t* cs, const uint32_t* pw, uint32_t sh) {
  // all K byte reads are independent: issued back to back, one wait; state
  // bytes are 0 or 1, so the index is a chain of shift-or steps
  uint32_t b[K];
#pragma unroll
  for (int k = 0; k < K; ++k) b[k] = cs[(k & 1) ? (pw[k >> 1] >> 16) : (pw[k >> 1] & 0xFFFFu)];
  uint32_t idx = b[K - 1];
#pragma unroll
  for (int k = K - 2; k >= 0; --k) idx = shl_or(idx, b[k], sh);
  return idx;
}

// The same gather from a state held as one 64-bit word (bit b = state byte b):
// the shift takes the position's low 6 bits.
template <int K>
__device__ __forceinline__ uint32_t gather_bits(unsigned long long st, const uint32_t* pw, uint32_t sh) {
  uint32_t b[K];
#pragma unroll
  for (int k = 0; k < K; ++k) b[k] = uint32_t(st >> (((k & 1) ? (pw[k >> 1] >> 16) : pw[k >> 1]) & 63u)) & 1u;
  uint32_t idx = b[K - 1];
#pragma unroll
  for (int k = K - 2; k >= 0; --k) idx = shl_or(idx, b[k], sh);
  return idx;
}

// The same gather from a packed state in LDS (bit b of the state = bit b % 32
// of word b / 32): one word read per parent, the bit taken by a field extract
// whose offset is the position's low 5 bits.
template <int K>
__device__ __forceinline__ uint32_t gather_lbits(const uint32_t* words, const uint32_t* pw, uint32_t sh) {
  uint32_t b[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint32_t p = (k & 1) ? (pw[k >> 1] >> 16) : (pw[k >> 1] & 0xFFFFu);
    b[k] = __builtin_amdgcn_ubfe(words[p >> 5], p & 31u, 1u);
  }
  uint32_t idx = b[K - 1];
#pragma unroll
  for (int k = K - 2; k >= 0; --k) idx = shl_or(idx, b[k], sh);
  return idx;
}

__device__ __forceinline__ uint32_t choose(uint32_t w, uint32_t t0, uint32_t t1, uint32_t t2, uint32_t nfn) {
  const uint32_t j = uint32_t(w >= t0) + uint32_t(w >= t1) + uint32_t(w >= t2);
  return min(j, nfn - 1u);
}

// The same choice from negated thresholds (2^64 - CUM[m] for m < l - 1, and
// 2^64 - 2^32, never reached, for the others): 3 + the three borrows.
struct NegThr {
  unsigned long long c0, c1, c2;
};

__device__ __forceinline__ NegThr neg_thresholds(uint32_t t0, uint32_t t1, uint32_t t2, uint32_t nfn) {
  constexpr unsigned long long kNever = 0xFFFFFFFF00000000ull;
  NegThr n;
  n.c0 = nfn > 1u ? 0ull - t0 : kNever;
  n.c1 = nfn > 2u ? 0ull - t1 : kNever;
  n.c2 = nfn > 3u ? 0ull - t2 : kNever;
  return n;
}

__device__ __forceinline__ uint32_t choose_neg(uint32_t w, const NegThr& n) {
  return 3u + borrow_hi(w, n.c0) + borrow_hi(w, n.c1) + borrow_hi(w, n.c2);
}

// Alias draw (Walker's method, Section 2.2) from one 32-bit word w over a
// table of L columns at `tab` (8-byte entries {threshold, alias}): the column
// is the high word of w * L, kept when the low word is below its threshold.
template <bool G>
__device__ __forceinline__ uint32_t alias_pick(const uint8_t* tab, uint32_t w, uint32_t L) {
  const unsigned long long prod = (unsigned long long)w * L;
  const uint32_t col = uint32_t(prod >> 32);
  const uint2 e = img_u2<G>(tab + 8u * col);
  return uint32_t(prod) < e.x ? col : e.y;
}

// Philox calls per lane in one fill of the ring (the host sizes fills to at
// most this many rounds of 64 calls; PBN_FILL_ROUNDS in the plan format).
constexpr int kFillRounds = PBN_FILL_ROUNDS;

// Layout of a plan's FN records (header fields) and the zero-position pair.
struct FnFmt {
  uint32_t units;     // 16-byte units per record
  uint32_t jshift;    // log2 of the bytes from predictor j's record to j + 1's
  uint32_t hoff;      // bytes from a record's first unit to its second
  uint32_t zp2;       // zero position in both halves of a word
  uint32_t var;       // two-unit plan, packed: a slot reading <= 5 parents keeps one unit
  uint32_t sh;        // 1, the shift of a gather step (a launch argument; see shl_or)
};

// FN record of predictor j of the slot (slot-record word `info`) whose
// predictor 0 is at image offset `base`: one 16-byte unit (5 positions,
// 32-entry table) or two units (7 positions; 128-entry table).  A
// gather-width-7 kernel reads two-unit plans, where a packed image keeps one
// unit for the slots that read at most 5 parents (fm.var: the slot's parent
// count decides, lane by lane); with MIXED (batches of plans of both kinds) it
// also reads one-unit plans.  A one-unit record read by this kernel has
// positions 5-7 = the zero position and table words 1-3 never selected.
// MODE: bit 0 MIXED, bit 1 image reads through global-address-space pointers.
template <int PM, int UM, int MODE>
__device__ __forceinline__ FnRec<Shape<PM, UM>::PW, Shape<PM, UM>::TTW> load_fn(const uint8_t* img, uint32_t base,
                                                                               uint32_t j, const FnFmt& fm,
                                                                               uint32_t info) {
  constexpr int TTW = Shape<PM, UM>::TTW;
  constexpr bool MIXED = (MODE & 1) != 0, G = (MODE & 2) != 0;
  FnRec<Shape<PM, UM>::PW, TTW> r;
  const bool two = fm.var ? PBN_SLOT_NU(info) > 5u : (!MIXED || fm.units == 2u);
  const uint32_t jshift = fm.var ? (two ? 5u : 4u) : fm.jshift;
  // records and units are 16-byte aligned: one 16-byte read per unit
  const uint8_t* rp = static_cast<const uint8_t*>(__builtin_assume_aligned(img + (base + (j << jshift)), 16));
  const uint4 a = img_u4<G>(rp);
  r.pw[0] = a.x;
  r.pw[1] = a.y;
  r.pw[2] = a.z;
  if constexpr (TTW == 1) {
    r.tt[0] = a.w;
  } else {
    if (two) {
      const uint4 b = img_u4<G>(rp + fm.hoff);
      r.pw[3] = a.w;
      r.tt[0] = b.x;
      r.tt[1] = b.y;
      r.tt[2] = b.z;
      r.tt[3] = b.w;
    } else {
      r.pw[3] = fm.zp2;
      r.tt[0] = a.w;
      r.tt[1] = r.tt[2] = r.tt[3] = 0u;
    }
  }
  return r;
}

// Look up an FN record's truth table over its parents in state `cs` (bytes in
// LDS) or, with REG, in the 64-bit state `st`.
template <int PM, int UM, bool REG = false, bool LBITS = false>
__device__ __forceinline__ uint32_t eval_fn(const FnRec<Shape<PM, UM>::PW, Shape<PM, UM>::TTW>& r, const uint8_t* cs,
                                            uint32_t sh, unsigned long long st = 0ull) {
  constexpr int TTW = Shape<PM, UM>::TTW;
  uint32_t idx;
  if constexpr (REG)
    idx = gather_bits<PM>(st, r.pw, sh);
  else if constexpr (LBITS)
    idx = gather_lbits<PM>(reinterpret_cast<const uint32_t*>(cs), r.pw, sh);
  else
    idx = gather<PM>(cs, r.pw, sh);
  uint32_t ttw = r.tt[0];
  if constexpr (TTW > 1) {
    // word idx / 32 of the 128-bit table, selected among scalars (an indexed
    // array here would be placed in scratch memory)
    const uint32_t t1 = r.tt[1], t2 = r.tt[2], t3 = r.tt[3];
    const uint32_t lo = (idx & 32u) ? t1 : ttw, hi = (idx & 32u) ? t3 : t2;
    ttw = (idx & 64u) ? hi : lo;
  }
  return __builtin_amdgcn_ubfe(ttw, idx, 1u);   // bit idx % 32
}

// Slot record of `slot` (lane slot % 64 of pass slot / 64) and what it points
// at: a table slot's union parents, a multi-predictor node's choice record, a
// one-predictor node's own FN record.
template <int PM, int UM, int MODE>
__device__ __forceinline__ void load_slot(SlotRegs<Shape<PM, UM>::XW, Shape<PM, UM>::TTW>& r, const uint8_t* img,
                                          uint32_t slot, const FnFmt& fm) {
  constexpr int XW = Shape<PM, UM>::XW, TTW = Shape<PM, UM>::TTW, PW = Shape<PM, UM>::PW, UW = Shape<PM, UM>::UW;
  constexpr bool G = (MODE & 2) != 0;
  const uint4 rec = img_u4<G>(img + 16u * slot);
  r.info = rec.x;
  r.base = rec.y;
  r.choice = rec.z;
  r.radix = rec.w;
  r.draw = 1u << 24;
  r.thr0 = r.thr1 = r.thr2 = 0xFFFFFFFFu;
#pragma unroll
  for (int k = 0; k < XW; ++k) r.pw[k] = 0;
#pragma unroll
  for (int k = 0; k < TTW; ++k) r.tt[k] = 0;
  if (UM > 0 && (rec.x & PBN_SLOT_TABLE)) {
    r.spos = 4u * slot;
    if (rec.x & PBN_SLOT_INLINE) {
      // union positions carried by the record (no multi-predictor members:
      // choice and radix are not read)
      r.pw[0] = rec.z;
      if constexpr (UW > 1) r.pw[1] = rec.w;
      if constexpr (UW > 2) r.pw[2] = PBN_SLOT_P4(rec.x) | (fm.zp2 & 0xFFFF0000u);
#pragma unroll
      for (int k = 3; k < UW; ++k) r.pw[k] = fm.zp2;
    } else {
#pragma unroll
      for (int k = 0; k < UW; ++k) r.pw[k] = img_u32<G>(img + (rec.y + 4u * k));
    }
  } else {
    r.spos = rec.w;   // FN slot or padded lane: its state byte
    if (PBN_SLOT_NMULTI(rec.x)) {
      const uint4 ch = img_u4<G>(img + rec.z);
      r.draw = ch.x;
      r.thr0 = ch.y;
      r.thr1 = ch.z;
      r.thr2 = ch.w;
    } else {
      // one-predictor node or padded lane (a dummy record)
      const auto f = load_fn<PM, UM, MODE>(img, rec.y, 0u, fm, rec.x);
#pragma unroll
      for (int k = 0; k < PW; ++k) r.pw[k] = f.pw[k];
#pragma unroll
      for (int k = 0; k < TTW; ++k) r.tt[k] = f.tt[k];
    }
  }
}

// TABLE slot: combined-function index from its multi-predictor members'
// choices (mixed radix), union parents, one table byte: member k's output in
// bit k (Section 3.3).
template <int PM, int UM, int MODE>
__device__ __forceinline__ uint32_t eval_table(const SlotRegs<Shape<PM, UM>::XW, Shape<PM, UM>::TTW>& r,
                                               const uint8_t* img, const uint8_t* cs, const uint8_t* rs, uint32_t sh) {
  constexpr bool G = (MODE & 2) != 0, ALIAS = (MODE & 4) != 0;
  uint32_t c = 0;
  const uint32_t nm = PBN_SLOT_NMULTI(r.info);
  if constexpr (ALIAS) {
    // one draw over the group's combined functions: record {word offset, L, ...}
    if (nm) {
      const uint2 hd = img_u2<G>(img + r.choice);
      c = alias_pick<G>(img + r.choice + 16u, *reinterpret_cast<const uint32_t*>(rs + hd.x), hd.y);
    }
  } else for (uint32_t m = 0; m < nm; ++m) {
    const uint4 ch = img_u4<G>(img + (r.choice + 16u * m));
    const uint32_t w = *reinterpret_cast<const uint32_t*>(rs + (ch.x & 0xFFFFFFu));
    c += choose(w, ch.y, ch.z, ch.w, ch.x >> 24) * ((r.radix >> (8u * m)) & 0xFFu);
  }
  uint32_t x;
  if constexpr ((MODE & 16) != 0)
    x = gather_lbits<(UM > 0 ? UM : 1)>(reinterpret_cast<const uint32_t*>(cs), r.pw, sh);
  else
    x = gather<(UM > 0 ? UM : 1)>(cs, r.pw, sh);
  const uint32_t list = (r.info & PBN_SLOT_INLINE) ? 0u : 32u;   // inline slots: the table at base
  const uint32_t v = img_u8<G>(img + (r.base + list + (c << PBN_SLOT_NU(r.info)) + x));
  return v;   // member k's output in bit k
}

// One slot: a table slot, a multi-predictor node (select from its drawn word,
// then read the chosen record) or a one-predictor node (record already held).
// `nt`: the slot's negated thresholds when held for the launch, else null.
template <int PM, int UM, int MODE>
__device__ __forceinline__ uint32_t eval_slot(const SlotRegs<Shape<PM, UM>::XW, Shape<PM, UM>::TTW>& r,
                                              const NegThr* nt, const uint8_t* img, const uint8_t* cs,
                                              const uint8_t* rs, const FnFmt& fm) {
  constexpr int PW = Shape<PM, UM>::PW, TTW = Shape<PM, UM>::TTW;
  if (UM > 0 && (r.info & PBN_SLOT_TABLE)) return eval_table<PM, UM, MODE>(r, img, cs, rs, fm.sh);
  FnRec<PW, TTW> f;
#pragma unroll
  for (int k = 0; k < PW; ++k) f.pw[k] = r.pw[k];
#pragma unroll
  for (int k = 0; k < TTW; ++k) f.tt[k] = r.tt[k];
  if (PBN_SLOT_NMULTI(r.info)) {
    const uint32_t w = *reinterpret_cast<const uint32_t*>(rs + (r.draw & 0xFFFFFFu));
    uint32_t j;
    if constexpr ((MODE & 4) != 0)
      j = alias_pick<(MODE & 2) != 0>(img + r.choice + 16u, w, r.thr0);   // alias record: {offset, L, ...}
    else
      j = nt ? choose_neg(w, *nt) : choose(w, r.thr0, r.thr1, r.thr2, r.draw >> 24);
    f = load_fn<PM, UM, MODE>(img, r.base, j, fm, r.info);
  }
  return eval_fn<PM, UM, false, (MODE & 16) != 0>(f, cs, fm.sh);
}

// One slot of a plan whose slot data are read from the image every pass:
// the slot record, then only what the slot's kind needs (a table slot's union
// positions and choice records, a multi-predictor node's choice record and
// chosen predictor record, a one-predictor node's record); returns the
// slot's output (member k in bit k) and the state position it writes.
template <int PM, int UM, int MODE>
__device__ __forceinline__ uint32_t eval_stream(const uint4 rec, const uint8_t* img, uint32_t slot, const uint8_t* cs,
                                                const uint8_t* rs, const FnFmt& fm, uint32_t& spos, bool& table) {
  constexpr int PW = Shape<PM, UM>::PW, TTW = Shape<PM, UM>::TTW, UW = Shape<PM, UM>::UW;
  constexpr bool G = (MODE & 2) != 0, LB = (MODE & 16) != 0;
  table = UM > 0 && (rec.x & PBN_SLOT_TABLE);
  if (UM > 0 && (rec.x & PBN_SLOT_TABLE)) {
    spos = 4u * slot;
    uint32_t pw[UW];
    uint32_t c = 0;
    if (rec.x & PBN_SLOT_INLINE) {
      pw[0] = rec.z;
      if constexpr (UW > 1) pw[1] = rec.w;
      if constexpr (UW > 2) pw[2] = PBN_SLOT_P4(rec.x) | (fm.zp2 & 0xFFFF0000u);
#pragma unroll
      for (int k = 3; k < UW; ++k) pw[k] = fm.zp2;
    } else {
#pragma unroll
      for (int k = 0; k < UW; ++k) pw[k] = img_u32<G>(img + (rec.y + 4u * k));
      const uint32_t nm = PBN_SLOT_NMULTI(rec.x);
      for (uint32_t m = 0; m < nm; ++m) {
        const uint4 ch = img_u4<G>(img + (rec.z + 16u * m));
        const uint32_t w = *reinterpret_cast<const uint32_t*>(rs + (ch.x & 0xFFFFFFu));
        c += choose(w, ch.y, ch.z, ch.w, ch.x >> 24) * ((rec.w >> (8u * m)) & 0xFFu);
      }
    }
    uint32_t x;
    if constexpr (LB)
      x = gather_lbits<(UM > 0 ? UM : 1)>(reinterpret_cast<const uint32_t*>(cs), pw, fm.sh);
    else
      x = gather<(UM > 0 ? UM : 1)>(cs, pw, fm.sh);
    const uint32_t list = (rec.x & PBN_SLOT_INLINE) ? 0u : 32u;   // inline slots: the table at y
    return img_u8<G>(img + (rec.y + list + (c << PBN_SLOT_NU(rec.x)) + x));
  }
  spos = rec.w;   // FN slot or padded lane: its state position
  uint32_t j = 0;
  if (PBN_SLOT_NMULTI(rec.x)) {
    const uint4 ch = img_u4<G>(img + rec.z);
    const uint32_t w = *reinterpret_cast<const uint32_t*>(rs + (ch.x & 0xFFFFFFu));
    j = choose(w, ch.y, ch.z, ch.w, ch.x >> 24);
  }
  const auto f = load_fn<PM, UM, MODE>(img, rec.y, j, fm, rec.x);
  (void)PW;
  (void)TTW;
  return eval_fn<PM, UM, false, LB>(f, cs, fm.sh);
}

// FN-only plans with slot data held in registers: every lane reads the record
// of its chosen predictor (one-predictor lanes and padded lanes choose 0: their
// thresholds are never reached), with no branch between lanes that select and
// lanes that do not, so the loads of several passes can be in flight together.
template <int PM, int UM, int MODE>
__device__ __forceinline__ uint32_t eval_fn_all(const SlotRegs<Shape<PM, UM>::XW, Shape<PM, UM>::TTW>& r,
                                                const NegThr& nt, const uint8_t* img, const uint8_t* cs,
                                                const uint8_t* rs, const FnFmt& fm, unsigned long long st = 0ull,
                                                const uint32_t* pre = nullptr) {
  const uint32_t w = pre ? *pre : *reinterpret_cast<const uint32_t*>(rs + (r.draw & 0xFFFFFFu));
  const auto f = load_fn<PM, UM, MODE>(img, r.base, choose_neg(w, nt), fm, r.info);
  return eval_fn<PM, UM, (MODE & 8) != 0>(f, cs, fm.sh, st);
}

// A pass whose lanes all hold one-predictor slots (or padding): the record
// load_slot keeps in registers is the one every step uses.
template <int PM, int UM, int MODE>
__device__ __forceinline__ uint32_t eval_fn_held(const SlotRegs<Shape<PM, UM>::XW, Shape<PM, UM>::TTW>& r,
                                                 const uint8_t* cs, const FnFmt& fm, unsigned long long st = 0ull) {
  constexpr int PW = Shape<PM, UM>::PW, TTW = Shape<PM, UM>::TTW;
  FnRec<PW, TTW> f;
#pragma unroll
  for (int k = 0; k < PW; ++k) f.pw[k] = r.pw[k];
#pragma unroll
  for (int k = 0; k < TTW; ++k) f.tt[k] = r.tt[k];
  return eval_fn<PM, UM, (MODE & 8) != 0>(f, cs, fm.sh, st);
}

// Store a slot's result: a table slot writes its word of member bytes (from
// the table byte's member bits), an FN slot (or padded lane) its one byte.
template <int UM>
__device__ __forceinline__ void store_slot(uint8_t* ns, uint32_t info, uint32_t spos, uint32_t out) {
  if (UM > 0 && (info & PBN_SLOT_TABLE))
    *reinterpret_cast<uint32_t*>(ns + spos) = __umul24(out, 0x204081u) & 0x01010101u;   // bit k -> byte k
  else
    ns[spos] = uint8_t(out);
}

// The keyed draws of one step of a plan with more than 64 Philox jobs per
// step, 64 at a time (job j: the first chain word for j = 0, else SEL block
// blk[j - 1]).  Job 0 is in the first round, and a step whose first chain
// word makes it perturbation-only (u >= Q[n]) reads no selection draw, so
// the later rounds are left out for it.
__device__ __forceinline__ void fill_step_keyed(uint4* ring, const uint32_t* blk, uint32_t njobs, uint32_t traj,
                                                uint32_t t, uint32_t lane, uint32_t k0, uint32_t k1, uint32_t qn_lo,
                                                uint32_t qn_hi) {
  for (uint32_t j = lane; j < njobs; j += 64u) {
    const uint4 x = philox(traj, t, j ? blk[j - 1u] : 0u, j ? PBN_STREAM_SEL : PBN_STREAM_PERT, k0, k1);
    ring[j] = x;
    if (j < 64u) {   // the first round: every lane takes part (njobs > 64), lane 0 holds job 0
      const uint32_t ulo = uniform(x.x), uhi = uniform(x.y);
      if (uhi > qn_hi || (uhi == qn_hi && ulo >= qn_lo)) break;
    }
  }
}

// A perturbation-only step (u >= Q[n], Eq. 1): walk the skip chain over all
// n original nodes of one trajectory, starting from its first drawn word u,
// and flip the kept nodes (bytes of `csb`, bits of the wave-uniform word
// `rst` with REG, or bits of the packed words at `csb` with LBITS).  Each draw counts the unperturbed nodes before the next
// perturbed one with ballots over Q (radix 64).  The chain's later draws are
// computed 64 at a time, one per lane (indices sbase .. sbase + 63), when the
// walk goes past them; a walk that flips again within them reads its next
// word with one lane read.  All lanes of the wave take part.  TOPREG: the
// top level's 64 entries of Q (entry stride0 (lane + 1), 0 past n) are held
// by the lanes in `qtop`, which saves a dependent read per draw.
template <bool G, bool REG, bool LBITS = false, bool TOPREG = false>
__device__ __forceinline__ void walk_chain(unsigned long long u, uint32_t n, uint32_t stride0,
                                           const unsigned long long* Q, const uint32_t* o2p, uint32_t traj, uint32_t t,
                                           uint32_t k0, uint32_t k1, uint32_t lane, uint8_t* csb,
                                           unsigned long long& rst, unsigned long long qtop = 0ull) {
  uint32_t j0 = 0;
  uint32_t sbase = 0u, spec_lo = 0u, spec_hi = 0u;
  bool have = false;
  for (;;) {
    uint32_t base = 0;
    for (uint32_t st = stride0;; st /= 64u) {
      const uint32_t h = base + st * (lane + 1u);
      const bool gt = TOPREG && st == stride0 ? qtop > u : h <= n && blob_u64<G>(Q + h) > u;
      base += st * uint32_t(__popcll(__ballot(gt)));
      if (st == 1u) break;
    }
    const uint32_t C = uniform(base);
    if (C >= n - j0) break;
    const uint32_t i = j0 + C;
    const uint32_t pos = blob_u32<G>(o2p + i);
    if constexpr (REG) {
      if (pos != PBN_NONE) rst ^= 1ull << uniform(pos);
    } else if constexpr (LBITS) {
      if (pos != PBN_NONE && lane == 0) reinterpret_cast<uint32_t*>(csb)[pos >> 5] ^= 1u << (pos & 31u);
    } else if (pos != PBN_NONE && lane == 0) {
      csb[pos] ^= 1u;
    }
    j0 = i + 1u;
    if (j0 >= n) break;
    if (!have || j0 - sbase >= 64u) {
      const uint4 x = philox(traj, t, j0 + lane, PBN_STREAM_PERT, k0, k1);
      spec_lo = x.x;
      spec_hi = x.y;
      sbase = j0;
      have = true;
    }
    const uint32_t off = j0 - sbase;   // wave-uniform lane index
    // the builtin returns int: take both words as unsigned 32-bit values
    u = (static_cast<unsigned long long>(uint32_t(__builtin_amdgcn_readlane(spec_hi, off))) << 32) |
        uint32_t(__builtin_amdgcn_readlane(spec_lo, off));
  }
}

// LDS copy of a plan's chain tables (several waves per trajectory): Q[0..n]
// (8 bytes each), then the original-to-position map o2p[0..n-1] (4 bytes
// each), each padded to 16 bytes.
__host__ __device__ constexpr uint32_t chain_q_bytes(uint32_t n) { return (8u * (n + 1u) + 15u) & ~15u; }
__host__ __device__ constexpr uint32_t chain_lds_bytes(uint32_t n) { return chain_q_bytes(n) + ((4u * n + 15u) & ~15u); }

// Everything one wavefront needs to advance one trajectory.
struct TrajArgs {
  const uint8_t* blob;              // plan blob (global memory)
  const uint8_t* img;               // plan image: LDS copy or the blob's own image
  uint8_t* wb;                      // this wave's LDS: state buffer(s) + ring
  unsigned long long seed;
  uint32_t traj;                    // global trajectory id (Philox counter word 0)
  uint32_t tl;                      // index within the launch's state/count arrays
  uint32_t ntraj;                   // trajectories of the launch (count layout)
  uint32_t step0, nsteps, count_from;
  uint32_t* state;                  // [ntraj][state_words]
  unsigned long long* counts;       // [ntargets][ntraj][3]
  const pbn_targets* tg;
  uint32_t* record;                 // this trajectory's indicator bits (target 0), or null
  uint32_t record_words;
  uint32_t gshift;                  // 1 (see shl_or)
  uint32_t wv, nw;                  // MODE bit 8: this wave's index among the trajectory's nw waves
  uint8_t* qo;                      // MODE bit 8: the workgroup's LDS for the chain tables (chain_lds_bytes)
};

// PM: parent bytes gathered per FN slot (>= the plan's largest predictor);
// UM: union bits gathered per TABLE slot (0: no table slots);
// NREG: 1 or 2, lane passes whose slot data stay in registers; their results
// are held in registers until all passes have read s(t), so s(t+1) overwrites
// s(t) in place (one state buffer per wave); 0: slot data reloaded every pass,
// results written to a second state buffer;
// MODE: bit 0, FN records of one or two units (batches of plans of both
// kinds); bit 1, image reads through global-address-space pointers; bit 2,
// alias sampling (Algorithms 1, 2 and 5's per-group draws) instead of the
// keyed draws; bit 3, the state held as one 64-bit wave-uniform word (bit b =
// state byte b) instead of bytes in LDS: one-pass FN-only plans whose slot
// bytes and zero word lie below 64, where s(t+1) is the pass's output ballot
// (padded lanes output 0, so the zero word stays 0); bit 5, with NREG = 0,
// each lane pass's slot records are read while the previous pass evaluates
// (one dependent global read less per pass for four more VGPRs); bit 7, with
// NREG = 1 or 2 and FN-only keyed plans, the last register-held pass holds no
// multi-predictor slot (no drawn word read, no threshold compare, and its
// records stay in registers); bit 8, with NREG = 0 and keyed draws, a.nw waves
// of one workgroup advance the trajectory together (this one is wave a.wv):
// they share its state buffers and ring, split each fill's Philox calls and
// each step's lane passes (wave w takes passes w, w + nw, ...), and meet at one
// workgroup barrier per step; wave 0 alone walks the perturbation chain (in
// place, between two barriers) and counts the targets.  Every wave takes the
// same branch of every step (the step's drawn word is read from the shared
// ring), so all reach the same barriers.
template <int PM, int UM, int NREG, int MODE>
__device__ __forceinline__ void run_traj(const TrajArgs& a) {
  constexpr int XW = Shape<PM, UM>::XW, TTW = Shape<PM, UM>::TTW;
  constexpr bool ALIAS = (MODE & 4) != 0;
  constexpr bool kPrefetch = (MODE & 32) != 0 && NREG == 0 && !ALIAS;
  constexpr bool kCached = NREG == 1 || NREG == 2;
  constexpr bool kLastNoSel = (MODE & 128) != 0 && kCached && UM == 0 && !ALIAS;
  constexpr bool kSingle = NREG != 0;   // one state buffer, updated in place
  constexpr int NR = kCached ? NREG : 1;
  // FN-only plans with register-held slots read target values from the pass
  // ballots (state byte b = bit b % 64 of pass b / 64's ballot)
  constexpr bool kBallotTargets = UM == 0 && kCached;
  // ... and mark a fill's perturbation-only steps before its steps (one scalar
  // bit per step), so that no step waits on its perturbation word to branch
  constexpr bool kPre = kBallotTargets;
  constexpr bool kRegState = (MODE & 8) != 0;
  static_assert(!kRegState || (NREG == 1 && UM == 0 && !ALIAS), "register state: one-pass FN-only keyed plans");
  constexpr bool kMW = (MODE & 256) != 0;
  static_assert(!kMW || (NREG == 0 && !ALIAS && (MODE & 2) != 0),
                "several waves per trajectory: streaming keyed plans with the image in global memory");
  const uint32_t wv = kMW ? a.wv : 0u, nw = kMW ? a.nw : 1u;
  const bool lead = !kMW || wv == 0u;   // counts targets and walks the chain
  // orders the trajectory's LDS traffic: its own lanes, or all its waves
  auto traj_sync = [&]() {
    if constexpr (kMW)
      __syncthreads();
    else
      wave_sync();
  };
  using Regs = SlotRegs<XW, TTW>;
  const pbn_plan_header* H = reinterpret_cast<const pbn_plan_header*>(a.blob);
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t n = H->n, npass = H->n_passes, njobs = H->n_jobs;
  const uint32_t fill = H->fill_steps, sd = H->state_dwords, zero_pos = H->zero_pos;
  FnFmt fm;
  fm.units = H->fn_units;
  fm.jshift = H->fn_jshift;
  fm.hoff = H->fn_hoff;
  fm.zp2 = zero_pos | (zero_pos << 16);
  fm.var = H->fn_var;
  fm.sh = a.gshift;
  const uint32_t zp2 = fm.zp2;
  const uint32_t sdp = (sd + 3u) & ~3u;   // state buffer, padded to 16 bytes
  const uint32_t* blk = reinterpret_cast<const uint32_t*>(a.blob + H->blk_off);
  const uint8_t* img = a.img;
  // the chain's tables are read from the image (LDS when the image is staged
  // there); several waves per trajectory (a latency-bound walk) copy them into
  // the workgroup's LDS first (ordered by the barrier after the state unpack)
  const unsigned long long* Q = reinterpret_cast<const unsigned long long*>(img + H->q_img);
  const uint32_t* o2p = reinterpret_cast<const uint32_t*>(img + H->o2p_img);
  constexpr bool kChainG = (MODE & 2) != 0 && !kMW;   // chain tables in global memory
  if constexpr (kMW) {
    auto* ql = reinterpret_cast<unsigned long long*>(a.qo);
    auto* ol = reinterpret_cast<uint32_t*>(a.qo + chain_q_bytes(H->n));
    for (uint32_t i = 64u * wv + lane; i <= H->n; i += 64u * nw) ql[i] = blob_u64<true>(Q + i);
    for (uint32_t i = 64u * wv + lane; i < H->n; i += 64u * nw) ol[i] = blob_u32<true>(o2p + i);
    Q = ql;
    o2p = ol;
  }
  uint32_t* sbuf0 = reinterpret_cast<uint32_t*>(a.wb);
  uint32_t* sbuf1 = kSingle ? sbuf0 : reinterpret_cast<uint32_t*>(a.wb + 4u * sdp);
  uint4* ring = reinterpret_cast<uint4*>(a.wb + (kSingle ? 4u : 8u) * sdp);   // after the state buffer(s)
  const uint32_t traj = a.traj;
  const uint32_t k0 = uint32_t(a.seed), k1 = uint32_t(a.seed >> 32);

  // unpack the packed state (bit b = state byte b), eight 4-bit groups per word
  const uint32_t W = H->state_words;
  uint32_t* gst = a.state + size_t(a.tl) * W;
  unsigned long long rst = 0ull;   // register-held state (kRegState)
  if constexpr (kRegState) rst = uniform64((W > 1u ? (static_cast<unsigned long long>(gst[1]) << 32) : 0ull) | gst[0]);
  for (uint32_t w = lane + 64u * wv; w < (kRegState ? 0u : W); w += 64u * nw) {
    const uint32_t word = gst[w];
#pragma unroll
    for (uint32_t i = 0; i < 8u; ++i) {
      sbuf0[8u * w + i] = (((word >> (4u * i)) & 0xFu) * 0x204081u) & 0x01010101u;
      if constexpr (!kSingle) sbuf1[8u * w + i] = 0;
    }
  }

  Regs cached[NR];
  NegThr nthr[NR];
  if constexpr (kCached) {
#pragma unroll
    for (int p = 0; p < NREG; ++p) {
      if (uint32_t(p) < npass) {
        load_slot<PM, UM, MODE>(cached[p], img, uint32_t(p) * 64u + lane, fm);
      } else {
        // no such pass: a one-predictor lane whose parents are all the zero
        // position and whose table is 0, writing 0 into the zero word
        cached[p] = Regs{};
        cached[p].base = H->dummy_fn;
        cached[p].draw = 1u << 24;
        cached[p].thr0 = cached[p].thr1 = cached[p].thr2 = 0xFFFFFFFFu;
        cached[p].spos = zero_pos;
#pragma unroll
        for (int k = 0; k < XW; ++k) cached[p].pw[k] = zp2;
      }
      nthr[p] = neg_thresholds(cached[p].thr0, cached[p].thr1, cached[p].thr2, cached[p].draw >> 24);
    }
  }

  // targets: lane k holds pair k; lane t counts target t
  const uint32_t npairs = a.tg->npairs, ntg = a.tg->ntargets;
  const uint32_t my_pos = lane < npairs ? a.tg->pos[lane] : zero_pos;
  const uint32_t my_val = lane < npairs ? a.tg->val[lane] : 0u;
  const unsigned long long my_mask = lane < ntg ? a.tg->mask[lane] : 0ull;
  auto target_z = [&](const uint8_t* s) -> bool {
    const uint32_t b = s[my_pos];
    const unsigned long long mism = __ballot(b != my_val);   // lanes past npairs read the zero word, expect 0
    return (mism & my_mask) == 0ull;
  };
  // ballot form of target t (lane t): bits that must be 1 (want) among the bits
  // it looks at (care), per pass (bit = slot = state byte of an FN-only plan);
  // a pair on any other byte is never 1
  uint32_t want_lo[NR], want_hi[NR], care_lo[NR], care_hi[NR];
  bool never = false;
#pragma unroll
  for (int p = 0; p < NR; ++p) want_lo[p] = want_hi[p] = care_lo[p] = care_hi[p] = 0u;
  if constexpr (kBallotTargets) {
    const uint32_t nslots = H->n_slots;
    for (unsigned long long m = my_mask; m; m &= m - 1ull) {
      const uint32_t k = uint32_t(__builtin_ctzll(m));
      const uint32_t pos = a.tg->pos[k], val = a.tg->val[k];
      const uint32_t bit = 1u << (pos & 31u), hi = (pos >> 5) & 1u;
      bool placed = false;
#pragma unroll
      for (int p = 0; p < NR; ++p) {
        if (pos < nslots && (pos >> 6) == uint32_t(p)) {
          care_lo[p] |= hi ? 0u : bit;
          care_hi[p] |= hi ? bit : 0u;
          if (val) {
            want_lo[p] |= hi ? 0u : bit;
            want_hi[p] |= hi ? bit : 0u;
          }
          placed = true;
        }
      }
      if (!placed && val) never = true;
    }
  }
  // one target (the common case): each lane's own care and want bits of
  // target 0 per register-held pass (0 or 1), so that a step's indicator is
  // one ballot of the lanes' mismatches, (out ^ want) & care, instead of a
  // masked compare of every pass's ballot on the target's lane; fewer vector
  // instructions for many waves, but one more branch in the step, so not for
  // the register-held state (one latency-bound trajectory)
  constexpr bool kOneTargetForm = kBallotTargets && !kRegState;
  const bool one_target = kOneTargetForm && ntg == 1u;
  uint32_t care_l[NR], want_l[NR];
  bool never0 = false;
#pragma unroll
  for (int p = 0; p < NR; ++p) care_l[p] = want_l[p] = 0u;
  if constexpr (kOneTargetForm) {
#pragma unroll
    for (int p = 0; p < NR; ++p) {
      const uint32_t c = lane < 32u ? uniform(care_lo[p]) >> lane : uniform(care_hi[p]) >> (lane - 32u);
      const uint32_t w = lane < 32u ? uniform(want_lo[p]) >> lane : uniform(want_hi[p]) >> (lane - 32u);
      care_l[p] = c & 1u;
      want_l[p] = w & 1u;
    }
    never0 = (__ballot(never) & 1ull) != 0ull;
  }
  traj_sync();

  // fixed Philox job of this lane when one fill covers several steps
  // plans whose slot data stay in registers have at most 64 jobs per step
  // (the host runs larger ones in the streaming form)
  const bool small_jobs = kCached || njobs <= 64u;
  const uint32_t bsteps = small_jobs ? min(fill, 32u) : 1u;   // steps per fill
  // a fill takes up to kFillRounds calls per lane: call lane + 64 r of a fill
  // is job (lane + 64 r) mod n_jobs of step (lane + 64 r) / n_jobs
  uint32_t my_s[kFillRounds], my_c2[kFillRounds], my_c3[kFillRounds];
#pragma unroll
  for (int r = 0; r < kFillRounds; ++r) {
    const uint32_t idx = lane + 64u * uint32_t(r);
    const uint32_t j = small_jobs ? idx % njobs : 0u;
    my_s[r] = small_jobs ? idx / njobs : 0u;
    my_c2[r] = ALIAS ? j : j ? blk[j - 1] : 0u;
    my_c3[r] = ALIAS ? PBN_STREAM_ALIAS : j ? PBN_STREAM_SEL : PBN_STREAM_PERT;
  }
  // alias sampling: Algorithm 2's groups, the pattern table, kept-node positions
  const uint32_t ag = ALIAS ? H->alias_g : 0u, ak = ALIAS ? H->alias_k : 1u;
  const uint32_t kmask_last = ALIAS ? (H->alias_kp >= 32u ? 0xFFFFFFFFu : (1u << H->alias_kp) - 1u) : 0u;
  const uint32_t leaf_thr = ALIAS ? H->leaf_thr : 0u;
  const uint8_t* pat = a.blob + (ALIAS ? H->pert_off : 0u);
  const uint32_t* kpos = reinterpret_cast<const uint32_t*>(a.blob + (ALIAS ? H->kpos_off : 0u));
  uint32_t stride0 = 1;
  while (stride0 * 64u < n) stride0 *= 64u;
  // several waves per trajectory (served queries, latency-bound chains): the
  // chain's top search level held in registers
  unsigned long long qtop = 0ull;
  if constexpr (kMW) {
    const uint32_t h = stride0 * (lane + 1u);
    qtop = h <= n ? blob_u64<kChainG>(Q + h) : 0ull;
  }
  const unsigned long long Qn = Q[n];
  const uint32_t qn_lo = uint32_t(Qn), qn_hi = uint32_t(Qn >> 32);

  // Target indicator z of each step is shifted into zacc (newest in bit 0);
  // at most every 32 steps the bits are folded into the counters: hits count
  // steps t >= count_from (state s(t+1)), changes count steps t >= count_from + 1
  // against the previous step's z (zlast: z before the oldest bit).
  uint32_t cur = 0;
  // register-held state: target t (lane t) from the state word itself
  auto target_reg = [&](unsigned long long b) -> bool {
    return !never && (masked_xor(uint32_t(b), care_lo[0], want_lo[0]) | masked_xor(uint32_t(b >> 32), care_hi[0], want_hi[0])) == 0u;
  };
  uint32_t zlast = 0u;
  if constexpr (kRegState)
    zlast = target_reg(rst) ? 1u : 0u;
  else if (lead)
    zlast = target_z(reinterpret_cast<const uint8_t*>(sbuf0)) ? 1u : 0u;
  uint32_t zacc = 0, nacc = 0;
  uint32_t hits = 0, n01 = 0, n10 = 0;
  uint32_t t = a.step0;
  uint32_t tacc = t;   // step of the oldest accumulated bit
  auto low_bits = [](long long m) -> uint32_t { return m <= 0 ? 0u : m >= 32 ? 0xFFFFFFFFu : (1u << m) - 1u; };
  // recorded indicator of target 0 (lane 0): bit (t - count_from) = z for the
  // transition of step t, steps count_from .. count_from + 32 record_words - 1
  auto record_bits = [&]() {
    uint64_t v = __builtin_bitreverse32(zacc) >> (32u - nacc);   // bit b: step tacc + b
    long long pos = (long long)tacc - (long long)a.count_from;
    long long cnt = nacc;
    if (pos < 0) {
      if (-pos >= cnt) return;
      v >>= -pos;
      cnt += pos;
      pos = 0;
    }
    const long long limit = 32ll * a.record_words;
    if (pos >= limit) return;
    if (pos + cnt > limit) {
      cnt = limit - pos;
      v &= (1ull << cnt) - 1ull;
    }
    const uint32_t w = uint32_t(pos >> 5);
    const uint64_t x = v << (pos & 31);
    a.record[w] |= uint32_t(x);
    if ((x >> 32) != 0ull && w + 1u < a.record_words) a.record[w + 1u] |= uint32_t(x >> 32);
  };
  auto fold = [&]() {
    if (nacc == 0u) return;
    if (a.record != nullptr && lead && lane == 0u) record_bits();
    const long long newest = (long long)tacc + nacc - 1;   // step of bit 0
    const uint32_t keep = low_bits(nacc);
    const uint32_t hm = low_bits(newest - (long long)a.count_from + 1) & keep;
    const uint32_t tm = low_bits(newest - (long long)a.count_from) & keep;
    const uint32_t prev = (zacc >> 1) | (zlast << (nacc - 1u));
    hits += __popc(zacc & hm);
    n01 += __popc(~prev & zacc & tm);
    n10 += __popc(prev & ~zacc & tm);
    zlast = zacc & 1u;
    zacc = 0u;
    tacc += nacc;
    nacc = 0u;
  };

  const uint32_t tend = a.step0 + a.nsteps;
  while (t < tend) {
    const uint32_t scount = small_jobs ? min(bsteps, tend - t) : 1u;
    if (nacc + scount > 32u) fold();
    if (small_jobs) {
#pragma unroll
      for (int r = 0; r < kFillRounds; ++r)
        if (lane + 64u * uint32_t(r) < scount * njobs && (!kMW || uint32_t(r) % nw == wv))
          ring[lane + 64u * uint32_t(r)] = philox(traj, t + my_s[r], my_c2[r], my_c3[r], k0, k1);
    } else if constexpr (ALIAS) {
      for (uint32_t j = lane; j < njobs; j += 64u) ring[j] = philox(traj, t, j, PBN_STREAM_ALIAS, k0, k1);
    } else if constexpr (kMW) {
      // several waves: wave 0 draws the first round (job 0, the step's first
      // chain word, among them); after a barrier every wave reads that word,
      // and the later rounds, split between the waves, are drawn only for a
      // step that is not perturbation-only
      if (wv == 0u) ring[lane] = philox(traj, t, lane ? blk[lane - 1u] : 0u, lane ? PBN_STREAM_SEL : PBN_STREAM_PERT,
                                        k0, k1);
      traj_sync();
      const uint2 pr = *reinterpret_cast<const uint2*>(ring);
      const uint32_t plo = uniform(pr.x), phi = uniform(pr.y);
      if (!(phi > qn_hi || (phi == qn_hi && plo >= qn_lo)))
        for (uint32_t j = 64u * (wv + 1u) + lane; j < njobs; j += 64u * nw)
          ring[j] = philox(traj, t, blk[j - 1u], PBN_STREAM_SEL, k0, k1);
    } else {
      fill_step_keyed(ring, blk, njobs, traj, t, lane, k0, k1, qn_lo, qn_hi);
    }
    traj_sync();
    if constexpr (ALIAS) {
      // Resolve the fill's perturbation draws ahead of the steps (they do not
      // depend on the state): word 1 of a step becomes its perturbed flag
      // (Algorithm 1's leaf draw, then any nonzero group pattern), words
      // 2 + 2q the patterns of Algorithm 2 (the last one masked to k' nodes).
      uint32_t* rw = reinterpret_cast<uint32_t*>(ring);
      const uint32_t spw = 4u * njobs;
      for (uint32_t s = lane; s < scount; s += 64u) rw[s * spw + 1u] = rw[s * spw] > leaf_thr ? 1u : 0u;
      wave_sync();
      for (uint32_t i = lane; i < scount * ag; i += 64u) {
        const uint32_t s = i / ag, q = i - s * ag;
        uint32_t* sw = rw + s * spw;
        const uint2 d = *reinterpret_cast<const uint2*>(sw + 2u + 2u * q);
        const uint32_t col = d.x >> (32u - ak);
        const uint2 e = img_u2<true>(pat + 8u * col);
        uint32_t c = d.y < e.x ? col : e.y;
        if (q == ag - 1u) c &= kmask_last;
        sw[2u + 2u * q] = c;
        if (c) sw[1] = 1u;
      }
      wave_sync();
    }
    uint32_t pmask = 0u;                 // kPre: bit s = step s of the fill is perturbation-only
    if constexpr (kPre) {
      bool pert = false;
      if (lane < scount) {
        const uint2 pr = *reinterpret_cast<const uint2*>(ring + lane * njobs);
        // alias sampling: word 1 is the step's resolved perturbed flag
        pert = ALIAS ? pr.y != 0u : pr.y > qn_hi || (pr.y == qn_hi && pr.x >= qn_lo);
      }
      pmask = uint32_t(__ballot(pert));   // scount <= 32
    }
    // register-held state (a latency-bound chain): each step's drawn word is
    // read one step ahead (the fill's last step re-reads its own)
    uint32_t wnext = 0u;
    if constexpr (kRegState)
      wnext = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const uint8_t*>(ring) + (cached[0].draw & 0xFFFFFFu));
    for (uint32_t s = 0; s < scount; ++s, ++t) {
      const uint8_t* rs = reinterpret_cast<const uint8_t*>(ring + s * njobs);
      const uint32_t wcur = wnext;
      if constexpr (kRegState)
        wnext = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const uint8_t*>(ring + min(s + 1u, scount - 1u) * njobs) +
                                                   (cached[0].draw & 0xFFFFFFu));
      uint32_t ulo = 0u, uhi = 0u;
      if constexpr (!kPre) {
        const uint2 pr = *reinterpret_cast<const uint2*>(rs);
        ulo = uniform(pr.x);
        uhi = uniform(pr.y);
      }
      const bool pert_step = kPre ? ((pmask >> s) & 1u) != 0u : uhi > qn_hi || (uhi == qn_hi && ulo >= qn_lo);
      uint8_t* csb = reinterpret_cast<uint8_t*>(cur ? sbuf1 : sbuf0);
      bool z = false;
      if (ALIAS && (kPre ? pert_step : uhi != 0u)) {
        // perturbation-only step (Algorithm 5): flip the nodes of every
        // group's pattern in place; pattern bit b of group q is kept node q k + b
        const uint32_t* rw = reinterpret_cast<const uint32_t*>(rs);
        for (uint32_t q = lane; q < ag; q += 64u) {
          for (uint32_t c = rw[2u + 2u * q]; c; c &= c - 1u) {
            const uint32_t pos = blob_u32<true>(kpos + q * ak + uint32_t(__builtin_ctz(c)));
            csb[pos] ^= 1u;
          }
        }
        wave_sync();
        z = target_z(csb);
      } else if (!ALIAS && pert_step) {
        // u >= Q[n]: perturbation-only step; walk the skip chain over all n
        // original nodes, flipping kept nodes in place
        if constexpr (kPre) {
          const uint2 pr = *reinterpret_cast<const uint2*>(rs);
          ulo = uniform(pr.x);
          uhi = uniform(pr.y);
        }
        if (lead)
          walk_chain<kChainG, kRegState, false, kMW>((static_cast<unsigned long long>(uhi) << 32) | ulo, n, stride0,
                                                     Q, o2p, traj, t, k0, k1, lane, csb, rst, qtop);
        traj_sync();
        if constexpr (kRegState)
          z = target_reg(rst);
        else if (lead)
          z = target_z(csb);
      } else {
        uint8_t* nsb = reinterpret_cast<uint8_t*>(cur ? sbuf0 : sbuf1);
        if constexpr (kCached) {
          // every pass reads s(t) before any writes s(t+1)
          uint32_t out[NREG];
#pragma unroll
          for (int p = 0; p < NREG; ++p) {
            if constexpr (UM == 0 && !ALIAS)
              out[p] = kLastNoSel && p == NREG - 1   // constant once the loop is unrolled
                           ? eval_fn_held<PM, UM, MODE>(cached[p], csb, fm, rst)
                           : eval_fn_all<PM, UM, MODE>(cached[p], nthr[p], img, csb, rs, fm, rst,
                                                       kRegState ? &wcur : nullptr);
            else
              out[p] = eval_slot<PM, UM, MODE>(cached[p], &nthr[p], img, csb, rs, fm);
          }
          if constexpr (kRegState) {
            // s(t+1): the pass's outputs (lane s = slot s = state byte s); padded
            // lanes, the zero word among them, output 0
            rst = __ballot(out[0] != 0u);
          } else {
#pragma unroll
            for (int p = 0; p < NREG; ++p) store_slot<UM>(nsb, cached[p].info, cached[p].spos, out[p]);
          }
          if constexpr (kBallotTargets) {
            if (kOneTargetForm && one_target) {
              uint32_t m = 0u;
#pragma unroll
              for (int p = 0; p < NREG; ++p) m |= (out[p] ^ want_l[p]) & care_l[p];
              z = !never0 && __ballot(m != 0u) == 0ull;
            } else {
              uint32_t mism = 0u;
#pragma unroll
              for (int p = 0; p < NREG; ++p) {
                const unsigned long long b = __ballot(out[p] != 0u);
                mism |= masked_xor(uint32_t(b), care_lo[p], want_lo[p]) | masked_xor(uint32_t(b >> 32), care_hi[p], want_hi[p]);
              }
              z = !never && mism == 0u;
            }
          }
        } else {
          constexpr bool G = (MODE & 2) != 0;
          uint4 nrec = kPrefetch && (!kMW || wv < npass) ? img_u4<G>(img + 16u * (wv * 64u + lane)) : uint4{};
          for (uint32_t p = wv; p < npass; p += nw) {
            if constexpr (ALIAS) {
              Regs r;
              load_slot<PM, UM, MODE>(r, img, p * 64u + lane, fm);
              store_slot<UM>(nsb, r.info, r.spos, eval_slot<PM, UM, MODE>(r, nullptr, img, csb, rs, fm));
            } else {
              uint4 rec;
              if constexpr (kPrefetch) {
                rec = nrec;
                if (p + nw < npass) nrec = img_u4<G>(img + 16u * ((p + nw) * 64u + lane));
              } else {
                rec = img_u4<G>(img + 16u * (p * 64u + lane));
              }
              uint32_t spos;
              bool table;
              const uint32_t out = eval_stream<PM, UM, MODE>(rec, img, p * 64u + lane, csb, rs, fm, spos, table);
              store_slot<UM>(nsb, table ? PBN_SLOT_TABLE : 0u, spos, out);
            }
          }
        }
        cur ^= 1u;
        if constexpr (!kRegState) traj_sync();
        if constexpr (!kBallotTargets)
          if (lead) z = target_z(nsb);
      }
      zacc = zacc + zacc + (z ? 1u : 0u);
      ++nacc;
    }
    traj_sync();
  }
  fold();

  if (lead && lane < ntg) {
    unsigned long long* c = a.counts + (size_t(lane) * a.ntraj + a.tl) * 3u;
    c[0] += hits;
    c[1] += n01;
    c[2] += n10;
  }
  if constexpr (kRegState) {
    if (lane < W) gst[lane] = lane == 0 ? uint32_t(rst) : lane == 1 ? uint32_t(rst >> 32) : 0u;
    return;
  }
  const uint32_t* fs = cur ? sbuf1 : sbuf0;
  for (uint32_t w = lane + 64u * wv; w < W; w += 64u * nw) {
    uint32_t word = 0;
#pragma unroll
    for (uint32_t i = 0; i < 8u; ++i) {
      const uint32_t v = fs[8u * w + i];
      const uint32_t nib = (v & 1u) | ((v >> 7) & 2u) | ((v >> 14) & 4u) | ((v >> 21) & 8u);
      word |= nib << (4u * i);
    }
    gst[w] = word;
  }
}

// Several trajectories per wavefront: FN-only keyed plans whose slots leave
// lanes of their last pass idle (C2: 85 slots in two passes of 64).  With K
// trajectories per wave, virtual slot v = 64 p + lane of pass p is slot v mod S
// of trajectory v / S (S slots per trajectory), so the K S virtual slots take
// ceil(K S / 64) passes instead of K ceil(S / 64).  Each trajectory keeps its
// own state buffer, drawn words and counters, and every result is the one the
// one-trajectory kernel gives.  Per step, the passes evaluate every virtual
// slot from s(t); trajectories perturbed in the step write nothing (their
// lanes store to a spare byte) and then walk their perturbation chains one
// after the other.  Target t of trajectory j is counted on lane t K + j.
struct MultiArgs {
  const uint8_t* blob;
  const uint8_t* img;
  uint8_t* wb;                      // this wave's LDS: K state buffers, a spare word, the ring
  unsigned long long seed;
  uint32_t traj0;                   // global id of the wave's trajectory 0
  uint32_t tl0;                     // its index in the launch's state/count arrays
  uint32_t nvalid;                  // trajectories of this wave (1 .. K)
  uint32_t K;                       // trajectories per wave
  uint32_t fill;                    // steps per Philox fill (fill K n_jobs <= 4 x 64, fill K <= 64)
  uint32_t ntraj, step0, nsteps, count_from;
  uint32_t* state;
  unsigned long long* counts;
  const pbn_targets* tg;
  uint32_t gshift;
};

template <int PM, int NP>
__device__ __forceinline__ void run_multi(const MultiArgs& a) {
  constexpr int UM = 0, MODE = 0;
  constexpr int XW = Shape<PM, UM>::XW, TTW = Shape<PM, UM>::TTW;
  using Regs = SlotRegs<XW, TTW>;
  const pbn_plan_header* H = reinterpret_cast<const pbn_plan_header*>(a.blob);
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t n = H->n, njobs = H->n_jobs, S = H->n_slots, zero_pos = H->zero_pos;
  const uint32_t K = a.K, nvalid = a.nvalid, kj = K * njobs;
  FnFmt fm;
  fm.units = H->fn_units;
  fm.jshift = H->fn_jshift;
  fm.hoff = H->fn_hoff;
  fm.zp2 = zero_pos | (zero_pos << 16);
  fm.var = H->fn_var;
  fm.sh = a.gshift;
  const uint32_t sbytes = 4u * ((H->state_dwords + 3u) & ~3u);   // one trajectory's buffer, 16-byte multiple
  uint8_t* sb = a.wb;
  uint8_t* spare = a.wb + K * sbytes;
  uint4* ring = reinterpret_cast<uint4*>(a.wb + K * sbytes + 16u);
  const uint32_t* blk = reinterpret_cast<const uint32_t*>(a.blob + H->blk_off);
  const uint8_t* img = a.img;
  const unsigned long long* Q = reinterpret_cast<const unsigned long long*>(img + H->q_img);
  const uint32_t* o2p = reinterpret_cast<const uint32_t*>(img + H->o2p_img);
  const uint32_t k0 = uint32_t(a.seed), k1 = uint32_t(a.seed >> 32);

  // unpack the packed states (bit b = state byte b); absent trajectories: zeros
  const uint32_t W = H->state_words;
  for (uint32_t j = 0; j < K; ++j) {
    uint32_t* buf = reinterpret_cast<uint32_t*>(sb + j * sbytes);
    const uint32_t* gst = a.state + size_t(a.tl0 + j) * W;
    for (uint32_t w = lane; w < W; w += 64u) {
      const uint32_t word = j < nvalid ? gst[w] : 0u;
#pragma unroll
      for (uint32_t i = 0; i < 8u; ++i) buf[8u * w + i] = (((word >> (4u * i)) & 0xFu) * 0x204081u) & 0x01010101u;
    }
  }

  // this lane's virtual slot in each pass: slot data held for the launch
  Regs cached[NP];
  NegThr nthr[NP];
  uint32_t sbase[NP], tj[NP];   // byte offset of the slot's trajectory buffer; that trajectory
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const uint32_t v = uint32_t(p) * 64u + lane;
    if (v < K * S) {
      const uint32_t j = v / S;
      load_slot<PM, UM, MODE>(cached[p], img, v - j * S, fm);
      cached[p].draw += j * njobs * 16u;   // the trajectory's drawn words within a step's segment
      sbase[p] = j * sbytes;
      tj[p] = j;
    } else {
      // no slot: predictor 0 of the dummy record (parents = the zero word,
      // table 0) writes 0 into the zero word of trajectory 0's buffer
      cached[p] = Regs{};
      cached[p].base = H->dummy_fn;
      cached[p].draw = 1u << 24;
      cached[p].thr0 = cached[p].thr1 = cached[p].thr2 = 0xFFFFFFFFu;
      cached[p].spos = zero_pos;
#pragma unroll
      for (int k = 0; k < XW; ++k) cached[p].pw[k] = fm.zp2;
      sbase[p] = 0u;
      tj[p] = 0u;
    }
    nthr[p] = neg_thresholds(cached[p].thr0, cached[p].thr1, cached[p].thr2, cached[p].draw >> 24);
  }

  // targets.  From the pass ballots: lane q = t K + j keeps, per pass, the
  // bits of target t's pairs in trajectory j (care) and those that must be 1
  // (want).  From a state buffer (perturbed trajectories): lane k reads pair
  // k, lane t tests target t.
  const uint32_t npairs = a.tg->npairs, ntg = a.tg->ntargets;
  const uint32_t qt = lane / K, qj = lane - qt * K;
  const bool qlive = qt < ntg;
  const uint32_t my_pos = lane < npairs ? a.tg->pos[lane] : zero_pos;
  const uint32_t my_val = lane < npairs ? a.tg->val[lane] : 0u;
  const unsigned long long my_mask = lane < ntg ? a.tg->mask[lane] : 0ull;
  uint32_t want_lo[NP], want_hi[NP], care_lo[NP], care_hi[NP];
  bool never = false;
#pragma unroll
  for (int p = 0; p < NP; ++p) want_lo[p] = want_hi[p] = care_lo[p] = care_hi[p] = 0u;
  if (qlive) {
    for (unsigned long long m = a.tg->mask[qt]; m; m &= m - 1ull) {
      const uint32_t k = uint32_t(__builtin_ctzll(m));
      const uint32_t pos = a.tg->pos[k], val = a.tg->val[k];
      if (pos >= S) {   // a removed node: reads the zero word
        if (val) never = true;
        continue;
      }
      const uint32_t v = qj * S + pos;
      const uint32_t bit = 1u << (v & 31u), hi = (v >> 5) & 1u;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        if ((v >> 6) == uint32_t(p)) {
          care_lo[p] |= hi ? 0u : bit;
          care_hi[p] |= hi ? bit : 0u;
          if (val) {
            want_lo[p] |= hi ? 0u : bit;
            want_hi[p] |= hi ? bit : 0u;
          }
        }
      }
    }
  }
  // target bits (bit t) of one trajectory's buffer
  auto target_bits = [&](const uint8_t* s) -> unsigned long long {
    const unsigned long long mism = __ballot(s[my_pos] != my_val);   // lanes past npairs read the zero word
    return __ballot(lane < ntg && (mism & my_mask) == 0ull);
  };
  wave_sync();

  // a fill of `fill` steps: call lane + 64 r is job (c mod kj) mod n_jobs of
  // trajectory (c mod kj) / n_jobs at step c / kj
  const uint32_t bsteps = a.fill;
  uint32_t my_s[kFillRounds], my_j[kFillRounds], my_c2[kFillRounds], my_c3[kFillRounds];
#pragma unroll
  for (int r = 0; r < kFillRounds; ++r) {
    const uint32_t idx = lane + 64u * uint32_t(r);
    const uint32_t st = idx / kj, rem = idx - st * kj, j = rem / njobs, job = rem - j * njobs;
    my_s[r] = st;
    my_j[r] = j;
    my_c2[r] = job ? blk[job - 1u] : 0u;
    my_c3[r] = job ? PBN_STREAM_SEL : PBN_STREAM_PERT;
  }
  uint32_t stride0 = 1;
  while (stride0 * 64u < n) stride0 *= 64u;
  const unsigned long long Qn = Q[n];
  const uint32_t qn_lo = uint32_t(Qn), qn_hi = uint32_t(Qn >> 32);
  const uint32_t kmask = (1u << K) - 1u, vmask = (1u << nvalid) - 1u;

  // indicators, as in the one-trajectory kernel, on lane q
  uint32_t zlast;
  {
    uint32_t z0 = 0u;
    for (uint32_t j = 0; j < K; ++j) {
      const unsigned long long b = target_bits(sb + j * sbytes);
      if (qj == j) z0 = uint32_t(b >> qt) & 1u;
    }
    zlast = z0;
  }
  uint32_t zacc = 0, nacc = 0, hits = 0, n01 = 0, n10 = 0;
  uint32_t t = a.step0, tacc = t;
  auto low_bits = [](long long m) -> uint32_t { return m <= 0 ? 0u : m >= 32 ? 0xFFFFFFFFu : (1u << m) - 1u; };
  auto fold = [&]() {
    if (nacc == 0u) return;
    const long long newest = (long long)tacc + nacc - 1;
    const uint32_t keep = low_bits(nacc);
    const uint32_t hm = low_bits(newest - (long long)a.count_from + 1) & keep;
    const uint32_t tm = low_bits(newest - (long long)a.count_from) & keep;
    const uint32_t prev = (zacc >> 1) | (zlast << (nacc - 1u));
    hits += __popc(zacc & hm);
    n01 += __popc(~prev & zacc & tm);
    n10 += __popc(prev & ~zacc & tm);
    zlast = zacc & 1u;
    zacc = 0u;
    tacc += nacc;
    nacc = 0u;
  };

  const uint32_t tend = a.step0 + a.nsteps;
  while (t < tend) {
    const uint32_t scount = min(bsteps, tend - t);
    if (nacc + scount > 32u) fold();
#pragma unroll
    for (int r = 0; r < kFillRounds; ++r)
      if (lane + 64u * uint32_t(r) < scount * kj)
        ring[lane + 64u * uint32_t(r)] = philox(a.traj0 + my_j[r], t + my_s[r], my_c2[r], my_c3[r], k0, k1);
    wave_sync();
    // bit s K + j: trajectory j is perturbed in step s of the fill
    bool pert = false;
    if (lane < scount * K) {
      const uint32_t st = lane / K, j = lane - st * K;
      const uint2 pr = *reinterpret_cast<const uint2*>(ring + st * kj + j * njobs);
      pert = j < nvalid && (pr.y > qn_hi || (pr.y == qn_hi && pr.x >= qn_lo));
    }
    const unsigned long long pmask = __ballot(pert);
    for (uint32_t s = 0; s < scount; ++s, ++t) {
      const uint8_t* rs = reinterpret_cast<const uint8_t*>(ring + s * kj);
      const uint32_t pb = uint32_t(pmask >> (s * K)) & kmask;
      bool z = false;
      if (pb != vmask) {
        // every pass reads s(t) before any writes s(t+1)
        uint32_t out[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) out[p] = eval_fn_all<PM, UM, MODE>(cached[p], nthr[p], img, sb + sbase[p], rs, fm);
        uint32_t mism = 0u;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const unsigned long long b = __ballot(out[p] != 0u);
          mism |= masked_xor(uint32_t(b), care_lo[p], want_lo[p]) | masked_xor(uint32_t(b >> 32), care_hi[p], want_hi[p]);
          uint8_t* dst = ((pb >> tj[p]) & 1u) ? spare : sb + sbase[p] + cached[p].spos;
          *dst = uint8_t(out[p]);
        }
        z = !never && mism == 0u;
        wave_sync();
      }
      for (uint32_t m = pb; m; m &= m - 1u) {
        // perturbation-only step of trajectory j (Eq. 1): its chain, then its targets
        const uint32_t j = uint32_t(__builtin_ctz(m));
        const uint2 pr = *reinterpret_cast<const uint2*>(rs + j * njobs * 16u);
        unsigned long long unused = 0ull;
        walk_chain<false, false>((static_cast<unsigned long long>(uniform(pr.y)) << 32) | uniform(pr.x), n, stride0,
                                 Q, o2p, a.traj0 + j, t, k0, k1, lane, sb + j * sbytes, unused);
        wave_sync();
        const unsigned long long b = target_bits(sb + j * sbytes);
        if (qj == j) z = ((b >> qt) & 1ull) != 0ull;
      }
      zacc = zacc + zacc + (z ? 1u : 0u);
      ++nacc;
    }
    wave_sync();
  }
  fold();

  if (qlive && qj < nvalid) {
    unsigned long long* c = a.counts + (size_t(qt) * a.ntraj + a.tl0 + qj) * 3u;
    c[0] += hits;
    c[1] += n01;
    c[2] += n10;
  }
  for (uint32_t j = 0; j < nvalid; ++j) {
    const uint32_t* fs = reinterpret_cast<const uint32_t*>(sb + j * sbytes);
    uint32_t* gst = a.state + size_t(a.tl0 + j) * W;
    for (uint32_t w = lane; w < W; w += 64u) {
      uint32_t word = 0;
#pragma unroll
      for (uint32_t i = 0; i < 8u; ++i) {
        const uint32_t v = fs[8u * w + i];
        const uint32_t nib = (v & 1u) | ((v >> 7) & 2u) | ((v >> 14) & 4u) | ((v >> 21) & 8u);
        word |= nib << (4u * i);
      }
      gst[w] = word;
    }
  }
}

// One network: one wavefront per trajectory, the plan image staged in LDS when
// it fits (IMG_LDS), shared by the workgroup's waves.  ALIAS: the plan's alias
// sampling draws.
template <bool IMG_LDS, int PM, int UM, int NREG, bool ALIAS, bool REGSTATE = false, bool NOSEL = false>
__global__ void __launch_bounds__(1024) k_simulate(SimParams a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  const pbn_plan_header* H = reinterpret_cast<const pbn_plan_header*>(a.blob);
  const uint32_t wave = uniform(threadIdx.x >> 6);   // wave-uniform: keeps per-trajectory data scalar
  const uint32_t img_bytes = H->image_bytes;
  const uint8_t* gimg = a.blob + H->image_off;
  uint32_t img_lds = 0;
  if constexpr (IMG_LDS) {
    for (uint32_t o = threadIdx.x * 16u; o < img_bytes; o += blockDim.x * 16u)
      *reinterpret_cast<uint4*>(smem + o) = *reinterpret_cast<const uint4*>(gimg + o);
    img_lds = (img_bytes + 15u) & ~15u;
  }
  __syncthreads();
  const uint32_t tl = blockIdx.x * a.wpb + wave;
  if (tl >= a.ntraj) return;
  TrajArgs t;
  t.blob = a.blob;
  if constexpr (IMG_LDS)
    t.img = smem;
  else
    t.img = gimg;
  t.wb = smem + img_lds + wave * a.wave_bytes;
  t.seed = a.seed;
  t.traj = a.traj0 + tl;
  t.tl = tl;
  t.ntraj = a.ntraj;
  t.step0 = a.step0;
  t.nsteps = a.nsteps;
  t.count_from = a.count_from;
  t.state = a.state;
  t.counts = a.counts;
  t.tg = &a.tg;
  t.record = a.record && tl < a.record_traj ? a.record + size_t(tl) * a.record_words : nullptr;
  t.record_words = a.record_words;
  t.gshift = a.gshift;
  run_traj<PM, UM, NREG, (ALIAS ? 4 : 0) | (REGSTATE ? 8 : 0) | 32 | (NOSEL ? 128 : 0)>(t);
}

// One network, K = a.tpw trajectories per wavefront (run_multi); NP lane
// passes.  Trajectories tl0 .. tl0 + K - 1 of wave w, tl0 = K w.
template <bool IMG_LDS, int PM, int NP>
__global__ void __launch_bounds__(1024) k_simulate_multi(SimParams a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  const pbn_plan_header* H = reinterpret_cast<const pbn_plan_header*>(a.blob);
  const uint32_t wave = uniform(threadIdx.x >> 6);
  const uint32_t img_bytes = H->image_bytes;
  const uint8_t* gimg = a.blob + H->image_off;
  uint32_t img_lds = 0;
  if constexpr (IMG_LDS) {
    for (uint32_t o = threadIdx.x * 16u; o < img_bytes; o += blockDim.x * 16u)
      *reinterpret_cast<uint4*>(smem + o) = *reinterpret_cast<const uint4*>(gimg + o);
    img_lds = (img_bytes + 15u) & ~15u;
  }
  __syncthreads();
  const uint32_t tl0 = (blockIdx.x * a.wpb + wave) * a.tpw;
  if (tl0 >= a.ntraj) return;
  MultiArgs m;
  m.blob = a.blob;
  m.img = IMG_LDS ? smem : gimg;
  m.wb = smem + img_lds + wave * a.wave_bytes;
  m.seed = a.seed;
  m.traj0 = a.traj0 + tl0;
  m.tl0 = tl0;
  m.nvalid = min(a.tpw, a.ntraj - tl0);
  m.K = a.tpw;
  m.fill = a.mfill;
  m.ntraj = a.ntraj;
  m.step0 = a.step0;
  m.nsteps = a.nsteps;
  m.count_from = a.count_from;
  m.state = a.state;
  m.counts = a.counts;
  m.tg = &a.tg;
  m.gshift = a.gshift;
  run_multi<PM, NP>(m);
}

// Packed-bit state (plans built with state_bits): the trajectory state in LDS
// is the packed state itself, two buffers of W words per wave (s(t), s(t+1)),
// about an eighth of the byte layout's LDS, so a workgroup of up to 16 waves
// keeps a large plan image in LDS beside them.  Parents are read as bits
// (gather_lbits).  Pass p writes its own segment of s(t+1) as whole words: a
// table pass (4 bits per lane) ORs the nibbles of 8 lanes with three
// row-shift DPP steps and every eighth lane stores a word; a pass of FN slots
// stores its output ballot (two words).  Keyed draws, slot data reloaded
// every pass (any number of passes); MODE bit 1: global-address-space image
// reads (not used by k_simulate_bits).
template <int PM, int UM, int MODE>
__device__ __forceinline__ void run_bits(const TrajArgs& a) {
  constexpr int M = MODE | 16;   // state as bits
  const pbn_plan_header* H = reinterpret_cast<const pbn_plan_header*>(a.blob);
  const pbn_pass_info* pinfo = reinterpret_cast<const pbn_pass_info*>(a.blob + H->pass_off);
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t n = H->n, npass = H->n_passes, njobs = H->n_jobs;
  const uint32_t fill = H->fill_steps, zero_pos = H->zero_pos;
  FnFmt fm;
  fm.units = H->fn_units;
  fm.jshift = H->fn_jshift;
  fm.hoff = H->fn_hoff;
  fm.zp2 = zero_pos | (zero_pos << 16);
  fm.var = H->fn_var;
  fm.sh = a.gshift;
  const uint32_t W = H->state_words, Wp = (W + 3u) & ~3u;
  // the two buffers, chosen by a select (an indexed pointer array would hide
  // from the compiler that both lie in LDS, and turn their reads into flat loads)
  uint32_t* const buf0 = reinterpret_cast<uint32_t*>(a.wb);
  uint32_t* const buf1 = buf0 + Wp;
  uint4* ring = reinterpret_cast<uint4*>(a.wb + 8u * Wp);
  const uint32_t* blk = reinterpret_cast<const uint32_t*>(a.blob + H->blk_off);
  const uint8_t* img = a.img;
  const unsigned long long* Q = reinterpret_cast<const unsigned long long*>(img + H->q_img);
  const uint32_t* o2p = reinterpret_cast<const uint32_t*>(img + H->o2p_img);
  const uint32_t traj = a.traj;
  const uint32_t k0 = uint32_t(a.seed), k1 = uint32_t(a.seed >> 32);

  uint32_t* gst = a.state + size_t(a.tl) * W;
  for (uint32_t w = lane; w < Wp; w += 64u) {
    buf0[w] = w < W ? gst[w] : 0u;
    buf1[w] = 0u;   // the zero word of s(t+1) stays 0: no pass writes it
  }

  const uint32_t npairs = a.tg->npairs, ntg = a.tg->ntargets;
  const uint32_t my_pos = lane < npairs ? a.tg->pos[lane] : zero_pos;
  const uint32_t my_val = lane < npairs ? a.tg->val[lane] : 0u;
  const unsigned long long my_mask = lane < ntg ? a.tg->mask[lane] : 0ull;
  auto target_z = [&](const uint32_t* words) -> bool {
    const uint32_t b = (words[my_pos >> 5] >> (my_pos & 31u)) & 1u;
    const unsigned long long mism = __ballot(b != my_val);   // lanes past npairs read the zero word
    return (mism & my_mask) == 0ull;
  };
  wave_sync();

  const bool small_jobs = njobs <= 64u;
  const uint32_t bsteps = small_jobs ? min(fill, 32u) : 1u;
  uint32_t my_s[kFillRounds], my_c2[kFillRounds], my_c3[kFillRounds];
#pragma unroll
  for (int r = 0; r < kFillRounds; ++r) {
    const uint32_t idx = lane + 64u * uint32_t(r);
    const uint32_t j = small_jobs ? idx % njobs : 0u;
    my_s[r] = small_jobs ? idx / njobs : 0u;
    my_c2[r] = j ? blk[j - 1] : 0u;
    my_c3[r] = j ? PBN_STREAM_SEL : PBN_STREAM_PERT;
  }
  uint32_t stride0 = 1;
  while (stride0 * 64u < n) stride0 *= 64u;
  const unsigned long long Qn = Q[n];
  const uint32_t qn_lo = uint32_t(Qn), qn_hi = uint32_t(Qn >> 32);
  const uint32_t nib_shift = 4u * (lane & 7u);

  uint32_t cur = 0;
  uint32_t zlast = target_z(buf0) ? 1u : 0u;
  uint32_t zacc = 0, nacc = 0, hits = 0, n01 = 0, n10 = 0;
  uint32_t t = a.step0, tacc = t;
  auto low_bits = [](long long m) -> uint32_t { return m <= 0 ? 0u : m >= 32 ? 0xFFFFFFFFu : (1u << m) - 1u; };
  auto fold = [&]() {
    if (nacc == 0u) return;
    const long long newest = (long long)tacc + nacc - 1;
    const uint32_t keep = low_bits(nacc);
    const uint32_t hm = low_bits(newest - (long long)a.count_from + 1) & keep;
    const uint32_t tm = low_bits(newest - (long long)a.count_from) & keep;
    const uint32_t prev = (zacc >> 1) | (zlast << (nacc - 1u));
    hits += __popc(zacc & hm);
    n01 += __popc(~prev & zacc & tm);
    n10 += __popc(prev & ~zacc & tm);
    zlast = zacc & 1u;
    zacc = 0u;
    tacc += nacc;
    nacc = 0u;
  };

  const uint32_t tend = a.step0 + a.nsteps;
  while (t < tend) {
    const uint32_t scount = small_jobs ? min(bsteps, tend - t) : 1u;
    if (nacc + scount > 32u) fold();
    if (small_jobs) {
#pragma unroll
      for (int r = 0; r < kFillRounds; ++r)
        if (lane + 64u * uint32_t(r) < scount * njobs)
          ring[lane + 64u * uint32_t(r)] = philox(traj, t + my_s[r], my_c2[r], my_c3[r], k0, k1);
    } else {
      fill_step_keyed(ring, blk, njobs, traj, t, lane, k0, k1, qn_lo, qn_hi);
    }
    wave_sync();
    for (uint32_t s = 0; s < scount; ++s, ++t) {
      const uint8_t* rs = reinterpret_cast<const uint8_t*>(ring + s * njobs);
      const uint2 pr = *reinterpret_cast<const uint2*>(rs);
      const uint32_t ulo = uniform(pr.x), uhi = uniform(pr.y);
      uint32_t* cw = cur ? buf1 : buf0;
      bool z;
      if (uhi > qn_hi || (uhi == qn_hi && ulo >= qn_lo)) {
        // perturbation-only step: flip the perturbed kept nodes' bits in place
        unsigned long long unused = 0ull;
        walk_chain<(MODE & 2) != 0, false, true>((static_cast<unsigned long long>(uhi) << 32) | ulo, n, stride0, Q,
                                                 o2p, traj, t, k0, k1, lane, reinterpret_cast<uint8_t*>(cw), unused);
        wave_sync();
        z = target_z(cw);
      } else {
        uint32_t* nw = cur ? buf0 : buf1;
        uint32_t seg = 0;   // word offset of pass p's segment
        for (uint32_t p = 0; p < npass; ++p) {
          const uint32_t flags = uniform(pinfo[p].flags);
          uint32_t spos;
          bool table;
          const uint4 rec = img_u4<(M & 2) != 0>(img + 16u * (p * 64u + lane));
          const uint32_t out = eval_stream<PM, UM, M>(rec, img, p * 64u + lane, reinterpret_cast<const uint8_t*>(cw), rs,
                                                      fm, spos, table);
          if (flags & PBN_PASS_TABLE) {
            // lane L's nibble at bits 4 (L mod 8) of word L / 8 of the segment
            uint32_t v = out << nib_shift;
            v |= __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xF, 0xF, true);   // row_shr:1
            v |= __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xF, 0xF, true);   // row_shr:2
            v |= __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xF, 0xF, true);   // row_shr:4
            if ((lane & 7u) == 7u) nw[seg + (lane >> 3)] = v;
            seg += 8u;
          } else {
            const unsigned long long b = __ballot(out != 0u);
            if (lane < 2u) nw[seg + lane] = lane ? uint32_t(b >> 32) : uint32_t(b);
            seg += 2u;
          }
        }
        cur ^= 1u;
        wave_sync();
        z = target_z(nw);
      }
      zacc = zacc + zacc + (z ? 1u : 0u);
      ++nacc;
    }
    wave_sync();
  }
  fold();

  if (lane < ntg) {
    unsigned long long* c = a.counts + (size_t(lane) * a.ntraj + a.tl) * 3u;
    c[0] += hits;
    c[1] += n01;
    c[2] += n10;
  }
  for (uint32_t w = lane; w < W; w += 64u) gst[w] = cur ? buf1[w] : buf0[w];
}

// One network with a packed-bit state (run_bits): one wavefront per
// trajectory, the plan image staged in LDS when it fits beside the waves'
// states and rings.
template <bool IMG_LDS, int PM, int UM>
__global__ void __launch_bounds__(1024) k_simulate_bits(SimParams a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  const pbn_plan_header* H = reinterpret_cast<const pbn_plan_header*>(a.blob);
  const uint32_t wave = uniform(threadIdx.x >> 6);
  const uint32_t img_bytes = H->image_bytes;
  const uint8_t* gimg = a.blob + H->image_off;
  uint32_t img_lds = 0;
  if constexpr (IMG_LDS) {
    for (uint32_t o = threadIdx.x * 16u; o < img_bytes; o += blockDim.x * 16u)
      *reinterpret_cast<uint4*>(smem + o) = *reinterpret_cast<const uint4*>(gimg + o);
    img_lds = (img_bytes + 15u) & ~15u;
  }
  __syncthreads();
  const uint32_t tl = blockIdx.x * a.wpb + wave;
  if (tl >= a.ntraj) return;
  TrajArgs t;
  t.blob = a.blob;
  t.img = IMG_LDS ? smem : gimg;
  t.wb = smem + img_lds + wave * a.wave_bytes;
  t.seed = a.seed;
  t.traj = a.traj0 + tl;
  t.tl = tl;
  t.ntraj = a.ntraj;
  t.step0 = a.step0;
  t.nsteps = a.nsteps;
  t.count_from = a.count_from;
  t.state = a.state;
  t.counts = a.counts;
  t.tg = &a.tg;
  t.record = nullptr;
  t.record_words = 0;
  t.gshift = a.gshift;
  run_bits<PM, UM, 0>(t);
}

// ---------------------------------------------------------------- batches
// Many networks of uneven size in one persistent launch.  Work is cut into
// tasks of `wpb` consecutive trajectories of one network, in nq queues of
// whole networks, ordered by the host (largest networks first within a
// queue).  The dispatcher sends workgroup b to XCD b mod 8 and, within the
// XCD, to its 32 CUs in turn, so the CU of a resident workgroup follows from
// b mod 256; with nq = 8 G, workgroup b starts on queue b mod nq, and the
// workgroups of a queue fill their own group of 32 / G CUs of one XCD, whose
// vector L1 caches then hold the images of few networks (one queue for the
// whole chip mixed the images of every network in flight on each CU).  A
// workgroup repeatedly claims the next task of its queue with one atomic
// increment; when its queue is empty it tries the other groups of its XCD,
// then those of the next XCDs (a queue found empty stays empty: its counter
// only grows), and it stops after the last one, so every wave reaches the
// exit.  The placement only decides which caches a task shares; any other
// placement gives the same results.  Plan images stay in global memory (the
// L2 serves them); each wave's LDS holds its trajectory's state buffers and
// Philox ring.
struct QueueBounds {
  uint32_t first[PBN_BATCH_QUEUES + 1];   // queue k: tasks first[k] .. first[k + 1] - 1
};

struct BatchParams {
  const pbn_work* items;
  const uint32_t* tasks;           // item of task k
  const uint32_t* task_first;      // first trajectory (local index) of task k
  uint32_t ntasks;                 // PBN_NONE: one queue of ctl->ntasks tasks, written on the device
  uint32_t wpb;                    // trajectories per task
  uint32_t wpt;                    // waves per trajectory (> 1: one trajectory per workgroup)
  uint32_t wave_bytes;             // LDS per trajectory: state buffers and ring; with wpt > 1 the chain
                                   // tables follow them (chain_lds_bytes of the largest network)
  uint32_t gshift;                 // 1: the gather step's shift, passed at run time (see shl_or)
  pbn_batch_ctl* ctl;              // device: queue counters and the step window
  uint32_t nq;                     // queues, 1 .. PBN_BATCH_QUEUES
  QueueBounds q;
};

// PF: each pass's slot records are read while the previous pass evaluates
// (run_traj MODE bit 5): launches too small to fill the chip at four waves
// per SIMD, where its four VGPRs cost no occupancy and the step latency of
// one trajectory is what counts (served queries).  MW: the workgroup's wpt
// waves advance one trajectory together (run_traj MODE bit 8), for a shorter
// step latency of the trajectories of large networks.
template <int PM, int UM, bool PF, bool MW>
__global__ void __launch_bounds__(1024) k_batch(BatchParams a, const pbn_work* __restrict__ items) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  // first 16 bytes: the claimed task, and how many queues thread 0 has found
  // empty (kept here, not in a register live across the trajectory body)
  uint32_t& claimed = *reinterpret_cast<uint32_t*>(smem);
  uint32_t& tried = *reinterpret_cast<uint32_t*>(smem + 4);
  const uint32_t wave = uniform(threadIdx.x >> 6);   // wave-uniform: keeps per-trajectory data scalar
  const uint32_t wstep0 = a.ctl->step0, nsteps = a.ctl->nsteps;
  if (threadIdx.x == 0) tried = 0;
  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t nq = a.nq, home = blockIdx.x % nq;
      const uint32_t groups = nq % 8u == 0 ? nq / 8u : 0u;   // CU groups per XCD
      uint32_t task = PBN_NONE, t = tried;
      for (; t < nq; ++t) {
        // the groups of the home XCD first (8 a + c runs over 0 .. nq - 1 once)
        const uint32_t k = groups ? (home + 8u * (t % groups) + t / groups) % nq : (home + t) % nq;
        // PBN_NONE: the schedule was written on the device (allocation-free launch)
        const uint32_t end = a.ntasks != PBN_NONE ? a.q.first[k + 1] : (k == 0 ? a.ctl->ntasks : 0u);
        if (a.q.first[k] >= end) continue;   // an empty queue costs no atomic
        const uint32_t c = atomicAdd(&a.ctl->next_task[k], 1u);
        if (c < end) {
          task = c;
          break;
        }
      }
      tried = t;
      claimed = task;
    }
    __syncthreads();
    const uint32_t task = uniform(claimed);   // the same for the workgroup: scalar loads of the task's item
    __syncthreads();
    if (task == PBN_NONE) return;        // uniform across the workgroup
    // the task's work item, read into wave-uniform values (scalar registers)
    const pbn_work& it = items[uniform(a.tasks[task])];
    const uint32_t slot = MW ? 0u : wave;   // the wave's trajectory within the task
    const uint32_t tl = uniform(a.task_first[task]) + slot;
    const uint32_t ntraj = uniform(it.ntraj);
    if (tl < ntraj) {
      const uint8_t* blob = static_cast<const uint8_t*>(it.d_plan);
      const pbn_plan_header* H = reinterpret_cast<const pbn_plan_header*>(blob);
      TrajArgs t;
      t.blob = blob;
      t.img = blob + H->image_off;
      t.wb = smem + 16u + slot * a.wave_bytes;
      t.seed = uniform64(it.seed);
      t.traj = uniform(it.traj0) + tl;
      t.tl = tl;
      t.ntraj = ntraj;
      t.step0 = uniform(it.step0) + wstep0;
      t.nsteps = nsteps;
      t.count_from = uniform(it.count_from);
      t.state = it.d_state;
      t.counts = reinterpret_cast<unsigned long long*>(it.d_counts);
      t.tg = it.d_targets;
      t.record = nullptr;
      t.record_words = 0;
      t.gshift = a.gshift;
      t.wv = MW ? wave : 0u;
      t.nw = MW ? a.wpt : 1u;
      t.qo = MW ? smem + 16u + a.wave_bytes : nullptr;
      // large launches run without the prefetch: its four VGPRs would take
      // this kernel from five to four waves per SIMD
      run_traj<PM, UM, 0, (PM == 7 ? 1 : 0) | 2 | (PF ? 32 : 0) | (MW ? 256 : 0)>(t);
    }
  }
}

// Graph-friendly control updates (no memset nodes): set each queue's counter
// to its first task before a batch pass, advance the step window after it.
__global__ void k_batch_begin(pbn_batch_ctl* ctl, QueueBounds q, uint32_t nq) {
  if (threadIdx.x < nq) ctl->next_task[threadIdx.x] = q.first[threadIdx.x];
}
__global__ void k_batch_end(pbn_batch_ctl* ctl) { ctl->step0 += ctl->nsteps; }

// ------------------------------------------------ allocation-free batches
// pbn_batch_launch_noalloc keeps what pbn_batch_launch takes from the caller
// as workspace -- the control block and the task schedule -- in one
// file-scope device array, so that the entry point allocates nothing.  Each
// GPU holds its own copy until the process ends; the host reaches it only
// through the address hipGetSymbolAddress returns for the current device.
constexpr uint32_t kNoAllocMaxItems = 4096u;    // work items per call
constexpr uint32_t kNoAllocMaxTasks = 65536u;   // tasks (waves_per_block trajectories of one item) per call
constexpr uint32_t kScratchCtlWords = 128u;     // the control block, alone in the first 512 bytes
static_assert(sizeof(pbn_batch_ctl) <= 4u * kScratchCtlWords, "control block exceeds its scratch region");
constexpr size_t kScratchWords = kScratchCtlWords + 2u * size_t(kNoAllocMaxTasks);
static __device__ __align__(256) uint32_t scratch[kScratchWords];   // 512.5 KiB

// The schedule of one allocation-free launch, written by one workgroup of
// 1024 threads: items in the caller's order, ceil(ntraj / wpb) tasks each
// (task k of an item starts at trajectory k wpb); the control block gets a
// zero task counter, the step window and the task count.  Items beyond
// kNoAllocMaxItems and tasks beyond kNoAllocMaxTasks are rejected on the host.
__global__ void __launch_bounds__(1024) k_noalloc_schedule(const pbn_work* items, uint32_t nitems, uint32_t wpb,
                                                          uint32_t step0, uint32_t nsteps, uint32_t* scr) {
  __shared__ uint32_t part[1024];
  const uint32_t t = threadIdx.x;
  const uint32_t chunk = (nitems + 1023u) / 1024u;
  const uint32_t lo = min(nitems, t * chunk), hi = min(nitems, lo + chunk);
  uint32_t mine = 0;
  for (uint32_t k = lo; k < hi; ++k) mine += (items[k].ntraj + wpb - 1u) / wpb;
  part[t] = mine;
  __syncthreads();
  for (uint32_t d = 1; d < 1024u; d <<= 1) {   // inclusive prefix sums
    const uint32_t v = t >= d ? part[t - d] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t* tasks = scr + kScratchCtlWords;
  uint32_t* first = tasks + kNoAllocMaxTasks;
  uint32_t at = part[t] - mine;
  for (uint32_t k = lo; k < hi; ++k) {
    const uint32_t cnt = (items[k].ntraj + wpb - 1u) / wpb;
    for (uint32_t f = 0; f < cnt && at < kNoAllocMaxTasks; ++f, ++at) {
      tasks[at] = k;
      first[at] = f * wpb;
    }
  }
  if (t == 1023u) {
    pbn_batch_ctl* ctl = reinterpret_cast<pbn_batch_ctl*>(scr);
    ctl->next_task[0] = 0;   // one queue
    ctl->step0 = step0;
    ctl->nsteps = nsteps;
    ctl->ntasks = min(part[1023], kNoAllocMaxTasks);
  }
}

// s(0): bit i of node i's INIT word, placed at the node's plan position.
__global__ void k_state_init(const uint8_t* blob, unsigned long long seed, uint32_t traj0, uint32_t ntraj,
                             uint32_t* state) {
  const pbn_plan_header* H = reinterpret_cast<const pbn_plan_header*>(blob);
  const uint32_t W = H->state_words, nbytes = 32u * W;
  const uint32_t* p2o = reinterpret_cast<const uint32_t*>(blob + H->p2o_off);
  const uint32_t k0 = uint32_t(seed), k1 = uint32_t(seed >> 32);
  const size_t total = size_t(ntraj) * W;
  for (size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < total; idx += size_t(gridDim.x) * blockDim.x) {
    const uint32_t tl = uint32_t(idx / W), w = uint32_t(idx % W);
    uint32_t word = 0, cached = PBN_NONE;
    uint4 x = make_uint4(0, 0, 0, 0);
    for (uint32_t b = 0; b < 32u; ++b) {
      const uint32_t pos = 32u * w + b;
      if (pos >= nbytes) break;
      const uint32_t o = p2o[pos];
      if (o == PBN_NONE) continue;
      if ((o >> 7) != cached) {
        cached = o >> 7;
        x = philox(traj0 + tl, 0u, cached, PBN_STREAM_INIT, k0, k1);
      }
      const uint32_t sel = (o >> 5) & 3u;
      const uint32_t src = sel == 0 ? x.x : sel == 1 ? x.y : sel == 2 ? x.z : x.w;
      word |= ((src >> (o & 31u)) & 1u) << b;
    }
    state[idx] = word;
  }
}

__global__ void k_to_original(const uint8_t* blob, const uint32_t* state, uint32_t ntraj, uint32_t* out) {
  const pbn_plan_header* H = reinterpret_cast<const pbn_plan_header*>(blob);
  const uint32_t W = H->state_words, n = H->n, WO = (n + 31u) / 32u;
  const uint32_t* o2p = reinterpret_cast<const uint32_t*>(blob + H->o2p_off);
  const size_t total = size_t(ntraj) * WO;
  for (size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < total; idx += size_t(gridDim.x) * blockDim.x) {
    const uint32_t tl = uint32_t(idx / WO), w = uint32_t(idx % WO);
    const uint32_t* st = state + size_t(tl) * W;
    uint32_t word = 0;
    for (uint32_t b = 0; b < 32u; ++b) {
      const uint32_t i = 32u * w + b;
      if (i >= n) break;
      const uint32_t pos = o2p[i];
      if (pos == PBN_NONE) continue;
      word |= ((st[pos >> 5] >> (pos & 31u)) & 1u) << b;
    }
    out[idx] = word;
  }
}

pbn_status fail(pbn_status code, const std::string& msg) {
  pbn::set_error(msg);
  return code;
}

pbn_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return PBN_OK;
  return fail(PBN_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

uint32_t grid_for(size_t work, uint32_t block) {
  const size_t g = (work + block - 1) / block;
  return uint32_t(std::min<size_t>(std::max<size_t>(g, 1), 65536));
}

constexpr uint32_t kLdsMax = 160u * 1024u;

// LDS of one wave: the state buffer(s) and the Philox ring (one fill:
// min(fill, 32) steps of n_jobs calls when the calls of a step fit in a wave,
// else one step).  `single`: the kernel updates one state buffer in place
// (plans of one or two lane passes in k_simulate).
uint32_t wave_lds_bytes(const pbn_plan* plan, bool single) {
  const uint32_t ring = plan->n_jobs <= 64 ? std::min(plan->fill_steps, 32u) * plan->n_jobs : plan->n_jobs;
  return (single ? 4u : 8u) * ((plan->state_dwords + 3u) & ~3u) + 16u * ring;
}

template <bool IMG_LDS, int PM, int UM, int NREG, bool ALIAS, bool REGSTATE = false, bool NOSEL = false>
pbn_status launch_sim(const SimParams& p, uint32_t blocks, uint32_t lds, hipStream_t stream) {
  auto* fn = k_simulate<IMG_LDS, PM, UM, NREG, ALIAS, REGSTATE, NOSEL>;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       int(kLdsMax));
    if (e != hipSuccess) return hip_check(e, "hipFuncSetAttribute");
    attr_set = true;
  }
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(64u * p.wpb), lds, stream, p);
  return hip_check(hipGetLastError(), "k_simulate launch");
}

// Instantiation choice: the smallest gather widths that cover the plan.
// nreg: 1 or 2, the lane passes whose slot data stay in registers; 0, the
// streaming form.  lastsel: the last of the nreg passes holds a
// multi-predictor slot.
template <bool IMG_LDS, int PM, int UM, bool ALIAS>
pbn_status dispatch_nreg(const SimParams& p, uint32_t nreg, bool lastsel, bool reg, uint32_t blocks, uint32_t lds,
                         hipStream_t s) {
  if constexpr (UM == 0 && !ALIAS) {
    // one pass, every state byte below 64: the state lives in a register
    if (reg) return launch_sim<IMG_LDS, PM, 0, 1, false, true>(p, blocks, lds, s);
    if (!lastsel && nreg == 1) return launch_sim<IMG_LDS, PM, 0, 1, false, false, true>(p, blocks, lds, s);
    if (!lastsel && nreg == 2) return launch_sim<IMG_LDS, PM, 0, 2, false, false, true>(p, blocks, lds, s);
  }
  if (nreg == 1) return launch_sim<IMG_LDS, PM, UM, 1, ALIAS>(p, blocks, lds, s);
  if (nreg == 2) return launch_sim<IMG_LDS, PM, UM, 2, ALIAS>(p, blocks, lds, s);
  return launch_sim<IMG_LDS, PM, UM, 0, ALIAS>(p, blocks, lds, s);
}

template <bool IMG_LDS, int PM, bool ALIAS>
pbn_status dispatch_um(const SimParams& p, uint32_t umax, uint32_t nreg, bool lastsel, bool reg, uint32_t blocks,
                       uint32_t lds, hipStream_t s) {
  if (umax == 0) return dispatch_nreg<IMG_LDS, PM, 0, ALIAS>(p, nreg, lastsel, reg, blocks, lds, s);
  if constexpr (!ALIAS) {
    if (umax <= 6) return dispatch_nreg<IMG_LDS, PM, 6, ALIAS>(p, nreg, true, false, blocks, lds, s);
  }
  if (umax <= 8) return dispatch_nreg<IMG_LDS, PM, 8, ALIAS>(p, nreg, true, false, blocks, lds, s);
  return dispatch_nreg<IMG_LDS, PM, 16, ALIAS>(p, nreg, true, false, blocks, lds, s);
}

template <bool IMG_LDS, bool ALIAS>
pbn_status dispatch_pm(const SimParams& p, uint32_t pmax, uint32_t umax, uint32_t nreg, bool lastsel, bool reg,
                       uint32_t blocks, uint32_t lds, hipStream_t s) {
  if (pmax <= 5) return dispatch_um<IMG_LDS, 5, ALIAS>(p, umax, nreg, lastsel, reg, blocks, lds, s);
  return dispatch_um<IMG_LDS, 7, ALIAS>(p, umax, nreg, lastsel, reg, blocks, lds, s);
}

template <bool IMG_LDS, int PM, int UM>
pbn_status launch_bits(const SimParams& p, uint32_t blocks, uint32_t lds, hipStream_t stream) {
  auto* fn = k_simulate_bits<IMG_LDS, PM, UM>;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       int(kLdsMax));
    if (e != hipSuccess) return hip_check(e, "hipFuncSetAttribute");
    attr_set = true;
  }
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(64u * p.wpb), lds, stream, p);
  return hip_check(hipGetLastError(), "k_simulate_bits launch");
}

template <bool IMG_LDS, int PM>
pbn_status dispatch_bits_um(const SimParams& p, uint32_t umax, uint32_t blocks, uint32_t lds, hipStream_t s) {
  if (umax == 0) return launch_bits<IMG_LDS, PM, 0>(p, blocks, lds, s);
  if (umax <= 6) return launch_bits<IMG_LDS, PM, 6>(p, blocks, lds, s);
  if (umax <= 8) return launch_bits<IMG_LDS, PM, 8>(p, blocks, lds, s);
  return launch_bits<IMG_LDS, PM, 16>(p, blocks, lds, s);
}

template <bool IMG_LDS, int PM, int NP>
pbn_status launch_multi(const SimParams& p, uint32_t blocks, uint32_t lds, hipStream_t stream) {
  auto* fn = k_simulate_multi<IMG_LDS, PM, NP>;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       int(kLdsMax));
    if (e != hipSuccess) return hip_check(e, "hipFuncSetAttribute");
    attr_set = true;
  }
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(64u * p.wpb), lds, stream, p);
  return hip_check(hipGetLastError(), "k_simulate_multi launch");
}

template <bool IMG_LDS, int PM>
pbn_status dispatch_multi_np(const SimParams& p, uint32_t np, uint32_t blocks, uint32_t lds, hipStream_t s) {
  switch (np) {
    case 1: return launch_multi<IMG_LDS, PM, 1>(p, blocks, lds, s);
    case 2: return launch_multi<IMG_LDS, PM, 2>(p, blocks, lds, s);
    case 3: return launch_multi<IMG_LDS, PM, 3>(p, blocks, lds, s);
    default: return launch_multi<IMG_LDS, PM, 4>(p, blocks, lds, s);
  }
}

// Steps per Philox fill with K trajectories per wave: the f <= 32 with
// f K n_jobs <= 4 x 64 calls and f K <= 64 whose calls use the largest share
// of their rounds of 64 lanes (ties: the larger f).
uint32_t multi_fill_steps(uint32_t njobs, uint32_t K) {
  uint32_t best = 1;
  double best_use = 0.0;
  for (uint32_t f = 1; f <= 32 && f * K * njobs <= uint32_t(kFillRounds) * 64u && f * K <= 64u; ++f) {
    const uint32_t calls = f * K * njobs, rounds = (calls + 63u) / 64u;
    const double use = double(calls) / double(rounds * 64u);
    if (use >= best_use - 1e-12) {
      best = f;
      best_use = use;
    }
  }
  return best;
}

pbn_status simulate_common(bool plain, const pbn_plan* plan, const void* d_plan, uint64_t seed, uint32_t traj0,
                           uint32_t ntraj, uint32_t step0, uint32_t nsteps, uint32_t count_from,
                           const pbn_targets* targets, uint32_t* d_state, uint64_t* d_counts,
                           const pbn_launch_opts* launch, void* stream) {
  pbn::clear_error();
  if (!plan || !d_plan || !targets || (ntraj && (!d_state || !d_counts)))
    return fail(PBN_EINVAL, "null argument");
  if (uint64_t(traj0) + ntraj > (1ull << 32)) return fail(PBN_ERANGE, "trajectory ids exceed 32 bits");
  if (uint64_t(step0) + nsteps > 0xFFFFFFFFull) return fail(PBN_ERANGE, "step counter exceeds 32 bits");
  if (targets->ntargets < 1 || targets->ntargets > 64 || targets->npairs > PBN_MAX_PAIRS)
    return fail(PBN_EINVAL, "bad targets (build them with pbn_targets_build)");
  for (uint32_t k = 0; k < targets->npairs; ++k)
    if (targets->pos[k] >= plan->info.state_bytes) return fail(PBN_EINVAL, "target position outside the plan");
  if (plain && plan->has_table) return fail(PBN_EINVAL, "the plain kernel needs a plan without table slots");
  if (ntraj == 0 || nsteps == 0) return PBN_OK;

  const uint32_t tpw = launch && launch->traj_per_wave > 1u ? launch->traj_per_wave : 1u;
  if (tpw > 1u) {
    // several trajectories per wave: FN-only keyed plans of at most 4 passes
    // of K slot sets, without indicator recording
    const uint32_t nps = (tpw * plan->info.n_slots + 63u) / 64u;
    if (tpw > 4u || plan->sampling || plan->info.max_union_bits != 0 || (launch && launch->d_record) ||
        tpw * plan->n_jobs > 64u || nps > 4u || targets->ntargets * tpw > 64u)
      return fail(PBN_EINVAL, "traj_per_wave > 1 needs a keyed FN-only plan whose K slot sets fit 4 lane passes, "
                              "K n_jobs <= 64, K targets <= 64 and no recording (K <= 4)");
  }
  const pbn_plan_header* ph = reinterpret_cast<const pbn_plan_header*>(plan->blob.data());
  const bool bits = ph->state_bits != 0;
  if (bits && (tpw > 1u || (launch && launch->d_record)))
    return fail(PBN_EINVAL, "plans with the packed-bit state run one trajectory per wave without recording");
  const uint32_t mfill = tpw > 1u ? multi_fill_steps(plan->n_jobs, tpw) : 0u;
  // slot data of plans of one or two lane passes stay in registers, unless a
  // step needs more than 64 Philox jobs (then the streaming form runs them)
  const bool cached = plan->info.n_passes <= 2u && plan->n_jobs <= 64u;
  const uint32_t ring_bytes = 16u * (plan->n_jobs <= 64 ? std::min(plan->fill_steps, 32u) * plan->n_jobs : plan->n_jobs);
  const uint32_t wave_bytes = tpw > 1u ? tpw * 4u * ((plan->state_dwords + 3u) & ~3u) + 16u + 16u * mfill * tpw * plan->n_jobs
                              : bits   ? 8u * ((ph->state_words + 3u) & ~3u) + ring_bytes
                                       : wave_lds_bytes(plan, cached);
  const bool img_lds = plan->info.image_in_lds != 0;
  const uint32_t img = img_lds ? ((plan->info.image_bytes + 15u) & ~15u) : 0u;
  uint32_t wpb = launch && launch->waves_per_block ? launch->waves_per_block : 4u;
  if (launch && launch->d_record && launch->record_words == 0)
    return fail(PBN_EINVAL, "record_words must be positive when recording");
  if (wpb > 16) return fail(PBN_EINVAL, "waves_per_block must be 1..16");
  while (wpb > 1 && img + wpb * wave_bytes > kLdsMax) --wpb;
  if (img + wpb * wave_bytes > kLdsMax)
    return fail(PBN_ELDS, "one trajectory's state and ring do not fit in LDS");
  SimParams p{};
  p.blob = static_cast<const uint8_t*>(d_plan);
  p.state = d_state;
  p.counts = reinterpret_cast<unsigned long long*>(d_counts);
  p.seed = seed;
  p.traj0 = traj0;
  p.ntraj = ntraj;
  p.step0 = step0;
  p.nsteps = nsteps;
  p.count_from = count_from;
  p.wpb = wpb;
  p.wave_bytes = wave_bytes;
  p.gshift = 1;
  p.tpw = tpw;
  p.mfill = mfill;
  p.tg = *targets;
  if (launch && launch->d_record) {
    p.record = launch->d_record;
    p.record_traj = launch->record_traj;
    p.record_words = launch->record_words;
  }
  const uint32_t waves = (ntraj + tpw - 1) / tpw;
  const uint32_t blocks = (waves + wpb - 1) / wpb;
  const uint32_t lds = img + wpb * wave_bytes;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint32_t pmax = plan->info.max_fn_parents, umax = plan->info.max_union_bits;
  const uint32_t npass = plan->info.n_passes;
  if (pmax > 7 || umax > 16) return fail(PBN_ELDS, "plan exceeds the kernel's gather widths");
  const uint32_t units = reinterpret_cast<const pbn_plan_header*>(plan->blob.data())->fn_units;
  if (units != (pmax > 5 ? 2u : 1u)) return fail(PBN_EINVAL, "plan FN record format does not match its parent count");
  if (bits) {
    if (pmax <= 5)
      return img_lds ? dispatch_bits_um<true, 5>(p, umax, blocks, lds, s) : dispatch_bits_um<false, 5>(p, umax, blocks, lds, s);
    return img_lds ? dispatch_bits_um<true, 7>(p, umax, blocks, lds, s) : dispatch_bits_um<false, 7>(p, umax, blocks, lds, s);
  }
  if (tpw > 1u) {
    const uint32_t nps = (tpw * plan->info.n_slots + 63u) / 64u;
    if (pmax <= 5)
      return img_lds ? dispatch_multi_np<true, 5>(p, nps, blocks, lds, s) : dispatch_multi_np<false, 5>(p, nps, blocks, lds, s);
    return img_lds ? dispatch_multi_np<true, 7>(p, nps, blocks, lds, s) : dispatch_multi_np<false, 7>(p, nps, blocks, lds, s);
  }
  // one-pass FN-only keyed plans whose slot bytes and zero word lie below 64
  // keep the state in a register (padded lanes' bytes, above the zero word,
  // are never read and stay 0)
  const uint32_t zero_pos = reinterpret_cast<const pbn_plan_header*>(plan->blob.data())->zero_pos;
  const bool reg = cached && npass == 1 && umax == 0 && !plan->sampling && zero_pos + 4u <= 64u;
  const uint32_t nreg = cached ? npass : 0u;
  // does the last register-held pass select a predictor anywhere?
  const pbn_pass_info* pinfo = reinterpret_cast<const pbn_pass_info*>(plan->blob.data() + ph->pass_off);
  const bool lastsel = nreg == 0u || (pinfo[nreg - 1u].flags & PBN_PASS_MULTI) != 0u;
  if (plan->sampling)
    return img_lds ? dispatch_pm<true, true>(p, pmax, umax, nreg, true, false, blocks, lds, s)
                   : dispatch_pm<false, true>(p, pmax, umax, nreg, true, false, blocks, lds, s);
  return img_lds ? dispatch_pm<true, false>(p, pmax, umax, nreg, lastsel, reg, blocks, lds, s)
                 : dispatch_pm<false, false>(p, pmax, umax, nreg, lastsel, reg, blocks, lds, s);
}

}  // namespace

extern "C" pbn_status pbn_state_init(const pbn_plan* plan, const void* d_plan, uint64_t seed, uint32_t traj0,
                                     uint32_t ntraj, uint32_t* d_state, void* stream) {
  pbn::clear_error();
  if (!plan || !d_plan || (ntraj && !d_state)) return fail(PBN_EINVAL, "null argument");
  if (uint64_t(traj0) + ntraj > (1ull << 32)) return fail(PBN_ERANGE, "trajectory ids exceed 32 bits");
  if (ntraj == 0) return PBN_OK;
  const size_t work = size_t(ntraj) * plan->info.state_words;
  hipLaunchKernelGGL(k_state_init, dim3(grid_for(work, 256)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const uint8_t*>(d_plan), (unsigned long long)seed, traj0, ntraj, d_state);
  return hip_check(hipGetLastError(), "k_state_init launch");
}

extern "C" pbn_status pbn_simulate(const pbn_plan* plan, const void* d_plan, uint64_t seed, uint32_t traj0,
                                   uint32_t ntraj, uint32_t step0, uint32_t nsteps, uint32_t count_from,
                                   const pbn_targets* targets, uint32_t* d_state, uint64_t* d_counts,
                                   const pbn_launch_opts* launch, void* stream) {
  return simulate_common(false, plan, d_plan, seed, traj0, ntraj, step0, nsteps, count_from, targets, d_state,
                         d_counts, launch, stream);
}

extern "C" pbn_status pbn_simulate_plain(const pbn_plan* plan, const void* d_plan, uint64_t seed, uint32_t traj0,
                                         uint32_t ntraj, uint32_t step0, uint32_t nsteps, uint32_t count_from,
                                         const pbn_targets* targets, uint32_t* d_state, uint64_t* d_counts,
                                         const pbn_launch_opts* launch, void* stream) {
  return simulate_common(true, plan, d_plan, seed, traj0, ntraj, step0, nsteps, count_from, targets, d_state,
                         d_counts, launch, stream);
}

extern "C" pbn_status pbn_rl_run(const pbn_plan* plan, const void* d_plan, uint64_t seed, uint32_t traj,
                                  const pbn_targets* targets, uint32_t* d_state, uint64_t* d_counts,
                                  uint32_t* d_record, uint32_t record_words, double precision, double conf,
                                  double eps, uint32_t kmax, uint64_t initial_steps, uint64_t max_steps,
                                  const pbn_launch_opts* launch, pbn_rl_out* out, void* stream) {
  pbn::clear_error();
  if (!plan || !d_plan || !targets || !d_state || !d_counts || !d_record || !out || record_words == 0)
    return fail(PBN_EINVAL, "null argument");
  const uint64_t cap = std::min<uint64_t>(32ull * record_words, max_steps);
  if (cap >= 0xFFFFFFFFull) return fail(PBN_ERANGE, "max_steps must stay below 2^32");
  hipStream_t s = static_cast<hipStream_t>(stream);
  pbn_status st = hip_check(hipMemsetAsync(d_record, 0, 4ull * record_words, s), "hipMemsetAsync");
  if (st == PBN_OK)
    st = hip_check(hipMemsetAsync(d_counts, 0, 24ull * targets->ntargets, s), "hipMemsetAsync");
  if (st == PBN_OK) st = pbn_state_init(plan, d_plan, seed, traj, 1, d_state, stream);
  if (st != PBN_OK) return st;
  pbn_launch_opts lo{};
  if (launch) lo = *launch;
  lo.record_traj = 1;
  lo.record_words = record_words;
  lo.d_record = d_record;
  std::vector<uint32_t> host;
  uint64_t done = 0, want = std::max<uint64_t>(std::min(initial_steps, cap), 64);
  for (;;) {
    want = std::min(want, cap);
    while (done < want) {   // launches of at most 2^24 steps
      const uint32_t chunk = uint32_t(std::min<uint64_t>(want - done, 1ull << 24));
      st = simulate_common(plan->has_table == 0, plan, d_plan, seed, traj, 1, uint32_t(done), chunk, 0, targets,
                           d_state, d_counts, &lo, stream);
      if (st != PBN_OK) return st;
      done += chunk;
    }
    const size_t words = size_t((done + 31) / 32);
    host.resize(words);
    st = hip_check(hipMemcpyAsync(host.data(), d_record, 4 * words, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    if (st == PBN_OK) st = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (st == PBN_OK) st = pbn_rl_diagnose(host.data(), done, precision, conf, eps, kmax, out);
    if (st != PBN_OK) return st;
    const double need = out->burn_in + out->n_required;
    if (std::isfinite(need) && double(done) >= need) return PBN_OK;
    if (done >= cap)
      return fail(PBN_ERANGE, "the sample size the diagnosis asks for exceeds max_steps or the record buffer");
    // extend to the diagnosed burn-in + sample size (doubling while the chain
    // has not changed state yet)
    want = std::isfinite(need) ? std::max<uint64_t>(uint64_t(std::ceil(need)), done + 1) : 2 * done;
  }
}

extern "C" pbn_status pbn_skart_run(const pbn_plan* plan, const void* d_plan, uint64_t seed, uint32_t traj,
                                     const pbn_targets* targets, uint32_t* d_state, uint64_t* d_counts,
                                     uint32_t* d_record, uint32_t record_words, double precision, double conf,
                                     uint64_t max_steps, const pbn_launch_opts* launch, pbn_skart_out* out,
                                     void* stream) {
  pbn::clear_error();
  if (!plan || !d_plan || !targets || !d_state || !d_counts || !d_record || !out || record_words == 0)
    return fail(PBN_EINVAL, "null argument");
  *out = pbn_skart_out{};
  const uint64_t cap = std::min<uint64_t>(32ull * record_words, max_steps);
  if (cap >= 0xFFFFFFFFull) return fail(PBN_ERANGE, "max_steps must stay below 2^32");
  hipStream_t s = static_cast<hipStream_t>(stream);
  pbn_status st = hip_check(hipMemsetAsync(d_record, 0, 4ull * record_words, s), "hipMemsetAsync");
  if (st == PBN_OK)
    st = hip_check(hipMemsetAsync(d_counts, 0, 24ull * targets->ntargets, s), "hipMemsetAsync");
  if (st == PBN_OK) st = pbn_state_init(plan, d_plan, seed, traj, 1, d_state, stream);
  if (st != PBN_OK) return st;
  pbn_launch_opts lo{};
  if (launch) lo = *launch;
  lo.record_traj = 1;
  lo.record_words = record_words;
  lo.d_record = d_record;
  std::vector<uint32_t> host;
  uint64_t done = 0, want = 1280;   // the procedure's first sample
  for (;;) {
    if (want > cap) {
      out->n_required = want;
      return fail(PBN_ERANGE, "the procedure asks for more steps than max_steps or the record buffer");
    }
    while (done < want) {   // launches of at most 2^24 steps
      const uint32_t chunk = uint32_t(std::min<uint64_t>(want - done, 1ull << 24));
      st = simulate_common(plan->has_table == 0, plan, d_plan, seed, traj, 1, uint32_t(done), chunk, 0, targets,
                           d_state, d_counts, &lo, stream);
      if (st != PBN_OK) return st;
      done += chunk;
    }
    const size_t words = size_t((done + 31) / 32);
    host.resize(words);
    st = hip_check(hipMemcpyAsync(host.data(), d_record, 4 * words, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    if (st == PBN_OK) st = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (st == PBN_OK) st = pbn_skart_analyze(host.data(), done, precision, conf, out);
    if (st != PBN_OK || out->done) return st;
    want = std::max<uint64_t>(out->n_required, done + 1);
  }
}

extern "C" pbn_status pbn_state_to_original(const pbn_plan* plan, const void* d_plan, const uint32_t* d_state,
                                            uint32_t ntraj, uint32_t* d_out, void* stream) {
  pbn::clear_error();
  if (!plan || !d_plan || (ntraj && (!d_state || !d_out))) return fail(PBN_EINVAL, "null argument");
  if (ntraj == 0) return PBN_OK;
  const size_t work = size_t(ntraj) * ((plan->info.n + 31) / 32);
  hipLaunchKernelGGL(k_to_original, dim3(grid_for(work, 256)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<const uint8_t*>(d_plan), d_state, ntraj, d_out);
  return hip_check(hipGetLastError(), "k_to_original launch");
}

// ------------------------------------------------------------------ batches

struct pbn_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

struct BatchShape {
  uint32_t pm = 5, um = 0, wave_bytes = 0;
  uint32_t chain_bytes = 0;   // LDS copy of the largest network's chain tables
};

pbn_status batch_shape(const pbn_plan* const* plans, uint32_t nitems, BatchShape& sh) {
  for (uint32_t k = 0; k < nitems; ++k) {
    const pbn_plan* p = plans[k];
    if (!p) return fail(PBN_EINVAL, "null plan in batch");
    if (p->sampling) return fail(PBN_EINVAL, "alias-sampling plans are not supported by the batch entry points");
    if (reinterpret_cast<const pbn_plan_header*>(p->blob.data())->state_bits)
      return fail(PBN_EINVAL, "plans with the packed-bit state are not supported by the batch entry points");
    if (p->info.max_fn_parents > 7 || p->info.max_union_bits > 16)
      return fail(PBN_ELDS, "plan exceeds the kernel's gather widths");
    if (p->info.max_fn_parents > 5) sh.pm = 7;
    sh.um = std::max(sh.um, p->info.max_union_bits);
    sh.wave_bytes = std::max(sh.wave_bytes, wave_lds_bytes(p, false));
    sh.chain_bytes = std::max(sh.chain_bytes, chain_lds_bytes(reinterpret_cast<const pbn_plan_header*>(p->blob.data())->n));
  }
  sh.um = sh.um == 0 ? 0 : sh.um <= 8 ? 8 : 16;
  return PBN_OK;
}

// `sched`: the allocation-free launch's schedule arguments (items, nitems,
// step window; p.ctl and p.tasks point into the device array), or null.
struct NoAllocSched {
  uint32_t nitems, step0, nsteps, ntasks;
};

template <int PM, int UM>
pbn_status launch_batch_t(const BatchParams& p, uint32_t lds, hipStream_t s, const NoAllocSched* sched = nullptr) {
  int dev = 0, ncu = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_check(e, "batch device query");
  // the slot-record prefetch when every wave of the launch fits the chip at
  // four waves per SIMD (four SIMDs per CU)
  const uint64_t waves = uint64_t(sched ? sched->ntasks : p.ntasks) * p.wpb * p.wpt;
  auto* fn = p.wpt > 1u                     ? k_batch<PM, UM, true, true>
             : waves <= uint64_t(ncu) * 16u ? k_batch<PM, UM, true, false>
                                            : k_batch<PM, UM, false, false>;
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize, int(kLdsMax));
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, int(64u * p.wpb * p.wpt), lds);
  if (e != hipSuccess) return hip_check(e, "batch occupancy query");
  const uint32_t resident = uint32_t(std::max(1, per_cu) * std::max(1, ncu));
  const uint32_t blocks = std::max(1u, std::min(sched ? sched->ntasks : p.ntasks, resident));
  if (sched) {
    hipLaunchKernelGGL(k_noalloc_schedule, dim3(1), dim3(1024), 0, s, p.items, sched->nitems, p.wpb, sched->step0,
                       sched->nsteps, reinterpret_cast<uint32_t*>(p.ctl));
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(64u * p.wpb * p.wpt), lds, s, p, p.items);
  } else {
    hipLaunchKernelGGL(k_batch_begin, dim3(1), dim3(PBN_BATCH_QUEUES), 0, s, p.ctl, p.q, p.nq);
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(64u * p.wpb * p.wpt), lds, s, p, p.items);
    hipLaunchKernelGGL(k_batch_end, dim3(1), dim3(1), 0, s, p.ctl);
  }
  return hip_check(hipGetLastError(), "k_batch launch");
}

pbn_status batch_enqueue(const pbn_plan* const* plans, uint32_t nitems, const pbn_work* d_items,
                         const uint32_t* d_tasks, const uint32_t* d_task_first, uint32_t ntasks,
                         const uint32_t* queue_first, uint32_t nq, pbn_batch_ctl* d_ctl, uint32_t wpb,
                         uint32_t wpt, hipStream_t s, const NoAllocSched* sched = nullptr) {
  if (!plans || !d_items || !d_tasks || !d_task_first || !d_ctl) return fail(PBN_EINVAL, "null argument");
  if (wpb < 1 || wpb > 16) return fail(PBN_EINVAL, "waves_per_block must be 1..16");
  if (wpt < 1 || wpt > 16 || (wpt > 1 && wpb != 1))
    return fail(PBN_EINVAL, "waves_per_traj must be 1..16, with one trajectory per task when above 1");
  if (nitems == 0 || ntasks == 0) return PBN_OK;
  QueueBounds q{};
  if (sched || !queue_first) {
    // one queue (the allocation-free launch bounds it on the device by the
    // schedule's task count)
    nq = 1;
    q.first[1] = ntasks;
  } else {
    if (nq < 1 || nq > PBN_BATCH_QUEUES) return fail(PBN_EINVAL, "nqueues must be 1..PBN_BATCH_QUEUES");
    if (queue_first[0] != 0 || queue_first[nq] != ntasks)
      return fail(PBN_EINVAL, "queue bounds must run from 0 to ntasks");
    for (uint32_t k = 0; k <= nq; ++k) {
      if (k > 0 && queue_first[k] < queue_first[k - 1]) return fail(PBN_EINVAL, "queue bounds must not decrease");
      q.first[k] = queue_first[k];
    }
  }
  BatchShape sh;
  pbn_status st = batch_shape(plans, nitems, sh);
  if (st != PBN_OK) return st;
  // several waves per trajectory copy the chain tables into LDS; when those of
  // the batch's largest network do not fit beside its states and ring, the
  // launch runs one wave per trajectory (the same results)
  if (wpt > 1u && 16u + wpb * sh.wave_bytes + sh.chain_bytes > kLdsMax) wpt = 1u;
  const uint32_t lds = 16u + wpb * sh.wave_bytes + (wpt > 1u ? sh.chain_bytes : 0u);
  if (lds > kLdsMax) return fail(PBN_ELDS, "states and rings of one workgroup exceed LDS");
  BatchParams p{};
  p.items = d_items;
  p.tasks = d_tasks;
  p.task_first = d_task_first;
  p.ntasks = ntasks;
  p.wpb = wpb;
  p.wpt = wpt;
  p.wave_bytes = sh.wave_bytes;
  p.gshift = 1;
  p.ctl = d_ctl;
  p.nq = nq;
  p.q = q;
  if (sh.pm == 5) {
    if (sh.um == 0) return launch_batch_t<5, 0>(p, lds, s, sched);
    if (sh.um == 8) return launch_batch_t<5, 8>(p, lds, s, sched);
    return launch_batch_t<5, 16>(p, lds, s, sched);
  }
  if (sh.um == 0) return launch_batch_t<7, 0>(p, lds, s, sched);
  if (sh.um == 8) return launch_batch_t<7, 8>(p, lds, s, sched);
  return launch_batch_t<7, 16>(p, lds, s, sched);
}

}  // namespace

extern "C" pbn_status pbn_batch_tasks(const pbn_plan* const* plans, const uint32_t* ntraj, uint32_t nitems,
                                      uint32_t wpb, uint32_t nqueues, uint32_t* tasks, uint32_t* task_first,
                                      uint32_t* queue_first, uint32_t* ntasks) {
  pbn::clear_error();
  if (!plans || !ntraj || !ntasks || wpb < 1 || wpb > 16) return fail(PBN_EINVAL, "bad argument");
  if (nqueues < 1 || nqueues > PBN_BATCH_QUEUES) return fail(PBN_EINVAL, "nqueues must be 1..PBN_BATCH_QUEUES");
  // per-step cost of one trajectory: lane passes and Philox jobs, then slots
  std::vector<uint64_t> cost(nitems);
  std::vector<uint32_t> order(nitems);
  for (uint32_t k = 0; k < nitems; ++k) {
    if (!plans[k]) return fail(PBN_EINVAL, "null plan in batch");
    if (plans[k]->sampling) return fail(PBN_EINVAL, "alias-sampling plans are not supported by the batch entry points");
    cost[k] = uint64_t(plans[k]->info.n_passes) * plans[k]->n_jobs + plans[k]->info.n_slots;
    order[k] = k;
  }
  // largest networks first, so the tail of each queue is made of short tasks
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return cost[a] > cost[b]; });
  // each network, in that order, to the queue with the least work so far
  // (ties: the lowest queue)
  std::vector<uint32_t> queue_of(nitems, 0);
  uint64_t load[PBN_BATCH_QUEUES] = {};
  for (uint32_t k : order) {
    uint32_t best = 0;
    for (uint32_t j = 1; j < nqueues; ++j)
      if (load[j] < load[best]) best = j;
    queue_of[k] = best;
    load[best] += cost[k] * ((uint64_t(ntraj[k]) + wpb - 1) / wpb);
  }
  uint32_t count = 0;
  for (uint32_t j = 0; j < nqueues; ++j) {
    if (queue_first) queue_first[j] = count;
    for (uint32_t k : order) {
      if (queue_of[k] != j) continue;
      for (uint32_t f = 0; f < ntraj[k]; f += wpb) {
        if (tasks) tasks[count] = k;
        if (task_first) task_first[count] = f;
        ++count;
      }
    }
  }
  if (queue_first) queue_first[nqueues] = count;
  *ntasks = count;
  return PBN_OK;
}

extern "C" pbn_status pbn_batch_launch(const pbn_plan* const* plans, uint32_t nitems, const pbn_work* d_items,
                                       const uint32_t* d_tasks, const uint32_t* d_task_first, uint32_t ntasks,
                                       const uint32_t* queue_first, uint32_t nqueues, pbn_batch_ctl* d_ctl,
                                       uint32_t waves_per_block, uint32_t waves_per_traj, void* stream) {
  pbn::clear_error();
  return batch_enqueue(plans, nitems, d_items, d_tasks, d_task_first, ntasks, queue_first, nqueues, d_ctl,
                       waves_per_block, waves_per_traj, static_cast<hipStream_t>(stream));
}

namespace {

// Device address of this file's `scratch` array on the current device, taken
// once per device (each GPU holds its own copy).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices] = {};

pbn_status noalloc_scratch(uint32_t** out) {
  int dev = 0;
  pbn_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (st != PBN_OK) return st;
  if (dev < 0 || dev >= kMaxDevices) return fail(PBN_ELIMIT, "device index beyond the library's table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    st = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
    if (st != PBN_OK) return st;
    g_scratch_ptr[dev] = static_cast<uint32_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return PBN_OK;
}

}  // namespace

extern "C" pbn_status pbn_batch_launch_noalloc(const pbn_plan* const* plans, const uint32_t* ntraj, uint32_t nitems,
                                               const pbn_work* d_items, uint32_t step0, uint32_t nsteps,
                                               uint32_t waves_per_block, void* stream) {
  pbn::clear_error();
  if (!plans || !ntraj || !d_items) return fail(PBN_EINVAL, "null argument");
  if (waves_per_block < 1 || waves_per_block > 16) return fail(PBN_EINVAL, "waves_per_block must be 1..16");
  if (nitems > kNoAllocMaxItems)
    return fail(PBN_ELIMIT, "nitems = " + std::to_string(nitems) + " exceeds the allocation-free launch's " +
                                std::to_string(kNoAllocMaxItems));
  if (uint64_t(step0) + nsteps > 0xFFFFFFFFull) return fail(PBN_ERANGE, "step counter exceeds 32 bits");
  uint64_t total = 0;
  for (uint32_t k = 0; k < nitems; ++k) total += (uint64_t(ntraj[k]) + waves_per_block - 1) / waves_per_block;
  if (total > kNoAllocMaxTasks)
    return fail(PBN_ELIMIT, "the batch needs " + std::to_string(total) + " tasks; the allocation-free launch holds " +
                                std::to_string(kNoAllocMaxTasks) + " (raise waves_per_block or split the batch)");
  if (nitems == 0 || total == 0 || nsteps == 0) return PBN_OK;
  uint32_t* scr = nullptr;
  pbn_status st = noalloc_scratch(&scr);
  if (st != PBN_OK) return st;
  const NoAllocSched sched{nitems, step0, nsteps, uint32_t(total)};
  return batch_enqueue(plans, nitems, d_items, scr + kScratchCtlWords, scr + kScratchCtlWords + kNoAllocMaxTasks,
                       PBN_NONE, nullptr, 1, reinterpret_cast<pbn_batch_ctl*>(scr), waves_per_block, 1,
                       static_cast<hipStream_t>(stream), &sched);
}

extern "C" pbn_status pbn_batch_graph_create(const pbn_plan* const* plans, uint32_t nitems, const pbn_work* d_items,
                                             const uint32_t* d_tasks, const uint32_t* d_task_first, uint32_t ntasks,
                                             const uint32_t* queue_first, uint32_t nqueues, pbn_batch_ctl* d_ctl,
                                             uint32_t waves_per_block, uint32_t waves_per_traj, uint32_t passes,
                                             pbn_graph** out) {
  pbn::clear_error();
  if (!out || passes == 0) return fail(PBN_EINVAL, "bad argument");
  *out = nullptr;
  hipStream_t s = nullptr;
  pbn_status st = hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreateWithFlags");
  if (st != PBN_OK) return st;
  st = hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  if (st == PBN_OK) {
    for (uint32_t k = 0; k < passes && st == PBN_OK; ++k)
      st = batch_enqueue(plans, nitems, d_items, d_tasks, d_task_first, ntasks, queue_first, nqueues, d_ctl,
                         waves_per_block, waves_per_traj, s);
    hipGraph_t g = nullptr;
    const pbn_status end = hip_check(hipStreamEndCapture(s, &g), "hipStreamEndCapture");
    if (st == PBN_OK) st = end;
    if (st == PBN_OK) {
      auto* pg = new pbn_graph;
      pg->graph = g;
      st = hip_check(hipGraphInstantiate(&pg->exec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
      if (st == PBN_OK)
        *out = pg;
      else {
        (void)hipGraphDestroy(g);
        delete pg;
      }
    } else if (g) {
      (void)hipGraphDestroy(g);
    }
  }
  (void)hipStreamDestroy(s);
  return st;
}

extern "C" pbn_status pbn_graph_launch(pbn_graph* g, void* stream) {
  pbn::clear_error();
  if (!g || !g->exec) return fail(PBN_EINVAL, "null graph");
  return hip_check(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)), "hipGraphLaunch");
}

extern "C" pbn_status pbn_graph_destroy(pbn_graph* g) {
  if (!g) return PBN_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return PBN_OK;
}
