// plan_format.h -- device blob of a prepared PBN (the output of Algorithm 5's
// Preparation, laid out for the step kernel).  Shared by the host builder and
// the HIP kernels; plain C layout, little-endian, every section 16-byte aligned.
//
// Step-kernel model: one wavefront simulates one trajectory.  The kept nodes
// are packed into "slots": a slot is either one node evaluated through its
// selected predictor function (FN slot) or a group of up to 4 nodes evaluated
// through one combined table (TABLE slot, Section 3.3).  Slot s is handled by
// lane s % 64 in pass s / 64; table slots come first.  The trajectory state
// lives in LDS as one byte per node value (0/1): table slot s (s < n_table)
// owns the word at byte 4 s (member k at byte k), FN slot s owns the byte at
// fn_base + (s - n_table); the zero word read by unused parent entries
// follows at zero_pos (the first 4-aligned byte after the last FN slot);
// padded lanes own bytes after it that only ever hold zeros.  Packed states in
// HBM use bit b for state byte b.
#pragma once
#include <stdint.h>

#define PBN_PLAN_MAGIC 0x314E4250u   // "PBN1"
#define PBN_WAVE 64
// A fill of the Philox ring computes fill_steps steps' calls in at most this
// many rounds of PBN_WAVE calls (fill_steps <= 32).
#define PBN_FILL_ROUNDS 4
#define PBN_NONE 0xFFFFFFFFu

// streams of the random-number contract
#define PBN_STREAM_INIT 1u
#define PBN_STREAM_PERT 2u
#define PBN_STREAM_SEL 3u

// slot-record info word
#define PBN_SLOT_VALID 0x80000000u
#define PBN_SLOT_TABLE 0x40000000u
// bits 0-2: number of members - 1; bits 3-5: multi-predictor members;
// bits 6-10: number of union parent bits (TABLE) / parent entries (FN, max over l)
#define PBN_SLOT_NMEM(i) (((i) & 7u) + 1u)
#define PBN_SLOT_NMULTI(i) (((i) >> 3) & 7u)
#define PBN_SLOT_NU(i) (((i) >> 6) & 31u)
// TABLE slot without multi-predictor members and with at most 5 union bits:
// its union positions sit in the slot record itself (z = p0 | p1 << 16,
// w = p2 | p3 << 16, info bits 11-26 = p4; the zero position where the union
// has fewer bits), so a lane pass reads no union list
#define PBN_SLOT_INLINE 0x20000000u
#define PBN_SLOT_P4(i) (((i) >> 11) & 0xFFFFu)

// pass-info flags
#define PBN_PASS_FN 1u
#define PBN_PASS_TABLE 2u
#define PBN_PASS_MULTI 4u

struct pbn_plan_header {
  uint32_t magic, version, blob_bytes, plan_id;
  uint32_t n;              // original nodes
  uint32_t n_kept;
  uint32_t n_slots;
  uint32_t n_passes;
  uint32_t state_dwords;   // LDS state buffer in words = 8 * state_words
  uint32_t state_words;    // packed words per trajectory = ceil((zero_pos + 4) / 32)
  uint32_t n_jobs;         // Philox calls per step: 1 + SEL blocks with a kept member
                           // (alias sampling: ceil((2 + 2 alias_g + n_sel) / 4))
  uint32_t fill_steps;     // steps whose jobs are computed per fill (n_jobs <= 64): the f <= 32
                           // with f n_jobs <= R * 64 that uses the most lanes of its rounds
                           // (ties: the larger f); R = PBN_FILL_ROUNDS for plans of <= 2
                           // lane passes, else 1
  uint32_t image_bytes;    // bytes of the image (slot, choice, fn records, tables)
  uint32_t image_off;      // blob offset of the image
  uint32_t q_off;          // blob offset of Q[0..n] (uint64)
  uint32_t o2p_off;        // blob offset of orig -> byte position (uint32[n])
  uint32_t p2o_off;        // blob offset of byte position -> orig (uint32[32 state_words])
  uint32_t blk_off;        // blob offset of SEL block ids (uint32[n_jobs - 1])
  uint32_t pass_off;       // blob offset of pass info (pbn_pass_info[n_passes])
  uint32_t zero_pos;       // byte position of the zero word
  uint32_t max_pmax;       // largest parent-entry count over all passes
  uint32_t image_in_lds;
  uint32_t has_table;
  uint32_t dummy_fn;       // image offset of an all-zero-position FN record (padded lanes)
  uint32_t n_table;        // table slots (slots 0 .. n_table - 1)
  uint32_t fn_base;        // byte position of the first FN slot (4 n_table)
  uint32_t fn_units;       // 16-byte units per FN record: 1 (<= 5 parents) or 2 (<= 7)
  uint32_t fn_jshift;      // log2 of the bytes from an FN slot's record of predictor j to j + 1
  uint32_t fn_hoff;        // bytes from a two-unit record's first unit to its second
  uint32_t sampling;       // 0 keyed draws; 1 alias sampling (the fields below)
  uint32_t q_img;          // image offset of a copy of Q[0..n] (uint64): read by the
                           // perturbation chain from wherever the image resides
  uint32_t o2p_img;        // image offset of a copy of the orig -> position map
  // alias sampling (Algorithms 1-2, Sections 2.2 / 3.2 / 3.3)
  uint32_t pert_off;       // blob offset of the pattern table: 2^alias_k entries {keep threshold, alias}
  uint32_t kpos_off;       // blob offset of kept-node byte positions (original-id order), n_kept entries
  uint32_t alias_k;        // nodes per perturbation group (Algorithm 2's k)
  uint32_t alias_g;        // groups
  uint32_t alias_kp;       // nodes of the last group (k')
  uint32_t leaf_thr;       // Algorithm 1: a leaf is perturbed when the drawn word exceeds this
  uint32_t n_sel;          // slots that draw a (combined) predictor function
  uint32_t fn_var;         // 1: packed two-unit plan whose slots with <= 5 parents keep one-unit
                           // records (predictor stride 16 units of the slot)
  uint32_t state_bits;     // 1: positions are bit indices of a packed state of pass segments
                           // (256 bits for a pass holding a table slot: lane L's member k at
                           // 4 L + k; else 64 bits: lane L at L), the zero word after the last
                           // segment; 0: byte positions (the layout described above)
};
// Alias sampling draws, per step t: Philox(traj, t, c, PBN_STREAM_ALIAS) for
// c = 0 .. n_jobs-1 give words w[0 .. 4 n_jobs) (word e of call c is w[4c+e]):
//   w[0]               Algorithm 1: a removed leaf is perturbed when w[0] > leaf_thr
//   w[1]               not drawn from (the kernel keeps the step's perturbed flag here)
//   w[2+2q], w[3+2q]   group q's pattern (Algorithm 2): column = the top alias_k
//                      bits of the first word, kept when the second word is below
//                      the column's threshold, else its alias; the last group's
//                      pattern is ANDed with the mask of its alias_kp low bits;
//                      bit b flips kept node q alias_k + b (original-id order)
//   w[2+2g+s]          selecting slot s (numbered by smallest member id): column =
//                      high word of w * L, kept when the low word is below the
//                      column's threshold, else its alias
// Tables come from Vose's construction in double; threshold = floor(keep 2^32),
// at most 2^32 - 1.
#define PBN_STREAM_ALIAS 4u

struct pbn_pass_info {
  uint32_t flags;   // PBN_PASS_*
  uint32_t pmax;    // parent entries to gather in FN slots of this pass
  uint32_t umax;    // union bits to gather in TABLE slots of this pass
  uint32_t mmax;    // multi-predictor members of TABLE slots in this pass
};

// Image sections (offsets relative to the image base):
//   [0, 16 * 64 * n_passes)  slot records (uint4 each)
//   choice records (uint4):   x = draw byte offset within a step's ring segment
//                                 | (l << 24);  y, z, w = thresholds CUM[0..2]
//                                 (unused = 0xFFFFFFFF); the first one is the
//                                 default record {0 | 1 << 24, unused x 3}
//   fn records (from a 128-byte aligned offset): fn_units 16-byte units each.
//     one unit  (every FN slot <= 5 parents): parent byte positions as 6
//               uint16 (unused = zero position), then the 32-bit truth table
//     two units (<= 7 parents): 8 uint16 positions; the second unit, fn_hoff
//               bytes later, holds the 128-bit truth table
//     Predictor j of a slot sits j << fn_jshift bytes after predictor 0.  An
//     image staged in LDS keeps slot s in unit 16 (s mod 8) of 128-byte rows
//     (stride 128 fn_units, fn_hoff = 128: lanes of one 16-byte read
//     hit distinct banks); otherwise records are packed (16 fn_units, 16).
//     The dummy records (all positions the zero word, table 0) come first.
//   tables:                   TABLE slot: 16 uint16 union-parent positions
//                             (unused = zero position), then the byte table
//                             T[c * 2^nu + x]; a PBN_SLOT_INLINE slot has the
//                             table alone (its positions are in its record)
//   alias records (alias sampling only, see below)
//   Q[0..n] (uint64) and the orig -> position map (uint32[n]), copies of the
//   blob's, at q_img / o2p_img
// Padded lanes (slot index >= n_slots) have info = 0, y = a dummy FN record,
// z = the default choice record and w = a state byte of their own above the
// zero word: they evaluate to 0 and write only that byte.
// Slot record (uint4):
//   x = info word (PBN_SLOT_*)
//   y = FN: image offset of the fn record of predictor 0 (predictor j at +32 j)
//       TABLE: image offset of the union-parent list (table follows at +32);
//       with PBN_SLOT_INLINE the offset of the table itself (the positions
//       are in z, w and the info word)
//   z = FN: image offset of the slot's choice record (one-predictor nodes and
//       padded lanes: the default record {ring offset 0, l = 1, no thresholds},
//       the first choice record of the image);
//       TABLE: offset of the first choice record of its multi-predictor members
//       (in member order), or 0
// With alias sampling, z of a selecting slot (a multi-predictor FN slot or a
// TABLE slot with multi-predictor members) is the image offset of its alias
// record: {byte offset of its word w[2+2g+s] in a step's draws, L, s, 0}, then
// L entries {threshold, alias} of 8 bytes; the outcome is the predictor j (FN)
// or the combined index c (TABLE).  Other slots keep the keyed-mode z.
//   w = TABLE: mixed-radix weights of the multi-predictor members, one byte
//       each (first member most significant digit); FN / padded lane: the
//       state byte the slot writes
