/*
 * pbn.h -- C ABI of the MI355X probabilistic Boolean network (PBN) simulator.
 *
 * Method: Mizera, Pang, Yuan, "Fast Simulation of Probabilistic Boolean
 * Networks" (arXiv:1605.00854).  The library simulates long trajectories of an
 * independent-synchronous PBN with perturbations (Section 2.1, Eq. 1) after the
 * paper's structure-based preparation: leaf-node reduction (Section 3.1,
 * Definition 1) and node grouping into combined predictor functions
 * (Section 3.3, Algorithms 3-4), assembled as in Algorithm 5.  Hit counters of
 * queried state sets feed the steady-state estimate (Section 4.2).
 *
 * Conventions
 *   - Every call returns pbn_status: PBN_OK (0) or a negative error code.
 *     pbn_last_error() returns a thread-local message for the last failure.
 *     No C++ exception or abort crosses this boundary.
 *   - Host arrays passed in are owned by the caller and copied; the library
 *     keeps no pointer to them after the call returns.
 *   - Opaque objects (pbn_net, pbn_plan) are owned by the library and freed by
 *     the matching *_destroy call (destroying NULL is a no-op).
 *   - Device buffers (d_*) are allocated by the caller on the current HIP
 *     device and passed as raw device pointers.  `stream` is a hipStream_t
 *     (NULL = legacy default stream).  Device calls only enqueue work; they do
 *     not synchronise.  Launch errors are reported through the return code.
 *
 * Random-number contract (the paper leaves the generator unspecified; this
 * fixed reading makes every trajectory a pure function of (seed, trajectory)):
 *   Philox4x32-10 with key = seed and counter (trajectory, step, index, stream),
 *   streams INIT = 1, PERT = 2, SEL = 3.  Perturbations of all n original nodes
 *   are drawn by a geometric skip chain over the integer table
 *   Q[h] = floor(v_h 2^64), v_h = fl(v_{h-1} fl(1 - p)); predictor selection of a
 *   node with l >= 2 predictors uses word (r & 3) of the SEL call with index
 *   r >> 2 (r = its rank among multi-predictor nodes of the full network)
 *   against thresholds CUM[m] = min(2^32, floor(S_m 2^32 + 1/2)) (2^32 is never
 *   reached: a predictor of probability 0 after a partial sum of 1 never fires).
 *   Reduction and grouping never change a kept node's trajectory.
 */
#ifndef PBN_H
#define PBN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pbn_status;

#define PBN_OK        0
#define PBN_EINVAL   -1   /* bad argument or malformed network                  */
#define PBN_ENOMEM   -2   /* host allocation failed                             */
#define PBN_ELIMIT   -3   /* input exceeds a documented limit of this library   */
#define PBN_ELDS     -4   /* plan cannot be laid out within the device limits   */
#define PBN_EHIP     -5   /* a HIP runtime call or kernel launch failed         */
#define PBN_ERANGE   -6   /* step or trajectory counter would overflow 32 bits  */
#define PBN_ENODEV   -7   /* no HIP device                                      */

/* Library limits. */
#define PBN_MAX_NODES          16000   /* nodes per network                      */
#define PBN_MAX_PREDICTORS         4   /* predictor functions per node, l(i)     */
#define PBN_MAX_FN_PARENTS        16   /* parents of one predictor function      */
#define PBN_MAX_GROUP_NODES        4   /* nodes per combined group               */
#define PBN_MAX_GROUP_PARENTS     16   /* parent bits indexing one group table   */
#define PBN_MAX_PAIRS             64   /* (node, value) pairs over all targets   */

/* Last error message of the calling thread ("" if none). */
const char* pbn_last_error(void);

/* ------------------------------------------------------------------ network
 * A PBN G(X, F) (Section 2.1): n binary nodes; node i has l(i) >= 1 predictor
 * functions with selection probabilities summing to 1; each predictor reads
 * its own ordered parent list; every node flips with probability p per step.
 *
 *   n          number of nodes, 1 .. PBN_MAX_NODES
 *   p          perturbation rate, 0 < p < 1 with 1 - p < 1 in double
 *   fn_off     [n+1]  predictors of node i are fn_off[i] .. fn_off[i+1]-1;
 *                     fn_off[0] = 0, 1 <= l(i) <= PBN_MAX_PREDICTORS
 *   sel_prob   [NF]   selection probabilities, finite, >= 0, per-node sum
 *                     within 1e-9 of 1 (NF = fn_off[n])
 *   par_off    [NF+1] parents of predictor f are parents[par_off[f] .. par_off[f+1]-1]
 *                     (0 .. PBN_MAX_FN_PARENTS of them)
 *   parents    node ids < n; parent k is bit k of the truth-table index
 *   tt_off     [NF+1] truth table of f is tt[tt_off[f] .. tt_off[f+1]-1], exactly
 *                     max(1, 2^phi / 64) 64-bit words for phi parents
 *   tt         LSB-first: the output for index j is bit (j % 64) of word j / 64;
 *                     bits at or above 2^phi must be zero
 * Errors: PBN_EINVAL (any rule above), PBN_ELIMIT (a limit), PBN_ENOMEM.
 * The integer quantisation of p and of the selection probabilities is done
 * here, once.
 */
typedef struct pbn_desc {
  uint32_t n;
  double p;
  const uint32_t* fn_off;
  const double* sel_prob;
  const uint32_t* par_off;
  const uint32_t* parents;
  const uint32_t* tt_off;
  const uint64_t* tt;
} pbn_desc;

typedef struct pbn_net pbn_net;
typedef struct pbn_plan pbn_plan;

pbn_status pbn_net_create(const pbn_desc* desc, pbn_net** out);
pbn_status pbn_net_destroy(pbn_net* net);

/* Integer tables of the random-number contract, for inspection and tests.
 *   q      [n+1] Q[h] for h = 0..n (Q[0] = 0: the certain event, never compared)
 *   cum    [3 n] thresholds of node i at cum[3 i + m], m < l(i) - 1, each at
 *                most 2^32 (2^32: never reached, the predictors after it have
 *                probability 0); the unused entries are 2^32
 *   rank   [n]   rank among nodes with >= 2 predictors, or -1                  */
pbn_status pbn_net_tables(const pbn_net* net, uint64_t* q, uint64_t* cum, int32_t* rank);

/* --------------------------------------------------------------------- plan
 * Preparation (Algorithm 5): leaf-node reduction (Definition 1), node grouping
 * (Equation 2, Algorithm 3, Algorithm 4, and grouping of single-predictor
 * nodes by shared parents, Section 3.3), combined predictor tables, and the
 * device layout.  `interest` lists the nodes of interest (every node a query
 * will read); they are never removed.
 *
 * Options:
 *   reduce             1: remove leaf nodes (Definition 1; their
 *                      perturbations still force a perturbation-only step, as
 *                      Algorithm 1 requires); 2: remove every node from which
 *                      no node of interest is reachable (the same argument
 *                      applied to whole regions, cycles included; a superset
 *                      of the leaves, same perturbation handling); 0: none
 *   group              1: group nodes into combined tables; 0: one predictor
 *                      evaluation per node
 *   weight_mode        weight of a multi-predictor node in Algorithms 3-4:
 *                      0 = l(i) (number of predictor functions, as in the paper),
 *                      1 = l(i) * 2^|P_i| (entries of its table over the union
 *                      P_i of its parents), so theta bounds table entries
 *   theta              Algorithm 4 limit on the sum over groups of the product
 *                      of member weights
 *   lds_budget_bytes   bytes of plan image (records + tables) that may be
 *                      staged in LDS; larger images stay in global memory
 *   max_table_entries  cap on (product of l) * 2^|union parents| per group
 *   max_parent_bits    cap on |union parents| per group (<= PBN_MAX_GROUP_PARENTS)
 *   max_group_nodes    cap on nodes per group (<= PBN_MAX_GROUP_NODES)
 *   sampling           0: the keyed draws (perturbation chain over all n
 *                      nodes, one selection word per multi-predictor node:
 *                      trajectories bit-identical whatever the reduction and
 *                      grouping); 1: the paper's sampling (Algorithm 1's leaf
 *                      draw, Algorithm 2's group perturbation through one alias
 *                      table of 2^k patterns, k <= 16, and one alias draw per
 *                      selecting slot over its (combined) predictor functions,
 *                      Sections 2.2, 3.2, 3.3): same distribution, different
 *                      draws; not supported by the batch entry points
 * Errors: PBN_EINVAL (bad node id, bad option), PBN_ELIMIT (a node needs a
 * table larger than max_table_entries), PBN_ELDS (layout exceeds device
 * limits), PBN_ENOMEM.
 */
typedef struct pbn_plan_opts {
  uint32_t reduce;
  uint32_t group;
  uint32_t weight_mode;
  uint32_t lds_budget_bytes;
  uint64_t theta;
  uint32_t max_table_entries;
  uint32_t max_parent_bits;
  uint32_t max_group_nodes;
  uint32_t sampling;
  uint32_t state_bits;  /* 0: one LDS byte per node while simulating; 1: packed
                           bits (keyed draws only): lane pass p owns a segment of
                           256 bits (4 per lane) when it holds a table slot, else
                           64 (1 per lane); the step kernel reads parents as bits
                           and writes each pass's results as whole words */
  uint32_t reserved;
} pbn_plan_opts;

/* Defaults: reduce = 1, group = 1, weight_mode = 1, theta = 65536,
 * lds_budget_bytes = 65536, max_table_entries = 4096, max_parent_bits = 12,
 * max_group_nodes = 4, sampling = 0, state_bits = 0. */
void pbn_plan_opts_default(pbn_plan_opts* opts);

pbn_status pbn_plan_build(const pbn_net* net, const uint32_t* interest, uint32_t n_interest,
                          const pbn_plan_opts* opts, pbn_plan** out);
pbn_status pbn_plan_destroy(pbn_plan* plan);

typedef struct pbn_plan_info {
  uint32_t n;               /* nodes of the original network                    */
  uint32_t n_kept;          /* nodes after reduction (n')                        */
  uint32_t n_slots;         /* evaluation slots: groups + single-node slots      */
  uint32_t n_table_slots;   /* slots evaluated through a combined table          */
  uint32_t n_passes;        /* ceil(n_slots / 64): lane passes per step          */
  uint32_t state_words;     /* 32-bit words of one packed trajectory state       */
  uint32_t n_jobs;          /* Philox calls per unperturbed step (1 + SEL blocks)*/
  uint32_t image_bytes;     /* records + tables read by the step kernel          */
  uint32_t table_bytes;     /* combined tables within the image                  */
  uint32_t image_in_lds;    /* 1 if the image is staged in LDS                   */
  uint32_t blob_bytes;      /* size of the exported device blob                  */
  uint32_t max_fn_parents;  /* largest parent count of a predictor in FN slots   */
  uint32_t max_union_bits;  /* largest |union parents| of a table slot           */
  uint32_t n_multi_groups;  /* groups holding >= 2 multi-predictor nodes         */
  uint32_t state_bytes;     /* LDS bytes of one trajectory state buffer          */
  uint32_t reserved[5];
} pbn_plan_info;

pbn_status pbn_plan_info_get(const pbn_plan* plan, pbn_plan_info* info);

/* Bit position of every original node in the packed plan state, or
 * 0xFFFFFFFF for a removed leaf.  pos: [n]. */
pbn_status pbn_plan_node_pos(const pbn_plan* plan, uint32_t* pos);

/* Slot of every original node (0xFFFFFFFF for leaves) and whether the slot is
 * evaluated through a combined table.  slot: [n], is_table: [n_slots]. */
pbn_status pbn_plan_slots(const pbn_plan* plan, uint32_t* slot, uint32_t* is_table);

/* Groups found by Algorithm 4 on the multi-predictor kept nodes, before any
 * device-limit split: flat member list and offsets (ngroups + 1 entries).
 * Call with NULL buffers to query the sizes. */
pbn_status pbn_plan_alg4_groups(const pbn_plan* plan, uint32_t* members, uint32_t* n_members,
                                uint32_t* offsets, uint32_t* n_groups);

/* Same for the grouping of single-predictor kept nodes by shared parents. */
pbn_status pbn_plan_single_groups(const pbn_plan* plan, uint32_t* members, uint32_t* n_members,
                                  uint32_t* offsets, uint32_t* n_groups);

/* Equation 2: smallest m >= 1 with m * (prod w)^(1/m) <= theta, or 0 when no m
 * satisfies it.  weights: [count] positive integers. */
pbn_status pbn_eq2_lower_bound(const uint64_t* weights, uint32_t count, uint64_t theta,
                               uint32_t* m_out);

/* Copy the device blob of the plan into host_buf.  *bytes: in = capacity,
 * out = size written (call with host_buf = NULL to query the size).  The
 * caller uploads the blob into device memory it owns and passes that pointer
 * as d_plan to the device calls below, together with the host plan. */
pbn_status pbn_plan_export(const pbn_plan* plan, void* host_buf, size_t* bytes);

/* ------------------------------------------------------------------ targets
 * Target state sets (queried steady-state events): target t is the
 * conjunction "node_k == value_k" over its pairs.  Built from original node
 * ids; every node must be kept by the plan (list it as of interest).
 *   node, value, target_of   [npairs] pair k belongs to target target_of[k]
 *   ntargets                 1 .. 64; npairs <= PBN_MAX_PAIRS
 * Errors: PBN_EINVAL (removed node, value not 0/1, empty target, bad counts). */
typedef struct pbn_targets {
  uint32_t ntargets;
  uint32_t npairs;
  uint32_t pos[PBN_MAX_PAIRS];    /* byte position of the pair's node in the step state */
  uint32_t val[PBN_MAX_PAIRS];
  uint64_t mask[64];              /* pairs of target t */
} pbn_targets;

pbn_status pbn_targets_build(const pbn_plan* plan, const uint32_t* node, const uint32_t* value,
                             const uint32_t* target_of, uint32_t npairs, uint32_t ntargets,
                             pbn_targets* out);

/* ----------------------------------------------------------- device calls
 * d_plan    device copy of pbn_plan_export(plan); must stay alive until the
 *           enqueued work completes
 * seed      64-bit Philox key
 * traj0     id of the first trajectory; trajectories traj0 .. traj0+ntraj-1
 * d_state   [ntraj][state_words] packed states in plan layout (bit = node at
 *           pbn_plan_node_pos), read and written in place
 *
 * pbn_state_init: s(0) of every trajectory from the INIT stream.
 * Errors: PBN_EINVAL, PBN_ERANGE (traj0 + ntraj > 2^32), PBN_EHIP.
 */
pbn_status pbn_state_init(const pbn_plan* plan, const void* d_plan, uint64_t seed, uint32_t traj0,
                          uint32_t ntraj, uint32_t* d_state, void* stream);

/* Launch tunables (0 = library choice) and optional recording of the hit
 * indicator of target 0 for the Raftery-Lewis diagnosis:
 *   d_record      device [record_traj][record_words] uint32, caller-owned and
 *                 zeroed by the caller; trajectory tl < record_traj of the
 *                 launch ORs bit (t - count_from) with z(t) = [s(t+1) in target
 *                 0] for steps count_from <= t < count_from + 32 record_words
 *                 (word w bit b = step count_from + 32 w + b).  NULL: none.
 * Errors: PBN_EINVAL when d_record is set and record_words is 0. */
typedef struct pbn_launch_opts {
  uint32_t waves_per_block;       /* wavefronts per workgroup, 1 .. 16        */
  uint32_t record_traj;
  uint32_t record_words;
  uint32_t traj_per_wave;         /* 0 or 1: one trajectory per wavefront;
                                     2 .. 4: that many trajectories share a
                                     wavefront's lane passes (keyed FN-only
                                     plans whose K slot sets fit 4 passes of
                                     64 lanes, K n_jobs <= 64, K targets <= 64,
                                     no recording; PBN_EINVAL otherwise).
                                     Results are identical for every value. */
  uint32_t* d_record;
} pbn_launch_opts;

/* pbn_simulate: advance every trajectory by nsteps transitions of Eq. 1,
 * global steps step0 .. step0+nsteps-1 (Algorithm 5's ParallelSimulation per
 * step), and accumulate per-target counters of the states reached:
 *   d_counts [ntargets][ntraj][3] uint64, added to (not overwritten):
 *     [0] hits: transitions t >= count_from whose result s(t+1) is in the target
 *     [1] 0->1 and [2] 1->0 changes of the hit indicator between consecutive
 *         counted states (t >= count_from + 1), for the two-state chain estimate.
 * Chunked calls (step0 advancing) give the same bits as one call.
 * Errors: PBN_EINVAL, PBN_ERANGE (step0 + nsteps >= 2^32), PBN_EHIP. */
pbn_status pbn_simulate(const pbn_plan* plan, const void* d_plan, uint64_t seed, uint32_t traj0,
                        uint32_t ntraj, uint32_t step0, uint32_t nsteps, uint32_t count_from,
                        const pbn_targets* targets, uint32_t* d_state, uint64_t* d_counts,
                        const pbn_launch_opts* launch, void* stream);

/* The plain per-node kernel (the paper's Method_old when the plan was built
 * with reduce = 0 and group = 0; Method_reduction with reduce = 1): same
 * contract, a step kernel compiled without combined-table evaluation.
 * Errors as pbn_simulate, and PBN_EINVAL if the plan holds table slots. */
pbn_status pbn_simulate_plain(const pbn_plan* plan, const void* d_plan, uint64_t seed,
                              uint32_t traj0, uint32_t ntraj, uint32_t step0, uint32_t nsteps,
                              uint32_t count_from, const pbn_targets* targets, uint32_t* d_state,
                              uint64_t* d_counts, const pbn_launch_opts* launch, void* stream);

/* Unpack plan-layout states to original node order: d_out [ntraj][ceil(n/32)]
 * words, bit i = node i; removed leaves read 0. */
pbn_status pbn_state_to_original(const pbn_plan* plan, const void* d_plan, const uint32_t* d_state,
                                 uint32_t ntraj, uint32_t* d_out, void* stream);

/* ---------------------------------------------------------------- estimate
 * Steady-state estimate of one target from per-unit counters (host, double
 * precision).  A unit is one trajectory, or one batch of one long trajectory
 * (batch means); every unit counted `steps_per_unit` states.
 *   counts   [units][3] as written by pbn_simulate for one target (hits, 0->1, 1->0)
 *   p_hat        sum hits / (units * steps_per_unit)
 *   half_width   t quantile (1 + conf) / 2 with units - 1 degrees of freedom times
 *                sd(unit means) / sqrt(units); NaN for one unit
 *   alpha, beta  two-state chain of the hit indicator: 0->1 changes per visit of
 *                state 0 and 1->0 changes per visit of state 1 (pooled over units)
 *   n_required   the two-state chain approach's sample size for precision
 *                `precision` at confidence `conf`:
 *                alpha beta (2 - alpha - beta) / (alpha + beta)^3 (z / precision)^2
 *   burn_in      log(1e-3 (alpha + beta) / max(alpha, beta)) / log|1 - alpha - beta|
 * Errors: PBN_EINVAL. */
typedef struct pbn_estimate_out {
  double p_hat;
  double half_width;
  double alpha, beta;
  double n_required;
  double burn_in;
  uint32_t units;
  uint32_t reserved;
} pbn_estimate_out;

pbn_status pbn_estimate(const uint64_t* counts, uint32_t units, uint64_t steps_per_unit, double conf,
                        double precision, pbn_estimate_out* out);

/* Raftery-Lewis single-chain diagnosis (the two-state Markov chain approach
 * the paper uses for its steady-state estimates, Section 4.2; Raftery and
 * Lewis, 1992) of one recorded hit-indicator sequence: bits[t >> 5] bit
 * (t & 31) = z_t for t = 0 .. nbits-1 (host array, caller-owned).
 *   k           thinning: the smallest k <= kmax whose k-thinned sequence
 *               z_0, z_k, ... prefers a first-order to a second-order Markov
 *               chain, BIC = G^2 - 2 log(L - 2) < 0 (kmax when none does)
 *   g2, bic     the statistic and BIC at that k
 *   alpha, beta 0->1 and 1->0 probabilities of the k-thinned chain
 *   burn_in     m* k original steps, m* = log(eps (alpha+beta) / max(alpha,
 *               beta)) / log|1 - alpha - beta|  (1 when alpha + beta = 1)
 *   n_required  N* k original steps, N* = alpha beta (2 - alpha - beta) /
 *               (alpha + beta)^3 (Phi^-1((1 + conf) / 2) / precision)^2
 *   p_hat       mean of z_t for t >= ceil(burn_in) (NaN if none)
 * burn_in and n_required are +inf when the thinned chain never changes state.
 * Errors: PBN_EINVAL (nbits < 3, kmax = 0, precision/eps <= 0, conf outside
 * (0, 1)). */
typedef struct pbn_rl_out {
  uint32_t k;
  uint32_t reserved;
  double g2, bic;
  double alpha, beta;
  double burn_in;
  double n_required;
  double p_hat;
  uint64_t steps;      /* nbits of the diagnosed sequence */
} pbn_rl_out;

pbn_status pbn_rl_diagnose(const uint32_t* bits, uint64_t nbits, double precision, double conf, double eps,
                           uint32_t kmax, pbn_rl_out* out);

/* Blocking driver of the two-state Markov chain approach on one trajectory
 * (id `traj`): s(0) from the INIT stream, then simulate from step 0 while
 * recording target 0's indicator, diagnose (pbn_rl_diagnose), and extend the
 * same trajectory to burn_in + n_required steps until the run is at least that
 * long.  The first diagnosis runs after initial_steps (at least 64).
 *   d_state [state_words], d_counts [ntargets][1][3], d_record [record_words]:
 *   caller-owned device buffers (zeroed or initialised here); the run is
 *   limited to min(max_steps, 32 record_words) < 2^32 steps.
 * `out` holds the last diagnosis.  Synchronises `stream`.  Errors: PBN_EINVAL,
 * PBN_ERANGE (the diagnosis asks for more steps than the limit; `out` is
 * filled), PBN_EHIP, and the errors of pbn_simulate. */
pbn_status pbn_rl_run(const pbn_plan* plan, const void* d_plan, uint64_t seed, uint32_t traj,
                      const pbn_targets* targets, uint32_t* d_state, uint64_t* d_counts, uint32_t* d_record,
                      uint32_t record_words, double precision, double conf, double eps, uint32_t kmax,
                      uint64_t initial_steps, uint64_t max_steps, const pbn_launch_opts* launch, pbn_rl_out* out,
                      void* stream);

/* The Skart stopping rule (Tafazzoli, Steiger and Wilson, 2011), the second
 * steady-state procedure the paper's authors name beside the two-state Markov
 * chain approach (Section 1), on one recorded hit-indicator sequence: bits[t >>
 * 5] bit (t & 31) = z_t for t = 0 .. nbits-1 (host array, caller-owned).
 * Steps, replayed from the start on every call:
 *   1  1280 batches of size m = 1; m doubles while the skewness of the last
 *      1024 batch means exceeds 4 in magnitude;
 *   2  von Neumann's ratio test (two-sided, size 0.20 exp(-0.184 b^2) after b
 *      failures) on every (d+1)-th batch mean, d = 0 .. 10 spacer batches; when
 *      every d fails, m <- ceil(sqrt(2) m), k <- max(ceil(0.9 k), 30);
 *   3  warm-up d m observations; the rest in min(k - d, 1024) batches; the
 *      interval mean -/+ G(t) sqrt(A S^2 / k) with Willink's skewness-adjusted
 *      G and A = max(1, (1 + phi) / (1 - phi)) from the lag-one correlation phi
 *      (clipped at 0.99); while the larger half-length exceeds `precision`, the
 *      sample grows by (half-length / precision)^2 (batches up to 1024, then
 *      batch size), or doubles when all batch means are equal.
 * A step that needs more than nbits observations stops there: done = 0 and
 * n_required = the observations it needs (a longer replay of the same
 * sequence takes the same decisions up to that step).  With done = 1,
 * n_required = the observations used and the interval fields hold the result.
 * Errors: PBN_EINVAL (null pointers, precision <= 0, conf outside (0, 1)). */
typedef struct pbn_skart_out {
  uint32_t done;
  uint32_t stage;           /* 1, 2, 3: the step reached */
  uint64_t n_required;
  uint64_t batch_size;      /* m of steps 1-2 */
  uint32_t batch_count;     /* k of steps 1-2 */
  uint32_t spacer;          /* d */
  uint32_t failures;        /* b */
  uint32_t ci_batches;      /* batches of the interval */
  uint64_t ci_batch_size;
  uint64_t warmup;          /* d m observations */
  double p_hat, lower, upper, half_width;
  double skewness, lag1, ar_factor;   /* of the interval's batch means */
  uint64_t steps;           /* nbits */
} pbn_skart_out;

pbn_status pbn_skart_analyze(const uint32_t* bits, uint64_t nbits, double precision, double conf,
                             pbn_skart_out* out);

/* Blocking Skart driver on one trajectory (id `traj`), like pbn_rl_run: s(0)
 * from the INIT stream, simulate from step 0 recording target 0's indicator,
 * run pbn_skart_analyze, and extend the same trajectory to the number of
 * observations it asks for until it finishes.  Buffers, limits and errors as
 * pbn_rl_run (PBN_ERANGE when the procedure asks for more than min(max_steps,
 * 32 record_words) steps; `out` holds the last analysis).  Synchronises
 * `stream`. */
pbn_status pbn_skart_run(const pbn_plan* plan, const void* d_plan, uint64_t seed, uint32_t traj,
                         const pbn_targets* targets, uint32_t* d_state, uint64_t* d_counts, uint32_t* d_record,
                         uint32_t record_words, double precision, double conf, uint64_t max_steps,
                         const pbn_launch_opts* launch, pbn_skart_out* out, void* stream);

/* Quantiles used by pbn_estimate: Student t with nu degrees of freedom, and the
 * standard normal.  p in (0, 1). */
double pbn_t_quantile(double p, double nu);
double pbn_normal_quantile(double p);

/* ----------------------------------------------------------------- batches
 * Many networks of uneven size advanced together by one persistent launch
 * (the step kernel of pbn_simulate, per trajectory, with a task loop on top).
 * A task is up to `waves_per_block` consecutive trajectories of one network.
 * The task list is cut into `nqueues` queues (at most PBN_BATCH_QUEUES), each
 * a run of whole networks.  Workgroup b claims tasks from queue b mod nqueues
 * with one atomic increment of that queue's counter, then from the other
 * queues once its own is empty, and exits when every queue is empty.  The
 * dispatcher sends workgroup b to XCD b mod 8 and, within the XCD, to its 32
 * CUs in turn; so with nqueues = 8 G the workgroups of a queue run on their
 * own group of 32 / G CUs of one XCD, and the CUs of a group share the
 * images of few networks in their vector L1 caches.  A workgroup whose queue
 * is empty tries the other groups of its XCD before other XCDs.  Every item is simulated
 * over the device-held step window [d_ctl->step0, d_ctl->step0 + d_ctl->nsteps);
 * each launch resets the queue counters first and advances step0 by nsteps
 * last, with small kernels (no memset, no allocation, no host
 * synchronisation), so launches can be captured into a HIP graph and
 * replayed.  Results are bit-identical to pbn_simulate on each network alone,
 * whatever the queues and whichever workgroup runs a task.
 *
 * pbn_work (device array, caller-owned, one per network):
 *   d_plan     device blob of plans[k];  d_targets  device copy of its pbn_targets
 *   d_state    [ntraj][state_words];     d_counts   [ntargets][ntraj][3] (added to)
 *   seed, traj0, ntraj, count_from as in pbn_simulate
 *   step0      offset of this item's window: it advances steps
 *              step0 + d_ctl->step0 .. + d_ctl->nsteps - 1 (callers must keep the
 *              sum below 2^32)
 * pbn_batch_tasks: host; the schedule.  Networks are dealt to `nqueues` queues
 *   (1..PBN_BATCH_QUEUES), largest first, each to the queue with the least
 *   work so far (work = tasks x a per-step cost from the plan's passes, Philox
 *   jobs and slots); within a queue, largest networks first.  tasks /
 *   task_first receive the item and first trajectory of each task in queue
 *   order, queue_first[nqueues + 1] the first task of each queue and the
 *   total (each may be NULL; all NULL to query *ntasks).
 * pbn_batch_launch: enqueue one pass on `stream`.  queue_first: host, the
 *   nqueues + 1 bounds from pbn_batch_tasks (non-decreasing, from 0 to
 *   ntasks), copied into the launch; NULL: one queue of all tasks (nqueues
 *   ignored).  waves_per_block: trajectories per task, as given to
 *   pbn_batch_tasks (one wave each).  waves_per_traj (1..16): with W > 1,
 *   W waves of one workgroup advance each trajectory together, sharing its
 *   state and draws in LDS and splitting each step's lane passes, for a
 *   shorter step latency on networks of many passes; tasks must then hold one
 *   trajectory (waves_per_block = 1).  The W waves keep a copy of the chain
 *   tables (12 bytes a node) in LDS; a launch whose largest network's tables
 *   do not fit beside its states runs one wave per trajectory instead.
 *   Results do not depend on W.
 * pbn_batch_graph_create: capture `passes` consecutive launches into a graph,
 *   replayed by pbn_graph_launch (each replay advances by passes * nsteps).
 * Errors: PBN_EINVAL, PBN_ELDS (one workgroup's states exceed LDS), PBN_EHIP. */
typedef struct pbn_work {
  const void* d_plan;
  const pbn_targets* d_targets;
  uint32_t* d_state;
  uint64_t* d_counts;
  uint64_t seed;
  uint32_t traj0, ntraj;
  uint32_t count_from;
  uint32_t step0;
} pbn_work;

#define PBN_BATCH_QUEUES 64

/* Control block of batched launches (device memory, caller-owned; the caller
 * sets step0 and nsteps, the library the rest). */
typedef struct pbn_batch_ctl {
  uint32_t step0;    /* first step of the next launch's window (advanced by each launch) */
  uint32_t nsteps;   /* steps per launch */
  uint32_t ntasks;   /* written by pbn_batch_launch_noalloc's own schedule; unused otherwise */
  uint32_t reserved; /* unused (keeps the counters 16-byte aligned) */
  uint32_t next_task[PBN_BATCH_QUEUES];   /* claim counters of the queues, reset by each launch */
} pbn_batch_ctl;

typedef struct pbn_graph pbn_graph;

pbn_status pbn_batch_tasks(const pbn_plan* const* plans, const uint32_t* ntraj, uint32_t nitems,
                           uint32_t waves_per_block, uint32_t nqueues, uint32_t* tasks, uint32_t* task_first,
                           uint32_t* queue_first, uint32_t* ntasks);
pbn_status pbn_batch_launch(const pbn_plan* const* plans, uint32_t nitems, const pbn_work* d_items,
                            const uint32_t* d_tasks, const uint32_t* d_task_first, uint32_t ntasks,
                            const uint32_t* queue_first, uint32_t nqueues, pbn_batch_ctl* d_ctl,
                            uint32_t waves_per_block, uint32_t waves_per_traj, void* stream);
pbn_status pbn_batch_graph_create(const pbn_plan* const* plans, uint32_t nitems, const pbn_work* d_items,
                                  const uint32_t* d_tasks, const uint32_t* d_task_first, uint32_t ntasks,
                                  const uint32_t* queue_first, uint32_t nqueues, pbn_batch_ctl* d_ctl,
                                  uint32_t waves_per_block, uint32_t waves_per_traj, uint32_t passes,
                                  pbn_graph** out);
pbn_status pbn_graph_launch(pbn_graph* graph, void* stream);

/* Allocation-free batch launch, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  Same computation as pbn_batch_launch with the step
 * window (step0, nsteps) passed by value: every trajectory of every item
 * advances from step step0 + item.step0 by nsteps steps; states and counters
 * (the items' caller-owned buffers) come out identical.
 *   plans[nitems]  host: the items' plans (kernel shape, as pbn_batch_launch)
 *   ntraj[nitems]  host: the items' trajectory counts (must equal d_items[k].ntraj)
 *   d_items        device: the work items, as pbn_batch_launch
 * The control block and the task schedule live in a device array of the
 * library (512.5 KiB per GPU, held until the process ends) instead of caller
 * buffers: at most 4096 items and 65 536 tasks of waves_per_block trajectories
 * per call (PBN_ELIMIT beyond).  Items run in the caller's order, from one
 * queue (list the largest networks first, as pbn_batch_tasks orders them).  The call makes no
 * device allocation, no memset and no host synchronisation; each call resets
 * the array's task counter with a kernel.  All calls on one GPU share that
 * GPU's array: calls that overlap on one GPU (several streams or host threads)
 * race and must be serialised by the caller.                                  */
pbn_status pbn_batch_launch_noalloc(const pbn_plan* const* plans, const uint32_t* ntraj, uint32_t nitems,
                                    const pbn_work* d_items, uint32_t step0, uint32_t nsteps,
                                    uint32_t waves_per_block, void* stream);
pbn_status pbn_graph_destroy(pbn_graph* graph);

/* --------------------------------------------------------------- probes
 * Measurement kernels for the step kernel's roofline (no simulation work).
 * The caller times them on `stream`; a launch performs
 * blocks x 256 threads x iters x 8 gathers.
 *
 * pbn_probe_lds_gather: random gathers of `width` bytes (1, 4 or 16) from a
 *   2^log2_bytes-byte LDS buffer (7 <= log2_bytes <= 16) per workgroup;
 *   pattern 0: random aligned addresses (bank conflicts as they fall),
 *   pattern 1: the lanes of a wave read bank-distinct words of random rows.
 * pbn_probe_vmem_gather: gathers of `width` bytes (1 or 16) from the
 *   caller's device buffer of at least 2^log2_bytes bytes (4 <= log2_bytes <=
 *   30) through the vector L1 and L2; pattern 0: random aligned addresses,
 *   pattern 1: lane L reads unit L of a random row of 64 x width bytes (a
 *   coalesced read; the buffer must hold one row).
 * d_sink: one device word, written only by an improbable value (keeps the
 * reads).  Errors: PBN_EINVAL for out-of-range arguments, PBN_EHIP.         */
pbn_status pbn_probe_lds_gather(uint32_t log2_bytes, uint32_t width, uint32_t pattern, uint32_t iters,
                                uint32_t blocks, uint32_t* d_sink, void* stream);
pbn_status pbn_probe_vmem_gather(const void* d_buf, uint32_t log2_bytes, uint32_t width, uint32_t pattern,
                                 uint32_t iters, uint32_t blocks, uint32_t* d_sink, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PBN_H */
