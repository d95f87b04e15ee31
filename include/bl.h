/*
 * bl.h - C interface of the MI355X (gfx950) candidate evaluator for the
 * GPU-accelerated heuristic search of M. G. Plessen, "GPU-accelerated
 * Logistics Optimisation for Biomass Production with Multiple Simultaneous
 * Harvesters Tours, Fields and Plants" (arXiv 1909.10286).
 *
 * The library evaluates many candidate solutions x_i of the multi-tour
 * harvest problem at once (Algorithm 1, GPU version, sec. 2.5): each
 * candidate is one remove-and-reinsert move (Alg. 1) applied to a base
 * solution; its evaluation checks the demand constraints (eq. (2)), runs the
 * embedded min-max assignment of HUs and of SUs (sec. 2.5 and Algorithm 2)
 * and costs the total path length (sec. 2.2) with the makespan gate of
 * sec. 2.5.
 *
 * Conventions
 *   - Every call returns a bl_status; 0 is success, negative values are
 *     errors.  No exception crosses this interface.  bl_last_error() gives a
 *     message for the last failing call on a context.
 *   - Host pointers are read (or written) during the call only; the caller
 *     keeps ownership.  Device pointers ("d_" prefix) are caller-owned device
 *     memory of the context's device, read or written asynchronously on the
 *     context's stream; the caller synchronises that stream before reading
 *     results.  Calls documented as synchronising wait for the stream.
 *   - A context is used by one host thread at a time.
 *   - Units: distances in metres, supplies and capacities in kg, areas in
 *     0.01 ha, yields in 0.1 t/ha, working rates in 0.01 ha/h, speeds in m/h,
 *     times in seconds.  All decisions are taken in exact integers.
 *   - Vertex numbering: 0 is the headquarter (HQ), 1..n_bps the biogas
 *     plants (BPs), n_bps+1..n_bps+n_fields the fields.
 */
#ifndef BL_H
#define BL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bl_status;
#define BL_OK 0
#define BL_EINVAL (-1)      /* bad argument, descriptor or instance data    */
#define BL_ENOMEM (-2)      /* device or host allocation failed             */
#define BL_EDEVICE (-3)     /* no usable GPU, or a HIP runtime error        */
#define BL_ESTATE (-4)      /* call out of order (e.g. step before start)   */
#define BL_EINFEASIBLE (-5) /* the initial solution misses a demand, eq. (2) */

/* Instance flags (bl_instance.flags). */
#define BL_FIXED_FIELD_BP 1u  /* sec. 2.6: a removed field returns to its own BP      */
#define BL_NO_EMBEDDED_MIN 2u /* Case 2 of sec. 3.2: units never move between tours   */
#define BL_GATE_OFF 4u        /* no makespan gate (Case 2)                             */
#define BL_GATE_STRICT 8u     /* discard when makespan >= T* (default: when > T*)      */
#define BL_FULL_WALK 16u      /* evaluate every candidate by walking all its routes,
                                 instead of from the base's per-tour and per-BP
                                 aggregates and the legs the move changes (same
                                 results; the walk is the plain reading of sec. 2.2) */
#define BL_WIDE_KEYS 32u      /* 64-bit keys in the rebalancing rounds even where the
                                 instance's time bounds allow 32-bit ones (same
                                 results; implies BL_SEGMENT_EVAL) */
#define BL_SEGMENT_EVAL 64u   /* evaluate each candidate on a segment of lanes, one
                                 tour per lane, also where the instance has at most
                                 12 tours and one lane per candidate (all its tours in
                                 registers) is the default (same results) */

/* Per-candidate flags written by bl_evaluate_batch. */
#define BL_CAND_INFEASIBLE 1u   /* eq. (2) violated; cost and makespan not evaluated */
#define BL_CAND_GATED 2u        /* makespan gate of sec. 2.5 discarded it            */
#define BL_CAND_CAP_HU 4u       /* HU rebalancing stopped at its round cap           */
#define BL_CAND_CAP_SU 8u       /* SU rebalancing (Alg. 2) stopped at its round cap  */
#define BL_CAND_INVALID 16u     /* move record out of range for the base             */
#define BL_CAND_INF_MAKESPAN 32u /* an active tour has no HU                         */

/* Solution slots held on the device per instance. */
#define BL_SLOT_BASE 0 /* base x that candidates are drawn from / applied to */
#define BL_SLOT_BEST 1 /* x* of the search                                   */
#define BL_SLOT_OLD 2  /* x_old of the search                                */

#define BL_INF_KEY 0xFFFFFFFFFFFFFFFFull
#define BL_INF_MAKESPAN 0x7FFFFFFF

typedef struct bl_ctx bl_ctx;

/*
 * Problem instance (sec. 2.1, Table 1).  Limits: 1 <= n_fields <= 32767,
 * 1 <= n_bps <= 4096, 1 <= n_tours <= 64 with n_tours <= n_hus <= 64 (sec. 2.1:
 * the number of tours is bounded by the number of HUs), 1 <= n_sus <= 128.
 * dist_m must be symmetric with a zero diagonal and entries < 2^24.  Every
 * field supply (area * yield, in kg), their total, the total area and every
 * field's shuttle distance 2 n_f D[f][b] must stay below 2^32; the total
 * supply must cover the total demand; working rates, speeds and the mean SU
 * capacity must be > 0 and fill times < 2^20 s.  The route-length bound
 * (n_fields + 1) * max distance must stay below 2^32 m and the path-length
 * bound (n_hus + n_sus) * route bound + shuttle total below 2^40 m, so that a
 * cost and a candidate index pack into one 64-bit key.  Violations give
 * BL_EINVAL.
 */
typedef struct {
  int32_t n_fields, n_bps, n_tours, n_hus, n_sus;
  const uint32_t *dist_m;       /* V x V row-major, V = 1 + n_bps + n_fields */
  const uint32_t *field_area;   /* [n_fields], 0.01 ha                      */
  const uint32_t *field_yield;  /* [n_fields], 0.1 t/ha                     */
  const uint32_t *bp_demand_kg; /* [n_bps], minimum demand d_b (eq. (2))    */
  const uint32_t *hu_rate;      /* [n_hus], working rate, 0.01 ha/h         */
  uint32_t hu_speed_mph;        /* HU road speed, m/h (> 0)                 */
  const uint32_t *su_cap_kg;    /* [n_sus], loading capacity                */
  const uint32_t *su_speed_mph; /* [n_sus], road speed (> 0)                */
  const uint32_t *su_fill_s;    /* [n_sus], in-field fill time              */
  const int32_t *xy_m;          /* [2 * V] or NULL: coordinates (learned screen features) */
  const uint16_t *init_hus_per_tour; /* [n_tours] or NULL: initial HU block sizes */
  const uint16_t *init_sus_per_tour; /* [n_tours] or NULL: initial SU block sizes */
  uint32_t flags;               /* BL_FIXED_FIELD_BP | BL_NO_EMBEDDED_MIN | BL_GATE_* | BL_FULL_WALK | BL_WIDE_KEYS | BL_SEGMENT_EVAL */
  uint32_t cap_hu, cap_su;      /* rebalancing round caps; 0 = units + tours */
} bl_instance;

/*
 * Solution x (sec. 2.5, Alg. 1): compressed lists.  Tour g visits BPs
 * tour_bp[tour_off[g] .. tour_off[g+1]) in order; BP b's fields, in harvest
 * order, are bp_field[bp_off[b] .. bp_off[b+1]) (BPs in id order).  hu_tour
 * and su_tour give each unit's tour.  The caller allocates every array.
 */
typedef struct {
  uint16_t *tour_off; /* [n_tours + 1] */
  uint16_t *tour_bp;  /* [n_bps]       */
  uint16_t *bp_off;   /* [n_bps + 1]   */
  uint16_t *bp_field; /* [n_fields]    */
  uint16_t *hu_tour;  /* [n_hus]       */
  uint16_t *su_tour;  /* [n_sus]       */
} bl_solution;

/* One search iteration (Algorithm 1, GPU version). */
typedef struct {
  uint64_t seed;          /* Philox key of the run                               */
  uint64_t eps_threshold; /* eq. (6): base = x* when u32 draw < this; 2^32 = always */
  uint32_t n;             /* candidates per iteration, 1 .. 2^24                 */
  uint32_t inst_index;    /* third Philox counter word (instance id in a batch)  */
} bl_search_params;

typedef struct {
  uint32_t it;          /* iterations done                     */
  uint32_t n_improved;  /* iterations that improved x*          */
  uint64_t cost_best_m; /* C* in metres                         */
  int64_t t_best_s;     /* T*: makespan of x*, seconds          */
} bl_search_state;

/* One row of the per-iteration trace (Fig. 3 quantities). */
typedef struct {
  uint64_t best_key;   /* min key of the iteration (BL_INF_KEY if all discarded) */
  uint64_t cost_m;     /* C* after the iteration                                 */
  int64_t makespan_s;  /* T* after the iteration                                 */
  uint32_t it;
  uint8_t indicator;   /* 0, 1 (field move improved x*), 2 (BP move improved x*) */
  uint8_t use_best;    /* eq. (6) picked x* as the base                          */
  uint8_t pad[2];
} bl_trace_row;

/* Context on GPU `device`; BL_EDEVICE when no GPU is usable. */
bl_status bl_create(int32_t device, bl_ctx **out);
void bl_destroy(bl_ctx *ctx);
/* Stream (hipStream_t, e.g. a torch stream handle) for all later work; NULL = default. */
bl_status bl_set_stream(bl_ctx *ctx, void *hip_stream);
const char *bl_status_str(bl_status s);
const char *bl_last_error(const bl_ctx *ctx);

/* Validate and copy an instance to the device (sec. 2.1 data, Table 1).
 * Writes its id to *inst.  Synchronising. */
bl_status bl_instance_upload(bl_ctx *ctx, const bl_instance *in, int32_t *inst);

/* How an uploaded instance is evaluated.  lane_eval: 1 when the evaluation
 * takes one candidate per lane (at most 12 tours, time bounds within 32
 * bits, no BL_SEGMENT_EVAL / BL_FULL_WALK / BL_WIDE_KEYS); tail_table: 1 when
 * the second pass of that evaluation keeps every thread's SU masks in LDS
 * (chosen at upload where it keeps the workgroups per CU; the environment
 * variable BL_LANE_TAIL=0 at upload turns it off); wg_per_cu: workgroups per
 * CU of the search evaluation; image_bytes: the instance image that every
 * evaluating workgroup stages in LDS.  No device work. */
typedef struct {
  int32_t lane_eval, tail_table, wg_per_cu;
  uint32_t image_bytes;
} bl_instance_info;
bl_status bl_instance_info_get(bl_ctx *ctx, int32_t inst, bl_instance_info *out);

/* The initial solution of Algorithm 1 on the host: BPs to tours by one nearest-neighbour
 * chain from HQ (floor(n_bps / n_tours) per tour, residual to the last),
 * fields in id order to the closest BP with unmet demand (then the closest
 * BP), each BP's fields chained from HQ, units in contiguous id blocks.
 * BL_EINFEASIBLE if some demand stays unmet. */
bl_status bl_init_solution(bl_ctx *ctx, int32_t inst, bl_solution *out);

/* Copy a solution to / from a device slot (BL_SLOT_*).  Upload validates the
 * partition (every field and BP exactly once, units in range) -> BL_EINVAL,
 * and, for BL_SLOT_BASE, prepares it as the base of bl_generate and
 * bl_evaluate_batch.  Download synchronises. */
bl_status bl_solution_upload(bl_ctx *ctx, int32_t inst, int32_t slot, const bl_solution *sol);
bl_status bl_solution_download(bl_ctx *ctx, int32_t inst, int32_t slot, bl_solution *sol);

/* Remove-and-reinsert moves for candidates first .. first+n-1 of iteration `iter` drawn
 * against the base slot: Philox4x32-10 block with counter (i, iter,
 * inst_index, 0) under key `seed`; vertex uniform over fields and BPs,
 * destination BP or tour uniform, slot uniform over the destination list
 * after the removal.  Record: bits 0-14 vertex, bit 15 kind (0 field, 1 BP),
 * bits 16-31 destination, bits 32-47 slot.  d_moves holds n u64.  Async. */
bl_status bl_generate(bl_ctx *ctx, int32_t inst, uint64_t seed, uint32_t iter, uint32_t inst_index,
                      uint32_t first, uint32_t n, uint64_t *d_moves);

/* Evaluate n <= 2^24 candidates (moves applied to the base slot) with makespan
 * gate T* = t_star_s.  Outputs, each nullable except d_key, n entries:
 * key = (path length in m) << 24 | i, or BL_INF_KEY when infeasible, gated or
 * invalid; cost in km as float (+inf if not evaluated); makespan in s
 * (BL_INF_MAKESPAN if infinite or not evaluated); BL_CAND_* flags.  Async. */
bl_status bl_evaluate_batch(bl_ctx *ctx, int32_t inst, const uint64_t *d_moves, uint32_t n,
                            int64_t t_star_s, uint64_t *d_key, float *d_cost_km,
                            int32_t *d_makespan_s, uint8_t *d_flags);

/* bl_evaluate_batch for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, outputs and errors, and the same kernels,
 * but the deferred-candidate list of the one-candidate-per-lane launch and
 * its counts live in a file-scope device array of the library (8 MiB + 256 B
 * per GPU, held until the process ends) instead of the instance's own
 * allocation.  Calls no allocating routine.  n <= 2^24 (BL_EINVAL beyond);
 * the array holds 2^20 deferred BP moves and 2^20 deferred field moves, a
 * launch that defers more finishes the rest in its first pass.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (other streams, other contexts
 * or threads) race and must be serialised by the caller.  BL_EDEVICE if the
 * array's device address could not be found when the context was created.
 * Not timed by bl_timing_enable.  Async. */
bl_status bl_evaluate_batch_static(bl_ctx *ctx, int32_t inst, const uint64_t *d_moves, uint32_t n,
                                   int64_t t_star_s, uint64_t *d_key, float *d_cost_km,
                                   int32_t *d_makespan_s, uint8_t *d_flags);

/* The argmin of Algorithm 1's GPU version (sec. 2.5): the minimum of n keys
 * from bl_evaluate_batch into *d_best (device), i.e. the cheapest candidate
 * that is feasible (eq. (2)) and not discarded by the makespan gate, or
 * BL_INF_KEY when there is none.  The smallest index wins ties because keys
 * carry the index.  d_key: n device keys (not read when n = 0); d_best: one
 * device u64, caller-owned.  BL_EINVAL for a null d_best, or a null d_key
 * with n > 0.  Async on the context's stream. */
bl_status bl_select_best(bl_ctx *ctx, const uint64_t *d_key, uint32_t n, uint64_t *d_best);

/* Start of Algorithm 1: evaluate the base slot with the gate off, store its minimised units
 * as x* and x_old, set C*, T*, and reset the trace (capacity trace_capacity
 * rows; further rows are counted but not stored).  Async. */
bl_status bl_search_start(bl_ctx *ctx, int32_t inst, uint32_t trace_capacity);

/* One iteration of Algorithm 1 (GPU version) entirely on the device: eq. (6)
 * base pick, n candidates generated and evaluated, argmin, reconstruction
 * of the winner, update of x* (strict decrease of C) and x_old.  No host
 * synchronisation; capturable in a HIP graph.  Async. */
bl_status bl_search_step(bl_ctx *ctx, int32_t inst, const bl_search_params *p);

/* Search counters; synchronising. */
bl_status bl_search_state_get(bl_ctx *ctx, int32_t inst, bl_search_state *out);
/* Copies min(max_rows, rows stored) trace rows; synchronising. */
bl_status bl_search_trace(bl_ctx *ctx, int32_t inst, bl_trace_row *out, uint32_t max_rows,
                          uint32_t *n_rows);

/*
 * Batches: many independent instances of uneven size searched together, one
 * persistent evaluation launch per iteration for all of them.  Members are
 * instances of the same context whose base slot is uploaded; each keeps its
 * own x*, x_old, state and trace (read with bl_search_state_get /
 * bl_search_trace on the member id).  Member k draws its candidates with
 * Philox counter word p->inst_index + k.  n_cand (1 .. 2^24) is the number of
 * candidates per member per iteration.
 */
typedef struct {
  /* Candidates per work item for members with < 100, 100-199 and >= 200
   * fields (powers of two, 64 .. 65536). */
  uint32_t tile[3];
  /* 0: members in id order; 1: members with more fields first. */
  uint32_t order_policy;
  /* One candidate per lane only (ignored otherwise).  1: each wave checks
   * eq. (2) for 64 candidates at a time and evaluates the feasible ones 64 at
   * a time from a queue in LDS (pays where many candidates break eq. (2));
   * 0: each lane evaluates its candidates in turn (fewer registers). */
  uint32_t feas_queue;
} bl_batch_schedule;

bl_status bl_batch_create(bl_ctx *ctx, const int32_t *inst_ids, int32_t n_inst, uint32_t n_cand,
                          int32_t *batch);
/* The start of Algorithm 1 for every member (as bl_search_start).  Async. */
bl_status bl_batch_start(bl_ctx *ctx, int32_t batch, uint32_t trace_capacity);
/* One iteration of Algorithm 1 for every member; p->n is ignored.  Async. */
bl_status bl_batch_step(bl_ctx *ctx, int32_t batch, const bl_search_params *p);
bl_status bl_batch_set_schedule(bl_ctx *ctx, int32_t batch, const bl_batch_schedule *s);
/* Search the schedule (tile per size class, member order) by timing the
 * batch's evaluation launch on the current bases, and apply the best one.
 * With cache_path, a previous result for the same member sizes and n_cand is
 * read from that JSON file instead, and a new result is added to it.  The
 * chosen schedule is written to *out (nullable).  Synchronising; the search
 * state is unchanged. */
bl_status bl_batch_autotune(bl_ctx *ctx, int32_t batch, const bl_search_params *p,
                            const char *cache_path, bl_batch_schedule *out);

/*
 * HIP graphs: n_steps iterations of bl_search_step (one instance) or of
 * bl_batch_step (a batch) captured once, then replayed with bl_graph_launch
 * on the context's stream.  The parameters are fixed at capture; capture
 * after bl_search_start / bl_batch_start (a later start invalidates the
 * graph).  Iterations keep advancing: each replay continues the search.
 */
bl_status bl_search_capture(bl_ctx *ctx, int32_t inst, const bl_search_params *p, uint32_t n_steps,
                            int32_t *graph);
bl_status bl_batch_capture(bl_ctx *ctx, int32_t batch, const bl_search_params *p, uint32_t n_steps,
                           int32_t *graph);
bl_status bl_graph_launch(bl_ctx *ctx, int32_t graph);

/*
 * Learned screen (not in the paper): a set encoder over the fields of a
 * candidate solution.  Per field f (BP b, route predecessor p):
 *   phi = [x_f, y_f, area, yield, x_b, y_b, D(f,b), D(p,f), 2 n_f D(f,b), D(HQ,f)]
 *   (scaled by the largest coordinate, area, yield, distance and shuttle
 *   distance; zero padded to 16) -> 128 -> 128 (ReLU), mean over the fields
 *   of each BP, mean over the BPs of each tour, concatenated with 8 tour
 *   features (HU and SU counts, rates and fill times, field and BP counts,
 *   return leg, 1) -> 64 (ReLU) -> 2 (path share, completion time); path =
 *   sum over active tours, makespan = max over active tours, both divided by
 *   the scales c0_m and t0_s.  bf16 MFMA with fp32 accumulation; fp32 master
 *   weights trained with Adam on (candidate, exact cost) pairs.
 * Weights are float32 in this order: W1 16x128, b1 128, W2 128x128, b2 128,
 * W3 136x64, b3 64, W4 64x2, b4 2 (27586 values, row-major).
 * The instance must have been uploaded with coordinates (xy_m) and at most
 * 128 BPs.  Candidates are moves against the instance's base slot.
 */
#define BL_SUR_PARAMS 27586

typedef struct {
  float lr, beta1, beta2, adam_eps; /* Adam                                        */
  uint32_t max_examples;            /* examples per predict / train call           */
  float c0_m, t0_s;                 /* target scales: path length (m), makespan (s) */
} bl_sur_config;

bl_status bl_sur_create(bl_ctx *ctx, int32_t inst, const float *weights, const bl_sur_config *cfg,
                        int32_t *sur);
bl_status bl_sur_get_weights(bl_ctx *ctx, int32_t sur, float *out);
bl_status bl_sur_set_weights(bl_ctx *ctx, int32_t sur, const float *weights);
/* Predictions for n moves: d_out[2 i] = path / c0, d_out[2 i + 1] = makespan / t0.  Async. */
bl_status bl_sur_predict(bl_ctx *ctx, int32_t sur, const uint64_t *d_moves, uint32_t n, float *d_out);
/* Sum over the n examples of the gradient of (P - C/c0)^2 + (M - T/t0)^2
 * into grads (host, BL_SUR_PARAMS floats) and the summed loss into *loss;
 * examples with an infinite cost or makespan are skipped.  Synchronising. */
bl_status bl_sur_gradients(bl_ctx *ctx, int32_t sur, const uint64_t *d_moves, const float *d_cost_km,
                           const int32_t *d_makespan_s, uint32_t n, float *grads, double *loss);
/* One Adam step on the mean loss of n <= max_examples examples (costs and
 * makespans as bl_evaluate_batch writes them).  d_loss (nullable, 2 floats):
 * loss sum and number of examples used.  Async. */
bl_status bl_sur_train_step(bl_ctx *ctx, int32_t sur, const uint64_t *d_moves,
                            const float *d_cost_km, const int32_t *d_makespan_s, uint32_t n,
                            float *d_loss);

/*
 * Learned screen (same surrogate, incremental inference).  The proposals of
 * an iteration are the n_proposals draws of bl_search_step for the same
 * seed, iteration and inst_index, taken against that iteration's base (the
 * eq. (6) pick).  Each proposal changes the features of at most three fields,
 * the pooled means of at most four BPs and the head inputs of at most two
 * tours, so its prediction is the base's with those parts recomputed: three
 * MLP rows per proposal instead of N_F.  A proposal is discarded when it
 * breaks the donor BP's demand (eq. (2)) or when its predicted makespan
 * exceeds the makespan gate, the incumbent makespan divided by t0_s plus
 * mk_margin; the others are ranked by predicted path (normalised by c0_m),
 * and the n_shortlist best (lowest index first among equal scores) form the
 * shortlist.  Discarded proposals rank after all others.
 */
typedef struct {
  uint32_t n_proposals;  /* 1 .. 2^24                                  */
  uint32_t n_shortlist;  /* 1 .. n_proposals                           */
  uint32_t n_fallback;   /* 0 .. 2^24 (screened step only)             */
  float mk_margin;       /* added to the normalised makespan gate       */
  float err_threshold;   /* screened step only, see below              */
  uint32_t n_control;    /* screened step only: 0 .. n_proposals       */
} bl_screen_params;

/* Screen the proposals of the coming iteration of instance `inst` (the one
 * the surrogate was created for; bl_search_start must have run) without
 * taking the iteration.  d_shortlist: n_shortlist u32 proposal indices in
 * ascending order (device, caller-owned).  d_score (nullable): n_proposals
 * floats, the predicted normalised path, +inf for a discarded proposal.
 * p->n is ignored.  Async. */
bl_status bl_sur_screen(bl_ctx *ctx, int32_t sur, const bl_search_params *p,
                        const bl_screen_params *sc, uint32_t *d_shortlist, float *d_score);

/* Screened search iteration: the iteration of bl_search_step (eq. (6) base
 * pick, argmin, commit) with the argmin taken over the shortlist of
 * bl_sur_screen and a control sample, proposals 0 .. n_control-1, all
 * evaluated exactly.  The exact results also judge the screen: when no
 * shortlisted candidate passes the exact gate, when the control sample's
 * best key is below the shortlist's and its cost below x*'s (the screen
 * missed an improvement that an unscreened sample found), or when the scatter of the predicted path around the
 * exact cost over the shortlisted candidates that have one (standard
 * deviation of predicted - exact, km, divided by the mean exact cost; a
 * common offset does not change the ranking and is not counted) exceeds
 * err_threshold, proposals 0 .. n_fallback-1 are evaluated exactly as well
 * (the plain iteration) before the argmin.  Ties
 * and the commit follow bl_search_step.  No host synchronisation.  p->n is
 * ignored.  Async. */
bl_status bl_sur_search_step(bl_ctx *ctx, int32_t sur, const bl_search_params *p,
                             const bl_screen_params *sc);

typedef struct {
  uint32_t iterations;   /* screened iterations run                    */
  uint32_t fallbacks;    /* of which evaluated the fallback proposals  */
  uint32_t last_used;    /* shortlisted candidates with an exact cost  */
  float last_error;      /* last scatter of the path error (+inf: none) */
} bl_sur_stats;

/* Counters of bl_sur_search_step.  Synchronising. */
bl_status bl_sur_stats_get(bl_ctx *ctx, int32_t sur, bl_sur_stats *out);

/* Kernel timing.  what = BL_TIMING_EVAL: every launch of the evaluation
 * kernel made by bl_search_step, bl_evaluate_batch or bl_batch_step is
 * bracketed by two HIP events on the context's stream; BL_TIMING_SCREEN:
 * every launch of the screen's scoring kernel (bl_sur_screen,
 * bl_sur_search_step); 0: off.  Launches inside a capture are not timed.
 * bl_timing_read synchronises, returns the summed kernel time in ms and the
 * number of bracketed launches since the last read, and resets both.
 * Another value of what: BL_EINVAL. */
#define BL_TIMING_EVAL 1
#define BL_TIMING_SCREEN 2
bl_status bl_timing_enable(bl_ctx *ctx, int32_t what);
bl_status bl_timing_read(bl_ctx *ctx, double *eval_ms, uint32_t *n_launches);

/* Measured bandwidth peaks of the device, the denominators a roofline can
 * use beside the published ones: *hbm_gbs from a streaming copy of 1 GiB
 * (bytes read + written per second, best of 5 timed copies), *lds_gbs from
 * conflict-free 16-byte LDS reads on every CU (bytes read per second, best
 * of 5).  Either pointer may be null.  Allocates and frees 2 GiB of device
 * memory; synchronises.  BL_ENOMEM if the buffers cannot be allocated. */
bl_status bl_measure_peaks(bl_ctx *ctx, double *hbm_gbs, double *lds_gbs);

#ifdef __cplusplus
}
#endif

#endif /* BL_H */
