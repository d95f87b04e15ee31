/*
 * bl.h - C interface of the MI355X (gfx950) candidate evaluator for the
 * GPU-accelerated heuristic search of M. G. Plessen, "GPU-accelerated
 * Logistics Optimisation for Biomass Production with Multiple Simultaneous
 * Harvesters Tours, Fields and Plants" (arXiv 1909.10286).
 *
 * The library evaluates many candidate solutions x_i of the multi-tour
 * harvest problem at once (Algorithm 1, GPU version, sec. 2.5): each
 * candidate is one remove-and-reinsert move (Step 8) applied to a base
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
 * field supply (area * yield, in kg) and their total must stay below 2^32,
 * and the total supply must cover the total demand.  Violations give
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
  uint32_t flags;               /* BL_FIXED_FIELD_BP | BL_NO_EMBEDDED_MIN | BL_GATE_* */
  uint32_t cap_hu, cap_su;      /* rebalancing round caps; 0 = units + tours */
} bl_instance;

/*
 * Solution x (sec. 2.5, Step 4): compressed lists.  Tour g visits BPs
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

/* Steps 1-3 of Algorithm 1 on the host: BPs to tours by one nearest-neighbour
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

/* Step 8 moves for candidates first .. first+n-1 of iteration `iter` drawn
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

/* Minimum of n keys into *d_best (device).  The smallest index wins ties
 * because keys carry the index.  Async. */
bl_status bl_select_best(bl_ctx *ctx, const uint64_t *d_key, uint32_t n, uint64_t *d_best);

/* Step 4: evaluate the base slot with the gate off, store its minimised units
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

/* Kernel timing.  While enabled, every launch of the evaluation kernel made
 * by bl_search_step or bl_evaluate_batch is bracketed by two HIP events on
 * the context's stream.  bl_timing_read synchronises, returns the summed
 * kernel time in ms and the number of bracketed launches since the last
 * read, and resets both. */
bl_status bl_timing_enable(bl_ctx *ctx, int32_t on);
bl_status bl_timing_read(bl_ctx *ctx, double *eval_ms, uint32_t *n_launches);

#ifdef __cplusplus
}
#endif

#endif /* BL_H */
