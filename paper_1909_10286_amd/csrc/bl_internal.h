// Internal layout shared by the host code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bl {

constexpr int kMaxFields = 32767;
constexpr int kMaxBps = 4096;
constexpr int kMaxTours = 64;
constexpr int kMaxHus = 64;
constexpr int kMaxSus = 128;
constexpr uint32_t kMaxCand = 1u << 24;
// Room for candidates whose long rebalancing tails an evaluation launch
// moves to its second pass; the ones beyond it finish in the first.
constexpr uint32_t kDeferCap = 1u << 20;
// Deferred-list room of bl_evaluate_batch_static, whose list and count live
// in a file-scope device array (eval.hip) instead of the instance's
// allocation.
constexpr uint32_t kStaticDeferCap = 1u << 20;

constexpr uint64_t kInfKey = ~0ull;
constexpr int64_t kInfT = INT64_MAX;
constexpr int64_t kNegInfT = INT64_MIN;
constexpr uint32_t kNone = 0xFFFFFFFFu;

enum : uint32_t { kFixedFieldBp = 1, kNoEmbeddedMin = 2, kGateOff = 4, kGateStrict = 8, kFullWalk = 16,
                  kWideKeys = 32, kSegmentEval = 64 };
enum : uint32_t {
  kCandInfeasible = 1, kCandGated = 2, kCandCapHu = 4, kCandCapSu = 8, kCandInvalid = 16,
  kCandInfMakespan = 32
};

// Word offsets (32-bit words) of the arrays of the per-instance image.  The
// image is one contiguous buffer that every evaluating workgroup copies into
// LDS unchanged.  The first `static_words` words never change after upload;
// the rest (the base view) is rewritten whenever the base solution changes.
struct ImageLayout {
  // static, per field id: area (0.01 ha), supply (kg), shuttle drives, D[HQ][f]
  uint32_t area, supply, nsh, dhq;
  uint32_t demand;                          // per BP, kg
  uint32_t hu_rate, su_fill, su_speed;      // per unit rank
  uint32_t hu_rank, su_rank;                // u16 per unit id -> rank
  // base view
  uint32_t seq;       // u16 per position: field at that position of the base
  uint32_t pos;       // u16 per field: its position
  uint32_t fbp;       // u16 per field: its BP
  uint32_t fidx;      // u16 per field: its index in the BP's list
  uint32_t prec;      // uint4 per position q: {D[field(q-1)][field(q)] (q=0: from HQ),
                      //   D[field][its BP], area, supply}
  uint32_t w_q;       // u32 per position: shuttle distance 2 * drives * D[field][its BP]
  uint32_t bp_start;  // u16 per BP: position of its first field
  uint32_t bp_len;    // u16 per BP: number of fields
  uint32_t bp_tour;   // u16 per BP: its tour
  uint32_t bp_idx;    // u16 per BP: its index in the tour's list
  uint32_t tour_off;  // u16 [NT+1]: CSR offsets of the tour lists
  uint32_t tour_bp;   // u16 [NB]: BPs in tour order
  uint32_t hu_mask;   // u64 per tour: HU ranks held
  uint32_t su_mask;   // 2 x u64 per tour: SU ranks held
  // base aggregates, from which a candidate's tours follow in O(1)
  uint32_t t_len;     // u32 per tour: route length L(g), m
  uint32_t t_area;    // u32 per tour: area
  uint32_t t_sh;      // u64 per tour: shuttle distance
  uint32_t t_msum;    // u32 per tour: sum over its BPs with fields of floor(sum D[f][b] / |F_b|)
  uint32_t t_mcnt;    // u32 per tour: number of its BPs with fields
  uint32_t t_start;   // u16 per tour: first position of its fields
  uint32_t t_end;     // u16 per tour: one past its last position
  uint32_t b_sd;      // u32 per BP: sum of D[f][b] over its fields
  uint32_t b_sup;     // u32 per BP: supply, kg
  uint32_t b_area;    // u32 per BP: area
  uint32_t b_sh;      // u64 per BP: shuttle distance
  uint32_t b_int;     // u32 per BP: legs between its consecutive fields
  uint32_t b_mean;    // u32 per BP: floor(sum D[f][b] / |F_b|), 0 without fields
  uint32_t b_skip;    // u32 per BP: leg joining its route neighbours once its fields leave
  uint32_t skip;      // u32 per position: leg joining the field's route neighbours once it leaves
  uint32_t n_viol;    // u32: BPs whose supply is below their demand
  uint32_t static_words, total_words;
};

struct DevSol {
  uint16_t *tour_off, *tour_bp, *bp_off, *bp_field, *hu_tour, *su_tour;
};

struct SearchState {
  uint32_t it;
  uint32_t n_improved;
  uint64_t cost_best;
  int64_t t_best;
  uint32_t use_best;
  uint32_t trace_rows;
};

struct TraceRow {
  uint64_t best_key;
  uint64_t cost_m;
  int64_t makespan_s;
  uint32_t it;
  uint8_t indicator, use_best, pad[2];
};

// The minimised units of the candidate that held the best key when the last
// workgroup of the second lane pass finished its own candidates (usually the
// iteration's winner), formed by that workgroup while the others run; the
// commit takes them instead of evaluating the winner again when the record
// is valid (the base preparation clears it each iteration) and its key and
// iteration match.
constexpr int kRecTours = 12;
struct WinRec {
  uint64_t key, cost;
  int64_t makespan;
  uint32_t it, valid;
  uint64_t hm[kRecTours], su_lo[kRecTours], su_hi[kRecTours];
};

// Everything a kernel needs to know about one instance (passed by value).
struct InstParams {
  int32_t NF, NB, NT, NHU, NSU, V;
  uint32_t flags, cap_hu, cap_su, v_hu;
  int32_t seg;        // lanes per candidate: power of two >= NT
  int32_t d_in_lds;   // the distance matrix is staged in LDS too
  int32_t narrow;     // times provably within (-2^26, 2^26 - 1) s and seg <= 16: 32-bit keys
  ImageLayout lay;
  const uint32_t *dist;
  uint32_t *image;
  DevSol sol[3];
  SearchState *st;
  TraceRow *trace;
  uint32_t trace_cap;
  uint64_t *best_key;  // per-instance argmin slot
  uint32_t *defer;     // [2 defer_cap] candidates whose SU rounds an evaluation launch left for its
                       // second pass: BP moves in the first defer_cap entries, field moves after them
  uint32_t *defer_cnt; // [2] their counts per class
  uint32_t defer_cap;  // entries per class; 0: no deferral
  uint32_t defer_zeroed; // host side: the base preparation of this iteration already cleared the count
  int32_t lane_tail;   // host side: the second lane pass keeps the SU masks in LDS (k_eval_lane_tail)
  WinRec *rec;         // the winner's units formed during the second pass (search and gather launches); null: none
  uint16_t *hu_id;     // rank -> HU id
  uint16_t *su_id;     // rank -> SU id
};

// A batch of instances evaluated by one persistent launch.
struct BatchParams {
  const InstParams *inst;    // [K] device copies of the members' parameters
  uint32_t K;
  uint32_t n;                // candidates per member per iteration
  uint64_t seed;
  uint64_t eps_thr;
  uint32_t index_base;       // member k uses Philox counter word index_base + k
  uint32_t total_items;
  const uint32_t *item_off;  // [K+1] first item of each schedule position
  const uint32_t *order;     // [K] schedule position -> member
  const uint32_t *tile;      // [K] candidates per item, by member
  uint32_t *queue;           // [1] next item to pop
  uint32_t walk;             // some member asks for the full walk (host side)
  uint32_t lane_n;           // > 0: one candidate per lane with this many tour slots (host side)
  uint32_t lane_small;       // every member has at most 32 HUs and 64 SUs (host side)
  uint32_t feas_queue;       // lane version: per-wave queue of the candidates that pass eq. (2) (host side)
};

// Kernel entry points (launch wrappers defined in eval.hip).
hipError_t launch_prepare(const InstParams &P, int mode, uint64_t seed, uint64_t eps_thr,
                          uint32_t inst_index, hipStream_t s);
hipError_t launch_generate(const InstParams &P, uint64_t seed, uint32_t iter, uint32_t inst_index,
                           uint32_t first, uint32_t n, uint64_t *out, hipStream_t s);
// Device address of the static array behind bl_evaluate_batch_static on the
// current device (2 kStaticDeferCap + 64 words).
hipError_t static_scratch_address(uint32_t **out);
hipError_t launch_eval_batch(const InstParams &P, const uint64_t *moves, uint32_t n,
                             int64_t t_star, uint64_t *key, float *cost, int32_t *mk,
                             uint8_t *flags, int grid, hipStream_t s);
// count_zeroed: the search-mode base preparation just before this launch
// cleared the deferred count (it does), so the launch skips its own clearing
// kernel.
hipError_t launch_eval_search(const InstParams &P, uint64_t seed, uint32_t n,
                              uint32_t inst_index, int grid, hipStream_t s,
                              const uint32_t *run_flag = nullptr, bool count_zeroed = false);
hipError_t launch_eval_gather(const InstParams &P, uint64_t seed, const uint32_t *idx, uint32_t n,
                              uint32_t inst_index, uint64_t *key, float *cost, int grid,
                              hipStream_t s);
hipError_t launch_commit(const InstParams &P, int mode, uint64_t seed, uint32_t inst_index,
                         hipStream_t s);
hipError_t launch_select(const uint64_t *keys, uint32_t n, uint64_t *out, hipStream_t s);
size_t eval_lds_bytes(const InstParams &P);
// Whether the evaluation launches take one candidate per lane (instances of
// at most 12 tours, unless a flag asks for the segment version).
bool lane_eval_on(const InstParams &P);
// Whether the second lane pass can take the kernel that keeps every
// thread's SU masks in LDS without losing workgroups per CU (off with the
// environment variable BL_LANE_TAIL=0).
bool lane_tail_on(const InstParams &P);
int eval_occupancy(const InstParams &P, bool search);
size_t batch_lds_bytes(uint32_t max_image_words);
int batch_occupancy(size_t lds, bool walk, int lane_n, bool lane_small, bool feas_queue);
// Tour slots of the one-candidate-per-lane batched kernel for members of at
// most max_nt tours (4, 8 or 12), 0 beyond 12.
int batch_lane_tours(int max_nt);
hipError_t launch_batch_start(const BatchParams &B, size_t lds, hipStream_t s);
hipError_t launch_batch_prepare(const BatchParams &B, size_t lds, hipStream_t s);
hipError_t launch_batch_eval(const BatchParams &B, int grid, size_t lds, hipStream_t s);
hipError_t launch_batch_commit(const BatchParams &B, size_t lds, hipStream_t s);

// Bandwidth probes (peaks.hip): a streaming device copy of `bytes`; a
// ds_read_b128 stream of `steps` reads per lane on peak_lds_blocks(n_cu)
// workgroups of 256 lanes (out: one word per lane).
hipError_t launch_peak_copy(const void *src, void *dst, size_t bytes, int n_cu, hipStream_t s);
size_t peak_lds_blocks(int n_cu);
hipError_t launch_peak_lds(uint32_t steps, uint32_t *out, int n_cu, hipStream_t s);

enum { kPrepFromBase = 0, kPrepSearch = 1 };
enum { kCommitStart = 0, kCommitStep = 1 };

}  // namespace bl
