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

constexpr uint64_t kInfKey = ~0ull;
constexpr int64_t kInfT = INT64_MAX;
constexpr int64_t kNegInfT = INT64_MIN;
constexpr uint32_t kNone = 0xFFFFFFFFu;

enum : uint32_t { kFixedFieldBp = 1, kNoEmbeddedMin = 2, kGateOff = 4, kGateStrict = 8, kFullWalk = 16,
                  kWideKeys = 32 };
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
};

// ---- learned screen (set encoder) ----
// Parameters, float32, in this order: W1 16x128, b1, W2 128x128, b2,
// W3 136x64 (rows 0..127 read the pooled field embedding, 128..135 the tour
// features), b3, W4 64x2, b4.
constexpr int kSurIn = 16, kSurK1 = 32, kSurH = 128, kSurU = 8, kSurA = 64;
constexpr int kSurOffW1 = 0, kSurOffB1 = 2048, kSurOffW2 = 2176, kSurOffB2 = 18560;
constexpr int kSurOffW3 = 18688, kSurOffB3 = 27392, kSurOffW4 = 27456, kSurOffB4 = 27584;
constexpr int kSurParams = 27586;

struct SurDev {
  float *W, *G, *Mo, *Ve;            // parameters, gradient sums, Adam moments
  uint16_t *w1t;                      // bf16 [128][32]: w1t[n][k] = W1[k][n] (k >= 16: 0)
  uint16_t *w2t;                      // bf16 [128][128]: w2t[n][k] = W2[k][n]
  uint16_t *w2n;                      // bf16 [128][128]: W2 as stored
  uint16_t *w3et;                     // bf16 [64][128]: w3et[n][k] = W3[k][n], k < 128
  uint16_t *w3en;                     // bf16 [128][64]: W3 rows 0..127 as stored
  const float *fstat;                 // [NF][8]: x, y, area, yield, D(HQ,f), 2 n_f / Ws
  const float *bxy;                   // [NB][2] scaled BP coordinates
  float inv_ds, inv_c0, inv_t0, inv_rates, inv_fills;
  uint32_t cap_ex;                    // examples per call (row buffers hold cap_ex * NF rows)
  uint16_t *phi;                      // [rows][32] bf16 features
  uint16_t *row_bp;                   // [rows] BP of the row's field in its candidate
  uint16_t *h1, *h2;                  // [rows][128] bf16 activations
  float *P;                           // [rows][64] h2 W3[0:128]
  float *dP;                          // [rows][64] loss gradient w.r.t. P
  float *ex_u;                        // [ex][NT][8]
  uint16_t *ex_cnt;                   // [ex][NB] fields per BP in the candidate
  uint16_t *ex_nb;                    // [ex][NT] BPs per tour
  uint16_t *ex_btour;                 // [ex][NB] tour of each BP in the candidate
  float *ex_pred;                     // [ex][2] predicted (path, makespan), scaled
  float *loss;                        // [2] loss sum, examples counted
  float *part_h;                      // [head waves][kHeadPart] per-wave sums of the head's gradients
  float *part_b;                      // [backward workgroups][kBwdPart] per-workgroup sums
};

// Partial gradient sums of one training step.  Head, per wave: W3 rows of
// the tour features (8 x 64), b3 (64), W4 (128), b4 (2), loss and count (2).
// Backward, per workgroup: W1, W2, W3 rows 0..127, and b1, b2 in two halves.
constexpr int kHeadPart = (kSurU + 3) * kSurA + 4;
constexpr int kBwdW1 = 0, kBwdW2 = kBwdW1 + kSurIn * kSurH, kBwdW3 = kBwdW2 + kSurH * kSurH;
constexpr int kBwdB1 = kBwdW3 + kSurH * kSurA, kBwdB2 = kBwdB1 + 2 * kSurH;
constexpr int kBwdPart = kBwdB2 + 2 * kSurH;
uint32_t sur_head_grid(uint32_t n, int n_cu);
uint32_t sur_bwd_grid(uint32_t rows, int n_cu);

// Screening of proposals through the learned screen.
struct ScreenDesc {          // what one proposal changes relative to the base (64 bytes)
  uint16_t f[3];             // fields whose features change (0xFFFF: none)
  uint16_t bold[3];          // their BP in the base
  uint16_t bnew[3];          // their BP in the candidate
  uint16_t ab[4];            // BPs whose pooled embedding changes (0xFFFF: none)
  int16_t dcnt[4];           // change of their field counts
  uint16_t tg[2];            // tours whose head input changes (0xFFFF: none)
  int16_t dnf[2], dnb[2];    // change of the tours' field and BP counts
  float u6[2];               // new return-leg feature of those tours
  uint16_t moved_bp;         // BP move: the BP (0xFFFF otherwise)
  uint16_t dst_tour;         // BP move: its destination tour
  uint8_t feasible, pad[5];
};

struct ScreenDev {
  float *Q;                  // [NB][64] sums of the base rows per BP
  float *R;                  // [NT][64] sums over the tour's BPs of the BP means
  float *U;                  // [NT][64] b3 + tour features through W3 rows 128..135
  float *ub6;                // [NT] base return-leg feature
  float *yb;                 // [NT][2] base head outputs
  int32_t *nbg, *nfg;        // [NT] BP / field counts
  float *scal;               // [4]: predicted base path, top-3 base completion outputs
  int32_t *top_g;            // [3] tours of those top-3 outputs
  uint32_t *keys;            // [n_prop] order-preserving score bits (0xFFFFFFFF: discarded)
  uint32_t *hist;            // [2048]
  uint32_t *sel;             // [8] radix-select state
  uint32_t *blk;             // [2 * 1024] per-block counts / offsets
  uint32_t *short_idx;       // [k] shortlisted proposal indices
  uint64_t *short_key;       // [k] their exact keys
  float *short_cost;         // [k] their exact costs, km
  uint32_t *flag;            // [1] 1: evaluate the plain fallback batch
  uint64_t *ctrl_key;        // [1] best exact key of the control sample
  float *stats;              // [4]: mean relative error, fallbacks, screened iterations, used
};

// Kernel entry points (launch wrappers defined in eval.hip).
hipError_t launch_prepare(const InstParams &P, int mode, uint64_t seed, uint64_t eps_thr,
                          uint32_t inst_index, hipStream_t s);
hipError_t launch_generate(const InstParams &P, uint64_t seed, uint32_t iter, uint32_t inst_index,
                           uint32_t first, uint32_t n, uint64_t *out, hipStream_t s);
hipError_t launch_eval_batch(const InstParams &P, const uint64_t *moves, uint32_t n,
                             int64_t t_star, uint64_t *key, float *cost, int32_t *mk,
                             uint8_t *flags, int grid, hipStream_t s);
hipError_t launch_eval_search(const InstParams &P, uint64_t seed, uint32_t n,
                              uint32_t inst_index, int grid, hipStream_t s,
                              const uint32_t *run_flag = nullptr);
hipError_t launch_eval_gather(const InstParams &P, uint64_t seed, const uint32_t *idx, uint32_t n,
                              uint32_t inst_index, uint64_t *key, float *cost, int grid,
                              hipStream_t s);
hipError_t launch_commit(const InstParams &P, int mode, uint64_t seed, uint32_t inst_index,
                         hipStream_t s);
hipError_t launch_select(const uint64_t *keys, uint32_t n, uint64_t *out, hipStream_t s);
size_t eval_lds_bytes(const InstParams &P);
int eval_occupancy(const InstParams &P, bool search);
size_t batch_lds_bytes(uint32_t max_image_words);
int batch_occupancy(size_t lds, bool walk);
hipError_t launch_batch_start(const BatchParams &B, size_t lds, hipStream_t s);
hipError_t launch_batch_prepare(const BatchParams &B, hipStream_t s);
hipError_t launch_batch_eval(const BatchParams &B, int grid, size_t lds, hipStream_t s);
hipError_t launch_batch_commit(const BatchParams &B, size_t lds, hipStream_t s);

size_t sur_w1t_elems();
size_t sur_w2_elems();
size_t sur_w3et_elems();
size_t sur_w3en_elems();
size_t sur_head_lds(const InstParams &P);
hipError_t sur_setup_attributes();
hipError_t launch_sur_pack(const SurDev &S, hipStream_t s);
hipError_t launch_sur_zero(float *p, uint32_t n, hipStream_t s);
hipError_t launch_sur_forward(const InstParams &P, const SurDev &S, const uint64_t *moves,
                              uint32_t n, int noop, bool keep_act, int n_cu, hipStream_t s);
hipError_t launch_sur_head(const InstParams &P, const SurDev &S, uint32_t n, int train,
                           const float *cost_km, const int32_t *mk, int n_cu, hipStream_t s);
hipError_t launch_sur_backward(const InstParams &P, const SurDev &S, uint32_t n, int n_cu,
                               hipStream_t s);
hipError_t launch_sur_adam(const SurDev &S, float lr, float b1, float b2, float eps, float scale,
                           uint32_t step, hipStream_t s);

hipError_t launch_screen_base(const InstParams &P, const SurDev &S, const ScreenDev &T, int n_cu,
                              hipStream_t s);
hipError_t launch_screen_score(const InstParams &P, const SurDev &S, const ScreenDev &T, uint64_t seed,
                               uint32_t inst_index, uint32_t n_prop, float mk_margin, int n_cu,
                               hipStream_t s);
hipError_t launch_screen_select(const ScreenDev &T, uint32_t n_prop, uint32_t k, hipStream_t s);
int screen_waves(const InstParams &P);
hipError_t launch_scr_export(const ScreenDev &T, uint32_t n, float *score, hipStream_t s);
hipError_t launch_scr_check(const InstParams &P, const SurDev &S, const ScreenDev &T, uint32_t k,
                            float err_thr, hipStream_t s);
hipError_t launch_scr_control_save(const InstParams &P, const ScreenDev &T, hipStream_t s);

enum { kPrepFromBase = 0, kPrepSearch = 1 };
enum { kCommitStart = 0, kCommitStep = 1 };

}  // namespace bl
