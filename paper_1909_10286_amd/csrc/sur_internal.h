// Internal declarations of the learned screen: parameters layout, device
// buffers and launch wrappers (defined in sur.hip).
#pragma once

#include "bl_internal.h"

namespace bl {

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

}  // namespace bl
