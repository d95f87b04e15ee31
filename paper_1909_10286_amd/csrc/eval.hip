// gfx950 kernels of the candidate evaluator: base preparation, move
// generation, candidate evaluation (walk, eq. (2) check, HU and SU min-max
// rebalancing, path-length cost, makespan gate), argmin, and the commit of
// the winner (Algorithm 1, GPU version, sec. 2.5 of the paper).
//
// Mapping.  One candidate is evaluated by a segment of S lanes of a 64-lane
// wavefront, S the smallest power of two >= N_T: lane t of the segment owns
// tour t.  Each lane walks its own tour of the candidate (the candidate is the
// base with the move applied by index remapping, never materialised), so the
// per-tour sums need no cross-lane traffic; the rebalancing rounds then run
// with one tour per lane, arg-max / arg-min / sums as butterfly reductions
// inside the segment and predicates as wave ballots.  Every branch that
// depends on the candidate is uniform across its segment.
//
// LDS holds a copy of the instance image (static per-field / per-unit tables
// plus the base view: field order, positions, successor distances, tour and
// BP lists, unit masks) and, when it fits, the full distance matrix.  Without
// the matrix in LDS, the walk takes every leg between fields that are
// consecutive in the base from the successor band and fetches only the legs
// created by the move (at most three per tour) from the matrix in HBM/L2.
#include <hip/hip_runtime.h>

#include "bl_internal.h"
#include "device.h"
#include "lane_eval.h"

namespace bl {

namespace {

// Modes: batch (move records given, per-candidate outputs), search (moves
// drawn for indices 0..n-1, argmin into the instance's slot) and gather
// (moves drawn for the indices listed in `gather`, per-entry outputs and the
// argmin).  `run_flag` (nullable): the launch does nothing while it is 0.
template <bool DLDS, int MODE, bool WALK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_eval(InstParams P, const uint64_t *__restrict__ moves,
                                              uint32_t n, int64_t t_star_arg, uint64_t seed,
                                              uint32_t inst_index, uint64_t *__restrict__ out_key,
                                              float *__restrict__ out_cost,
                                              int32_t *__restrict__ out_mk,
                                              uint8_t *__restrict__ out_flags,
                                              const uint32_t *__restrict__ gather,
                                              const uint32_t *__restrict__ run_flag) {
  if (run_flag && *run_flag == 0u) return;
  uint32_t *lds = reinterpret_cast<uint32_t *>(g_lds4);
  const uint32_t img_words = round4(P.lay.total_words);
  stage(lds, P.image, P.lay.total_words);
  if (DLDS) stage(lds + img_words, P.dist, (uint32_t)(P.V * P.V));
  __syncthreads();
  const View V = make_view(lds, P.lay, DLDS ? lds + img_words : P.dist);

  const int S = P.seg;
  const int lane = threadIdx.x & 63;
  const int t = lane & (S - 1);
  const int seg_base = lane & ~(S - 1);
  const uint64_t seg_mask = S == 64 ? ~0ull : ((1ull << S) - 1ull);
  const int segs_per_wave = 64 / S;
  const int waves_per_block = blockDim.x >> 6;
  const uint32_t gseg = ((blockIdx.x * waves_per_block + (threadIdx.x >> 6)) * segs_per_wave) +
                        (uint32_t)(lane / S);
  const uint32_t nseg = gridDim.x * waves_per_block * segs_per_wave;

  uint32_t it = 0;
  int64_t t_star = t_star_arg;
  if (MODE != kModeBatch) {
    it = P.st->it;
    t_star = P.st->t_best;
  }
  uint64_t best = kInfKey;
  for (uint32_t c = gseg; c < n; c += nseg) {
    const uint32_t ci = MODE == kModeGather ? gather[c] : c;
    const uint64_t w = MODE == kModeBatch ? moves[c] : draw_move(seed, ci, it, inst_index, V, P);
    const CandResult r = eval_one<WALK>(V, P, w, ci, t, S, seg_base, seg_mask, t_star);
    if (MODE != kModeSearch && t == 0) {
      if (out_key) out_key[c] = r.key;
      if (out_cost) out_cost[c] = r.cost_km;
      if (out_mk) out_mk[c] = r.mk;
      if (out_flags) out_flags[c] = (uint8_t)r.flags;
    }
    best = r.key < best ? r.key : best;
  }
  if (MODE != kModeBatch) wave_min_to(best, P.best_key);
}

// The same launch with one candidate per lane (lane_eval.h): for instances of
// at most kLaneMaxTours tours, unless a flag asks for the segment version.
// phase 0: candidates 0 .. n-1; one whose SU rounds go past kSuDeferRounds
// rounds is appended to the instance's deferred list (while it has room)
// instead of holding its wave in a long tail of rounds.  phase 1: the
// deferred candidates, densely, with no limit.  A deferred candidate is
// evaluated again from the start, so the limit trades that repeated work
// against the tail.  Measured: one round is fastest at 5 and at 10 tours (of
// 1, 2, 3) now that the second pass keeps its SU masks in LDS; with that pass
// in registers, 3 rounds had been fastest at 5 tours.
constexpr int kSuDeferRounds = 1;

// The deferred list holds two classes, each in a part of its own with a
// count of its own: BP moves (class 0) and field moves (class 1).  A BP move
// carries a whole BP's fields and changes its tours' mean distances more, so
// its SU tails run longer (clust500 after 200 iterations: 20 rounds on
// average, up to 66, against 10, up to 19, for field moves); the second pass
// takes the BP moves first, in waves of their own, and the field moves after
// them.  A workgroup collects its deferred candidates in LDS and appends them
// to the list at its end with one atomic per class: with one global atomic
// per deferring lane or wave the shared counters were the bottleneck of the
// first pass.
constexpr int kWgDefer = 512;   // per class and workgroup

// Orders LDS traffic between the lanes of one wave.
__device__ __forceinline__ void lane_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Candidates a wave holds back between its feasibility checks and their
// evaluation: up to 63 left over plus one batch of 64.
constexpr int kLaneQueue = 128;

// Per-candidate outputs of the batch and gather modes.
template <int MODE>
__device__ __forceinline__ void lane_write(uint32_t c, const CandResult &r, uint64_t *out_key, float *out_cost,
                                           int32_t *out_mk, uint8_t *out_flags) {
  if (MODE == kModeSearch) return;
  if (out_key) out_key[c] = r.key;
  if (out_cost) out_cost[c] = r.cost_km;
  if (out_mk) out_mk[c] = r.mk;
  if (out_flags) out_flags[c] = (uint8_t)r.flags;
}

// A candidate's outputs from its evaluation: key (cost, then index; none
// when gated or infeasible), cost in km, makespan and flags.
__device__ __forceinline__ CandResult lane_result(const LaneOut &o, uint32_t ci, int64_t t_star, uint32_t flags) {
  CandResult r{kInfKey, __builtin_inff(), 0x7FFFFFFF, o.flags};
  if (o.feasible) {
    r.cost_km = (float)((double)o.cost / 1000.0);
    r.mk = o.makespan >= 0x7FFFFFFFll ? 0x7FFFFFFF : (int32_t)o.makespan;
    if (is_gated(o.makespan, t_star, flags))
      r.flags |= kCandGated;
    else
      r.key = (o.cost << 24) | (uint64_t)ci;
  }
  return r;
}

// Waves per SIMD the lane kernel is compiled for: 2 (at most 256 VGPRs).
// Left to itself the compiler takes 264 registers at 10 tours and drops to
// one wave (clust500: 1.72 ms per evaluation step against 1.19 ms bounded);
// at 5 tours, 3 waves (168 VGPRs, a few spills) measured 2 % slower than 2.
constexpr int kLaneWaves = 2;

template <int N, bool SMALL, int MODE>
__global__ __launch_bounds__(256, kLaneWaves) void k_eval_lane(InstParams P, int phase, const uint64_t *__restrict__ moves,
                                                   uint32_t n, int64_t t_star_arg, uint64_t seed,
                                                   uint32_t inst_index, uint64_t *__restrict__ out_key,
                                                   float *__restrict__ out_cost,
                                                   int32_t *__restrict__ out_mk,
                                                   uint8_t *__restrict__ out_flags,
                                                   const uint32_t *__restrict__ gather,
                                                   const uint32_t *__restrict__ run_flag) {
  if (run_flag && *run_flag == 0u) return;
  // The counter goes on counting past the list's room (those candidates
  // finish in the first pass), so the second pass takes at most defer_cap.
  // The list holds defer_cap entries per class: BP moves first, then field
  // moves.
  const uint32_t cap = P.defer_cap;
  const uint32_t n_bp = phase == 0 ? 0u : min(P.defer_cnt[0], cap);
  const uint32_t total = phase == 0 ? n : n_bp + min(P.defer_cnt[1], cap);
  if (phase == 1 && blockIdx.x * blockDim.x >= total) return;
  __shared__ LaneBase s_base;
  __shared__ uint64_t s_qw[4][kLaneQueue];
  __shared__ uint32_t s_qc[4][kLaneQueue];
  __shared__ uint32_t s_dq[2][kWgDefer];
  __shared__ uint32_t s_dqn[2], s_dbase[2];
  if (threadIdx.x < 2) s_dqn[threadIdx.x] = 0u;
  uint32_t *lds = reinterpret_cast<uint32_t *>(g_lds4);
  stage(lds, P.image, P.lay.total_words);
  __syncthreads();
  // The distance matrix stays in global memory: a candidate reads at most a
  // few legs of it.
  const View V = make_view(lds, P.lay, P.dist);
  lane_base_fill(s_base, V, P, N);
  __syncthreads();
  uint32_t it = 0;
  int64_t t_star = t_star_arg;
  if (MODE != kModeBatch) {
    it = P.st->it;
    t_star = P.st->t_best;
  }
  const int su_limit = phase == 0 && P.defer_cap ? kSuDeferRounds : 0;
  uint64_t best = kInfKey;
  // Full evaluation of feasible candidate c (move word w), from round limit
  // lim0.  A candidate whose SU rounds pass the limit goes to the
  // workgroup's buffer (or, when that is full, straight to the list); when
  // the list is full too it is evaluated again here with no limit (one copy
  // of the evaluation in the code, run once or twice).
  auto evaluate = [&](uint32_t c, uint64_t w, int lim0) {
    const uint32_t ci = MODE == kModeGather ? gather[c] : c;
    const Move m = decode_move(w, V, P);
    CandResult r{kInfKey, __builtin_inff(), 0x7FFFFFFF, 0u};
    LaneOut o;
    for (int lim = lim0;; lim = 0) {
      o = eval_lane<N, SMALL>(V, P, s_base, m, lim);
      if (!o.deferred) break;
      const int cls = m.kind == 0 ? 1 : 0;
      const uint32_t ls = atomicAdd(&s_dqn[cls], 1u);
      if (ls < (uint32_t)kWgDefer) {
        s_dq[cls][ls] = c;
        return;
      }
      const uint32_t slot = atomicAdd(P.defer_cnt + cls, 1u);
      if (slot < cap) {
        P.defer[cls * cap + slot] = c;
        return;
      }
    }
    r = lane_result(o, ci, t_star, P.flags);
    lane_write<MODE>(c, r, out_key, out_cost, out_mk, out_flags);
    best = r.key < best ? r.key : best;
  };
  // Each wave checks 64 candidates at a time for validity and eq. (2) (the
  // others get their outputs at once) and queues the feasible ones in LDS;
  // whenever 64 are queued, every lane evaluates one.  About half the
  // candidates break eq. (2); without the queue their lanes would idle
  // through the rebalancing rounds of the feasible ones.  In the second
  // pass the candidates are the deferred list's, all feasible.
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint64_t *qw = s_qw[wave];
  uint32_t *qc = s_qc[wave];
  uint32_t qn = 0;   // wave-uniform
  const uint32_t wstride = gridDim.x * (blockDim.x >> 6) * 64u;
  for (uint32_t i0 = (blockIdx.x * (blockDim.x >> 6) + (uint32_t)wave) * 64u;; i0 += wstride) {
    const bool more = i0 < total;
    if (more) {
      const uint32_t i = i0 + (uint32_t)lane;
      bool feas = false;
      uint64_t w = 0;
      uint32_t c = 0;
      if (i < total) {
        c = phase == 0 ? i : P.defer[i < n_bp ? i : cap + (i - n_bp)];
        const uint32_t ci = MODE == kModeGather ? gather[c] : c;
        w = MODE == kModeBatch ? moves[c] : draw_move(seed, ci, it, inst_index, V, P);
        const Move m = decode_move(w, V, P);
        CandResult r{kInfKey, __builtin_inff(), 0x7FFFFFFF, 0u};
        if (!m.valid)
          r.flags = kCandInvalid;
        else if (!delta_feasible(V, m))
          r.flags = kCandInfeasible;
        else
          feas = true;
        if (!feas) lane_write<MODE>(c, r, out_key, out_cost, out_mk, out_flags);
      }
      const uint64_t bal = __ballot(feas);
      if (feas) {
        const uint32_t at = qn + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        qw[at] = w;
        qc[at] = c;
      }
      qn += (uint32_t)__popcll(bal);
    }
    while (qn >= 64u || (!more && qn > 0u)) {
      lane_wave_sync();
      const uint32_t take = qn < 64u ? qn : 64u;
      if ((uint32_t)lane < take) evaluate(qc[qn - take + lane], qw[qn - take + lane], su_limit);
      lane_wave_sync();
      qn -= take;
    }
    if (!more) break;
  }
  if (su_limit) {
    // The workgroup's deferred candidates join the list; any the list has
    // no room for are finished here.
    __syncthreads();
    if (threadIdx.x < 2) {
      const uint32_t k = min(s_dqn[threadIdx.x], (uint32_t)kWgDefer);
      s_dbase[threadIdx.x] = k ? atomicAdd(P.defer_cnt + threadIdx.x, k) : 0u;
    }
    __syncthreads();
#pragma unroll 1
    for (int cls = 0; cls < 2; ++cls) {
      const uint32_t k = min(s_dqn[cls], (uint32_t)kWgDefer), base = s_dbase[cls];
      for (uint32_t i = threadIdx.x; i < k; i += blockDim.x) {
        const uint32_t c = s_dq[cls][i];
        if (base + i < cap) {
          P.defer[cls * cap + base + i] = c;
        } else {
          const uint32_t ci = MODE == kModeGather ? gather[c] : c;
          evaluate(c, MODE == kModeBatch ? moves[c] : draw_move(seed, ci, it, inst_index, V, P), 0);
        }
      }
    }
  }
  if (MODE != kModeBatch) wave_min_to(best, P.best_key);
}

// Evaluates the candidate that holds the instance's best key (the first
// pass's best, or a better one the second pass already found) with the
// segment version, as the commit would, and keeps its minimised units in
// P.rec with its key and iteration.  Run by one workgroup of the second
// pass; the commit uses the record only where its key is the iteration's
// final best.
// `staged`: the image is already in LDS.
__device__ void winner_units(const InstParams &P, uint64_t seed, uint32_t inst_index, bool staged) {
  __shared__ uint64_t s_key;
  if (threadIdx.x == 0) s_key = *(volatile uint64_t *)P.best_key;
  uint32_t *lds = reinterpret_cast<uint32_t *>(g_lds4);
  if (!staged) stage(lds, P.image, P.lay.total_words);
  __syncthreads();
  const uint64_t key = s_key;
  if (key == kInfKey || threadIdx.x >= 64) return;
  const View V = make_view(lds, P.lay, P.dist);
  const uint32_t it = P.st->it;
  const Move m = decode_move(draw_move(seed, (uint32_t)(key & 0xFFFFFFu), it, inst_index, V, P), V, P);
  const int S = P.seg;
  const int t = threadIdx.x & (S - 1);
  const uint64_t seg_mask = S == 64 ? ~0ull : ((1ull << S) - 1ull);
  const int seg_base = threadIdx.x & ~(S - 1);
  if (seg_base != 0) return;
  const EvalOut o = eval_candidate<false, 0>(V, P, m, t, S, seg_base, seg_mask);
  WinRec &w = *P.rec;
  if (t < P.NT && t < kRecTours) {
    w.hm[t] = o.hu_mask;
    w.su_lo[t] = o.su_mask.lo;
    w.su_hi[t] = o.su_mask.hi;
  }
  if (t == 0) {
    w.key = key;
    w.cost = o.cost;
    w.makespan = o.makespan;
    w.it = it;
  }
  __threadfence();
  if (t == 0) w.valid = 1u;
}

// The second pass over the deferred list where the SU masks of every thread
// fit in LDS beside the image (rows of N entries after it, ltbl_get): a
// round then reads and writes the two tours' masks in LDS instead of
// selecting over every tour's registers.  Every deferred candidate passed
// eq. (2), so the pass needs no queue, and nothing is deferred again.
template <int N, bool SMALL, int MODE>
__global__ __launch_bounds__(256, kLaneWaves) void k_eval_lane_tail(InstParams P, const uint64_t *__restrict__ moves,
                                                        uint32_t n, int64_t t_star_arg, uint64_t seed,
                                                        uint32_t inst_index, uint64_t *__restrict__ out_key,
                                                        float *__restrict__ out_cost,
                                                        int32_t *__restrict__ out_mk,
                                                        uint8_t *__restrict__ out_flags,
                                                        const uint32_t *__restrict__ gather,
                                                        const uint32_t *__restrict__ run_flag) {
  if (run_flag && *run_flag == 0u) return;
  // In search and gather launches the last workgroup also forms the units of
  // the best candidate so far, after its own candidates: they are the last
  // field moves of the list (short tails), so it is done long before the
  // waves of long BP tails are.
  const bool extra = MODE != kModeBatch && P.rec && blockIdx.x == gridDim.x - 1;
  const uint32_t cap = P.defer_cap;
  const uint32_t n_bp = min(P.defer_cnt[0], cap);
  const uint32_t total = n_bp + min(P.defer_cnt[1], cap);
  if (blockIdx.x * blockDim.x >= total) {
    if (extra) winner_units(P, seed, inst_index, false);
    return;
  }
  __shared__ LaneBase s_base;
  uint32_t *lds = reinterpret_cast<uint32_t *>(g_lds4);
  stage(lds, P.image, P.lay.total_words);
  __syncthreads();
  const View V = make_view(lds, P.lay, P.dist);
  lane_base_fill(s_base, V, P, N);
  __syncthreads();
  uint64_t *row0 = reinterpret_cast<uint64_t *>(lds + round4(P.lay.total_words)) + (SMALL ? 1 : 2) * threadIdx.x;
  uint32_t it = 0;
  int64_t t_star = t_star_arg;
  if (MODE != kModeBatch) {
    it = P.st->it;
    t_star = P.st->t_best;
  }
  uint64_t best = kInfKey;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const uint32_t c = P.defer[i < n_bp ? i : cap + (i - n_bp)];
    const uint32_t ci = MODE == kModeGather ? gather[c] : c;
    const uint64_t w = MODE == kModeBatch ? moves[c] : draw_move(seed, ci, it, inst_index, V, P);
    const Move m = decode_move(w, V, P);
    const LaneOut o = eval_lane<N, SMALL, true>(V, P, s_base, m, 0, row0);
    const CandResult r = lane_result(o, ci, t_star, P.flags);
    lane_write<MODE>(c, r, out_key, out_cost, out_mk, out_flags);
    best = r.key < best ? r.key : best;
  }
  if (MODE != kModeBatch) wave_min_to(best, P.best_key);
  if (extra) {
    __syncthreads();
    winner_units(P, seed, inst_index, true);
  }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v) { *p = v; }

// Base preparation: optional eq. (6) pick (copy x* or x_old to the base
// slot), then the base view written into the instance image.  Run by one
// whole workgroup.
// The base view is built in LDS (`limg`, the image's size) from the
// static part staged there, and copied to the image in one coalesced pass
// at the end; sums over a BP's or a tour's positions are LDS integer
// atomics, one per position, so the result does not depend on their order.
__device__ void prepare_body(const InstParams &P, int mode, uint64_t seed, uint64_t eps_thr,
                             uint32_t inst_index, int &s_src, uint32_t *limg) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const ImageLayout &L = P.lay;
  for (uint32_t i = tid; i < L.static_words; i += nt) limg[i] = P.image[i];
  if (mode == kPrepSearch) {
    if (tid == 0) {
      const U4 w = philox4x32(U4{0u, P.st->it, inst_index, 1u}, (uint32_t)seed,
                              (uint32_t)(seed >> 32));
      const bool use_best = (uint64_t)w.x < eps_thr;
      P.st->use_best = use_best ? 1u : 0u;
      s_src = use_best ? 1 : 2;
    }
    __syncthreads();
    const DevSol &src = P.sol[s_src];
    const DevSol &dst = P.sol[0];
    for (int i = tid; i <= P.NT; i += nt) dst.tour_off[i] = src.tour_off[i];
    for (int i = tid; i < P.NB; i += nt) dst.tour_bp[i] = src.tour_bp[i];
    for (int i = tid; i <= P.NB; i += nt) dst.bp_off[i] = src.bp_off[i];
    for (int i = tid; i < P.NF; i += nt) dst.bp_field[i] = src.bp_field[i];
    for (int i = tid; i < P.NHU; i += nt) dst.hu_tour[i] = src.hu_tour[i];
    for (int i = tid; i < P.NSU; i += nt) dst.su_tour[i] = src.su_tour[i];
    __syncthreads();
  }
  const DevSol &x = P.sol[0];
  uint32_t *img = limg;
  uint16_t *seq = (uint16_t *)(img + L.seq), *pos = (uint16_t *)(img + L.pos);
  uint16_t *fbp = (uint16_t *)(img + L.fbp), *fidx = (uint16_t *)(img + L.fidx);
  uint16_t *bp_start = (uint16_t *)(img + L.bp_start), *bp_len = (uint16_t *)(img + L.bp_len);
  uint16_t *bp_tour = (uint16_t *)(img + L.bp_tour), *bp_idx = (uint16_t *)(img + L.bp_idx);
  uint16_t *tour_off = (uint16_t *)(img + L.tour_off), *tour_bp = (uint16_t *)(img + L.tour_bp);
  uint16_t *t_start = (uint16_t *)(img + L.t_start), *t_end = (uint16_t *)(img + L.t_end);
  uint4 *prec = (uint4 *)(img + L.prec);
  uint32_t *w_q = img + L.w_q;
  const uint32_t *f_area = img + L.area, *f_supply = img + L.supply, *f_nsh = img + L.nsh;
  const uint32_t *f_dhq = img + L.dhq, *demand = img + L.demand;
  const uint16_t *hu_rank = (const uint16_t *)(img + L.hu_rank);
  const uint16_t *su_rank = (const uint16_t *)(img + L.su_rank);
  uint32_t *b_sd = img + L.b_sd, *b_sup = img + L.b_sup, *b_area = img + L.b_area;
  uint32_t *b_int = img + L.b_int;
  unsigned long long *b_sh = (unsigned long long *)(img + L.b_sh);
  uint32_t *t_len = img + L.t_len, *t_area = img + L.t_area, *t_msum = img + L.t_msum;
  uint32_t *t_mcnt = img + L.t_mcnt;
  uint64_t *t_sh = (uint64_t *)(img + L.t_sh);
  unsigned long long *hu_mask = (unsigned long long *)(img + L.hu_mask);
  unsigned long long *su_mask = (unsigned long long *)(img + L.su_mask);

  // The base view's words start at zero (the sums and masks below add into them).
  for (uint32_t i = L.static_words + tid; i < L.total_words; i += nt) img[i] = 0u;
  __syncthreads();
  for (int i = tid; i <= P.NT; i += nt) tour_off[i] = x.tour_off[i];
  // The BP of each slot of the id-ordered field lists, kept for now in the
  // skip legs' words (written only after it is last read).
  uint32_t *owner = img + L.skip;
  for (int i = tid; i < P.NB; i += nt) {
    tour_bp[i] = x.tour_bp[i];
    const int o0 = x.bp_off[i], o1 = x.bp_off[i + 1];
    bp_len[i] = (uint16_t)(o1 - o0);
    for (int j = o0; j < o1; ++j) owner[j] = (uint32_t)i;
  }
  __syncthreads();
  if (tid == 0) {
    // BP start positions in tour order (serial prefix over the BPs).
    uint32_t run = 0;
    for (int g = 0; g < P.NT; ++g) {
      t_start[g] = (uint16_t)run;
      for (int j = tour_off[g]; j < tour_off[g + 1]; ++j) {
        const int b = tour_bp[j];
        bp_tour[b] = (uint16_t)g;
        bp_idx[b] = (uint16_t)(j - tour_off[g]);
        bp_start[b] = (uint16_t)run;
        run += bp_len[b];
      }
      t_end[g] = (uint16_t)run;
    }
    *P.best_key = kInfKey;
    if (mode == kPrepSearch && P.defer_cap) {   // the evaluation launch's deferred counts
      P.defer_cnt[0] = 0u;
      P.defer_cnt[1] = 0u;
    }
    if (P.rec) P.rec->valid = 0u;   // only this iteration's second pass may form the winner's units
  }
  __syncthreads();
  const uint32_t nb1 = 1u + (uint32_t)P.NB;
  for (int i = tid; i < P.NF; i += nt) {
    const int b = (int)owner[i];
    const int k = i - x.bp_off[b];
    const int f = x.bp_field[i];
    const int q = bp_start[b] + k;
    seq[q] = (uint16_t)f;
    pos[f] = (uint16_t)q;
    fbp[f] = (uint16_t)b;
    fidx[f] = (uint16_t)k;
    const uint32_t d = P.dist[(size_t)(nb1 + f) * P.V + 1 + b];
    prec[q].y = d;
    prec[q].z = f_area[f];
    prec[q].w = f_supply[f];
    w_q[q] = 2u * f_nsh[f] * d;
  }
  __syncthreads();
  // Per position: the leg into it, the leg that closes the route when its
  // field leaves, and its share of its BP's and tour's sums (every sum is
  // the one the full walk forms, over the same fields).
  for (int q = tid; q < P.NF; q += nt) {
    const int f = seq[q], b = fbp[f], g = bp_tour[b];
    const uint32_t a = q == 0 ? 0u : nb1 + seq[q - 1];
    const uint32_t leg = P.dist[(size_t)a * P.V + nb1 + f];
    prec[q].x = leg;
    const int po = q > (int)t_start[g] ? seq[q - 1] : -1, no = q + 1 < (int)t_end[g] ? seq[q + 1] : -1;
    img[L.skip + q] = po < 0 ? (no < 0 ? 0u : f_dhq[no])
                             : (no < 0 ? f_dhq[po] : P.dist[(size_t)(nb1 + po) * P.V + nb1 + no]);
    const uint4 r = prec[q];
    atomicAdd(&b_sd[b], r.y);
    atomicAdd(&b_area[b], r.z);
    atomicAdd(&b_sup[b], r.w);
    atomicAdd(&b_sh[b], (unsigned long long)w_q[q]);
    if (q > (int)bp_start[b]) atomicAdd(&b_int[b], leg);
    if (q > (int)t_start[g]) atomicAdd(&t_len[g], leg);
  }
  __syncthreads();
  for (int b = tid; b < P.NB; b += nt) {
    img[L.b_mean + b] = bp_len[b] ? b_sd[b] / bp_len[b] : 0u;
    // The leg that closes the route when the BP's fields leave it.
    uint32_t bridge = 0;
    if (bp_len[b]) {
      const int g = bp_tour[b], q0 = bp_start[b], q1 = q0 + bp_len[b];
      const int po = q0 > (int)t_start[g] ? seq[q0 - 1] : -1, no = q1 < (int)t_end[g] ? seq[q1] : -1;
      bridge = po < 0 ? (no < 0 ? 0u : f_dhq[no])
                      : (no < 0 ? f_dhq[po] : P.dist[(size_t)(nb1 + po) * P.V + nb1 + no]);
    }
    img[L.b_skip + b] = bridge;
  }
  for (int g = tid; g < P.NT; g += nt) {
    uint32_t ar = 0, ms = 0, mc = 0;
    uint64_t sh = 0;
    for (int j = tour_off[g]; j < tour_off[g + 1]; ++j) {
      const int b = tour_bp[j];
      ar += b_area[b];
      sh += b_sh[b];
      if (bp_len[b]) {
        ms += b_sd[b] / bp_len[b];
        mc += 1;
      }
    }
    const int q0 = t_start[g], q1 = t_end[g];
    // The legs between the tour's fields are summed above; the two legs to
    // and from HQ close the route.
    if (q1 > q0) t_len[g] += f_dhq[seq[q0]] + f_dhq[seq[q1 - 1]];
    t_area[g] = ar;
    t_sh[g] = sh;
    t_msum[g] = ms;
    t_mcnt[g] = mc;
  }
  if (tid == 0) {
    uint32_t v = 0;
    for (int b = 0; b < P.NB; ++b) v += b_sup[b] < demand[b] ? 1u : 0u;
    img[L.n_viol] = v;
  }
  // Unit masks per tour: one thread per unit sets its rank bit (bitwise OR,
  // so the order does not matter).
  for (int h = tid; h < P.NHU; h += nt) atomicOr(&hu_mask[x.hu_tour[h]], 1ull << hu_rank[h]);
  for (int u = tid; u < P.NSU; u += nt) {
    const int r = su_rank[u];
    atomicOr(&su_mask[2 * x.su_tour[u] + (r >> 6)], 1ull << (r & 63));
  }
  __syncthreads();
  for (uint32_t i = L.static_words + tid; i < L.total_words; i += nt) P.image[i] = img[i];
}

__global__ __launch_bounds__(1024) void k_prepare(InstParams P, int mode, uint64_t seed,
                                                  uint64_t eps_thr, uint32_t inst_index) {
  __shared__ int s_src;
  prepare_body(P, mode, seed, eps_thr, inst_index, s_src, reinterpret_cast<uint32_t *>(g_lds4));
}

// Moves for candidates first..first+n-1 (one thread each), read from the
// image in global memory.
__global__ void k_generate(InstParams P, uint64_t seed, uint32_t iter, uint32_t inst_index,
                           uint32_t first, uint32_t n, uint64_t *__restrict__ out) {
  const View V = make_view(P.image, P.lay, P.dist);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    out[i] = draw_move(seed, first + i, iter, inst_index, V, P);
}

__global__ void k_fill_u64(uint64_t *p, uint64_t v) { *p = v; }

__global__ void k_select(const uint64_t *__restrict__ keys, uint32_t n, uint64_t *out) {
  uint64_t best = kInfKey;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    best = k < best ? k : best;
  }
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t o = __shfl_xor((unsigned long long)best, off, 64);
    best = o < best ? o : best;
  }
  if ((threadIdx.x & 63) == 0 && best != kInfKey)
    atomicMin((unsigned long long *)out, (unsigned long long)best);
}

// Commit (one workgroup).  Start mode: the start of Algorithm 1, the base with
// a no-op move and the gate off becomes x* and x_old.  Step mode: the winner
// of the iteration is rebuilt from its draw, x_old <- x_new, and x* <- x_new
// on a strict decrease of C; one trace row.
// use_rec: the winner's units may come from the second lane pass's record
// (single-instance search and gather launches).
__device__ void commit_body(const InstParams &P, const View &V, int mode, uint64_t seed,
                            uint32_t inst_index, bool use_rec) {
  __shared__ uint64_t s_mv;
  __shared__ int s_win, s_improved;
  __shared__ uint64_t s_cost;
  __shared__ int64_t s_mk;
  const int tid = threadIdx.x, nt = blockDim.x;
  const uint32_t it = mode == kCommitStep ? P.st->it : 0u;
  const uint64_t bkey = mode == kCommitStep ? *P.best_key : 0ull;
  if (tid == 0) {
    if (mode == kCommitStart) {
      const int f0 = V.seq[0];
      s_mv = (uint64_t)f0 | ((uint64_t)V.fbp[f0] << 16) | ((uint64_t)V.fidx[f0] << 32);
      s_win = 1;
    } else if (bkey == kInfKey) {
      s_win = 0;
    } else {
      s_mv = draw_move(seed, (uint32_t)(bkey & 0xFFFFFFu), it, inst_index, V, P);
      s_win = 1;
    }
  }
  __syncthreads();
  const int win = s_win;
  const DevSol &base = P.sol[0];
  const DevSol &xo = P.sol[2];
  const DevSol &xb = P.sol[1];
  if (!win) {
    for (int i = tid; i <= P.NT; i += nt) xo.tour_off[i] = base.tour_off[i];
    for (int i = tid; i < P.NB; i += nt) xo.tour_bp[i] = base.tour_bp[i];
    for (int i = tid; i <= P.NB; i += nt) xo.bp_off[i] = base.bp_off[i];
    for (int i = tid; i < P.NF; i += nt) xo.bp_field[i] = base.bp_field[i];
    for (int i = tid; i < P.NHU; i += nt) xo.hu_tour[i] = base.hu_tour[i];
    for (int i = tid; i < P.NSU; i += nt) xo.su_tour[i] = base.su_tour[i];
    if (tid == 0) {
      SearchState *st = P.st;
      if (st->trace_rows < P.trace_cap) {
        TraceRow r;
        r.best_key = kInfKey;
        r.cost_m = st->cost_best;
        r.makespan_s = st->t_best;
        r.it = it;
        r.indicator = 0;
        r.use_best = (uint8_t)st->use_best;
        r.pad[0] = r.pad[1] = 0;
        P.trace[st->trace_rows] = r;
      }
      st->trace_rows += 1;
      st->it = it + 1;
    }
    return;
  }
  const Move m = decode_move(s_mv, V, P);
  // The winner's units from the second pass's record where it holds this
  // iteration's winner; else wave 0 evaluates the winner and writes them.
  const bool from_rec = use_rec && mode == kCommitStep && P.rec && P.rec->valid && P.rec->key == bkey &&
                        P.rec->it == it;
  if (from_rec) {
    const WinRec &w = *P.rec;
    for (int t = tid; t < P.NT; t += nt) {
      for (uint64_t mm = w.hm[t]; mm; mm &= mm - 1)
        xo.hu_tour[P.hu_id[__ffsll((unsigned long long)mm) - 1]] = (uint16_t)t;
      M128 sm{w.su_lo[t], w.su_hi[t]};
      while (!m_empty(sm)) xo.su_tour[P.su_id[m_pop_low(sm)]] = (uint16_t)t;
    }
    if (tid == 0) {
      s_cost = w.cost;
      s_mk = w.makespan;
    }
  } else if (tid < 64) {
    // Wave 0 evaluates the winner and writes its minimised units.
    const int S = P.seg;
    const int t = tid & (S - 1);
    const uint64_t seg_mask = S == 64 ? ~0ull : ((1ull << S) - 1ull);
    const int seg_base = tid & ~(S - 1);
    if (seg_base == 0) {
      const EvalOut o = (P.flags & kFullWalk) ? eval_candidate<true, 0>(V, P, m, t, S, seg_base, seg_mask)
                                              : eval_candidate<false, 0>(V, P, m, t, S, seg_base, seg_mask);
      if (t < P.NT) {
        for (uint64_t mm = o.hu_mask; mm; mm &= mm - 1)
          xo.hu_tour[P.hu_id[__ffsll((unsigned long long)mm) - 1]] = (uint16_t)t;
        M128 sm = o.su_mask;
        while (!m_empty(sm)) xo.su_tour[P.su_id[m_pop_low(sm)]] = (uint16_t)t;
      }
      if (t == 0) {
        s_cost = o.cost;
        s_mk = o.makespan;
      }
    }
  }
  // x_new = base with the move applied, into the x_old slot.
  if (m.kind == 0) {
    for (int i = tid; i <= P.NT; i += nt) xo.tour_off[i] = base.tour_off[i];
    for (int i = tid; i < P.NB; i += nt) xo.tour_bp[i] = base.tour_bp[i];
    for (int b = tid; b <= P.NB; b += nt)
      xo.bp_off[b] = (uint16_t)(base.bp_off[b] - (b > m.src ? 1 : 0) + (b > m.dst ? 1 : 0));
    __syncthreads();
    for (int i = tid; i < P.NF; i += nt) {
      int lo = 0, hi = P.NB;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int)xo.bp_off[mid] <= i) lo = mid; else hi = mid;
      }
      xo.bp_field[i] = (uint16_t)cand_field(V, m, lo, i - xo.bp_off[lo]);
    }
  } else {
    for (int i = tid; i <= P.NB; i += nt) xo.bp_off[i] = base.bp_off[i];
    for (int i = tid; i < P.NF; i += nt) xo.bp_field[i] = base.bp_field[i];
    for (int g = tid; g <= P.NT; g += nt)
      xo.tour_off[g] = (uint16_t)(base.tour_off[g] - (g > m.src ? 1 : 0) + (g > m.dst ? 1 : 0));
    __syncthreads();
    for (int i = tid; i < P.NB; i += nt) {
      int lo = 0, hi = P.NT;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int)xo.tour_off[mid] <= i) lo = mid; else hi = mid;
      }
      xo.tour_bp[i] = (uint16_t)cand_tour_bp(V, m, lo, i - xo.tour_off[lo]);
    }
  }
  __syncthreads();
  if (tid == 0) {
    SearchState *st = P.st;
    int improved = 0;
    if (mode == kCommitStart) {
      st->it = 0;
      st->n_improved = 0;
      st->trace_rows = 0;
      st->use_best = 0;
      st->cost_best = s_cost;
      st->t_best = s_mk;
      improved = 1;
    } else {
      if (s_cost < st->cost_best) {
        st->cost_best = s_cost;
        st->t_best = s_mk;
        st->n_improved += 1;
        improved = m.kind == 0 ? 1 : 2;
      }
      if (st->trace_rows < P.trace_cap) {
        TraceRow r;
        r.best_key = bkey;
        r.cost_m = st->cost_best;
        r.makespan_s = st->t_best;
        r.it = it;
        r.indicator = (uint8_t)improved;
        r.use_best = (uint8_t)st->use_best;
        r.pad[0] = r.pad[1] = 0;
        P.trace[st->trace_rows] = r;
      }
      st->trace_rows += 1;
      st->it = it + 1;
    }
    s_improved = improved;
  }
  __syncthreads();
  if (s_improved) {
    for (int i = tid; i <= P.NT; i += nt) xb.tour_off[i] = xo.tour_off[i];
    for (int i = tid; i < P.NB; i += nt) xb.tour_bp[i] = xo.tour_bp[i];
    for (int i = tid; i <= P.NB; i += nt) xb.bp_off[i] = xo.bp_off[i];
    for (int i = tid; i < P.NF; i += nt) xb.bp_field[i] = xo.bp_field[i];
    for (int i = tid; i < P.NHU; i += nt) xb.hu_tour[i] = xo.hu_tour[i];
    for (int i = tid; i < P.NSU; i += nt) xb.su_tour[i] = xo.su_tour[i];
  }
}

template <bool DLDS>
__global__ __launch_bounds__(256) void k_commit(InstParams P, int mode, uint64_t seed,
                                                uint32_t inst_index) {
  uint32_t *lds = reinterpret_cast<uint32_t *>(g_lds4);
  const uint32_t img_words = round4(P.lay.total_words);
  stage(lds, P.image, P.lay.total_words);
  if (DLDS) stage(lds + img_words, P.dist, (uint32_t)(P.V * P.V));
  __syncthreads();
  const View V = make_view(lds, P.lay, DLDS ? lds + img_words : P.dist);
  commit_body(P, V, mode, seed, inst_index, true);
}

// ------------------------------------------------- batches of instances --
// One iteration for K instances: a prepare and a commit workgroup per
// instance, and one persistent evaluation grid that pops (instance, tile)
// items from a device queue in the scheduled order.  A workgroup restages
// LDS only when its next item belongs to another instance.

__global__ void k_batch_reset(uint32_t *queue) {
  if (threadIdx.x == 0) queue[0] = 0u;
}

__global__ __launch_bounds__(256) void k_prepare_multi(BatchParams B, int mode) {
  __shared__ int s_src;
  const uint32_t k = blockIdx.x;
  prepare_body(B.inst[k], mode, B.seed, B.eps_thr, B.index_base + k, s_src, reinterpret_cast<uint32_t *>(g_lds4));
}

__global__ __launch_bounds__(256) void k_commit_multi(BatchParams B, int mode) {
  const uint32_t k = blockIdx.x;
  const InstParams &P = B.inst[k];
  uint32_t *lds = reinterpret_cast<uint32_t *>(g_lds4);
  stage(lds, P.image, P.lay.total_words);
  __syncthreads();
  const View V = make_view(lds, P.lay, P.dist);
  commit_body(P, V, mode, B.seed, B.index_base + k, false);
}

// The batched evaluation with one candidate per lane, for batches whose
// members all have at most N tours and 32-bit time bounds: a member's tours
// beyond its own count are empty and inactive (eval_lane's nt), so one
// instantiation serves members of any smaller tour count.  A candidate whose
// SU rounds run past kSuDeferRounds is queued in LDS (up to
// kLocalDefer per item) and evaluated again, densely, once the item's other
// candidates are done.
constexpr uint32_t kLocalDefer = 1024;

// QUEUE: the per-wave feasibility queue of k_eval_lane (the schedule's
// feas_queue; the autotuner times both).  It pays where many candidates break
// eq. (2) (batch256: 3.63 to 3.40 ms per iteration) and costs registers where
// few do (the paper-scale replica: 0.254 to 0.289 ms).
template <int N, bool SMALL, bool QUEUE>
__global__ __launch_bounds__(256, QUEUE ? kLaneWaves : 1) void k_eval_multi_lane(BatchParams B) {
  uint32_t *lds = reinterpret_cast<uint32_t *>(g_lds4);
  __shared__ uint32_t s_item, s_qn;
  __shared__ uint32_t s_q[kLocalDefer];
  __shared__ LaneBase s_base;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int cur = -1;
  while (true) {
    if (threadIdx.x == 0) {
      s_item = atomicAdd(B.queue, 1u);
      s_qn = 0;
    }
    __syncthreads();
    const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);  // uniform: scalar loads below
    if (item >= B.total_items) break;
    int lo = 0, hi = (int)B.K;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (B.item_off[mid] <= item) lo = mid; else hi = mid;
    }
    const uint32_t k = B.order[lo];
    const InstParams &P = B.inst[k];
    const View V = make_view(lds, P.lay, P.dist);
    if ((int)k != cur) {   // uniform over the workgroup
      stage(lds, P.image, P.lay.total_words);
      __syncthreads();
      lane_base_fill(s_base, V, P, P.NT);
      cur = (int)k;
    }
    __syncthreads();
    const uint32_t tile = B.tile[k];
    const uint32_t c0 = (item - B.item_off[lo]) * tile;
    const uint32_t c1 = c0 + tile < B.n ? c0 + tile : B.n;
    const uint32_t it = P.st->it;
    const int64_t t_star = P.st->t_best;
    const uint32_t idx = B.index_base + k;
    const int nt = P.NT;
    const int su_limit = kSuDeferRounds;
    uint64_t best = kInfKey;
    // A candidate whose SU rounds pass su_limit goes to the work item's tail
    // queue (or, when that is full, is finished here).  Without QUEUE each
    // lane takes the item's candidates in turn; with it, as in k_eval_lane,
    // each wave checks 64 candidates at a time for validity and eq. (2) and
    // evaluates the feasible ones 64 at a time from a queue in LDS.
    auto evaluate = [&](uint32_t c, uint64_t w) {
      const Move m = decode_move(w, V, P);
      LaneOut o;
      for (int lim = su_limit;; lim = 0) {
        o = eval_lane<N, SMALL>(V, P, s_base, m, lim);
        if (!o.deferred) break;
        const uint32_t slot = atomicAdd(&s_qn, 1u);
        if (slot < kLocalDefer) {
          s_q[slot] = c;
          return;
        }
      }
      if (o.feasible && !is_gated(o.makespan, t_star, P.flags)) {
        const uint64_t key = (o.cost << 24) | (uint64_t)c;
        best = key < best ? key : best;
      }
    };
    if constexpr (!QUEUE) {
      for (uint32_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
        const uint64_t w = draw_move(B.seed, c, it, idx, V, P);
        if (decode_move(w, V, P).valid) evaluate(c, w);
      }
    } else {
      __shared__ uint64_t s_qw[4][kLaneQueue];
      __shared__ uint32_t s_qc[4][kLaneQueue];
      uint64_t *qw = s_qw[wave];
      uint32_t *qc = s_qc[wave];
      uint32_t qn = 0;   // wave-uniform
      for (uint32_t i0 = c0 + (uint32_t)wave * 64u;; i0 += blockDim.x) {
        const bool more = i0 < c1;
        if (more) {
          const uint32_t c = i0 + (uint32_t)lane;
          bool feas = false;
          uint64_t w = 0;
          if (c < c1) {
            w = draw_move(B.seed, c, it, idx, V, P);
            const Move m = decode_move(w, V, P);
            feas = m.valid && delta_feasible(V, m);
          }
          const uint64_t bal = __ballot(feas);
          if (feas) {
            const uint32_t at = qn + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            qw[at] = w;
            qc[at] = c;
          }
          qn += (uint32_t)__popcll(bal);
        }
        while (qn >= 64u || (!more && qn > 0u)) {
          lane_wave_sync();
          const uint32_t take = qn < 64u ? qn : 64u;
          if ((uint32_t)lane < take) evaluate(qc[qn - take + lane], qw[qn - take + lane]);
          lane_wave_sync();
          qn -= take;
        }
        if (!more) break;
      }
    }
    __syncthreads();
    const uint32_t qd = s_qn < kLocalDefer ? s_qn : kLocalDefer;
    for (uint32_t i = threadIdx.x; i < qd; i += blockDim.x) {
      const uint32_t c = s_q[i];
      const Move m = decode_move(draw_move(B.seed, c, it, idx, V, P), V, P);
      const LaneOut o = eval_lane<N, SMALL>(V, P, s_base, m, 0);
      if (o.feasible && !is_gated(o.makespan, t_star, P.flags)) {
        const uint64_t key = (o.cost << 24) | (uint64_t)c;
        best = key < best ? key : best;
      }
    }
    wave_min_to(best, P.best_key);
    __syncthreads();
  }
}

template <bool WALK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_eval_multi(BatchParams B) {
  uint32_t *lds = reinterpret_cast<uint32_t *>(g_lds4);
  __shared__ uint32_t s_item;
  const int lane = threadIdx.x & 63;
  int cur = -1;
  while (true) {
    if (threadIdx.x == 0) s_item = atomicAdd(B.queue, 1u);
    __syncthreads();
    const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);  // uniform: scalar loads below
    if (item >= B.total_items) break;
    int lo = 0, hi = (int)B.K;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (B.item_off[mid] <= item) lo = mid; else hi = mid;
    }
    const uint32_t k = B.order[lo];
    const InstParams &P = B.inst[k];
    if ((int)k != cur) {
      stage(lds, P.image, P.lay.total_words);
      cur = (int)k;
    }
    __syncthreads();
    const View V = make_view(lds, P.lay, P.dist);
    const int S = P.seg;
    const int t = lane & (S - 1);
    const int seg_base = lane & ~(S - 1);
    const uint64_t seg_mask = S == 64 ? ~0ull : ((1ull << S) - 1ull);
    const uint32_t segs = (blockDim.x >> 6) * (uint32_t)(64 / S);
    const uint32_t wseg = (threadIdx.x >> 6) * (uint32_t)(64 / S) + (uint32_t)(lane / S);
    const uint32_t tile = B.tile[k];
    const uint32_t c0 = (item - B.item_off[lo]) * tile;
    const uint32_t c1 = c0 + tile < B.n ? c0 + tile : B.n;
    const uint32_t it = P.st->it;
    const int64_t t_star = P.st->t_best;
    const uint32_t idx = B.index_base + k;
    uint64_t best = kInfKey;
    for (uint32_t c = c0 + wseg; c < c1; c += segs) {
      const uint64_t w = draw_move(B.seed, c, it, idx, V, P);
      const CandResult r = eval_one<WALK>(V, P, w, c, t, S, seg_base, seg_mask, t_star);
      best = r.key < best ? r.key : best;
    }
    wave_min_to(best, P.best_key);
    __syncthreads();
  }
}

}  // namespace

size_t eval_lds_bytes(const InstParams &P) {
  size_t w = round4(P.lay.total_words);
  if (P.d_in_lds) w += (size_t)P.V * (size_t)P.V;
  return w * 4;
}

hipError_t launch_prepare(const InstParams &P, int mode, uint64_t seed, uint64_t eps_thr,
                          uint32_t inst_index, hipStream_t s) {
  hipLaunchKernelGGL(k_prepare, dim3(1), dim3(1024), (size_t)round4(P.lay.total_words) * 4, s, P, mode, seed, eps_thr,
                     inst_index);
  return hipGetLastError();
}

hipError_t launch_generate(const InstParams &P, uint64_t seed, uint32_t iter, uint32_t inst_index,
                           uint32_t first, uint32_t n, uint64_t *out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t blocks = (n + 255u) / 256u < 4096u ? (n + 255u) / 256u : 4096u;
  hipLaunchKernelGGL(k_generate, dim3(blocks), dim3(256), 0, s, P, seed, iter, inst_index, first,
                     n, out);
  return hipGetLastError();
}

// The instantiation for the instance: distance matrix in LDS or not, full
// walk or delta evaluation.
size_t lane_lds_bytes(const InstParams &P) { return (size_t)round4(P.lay.total_words) * 4; }
bool lane_small(const InstParams &P) { return P.NHU <= 32 && P.NSU <= 64; }

size_t lane_tail_lds_bytes(const InstParams &P, bool small) {
  return lane_lds_bytes(P) + (size_t)P.NT * 256 * (small ? ltbl_entry_bytes<true>() : ltbl_entry_bytes<false>());
}

template <int MODE, bool SMALL, class... A>
hipError_t launch_lane_tail(const InstParams &P, int grid, hipStream_t s, A... a) {
  const size_t lds = lane_tail_lds_bytes(P, SMALL);
  switch (P.NT) {
#define BL_TAIL_CASE(N) \
    case N: hipLaunchKernelGGL((k_eval_lane_tail<N, SMALL, MODE>), dim3(grid), dim3(256), lds, s, P, a...); break;
    BL_TAIL_CASE(1) BL_TAIL_CASE(2) BL_TAIL_CASE(3) BL_TAIL_CASE(4)
    BL_TAIL_CASE(5) BL_TAIL_CASE(6) BL_TAIL_CASE(7) BL_TAIL_CASE(8)
    BL_TAIL_CASE(9) BL_TAIL_CASE(10) BL_TAIL_CASE(11) BL_TAIL_CASE(12)
#undef BL_TAIL_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int MODE, bool SMALL, class... A>
hipError_t launch_lane_phase(const InstParams &P, int phase, int grid, hipStream_t s, A... a) {
  if (phase == 1 && P.lane_tail) return launch_lane_tail<MODE, SMALL>(P, grid, s, a...);
  const size_t lds = lane_lds_bytes(P);
  switch (P.NT) {
#define BL_LANE_CASE(N) \
    case N: hipLaunchKernelGGL((k_eval_lane<N, SMALL, MODE>), dim3(grid), dim3(256), lds, s, P, phase, a...); break;
    BL_LANE_CASE(1) BL_LANE_CASE(2) BL_LANE_CASE(3) BL_LANE_CASE(4)
    BL_LANE_CASE(5) BL_LANE_CASE(6) BL_LANE_CASE(7) BL_LANE_CASE(8)
    BL_LANE_CASE(9) BL_LANE_CASE(10) BL_LANE_CASE(11) BL_LANE_CASE(12)
#undef BL_LANE_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The two phases of one evaluation launch, the deferred list emptied first
// (by a kernel, so that the sequence can be captured in a graph).
template <int MODE, bool SMALL, class... A>
hipError_t launch_lane(const InstParams &P, int grid, hipStream_t s, A... a) {
  if (P.defer_cap && !P.defer_zeroed)
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(1), 0, s, reinterpret_cast<uint64_t *>(P.defer_cnt), 0ull);
  hipError_t e = launch_lane_phase<MODE, SMALL>(P, 0, grid, s, a...);
  if (e != hipSuccess || !P.defer_cap) return e;
  return launch_lane_phase<MODE, SMALL>(P, 1, grid, s, a...);
}

template <int MODE, class... A>
hipError_t launch_k_eval(const InstParams &P, int grid, hipStream_t s, A... a) {
  const size_t lds = eval_lds_bytes(P);
  if (lane_eval_on(P))
    return lane_small(P) ? launch_lane<MODE, true>(P, grid, s, a...) : launch_lane<MODE, false>(P, grid, s, a...);
  const bool walk = (P.flags & kFullWalk) != 0;
  if (P.d_in_lds) {
    if (walk)
      hipLaunchKernelGGL((k_eval<true, MODE, true>), dim3(grid), dim3(256), lds, s, P, a...);
    else
      hipLaunchKernelGGL((k_eval<true, MODE, false>), dim3(grid), dim3(256), lds, s, P, a...);
  } else {
    if (walk)
      hipLaunchKernelGGL((k_eval<false, MODE, true>), dim3(grid), dim3(256), lds, s, P, a...);
    else
      hipLaunchKernelGGL((k_eval<false, MODE, false>), dim3(grid), dim3(256), lds, s, P, a...);
  }
  return hipGetLastError();
}

// The instance's parameters for one evaluation launch: the second pass only
// where every lane takes at least two candidates in the first.  Below that
// the waves are few, and the extra launches cost more than the tails they
// would shorten (tiny12, 4096 candidates: 23 us in one pass, 36 us in two).
static InstParams pass_params(const InstParams &P, uint32_t n, int grid) {
  InstParams Q = P;
  if ((uint64_t)n < 2ull * (uint64_t)grid * 256ull) Q.defer_cap = 0;
  return Q;
}

// The deferred-candidate list (kStaticDeferCap words per class, two
// classes) and its counts of bl_evaluate_batch_static, for callers that
// cannot allocate: 8 MiB + 256 B that every GPU the library runs on holds
// until the process ends.  In host
// code `scratch` names a host-side stand-in; its device address comes from
// static_scratch_address, once per device.
static __device__ __align__(256) uint32_t scratch[2 * kStaticDeferCap + 64];

hipError_t static_scratch_address(uint32_t **out) {
  return hipGetSymbolAddress(reinterpret_cast<void **>(out), HIP_SYMBOL(scratch));
}

hipError_t launch_eval_batch(const InstParams &P, const uint64_t *moves, uint32_t n,
                             int64_t t_star, uint64_t *key, float *cost, int32_t *mk,
                             uint8_t *flags, int grid, hipStream_t s) {
  if (n == 0) return hipSuccess;
  return launch_k_eval<kModeBatch>(pass_params(P, n, grid), grid, s, moves, n, t_star, (uint64_t)0, (uint32_t)0, key, cost,
                                   mk, flags, (const uint32_t *)nullptr, (const uint32_t *)nullptr);
}

hipError_t launch_eval_search(const InstParams &P, uint64_t seed, uint32_t n,
                              uint32_t inst_index, int grid, hipStream_t s,
                              const uint32_t *run_flag, bool count_zeroed) {
  if (n == 0) return hipSuccess;
  InstParams Q = pass_params(P, n, grid);
  Q.defer_zeroed = count_zeroed ? 1u : 0u;
  return launch_k_eval<kModeSearch>(Q, grid, s, (const uint64_t *)nullptr, n, (int64_t)0, seed,
                                    inst_index, (uint64_t *)nullptr, (float *)nullptr,
                                    (int32_t *)nullptr, (uint8_t *)nullptr, (const uint32_t *)nullptr,
                                    run_flag);
}

hipError_t launch_eval_gather(const InstParams &P, uint64_t seed, const uint32_t *idx, uint32_t n,
                              uint32_t inst_index, uint64_t *key, float *cost, int grid,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  return launch_k_eval<kModeGather>(pass_params(P, n, grid), grid, s, (const uint64_t *)nullptr, n, (int64_t)0, seed,
                                    inst_index, key, cost, (int32_t *)nullptr, (uint8_t *)nullptr, idx,
                                    (const uint32_t *)nullptr);
}

hipError_t launch_commit(const InstParams &P, int mode, uint64_t seed, uint32_t inst_index,
                         hipStream_t s) {
  const size_t lds = eval_lds_bytes(P);
  if (P.d_in_lds)
    hipLaunchKernelGGL((k_commit<true>), dim3(1), dim3(256), lds, s, P, mode, seed, inst_index);
  else
    hipLaunchKernelGGL((k_commit<false>), dim3(1), dim3(256), lds, s, P, mode, seed, inst_index);
  return hipGetLastError();
}

hipError_t launch_select(const uint64_t *keys, uint32_t n, uint64_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(1), 0, s, out, kInfKey);
  if (n == 0) return hipGetLastError();
  const uint32_t blocks = (n + 255u) / 256u < 2048u ? (n + 255u) / 256u : 2048u;
  hipLaunchKernelGGL(k_select, dim3(blocks), dim3(256), 0, s, keys, n, out);
  return hipGetLastError();
}

bool lane_eval_on(const InstParams &P) {
  return P.narrow && P.NT >= 1 && P.NT <= kLaneMaxTours && !(P.flags & (kFullWalk | kWideKeys | kSegmentEval));
}

template <bool SMALL, int MODE>
int lane_occupancy(const InstParams &P, size_t lds) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (P.NT) {
#define BL_LANE_OCC(N) \
    case N: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval_lane<N, SMALL, MODE>, 256, lds); break;
    BL_LANE_OCC(1) BL_LANE_OCC(2) BL_LANE_OCC(3) BL_LANE_OCC(4)
    BL_LANE_OCC(5) BL_LANE_OCC(6) BL_LANE_OCC(7) BL_LANE_OCC(8)
    BL_LANE_OCC(9) BL_LANE_OCC(10) BL_LANE_OCC(11) BL_LANE_OCC(12)
#undef BL_LANE_OCC
    default: break;
  }
  return e == hipSuccess && nb > 0 ? nb : 1;
}

template <bool SMALL>
int lane_tail_occupancy(const InstParams &P, size_t lds) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (P.NT) {
#define BL_TAIL_OCC(N) \
    case N: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval_lane_tail<N, SMALL, kModeSearch>, 256, lds); break;
    BL_TAIL_OCC(1) BL_TAIL_OCC(2) BL_TAIL_OCC(3) BL_TAIL_OCC(4)
    BL_TAIL_OCC(5) BL_TAIL_OCC(6) BL_TAIL_OCC(7) BL_TAIL_OCC(8)
    BL_TAIL_OCC(9) BL_TAIL_OCC(10) BL_TAIL_OCC(11) BL_TAIL_OCC(12)
#undef BL_TAIL_OCC
    default: break;
  }
  return e == hipSuccess ? nb : 0;
}

bool lane_tail_on(const InstParams &P) {
  if (!lane_eval_on(P)) return false;
  if (const char *env = getenv("BL_LANE_TAIL"))
    if (atoi(env) == 0) return false;
  const bool small = lane_small(P);
  const size_t lds = lane_tail_lds_bytes(P, small);
  if (lds > 160 * 1024) return false;
  const int occ = small ? lane_tail_occupancy<true>(P, lds) : lane_tail_occupancy<false>(P, lds);
  return occ > 0 && occ >= eval_occupancy(P, true);
}

int eval_occupancy(const InstParams &P, bool search) {
  int nb = 0;
  const size_t lds = eval_lds_bytes(P);
  if (lane_eval_on(P)) {
    const size_t ll = lane_lds_bytes(P);
    if (lane_small(P)) return search ? lane_occupancy<true, kModeSearch>(P, ll) : lane_occupancy<true, kModeBatch>(P, ll);
    return search ? lane_occupancy<false, kModeSearch>(P, ll) : lane_occupancy<false, kModeBatch>(P, ll);
  }
  hipError_t e;
  const bool walk = (P.flags & kFullWalk) != 0;
  if (P.d_in_lds)
    e = walk ? (search ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval<true, kModeSearch, true>, 256, lds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval<true, kModeBatch, true>, 256, lds))
             : (search ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval<true, kModeSearch, false>, 256, lds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval<true, kModeBatch, false>, 256, lds));
  else
    e = walk ? (search ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval<false, kModeSearch, true>, 256, lds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval<false, kModeBatch, true>, 256, lds))
             : (search ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval<false, kModeSearch, false>, 256, lds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval<false, kModeBatch, false>, 256, lds));
  return e == hipSuccess && nb > 0 ? nb : 1;
}

size_t batch_lds_bytes(uint32_t max_image_words) { return (size_t)round4(max_image_words) * 4; }

template <int N, bool SMALL>
int multi_lane_occupancy(size_t lds, bool queue) {
  int nb = 0;
  const hipError_t e = queue ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval_multi_lane<N, SMALL, true>, 256, lds)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval_multi_lane<N, SMALL, false>, 256, lds);
  return e == hipSuccess && nb > 0 ? nb : 1;
}

int batch_occupancy(size_t lds, bool walk, int lane_n, bool lane_small, bool queue) {
  switch (lane_n) {
    case 4: return lane_small ? multi_lane_occupancy<4, true>(lds, queue) : multi_lane_occupancy<4, false>(lds, queue);
    case 8: return lane_small ? multi_lane_occupancy<8, true>(lds, queue) : multi_lane_occupancy<8, false>(lds, queue);
    case 12: return lane_small ? multi_lane_occupancy<12, true>(lds, queue) : multi_lane_occupancy<12, false>(lds, queue);
    default: break;
  }
  int nb = 0;
  const hipError_t e = walk ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval_multi<true>, 256, lds)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval_multi<false>, 256, lds);
  return e == hipSuccess && nb > 0 ? nb : 1;
}

int batch_lane_tours(int max_nt) { return max_nt <= 4 ? 4 : (max_nt <= 8 ? 8 : (max_nt <= kLaneMaxTours ? 12 : 0)); }

hipError_t launch_batch_start(const BatchParams &B, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_prepare_multi, dim3(B.K), dim3(256), lds, s, B, (int)kPrepFromBase);
  hipLaunchKernelGGL(k_commit_multi, dim3(B.K), dim3(256), lds, s, B, (int)kCommitStart);
  return hipGetLastError();
}

hipError_t launch_batch_eval(const BatchParams &B, int grid, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, B.queue);
  switch (B.lane_n) {
#define BL_MULTI_LANE(N) \
    case N: \
      if (B.feas_queue) { \
        if (B.lane_small) hipLaunchKernelGGL((k_eval_multi_lane<N, true, true>), dim3(grid), dim3(256), lds, s, B); \
        else hipLaunchKernelGGL((k_eval_multi_lane<N, false, true>), dim3(grid), dim3(256), lds, s, B); \
      } else { \
        if (B.lane_small) hipLaunchKernelGGL((k_eval_multi_lane<N, true, false>), dim3(grid), dim3(256), lds, s, B); \
        else hipLaunchKernelGGL((k_eval_multi_lane<N, false, false>), dim3(grid), dim3(256), lds, s, B); \
      } \
      return hipGetLastError();
    BL_MULTI_LANE(4) BL_MULTI_LANE(8) BL_MULTI_LANE(12)
#undef BL_MULTI_LANE
    default: break;
  }
  if (B.walk)
    hipLaunchKernelGGL(k_eval_multi<true>, dim3(grid), dim3(256), lds, s, B);
  else
    hipLaunchKernelGGL(k_eval_multi<false>, dim3(grid), dim3(256), lds, s, B);
  return hipGetLastError();
}

hipError_t launch_batch_prepare(const BatchParams &B, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_prepare_multi, dim3(B.K), dim3(256), lds, s, B, (int)kPrepSearch);
  return hipGetLastError();
}

hipError_t launch_batch_commit(const BatchParams &B, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(k_commit_multi, dim3(B.K), dim3(256), lds, s, B, (int)kCommitStep);
  return hipGetLastError();
}

}  // namespace bl
