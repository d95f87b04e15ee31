// One candidate per lane: the evaluation of device.h's segment version
// (eval_candidate, delta mode) with every tour of the candidate in registers
// of one lane instead of one tour per lane.  NTC is the instance's tour count
// (compile time, at most kLaneMaxTours); per-tour values live in arrays that
// the unrolled loops index with constants, and values of a tour picked at run
// time (g_max, g_min) are read by select chains.  The rules, ties and integer
// results are the segment version's, which the tests compare it with.
#pragma once

#include <type_traits>

#include "device.h"

namespace bl {

namespace {

constexpr int kLaneMaxTours = 12;

// Times in the rounds: 32-bit, which the instance's time bounds allow (the
// lane version runs only on instances whose completion and waiting times
// stay within (-2^26, 2^26), checked at upload); +inf and -inf are the
// extremes of the type.
using tm_t = int32_t;
constexpr tm_t kTInf = INT32_MAX, kTNegInf = INT32_MIN;

// Base values per tour, the same for every candidate of a launch (one copy
// per workgroup in LDS): rate sum of the tour's HUs, fill-time sum of its
// SUs, its critical SU, and its road time, completion time and waiting time
// with the base's units.  A move changes two tours; every other tour of a
// candidate starts from these values, and its waiting time stays the
// base's unless the HU rebalancing moves one of its HUs.
struct LaneBase {
  // The base's tour aggregates and unit masks, copied from the image so that
  // the evaluation addresses them at fixed offsets (a few scalar registers
  // fewer than the image's arrays need).  Zero beyond the instance's tours.
  uint64_t sh[kLaneMaxTours];     // shuttle distance
  uint64_t hu_mask[kLaneMaxTours];
  uint64_t su_lo[kLaneMaxTours], su_hi[kLaneMaxTours];
  uint32_t len[kLaneMaxTours], area[kLaneMaxTours], msum[kLaneMaxTours], mcnt[kLaneMaxTours];
  int32_t nf[kLaneMaxTours];      // fields
  uint32_t R[kLaneMaxTours];
  uint32_t load[kLaneMaxTours];
  int32_t top[kLaneMaxTours];  // critical SU (largest fill time) of the base, -1 without SUs
  uint32_t lc[kLaneMaxTours];  // floor(3600 L / v_HU)
  tm_t T[kLaneMaxTours];       // completion time (0 for an inactive tour)
  tm_t W[kLaneMaxTours];       // waiting time, eq. (5) (0 for an inactive tour)
  uint32_t dm[kLaneMaxTours];  // mean field-BP distance (Alg. 2), 0 without fields
  int32_t KT[kLaneMaxTours];   // rebalancing keys (lkey) of T and W
  int32_t KW[kLaneMaxTours];
  uint32_t actm;               // tours with fields
  uint32_t su_has;             // tours holding SUs
  uint64_t shsum;              // shuttle distance over all tours
  double rcp[kMaxHus + 1];   // rcp[k] = 1/k (k >= 1): the reciprocals udiv_small takes
};

__device__ __forceinline__ tm_t lane_tcompl(uint32_t lc, uint32_t A, uint32_t rate) {
  return rate == 0 ? kTInf : (tm_t)(lc + (uint32_t)udiv(3600ull * A, rate));
}

// Rebalancing keys: a tour's value and index in one 32-bit integer,
// (ord << 4) | (15 - t), where ord is the value clamped to [-2^26 - 1, 2^26].
// Every finite value lies strictly inside that range (the narrow bound), so
// the clamp only maps +inf to 2^26 and -inf to -2^26 - 1 and keeps the
// order; an inactive tour takes ord = -2^26 - 1, below every active tour.
// The largest key is then the lowest-index arg-max over active tours, and
// key ^ 15 orders equal values by increasing index (the arg-min's rule).
constexpr int32_t kOrdHi = 1 << 26, kOrdLo = -(1 << 26) - 1;
__device__ __forceinline__ int32_t lkey(tm_t v, int t) {
  const int32_t o = v < kOrdLo ? kOrdLo : (v > kOrdHi ? kOrdHi : v);
  return (int32_t)(((uint32_t)o << 4) | (uint32_t)(15 - t));
}
__device__ __forceinline__ int32_t lkey_inactive(int t) { return lkey(kOrdLo, t); }
__device__ __forceinline__ int32_t lkey_ord(int32_t k) { return k >> 4; }
__device__ __forceinline__ tm_t lord_value(int32_t o) {
  return o >= kOrdHi ? kTInf : (o <= kOrdLo ? kTNegInf : (tm_t)o);
}
__device__ __forceinline__ int32_t lmed3(int32_t a, int32_t b, int32_t c) {
  return max(min(a, b), min(max(a, b), c));
}
// Fills `B` for the tours 0..nt-1 of the base in V (zero and inactive
// beyond), and the reciprocal table.  Called by a whole workgroup; the caller
// synchronises before and after.
__device__ __forceinline__ void lane_base_fill(LaneBase &B, const View &V, const InstParams &P, int nt) {
  if (threadIdx.x < kLaneMaxTours) {
    const int t = threadIdx.x;
    uint32_t R = 0, ld = 0, lc = 0, nhu = 0, dm = 0;
    int top = -1;
    tm_t T = 0, W = 0;
    if (t < nt) {
      for (uint64_t mm = V.hu_mask[t]; mm; mm &= mm - 1) {
        R += V.hu_rate[__ffsll((unsigned long long)mm) - 1];
        ++nhu;
      }
      M128 sm{V.su_mask[2 * t], V.su_mask[2 * t + 1]};
      if (!m_empty(sm)) top = m_top(sm);
      while (!m_empty(sm)) ld += V.su_fill[m_pop_low(sm)];
      lc = (uint32_t)udiv(3600ull * V.t_len[t], P.v_hu);
      if ((int)V.t_end[t] > (int)V.t_start[t]) {
        T = lane_tcompl(lc, V.t_area[t], R);
        const uint32_t mc = V.t_mcnt[t];
        dm = mc ? V.t_msum[t] / mc : 0u;
        W = (top < 0 || nhu == 0) ? kTInf
                                  : (tm_t)udiv(7200ull * dm, V.su_speed[top]) - (tm_t)udiv(ld - V.su_fill[top], nhu);
      }
    }
    const bool live = t < nt;
    B.sh[t] = live ? V.t_sh[t] : 0ull;
    B.hu_mask[t] = live ? V.hu_mask[t] : 0ull;
    B.su_lo[t] = live ? V.su_mask[2 * t] : 0ull;
    B.su_hi[t] = live ? V.su_mask[2 * t + 1] : 0ull;
    B.len[t] = live ? V.t_len[t] : 0u;
    B.area[t] = live ? V.t_area[t] : 0u;
    B.msum[t] = live ? V.t_msum[t] : 0u;
    B.mcnt[t] = live ? V.t_mcnt[t] : 0u;
    B.nf[t] = live ? (int)V.t_end[t] - (int)V.t_start[t] : 0;
    B.R[t] = R;
    B.load[t] = ld;
    B.top[t] = top;
    B.lc[t] = lc;
    B.T[t] = T;
    B.W[t] = W;
    B.dm[t] = dm;
    const bool act = live && (int)V.t_end[t] > (int)V.t_start[t];
    B.KT[t] = act ? lkey(T, t) : lkey_inactive(t);
    B.KW[t] = act ? lkey(W, t) : lkey_inactive(t);
  }
  if (threadIdx.x == 0) {
    uint32_t actm = 0, su_has = 0;
    uint64_t shsum = 0;
    for (int t = 0; t < nt; ++t) {
      if ((int)V.t_end[t] > (int)V.t_start[t]) actm |= 1u << t;
      if ((V.su_mask[2 * t] | V.su_mask[2 * t + 1]) != 0) su_has |= 1u << t;
      shsum += V.t_sh[t];
    }
    B.actm = actm;
    B.su_has = su_has;
    B.shsum = shsum;
  }
  for (int k = threadIdx.x; k <= kMaxHus; k += blockDim.x) B.rcp[k] = k ? 1.0 / (double)k : 0.0;
}

// The value in a VGPR as far as the optimiser knows, so that a select
// chain over the tours stays a chain of selects instead of becoming an
// indexed load from a stack copy of the array.  lpick applies it to each
// step's result, which dies at once, so that it costs no register copy.
template <class T>
__device__ __forceinline__ T lopaque(T x) {
  __asm__ volatile("" : "+v"(x));
  return x;
}

template <int N, class T>
__device__ __forceinline__ T lpick(const T (&a)[N], int i) {
  T r = a[0];
#pragma unroll
  for (int k = 1; k < N; ++k) r = lopaque(i == k ? a[k] : r);
  return r;
}

// What a move changes in the base's tour aggregates: the legs it cuts and
// creates and the sums that travel with the moved field or BP (the segment
// version's tour_delta, formed once for both tours).
struct Change {
  bool any;
  int Ts, Td;
  int64_t dLs, dLd;
  uint32_t mv_area, mv_nf;
  uint64_t sh_out, sh_in;
  int32_t ms_s, ms_d, mc_s, mc_d;
};

__device__ __forceinline__ Change move_change(const View &V, const InstParams &P, const Move &m,
                                              const Nbrs &nb) {
  Change c;
  c.any = nb.first >= 0;
  const bool fm = m.kind == 0;
  c.Ts = fm ? (int)V.bp_tour[m.src] : m.src;
  c.Td = fm ? (int)V.bp_tour[m.dst] : m.dst;
  c.dLs = c.dLd = 0;
  c.mv_area = c.mv_nf = 0;
  c.sh_out = c.sh_in = 0;
  c.ms_s = c.ms_d = c.mc_s = c.mc_d = 0;
  if (!c.any) return c;
  const bool cross = fm && m.src != m.dst;
  const size_t nb1 = 1 + (size_t)P.NB;
  const uint32_t l_in = route_leg(V, P, nb.pnew, nb.first);
  const uint32_t l_out = route_leg(V, P, nb.last, nb.nnew);
  const uint32_t dfd = cross ? V.D[(nb1 + (size_t)m.v) * (size_t)P.V + 1 + (size_t)m.dst] : 0u;
  const uint32_t bridge = fm ? V.skip[nb.q0] : V.b_skip[m.v];
  const uint32_t lin = nb.pold < 0 ? V.dhq[nb.first] : V.prec[nb.q0].x;
  const uint32_t lout = nb.nold < 0 ? V.dhq[nb.last] : V.prec[nb.q1].x;
  const int64_t inner = fm ? 0 : (int64_t)V.b_int[m.v];
  uint32_t gap;
  if (nb.pnew == nb.pold && nb.nnew == nb.nold) {
    gap = bridge;
  } else if (nb.pnew < 0 || nb.nnew < 0) {
    gap = nb.pnew < 0 ? (nb.nnew < 0 ? 0u : V.dhq[nb.nnew]) : V.dhq[nb.pnew];
  } else {
    const int qn = V.pos[nb.nnew];
    gap = V.seq[qn - 1] == nb.pnew ? V.prec[qn].x : route_leg(V, P, nb.pnew, nb.nnew);
  }
  c.dLs = (int64_t)bridge - (int64_t)lin - (int64_t)lout - inner;
  c.dLd = (int64_t)l_in + (int64_t)l_out - (int64_t)gap + inner;
  if (fm) {
    const int f = m.v;
    c.mv_area = V.area[f];
    c.mv_nf = 1;
    c.sh_out = V.w_q[nb.q0];
    c.sh_in = cross ? 2ull * (uint64_t)V.nsh[f] * (uint64_t)dfd : c.sh_out;
    if (cross) {
      const int bs = m.src, bd = m.dst;
      const uint32_t cs = V.bp_len[bs], cd = V.bp_len[bd];
      c.ms_s = (int32_t)bp_mean(V.b_sd[bs] - V.prec[nb.q0].y, cs - 1) - (int32_t)V.b_mean[bs];
      c.mc_s = cs == 1 ? -1 : 0;
      c.ms_d = (int32_t)bp_mean(V.b_sd[bd] + dfd, cd + 1) - (int32_t)V.b_mean[bd];
      c.mc_d = cd == 0 ? 1 : 0;
    }
  } else {
    const int b = m.v;
    c.mv_area = V.b_area[b];
    c.mv_nf = V.bp_len[b];
    c.sh_out = c.sh_in = V.b_sh[b];
    c.ms_s = -(int32_t)V.b_mean[b];
    c.ms_d = (int32_t)V.b_mean[b];
    c.mc_s = -1;
    c.mc_d = 1;
  }
  return c;
}

__device__ __forceinline__ tm_t lane_twait(const View &V, const LaneBase &B, const M128 &msk, uint32_t ld,
                                           uint32_t nhu, uint32_t dm) {
  if (m_empty(msk) || nhu == 0) return kTInf;
  const int s = m_top(msk);
  const double r = B.rcp[nhu];
  return (tm_t)udiv(7200ull * dm, V.su_speed[s]) - (tm_t)udiv_small(ld - V.su_fill[s], nhu, r);
}

// The three largest keys, m1 >= m2 >= m3 (INT32_MIN where N is smaller).
template <int N>
__device__ __forceinline__ void lane_top3(const int32_t (&k)[N], int32_t &m1, int32_t &m2, int32_t &m3) {
  m1 = m2 = m3 = INT32_MIN;
#pragma unroll
  for (int t = 0; t < N; ++t) {
    const int32_t x = k[t];
    m3 = lmed3(m2, m3, x);
    m2 = lmed3(m1, m2, x);
    m1 = max(m1, x);
  }
}

struct LaneOut {
  uint64_t cost;
  int64_t makespan;
  uint32_t flags;
  bool feasible;
  bool deferred;   // stopped before its SU rounds were done (see su_limit)
};

__device__ __forceinline__ int lane_popc(uint32_t x) { return __popc(x); }
__device__ __forceinline__ int lane_popc(uint64_t x) { return __popcll((unsigned long long)x); }
__device__ __forceinline__ int lane_ffs(uint32_t x) { return __ffs(x); }
__device__ __forceinline__ int lane_ffs(uint64_t x) { return __ffsll((unsigned long long)x); }

// A lane's SU masks kept in LDS instead of registers: a table of N rows of
// 256 entries (one per thread of the workgroup), `row0` pointing at the
// lane's entry of row 0.  One 64-bit word per entry when SMALL, two
// otherwise.  Reading or writing a tour's mask is then one LDS access
// instead of a select over every tour; the banks a wave touches do not
// depend on the tours its lanes pick.
template <bool SMALL>
__device__ __forceinline__ M128 ltbl_get(const uint64_t *row0, int t) {
  if constexpr (SMALL) {
    return M128{row0[t * 256], 0ull};
  } else {
    const ulonglong2 x = reinterpret_cast<const ulonglong2 *>(row0)[t * 256];
    return M128{x.x, x.y};
  }
}
template <bool SMALL>
__device__ __forceinline__ void ltbl_set(uint64_t *row0, int t, const M128 &m) {
  if constexpr (SMALL)
    row0[t * 256] = m.lo;
  else
    reinterpret_cast<ulonglong2 *>(row0)[t * 256] = ulonglong2{m.lo, m.hi};
}
template <bool SMALL>
constexpr size_t ltbl_entry_bytes() { return SMALL ? 8 : 16; }

// SMALL: at most 32 HUs and 64 SUs, so that an HU mask is one 32-bit word
// and an SU mask one 64-bit word (the high half of M128 stays zero, which
// the compiler folds away).
//
// su_limit > 0: when the SU rounds would go past su_limit rounds the
// evaluation stops with `deferred` set and no result; the caller evaluates
// the candidate again later with su_limit = 0 (no limit).
//
// Tours from the instance's tour count up to N come from `B` as empty and
// inactive and as holding no units (lane_base_fill): they are then never
// g_max, g2 or a donor, add nothing to the cost, and the result is that of
// N = the tour count.
//
// TBL: the SU masks live in the LDS table at `row0` (ltbl_get) during the
// SU rounds; the rows are written at their start.
template <int N, bool SMALL, bool TBL = false>
__device__ __forceinline__ LaneOut eval_lane(const View &V, const InstParams &P, const LaneBase &B,
                                             const Move &m, int su_limit, uint64_t *row0 = nullptr) {
  using HM = typename std::conditional<SMALL, uint32_t, uint64_t>::type;
  LaneOut o;
  o.flags = 0;
  o.deferred = false;
  const Nbrs nb = move_nbrs(V, m);
  if (!delta_feasible(V, m)) {
    o.feasible = false;
    o.flags = kCandInfeasible;
    o.cost = 0;
    o.makespan = kInfT;
    return o;
  }
  o.feasible = true;
  const Change ch = move_change(V, P, m, nb);
  // ---- tours of the candidate ----
  // The move changes its two tours (one, when both ends lie in the same
  // tour); every other tour keeps the base's values.
  const int Ts = ch.Ts, Td = ch.Td;
  const bool same = Ts == Td;
  uint32_t LS = 0, LD = 0, AS = 0, AD = 0, dmS = 0, dmD = 0;
  uint32_t actm = B.actm;
  uint64_t shsum = B.shsum;
  if (ch.any) {
    const int64_t dS = ch.dLs + (same ? ch.dLd : 0), dD = ch.dLd + (same ? ch.dLs : 0);
    LS = (uint32_t)((int64_t)B.len[Ts] + dS);
    LD = (uint32_t)((int64_t)B.len[Td] + dD);
    AS = same ? B.area[Ts] : B.area[Ts] - ch.mv_area;
    AD = same ? B.area[Td] : B.area[Td] + ch.mv_area;
    const int32_t msS = ch.ms_s + (same ? ch.ms_d : 0), mcS = ch.mc_s + (same ? ch.mc_d : 0);
    const int32_t msD = ch.ms_d + (same ? ch.ms_s : 0), mcD = ch.mc_d + (same ? ch.mc_s : 0);
    const uint32_t ms1 = (uint32_t)((int32_t)B.msum[Ts] + msS), mc1 = (uint32_t)((int32_t)B.mcnt[Ts] + mcS);
    const uint32_t ms2 = (uint32_t)((int32_t)B.msum[Td] + msD), mc2 = (uint32_t)((int32_t)B.mcnt[Td] + mcD);
    dmS = mc1 ? ms1 / mc1 : 0u;
    dmD = mc2 ? ms2 / mc2 : 0u;
    const int nfS = B.nf[Ts] - (same ? 0 : (int)ch.mv_nf), nfD = B.nf[Td] + (same ? 0 : (int)ch.mv_nf);
    actm = (actm & ~(1u << Ts) & ~(1u << Td)) | ((nfS > 0 ? 1u : 0u) << Ts) | ((nfD > 0 ? 1u : 0u) << Td);
    shsum = shsum - ch.sh_out + ch.sh_in;
  }
  // Road and completion times of the two tours (the base's where the move
  // changes nothing).
  const uint32_t lcS = ch.any ? (uint32_t)udiv(3600ull * LS, P.v_hu) : 0u;
  const uint32_t lcD = ch.any ? (uint32_t)udiv(3600ull * LD, P.v_hu) : 0u;
  const int32_t ktS = ((actm >> Ts) & 1u) ? lkey(lane_tcompl(lcS, AS, B.R[Ts]), Ts) : lkey_inactive(Ts);
  const int32_t ktD = ((actm >> Td) & 1u) ? lkey(lane_tcompl(lcD, AD, B.R[Td]), Td) : lkey_inactive(Td);
  // One pass over the tours, so that the comparisons with the move's tours
  // die with it.
  uint32_t L[N], A[N], dm[N], lc[N];
  int32_t KT[N];   // rebalancing keys of the completion times (lkey)
#pragma unroll
  for (int t = 0; t < N; ++t) {
    const bool isS = ch.any && t == Ts, isD = ch.any && t == Td;
    L[t] = isS ? LS : (isD ? LD : B.len[t]);
    A[t] = isS ? AS : (isD ? AD : B.area[t]);
    dm[t] = isS ? dmS : (isD ? dmD : B.dm[t]);
    lc[t] = isS ? lcS : (isD ? lcD : B.lc[t]);
    KT[t] = isS ? ktS : (isD ? ktD : B.KT[t]);
  }
  HM hm[N];
  M128 sm[N];
  uint32_t R[N], load[N];
#pragma unroll
  for (int t = 0; t < N; ++t) {
    hm[t] = (HM)B.hu_mask[t];
    if constexpr (!TBL) sm[t] = M128{B.su_lo[t], SMALL ? 0ull : B.su_hi[t]};
    R[t] = B.R[t];
    load[t] = B.load[t];
  }
  const bool embedded = !(P.flags & kNoEmbeddedMin);
  // ---- HU min-max rebalancing: completion time ----
  uint32_t hu_moved = 0;   // tours whose HUs the rounds changed
  if (embedded) {
    uint32_t hasu = 0;   // tours holding HUs
#pragma unroll
    for (int t = 0; t < N; ++t)
      if (hm[t]) hasu |= 1u << t;
    int rounds = 0;
    while (true) {
      int32_t m1, m2, m3;
      lane_top3(KT, m1, m2, m3);
      if (lkey_ord(m1) <= kOrdLo) break;   // no active tour
      const int gmax = 15 - (m1 & 15);
      const int t2 = 15 - (m2 & 15);        // the tour of the second key (15: none)
      const bool has2 = lkey_ord(m2) > kOrdLo;
      const tm_t c2 = lord_value(lkey_ord(m2));
      const uint32_t nmax = hasu & ~(1u << gmax);
      const uint32_t d1 = has2 ? nmax & ~(1u << t2) : nmax;
      const uint32_t dmask = d1 ? d1 : nmax;
      int32_t kmin = INT32_MAX;
#pragma unroll
      for (int t = 0; t < N; ++t) kmin = min(kmin, ((dmask >> t) & 1u) ? (KT[t] ^ 15) : INT32_MAX);
      if (kmin == INT32_MAX) break;
      const int gmin = kmin & 15;
      if (rounds == (int)P.cap_hu) {
        o.flags |= kCandCapHu;
        break;
      }
      const HM hmin = lpick(hm, gmin);
      HM cands = hmin;
      const uint32_t lcx = lpick(lc, gmax);
      const uint32_t ax = lpick(A, gmax), rx = lpick(R, gmax);
      int u = 0;
      tm_t trial = 0;   // g_max's completion time with the unit tried last
      while (cands) {
        u = lane_ffs(cands) - 1;
        cands &= cands - 1;
        trial = (tm_t)(lcx + (uint32_t)udiv(3600ull * ax, rx + V.hu_rate[u]));
        if (!has2 || trial < c2 || cands == 0) break;
      }
      const uint32_t ru = V.hu_rate[u];
      const HM bit = (HM)1 << u;
      // The two tours that change, recomputed; an inactive g_min keeps its
      // key, and g_max's new time is the trial of the unit moved (rates are
      // positive).  The round is kept only if the largest time falls.
      const uint32_t Rmin = lpick(R, gmin) - ru, Rmax = rx + ru;
      const int32_t kmin1 = ((actm >> gmin) & 1u)
                                ? lkey(lane_tcompl(lpick(lc, gmin), lpick(A, gmin), Rmin), gmin)
                                : (kmin ^ 15);
      const int32_t kmax1 = lkey(trial, gmax);
      const int32_t rest = gmin == t2 ? m3 : m2;
      ++rounds;
      const bool keep = lkey_ord(max(rest, max(kmin1, kmax1))) < lkey_ord(m1);
#pragma unroll
      for (int t = 0; t < N; ++t) {
        const bool mn = keep && t == gmin, mx = keep && t == gmax;
        hm[t] = mn ? (hm[t] & ~bit) : (mx ? (hm[t] | bit) : hm[t]);
        R[t] = mn ? Rmin : (mx ? Rmax : R[t]);
        KT[t] = mn ? kmin1 : (mx ? kmax1 : KT[t]);
      }
      if (!keep) break;
      hasu |= 1u << gmax;
      if (!(hmin & ~bit)) hasu &= ~(1u << gmin);
      hu_moved |= (1u << gmin) | (1u << gmax);
    }
  }
  // Makespan: the largest completion time over active tours.
  int32_t kt_max = INT32_MIN;
#pragma unroll
  for (int t = 0; t < N; ++t) kt_max = max(kt_max, KT[t]);
  const tm_t tmax = lkey_ord(kt_max) <= kOrdLo ? kTNegInf : lord_value(lkey_ord(kt_max));
  // ---- SU min-max rebalancing, Alg. 2: waiting time ----
  // Waiting times: the base's, but for the move's two tours and the tours
  // whose HU count the rounds changed.  The SU masks are still the base's,
  // so a tour's critical SU and fill-time sum are the base's.  Per tour, the
  // HU count and the mean distance share one word (nhu << 25 | dm; dm < 2^24,
  // nhu <= 64), so that one select chain picks both.
  // The base's keys, recomputed for the move's two tours (inactive ones
  // take the inactive key) and the tours whose HU count changed.
  uint32_t nd[N];
  int32_t K[N];   // rebalancing keys of the waiting times (lkey)
#pragma unroll
  for (int t = 0; t < N; ++t) {
    nd[t] = dm[t] | ((uint32_t)lane_popc(hm[t]) << 25);
    K[t] = B.KW[t];
  }
  const uint32_t moved = ch.any ? (1u << Ts) | (1u << Td) : 0u;
  for (uint32_t redo = (hu_moved & actm) | moved; redo; redo &= redo - 1) {
    const int g = lane_ffs(redo) - 1;
    const uint32_t ndg = lpick(nd, g);
    const uint32_t nh = ndg >> 25;
    const int s = B.top[g];
    const tm_t Wg = (s < 0 || nh == 0) ? kTInf
                                       : (tm_t)udiv(7200ull * (ndg & 0x1FFFFFFu), V.su_speed[s]) -
                                             (tm_t)udiv_small(B.load[g] - V.su_fill[s], nh, B.rcp[nh]);
    const int32_t kg = ((actm >> g) & 1u) ? lkey(Wg, g) : lkey_inactive(g);
#pragma unroll
    for (int t = 0; t < N; ++t) K[t] = t == g ? kg : K[t];
  }
  if (embedded) {
    uint32_t hasu = 0;   // tours holding SUs
    if constexpr (TBL) {
      hasu = B.su_has;
#pragma unroll
      for (int t = 0; t < N; ++t) ltbl_set<SMALL>(row0, t, M128{B.su_lo[t], SMALL ? 0ull : B.su_hi[t]});
    } else {
#pragma unroll
      for (int t = 0; t < N; ++t)
        if (!m_empty(sm[t])) hasu |= 1u << t;
    }
    int rounds = 0;
    while (true) {
      int32_t m1, m2, m3;
      lane_top3(K, m1, m2, m3);
      if (lkey_ord(m1) <= kOrdLo) break;   // no active tour
      const int gmax = 15 - (m1 & 15);
      const int t2 = 15 - (m2 & 15);        // the tour of the second key (15: none)
      const bool has2 = lkey_ord(m2) > kOrdLo;
      const tm_t w2 = lord_value(lkey_ord(m2));
      // Donors: tours holding units outside {g_max, g2}, else outside
      // {g_max}; the arg-min of their keys (inactive tours lowest).
      const uint32_t nmax = hasu & ~(1u << gmax);
      const uint32_t d1 = has2 ? nmax & ~(1u << t2) : nmax;
      const uint32_t dmask = d1 ? d1 : nmax;
      int32_t kmin = INT32_MAX;
#pragma unroll
      for (int t = 0; t < N; ++t) kmin = min(kmin, ((dmask >> t) & 1u) ? (K[t] ^ 15) : INT32_MAX);
      if (kmin == INT32_MAX) break;
      const int gmin = kmin & 15;
      if (rounds == (int)P.cap_su) {
        o.flags |= kCandCapSu;
        break;
      }
      if (su_limit > 0 && rounds == su_limit) {
        o.deferred = true;
        return o;
      }
      M128 cands_all, smx;
      if constexpr (TBL) {
        cands_all = ltbl_get<SMALL>(row0, gmin);
        smx = ltbl_get<SMALL>(row0, gmax);
      } else {
        uint64_t slo[N], shi[N];
#pragma unroll
        for (int t = 0; t < N; ++t) {
          slo[t] = sm[t].lo;
          shi[t] = sm[t].hi;
        }
        cands_all = M128{lpick(slo, gmin), lpick(shi, gmin)};
        smx = M128{lpick(slo, gmax), lpick(shi, gmax)};
      }
      const int topx = m_empty(smx) ? -1 : m_top(smx);
      const uint32_t ndx = lpick(nd, gmax);
      const uint32_t ldx = lpick(load, gmax), nhx = ndx >> 25, dmx = ndx & 0x1FFFFFFu;
      const uint64_t rt_top = (nhx != 0 && topx >= 0) ? udiv(7200ull * dmx, V.su_speed[topx]) : 0ull;
      const double r_nhx = B.rcp[nhx];
      // The donor's units are tried in rank order: the first whose move takes
      // g_max's waiting time below w2 moves, else the last (without g2 the
      // first; without HUs every trial is infinite, so the last).  Each form
      // of the trial falls below w2 exactly when one integer of the unit
      // passes a bound formed once per round, so the scan compares integers
      // and only the chosen unit's waiting time is computed:
      //  - a unit ranked below g_max's critical SU topx leaves topx critical,
      //    trial = rt_top - floor((C + f_u) / nhx) with C = ldx - f_topx: below
      //    w2 iff f_u >= nhx * J - C, J = rt_top - w2 + 1 (every unit if J <= 0);
      //  - a unit ranked above it becomes critical, trial = floor(7200 dmx /
      //    v_u) - floor(ldx / nhx): below w2 iff K = w2 + floor(ldx / nhx) > 0
      //    and v_u >= floor(7200 dmx / K) + 1.
      // (All times are below 2^26 s here, so neither side wraps.)
      int u;
      {
        M128 cands = cands_all;
        if (!has2 || nhx == 0) {
          u = has2 ? m_top(cands) : m_pop_low(cands);
        } else {
          const int64_t J = (int64_t)rt_top - (int64_t)w2 + 1;
          const uint32_t C = topx >= 0 ? ldx - V.su_fill[topx] : 0u;
          const int64_t fa = J <= 0 ? 0 : (int64_t)nhx * J - (int64_t)C;
          const uint32_t fbound = fa <= 0 ? 0u : (fa >= (int64_t)UINT32_MAX ? UINT32_MAX : (uint32_t)fa);
          const int64_t Kb = (int64_t)w2 + (int64_t)udiv_small(ldx, nhx, r_nhx);
          const uint64_t vbound = Kb <= 0 ? ~0ull : udiv_wide(7200ull * dmx, (uint64_t)Kb) + 1ull;
          while (true) {
            u = m_pop_low(cands);
            const bool ok = u < topx ? V.su_fill[u] >= fbound : (uint64_t)V.su_speed[u] >= vbound;
            if (ok || m_empty(cands)) break;
          }
        }
      }
      tm_t trial = kTInf;   // g_max's waiting time with unit u
      if (nhx != 0) {
        const int s = u > topx ? u : topx;
        const uint64_t rt = u > topx ? udiv(7200ull * dmx, V.su_speed[u]) : rt_top;
        trial = (tm_t)rt - (tm_t)udiv_small(ldx + V.su_fill[u] - V.su_fill[s], nhx, r_nhx);
      }
      const uint32_t fu = V.su_fill[u];
      // The two tours after the move; the round is kept only if the largest
      // waiting time over active tours falls.  g_max's new time is the trial
      // of the unit moved (its critical SU is the larger of the two, its load
      // and HU count as in the trial); an inactive g_min keeps its key.
      const uint64_t ulo = (SMALL || u < 64) ? 1ull << u : 0ull, uhi = (SMALL || u < 64) ? 0ull : 1ull << (u - 64);
      const M128 smin_new{cands_all.lo & ~ulo, cands_all.hi & ~uhi}, smax_new{smx.lo | ulo, smx.hi | uhi};
      const uint32_t ldmin = lpick(load, gmin) - fu;
      const uint32_t ndmin = lpick(nd, gmin);
      const int32_t kmin1 = ((actm >> gmin) & 1u)
                                ? lkey(lane_twait(V, B, smin_new, ldmin, ndmin >> 25, ndmin & 0x1FFFFFFu), gmin)
                                : (kmin ^ 15);
      const int32_t kmax1 = lkey(trial, gmax);
      // The largest key outside {g_max, g_min}: m2, or m3 when g_min holds m2.
      const int32_t rest = gmin == t2 ? m3 : m2;
      ++rounds;
      const bool keep = lkey_ord(max(rest, max(kmin1, kmax1))) < lkey_ord(m1);
#pragma unroll
      for (int t = 0; t < N; ++t) {
        const bool mn = keep && t == gmin, mx = keep && t == gmax;
        if constexpr (!TBL) {
          sm[t].lo = mn ? smin_new.lo : (mx ? smax_new.lo : sm[t].lo);
          sm[t].hi = mn ? smin_new.hi : (mx ? smax_new.hi : sm[t].hi);
        }
        load[t] = mn ? ldmin : (mx ? ldx + fu : load[t]);
        K[t] = mn ? kmin1 : (mx ? kmax1 : K[t]);
      }
      if constexpr (TBL) {
        if (keep) {
          ltbl_set<SMALL>(row0, gmin, smin_new);
          ltbl_set<SMALL>(row0, gmax, smax_new);
        }
      }
      if (!keep) break;
      hasu |= 1u << gmax;
      if (m_empty(smin_new)) hasu &= ~(1u << gmin);
    }
  }
  // ---- path length (sec. 2.2) ----
  uint64_t cost = shsum;
#pragma unroll
  for (int t = 0; t < N; ++t) {
    M128 st;
    if constexpr (TBL)
      st = embedded ? ltbl_get<SMALL>(row0, t) : M128{B.su_lo[t], SMALL ? 0ull : B.su_hi[t]};
    else
      st = sm[t];
    cost += (uint64_t)(lane_popc(hm[t]) + m_pop(st)) * (uint64_t)L[t];
  }
  o.cost = cost;
  o.makespan = tmax == kTInf ? kInfT : (tmax == kTNegInf ? kNegInfT : (int64_t)tmax);
  if (tmax == kTInf) o.flags |= kCandInfMakespan;
  return o;
}

}  // namespace

}  // namespace bl
