// gfx950 kernels of the candidate evaluator: base preparation, Step 8 move
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

namespace bl {

namespace {

// ------------------------------------------------------------- Philox ----
// Philox4x32-10 (Salmon et al., SC'11).
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ uint32_t scale_word(uint32_t w, uint32_t m) { return __umulhi(w, m); }

// Exact floor(p / q) for p + q < 2^53 (p, q >= 0, q > 0): the correctly
// rounded double quotient cannot reach the next integer below that bound.
__device__ __forceinline__ uint64_t udiv(uint64_t p, uint32_t q) {
  return (uint64_t)((double)p / (double)q);
}

// --------------------------------------------------------- the LDS view --
struct View {
  const uint32_t *area, *supply, *nsh, *dhq, *demand, *hu_rate, *su_fill, *su_speed;
  const uint16_t *hu_rank, *su_rank;
  const uint16_t *seq, *pos, *fbp, *fidx, *bp_start, *bp_len, *bp_tour, *bp_idx, *tour_off, *tour_bp;
  const uint32_t *leg_in, *dfb;
  const uint64_t *hu_mask, *su_mask;
  const uint32_t *D;
};

__device__ __forceinline__ View make_view(const uint32_t *img, const ImageLayout &L,
                                          const uint32_t *D) {
  View v;
  v.area = img + L.area;
  v.supply = img + L.supply;
  v.nsh = img + L.nsh;
  v.dhq = img + L.dhq;
  v.demand = img + L.demand;
  v.hu_rate = img + L.hu_rate;
  v.su_fill = img + L.su_fill;
  v.su_speed = img + L.su_speed;
  v.hu_rank = (const uint16_t *)(img + L.hu_rank);
  v.su_rank = (const uint16_t *)(img + L.su_rank);
  v.seq = (const uint16_t *)(img + L.seq);
  v.pos = (const uint16_t *)(img + L.pos);
  v.fbp = (const uint16_t *)(img + L.fbp);
  v.fidx = (const uint16_t *)(img + L.fidx);
  v.leg_in = img + L.leg_in;
  v.dfb = img + L.dfb;
  v.bp_start = (const uint16_t *)(img + L.bp_start);
  v.bp_len = (const uint16_t *)(img + L.bp_len);
  v.bp_tour = (const uint16_t *)(img + L.bp_tour);
  v.bp_idx = (const uint16_t *)(img + L.bp_idx);
  v.tour_off = (const uint16_t *)(img + L.tour_off);
  v.tour_bp = (const uint16_t *)(img + L.tour_bp);
  v.hu_mask = (const uint64_t *)(img + L.hu_mask);
  v.su_mask = (const uint64_t *)(img + L.su_mask);
  v.D = D;
  return v;
}

// ---------------------------------------------------------------- moves --
struct Move {
  int kind;  // 0 field, 1 BP
  int v;     // field id or BP id
  int dst;   // destination BP (field) or tour (BP)
  int slot;  // position in the destination list after the removal
  int src;   // BP of the field / tour of the BP in the base
  int r;     // index of the vertex in its base list
  bool valid;
};

__device__ __forceinline__ int tour_len(const View &V, int g) {
  return (int)V.tour_off[g + 1] - (int)V.tour_off[g];
}

__device__ __forceinline__ Move decode_move(uint64_t w, const View &V, const InstParams &P) {
  Move m;
  m.v = (int)(w & 0x7FFF);
  m.kind = (int)((w >> 15) & 1);
  m.dst = (int)((w >> 16) & 0xFFFF);
  m.slot = (int)((w >> 32) & 0xFFFF);
  m.src = 0;
  m.r = 0;
  if (m.kind == 0) {
    m.valid = m.v < P.NF && m.dst < P.NB;
    if (m.valid) {
      m.src = V.fbp[m.v];
      m.r = V.fidx[m.v];
      const int room = (int)V.bp_len[m.dst] - (m.dst == m.src ? 1 : 0);
      m.valid = m.slot <= room;
    }
  } else {
    m.valid = m.v < P.NB && m.dst < P.NT;
    if (m.valid) {
      m.src = V.bp_tour[m.v];
      m.r = V.bp_idx[m.v];
      const int room = tour_len(V, m.dst) - (m.dst == m.src ? 1 : 0);
      m.valid = m.slot <= room;
    }
  }
  return m;
}

// Step 8 draw of candidate i of iteration `it` (counter (i, it, inst, 0)).
__device__ __forceinline__ uint64_t draw_move(uint64_t seed, uint32_t i, uint32_t it,
                                              uint32_t inst_index, const View &V,
                                              const InstParams &P) {
  const U4 w = philox4x32(U4{i, it, inst_index, 0u}, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint32_t v = scale_word(w.x, (uint32_t)(P.NF + P.NB));
  uint32_t kind, vert, dst, room, src;
  if (v < (uint32_t)P.NF) {
    kind = 0;
    vert = v;
    src = V.fbp[v];
    dst = (P.flags & kFixedFieldBp) ? src : scale_word(w.y, (uint32_t)P.NB);
    room = V.bp_len[dst] - (dst == src ? 1u : 0u);
  } else {
    kind = 1;
    vert = v - (uint32_t)P.NF;
    src = V.bp_tour[vert];
    dst = scale_word(w.y, (uint32_t)P.NT);
    room = (uint32_t)tour_len(V, (int)dst) - (dst == src ? 1u : 0u);
  }
  const uint32_t slot = scale_word(w.z, room + 1u);
  return (uint64_t)vert | ((uint64_t)kind << 15) | ((uint64_t)dst << 16) | ((uint64_t)slot << 32);
}

// Element j of tour g's BP list in the candidate.
__device__ __forceinline__ int cand_tour_bp(const View &V, const Move &m, int g, int j) {
  if (m.kind == 1) {
    if (g == m.dst) {
      if (j == m.slot) return m.v;
      if (j > m.slot) j -= 1;
    }
    if (g == m.src && j >= m.r) j += 1;
  }
  return V.tour_bp[V.tour_off[g] + j];
}

__device__ __forceinline__ int cand_tour_len(const View &V, const Move &m, int g) {
  int n = tour_len(V, g);
  if (m.kind == 1) n += (g == m.dst ? 1 : 0) - (g == m.src ? 1 : 0);
  return n;
}

__device__ __forceinline__ int cand_bp_len(const View &V, const Move &m, int b) {
  int n = V.bp_len[b];
  if (m.kind == 0) n += (b == m.dst ? 1 : 0) - (b == m.src ? 1 : 0);
  return n;
}

// Element k of BP b's field list in the candidate: field id and its base position.
__device__ __forceinline__ void cand_field(const View &V, const Move &m, int b, int k, int &f,
                                           int &q) {
  if (m.kind == 0) {
    if (b == m.dst) {
      if (k == m.slot) {
        f = m.v;
        q = V.pos[f];
        return;
      }
      if (k > m.slot) k -= 1;
    }
    if (b == m.src && k >= m.r) k += 1;
  }
  q = V.bp_start[b] + k;
  f = V.seq[q];
}

// ------------------------------------------------- segment reductions --
// (value, tour) packed so that one unsigned max / min is the arg-max /
// arg-min with the lowest tour winning ties.  Values live in (-2^57, 2^57).
constexpr int64_t kValOff = (int64_t)1 << 57;
constexpr int64_t kValInf = ((int64_t)1 << 57) - 1;   // +inf inside the packing
constexpr int64_t kValNegInf = -((int64_t)1 << 57) + 1;

__device__ __forceinline__ int64_t clampv(int64_t v) {
  return v == kInfT ? kValInf : (v == kNegInfT ? kValNegInf : v);
}
__device__ __forceinline__ int64_t unclampv(int64_t v) {
  return v == kValInf ? kInfT : (v == kValNegInf ? kNegInfT : v);
}
__device__ __forceinline__ uint64_t pack_max(int64_t v, int t) {
  return ((uint64_t)(clampv(v) + kValOff) << 6) | (uint64_t)(63 - t);
}
__device__ __forceinline__ uint64_t pack_min(int64_t v, int t) {
  return ((uint64_t)(clampv(v) + kValOff) << 6) | (uint64_t)t;
}
__device__ __forceinline__ int64_t unpack_val(uint64_t k) {
  return unclampv((int64_t)(k >> 6) - kValOff);
}
__device__ __forceinline__ int unpack_max_t(uint64_t k) { return 63 - (int)(k & 63); }
__device__ __forceinline__ int unpack_min_t(uint64_t k) { return (int)(k & 63); }

__device__ __forceinline__ uint64_t seg_max_u64(uint64_t v, int S) {
  for (int off = 1; off < S; off <<= 1) {
    const uint64_t o = __shfl_xor((unsigned long long)v, off, S);
    v = o > v ? o : v;
  }
  return v;
}
__device__ __forceinline__ uint64_t seg_min_u64(uint64_t v, int S) {
  for (int off = 1; off < S; off <<= 1) {
    const uint64_t o = __shfl_xor((unsigned long long)v, off, S);
    v = o < v ? o : v;
  }
  return v;
}
__device__ __forceinline__ uint64_t seg_sum_u64(uint64_t v, int S) {
  for (int off = 1; off < S; off <<= 1) v += __shfl_xor((unsigned long long)v, off, S);
  return v;
}
__device__ __forceinline__ uint64_t bcast_u64(uint64_t v, int t, int S) {
  return __shfl((unsigned long long)v, t, S);
}
__device__ __forceinline__ int64_t bcast_i64(int64_t v, int t, int S) {
  return __shfl((long long)v, t, S);
}
__device__ __forceinline__ uint32_t bcast_u32(uint32_t v, int t, int S) {
  return __shfl(v, t, S);
}
// Bits of this lane's segment in a wave ballot, shifted down to bit 0.
__device__ __forceinline__ uint64_t seg_ballot(bool p, int seg_base, uint64_t seg_mask) {
  return (__ballot(p) >> seg_base) & seg_mask;
}

// ------------------------------------------------------ unit masks ------
struct M128 {
  uint64_t lo, hi;
};
__device__ __forceinline__ bool m_empty(const M128 &m) { return (m.lo | m.hi) == 0; }
__device__ __forceinline__ int m_top(const M128 &m) {
  return m.hi ? 127 - __clzll(m.hi) : 63 - __clzll(m.lo);
}
__device__ __forceinline__ int m_pop(const M128 &m) { return __popcll(m.lo) + __popcll(m.hi); }
__device__ __forceinline__ void m_set(M128 &m, int k) {
  if (k < 64) m.lo |= 1ull << k; else m.hi |= 1ull << (k - 64);
}
__device__ __forceinline__ void m_clear(M128 &m, int k) {
  if (k < 64) m.lo &= ~(1ull << k); else m.hi &= ~(1ull << (k - 64));
}
// Remove and return the lowest set bit.
__device__ __forceinline__ int m_pop_low(M128 &m) {
  if (m.lo) {
    const int k = __ffsll((unsigned long long)m.lo) - 1;
    m.lo &= m.lo - 1;
    return k;
  }
  const int k = __ffsll((unsigned long long)m.hi) - 1;
  m.hi &= m.hi - 1;
  return 64 + k;
}

// ------------------------------------------------- candidate evaluation --
struct EvalOut {
  uint64_t cost;     // path length, metres
  int64_t makespan;  // max completion time over active tours, s (kInfT if infinite)
  uint32_t flags;
  bool feasible;
  // per lane (tour t): final units
  uint64_t hu_mask;
  M128 su_mask;
};

__device__ __forceinline__ uint32_t leg_between(const View &V, const InstParams &P, int fprev,
                                                int qprev, int f, int q) {
  if (fprev < 0) return V.dhq[f];
  if (q == qprev + 1) return V.leg_in[q];
  const int nb1 = 1 + P.NB;
  return V.D[(size_t)(nb1 + fprev) * (size_t)P.V + (size_t)(nb1 + f)];
}

// Evaluate one candidate on the S lanes of a segment (lane t owns tour t).
// `gate`: 0 = off, 1 = discard when makespan > t_star, 2 = when >= t_star.
__device__ EvalOut eval_candidate(const View &V, const InstParams &P, const Move &m, int t,
                                  int S, int seg_base, uint64_t seg_mask) {
  EvalOut o;
  o.flags = 0;
  const bool lane_tour = t < P.NT;
  // ---- walk of tour t: length, area, shuttles, per-BP means, eq. (2) ----
  uint32_t L = 0, A = 0, sum_mean = 0, n_mean = 0;
  uint64_t shuttle = 0;
  bool feas = true, act = false;
  if (lane_tour) {
    const int nbt = cand_tour_len(V, m, t);
    int fprev = -1, qprev = -2;
    for (int j = 0; j < nbt; ++j) {
      const int b = cand_tour_bp(V, m, t, j);
      const int nfb = cand_bp_len(V, m, b);
      uint32_t sd = 0, sup = 0;
      for (int k = 0; k < nfb; ++k) {
        int f, q;
        cand_field(V, m, b, k, f, q);
        L += leg_between(V, P, fprev, qprev, f, q);
        uint32_t dfb;
        if (m.kind == 0 && f == m.v && m.dst != m.src)
          dfb = V.D[(size_t)(1 + P.NB + f) * (size_t)P.V + (size_t)(1 + b)];
        else
          dfb = V.dfb[q];
        A += V.area[f];
        sup += V.supply[f];
        sd += dfb;
        shuttle += 2ull * (uint64_t)V.nsh[f] * (uint64_t)dfb;
        fprev = f;
        qprev = q;
      }
      if (nfb > 0) {
        sum_mean += sd / (uint32_t)nfb;
        n_mean += 1;
      }
      feas = feas && sup >= V.demand[b];
    }
    if (fprev >= 0) {
      L += V.dhq[fprev];
      act = true;
    }
  }
  o.feasible = seg_ballot(!feas, seg_base, seg_mask) == 0;
  uint64_t hm = lane_tour ? V.hu_mask[t] : 0ull;
  M128 sm = lane_tour ? M128{V.su_mask[2 * t], V.su_mask[2 * t + 1]} : M128{0ull, 0ull};
  if (!o.feasible) {
    o.flags = kCandInfeasible;
    o.cost = 0;
    o.makespan = kInfT;
    o.hu_mask = hm;
    o.su_mask = sm;
    return o;
  }
  const bool embedded = !(P.flags & kNoEmbeddedMin);
  // ---- HU min-max rebalancing: completion time ----
  const uint64_t lc = udiv(3600ull * L, P.v_hu);  // road part of the completion time
  uint32_t R = 0;
  for (uint64_t mm = hm; mm; mm &= mm - 1) R += V.hu_rate[__ffsll((unsigned long long)mm) - 1];
  auto tcompl = [&](uint32_t rate) -> int64_t {
    return rate == 0 ? kInfT : (int64_t)(lc + udiv(3600ull * A, rate));
  };
  int64_t T = act ? tcompl(R) : 0;
  if (embedded) {
    int rounds = 0;
    while (true) {
      const uint64_t kx = seg_max_u64(act ? pack_max(T, t) : 0ull, S);
      if (kx == 0) break;
      const int gmax = unpack_max_t(kx);
      const int64_t top = unpack_val(kx);
      const uint64_t k2 = seg_max_u64((act && t != gmax) ? pack_max(T, t) : 0ull, S);
      const bool has2 = k2 != 0;
      const int g2 = has2 ? unpack_max_t(k2) : -1;
      const int64_t t2 = has2 ? unpack_val(k2) : 0;
      const bool hasu = hm != 0;
      uint64_t dm = seg_ballot(hasu && t != gmax && t != g2, seg_base, seg_mask);
      if (!dm) dm = seg_ballot(hasu && t != gmax, seg_base, seg_mask);
      if (!dm) break;
      if (rounds == (int)P.cap_hu) {
        o.flags |= kCandCapHu;
        break;
      }
      const bool donor = (dm >> t) & 1;
      const uint64_t kn = seg_min_u64(donor ? pack_min(act ? T : kNegInfT, t) : ~0ull, S);
      const int gmin = unpack_min_t(kn);
      uint64_t cands = bcast_u64(hm, gmin, S);
      const uint64_t lcx = bcast_u64(lc, gmax, S);
      const uint32_t ax = bcast_u32(A, gmax, S);
      const uint32_t rx = bcast_u32(R, gmax, S);
      int u = 0;
      while (cands) {
        u = __ffsll((unsigned long long)cands) - 1;
        cands &= cands - 1;
        const int64_t trial = (int64_t)(lcx + udiv(3600ull * ax, rx + V.hu_rate[u]));
        if (!has2 || trial < t2 || cands == 0) break;
      }
      const uint32_t ru = V.hu_rate[u];
      if (t == gmin) { hm &= ~(1ull << u); R -= ru; }
      if (t == gmax) { hm |= 1ull << u; R += ru; }
      if (act) T = tcompl(R);
      ++rounds;
      const int64_t ntop = unpack_val(seg_max_u64(act ? pack_max(T, t) : 0ull, S));
      if (ntop < top) continue;
      if (t == gmin) { hm |= 1ull << u; R += ru; }
      if (t == gmax) { hm &= ~(1ull << u); R -= ru; }
      if (act) T = tcompl(R);
      break;
    }
  }
  const int64_t tmax = unpack_val(seg_max_u64(act ? pack_max(T, t) : 0ull, S));
  // ---- SU min-max rebalancing, Alg. 2: waiting time ----
  const uint32_t nhu = (uint32_t)__popcll(hm);
  const uint32_t dm_t = n_mean ? sum_mean / n_mean : 0u;
  uint32_t load = 0;
  {
    M128 mm = sm;
    while (!m_empty(mm)) load += V.su_fill[m_pop_low(mm)];
  }
  auto twait = [&](const M128 &msk, uint32_t ld) -> int64_t {
    if (m_empty(msk) || nhu == 0) return kInfT;
    const int s = m_top(msk);
    return (int64_t)udiv(7200ull * dm_t, V.su_speed[s]) - (int64_t)((ld - V.su_fill[s]) / nhu);
  };
  if (embedded) {
    int64_t W = act ? twait(sm, load) : 0;
    int rounds = 0;
    while (true) {
      const uint64_t kx = seg_max_u64(act ? pack_max(W, t) : 0ull, S);
      if (kx == 0) break;
      const int gmax = unpack_max_t(kx);
      const int64_t top = unpack_val(kx);
      const uint64_t k2 = seg_max_u64((act && t != gmax) ? pack_max(W, t) : 0ull, S);
      const bool has2 = k2 != 0;
      const int g2 = has2 ? unpack_max_t(k2) : -1;
      const int64_t w2 = has2 ? unpack_val(k2) : 0;
      const bool hasu = !m_empty(sm);
      uint64_t dmk = seg_ballot(hasu && t != gmax && t != g2, seg_base, seg_mask);
      if (!dmk) dmk = seg_ballot(hasu && t != gmax, seg_base, seg_mask);
      if (!dmk) break;
      if (rounds == (int)P.cap_su) {
        o.flags |= kCandCapSu;
        break;
      }
      const bool donor = (dmk >> t) & 1;
      const uint64_t kn = seg_min_u64(donor ? pack_min(act ? W : kNegInfT, t) : ~0ull, S);
      const int gmin = unpack_min_t(kn);
      M128 cands{bcast_u64(sm.lo, gmin, S), bcast_u64(sm.hi, gmin, S)};
      const M128 mx{bcast_u64(sm.lo, gmax, S), bcast_u64(sm.hi, gmax, S)};
      const uint32_t ldx = bcast_u32(load, gmax, S);
      const uint32_t nhx = bcast_u32(nhu, gmax, S);
      const uint32_t dmx = bcast_u32(dm_t, gmax, S);
      const int topx = m_empty(mx) ? -1 : m_top(mx);
      int u = 0;
      while (!m_empty(cands)) {
        u = m_pop_low(cands);
        int64_t trial;
        if (nhx == 0) {
          trial = kInfT;
        } else {
          const int s = u > topx ? u : topx;
          const uint32_t ld = ldx + V.su_fill[u];
          trial = (int64_t)udiv(7200ull * dmx, V.su_speed[s]) - (int64_t)((ld - V.su_fill[s]) / nhx);
        }
        if (!has2 || trial < w2 || m_empty(cands)) break;
      }
      const uint32_t fu = V.su_fill[u];
      if (t == gmin) { m_clear(sm, u); load -= fu; }
      if (t == gmax) { m_set(sm, u); load += fu; }
      if (act) W = twait(sm, load);
      ++rounds;
      const int64_t ntop = unpack_val(seg_max_u64(act ? pack_max(W, t) : 0ull, S));
      if (ntop < top) continue;
      if (t == gmin) { m_set(sm, u); load += fu; }
      if (t == gmax) { m_clear(sm, u); load -= fu; }
      if (act) W = twait(sm, load);
      break;
    }
  }
  // ---- path length (sec. 2.2) ----
  const uint64_t units = lane_tour ? (uint64_t)(__popcll(hm) + m_pop(sm)) : 0ull;
  o.cost = seg_sum_u64(units * (uint64_t)L + shuttle, S);
  o.makespan = tmax;
  if (tmax == kInfT) o.flags |= kCandInfMakespan;
  o.hu_mask = hm;
  o.su_mask = sm;
  return o;
}

__device__ __forceinline__ bool is_gated(int64_t mk, int64_t t_star, uint32_t flags) {
  if (flags & kGateOff) return false;
  if (flags & kGateStrict) return mk >= t_star;
  return mk > t_star;
}

// ------------------------------------------------------- LDS staging ----
__device__ __forceinline__ void stage(uint32_t *lds, const uint32_t *src, uint32_t words) {
  const uint32_t n4 = words >> 2;
  const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
  uint4 *d4 = reinterpret_cast<uint4 *>(lds);
  for (uint32_t i = threadIdx.x; i < n4; i += blockDim.x) d4[i] = s4[i];
  for (uint32_t i = (n4 << 2) + threadIdx.x; i < words; i += blockDim.x) lds[i] = src[i];
}

__host__ __device__ __forceinline__ uint32_t round4(uint32_t w) { return (w + 3u) & ~3u; }

extern __shared__ uint4 g_lds4[];

// ----------------------------------------------------------- kernels ----
enum { kModeBatch = 0, kModeSearch = 1 };

template <bool DLDS, int MODE>
__global__ __launch_bounds__(256) void k_eval(InstParams P, const uint64_t *__restrict__ moves,
                                              uint32_t n, int64_t t_star_arg, uint64_t seed,
                                              uint32_t inst_index, uint64_t *__restrict__ out_key,
                                              float *__restrict__ out_cost,
                                              int32_t *__restrict__ out_mk,
                                              uint8_t *__restrict__ out_flags) {
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
  if (MODE == kModeSearch) {
    it = P.st->it;
    t_star = P.st->t_best;
  }
  uint64_t best = kInfKey;
  for (uint32_t c = gseg; c < n; c += nseg) {
    const uint64_t w = MODE == kModeSearch ? draw_move(seed, c, it, inst_index, V, P) : moves[c];
    const Move m = decode_move(w, V, P);
    uint64_t key = kInfKey;
    float cost_km = __builtin_inff();
    int32_t mk = 0x7FFFFFFF;
    uint32_t fl;
    if (!m.valid) {
      fl = kCandInvalid;
    } else {
      const EvalOut o = eval_candidate(V, P, m, t, S, seg_base, seg_mask);
      fl = o.flags;
      if (o.feasible) {
        cost_km = (float)((double)o.cost / 1000.0);
        mk = o.makespan >= 0x7FFFFFFFll ? 0x7FFFFFFF : (int32_t)o.makespan;
        if (is_gated(o.makespan, t_star, P.flags))
          fl |= kCandGated;
        else
          key = (o.cost << 24) | (uint64_t)c;
      }
    }
    if (MODE == kModeBatch && t == 0) {
      out_key[c] = key;
      if (out_cost) out_cost[c] = cost_km;
      if (out_mk) out_mk[c] = mk;
      if (out_flags) out_flags[c] = (uint8_t)fl;
    }
    best = key < best ? key : best;
  }
  if (MODE == kModeSearch) {
    for (int off = 1; off < 64; off <<= 1) {
      const uint64_t o = __shfl_xor((unsigned long long)best, off, 64);
      best = o < best ? o : best;
    }
    if (lane == 0 && best != kInfKey) atomicMin((unsigned long long *)P.best_key, (unsigned long long)best);
  }
}

// Base preparation: optional eq. (6) pick (copy x* or x_old to the base
// slot), then the base view written into the instance image.  One workgroup.
__global__ __launch_bounds__(1024) void k_prepare(InstParams P, int mode, uint64_t seed,
                                                  uint64_t eps_thr, uint32_t inst_index) {
  __shared__ int s_src;
  const int tid = threadIdx.x, nt = blockDim.x;
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
  uint32_t *img = P.image;
  const ImageLayout &L = P.lay;
  uint16_t *seq = (uint16_t *)(img + L.seq), *pos = (uint16_t *)(img + L.pos);
  uint16_t *fbp = (uint16_t *)(img + L.fbp), *fidx = (uint16_t *)(img + L.fidx);
  uint16_t *bp_start = (uint16_t *)(img + L.bp_start), *bp_len = (uint16_t *)(img + L.bp_len);
  uint16_t *bp_tour = (uint16_t *)(img + L.bp_tour), *bp_idx = (uint16_t *)(img + L.bp_idx);
  uint16_t *tour_off = (uint16_t *)(img + L.tour_off), *tour_bp = (uint16_t *)(img + L.tour_bp);
  uint32_t *leg_in = img + L.leg_in, *dfb = img + L.dfb;
  uint64_t *hu_mask = (uint64_t *)(img + L.hu_mask), *su_mask = (uint64_t *)(img + L.su_mask);
  const uint16_t *hu_rank = (const uint16_t *)(img + L.hu_rank);
  const uint16_t *su_rank = (const uint16_t *)(img + L.su_rank);

  for (int i = tid; i <= P.NT; i += nt) tour_off[i] = x.tour_off[i];
  for (int i = tid; i < P.NB; i += nt) tour_bp[i] = x.tour_bp[i];
  for (int i = tid; i < P.NB; i += nt) bp_len[i] = (uint16_t)(x.bp_off[i + 1] - x.bp_off[i]);
  __syncthreads();
  if (tid == 0) {
    // BP start positions in tour order (serial prefix over the BPs).
    uint32_t run = 0;
    for (int g = 0; g < P.NT; ++g)
      for (int j = x.tour_off[g]; j < x.tour_off[g + 1]; ++j) {
        const int b = x.tour_bp[j];
        bp_tour[b] = (uint16_t)g;
        bp_idx[b] = (uint16_t)(j - x.tour_off[g]);
        bp_start[b] = (uint16_t)run;
        run += bp_len[b];
      }
    *P.best_key = kInfKey;
  }
  __syncthreads();
  const uint32_t nb1 = 1u + (uint32_t)P.NB;
  for (int i = tid; i < P.NF; i += nt) {
    // BP owning slot i of the id-ordered field lists (upper bound search).
    int lo = 0, hi = P.NB;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if ((int)x.bp_off[mid] <= i) lo = mid; else hi = mid;
    }
    const int b = lo;
    const int k = i - x.bp_off[b];
    const int f = x.bp_field[i];
    const int q = bp_start[b] + k;
    seq[q] = (uint16_t)f;
    pos[f] = (uint16_t)q;
    fbp[f] = (uint16_t)b;
    fidx[f] = (uint16_t)k;
    dfb[q] = P.dist[(size_t)(nb1 + f) * P.V + 1 + b];
  }
  __syncthreads();
  for (int q = tid; q < P.NF; q += nt) {
    const uint32_t a = q == 0 ? 0u : nb1 + seq[q - 1];
    leg_in[q] = P.dist[(size_t)a * P.V + nb1 + seq[q]];
  }
  for (int g = tid; g < P.NT; g += nt) {
    uint64_t hm = 0, lo = 0, hi = 0;
    for (int h = 0; h < P.NHU; ++h)
      if (x.hu_tour[h] == g) hm |= 1ull << hu_rank[h];
    for (int s = 0; s < P.NSU; ++s)
      if (x.su_tour[s] == g) {
        const int r = su_rank[s];
        if (r < 64) lo |= 1ull << r; else hi |= 1ull << (r - 64);
      }
    hu_mask[g] = hm;
    su_mask[2 * g] = lo;
    su_mask[2 * g + 1] = hi;
  }
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

// Commit (one workgroup).  Start mode: Step 4 of Algorithm 1, the base with
// a no-op move and the gate off becomes x* and x_old.  Step mode: the winner
// of the iteration is rebuilt from its draw, x_old <- x_new, and x* <- x_new
// on a strict decrease of C; one trace row.
template <bool DLDS>
__global__ __launch_bounds__(256) void k_commit(InstParams P, int mode, uint64_t seed,
                                                uint32_t inst_index) {
  uint32_t *lds = reinterpret_cast<uint32_t *>(g_lds4);
  const uint32_t img_words = round4(P.lay.total_words);
  stage(lds, P.image, P.lay.total_words);
  if (DLDS) stage(lds + img_words, P.dist, (uint32_t)(P.V * P.V));
  __syncthreads();
  const View V = make_view(lds, P.lay, DLDS ? lds + img_words : P.dist);
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
  // Wave 0 evaluates the winner and writes its minimised units.
  if (tid < 64) {
    const int S = P.seg;
    const int t = tid & (S - 1);
    const uint64_t seg_mask = S == 64 ? ~0ull : ((1ull << S) - 1ull);
    const int seg_base = tid & ~(S - 1);
    if (seg_base == 0) {
      const EvalOut o = eval_candidate(V, P, m, t, S, seg_base, seg_mask);
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
      int f, q;
      cand_field(V, m, lo, i - xo.bp_off[lo], f, q);
      xo.bp_field[i] = (uint16_t)f;
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

}  // namespace

size_t eval_lds_bytes(const InstParams &P) {
  size_t w = round4(P.lay.total_words);
  if (P.d_in_lds) w += (size_t)P.V * (size_t)P.V;
  return w * 4;
}

hipError_t launch_prepare(const InstParams &P, int mode, uint64_t seed, uint64_t eps_thr,
                          uint32_t inst_index, hipStream_t s) {
  hipLaunchKernelGGL(k_prepare, dim3(1), dim3(1024), 0, s, P, mode, seed, eps_thr, inst_index);
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

hipError_t launch_eval_batch(const InstParams &P, const uint64_t *moves, uint32_t n,
                             int64_t t_star, uint64_t *key, float *cost, int32_t *mk,
                             uint8_t *flags, int grid, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t lds = eval_lds_bytes(P);
  if (P.d_in_lds)
    hipLaunchKernelGGL((k_eval<true, kModeBatch>), dim3(grid), dim3(256), lds, s, P, moves, n,
                       t_star, 0ull, 0u, key, cost, mk, flags);
  else
    hipLaunchKernelGGL((k_eval<false, kModeBatch>), dim3(grid), dim3(256), lds, s, P, moves, n,
                       t_star, 0ull, 0u, key, cost, mk, flags);
  return hipGetLastError();
}

hipError_t launch_eval_search(const InstParams &P, uint64_t seed, uint32_t n,
                              uint32_t inst_index, int grid, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t lds = eval_lds_bytes(P);
  if (P.d_in_lds)
    hipLaunchKernelGGL((k_eval<true, kModeSearch>), dim3(grid), dim3(256), lds, s, P, nullptr, n,
                       0ll, seed, inst_index, nullptr, nullptr, nullptr, nullptr);
  else
    hipLaunchKernelGGL((k_eval<false, kModeSearch>), dim3(grid), dim3(256), lds, s, P, nullptr, n,
                       0ll, seed, inst_index, nullptr, nullptr, nullptr, nullptr);
  return hipGetLastError();
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

int eval_occupancy(const InstParams &P, bool search) {
  int nb = 0;
  const size_t lds = eval_lds_bytes(P);
  hipError_t e;
  if (P.d_in_lds)
    e = search ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval<true, kModeSearch>, 256, lds)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval<true, kModeBatch>, 256, lds);
  else
    e = search ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval<false, kModeSearch>, 256, lds)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eval<false, kModeBatch>, 256, lds);
  return e == hipSuccess && nb > 0 ? nb : 1;
}

}  // namespace bl
