// Device helpers shared by the evaluator and the learned-screen kernels:
// Philox, the LDS view of an instance image, remove-and-reinsert move decoding and the
// candidate view, segment reductions, unit masks, the full evaluation of one
// candidate (walk, eq. (2), HU and SU rebalancing, cost) and LDS staging.
#pragma once

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

// udiv with a 64-bit divisor: exact for p + q < 2^53, q > 0, and 0 for any
// q > p (p < 2^53): the quotient then rounds to at most 1 - 2^-53.
__device__ __forceinline__ uint64_t udiv_wide(uint64_t p, uint64_t q) {
  return (uint64_t)((double)p / (double)q);
}

// floor(n / d) for n < 2^31 and 0 < d < 2^16 from r = 1/d (double): n * r
// is within 2^-19 of n / d, whose fraction is at most 1 - 2^-16, so the
// truncation is floor(n / d) or one below it (exact quotients); one check,
// whose product stays below 2^32, fixes the latter.  r is computed once per
// divisor by the caller.  (SU loads are below 2^27: fill times < 2^20 s.)
__device__ __forceinline__ uint32_t udiv_small(uint32_t n, uint32_t d, double r) {
  uint32_t q = (uint32_t)((double)n * r);
  if ((q + 1u) * d <= n) ++q;
  return q;
}

// --------------------------------------------------------- the LDS view --
struct View {
  const uint32_t *area, *supply, *nsh, *dhq, *demand, *hu_rate, *su_fill, *su_speed;
  const uint16_t *hu_rank, *su_rank;
  const uint16_t *seq, *pos, *fbp, *fidx, *bp_start, *bp_len, *bp_tour, *bp_idx, *tour_off, *tour_bp;
  const uint4 *prec;   // per position: {leg in, D[field][BP], area, supply}
  const uint32_t *w_q;  // per position: shuttle distance
  const uint64_t *hu_mask, *su_mask;
  const uint32_t *t_len, *t_area, *t_msum, *t_mcnt, *b_sd, *b_sup, *b_area, *b_int, *b_mean, *b_skip,
      *skip, *n_viol;
  const uint64_t *t_sh, *b_sh;
  const uint16_t *t_start, *t_end;
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
  v.prec = (const uint4 *)(img + L.prec);
  v.w_q = img + L.w_q;
  v.bp_start = (const uint16_t *)(img + L.bp_start);
  v.bp_len = (const uint16_t *)(img + L.bp_len);
  v.bp_tour = (const uint16_t *)(img + L.bp_tour);
  v.bp_idx = (const uint16_t *)(img + L.bp_idx);
  v.tour_off = (const uint16_t *)(img + L.tour_off);
  v.tour_bp = (const uint16_t *)(img + L.tour_bp);
  v.hu_mask = (const uint64_t *)(img + L.hu_mask);
  v.su_mask = (const uint64_t *)(img + L.su_mask);
  v.t_len = img + L.t_len;
  v.t_area = img + L.t_area;
  v.t_msum = img + L.t_msum;
  v.t_mcnt = img + L.t_mcnt;
  v.b_sd = img + L.b_sd;
  v.b_sup = img + L.b_sup;
  v.b_area = img + L.b_area;
  v.b_int = img + L.b_int;
  v.b_mean = img + L.b_mean;
  v.b_skip = img + L.b_skip;
  v.skip = img + L.skip;
  v.n_viol = img + L.n_viol;
  v.t_sh = (const uint64_t *)(img + L.t_sh);
  v.b_sh = (const uint64_t *)(img + L.b_sh);
  v.t_start = (const uint16_t *)(img + L.t_start);
  v.t_end = (const uint16_t *)(img + L.t_end);
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

// Remove-and-reinsert draw of candidate i of iteration `it` (counter (i, it, inst, 0)).
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

// Field id of element k of BP b's field list in the candidate.
__device__ __forceinline__ int cand_field(const View &V, const Move &m, int b, int k) {
  if (m.kind == 0) {
    if (b == m.dst) {
      if (k == m.slot) return m.v;
      if (k > m.slot) k -= 1;
    }
    if (b == m.src && k >= m.r) k += 1;
  }
  return V.seq[V.bp_start[b] + k];
}

// BP b's candidate field list as base-position runs around the inserted
// field: run0, [moved field if ins0], run1, [moved field if ins1], run2.
struct Pieces {
  int a0, a1, b0, b1, c0, c1;
  bool ins0, ins1;
};

__device__ __forceinline__ Pieces bp_pieces(const View &V, const Move &m, int b) {
  const int st = V.bp_start[b], len = V.bp_len[b];
  Pieces p{st, st + len, 0, 0, 0, 0, false, false};
  if (m.kind != 0) return p;
  const bool is_src = b == m.src, is_dst = b == m.dst;
  const int r = m.r, s = m.slot;
  if (is_src && !is_dst) {
    p.a1 = st + r;
    p.b0 = st + r + 1;
    p.b1 = st + len;
  } else if (is_dst && !is_src) {
    p.a1 = st + s;
    p.ins0 = true;
    p.b0 = st + s;
    p.b1 = st + len;
  } else if (is_src && is_dst) {
    if (s <= r) {
      p.a1 = st + s;
      p.ins0 = true;
      p.b0 = st + s;
      p.b1 = st + r;
      p.c0 = st + r + 1;
      p.c1 = st + len;
    } else {
      p.a1 = st + r;
      p.b0 = st + r + 1;
      p.b1 = st + s + 1;
      p.ins1 = true;
      p.c0 = st + s + 1;
      p.c1 = st + len;
    }
  }
  return p;
}

// ------------------------------------------------ delta evaluation ----
// Route neighbours of the moved vertex: the field, or the BP's run of fields
// [q0, q1) in base positions.  pold/nold surround it in the base; pnew/nnew
// surround its insertion point in the route after its removal.  -1 is HQ.
// An empty moved BP leaves every route unchanged (first = -1).
struct Nbrs {
  int q0, q1, first, last, pold, nold, pnew, nnew;
};

__device__ __forceinline__ Nbrs move_nbrs(const View &V, const Move &m) {
  Nbrs n;
  if (m.kind == 0) {
    const int f = m.v, bs = m.src, bd = m.dst, r = m.r, s = m.slot;
    const int Ts = V.bp_tour[bs], Td = V.bp_tour[bd];
    const int qf = V.pos[f];
    n.q0 = qf;
    n.q1 = qf + 1;
    n.first = n.last = f;
    n.pold = qf > (int)V.t_start[Ts] ? V.seq[qf - 1] : -1;
    n.nold = qf + 1 < (int)V.t_end[Ts] ? V.seq[qf + 1] : -1;
    const int st = V.bp_start[bd], len = V.bp_len[bd];
    const int room = len - (bd == bs ? 1 : 0);
    if (s > 0) {
      int k = s - 1;
      if (bd == bs && k >= r) ++k;
      n.pnew = V.seq[st + k];
    } else {
      int pp = st - 1;
      if (pp == qf) --pp;
      n.pnew = pp >= (int)V.t_start[Td] ? V.seq[pp] : -1;
    }
    if (s < room) {
      int k = s;
      if (bd == bs && k >= r) ++k;
      n.nnew = V.seq[st + k];
    } else {
      int pp = st + len;
      if (pp == qf) ++pp;
      n.nnew = pp < (int)V.t_end[Td] ? V.seq[pp] : -1;
    }
  } else {
    const int b = m.v, s = m.slot, r = m.r, Ts = m.src, Td = m.dst;
    const int q0 = V.bp_start[b], q1 = q0 + V.bp_len[b];
    n.q0 = q0;
    n.q1 = q1;
    n.first = n.last = n.pold = n.nold = n.pnew = n.nnew = -1;
    if (q1 == q0) return n;
    n.first = V.seq[q0];
    n.last = V.seq[q1 - 1];
    n.pold = q0 > (int)V.t_start[Ts] ? V.seq[q0 - 1] : -1;
    n.nold = q1 < (int)V.t_end[Ts] ? V.seq[q1] : -1;
    const int room = tour_len(V, Td) - (Td == Ts ? 1 : 0);
    int ip;
    if (s < room) {
      int j = s;
      if (Td == Ts && j >= r) ++j;
      ip = V.bp_start[V.tour_bp[V.tour_off[Td] + j]];
    } else {
      ip = V.t_end[Td];
    }
    int pp = ip - 1;
    if (pp >= q0 && pp < q1) pp = q0 - 1;
    n.pnew = pp >= (int)V.t_start[Td] ? V.seq[pp] : -1;
    pp = ip;
    if (pp >= q0 && pp < q1) pp = q1;
    n.nnew = pp < (int)V.t_end[Td] ? V.seq[pp] : -1;
  }
  return n;
}

// Road distance between two fields, HQ standing for -1 on either side.
__device__ __forceinline__ uint32_t route_leg(const View &V, const InstParams &P, int a, int b) {
  if (a < 0) return b < 0 ? 0u : V.dhq[b];
  if (b < 0) return V.dhq[a];
  const size_t nb1 = 1 + (size_t)P.NB;
  return V.D[(nb1 + (size_t)a) * (size_t)P.V + nb1 + (size_t)b];
}

__device__ __forceinline__ uint32_t bp_mean(uint32_t sd, uint32_t cnt) { return cnt ? sd / cnt : 0u; }

// Tour t of the candidate from the base's aggregates: only the source and
// destination tours change, by the legs the move cuts and creates and by the
// moved fields' sums.  Every lane of the segment forms the same changes (the
// move is uniform over the segment), so the distance-matrix reads of the two
// created legs are issued together; lane t then applies the source part
// and/or the destination part.  Integer results equal the full walk's.
__device__ __forceinline__ void tour_delta(const View &V, const InstParams &P, const Move &m,
                                           const Nbrs &nb, int t, uint32_t &L, uint32_t &A,
                                           uint64_t &sh, uint32_t &msum, uint32_t &mcnt, bool &act) {
  L = V.t_len[t];
  A = V.t_area[t];
  sh = V.t_sh[t];
  msum = V.t_msum[t];
  mcnt = V.t_mcnt[t];
  int nf = (int)V.t_end[t] - (int)V.t_start[t];
  if (nb.first >= 0) {  // an empty moved BP changes no route and no sum
    const bool fm = m.kind == 0;
    const int Ts = fm ? (int)V.bp_tour[m.src] : m.src;
    const int Td = fm ? (int)V.bp_tour[m.dst] : m.dst;
    const bool cross = fm && m.src != m.dst;
    const size_t nb1 = 1 + (size_t)P.NB;
    // The created legs and the moved field's distance to its new BP.
    const uint32_t l_in = route_leg(V, P, nb.pnew, nb.first);
    const uint32_t l_out = route_leg(V, P, nb.last, nb.nnew);
    const uint32_t dfd = cross ? V.D[(nb1 + (size_t)m.v) * (size_t)P.V + 1 + (size_t)m.dst] : 0u;
    // The cut legs (position records) and the leg that closes the gap.
    const uint32_t bridge = fm ? V.skip[nb.q0] : V.b_skip[m.v];
    const uint32_t lin = nb.pold < 0 ? V.dhq[nb.first] : V.prec[nb.q0].x;
    const uint32_t lout = nb.nold < 0 ? V.dhq[nb.last] : V.prec[nb.q1].x;
    const int64_t inner = fm ? 0 : (int64_t)V.b_int[m.v];
    uint32_t gap;
    if (nb.pnew == nb.pold && nb.nnew == nb.nold) {
      gap = bridge;
    } else if (nb.pnew < 0 || nb.nnew < 0) {
      gap = nb.pnew < 0 ? (nb.nnew < 0 ? 0u : V.dhq[nb.nnew]) : V.dhq[nb.pnew];
    } else {  // consecutive in the base
      const int qn = V.pos[nb.nnew];
      gap = V.seq[qn - 1] == nb.pnew ? V.prec[qn].x : route_leg(V, P, nb.pnew, nb.nnew);
    }
    // Sums that move with the vertex.
    uint32_t mv_area, mv_nf;
    uint64_t sh_out, sh_in;
    int32_t ms_s = 0, ms_d = 0, mc_s = 0, mc_d = 0;
    if (fm) {
      const int f = m.v;
      mv_area = V.area[f];
      mv_nf = 1;
      sh_out = V.w_q[nb.q0];
      sh_in = cross ? 2ull * (uint64_t)V.nsh[f] * (uint64_t)dfd : sh_out;
      if (cross) {
        const int bs = m.src, bd = m.dst;
        const uint32_t cs = V.bp_len[bs], cd = V.bp_len[bd];
        ms_s = (int32_t)bp_mean(V.b_sd[bs] - V.prec[nb.q0].y, cs - 1) - (int32_t)V.b_mean[bs];
        mc_s = cs == 1 ? -1 : 0;
        ms_d = (int32_t)bp_mean(V.b_sd[bd] + dfd, cd + 1) - (int32_t)V.b_mean[bd];
        mc_d = cd == 0 ? 1 : 0;
      }
    } else {
      const int b = m.v;
      mv_area = V.b_area[b];
      mv_nf = V.bp_len[b];
      sh_out = sh_in = V.b_sh[b];
      ms_s = -(int32_t)V.b_mean[b];
      ms_d = (int32_t)V.b_mean[b];
      mc_s = -1;
      mc_d = 1;
    }
    int64_t Lx = L;
    if (t == Ts) {
      Lx += (int64_t)bridge - (int64_t)lin - (int64_t)lout - inner;
      A -= mv_area;
      sh -= sh_out;
      msum = (uint32_t)((int32_t)msum + ms_s);
      mcnt = (uint32_t)((int32_t)mcnt + mc_s);
      nf -= (int)mv_nf;
    }
    if (t == Td) {
      Lx += (int64_t)l_in + (int64_t)l_out - (int64_t)gap + inner;
      A += mv_area;
      sh += sh_in;
      msum = (uint32_t)((int32_t)msum + ms_d);
      mcnt = (uint32_t)((int32_t)mcnt + mc_d);
      nf += (int)mv_nf;
    }
    L = (uint32_t)Lx;
  }
  act = nf > 0;
}

// eq. (2) for the candidate: the base's violations corrected at the two BPs
// a field move changes.  Uniform over the segment.
__device__ __forceinline__ bool delta_feasible(const View &V, const Move &m) {
  int viol = (int)V.n_viol[0];
  if (m.kind == 0 && m.src != m.dst) {
    const int bs = m.src, bd = m.dst;
    const uint32_t sf = V.supply[m.v], ss = V.b_sup[bs], sd = V.b_sup[bd];
    const uint32_t ds = V.demand[bs], dd = V.demand[bd];
    viol += (int)(ss - sf < ds) - (int)(ss < ds) + (int)(sd + sf < dd) - (int)(sd < dd);
  }
  return viol == 0;
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

// Butterfly partner exchange inside a segment.  Up to 16 lanes the partner
// comes through DPP (quad permutes, then the 8- and 16-lane mirrors, which
// pair the two halves after the smaller groups are reduced); wider segments
// use a cross-lane permute.
template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
  // Every lane's partner exists for these patterns, so no old value is kept.
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)v, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, true);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7-i within 8 lanes
constexpr int kDppMirror = 0x140;     // lane i <-> 15-i within 16 lanes

template <class Op>
__device__ __forceinline__ uint64_t seg_reduce_u64(uint64_t v, int S, Op op) {
  if (S >= 2) v = op(v, dpp64<kDppXor1>(v));
  if (S >= 4) v = op(v, dpp64<kDppXor2>(v));
  if (S >= 8) v = op(v, dpp64<kDppHalfMirror>(v));
  if (S >= 16) v = op(v, dpp64<kDppMirror>(v));
  if (S >= 32) v = op(v, (uint64_t)__shfl_xor((unsigned long long)v, 16, S));
  if (S >= 64) v = op(v, (uint64_t)__shfl_xor((unsigned long long)v, 32, S));
  return v;
}
// 32-bit keys for instances whose times stay within (-2^26, 2^26 - 1) s and
// segments of at most 16 lanes: the value + 2^26 in 27 bits above a 5-bit
// tour field (the infinities take the end codes), so each butterfly step is
// one DPP move and one max or min.
constexpr int64_t kNarrowOff = (int64_t)1 << 26;
constexpr uint32_t kNarrowInf = (1u << 27) - 1u;
__device__ __forceinline__ uint32_t nclamp(int64_t v) {
  return v == kInfT ? kNarrowInf : (v == kNegInfT ? 0u : (uint32_t)(v + kNarrowOff));
}
__device__ __forceinline__ int64_t nunclamp(uint32_t b) {
  return b == kNarrowInf ? kInfT : (b == 0u ? kNegInfT : (int64_t)b - kNarrowOff);
}
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}
template <bool MAX>
__device__ __forceinline__ uint32_t seg_reduce_u32(uint32_t v, int S) {
  auto op = [](uint32_t a, uint32_t b) { return MAX ? (a > b ? a : b) : (a < b ? a : b); };
  if (S >= 2) v = op(v, dpp32<kDppXor1>(v));
  if (S >= 4) v = op(v, dpp32<kDppXor2>(v));
  if (S >= 8) v = op(v, dpp32<kDppHalfMirror>(v));
  if (S >= 16) v = op(v, dpp32<kDppMirror>(v));
  return v;
}

// Key operations of the rebalancing rounds, 64-bit (any instance) or 32-bit
// (narrow instances).
template <bool NK>
struct Keys {
  using K = uint64_t;
  static constexpr K kNone = 0ull, kNoneMin = ~0ull;
  __device__ static K pmax(int64_t v, int t) { return pack_max(v, t); }
  __device__ static K pmin(int64_t v, int t) { return pack_min(v, t); }
  __device__ static int64_t val(K k) { return unpack_val(k); }
  __device__ static int tmax(K k) { return unpack_max_t(k); }
  __device__ static int tmin(K k) { return unpack_min_t(k); }
};
template <>
struct Keys<true> {
  using K = uint32_t;
  static constexpr K kNone = 0u, kNoneMin = ~0u;
  __device__ static K pmax(int64_t v, int t) { return (nclamp(v) << 5) | (uint32_t)(31 - t); }
  __device__ static K pmin(int64_t v, int t) { return (nclamp(v) << 5) | (uint32_t)t; }
  __device__ static int64_t val(K k) { return nunclamp(k >> 5); }
  __device__ static int tmax(K k) { return 31 - (int)(k & 31u); }
  __device__ static int tmin(K k) { return (int)(k & 31u); }
};

__device__ __forceinline__ uint64_t seg_max_u64(uint64_t v, int S) {
  return seg_reduce_u64(v, S, [](uint64_t a, uint64_t b) { return a > b ? a : b; });
}
__device__ __forceinline__ uint64_t seg_min_u64(uint64_t v, int S) {
  return seg_reduce_u64(v, S, [](uint64_t a, uint64_t b) { return a < b ? a : b; });
}
__device__ __forceinline__ uint32_t seg_max_k(uint32_t v, int S) { return seg_reduce_u32<true>(v, S); }
__device__ __forceinline__ uint32_t seg_min_k(uint32_t v, int S) { return seg_reduce_u32<false>(v, S); }
__device__ __forceinline__ uint64_t seg_max_k(uint64_t v, int S) { return seg_max_u64(v, S); }
__device__ __forceinline__ uint64_t seg_min_k(uint64_t v, int S) { return seg_min_u64(v, S); }
__device__ __forceinline__ uint64_t seg_sum_u64(uint64_t v, int S) {
  return seg_reduce_u64(v, S, [](uint64_t a, uint64_t b) { return a + b; });
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

// Evaluate one candidate on the S lanes of a segment (lane t owns tour t).
// `gate`: 0 = off, 1 = discard when makespan > t_star, 2 = when >= t_star.
// SS > 0 fixes the segment width at compile time (the reductions and
// broadcasts then have no width tests); SS == 0 takes it from S_rt.
template <bool WALK, int SS>
__device__ __forceinline__ EvalOut eval_candidate(const View &V, const InstParams &P, const Move &m, int t,
                                  int S_rt, int seg_base, uint64_t seg_mask) {
  const int S = SS > 0 ? SS : S_rt;
  // Compile-time widths run only for narrow instances (see eval_candidate_s).
  using KY = Keys<(SS > 0)>;
  using K = typename KY::K;
  EvalOut o;
  o.flags = 0;
  const bool lane_tour = t < P.NT;
  // ---- walk of tour t: length, area, shuttles, per-BP means, eq. (2) ----
  // Every field of the tour is visited.  A BP's candidate field list is at
  // most three runs of consecutive base positions around the moved field;
  // inside a run the leg into each field is the base successor distance.
  uint32_t L = 0, A = 0, sum_mean = 0, n_mean = 0;
  uint64_t shuttle = 0;
  bool feas = true, act = false;
  if constexpr (!WALK) {
    const Nbrs nb = move_nbrs(V, m);
    if (lane_tour) tour_delta(V, P, m, nb, t, L, A, shuttle, sum_mean, n_mean, act);
    feas = delta_feasible(V, m);
  } else if (lane_tour) {
    const int nbt = cand_tour_len(V, m, t);
    const size_t Vn = (size_t)P.V;
    const int nb1 = 1 + P.NB;
    int fprev = -1, qprev = -2;
    for (int j = 0; j < nbt; ++j) {
      const int b = cand_tour_bp(V, m, t, j);
      const Pieces pc = bp_pieces(V, m, b);
      uint32_t sd = 0, sup = 0, cnt = 0;
      auto run = [&](int q0, int q1) {
        if (q0 >= q1) return;
        const int f0 = V.seq[q0];
        uint4 r = V.prec[q0];
        L += fprev < 0 ? V.dhq[f0]
                       : (q0 == qprev + 1 ? r.x : V.D[(size_t)(nb1 + fprev) * Vn + nb1 + f0]);
        sd += r.y;
        A += r.z;
        sup += r.w;
        shuttle += V.w_q[q0];
        for (int q = q0 + 1; q < q1; ++q) {
          r = V.prec[q];
          L += r.x;
          sd += r.y;
          A += r.z;
          sup += r.w;
          shuttle += V.w_q[q];
        }
        cnt += (uint32_t)(q1 - q0);
        fprev = V.seq[q1 - 1];
        qprev = q1 - 1;
      };
      auto ins = [&]() {
        const int f = m.v;
        const uint32_t dfb = V.D[(size_t)(nb1 + f) * Vn + 1 + b];
        L += fprev < 0 ? V.dhq[f] : V.D[(size_t)(nb1 + fprev) * Vn + nb1 + f];
        A += V.area[f];
        sup += V.supply[f];
        sd += dfb;
        shuttle += 2ull * (uint64_t)V.nsh[f] * (uint64_t)dfb;
        cnt += 1;
        fprev = f;
        qprev = V.pos[f];
      };
      run(pc.a0, pc.a1);
      if (pc.ins0) ins();
      run(pc.b0, pc.b1);
      if (pc.ins1) ins();
      run(pc.c0, pc.c1);
      if (cnt > 0) {
        sum_mean += sd / cnt;
        n_mean += 1;
      }
      feas = feas && sup >= V.demand[b];
    }
    if (fprev >= 0) {
      L += V.dhq[fprev];
      act = true;
    }
  }
  if constexpr (WALK)
    o.feasible = seg_ballot(!feas, seg_base, seg_mask) == 0;
  else
    o.feasible = feas;
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
      const K kx = seg_max_k(act ? KY::pmax(T, t) : KY::kNone, S);
      if (kx == KY::kNone) break;
      const int gmax = KY::tmax(kx);
      const int64_t top = KY::val(kx);
      const K k2 = seg_max_k((act && t != gmax) ? KY::pmax(T, t) : KY::kNone, S);
      const bool has2 = k2 != KY::kNone;
      const int g2 = has2 ? KY::tmax(k2) : -1;
      const int64_t t2 = has2 ? KY::val(k2) : 0;
      const bool hasu = hm != 0;
      uint64_t dm = seg_ballot(hasu && t != gmax && t != g2, seg_base, seg_mask);
      if (!dm) dm = seg_ballot(hasu && t != gmax, seg_base, seg_mask);
      if (!dm) break;
      if (rounds == (int)P.cap_hu) {
        o.flags |= kCandCapHu;
        break;
      }
      const bool donor = (dm >> t) & 1;
      const K kn = seg_min_k(donor ? KY::pmin(act ? T : kNegInfT, t) : KY::kNoneMin, S);
      const int gmin = KY::tmin(kn);
      uint64_t cands = bcast_u64(hm, gmin, S);
      uint64_t lcx;
      if constexpr (SS > 0)  // narrow: the road part of a completion time is < 2^26
        lcx = bcast_u32((uint32_t)lc, gmax, S);
      else
        lcx = bcast_u64(lc, gmax, S);
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
      const int64_t T_before = T;
      if (t == gmin) { hm &= ~(1ull << u); R -= ru; }
      if (t == gmax) { hm |= 1ull << u; R += ru; }
      if (act) T = tcompl(R);
      ++rounds;
      const int64_t ntop = KY::val(seg_max_k(act ? KY::pmax(T, t) : KY::kNone, S));
      if (ntop < top) continue;
      // Not kept: undo.
      if (t == gmin) { hm |= 1ull << u; R += ru; }
      if (t == gmax) { hm &= ~(1ull << u); R -= ru; }
      T = T_before;
      break;
    }
  }
  const int64_t tmax = KY::val(seg_max_k(act ? KY::pmax(T, t) : KY::kNone, S));
  // ---- SU min-max rebalancing, Alg. 2: waiting time ----
  const uint32_t nhu = (uint32_t)__popcll(hm);
  const uint32_t dm_t = n_mean ? sum_mean / n_mean : 0u;
  uint32_t load = 0;
  {
    M128 mm = sm;
    while (!m_empty(mm)) load += V.su_fill[m_pop_low(mm)];
  }
  const double r_nhu = nhu ? 1.0 / (double)nhu : 0.0;
  auto twait = [&](const M128 &msk, uint32_t ld) -> int64_t {
    if (m_empty(msk) || nhu == 0) return kInfT;
    const int s = m_top(msk);
    return (int64_t)udiv(7200ull * dm_t, V.su_speed[s]) - (int64_t)udiv_small(ld - V.su_fill[s], nhu, r_nhu);
  };
  if (embedded) {
    int64_t W = act ? twait(sm, load) : 0;
    int rounds = 0;
    while (true) {
      const K kx = seg_max_k(act ? KY::pmax(W, t) : KY::kNone, S);
      if (kx == KY::kNone) break;
      const int gmax = KY::tmax(kx);
      const int64_t top = KY::val(kx);
      const K k2 = seg_max_k((act && t != gmax) ? KY::pmax(W, t) : KY::kNone, S);
      const bool has2 = k2 != KY::kNone;
      const int g2 = has2 ? KY::tmax(k2) : -1;
      const int64_t w2 = has2 ? KY::val(k2) : 0;
      const bool hasu = !m_empty(sm);
      uint64_t dmk = seg_ballot(hasu && t != gmax && t != g2, seg_base, seg_mask);
      if (!dmk) dmk = seg_ballot(hasu && t != gmax, seg_base, seg_mask);
      if (!dmk) break;
      if (rounds == (int)P.cap_su) {
        o.flags |= kCandCapSu;
        break;
      }
      const bool donor = (dmk >> t) & 1;
      const K kn = seg_min_k(donor ? KY::pmin(act ? W : kNegInfT, t) : KY::kNoneMin, S);
      const int gmin = KY::tmin(kn);
      M128 cands{bcast_u64(sm.lo, gmin, S), bcast_u64(sm.hi, gmin, S)};
      // g_max's critical SU, load, HU count and mean distance (< 2^24, so it
      // shares a word with the HU count).
      const int topx = (int)bcast_u32((uint32_t)(m_empty(sm) ? -1 : m_top(sm)), gmax, S);
      const uint32_t ldx = bcast_u32(load, gmax, S);
      const uint32_t nd = bcast_u32((nhu << 24) | dm_t, gmax, S);
      const uint32_t nhx = nd >> 24, dmx = nd & 0xFFFFFFu;
      // Round trip of g_max's critical SU: the trial's unless the unit tried
      // outranks it.
      const uint64_t rt_top = (nhx != 0 && topx >= 0) ? udiv(7200ull * dmx, V.su_speed[topx]) : 0ull;
      const double r_nhx = nhx ? 1.0 / (double)nhx : 0.0;
      // The donor's units in rank order: the first whose move takes g_max's
      // waiting time below w2, else the last (the first without g2, the last
      // without HUs).  As in the lane version, each form of the trial is
      // below w2 exactly when one integer of the unit passes a bound formed
      // once per round: f_u >= nhx * (rt_top - w2 + 1) - (ldx - f_topx) for a
      // unit ranked below the critical SU topx, v_u >= floor(7200 dmx / K) + 1
      // with K = w2 + floor(ldx / nhx) > 0 for one ranked above it (K
      // saturates where w2 is +inf: every finite trial is below it).
      int u = 0;
      if (!has2 || nhx == 0) {
        u = has2 ? m_top(cands) : m_pop_low(cands);
      } else {
        const int64_t J = (int64_t)rt_top - w2 + 1;
        const uint32_t C = topx >= 0 ? ldx - V.su_fill[topx] : 0u;
        const int64_t fa = J <= 0 ? 0 : (int64_t)nhx * J - (int64_t)C;
        const uint32_t fbound = fa <= 0 ? 0u : (fa >= (int64_t)UINT32_MAX ? UINT32_MAX : (uint32_t)fa);
        const int64_t q = (int64_t)udiv_small(ldx, nhx, r_nhx);
        const int64_t Kb = w2 > INT64_MAX - q ? INT64_MAX : w2 + q;
        const uint64_t vbound = Kb <= 0 ? ~0ull : udiv_wide(7200ull * dmx, (uint64_t)Kb) + 1ull;
        while (true) {
          u = m_pop_low(cands);
          const bool ok = u < topx ? V.su_fill[u] >= fbound : (uint64_t)V.su_speed[u] >= vbound;
          if (ok || m_empty(cands)) break;
        }
      }
      const uint32_t fu = V.su_fill[u];
      if (t == gmin) { m_clear(sm, u); load -= fu; }
      if (t == gmax) { m_set(sm, u); load += fu; }
      if (act) W = twait(sm, load);
      ++rounds;
      const int64_t ntop = KY::val(seg_max_k(act ? KY::pmax(W, t) : KY::kNone, S));
      if (ntop < top) continue;
      // Not kept: undo (W is not used after the loop).
      if (t == gmin) { m_set(sm, u); load += fu; }
      if (t == gmax) { m_clear(sm, u); load -= fu; }
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
enum { kModeBatch = 0, kModeSearch = 1, kModeGather = 2 };

struct CandResult {
  uint64_t key;
  float cost_km;
  int32_t mk;
  uint32_t flags;
};

// Full evaluation of move word w as candidate c (all segment lanes call it).
// The evaluation for the instance's segment width: compile-time widths and
// 32-bit keys for narrow instances (at most 16 lanes), the run-time width and
// 64-bit keys otherwise.
template <bool WALK>
__device__ __forceinline__ EvalOut eval_candidate_s(const View &V, const InstParams &P, const Move &m,
                                                    int t, int S, int seg_base, uint64_t seg_mask) {
  if (!P.narrow) return eval_candidate<WALK, 0>(V, P, m, t, S, seg_base, seg_mask);
  switch (S) {
    case 1: return eval_candidate<WALK, 1>(V, P, m, t, S, seg_base, seg_mask);
    case 2: return eval_candidate<WALK, 2>(V, P, m, t, S, seg_base, seg_mask);
    case 4: return eval_candidate<WALK, 4>(V, P, m, t, S, seg_base, seg_mask);
    case 8: return eval_candidate<WALK, 8>(V, P, m, t, S, seg_base, seg_mask);
    case 16: return eval_candidate<WALK, 16>(V, P, m, t, S, seg_base, seg_mask);
    default: return eval_candidate<WALK, 0>(V, P, m, t, S, seg_base, seg_mask);
  }
}

template <bool WALK>
__device__ __forceinline__ CandResult eval_one(const View &V, const InstParams &P, uint64_t w,
                                               uint32_t c, int t, int S, int seg_base,
                                               uint64_t seg_mask, int64_t t_star) {
  const Move m = decode_move(w, V, P);
  CandResult r{kInfKey, __builtin_inff(), 0x7FFFFFFF, 0u};
  if (!m.valid) {
    r.flags = kCandInvalid;
    return r;
  }
  const EvalOut o = eval_candidate_s<WALK>(V, P, m, t, S, seg_base, seg_mask);
  r.flags = o.flags;
  if (o.feasible) {
    r.cost_km = (float)((double)o.cost / 1000.0);
    r.mk = o.makespan >= 0x7FFFFFFFll ? 0x7FFFFFFF : (int32_t)o.makespan;
    if (is_gated(o.makespan, t_star, P.flags))
      r.flags |= kCandGated;
    else
      r.key = (o.cost << 24) | (uint64_t)c;
  }
  return r;
}

// Wave-wide minimum of `best`; lane 0 folds it into *slot with one atomic.
__device__ __forceinline__ void wave_min_to(uint64_t best, uint64_t *slot) {
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t o = __shfl_xor((unsigned long long)best, off, 64);
    best = o < best ? o : best;
  }
  if ((threadIdx.x & 63) == 0 && best != kInfKey)
    atomicMin((unsigned long long *)slot, (unsigned long long)best);
}


}  // namespace

}  // namespace bl
