// gfx950 kernels of the learned screen: a set encoder over the fields of a
// candidate solution.  Per field: 16 features -> 128 -> 128 (ReLU) on bf16
// MFMA with fp32 accumulation, then projected by the pooled-embedding rows of
// W3 (128 -> 64) before pooling; mean over the fields of each BP, mean over
// the BPs of each tour, plus the tour features through the remaining rows of
// W3, ReLU, 64 -> 2 (path share, completion time); path = sum over active
// tours, makespan = max over active tours.  Projecting before pooling is the
// same function as pooling then projecting (both steps are linear), and lets
// the screen update a candidate from its base through the few fields whose
// features changed.
//
// Training runs full forward and backward passes per example on the rows of
// every field: features (k_sur_feat), MLP forward (k_sur_fwd), pool and head
// forward/backward (k_sur_head), MLP backward with weight gradients
// (k_sur_bwd), Adam (k_sur_adam) and the bf16 operand refresh (k_sur_pack).
//
// MFMA operand layout of v_mfma_f32_16x16x32_bf16 (checked by a probe): lane
// l holds A[row l%16][k 8*(l/16) .. +8], B[k 8*(l/16) .. +8][col l%16]; the
// result D[row 4*(l/16)+i][col l%16], i = 0..3.  Weight rows in LDS are padded
// by 8 bf16 so that the 16 rows read together fall into different banks.
#include <hip/hip_runtime.h>

#include "bl_internal.h"
#include "sur_internal.h"
#include "device.h"

namespace bl {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kLd1 = 40;    // row stride (bf16) of w1t and of transposed row tiles
constexpr int kLd2 = 136;   // row stride of 128-wide operands
constexpr int kLd3 = 72;    // row stride of 64-wide operands

__device__ __forceinline__ floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ uint16_t to_bf16(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}
__device__ __forceinline__ float from_bf16(uint16_t b) {
  return (float)__builtin_bit_cast(__bf16, b);
}
__device__ __forceinline__ bf16x8 ld8(const uint16_t *p) {
  return *reinterpret_cast<const bf16x8 *>(p);
}
__device__ __forceinline__ bf16x8 zero8() {
  bf16x8 z;
  for (int j = 0; j < 8; ++j) z[j] = (__bf16)0.0f;
  return z;
}
// Orders LDS traffic between the lanes of one wave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}
__device__ __forceinline__ float wave_sum(float v) {
  for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Visits the fields of tour t of the candidate in route order:
// fn(field, BP, leg into the field, field-BP distance).
template <class Fn>
__device__ __forceinline__ void walk_fields(const View &V, const InstParams &P, const Move &m,
                                            int t, Fn fn) {
  const int nbt = cand_tour_len(V, m, t);
  const size_t Vn = (size_t)P.V;
  const int nb1 = 1 + P.NB;
  int fprev = -1, qprev = -2;
  for (int j = 0; j < nbt; ++j) {
    const int b = cand_tour_bp(V, m, t, j);
    const Pieces pc = bp_pieces(V, m, b);
    auto run = [&](int q0, int q1) {
      for (int q = q0; q < q1; ++q) {
        const int f = V.seq[q];
        const uint4 r = V.prec[q];
        const uint32_t leg = fprev < 0 ? V.dhq[f]
                                       : (q == qprev + 1 ? r.x : V.D[(size_t)(nb1 + fprev) * Vn + nb1 + f]);
        fn(f, b, leg, r.y);
        fprev = f;
        qprev = q;
      }
    };
    auto ins = [&]() {
      const int f = m.v;
      const uint32_t dfb = V.D[(size_t)(nb1 + f) * Vn + 1 + b];
      const uint32_t leg = fprev < 0 ? V.dhq[f] : V.D[(size_t)(nb1 + fprev) * Vn + nb1 + f];
      fn(f, b, leg, dfb);
      fprev = f;
      qprev = V.pos[f];
    };
    run(pc.a0, pc.a1);
    if (pc.ins0) ins();
    run(pc.b0, pc.b1);
    if (pc.ins1) ins();
    run(pc.c0, pc.c1);
  }
}

// One feature row (16 values, zero padded to 32 bf16 = 64 bytes).
__device__ __forceinline__ void write_row(uint16_t *dst, const float *v) {
  uint32_t w[8];
  for (int j = 0; j < 8; ++j) w[j] = (uint32_t)to_bf16(v[2 * j]) | ((uint32_t)to_bf16(v[2 * j + 1]) << 16);
  uint4 *d = reinterpret_cast<uint4 *>(dst);
  d[0] = uint4{w[0], w[1], w[2], w[3]};
  d[1] = uint4{w[4], w[5], w[6], w[7]};
  d[2] = uint4{0u, 0u, 0u, 0u};
  d[3] = uint4{0u, 0u, 0u, 0u};
}

// Features of n candidates (one per segment, lane t = tour t): rows in
// candidate route order, example e owning rows e*NF .. e*NF + NF - 1.
// noop: one example, the base itself.  Invalid move records are treated as
// the base.
__global__ __launch_bounds__(256) void k_sur_feat(InstParams P, SurDev S, const uint64_t *moves,
                                                  uint32_t n, int noop) {
  uint32_t *lds = reinterpret_cast<uint32_t *>(g_lds4);
  stage(lds, P.image, P.lay.total_words);
  __syncthreads();
  const View V = make_view(lds, P.lay, P.dist);
  const int SG = P.seg;
  const int lane = threadIdx.x & 63;
  const int t = lane & (SG - 1);
  const int segs_per_wave = 64 / SG;
  const uint32_t gseg = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * segs_per_wave +
                        (uint32_t)(lane / SG);
  const uint32_t nseg = gridDim.x * (blockDim.x >> 6) * segs_per_wave;
  const int f0 = V.seq[0];
  const uint64_t noop_w = (uint64_t)f0 | ((uint64_t)V.fbp[f0] << 16) | ((uint64_t)V.fidx[f0] << 32);
  for (uint32_t e = gseg; e < n; e += nseg) {
    Move m = decode_move(noop ? noop_w : moves[e], V, P);
    if (!m.valid) m = decode_move(noop_w, V, P);
    int nf_t = 0, nb_t = 0;
    if (t < P.NT) {
      nb_t = cand_tour_len(V, m, t);
      for (int j = 0; j < nb_t; ++j) nf_t += cand_bp_len(V, m, cand_tour_bp(V, m, t, j));
    }
    int incl = nf_t;
    for (int off = 1; off < SG; off <<= 1) {
      const int y = __shfl_up(incl, off, SG);
      if (t >= off) incl += y;
    }
    if (t >= P.NT) continue;
    uint32_t row = e * (uint32_t)P.NF + (uint32_t)(incl - nf_t);
    int last = -1;
    walk_fields(V, P, m, t, [&](int f, int b, uint32_t leg, uint32_t dfb) {
      const float *fs = S.fstat + (size_t)f * 8;
      float v[16] = {fs[0], fs[1], fs[2], fs[3], S.bxy[2 * b], S.bxy[2 * b + 1],
                     (float)dfb * S.inv_ds, (float)leg * S.inv_ds, fs[5] * (float)dfb, fs[4],
                     0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      write_row(S.phi + (size_t)row * kSurK1, v);
      S.row_bp[row] = (uint16_t)b;
      ++row;
      last = f;
    });
    // Tour features, with the units of the base (before rebalancing).
    const uint64_t hm = V.hu_mask[t];
    const uint64_t slo = V.su_mask[2 * t], shi = V.su_mask[2 * t + 1];
    float rates = 0.f, fills = 0.f;
    for (uint64_t mm = hm; mm; mm &= mm - 1) rates += (float)V.hu_rate[__ffsll((unsigned long long)mm) - 1];
    for (uint64_t mm = slo; mm; mm &= mm - 1) fills += (float)V.su_fill[__ffsll((unsigned long long)mm) - 1];
    for (uint64_t mm = shi; mm; mm &= mm - 1) fills += (float)V.su_fill[63 + __ffsll((unsigned long long)mm)];
    float *u = S.ex_u + ((size_t)e * P.NT + t) * kSurU;
    u[0] = (float)__popcll(hm) / (float)P.NHU;
    u[1] = (float)(__popcll(slo) + __popcll(shi)) / (float)P.NSU;
    u[2] = rates * S.inv_rates;
    u[3] = fills * S.inv_fills;
    u[4] = (float)nf_t / (float)P.NF;
    u[5] = (float)nb_t / (float)P.NB;
    u[6] = last >= 0 ? (float)V.dhq[last] * S.inv_ds : 0.f;
    u[7] = 1.f;
    S.ex_nb[(size_t)e * P.NT + t] = (uint16_t)nb_t;
    for (int j = 0; j < nb_t; ++j) {
      const int b = cand_tour_bp(V, m, t, j);
      S.ex_cnt[(size_t)e * P.NB + b] = (uint16_t)cand_bp_len(V, m, b);
      S.ex_btour[(size_t)e * P.NB + b] = (uint16_t)t;
    }
  }
}

// Per-field MLP over rows: P = relu(relu(phi W1 + b1) W2 + b2) W3[0:128].
// One wave per 16-row tile; weights staged in LDS per workgroup.
__global__ __launch_bounds__(256) void k_sur_fwd(SurDev S, const uint16_t *phi, uint32_t n_rows,
                                                 float *Pout, uint16_t *h1out, uint16_t *h2out) {
  uint16_t *w1t = reinterpret_cast<uint16_t *>(g_lds4);
  uint16_t *w2t = w1t + 128 * kLd1;
  uint16_t *w3et = w2t + 128 * kLd2;
  float *b1 = reinterpret_cast<float *>(w3et + 64 * kLd2);
  float *b2 = b1 + 128;
  uint16_t *hbuf = reinterpret_cast<uint16_t *>(b2 + 128);
  for (int i = threadIdx.x; i < 128 * kLd1; i += blockDim.x) w1t[i] = S.w1t[i];
  for (int i = threadIdx.x; i < 128 * kLd2; i += blockDim.x) w2t[i] = S.w2t[i];
  for (int i = threadIdx.x; i < 64 * kLd2; i += blockDim.x) w3et[i] = S.w3et[i];
  for (int i = threadIdx.x; i < 128; i += blockDim.x) {
    b1[i] = S.W[kSurOffB1 + i];
    b2[i] = S.W[kSurOffB2 + i];
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, kb = lane >> 4;
  uint16_t *hb = hbuf + wave * 16 * kLd2;
  const uint32_t tiles = (n_rows + 15) / 16;
  const uint32_t wpb = blockDim.x >> 6;
  for (uint32_t tile = blockIdx.x * wpb + wave; tile < tiles; tile += gridDim.x * wpb) {
    const uint32_t row0 = tile * 16;
    const bool va = row0 + r < n_rows;
    const bf16x8 a1 = va ? ld8(phi + (size_t)(row0 + r) * kSurK1 + kb * 8) : zero8();
    for (int nt = 0; nt < 8; ++nt) {
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma(a1, ld8(w1t + (nt * 16 + r) * kLd1 + kb * 8), acc);
      for (int i = 0; i < 4; ++i)
        hb[(4 * kb + i) * kLd2 + nt * 16 + r] = to_bf16(fmaxf(acc[i] + b1[nt * 16 + r], 0.f));
    }
    wave_sync();
    if (h1out) {
      const int rr = lane >> 2, cc = (lane & 3) * 32;
      if (row0 + rr < n_rows)
        for (int j = 0; j < 4; ++j)
          *reinterpret_cast<uint4 *>(h1out + (size_t)(row0 + rr) * 128 + cc + 8 * j) =
              *reinterpret_cast<const uint4 *>(hb + rr * kLd2 + cc + 8 * j);
    }
    floatx4 acc2[8];
    for (int nt = 0; nt < 8; ++nt) acc2[nt] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < 4; ++ks) {
      const bf16x8 a = ld8(hb + r * kLd2 + ks * 32 + kb * 8);
      for (int nt = 0; nt < 8; ++nt)
        acc2[nt] = mfma(a, ld8(w2t + (nt * 16 + r) * kLd2 + ks * 32 + kb * 8), acc2[nt]);
    }
    wave_sync();
    for (int nt = 0; nt < 8; ++nt)
      for (int i = 0; i < 4; ++i)
        hb[(4 * kb + i) * kLd2 + nt * 16 + r] = to_bf16(fmaxf(acc2[nt][i] + b2[nt * 16 + r], 0.f));
    wave_sync();
    if (h2out) {
      const int rr = lane >> 2, cc = (lane & 3) * 32;
      if (row0 + rr < n_rows)
        for (int j = 0; j < 4; ++j)
          *reinterpret_cast<uint4 *>(h2out + (size_t)(row0 + rr) * 128 + cc + 8 * j) =
              *reinterpret_cast<const uint4 *>(hb + rr * kLd2 + cc + 8 * j);
    }
    for (int nt = 0; nt < 4; ++nt) {
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int ks = 0; ks < 4; ++ks)
        acc = mfma(ld8(hb + r * kLd2 + ks * 32 + kb * 8), ld8(w3et + (nt * 16 + r) * kLd2 + ks * 32 + kb * 8), acc);
      for (int i = 0; i < 4; ++i) {
        const uint32_t row = row0 + 4 * kb + i;
        if (row < n_rows) Pout[(size_t)row * kSurA + nt * 16 + r] = acc[i];
      }
    }
    wave_sync();
  }
}

// Pool and head, one wave per example (lane c = column c of the 64-wide
// projected embeddings).  train = 0: predictions; train = 1: loss against
// the exact cost / makespan, gradients of the head parameters (summed into
// S.G) and of every row's P (into S.dP).
__global__ __launch_bounds__(256) void k_sur_head(InstParams P, SurDev S, uint32_t n_ex, int train,
                                                  const float *cost_km, const int32_t *mk) {
  float *Q = reinterpret_cast<float *>(g_lds4) + (size_t)(threadIdx.x >> 6) * P.NB * kSurA;
  const int c = threadIdx.x & 63;
  const uint32_t wpb = blockDim.x >> 6;
  float w3u[kSurU];
  for (int j = 0; j < kSurU; ++j) w3u[j] = S.W[kSurOffW3 + (kSurH + j) * kSurA + c];
  const float b3 = S.W[kSurOffB3 + c];
  const float w40 = S.W[kSurOffW4 + c * 2], w41 = S.W[kSurOffW4 + c * 2 + 1];
  const float b40 = S.W[kSurOffB4], b41 = S.W[kSurOffB4 + 1];
  float gw3u[kSurU] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float gb3 = 0.f, gw40 = 0.f, gw41 = 0.f, gb40 = 0.f, gb41 = 0.f, lsum = 0.f, lcnt = 0.f;
  for (uint32_t e = blockIdx.x * wpb + (threadIdx.x >> 6); e < n_ex; e += gridDim.x * wpb) {
    const size_t r0 = (size_t)e * P.NF;
    const uint16_t *cnt = S.ex_cnt + (size_t)e * P.NB;
    const uint16_t *bt = S.ex_btour + (size_t)e * P.NB;
    for (int b = 0; b < P.NB; ++b) Q[b * kSurA + c] = 0.f;
    for (int r = 0; r < P.NF; ++r) Q[S.row_bp[r0 + r] * kSurA + c] += S.P[(r0 + r) * kSurA + c];
    auto tour_z = [&](int g, float &nbf) {
      const int nb = S.ex_nb[(size_t)e * P.NT + g];
      float R = 0.f;
      for (int b = 0; b < P.NB; ++b)
        if (bt[b] == g && cnt[b] > 0 && nb > 0) R += Q[b * kSurA + c] / (float)cnt[b];
      const float *u = S.ex_u + ((size_t)e * P.NT + g) * kSurU;
      float z = (nb > 0 ? R / (float)nb : 0.f) + b3;
      for (int j = 0; j < kSurU; ++j) z += u[j] * w3u[j];
      nbf = (float)nb;
      return z;
    };
    float psum = 0.f, mbest = 0.f;
    int gm = -1;
    for (int g = 0; g < P.NT; ++g) {
      float nbf;
      const float a = fmaxf(tour_z(g, nbf), 0.f);
      const float y0 = wave_sum(a * w40) + b40, y1 = wave_sum(a * w41) + b41;
      if (S.ex_u[((size_t)e * P.NT + g) * kSurU + 4] > 0.f) {
        psum += y0;
        if (gm < 0 || y1 > mbest) mbest = y1, gm = g;
      }
    }
    if (!train) {
      if (c == 0) {
        S.ex_pred[2 * e] = psum;
        S.ex_pred[2 * e + 1] = mbest;
      }
      continue;
    }
    const float ck = cost_km[e];
    const int32_t mv = mk[e];
    const bool ok = __builtin_isfinite(ck) && mv != 0x7FFFFFFF && gm >= 0;
    if (!ok) {
      for (int r = 0; r < P.NF; ++r) S.dP[(r0 + r) * kSurA + c] = 0.f;
      continue;
    }
    const float pt = ck * 1000.f * S.inv_c0, mt = (float)mv * S.inv_t0;
    const float dpp = 2.f * (psum - pt), dmm = 2.f * (mbest - mt);
    lsum += (psum - pt) * (psum - pt) + (mbest - mt) * (mbest - mt);
    lcnt += 1.f;
    for (int g = 0; g < P.NT; ++g) {
      float nbf;
      const float z = tour_z(g, nbf);
      const float a = fmaxf(z, 0.f);
      const bool act = S.ex_u[((size_t)e * P.NT + g) * kSurU + 4] > 0.f;
      const float dy0 = act ? dpp : 0.f, dy1 = g == gm ? dmm : 0.f;
      gw40 += a * dy0;
      gw41 += a * dy1;
      gb40 += dy0;
      gb41 += dy1;
      const float dz = z > 0.f ? w40 * dy0 + w41 * dy1 : 0.f;
      const float *u = S.ex_u + ((size_t)e * P.NT + g) * kSurU;
      for (int j = 0; j < kSurU; ++j) gw3u[j] += u[j] * dz;
      gb3 += dz;
      const float dR = nbf > 0.f ? dz / nbf : 0.f;
      for (int b = 0; b < P.NB; ++b)
        if (bt[b] == g && cnt[b] > 0) Q[b * kSurA + c] = dR / (float)cnt[b];
    }
    for (int r = 0; r < P.NF; ++r) S.dP[(r0 + r) * kSurA + c] = Q[S.row_bp[r0 + r] * kSurA + c];
  }
  if (train) {
    // This wave's sums, added up in a fixed order by k_sur_gsum.
    float *part = S.part_h + (size_t)(blockIdx.x * wpb + (threadIdx.x >> 6)) * kHeadPart;
    for (int j = 0; j < kSurU; ++j) part[j * kSurA + c] = gw3u[j];
    part[kSurU * kSurA + c] = gb3;
    part[(kSurU + 1) * kSurA + 2 * c] = gw40;
    part[(kSurU + 1) * kSurA + 2 * c + 1] = gw41;
    if (c == 0) {
      part[(kSurU + 3) * kSurA] = gb40;
      part[(kSurU + 3) * kSurA + 1] = gb41;
      part[(kSurU + 3) * kSurA + 2] = lsum;
      part[(kSurU + 3) * kSurA + 3] = lcnt;
    }
  }
}

// MLP backward over rows, one 32-row chunk per workgroup step: row gradients
// through layers 3, 2, 1 on MFMA, then the weight gradients (K = the 32 rows)
// accumulated per wave and summed into S.G at the end.
__global__ __launch_bounds__(256) void k_sur_bwd(SurDev S, uint32_t n_rows) {
  uint16_t *w2n = reinterpret_cast<uint16_t *>(g_lds4);      // [128][kLd2]
  uint16_t *w3en = w2n + 128 * kLd2;                         // [128][kLd3]
  uint16_t *dPr = w3en + 128 * kLd3;                         // [32][kLd3]
  uint16_t *dz2r = dPr + 32 * kLd3;                          // [32][kLd2]
  uint16_t *phiT = dz2r + 32 * kLd2;                         // [16][kLd1]
  uint16_t *h1T = phiT + 16 * kLd1;                          // [128][kLd1]
  uint16_t *h2T = h1T + 128 * kLd1;
  uint16_t *dPT = h2T + 128 * kLd1;                          // [64][kLd1]
  uint16_t *dz2T = dPT + 64 * kLd1;                          // [128][kLd1]
  uint16_t *dz1T = dz2T + 128 * kLd1;
  for (int i = threadIdx.x; i < 128 * kLd2; i += blockDim.x) w2n[i] = S.w2n[i];
  for (int i = threadIdx.x; i < 128 * kLd3; i += blockDim.x) w3en[i] = S.w3en[i];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, kb = lane >> 4;
  floatx4 acc3[8], acc2[16], acc1[2];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc3[k] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 16; ++k) acc2[k] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 2; ++k) acc1[k] = floatx4{0.f, 0.f, 0.f, 0.f};
  float gb2[4] = {0.f, 0.f, 0.f, 0.f}, gb1[4] = {0.f, 0.f, 0.f, 0.f};
  const uint32_t chunks = (n_rows + 31) / 32;
  // A chunk's rows are loaded into registers one chunk ahead, so that the
  // loads of chunk ch + gridDim.x are in flight while chunk ch is on MFMA.
  // Thread t holds elements t + 256 k of the chunk's dP (32 x 64), h1 and h2
  // (32 x 128) and phi (32 x 16) tiles; rows past n_rows are zero.
  static_assert(32 * 64 % 256 == 0 && 32 * 128 % 256 == 0 && 32 * 16 % 256 == 0, "tile split");
  float pf_dp[32 * 64 / 256];
  uint16_t pf_h1[32 * 128 / 256], pf_h2[32 * 128 / 256], pf_phi[32 * 16 / 256];
  auto fetch = [&](uint32_t row0) {
#pragma unroll
    for (int k = 0; k < 32 * 64 / 256; ++k) {
      const int i = threadIdx.x + 256 * k, rr = i >> 6, cc = i & 63;
      pf_dp[k] = row0 + rr < n_rows ? S.dP[(size_t)(row0 + rr) * kSurA + cc] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < 32 * 128 / 256; ++k) {
      const int i = threadIdx.x + 256 * k, rr = i >> 7, cc = i & 127;
      const bool v = row0 + rr < n_rows;
      pf_h1[k] = v ? S.h1[(size_t)(row0 + rr) * 128 + cc] : (uint16_t)0;
      pf_h2[k] = v ? S.h2[(size_t)(row0 + rr) * 128 + cc] : (uint16_t)0;
    }
#pragma unroll
    for (int k = 0; k < 32 * 16 / 256; ++k) {
      const int i = threadIdx.x + 256 * k, rr = i >> 4, cc = i & 15;
      pf_phi[k] = row0 + rr < n_rows ? S.phi[(size_t)(row0 + rr) * kSurK1 + cc] : (uint16_t)0;
    }
  };
  if (blockIdx.x < chunks) fetch(blockIdx.x * 32);
  for (uint32_t ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 32 * 64 / 256; ++k) {
      const int i = threadIdx.x + 256 * k, rr = i >> 6, cc = i & 63;
      const uint16_t bv = to_bf16(pf_dp[k]);
      dPr[rr * kLd3 + cc] = bv;
      dPT[cc * kLd1 + rr] = bv;
    }
#pragma unroll
    for (int k = 0; k < 32 * 128 / 256; ++k) {
      const int i = threadIdx.x + 256 * k, rr = i >> 7, cc = i & 127;
      h1T[cc * kLd1 + rr] = pf_h1[k];
      h2T[cc * kLd1 + rr] = pf_h2[k];
    }
#pragma unroll
    for (int k = 0; k < 32 * 16 / 256; ++k) {
      const int i = threadIdx.x + 256 * k, rr = i >> 4, cc = i & 15;
      phiT[cc * kLd1 + rr] = pf_phi[k];
    }
    __syncthreads();
    if (ch + gridDim.x < chunks) fetch((ch + gridDim.x) * 32);
    // dz2 = (dP W3e^T) * (h2 > 0): 16 tiles (2 row tiles x 8 column tiles), 4 per wave.
    for (int k = 0; k < 4; ++k) {
      const int tile = wave * 4 + k, rt = tile >> 3, nt = tile & 7;
      floatx4 d = {0.f, 0.f, 0.f, 0.f};
      for (int ks = 0; ks < 2; ++ks)
        d = mfma(ld8(dPr + (rt * 16 + r) * kLd3 + ks * 32 + kb * 8),
                 ld8(w3en + (nt * 16 + r) * kLd3 + ks * 32 + kb * 8), d);
      const int col = nt * 16 + r;
      for (int i = 0; i < 4; ++i) {
        const int row = rt * 16 + 4 * kb + i;
        const float g = from_bf16(h2T[col * kLd1 + row]) > 0.f ? d[i] : 0.f;
        gb2[k] += g;
        const uint16_t bg = to_bf16(g);
        dz2r[row * kLd2 + col] = bg;
        dz2T[col * kLd1 + row] = bg;
      }
    }
    __syncthreads();
    // dz1 = (dz2 W2^T) * (h1 > 0).
    for (int k = 0; k < 4; ++k) {
      const int tile = wave * 4 + k, rt = tile >> 3, nt = tile & 7;
      floatx4 d = {0.f, 0.f, 0.f, 0.f};
      for (int ks = 0; ks < 4; ++ks)
        d = mfma(ld8(dz2r + (rt * 16 + r) * kLd2 + ks * 32 + kb * 8),
                 ld8(w2n + (nt * 16 + r) * kLd2 + ks * 32 + kb * 8), d);
      const int col = nt * 16 + r;
      for (int i = 0; i < 4; ++i) {
        const int row = rt * 16 + 4 * kb + i;
        const float g = from_bf16(h1T[col * kLd1 + row]) > 0.f ? d[i] : 0.f;
        gb1[k] += g;
        dz1T[col * kLd1 + row] = to_bf16(g);
      }
    }
    __syncthreads();
    // Weight gradients, K = the 32 rows: dW3e 8 x 4 tiles (8 per wave), dW2
    // 8 x 8 tiles (16 per wave), dW1 1 x 8 tiles (2 per wave).
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int tile = wave * 8 + k;
      acc3[k] = mfma(ld8(h2T + ((tile >> 2) * 16 + r) * kLd1 + kb * 8),
                     ld8(dPT + ((tile & 3) * 16 + r) * kLd1 + kb * 8), acc3[k]);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int tile = wave * 16 + k;
      acc2[k] = mfma(ld8(h1T + ((tile >> 3) * 16 + r) * kLd1 + kb * 8),
                     ld8(dz2T + ((tile & 7) * 16 + r) * kLd1 + kb * 8), acc2[k]);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int tile = wave * 2 + k;
      acc1[k] = mfma(ld8(phiT + r * kLd1 + kb * 8), ld8(dz1T + (tile * 16 + r) * kLd1 + kb * 8),
                     acc1[k]);
    }
  }
  // This workgroup's sums (every entry written by exactly one lane), added
  // up in a fixed order by k_sur_gsum.  The bias sums come in two halves,
  // one per 16-row tile of the chunk.
  float *part = S.part_b + (size_t)blockIdx.x * kBwdPart;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int tile = wave * 8 + k;
    for (int i = 0; i < 4; ++i)
      part[kBwdW3 + ((tile >> 2) * 16 + 4 * kb + i) * kSurA + (tile & 3) * 16 + r] = acc3[k][i];
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int tile = wave * 16 + k;
    for (int i = 0; i < 4; ++i)
      part[kBwdW2 + ((tile >> 3) * 16 + 4 * kb + i) * kSurH + (tile & 7) * 16 + r] = acc2[k][i];
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int tile = wave * 2 + k;
    for (int i = 0; i < 4; ++i) part[kBwdW1 + (4 * kb + i) * kSurH + tile * 16 + r] = acc1[k][i];
  }
  for (int k = 0; k < 4; ++k) {
    const int tile = wave * 4 + k, rt = tile >> 3, nt = tile & 7;
    float v2 = gb2[k], v1 = gb1[k];
    v2 += __shfl_xor(v2, 16, 64);
    v2 += __shfl_xor(v2, 32, 64);
    v1 += __shfl_xor(v1, 16, 64);
    v1 += __shfl_xor(v1, 32, 64);
    if (kb == 0) {
      part[kBwdB2 + rt * kSurH + nt * 16 + r] = v2;
      part[kBwdB1 + rt * kSurH + nt * 16 + r] = v1;
    }
  }
}

// Gradient (and loss) sums of one training step from the partial sums of
// the head's waves and the backward pass's workgroups.  A workgroup of 16
// waves takes 64 consecutive elements: wave w adds partials w, w + 16, ...
// in order, then the 16 wave sums are added in order: the result does not
// depend on scheduling.
__device__ __forceinline__ int gsum_source(uint32_t i, uint32_t &o, uint32_t &o2) {
  o2 = 0xFFFFFFFFu;
  if (i >= (uint32_t)(kSurOffW3 + kSurH * kSurA)) {   // head: W3 rows of the tour features, b3, W4, b4
    if (i < (uint32_t)kSurOffB3) o = i - (kSurOffW3 + kSurH * kSurA);
    else if (i < (uint32_t)kSurOffW4) o = kSurU * kSurA + (i - kSurOffB3);
    else if (i < (uint32_t)kSurOffB4) o = (kSurU + 1) * kSurA + (i - kSurOffW4);
    else o = (kSurU + 3) * kSurA + (i - kSurOffB4);
    return 0;
  }
  if (i < (uint32_t)kSurOffB1) o = kBwdW1 + (i - kSurOffW1);
  else if (i < (uint32_t)kSurOffW2) o = kBwdB1 + (i - kSurOffB1), o2 = o + kSurH;
  else if (i < (uint32_t)kSurOffB2) o = kBwdW2 + (i - kSurOffW2);
  else if (i < (uint32_t)kSurOffW3) o = kBwdB2 + (i - kSurOffB2), o2 = o + kSurH;
  else o = kBwdW3 + (i - kSurOffW3);
  return 1;
}

__global__ __launch_bounds__(1024) void k_sur_gsum(SurDev S, uint32_t n_head, uint32_t n_bwd) {
  __shared__ float red[16][65];
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
  // Elements kSurParams, kSurParams + 1 stand for the loss sum and count.
  const uint32_t i = blockIdx.x * 64 + c;
  float acc = 0.f;
  if (i < (uint32_t)kSurParams + 2) {
    uint32_t o, o2;
    const int bwd = i < (uint32_t)kSurParams ? gsum_source(i, o, o2) : (o = (kSurU + 3) * kSurA + 2 + (i - kSurParams), o2 = 0xFFFFFFFFu, 0);
    if (bwd) {
      for (uint32_t b = w; b < n_bwd; b += 16) {
        acc += S.part_b[(size_t)b * kBwdPart + o];
        if (o2 != 0xFFFFFFFFu) acc += S.part_b[(size_t)b * kBwdPart + o2];
      }
    } else {
      for (uint32_t h = w; h < n_head; h += 16) acc += S.part_h[(size_t)h * kHeadPart + o];
    }
  }
  red[w][c] = acc;
  __syncthreads();
  if (w == 0 && i < (uint32_t)kSurParams + 2) {
    float t = 0.f;
    for (int k = 0; k < 16; ++k) t += red[k][c];
    if (i < (uint32_t)kSurParams) S.G[i] = t;
    else S.loss[i - kSurParams] = t;
  }
}

__global__ void k_sur_adam(SurDev S, float lr, float beta1, float beta2, float eps, float scale,
                           float bc1, float bc2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kSurParams; i += gridDim.x * blockDim.x) {
    const float g = S.G[i] * scale;
    const float m = beta1 * S.Mo[i] + (1.f - beta1) * g;
    const float v = beta2 * S.Ve[i] + (1.f - beta2) * g * g;
    S.Mo[i] = m;
    S.Ve[i] = v;
    S.W[i] -= lr * (m / bc1) / (sqrtf(v / bc2) + eps);
    S.G[i] = 0.f;
  }
}

// bf16 operand copies of the weights (zero padding included).
__global__ void k_sur_pack(SurDev S) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  for (int i = tid; i < 128 * kLd1; i += nt) {
    const int n = i / kLd1, k = i % kLd1;
    S.w1t[i] = to_bf16(k < kSurIn ? S.W[kSurOffW1 + k * kSurH + n] : 0.f);
  }
  for (int i = tid; i < 128 * kLd2; i += nt) {
    const int n = i / kLd2, k = i % kLd2;
    S.w2t[i] = to_bf16(k < kSurH ? S.W[kSurOffW2 + k * kSurH + n] : 0.f);
    S.w2n[i] = to_bf16(k < kSurH ? S.W[kSurOffW2 + n * kSurH + k] : 0.f);
  }
  for (int i = tid; i < 64 * kLd2; i += nt) {
    const int n = i / kLd2, k = i % kLd2;
    S.w3et[i] = to_bf16(k < kSurH ? S.W[kSurOffW3 + k * kSurA + n] : 0.f);
  }
  for (int i = tid; i < 128 * kLd3; i += nt) {
    const int n = i / kLd3, k = i % kLd3;
    S.w3en[i] = to_bf16(k < kSurA ? S.W[kSurOffW3 + n * kSurA + k] : 0.f);
  }
}

__global__ void k_sur_zero(float *p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.f;
}

// ------------------------------------------------------------- screening --
// A proposal changes the features of at most three fields (the moved field
// or the moved BP's first field, and the fields whose route predecessor
// changes), the pooled means of at most four BPs and the head inputs of at
// most two tours.  Its prediction is the base's with those parts replaced.

// Order-preserving bits of a float score (smaller score, smaller key).
__device__ __forceinline__ uint32_t score_key(float v) {
  const uint32_t u = __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_score(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

// Base tables from the base's forward rows (example 0, projected rows in
// base position order): BP sums, then per tour the sum of BP means, the tour
// feature term and the head outputs; then the predicted base path and the
// three largest completion outputs.  One workgroup of 16 waves, lane c =
// column c.
__global__ __launch_bounds__(1024) void k_scr_tables(InstParams P, SurDev S, ScreenDev T) {
  const View V = make_view(P.image, P.lay, P.dist);
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int b = w; b < P.NB; b += nw) {
    float s = 0.f;
    const int st = V.bp_start[b], len = V.bp_len[b];
    for (int q = st; q < st + len; ++q) s += S.P[q * kSurA + c];
    T.Q[b * kSurA + c] = s;
  }
  __syncthreads();
  float w3u[kSurU];
  for (int j = 0; j < kSurU; ++j) w3u[j] = S.W[kSurOffW3 + (kSurH + j) * kSurA + c];
  const float b3 = S.W[kSurOffB3 + c];
  const float w40 = S.W[kSurOffW4 + 2 * c], w41 = S.W[kSurOffW4 + 2 * c + 1];
  const float b40 = S.W[kSurOffB4], b41 = S.W[kSurOffB4 + 1];
  for (int g = w; g < P.NT; g += nw) {
    const int nb = tour_len(V, g);
    float R = 0.f;
    int nf = 0;
    for (int j = 0; j < nb; ++j) {
      const int b = V.tour_bp[V.tour_off[g] + j];
      const int len = V.bp_len[b];
      nf += len;
      if (len > 0) R += T.Q[b * kSurA + c] / (float)len;
    }
    const float *u = S.ex_u + (size_t)g * kSurU;
    float U = b3;
    for (int j = 0; j < kSurU; ++j) U += u[j] * w3u[j];
    const float a = fmaxf((nb > 0 ? R / (float)nb : 0.f) + U, 0.f);
    const float y0 = wave_sum(a * w40) + b40, y1 = wave_sum(a * w41) + b41;
    T.R[g * kSurA + c] = R;
    T.U[g * kSurA + c] = U;
    if (c == 0) {
      T.yb[2 * g] = y0;
      T.yb[2 * g + 1] = y1;
      T.nbg[g] = nb;
      T.nfg[g] = nf;
      T.ub6[g] = u[6];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float psum = 0.f;
    for (int g = 0; g < P.NT; ++g)
      if (T.nfg[g] > 0) psum += T.yb[2 * g];
    // Three largest completion outputs over active tours (ties to the lower tour).
    int tg[3] = {-1, -1, -1};
    for (int k = 0; k < 3; ++k)
      for (int g = 0; g < P.NT; ++g) {
        if (T.nfg[g] == 0 || g == tg[0] || g == tg[1]) continue;
        if (tg[k] < 0 || T.yb[2 * g + 1] > T.yb[2 * tg[k] + 1]) tg[k] = g;
      }
    T.scal[0] = psum;
    for (int k = 0; k < 3; ++k) {
      T.top_g[k] = tg[k];
      T.scal[1 + k] = tg[k] >= 0 ? T.yb[2 * tg[k] + 1] : 0.f;
    }
  }
}

// The 16 features of field f served from BP b after route predecessor pred
// (-1: the tour's first field, reached from HQ).
__device__ __forceinline__ void feature_vals(const View &V, const InstParams &P, const SurDev &S,
                                             int f, int b, int pred, float v[16]) {
  const int nb1 = 1 + P.NB;
  const size_t Vn = (size_t)P.V;
  const float *fs = S.fstat + (size_t)f * 8;
  const uint32_t dfb = V.D[(size_t)(nb1 + f) * Vn + 1 + b];
  const uint32_t leg = pred < 0 ? V.dhq[f] : V.D[(size_t)(nb1 + pred) * Vn + nb1 + f];
  v[0] = fs[0];
  v[1] = fs[1];
  v[2] = fs[2];
  v[3] = fs[3];
  v[4] = S.bxy[2 * b];
  v[5] = S.bxy[2 * b + 1];
  v[6] = (float)dfb * S.inv_ds;
  v[7] = (float)leg * S.inv_ds;
  v[8] = fs[5] * (float)dfb;
  v[9] = fs[4];
  for (int j = 10; j < 16; ++j) v[j] = 0.f;
}

__device__ __forceinline__ void add_bp(ScreenDesc &d, int b, int dc) {
  bool done = false;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    if (!done && d.ab[a] == (uint16_t)b) {
      d.dcnt[a] += (int16_t)dc;
      done = true;
    } else if (!done && d.ab[a] == 0xFFFF) {
      d.ab[a] = (uint16_t)b;
      d.dcnt[a] = (int16_t)dc;
      done = true;
    }
  }
}

// A descriptor as 15 words (for the exchange between lanes) and back.
constexpr int kDescWords = 15;
__device__ __forceinline__ uint32_t pk16(uint32_t lo, uint32_t hi) { return (lo & 0xFFFFu) | (hi << 16); }
__device__ __forceinline__ void desc_pack(const ScreenDesc &d, uint32_t w[kDescWords]) {
  w[0] = pk16(d.f[0], d.f[1]);
  w[1] = pk16(d.f[2], d.bold[0]);
  w[2] = pk16(d.bold[1], d.bold[2]);
  w[3] = pk16(d.bnew[0], d.bnew[1]);
  w[4] = pk16(d.bnew[2], d.ab[0]);
  w[5] = pk16(d.ab[1], d.ab[2]);
  w[6] = pk16(d.ab[3], d.moved_bp);
  w[7] = pk16((uint16_t)d.dcnt[0], (uint16_t)d.dcnt[1]);
  w[8] = pk16((uint16_t)d.dcnt[2], (uint16_t)d.dcnt[3]);
  w[9] = pk16(d.tg[0], d.tg[1]);
  w[10] = pk16((uint16_t)d.dnf[0], (uint16_t)d.dnf[1]);
  w[11] = pk16((uint16_t)d.dnb[0], (uint16_t)d.dnb[1]);
  w[12] = __float_as_uint(d.u6[0]);
  w[13] = __float_as_uint(d.u6[1]);
  w[14] = pk16(d.dst_tour, d.feasible);
}
__device__ __forceinline__ void desc_unpack(const uint32_t w[kDescWords], ScreenDesc &d) {
  auto lo = [](uint32_t x) { return (uint16_t)(x & 0xFFFFu); };
  auto hi = [](uint32_t x) { return (uint16_t)(x >> 16); };
  d.f[0] = lo(w[0]);
  d.f[1] = hi(w[0]);
  d.f[2] = lo(w[1]);
  d.bold[0] = hi(w[1]);
  d.bold[1] = lo(w[2]);
  d.bold[2] = hi(w[2]);
  d.bnew[0] = lo(w[3]);
  d.bnew[1] = hi(w[3]);
  d.bnew[2] = lo(w[4]);
  d.ab[0] = hi(w[4]);
  d.ab[1] = lo(w[5]);
  d.ab[2] = hi(w[5]);
  d.ab[3] = lo(w[6]);
  d.moved_bp = hi(w[6]);
  d.dcnt[0] = (int16_t)lo(w[7]);
  d.dcnt[1] = (int16_t)hi(w[7]);
  d.dcnt[2] = (int16_t)lo(w[8]);
  d.dcnt[3] = (int16_t)hi(w[8]);
  d.tg[0] = lo(w[9]);
  d.tg[1] = hi(w[9]);
  d.dnf[0] = (int16_t)lo(w[10]);
  d.dnf[1] = (int16_t)hi(w[10]);
  d.dnb[0] = (int16_t)lo(w[11]);
  d.dnb[1] = (int16_t)hi(w[11]);
  d.u6[0] = __uint_as_float(w[12]);
  d.u6[1] = __uint_as_float(w[13]);
  d.dst_tour = lo(w[14]);
  d.feasible = (uint8_t)hi(w[14]);
}

// What move m changes relative to the base: its descriptor, and per changed
// feature row k the field rf[k] (-1: none), its BP rb[k] and its route
// predecessor rp[k].  The rows are the moved run's first field, the field
// after the insertion point and the field after the gap it leaves.
__device__ __forceinline__ void describe(const View &V, const SurDev &S, const ScreenDev &T,
                                         const Move &m, ScreenDesc &d, int rf[3], int rb[3],
                                         int rp[3]) {
  for (int k = 0; k < 3; ++k) {
    d.f[k] = d.bold[k] = d.bnew[k] = 0xFFFF;
    rf[k] = -1;
    rb[k] = 0;
    rp[k] = -1;
  }
  for (int k = 0; k < 4; ++k) {
    d.ab[k] = 0xFFFF;
    d.dcnt[k] = 0;
  }
  d.tg[0] = d.tg[1] = 0xFFFF;
  d.dnf[0] = d.dnf[1] = d.dnb[0] = d.dnb[1] = 0;
  d.u6[0] = d.u6[1] = 0.f;
  d.moved_bp = d.dst_tour = 0xFFFF;
  d.feasible = 1;
  for (int k = 0; k < 5; ++k) d.pad[k] = 0;
  int Ts, Td, newlast_d = -2, newlast_s = -2;  // -2: unchanged, -1: tour empty
  const Nbrs nb = move_nbrs(V, m);
  int b0;
  if (m.kind == 0) {
    const int f = m.v, bs = m.src, bd = m.dst;
    Ts = V.bp_tour[bs];
    Td = V.bp_tour[bd];
    if (bs != bd && V.b_sup[bs] - V.supply[f] < V.demand[bs]) d.feasible = 0;
    add_bp(d, bs, bs == bd ? 0 : -1);
    add_bp(d, bd, bs == bd ? 0 : 1);
    if (Ts != Td) {
      d.dnf[0] = -1;
      d.dnf[1] = 1;
    }
    b0 = bd;
    d.bold[0] = (uint16_t)bs;
  } else {
    const int b = m.v, len = V.bp_len[b];
    Ts = m.src;
    Td = m.dst;
    d.moved_bp = (uint16_t)b;
    d.dst_tour = (uint16_t)Td;
    add_bp(d, b, 0);
    if (Ts != Td) {
      d.dnf[0] = (int16_t)-len;
      d.dnf[1] = (int16_t)len;
      d.dnb[0] = -1;
      d.dnb[1] = 1;
    }
    b0 = b;
    if (len > 0) d.bold[0] = (uint16_t)b;
  }
  if (nb.first >= 0) {
    rf[0] = nb.first;
    rb[0] = b0;
    rp[0] = nb.pnew;
    if (nb.nnew >= 0) {
      rf[1] = nb.nnew;
      rb[1] = V.fbp[nb.nnew];
      rp[1] = nb.last;
      d.bold[1] = (uint16_t)rb[1];
    }
    if (nb.nold >= 0 && nb.nold != nb.nnew) {
      rf[2] = nb.nold;
      rb[2] = V.fbp[nb.nold];
      rp[2] = nb.pold;
      d.bold[2] = (uint16_t)rb[2];
    }
    if (nb.nnew < 0) newlast_d = nb.last;
    if (nb.nold < 0) newlast_s = nb.pold;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (rf[k] < 0) continue;
    d.f[k] = (uint16_t)rf[k];
    d.bnew[k] = (uint16_t)rb[k];
    add_bp(d, rb[k], 0);
    add_bp(d, d.bold[k], 0);
  }
  // Affected tours and their new return legs.
  auto last_feat = [&](int g, int nl) -> float {
    if (nl == -2) return T.ub6[g];
    return nl >= 0 ? (float)V.dhq[nl] * S.inv_ds : 0.f;
  };
  if (Ts == Td) {
    d.tg[0] = (uint16_t)Ts;
    d.dnf[0] = 0;
    d.dnb[0] = 0;
    d.u6[0] = last_feat(Ts, newlast_d != -2 ? newlast_d : newlast_s);
  } else {
    d.tg[0] = (uint16_t)Ts;
    d.tg[1] = (uint16_t)Td;
    d.u6[0] = last_feat(Ts, newlast_s);
    d.u6[1] = last_feat(Td, newlast_d);
  }
}

// LDS of the fused screen kernel (byte offsets): bf16 weight operands, the
// base tables, the instance image, then per wave the changed feature rows of
// its 64 proposals.
constexpr uint32_t kFuseW1 = 0;
constexpr uint32_t kFuseW2 = kFuseW1 + 128 * kLd1 * 2;
constexpr uint32_t kFuseW3 = kFuseW2 + 128 * kLd2 * 2;
constexpr uint32_t kFuseB1 = kFuseW3 + 64 * kLd2 * 2;
constexpr uint32_t kFuseB2 = kFuseB1 + 128 * 4;
constexpr uint32_t kFuseTab = kFuseB2 + 128 * 4;
constexpr uint32_t kFuseWaveBytes = 3 * 64 * 32;   // 3 rows of 16 bf16 per proposal
constexpr int kFuseMaxWaves = 8;
constexpr int kTabLd = kSurA + 4;   // row stride (floats) of the LDS tables: rows read together
                                    // by different lanes start in different banks
constexpr uint32_t kFuseLdsMax = 160 * 1024;

struct FuseLayout {
  uint32_t q, rz, cst, yb, nbg, nfg, scal, topg;  // word offsets in the table area
  uint32_t img, rows, total;                      // byte offsets
};

__host__ __device__ inline FuseLayout fuse_layout(int NB, int NT, uint32_t img_words, int waves) {
  FuseLayout L;
  L.q = 0;                       // [NB] BP sums of the base's projected rows
  L.rz = L.q + NB * kTabLd;      // [NT][3] head input of each tour before the changes, for a
                                 // BP count change of -1, 0, +1 (see below)
  L.cst = L.rz + 3 * NT * kTabLd;  // 4 rows: W3 rows of the field count (pre-divided) and of
                                   // the return leg, and the two head columns
  L.yb = L.cst + 4 * kTabLd;
  L.nbg = L.yb + 2 * NT;
  L.nfg = L.nbg + NT;
  L.scal = L.nfg + NT;
  L.topg = L.scal + 4;
  const uint32_t tab_words = L.topg + 4;
  L.img = kFuseTab + ((tab_words * 4 + 15u) & ~15u);
  L.rows = L.img + ((img_words * 4 + 15u) & ~15u);
  L.total = L.rows + (uint32_t)waves * kFuseWaveBytes;
  return L;
}

// Two floats rounded to bf16 (round to nearest even), then ReLU on the
// packed halves as signed 16-bit integers (a negative bf16 has its sign bit
// set; rounding keeps signs, so this equals rounding after the ReLU).
__device__ __forceinline__ uint32_t relu_bf16x2(float a, float b) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef short i16x2 __attribute__((ext_vector_type(2)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  const bf16x2 v = __builtin_convertvector((f32x2){a, b}, bf16x2);
  const i16x2 m = __builtin_elementwise_max(__builtin_bit_cast(i16x2, v), (i16x2){0, 0});
  return __builtin_bit_cast(uint32_t, m);
}
__device__ __forceinline__ bf16x8 pack8(const uint32_t w[4]) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 v = {w[0], w[1], w[2], w[3]};
  return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float4 fma4(float a, float4 x, float4 y) {
  return float4{fmaf(a, x.x, y.x), fmaf(a, x.y, y.y), fmaf(a, x.z, y.z), fmaf(a, x.w, y.w)};
}
__device__ __forceinline__ float4 relu4(float4 x) {
  return float4{fmaxf(x.x, 0.f), fmaxf(x.y, 0.f), fmaxf(x.z, 0.f), fmaxf(x.w, 0.f)};
}
__device__ __forceinline__ float dot4(float4 a, float4 b) {
  return fmaf(a.w, b.w, fmaf(a.z, b.z, fmaf(a.y, b.y, a.x * b.x)));
}

// Screen of proposals i0 .. i0 + cnt - 1, fused: one wave takes 64 proposals
// at a time.  Each lane draws one proposal and builds its descriptor and its
// (up to three) changed feature rows; then, 16 proposals at a time, the MLP
// runs on bf16 MFMA with the weights as the A operand and the rows as the B
// operand (the product transposed), so that a layer's fp32 outputs, after
// bias, ReLU and rounding to bf16, are already the next layer's B operand in
// registers: the K order inside each 32-wide slab is permuted to match the
// output layout, in the weights staged to LDS.  Lane l then holds columns
// 16 mt + 4 (l / 16) + i (mt, i < 4) of the projected rows of proposal l % 16
// of the group, and the four lanes of a proposal update the base's BP means,
// tour inputs and head outputs for those columns and add them up.
__global__ __launch_bounds__(512, 1) void k_scr_fused(InstParams P, SurDev S, ScreenDev T,
                                                      uint64_t seed, uint32_t inst_index,
                                                      uint32_t i0, uint32_t cnt, float mk_margin) {
  uint8_t *lds = reinterpret_cast<uint8_t *>(g_lds4);
  const int NB = P.NB, NT = P.NT;
  const int nwaves = blockDim.x >> 6;
  const FuseLayout L = fuse_layout(NB, NT, P.lay.total_words, nwaves);
  uint16_t *w1 = reinterpret_cast<uint16_t *>(lds + kFuseW1);
  uint16_t *w2 = reinterpret_cast<uint16_t *>(lds + kFuseW2);
  uint16_t *w3 = reinterpret_cast<uint16_t *>(lds + kFuseW3);
  float *b1 = reinterpret_cast<float *>(lds + kFuseB1);
  float *b2 = reinterpret_cast<float *>(lds + kFuseB2);
  float *tab = reinterpret_cast<float *>(lds + kFuseTab);
  uint32_t *img = reinterpret_cast<uint32_t *>(lds + L.img);
  // Staging.  Within slab ks of 32 inputs, position 8 q + j holds input
  // 32 ks + 4 q + j (j < 4) or 32 ks + 16 + 4 q + j - 4 (j >= 4).
  for (int i = threadIdx.x; i < 128 * kLd1; i += blockDim.x) w1[i] = S.w1t[i];
  for (int i = threadIdx.x; i < 128 * 128; i += blockDim.x) {
    const int m = i >> 7, kk = i & 127, ks = kk >> 5, q = (kk >> 3) & 3, j = kk & 7;
    const int src = 32 * ks + (j < 4 ? 4 * q + j : 16 + 4 * q + j - 4);
    w2[m * kLd2 + kk] = S.w2t[m * kLd2 + src];
    if (m < 64) w3[m * kLd2 + kk] = S.w3et[m * kLd2 + src];
  }
  for (int i = threadIdx.x; i < 128; i += blockDim.x) {
    b1[i] = S.W[kSurOffB1 + i];
    b2[i] = S.W[kSurOffB2 + i];
  }
  // Head input of tour g, column c, when its BP count changes by e and
  // nothing else: R/(nb + e) + U + e w3[BP count] / NB - ub6 w3[return leg]
  // (the proposal adds its own return leg and field count terms).
  for (int i = threadIdx.x; i < NB * kSurA; i += blockDim.x) tab[L.q + (i >> 6) * kTabLd + (i & 63)] = T.Q[i];
  for (int i = threadIdx.x; i < 3 * NT * kSurA; i += blockDim.x) {
    const int g = i / (3 * kSurA), e = (i / kSurA) % 3 - 1, c = i & 63;
    const int nb = T.nbg[g] + e;
    const float w5 = S.W[kSurOffW3 + (kSurH + 5) * kSurA + c] / (float)P.NB;
    const float w6 = S.W[kSurOffW3 + (kSurH + 6) * kSurA + c];
    tab[L.rz + (3 * g + e + 1) * kTabLd + c] =
        (nb > 0 ? T.R[g * kSurA + c] / (float)nb : 0.f) + T.U[g * kSurA + c] + (float)e * w5 - T.ub6[g] * w6;
  }
  for (int c = threadIdx.x; c < kSurA; c += blockDim.x) {
    tab[L.cst + c] = S.W[kSurOffW3 + (kSurH + 4) * kSurA + c] / (float)P.NF;
    tab[L.cst + kTabLd + c] = S.W[kSurOffW3 + (kSurH + 6) * kSurA + c];
    tab[L.cst + 2 * kTabLd + c] = S.W[kSurOffW4 + 2 * c];
    tab[L.cst + 3 * kTabLd + c] = S.W[kSurOffW4 + 2 * c + 1];
  }
  for (int g = threadIdx.x; g < NT; g += blockDim.x) {
    tab[L.yb + 2 * g] = T.yb[2 * g];
    tab[L.yb + 2 * g + 1] = T.yb[2 * g + 1];
    tab[L.nbg + g] = (float)T.nbg[g];
    tab[L.nfg + g] = (float)T.nfg[g];
  }
  if (threadIdx.x < 4) tab[L.scal + threadIdx.x] = T.scal[threadIdx.x];
  if (threadIdx.x < 3) tab[L.topg + threadIdx.x] = (float)T.top_g[threadIdx.x];
  stage(img, P.image, P.lay.total_words);
  __syncthreads();
  const View V = make_view(img, P.lay, P.dist);
  const uint32_t it = P.st->it;
  const float gate = (float)P.st->t_best * S.inv_t0 + mk_margin;
  const float b40 = S.W[kSurOffB4], b41 = S.W[kSurOffB4 + 1];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, q = lane >> 4;
  // Feature rows: [row k][half][proposal][4 words] (each half holds 8 bf16).
  uint32_t *rows = reinterpret_cast<uint32_t *>(lds + L.rows + wave * kFuseWaveBytes);
  const uint32_t ntask = (cnt + 63) / 64;
  for (uint32_t task = blockIdx.x * nwaves + wave; task < ntask; task += gridDim.x * nwaves) {
    // Phase 1: one proposal per lane.
    uint32_t own[kDescWords];
    {
      const uint32_t j = task * 64 + lane;
      int rf[3] = {-1, -1, -1}, rb[3] = {0, 0, 0}, rp[3] = {-1, -1, -1};
      ScreenDesc dd;
      if (j < cnt) {
        const Move m = decode_move(draw_move(seed, i0 + j, it, inst_index, V, P), V, P);
        describe(V, S, T, m, dd, rf, rb, rp);
        desc_pack(dd, own);
      } else {
        for (int w = 0; w < kDescWords; ++w) own[w] = 0;   // infeasible: no key is written
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        uint32_t pk[8];
        if (rf[k] >= 0) {
          float v[16];
          feature_vals(V, P, S, rf[k], rb[k], rp[k], v);
          for (int x = 0; x < 8; ++x) pk[x] = (uint32_t)to_bf16(v[2 * x]) | ((uint32_t)to_bf16(v[2 * x + 1]) << 16);
        } else {
          for (int x = 0; x < 8; ++x) pk[x] = 0u;
        }
        *reinterpret_cast<uint4 *>(rows + ((2 * k) * 64 + lane) * 4) = uint4{pk[0], pk[1], pk[2], pk[3]};
        *reinterpret_cast<uint4 *>(rows + ((2 * k + 1) * 64 + lane) * 4) = uint4{pk[4], pk[5], pk[6], pk[7]};
      }
    }
    wave_sync();
    // Phase 2: 16 proposals at a time.
#pragma unroll 1
    for (int grp = 0; grp < 4; ++grp) {
      // Keeps the weight operands from being hoisted out of the loop into
      // registers (they are re-read from LDS for every group).
      __asm__ volatile("" ::: "memory");
      const int p = 16 * grp + r;
      // The descriptor of proposal p.
      ScreenDesc d;
      {
        uint32_t ew[kDescWords];
#pragma unroll
        for (int w = 0; w < kDescWords; ++w) ew[w] = (uint32_t)__shfl((int)own[w], p, 64);
        desc_unpack(ew, d);
      }
      // Base rows of the changed fields (global memory: issued before the MLP).
      int prow[3];
      float4 pb[3][4];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        prow[k] = d.f[k] != 0xFFFF ? V.pos[d.f[k]] : 0;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
          pb[k][mt] = *reinterpret_cast<const float4 *>(S.P + (size_t)prow[k] * kSurA + 16 * mt + 4 * q);
      }
      // Layer 1: 16 (padded to 32) -> 128, bias (as the accumulator's start),
      // ReLU.  All 24 products are issued before the first result is used.
      bf16x8 h1[3][4];
      {
        bf16x8 x[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) x[k] = q < 2 ? ld8(reinterpret_cast<const uint16_t *>(rows + ((2 * k + q) * 64 + p) * 4)) : zero8();
        floatx4 acc[3][8];
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) {
          const bf16x8 a = ld8(w1 + (nt * 16 + r) * kLd1 + 8 * q);
          const floatx4 bb = *reinterpret_cast<const floatx4 *>(b1 + nt * 16 + 4 * q);
#pragma unroll
          for (int k = 0; k < 3; ++k) acc[k][nt] = mfma(a, x[k], bb);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) {
            const uint32_t w[4] = {relu_bf16x2(acc[k][2 * ks][0], acc[k][2 * ks][1]),
                                   relu_bf16x2(acc[k][2 * ks][2], acc[k][2 * ks][3]),
                                   relu_bf16x2(acc[k][2 * ks + 1][0], acc[k][2 * ks + 1][1]),
                                   relu_bf16x2(acc[k][2 * ks + 1][2], acc[k][2 * ks + 1][3])};
            h1[k][ks] = pack8(w);
          }
      }
      // Layer 2: 128 -> 128, bias, ReLU; output tiles in pairs (six
      // independent accumulation chains).
      bf16x8 h2[3][4];
#pragma unroll
      for (int mp = 0; mp < 4; ++mp) {
        floatx4 acc[2][3];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const floatx4 bb = *reinterpret_cast<const floatx4 *>(b2 + (2 * mp + h) * 16 + 4 * q);
          acc[h][0] = acc[h][1] = acc[h][2] = bb;
        }
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const bf16x8 a = ld8(w2 + ((2 * mp + h) * 16 + r) * kLd2 + 32 * ks + 8 * q);
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[h][k] = mfma(a, h1[k][ks], acc[h][k]);
          }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const uint32_t w[4] = {relu_bf16x2(acc[0][k][0], acc[0][k][1]), relu_bf16x2(acc[0][k][2], acc[0][k][3]),
                                 relu_bf16x2(acc[1][k][0], acc[1][k][1]), relu_bf16x2(acc[1][k][2], acc[1][k][3])};
          h2[k][mp] = pack8(w);
        }
      }
      // Layer 3: the pooled-embedding rows of W3, 128 -> 64, no bias (twelve
      // independent chains).
      floatx4 pn[3][4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int k = 0; k < 3; ++k) pn[k][mt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          const bf16x8 a = ld8(w3 + (mt * 16 + r) * kLd2 + 32 * ks + 8 * q);
#pragma unroll
          for (int k = 0; k < 3; ++k) pn[k][mt] = mfma(a, h2[k][ks], pn[k][mt]);
        }
      // Per-lane coefficients: the head input of tour tt is its table row
      // plus sum_a cq[tt][a] Q[b_a] + sum_k (cn[tt][k] Pnew_k - cb[tt][k] Pbase_k)
      // (the changes of its BP means, over its new BP count) plus the field
      // count and return leg terms.
      const int g0 = d.tg[0] == 0xFFFF ? 0 : d.tg[0];
      const bool has1 = d.tg[1] != 0xFFFF;
      const int g1 = has1 ? d.tg[1] : g0;
      const int nb0 = (int)tab[L.nbg + g0] + d.dnb[0], nb1_ = (int)tab[L.nbg + g1] + d.dnb[1];
      const float i0n = nb0 > 0 ? rcp((float)nb0) : 0.f, i1n = nb1_ > 0 ? rcp((float)nb1_) : 0.f;
      float cq[2][4], en[2][4];
      int qrow[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int b = d.ab[a];
        const bool ok = b != 0xFFFF;
        const int bb = ok ? b : 0;
        qrow[a] = bb;
        const int bt = V.bp_tour[bb];
        const int ct = bb == d.moved_bp ? d.dst_tour : bt;
        const int cb = V.bp_len[bb], cn = cb + d.dcnt[a];
        const float io = ok && cb > 0 ? rcp((float)cb) : 0.f;
        const float in = ok && cn > 0 ? rcp((float)cn) : 0.f;
        en[0][a] = ct == g0 ? in * i0n : 0.f;
        en[1][a] = has1 && ct == g1 ? in * i1n : 0.f;
        cq[0][a] = en[0][a] - (bt == g0 ? io * i0n : 0.f);
        cq[1][a] = en[1][a] - (has1 && bt == g1 ? io * i1n : 0.f);
      }
      float cn_[2][3], cb_[2][3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const bool fv = d.f[k] != 0xFFFF;
        cn_[0][k] = cn_[1][k] = cb_[0][k] = cb_[1][k] = 0.f;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          if (fv && d.ab[a] != 0xFFFF && d.bnew[k] == d.ab[a]) {
            cn_[0][k] += en[0][a];
            cn_[1][k] += en[1][a];
          }
          if (fv && d.ab[a] != 0xFFFF && d.bold[k] == d.ab[a]) {
            cb_[0][k] += en[0][a];
            cb_[1][k] += en[1][a];
          }
        }
      }
      const float* rz0 = tab + L.rz + (3 * g0 + d.dnb[0] + 1) * kTabLd;
      const float* rz1 = tab + L.rz + (3 * g1 + d.dnb[1] + 1) * kTabLd;
      const float f0 = (float)d.dnf[0], f1 = (float)d.dnf[1];
      const float u60 = d.u6[0], u61 = d.u6[1];
      float y00 = 0.f, y01 = 0.f, y10 = 0.f, y11 = 0.f;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        // Bounds the loads in flight to one 4-column slice.
        __asm__ volatile("" ::: "memory");
        const int co = 16 * mt + 4 * q;
        float4 s0 = *reinterpret_cast<const float4 *>(rz0 + co);
        float4 s1 = *reinterpret_cast<const float4 *>(rz1 + co);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const float4 t = *reinterpret_cast<const float4 *>(tab + L.q + qrow[a] * kTabLd + co);
          s0 = fma4(cq[0][a], t, s0);
          s1 = fma4(cq[1][a], t, s1);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const float4 pnk = {pn[k][mt][0], pn[k][mt][1], pn[k][mt][2], pn[k][mt][3]};
          s0 = fma4(cn_[0][k], pnk, fma4(-cb_[0][k], pb[k][mt], s0));
          s1 = fma4(cn_[1][k], pnk, fma4(-cb_[1][k], pb[k][mt], s1));
        }
        const float4 c4 = *reinterpret_cast<const float4 *>(tab + L.cst + co);
        const float4 c6 = *reinterpret_cast<const float4 *>(tab + L.cst + kTabLd + co);
        const float4 v0 = *reinterpret_cast<const float4 *>(tab + L.cst + 2 * kTabLd + co);
        const float4 v1 = *reinterpret_cast<const float4 *>(tab + L.cst + 3 * kTabLd + co);
        const float4 a0 = relu4(fma4(u60, c6, fma4(f0, c4, s0)));
        const float4 a1 = relu4(fma4(u61, c6, fma4(f1, c4, s1)));
        y00 += dot4(a0, v0);
        y01 += dot4(a0, v1);
        y10 += dot4(a1, v0);
        y11 += dot4(a1, v1);
      }
#pragma unroll
      for (int off = 16; off < 64; off <<= 1) {
        y00 += __shfl_xor(y00, off, 64);
        y01 += __shfl_xor(y01, off, 64);
        y10 += __shfl_xor(y10, off, 64);
        y11 += __shfl_xor(y11, off, 64);
      }
      // Predicted path and makespan from the base's.
      float pp = tab[L.scal];
      float mm = -__builtin_inff();
      for (int k = 0; k < 3; ++k) {
        const int g = (int)tab[L.topg + k];
        if (g >= 0 && g != d.tg[0] && g != d.tg[1]) {
          mm = tab[L.scal + 1 + k];
          break;
        }
      }
      {
        const int nf = (int)tab[L.nfg + g0];
        if (nf > 0) pp -= tab[L.yb + 2 * g0];
        if (nf + d.dnf[0] > 0) {
          pp += y00 + b40;
          mm = fmaxf(mm, y01 + b41);
        }
      }
      if (has1) {
        const int nf = (int)tab[L.nfg + g1];
        if (nf > 0) pp -= tab[L.yb + 2 * g1];
        if (nf + d.dnf[1] > 0) {
          pp += y10 + b40;
          mm = fmaxf(mm, y11 + b41);
        }
      }
      const uint32_t j = task * 64 + p;
      if (q == 0 && j < cnt) T.keys[i0 + j] = d.feasible && mm <= gate ? score_key(pp) : 0xFFFFFFFFu;
    }
    wave_sync();
  }
}

// Radix selection of the k smallest score keys (three digit passes of
// 11, 11 and 10 bits), then an order-preserving compaction: every key below
// the k-th and the lowest-index ties at it.
__global__ void k_topk_hist(const uint32_t *keys, uint32_t n, int pass, const uint32_t *sel,
                            uint32_t *hist) {
  __shared__ uint32_t h[2048];
  for (int i = threadIdx.x; i < 2048; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const uint32_t p1 = sel[0], p12 = (sel[0] << 11) | sel[1];
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t k = keys[i];
    if (pass == 0)
      atomicAdd(&h[k >> 21], 1u);
    else if (pass == 1) {
      if ((k >> 21) == p1) atomicAdd(&h[(k >> 10) & 0x7FF], 1u);
    } else if ((k >> 10) == p12) {
      atomicAdd(&h[k & 0x3FF], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 2048; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// sel: [0..2] digits, [3] ranks still to take, [4] threshold key, [5] k.
__global__ void k_topk_pick(uint32_t *hist, uint32_t *sel, int pass, uint32_t k) {
  __shared__ uint32_t part[256];
  const int t = threadIdx.x;
  const uint32_t need = pass == 0 ? k : sel[3];
  uint32_t s = 0;
  for (int i = 0; i < 8; ++i) s += hist[t * 8 + i];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    uint32_t run = 0;
    int bin = 2047;
    uint32_t below = 0;
    bool found = false;
    for (int w = 0; w < 256 && !found; ++w) {
      if (run + part[w] >= need) {
        uint32_t r2 = run;
        for (int i = 0; i < 8; ++i) {
          const uint32_t hv = hist[w * 8 + i];
          if (r2 + hv >= need) {
            bin = w * 8 + i;
            below = r2;
            found = true;
            break;
          }
          r2 += hv;
        }
      }
      run += part[w];
    }
    if (!found) below = run;  // fewer keys than k: take them all
    sel[pass] = (uint32_t)bin;
    sel[3] = need - below;
    if (pass == 0) sel[5] = k;
    if (pass == 2) sel[4] = (sel[0] << 21) | (sel[1] << 10) | sel[2];
  }
  __syncthreads();
  for (int i = t; i < 2048; i += blockDim.x) hist[i] = 0;
}

__device__ __forceinline__ void block_counts(uint32_t n, uint32_t &lo, uint32_t &hi) {
  const uint32_t per = (n + gridDim.x - 1) / gridDim.x;
  lo = blockIdx.x * per;
  hi = lo + per < n ? lo + per : n;
  if (lo > n) lo = n;
}

__global__ void k_topk_count(const uint32_t *keys, uint32_t n, const uint32_t *sel, uint32_t *blk) {
  __shared__ uint32_t c_lt, c_eq;
  if (threadIdx.x == 0) c_lt = c_eq = 0;
  __syncthreads();
  uint32_t lo, hi;
  block_counts(n, lo, hi);
  const uint32_t T = sel[4];
  uint32_t lt = 0, eq = 0;
  for (uint32_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const uint32_t k = keys[i];
    lt += k < T;
    eq += k == T;
  }
  atomicAdd(&c_lt, lt);
  atomicAdd(&c_eq, eq);
  __syncthreads();
  if (threadIdx.x == 0) {
    blk[blockIdx.x] = c_lt;
    blk[gridDim.x + blockIdx.x] = c_eq;
  }
}

// Per block: exclusive prefix of the keys equal to the threshold, then of
// the selected keys (those below it, and the first still-needed ties in index
// order).  nblk == blockDim.x == 1024, one workgroup.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const uint32_t x = t >= off ? sh[t - off] : 0u;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  const uint32_t incl = sh[t];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(1024) void k_topk_scan(uint32_t *blk, uint32_t nblk, const uint32_t *sel) {
  __shared__ uint32_t sh[1024];
  const uint32_t i = threadIdx.x;
  const uint32_t need_eq = sel[3];
  const uint32_t lt = blk[i], eq = blk[nblk + i];
  const uint32_t e = block_excl_scan(eq, sh);
  const uint32_t take = e >= need_eq ? 0u : (need_eq - e < eq ? need_eq - e : eq);
  const uint32_t t = block_excl_scan(lt + take, sh);
  blk[i] = t;
  blk[nblk + i] = e;
}

// The selected indices in ascending order: below the threshold, or equal to
// it within the first sel[3] such keys.
__global__ void k_topk_write(const uint32_t *keys, uint32_t n, const uint32_t *sel, const uint32_t *blk,
                             uint32_t *out) {
  __shared__ uint32_t w_sel[8], w_eq[8];
  uint32_t lo, hi;
  block_counts(n, lo, hi);
  const uint32_t T = sel[4], need_eq = sel[3];
  uint32_t off_sel = blk[blockIdx.x], off_eq = blk[gridDim.x + blockIdx.x];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (uint32_t base = lo; base < hi; base += blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t key = i < hi ? keys[i] : 0xFFFFFFFFu;
    const bool is_lt = i < hi && key < T, is_eq = i < hi && key == T;
    // Rank of this tie among the block's ties so far.
    const uint64_t be = __ballot(is_eq);
    if (lane == 0) w_eq[wave] = (uint32_t)__popcll(be);
    __syncthreads();
    uint32_t pe = 0, te = 0;
    for (int w = 0; w < nw; ++w) {
      if (w < wave) pe += w_eq[w];
      te += w_eq[w];
    }
    const bool take = is_lt || (is_eq && off_eq + pe + (uint32_t)__popcll(be & below) < need_eq);
    const uint64_t bs = __ballot(take);
    if (lane == 0) w_sel[wave] = (uint32_t)__popcll(bs);
    __syncthreads();
    uint32_t ps = 0, ts = 0;
    for (int w = 0; w < nw; ++w) {
      if (w < wave) ps += w_sel[w];
      ts += w_sel[w];
    }
    if (take) out[off_sel + ps + (uint32_t)__popcll(bs & below)] = i;
    off_sel += ts;
    off_eq += te;
    __syncthreads();
  }
}

// Scores of the screened proposals as floats (+inf: discarded).
__global__ void k_scr_export(const uint32_t *keys, uint32_t n, float *out) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t k = keys[i];
    out[i] = k == 0xFFFFFFFFu ? __builtin_inff() : key_score(k);
  }
}

// How well the screen ranks.  Scatter: the standard deviation of (predicted -
// exact) path over the shortlisted candidates with an exact cost, divided by
// their mean exact cost (a common offset does not change the ranking, so it
// is not counted).  Fallback when no shortlisted candidate passed the exact
// gate, when the control sample's best key beats the shortlist's, or when
// the scatter exceeds the threshold.  Per-block partial sums (double) and
// key minima into part[5 * gridDim.x], then one thread combines them in
// block order (deterministic).
__global__ __launch_bounds__(256) void k_scr_check_part(SurDev S, ScreenDev T, uint32_t k, double *part) {
  __shared__ double s_v[4][256];
  __shared__ uint64_t s_min[256];
  double r1 = 0.0, r2 = 0.0, ex = 0.0, cnt = 0.0;
  uint64_t kmin = kInfKey;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < k; j += gridDim.x * blockDim.x) {
    const uint64_t xk = T.short_key[j];
    kmin = xk < kmin ? xk : kmin;
    const float cost = T.short_cost[j];
    const uint32_t key = T.keys[T.short_idx[j]];
    if (!__builtin_isfinite(cost) || key == 0xFFFFFFFFu || cost <= 0.f) continue;
    const double r = (double)key_score(key) / (double)S.inv_c0 * 1e-3 - (double)cost;
    r1 += r;
    r2 += r * r;
    ex += (double)cost;
    cnt += 1.0;
  }
  s_v[0][threadIdx.x] = r1;
  s_v[1][threadIdx.x] = r2;
  s_v[2][threadIdx.x] = ex;
  s_v[3][threadIdx.x] = cnt;
  s_min[threadIdx.x] = kmin;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      for (int q = 0; q < 4; ++q) s_v[q][threadIdx.x] += s_v[q][threadIdx.x + off];
      const uint64_t o = s_min[threadIdx.x + off];
      if (o < s_min[threadIdx.x]) s_min[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) part[5 * blockIdx.x + threadIdx.x] = s_v[threadIdx.x][0];
  if (threadIdx.x == 4) reinterpret_cast<uint64_t *>(part)[5 * blockIdx.x + 4] = s_min[0];
}

__global__ void k_scr_check(InstParams P, ScreenDev T, const double *part, uint32_t nblk, float err_thr) {
  if (threadIdx.x == 0) {
    double r1 = 0.0, r2 = 0.0, ex = 0.0, cnt = 0.0;
    uint64_t smin = kInfKey;
    for (uint32_t i = 0; i < nblk; ++i) {
      r1 += part[5 * i];
      r2 += part[5 * i + 1];
      ex += part[5 * i + 2];
      cnt += part[5 * i + 3];
      const uint64_t m = reinterpret_cast<const uint64_t *>(part)[5 * i + 4];
      smin = m < smin ? m : smin;
    }
    float scatter = __builtin_inff();
    if (cnt > 0.0) {
      const double mean = r1 / cnt, var = r2 / cnt - mean * mean;
      scatter = (float)(sqrt(var > 0.0 ? var : 0.0) / (ex / cnt));
    }
    // The screen lost when the control sample improves on x* and beats the
    // shortlist (late in a search neither improves, and the least bad move of
    // an unscreened sample is no reason to evaluate the plain batch).
    const uint64_t ck = *T.ctrl_key;
    const bool lost = ck < smin && (ck >> 24) < P.st->cost_best;
    const uint32_t fb = (smin == kInfKey || lost || scatter > err_thr) ? 1u : 0u;
    *T.flag = fb;
    T.stats[0] = scatter;
    T.stats[1] += (float)fb;
    T.stats[2] += 1.f;
    T.stats[3] = (float)cnt;
  }
}

// The control sample's best key (the instance's argmin slot after its
// launch), kept before the shortlist joins the argmin.
__global__ void k_scr_control_save(const uint64_t *best_key, uint64_t *ctrl_key) { *ctrl_key = *best_key; }

}  // namespace

// Sizes of the bf16 operand copies (elements).
size_t sur_w1t_elems() { return 128 * kLd1; }
size_t sur_w2_elems() { return 128 * kLd2; }
size_t sur_w3et_elems() { return 64 * kLd2; }
size_t sur_w3en_elems() { return 128 * kLd3; }

hipError_t launch_sur_pack(const SurDev &S, hipStream_t s) {
  hipLaunchKernelGGL(k_sur_pack, dim3(64), dim3(256), 0, s, S);
  return hipGetLastError();
}

hipError_t launch_sur_zero(float *p, uint32_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_sur_zero, dim3(64), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// Features, forward MLP and head for n examples drawn against the base.
hipError_t launch_sur_forward(const InstParams &P, const SurDev &S, const uint64_t *moves,
                              uint32_t n, int noop, bool keep_act, int n_cu, hipStream_t s) {
  const size_t lds_img = (size_t)round4(P.lay.total_words) * 4;
  const uint32_t per_block = 4u * (64u / (uint32_t)P.seg);
  const uint32_t fb = std::min<uint32_t>((n + per_block - 1) / per_block, (uint32_t)n_cu * 4);
  hipLaunchKernelGGL(k_sur_feat, dim3(fb), dim3(256), lds_img, s, P, S, moves, n, noop);
  const uint32_t rows = n * (uint32_t)P.NF;
  const size_t lds_fwd = (size_t)(128 * kLd1 + 128 * kLd2 + 64 * kLd2) * 2 + 256 * 4 + 4 * 16 * kLd2 * 2;
  const uint32_t tiles = (rows + 15) / 16;
  const uint32_t gb = std::min<uint32_t>((tiles + 3) / 4, (uint32_t)n_cu * 2);
  hipLaunchKernelGGL(k_sur_fwd, dim3(gb), dim3(256), lds_fwd, s, S, S.phi, rows, S.P,
                     keep_act ? S.h1 : nullptr, keep_act ? S.h2 : nullptr);
  return hipGetLastError();
}

uint32_t sur_head_grid(uint32_t n, int n_cu) { return std::min<uint32_t>((n + 3) / 4, (uint32_t)n_cu * 4); }
uint32_t sur_bwd_grid(uint32_t rows, int n_cu) { return std::min<uint32_t>((rows + 31) / 32, (uint32_t)n_cu); }

hipError_t launch_sur_head(const InstParams &P, const SurDev &S, uint32_t n, int train,
                           const float *cost_km, const int32_t *mk, int n_cu, hipStream_t s) {
  const size_t lds = (size_t)4 * P.NB * kSurA * 4;
  const uint32_t gb = sur_head_grid(n, n_cu);
  hipLaunchKernelGGL(k_sur_head, dim3(gb), dim3(256), lds, s, P, S, n, train, cost_km, mk);
  return hipGetLastError();
}

hipError_t launch_sur_backward(const InstParams &P, const SurDev &S, uint32_t n, int n_cu,
                               hipStream_t s) {
  const uint32_t rows = n * (uint32_t)P.NF;
  const size_t lds = (size_t)(128 * kLd2 + 128 * kLd3 + 32 * kLd3 + 32 * kLd2 + 16 * kLd1 +
                              128 * kLd1 * 2 + 64 * kLd1 + 128 * kLd1 * 2) * 2;
  const uint32_t gb = sur_bwd_grid(rows, n_cu);
  hipLaunchKernelGGL(k_sur_bwd, dim3(gb), dim3(256), lds, s, S, rows);
  hipLaunchKernelGGL(k_sur_gsum, dim3((kSurParams + 2 + 63) / 64), dim3(1024), 0, s, S,
                     4 * sur_head_grid(n, n_cu), gb);
  return hipGetLastError();
}

hipError_t launch_sur_adam(const SurDev &S, float lr, float b1, float b2, float eps, float scale,
                           uint32_t step, hipStream_t s) {
  const float bc1 = 1.f - powf(b1, (float)step), bc2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_sur_adam, dim3(64), dim3(256), 0, s, S, lr, b1, b2, eps, scale, bc1, bc2);
  return hipGetLastError();
}

size_t sur_head_lds(const InstParams &P) { return (size_t)4 * P.NB * kSurA * 4; }

// Waves per workgroup of the fused screen kernel on instance P (0: its
// tables and image leave no room for one wave in LDS).
int screen_waves(const InstParams &P) {
  for (int w = kFuseMaxWaves; w >= 1; --w)
    if (fuse_layout(P.NB, P.NT, P.lay.total_words, w).total <= kFuseLdsMax) return w;
  return 0;
}

// The screen of one iteration in three launches: the base's forward pass
// and tables; the fused kernel's score keys of proposals 0 .. n_prop - 1;
// the k best-predicted proposal indices into T.short_idx.
hipError_t launch_screen_base(const InstParams &P, const SurDev &S, const ScreenDev &T, int n_cu,
                              hipStream_t s) {
  hipError_t e = launch_sur_forward(P, S, nullptr, 1, 1, false, n_cu, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scr_tables, dim3(1), dim3(1024), 0, s, P, S, T);
  return hipGetLastError();
}

hipError_t launch_screen_score(const InstParams &P, const SurDev &S, const ScreenDev &T, uint64_t seed,
                               uint32_t inst_index, uint32_t n_prop, float mk_margin, int n_cu,
                               hipStream_t s) {
  const int waves = screen_waves(P);
  if (waves == 0) return hipErrorInvalidValue;
  const uint32_t lds = fuse_layout(P.NB, P.NT, P.lay.total_words, waves).total;
  const uint32_t tasks = (n_prop + 63) / 64;
  const uint32_t grid = std::min<uint32_t>((tasks + waves - 1) / waves, (uint32_t)n_cu);
  hipLaunchKernelGGL(k_scr_fused, dim3(grid), dim3(64 * waves), lds, s, P, S, T, seed, inst_index, 0u,
                     n_prop, mk_margin);
  return hipGetLastError();
}

hipError_t launch_screen_select(const ScreenDev &T, uint32_t n_prop, uint32_t k, hipStream_t s) {
  hipLaunchKernelGGL(k_sur_zero, dim3(8), dim3(256), 0, s, reinterpret_cast<float *>(T.hist), 2048u);
  hipLaunchKernelGGL(k_sur_zero, dim3(1), dim3(64), 0, s, reinterpret_cast<float *>(T.sel), 8u);
  for (int pass = 0; pass < 3; ++pass) {
    hipLaunchKernelGGL(k_topk_hist, dim3(1024), dim3(256), 0, s, T.keys, n_prop, pass, T.sel, T.hist);
    hipLaunchKernelGGL(k_topk_pick, dim3(1), dim3(256), 0, s, T.hist, T.sel, pass, k);
  }
  hipLaunchKernelGGL(k_topk_count, dim3(1024), dim3(256), 0, s, T.keys, n_prop, T.sel, T.blk);
  hipLaunchKernelGGL(k_topk_scan, dim3(1), dim3(1024), 0, s, T.blk, 1024u, T.sel);
  hipLaunchKernelGGL(k_topk_write, dim3(1024), dim3(256), 0, s, T.keys, n_prop, T.sel, T.blk, T.short_idx);
  return hipGetLastError();
}

hipError_t launch_scr_control_save(const InstParams &P, const ScreenDev &T, hipStream_t s) {
  hipLaunchKernelGGL(k_scr_control_save, dim3(1), dim3(1), 0, s, P.best_key, T.ctrl_key);
  return hipGetLastError();
}

hipError_t launch_scr_export(const ScreenDev &T, uint32_t n, float *score, hipStream_t s) {
  const uint32_t gb = std::min<uint32_t>((n + 255) / 256, 1024u);
  hipLaunchKernelGGL(k_scr_export, dim3(gb), dim3(256), 0, s, T.keys, n, score);
  return hipGetLastError();
}

hipError_t launch_scr_check(const InstParams &P, const SurDev &S, const ScreenDev &T, uint32_t k,
                            float err_thr, hipStream_t s) {
  // The radix-select block counts are no longer needed: their buffer holds
  // the partial sums.
  const uint32_t nb = std::min<uint32_t>((k + 255) / 256, 192u);  // 5 words of 8 bytes each fit T.blk
  double *part = reinterpret_cast<double *>(T.blk);
  hipLaunchKernelGGL(k_scr_check_part, dim3(nb), dim3(256), 0, s, S, T, k, part);
  hipLaunchKernelGGL(k_scr_check, dim3(1), dim3(64), 0, s, P, T, part, nb, err_thr);
  return hipGetLastError();
}

hipError_t sur_setup_attributes() {
  const int fwd = (128 * kLd1 + 128 * kLd2 + 64 * kLd2) * 2 + 256 * 4 + 4 * 16 * kLd2 * 2;
  const int bwd = (128 * kLd2 + 128 * kLd3 + 32 * kLd3 + 32 * kLd2 + 16 * kLd1 + 128 * kLd1 * 2 +
                   64 * kLd1 + 128 * kLd1 * 2) * 2;
  hipError_t e = hipFuncSetAttribute((const void *)k_sur_fwd,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, fwd);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)k_sur_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, bwd);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void *)k_scr_fused, hipFuncAttributeMaxDynamicSharedMemorySize,
                          kFuseLdsMax);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void *)k_sur_head, hipFuncAttributeMaxDynamicSharedMemorySize,
                             160 * 1024);
}

}  // namespace bl
