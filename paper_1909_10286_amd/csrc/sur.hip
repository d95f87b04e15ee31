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
    for (int j = 0; j < kSurU; ++j) atomicAdd(&S.G[kSurOffW3 + (kSurH + j) * kSurA + c], gw3u[j]);
    atomicAdd(&S.G[kSurOffB3 + c], gb3);
    atomicAdd(&S.G[kSurOffW4 + c * 2], gw40);
    atomicAdd(&S.G[kSurOffW4 + c * 2 + 1], gw41);
    if (c == 0) {
      atomicAdd(&S.G[kSurOffB4], gb40);
      atomicAdd(&S.G[kSurOffB4 + 1], gb41);
      atomicAdd(&S.loss[0], lsum);
      atomicAdd(&S.loss[1], lcnt);
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
  for (uint32_t ch = blockIdx.x; ch < chunks; ch += gridDim.x) {
    const uint32_t row0 = ch * 32;
    __syncthreads();
    for (int i = threadIdx.x; i < 32 * 64; i += blockDim.x) {
      const int rr = i >> 6, cc = i & 63;
      const float v = row0 + rr < n_rows ? S.dP[(size_t)(row0 + rr) * kSurA + cc] : 0.f;
      const uint16_t bv = to_bf16(v);
      dPr[rr * kLd3 + cc] = bv;
      dPT[cc * kLd1 + rr] = bv;
    }
    for (int i = threadIdx.x; i < 32 * 128; i += blockDim.x) {
      const int rr = i >> 7, cc = i & 127;
      const bool v = row0 + rr < n_rows;
      h1T[cc * kLd1 + rr] = v ? S.h1[(size_t)(row0 + rr) * 128 + cc] : (uint16_t)0;
      h2T[cc * kLd1 + rr] = v ? S.h2[(size_t)(row0 + rr) * 128 + cc] : (uint16_t)0;
    }
    for (int i = threadIdx.x; i < 32 * 16; i += blockDim.x) {
      const int rr = i >> 4, cc = i & 15;
      phiT[cc * kLd1 + rr] = row0 + rr < n_rows ? S.phi[(size_t)(row0 + rr) * kSurK1 + cc] : (uint16_t)0;
    }
    __syncthreads();
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
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int tile = wave * 8 + k;
    for (int i = 0; i < 4; ++i)
      atomicAdd(&S.G[kSurOffW3 + ((tile >> 2) * 16 + 4 * kb + i) * kSurA + (tile & 3) * 16 + r],
                acc3[k][i]);
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int tile = wave * 16 + k;
    for (int i = 0; i < 4; ++i)
      atomicAdd(&S.G[kSurOffW2 + ((tile >> 3) * 16 + 4 * kb + i) * kSurH + (tile & 7) * 16 + r],
                acc2[k][i]);
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int tile = wave * 2 + k;
    for (int i = 0; i < 4; ++i)
      atomicAdd(&S.G[kSurOffW1 + (4 * kb + i) * kSurH + tile * 16 + r], acc1[k][i]);
  }
  for (int k = 0; k < 4; ++k) {
    const int nt = (wave * 4 + k) & 7;
    float v2 = gb2[k], v1 = gb1[k];
    v2 += __shfl_xor(v2, 16, 64);
    v2 += __shfl_xor(v2, 32, 64);
    v1 += __shfl_xor(v1, 16, 64);
    v1 += __shfl_xor(v1, 32, 64);
    if (kb == 0) {
      atomicAdd(&S.G[kSurOffB2 + nt * 16 + r], v2);
      atomicAdd(&S.G[kSurOffB1 + nt * 16 + r], v1);
    }
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

__device__ __forceinline__ void feature_row(const View &V, const InstParams &P, const SurDev &S,
                                            uint16_t *dst, int f, int b, int pred) {
  const int nb1 = 1 + P.NB;
  const size_t Vn = (size_t)P.V;
  const float *fs = S.fstat + (size_t)f * 8;
  const uint32_t dfb = V.D[(size_t)(nb1 + f) * Vn + 1 + b];
  const uint32_t leg = pred < 0 ? V.dhq[f] : V.D[(size_t)(nb1 + pred) * Vn + nb1 + f];
  float v[16] = {fs[0], fs[1], fs[2], fs[3], S.bxy[2 * b], S.bxy[2 * b + 1],
                 (float)dfb * S.inv_ds, (float)leg * S.inv_ds, fs[5] * (float)dfb, fs[4],
                 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  write_row(dst, v);
}

__device__ __forceinline__ void add_bp(ScreenDesc &d, int b, int dc) {
  for (int a = 0; a < 4; ++a) {
    if (d.ab[a] == (uint16_t)b) {
      d.dcnt[a] += (int16_t)dc;
      return;
    }
    if (d.ab[a] == 0xFFFF) {
      d.ab[a] = (uint16_t)b;
      d.dcnt[a] = (int16_t)dc;
      return;
    }
  }
}

// Descriptor and changed feature rows (3 per proposal) of proposals
// i0 .. i0 + cnt - 1, one thread each.
__global__ __launch_bounds__(256) void k_scr_rows(InstParams P, SurDev S, ScreenDev T, uint64_t seed,
                                                  uint32_t inst_index, uint32_t i0, uint32_t cnt) {
  uint32_t *lds = reinterpret_cast<uint32_t *>(g_lds4);
  stage(lds, P.image, P.lay.total_words);
  __syncthreads();
  const View V = make_view(lds, P.lay, P.dist);
  const uint32_t it = P.st->it;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < cnt; j += gridDim.x * blockDim.x) {
    const Move m = decode_move(draw_move(seed, i0 + j, it, inst_index, V, P), V, P);
    ScreenDesc d;
    for (int k = 0; k < 3; ++k) d.f[k] = d.bold[k] = d.bnew[k] = 0xFFFF;
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
    int rf[3] = {-1, -1, -1}, rb[3] = {0, 0, 0}, rp[3] = {-1, -1, -1};
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
    // Rows whose route predecessor or BP changes: the moved run's first
    // field, the field after the insertion point and the one after the gap.
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
      uint16_t *row = T.phi + ((size_t)j * 3 + k) * kSurK1;
      if (rf[k] >= 0) {
        d.f[k] = (uint16_t)rf[k];
        d.bnew[k] = (uint16_t)rb[k];
        add_bp(d, rb[k], 0);
        add_bp(d, d.bold[k], 0);
        feature_row(V, P, S, row, rf[k], rb[k], rp[k]);
      } else {
        float z[16] = {0.f};
        write_row(row, z);
      }
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
    T.desc[j] = d;
  }
}

// Predicted (path, makespan) of proposals i0 .. i0+cnt-1 from their
// descriptors and projected rows; writes their score keys (predicted path,
// or discarded when infeasible or above the makespan gate).  One wave per
// proposal, lane c = embedding column c: every row read is one coalesced
// 256-byte line.
__global__ __launch_bounds__(256) void k_scr_score(InstParams P, SurDev S, ScreenDev T, uint32_t i0,
                                                   uint32_t cnt, float mk_margin) {
  const View V = make_view(P.image, P.lay, P.dist);
  const int c = threadIdx.x & 63;
  const float gate = (float)P.st->t_best * S.inv_t0 + mk_margin;
  const float b40 = S.W[kSurOffB4], b41 = S.W[kSurOffB4 + 1];
  const float w3u4 = S.W[kSurOffW3 + (kSurH + 4) * kSurA + c] / (float)P.NF;
  const float w3u5 = S.W[kSurOffW3 + (kSurH + 5) * kSurA + c] / (float)P.NB;
  const float w3u6 = S.W[kSurOffW3 + (kSurH + 6) * kSurA + c];
  const float w40 = S.W[kSurOffW4 + 2 * c], w41 = S.W[kSurOffW4 + 2 * c + 1];
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint32_t nwave = (gridDim.x * blockDim.x) >> 6;
  for (uint32_t j = wave; j < cnt; j += nwave) {
    const ScreenDesc d = T.desc[j];
    uint32_t key = 0xFFFFFFFFu;
    if (d.feasible) {
      // BP means before and after, column c.
      float eo[4], en[4];
      int bt[4], ct[4];
      const float *pr = T.P + (size_t)j * 3 * kSurA;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        eo[a] = en[a] = 0.f;
        bt[a] = ct[a] = -1;
        const int b = d.ab[a];
        if (b == 0xFFFF) continue;
        bt[a] = V.bp_tour[b];
        ct[a] = b == d.moved_bp ? d.dst_tour : bt[a];
        const int cb = V.bp_len[b], cn = cb + d.dcnt[a];
        const float qo = T.Q[b * kSurA + c];
        float qn = qo;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          if (d.f[k] == 0xFFFF) continue;
          if (d.bold[k] == b) qn -= S.P[(size_t)V.pos[d.f[k]] * kSurA + c];
          if (d.bnew[k] == b) qn += pr[k * kSurA + c];
        }
        eo[a] = cb > 0 ? qo / (float)cb : 0.f;
        en[a] = cn > 0 ? qn / (float)cn : 0.f;
      }
      float y0[2] = {0.f, 0.f}, y1[2] = {0.f, 0.f};
#pragma unroll
      for (int tt = 0; tt < 2; ++tt) {
        if (d.tg[tt] == 0xFFFF) continue;
        const int g = d.tg[tt];
        float R = T.R[g * kSurA + c];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          if (bt[a] == g) R -= eo[a];
          if (ct[a] == g) R += en[a];
        }
        const int nbn = T.nbg[g] + d.dnb[tt];
        const float z = (nbn > 0 ? R / (float)nbn : 0.f) + T.U[g * kSurA + c] + (float)d.dnf[tt] * w3u4 +
                        (float)d.dnb[tt] * w3u5 + (d.u6[tt] - T.ub6[g]) * w3u6;
        const float act = fmaxf(z, 0.f);
        y0[tt] = wave_sum(act * w40) + b40;
        y1[tt] = wave_sum(act * w41) + b41;
      }
      float pp = T.scal[0];
      float mm = -__builtin_inff();
      for (int k = 0; k < 3; ++k) {
        const int g = T.top_g[k];
        if (g >= 0 && g != d.tg[0] && g != d.tg[1]) {
          mm = T.scal[1 + k];
          break;
        }
      }
      for (int tt = 0; tt < 2; ++tt) {
        if (d.tg[tt] == 0xFFFF) continue;
        const int g = d.tg[tt];
        if (T.nfg[g] > 0) pp -= T.yb[2 * g];
        if (T.nfg[g] + d.dnf[tt] > 0) {
          pp += y0[tt];
          mm = fmaxf(mm, y1[tt]);
        }
      }
      if (mm <= gate) key = score_key(pp);
    }
    if (c == 0) T.keys[i0 + j] = key;
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

// The judge of the screen.  Scatter: the standard deviation of (predicted -
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
    const bool lost = *T.ctrl_key < smin;
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

hipError_t launch_sur_head(const InstParams &P, const SurDev &S, uint32_t n, int train,
                           const float *cost_km, const int32_t *mk, int n_cu, hipStream_t s) {
  const size_t lds = (size_t)4 * P.NB * kSurA * 4;
  const uint32_t gb = std::min<uint32_t>((n + 3) / 4, (uint32_t)n_cu * 4);
  hipLaunchKernelGGL(k_sur_head, dim3(gb), dim3(256), lds, s, P, S, n, train, cost_km, mk);
  return hipGetLastError();
}

hipError_t launch_sur_backward(const InstParams &P, const SurDev &S, uint32_t n, int n_cu,
                               hipStream_t s) {
  const uint32_t rows = n * (uint32_t)P.NF;
  const size_t lds = (size_t)(128 * kLd2 + 128 * kLd3 + 32 * kLd3 + 32 * kLd2 + 16 * kLd1 +
                              128 * kLd1 * 2 + 64 * kLd1 + 128 * kLd1 * 2) * 2;
  const uint32_t gb = std::min<uint32_t>((rows + 31) / 32, (uint32_t)n_cu);
  hipLaunchKernelGGL(k_sur_bwd, dim3(gb), dim3(256), lds, s, S, rows);
  return hipGetLastError();
}

hipError_t launch_sur_adam(const SurDev &S, float lr, float b1, float b2, float eps, float scale,
                           uint32_t step, hipStream_t s) {
  const float bc1 = 1.f - powf(b1, (float)step), bc2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_sur_adam, dim3(64), dim3(256), 0, s, S, lr, b1, b2, eps, scale, bc1, bc2);
  return hipGetLastError();
}

size_t sur_head_lds(const InstParams &P) { return (size_t)4 * P.NB * kSurA * 4; }

// Screen n_prop proposals against the base: base forward and tables, then
// chunks of descriptors + changed rows -> MLP rows -> scores, then the k
// best-predicted proposal indices into T.short_idx.
hipError_t launch_screen(const InstParams &P, const SurDev &S, const ScreenDev &T, uint64_t seed,
                         uint32_t inst_index, uint32_t n_prop, uint32_t k, float mk_margin,
                         uint32_t chunk, int n_cu, hipStream_t s) {
  hipError_t e = launch_sur_forward(P, S, nullptr, 1, 1, false, n_cu, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scr_tables, dim3(1), dim3(1024), 0, s, P, S, T);
  const size_t lds_img = (size_t)round4(P.lay.total_words) * 4;
  const size_t lds_fwd = (size_t)(128 * kLd1 + 128 * kLd2 + 64 * kLd2) * 2 + 256 * 4 + 4 * 16 * kLd2 * 2;
  for (uint32_t i0 = 0; i0 < n_prop; i0 += chunk) {
    const uint32_t cnt = std::min(chunk, n_prop - i0);
    const uint32_t gb = std::min<uint32_t>((cnt + 255) / 256, (uint32_t)n_cu * 4);
    hipLaunchKernelGGL(k_scr_rows, dim3(gb), dim3(256), lds_img, s, P, S, T, seed, inst_index, i0, cnt);
    const uint32_t rows = 3 * cnt, tiles = (rows + 15) / 16;
    const uint32_t gf = std::min<uint32_t>((tiles + 3) / 4, (uint32_t)n_cu * 2);
    hipLaunchKernelGGL(k_sur_fwd, dim3(gf), dim3(256), lds_fwd, s, S, T.phi, rows, T.P, nullptr, nullptr);
    const uint32_t gs = std::min<uint32_t>((cnt + 3) / 4, (uint32_t)n_cu * 8);
    hipLaunchKernelGGL(k_scr_score, dim3(gs), dim3(256), 0, s, P, S, T, i0, cnt, mk_margin);
  }
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
  return hipFuncSetAttribute((const void *)k_sur_head, hipFuncAttributeMaxDynamicSharedMemorySize,
                             160 * 1024);
}

}  // namespace bl
