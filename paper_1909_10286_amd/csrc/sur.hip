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
