// Host side of the C interface: contexts, instance validation and upload,
// the initial solution (Steps 1-3 of Algorithm 1), solution slots, and the
// launch sequence of the device-resident search iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/bl.h"
#include "bl_internal.h"

namespace bl {
int eval_occupancy(const InstParams &P, bool search);
}

using namespace bl;

namespace {

struct Instance {
  // host copies
  int NF = 0, NB = 0, NT = 0, NHU = 0, NSU = 0, V = 0;
  std::vector<uint32_t> dist, area, yld, demand, hu_rate, su_cap, su_speed, su_fill;
  std::vector<uint16_t> init_hu, init_su;
  std::vector<uint64_t> supply;
  uint32_t v_hu = 0, flags = 0;
  // device
  InstParams P{};
  uint32_t *d_dist = nullptr, *d_image = nullptr;
  uint16_t *d_sol = nullptr, *d_units = nullptr;
  SearchState *d_st = nullptr;
  TraceRow *d_trace = nullptr;
  uint64_t *d_best = nullptr;
  bool base_ready = false, started = false;
  int occ_batch = 1, occ_search = 1;
};

}  // namespace

struct bl_ctx {
  int device = 0;
  int n_cu = 256;
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<std::unique_ptr<Instance>> inst;
  // kernel timing: event pairs recorded around evaluation launches
  bool timing = false;
  std::vector<hipEvent_t> events;
  size_t events_used = 0;
};

namespace {

bl_status fail(bl_ctx *c, bl_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return s;
}

bl_status hip_fail(bl_ctx *c, hipError_t e, const char *where) {
  return fail(c, e == hipErrorOutOfMemory ? BL_ENOMEM : BL_EDEVICE, "%s: %s", where,
              hipGetErrorString(e));
}

#define HIP_TRY(c, expr)                                \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hip_fail(c, e_, #expr); \
  } while (0)

Instance *get_inst(bl_ctx *c, int32_t id) {
  if (!c || id < 0 || id >= (int32_t)c->inst.size()) return nullptr;
  return c->inst[id].get();
}

uint32_t next_pow2(uint32_t v) {
  uint32_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Word-offset allocator for the image.
struct Alloc {
  uint32_t words = 0;
  uint32_t u32(uint32_t n) {
    const uint32_t o = words;
    words += n;
    return o;
  }
  uint32_t u16(uint32_t n) { return u32((n + 1) / 2); }
  uint32_t u64(uint32_t n) {
    words = (words + 1) & ~1u;
    return u32(2 * n);
  }
};

void free_instance(Instance *I) {
  (void)hipFree(I->d_dist);
  (void)hipFree(I->d_image);
  (void)hipFree(I->d_sol);
  (void)hipFree(I->d_units);
  (void)hipFree(I->d_st);
  (void)hipFree(I->d_trace);
  (void)hipFree(I->d_best);
}

// Solution slot layout inside one u16 buffer.
struct SolLayout {
  size_t tour_off, tour_bp, bp_off, bp_field, hu_tour, su_tour, total;
};
SolLayout sol_layout(const Instance &I) {
  SolLayout L;
  size_t o = 0;
  L.tour_off = o; o += I.NT + 1;
  L.tour_bp = o; o += I.NB;
  L.bp_off = o; o += I.NB + 1;
  L.bp_field = o; o += I.NF;
  L.hu_tour = o; o += I.NHU;
  L.su_tour = o; o += I.NSU;
  L.total = (o + 127) & ~size_t(127);
  return L;
}

bl_status validate_solution(bl_ctx *c, const Instance &I, const bl_solution *s) {
  if (!s || !s->tour_off || !s->tour_bp || !s->bp_off || !s->bp_field || !s->hu_tour || !s->su_tour)
    return fail(c, BL_EINVAL, "solution: null array");
  if (s->tour_off[0] != 0 || s->tour_off[I.NT] != I.NB)
    return fail(c, BL_EINVAL, "solution: tour offsets must run 0..n_bps");
  for (int g = 0; g < I.NT; ++g)
    if (s->tour_off[g] > s->tour_off[g + 1]) return fail(c, BL_EINVAL, "solution: tour offsets decrease");
  if (s->bp_off[0] != 0 || s->bp_off[I.NB] != I.NF)
    return fail(c, BL_EINVAL, "solution: BP offsets must run 0..n_fields");
  for (int b = 0; b < I.NB; ++b)
    if (s->bp_off[b] > s->bp_off[b + 1]) return fail(c, BL_EINVAL, "solution: BP offsets decrease");
  std::vector<char> seen_b(I.NB, 0), seen_f(I.NF, 0);
  for (int j = 0; j < I.NB; ++j) {
    const int b = s->tour_bp[j];
    if (b >= I.NB || seen_b[b]) return fail(c, BL_EINVAL, "solution: BP %d missing or repeated", b);
    seen_b[b] = 1;
  }
  for (int i = 0; i < I.NF; ++i) {
    const int f = s->bp_field[i];
    if (f >= I.NF || seen_f[f]) return fail(c, BL_EINVAL, "solution: field %d missing or repeated", f);
    seen_f[f] = 1;
  }
  for (int h = 0; h < I.NHU; ++h)
    if (s->hu_tour[h] >= I.NT) return fail(c, BL_EINVAL, "solution: HU %d tour out of range", h);
  for (int u = 0; u < I.NSU; ++u)
    if (s->su_tour[u] >= I.NT) return fail(c, BL_EINVAL, "solution: SU %d tour out of range", u);
  return BL_OK;
}

// Records one timing event (when enabled); returns false on a HIP error.
hipError_t timing_mark(bl_ctx *c) {
  if (!c->timing) return hipSuccess;
  if (c->events_used == c->events.size()) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    c->events.push_back(e);
  }
  return hipEventRecord(c->events[c->events_used++], c->stream);
}

int grid_for(const bl_ctx *c, const Instance &I, uint32_t n, bool search) {
  const uint32_t per_block = 4u * (64u / (uint32_t)I.P.seg);
  const uint32_t need = (n + per_block - 1) / per_block;
  const uint32_t cap = (uint32_t)c->n_cu * (uint32_t)(search ? I.occ_search : I.occ_batch);
  return (int)std::max<uint32_t>(1u, std::min(need, cap));
}

}  // namespace

extern "C" {

const char *bl_status_str(bl_status s) {
  switch (s) {
    case BL_OK: return "ok";
    case BL_EINVAL: return "invalid argument";
    case BL_ENOMEM: return "out of memory";
    case BL_EDEVICE: return "device error";
    case BL_ESTATE: return "call out of order";
    case BL_EINFEASIBLE: return "infeasible initial solution";
    default: return "unknown status";
  }
}

const char *bl_last_error(const bl_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

bl_status bl_create(int32_t device, bl_ctx **out) {
  if (!out) return BL_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return BL_EDEVICE;
  if (device < 0 || device >= n) return BL_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return BL_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return BL_EDEVICE;
  bl_ctx *c = new (std::nothrow) bl_ctx();
  if (!c) return BL_ENOMEM;
  c->device = device;
  c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  *out = c;
  return BL_OK;
}

void bl_destroy(bl_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  (void)hipDeviceSynchronize();
  for (auto &I : ctx->inst) free_instance(I.get());
  for (auto e : ctx->events) (void)hipEventDestroy(e);
  delete ctx;
}

bl_status bl_set_stream(bl_ctx *ctx, void *hip_stream) {
  if (!ctx) return BL_EINVAL;
  ctx->stream = (hipStream_t)hip_stream;
  return BL_OK;
}

bl_status bl_instance_upload(bl_ctx *c, const bl_instance *in, int32_t *inst_id) {
  if (!c || !in || !inst_id) return fail(c, BL_EINVAL, "null argument");
  const int NF = in->n_fields, NB = in->n_bps, NT = in->n_tours, NHU = in->n_hus, NSU = in->n_sus;
  if (NF < 1 || NF > kMaxFields) return fail(c, BL_EINVAL, "n_fields %d out of 1..%d", NF, kMaxFields);
  if (NB < 1 || NB > kMaxBps) return fail(c, BL_EINVAL, "n_bps %d out of 1..%d", NB, kMaxBps);
  if (NT < 1 || NT > kMaxTours) return fail(c, BL_EINVAL, "n_tours %d out of 1..%d", NT, kMaxTours);
  if (NHU < NT || NHU > kMaxHus) return fail(c, BL_EINVAL, "n_hus %d must be in n_tours..%d", NHU, kMaxHus);
  if (NSU < 1 || NSU > kMaxSus) return fail(c, BL_EINVAL, "n_sus %d out of 1..%d", NSU, kMaxSus);
  if (!in->dist_m || !in->field_area || !in->field_yield || !in->bp_demand_kg || !in->hu_rate ||
      !in->su_cap_kg || !in->su_speed_mph || !in->su_fill_s)
    return fail(c, BL_EINVAL, "null instance array");
  if (in->hu_speed_mph == 0) return fail(c, BL_EINVAL, "hu_speed_mph must be > 0");
  if (in->flags & ~15u) return fail(c, BL_EINVAL, "unknown flags 0x%x", in->flags);
  auto I = std::make_unique<Instance>();
  I->NF = NF; I->NB = NB; I->NT = NT; I->NHU = NHU; I->NSU = NSU;
  const int V = 1 + NB + NF;
  I->V = V;
  I->dist.assign(in->dist_m, in->dist_m + (size_t)V * V);
  uint32_t dmax = 0;
  for (int i = 0; i < V; ++i) {
    if (I->dist[(size_t)i * V + i] != 0) return fail(c, BL_EINVAL, "dist_m diagonal must be 0");
    for (int j = i + 1; j < V; ++j) {
      const uint32_t a = I->dist[(size_t)i * V + j];
      if (a != I->dist[(size_t)j * V + i]) return fail(c, BL_EINVAL, "dist_m not symmetric at (%d,%d)", i, j);
      if (a >= (1u << 24)) return fail(c, BL_EINVAL, "dist_m entry >= 2^24 at (%d,%d)", i, j);
      dmax = std::max(dmax, a);
    }
  }
  I->area.assign(in->field_area, in->field_area + NF);
  I->yld.assign(in->field_yield, in->field_yield + NF);
  I->demand.assign(in->bp_demand_kg, in->bp_demand_kg + NB);
  I->hu_rate.assign(in->hu_rate, in->hu_rate + NHU);
  I->su_cap.assign(in->su_cap_kg, in->su_cap_kg + NSU);
  I->su_speed.assign(in->su_speed_mph, in->su_speed_mph + NSU);
  I->su_fill.assign(in->su_fill_s, in->su_fill_s + NSU);
  I->v_hu = in->hu_speed_mph;
  I->flags = in->flags;
  for (int h = 0; h < NHU; ++h)
    if (I->hu_rate[h] == 0) return fail(c, BL_EINVAL, "hu_rate[%d] must be > 0", h);
  uint64_t capsum = 0;
  for (int s = 0; s < NSU; ++s) {
    if (I->su_speed[s] == 0) return fail(c, BL_EINVAL, "su_speed_mph[%d] must be > 0", s);
    if (I->su_fill[s] >= (1u << 20)) return fail(c, BL_EINVAL, "su_fill_s[%d] >= 2^20", s);
    capsum += I->su_cap[s];
  }
  const uint64_t cbar = capsum / (uint64_t)NSU;
  if (cbar == 0) return fail(c, BL_EINVAL, "mean SU capacity is 0");
  // eq. (3) supply per field, eq. (4) shuttle drives with the mean capacity.
  I->supply.resize(NF);
  uint64_t tot_supply = 0, tot_area = 0, shuttle_bound = 0;
  std::vector<uint32_t> nsh(NF);
  for (int f = 0; f < NF; ++f) {
    const uint64_t s = (uint64_t)I->area[f] * (uint64_t)I->yld[f];
    I->supply[f] = s;
    tot_supply += s;
    tot_area += I->area[f];
    nsh[f] = (uint32_t)((s + cbar - 1) / cbar);
    shuttle_bound += 2ull * nsh[f] * dmax;
  }
  if (tot_supply >= (1ull << 32)) return fail(c, BL_EINVAL, "total supply >= 2^32 kg");
  if (tot_area >= (1ull << 32)) return fail(c, BL_EINVAL, "total area >= 2^32");
  uint64_t tot_demand = 0;
  for (int b = 0; b < NB; ++b) tot_demand += I->demand[b];
  if (tot_demand > tot_supply) return fail(c, BL_EINVAL, "total demand exceeds total supply");
  const uint64_t lmax = (uint64_t)(NF + 1) * dmax;
  if (lmax >= (1ull << 32)) return fail(c, BL_EINVAL, "tour length bound >= 2^32 m");
  if ((uint64_t)(NHU + NSU) * lmax + shuttle_bound >= (1ull << 40))
    return fail(c, BL_EINVAL, "path length bound >= 2^40 m (key packing)");
  if (in->init_hus_per_tour) {
    I->init_hu.assign(in->init_hus_per_tour, in->init_hus_per_tour + NT);
    int s = 0;
    for (auto v : I->init_hu) s += v;
    if (s != NHU) return fail(c, BL_EINVAL, "init_hus_per_tour must sum to n_hus");
  }
  if (in->init_sus_per_tour) {
    I->init_su.assign(in->init_sus_per_tour, in->init_sus_per_tour + NT);
    int s = 0;
    for (auto v : I->init_su) s += v;
    if (s != NSU) return fail(c, BL_EINVAL, "init_sus_per_tour must sum to n_sus");
  }
  // Unit ranks: HUs by (rate, id); SUs by (fill time, id descending), so the
  // highest rank among a tour's SUs is the critical one (largest fill time,
  // lowest id among equals).
  std::vector<int> hu_ord(NHU), su_ord(NSU);
  std::iota(hu_ord.begin(), hu_ord.end(), 0);
  std::iota(su_ord.begin(), su_ord.end(), 0);
  std::sort(hu_ord.begin(), hu_ord.end(), [&](int a, int b) {
    return I->hu_rate[a] != I->hu_rate[b] ? I->hu_rate[a] < I->hu_rate[b] : a < b;
  });
  std::sort(su_ord.begin(), su_ord.end(), [&](int a, int b) {
    return I->su_fill[a] != I->su_fill[b] ? I->su_fill[a] < I->su_fill[b] : a > b;
  });
  // Image layout.
  ImageLayout L{};
  Alloc al;
  L.area = al.u32(NF); L.supply = al.u32(NF); L.nsh = al.u32(NF); L.dhq = al.u32(NF);
  L.demand = al.u32(NB);
  L.hu_rate = al.u32(NHU); L.su_fill = al.u32(NSU); L.su_speed = al.u32(NSU);
  L.hu_rank = al.u16(NHU); L.su_rank = al.u16(NSU);
  L.static_words = al.words;
  L.seq = al.u16(NF); L.pos = al.u16(NF); L.fbp = al.u16(NF); L.fidx = al.u16(NF);
  L.leg_in = al.u32(NF); L.dfb = al.u32(NF);
  L.bp_start = al.u16(NB); L.bp_len = al.u16(NB); L.bp_tour = al.u16(NB); L.bp_idx = al.u16(NB);
  L.tour_off = al.u16(NT + 1); L.tour_bp = al.u16(NB);
  L.hu_mask = al.u64(NT); L.su_mask = al.u64(2 * NT);
  L.total_words = (al.words + 3) & ~3u;
  std::vector<uint32_t> img(L.total_words, 0);
  for (int f = 0; f < NF; ++f) {
    img[L.area + f] = I->area[f];
    img[L.supply + f] = (uint32_t)I->supply[f];
    img[L.nsh + f] = nsh[f];
    img[L.dhq + f] = I->dist[(size_t)(1 + NB + f)];
  }
  for (int b = 0; b < NB; ++b) img[L.demand + b] = I->demand[b];
  std::vector<uint16_t> hu_id(NHU), su_id(NSU);
  uint16_t *hu_rank = (uint16_t *)(img.data() + L.hu_rank);
  uint16_t *su_rank = (uint16_t *)(img.data() + L.su_rank);
  for (int r = 0; r < NHU; ++r) {
    img[L.hu_rate + r] = I->hu_rate[hu_ord[r]];
    hu_rank[hu_ord[r]] = (uint16_t)r;
    hu_id[r] = (uint16_t)hu_ord[r];
  }
  for (int r = 0; r < NSU; ++r) {
    img[L.su_fill + r] = I->su_fill[su_ord[r]];
    img[L.su_speed + r] = I->su_speed[su_ord[r]];
    su_rank[su_ord[r]] = (uint16_t)r;
    su_id[r] = (uint16_t)su_ord[r];
  }
  // Device buffers.
  HIP_TRY(c, hipSetDevice(c->device));
  Instance *R = I.get();
  auto cleanup = [&](bl_status s) {
    free_instance(R);
    return s;
  };
  hipError_t e;
  if ((e = hipMalloc(&R->d_dist, (size_t)V * V * 4)) != hipSuccess) return cleanup(hip_fail(c, e, "hipMalloc dist"));
  if ((e = hipMalloc(&R->d_image, (size_t)L.total_words * 4)) != hipSuccess) return cleanup(hip_fail(c, e, "hipMalloc image"));
  const SolLayout SL = sol_layout(*R);
  if ((e = hipMalloc(&R->d_sol, SL.total * 3 * sizeof(uint16_t))) != hipSuccess) return cleanup(hip_fail(c, e, "hipMalloc sol"));
  if ((e = hipMalloc(&R->d_units, (size_t)(NHU + NSU) * sizeof(uint16_t))) != hipSuccess) return cleanup(hip_fail(c, e, "hipMalloc units"));
  if ((e = hipMalloc(&R->d_st, sizeof(SearchState))) != hipSuccess) return cleanup(hip_fail(c, e, "hipMalloc state"));
  if ((e = hipMalloc(&R->d_best, 64)) != hipSuccess) return cleanup(hip_fail(c, e, "hipMalloc key"));
  if ((e = hipMemcpy(R->d_dist, R->dist.data(), (size_t)V * V * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(R->d_image, img.data(), (size_t)L.total_words * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(R->d_units, hu_id.data(), NHU * 2, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(R->d_units + NHU, su_id.data(), NSU * 2, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemset(R->d_st, 0, sizeof(SearchState))) != hipSuccess)
    return cleanup(hip_fail(c, e, "upload"));
  InstParams &P = R->P;
  P.NF = NF; P.NB = NB; P.NT = NT; P.NHU = NHU; P.NSU = NSU; P.V = V;
  P.flags = in->flags;
  P.cap_hu = in->cap_hu ? in->cap_hu : (uint32_t)(NHU + NT);
  P.cap_su = in->cap_su ? in->cap_su : (uint32_t)(NSU + NT);
  P.v_hu = in->hu_speed_mph;
  P.seg = (int32_t)next_pow2((uint32_t)NT);
  size_t dlds_max = 64 * 1024;
  if (const char *env = getenv("BL_D_LDS_MAX_BYTES")) dlds_max = (size_t)strtoull(env, nullptr, 10);
  P.d_in_lds = ((size_t)L.total_words + (size_t)V * V) * 4 <= dlds_max ? 1 : 0;
  P.lay = L;
  P.dist = R->d_dist;
  P.image = R->d_image;
  for (int k = 0; k < 3; ++k) {
    uint16_t *base = R->d_sol + SL.total * k;
    P.sol[k] = DevSol{base + SL.tour_off, base + SL.tour_bp, base + SL.bp_off,
                      base + SL.bp_field, base + SL.hu_tour, base + SL.su_tour};
  }
  P.st = R->d_st;
  P.trace = nullptr;
  P.trace_cap = 0;
  P.best_key = R->d_best;
  P.hu_id = R->d_units;
  P.su_id = R->d_units + NHU;
  if (eval_lds_bytes(P) > 160 * 1024) return cleanup(fail(c, BL_EINVAL, "instance image exceeds LDS"));
  R->occ_batch = eval_occupancy(P, false);
  R->occ_search = eval_occupancy(P, true);
  c->inst.push_back(std::move(I));
  *inst_id = (int32_t)c->inst.size() - 1;
  return BL_OK;
}

// Steps 1-3 of Algorithm 1 (sec. 2.5), on the host.
bl_status bl_init_solution(bl_ctx *c, int32_t id, bl_solution *out) {
  Instance *I = get_inst(c, id);
  if (!I) return fail(c, BL_EINVAL, "bad instance id %d", id);
  if (!out || !out->tour_off || !out->tour_bp || !out->bp_off || !out->bp_field || !out->hu_tour ||
      !out->su_tour)
    return fail(c, BL_EINVAL, "solution: null array");
  const int NF = I->NF, NB = I->NB, NT = I->NT, V = I->V;
  auto D = [&](int a, int b) { return I->dist[(size_t)a * V + b]; };
  // Step 1: nearest-neighbour chain over the BPs from HQ, ties to the lower id.
  std::vector<int> chain;
  std::vector<char> used(NB, 0);
  int cur = 0;
  for (int k = 0; k < NB; ++k) {
    int best = -1;
    for (int b = 0; b < NB; ++b)
      if (!used[b] && (best < 0 || D(cur, 1 + b) < D(cur, 1 + best))) best = b;
    used[best] = 1;
    chain.push_back(best);
    cur = 1 + best;
  }
  const int per = NB / NT;
  for (int g = 0; g <= NT; ++g) out->tour_off[g] = (uint16_t)(g < NT ? g * per : NB);
  for (int j = 0; j < NB; ++j) out->tour_bp[j] = (uint16_t)chain[j];
  // Step 2: fields in id order to the closest BP with unmet demand, then to
  // the closest BP.
  std::vector<uint64_t> got(NB, 0);
  std::vector<std::vector<int>> lists(NB);
  for (int f = 0; f < NF; ++f) {
    bool any_unmet = false;
    for (int b = 0; b < NB; ++b) any_unmet |= got[b] < I->demand[b];
    int best = -1;
    for (int b = 0; b < NB; ++b) {
      if (any_unmet && got[b] >= I->demand[b]) continue;
      if (best < 0 || D(1 + NB + f, 1 + b) < D(1 + NB + f, 1 + best)) best = b;
    }
    lists[best].push_back(f);
    got[best] += I->supply[f];
  }
  for (int b = 0; b < NB; ++b)
    if (got[b] < I->demand[b]) return fail(c, BL_EINFEASIBLE, "BP %d demand unmet by the greedy assignment", b);
  // Step 3: per BP, nearest-neighbour chain over its fields from HQ.
  int o = 0;
  for (int b = 0; b < NB; ++b) {
    out->bp_off[b] = (uint16_t)o;
    std::vector<int> left = lists[b];
    int at = 0;
    while (!left.empty()) {
      size_t bi = 0;
      for (size_t k = 1; k < left.size(); ++k) {
        const uint32_t dk = D(at, 1 + NB + left[k]), db = D(at, 1 + NB + left[bi]);
        if (dk < db || (dk == db && left[k] < left[bi])) bi = k;
      }
      const int f = left[bi];
      left.erase(left.begin() + bi);
      out->bp_field[o++] = (uint16_t)f;
      at = 1 + NB + f;
    }
  }
  out->bp_off[NB] = (uint16_t)o;
  // Units: contiguous id blocks.
  auto blocks = [&](int n, const std::vector<uint16_t> &counts, uint16_t *dst) {
    int u = 0;
    for (int g = 0; g < NT; ++g) {
      const int k = counts.empty() ? (g < NT - 1 ? n / NT : n - (n / NT) * (NT - 1)) : counts[g];
      for (int j = 0; j < k; ++j) dst[u++] = (uint16_t)g;
    }
  };
  blocks(I->NHU, I->init_hu, out->hu_tour);
  blocks(I->NSU, I->init_su, out->su_tour);
  return BL_OK;
}

bl_status bl_solution_upload(bl_ctx *c, int32_t id, int32_t slot, const bl_solution *s) {
  Instance *I = get_inst(c, id);
  if (!I) return fail(c, BL_EINVAL, "bad instance id %d", id);
  if (slot < 0 || slot > 2) return fail(c, BL_EINVAL, "bad slot %d", slot);
  bl_status st = validate_solution(c, *I, s);
  if (st != BL_OK) return st;
  const DevSol &d = I->P.sol[slot];
  hipStream_t q = c->stream;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(d.tour_off, s->tour_off, (I->NT + 1) * 2, hipMemcpyHostToDevice, q));
  HIP_TRY(c, hipMemcpyAsync(d.tour_bp, s->tour_bp, I->NB * 2, hipMemcpyHostToDevice, q));
  HIP_TRY(c, hipMemcpyAsync(d.bp_off, s->bp_off, (I->NB + 1) * 2, hipMemcpyHostToDevice, q));
  HIP_TRY(c, hipMemcpyAsync(d.bp_field, s->bp_field, I->NF * 2, hipMemcpyHostToDevice, q));
  HIP_TRY(c, hipMemcpyAsync(d.hu_tour, s->hu_tour, I->NHU * 2, hipMemcpyHostToDevice, q));
  HIP_TRY(c, hipMemcpyAsync(d.su_tour, s->su_tour, I->NSU * 2, hipMemcpyHostToDevice, q));
  if (slot == BL_SLOT_BASE) {
    HIP_TRY(c, launch_prepare(I->P, kPrepFromBase, 0, 0, 0, q));
    I->base_ready = true;
  }
  // The host arrays may be released by the caller after return.
  HIP_TRY(c, hipStreamSynchronize(q));
  return BL_OK;
}

bl_status bl_solution_download(bl_ctx *c, int32_t id, int32_t slot, bl_solution *s) {
  Instance *I = get_inst(c, id);
  if (!I) return fail(c, BL_EINVAL, "bad instance id %d", id);
  if (slot < 0 || slot > 2) return fail(c, BL_EINVAL, "bad slot %d", slot);
  if (!s || !s->tour_off || !s->tour_bp || !s->bp_off || !s->bp_field || !s->hu_tour || !s->su_tour)
    return fail(c, BL_EINVAL, "solution: null array");
  const DevSol &d = I->P.sol[slot];
  hipStream_t q = c->stream;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(s->tour_off, d.tour_off, (I->NT + 1) * 2, hipMemcpyDeviceToHost, q));
  HIP_TRY(c, hipMemcpyAsync(s->tour_bp, d.tour_bp, I->NB * 2, hipMemcpyDeviceToHost, q));
  HIP_TRY(c, hipMemcpyAsync(s->bp_off, d.bp_off, (I->NB + 1) * 2, hipMemcpyDeviceToHost, q));
  HIP_TRY(c, hipMemcpyAsync(s->bp_field, d.bp_field, I->NF * 2, hipMemcpyDeviceToHost, q));
  HIP_TRY(c, hipMemcpyAsync(s->hu_tour, d.hu_tour, I->NHU * 2, hipMemcpyDeviceToHost, q));
  HIP_TRY(c, hipMemcpyAsync(s->su_tour, d.su_tour, I->NSU * 2, hipMemcpyDeviceToHost, q));
  HIP_TRY(c, hipStreamSynchronize(q));
  return BL_OK;
}

bl_status bl_generate(bl_ctx *c, int32_t id, uint64_t seed, uint32_t iter, uint32_t inst_index,
                      uint32_t first, uint32_t n, uint64_t *d_moves) {
  Instance *I = get_inst(c, id);
  if (!I) return fail(c, BL_EINVAL, "bad instance id %d", id);
  if (!I->base_ready) return fail(c, BL_ESTATE, "no base solution uploaded");
  if (n && !d_moves) return fail(c, BL_EINVAL, "null move buffer");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, launch_generate(I->P, seed, iter, inst_index, first, n, d_moves, c->stream));
  return BL_OK;
}

bl_status bl_evaluate_batch(bl_ctx *c, int32_t id, const uint64_t *d_moves, uint32_t n,
                            int64_t t_star_s, uint64_t *d_key, float *d_cost_km,
                            int32_t *d_makespan_s, uint8_t *d_flags) {
  Instance *I = get_inst(c, id);
  if (!I) return fail(c, BL_EINVAL, "bad instance id %d", id);
  if (!I->base_ready) return fail(c, BL_ESTATE, "no base solution uploaded");
  if (n > kMaxCand) return fail(c, BL_EINVAL, "n %u > 2^24", n);
  if (n && (!d_moves || !d_key)) return fail(c, BL_EINVAL, "null move or key buffer");
  HIP_TRY(c, hipSetDevice(c->device));
  if (n == 0) return BL_OK;
  HIP_TRY(c, timing_mark(c));
  HIP_TRY(c, launch_eval_batch(I->P, d_moves, n, t_star_s, d_key, d_cost_km, d_makespan_s, d_flags,
                               grid_for(c, *I, n, false), c->stream));
  HIP_TRY(c, timing_mark(c));
  return BL_OK;
}

bl_status bl_select_best(bl_ctx *c, const uint64_t *d_key, uint32_t n, uint64_t *d_best) {
  if (!c) return BL_EINVAL;
  if (!d_best || (n && !d_key)) return fail(c, BL_EINVAL, "null buffer");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, launch_select(d_key, n, d_best, c->stream));
  return BL_OK;
}

bl_status bl_search_start(bl_ctx *c, int32_t id, uint32_t trace_capacity) {
  Instance *I = get_inst(c, id);
  if (!I) return fail(c, BL_EINVAL, "bad instance id %d", id);
  if (!I->base_ready) return fail(c, BL_ESTATE, "no base solution uploaded");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (trace_capacity != I->P.trace_cap) {
    (void)hipFree(I->d_trace);
    I->d_trace = nullptr;
    I->P.trace_cap = 0;
    I->P.trace = nullptr;
    if (trace_capacity) {
      HIP_TRY(c, hipMalloc(&I->d_trace, (size_t)trace_capacity * sizeof(TraceRow)));
      I->P.trace = I->d_trace;
      I->P.trace_cap = trace_capacity;
    }
  }
  HIP_TRY(c, launch_commit(I->P, kCommitStart, 0, 0, c->stream));
  I->started = true;
  return BL_OK;
}

bl_status bl_search_step(bl_ctx *c, int32_t id, const bl_search_params *p) {
  Instance *I = get_inst(c, id);
  if (!I) return fail(c, BL_EINVAL, "bad instance id %d", id);
  if (!p) return fail(c, BL_EINVAL, "null params");
  if (!I->started) return fail(c, BL_ESTATE, "bl_search_start not called");
  if (p->n == 0 || p->n > kMaxCand) return fail(c, BL_EINVAL, "n %u out of 1..2^24", p->n);
  if (p->eps_threshold > (1ull << 32)) return fail(c, BL_EINVAL, "eps_threshold > 2^32");
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t q = c->stream;
  HIP_TRY(c, launch_prepare(I->P, kPrepSearch, p->seed, p->eps_threshold, p->inst_index, q));
  HIP_TRY(c, timing_mark(c));
  HIP_TRY(c, launch_eval_search(I->P, p->seed, p->n, p->inst_index, grid_for(c, *I, p->n, true), q));
  HIP_TRY(c, timing_mark(c));
  HIP_TRY(c, launch_commit(I->P, kCommitStep, p->seed, p->inst_index, q));
  return BL_OK;
}

bl_status bl_search_state_get(bl_ctx *c, int32_t id, bl_search_state *out) {
  Instance *I = get_inst(c, id);
  if (!I) return fail(c, BL_EINVAL, "bad instance id %d", id);
  if (!out) return fail(c, BL_EINVAL, "null output");
  SearchState st;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(&st, I->d_st, sizeof st, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  out->it = st.it;
  out->n_improved = st.n_improved;
  out->cost_best_m = st.cost_best;
  out->t_best_s = st.t_best;
  return BL_OK;
}

bl_status bl_search_trace(bl_ctx *c, int32_t id, bl_trace_row *out, uint32_t max_rows,
                          uint32_t *n_rows) {
  Instance *I = get_inst(c, id);
  if (!I) return fail(c, BL_EINVAL, "bad instance id %d", id);
  if (!n_rows || (max_rows && !out)) return fail(c, BL_EINVAL, "null output");
  static_assert(sizeof(bl_trace_row) == sizeof(TraceRow), "trace row layout");
  SearchState st;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(&st, I->d_st, sizeof st, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  uint32_t rows = std::min(st.trace_rows, I->P.trace_cap);
  rows = std::min(rows, max_rows);
  if (rows) {
    HIP_TRY(c, hipMemcpyAsync(out, I->d_trace, rows * sizeof(TraceRow), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  *n_rows = rows;
  return BL_OK;
}

bl_status bl_timing_enable(bl_ctx *c, int32_t on) {
  if (!c) return BL_EINVAL;
  c->timing = on != 0;
  return BL_OK;
}

bl_status bl_timing_read(bl_ctx *c, double *eval_ms, uint32_t *n_launches) {
  if (!c || !eval_ms || !n_launches) return fail(c, BL_EINVAL, "null output");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  double total = 0.0;
  for (size_t k = 0; k + 1 < c->events_used; k += 2) {
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->events[k], c->events[k + 1]));
    total += ms;
  }
  *eval_ms = total;
  *n_launches = (uint32_t)(c->events_used / 2);
  c->events_used = 0;
  return BL_OK;
}

}  // extern "C"
