// Host side of the C interface: contexts, instance validation and upload,
// the initial solution of Algorithm 1, solution slots, and the
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
#include <mutex>
#include <vector>

#include "../../include/bl.h"
#include "bl_internal.h"
#include "sur_internal.h"

namespace bl {
int eval_occupancy(const InstParams &P, bool search);
}

using namespace bl;

namespace {

struct Instance {
  // host copies
  int NF = 0, NB = 0, NT = 0, NHU = 0, NSU = 0, V = 0;
  std::vector<uint32_t> dist, area, yld, demand, hu_rate, su_cap, su_speed, su_fill;
  std::vector<int32_t> xy;  // 2 * V coordinates, empty when not given
  std::vector<uint16_t> init_hu, init_su;
  std::vector<uint64_t> supply;
  uint32_t v_hu = 0, flags = 0;
  // device
  InstParams P{};
  uint32_t *d_dist = nullptr, *d_image = nullptr;
  uint16_t *d_sol = nullptr, *d_units = nullptr;
  SearchState *d_st = nullptr;
  TraceRow *d_trace = nullptr;
  uint64_t *d_best = nullptr;   // argmin slot (8 B), then the deferred-candidate counts (2 x 4 B)
  uint32_t *d_defer = nullptr;  // deferred-candidate list of the one-candidate-per-lane launches (2 classes)
  WinRec *d_rec = nullptr;      // the winner's units formed during their second pass
  bool base_ready = false, started = false;
  int occ_batch = 1, occ_search = 1;
};

// Learned screen of one instance.
struct Sur {
  int32_t inst = -1;
  bl_sur_config cfg{};
  SurDev D{};
  std::vector<void *> allocs;
  uint32_t step = 0;
  ScreenDev T{};                 // screening buffers, allocated on first use
  std::vector<void *> t_allocs;
  uint32_t t_nprop = 0, t_k = 0;
};

struct Batch {
  std::vector<int32_t> members;
  uint32_t n = 0;
  bl_batch_schedule sched{{1024, 1024, 1024}, 1, 1};
  InstParams *d_inst = nullptr;  // [K]
  uint32_t *d_sched = nullptr;   // item_off[K+1] | order[K] | tile[K] | queue[1]
  uint32_t total_items = 0;
  uint32_t max_image_words = 0;
  size_t lds = 0;
  int occ[2] = {1, 1};   // workgroups per CU without and with the feasibility queue
  bool walk = false;  // some member asks for the full walk
  int lane_n = 0;     // > 0: one candidate per lane, this many tour slots
  bool lane_small = false;
  bool started = false;
};

}  // namespace

struct bl_ctx {
  int device = 0;
  int n_cu = 256;
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<std::unique_ptr<Instance>> inst;
  std::vector<std::unique_ptr<Batch>> batches;
  std::vector<std::unique_ptr<Sur>> surs;
  std::vector<hipGraphExec_t> graphs;
  hipStream_t capture_stream = nullptr;  // private stream used only while capturing
  bool capturing = false;
  // kernel timing: event pairs recorded around launches of one kind
  int timing = 0;
  std::vector<hipEvent_t> events;
  size_t events_used = 0;
  uint32_t *scratch = nullptr;   // device address of the static array (bl_evaluate_batch_static)
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
  uint32_t u128(uint32_t n) {
    words = (words + 3) & ~3u;
    return u32(4 * n);
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
  (void)hipFree(I->d_defer);
  (void)hipFree(I->d_rec);
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

// Records one timing event when launches of this kind are being timed.
enum { kTimeEval = BL_TIMING_EVAL, kTimeScreen = BL_TIMING_SCREEN };
hipError_t timing_mark(bl_ctx *c, int kind = kTimeEval) {
  if (c->timing != kind || c->capturing) return hipSuccess;
  if (c->events_used == c->events.size()) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    c->events.push_back(e);
  }
  return hipEventRecord(c->events[c->events_used++], c->stream);
}

hipStream_t work_stream(const bl_ctx *c) { return c->capturing ? c->capture_stream : c->stream; }

bl_status alloc_trace(bl_ctx *c, Instance *I, uint32_t cap) {
  if (cap == I->P.trace_cap) return BL_OK;
  (void)hipFree(I->d_trace);
  I->d_trace = nullptr;
  I->P.trace_cap = 0;
  I->P.trace = nullptr;
  if (cap) {
    HIP_TRY(c, hipMalloc(&I->d_trace, (size_t)cap * sizeof(TraceRow)));
    I->P.trace = I->d_trace;
    I->P.trace_cap = cap;
  }
  return BL_OK;
}

int grid_for(const bl_ctx *c, const Instance &I, uint32_t n, bool search) {
  // Candidates one workgroup of 256 lanes takes at a time.
  const uint32_t per_block = lane_eval_on(I.P) ? 256u : 4u * (64u / (uint32_t)I.P.seg);
  const uint32_t need = (n + per_block - 1) / per_block;
  const uint32_t cap = (uint32_t)c->n_cu * (uint32_t)(search ? I.occ_search : I.occ_batch);
  return (int)std::max<uint32_t>(1u, std::min(need, cap));
}

bl_status search_step_on(bl_ctx *c, Instance *I, const bl_search_params *p, hipStream_t q) {
  HIP_TRY(c, launch_prepare(I->P, kPrepSearch, p->seed, p->eps_threshold, p->inst_index, q));
  HIP_TRY(c, timing_mark(c));
  HIP_TRY(c, launch_eval_search(I->P, p->seed, p->n, p->inst_index, grid_for(c, *I, p->n, true), q, nullptr,
                                true));
  HIP_TRY(c, timing_mark(c));
  HIP_TRY(c, launch_commit(I->P, kCommitStep, p->seed, p->inst_index, q));
  return BL_OK;
}

// ---------------------------------------------------------------- batches

Batch *get_batch(bl_ctx *c, int32_t id) {
  if (!c || id < 0 || id >= (int32_t)c->batches.size()) return nullptr;
  return c->batches[id].get();
}

int size_class(int nf) { return nf < 100 ? 0 : (nf < 200 ? 1 : 2); }

bl_status upload_member_params(bl_ctx *c, Batch &B) {
  std::vector<InstParams> ps;
  for (int32_t id : B.members) ps.push_back(c->inst[id]->P);
  HIP_TRY(c, hipMemcpy(B.d_inst, ps.data(), ps.size() * sizeof(InstParams), hipMemcpyHostToDevice));
  return BL_OK;
}

bl_status apply_schedule(bl_ctx *c, Batch &B, const bl_batch_schedule &s) {
  for (int k = 0; k < 3; ++k) {
    const uint32_t t = s.tile[k];
    if (t < 64 || t > 65536 || (t & (t - 1)))
      return fail(c, BL_EINVAL, "tile[%d] = %u must be a power of two in 64..65536", k, t);
  }
  if (s.order_policy > 1) return fail(c, BL_EINVAL, "order_policy must be 0 or 1");
  if (s.feas_queue > 1) return fail(c, BL_EINVAL, "feas_queue must be 0 or 1");
  const uint32_t K = (uint32_t)B.members.size();
  std::vector<uint32_t> order(K);
  std::iota(order.begin(), order.end(), 0u);
  if (s.order_policy == 1)
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
      return c->inst[B.members[a]]->NF > c->inst[B.members[b]]->NF;
    });
  std::vector<uint32_t> tile(K), off(K + 1, 0);
  for (uint32_t k = 0; k < K; ++k) tile[k] = s.tile[size_class(c->inst[B.members[k]]->NF)];
  for (uint32_t p = 0; p < K; ++p) off[p + 1] = off[p] + (B.n + tile[order[p]] - 1) / tile[order[p]];
  std::vector<uint32_t> buf;
  buf.insert(buf.end(), off.begin(), off.end());
  buf.insert(buf.end(), order.begin(), order.end());
  buf.insert(buf.end(), tile.begin(), tile.end());
  buf.push_back(0u);
  HIP_TRY(c, hipMemcpy(B.d_sched, buf.data(), buf.size() * 4, hipMemcpyHostToDevice));
  B.total_items = off[K];
  B.sched = s;
  return BL_OK;
}

BatchParams batch_params(const Batch &B, const bl_search_params *p) {
  const uint32_t K = (uint32_t)B.members.size();
  BatchParams bp;
  bp.inst = B.d_inst;
  bp.K = K;
  bp.n = B.n;
  bp.seed = p ? p->seed : 0;
  bp.eps_thr = p ? p->eps_threshold : 0;
  bp.index_base = p ? p->inst_index : 0;
  bp.total_items = B.total_items;
  bp.item_off = B.d_sched;
  bp.order = B.d_sched + K + 1;
  bp.tile = B.d_sched + 2 * K + 1;
  bp.queue = B.d_sched + 3 * K + 1;
  bp.walk = B.walk ? 1u : 0u;
  bp.lane_n = (uint32_t)B.lane_n;
  bp.lane_small = B.lane_small ? 1u : 0u;
  bp.feas_queue = B.sched.feas_queue;
  return bp;
}

int batch_grid(const bl_ctx *c, const Batch &B) {
  const int occ = B.occ[B.sched.feas_queue ? 1 : 0];
  return (int)std::max<uint32_t>(1u, std::min<uint32_t>(B.total_items, (uint32_t)(c->n_cu * occ)));
}

bl_status batch_step_on(bl_ctx *c, Batch &B, const bl_search_params *p, hipStream_t q) {
  const BatchParams bp = batch_params(B, p);
  HIP_TRY(c, launch_batch_prepare(bp, B.lds, q));
  HIP_TRY(c, timing_mark(c));
  HIP_TRY(c, launch_batch_eval(bp, batch_grid(c, B), B.lds, q));
  HIP_TRY(c, timing_mark(c));
  HIP_TRY(c, launch_batch_commit(bp, B.lds, q));
  return BL_OK;
}

// FNV-1a over the member sizes and the candidate count.
std::string batch_signature(const bl_ctx *c, const Batch &B) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 0xFF;
      h *= 1099511628211ull;
    }
  };
  mix(B.members.size());
  mix(B.n);
  for (int32_t id : B.members) {
    const Instance &I = *c->inst[id];
    mix(I.NF);
    mix(I.NB);
    mix(I.NT);
    mix(I.NHU);
    mix(I.NSU);
  }
  mix((uint64_t)B.lane_n);   // the kernel the schedule was timed with
  char buf[32];
  snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
  return buf;
}

bool read_file(const char *path, std::string &out) {
  FILE *f = fopen(path, "rb");
  if (!f) return false;
  char buf[4096];
  size_t k;
  while ((k = fread(buf, 1, sizeof buf, f)) > 0) out.append(buf, k);
  fclose(f);
  return true;
}

bool cache_lookup(const std::string &text, const std::string &sig, bl_batch_schedule &s) {
  const size_t at = text.find("\"" + sig + "\"");
  if (at == std::string::npos) return false;
  unsigned a, b, d, pol, fq;
  if (sscanf(text.c_str() + at + sig.size() + 2,
             " : {\"tile\": [%u, %u, %u], \"order_policy\": %u, \"feas_queue\": %u", &a, &b, &d, &pol, &fq) != 5)
    return false;
  s.tile[0] = a;
  s.tile[1] = b;
  s.tile[2] = d;
  s.order_policy = pol;
  s.feas_queue = fq;
  return true;
}

bool cache_store(const char *path, std::string text, const std::string &sig,
                 const bl_batch_schedule &s, double ms) {
  char entry[256];
  snprintf(entry, sizeof entry,
           "  \"%s\": {\"tile\": [%u, %u, %u], \"order_policy\": %u, \"feas_queue\": %u, \"eval_ms\": %.4f}",
           sig.c_str(), s.tile[0], s.tile[1], s.tile[2], s.order_policy, s.feas_queue, ms);
  const size_t close = text.rfind('}');
  if (text.find('"') == std::string::npos || close == std::string::npos)
    text = std::string("{\n") + entry + "\n}\n";
  else
    text = text.substr(0, text.find_last_not_of(" \n\t", close - 1) + 1) + ",\n" + entry + "\n}\n";
  FILE *f = fopen(path, "wb");
  if (!f) return false;
  const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
  return fclose(f) == 0 && ok;
}

// ----------------------------------------------------------------- graphs

template <class Body>
bl_status capture_steps(bl_ctx *c, uint32_t n_steps, Body body, int32_t *graph) {
  if (!graph || n_steps == 0) return fail(c, BL_EINVAL, "bad graph arguments");
  if (!c->capture_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeRelaxed));
  c->capturing = true;
  bl_status st = BL_OK;
  for (uint32_t s = 0; s < n_steps && st == BL_OK; ++s) st = body(c->capture_stream);
  c->capturing = false;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->capture_stream, &g);
  if (st != BL_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) return hip_fail(c, e2, "hipGraphInstantiate");
  c->graphs.push_back(ex);
  *graph = (int32_t)c->graphs.size() - 1;
  return BL_OK;
}

// Device addresses of the static array behind bl_evaluate_batch_static,
// looked up once per device (each GPU holds its own copy of the array).
std::mutex g_scratch_mu;
std::vector<uint32_t *> g_scratch;

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
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch.size() < (size_t)n) g_scratch.resize((size_t)n, nullptr);
    if (!g_scratch[device]) {
      uint32_t *p = nullptr;
      // On failure the entry point that needs the array reports it.
      if (static_scratch_address(&p) == hipSuccess) g_scratch[device] = p;
      else (void)hipGetLastError();
    }
    c->scratch = g_scratch[device];
  }
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
  for (auto g : ctx->graphs) (void)hipGraphExecDestroy(g);
  for (auto &B : ctx->batches) {
    (void)hipFree(B->d_inst);
    (void)hipFree(B->d_sched);
  }
  for (auto &S : ctx->surs) {
    for (void *p : S->allocs) (void)hipFree(p);
    for (void *p : S->t_allocs) (void)hipFree(p);
  }
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
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
  if (in->flags & ~127u) return fail(c, BL_EINVAL, "unknown flags 0x%x", in->flags);
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
  if (in->xy_m) I->xy.assign(in->xy_m, in->xy_m + 2 * (size_t)V);
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
  for (int f = 0; f < NF; ++f) {
    uint32_t dfmax = 0;
    for (int b = 0; b < NB; ++b) dfmax = std::max(dfmax, I->dist[(size_t)(1 + NB + f) * V + 1 + b]);
    if (2ull * nsh[f] * dfmax >= (1ull << 32))
      return fail(c, BL_EINVAL, "shuttle distance of field %d >= 2^32 m", f);
  }
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
  L.prec = al.u128(NF); L.w_q = al.u32(NF);
  L.bp_start = al.u16(NB); L.bp_len = al.u16(NB); L.bp_tour = al.u16(NB); L.bp_idx = al.u16(NB);
  L.tour_off = al.u16(NT + 1); L.tour_bp = al.u16(NB);
  L.hu_mask = al.u64(NT); L.su_mask = al.u64(2 * NT);
  L.t_len = al.u32(NT); L.t_area = al.u32(NT); L.t_sh = al.u64(NT); L.t_msum = al.u32(NT);
  L.t_mcnt = al.u32(NT); L.t_start = al.u16(NT); L.t_end = al.u16(NT);
  L.b_sd = al.u32(NB); L.b_sup = al.u32(NB); L.b_area = al.u32(NB); L.b_sh = al.u64(NB);
  L.b_int = al.u32(NB); L.b_mean = al.u32(NB); L.b_skip = al.u32(NB); L.skip = al.u32(NF);
  L.n_viol = al.u32(1);
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
  // Staging the whole matrix pays only while it is small: a large LDS
  // footprint costs more occupancy than the band-plus-L2 lookups it saves.
  size_t dlds_max = 16 * 1024;
  if (const char *env = getenv("BL_D_LDS_MAX_BYTES")) dlds_max = (size_t)strtoull(env, nullptr, 10);
  P.d_in_lds = ((size_t)L.total_words + (size_t)V * V) * 4 <= dlds_max ? 1 : 0;
  {
    // Bounds of every completion time (route bound over the HU speed plus the
    // whole area at the slowest rate) and waiting time (longest round trip at
    // the slowest SU, or every fill time): when both fit 26 bits and the
    // segment has at most 16 lanes, the rebalancing keys are 32-bit.
    uint32_t rmin = ~0u, vmin = ~0u;
    uint64_t fills = 0;
    for (uint32_t r : I->hu_rate) rmin = std::min(rmin, r);
    for (uint32_t v : I->su_speed) vmin = std::min(vmin, v);
    for (uint32_t f : I->su_fill) fills += f;
    const double tb = 3600.0 * (double)lmax / (double)in->hu_speed_mph + 3600.0 * (double)tot_area / (double)rmin;
    const double wb = std::max(7200.0 * (double)dmax / (double)vmin, (double)fills);
    const double lim = (double)((1ll << 26) - 4);
    P.narrow = (tb < lim && wb < lim && P.seg <= 16 && !(in->flags & kWideKeys)) ? 1 : 0;
  }
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
  P.defer = nullptr;
  P.defer_zeroed = 0;
  P.defer_cnt = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(R->d_best) + 8);
  P.defer_cap = 0;
  if (lane_eval_on(P)) {
    if ((e = hipMalloc(&R->d_defer, (size_t)kDeferCap * 8)) != hipSuccess)
      return cleanup(hip_fail(c, e, "hipMalloc deferred list"));
    P.defer = R->d_defer;
    P.defer_cap = kDeferCap;
  }
  R->occ_batch = eval_occupancy(P, false);
  R->occ_search = eval_occupancy(P, true);
  P.lane_tail = lane_tail_on(P) ? 1 : 0;
  P.rec = nullptr;
  if (P.lane_tail) {
    if ((e = hipMalloc(&R->d_rec, sizeof(WinRec))) != hipSuccess ||
        (e = hipMemset(R->d_rec, 0, sizeof(WinRec))) != hipSuccess)
      return cleanup(hip_fail(c, e, "hipMalloc winner record"));
    P.rec = R->d_rec;
  }
  c->inst.push_back(std::move(I));
  *inst_id = (int32_t)c->inst.size() - 1;
  return BL_OK;
}

// The initial solution of Algorithm 1 (sec. 2.5), on the host.
bl_status bl_init_solution(bl_ctx *c, int32_t id, bl_solution *out) {
  Instance *I = get_inst(c, id);
  if (!I) return fail(c, BL_EINVAL, "bad instance id %d", id);
  if (!out || !out->tour_off || !out->tour_bp || !out->bp_off || !out->bp_field || !out->hu_tour ||
      !out->su_tour)
    return fail(c, BL_EINVAL, "solution: null array");
  const int NF = I->NF, NB = I->NB, NT = I->NT, V = I->V;
  auto D = [&](int a, int b) { return I->dist[(size_t)a * V + b]; };
  // BPs to tours: nearest-neighbour chain over the BPs from HQ, ties to the lower id.
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
  // Fields to BPs: in id order to the closest BP with unmet demand, then to
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
  // Field order: per BP, nearest-neighbour chain over its fields from HQ.
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

bl_status bl_evaluate_batch_static(bl_ctx *c, int32_t id, const uint64_t *d_moves, uint32_t n,
                                   int64_t t_star_s, uint64_t *d_key, float *d_cost_km,
                                   int32_t *d_makespan_s, uint8_t *d_flags) {
  Instance *I = get_inst(c, id);
  if (!I) return fail(c, BL_EINVAL, "bad instance id %d", id);
  if (!I->base_ready) return fail(c, BL_ESTATE, "no base solution uploaded");
  if (n > kMaxCand) return fail(c, BL_EINVAL, "n %u > 2^24", n);
  if (n && (!d_moves || !d_key)) return fail(c, BL_EINVAL, "null move or key buffer");
  if (!c->scratch) return fail(c, BL_EDEVICE, "static scratch array unavailable on device %d", c->device);
  HIP_TRY(c, hipSetDevice(c->device));
  if (n == 0) return BL_OK;
  // The same launch, its deferred list and counts in the static array (the
  // counts are cleared by a kernel at the start of the launch).  No timing
  // events: their first use would create events.
  InstParams Q = I->P;
  if (Q.defer_cap) {
    Q.defer = c->scratch;
    Q.defer_cnt = c->scratch + 2 * kStaticDeferCap;
    Q.defer_cap = kStaticDeferCap;
  }
  HIP_TRY(c, launch_eval_batch(Q, d_moves, n, t_star_s, d_key, d_cost_km, d_makespan_s, d_flags,
                               grid_for(c, *I, n, false), c->stream));
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
  bl_status st = alloc_trace(c, I, trace_capacity);
  if (st != BL_OK) return st;
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
  return search_step_on(c, I, p, work_stream(c));
}

bl_status bl_instance_info_get(bl_ctx *c, int32_t id, bl_instance_info *out) {
  Instance *I = get_inst(c, id);
  if (!I) return fail(c, BL_EINVAL, "bad instance id %d", id);
  if (!out) return fail(c, BL_EINVAL, "null output");
  out->lane_eval = lane_eval_on(I->P) ? 1 : 0;
  out->tail_table = I->P.lane_tail ? 1 : 0;
  out->wg_per_cu = I->occ_search;
  out->image_bytes = I->P.lay.total_words * 4u;
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

bl_status bl_batch_create(bl_ctx *c, const int32_t *ids, int32_t n_inst, uint32_t n_cand,
                          int32_t *batch) {
  if (!c) return BL_EINVAL;
  if (!ids || !batch || n_inst < 1) return fail(c, BL_EINVAL, "bad batch arguments");
  if (n_cand == 0 || n_cand > kMaxCand) return fail(c, BL_EINVAL, "n_cand %u out of 1..2^24", n_cand);
  auto B = std::make_unique<Batch>();
  for (int32_t k = 0; k < n_inst; ++k) {
    Instance *I = get_inst(c, ids[k]);
    if (!I) return fail(c, BL_EINVAL, "bad instance id %d", ids[k]);
    if (!I->base_ready) return fail(c, BL_ESTATE, "member %d has no base solution", ids[k]);
    for (int32_t j = 0; j < k; ++j)
      if (ids[j] == ids[k]) return fail(c, BL_EINVAL, "instance %d listed twice", ids[k]);
    B->members.push_back(ids[k]);
    B->max_image_words = std::max(B->max_image_words, I->P.lay.total_words);
    if (I->P.flags & kFullWalk) B->walk = true;
  }
  // One candidate per lane when every member allows it (lane_eval_on), with
  // tour slots for the largest member; else one segment per candidate.
  bool lane = true, small = true;
  int max_nt = 0;
  for (int32_t id : B->members) {
    const InstParams &P = c->inst[id]->P;
    lane = lane && lane_eval_on(P);
    small = small && P.NHU <= 32 && P.NSU <= 64;
    max_nt = std::max(max_nt, (int)P.NT);
  }
  B->lane_n = lane ? batch_lane_tours(max_nt) : 0;
  B->lane_small = small;
  B->n = n_cand;
  B->lds = batch_lds_bytes(B->max_image_words);
  if (B->lds > 160 * 1024) return fail(c, BL_EINVAL, "member image exceeds LDS");
  HIP_TRY(c, hipSetDevice(c->device));
  for (int q = 0; q < 2; ++q) B->occ[q] = batch_occupancy(B->lds, B->walk, B->lane_n, B->lane_small, q == 1);
  const size_t K = B->members.size();
  HIP_TRY(c, hipMalloc(&B->d_inst, K * sizeof(InstParams)));
  if (hipMalloc(&B->d_sched, (3 * K + 2) * sizeof(uint32_t)) != hipSuccess) {
    (void)hipFree(B->d_inst);
    return fail(c, BL_ENOMEM, "batch schedule allocation");
  }
  Batch *R = B.get();
  c->batches.push_back(std::move(B));
  bl_status st = upload_member_params(c, *R);
  if (st == BL_OK) st = apply_schedule(c, *R, R->sched);
  if (st != BL_OK) return st;
  *batch = (int32_t)c->batches.size() - 1;
  return BL_OK;
}

bl_status bl_batch_start(bl_ctx *c, int32_t id, uint32_t trace_capacity) {
  Batch *B = get_batch(c, id);
  if (!B) return fail(c, BL_EINVAL, "bad batch id %d", id);
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int32_t m : B->members) {
    bl_status st = alloc_trace(c, c->inst[m].get(), trace_capacity);
    if (st != BL_OK) return st;
  }
  bl_status st = upload_member_params(c, *B);
  if (st != BL_OK) return st;
  HIP_TRY(c, launch_batch_start(batch_params(*B, nullptr), B->lds, c->stream));
  for (int32_t m : B->members) c->inst[m]->started = true;
  B->started = true;
  return BL_OK;
}

bl_status bl_batch_step(bl_ctx *c, int32_t id, const bl_search_params *p) {
  Batch *B = get_batch(c, id);
  if (!B) return fail(c, BL_EINVAL, "bad batch id %d", id);
  if (!p) return fail(c, BL_EINVAL, "null params");
  if (!B->started) return fail(c, BL_ESTATE, "bl_batch_start not called");
  if (p->eps_threshold > (1ull << 32)) return fail(c, BL_EINVAL, "eps_threshold > 2^32");
  HIP_TRY(c, hipSetDevice(c->device));
  return batch_step_on(c, *B, p, work_stream(c));
}

bl_status bl_batch_set_schedule(bl_ctx *c, int32_t id, const bl_batch_schedule *s) {
  Batch *B = get_batch(c, id);
  if (!B) return fail(c, BL_EINVAL, "bad batch id %d", id);
  if (!s) return fail(c, BL_EINVAL, "null schedule");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return apply_schedule(c, *B, *s);
}

bl_status bl_batch_autotune(bl_ctx *c, int32_t id, const bl_search_params *p, const char *cache_path,
                            bl_batch_schedule *out) {
  Batch *B = get_batch(c, id);
  if (!B) return fail(c, BL_EINVAL, "bad batch id %d", id);
  if (!p) return fail(c, BL_EINVAL, "null params");
  if (!B->started) return fail(c, BL_ESTATE, "bl_batch_start not called");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const std::string sig = batch_signature(c, *B);
  std::string text;
  const bool have_file = cache_path && read_file(cache_path, text);
  bl_batch_schedule best{};
  if (have_file && cache_lookup(text, sig, best)) {
    bl_status st = apply_schedule(c, *B, best);
    if (st != BL_OK) return st;
    if (out) *out = best;
    return BL_OK;
  }
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  // Median of three timed evaluation launches (the bases stay as they are;
  // only the per-member argmin slots are touched, and the next prepare resets
  // them).
  auto time_sched = [&](const bl_batch_schedule &s, double &ms) -> bl_status {
    bl_status st = apply_schedule(c, *B, s);
    if (st != BL_OK) return st;
    const BatchParams bp = batch_params(*B, p);
    double t[3];
    for (int r = 0; r < 3; ++r) {
      HIP_TRY(c, hipEventRecord(e0, c->stream));
      HIP_TRY(c, launch_batch_eval(bp, batch_grid(c, *B), B->lds, c->stream));
      HIP_TRY(c, hipEventRecord(e1, c->stream));
      HIP_TRY(c, hipEventSynchronize(e1));
      float f = 0.f;
      HIP_TRY(c, hipEventElapsedTime(&f, e0, e1));
      t[r] = f;
    }
    std::sort(t, t + 3);
    ms = t[1];
    return BL_OK;
  };
  bool present[3] = {false, false, false};
  for (int32_t m : B->members) present[size_class(c->inst[m]->NF)] = true;
  const uint32_t tiles[] = {256, 512, 1024, 2048, 4096};
  best = bl_batch_schedule{{1024, 1024, 1024}, 1, 1};
  double best_ms = 0;
  bl_status st = time_sched(best, best_ms);
  // Coordinate descent: one size class at a time, then the member order,
  // then the feasibility queue.
  for (int k = 0; k < 3 && st == BL_OK; ++k) {
    if (!present[k]) continue;
    for (uint32_t t : tiles) {
      bl_batch_schedule s = best;
      s.tile[k] = t;
      double ms = 0;
      if ((st = time_sched(s, ms)) != BL_OK) break;
      if (ms < best_ms) best_ms = ms, best = s;
    }
  }
  if (st == BL_OK) {
    bl_batch_schedule s = best;
    s.order_policy = 1 - s.order_policy;
    double ms = 0;
    st = time_sched(s, ms);
    if (st == BL_OK && ms < best_ms) best_ms = ms, best = s;
  }
  if (st == BL_OK && B->lane_n > 0) {
    bl_batch_schedule s = best;
    s.feas_queue = 1 - s.feas_queue;
    double ms = 0;
    st = time_sched(s, ms);
    if (st == BL_OK && ms < best_ms) best_ms = ms, best = s;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != BL_OK) return st;
  st = apply_schedule(c, *B, best);
  if (st != BL_OK) return st;
  if (cache_path && !cache_store(cache_path, have_file ? text : std::string(), sig, best, best_ms))
    return fail(c, BL_EINVAL, "cannot write cache %s", cache_path);
  if (out) *out = best;
  return BL_OK;
}

bl_status bl_search_capture(bl_ctx *c, int32_t id, const bl_search_params *p, uint32_t n_steps,
                            int32_t *graph) {
  Instance *I = get_inst(c, id);
  if (!I) return fail(c, BL_EINVAL, "bad instance id %d", id);
  if (!p) return fail(c, BL_EINVAL, "null params");
  if (!I->started) return fail(c, BL_ESTATE, "bl_search_start not called");
  if (p->n == 0 || p->n > kMaxCand) return fail(c, BL_EINVAL, "n %u out of 1..2^24", p->n);
  if (p->eps_threshold > (1ull << 32)) return fail(c, BL_EINVAL, "eps_threshold > 2^32");
  HIP_TRY(c, hipSetDevice(c->device));
  return capture_steps(c, n_steps, [&](hipStream_t q) { return search_step_on(c, I, p, q); }, graph);
}

bl_status bl_batch_capture(bl_ctx *c, int32_t id, const bl_search_params *p, uint32_t n_steps,
                           int32_t *graph) {
  Batch *B = get_batch(c, id);
  if (!B) return fail(c, BL_EINVAL, "bad batch id %d", id);
  if (!p) return fail(c, BL_EINVAL, "null params");
  if (!B->started) return fail(c, BL_ESTATE, "bl_batch_start not called");
  if (p->eps_threshold > (1ull << 32)) return fail(c, BL_EINVAL, "eps_threshold > 2^32");
  HIP_TRY(c, hipSetDevice(c->device));
  return capture_steps(c, n_steps, [&](hipStream_t q) { return batch_step_on(c, *B, p, q); }, graph);
}

bl_status bl_graph_launch(bl_ctx *c, int32_t graph) {
  if (!c) return BL_EINVAL;
  if (graph < 0 || graph >= (int32_t)c->graphs.size()) return fail(c, BL_EINVAL, "bad graph id %d", graph);
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipGraphLaunch(c->graphs[graph], c->stream));
  return BL_OK;
}

}  // extern "C"

// ---------------------------------------------------------- learned screen

namespace {

Sur *get_sur(bl_ctx *c, int32_t id) {
  if (!c || id < 0 || id >= (int32_t)c->surs.size()) return nullptr;
  return c->surs[id].get();
}

template <class T>
bl_status sur_alloc(bl_ctx *c, Sur &S, T *&p, size_t n) {
  void *q = nullptr;
  HIP_TRY(c, hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)));
  S.allocs.push_back(q);
  p = (T *)q;
  return BL_OK;
}

bl_status sur_grads_on(bl_ctx *c, Sur &S, Instance &I, const uint64_t *d_moves, const float *cost,
                       const int32_t *mk, uint32_t n) {
  HIP_TRY(c, launch_sur_zero(S.D.loss, 2, c->stream));
  HIP_TRY(c, launch_sur_forward(I.P, S.D, d_moves, n, 0, true, c->n_cu, c->stream));
  HIP_TRY(c, launch_sur_head(I.P, S.D, n, 1, cost, mk, c->n_cu, c->stream));
  HIP_TRY(c, launch_sur_backward(I.P, S.D, n, c->n_cu, c->stream));
  return BL_OK;
}

}  // namespace

extern "C" {

bl_status bl_sur_create(bl_ctx *c, int32_t inst, const float *weights, const bl_sur_config *cfg,
                        int32_t *sur) {
  Instance *I = get_inst(c, inst);
  if (!I) return fail(c, BL_EINVAL, "bad instance id %d", inst);
  if (!weights || !cfg || !sur) return fail(c, BL_EINVAL, "null argument");
  if (I->xy.empty()) return fail(c, BL_EINVAL, "the instance was uploaded without coordinates");
  if (I->NB > 128) return fail(c, BL_EINVAL, "the learned screen supports at most 128 BPs");
  if (cfg->max_examples == 0 || !(cfg->c0_m > 0.f) || !(cfg->t0_s > 0.f) || !(cfg->lr > 0.f))
    return fail(c, BL_EINVAL, "bad surrogate configuration");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, sur_setup_attributes());
  auto S = std::make_unique<Sur>();
  S->inst = inst;
  S->cfg = *cfg;
  SurDev &D = S->D;
  const int NF = I->NF, NB = I->NB, NT = I->NT, V = I->V;
  // Scales: largest |coordinate|, area, yield, distance, shuttle distance.
  double ls = 1, as = 1, ys = 1, ds = 1, ws = 1;
  for (int32_t v : I->xy) ls = std::max(ls, (double)std::abs(v));
  for (int f = 0; f < NF; ++f) {
    as = std::max(as, (double)I->area[f]);
    ys = std::max(ys, (double)I->yld[f]);
  }
  for (uint32_t d : I->dist) ds = std::max(ds, (double)d);
  uint64_t capsum = 0;
  for (uint32_t cap : I->su_cap) capsum += cap;
  const uint64_t cbar = capsum / (uint64_t)I->NSU;
  std::vector<double> nsh(NF);
  for (int f = 0; f < NF; ++f) {
    nsh[f] = (double)((I->supply[f] + cbar - 1) / cbar);
    uint32_t dm = 0;
    for (int b = 0; b < NB; ++b) dm = std::max(dm, I->dist[(size_t)(1 + NB + f) * V + 1 + b]);
    ws = std::max(ws, 2.0 * nsh[f] * dm);
  }
  std::vector<float> fstat((size_t)NF * 8, 0.f), bxy((size_t)NB * 2);
  for (int f = 0; f < NF; ++f) {
    const int v = 1 + NB + f;
    fstat[f * 8 + 0] = (float)(I->xy[2 * v] / ls);
    fstat[f * 8 + 1] = (float)(I->xy[2 * v + 1] / ls);
    fstat[f * 8 + 2] = (float)(I->area[f] / as);
    fstat[f * 8 + 3] = (float)(I->yld[f] / ys);
    fstat[f * 8 + 4] = (float)(I->dist[v] / ds);
    fstat[f * 8 + 5] = (float)(2.0 * nsh[f] / ws);
  }
  for (int b = 0; b < NB; ++b) {
    bxy[2 * b] = (float)(I->xy[2 * (1 + b)] / ls);
    bxy[2 * b + 1] = (float)(I->xy[2 * (1 + b) + 1] / ls);
  }
  double rates = 0, fills = 0;
  for (uint32_t r : I->hu_rate) rates += r;
  for (uint32_t f : I->su_fill) fills += f;
  D.inv_ds = (float)(1.0 / ds);
  D.inv_c0 = 1.f / cfg->c0_m;
  D.inv_t0 = 1.f / cfg->t0_s;
  D.inv_rates = (float)(1.0 / rates);
  D.inv_fills = (float)(fills > 0 ? 1.0 / fills : 0.0);
  D.cap_ex = cfg->max_examples;
  const size_t rows = (size_t)cfg->max_examples * NF;
  Sur &R = *S;
  bl_status st = BL_OK;
  float *fs_d = nullptr, *bxy_d = nullptr;
  if ((st = sur_alloc(c, R, D.W, kSurParams)) || (st = sur_alloc(c, R, D.G, kSurParams)) ||
      (st = sur_alloc(c, R, D.Mo, kSurParams)) || (st = sur_alloc(c, R, D.Ve, kSurParams)) ||
      (st = sur_alloc(c, R, D.w1t, sur_w1t_elems())) || (st = sur_alloc(c, R, D.w2t, sur_w2_elems())) ||
      (st = sur_alloc(c, R, D.w2n, sur_w2_elems())) || (st = sur_alloc(c, R, D.w3et, sur_w3et_elems())) ||
      (st = sur_alloc(c, R, D.w3en, sur_w3en_elems())) || (st = sur_alloc(c, R, fs_d, fstat.size())) ||
      (st = sur_alloc(c, R, bxy_d, bxy.size())) || (st = sur_alloc(c, R, D.phi, rows * kSurK1)) ||
      (st = sur_alloc(c, R, D.row_bp, rows)) || (st = sur_alloc(c, R, D.h1, rows * kSurH)) ||
      (st = sur_alloc(c, R, D.h2, rows * kSurH)) || (st = sur_alloc(c, R, D.P, rows * kSurA)) ||
      (st = sur_alloc(c, R, D.dP, rows * kSurA)) ||
      (st = sur_alloc(c, R, D.ex_u, (size_t)cfg->max_examples * NT * kSurU)) ||
      (st = sur_alloc(c, R, D.ex_cnt, (size_t)cfg->max_examples * NB)) ||
      (st = sur_alloc(c, R, D.ex_nb, (size_t)cfg->max_examples * NT)) ||
      (st = sur_alloc(c, R, D.ex_btour, (size_t)cfg->max_examples * NB)) ||
      (st = sur_alloc(c, R, D.ex_pred, (size_t)cfg->max_examples * 2)) ||
      (st = sur_alloc(c, R, D.loss, 2)) ||
      (st = sur_alloc(c, R, D.part_h, (size_t)sur_head_grid(cfg->max_examples, c->n_cu) * 4 * kHeadPart)) ||
      (st = sur_alloc(c, R, D.part_b, (size_t)sur_bwd_grid(rows, c->n_cu) * kBwdPart))) {
    for (void *p : R.allocs) (void)hipFree(p);
    return st;
  }
  D.fstat = fs_d;
  D.bxy = bxy_d;
  HIP_TRY(c, hipMemcpy(fs_d, fstat.data(), fstat.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(bxy_d, bxy.data(), bxy.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(D.W, weights, kSurParams * 4, hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemset(D.G, 0, kSurParams * 4));
  HIP_TRY(c, hipMemset(D.Mo, 0, kSurParams * 4));
  HIP_TRY(c, hipMemset(D.Ve, 0, kSurParams * 4));
  HIP_TRY(c, launch_sur_pack(D, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->surs.push_back(std::move(S));
  *sur = (int32_t)c->surs.size() - 1;
  return BL_OK;
}

bl_status bl_sur_get_weights(bl_ctx *c, int32_t id, float *out) {
  Sur *S = get_sur(c, id);
  if (!S || !out) return fail(c, BL_EINVAL, "bad surrogate or null output");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(out, S->D.W, kSurParams * 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return BL_OK;
}

bl_status bl_sur_set_weights(bl_ctx *c, int32_t id, const float *w) {
  Sur *S = get_sur(c, id);
  if (!S || !w) return fail(c, BL_EINVAL, "bad surrogate or null weights");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(S->D.W, w, kSurParams * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, launch_sur_pack(S->D, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return BL_OK;
}

bl_status bl_sur_predict(bl_ctx *c, int32_t id, const uint64_t *d_moves, uint32_t n, float *d_out) {
  Sur *S = get_sur(c, id);
  if (!S) return fail(c, BL_EINVAL, "bad surrogate id %d", id);
  Instance *I = c->inst[S->inst].get();
  if (!I->base_ready) return fail(c, BL_ESTATE, "no base solution uploaded");
  if (n && (!d_moves || !d_out)) return fail(c, BL_EINVAL, "null buffer");
  HIP_TRY(c, hipSetDevice(c->device));
  for (uint32_t done = 0; done < n; done += S->D.cap_ex) {
    const uint32_t k = std::min(n - done, S->D.cap_ex);
    HIP_TRY(c, launch_sur_forward(I->P, S->D, d_moves + done, k, 0, false, c->n_cu, c->stream));
    HIP_TRY(c, launch_sur_head(I->P, S->D, k, 0, nullptr, nullptr, c->n_cu, c->stream));
    HIP_TRY(c, hipMemcpyAsync(d_out + 2 * (size_t)done, S->D.ex_pred, (size_t)k * 8,
                              hipMemcpyDeviceToDevice, c->stream));
  }
  return BL_OK;
}

bl_status bl_sur_gradients(bl_ctx *c, int32_t id, const uint64_t *d_moves, const float *d_cost_km,
                           const int32_t *d_makespan_s, uint32_t n, float *grads, double *loss) {
  Sur *S = get_sur(c, id);
  if (!S) return fail(c, BL_EINVAL, "bad surrogate id %d", id);
  Instance *I = c->inst[S->inst].get();
  if (!I->base_ready) return fail(c, BL_ESTATE, "no base solution uploaded");
  if (n == 0 || n > S->D.cap_ex) return fail(c, BL_EINVAL, "n %u out of 1..max_examples", n);
  if (!d_moves || !d_cost_km || !d_makespan_s || !grads || !loss) return fail(c, BL_EINVAL, "null buffer");
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, launch_sur_zero(S->D.G, kSurParams, c->stream));
  bl_status st = sur_grads_on(c, *S, *I, d_moves, d_cost_km, d_makespan_s, n);
  if (st != BL_OK) return st;
  float l[2];
  HIP_TRY(c, hipMemcpyAsync(grads, S->D.G, kSurParams * 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(l, S->D.loss, 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, launch_sur_zero(S->D.G, kSurParams, c->stream));
  *loss = l[0];
  return BL_OK;
}

bl_status bl_sur_train_step(bl_ctx *c, int32_t id, const uint64_t *d_moves, const float *d_cost_km,
                            const int32_t *d_makespan_s, uint32_t n, float *d_loss) {
  Sur *S = get_sur(c, id);
  if (!S) return fail(c, BL_EINVAL, "bad surrogate id %d", id);
  Instance *I = c->inst[S->inst].get();
  if (!I->base_ready) return fail(c, BL_ESTATE, "no base solution uploaded");
  if (n == 0 || n > S->D.cap_ex) return fail(c, BL_EINVAL, "n %u out of 1..max_examples", n);
  if (!d_moves || !d_cost_km || !d_makespan_s) return fail(c, BL_EINVAL, "null buffer");
  HIP_TRY(c, hipSetDevice(c->device));
  bl_status st = sur_grads_on(c, *S, *I, d_moves, d_cost_km, d_makespan_s, n);
  if (st != BL_OK) return st;
  S->step += 1;
  const bl_sur_config &g = S->cfg;
  HIP_TRY(c, launch_sur_adam(S->D, g.lr, g.beta1, g.beta2, g.adam_eps, 1.f / (float)n, S->step, c->stream));
  HIP_TRY(c, launch_sur_pack(S->D, c->stream));
  if (d_loss) HIP_TRY(c, hipMemcpyAsync(d_loss, S->D.loss, 8, hipMemcpyDeviceToDevice, c->stream));
  return BL_OK;
}

}  // extern "C"

namespace {

template <class T>
bl_status scr_alloc(bl_ctx *c, Sur &S, T *&p, size_t n) {
  void *q = nullptr;
  HIP_TRY(c, hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)));
  S.t_allocs.push_back(q);
  p = (T *)q;
  return BL_OK;
}

bl_status screen_buffers(bl_ctx *c, Sur &S, const Instance &I, uint32_t nprop, uint32_t k) {
  if (S.T.keys && S.t_nprop >= nprop && S.t_k >= k) return BL_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (void *p : S.t_allocs) (void)hipFree(p);
  S.t_allocs.clear();
  ScreenDev &T = S.T;
  const size_t NB = I.NB, NT = I.NT;
  bl_status st = BL_OK;
  if ((st = scr_alloc(c, S, T.Q, NB * kSurA)) ||
      (st = scr_alloc(c, S, T.R, NT * kSurA)) || (st = scr_alloc(c, S, T.U, NT * kSurA)) ||
      (st = scr_alloc(c, S, T.ub6, NT)) || (st = scr_alloc(c, S, T.yb, 2 * NT)) ||
      (st = scr_alloc(c, S, T.nbg, NT)) || (st = scr_alloc(c, S, T.nfg, NT)) ||
      (st = scr_alloc(c, S, T.scal, 4)) ||
      (st = scr_alloc(c, S, T.top_g, 3)) ||
      (st = scr_alloc(c, S, T.keys, nprop)) || (st = scr_alloc(c, S, T.hist, 2048)) ||
      (st = scr_alloc(c, S, T.sel, 8)) || (st = scr_alloc(c, S, T.blk, 2048)) ||
      (st = scr_alloc(c, S, T.short_idx, k)) || (st = scr_alloc(c, S, T.short_key, k)) ||
      (st = scr_alloc(c, S, T.short_cost, k)) || (st = scr_alloc(c, S, T.flag, 1)) ||
      (st = scr_alloc(c, S, T.ctrl_key, 1)) ||
      (st = scr_alloc(c, S, T.stats, 4))) {
    for (void *p : S.t_allocs) (void)hipFree(p);
    S.t_allocs.clear();
    S.T = ScreenDev{};
    return st;
  }
  HIP_TRY(c, hipMemset(T.stats, 0, 16));
  HIP_TRY(c, hipMemset(T.flag, 0, 4));
  S.t_nprop = nprop;
  S.t_k = k;
  return BL_OK;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// Validation, buffers, base pick and screen of one iteration's proposals.
bl_status screen_on(bl_ctx *c, Sur *S, const bl_search_params *p, const bl_screen_params *sc,
                    Instance *&I, hipStream_t &q) {
  if (!S) return fail(c, BL_EINVAL, "bad surrogate id");
  I = c->inst[S->inst].get();
  if (!p || !sc) return fail(c, BL_EINVAL, "null params");
  if (!I->started) return fail(c, BL_ESTATE, "bl_search_start not called");
  if (sc->n_proposals == 0 || sc->n_proposals > kMaxCand)
    return fail(c, BL_EINVAL, "n_proposals out of 1..2^24");
  if (sc->n_shortlist == 0 || sc->n_shortlist > sc->n_proposals)
    return fail(c, BL_EINVAL, "n_shortlist out of 1..n_proposals");
  if (sc->n_fallback > kMaxCand) return fail(c, BL_EINVAL, "n_fallback > 2^24");
  if (sc->n_control > sc->n_proposals) return fail(c, BL_EINVAL, "n_control > n_proposals");
  if (p->eps_threshold > (1ull << 32)) return fail(c, BL_EINVAL, "eps_threshold > 2^32");
  HIP_TRY(c, hipSetDevice(c->device));
  if (c->capturing && !(S->T.keys && S->t_nprop >= sc->n_proposals && S->t_k >= sc->n_shortlist))
    return fail(c, BL_ESTATE, "run one screened call of this size before capturing it");
  if (screen_waves(I->P) == 0)
    return fail(c, BL_EINVAL, "instance too large for the screen's LDS layout (image + BP and tour tables)");
  bl_status st = screen_buffers(c, *S, *I, sc->n_proposals, sc->n_shortlist);
  if (st != BL_OK) return st;
  q = work_stream(c);
  HIP_TRY(c, launch_prepare(I->P, kPrepSearch, p->seed, p->eps_threshold, p->inst_index, q));
  HIP_TRY(c, launch_screen_base(I->P, S->D, S->T, c->n_cu, q));
  HIP_TRY(c, timing_mark(c, kTimeScreen));
  HIP_TRY(c, launch_screen_score(I->P, S->D, S->T, p->seed, p->inst_index, sc->n_proposals, sc->mk_margin,
                                 c->n_cu, q));
  HIP_TRY(c, timing_mark(c, kTimeScreen));
  HIP_TRY(c, launch_screen_select(S->T, sc->n_proposals, sc->n_shortlist, q));
  return BL_OK;
}

}  // namespace

extern "C" {

bl_status bl_sur_screen(bl_ctx *c, int32_t id, const bl_search_params *p, const bl_screen_params *sc,
                        uint32_t *d_shortlist, float *d_score) {
  if (!d_shortlist) return fail(c, BL_EINVAL, "null shortlist buffer");
  Sur *S = get_sur(c, id);
  Instance *I = nullptr;
  hipStream_t q = nullptr;
  bl_status st = screen_on(c, S, p, sc, I, q);
  if (st != BL_OK) return st;
  HIP_TRY(c, hipMemcpyAsync(d_shortlist, S->T.short_idx, (size_t)sc->n_shortlist * 4,
                            hipMemcpyDeviceToDevice, q));
  if (d_score) HIP_TRY(c, launch_scr_export(S->T, sc->n_proposals, d_score, q));
  return BL_OK;
}

bl_status bl_sur_search_step(bl_ctx *c, int32_t id, const bl_search_params *p,
                             const bl_screen_params *sc) {
  Sur *S = get_sur(c, id);
  Instance *I = nullptr;
  hipStream_t q = nullptr;
  bl_status st = screen_on(c, S, p, sc, I, q);
  if (st != BL_OK) return st;
  // The control sample first: its best key is the instance's argmin slot
  // until the shortlist joins.
  HIP_TRY(c, launch_eval_search(I->P, p->seed, sc->n_control, p->inst_index,
                                grid_for(c, *I, std::max(sc->n_control, 1u), true), q, nullptr));
  HIP_TRY(c, launch_scr_control_save(I->P, S->T, q));
  HIP_TRY(c, launch_eval_gather(I->P, p->seed, S->T.short_idx, sc->n_shortlist, p->inst_index,
                                S->T.short_key, S->T.short_cost, grid_for(c, *I, sc->n_shortlist, true), q));
  HIP_TRY(c, launch_scr_check(I->P, S->D, S->T, sc->n_shortlist, sc->err_threshold, q));
  if (sc->n_fallback)
    HIP_TRY(c, launch_eval_search(I->P, p->seed, sc->n_fallback, p->inst_index,
                                  grid_for(c, *I, sc->n_fallback, true), q, S->T.flag));
  HIP_TRY(c, launch_commit(I->P, kCommitStep, p->seed, p->inst_index, q));
  return BL_OK;
}

bl_status bl_sur_stats_get(bl_ctx *c, int32_t id, bl_sur_stats *out) {
  Sur *S = get_sur(c, id);
  if (!S || !out) return fail(c, BL_EINVAL, "bad surrogate or null output");
  *out = bl_sur_stats{0, 0, 0, 0.f};
  if (!S->T.stats) return BL_OK;
  float st[4];
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(st, S->T.stats, 16, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  out->iterations = (uint32_t)st[2];
  out->fallbacks = (uint32_t)st[1];
  out->last_used = (uint32_t)st[3];
  out->last_error = st[0];
  return BL_OK;
}

bl_status bl_timing_enable(bl_ctx *c, int32_t what) {
  if (!c) return BL_EINVAL;
  if (what < 0 || what > BL_TIMING_SCREEN) return fail(c, BL_EINVAL, "timing: 0, BL_TIMING_EVAL or BL_TIMING_SCREEN");
  c->timing = what;
  return BL_OK;
}

bl_status bl_measure_peaks(bl_ctx *c, double *hbm_gbs, double *lds_gbs) {
  if (!c) return BL_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  auto best_ms = [&](auto launch, float &out) -> hipError_t {
    hipError_t e = launch();  // warm-up
    if (e != hipSuccess) return e;
    out = 1e30f;
    for (int r = 0; r < 5; ++r) {
      if ((e = hipEventRecord(e0, c->stream)) != hipSuccess || (e = launch()) != hipSuccess ||
          (e = hipEventRecord(e1, c->stream)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess)
        return e;
      float ms = 0.f;
      if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return e;
      out = std::min(out, ms);
    }
    return hipSuccess;
  };
  bl_status st = BL_OK;
  if (hbm_gbs) {
    const size_t bytes = (size_t)1 << 30;
    void *a = nullptr, *b = nullptr;
    hipError_t e = hipMalloc(&a, bytes);
    if (e == hipSuccess) e = hipMalloc(&b, bytes);
    if (e == hipSuccess) e = hipMemsetAsync(a, 1, bytes, c->stream);
    float ms = 0.f;
    if (e == hipSuccess) e = best_ms([&] { return launch_peak_copy(a, b, bytes, c->n_cu, c->stream); }, ms);
    if (e == hipSuccess) *hbm_gbs = 2.0 * (double)bytes / (ms * 1e-3) / 1e9;
    else st = hip_fail(c, e, "HBM copy probe");
    (void)hipFree(a);
    (void)hipFree(b);
  }
  if (lds_gbs && st == BL_OK) {
    const uint32_t steps = 1u << 14;
    const size_t lanes = peak_lds_blocks(c->n_cu) * 256;
    uint32_t *out = nullptr;
    hipError_t e = hipMalloc(&out, lanes * 4);
    float ms = 0.f;
    if (e == hipSuccess) e = best_ms([&] { return launch_peak_lds(steps, out, c->n_cu, c->stream); }, ms);
    if (e == hipSuccess) *lds_gbs = (double)lanes * steps * 16.0 / (ms * 1e-3) / 1e9;
    else st = hip_fail(c, e, "LDS read probe");
    (void)hipFree(out);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
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
