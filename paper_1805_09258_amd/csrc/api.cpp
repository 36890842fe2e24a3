// api.cpp -- the C ABI of librc (see include/rc.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "learned.hpp"
#include "render.hpp"
#include "j08.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define RC_HIP(call)                                                                                   \
  do {                                                                                                 \
    hipError_t e_ = (call);                                                                            \
    if (e_ != hipSuccess) return fail(RC_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));      \
  } while (0)

bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// One record-kernel launch of a batched call.
struct Launch {
  rc::RecordArgs args;
  int grid;
  size_t lds;
};

struct GraphCache {
  bool valid = false;
  std::vector<Launch> plan;
  int stack = 0;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void clear() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    valid = false;
  }
};

}  // namespace

struct rc_scene {
  int device = 0;
  int n_cu = 0;
  std::string arch;
  int64_t T = 0;
  int64_t n_nodes = 0;
  int depth = 0;
  float pad = 0.f;
  float box_lo[3], box_hi[3];
  float4* nodes = nullptr;
  float4* tris = nullptr;     // three copies of the triangle records (copy k permuted for kz = k)
  int tri_stride = 0;         // float4 words per copy
  float4* shade = nullptr;
  double4* plane = nullptr;
  float* emission = nullptr;
  std::vector<float> tri_host;  // the input triangles (light bins are built from them)
  // per-light triangle bins of the last light set (positions), device copies
  struct {
    int n = 0;
    float pos[RC_MAX_LIGHTS][3];
    int4* desc = nullptr;
    int* offs = nullptr;
    float4* ent = nullptr;
    int64_t n_entries = 0;
    int64_t bytes = 0;
    void clear() {
      if (desc) (void)hipFree(desc);
      if (offs) (void)hipFree(offs);
      if (ent) (void)hipFree(ent);
      desc = nullptr;
      offs = nullptr;
      ent = nullptr;
      n = 0;
      n_entries = 0;
      bytes = 0;
    }
  } lb;
  int64_t device_bytes = 0;  // nodes, triangle copies, shading, planes, emission
  float2* hits = nullptr;    // primary hits of the last batched call with a hits pass
  size_t hits_bytes = 0;
  unsigned int* vis = nullptr;  // their vertices' visibility bits (shadow pass)
  size_t vis_bytes = 0;
  std::mutex mu;
  GraphCache graph;
  ~rc_scene() {
    graph.clear();
    lb.clear();
    if (hits) (void)hipFree(hits);
    if (vis) (void)hipFree(vis);
    if (nodes) (void)hipFree(nodes);
    if (tris) (void)hipFree(tris);
    if (shade) (void)hipFree(shade);
    if (plane) (void)hipFree(plane);
    if (emission) (void)hipFree(emission);
  }
};

namespace {

// queue area (kQueueWords words, see kernels.hpp); then the bucket counts and
// cursors of the device-built queue, the queue order itself,
constexpr size_t kWsQueue = 0, kWsHist = 4 * rc::kQueueWords, kWsCursor = kWsHist + 4 * rc::kOrderBuckets,
                 kWsOrder = kWsCursor + 4 * rc::kOrderBuckets;
// after the queue order: per-record part counters, then per-part partial sums
// launch configurations ("tiles"): persistent grid as a multiple of the
// resident wave capacity, idle lanes that trigger a refill of the shadow
// loop, lanes waiting at a leaf that trigger a triangle step, and the
// resident wavefronts per SIMD the LDS row width is sized for (fewer: wider
// rows, fewer column sectors, but less latency hiding)
struct Tile {
  float grid;
  int refill_min, leaf_batch, lds_waves;
};
constexpr int kNTiles = 10;
constexpr Tile kTiles[kNTiles] = {{1.0f, 12, 0, 4}, {2.0f, 12, 0, 4}, {1.0f, 8, 0, 4},  {1.0f, 16, 0, 4},
                                  {1.0f, 12, 8, 4}, {2.0f, 12, 8, 4}, {0.5f, 12, 0, 4}, {1.0f, 24, 0, 4},
                                  {1.0f, 12, 0, 3}, {1.0f, 12, 0, 2}};

constexpr size_t ws_split_offset(int64_t P) {
  return (kWsOrder + 4 * (size_t)(P > 0 ? P : 0) + 255) & ~size_t(255);
}
constexpr size_t ws_partial_offset(int64_t Pm) { return (4 * (size_t)Pm + 255) & ~size_t(255); }
constexpr size_t ws_bytes(int64_t P) {
  return ws_split_offset(P) + ws_partial_offset(P < rc::kSplitMaxRecords ? P : rc::kSplitMaxRecords) +
         (size_t)(P < rc::kSplitMaxRecords ? P : rc::kSplitMaxRecords) * rc::kMaxSplits * 20 * sizeof(double);
}

// Workspace of rc_records_noalloc: one per device, in the library's device
// image (no allocation at call time).  Host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocBytes = ws_bytes(RC_NOALLOC_MAX_RECORDS);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (the current device), looked up
// once per device.
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(RC_ENODEV, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(RC_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return RC_OK;
}

int check_inputs(const rc_scene* s, const rc_medium* m, const rc_point_light* lights, int n_lights, const float* pos,
                 const int32_t* nth, const int32_t* nph, int64_t P, const rc_params* p, double* value, double* grad,
                 double* hess, void* ws) {
  if (!s) return fail(RC_EINVAL, "scene is NULL");
  if (!m || !std::isfinite(m->sigma_s) || !std::isfinite(m->sigma_a) || m->sigma_s < 0 || m->sigma_a < 0)
    return fail(RC_EINVAL, "medium coefficients must be finite and >= 0");
  if (n_lights < 0 || n_lights > RC_MAX_LIGHTS) return fail(RC_EINVAL, "n_lights must be in [0, %d]", RC_MAX_LIGHTS);
  if (n_lights > 0 && !lights) return fail(RC_EINVAL, "lights is NULL");
  for (int l = 0; l < n_lights; l++)
    if (!finite3(lights[l].pos) || !std::isfinite(lights[l].intensity) || lights[l].intensity < 0)
      return fail(RC_EINVAL, "light %d is not finite or has negative intensity", l);
  if (P < 0 || P > 0x7fffffff) return fail(RC_EINVAL, "P out of range");
  if (!p) return fail(RC_EINVAL, "params is NULL");
  if (!(p->ring_step > 0.f) || !std::isfinite(p->ring_step)) return fail(RC_EINVAL, "ring_step must be > 0");
  if (p->max_rings < 1 || p->max_rings > RC_MAX_RINGS) return fail(RC_EINVAL, "max_rings must be in [1, %d]", RC_MAX_RINGS);
  if (p->max_n_phi < 5 || p->max_n_phi > RC_MAX_NPHI) return fail(RC_EINVAL, "max_n_phi must be in [5, %d]", RC_MAX_NPHI);
  if (p->max_n_theta < 0 || (p->max_n_theta > 0 && (int64_t)p->max_n_theta * p->max_n_phi + 2 > (1 << 24)))
    return fail(RC_EINVAL, "max_n_theta must be 0 or at most 2^24 / max_n_phi");
  if (p->precision != 0 && p->precision != 1) return fail(RC_EINVAL, "precision must be 0 or 1");
  if (p->common_random != 0 && p->common_random != 1) return fail(RC_EINVAL, "common_random must be 0 or 1");
  if (p->shadow_bvh != 0 && p->shadow_bvh != 1) return fail(RC_EINVAL, "shadow_bvh must be 0 or 1");
  if (p->shadow_pass != 0 && p->shadow_pass != 1) return fail(RC_EINVAL, "shadow_pass must be 0 or 1");
  if (p->splits < 0 || p->splits > rc::kMaxSplits) return fail(RC_EINVAL, "splits must be in [0, %d]", rc::kMaxSplits);
  if (p->splits > 1 && P > rc::kSplitMaxRecords)
    return fail(RC_EINVAL, "splits > 1 needs P <= %d", rc::kSplitMaxRecords);
  if (p->rec_base < 0) return fail(RC_EINVAL, "rec_base must be >= 0");
  if (P > 0 && (!pos || !nth || !nph || !value || !grad || !hess))
    return fail(RC_EINVAL, "NULL input or output pointer");
  if (P > 0 && !ws) return fail(RC_EINVAL, "workspace is NULL");
  return RC_OK;
}

// LDS row width.  The record kernel's register budget allows W = 16 or 12
// wavefronts per CU (record_waves_per_simd); rows are held whole when that
// fits the LDS, else in sectors of w columns (plus one) with the widest
// w <= 32 for which a wavefront's LDS (stack, two rows, offsets) stays within
// 1/W of the CU's 160 KB.  Measured at 64 columns: whole rows at 8 wavefronts
// per CU gave 0.79x the records/s of 33-column LDS rows at 12, and 26-column
// LDS rows at 16 gave 1.09x those at 12.
int lds_cols_for(int max_n_phi, int stack, int max_rings, int lds_waves = 0) {
  const int wps = lds_waves > 0 ? std::min(lds_waves, rc::record_waves_per_simd(stack)) : rc::record_waves_per_simd(stack);
  const size_t budget = (size_t)160 * 1024 / (4 * wps);
  if (rc::record_lds_bytes(stack, max_n_phi, max_rings) <= budget) return max_n_phi;
  for (int w = std::min(32, max_n_phi - 1); w >= 8; w--)
    if (rc::record_lds_bytes(stack, w + 1, max_rings) <= budget) return w + 1;
  return std::min(max_n_phi, 33);  // deep stacks or many rings: fewer wavefronts
}

// Build and upload the light bins of these light positions unless the scene
// already holds them.  Caller holds s->mu.
int ensure_light_bins(rc_scene* s, const rc_point_light* lights, int n_lights, int B) {
  if (n_lights <= 0) return RC_OK;
  bool same = s->lb.n == n_lights && s->lb.desc != nullptr;
  for (int l = 0; same && l < n_lights; l++)
    same = std::memcmp(s->lb.pos[l], lights[l].pos, sizeof(float) * 3) == 0;
  if (same && B == 0) return RC_OK;
  if (B == 0) B = rc::light_bins_size_for(s->T);
  std::vector<rc::LightBinsHost> h((size_t)n_lights);
  std::vector<std::string> errs((size_t)n_lights);
  std::vector<int> rcs((size_t)n_lights, RC_OK);
  {
    std::vector<std::thread> th;
    for (int l = 0; l < n_lights; l++)
      th.emplace_back([&, l] {
        rcs[l] = rc::build_light_bins(s->tri_host.data(), s->T, s->pad, lights[l].pos, B, h[l], errs[l]);
      });
    for (auto& t : th) t.join();
  }
  for (int l = 0; l < n_lights; l++)
    if (rcs[l] != RC_OK) return fail(rcs[l], "%s", errs[l].c_str());
  // concatenate: offsets shifted to absolute entry indices
  std::vector<int32_t> offs;
  std::vector<float> ent;
  std::vector<int4> desc(2 * (size_t)n_lights);
  int64_t ebase = 0;
  for (int l = 0; l < n_lights; l++) {
    const int64_t obase = (int64_t)offs.size();
    if (ebase + (int64_t)(h[l].entries.size() / 12) >= ((int64_t)1 << 31) || obase + (int64_t)h[l].offs.size() >= ((int64_t)1 << 31))
      return fail(RC_EINVAL, "light bins: more than 2^31 entries or bins");
    // index words (each bin's first entry, each level's end) move by the
    // entries of the lights before; the distance words stay as they are
    for (size_t i = 0; i < h[l].offs.size(); i++) offs.push_back(h[l].offs[i]);
    for (int k = 0; k < h[l].nlev; k++) {
      const int64_t Bk = h[l].B >> (2 * k);
      for (int64_t i = 0; i <= 12 * Bk * Bk; i += 2) offs[(size_t)(obase + h[l].lev_off[k] + i)] += (int32_t)ebase;
    }
    ent.insert(ent.end(), h[l].entries.begin(), h[l].entries.end());
    int lo[rc::kLbMaxLevels] = {0, 0, 0, 0};
    for (int k = 0; k < h[l].nlev; k++) lo[k] = (int)(obase + h[l].lev_off[k]);
    desc[2 * l] = make_int4(h[l].B, h[l].nlev, lo[0], lo[1]);
    desc[2 * l + 1] = make_int4(lo[2], lo[3], 0, 0);
    ebase += (int64_t)(h[l].entries.size() / 12);
  }
  ent.resize(ent.size() + 4, 0.f);
  s->graph.clear();  // launches captured with the old buffers
  s->lb.clear();
  auto up = [&](void** dst, const void* src, size_t bytes) -> int {
    if (hipMalloc(dst, std::max<size_t>(bytes, 16)) != hipSuccess) return fail(RC_ENOMEM, "hipMalloc %zu", bytes);
    if (bytes && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return fail(RC_EDEVICE, "hipMemcpy");
    return RC_OK;
  };
  int r = up((void**)&s->lb.desc, desc.data(), desc.size() * sizeof(int4));
  if (!r) r = up((void**)&s->lb.offs, offs.data(), offs.size() * 4);
  if (!r) r = up((void**)&s->lb.ent, ent.data(), ent.size() * 4);
  if (r) {
    s->lb.clear();
    return r;
  }
  s->lb.n = n_lights;
  for (int l = 0; l < n_lights; l++) std::memcpy(s->lb.pos[l], lights[l].pos, sizeof(float) * 3);
  s->lb.n_entries = ebase;
  s->lb.bytes = (int64_t)(desc.size() * sizeof(int4) + offs.size() * 4 + ent.size() * 4);
  return RC_OK;
}

rc::RecordArgs make_args(const rc_scene* s, const rc_medium* m, const rc_point_light* lights, int n_lights,
                         const float* pos, const int32_t* nth, const int32_t* nph, int64_t P, const rc_params* p,
                         double* value, double* grad, double* hess, void* ws, const int32_t* order) {
  rc::RecordArgs a;
  std::memset(&a, 0, sizeof a);  // padding too: the graph cache compares whole structs
  a.nodes = s->nodes;
  a.tris = s->tris;
  a.tri_stride = s->tri_stride;
  a.shade = s->shade;
  a.plane = s->plane;
  a.emission = s->emission;
  a.box_lo = make_float3(s->box_lo[0], s->box_lo[1], s->box_lo[2]);
  a.box_hi = make_float3(s->box_hi[0], s->box_hi[1], s->box_hi[2]);
  a.n_lights = n_lights;
  for (int l = 0; l < n_lights; l++)
    a.lights[l] = make_float4(lights[l].pos[0], lights[l].pos[1], lights[l].pos[2], lights[l].intensity);
  a.sigma_s = m->sigma_s;
  a.sigma_a = m->sigma_a;
  a.pos = pos;
  a.n_theta = nth;
  a.n_phi = nph;
  a.P = (int)P;
  a.rec_base = p->rec_base;
  a.common_random = p->common_random;
  a.ring_step = p->ring_step;
  a.max_rings = p->max_rings;
  a.max_n_phi = p->max_n_phi;
  a.lds_cols = lds_cols_for(p->max_n_phi, rc::stack_variant(s->depth), p->max_rings);
  a.precision = p->precision;
  a.seed = p->seed;
  a.value = value;
  a.grad = grad;
  a.hess = hess;
  a.order = order;
  a.queue = reinterpret_cast<unsigned int*>(static_cast<char*>(ws) + kWsQueue);
  a.range = nullptr;  // slots 0..P-1
  a.next = a.queue;
  a.hits = nullptr;  // the record kernel traces its primary rays
  a.hit_stride = 0;
  a.max_n_theta = p->max_n_theta;
  a.trace_stack = rc::stack_variant(s->depth);
  a.vis = nullptr;
  a.vis_words = 0;
  a.vis_shift = 0;
  a.counters = reinterpret_cast<unsigned long long*>(p->counters);
  a.splits = 1;
  a.refill_min = kTiles[0].refill_min;
  a.leaf_batch = kTiles[0].leaf_batch;
  if (p->shadow_bvh == 0 && n_lights > 0 && s->lb.n == n_lights) {
    a.lb_desc = s->lb.desc;
    a.lb_offs = s->lb.offs;
    a.lb_ent = s->lb.ent;
  }
  return a;
}

// Wavefronts per record: explicit (params->splits) or chosen to minimise a
// makespan model of the persistent launch: the work spread over the resident
// wavefronts, P (1 + (S - 1) / 12) / resident record-times, plus the tail of
// one part, 1 / S.  Each extra part costs about 1/12 of a record: one
// recomputed row of ~16 plus its own queue pop, partial sums and share of the
// final reduction (measured at 10 000 records on 4 096 resident wavefronts:
// 2 parts 1.3 % faster than 3, where a cost of 1/16 per part picked 3).
void set_splits(rc::RecordArgs& a, const rc_params* p, int64_t P, int64_t resident, void* ws) {
  int S = p->splits;
  if (S == 0) {
    S = 1;
    if (P <= rc::kSplitMaxRecords && P > 0) {
      const double rows = 12.0;
      double best = 1e300;
      for (int k = 1; k <= rc::kMaxSplits; k++) {
        const double t = (double)P * (1.0 + (k - 1) / rows) / (double)resident + 1.0 / k;
        if (t < best - 1e-9) {
          best = t;
          S = k;
        }
      }
    }
  }
  a.splits = S;
  if (S > 1) {
    char* base = static_cast<char*>(ws) + ws_split_offset(P);
    a.done = reinterpret_cast<unsigned int*>(base);
    a.partial = reinterpret_cast<double*>(base + ws_partial_offset(std::min<int64_t>(P, rc::kSplitMaxRecords)));
  }
}

// Hits pass of rc_records_batched: with an n_theta bound and no counters.
bool hits_mode(const rc_params* p) { return p->max_n_theta > 0 && !p->counters; }

int plan(const rc_scene* s, const rc_params* p, int64_t P, int tile, int& stack, size_t& lds, int& grid,
         int64_t* resident_out = nullptr, bool hits = false) {
  // with the hits pass and light bins the record kernel traverses nothing
  stack = (hits && p->shadow_bvh == 0) ? rc::kHitsStack : rc::stack_variant(s->depth);
  const int t = (tile >= 0 && tile < kNTiles) ? tile : 0;
  lds = rc::record_lds_bytes(stack, lds_cols_for(p->max_n_phi, stack, p->max_rings, kTiles[t].lds_waves),
                             p->max_rings);
  if (lds > 160 * 1024) return fail(RC_EINVAL, "max_n_phi x max_rings needs %zu bytes of LDS (> 160 KiB)", lds);
  hipError_t e = rc::prepare_record(stack, p->counters != nullptr, p->precision == 1, lds);
  if (e != hipSuccess) return fail(RC_EDEVICE, "kernel attribute: %s", hipGetErrorString(e));
  int occ = rc::record_occupancy(stack, p->counters != nullptr, p->precision == 1, lds);
  if (occ < 1) occ = 1;
  int64_t resident = (int64_t)occ * s->n_cu;
  if (resident_out) *resident_out = resident;
  int64_t gsz = (int64_t)std::llround((double)resident * kTiles[t].grid);
  gsz = std::max<int64_t>(1, std::min<int64_t>(gsz, P * (int64_t)rc::kMaxSplits));
  grid = (int)gsz;
  return RC_OK;
}

// The launches of one call.  Every counter that must start at zero (queue,
// class cursors, part counters) is cleared by a kernel first; the partial sums
// of split records are written before they are read.
hipError_t run_plan(const Launch* plan, size_t n, int stack, hipStream_t st) {
  const rc::RecordArgs& a0 = plan[0].args;
  hipError_t e = rc::launch_reset(a0.queue, st);
  if (e == hipSuccess && a0.hits) {
    // the pass covers every class: the call's n_phi bound is the widest launch's
    rc::RecordArgs pa = a0;
    for (size_t i = 1; i < n; i++) pa.max_n_phi = std::max(pa.max_n_phi, plan[i].args.max_n_phi);
    e = rc::launch_primary(pa, pa.trace_stack, a0.P, st);
  }
  if (e == hipSuccess && a0.splits > 1) e = rc::launch_zero_u32(a0.done, a0.P, st);
  for (size_t i = 0; i < n && e == hipSuccess; i++) {
    const Launch& l = plan[i];
    e = rc::launch_record(l.args, stack, l.args.counters != nullptr, l.args.precision == 1, l.grid, l.lds, st);
  }
  return e;
}
hipError_t run_plan(const std::vector<Launch>& plan, int stack, hipStream_t st) {
  return run_plan(plan.data(), plan.size(), stack, st);
}

int launch_direct(rc_scene* s, const rc::RecordArgs& a, int stack, size_t lds, int grid, hipStream_t st) {
  (void)s;
  const Launch one{a, grid, lds};
  RC_HIP(run_plan(&one, 1, stack, st));
  return RC_OK;
}

}  // namespace

extern "C" {

const char* rc_last_error(void) { return g_last_error.c_str(); }
const char* rc_version(void) { return "librc 0.1 (gfx950)"; }

int rc_scene_create(const float* tri, const float* albedo, const float* emission, int64_t T, const float box_lo[3],
                    const float box_hi[3], rc_scene** out) {
  if (!out) return fail(RC_EINVAL, "out is NULL");
  *out = nullptr;
  if (T < 0) return fail(RC_EINVAL, "T < 0");
  if (T > 0 && (!tri || !albedo)) return fail(RC_EINVAL, "tri/albedo NULL");
  if (!box_lo || !box_hi || !finite3(box_lo) || !finite3(box_hi)) return fail(RC_EINVAL, "box not finite");
  for (int k = 0; k < 3; k++)
    if (!(box_hi[k] > box_lo[k])) return fail(RC_EINVAL, "empty box");
  float tol[3];
  for (int k = 0; k < 3; k++) tol[k] = 1e-4f * (box_hi[k] - box_lo[k]);
  for (int64_t i = 0; i < 9 * T; i++) {
    if (!std::isfinite(tri[i])) return fail(RC_EINVAL, "triangle %lld not finite", (long long)(i / 9));
    int k = (int)(i % 3);
    if (tri[i] < box_lo[k] - tol[k] || tri[i] > box_hi[k] + tol[k])
      return fail(RC_EINVAL, "triangle %lld outside the medium box", (long long)(i / 9));
  }
  for (int64_t i = 0; i < T; i++) {
    if (!std::isfinite(albedo[i]) || albedo[i] < 0) return fail(RC_EINVAL, "albedo %lld invalid", (long long)i);
    if (emission && (!std::isfinite(emission[i]) || emission[i] < 0))
      return fail(RC_EINVAL, "emission %lld invalid", (long long)i);
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(RC_ENODEV, "no HIP device");
  int dev = 0;
  RC_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  RC_HIP(hipGetDeviceProperties(&prop, dev));
  std::string arch = prop.gcnArchName;
  if (arch.find("gfx950") == std::string::npos) return fail(RC_ENODEV, "device %d is %s, not gfx950", dev, arch.c_str());

  rc::HostBvh bvh;
  std::string err;
  float pad = rc::bvh_pad_for(tri, T, box_lo, box_hi);
  int rc_ = rc::build_bvh(tri, T, pad, bvh, err);
  if (rc_ != RC_OK) return fail(rc_, "BVH build: %s", err.c_str());

  rc_scene* s = new (std::nothrow) rc_scene();
  if (!s) return fail(RC_ENOMEM, "host allocation");
  s->device = dev;
  s->n_cu = prop.multiProcessorCount;
  s->arch = arch;
  s->T = T;
  s->n_nodes = (int64_t)bvh.nodes.size() / 16;
  s->depth = bvh.depth;
  s->pad = pad;
  for (int k = 0; k < 3; k++) { s->box_lo[k] = box_lo[k]; s->box_hi[k] = box_hi[k]; }
  s->tri_host.assign(tri, tri + 9 * T);
  // per-triangle shading data
  std::vector<float> shade(4 * std::max<int64_t>(T, 1), 0.f), em(std::max<int64_t>(T, 1), 0.f);
  // FP64 plane of each triangle (unit normal n from the FP32 vertices, n . v0):
  // the hit distance the derivative terms use is the exact ray-plane distance
  // of the decided triangle
  std::vector<double> plane(4 * std::max<int64_t>(T, 1), 0.0);
  for (int64_t i = 0; i < T; i++) {
    const float* t = tri + 9 * i;
    double e1[3] = {(double)t[3] - t[0], (double)t[4] - t[1], (double)t[5] - t[2]};
    double e2[3] = {(double)t[6] - t[0], (double)t[7] - t[1], (double)t[8] - t[2]};
    double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    double ln = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int k = 0; k < 3; k++) shade[4 * i + k] = ln > 0 ? (float)(n[k] / ln) : 0.f;
    shade[4 * i + 3] = albedo[i];
    for (int k = 0; k < 3; k++) plane[4 * i + k] = ln > 0 ? n[k] / ln : 0.0;
    plane[4 * i + 3] = (plane[4 * i] * t[0] + plane[4 * i + 1] * t[1]) + plane[4 * i + 2] * t[2];
    em[i] = emission ? emission[i] : 0.f;
  }
  auto up = [&](void** dst, const void* src, size_t bytes) -> int {
    if (hipMalloc(dst, std::max<size_t>(bytes, 16)) != hipSuccess) return fail(RC_ENOMEM, "hipMalloc %zu", bytes);
    if (bytes && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
      return fail(RC_EDEVICE, "hipMemcpy");
    return RC_OK;
  };
  // Three copies of the triangle records, copy k with every vertex permuted
  // to (v[(k+1)%3], v[(k+2)%3], v[k]): a ray whose largest direction
  // component is k reads copy k, so the watertight test selects nothing per
  // vertex.  One padding word after the last record of the last copy keeps
  // the traversal's fourth 16-byte load in bounds.
  const size_t per_copy = bvh.tris.size();  // floats, 12 per triangle
  s->tri_stride = (int)(per_copy / 4);
  std::vector<float> tris3(3 * per_copy + 4, 0.f);
  for (int k = 0; k < 3; k++)
    for (size_t i = 0; i < per_copy; i += 4) {
      const float* q = bvh.tris.data() + i;
      float* o = tris3.data() + k * per_copy + i;
      o[0] = q[(k + 1) % 3];
      o[1] = q[(k + 2) % 3];
      o[2] = q[k];
      o[3] = q[3];  // id bits (first word) or 0
    }
  int r = up((void**)&s->nodes, bvh.nodes.data(), bvh.nodes.size() * 4);
  if (!r) r = up((void**)&s->tris, tris3.data(), tris3.size() * 4);
  if (!r) r = up((void**)&s->shade, shade.data(), shade.size() * 4);
  if (!r) r = up((void**)&s->plane, plane.data(), plane.size() * 8);
  if (!r) r = up((void**)&s->emission, em.data(), em.size() * 4);
  s->device_bytes = (int64_t)(bvh.nodes.size() * 4 + tris3.size() * 4 + shade.size() * 4 + plane.size() * 8 +
                              em.size() * 4);
  if (r) {
    delete s;
    return r;
  }
  *out = s;
  return RC_OK;
}

int rc_scene_destroy(rc_scene* s) {
  if (!s) return fail(RC_EINVAL, "scene is NULL");
  delete s;
  return RC_OK;
}

int rc_scene_info(const rc_scene* s, rc_scene_stats* o) {
  if (!s || !o) return fail(RC_EINVAL, "NULL argument");
  o->n_tri = s->T;
  o->n_nodes = s->n_nodes;
  o->depth = s->depth;
  o->leaf_max = rc::kLeafMax;
  o->node_bytes = 64;
  o->tri_bytes = 48;
  o->pad = s->pad;
  o->device_bytes = s->device_bytes;
  o->light_bin_bytes = s->lb.bytes;
  o->light_bin_entries = s->lb.n_entries;
  return RC_OK;
}

int64_t rc_bvh_build_host(const float* tri, int64_t T, const float box_lo[3], const float box_hi[3], float* nodes,
                          int64_t max_nodes, float* tris, rc_scene_stats* stats) {
  if (T < 0 || (T > 0 && !tri) || !box_lo || !box_hi) return fail(RC_EINVAL, "invalid arguments");
  rc::HostBvh bvh;
  std::string err;
  float pad = rc::bvh_pad_for(tri, T, box_lo, box_hi);
  int r = rc::build_bvh(tri, T, pad, bvh, err);
  if (r != RC_OK) return fail(r, "BVH build: %s", err.c_str());
  int64_t nn = (int64_t)bvh.nodes.size() / 16;
  if (nodes) {
    if (max_nodes < nn) return fail(RC_EINVAL, "max_nodes %lld < %lld", (long long)max_nodes, (long long)nn);
    std::memcpy(nodes, bvh.nodes.data(), bvh.nodes.size() * 4);
  }
  if (tris) std::memcpy(tris, bvh.tris.data(), bvh.tris.size() * 4);
  if (stats) {
    stats->n_tri = T;
    stats->n_nodes = nn;
    stats->depth = bvh.depth;
    stats->leaf_max = rc::kLeafMax;
    stats->node_bytes = 64;
    stats->tri_bytes = 48;
    stats->pad = pad;
    stats->device_bytes = 0;  // nothing uploaded
    stats->light_bin_bytes = 0;
    stats->light_bin_entries = 0;
  }
  return nn;
}

size_t rc_workspace_size(int64_t P) { return ws_bytes(std::max<int64_t>(P, 0)); }

int64_t rc_workspace_errors(const void* ws, void* stream) {
  if (!ws) return fail(RC_EINVAL, "workspace is NULL");
  unsigned int q[2];
  hipStream_t st = static_cast<hipStream_t>(stream);
  RC_HIP(hipMemcpyAsync(q, ws, sizeof q, hipMemcpyDeviceToHost, st));
  RC_HIP(hipStreamSynchronize(st));
  return (int64_t)q[1];
}

int rc_records(const rc_scene* scene, const rc_medium* medium, const rc_point_light* lights, int n_lights,
               const float* pos, const int32_t* n_theta, const int32_t* n_phi, int64_t P, const rc_params* params,
               double* value, double* grad, double* hess, void* workspace, void* stream) {
  int r = check_inputs(scene, medium, lights, n_lights, pos, n_theta, n_phi, P, params, value, grad, hess, workspace);
  if (r) return r;
  if (P == 0) return RC_OK;
  rc_scene* s = const_cast<rc_scene*>(scene);
  if (params->shadow_bvh == 0) {
    std::lock_guard<std::mutex> lk(s->mu);
    if ((r = ensure_light_bins(s, lights, n_lights, 0))) return r;
  }
  int stack, grid;
  size_t lds;
  int64_t resident = 0;
  if ((r = plan(s, params, P, 0, stack, lds, grid, &resident))) return r;
  rc::RecordArgs a = make_args(s, medium, lights, n_lights, pos, n_theta, n_phi, P, params, value, grad, hess,
                               workspace, nullptr);
  set_splits(a, params, P, resident, workspace);
  grid = (int)std::min<int64_t>(grid, P * (int64_t)a.splits);
  return launch_direct(s, a, stack, lds, grid, static_cast<hipStream_t>(stream));
}

int rc_records_noalloc(const rc_scene* scene, const rc_medium* medium, const rc_point_light* lights, int n_lights,
                       const float* pos, const int32_t* n_theta, const int32_t* n_phi, int64_t P,
                       const rc_params* params, double* value, double* grad, double* hess, void* stream) {
  if (P > RC_NOALLOC_MAX_RECORDS)
    return fail(RC_EINVAL, "rc_records_noalloc takes at most %d records (%lld given)", RC_NOALLOC_MAX_RECORDS,
                (long long)P);
  if (!scene) return fail(RC_EINVAL, "scene is NULL");
  int dev = -1;
  RC_HIP(hipGetDevice(&dev));
  if (dev != scene->device) return fail(RC_EINVAL, "scene is on device %d, current device is %d", scene->device, dev);
  void* ws = nullptr;
  int r = scratch_address(dev, &ws);
  if (r) return r;
  r = check_inputs(scene, medium, lights, n_lights, pos, n_theta, n_phi, P, params, value, grad, hess, ws);
  if (r) return r;
  if (P == 0) return RC_OK;
  rc_scene* s = const_cast<rc_scene*>(scene);
  rc_params pr = *params;
  int stack, grid;
  size_t lds;
  int64_t resident = 0;
  std::lock_guard<std::mutex> lk(s->mu);
  if (pr.shadow_bvh == 0 && n_lights > 0) {
    // light bins only if the scene already holds them for these lights
    // (building them allocates); otherwise the BVH gives the same segments
    bool same = s->lb.n == n_lights && s->lb.desc != nullptr;
    for (int l = 0; same && l < n_lights; l++) same = std::memcmp(s->lb.pos[l], lights[l].pos, sizeof(float) * 3) == 0;
    if (!same) pr.shadow_bvh = 1;
  }
  if ((r = plan(s, &pr, P, 0, stack, lds, grid, &resident))) return r;
  rc::RecordArgs a =
      make_args(s, medium, lights, n_lights, pos, n_theta, n_phi, P, &pr, value, grad, hess, ws, nullptr);
  set_splits(a, &pr, P, resident, ws);
  grid = (int)std::min<int64_t>(grid, P * (int64_t)a.splits);
  return launch_direct(s, a, stack, lds, grid, static_cast<hipStream_t>(stream));
}

int64_t rc_records_noalloc_errors(void* stream) {
  int dev = -1;
  RC_HIP(hipGetDevice(&dev));
  void* ws = nullptr;
  int r = scratch_address(dev, &ws);
  if (r) return r;
  return rc_workspace_errors(ws, stream);
}

int rc_records_batched(const rc_scene* scene, const rc_medium* medium, const rc_point_light* lights, int n_lights,
                       const float* pos, const int32_t* n_theta, const int32_t* n_phi, int64_t P,
                       const rc_params* params, const int32_t* order, int use_graph, int tile, double* value,
                       double* grad, double* hess, void* workspace, void* stream) {
  int r = check_inputs(scene, medium, lights, n_lights, pos, n_theta, n_phi, P, params, value, grad, hess, workspace);
  if (r) return r;
  if (tile < -1 || tile >= kNTiles) return fail(RC_EINVAL, "tile must be in [-1, %d)", kNTiles);
  if (P == 0) return RC_OK;
  rc_scene* s = const_cast<rc_scene*>(scene);
  if (params->shadow_bvh == 0) {
    std::lock_guard<std::mutex> lk(s->mu);
    if ((r = ensure_light_bins(s, lights, n_lights, 0))) return r;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  int stack, grid;
  size_t lds;
  int64_t resident = 0;
  bool hits = hits_mode(params);
  if (hits) {
    // the scene's hit buffer, grown to this batch; without the memory the
    // record kernel traces its own primary rays
    const int64_t stride = (int64_t)params->max_n_theta * params->max_n_phi + 2;
    const size_t need = (size_t)((P + 63) / 64) * 64 * (size_t)stride * sizeof(float2);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->hits_bytes < need) {
      s->graph.clear();  // launches captured with the old buffer
      if (s->hits) (void)hipFree(s->hits);
      s->hits = nullptr;
      s->hits_bytes = 0;
      if (hipMalloc((void**)&s->hits, need) == hipSuccess) {
        s->hits_bytes = need;
      } else {
        s->hits = nullptr;
        (void)hipGetLastError();
        hits = false;
      }
    }
  }
  if ((r = plan(s, params, P, tile, stack, lds, grid, &resident, hits))) return r;
  char* ws = static_cast<char*>(workspace);
  const int32_t* ord = order;
  unsigned int* q = reinterpret_cast<unsigned int*>(ws + kWsQueue);
  if (!ord) {
    int32_t* o = reinterpret_cast<int32_t*>(ws + kWsOrder);
    RC_HIP(rc::launch_order(n_theta, n_phi, pos, make_float3(s->box_lo[0], s->box_lo[1], s->box_lo[2]),
                            make_float3(s->box_hi[0], s->box_hi[1], s->box_hi[2]), (int)P, params->max_n_phi,
                            reinterpret_cast<unsigned int*>(ws + kWsHist), reinterpret_cast<unsigned int*>(ws + kWsCursor),
                            o, q + rc::kQueueRange, st));
    ord = o;
  }
  rc::RecordArgs a = make_args(s, medium, lights, n_lights, pos, n_theta, n_phi, P, params, value, grad, hess,
                               workspace, ord);
  set_splits(a, params, P, resident, workspace);
  a.refill_min = kTiles[tile < 0 ? 0 : tile].refill_min;
  a.leaf_batch = kTiles[tile < 0 ? 0 : tile].leaf_batch;
  a.lds_cols = lds_cols_for(params->max_n_phi, stack, params->max_rings, kTiles[tile < 0 ? 0 : tile].lds_waves);
  if (hits) {  // hits pass: every primary ray of the batch traced first, coherently
    a.hits = s->hits;
    a.hit_stride = params->max_n_theta * params->max_n_phi + 2;
    // shadow pass: the same pass walks the vertices' shadow segments
    int B = 1, shift = 0;
    while (B < n_lights) {
      B <<= 1;
      shift++;
    }
    const int words = (params->max_rings + 1 + 32 / B - 1) / (32 / B);
    if (params->shadow_pass && params->shadow_bvh == 0 && n_lights > 0 && a.lb_desc && words <= rc::kVisMaxWords) {
      const size_t need = (size_t)((P + 63) / 64) * 64 * (size_t)a.hit_stride * (size_t)words * 4;
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->vis_bytes < need) {
        s->graph.clear();
        if (s->vis) (void)hipFree(s->vis);
        s->vis = nullptr;
        s->vis_bytes = 0;
        if (hipMalloc((void**)&s->vis, need) == hipSuccess) {
          s->vis_bytes = need;
        } else {
          s->vis = nullptr;
          (void)hipGetLastError();
        }
      }
      if (s->vis) {
        a.vis = s->vis;
        a.vis_words = words;
        a.vis_shift = shift;
      }
    }
  }
  std::vector<Launch> launches;
  if (!order && a.splits == 1 && P > rc::kSplitMaxRecords) {
    // Large batches from the internal queue: one launch per n_phi class, each
    // with the LDS (and so the occupancy) its rows need; a class's launch
    // takes only its queue range and exits at once if the class is empty.
    int prev_cap = 0;
    size_t lds_max = 0;
    for (int k = 0; k < rc::kOrderClasses && prev_cap < params->max_n_phi; k++) {
      const int cap = std::min(rc::kClassCap[k], params->max_n_phi);
      rc_params pk = *params;
      pk.max_n_phi = cap;
      int sk, gk;
      size_t lk;
      int64_t rk = 0;
      if ((r = plan(s, &pk, P, tile, sk, lk, gk, &rk, hits))) return r;
      rc::RecordArgs ak = a;
      ak.max_n_phi = cap;
      ak.lds_cols = lds_cols_for(cap, stack, params->max_rings, kTiles[tile < 0 ? 0 : tile].lds_waves);
      ak.range = q + rc::kQueueRange + 2 * k;
      ak.next = q + rc::kQueueClassNext + k;
      launches.push_back(Launch{ak, gk, lk});
      lds_max = std::max(lds_max, lk);
      prev_cap = rc::kClassCap[k];
    }
    if (hipError_t e = rc::prepare_record(stack, a.counters != nullptr, a.precision == 1, lds_max))
      return fail(RC_EDEVICE, "kernel attribute: %s", hipGetErrorString(e));
  } else {
    launches.push_back(Launch{a, (int)std::min<int64_t>(grid, P * (int64_t)a.splits), lds});
  }
  if (!use_graph || st == nullptr) {
    RC_HIP(run_plan(launches, stack, st));
    return RC_OK;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  GraphCache& gc = s->graph;
  bool same = gc.valid && gc.stack == stack && gc.stream == st && gc.plan.size() == launches.size();
  for (size_t i = 0; same && i < launches.size(); i++)
    same = gc.plan[i].grid == launches[i].grid && gc.plan[i].lds == launches[i].lds &&
           std::memcmp(&gc.plan[i].args, &launches[i].args, sizeof(rc::RecordArgs)) == 0;
  if (!same) {
    gc.clear();
    RC_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t e2 = run_plan(launches, stack, st);
    hipGraph_t g = nullptr;
    hipError_t e3 = hipStreamEndCapture(st, &g);
    if (e2 != hipSuccess || e3 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(RC_EDEVICE, "graph capture failed: %s", hipGetErrorString(e2 != hipSuccess ? e2 : e3));
    }
    hipGraphExec_t ex = nullptr;
    hipError_t e4 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e4 != hipSuccess) {
      (void)hipGraphDestroy(g);
      return fail(RC_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e4));
    }
    gc.graph = g;
    gc.exec = ex;
    gc.plan = launches;
    gc.stack = stack;
    gc.stream = st;
    gc.valid = true;
  }
  RC_HIP(hipGraphLaunch(gc.exec, st));
  return RC_OK;
}

int rc_records_wait(const void* workspace, int timeout_ms, void* stream) {
  if (!workspace || timeout_ms < 0) return fail(RC_EINVAL, "workspace is NULL or timeout_ms < 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  // nothing here may wait on `stream`: no allocation of pinned memory, no
  // copy on the null stream; progress is read into pageable memory through a
  // non-blocking stream
  hipEvent_t ev = nullptr;
  hipStream_t side = nullptr;
  unsigned int hostv = 0;
  unsigned int* host = &hostv;
  auto done = [&](int code) {
    if (ev) (void)hipEventDestroy(ev);
    if (side) (void)hipStreamDestroy(side);
    return code;
  };
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess || hipEventRecord(ev, st) != hipSuccess ||
      hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess)
    return done(fail(RC_EDEVICE, "watchdog setup failed"));
  const unsigned int* progress = static_cast<const unsigned int*>(workspace) + rc::kQueueDone;
  unsigned int last = 0xffffffffu;
  auto t_last = std::chrono::steady_clock::now();
  while (true) {
    const hipError_t q = hipEventQuery(ev);
    if (q == hipSuccess) return done(RC_OK);
    if (q != hipErrorNotReady) return done(fail(RC_EDEVICE, "stream failed: %s", hipGetErrorString(q)));
    if (hipMemcpyAsync(host, progress, sizeof(unsigned int), hipMemcpyDeviceToHost, side) != hipSuccess ||
        hipStreamSynchronize(side) != hipSuccess)
      return done(fail(RC_EDEVICE, "progress read failed"));
    const auto now = std::chrono::steady_clock::now();
    if (*host != last) {
      last = *host;
      t_last = now;
    } else if (std::chrono::duration_cast<std::chrono::milliseconds>(now - t_last).count() >= timeout_ms) {
      return done(fail(RC_ETIMEOUT, "no record finished for %d ms (%u finished)", timeout_ms, last));
    }
    std::this_thread::sleep_for(std::chrono::microseconds(500));
  }
}

int rc_tile_info(int tile, float* grid, int* refill_min, int* leaf_batch, int* lds_waves) {
  if (tile < 0 || tile >= kNTiles) return fail(RC_EINVAL, "tile must be in [0, %d)", kNTiles);
  if (!grid || !refill_min || !leaf_batch || !lds_waves) return fail(RC_EINVAL, "NULL output");
  *grid = kTiles[tile].grid;
  *refill_min = kTiles[tile].refill_min;
  *leaf_batch = kTiles[tile].leaf_batch;
  *lds_waves = kTiles[tile].lds_waves;
  return RC_OK;
}

int rc_autotune(const rc_scene* scene, const rc_medium* medium, const rc_point_light* lights, int n_lights,
                const float* pos, const int32_t* n_theta, const int32_t* n_phi, int64_t P, const rc_params* params,
                double* value, double* grad, double* hess, void* workspace, const char* cache_path, int* best_tile,
                float* ms_out, int* n_tiles, void* stream) {
  int r = check_inputs(scene, medium, lights, n_lights, pos, n_theta, n_phi, P, params, value, grad, hess, workspace);
  if (r) return r;
  if (!best_tile) return fail(RC_EINVAL, "best_tile is NULL");
  if (n_tiles) *n_tiles = kNTiles;
  *best_tile = 0;
  if (P == 0) return RC_OK;
  const rc_scene* s = scene;
  std::ostringstream key;
  key << s->arch << "|T=" << s->T << "|P=" << P << "|nphi=" << params->max_n_phi << "|rings=" << params->max_rings
      << "|L=" << n_lights;
  if (cache_path && !ms_out) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      auto p = line.rfind(' ');
      if (p != std::string::npos && line.substr(0, p) == key.str()) {
        int t = std::atoi(line.c_str() + p + 1);
        if (t >= 0 && t < kNTiles) {
          *best_tile = t;
          return RC_OK;
        }
      }
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  RC_HIP(hipEventCreate(&e0));
  RC_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  for (int t = 0; t < kNTiles; t++) {
    float tot = 0.f;
    for (int rep = 0; rep < 3; rep++) {
      RC_HIP(hipEventRecord(e0, st));
      r = rc_records_batched(scene, medium, lights, n_lights, pos, n_theta, n_phi, P, params, nullptr, 0, t, value,
                             grad, hess, workspace, stream);
      if (r) return r;
      RC_HIP(hipEventRecord(e1, st));
      RC_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      RC_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) tot += ms;  // first repetition warms up
    }
    tot *= 0.5f;
    if (ms_out) ms_out[t] = tot;
    if (tot < best) {
      best = tot;
      *best_tile = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (cache_path) {
    std::ofstream out(cache_path, std::ios::app);
    out << key.str() << " " << *best_tile << "\n";
  }
  return RC_OK;
}

int rc_radius(const double* value, const double* hess, int64_t P, float eps, float r_min, float r_max, float* R,
              float* axes, void* stream) {
  if (P < 0 || P > 0x7fffffff) return fail(RC_EINVAL, "P out of range");
  if (P > 0 && (!value || !hess || !R)) return fail(RC_EINVAL, "NULL pointer");
  if (!(eps > 0.f) || !(r_min > 0.f) || !(r_max >= r_min) || !std::isfinite(r_max))
    return fail(RC_EINVAL, "need eps > 0 and 0 < r_min <= r_max");
  if (P == 0) return RC_OK;
  RC_HIP(rc::launch_radius(value, hess, (int)P, eps, r_min, r_max, R, axes, static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_trace_rays(const rc_scene* s, const float* orig, const float* dir, int64_t n, int32_t* hit_id, float* t,
                  int32_t* front, void* stream) {
  if (!s || n < 0 || n > 0x7fffffff) return fail(RC_EINVAL, "invalid arguments");
  if (n > 0 && (!orig || !dir || !hit_id || !t || !front)) return fail(RC_EINVAL, "NULL pointer");
  RC_HIP(rc::launch_trace_rays(s->nodes, s->tris, s->tri_stride, s->depth, orig, dir, (int)n, hit_id, t, front,
                               make_float3(s->box_lo[0], s->box_lo[1], s->box_lo[2]),
                               make_float3(s->box_hi[0], s->box_hi[1], s->box_hi[2]), static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_occluded_rays(const rc_scene* s, const float* orig, const float* seg, const int32_t* skip, int64_t n,
                     int32_t* occ, void* stream) {
  if (!s || n < 0 || n > 0x7fffffff) return fail(RC_EINVAL, "invalid arguments");
  if (n > 0 && (!orig || !seg || !occ)) return fail(RC_EINVAL, "NULL pointer");
  RC_HIP(rc::launch_occluded_rays(s->nodes, s->tris, s->tri_stride, s->depth, orig, seg, skip, (int)n, occ,
                                  static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_light_bins_build(rc_scene* s, const rc_point_light* lights, int n_lights, int B) {
  if (!s) return fail(RC_EINVAL, "scene is NULL");
  if (n_lights < 1 || n_lights > RC_MAX_LIGHTS || !lights) return fail(RC_EINVAL, "n_lights must be in [1, %d]", RC_MAX_LIGHTS);
  for (int l = 0; l < n_lights; l++)
    if (!finite3(lights[l].pos)) return fail(RC_EINVAL, "light %d is not finite", l);
  if (B != 0 && (B < 2 || B > 4096 || (B & (B - 1)))) return fail(RC_EINVAL, "B must be 0 or a power of two in [2, 4096]");
  std::lock_guard<std::mutex> lk(s->mu);
  if (B != 0) s->lb.n = 0;  // explicit size: always rebuild
  return ensure_light_bins(s, lights, n_lights, B);
}

int rc_light_occluded(const rc_scene* s, int light, const float* pts, const int32_t* skip, int64_t n, int32_t* occ,
                      void* stream) {
  if (!s || n < 0 || n > 0x7fffffff) return fail(RC_EINVAL, "invalid arguments");
  if (!s->lb.desc || light < 0 || light >= s->lb.n) return fail(RC_EINVAL, "no light bins for light %d", light);
  if (n > 0 && (!pts || !occ)) return fail(RC_EINVAL, "NULL pointer");
  const float4 L = make_float4(s->lb.pos[light][0], s->lb.pos[light][1], s->lb.pos[light][2], 0.f);
  RC_HIP(rc::launch_light_occluded(s->lb.desc, s->lb.offs, s->lb.ent, light, L, pts, skip, (int)n, occ,
                                   static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int64_t rc_light_bins_host(const float* tri, int64_t T, const float box_lo[3], const float box_hi[3],
                           const float light[3], int B, int* B_out, int* levels, int64_t* level_off, int32_t* offs,
                           int64_t cap_offs, int64_t* n_offs, float* entries, int64_t cap_entries) {
  if (T < 0 || (T > 0 && !tri) || !box_lo || !box_hi || !light || !finite3(light))
    return fail(RC_EINVAL, "invalid arguments");
  if (B != 0 && (B < 2 || B > 4096 || (B & (B - 1)))) return fail(RC_EINVAL, "B must be 0 or a power of two in [2, 4096]");
  rc::LightBinsHost h;
  std::string err;
  const float scale = rc::bvh_pad_for(tri, T, box_lo, box_hi);
  int r = rc::build_light_bins(tri, T, scale, light, B ? B : rc::light_bins_size_for(T), h, err);
  if (r != RC_OK) return fail(r, "%s", err.c_str());
  const int64_t ne = (int64_t)(h.entries.size() / 12), no = (int64_t)h.offs.size();
  if (B_out) *B_out = h.B;
  if (levels) *levels = h.nlev;
  if (level_off)
    for (int k = 0; k < rc::kLbMaxLevels; k++) level_off[k] = k < h.nlev ? h.lev_off[k] : 0;
  if (n_offs) *n_offs = no;
  if (offs && cap_offs >= no) std::memcpy(offs, h.offs.data(), (size_t)no * 4);
  if (entries && cap_entries >= ne) std::memcpy(entries, h.entries.data(), (size_t)ne * 48);
  return ne;
}

/* ------------------------------------------------------------------ */
/* Learned placement                                                    */
/* ------------------------------------------------------------------ */
int rc_probe(const rc_scene* s, const rc_medium* m, const rc_point_light* lights, int n_lights, const float* cand,
             int64_t C, uint64_t seed, int64_t id_base, int common_random, float* feat32, uint16_t* feat_bf16,
             void* stream) {
  if (!s) return fail(RC_EINVAL, "scene is NULL");
  if (!m || !std::isfinite(m->sigma_s) || !std::isfinite(m->sigma_a) || m->sigma_s < 0 || m->sigma_a < 0)
    return fail(RC_EINVAL, "medium coefficients must be finite and >= 0");
  if (n_lights < 0 || n_lights > RC_MAX_LIGHTS || (n_lights > 0 && !lights)) return fail(RC_EINVAL, "bad lights");
  if (C < 0 || C > 0x7fffffff || id_base < 0) return fail(RC_EINVAL, "C or id_base out of range");
  if (common_random != 0 && common_random != 1) return fail(RC_EINVAL, "common_random must be 0 or 1");
  if (C > 0 && (!cand || (!feat32 && !feat_bf16))) return fail(RC_EINVAL, "NULL candidate or feature pointer");
  if (C == 0) return RC_OK;
  rc::ProbeArgs a;
  std::memset(&a, 0, sizeof a);
  a.nodes = s->nodes;
  a.tris = s->tris;
  a.tri_stride = s->tri_stride;
  a.shade = s->shade;
  a.emission = s->emission;
  a.box_lo = make_float3(s->box_lo[0], s->box_lo[1], s->box_lo[2]);
  a.box_hi = make_float3(s->box_hi[0], s->box_hi[1], s->box_hi[2]);
  a.n_lights = n_lights;
  for (int l = 0; l < n_lights; l++)
    a.lights[l] = make_float4(lights[l].pos[0], lights[l].pos[1], lights[l].pos[2], lights[l].intensity);
  a.sigma_s = m->sigma_s;
  a.sigma_a = m->sigma_a;
  a.cand = cand;
  a.C = (int)C;
  a.seed = seed;
  a.id_base = id_base;
  a.common_random = common_random;
  a.feat32 = feat32;
  a.feat16 = reinterpret_cast<__bf16*>(feat_bf16);
  if (n_lights > 0) {  // shadow segments from the light bins of these lights
    rc_scene* sm = const_cast<rc_scene*>(s);
    std::lock_guard<std::mutex> lk(sm->mu);
    int r = ensure_light_bins(sm, lights, n_lights, 0);
    if (r) return r;
    a.lb_desc = sm->lb.desc;
    a.lb_offs = sm->lb.offs;
    a.lb_ent = sm->lb.ent;
  }
  RC_HIP(rc::launch_probe(a, s->depth, static_cast<hipStream_t>(stream)));
  return RC_OK;
}

// sample counts of the MLP calls (grid-stride loops index samples with int)
constexpr int64_t kMlpMaxSamples = int64_t(1) << 30;

size_t rc_mlp_param_bytes(void) { return rc::kMlpParamBytes; }
int64_t rc_mlp_n_params(void) { return rc::kMlpGradFloats; }
size_t rc_mlp_train_workspace_bytes(int64_t n) {
  const int64_t tiles = (std::max<int64_t>(n, 1) + 63) / 64;
  return (size_t)tiles * rc::kMlpGradFloats * sizeof(float);
}

int rc_mlp_init(void* params, float* state, uint64_t seed, void* stream) {
  if (!params || !state) return fail(RC_EINVAL, "NULL pointer");
  RC_HIP(rc::launch_mlp_init(params, state, seed, static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_mlp_load(void* params, const float* state, void* stream) {
  if (!params || !state) return fail(RC_EINVAL, "NULL pointer");
  RC_HIP(rc::launch_mlp_sync(params, state, static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_mlp_fit_features(void* params, const float* X, int64_t n, void* workspace, void* stream) {
  if (!params || (n > 0 && (!X || !workspace))) return fail(RC_EINVAL, "NULL pointer");
  if (n < 2 || n > kMlpMaxSamples) return fail(RC_EINVAL, "need 2 <= n <= 2^30 samples");
  RC_HIP(rc::launch_feature_stats(X, (int)n, static_cast<float*>(workspace), 256, params,
                                  static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_mlp_forward(const void* params, const float* X, int64_t n, float* out, void* stream) {
  if (!params || n < 0 || n > kMlpMaxSamples || (n > 0 && (!X || !out))) return fail(RC_EINVAL, "invalid arguments");
  RC_HIP(rc::launch_mlp_forward(params, X, (int)n, out, static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_mlp_radius(const void* params, const float* X, int64_t n, float safety, float r_min, float r_max, float* R,
                  void* stream) {
  if (!params || n < 0 || n > kMlpMaxSamples || (n > 0 && (!X || !R))) return fail(RC_EINVAL, "invalid arguments");
  if (!(safety > 0.f) || !std::isfinite(safety) || !(r_min > 0.f) || !(r_max >= r_min) || !std::isfinite(r_max))
    return fail(RC_EINVAL, "need safety > 0 and 0 < r_min <= r_max finite");
  RC_HIP(rc::launch_mlp_radius(params, X, (int)n, safety, r_min, r_max, R, static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_mlp_train_step(void* params, float* state, const float* X, const float* target, int64_t n, float lr,
                      int64_t step, void* workspace, float* loss, float* grad, void* stream) {
  if (!params || !state || !X || !target || !workspace) return fail(RC_EINVAL, "NULL pointer");
  if (n < 1 || n > kMlpMaxSamples || !(lr >= 0.f) || step < 1)
    return fail(RC_EINVAL, "need 1 <= n <= 2^30, lr >= 0, step >= 1");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int tiles = (int)((n + 63) / 64);
  float* partial = static_cast<float*>(workspace);
  RC_HIP(rc::launch_mlp_grad(params, X, target, (int)n, partial, st));
  const float b1c = (float)(1.0 - std::pow(0.9, (double)step));
  const float b2c = (float)(1.0 - std::pow(0.999, (double)step));
  RC_HIP(rc::launch_mlp_adam(params, state, state + rc::kMlpGradFloats, state + 2 * rc::kMlpGradFloats, partial,
                             tiles, lr, b1c, b2c, grad, loss, st));
  return RC_OK;
}

int rc_place_gather(const float* cand, const float* radius, const int32_t* order, int64_t C, const uint8_t* covered,
                    int32_t* state, int32_t* batch_idx, float* batch_pos, float* batch_R, int batch, void* stream) {
  if (C < 0 || C > 0x7fffffff || batch < 1 || batch > rc::kPlaceMaxBatch)
    return fail(RC_EINVAL, "C out of range or batch not in [1, %d]", rc::kPlaceMaxBatch);
  if (!cand || !covered || !state || !batch_idx || !batch_pos || (radius && !batch_R))
    return fail(RC_EINVAL, "NULL pointer");
  RC_HIP(rc::launch_place_gather(cand, radius, order, (int)C, covered, state, batch_idx, batch_pos, batch_R, batch,
                                 static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_place_accept(const float* cand, const int32_t* batch_idx, const float* batch_R, uint8_t* covered,
                    int32_t* state, int32_t* accepted, float* accepted_R, float* accepted_pos,
                    const double* batch_value, const double* batch_grad, double* cache_value, double* cache_grad,
                    const float* batch_form, float* accepted_form, void* stream) {
  if (!cand || !batch_idx || !batch_R || !covered || !state || !accepted || !accepted_R)
    return fail(RC_EINVAL, "NULL pointer");
  if (!batch_form != !accepted_form) return fail(RC_EINVAL, "batch_form and accepted_form: both or neither");
  const bool any = batch_value || batch_grad || cache_value || cache_grad;
  const bool all = batch_value && batch_grad && cache_value && cache_grad;
  if (any && !all) return fail(RC_EINVAL, "batch_value, batch_grad, cache_value, cache_grad: all or none");
  RC_HIP(rc::launch_place_accept(cand, batch_idx, batch_R, batch_form, covered, state, accepted, accepted_R,
                                 accepted_form, accepted_pos, batch_value, batch_grad, cache_value, cache_grad,
                                 static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_place_cover(const float* cand, int64_t C, uint8_t* covered, const int32_t* state, const int32_t* accepted,
                   const float* accepted_R, int64_t first, int64_t count, const float* accepted_form, void* stream) {
  if (C < 0 || C > 0x7fffffff || !cand || !covered || !accepted || !accepted_R || (first < 0 && !state))
    return fail(RC_EINVAL, "invalid arguments");
  if (first > 0x7fffffff || count < 0 || count > 0x7fffffff) return fail(RC_EINVAL, "first/count out of range");
  RC_HIP(rc::launch_place_cover(cand, (int)C, covered, state, accepted, accepted_R, accepted_form, (int)first,
                                (int)count, static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_place_cover_grid(const float* cand, const int32_t dims[3], const float lo[3], const float cell[3],
                        uint8_t* covered, const int32_t* state, const int32_t* accepted, const float* accepted_R,
                        int64_t first, int64_t count, const float* accepted_form, void* stream) {
  if (!cand || !dims || !lo || !cell || !covered || !accepted || !accepted_R || (first < 0 && !state))
    return fail(RC_EINVAL, "NULL pointer");
  if (first > 0x7fffffff || count < 0 || count > 0x7fffffff) return fail(RC_EINVAL, "first/count out of range");
  int64_t cells = 1;
  for (int d = 0; d < 3; d++) {
    if (dims[d] < 1) return fail(RC_EINVAL, "grid dimensions must be >= 1");
    if (!(cell[d] > 0.f) || !std::isfinite(cell[d]) || !std::isfinite(lo[d]))
      return fail(RC_EINVAL, "grid origin and cell size must be finite, cell > 0");
    cells *= dims[d];
  }
  if (cells > 0x7fffffff) return fail(RC_EINVAL, "grid has more than 2^31 - 1 cells");
  rc::PlaceGrid g;
  g.nx = dims[0];
  g.ny = dims[1];
  g.nz = dims[2];
  g.lo = make_float3(lo[0], lo[1], lo[2]);
  g.inv_h = make_float3(1.f / cell[0], 1.f / cell[1], 1.f / cell[2]);
  RC_HIP(rc::launch_place_cover_grid(cand, g, covered, state, accepted, accepted_R, accepted_form, (int)first,
                                     (int)count, rc::kPlaceMaxBatch, static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_interp(const float* cache_pos, const double* cache_value, const double* cache_grad, const float* cache_R,
              int64_t K, const float* query, int64_t Q, double* out, int32_t* hits, const double* ref_value,
              double* err_partial, const float* cache_form, void* stream) {
  if (K < 0 || K > 0x7fffffff || Q < 0 || Q > 0x7fffffff) return fail(RC_EINVAL, "K or Q out of range");
  if ((K > 0 && (!cache_pos || !cache_value || !cache_grad || !cache_R)) || (Q > 0 && (!query || !out)) ||
      (ref_value && !err_partial))
    return fail(RC_EINVAL, "NULL pointer");
  RC_HIP(rc::launch_interp(cache_pos, cache_value, cache_grad, cache_R, cache_form, (int)K, query, (int)Q, out, hits,
                           ref_value, err_partial, static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_interp_log(const float* cache_pos, const double* cache_value, const double* cache_grad, const float* cache_R,
                  int64_t K, const float* query, int64_t Q, double* out, int32_t* hits, void* stream) {
  if (K < 0 || K > 0x7fffffff || Q < 0 || Q > 0x7fffffff) return fail(RC_EINVAL, "K or Q out of range");
  if ((K > 0 && (!cache_pos || !cache_value || !cache_grad || !cache_R)) || (Q > 0 && (!query || !out)))
    return fail(RC_EINVAL, "NULL pointer");
  RC_HIP(rc::launch_interp_log(cache_pos, cache_value, cache_grad, cache_R, (int)K, query, (int)Q, out, hits,
                               static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_ellipsoid_form(const float* axes, int64_t K, float* form, float* r_max, void* stream) {
  if (K < 0 || K > 0x7fffffff) return fail(RC_EINVAL, "K out of range");
  if (K > 0 && (!axes || !form)) return fail(RC_EINVAL, "NULL pointer");
  RC_HIP(rc::launch_ellipsoid_form(axes, (int)K, form, r_max, static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_march_count(const rc_scene* s, const float* orig, const float* dir, const float* xi, int64_t n, double step,
                   float* t_end, int64_t* offsets, void* stream) {
  if (!s || n < 0 || n > 0x7fffffff) return fail(RC_EINVAL, "invalid arguments");
  if (!offsets || (n > 0 && (!orig || !dir || !xi || !t_end))) return fail(RC_EINVAL, "NULL pointer");
  double diag = 0.0;
  for (int a = 0; a < 3; a++) diag += ((double)s->box_hi[a] - s->box_lo[a]) * ((double)s->box_hi[a] - s->box_lo[a]);
  diag = std::sqrt(diag);
  if (!(step > 0.0) || !std::isfinite(step) || diag / step > (double)RC_MARCH_MAX_POINTS_PER_RAY)
    return fail(RC_EINVAL, "step must be positive with box diagonal / step <= %d", RC_MARCH_MAX_POINTS_PER_RAY);
  RC_HIP(rc::launch_march_count(s->nodes, s->tris, s->tri_stride, s->depth, orig, dir, xi, (int)n, step,
                                make_float3(s->box_lo[0], s->box_lo[1], s->box_lo[2]),
                                make_float3(s->box_hi[0], s->box_hi[1], s->box_hi[2]), t_end,
                                reinterpret_cast<long long*>(offsets), static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_march_emit(const float* orig, const float* dir, const float* xi, int64_t n, double step, double sigma_s,
                  double sigma_t, const int64_t* offsets, float* points, double* weight, void* stream) {
  if (n < 0 || n > 0x7fffffff) return fail(RC_EINVAL, "n out of range");
  if (!(step > 0.0) || !std::isfinite(step) || !std::isfinite(sigma_s) || !std::isfinite(sigma_t) || sigma_s < 0 ||
      sigma_t < 0)
    return fail(RC_EINVAL, "step must be positive and the coefficients finite and non-negative");
  if (n > 0 && (!orig || !dir || !xi || !offsets || !points || !weight)) return fail(RC_EINVAL, "NULL pointer");
  RC_HIP(rc::launch_march_emit(orig, dir, xi, (int)n, step, sigma_s, sigma_t,
                               reinterpret_cast<const long long*>(offsets), points, weight,
                               static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_composite(const int64_t* offsets, int64_t n_rays, int32_t spp, const double* weight, const double* L,
                 double* pixel, void* stream) {
  if (n_rays < 0 || n_rays > 0x7fffffff || spp < 1 || n_rays % spp != 0)
    return fail(RC_EINVAL, "n_rays must be a non-negative multiple of spp >= 1");
  if (n_rays > 0 && (!offsets || !pixel)) return fail(RC_EINVAL, "NULL pointer");
  RC_HIP(rc::launch_composite(reinterpret_cast<const long long*>(offsets), (int)(n_rays / spp), spp, weight, L, pixel,
                              static_cast<hipStream_t>(stream)));
  return RC_OK;
}

int rc_j08_records(const rc_scene* s, const rc_medium* m, const rc_point_light* lights, int n_lights,
                   const float* pos, const int32_t* n_theta, const int32_t* n_phi, int64_t P, const rc_params* params,
                   float eps, float r_min, float r_max, double* value, double* grad, double* moments, float* R,
                   void* stream) {
  if (!s) return fail(RC_EINVAL, "scene is NULL");
  if (!m || !std::isfinite(m->sigma_s) || !std::isfinite(m->sigma_a) || m->sigma_s < 0 || m->sigma_a < 0)
    return fail(RC_EINVAL, "medium coefficients must be finite and >= 0");
  if (n_lights < 0 || n_lights > RC_MAX_LIGHTS || (n_lights > 0 && !lights)) return fail(RC_EINVAL, "bad lights");
  if (!params || !(params->ring_step > 0.f) || params->max_rings < 0 || params->max_rings > RC_MAX_RINGS ||
      params->rec_base < 0 || (params->common_random != 0 && params->common_random != 1))
    return fail(RC_EINVAL, "bad params");
  if (!(eps > 0.f) || !(r_min > 0.f) || !(r_max >= r_min) || !std::isfinite(r_max))
    return fail(RC_EINVAL, "need eps > 0 and 0 < r_min <= r_max finite");
  if (P < 0 || P > 0x7fffffff) return fail(RC_EINVAL, "P out of range");
  if (P > 0 && (!pos || !n_theta || !n_phi || !value || !grad || !moments || !R)) return fail(RC_EINVAL, "NULL pointer");
  if (P == 0) return RC_OK;
  rc::J08Args a;
  std::memset(&a, 0, sizeof a);
  a.nodes = s->nodes;
  a.tris = s->tris;
  a.tri_stride = s->tri_stride;
  a.shade = s->shade;
  a.emission = s->emission;
  a.box_lo = make_float3(s->box_lo[0], s->box_lo[1], s->box_lo[2]);
  a.box_hi = make_float3(s->box_hi[0], s->box_hi[1], s->box_hi[2]);
  a.n_lights = n_lights;
  for (int l = 0; l < n_lights; l++)
    a.lights[l] = make_float4(lights[l].pos[0], lights[l].pos[1], lights[l].pos[2], lights[l].intensity);
  a.sigma_s = m->sigma_s;
  a.sigma_a = m->sigma_a;
  a.ring_step = params->ring_step;
  a.max_rings = params->max_rings;
  a.seed = params->seed;
  a.rec_base = params->rec_base;
  a.common_random = params->common_random;
  a.pos = pos;
  a.n_theta = n_theta;
  a.n_phi = n_phi;
  a.P = (int)P;
  a.eps = eps;
  a.r_min = r_min;
  a.r_max = r_max;
  a.value = value;
  a.grad = grad;
  a.moments = moments;
  a.R = R;
  if (n_lights > 0) {  // shadow segments from the light bins of these lights
    rc_scene* sm = const_cast<rc_scene*>(s);
    std::lock_guard<std::mutex> lk(sm->mu);
    int r = ensure_light_bins(sm, lights, n_lights, 0);
    if (r) return r;
    a.lb_desc = sm->lb.desc;
    a.lb_offs = sm->lb.offs;
    a.lb_ent = sm->lb.ent;
  }
  RC_HIP(rc::launch_j08(a, s->depth, static_cast<hipStream_t>(stream)));
  return RC_OK;
}

}  // extern "C"
