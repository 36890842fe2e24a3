// kernels.hpp -- launch interface between the host API and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "limits.hpp"
#include "rc.h"

namespace rc {

// Device-built queue: records grouped by n_phi class (widest first), then by
// cost (octaves of N = n_theta * n_phi, largest first), then by cell of an
// 8x8x8 grid over the medium box in Morton order, so that the records in
// flight at any time lie close together and share the caches.
constexpr int kOrderClasses = 5;  // n_phi classes: <= 16, 32, 64, 128, 256
constexpr int kClassCap[kOrderClasses] = {16, 32, 64, 128, 256};
constexpr int kOrderCost = 16;    // cost buckets (octaves of N)
constexpr int kOrderCells = 512;  // Morton cells (8 x 8 x 8)
constexpr int kOrderGroup = kOrderCost * kOrderCells;            // buckets of one class
constexpr int kOrderBuckets = kOrderClasses * kOrderGroup;       // 40960
constexpr int kOrderScanThreads = 1024;
static_assert(kOrderBuckets % kOrderScanThreads == 0, "order scan chunks");
// workspace queue words: [0] pop counter of a single launch, [1] invalid
// records, [2..6] pop counter of each class launch, [8] records finished
// (progress, read by the host watchdog), [16..25] queue range [lo, hi) of each class
constexpr int kQueueWords = 64;
constexpr int kQueueClassNext = 2;
constexpr int kQueueDone = 8;
constexpr int kQueueRange = 16;
// LDS stack of the record kernel when its primary rays come from the hits
// pass and its shadow segments from the light bins: only the bin lists of a
// segment (two words per level) use it
constexpr int kHitsStack = 2 * kLbMaxLevels;

struct RecordArgs {
  const float4* nodes;
  const float4* tris;      // three copies of the triangle records, copy k permuted for kz = k
  int tri_stride;          // float4 words per copy
  const float4* shade;     // per triangle: unit normal (xyz), albedo (w)
  const double4* plane;    // per triangle: FP64 unit normal (xyz), normal . v0 (w)
  const float* emission;   // per triangle
  float3 box_lo, box_hi;
  int n_lights;
  float4 lights[RC_MAX_LIGHTS];
  float sigma_s, sigma_a;
  const float* pos;
  const int* n_theta;
  const int* n_phi;
  int P;
  long long rec_base;
  int common_random;       // 1: every record draws with id rec_base
  float ring_step;
  int max_rings;
  int max_n_phi;           // largest n_phi accepted (records above it are invalid)
  int lds_cols;            // columns of an LDS row (wider rows are done in sectors)
  int precision;
  unsigned long long seed;
  double* value;
  double* grad;
  double* hess;
  const int* order;        // queue order or nullptr (identity)
  unsigned int* queue;     // queue words (kQueueWords): [1] invalid records, progress, ranges, counters
  // shadow segments from light bins (nullptr: BVH traversal): per light two
  // int4 (B, levels, level offsets 0..3), the bin offsets (CSR over levels,
  // faces, bins) and the entries (3 float4: permuted vertices, id bits,
  // stored distance from the light)
  const int4* lb_desc;
  const int* lb_offs;
  const float4* lb_ent;
  int splits;              // wavefronts per record (each owns a range of rows)
  int refill_min;          // shadow loop: idle lanes that trigger a refill
  int leaf_batch;          // traversal: lanes waiting at a leaf that trigger a triangle step
  double* partial;         // [P][splits][20] partial sums (splits > 1)
  unsigned int* done;      // [P] parts finished (splits > 1; zero before launch)
  const unsigned int* range;  // device [lo, hi): queue slots of this launch, or nullptr (all)
  unsigned int* next;         // pop counter of this launch
  unsigned long long* counters;
  // primary hits traced by primary_kernel (or nullptr: the record kernel
  // traces them): (t, code bits) of direction d of the record at queue slot
  // q at hits[((q / 64) * hit_stride + d) * 64 + q % 64]; d = 0 north pole,
  // 1 + a * n_phi + col stratum (a, col), N + 1 south pole
  float2* hits;
  int hit_stride;             // max_n_theta * max_n_phi + 2
  int max_n_theta;            // records above it are invalid (with hits)
  int trace_stack;            // traversal stack of the BVH (primary_kernel)
  // visibility bits of every vertex of every primary ray, walked by
  // primary_kernel (or nullptr): word w of ray (q, d) at
  // vis[(((q / 64) * hit_stride + d) * vis_words + w) * 64 + q % 64]; vertex
  // kk (0 the surface vertex, 1 + i ring i) holds its light bits at bit
  // kk << vis_shift of the ray's words
  unsigned int* vis;
  int vis_words, vis_shift;
};
constexpr int kVisMaxWords = 4;

int stack_variant(int depth);
size_t record_lds_bytes(int stack, int max_n_phi, int max_rings);
// Resident wavefronts per SIMD the record kernel is compiled for: 4 (128
// VGPRs) with a traversal stack of up to 24 entries, else 3 (168 VGPRs; a
// deeper stack takes too much LDS for 16 wavefronts per CU to keep useful
// row widths).  The LDS row width is chosen for the same occupancy.
constexpr int record_waves_per_simd(int stack) { return stack <= 24 ? 4 : 3; }
int record_occupancy(int stack, bool count, bool f64, size_t lds);
hipError_t prepare_record(int stack, bool count, bool f64, size_t lds);
hipError_t launch_record(const RecordArgs& a, int stack, bool count, bool f64, int grid, size_t lds, hipStream_t s);
hipError_t launch_reset(unsigned int* q, hipStream_t s);
// primary hits of queue slots [0, nq) into a.hits (every direction of every record)
hipError_t launch_primary(const RecordArgs& a, int stack, int nq, hipStream_t s);
hipError_t launch_zero_u32(unsigned int* p, int n, hipStream_t s);
constexpr int kMaxSplits = 8;        // wavefronts per record at most
constexpr int kSplitMaxRecords = 16384;  // batches up to this size may split records
hipError_t launch_order(const int* nth, const int* nph, const float* pos, float3 box_lo, float3 box_hi, int P,
                        int max_nph, unsigned int* hist, unsigned int* cursor, int* order, unsigned int* class_range,
                        hipStream_t s);
hipError_t launch_radius(const double* value, const double* hess, int P, float eps, float r_min, float r_max, float* R,
                         float* axes, hipStream_t s);

hipError_t launch_light_occluded(const int4* desc, const int* offs, const float4* ent, int l, float4 L,
                                 const float* pts, const int* skip, int n, int* occ, hipStream_t s);
hipError_t launch_trace_rays(const float4* nodes, const float4* tris, int tri_stride, int depth, const float* o,
                             const float* d, int n,
                             int* hit, float* t, int* front, float3 lo, float3 hi, hipStream_t s);
hipError_t launch_occluded_rays(const float4* nodes, const float4* tris, int tri_stride, int depth, const float* o,
                                const float* d,
                                const int* skip, int n, int* occ, hipStream_t s);

}  // namespace rc
