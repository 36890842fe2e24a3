// learned.hpp -- launch interface of the learned-placement kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rc.h"

namespace rc {

// parameter block: FP32 section (floats) then BF16 W1 [128][32], W2 [128][128], W2^T [128][128]
constexpr int kMlpShift = 0, kMlpScale = 32, kMlpB1 = 64, kMlpB2 = 192, kMlpW3 = 320, kMlpB3 = 448;
constexpr int kMlpFloats = 464;  // padded so the BF16 section is 16-byte aligned
constexpr size_t kMlpParamBytes = kMlpFloats * 4 + (size_t)(128 * 32 + 2 * 128 * 128) * 2;
// gradient / master-weight layout (floats)
constexpr int kGradW1 = 0, kGradB1 = 4096, kGradW2 = 4224, kGradB2 = 20608, kGradW3 = 20736, kGradB3 = 20864,
              kGradLoss = 20865;
constexpr int kMlpGradFloats = 20866;

constexpr int kPlaceMaxBatch = 4096;  // candidates gathered / decided per round
constexpr int kPlaceThreads = 1024;   // one workgroup for gather and accept
constexpr int kPlaceStatus = 5;       // state[5 + j]: batch entry j undecided (0), accepted (1), rejected (2)
constexpr int kPlacePasses = 3;       // wide resolve passes before the final one-workgroup pass
constexpr int kPlaceResolveThreads = 1024;  // 16 waves per resolve workgroup, one batch entry each
static_assert(RC_PLACE_STATE_INTS == kPlaceStatus + kPlaceMaxBatch, "placement state layout");

// cell grid of grid candidates: index (ix * ny + iy) * nz + iz
struct PlaceGrid {
  int nx, ny, nz;
  float3 lo, inv_h;
};

struct ProbeArgs {
  const float4* nodes;
  const float4* tris;      // three copies, copy k permuted for kz = k
  int tri_stride;          // float4 words per copy
  const float4* shade;
  const float* emission;
  float3 box_lo, box_hi;
  int n_lights;
  float4 lights[RC_MAX_LIGHTS];
  float sigma_s, sigma_a;
  const float* cand;
  int C;
  unsigned long long seed;
  long long id_base;
  int common_random;  // 1: every candidate draws with id id_base
  float* feat32;
  __bf16* feat16;
  // light bins of these lights (shadow segments from the bins), or nullptr
  // (BVH traversal); both give the answer of testing every triangle
  const int4* lb_desc;
  const int* lb_offs;
  const float4* lb_ent;
};

int stack_variant(int depth);
hipError_t launch_probe(const ProbeArgs& a, int depth, hipStream_t s);
hipError_t launch_mlp_forward(const void* params, const float* X, int n, float* out, hipStream_t s);
hipError_t launch_mlp_radius(const void* params, const float* X, int n, float safety, float r_min, float r_max,
                             float* R, hipStream_t s);
hipError_t launch_mlp_grad(const void* params, const float* X, const float* target, int n, float* partial,
                           hipStream_t s);
hipError_t launch_mlp_adam(void* params, float* master, float* m, float* v, const float* partial, int tiles, float lr,
                           float b1c, float b2c, float* grad_out, float* loss_out, hipStream_t s);
hipError_t launch_feature_stats(const float* X, int n, float* partial, int blocks, void* params, hipStream_t s);
hipError_t launch_place_gather(const float* cand, const float* radius, const int* order, int C,
                               const unsigned char* covered, int* state, int* batch_idx, float* batch_pos,
                               float* batch_R, int batch, hipStream_t s);
hipError_t launch_place_accept(const float* cand, const int* batch_idx, const float* batch_R, const float* batch_form,
                               unsigned char* covered, int* state, int* accepted, float* accepted_R,
                               float* accepted_form, float* accepted_pos, const double* bval, const double* bgrad,
                               double* cval, double* cgrad, hipStream_t s);
hipError_t launch_place_cover(const float* cand, int C, unsigned char* covered, const int* state, const int* accepted,
                              const float* accepted_R, const float* accepted_form, int first, int count,
                              hipStream_t s);
hipError_t launch_place_cover_grid(const float* cand, const PlaceGrid& g, unsigned char* covered, const int* state,
                                   const int* accepted, const float* accepted_R, const float* accepted_form, int first,
                                   int count, int max_points, hipStream_t s);
hipError_t launch_interp(const float* cpos, const double* cval, const double* cgrad, const float* cR,
                         const float* cform, int K, const float* q, int Q, double* out, int* hits, const double* ref,
                         double* err, hipStream_t s);
hipError_t launch_interp_log(const float* cpos, const double* cval, const double* cgrad, const float* cR, int K,
                             const float* q, int Q, double* out, int* hits, hipStream_t s);
hipError_t launch_ellipsoid_form(const float* axes, int K, float* form, float* Rmax, hipStream_t s);
hipError_t launch_mlp_init(void* params, float* state, unsigned long long seed, hipStream_t s);
hipError_t launch_mlp_sync(void* params, const float* master, hipStream_t s);

}  // namespace rc
