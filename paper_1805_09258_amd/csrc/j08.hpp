// j08.hpp -- launch interface of the comparison method's records: values,
// occlusion-unaware gradients and gradient-norm radii.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rc.h"

namespace rc {

struct J08Args {
  const float4* nodes;
  const float4* tris;
  int tri_stride;
  const float4* shade;
  const float* emission;
  float3 box_lo, box_hi;
  int n_lights;
  float4 lights[RC_MAX_LIGHTS];
  float sigma_s, sigma_a, ring_step;
  int max_rings;
  unsigned long long seed;
  long long rec_base;
  int common_random;
  const float* pos;
  const int* n_theta;
  const int* n_phi;
  int P;
  const int4* lb_desc;  // light bins of these lights (nullptr when there are none)
  const int* lb_offs;
  const float4* lb_ent;
  float eps, r_min, r_max;
  double* value;    // [P][2]
  double* grad;     // [P][2][3]
  double* moments;  // [P][2]
  float* R;         // [P]
};

int stack_variant(int depth);
hipError_t launch_j08(const J08Args& a, int depth, hipStream_t s);

}  // namespace rc
