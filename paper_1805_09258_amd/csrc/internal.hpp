// internal.hpp -- shared between the host API and the kernels of librc.
#pragma once
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "limits.hpp"
#include "rc.h"

namespace rc {

// Node layout (64 bytes, four 16-byte words), a binary BVH whose nodes store
// both children's padded boxes so one fetch decides both:
//   w0 = (c0.lo.x, c0.hi.x, c0.lo.y, c0.hi.y)
//   w1 = (c1.lo.x, c1.hi.x, c1.lo.y, c1.hi.y)
//   w2 = (c0.lo.z, c0.hi.z, c1.lo.z, c1.hi.z)
//   w3 = (child0, child1, 0, 0) as int bits: >= 0 internal node index,
//        < 0 leaf ~((first << 3) | (count - 1)).
// Triangle layout (48 bytes): (v0.xyz, id bits), (v1.xyz, 0), (v2.xyz, 0),
// the vertices as given (the watertight hit test projects them along the ray).
constexpr int kLeafMax = 4;
constexpr int kMaxDepth = 60;

struct HostBvh {
  std::vector<float> nodes;   // [n_nodes * 16]
  std::vector<float> tris;    // [T * 12]
  int depth = 0;
  float pad = 0.f;
};

// Traversal stack entries of the record kernel variant for a BVH of this
// depth (16, 24, 32, 48 or 64; kernels.hip).
int stack_variant(int depth);

// Build on the host. pad = scene coordinate scale (bvh_pad_for).
int build_bvh(const float* tri, int64_t T, float pad, HostBvh& out, std::string& err);

// Scene coordinate scale (largest |coordinate| or box side) that sets the
// FP32 error of an accepted ray/triangle hit.
float bvh_pad_for(const float* tri, int64_t T, const float* lo, const float* hi);
// Box padding of one triangle (16 x the FP32 error bound of an accepted hit, see bvh.cpp).
float triangle_pad(const float* t, float scale);

// Per-light triangle bins (lightbins.cpp): levels of B / 4^k bins per cube
// face side (k < levels <= kLbMaxLevels).  offs: for each level (from
// lev_off[k]) two words per bin, the first entry's index and its stored
// distance as float bits (+inf if empty), then one word, the end of the
// level's last bin (a bin's entries end where the next bin's begin).
// entries: 12 floats each, the triangle's vertices permuted for the face's
// axis, its id bits (word 3), its distance from the light minus the hit-test
// error, rounded down (word 7), and the next entry's distance in the bin
// (word 11, +inf for the last); a bin's entries by increasing distance.
struct LightBinsHost {
  int B = 0, nlev = 0;
  int64_t lev_off[kLbMaxLevels] = {0, 0, 0, 0};
  std::vector<int32_t> offs;
  std::vector<float> entries;
};
int light_bins_levels(int B);
int light_bins_size_for(int64_t T);
int build_light_bins(const float* tri, int64_t T, float scale, const float light[3], int B, LightBinsHost& out,
                     std::string& err);

}  // namespace rc
