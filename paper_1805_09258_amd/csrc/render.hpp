// render.hpp -- launch interface of the render-pass kernels (camera-ray
// marching through the medium and pixel compositing).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rc {

int stack_variant(int depth);

constexpr int kScanThreads = 1024;  // one workgroup scans the per-ray counts
constexpr int kScanPerThread = 16;  // consecutive counts per thread and tile

hipError_t launch_march_count(const float4* nodes, const float4* tris, int tri_stride, int depth, const float* o,
                              const float* d, const float* xi, int n, double step, float3 lo, float3 hi,
                              float* t_end, long long* offsets, hipStream_t s);
hipError_t launch_march_emit(const float* o, const float* d, const float* xi, int n, double step, double sigma_s,
                             double sigma_t, const long long* offsets, float* points, double* weight, hipStream_t s);
hipError_t launch_composite(const long long* offsets, int n_pixels, int spp, const double* weight, const double* L,
                            double* pixel, hipStream_t s);

}  // namespace rc
