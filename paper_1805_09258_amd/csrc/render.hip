// render.hip -- the render pass that consumes a radiance cache (Sec. 6,
// "Implementation"; Results in 3D): camera rays are marched uniformly
// through the medium (step 0.1 in the paper) and the in-scattered radiance
// at each march point comes from the cache.  Three kernels:
//   march_count: closest surface hit of each camera ray (the BVH traversal of
//                the record kernel), the number of march points before it,
//                and an in-place scan of the counts into offsets;
//   march_emit:  the march points (positions and quadrature weights);
//   composite:   pixel = mean over its rays of sum(weight * L).
// Positions, counts and weights are formed in FP64 from FP32 inputs (the
// library is compiled without FP contraction), so that they are a fixed
// function of the inputs.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "render.hpp"

namespace rc {

namespace {

// Number of k >= 0 with (k + xi) * step < t: the smallest k with
// (k + xi) * step >= t (monotone in k).  k + xi is exact in FP64.
RC_DEV long long march_points(float t, float xi, double step) {
  const double te = t, x = xi;
  const double g = te / step - x;
  long long k = g > 0.0 ? (long long)ceil(g) : 0;
  while (k > 0 && ((double)(k - 1) + x) * step >= te) k--;
  while (((double)k + x) * step < te) k++;
  return k;
}

}  // namespace

template <int STACK>
__global__ __launch_bounds__(64) void march_count_kernel(const float4* __restrict__ nodes,
                                                         const float4* __restrict__ tris, int tri_stride,
                                                         const float* __restrict__ o, const float* __restrict__ d,
                                                         const float* __restrict__ xi, int n, double step, float3 lo,
                                                         float3 hi, float* __restrict__ t_end,
                                                         long long* __restrict__ offsets) {
  __shared__ int stack[STACK * kWave];
  const int i = blockIdx.x * kWave + threadIdx.x;
  if (i == 0) offsets[0] = 0;
  if (i >= n) return;
  const float3 oo = make_float3(o[3 * i], o[3 * i + 1], o[3 * i + 2]);
  const float3 dd = make_float3(d[3 * i], d[3 * i + 1], d[3 * i + 2]);
  int id;
  float tt;
  bool fr;
  TraceCount tc;
  trace_closest<false>(nodes, tris, tri_stride, oo, dd, stack + threadIdx.x, 0, id, tt, fr, tc);
  if (id < 0) tt = box_exit(oo, dd, lo, hi);
  // a ray that neither hits nor leaves the box (zero direction) has no points
  const bool ok = tt < 3.0e38f;
  t_end[i] = tt;
  offsets[i + 1] = ok ? march_points(tt, xi[i], step) : 0;
}

// In-place inclusive scan of offsets[1..n] by one workgroup: tiles of
// kScanThreads * kScanPerThread counts, each thread summing kScanPerThread
// consecutive ones, a wave prefix sum of the thread sums by lane shuffles,
// the wave totals combined through LDS, and a carry from tile to tile.
__global__ __launch_bounds__(kScanThreads) void scan_counts_kernel(long long* __restrict__ offsets, int n) {
  constexpr int kWaves = kScanThreads / kWave;
  __shared__ long long wtot[kWaves];
  const int t = threadIdx.x, lane = t & (kWave - 1), wv = t / kWave;
  long long* c = offsets + 1;
  long long carry = 0;  // the same in every thread
  constexpr int kTile = kScanThreads * kScanPerThread;
  for (long long base = 0; base < n; base += kTile) {
    long long v[kScanPerThread];
    long long sum = 0;
#pragma unroll
    for (int e = 0; e < kScanPerThread; e++) {
      const long long j = base + (long long)t * kScanPerThread + e;
      v[e] = j < n ? c[j] : 0;
      sum += v[e];
    }
    long long incl = sum;
#pragma unroll
    for (int sh = 1; sh < kWave; sh <<= 1) {
      const long long u = __shfl_up(incl, sh, kWave);
      if (lane >= sh) incl += u;
    }
    if (lane == kWave - 1) wtot[wv] = incl;
    __syncthreads();
    long long off = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) {
      const long long x = wtot[w];
      total += x;
      off += w < wv ? x : 0;
    }
    long long run = carry + off + incl - sum;
#pragma unroll
    for (int e = 0; e < kScanPerThread; e++) {
      const long long j = base + (long long)t * kScanPerThread + e;
      run += v[e];
      if (j < n) c[j] = run;
    }
    carry += total;
    __syncthreads();  // wtot is rewritten by the next tile
  }
}

// One thread per ray writes its points: t_k = (k + xi) step, position
// o + t_k d rounded once to FP32, weight step sigma_s exp(-sigma_t t_k).
__global__ __launch_bounds__(256) void march_emit_kernel(const float* __restrict__ o, const float* __restrict__ d,
                                                         const float* __restrict__ xi, int n, double step,
                                                         double sigma_s, double sigma_t,
                                                         const long long* __restrict__ offsets,
                                                         float* __restrict__ points, double* __restrict__ weight) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long a = offsets[i], m = offsets[i + 1] - a;
  const double ox = o[3 * i], oy = o[3 * i + 1], oz = o[3 * i + 2];
  const double dx = d[3 * i], dy = d[3 * i + 1], dz = d[3 * i + 2];
  const double x = xi[i], ws = step * sigma_s;
  for (long long k = 0; k < m; k++) {
    const double t = ((double)k + x) * step;
    float* p = points + 3 * (a + k);
    p[0] = (float)(ox + t * dx);
    p[1] = (float)(oy + t * dy);
    p[2] = (float)(oz + t * dz);
    weight[a + k] = ws * exp(-sigma_t * t);
  }
}

// Pixels: one thread per ray sums weight * L over the ray's points (in
// order) into LDS; then one thread per pixel adds its spp ray sums in ray
// order and divides by spp.  A workgroup holds 256 / spp whole pixels.
__global__ __launch_bounds__(256) void composite_kernel(const long long* __restrict__ offsets, int n_pixels, int spp,
                                                        const double* __restrict__ weight,
                                                        const double* __restrict__ L, double* __restrict__ pixel) {
  __shared__ double ray[256];
  const int per = 256 / spp;  // pixels per workgroup (spp <= 256)
  const int p0 = blockIdx.x * per;
  const int t = threadIdx.x;
  const long long r = (long long)p0 * spp + t;
  if (t < per * spp && r < (long long)n_pixels * spp) {
    double acc = 0.0;
    for (long long j = offsets[r]; j < offsets[r + 1]; j++) acc += weight[j] * L[j];
    ray[t] = acc;
  }
  __syncthreads();
  const int p = p0 + t;
  if (t < per && p < n_pixels) {
    double acc = 0.0;
    for (int k = 0; k < spp; k++) acc += ray[t * spp + k];
    pixel[p] = acc / spp;
  }
}

// More than 256 samples per pixel: one thread per pixel, rays in order.
__global__ __launch_bounds__(256) void composite_wide_kernel(const long long* __restrict__ offsets, int n_pixels,
                                                             int spp, const double* __restrict__ weight,
                                                             const double* __restrict__ L,
                                                             double* __restrict__ pixel) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pixels) return;
  double acc = 0.0;
  for (long long r = (long long)p * spp; r < (long long)(p + 1) * spp; r++) {
    double rs = 0.0;
    for (long long j = offsets[r]; j < offsets[r + 1]; j++) rs += weight[j] * L[j];
    acc += rs;
  }
  pixel[p] = acc / spp;
}

hipError_t launch_march_count(const float4* nodes, const float4* tris, int tri_stride, int depth, const float* o,
                              const float* d, const float* xi, int n, double step, float3 lo, float3 hi,
                              float* t_end, long long* offsets, hipStream_t s) {
  const int blocks = n > 0 ? (n + kWave - 1) / kWave : 1;  // one block writes offsets[0] even for n = 0
  const int st = stack_variant(depth);
  if (st <= 16)
    hipLaunchKernelGGL(march_count_kernel<16>, dim3(blocks), dim3(kWave), 0, s, nodes, tris, tri_stride, o, d, xi, n,
                       step, lo, hi, t_end, offsets);
  else if (st <= 32)
    hipLaunchKernelGGL(march_count_kernel<32>, dim3(blocks), dim3(kWave), 0, s, nodes, tris, tri_stride, o, d, xi, n,
                       step, lo, hi, t_end, offsets);
  else if (st <= 48)
    hipLaunchKernelGGL(march_count_kernel<48>, dim3(blocks), dim3(kWave), 0, s, nodes, tris, tri_stride, o, d, xi, n,
                       step, lo, hi, t_end, offsets);
  else
    hipLaunchKernelGGL(march_count_kernel<64>, dim3(blocks), dim3(kWave), 0, s, nodes, tris, tri_stride, o, d, xi, n,
                       step, lo, hi, t_end, offsets);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n == 0) return e;
  hipLaunchKernelGGL(scan_counts_kernel, dim3(1), dim3(kScanThreads), 0, s, offsets, n);
  return hipGetLastError();
}

hipError_t launch_march_emit(const float* o, const float* d, const float* xi, int n, double step, double sigma_s,
                             double sigma_t, const long long* offsets, float* points, double* weight, hipStream_t s) {
  const int blocks = (n + 255) / 256;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(march_emit_kernel, dim3(blocks), dim3(256), 0, s, o, d, xi, n, step, sigma_s, sigma_t, offsets,
                     points, weight);
  return hipGetLastError();
}

hipError_t launch_composite(const long long* offsets, int n_pixels, int spp, const double* weight, const double* L,
                            double* pixel, hipStream_t s) {
  if (n_pixels <= 0) return hipSuccess;
  if (spp <= 256) {
    const int per = 256 / spp;
    const int blocks = (n_pixels + per - 1) / per;
    hipLaunchKernelGGL(composite_kernel, dim3(blocks), dim3(256), 0, s, offsets, n_pixels, spp, weight, L, pixel);
  } else {
    hipLaunchKernelGGL(composite_wide_kernel, dim3((n_pixels + 255) / 256), dim3(256), 0, s, offsets, n_pixels, spp,
                       weight, L, pixel);
  }
  return hipGetLastError();
}

}  // namespace rc
