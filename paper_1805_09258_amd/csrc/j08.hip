// j08.hip -- records of the comparison method (Jarosz et al. 2008, as the
// paper summarises it in Sec. 3 and supplement Eqs. S.3-S.4): the same
// stratified directions, hits, shading and medium rings as a record's Monte
// Carlo value, with occlusion-unaware gradients and the gradient-norm radius
// of Eq. jaroszRadius.
//   single scattering: a direction's sample keeps its hit point y fixed as x
//     moves; its gradient is the sample times grad ln T + grad ln G with
//     T = exp(-mu r), G = (yx . n) / r^3, yx = x - y;
//   multiple scattering: the path x -> ring vertex m -> light moves
//     rigidly, so only the light connection I exp(-mu d) / d^2 changes
//     (visibility held): contribution * (-mu - 2 / d) (m - l) / d;
//   radius: eps * sum_k L_k / sum_k |grad L_k| over the directions k.
// One workgroup of kJ08Waves wavefronts per record, one direction per lane
// (wavefront v takes the 64-direction chunks v, v + kJ08Waves, ...); per-lane
// FP64 sums, reduced across each wavefront and then over the wavefronts in
// order through LDS.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "j08.hpp"

namespace rc {

namespace {

RC_DEV double wave_sum(double v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, kWave);
  return v;
}

}  // namespace

constexpr int kJ08Waves = 4;  // wavefronts per record

template <int STACK>
__global__ __launch_bounds__(kWave * kJ08Waves) void j08_kernel(J08Args g) {
  __shared__ int stack[kJ08Waves * STACK * kWave];
  __shared__ double part[kJ08Waves][10];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  int* stk = stack + wv * STACK * kWave + lane;
  TraceCount tc;
  const double mu = (double)g.sigma_s + (double)g.sigma_a;
  const float muf = g.sigma_s + g.sigma_a;
  const double ms_scale = (double)g.sigma_s / (4.0 * kPi);
  for (int rec = blockIdx.x; rec < g.P; rec += gridDim.x) {
    const int nth = g.n_theta[rec], nph = g.n_phi[rec];
    if (nth < 2 || nph < 5 || nph > RC_MAX_NPHI) {  // invalid sample counts: NaN outputs (same for the workgroup)
      if (threadIdx.x < 2) {
        g.value[2 * rec + lane] = __builtin_nan("");
        g.moments[2 * rec + lane] = __builtin_nan("");
        for (int k = 0; k < 3; k++) g.grad[6 * rec + 3 * lane + k] = __builtin_nan("");
      }
      if (threadIdx.x == 0) g.R[rec] = __builtin_nanf("");
      continue;
    }
    const float3 x = make_float3(g.pos[3 * rec], g.pos[3 * rec + 1], g.pos[3 * rec + 2]);
    const uint64_t key = record_key(g.seed, (uint64_t)(g.rec_base + (g.common_random ? 0 : rec)));
    const float xr = uniform24(key, kRingIdx, 0);
    const int N = nth * nph;
    double vs = 0.0, vm = 0.0, lsum = 0.0, nsum = 0.0;
    double gs[3] = {0.0, 0.0, 0.0}, gm[3] = {0.0, 0.0, 0.0};
    for (int base = wv * kWave; base < N; base += kWave * kJ08Waves) {
      const int s = base + lane;
      if (s >= N) continue;
      const int a = s / nph, b = s - a * nph;
      const float3 w = stratum_direction(key, a, b, nth, nph);
      int id;
      float t;
      bool fr;
      trace_closest<false>(g.nodes, g.tris, g.tri_stride, x, w, stk, 0, id, t, fr, tc);
      if (id < 0) t = box_exit(x, w, g.box_lo, g.box_hi);
      const double wx = w.x, wy = w.y, wz = w.z;
      const double wn = sqrt(wx * wx + wy * wy + wz * wz);
      double gk[3] = {0.0, 0.0, 0.0}, Lk = 0.0;
      if (id >= 0) {  // surface sample, hit point held fixed
        const float4 sh = g.shade[id];
        const float nsign = fr ? 1.f : -1.f;
        const float3 nrm = make_float3(nsign * sh.x, nsign * sh.y, nsign * sh.z);
        const float3 y = axpy3(t, w, x);
        const int bits = g.n_lights > 0 ? light_bits<false>(g.lights, g.n_lights, g.lb_desc, g.lb_offs, g.lb_ent, y,
                                                            id, nrm, stk, tc)
                                        : 0;
        float Ls = g.emission[id];
        for (int l = 0; l < g.n_lights; l++) {
          if (!((bits >> l) & 1)) continue;
          const float4 L = g.lights[l];
          const float3 seg = make_float3(L.x - y.x, L.y - y.y, L.z - y.z);
          const float dist = sqrtf(dot3(seg, seg));
          const float c = dot3(nrm, seg) / dist;
          Ls += sh.w * (float)(1.0 / kPi) * L.w * c * expf(-muf * dist) / (dist * dist);
        }
        const double tt = t, r = tt * wn;
        const double S = exp(-mu * r) * (double)Ls;
        const double yx[3] = {-tt * wx, -tt * wy, -tt * wz};
        const double n3[3] = {sh.x, sh.y, sh.z};
        const double yn = yx[0] * n3[0] + yx[1] * n3[1] + yx[2] * n3[2];
#pragma unroll
        for (int i = 0; i < 3; i++) {
          gk[i] = S * (-mu * yx[i] / r + n3[i] / yn - 3.0 * yx[i] / (r * r));
          gs[i] += gk[i];
        }
        Lk += S;
        vs += S;
      }
      // medium ring vertices in front of the hit, paths moved rigidly
      for (int i = 0; i < g.max_rings && g.n_lights > 0; i++) {
        const float ri = ring_distance(i, xr, g.ring_step);
        if (!(ri < t)) break;
        const float3 y = axpy3(ri, w, x);
        const int bits = light_bits<false>(g.lights, g.n_lights, g.lb_desc, g.lb_offs, g.lb_ent, y, -1,
                                           make_float3(0.f, 0.f, 0.f), stk, tc);
        if (!bits) continue;
        const double r64 = ((double)i + (double)xr) * (double)g.ring_step;
        const double y64[3] = {(double)x.x + r64 * wx, (double)x.y + r64 * wy, (double)x.z + r64 * wz};
        const double att = (double)g.ring_step * exp(-mu * r64 * wn) * ms_scale;
        for (int l = 0; l < g.n_lights; l++) {
          if (!((bits >> l) & 1)) continue;
          const float4 L = g.lights[l];
          const double ml[3] = {y64[0] - (double)L.x, y64[1] - (double)L.y, y64[2] - (double)L.z};
          const double d = sqrt(ml[0] * ml[0] + ml[1] * ml[1] + ml[2] * ml[2]);
          const double c = att * (double)L.w * exp(-mu * d) / (d * d);
          Lk += c;
          vm += c;
#pragma unroll
          for (int q = 0; q < 3; q++) {
            const double gq = c * (-mu - 2.0 / d) * ml[q] / d;
            gk[q] += gq;
            gm[q] += gq;
          }
        }
      }
      lsum += Lk;
      nsum += sqrt(gk[0] * gk[0] + gk[1] * gk[1] + gk[2] * gk[2]);
    }
    vs = wave_sum(vs);
    vm = wave_sum(vm);
    lsum = wave_sum(lsum);
    nsum = wave_sum(nsum);
#pragma unroll
    for (int i = 0; i < 3; i++) {
      gs[i] = wave_sum(gs[i]);
      gm[i] = wave_sum(gm[i]);
    }
    if (lane == 0) {
      part[wv][0] = vs, part[wv][1] = vm, part[wv][2] = lsum, part[wv][3] = nsum;
      for (int i = 0; i < 3; i++) part[wv][4 + i] = gs[i], part[wv][7 + i] = gm[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double t[10];
      for (int q = 0; q < 10; q++) {
        t[q] = 0.0;
        for (int v = 0; v < kJ08Waves; v++) t[q] += part[v][q];
      }
      const double inv = 1.0 / N;
      g.value[2 * rec] = t[0] * inv;
      g.value[2 * rec + 1] = t[1] * inv;
      for (int i = 0; i < 3; i++) {
        g.grad[6 * rec + i] = t[4 + i] * inv;
        g.grad[6 * rec + 3 + i] = t[7 + i] * inv;
      }
      g.moments[2 * rec] = t[2] * inv;
      g.moments[2 * rec + 1] = t[3] * inv;
      const double R = t[3] > 0.0 ? (double)g.eps * t[2] / t[3] : (double)g.r_max;
      g.R[rec] = (float)fmin(fmax(R, (double)g.r_min), (double)g.r_max);
    }
    __syncthreads();  // part is rewritten by the next record
  }
}

hipError_t launch_j08(const J08Args& a, int depth, hipStream_t s) {
  if (a.P <= 0) return hipSuccess;
  const int grid = a.P < 65536 ? a.P : 65536;
  const int st = stack_variant(depth);
  const dim3 block(kWave * kJ08Waves);
  if (st <= 16) hipLaunchKernelGGL(j08_kernel<16>, dim3(grid), block, 0, s, a);
  else if (st <= 32) hipLaunchKernelGGL(j08_kernel<32>, dim3(grid), block, 0, s, a);
  else if (st <= 48) hipLaunchKernelGGL(j08_kernel<48>, dim3(grid), block, 0, s, a);
  else hipLaunchKernelGGL(j08_kernel<64>, dim3(grid), block, 0, s, a);
  return hipGetLastError();
}

}  // namespace rc
