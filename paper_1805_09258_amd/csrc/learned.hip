// learned.hip -- learned cache placement on gfx950 (project-defined, not in
// the paper): a 64-ray probe per candidate point, a 32 -> 128 -> 128 -> 1 MLP
// (GELU, BF16 weights, FP32 accumulation on MFMA) that predicts the log of
// the validity radius of Sec. 5 (Eq. radiusAniso3D), its training step
// (forward, backward, Adam), greedy cover placement, and the interpolation of
// a cache (Eq. radianceTaylor) to measure rendered-cache error.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "learned.hpp"

namespace rc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

RC_DEV float wsum(float v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, kWave);
  return v;
}
RC_DEV float wmin(float v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v = fminf(v, __shfl_xor(v, s, kWave));
  return v;
}
RC_DEV float wmax(float v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v = fmaxf(v, __shfl_xor(v, s, kWave));
  return v;
}
// sum over the 16 lanes of a strata row (lanes 16r .. 16r+15)
RC_DEV float rowsum16(float v) {
#pragma unroll
  for (int s = 8; s >= 1; s >>= 1) v += __shfl_xor(v, s, kWave);
  return v;
}

// tanh-form GELU and its derivative (Hendrycks & Gimpel 2016)
RC_DEV float gelu(float x) {
  const float k = 0.7978845608028654f;
  float u = k * (x + 0.044715f * x * x * x);
  return 0.5f * x * (1.0f + tanhf(u));
}
RC_DEV float gelu_grad(float x) {
  const float k = 0.7978845608028654f;
  float u = k * (x + 0.044715f * x * x * x);
  float t = tanhf(u);
  float du = k * (1.0f + 3.0f * 0.044715f * x * x);
  return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * du;
}

}  // namespace

// ---------------------------------------------------------------------------
// Probe: one wavefront per candidate, one lane per direction of a 4 x 16
// strata grid.  Each lane traces its direction (closest hit), shades the hit
// with shadow rays (Lambertian, lit side facing x, point lights, emission)
// and attenuates it to x; lanes 0..L-1 also test the visibility of light l
// from x.  Wave reductions turn these into 32 features.
// ---------------------------------------------------------------------------
template <int STACK>
__global__ __launch_bounds__(64) void probe_kernel(ProbeArgs g) {
  __shared__ int stack[STACK * kWave];
  __shared__ float Ls_row[kWave];
  __shared__ float sw[3][kWave], st_[kWave];  // each direction and its hit distance
  __shared__ int scode[kWave];                  // (triangle << 1) | front, or -1
  __shared__ int vbits[kWave + 1];              // unblocked lights per hit; [64]: from x
  const int lane = threadIdx.x;
  int* stk = stack + lane;
  TraceCount tc;
  const float mu = g.sigma_s + g.sigma_a;
  const int nx = g.n_lights < 4 ? g.n_lights : 4;  // lights whose visibility from x is a feature
  for (int c = blockIdx.x; c < g.C; c += gridDim.x) {
    const float3 x = make_float3(g.cand[3 * c], g.cand[3 * c + 1], g.cand[3 * c + 2]);
    const uint64_t key = record_key(g.seed, (uint64_t)(g.id_base + (g.common_random ? 0 : c)));
    const int a = lane >> 4, b = lane & 15;
    const float3 w = stratum_direction(key, a, b, 4, 16);
    int id;
    float t;
    bool fr;
    trace_closest<false>(g.nodes, g.tris, g.tri_stride, x, w, stk, 0, id, t, fr, tc);
    const bool hit = id >= 0;
    if (!hit) t = box_exit(x, w, g.box_lo, g.box_hi);
    sw[0][lane] = w.x;
    sw[1][lane] = w.y;
    sw[2][lane] = w.z;
    st_[lane] = t;
    scode[lane] = hit ? ((id << 1) | (fr ? 1 : 0)) : -1;
    vbits[lane] = 0;
    if (lane == 0) vbits[kWave] = 0;
    __syncthreads();
    // Shadow segments: hit point to light l (skipped when the hit's lit side
    // faces away) for every lane's hit and light, and x to light l for
    // l < min(L, 4).  From the light bins: each lane walks its hit's lights
    // in turn, lanes 0..min(L,4)-1 also the segment from x.
    if (g.lb_desc) {
      int bits = 0;
      if (hit) {
        const float4 sh = g.shade[id];
        const float nsign = fr ? 1.f : -1.f;
        bits = light_bits<false>(g.lights, g.n_lights, g.lb_desc, g.lb_offs, g.lb_ent, axpy3(t, w, x), id,
                                 make_float3(nsign * sh.x, nsign * sh.y, nsign * sh.z), stk, tc);
      }
      vbits[lane] = bits;
      if (lane < nx && light_visible<false>(g.lights[lane], lane, g.lb_desc, g.lb_offs, g.lb_ent, x, -1, stk, tc))
        atomicOr(&vbits[kWave], 1 << lane);
    } else {
    // From the BVH, as a list of tasks: (direction k, light l) for
    // k + 64 l < 64 L, then (x, light l) for l < min(L, 4).  Each loop
    // iteration advances every busy lane by one node or one triangle; a lane
    // whose segment is resolved takes the next task, so lanes stay busy while
    // segments of different lengths finish.
    {
      const int total = kWave * g.n_lights + nx;
      int next = 0;
      bool active = false;
      int node = 0, sp = 0, lf = 0, ln = 0, skip = -1, dst = 0, bit = 0;
      float3 o = make_float3(0.f, 0.f, 0.f), d = o, inv = o, oi = o;
      WtRay wr = wt_ray(o, d);
      while (true) {
        const uint64_t idle = __ballot(!active);
        if (next < total && (__popcll(idle) >= 8 || idle == ~0ull)) {
          if (!active) {
            const int task = next + mask_rank(idle);
            if (task < total) {
              active = true;
              if (task < kWave * g.n_lights) {
                const int k = task & (kWave - 1), l = task >> 6;
                const int code = scode[k];
                const float4 L = g.lights[l];
                if (code < 0) {
                  active = false;
                } else {
                  const float3 wk = make_float3(sw[0][k], sw[1][k], sw[2][k]);
                  o = axpy3(st_[k], wk, x);
                  d = make_float3(L.x - o.x, L.y - o.y, L.z - o.z);
                  skip = code >> 1;
                  const float4 sh = g.shade[skip];
                  const float nsign = (code & 1) ? 1.f : -1.f;
                  const float cs = nsign * dot3(make_float3(sh.x, sh.y, sh.z), d) / sqrtf(dot3(d, d));
                  if (!(cs > 0.f)) active = false;
                  dst = k;
                  bit = 1 << l;
                }
              } else {
                const int l = task - kWave * g.n_lights;
                const float4 L = g.lights[l];
                o = x;
                d = make_float3(L.x - x.x, L.y - x.y, L.z - x.z);
                skip = -1;
                dst = kWave;
                bit = 1 << l;
              }
              wr = wt_ray(o, d);
              ray_inv(d, o, inv, oi);
              node = 0;
              sp = 0;
              ln = 0;
            }
          }
          next += __popcll(idle);
        }
        if (__ballot(active) == 0ull) {
          if (next >= total) break;
          continue;
        }
        if (active) {
          bool done = false, blocked = false;
          const float4* src = (ln > 0) ? (g.tris + wr.kz * g.tri_stride + 3 * lf) : (g.nodes + 4 * node);
          const float4 q0 = src[0], q1 = src[1], q2 = src[2], q3 = src[3];
          if (ln > 0) {
            float th;
            bool fh;
            if (__float_as_int(q0.w) != skip && hit_triangle(wr, q0, q1, q2, 1e-4f, 1.0f, th, fh)) {
              done = true;
              blocked = true;
            } else {
              lf++;
              ln--;
              if (ln == 0) {
                if (sp == 0) {
                  done = true;
                } else {
                  const int cc = stk[--sp * kWave];
                  if (cc < 0) {
                    lf = leaf_first(cc);
                    ln = leaf_count(cc);
                  } else {
                    node = cc;
                  }
                }
              }
            }
          } else {
            const float ta = slab(q0.x, q0.y, q0.z, q0.w, q2.x, q2.y, inv, oi, 0.0f, 1.0f);
            const float tb = slab(q1.x, q1.y, q1.z, q1.w, q2.z, q2.w, inv, oi, 0.0f, 1.0f);
            const int ca = __float_as_int(q3.x), cb = __float_as_int(q3.y);
            const bool ha = ta < __builtin_huge_valf(), hb = tb < __builtin_huge_valf();
            int nxn;
            if (ha && hb) {
              nxn = ta <= tb ? ca : cb;
              stk[sp++ * kWave] = ta <= tb ? cb : ca;
            } else if (ha || hb) {
              nxn = ha ? ca : cb;
            } else {
              nxn = sp == 0 ? 0x7fffffff : stk[--sp * kWave];
            }
            if (nxn == 0x7fffffff) {
              done = true;
            } else if (nxn < 0) {
              lf = leaf_first(nxn);
              ln = leaf_count(nxn);
            } else {
              node = nxn;
            }
          }
          if (done) {
            active = false;
            if (!blocked) atomicOr(&vbits[dst], bit);
          }
        }
      }
    }
    }  // BVH shadow segments
    __syncthreads();
    // radiance of each hit: emission plus the unblocked lights, in order
    float Ls = hit ? g.emission[id] : 0.f;
    if (hit) {
      const int bits = vbits[lane];
      const float3 y = axpy3(t, w, x);
      const float4 sh = g.shade[id];
      const float nsign = fr ? 1.f : -1.f;
      for (int l = 0; l < g.n_lights; l++) {
        const float4 L = g.lights[l];
        const float3 seg = make_float3(L.x - y.x, L.y - y.y, L.z - y.z);
        const float dist = sqrtf(dot3(seg, seg));
        const float cs = nsign * dot3(make_float3(sh.x, sh.y, sh.z), seg) / dist;
        if (cs > 0.f && ((bits >> l) & 1))
          Ls += sh.w * (float)(1.0 / kPi) * L.w * cs * expf(-mu * dist) / (dist * dist);
      }
    }
    const float wn = sqrtf(dot3(w, w));
    const float dist = fmaxf(t * wn, 1e-6f);
    const float Lt = expf(-mu * dist) * Ls;          // radiance arriving at x
    // direct light from x: visibility and unshadowed irradiance proxy
    float vis = 0.f, dirl = 0.f;
    if (lane < nx) {
      const float4 L = g.lights[lane];
      const float3 seg = make_float3(L.x - x.x, L.y - x.y, L.z - x.z);
      const float d2 = dot3(seg, seg);
      vis = ((vbits[kWave] >> lane) & 1) ? 1.f : 0.f;
      dirl = logf(L.w * expf(-mu * sqrtf(d2)) / d2 + 1e-6f);
    }
    // neighbour contrast along phi within the strata row
    Ls_row[lane] = Lt;
    __syncthreads();
    const float Lnb = Ls_row[(a << 4) | ((b + 1) & 15)];
    __syncthreads();
    const float ld = logf(dist);
    const float inv = 1.f / dist;
    float f[32];
    f[0] = wmin(ld);
    f[1] = wsum(ld) * (1.f / 64.f);
    {
      float d0 = ld - f[1];
      f[2] = sqrtf(wsum(d0 * d0) * (1.f / 64.f));
    }
    f[3] = wmax(ld);
    f[4] = wsum(hit ? 0.f : 1.f) * (1.f / 64.f);
    f[5] = logf(wsum(inv) * (1.f / 64.f));
    const float mL = wsum(Lt) * (1.f / 64.f);
    f[6] = logf(mL + 1e-6f);
    {
      float d0 = Lt - mL;
      f[7] = sqrtf(wsum(d0 * d0) * (1.f / 64.f)) / (mL + 1e-6f);
    }
    f[8] = logf(wmax(Lt) + 1e-6f);
    for (int l = 0; l < 4; l++) {
      f[9 + l] = __shfl(vis, l, kWave);
      f[13 + l] = (l < g.n_lights) ? __shfl(dirl, l, kWave) : 0.f;
    }
    const float sL = wsum(Lt) + 1e-12f;
    f[17] = wsum(Lt * w.x) / sL;
    f[18] = wsum(Lt * w.y) / sL;
    f[19] = wsum(Lt * w.z) / sL;
    const float sI = wsum(inv);
    f[20] = wsum(inv * w.x) / sI;
    f[21] = wsum(inv * w.y) / sI;
    f[22] = wsum(inv * w.z) / sI;
    const float rld = rowsum16(ld) * (1.f / 16.f);
    const float rll = rowsum16(logf(Lt + 1e-6f)) * (1.f / 16.f);
    for (int r = 0; r < 4; r++) {
      f[23 + r] = __shfl(rld, 16 * r, kWave);
      f[27 + r] = __shfl(rll, 16 * r, kWave);
    }
    f[31] = wsum(fabsf(Lt - Lnb)) / sL;
    // lane k < 32 writes feature k (FP32 and BF16 copies)
    float mine = 0.f;
#pragma unroll
    for (int k = 0; k < 32; k++)
      if (lane == k) mine = f[k];
    if (lane < 32) {
      if (g.feat32) g.feat32[(size_t)c * 32 + lane] = mine;
      if (g.feat16) g.feat16[(size_t)c * 32 + lane] = (__bf16)mine;
    }
  }
}

// ---------------------------------------------------------------------------
// MLP.  Parameter block (see rc.h): standardisation (shift, scale) of the 32
// features, biases and the last layer in FP32, W1 [128][32], W2 [128][128] and
// W2^T in BF16.  One wavefront handles 16 samples with
// v_mfma_f32_16x16x32_bf16 (A: lane l holds row l%16, k = 8(l/16)+i;
// B: column l%16, k = 8(l/16)+i; D: column l%16, rows 4(l/16)+i).
// ---------------------------------------------------------------------------
struct MlpView {
  const float *shift, *scale, *b1, *b2, *w3, *b3;
  const __bf16 *W1, *W2, *W2T;
};
RC_DEV MlpView mlp_view(const void* p) {
  const float* f = static_cast<const float*>(p);
  MlpView v;
  v.shift = f + kMlpShift;
  v.scale = f + kMlpScale;
  v.b1 = f + kMlpB1;
  v.b2 = f + kMlpB2;
  v.w3 = f + kMlpW3;
  v.b3 = f + kMlpB3;
  const __bf16* h = reinterpret_cast<const __bf16*>(f + kMlpFloats);
  v.W1 = h;
  v.W2 = h + 128 * 32;
  v.W2T = h + 128 * 32 + 128 * 128;
  return v;
}

// Forward pass of 16 samples (rows s0..s0+15 of X, FP32 features); fills the
// activations the backward pass needs.  A1 (BF16, [16][128], row-major) goes
// to LDS; Z1 and Z2 stay in registers in the D layout: z1[nb][i] is sample
// 4(l/16)+i, unit 16 nb + l%16.
RC_DEV void mlp_forward16(const MlpView& P, const float* __restrict__ X, int s0, int n, __bf16* A1s,
                          float z1[8][4], float z2[8][4], float y[4]) {
  const int l = threadIdx.x & 63;
  const int r = l & 15, q = l >> 4;
  // A operand: standardised features of sample s0 + r, k = 8q .. 8q+7
  bf16x8 xa;
  {
    const int s = s0 + r;
#pragma unroll
    for (int i = 0; i < 8; i++) {
      const int k = 8 * q + i;
      float v = (s < n) ? (X[(size_t)s * 32 + k] - P.shift[k]) * P.scale[k] : 0.f;
      xa[i] = (__bf16)v;
    }
  }
#pragma unroll
  for (int nb = 0; nb < 8; nb++) {
    bf16x8 wb = *reinterpret_cast<const bf16x8*>(P.W1 + (16 * nb + r) * 32 + 8 * q);
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa, wb, acc, 0, 0, 0);
    const float bias = P.b1[16 * nb + r];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      z1[nb][i] = acc[i] + bias;
      A1s[(4 * q + i) * 128 + 16 * nb + r] = (__bf16)gelu(z1[nb][i]);
    }
  }
  // A1 rows written by other lanes of this wavefront become visible
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // layer 2: K = 128 in four steps of 32
  floatx4 acc2[8];
#pragma unroll
  for (int nb = 0; nb < 8; nb++) acc2[nb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < 4; ks++) {
    const bf16x8 aa = *reinterpret_cast<const bf16x8*>(A1s + r * 128 + 32 * ks + 8 * q);
#pragma unroll
    for (int nb = 0; nb < 8; nb++) {
      const bf16x8 wb = *reinterpret_cast<const bf16x8*>(P.W2 + (16 * nb + r) * 128 + 32 * ks + 8 * q);
      acc2[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aa, wb, acc2[nb], 0, 0, 0);
    }
  }
  float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int nb = 0; nb < 8; nb++) {
    const float bias = P.b2[16 * nb + r], w3 = P.w3[16 * nb + r];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      z2[nb][i] = acc2[nb][i] + bias;
      part[i] += gelu(z2[nb][i]) * w3;
    }
  }
  // reduce over the 16 lanes holding the same samples (same q)
#pragma unroll
  for (int i = 0; i < 4; i++) {
    float v = part[i];
#pragma unroll
    for (int s = 8; s >= 1; s >>= 1) v += __shfl_xor(v, s, kWave);
    y[i] = v + P.b3[0];
  }
}

// RADIUS: out = clamp(safety * exp(y), r_min, r_max) instead of y.
template <bool RADIUS>
__global__ __launch_bounds__(256) void mlp_forward_kernel(const void* params, const float* __restrict__ X, int n,
                                                          float* __restrict__ out, float safety, float r_min,
                                                          float r_max) {
  __shared__ __bf16 A1[4][16 * 128];
  const MlpView P = mlp_view(params);
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  for (int s0 = (blockIdx.x * 4 + wv) * 16; s0 < n; s0 += gridDim.x * 64) {
    float z1[8][4], z2[8][4], y[4];
    mlp_forward16(P, X, s0, n, A1[wv], z1, z2, y);
    if ((l & 15) == 0) {
      const int q = l >> 4;
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int s = s0 + 4 * q + i;
        if (s < n) out[s] = RADIUS ? fminf(fmaxf(safety * expf(y[i]), r_min), r_max) : y[i];
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Training: one workgroup (4 wavefronts, 64 samples) computes the forward
// pass, the loss and the gradient of every parameter for its samples, and
// writes them to its slot of a partial-gradient buffer; a second kernel sums
// the slots in a fixed order and applies Adam.
__global__ __launch_bounds__(256) void mlp_grad_kernel(const void* params, const float* __restrict__ X,
                                                       const float* __restrict__ target, int n, float inv_batch,
                                                       float* __restrict__ partial) {
  __shared__ __bf16 A1[64 * 128];   // layer-1 activations of the tile
  __shared__ __bf16 dZ2[64 * 128];  // layer-2 pre-activation gradients
  __shared__ __bf16 dZ1[64 * 128];  // layer-1 pre-activation gradients
  __shared__ __bf16 Xs[64 * 32];    // standardised inputs
  __shared__ float red[4][3 * 128 + 2];
  const MlpView P = mlp_view(params);
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, q = l >> 4;
  const int s0 = blockIdx.x * 64 + wv * 16;
  float z1[8][4], z2[8][4], y[4];
  mlp_forward16(P, X, s0, n, A1 + wv * 16 * 128, z1, z2, y);
  // standardised inputs of this wave's rows, for dW1
  for (int e = l; e < 16 * 32; e += 64) {
    const int sr = e >> 5, k = e & 31, s = s0 + sr;
    Xs[(wv * 16 + sr) * 32 + k] = (__bf16)((s < n) ? (X[(size_t)s * 32 + k] - P.shift[k]) * P.scale[k] : 0.f);
  }
  // dL/dy for the mean squared error, samples outside the batch contribute 0
  float dy[4], loss = 0.f;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const int s = s0 + 4 * q + i;
    const float e = (s < n) ? (y[i] - target[s]) : 0.f;
    dy[i] = 2.f * e * inv_batch;
    loss += (r == 0) ? e * e : 0.f;
  }
  // dw3, db2, dZ2 (D layout: lane holds unit 16nb + r, samples 4q + i)
  float gw3[8], gb2[8];
#pragma unroll
  for (int nb = 0; nb < 8; nb++) {
    const float w3 = P.w3[16 * nb + r];
    float a = 0.f, bsum = 0.f;
#pragma unroll
    for (int i = 0; i < 4; i++) {
      a += dy[i] * gelu(z2[nb][i]);
      const float dz = dy[i] * w3 * gelu_grad(z2[nb][i]);
      bsum += dz;
      dZ2[(wv * 16 + 4 * q + i) * 128 + 16 * nb + r] = (__bf16)dz;
    }
    gw3[nb] = a;
    gb2[nb] = bsum;
  }
  __syncthreads();
  // dA1 = dZ2 W2 for this wave's 16 rows (A: dZ2 rows, B: W2^T), then dZ1
  float gb1[8];
  {
    floatx4 acc[8];
#pragma unroll
    for (int nb = 0; nb < 8; nb++) acc[nb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4; ks++) {
      const bf16x8 aa = *reinterpret_cast<const bf16x8*>(dZ2 + (wv * 16 + r) * 128 + 32 * ks + 8 * q);
#pragma unroll
      for (int nb = 0; nb < 8; nb++) {
        // B[k = unit j of layer 2][n = unit i of layer 1] = W2[j][i] = W2T[i][j]
        const bf16x8 wb = *reinterpret_cast<const bf16x8*>(P.W2T + (16 * nb + r) * 128 + 32 * ks + 8 * q);
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aa, wb, acc[nb], 0, 0, 0);
      }
    }
#pragma unroll
    for (int nb = 0; nb < 8; nb++) {
      float bsum = 0.f;
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const float dz = acc[nb][i] * gelu_grad(z1[nb][i]);
        bsum += dz;
        dZ1[(wv * 16 + 4 * q + i) * 128 + 16 * nb + r] = (__bf16)dz;
      }
      gb1[nb] = bsum;
    }
  }
  // per-unit sums over the 4 lane groups of the wave, then over waves
#pragma unroll
  for (int nb = 0; nb < 8; nb++) {
    float a = gw3[nb], b2 = gb2[nb], b1 = gb1[nb];
    a += __shfl_xor(a, 16, kWave);
    a += __shfl_xor(a, 32, kWave);
    b2 += __shfl_xor(b2, 16, kWave);
    b2 += __shfl_xor(b2, 32, kWave);
    b1 += __shfl_xor(b1, 16, kWave);
    b1 += __shfl_xor(b1, 32, kWave);
    if (q == 0) {
      red[wv][16 * nb + r] = a;
      red[wv][128 + 16 * nb + r] = b2;
      red[wv][256 + 16 * nb + r] = b1;
    }
  }
  {
    float ls = loss;
    for (int s = 32; s >= 1; s >>= 1) ls += __shfl_xor(ls, s, kWave);
    float ds = (r == 0) ? (dy[0] + dy[1] + dy[2] + dy[3]) : 0.f;
    for (int s = 32; s >= 1; s >>= 1) ds += __shfl_xor(ds, s, kWave);
    if (l == 0) {
      red[wv][384] = ls;
      red[wv][385] = ds;
    }
  }
  __syncthreads();
  float* out = partial + (size_t)blockIdx.x * kMlpGradFloats;
  for (int e = threadIdx.x; e < 386; e += 256) {
    const float v = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
    if (e < 128) out[kGradW3 + e] = v;
    else if (e < 256) out[kGradB2 + e - 128] = v;
    else if (e < 384) out[kGradB1 + e - 256] = v;
    else if (e == 384) out[kGradLoss] = v;
    else out[kGradB3] = v;
  }
  // dW2[j][i] = sum_s dZ2[s][j] A1[s][i]: M = j, N = i, K = 64 samples.
  // 64 output tiles of 16x16, 16 per wave, two K steps each.
  for (int t = wv; t < 64; t += 4) {
    const int mj = t >> 3, ni = t & 7;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ks++) {
      bf16x8 aa, bb;
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const int s = 32 * ks + 8 * q + i;
        aa[i] = dZ2[s * 128 + 16 * mj + r];
        bb[i] = A1[s * 128 + 16 * ni + r];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aa, bb, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; i++) out[kGradW2 + (16 * mj + 4 * q + i) * 128 + 16 * ni + r] = acc[i];
  }
  // dW1[j][k] = sum_s dZ1[s][j] X[s][k]: M = j (128), N = k (32), K = 64.
  for (int t = wv; t < 16; t += 4) {
    const int mj = t >> 1, nk = t & 1;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ks++) {
      bf16x8 aa, bb;
#pragma unroll
      for (int i = 0; i < 8; i++) {
        const int s = 32 * ks + 8 * q + i;
        aa[i] = dZ1[s * 128 + 16 * mj + r];
        bb[i] = Xs[s * 32 + 16 * nk + r];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aa, bb, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; i++) out[kGradW1 + (16 * mj + 4 * q + i) * 32 + 16 * nk + r] = acc[i];
  }
}

// Sum the partial gradients of `tiles` workgroups in order; Adam (Kingma &
// Ba 2015, bias-corrected) on the FP32 master weights; refresh the BF16
// copies (W1, W2, W2^T) and FP32 biases of the parameter block.
__global__ void mlp_adam_kernel(void* params, float* __restrict__ master, float* __restrict__ m,
                                float* __restrict__ v, const float* __restrict__ partial, int tiles, float lr,
                                float b1c, float b2c, float* __restrict__ grad_out, float* __restrict__ loss_out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kMlpGradFloats) return;
  float g = 0.f;
  for (int t = 0; t < tiles; t++) g += partial[(size_t)t * kMlpGradFloats + e];
  if (e == kGradLoss) {
    if (loss_out) *loss_out = g;
    return;
  }
  if (grad_out) grad_out[e] = g;
  const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  const float mm = beta1 * m[e] + (1.f - beta1) * g;
  const float vv = beta2 * v[e] + (1.f - beta2) * g * g;
  m[e] = mm;
  v[e] = vv;
  const float w = master[e] - lr * (mm / b1c) / (sqrtf(vv / b2c) + eps);
  master[e] = w;
  float* f = static_cast<float*>(params);
  __bf16* h = reinterpret_cast<__bf16*>(f + kMlpFloats);
  if (e >= kGradW1 && e < kGradW1 + 128 * 32) {
    h[e - kGradW1] = (__bf16)w;
  } else if (e >= kGradW2 && e < kGradW2 + 128 * 128) {
    const int jj = (e - kGradW2) >> 7, ii = (e - kGradW2) & 127;
    h[128 * 32 + jj * 128 + ii] = (__bf16)w;
    h[128 * 32 + 128 * 128 + ii * 128 + jj] = (__bf16)w;
  } else if (e >= kGradB1 && e < kGradB1 + 128) {
    f[kMlpB1 + e - kGradB1] = w;
  } else if (e >= kGradB2 && e < kGradB2 + 128) {
    f[kMlpB2 + e - kGradB2] = w;
  } else if (e >= kGradW3 && e < kGradW3 + 128) {
    f[kMlpW3 + e - kGradW3] = w;
  } else if (e == kGradB3) {
    f[kMlpB3] = w;
  }
}


// Deterministic initialisation: Glorot-uniform weights from the counter-based
// generator, zero biases, identity standardisation, zero Adam moments.
__global__ void mlp_init_kernel(void* params, float* __restrict__ state, unsigned long long seed) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kMlpGradFloats) return;
  const uint64_t key = record_key(seed, 0x4d4c50ull);
  const float u = 2.f * uniform24(key, (uint64_t)e, 0) - 1.f;
  float w = 0.f;
  if (e < kGradB1) w = u * sqrtf(6.f / (32.f + 128.f));
  else if (e >= kGradW2 && e < kGradB2) w = u * sqrtf(6.f / (128.f + 128.f));
  else if (e >= kGradW3 && e < kGradB3) w = u * sqrtf(6.f / (128.f + 1.f));
  float* master = state;
  float* m = state + kMlpGradFloats;
  float* v = state + 2 * kMlpGradFloats;
  master[e] = w;
  m[e] = 0.f;
  v[e] = 0.f;
  float* f = static_cast<float*>(params);
  __bf16* h = reinterpret_cast<__bf16*>(f + kMlpFloats);
  if (e < 32) {
    f[kMlpShift + e] = 0.f;
    f[kMlpScale + e] = 1.f;
  }
  if (e >= kGradW1 && e < kGradW1 + 128 * 32) h[e - kGradW1] = (__bf16)w;
  else if (e >= kGradW2 && e < kGradW2 + 128 * 128) {
    const int jj = (e - kGradW2) >> 7, ii = (e - kGradW2) & 127;
    h[128 * 32 + jj * 128 + ii] = (__bf16)w;
    h[128 * 32 + 128 * 128 + ii * 128 + jj] = (__bf16)w;
  } else if (e >= kGradB1 && e < kGradB1 + 128) f[kMlpB1 + e - kGradB1] = w;
  else if (e >= kGradB2 && e < kGradB2 + 128) f[kMlpB2 + e - kGradB2] = w;
  else if (e >= kGradW3 && e < kGradW3 + 128) f[kMlpW3 + e - kGradW3] = w;
  else if (e == kGradB3) f[kMlpB3] = w;
}

// Refresh the parameter block from FP32 master weights (after loading them).
__global__ void mlp_sync_kernel(void* params, const float* __restrict__ master) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kMlpGradFloats || e == kGradLoss) return;
  const float w = master[e];
  float* f = static_cast<float*>(params);
  __bf16* h = reinterpret_cast<__bf16*>(f + kMlpFloats);
  if (e >= kGradW1 && e < kGradW1 + 128 * 32) h[e - kGradW1] = (__bf16)w;
  else if (e >= kGradW2 && e < kGradW2 + 128 * 128) {
    const int jj = (e - kGradW2) >> 7, ii = (e - kGradW2) & 127;
    h[128 * 32 + jj * 128 + ii] = (__bf16)w;
    h[128 * 32 + 128 * 128 + ii * 128 + jj] = (__bf16)w;
  } else if (e >= kGradB1 && e < kGradB1 + 128) f[kMlpB1 + e - kGradB1] = w;
  else if (e >= kGradB2 && e < kGradB2 + 128) f[kMlpB2 + e - kGradB2] = w;
  else if (e >= kGradW3 && e < kGradW3 + 128) f[kMlpW3 + e - kGradW3] = w;
  else if (e == kGradB3) f[kMlpB3] = w;
}

// Per-feature mean and 1/std over n samples (two-stage, fixed order).
__global__ void feature_stats_kernel(const float* __restrict__ X, int n, float* __restrict__ partial) {
  // partial[block][64]: sums and sums of squares of the 32 features
  __shared__ float s1[256], s2[256];
  const int k = threadIdx.x & 31, lane_row = threadIdx.x >> 5;  // 8 rows per step
  float a = 0.f, b = 0.f;
  for (int s = blockIdx.x * 8 + lane_row; s < n; s += gridDim.x * 8) {
    const float v = X[(size_t)s * 32 + k];
    a += v;
    b += v * v;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  if (threadIdx.x < 32) {
    float A = 0.f, B = 0.f;
    for (int r = 0; r < 8; r++) {
      A += s1[r * 32 + k];
      B += s2[r * 32 + k];
    }
    partial[blockIdx.x * 64 + k] = A;
    partial[blockIdx.x * 64 + 32 + k] = B;
  }
}
__global__ void feature_stats_finish(const float* __restrict__ partial, int blocks, int n, void* params) {
  const int k = threadIdx.x;
  if (k >= 32) return;
  double A = 0.0, B = 0.0;
  for (int b = 0; b < blocks; b++) {
    A += partial[b * 64 + k];
    B += partial[b * 64 + 32 + k];
  }
  const double mean = A / n;
  const double var = B / n - mean * mean;
  float* f = static_cast<float*>(params);
  f[kMlpShift + k] = (float)mean;
  f[kMlpScale + k] = (float)(1.0 / sqrt(var > 1e-12 ? var : 1e-12));
}

// ---------------------------------------------------------------------------
// Greedy cover placement: the exact sequential greedy over candidates in
// visiting order (a candidate is accepted unless an accepted point lies closer
// than that point's radius), run in rounds.  Device state (int):
//   [0] cursor: every candidate visited before it is decided
//   [1] accepted so far          [2] first index accepted in the last round
//   [3] accepted in the last round   [4] size of the gathered batch
// gather: one workgroup collects the next `batch` undecided candidates after
//         the cursor, in visiting order;
// accept: one workgroup decides the batch against the points accepted earlier
//         in the same batch (earlier rounds are already folded into
//         `covered`), by a monotone fixed point that reproduces the
//         sequential rule; appends the accepted points;
// cover:  candidates within the radius of the points just accepted become
//         covered (brute force, or through the cell grid of grid candidates).
// Every squared-distance test is ((dx*dx + dy*dy) + dz*dz) < R*R in FP32 with
// dx = candidate - accepted point, so all three kernels decide alike.
// ---------------------------------------------------------------------------
RC_DEV bool within(float cx, float cy, float cz, float px, float py, float pz, float R) {
  const float dx = cx - px, dy = cy - py, dz = cz - pz;
  return dx * dx + dy * dy + dz * dz < R * R;
}
// Anisotropic points (Eq. radiusAniso3D): inside the ellipsoid of the form
// m = (m00, m01, m02, m11, m12, m22) iff d^T M d < 1, d = candidate - point,
// every product and sum in FP32 in this order.
RC_DEV float form_q(float dx, float dy, float dz, const float* __restrict__ m) {
  const float diag = (m[0] * (dx * dx) + m[3] * (dy * dy)) + m[5] * (dz * dz);
  const float off = (m[1] * (dx * dy) + m[2] * (dx * dz)) + m[4] * (dy * dz);
  return diag + 2.f * off;
}
RC_DEV bool within_form(float cx, float cy, float cz, float px, float py, float pz, const float* __restrict__ m) {
  return form_q(cx - px, cy - py, cz - pz, m) < 1.f;
}
// Is candidate c inside the valid region of point p with radius R (ball) or
// form m (ellipsoid, if m is not null)?
RC_DEV bool inside(float cx, float cy, float cz, float px, float py, float pz, float R, const float* __restrict__ m) {
  return m ? within_form(cx, cy, cz, px, py, pz, m) : within(cx, cy, cz, px, py, pz, R);
}

// Verdict of batch entry j from the entries i < j, one lane per i: 2 if an
// accepted entry covers j, 0 if an undecided one does (and no accepted one),
// else 1.  ps: x, y, z, R of the batch; form: the batch's ellipsoids
// ([batch][6]) or null (balls); status(i) reads entry i's state (0
// undecided, 1 accepted, 2 rejected).  Called by all 64 lanes of a wave.
template <typename Status>
RC_DEV int wave_verdict(const float4* ps, const float* __restrict__ form, int j, Status status, int lane) {
  const float4 pj = ps[j];
  bool und = false;
  for (int i0 = 0; i0 < j; i0 += kWave) {
    const int i = i0 + lane;
    bool acc = false;
    if (i < j) {
      const float4 pi = ps[i];
      if (inside(pj.x, pj.y, pj.z, pi.x, pi.y, pi.z, pi.w, form ? form + 6 * i : nullptr)) {
        const int si = status(i);
        acc = si == 1;
        und = und || si == 0;
      }
    }
    if (__ballot(acc)) return 2;
  }
  return __ballot(und) ? 0 : 1;
}

// Gather: the next `batch` undecided candidates in visiting order from the
// cursor state[0]; each chunk gives every thread kGatherPer consecutive
// candidates, ranks the undecided ones by a workgroup prefix sum, and cuts
// the chunk after the last one that fits.
constexpr int kGatherPer = 4;

__global__ __launch_bounds__(kPlaceThreads) void place_gather_kernel(const float* __restrict__ cand,
                                                                     const float* __restrict__ radius,
                                                                     const int* __restrict__ order, int C,
                                                                     const unsigned char* __restrict__ covered,
                                                                     int* __restrict__ state,
                                                                     int* __restrict__ batch_idx,
                                                                     float* __restrict__ batch_pos,
                                                                     float* __restrict__ batch_R, int batch) {
  __shared__ int wtot[kPlaceThreads / kWave];
  __shared__ int s_stop;
  const int t = threadIdx.x, lane = t & (kWave - 1), wv = t / kWave;
  constexpr int kChunk = kPlaceThreads * kGatherPer;
  for (int j = t; j < kPlaceMaxBatch; j += kPlaceThreads) state[kPlaceStatus + j] = 0;  // all undecided
  int cursor = state[0];
  int have = 0;
  while (cursor < C && have < batch) {
    int idx[kGatherPer];
    bool u[kGatherPer];
    int cnt = 0;
#pragma unroll
    for (int e = 0; e < kGatherPer; e++) {
      const long long k = (long long)cursor + t * kGatherPer + e;
      idx[e] = -1;
      u[e] = false;
      if (k < C) {
        idx[e] = order ? order[k] : (int)k;
        u[e] = !covered[idx[e]];
      }
      cnt += u[e] ? 1 : 0;
    }
    int incl = cnt;  // inclusive prefix of the counts within the wave
#pragma unroll
    for (int sh = 1; sh < kWave; sh <<= 1) {
      const int v = __shfl_up(incl, sh, kWave);
      if (lane >= sh) incl += v;
    }
    if (lane == kWave - 1) wtot[wv] = incl;
    __syncthreads();
    int off = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kPlaceThreads / kWave; w++) {
      const int v = wtot[w];
      total += v;
      off += (w < wv) ? v : 0;
    }
    const int rank0 = off + incl - cnt;  // rank of this thread's first undecided candidate in the chunk
    const int room = batch - have;
    int consumed = kChunk;
    if (total > room) {  // uniform across the workgroup
      if (rank0 <= room - 1 && room - 1 < rank0 + cnt) {
        int r = rank0;
#pragma unroll
        for (int e = 0; e < kGatherPer; e++)
          if (u[e]) {
            if (r == room - 1) s_stop = t * kGatherPer + e;  // the last candidate that fits
            r++;
          }
      }
      __syncthreads();
      consumed = s_stop + 1;
    }
    int r = rank0;
#pragma unroll
    for (int e = 0; e < kGatherPer; e++)
      if (u[e]) {
        if (r < room) {
          const int q = have + r, i = idx[e];
          batch_idx[q] = i;
          batch_pos[3 * q] = cand[3 * i];
          batch_pos[3 * q + 1] = cand[3 * i + 1];
          batch_pos[3 * q + 2] = cand[3 * i + 2];
          if (radius) batch_R[q] = radius[i];
        }
        r++;
      }
    have += total < room ? total : room;
    cursor = ((long long)cursor + consumed < C) ? cursor + consumed : C;
    __syncthreads();  // wtot and s_stop are rewritten by the next chunk
  }
  if (t == 0) {
    state[0] = cursor;
    state[4] = have;
  }
}

// One pass of the fixed point below, spread over many workgroups: each wave
// takes one undecided entry j, its lanes scan the entries i < j (positions
// staged in LDS), and j is rejected by an accepted coverer, accepted when all
// its coverers are rejected, else left undecided.  Status words
// (state[kPlaceStatus + j]) only ever go from undecided to decided, so passes
// racing with each other are harmless.
__global__ __launch_bounds__(kPlaceResolveThreads) void place_resolve_kernel(const float* __restrict__ cand,
                                                                           const int* __restrict__ batch_idx,
                                                                           const float* __restrict__ batch_R,
                                                                           const float* __restrict__ batch_form,
                                                                           int* __restrict__ state) {
  __shared__ float4 ps[kPlaceMaxBatch];
  constexpr int kWaves = kPlaceResolveThreads / kWave;
  const int m = min(state[4], kPlaceMaxBatch);
  const int j0 = blockIdx.x * kWaves;
  if (j0 >= m) return;
  const int jn = min(m, j0 + kWaves);  // entries i < jn are read
  for (int i = threadIdx.x; i < jn; i += kPlaceResolveThreads) {
    const int c = batch_idx[i];
    ps[i] = make_float4(cand[3 * c], cand[3 * c + 1], cand[3 * c + 2], batch_R[i]);
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int j = j0 + threadIdx.x / kWave;
  volatile int* stv = state + kPlaceStatus;
  if (j >= m || stv[j] != 0) return;
  const int verdict = wave_verdict(ps, batch_form, j, [stv](int i) { return stv[i]; }, lane);
  if (verdict != 0 && lane == 0) stv[j] = verdict;
}

// Batch entry j is accepted iff no accepted entry i < j covers it.  Each pass
// decides every entry whose covering predecessors are all decided: rejected
// as soon as one accepted predecessor covers it, accepted once every covering
// predecessor is rejected.  Decisions never change once made, so reading a
// neighbour's state while it is being written in the same pass only delays a
// decision; the smallest undecided entry is always decided in the next pass.
__global__ __launch_bounds__(kPlaceThreads) void place_accept_kernel(
    const float* __restrict__ cand, const int* __restrict__ batch_idx, const float* __restrict__ batch_R,
    const float* __restrict__ batch_form, unsigned char* __restrict__ covered, int* __restrict__ state,
    int* __restrict__ accepted, float* __restrict__ accepted_R, float* __restrict__ accepted_form,
    float* __restrict__ accepted_pos, const double* __restrict__ bval, const double* __restrict__ bgrad,
    double* __restrict__ cval, double* __restrict__ cgrad) {
  __shared__ float4 ps[kPlaceMaxBatch];  // x, y, z, R of the batch
  __shared__ unsigned char st[kPlaceMaxBatch];  // 0 undecided, 1 accepted, 2 rejected
  __shared__ int wtot[kPlaceThreads / kWave];
  __shared__ int s_und;
  const int t = threadIdx.x, lane = t & (kWave - 1), wv = t / kWave;
  const int m = min(state[4], kPlaceMaxBatch);  // gather never stores more
  const int base = state[1];
  for (int j = t; j < m; j += kPlaceThreads) {
    const int c = batch_idx[j];
    ps[j] = make_float4(cand[3 * c], cand[3 * c + 1], cand[3 * c + 2], batch_R[j]);
    st[j] = (unsigned char)state[kPlaceStatus + j];  // decided by the resolve passes, or 0
  }
  for (;;) {
    __syncthreads();
    if (t == 0) s_und = 0;
    __syncthreads();
    int und = 0;
    for (int j = wv; j < m; j += kPlaceThreads / kWave) {  // one wave per entry
      if (*(volatile unsigned char*)&st[j] != 0) continue;
      volatile unsigned char* stv = st;
      const int verdict = wave_verdict(ps, batch_form, j, [stv](int i) { return (int)stv[i]; }, lane);
      if (verdict != 0) {
        if (lane == 0) *(volatile unsigned char*)&st[j] = (unsigned char)verdict;
      } else {
        und++;
      }
    }
    if (und && lane == 0) atomicAdd(&s_und, und);
    __syncthreads();
    if (s_und == 0) break;
  }
  // append the accepted entries in batch order
  int prior = 0;
  for (int j0 = 0; j0 < m; j0 += kPlaceThreads) {
    const int j = j0 + t;
    const bool a = j < m && st[j] == 1;
    const unsigned long long mask = __ballot(a);
    if (lane == 0) wtot[wv] = __popcll(mask);
    __syncthreads();
    int off = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kPlaceThreads / kWave; w++) {
      const int v = wtot[w];
      total += v;
      off += (w < wv) ? v : 0;
    }
    if (a) {
      const int dst = base + prior + off + __popcll(mask & ((1ull << lane) - 1ull));
      const float4 p = ps[j];
      accepted[dst] = batch_idx[j];
      accepted_R[dst] = p.w;
      if (accepted_form) {
#pragma unroll
        for (int e = 0; e < 6; e++) accepted_form[6 * dst + e] = batch_form[6 * j + e];
      }
      if (accepted_pos) {
        accepted_pos[3 * dst] = p.x;
        accepted_pos[3 * dst + 1] = p.y;
        accepted_pos[3 * dst + 2] = p.z;
      }
      if (cval) {
        cval[2 * dst] = bval[2 * j];
        cval[2 * dst + 1] = bval[2 * j + 1];
#pragma unroll
        for (int e = 0; e < 6; e++) cgrad[6 * dst + e] = bgrad[6 * j + e];
      }
    }
    prior += total;
    __syncthreads();
  }
  // every batch member is decided; rejected ones are covered by an accepted one
  for (int j = t; j < m; j += kPlaceThreads) covered[batch_idx[j]] = 1;
  if (t == 0) {
    state[2] = base;
    state[3] = prior;
    state[1] = base + prior;
  }
}

// Cover by the accepted points b .. b + nn - 1 (a round's, or an explicit
// range): one candidate per thread; the points are staged through LDS 256 at
// a time, keeping only those whose bounding ball (the radius, or an
// ellipsoid's largest radius) reaches the box of the workgroup's candidates
// that are still uncovered.  Covering is an OR over the points, so the
// order of the tests does not change the result.
__global__ __launch_bounds__(256) void place_cover_kernel(const float* __restrict__ cand, int C,
                                                          unsigned char* __restrict__ covered,
                                                          const int* __restrict__ state,
                                                          const int* __restrict__ accepted,
                                                          const float* __restrict__ accepted_R,
                                                          const float* __restrict__ accepted_form, int first,
                                                          int count) {
  __shared__ float4 sp[256];
  __shared__ float sf[256 * 6];
  __shared__ float box[4][6];
  __shared__ int kept[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int b = first >= 0 ? first : state[2];
  const int nn = first >= 0 ? count : state[3];
  bool need = i < C && !covered[i];
  const float cx = need ? cand[3 * i] : 0.f, cy = need ? cand[3 * i + 1] : 0.f, cz = need ? cand[3 * i + 2] : 0.f;
  {
    const float inf = __builtin_huge_valf();
    const float b0 = wmin(need ? cx : inf), b1 = wmin(need ? cy : inf), b2 = wmin(need ? cz : inf);
    const float b3 = wmax(need ? cx : -inf), b4 = wmax(need ? cy : -inf), b5 = wmax(need ? cz : -inf);
    if (lane == 0) {
      box[wv][0] = b0, box[wv][1] = b1, box[wv][2] = b2;
      box[wv][3] = b3, box[wv][4] = b4, box[wv][5] = b5;
    }
  }
  __syncthreads();
  float lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    lo[a] = fminf(fminf(box[0][a], box[1][a]), fminf(box[2][a], box[3][a]));
    hi[a] = fmaxf(fmaxf(box[0][3 + a], box[1][3 + a]), fmaxf(box[2][3 + a], box[3][3 + a]));
  }
  for (int base = 0; base < nn; base += 256) {
    if (!__syncthreads_or(need)) break;  // every candidate of the workgroup is covered
    const int a = base + threadIdx.x;
    bool keep = false;
    float4 pr = make_float4(0.f, 0.f, 0.f, 0.f);
    if (a < nn) {
      const int p = accepted[b + a];
      pr = make_float4(cand[3 * p], cand[3 * p + 1], cand[3 * p + 2], accepted_R[b + a]);
      // a point inside by the FP32 test is within R (1 + 1e-6) of the centre
      // (balls, and ellipsoids of largest radius R); cull only finite R > 0
      const float ex = fmaxf(fmaxf(lo[0] - pr.x, pr.x - hi[0]), 0.f);
      const float ey = fmaxf(fmaxf(lo[1] - pr.y, pr.y - hi[1]), 0.f);
      const float ez = fmaxf(fmaxf(lo[2] - pr.z, pr.z - hi[2]), 0.f);
      const float rm = pr.w * 1.0001f;
      keep = !(pr.w > 0.f && pr.w < 3.0e38f) || !((ex * ex + ey * ey) + ez * ez > rm * rm);
    }
    const unsigned long long mask = __ballot(keep);
    if (lane == 0) kept[wv] = __popcll(mask);
    __syncthreads();
    int at = __popcll(mask & ((1ull << lane) - 1ull)), m = 0;
#pragma unroll
    for (int w = 0; w < 4; w++) {
      at += w < wv ? kept[w] : 0;
      m += kept[w];
    }
    if (keep) {
      sp[at] = pr;
      if (accepted_form)
        for (int e = 0; e < 6; e++) sf[6 * at + e] = accepted_form[6 * (b + a) + e];
    }
    __syncthreads();
    if (need) {
      for (int j = 0; j < m; j++) {
        const float4 q = sp[j];
        if (inside(cx, cy, cz, q.x, q.y, q.z, q.w, accepted_form ? sf + 6 * j : nullptr)) {
          covered[i] = 1;
          need = false;
          break;
        }
      }
    }
  }
}

// Grid candidates: candidate (ix, iy, iz) has index (ix * ny + iy) * nz + iz
// and lies in cell lo + [i, i + 1) * h.  One wavefront per accepted point
// visits the cells of the point's bounding box grown by one cell (so that
// rounding at cell faces cannot hide a candidate) and marks the candidates
// within its radius (or ellipsoid, whose bounding box sets the cells).
__global__ __launch_bounds__(256) void place_cover_grid_kernel(const float* __restrict__ cand, PlaceGrid g,
                                                               unsigned char* __restrict__ covered,
                                                               const int* __restrict__ state,
                                                               const int* __restrict__ accepted,
                                                               const float* __restrict__ accepted_R,
                                                               const float* __restrict__ accepted_form, int first,
                                                               int count) {
  const int lane = threadIdx.x & (kWave - 1);
  const int b = first >= 0 ? first : state[2];
  const int nn = first >= 0 ? count : state[3];
  for (int a = blockIdx.x * 4 + (threadIdx.x >> 6); a < nn; a += gridDim.x * 4) {
    const int p = accepted[b + a];
    const float px = cand[3 * p], py = cand[3 * p + 1], pz = cand[3 * p + 2];
    const float R = accepted_R[b + a];  // ball radius, or the ellipsoid's largest radius
    if (!(R > 0.f) || !(R < 3.0e38f)) continue;
    const float* m = accepted_form ? accepted_form + 6 * (b + a) : nullptr;
    // search half-extent per axis: R, or for an ellipsoid sqrt((M^-1)_dd) (its
    // bounding box, from the adjugate in FP64, never above R)
    float ext[3] = {R, R, R};
    if (m) {
      const double f0 = m[0], f1 = m[1], f2 = m[2], f3 = m[3], f4 = m[4], f5 = m[5];
      const double a00 = f3 * f5 - f4 * f4, a11 = f0 * f5 - f2 * f2, a22 = f0 * f3 - f1 * f1;
      const double det = f0 * a00 - f1 * (f1 * f5 - f2 * f4) + f2 * (f1 * f4 - f2 * f3);
      if (det > 0.0) {
        ext[0] = fminf(R, (float)(sqrt(fmax(a00 / det, 0.0)) * 1.0001));
        ext[1] = fminf(R, (float)(sqrt(fmax(a11 / det, 0.0)) * 1.0001));
        ext[2] = fminf(R, (float)(sqrt(fmax(a22 / det, 0.0)) * 1.0001));
      }
    }
    int lo3[3], n3[3];
    const float pc[3] = {px, py, pz};
    const float glo[3] = {g.lo.x, g.lo.y, g.lo.z}, gih[3] = {g.inv_h.x, g.inv_h.y, g.inv_h.z};
    const int gn[3] = {g.nx, g.ny, g.nz};
#pragma unroll
    for (int d = 0; d < 3; d++) {
      float f0 = floorf((pc[d] - ext[d] - glo[d]) * gih[d]) - 1.f;
      float f1 = floorf((pc[d] + ext[d] - glo[d]) * gih[d]) + 1.f;
      f0 = fmaxf(f0, 0.f);
      f1 = fminf(f1, (float)(gn[d] - 1));
      lo3[d] = (int)f0;
      n3[d] = (f1 >= f0) ? (int)f1 - (int)f0 + 1 : 0;
    }
    const int nyz = n3[1] * n3[2];
    const long long ncell = (long long)n3[0] * nyz;
    for (long long e = lane; e < ncell; e += kWave) {
      const int ee = (int)e;
      const int ix = lo3[0] + ee / nyz, r = ee % nyz;
      const int iy = lo3[1] + r / n3[2], iz = lo3[2] + r % n3[2];
      const int c = (ix * g.ny + iy) * g.nz + iz;
      if (covered[c]) continue;
      if (inside(cand[3 * c], cand[3 * c + 1], cand[3 * c + 2], px, py, pz, R, m)) covered[c] = 1;
    }
  }
}

// ---------------------------------------------------------------------------
// Cache interpolation (Eq. radianceTaylor): first-order Taylor from every
// cache point whose radius contains x', cubic kernel w = 3d^2 - 2d^3,
// d = 1 - |x' - x_k| / R_k; FP64 accumulation.  Every query visits the cache
// points in index order; a workgroup skips the balls that cannot reach the
// bounding box of its 256 queries (conservative FP32 test, with the kept
// points compacted in order, so each query sums the same points in the same
// order as a visit of all of them).  Anisotropic points: membership
// d^T M d < 1 (FP32) and d = 1 - sqrt(d^T M d) (FP64); no culling.
// ---------------------------------------------------------------------------
// cval [K][2] and cgrad [K][2][3] are records (the two channels are summed);
// if ref [Q][2] is given, block b writes (sum (L - L_ref)^2, sum L_ref^2) over
// its covered queries to err[2b], err[2b+1].
// LOG: the comparison method's extrapolation (Eq. jaroszExtrapolation): the
// same weights over first-order expansions of ln L (value ln L_k, gradient
// grad L_k / L_k; points with L_k <= 0 take no part), exponentiated.
template <bool LOG>
__global__ __launch_bounds__(256) void interp_kernel(const float* __restrict__ cpos, const double* __restrict__ cval,
                                                     const double* __restrict__ cgrad, const float* __restrict__ cR,
                                                     const float* __restrict__ cform, int K,
                                                     const float* __restrict__ q, int Q, double* __restrict__ out,
                                                     int* __restrict__ hits, const double* __restrict__ ref,
                                                     double* __restrict__ err) {
  __shared__ double rs[2][256];
  __shared__ float sp[256 * 4];
  __shared__ float sf[256 * 6];
  __shared__ double sv[256 * 4];
  __shared__ float box[4][6];  // per wave: min x, y, z, max x, y, z of its queries
  __shared__ int kept[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const float qx = i < Q ? q[3 * i] : 0.f, qy = i < Q ? q[3 * i + 1] : 0.f, qz = i < Q ? q[3 * i + 2] : 0.f;
  {
    const float inf = __builtin_huge_valf();
    const float b0 = wmin(i < Q ? qx : inf), b1 = wmin(i < Q ? qy : inf), b2 = wmin(i < Q ? qz : inf);
    const float b3 = wmax(i < Q ? qx : -inf), b4 = wmax(i < Q ? qy : -inf), b5 = wmax(i < Q ? qz : -inf);
    if (lane == 0) {
      box[wv][0] = b0, box[wv][1] = b1, box[wv][2] = b2;
      box[wv][3] = b3, box[wv][4] = b4, box[wv][5] = b5;
    }
  }
  __syncthreads();
  float lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    lo[a] = fminf(fminf(box[0][a], box[1][a]), fminf(box[2][a], box[3][a]));
    hi[a] = fmaxf(fmaxf(box[0][3 + a], box[1][3 + a]), fmaxf(box[2][3 + a], box[3][3 + a]));
  }
  double num = 0.0, den = 0.0;
  int nh = 0;
  for (int base = 0; base < K; base += 256) {
    const int k = base + threadIdx.x;
    bool keep = false;
    float c0 = 0.f, c1 = 0.f, c2 = 0.f, cr = 0.f;
    if (k < K) {
      c0 = cpos[3 * k], c1 = cpos[3 * k + 1], c2 = cpos[3 * k + 2], cr = cform ? 0.f : cR[k];
      if (LOG && !(cval[2 * k] + cval[2 * k + 1] > 0.0)) {
        keep = false;
      } else if (cform) {
        keep = true;
      } else {
        // distance from the ball's centre to the queries' box; a query inside
        // the ball by the FP32 test is no further than R (1 + 1e-6) from it,
        // so a margin of 1e-4 R keeps every ball that can hold one
        const float ex = fmaxf(fmaxf(lo[0] - c0, c0 - hi[0]), 0.f);
        const float ey = fmaxf(fmaxf(lo[1] - c1, c1 - hi[1]), 0.f);
        const float ez = fmaxf(fmaxf(lo[2] - c2, c2 - hi[2]), 0.f);
        const float rm = cr * 1.0001f + 1e-30f;
        keep = !((ex * ex + ey * ey) + ez * ez > rm * rm);
      }
    }
    const unsigned long long mask = __ballot(keep);
    __syncthreads();  // the previous tile's LDS rows are read
    if (lane == 0) kept[wv] = __popcll(mask);
    __syncthreads();
    int at = __popcll(mask & ((1ull << lane) - 1ull)), m = 0;
#pragma unroll
    for (int w = 0; w < 4; w++) {
      at += w < wv ? kept[w] : 0;
      m += kept[w];
    }
    if (keep) {
      sp[4 * at] = c0;
      sp[4 * at + 1] = c1;
      sp[4 * at + 2] = c2;
      sp[4 * at + 3] = cr;
      if (cform)
        for (int e = 0; e < 6; e++) sf[6 * at + e] = cform[6 * k + e];
      const double lv = cval[2 * k] + cval[2 * k + 1];
      const double gx = cgrad[6 * k] + cgrad[6 * k + 3], gy = cgrad[6 * k + 1] + cgrad[6 * k + 4],
                   gz = cgrad[6 * k + 2] + cgrad[6 * k + 5];
      sv[4 * at] = LOG ? log(lv) : lv;
      sv[4 * at + 1] = LOG ? gx / lv : gx;
      sv[4 * at + 2] = LOG ? gy / lv : gy;
      sv[4 * at + 3] = LOG ? gz / lv : gz;
    }
    __syncthreads();
    for (int j = 0; j < m; j++) {
      const float dx = qx - sp[4 * j], dy = qy - sp[4 * j + 1], dz = qz - sp[4 * j + 2], R = sp[4 * j + 3];
      bool in;
      double d;  // 1 - normalised distance: 1 at the point, 0 on the region's boundary
      if (cform) {
        const float* m = sf + 6 * j;
        in = form_q(dx, dy, dz, m) < 1.f;
        // the weight from the form in FP64 (the FP32 value cancels near the point)
        const double ex = (double)qx - (double)sp[4 * j], ey = (double)qy - (double)sp[4 * j + 1],
                     ez = (double)qz - (double)sp[4 * j + 2];
        const double diag = ((double)m[0] * (ex * ex) + (double)m[3] * (ey * ey)) + (double)m[5] * (ez * ez);
        const double off = ((double)m[1] * (ex * ey) + (double)m[2] * (ex * ez)) + (double)m[4] * (ey * ez);
        d = 1.0 - sqrt(fmax(diag + 2.0 * off, 0.0));
      } else {
        const float d2 = dx * dx + dy * dy + dz * dz;
        in = d2 < R * R;
        d = 1.0 - sqrt((double)d2) / (double)R;
      }
      if (in) {
        const double w = 3.0 * d * d - 2.0 * d * d * d;
        const double L = sv[4 * j] + sv[4 * j + 1] * dx + sv[4 * j + 2] * dy + sv[4 * j + 3] * dz;
        num += w * L;
        den += w;
        nh++;
      }
    }
  }
  const double L = den > 0.0 ? (LOG ? exp(num / den) : num / den) : 0.0;
  if (i < Q) {
    out[i] = L;
    if (hits) hits[i] = den > 0.0 ? nh : 0;
  }
  if (ref) {
    const double Lr = (i < Q && den > 0.0) ? ref[2 * i] + ref[2 * i + 1] : 0.0;
    const double dv = (i < Q && den > 0.0) ? (L - Lr) : 0.0;
    rs[0][threadIdx.x] = dv * dv;
    rs[1][threadIdx.x] = Lr * Lr;
    __syncthreads();
    for (int st = 128; st >= 1; st >>= 1) {
      if (threadIdx.x < st) {
        rs[0][threadIdx.x] += rs[0][threadIdx.x + st];
        rs[1][threadIdx.x] += rs[1][threadIdx.x + st];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      err[2 * blockIdx.x] = rs[0][0];
      err[2 * blockIdx.x + 1] = rs[1][0];
    }
  }
}

// Ellipsoid of an anisotropic point from the axes the radius kernel writes
// ([12]: R_1..R_3, then the unit eigenvectors as rows): form entries
// sum_i (v_i[a] v_i[b]) / (R_i R_i) in FP64 (axis order), rounded to FP32,
// and the largest radius (bounds the ellipsoid).
__global__ void ellipsoid_form_kernel(const float* __restrict__ axes, int K, float* __restrict__ form,
                                      float* __restrict__ Rmax) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const float* a = axes + 12 * k;
  double R2[3], v[3][3];
  for (int i = 0; i < 3; i++) {
    R2[i] = (double)a[i] * (double)a[i];
    for (int c = 0; c < 3; c++) v[i][c] = (double)a[3 + 3 * i + c];
  }
  const int ea[6] = {0, 0, 0, 1, 1, 2}, eb[6] = {0, 1, 2, 1, 2, 2};
  for (int e = 0; e < 6; e++) {
    const double t0 = (v[0][ea[e]] * v[0][eb[e]]) / R2[0];
    const double t1 = (v[1][ea[e]] * v[1][eb[e]]) / R2[1];
    const double t2 = (v[2][ea[e]] * v[2][eb[e]]) / R2[2];
    form[6 * k + e] = (float)((t0 + t1) + t2);
  }
  if (Rmax) Rmax[k] = fmaxf(fmaxf(a[0], a[1]), a[2]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_probe(const ProbeArgs& a, int depth, hipStream_t s) {
  if (a.C <= 0) return hipSuccess;
  int grid = a.C < 65536 ? a.C : 65536;
  const int st = stack_variant(depth);
  if (st <= 16) hipLaunchKernelGGL(probe_kernel<16>, dim3(grid), dim3(kWave), 0, s, a);
  else if (st <= 32) hipLaunchKernelGGL(probe_kernel<32>, dim3(grid), dim3(kWave), 0, s, a);
  else if (st <= 48) hipLaunchKernelGGL(probe_kernel<48>, dim3(grid), dim3(kWave), 0, s, a);
  else hipLaunchKernelGGL(probe_kernel<64>, dim3(grid), dim3(kWave), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const void* params, const float* X, int n, float* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int blocks = (n + 63) / 64;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(mlp_forward_kernel<false>, dim3(blocks), dim3(256), 0, s, params, X, n, out, 1.f, 0.f, 0.f);
  return hipGetLastError();
}

hipError_t launch_mlp_radius(const void* params, const float* X, int n, float safety, float r_min, float r_max,
                             float* R, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int blocks = (n + 63) / 64;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(mlp_forward_kernel<true>, dim3(blocks), dim3(256), 0, s, params, X, n, R, safety, r_min, r_max);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const void* params, const float* X, const float* target, int n, float* partial,
                           hipStream_t s) {
  const int tiles = (n + 63) / 64;
  if (tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(tiles), dim3(256), 0, s, params, X, target, n, 1.0f / (float)n, partial);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(void* params, float* master, float* m, float* v, const float* partial, int tiles, float lr,
                           float b1c, float b2c, float* grad_out, float* loss_out, hipStream_t s) {
  const int blocks = (kMlpGradFloats + 255) / 256;
  hipLaunchKernelGGL(mlp_adam_kernel, dim3(blocks), dim3(256), 0, s, params, master, m, v, partial, tiles, lr, b1c, b2c,
                     grad_out, loss_out);
  return hipGetLastError();
}

hipError_t launch_feature_stats(const float* X, int n, float* partial, int blocks, void* params, hipStream_t s) {
  hipLaunchKernelGGL(feature_stats_kernel, dim3(blocks), dim3(256), 0, s, X, n, partial);
  hipLaunchKernelGGL(feature_stats_finish, dim3(1), dim3(64), 0, s, partial, blocks, n, params);
  return hipGetLastError();
}

hipError_t launch_place_gather(const float* cand, const float* radius, const int* order, int C,
                               const unsigned char* covered, int* state, int* batch_idx, float* batch_pos,
                               float* batch_R, int batch, hipStream_t s) {
  hipLaunchKernelGGL(place_gather_kernel, dim3(1), dim3(kPlaceThreads), 0, s, cand, radius, order, C, covered, state,
                     batch_idx, batch_pos, batch_R, batch);
  return hipGetLastError();
}

hipError_t launch_place_accept(const float* cand, const int* batch_idx, const float* batch_R, const float* batch_form,
                               unsigned char* covered, int* state, int* accepted, float* accepted_R,
                               float* accepted_form, float* accepted_pos, const double* bval, const double* bgrad,
                               double* cval, double* cgrad, hipStream_t s) {
  // a few wide passes decide almost every entry; the one-workgroup kernel
  // finishes whatever chains of coverers remain and appends the result
  for (int pass = 0; pass < kPlacePasses; pass++)
    hipLaunchKernelGGL(place_resolve_kernel, dim3(kPlaceMaxBatch / (kPlaceResolveThreads / kWave)),
                       dim3(kPlaceResolveThreads), 0, s, cand, batch_idx, batch_R, batch_form, state);
  hipLaunchKernelGGL(place_accept_kernel, dim3(1), dim3(kPlaceThreads), 0, s, cand, batch_idx, batch_R, batch_form,
                     covered, state, accepted, accepted_R, accepted_form, accepted_pos, bval, bgrad, cval, cgrad);
  return hipGetLastError();
}

hipError_t launch_place_cover(const float* cand, int C, unsigned char* covered, const int* state, const int* accepted,
                              const float* accepted_R, const float* accepted_form, int first, int count,
                              hipStream_t s) {
  const int blocks = (C + 255) / 256;
  if (blocks > 0)
    hipLaunchKernelGGL(place_cover_kernel, dim3(blocks), dim3(256), 0, s, cand, C, covered, state, accepted, accepted_R,
                       accepted_form, first, count);
  return hipGetLastError();
}

hipError_t launch_place_cover_grid(const float* cand, const PlaceGrid& g, unsigned char* covered, const int* state,
                                   const int* accepted, const float* accepted_R, const float* accepted_form, int first,
                                   int count, int max_points, hipStream_t s) {
  int pts = first >= 0 ? count : max_points;
  if (pts <= 0) return hipSuccess;
  int blocks = (pts + 3) / 4;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(place_cover_grid_kernel, dim3(blocks), dim3(256), 0, s, cand, g, covered, state, accepted,
                     accepted_R, accepted_form, first, count);
  return hipGetLastError();
}

hipError_t launch_interp(const float* cpos, const double* cval, const double* cgrad, const float* cR,
                         const float* cform, int K, const float* q, int Q, double* out, int* hits, const double* ref,
                         double* err, hipStream_t s) {
  const int blocks = (Q + 255) / 256;
  if (blocks > 0)
    hipLaunchKernelGGL(interp_kernel<false>, dim3(blocks), dim3(256), 0, s, cpos, cval, cgrad, cR, cform, K, q, Q,
                       out, hits, ref, err);
  return hipGetLastError();
}

hipError_t launch_interp_log(const float* cpos, const double* cval, const double* cgrad, const float* cR, int K,
                             const float* q, int Q, double* out, int* hits, hipStream_t s) {
  const int blocks = (Q + 255) / 256;
  if (blocks > 0)
    hipLaunchKernelGGL(interp_kernel<true>, dim3(blocks), dim3(256), 0, s, cpos, cval, cgrad, cR, nullptr, K, q, Q,
                       out, hits, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_ellipsoid_form(const float* axes, int K, float* form, float* Rmax, hipStream_t s) {
  const int blocks = (K + 255) / 256;
  if (blocks > 0) hipLaunchKernelGGL(ellipsoid_form_kernel, dim3(blocks), dim3(256), 0, s, axes, K, form, Rmax);
  return hipGetLastError();
}

hipError_t launch_mlp_init(void* params, float* state, unsigned long long seed, hipStream_t s) {
  hipLaunchKernelGGL(mlp_init_kernel, dim3((kMlpGradFloats + 255) / 256), dim3(256), 0, s, params, state, seed);
  return hipGetLastError();
}

hipError_t launch_mlp_sync(void* params, const float* master, hipStream_t s) {
  hipLaunchKernelGGL(mlp_sync_kernel, dim3((kMlpGradFloats + 255) / 256), dim3(256), 0, s, params, master);
  return hipGetLastError();
}

}  // namespace rc
