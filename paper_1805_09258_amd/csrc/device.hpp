// device.hpp -- device-side building blocks of the record kernel (gfx950).
//
// The whole library is compiled with -ffp-contract=off: the FP32 decision
// formulas below (direction rounding, ray/triangle test, shadow-ray origins,
// ring distances, quad diagonals) must round exactly as written, because the
// same published formulas decide the same discrete events on the CPU
// reference.  Where fused multiply-adds are wanted (box slab tests), they are
// written explicitly with fmaf.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define RC_DEV __device__ __forceinline__

namespace rc {

constexpr double kPi = 3.14159265358979323846;
constexpr float kPiF = 3.14159265358979323846f;
constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Counter-based random numbers: splitmix64 (Steele, Lea, Flood 2014) used as
// a hash of (seed, record, sample index, dimension).
// ---------------------------------------------------------------------------
RC_DEV uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
RC_DEV uint64_t record_key(uint64_t seed, uint64_t rec) { return splitmix64(splitmix64(seed) ^ rec); }
RC_DEV float uniform24(uint64_t key, uint64_t idx, uint64_t dim) {
  return (float)(splitmix64(splitmix64(key ^ idx) ^ dim) >> 40) * 0x1p-24f;
}
constexpr uint64_t kRingIdx = 0xFFFFFFFFull;

// Jittered sample of stratum (a, b) of the equal-solid-angle (z, phi) grid,
// evaluated in FP64 and rounded once to FP32 (Sec. 6, Implementation).
RC_DEV float3 stratum_direction(uint64_t key, int a, int b, int nth, int nph) {
  uint64_t idx = (uint64_t)a * (uint64_t)nph + (uint64_t)b;
  double xi0 = uniform24(key, idx, 0), xi1 = uniform24(key, idx, 1);
  double u = ((double)a + xi0) / (double)nth;
  double v = ((double)b + xi1) / (double)nph;
  double z = 1.0 - 2.0 * u;
  double phi = (2.0 * kPi) * v;
  double zz = z * z;
  double st = sqrt(fmax(0.0, 1.0 - zz));
  return make_float3((float)(st * cos(phi)), (float)(st * sin(phi)), (float)z);
}

RC_DEV float ring_distance(int i, float xi, float step) { return ((float)i + xi) * step; }

// Set bits of a wavefront mask below the calling lane (mbcnt: nothing held
// across loop iterations, unlike a materialised lane mask).
RC_DEV int mask_rank(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// ---------------------------------------------------------------------------
// FP32 vector helpers (decision formulas: no fused operations)
// ---------------------------------------------------------------------------
RC_DEV float3 sub3(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
RC_DEV float3 cross3(float3 a, float3 b) {
  return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
RC_DEV float dot3(float3 a, float3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
RC_DEV float3 axpy3(float t, float3 w, float3 x) { return make_float3(x.x + t * w.x, x.y + t * w.y, x.z + t * w.z); }
RC_DEV float det3(float3 a, float3 b, float3 c) { return dot3(a, cross3(b, c)); }

// Watertight ray/triangle test (Woop, Benthin and Wald, "Watertight
// Ray/Triangle Intersection", JCGT 2(1), 2013), written without divisions.
// kz is the axis of the largest |d| component (ties to the lower axis) and
// (kx, ky) = (kz + 1, kz + 2) mod 3.  Each vertex v is projected along the ray
// to the 2-D point
//   p(v) = (d_kz a_kx - d_kx a_kz,  d_kz a_ky - d_ky a_kz),   a = v - o,
// in FP32 (d_kz times the sheared coordinates of the published test).  The
// edge functions U = p(v1) x p(v2), V = p(v2) x p(v0), W = p(v0) x p(v1) are
// FP64 from the FP32 points: the products are exact and one rounding keeps
// each sign exact, so which side of every projected edge the ray passes is
// decided exactly and a ray through an edge shared by two triangles of a
// closed mesh is never lost, at any angle.  Hit iff U, V, W are all >= 0 or
// all <= 0 and D = U + V + W != 0; then
//   t = (U a_kz(v0) + V a_kz(v1) + W a_kz(v2)) / (D d_kz)
// in FP64, rounded once to FP32, and tmin < t < tmax.  D d_kz has the sign of
// d . ((v1 - v0) x (v2 - v0)), so front (the ray travels against that normal)
// is D d_kz < 0.
//
// The ray is kept in the permuted frame (x, y, z) = (kx, ky, kz), and the
// triangle array holds three copies of every triangle, copy k with its
// vertices in the frame of kz = k, so the test itself selects nothing.
struct WtRay {
  float3 o, d;  // origin and direction, permuted
  int kz;
};
RC_DEV float3 permute3(float3 v, int kz) {
  const bool b0 = kz == 0, b1 = kz == 1;
  return make_float3(b0 ? v.y : (b1 ? v.z : v.x), b0 ? v.z : (b1 ? v.x : v.y), b0 ? v.x : (b1 ? v.y : v.z));
}
RC_DEV WtRay wt_ray(float3 o, float3 d) {
  const float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
  int k = 0;
  float m = ax;
  if (ay > m) {
    k = 1;
    m = ay;
  }
  if (az > m) k = 2;
  WtRay r;
  r.o = permute3(o, k);
  r.d = permute3(d, k);
  r.kz = k;
  return r;
}
// Triangle record in the copy of the ray's kz: A = (v0, id bits), B = (v1, 0),
// C = (v2, 0), each vertex permuted to (v_kx, v_ky, v_kz).
RC_DEV bool hit_triangle(const WtRay& r, float4 A, float4 B, float4 C, float tmin, float tmax, float& tout,
                         bool& front) {
  const float3 a0 = sub3(make_float3(A.x, A.y, A.z), r.o);
  const float3 a1 = sub3(make_float3(B.x, B.y, B.z), r.o);
  const float3 a2 = sub3(make_float3(C.x, C.y, C.z), r.o);
  const double px0 = r.d.z * a0.x - r.d.x * a0.z, py0 = r.d.z * a0.y - r.d.y * a0.z;
  const double px1 = r.d.z * a1.x - r.d.x * a1.z, py1 = r.d.z * a1.y - r.d.y * a1.z;
  const double px2 = r.d.z * a2.x - r.d.x * a2.z, py2 = r.d.z * a2.y - r.d.y * a2.z;
  const double U = px1 * py2 - py1 * px2;
  const double V = px2 * py0 - py2 * px0;
  const double W = px0 * py1 - py0 * px1;
  if ((U < 0.0 || V < 0.0 || W < 0.0) && (U > 0.0 || V > 0.0 || W > 0.0)) return false;
  const double D = (U + V) + W;
  if (D == 0.0) return false;
  const double num = (U * (double)a0.z + V * (double)a1.z) + W * (double)a2.z;
  const double den = D * (double)r.d.z;
  const float t = (float)(num / den);
  if (!(t > tmin && t < tmax)) return false;
  tout = t;
  front = den < 0.0;
  return true;
}

// Per-light triangle bins: for the segment o -> o + d ending at light l
// (wr = wt_ray(o, d)), the bin of each level that holds the direction from
// the light to o, e = -d: face 2 kz + (e_kz > 0 ? 0 : 1), tangent coordinates
// (e_kx, e_ky) / |e_kz|, nested levels of B >> 2k bins per side.  h[k] is
// the index of that bin's header (first entry, its distance bits; the next
// word starts the next bin).  Returns the level count (0 if o is at the
// light).  desc[2 l] = (B, levels, level offset 0, 1), desc[2 l + 1] =
// (level offset 2, 3, -, -).
RC_DEV int lb_bins(const int4* __restrict__ desc, int l, const WtRay& wr, int (&h)[4]) {
  const int4 ds0 = desc[2 * l], ds1 = desc[2 * l + 1];
  const int B = ds0.x, nlev = ds0.y;
  const float ez = -wr.d.z, ex = -wr.d.x, ey = -wr.d.y;
  if (!(fabsf(ez) > 0.0f)) return 0;
  const float ia = 1.0f / fabsf(ez);
  const int face = 2 * wr.kz + (ez > 0.0f ? 0 : 1);
  const float hb = 0.5f * (float)B;
  const int iu = min(max((int)((ex * ia + 1.0f) * hb), 0), B - 1);
  const int iv = min(max((int)((ey * ia + 1.0f) * hb), 0), B - 1);
  const int lo[4] = {ds0.z, ds0.w, ds1.x, ds1.y};
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int Bk = B >> (2 * k);
    h[k] = lo[k] + 2 * ((face * Bk + (iu >> (2 * k))) * Bk + (iv >> (2 * k)));
  }
  return nlev;
}

// FP32 distance to the exit of the medium box (rays that hit nothing).
RC_DEV float box_exit(float3 o, float3 d, float3 lo, float3 hi) {
  float t = __builtin_huge_valf();
  if (d.x > 0.0f) t = fminf(t, (hi.x - o.x) / d.x); else if (d.x < 0.0f) t = fminf(t, (lo.x - o.x) / d.x);
  if (d.y > 0.0f) t = fminf(t, (hi.y - o.y) / d.y); else if (d.y < 0.0f) t = fminf(t, (lo.y - o.y) / d.y);
  if (d.z > 0.0f) t = fminf(t, (hi.z - o.z) / d.z); else if (d.z < 0.0f) t = fminf(t, (lo.z - o.z) / d.z);
  return t > 0.0f ? t : 0.0f;
}

// The same exit distance in FP64 (the continuous value of an escaping ray).
RC_DEV double box_exit64(float3 o, float3 d, float3 lo, float3 hi) {
  double t = 1e300;
  if (d.x > 0.0f) t = fmin(t, ((double)hi.x - o.x) / d.x); else if (d.x < 0.0f) t = fmin(t, ((double)lo.x - o.x) / d.x);
  if (d.y > 0.0f) t = fmin(t, ((double)hi.y - o.y) / d.y); else if (d.y < 0.0f) t = fmin(t, ((double)lo.y - o.y) / d.y);
  if (d.z > 0.0f) t = fmin(t, ((double)hi.z - o.z) / d.z); else if (d.z < 0.0f) t = fmin(t, ((double)lo.z - o.z) / d.z);
  return t > 0.0 ? t : 0.0;
}

// ---------------------------------------------------------------------------
// BVH traversal.  Boxes are padded by more than the FP32 error of an accepted
// hit, so pruning never removes a triangle whose hit test would pass: the
// closest hit (smallest t, ties to the lowest triangle id) and the any-hit
// answer equal those of testing every triangle.
// The per-lane stack lives in LDS: entry k of lane l at stk[k * 64] (stk is
// pre-offset by the lane).
// ---------------------------------------------------------------------------
struct TraceCount {
  uint32_t nodes = 0, tris = 0;
};

RC_DEV int leaf_first(int code) { return (~code) >> 3; }
RC_DEV int leaf_count(int code) { return ((~code) & 7) + 1; }

RC_DEV void ray_inv(float3 d, float3 o, float3& inv, float3& oi) {
  const float eps = 1e-20f;
  float dx = fabsf(d.x) > eps ? d.x : copysignf(eps, d.x);
  float dy = fabsf(d.y) > eps ? d.y : copysignf(eps, d.y);
  float dz = fabsf(d.z) > eps ? d.z : copysignf(eps, d.z);
  // hardware reciprocal (1 ulp): only the padded-box slab tests use it
  inv = make_float3(__builtin_amdgcn_rcpf(dx), __builtin_amdgcn_rcpf(dy), __builtin_amdgcn_rcpf(dz));
  oi = make_float3(o.x * inv.x, o.y * inv.y, o.z * inv.z);
}

// slab test of one child box; returns the entry distance or +inf on a miss
RC_DEV float slab(float lx, float hx, float ly, float hy, float lz, float hz, float3 inv, float3 oi, float t0,
                  float t1) {
  float ax = fmaf(lx, inv.x, -oi.x), bx = fmaf(hx, inv.x, -oi.x);
  float ay = fmaf(ly, inv.y, -oi.y), by = fmaf(hy, inv.y, -oi.y);
  float az = fmaf(lz, inv.z, -oi.z), bz = fmaf(hz, inv.z, -oi.z);
  float tn = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), t0));
  float tf = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), t1));
  return tn <= tf ? tn : __builtin_huge_valf();
}

// Closest hit (smallest t, ties to the lowest triangle id): one node or one
// triangle per loop iteration, with a single stack pop and dispatch for both
// kinds of step.  leaf_batch 0: every lane takes its next step in every
// iteration.  leaf_batch k > 0: the lanes still tracing take the same kind of
// step in an iteration, triangle tests once at least k of them wait at a leaf
// (or none has a node step left), node steps otherwise.  Testing a leaf later
// only means nodes are culled against a larger best distance meanwhile; the
// result is the same.
template <bool COUNT>
RC_DEV void trace_closest(const float4* __restrict__ nodes, const float4* __restrict__ tris, int tri_stride, float3 o,
                          float3 d, int* stk, int leaf_batch, int& best_id, float& best_t, bool& best_front,
                          TraceCount& cnt) {
  constexpr int kEnd = 0x7fffffff, kStay = 0x7ffffffe;
  const WtRay wr = wt_ray(o, d);
  const float4* const tk = tris + wr.kz * tri_stride;
  float3 inv, oi;
  ray_inv(d, o, inv, oi);
  best_id = -1;
  best_t = __builtin_huge_valf();
  best_front = false;
  int sp = 0, node = 0, lf = 0, ln = 0;
  while (true) {
    const uint64_t here = __ballot(true), at_leaf = __ballot(ln > 0);
    const bool tri_step = at_leaf != 0ull && (__popcll(at_leaf) >= leaf_batch || at_leaf == here);
    if (leaf_batch > 0 && (ln > 0) != tri_step) continue;
    const float4* src = (ln > 0) ? (tk + 3 * lf) : (nodes + 4 * node);
    const float4 q0 = src[0], q1 = src[1], q2 = src[2], q3 = src[3];
    int nx = kStay;
    bool pop = false;
    if (ln > 0) {
      if (COUNT) cnt.tris++;
      float t;
      bool fr;
      if (hit_triangle(wr, q0, q1, q2, 0.0f, __builtin_huge_valf(), t, fr)) {
        const int id = __float_as_int(q0.w);
        if (t < best_t || (t == best_t && id < best_id)) {
          best_t = t;
          best_id = id;
          best_front = fr;
        }
      }
      lf++;
      ln--;
      pop = ln == 0;
    } else {
      if (COUNT) cnt.nodes++;
      const float ta = slab(q0.x, q0.y, q0.z, q0.w, q2.x, q2.y, inv, oi, 0.0f, best_t);
      const float tb = slab(q1.x, q1.y, q1.z, q1.w, q2.z, q2.w, inv, oi, 0.0f, best_t);
      const int ca = __float_as_int(q3.x), cb = __float_as_int(q3.y);
      const bool ha = ta < __builtin_huge_valf(), hb = tb < __builtin_huge_valf();
      if (ha && hb) {
        nx = ta <= tb ? ca : cb;
        stk[sp++ * kWave] = ta <= tb ? cb : ca;
      } else if (ha || hb) {
        nx = ha ? ca : cb;
      } else {
        pop = true;
      }
    }
    if (pop) nx = sp == 0 ? kEnd : stk[--sp * kWave];
    if (nx == kEnd) return;
    if (nx != kStay) {
      if (nx < 0) {
        lf = leaf_first(nx);
        ln = leaf_count(nx);
      } else {
        node = nx;
      }
    }
  }
}

// Is the segment o -> light l unblocked?  From the light bins: the segment
// reads one header per level and then only the entries within its reach,
// nearest to the light first, stopping at the first hit (the entry of the
// vertex's own triangle `skip` excepted); the lists whose first entry is
// within reach are kept as (first, end) pairs in the lane's stack slots
// (stride 64) and walked in one loop, so a wavefront runs as long as its
// longest walk, not as the sum over levels of each level's longest list.
template <bool COUNT>
RC_DEV bool light_visible(float4 Lp, int l, const int4* lb_desc, const int* lb_offs, const float4* lb_ent, float3 o,
                          int skip, int* stk, TraceCount& tc) {
  const float3 d = make_float3(Lp.x - o.x, Lp.y - o.y, Lp.z - o.z);
  const WtRay wr = wt_ray(o, d);
  int h[4];
  const int nlev = lb_bins(lb_desc, l, wr, h);
  // the largest stored distance from the light that can still block
  const float reach = __builtin_amdgcn_sqrtf(dot3(d, d)) * (1.0f + 0x1p-20f);
  int nl = 0;
  for (int q = 0; q < nlev; q++) {
    if (COUNT) tc.nodes++;
    const int* hd = lb_offs + h[q];
    if (__int_as_float(hd[1]) <= reach) {
      stk[(2 * nl) * kWave] = hd[0];
      stk[(2 * nl + 1) * kWave] = hd[2];
      nl++;
    }
  }
  bool live = nl > 0;
  int cur = live ? stk[0] : 0, end = live ? stk[kWave] : 0, nxt = 1;
  while (live) {
    if (COUNT) tc.tris++;
    const float4* en = lb_ent + 3 * cur;
    const float4 q0 = en[0], q1 = en[1], q2 = en[2];
    float t;
    bool fr;
    if (__float_as_int(q0.w) != skip && hit_triangle(wr, q0, q1, q2, 1e-4f, 1.0f, t, fr)) {
      return false;
    } else if (++cur == end || q2.w > reach) {  // this list is done: the next one, if any
      if (nxt < nl) {
        cur = stk[(2 * nxt) * kWave];
        end = stk[(2 * nxt + 1) * kWave];
        nxt++;
      } else {
        live = false;
      }
    }
  }
  return true;
}

// Visibility bits of one vertex o (bit l: the segment to light l is
// unblocked), light by light as light_visible walks them (the same
// decisions, written as one loop so the record kernel keeps its register
// allocation).  A surface vertex (skip = its own triangle, nrm = its lit-side
// normal) gets no bit for a light behind its lit side.
template <bool COUNT>
RC_DEV int light_bits(const float4* lights, int n_lights, const int4* lb_desc, const int* lb_offs,
                      const float4* lb_ent, float3 o, int skip, float3 nrm, int* stk, TraceCount& tc) {
  int bits = 0;
  for (int l = 0; l < n_lights; l++) {
    const float4 Lp = lights[l];
    const float3 d = make_float3(Lp.x - o.x, Lp.y - o.y, Lp.z - o.z);
    if (skip >= 0 && !(dot3(nrm, d) > 0.f)) continue;  // light behind the lit side
    const WtRay wr = wt_ray(o, d);
    int h[4];
    const int nlev = lb_bins(lb_desc, l, wr, h);
    const float reach = __builtin_amdgcn_sqrtf(dot3(d, d)) * (1.0f + 0x1p-20f);
    int nl = 0;
    for (int q = 0; q < nlev; q++) {
      if (COUNT) tc.nodes++;
      const int* hd = lb_offs + h[q];
      if (__int_as_float(hd[1]) <= reach) {
        stk[(2 * nl) * kWave] = hd[0];
        stk[(2 * nl + 1) * kWave] = hd[2];
        nl++;
      }
    }
    bool blocked = false, live = nl > 0;
    int cur = live ? stk[0] : 0, end = live ? stk[kWave] : 0, nxt = 1;
    while (live) {
      if (COUNT) tc.tris++;
      const float4* en = lb_ent + 3 * cur;
      const float4 q0 = en[0], q1 = en[1], q2 = en[2];
      float t;
      bool fr;
      if (__float_as_int(q0.w) != skip && hit_triangle(wr, q0, q1, q2, 1e-4f, 1.0f, t, fr)) {
        blocked = true;
        live = false;
      } else if (++cur == end || q2.w > reach) {  // this list is done: the next one, if any
        if (nxt < nl) {
          cur = stk[(2 * nxt) * kWave];
          end = stk[(2 * nxt + 1) * kWave];
          nxt++;
        } else {
          live = false;
        }
      }
    }
    if (!blocked) bits |= 1 << l;
  }
  return bits;
}

// Shadow segment o -> o + d: blocked iff some triangle other than `skip` is
// hit with 1e-4 < t < 1.
template <bool COUNT>
RC_DEV bool occluded(const float4* __restrict__ nodes, const float4* __restrict__ tris, int tri_stride, float3 o,
                     float3 d, int skip, int* stk, TraceCount& cnt) {
  const WtRay wr = wt_ray(o, d);
  const float4* const tk = tris + wr.kz * tri_stride;
  float3 inv, oi;
  ray_inv(d, o, inv, oi);
  int sp = 0;
  int node = 0;
  while (true) {
    while (node >= 0) {
      const float4* nd = nodes + 4 * node;
      float4 w0 = nd[0], w1 = nd[1], w2 = nd[2], w3 = nd[3];
      if (COUNT) cnt.nodes++;
      float ta = slab(w0.x, w0.y, w0.z, w0.w, w2.x, w2.y, inv, oi, 0.0f, 1.0f);
      float tb = slab(w1.x, w1.y, w1.z, w1.w, w2.z, w2.w, inv, oi, 0.0f, 1.0f);
      int ca = __float_as_int(w3.x), cb = __float_as_int(w3.y);
      bool ha = ta < __builtin_huge_valf(), hb = tb < __builtin_huge_valf();
      if (ha && hb) {
        int nearc = ta <= tb ? ca : cb, farc = ta <= tb ? cb : ca;
        stk[sp * kWave] = farc;
        sp++;
        node = nearc;
      } else if (ha) {
        node = ca;
      } else if (hb) {
        node = cb;
      } else {
        if (sp == 0) return false;
        sp--;
        node = stk[sp * kWave];
      }
    }
    int first = leaf_first(node), n = leaf_count(node);
    for (int k = 0; k < n; k++) {
      const float4* tr = tk + 3 * (first + k);
      float4 A = tr[0], B = tr[1], C = tr[2];
      if (COUNT) cnt.tris++;
      float t;
      bool fr;
      if (__float_as_int(A.w) != skip && hit_triangle(wr, A, B, C, 1e-4f, 1.0f, t, fr)) return true;
    }
    if (sp == 0) return false;
    sp--;
    node = stk[sp * kWave];
  }
}

// ---------------------------------------------------------------------------
// One triangle's contribution to the gradient and Hessian
// (Eqs. SSSegALGradientSimp / SSSegALHessianSimp):
//   g = wL (T grad F + F grad T)
//   H = wL (T HF + grad T grad F^T + grad F grad T^T + F HT)
// with the triangle's solid angle Omega = 2 atan2(|A|, B), F = Omega/(4 pi)
// (App. C), its gradient (B grad|A| - |A| grad B) / (2 pi D), D = A^2 + B^2,
// and its Hessian written in symmetric form
//   HF = [ -|A| J(grad B) / D
//          + ((A^2 - B^2)(a b^T + b a^T) - 2 |A| B (a a^T - b b^T)) / D^2 ] / (2 pi)
// where a = grad|A| (J(grad A) = 0, App. C) and b = grad B.  Transmittance
// T = exp(-mu r) to the far vertex and its derivatives (App. A).
// Vertices are given relative to x (r_k = y_k - x); `far` indexes the far
// vertex.  Outputs g[3] and h[6] (xx, xy, xz, yy, yz, zz).
// ---------------------------------------------------------------------------
template <typename R>
struct V3 {
  R x, y, z;
};
template <typename R>
RC_DEV V3<R> mk(R x, R y, R z) { return V3<R>{x, y, z}; }
template <typename R>
RC_DEV V3<R> operator+(V3<R> a, V3<R> b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
template <typename R>
RC_DEV V3<R> operator-(V3<R> a, V3<R> b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
template <typename R>
RC_DEV V3<R> operator*(R s, V3<R> a) { return mk(s * a.x, s * a.y, s * a.z); }
template <typename R>
RC_DEV R dotv(V3<R> a, V3<R> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename R>
RC_DEV V3<R> crossv(V3<R> a, V3<R> b) { return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }

// symmetric outer-product helpers on 6-vectors (xx, xy, xz, yy, yz, zz)
template <typename R>
RC_DEV void sym_add_outer2(R* h, R s, V3<R> a, V3<R> b) {  // h += s (a b^T + b a^T)
  h[0] += s * (2 * a.x * b.x);
  h[1] += s * (a.x * b.y + a.y * b.x);
  h[2] += s * (a.x * b.z + a.z * b.x);
  h[3] += s * (2 * a.y * b.y);
  h[4] += s * (a.y * b.z + a.z * b.y);
  h[5] += s * (2 * a.z * b.z);
}
template <typename R>
RC_DEV void sym_add_outer(R* h, R s, V3<R> a) {  // h += s a a^T
  h[0] += s * a.x * a.x;
  h[1] += s * a.x * a.y;
  h[2] += s * a.x * a.z;
  h[3] += s * a.y * a.y;
  h[4] += s * a.y * a.z;
  h[5] += s * a.z * a.z;
}

template <typename R>
RC_DEV R r_atan2(R y, R x);
template <>
RC_DEV float r_atan2<float>(float y, float x) { return atan2f(y, x); }
template <>
RC_DEV double r_atan2<double>(double y, double x) { return atan2(y, x); }
template <typename R>
RC_DEV R r_sqrt(R v);
template <>
RC_DEV float r_sqrt<float>(float v) { return sqrtf(v); }
template <>
RC_DEV double r_sqrt<double>(double v) { return sqrt(v); }
template <typename R>
RC_DEV R r_exp(R v);
template <>
RC_DEV float r_exp<float>(float v) { return expf(v); }
template <>
RC_DEV double r_exp<double>(double v) { return exp(v); }

// Returns false (no term) for a degenerate triangle: A = 0 (the vertices
// coplanar with x: a term of zero measure) or all vertices at x.
// q_k = t_k w_k: vertex k at ray distance t_k along direction w_k.
// detw = w1 . (w2 x w3), supplied by the caller in FP64 precision: for thin
// (near-zero-area) triangles it is one of the two quantities FP32 cannot
// resolve (cs below is the other), and A = q1 . (q2 x q3) = t1 t2 t3 detw
// exactly.
//
// F is invariant under scaling of the vertices about x, grad F scales as 1/s
// and HF as 1/s^2: the form factor is evaluated on vertices divided by
// s = max_k |r_k| and rescaled, which keeps B ~ |r|^3 and 1/D^2 ~ |r|^-12 inside
// the FP32 range for vertices arbitrarily close to x.
//
// cs = (q2 - q1) x (q3 - q1) = q1 x q2 + q2 x q3 + q3 x q1 is supplied in
// FP64 as well: it is grad A up to sign, and for thin triangles (vertices
// nearly collinear as seen from x) its three cross products nearly cancel,
// which costs FP32 all its digits (per-term Hessian errors up to 5e-2 on
// 1M-triangle scenes; 2e-6 with cs in FP64).
template <typename R>
RC_DEV bool triangle_term(V3<R> q1, V3<R> q2, V3<R> q3, R t1, R t2, R t3, R detw, V3<double> cs, int far, R wL,
                          R mu, R* g, R* h) {
  const R inv2pi = (R)(1.0 / (2.0 * kPi));
  R m1 = r_sqrt(dotv(q1, q1)), m2 = r_sqrt(dotv(q2, q2)), m3 = r_sqrt(dotv(q3, q3));
  R sc = m1 > m2 ? (m1 > m3 ? m1 : m3) : (m2 > m3 ? m2 : m3);
  if (!(sc > (R)0)) return false;
  R isc = (R)1 / sc;
  V3<R> r1 = isc * q1, r2 = isc * q2, r3 = isc * q3;
  R l1 = m1 * isc, l2 = m2 * isc, l3 = m3 * isc;
  R A = ((t1 * isc) * (t2 * isc) * (t3 * isc)) * detw;
  R d12 = dotv(r1, r2), d23 = dotv(r2, r3), d13 = dotv(r1, r3);
  R B = l1 * l2 * l3 + d12 * l3 + d23 * l1 + d13 * l2;
  R absA = A < 0 ? -A : A;
  R sg = A < 0 ? (R)-1 : (R)1;
  if (A == (R)0) return false;
  V3<R> u1 = ((R)1 / l1) * r1, u2 = ((R)1 / l2) * r2, u3 = ((R)1 / l3) * r3;
  const double isc2 = (double)isc * (double)isc;
  V3<R> a = (-sg) * mk((R)(cs.x * isc2), (R)(cs.y * isc2), (R)(cs.z * isc2));
  // b = grad B, with grad l_k = -u_k
  V3<R> b = (-(l2 * l3 + d23)) * u1 + (-(l1 * l3 + d13)) * u2 + (-(l1 * l2 + d12)) * u3;
  b = b - l3 * (r1 + r2) - l1 * (r2 + r3) - l2 * (r1 + r3);
  // Work with a/sqrt(D) and b/sqrt(D), D = A^2 + B^2, so that every
  // coefficient below ((A^2 - B^2)/D, |A| B / D, |A|/sqrt(D), B/sqrt(D)) is
  // bounded by 1 and no intermediate overflows when two vertices are much
  // closer to x than the third (B ~ l1 l2 l3 tiny).
  R rho = absA > (B < 0 ? -B : B) ? absA : (B < 0 ? -B : B);
  R an = absA / rho, bn = B / rho;
  R sD = rho * r_sqrt(an * an + bn * bn);  // sqrt(D)
  R isD = (R)1 / sD;
  R cA = absA * isD, cB = B * isD;           // |A|/sqrt(D), B/sqrt(D)
  V3<R> al = isD * a, be = isD * b;          // a/sqrt(D), b/sqrt(D)
  R F = r_atan2(absA, B) * inv2pi;  // Omega / (4 pi) with Omega = 2 atan2(|A|, B)
  V3<R> gF = (inv2pi * isc) * (cB * al - cA * be);
  // J(grad B), symmetric
  R JB[6] = {0, 0, 0, 0, 0, 0};
  R k1 = (l2 * l3 + d23) / l1, k2 = (l1 * l3 + d13) / l2, k3 = (l1 * l2 + d12) / l3;
  R diag = k1 + k2 + k3 + (R)2 * (l1 + l2 + l3);
  JB[0] = diag;
  JB[3] = diag;
  JB[5] = diag;
  sym_add_outer(JB, -k1, u1);
  sym_add_outer(JB, -k2, u2);
  sym_add_outer(JB, -k3, u3);
  sym_add_outer2(JB, l1, u2, u3);
  sym_add_outer2(JB, l2, u1, u3);
  sym_add_outer2(JB, l3, u1, u2);
  sym_add_outer2(JB, (R)1, u3, r1 + r2);
  sym_add_outer2(JB, (R)1, u1, r2 + r3);
  sym_add_outer2(JB, (R)1, u2, r1 + r3);
  // HF = [ -|A| J(grad B)/D + ((A^2-B^2)/D)(al be^T + be al^T) - 2(|A| B/D)(al al^T - be be^T) ] / (2 pi)
  R HF[6];
  R c0 = -cA * isD;
  for (int k = 0; k < 6; k++) HF[k] = c0 * JB[k];
  sym_add_outer2(HF, (cA - cB) * (cA + cB), al, be);
  sym_add_outer(HF, (R)-2 * cA * cB, al);
  sym_add_outer(HF, (R)2 * cA * cB, be);
  const R hs = inv2pi * isc * isc;
  for (int k = 0; k < 6; k++) HF[k] *= hs;
  // transmittance to the far vertex (true distances), u = x - y_far = -r_far
  V3<R> rf = far == 0 ? r1 : (far == 1 ? r2 : r3);
  R lf = (far == 0 ? l1 : (far == 1 ? l2 : l3)) * sc;
  V3<R> uf = (sc / lf) * rf;
  R T = r_exp(-mu * lf);
  V3<R> gT = (mu * T) * uf;
  // HT = -(mu T / r)(I - (1 + mu r) uf uf^T)
  R cH = -mu * T / lf;
  R HT[6] = {cH, 0, 0, cH, 0, cH};
  sym_add_outer(HT, -cH * ((R)1 + mu * lf), uf);
  g[0] = wL * (T * gF.x + F * gT.x);
  g[1] = wL * (T * gF.y + F * gT.y);
  g[2] = wL * (T * gF.z + F * gT.z);
  R hh[6];
  for (int k = 0; k < 6; k++) hh[k] = T * HF[k] + F * HT[k];
  sym_add_outer2(hh, (R)1, gT, gF);
  for (int k = 0; k < 6; k++) h[k] = wL * hh[k];
  return true;
}

// Neumaier compensated accumulation in FP32
RC_DEV void kadd(float& s, float& c, float x) {
  float t = s + x;
  if (fabsf(s) >= fabsf(x)) c += (s - t) + x;
  else c += (x - t) + s;
  s = t;
}

}  // namespace rc
