// kernels.hip -- HIP kernels of librc for gfx950 (AMD Instinct MI355X).
//
// record_kernel: one wavefront computes one whole radiance-cache record
// (Sec. 4 and Sec. 6 of Marco et al. 2018).  The grid is persistent: each
// wavefront pops record indices from a queue counter until the queue is
// empty.  Per record the wave walks the strata rows from the north pole to
// the south pole, keeping two rows on chip (LDS):
//   1. trace the row's directions (closest hit over the BVH) and count the
//      medium rings in front of each hit;
//   2. shade every surface vertex and ring vertex of the row with one shadow
//      ray per point light; the (vertex, light) tasks of the row are
//      compacted across the 64 lanes;
//   3. accumulate the Monte Carlo value of the row's strata;
//   4. form the triangles between the previous row and this one (polar fans
//      at the ends, two triangles per quad elsewhere) and evaluate every
//      (triangle, ring) term, again compacted across lanes, into per-lane
//      compensated FP32 sums (FP32 terms whose two thin-triangle
//      quantities, the direction determinant and grad A, are FP64);
// and finally reduces the 64 lanes in FP64 with cross-lane shuffles.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"

namespace rc {

namespace {

// One strata row in LDS, structure of arrays over the row's columns:
// direction, hit distance (the FP32 decision value), hit code
// ((triangle << 1) | front, or -1), rings in front of the hit, surface
// radiance, surface light-visibility bits, the continuous hit distance as a
// correction to the decision value (FP64 exact ray-plane distance of the
// decided triangle, or FP64 box exit, minus t; rounded to FP32), and ring
// radiance [ring][column] (holding light-visibility bits until shaded).
constexpr int kRowFields = 9;
struct Row {
  float *wx, *wy, *wz, *t, *Ls, *tlo, *Lm;
  int *code, *M, *visS;
};

RC_DEV Row row_view(float* base, int cap) {
  Row r;
  r.wx = base;
  r.wy = base + cap;
  r.wz = base + 2 * cap;
  r.t = base + 3 * cap;
  r.code = (int*)(base + 4 * cap);
  r.M = (int*)(base + 5 * cap);
  r.Ls = base + 6 * cap;
  r.visS = (int*)(base + 7 * cap);
  r.tlo = base + 8 * cap;
  r.Lm = base + kRowFields * cap;  // [max_rings][cap]
  return r;
}

RC_DEV int wave_inclusive_scan(int v, int lane) {
#pragma unroll
  for (int s = 1; s < kWave; s <<= 1) {
    int o = __shfl_up(v, s, kWave);
    if (lane >= s) v += o;
  }
  return v;
}

// largest j in [0, n) with off[j] <= x (off non-decreasing, off[0] = 0)
RC_DEV int find_slot(const int* off, int n, int x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// largest j in [0, n) with off[j] - j <= x (off[j] - j non-decreasing)
RC_DEV int find_slot_minus(const int* off, int n, int x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] - mid <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Direction of column `col` of row a: row -1 is the north pole, row nth the
// south pole, rows 0..nth-1 the strata rows.
RC_DEV float3 row_direction(uint64_t key, int a, int col, int nth, int nph) {
  if (a < 0) return make_float3(0.f, 0.f, 1.f);
  if (a == nth) return make_float3(0.f, 0.f, -1.f);
  return stratum_direction(key, a, col, nth, nph);
}

// Position of direction (row a, column col) in a record's list of primary
// rays: north pole 0, stratum (a, col) 1 + a * nph + col, south pole N + 1.
RC_DEV int dir_index(int a, int col, int nth, int nph) {
  return a < 0 ? 0 : (a == nth ? nth * nph + 1 : 1 + a * nph + col);
}
RC_DEV size_t hit_slot(int qr, int d, int stride) {
  return ((size_t)(qr >> 6) * (size_t)stride + (size_t)d) * kWave + (size_t)(qr & (kWave - 1));
}

RC_DEV double wave_sum(double v) {
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) v += __shfl_xor(v, s, kWave);
  return v;
}

// Add one term's 9 outputs (gradient 3, Hessian 6) to a channel's
// compensated pairs.
RC_DEV void add_term(float* acc, float* accc, const float* t) {
#pragma unroll
  for (int k = 0; k < 9; k++) kadd(acc[k], accc[k], t[k]);
}

// The same with each output given as an FP32 (hi, lo) split of an FP64 value:
// hi then lo, per output.
RC_DEV void add_term2(float* acc, float* accc, const float* hi, const float* lo) {
#pragma unroll
  for (int k = 0; k < 9; k++) {
    kadd(acc[k], accc[k], hi[k]);
    kadd(acc[k], accc[k], lo[k]);
  }
}

}  // namespace

template <int STACK, bool COUNT, bool F64>
// Register budget for record_waves_per_simd(STACK) wavefronts per SIMD (the
// compiler spills values of the cooler phases, none inside the traversal
// loops): traversal is latency-bound, so more resident wavefronts beat the
// spills.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(record_waves_per_simd(STACK),
                                                                     record_waves_per_simd(STACK)))) void
record_kernel(RecordArgs g) {
  extern __shared__ float lds[];
  // the smallest stack variant holds no traversal: its primary hits come
  // from the hits pass and its shadow segments from the light bins
  constexpr bool kOwnRays = STACK > kHitsStack;
  const int lane = threadIdx.x;
  const int cap = g.lds_cols;  // columns of an LDS row
  const int MR = g.max_rings;
  int* stk = reinterpret_cast<int*>(lds) + lane;
  float* rows = lds + STACK * kWave;
  const int row_words = cap * (kRowFields + MR);
  int* off = reinterpret_cast<int*>(rows + 2 * row_words);  // [2 * cap + 1]
  // per-record FP64 accumulators (lane 0 writes): 2 values + 2 x 9 derivatives
  double* racc = reinterpret_cast<double*>(off + ((2 * cap + 2) & ~1));

  const float mu = g.sigma_s + g.sigma_a;
  const float ms_scale = g.sigma_s * (float)(1.0 / (4.0 * kPi));
  TraceCount tc;
  uint32_t n_rays = 0, n_terms = 0;
  uint64_t cyc[4] = {0, 0, 0, 0};  // counting variant: shader clocks per phase
  uint64_t sh_iter = 0, sh_busy = 0, sh_refill = 0, sh_lanes = 0;  // counting variant: shadow loop
  uint64_t t_mark = 0;

  const int S = g.splits;  // wavefronts per record (row ranges); 1 for large batches
  // queue slots [lo, hi) of this launch: all of them, or one class of records
  const int q_lo = g.range ? (int)g.range[0] : 0;
  const int q_n = g.range ? (int)g.range[1] - q_lo : g.P;
  while (true) {
    int q = 0;  // item = queue slot * S + part
    if (lane == 0) q = (int)atomicAdd(g.next, 1u);
    q = __shfl(q, 0, kWave);
    if ((long long)q >= (long long)q_n * S) break;
    const int qr = q_lo + q / S, part = q - (q / S) * S;
    const int rec = g.order ? g.order[qr] : qr;
    if (rec < 0 || rec >= g.P) {  // corrupt queue entry: count it, touch nothing
      if (lane == 0 && part == 0) atomicAdd(&g.queue[1], 1u);
      continue;
    }
    const float3 x = make_float3(g.pos[3 * rec], g.pos[3 * rec + 1], g.pos[3 * rec + 2]);
    const int nth = g.n_theta[rec], nph = g.n_phi[rec];
    const bool bad = !(nth >= 2 && nph >= 5 && nph <= g.max_n_phi) || (g.hits && nth > g.max_n_theta) ||
                     !(x.x >= g.box_lo.x && x.x <= g.box_hi.x) ||
                     !(x.y >= g.box_lo.y && x.y <= g.box_hi.y) || !(x.z >= g.box_lo.z && x.z <= g.box_hi.z);
    if (bad) {
      if (part != 0) continue;  // the first part reports it
      if (lane < 2) {
        g.value[2 * rec + lane] = __builtin_nan("");
        for (int k = 0; k < 3; k++) g.grad[6 * rec + 3 * lane + k] = __builtin_nan("");
        for (int k = 0; k < 6; k++) g.hess[12 * rec + 6 * lane + k] = __builtin_nan("");
      }
      if (lane == 0) atomicAdd(&g.queue[1], 1u);
      continue;
    }
    const int N = nth * nph;
    const uint64_t key = record_key(g.seed, (uint64_t)(g.rec_base + (g.common_random ? 0 : rec)));
    const float xr = uniform24(key, kRingIdx, 0);

    if (lane < 20) racc[lane] = 0.0;

    // rows: -1 north pole, 0..nth-1 strata rows, nth south pole.  Part k of S
    // owns rows a_own..a_hi (values and the bands ending at them); a later
    // part also recomputes the row before a_own, which its first band needs.
    const int nr = nth + 2;
    const int r0 = (int)(((long long)part * nr) / S), r1 = (int)(((long long)(part + 1) * nr) / S);
    const int a_own = r0 - 1, a_hi = r1 - 2;
    const int a_lo = (part > 0 && r1 > r0) ? a_own - 1 : a_own;
    // Columns: a row wider than the LDS rows is done in sectors of at most
    // cap - 1 owned columns plus the next sector's first column (the quads
    // between them need it); each sector walks the rows again (poles included).
    // Local column j of sector s is global column (b0 + j) mod n_phi.
    const bool sectored = nph > cap;
    const int nsec = sectored ? (nph + cap - 2) / (cap - 1) : 1;  // sectors of at most cap - 1 columns,
    const int wsec = (nph + nsec - 1) / nsec;                     // balanced
    for (int sec = 0; sec < nsec; sec++) {
    const int b0 = sec * wsec;
    const int nown = min(wsec, nph - b0);           // owned columns (strata, quads)
    const int ncol = sectored ? nown + 1 : nph;      // columns held
    // rows g_lo..g_hi had their primary rays traced in one pass; with more
    // than one row, lane k holds the closest hit of ray k of the pass
    int g_lo = a_lo, g_hi = a_lo - 1;
    float held_t = 0.f;
    int held_code = -1;
    for (int a = a_lo; a <= a_hi; a++) {
      const bool own = a >= a_own;
      float* const baseR = rows + ((a + 1) & 1) * row_words;
      float* const baseP = rows + (a & 1) * row_words;
      const Row R = row_view(baseR, cap);
      const Row P = row_view(baseP, cap);
      const bool pole = (a < 0 || a == nth);
      const int n = pole ? 1 : ncol;
      // counted once per record: owned columns, and the poles in the first sector
      const int n_cnt = pole ? (sec == 0 ? 1 : 0) : nown;
      // ---- 1. primary rays ------------------------------------------------
      // Narrow rows leave lanes idle, so the closest hits of this row and of
      // as many following rows as fit in the wavefront are traced in one pass
      // (a pole row has one column).  A row traced alone keeps its hits in
      // its LDS row; a pass over several rows keeps them in registers.
      if (COUNT) t_mark = clock64();
      if (kOwnRays && !g.hits && a > g_hi) {
        g_lo = a;
        g_hi = a;
        int tot = n;
        while (g_hi < a_hi) {
          const int nn = (g_hi + 1 == nth) ? 1 : ncol;
          if (tot + nn > kWave) break;
          g_hi++;
          tot += nn;
        }
        for (int base = 0; base < tot; base += kWave) {
          int c = base + lane;
          if (c < tot) {
            int r = a;
            for (int m = (r < 0 || r == nth) ? 1 : ncol; c >= m; m = (r < 0 || r == nth) ? 1 : ncol) {
              c -= m;
              r++;
            }
            const float3 w = row_direction(key, r, sectored ? (b0 + c) % nph : c, nth, nph);
            int id;
            float t;
            bool fr;
            trace_closest<COUNT>(g.nodes, g.tris, g.tri_stride, x, w, stk, g.leaf_batch, id, t, fr, tc);
            const int code = id >= 0 ? ((id << 1) | (fr ? 1 : 0)) : -1;
            if (g_hi == a) {
              R.t[c] = t;
              R.code[c] = code;
            } else {
              held_t = t;
              held_code = code;
            }
          }
        }
      }
      // this row's hits: from the LDS row, or from the lanes of the pass
      const bool grouped = g_hi > g_lo;
      float gt = 0.f;
      int gcode = -1;
      if (grouped) {
        int o = 0;  // first ray of row a in the pass
        for (int r = g_lo; r < a; r++) o += (r < 0 || r == nth) ? 1 : ncol;
        const int src = min(o + lane, kWave - 1);
        gt = __shfl(held_t, src, kWave);
        gcode = __shfl(held_code, src, kWave);
      }
      for (int base = 0; base < n; base += kWave) {
        int j = base + lane;
        if (j < n) {
          const int col = sectored ? (b0 + j) % nph : j;
          const float3 w = row_direction(key, a, col, nth, nph);
          float t;
          int code;
          if (!kOwnRays || g.hits) {  // traced by primary_kernel
            const float2 h = g.hits[hit_slot(qr, dir_index(a, col, nth, nph), g.hit_stride)];
            t = h.x;
            code = __float_as_int(h.y);
          } else {
            t = grouped ? gt : R.t[j];
            code = grouped ? gcode : R.code[j];
          }
          double t64;
          if (code < 0) {
            t = box_exit(x, w, g.box_lo, g.box_hi);
            t64 = box_exit64(x, w, g.box_lo, g.box_hi);
          } else {
            const double4 pl = g.plane[code >> 1];
            t64 = (pl.w - ((pl.x * x.x + pl.y * x.y) + pl.z * x.z)) / ((pl.x * w.x + pl.y * w.y) + pl.z * w.z);
          }
          R.tlo[j] = (float)(t64 - (double)t);
          int M = 0;
          while (M < MR && ring_distance(M, xr, g.ring_step) < t) M++;
          R.wx[j] = w.x;
          R.wy[j] = w.y;
          R.wz[j] = w.z;
          R.t[j] = t;
          R.code[j] = code;
          R.M[j] = M;
          R.Ls[j] = code >= 0 ? g.emission[code >> 1] : 0.f;
          R.visS[j] = 0;
          for (int i = 0; i < M; i++) reinterpret_cast<int*>(R.Lm)[i * cap + j] = 0;
          if (COUNT && own && j < n_cnt) n_rays++;
        }
      }
      __syncthreads();
      if (COUNT) { uint64_t t = clock64(); cyc[0] += t - t_mark; t_mark = t; }
      // ---- 2. shadow rays ---------------------------------------------------
      // Every surface vertex and ring vertex of the row needs one shadow
      // segment per point light; unblocked segments set the light's bit on the
      // vertex.  Lanes take vertices in column order, so neighbouring lanes
      // trace coherent segments, and decode each vertex once.
      if (g.n_lights > 0) {
        int carry = 0;
        for (int base = 0; base < n; base += kWave) {
          int j = base + lane;
          int c = (j < n) ? ((R.code[j] >= 0 ? 1 : 0) + R.M[j]) : 0;
          int inc = wave_inclusive_scan(c, lane);
          if (j < n) off[j] = carry + inc - c;
          carry += __shfl(inc, kWave - 1, kWave);
        }
        // wave-uniform counts, kept in scalar registers
        const int nvert = __builtin_amdgcn_readfirstlane(carry);
        const int NL = g.n_lights;
        __syncthreads();
        if (g.vis) {
          // walked by the hits pass: the vertices' bits of each column's ray
          for (int base = 0; base < n; base += kWave) {
            const int j = base + lane;
            if (j >= n) continue;
            const int col = sectored ? (b0 + j) % nph : j;
            const size_t w0 =
                ((size_t)(qr >> 6) * (size_t)g.hit_stride + (size_t)dir_index(a, col, nth, nph)) * (size_t)g.vis_words;
            unsigned int words[kVisMaxWords];
#pragma unroll
            for (int q = 0; q < kVisMaxWords; q++)
              words[q] = q < g.vis_words ? g.vis[(w0 + q) * kWave + (size_t)(qr & (kWave - 1))] : 0u;
            const unsigned int mask = (1u << NL) - 1u;
            auto vbits = [&](int kk) {
              const int pos = kk << g.vis_shift;
              unsigned int wd = 0u;
#pragma unroll
              for (int q = 0; q < kVisMaxWords; q++)
                if (q == (pos >> 5)) wd = words[q];
              return (int)((wd >> (pos & 31)) & mask);
            };
            const int code = R.code[j], M = R.M[j];
            if (code >= 0) R.visS[j] = vbits(0);
            for (int i = 0; i < M; i++) reinterpret_cast<int*>(R.Lm)[i * cap + j] = vbits(1 + i);
            if (COUNT && own && j < n_cnt) n_rays += NL * ((code >= 0 ? 1 : 0) + M);
          }
        } else if (!kOwnRays || g.lb_desc) {
          // Light bins: a segment reads one header per level and then only
          // the few entries within its reach (one to three on average), so a
          // lane walks all lights of its vertex in turn: decode once, per
          // light the bin headers and the entry list, and one store of the
          // vertex's visibility bits.
          for (int base = 0; base < nvert; base += kWave) {
            const int v = base + lane;
            if (v >= nvert) continue;
            const int j = find_slot(off, n, v);
            const int k = v - off[j];
            const int code = R.code[j];
            const float3 w = make_float3(R.wx[j], R.wy[j], R.wz[j]);
            int skip = -1, slot;
            float3 o, nrm = make_float3(0.f, 0.f, 0.f);
            if (code >= 0 && k == 0) {
              skip = code >> 1;
              o = axpy3(R.t[j], w, x);
              slot = -1 - j;  // surface vertex of column j
              const float4 sh = g.shade[skip];
              const float nsign = (code & 1) ? 1.f : -1.f;
              nrm = make_float3(nsign * sh.x, nsign * sh.y, nsign * sh.z);
            } else {
              const int i = k - (code >= 0 ? 1 : 0);
              o = axpy3(ring_distance(i, xr, g.ring_step), w, x);
              slot = i * cap + j;
            }
            if (COUNT && own && j < n_cnt) n_rays += NL;
            const int bits = light_bits<COUNT>(g.lights, g.n_lights, g.lb_desc, g.lb_offs, g.lb_ent, o, skip, nrm, stk, tc);
            if (slot < 0) R.visS[-1 - slot] = bits;
            else reinterpret_cast<int*>(R.Lm)[slot] = bits;
          }
        } else {
        int next = 0;          // next vertex to hand out (wave-uniform)
        bool active = false;   // a segment in progress
        // the lane's vertex: origin, oriented surface normal (surface
        // vertices), own triangle (skip >= 0: a surface vertex), visibility
        // slot, and the light of its current or next segment (NL: no vertex)
        int lcur = NL, skip = -1, slot = 0;
        float3 o = make_float3(0.f, 0.f, 0.f), nrm = o;
        // the current segment: BVH traversal state, or light-bin lists
        int node = 0, sp = 0, lf = 0, ln = 0;
        float3 d = o, inv = o, oi = o;
        WtRay wr = wt_ray(o, d);
        while (true) {
          const uint64_t idle = __ballot(!active);
          const uint64_t fresh = __ballot(!active && lcur >= NL);  // idle lanes without a vertex
          const bool more = next < nvert || (idle & ~fresh) != 0ull;
          const bool refill = more && (__popcll(idle) >= g.refill_min || idle == ~0ull);
          if (refill && !active) {
            if (lcur >= NL) {
              const int v = next + mask_rank(fresh);
              if (v < nvert) {
                const int j = find_slot(off, n, v);
                const int k = v - off[j];
                const int code = R.code[j];
                const float3 w = make_float3(R.wx[j], R.wy[j], R.wz[j]);
                if (code >= 0 && k == 0) {
                  skip = code >> 1;
                  o = axpy3(R.t[j], w, x);
                  slot = -1 - j;  // surface vertex of column j
                  const float4 sh = g.shade[skip];
                  const float nsign = (code & 1) ? 1.f : -1.f;
                  nrm = make_float3(nsign * sh.x, nsign * sh.y, nsign * sh.z);
                } else {
                  const int i = k - (code >= 0 ? 1 : 0);
                  skip = -1;
                  o = axpy3(ring_distance(i, xr, g.ring_step), w, x);
                  slot = i * cap + j;
                }
                lcur = 0;
                if (COUNT && own && j < n_cnt) n_rays += NL;
              }
            }
            // set up the segment to the next light that needs one: lights
            // behind a surface's lit side need none, and a segment whose
            // light bins hold nothing within reach is clear at once
            while (lcur < NL && !active) {
              const float4 Lp = g.lights[lcur];
              d = make_float3(Lp.x - o.x, Lp.y - o.y, Lp.z - o.z);
              if (skip >= 0 && !(dot3(nrm, d) > 0.f)) {
                lcur++;
                continue;
              }
              wr = wt_ray(o, d);
              {
                ray_inv(d, o, inv, oi);
                node = 0;
                sp = 0;
                ln = 0;
              }
              active = true;
            }
          }
          if (refill) next = __builtin_amdgcn_readfirstlane(next + __popcll(fresh));
          const uint64_t busy = __ballot(active);
          if (COUNT) {
            sh_iter++;
            sh_busy += __popcll(busy);
            if (refill) {
              sh_refill++;
              sh_lanes += __popcll(busy & idle);
            }
          }
          if (busy == 0ull) {
            if (next >= nvert && __ballot(lcur < NL) == 0ull) break;
            continue;
          }
          // leaf_batch 0: every busy lane takes its next step (node or
          // triangle) in every iteration.  leaf_batch k > 0: one kind of step
          // per iteration for the whole wavefront, triangle tests once at
          // least k lanes wait at a leaf (or no lane has a node step left),
          // node steps otherwise; lanes of the other kind wait.
          const uint64_t at_leaf = __ballot(active && ln > 0);
          const bool tri_step = at_leaf != 0ull && (__popcll(at_leaf) >= g.leaf_batch || at_leaf == busy);
          if (active && (g.leaf_batch == 0 || (ln > 0) == tri_step)) {
            bool done = false, blocked = false;
            // one fetch per lane per iteration: the next triangle of the current
            // leaf, or the current node (the triangle array carries one word of
            // padding so the fourth load of the last triangle stays in bounds)
            const float4* src = (ln > 0) ? (g.tris + wr.kz * g.tri_stride + 3 * lf) : (g.nodes + 4 * node);
            const float4 q0 = src[0], q1 = src[1], q2 = src[2], q3 = src[3];
            // next: the code to visit next (a node >= 0, a leaf < 0, kEnd when
            // the stack is exhausted) or kStay to go on in the current leaf
            constexpr int kEnd = 0x7fffffff, kStay = 0x7ffffffe;
            int nx = kStay;
            bool pop = false;
            if (ln > 0) {
              if (COUNT) tc.tris++;
              float t;
              bool fr;
              if (__float_as_int(q0.w) != skip && hit_triangle(wr, q0, q1, q2, 1e-4f, 1.0f, t, fr)) {
                done = true;
                blocked = true;
              } else {
                lf++;
                ln--;
                pop = ln == 0;
              }
            } else {
              if (COUNT) tc.nodes++;
              const float ta = slab(q0.x, q0.y, q0.z, q0.w, q2.x, q2.y, inv, oi, 0.0f, 1.0f);
              const float tb = slab(q1.x, q1.y, q1.z, q1.w, q2.z, q2.w, inv, oi, 0.0f, 1.0f);
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
            if (nx == kEnd) {
              done = true;
            } else if (nx != kStay) {
              if (nx < 0) {  // a leaf
                lf = leaf_first(nx);
                ln = leaf_count(nx);
              } else {
                node = nx;
              }
            }
            if (done) {
              active = false;
              if (!blocked) {
                if (slot < 0) atomicOr(&R.visS[-1 - slot], 1 << lcur);
                else atomicOr(reinterpret_cast<int*>(R.Lm) + slot, 1 << lcur);
              }
              lcur++;
            }
          }
        }
        }  // BVH shadow segments
        __syncthreads();
        // radiance from the visibility bits, lights summed in order
        for (int v = lane; v < nvert; v += kWave) {
          const int j = find_slot(off, n, v);
          const int k = v - off[j];
          const int code = R.code[j];
          const float3 w = make_float3(R.wx[j], R.wy[j], R.wz[j]);
          if (code >= 0 && k == 0) {
            const int bits = R.visS[j];
            const int id = code >> 1;
            const float3 y = axpy3(R.t[j], w, x);
            const float4 sh = g.shade[id];
            const float nsign = (code & 1) ? 1.f : -1.f;
            float Lsum = R.Ls[j];
            for (int l = 0; l < g.n_lights; l++) {
              if (!((bits >> l) & 1)) continue;
              const float4 L = g.lights[l];
              const float3 seg = make_float3(L.x - y.x, L.y - y.y, L.z - y.z);
              const float dist = sqrtf(dot3(seg, seg));
              const float c = nsign * dot3(make_float3(sh.x, sh.y, sh.z), seg) / dist;
              Lsum += sh.w * (float)(1.0 / kPi) * L.w * c * expf(-mu * dist) / (dist * dist);
            }
            R.Ls[j] = Lsum;
          } else {
            const int i = k - (code >= 0 ? 1 : 0);
            const int bits = reinterpret_cast<int*>(R.Lm)[i * cap + j];
            const float3 y = axpy3(ring_distance(i, xr, g.ring_step), w, x);
            float Lsum = 0.f;
            for (int l = 0; l < g.n_lights; l++) {
              if (!((bits >> l) & 1)) continue;
              const float4 L = g.lights[l];
              const float3 seg = make_float3(L.x - y.x, L.y - y.y, L.z - y.z);
              const float dist2 = dot3(seg, seg);
              Lsum += ms_scale * L.w * expf(-mu * sqrtf(dist2)) / dist2;
            }
            R.Lm[i * cap + j] = Lsum;
          }
        }
        __syncthreads();
      } else {
        // no lights: ring radiance is zero (slots were cleared as ints)
      }
      if (COUNT) { uint64_t t = clock64(); cyc[1] += t - t_mark; t_mark = t; }
      // ---- 3. Monte Carlo value of the strata in this row -----------------
      if (!pole && own) {
        float vs = 0.f, vsc = 0.f, vm = 0.f, vmc = 0.f;
        for (int base = 0; base < nown; base += kWave) {
          int j = base + lane;
          if (j < nown) {
            float3 w = make_float3(R.wx[j], R.wy[j], R.wz[j]);
            float wn = sqrtf(dot3(w, w));
            kadd(vs, vsc, expf(-mu * (R.t[j] + R.tlo[j]) * wn) * R.Ls[j]);
            for (int i = 0; i < R.M[j]; i++)
              kadd(vm, vmc, g.ring_step * expf(-mu * ring_distance(i, xr, g.ring_step) * wn) * R.Lm[i * cap + j]);
          }
        }
        double s0 = wave_sum((double)vs + (double)vsc);
        double s1 = wave_sum((double)vm + (double)vmc);
        if (lane == 0) {
          racc[0] += s0;
          racc[1] += s1;
        }
      }
      if (COUNT) { uint64_t t = clock64(); cyc[2] += t - t_mark; t_mark = t; }
      // ---- 4. triangles between the previous row and this one -------------
      if (a >= 0 && own) {
        // kind 0: north fan (P = pole, R = row 0); 1: band; 2: south fan
        const int kind = (a == 0) ? 0 : (a == nth ? 2 : 1);
        const int ntri = (kind == 1) ? 2 * nown : nown;
        const int prow = a - 1;  // strata row index of P (for vertex ids)
        int carry = 0;
        for (int base = 0; base < ntri; base += kWave) {
          int tI = base + lane;
          int c = 0;
          if (tI < ntri) {
            int m0, m1, m2;
            int b = (kind == 1) ? (tI >> 1) : tI;
            int b1 = (b + 1 == ncol) ? 0 : b + 1;
            if (kind == 0) { m0 = P.M[0]; m1 = R.M[b]; m2 = R.M[b1]; }
            else if (kind == 2) { m0 = R.M[0]; m1 = P.M[b1]; m2 = P.M[b]; }
            else { m0 = max(P.M[b], P.M[b1]); m1 = R.M[b]; m2 = R.M[b1]; }
            c = 1 + max(m0, max(m1, m2));
          }
          int inc = wave_inclusive_scan(c, lane);
          if (tI < ntri) off[tI] = carry + inc - c;
          carry += __shfl(inc, kWave - 1, kWave);
        }
        const int total = carry;
        __syncthreads();
        // Two passes, the surface terms (one per triangle) and then the medium
        // terms, so each pass keeps only its channel's 9 compensated sums live.
        // Triangle tI holds items off[tI] .. off[tI+1]-1: its surface term and
        // then its medium rings, so its rings start at off[tI] - tI among the
        // medium items.
        for (int chn = 0; chn < 2; chn++) {
        float acc[9], accc[9];
#pragma unroll
        for (int k = 0; k < 9; k++) { acc[k] = 0.f; accc[k] = 0.f; }
        const int n_items = chn == 0 ? ntri : total - ntri;
        for (int base = 0; base < n_items; base += kWave) {
          int item = base + lane;
          if (item >= n_items) continue;
          int tI, ring;  // ring -1: surface ring
          if (chn == 0) {
            tI = item;
            ring = -1;
          } else {
            tI = find_slot_minus(off, ntri, item);
            ring = item - (off[tI] - tI);
          }
          // the triangle's three vertices: (row pointer, column, global id)
          const float* vb[3];  // row base of each vertex
          int col[3], gid[3];
          // local columns b, b1 of the quad; global columns gb, gb1 (vertex ids)
          if (kind == 0) {
            int b = tI, b1 = (b + 1 == ncol) ? 0 : b + 1;
            const int gb = (b0 + b) % nph, gb1 = (b0 + b1) % nph;
            vb[0] = baseP; col[0] = 0; gid[0] = 0;
            vb[1] = baseR; col[1] = b; gid[1] = 1 + gb;
            vb[2] = baseR; col[2] = b1; gid[2] = 1 + gb1;
          } else if (kind == 2) {
            int b = tI, b1 = (b + 1 == ncol) ? 0 : b + 1;
            const int gb = (b0 + b) % nph, gb1 = (b0 + b1) % nph;
            vb[0] = baseR; col[0] = 0; gid[0] = N + 1;
            vb[1] = baseP; col[1] = b1; gid[1] = 1 + prow * nph + gb1;
            vb[2] = baseP; col[2] = b; gid[2] = 1 + prow * nph + gb;
          } else {
            int b = tI >> 1, b1 = (b + 1 == ncol) ? 0 : b + 1;
            const int gb = (b0 + b) % nph, gb1 = (b0 + b1) % nph;
            float3 wP = make_float3(P.wx[b], P.wy[b], P.wz[b]);
            float3 wQ = make_float3(P.wx[b1], P.wy[b1], P.wz[b1]);
            float3 wR = make_float3(R.wx[b], R.wy[b], R.wz[b]);
            float3 wS = make_float3(R.wx[b1], R.wy[b1], R.wz[b1]);
            bool d1 = det3(wP, wR, wS) > 0.f && det3(wP, wS, wQ) > 0.f;
            int gP = 1 + prow * nph + gb, gQ = 1 + prow * nph + gb1, gR = 1 + a * nph + gb, gS = 1 + a * nph + gb1;
            bool second = tI & 1;
            if (d1) {
              if (!second) { vb[0] = baseP; col[0] = b; gid[0] = gP; vb[1] = baseR; col[1] = b; gid[1] = gR; vb[2] = baseR; col[2] = b1; gid[2] = gS; }
              else { vb[0] = baseP; col[0] = b; gid[0] = gP; vb[1] = baseR; col[1] = b1; gid[1] = gS; vb[2] = baseP; col[2] = b1; gid[2] = gQ; }
            } else {
              if (!second) { vb[0] = baseP; col[0] = b; gid[0] = gP; vb[1] = baseR; col[1] = b; gid[1] = gR; vb[2] = baseP; col[2] = b1; gid[2] = gQ; }
              else { vb[0] = baseP; col[0] = b1; gid[0] = gQ; vb[1] = baseR; col[1] = b; gid[1] = gR; vb[2] = baseR; col[2] = b1; gid[2] = gS; }
            }
          }
          // per vertex: the decision distance (FP32: ring distance or hit
          // distance, picks the far vertex), the continuous distance (the
          // geometry of the term) and its low part (FP64 terms)
          float dec[3], tau[3], tlo[3], Lv[3];
          bool on_ring[3];
          float3 wv[3];
          const float rr = ring >= 0 ? ring_distance(ring, xr, g.ring_step) : 0.f;
#pragma unroll
          for (int k = 0; k < 3; k++) {
            const float* b = vb[k];
            int c = col[k];
            // field offsets as laid out by row_view
            wv[k] = make_float3(b[c], b[cap + c], b[2 * cap + c]);
            const float tk = b[3 * cap + c], lk = b[8 * cap + c];
            bool front = false;
            if (ring < 0) {
              Lv[k] = b[6 * cap + c];
            } else {
              front = ring < reinterpret_cast<const int*>(b)[5 * cap + c];
              Lv[k] = front ? b[(kRowFields + ring) * cap + c] : 0.f;
            }
            on_ring[k] = front;
            dec[k] = front ? rr : tk;
            tau[k] = front ? rr : tk + lk;
            tlo[k] = front ? 0.f : lk;
          }
          // far vertex: largest decision distance, ties to the smaller vertex
          // id (the running maximum is kept in plain variables, so no array is
          // indexed at run time)
          int far = 0;
          float tf = dec[0];
          int gf = gid[0];
#pragma unroll
          for (int k = 1; k < 3; k++)
            if (dec[k] > tf || (dec[k] == tf && gid[k] < gf)) { far = k; tf = dec[k]; gf = gid[k]; }
          float Lf = far == 0 ? Lv[0] : (far == 1 ? Lv[1] : Lv[2]);
          if (Lf == 0.f) continue;
          // direction determinant in FP64 (thin triangles); A = tau1 tau2 tau3 detw
          double dw = (double)wv[0].x * ((double)wv[1].y * wv[2].z - (double)wv[1].z * wv[2].y) +
                      (double)wv[0].y * ((double)wv[1].z * wv[2].x - (double)wv[1].x * wv[2].z) +
                      (double)wv[0].z * ((double)wv[1].x * wv[2].y - (double)wv[1].y * wv[2].x);
          if (!F64) {
            float wL = ring < 0 ? Lf : g.ring_step * Lf;
            float gg[3], hh[6];
            V3<float> r1 = mk(tau[0] * wv[0].x, tau[0] * wv[0].y, tau[0] * wv[0].z);
            V3<float> r2 = mk(tau[1] * wv[1].x, tau[1] * wv[1].y, tau[1] * wv[1].z);
            V3<float> r3 = mk(tau[2] * wv[2].x, tau[2] * wv[2].y, tau[2] * wv[2].z);
            // grad A up to sign, in FP64 from the same vertices (thin triangles)
            const V3<double> p1 = mk((double)tau[0] * wv[0].x, (double)tau[0] * wv[0].y, (double)tau[0] * wv[0].z);
            const V3<double> p2 = mk((double)tau[1] * wv[1].x, (double)tau[1] * wv[1].y, (double)tau[1] * wv[1].z);
            const V3<double> p3 = mk((double)tau[2] * wv[2].x, (double)tau[2] * wv[2].y, (double)tau[2] * wv[2].z);
            const V3<double> cs = crossv(p2 - p1, p3 - p1);
            if (triangle_term<float>(r1, r2, r3, tau[0], tau[1], tau[2], (float)dw, cs, far, wL, mu, gg, hh)) {
              const float t9[9] = {gg[0], gg[1], gg[2], hh[0], hh[1], hh[2], hh[3], hh[4], hh[5]};
              add_term(acc, accc, t9);
            }
          } else {
            // study mode: the whole term in FP64, folded into the compensated
            // pair as a (hi, lo) split
            const double r64 = ((double)ring + (double)xr) * (double)g.ring_step;
            double dtau[3];
#pragma unroll
            for (int k = 0; k < 3; k++) dtau[k] = on_ring[k] ? r64 : (double)dec[k] + (double)tlo[k];
            V3<double> r1 = mk(dtau[0] * wv[0].x, dtau[0] * wv[0].y, dtau[0] * wv[0].z);
            V3<double> r2 = mk(dtau[1] * wv[1].x, dtau[1] * wv[1].y, dtau[1] * wv[1].z);
            V3<double> r3 = mk(dtau[2] * wv[2].x, dtau[2] * wv[2].y, dtau[2] * wv[2].z);
            double g64[3], h64[6];
            double wL64 = ring < 0 ? (double)Lf : (double)g.ring_step * (double)Lf;
            const V3<double> cs = crossv(r2 - r1, r3 - r1);
            if (triangle_term<double>(r1, r2, r3, dtau[0], dtau[1], dtau[2], dw, cs, far, wL64, (double)mu, g64,
                                      h64)) {
              float hi[9], lo[9];
#pragma unroll
              for (int k = 0; k < 9; k++) {
                const double x = k < 3 ? g64[k] : h64[k - 3];
                hi[k] = (float)x;
                lo[k] = (float)(x - (double)hi[k]);
              }
              add_term2(acc, accc, hi, lo);
            }
          }
          if (COUNT) n_terms++;
        }
        // band partial sums: lanes -> FP64 across the wave -> record accumulator
#pragma unroll
        for (int k = 0; k < 9; k++) {
          double sk = wave_sum((double)acc[k] + (double)accc[k]);
          if (lane == 0) racc[2 + 9 * chn + k] += sk;
        }
        }  // channels
      }
      __syncthreads();
      if (COUNT) { uint64_t t = clock64(); cyc[3] += t - t_mark; t_mark = t; }
    }
    }  // sectors
    // ---- store ------------------------------------------------------------
    if (S > 1) {
      // parts leave FP64 partial sums; the last part to finish adds them in
      // part order (deterministic) and stores the record
      double* pp = g.partial + ((size_t)rec * S + part) * 20;
      if (lane < 20) pp[lane] = racc[lane];
      __threadfence();
      unsigned int old = 0;
      if (lane == 0) old = atomicAdd(&g.done[rec], 1u);
      old = __shfl(old, 0, kWave);
      if (old != (unsigned int)(S - 1)) continue;
      __threadfence();
      if (lane < 20) {
        double sum = 0.0;
        for (int k = 0; k < S; k++)
          sum += __hip_atomic_load(g.partial + ((size_t)rec * S + k) * 20 + lane, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        racc[lane] = sum;
      }
      __syncthreads();
    }
    if (lane < 2) g.value[2 * rec + lane] = racc[lane] / (double)N;
    if (lane == 0) atomicAdd(&g.queue[kQueueDone], 1u);  // progress, read by the host watchdog
    if (lane < 18) {
      int c = lane / 9, k = lane % 9;
      if (k < 3) g.grad[6 * rec + 3 * c + k] = racc[2 + lane];
      else g.hess[12 * rec + 6 * c + (k - 3)] = racc[2 + lane];
    }
    __syncthreads();
  }
  if (COUNT) {
    // wave-level totals, one atomic per wave
    double r = wave_sum((double)n_rays), nd = wave_sum((double)tc.nodes), tr = wave_sum((double)tc.tris),
           te = wave_sum((double)n_terms);
    if (lane == 0) {
      atomicAdd(&g.counters[0], (unsigned long long)r);
      atomicAdd(&g.counters[1], (unsigned long long)nd);
      atomicAdd(&g.counters[2], (unsigned long long)tr);
      atomicAdd(&g.counters[3], (unsigned long long)te);
      for (int k = 0; k < 4; k++) atomicAdd(&g.counters[4 + k], (unsigned long long)cyc[k]);
      atomicAdd(&g.counters[8], (unsigned long long)sh_iter);
      atomicAdd(&g.counters[9], (unsigned long long)sh_busy);
      atomicAdd(&g.counters[10], (unsigned long long)sh_refill);
      atomicAdd(&g.counters[11], (unsigned long long)sh_lanes);
    }
  }
}

// ---------------------------------------------------------------------------
// primary rays of a whole batch, coherent: workgroup (b, d) traces direction
// d of the 64 records at queue slots 64 b .. 64 b + 63 (nearby points with the
// device-built queue, one stratum: nearly parallel rays), one lane per record,
// with the record kernel's closest-hit traversal (so the same hits).
// ---------------------------------------------------------------------------
template <int STACK>
__global__ __launch_bounds__(64) void primary_kernel(RecordArgs g, int nq, int blk0) {
  __shared__ int stack_lds[STACK * kWave];
  const int lane = threadIdx.x;
  // grid (direction, block): consecutive workgroups take the directions of
  // one block of records
  const int d = blockIdx.x, blk = blk0 + (int)blockIdx.y;
  const int qr = blk * kWave + lane;
  if (qr >= nq) return;
  const int rec = g.order ? g.order[qr] : qr;
  if (rec < 0 || rec >= g.P) return;
  const int nth = g.n_theta[rec], nph = g.n_phi[rec];
  const float3 x = make_float3(g.pos[3 * rec], g.pos[3 * rec + 1], g.pos[3 * rec + 2]);
  // the record kernel's validity test: invalid records are not traced
  if (!(nth >= 2 && nph >= 5 && nph <= g.max_n_phi && nth <= g.max_n_theta) ||
      !(x.x >= g.box_lo.x && x.x <= g.box_hi.x) || !(x.y >= g.box_lo.y && x.y <= g.box_hi.y) ||
      !(x.z >= g.box_lo.z && x.z <= g.box_hi.z))
    return;
  const int N = nth * nph;
  if (d > N + 1) return;
  int a, col = 0;
  if (d == 0) {
    a = -1;
  } else if (d == N + 1) {
    a = nth;
  } else {
    a = (d - 1) / nph;
    col = (d - 1) - a * nph;
  }
  const uint64_t key = record_key(g.seed, (uint64_t)(g.rec_base + (g.common_random ? 0 : rec)));
  const float3 w = row_direction(key, a, col, nth, nph);
  int id;
  float t;
  bool fr;
  TraceCount tc;
  trace_closest<false>(g.nodes, g.tris, g.tri_stride, x, w, stack_lds + lane, g.leaf_batch, id, t, fr, tc);
  const int code = id >= 0 ? ((id << 1) | (fr ? 1 : 0)) : -1;
  g.hits[hit_slot(qr, d, g.hit_stride)] = make_float2(t, __int_as_float(code));
  if (g.vis) {
    // the ray's vertices as the record kernel takes them: the surface vertex
    // (a hit) and the ring vertices in front of the hit or box exit
    const float xr = uniform24(key, kRingIdx, 0);
    const float tt = code < 0 ? box_exit(x, w, g.box_lo, g.box_hi) : t;
    int M = 0;
    while (M < g.max_rings && ring_distance(M, xr, g.ring_step) < tt) M++;
    unsigned int words[kVisMaxWords] = {0u, 0u, 0u, 0u};
    for (int kk = code >= 0 ? 0 : 1; kk <= M; kk++) {
      int skip = -1;
      float3 o, nrm = make_float3(0.f, 0.f, 0.f);
      if (kk == 0) {
        skip = code >> 1;
        o = axpy3(t, w, x);
        const float4 sh = g.shade[skip];
        const float nsign = (code & 1) ? 1.f : -1.f;
        nrm = make_float3(nsign * sh.x, nsign * sh.y, nsign * sh.z);
      } else {
        o = axpy3(ring_distance(kk - 1, xr, g.ring_step), w, x);
      }
      const unsigned int bits = (unsigned int)light_bits<false>(g.lights, g.n_lights, g.lb_desc, g.lb_offs, g.lb_ent, o, skip, nrm, stack_lds + lane, tc);
      const int pos = kk << g.vis_shift;
#pragma unroll
      for (int q = 0; q < kVisMaxWords; q++)
        if (q == (pos >> 5)) words[q] |= bits << (pos & 31);
    }
    const size_t w0 = ((size_t)blk * (size_t)g.hit_stride + (size_t)d) * (size_t)g.vis_words;
#pragma unroll
    for (int q = 0; q < kVisMaxWords; q++)
      if (q < g.vis_words) g.vis[(w0 + q) * kWave + lane] = words[q];
  }
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
// clears the queue words that must start at zero: pop counters, invalid
// records, progress
__global__ void reset_queue_kernel(unsigned int* q) {
  const int t = threadIdx.x;
  if (t < kQueueClassNext + kOrderClasses || t == kQueueDone) q[t] = 0u;
}

// Queue order (see kernels.hpp): bucket of a record = class block (widest
// n_phi class first), cost octave (largest first), Morton cell of the box's
// 8x8x8 grid.  Records with n_phi above the call's max_n_phi (invalid: the
// record kernel writes NaN and counts it) are queued in max_n_phi's class so
// that one of the launches pops them; points outside the box (also invalid)
// are clamped to the nearest cell.
RC_DEV int order_class(int nph) { return nph <= 16 ? 0 : (nph <= 32 ? 1 : (nph <= 64 ? 2 : (nph <= 128 ? 3 : 4))); }
RC_DEV int order_bucket(int nth, int nph, int max_nph, float x, float y, float z, float3 lo, float3 inv) {
  const float n = fmaxf((float)nth * (float)nph, 1.f);
  const int cb = min(max((int)log2f(n), 0), kOrderCost - 1);
  // fminf/fmaxf drop a NaN coordinate (cell 0)
  const int cx = (int)fminf(fmaxf((x - lo.x) * inv.x, 0.f), 7.f);
  const int cy = (int)fminf(fmaxf((y - lo.y) * inv.y, 0.f), 7.f);
  const int cz = (int)fminf(fmaxf((z - lo.z) * inv.z, 0.f), 7.f);
  int cell = 0;
  for (int b = 2; b >= 0; b--) cell = (cell << 3) | (((cx >> b) & 1) << 2) | (((cy >> b) & 1) << 1) | ((cz >> b) & 1);
  const int blk = kOrderClasses - 1 - order_class(min(nph, max_nph));
  return (blk * kOrderCost + (kOrderCost - 1 - cb)) * kOrderCells + cell;
}
__global__ void order_hist_kernel(const int* nth, const int* nph, const float* pos, float3 lo, float3 inv, int P,
                                  int max_nph, unsigned int* hist) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  atomicAdd(&hist[order_bucket(nth[i], nph[i], max_nph, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], lo, inv)], 1u);
}
// Exclusive prefix sums of the bucket counts (the first queue slot of each
// bucket) and the [lo, hi) queue range of each class, by one block: each
// thread sums a run of buckets, the run sums are scanned in LDS, then each
// thread writes its run.
__global__ __launch_bounds__(kOrderScanThreads) void order_scan_kernel(const unsigned int* hist, unsigned int* cursor,
                                                                       unsigned int* class_range) {
  constexpr int kRun = kOrderBuckets / kOrderScanThreads;
  __shared__ unsigned int part[kOrderScanThreads];
  const int t = threadIdx.x;
  unsigned int sum = 0;
  for (int i = 0; i < kRun; i++) sum += hist[t * kRun + i];
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < kOrderScanThreads; off <<= 1) {
    const unsigned int v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  unsigned int run = part[t] - sum;
  for (int i = 0; i < kRun; i++) {
    const int b = t * kRun + i;
    if (b % kOrderGroup == 0) {  // class block blk starts here (and block blk - 1 ends)
      const int blk = b / kOrderGroup;
      class_range[2 * (kOrderClasses - 1 - blk)] = run;
      if (blk > 0) class_range[2 * (kOrderClasses - blk) + 1] = run;
    }
    cursor[b] = run;
    run += hist[b];
  }
  if (t == kOrderScanThreads - 1) class_range[1] = run;  // the last block: class 0
}
__global__ void order_scatter_kernel(const int* nth, const int* nph, const float* pos, float3 lo, float3 inv, int P,
                                     int max_nph, unsigned int* cursor, int* order) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const int b = order_bucket(nth[i], nph[i], max_nph, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], lo, inv);
  unsigned int p = atomicAdd(&cursor[b], 1u);
  order[p] = i;
}
__global__ void zero_u32_kernel(unsigned int* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// validity radius: Jacobi eigen-decomposition of the summed 3x3 Hessian (FP64)
// ---------------------------------------------------------------------------
__global__ void radius_kernel(const double* __restrict__ value, const double* __restrict__ hess, int P, float eps,
                              float r_min, float r_max, float* __restrict__ R, float* __restrict__ axes) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  double L = value[2 * i] + value[2 * i + 1];
  const double* h0 = hess + 12 * i;
  double h[6];
  for (int k = 0; k < 6; k++) h[k] = h0[k] + h0[6 + k];
  double a[3][3] = {{h[0], h[1], h[2]}, {h[1], h[3], h[4]}, {h[2], h[4], h[5]}};
  double v[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int sweep = 0; sweep < 12; sweep++) {
    double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    double dg = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (!(off > 1e-30 * dg) || off == 0.0) break;
    for (int p = 0; p < 2; p++)
      for (int q = p + 1; q < 3; q++) {
        if (a[p][q] == 0.0) continue;
        double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; k++) {  // A <- A J (columns p, q)
          double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - s * akq;
          a[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; k++) {  // A <- J^T A (rows p, q)
          double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - s * aqk;
          a[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; k++) {
          double vkp = v[k][p], vkq = v[k][q];
          v[k][p] = c * vkp - s * vkq;
          v[k][q] = s * vkp + c * vkq;
        }
      }
  }
  double lam[3] = {a[0][0], a[1][1], a[2][2]};
  double Ri[3];
  for (int k = 0; k < 3; k++) {
    double al = fabs(lam[k]);
    double r;
    if (!(L > 0.0)) r = r_min;
    else if (al == 0.0) r = r_max;
    else r = pow(15.0 * L * (double)eps / (4.0 * kPi * al), 0.2);
    if (!(r >= (double)r_min)) r = r_min;  // also catches NaN
    if (r > (double)r_max) r = r_max;
    Ri[k] = r;
  }
  R[i] = (float)fmin(Ri[0], fmin(Ri[1], Ri[2]));
  if (axes) {
    for (int k = 0; k < 3; k++) axes[12 * i + k] = (float)Ri[k];
    for (int k = 0; k < 3; k++)
      for (int c = 0; c < 3; c++) axes[12 * i + 3 + 3 * k + c] = (float)v[c][k];  // row k = eigenvector k
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
size_t record_lds_bytes(int stack, int max_n_phi, int max_rings) {
  size_t words = (size_t)stack * kWave + 2 * (size_t)max_n_phi * (kRowFields + max_rings) + ((2 * (size_t)max_n_phi + 2) & ~size_t(1));
  return words * 4 + 20 * sizeof(double);
}

template <int S, bool C, bool D>
static const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&record_kernel<S, C, D>);
}

// kernel variants: stack depth {8 (hits pass and light bins), 16, 24, 32, 48, 64} x counting x FP64 study mode
static int stack_index(int stack) {
  return stack <= kHitsStack ? 0 : stack <= 16 ? 1 : (stack <= 24 ? 2 : (stack <= 32 ? 3 : (stack <= 48 ? 4 : 5)));
}
#define RC_KVARIANTS(S) \
  {{kernel_ptr<S, false, false>(), kernel_ptr<S, false, true>()}, {kernel_ptr<S, true, false>(), kernel_ptr<S, true, true>()}}
static const void* select_kernel(int stack, bool count, bool f64) {
  static const void* const table[6][2][2] = {RC_KVARIANTS(kHitsStack), RC_KVARIANTS(16), RC_KVARIANTS(24),
                                             RC_KVARIANTS(32),         RC_KVARIANTS(48), RC_KVARIANTS(64)};
  return table[stack_index(stack)][count ? 1 : 0][f64 ? 1 : 0];
}

// the stack holds at most (depth - 1) postponed children on one root-to-leaf path
int stack_variant(int depth) { return depth <= 16 ? 16 : (depth <= 24 ? 24 : (depth <= 32 ? 32 : (depth <= 48 ? 48 : 64))); }

int record_occupancy(int stack, bool count, bool f64, size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, select_kernel(stack, count, f64), kWave, lds) != hipSuccess)
    return 0;
  return n;
}

hipError_t prepare_record(int stack, bool count, bool f64, size_t lds) {
  return hipFuncSetAttribute(select_kernel(stack, count, f64), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_record(const RecordArgs& a, int stack, bool count, bool f64, int grid, size_t lds, hipStream_t s) {
  // the stackless variant needs the hits pass and, with lights, the light bins
  if (stack <= kHitsStack && (!a.hits || (a.n_lights > 0 && !a.lb_desc))) return hipErrorInvalidValue;
  void* args[] = {const_cast<RecordArgs*>(&a)};
  return hipLaunchKernel(select_kernel(stack, count, f64), dim3(grid), dim3(kWave), args, lds, s);
}

hipError_t launch_primary(const RecordArgs& a, int stack, int nq, hipStream_t s) {
  const int nblk = (nq + kWave - 1) / kWave;
  constexpr int kBlocks = 65535;  // grid y per launch
  for (int b0 = 0; b0 < nblk; b0 += kBlocks) {
    const dim3 grid(a.hit_stride, nblk - b0 < kBlocks ? nblk - b0 : kBlocks);
    switch (stack <= 16 ? 0 : (stack <= 24 ? 1 : (stack <= 32 ? 2 : (stack <= 48 ? 3 : 4)))) {
      case 0: hipLaunchKernelGGL(primary_kernel<16>, grid, dim3(kWave), 0, s, a, nq, b0); break;
      case 1: hipLaunchKernelGGL(primary_kernel<24>, grid, dim3(kWave), 0, s, a, nq, b0); break;
      case 2: hipLaunchKernelGGL(primary_kernel<32>, grid, dim3(kWave), 0, s, a, nq, b0); break;
      case 3: hipLaunchKernelGGL(primary_kernel<48>, grid, dim3(kWave), 0, s, a, nq, b0); break;
      default: hipLaunchKernelGGL(primary_kernel<64>, grid, dim3(kWave), 0, s, a, nq, b0); break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_reset(unsigned int* q, hipStream_t s) {
  hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, q);
  return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned int* p, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(zero_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_order(const int* nth, const int* nph, const float* pos, float3 box_lo, float3 box_hi, int P,
                        int max_nph, unsigned int* hist, unsigned int* cursor, int* order, unsigned int* class_range,
                        hipStream_t s) {
  const float3 inv = make_float3(8.f / (box_hi.x - box_lo.x), 8.f / (box_hi.y - box_lo.y), 8.f / (box_hi.z - box_lo.z));
  hipLaunchKernelGGL(zero_u32_kernel, dim3(kOrderBuckets / 256), dim3(256), 0, s, hist, kOrderBuckets);
  int blocks = (P + 255) / 256;
  if (blocks > 0)
    hipLaunchKernelGGL(order_hist_kernel, dim3(blocks), dim3(256), 0, s, nth, nph, pos, box_lo, inv, P, max_nph, hist);
  hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(kOrderScanThreads), 0, s, hist, cursor, class_range);
  if (blocks > 0)
    hipLaunchKernelGGL(order_scatter_kernel, dim3(blocks), dim3(256), 0, s, nth, nph, pos, box_lo, inv, P, max_nph,
                       cursor, order);
  return hipGetLastError();
}

hipError_t launch_radius(const double* value, const double* hess, int P, float eps, float r_min, float r_max, float* R,
                         float* axes, hipStream_t s) {
  int blocks = (P + 127) / 128;
  if (blocks > 0)
    hipLaunchKernelGGL(radius_kernel, dim3(blocks), dim3(128), 0, s, value, hess, P, eps, r_min, r_max, R, axes);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ray queries (traversal checks): one ray per lane
// ---------------------------------------------------------------------------
template <int STACK>
__global__ __launch_bounds__(64) void trace_rays_kernel(const float4* __restrict__ nodes,
                                                        const float4* __restrict__ tris, int tri_stride,
                                                        const float* __restrict__ o,
                                                        const float* __restrict__ d, int n, int* __restrict__ hit,
                                                        float* __restrict__ t, int* __restrict__ front,
                                                        float3 lo, float3 hi) {
  __shared__ int stack[STACK * kWave];
  int i = blockIdx.x * kWave + threadIdx.x;
  if (i >= n) return;
  float3 oo = make_float3(o[3 * i], o[3 * i + 1], o[3 * i + 2]);
  float3 dd = make_float3(d[3 * i], d[3 * i + 1], d[3 * i + 2]);
  int id;
  float tt;
  bool fr;
  TraceCount tc;
  trace_closest<false>(nodes, tris, tri_stride, oo, dd, stack + threadIdx.x, 0, id, tt, fr, tc);
  if (id < 0) tt = box_exit(oo, dd, lo, hi);
  hit[i] = id;
  t[i] = tt;
  front[i] = fr ? 1 : 0;
}

template <int STACK>
__global__ __launch_bounds__(64) void occluded_rays_kernel(const float4* __restrict__ nodes,
                                                           const float4* __restrict__ tris, int tri_stride,
                                                           const float* __restrict__ o, const float* __restrict__ d,
                                                           const int* __restrict__ skip, int n, int* __restrict__ occ) {
  __shared__ int stack[STACK * kWave];
  int i = blockIdx.x * kWave + threadIdx.x;
  if (i >= n) return;
  float3 oo = make_float3(o[3 * i], o[3 * i + 1], o[3 * i + 2]);
  float3 dd = make_float3(d[3 * i], d[3 * i + 1], d[3 * i + 2]);
  TraceCount tc;
  occ[i] = occluded<false>(nodes, tris, tri_stride, oo, dd, skip ? skip[i] : -1, stack + threadIdx.x, tc) ? 1 : 0;
}

// segments p -> light through the light bins, one per lane (the same bin
// lookup and entry loop as the record kernel's shadow segments)
__global__ __launch_bounds__(64) void light_occluded_kernel(const int4* __restrict__ desc,
                                                            const int* __restrict__ offs,
                                                            const float4* __restrict__ ent, int l, float4 L,
                                                            const float* __restrict__ pts,
                                                            const int* __restrict__ skip, int n,
                                                            int* __restrict__ occ) {
  const int i = blockIdx.x * kWave + threadIdx.x;
  if (i >= n) return;
  const float3 o = make_float3(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]);
  const float3 d = make_float3(L.x - o.x, L.y - o.y, L.z - o.z);
  const int sk = skip ? skip[i] : -1;
  const WtRay wr = wt_ray(o, d);
  int h[4];
  const int nlev = lb_bins(desc, l, wr, h);
  const float reach = sqrtf(dot3(d, d)) * (1.0f + 0x1p-20f);
  int res = 0;
  for (int k = 0; k < 4 && !res; k++) {
    if (k >= nlev || __int_as_float(offs[h[k] + 1]) > reach) continue;
    const int e1 = offs[h[k] + 2];
    for (int e = offs[h[k]]; e < e1; e++) {
      const float4 q0 = ent[3 * e], q1 = ent[3 * e + 1], q2 = ent[3 * e + 2];
      float t;
      bool fr;
      if (__float_as_int(q0.w) != sk && hit_triangle(wr, q0, q1, q2, 1e-4f, 1.0f, t, fr)) {
        res = 1;
        break;
      }
      if (q2.w > reach) break;
    }
  }
  occ[i] = res;
}

hipError_t launch_light_occluded(const int4* desc, const int* offs, const float4* ent, int l, float4 L,
                                 const float* pts, const int* skip, int n, int* occ, hipStream_t s) {
  const int blocks = (n + kWave - 1) / kWave;
  if (blocks > 0)
    hipLaunchKernelGGL(light_occluded_kernel, dim3(blocks), dim3(kWave), 0, s, desc, offs, ent, l, L, pts, skip, n,
                       occ);
  return hipGetLastError();
}

hipError_t launch_trace_rays(const float4* nodes, const float4* tris, int tri_stride, int depth, const float* o,
                             const float* d, int n,
                             int* hit, float* t, int* front, float3 lo, float3 hi, hipStream_t s) {
  int blocks = (n + kWave - 1) / kWave;
  if (blocks == 0) return hipSuccess;
  int st = stack_variant(depth);
  if (st <= 16) hipLaunchKernelGGL(trace_rays_kernel<16>, dim3(blocks), dim3(kWave), 0, s, nodes, tris, tri_stride, o, d, n, hit, t, front, lo, hi);
  else if (st <= 32) hipLaunchKernelGGL(trace_rays_kernel<32>, dim3(blocks), dim3(kWave), 0, s, nodes, tris, tri_stride, o, d, n, hit, t, front, lo, hi);
  else if (st <= 48) hipLaunchKernelGGL(trace_rays_kernel<48>, dim3(blocks), dim3(kWave), 0, s, nodes, tris, tri_stride, o, d, n, hit, t, front, lo, hi);
  else hipLaunchKernelGGL(trace_rays_kernel<64>, dim3(blocks), dim3(kWave), 0, s, nodes, tris, tri_stride, o, d, n, hit, t, front, lo, hi);
  return hipGetLastError();
}

hipError_t launch_occluded_rays(const float4* nodes, const float4* tris, int tri_stride, int depth, const float* o,
                                const float* d,
                                const int* skip, int n, int* occ, hipStream_t s) {
  int blocks = (n + kWave - 1) / kWave;
  if (blocks == 0) return hipSuccess;
  int st = stack_variant(depth);
  if (st <= 16) hipLaunchKernelGGL(occluded_rays_kernel<16>, dim3(blocks), dim3(kWave), 0, s, nodes, tris, tri_stride, o, d, skip, n, occ);
  else if (st <= 32) hipLaunchKernelGGL(occluded_rays_kernel<32>, dim3(blocks), dim3(kWave), 0, s, nodes, tris, tri_stride, o, d, skip, n, occ);
  else if (st <= 48) hipLaunchKernelGGL(occluded_rays_kernel<48>, dim3(blocks), dim3(kWave), 0, s, nodes, tris, tri_stride, o, d, skip, n, occ);
  else hipLaunchKernelGGL(occluded_rays_kernel<64>, dim3(blocks), dim3(kWave), 0, s, nodes, tris, tri_stride, o, d, skip, n, occ);
  return hipGetLastError();
}

}  // namespace rc
