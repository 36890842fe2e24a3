/*
 * rco.c -- FP64 CPU oracle for occlusion-aware second-order radiance-cache
 * records in a homogeneous isotropic medium (Marco, Jarabo, Jarosz, Gutierrez,
 * "Second-Order Occlusion-Aware Volumetric Radiance Caching", ACM TOG 37(2),
 * 2018).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is
 * checked against.  Only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code with the GPU library:
 * nothing here includes, links or generates anything used there, and it does
 * not include anything from there.
 *
 * What it computes (one record per cache point x, two channels):
 *   channel 0 "SS": radiance reaching x from the first surface along each
 *                   direction (surface ring, Sec. 4, Eq. ApprxRadiance with
 *                   pdf = 1 for the surface ring);
 *   channel 1 "MS": radiance in-scattered towards x by medium points lit
 *                   directly by the point lights (concentric medium rings,
 *                   Sec. 4 and Sec. 6 "Implementation": uniform ray-marching
 *                   distances, zero-radiance vertex at the surface when an
 *                   occluder is closer than the ring).
 * For each channel:
 *   value    : the unbiased Monte Carlo estimate of Eq. outLF with uniform
 *              stratified sphere sampling (Sec. 4, last paragraph: the value is
 *              computed by plain Monte Carlo, only the derivatives use the
 *              triangulation);
 *   gradient : sum over triangles of Eq. SSSegALGradientSimp, weighted by
 *              1/pdf(ring) (Eq. SegmentRadianceGradient);
 *   Hessian  : sum over triangles of Eq. SSSegALHessianSimp, weighted by
 *              1/pdf(ring) (Eq. SegmentRadianceHessian).
 * Per triangle the radiance, transmittance and scattering are taken at its
 * furthest vertex (Eq. ApproxSegmentRadiance and the assumptions before it);
 * the form factor is the triangle solid angle over 4 pi (App. C,
 * Eq. FFDDDMediaSurfArea); its gradient is Eq. TriToMediaFFGradient and its
 * Hessian is the paper's Eq. TriToMediaFFHessian, evaluated literally (with
 * J(grad|A|) = 0 as App. C shows), except for one correction: the boxed
 * expression for grad A in App. C has the signs of two cross products
 * flipped; we use grad A = -(r1 x r2 + r2 x r3 + r3 x r1), the derivative of
 * the triple product, which the finite-difference pins confirm.
 * Transmittance derivatives follow App. A.
 *
 * Normalisation: the record is  integral of f_s * L_i over the sphere with
 * f_s = 1/(4 pi) (Eq. outLF with the isotropic phase function; the
 * scattering coefficient at x itself is left to the caller).  Each triangle's
 * form factor Omega/(4 pi) already carries f_s, so value and derivatives share
 * one normalisation.
 *
 * Precision: every continuous quantity is FP64.  Discrete decisions that the
 * GPU kernel takes in FP32 (which triangle a ray hits, whether a shadow ray is
 * blocked, whether a ring lies in front of the hit, which triangle vertex is
 * furthest, which quad diagonal is used) are taken here in FP32 with the same
 * published formulas, so that both sides take the same decisions; the FP64
 * values are then recomputed from those decisions.  The decision rules are:
 *   - ray/triangle: the watertight test of Woop, Benthin and Wald (JCGT
 *     2013) in a division-free form (see wt32): FP32 projection of the
 *     vertices along the ray, 2-D edge functions with exact signs (FP64
 *     from the FP32 points), so every ray that meets a closed mesh hits it,
 *     at any angle and any distance from a surface (Sec. 4 takes each
 *     sample at the first surface seen from x);
 *   - closest hit: smallest FP32 t, ties to the lowest triangle index;
 *   - shadow rays: segment y -> light, hit if 1e-4 < t < 1 (t in units of the
 *     unnormalised segment), the surface vertex's own triangle excluded;
 *   - escaping rays: FP32 slab exit of the medium box.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define RCO_PI 3.14159265358979323846
#define RCO_OK 0
#define RCO_EINVAL (-1)
#define RCO_ENOMEM (-2)

/* ------------------------------------------------------------------ */
/* counter-based random numbers: splitmix64 (Steele, Lea, Flood 2014)   */
/* ------------------------------------------------------------------ */
static uint64_t sm64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
/* per-record key and a uniform float in [0,1) with 24 random bits */
static uint64_t rec_key(uint64_t seed, uint64_t rec) { return sm64(sm64(seed) ^ rec); }
static float unif(uint64_t key, uint64_t idx, uint64_t dim) {
  return (float)(sm64(sm64(key ^ idx) ^ dim) >> 40) * 0x1p-24f;
}
#define RCO_RING_IDX 0xFFFFFFFFull

/* ------------------------------------------------------------------ */
/* small FP32 vector helpers (decisions only; compiled without FMA)     */
/* ------------------------------------------------------------------ */
typedef struct { float x, y, z; } f3;
static f3 f3_sub(f3 a, f3 b) { f3 r = {a.x - b.x, a.y - b.y, a.z - b.z}; return r; }
static f3 f3_cross(f3 a, f3 b) {
  f3 r = {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
  return r;
}
static float f3_dot(f3 a, f3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }

/* ------------------------------------------------------------------ */
/* small FP64 helpers                                                   */
/* ------------------------------------------------------------------ */
static double d3_dot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void d3_cross(const double* a, const double* b, double* r) {
  double t0 = a[1] * b[2] - a[2] * b[1], t1 = a[2] * b[0] - a[0] * b[2], t2 = a[0] * b[1] - a[1] * b[0];
  r[0] = t0; r[1] = t1; r[2] = t2;
}
static double d3_norm(const double* a) { return sqrt(d3_dot(a, a)); }

/* ------------------------------------------------------------------ */
/* scene                                                                */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t T;
  f3 *v0, *v1, *v2;   /* FP32 vertices (decision data) */
  double* n64;        /* unit geometric normal e1 x e2 (FP64 from the FP32 vertices) [T][3] */
  double* v064;       /* v0 in FP64 [T][3] */
  float *albedo, *emission;
  f3 lo, hi;          /* medium box */
  /* acceleration: k-ary hierarchy of padded boxes over Morton-sorted triangles */
  int64_t* perm;      /* sorted triangle index */
  int nlev;           /* level 0 = groups of triangles, nlev-1 = top */
  int64_t* lev_n;     /* nodes per level */
  double** lev_box;   /* [lev][node][6] lo.xyz hi.xyz */
  double pad;
} rco_scene;

#define RCO_FAN 16

static uint64_t morton_expand(uint64_t v) { /* 21 bits -> every third bit */
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}
/* Padding of the triangle boxes.  A hit accepted by wt32 lies at a point
 * o + t d that is a convex combination of the vertices, each moved by at most
 * ~8 units of FP32 rounding (2^-24) times the largest vertex-to-origin
 * coordinate: the FP32 projection and the FP32 rounding of t are the only
 * inexact steps (the barycentric weights are FP64 with exact signs).  So every
 * accepted hit point lies within 16 * 2^-24 * scale of the triangle's box
 * (scale = the medium box's largest side, which bounds every vertex-to-origin
 * distance); the boxes are padded by 2^-16 * scale, 16 times that bound, so
 * culling never removes a triangle the test would accept. */
static double tri_pad(double scale) { return ldexp(scale, -16); }
typedef struct { uint64_t key; int64_t idx; } kv;
static int kv_cmp(const void* a, const void* b) {
  const kv* x = (const kv*)a; const kv* y = (const kv*)b;
  if (x->key < y->key) return -1;
  if (x->key > y->key) return 1;
  return (x->idx < y->idx) ? -1 : (x->idx > y->idx);
}

void rco_scene_destroy(rco_scene* s) {
  if (!s) return;
  free(s->v0); free(s->v1); free(s->v2); free(s->n64); free(s->v064);
  free(s->albedo); free(s->emission); free(s->perm);
  if (s->lev_box) for (int l = 0; l < s->nlev; l++) free(s->lev_box[l]);
  free(s->lev_box); free(s->lev_n);
  free(s);
}

int rco_scene_create(const float* tri, const float* albedo, const float* emission, int64_t T,
                     const float* box_lo, const float* box_hi, rco_scene** out) {
  if (!out || T < 0 || (T > 0 && (!tri || !albedo)) || !box_lo || !box_hi) return RCO_EINVAL;
  rco_scene* s = (rco_scene*)calloc(1, sizeof(rco_scene));
  if (!s) return RCO_ENOMEM;
  s->T = T;
  int64_t Tn = T > 0 ? T : 1;
  s->v0 = (f3*)malloc(sizeof(f3) * Tn); s->v1 = (f3*)malloc(sizeof(f3) * Tn); s->v2 = (f3*)malloc(sizeof(f3) * Tn);
  s->n64 = (double*)malloc(sizeof(double) * 3 * Tn);
  s->v064 = (double*)malloc(sizeof(double) * 3 * Tn);
  s->albedo = (float*)malloc(sizeof(float) * Tn); s->emission = (float*)calloc(Tn, sizeof(float));
  s->perm = (int64_t*)malloc(sizeof(int64_t) * Tn);
  if (!s->v0 || !s->v1 || !s->v2 || !s->n64 || !s->v064 || !s->albedo || !s->emission || !s->perm) {
    rco_scene_destroy(s); return RCO_ENOMEM;
  }
  s->lo.x = box_lo[0]; s->lo.y = box_lo[1]; s->lo.z = box_lo[2];
  s->hi.x = box_hi[0]; s->hi.y = box_hi[1]; s->hi.z = box_hi[2];
  double ext = 0.0;
  for (int a = 0; a < 3; a++) ext = fmax(ext, (double)box_hi[a] - (double)box_lo[a]);
  for (int64_t j = 0; j < T; j++) {
    const float* t = tri + 9 * j;
    f3 a = {t[0], t[1], t[2]}, b = {t[3], t[4], t[5]}, c = {t[6], t[7], t[8]};
    s->v0[j] = a; s->v1[j] = b; s->v2[j] = c;
    double A[3] = {t[0], t[1], t[2]}, B[3] = {t[3], t[4], t[5]}, C[3] = {t[6], t[7], t[8]};
    double E1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]}, E2[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
    double N[3]; d3_cross(E1, E2, N);
    double ln = d3_norm(N);
    for (int k = 0; k < 3; k++) { s->n64[3 * j + k] = ln > 0 ? N[k] / ln : 0.0; s->v064[3 * j + k] = A[k]; }
    s->albedo[j] = albedo[j];
    s->emission[j] = emission ? emission[j] : 0.0f;
    for (int k = 0; k < 9; k++) ext = fmax(ext, fabs((double)t[k] - (double)box_lo[k % 3]));
  }
  /* scale for the box padding (see tri_pad) */
  s->pad = ext > 0 ? ext : 1.0;
  /* Morton order of centroids inside the scene bounds */
  double smin[3] = {1e300, 1e300, 1e300}, smax[3] = {-1e300, -1e300, -1e300};
  for (int64_t j = 0; j < T; j++)
    for (int k = 0; k < 9; k++) { smin[k % 3] = fmin(smin[k % 3], tri[9 * j + k]); smax[k % 3] = fmax(smax[k % 3], tri[9 * j + k]); }
  kv* keys = (kv*)malloc(sizeof(kv) * Tn);
  if (!keys) { rco_scene_destroy(s); return RCO_ENOMEM; }
  for (int64_t j = 0; j < T; j++) {
    uint64_t m = 0;
    for (int k = 0; k < 3; k++) {
      double c = ((double)tri[9 * j + k] + tri[9 * j + 3 + k] + tri[9 * j + 6 + k]) / 3.0;
      double w = smax[k] - smin[k];
      double u = w > 0 ? (c - smin[k]) / w : 0.0;
      uint64_t q = (uint64_t)fmin(fmax(u * 2097151.0, 0.0), 2097151.0);
      m |= morton_expand(q) << k;
    }
    keys[j].key = m; keys[j].idx = j;
  }
  qsort(keys, (size_t)T, sizeof(kv), kv_cmp);
  for (int64_t j = 0; j < T; j++) s->perm[j] = keys[j].idx;
  free(keys);
  /* levels */
  int cap = 16;
  s->lev_n = (int64_t*)malloc(sizeof(int64_t) * cap);
  s->lev_box = (double**)calloc(cap, sizeof(double*));
  int64_t nprev = T;
  int l = 0;
  do {
    int64_t n = (nprev + RCO_FAN - 1) / RCO_FAN;
    if (n == 0) n = 1;
    s->lev_n[l] = n;
    s->lev_box[l] = (double*)malloc(sizeof(double) * 6 * n);
    for (int64_t i = 0; i < n; i++) {
      double* b = s->lev_box[l] + 6 * i;
      b[0] = b[1] = b[2] = 1e300; b[3] = b[4] = b[5] = -1e300;
      for (int64_t c = i * RCO_FAN; c < (i + 1) * RCO_FAN && c < nprev; c++) {
        if (l == 0) {
          const float* t = tri + 9 * s->perm[c];
          double pd = tri_pad(s->pad);
          for (int k = 0; k < 9; k++) {
            b[k % 3] = fmin(b[k % 3], (double)t[k] - pd);
            b[3 + k % 3] = fmax(b[3 + k % 3], (double)t[k] + pd);
          }
        } else {
          const double* cb = s->lev_box[l - 1] + 6 * c;
          for (int k = 0; k < 3; k++) { b[k] = fmin(b[k], cb[k]); b[3 + k] = fmax(b[3 + k], cb[3 + k]); }
        }
      }
    }
    nprev = n; l++;
  } while (nprev > RCO_FAN && l < cap);
  s->nlev = l;
  *out = s;
  return RCO_OK;
}

/* ------------------------------------------------------------------ */
/* FP32 decision: watertight ray/triangle test                          */
/* ------------------------------------------------------------------ */
/* Woop, Benthin and Wald, "Watertight Ray/Triangle Intersection", JCGT 2(1),
 * 2013, written without divisions.  With kz the axis of the largest |d|
 * component (ties to the lower axis) and (kx, ky) = (kz+1, kz+2) mod 3, each
 * vertex v is projected along the ray to the 2-D point
 *   p(v) = (d_kz a_kx - d_kx a_kz,  d_kz a_ky - d_ky a_kz),  a = v - o,
 * in FP32 without fused operations (d_kz times the published sheared
 * coordinates).  The edge functions U = p(v1) x p(v2), V = p(v2) x p(v0),
 * W = p(v0) x p(v1) are FP64 from the FP32 points: the products are exact
 * and one rounding keeps every sign exact, so the origin's side of each
 * projected edge is decided exactly and a ray through an edge shared by two
 * triangles is never lost.  Hit iff U, V, W are all >= 0 or all <= 0 and
 * D = U + V + W != 0; then t = (U a_kz(v0) + V a_kz(v1) + W a_kz(v2)) /
 * (D d_kz) in FP64, rounded once to FP32, and tmin < t < tmax.  D d_kz has the
 * sign of d . ((v1 - v0) x (v2 - v0)), so front (the ray travels against that
 * normal) is D d_kz < 0. */
static int ray_axis(f3 d) {
  float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
  int k = 0;
  float m = ax;
  if (ay > m) { k = 1; m = ay; }
  if (az > m) k = 2;
  return k;
}
static float f3_at(f3 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }
static int wt32(const rco_scene* s, int64_t j, f3 o, f3 d, int kz, float tmin, float tmax, float* tout, int* front) {
  const int kx = (kz + 1) % 3, ky = (kz + 2) % 3;
  const f3 vs[3] = {s->v0[j], s->v1[j], s->v2[j]};
  const float dx = f3_at(d, kx), dy = f3_at(d, ky), dz = f3_at(d, kz);
  double px[3], py[3], pz[3];
  for (int i = 0; i < 3; i++) {
    f3 a = f3_sub(vs[i], o);
    float ax = f3_at(a, kx), ay = f3_at(a, ky), az = f3_at(a, kz);
    float qx = dz * ax - dx * az;
    float qy = dz * ay - dy * az;
    px[i] = qx; py[i] = qy; pz[i] = az;
  }
  double U = px[1] * py[2] - py[1] * px[2];
  double V = px[2] * py[0] - py[2] * px[0];
  double W = px[0] * py[1] - py[0] * px[1];
  if ((U < 0.0 || V < 0.0 || W < 0.0) && (U > 0.0 || V > 0.0 || W > 0.0)) return 0;
  double D = (U + V) + W;
  if (D == 0.0) return 0;
  double num = (U * pz[0] + V * pz[1]) + W * pz[2];
  double den = D * (double)dz;
  float t = (float)(num / den);
  if (!(t > tmin && t < tmax)) return 0;
  *tout = t;
  *front = den < 0.0;
  return 1;
}

/* FP64 slab test of a padded box against the ray o + t d, t in [t0, t1] */
static int box_hit(const double* b, const double* o, const double* d, double t0, double t1) {
  for (int k = 0; k < 3; k++) {
    if (d[k] == 0.0) {
      if (o[k] < b[k] || o[k] > b[3 + k]) return 0;
    } else {
      double ta = (b[k] - o[k]) / d[k], tb = (b[3 + k] - o[k]) / d[k];
      if (ta > tb) { double tt = ta; ta = tb; tb = tt; }
      if (ta > t0) t0 = ta;
      if (tb < t1) t1 = tb;
      if (t0 > t1) return 0;
    }
  }
  return 1;
}

typedef struct { int hit; int64_t id; float t; int front; } hit32;

/* Closest hit.  The hierarchy only skips boxes the ray cannot reach with a
 * t at or below the current best, so the result equals testing every
 * triangle (checked against brute force by the tests). */
static void closest_rec(const rco_scene* s, int lev, int64_t node, const double* o64, const double* d64,
                        f3 o, f3 d, int kz, hit32* best) {
  double tmax = best->hit ? (double)best->t * (1.0 + 1e-6) + 1e-6 : 1e300;
  if (!box_hit(s->lev_box[lev] + 6 * node, o64, d64, 0.0, tmax)) return;
  int64_t nchild = (lev == 0) ? s->T : s->lev_n[lev - 1];
  for (int64_t c = node * RCO_FAN; c < (node + 1) * RCO_FAN && c < nchild; c++) {
    if (lev == 0) {
      int64_t j = s->perm[c];
      float t; int fr;
      if (wt32(s, j, o, d, kz, 0.0f, INFINITY, &t, &fr)) {
        if (!best->hit || t < best->t || (t == best->t && j < best->id)) {
          best->hit = 1; best->id = j; best->t = t; best->front = fr;
        }
      }
    } else {
      closest_rec(s, lev - 1, c, o64, d64, o, d, kz, best);
    }
  }
}
static hit32 trace_closest(const rco_scene* s, f3 o, f3 d) {
  hit32 best = {0, -1, 0.0f, 0};
  if (s->T == 0) return best;
  double o64[3] = {o.x, o.y, o.z}, d64[3] = {d.x, d.y, d.z};
  int kz = ray_axis(d);
  int top = s->nlev - 1;
  for (int64_t n = 0; n < s->lev_n[top]; n++) closest_rec(s, top, n, o64, d64, o, d, kz, &best);
  return best;
}
static hit32 trace_closest_brute(const rco_scene* s, f3 o, f3 d) {
  hit32 best = {0, -1, 0.0f, 0};
  int kz = ray_axis(d);
  for (int64_t j = 0; j < s->T; j++) {
    float t; int fr;
    if (wt32(s, j, o, d, kz, 0.0f, INFINITY, &t, &fr))
      if (!best.hit || t < best.t || (t == best.t && j < best.id)) { best.hit = 1; best.id = j; best.t = t; best.front = fr; }
  }
  return best;
}

static int occluded_rec(const rco_scene* s, int lev, int64_t node, const double* o64, const double* d64,
                        f3 o, f3 d, int kz, int64_t skip) {
  if (!box_hit(s->lev_box[lev] + 6 * node, o64, d64, 0.0, 1.0)) return 0;
  int64_t nchild = (lev == 0) ? s->T : s->lev_n[lev - 1];
  for (int64_t c = node * RCO_FAN; c < (node + 1) * RCO_FAN && c < nchild; c++) {
    if (lev == 0) {
      int64_t j = s->perm[c];
      float t; int fr;
      if (j != skip && wt32(s, j, o, d, kz, 1e-4f, 1.0f, &t, &fr)) return 1;
    } else if (occluded_rec(s, lev - 1, c, o64, d64, o, d, kz, skip)) {
      return 1;
    }
  }
  return 0;
}
/* shadow segment from o to o + d (d = light - o), own triangle `skip` excluded */
static int occluded(const rco_scene* s, f3 o, f3 d, int64_t skip) {
  if (s->T == 0) return 0;
  double o64[3] = {o.x, o.y, o.z}, d64[3] = {d.x, d.y, d.z};
  int kz = ray_axis(d);
  int top = s->nlev - 1;
  for (int64_t n = 0; n < s->lev_n[top]; n++)
    if (occluded_rec(s, top, n, o64, d64, o, d, kz, skip)) return 1;
  return 0;
}
static int occluded_brute(const rco_scene* s, f3 o, f3 d, int64_t skip) {
  int kz = ray_axis(d);
  for (int64_t j = 0; j < s->T; j++) {
    float t; int fr;
    if (j != skip && wt32(s, j, o, d, kz, 1e-4f, 1.0f, &t, &fr)) return 1;
  }
  return 0;
}

/* FP32 exit distance from the medium box (rays that hit nothing) */
static float box_exit32(const rco_scene* s, f3 o, f3 d) {
  float t = INFINITY;
  float oo[3] = {o.x, o.y, o.z}, dv[3] = {d.x, d.y, d.z};
  float lo[3] = {s->lo.x, s->lo.y, s->lo.z}, hi[3] = {s->hi.x, s->hi.y, s->hi.z};
  for (int k = 0; k < 3; k++) {
    if (dv[k] > 0.0f) t = fminf(t, (hi[k] - oo[k]) / dv[k]);
    else if (dv[k] < 0.0f) t = fminf(t, (lo[k] - oo[k]) / dv[k]);
  }
  return t > 0.0f ? t : 0.0f;
}
static double box_exit64(const rco_scene* s, const double* o, const double* d) {
  double t = 1e300;
  double lo[3] = {s->lo.x, s->lo.y, s->lo.z}, hi[3] = {s->hi.x, s->hi.y, s->hi.z};
  for (int k = 0; k < 3; k++) {
    if (d[k] > 0.0) t = fmin(t, (hi[k] - o[k]) / d[k]);
    else if (d[k] < 0.0) t = fmin(t, (lo[k] - o[k]) / d[k]);
  }
  return t > 0.0 ? t : 0.0;
}

/* exported tracing entry points (for the traversal tests): FP32 decisions */
int rco_trace(const rco_scene* s, const float* orig, const float* dir, int64_t n, int brute,
              int64_t* hit_id, float* t32, int32_t* front) {
  if (!s || !orig || !dir || n < 0) return RCO_EINVAL;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; i++) {
    f3 o = {orig[3 * i], orig[3 * i + 1], orig[3 * i + 2]}, d = {dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
    hit32 h = brute ? trace_closest_brute(s, o, d) : trace_closest(s, o, d);
    hit_id[i] = h.hit ? h.id : -1;
    t32[i] = h.hit ? h.t : box_exit32(s, o, d);
    if (front) front[i] = h.front;
  }
  return RCO_OK;
}
int rco_occluded(const rco_scene* s, const float* orig, const float* seg, const int64_t* skip, int64_t n,
                 int brute, int32_t* occ) {
  if (!s || !orig || !seg || n < 0) return RCO_EINVAL;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; i++) {
    f3 o = {orig[3 * i], orig[3 * i + 1], orig[3 * i + 2]}, d = {seg[3 * i], seg[3 * i + 1], seg[3 * i + 2]};
    int64_t sk = skip ? skip[i] : -1;
    occ[i] = brute ? occluded_brute(s, o, d, sk) : occluded(s, o, d, sk);
  }
  return RCO_OK;
}

/* ------------------------------------------------------------------ */
/* App. A: homogeneous transmittance and its derivatives               */
/* ------------------------------------------------------------------ */
/* x: shaded point, y: source point. u = x - y, r = |u|.
 * T = exp(-mu r); grad T = -mu (u/r) T;
 * H T = -mu (I/r - u u^T / r^3 - mu u u^T / r^2) T.                     */
void rco_transmittance(const double* x, const double* y, double mu, double* T, double* gT, double* HT) {
  double u[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
  double r = d3_norm(u);
  double t = exp(-mu * r);
  *T = t;
  for (int i = 0; i < 3; i++) gT[i] = -mu * (u[i] / r) * t;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double I = (i == j) ? 1.0 : 0.0;
      HT[3 * i + j] = -mu * (I / r - u[i] * u[j] / (r * r * r) - mu * u[i] * u[j] / (r * r)) * t;
    }
}

/* ------------------------------------------------------------------ */
/* App. C: triangle-to-medium form factor and its derivatives           */
/* ------------------------------------------------------------------ */
/* r1, r2, r3: vertex positions relative to x (r_i = y_i - x).
 * Omega = 2 atan(|A|/B) with pi added for negative arctangents, i.e.
 * 2 atan2(|A|, B); F = Omega / (4 pi).                                  */
void rco_formfactor(const double* r1, const double* r2, const double* r3, double* F, double* gF, double* HF) {
  const double* r[3] = {r1, r2, r3};
  double l[3] = {d3_norm(r1), d3_norm(r2), d3_norm(r3)};
  double c23[3], c12[3], c31[3];
  d3_cross(r2, r3, c23); d3_cross(r1, r2, c12); d3_cross(r3, r1, c31);
  double A = d3_dot(r1, c23);
  double d12 = d3_dot(r1, r2), d23 = d3_dot(r2, r3), d13 = d3_dot(r1, r3);
  double B = l[0] * l[1] * l[2] + d12 * l[2] + d23 * l[0] + d13 * l[1];
  double absA = fabs(A);
  double sgn = (A > 0) ? 1.0 : ((A < 0) ? -1.0 : 0.0);
  *F = 2.0 * atan2(absA, B) / (4.0 * RCO_PI);
  /* grad A (derivative of the triple product; App. C's boxed form corrected) */
  double gA[3], gabsA[3];
  for (int i = 0; i < 3; i++) { gA[i] = -(c12[i] + c23[i] + c31[i]); gabsA[i] = sgn * gA[i]; }
  /* grad r_i = -r_i / |r_i| */
  double gr[3][3];
  for (int k = 0; k < 3; k++)
    for (int i = 0; i < 3; i++) gr[k][i] = -r[k][i] / l[k];
  /* grad B: grad(l1 l2 l3) + sum over (i,j,k) of grad((r_i.r_j) l_k) */
  double gB[3];
  for (int i = 0; i < 3; i++) {
    double g = l[1] * l[2] * gr[0][i] + l[0] * l[2] * gr[1][i] + l[0] * l[1] * gr[2][i];
    g += d12 * gr[2][i] - l[2] * (r1[i] + r2[i]);
    g += d23 * gr[0][i] - l[0] * (r2[i] + r3[i]);
    g += d13 * gr[1][i] - l[1] * (r1[i] + r3[i]);
    gB[i] = g;
  }
  double D = absA * absA + B * B;
  for (int i = 0; i < 3; i++) gF[i] = (B * gabsA[i] - absA * gB[i]) / (2.0 * RCO_PI * D);
  /* J(grad r_k) = I / l_k - r_k r_k^T / l_k^3 */
  double Jr[3][9];
  for (int k = 0; k < 3; k++)
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++)
        Jr[k][3 * i + j] = ((i == j) ? 1.0 / l[k] : 0.0) - r[k][i] * r[k][j] / (l[k] * l[k] * l[k]);
  /* J(grad B) */
  double JB[9];
  static const int tri_ij[3][3] = {{0, 1, 2}, {1, 2, 0}, {0, 2, 1}}; /* (i, j, k): (r_i . r_j) l_k */
  double dots[3] = {d12, d23, d13};
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      /* J(grad(l1 l2 l3)) */
      double v = l[1] * l[2] * Jr[0][3 * i + j] + l[0] * (gr[2][i] * gr[1][j] + gr[1][i] * gr[2][j])
               + l[0] * l[2] * Jr[1][3 * i + j] + l[1] * (gr[2][i] * gr[0][j] + gr[0][i] * gr[2][j])
               + l[0] * l[1] * Jr[2][3 * i + j] + l[2] * (gr[1][i] * gr[0][j] + gr[0][i] * gr[1][j]);
      /* J(grad((r_a . r_b) l_c)) = (r_a.r_b) J(grad l_c) + 2 l_c I - grad l_c (r_a+r_b)^T - (r_a+r_b) grad l_c^T */
      for (int m = 0; m < 3; m++) {
        int a = tri_ij[m][0], b = tri_ij[m][1], c = tri_ij[m][2];
        double sab_i = r[a][i] + r[b][i], sab_j = r[a][j] + r[b][j];
        v += dots[m] * Jr[c][3 * i + j] + ((i == j) ? 2.0 * l[c] : 0.0) - gr[c][i] * sab_j - sab_i * gr[c][j];
      }
      JB[3 * i + j] = v;
    }
  /* J(grad|A|) = (A J(grad A) + grad A grad A^T)/|A| - A^2 grad A grad A^T/|A|^3, and
   * J(grad A) = 0, so J(grad|A|) = 0 for A != 0. */
  /* Eq. TriToMediaFFHessian, literally:
   * HF = 1/(2 pi) [ (g|A| gB^T - gB g|A|^T)/D + (B J(g|A|) - |A| J(gB))/D
   *                 - (B g|A| - |A| gB)(grad(|A|^2) + grad(B^2))^T / D^2 ]  */
  double gA2[3], gB2[3];
  for (int i = 0; i < 3; i++) { gA2[i] = 2.0 * absA * gabsA[i]; gB2[i] = 2.0 * B * gB[i]; }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double t1 = (gabsA[i] * gB[j] - gB[i] * gabsA[j]) / D;
      double t2 = (B * 0.0 - absA * JB[3 * i + j]) / D;
      double t3 = (B * gabsA[i] - absA * gB[i]) * (gA2[j] + gB2[j]) / (D * D);
      HF[3 * i + j] = (t1 + t2 - t3) / (2.0 * RCO_PI);
    }
}

/* ------------------------------------------------------------------ */
/* record computation                                                   */
/* ------------------------------------------------------------------ */
typedef struct {
  float sigma_s, sigma_a;
  const float* lights; int L;
  float ring_step; int max_rings;
  uint64_t seed;
} rco_params;

typedef struct {
  int nth, nph, nv;          /* nv = N + 2 (two poles) */
  f3* w32;                   /* direction (FP32, as sampled) */
  float* t32;                /* FP32 hit / exit distance (decision value) */
  double* t64;               /* FP64 distance recomputed from the decision */
  int64_t* hit;              /* triangle index or -1 */
  int* front;
  double* Ls;                /* surface vertex radiance */
  int* M;                    /* rings in front of the hit */
  double* Lm;                /* [nv][max_rings] ring vertex radiance */
  float* r32; double* r64;   /* ring distances */
  int64_t shadow_rays;
} rco_verts;

static void verts_free(rco_verts* v) {
  free(v->w32); free(v->t32); free(v->t64); free(v->hit); free(v->front); free(v->Ls); free(v->M);
  free(v->Lm); free(v->r32); free(v->r64);
}

/* vertex id: 0 north pole, 1 + a*nph + b stratum (a,b), N+1 south pole */
static int vid(const rco_verts* v, int a, int b) { return 1 + a * v->nph + ((b % v->nph + v->nph) % v->nph); }

/* Direction of stratum (a, b): equal-solid-angle strata in (z, phi),
 * jittered (Sec. 6, Implementation).  The sample is computed in FP64 and
 * rounded to FP32; the FP32 vector is the sample direction used everywhere. */
static f3 stratum_dir(uint64_t key, int a, int b, int nth, int nph) {
  uint64_t idx = (uint64_t)a * (uint64_t)nph + (uint64_t)b;
  double xi0 = unif(key, idx, 0), xi1 = unif(key, idx, 1);
  double u = ((double)a + xi0) / (double)nth;
  double v = ((double)b + xi1) / (double)nph;
  double z = 1.0 - 2.0 * u;
  double phi = (2.0 * RCO_PI) * v;
  double zz = z * z;
  double st = sqrt(fmax(0.0, 1.0 - zz));
  f3 w = {(float)(st * cos(phi)), (float)(st * sin(phi)), (float)z};
  return w;
}

/* surface radiance at the hit of direction k (Lambertian, two-sided: the side
 * facing x is lit; point lights with shadow rays; plus emission). */
static double shade_surface(const rco_scene* s, const rco_params* p, f3 x32, const double* x64, f3 w,
                            float t32, double t64, int64_t j, int front, int64_t* nrays) {
  double L = s->emission[j];
  double mu = (double)p->sigma_s + (double)p->sigma_a;
  double y64[3] = {x64[0] + t64 * w.x, x64[1] + t64 * w.y, x64[2] + t64 * w.z};
  f3 y32 = {x32.x + t32 * w.x, x32.y + t32 * w.y, x32.z + t32 * w.z};
  double nf[3];
  for (int k = 0; k < 3; k++) nf[k] = front ? s->n64[3 * j + k] : -s->n64[3 * j + k];
  for (int l = 0; l < p->L; l++) {
    const float* lp = p->lights + 4 * l;
    (*nrays)++;
    double dl[3] = {lp[0] - y64[0], lp[1] - y64[1], lp[2] - y64[2]};
    double dist = d3_norm(dl);
    double c = d3_dot(nf, dl) / dist;
    if (!(c > 0.0)) continue;
    f3 seg = {lp[0] - y32.x, lp[1] - y32.y, lp[2] - y32.z};
    if (occluded(s, y32, seg, j)) continue;
    L += ((double)s->albedo[j] / RCO_PI) * (double)lp[3] * c * exp(-mu * dist) / (dist * dist);
  }
  return L;
}

/* medium vertex radiance: sigma_s f_s sum_l I_l exp(-mu d_l) V_l / d_l^2 */
static double shade_medium(const rco_scene* s, const rco_params* p, f3 x32, const double* x64, f3 w,
                           float r32, double r64, int64_t* nrays) {
  double mu = (double)p->sigma_s + (double)p->sigma_a;
  double y64[3] = {x64[0] + r64 * w.x, x64[1] + r64 * w.y, x64[2] + r64 * w.z};
  f3 y32 = {x32.x + r32 * w.x, x32.y + r32 * w.y, x32.z + r32 * w.z};
  double L = 0.0;
  for (int l = 0; l < p->L; l++) {
    const float* lp = p->lights + 4 * l;
    (*nrays)++;
    f3 seg = {lp[0] - y32.x, lp[1] - y32.y, lp[2] - y32.z};
    if (occluded(s, y32, seg, -1)) continue;
    double dl[3] = {lp[0] - y64[0], lp[1] - y64[1], lp[2] - y64[2]};
    double dist = d3_norm(dl);
    L += (double)lp[3] * exp(-mu * dist) / (dist * dist);
  }
  return (double)p->sigma_s / (4.0 * RCO_PI) * L;
}

static int build_verts(const rco_scene* s, const rco_params* p, const float* xin, int nth, int nph,
                       uint64_t rec, rco_verts* v) {
  memset(v, 0, sizeof(*v));
  v->nth = nth; v->nph = nph; v->nv = nth * nph + 2;
  int nv = v->nv, R = p->max_rings;
  v->w32 = (f3*)malloc(sizeof(f3) * nv); v->t32 = (float*)malloc(sizeof(float) * nv);
  v->t64 = (double*)malloc(sizeof(double) * nv); v->hit = (int64_t*)malloc(sizeof(int64_t) * nv);
  v->front = (int*)malloc(sizeof(int) * nv); v->Ls = (double*)malloc(sizeof(double) * nv);
  v->M = (int*)malloc(sizeof(int) * nv); v->Lm = (double*)calloc((size_t)nv * (R > 0 ? R : 1), sizeof(double));
  v->r32 = (float*)malloc(sizeof(float) * (R > 0 ? R : 1)); v->r64 = (double*)malloc(sizeof(double) * (R > 0 ? R : 1));
  if (!v->w32 || !v->t32 || !v->t64 || !v->hit || !v->front || !v->Ls || !v->M || !v->Lm || !v->r32 || !v->r64) {
    verts_free(v); return RCO_ENOMEM;
  }
  uint64_t key = rec_key(p->seed, rec);
  float xr = unif(key, RCO_RING_IDX, 0);
  for (int i = 0; i < R; i++) {
    v->r32[i] = ((float)i + xr) * p->ring_step;
    v->r64[i] = ((double)i + (double)xr) * (double)p->ring_step;
  }
  f3 x32 = {xin[0], xin[1], xin[2]};
  double x64[3] = {xin[0], xin[1], xin[2]};
  /* directions */
  f3 np = {0.0f, 0.0f, 1.0f}, sp = {0.0f, 0.0f, -1.0f};
  v->w32[0] = np; v->w32[nv - 1] = sp;
  for (int a = 0; a < nth; a++)
    for (int b = 0; b < nph; b++) v->w32[vid(v, a, b)] = stratum_dir(key, a, b, nth, nph);
  /* trace, shade */
  for (int k = 0; k < nv; k++) {
    f3 w = v->w32[k];
    double w64[3] = {w.x, w.y, w.z};
    hit32 h = trace_closest(s, x32, w);
    v->hit[k] = h.hit ? h.id : -1;
    v->front[k] = h.front;
    if (h.hit) {
      v->t32[k] = h.t;
      /* exact ray-plane distance in FP64 for the decided triangle */
      const double* n = s->n64 + 3 * h.id;
      const double* a0 = s->v064 + 3 * h.id;
      double num = (a0[0] - x64[0]) * n[0] + (a0[1] - x64[1]) * n[1] + (a0[2] - x64[2]) * n[2];
      v->t64[k] = num / d3_dot(w64, n);
    } else {
      v->t32[k] = box_exit32(s, x32, w);
      v->t64[k] = box_exit64(s, x64, w64);
    }
    v->Ls[k] = h.hit ? shade_surface(s, p, x32, x64, w, v->t32[k], v->t64[k], h.id, h.front, &v->shadow_rays) : 0.0;
    int M = 0;
    while (M < R && v->r32[M] < v->t32[k]) M++;
    v->M[k] = M;
    for (int i = 0; i < M; i++)
      v->Lm[(size_t)k * R + i] = shade_medium(s, p, x32, x64, w, v->r32[i], v->r64[i], &v->shadow_rays);
  }
  return RCO_OK;
}

/* Triangles of the angular subdivision: polar fans plus two triangles per
 * quad between adjacent strata rows (Sec. 4: adjacent strata are joined).
 * The quad diagonal (a,b)-(a+1,b+1) is used unless one of its triangles is
 * not positively oriented on the FP32 directions; then (a,b+1)-(a+1,b). */
static float det32(f3 a, f3 b, f3 c) { return f3_dot(a, f3_cross(b, c)); }
typedef struct { int v[3]; } tri3;
static int build_tris(const rco_verts* v, tri3* out) {
  int n = 0, nth = v->nth, nph = v->nph, S = v->nv - 1;
  for (int b = 0; b < nph; b++) { out[n].v[0] = 0; out[n].v[1] = vid(v, 0, b); out[n].v[2] = vid(v, 0, b + 1); n++; }
  for (int a = 0; a + 1 < nth; a++)
    for (int b = 0; b < nph; b++) {
      int P = vid(v, a, b), Q = vid(v, a, b + 1), R = vid(v, a + 1, b), Sq = vid(v, a + 1, b + 1);
      if (det32(v->w32[P], v->w32[R], v->w32[Sq]) > 0.0f && det32(v->w32[P], v->w32[Sq], v->w32[Q]) > 0.0f) {
        out[n].v[0] = P; out[n].v[1] = R; out[n].v[2] = Sq; n++;
        out[n].v[0] = P; out[n].v[1] = Sq; out[n].v[2] = Q; n++;
      } else {
        out[n].v[0] = P; out[n].v[1] = R; out[n].v[2] = Q; n++;
        out[n].v[0] = Q; out[n].v[1] = R; out[n].v[2] = Sq; n++;
      }
    }
  for (int b = 0; b < nph; b++) { out[n].v[0] = S; out[n].v[1] = vid(v, nth - 1, b + 1); out[n].v[2] = vid(v, nth - 1, b); n++; }
  return n;
}

/* Accumulate one triangle's Eq. SSSegALGradientSimp / SSSegALHessianSimp
 * term, with r_i = y_i - x_eval and y_far its furthest vertex. */
typedef struct { double G[3], H[9], V, SG, SH; int64_t n; } acc_t;
static void add_term(acc_t* acc, const double* y1, const double* y2, const double* y3, const double* yfar,
                     const double* xe, double wL, double mu) {
  double r1[3], r2[3], r3[3];
  for (int i = 0; i < 3; i++) { r1[i] = y1[i] - xe[i]; r2[i] = y2[i] - xe[i]; r3[i] = y3[i] - xe[i]; }
  double F, gF[3], HF[9], T, gT[3], HT[9];
  rco_formfactor(r1, r2, r3, &F, gF, HF);
  rco_transmittance(xe, yfar, mu, &T, gT, HT);
  double g[3], h[9], ng = 0.0, nh = 0.0;
  for (int i = 0; i < 3; i++) { g[i] = wL * (T * gF[i] + F * gT[i]); ng += g[i] * g[i]; }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      h[3 * i + j] = wL * (T * HF[3 * i + j] + gT[i] * gF[j] + gF[i] * gT[j] + F * HT[3 * i + j]);
      nh += h[3 * i + j] * h[3 * i + j];
    }
  for (int i = 0; i < 3; i++) acc->G[i] += g[i];
  for (int i = 0; i < 9; i++) acc->H[i] += h[i];
  acc->V += wL * T * F;
  acc->SG += sqrt(ng);
  acc->SH += sqrt(nh);
  acc->n++;
}

/* Monte Carlo value (Eq. outLF): mean over the N strata (poles excluded) of
 * the surface radiance attenuated to x (SS) and of the ring radiances in
 * front of the hit, attenuated to x and weighted by 1/pdf = ring_step (MS) */
static void mc_value(const rco_verts* v, const rco_params* p, double* val) {
  const int N = v->nth * v->nph, R = p->max_rings;
  const double mu = (double)p->sigma_s + (double)p->sigma_a;
  double VS = 0.0, VM = 0.0;
  for (int k = 1; k <= N; k++) {
    f3 w = v->w32[k];
    double wn = sqrt((double)w.x * w.x + (double)w.y * w.y + (double)w.z * w.z);
    VS += exp(-mu * v->t64[k] * wn) * v->Ls[k];
    for (int i = 0; i < v->M[k]; i++) VM += (double)p->ring_step * exp(-mu * v->r64[i] * wn) * v->Lm[(size_t)k * R + i];
  }
  val[0] = VS / N; val[1] = VM / N;
}

/* far vertex: the largest FP32 decision distance, ties to the lowest id */
static int far_vertex(const int* ids, const float* dist) {
  int best = 0;
  for (int k = 1; k < 3; k++)
    if (dist[k] > dist[best] || (dist[k] == dist[best] && ids[k] < ids[best])) best = k;
  return best;
}

/* stats layout (per record) */
#define RCO_NSTAT 12
/* 0 rays traced (primary + shadow), 1 terms SS, 2 terms MS, 3 S_G SS, 4 S_H SS, 5 S_G MS, 6 S_H MS,
 * 7 triangulated value SS, 8 triangulated value MS, 9 max relative Hessian asymmetry,
 * 10 largest ring count, 11 number of triangles */

static int one_record(const rco_scene* s, const rco_params* p, const float* x, int nth, int nph, uint64_t rec,
                      const double* xeval, double* val, double* grad, double* hess, double* stats) {
  rco_verts v;
  int rc = build_verts(s, p, x, nth, nph, rec, &v);
  if (rc) return rc;
  int N = nth * nph, R = p->max_rings;
  double mu = (double)p->sigma_s + (double)p->sigma_a;
  double x64[3] = {x[0], x[1], x[2]};
  const double* xe = xeval ? xeval : x64;
  mc_value(&v, p, val);
  /* triangulated derivatives */
  tri3* tris = (tri3*)malloc(sizeof(tri3) * 2 * N);
  if (!tris) { verts_free(&v); return RCO_ENOMEM; }
  int ntri = build_tris(&v, tris);
  acc_t acc[2];
  memset(acc, 0, sizeof(acc));
  int maxM = 0;
  for (int k = 0; k < v.nv; k++) if (v.M[k] > maxM) maxM = v.M[k];
  for (int t = 0; t < ntri; t++) {
    const int* id = tris[t].v;
    double y[3][3];
    float dd[3];
    /* surface ring: every vertex at its hit (or box exit) */
    for (int q = 0; q < 3; q++) {
      f3 w = v.w32[id[q]];
      double tt = v.t64[id[q]];
      y[q][0] = x64[0] + tt * w.x; y[q][1] = x64[1] + tt * w.y; y[q][2] = x64[2] + tt * w.z;
      dd[q] = v.t32[id[q]];
    }
    int f = far_vertex(id, dd);
    double L = v.Ls[id[f]];
    if (L != 0.0) add_term(&acc[0], y[0], y[1], y[2], y[f], xe, L, mu);
    /* medium rings: vertex at r_i if the ring is in front of the hit, else at the hit with zero radiance */
    int mmax = v.M[id[0]];
    if (v.M[id[1]] > mmax) mmax = v.M[id[1]];
    if (v.M[id[2]] > mmax) mmax = v.M[id[2]];
    for (int i = 0; i < mmax; i++) {
      double Lq[3];
      for (int q = 0; q < 3; q++) {
        f3 w = v.w32[id[q]];
        int in_front = i < v.M[id[q]];
        double tt = in_front ? v.r64[i] : v.t64[id[q]];
        y[q][0] = x64[0] + tt * w.x; y[q][1] = x64[1] + tt * w.y; y[q][2] = x64[2] + tt * w.z;
        dd[q] = in_front ? v.r32[i] : v.t32[id[q]];
        Lq[q] = in_front ? v.Lm[(size_t)id[q] * R + i] : 0.0;
      }
      f = far_vertex(id, dd);
      if (Lq[f] != 0.0) add_term(&acc[1], y[0], y[1], y[2], y[f], xe, (double)p->ring_step * Lq[f], mu);
    }
  }
  double asym = 0.0;
  for (int c = 0; c < 2; c++) {
    double fro = 0.0, dif = 0.0;
    for (int i = 0; i < 9; i++) fro += acc[c].H[i] * acc[c].H[i];
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) { double d = acc[c].H[3 * i + j] - acc[c].H[3 * j + i]; dif += d * d; }
    if (fro > 0) asym = fmax(asym, sqrt(dif / fro));
    for (int i = 0; i < 3; i++) grad[3 * c + i] = acc[c].G[i];
    const double* H = acc[c].H;
    hess[6 * c + 0] = H[0];
    hess[6 * c + 1] = 0.5 * (H[1] + H[3]);
    hess[6 * c + 2] = 0.5 * (H[2] + H[6]);
    hess[6 * c + 3] = H[4];
    hess[6 * c + 4] = 0.5 * (H[5] + H[7]);
    hess[6 * c + 5] = H[8];
  }
  if (stats) {
    stats[0] = (double)(v.nv + v.shadow_rays);
    stats[1] = (double)acc[0].n; stats[2] = (double)acc[1].n;
    stats[3] = acc[0].SG; stats[4] = acc[0].SH; stats[5] = acc[1].SG; stats[6] = acc[1].SH;
    stats[7] = acc[0].V; stats[8] = acc[1].V;
    stats[9] = asym; stats[10] = (double)maxM; stats[11] = (double)ntri;
  }
  free(tris);
  verts_free(&v);
  return RCO_OK;
}

int rco_nstat(void) { return RCO_NSTAT; }

/* Records for P cache points.
 *   value [P][2] (SS, MS), grad [P][2][3], hess [P][2][6] (xx, xy, xz, yy, yz, zz),
 *   stats [P][RCO_NSTAT] or NULL.
 *   rec_id [P]: the record index that keys the random numbers.
 *   xeval [P][3] or NULL: evaluate the triangulated derivatives at xeval with
 *   the vertices frozen at pos (finite-difference checks); the value output
 *   stays the Monte Carlo value at pos.
 *   nthreads <= 0: OpenMP default. */
int rco_records(const rco_scene* s, float sigma_s, float sigma_a, const float* lights, int L,
                const float* pos, const int32_t* n_theta, const int32_t* n_phi, const uint64_t* rec_id, int64_t P,
                float ring_step, int max_rings, uint64_t seed, const double* xeval,
                double* value, double* grad, double* hess, double* stats, int nthreads) {
  if (!s || P < 0 || (P > 0 && (!pos || !n_theta || !n_phi || !rec_id || !value || !grad || !hess))) return RCO_EINVAL;
  if (L < 0 || (L > 0 && !lights) || !(ring_step > 0.0f) || max_rings < 0 || sigma_s < 0 || sigma_a < 0) return RCO_EINVAL;
  for (int64_t i = 0; i < P; i++)
    if (n_theta[i] < 2 || n_phi[i] < 5) return RCO_EINVAL;
  rco_params p = {sigma_s, sigma_a, lights, L, ring_step, max_rings, seed};
  int err = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
  for (int64_t i = 0; i < P; i++) {
    int rc = one_record(s, &p, pos + 3 * i, n_theta[i], n_phi[i], rec_id[i], xeval ? xeval + 3 * i : NULL,
                        value + 2 * i, grad + 6 * i, hess + 12 * i, stats ? stats + RCO_NSTAT * i : NULL);
    if (rc) err |= 1;
  }
  return err ? RCO_ENOMEM : RCO_OK;
}

/* The Monte Carlo values of records only (the value part of rco_records,
 * without the triangulation): brute-force references at large N. */
int rco_values(const rco_scene* s, float sigma_s, float sigma_a, const float* lights, int L,
               const float* pos, const int32_t* n_theta, const int32_t* n_phi, const uint64_t* rec_id, int64_t P,
               float ring_step, int max_rings, uint64_t seed, double* value, int nthreads) {
  if (!s || P < 0 || (P > 0 && (!pos || !n_theta || !n_phi || !rec_id || !value))) return RCO_EINVAL;
  if (L < 0 || (L > 0 && !lights) || !(ring_step > 0.0f) || max_rings < 0 || sigma_s < 0 || sigma_a < 0) return RCO_EINVAL;
  for (int64_t i = 0; i < P; i++)
    if (n_theta[i] < 2 || n_phi[i] < 5) return RCO_EINVAL;
  rco_params p = {sigma_s, sigma_a, lights, L, ring_step, max_rings, seed};
  int err = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
  for (int64_t i = 0; i < P; i++) {
    rco_verts v;
    if (build_verts(s, &p, pos + 3 * i, n_theta[i], n_phi[i], rec_id[i], &v)) { err |= 1; continue; }
    mc_value(&v, &p, value + 2 * i);
    verts_free(&v);
  }
  return err ? RCO_ENOMEM : RCO_OK;
}

/* Occlusion-unaware per-sample gradients of the comparison method (the
 * gradients of Jarosz et al. 2008 summarised in Sec. 3 and supplement
 * Eqs. S.3-S.4), from the same samples as the record's Monte Carlo value.
 * Single scattering: each direction's sample keeps its hit point y fixed as x
 * moves; in surface-area form the sample is L_s T G / pdf_A, so its gradient
 * is the sample times grad ln T + grad ln G, with T = exp(-mu r),
 * G = (yx . n) / r^3, yx = x - y, r = |yx|: grad ln T = -mu yx / r and
 * grad ln G = n / (yx . n) - 3 yx / r^2.  Multiple scattering: the path
 * x -> ring vertex m -> light moves rigidly with x, so only the light
 * connection I exp(-mu d) / d^2 (d = |l - m|, visibility held) changes:
 * gradient = contribution * (-mu - 2 / d) (m - l) / d.  Per direction k the
 * sample is L_k = SS_k + MS_k with gradient g_k; outputs: grad [2][3]
 * (SS, MS; means over the N directions like the value), and the means of
 * L_k and of |g_k| (the radius of Eq. jaroszRadius is
 * eps * sum L_k / sum |g_k|). */
static void j08_grad(const rco_scene* s, const rco_params* p, const float* xin, const rco_verts* v, double* grad,
                     double* lmean, double* gmean) {
  const int N = v->nth * v->nph;
  const double mu = (double)p->sigma_s + (double)p->sigma_a;
  const double x64[3] = {xin[0], xin[1], xin[2]};
  const f3 x32 = {xin[0], xin[1], xin[2]};
  double gs[3] = {0, 0, 0}, gm[3] = {0, 0, 0}, lsum = 0.0, nsum = 0.0;
  for (int k = 1; k <= N; k++) {
    const f3 w = v->w32[k];
    const double wn = sqrt((double)w.x * w.x + (double)w.y * w.y + (double)w.z * w.z);
    double gk[3] = {0, 0, 0}, Lk = 0.0;
    if (v->hit[k] >= 0) {
      const double r = v->t64[k] * wn;
      const double S = exp(-mu * r) * v->Ls[k];
      const double* n = s->n64 + 3 * v->hit[k];
      const double yx[3] = {-v->t64[k] * w.x, -v->t64[k] * w.y, -v->t64[k] * w.z};
      const double yn = d3_dot(yx, n);
      for (int i = 0; i < 3; i++) gk[i] = S * (-mu * yx[i] / r + n[i] / yn - 3.0 * yx[i] / (r * r));
      Lk += S;
      for (int i = 0; i < 3; i++) gs[i] += gk[i];
    }
    for (int i = 0; i < v->M[k]; i++) {
      const double y64[3] = {x64[0] + v->r64[i] * w.x, x64[1] + v->r64[i] * w.y, x64[2] + v->r64[i] * w.z};
      const f3 y32 = {x32.x + v->r32[i] * w.x, x32.y + v->r32[i] * w.y, x32.z + v->r32[i] * w.z};
      const double att = (double)p->ring_step * exp(-mu * v->r64[i] * wn) * (double)p->sigma_s / (4.0 * RCO_PI);
      for (int l = 0; l < p->L; l++) {
        const float* lp = p->lights + 4 * l;
        const f3 seg = {lp[0] - y32.x, lp[1] - y32.y, lp[2] - y32.z};
        if (occluded(s, y32, seg, -1)) continue;
        const double ml[3] = {y64[0] - lp[0], y64[1] - lp[1], y64[2] - lp[2]};
        const double d = d3_norm(ml);
        const double c = att * (double)lp[3] * exp(-mu * d) / (d * d);
        Lk += c;
        for (int q = 0; q < 3; q++) {
          const double g = c * (-mu - 2.0 / d) * ml[q] / d;
          gk[q] += g;
          gm[q] += g;
        }
      }
    }
    lsum += Lk;
    nsum += d3_norm(gk);
  }
  for (int i = 0; i < 3; i++) {
    grad[i] = gs[i] / N;
    grad[3 + i] = gm[i] / N;
  }
  *lmean = lsum / N;
  *gmean = nsum / N;
}

/* Values, occlusion-unaware gradients [P][2][3] and the means of the
 * per-direction samples and of their gradient norms [P][2] for P points. */
int rco_j08(const rco_scene* s, float sigma_s, float sigma_a, const float* lights, int L, const float* pos,
            const int32_t* n_theta, const int32_t* n_phi, const uint64_t* rec_id, int64_t P, float ring_step,
            int max_rings, uint64_t seed, double* value, double* grad, double* moments, int nthreads) {
  if (!s || P < 0 || (P > 0 && (!pos || !n_theta || !n_phi || !rec_id || !value || !grad || !moments)))
    return RCO_EINVAL;
  if (L < 0 || (L > 0 && !lights) || !(ring_step > 0.0f) || max_rings < 0 || sigma_s < 0 || sigma_a < 0) return RCO_EINVAL;
  for (int64_t i = 0; i < P; i++)
    if (n_theta[i] < 2 || n_phi[i] < 5) return RCO_EINVAL;
  rco_params p = {sigma_s, sigma_a, lights, L, ring_step, max_rings, seed};
  int err = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
  for (int64_t i = 0; i < P; i++) {
    rco_verts v;
    if (build_verts(s, &p, pos + 3 * i, n_theta[i], n_phi[i], rec_id[i], &v)) { err |= 1; continue; }
    mc_value(&v, &p, value + 2 * i);
    j08_grad(s, &p, pos + 3 * i, &v, grad + 6 * i, moments + 2 * i, moments + 2 * i + 1);
    verts_free(&v);
  }
  return err ? RCO_ENOMEM : RCO_OK;
}

/* The per-record sample directions (FP32), exported for tests of the
 * sampling layout (strata, equal solid angle, poles). [N+2][3] */
int rco_directions(uint64_t seed, uint64_t rec, int nth, int nph, float* out) {
  if (nth < 1 || nph < 1 || !out) return RCO_EINVAL;
  uint64_t key = rec_key(seed, rec);
  int N = nth * nph;
  out[0] = 0.0f; out[1] = 0.0f; out[2] = 1.0f;
  for (int a = 0; a < nth; a++)
    for (int b = 0; b < nph; b++) {
      f3 w = stratum_dir(key, a, b, nth, nph);
      int k = 1 + a * nph + b;
      out[3 * k] = w.x; out[3 * k + 1] = w.y; out[3 * k + 2] = w.z;
    }
  out[3 * (N + 1)] = 0.0f; out[3 * (N + 1) + 1] = 0.0f; out[3 * (N + 1) + 2] = -1.0f;
  return RCO_OK;
}

/* The triangle list of the angular subdivision for given directions. [2N][3] */
int rco_triangles(const float* dirs, int nth, int nph, int32_t* out) {
  if (!dirs || !out || nth < 1 || nph < 3) return RCO_EINVAL;
  rco_verts v;
  memset(&v, 0, sizeof(v));
  v.nth = nth; v.nph = nph; v.nv = nth * nph + 2;
  v.w32 = (f3*)malloc(sizeof(f3) * v.nv);
  tri3* t = (tri3*)malloc(sizeof(tri3) * 2 * nth * nph);
  if (!v.w32 || !t) { free(v.w32); free(t); return RCO_ENOMEM; }
  for (int k = 0; k < v.nv; k++) { v.w32[k].x = dirs[3 * k]; v.w32[k].y = dirs[3 * k + 1]; v.w32[k].z = dirs[3 * k + 2]; }
  int n = build_tris(&v, t);
  for (int i = 0; i < n; i++) for (int q = 0; q < 3; q++) out[3 * i + q] = t[i].v[q];
  free(v.w32); free(t);
  return n;
}

/* uniform float of the counter-based generator (for tests of the generator) */
float rco_unif(uint64_t seed, uint64_t rec, uint64_t idx, uint64_t dim) { return unif(rec_key(seed, rec), idx, dim); }
uint64_t rco_splitmix64(uint64_t x) { return sm64(x); }

/* ------------------------------------------------------------------ */
/* Probe features for learned placement (project-defined, not in the   */
/* paper).  A 4 x 16 jittered strata grid from the same sampler; per     */
/* direction: distance to the first hit (or box exit), Lambertian        */
/* radiance of the hit with shadow rays, attenuated to x; plus the        */
/* visibility of lights 0..3 from x.  32 features, each defined below.    */
/* ------------------------------------------------------------------ */
int rco_probe(const rco_scene* s, float sigma_s, float sigma_a, const float* lights, int L, const float* cand,
              int64_t C, uint64_t seed, const uint64_t* ids, double* feat) {
  if (!s || C < 0 || (C > 0 && (!cand || !ids || !feat)) || L < 0 || (L > 0 && !lights)) return RCO_EINVAL;
  rco_params p = {sigma_s, sigma_a, lights, L, 0.1f, 0, seed};
  const double mu = (double)sigma_s + (double)sigma_a;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t c = 0; c < C; c++) {
    const float* xin = cand + 3 * c;
    f3 x32 = {xin[0], xin[1], xin[2]};
    double x64[3] = {xin[0], xin[1], xin[2]};
    uint64_t key = rec_key(seed, ids[c]);
    double dist[64], Lt[64], wv[64][3];
    int hitk[64];
    int64_t dummy = 0;
    for (int k = 0; k < 64; k++) {
      int a = k / 16, b = k % 16;
      f3 w = stratum_dir(key, a, b, 4, 16);
      double w64[3] = {w.x, w.y, w.z};
      hit32 h = trace_closest(s, x32, w);
      double t64;
      float t32;
      if (h.hit) {
        const double* n = s->n64 + 3 * h.id;
        const double* a0 = s->v064 + 3 * h.id;
        double num = (a0[0] - x64[0]) * n[0] + (a0[1] - x64[1]) * n[1] + (a0[2] - x64[2]) * n[2];
        t64 = num / d3_dot(w64, n);
        t32 = h.t;
      } else {
        t32 = box_exit32(s, x32, w);
        t64 = box_exit64(s, x64, w64);
      }
      double Ls = h.hit ? shade_surface(s, &p, x32, x64, w, t32, t64, h.id, h.front, &dummy) : 0.0;
      double wn = sqrt(d3_dot(w64, w64));
      double dd = t64 * wn;
      if (dd < 1e-6) dd = 1e-6;
      dist[k] = dd;
      Lt[k] = exp(-mu * dd) * Ls;
      hitk[k] = h.hit;
      for (int q = 0; q < 3; q++) wv[k][q] = w64[q];
    }
    double* f = feat + 32 * c;
    double mn = 1e300, mx = -1e300, sl = 0, sinv = 0, sL = 0, maxL = -1e300, esc = 0;
    for (int k = 0; k < 64; k++) {
      double ld = log(dist[k]);
      mn = fmin(mn, ld);
      mx = fmax(mx, ld);
      sl += ld;
      sinv += 1.0 / dist[k];
      sL += Lt[k];
      maxL = fmax(maxL, Lt[k]);
      esc += hitk[k] ? 0.0 : 1.0;
    }
    double ml = sl / 64, mL = sL / 64, vl = 0, vL = 0;
    for (int k = 0; k < 64; k++) {
      vl += (log(dist[k]) - ml) * (log(dist[k]) - ml);
      vL += (Lt[k] - mL) * (Lt[k] - mL);
    }
    f[0] = mn;                                   /* min log distance */
    f[1] = ml;                                   /* mean log distance */
    f[2] = sqrt(vl / 64);                        /* std of log distance */
    f[3] = mx;                                   /* max log distance */
    f[4] = esc / 64;                             /* escaped fraction */
    f[5] = log(sinv / 64);                       /* log mean inverse distance */
    f[6] = log(mL + 1e-6);                       /* log mean radiance */
    f[7] = sqrt(vL / 64) / (mL + 1e-6);          /* coefficient of variation */
    f[8] = log(maxL + 1e-6);                     /* log max radiance */
    for (int l = 0; l < 4; l++) {                /* lights seen from x, unshadowed irradiance */
      if (l < L) {
        const float* lp = lights + 4 * l;
        f3 seg = {lp[0] - x32.x, lp[1] - x32.y, lp[2] - x32.z};
        f[9 + l] = occluded(s, x32, seg, -1) ? 0.0 : 1.0;
        double d[3] = {(double)lp[0] - x64[0], (double)lp[1] - x64[1], (double)lp[2] - x64[2]};
        double d2 = d3_dot(d, d);
        f[13 + l] = log((double)lp[3] * exp(-mu * sqrt(d2)) / d2 + 1e-6);
      } else {
        f[9 + l] = 0.0;
        f[13 + l] = 0.0;
      }
    }
    double sLt = sL + 1e-12;
    for (int q = 0; q < 3; q++) {
      double aL = 0, aI = 0;
      for (int k = 0; k < 64; k++) {
        aL += Lt[k] * wv[k][q];
        aI += wv[k][q] / dist[k];
      }
      f[17 + q] = aL / sLt;                      /* radiance-weighted mean direction */
      f[20 + q] = aI / sinv;                     /* inverse-distance-weighted mean direction */
    }
    for (int r = 0; r < 4; r++) {                /* per strata row: mean log distance, mean log radiance */
      double a1 = 0, a2 = 0;
      for (int b = 0; b < 16; b++) {
        a1 += log(dist[16 * r + b]);
        a2 += log(Lt[16 * r + b] + 1e-6);
      }
      f[23 + r] = a1 / 16;
      f[27 + r] = a2 / 16;
    }
    double con = 0;                              /* contrast with the next column of the same row */
    for (int k = 0; k < 64; k++) con += fabs(Lt[k] - Lt[16 * (k / 16) + (k % 16 + 1) % 16]);
    f[31] = con / sLt;
  }
  return RCO_OK;
}
