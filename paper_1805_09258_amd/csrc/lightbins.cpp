// lightbins.cpp -- host builder of the per-light triangle bins that answer
// the record kernel's shadow segments.
//
// Every shadow segment of a record ends at one of the point lights (Sec. 6:
// point lights handled by shadow rays).  Seen from a light L, a triangle
// covers a region of directions; a segment y -> L can only be blocked by a
// triangle whose region contains the direction of y - L and whose distance
// from L is below |y - L|.  The directions around L are split into the six
// faces of a cube, each face into B x B bins in the tangent coordinates
// (u, v) = (e_kx, e_ky) / |e_kz| of a direction e (kz the axis of its largest
// component, (kx, ky) = (kz + 1, kz + 2) mod 3, face 2 kz for e_kz > 0 and
// 2 kz + 1 otherwise).  Coarser levels of B / 4^k bins (nested) take the
// triangles whose region covers more than 32 x 32 bins of a finer level, so a
// wall or a slab lands in a few coarse bins instead of thousands of fine
// ones.  Each bin lists its triangles by increasing distance from L.
//
// The lists are conservative for the watertight ray/triangle test: a hit it
// accepts lies within eps = 64 * 2^-24 * scale of the triangle (the FP32
// projection along the ray and the FP32 rounding of t are its only inexact
// steps), so the direction from L to the hit point is within
// a = eps / (dmin - eps) of the triangle's region (dmin: the triangle's
// distance from L).  Each region is clipped to each face's pyramid widened by
// 3a + 1e-5 in (u, v) (tangent coordinates stretch angles by at most 3 on a
// face), its (u, v) box padded by the same amount, and each entry's distance
// is a lower bound on the distance from L of the triangle's points seen
// through the padded bin, minus eps, rounded down; the 1e-5 covers the FP32
// rounding of the bin coordinates of a query.  Triangles that pass within 2 eps of L, or
// whose clipped region reaches the apex, cover every bin of the face.
// A segment's answer from the bins is therefore the answer of testing every
// triangle.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.hpp"

namespace rc {
namespace {

struct V {
  double x, y, z;
};
V sub(V a, V b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
V add(V a, V b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
V mul(double s, V a) { return {s * a.x, s * a.y, s * a.z}; }
double dot(V a, V b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
double norm(V a) { return std::sqrt(dot(a, a)); }

// distance from p to the triangle (a, b, c): closest point by Voronoi regions
// of the vertices, edges and face
double point_triangle_distance(V p, V a, V b, V c) {
  const V ab = sub(b, a), ac = sub(c, a), ap = sub(p, a);
  const double d1 = dot(ab, ap), d2 = dot(ac, ap);
  if (d1 <= 0 && d2 <= 0) return norm(ap);
  const V bp = sub(p, b);
  const double d3 = dot(ab, bp), d4 = dot(ac, bp);
  if (d3 >= 0 && d4 <= d3) return norm(bp);
  const double vc = d1 * d4 - d3 * d2;
  if (vc <= 0 && d1 >= 0 && d3 <= 0) return norm(sub(p, add(a, mul(d1 / (d1 - d3), ab))));
  const V cp = sub(p, c);
  const double d5 = dot(ab, cp), d6 = dot(ac, cp);
  if (d6 >= 0 && d5 <= d6) return norm(cp);
  const double vb = d5 * d2 - d1 * d6;
  if (vb <= 0 && d2 >= 0 && d6 <= 0) return norm(sub(p, add(a, mul(d2 / (d2 - d6), ac))));
  const double va = d3 * d6 - d5 * d4;
  if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0) {
    const double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    return norm(sub(p, add(b, mul(w, sub(c, b)))));
  }
  const double den = 1.0 / (va + vb + vc);
  const double v = vb * den, w = vc * den;
  // the face: distance to the plane (more accurate than the reconstructed point)
  V n = {ab.y * ac.z - ab.z * ac.y, ab.z * ac.x - ab.x * ac.z, ab.x * ac.y - ab.y * ac.x};
  const double nn = norm(n);
  if (nn > 0) return std::fabs(dot(ap, n)) / nn;
  return norm(sub(p, add(a, add(mul(v, ab), mul(w, ac)))));
}

double comp(V a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

// polygon clipping against the half-space f(p) >= 0 (Sutherland-Hodgman)
template <class F>
int clip(const V* in, int n, V* out, F f) {
  int m = 0;
  for (int i = 0; i < n; i++) {
    const V p = in[i], q = in[(i + 1) % n];
    const double fp = f(p), fq = f(q);
    if (fp >= 0) out[m++] = p;
    if ((fp >= 0) != (fq >= 0)) {
      const double t = fp / (fp - fq);
      out[m++] = add(p, mul(t, sub(q, p)));
    }
  }
  return m;
}

struct Span {
  int face, level, iu0, iu1, iv0, iv1;
};

}  // namespace

int light_bins_levels(int B) {
  int n = 0;
  for (int b = B; b >= 2 && n < kLbMaxLevels; b >>= 2) n++;
  return n;
}

int build_light_bins(const float* tri, int64_t T, float scale, const float light[3], int B, LightBinsHost& out,
                     std::string& err) {
  if (B < 2 || (B & (B - 1))) {
    err = "light bins: B must be a power of two >= 2";
    return RC_EINVAL;
  }
  out = LightBinsHost();
  out.B = B;
  out.nlev = light_bins_levels(B);
  const double eps = std::ldexp((double)scale, -24) * 64.0;
  const V L = {light[0], light[1], light[2]};
  // per (triangle, face): the level and bin rectangle it covers
  std::vector<Span> spans;
  std::vector<int32_t> span_tri;
  // per triangle: distance from L, unit plane normal facing away from L and
  // the plane's distance from L (0 if degenerate), padding in (u, v)
  std::vector<double> tdmin((size_t)std::max<int64_t>(T, 1)), tpad(tdmin.size()), th(tdmin.size());
  std::vector<V> tn(tdmin.size());
  spans.reserve((size_t)T * 2);
  for (int64_t j = 0; j < T; j++) {
    const float* t = tri + 9 * j;
    const V a = {t[0], t[1], t[2]}, b = {t[3], t[4], t[5]}, c = {t[6], t[7], t[8]};
    const double dmin = point_triangle_distance(L, a, b, c);
    tdmin[j] = dmin;
    const V e1 = sub(b, a), e2 = sub(c, a);
    V n = {e1.y * e2.z - e1.z * e2.y, e1.z * e2.x - e1.x * e2.z, e1.x * e2.y - e1.y * e2.x};
    const double nn = norm(n);
    double h = 0.0;
    if (nn > 0) {
      n = mul(1.0 / nn, n);
      h = dot(n, sub(a, L));
      if (h < 0) {
        n = mul(-1.0, n);
        h = -h;
      }
    }
    tn[j] = n;
    th[j] = h;
    const bool near = !(dmin > 2.0 * eps);
    const double alpha = near ? 1.0 : eps / (dmin - eps);
    const double pad = 3.0 * alpha + 1e-5;
    tpad[j] = pad;
    const V rel[3] = {sub(a, L), sub(b, L), sub(c, L)};
    for (int ax = 0; ax < 3; ax++) {
      const int kx = (ax + 1) % 3, ky = (ax + 2) % 3;
      for (int sg = 0; sg < 2; sg++) {
        const double s = sg == 0 ? 1.0 : -1.0;
        V poly[16], tmp[16];
        int n = 3;
        for (int q = 0; q < 3; q++) poly[q] = {comp(rel[q], kx), comp(rel[q], ky), s * comp(rel[q], ax)};
        bool full = near;
        if (!full) {
          const double w = 1.0 + pad;
          n = clip(poly, n, tmp, [w](V p) { return w * p.z - p.x; });
          n = clip(tmp, n, poly, [w](V p) { return w * p.z + p.x; });
          n = clip(poly, n, tmp, [w](V p) { return w * p.z - p.y; });
          n = clip(tmp, n, poly, [w](V p) { return w * p.z + p.y; });
          if (n == 0) continue;
        }
        double u0 = -1.0, u1 = 1.0, v0 = -1.0, v1 = 1.0;
        if (!full) {
          double zmin = poly[0].z;
          for (int q = 1; q < n; q++) zmin = std::min(zmin, poly[q].z);
          if (!(zmin > 1e-9 * (double)scale)) {
            full = true;
          } else {
            u0 = v0 = 1e300;
            u1 = v1 = -1e300;
            for (int q = 0; q < n; q++) {
              const double u = poly[q].x / poly[q].z, v = poly[q].y / poly[q].z;
              u0 = std::min(u0, u);
              u1 = std::max(u1, u);
              v0 = std::min(v0, v);
              v1 = std::max(v1, v);
            }
            u0 -= pad;
            u1 += pad;
            v0 -= pad;
            v1 += pad;
          }
        }
        // finest level whose rectangle has at most 32 x 32 bins (else the coarsest)
        Span sp{2 * ax + sg, 0, 0, 0, 0, 0};
        for (int k = 0; k < out.nlev; k++) {
          const int Bk = B >> (2 * k);
          auto bin = [Bk](double u) {
            double f = std::floor((u + 1.0) * 0.5 * Bk);
            return (int)std::min<double>(std::max<double>(f, 0.0), Bk - 1);
          };
          sp.level = k;
          sp.iu0 = bin(u0);
          sp.iu1 = bin(u1);
          sp.iv0 = bin(v0);
          sp.iv1 = bin(v1);
          if ((int64_t)(sp.iu1 - sp.iu0 + 1) * (sp.iv1 - sp.iv0 + 1) <= 1024) break;
        }
        spans.push_back(sp);
        span_tri.push_back((int32_t)j);
      }
    }
  }
  // CSR over (level, face, bin): counts, prefix sums, fill, sort by distance
  int64_t total_bins = 0;
  std::vector<int64_t> lev_bin(out.nlev);  // first bin of each level in the flat count array
  for (int k = 0; k < out.nlev; k++) {
    const int64_t Bk = B >> (2 * k);
    lev_bin[k] = total_bins + k;  // each level's starts end with its own sentinel
    total_bins += 6 * Bk * Bk;
  }
  auto bin_index = [&](int level, int face, int iu, int iv) {
    const int64_t Bk = B >> (2 * level);
    return lev_bin[level] + ((int64_t)face * Bk + iu) * Bk + iv;
  };
  // Stored distance of each (triangle, bin) entry: the distance from L of the
  // part of the triangle seen through the padded bin (the triangle clipped to
  // the bin's pyramid: the closest point of a convex planar polygon), minus
  // eps, rounded down; +inf when nothing of the triangle is seen through it
  // (the bin lies in a corner of the triangle's (u, v) box), and such entries
  // are dropped.  Walls and slabs so stay out of the lists of segments that
  // do not reach them.
  auto entry_distance = [&](int32_t j, int level, int face, int iu, int iv) -> float {
    const double Bk = (double)(B >> (2 * level)), pad = tpad[j];
    const double u0 = -1.0 + 2.0 * iu / Bk - pad, u1 = -1.0 + 2.0 * (iu + 1) / Bk + pad;
    const double v0 = -1.0 + 2.0 * iv / Bk - pad, v1 = -1.0 + 2.0 * (iv + 1) / Bk + pad;
    const int ax = face >> 1, kx = (ax + 1) % 3, ky = (ax + 2) % 3;
    const double sz = (face & 1) ? -1.0 : 1.0;
    const float* t = tri + 9 * (int64_t)j;
    V poly[16], tmp[16];
    for (int q = 0; q < 3; q++) {
      const V r = {t[3 * q] - L.x, t[3 * q + 1] - L.y, t[3 * q + 2] - L.z};
      poly[q] = {comp(r, kx), comp(r, ky), sz * comp(r, ax)};
    }
    int n = clip(poly, 3, tmp, [u0](V p) { return p.x - u0 * p.z; });
    n = clip(tmp, n, poly, [u1](V p) { return u1 * p.z - p.x; });
    n = clip(poly, n, tmp, [v0](V p) { return p.y - v0 * p.z; });
    n = clip(tmp, n, poly, [v1](V p) { return v1 * p.z - p.y; });
    if (n == 0) return INFINITY;
    // closest point of the polygon to the origin (L): the plane's foot if
    // inside, else the nearest edge point
    double d = 1e300;
    const V nrm = tn[j];
    const V nf = {comp(nrm, kx), comp(nrm, ky), sz * comp(nrm, ax)};
    const double hp = dot(nf, poly[0]);
    bool inside = n >= 3 && norm(nf) > 0;
    const V foot = mul(hp, nf);
    double sgn = 0;
    for (int q = 0; q < n && inside; q++) {
      const V a = poly[q], b = poly[(q + 1) % n];
      const V e = sub(b, a), f = sub(foot, a);
      const V c = {e.y * f.z - e.z * f.y, e.z * f.x - e.x * f.z, e.x * f.y - e.y * f.x};
      const double sd = dot(c, nf);
      if (sd != 0) {
        if (sgn == 0) sgn = sd;
        else if ((sd > 0) != (sgn > 0)) inside = false;
      }
    }
    if (inside) d = std::fabs(hp);
    for (int q = 0; q < n; q++) {
      const V a = poly[q], b = poly[(q + 1) % n];
      const V e = sub(b, a);
      const double ee = dot(e, e);
      double tq = ee > 0 ? -dot(a, e) / ee : 0.0;
      tq = std::min(1.0, std::max(0.0, tq));
      d = std::min(d, norm(add(a, mul(tq, e))));
    }
    d = std::max(d, tdmin[j]);
    const double ds = d - eps;
    float df = (float)ds;
    if ((double)df > ds) df = std::nextafter(df, -INFINITY);
    return df;
  };
  std::vector<int64_t> cnt((size_t)(total_bins + out.nlev), 0);
  // entries: (bin, distance, triangle) of every span bin that sees the triangle
  struct Ent {
    int64_t bin;
    float d;
    int32_t j;
  };
  std::vector<Ent> ents;
  ents.reserve(spans.size() * 4);
  for (size_t s = 0; s < spans.size(); s++) {
    const Span& sp = spans[s];
    for (int iu = sp.iu0; iu <= sp.iu1; iu++)
      for (int iv = sp.iv0; iv <= sp.iv1; iv++) {
        const float d = entry_distance(span_tri[s], sp.level, sp.face, iu, iv);
        if (!(d < INFINITY)) continue;
        const int64_t b = bin_index(sp.level, sp.face, iu, iv);
        ents.push_back({b, d, span_tri[s]});
        cnt[b]++;
      }
  }
  int64_t run = 0;
  for (int k = 0; k < out.nlev; k++) {
    const int64_t Bk = B >> (2 * k);
    const int64_t lo = lev_bin[k], hi = lo + 6 * Bk * Bk;
    for (int64_t i = lo; i < hi; i++) {
      const int64_t c = cnt[i];
      cnt[i] = run;
      run += c;
    }
    cnt[hi] = run;  // sentinel: end of the level's last bin
  }
  if (run >= ((int64_t)1 << 31)) {
    err = "light bins: too many entries";
    return RC_EINVAL;
  }
  std::vector<int32_t> ids((size_t)run);
  std::vector<float> edist((size_t)run);
  std::vector<int64_t> cur(cnt.begin(), cnt.end());
  for (const Ent& e : ents) {
    const int64_t k = cur[e.bin]++;
    ids[(size_t)k] = e.j;
    edist[(size_t)k] = e.d;
  }
  std::vector<Ent>().swap(ents);
  // bin headers, two words per bin: the first entry's index and its stored
  // distance (+inf for an empty bin); the level's last word is the end of
  // its last bin
  out.offs.assign((size_t)(2 * total_bins + out.nlev), 0);
  for (int k = 0; k < out.nlev; k++) out.lev_off[k] = 2 * lev_bin[k] - k;
  out.entries.assign((size_t)run * 12, 0.f);
  for (int k = 0; k < out.nlev; k++) {
    const int64_t Bk = B >> (2 * k);
    const int64_t nb = 6 * Bk * Bk;
    out.offs[(size_t)(out.lev_off[k] + 2 * nb)] = (int32_t)cnt[(size_t)(lev_bin[k] + nb)];
    for (int face = 0; face < 6; face++) {
      const int ax = face >> 1;
      for (int64_t bi = 0; bi < Bk * Bk; bi++) {
        const int64_t slot = lev_bin[k] + face * Bk * Bk + bi;
        const int64_t lo = cnt[slot], hi = cnt[slot + 1];
        std::vector<std::pair<float, int32_t>> srt;
        srt.reserve((size_t)(hi - lo));
        for (int64_t e = lo; e < hi; e++) srt.emplace_back(edist[(size_t)e], ids[(size_t)e]);
        std::sort(srt.begin(), srt.end());
        for (int64_t e = lo; e < hi; e++) {
          edist[(size_t)e] = srt[(size_t)(e - lo)].first;
          ids[(size_t)e] = srt[(size_t)(e - lo)].second;
        }
        const int64_t h = out.lev_off[k] + 2 * (face * Bk * Bk + bi);
        out.offs[(size_t)h] = (int32_t)lo;
        const float dfirst = lo < hi ? edist[(size_t)lo] : INFINITY;
        std::memcpy(&out.offs[(size_t)h + 1], &dfirst, 4);
        for (int64_t e = lo; e < hi; e++) {
          const int32_t j = ids[(size_t)e];
          const float* t = tri + 9 * (int64_t)j;
          float* o = out.entries.data() + 12 * e;
          for (int vtx = 0; vtx < 3; vtx++) {
            o[4 * vtx + 0] = t[3 * vtx + (ax + 1) % 3];
            o[4 * vtx + 1] = t[3 * vtx + (ax + 2) % 3];
            o[4 * vtx + 2] = t[3 * vtx + ax];
          }
          std::memcpy(&o[3], &j, 4);
          o[7] = edist[(size_t)e];
          o[11] = e + 1 < hi ? edist[(size_t)e + 1] : INFINITY;  // the next entry's distance
        }
      }
    }
  }
  return RC_OK;
}

int light_bins_size_for(int64_t T) {
  // about 2 sqrt(T) bins per face side at the finest level, a power of two in
  // [16, 2048] (measured launch times: 100k triangles with slabs 463 ms at 512,
  // 467 at 1024; 1M triangles 5237 ms at 512, 4819 at 1024, 4688 at 2048 with
  // 3.9 GB of bins for four lights)
  const double want = 2.0 * std::sqrt((double)std::max<int64_t>(T, 1));
  int B = 16;
  while (B < 2048 && (double)B * 1.41421356 < want) B <<= 1;
  return B;
}

}  // namespace rc
