// bvh.cpp -- host builder of the flat binary BVH traversed by the record
// kernel.  Binned surface-area heuristic (32 bins per axis over centroid
// bounds), leaves of at most kLeafMax triangles, object-median fallback when
// the heuristic finds no split or the tree gets deep.  A node of at most
// kLeafMax triangles is split further when the heuristic prices the split
// below testing every triangle, with one traversal step and one triangle test
// costing the same (each is one iteration of the kernel's traversal loop);
// such splits stop at the depth that keeps the traversal stack of the plain
// build, so a tighter tree never costs the kernel LDS.  When a tree bounded
// to the next smaller stack (median splits wherever the heuristic's split
// could not be finished as a balanced tree within the bound) prices within
// 3 % of the unbounded one, the bounded tree is kept: its smaller stack lets
// more wavefronts share a CU.  The paper relies on
// Embree for tracing (Sec. 6) and describes no acceleration structure; this
// one is laid out for the GPU: both children's boxes in one 64-byte node, and
// the triangles of a leaf contiguous in the order the leaf lists them.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "internal.hpp"

namespace rc {
namespace {

struct Prim {
  float lo[3], hi[3], c[3];
  int32_t id;
};

struct Box {
  float lo[3] = {std::numeric_limits<float>::infinity(), std::numeric_limits<float>::infinity(),
                 std::numeric_limits<float>::infinity()};
  float hi[3] = {-std::numeric_limits<float>::infinity(), -std::numeric_limits<float>::infinity(),
                 -std::numeric_limits<float>::infinity()};
  void grow(const float* l, const float* h) {
    for (int k = 0; k < 3; k++) {
      lo[k] = std::min(lo[k], l[k]);
      hi[k] = std::max(hi[k], h[k]);
    }
  }
  void grow(const Box& b) { grow(b.lo, b.hi); }
  double area() const {
    if (!(hi[0] >= lo[0])) return 0.0;
    double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    return 2.0 * (dx * dy + dy * dz + dz * dx);
  }
};

struct Builder {
  std::vector<Prim>& prims;
  const float* tri;
  float pad;
  std::vector<float>& nodes;
  std::vector<float>& tris;
  int max_depth_seen = 0;

  Box bounds(int64_t b, int64_t e) const {
    Box bx;
    for (int64_t i = b; i < e; i++) bx.grow(prims[i].lo, prims[i].hi);
    return bx;
  }

  static int32_t as_i(float f) {
    int32_t i;
    std::memcpy(&i, &f, 4);
    return i;
  }
  static float as_f(int32_t i) {
    float f;
    std::memcpy(&f, &i, 4);
    return f;
  }

  int32_t make_leaf(int64_t b, int64_t e) {
    int64_t first = (int64_t)tris.size() / 12;
    for (int64_t i = b; i < e; i++) {
      const float* t = tri + 9 * (int64_t)prims[i].id;
      float rec[12] = {t[0], t[1], t[2], as_f(prims[i].id), t[3], t[4], t[5], 0.f, t[6], t[7], t[8], 0.f};
      tris.insert(tris.end(), rec, rec + 12);
    }
    int64_t cnt = e - b;
    return ~(int32_t)((first << 3) | (cnt - 1));
  }

  // Large triangles (room walls, slab faces) whose boxes span most of the
  // node would inflate every subtree they land in; they are split off into
  // their own subtree first.  Returns mid or -1 if nothing to separate.
  int64_t split_large(int64_t b, int64_t e) {
    Box nb = bounds(b, e);
    float ext = std::max({nb.hi[0] - nb.lo[0], nb.hi[1] - nb.lo[1], nb.hi[2] - nb.lo[2]});
    auto big = [&](const Prim& p) {
      float s = std::max({p.hi[0] - p.lo[0], p.hi[1] - p.lo[1], p.hi[2] - p.lo[2]});
      return s > 0.5f * ext;
    };
    int64_t nbig = 0;
    for (int64_t i = b; i < e; i++) nbig += big(prims[i]) ? 1 : 0;
    if (nbig == 0 || nbig == e - b || nbig > (e - b) / 2) return -1;
    auto it = std::stable_partition(prims.begin() + b, prims.begin() + e, big);
    return it - prims.begin();
  }

  // depth below which nodes of at most kLeafMax triangles may still be split
  int leaf_split_depth = 0;
  // bound on the final depth (0: none)
  int depth_bound = 0;
  // surface-area cost of the tree built so far: box area per node visit plus
  // box area x triangles per leaf (one traversal step = one triangle test)
  double sah = 0.0;

  // a child of n triangles at depth d can still be finished as a balanced
  // tree (leaves of kLeafMax) within depth_bound
  bool fits(int64_t n, int d) const {
    if (depth_bound <= 0) return true;
    int64_t cap = kLeafMax;
    for (int l = d; l < depth_bound - 1 && cap < (int64_t(1) << 40); l++) cap *= 2;
    return n <= cap;
  }

  // Split [b, e) -> mid; returns mid (b < mid < e).  leaf_cheaper (if given):
  // the heuristic's best split costs no less than testing all triangles.
  int64_t split(int64_t b, int64_t e, int depth, bool* leaf_cheaper = nullptr) {
    int64_t n = e - b;
    if (leaf_cheaper) *leaf_cheaper = true;
    if (n > 2 * kLeafMax) {
      int64_t m = split_large(b, e);
      if (m > b && m < e && fits(m - b, depth + 1) && fits(e - m, depth + 1)) return m;
    }
    Box cb;
    for (int64_t i = b; i < e; i++) cb.grow(prims[i].c, prims[i].c);
    int axis = 0;
    float ext = cb.hi[0] - cb.lo[0];
    for (int k = 1; k < 3; k++)
      if (cb.hi[k] - cb.lo[k] > ext) { ext = cb.hi[k] - cb.lo[k]; axis = k; }
    auto median = [&](int ax) {
      int64_t mid = b + n / 2;
      std::nth_element(prims.begin() + b, prims.begin() + mid, prims.begin() + e,
                       [ax](const Prim& p, const Prim& q) { return p.c[ax] < q.c[ax] || (p.c[ax] == q.c[ax] && p.id < q.id); });
      return mid;
    };
    if (!(ext > 0.f) || depth > 40) return median(axis);
    constexpr int NB = 32;
    double best = std::numeric_limits<double>::infinity();
    int best_axis = -1, best_bin = -1;
    for (int ax = 0; ax < 3; ax++) {
      float lo = cb.lo[ax], w = cb.hi[ax] - cb.lo[ax];
      if (!(w > 0.f)) continue;
      Box bb[NB];
      int64_t cnt[NB] = {0};
      for (int64_t i = b; i < e; i++) {
        int k = (int)((prims[i].c[ax] - lo) / w * NB);
        k = std::min(std::max(k, 0), NB - 1);
        cnt[k]++;
        bb[k].grow(prims[i].lo, prims[i].hi);
      }
      double ra[NB];
      int64_t rc[NB];
      Box acc;
      int64_t c = 0;
      for (int k = NB - 1; k > 0; k--) {
        acc.grow(bb[k]);
        c += cnt[k];
        ra[k] = acc.area();
        rc[k] = c;
      }
      Box accl;
      int64_t cl = 0;
      for (int k = 0; k < NB - 1; k++) {
        accl.grow(bb[k]);
        cl += cnt[k];
        if (cl == 0 || rc[k + 1] == 0) continue;
        double cost = accl.area() * (double)cl + ra[k + 1] * (double)rc[k + 1];
        if (cost < best) { best = cost; best_axis = ax; best_bin = k; }
      }
    }
    if (leaf_cheaper && best_axis >= 0) {
      // cost of the split in triangle tests: one step for the node, then the
      // children's triangles weighted by the chance of entering each child
      const double A = bounds(b, e).area();
      *leaf_cheaper = !(A > 0.0) || 1.0 + best / A >= (double)n;
    }
    if (best_axis < 0) return median(axis);
    float lo = cb.lo[best_axis], w = cb.hi[best_axis] - cb.lo[best_axis];
    auto mid_it = std::partition(prims.begin() + b, prims.begin() + e, [&](const Prim& p) {
      int k = (int)((p.c[best_axis] - lo) / w * NB);
      k = std::min(std::max(k, 0), NB - 1);
      return k <= best_bin;
    });
    int64_t mid = mid_it - prims.begin();
    if (mid <= b || mid >= e) return median(axis);
    if (!fits(mid - b, depth + 1) || !fits(e - mid, depth + 1)) return median(best_axis);
    return mid;
  }

  // Build the subtree over [b, e); returns its child code.
  int32_t build(int64_t b, int64_t e, int depth) {
    max_depth_seen = std::max(max_depth_seen, depth);
    int64_t n = e - b;
    bool leaf = n <= kLeafMax && (n == 1 || depth + 1 >= leaf_split_depth);
    int64_t mid = 0;
    if (!leaf) {
      bool leaf_cheaper = false;
      mid = split(b, e, depth, n <= kLeafMax ? &leaf_cheaper : nullptr);
      leaf = n <= kLeafMax && leaf_cheaper;
    }
    if (leaf) {
      sah += bounds(b, e).area() * (double)n;
      return make_leaf(b, e);
    }
    int64_t idx = (int64_t)nodes.size() / 16;
    nodes.resize(nodes.size() + 16, 0.f);
    Box l = bounds(b, mid), r = bounds(mid, e);
    Box lr = l;
    lr.grow(r);
    sah += lr.area();
    int32_t c0 = build(b, mid, depth + 1);
    int32_t c1 = build(mid, e, depth + 1);
    write_node(idx, l, r, c0, c1);
    return (int32_t)idx;
  }

  void write_node(int64_t idx, const Box& l, const Box& r, int32_t c0, int32_t c1) {
    float* nd = nodes.data() + 16 * idx;
    auto plo = [&](float v) { return v - pad; };
    auto phi = [&](float v) { return v + pad; };
    nd[0] = plo(l.lo[0]); nd[1] = phi(l.hi[0]); nd[2] = plo(l.lo[1]); nd[3] = phi(l.hi[1]);
    nd[4] = plo(r.lo[0]); nd[5] = phi(r.hi[0]); nd[6] = plo(r.lo[1]); nd[7] = phi(r.hi[1]);
    nd[8] = plo(l.lo[2]); nd[9] = phi(l.hi[2]); nd[10] = plo(r.lo[2]); nd[11] = phi(r.hi[2]);
    nd[12] = as_f(c0); nd[13] = as_f(c1); nd[14] = 0.f; nd[15] = 0.f;
  }
};

}  // namespace

float bvh_pad_for(const float* tri, int64_t T, const float* lo, const float* hi) {
  double m = 0.0;
  for (int k = 0; k < 3; k++) m = std::max({m, std::fabs((double)lo[k]), std::fabs((double)hi[k]),
                                            (double)hi[k] - (double)lo[k]});
  for (int64_t i = 0; i < 9 * T; i++) m = std::max(m, std::fabs((double)tri[i]));
  return (float)(m > 0 ? m : 1.0);
}

// Padding of one triangle's box.  A hit accepted by the watertight test is
// the point o + t d with t rounded once to FP32 from a value that is exact for
// vertices moved by a few units of FP32 rounding (the projection along the ray
// is the only other inexact step; the edge functions keep exact signs), so it
// lies within ~16 * 2^-24 * scale of the triangle's box; the slab tests of the
// traversal (hardware reciprocal, fused multiply-add) err by a few units of
// rounding of the coordinates, also below that.  The pad is 2^-16 * scale,
// 16 times the bound, and independent of the triangle's shape.
float triangle_pad(const float* /*t*/, float scale) { return std::ldexp(scale, -16); }

int build_bvh(const float* tri, int64_t T, float pad, HostBvh& out, std::string& err) {
  out.nodes.clear();
  out.tris.clear();
  out.pad = pad;
  if (T >= (int64_t(1) << 28)) {
    err = "too many triangles";
    return RC_EINVAL;
  }
  std::vector<Prim> prims((size_t)T);
  for (int64_t i = 0; i < T; i++) {
    Prim& p = prims[i];
    const float* t = tri + 9 * i;
    float pi = triangle_pad(t, pad);
    for (int k = 0; k < 3; k++) {
      p.lo[k] = std::min({t[k], t[3 + k], t[6 + k]}) - pi;
      p.hi[k] = std::max({t[k], t[3 + k], t[6 + k]}) + pi;
      p.c[k] = (t[k] + t[3 + k] + t[6 + k]) * (1.0f / 3.0f);
    }
    p.id = (int32_t)i;
  }
  std::vector<Prim> prims0 = prims;
  // One build of the whole tree (root always internal: the traversal starts
  // by testing both of its children); returns its depth.
  auto build_tree = [&](int leaf_split_depth, int depth_bound, std::vector<float>& nodes,
                        std::vector<float>& tris, double& sah) {
    prims = prims0;
    nodes.assign(16, 0.f);
    tris.clear();
    Builder bd{prims, tri, 0.0f, nodes, tris};
    bd.leaf_split_depth = leaf_split_depth;
    bd.depth_bound = depth_bound;
    int64_t mid = bd.split(0, T, 0);
    Box l = bd.bounds(0, mid), r = bd.bounds(mid, T);
    Box lr = l;
    lr.grow(r);
    bd.sah = lr.area();
    int32_t c0 = bd.build(0, mid, 1);
    int32_t c1 = bd.build(mid, T, 1);
    bd.write_node(0, l, r, c0, c1);
    sah = bd.sah;
    return bd.max_depth_seen + 1;
  };
  if (T <= kLeafMax) {
    Builder bd{prims, tri, 0.0f, out.nodes, out.tris};
    out.nodes.resize(16, 0.f);
    Box empty;  // inverted box: never hit
    int32_t c0 = T > 0 ? bd.make_leaf(0, T) : ~0;
    Box l = T > 0 ? bd.bounds(0, T) : empty;
    bd.write_node(0, l, empty, c0, ~0);
    // the empty child keeps its inverted box (padding must not make it valid)
    float* nd = out.nodes.data();
    nd[4] = std::numeric_limits<float>::infinity(); nd[5] = -std::numeric_limits<float>::infinity();
    nd[6] = std::numeric_limits<float>::infinity(); nd[7] = -std::numeric_limits<float>::infinity();
    nd[10] = std::numeric_limits<float>::infinity(); nd[11] = -std::numeric_limits<float>::infinity();
    if (T == 0) {
      nd[0] = std::numeric_limits<float>::infinity(); nd[1] = -std::numeric_limits<float>::infinity();
      nd[2] = std::numeric_limits<float>::infinity(); nd[3] = -std::numeric_limits<float>::infinity();
      nd[8] = std::numeric_limits<float>::infinity(); nd[9] = -std::numeric_limits<float>::infinity();
    }
    out.depth = 1;
    return RC_OK;
  }
  // plain build (no splits below kLeafMax triangles): its depth sets the stack
  double sah = 0.0;
  std::vector<float> nodes_b, tris_b;
  const int d0 = build_tree(0, 0, nodes_b, tris_b, sah);
  const int s0 = stack_variant(d0);
  // the tree the kernel gets: small nodes split down to that stack's depth
  out.depth = build_tree(s0, 0, out.nodes, out.tris, sah);
  // or a tree bounded to the next smaller stack, if it prices within 3 %
  const int sb = s0 == 64 ? 48 : (s0 == 48 ? 32 : (s0 == 32 ? 24 : (s0 == 24 ? 16 : 0)));
  if (sb > 0) {
    double sah_b = 0.0;
    const int db = build_tree(sb, sb, nodes_b, tris_b, sah_b);
    if (db <= sb && sah_b <= 1.03 * sah) {
      out.nodes.swap(nodes_b);
      out.tris.swap(tris_b);
      out.depth = db;
    }
  }
  if (out.depth > kMaxDepth) {
    err = "BVH deeper than the traversal stack";
    return RC_EINVAL;
  }
  return RC_OK;
}

}  // namespace rc
