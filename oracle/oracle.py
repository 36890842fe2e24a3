"""Python side of the FP64 CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It loads ``oracle/liboracle.so`` (built from
``oracle/rco.c`` by ``oracle/build.py``) and adds the parts of the method that
are plain linear algebra, written here in numpy:

* the validity radius of a record (Sec. 5, Eq. radiusAniso3D, with the
  isotropic choice of the largest |eigenvalue| as in Sec. 6) and the
  ellipsoid of an anisotropic cache point;
* the sequential greedy cover (Sec. 6 insertion rule) with balls or ellipsoids;
* the multi-point interpolation of a cache (Sec. 5, Eq. radianceTaylor, with
  the cubic kernel);
* the render pass that consumes a cache (Sec. 6 "Implementation"): uniform
  ray marching of camera rays and the pixel estimates;
* an FP64 reference of the small MLP used for learned placement (not part of
  the paper).

Nothing here is shared with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_LIB = None


_LIB_PATH = None  # None: oracle/liboracle.so


def use_library(path=None):
    """Load the oracle from another build of rco.c (tests of the pins build
    copies with planted mistakes); None restores oracle/liboracle.so."""
    global _LIB, _LIB_PATH
    _LIB, _LIB_PATH = None, path


def lib():
    global _LIB
    if _LIB is None:
        path = Path(_LIB_PATH) if _LIB_PATH is not None else _HERE / "liboracle.so"
        if not path.exists():
            from . import build as _b  # noqa: F401  (oracle/build.py)
            _b.build()
        L = C.CDLL(str(path))
        vp, i64, f32, i32, u64 = C.c_void_p, C.c_int64, C.c_float, C.c_int, C.c_uint64
        L.rco_scene_create.argtypes = [vp, vp, vp, i64, vp, vp, C.POINTER(vp)]
        L.rco_scene_create.restype = i32
        L.rco_scene_destroy.argtypes = [vp]
        L.rco_scene_destroy.restype = None
        L.rco_records.argtypes = [vp, f32, f32, vp, i32, vp, vp, vp, vp, i64, f32, i32, u64, vp,
                                  vp, vp, vp, vp, i32]
        L.rco_records.restype = i32
        L.rco_values.argtypes = [vp, f32, f32, vp, i32, vp, vp, vp, vp, i64, f32, i32, u64, vp, i32]
        L.rco_values.restype = i32
        L.rco_j08.argtypes = [vp, f32, f32, vp, i32, vp, vp, vp, vp, i64, f32, i32, u64, vp, vp, vp, i32]
        L.rco_j08.restype = i32
        L.rco_trace.argtypes = [vp, vp, vp, i64, i32, vp, vp, vp]
        L.rco_trace.restype = i32
        L.rco_occluded.argtypes = [vp, vp, vp, vp, i64, i32, vp]
        L.rco_occluded.restype = i32
        L.rco_formfactor.argtypes = [vp, vp, vp, vp, vp, vp]
        L.rco_formfactor.restype = None
        L.rco_transmittance.argtypes = [vp, vp, C.c_double, vp, vp, vp]
        L.rco_transmittance.restype = None
        L.rco_directions.argtypes = [u64, u64, i32, i32, vp]
        L.rco_directions.restype = i32
        L.rco_triangles.argtypes = [vp, i32, i32, vp]
        L.rco_triangles.restype = i32
        L.rco_unif.argtypes = [u64, u64, u64, u64]
        L.rco_unif.restype = f32
        L.rco_splitmix64.argtypes = [u64]
        L.rco_splitmix64.restype = u64
        L.rco_nstat.restype = i32
        L.rco_probe.argtypes = [vp, f32, f32, vp, i32, vp, i64, u64, vp, vp]
        L.rco_probe.restype = i32
        _LIB = L
    return _LIB


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


STAT_NAMES = ["rays", "terms_ss", "terms_ms", "SG_ss", "SH_ss", "SG_ms", "SH_ms", "tri_value_ss",
              "tri_value_ms", "hess_asym", "max_rings_used", "n_triangles"]


class Scene:
    """Host copy of a triangle scene with the oracle's own acceleration."""

    def __init__(self, tri, albedo, emission=None, box_lo=(0, 0, 0), box_hi=(1, 1, 1)):
        self.tri = _c(tri, np.float32).reshape(-1, 9)
        self.albedo = _c(albedo, np.float32)
        self.emission = None if emission is None else _c(emission, np.float32)
        self.box_lo = _c(box_lo, np.float32)
        self.box_hi = _c(box_hi, np.float32)
        h = C.c_void_p()
        rc = lib().rco_scene_create(_p(self.tri), _p(self.albedo), _p(self.emission), self.tri.shape[0],
                                    _p(self.box_lo), _p(self.box_hi), C.byref(h))
        if rc != 0:
            raise RuntimeError(f"rco_scene_create failed ({rc})")
        self._h = h

    @classmethod
    def from_workload(cls, w):
        return cls(w.tri, w.albedo, w.emission, w.box_lo, w.box_hi)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().rco_scene_destroy(h)
            self._h = None

    def trace(self, orig, dirs, brute=False):
        o = _c(orig, np.float32).reshape(-1, 3)
        d = _c(dirs, np.float32).reshape(-1, 3)
        n = o.shape[0]
        hid = np.empty(n, np.int64)
        t = np.empty(n, np.float32)
        fr = np.empty(n, np.int32)
        rc = lib().rco_trace(self._h, _p(o), _p(d), n, int(brute), _p(hid), _p(t), _p(fr))
        assert rc == 0
        return hid, t, fr

    def occluded(self, orig, seg, skip=None, brute=False):
        o = _c(orig, np.float32).reshape(-1, 3)
        d = _c(seg, np.float32).reshape(-1, 3)
        n = o.shape[0]
        sk = None if skip is None else _c(skip, np.int64)
        occ = np.empty(n, np.int32)
        rc = lib().rco_occluded(self._h, _p(o), _p(d), _p(sk), n, int(brute), _p(occ))
        assert rc == 0
        return occ.astype(bool)


def records(scene: Scene, sigma_s, sigma_a, lights, pos, n_theta, n_phi, rec_id=None, ring_step=0.1,
            max_rings=20, seed=0, xeval=None, nthreads=0, want_stats=True):
    """Oracle records.  Returns dict(value [P,2], grad [P,2,3], hess [P,2,6], stats [P,12])."""
    pos = _c(pos, np.float32).reshape(-1, 3)
    P = pos.shape[0]
    nt = _c(np.broadcast_to(n_theta, (P,)), np.int32)
    npf = _c(np.broadcast_to(n_phi, (P,)), np.int32)
    rid = _c(np.arange(P) if rec_id is None else rec_id, np.uint64)
    li = _c(lights, np.float32).reshape(-1, 4)
    xe = None if xeval is None else _c(xeval, np.float64).reshape(-1, 3)
    val = np.zeros((P, 2))
    grad = np.zeros((P, 2, 3))
    hess = np.zeros((P, 2, 6))
    st = np.zeros((P, len(STAT_NAMES))) if want_stats else None
    rc = lib().rco_records(scene._h, float(sigma_s), float(sigma_a), _p(li), li.shape[0], _p(pos), _p(nt), _p(npf),
                           _p(rid), P, float(ring_step), int(max_rings), int(seed) & (2**64 - 1), _p(xe),
                           _p(val), _p(grad), _p(hess), _p(st), int(nthreads))
    if rc != 0:
        raise ValueError(f"rco_records failed ({rc})")
    out = {"value": val, "grad": grad, "hess": hess}
    if want_stats:
        out["stats"] = st
    return out


def values(scene: Scene, sigma_s, sigma_a, lights, pos, n_theta, n_phi, rec_id=None, ring_step=0.1,
           max_rings=20, seed=0, nthreads=0):
    """Monte Carlo values only (no triangulation): [P, 2]."""
    pos = _c(pos, np.float32).reshape(-1, 3)
    P = pos.shape[0]
    nt = _c(np.broadcast_to(n_theta, (P,)), np.int32)
    npf = _c(np.broadcast_to(n_phi, (P,)), np.int32)
    rid = _c(np.arange(P) if rec_id is None else np.broadcast_to(rec_id, (P,)), np.uint64)
    li = _c(lights, np.float32).reshape(-1, 4)
    val = np.zeros((P, 2))
    rc = lib().rco_values(scene._h, float(sigma_s), float(sigma_a), _p(li), li.shape[0], _p(pos), _p(nt), _p(npf),
                          _p(rid), P, float(ring_step), int(max_rings), int(seed) & (2**64 - 1), _p(val),
                          int(nthreads))
    if rc != 0:
        raise ValueError(f"rco_values failed ({rc})")
    return val


def j08(scene: Scene, sigma_s, sigma_a, lights, pos, n_theta, n_phi, rec_id=None, ring_step=0.1, max_rings=20,
        seed=0, nthreads=0):
    """The comparison method's occlusion-unaware gradients (Jarosz et al.
    2008: surface hit points held fixed, medium paths moved rigidly;
    supplement Eqs. S.3-S.4) from the record's own samples.  Returns (value
    [P][2], grad [P][2][3], moments [P][2] = means over the directions of the
    per-direction sample L_k and of its gradient norm |grad L_k|)."""
    pos = _c(pos, np.float32).reshape(-1, 3)
    P = pos.shape[0]
    nt = _c(np.broadcast_to(n_theta, (P,)), np.int32)
    npf = _c(np.broadcast_to(n_phi, (P,)), np.int32)
    rid = _c(np.arange(P) if rec_id is None else rec_id, np.uint64)
    li = _c(lights, np.float32).reshape(-1, 4)
    val = np.zeros((P, 2))
    grad = np.zeros((P, 2, 3))
    mom = np.zeros((P, 2))
    rc = lib().rco_j08(scene._h, float(sigma_s), float(sigma_a), _p(li), li.shape[0], _p(pos), _p(nt), _p(npf),
                       _p(rid), P, float(ring_step), int(max_rings), int(seed) & (2**64 - 1), _p(val), _p(grad),
                       _p(mom), int(nthreads))
    if rc != 0:
        raise ValueError(f"rco_j08 failed ({rc})")
    return val, grad, mom


def j08_radius(moments, eps, r_min, r_max):
    """Eq. jaroszRadius: R = eps * sum_k L_k / sum_k |grad L_k| over the
    record's per-direction samples, clamped to [r_min, r_max] (the paper's
    comparison clamps to a minimum radius); moments [P][2] from j08()."""
    m = np.asarray(moments, np.float64).reshape(-1, 2)
    with np.errstate(divide="ignore", invalid="ignore"):
        R = np.where(m[:, 1] > 0, eps * m[:, 0] / m[:, 1], np.inf)
    return np.clip(R, r_min, r_max).astype(np.float32)


def records_for(w, idx=None, xeval=None, nthreads=0, scene=None):
    """Oracle records for (a subset of) a workload; record ids are the indices."""
    idx = np.arange(w.n_rec) if idx is None else np.asarray(idx)
    sc = scene if scene is not None else Scene.from_workload(w)
    return records(sc, w.sigma_s, w.sigma_a, w.lights, w.pos[idx], w.n_theta[idx], w.n_phi[idx], rec_id=idx,
                   ring_step=w.ring_step, max_rings=w.max_rings, seed=w.seed, xeval=xeval, nthreads=nthreads)


def probe(scene: Scene, sigma_s, sigma_a, lights, cand, seed, ids=None):
    """32 probe features per candidate (FP64 values, FP32 decisions)."""
    cand = _c(cand, np.float32).reshape(-1, 3)
    n = cand.shape[0]
    ids = _c(np.arange(n) if ids is None else ids, np.uint64)
    li = _c(lights, np.float32).reshape(-1, 4)
    feat = np.zeros((n, 32))
    rc = lib().rco_probe(scene._h, float(sigma_s), float(sigma_a), _p(li), li.shape[0], _p(cand), n,
                         int(seed) & (2**64 - 1), _p(ids), _p(feat))
    if rc != 0:
        raise ValueError(f"rco_probe failed ({rc})")
    return feat


def _within32(q, p, R):
    """|q - p|^2 < R^2 taken in FP32 as ((dx*dx + dy*dy) + dz*dz) < R*R: the one
    discrete decision of cover and interpolation, made in single precision so
    that both implementations decide alike."""
    d = np.asarray(q, np.float32) - np.asarray(p, np.float32)
    d2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    R = np.asarray(R, np.float32)
    return d2 < R * R


def ellipsoid_form(Ri, vecs):
    """Anisotropic cache point (Sec. 5, Eq. radiusAniso3D: the valid region is
    an ellipsoid with principal radii R_i along the Hessian's eigenvectors):
    the quadratic form M = sum_i v_i v_i^T / R_i^2, so that x' lies inside iff
    (x' - x)^T M (x' - x) < 1.  Ri [K,3] and vecs [K,3,3] (row i = unit
    eigenvector i) are the FP32 values a cache stores; each entry
    sum_i (v_i[a] v_i[b]) / (R_i R_i) is formed in FP64 (terms added in axis
    order) and rounded once to FP32.  Returns float32 [K,6] =
    (m00, m01, m02, m11, m12, m22)."""
    R = np.asarray(Ri, np.float32).astype(np.float64).reshape(-1, 3)
    V = np.asarray(vecs, np.float32).astype(np.float64).reshape(-1, 3, 3)
    out = np.zeros((len(R), 6), np.float32)
    for e, (a, b) in enumerate(((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))):
        t = [(V[:, i, a] * V[:, i, b]) / (R[:, i] * R[:, i]) for i in range(3)]
        out[:, e] = ((t[0] + t[1]) + t[2]).astype(np.float32)
    return out


def _within_form32(q, p, form):
    """(q - p)^T M (q - p) < 1 in FP32, evaluated as
    ((m00 dx^2 + m11 dy^2) + m22 dz^2) + 2 ((m01 dx dy + m02 dx dz) + m12 dy dz)
    with every product and sum rounded to FP32 in that order (the cover and
    interpolation decision of anisotropic points, taken alike on both sides)."""
    d = np.asarray(q, np.float32) - np.asarray(p, np.float32)
    m = np.asarray(form, np.float32)
    dx, dy, dz = d[..., 0], d[..., 1], d[..., 2]
    diag = (m[..., 0] * (dx * dx) + m[..., 3] * (dy * dy)) + m[..., 5] * (dz * dz)
    off = (m[..., 1] * (dx * dy) + m[..., 2] * (dx * dz)) + m[..., 4] * (dy * dz)
    return (diag + np.float32(2) * off) < np.float32(1)


def greedy_cover(cand, radius, form=None):
    """Sequential greedy cover (Sec. 6 insertion rule applied to a candidate
    list): visit the candidates in index order and accept one unless an already
    accepted point p lies inside p's valid region: the ball of p's radius, or,
    with form [C,6] (anisotropic points), p's ellipsoid.  Returns the accepted
    indices in acceptance order."""
    cand = np.asarray(cand, np.float32)
    radius = np.asarray(radius, np.float32)
    acc = []
    for i in range(len(cand)):
        if acc:
            inside = (_within32(cand[i], cand[acc], radius[acc]) if form is None
                      else _within_form32(cand[i], cand[acc], np.asarray(form, np.float32)[acc]))
            if np.any(inside):
                continue
        acc.append(i)
    return np.array(acc, np.int64)


def formfactor(r1, r2, r3):
    """App. C: F, grad F, Hessian F for vertices r_i = y_i - x (FP64)."""
    a = [_c(r, np.float64) for r in (r1, r2, r3)]
    F = np.zeros(1)
    g = np.zeros(3)
    H = np.zeros(9)
    lib().rco_formfactor(_p(a[0]), _p(a[1]), _p(a[2]), _p(F), _p(g), _p(H))
    return F[0], g, H.reshape(3, 3)


def transmittance(x, y, mu):
    """App. A: T, grad T, Hessian T w.r.t. the shaded point x."""
    xx = _c(x, np.float64)
    yy = _c(y, np.float64)
    T = np.zeros(1)
    g = np.zeros(3)
    H = np.zeros(9)
    lib().rco_transmittance(_p(xx), _p(yy), float(mu), _p(T), _p(g), _p(H))
    return T[0], g, H.reshape(3, 3)


def directions(seed, rec, nth, nph):
    out = np.zeros((nth * nph + 2, 3), np.float32)
    assert lib().rco_directions(int(seed), int(rec), nth, nph, _p(out)) == 0
    return out


def triangles(dirs, nth, nph):
    d = _c(dirs, np.float32).reshape(-1, 3)
    out = np.zeros((2 * nth * nph, 3), np.int32)
    n = lib().rco_triangles(_p(d), nth, nph, _p(out))
    assert n == 2 * nth * nph
    return out


def unif(seed, rec, idx, dim):
    return float(lib().rco_unif(int(seed), int(rec), int(idx), int(dim)))


def splitmix64(x):
    return int(lib().rco_splitmix64(int(x) & (2**64 - 1)))


# --------------------------------------------------------------------------
# Sec. 5: validity radius (Eq. radiusAniso3D)
# --------------------------------------------------------------------------
def hess6_to_mat(h6):
    h6 = np.asarray(h6, np.float64)
    H = np.empty(h6.shape[:-1] + (3, 3))
    H[..., 0, 0] = h6[..., 0]
    H[..., 0, 1] = H[..., 1, 0] = h6[..., 1]
    H[..., 0, 2] = H[..., 2, 0] = h6[..., 2]
    H[..., 1, 1] = h6[..., 3]
    H[..., 1, 2] = H[..., 2, 1] = h6[..., 4]
    H[..., 2, 2] = h6[..., 5]
    return H


def radius(value, hess6, eps, r_min, r_max, anisotropic=False):
    """R_i = (15 L eps / (4 pi |lambda_i|))^(1/5) per eigen-axis of the radiance
    Hessian (Eq. radiusAniso3D); the isotropic radius uses the largest
    |lambda| (Sec. 6: isotropic points with the smallest principal axis).
    Radii are clamped to [r_min, r_max]; lambda = 0 gives r_max; L <= 0 gives
    r_min.  value [P], hess6 [P,6] (already summed over channels)."""
    L = np.asarray(value, np.float64)
    H = hess6_to_mat(hess6)
    lam, vec = np.linalg.eigh(H)
    absl = np.abs(lam)
    with np.errstate(divide="ignore", invalid="ignore"):
        Ri = (15.0 * L[:, None] * eps / (4.0 * np.pi * absl)) ** 0.2
    Ri = np.where(absl == 0, r_max, Ri)
    Ri = np.where(L[:, None] <= 0, r_min, Ri)
    Ri = np.clip(Ri, r_min, r_max)
    R = Ri.min(axis=1)
    if anisotropic:
        return R, Ri, vec
    return R


# --------------------------------------------------------------------------
# Sec. 5: interpolation from several cache points (Eq. radianceTaylor)
# --------------------------------------------------------------------------
def interpolate(cache_pos, cache_val, cache_grad, cache_R, query, cache_form=None):
    """L(x') = sum_k [L_k + grad L_k . (x' - x_k)] w_k / sum_k w_k over the
    cache points whose valid region contains x', with w = 3d^2 - 2d^3,
    d = 1 - |x' - x_k| / R_k.  Returns (L [Q], covered [Q]).
    The membership test |x' - x_k| < R_k is taken in FP32 (see _within32);
    everything else is FP64.  With cache_form [K,6] (anisotropic points) the
    region is the ellipsoid (see _within_form32) and d = 1 - sqrt(q) with
    q = (x' - x_k)^T M_k (x' - x_k) in FP64: the normalised distance that is 1
    on the ellipsoid, as |x' - x_k| / R_k is on the sphere."""
    cp = np.asarray(cache_pos, np.float64)
    cv = np.asarray(cache_val, np.float64)
    cg = np.asarray(cache_grad, np.float64)
    cR = np.asarray(cache_R, np.float64)
    q = np.asarray(query, np.float64)
    q32, cp32, cR32 = (np.asarray(a, np.float32) for a in (query, cache_pos, cache_R))
    F = None if cache_form is None else np.asarray(cache_form, np.float32)
    out = np.zeros(len(q))
    cov = np.zeros(len(q), bool)
    for i, x in enumerate(q):
        dx = x[None, :] - cp
        if F is None:
            m = _within32(q32[i][None, :], cp32, cR32)
        else:
            m = _within_form32(q32[i][None, :], cp32, F)
        if not m.any():
            continue
        if F is None:
            dist = np.sqrt((dx * dx).sum(1))
            d = 1.0 - dist[m] / cR[m]
        else:
            f = F[m].astype(np.float64)
            e = dx[m]
            qf = ((f[:, 0] * e[:, 0] ** 2 + f[:, 3] * e[:, 1] ** 2 + f[:, 5] * e[:, 2] ** 2)
                  + 2 * (f[:, 1] * e[:, 0] * e[:, 1] + f[:, 2] * e[:, 0] * e[:, 2] + f[:, 4] * e[:, 1] * e[:, 2]))
            d = 1.0 - np.sqrt(np.maximum(qf, 0.0))
        w = 3 * d * d - 2 * d * d * d
        num = ((cv[m] + (cg[m] * dx[m]).sum(1)) * w).sum()
        den = w.sum()
        if den > 0:
            out[i] = num / den
            cov[i] = True
    return out, cov


def interpolate_log(cache_pos, cache_val, cache_grad, cache_R, query):
    """The comparison method's extrapolation (Eq. jaroszExtrapolation):
    L(x') = exp( sum_k [ln L_k + (grad L_k / L_k) . (x' - x_k)] w_k / sum_k w_k )
    over the cache points whose radius contains x' (FP32 test as in
    interpolate) with the same cubic weights; cache points with L_k <= 0 have
    no logarithm and take no part.  Returns (L [Q], covered [Q])."""
    cp = np.asarray(cache_pos, np.float64)
    cv = np.asarray(cache_val, np.float64)
    cg = np.asarray(cache_grad, np.float64)
    cR = np.asarray(cache_R, np.float64)
    q = np.asarray(query, np.float64)
    q32, cp32, cR32 = (np.asarray(a, np.float32) for a in (query, cache_pos, cache_R))
    out = np.zeros(len(q))
    cov = np.zeros(len(q), bool)
    for i, x in enumerate(q):
        m = _within32(q32[i][None, :], cp32, cR32) & (cv > 0)
        if not m.any():
            continue
        dx = x[None, :] - cp[m]
        d = 1.0 - np.sqrt((dx * dx).sum(1)) / cR[m]
        w = 3 * d * d - 2 * d * d * d
        lnL = np.log(cv[m]) + ((cg[m] / cv[m][:, None]) * dx).sum(1)
        den = w.sum()
        if den > 0:
            out[i] = np.exp((lnL * w).sum() / den)
            cov[i] = True
    return out, cov


# --------------------------------------------------------------------------
# Sec. 6 "Implementation" and Results in 3D: the render pass that consumes the
# cache (uniform ray marching of camera rays, step 0.1, 16 samples per pixel)
# --------------------------------------------------------------------------
def march(t_end, xi, step, sigma_s, sigma_t, orig, dirs):
    """Uniform ray marching of camera rays through the medium.  Ray r starts
    at orig[r] (inside the medium box) and ends at t_end[r] (its first surface
    hit, or where it leaves the box); its march points lie at
    t_k = (k + xi[r]) * step for k = 0, 1, 2, ... while t_k < t_end[r]
    (k + xi is exact in FP64, the product is rounded once).  A point's
    position is o + t_k d formed in FP64 and rounded once to FP32, and its
    weight is step * sigma_s * exp(-sigma_t * t_k): the midpoint-rule term of
    the in-scattering integral along the ray, attenuated by the transmittance
    from the eye, so that a pixel's medium radiance is the sum of
    weight * L_in over its points.  Points of a ray are enumerated one by one
    (brute force).  Returns (offsets int64 [N+1], points float32 [M][3],
    weights float64 [M])."""
    t_end = np.asarray(t_end, np.float32)
    xi = np.asarray(xi, np.float32)
    o = np.asarray(orig, np.float32).astype(np.float64)
    d = np.asarray(dirs, np.float32).astype(np.float64)
    step = float(step)
    offs = [0]
    pts, wts = [], []
    for r in range(len(t_end)):
        k = 0
        while True:
            t = (k + float(xi[r])) * step
            if not t < float(t_end[r]):
                break
            pts.append(o[r] + t * d[r])
            wts.append(step * sigma_s * np.exp(-sigma_t * t))
            k += 1
        offs.append(offs[-1] + k)
    P = np.asarray(pts, np.float64).reshape(-1, 3).astype(np.float32)
    return np.asarray(offs, np.int64), P, np.asarray(wts, np.float64)


def composite(offsets, spp, weights, L):
    """Pixel estimates of the render pass: pixel p averages its spp rays
    (rays p*spp .. p*spp + spp - 1), each ray contributing the sum of
    weight * L over its march points.  FP64.  Returns [N / spp]."""
    offsets = np.asarray(offsets, np.int64)
    w = np.asarray(weights, np.float64)
    L = np.asarray(L, np.float64)
    n_pix = (len(offsets) - 1) // spp
    out = np.zeros(n_pix)
    for p in range(n_pix):
        acc = 0.0
        for r in range(p * spp, (p + 1) * spp):
            a, b = offsets[r], offsets[r + 1]
            acc += float(np.dot(w[a:b], L[a:b]))
        out[p] = acc / spp
    return out


# --------------------------------------------------------------------------
# FP64 reference of the placement MLP (project-defined, not in the paper)
# --------------------------------------------------------------------------
def gelu(x):
    """tanh-form GELU (Hendrycks & Gimpel 2016)."""
    k = np.sqrt(2.0 / np.pi)
    return 0.5 * x * (1.0 + np.tanh(k * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    k = np.sqrt(2.0 / np.pi)
    u = k * (x + 0.044715 * x ** 3)
    t = np.tanh(u)
    du = k * (1.0 + 3 * 0.044715 * x * x)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * du


def mlp_forward(params, X):
    """params: dict W1 [128,32], b1 [128], W2 [128,128], b2, W3 [1,128], b3 [1]."""
    X = np.asarray(X, np.float64)
    z1 = X @ params["W1"].T + params["b1"]
    a1 = gelu(z1)
    z2 = a1 @ params["W2"].T + params["b2"]
    a2 = gelu(z2)
    y = a2 @ params["W3"].T + params["b3"]
    return y[:, 0], (X, z1, a1, z2, a2)


def mlp_loss_grad(params, X, target):
    """Mean squared error and its gradient w.r.t. every parameter (FP64)."""
    y, (X, z1, a1, z2, a2) = mlp_forward(params, X)
    B = X.shape[0]
    r = y - np.asarray(target, np.float64)
    loss = float((r * r).mean())
    dy = (2.0 / B) * r[:, None]
    g = {}
    g["W3"] = dy.T @ a2
    g["b3"] = dy.sum(0)
    da2 = dy @ params["W3"]
    dz2 = da2 * gelu_grad(z2)
    g["W2"] = dz2.T @ a1
    g["b2"] = dz2.sum(0)
    da1 = dz2 @ params["W2"]
    dz1 = da1 * gelu_grad(z1)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return loss, g


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba 2015), bias-corrected, one step; updates in place."""
    for k in params:
        m[k] = b1 * m[k] + (1 - b1) * grads[k]
        v[k] = b2 * v[k] + (1 - b2) * grads[k] ** 2
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params


def cpu_info():
    n = os.cpu_count() or 1
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": n, "model": model}
