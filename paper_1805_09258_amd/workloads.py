"""Seeded synthetic workloads for radiance-cache record computation.

This module only *generates inputs*: scene triangles, albedo/emission, the
medium box, point lights, medium coefficients, cache positions and per-record
stratum counts.  It holds none of the method's arithmetic (no sampling of
directions, no tracing, no form factors), so both the HIP path and the CPU
oracle can consume what it produces.

The paper's own scenes (Statues, Strips, Patio, Cornell Holes, Staircase,
Whiteroom; Sec. 6) are not available; these synthetic scenes stand in for
them.  They are shaped like the paper's occluder-rich interiors: a closed room
(walls, floor, ceiling), thin axis-aligned slabs standing in for window frames
and strips, and a soup of small triangles standing in for clutter.  The
participating medium is homogeneous and isotropic, as the paper restricts
itself to (Sec. 4, last paragraph before the error-control section).

All arrays are numpy; float32 for geometry and positions, int32 for counts.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload",
    "strata_shape",
    "room_triangles",
    "slab_triangles",
    "soup_triangles",
    "make_c1",
    "make_c2",
    "make_c3",
    "make_c4_scene",
    "make_c5",
    "make",
    "default_max_rings",
    "GridCandidates",
    "uniform_points",
]


@dataclass
class Workload:
    name: str
    tri: np.ndarray            # float32 [T, 9]  (v0, v1, v2)
    albedo: np.ndarray         # float32 [T]     Lambertian reflectance
    emission: np.ndarray       # float32 [T]     emitted radiance (two-sided)
    box_lo: np.ndarray         # float32 [3]     medium extent (axis-aligned box)
    box_hi: np.ndarray         # float32 [3]
    lights: np.ndarray         # float32 [L, 4]  (x, y, z, intensity)
    sigma_s: float
    sigma_a: float
    pos: np.ndarray            # float32 [P, 3]  cache positions
    n_theta: np.ndarray        # int32 [P]
    n_phi: np.ndarray          # int32 [P]
    ring_step: float
    max_rings: int
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def n_tri(self) -> int:
        return int(self.tri.shape[0])

    @property
    def n_rec(self) -> int:
        return int(self.pos.shape[0])

    def subset(self, idx) -> "Workload":
        idx = np.asarray(idx)
        return Workload(self.name + "[sub]", self.tri, self.albedo, self.emission, self.box_lo,
                        self.box_hi, self.lights, self.sigma_s, self.sigma_a,
                        np.ascontiguousarray(self.pos[idx]), np.ascontiguousarray(self.n_theta[idx]),
                        np.ascontiguousarray(self.n_phi[idx]), self.ring_step, self.max_rings,
                        self.seed, dict(self.meta, parent_index=idx))


def strata_shape(n: int) -> tuple[int, int]:
    """Split a requested direction count N into an (n_theta, n_phi) grid.

    n_theta = 2^floor(log2(N)/2 - 1/2), n_phi = round(N / n_theta): 64 -> 4x16,
    256 -> 8x32, 1024 -> 16x64, 2048 -> 32x64, 4096 -> 32x128.  The paper only
    says the sphere is split into equal-solid-angle strata (Sec. 6,
    Implementation); the grid shape is this project's choice.
    """
    n = int(n)
    if n < 16:
        raise ValueError("need at least 16 directions")
    nt = 2 ** int(math.floor(math.log2(n) / 2.0 - 0.5))
    nt = max(nt, 2)
    npf = int(round(n / nt))
    return nt, max(npf, 5)


def default_max_rings(box_lo, box_hi, ring_step: float) -> int:
    """Rings needed so that no direction is truncated: ceil(diag / step) + 1."""
    d = float(np.linalg.norm(np.asarray(box_hi, np.float64) - np.asarray(box_lo, np.float64)))
    return int(math.ceil(d / ring_step)) + 1


def _quad(a, b, c, d):
    # quad a-b-c-d (counter-clockwise) as two triangles
    return [np.concatenate([a, b, c]), np.concatenate([a, c, d])]


def room_triangles(lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)) -> np.ndarray:
    """12 triangles: the six faces of an axis-aligned box (normals inward)."""
    lo = np.asarray(lo, np.float32)
    hi = np.asarray(hi, np.float32)
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    P = lambda x, y, z: np.array([x, y, z], np.float32)  # noqa: E731
    tris = []
    tris += _quad(P(x0, y0, z0), P(x1, y0, z0), P(x1, y0, z1), P(x0, y0, z1))  # floor y=y0
    tris += _quad(P(x0, y1, z0), P(x0, y1, z1), P(x1, y1, z1), P(x1, y1, z0))  # ceiling y=y1
    tris += _quad(P(x0, y0, z0), P(x0, y0, z1), P(x0, y1, z1), P(x0, y1, z0))  # x=x0
    tris += _quad(P(x1, y0, z0), P(x1, y1, z0), P(x1, y1, z1), P(x1, y0, z1))  # x=x1
    tris += _quad(P(x0, y0, z0), P(x0, y1, z0), P(x1, y1, z0), P(x1, y0, z0))  # z=z0
    tris += _quad(P(x0, y0, z1), P(x1, y0, z1), P(x1, y1, z1), P(x0, y1, z1))  # z=z1
    return np.stack(tris).astype(np.float32)


def _box_tris(lo, hi) -> np.ndarray:
    return room_triangles(lo, hi)


def slab_triangles(rng: np.random.Generator, n_slabs: int, thickness=0.02,
                   extent=(0.2, 0.6), lo=0.0, hi=1.0):
    """Axis-aligned thin boxes (12 triangles each), fully inside [lo, hi]^3.

    Returns (triangles [12*n_slabs, 9], list of (box_lo, box_hi))."""
    tris, boxes = [], []
    for _ in range(n_slabs):
        thin = int(rng.integers(0, 3))
        size = np.empty(3)
        for ax in range(3):
            size[ax] = thickness if ax == thin else rng.uniform(extent[0], extent[1])
        c = np.array([rng.uniform(lo + s / 2 + 1e-3, hi - s / 2 - 1e-3) for s in size])
        blo = (c - size / 2).astype(np.float32)
        bhi = (c + size / 2).astype(np.float32)
        tris.append(_box_tris(blo, bhi))
        boxes.append((blo, bhi))
    if not tris:
        return np.zeros((0, 9), np.float32), boxes
    return np.concatenate(tris).astype(np.float32), boxes


def soup_triangles(rng: np.random.Generator, n: int, edge: float, lo=0.0, hi=1.0) -> np.ndarray:
    """Equilateral triangles with edge `edge`, centres uniform in the box shrunk
    by the circumradius (so every triangle lies inside), uniformly random
    orientation (random rotation of a reference triangle)."""
    if n == 0:
        return np.zeros((0, 9), np.float32)
    rc = edge / math.sqrt(3.0)  # circumradius
    margin = rc + 1e-4
    c = rng.uniform(lo + margin, hi - margin, size=(n, 3))
    # random rotations from normalised Gaussian quaternions
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    ref = np.array([[rc, 0, 0],
                    [rc * math.cos(2 * math.pi / 3), rc * math.sin(2 * math.pi / 3), 0],
                    [rc * math.cos(4 * math.pi / 3), rc * math.sin(4 * math.pi / 3), 0]])
    v = np.einsum("nij,kj->nki", R, ref) + c[:, None, :]
    return v.reshape(n, 9).astype(np.float32)


def _inside_any(p: np.ndarray, boxes, pad=0.0) -> np.ndarray:
    m = np.zeros(len(p), bool)
    for blo, bhi in boxes:
        m |= np.all((p >= blo - pad) & (p <= bhi + pad), axis=1)
    return m


def _points(rng, n, boxes=(), lo=0.0, hi=1.0):
    out = np.empty((0, 3))
    while len(out) < n:
        p = rng.uniform(lo, hi, size=(2 * (n - len(out)) + 16, 3))
        if boxes:
            p = p[~_inside_any(p, boxes, pad=1e-3)]
        out = np.concatenate([out, p])
    return out[:n].astype(np.float32)


def _c2_lights(intensity=2.5):
    return np.array([[x, 0.95, z, intensity] for x in (0.25, 0.75) for z in (0.25, 0.75)], np.float32)


def _fixed_strata(P, n):
    nt, npf = strata_shape(n)
    return np.full(P, nt, np.int32), np.full(P, npf, np.int32)


def make_c1(seed: int = 1, P: int = 64, n_dirs: int = 256) -> Workload:
    """FP64-checkable: 16 random triangles in the unit cube (no walls),
    sigma_s=0.5, sigma_a=0.1, one light I=10 at (0.5,0.95,0.5), 64 points,
    256 directions (8x32), ring step 0.1."""
    rng = np.random.default_rng(seed)
    tri = rng.uniform(0.0, 1.0, size=(16, 9)).astype(np.float32)
    T = tri.shape[0]
    lo = np.zeros(3, np.float32)
    hi = np.ones(3, np.float32)
    nt, npf = _fixed_strata(P, n_dirs)
    pos = rng.uniform(0.0, 1.0, size=(P, 3)).astype(np.float32)
    return Workload("C1", tri, np.full(T, 0.7, np.float32), np.zeros(T, np.float32), lo, hi,
                    np.array([[0.5, 0.95, 0.5, 10.0]], np.float32), 0.5, 0.1, pos, nt, npf,
                    0.1, default_max_rings(lo, hi, 0.1), seed)


def make_c2(seed: int = 2, P: int = 10_000, n_dirs: int = 1024, n_soup: int = 10_000) -> Workload:
    """Closed unit room (12 triangles) + 10k-triangle soup (edge 0.02),
    sigma_s=1.0, sigma_a=0.2, four lights I=2.5 at (0.25|0.75, 0.95, 0.25|0.75),
    points uniform in the room, 1024 directions (16x64), ring step 0.1."""
    rng = np.random.default_rng(seed)
    tri = np.concatenate([room_triangles(), soup_triangles(rng, n_soup, 0.02)])
    T = tri.shape[0]
    lo = np.zeros(3, np.float32)
    hi = np.ones(3, np.float32)
    pos = _points(rng, P)
    nt, npf = _fixed_strata(P, n_dirs)
    return Workload("C2", tri, np.full(T, 0.7, np.float32), np.zeros(T, np.float32), lo, hi,
                    _c2_lights(), 1.0, 0.2, pos, nt, npf, 0.1, default_max_rings(lo, hi, 0.1), seed)


def _slab_scene(rng, n_total: int):
    room = room_triangles()
    slabs, boxes = slab_triangles(rng, 20)
    n_soup = n_total - room.shape[0] - slabs.shape[0]
    # keep the soup's optical depth equal to the 10k-triangle, edge-0.02 soup
    edge = 0.02 * math.sqrt(1e4 / n_soup)
    soup = soup_triangles(rng, n_soup, edge)
    return np.concatenate([room, slabs, soup]).astype(np.float32), boxes, edge


def make_c3(seed: int = 3, P: int = 200_000, n_tri: int = 100_000,
            n_min: int = 256, n_max: int = 4096) -> Workload:
    """Batched: 100k triangles (room + 20 slabs + soup), 200k points with
    direction counts log-uniform in [256, 4096], medium and lights as C2."""
    rng = np.random.default_rng(seed)
    tri, boxes, edge = _slab_scene(rng, n_tri)
    T = tri.shape[0]
    lo = np.zeros(3, np.float32)
    hi = np.ones(3, np.float32)
    pos = _points(rng, P, boxes)
    n = np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=P))
    shapes = np.array([strata_shape(int(round(v))) for v in n], np.int32)
    return Workload("C3", tri, np.full(T, 0.7, np.float32), np.zeros(T, np.float32), lo, hi,
                    _c2_lights(), 1.0, 0.2, pos, np.ascontiguousarray(shapes[:, 0]),
                    np.ascontiguousarray(shapes[:, 1]), 0.1, default_max_rings(lo, hi, 0.1), seed,
                    {"soup_edge": edge, "slabs": boxes})


def make_c4_scene(seed: int, P: int = 10_000, n_dirs: int = 1024) -> Workload:
    """One scene of the C2 family (training uses seeds 1000..1099)."""
    w = make_c2(seed=seed, P=P, n_dirs=n_dirs)
    w.name = "C4-scene"
    return w


def make_c5(seed: int = 5, P: int = 1_000_000, n_tri: int = 1_000_000, n_dirs: int = 2048) -> Workload:
    """Large scene: 1M triangles (room + 20 slabs + soup), 1M points at 2048
    directions (32x64), sigma_s=2.0, sigma_a=0.5, lights as C2."""
    rng = np.random.default_rng(seed)
    tri, boxes, edge = _slab_scene(rng, n_tri)
    T = tri.shape[0]
    lo = np.zeros(3, np.float32)
    hi = np.ones(3, np.float32)
    pos = _points(rng, P, boxes)
    nt, npf = _fixed_strata(P, n_dirs)
    return Workload("C5", tri, np.full(T, 0.7, np.float32), np.zeros(T, np.float32), lo, hi,
                    _c2_lights(), 2.0, 0.5, pos, nt, npf, 0.1, default_max_rings(lo, hi, 0.1), seed,
                    {"soup_edge": edge, "slabs": boxes})


def make(name: str, **kw) -> Workload:
    return {"C1": make_c1, "C2": make_c2, "C3": make_c3, "C5": make_c5}[name.upper()](**kw)


class GridCandidates:
    """Candidate cache points for placement: one point per cell of an
    n x n x n grid over the medium box, jittered inside its cell (kept 1e-3
    of a cell away from the faces so FP32 rounding cannot move it out), and
    a seeded random visiting order.  Index (ix * n + iy) * n + iz."""

    def __init__(self, n: int, box_lo, box_hi, seed: int):
        rng = np.random.default_rng(seed)
        lo = np.asarray(box_lo, np.float64)
        hi = np.asarray(box_hi, np.float64)
        h = (hi - lo) / n
        ix, iy, iz = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        cell = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], 1).astype(np.float64)
        u = rng.uniform(1e-3, 1.0 - 1e-3, size=cell.shape)
        self.pos = (lo + (cell + u) * h).astype(np.float32)
        self.order = rng.permutation(n ** 3).astype(np.int32)
        self.dims = np.array([n, n, n], np.int32)
        self.lo = lo.astype(np.float32)
        self.cell = h.astype(np.float32)

    @property
    def n(self) -> int:
        return self.pos.shape[0]


def uniform_points(n: int, box_lo, box_hi, seed: int) -> np.ndarray:
    """n points uniform in the box (test points for cache error)."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(box_lo, np.float64)
    hi = np.asarray(box_hi, np.float64)
    return (lo + rng.uniform(0, 1, (n, 3)) * (hi - lo)).astype(np.float32)


class CameraRays:
    """Camera rays of a render pass: a pinhole camera at eye looking at
    look_at (vertical field of view fov_deg, square pixels), width x height
    pixels with spp jittered rays each, ordered pixel by pixel (ray
    p * spp + s is sample s of pixel p, pixels row-major from the top-left),
    and one uniform march offset xi per ray.  Directions are formed in FP64,
    normalised and rounded once to FP32; every random number is drawn here
    from the seed.  The eye must lie inside the medium box."""

    def __init__(self, width: int, height: int, spp: int, eye, look_at, fov_deg: float, seed: int,
                 up=(0.0, 1.0, 0.0), shuffle=False):
        rng = np.random.default_rng(seed)
        self.width, self.height, self.spp = int(width), int(height), int(spp)
        eye = np.asarray(eye, np.float64)
        fwd = np.asarray(look_at, np.float64) - eye
        fwd /= np.linalg.norm(fwd)
        right = np.cross(fwd, np.asarray(up, np.float64))
        right /= np.linalg.norm(right)
        upv = np.cross(right, fwd)
        th = np.tan(np.radians(fov_deg) / 2)
        n = self.width * self.height * self.spp
        pix = np.arange(n) // self.spp
        px = (pix % self.width).astype(np.float64)
        py = (pix // self.width).astype(np.float64)
        j = rng.uniform(0.0, 1.0, (n, 2))
        u = (2.0 * (px + j[:, 0]) / self.width - 1.0) * th * self.width / self.height
        v = (1.0 - 2.0 * (py + j[:, 1]) / self.height) * th
        d = fwd[None, :] + u[:, None] * right[None, :] + v[:, None] * upv[None, :]
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        self.dirs = d.astype(np.float32)
        self.orig = np.tile(eye.astype(np.float32)[None, :], (n, 1))
        self.xi = rng.uniform(0.0, 1.0, n).astype(np.float32)
        if shuffle:  # rays in a seeded random order (a uniform sampling of the camera's rays, not pixel order)
            perm = rng.permutation(n)
            self.dirs, self.orig, self.xi = self.dirs[perm], self.orig[perm], self.xi[perm]

    @property
    def n(self) -> int:
        return self.dirs.shape[0]

    @property
    def n_pixels(self) -> int:
        return self.width * self.height


def render_camera(width=128, height=128, spp=16, seed=8, shuffle=False):
    """The render-pass camera in the closed-room scenes: eye near the z = 0
    wall, looking at the far wall through the medium (60 degree field of
    view); shuffle: rays in a seeded random order."""
    return CameraRays(width, height, spp, eye=(0.5, 0.5, 0.04), look_at=(0.5, 0.5, 1.0), fov_deg=60.0, seed=seed,
                      shuffle=shuffle)
