"""The render pass that consumes the radiance cache (Sec. 6 "Implementation";
Results in 3D: 16 samples per pixel, uniform ray marching with step 0.1).

1. Pre-population: camera rays (one per pixel, visited in a random order:
   a uniform sampling of the camera's rays) are marched through the medium
   and their march points are the candidates of a plain greedy placement
   (the error-metric insertion rule of Sec. 5 and 6).
2. Render: every sample ray is marched; at each march point, in camera
   order, the cache either holds a valid point (the radius test of
   Eq. radiusAniso3D) or a record is computed there and inserted.  This is
   the same greedy rule continued over the render points with the
   pre-populated cache already in place, so it runs as further plain rounds.
3. The in-scattered radiance at every march point is interpolated from the
   final cache (Eq. radianceTaylor) and the pixels are composited.

With CacheConfig(method="j08") the same pass runs the paper's comparison
method: its records and gradient-norm radii place the cache, and the march
points read it in log space.

Every step runs in the library's kernels (rc.*); this module sequences the
calls and holds device buffers.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

from . import rc
from . import workloads as W
from .placement import CacheConfig, PlacementResult, Placer, SceneContext


@dataclass
class MarchCandidates:
    """Candidates of a placement that are march points (device float[C][3],
    visited in index order, no grid)."""
    pos: object
    order: object = None
    dims: object = None

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


@dataclass
class Marched:
    offsets: object   # device int64 [N + 1]
    points: object    # device float32 [M][3]
    weight: object    # device float64 [M]
    t_end: object     # device float32 [N]

    @property
    def n_points(self) -> int:
        return int(self.points.shape[0])


def march(ctx: SceneContext, cam: W.CameraRays, step: float, device) -> Marched:
    """The march points of a camera's rays (rc_march_count, rc_march_emit)."""
    import torch
    w = ctx.w
    T = lambda a: torch.as_tensor(a, device=device)  # noqa: E731
    o, d, xi = T(cam.orig), T(cam.dirs), T(cam.xi)
    N = cam.n
    t_end = torch.empty(N, dtype=torch.float32, device=device)
    offs = torch.empty(N + 1, dtype=torch.int64, device=device)
    rc.rc_march_count(ctx.scene.handle, o, d, xi, step, t_end, offs)
    M = int(offs[-1].item())
    pts = torch.empty((M, 3), dtype=torch.float32, device=device)
    wt = torch.empty(M, dtype=torch.float64, device=device)
    rc.rc_march_emit(o, d, xi, step, w.sigma_s, w.sigma_s + w.sigma_a, offs, pts, wt)
    return Marched(offs, pts, wt, t_end)


def _empty_cache(device):
    import torch
    z = lambda *shape, dt=torch.float32: torch.zeros(shape, dtype=dt, device=device)  # noqa: E731
    return PlacementResult(z(0, 3), z(0, 2, dt=torch.float64), z(0, 2, 3, dt=torch.float64), z(0), 0,
                           {"records": 0, "rounds": 0})


def _empty_render(cam, prepop, m0, m1, res0, device, t0, t1, ev):
    """The render of rays with no march points and no cache: zero pixels."""
    import torch
    pix = torch.zeros(cam.n_pixels, dtype=torch.float64, device=device)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    stats = {"rays": cam.n, "march_points": 0, "prepop_rays": prepop.n, "prepop_points": m0.n_points,
             "prepop_records": 0, "prepop_cache": 0, "prepop_rounds": 0, "render_records": 0, "render_rounds": 0,
             "cache_points": 0, "inserted": 0, "uncovered_after": 0, "seconds_prepop": t1 - t0,
             "seconds_render": t2 - t1, "pixel_mean": 0.0, "march_points_per_s": 0.0, "ms": {}}
    z = torch.zeros(0, dtype=torch.float64, device=device)
    return pix, stats, (m1, res0, z, torch.zeros(0, dtype=torch.int32, device=device), None, None)


def render(ctx: SceneContext, cam: W.CameraRays, prepop: W.CameraRays, cfg: CacheConfig, device, step=0.1,
           batch=None, prepop_batch=None):
    """Pre-populate a cache from prepop's rays (in their order; rounds of
    prepop_batch candidates), render cam's rays through it (inserting records
    where the cache has no valid point; rounds of batch), and composite.
    Batch sizes default to cfg.batch.  Returns (pixels [n_pixels] device
    float64, stats, device buffers)."""
    import torch
    ev = []

    def mark(name):
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        ev.append((name, e))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mark("start")
    m0 = march(ctx, prepop, step, device)
    mark("march_prepop")
    if m0.n_points:
        pre = Placer(ctx, MarchCandidates(m0.points), cfg, device)
        res0 = pre.plain(prepop_batch if prepop_batch is not None else batch)
    else:  # no pre-population: the render inserts every cache point
        res0 = _empty_cache(device)
    K0 = res0.K
    mark("place_prepop")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # render: the candidates are the cache's K0 points followed by the render
    # march points; the cache entries are in place (accepted, covered) and
    # cover the render points before the rounds continue from candidate K0
    mark("render_start")
    m1 = march(ctx, cam, step, device)
    mark("march_render")
    cand = torch.cat([res0.pos, m1.points])
    if cand.shape[0] == 0:  # nothing cached and no march points
        return _empty_render(cam, prepop, m0, m1, res0, device, t0, t1, ev)
    pl = Placer(ctx, MarchCandidates(cand), cfg, device)
    pl.covered[:K0] = 1
    pl.acc[:K0] = torch.arange(K0, dtype=torch.int32, device=device)
    pl.accR[:K0] = res0.R
    pl.accpos[:K0] = res0.pos
    pl.cval[:K0] = res0.value
    pl.cgrad[:K0] = res0.grad
    pl.state[0] = K0   # gather cursor
    pl.state[1] = K0   # cache size
    if K0:
        rc.rc_place_cover(pl.cand, pl.covered, None, pl.acc, pl.accR, 0, K0)
    rounds, records = pl._plain_rounds(batch)
    mark("insert_misses")
    res = pl._result({})
    # radiance at every march point from the final cache, and the pixels
    M = m1.n_points
    L = torch.zeros(M, dtype=torch.float64, device=device)
    hits = torch.zeros(M, dtype=torch.int32, device=device)
    if cfg.method == "j08":  # the comparison method reads its cache in log space (Eq. jaroszExtrapolation)
        rc.rc_interp_log(res.pos, res.value, res.grad, res.R, m1.points, L, hits)
    else:
        rc.rc_interp(res.pos, res.value, res.grad, res.R, m1.points, L, hits)
    mark("interpolate")
    pix = torch.empty(cam.n_pixels, dtype=torch.float64, device=device)
    rc.rc_composite(m1.offsets, cam.spp, m1.weight, L, pix)
    mark("composite")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    uncovered = int((hits == 0).sum().item())
    stats = {"rays": cam.n, "march_points": M, "prepop_rays": prepop.n, "prepop_points": m0.n_points,
             "prepop_records": res0.stats["records"], "prepop_cache": K0, "prepop_rounds": res0.stats["rounds"],
             "render_records": records, "render_rounds": rounds, "cache_points": res.K,
             "inserted": res.K - K0, "uncovered_after": uncovered,
             "seconds_prepop": t1 - t0, "seconds_render": t2 - t1,
             "pixel_mean": float(pix.mean().item()) if cam.n_pixels else 0.0}
    stats["march_points_per_s"] = M / stats["seconds_render"] if stats["seconds_render"] > 0 else 0.0
    # milliseconds of device time between consecutive marks (host waits included)
    stats["ms"] = {n: ev[i - 1][1].elapsed_time(e) for i, (n, e) in enumerate(ev) if i > 0 and n != "render_start"}
    return pix, stats, (m1, res, L, hits, cand, pl)
