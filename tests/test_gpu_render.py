"""The render pass (Sec. 6 "Implementation"; Results in 3D) on the GPU
against the oracle, through the C ABI.

March counts, offsets and positions are compared bit for bit (both sides form
them in FP64 from the same FP32 inputs and the same closest hits); weights to
1e-15 relative (the FP64 exponential of two math libraries); pixels to 1e-12
relative (FP64 sums in another order).  The end-to-end pass is checked against
the sequential insertion rule it implements: the cache it ends with is the one
that visiting the march points in camera order and inserting a point at every
one no earlier point covers produces.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1805_09258_amd import rc  # noqa: E402
from paper_1805_09258_amd import render as RD  # noqa: E402
from paper_1805_09258_amd import workloads as W  # noqa: E402
from paper_1805_09258_amd.placement import CacheConfig, SceneContext  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _rays(rng, n, cam_seed=5):
    """Camera rays of a small image plus rays from random points inside the
    room in random directions, with offsets including 0 and values next to 1."""
    cam = W.CameraRays(16, 8, 4, eye=(0.5, 0.5, 0.04), look_at=(0.5, 0.5, 1.0), fov_deg=60.0, seed=cam_seed)
    m = max(n - cam.n, 0)
    o = rng.uniform(0.05, 0.95, (m, 3)).astype(np.float32)
    d = rng.normal(size=(m, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    o = np.concatenate([cam.orig, o])[:n]
    d = np.concatenate([cam.dirs, d])[:n]
    xi = rng.uniform(0, 1, n).astype(np.float32)
    xi[::7] = 0.0
    xi[3::11] = np.nextafter(np.float32(1), np.float32(0))
    return np.ascontiguousarray(o), np.ascontiguousarray(d), xi


def _march_gpu(sc, o, d, xi, step, ss, st, dev):
    T = lambda a: torch.as_tensor(a, device=dev)  # noqa: E731
    n = o.shape[0]
    t = torch.full((n,), -1.0, dtype=torch.float32, device=dev)
    offs = torch.full((n + 1,), -1, dtype=torch.int64, device=dev)
    to, td, tx = T(o), T(d), T(xi)
    rc.rc_march_count(sc.handle, to, td, tx, step, t, offs)
    M = int(offs[-1].item())
    pts = torch.empty((M, 3), dtype=torch.float32, device=dev)
    wt = torch.empty(M, dtype=torch.float64, device=dev)
    rc.rc_march_emit(to, td, tx, step, ss, st, offs, pts, wt)
    torch.cuda.synchronize()
    return offs.cpu().numpy(), pts.cpu().numpy(), wt.cpu().numpy(), t.cpu().numpy()


@pytest.mark.parametrize("n,step", [(1, 0.1), (63, 0.1), (2 * 8192 + 37, 0.1), (3000, 0.013)])
def test_march_equals_oracle_bit_for_bit(dev, n, step):
    rng = np.random.default_rng(n)
    w = W.make_c2(seed=21, P=1, n_soup=2000)
    o, d, xi = _rays(rng, n)
    sc = rc.Scene.from_workload(w)
    ss, st = w.sigma_s, w.sigma_s + w.sigma_a
    offs, pts, wt, t = _march_gpu(sc, o, d, xi, step, ss, st, dev)
    sc.close()
    _, ot, _ = O.Scene.from_workload(w).trace(o, d, brute=True)
    assert np.array_equal(t.view(np.int32), ot.view(np.int32))
    oo, op, ow = O.march(ot, xi, step, ss, st, o, d)
    _say(f"march n={n} step={step}: {oo[-1]} points")
    assert np.array_equal(offs, oo)
    assert np.array_equal(pts.view(np.int32), op.view(np.int32))
    np.testing.assert_allclose(wt, ow, rtol=1e-15, atol=0)


def test_march_of_no_rays_and_composite_of_empty_rays(dev):
    w = W.make_c2(seed=21, P=1, n_soup=200)
    sc = rc.Scene.from_workload(w)
    z3 = np.zeros((0, 3), np.float32)
    offs, pts, wt, t = _march_gpu(sc, z3, z3, np.zeros(0, np.float32), 0.1, 1.0, 1.2, dev)
    assert offs.tolist() == [0] and pts.shape == (0, 3)
    # a step too small for the box is refused before any launch
    with pytest.raises(rc.RCError):
        _march_gpu(sc, np.full((4, 3), 0.5, np.float32), np.tile(np.float32([[0, 0, 1]]), (4, 1)),
                   np.zeros(4, np.float32), 1e-7, 1.0, 1.2, dev)
    # rays with no points (offsets equal) give zero pixels
    o = torch.zeros(9, dtype=torch.int64, device=dev)
    pix = torch.full((4,), float("nan"), dtype=torch.float64, device=dev)
    rc.rc_composite(o, 2, None, None, pix)
    torch.cuda.synchronize()
    assert pix.cpu().numpy().tolist() == [0.0] * 4
    sc.close()


@pytest.mark.parametrize("spp", [1, 3, 4, 16, 300])
def test_composite_equals_oracle(dev, spp):
    rng = np.random.default_rng(40 + spp)
    w = W.make_c2(seed=22, P=1, n_soup=2000)
    n = spp * 777
    o, d, xi = _rays(rng, n)
    sc = rc.Scene.from_workload(w)
    offs, pts, wt, t = _march_gpu(sc, o, d, xi, 0.1, w.sigma_s, w.sigma_s + w.sigma_a, dev)
    sc.close()
    L = rng.uniform(0, 3, offs[-1])
    T = lambda a: torch.as_tensor(a, device=dev)  # noqa: E731
    pix = torch.empty(n // spp, dtype=torch.float64, device=dev)
    rc.rc_composite(T(offs), spp, T(wt), T(L), pix)
    torch.cuda.synchronize()
    ref = O.composite(offs, spp, wt, L)
    np.testing.assert_allclose(pix.cpu().numpy(), ref, rtol=1e-12, atol=1e-300)


def _within32(q, p, R):
    d = q.astype(np.float32) - p.astype(np.float32)
    d2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
    return d2 < R.astype(np.float32) * R.astype(np.float32)


def _check_insertion_rule(cand, acc, R, K0):
    """acc: candidate indices of the cache in insertion order (the first K0
    pre-populated, at candidates 0..K0-1); R their radii.  Every inserted
    point lies in no earlier point's ball; every render candidate lies in the
    ball of a point inserted no later than itself."""
    assert np.array_equal(acc[:K0], np.arange(K0))
    ins = acc[K0:]
    assert (np.diff(ins) > 0).all() and (ins >= K0).all()
    P = cand[acc]
    for j in range(K0, len(acc)):
        assert not _within32(cand[acc[j]][None], P[:j], R[:j]).any(), f"inserted point {j} was covered"
    C = cand.shape[0]
    ok = np.zeros(C, bool)
    first = np.full(C, np.iinfo(np.int64).max)
    for j in range(len(acc)):
        m = _within32(cand, P[j][None], np.float32(R[j])) | (np.arange(C) == acc[j])
        first = np.where(m & ~ok, acc[j], first)
        ok |= m
    assert ok[K0:].all(), "a render point is not covered"
    assert (first[K0:] <= np.arange(K0, C)).all(), "a render point is covered only by a later insertion"


def test_render_pass_follows_the_sequential_insertion_rule(dev):
    w = W.make_c2(seed=31, P=1, n_soup=2000)
    ctx = SceneContext(w)
    cfg = CacheConfig(n_theta=8, n_phi=32, batch=1024)
    cam = W.CameraRays(24, 16, 4, eye=(0.5, 0.5, 0.04), look_at=(0.5, 0.5, 1.0), fov_deg=60.0, seed=3)
    pre = W.CameraRays(24, 16, 1, eye=(0.5, 0.5, 0.04), look_at=(0.5, 0.5, 1.0), fov_deg=60.0, seed=4)
    pix, st, (m1, res, L, hits, cand, pl) = RD.render(ctx, cam, pre, cfg, dev, batch=256)
    _say("render", st)
    assert st["uncovered_after"] == 0 and st["inserted"] > 0 and st["prepop_cache"] > 0
    assert (hits > 0).all()
    K, K0 = res.K, st["prepop_cache"]
    acc = pl.acc[:K].cpu().numpy().astype(np.int64)
    _check_insertion_rule(cand.cpu().numpy(), acc, res.R.cpu().numpy(), K0)
    # the pixels are the composite of the interpolated radiance
    ref = O.composite(m1.offsets.cpu().numpy(), cam.spp, m1.weight.cpu().numpy(), L.cpu().numpy())
    np.testing.assert_allclose(pix.cpu().numpy(), ref, rtol=1e-12)
    assert np.isfinite(pix.cpu().numpy()).all() and pix.mean().item() > 0
    # deterministic: a second pass gives the same pixels, bit for bit
    pix2, st2, _ = RD.render(ctx, cam, pre, cfg, dev, batch=256)
    assert np.array_equal(pix.cpu().numpy(), pix2.cpu().numpy()) and st2["cache_points"] == st["cache_points"]
    ctx.close()


def test_render_pass_at_full_size_sampled(dev):
    """The 128 x 128 x 16 render of the closed-room scene as the benchmark
    runs it: march points of a seeded 1 % sample of the rays equal the
    oracle's bit for bit (the oracle traces each sampled ray itself), and
    every march point ends covered."""
    w = W.make_c2(P=1)
    ctx = SceneContext(w)
    cam = W.render_camera()
    pre = W.render_camera(spp=1, seed=9, shuffle=True)
    pix, st, (m1, res, L, hits, cand, pl) = RD.render(ctx, cam, pre, CacheConfig(), dev, prepop_batch=512)
    _say("full-size render", st)
    assert st["uncovered_after"] == 0 and (hits > 0).all()
    rng = np.random.default_rng(77)
    idx = np.sort(rng.choice(cam.n, cam.n // 100, replace=False))
    o, d, xi = cam.orig[idx], cam.dirs[idx], cam.xi[idx]
    _, ot, _ = O.Scene.from_workload(w).trace(o, d)
    offs = m1.offsets.cpu().numpy()
    assert np.array_equal(m1.t_end.cpu().numpy()[idx].view(np.int32), ot.view(np.int32))
    oo, op, ow = O.march(ot, xi, 0.1, w.sigma_s, w.sigma_s + w.sigma_a, o, d)
    pts, wt = m1.points.cpu().numpy(), m1.weight.cpu().numpy()
    sel = np.concatenate([np.arange(offs[i], offs[i + 1]) for i in idx])
    assert np.array_equal(np.diff(oo), (offs[idx + 1] - offs[idx]))
    assert np.array_equal(pts[sel].view(np.int32), op.view(np.int32))
    np.testing.assert_allclose(wt[sel], ow, rtol=1e-15, atol=0)
    ctx.close()


def test_interpolation_of_march_points_matches_oracle(dev):
    """Queries that are march points (consecutive queries close together, so
    a workgroup skips most cache balls) and queries just inside and just
    outside ball boundaries: the same members, counts and radiance as the
    oracle's visit of every cache point."""
    rng = np.random.default_rng(91)
    w = W.make_c2(seed=23, P=1, n_soup=2000)
    o, d, xi = _rays(rng, 512)
    sc = rc.Scene.from_workload(w)
    offs, pts, wt, t = _march_gpu(sc, o, d, xi, 0.1, w.sigma_s, w.sigma_s + w.sigma_a, dev)
    sc.close()
    K = 700
    cp = rng.uniform(0, 1, (K, 3)).astype(np.float32)
    cR = np.exp(rng.uniform(np.log(0.01), np.log(0.15), K)).astype(np.float32)
    cv = rng.uniform(0, 2, (K, 2))
    cg = rng.normal(size=(K, 2, 3))
    u = rng.normal(size=(600, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    j = rng.integers(0, K, 600)
    s = np.where(np.arange(600) % 2 == 0, 1 - 3e-7, 1 + 3e-7)
    edge = (cp[j].astype(np.float64) + (s * cR[j])[:, None] * u).astype(np.float32)
    q = np.ascontiguousarray(np.concatenate([pts, edge]))
    Q = q.shape[0]
    T = lambda a: torch.as_tensor(a, device=dev)  # noqa: E731
    out = torch.full((Q,), float("nan"), dtype=torch.float64, device=dev)
    hits = torch.zeros(Q, dtype=torch.int32, device=dev)
    rc.rc_interp(T(cp), T(cv), T(cg), T(cR), T(q), out, hits)
    torch.cuda.synchronize()
    L, cov = O.interpolate(cp, cv.sum(1), cg.sum(1), cR, q)
    members = np.array([O._within32(q[i][None], cp, cR).sum() for i in range(Q)])
    _say(f"interp: {Q} queries ({pts.shape[0]} march points), {cov.sum()} covered, mean members {members.mean():.1f}")
    np.testing.assert_array_equal(hits.cpu().numpy(), np.where(cov, members, 0))
    np.testing.assert_allclose(out.cpu().numpy(), L, rtol=1e-6, atol=1e-6)


def test_render_pass_without_prepopulation_and_without_rays(dev):
    """No pre-population rays: every cache point is inserted at render time,
    under the same rule; no render rays: no pixels and nothing placed."""
    w = W.make_c2(seed=32, P=1, n_soup=2000)
    ctx = SceneContext(w)
    cfg = CacheConfig(n_theta=8, n_phi=32, batch=512)
    cam = W.CameraRays(12, 8, 2, eye=(0.5, 0.5, 0.04), look_at=(0.5, 0.5, 1.0), fov_deg=60.0, seed=6)
    none = W.CameraRays(0, 1, 1, eye=(0.5, 0.5, 0.04), look_at=(0.5, 0.5, 1.0), fov_deg=60.0, seed=7)
    assert none.n == 0
    pix, st, (m1, res, L, hits, cand, pl) = RD.render(ctx, cam, none, cfg, dev)
    _say("render without pre-population", st)
    assert st["prepop_cache"] == 0 and st["cache_points"] == st["inserted"] > 0 and st["uncovered_after"] == 0
    _check_insertion_rule(cand.cpu().numpy(), pl.acc[:res.K].cpu().numpy().astype(np.int64), res.R.cpu().numpy(), 0)
    pix0, st0, _ = RD.render(ctx, none, none, cfg, dev)
    assert pix0.shape[0] == 0 and st0["cache_points"] == 0 and st0["march_points"] == 0
    ctx.close()


def test_render_pass_of_the_comparison_method(dev):
    """The same pass with the comparison method's records, radii and
    log-space reads: the insertion rule holds, every march point is read
    from a valid cache point, and the pixels are finite and positive on
    average."""
    w = W.make_c2(seed=33, P=1, n_soup=2000)
    ctx = SceneContext(w)
    cfg = CacheConfig(n_theta=8, n_phi=32, batch=256, method="j08", j08_eps=0.7)
    cam = W.CameraRays(16, 12, 2, eye=(0.5, 0.5, 0.04), look_at=(0.5, 0.5, 1.0), fov_deg=60.0, seed=12)
    pre = W.CameraRays(16, 12, 1, eye=(0.5, 0.5, 0.04), look_at=(0.5, 0.5, 1.0), fov_deg=60.0, seed=13, shuffle=True)
    pix, st, (m1, res, L, hits, cand, pl) = RD.render(ctx, cam, pre, cfg, dev)
    _say("comparison-method render", st)
    assert res.log_space and st["uncovered_after"] == 0 and (hits > 0).all()
    _check_insertion_rule(cand.cpu().numpy(), pl.acc[:res.K].cpu().numpy().astype(np.int64), res.R.cpu().numpy(),
                          st["prepop_cache"])
    p = pix.cpu().numpy()
    assert np.isfinite(p).all() and p.mean() > 0
    ctx.close()
