"""GPU (HIP, gfx950) records against the FP64 CPU oracle, through the C ABI.

Both sides draw the same sample directions from the same counter-based
generator and take the same FP32 discrete decisions, so records are compared
element by element: value to 1e-4, gradient to 1e-3 and Hessian (Frobenius)
to 5e-3 relative error, with the cancellation floor described in _compare.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1805_09258_amd import rc  # noqa: E402
from paper_1805_09258_amd import workloads as W  # noqa: E402
from tests._compare import assert_parity, rel_errors  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def gpu_records(w, batched=False, use_graph=False, precision=0, counters=None, stream=None):
    sc = rc.Scene.from_workload(w)
    dw = rc.DeviceWorkload(w)
    v, g, h, ws = rc.compute_records(sc, dw, batched=batched, use_graph=use_graph, precision=precision,
                                     counters=counters, stream=stream)
    torch.cuda.synchronize()
    errs = rc.rc_workspace_errors(ws)
    out = (v.cpu().numpy(), g.cpu().numpy(), h.cpu().numpy())
    sc.close()
    return out, errs


def test_ray_queries_equal_oracle_brute_force(dev):
    w = W.make_c2(P=4, n_soup=3000)
    _say("rays: C2-like scene", w.n_tri, "triangles")
    sc = rc.Scene.from_workload(w)
    osc = O.Scene.from_workload(w)
    rng = np.random.default_rng(8)
    n = 20000
    o = rng.uniform(0.01, 0.99, size=(n, 3)).astype(np.float32)
    d = rng.normal(size=(n, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    to = torch.as_tensor(o, device=dev)
    td = torch.as_tensor(d, device=dev)
    hid = torch.empty(n, dtype=torch.int32, device=dev)
    tt = torch.empty(n, dtype=torch.float32, device=dev)
    fr = torch.empty(n, dtype=torch.int32, device=dev)
    rc.rc_trace_rays(sc.handle, to, td, hid, tt, fr)
    torch.cuda.synchronize()
    ohid, ot, ofr = osc.trace(o, d, brute=True)
    assert np.array_equal(hid.cpu().numpy(), ohid.astype(np.int32))
    assert np.array_equal(tt.cpu().numpy().view(np.int32), ot.view(np.int32))      # bitwise
    assert np.array_equal(fr.cpu().numpy()[ohid >= 0], ofr[ohid >= 0])
    # shadow segments from the hit points to random targets
    hit = ohid >= 0
    y = (o + ot[:, None] * d).astype(np.float32)
    seg = (rng.uniform(0, 1, size=(n, 3)).astype(np.float32) - y).astype(np.float32)
    skip = np.where(hit, ohid, -1).astype(np.int32)
    occ = torch.empty(n, dtype=torch.int32, device=dev)
    rc.rc_occluded_rays(sc.handle, torch.as_tensor(y, device=dev), torch.as_tensor(seg, device=dev),
                        torch.as_tensor(skip, device=dev), occ)
    torch.cuda.synchronize()
    oocc = osc.occluded(y, seg, skip.astype(np.int64), brute=True)
    assert np.array_equal(occ.cpu().numpy().astype(bool), oocc)
    sc.close()


def test_light_bin_segments_equal_oracle_brute_force(dev):
    """Shadow segments y -> light answered from the per-light bins on the GPU
    equal the oracle's brute-force answers, for random points and for points
    whose segments skim triangle edges, run along cube-face boundaries seen
    from the light or start next to it."""
    from tests.test_abi_host import _adversarial_points
    w = W.make_c2(P=4, n_soup=3000, seed=17)
    sc = rc.Scene.from_workload(w)
    osc = O.Scene.from_workload(w)
    rc.rc_light_bins_build(sc.handle, w.lights)
    rng = np.random.default_rng(9)
    for li in range(len(w.lights)):
        L = w.lights[li, :3].astype(np.float32)
        pts = np.concatenate([rng.uniform(w.box_lo, w.box_hi, (250000, 3)),
                              _adversarial_points(w.tri, L.astype(np.float64), rng, 20000)]).astype(np.float32)
        pts = pts[np.all((pts > w.box_lo) & (pts < w.box_hi), axis=1)]
        skip = np.where(rng.uniform(size=len(pts)) < 0.3, rng.integers(0, w.n_tri, len(pts)), -1).astype(np.int32)
        occ = torch.empty(len(pts), dtype=torch.int32, device=dev)
        _say(f"light {li}: {len(pts)} segments")
        rc.rc_light_occluded(sc.handle, li, torch.as_tensor(pts, device=dev), torch.as_tensor(skip, device=dev), occ)
        torch.cuda.synchronize()
        # the oracle's hierarchy answers as brute force does (pinned by the oracle tests)
        ref = osc.occluded(pts, (L[None, :] - pts).astype(np.float32), skip=skip.astype(np.int64))
        got = occ.cpu().numpy().astype(bool)
        assert np.array_equal(got, ref), (li, int((got != ref).sum()))
        assert 0.05 < ref.mean() < 0.95
        # the same light at another position of the light set answers the same
        rc.rc_light_bins_build(sc.handle, w.lights[::-1].copy())
        occ2 = torch.empty_like(occ)
        rc.rc_light_occluded(sc.handle, len(w.lights) - 1 - li, torch.as_tensor(pts, device=dev),
                             torch.as_tensor(skip, device=dev), occ2)
        torch.cuda.synchronize()
        assert torch.equal(occ, occ2), li
        rc.rc_light_bins_build(sc.handle, w.lights)
    sc.close()


def test_light_bin_and_bvh_shadows_give_identical_records(dev):
    """Records whose shadow segments come from the light bins equal, bit for
    bit, records whose shadow segments traverse the BVH."""
    w = W.make_c2(P=300, n_soup=4000, seed=18)
    sc = rc.Scene.from_workload(w)
    dw = rc.DeviceWorkload(w)
    out = []
    for bvh in (False, True):
        # records traced in the kernel, so both runs share one LDS layout (the
        # summation order of a record depends on its row width)
        v, g, h, ws = rc.compute_records(sc, dw, batched=True, shadow_bvh=bvh, hits_pass=False)
        torch.cuda.synchronize()
        assert rc.rc_workspace_errors(ws) == 0
        out.append((v.clone(), g.clone(), h.clone()))
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a, b)
    sc.close()


def test_c1_all_records_match_oracle(dev):
    w = W.make_c1()
    _say("C1: 64 records x 256 directions, 16 triangles")
    cnt = torch.zeros(12, dtype=torch.int64, device=dev)
    (v, g, h), errs = gpu_records(w, counters=cnt)
    assert errs == 0
    ref = O.records_for(w)
    assert_parity(v, g, h, ref, "C1")
    # identical discrete decisions: the traced-ray count matches exactly
    assert int(cnt[0].item()) == int(ref["stats"][:, 0].sum())
    assert int(cnt[3].item()) == int(ref["stats"][:, 1].sum() + ref["stats"][:, 2].sum())


@pytest.mark.parametrize("splits", [1, 2, 3, 8])
def test_records_split_over_wavefronts_match_oracle(dev, splits):
    """A record's strata rows split over several wavefronts (each recomputing
    its boundary row) give the oracle's record, with the same traced rays and
    terms, and agree with the unsplit record to FP64 rounding."""
    w = W.make_c1(P=40)
    sc = rc.Scene.from_workload(w)
    dw = rc.DeviceWorkload(w)
    cnt = torch.zeros(12, dtype=torch.int64, device=dev)
    v, g, h, ws = rc.compute_records(sc, dw, batched=True, counters=cnt, splits=splits)
    v1, g1, h1, _ = rc.compute_records(sc, dw, batched=True, splits=1)
    torch.cuda.synchronize()
    assert rc.rc_workspace_errors(ws) == 0
    ref = O.records_for(w)
    a = (v.cpu().numpy(), g.cpu().numpy(), h.cpu().numpy())
    assert_parity(*a, ref, f"C1, {splits} parts")
    assert int(cnt[0].item()) == int(ref["stats"][:, 0].sum())
    assert int(cnt[3].item()) == int(ref["stats"][:, 1].sum() + ref["stats"][:, 2].sum())
    for x, y in zip(a, (v1.cpu().numpy(), g1.cpu().numpy(), h1.cpu().numpy())):
        np.testing.assert_allclose(x, y, rtol=1e-12, atol=1e-12 * np.abs(y).max())
    sc.close()


@pytest.mark.parametrize("nth,nph,splits", [(4, 100, 1), (3, 129, 1), (2, 256, 1), (6, 100, 3)])
def test_wide_rows_done_in_column_sectors_match_oracle(dev, nth, nph, splits):
    """Rows wider than 64 columns are traced and triangulated in sectors of 64
    columns (plus the next sector's first); records, ray and term counts equal
    the oracle's, also combined with row parts."""
    w = W.make_c1(P=24)
    w.n_theta = np.full(w.n_rec, nth, np.int32)
    w.n_phi = np.full(w.n_rec, nph, np.int32)
    sc = rc.Scene.from_workload(w)
    dw = rc.DeviceWorkload(w)
    cnt = torch.zeros(12, dtype=torch.int64, device=dev)
    v, g, h, ws = rc.compute_records(sc, dw, batched=True, counters=cnt, splits=splits)
    torch.cuda.synchronize()
    assert rc.rc_workspace_errors(ws) == 0
    ref = O.records_for(w)
    assert_parity(v.cpu().numpy(), g.cpu().numpy(), h.cpu().numpy(), ref, f"{nth}x{nph}, {splits} parts")
    assert int(cnt[0].item()) == int(ref["stats"][:, 0].sum())
    assert int(cnt[3].item()) == int(ref["stats"][:, 1].sum() + ref["stats"][:, 2].sum())
    sc.close()


def test_small_batches_split_automatically_on_the_c2_scene(dev):
    w = W.make_c2().subset(np.arange(37))
    sc = rc.Scene.from_workload(w)
    dw = rc.DeviceWorkload(w)
    v, g, h, ws = rc.compute_records(sc, dw, batched=True, use_graph=False)
    torch.cuda.synchronize()
    assert rc.rc_workspace_errors(ws) == 0
    idx = np.arange(0, 37, 3)
    ref = O.records_for(w, idx)
    assert_parity(v.cpu().numpy()[idx], g.cpu().numpy()[idx], h.cpu().numpy()[idx], ref, "C2 scene, 37 records")
    with pytest.raises(rc.RCError):
        big = W.make_c1(P=16385)
        dwb = rc.DeviceWorkload(big)
        rc.compute_records(rc.Scene.from_workload(big), dwb, splits=2)
    sc.close()


def test_c2_full_size_sampled_records_match_oracle(dev):
    """C2 at its full size (10k records, 1024 directions, 10k-triangle soup in a
    closed room, 4 lights) in the benchmark's launch configuration (batched
    persistent launch from a device-built queue, graph replay); a seeded 1 %
    sample of the records (100) is recomputed by the oracle."""
    w = W.make_c2()
    _say("C2 full:", w.n_rec, "records,", w.n_tri, "triangles")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        (v, g, h), errs = gpu_records(w, batched=True, use_graph=True, stream=s)
    assert errs == 0
    idx = np.sort(np.random.default_rng(123).choice(w.n_rec, size=w.n_rec // 100, replace=False))  # 1 %
    ref = O.records_for(w, idx)
    assert_parity(v[idx], g[idx], h[idx], ref, "C2 1% sample")
    assert np.all(np.isfinite(v)) and np.all(np.isfinite(g)) and np.all(np.isfinite(h))


def test_ragged_strata_shapes_in_one_call(dev):
    """Mixed (n_theta, n_phi) in one launch: the minimum grid (2 x 5), rows
    wider than a wavefront (100, 128 columns: two passes per row), a ragged
    tail, and large N."""
    base = W.make_c2(P=12, n_soup=2000, seed=31)
    shapes = [(2, 5), (2, 6), (3, 7), (4, 16), (8, 32), (5, 100), (16, 64), (8, 128), (32, 128), (7, 65),
              (2, 200), (13, 37)]
    w = base
    w.n_theta = np.array([s[0] for s in shapes], np.int32)
    w.n_phi = np.array([s[1] for s in shapes], np.int32)
    _say("ragged shapes", shapes)
    (v, g, h), errs = gpu_records(w)
    assert errs == 0
    ref = O.records_for(w)
    assert_parity(v, g, h, ref, "ragged")


def test_empty_and_invalid_records(dev):
    w = W.make_c1(P=6)
    sc = rc.Scene.from_workload(w)
    # P = 0: a no-op
    w0 = W.make_c1(P=6)
    dw0 = rc.DeviceWorkload(w0)
    dw0.pos = dw0.pos[:0]
    dw0.n_theta = dw0.n_theta[:0]
    dw0.n_phi = dw0.n_phi[:0]
    rc.compute_records(sc, dw0)
    # invalid device inputs: n_phi too small, position outside the box
    w.n_phi = w.n_phi.copy()
    w.n_phi[1] = 3
    w.pos = w.pos.copy()
    w.pos[4] = [1.5, 0.5, 0.5]
    dw = rc.DeviceWorkload(w)
    dw.max_n_phi = 32
    v, g, h, ws = rc.compute_records(sc, dw)
    torch.cuda.synchronize()
    assert rc.rc_workspace_errors(ws) == 2
    v, g, h = v.cpu().numpy(), g.cpu().numpy(), h.cpu().numpy()
    assert np.all(np.isnan(v[[1, 4]])) and np.all(np.isnan(h[[1, 4]]))
    ok = [0, 2, 3, 5]
    ref = O.records_for(w, np.array(ok))
    assert_parity(v[ok], g[ok], h[ok], ref, "valid records next to invalid ones")
    sc.close()


def test_large_batch_with_n_phi_above_its_bound(dev):
    """Large batches (more than 16384 records) run one launch per n_phi class
    up to max_n_phi's class; a record whose n_phi exceeds max_n_phi, in a
    higher class, is still popped: its outputs are NaN and it is counted, and
    every other record is computed."""
    P = 20000
    w = W.make_c1(P=P)
    w.n_theta = np.full(P, 4, np.int32)
    w.n_phi = np.full(P, 8, np.int32)
    w.n_phi[[7, 12345]] = [40, 200]     # classes <= 64 and <= 256, above max_n_phi = 32
    w.n_phi[100] = 24
    sc = rc.Scene.from_workload(w)
    dw = rc.DeviceWorkload(w)
    dw.max_n_phi = 32
    v, g, h, ws = rc.compute_records(sc, dw, batched=True)
    torch.cuda.synchronize()
    assert rc.rc_workspace_errors(ws) == 2
    v, g, h = v.cpu().numpy(), g.cpu().numpy(), h.cpu().numpy()
    assert np.all(np.isnan(v[[7, 12345]])) and np.all(np.isnan(g[[7, 12345]])) and np.all(np.isnan(h[[7, 12345]]))
    ok = np.setdiff1d(np.arange(P), [7, 12345])
    assert np.all(np.isfinite(v[ok])) and np.all(np.isfinite(h[ok]))
    idx = np.array([0, 100, 19999])
    ref = O.records_for(w, idx)
    assert_parity(v[idx], g[idx], h[idx], ref, "large batch next to out-of-bound n_phi")
    sc.close()


def test_watchdog_times_out_while_the_stream_is_held_and_returns_once_it_runs(dev):
    """rc_records_wait reports ETIMEOUT when no record finishes within the
    limit, and returns normally once the records run.  The stall is forced
    from the host: a host function that sleeps holds the stream, so no kernel
    ever waits on anything."""
    import ctypes
    import time
    w = W.make_c1(P=64)
    sc = rc.Scene.from_workload(w)
    dw = rc.DeviceWorkload(w)
    ws = dw.workspace()
    s = torch.cuda.Stream()
    rc.compute_records(sc, dw, batched=True, workspace=ws, stream=s)  # builds and caches the light bins
    torch.cuda.synchronize()
    hip = ctypes.CDLL("libamdhip64.so")
    hold = ctypes.CFUNCTYPE(None, ctypes.c_void_p)(lambda _: time.sleep(1.5))
    hip.hipLaunchHostFunc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert hip.hipLaunchHostFunc(ctypes.c_void_p(s.cuda_stream), ctypes.cast(hold, ctypes.c_void_p), None) == 0
    with torch.cuda.stream(s):
        v, g, h, _ = rc.compute_records(sc, dw, batched=True, workspace=ws, stream=s)
    t0 = time.time()
    with pytest.raises(rc.RCError) as e:
        rc.rc_records_wait(ws, 300, stream=s)
    assert e.value.code == rc.RC_ETIMEOUT and time.time() - t0 < 1.4
    assert rc.rc_records_wait(ws, 10000, stream=s) == 0
    torch.cuda.synchronize()
    assert rc.rc_workspace_errors(ws) == 0 and bool(torch.isfinite(v).all())
    ref = O.records_for(w, np.arange(4))
    assert_parity(v[:4].cpu().numpy(), g[:4].cpu().numpy(), h[:4].cpu().numpy(), ref, "records after the watchdog")
    sc.close()


def test_deterministic_batched_and_graph_replays_bitwise_equal(dev):
    w = W.make_c2(P=300, n_soup=3000, seed=41)
    w.n_theta = np.where(np.arange(300) % 3 == 0, 16, 8).astype(np.int32)
    w.n_phi = np.where(np.arange(300) % 3 == 0, 64, 32).astype(np.int32)
    sc = rc.Scene.from_workload(w)
    dw = rc.DeviceWorkload(w)
    ra = rc.compute_records(sc, dw)
    torch.cuda.synchronize()
    a = [t.clone() for t in ra[:3]]
    rb = rc.compute_records(sc, dw)
    torch.cuda.synchronize()
    b = [t.clone() for t in rb[:3]]
    _say("direct launches: invalid", rc.rc_workspace_errors(ra[3]), rc.rc_workspace_errors(rb[3]),
         "non-finite", int((~torch.isfinite(a[0])).sum()), int((~torch.isfinite(b[0])).sum()))
    assert bool(torch.isfinite(a[0]).all()) and bool(torch.isfinite(a[2]).all())
    s = torch.cuda.Stream()
    out = dw.outputs()
    ws = dw.workspace()
    reps = []
    hreps = []
    with torch.cuda.stream(s):
        for r in range(3):
            for t in out:
                t.fill_(float("nan"))          # eager work between graph replays
            # the record kernel's own traversal: the direct launches' layout
            rc.compute_records(sc, dw, batched=True, use_graph=True, out=out, workspace=ws, stream=s,
                               hits_pass=False)
            s.synchronize()
            reps.append([t.clone() for t in out])
        for r in range(3):  # with the primary-hit pass (its own graph)
            for t in out:
                t.fill_(float("nan"))
            prm = rc.make_params(w.ring_step, w.max_rings, dw.max_n_phi, w.seed, max_n_theta=dw.max_n_theta)
            rc.rc_records_batched(sc.handle, w.sigma_s, w.sigma_a, w.lights, dw.pos, dw.n_theta, dw.n_phi, prm,
                                  None, True, -1, out[0], out[1], out[2], ws, s)
            s.synchronize()
            hreps.append([t.clone() for t in out])
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    for rep in reps:
        for x, y in zip(a, rep):
            assert torch.equal(x, y)
    for rep in hreps[1:]:
        for x, y in zip(hreps[0], rep):
            assert torch.equal(x, y)
    assert all(bool(torch.isfinite(t).all()) for t in hreps[0])
    sc.close()


def test_fp64_study_mode_agrees(dev):
    w = W.make_c2(P=16, n_soup=2000, seed=51)
    (v0, g0, h0), _ = gpu_records(w, precision=0)
    (v1, g1, h1), _ = gpu_records(w, precision=1)
    ref = O.records_for(w)
    e0 = rel_errors(v0, g0, h0, ref)
    e1 = rel_errors(v1, g1, h1, ref)
    _say("FP32 path max errors", [float(e.max()) for e in e0[:3]], "FP64 study", [float(e.max()) for e in e1[:3]])
    assert_parity(v1, g1, h1, ref, "FP64 study mode")
    assert_parity(v0, g0, h0, ref, "FP32 terms")
    assert np.array_equal(v0, v1)          # value path is the same in both modes
    # the term arithmetic is not the accuracy bottleneck: FP32 inputs (hit
    # distances, vertex radiances) dominate, so both modes land close together
    assert e0[1].max() <= 4 * e1[1].max() + 1e-9 and e0[2].max() <= 4 * e1[2].max() + 1e-9


def test_radius_matches_oracle(dev):
    rng = np.random.default_rng(5)
    P = 2000
    value = np.abs(rng.normal(size=(P, 2))) + 0.01
    value[:5] = 0.0                                  # L <= 0 -> r_min
    hess = rng.normal(size=(P, 2, 6)) * 10 ** rng.uniform(-3, 2, size=(P, 1, 1))
    hess[5:8] = 0.0                                  # lambda = 0 -> r_max
    tv = torch.as_tensor(value, device=dev)
    th = torch.as_tensor(hess, device=dev)
    R = torch.empty(P, dtype=torch.float32, device=dev)
    axes = torch.empty((P, 12), dtype=torch.float32, device=dev)
    rc.rc_radius(tv, th, 1.5e-4, 1e-3, 0.4, R, axes)
    torch.cuda.synchronize()
    Ro, Rio, vec = O.radius(value.sum(1), hess.sum(1), 1.5e-4, 1e-3, 0.4, anisotropic=True)
    assert np.allclose(R.cpu().numpy(), Ro, rtol=2e-6, atol=0)
    ax = axes.cpu().numpy()
    assert np.allclose(np.sort(ax[:, :3], 1), np.sort(Rio, 1), rtol=2e-6)
    # eigenvectors: orthonormal, and H v = lambda v
    Hm = O.hess6_to_mat(hess.sum(1))
    V = ax[:, 3:].reshape(P, 3, 3).astype(np.float64)
    assert np.allclose(np.einsum("pij,pkj->pik", V, V), np.eye(3), atol=1e-5)
    lam = np.einsum("pki,pij,pkj->pk", V, Hm, V)
    res = np.einsum("pij,pkj->pki", Hm, V) - lam[..., None] * V
    assert np.all(np.linalg.norm(res, axis=-1) <= 1e-5 * np.abs(np.linalg.eigvalsh(Hm)).max(1, keepdims=True) + 1e-30)


def test_autotune_picks_a_configuration(dev, tmp_path):
    w = W.make_c2(P=2000, n_soup=3000, seed=61)
    sc = rc.Scene.from_workload(w)
    dw = rc.DeviceWorkload(w)
    v, g, h = dw.outputs()
    ws = dw.workspace()
    prm = rc.make_params(w.ring_step, w.max_rings, dw.max_n_phi, w.seed)
    cache = tmp_path / "tune.txt"
    best, ms = rc.rc_autotune(sc.handle, w.sigma_s, w.sigma_a, w.lights, dw.pos, dw.n_theta, dw.n_phi, prm, v, g, h,
                              ws, cache_path=cache)
    _say("autotune ms per tile", ms, "best", best)
    assert 0 <= best < len(ms) and ms[best] == min(ms)
    assert cache.read_text().strip().endswith(f" {best}")
    best2, _ = rc.rc_autotune(sc.handle, w.sigma_s, w.sigma_a, w.lights, dw.pos, dw.n_theta, dw.n_phi, prm, v, g, h,
                              ws, cache_path=cache, measure=False)
    assert best2 == best
    sc.close()


def test_points_very_close_to_surfaces(dev):
    """Cache points 1e-2 .. 1e-6 away from a wall and from a soup triangle:
    vertices almost at x (huge 1/r terms) must stay finite and match."""
    w = W.make_c2(P=4, n_soup=500, seed=71)
    t0 = w.tri[12].reshape(3, 3).astype(np.float64)       # first soup triangle
    c = t0.mean(0)
    n = np.cross(t0[1] - t0[0], t0[2] - t0[0])
    n /= np.linalg.norm(n)
    pts = []
    for h in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
        pts.append([0.37, h, 0.61])                        # above the floor
        pts.append(c + h * n)                              # above a soup triangle
    w.pos = np.array(pts, np.float32)
    w.n_theta = np.full(len(pts), 8, np.int32)
    w.n_phi = np.full(len(pts), 32, np.int32)
    (v, g, h), errs = gpu_records(w)
    assert errs == 0
    assert np.all(np.isfinite(v)) and np.all(np.isfinite(g)) and np.all(np.isfinite(h))
    ref = O.records_for(w)
    assert_parity(v, g, h, ref, "near-surface points")


@pytest.mark.parametrize("case", ["mixed classes", "split records"])
def test_primary_hits_pass_gives_identical_records(dev, case):
    """With the batch's largest n_theta given, the primary rays are traced in a
    separate coherent pass and read back by the record kernel: the records
    equal, bit for bit, those of the record kernel's own traversal.  Both runs
    take their shadow segments from the BVH, which keeps the record kernel's
    LDS layout (with light bins the pass also selects a kernel without a
    traversal stack and wider rows: other summation order, covered by the
    oracle parity tests)."""
    if case == "mixed classes":
        w = W.make_c3().subset(np.arange(20000))  # several n_phi classes, launched per class
    else:
        w = W.make_c2(P=3000, n_soup=4000, seed=19)  # small batch: records split over wavefronts
    sc = rc.Scene.from_workload(w)
    dw = rc.DeviceWorkload(w)
    out = []
    for mnt in (0, dw.max_n_theta):
        v, g, h = dw.outputs()
        ws = dw.workspace()
        prm = rc.make_params(w.ring_step, w.max_rings, dw.max_n_phi, w.seed, max_n_theta=mnt, shadow_bvh=True)
        rc.rc_records_batched(sc.handle, w.sigma_s, w.sigma_a, w.lights, dw.pos, dw.n_theta, dw.n_phi, prm, None,
                              True, -1, v, g, h, ws)
        torch.cuda.synchronize()
        assert rc.rc_workspace_errors(ws) == 0
        out.append((v, g, h))
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a, b)
    sc.close()


def test_primary_hits_pass_rejects_records_above_the_n_theta_bound(dev):
    w = W.make_c2(P=20000, n_soup=2000, seed=20)
    w.n_theta[[5, 17000]] = 32  # above the bound given below
    sc = rc.Scene.from_workload(w)
    dw = rc.DeviceWorkload(w)
    v, g, h = dw.outputs()
    ws = dw.workspace()
    prm = rc.make_params(w.ring_step, w.max_rings, dw.max_n_phi, w.seed, max_n_theta=16)
    rc.rc_records_batched(sc.handle, w.sigma_s, w.sigma_a, w.lights, dw.pos, dw.n_theta, dw.n_phi, prm, None,
                          False, -1, v, g, h, ws)
    torch.cuda.synchronize()
    assert rc.rc_workspace_errors(ws) == 2
    vv = v.cpu().numpy()
    assert np.isnan(vv[[5, 17000]]).all() and np.isfinite(np.delete(vv, [5, 17000], axis=0)).all()
    sc.close()


@pytest.mark.parametrize("case", ["mixed classes", "split records"])
def test_shadow_pass_gives_identical_records(dev, case):
    """With the shadow pass the hits pass also walks every vertex's shadow
    segments and the record kernel reads the visibility bits: the records
    equal, bit for bit, those whose segments the record kernel walks itself
    (both runs use the hits pass, so both share one LDS layout)."""
    if case == "mixed classes":
        w = W.make_c3().subset(np.arange(20000))
    else:
        w = W.make_c2(P=3000, n_soup=4000, seed=21)
    sc = rc.Scene.from_workload(w)
    dw = rc.DeviceWorkload(w)
    out = []
    for sp in (False, True):
        v, g, h = dw.outputs()
        ws = dw.workspace()
        prm = rc.make_params(w.ring_step, w.max_rings, dw.max_n_phi, w.seed, max_n_theta=dw.max_n_theta,
                             shadow_pass=sp)
        rc.rc_records_batched(sc.handle, w.sigma_s, w.sigma_a, w.lights, dw.pos, dw.n_theta, dw.n_phi, prm, None,
                              True, -1, v, g, h, ws)
        torch.cuda.synchronize()
        assert rc.rc_workspace_errors(ws) == 0
        out.append((v, g, h))
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a, b)
    sc.close()
