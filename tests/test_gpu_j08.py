"""The comparison method's records (occlusion-unaware gradients, supplement
Eqs. S.3-S.4; gradient-norm radius, Eq. jaroszRadius) on the GPU against
the oracle, through the C ABI.

Values to 1e-4 relative (as records); gradients to 2e-3 of the mean
per-direction gradient norm (the estimator's own scale: a grazing hit's
1/(yx . n) term amplifies the FP32 normal's rounding in a single sample);
the moments and the radius to 2e-3 relative.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1805_09258_amd import rc  # noqa: E402
from paper_1805_09258_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
EPS, RMIN, RMAX = 0.3, 1e-3, 0.43


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def gpu_j08(w, dev, n_theta=None, rec_base=0):
    sc = rc.Scene.from_workload(w)
    T = lambda a: torch.as_tensor(a, device=dev)  # noqa: E731
    P = w.n_rec
    val = torch.full((P, 2), -1.0, dtype=torch.float64, device=dev)
    grad = torch.full((P, 2, 3), -1.0, dtype=torch.float64, device=dev)
    mom = torch.full((P, 2), -1.0, dtype=torch.float64, device=dev)
    R = torch.full((P,), -1.0, dtype=torch.float32, device=dev)
    prm = rc.make_params(w.ring_step, w.max_rings, int(w.n_phi.max()), w.seed, rec_base=rec_base)
    nt = w.n_theta if n_theta is None else n_theta
    rc.rc_j08_records(sc.handle, w.sigma_s, w.sigma_a, w.lights, T(w.pos), T(nt), T(w.n_phi), prm, EPS, RMIN, RMAX,
                      val, grad, mom, R)
    torch.cuda.synchronize()
    sc.close()
    return val.cpu().numpy(), grad.cpu().numpy(), mom.cpu().numpy(), R.cpu().numpy()


def _compare(got, ref, idx, tag):
    v, g, m, R = got
    ov, og, om = ref
    v, g, m, R = v[idx], g[idx], m[idx], R[idx]
    scale = np.maximum(np.abs(ov).sum(1, keepdims=True), 1e-300)
    ev = (np.abs(v - ov) / scale).max()
    eg = (np.abs(g - og).max(2).max(1) / np.maximum(om[:, 1], 1e-300)).max()
    em = (np.abs(m - om) / np.maximum(np.abs(om), 1e-300)).max()
    oR = O.j08_radius(om, EPS, RMIN, RMAX)
    eR = (np.abs(R - oR) / oR).max()
    _say(f"{tag}: max rel err value {ev:.2e}, gradient {eg:.2e} (of the mean |grad L_k|), moments {em:.2e}, R {eR:.2e}")
    assert ev < 1e-4 and eg < 2e-3 and em < 2e-3 and eR < 2e-3


def test_c1_all_records_match_oracle(dev):
    w = W.make_c1()
    got = gpu_j08(w, dev)
    ref = O.j08(O.Scene.from_workload(w), w.sigma_s, w.sigma_a, w.lights, w.pos, w.n_theta, w.n_phi,
                ring_step=w.ring_step, max_rings=w.max_rings, seed=w.seed)
    _compare(got, ref, np.arange(w.n_rec), "C1 j08")


def test_c2_one_percent_of_the_full_launch_matches_oracle(dev):
    w = W.make_c2()
    got = gpu_j08(w, dev)
    idx = np.sort(np.random.default_rng(5).choice(w.n_rec, w.n_rec // 100, replace=False))
    ref = O.j08(O.Scene.from_workload(w), w.sigma_s, w.sigma_a, w.lights, w.pos[idx], w.n_theta[idx], w.n_phi[idx],
                rec_id=idx, ring_step=w.ring_step, max_rings=w.max_rings, seed=w.seed)
    _compare(got, ref, idx, "C2 1% j08")
    # same value samples as the records: the values equal rc_records' values
    # to the value tolerance (the record kernel sums in compensated FP32 with
    # corrected hit distances, this kernel in FP64 from the FP32 distances)
    sc = rc.Scene.from_workload(w)
    dw = rc.DeviceWorkload(w, device=dev)
    v, g, h, ws = rc.compute_records(sc, dw, batched=True)
    torch.cuda.synchronize()
    sc.close()
    np.testing.assert_allclose(got[0], v.cpu().numpy(), rtol=1e-4, atol=1e-12)


def test_invalid_sample_counts_give_nan_and_calls_are_deterministic(dev):
    w = W.make_c1(P=20)
    nt = w.n_theta.copy()
    nt[[3, 11]] = 1
    v, g, m, R = gpu_j08(w, dev, n_theta=nt)
    bad = np.zeros(20, bool)
    bad[[3, 11]] = True
    assert np.isnan(v[bad]).all() and np.isnan(g[bad]).all() and np.isnan(R[bad]).all()
    assert np.isfinite(v[~bad]).all() and np.isfinite(R[~bad]).all()
    v2, g2, m2, R2 = gpu_j08(w, dev, n_theta=nt)
    assert np.array_equal(v[~bad], v2[~bad]) and np.array_equal(g[~bad], g2[~bad]) and np.array_equal(R, R2,
                                                                                                     equal_nan=True)
    with pytest.raises(rc.RCError):
        sc = rc.Scene.from_workload(w)
        try:
            prm = rc.make_params(w.ring_step, w.max_rings, 32, w.seed)
            z = torch.zeros(1, device=dev)
            rc.rc_j08_records(sc.handle, w.sigma_s, w.sigma_a, w.lights, torch.zeros((1, 3), device=dev),
                              torch.ones(1, dtype=torch.int32, device=dev), torch.ones(1, dtype=torch.int32, device=dev),
                              prm, 0.0, RMIN, RMAX, z, z, z, z)  # eps must be > 0
        finally:
            sc.close()


@pytest.mark.parametrize("K,Q", [(1, 40), (300, 3000)])
def test_log_space_extrapolation_matches_oracle(dev, K, Q):
    """rc_interp_log against the oracle's Eq. jaroszExtrapolation: members
    and counts exactly, values to 1e-6 like rc_interp (the GPU forms the
    offset x' - x_k in FP32, relative error 6e-8, and the exponent multiplies
    it by grad L_k / L_k, up to about 60 here); a point with a non-positive
    value takes no part."""
    rng = np.random.default_rng(K + 3)
    cp = rng.uniform(0.2, 0.8, (K, 3)).astype(np.float32)
    cv = rng.uniform(0.05, 2.0, (K, 2))
    cv[0] = [-0.5, 0.2]  # sum <= 0: excluded
    cg = rng.normal(size=(K, 2, 3))
    cR = rng.uniform(0.05, 0.3, K).astype(np.float32)
    q = rng.uniform(0.15, 0.85, (Q, 3)).astype(np.float32)
    if K == 1:
        cv[0] = [0.7, 0.4]
        q = (cp[0] + rng.uniform(-1, 1, (Q, 3)) * cR[0]).astype(np.float32)
    T = lambda a: torch.as_tensor(a, device=dev)  # noqa: E731
    out = torch.full((Q,), float("nan"), dtype=torch.float64, device=dev)
    hits = torch.full((Q,), -1, dtype=torch.int32, device=dev)
    rc.rc_interp_log(T(cp), T(cv), T(cg), T(cR), T(q), out, hits)
    torch.cuda.synchronize()
    L, cov = O.interpolate_log(cp, cv.sum(1), cg.sum(1), cR, q)
    pos = cv.sum(1) > 0
    members = np.array([(O._within32(q[i][None], cp, cR) & pos).sum() for i in range(Q)])
    np.testing.assert_array_equal(hits.cpu().numpy(), np.where(cov, members, 0))
    assert cov.sum() > Q // 10
    np.testing.assert_allclose(out.cpu().numpy(), L, rtol=1e-6, atol=0)


def test_comparison_method_cache_obeys_the_insertion_rule(dev):
    """A cache of the comparison method (its radius, eps 0.3) over a grid of
    candidates in a seeded visiting order: every candidate ends inside a
    cached ball, no cached point lies inside the ball of a point cached
    before it, and the cache is read in log space."""
    from paper_1805_09258_amd.placement import CacheConfig, Placer, SceneContext, cache_error, direct_records
    w = W.make_c4_scene(77, P=1)
    ctx = SceneContext(w)
    cands = W.GridCandidates(20, w.box_lo, w.box_hi, seed=78)
    cfg = CacheConfig(n_theta=8, n_phi=32, batch=512, method="j08")
    res = Placer(ctx, cands, cfg, dev).plain()
    _say("comparison method cache", res.stats, res.K)
    assert res.K > 0 and res.log_space
    pos = cands.pos.astype(np.float32)
    acc_pos = res.pos.cpu().numpy()
    R = res.R.cpu().numpy()
    inside = np.zeros(cands.n, bool)
    for k in range(res.K):
        if k:
            assert not O._within32(acc_pos[k][None], acc_pos[:k], R[:k]).any(), f"cached point {k} was covered"
        inside |= O._within32(pos, acc_pos[k][None], R[k]) | (np.abs(pos - acc_pos[k]).max(1) == 0)
    assert inside.all()
    q = torch.as_tensor(W.uniform_points(2000, w.box_lo, w.box_hi, 79), device=dev)
    ref, _, _ = direct_records(ctx, q, cfg.n_theta, cfg.n_phi, cfg.record_id, dev, common_random=True)
    e = cache_error(res, q, ref, dev)
    _say("comparison method cache error", e)
    # its radii (median about 0.024 at eps 0.3) are below this grid's spacing
    # (0.05): the balls cover the candidates, not the whole box
    assert np.isfinite(e["rel_l2"]) and 0.2 < e["covered"] < 1.0
    with pytest.raises(ValueError):
        Placer(ctx, cands, CacheConfig(method="j08", anisotropic=True), dev)
    ctx.close()


def test_c3_mixed_sample_counts_match_oracle(dev):
    """128 points of the 100k-triangle slab scene with 256 to 4096 directions
    each (several strata shapes in one launch, a deeper BVH)."""
    w = W.make_c3().subset(np.arange(128))
    got = gpu_j08(w, dev)
    ref = O.j08(O.Scene.from_workload(w), w.sigma_s, w.sigma_a, w.lights, w.pos, w.n_theta, w.n_phi,
                ring_step=w.ring_step, max_rings=w.max_rings, seed=w.seed)
    _say(f"C3 sample counts {int((w.n_theta * w.n_phi).min())}..{int((w.n_theta * w.n_phi).max())}")
    _compare(got, ref, np.arange(w.n_rec), "C3[128] j08")
