"""GPU learned-placement kernels against the CPU oracle, through the C ABI:
the 64-ray probe, the BF16-MFMA MLP (forward, gradient, Adam), the feature
standardisation, greedy cover placement and cache interpolation."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1805_09258_amd import rc  # noqa: E402
from paper_1805_09258_amd import workloads as W  # noqa: E402
from tests._compare import assert_parity  # noqa: E402

pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -9      # unit roundoff of bfloat16 (8 significant bits, round to nearest)
GELU_SLOPE_MAX = 1.13   # sup |d/dx gelu_tanh(x)| (about 1.129)


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


# ---------------------------------------------------------------------------
# probe
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("C", [1, 333])
def test_probe_features_match_oracle(dev, C):
    w = W.make_c2(P=C, n_soup=10000)
    _say("probe: C2 scene,", C, "candidates")
    sc = rc.Scene.from_workload(w)
    cand = torch.as_tensor(w.pos, device=dev)
    f32 = torch.full((C, 32), float("nan"), device=dev)
    f16 = torch.zeros((C, 32), dtype=torch.bfloat16, device=dev)
    rc.rc_probe(sc.handle, w.sigma_s, w.sigma_a, w.lights, cand, 55, 1000, f32, f16.view(torch.int16))
    torch.cuda.synchronize()
    got = f32.cpu().numpy().astype(np.float64)
    ref = O.probe(O.Scene.from_workload(w), w.sigma_s, w.sigma_a, w.lights, w.pos, 55, ids=np.arange(C) + 1000)
    err = np.abs(got - ref) / (1e-4 + 1e-4 * np.abs(ref))
    _say("probe max scaled error", float(err.max()))
    assert np.all(np.isfinite(got))
    assert err.max() <= 1.0, np.unravel_index(err.argmax(), err.shape)
    # the BF16 copy is the FP32 feature rounded to nearest
    assert torch.equal(f16.cpu(), f32.cpu().to(torch.bfloat16))
    sc.close()


def test_probe_empty_input_and_errors(dev):
    w = W.make_c1()
    sc = rc.Scene.from_workload(w)
    cand = torch.zeros((0, 3), device=dev)
    rc.rc_probe(sc.handle, w.sigma_s, w.sigma_a, w.lights, cand, 1, 0, torch.zeros((0, 32), device=dev))
    with pytest.raises(rc.RCError):
        rc.rc_probe(sc.handle, -1.0, w.sigma_a, w.lights, torch.zeros((2, 3), device=dev), 1, 0,
                    torch.zeros((2, 32), device=dev))
    sc.close()


# ---------------------------------------------------------------------------
# MLP
# ---------------------------------------------------------------------------
def _new_mlp(dev, seed=5):
    params = torch.zeros(rc.rc_mlp_param_bytes(), dtype=torch.uint8, device=dev)
    state = torch.zeros(3 * rc.rc_mlp_n_params(), dtype=torch.float32, device=dev)
    rc.rc_mlp_init(params, state, seed)
    return params, state


def _unpack(master):
    """The FP32 master layout W1[128][32], b1, W2[128][128], b2, w3, b3."""
    m = np.asarray(master, np.float64)
    o = 0
    out = {}
    for k, shp in (("W1", (128, 32)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)), ("W3", (1, 128)),
                   ("b3", (1,))):
        n = int(np.prod(shp))
        out[k] = m[o:o + n].reshape(shp)
        o += n
    return out


def _std(params):
    f = params[:464 * 4].view(torch.float32).cpu().numpy().astype(np.float64)
    return f[:32], f[32:64]


def _features(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 32)) * rng.uniform(0.5, 3.0, 32) + rng.uniform(-4, 4, 32)
    return X.astype(np.float32)


GELU_CURV_MAX = 0.80    # sup |d2/dx2 gelu_tanh(x)| (about 0.798)


def _forward_bound(P, Xs, parts=False):
    """First-order bound on |y_bf16 - y_exact| from rounding the standardised
    inputs, W1, W2 and the layer-1 activations to bfloat16 (FP32 accumulation
    and the FP32 last layer add far less, covered by the 1e-6 terms).  With
    parts=True also returns the bounds on the two pre-activations."""
    u = U_BF16
    z1 = Xs @ P["W1"].T + P["b1"]
    a1 = O.gelu(z1)
    dz1 = 2 * u * (np.abs(Xs) @ np.abs(P["W1"]).T) + 1e-6
    da1 = GELU_SLOPE_MAX * dz1 + u * np.abs(a1)
    dz2 = u * (np.abs(a1) @ np.abs(P["W2"]).T) + da1 @ np.abs(P["W2"]).T + 1e-6
    z2 = a1 @ P["W2"].T + P["b2"]
    dy = (GELU_SLOPE_MAX * dz2) @ np.abs(P["W3"][0]) + 1e-6 * (1 + np.abs(O.gelu(z2)) @ np.abs(P["W3"][0]))
    return (dy, dz1, dz2) if parts else dy


def _grad_bound(P, Xs, target):
    """First-order running-error bound of the BF16 backward pass: errors of the
    forward pass carried into dL/dy and into the GELU slopes, plus rounding of
    dZ2, dZ1, the activations, the inputs and W2 to bfloat16."""
    u = U_BF16
    n = Xs.shape[0]
    _, (_, z1, a1, z2, a2) = O.mlp_forward(P, Xs)
    y = a2 @ P["W3"][0] + P["b3"][0]
    ey, ez1, ez2 = _forward_bound(P, Xs, parts=True)
    dy = (2.0 / n) * (y - target)
    e_dy = (2.0 / n) * ey
    w3 = np.abs(P["W3"][0])
    dz2 = np.abs(dy[:, None] * P["W3"][0] * O.gelu_grad(z2))
    e_dz2 = (e_dy[:, None] * w3 * GELU_SLOPE_MAX + np.abs(dy)[:, None] * w3 * GELU_CURV_MAX * ez2)
    ea1 = GELU_SLOPE_MAX * ez1
    E = {"b3": np.array([e_dy.sum()]),
         "W3": (e_dy @ np.abs(a2) + np.abs(dy) @ (GELU_SLOPE_MAX * ez2))[None, :],
         "b2": e_dz2.sum(0),
         "W2": (e_dz2 + u * dz2).T @ np.abs(a1) + dz2.T @ (u * np.abs(a1) + ea1)}
    W2 = np.abs(P["W2"])
    dA1 = dz2 @ W2
    e_dA1 = (e_dz2 + u * dz2) @ W2 + dz2 @ (u * W2)
    dz1 = dA1 * GELU_SLOPE_MAX
    e_dz1 = e_dA1 * GELU_SLOPE_MAX + dA1 * GELU_CURV_MAX * ez1
    E["b1"] = e_dz1.sum(0)
    E["W1"] = (e_dz1 + u * dz1).T @ np.abs(Xs) + dz1.T @ (u * np.abs(Xs))
    return E


@pytest.mark.parametrize("n", [1, 16, 1000, 70001])
def test_mlp_forward_within_bf16_bound_of_fp64_oracle(dev, n):
    params, state = _new_mlp(dev)
    X = _features(n, 3)
    tX = torch.as_tensor(X, device=dev)
    ws = torch.zeros(rc.rc_mlp_train_workspace_bytes(1), dtype=torch.uint8, device=dev)
    if n >= 2:
        rc.rc_mlp_fit_features(params, tX, ws)
    out = torch.full((n,), float("nan"), device=dev)
    rc.rc_mlp_forward(params, tX, out)
    torch.cuda.synchronize()
    P = _unpack(state[:rc.rc_mlp_n_params()].cpu().numpy())
    shift, scale = _std(params)
    if n >= 2:
        np.testing.assert_allclose(shift, X.astype(np.float64).mean(0), rtol=1e-5, atol=1e-5)
        np.testing.assert_allclose(scale, 1 / X.astype(np.float64).std(0), rtol=1e-4)
    Xs = (X.astype(np.float64) - shift) * scale
    y_ref, _ = O.mlp_forward(P, Xs)
    y = out.cpu().numpy().astype(np.float64)
    bound = _forward_bound(P, Xs)
    ratio = np.abs(y - y_ref) / bound
    _say(f"mlp forward n={n}: max |dy|/bound {ratio.max():.3f}, rms dy {np.sqrt(np.mean((y - y_ref) ** 2)):.2e}")
    assert np.all(np.isfinite(y))
    assert ratio.max() <= 1.0
    # statistical check: independent BF16 roundings leave a few u of relative
    # error; 10 u flags a systematic mistake the worst-case bound would hide
    _, (_, _, _, _, a2) = O.mlp_forward(P, Xs)
    scale_y = np.abs(a2) @ np.abs(P["W3"][0]) + abs(P["b3"][0])  # size of the terms summed into y
    assert np.sqrt(np.mean((y - y_ref) ** 2)) <= 10 * U_BF16 * np.sqrt(np.mean(scale_y ** 2))


def test_mlp_gradient_within_bf16_bound_of_fp64_oracle(dev):
    n = 1000  # 16 tiles of 64, ragged last tile
    params, state = _new_mlp(dev, seed=9)
    X = _features(n, 4)
    tX = torch.as_tensor(X, device=dev)
    ws = torch.zeros(rc.rc_mlp_train_workspace_bytes(n), dtype=torch.uint8, device=dev)
    rc.rc_mlp_fit_features(params, tX, ws)
    torch.cuda.synchronize()
    P = _unpack(state[:rc.rc_mlp_n_params()].cpu().numpy())
    shift, scale = _std(params)
    Xs = (X.astype(np.float64) - shift) * scale
    y0, _ = O.mlp_forward(P, Xs)
    rng = np.random.default_rng(1)
    target = (y0 + rng.normal(size=n)).astype(np.float32)
    grad = torch.zeros(rc.rc_mlp_n_params(), device=dev)
    loss = torch.zeros(1, device=dev)
    rc.rc_mlp_train_step(params, state, tX, torch.as_tensor(target, device=dev), 0.0, 1, ws, loss, grad)
    torch.cuda.synchronize()
    lref, gref = O.mlp_loss_grad(P, Xs, target)
    g = _unpack(grad.cpu().numpy())
    E = _grad_bound(P, Xs, target.astype(np.float64))
    for k in gref:
        err = np.abs(g[k] - gref[k])
        lim = 2 * E[k] + 1e-9
        _say(f"grad {k}: max err/limit {np.max(err / lim):.3f}, rel L2 "
             f"{np.linalg.norm(g[k] - gref[k]) / np.linalg.norm(gref[k]):.2e}")
        assert np.all(err <= lim), k
        assert np.linalg.norm(g[k] - gref[k]) <= 10 * U_BF16 * np.linalg.norm(gref[k]), k
    assert float(loss.cpu()) == pytest.approx(lref * n, rel=0.05)


def test_adam_steps_follow_the_oracle(dev):
    n, lr = 512, 1e-3
    params, state = _new_mlp(dev, seed=11)
    X = _features(n, 6)
    tX = torch.as_tensor(X, device=dev)
    ws = torch.zeros(rc.rc_mlp_train_workspace_bytes(n), dtype=torch.uint8, device=dev)
    rc.rc_mlp_fit_features(params, tX, ws)
    torch.cuda.synchronize()
    P = _unpack(state[:rc.rc_mlp_n_params()].cpu().numpy())
    P0 = {k: v.copy() for k, v in P.items()}
    shift, scale = _std(params)
    Xs = (X.astype(np.float64) - shift) * scale
    target = np.sin(Xs[:, 0]) + 0.5 * Xs[:, 1]
    tt = torch.as_tensor(target.astype(np.float32), device=dev)
    # step 1: where the oracle gradient is far above the BF16 error, the update is -lr sign(g)
    rc.rc_mlp_train_step(params, state, tX, tt, lr, 1, ws)
    torch.cuda.synchronize()
    P1 = _unpack(state[:rc.rc_mlp_n_params()].cpu().numpy())
    _, g1 = O.mlp_loss_grad(P0, Xs, target)
    for k in P1:
        big = np.abs(g1[k]) > 0.2 * np.abs(g1[k]).max()
        np.testing.assert_allclose((P1[k] - P0[k])[big], -lr * np.sign(g1[k][big]), rtol=1e-3, atol=1e-9)
    # moments: m = 0.1 g, v = 0.001 g^2 after one step
    m1 = _unpack(state[rc.rc_mlp_n_params():2 * rc.rc_mlp_n_params()].cpu().numpy())
    v1 = _unpack(state[2 * rc.rc_mlp_n_params():].cpu().numpy())
    for k in m1:
        big = np.abs(g1[k]) > 0.2 * np.abs(g1[k]).max()
        np.testing.assert_allclose(m1[k][big], 0.1 * g1[k][big], rtol=0.05)
        np.testing.assert_allclose(v1[k][big], 1e-3 * g1[k][big] ** 2, rtol=0.1)
    # 20 steps on both sides: the trajectories stay together and the loss falls
    Po = {k: v.copy() for k, v in P0.items()}
    mo = {k: np.zeros_like(v) for k, v in P0.items()}
    vo = {k: np.zeros_like(v) for k, v in P0.items()}
    loss0 = O.mlp_loss_grad(P0, Xs, target)[0]
    for t in range(1, 21):
        _, gg = O.mlp_loss_grad(Po, Xs, target)
        O.adam_step(Po, gg, mo, vo, t, lr)
        if t > 1:
            rc.rc_mlp_train_step(params, state, tX, tt, lr, t, ws)
    torch.cuda.synchronize()
    Pg = _unpack(state[:rc.rc_mlp_n_params()].cpu().numpy())
    d = np.concatenate([np.abs(Pg[k] - Po[k]).ravel() for k in Po])
    _say(f"adam 20 steps: median |dw| {np.median(d):.2e}, p99 {np.quantile(d, 0.99):.2e} (lr {lr})")
    assert np.median(d) < 0.5 * lr and np.quantile(d, 0.99) < 5 * lr
    assert O.mlp_loss_grad(Pg, Xs, target)[0] < 0.95 * loss0


def test_mlp_load_round_trip(dev):
    params, state = _new_mlp(dev, seed=2)
    X = torch.as_tensor(_features(100, 1), device=dev)
    a = torch.empty(100, device=dev)
    rc.rc_mlp_forward(params, X, a)
    p2 = torch.zeros_like(params)
    p2[:464 * 4] = params[:464 * 4]  # keep standardisation
    rc.rc_mlp_load(p2, state)
    b = torch.empty(100, device=dev)
    rc.rc_mlp_forward(p2, X, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(params, p2)


# ---------------------------------------------------------------------------
# placement and interpolation
# ---------------------------------------------------------------------------
def gpu_greedy(cand, R, batch, dev):
    """Rounds of gather / accept / cover until every candidate is decided."""
    C = cand.shape[0]
    tc = torch.as_tensor(cand, device=dev)
    tR = torch.as_tensor(R, device=dev)
    covered = torch.zeros(C, dtype=torch.uint8, device=dev)
    state = torch.zeros(rc.RC_PLACE_STATE_INTS, dtype=torch.int32, device=dev)
    bi = torch.zeros(batch, dtype=torch.int32, device=dev)
    bp = torch.zeros((batch, 3), device=dev)
    bR = torch.zeros(batch, device=dev)
    acc = torch.full((C,), -1, dtype=torch.int32, device=dev)
    accR = torch.zeros(C, device=dev)
    rounds = 0
    while True:
        rc.rc_place_gather(tc, tR, covered, state, bi, bp, bR, batch)
        if int(state[4].item()) == 0:
            break
        rc.rc_place_accept(tc, bi, bR, covered, state, acc, accR)
        rc.rc_place_cover(tc, covered, state, acc, accR)
        rounds += 1
        assert rounds <= C
    torch.cuda.synchronize()
    k = int(state[1].item())
    assert int(state[0].item()) == C and bool(covered.bool().all())
    return acc[:k].cpu().numpy().astype(np.int64), accR[:k].cpu().numpy(), rounds


@pytest.mark.parametrize("C,batch,seed", [(1, 1, 0), (700, 1, 1), (5000, 64, 2), (20000, 1024, 3), (3001, 1000, 4)])
def test_greedy_cover_equals_sequential_oracle(dev, C, batch, seed):
    rng = np.random.default_rng(seed)
    cand = rng.uniform(0, 1, (C, 3)).astype(np.float32)
    R = np.exp(rng.uniform(np.log(0.01), np.log(0.2), C)).astype(np.float32)
    acc, accR, rounds = gpu_greedy(cand, R, batch, dev)
    want = O.greedy_cover(cand, R)
    _say(f"cover C={C} batch={batch}: {len(want)} accepted in {rounds} rounds")
    np.testing.assert_array_equal(acc, want)
    np.testing.assert_array_equal(accR, R[want])


def test_greedy_cover_rejects_bad_batch(dev):
    t = torch.zeros((4, 3), device=dev)
    with pytest.raises(rc.RCError):
        rc.rc_place_gather(t, None, torch.zeros(4, dtype=torch.uint8, device=dev),
                           torch.zeros(rc.RC_PLACE_STATE_INTS, dtype=torch.int32, device=dev), torch.zeros(5000, dtype=torch.int32,
                                                                                      device=dev),
                           torch.zeros((5000, 3), device=dev), torch.zeros(5000, device=dev), 5000)


@pytest.mark.parametrize("K,Q", [(1, 1), (300, 2000), (2600, 777)])
def test_interpolation_matches_oracle(dev, K, Q):
    rng = np.random.default_rng(K)
    cp = rng.uniform(0, 1, (K, 3)).astype(np.float32)
    cv = rng.uniform(0, 2, (K, 2))
    cg = rng.normal(size=(K, 2, 3))
    cR = rng.uniform(0.05, 0.3, K).astype(np.float32)
    q = rng.uniform(0, 1, (Q, 3)).astype(np.float32)
    ref_v = rng.uniform(0, 2, (Q, 2))
    out = torch.full((Q,), float("nan"), dtype=torch.float64, device=dev)
    hits = torch.zeros(Q, dtype=torch.int32, device=dev)
    nb = (Q + 255) // 256
    err = torch.zeros(2 * nb, dtype=torch.float64, device=dev)
    T = lambda a: torch.as_tensor(a, device=dev)  # noqa: E731
    rc.rc_interp(T(cp), T(cv), T(cg), T(cR), T(q), out, hits, T(ref_v), err)
    torch.cuda.synchronize()
    L, cov = O.interpolate(cp, cv.sum(1), cg.sum(1), cR, q)
    got = out.cpu().numpy()
    np.testing.assert_array_equal(hits.cpu().numpy() > 0, cov)
    np.testing.assert_allclose(got, L, rtol=1e-6, atol=1e-6)
    e = err.cpu().numpy().reshape(-1, 2).sum(0)
    rv = ref_v.sum(1)
    # the GPU's Taylor term uses the FP32 offset x' - x_k (relative error 6e-8)
    np.testing.assert_allclose(e, [np.sum((L[cov] - rv[cov]) ** 2), np.sum(rv[cov] ** 2)], rtol=1e-6)


@pytest.mark.parametrize("C,batch,seed", [(9000, 4096, 5), (4096, 4096, 6), (30000, 777, 7)])
def test_greedy_cover_in_visiting_order_equals_oracle(dev, C, batch, seed):
    """A permutation as visiting order and the largest batch."""
    rng = np.random.default_rng(seed)
    cand = rng.uniform(0, 1, (C, 3)).astype(np.float32)
    R = np.exp(rng.uniform(np.log(0.005), np.log(0.1), C)).astype(np.float32)
    order = rng.permutation(C).astype(np.int32)
    tc, tR, to = (torch.as_tensor(a, device=dev) for a in (cand, R, order))
    covered = torch.zeros(C, dtype=torch.uint8, device=dev)
    state = torch.zeros(rc.RC_PLACE_STATE_INTS, dtype=torch.int32, device=dev)
    bi = torch.zeros(batch, dtype=torch.int32, device=dev)
    bp = torch.zeros((batch, 3), device=dev)
    bR = torch.zeros(batch, device=dev)
    acc = torch.full((C,), -1, dtype=torch.int32, device=dev)
    accR = torch.zeros(C, device=dev)
    accpos = torch.zeros((C, 3), device=dev)
    rounds = 0
    while True:
        rc.rc_place_gather(tc, tR, covered, state, bi, bp, bR, batch, order=to)
        if int(state[4].item()) == 0:
            break
        rc.rc_place_accept(tc, bi, bR, covered, state, acc, accR, accpos)
        rc.rc_place_cover(tc, covered, state, acc, accR)
        rounds += 1
    torch.cuda.synchronize()
    k = int(state[1].item())
    want = order[O.greedy_cover(cand[order], R[order])]
    _say(f"ordered cover C={C} batch={batch}: {len(want)} accepted in {rounds} rounds")
    np.testing.assert_array_equal(acc[:k].cpu().numpy(), want)
    np.testing.assert_array_equal(accpos[:k].cpu().numpy(), cand[want])


def test_accept_copies_records_of_accepted_slots(dev):
    rng = np.random.default_rng(3)
    C, B = 500, 64
    cand = rng.uniform(0, 1, (C, 3)).astype(np.float32)
    R = np.full(C, 0.15, np.float32)
    tc, tR = torch.as_tensor(cand, device=dev), torch.as_tensor(R, device=dev)
    covered = torch.zeros(C, dtype=torch.uint8, device=dev)
    state = torch.zeros(rc.RC_PLACE_STATE_INTS, dtype=torch.int32, device=dev)
    bi = torch.zeros(B, dtype=torch.int32, device=dev)
    bp = torch.zeros((B, 3), device=dev)
    bR = torch.zeros(B, device=dev)
    acc = torch.zeros(C, dtype=torch.int32, device=dev)
    accR = torch.zeros(C, device=dev)
    cval = torch.zeros((C, 2), dtype=torch.float64, device=dev)
    cgrad = torch.zeros((C, 2, 3), dtype=torch.float64, device=dev)
    seen = {}
    while True:
        rc.rc_place_gather(tc, tR, covered, state, bi, bp, bR, B)
        m = int(state[4].item())
        if m == 0:
            break
        # a record stand-in that names its candidate: value = (idx, -idx), grad = idx * (1..6)
        idx = bi[:m].double()
        bval = torch.stack([idx, -idx], 1).contiguous()
        bgrad = (idx[:, None] * torch.arange(1, 7, device=dev, dtype=torch.float64)).view(m, 2, 3).contiguous()
        bval = torch.cat([bval, torch.zeros((B - m, 2), dtype=torch.float64, device=dev)])
        bgrad = torch.cat([bgrad, torch.zeros((B - m, 2, 3), dtype=torch.float64, device=dev)])
        rc.rc_place_accept(tc, bi, bR, covered, state, acc, accR, None, bval, bgrad, cval, cgrad)
        rc.rc_place_cover(tc, covered, state, acc, accR)
    torch.cuda.synchronize()
    k = int(state[1].item())
    a = acc[:k].cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(cval[:k].cpu().numpy(), np.stack([a, -a], 1))
    np.testing.assert_array_equal(cgrad[:k].cpu().numpy().reshape(k, 6), a[:, None] * np.arange(1, 7))
    np.testing.assert_array_equal(acc[:k].cpu().numpy(), O.greedy_cover(cand, R))


@pytest.mark.parametrize("n", [9, 40])
def test_grid_cover_equals_definition(dev, n):
    g = W.GridCandidates(n, (0, 0, 0), (1.0, 1.5, 0.8), seed=n)
    rng = np.random.default_rng(n)
    K = 60
    pick = rng.choice(g.n, K, replace=False).astype(np.int32)
    R = np.exp(rng.uniform(np.log(0.01), np.log(0.6), K)).astype(np.float32)
    R[:3] = [0.0, 5.0, 1e-7]  # no cover, everything, only itself
    tc = torch.as_tensor(g.pos, device=dev)
    covered = torch.zeros(g.n, dtype=torch.uint8, device=dev)
    acc, accR = torch.as_tensor(pick, device=dev), torch.as_tensor(R, device=dev)
    rc.rc_place_cover_grid(tc, g.dims, g.lo, g.cell, covered, None, acc, accR, 0, K)
    torch.cuda.synchronize()
    want = np.zeros(g.n, bool)
    for p, r in zip(pick, R):
        want |= O._within32(g.pos, g.pos[p][None, :], r)
    np.testing.assert_array_equal(covered.cpu().numpy().astype(bool), want)
    with pytest.raises(rc.RCError):
        rc.rc_place_cover_grid(tc, [n, n, 0], g.lo, g.cell, covered, None, acc, accR, 0, K)


def test_mlp_radius_is_clamped_exp_of_forward(dev):
    params, state = _new_mlp(dev, seed=4)
    X = torch.as_tensor(_features(3000, 8), device=dev)
    y = torch.empty(3000, device=dev)
    R = torch.empty(3000, device=dev)
    rc.rc_mlp_forward(params, X, y)
    rc.rc_mlp_radius(params, X, 0.7, 0.05, 2.0, R)
    torch.cuda.synchronize()
    want = np.clip(0.7 * np.exp(y.cpu().numpy().astype(np.float64)), 0.05, 2.0)
    np.testing.assert_allclose(R.cpu().numpy(), want, rtol=2e-6)
    assert 0 < np.mean(want == 0.05) < 1 or 0 < np.mean(want == 2.0) < 1


def test_common_random_records_and_probe_match_oracle(dev):
    w = W.make_c1(P=24)
    sc = rc.Scene.from_workload(w)
    dw = rc.DeviceWorkload(w)
    v, g, h = dw.outputs()
    ws = dw.workspace()
    prm = rc.make_params(w.ring_step, w.max_rings, dw.max_n_phi, w.seed, rec_base=77, common_random=True)
    rc.rc_records(sc.handle, w.sigma_s, w.sigma_a, w.lights, dw.pos, dw.n_theta, dw.n_phi, prm, v, g, h, ws)
    f = torch.zeros((w.n_rec, 32), device=dev)
    rc.rc_probe(sc.handle, w.sigma_s, w.sigma_a, w.lights, dw.pos, w.seed, 5, f, common_random=True)
    torch.cuda.synchronize()
    ids = np.full(w.n_rec, 77)
    osc = O.Scene.from_workload(w)
    ref = O.records(osc, w.sigma_s, w.sigma_a, w.lights, w.pos, w.n_theta, w.n_phi, rec_id=ids,
                    ring_step=w.ring_step, max_rings=w.max_rings, seed=w.seed)
    assert_parity(v.cpu().numpy(), g.cpu().numpy(), h.cpu().numpy(), ref, "common random numbers")
    fr = O.probe(osc, w.sigma_s, w.sigma_a, w.lights, w.pos, w.seed, ids=np.full(w.n_rec, 5))
    err = np.abs(f.cpu().numpy() - fr) / (1e-4 + 1e-4 * np.abs(fr))
    assert err.max() <= 1.0
    sc.close()
