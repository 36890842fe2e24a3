"""The learned placement pipeline end to end on the GPU: the MLP trained by the
library's own kernels on records the method generates, what it gains over a
constant prediction, and the validity of the caches both pipelines build."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1805_09258_amd import placement as PL  # noqa: E402
from paper_1805_09258_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def trained(dev):
    cfg = PL.CacheConfig(batch=2048)
    X, y = PL.training_set(range(1000, 1004), 5000, cfg, dev)
    mlp = PL.Mlp.new(dev, seed=1)
    hist = PL.train(mlp, X, y, epochs=20, batch=512, log=_say)
    return cfg, mlp, float(y.mean().item()), hist


def _all_covered(cands, res):
    """Every candidate lies inside the (true) radius of some cache point, with
    the FP32 distance test of the insertion rule."""
    P = res.pos.cpu().numpy()
    R = res.R.cpu().numpy()
    ok = np.zeros(cands.n, bool)
    for s in range(0, len(P), 256):
        for p, r in zip(P[s:s + 256], R[s:s + 256]):
            ok |= O._within32(cands.pos, p[None, :], r)
    return ok


def test_trained_network_beats_a_constant_prediction(dev, trained):
    cfg, mlp, ymean, hist = trained
    assert hist[-1] < 0.5 * hist[0]
    Xv, yv = PL.training_set([1099], 5000, cfg, dev)
    mse_net = float(((PL.predict_log_radius(mlp, Xv) - yv) ** 2).mean().item())
    mse_const = float(((yv - ymean) ** 2).mean().item())
    untrained = PL.Mlp.new(dev, seed=1)
    torch.cuda.synchronize()
    mse_init = float(((PL.predict_log_radius(untrained, Xv) - yv) ** 2).mean().item())
    _say(f"held-out log-radius MSE: trained {mse_net:.4f}, constant {mse_const:.4f}, untrained {mse_init:.4f}")
    assert mse_net < 0.5 * mse_const
    assert mse_net < mse_init


def test_both_pipelines_build_valid_caches_and_learned_needs_fewer_record_rounds(dev, trained):
    cfg, mlp, _, _ = trained
    we = W.make_c4_scene(4242, P=1)
    ctx = PL.SceneContext(we)
    cands = W.GridCandidates(40, we.box_lo, we.box_hi, seed=4243)
    placer = PL.Placer(ctx, cands, cfg, dev)
    rp = placer.plain()
    _say("plain", rp.stats)
    assert rp.K > 0 and _all_covered(cands, rp).all()
    assert np.all(np.isfinite(rp.value.cpu().numpy())) and np.all(np.isfinite(rp.grad.cpu().numpy()))
    rl = placer.learned(mlp, 1.0)
    _say("learned", rl.stats)
    assert rl.K > 0 and _all_covered(cands, rl).all()
    Rl = rl.R.cpu().numpy()
    assert np.all((Rl >= cfg.r_min) & (Rl <= cfg.r_max))
    # the network decides the rounds: probes pick the points, and fewer full
    # records are computed than the plain rounds compute
    assert rl.stats["probes"] >= rl.stats["records_learned"]
    assert rl.stats["records"] < rp.stats["records"]
    ctx.close()


def test_learned_placement_is_deterministic(dev, trained):
    cfg, mlp, _, _ = trained
    we = W.make_c4_scene(4242, P=1)
    ctx = PL.SceneContext(we)
    cands = W.GridCandidates(24, we.box_lo, we.box_hi, seed=1)
    placer = PL.Placer(ctx, cands, cfg, dev)
    a = placer.learned(mlp, 0.9)
    pa, va = a.pos.clone(), a.value.clone()
    b = placer.learned(mlp, 0.9)
    assert a.K == b.K and torch.equal(pa, b.pos) and torch.equal(va, b.value)
    ctx.close()
