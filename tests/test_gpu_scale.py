"""Records on the large scenes against the FP64 oracle, sampled: the 100k-
triangle batched workload with mixed sample counts (cost-ordered queue,
autotuned launch, graph replay) and the 1M-triangle scene, where the
per-output error of the FP32 path and of the all-FP64 term mode is reported
on the sample."""
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


def _run(w, dev, precision=0, autotune=False, graph=False):
    sc = rc.Scene.from_workload(w)
    dw = rc.DeviceWorkload(w, device=dev)
    v, g, h = dw.outputs()
    ws = dw.workspace()
    tile = -1
    if autotune:
        prm = rc.make_params(w.ring_step, w.max_rings, dw.max_n_phi, w.seed)
        tile, ms = rc.rc_autotune(sc.handle, w.sigma_s, w.sigma_a, w.lights, dw.pos, dw.n_theta, dw.n_phi, prm,
                                  v, g, h, ws)
        _say(f"autotune: tile {tile}, {['%.1f' % m for m in ms]} ms")
    rc.compute_records(sc, dw, batched=True, use_graph=graph, tile=tile, precision=precision, out=(v, g, h),
                       workspace=ws)
    if graph:  # replay once more: the captured launch must give the same records
        v0 = v.clone()
        rc.compute_records(sc, dw, batched=True, use_graph=True, tile=tile, precision=precision, out=(v, g, h),
                           workspace=ws)
        torch.cuda.synchronize()
        assert torch.equal(v0, v)
    torch.cuda.synchronize()
    assert rc.rc_workspace_errors(ws) == 0
    out = (v.cpu().numpy(), g.cpu().numpy(), h.cpu().numpy())
    sc.close()
    return out


@pytest.mark.parametrize("P", [3000, 20000])
def test_c3_batched_mixed_sample_counts_sampled_parity(dev, P):
    """3000 records run as one launch (records split over wavefronts); 20000
    as one launch per n_phi class (each with its own LDS size)."""
    full = W.make_c3()
    w = full.subset(np.arange(P))
    _say("C3 scene:", w.n_tri, "triangles; N in", int((w.n_theta * w.n_phi).min()), "..",
         int((w.n_theta * w.n_phi).max()))
    v, g, h = _run(w, dev, autotune=True, graph=True)
    rng = np.random.default_rng(33)
    idx = np.sort(rng.choice(w.n_rec, 16, replace=False))
    ref = O.records_for(w, idx)
    assert_parity(v[idx], g[idx], h[idx], ref, "C3 sample")


def test_c5_million_triangles_sampled_precision(dev):
    full = W.make_c5(P=2048)
    w = full.subset(np.arange(1024))
    _say("C5 scene:", w.n_tri, "triangles")
    v, g, h = _run(w, dev)
    v64, g64, h64 = _run(w, dev, precision=1)
    rng = np.random.default_rng(55)
    idx = np.sort(rng.choice(w.n_rec, 160, replace=False))
    ref = O.records_for(w, idx)
    for name, (a, b, c) in (("fp32 terms", (v, g, h)), ("fp64 terms", (v64, g64, h64))):
        ev, eg, eh, _, _ = rel_errors(a[idx], b[idx], c[idx], ref)
        q = lambda e: f"median {np.median(e):.1e} p99 {np.quantile(e, .99):.1e} max {e.max():.1e}"  # noqa: E731
        _say(f"C5 {name}, 160 records x 2 channels: value {q(ev)}; gradient {q(eg)}; Hessian {q(eh)}")
    assert_parity(v[idx], g[idx], h[idx], ref, "C5 sample")
    assert_parity(v64[idx], g64[idx], h64[idx], ref, "C5 sample, FP64 terms")
