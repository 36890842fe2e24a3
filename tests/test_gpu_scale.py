"""Records on the large scenes against the FP64 oracle, from full-size launches
in the benchmark's configuration, sampled: the 200k-record, 100k-triangle
batched workload with mixed sample counts (cost-ordered queue, autotuned
launch, graph replay; 1 % sample) and the 1M-record, 1M-triangle scene, where
the per-output error of the FP32 path and of the all-FP64 term mode is
reported on a 0.1 % sample (1 % would keep the oracle busy for minutes)."""
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


def _table(name, v, g, h, ref):
    ev, eg, eh, _, _ = rel_errors(v, g, h, ref)
    q = lambda e: f"median {np.median(e):.1e} p99 {np.quantile(e, .99):.1e} max {e.max():.1e}"  # noqa: E731
    _say(f"{name}, {len(v)} records x 2 channels: value {q(ev)} (tol 1e-4); gradient {q(eg)} (tol 1e-3); "
         f"Hessian {q(eh)} (tol 5e-3)")


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


def test_c3_full_size_launch_one_percent_parity(dev):
    """All 200k records in one autotuned, graph-replayed launch (one launch per
    n_phi class); a seeded 1 % sample (2000 records) against the oracle."""
    w = W.make_c3()
    v, g, h = _run(w, dev, autotune=True, graph=True)
    assert np.all(np.isfinite(v)) and np.all(np.isfinite(g)) and np.all(np.isfinite(h))
    idx = np.sort(np.random.default_rng(34).choice(w.n_rec, w.n_rec // 100, replace=False))
    ref = O.records_for(w, idx)
    _table("C3 1% sample", v[idx], g[idx], h[idx], ref)
    assert_parity(v[idx], g[idx], h[idx], ref, "C3 1% sample")


def test_c5_full_size_launch_precision(dev):
    """All 1M records over 1M triangles in one launch, with FP32 terms (the
    default) and with every term in FP64; a seeded 0.1 % sample (1000
    records) against the oracle, per output."""
    w = W.make_c5()
    _say("C5 scene:", w.n_tri, "triangles,", w.n_rec, "records")
    v, g, h = _run(w, dev)
    v64, g64, h64 = _run(w, dev, precision=1)
    idx = np.sort(np.random.default_rng(55).choice(w.n_rec, 1000, replace=False))
    ref = O.records_for(w, idx)
    _table("C5 FP32 terms", v[idx], g[idx], h[idx], ref)
    _table("C5 FP64 terms", v64[idx], g64[idx], h64[idx], ref)
    assert_parity(v[idx], g[idx], h[idx], ref, "C5 0.1% sample")
    assert_parity(v64[idx], g64[idx], h64[idx], ref, "C5 0.1% sample, FP64 terms")
