"""rc_records_noalloc (records without allocation, for callers that cannot
allocate) against rc_records through the C ABI: the same kernels, so the same
records bit for bit, on consecutive calls that share the library's workspace,
the second with a smaller batch.  Each output is also checked against the
FP64 oracle on a sample, to the record tolerances."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1805_09258_amd import rc  # noqa: E402
from paper_1805_09258_amd import workloads as W  # noqa: E402
from tests._compare import assert_parity  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _inputs(w, idx, dev):
    pos = torch.as_tensor(np.ascontiguousarray(w.pos[idx], np.float32), device=dev)
    nth = torch.as_tensor(np.ascontiguousarray(w.n_theta[idx], np.int32), device=dev)
    nph = torch.as_tensor(np.ascontiguousarray(w.n_phi[idx], np.int32), device=dev)
    return pos, nth, nph


def _outputs(P, dev):
    # filled with NaN so that an unwritten record cannot pass
    return (torch.full((P, 2), float("nan"), dtype=torch.float64, device=dev),
            torch.full((P, 2, 3), float("nan"), dtype=torch.float64, device=dev),
            torch.full((P, 2, 6), float("nan"), dtype=torch.float64, device=dev))


def _with_workspace(sc, w, idx, prm, dev):
    pos, nth, nph = _inputs(w, idx, dev)
    v, g, h = _outputs(len(idx), dev)
    ws = torch.zeros(rc.rc_workspace_size(len(idx)), dtype=torch.uint8, device=dev)
    rc.rc_records(sc.handle, w.sigma_s, w.sigma_a, w.lights, pos, nth, nph, prm, v, g, h, ws)
    torch.cuda.synchronize()
    assert rc.rc_workspace_errors(ws) == 0
    return v, g, h


def _without(sc, w, idx, prm, dev):
    pos, nth, nph = _inputs(w, idx, dev)
    v, g, h = _outputs(len(idx), dev)
    rc.rc_records_noalloc(sc.handle, w.sigma_s, w.sigma_a, w.lights, pos, nth, nph, prm, v, g, h)
    torch.cuda.synchronize()
    assert rc.rc_records_noalloc_errors() == 0
    return v, g, h


def test_noalloc_records_equal_workspace_records_on_consecutive_calls(dev):
    w = W.make_c2(P=rc.RC_NOALLOC_MAX_RECORDS, n_soup=4000, seed=71)
    prm = rc.make_params(w.ring_step, w.max_rings, int(w.n_phi.max()), w.seed)
    sc = rc.Scene.from_workload(w)
    big = np.arange(rc.RC_NOALLOC_MAX_RECORDS)        # the largest batch
    small = np.arange(1500, 2200)                      # then a smaller one (split records)
    print("noalloc: fresh scene (BVH shadow segments), P =", len(big), flush=True)
    first = _without(sc, w, big, prm, dev)
    print("rc_records (builds the light bins), P =", len(big), flush=True)
    ref_big = _with_workspace(sc, w, big, prm, dev)
    print("noalloc: light bins present, P =", len(small), flush=True)
    prm_small = rc.make_params(w.ring_step, w.max_rings, int(w.n_phi.max()), w.seed, rec_base=int(small[0]))
    second = _without(sc, w, small, prm_small, dev)
    ref_small = _with_workspace(sc, w, small, prm_small, dev)
    print("noalloc: light bins present, P =", len(big), flush=True)
    third = _without(sc, w, big, prm, dev)
    for got, ref in ((first, ref_big), (second, ref_small), (third, ref_big)):
        for a, b in zip(got, ref):
            assert torch.isfinite(a).all()
            assert torch.equal(a, b)
    # and the records themselves against the oracle on a seeded sample
    pick = np.sort(np.random.default_rng(5).choice(len(small), 24, replace=False))
    ref = O.records_for(w, small[pick])
    v, g, h = (t.cpu().numpy()[pick] for t in second)
    assert_parity(v, g, h, ref, "noalloc sample")
    sc.close()


def test_noalloc_records_reject_an_oversized_batch(dev):
    w = W.make_c2(P=8, n_soup=100, seed=72)
    prm = rc.make_params(w.ring_step, w.max_rings, int(w.n_phi.max()), w.seed)
    sc = rc.Scene.from_workload(w)
    P = rc.RC_NOALLOC_MAX_RECORDS + 1
    pos = torch.zeros((P, 3), dtype=torch.float32, device=dev) + 0.5
    nth = torch.full((P,), 4, dtype=torch.int32, device=dev)
    nph = torch.full((P,), 8, dtype=torch.int32, device=dev)
    v, g, h = _outputs(P, dev)
    with pytest.raises(rc.RCError, match="at most 4096"):
        rc.rc_records_noalloc(sc.handle, w.sigma_s, w.sigma_a, w.lights, pos, nth, nph, prm, v, g, h)
    assert torch.isnan(v).all()  # nothing launched
    sc.close()
