"""Pins of the oracle's learned-placement parts (probe features, greedy cover).

The probe features are recomputed here from plain geometry (ray-plane and
ray-box distances written out in numpy, the Lambertian shading formula, the
exponential attenuation) on scenes where every probe ray's fate is known in
closed form; greedy cover is checked against its defining properties and
against exhaustive search on tiny inputs.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O

SEED = 91


def _probe_dirs(seed, cid):
    d = O.directions(seed, cid, 4, 16)[1:-1].astype(np.float64)  # drop the poles: 4 x 16 strata, row-major
    return d


def _box_exit(x, w, lo, hi):
    t = np.inf
    for k in range(3):
        if w[k] > 0:
            t = min(t, (hi[k] - x[k]) / w[k])
        elif w[k] < 0:
            t = min(t, (lo[k] - x[k]) / w[k])
    return t


def _features(dist, Lt, hit, w, light_vis, light_irr):
    """The 32 features from per-direction distance, arriving radiance, hit flag."""
    ld = np.log(dist)
    f = np.zeros(32)
    f[0], f[1], f[2], f[3] = ld.min(), ld.mean(), ld.std(), ld.max()
    f[4] = 1.0 - hit.mean()
    f[5] = np.log(np.mean(1.0 / dist))
    mL = Lt.mean()
    f[6] = np.log(mL + 1e-6)
    f[7] = Lt.std() / (mL + 1e-6)
    f[8] = np.log(Lt.max() + 1e-6)
    f[9:13] = light_vis
    f[13:17] = light_irr
    sL = Lt.sum() + 1e-12
    f[17:20] = (Lt[:, None] * w).sum(0) / sL
    f[20:23] = (w / dist[:, None]).sum(0) / (1.0 / dist).sum()
    f[23:27] = ld.reshape(4, 16).mean(1)
    f[27:31] = np.log(Lt + 1e-6).reshape(4, 16).mean(1)
    f[31] = np.abs(Lt.reshape(4, 16) - np.roll(Lt.reshape(4, 16), -1, axis=1)).sum() / sL
    return f


@pytest.mark.parametrize("cid", [0, 5, 17])
def test_probe_over_a_lit_emitting_floor_matches_geometry(cid):
    """Wide floor z = 0 (emission 0.4, albedo 0.5) in a flat box, medium
    mu = 0.5, two point lights above: every downward probe ray that lands
    inside the box hits the floor at t = h / |w_z|; the rest leave the box."""
    Wd, top = 10.0, 1.0
    lo, hi = np.array([-Wd, -Wd, 0.0]), np.array([Wd, Wd, top])
    floor = np.array([[-Wd, -Wd, 0, Wd, -Wd, 0, Wd, Wd, 0], [-Wd, -Wd, 0, Wd, Wd, 0, -Wd, Wd, 0]], np.float32)
    rho, Le = 0.5, 0.4
    sc = O.Scene(floor, np.full(2, rho, np.float32), np.full(2, Le, np.float32), lo, hi)
    lights = np.array([[0.3, -0.2, 0.8, 3.0], [-1.5, 0.7, 0.5, 1.5]], np.float32)
    ss, sa = 0.3, 0.2
    mu = ss + sa
    x = np.array([0.25, -0.1, 0.35], np.float32)
    f = O.probe(sc, ss, sa, lights, x[None], SEED, ids=[cid])[0]

    x64 = x.astype(np.float64)
    w = _probe_dirs(SEED, cid)
    dist, Lt, hit = np.zeros(64), np.zeros(64), np.zeros(64, bool)
    for k in range(64):
        te = _box_exit(x64, w[k], lo, hi)
        th = -x64[2] / w[k][2] if w[k][2] < 0 else np.inf
        wn = np.linalg.norm(w[k])
        if th <= te:
            y = x64 + th * w[k]
            Ls = Le
            for lp in lights.astype(np.float64):
                dl = lp[:3] - y
                d = np.linalg.norm(dl)
                Ls += rho / np.pi * lp[3] * (dl[2] / d) * np.exp(-mu * d) / d ** 2
            dist[k], Lt[k], hit[k] = th * wn, np.exp(-mu * th * wn) * Ls, True
        else:
            dist[k], Lt[k] = te * wn, 0.0
    vis = np.array([1.0, 1.0, 0.0, 0.0])
    irr = np.zeros(4)
    for l, lp in enumerate(lights.astype(np.float64)):
        d = np.linalg.norm(lp[:3] - x64)
        irr[l] = np.log(lp[3] * np.exp(-mu * d) / d ** 2 + 1e-6)
    ref = _features(dist, Lt, hit, w, vis, irr)
    np.testing.assert_allclose(f, ref, rtol=2e-6, atol=2e-6)
    assert 0 < hit.sum() < 64


def test_probe_in_an_empty_box_sees_only_the_walls_of_the_medium():
    lo, hi = np.zeros(3), np.ones(3)
    sc = O.Scene(np.zeros((0, 9), np.float32), np.zeros(0, np.float32), None, lo, hi)
    lights = np.array([[0.5, 0.9, 0.5, 2.0]], np.float32)
    x = np.array([0.5, 0.5, 0.5], np.float32)
    f = O.probe(sc, 0.3, 0.2, lights, x[None], SEED, ids=[3])[0]
    w = _probe_dirs(SEED, 3)
    dist = np.array([_box_exit(x.astype(np.float64), wk, lo, hi) * np.linalg.norm(wk) for wk in w])
    ref = _features(dist, np.zeros(64), np.zeros(64, bool), w, [1, 0, 0, 0],
                    [np.log(2.0 * np.exp(-0.5 * 0.4) / 0.16 + 1e-6), 0, 0, 0])
    np.testing.assert_allclose(f, ref, rtol=2e-6, atol=2e-6)
    assert f[4] == 1.0 and f[17] == 0.0 and f[31] == 0.0


def test_probe_light_visibility_follows_an_occluding_square():
    """A square at z = 0.6 over the point hides light 0 straight above and not
    light 1 off to the side; light slots beyond the light count read 0."""
    sq = np.array([[-0.2, -0.2, 0.6, 0.2, -0.2, 0.6, 0.2, 0.2, 0.6],
                   [-0.2, -0.2, 0.6, 0.2, 0.2, 0.6, -0.2, 0.2, 0.6]], np.float32)
    sc = O.Scene(sq, np.full(2, 0.5, np.float32), None, (-1, -1, 0), (1, 1, 1))
    lights = np.array([[0.0, 0.0, 0.9, 1.0], [0.8, 0.0, 0.5, 1.0]], np.float32)
    f = O.probe(sc, 0.0, 0.0, lights, np.array([[0.0, 0.0, 0.3]], np.float32), SEED)[0]
    assert f[9] == 0.0 and f[10] == 1.0 and f[11] == 0.0 and f[12] == 0.0
    assert f[15] == 0.0 and f[16] == 0.0
    assert f[13] == pytest.approx(np.log(1.0 / 0.36 + 1e-6), rel=1e-6)  # light and point are FP32 inputs


def test_probe_is_a_function_of_seed_and_id_only():
    rng = np.random.default_rng(4)
    tri = rng.uniform(0, 1, (30, 9)).astype(np.float32)
    sc = O.Scene(tri, np.full(30, 0.7, np.float32), None, (0, 0, 0), (1, 1, 1))
    li = np.array([[0.5, 0.95, 0.5, 5.0]], np.float32)
    c = rng.uniform(0, 1, (6, 3)).astype(np.float32)
    a = O.probe(sc, 0.5, 0.1, li, c, 7, ids=np.arange(10, 16))
    b = O.probe(sc, 0.5, 0.1, li, c[::-1], 7, ids=np.arange(10, 16)[::-1])[::-1]
    np.testing.assert_array_equal(a, b)
    assert np.all(np.isfinite(a))
    assert not np.array_equal(a, O.probe(sc, 0.5, 0.1, li, c, 8, ids=np.arange(10, 16)))


# ---------------------------------------------------------------------------
# greedy cover
# ---------------------------------------------------------------------------
def _check_greedy(cand, R, acc):
    """The defining properties of the sequential greedy cover."""
    cand = np.asarray(cand, np.float64)
    acc = list(acc)
    assert acc == sorted(acc) and len(set(acc)) == len(acc)
    aset = set(acc)
    for i in range(len(cand)):
        earlier = [p for p in acc if p < i]
        covered = any(np.sum((cand[i] - cand[p]) ** 2) < R[p] ** 2 for p in earlier)
        assert (i in aset) == (not covered), i


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_greedy_cover_has_its_defining_properties(seed):
    rng = np.random.default_rng(seed)
    n = 300
    cand = rng.uniform(0, 1, (n, 3)).astype(np.float32)
    R = rng.uniform(0.02, 0.25, n).astype(np.float32)
    acc = O.greedy_cover(cand, R)
    _check_greedy(cand, R.astype(np.float64), acc)
    assert 1 < len(acc) < n


def test_greedy_cover_exhaustive_on_tiny_inputs():
    """Points on a line with every radius pattern from a small set: the result
    equals a hand enumeration of the insertion rule."""
    xs = np.array([0.0, 0.27, 0.52, 0.93, 1.0])  # no distance within 1e-6 of a radius
    cand = np.stack([xs, np.zeros(5), np.zeros(5)], 1).astype(np.float32)
    for radii in itertools.product([0.1, 0.35, 0.65], repeat=5):
        R = np.array(radii, np.float32)
        want = []
        for i in range(5):
            if not any(abs(xs[i] - xs[p]) < radii[p] for p in want):
                want.append(i)
        assert list(O.greedy_cover(cand, R)) == want, radii


def test_greedy_cover_edge_cases():
    assert len(O.greedy_cover(np.zeros((0, 3), np.float32), np.zeros(0, np.float32))) == 0
    one = O.greedy_cover(np.array([[0.1, 0.2, 0.3]], np.float32), np.array([0.5], np.float32))
    assert list(one) == [0]
    same = np.tile(np.array([[0.5, 0.5, 0.5]], np.float32), (4, 1))
    assert list(O.greedy_cover(same, np.full(4, 0.1, np.float32))) == [0]
    # zero radius covers nothing, not even a coincident point
    assert list(O.greedy_cover(same, np.zeros(4, np.float32))) == [0, 1, 2, 3]
