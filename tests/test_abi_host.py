"""C-ABI checks that need no GPU: the library loads, exports every entry
point the header declares, validates arguments on the host, and builds a
well-formed BVH."""
import ctypes as C
import re
from pathlib import Path

import numpy as np
import pytest

from paper_1805_09258_amd import rc
from paper_1805_09258_amd import workloads as W

ROOT = Path(__file__).resolve().parent.parent


def header_symbols():
    txt = (ROOT / "include" / "rc.h").read_text()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rc_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = rc.lib()
    syms = header_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(rc.EXPORTS) == syms


def test_version_and_workspace_size():
    assert "gfx950" in rc.rc_version()
    assert rc.rc_workspace_size(0) >= 256
    assert rc.rc_workspace_size(1000) >= rc.rc_workspace_size(0) + 4000
    assert rc.rc_workspace_size(1000) % 256 == 0


def test_host_validation_rejects_bad_arguments_without_touching_a_device():
    L = rc.lib()
    med = rc.rc_medium(1.0, 0.2)
    prm = rc.make_params(0.1, 20, 64, 1)
    lights, nl = rc._lights(np.zeros((1, 4), np.float32))
    # NULL scene
    assert L.rc_records(None, C.byref(med), lights, nl, None, None, None, 1, C.byref(prm), None, None, None, None,
                        None) == rc.RC_EINVAL
    assert "scene" in rc.lib().rc_last_error().decode()
    fake = C.c_void_p(1)  # never dereferenced: validation fails first
    bad_med = rc.rc_medium(-1.0, 0.2)
    assert L.rc_records(fake, C.byref(bad_med), lights, nl, None, None, None, 1, C.byref(prm), None, None, None,
                        None, None) == rc.RC_EINVAL
    for field, val in [("ring_step", 0.0), ("max_rings", 0), ("max_rings", 65), ("max_n_phi", 4),
                       ("max_n_phi", 257), ("precision", 2), ("rec_base", -1)]:
        p2 = rc.make_params(0.1, 20, 64, 1)
        setattr(p2, field, val)
        assert L.rc_records(fake, C.byref(med), lights, nl, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), 1,
                            C.byref(p2), C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), C.c_void_p(8),
                            None) == rc.RC_EINVAL, field
    # too many lights, negative intensity, NULL outputs, NULL workspace
    many, nmany = rc._lights(np.zeros((17, 4), np.float32))
    assert L.rc_records(fake, C.byref(med), many, nmany, None, None, None, 0, C.byref(prm), None, None, None, None,
                        None) == rc.RC_EINVAL
    neg, nneg = rc._lights(np.array([[0.5, 0.5, 0.5, -1.0]], np.float32))
    assert L.rc_records(fake, C.byref(med), neg, nneg, None, None, None, 0, C.byref(prm), None, None, None, None,
                        None) == rc.RC_EINVAL
    assert L.rc_records(fake, C.byref(med), lights, nl, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), 1,
                        C.byref(prm), None, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), None) == rc.RC_EINVAL
    assert L.rc_records(fake, C.byref(med), lights, nl, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), 1,
                        C.byref(prm), C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), None, None) == rc.RC_EINVAL
    # P = 0 is a valid no-op
    assert L.rc_records(fake, C.byref(med), lights, nl, None, None, None, 0, C.byref(prm), None, None, None, None,
                        None) == rc.RC_OK
    # radius
    assert L.rc_radius(None, None, -1, 1e-4, 1e-3, 0.3, None, None, None) == rc.RC_EINVAL
    assert L.rc_radius(C.c_void_p(8), C.c_void_p(8), 4, 0.0, 1e-3, 0.3, C.c_void_p(8), None, None) == rc.RC_EINVAL
    assert L.rc_radius(C.c_void_p(8), C.c_void_p(8), 4, 1e-4, 0.5, 0.3, C.c_void_p(8), None, None) == rc.RC_EINVAL
    assert L.rc_radius(None, None, 0, 1e-4, 1e-3, 0.3, None, None, None) == rc.RC_OK


def test_scene_create_validates_before_device():
    w = W.make_c1()
    with pytest.raises(rc.RCError) as e:
        rc.rc_scene_create(w.tri, w.albedo, None, np.array([0, 0, 0.]), np.array([1, 1, 0.]))  # empty box
    assert e.value.code == rc.RC_EINVAL
    out = w.tri.copy()
    out[0, 0] = 5.0
    with pytest.raises(rc.RCError) as e:
        rc.rc_scene_create(out, w.albedo, None, w.box_lo, w.box_hi)  # triangle outside the medium
    assert e.value.code == rc.RC_EINVAL
    nan = w.tri.copy()
    nan[3, 4] = np.nan
    with pytest.raises(rc.RCError) as e:
        rc.rc_scene_create(nan, w.albedo, None, w.box_lo, w.box_hi)
    assert e.value.code == rc.RC_EINVAL


def _check_bvh(tri, lo, hi):
    nodes, tris, st = rc.rc_bvh_build_host(tri, lo, hi)
    T = tri.shape[0]
    pad = st["pad"]
    ids = tris[:, 3].view(np.int32)
    assert sorted(ids.tolist()) == list(range(T))          # each triangle exactly once
    # stored vertices are the given FP32 vertices (the watertight test projects them)
    t = tri[ids]
    assert np.array_equal(tris[:, 0:3], t[:, 0:3])
    assert np.array_equal(tris[:, 4:7], t[:, 3:6])
    assert np.array_equal(tris[:, 8:11], t[:, 6:9])
    codes = nodes[:, 12:14].view(np.int32)
    depth = 0
    seen = set()

    def walk(code, lo_b, hi_b, d):
        nonlocal depth
        depth = max(depth, d)
        if code >= 0:
            assert code not in seen
            seen.add(code)
            nd = nodes[code]
            boxes = [((nd[0], nd[2], nd[8]), (nd[1], nd[3], nd[9])), ((nd[4], nd[6], nd[10]), (nd[5], nd[7], nd[11]))]
            for c, (bl, bh) in zip(codes[code], boxes):
                if np.all(np.array(bl) > np.array(bh)):
                    continue                              # empty child: inverted box, never entered
                walk(int(c), np.array(bl), np.array(bh), d + 1)
        else:
            first, cnt = (~code) >> 3, ((~code) & 7) + 1
            assert cnt <= st["leaf_max"]
            pd = np.ldexp(pad, -16)
            for r in tris[first:first + cnt]:
                tv = tri[r[3:4].view(np.int32)[0]].reshape(3, 3).astype(np.float64)
                # every triangle lies inside its leaf box with the padding
                assert np.all(tv.min(0) - 0.99 * pd >= lo_b) and np.all(tv.max(0) + 0.99 * pd <= hi_b)

    walk(0, None, None, 0)
    assert len(seen) == nodes.shape[0]
    assert depth <= st["depth"]
    return st


def test_bvh_structure_small_and_soup():
    w1 = W.make_c1()
    _check_bvh(w1.tri, w1.box_lo, w1.box_hi)
    w2 = W.make_c2(P=4, n_soup=2000)
    st = _check_bvh(w2.tri, w2.box_lo, w2.box_hi)
    assert st["depth"] < 32
    few = w1.tri[:3]
    _check_bvh(few, w1.box_lo, w1.box_hi)


def test_bvh_structure_of_deeper_scenes():
    """Scenes whose plain build needs a deeper traversal stack, so the builder
    also prices a tree bounded to the next smaller stack and keeps one of
    the two: whichever it keeps holds every triangle once, inside padded boxes,
    and no deeper than it reports."""
    w3 = W.make_c3(P=1, n_tri=20_000)
    st = _check_bvh(w3.tri, w3.box_lo, w3.box_hi)
    assert st["depth"] <= 24
    w5 = W.make_c5(P=1, n_tri=60_000)
    st = _check_bvh(w5.tri, w5.box_lo, w5.box_hi)
    assert st["depth"] <= 24


def test_bvh_structure_of_degenerate_scenes():
    """Coincident triangles (zero centroid extent: median splits only) and
    triangles strung along one line (one useful split axis) still give a valid
    tree, with the small-node and depth rules in play."""
    rng = np.random.default_rng(7)
    lo, hi = np.zeros(3, np.float32), np.ones(3, np.float32)
    one = np.array([0.4, 0.4, 0.4, 0.45, 0.4, 0.4, 0.4, 0.45, 0.42], np.float32)
    same = np.tile(one, (300, 1))
    st = _check_bvh(same, lo, hi)
    assert st["n_tri"] == 300
    x = np.sort(rng.uniform(0.05, 0.9, 5000)).astype(np.float32)
    line = np.stack([x, np.full_like(x, 0.5), np.full_like(x, 0.5), x + 0.01, np.full_like(x, 0.5),
                     np.full_like(x, 0.5), x, np.full_like(x, 0.51), np.full_like(x, 0.5)], axis=1)
    st = _check_bvh(line, lo, hi)
    assert st["depth"] <= 24


def test_bvh_padding_covers_fp32_hit_error():
    """The BVH pads each triangle's box by 2^-16 * scale (scale: the largest
    |coordinate| or box side).  The FP32 hit test (shared decision rule) must
    accept no point farther than a quarter of that from the triangle's box:
    checked on rays aimed at triangle edges, down to grazing incidence (1e-7
    rad), with exact FP64 geometry."""
    from oracle import oracle as O
    rng = np.random.default_rng(0)
    tri = rng.uniform(0, 1, size=(400, 9)).astype(np.float32)
    sc = O.Scene(tri, np.zeros(400, np.float32), None, (0, 0, 0), (1, 1, 1))
    _, _, st = rc.rc_bvh_build_host(tri, np.zeros(3, np.float32), np.ones(3, np.float32))
    pd = np.ldexp(st["pad"], -16)
    n = 40000
    k = rng.integers(0, 400, n)
    v = tri[k].reshape(n, 3, 3).astype(np.float64)
    s = rng.uniform(0, 1, n)
    e = rng.integers(0, 3, n)
    a, b = v[np.arange(n), e], v[np.arange(n), (e + 1) % 3]
    tgt = a + s[:, None] * (b - a)                        # points on edges
    nrm = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    tang = rng.normal(size=(n, 3))
    tang -= (tang * nrm).sum(1, keepdims=True) * nrm
    tang /= np.linalg.norm(tang, axis=1, keepdims=True)
    cosg = 10 ** rng.uniform(-7, 0, n)                    # down to grazing
    d = (np.sqrt(1 - cosg ** 2)[:, None] * tang - cosg[:, None] * nrm)
    o = tgt - 0.7 * d
    hid, t, _ = sc.trace(o.astype(np.float32), d.astype(np.float32), brute=True)
    hit = hid >= 0
    P = o.astype(np.float32).astype(np.float64) + t[:, None].astype(np.float64) * d.astype(np.float32)
    tb = tri[hid[hit]].reshape(-1, 3, 3).astype(np.float64)
    out = np.maximum(tb.min(1) - P[hit], P[hit] - tb.max(1)).max(1)
    assert hit.sum() > 10000
    assert out.max() < pd / 4, (out.max(), pd)


def test_binding_constants_match_header():
    import re
    text = (Path(__file__).resolve().parent.parent / "include" / "rc.h").read_text()
    defs = dict(re.findall(r"#define (RC_[A-Z_]+) (-?\d+)", text))
    assert int(defs["RC_PLACE_STATE_INTS"]) == rc.RC_PLACE_STATE_INTS
    assert (int(defs["RC_MAX_LIGHTS"]), int(defs["RC_MAX_RINGS"]), int(defs["RC_MAX_NPHI"])) == (
        rc.RC_MAX_LIGHTS, rc.RC_MAX_RINGS, rc.RC_MAX_NPHI)
