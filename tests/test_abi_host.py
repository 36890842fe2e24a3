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


def _bin_candidates(b, L, y):
    """Triangle ids the kernels test for the segment y -> L: every entry of
    the segment's bin on each level up to the first stored distance beyond
    the segment (the same FP32 bin arithmetic as the kernels)."""
    d = (np.float32(L) - np.float32(y)).astype(np.float32)
    ad = np.abs(d)
    kz = 0
    if ad[1] > ad[kz]:
        kz = 1
    if ad[2] > ad[kz]:
        kz = 2
    kx, ky = (kz + 1) % 3, (kz + 2) % 3
    ez, ex, ey = -d[kz], -d[kx], -d[ky]
    if not abs(ez) > 0:
        return []
    ia = np.float32(1.0) / np.float32(abs(ez))
    face = 2 * kz + (0 if ez > 0 else 1)
    B = b["B"]
    hb = np.float32(0.5) * np.float32(B)
    iu = min(max(int(np.float32((np.float32(ex * ia) + np.float32(1)) * hb)), 0), B - 1)
    iv = min(max(int(np.float32((np.float32(ey * ia) + np.float32(1)) * hb)), 0), B - 1)
    reach = np.float32(np.sqrt(np.float32(d @ d))) * np.float32(1 + 2.0 ** -20)
    ids = []
    offs = b["offs"]
    for k in range(b["levels"]):
        Bk = B >> (2 * k)
        h = b["level_off"][k] + 2 * ((face * Bk + (iu >> (2 * k))) * Bk + (iv >> (2 * k)))
        if offs[h + 1:h + 2].view(np.float32)[0] > reach:
            continue
        for e in range(offs[h], offs[h + 2]):
            assert b["entries"][e, 7] <= reach
            ids.append(int(b["entries"][e, 3:4].view(np.int32)[0]))
            if b["entries"][e, 11] > reach:
                break
    return ids


def _adversarial_points(tri, L, rng, n):
    """Points whose segment to the light skims triangle edges and vertices,
    lies on cube-face boundaries seen from the light, or starts next to it."""
    t3 = tri.reshape(-1, 3, 3).astype(np.float64)
    j = rng.integers(0, len(t3), n)
    e = rng.integers(0, 3, n)
    s = rng.uniform(0, 1, n)
    a, b_ = t3[j, e], t3[j, (e + 1) % 3]
    p = a + s[:, None] * (b_ - a)
    far = L + rng.uniform(1.02, 3.0, (n, 1)) * (p - L)
    diag = np.stack([np.full(n, 1.0), rng.choice([-1.0, 1.0], n), rng.uniform(-1, 1, n)], 1)
    diag = L + rng.uniform(0.05, 0.8, (n, 1)) * rng.permuted(diag, axis=1)
    near = L + rng.normal(size=(n, 3)) * 10 ** rng.uniform(-4, -1, (n, 1))
    return np.concatenate([far, diag, near])


@pytest.mark.parametrize("scene", ["c2", "c3", "degenerate"])
def test_light_bins_answer_every_segment_like_all_triangles(scene):
    """The bins of a light list, for every segment y -> light, a superset of
    the triangles the watertight test can accept on it: testing only a
    segment's bin candidates (oracle decision rule) gives the answer of
    testing every triangle, on random segments and on segments that skim
    edges, run along cube-face boundaries or start next to the light."""
    from oracle import oracle as O
    rng = np.random.default_rng({"c2": 3, "c3": 4, "degenerate": 5}[scene])
    if scene == "c2":
        w = W.make_c2(P=1, n_soup=1500, seed=41)
    elif scene == "c3":
        w = W.make_c3(P=1, n_tri=3000, seed=42)
    else:
        w = W.make_c2(P=1, n_soup=200, seed=43)
        # triangles through the light, next to it and edge-on to it
        L = w.lights[0, :3].astype(np.float64)
        extra = np.array([np.r_[L + [-0.1, 0, -0.1], L + [0.1, 0, -0.1], L + [0, 0, 0.1]],
                          np.r_[L + [1e-5, -0.05, -0.05], L + [1e-5, 0.05, -0.05], L + [1e-5, 0, 0.05]],
                          np.r_[L + [-0.2, -0.3, 0.0], L + [0.2, -0.3, 0.0], L + [0.0, -0.3, 1e-7]]], np.float32)
        w.tri = np.concatenate([w.tri, extra])
        w.albedo = np.concatenate([w.albedo, np.full(3, 0.7, np.float32)])
    sc = O.Scene(w.tri, w.albedo, None, w.box_lo, w.box_hi)
    for li in range(min(2, len(w.lights))):
        L = w.lights[li, :3].astype(np.float32)
        b = rc.rc_light_bins_host(w.tri, w.box_lo, w.box_hi, L)
        assert b["levels"] >= 1 and b["entries"].shape[0] > 0
        pts = np.concatenate([rng.uniform(w.box_lo, w.box_hi, (600, 3)),
                              _adversarial_points(w.tri, L.astype(np.float64), rng, 300)]).astype(np.float32)
        pts = pts[np.all((pts > w.box_lo) & (pts < w.box_hi), axis=1)]
        skip = np.where(rng.uniform(size=len(pts)) < 0.2, rng.integers(0, w.n_tri, len(pts)), -1)
        seg = (L[None, :] - pts).astype(np.float32)
        full = sc.occluded(pts, seg, skip=skip, brute=True)
        mism = 0
        for i in range(len(pts)):
            ids = sorted(set(_bin_candidates(b, L, pts[i])))
            if not ids:
                sub = False
            else:
                ssc = O.Scene(w.tri[ids], w.albedo[ids], None, w.box_lo, w.box_hi)
                sk = ids.index(skip[i]) if skip[i] in ids else -1
                sub = bool(ssc.occluded(pts[i:i + 1], seg[i:i + 1], skip=np.array([sk]), brute=True)[0])
            mism += int(sub != bool(full[i]))
        assert mism == 0, (scene, li, mism, len(pts))
        assert full.sum() >= 10


def test_watchdog_rejects_bad_arguments_without_a_device():
    ws = np.zeros(64, np.uint32)
    assert rc.lib().rc_records_wait(None, 100, None) == rc.RC_EINVAL
    assert rc.lib().rc_records_wait(ws.ctypes.data_as(rc.C.c_void_p), -1, None) == rc.RC_EINVAL


def test_noalloc_records_reject_batches_above_the_limit_without_a_device():
    """rc_records_noalloc rejects more than RC_NOALLOC_MAX_RECORDS records
    before it touches a device."""
    L = rc.lib()
    prm = rc.make_params(0.1, 8, 64, 1)
    med = rc.rc_medium(1.0, 0.2)
    P = rc.RC_NOALLOC_MAX_RECORDS + 1
    r = L.rc_records_noalloc(None, rc.C.byref(med), None, 0, None, None, None, P, rc.C.byref(prm), None, None, None,
                             None)
    assert r == rc.RC_EINVAL
    assert b"at most 4096" in L.rc_last_error()
    assert L.rc_records_noalloc(None, rc.C.byref(med), None, 0, None, None, None, 16, rc.C.byref(prm), None, None,
                                None, None) == rc.RC_EINVAL


def test_tile_table_is_readable_without_a_device():
    tiles = [rc.rc_tile_info(t) for t in range(10)]
    assert tiles[0] == {"grid": 1.0, "refill_min": 12, "leaf_batch": 0, "lds_waves": 4}
    assert {t["lds_waves"] for t in tiles} == {2, 3, 4}
    with pytest.raises(rc.RCError):
        rc.rc_tile_info(10)


def test_render_pass_entries_reject_bad_arguments_without_a_device():
    L = rc.lib()
    vp = rc.C.c_void_p
    for step in (0.0, -0.1, float("nan"), float("inf")):  # march step
        assert L.rc_march_emit(vp(8), vp(8), vp(8), 4, step, 1.0, 1.2, vp(8), vp(8), vp(8), None) == rc.RC_EINVAL
    assert L.rc_march_count(None, vp(8), vp(8), vp(8), 4, 0.1, vp(8), vp(8), None) == rc.RC_EINVAL
    assert L.rc_march_emit(vp(8), vp(8), vp(8), -1, 0.1, 1.0, 1.2, vp(8), vp(8), vp(8), None) == rc.RC_EINVAL
    assert L.rc_march_emit(vp(8), vp(8), vp(8), 4, 0.1, -1.0, 1.2, vp(8), vp(8), vp(8), None) == rc.RC_EINVAL
    assert L.rc_march_emit(None, vp(8), vp(8), 4, 0.1, 1.0, 1.2, vp(8), vp(8), vp(8), None) == rc.RC_EINVAL
    # pixels: spp must divide the ray count
    assert L.rc_composite(vp(8), 10, 3, vp(8), vp(8), vp(8), None) == rc.RC_EINVAL
    assert L.rc_composite(vp(8), 10, 0, vp(8), vp(8), vp(8), None) == rc.RC_EINVAL
    assert L.rc_composite(None, 8, 2, vp(8), vp(8), vp(8), None) == rc.RC_EINVAL
    assert rc.RC_MARCH_MAX_POINTS_PER_RAY == 1 << 20


def test_comparison_method_entries_reject_bad_arguments_without_a_device():
    L = rc.lib()
    vp = rc.C.c_void_p
    med = rc.rc_medium(1.0, 0.2)
    prm = rc.make_params(0.1, 20, 64, 1)
    args = (rc.C.byref(med), None, 0, vp(8), vp(8), vp(8), 4, rc.C.byref(prm))
    outs = (vp(8), vp(8), vp(8), vp(8), None)
    assert L.rc_j08_records(None, *args, 0.3, 1e-3, 0.4, *outs) == rc.RC_EINVAL  # no scene
    assert L.rc_interp_log(vp(8), vp(8), vp(8), vp(8), -1, vp(8), 4, vp(8), None, None) == rc.RC_EINVAL
    assert L.rc_interp_log(None, None, None, None, 3, vp(8), 4, vp(8), None, None) == rc.RC_EINVAL
    assert L.rc_interp_log(vp(8), vp(8), vp(8), vp(8), 3, None, 4, vp(8), None, None) == rc.RC_EINVAL
