"""Pins of the FP64 CPU oracle against things other than itself.

Each test checks the oracle against mathematics or published values:
closed forms, invariants, finite differences of independently computed
quantities, brute force, and a published generator test vector.  A plausible
mistake in the oracle (a dropped term, a wrong sign or index, a transposed
operand, a wrong constant) fails at least one of these.
"""
import math
from pathlib import Path

import numpy as np
import pytest
from scipy.special import expn

from oracle import oracle as O
from paper_1805_09258_amd import workloads as W

GOLDEN = Path(__file__).resolve().parent / "golden"
NO_LIGHTS = np.zeros((0, 4), np.float32)


# ---------------------------------------------------------------------------
# random numbers and sampling layout
# ---------------------------------------------------------------------------
def test_splitmix64_published_vector():
    vals = [int(l) for l in (GOLDEN / "splitmix64_seed1234567.txt").read_text().split("\n")
            if l.strip() and not l.startswith("#")]
    g = 0x9E3779B97F4A7C15
    got = [O.splitmix64((1234567 + i * g) % 2**64) for i in range(len(vals))]
    assert got == vals


def test_uniform_floats_are_24bit_and_uniform():
    u = np.array([O.unif(9, r, i, d) for r in range(40) for i in range(500) for d in range(2)])
    assert np.all(u >= 0) and np.all(u < 1)
    assert np.all(np.floor(u * 2**24) == u * 2**24)
    h, _ = np.histogram(u, bins=16, range=(0, 1))
    e = len(u) / 16
    chi2 = ((h - e) ** 2 / e).sum()
    assert chi2 < 40.0  # 15 dof, p ~ 5e-4
    # different dims / records decorrelated
    a = np.array([O.unif(9, 3, i, 0) for i in range(4000)])
    b = np.array([O.unif(9, 3, i, 1) for i in range(4000)])
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.05


@pytest.mark.parametrize("nth,nph", [(4, 16), (8, 32), (16, 64), (5, 7)])
def test_directions_lie_in_their_equal_area_strata(nth, nph):
    d = O.directions(11, 5, nth, nph).astype(np.float64)
    N = nth * nph
    assert d.shape == (N + 2, 3)
    assert np.array_equal(d[0], [0, 0, 1]) and np.array_equal(d[-1], [0, 0, -1])
    nrm = np.linalg.norm(d, axis=1)
    assert np.all(np.abs(nrm - 1) < 3e-7)
    for a in range(nth):
        for b in range(nph):
            w = d[1 + a * nph + b]
            z = w[2]
            # z-bands of equal width have equal area (Archimedes), phi split evenly
            assert 1 - 2 * (a + 1) / nth - 1e-6 <= z <= 1 - 2 * a / nth + 1e-6
            phi = math.atan2(w[1], w[0]) % (2 * math.pi)
            lo, hi = 2 * math.pi * b / nph, 2 * math.pi * (b + 1) / nph
            assert lo - 1e-5 <= phi <= hi + 1e-5 or (b == 0 and phi > 2 * math.pi - 1e-5)


def test_directions_uniform_on_sphere():
    # moments of the uniform distribution: E[w] = 0, E[w w^T] = I/3
    d = np.concatenate([O.directions(3, r, 8, 32)[1:-1] for r in range(60)]).astype(np.float64)
    assert np.abs(d.mean(0)).max() < 3e-3
    M = d.T @ d / len(d)
    assert np.abs(M - np.eye(3) / 3).max() < 3e-3


# ---------------------------------------------------------------------------
# angular triangulation: a closed, consistently oriented star mesh
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nth,nph,rec", [(4, 16, 0), (8, 32, 1), (16, 64, 2), (8, 32, 77)])
def test_triangulation_is_closed_star_mesh(nth, nph, rec):
    d = O.directions(5, rec, nth, nph)
    t = O.triangles(d, nth, nph)
    N = nth * nph
    assert t.shape == (2 * N, 3)
    dd = d.astype(np.float64)
    det = np.einsum("ij,ij->i", dd[t[:, 0]], np.cross(dd[t[:, 1]], dd[t[:, 2]]))
    assert np.all(det > 0)                       # no folded triangle
    edges = {}
    for a, b, c in t:
        for u, v in ((a, b), (b, c), (c, a)):
            edges[(u, v)] = edges.get((u, v), 0) + 1
    assert all(n == 1 for n in edges.values())
    assert all((v, u) in edges for (u, v) in edges)   # every edge shared, opposite orientation
    V, E, F = N + 2, len(edges) // 2, len(t)
    assert V - E + F == 2                        # sphere topology
    # with every vertex pushed to an arbitrary distance, the mesh still
    # encloses x: total solid angle 4 pi and translation-invariant (grad = H = 0)
    rng = np.random.default_rng(rec)
    dist = rng.uniform(0.05, 3.0, size=N + 2)
    Y = dd * dist[:, None]
    Fs, G, H, S = 0.0, np.zeros(3), np.zeros((3, 3)), 0.0
    for a, b, c in t:
        f, g, h = O.formfactor(Y[a], Y[b], Y[c])
        Fs += f
        G += g
        H += h
        S += np.abs(h).sum()
    assert abs(Fs - 1.0) < 1e-12
    assert np.abs(G).max() < 1e-11 * max(1.0, S)
    assert np.abs(H).max() < 1e-11 * S


# ---------------------------------------------------------------------------
# App. C: triangle form factor
# ---------------------------------------------------------------------------
def test_formfactor_octant_triangle():
    F, _, _ = O.formfactor([1, 0, 0], [0, 1, 0], [0, 0, 1])
    assert abs(F - 1.0 / 8.0) < 1e-15               # one octant = pi/2 sr


def test_formfactor_large_triangle_above_pi_branch():
    # a large near-planar triangle seen from just above its centroid covers
    # almost a hemisphere: Omega > pi needs the branch of atan2 (pi added)
    F, _, _ = O.formfactor([100, -50, -1e-2], [-100, -50, -1e-2], [0, 100, -1e-2])
    assert 0.25 < F < 0.5


def _quad_solid_angle(y1, y2, y3, n=400):
    """Solid angle by midpoint quadrature of cos(theta)/r^2 over the triangle."""
    y1, y2, y3 = map(np.asarray, (y1, y2, y3))
    e1, e2 = y2 - y1, y3 - y1
    nrm = np.cross(e1, e2)
    area = np.linalg.norm(nrm) / 2
    nh = nrm / np.linalg.norm(nrm)
    s = 0.0
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    m = (i + j) < n
    for off in ((1 / 3, 1 / 3), (2 / 3, 2 / 3)):
        u = (i[m] + off[0]) / n
        v = (j[m] + off[1]) / n
        ok = u + v <= 1
        p = y1 + u[ok, None] * e1 + v[ok, None] * e2
        r = np.linalg.norm(p, axis=1)
        s += np.sum(np.abs(p @ nh) / r ** 3)
    return s * area / n ** 2


@pytest.mark.parametrize("seed", range(4))
def test_formfactor_matches_solid_angle_quadrature(seed):
    rng = np.random.default_rng(seed)
    y = rng.uniform(-1, 1, size=(3, 3)) + np.array([0, 0, 1.5])
    F, _, _ = O.formfactor(*y)
    Om = _quad_solid_angle(*y)
    assert abs(F - Om / (4 * np.pi)) < 2e-4 * max(F, 1e-3)


def _fd(f, x, h):
    x = np.asarray(x, np.float64)
    g = np.zeros((3,) + np.shape(f(x)))
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        g[i] = (f(x + e) - f(x - e)) / (2 * h)
    return g


@pytest.mark.parametrize("seed", range(6))
def test_formfactor_derivatives_vs_finite_differences(seed):
    rng = np.random.default_rng(100 + seed)
    y = rng.uniform(-1, 1, size=(3, 3)) + rng.uniform(-1, 1, 3) * 3
    x0 = rng.uniform(-0.5, 0.5, 3)

    def Fx(x):
        return O.formfactor(*(y - x))[0]

    def Gx(x):
        return O.formfactor(*(y - x))[1]

    F, g, H = O.formfactor(*(y - x0))
    gfd = _fd(Fx, x0, 1e-5)
    Hfd = _fd(Gx, x0, 1e-5)            # rows: d/dx_i of grad
    assert np.linalg.norm(g - gfd) <= 1e-7 * np.linalg.norm(g) + 1e-12
    assert np.linalg.norm(H - Hfd.T) <= 1e-6 * np.linalg.norm(H) + 1e-10
    assert np.linalg.norm(H - H.T) <= 1e-12 * np.linalg.norm(H)


def test_paper_boxed_gradA_sign_reading():
    """App. C boxes grad A = <r3 - r2> r1 - (r2 x r3).  Finite differences of
    A = r1 . (r2 x r3) (r_i = y_i - x) contradict it and confirm
    grad A = -(r1 x r2 + r2 x r3 + r3 x r1), the reading the oracle uses."""
    rng = np.random.default_rng(5)
    y = rng.uniform(-1, 1, size=(3, 3))
    x0 = rng.uniform(-0.3, 0.3, 3)

    def A(x):
        r = y - x
        return float(np.dot(r[0], np.cross(r[1], r[2])))

    gfd = _fd(A, x0, 1e-6)
    r1, r2, r3 = y - x0
    boxed = np.cross(r3 - r2, r1) - np.cross(r2, r3)
    ours = -(np.cross(r1, r2) + np.cross(r2, r3) + np.cross(r3, r1))
    assert np.linalg.norm(ours - gfd) < 1e-8 * np.linalg.norm(gfd)
    assert np.linalg.norm(boxed - gfd) > 0.1 * np.linalg.norm(gfd)
    # and the oracle's grad F is consistent with the corrected grad A
    F, g, _ = O.formfactor(r1, r2, r3)
    gfdF = _fd(lambda x: O.formfactor(*(y - x))[0], x0, 1e-6)
    assert np.linalg.norm(g - gfdF) < 1e-6 * np.linalg.norm(g)


# ---------------------------------------------------------------------------
# App. A: transmittance
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mu", [0.0, 0.3, 2.5])
def test_transmittance_closed_form_and_fd(mu):
    y = np.array([0.3, -0.2, 0.9])
    x0 = np.array([-0.1, 0.25, 0.05])
    T, g, H = O.transmittance(x0, y, mu)
    assert abs(T - math.exp(-mu * np.linalg.norm(x0 - y))) < 1e-15
    gfd = _fd(lambda x: O.transmittance(x, y, mu)[0], x0, 1e-5)
    Hfd = _fd(lambda x: O.transmittance(x, y, mu)[1], x0, 1e-5)
    assert np.linalg.norm(g - gfd) <= 1e-8 * max(np.linalg.norm(g), 1e-12) + 1e-14
    assert np.linalg.norm(H - Hfd) <= 1e-7 * max(np.linalg.norm(H), 1e-12) + 1e-12


# ---------------------------------------------------------------------------
# whole records: closed forms
# ---------------------------------------------------------------------------
def _emitting_box_scene(extra_tri=None, lo=(0, 0, 0), hi=(1, 1, 1)):
    box = W.room_triangles(lo, hi)
    tri = box if extra_tri is None else np.concatenate([box, extra_tri])
    em = np.zeros(len(tri), np.float32)
    em[:12] = 1.0
    return O.Scene(tri.astype(np.float32), np.zeros(len(tri), np.float32), em, lo, hi)


def test_uniform_unoccluded_field_has_zero_derivatives():
    sc = _emitting_box_scene()
    rng = np.random.default_rng(3)
    pts = rng.uniform(0.1, 0.9, size=(12, 3)).astype(np.float32)
    r = O.records(sc, 0.0, 0.0, NO_LIGHTS, pts, 8, 32, ring_step=0.1, max_rings=20, seed=4)
    st = r["stats"]
    assert np.allclose(r["value"][:, 0], 1.0, atol=1e-15)
    assert np.allclose(r["value"][:, 1], 0.0)
    assert np.allclose(st[:, 7], 1.0, atol=1e-12)                 # sum of form factors
    assert np.all(np.linalg.norm(r["grad"][:, 0], axis=1) < 1e-11 * st[:, 3])
    assert np.all(np.linalg.norm(r["hess"][:, 0], axis=1) < 1e-11 * st[:, 4])



NEAR_SURFACE = [(0.5, 0.5, "h"), (0.3, 0.6, "1-h"), ("h", "h", 0.5), ("1-h", 0.4, "1-h"), ("h", "h", "h"),
                ("1-h", "1-h", "1-h"), ("h", "1-h", "h")]


def _near_point(spec, h):
    return [h if c == "h" else (1 - h if c == "1-h" else c) for c in spec]


@pytest.mark.parametrize("h", [1e-3, 1e-4, 1e-5])
def test_closed_emitting_box_seen_from_points_next_to_walls_edges_and_corners(h):
    """Sec. 4 takes each sample at the first surface seen from x.  Inside a
    closed emitting box in vacuum every direction sees a wall, so V_SS = 1
    and the triangulated gradient and Hessian vanish (the fan of hit points
    is a closed star mesh around x) for points arbitrarily close to a wall,
    an edge or a corner; a ray/triangle test that drops grazing rays loses
    directions here and the value falls short of 1."""
    sc = _emitting_box_scene()
    pts = np.array([_near_point(s_, h) for s_ in NEAR_SURFACE], np.float32)
    for seed in (5, 6):
        r = O.records(sc, 0.0, 0.0, NO_LIGHTS, pts, 32, 128, ring_step=0.1, max_rings=20, seed=seed)
        st = r["stats"]
        assert np.abs(r["value"][:, 0] - 1.0).max() < 1e-6, r["value"][:, 0]
        assert np.allclose(r["value"][:, 1], 0.0)
        assert np.abs(st[:, 7] - 1.0).max() < 1e-9                  # sum of form factors
        assert np.all(np.linalg.norm(r["grad"][:, 0], axis=1) <= 1e-11 * st[:, 3])
        assert np.all(np.linalg.norm(r["hess"][:, 0], axis=1) <= 1e-11 * st[:, 4])


def _closed_meshes():
    """Closed triangle meshes around the origin with shared vertices: an
    octahedron, a cube split along its face diagonals, and a subdivided
    icosphere-like mesh (random radial perturbation)."""
    octa_v = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.float64)
    octa_f = [(0, 2, 4), (2, 1, 4), (1, 3, 4), (3, 0, 4), (2, 0, 5), (1, 2, 5), (3, 1, 5), (0, 3, 5)]
    cube = W.room_triangles((-1, -1, -1), (1, 1, 1)).reshape(-1, 3, 3).astype(np.float64)
    rng = np.random.default_rng(11)
    v, f = octa_v.copy(), list(octa_f)
    for _ in range(3):   # loop subdivision of the faces (midpoints shared between neighbours)
        mids, nf = {}, []
        def mid(a, b):
            k = (min(a, b), max(a, b))
            if k not in mids:
                mids[k] = len(v_list)
                v_list.append((v_list[a] + v_list[b]) / 2)
            return mids[k]
        v_list = list(v)
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        v, f = np.array(v_list), nf
    v = v / np.linalg.norm(v, axis=1, keepdims=True) * rng.uniform(0.7, 1.3, size=(len(v), 1))
    sphere = v[np.array(f)]
    return [octa_v[np.array(octa_f)], cube, sphere]


def test_rays_through_shared_edges_and_vertices_of_closed_meshes_always_hit():
    """Watertightness: rays from inside a closed mesh aimed exactly at its
    vertices, at points of its edges, and in random directions always hit
    one of its triangles (brute force and hierarchy agree)."""
    rng = np.random.default_rng(12)
    for mesh in _closed_meshes():
        tri = mesh.reshape(-1, 9).astype(np.float32)
        sc = O.Scene(tri, np.zeros(len(tri), np.float32), None, (-2, -2, -2), (2, 2, 2))
        t3 = tri.reshape(-1, 3, 3).astype(np.float64)
        targets = [t3.reshape(-1, 3)]
        for a, b in ((0, 1), (1, 2), (2, 0)):
            for f in (0.5, 0.25, rng.uniform()):
                targets.append(t3[:, a] + f * (t3[:, b] - t3[:, a]))
        targets = np.concatenate(targets)
        for o in (np.zeros(3), rng.uniform(-0.2, 0.2, 3), np.array([0.3, -0.1, 0.05])):
            o32 = np.broadcast_to(o, targets.shape).astype(np.float32)
            d = (targets - o32).astype(np.float32)
            d = np.concatenate([d, rng.normal(size=(3000, 3)).astype(np.float32)])
            o32 = np.broadcast_to(o, d.shape).astype(np.float32)
            for brute in (True, False):
                hid, t, _ = sc.trace(o32, d, brute=brute)
                assert (hid >= 0).all(), (len(tri), int((hid < 0).sum()))


def _grazing_rays(tri, rng, n):
    """Rays that skim random triangles: origin near the triangle's plane,
    direction in the plane tilted by 1e-7 .. 1e-2 rad, aimed at the triangle
    or just past one of its edges."""
    T = len(tri)
    t3 = tri.reshape(-1, 3, 3).astype(np.float64)
    j = rng.integers(0, T, n)
    v0, v1, v2 = t3[j, 0], t3[j, 1], t3[j, 2]
    nrm = np.cross(v1 - v0, v2 - v0)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    bc = rng.dirichlet([1, 1, 1], size=n) * 1.1 - 0.033
    tgt = bc[:, :1] * v0 + bc[:, 1:2] * v1 + bc[:, 2:] * v2
    u = rng.normal(size=(n, 3))
    u -= (u * nrm).sum(1, keepdims=True) * nrm
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    ang = 10.0 ** rng.uniform(-7, -2, n) * rng.choice([-1, 1], n)
    d = u * np.cos(ang)[:, None] + nrm * np.sin(ang)[:, None]
    dist = rng.uniform(0.01, 0.5, n)
    o = tgt - d * dist[:, None]
    return o.astype(np.float32), (d * rng.uniform(0.5, 2.0, (n, 1))).astype(np.float32)


def test_grazing_rays_hierarchy_equals_brute_force_and_hits_stay_in_padding():
    """Rays skimming triangles at 1e-7 .. 1e-2 rad: the hierarchy of padded
    boxes gives the brute-force closest hit and any-hit answers, and every
    accepted hit point o + t d lies within 16 * 2^-24 * scale of its
    triangle's box (the bound the box padding of 2^-16 * scale covers)."""
    w = W.make_c2(P=4, n_soup=2000)
    sc = O.Scene.from_workload(w)
    rng = np.random.default_rng(13)
    o, d = _grazing_rays(w.tri, rng, 20000)
    keep = np.all((o > 0.0) & (o < 1.0), axis=1)
    o, d = o[keep], d[keep]
    a = sc.trace(o, d, brute=False)
    b = sc.trace(o, d, brute=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    hit = a[0] >= 0
    assert hit.mean() > 0.3
    t3 = w.tri.reshape(-1, 3, 3).astype(np.float64)[a[0][hit]]
    hp = o[hit].astype(np.float64) + a[1][hit].astype(np.float64)[:, None] * d[hit].astype(np.float64)
    out = np.maximum(t3.min(1) - hp, hp - t3.max(1)).max(1)
    scale = float((w.box_hi - w.box_lo).max())
    assert out.max() <= 16 * 2.0 ** -24 * scale, out.max()
    seg = d * rng.uniform(0.2, 3.0, (len(d), 1)).astype(np.float32)
    assert np.array_equal(sc.occluded(o, seg), sc.occluded(o, seg, brute=True))


def _rect_omega(p, x1, x2, y1, y2):
    """Solid angle of the rectangle [x1,x2]x[y1,y2] in the plane z = 0 seen
    from p (textbook corner formula)."""
    h = p[2]

    def F(a, b):
        return np.arctan(a * b / (h * np.sqrt(a * a + b * b + h * h)))

    X1, X2, Y1, Y2 = x1 - p[0], x2 - p[0], y1 - p[1], y2 - p[1]
    return F(X2, Y2) - F(X1, Y2) - F(X2, Y1) + F(X1, Y1)


def _fd_grad_hess(f, p, h=1e-4):
    g = np.zeros(3)
    H = np.zeros((3, 3))
    E = np.eye(3) * h
    for i in range(3):
        g[i] = (f(p + E[i]) - f(p - E[i])) / (2 * h)
        for j in range(3):
            H[i, j] = (f(p + E[i] + E[j]) - f(p + E[i] - E[j]) - f(p - E[i] + E[j]) + f(p - E[i] - E[j])) / (4 * h * h)
    return g, H


def test_black_occluder_in_uniform_field_converges_to_closed_form():
    """Vacuum, every wall of the box emits 1, a black rectangle hangs inside.
    V(x) = 1 - Omega_rect(x)/(4 pi) exactly; its gradient and Hessian are the
    occlusion derivatives.  The triangulated estimator is biased but
    consistent (Sec. 4): errors must fall roughly like N^-1/2."""
    x1, x2, y1, y2 = -0.3, 0.3, -0.2, 0.2
    rect = np.array([[x1, y1, 0, x2, y1, 0, x2, y2, 0], [x1, y1, 0, x2, y2, 0, x1, y2, 0]], np.float32)
    sc = _emitting_box_scene(rect, (-1, -1, -1), (1, 1, 1))
    pts = np.array([[0.25, 0.1, 0.15], [0.0, 0.0, 0.3], [0.35, -0.1, 0.1], [-0.5, 0.3, 0.4]], np.float32)
    errs = {}
    for N in (1024, 4096, 16384):
        nt, npf = W.strata_shape(N)
        eg, eh = [], []
        for s in range(4):
            r = O.records(sc, 0.0, 0.0, NO_LIGHTS, pts, nt, npf, ring_step=0.1, max_rings=0, seed=100 + s)
            for k, p in enumerate(pts.astype(np.float64)):
                f = lambda q: 1 - _rect_omega(q, x1, x2, y1, y2) / (4 * np.pi)  # noqa: E731
                g, H = _fd_grad_hess(f, p)
                if N == 16384:
                    assert abs(r["value"][k, 0] - f(p)) < 3e-3
                eg.append(np.linalg.norm(r["grad"][k, 0] - g) / np.linalg.norm(g))
                eh.append(np.linalg.norm(O.hess6_to_mat(r["hess"][k, 0]) - H) / np.linalg.norm(H))
        errs[N] = (np.mean(eg), np.mean(eh))
    slope_g = math.log(errs[16384][0] / errs[1024][0]) / math.log(16)
    slope_h = math.log(errs[16384][1] / errs[1024][1]) / math.log(16)
    assert slope_g < -0.35 and slope_h < -0.35, errs
    assert errs[16384][0] < 0.10 and errs[16384][1] < 0.10, errs


def test_emitting_plane_under_medium_matches_exponential_integrals():
    """Emitter L_e = 1 on z = 0, homogeneous absorbing medium above, point at
    height h: V = E2(mu h)/2, dV/dz = -mu E1(mu h)/2,
    d2V/dz2 = mu exp(-mu h)/(2h), lateral derivatives 0."""
    Wd = 30.0
    floor = np.array([[-Wd, -Wd, 0, Wd, -Wd, 0, Wd, Wd, 0], [-Wd, -Wd, 0, Wd, Wd, 0, -Wd, Wd, 0]], np.float32)
    sc = O.Scene(floor, np.zeros(2, np.float32), np.ones(2, np.float32), (-Wd, -Wd, 0), (Wd, Wd, 4))
    mu, h = 1.0, 0.5
    V = expn(2, mu * h) / 2
    Gz = -mu * expn(1, mu * h) / 2
    Hzz = mu * math.exp(-mu * h) / (2 * h)
    res = {}
    for N in (1024, 16384):
        nt, npf = W.strata_shape(N)
        r = O.records(sc, 0.0, mu, NO_LIGHTS, np.array([[0.1, -0.2, h]] * 8, np.float32), nt, npf,
                      ring_step=0.1, max_rings=0, seed=7)
        res[N] = (r["value"][:, 0].mean(), r["grad"][:, 0].mean(0), r["hess"][:, 0].mean(0))
    v, g, H = res[16384]
    assert abs(v - V) < 2e-4
    assert abs(g[2] - Gz) / abs(Gz) < 0.02
    assert abs(H[5] - Hzz) / Hzz < 0.02
    assert np.abs(g[:2]).max() < 1e-3 and abs(H[1]) < 1e-2 and abs(H[2]) < 1e-2 and abs(H[4]) < 1e-2
    # consistency: the error shrinks with N
    assert abs(res[16384][1][2] - Gz) < 0.5 * abs(res[1024][1][2] - Gz)
    assert abs(res[16384][2][5] - Hzz) < 0.5 * abs(res[1024][2][5] - Hzz)


def test_record_derivatives_are_exact_calculus_of_triangulated_value():
    """With the vertices frozen, the oracle's gradient and Hessian must be the
    exact derivatives of sum_j w L_far T(x, y_far) F_j(x): checked by central
    differences of the triangulated value and of the gradient."""
    w = W.make_c1(P=6)
    sc = O.Scene.from_workload(w)
    idx = np.arange(6)
    base = O.records_for(w, idx, scene=sc, xeval=w.pos.astype(np.float64))
    h = 1e-6
    for c, st in ((0, 7), (1, 8)):
        gfd = np.zeros((6, 3))
        Hfd = np.zeros((6, 3, 3))
        for i in range(3):
            e = np.zeros(3)
            e[i] = h
            rp = O.records_for(w, idx, scene=sc, xeval=w.pos.astype(np.float64) + e)
            rm = O.records_for(w, idx, scene=sc, xeval=w.pos.astype(np.float64) - e)
            gfd[:, i] = (rp["stats"][:, st] - rm["stats"][:, st]) / (2 * h)
            Hfd[:, i, :] = (rp["grad"][:, c] - rm["grad"][:, c]) / (2 * h)
        G = base["grad"][:, c]
        H = O.hess6_to_mat(base["hess"][:, c])
        for k in range(6):
            sg = base["stats"][k, 3 + 2 * c]
            sh = base["stats"][k, 4 + 2 * c]
            assert np.linalg.norm(G[k] - gfd[k]) <= 1e-6 * sg + 1e-12
            assert np.linalg.norm(H[k] - 0.5 * (Hfd[k] + Hfd[k].T)) <= 1e-5 * sh + 1e-10


def test_hessian_paper_form_is_symmetric_on_records():
    w = W.make_c1(P=16)
    r = O.records_for(w)
    assert np.all(r["stats"][:, 9] < 1e-9)


def test_mc_value_of_uniform_medium_vertex_radiance():
    """MS channel in an open box with no geometry, one light, no absorption
    along the light path: compare the ring Monte Carlo estimator with direct
    numerical integration over a sphere of directions and distances."""
    lo, hi = np.zeros(3, np.float32), np.ones(3, np.float32)
    sc = O.Scene(np.zeros((0, 9), np.float32), np.zeros(0, np.float32), None, lo, hi)
    light = np.array([[0.5, 0.95, 0.5, 10.0]], np.float32)
    x = np.array([[0.4, 0.3, 0.55]], np.float32)
    ss, sa = 0.5, 0.1
    mu = ss + sa
    vals = [O.records(sc, ss, sa, light, x, 16, 64, rec_id=[r], ring_step=0.05, max_rings=40,
                      seed=21)["value"][0, 1] for r in range(24)]
    # reference: (1/4pi) int dw int_0^s(w) mu_s/(4pi) I e^{-mu t} e^{-mu d}/d^2 dt
    n = 200
    u = (np.arange(n) + 0.5) / n
    z = 1 - 2 * u
    phi = 2 * np.pi * (np.arange(2 * n) + 0.5) / (2 * n)
    Z, PH = np.meshgrid(z, phi, indexing="ij")
    st = np.sqrt(1 - Z * Z)
    dirs = np.stack([st * np.cos(PH), st * np.sin(PH), Z], -1).reshape(-1, 3)
    x0 = x[0].astype(np.float64)
    with np.errstate(divide="ignore"):
        t_exit = np.min(np.where(dirs > 0, (1 - x0) / dirs, np.where(dirs < 0, -x0 / dirs, np.inf)), axis=1)
    ref = 0.0
    m = 400
    for k, wv in enumerate(dirs):
        t = (np.arange(m) + 0.5) / m * t_exit[k]
        y = x0 + t[:, None] * wv
        d = np.linalg.norm(light[0, :3].astype(np.float64) - y, axis=1)
        f = ss / (4 * np.pi) * 10.0 * np.exp(-mu * t) * np.exp(-mu * d) / d ** 2
        ref += f.sum() * t_exit[k] / m
    ref *= (4 * np.pi / len(dirs)) / (4 * np.pi)
    assert abs(np.mean(vals) - ref) / ref < 0.01


# ---------------------------------------------------------------------------
# ray decisions
# ---------------------------------------------------------------------------
def test_hierarchical_trace_equals_brute_force():
    w = W.make_c2(P=4, n_soup=3000)
    sc = O.Scene.from_workload(w)
    rng = np.random.default_rng(8)
    n = 6000
    o = rng.uniform(0.02, 0.98, size=(n, 3)).astype(np.float32)
    d = rng.normal(size=(n, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    a = sc.trace(o, d, brute=False)
    b = sc.trace(o, d, brute=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    seg = (rng.uniform(0, 1, size=(n, 3)) - o).astype(np.float32)
    skip = np.where(a[0] >= 0, a[0], -1)
    assert np.array_equal(sc.occluded(o, seg, skip), sc.occluded(o, seg, skip, brute=True))


def test_trace_decisions_agree_with_exact_geometry_away_from_edges():
    """Rays aimed at interior points of random triangles (barycentric margin
    >= 0.05, no nearer triangle) must hit exactly that triangle at the exact
    FP64 distance (to FP32 rounding)."""
    rng = np.random.default_rng(2)
    tri = rng.uniform(-1, 1, size=(30, 3, 3))
    tri[:, :, 2] += np.arange(30)[:, None] * 0.0 + 5.0 + np.arange(30)[:, None] * 0.5
    sc = O.Scene(tri.reshape(-1, 9).astype(np.float32), np.zeros(30, np.float32), None, (-10, -10, -10), (10, 10, 30))
    o = np.zeros((30, 3), np.float32)
    bc = rng.dirichlet([1, 1, 1], size=30) * 0.85 + 0.05
    tgt = np.einsum("nk,nkj->nj", bc, tri)
    d = (tgt / np.linalg.norm(tgt, axis=1, keepdims=True)).astype(np.float32)
    hid, t, _ = sc.trace(o, d, brute=True)
    # exact first hit in FP64 (Moller-Trumbore in numpy, double precision)
    for i in range(30):
        best, bj = np.inf, -1
        for j in range(30):
            v0, v1, v2 = tri[j]
            e1, e2 = v1 - v0, v2 - v0
            p = np.cross(d[i].astype(np.float64), e2)
            det = e1 @ p
            s = -v0
            u = s @ p / det
            q = np.cross(s, e1)
            v = d[i].astype(np.float64) @ q / det
            tt = e2 @ q / det
            if u >= 0 and v >= 0 and u + v <= 1 and tt > 0 and tt < best:
                best, bj = tt, j
        assert hid[i] == bj
        assert abs(t[i] - best) <= 1e-5 * best


# ---------------------------------------------------------------------------
# Sec. 5: radius and interpolation
# ---------------------------------------------------------------------------
def test_radius_constant_integrates_the_error_bound_to_eps():
    """With R = (15 L eps / (4 pi |lambda|))^(1/5) the bound of Eq. S.11 for a
    single axis, integral over the ball of |lambda| x1^2 / L, equals eps."""
    L, lam, eps = 0.7, -3.2, 1.5e-4
    H = np.zeros(6)
    H[0] = lam
    R = O.radius(np.array([L]), H[None, :], eps, 1e-9, 1e9)[0]
    # spherical-shell quadrature of x1^2 over the ball: 4 pi R^5 / 15
    n = 2000
    r = (np.arange(n) + 0.5) / n * R
    ct = (np.arange(n) + 0.5) / n * 2 - 1
    integ = 0.0
    for c in ct[::10]:
        integ += np.sum(r ** 2 * r ** 2 * c ** 2) * (R / n) * (2.0 / (n / 10)) * 2 * np.pi
    assert abs(abs(lam) * integ / L - eps) / eps < 1e-3
    # two dimensions: the paper's 2-D constant (4/pi) comes from pi R^4 / 4
    R2 = (4 * L * eps / (np.pi * abs(lam))) ** 0.25
    ints = np.sum(((np.arange(n) + 0.5) / n * R2) ** 3) * (R2 / n) * np.pi  # int r^2 cos^2 r dr dphi
    assert abs(abs(lam) * ints / L - eps) / eps < 1e-3


def test_radius_edge_cases_and_isotropic_choice():
    H = np.array([[1.0, 0, 0, -8.0, 0, 2.0], [0, 0, 0, 0, 0, 0], [1, 0, 0, 1, 0, 1], [1, 0, 0, 1, 0, 1]])
    L = np.array([1.0, 1.0, 0.0, 2.0])
    R, Ri, vec = O.radius(L, H, 1.5e-4, 1e-3, 0.4, anisotropic=True)
    assert abs(R[0] - (15 * 1.0 * 1.5e-4 / (4 * np.pi * 8.0)) ** 0.2) < 1e-12   # largest |lambda|
    assert R[1] == 0.4                      # lambda = 0 -> r_max
    assert R[2] == 1e-3                     # L <= 0 -> r_min
    assert np.all(Ri[0] >= R[0])
    # rotating the Hessian rotates the axes and keeps the radii
    Q = np.linalg.qr(np.random.default_rng(0).normal(size=(3, 3)))[0]
    Hm = O.hess6_to_mat(H[0])
    Hr = Q @ Hm @ Q.T
    h6 = np.array([Hr[0, 0], Hr[0, 1], Hr[0, 2], Hr[1, 1], Hr[1, 2], Hr[2, 2]])
    assert abs(O.radius(L[:1], h6[None], 1.5e-4, 1e-3, 0.4)[0] - R[0]) < 1e-12


def test_interpolation_reproduces_linear_fields_and_kernel():
    rng = np.random.default_rng(1)
    cp = rng.uniform(0, 1, size=(20, 3))
    a, g = 0.7, np.array([0.3, -0.2, 0.5])
    cv = a + cp @ g
    cg = np.tile(g, (20, 1))
    cR = np.full(20, 0.45)
    q = rng.uniform(0.2, 0.8, size=(50, 3))
    L, cov = O.interpolate(cp, cv, cg, cR, q)
    assert cov.all()
    assert np.allclose(L, a + q @ g, atol=1e-12)      # first-order Taylor is exact for linear fields
    # kernel: single point, weight irrelevant; outside radius -> not covered
    L1, c1 = O.interpolate(cp[:1], cv[:1], cg[:1] * 0, np.array([0.1]), cp[:1] + [0.2, 0, 0])
    assert not c1[0]
    # two points, equal values 1 and 3: weights 3d^2 - 2d^3 at d = 1 - dist/R
    cp2 = np.array([[0, 0, 0], [1, 0, 0]], float)
    L2, _ = O.interpolate(cp2, np.array([1.0, 3.0]), np.zeros((2, 3)), np.array([2.0, 2.0]), [[0.25, 0, 0]])
    d1, d2 = 1 - 0.25 / 2, 1 - 0.75 / 2
    w1, w2 = 3 * d1 ** 2 - 2 * d1 ** 3, 3 * d2 ** 2 - 2 * d2 ** 3
    assert abs(L2[0] - (w1 * 1 + w2 * 3) / (w1 + w2)) < 1e-14


# ---------------------------------------------------------------------------
# MLP reference
# ---------------------------------------------------------------------------
def _mlp_params(rng):
    return {"W1": rng.normal(size=(128, 32)) * 0.2, "b1": rng.normal(size=128) * 0.1,
            "W2": rng.normal(size=(128, 128)) * 0.1, "b2": rng.normal(size=128) * 0.1,
            "W3": rng.normal(size=(1, 128)) * 0.1, "b3": rng.normal(size=1) * 0.1}


def test_gelu_matches_erf_form_closely_and_its_derivative():
    from scipy.special import erf
    x = np.linspace(-5, 5, 2001)
    exact = 0.5 * x * (1 + erf(x / np.sqrt(2)))
    assert np.abs(O.gelu(x) - exact).max() < 1e-3          # tanh approximation of the erf form
    h = 1e-6
    assert np.abs(O.gelu_grad(x) - (O.gelu(x + h) - O.gelu(x - h)) / (2 * h)).max() < 1e-8


def test_mlp_gradients_vs_finite_differences():
    rng = np.random.default_rng(4)
    p = _mlp_params(rng)
    X = rng.normal(size=(16, 32))
    y = rng.normal(size=16)
    loss, g = O.mlp_loss_grad(p, X, y)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(5, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = O.mlp_loss_grad(p, X, y)
            flat[idx] = old - h
            lm, _ = O.mlp_loss_grad(p, X, y)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(g[k].reshape(-1)[idx] - fd) <= 1e-6 * max(1.0, abs(fd))


def test_adam_first_step_is_signed_lr():
    p = {"a": np.array([1.0, -2.0, 3.0])}
    g = {"a": np.array([0.5, -1e-3, 2.0])}
    m = {"a": np.zeros(3)}
    v = {"a": np.zeros(3)}
    O.adam_step(p, g, m, v, 1, 0.01)
    assert np.allclose(p["a"], [1.0 - 0.01, -2.0 + 0.01, 3.0 - 0.01], atol=1e-7)


def test_lit_lambertian_floor_matches_surface_quadrature():
    """SS value of a point above a Lambertian floor lit by a point light in a
    homogeneous medium, against direct quadrature over the floor:
    V = 1/(4 pi) int (rho/pi) I cos_l e^{-mu d_l} / d_l^2 e^{-mu r} cos_y / r^2 dA."""
    Wd = 2.0
    floor = np.array([[-Wd, -Wd, 0, Wd, -Wd, 0, Wd, Wd, 0], [-Wd, -Wd, 0, Wd, Wd, 0, -Wd, Wd, 0]], np.float32)
    sc = O.Scene(floor, np.full(2, 0.5, np.float32), None, (-Wd, -Wd, 0), (Wd, Wd, 3))
    light = np.array([[0.3, 0.2, 1.0, 5.0]], np.float32)
    x = np.array([-0.2, 0.1, 0.4])
    ss, sa = 0.0, 0.4
    mu = ss + sa
    vals = [O.records(sc, ss, sa, light, x[None].astype(np.float32), 32, 128, rec_id=[r], ring_step=0.1,
                      max_rings=0, seed=3)["value"][0, 0] for r in range(6)]
    n = 1200
    g = (np.arange(n) + 0.5) / n * 2 * Wd - Wd
    X, Y = np.meshgrid(g, g, indexing="ij")
    P = np.stack([X, Y, np.zeros_like(X)], -1)
    dl = light[0, :3].astype(np.float64) - P
    d = np.linalg.norm(dl, axis=-1)
    cl = dl[..., 2] / d
    Ls = 0.5 / np.pi * 5.0 * cl * np.exp(-mu * d) / d ** 2
    rv = x - P
    r = np.linalg.norm(rv, axis=-1)
    cy = rv[..., 2] / r
    ref = np.sum(Ls * np.exp(-mu * r) * cy / r ** 2) * (2 * Wd / n) ** 2 / (4 * np.pi)
    assert abs(np.mean(vals) - ref) / ref < 3e-3


# ---------------------------------------------------------------------------
# Medium rings: gradient against finite differences of brute-force values
# ---------------------------------------------------------------------------
MS_SQUARE = np.array([[0.35, 0.35, 0.6, 0.65, 0.35, 0.6, 0.65, 0.65, 0.6],
                      [0.35, 0.35, 0.6, 0.65, 0.65, 0.6, 0.35, 0.65, 0.6]], np.float32)
# one light outside the medium box, in the square's plane: it lights every
# medium point (the square casts no shadow into the box) and no ring vertex
# comes near it, so the medium radiance is smooth and only the square's
# occlusion of the rings, as seen from x, is discontinuous
MS_LIGHT = np.array([[1.6, 0.5, 0.6, 40.0]], np.float32)
MS_POINTS = np.array([[0.5, 0.5, 0.45], [0.42, 0.55, 0.5], [0.58, 0.45, 0.4]])


def ms_fd_gradient(sc, h=0.01, nbf=(256, 1024), seeds=16, sigma=(1.0, 0.2), step=0.1, max_rings=20):
    """Central differences of brute-force Monte Carlo MS values (nbf strata,
    common random numbers at x +- h e_i), averaged over seeds: mean, stderr."""
    E = np.eye(3)
    pos = np.array([p + sg * h * E[i] for p in MS_POINTS for i in range(3) for sg in (1, -1)], np.float32)
    P = pos.reshape(len(MS_POINTS), 3, 2, 3).astype(np.float64)
    G = np.zeros((seeds, len(MS_POINTS), 3))
    for s in range(seeds):
        v = O.values(sc, sigma[0], sigma[1], MS_LIGHT, pos, nbf[0], nbf[1], rec_id=3, ring_step=step,
                     max_rings=max_rings, seed=2000 + s)[:, 1].reshape(len(MS_POINTS), 3, 2)
        for i in range(3):
            G[s, :, i] = (v[:, i, 0] - v[:, i, 1]) / (P[:, i, 0, i] - P[:, i, 1, i])
    return G.mean(0), G.std(0) / np.sqrt(seeds)


def ms_triangulated_gradient(sc, N, seeds=16, sigma=(1.0, 0.2), step=0.1, max_rings=20):
    nt, npf = W.strata_shape(N)
    g = [O.records(sc, sigma[0], sigma[1], MS_LIGHT, MS_POINTS.astype(np.float32), nt, npf, ring_step=step,
                   max_rings=max_rings, seed=500 + s)["grad"][:, 1] for s in range(seeds)]
    return np.mean(g, 0)


def ms_gradient_errors():
    """Relative error of the triangulated MS gradient (mean over seeds) against
    the finite-difference reference, per N in (1k, 4k, 16k), averaged over
    the points; and the reference's own relative standard error."""
    sc = O.Scene(MS_SQUARE, np.zeros(2, np.float32), None, (0, 0, 0), (1, 1, 1))
    ref, se = ms_fd_gradient(sc)
    errs = []
    for N in (1024, 4096, 16384):
        g = ms_triangulated_gradient(sc, N)
        errs.append(float(np.mean(np.linalg.norm(g - ref, axis=1) / np.linalg.norm(ref, axis=1))))
    del sc
    return np.array(errs), float(np.max(np.linalg.norm(se, axis=1) / np.linalg.norm(ref, axis=1)))


def test_medium_ring_gradient_converges_to_fd_of_brute_force_values():
    """Sec. 4: occluders closer than a ring put its vertex at the occluder with
    zero radiance, so the medium-ring gradient carries the occlusion of the
    medium behind them.  A black square in front of points in a lit medium:
    the triangulated MS gradient converges, with N^-1/2 or faster, to central
    differences of brute-force Monte Carlo values (65 536 strata, common random
    numbers, 16 seeds), whose standard error stays below 4 %."""
    errs, rel_se = ms_gradient_errors()
    print("MS gradient errors at 1k, 4k, 16k:", np.round(errs, 4), "reference rel. stderr", round(rel_se, 4))
    assert rel_se < 0.04, rel_se
    slope = np.polyfit(np.log([1024, 4096, 16384]), np.log(errs), 1)[0]
    assert slope <= -0.35 and errs[-1] <= 0.08, (errs, slope)


# ---------------------------------------------------------------------------
# Anisotropic cache points (Sec. 5, Eq. radiusAniso3D: ellipsoidal valid
# regions along the Hessian's eigenvectors)
# ---------------------------------------------------------------------------
def _random_axes(rng, K, lo=0.02, hi=0.3):
    R = rng.uniform(lo, hi, (K, 3)).astype(np.float32)
    V = np.stack([np.linalg.qr(rng.normal(size=(3, 3)))[0].T for _ in range(K)]).astype(np.float32)
    return R, V


def _form_matrix(f):
    f = np.asarray(f, np.float64)
    return np.array([[f[0], f[1], f[2]], [f[1], f[3], f[4]], [f[2], f[4], f[5]]])


def test_ellipsoid_form_has_the_axes_as_eigenvectors():
    rng = np.random.default_rng(501)
    R, V = _random_axes(rng, 64)
    F = O.ellipsoid_form(R, V)
    for k in range(64):
        M = _form_matrix(F[k])
        for i in range(3):
            v = V[k, i].astype(np.float64)
            np.testing.assert_allclose(M @ v, v / float(R[k, i]) ** 2, rtol=0, atol=2e-5 / float(R[k, i]) ** 2)


def test_ellipsoid_membership_along_and_off_the_axes():
    rng = np.random.default_rng(502)
    R, V = _random_axes(rng, 40)
    F = O.ellipsoid_form(R, V)
    p = rng.uniform(0.3, 0.7, (40, 3)).astype(np.float32)
    for k in range(40):
        for i in range(3):
            for s, inside in ((0.999, True), (1.001, False), (-0.999, True), (-1.001, False)):
                q = (p[k].astype(np.float64) + s * float(R[k, i]) * V[k, i]).astype(np.float32)
                assert bool(O._within_form32(q, p[k], F[k])) == inside, (k, i, s)
    # random offsets: the FP32 decision equals the exact one away from the surface
    for k in range(40):
        d = rng.uniform(-0.35, 0.35, (500, 3))
        q = (p[k].astype(np.float64) + d).astype(np.float32)
        dd = q.astype(np.float64) - p[k].astype(np.float64)
        exact = ((dd @ V[k].astype(np.float64).T) ** 2 / R[k].astype(np.float64) ** 2).sum(1)
        got = O._within_form32(q, p[k][None, :], F[k][None, :])
        far = np.abs(exact - 1) > 1e-4
        assert far.sum() > 400
        assert np.array_equal(got[far], exact[far] < 1)


def test_equal_radii_ellipsoid_is_the_ball():
    rng = np.random.default_rng(503)
    C = 400
    cand = rng.uniform(0, 1, (C, 3)).astype(np.float32)
    Rb = np.float32(0.11)
    R = np.full((C, 3), Rb, np.float32)
    _, V = _random_axes(rng, C)
    F = O.ellipsoid_form(R, V)
    np.testing.assert_allclose(F[:, [0, 3, 5]], 1 / float(Rb) ** 2, rtol=2e-6)
    np.testing.assert_allclose(F[:, [1, 2, 4]], 0, atol=2e-6 / float(Rb) ** 2)
    # keep candidates whose pairwise distances stay clear of R, where rounding could differ
    d = np.linalg.norm(cand[:, None, :].astype(np.float64) - cand[None, :, :], axis=-1)
    near = (np.abs(d - float(Rb)) < 1e-4 * float(Rb)).any(1)
    cand = cand[~near]
    keep_f = F[~near]
    a = O.greedy_cover(cand, np.full(len(cand), Rb, np.float32))
    b = O.greedy_cover(cand, np.full(len(cand), Rb, np.float32), form=keep_f)
    assert len(a) > 20 and np.array_equal(a, b)


def test_anisotropic_greedy_cover_satisfies_the_sequential_rule():
    """Brute force: each candidate is accepted iff no earlier accepted point's
    ellipsoid contains it (the rule characterises the sequential output)."""
    rng = np.random.default_rng(504)
    C = 300
    cand = rng.uniform(0, 1, (C, 3)).astype(np.float32)
    R, V = _random_axes(rng, C, 0.03, 0.25)
    F = O.ellipsoid_form(R, V)
    acc = O.greedy_cover(cand, R.min(1), form=F)
    is_acc = np.zeros(C, bool)
    is_acc[acc] = True
    assert np.all(np.diff(acc) > 0) and 10 < len(acc) < C
    for i in range(C):
        earlier = [j for j in acc if j < i]
        inside = any(bool(O._within_form32(cand[i], cand[j], F[j])) for j in earlier)
        assert is_acc[i] == (not inside), i
    # anisotropy matters: the ball of the smallest radius gives another cover
    assert not np.array_equal(acc, O.greedy_cover(cand, R.min(1)))


def test_anisotropic_interpolation_single_point_and_ball_limit():
    rng = np.random.default_rng(505)
    R, V = _random_axes(rng, 1, 0.1, 0.3)
    F = O.ellipsoid_form(R, V)
    p = np.array([[0.5, 0.5, 0.5]], np.float32)
    val = np.array([2.0])
    grad = np.array([[0.3, -0.2, 0.5]])
    for i in range(3):
        for s in (0.25, 0.5, 0.9):
            q = (p[0].astype(np.float64) + s * float(R[0, i]) * V[0, i]).astype(np.float32)
            L, cov = O.interpolate(p, val, grad, R.min(1), q[None, :], cache_form=F)
            assert cov[0]
            np.testing.assert_allclose(L[0], 2.0 + grad[0] @ (q.astype(np.float64) - p[0]), rtol=1e-12)
        q = (p[0].astype(np.float64) + 1.01 * float(R[0, i]) * V[0, i]).astype(np.float32)
        L, cov = O.interpolate(p, val, grad, R.min(1), q[None, :], cache_form=F)
        assert not cov[0] and L[0] == 0
    # several points with equal radii: the ellipsoid weights are the ball's
    K = 30
    cp = rng.uniform(0.3, 0.7, (K, 3)).astype(np.float32)
    Rb = np.full(K, 0.15, np.float32)
    _, VV = _random_axes(rng, K)
    FF = O.ellipsoid_form(np.repeat(Rb[:, None], 3, 1), VV)
    cv = rng.uniform(1, 2, K)
    cg = rng.normal(size=(K, 3))
    qs = rng.uniform(0.3, 0.7, (200, 3)).astype(np.float32)
    d = np.linalg.norm(qs[:, None, :].astype(np.float64) - cp[None].astype(np.float64), axis=-1)
    qs = qs[~(np.abs(d - 0.15) < 1e-4).any(1)]
    a, ca = O.interpolate(cp, cv, cg, Rb, qs)
    b, cb = O.interpolate(cp, cv, cg, Rb, qs, cache_form=FF)
    assert np.array_equal(ca, cb) and ca.sum() > 100
    np.testing.assert_allclose(b, a, rtol=1e-5)


# ---------------------------------------------------------------------------
# the render pass (Sec. 6 "Implementation"; Results in 3D: march step 0.1)
# ---------------------------------------------------------------------------
def _room_rays(rng, n):
    """Rays from the centre region of the empty unit room: FP32 origins and
    unit directions, the oracle's closest hits, and the exact FP64 distances
    to the walls (the room is the only geometry)."""
    o = rng.uniform(0.3, 0.7, (n, 3)).astype(np.float32)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d = d.astype(np.float32)
    d[:6] = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.float32)
    sc = O.Scene(W.room_triangles(), np.full(12, 0.5, np.float32))
    hid, t, _ = sc.trace(o, d, brute=True)
    o64, d64 = o.astype(np.float64), d.astype(np.float64)
    with np.errstate(divide="ignore"):
        wall = np.where(d64 > 0, (1.0 - o64) / d64, np.where(d64 < 0, -o64 / d64, np.inf)).min(1)
    return o, d, hid, t, wall


def test_march_points_in_an_empty_room_follow_the_closed_form():
    """Every ray from inside the closed room ends on a wall at the exact wall
    distance; its march points are the ceil(t/step - xi) points (k + xi) step
    along the ray, inside the room."""
    rng = np.random.default_rng(71)
    n = 400
    o, d, hid, t, wall = _room_rays(rng, n)
    assert (hid >= 0).all()
    np.testing.assert_allclose(t, wall, rtol=2e-6)
    xi = rng.uniform(0, 1, n).astype(np.float32)
    step = 0.1
    offs, P, wts = O.march(t, xi, step, 1.0, 1.2, o, d)
    r = t.astype(np.float64) / step - xi.astype(np.float64)
    assert np.abs(r - np.round(r)).min() > 1e-9  # no ray ends on a march point
    np.testing.assert_array_equal(np.diff(offs), np.maximum(np.ceil(r), 0).astype(np.int64))
    ray = np.repeat(np.arange(n), np.diff(offs))
    k = np.arange(offs[-1]) - offs[:-1][ray]
    tk = (k + xi[ray].astype(np.float64)) * step
    np.testing.assert_allclose(np.linalg.norm(P.astype(np.float64) - o[ray].astype(np.float64), axis=1), tk,
                               rtol=1e-6, atol=1e-7)
    assert ((P >= 0) & (P <= 1)).all()
    # the points of a ray lie on it: cross((p - o), d) = 0
    c = np.cross(P.astype(np.float64) - o[ray].astype(np.float64), d[ray].astype(np.float64))
    assert np.abs(c).max() < 1e-6


def test_march_weights_average_to_the_transmittance_integral():
    """With a uniform offset xi, the march points of one ray stratify [0, t):
    the average of sum_k weight_k over xi is the integral of
    sigma_s exp(-sigma_t s) over [0, t), i.e. sigma_s (1 - exp(-sigma_t t)) /
    sigma_t (the medium radiance of a pixel seeing unit in-scattered radiance
    everywhere).  Averaged over 4000 evenly spaced offsets."""
    step, ss, st = 0.1, 0.8, 1.7
    for t_end in (0.05, 0.37, 1.0, 1.6180339):
        m = 4000
        xi = ((np.arange(m) + 0.5) / m).astype(np.float32)
        o = np.zeros((m, 3), np.float32)
        dd = np.tile(np.array([[0, 0, 1]], np.float32), (m, 1))
        offs, P, w = O.march(np.full(m, t_end, np.float32), xi, step, ss, st, o, dd)
        per_ray = np.bincount(np.repeat(np.arange(m), np.diff(offs)), weights=w, minlength=m)
        exact = ss * (1 - math.exp(-st * float(np.float32(t_end)))) / st
        assert abs(per_ray.mean() - exact) < 1e-6 * exact + 1e-7


def test_composite_of_constant_radiance_is_a_geometric_series():
    """Constant in-scattered radiance c: a ray with n points contributes
    step sigma_s c exp(-sigma_t xi step) (1 - r^n) / (1 - r), r = exp(-sigma_t
    step); a pixel averages its spp rays."""
    rng = np.random.default_rng(72)
    spp, n_pix = 4, 50
    N = spp * n_pix
    t = rng.uniform(0, 1.5, N).astype(np.float32)
    xi = rng.uniform(0, 1, N).astype(np.float32)
    step, ss, st, c = 0.1, 1.0, 1.2, 2.5
    o = np.zeros((N, 3), np.float32)
    dd = np.tile(np.array([[1, 0, 0]], np.float32), (N, 1))
    offs, P, w = O.march(t, xi, step, ss, st, o, dd)
    pix = O.composite(offs, spp, w, np.full(len(w), c))
    n = np.diff(offs)
    r = math.exp(-st * step)
    ray = step * ss * c * np.exp(-st * xi.astype(np.float64) * step) * (1 - r ** n) / (1 - r)
    np.testing.assert_allclose(pix, ray.reshape(n_pix, spp).mean(1), rtol=1e-12)
    # each pixel sees only its own rays: per-ray distinct radiance
    Lr = rng.uniform(0, 1, N)
    pix2 = O.composite(offs, spp, w, Lr[np.repeat(np.arange(N), n)])
    np.testing.assert_allclose(pix2, (ray / c * Lr).reshape(n_pix, spp).mean(1), rtol=1e-12)


# ---------------------------------------------------------------------------
# the comparison method's occlusion-unaware gradients (Jarosz et al. 2008;
# supplement Eqs. S.3-S.4) and its radius (Eq. jaroszRadius)
# ---------------------------------------------------------------------------
def _emitting_plane():
    Wd = 30.0
    floor = np.array([[-Wd, -Wd, 0, Wd, -Wd, 0, Wd, Wd, 0], [-Wd, -Wd, 0, Wd, Wd, 0, -Wd, Wd, 0]], np.float32)
    return O.Scene(floor, np.zeros(2, np.float32), np.ones(2, np.float32), (-Wd, -Wd, 0), (Wd, Wd, 4))


def test_j08_gradient_of_an_emitting_plane_is_the_exact_gradient():
    """Emitter L_e = 1 on z = 0 under an absorbing medium, nothing occluding:
    holding the hit points fixed loses nothing, so the occlusion-unaware
    gradient converges to dV/dz = -mu E1(mu h)/2 (lateral 0), and the mean of
    the per-direction gradient norms to the hemisphere integral
    (1/2) int_0^1 exp(-mu h/c) |(mu + 3c/h) u + e_z/h| dc (u the unit
    direction to the hit, u_z = -c), evaluated by quadrature."""
    from scipy.integrate import quad
    sc = _emitting_plane()
    mu, h = 1.0, 0.5
    Gz = -mu * expn(1, mu * h) / 2

    def norm(c):
        a = mu + 3 * c / h
        return math.exp(-mu * h / c) * math.sqrt(a * a - 2 * a * c / h + 1 / (h * h)) / 2
    gnorm = quad(norm, 0, 1, limit=200)[0]
    res = {}
    for N in (1024, 16384):
        nt, npf = W.strata_shape(N)
        v, g, m = O.j08(sc, 0.0, mu, NO_LIGHTS, np.array([[0.1, -0.2, h]] * 8, np.float32), nt, npf,
                        rec_id=np.arange(8), ring_step=0.1, max_rings=0, seed=7)
        res[N] = (g[:, 0].mean(0), m.mean(0), v[:, 0].mean())
    g, m, v = res[16384]
    assert abs(g[2] - Gz) / abs(Gz) < 0.02 and np.abs(g[:2]).max() < 2e-3 * abs(Gz)
    assert abs(res[16384][0][2] - Gz) < 0.5 * abs(res[1024][0][2] - Gz)
    assert abs(m[0] - v) < 1e-12 and abs(m[0] - expn(2, mu * h) / 2) < 2e-4
    assert abs(m[1] - gnorm) / gnorm < 0.02


def test_j08_medium_gradient_is_the_rigid_path_derivative():
    """A point light in an open absorbing medium, nothing occluding: moving x
    moves every sampled path rigidly when the random numbers are held (same
    record id), so the multiple-scattering gradient must equal the central
    difference of the record's own Monte Carlo values (rings far from the
    box, where the medium has absorbed everything)."""
    Wd = 20.0
    tri = np.array([[Wd - 1, Wd - 1, Wd - 1, Wd - 0.5, Wd - 1, Wd - 1, Wd - 1, Wd - 0.5, Wd - 1]], np.float32)
    sc = O.Scene(tri, np.zeros(1, np.float32), None, (-Wd, -Wd, -Wd), (Wd, Wd, Wd))
    light = np.array([[0.3, 0.45, -0.2, 5.0]], np.float32)
    ss, sa = 1.0, 1.0
    x = np.array([0.05, 0.1, 0.0])
    kw = dict(ring_step=0.1, max_rings=60, seed=11)
    v, g, m = O.j08(sc, ss, sa, light, x[None].astype(np.float32), 16, 64, rec_id=[3], **kw)
    h = 2e-3
    fd = np.zeros(3)
    for i in range(3):
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        vp = O.values(sc, ss, sa, light, xp[None].astype(np.float32), 16, 64, rec_id=[3], **kw)[0, 1]
        vm = O.values(sc, ss, sa, light, xm[None].astype(np.float32), 16, 64, rec_id=[3], **kw)[0, 1]
        fd[i] = (vp - vm) / (2 * h)
    assert np.linalg.norm(fd) > 0.05 * v[0, 1]
    np.testing.assert_allclose(g[0, 1], fd, rtol=2e-3, atol=2e-3 * np.linalg.norm(fd))
    assert np.abs(g[0, 0]).max() == 0.0 and v[0, 0] == 0.0  # nothing emits or reflects


def test_j08_radius_scales_with_eps_and_ignores_the_radiance_scale():
    """Eq. jaroszRadius uses the ratio of summed radiance to summed gradient
    norms: linear in eps, unchanged when every light (and so every sample)
    is scaled, and clamped to [r_min, r_max]."""
    w = W.make_c1(P=6)
    sc = O.Scene.from_workload(w)
    args = (sc, w.sigma_s, w.sigma_a)
    _, _, m1 = O.j08(*args, w.lights, w.pos, w.n_theta, w.n_phi, ring_step=w.ring_step, max_rings=w.max_rings,
                     seed=w.seed)
    L2 = w.lights.copy()
    L2[:, 3] *= 8.0
    _, _, m2 = O.j08(*args, L2, w.pos, w.n_theta, w.n_phi, ring_step=w.ring_step, max_rings=w.max_rings, seed=w.seed)
    np.testing.assert_allclose(m2, 8.0 * m1, rtol=1e-12)
    R1 = O.j08_radius(m1, 0.1, 1e-6, 1e6)
    np.testing.assert_allclose(O.j08_radius(m2, 0.1, 1e-6, 1e6), R1, rtol=1e-6)
    np.testing.assert_allclose(O.j08_radius(m1, 0.2, 1e-6, 1e6), 2 * R1, rtol=1e-6)
    assert (O.j08_radius(m1, 0.1, 0.05, 0.06) >= 0.05).all() and (O.j08_radius(m1, 0.1, 0.05, 0.06) <= 0.06).all()


def test_log_space_extrapolation_is_exact_for_exponential_fields():
    """Eq. jaroszExtrapolation averages first-order expansions of ln L: for
    L = exp(a + g . x) (so grad L_k / L_k = g) every expansion equals ln L(x')
    and the result is exp(a + g . x') exactly, whatever the weights; one
    cache point gives L_k exp(g_k . (x' - x_k)); a point with L_k <= 0 takes
    no part."""
    rng = np.random.default_rng(81)
    K, Q = 40, 300
    cp = rng.uniform(0.2, 0.8, (K, 3)).astype(np.float32)
    a, gv = 0.3, np.array([1.5, -2.0, 0.7])
    cv = np.exp(a + cp.astype(np.float64) @ gv)
    cg = cv[:, None] * gv[None, :]
    cR = rng.uniform(0.15, 0.4, K).astype(np.float32)
    q = rng.uniform(0.2, 0.8, (Q, 3)).astype(np.float32)
    L, cov = O.interpolate_log(cp, cv, cg, cR, q)
    assert cov.sum() > Q // 2
    np.testing.assert_allclose(L[cov], np.exp(a + q[cov].astype(np.float64) @ gv), rtol=1e-12)
    Lin, _ = O.interpolate(cp, cv, cg, cR, q)  # linear space is not exact here
    assert np.abs(Lin[cov] / np.exp(a + q[cov].astype(np.float64) @ gv) - 1).max() > 1e-3
    one, c1 = O.interpolate_log(cp[:1], cv[:1], cg[:1] * 0.5, cR[:1], q)
    d = q[c1].astype(np.float64) - cp[0].astype(np.float64)
    np.testing.assert_allclose(one[c1], cv[0] * np.exp(d @ (0.5 * gv)), rtol=1e-12)
    neg = cv.copy()
    neg[0] = -1.0
    _, cn = O.interpolate_log(cp[:1], neg[:1], cg[:1], cR[:1], q)
    assert not cn.any()
