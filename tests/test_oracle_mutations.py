"""The oracle's pins catch plausible mistakes: each case builds a copy of the
oracle's C source with one planted mistake, loads it in place of the oracle,
and requires the named pin to fail on it.  CPU only; the copies live in a
temporary directory."""
import inspect

import numpy as np

import pytest

from oracle import build as OB
from oracle import oracle as O
from tests import test_oracle_pins as pins

SRC = OB.HERE / "rco.c"

# (name, text in rco.c, replacement, pins of which at least one must fail)
MUTATIONS = [
    # Sec. 4: an occluder closer than the ring puts the vertex at the occluder
    ("ring vertex kept at its ring distance behind an occluder",
     "double tt = in_front ? v.r64[i] : v.t64[id[q]];", "double tt = v.r64[i];",
     ["test_medium_ring_gradient_converges_to_fd_of_brute_force_values"]),
    ("far-vertex choice by the ring distance of the clamped vertex",
     "dd[q] = in_front ? v.r32[i] : v.t32[id[q]];", "dd[q] = v.r32[i];",
     ["test_medium_ring_gradient_converges_to_fd_of_brute_force_values"]),
    # App. A: transmittance gradient
    ("sign of grad T", "gT[i] = -mu * (u[i] / r) * t;", "gT[i] = mu * (u[i] / r) * t;",
     [("test_transmittance_closed_form_and_fd", {"mu": 0.3})]),
    # Eq. SSSegALHessianSimp: the F * HT term
    ("dropped F HT term of the Hessian", "gF[i] * gT[j] + F * HT[3 * i + j]);", "gF[i] * gT[j]);",
     ["test_record_derivatives_are_exact_calculus_of_triangulated_value",
      "test_emitting_plane_under_medium_matches_exponential_integrals"]),
    # comparison method's gradients (supplement Eq. S.4; rigid medium paths)
    ("sign of the 3 yx / r^2 term of grad ln G", "- 3.0 * yx[i] / (r * r));", "+ 3.0 * yx[i] / (r * r));",
     ["test_j08_gradient_of_an_emitting_plane_is_the_exact_gradient"]),
    ("inverse-square falloff differentiated as 1/d", "(-mu - 2.0 / d) * ml[q] / d;", "(-mu - 1.0 / d) * ml[q] / d;",
     ["test_j08_medium_gradient_is_the_rigid_path_derivative"]),
    ("sign of grad ln T of the fixed-hit sample", "gk[i] = S * (-mu * yx[i] / r +", "gk[i] = S * (mu * yx[i] / r +",
     ["test_j08_gradient_of_an_emitting_plane_is_the_exact_gradient"]),
    # far vertex (the first to be occluded): nearest instead
    ("nearest instead of furthest vertex", "if (dist[k] > dist[best] ||", "if (dist[k] < dist[best] ||",
     ["test_black_occluder_in_uniform_field_converges_to_closed_form",
      "test_medium_ring_gradient_converges_to_fd_of_brute_force_values"]),
]


def _call(pin):
    name, given = (pin, {}) if isinstance(pin, str) else pin
    fn = getattr(pins, name)
    params = inspect.signature(fn).parameters
    # parametrized pins: their first parameter set unless given
    marks = getattr(fn, "pytestmark", [])
    args = {}
    for m in marks:
        if m.name == "parametrize":
            names = [n.strip() for n in m.args[0].split(",")]
            vals = m.args[1][0]
            vals = vals if len(names) > 1 else (vals,)
            args.update(dict(zip(names, vals)))
    args.update(given)
    fn(**{k: v for k, v in args.items() if k in params})


@pytest.mark.parametrize("name,old,new,pin_names", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(tmp_path, name, old, new, pin_names):
    text = SRC.read_text()
    assert text.count(old) == 1, f"mutation site not unique: {old}"
    src = tmp_path / "rco_mut.c"
    src.write_text(text.replace(old, new))
    so = tmp_path / "liboracle_mut.so"
    OB.build(src=src, out=so)
    failed = []
    try:
        O.use_library(so)
        for pn in pin_names:
            try:
                _call(pn)
            except AssertionError:
                failed.append(pn)
    finally:
        O.use_library(None)
    assert failed, f"no pin caught: {name}"  # the pins pass on the oracle itself (test_oracle_pins)


# Planted mistakes in the oracle's numpy parts (anisotropic cache points)
def _form_transposed(orig):
    def f(Ri, vecs):
        return orig(Ri, np.transpose(np.asarray(vecs, np.float32).reshape(-1, 3, 3), (0, 2, 1)))
    return f


def _within_without_factor_two(orig):
    def f(q, p, form):
        d = np.asarray(q, np.float32) - np.asarray(p, np.float32)
        m = np.asarray(form, np.float32)
        dx, dy, dz = d[..., 0], d[..., 1], d[..., 2]
        diag = (m[..., 0] * (dx * dx) + m[..., 3] * (dy * dy)) + m[..., 5] * (dz * dz)
        off = (m[..., 1] * (dx * dy) + m[..., 2] * (dx * dz)) + m[..., 4] * (dy * dz)
        return (diag + off) < np.float32(1)
    return f


def _march_from_k1(orig):
    def f(t_end, xi, step, sigma_s, sigma_t, o, d):
        return orig(t_end, np.asarray(xi, np.float32) + np.float32(1), step, sigma_s, sigma_t, o, d)
    return f


def _march_without_sigma_s(orig):
    def f(t_end, xi, step, sigma_s, sigma_t, o, d):
        return orig(t_end, xi, step, 1.0, sigma_t, o, d)
    return f


def _composite_summing_rays(orig):
    def f(offsets, spp, weights, L):
        return orig(offsets, spp, weights, L) * spp
    return f


def _log_interp_in_linear_space(orig):
    def f(cache_pos, cache_val, cache_grad, cache_R, query):
        return O.interpolate(cache_pos, cache_val, cache_grad, cache_R, query)
    return f


PY_MUTATIONS = [
    ("log-space extrapolation done in linear space", "interpolate_log", _log_interp_in_linear_space,
     ["test_log_space_extrapolation_is_exact_for_exponential_fields"]),
    ("march starts one step late", "march", _march_from_k1,
     ["test_march_points_in_an_empty_room_follow_the_closed_form"]),
    ("march weight without the scattering coefficient", "march", _march_without_sigma_s,
     ["test_march_weights_average_to_the_transmittance_integral"]),
    ("pixel sums its rays instead of averaging them", "composite", _composite_summing_rays,
     ["test_composite_of_constant_radiance_is_a_geometric_series"]),
    ("ellipsoid built from eigenvector columns", "ellipsoid_form", _form_transposed,
     ["test_ellipsoid_form_has_the_axes_as_eigenvectors"]),
    ("off-diagonal terms of the form counted once", "_within_form32", _within_without_factor_two,
     ["test_ellipsoid_membership_along_and_off_the_axes"]),
]


@pytest.mark.parametrize("name,attr,make,pin_names", PY_MUTATIONS, ids=[m[0] for m in PY_MUTATIONS])
def test_planted_numpy_mistake_fails_a_pin(monkeypatch, name, attr, make, pin_names):
    monkeypatch.setattr(O, attr, make(getattr(O, attr)))
    failed = []
    for pn in pin_names:
        try:
            _call(pn)
        except AssertionError:
            failed.append(pn)
    assert failed, f"no pin caught: {name}"
