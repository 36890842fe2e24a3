"""Thin Python binding of librc (the C ABI declared in include/rc.h).

Argument marshalling only: every step of the computation runs in librc's HIP
kernels.  PyTorch supplies device memory and streams.  The functions keep the
C names (rc_scene_create, rc_records, ...); `Scene` and `compute_records` are
conveniences that allocate the outputs as torch tensors.

Loading fails loudly if the library has not been built (run
``python paper_1805_09258_amd/build.py``); there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from pathlib import Path

import numpy as np

_PKG = Path(__file__).resolve().parent
LIB_PATH = Path(os.environ.get("RC_LIBRARY", str(_PKG / "librc.so")))

RC_OK, RC_EINVAL, RC_ENOMEM, RC_EDEVICE, RC_ENODEV = 0, -1, -2, -3, -4
RC_MAX_LIGHTS, RC_MAX_RINGS, RC_MAX_NPHI = 16, 64, 256
RC_ETIMEOUT = -5
RC_NOALLOC_MAX_RECORDS = 4096  # largest batch of rc_records_noalloc
RC_MARCH_MAX_POINTS_PER_RAY = 1 << 20  # bound on medium box diagonal / march step
RC_PLACE_STATE_INTS = 4101  # placement state: 5 counters + one status word per gathered candidate


class RCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"librc error {code}: {msg}")
        self.code = code


class rc_medium(C.Structure):
    _fields_ = [("sigma_s", C.c_float), ("sigma_a", C.c_float)]


class rc_point_light(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("intensity", C.c_float)]


class rc_params(C.Structure):
    _fields_ = [("ring_step", C.c_float), ("max_rings", C.c_int32), ("max_n_phi", C.c_int32),
                ("precision", C.c_int32), ("common_random", C.c_int32), ("splits", C.c_int32),
                ("seed", C.c_uint64),
                ("rec_base", C.c_int64),
                ("counters", C.c_void_p),
                ("shadow_bvh", C.c_int32),
                ("max_n_theta", C.c_int32),
                ("shadow_pass", C.c_int32)]


class rc_scene_stats(C.Structure):
    _fields_ = [("n_tri", C.c_int64), ("n_nodes", C.c_int64), ("depth", C.c_int32), ("leaf_max", C.c_int32),
                ("node_bytes", C.c_int64), ("tri_bytes", C.c_int64), ("pad", C.c_float),
                ("device_bytes", C.c_int64), ("light_bin_bytes", C.c_int64), ("light_bin_entries", C.c_int64)]


EXPORTS = ["rc_scene_create", "rc_scene_destroy", "rc_scene_info", "rc_bvh_build_host", "rc_workspace_size",
           "rc_workspace_errors", "rc_records", "rc_records_noalloc", "rc_records_noalloc_errors", "rc_records_batched", "rc_records_wait", "rc_autotune", "rc_tile_info", "rc_radius",
           "rc_trace_rays", "rc_occluded_rays", "rc_light_bins_build", "rc_light_occluded", "rc_light_bins_host",
           "rc_probe", "rc_mlp_param_bytes", "rc_mlp_n_params", "rc_mlp_init",
           "rc_mlp_load", "rc_mlp_fit_features", "rc_mlp_forward", "rc_mlp_radius", "rc_mlp_train_workspace_bytes",
           "rc_mlp_train_step", "rc_place_gather", "rc_place_accept", "rc_place_cover", "rc_place_cover_grid",
           "rc_ellipsoid_form", "rc_interp", "rc_march_count", "rc_march_emit", "rc_composite",
           "rc_j08_records", "rc_interp_log",
           "rc_last_error", "rc_version"]

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1805_09258_amd/build.py")
        L = C.CDLL(str(LIB_PATH))
        vp, i64, i32, f32, sz = C.c_void_p, C.c_int64, C.c_int, C.c_float, C.c_size_t
        L.rc_scene_create.argtypes = [vp, vp, vp, i64, vp, vp, C.POINTER(vp)]
        L.rc_scene_create.restype = i32
        L.rc_scene_destroy.argtypes = [vp]
        L.rc_scene_destroy.restype = i32
        L.rc_scene_info.argtypes = [vp, C.POINTER(rc_scene_stats)]
        L.rc_scene_info.restype = i32
        L.rc_bvh_build_host.argtypes = [vp, i64, vp, vp, vp, i64, vp, C.POINTER(rc_scene_stats)]
        L.rc_bvh_build_host.restype = i64
        L.rc_workspace_size.argtypes = [i64]
        L.rc_workspace_size.restype = sz
        L.rc_workspace_errors.argtypes = [vp, vp]
        L.rc_workspace_errors.restype = i64
        rec = [vp, C.POINTER(rc_medium), C.POINTER(rc_point_light), i32, vp, vp, vp, i64, C.POINTER(rc_params)]
        L.rc_records.argtypes = rec + [vp, vp, vp, vp, vp]
        L.rc_records.restype = i32
        L.rc_records_noalloc.argtypes = rec + [vp, vp, vp, vp]
        L.rc_records_noalloc.restype = i32
        L.rc_records_noalloc_errors.argtypes = [vp]
        L.rc_records_noalloc_errors.restype = i64
        L.rc_records_batched.argtypes = rec + [vp, i32, i32, vp, vp, vp, vp, vp]
        L.rc_records_batched.restype = i32
        L.rc_records_wait.argtypes = [vp, i32, vp]
        L.rc_records_wait.restype = i32
        L.rc_autotune.argtypes = rec + [vp, vp, vp, vp, C.c_char_p, C.POINTER(i32), vp, C.POINTER(i32), vp]
        L.rc_autotune.restype = i32
        L.rc_tile_info.argtypes = [i32, C.POINTER(f32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.rc_tile_info.restype = i32
        L.rc_radius.argtypes = [vp, vp, i64, f32, f32, f32, vp, vp, vp]
        L.rc_radius.restype = i32
        L.rc_trace_rays.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp]
        L.rc_trace_rays.restype = i32
        L.rc_occluded_rays.argtypes = [vp, vp, vp, vp, i64, vp, vp]
        L.rc_occluded_rays.restype = i32
        L.rc_light_bins_build.argtypes = [vp, C.POINTER(rc_point_light), i32, i32]
        L.rc_light_bins_build.restype = i32
        L.rc_light_occluded.argtypes = [vp, i32, vp, vp, i64, vp, vp]
        L.rc_light_occluded.restype = i32
        L.rc_light_bins_host.argtypes = [vp, i64, vp, vp, vp, i32, C.POINTER(i32), C.POINTER(i32), vp, vp, i64,
                                         C.POINTER(i64), vp, i64]
        L.rc_light_bins_host.restype = i64
        u64 = C.c_uint64
        L.rc_probe.argtypes = [vp, C.POINTER(rc_medium), C.POINTER(rc_point_light), i32, vp, i64, u64, i64, i32, vp,
                               vp, vp]
        L.rc_probe.restype = i32
        L.rc_mlp_param_bytes.restype = sz
        L.rc_mlp_n_params.restype = i64
        L.rc_mlp_init.argtypes = [vp, vp, u64, vp]
        L.rc_mlp_init.restype = i32
        L.rc_mlp_load.argtypes = [vp, vp, vp]
        L.rc_mlp_load.restype = i32
        L.rc_mlp_fit_features.argtypes = [vp, vp, i64, vp, vp]
        L.rc_mlp_fit_features.restype = i32
        L.rc_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
        L.rc_mlp_forward.restype = i32
        L.rc_mlp_radius.argtypes = [vp, vp, i64, f32, f32, f32, vp, vp]
        L.rc_mlp_radius.restype = i32
        L.rc_mlp_train_workspace_bytes.argtypes = [i64]
        L.rc_mlp_train_workspace_bytes.restype = sz
        L.rc_mlp_train_step.argtypes = [vp, vp, vp, vp, i64, f32, i64, vp, vp, vp, vp]
        L.rc_mlp_train_step.restype = i32
        L.rc_place_gather.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, i32, vp]
        L.rc_place_gather.restype = i32
        L.rc_place_accept.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.rc_place_accept.restype = i32
        L.rc_place_cover.argtypes = [vp, i64, vp, vp, vp, vp, i64, i64, vp, vp]
        L.rc_place_cover.restype = i32
        L.rc_place_cover_grid.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, i64, i64, vp, vp]
        L.rc_place_cover_grid.restype = i32
        L.rc_ellipsoid_form.argtypes = [vp, i64, vp, vp, vp]
        L.rc_ellipsoid_form.restype = i32
        L.rc_interp.argtypes = [vp, vp, vp, vp, i64, vp, i64, vp, vp, vp, vp, vp, vp]
        L.rc_interp.restype = i32
        f64 = C.c_double
        L.rc_march_count.argtypes = [vp, vp, vp, vp, i64, f64, vp, vp, vp]
        L.rc_march_count.restype = i32
        L.rc_march_emit.argtypes = [vp, vp, vp, i64, f64, f64, f64, vp, vp, vp, vp]
        L.rc_march_emit.restype = i32
        L.rc_composite.argtypes = [vp, i64, i32, vp, vp, vp, vp]
        L.rc_composite.restype = i32
        L.rc_j08_records.argtypes = [vp, C.POINTER(rc_medium), C.POINTER(rc_point_light), i32, vp, vp, vp, i64,
                                     C.POINTER(rc_params), f32, f32, f32, vp, vp, vp, vp, vp]
        L.rc_j08_records.restype = i32
        L.rc_interp_log.argtypes = [vp, vp, vp, vp, i64, vp, i64, vp, vp, vp]
        L.rc_interp_log.restype = i32
        L.rc_last_error.restype = C.c_char_p
        L.rc_version.restype = C.c_char_p
        _LIB = L
    return _LIB


def _check(code):
    if code < 0:
        raise RCError(code, lib().rc_last_error().decode(errors="replace"))
    return code


def _np(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _ptr(t):
    """Raw pointer of a torch tensor or numpy array (None -> NULL)."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return C.c_void_p(t.data_ptr())
    return t.ctypes.data_as(C.c_void_p)


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream) if hasattr(stream, "cuda_stream") else C.c_void_p(stream)


def _lights(lights):
    li = np.ascontiguousarray(lights, np.float32).reshape(-1, 4)
    arr = (rc_point_light * max(len(li), 1))()
    for i, (x, y, z, I) in enumerate(li):
        arr[i].pos[0], arr[i].pos[1], arr[i].pos[2], arr[i].intensity = x, y, z, I
    return arr, len(li)


# ---------------------------------------------------------------------------
# C-named entry points
# ---------------------------------------------------------------------------
def rc_scene_create(tri, albedo, emission, box_lo, box_hi):
    tri = np.ascontiguousarray(tri, np.float32).reshape(-1, 9)
    alb = np.ascontiguousarray(albedo, np.float32)
    em = None if emission is None else np.ascontiguousarray(emission, np.float32)
    lo = np.ascontiguousarray(box_lo, np.float32)
    hi = np.ascontiguousarray(box_hi, np.float32)
    h = C.c_void_p()
    _check(lib().rc_scene_create(_ptr(tri), _ptr(alb), _ptr(em), tri.shape[0], _ptr(lo), _ptr(hi), C.byref(h)))
    return h


def rc_scene_destroy(h):
    return _check(lib().rc_scene_destroy(h))


def rc_scene_info(h):
    st = rc_scene_stats()
    _check(lib().rc_scene_info(h, C.byref(st)))
    return {k: getattr(st, k) for k, _ in rc_scene_stats._fields_}


def rc_bvh_build_host(tri, box_lo, box_hi):
    tri = np.ascontiguousarray(tri, np.float32).reshape(-1, 9)
    lo = np.ascontiguousarray(box_lo, np.float32)
    hi = np.ascontiguousarray(box_hi, np.float32)
    st = rc_scene_stats()
    n = _check(lib().rc_bvh_build_host(_ptr(tri), tri.shape[0], _ptr(lo), _ptr(hi), None, 0, None, C.byref(st)))
    nodes = np.zeros((n, 16), np.float32)
    tris = np.zeros((tri.shape[0], 12), np.float32)
    _check(lib().rc_bvh_build_host(_ptr(tri), tri.shape[0], _ptr(lo), _ptr(hi), _ptr(nodes), n, _ptr(tris),
                                   C.byref(st)))
    return nodes, tris, {k: getattr(st, k) for k, _ in rc_scene_stats._fields_}


def rc_workspace_size(P):
    return int(lib().rc_workspace_size(int(P)))


def rc_workspace_errors(ws, stream=None):
    return _check(lib().rc_workspace_errors(_ptr(ws), _stream(stream)))


def make_params(ring_step, max_rings, max_n_phi, seed, rec_base=0, precision=0, counters=None, common_random=False,
                splits=0, shadow_bvh=False, max_n_theta=0, shadow_pass=False):
    return rc_params(float(ring_step), int(max_rings), int(max_n_phi), int(precision), int(bool(common_random)),
                     int(splits), int(seed) & (2**64 - 1), int(rec_base),
                     None if counters is None else counters.data_ptr(), int(bool(shadow_bvh)), int(max_n_theta),
                     int(bool(shadow_pass)))


def rc_records_wait(workspace, timeout_ms, stream=None):
    return _check(lib().rc_records_wait(_ptr(workspace), int(timeout_ms), _stream(stream)))


def rc_light_bins_build(scene, lights, B=0):
    arr, nl = _lights(lights)
    return _check(lib().rc_light_bins_build(scene, arr, nl, int(B)))


def rc_light_occluded(scene, light, pts, skip, occ, stream=None):
    n = int(pts.shape[0])
    return _check(lib().rc_light_occluded(scene, int(light), _ptr(pts), _ptr(skip), n, _ptr(occ), _stream(stream)))


def rc_light_bins_host(tri, box_lo, box_hi, light, B=0):
    """Host-built bins of one light: dict(B, levels, level_off, offs, entries[n][12])."""
    tri = np.ascontiguousarray(tri, np.float32).reshape(-1, 9)
    lo = np.ascontiguousarray(box_lo, np.float32)
    hi = np.ascontiguousarray(box_hi, np.float32)
    L = np.ascontiguousarray(light, np.float32)
    Bo, nl, no = C.c_int(0), C.c_int(0), C.c_int64(0)
    lev = np.zeros(4, np.int64)
    ne = _check(lib().rc_light_bins_host(_np(tri), tri.shape[0], _np(lo), _np(hi), _np(L), int(B), C.byref(Bo),
                                         C.byref(nl), _np(lev), None, 0, C.byref(no), None, 0))
    offs = np.zeros(no.value, np.int32)
    ent = np.zeros((ne, 12), np.float32)
    _check(lib().rc_light_bins_host(_np(tri), tri.shape[0], _np(lo), _np(hi), _np(L), int(B), C.byref(Bo),
                                    C.byref(nl), _np(lev), _np(offs), no.value, C.byref(no), _np(ent), ne))
    return {"B": Bo.value, "levels": nl.value, "level_off": lev[:nl.value].copy(), "offs": offs, "entries": ent}


def rc_records(scene, sigma_s, sigma_a, lights, pos, n_theta, n_phi, params, value, grad, hess, workspace,
               stream=None):
    med = rc_medium(float(sigma_s), float(sigma_a))
    arr, nl = _lights(lights)
    P = int(pos.shape[0])
    return _check(lib().rc_records(scene, C.byref(med), arr, nl, _ptr(pos), _ptr(n_theta), _ptr(n_phi), P,
                                   C.byref(params), _ptr(value), _ptr(grad), _ptr(hess), _ptr(workspace),
                                   _stream(stream)))


def rc_records_noalloc(scene, sigma_s, sigma_a, lights, pos, n_theta, n_phi, params, value, grad, hess, stream=None):
    med = rc_medium(float(sigma_s), float(sigma_a))
    arr, nl = _lights(lights)
    P = int(pos.shape[0])
    return _check(lib().rc_records_noalloc(scene, C.byref(med), arr, nl, _ptr(pos), _ptr(n_theta), _ptr(n_phi), P,
                                           C.byref(params), _ptr(value), _ptr(grad), _ptr(hess), _stream(stream)))


def rc_records_noalloc_errors(stream=None):
    return _check(lib().rc_records_noalloc_errors(_stream(stream)))


def rc_records_batched(scene, sigma_s, sigma_a, lights, pos, n_theta, n_phi, params, order, use_graph, tile, value,
                       grad, hess, workspace, stream=None):
    med = rc_medium(float(sigma_s), float(sigma_a))
    arr, nl = _lights(lights)
    P = int(pos.shape[0])
    return _check(lib().rc_records_batched(scene, C.byref(med), arr, nl, _ptr(pos), _ptr(n_theta), _ptr(n_phi), P,
                                           C.byref(params), _ptr(order), int(use_graph), int(tile), _ptr(value),
                                           _ptr(grad), _ptr(hess), _ptr(workspace), _stream(stream)))


def rc_autotune(scene, sigma_s, sigma_a, lights, pos, n_theta, n_phi, params, value, grad, hess, workspace,
                cache_path=None, measure=True, stream=None):
    med = rc_medium(float(sigma_s), float(sigma_a))
    arr, nl = _lights(lights)
    P = int(pos.shape[0])
    best = C.c_int(0)
    nt = C.c_int(0)
    ms = np.zeros(16, np.float32)
    _check(lib().rc_autotune(scene, C.byref(med), arr, nl, _ptr(pos), _ptr(n_theta), _ptr(n_phi), P,
                             C.byref(params), _ptr(value), _ptr(grad), _ptr(hess), _ptr(workspace),
                             None if cache_path is None else str(cache_path).encode(), C.byref(best),
                             _ptr(ms) if measure else None, C.byref(nt), _stream(stream)))
    return best.value, (ms[:nt.value].tolist() if measure else None)


def rc_tile_info(tile):
    g, r, l, w = C.c_float(0), C.c_int(0), C.c_int(0), C.c_int(0)
    _check(lib().rc_tile_info(int(tile), C.byref(g), C.byref(r), C.byref(l), C.byref(w)))
    return {"grid": g.value, "refill_min": r.value, "leaf_batch": l.value, "lds_waves": w.value}


def rc_radius(value, hess, eps, r_min, r_max, R, axes=None, stream=None):
    P = int(value.shape[0])
    return _check(lib().rc_radius(_ptr(value), _ptr(hess), P, float(eps), float(r_min), float(r_max), _ptr(R),
                                  _ptr(axes), _stream(stream)))


def rc_trace_rays(scene, orig, dirs, hit_id, t, front, stream=None):
    return _check(lib().rc_trace_rays(scene, _ptr(orig), _ptr(dirs), int(orig.shape[0]), _ptr(hit_id), _ptr(t),
                                      _ptr(front), _stream(stream)))


def rc_occluded_rays(scene, orig, seg, skip, occ, stream=None):
    return _check(lib().rc_occluded_rays(scene, _ptr(orig), _ptr(seg), _ptr(skip), int(orig.shape[0]), _ptr(occ),
                                         _stream(stream)))


def rc_probe(scene, sigma_s, sigma_a, lights, cand, seed, id_base, feat32=None, feat_bf16=None, stream=None,
             common_random=False):
    med = rc_medium(float(sigma_s), float(sigma_a))
    arr, nl = _lights(lights)
    return _check(lib().rc_probe(scene, C.byref(med), arr, nl, _ptr(cand), int(cand.shape[0]), int(seed) & (2**64 - 1),
                                 int(id_base), int(bool(common_random)), _ptr(feat32), _ptr(feat_bf16),
                                 _stream(stream)))


def rc_mlp_param_bytes():
    return int(lib().rc_mlp_param_bytes())


def rc_mlp_n_params():
    return int(lib().rc_mlp_n_params())


def rc_mlp_init(params, state, seed, stream=None):
    return _check(lib().rc_mlp_init(_ptr(params), _ptr(state), int(seed), _stream(stream)))


def rc_mlp_load(params, state, stream=None):
    return _check(lib().rc_mlp_load(_ptr(params), _ptr(state), _stream(stream)))


def rc_mlp_fit_features(params, X, workspace, stream=None):
    return _check(lib().rc_mlp_fit_features(_ptr(params), _ptr(X), int(X.shape[0]), _ptr(workspace), _stream(stream)))


def rc_mlp_forward(params, X, out, stream=None):
    return _check(lib().rc_mlp_forward(_ptr(params), _ptr(X), int(X.shape[0]), _ptr(out), _stream(stream)))


def rc_mlp_radius(params, X, safety, r_min, r_max, R, stream=None):
    return _check(lib().rc_mlp_radius(_ptr(params), _ptr(X), int(X.shape[0]), float(safety), float(r_min),
                                      float(r_max), _ptr(R), _stream(stream)))


def rc_mlp_train_workspace_bytes(n):
    return int(lib().rc_mlp_train_workspace_bytes(int(n)))


def rc_mlp_train_step(params, state, X, target, lr, step, workspace, loss=None, grad=None, stream=None):
    return _check(lib().rc_mlp_train_step(_ptr(params), _ptr(state), _ptr(X), _ptr(target), int(X.shape[0]),
                                          float(lr), int(step), _ptr(workspace), _ptr(loss), _ptr(grad),
                                          _stream(stream)))


def rc_place_gather(cand, radius, covered, state, batch_idx, batch_pos, batch_R, batch, order=None, stream=None):
    return _check(lib().rc_place_gather(_ptr(cand), _ptr(radius), _ptr(order), int(cand.shape[0]), _ptr(covered),
                                        _ptr(state), _ptr(batch_idx), _ptr(batch_pos), _ptr(batch_R), int(batch),
                                        _stream(stream)))


def rc_place_accept(cand, batch_idx, batch_R, covered, state, accepted, accepted_R, accepted_pos=None,
                    batch_value=None, batch_grad=None, cache_value=None, cache_grad=None, batch_form=None,
                    accepted_form=None, stream=None):
    return _check(lib().rc_place_accept(_ptr(cand), _ptr(batch_idx), _ptr(batch_R), _ptr(covered), _ptr(state),
                                        _ptr(accepted), _ptr(accepted_R), _ptr(accepted_pos), _ptr(batch_value),
                                        _ptr(batch_grad), _ptr(cache_value), _ptr(cache_grad), _ptr(batch_form),
                                        _ptr(accepted_form), _stream(stream)))


def rc_place_cover(cand, covered, state, accepted, accepted_R, first=-1, count=0, accepted_form=None, stream=None):
    return _check(lib().rc_place_cover(_ptr(cand), int(cand.shape[0]), _ptr(covered), _ptr(state), _ptr(accepted),
                                       _ptr(accepted_R), int(first), int(count), _ptr(accepted_form),
                                       _stream(stream)))


def rc_place_cover_grid(cand, dims, lo, cell, covered, state, accepted, accepted_R, first=-1, count=0,
                        accepted_form=None, stream=None):
    d = np.ascontiguousarray(dims, np.int32)
    l0 = np.ascontiguousarray(lo, np.float32)
    ce = np.ascontiguousarray(cell, np.float32)
    return _check(lib().rc_place_cover_grid(_ptr(cand), _ptr(d), _ptr(l0), _ptr(ce), _ptr(covered), _ptr(state),
                                            _ptr(accepted), _ptr(accepted_R), int(first), int(count),
                                            _ptr(accepted_form), _stream(stream)))


def rc_ellipsoid_form(axes, form, r_max=None, stream=None):
    return _check(lib().rc_ellipsoid_form(_ptr(axes), int(axes.shape[0]), _ptr(form), _ptr(r_max),
                                          _stream(stream)))


def rc_interp(cache_pos, cache_value, cache_grad, cache_R, query, out, hits=None, ref_value=None, err_partial=None,
              cache_form=None, stream=None):
    return _check(lib().rc_interp(_ptr(cache_pos), _ptr(cache_value), _ptr(cache_grad), _ptr(cache_R),
                                  int(cache_pos.shape[0]), _ptr(query), int(query.shape[0]), _ptr(out), _ptr(hits),
                                  _ptr(ref_value), _ptr(err_partial), _ptr(cache_form), _stream(stream)))


def rc_march_count(scene, orig, dirs, xi, step, t_end, offsets, stream=None):
    return _check(lib().rc_march_count(scene, _ptr(orig), _ptr(dirs), _ptr(xi), int(orig.shape[0]), float(step),
                                       _ptr(t_end), _ptr(offsets), _stream(stream)))


def rc_march_emit(orig, dirs, xi, step, sigma_s, sigma_t, offsets, points, weight, stream=None):
    return _check(lib().rc_march_emit(_ptr(orig), _ptr(dirs), _ptr(xi), int(orig.shape[0]), float(step),
                                      float(sigma_s), float(sigma_t), _ptr(offsets), _ptr(points), _ptr(weight),
                                      _stream(stream)))


def rc_composite(offsets, spp, weight, L, pixel, stream=None):
    return _check(lib().rc_composite(_ptr(offsets), int(offsets.shape[0]) - 1, int(spp), _ptr(weight), _ptr(L),
                                     _ptr(pixel), _stream(stream)))


def rc_j08_records(scene, sigma_s, sigma_a, lights, pos, n_theta, n_phi, params, eps, r_min, r_max, value, grad,
                   moments, R, stream=None):
    li, n = _lights(lights)
    med = rc_medium(float(sigma_s), float(sigma_a))
    return _check(lib().rc_j08_records(scene, C.byref(med), li, n, _ptr(pos), _ptr(n_theta), _ptr(n_phi),
                                       int(pos.shape[0]), C.byref(params), float(eps), float(r_min), float(r_max),
                                       _ptr(value), _ptr(grad), _ptr(moments), _ptr(R), _stream(stream)))


def rc_interp_log(cache_pos, cache_value, cache_grad, cache_R, query, out, hits=None, stream=None):
    return _check(lib().rc_interp_log(_ptr(cache_pos), _ptr(cache_value), _ptr(cache_grad), _ptr(cache_R),
                                      int(cache_pos.shape[0]), _ptr(query), int(query.shape[0]), _ptr(out), _ptr(hits),
                                      _stream(stream)))


def rc_version():
    return lib().rc_version().decode()


# ---------------------------------------------------------------------------
# conveniences
# ---------------------------------------------------------------------------
class Scene:
    """Device scene handle built from host arrays (owned; freed on close)."""

    def __init__(self, tri, albedo, emission=None, box_lo=(0, 0, 0), box_hi=(1, 1, 1)):
        self.box_lo = np.asarray(box_lo, np.float32)
        self.box_hi = np.asarray(box_hi, np.float32)
        self.handle = rc_scene_create(tri, albedo, emission, self.box_lo, self.box_hi)

    @classmethod
    def from_workload(cls, w):
        return cls(w.tri, w.albedo, w.emission, w.box_lo, w.box_hi)

    def info(self):
        return rc_scene_info(self.handle)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            rc_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceWorkload:
    """Device copies (torch, cuda:0) of a workload's per-record inputs."""

    def __init__(self, w, device="cuda"):
        import torch
        self.w = w
        self.pos = torch.as_tensor(np.ascontiguousarray(w.pos, np.float32), device=device)
        self.n_theta = torch.as_tensor(np.ascontiguousarray(w.n_theta, np.int32), device=device)
        self.n_phi = torch.as_tensor(np.ascontiguousarray(w.n_phi, np.int32), device=device)
        self.max_n_phi = int(np.max(w.n_phi)) if len(w.n_phi) else 5
        self.max_n_theta = int(np.max(w.n_theta)) if len(w.n_theta) else 2
        # the primary-hit buffer of a hits pass: 8 B per slot, each record
        # reserving max_n_theta * max_n_phi + 2 slots; the share the rays fill
        P = len(w.n_theta)
        slots = ((P + 63) // 64) * 64 * (self.max_n_theta * self.max_n_phi + 2)
        self.hits_bytes = 8 * slots
        self.hits_fill = float((w.n_theta.astype(np.int64) * w.n_phi + 2).sum()) / slots if P else 0.0

    def hits_bound(self):
        """max_n_theta for rc_params when the hits pass pays: its buffer at most
        32 GiB and at least a quarter filled (measured faster at fills of 0.34
        and 1.0, with the wider-row record kernel it enables), else 0."""
        return self.max_n_theta if (self.hits_bytes <= 32 << 30 and self.hits_fill >= 0.25) else 0

    def outputs(self):
        import torch
        P = self.pos.shape[0]
        dev = self.pos.device
        return (torch.empty((P, 2), dtype=torch.float64, device=dev),
                torch.empty((P, 2, 3), dtype=torch.float64, device=dev),
                torch.empty((P, 2, 6), dtype=torch.float64, device=dev))

    def workspace(self):
        import torch
        return torch.zeros(rc_workspace_size(self.pos.shape[0]), dtype=torch.uint8, device=self.pos.device)


def compute_records(scene: Scene, dw: DeviceWorkload, batched=False, use_graph=False, tile=-1, order=None,
                    precision=0, counters=None, out=None, workspace=None, stream=None, splits=0, shadow_bvh=False,
                    hits_pass=True, shadow_pass=False):
    """Records for every point of a DeviceWorkload; returns (value, grad, hess, workspace).
    hits_pass: give rc_records_batched the batch's largest n_theta (primary rays
    traced in a separate coherent pass, ignored with counters) when
    DeviceWorkload.hits_bound says the pass pays."""
    w = dw.w
    value, grad, hess = out if out is not None else dw.outputs()
    ws = workspace if workspace is not None else dw.workspace()
    prm = make_params(w.ring_step, w.max_rings, dw.max_n_phi, w.seed, 0, precision, counters, splits=splits,
                      shadow_bvh=shadow_bvh,
                      max_n_theta=dw.hits_bound() if (hits_pass and batched and counters is None) else 0,
                      shadow_pass=shadow_pass)
    if batched:
        rc_records_batched(scene.handle, w.sigma_s, w.sigma_a, w.lights, dw.pos, dw.n_theta, dw.n_phi, prm, order,
                           use_graph, tile, value, grad, hess, ws, stream)
    else:
        rc_records(scene.handle, w.sigma_s, w.sigma_a, w.lights, dw.pos, dw.n_theta, dw.n_phi, prm, value, grad,
                   hess, ws, stream)
    return value, grad, hess, ws
