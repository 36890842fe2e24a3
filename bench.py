#!/usr/bin/env python3
"""Benchmark: radiance-cache records (value + gradient + Hessian) per second.

Headline workload (default): 1M cache points uniform in a closed room with
20 occluder slabs and a random triangle soup (1M triangles), 2048 stratified
directions per point (32 x 64), sigma_s = 2.0, sigma_a = 0.5, four point
lights, ring step 0.1; seeded synthetic inputs resident in device memory
before timing.

One step = the whole record path over the batch: the device-built queue and
the persistent, graph-replayed record kernel (directions, BVH traversal,
light-bin shadow segments, shading, rings, triangulation, per-triangle
derivative terms, reductions) followed by the validity-radius kernel.

Prints one JSON line.  Extra fields: Mrays/s (counted rays), the roofline of
the dominant kernel (record_kernel: VALU issue, from the committed counter
summary of the same kernel source, over the live kernel time), the FP64 CPU
oracle's rate on a bounded sample of the same workload together with the
per-output error of the timed launch's records on that sample, the two
smaller record workloads (10k points over 10k triangles; 200k points with
mixed sample counts over 100k triangles), the render pass that consumes a
cache (128 x 128 pixels x 16 samples marched with step 0.1, misses inserted)
and the learned-vs-plain placement comparison.

`--summarize-counters DIR` turns the CSV output of the rocprofv3 counter
passes (and of `--copy-calibration` runs) into the counter summary that the
roofline reads; the commands are listed in the summary itself.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a wave64 VALU
# instruction occupies its SIMD for 4 cycles), in 1e12 lane-operations per s
VALU_PEAK = 256 * 4 * 16 * 2.4e9 / 1e12
METRIC = "cache records/s (value+grad+Hessian) & Mrays/s; learned vs plain at equal error"
WORKLOAD_TEXT = {
    "c2": "10k points, closed unit room + 10k-triangle soup (edge 0.02), 1024 directions (16x64), "
          "sigma_s=1.0 sigma_a=0.2, 4 point lights, ring step 0.1",
    "c3": "200k points, room + 20 slabs + soup (100k triangles), directions log-uniform in [256, 4096], "
          "sigma_s=1.0 sigma_a=0.2, 4 point lights, ring step 0.1, one batched launch",
    "c5": "1M points, room + 20 slabs + soup (1M triangles), 2048 directions (32x64), sigma_s=2.0 "
          "sigma_a=0.5, 4 point lights, ring step 0.1",
}
RENDER_PREPOP_BATCH = 512  # pre-population rounds (fastest of 256..4096 with shuffled rays)
EXTRA_STEPS = {"c2": (20, 2), "c3": (5, 1), "c5": (2, 1)}
COUNTERS = ROOT / "profiles" / "record_kernel_counters.json"


def log(*a):
    print(f"[{time.strftime('%H:%M:%S')}]", *a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """sha256 prefix of the sources that make the record kernel and its launches
    (every file of paper_1805_09258_amd/csrc but the learned-placement,
    render-pass and comparison-method ones, which build other kernels)."""
    h = hashlib.sha256()
    for p in sorted((ROOT / "paper_1805_09258_amd" / "csrc").glob("*")):
        if p.suffix in (".hip", ".hpp", ".cpp") and not p.stem.startswith(("learned", "render", "j08")):
            h.update(p.read_bytes())
    return h.hexdigest()[:16]


def committed_counters(workload):
    """Per-dispatch counters of record_kernel on this workload from the committed
    summary, if it was taken on the current kernel source; else None."""
    if not COUNTERS.exists():
        return None
    try:
        d = json.loads(COUNTERS.read_text())
    except ValueError:
        return None
    if d.get("kernel_source_sha") != kernel_source_hash():
        return None
    return d.get("workloads", {}).get(workload)


def compulsory_bytes(w, info):
    """Bytes one launch must move at least: per-record inputs (position, two
    sample counts) and FP64 outputs (2-channel value, gradient, Hessian), the
    scene's device structures and the light bins, each once."""
    per_rec = 12 + 8 + 8 * (2 + 6 + 12)
    return w.n_rec * per_rec + info["device_bytes"] + info["light_bin_bytes"]


def cpu_baseline(w, outputs, budget_s=15.0):
    """The FP64 oracle, as it stands, on a bounded sample of the workload; the
    timed launch's records on the same sample are compared with it."""
    from oracle import oracle as O
    from tests._compare import ETA, TOL_G, TOL_H, TOL_V, rel_errors
    t_scene = time.perf_counter()
    sc = O.Scene.from_workload(w)
    t_scene = time.perf_counter() - t_scene
    rng = np.random.default_rng(2024)
    idx = np.sort(rng.choice(w.n_rec, size=16, replace=False))
    t0 = time.perf_counter()
    O.records_for(w, idx, scene=sc)
    t1 = time.perf_counter() - t0
    n = int(min(w.n_rec, max(16, 16 * budget_s / max(t1, 1e-3))))
    idx = np.sort(rng.choice(w.n_rec, size=n, replace=False))
    t0 = time.perf_counter()
    ref = O.records_for(w, idx, scene=sc)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = min(cores, os.cpu_count() or cores)
    value, grad, hess = (t.cpu().numpy()[idx] for t in outputs)
    ev, eg, eh, _, _ = rel_errors(value, grad, hess, ref)

    def q(e, tol):
        return {"median": float(np.median(e)), "p99": float(np.quantile(e, 0.99)), "max": float(e.max()),
                "tol": tol}
    return {"value": n / dt, "unit": "records/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} of {w.n_rec} records (seeded), same scene and sample counts, {dt:.1f} s "
                      f"(+{t_scene:.1f} s for the oracle's own BVH, not counted)",
            "cpu": O.cpu_info()["model"],
            "precision_vs_oracle": {"records": n, "channels": 2, "value": q(ev, TOL_V), "gradient": q(eg, TOL_G),
                                    "hessian_frobenius": q(eh, TOL_H),
                                    "note": f"relative errors of the timed launch's records; gradient and Hessian "
                                            f"denominators floored at {ETA} x the sum of per-triangle term norms"}}


def learned_vs_plain(dev):
    """Learned vs plain cache placement over one held-out scene of the 10k-
    triangle family: candidates resolved per second by each pipeline, and each
    cache's error against the dense plain cache (records at the test points
    with the random numbers every cached record uses)."""
    from paper_1805_09258_amd import placement as PL
    r = PL.compare(dev, log=log)
    lp, pl = r["learned"], r["plain"]
    keep = ("seconds", "rounds", "records", "accepted", "rel_l2", "median_rel", "rel_l2_far_from_lights",
            "covered", "mean_hits", "batch")
    res = {"candidates": r["candidates"],
           "plain": {k: pl[k] for k in keep if k in pl},
           "learned": {k: lp[k] for k in keep + ("probes", "records_learned", "passes", "uncovered_after_judge",
                                                 "fallback_rounds", "fallback_records", "seconds_rounds",
                                                 "seconds_records_judge", "seconds_fallback", "safety") if k in lp},
           "independent_records_error": r["independent_records"],
           "training": {k: r[k] for k in ("train_samples", "train_data_seconds", "train_seconds", "train_mse",
                                          "heldout_mse_net", "heldout_mse_constant")},
           "safety_by_validation": r["safety_validation"],
           "plain_by_batch": r["plain_by_batch"]}
    for k in ("reference", "epsilon", "error_band"):
        res[k] = r[k]
    an = r["anisotropic_plain"]
    res["anisotropic_plain"] = {k: an[k] for k in keep if k in an}
    res["j08_by_eps"] = {e: {k: v[k] for k in keep + ("eps_j08",) if k in v} for e, v in r["j08_by_eps"].items()}
    eq = r["j08_equal_error"]
    res["j08_equal_error"] = None if eq is None else {k: eq[k] for k in keep + ("eps_j08",) if k in eq}
    if eq is not None:
        res["j08_equal_error"]["candidates_per_s"] = r["candidates"] / eq["seconds"]
        res["j08_equal_error"]["points_over_ours"] = eq["accepted"] / pl["accepted"]
        res["j08_equal_error"]["seconds_over_ours"] = eq["seconds"] / pl["seconds"]
    res["anisotropic_plain"]["candidates_per_s"] = r["candidates"] / an["seconds"]
    res["plain"]["candidates_per_s"] = r["candidates"] / pl["seconds"]
    res["learned"]["candidates_per_s"] = r["candidates"] / lp["seconds"]
    res["speedup"] = pl["seconds"] / lp["seconds"]
    return res


def render_pass(dev, reps=3):
    """The render pass that consumes the cache: 128 x 128 pixels x 16 samples
    marched with step 0.1 through the closed-room scene of 10k triangles,
    the cache pre-populated from one ray per pixel and completed at the
    render's march points; one untimed pass, then the median of reps."""
    from dataclasses import replace
    from paper_1805_09258_amd import placement as PL
    from paper_1805_09258_amd import render as RD
    from paper_1805_09258_amd import workloads as W
    w = W.make_c2(P=1)
    ctx = PL.SceneContext(w)
    cam, pre = W.render_camera(), W.render_camera(spp=1, seed=9, shuffle=True)
    cfg = PL.CacheConfig()
    RD.render(ctx, cam, pre, cfg, dev, prepop_batch=RENDER_PREPOP_BATCH)
    runs = sorted((RD.render(ctx, cam, pre, cfg, dev, prepop_batch=RENDER_PREPOP_BATCH)[1] for _ in range(reps)),
                  key=lambda r: r["seconds_prepop"] + r["seconds_render"])
    ctx.close()
    st = runs[reps // 2]
    st["seconds_render_runs"] = [r["seconds_render"] for r in runs]
    st["workload"] = (f"{cam.width} x {cam.height} pixels x {cam.spp} samples, march step 0.1, pre-population "
                      f"from {pre.spp} ray per pixel in random order (rounds of {RENDER_PREPOP_BATCH}); closed unit "
                      f"room + 10k triangles, 4 point lights; {cfg.n_theta * cfg.n_phi}-direction records, "
                      f"eps {cfg.eps}; misses in rounds of {cfg.batch}")
    st["seconds_per_frame"] = st["seconds_prepop"] + st["seconds_render"]
    st["records_per_march_point"] = (st["prepop_records"] + st["render_records"]) / st["march_points"]
    # the comparison method's render at the tolerance where its cache reaches this method's cache error
    cj = replace(cfg, method="j08", j08_eps=0.7)
    ctx = PL.SceneContext(w)
    RD.render(ctx, cam, pre, cj, dev, prepop_batch=RENDER_PREPOP_BATCH)
    rj = sorted((RD.render(ctx, cam, pre, cj, dev, prepop_batch=RENDER_PREPOP_BATCH)[1] for _ in range(reps)),
                key=lambda r: r["seconds_prepop"] + r["seconds_render"])[reps // 2]
    ctx.close()
    keep = ("prepop_records", "prepop_cache", "render_records", "cache_points", "inserted", "uncovered_after",
            "seconds_prepop", "seconds_render", "pixel_mean", "ms")
    st["comparison_method"] = dict({k: rj[k] for k in keep}, eps_j08=cj.j08_eps,
                                   seconds_per_frame=rj["seconds_prepop"] + rj["seconds_render"])
    return st


def j08_vs_ours(dev, reps=5, eps_j08=0.3):
    """The comparison method's records (occlusion-unaware gradients and the
    gradient-norm radius, eps = 0.3 as in the paper's Patio comparison)
    against this method's records on the 10k-point workload: records/s of
    each (same samples) and the radius distribution of each at its own
    tolerance (the paper reports that the gradient-norm radius piles up at
    the minimum radius near surfaces and lights)."""
    import torch
    from paper_1805_09258_amd import placement as PL
    from paper_1805_09258_amd import rc
    from paper_1805_09258_amd import workloads as W
    w = W.make_c2()
    sc = rc.Scene.from_workload(w)
    dw = rc.DeviceWorkload(w, device=dev)
    P = w.n_rec
    cfg = PL.CacheConfig()
    val = torch.zeros((P, 2), dtype=torch.float64, device=dev)
    grad = torch.zeros((P, 2, 3), dtype=torch.float64, device=dev)
    mom = torch.zeros((P, 2), dtype=torch.float64, device=dev)
    Rj = torch.zeros(P, dtype=torch.float32, device=dev)
    prm = rc.make_params(w.ring_step, w.max_rings, int(w.n_phi.max()), w.seed)

    def j08():
        rc.rc_j08_records(sc.handle, w.sigma_s, w.sigma_a, w.lights, dw.pos, dw.n_theta, dw.n_phi, prm, eps_j08,
                          cfg.r_min, cfg.r_max, val, grad, mom, Rj)

    def timed(fn):
        fn()
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[reps // 2]
    tj = timed(j08)
    out = dw.outputs()
    ws = dw.workspace()
    to = timed(lambda: rc.compute_records(sc, dw, batched=True, out=out, workspace=ws, hits_pass=True))
    v, g, h = out[:3] if isinstance(out, tuple) else out
    Ro = torch.zeros(P, dtype=torch.float32, device=dev)
    rc.rc_radius(v, h, cfg.eps, cfg.r_min, cfg.r_max, Ro)
    torch.cuda.synchronize()
    sc.close()

    def dist(R):
        R = R.double()
        return {"median": float(R.median().item()), "at_r_min": float((R <= cfg.r_min * 1.0001).double().mean().item()),
                "mean": float(R.mean().item())}
    return {"workload": "10k points, closed unit room + 10k-triangle soup, 1024 directions, 4 point lights",
            "j08": {"seconds": tj, "records_per_s": P / tj, "eps": eps_j08, "radius": dist(Rj)},
            "ours": {"seconds": to, "records_per_s": P / to, "eps": cfg.eps, "radius": dist(Ro)},
            "time_per_record_ratio": tj / to, "r_min": cfg.r_min, "r_max": cfg.r_max}


def measure(name, dev, steps, warmup, count=True):
    """Build the workload and scene, autotune the launch, time `steps` steps
    (HIP events on the launch stream around the record launch; wall clock
    around the whole step) and return the figures and device outputs."""
    import torch
    from paper_1805_09258_amd import rc
    from paper_1805_09258_amd import workloads as W
    w = W.make(name)
    ndir = (w.n_theta.astype(np.int64) * w.n_phi).astype(np.float64)
    log(f"workload {name}: {w.n_rec} records, {w.n_tri} triangles, N mean {ndir.mean():.0f} "
        f"[{ndir.min():.0f}, {ndir.max():.0f}]")
    scene = rc.Scene.from_workload(w)
    dw = rc.DeviceWorkload(w, device=dev)
    value, grad, hess = dw.outputs()
    ws = dw.workspace()
    R = torch.empty(w.n_rec, dtype=torch.float32, device=dev)
    stream = torch.cuda.Stream()
    eps, r_min, r_max = 1.5e-4, 1e-3, 0.25 * float(np.linalg.norm(w.box_hi - w.box_lo))
    res = {"workload": WORKLOAD_TEXT[name], "records_per_step": w.n_rec, "n_triangles": w.n_tri,
           "directions_mean": float(ndir.mean())}
    rays = None
    if count:
        # untimed: algorithmic work of one launch (rays, fetches, terms, per-phase clocks), counted
        # with one wavefront per record so that rows recomputed by split records are not counted
        cnt = torch.zeros(12, dtype=torch.int64, device=dev)
        with torch.cuda.stream(stream):
            rc.compute_records(scene, dw, batched=True, counters=cnt, out=(value, grad, hess), workspace=ws,
                               stream=stream, splits=1 if w.n_rec <= 16384 else 0)
        stream.synchronize()
        (rays, nodes, tris, terms, c0, c1, c2, c3, sh_iter, sh_busy, sh_refill,
         sh_lanes) = (int(x) for x in cnt.cpu().tolist())
        ctot = max(c0 + c1 + c2 + c3, 1)
        res["counts"] = {"rays": rays, "node_fetches": nodes, "triangle_tests": tris, "triangle_terms": terms,
                         "phase_clock_fraction": {"primary_rays": c0 / ctot, "shadow_segments": c1 / ctot,
                                                  "mc_value": c2 / ctot, "triangle_terms": c3 / ctot},
                         "note": "node fetches come from the primary rays' BVH traversal; triangle tests include "
                                 "the light-bin entries the shadow segments test"}
        if sh_iter:  # the BVH shadow loop (light bins off)
            res["counts"]["shadow_loop"] = {"iterations": sh_iter, "lane_utilisation": sh_busy / max(64 * sh_iter, 1),
                                            "refills": sh_refill, "lanes_per_refill": sh_lanes / max(sh_refill, 1)}
        log(f"counted launch: {rays} rays, {nodes} node fetches, {tris} triangle tests, {terms} terms")
    # untimed: the launch configuration, chosen by the autotuner over the persistent-grid tiles
    # (measured on the first 20k records)
    prm = rc.make_params(w.ring_step, w.max_rings, dw.max_n_phi, w.seed, max_n_theta=dw.hits_bound())
    nt = min(w.n_rec, 20_000)
    tile, tile_ms = rc.rc_autotune(scene.handle, w.sigma_s, w.sigma_a, w.lights, dw.pos[:nt], dw.n_theta[:nt],
                                   dw.n_phi[:nt], prm, value[:nt], grad[:nt], hess[:nt], ws, stream=stream)
    stream.synchronize()
    log(f"autotune: tile {tile} ({', '.join(f'{t:.1f}' for t in tile_ms)} ms)")

    def step(ev=None):
        with torch.cuda.stream(stream):
            if ev is not None:
                ev[0].record(stream)
            rc.compute_records(scene, dw, batched=True, use_graph=True, tile=tile, out=(value, grad, hess),
                               workspace=ws, stream=stream)
            if ev is not None:
                ev[1].record(stream)
            rc.rc_radius(value, hess, eps, r_min, r_max, R, None, stream=stream)

    for i in range(warmup):
        step()
        stream.synchronize()
        log(f"{name} warmup {i + 1}/{warmup}")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(evs[i])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    errs = rc.rc_workspace_errors(ws)
    assert errs == 0, f"{errs} invalid records"
    info = scene.info()
    scene.close()
    res.update({"records_per_s": w.n_rec * steps / dt, "ms_per_step": dt / steps * 1e3,
                "record_launch_ms": kern_ms, "steps": steps, "warmup": warmup,
                "bvh_nodes": info["n_nodes"], "bvh_depth": info["depth"],
                "scene_device_bytes": info["device_bytes"], "light_bin_bytes": info["light_bin_bytes"],
                "light_bin_entries": info["light_bin_entries"],
                "tile": tile, "tile_settings": rc.rc_tile_info(tile), "tile_ms": tile_ms,
                "compulsory_bytes": compulsory_bytes(w, info)})
    if rays is not None:
        res["mrays_per_s"] = rays * steps / dt / 1e6
        res["rays_per_record"] = rays / w.n_rec
    log(f"{name}: {steps} steps, {res['ms_per_step']:.3f} ms/step, record launch {kern_ms:.3f} ms, "
        f"{res['records_per_s']:.0f} records/s")
    return w, res, (value, grad, hess)


def roofline(name, res):
    """VALU-issue roofline of one record step (the primary-hit pass and the
    record kernel's launches): lane-operations issued per step (SQ_INSTS_VALU
    x 64 from the committed counters of this kernel source) over the live step
    time, and per kernel from the counter passes; traffic beyond L2 from
    FETCH_SIZE/WRITE_SIZE scaled by a plain copy's reading."""
    c = committed_counters(name)
    kern_s = res["record_launch_ms"] * 1e-3
    out = {"bound": "alu", "achieved": None, "peak": VALU_PEAK, "unit": "T VALU lane-ops/s", "frac": None,
           "traffic": None, "kernel": "record step: primary_kernel (hits pass) + record_kernel",
           "kernel_ms": res["record_launch_ms"], "compulsory_bytes": res["compulsory_bytes"]}
    if c is None:
        out["note"] = "no counter summary for this kernel source: achieved and traffic unmeasured"
        return out
    lane_ops = c["per_dispatch"]["SQ_INSTS_VALU"] * 64
    out["achieved"] = lane_ops / kern_s / 1e12
    out["frac"] = out["achieved"] / VALU_PEAK
    out["valu_lane_ops_per_launch"] = lane_ops
    out["profiled_kernel_ms"] = c["duration_ms"]
    d = c.get("derived", {})
    for k in ("valu_busy", "waves_per_simd", "vmem_wait_frac", "tcp_hit", "tcc_hit", "clock_ghz"):
        if k in d:
            out[k] = d[k]
    per_k = {}
    for kn, e in c.get("by_kernel", {}).items():
        k = {"profiled_ms": e.get("ms")}
        if "valu_lane_ops_per_s" in e:
            k["achieved"] = e["valu_lane_ops_per_s"] / 1e12
            k["frac"] = k["achieved"] / VALU_PEAK
        if "valu_busy" in e:
            k["valu_busy"] = e["valu_busy"]
        if "TCC_HIT_sum" in e and "TCC_MISS_sum" in e:
            k["tcc_hit"] = e["TCC_HIT_sum"] / max(e["TCC_HIT_sum"] + e["TCC_MISS_sum"], 1)
        per_k[kn.replace("rc::", "")] = k
    if per_k:
        out["by_kernel"] = per_k
    if "hbm_bytes" in c:
        out["traffic"] = c["hbm_bytes"]
        out["traffic_gbs"] = c["hbm_bytes"] / kern_s / 1e9
        out["traffic_over_compulsory"] = c["hbm_bytes"] / res["compulsory_bytes"]
    return out


# ---------------------------------------------------------------------------------------------
# counter summary (rocprofv3 CSV -> profiles/record_kernel_counters.json)

def _read_pmc(d):
    """{(pass, dispatch): {name, dur_ns, grid, counters...}} from rocprofv3 CSV under d/<pass>/."""
    rows = {}
    for f in sorted(glob.glob(f"{d}/*/*_counter_collection.csv")):
        tag = Path(f).parent.name
        for r in csv.DictReader(open(f)):
            key = (tag, int(r["Dispatch_Id"]))
            e = rows.setdefault(key, {"name": r["Kernel_Name"], "grid": int(r["Grid_Size"]),
                                      "dur_ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"]),
                                      "vgpr": int(r["VGPR_Count"]), "scratch": int(r["Scratch_Size"]),
                                      "lds": int(r["LDS_Block_Size"])})
            e[r["Counter_Name"]] = float(r["Counter_Value"])
    return rows


def summarize_counters(d, workload, steps, copy_dir=None, launches=1):
    """Counters of the timed steps: per pass, the last `steps` steps of
    `launches` dispatches each (the primary-hit pass, in chunks, and one
    record_kernel launch per n_phi class of a batched launch, empty classes
    included), summed per step, averaged over steps and passes; also per
    kernel."""
    rows = _read_pmc(d)
    per, durs, meta = {}, [], None
    by_kernel = {}
    info_keys = ("name", "grid", "dur_ns", "vgpr", "scratch", "lds")
    for tag in sorted({k[0] for k in rows}):
        ks = [k for k in sorted(rows) if k[0] == tag and ("record_kernel" in rows[k]["name"] or
                                                           "primary_kernel" in rows[k]["name"])
              and ", true," not in rows[k]["name"]]
        if len(ks) < steps * launches:
            continue
        ks = ks[-steps * launches:]
        for st in range(steps):
            grp = ks[st * launches:(st + 1) * launches]
            meta = max((rows[k] for k in grp if "record_kernel" in rows[k]["name"]), key=lambda r: r["dur_ns"])
            durs.append(sum(rows[k]["dur_ns"] for k in grp) / 1e6)
            tot, kt = {}, {}
            for k in grp:
                kn = rows[k]["name"].split("(")[0].replace("void ", "")
                e = kt.setdefault(kn, {"ms": 0.0})
                e["ms"] += rows[k]["dur_ns"] / 1e6
                for c, v in rows[k].items():
                    if c not in info_keys:
                        tot[c] = tot.get(c, 0.0) + v
                        e[c] = e.get(c, 0.0) + v
            for c, v in tot.items():
                per.setdefault(c, []).append(v)
            for kn, e in kt.items():
                for c, v in e.items():
                    by_kernel.setdefault(kn, {}).setdefault(c, []).append(v)
    m = {c: float(np.mean(v)) for c, v in per.items()}
    # per kernel: each counter averaged over the steps that read it (its pass)
    kern = {kn: {c: float(np.mean(v)) for c, v in e.items()} for kn, e in by_kernel.items()}
    for kn, e in kern.items():
        if "SQ_INSTS_VALU" in e and e.get("ms"):
            e["valu_lane_ops_per_s"] = e["SQ_INSTS_VALU"] * 64 / (e["ms"] * 1e-3)
        if "SQ_ACTIVE_INST_VALU" in e and e.get("GRBM_GUI_ACTIVE"):
            e["valu_busy"] = e["SQ_ACTIVE_INST_VALU"] * 4 / (e["GRBM_GUI_ACTIVE"] / 8 * 1024)
    cu, simd = 256, 1024
    derived = {}
    if "GRBM_GUI_ACTIVE" in m:
        gui = m["GRBM_GUI_ACTIVE"] / 8  # summed over the 8 XCDs
        derived["clock_ghz"] = gui / (np.mean(durs) * 1e6)
        if "SQ_ACTIVE_INST_VALU" in m:
            # per-wave VALU issue cycles (quad-cycles, x4) over the SIMD cycles of the launch
            derived["valu_busy"] = m["SQ_ACTIVE_INST_VALU"] * 4 / (gui * simd)
        if "SQ_WAVE_CYCLES" in m:
            derived["waves_per_simd"] = m["SQ_WAVE_CYCLES"] * 4 / (gui * simd)
    if "SQ_WAIT_INST_ANY" in m and "SQ_WAVE_CYCLES" in m:
        derived["vmem_wait_frac"] = m["SQ_WAIT_INST_ANY"] / m["SQ_WAVE_CYCLES"]
    if "TCP_TOTAL_CACHE_ACCESSES_sum" in m and "TCP_TCC_READ_REQ_sum" in m:
        derived["tcp_hit"] = 1 - m["TCP_TCC_READ_REQ_sum"] / max(m["TCP_TOTAL_CACHE_ACCESSES_sum"], 1)
    if "TCC_HIT_sum" in m and "TCC_MISS_sum" in m:
        derived["tcc_hit"] = m["TCC_HIT_sum"] / max(m["TCC_HIT_sum"] + m["TCC_MISS_sum"], 1)
    out = {"kernel": meta["name"] if meta else None, "grid": meta["grid"] if meta else None,
           "vgpr": meta["vgpr"] if meta else None, "scratch_bytes_per_lane": meta["scratch"] if meta else None,
           "lds_bytes": meta["lds"] if meta else None, "steps": len(durs), "launches_per_step": launches,
           "duration_ms": float(np.mean(durs)) if durs else None, "per_dispatch": m, "derived": derived,
           "by_kernel": kern}
    if copy_dir:
        crows = _read_pmc(copy_dir)
        fs = [r["FETCH_SIZE"] for r in crows.values() if "FETCH_SIZE" in r and r["dur_ns"] > 1e5]
        wsz = [r["WRITE_SIZE"] for r in crows.values() if "WRITE_SIZE" in r and r["dur_ns"] > 1e5]
        nbytes = 1 << 30
        cal = {"bytes_copied": nbytes}
        if fs:
            cal["fetch_size_kib"] = fs
            cal["fetch_scale"] = nbytes / (np.median(fs) * 1024)
        if wsz:
            cal["write_size_kib"] = wsz
            cal["write_scale"] = nbytes / (np.median(wsz) * 1024)
        out["copy_calibration"] = cal
        if "FETCH_SIZE" in m and "WRITE_SIZE" in m and "fetch_scale" in cal and "write_scale" in cal:
            out["hbm_fetch_bytes"] = m["FETCH_SIZE"] * 1024 * cal["fetch_scale"]
            out["hbm_write_bytes"] = m["WRITE_SIZE"] * 1024 * cal["write_scale"]
            out["hbm_bytes"] = out["hbm_fetch_bytes"] + out["hbm_write_bytes"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5", choices=["c2", "c3", "c5"],
                    help="c5 (default: 1M points over 1M triangles); c2 = 10k points over 10k triangles; "
                         "c3 = 200k points with mixed sample counts over 100k triangles")
    ap.add_argument("--extra", default="c2,c3",
                    help="comma-separated smaller workloads also measured (own step counts), or 'none'")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-plain placement comparison")
    ap.add_argument("--no-render", action="store_true", help="skip the render pass that consumes the cache")
    ap.add_argument("--render-only", action="store_true", help="only the render pass (its own JSON line)")
    ap.add_argument("--no-j08", action="store_true", help="skip the comparison method's records")
    ap.add_argument("--no-count", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 1 GiB float32 buffer three times (scales the HBM byte counters)")
    ap.add_argument("--summarize-counters", metavar="DIR", default=None,
                    help="write the counter summary from rocprofv3 CSV passes under DIR (and DIR/copy)")
    ap.add_argument("--commands", default="", help=argparse.SUPPRESS)
    ap.add_argument("--launches-per-step", type=int, default=1, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (--gpus {args.gpus} requested); records are independent "
              "and the multi-GPU path is not built.", file=sys.stderr)
        sys.exit(2)

    if args.summarize_counters:
        d = Path(args.summarize_counters)
        s = summarize_counters(d, args.workload, args.steps, copy_dir=d / "copy" if (d / "copy").exists() else None,
                               launches=args.launches_per_step)
        s["kernel_source_sha"] = kernel_source_hash()
        s["commands"] = [c for c in args.commands.split(";;") if c]
        doc = json.loads(COUNTERS.read_text()) if COUNTERS.exists() else {}
        if doc.get("kernel_source_sha") != s["kernel_source_sha"]:
            doc = {"kernel_source_sha": s["kernel_source_sha"], "workloads": {}}
        doc["workloads"][args.workload] = s
        COUNTERS.write_text(json.dumps(doc, indent=1) + "\n")
        print(json.dumps(s, indent=1))
        return

    import torch
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copied 3 x 1 GiB")
        return
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.render_only:
        print(json.dumps({"render_pass": render_pass(dev)}), flush=True)
        return

    w, res, outputs = measure(args.workload, dev, args.steps, args.warmup, count=not args.no_count)
    out = {
        "metric": METRIC,
        "value": res["records_per_s"],
        "unit": "records/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {k: res[k] for k in ("workload", "records_per_step", "n_triangles", "directions_mean",
                                       "bvh_nodes", "bvh_depth", "light_bin_entries", "tile", "tile_settings",
                                       "tile_ms")},
        "mrays_per_s": res.get("mrays_per_s"),
        "rays_per_record": res.get("rays_per_record"),
        "roofline": roofline(args.workload, res),
    }
    if "counts" in res:
        out["counts"] = res["counts"]
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w, outputs)
        log(f"cpu baseline {out['cpu_baseline']['value']:.2f} records/s")
    del outputs
    torch.cuda.empty_cache()
    extra = [] if args.extra == "none" else [e for e in args.extra.split(",") if e and e != args.workload]
    if extra:
        out["workloads"] = {}
    for e in extra:
        st, wu = EXTRA_STEPS[e]
        _, r, o = measure(e, dev, st, wu)
        del o
        torch.cuda.empty_cache()
        r["roofline"] = roofline(e, r)
        out["workloads"][e] = r
    if not args.no_render:
        log("render pass ...")
        out["render_pass"] = render_pass(dev)
        log("render pass", out["render_pass"])
    if not args.no_j08:
        log("comparison method's records ...")
        out["j08_vs_ours"] = j08_vs_ours(dev)
        log("j08 vs ours", out["j08_vs_ours"])
    if not args.no_learned:
        log("learned vs plain placement ...")
        out["learned_vs_plain"] = learned_vs_plain(dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
