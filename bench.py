#!/usr/bin/env python3
"""Benchmark of the differentiable camera + lidar Gaussian rasterizer on one MI355X.

Workload (default): a 128-beam x 2048-azimuth spinning lidar (100 ms rolling-shutter sweep,
15 m/s ego velocity) plus one 1920x1080 rolling-shutter camera at the lidar origin, over 2M
synthetic Gaussians in a 300 x 300 x 6 m box; forward + backward (projection, binning, depth
sort, compositing, adjoint) every step.  The lidar carries measured ranges, so each step also
sums the line-of-sight opacities of its rays and back-propagates their upstream gradient.
Inputs are resident in HBM before timing starts.

Three forms of the same step are timed:
  plain   -- per-sensor calls (project -> bin/sort -> rasterize_fwd -> rasterize_bwd per sensor);
  batched -- one call per stage for both sensors (one projection launch, one bin/sort building
             a cost-ordered work queue, persistent forward and adjoint rasterisers);
  graph   -- the batched step captured once as a hipGraph (splat_pipeline_*) and replayed.
Each is checked against the FP64 oracle on sampled rays before timing, and also timed
forward-only (project -> bin/sort -> rasterize_fwd).

Prints one JSON line.  `value` is the batched form's rays (pixels + lidar rays) per second of whole
fwd+bwd steps, in Mrays/s, launched from the stream or replayed from the captured graph, whichever
is faster (`config.launch` says which); every form is reported beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s fwd+bwd, 128x2048 lidar + 1080p camera; batched vs plain at 1e-4 err"

# MI355X published peaks
PEAK_FP32_TFLOPS = 157.3            # FP32, datasheet (vector packed FMA; also the dense FP32 matrix-core rate)
PEAK_HBM_GBS = 8000.0               # HBM3E, datasheet
SEED_COMPOSE = 16816 + 11           # seed of the composition workload
SEED_POINTS = 16816 + 12            # seed of the lidar points-to-rays workload
SEED_DECODER = 16816 + 13           # seed of the lidar decoder workload (weights, features)
SEED_CNN = 16816 + 14               # seed of the camera decoder workload
SEED_RELOC = 16816 + 15             # seed of the relocation workload (dead set, draws)
# algorithmic FP32 work per evaluated (ray, Gaussian) pair of the forward compositing loop:
# Delta (6), sigma (9), exp (1), alpha (1), transmittance (2), weight (1), feature and depth
# blends (2 C + 2), plus the lidar range correction (2) and azimuth reduction (3);
# the adjoint recomputes the pair and back-propagates through it: about 3x the forward.
FLOP_PER_PAIR = {"camera": 22 + 2 * 16, "lidar": 22 + 2 * 8 + 5}
BWD_FACTOR = 3.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=2_000_000, help="Gaussians")
    ap.add_argument("--modes", default="plain,batched,graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compose", action="store_true", help="skip the composition, points-to-rays, MCMC regulariser and decoder measurements")
    ap.add_argument("--c5", action="store_true",
                    help="instead of the headline step: the 60-sensor sweep workload (3M Gaussians, 48 lidar sweeps "
                         "+ 12 cameras) with per-sensor latency p50/p99 from in-kernel clocks")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the per-config (C1-C4) plain / batched lines")
    ap.add_argument("--cpu-rays", type=int, default=256, help="camera pixels in the CPU oracle sample")
    ap.add_argument("--cpu-lidar-rays", type=int, default=64, help="lidar rays in the CPU oracle sample")
    ap.add_argument("--profile-steps", action="store_true", help="skip parity and CPU legs (for rocprofv3)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the scene's tile shapes")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with two 1 GiB device copies (reference kernel for rocprofv3 byte counters)")
    ap.add_argument("--camera-tile", default=None, help="WxH: fixed camera tile (skips autotuning)")
    ap.add_argument("--lidar-tile", default=None,
                    help="AZxM: fixed lidar tiles of AZ azimuth steps, elevation tiles merged by M (skips autotuning)")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the path is measured on one GPU's "
              f"share; its multi-GPU form (replicated Gaussians, sensors split across GPUs, one gradient "
              f"all-reduce) is a design, not a measured configuration.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2411_16816_amd import binding as B
    from scenes import synthetic as S

    if args.c5:
        print(json.dumps(c5_latency(args, "cuda")), flush=True)
        return
    t0 = time.time()
    sc = S.headline(n=args.n)
    cam, lid = sc.cameras[0], sc.lidars[0]
    g = sc.gaussians
    log(f"scene {sc.name}: {g.n} Gaussians, {sc.n_rays} rays/step, generated in {time.time() - t0:.1f}s")
    dev = "cuda"
    G = B.GaussTensors.from_numpy(g, dev)
    tiles = {"camera": [int(cam.tile_w), int(cam.tile_h)], "lidar_az_tiles": int(lid.n_az_tiles),
             "lidar_el_tiles": int(lid.n_el_tiles)}
    tune_report = None
    if args.camera_tile or args.lidar_tile:
        from paper_2411_16816_amd import autotune
        if args.camera_tile:
            tw, th = (int(x) for x in args.camera_tile.lower().split("x"))
            cam = next(c for c in autotune.camera_candidates(cam) if (c.tile_w, c.tile_h) == (tw, th))
        if args.lidar_tile:
            taz, m = (int(x) for x in args.lidar_tile.lower().split("x"))
            n_el = (lid.n_el_tiles + m - 1) // m
            lid = next(l for l in autotune.lidar_candidates(lid) if autotune._shape(l, False) == (taz, n_el))
        tiles = {"camera": [int(cam.tile_w), int(cam.tile_h)], "lidar_az_tiles": int(lid.n_az_tiles),
                 "lidar_el_tiles": int(lid.n_el_tiles)}
    elif not args.no_autotune:
        from paper_2411_16816_amd import autotune
        t1 = time.time()
        cams, lids, rep = autotune.tune_rig([cam], [lid], G, log=log)
        cam, lid = cams[0], lids[0]
        tiles = {"camera": [int(cam.tile_w), int(cam.tile_h)], "lidar_az_tiles": int(lid.n_az_tiles),
                 "lidar_el_tiles": int(lid.n_el_tiles)}
        tune_report = {("camera" if k == 0 else "lidar"): [[list(sh), round(ms, 4)] for sh, ms in v[1]]
                       for k, v in rep.items()}
        tune_report["source"] = "search" if any(v[1] for v in rep.values()) else \
            f"cache ({os.path.relpath(autotune.CACHE_PATH, ROOT)})"
        log(f"autotuned tiles {tiles} in {time.time() - t1:.1f}s ({tune_report['source']})")
    rig = B.Rig([cam], [lid], dev)
    stream = torch.cuda.current_stream()
    stages = ["project", "bin_sort", "raster_fwd", "raster_bwd"]
    results = {}
    for mode in args.modes.split(","):
        if mode == "plain":
            passes = [B.SensorPass(rig, 0, 1, g.n, 1, dev), B.SensorPass(rig, 1, 1, g.n, 1, dev)]
        else:
            passes = [B.SensorPass(rig, 0, 2, g.n, 1, dev, batched=True)]
        Ks = [sp.fit_capacity(G, 1.15) for sp in passes]
        # upstream gradients drawn per sensor; the batched form takes their concatenation, so that
        # every form differentiates the same loss
        # (dF, dD, dA, d_los): the line-of-sight weight is drawn for lidar rays, zero for pixels
        per_sensor = []
        for k, sensor in enumerate((cam, lid)):
            _, dD, dA = S.upstream_grads(1000 + k, sensor.n_rays, 1)
            dF = np.random.default_rng(1100 + k).normal(size=sensor.n_rays * sensor.n_channels).astype(np.float32)
            dl = (np.random.default_rng(1200 + k).normal(size=sensor.n_rays).astype(np.float32) if k == 1 else
                  np.zeros(sensor.n_rays, np.float32))
            per_sensor.append((dF, dD.reshape(-1), dA.reshape(-1), dl))
        if mode == "plain":
            host_ups = per_sensor
        else:
            host_ups = [tuple(np.concatenate([per_sensor[0][i], per_sensor[1][i]]) for i in range(4))]
        ups = [tuple(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev) for a in u) for u in host_ups]
        for sp, u in zip(passes, ups):
            assert u[0].numel() == sp.n_feat and u[1].numel() == sp.n_rays and u[3].numel() == sp.n_rays, \
                "upstream gradient shapes"
        grads = B.zeros_like_grads(G)
        pipe = pipe_fwd = None
        if mode == "graph":
            pipe = B.Pipeline(passes[0], G, B.BOX, grads, *ups[0][:3], zero_grads=False, d_los=ups[0][3])
            pipe_fwd = B.Pipeline(passes[0], G, B.BOX)

        def step(events=None):
            if pipe is not None:
                pipe.run()
                return
            for k, sp in enumerate(passes):
                ev = events[k] if events is not None else None
                if ev: ev["project"][0].record(stream)
                sp.project(G)
                if ev: ev["project"][1].record(stream); ev["bin_sort"][0].record(stream)
                sp.bin_sort()
                if ev: ev["bin_sort"][1].record(stream); ev["raster_fwd"][0].record(stream)
                sp.raster_fwd(G, timer=ev["k_fwd"] if ev else None)
                if ev: ev["raster_fwd"][1].record(stream); ev["raster_bwd"][0].record(stream)
                sp.raster_bwd(G, *ups[k][:3], grads, timer=ev["k_bwd"] if ev else None, d_los=ups[k][3])
                if ev: ev["raster_bwd"][1].record(stream)

        for sp in passes:
            sp.status.zero_()
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        for k, sp in enumerate(passes):
            st = B.read_status(sp.status)
            if st.overflow:
                raise SystemExit(f"{mode}: intersection overflow on pass {k}: need {st.n_isect}, have {st.k_cap}")
        parity = None
        if not (args.no_parity or args.profile_steps):
            parity = check_parity(passes, rig, g)
            log(f"{mode} parity: {parity}")
        mk = lambda: torch.cuda.Event(enable_timing=True)
        evs = [[{s: (mk(), mk()) for s in stages + ["k_fwd", "k_bwd"]} for _ in passes] for _ in range(args.steps)]
        for e in evs:          # the library records these events: create them on this stream first
            for d in e:
                for a, b in d.values():
                    a.record(stream)
                    b.record(stream)
        start, end = mk(), mk()
        marks = [mk() for _ in range(args.steps - 1)]   # step boundaries inside the timed region
        torch.cuda.synchronize()
        start.record(stream)
        for i in range(args.steps):
            step(evs[i])
            if i < args.steps - 1:
                marks[i].record(stream)
        end.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(end) / args.steps
        bounds = [start] + marks + [end]
        per_step = np.array([bounds[i].elapsed_time(bounds[i + 1]) for i in range(args.steps)])
        step_ms = {"median": round(float(np.median(per_step)), 4), "p99": round(float(np.percentile(per_step, 99)), 4),
                   "min": round(float(per_step.min()), 4), "max": round(float(per_step.max()), 4)}
        # state after the warm-up and timed steps, for the agreement check between the forms
        snap_out = {}
        for k, sp in enumerate(passes):
            o = sp.outputs()
            for key in ("feat", "depth", "alpha", "t_final", "last"):
                snap_out.setdefault(key, []).append(o[key].clone())
        snap_out = {key: torch.cat(v) for key, v in snap_out.items()}
        # the median and the line-of-sight sum are written for lidar rays only
        for key in ("median", "los"):
            snap_out[f"{key}_lidar"] = (passes[1].outputs()[key].clone() if mode == "plain" else
                                        passes[0].outputs()[key][passes[0].sensor_slices(1)[0]].clone())
        snap_grad = {name: getattr(grads, name).clone() for name in GRAD_FIELDS}
        rays = sum(sp.n_rays for sp in passes)
        names = ["camera", "lidar"] if mode == "plain" else ["both"]
        stage_ms = {} if pipe is not None else {
            f"{s}_{names[k]}": float(np.mean([e[k][s][0].elapsed_time(e[k][s][1]) for e in evs]))
            for k in range(len(passes)) for s in stages}
        # the rasteriser kernels alone (events recorded by the library around the kernel launch)
        kernel_ms = {} if pipe is not None else {
            f"{s}_{names[k]}": float(np.mean([e[k][s][0].elapsed_time(e[k][s][1]) for e in evs]))
            for k in range(len(passes)) for s in ("k_fwd", "k_bwd")}

        # forward only (project -> bin/sort -> rasterize_fwd), same step count
        def fwd_step():
            if pipe_fwd is not None:
                pipe_fwd.run()
                return
            for sp in passes:
                sp.project(G)
                sp.bin_sort()
                sp.raster_fwd(G)

        for _ in range(max(1, args.warmup)):
            fwd_step()
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(args.steps):
            fwd_step()
        end.record(stream)
        torch.cuda.synchronize()
        ms_fwd = start.elapsed_time(end) / args.steps
        # evaluated pairs (one extra forward with the counter on, outside the timed region)
        pairs = []
        for sp in passes:
            sp.status.zero_()
            sp.raster_fwd(G, count_pairs=True)
        torch.cuda.synchronize()
        sts = [B.read_status(sp.status) for sp in passes]
        pairs = [int(x.n_pairs) for x in sts]
        stopped = [int(x.n_stopped) for x in sts]
        results[mode] = dict(ms=ms, value=rays / (ms * 1e-3) / 1e6, stage_ms=stage_ms, kernel_ms=kernel_ms,
                             parity=parity, K=Ks, step_ms=step_ms, snap_out=snap_out, snap_grad=snap_grad,
                             pairs=pairs, stopped=stopped, rays=rays, ms_fwd=ms_fwd, value_fwd=rays / (ms_fwd * 1e-3) / 1e6)
        log(f"{mode}: {ms:.3f} ms/step, {results[mode]['value']:.1f} Mrays/s (forward only {ms_fwd:.3f} ms, "
            f"{results[mode]['value_fwd']:.1f} Mrays/s); stages "
            + json.dumps({k: round(v, 4) for k, v in stage_ms.items()}) + f"; pairs {pairs}")
        if pipe is not None:
            pipe.close()
            pipe_fwd.close()
        del passes, grads, pipe, pipe_fwd

    # the batched form, launched from the stream or replayed from the captured graph, whichever
    # runs faster on this machine
    batched_forms = [m for m in ("batched", "graph") if m in results]
    main_mode = max(batched_forms, key=lambda m: results[m]["value"]) if batched_forms else "plain"
    R = results[main_mode]
    roof = roofline(results, tiles) if "batched" in results else None
    cpu = None
    if not (args.no_cpu_baseline or args.profile_steps):
        cpu = cpu_baseline(g, cam, lid, args.cpu_rays, args.cpu_lidar_rays)
    out = {
        "metric": METRIC, "value": round(R["value"], 3), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(R["ms"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "lidar 128x2048 (100 ms RS, 15 m/s ego, line-of-sight sum) + 1920x1080 RS camera, "
                               "2M Gaussians, fwd+bwd",
                   "mode": "batched" if main_mode != "plain" else "plain",
                   "launch": "hipGraph replay" if main_mode == "graph" else "stream",
                   "gaussians": g.n, "rays_per_step": R["rays"], "tiles": tiles},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forward_only": {"value": round(R["value_fwd"], 3), "unit": "Mrays/s", "ms_per_step": round(R["ms_fwd"], 4)},
        "modes": {m: {"value": round(r["value"], 3), "ms_per_step": round(r["ms"], 4),
                      "forward_only_value": round(r["value_fwd"], 3), "forward_only_ms": round(r["ms_fwd"], 4),
                      "stage_ms": {k: round(v, 4) for k, v in r["stage_ms"].items()},
                      "intersections": r["K"], "evaluated_pairs": r["pairs"],
                      "pairs_per_ray": round(sum(r["pairs"]) / r["rays"], 2),
                      "early_stop_rate": round(sum(r["stopped"]) / r["rays"], 4), "parity": r["parity"]}
                  for m, r in results.items()},
    }
    for m, r in results.items():
        out["modes"][m]["step_ms"] = r["step_ms"]
    if not (args.no_configs or args.profile_steps):
        out["configs"] = {f"C{k}": config_bench(args, dev, k) for k in (1, 2, 3, 4)}
        # C5 in its batched form only (one call per stage for all 60 sensors): 60 plain passes at
        # once would hold a list and an adjoint workspace per sensor, beyond the GPU's memory
        out["configs"]["C5"] = c5_latency(args, dev, parity_sensors=[0, 11, 12, 28, 59])
    if not args.no_compose:
        out["compose"] = compose_bench(args, dev)
        out["points_to_rays"] = points_bench(args, dev, lid)
        out["mcmc_regularizer"] = mcmc_bench(args, dev, G, g)
        out["lidar_decoder"] = decoder_bench(args, dev, lid)
        out["camera_decoder"] = cnn_bench(args, dev, cam)
    agree = mode_agreement(results)
    if agree:
        out["agreement"] = agree
    if tune_report is not None:
        out["autotune_ms"] = tune_report
    if "plain" in results:
        for m in ("batched", "graph"):
            if m in results:
                out[f"{m}_over_plain"] = round(results[m]["value"] / results["plain"]["value"], 4)
    print(json.dumps(out), flush=True)
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration: 2 copies of 1 GiB")


GRAD_FIELDS = ("means", "log_scales", "quats", "opacities", "velocities", "features")


def mode_agreement(results):
    """Each form against the plain per-sensor calls on the same inputs, after the same warm-up +
    timed steps: forward outputs must be bit-identical (median and line-of-sight sum: lidar rays
    only); the accumulated gradients must agree within 1e-4 (relative norm per field)."""
    if "plain" not in results:
        return None
    ref = results["plain"]
    out = {}
    for m, r in results.items():
        if m == "plain":
            continue
        fwd_equal = True
        for key, x in r["snap_out"].items():
            y = ref["snap_out"][key]
            fwd_equal = fwd_equal and x.shape == y.shape and bool(torch_equal(x, y))
        worst = 0.0
        for name in GRAD_FIELDS:
            x = r["snap_grad"][name].double()
            y = ref["snap_grad"][name].double()
            ny = float(y.norm())
            if ny > 0:
                worst = max(worst, float((x - y).norm()) / ny)
        out[f"{m}_vs_plain"] = {"forward_bit_equal": fwd_equal, "grad_rel_err": float(f"{worst:.3g}"),
                                "pass": bool(fwd_equal and worst <= 1e-4)}
    for r in results.values():
        r.pop("snap_out", None)
        r.pop("snap_grad", None)
    return out


def torch_equal(x, y):
    import torch
    return torch.equal(x, y)


def check_parity(passes, rig, g):
    """Sampled-ray parity of the timed configuration against the FP64 oracle (1e-4 rel, 1e-5 abs)."""
    from oracle import render as rd
    res = {}
    rng = np.random.default_rng(7)
    for sp in passes:
        for k in range(sp.count):
            sensor = rig.sensors[sp.first + k]
            rs, fs, C = sp.sensor_slices(k)
            n = rs.stop - rs.start
            idx = np.sort(rng.choice(n, size=48, replace=False))
            o = sp.outputs()
            F = o["feat"][fs].reshape(-1, C)[idx].cpu().numpy()
            D = o["depth"][rs][idx].cpu().numpy()
            A = o["alpha"][rs][idx].cpu().numpy()
            ref = rd.render_sensor(g, sensor, idx)
            ok = ~ref["near"]
            worst = 0.0
            checks = [(F, ref["F"].numpy()), (D, ref["D"].numpy()), (A, ref["A"].numpy())]
            if o["los"] is not None and not hasattr(sensor, "fx"):
                checks.append((o["los"][rs][idx].cpu().numpy(), ref["los"].numpy()))
            for a, r in checks:
                a, r = a[ok], r[ok]
                err = np.abs(a - r) / (1e-5 + 1e-4 * np.abs(r))
                worst = max(worst, float(err.max()) if err.size else 0.0)
            kind = "camera" if hasattr(sensor, "fx") else "lidar"
            res[kind] = {"rays": int(len(idx)), "near_excluded": int((~ok).sum()),
                         "max_err_over_tol": round(worst, 4), "pass": bool(worst <= 1.0)}
    return res


# kernel whose roofline is reported: the batched adjoint rasteriser, the longest kernel of the step
ROOF_KERNEL = "k_raster_bwd_queue<16, 8, false, 4>"   # camera + lidar call, queue grouped by kind
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_raster_bwd_queue_headline.md")
KERNEL_SOURCES = ["paper_2411_16816_amd/csrc/raster.hip", "paper_2411_16816_amd/csrc/splat_common.hpp",
                  "paper_2411_16816_amd/csrc/wave_ops.hpp", "paper_2411_16816_amd/csrc/kernels.hpp",
                  "include/splat.h"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(tiles):
    """HBM bytes per launch of ROOF_KERNEL from the committed rocprofv3 --pmc summary, or None
    when the summary is missing, was taken on other kernel sources or on another tile layout."""
    try:
        txt = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    vals = dict(line[2:].split(": ", 1) for line in txt.splitlines() if line.startswith("- ") and ": " in line)
    if vals.get("source_hash", "").strip() != kernel_source_hash():
        return None
    if vals.get("tiles", "").strip() != json.dumps(tiles, sort_keys=True):
        return None
    try:
        return int(vals["traffic_bytes_per_launch"].strip())
    except (KeyError, ValueError):
        return None


def roofline(results, tiles):
    """VALU roofline of the batched adjoint rasteriser kernel.  Time: the kernel alone, from
    events the library records around its launch (splat_time_next_raster), averaged over the
    timed steps.  Algorithmic FLOP = evaluated pairs x FLOP per pair x 3."""
    r = results["batched"]
    plain = results.get("plain", r)
    pc = plain["pairs"]
    if len(pc) == 2:
        flop_fwd = pc[0] * FLOP_PER_PAIR["camera"] + pc[1] * FLOP_PER_PAIR["lidar"]
    else:
        flop_fwd = pc[0] * 0.5 * (FLOP_PER_PAIR["camera"] + FLOP_PER_PAIR["lidar"])
    flop_bwd = BWD_FACTOR * flop_fwd
    t_bwd = r["kernel_ms"]["k_bwd_both"] * 1e-3
    t_fwd = r["kernel_ms"]["k_fwd_both"] * 1e-3
    ach = flop_bwd / t_bwd / 1e12
    traffic = measured_traffic(tiles)
    return {"bound": "alu", "kernel": ROOF_KERNEL, "achieved": round(ach, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
            "kernel_ms": round(t_bwd * 1e3, 4), "algorithmic_flop": int(flop_bwd), "evaluated_pairs": int(sum(pc)),
            "hbm_gbs": None if traffic is None else round(traffic / t_bwd / 1e9, 1),
            "forward": {"kernel": "k_raster_fwd_queue<16, 8, false>", "kernel_ms": round(t_fwd * 1e3, 4),
                        "achieved": round(flop_fwd / t_fwd / 1e12, 3),
                        "frac": round(flop_fwd / t_fwd / 1e12 / PEAK_FP32_TFLOPS, 4)}}


def c5_parity(sc, sp, first, sensors, rays=4):
    """Forward outputs of `rays` sampled rays of each listed sensor (rig index) against the oracle."""
    from oracle import render as rd
    rig_sensors = list(sc.cameras) + list(sc.lidars)
    prng = np.random.default_rng(1905)
    worst, near, n = 0.0, 0, 0
    o = sp.outputs()
    for k in sensors:
        s_ = rig_sensors[k]
        idx = np.sort(prng.choice(s_.n_rays, size=rays, replace=False))
        ref = rd.render_sensor(sc.gaussians, s_, idx)
        rs, fs, C = sp.sensor_slices(k - first)
        ok = ~ref["near"]
        near += int((~ok).sum())
        n += len(idx)
        for a, r in ((o["feat"][fs].reshape(-1, C)[idx], ref["F"]), (o["depth"][rs][idx], ref["D"]),
                     (o["alpha"][rs][idx], ref["A"])):
            a, r = a.cpu().numpy(), r.numpy()
            err = np.abs(a[ok] - r[ok]) / (1e-5 + 1e-4 * np.abs(r[ok]))
            worst = max(worst, float(err.max()) if err.size else 0.0)
    return {"rays": n, "sensors": list(sensors), "near_excluded": near, "max_err_over_tol": round(worst, 4),
            "pass": bool(worst <= 1.0)}


def c5_latency(args, dev, parity_sensors=None):
    """The sweep workload: 3M Gaussians, 48 lidar sweeps (16 each of 32, 64 and 128 beams,
    1024-2048 azimuth steps) and 12 1080p cameras, all 60 sensors in one batched call per stage
    (persistent rasterisers; about 1.9e9 list entries, so the adjoint keeps no per-entry rows).
    Per-sensor latency = (device clock when the sensor's last work item finished) - (device
    clock stamped on the stream when the step started), fwd-only and fwd+bwd; p50 / p99 over
    the sensors and the timed steps."""
    import torch
    from paper_2411_16816_amd import binding as B
    from scenes import synthetic as S
    t0 = time.time()
    sc = S.config_5()
    n_cam = len(sc.cameras)
    log(f"C5: {sc.gaussians.n} Gaussians, {n_cam} cameras, {len(sc.lidars)} lidars, built in {time.time() - t0:.1f}s")
    rig = B.Rig(sc.cameras, sc.lidars, dev)
    G = B.GaussTensors.from_numpy(sc.gaussians, dev)
    hz = B.device_clock_hz()
    groups = [(0, n_cam + len(sc.lidars))]
    stream = torch.cuda.current_stream()
    lat = {"fwd": {"camera": [], "lidar": []}, "fwd_bwd": {"camera": [], "lidar": []}}
    ms = {"fwd": 0.0, "fwd_bwd": 0.0}
    rays_total = 0
    mk = lambda: torch.cuda.Event(enable_timing=True)
    for first, count in groups:
        sp = B.SensorPass(rig, first, count, sc.gaussians.n, 1, dev, batched=True)
        K = sp.fit_capacity(G, 1.05)
        rng = np.random.default_rng(700 + first)
        dF = torch.from_numpy(rng.normal(size=sp.n_feat).astype(np.float32)).to(dev)
        dD = torch.from_numpy((0.01 * rng.normal(size=sp.n_rays)).astype(np.float32)).to(dev)
        dA = torch.from_numpy(rng.normal(size=sp.n_rays).astype(np.float32)).to(dev)
        grads = B.zeros_like_grads(G)
        clk = torch.zeros(args.steps + 1, dtype=torch.int64, device=dev)
        kinds = ["camera" if first + k < n_cam else "lidar" for k in range(count)]
        for phase in ("fwd", "fwd_bwd"):
            done = torch.zeros(args.steps + 1, count, dtype=torch.int64, device=dev)

            def step(i):
                B.device_clock(clk, i)
                sp.project(G)
                sp.bin_sort()
                sp.raster_fwd(G, sensor_done=done[i] if phase == "fwd" else None)
                if phase == "fwd_bwd":
                    sp.raster_bwd(G, dF, dD, dA, grads, sensor_done=done[i])

            step(args.steps)   # warm-up (slot `steps`, discarded)
            torch.cuda.synchronize()
            a, b = mk(), mk()
            a.record(stream)
            for i in range(args.steps):
                step(i)
            b.record(stream)
            torch.cuda.synchronize()
            ms[phase] += a.elapsed_time(b) / args.steps
            d = done[:args.steps].cpu().numpy().astype(np.float64)
            c = clk[:args.steps].cpu().numpy().astype(np.float64)
            for k in range(count):
                lat[phase][kinds[k]].extend(((d[:, k] - c) / hz * 1e3).tolist())
        st_ = B.read_status(sp.status)
        if st_.overflow:
            raise SystemExit(f"C5 group {first}: overflow")
        rays_total += sp.n_rays
        log(f"C5 group [{first}, {first + count}): {K} entries, {sp.n_rays} rays")
        if parity_sensors:   # the last step's outputs against the oracle on sampled rays
            parity = c5_parity(sc, sp, first, parity_sensors)
        del sp, grads
        torch.cuda.empty_cache()
    pct = lambda v, q: round(float(np.percentile(np.asarray(v), q)), 4)
    out = {"metric": "C5 sweep: per-sensor latency p50/p99 and Mrays/s, fwd and fwd+bwd", "n_gpus": 1,
           "steps": args.steps, "data": "synthetic", "dtype": "f32",
           "config": {"workload": "3M Gaussians, 48 lidar sweeps (16 x 32 / 64 / 128 beams, 1024-2048 az) + "
                                  "12 RS cameras 1920x1080", "calls_per_step": len(groups),
                      "groups": [list(g_) for g_ in groups], "rays_per_step": rays_total}}
    if parity_sensors:
        out["parity"] = parity
        log(f"C5 parity {parity}")
    for phase in ("fwd", "fwd_bwd"):
        out[phase] = {"ms_per_step": round(ms[phase], 4), "Mrays_per_s": round(rays_total / (ms[phase] * 1e-3) / 1e6, 3),
                      "latency_ms": {k: {"p50": pct(v, 50), "p99": pct(v, 99), "n": len(v)}
                                     for k, v in lat[phase].items()}}
        log(f"C5 {phase}: {ms[phase]:.3f} ms/step; latency {out[phase]['latency_ms']}")
    return out


CONFIG_NAMES = {1: "C1 plain lidar forward: 4096 Gaussians, 32 x 1024 global-shutter lidar",
                2: "C2 camera fwd+bwd: 500k Gaussians (road slab), 1920x1080 RS camera",
                3: "C3 lidar fwd+bwd: 2M Gaussians, 128 x 2048 lidar, 100 ms RS sweep, 15 m/s ego",
                4: "C4 rig fwd+bwd: 1.5M Gaussians, 6 RS cameras (2x 1920x1080, 2x 1280x720, 2x 960x640) "
                   "+ 64 x 1800 lidar"}


def config_bench(args, dev, k, parity_rays=8):
    """Config k timed in both forms: plain (one call per stage per sensor) and batched (one call
    per stage for all sensors, persistent rasterisers); fwd+bwd per step (C1: forward only, as
    the config states).  Median and p99 over the timed steps; both forms checked against the
    oracle on the same sampled rays, forward outputs bit-equal between the forms and gradients
    within 1e-4."""
    import torch
    from oracle import render as rd
    from paper_2411_16816_amd import binding as B
    from scenes import synthetic as S
    sc = S.make_config(k)
    g = sc.gaussians
    sensors = list(sc.cameras) + list(sc.lidars)
    G = B.GaussTensors.from_numpy(g, dev)
    rig = B.Rig(sc.cameras, sc.lidars, dev)
    fwd_only = k == 1
    stream = torch.cuda.current_stream()
    mk = lambda: torch.cuda.Event(enable_timing=True)
    rng = np.random.default_rng(900 + k)
    ups = []
    for s_ in sensors:
        ups.append((rng.normal(size=s_.n_rays * s_.n_channels).astype(np.float32),
                    (0.1 * rng.normal(size=s_.n_rays)).astype(np.float32), rng.normal(size=s_.n_rays).astype(np.float32)))
    prng = np.random.default_rng(1900 + k)
    pidx = [np.sort(prng.choice(s_.n_rays, size=min(parity_rays, s_.n_rays), replace=False)) for s_ in sensors]
    refs = [rd.render_sensor(g, s_, idx) for s_, idx in zip(sensors, pidx)]
    out = {"workload": CONFIG_NAMES[k], "gaussians": g.n, "rays_per_step": int(sum(s_.n_rays for s_ in sensors)),
           "step": "forward" if fwd_only else "fwd+bwd"}
    snaps = {}
    for mode in ("plain", "batched"):
        if mode == "plain":
            passes = [B.SensorPass(rig, i, 1, g.n, 1, dev) for i in range(len(sensors))]
            pups = [[torch.from_numpy(a).to(dev) for a in u] for u in ups]
        else:
            passes = [B.SensorPass(rig, 0, len(sensors), g.n, 1, dev, batched=True)]
            pups = [[torch.from_numpy(np.concatenate([u[j] for u in ups])).to(dev) for j in range(3)]]
        K = [sp.fit_capacity(G, 1.1) for sp in passes]
        grads = B.zeros_like_grads(G)

        def step():
            for sp, u in zip(passes, pups):
                sp.project(G)
                sp.bin_sort()
                sp.raster_fwd(G)
                if not fwd_only:
                    sp.raster_bwd(G, *u, grads)

        for _ in range(max(1, args.warmup)):
            step()
        torch.cuda.synchronize()
        evs = [mk() for _ in range(args.steps + 1)]
        evs[0].record(stream)
        for i in range(args.steps):
            step()
            evs[i + 1].record(stream)
        torch.cuda.synchronize()
        per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
        med = float(np.median(per))
        # parity: the outputs of the last step against the oracle on the sampled rays
        worst, near, outs = 0.0, 0, []
        for si, (s_, idx, ref) in enumerate(zip(sensors, pidx, refs)):
            sp = passes[si] if mode == "plain" else passes[0]
            kk = 0 if mode == "plain" else si
            rs, fs, C = sp.sensor_slices(kk)
            o = sp.outputs()
            F = o["feat"][fs].reshape(-1, C)[idx].cpu().numpy()
            D = o["depth"][rs][idx].cpu().numpy()
            A = o["alpha"][rs][idx].cpu().numpy()
            ok = ~ref["near"]
            near += int((~ok).sum())
            for a, r in ((F, ref["F"].numpy()), (D, ref["D"].numpy()), (A, ref["A"].numpy())):
                err = np.abs(a[ok] - r[ok]) / (1e-5 + 1e-4 * np.abs(r[ok]))
                worst = max(worst, float(err.max()) if err.size else 0.0)
            outs.append((o["feat"][fs].clone(), o["depth"][rs].clone(), o["alpha"][rs].clone()))
        snaps[mode] = (outs, {n_: getattr(grads, n_).double().clone() for n_ in GRAD_FIELDS
                              if getattr(grads, n_) is not None})
        out[mode] = {"ms_per_step": round(med, 4), "p99_ms": round(float(np.percentile(per, 99)), 4),
                     "Mrays_per_s": round(out["rays_per_step"] / (med * 1e-3) / 1e6, 3), "intersections": K,
                     "calls_per_stage": len(passes),
                     "parity": {"rays": int(sum(len(i) for i in pidx)), "near_excluded": near,
                                "max_err_over_tol": round(worst, 4), "pass": bool(worst <= 1.0)}}
        log(f"{CONFIG_NAMES[k].split(':')[0]} {mode}: {med:.3f} ms/step, {out[mode]['Mrays_per_s']} Mrays/s, "
            f"parity {out[mode]['parity']}")
        del passes, grads
        torch.cuda.empty_cache()
    fwd_equal = all(torch.equal(a, b) for x, y in zip(snaps["plain"][0], snaps["batched"][0]) for a, b in zip(x, y))
    worst = 0.0
    for n_ in snaps["plain"][1]:
        x, y = snaps["batched"][1][n_], snaps["plain"][1][n_]
        ny = float(y.norm())
        if ny > 0:
            worst = max(worst, float((x - y).norm()) / ny)
    out["batched_over_plain"] = round(out["plain"]["ms_per_step"] / out["batched"]["ms_per_step"], 4)
    out["agreement"] = {"forward_bit_equal": bool(fwd_equal), "grad_rel_err": float(f"{worst:.3g}"),
                        "pass": bool(fwd_equal and worst <= 1e-4)}
    return out


def compose_bench(args, dev):
    """Scene-graph composition (splat_compose, splat_compose_bwd) on 2M Gaussians of which 30 %
    belong to 64 car-sized actors, timed with HIP events around each call over the timed steps,
    against the HBM roofline (algorithmic bytes: every array read or written once)."""
    import torch
    from oracle import compose as oc
    from paper_2411_16816_amd import binding as B
    from scenes import synthetic as S
    sc = S.actor_scene(SEED_COMPOSE, 2_000_000, 64)
    g = sc.gaussians
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    mu, q, v, aid = f(g.means), f(g.quats), f(g.velocities), torch.from_numpy(sc.actor_id).to(dev)
    A = B.ActorTensors(f(sc.rot), f(sc.trans), f(sc.rot_offset), f(sc.trans_offset), f(sc.lin_vel),
                       f(sc.lin_vel_offset), f(sc.ang_vel))
    r = np.random.default_rng(9)
    gm, gq, gv = (f(r.normal(size=s_)) for s_ in ((g.n, 3), (g.n, 4), (g.n, 3)))
    dm, dq, dv = torch.zeros_like(mu), torch.zeros_like(q), torch.zeros_like(v)
    da = {k: torch.zeros_like(getattr(A, k)) for k in B.ACTOR_GRAD_FIELDS}
    ws = torch.empty(int(B.load().splat_compose_workspace_bytes(A.n)), dtype=torch.uint8, device=dev)
    for _ in range(args.warmup):
        mw, qw, vw = B.compose(mu, q, aid, A, v)
        B.compose_bwd(mu, q, aid, A, gm, gq, gv, dm, dq, dv, da, ws)
    stream = torch.cuda.current_stream()
    mk = lambda: torch.cuda.Event(enable_timing=True)
    ev = [(mk(), mk(), mk()) for _ in range(args.steps)]
    torch.cuda.synchronize()
    for e0, e1, e2 in ev:
        e0.record(stream)
        mw, qw, vw = B.compose(mu, q, aid, A, v)
        e1.record(stream)
        B.compose_bwd(mu, q, aid, A, gm, gq, gv, dm, dq, dv, da, ws)
        e2.record(stream)
    torch.cuda.synchronize()
    t_f = float(np.median([a.elapsed_time(b) for a, b, _ in ev])) * 1e-3
    t_b = float(np.median([b.elapsed_time(c) for _, b, c in ev])) * 1e-3
    n, n_static = g.n, int((sc.actor_id < 0).sum())
    bytes_f = n * (12 + 16 + 4 + 12 + 16 + 12) + n_static * 12
    bytes_b = n * (12 + 16 + 12 + 4 + 12 + 16 + 24 + 32) + n_static * 24
    # sampled parity of the world arrays against the oracle
    idx = np.sort(np.random.default_rng(3).choice(n, 4096, replace=False))
    t = lambda a: torch.from_numpy(np.asarray(a, np.float64))
    sub_id = sc.actor_id[idx]
    ref = oc.compose(t(g.means[idx]), t(g.quats[idx]), sub_id, t(sc.rot), t(sc.trans), t(sc.rot_offset),
                     t(sc.trans_offset), t(sc.lin_vel), t(sc.lin_vel_offset), t(sc.ang_vel), t(g.velocities[idx]))
    worst = 0.0
    for got, want in zip((mw, qw, vw), ref):
        a_ = got[torch.from_numpy(idx).to(dev)].double().cpu().numpy()
        w_ = want.numpy()
        worst = max(worst, float((np.abs(a_ - w_) / (1e-5 + 1e-4 * np.abs(w_))).max()))
    ach_f, ach_b = bytes_f / t_f / 1e9, bytes_b / t_b / 1e9
    log(f"compose: fwd {t_f * 1e3:.4f} ms ({ach_f:.0f} GB/s), bwd {t_b * 1e3:.4f} ms ({ach_b:.0f} GB/s)")
    return {"workload": "2M Gaussians, 30 % in 64 rigid actors (cars), world means / rotations / velocities",
            "fwd_ms": round(t_f * 1e3, 4), "bwd_ms": round(t_b * 1e3, 4),
            "roofline": {"bound": "hbm", "unit": "GB/s", "peak": PEAK_HBM_GBS,
                         "fwd": {"achieved": round(ach_f, 1), "frac": round(ach_f / PEAK_HBM_GBS, 4),
                                 "bytes_per_launch": int(bytes_f)},
                         "bwd": {"achieved": round(ach_b, 1), "frac": round(ach_b / PEAK_HBM_GBS, 4),
                                 "bytes_per_launch": int(bytes_b)}},
            "parity": {"gaussians": 4096, "max_err_over_tol": round(worst, 4), "pass": bool(worst <= 1.0)}}


def points_bench(args, dev, lid):
    """Lidar points to rasterisation rays (splat_lidar_points_to_rays) for one 128 x 2048 sweep and
    for 64 sweeps in one launch, timed with HIP events around each call on the launching stream,
    against the HBM roofline (28 B per point: point and time read, azimuth, elevation and range
    written once)."""
    import torch
    from oracle import points as op
    from paper_2411_16816_amd import binding as B
    from scenes import synthetic as S
    out = {"workload": "ego-motion-compensated world points of a 128 x 2048 sweep (100 ms, 15 m/s) -> "
                       "azimuth / elevation / measured range", "bytes_per_point": 28, "sizes": {}}
    stream = torch.cuda.current_stream()
    mk = lambda: torch.cuda.Event(enable_timing=True)
    worst = 0.0
    for label, n in (("one_sweep", lid.n_rays), ("64_sweeps", 64 * lid.n_rays)):
        pts, t = S.lidar_points(SEED_POINTS, n)
        P, T = torch.from_numpy(pts).to(dev), torch.from_numpy(t).to(dev)
        o = tuple(torch.empty(n, dtype=torch.float32, device=dev) for _ in range(3))
        for _ in range(max(1, args.warmup)):
            B.points_to_rays(P, T, lid.R, lid.t, lid.lin_vel, lid.ang_vel, out=o)
        ev = [(mk(), mk()) for _ in range(args.steps)]
        torch.cuda.synchronize()
        for e0, e1 in ev:
            e0.record(stream)
            B.points_to_rays(P, T, lid.R, lid.t, lid.lin_vel, lid.ang_vel, out=o)
            e1.record(stream)
        torch.cuda.synchronize()
        sec = float(np.median([a.elapsed_time(b) for a, b in ev])) * 1e-3
        ach = 28.0 * n / sec / 1e9
        idx = np.sort(np.random.default_rng(5).choice(n, 4096, replace=False))
        ref = op.points_to_rays(pts[idx], t[idx], lid.R, lid.t, lid.lin_vel, lid.ang_vel)
        ii = torch.from_numpy(idx).to(dev)
        for k, (got, want) in enumerate(zip(o, ref)):
            a_ = got[ii].double().cpu().numpy()
            d = np.abs(((a_ - want + np.pi) % (2 * np.pi)) - np.pi) if k == 0 else np.abs(a_ - want)
            worst = max(worst, float((d / (1e-5 + 1e-4 * np.abs(want))).max()))
        out["sizes"][label] = {"points": n, "ms": round(sec * 1e3, 4), "achieved_GBs": round(ach, 1),
                               "frac": round(ach / PEAK_HBM_GBS, 4)}
        log(f"points_to_rays {label}: {n} points, {sec * 1e3:.4f} ms ({ach:.0f} GB/s)")
        del P, T, o
    out["roofline"] = {"bound": "hbm", "unit": "GB/s", "peak": PEAK_HBM_GBS}
    out["parity"] = {"points": 2 * 4096, "max_err_over_tol": round(worst, 4), "pass": bool(worst <= 1.0)}
    return out


def mcmc_bench(args, dev, G, g):
    """MCMC regulariser (splat_mcmc_regularizer) over the step's 2M Gaussians: value and
    opacity / log-scale gradients, timed with HIP events around each call on the launching
    stream, against the HBM roofline (48 B per Gaussian: opacity and log-scales read, their
    gradients read and written)."""
    import torch
    from oracle import mcmc
    from paper_2411_16816_amd import binding as B
    val = torch.zeros(1, device=dev)
    gr = B.zeros_like_grads(G)
    for _ in range(max(1, args.warmup)):
        B.mcmc_regularizer(G, val, gr)
    stream = torch.cuda.current_stream()
    mk = lambda: torch.cuda.Event(enable_timing=True)
    ev = [(mk(), mk()) for _ in range(args.steps)]
    val.zero_()
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record(stream)
        B.mcmc_regularizer(G, val, gr)
        e1.record(stream)
    torch.cuda.synchronize()
    sec = float(np.median([a.elapsed_time(b_) for a, b_ in ev])) * 1e-3
    ach = 48.0 * g.n / sec / 1e9
    with torch.no_grad():
        L = float(mcmc.regulariser(g.opacities, g.log_scales, g.quats))
    err = abs(float(val) / args.steps - L) / L
    log(f"mcmc_regularizer: {g.n} Gaussians, {sec * 1e3:.4f} ms ({ach:.0f} GB/s), value rel err {err:.2e}")
    out = {"workload": f"{g.n} Gaussians of the step, value + opacity / log-scale gradients",
           "ms": round(sec * 1e3, 4), "bytes_per_gaussian": 48,
           "roofline": {"bound": "hbm", "unit": "GB/s", "peak": PEAK_HBM_GBS, "achieved": round(ach, 1),
                        "frac": round(ach / PEAK_HBM_GBS, 4)},
           "parity": {"value_rel_err": float(f"{err:.3g}"), "pass": bool(err <= 1e-4)}}
    # relocation: 10 % of the Gaussians dead; the arrays are restored before every call (outside
    # the timed events), since the call relocates in place
    rng = np.random.default_rng(SEED_RELOC)
    dead = rng.choice(g.n, g.n // 10, replace=False)
    o_dead = G.opacities.clone()
    o_dead[torch.from_numpy(dead).to(dev)] = torch.from_numpy(rng.uniform(0, 0.005, len(dead)).astype(np.float32)).to(dev)
    fields = ("means", "log_scales", "quats", "opacities", "velocities", "features")
    pristine = {f: getattr(G, f).clone() for f in fields if getattr(G, f) is not None and f != "opacities"}
    pristine["opacities"] = o_dead
    work = B.GaussTensors(*(pristine[f].clone() if f in pristine else None for f in fields))
    u = torch.from_numpy(rng.integers(0, 1 << 32, g.n, dtype=np.uint64).astype(np.uint32).view(np.int32)).to(dev)
    ws = torch.empty(int(B.load().splat_mcmc_relocate_workspace_bytes(g.n)), dtype=torch.uint8, device=dev)
    ev = [(mk(), mk()) for _ in range(args.steps)]
    for k in range(max(1, args.warmup) + args.steps):
        for f, t in pristine.items():
            getattr(work, f).copy_(t)
        if k >= max(1, args.warmup):
            ev[k - max(1, args.warmup)][0].record(stream)
        tgt, moved = B.mcmc_relocate(work, u, ws=ws)
        if k >= max(1, args.warmup):
            ev[k - max(1, args.warmup)][1].record(stream)
    torch.cuda.synchronize()
    sec_r = float(np.median([a.elapsed_time(b_) for a, b_ in ev])) * 1e-3
    log(f"mcmc_relocate: {g.n} Gaussians, {len(dead)} dead, {sec_r * 1e3:.4f} ms")
    out["relocate"] = {"workload": f"{g.n} Gaussians, {len(dead)} dead (opacity <= 0.005), copies capped at 51",
                       "ms": round(sec_r * 1e3, 4), "relocated": int(moved)}
    return out


def decoder_bench(args, dev, lid):
    """Lidar decoder (splat_lidar_decode / _bwd, 8 feature channels, hidden width 32) on one
    128 x 2048 sweep and on 64 sweeps in one launch, timed with HIP events around each call;
    forward against the HBM roofline (48 B per ray: feature row, angles, two outputs) and its
    FLOP (2 x (32 x 11 + 64) per ray) against the FP32 peak."""
    import torch
    from oracle import decoders as dec
    from paper_2411_16816_amd import binding as B
    rng = np.random.default_rng(SEED_DECODER)
    C = 8
    W = [rng.normal(0, 0.5, (32, C + 3)), rng.normal(0, 0.2, 32), rng.normal(0, 0.5, (2, 32)), rng.normal(0, 0.2, 2)]
    W = [w.astype(np.float32) for w in W]
    mlp = B.LidarMLP(*(torch.from_numpy(w).to(dev) for w in W))
    stream = torch.cuda.current_stream()
    mk = lambda: torch.cuda.Event(enable_timing=True)
    out = {"workload": "lidar decoder, 8 feature channels + ray direction -> intensity, ray drop (hidden 32)",
           "bytes_per_ray_fwd": 48, "flop_per_ray_fwd": 2 * (32 * (C + 3) + 64), "sizes": {}}
    worst = 0.0
    for label, reps in (("one_sweep", 1), ("64_sweeps", 64)):
        n = lid.n_rays * reps
        F = torch.from_numpy(rng.normal(size=(n, C)).astype(np.float32)).to(dev)
        az = torch.from_numpy(np.tile(lid.ray_az.astype(np.float32), reps)).to(dev)
        el = torch.from_numpy(np.tile(lid.ray_el.astype(np.float32), reps)).to(dev)
        dI = torch.from_numpy(rng.normal(size=n).astype(np.float32)).to(dev)
        dP = torch.from_numpy(rng.normal(size=n).astype(np.float32)).to(dev)
        dF = torch.zeros_like(F)
        dm = {f: torch.zeros_like(getattr(mlp, f)) for f in B.MLP_FIELDS}
        ws = torch.empty(int(B.load().splat_lidar_decode_workspace_bytes(n, C)), dtype=torch.uint8, device=dev)
        for _ in range(max(1, args.warmup)):
            I, P = B.lidar_decode(F, az, el, mlp)
            B.lidar_decode_bwd(F, az, el, mlp, dI, dP, dF, dm, ws)
        ev = [(mk(), mk(), mk()) for _ in range(args.steps)]
        torch.cuda.synchronize()
        for e0, e1, e2 in ev:
            e0.record(stream)
            I, P = B.lidar_decode(F, az, el, mlp)
            e1.record(stream)
            B.lidar_decode_bwd(F, az, el, mlp, dI, dP, dF, dm, ws)
            e2.record(stream)
        torch.cuda.synchronize()
        t_f = float(np.median([a.elapsed_time(b_) for a, b_, _ in ev])) * 1e-3
        t_b = float(np.median([b_.elapsed_time(c) for _, b_, c in ev])) * 1e-3
        idx = np.sort(np.random.default_rng(5).choice(n, 4096, replace=False))
        ii = torch.from_numpy(idx).to(dev)
        with torch.no_grad():
            rI, rP = dec.lidar_mlp(F[ii].double().cpu(), az[ii].cpu().numpy(), el[ii].cpu().numpy(), *W)
        for got, want in ((I[ii], rI), (P[ii], rP)):
            a_, w_ = got.double().cpu().numpy(), want.numpy()
            worst = max(worst, float((np.abs(a_ - w_) / (1e-5 + 1e-4 * np.abs(w_))).max()))
        gbs = 48.0 * n / t_f / 1e9
        out["sizes"][label] = {"rays": n, "fwd_ms": round(t_f * 1e3, 4), "bwd_ms": round(t_b * 1e3, 4),
                               "fwd_GBs": round(gbs, 1), "fwd_hbm_frac": round(gbs / PEAK_HBM_GBS, 4),
                               "fwd_TFLOPs": round(out["flop_per_ray_fwd"] * n / t_f / 1e12, 2)}
        log(f"lidar decoder {label}: {n} rays, fwd {t_f * 1e3:.4f} ms ({gbs:.0f} GB/s), bwd {t_b * 1e3:.4f} ms")
        del F, az, el, dI, dP, dF, ws
    out["roofline"] = {"bound": "hbm", "unit": "GB/s", "peak": PEAK_HBM_GBS}
    out["parity"] = {"rays": 2 * 4096, "max_err_over_tol": round(worst, 4), "pass": bool(worst <= 1.0)}
    return out


def cnn_bench(args, dev, cam):
    """Camera decoder (splat_camera_decode / _bwd) on the 1920 x 1080 camera, 16 feature channels
    + direction + 8-float embedding, timed with HIP events around each call.  Algorithmic FLOP:
    the five 3x3 convolutions (2 x 9 x C_in x 32 per pixel each, C_in = 27 for the stem) and the
    1x1 head; the adjoint counts the input- and weight-gradient convolutions (twice the forward)
    plus the head.  Against the FP32 matrix-core peak."""
    import torch
    from oracle import decoders as dec
    from paper_2411_16816_amd import binding as B
    rng = np.random.default_rng(SEED_CNN)
    Df, E = cam.n_channels, 8
    cin = Df + 3 + E
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    Wn = {"embed": rng.normal(0, 1, E), "w_in": rng.normal(0, np.sqrt(2 / (9 * cin)), (32, cin, 3, 3)),
          "b_in": rng.normal(0, 0.05, 32), "w_block": [rng.normal(0, 0.5 * np.sqrt(2 / 288), (32, 32, 3, 3)) for _ in range(4)],
          "b_block": [rng.normal(0, 0.05, 32) for _ in range(4)], "w_out": rng.normal(0, np.sqrt(1 / 32), (6, 32)),
          "b_out": rng.normal(0, 0.1, 6)}
    cnn = B.CameraCNN(d(Wn["embed"]), d(Wn["w_in"]), d(Wn["b_in"]), [d(w) for w in Wn["w_block"]],
                      [d(x) for x in Wn["b_block"]], d(Wn["w_out"]), d(Wn["b_out"]))
    H, W = cam.height, cam.width
    n = H * W
    F = d(rng.normal(size=n * Df))
    dI = d(rng.normal(size=n * 3))
    dF = torch.zeros_like(F)
    dc = {"embed": torch.zeros_like(cnn.embed), "w_in": torch.zeros_like(cnn.w_in), "b_in": torch.zeros_like(cnn.b_in),
          "w_block": [torch.zeros_like(x) for x in cnn.w_block], "b_block": [torch.zeros_like(x) for x in cnn.b_block],
          "w_out": torch.zeros_like(cnn.w_out), "b_out": torch.zeros_like(cnn.b_out)}
    ws = B.camera_decode_workspace(cam, dev)
    for _ in range(max(1, args.warmup)):
        I = B.camera_decode(cam, F, cnn, ws)
        B.camera_decode_bwd(cam, F, cnn, dI, dF, dc, ws)
    stream = torch.cuda.current_stream()
    mk = lambda: torch.cuda.Event(enable_timing=True)
    ev = [(mk(), mk(), mk()) for _ in range(args.steps)]
    torch.cuda.synchronize()
    for e0, e1, e2 in ev:
        e0.record(stream)
        I = B.camera_decode(cam, F, cnn, ws)
        e1.record(stream)
        B.camera_decode_bwd(cam, F, cnn, dI, dF, dc, ws)
        e2.record(stream)
    torch.cuda.synchronize()
    t_f = float(np.median([a.elapsed_time(b_) for a, b_, _ in ev])) * 1e-3
    t_b = float(np.median([b_.elapsed_time(c) for _, b_, c in ev])) * 1e-3
    conv_px = 2 * 9 * cin * 32 + 4 * 2 * 9 * 32 * 32
    flop_f = n * (conv_px + 2 * 6 * 32 + 3 * 2)
    flop_b = n * (2 * conv_px + 2 * 2 * 6 * 32)
    # parity: a 24 x 24 crop (5-pixel margin: the receptive field) against the FP64 oracle
    import dataclasses
    x0, y0, m = 700, 500, 5
    Fh = F.view(H, W, Df)[y0 - m:y0 + 24 + m, x0 - m:x0 + 24 + m].double().cpu()
    sub = dataclasses.replace(cam, width=34, height=34, cx=cam.cx - (x0 - m), cy=cam.cy - (y0 - m))
    with torch.no_grad():
        ref = dec.camera_cnn(Fh, sub, Wn["embed"].astype(np.float32), Wn["w_in"].astype(np.float32),
                             Wn["b_in"].astype(np.float32), [w.astype(np.float32) for w in Wn["w_block"]],
                             [x.astype(np.float32) for x in Wn["b_block"]], Wn["w_out"].astype(np.float32),
                             Wn["b_out"].astype(np.float32))[m:m + 24, m:m + 24].numpy()
    got = I.view(H, W, 3)[y0:y0 + 24, x0:x0 + 24].double().cpu().numpy()
    worst = float((np.abs(got - ref) / (1e-5 + 1e-4 * np.abs(ref))).max())
    tf, tb = flop_f / t_f / 1e12, flop_b / t_b / 1e12
    log(f"camera decoder 1080p: fwd {t_f * 1e3:.3f} ms ({tf:.1f} TFLOP/s), bwd {t_b * 1e3:.3f} ms ({tb:.1f} TFLOP/s)")
    return {"workload": f"camera decoder on {W}x{H}: {Df} feature channels + direction + {E}-float embedding, "
                        "3x3 stem, two residual blocks of width 32, 1x1 head",
            "fwd_ms": round(t_f * 1e3, 4), "bwd_ms": round(t_b * 1e3, 4),
            "roofline": {"bound": "mfma", "unit": "TFLOP/s", "peak": PEAK_FP32_TFLOPS,
                         "fwd": {"achieved": round(tf, 2), "frac": round(tf / PEAK_FP32_TFLOPS, 4), "flop": int(flop_f)},
                         "bwd": {"achieved": round(tb, 2), "frac": round(tb / PEAK_FP32_TFLOPS, 4), "flop": int(flop_b)}},
            "parity": {"pixels": 576, "max_err_over_tol": round(worst, 4), "pass": bool(worst <= 1.0)}}


# ---- CPU baseline: the FP64 oracle on the host's cores ----------------------------------------
_ORC = {}
MAX_ORACLE_WORKERS = 15


def _oracle_init(n_gauss, barrier):
    """Pool worker set-up: the seeded scene and its FP64 projections (one thread per worker)."""
    import torch
    from oracle import geometry as og
    from scenes import synthetic as S
    torch.set_num_threads(1)
    t0 = time.perf_counter()
    sc = S.headline(n=n_gauss)
    p = og.Params.from_gaussians(sc.gaussians)
    for k, sensor in enumerate((sc.cameras[0], sc.lidars[0])):
        _ORC[k] = (sensor, og.project(p, sensor), p.features)
    _ORC["setup_s"] = time.perf_counter() - t0
    _ORC["barrier"] = barrier


def _oracle_ready(_):
    _ORC["barrier"].wait(timeout=600)   # every worker has finished its set-up
    return _ORC["setup_s"]


def _oracle_task(args):
    """Render (and differentiate) one chunk of rays against every Gaussian; returns seconds."""
    import dataclasses
    import torch
    from oracle import grad as ogr
    from oracle import render as rd
    k, ray_idx, with_grad, seed = args
    sensor, proj, feats = _ORC[k]
    rays = rd.lidar_rays(sensor, ray_idx) if k == 1 else rd.camera_rays(sensor, ray_idx)
    t0 = time.perf_counter()
    if with_grad:
        # gradients with respect to the projected records and the features: the adjoint of the
        # compositing per ray (the projection adjoint is a per-Gaussian cost, like the projection)
        leaves = {f.name: getattr(proj, f.name).detach().clone().requires_grad_(True)
                  for f in dataclasses.fields(proj)
                  if isinstance(getattr(proj, f.name), torch.Tensor) and getattr(proj, f.name).is_floating_point()}
        pl = dataclasses.replace(proj, **leaves)
        fl = feats.detach().clone().requires_grad_(True)
        out = rd.render(pl, sensor, fl, rays)
        r = np.random.default_rng(seed)
        n, C = len(ray_idx), sensor.n_channels
        t = lambda a: torch.from_numpy(a)
        loss = ogr.weighted_loss(out, t(r.normal(size=(n, C))), t(r.normal(size=n)), t(r.normal(size=n)),
                                 t(r.normal(size=n)) if k == 1 else None)
        loss.backward()
    else:
        with torch.no_grad():
            rd.render(proj, sensor, feats, rays)
    return time.perf_counter() - t0


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, cam, lid, n_cam_rays, n_lid_rays):
    """The FP64 oracle (brute force over every Gaussian per ray) on the host's cores: a pool of
    single-threaded worker processes, one per core of this process's CPU share, each holding
    the seeded scene and its FP64 projections.  A seeded sample of camera pixels and lidar rays is
    rendered forward only and then forward + backward (the compositing adjoint, down to the
    projected records and the features); each sensor's wall-clock rate over the pool is combined
    with the workload's mix of pixels and lidar rays into rays per second of a whole step.  The
    per-Gaussian work (scene set-up, projection and its adjoint) is a fixed cost per step and is
    reported, not included."""
    import multiprocessing as mp
    cores = len(os.sched_getaffinity(0))
    share = os.environ.get("OMP_NUM_THREADS")
    if share and share.isdigit() and int(share) > 0:
        cores = min(cores, int(share))
    # this process holds the GPU; the workers get none (hidden before they start), and with
    # this process they stay within 16 processes even if a worker opened the device
    cores = max(1, min(cores, MAX_ORACLE_WORKERS))
    rng = np.random.default_rng(11)
    samples = {0: np.sort(rng.choice(cam.n_rays, size=n_cam_rays, replace=False)),
               1: np.sort(rng.choice(lid.n_rays, size=n_lid_rays, replace=False))}
    per_task = {0: 8, 1: 2}
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(cores)
    rates = {}
    hidden = ("HIP_VISIBLE_DEVICES", "ROCR_VISIBLE_DEVICES", "CUDA_VISIBLE_DEVICES")
    saved = {k: os.environ.get(k) for k in hidden}
    for k in hidden:
        os.environ[k] = ""
    try:
        pool = ctx.Pool(cores, initializer=_oracle_init, initargs=(g.n, barrier))
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    with pool:
        setup = pool.map_async(_oracle_ready, range(cores), chunksize=1).get(timeout=900)
        for with_grad in (False, True):
            for k in (0, 1):
                idx = samples[k]
                tasks = [(k, idx[i:i + per_task[k]], with_grad, 100 + i) for i in range(0, len(idx), per_task[k])]
                t0 = time.perf_counter()
                pool.map_async(_oracle_task, tasks, chunksize=1).get(timeout=900)
                rates[(k, with_grad)] = len(idx) / (time.perf_counter() - t0)
    n_rays = {0: cam.n_rays, 1: lid.n_rays}
    step_s = lambda wg: sum(n_rays[k] / rates[(k, wg)] for k in (0, 1))
    total = cam.n_rays + lid.n_rays
    fb = total / step_s(True) / 1e6
    fwd = total / step_s(False) / 1e6
    return {"value": round(fb, 8), "unit": "Mrays/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_cam_rays} camera pixels + {n_lid_rays} lidar rays of the workload, FP64 brute force, "
                      f"{cores} single-threaded worker processes; rates per sensor weighted by the step's "
                      f"{cam.n_rays} pixels and {lid.n_rays} lidar rays; per-Gaussian set-up and projection "
                      f"({max(setup):.1f} s per worker) not included",
            "forward_only": round(fwd, 8),
            "per_sensor_rays_per_s": {"camera_fwd": round(rates[(0, False)], 3), "lidar_fwd": round(rates[(1, False)], 3),
                                      "camera_fwd_bwd": round(rates[(0, True)], 3),
                                      "lidar_fwd_bwd": round(rates[(1, True)], 3)},
            "cpu_model": _cpu_model()}


if __name__ == "__main__":
    main()
