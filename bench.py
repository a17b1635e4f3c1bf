#!/usr/bin/env python3
"""Benchmark: 1080p photon-field ray-marched frames on one MI355X.

Workload (config "field inference render"): 512^3 float16 synthetic volume (64 blobs, 4 octaves),
3 point lights, photon cache traced from 2^22 photons into 128^3 x 5 HG bins, field trained with
the photon-cache recipe (16 levels x 2 features, base 16, growth 1.5, 2^19 table, 3 x 64 ReLU
MLP, batch 2^18, 2000 steps, L2), rendered at 1920x1080, 1 spp, step 0.5 voxel, <= 1024 steps,
transmittance cut-off 1e-3, field every 4 steps, FP16 matrix-core MLP, light-transmittance volume.

A step is one full frame of the hot path (ray generation, density, transfer function,
transmittance, direct light, field queries, compositing).  Scene set-up, tracing and training
happen before the timed region (their times are reported separately).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel):
    """Calibrated FETCH_SIZE + WRITE_SIZE bytes per frame of `kernel` (all its launches of one
    frame), taken from the committed counter summaries, or None when there is none for it or the
    kernel sources have changed since."""
    import glob
    import hashlib
    rec = None
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_hbm_traffic.md"))):
        with open(path) as f:
            for l in f:
                if l.startswith("traffic-record:"):
                    r = json.loads(l.split(":", 1)[1])
                    if r["kernel"].split("<")[0] == kernel:
                        rec = r
    if rec is None:
        return None
    h = hashlib.sha256()
    for name in rec["sources"]:
        with open(os.path.join(ROOT, "paper_2304_07338_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return int(rec["fetch_bytes"]) + int(rec["write_bytes"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="smaller training (setup only)")
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--precision", default="f16", choices=["f16", "bf16", "f32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=80, help="lattice side of the oracle sample")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 64-job launch")
    ap.add_argument("--no-first-interaction", action="store_true",
                    help="skip the Algorithm 2 renderer timings")
    ap.add_argument("--no-photon-map", action="store_true",
                    help="skip the photon-map (Eq. 5) training timings")
    ap.add_argument("--pm-radius", type=float, default=0.08,
                    help="final KNN query radius of the photon-map schedule (cube units)")
    ap.add_argument("--pm-grid", type=int, default=64)
    ap.add_argument("--pm-steps", type=int, default=10)
    ap.add_argument("--strategy", default="auto", choices=["auto", "fused", "wavefront", "wavefront_serial"],
                    help="form of the field-lit render")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the precision / spp / g / direct-light variants of the frame")
    ap.add_argument("--no-matched", action="store_true",
                    help="skip the matched-RMSE comparison with the path tracer on the frame")
    ap.add_argument("--mr2-ref-spp", type=int, default=1024,
                    help="reference spp of the matched-RMSE comparison on the benchmark frame")
    ap.add_argument("--matched-rmse", action="store_true",
                    help="run the large-scale comparison with the path tracer instead")
    ap.add_argument("--mr-n", type=int, default=1024, help="volume side of the comparison")
    ap.add_argument("--mr-width", type=int, default=1920)
    ap.add_argument("--mr-height", type=int, default=1080)
    ap.add_argument("--mr-ref-spp", type=int, default=4096)
    ap.add_argument("--mr-photons", type=int, default=24, help="log2 photons per re-trace")
    ap.add_argument("--studies", action="store_true",
                    help="run the phase-awareness and noise studies instead")
    ap.add_argument("--st-photons", type=int, default=22, help="log2 photons per study trace")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the renderer runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding over several GPUs is described, not implemented)", file=sys.stderr)
        sys.exit(2)

    if args.matched_rmse:
        print(json.dumps(matched_rmse(args)), flush=True)
        return
    if args.studies:
        print(json.dumps(studies(args)), flush=True)
        return

    import numpy as np
    import torch

    from paper_2304_07338_amd import scenegen as sg
    from paper_2304_07338_amd import workloads as wl
    from paper_2304_07338_amd.pfn import (Context, FieldConfig, PfnError, RenderConfig,
                                          TrainConfig, DIRECT_LIGHT_VOLUME, INDIRECT_CACHE,
                                          INDIRECT_FIELD)
    from paper_2304_07338_amd import _ffi

    w = wl.C2
    dev = "cuda:0"
    t0 = time.time()
    vol, tf, lights = wl.make_scene(w, device=dev)
    la = sg.lights_array(lights)
    torch.cuda.synchronize()
    log(f"[setup] volume {w.n}^3 {w.vol_dtype} generated in {time.time() - t0:.1f}s")
    ctx = Context(0)
    ctx.set_render_strategy(args.strategy)
    ctx.set_volume(vol.contiguous())
    ctx.set_transfer_function(tf, w.extinction)
    ctx.set_lights(la)
    t1 = time.time()
    ctx.build_light_volume(0.5)
    ctx.sync()
    lv_s = time.time() - t1
    log(f"[setup] light volume built in {lv_s:.2f}s")

    n_photons = 1 << 22
    ctx.timing_enable(True)
    t1 = time.time()
    st = ctx.trace_photon_cache(n_photons, wl.C1_G_BINS, cache_res=128, seed=6,
                                max_collisions=8, rr_start=3)
    trace_s = time.time() - t1
    trace_ms, _ = ctx.timing_get(_ffi.TK_TRACE)
    log(f"[setup] traced {n_photons} photons ({st['n_records']} records) in {trace_s:.2f}s "
        f"(kernel {trace_ms:.1f} ms), kappa {st['kappa']:.4g}")

    fcfg = FieldConfig()
    ctx.field_select(0)
    ctx.field_init(fcfg, seed=1)
    train_info = {"trained": False}
    try:
        tcfg = TrainConfig(steps=200 if args.quick else args.train_steps, log2_batch=18,
                           precision="f16", seed=7)
        ctx.sync()
        t1 = time.time()
        hist = ctx.train_field(tcfg)
        train_s = time.time() - t1
        train_info = {"trained": True, "steps": tcfg.steps, "batch": 1 << tcfg.log2_batch,
                      "seconds": round(train_s, 3), "steps_per_s": round(tcfg.steps / train_s, 1),
                      "final_loss": float(np.mean(hist[-20:]))}
        log(f"[setup] trained {tcfg.steps} steps in {train_s:.2f}s, loss {hist[0]:.4g} -> "
            f"{train_info['final_loss']:.4g}")
    except PfnError as e:
        log(f"[setup] training unavailable ({e}); the field keeps its initial parameters")

    cam = wl.camera(w, 0)
    rc = RenderConfig(spp=1, step_voxels=0.5, max_steps=1024, t_min=1e-3, field_stride=4, g=0.4,
                      indirect=INDIRECT_FIELD, direct=DIRECT_LIGHT_VOLUME,
                      field_precision=args.precision, field_slot=0)
    out = torch.empty((w.height, w.width, 3), dtype=torch.float32, device=dev)

    # counting pass (not timed): march steps and field queries of this frame
    ctx.count_enable(True)
    ctx.render_frame(cam, rc, out)
    steps_f, queries_f = ctx.count_get()
    ctx.count_enable(False)
    log(f"[setup] frame: {steps_f} march steps, {queries_f} field queries")
    # the library's autotuner picks the render form and ray-tile shape for this frame (not timed)
    tuned = ctx.autotune_batch([cam], [rc], [out], iters=2)
    log(f"[setup] autotuned frame: {tuned}")

    for _ in range(args.warmup):
        ctx.render_frame(cam, rc, out)
    torch.cuda.synchronize()
    ctx.timing_reset()
    ctx.timing_enable(True)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(args.steps):
        ctx.render_frame(cam, rc, out)
    torch.cuda.synchronize()
    te = time.perf_counter()
    march_ms, launches = ctx.timing_get(_ffi.TK_MARCH)
    ktimes = {k: ctx.timing_get(i) for k, i in (("wf_march_kernel", _ffi.TK_WF_MARCH),
                                                 ("wf_encode_kernel", _ffi.TK_WF_ENCODE),
                                                 ("wf_dir_kernel", _ffi.TK_WF_DIR),
                                                 ("wf_field_kernel", _ffi.TK_WF_FIELD),
                                                 ("wf_resolve_kernel", _ffi.TK_WF_RESOLVE))}
    ctx.timing_enable(False)
    ms_per_step = (te - ts) * 1000.0 / args.steps
    frame_ms = march_ms / max(launches, 1)
    fps = 1000.0 / ms_per_step
    img_mean = float(out.mean())

    # algorithmic bytes of one frame: per step 8 density corners + 8 light-volume texels
    # (4 x f16); per field query 16 levels x (8 + 4) corners x 2 features
    vbytes = 2 if w.vol_dtype == "f16" else 4
    feat_bytes = {"f16": 4, "bf16": 4, "f32": 8}[args.precision]
    step_bytes = 8 * vbytes + 8 * 8
    bytes_frame = steps_f * step_bytes + queries_f * 16 * 12 * feat_bytes
    mlp_flop = 2 * (65 * 64 + 64 * 64 * 2 + 64 * 3)  # 3 hidden layers of 64, FLOP per query
    kernels = {}
    if ktimes["wf_march_kernel"][1] > 0:
        # wavefront form: per kernel, per frame
        # the position encoding reads a query's 16 x 8 grid corners and its position once and
        # writes its 16 features (the XCDs that read the position again add no algorithmic
        # bytes); the direction encoding reads 16 x 4 corners and writes 16 features per ray
        # of a round
        per = {"wf_march_kernel": (steps_f * step_bytes + queries_f * 24, 0),
               "wf_encode_kernel": (queries_f * (16 * 8 * feat_bytes + 16 * feat_bytes + 12), 0),
               "wf_dir_kernel": (None, 0),  # per ray of a round; rays per round not counted
               "wf_field_kernel": (queries_f * (16 * feat_bytes + 12), queries_f * mlp_flop),
               "wf_resolve_kernel": (0, 0)}
        for k, (ms, n) in ktimes.items():
            kms = ms / args.steps
            b, fl = per[k]
            kernels[k] = {"ms_per_frame": round(kms, 4), "launches_per_frame": n / args.steps,
                          "algorithmic_bytes_per_frame": None if b is None else int(b),
                          "GB_s": round(b / (kms * 1e-3) / 1e9, 2)
                          if b is not None and kms > 0 else None}
            if fl:
                kernels[k]["TFLOP_s"] = round(fl / (kms * 1e-3) / 1e12, 3)
        dom = max((k for k in kernels if k not in ("wf_resolve_kernel", "wf_dir_kernel")),
                  key=lambda k: kernels[k]["ms_per_frame"])
        dom_bytes = kernels[dom]["algorithmic_bytes_per_frame"]
        dom_ms = kernels[dom]["ms_per_frame"]
    else:
        dom, dom_bytes, dom_ms = "march_kernel", bytes_frame, frame_ms
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9

    # plain cache gather render of the same frame (no network)
    rc_cache = RenderConfig(**{**rc.__dict__, "indirect": INDIRECT_CACHE})
    tuned_cache = ctx.autotune_batch([cam], [rc_cache], [out], iters=2)
    for _ in range(2):
        ctx.render_frame(cam, rc_cache, out)
    torch.cuda.synchronize()
    tc0 = time.perf_counter()
    n_cache = max(3, args.steps // 2)
    for _ in range(n_cache):
        ctx.render_frame(cam, rc_cache, out)
    torch.cuda.synchronize()
    cache_ms = (time.perf_counter() - tc0) * 1000.0 / n_cache
    ctx.autotune_batch([cam], [rc], [out], iters=2)  # the field frame's form and tile again

    fi_info = None if args.no_first_interaction else first_interaction_bench(ctx, cam, rc, args)
    variants = None if args.no_variants else frame_variants(ctx, cam, rc, out, args)
    matched = None if args.no_matched else matched_rmse_frame(ctx, cam, rc, out, ms_per_step,
                                                              cache_ms, args)

    result = {
        "metric": "1080p fps + field queries/s: photon field vs path tracer at matched RMSE",
        "value": round(fps, 3),
        "unit": "fps",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f16": "f16-mfma/f32", "bf16": "bf16-mfma/f32", "f32": "f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": w.name, "volume": f"{w.n}^3 {w.vol_dtype}", "resolution": "1920x1080",
                   "spp": 1, "field_stride": 4, "max_steps": 1024, "t_min": 1e-3,
                   "direct": "light_volume", "photons": n_photons, "cache": "128^3 x 5 bins",
                   "field": "16 lv x 2 feat, T=2^19, 3x64 MLP", "g": 0.4},
        "field_queries_per_s": round(queries_f * fps, 1),
        "field_queries_per_frame": int(queries_f),
        "march_steps_per_frame": int(steps_f),
        "cache_gather_fps": round(1000.0 / cache_ms, 3),
        "cache_gather_autotuned": {k: tuned_cache[k] for k in ("strategy", "tile_w", "block_w",
                                                              "block_h", "persistent")},
        "roofline": roofline_entry(dom, dom_bytes, dom_ms, achieved, args),
        "frame": {"autotuned": {k: tuned[k] for k in ("strategy", "tile_w", "block_w",
                                                       "block_h", "persistent")},
                  "gpu_ms": round(frame_ms, 4), "algorithmic_bytes": int(bytes_frame),
                  "GB_s": round(bytes_frame / (frame_ms * 1e-3) / 1e9, 2),
                  "strategy": "wavefront" if kernels else "fused", "kernels": kernels},
        "trace": {"photons": n_photons, "seconds": round(trace_s, 3),
                  "kernel_ms": round(trace_ms, 3),
                  "photons_per_s": round(n_photons / (trace_ms * 1e-3), 1) if trace_ms else None},
        "train": train_info,
        "image_mean": img_mean,
    }

    if matched is not None:
        result["matched_rmse"] = matched
    if variants is not None:
        result["variants"] = variants
    if fi_info is not None:
        result["first_interaction"] = fi_info
    if not args.no_photon_map:
        result["photon_map_training"] = photon_map_bench(ctx, args)
    if not args.no_batch:
        result["batch"] = batch_bench(args)

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args, w, vol, tf, la, ctx, cam, fcfg, rc)

    print(json.dumps(result), flush=True)
    ctx.close()


def address_record(kernel):
    """The address-path record of `kernel` from the committed counter summaries (texture
    addresser busy fraction with the kernel alone on the chip, and the probe's ceilings), or
    None when there is none or the kernel sources have changed since."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_counters.md"))):
        with open(path) as f:
            for l in f:
                if l.startswith("address-record:"):
                    r = json.loads(l.split(":", 1)[1])
                    if r["kernel"].split("<")[0] != kernel:
                        continue
                    h = hashlib.sha256()
                    for name in r["sources"]:
                        with open(os.path.join(ROOT, "paper_2304_07338_amd", "csrc", name), "rb") as g:
                            h.update(g.read())
                    return r if h.hexdigest() == r["sources_sha256"] else None
    return None


def roofline_entry(kernel, alg_bytes, kernel_ms, achieved, args):
    """Roofline row of the frame's dominant kernel: algorithmic bytes per frame over its
    event-timed duration per frame (it shares the chip with the other rounds' kernels), against
    8 TB/s; the calibrated HBM traffic of its launches and that traffic's rate; and its binding
    ceiling, the vector-memory address path, with the addresser's busy fraction measured by
    counters."""
    traffic = measured_traffic(kernel) if args.precision == "f16" else None
    r = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic, "kernel": kernel,
         "kernel_ms_per_frame": round(kernel_ms, 4), "algorithmic_bytes_per_frame": int(alg_bytes)}
    if traffic is not None:
        gbs = traffic / (kernel_ms * 1e-3) / 1e9
        r["traffic_GB_s"] = round(gbs, 1)
        r["traffic_frac"] = round(gbs / HBM_PEAK_GBS, 4)
    rec = address_record(kernel) if args.precision == "f16" else None
    if rec is not None:
        r["binding"] = {"ceiling": "vector-memory address path (one lane address per CU clock)",
                        "counter": "TA_TA_BUSY", "busy_frac": rec["ta_busy_frac"],
                        "probe_lanes_per_cu_clock": rec["address_ceiling_lanes_per_cu_clock"]}
    return r


def _timed_frames(ctx, cam, cfg, out, reps):
    import torch
    ctx.render_frame(cam, cfg, out)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(reps):
        ctx.render_frame(cam, cfg, out)
    torch.cuda.synchronize()
    return (time.perf_counter() - ts) * 1000.0 / reps


def frame_variants(ctx, cam, rc, out, args):
    """The benchmark frame with one setting changed at a time: the field's arithmetic (BF16
    matrix cores, FP32), samples per pixel (2, 4, 8), g between the trained bins (0.2), and the
    direct light from exact shadow rays instead of the light-transmittance volume (on a 256x256
    frame of the same view, where the shadow rays are affordable), with the relative RMSE
    between the two direct-light forms (the light volume's bias)."""
    import torch
    from paper_2304_07338_amd import scenegen as sg
    from paper_2304_07338_amd.pfn import RenderConfig, DIRECT_SHADOW_RAYS
    res = {"field_precision": {}, "spp": {}, "g": {}}
    reps = 5
    for prec in ("bf16", "f32"):
        ms = _timed_frames(ctx, cam, RenderConfig(**{**rc.__dict__, "field_precision": prec}),
                           out, reps)
        res["field_precision"][prec] = {"ms_per_frame": round(ms, 3), "fps": round(1000 / ms, 3)}
        log(f"[variants] field {prec}: {ms:.2f} ms")
    for spp in (2, 4, 8):
        ms = _timed_frames(ctx, cam, RenderConfig(**{**rc.__dict__, "spp": spp, "seed": 5}), out,
                           reps)
        res["spp"][str(spp)] = {"ms_per_frame": round(ms, 3), "fps": round(1000 / ms, 3)}
        log(f"[variants] {spp} spp: {ms:.2f} ms")
    ms = _timed_frames(ctx, cam, RenderConfig(**{**rc.__dict__, "g": 0.2}), out, reps)
    res["g"]["0.2"] = {"ms_per_frame": round(ms, 3), "fps": round(1000 / ms, 3)}
    log(f"[variants] g 0.2: {ms:.2f} ms")
    small = sg.Camera(cam.eye, cam.target, cam.up, cam.fov_y_deg, 256, 256)
    o_lv = torch.empty((256, 256, 3), dtype=torch.float32, device="cuda:0")
    o_sr = torch.empty_like(o_lv)
    ms_lv = _timed_frames(ctx, small, rc, o_lv, 3)
    ms_sr = _timed_frames(ctx, small, RenderConfig(**{**rc.__dict__, "direct": DIRECT_SHADOW_RAYS}),
                          o_sr, 3)
    e = ctx.image_error(o_lv, o_sr)
    res["direct_light_256x256"] = {"light_volume_ms": round(ms_lv, 3),
                                   "shadow_rays_ms": round(ms_sr, 3),
                                   "light_volume_rel_rmse_vs_shadow_rays": e[1],
                                   "light_volume_psnr_vs_shadow_rays": e[2]}
    log(f"[variants] 256x256 light volume {ms_lv:.2f} ms vs shadow rays {ms_sr:.2f} ms, "
        f"rel-RMSE {e[1]:.4g}")
    res["paper_encoding"] = paper_encoding_costs(ctx, cam, rc, out, reps)
    return res


def paper_encoding_costs(ctx, cam, rc, out, reps):
    """The paper's encoding and network (Section 3.4: 16 levels x 8 features, growth 2, table
    2^19, 5 hidden layers) in a field slot of its own: the benchmark frame lit by it, and
    training steps of the paper's recipe (batches of 2^16, relative L2, Section 3.5.1) beside
    steps of the configuration's recipe on the same field.  The march, query count and launch
    shapes do not depend on the parameter values, so the field is trained for the timing only."""
    import torch
    from paper_2304_07338_amd.pfn import FieldConfig, PfnError, RenderConfig, TrainConfig
    slot = (rc.field_slot + 1) % 8
    fc = FieldConfig(levels=16, feats_per_level=8, growth=2.0, log2_table=19, hidden_layers=5)
    ctx.field_select(slot)
    ctx.field_init(fc, seed=5)
    res = {"field": {"levels": 16, "feats_per_level": 8, "growth": 2.0, "log2_table": 19,
                     "hidden_layers": 5, "n_params": ctx.field_num_params()}}
    try:
        for name, tc in (("paper_recipe", TrainConfig(steps=100, log2_batch=16, loss="rel",
                                                      seed=5)),
                         ("batch_2p18_l2", TrainConfig(steps=50, log2_batch=18, seed=5))):
            ctx.train_field(TrainConfig(**{**tc.__dict__, "steps": 3}))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.train_field(tc)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1000.0 / tc.steps
            res[f"train_{name}"] = {"batch": 1 << tc.log2_batch, "loss": tc.loss,
                                    "ms_per_step": round(ms, 3)}
            log(f"[variants] paper encoding, training {name}: {ms:.3f} ms per step")
        try:
            ms = _timed_frames(ctx, cam, RenderConfig(**{**rc.__dict__, "field_slot": slot}),
                               out, reps)
            res["frame"] = {"ms_per_frame": round(ms, 3), "fps": round(1000 / ms, 3)}
            log(f"[variants] paper encoding frame: {ms:.2f} ms")
        except PfnError as e:  # the fused strategy renders 2-feature fields only
            res["frame"] = str(e)
    finally:
        ctx.field_select(rc.field_slot)
    return res


def matched_rmse_frame(ctx, cam, rc, out, field_ms, cache_ms, args):
    """The benchmark frame against the Monte Carlo path tracer at equal error (the comparison
    of Section 4.3.1, on this GPU): a path-traced reference of --mr2-ref-spp samples (8 bounces,
    HG sampling, Russian roulette from bounce 3), the field frame as timed (1 spp), the plain
    cache gather, and the path tracer at 16..256 spp.  The path tracer's squared error is fitted
    as c^2 (1/spp + 1/ref_spp), solved for the spp at which it equals the field's, and its time
    interpolated there; the speedup is that time over the field frame's.  Both frames' times
    are the ones measured in their autotuned forms (field_ms, cache_ms)."""
    import numpy as np
    import torch
    from paper_2304_07338_amd.pfn import RenderConfig, INDIRECT_CACHE
    g = rc.g
    chunk = min(256, args.mr2_ref_spp)
    n_chunks = max(1, args.mr2_ref_spp // chunk)
    ref = torch.zeros_like(out)
    part = torch.empty_like(out)
    for c in range(n_chunks):
        ctx.render_path_traced(cam, chunk, max_bounces=8, g=g, rr_start=3, seed=3000 + c,
                               out=part)
        ref += part
        torch.cuda.synchronize()
    ref /= n_chunks
    log(f"[matched] reference {n_chunks * chunk} spp done")
    ctx.render_frame(cam, rc, out)
    e_field = ctx.image_error(out, ref)
    ctx.render_frame(cam, RenderConfig(**{**rc.__dict__, "indirect": INDIRECT_CACHE}), out)
    e_cache = ctx.image_error(out, ref)
    pt_spp = [16, 32, 64, 128, 256]
    pts = []
    img = torch.empty_like(out)
    for spp in pt_spp:
        torch.cuda.synchronize()
        ts = time.perf_counter()
        ctx.render_path_traced(cam, spp, max_bounces=8, g=g, rr_start=3, seed=4000 + spp, out=img)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - ts) * 1000.0
        pts.append((spp, ms, ctx.image_error(img, ref)[0]))
        log(f"[matched] path tracer {spp} spp: {ms:.1f} ms, RMSE {pts[-1][2]:.4g}")
    spp_a = np.array([p[0] for p in pts], dtype=np.float64)
    t_a = np.array([p[1] for p in pts])
    e_a = np.array([p[2] for p in pts])
    ref_spp = n_chunks * chunk
    basis = 1.0 / spp_a + 1.0 / ref_spp
    c2 = float(np.sum(e_a ** 2 * basis) / np.sum(basis ** 2))
    slope, icpt = np.polyfit(spp_a, t_a, 1)
    inv = e_field[0] ** 2 / c2 - 1.0 / ref_spp
    spp_star = speedup = None
    if inv <= 0:
        note = "the field's error is below the reference's own noise"
    else:
        spp_star = 1.0 / inv
        note = ("interpolated" if pt_spp[0] <= spp_star <= pt_spp[-1] else
                "extrapolated above 256 spp" if spp_star > pt_spp[-1] else
                "the path tracer reaches the field's error below 16 spp")
        speedup = max(icpt + slope * spp_star, 0.0) / field_ms
    log(f"[matched] field RMSE {e_field[0]:.4g}, cache {e_cache[0]:.4g}; matched spp {spp_star} "
        f"({note}), speedup {speedup}")
    return {"g": g, "reference_spp": ref_spp,
            "field": {"ms": round(field_ms, 3), "rmse": e_field[0], "rel_rmse": e_field[1],
                      "psnr": e_field[2]},
            "cache_gather": {"ms": round(cache_ms, 3), "rmse": e_cache[0], "rel_rmse": e_cache[1],
                             "psnr": e_cache[2]},
            "path_tracer": [{"spp": p[0], "ms": round(p[1], 3), "rmse": p[2]} for p in pts],
            "spp_matched": spp_star, "note": note, "speedup_at_matched_rmse": speedup}


def first_interaction_bench(ctx, cam, rc, args):
    """The paper's own renderer (Section 3.6, Algorithm 2) on the benchmark scene and its trained
    field at 1 spp: delta-tracked first interaction along the pixel-centre ray, one batched field
    pass over the compacted interactions, next-event estimation with delta-tracking visibility,
    composition.  Timed at 720p (the resolution of the paper's Table 2) and 1080p, per kernel,
    beside the Monte Carlo path tracer at 1 spp with paths of at most 16 collisions (the
    comparison of Table 2).  The paper's figures are another GPU's and another dataset's:
    context, not a target."""
    import torch
    from paper_2304_07338_amd import scenegen as sg
    from paper_2304_07338_amd import _ffi
    from paper_2304_07338_amd.pfn import RenderConfig
    res = {}
    for W, H in ((1280, 720), (1920, 1080)):
        c = sg.Camera(cam.eye, cam.target, cam.up, cam.fov_y_deg, W, H)
        cfg = RenderConfig(**{**rc.__dict__, "spp": 1, "seed": 11})
        out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda:0")
        ctx.count_enable(True)
        ctx.render_first_interaction(c, cfg, out)
        _, inter = ctx.count_get()
        ctx.count_enable(False)
        for _ in range(3):
            ctx.render_first_interaction(c, cfg, out)
        torch.cuda.synchronize()
        ctx.timing_reset()
        ctx.timing_enable(True)
        n = args.steps
        ts = time.perf_counter()
        for _ in range(n):
            ctx.render_first_interaction(c, cfg, out)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - ts) * 1000.0 / n
        kms = {k: ctx.timing_get(i)[0] / n for k, i in (
            ("sample", _ffi.TK_FI_SAMPLE), ("nee", _ffi.TK_FI_NEE),
            ("field_encode", _ffi.TK_WF_ENCODE), ("field_dir", _ffi.TK_WF_DIR),
            ("field_mlp", _ffi.TK_WF_FIELD),
            ("resolve", _ffi.TK_WF_RESOLVE), ("frame", _ffi.TK_MARCH))}
        ctx.timing_enable(False)
        mean = float(out.mean())
        # the path tracer at 1 spp, paths of at most 16 collisions, no roulette
        ctx.render_path_traced(c, 1, max_bounces=16, g=rc.g, seed=3, out=out)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for _ in range(n):
            ctx.render_path_traced(c, 1, max_bounces=16, g=rc.g, seed=3, out=out)
        torch.cuda.synchronize()
        pt_ms = (time.perf_counter() - tp) * 1000.0 / n
        key = f"{W}x{H}"
        res[key] = {"ms_per_frame": round(wall, 4), "gpu_ms": round(kms["frame"], 4),
                    "kernels_ms": {k: round(v, 4) for k, v in kms.items() if k != "frame"},
                    "interactions_per_frame": int(inter),
                    "field_queries_per_s": round(inter / (wall * 1e-3), 1),
                    "path_tracer_16_ms": round(pt_ms, 4),
                    "speedup_vs_path_tracer": round(pt_ms / wall, 3), "image_mean": mean}
        log(f"[alg2] {key}: {wall:.3f} ms/frame ({kms['frame']:.3f} ms GPU; sample "
            f"{kms['sample']:.3f}, NEE {kms['nee']:.3f}, field {kms['field_encode']:.3f} + "
            f"{kms['field_dir']:.3f} + {kms['field_mlp']:.3f}, resolve {kms['resolve']:.3f}), "
            f"{inter} interactions; "
            f"path tracer (16 collisions) {pt_ms:.3f} ms")
    return {"workload": "c2 scene, Algorithm 2 renderer, 1 spp, f16 field",
            "g": rc.g, "indirect": "field", "per_resolution": res,
            "paper_table2_overall_ms": {"L_d": 7.08, "L_i": 5.07, "L": 12.42,
                                        "path_tracer_L": 57.97, "speedup_L": 4.58,
                                        "note": "720p, 1 spp, RTX 3090, averages over seven "
                                                "datasets' fly-throughs: context only"}}


def photon_map_bench(ctx, args):
    """Training on the photon-map targets of Eq. (5) (Section 3.3) with the staggered KNN schedule
    of Section 3.5.2: the map of the benchmark trace (HG bins and grid cells), K = 1024, batches
    of 2^16 as in the paper.  One step = batch, KNN estimates, Eq. (6), forward/backward, Adam.
    Timed at each radius of the schedule; the schedule's time over 3000 steps (36/27/27/10 % of
    them at radius/8, /4, /2, /1) is compared with 3000 steps at the final radius (the naive
    schedule), the comparison of the paper's Figure 10.  Trains a separate field slot."""
    import torch
    from paper_2304_07338_amd import _ffi
    from paper_2304_07338_amd.pfn import FieldConfig, TrainConfig
    t0 = time.time()
    ctx.photon_map_build(args.pm_grid)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    ctx.field_select(1)
    ctx.field_init(FieldConfig(), seed=9)
    stages = []
    for frac, share in ((0.125, 0.36), (0.25, 0.27), (0.5, 0.27), (1.0, 0.10)):
        r = args.pm_radius * frac
        cfg = TrainConfig(steps=args.pm_steps, log2_batch=16, precision="f16", seed=13,
                          target="photon_map", knn_k=1024, radius=r, staggered=False)
        ctx.train_field(TrainConfig(**{**cfg.__dict__, "steps": 2}))
        torch.cuda.synchronize()
        ctx.timing_reset()
        ctx.timing_enable(True)
        ts = time.perf_counter()
        ctx.train_field(cfg)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - ts) * 1000.0 / cfg.steps
        est_ms = ctx.timing_get(_ffi.TK_PM_ESTIMATE)[0] / cfg.steps
        ctx.timing_enable(False)
        stages.append({"radius": round(r, 5), "share": share, "ms_per_step": round(ms, 4),
                       "knn_ms_per_step": round(est_ms, 4)})
        log(f"[pmap] radius {r:.4f}: {ms:.3f} ms per step ({est_ms:.3f} ms of KNN estimates)")
    ctx.field_select(0)
    staggered_s = sum(st["share"] * 3000 * st["ms_per_step"] for st in stages) / 1000.0
    naive_s = 3000 * stages[-1]["ms_per_step"] / 1000.0
    log(f"[pmap] 3000 steps: staggered {staggered_s:.2f} s, naive {naive_s:.2f} s")
    return {"workload": "c2 trace (2^22 photons, 5 HG bins), K = 1024, batch 2^16",
            "grid": args.pm_grid, "build_s": round(build_s, 3), "stages": stages,
            "train_3000_steps_s": {"staggered": round(staggered_s, 3),
                                   "naive": round(naive_s, 3),
                                   "speedup": round(naive_s / staggered_s, 3)}}


def batch_bench(args):
    """Batched launch: 64 uneven renders (16 views with sides in [256, 1024] x 4 single-light
    field slots, each job at its own g) of the 256^3 f32 volume.  Timed three ways: as one
    graph-captured launch of the fused kernel (tile shape, block arrangement and persistent mode
    tuned); in the form the autotuner picks between that and the wavefront rounds (one pass per
    field slot, not graph-captured); and as 64 separate fused launches.  The four fields keep
    their initial parameters: the work of a frame (steps, field queries, gathers and
    matrix-core tiles) does not depend on the parameter values."""
    import torch
    from paper_2304_07338_amd import scenegen as sg
    from paper_2304_07338_amd import workloads as wl
    from paper_2304_07338_amd.pfn import Context, FieldConfig, INDIRECT_FIELD
    w = wl.C3
    vol, tf, lights = wl.make_scene(w, device="cuda:0")
    ctx = Context(0)
    ctx.set_volume(vol.contiguous())
    ctx.set_transfer_function(tf, w.extinction)
    ctx.set_lights(sg.lights_array(lights))
    ctx.build_light_volume(0.5)
    for l in range(w.n_lights):
        ctx.field_select(l)
        ctx.field_init(FieldConfig(), seed=100 + l)
    cams, cfgs = wl.batch_jobs(w)
    for c in cfgs:
        c.indirect = INDIRECT_FIELD
        c.field_precision = args.precision
    outs = [torch.empty((c.height, c.width, 3), dtype=torch.float32, device="cuda:0") for c in cams]
    pixels = sum(c.width * c.height for c in cams)

    def timed_batch(reps):
        ctx.render_batch(cams, cfgs, outs)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for _ in range(reps):
            ctx.render_batch(cams, cfgs, outs)
        torch.cuda.synchronize()
        return (time.perf_counter() - ts) * 1000.0 / reps

    # the fused kernel: one graph-captured (persistent) launch per batch, tuned
    t0 = time.time()
    ctx.set_render_strategy("fused")
    ctx.set_launch_mode(0, True)
    fbest = ctx.autotune_batch(cams, cfgs, outs, iters=1)
    ctx.set_tile_config(fbest["tile_w"], fbest["block_w"], fbest["block_h"])
    ctx.set_launch_mode(fbest["persistent"], True)
    graph_ms = timed_batch(args.batch_steps)
    # both forms: the autotuner reuses the fused result above, times the wavefront rounds and
    # makes the faster the context's form (graph replay applies to the fused kernel only)
    ctx.set_render_strategy("auto")
    best = ctx.autotune_batch(cams, cfgs, outs, iters=1)
    tune_s = time.time() - t0
    batch_ms = timed_batch(args.batch_steps)
    # the same 64 renders as separate launches of the fused kernel (default tiles, no graph)
    ctx.set_launch_mode(0, False)
    ctx.set_tile_config(8, 2, 2)
    ctx.set_render_strategy("fused")
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for c, f, o in zip(cams, cfgs, outs):
        ctx.render_frame(c, f, o)
    torch.cuda.synchronize()
    single_ms = (time.perf_counter() - ts) * 1000.0
    ctx.close()
    log(f"[batch] 64 jobs, {pixels} pixels: {batch_ms:.2f} ms per batch in the tuned form "
        f"({best}), {graph_ms:.2f} ms as one graph-captured fused launch ({fbest}), "
        f"{single_ms:.2f} ms as 64 fused launches; tuning {tune_s:.1f}s")
    return {"workload": w.name, "jobs": len(cams), "pixels": pixels,
            "ms_per_batch": round(batch_ms, 4), "jobs_per_s": round(len(cams) * 1000.0 / batch_ms, 2),
            "pixels_per_s": round(pixels * 1000.0 / batch_ms, 1),
            "ms_graph_captured_fused": round(graph_ms, 4),
            "fused_tuned": {k: fbest[k] for k in ("tile_w", "block_w", "block_h", "persistent")},
            "ms_as_separate_fused_launches": round(single_ms, 4),
            "autotuned": {k: best[k] for k in ("tile_w", "block_w", "block_h", "persistent",
                                               "strategy")},
            "autotune_s": round(tune_s, 2),
            "fields": "4 single-light fields at their initial parameters"}


def matched_rmse(args):
    """Large-scale comparison on one GPU: the photon-field render against a Monte Carlo path
    tracer (8 bounces, HG sampling, Russian roulette from bounce 3) at equal error.

    Scene: 1024^3 f16 (256 blobs, 6 octaves), 3 lights.  Two edits (a new transfer function,
    then a moved light) each re-trace 2^24 photons into a 128^3 x 5-bin cache and retrain the
    field with the cache-and-train recipe; the edit-to-first-frame latency covers light volume,
    trace, training and the first frame.  On the final scene: the field render (4 spp, field
    every 4 steps, light-transmittance volume, FP16 matrix cores) and the plain cache gather at
    g = 0.4 (a trained bin) and 0.2 (between bins), and the path tracer at 16..256 spp, each
    judged against a path-traced reference at --mr-ref-spp.  The path tracer's error is fitted
    as c^2 (1/spp + 1/ref_spp) (its own noise plus the reference's), solved for the spp at which
    it equals the field's error, and its time interpolated there."""
    import numpy as np
    import torch
    from paper_2304_07338_amd import scenegen as sg
    from paper_2304_07338_amd import workloads as wl
    from paper_2304_07338_amd.pfn import (Context, FieldConfig, RenderConfig, TrainConfig,
                                          DIRECT_LIGHT_VOLUME, INDIRECT_CACHE, INDIRECT_FIELD)
    w = wl.C4
    W, H = args.mr_width, args.mr_height
    n = args.mr_n
    t0 = time.time()
    vol, tf, lights = wl.make_scene(w, device="cuda:0", n=n)
    torch.cuda.synchronize()
    log(f"[mr] volume {n}^3 {w.vol_dtype} in {time.time() - t0:.1f}s")
    ctx = Context(0)
    ctx.set_volume(vol.contiguous())
    del vol
    la = sg.lights_array(lights)
    cam = wl.camera(w, 0, W, H)
    steps_cap = int(math.ceil(n * math.sqrt(3.0) * 2.0))
    out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda:0")

    def field_rc(g, indirect=INDIRECT_FIELD):
        return RenderConfig(spp=4, step_voxels=0.5, max_steps=steps_cap, t_min=1e-3,
                            field_stride=4, g=g, indirect=indirect, direct=DIRECT_LIGHT_VOLUME,
                            field_precision="f16", field_slot=0, seed=3)

    def rebuild(tf_table, lights_arr, seed):
        """set the scene, rebuild every derived quantity and render the first frame"""
        torch.cuda.synchronize()
        ts = time.perf_counter()
        marks = []

        def mark(name):  # stage boundaries (a synchronisation each, microseconds)
            torch.cuda.synchronize()
            marks.append((name, time.perf_counter()))

        ctx.set_transfer_function(tf_table, w.extinction)
        ctx.set_lights(lights_arr)
        ctx.build_light_volume(0.5)
        mark("light_volume")
        st = ctx.trace_photon_cache(1 << args.mr_photons, wl.C1_G_BINS, cache_res=128,
                                    seed=seed, max_collisions=8, rr_start=3)
        mark("trace_and_cache")
        ctx.field_init(FieldConfig(), seed=seed)
        hist = ctx.train_field(TrainConfig(steps=args.train_steps, log2_batch=18, seed=seed))
        mark("train")
        ctx.render_frame(cam, field_rc(0.4), out)
        mark("first_frame")
        prev, stages = ts, {}
        for name, t in marks:
            stages[name] = round(t - prev, 3)
            prev = t
        log(f"[mr] stages (s): {stages}")
        stage_log.append(stages)
        return marks[-1][1] - ts, st, float(np.mean(hist[-20:]))

    stage_log = []

    lat0, st, loss = rebuild(tf, la, 11)
    log(f"[mr] initial build + first frame {lat0:.2f}s ({st['n_records']} records, loss {loss:.4g})")
    # the field frame's form and tile, tuned once (the edits' first frames and the timings below
    # use them; the results are cached per frame shape and form)
    ta = time.perf_counter()
    tuned = {"field": ctx.autotune_batch([cam], [field_rc(0.4)], [out], iters=1),
             "cache_gather": ctx.autotune_batch([cam], [field_rc(0.4, INDIRECT_CACHE)], [out],
                                                iters=1)}
    ctx.autotune_batch([cam], [field_rc(0.4)], [out], iters=1)
    log(f"[mr] autotuned in {time.perf_counter() - ta:.1f}s: {tuned}")
    tf2 = sg.make_transfer_function(w.seed + 17)
    lat_tf, _, loss = rebuild(tf2, la, 12)
    log(f"[mr] transfer-function edit -> first frame {lat_tf:.2f}s (loss {loss:.4g})")
    la2 = la.copy()
    moved = sg.make_lights(1, w.seed + 29)[0]
    la2[0, :3] = moved.pos
    lat_light, _, loss = rebuild(tf2, la2, 13)
    log(f"[mr] light edit -> first frame {lat_light:.2f}s (loss {loss:.4g})")

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - ts) * 1000.0 / reps

    per_g = {}
    pt_spp = [16, 32, 64, 128, 256]
    for g in (0.4, 0.2):
        # the reference: the mean of independent path-traced renders of at most 512 spp each
        chunk = min(512, args.mr_ref_spp)
        n_chunks = max(1, args.mr_ref_spp // chunk)
        ref = torch.zeros_like(out)
        part = torch.empty_like(out)
        for c in range(n_chunks):
            ctx.render_path_traced(cam, chunk, max_bounces=8, g=g, rr_start=3, seed=1000 + c,
                                   out=part)
            ref += part
            torch.cuda.synchronize()
            log(f"[mr] g={g} reference {(c + 1) * chunk}/{n_chunks * chunk} spp")
        ref /= n_chunks
        ctx.autotune_batch([cam], [field_rc(g)], [out], iters=1)  # cached: the tuned form
        field_ms = timed(lambda: ctx.render_frame(cam, field_rc(g), out), 3)
        e_field = ctx.image_error(out, ref)
        ctx.autotune_batch([cam], [field_rc(g, INDIRECT_CACHE)], [out], iters=1)
        cache_ms = timed(lambda: ctx.render_frame(cam, field_rc(g, INDIRECT_CACHE), out), 3)
        e_cache = ctx.image_error(out, ref)
        pts = []
        for spp in pt_spp:
            img = torch.empty_like(out)
            ms = timed(lambda: ctx.render_path_traced(cam, spp, max_bounces=8, g=g, rr_start=3,
                                                      seed=2000 + spp, out=img), 1)
            pts.append((spp, ms, ctx.image_error(img, ref)[0]))
            log(f"[mr] g={g} PT {spp} spp: {ms:.1f} ms, RMSE {pts[-1][2]:.4g}")
        spp_a = np.array([p[0] for p in pts], dtype=np.float64)
        t_a = np.array([p[1] for p in pts])
        e_a = np.array([p[2] for p in pts])
        basis = 1.0 / spp_a + 1.0 / args.mr_ref_spp
        c2 = float(np.sum(e_a ** 2 * basis) / np.sum(basis ** 2))
        slope, icpt = np.polyfit(spp_a, t_a, 1)
        inv = e_field[0] ** 2 / c2 - 1.0 / args.mr_ref_spp
        if inv <= 0:
            spp_star, note = None, "field error below the reference's own noise level"
            speedup = None
        else:
            spp_star = 1.0 / inv
            note = ("interpolated" if pt_spp[0] <= spp_star <= pt_spp[-1] else
                    "extrapolated: the field is more accurate than the path tracer at 256 spp"
                    if spp_star > pt_spp[-1] else
                    "the path tracer reaches the field's error below 16 spp")
            t_star = max(icpt + slope * spp_star, 0.0)
            speedup = t_star / field_ms
        per_g[str(g)] = {
            "field": {"ms": round(field_ms, 3), "rmse": e_field[0], "rel_rmse": e_field[1],
                      "psnr": e_field[2]},
            "cache_gather": {"ms": round(cache_ms, 3), "rmse": e_cache[0], "rel_rmse": e_cache[1],
                             "psnr": e_cache[2]},
            "path_tracer": [{"spp": p[0], "ms": round(p[1], 3), "rmse": p[2]} for p in pts],
            "pt_noise_c": math.sqrt(c2), "spp_matched": spp_star, "note": note,
            "speedup_at_matched_rmse": speedup}
        log(f"[mr] g={g}: field {field_ms:.1f} ms RMSE {e_field[0]:.4g}; cache {cache_ms:.1f} ms "
            f"RMSE {e_cache[0]:.4g}; matched spp {spp_star} ({note}), speedup {speedup}")
    ctx.close()
    sp = per_g["0.4"]["speedup_at_matched_rmse"]
    return {
        "metric": "photon field vs path tracer at matched RMSE (time ratio)",
        "value": round(sp, 3) if sp is not None else None, "unit": "x", "n_gpus": 1,
        "higher_is_better": True, "vs_baseline": None, "dtype": "f16-mfma/f32",
        "data": "synthetic",
        "config": {"workload": w.name if n == w.n and (W, H) == (1920, 1080) else
                   f"{w.name} at {n}^3, {W}x{H}", "volume": f"{n}^3 f16", "resolution": f"{W}x{H}",
                   "field_spp": 4, "max_steps": steps_cap, "pt_spp": pt_spp,
                   "reference_spp": args.mr_ref_spp, "photons_per_trace": 1 << args.mr_photons,
                   "train_steps": args.train_steps},
        "autotuned": {k: {kk: v[kk] for kk in ("strategy", "tile_w", "block_w", "block_h",
                                                "persistent")} for k, v in tuned.items()},
        "edit_to_first_frame_s": {"initial": round(lat0, 3), "transfer_function": round(lat_tf, 3),
                                  "light": round(lat_light, 3)},
        "edit_stages_s": {"initial": stage_log[0], "transfer_function": stage_log[1],
                          "light": stage_log[2]},
        "per_g": per_g,
    }


def ssim_map(img, ref):
    """Per-pixel SSIM (Wang et al. 2004: Gaussian window sigma 1.5 truncated at 3.5 sigma,
    K1 = 0.01, K2 = 0.03) of the luminance (RGB mean) of two images, with the reference's
    maximum as the dynamic range L; borders are reflected."""
    import numpy as np
    from scipy.ndimage import gaussian_filter
    a = np.asarray(img, dtype=np.float64).mean(-1)
    b = np.asarray(ref, dtype=np.float64).mean(-1)
    L = max(float(b.max()), 1e-30)
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    f = lambda x: gaussian_filter(x, 1.5, truncate=3.5)
    ma, mb = f(a), f(b)
    va, vb, cab = f(a * a) - ma * ma, f(b * b) - mb * mb, f(a * b) - ma * mb
    return ((2 * ma * mb + c1) * (2 * cab + c2)) / ((ma * ma + mb * mb + c1) * (va + vb + c2))


def ssim(img, ref):
    """Mean SSIM over the image (ssim_map)."""
    return float(ssim_map(img, ref).mean())


def studies(args):
    """Phase-function awareness and stochastic noise (Sections 4.3 and 4.5 of the paper), on the
    256^3 f32 synthetic scene with 3 lights at 640x480.

    Phase awareness: fields trained on a trace with G = {-0.75, 0, 0.75}, one with g drawn from
    G and one with g uniform in [-0.75, 0.75] (targets linear in g between the bins), render L_i
    (the field-lit ray-marched frame minus the direct-only frame) at g in {-0.75, -0.35, 0, 0.35,
    0.75}; each is compared with the L_i of a separate single-bin photon cache traced at exactly
    that g (so g = +-0.35 are phases the pool-trained field never saw).  The error between two
    independent reference traces at g = 0 is the tracing floor.

    Network settings: the configuration against the paper's encoding and network (16 levels x 8
    features, growth 2, 5 hidden layers, batches of 2^16, relative or plain L2), trained on a
    5-phase trace and judged at g = 0.4 and 0.2, with training time and 640x480 frame time.

    Noise: the Algorithm 2 renderer with the field and the path tracer (at most 16 collisions)
    at 1, 4 and 8 spp; the noise of each is the RMS difference of two frames with different
    seeds over sqrt 2, relative to the mean of a 1024-spp path-traced frame."""
    import numpy as np
    import torch
    from paper_2304_07338_amd import scenegen as sg
    from paper_2304_07338_amd import workloads as wl
    from paper_2304_07338_amd.pfn import (Context, FieldConfig, RenderConfig, TrainConfig,
                                          DIRECT_LIGHT_VOLUME, INDIRECT_CACHE, INDIRECT_FIELD,
                                          INDIRECT_NONE)
    w = wl.C1
    W, H = 640, 480
    vol, tf, lights = wl.make_scene(w, device="cuda:0")
    ctx = Context(0)
    ctx.set_volume(vol.contiguous())
    ctx.set_transfer_function(tf, w.extinction)
    la = sg.lights_array(lights)
    ctx.set_lights(la)
    ctx.build_light_volume(0.5)
    cam = wl.camera(w, 0, W, H)
    G3 = (-0.75, 0.0, 0.75)
    photons = 1 << args.st_photons
    st = ctx.trace_photon_cache(photons, G3, cache_res=128, seed=21, max_collisions=8,
                                rr_start=3)
    # slot 0: g drawn from the pool G (Section 3.5.1); slot 6: g uniform over [-0.75, 0.75]
    # against the trace's cache linear in g between its bins
    for slot, gs in ((0, "pool"), (6, "uniform")):
        ctx.field_select(slot)
        ctx.field_init(FieldConfig(), seed=21)
        hist = ctx.train_field(TrainConfig(steps=args.train_steps, log2_batch=18, seed=21,
                                           g_sampling=gs))
        log(f"[st] trained on G = {G3} ({gs} g): {st['n_records']} records, loss "
            f"{np.mean(hist[-20:]):.4g}")

    def rc(g, indirect, spp=1, seed=3):
        return RenderConfig(spp=spp, step_voxels=0.5, max_steps=1024, t_min=1e-3, field_stride=4,
                            g=g, indirect=indirect, direct=DIRECT_LIGHT_VOLUME,
                            field_precision="f16", field_slot=0, seed=seed)

    def frame(cfg):
        out = ctx.render_frame(cam, cfg)
        torch.cuda.synchronize()
        return out.cpu().numpy().astype(np.float64)

    def li_field(g, slot=0):
        cfg = rc(g, INDIRECT_FIELD)
        cfg.field_slot = slot
        return frame(cfg) - frame(rc(g, INDIRECT_NONE))

    field_li = {g: li_field(g) for g in (-0.75, -0.35, 0.0, 0.35, 0.75)}
    field_li_u = {g: li_field(g, 6) for g in (-0.75, -0.35, 0.0, 0.35, 0.75)}
    # the training trace's own cache, linear in g between its bins: the estimate without network
    cache_li = {g: frame(rc(g, INDIRECT_CACHE)) - frame(rc(g, INDIRECT_NONE))
                for g in (-0.75, -0.35, 0.0, 0.35, 0.75)}

    def li_reference(g, seed):
        ctx.trace_photon_cache(photons, (g,), cache_res=128, seed=seed, max_collisions=8,
                               rr_start=3)
        return frame(rc(g, INDIRECT_CACHE)) - frame(rc(g, INDIRECT_NONE))

    phase = []
    for i, g in enumerate((-0.75, -0.35, 0.0, 0.35, 0.75)):
        ref = li_reference(g, 100 + i)
        f, fu, c = field_li[g], field_li_u[g], cache_li[g]
        rel = lambda a: float(np.sqrt(np.mean((a - ref) ** 2)) / ref.mean())
        phase.append({"g": g, "in_training_set": g in G3, "rel_rmse": rel(f), "ssim": ssim(f, ref),
                      "uniform_g_rel_rmse": rel(fu), "uniform_g_ssim": ssim(fu, ref),
                      "cache_interp_rel_rmse": rel(c), "cache_interp_ssim": ssim(c, ref),
                      "li_mean": float(ref.mean()), "field_li_mean": float(f.mean()),
                      "uniform_g_li_mean": float(fu.mean())})
        log(f"[st] g={g:+.2f} ({'trained' if g in G3 else 'unseen '}): L_i rel-RMSE "
            f"{phase[-1]['rel_rmse']:.4f}, SSIM {phase[-1]['ssim']:.4f} (field mean "
            f"{f.mean():.4g} vs {ref.mean():.4g}); uniform g: rel-RMSE "
            f"{phase[-1]['uniform_g_rel_rmse']:.4f}, SSIM {phase[-1]['uniform_g_ssim']:.4f} "
            f"(mean {fu.mean():.4g}); 3-bin cache in g: rel-RMSE {rel(c):.4f}, "
            f"SSIM {phase[-1]['cache_interp_ssim']:.4f}")
    a, b = li_reference(0.0, 300), li_reference(0.0, 301)
    floor = {"rel_rmse": float(np.sqrt(np.mean((a - b) ** 2)) / b.mean()), "ssim": ssim(a, b)}
    log(f"[st] two reference traces at g=0: rel-RMSE {floor['rel_rmse']:.4f}, "
        f"SSIM {floor['ssim']:.4f}")

    # noise: Algorithm 2 renderer with the field against the path tracer
    g = 0.0
    def fi(spp, seed):
        out = ctx.render_first_interaction(cam, rc(g, INDIRECT_FIELD, spp=spp, seed=seed))
        torch.cuda.synchronize()
        return out.cpu().numpy().astype(np.float64)

    def pt(spp, seed):
        out = ctx.render_path_traced(cam, spp, max_bounces=16, g=g, seed=seed)
        torch.cuda.synchronize()
        return out.cpu().numpy().astype(np.float64)

    ref = pt(1024, 999)
    noise = []
    for spp in (1, 4, 8):
        nf = float(np.sqrt(np.mean((fi(spp, 1) - fi(spp, 2)) ** 2) / 2) / ref.mean())
        npt = float(np.sqrt(np.mean((pt(spp, 1) - pt(spp, 2)) ** 2) / 2) / ref.mean())
        noise.append({"spp": spp, "field_first_interaction": nf, "path_tracer": npt})
        log(f"[st] {spp} spp: relative noise field {nf:.4f}, path tracer {npt:.4f}")
    # the configuration against the paper's network settings (Sections 3.4 and 3.5.1: 16 levels
    # x 8 features, growth 2, 5 hidden layers, batches of 2^16, relative L2), with g from the
    # pool and uniform in [-0.8, 0.8]; trained on one 5-phase trace and judged on L_i against
    # single-phase reference traces
    st5 = ctx.trace_photon_cache(photons, wl.C1_G_BINS, cache_res=128, seed=31, max_collisions=8,
                                 rr_start=3)
    paper = FieldConfig(hidden_layers=5, growth=2.0, levels=16, feats_per_level=8)
    variants = {
        "configuration": (FieldConfig(), TrainConfig(steps=args.train_steps, log2_batch=18,
                                                     seed=31)),
        "configuration_uniform_g": (FieldConfig(),
                                    TrainConfig(steps=args.train_steps, log2_batch=18, seed=31,
                                                g_sampling="uniform")),
        "paper_network_rel_l2": (paper, TrainConfig(steps=args.train_steps, log2_batch=16,
                                                    seed=31, loss="rel")),
        "paper_network_l2": (paper, TrainConfig(steps=args.train_steps, log2_batch=16, seed=31)),
        "paper_network_rel_l2_uniform_g": (paper, TrainConfig(steps=args.train_steps,
                                                              log2_batch=16, seed=31, loss="rel",
                                                              g_sampling="uniform")),
    }
    ab = {}
    for slot, (name, (fc, tc)) in enumerate(variants.items()):
        ctx.field_select(1 + slot)
        ctx.field_init(fc, seed=31)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        hist = ctx.train_field(tc)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - ts
        cfg = rc(0.4, INDIRECT_FIELD)
        cfg.field_slot = 1 + slot
        frame(cfg)
        tf0 = time.perf_counter()
        for _ in range(5):
            ctx.render_frame(cam, cfg)
        torch.cuda.synchronize()
        ab[name] = {"levels": fc.levels, "feats_per_level": fc.feats_per_level,
                    "hidden_layers": fc.hidden_layers, "growth": fc.growth,
                    "n_params": ctx.field_num_params(),
                    "batch": 1 << tc.log2_batch, "loss": tc.loss, "g_sampling": tc.g_sampling,
                    "train_s": round(train_s, 3),
                    "frame_ms": round((time.perf_counter() - tf0) * 200.0, 3),
                    "final_loss": float(np.mean(hist[-20:])), "per_g": {}}
    for i, g in enumerate((0.4, 0.2)):
        ref = li_reference(g, 400 + i)
        for slot, name in enumerate(variants):
            cfg = rc(g, INDIRECT_FIELD)
            cfg.field_slot = 1 + slot
            f = frame(cfg) - frame(rc(g, INDIRECT_NONE))
            ab[name]["per_g"][str(g)] = {
                "rel_rmse": float(np.sqrt(np.mean((f - ref) ** 2)) / ref.mean()),
                "ssim": ssim(f, ref)}
            log(f"[st] {name} g={g}: L_i rel-RMSE {ab[name]['per_g'][str(g)]['rel_rmse']:.4f}, "
                f"SSIM {ab[name]['per_g'][str(g)]['ssim']:.4f}, train {ab[name]['train_s']} s")
    ctx.field_select(0)
    ctx.close()
    return {"metric": "phase-function awareness and stochastic noise", "value": None,
            "unit": None, "n_gpus": 1, "data": "synthetic",
            "config": {"workload": f"{w.name} at {W}x{H}", "training_bins": list(G3),
                       "photons_per_trace": photons, "train_steps": args.train_steps},
            "phase_awareness": phase, "tracing_floor_g0": floor, "noise": noise,
            "network_settings": {"trace": f"{st5['n_records']} records, bins {list(wl.C1_G_BINS)}",
                                 "variants": ab}}


def cpu_baseline(args, w, vol, tf, la, ctx, cam, fcfg, rc):
    """The FP64 oracle rendering a lattice sample of the same frame on the host cores."""
    import numpy as np
    from oracle import pyoracle as orc
    t0 = time.time()
    dens = vol.float().cpu().numpy().astype(np.float64)
    os_ = orc.OracleScene(dens, tf, w.extinction, la)
    params = ctx.field_get_params().cpu().numpy().astype(np.float64)
    nb, res, kappa = ctx.cache_info()
    desc = orc.field_desc(levels=fcfg.levels, feats=fcfg.feats_per_level, base_res=fcfg.base_res,
                          growth=fcfg.growth, log2_table=fcfg.log2_table,
                          hidden_layers=fcfg.hidden_layers, width=fcfg.width, psi=fcfg.psi)
    k = args.cpu_sample
    xs = (np.arange(k) + 0.5) * w.width / k
    ys = (np.arange(k) + 0.5) * w.height / k
    pix = np.array([int(y) * w.width + int(x) for y in ys for x in xs], dtype=np.int64)
    op = orc.render_params(spp=1, step_voxels=0.5, max_steps=1024, t_min=1e-3, field_stride=4,
                           g=rc.g, indirect=orc.IND_FIELD, direct=orc.DIR_LIGHTVOL,
                           lv_step_voxels=0.5)
    prep = time.time() - t0
    t1 = time.time()
    orc.render_pixels(os_, cam, op, pixels=pix, field=(desc, params, 1, kappa))
    dt = time.time() - t1
    frame_s = dt * (w.width * w.height) / len(pix)
    log(f"[cpu] oracle: {len(pix)} pixels in {dt:.1f}s ({orc.num_threads()} threads, prep {prep:.1f}s)")
    return {"value": round(1.0 / frame_s, 8), "unit": "fps", "cores": orc.num_threads(),
            "kind": "oracle",
            "sample": f"{len(pix)} of {w.width * w.height} pixels on a {k}x{k} lattice of the "
                      f"same frame; frame time extrapolated ({dt:.1f}s for the sample)"}


if __name__ == "__main__":
    main()
