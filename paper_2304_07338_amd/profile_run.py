"""Profiling driver: renders the 1080p photon-field frame of the benchmark (512^3 f16 volume,
field every 4 steps, FP16 matrix cores) a few times, plus one plain device copy of 1 GiB whose
memory counters calibrate the HBM traffic counters.  The field keeps its initial parameters:
the memory access pattern of a ray-marched frame does not depend on the parameter values.
With --renderer first_interaction it renders the same view with the Algorithm 2 renderer at 1
spp instead (at --width x --height).  With --train-steps N it then runs N training steps of the
benchmark's recipe (batch 2^18, FP16 matrix cores) on the traced cache, for the training kernels'
counters.  With --paper-encoding the field is the paper's (16 levels x 8 features, growth 2, 5
hidden layers) instead of the configuration's.

    python -m paper_2304_07338_amd.profile_run [--frames 3] [--strategy auto|fused|wavefront]
        [--renderer march|first_interaction] [--width 1920 --height 1080] [--train-steps 0]
        [--paper-encoding]
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=3)
    ap.add_argument("--precision", default="f16")
    ap.add_argument("--strategy", default="auto",
                    choices=["auto", "fused", "wavefront", "wavefront_serial"])
    ap.add_argument("--renderer", default="march", choices=["march", "first_interaction"])
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--train-steps", type=int, default=0)
    ap.add_argument("--paper-encoding", action="store_true",
                    help="the paper's field: 16 levels x 8 features, growth 2, 5 hidden layers")
    args = ap.parse_args()
    import torch
    from paper_2304_07338_amd import scenegen as sg
    from paper_2304_07338_amd import workloads as wl
    from paper_2304_07338_amd.pfn import (Context, FieldConfig, RenderConfig, TrainConfig,
                                          DIRECT_LIGHT_VOLUME, INDIRECT_FIELD)
    w = wl.C2
    vol, tf, lights = wl.make_scene(w, device="cuda:0")
    ctx = Context(0)
    ctx.set_render_strategy(args.strategy)
    ctx.set_volume(vol.contiguous())
    ctx.set_transfer_function(tf, w.extinction)
    ctx.set_lights(sg.lights_array(lights))
    ctx.build_light_volume(0.5)
    ctx.trace_photon_cache(1 << 22, wl.C1_G_BINS, cache_res=128, seed=6)
    fc = FieldConfig(feats_per_level=8, growth=2.0, hidden_layers=5) if args.paper_encoding \
        else FieldConfig()
    ctx.field_init(fc, seed=1)
    cam0 = wl.camera(w, 0)
    cam = sg.Camera(cam0.eye, cam0.target, cam0.up, cam0.fov_y_deg, args.width, args.height)
    rc = RenderConfig(spp=1, step_voxels=0.5, max_steps=1024, t_min=1e-3, field_stride=4, g=0.4,
                      indirect=INDIRECT_FIELD, direct=DIRECT_LIGHT_VOLUME,
                      field_precision=args.precision)
    out = torch.empty((cam.height, cam.width, 3), dtype=torch.float32, device="cuda:0")
    render = ctx.render_first_interaction if args.renderer == "first_interaction" else \
        ctx.render_frame
    for i in range(args.frames):
        render(cam, rc, out)
        torch.cuda.synchronize()
        print(f"frame {i} done", flush=True)
    if args.train_steps > 0:
        ctx.train_field(TrainConfig(steps=args.train_steps, log2_batch=18, precision="f16",
                                    seed=7))
        print(f"{args.train_steps} training steps done", flush=True)
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)  # 1 GiB read + 1 GiB write
    torch.cuda.synchronize()
    print("calibration copy done (1 GiB)", flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
