"""Benchmark: ms/frame for a 256^3 hierarchical surface + a 512^2 mesh-free render.

One step = one frame of the hot path on synthetic inputs already resident in HBM:
  * pifu_occupancy_grid: 256^3 cells (257^3 nodes) from a 32^3 coarse level, PIFu-size
    MLP (256+z)->1024->512->256->128->1 with feature skips over a 256 ch x 128 x 128
    feature map;
  * pifu_render_view: 512 x 512 image, 256 depth cells, from a 64 x 64 x 32 coarse
    level, view rotated 90 degrees about y, colour MLP (256+z+occ)->512->256->3 over
    a second 256 ch x 128 x 128 map.
Prints one JSON line (see the design doc for the fields).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0
FP8_MFMA_PEAK_TFLOPS = 5000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--form", default="fp32", choices=["fp32"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget of the oracle timing sample (cpu_baseline)")
    ap.add_argument("--no-cpu", action="store_true")
    return ap.parse_args()


def cpu_baseline(points_per_frame, budget_s):
    """Times the FP64 oracle's occupancy MLP on a bounded sample of points and scales
    it to the frame's number of evaluated points."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import synth
    from oracle import pifu_oracle as O
    feat = synth.pifu_features()
    spec = synth.pifu_mlp()
    fld = O.Field("mlp", feat=feat, mlp=spec)
    pts = synth.precision_points(200000, 7)
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and done < pts.shape[0]:
        O.field_logit(fld, pts[done:done + 8192])
        done += 8192
    dt = time.perf_counter() - t0
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    per_pt = dt / done
    return {"value": per_pt * points_per_frame * 1e3, "unit": "ms/frame", "cores": threads,
            "kind": "oracle",
            "sample": f"FP64 oracle occupancy MLP on {done} points ({dt:.1f} s), scaled to the "
                      f"frame's {points_per_frame} MLP-evaluated points (occupancy grid + render); "
                      f"level logic and colour MLP not included"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is described in DESIGN.md only)"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2007_13988_amd as P
    import synth

    torch.cuda.set_device(0)
    feat = synth.pifu_features()
    spec = synth.pifu_mlp()
    occ_field = P.DeviceField.mlp_field(feat, spec)
    col_field = P.DeviceField.mlp_field(synth.color_features(), synth.color_mlp())
    view = synth.yaw_view(90.0)
    bg = (0.0, 0.0, 0.0)
    prec = "fp32"
    gopts = P.grid_opts(8, 5, precision=prec, guard_logit=1e-3)
    gout = P.GridOutputs(occ_field, gopts)
    ropts = P.render_opts(9, 8, 6, precision=prec, guard_logit=1e-3)
    rout = P.RenderOutputs(occ_field, col_field, ropts)
    stream = torch.cuda.current_stream()

    def frame():
        P.occupancy_grid_into(occ_field, gout, stream)
        P.render_view_into(occ_field, col_field, view, bg, rout, stream)

    for _ in range(args.warmup):
        frame()
    torch.cuda.synchronize()
    P.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_occ = 0.0
    for _ in range(args.steps):
        a = time.perf_counter()
        P.occupancy_grid_into(occ_field, gout, stream)
        t_occ += time.perf_counter() - a
        P.render_view_into(occ_field, col_field, view, bg, rout, stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = P.profile_read()
    P.profile_enable(False)

    ms = elapsed / args.steps * 1e3
    gst = [s.as_dict() for s in gout.stats]
    rst = [s.as_dict() for s in rout.stats]
    occ_pts = sum(s["mlp_points"] for s in gst)
    ren_pts = sum(s["mlp_points"] for s in rst)
    hits = rst[-1]["hits"]
    pts_frame = occ_pts + ren_pts
    g = prof["gemm_f32"]
    avg_ms = g["total_ms"] / max(g["launches"], 1)
    flops_per_launch = g["flops"] / max(g["launches"], 1)
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    roofline = {"kernel": "k_gemm_f32 (MLP hidden layers, FP32 MFMA)", "bound": "mfma",
                "achieved": round(achieved, 2), "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_MFMA_PEAK_TFLOPS, 4), "traffic": None,
                "launches_per_step": g["launches"] / args.steps,
                "avg_launch_ms": round(avg_ms, 4),
                "flops_per_launch": flops_per_launch}
    mlp_flops = spec.flops_per_point()
    out = {
        "metric": "ms/frame to 256^3 surface + 512^2 render",
        "value": round(ms, 3), "unit": "ms/frame", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "hierarchical occupancy grid 256^3 cells from 32^3 + mesh-free "
                               "render 512x512x256 from 64x64x32, yaw 90",
                   "form": args.form,
                   "occupancy_mlp": "(256+z)->1024->512->256->128->1 skip, 256ch x 128^2 features",
                   "color_mlp": "(256+z+occ)->512->256->3", "guard_logit": 1e-3},
        "ms_occupancy_grid": round(t_occ / args.steps * 1e3, 3),
        "mlp_queries_per_s": round(pts_frame / (ms * 1e-3), 1),
        "mlp_points_per_frame": {"occupancy_grid": occ_pts, "render": ren_pts, "color_hits": hits},
        "dense_points_256": 257 ** 3,
        "acceleration_vs_dense": round(257 ** 3 / max(occ_pts, 1), 2),
        "occupancy_mlp_tflops_effective": round(pts_frame * mlp_flops / (ms * 1e-3) / 1e12, 2),
        "roofline": roofline,
        "kernels": {k: {"launches": v["launches"] / args.steps,
                        "ms_per_step": round(v["total_ms"] / args.steps, 3)} for k, v in prof.items()
                    if v["launches"]},
        "levels_occupancy": gst, "levels_render": rst,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(pts_frame, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
