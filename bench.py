"""Benchmark of the CT projector hot path on one MI355X.

Metric: GUPS (voxel-view updates per second) of the forward + adjoint pair
on the 3-D circular cone-beam workload 256^3 x 360 views (512^2 detector,
SID 750 mm, SDD 1200 mm, 12 random ellipsoids, FP32):

    GUPS_pair = nx*ny*nz*n_views / (t_A + t_AT)

One step = pn_forward (work-copy relayout + forward kernel) followed by
pn_adjoint of its result.  Inputs are resident in HBM before timing starts.

Also reported: per-operator GUPS (A, A^T, voxel-driven back-projection),
the BF16-storage pair, the batched form, the roofline of the dominant
kernel and the FP64 CPU oracle timed on this host on a sample of views.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--cpu-views", type=int, default=16, help="views of the oracle CPU sample")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB elementwise copy kernel (counter calibration)")
    ap.add_argument("--profile-once", action="store_true",
                    help="run one forward and one adjoint only (for counter collection)")
    return ap.parse_args()


def timed(fn, reps, stream):
    import torch

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for s, e in evs:
        s.record(stream)
        fn()
        e.record(stream)
    torch.cuda.synchronize()
    ms = sorted(s.elapsed_time(e) for s, e in evs)
    return ms[len(ms) // 2], sum(ms) / len(ms)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2511_08427_amd as pn
    import workloads as W

    cfg = W.CONFIGS["cone3d_256"]
    shp, sp, det, ds = cfg["vol_shape"], cfg["vol_spacing"], cfg["det_shape"], cfg["det_spacing"]
    nviews = cfg["n_views"]
    upd = float(np.prod(shp)) * nviews
    log("building phantom and geometry")
    vol = W.ellipsoid_phantom_3d(cfg["seeds"][0], shp, sp, cfg["n_ellipsoids"])[0]
    geom = pn.cone_geometry(shp, sp, det, ds, nviews, cfg["sid"], cfg["sdd"])
    x = torch.from_numpy(vol).float().cuda()
    stream = torch.cuda.current_stream()
    sino = torch.empty(geom.sino_shape(), device="cuda")

    def step():
        y = pn.forward(x, geom)
        a = pn.adjoint(y, geom)
        return y, a

    if args.calib_copy:
        src = torch.ones(64 * 1024 * 1024, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)  # reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        log("calibration copy: 268435456 bytes read + 268435456 bytes written")
    if args.profile_once:
        step()
        torch.cuda.synchronize()
        log("profile-once: one forward + one adjoint done")
        return

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    value = upd * args.steps / wall / 1e9
    log(f"pair: {ms_step:.3f} ms/step, {value:.1f} GUPS")

    # per-operator times (HIP events on the stream the library launches on)
    reps = max(5, args.steps)
    y = pn.forward(x, geom)
    t_fwd, t_fwd_mean = timed(lambda: pn.forward(x, geom), reps, stream)
    t_adj, t_adj_mean = timed(lambda: pn.adjoint(y, geom), reps, stream)
    t_bp, _ = timed(lambda: pn.backproject(y, geom), reps, stream)
    log(f"A {t_fwd:.3f} ms, AT {t_adj:.3f} ms, BP {t_bp:.3f} ms")

    variants = {
        "forward_gups": upd / (t_fwd * 1e-3) / 1e9,
        "adjoint_gups": upd / (t_adj * 1e-3) / 1e9,
        "backproject_gups": upd / (t_bp * 1e-3) / 1e9,
        "forward_ms": t_fwd,
        "adjoint_ms": t_adj,
        "backproject_ms": t_bp,
    }
    if not args.no_variants:
        xb = x.to(torch.bfloat16)
        yb = pn.forward(xb, geom)
        tb_f, _ = timed(lambda: pn.forward(xb, geom), reps, stream)
        tb_a, _ = timed(lambda: pn.adjoint(yb, geom), reps, stream)
        variants["bf16_pair_gups"] = upd / ((tb_f + tb_a) * 1e-3) / 1e9
        variants["bf16_forward_ms"] = tb_f
        variants["bf16_adjoint_ms"] = tb_a
        log(f"bf16: A {tb_f:.3f} ms, AT {tb_a:.3f} ms")

    # roofline of the dominant operator under the per-view streaming model:
    # each voxel-view update moves the stored voxel once plus its share of
    # the view's detector row data: 4 + 4*nu*nv/(nx*ny*nz) bytes (FP32)
    bytes_per_upd = 4.0 + 4.0 * det[0] * det[1] / float(np.prod(shp))
    dom_name, dom_ms = ("forward", t_fwd_mean) if t_fwd_mean >= t_adj_mean else ("adjoint", t_adj_mean)
    achieved = bytes_per_upd * upd / (dom_ms * 1e-3) / 1e9
    roofline = {
        "bound": "hbm",
        "kernel": dom_name,
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": None,
        "bytes_per_update": bytes_per_upd,
    }

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O

        nv_s = args.cpu_views
        log(f"cpu baseline: oracle on {nv_s} of {nviews} views")
        go = O.circular_cone(shp, sp, det, ds, nviews, cfg["angular_range"], cfg["sid"], cfg["sdd"])
        step_v = nviews // nv_s
        sub = dict(go)
        sub["P"] = np.ascontiguousarray(go["P"][::step_v][:nv_s])
        threads = O.max_threads()
        t0 = time.perf_counter()
        ys = O.forward(vol, sub)
        t1 = time.perf_counter()
        O.adjoint(ys, sub)
        t2 = time.perf_counter()
        upd_s = float(np.prod(shp)) * nv_s
        cpu = {
            "value": round(upd_s / (t2 - t0) / 1e9, 4),
            "unit": "GUPS",
            "cores": threads,
            "kind": "oracle",
            "sample": f"forward+adjoint of the 256^3 phantom over {nv_s} of the 360 views (every {step_v}th), "
                      f"FP64, {threads} OpenMP threads; A {t1 - t0:.2f} s, AT {t2 - t1:.2f} s",
        }
        log(f"cpu: {cpu['value']} GUPS")

    out = {
        "metric": "GUPS (voxel·views/s) fwd+adjoint, cone 256³×360, FP32 vs BF16-store/batched",
        "value": round(value, 2),
        "unit": "GUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "cone3d_256: 256^3 FP32 volume (0.5 mm, 12 random ellipsoids, seed 3), 360 views over "
                        "360 deg, 512x512 detector at 1.0 mm, SID 750 mm, SDD 1200 mm; step = A then A^T",
            "global_batch": 1,
            "parallelism": "single-gpu",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in variants.items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
