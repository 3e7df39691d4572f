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
# the projector kernels' sources: the counters in profiles/ hold for the
# sha256 of these files, concatenated in this order
KERNEL_SRCS = [os.path.join(ROOT, "paper_2511_08427_amd", "csrc", f)
               for f in ("pn_kernels.hip", "pn_ray.hpp", "pn_common.hpp", "pn_device.hpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cone3d_256_hbm_traffic.md")
COUNTER_FILE = os.path.join(ROOT, "profiles", "cone3d_256_counters.md")


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
                    help="run one forward, adjoint, back-projection and filter only (for counter collection)")
    ap.add_argument("--profile-sampler", action="store_true",
                    help="run one staged forward and back-projection and one sampler-interpolation forward "
                         "and back-projection per image only (for counter collection)")
    ap.add_argument("--profile-splat", action="store_true",
                    help="run the splat of the back-projected sinogram twice only (for counter collection)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 32-problem batched variant")
    ap.add_argument("--unrolled512", action="store_true",
                    help="also time the 512^3 x 720 unrolled 10-step reconstruction (FP32 and BF16 storage)")
    return ap.parse_args()


def profiled_value(path, key):
    """A per-call figure from a committed rocprofv3 summary, or None when the
    kernels have changed since it was taken (source sha256 recorded there)."""
    import hashlib

    try:
        text = open(path).read()
        h = hashlib.sha256()
        for f in KERNEL_SRCS:
            h.update(open(f, "rb").read())
        src = h.hexdigest()
    except OSError:
        return None
    sha = val = None
    for line in text.splitlines():
        if line.startswith("kernel_source_sha256:"):
            sha = line.split(":", 1)[1].strip()
        if line.startswith(key + ":"):
            val = float(line.split(":", 1)[1])
    return val if sha == src else None


def measured_traffic(op):
    """HBM bytes per call of `op` from the committed FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernels have changed since it was taken."""
    return profiled_value(TRAFFIC_FILE, f"traffic_bytes_per_call {op}")


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


def batched_variant(pn, W, np, torch, stream):
    """Aggregate GUPS of pn_forward_batched + pn_adjoint_batched over the
    seeded 32-problem uneven cone-beam list (64^3..256^3, 90..720 views,
    128^2..512^2 detectors; perturbed, helical and sinusoidal orbits)."""
    import math

    log("batched: building 32 problems")
    pairs, upd = [], 0.0
    for p in W.batched_problem_list():
        n = p["vol_shape"]
        draws = W.perturbation_draws(p["perturb_seed"], p["n_views"]) if p["trajectory"] == "perturbed" else None
        g = pn.cone_geometry(n, p["vol_spacing"], p["det_shape"], p["det_spacing"], p["n_views"], p["sid"],
                             p["sdd"], p["angular_range"], p["trajectory"], p["pitch"], draws)
        vol = W.ellipsoid_phantom_3d(p["phantom_seed"], n, p["vol_spacing"], p["n_ellipsoids"])[0]
        pairs.append((torch.from_numpy(vol).float().cuda(), g))
        upd += float(np.prod(n)) * p["n_views"]
    sinos = pn.forward_batched(pairs)
    sp = [(y, g) for y, (_, g) in zip(sinos, pairs)]
    pn.adjoint_batched(sp)
    torch.cuda.synchronize()
    tf, _ = timed(lambda: pn.forward_batched(pairs), 3, stream)
    ta, _ = timed(lambda: pn.adjoint_batched(sp), 3, stream)
    log(f"batched: A {tf:.2f} ms, AT {ta:.2f} ms over {upd / 1e9:.1f} G updates")
    # the same 32 problems as one single call each, back to back
    tsf, _ = timed(lambda: [pn.forward(x, g) for x, g in pairs], 3, stream)
    tsa, _ = timed(lambda: [pn.adjoint(y, g) for y, g in sp], 3, stream)
    log(f"single calls: A {tsf:.2f} ms, AT {tsa:.2f} ms")
    # batch plans: one launch per kernel group, replayed from the library's graph
    fplan = pn.BatchPlan("forward", pairs)
    aplan = pn.BatchPlan("adjoint", sp)
    fplan.run()
    aplan.run()
    torch.cuda.synchronize()
    tpf, _ = timed(fplan.run, 3, stream)
    tpa, _ = timed(aplan.run, 3, stream)
    log(f"batch plans (graph replay): A {tpf:.2f} ms, AT {tpa:.2f} ms")
    fplan.close()
    aplan.close()
    return {
        "batch_plan_pair_gups": upd / ((tpf + tpa) * 1e-3) / 1e9,
        "batch_plan_forward_ms": tpf,
        "batch_plan_adjoint_ms": tpa,
        "batched_pair_gups": upd / ((tf + ta) * 1e-3) / 1e9,
        "batched_forward_ms": tf,
        "batched_adjoint_ms": ta,
        "batched_updates": upd,
        "batched_list_single_calls_pair_gups": upd / ((tsf + tsa) * 1e-3) / 1e9,
        "batched_list_single_forward_ms": tsf,
        "batched_list_single_adjoint_ms": tsa,
    }


def unrolled_variant(pn, W, np, torch):
    """Ten checkpointed gradient steps x <- x - alpha A^T (A x - y) on the
    512^3 x 720 workload (1024^2 detector at 0.5 mm), forward and backward
    through the loop, with FP32 and with BF16 storage.  y is Poisson data
    (I0 = 1e5, kappa = 4 / max(A x_true), counts drawn on the GPU from a
    generator seeded 55); alpha = 1/L from 20 power iterations of A^T A."""
    cfg = W.CONFIGS["cone3d_512"]
    shp, sp, det, ds = cfg["vol_shape"], cfg["vol_spacing"], cfg["det_shape"], cfg["det_spacing"]
    log("unrolled512: phantom")
    geom = pn.cone_geometry(shp, sp, det, ds, cfg["n_views"], cfg["sid"], cfg["sdd"])
    x_true = torch.from_numpy(W.ellipsoid_phantom_3d(cfg["seeds"][0], shp, sp, cfg["n_ellipsoids"])[0]).float().cuda()
    with torch.no_grad():
        p = pn.forward(x_true, geom)
        kappa = 4.0 / float(p.max())
        gen = torch.Generator(device="cuda")
        gen.manual_seed(cfg["poisson_seed"])
        counts = torch.poisson(cfg["I0"] * torch.exp(-kappa * p), generator=gen)
        y = -torch.log(torch.clamp(counts, min=1.0) / cfg["I0"]) / kappa
        del p, counts
        gen.manual_seed(cfg["poisson_seed"] + 1)
        v = torch.randn(x_true.shape, device="cuda", generator=gen)
        log("unrolled512: power iterations")
        for _ in range(20):
            w = pn.adjoint(pn.forward(v, geom), geom)
            lam = float(w.norm() / v.norm())
            v = w / w.norm()
        del v, w
    alpha = 1.0 / lam
    upd = float(np.prod(shp)) * cfg["n_views"]
    steps = cfg["unrolled_steps"]
    out = {"alpha": alpha, "steps": steps, "kappa": kappa}
    results = {}
    for name, dt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
        x0 = torch.zeros(shp, device="cuda", dtype=dt, requires_grad=True)
        yd = y.to(dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xk = pn.unrolled_gd(x0, yd, geom, alpha, steps, checkpoint=True)
        loss = 0.5 * (xk.float() - x_true).square().sum()
        loss.backward()
        torch.cuda.synchronize()
        dt_s = time.perf_counter() - t0
        # operator calls: 2 per step forward; recompute (2) + backward (2) per step
        calls = 6 * steps
        results[name] = xk.detach().float()
        out[f"{name}_seconds"] = round(dt_s, 3)
        out[f"{name}_operator_gups"] = round(calls * upd / dt_s / 1e9, 1)
        out[f"{name}_rel_error_vs_truth"] = float((xk.detach().float() - x_true).norm() / x_true.norm())
        log(f"unrolled512 {name}: {dt_s:.2f} s, {out[f'{name}_operator_gups']} GUPS over {calls} operator calls")
        del x0, xk, loss
    out["bf16_vs_f32_rel"] = float((results["bf16"] - results["f32"]).norm() / results["f32"].norm())
    return out


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
    if args.profile_sampler:
        pn.forward(x, geom)
        pn.forward_sampled(x, geom, "bordered")
        pn.forward_sampled(x, geom, "direct")
        y = pn.forward(x, geom)
        pn.backproject(y, geom)
        pn.backproject_sampled(y, geom, "bordered")
        pn.backproject_sampled(y, geom, "direct")
        torch.cuda.synchronize()
        log("profile-sampler: staged and sampler forward and back-projection done")
        return
    if args.profile_splat:
        bpv = pn.backproject(pn.forward(x, geom), geom)
        pn.splat(bpv, geom)
        pn.splat(bpv, geom)
        torch.cuda.synchronize()
        log("profile-splat: two splats of the back-projected sinogram done")
        return
    if args.profile_once:
        y, _ = step()
        pn.backproject(y, geom)
        pn.fbp_filter(y, geom, "shepp-logan")
        torch.cuda.synchronize()
        log("profile-once: one forward, adjoint, back-projection and Shepp-Logan filter done")
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
    # the back-projection's transpose (its gradient), volume -> sinogram
    bpv = pn.backproject(y, geom)
    t_splat, _ = timed(lambda: pn.splat(bpv, geom), reps, stream)
    log(f"splat (BP transpose) {t_splat:.3f} ms")
    # FDK: the row filter (a linear convolution, nu^2 multiply-adds per
    # detector row, as a Toeplitz product on the matrix cores) followed by
    # the back-projection
    t_filt, _ = timed(lambda: pn.fbp_filter(y, geom), reps, stream)
    t_filt_sl, _ = timed(lambda: pn.fbp_filter(y, geom, "shepp-logan"), reps, stream)
    t_fdk, _ = timed(lambda: pn.fbp(y, geom), reps, stream)
    filt_flop = 2.0 * geom.n_views * geom.det_shape[0] * geom.det_shape[1] ** 2
    # artifact simulation on the sinogram: Gaussian noise (read + write of
    # every element)
    yn = y.clone()
    t_noise, _ = timed(lambda: pn.gaussian_noise_(yn, 0.0, 0.01, seed=1), reps, stream)
    noise_gbs = 2 * yn.numel() * 4 / (t_noise * 1e-3) / 1e9
    log(f"Gaussian noise on the sinogram: {t_noise:.3f} ms ({noise_gbs:.0f} GB/s)")
    # the other sinogram-domain simulators: detector jitter (shifted copy),
    # gantry blur (9-tap line kernel per view), ring artifacts (32 columns
    # over half of the views, in place)
    t_jit, _ = timed(lambda: pn.detector_jitter(y, 2, seed=3), reps, stream)
    t_blur, _ = timed(lambda: pn.gantry_blur(y, 0.0, 2 * math.pi / nviews, 9), reps, stream)
    ring_cols = list(range(100, 420, 10))
    t_ring, _ = timed(lambda: pn.ring_artifacts_(yn, ring_cols, 0.5, (0, nviews // 2)), reps, stream)
    copy_bytes = 2 * y.numel() * 4
    log(f"jitter {t_jit:.3f} ms ({copy_bytes / (t_jit * 1e-3) / 1e9:.0f} GB/s), blur {t_blur:.3f} ms "
        f"({copy_bytes / (t_blur * 1e-3) / 1e9:.0f} GB/s), ring {t_ring:.3f} ms")
    # a plain device-to-device copy of the sinogram (read + write), the
    # achievable streaming bandwidth on this GPU
    yc = torch.empty_like(y)
    t_copy, _ = timed(lambda: yc.copy_(y), reps, stream)
    copy_gbs = copy_bytes / (t_copy * 1e-3) / 1e9
    log(f"copy of the sinogram: {t_copy:.3f} ms ({copy_gbs:.0f} GB/s)")
    log(f"FDK: Ram-Lak filter {t_filt:.3f} ms, Shepp-Logan filter {t_filt_sl:.3f} ms "
        f"({filt_flop / (t_filt_sl * 1e-3) / 1e12:.1f} TFLOP/s), filter + BP {t_fdk:.3f} ms")

    variants = {
        "forward_gups": upd / (t_fwd * 1e-3) / 1e9,
        "adjoint_gups": upd / (t_adj * 1e-3) / 1e9,
        "backproject_gups": upd / (t_bp * 1e-3) / 1e9,
        "forward_ms": t_fwd,
        "adjoint_ms": t_adj,
        "backproject_ms": t_bp,
        "splat_ms": t_splat,
        "splat_gups": upd / (t_splat * 1e-3) / 1e9,
        "fdk_filter_ms": t_filt,
        "fdk_filter_shepp_logan_ms": t_filt_sl,
        "fdk_filter_shepp_logan_tflops": filt_flop / (t_filt_sl * 1e-3) / 1e12,
        "fdk_ms": t_fdk,
        "noise_ms": t_noise,
        "noise_gbps": noise_gbs,
        "jitter_ms": t_jit,
        "jitter_gbps": copy_bytes / (t_jit * 1e-3) / 1e9,
        "blur_ms": t_blur,
        "blur_gbps": copy_bytes / (t_blur * 1e-3) / 1e9,
        "ring_ms": t_ring,
        "copy_gbps": copy_gbs,
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
        # sampler interpolation: every tap a load through the caches, from
        # the bordered copies (extra memory, as the staged projector) or from
        # the volume itself (none); with FP32 and with 8-bit weights
        for key, src, bits in (("sampler_bordered", "bordered", 0), ("sampler_direct", "direct", 0),
                               ("sampler_bordered_w8", "bordered", 8)):
            pn.forward_sampled(x, geom, src, bits)
            t_s, _ = timed(lambda: pn.forward_sampled(x, geom, src, bits), reps, stream)
            variants[f"{key}_forward_ms"] = t_s
            variants[f"{key}_forward_gups"] = upd / (t_s * 1e-3) / 1e9
            log(f"sampler ({src}, weight_bits {bits}): A {t_s:.3f} ms")
        # the back-projection with sampler interpolation (no LDS rectangles)
        for key, src in (("bp_sampler_bordered", "bordered"), ("bp_sampler_direct", "direct")):
            pn.backproject_sampled(y, geom, src)
            t_s, _ = timed(lambda: pn.backproject_sampled(y, geom, src), reps, stream)
            variants[f"{key}_ms"] = t_s
            variants[f"{key}_gups"] = upd / (t_s * 1e-3) / 1e9
            log(f"sampler ({src}): BP {t_s:.3f} ms")

    if not args.no_variants and not args.no_batched:
        variants.update(batched_variant(pn, W, np, torch, stream))
    if args.unrolled512:
        variants["unrolled512"] = unrolled_variant(pn, W, np, torch)

    # roofline of the dominant operator under the per-view streaming model:
    # each voxel-view update moves the stored voxel once plus its share of
    # the view's detector data: 4 + 4*nu*nv/(nx*ny*nz) bytes (FP32).  The
    # unit is one call of the operator (all its kernels), timed with HIP
    # events on the stream the library launches on.
    bytes_per_upd = 4.0 + 4.0 * det[0] * det[1] / float(np.prod(shp))
    dom_name, dom_ms = ("forward", t_fwd_mean) if t_fwd_mean >= t_adj_mean else ("adjoint", t_adj_mean)
    achieved = bytes_per_upd * upd / (dom_ms * 1e-3) / 1e9
    roofline = {
        "bound": "hbm",
        "kernel": "pn_forward (relayouts + forward_kernel)" if dom_name == "forward"
        else "pn_adjoint (adjoint_fused_kernel: all pass axes in one launch)",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(dom_name),
        "bytes_per_update": bytes_per_upd,
        "algorithmic_bytes_per_call": bytes_per_upd * upd,
        "call_ms": round(dom_ms, 4),
    }
    # what the counters say about the same kernel (committed rocprofv3
    # summary of the same source; null once the kernels have changed)
    busy = profiled_value(COUNTER_FILE, f"valu_busy_percent {dom_name}")
    if busy is not None:
        roofline["counters"] = {
            "valu_busy_percent": busy,
            "valu_instructions_per_call": profiled_value(COUNTER_FILE, f"valu_instructions_per_call {dom_name}"),
            "lds_bank_conflict_percent": profiled_value(COUNTER_FILE, f"lds_bank_conflict_percent {dom_name}"),
            "l2_hit_percent": profiled_value(COUNTER_FILE, f"l2_hit_percent {dom_name}"),
            "occupancy_percent": profiled_value(COUNTER_FILE, f"occupancy_percent {dom_name}"),
            "source": "profiles/cone3d_256_counters.md",
        }
    # the same achieved rate against a plain device copy measured here
    if variants.get("copy_gbps"):
        roofline["frac_of_measured_copy"] = round(achieved / variants["copy_gbps"], 4)

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
