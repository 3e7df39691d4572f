"""Batch plans (pn_batch_create / pn_batch_run) through the C ABI: one
launch per kernel group over a fixed problem list, replayed from a HIP graph
the library captures.

Every output must equal the batched call's (itself tied to the single calls
and, at full size, to the oracle) bit for bit, on every replay: the inputs
are changed in place between replays, with eager work and synchronisation in
between, and each replay is checked against the eager batched result of the
current inputs.
"""
import math
import sys

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-batch-plan] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pn():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2511_08427_amd as pn

    return pn


def _problems(pn):
    """17 problems: mixed sizes and trajectories, one geometry used three
    times, two 2-D problems and one with no views."""
    out = []
    kinds = ["circular", "helical", "sinusoidal", "perturbed"]
    for i in range(12):
        n = (12 + 3 * i, 14 + 2 * i, 10 + i)
        det = (18 + i, 21 + 2 * i)
        kind = kinds[i % 4]
        draws = W.perturbation_draws(900 + i, 7 + i) if kind == "perturbed" else None
        g = pn.cone_geometry(n, (0.9, 0.8, 1.0), det, (1.3, 1.2), 7 + i, 400.0, 650.0, 2 * math.pi, kind, 0.5, draws)
        out.append((g, W.ellipsoid_phantom_3d(600 + i, n, (0.9, 0.8, 1.0), 5)[0]))
    g0, v0 = out[0]
    out.append((g0, v0[::-1].copy()))
    out.append((g0, 0.5 * v0))
    for s in (2, 3):
        g = pn.fan_geometry((40 + 7 * s, 33), (0.6, 0.6), 70, 0.6, 30 + s, 500.0, 800.0)
        out.append((g, W.ellipse_phantom_2d(s, (40 + 7 * s, 33), (0.6, 0.6))[0]))
    g_empty = pn.Geometry(3, "cone", (9, 8, 7), (1.0,) * 3, (10, 11), np.zeros((0, 3, 4)))
    out.append((g_empty, np.ones((9, 8, 7))))
    return out


def _check(outs, refs, what):
    for i, (o, r) in enumerate(zip(outs, refs)):
        assert o.dtype == r.dtype and torch.equal(o, r), f"{what}: problem {i}"


@pytest.mark.parametrize("dt", [torch.float32, torch.bfloat16])
def test_batch_plans_replay_like_batched_calls(pn, dt):
    _say(f"batch plans, 17 problems, {dt}")
    probs = _problems(pn)
    xs = [(torch.from_numpy(v.reshape(g.vol_shape)).float().to(dt).cuda(), g) for g, v in probs]
    ys = [(y.clone(), g) for y, (_, g) in zip(pn.forward_batched(xs), xs)]
    plans = {"forward": pn.BatchPlan("forward", xs), "adjoint": pn.BatchPlan("adjoint", ys),
             "backproject": pn.BatchPlan("backproject", ys, out_dtype=torch.float32)}
    eager = {"forward": lambda: pn.forward_batched(xs), "adjoint": lambda: pn.adjoint_batched(ys),
             "backproject": lambda: pn.backproject_batched(ys, out_dtype=torch.float32)}
    for rep in range(3):
        if rep:
            # new input contents, same buffers
            for x, _ in xs:
                x.mul_(0.75).add_(0.01)
            for y, _ in ys:
                y.mul_(1.5)
            pn.adjoint(pn.forward(xs[0][0], xs[0][1]), xs[0][1])  # eager work on the same plans
            torch.cuda.synchronize()
        for name, plan in plans.items():
            outs = plan.run()
            refs = eager[name]()
            torch.cuda.synchronize()
            _check(outs, refs, f"{name} replay {rep}")
    for plan in plans.values():
        plan.close()


def test_batch_plan_survives_cache_release(pn):
    _say("batch plan across pn_release_caches")
    probs = _problems(pn)[:5]
    xs = [(torch.from_numpy(v.reshape(g.vol_shape)).float().cuda(), g) for g, v in probs]
    plan = pn.BatchPlan("forward", xs)
    ref = [o.clone() for o in plan.run()]
    torch.cuda.synchronize()
    pn.release_caches()
    _check(plan.run(), ref, "after release")
    torch.cuda.synchronize()
    plan.close()
    pn.release_caches()
    _check(pn.forward_batched(xs), ref, "after close")


def test_batch_plan_32_problem_list(pn):
    _say("batch plans on the 32-problem uneven list")
    pairs = []
    for p in W.batched_problem_list():
        n = p["vol_shape"]
        draws = W.perturbation_draws(p["perturb_seed"], p["n_views"]) if p["trajectory"] == "perturbed" else None
        g = pn.cone_geometry(n, p["vol_spacing"], p["det_shape"], p["det_spacing"], p["n_views"], p["sid"],
                             p["sdd"], p["angular_range"], p["trajectory"], p["pitch"], draws)
        vol = W.ellipsoid_phantom_3d(p["phantom_seed"], n, p["vol_spacing"], p["n_ellipsoids"])[0]
        pairs.append((torch.from_numpy(vol).float().cuda(), g))
    fplan = pn.BatchPlan("forward", pairs)
    ys = [(y, g) for y, (_, g) in zip(fplan.run(), pairs)]
    torch.cuda.synchronize()
    _check([y for y, _ in ys], pn.forward_batched(pairs), "forward")
    aplan = pn.BatchPlan("adjoint", ys)
    outs = aplan.run()
    torch.cuda.synchronize()
    _check(outs, pn.adjoint_batched(ys), "adjoint")
    aplan.close()
    fplan.close()


def test_batch_plan_errors(pn):
    with pytest.raises(ValueError):
        pn.BatchPlan("forward", [])
    with pytest.raises(ValueError):
        pn.BatchPlan("transpose", [(torch.zeros(4, 4, 4, device="cuda"), None)])
    g = pn.cone_geometry((8, 8, 8), (1.0,) * 3, (10, 10), (1.0, 1.0), 4, 400.0, 650.0)
    with pytest.raises(ValueError):  # wrong input shape
        pn.BatchPlan("forward", [(torch.zeros(8, 8, 9, device="cuda"), g)])
