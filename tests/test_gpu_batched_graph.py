"""Batched work lists and graph capture on the GPU (through the C ABI).

* A batched call launches one kernel per operator for up to 12 problems,
  ordered by cost; problems of the same geometry, 2-D and 3-D problems and
  problems without views go to separate work lists.  Every output must be
  bitwise equal to the single-problem call, which the parity tests tie to
  the oracle.
* The library's calls are stream-ordered and allocate nothing once a plan
  exists, so they can be captured in a graph; each replay (with eager work
  and synchronisation between replays) must equal the eager result.
"""
import math
import sys

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-batched] {msg}", flush=True)
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
        out.append((g, W.ellipse_phantom_2d(s, (40 + 7 * s, 33), (0.6, 0.6))[0][None]))
    g_empty = pn.Geometry(3, "cone", (9, 8, 7), (1.0,) * 3, (10, 11), np.zeros((0, 3, 4)))
    out.append((g_empty, np.ones((9, 8, 7))))
    return out


def test_batched_work_lists_equal_single(pn):
    _say("batched: 17 problems, repeated geometry, 2-D/3-D, no views")
    probs = _problems(pn)
    xs = [(torch.from_numpy(v.reshape(g.vol_shape)).float().cuda(), g) for g, v in probs]
    singles = [pn.forward(x, g) for x, g in xs]
    outs = pn.forward_batched(xs)
    for i, (o, s) in enumerate(zip(outs, singles)):
        assert torch.equal(o, s), f"forward problem {i}"
    sp = [(s, g) for s, (_, g) in zip(singles, xs)]
    for i, (o, (s, g)) in enumerate(zip(pn.adjoint_batched(sp), sp)):
        assert torch.equal(o, pn.adjoint(s, g)), f"adjoint problem {i}"
    for i, (o, (s, g)) in enumerate(zip(pn.backproject_batched(sp), sp)):
        assert torch.equal(o, pn.backproject(s, g)), f"backproject problem {i}"


def test_batched_16bit_outputs_equal_single(pn):
    _say("batched: bf16 storage")
    probs = _problems(pn)[:5]
    xs = [(torch.from_numpy(v.reshape(g.vol_shape)).to(torch.bfloat16).cuda(), g) for g, v in probs]
    singles = [pn.forward(x, g) for x, g in xs]
    for o, s in zip(pn.forward_batched(xs), singles):
        assert o.dtype == torch.bfloat16 and torch.equal(o, s)
    sp = [(s, g) for s, (_, g) in zip(singles, xs)]
    for o, (s, g) in zip(pn.adjoint_batched(sp), sp):
        assert torch.equal(o, pn.adjoint(s, g))


def test_graph_capture_replays_match_eager(pn):
    _say("graph capture: forward + adjoint + batched forward")
    g = pn.cone_geometry((24, 28, 26), (0.8, 0.8, 0.8), (30, 34), (1.2, 1.2), 24, 400.0, 650.0)
    vol = W.ellipsoid_phantom_3d(31, (24, 28, 26), (0.8, 0.8, 0.8), 6)[0]
    x = torch.from_numpy(vol).float().cuda()
    probs = [(x, g), (x[:, ::2].contiguous(), pn.cone_geometry((24, 14, 26), (0.8, 1.6, 0.8), (30, 34), (1.2, 1.2),
                                                              18, 400.0, 650.0))]
    # eager results (also create the plans: plan set-up allocates and copies)
    y_ref = pn.forward(x, g)
    a_ref = pn.adjoint(y_ref, g)
    b_ref = pn.forward_batched(probs)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up on the capture stream
        pn.forward(x, g)
        pn.forward_batched(probs)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        y = pn.forward(x, g)
        a = pn.adjoint(y, g)
        b = pn.forward_batched(probs)
    for rep in range(4):
        # eager work between replays touches the same plans and buffers
        pn.adjoint(pn.forward(2.0 * x, g), g)
        torch.cuda.synchronize()
        y.zero_()
        a.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref), f"replay {rep}: forward"
        assert torch.equal(a, a_ref), f"replay {rep}: adjoint"
        for o, r in zip(b, b_ref):
            assert torch.equal(o, r), f"replay {rep}: batched forward"
