"""The allocation-free adjoint entry point (pn_adjoint_noalloc) against
pn_adjoint, through the C ABI.

Both run the same kernels with the same (default) block shape, and the
adjoint's fixed-point accumulation is deterministic, so the outputs must be
bitwise equal; they must also meet the FP32 parity bar against each other
(rel-L2 <= 1e-5), which bitwise equality implies.  Calls in a row: a cone
problem, then a smaller one (other geometry, the scratch array's tables are
replaced), then the smaller geometry again with a batch of 2 (tables re-used),
then 16-bit storage (the FP32 accumulator in the scratch array), then a 2-D
fan problem.  A problem too large for the scratch array is refused with
PN_EINVAL before anything is enqueued (its buffers are full size, so nothing
could be written out of bounds either way).
"""
import math
import sys

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-noalloc] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pn():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2511_08427_amd as pn

    return pn


def _rel(a, b):
    a, b = a.double(), b.double()
    return float((a - b).norm() / b.norm())


def _same(pn, y, g, out_dtype=None):
    ref = pn.adjoint(y, g, out_dtype=out_dtype)
    got = pn.adjoint_noalloc(y, g, out_dtype=out_dtype)
    torch.cuda.synchronize()
    assert got.dtype == ref.dtype and got.shape == ref.shape
    assert _rel(got, ref) <= 1e-5
    assert torch.equal(got, ref)


def test_noalloc_adjoint_equals_adjoint(pn):
    _say("noalloc: cone 36x44x40, 30 views")
    shp, sp, det, ds = (36, 44, 40), (0.5, 0.5, 0.5), (37, 45), (1.0, 1.0)
    g1 = pn.cone_geometry(shp, sp, det, ds, 30, 750.0, 1200.0)
    y1 = pn.forward(torch.from_numpy(W.ellipsoid_phantom_3d(3, shp, sp)[0]).float().cuda(), g1)
    _same(pn, y1, g1)
    _say("noalloc: smaller helical problem 20x22x18, 16 views")
    shp2, sp2, det2, ds2 = (20, 22, 18), (0.8, 0.8, 0.8), (26, 28), (1.2, 1.2)
    g2 = pn.cone_geometry(shp2, sp2, det2, ds2, 16, 400.0, 650.0, 2 * math.pi, "helical", 0.5)
    x2 = torch.from_numpy(W.ellipsoid_phantom_3d(32, shp2, sp2, 6)[0]).float().cuda()
    y2 = pn.forward(x2, g2)
    _same(pn, y2, g2)
    _say("noalloc: same geometry again, batch of 2")
    y2b = pn.forward(torch.stack([x2, 0.25 * x2.flip(0).contiguous()]), g2)
    _same(pn, y2b, g2)
    _say("noalloc: bf16 storage, bf16 and fp32 outputs")
    _same(pn, y2b.to(torch.bfloat16), g2)
    _same(pn, y1.to(torch.bfloat16), g1, out_dtype=torch.float32)
    _say("noalloc: 2-D fan")
    g3 = pn.fan_geometry((100, 90), (0.5, 0.5), 150, 0.5, 96, 1000.0, 1500.0)
    y3 = pn.forward(torch.from_numpy(W.ellipse_phantom_2d(2, (100, 90), (0.5, 0.5))[0]).float().cuda(), g3)
    _same(pn, y3, g3)
    _say("noalloc: back to the first geometry")
    _same(pn, 0.5 * y1, g1)


def test_noalloc_refuses_oversized_problems(pn):
    _say("noalloc: 512^3 x 720 views is refused")
    cfg = W.CONFIGS["cone3d_512"]
    g = pn.cone_geometry(cfg["vol_shape"], cfg["vol_spacing"], cfg["det_shape"], cfg["det_spacing"], cfg["n_views"],
                         cfg["sid"], cfg["sdd"])
    y = torch.zeros(g.sino_shape(), device="cuda")
    with pytest.raises(pn.PnError) as e:
        pn.adjoint_noalloc(y, g)
    assert "scratch" in str(e.value)
    # the refused call enqueued nothing and left the array usable
    shp, sp, det, ds = (16, 18, 14), (0.9, 0.9, 0.9), (22, 24), (1.3, 1.3)
    g2 = pn.cone_geometry(shp, sp, det, ds, 12, 420.0, 700.0)
    y2 = pn.forward(torch.from_numpy(W.ellipsoid_phantom_3d(33, shp, sp, 5)[0]).float().cuda(), g2)
    _same(pn, y2, g2)
