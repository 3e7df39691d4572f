"""GPU parity of the sampler-interpolation forward projector
(pn_forward_sampled, through the C ABI) against the FP64 oracle (paper
Sec. 2.1, interpolation: texture sampling versus interpolation written in
the kernel).

* FP32 weights (weight_bits = 0): the same operator A as pn_forward, so the
  bar is the forward's: rel-L2 <= 1e-5 for FP32 storage, <= 1e-2 for 16-bit
  storage, on the parity cases of the staged projector (2-D fan, ragged
  cone, anisotropic cone, helical, a skewed parallel beam) and on sampled
  rays of the full 256^3 x 360 cone workload.  Both sources (the bordered
  copies and the caller's volume) do the same FP32 arithmetic on the same
  taps (zeros outside the grid either way), so they agree bit for bit.

* Rounded weights (weight_bits = B): the oracle's sampler variant rounds
  each in-plane weight to a multiple of 2^-B.  That operator is
  discontinuous: where the exact crossing lies within the kernel's FP32
  position error d of a rounding tie, the two sides may round differently
  and a sample moves by 2^-B |v1 - v0|.  Two bars:
  - a tie-free geometry (parallel beams with dyadic slopes, every crossing
    fraction at least 0.1 2^-B from a tie, checked here in FP64) leaves no
    such sample, so it is held to the FP32 bar;
  - on general geometry a fraction ~2 d 2^B of the samples may flip, while
    the rounding itself moves every sample by up to 2^-(B+1) |v1 - v0|, so
    the GPU-to-oracle distance is ~sqrt(24 d 2^B) of the rounding effect
    (~0.2 for B = 8 and d ~ 5e-6 at these sizes); it must stay below half
    of it, and the GPU's own rounding effect must match the oracle's
    within 20%.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
import test_gpu_parity as P
import workloads as W

pytestmark = pytest.mark.gpu
TOL32 = 1e-5
TOL16 = 1e-2


def _say(msg):
    print(f"[gpu-sampler] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pn():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2511_08427_amd as pn

    return pn


rel, cpu, gpu = P.rel, P.cpu, P.gpu

CASES = ["fan2d_ragged", "cone3d_ragged", "cone3d_anisotropic", "cone3d_helical", "cone3d_parallel_beam",
         "parallel2d_long_x"]


@pytest.mark.parametrize("name", CASES)
def test_sampler_fp32_weights_match_oracle(pn, name):
    _say(f"{name}: sampler, FP32 weights")
    gp, go, vols = P.make_case(pn, name)
    x = gpu(np.stack(vols))
    ref = np.stack([O.forward(v, go) for v in vols])
    yb = pn.forward_sampled(x, gp, "bordered")
    yv = pn.forward_sampled(x, gp, "direct")
    torch.cuda.synchronize()
    assert rel(cpu(yb), ref) <= TOL32, rel(cpu(yb), ref)
    assert torch.equal(yb, yv)
    # the staged projector computes the same operator
    assert rel(cpu(yb), cpu(pn.forward(x, gp))) <= TOL32


@pytest.mark.parametrize("dt", [torch.bfloat16, torch.float16])
def test_sampler_16bit_storage(pn, dt):
    _say(f"cone3d_ragged: sampler, {dt} storage")
    gp, go, vols = P.make_case(pn, "cone3d_ragged")
    x = gpu(np.stack(vols), dt)
    ref = np.stack([O.forward(v, go) for v in vols])
    for src in ("bordered", "direct"):
        y = pn.forward_sampled(x, gp, src)
        assert y.dtype == dt
        assert rel(cpu(y), ref) <= TOL16
    y32 = pn.forward_sampled(x, gp, "direct", out_dtype=torch.float32)
    # FP32 output of a 16-bit volume: the oracle of the rounded volume
    ref_r = np.stack([O.forward(v, go) for v in cpu(x)])
    assert rel(cpu(y32), ref_r) <= TOL32


def _tie_free_case(pn):
    """Parallel beams whose rays have dyadic slopes (1/4, 1/2) in index
    space and whose detector pixels sit at index offsets 0.1 + 0.75 k, so
    every crossing fraction is 0.1 + (multiple of 1/16)."""
    shp = (20, 24, 28)  # z, y, x; unit spacing, centred
    det = (24, 28)
    o = -0.5 * (np.array([shp[2], shp[1], shp[0]]) - 1.0)  # x, y, z of voxel (0, 0, 0)
    dirs = [(1.0, 0.25, 0.0), (1.0, -0.5, 0.25), (0.25, 1.0, 0.5), (-0.5, 0.25, 1.0), (1.0, 0.0, -0.25)]
    Pp, Po = [], []
    for d in dirs:
        d = np.array(d)
        a = int(np.argmax(np.abs(d)))
        f, s = [i for i in range(3) if i != a]
        eu, ev = np.zeros(3), np.zeros(3)
        eu[f], ev[s] = 0.75, 0.75
        base = np.zeros(3)
        base[f] = base[s] = 0.1
        # pixel (c, r) at index point base + c eu + r ev of plane a = 0
        C = o + base + 0.5 * (det[1] - 1) * eu + 0.5 * (det[0] - 1) * ev
        Pp.append((d, C, eu, ev))
        Po.append(O.parallel3d_matrix(d, C, eu, ev, det))
    d, C, eu, ev = (np.stack(v) for v in zip(*Pp))
    gp = pn.Geometry(3, "parallel", shp, (1.0, 1.0, 1.0), det, pn.parallel3d_matrices(d, C, eu, ev, det))
    go = O.cone_geometry(shp, (1.0, 1.0, 1.0), det, (1.0, 1.0), np.stack(Po), parallel=True)
    # every crossing of every ray, in FP64 index space: fractions away from ties
    fr = []
    for dd, bb in zip(dirs, Pp):
        dd = np.array(dd)
        a = int(np.argmax(np.abs(dd)))
        for r in range(det[0]):
            for c in range(det[1]):
                X = bb[1] - o + (c - 0.5 * (det[1] - 1)) * bb[2] + (r - 0.5 * (det[0] - 1)) * bb[3]
                m = np.arange([shp[2], shp[1], shp[0]][a], dtype=float)
                pts = X[None, :] + ((m - X[a]) / dd[a])[:, None] * dd[None, :]
                fr.append(np.delete(pts, a, axis=1).ravel())
    fr = np.concatenate(fr)
    return gp, go, fr


@pytest.mark.parametrize("bits", [4, 8])
def test_rounded_weights_tie_free_geometry(pn, bits):
    _say(f"tie-free parallel beams, weight_bits {bits}")
    gp, go, fr = _tie_free_case(pn)
    t = (fr - np.floor(fr)) * 2.0 ** bits
    assert np.abs(t - np.floor(t) - 0.5).min() >= 0.099  # no crossing near a rounding tie
    rng = np.random.default_rng(31)
    vols = rng.random((2,) + gp.vol_shape)
    x = gpu(vols)
    ref_q = np.stack([O.forward(v, go, weight_bits=bits) for v in vols])
    ref = np.stack([O.forward(v, go) for v in vols])
    for src in ("bordered", "direct"):
        y = cpu(pn.forward_sampled(x, gp, src, weight_bits=bits))
        assert rel(y, ref_q) <= TOL32, (src, rel(y, ref_q))
        assert rel(y, ref) > 10 * TOL32  # the rounding is there
    y0 = cpu(pn.forward_sampled(x, gp, "bordered"))
    assert rel(y0, ref) <= TOL32


def test_rounded_weights_exact_ties_round_upward(pn):
    """Rays along +x through index rows (j + 3/16, k + 5/16): every crossing
    is exactly on a tie of the 2^-3 lattice, which rounds upward (weights
    2/8 and 3/8); the expected values are plain sums of the volume's rows."""
    _say("exact rounding ties, weight_bits 3")
    shape, det = (6, 7, 8), (6, 7)
    d, C, eu, ev = [1.0, 0, 0], [0, 3 / 16, 5 / 16], [0, 1.0, 0], [0, 0, 1.0]
    gp = pn.Geometry(3, "parallel", shape, (1.0, 1.0, 1.0), det, pn.parallel3d_matrices(
        np.array([d]), np.array([C]), np.array([eu]), np.array([ev]), det))
    go = O.cone_geometry(shape, (1.0, 1.0, 1.0), det, (1.0, 1.0), O.parallel3d_matrix(d, C, eu, ev, det)[None],
                         parallel=True)
    vol = np.random.default_rng(18).random(shape)
    pad = np.pad(vol, ((0, 1), (0, 1), (0, 0))).sum(axis=2)
    wy, wz = 2 / 8, 3 / 8
    expect = ((1 - wy) * (1 - wz) * pad[:-1, :-1] + wy * (1 - wz) * pad[:-1, 1:] + (1 - wy) * wz * pad[1:, :-1]
              + wy * wz * pad[1:, 1:])
    assert np.abs(O.forward(vol, go, weight_bits=3)[0] - expect).max() < 1e-12
    for src in ("bordered", "direct"):
        y = cpu(pn.forward_sampled(gpu(vol), gp, src, weight_bits=3))[0]
        assert np.abs(y - expect).max() <= 1e-5 * np.abs(expect).max(), src


@pytest.mark.parametrize("name,bits", [("cone3d_ragged", 8), ("cone3d_helical", 8), ("fan2d_ragged", 6),
                                       ("cone3d_anisotropic", 4)])
def test_rounded_weights_general_geometry(pn, name, bits):
    _say(f"{name}: weight_bits {bits}")
    gp, go, vols = P.make_case(pn, name)
    rng = np.random.default_rng(32)
    vols = [0.5 * v + 0.5 * rng.random(v.shape) for v in vols]  # edges everywhere
    x = gpu(np.stack(vols))
    ref = np.stack([O.forward(v, go) for v in vols])
    ref_q = np.stack([O.forward(v, go, weight_bits=bits) for v in vols])
    yb = pn.forward_sampled(x, gp, "bordered", weight_bits=bits)
    yv = pn.forward_sampled(x, gp, "direct", weight_bits=bits)
    assert torch.equal(yb, yv)
    y = cpu(yb)
    effect = rel(ref_q, ref)
    assert effect > 10 * TOL32
    assert rel(y, ref_q) <= 0.5 * effect, (rel(y, ref_q), effect)
    assert abs(rel(y, ref) / effect - 1.0) <= 0.2
    _say(f"{name}: B={bits} rounding error vs A {rel(y, ref):.3e} (oracle {effect:.3e}), "
         f"GPU vs rounded oracle {rel(y, ref_q):.3e}")


def test_sampler_full_size_cone256_sampled(pn):
    cfg = W.CONFIGS["cone3d_256"]
    shp, sp, det, ds = cfg["vol_shape"], cfg["vol_spacing"], cfg["det_shape"], cfg["det_spacing"]
    gp = pn.cone_geometry(shp, sp, det, ds, cfg["n_views"], cfg["sid"], cfg["sdd"])
    go = O.circular_cone(shp, sp, det, ds, cfg["n_views"], cfg["angular_range"], cfg["sid"], cfg["sdd"])
    vol = W.ellipsoid_phantom_3d(cfg["seeds"][0], shp, sp, cfg["n_ellipsoids"])[0]
    x = gpu(vol)
    rng = np.random.default_rng(124)
    n = 3000
    view, row, col = rng.integers(0, 360, n), rng.integers(0, 512, n), rng.integers(0, 512, n)
    ref = O.forward_rays(vol, go, view, row, col)
    for src in ("bordered", "direct"):
        _say(f"full-size cone 256^3 x 360: sampler ({src})")
        y = pn.forward_sampled(x, gp, src).cpu().numpy()
        assert rel(y[view, row, col], ref) <= TOL32
        mid = np.arange(512)
        refm = O.forward_rays(vol, go, np.full(512, 91), np.full(512, 256), mid)
        assert rel(y[91, 256], refm) <= TOL32
    _say("full-size cone 256^3 x 360: sampler, weight_bits 8")
    yq = pn.forward_sampled(x, gp, "bordered", weight_bits=8).cpu().numpy()
    ref_q = O.forward_rays(vol, go, view, row, col, weight_bits=8)
    # on this smooth phantom the rounding moves the rays by ~4e-5 (rel-L2);
    # positions up to 256 make the FP32 position error d larger than in the
    # small cases, so only the size of the effect is compared here: the
    # flips add ~sqrt(24 d 2^B) <~ 0.4 of it in quadrature (<= 8%)
    effect = rel(ref_q, ref)
    got = rel(yq[view, row, col], ref)
    assert abs(got / effect - 1.0) <= 0.2, (got, effect)
    _say(f"cone 256^3, B=8: rounding error vs A {got:.3e} (oracle {effect:.3e}), "
         f"GPU vs rounded oracle {rel(yq[view, row, col], ref_q):.3e}")


def test_sampler_layer_and_gradient(pn):
    _say("ConeProjection3D(interp='sampler'): values and gradient")
    gp, go, vols = P.make_case(pn, "cone3d_anisotropic")
    x = gpu(np.stack(vols)).requires_grad_(True)
    for interp, src in (("sampler", "bordered"), ("sampler-direct", "direct")):
        layer = pn.ConeProjection3D(gp, interp=interp, weight_bits=8)
        y = layer(x)
        assert torch.equal(y.detach(), pn.forward_sampled(x.detach(), gp, src, weight_bits=8))
        g = torch.rand_like(y)
        (y * g).sum().backward()
        assert torch.equal(x.grad, pn.adjoint(g, gp))
        x.grad = None


def test_sampler_edge_cases_and_errors(pn):
    _say("sampler edge cases")
    shp = (8, 8, 8)
    g = pn.cone_geometry(shp, (1.0, 1.0, 1.0), (6, 6), (1.0, 1.0), 5, 100.0, 160.0, vol_origin=(200.0, 0.0, 0.0))
    for src in ("bordered", "direct"):
        y = pn.forward_sampled(torch.ones((1,) + shp, device="cuda"), g, src, weight_bits=3)
        assert float(y.abs().max()) == 0.0
    g0 = pn.Geometry(3, "cone", shp, (1.0,) * 3, (6, 6), np.zeros((0, 3, 4)))
    assert pn.forward_sampled(torch.ones(shp, device="cuda"), g0).shape == g0.sino_shape()
    assert pn.forward_sampled(torch.ones((0,) + shp, device="cuda"), g).shape[0] == 0
    g1 = pn.cone_geometry((1, 1, 1), (1.0, 1.0, 1.0), (1, 1), (1.0, 1.0), 4, 50.0, 80.0)
    go1 = O.circular_cone((1, 1, 1), (1.0, 1.0, 1.0), (1, 1), (1.0, 1.0), 4, 2 * math.pi, 50.0, 80.0)
    v = np.full((1, 1, 1), 2.5)
    for src in ("bordered", "direct"):
        assert rel(cpu(pn.forward_sampled(gpu(v), g1, src)), O.forward(v, go1)) <= TOL32
    with pytest.raises(ValueError):
        pn.forward_sampled(torch.ones(shp, device="cuda"), g, "texture")
    for bad in (-1, 17):
        with pytest.raises(pn.PnError):
            pn.forward_sampled(torch.ones(shp, device="cuda"), g, "direct", weight_bits=bad)


# ------------------------------------------------ sampler back-projection --


def _sino_case(pn, name):
    gp, go, vols = P.make_case(pn, name)
    q = np.stack([O.forward(v, go) for v in vols]).astype(np.float32).astype(np.float64)
    return gp, go, q


@pytest.mark.parametrize("name", CASES)
def test_bp_sampler_fp32_weights_match_oracle(pn, name):
    _say(f"{name}: sampler back-projection, FP32 weights")
    gp, go, q = _sino_case(pn, name)
    y = gpu(q)
    ref = np.stack([O.backproject(qq, go) for qq in q])
    bb = pn.backproject_sampled(y, gp, "bordered")
    bd = pn.backproject_sampled(y, gp, "direct")
    torch.cuda.synchronize()
    assert rel(cpu(bb), ref) <= TOL32, rel(cpu(bb), ref)
    assert torch.equal(bb, bd)
    assert rel(cpu(bb), cpu(pn.backproject(y, gp))) <= TOL32


@pytest.mark.parametrize("dt", [torch.bfloat16, torch.float16])
def test_bp_sampler_16bit_storage(pn, dt):
    _say(f"cone3d_ragged: sampler back-projection, {dt} storage")
    gp, go, q = _sino_case(pn, "cone3d_ragged")
    y = gpu(q, dt)
    ref_r = np.stack([O.backproject(qq, go) for qq in cpu(y)])
    for src in ("bordered", "direct"):
        b = pn.backproject_sampled(y, gp, src, out_dtype=torch.float32)
        assert rel(cpu(b), ref_r) <= TOL32
    b16 = pn.backproject_sampled(y, gp, "bordered")
    assert b16.dtype == dt and rel(cpu(b16), ref_r) <= TOL16


def test_bp_rounded_weights_exact_ties_round_upward(pn):
    """Rays along +x onto a panel shifted by (3/16, 5/16) pixel: every
    voxel projects exactly onto ties of the 2^-3 lattice (fractions 13/16
    and 11/16), which round up to 7/8 and 6/8."""
    _say("sampler back-projection, exact rounding ties")
    shape, det = (6, 7, 8), (6, 7)
    d, C, eu, ev = [1.0, 0, 0], [0, 3 / 16, 5 / 16], [0, 1.0, 0], [0, 0, 1.0]
    gp = pn.Geometry(3, "parallel", shape, (1.0, 1.0, 1.0), det, pn.parallel3d_matrices(
        np.array([d]), np.array([C]), np.array([eu]), np.array([ev]), det))
    img = np.random.default_rng(20).random(det)
    pad = np.pad(img, ((1, 0), (1, 0)))
    for bits, (wu, wv) in ((3, (7 / 8, 6 / 8)), (0, (13 / 16, 11 / 16))):
        col = (1 - wu) * pad[:, :-1] + wu * pad[:, 1:]
        expect = np.broadcast_to(((1 - wv) * col[:-1, :] + wv * col[1:, :])[:, :, None], shape)
        for src in ("bordered", "direct"):
            got = cpu(pn.backproject_sampled(gpu(img[None]), gp, src, weight_bits=bits))
            assert np.abs(got - expect).max() <= 1e-5 * np.abs(expect).max(), (bits, src)


@pytest.mark.parametrize("name,bits", [("cone3d_ragged", 8), ("fan2d_ragged", 6), ("cone3d_anisotropic", 4)])
def test_bp_rounded_weights_general_geometry(pn, name, bits):
    """The flip bound of the module docstring, for detector positions U/W."""
    _say(f"{name}: sampler back-projection, weight_bits {bits}")
    gp, go, _ = _sino_case(pn, name)
    rng = np.random.default_rng(33)
    q = rng.random((1,) + gp.sino_shape())
    ref = O.backproject(q[0], go)
    ref_q = O.backproject(q[0], go, weight_bits=bits)
    bb = pn.backproject_sampled(gpu(q), gp, "bordered", weight_bits=bits)
    assert torch.equal(bb, pn.backproject_sampled(gpu(q), gp, "direct", weight_bits=bits))
    y = cpu(bb)[0]
    effect = rel(ref_q, ref)
    assert effect > 10 * TOL32
    assert rel(y, ref_q) <= 0.5 * effect, (rel(y, ref_q), effect)
    assert abs(rel(y, ref) / effect - 1.0) <= 0.2
    _say(f"{name}: BP B={bits} rounding error vs B {rel(y, ref):.3e} (oracle {effect:.3e}), "
         f"GPU vs rounded oracle {rel(y, ref_q):.3e}")


def test_bp_sampler_full_size_cone256_sampled(pn):
    cfg = W.CONFIGS["cone3d_256"]
    shp, sp, det, ds = cfg["vol_shape"], cfg["vol_spacing"], cfg["det_shape"], cfg["det_spacing"]
    gp = pn.cone_geometry(shp, sp, det, ds, cfg["n_views"], cfg["sid"], cfg["sdd"])
    go = O.circular_cone(shp, sp, det, ds, cfg["n_views"], cfg["angular_range"], cfg["sid"], cfg["sdd"])
    vol = W.ellipsoid_phantom_3d(cfg["seeds"][0], shp, sp, cfg["n_ellipsoids"])[0]
    y = pn.forward(gpu(vol), gp)
    yc = y.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(125)
    i, j, k = rng.integers(0, 256, 1500), rng.integers(0, 256, 1500), rng.integers(0, 256, 1500)
    ref = O.backproject_voxels(yc, go, i, j, k)
    for src in ("bordered", "direct"):
        _say(f"full-size cone 256^3 x 360: sampler back-projection ({src})")
        b = pn.backproject_sampled(y, gp, src).cpu().numpy()
        assert rel(b[k, j, i], ref) <= TOL32


def test_bp_sampler_layer_and_gradient(pn):
    _say("ConeBackProjection3D(interp='sampler'): values and gradient")
    gp, go, q = _sino_case(pn, "cone3d_anisotropic")
    y = gpu(q).requires_grad_(True)
    for interp, src in (("sampler", "bordered"), ("sampler-direct", "direct")):
        layer = pn.ConeBackProjection3D(gp, interp=interp, weight_bits=8)
        x = layer(y)
        assert torch.equal(x.detach(), pn.backproject_sampled(y.detach(), gp, src, weight_bits=8))
        g = torch.rand_like(x)
        (x * g).sum().backward()
        # the splat adds with float atomics: equal up to FP32 rounding
        assert rel(cpu(y.grad), cpu(pn.splat(g, gp))) <= 1e-6
        y.grad = None


def test_bp_sampler_edge_cases_and_errors(pn):
    _say("sampler back-projection edge cases")
    shp = (8, 8, 8)
    g0 = pn.Geometry(3, "cone", shp, (1.0,) * 3, (6, 6), np.zeros((0, 3, 4)))
    for src in ("bordered", "direct"):
        z = pn.backproject_sampled(torch.zeros((1,) + g0.sino_shape(), device="cuda"), g0, src)
        assert z.shape == (1,) + shp and float(z.abs().max()) == 0.0
    g = pn.cone_geometry(shp, (1.0, 1.0, 1.0), (6, 6), (1.0, 1.0), 5, 100.0, 160.0)
    assert pn.backproject_sampled(torch.ones((0,) + g.sino_shape(), device="cuda"), g).shape[0] == 0
    g1 = pn.cone_geometry((1, 1, 1), (1.0, 1.0, 1.0), (1, 1), (1.0, 1.0), 4, 50.0, 80.0)
    go1 = O.circular_cone((1, 1, 1), (1.0, 1.0, 1.0), (1, 1), (1.0, 1.0), 4, 2 * math.pi, 50.0, 80.0)
    s1 = np.full((4, 1, 1), 1.5)
    for src in ("bordered", "direct"):
        assert rel(cpu(pn.backproject_sampled(gpu(s1), g1, src)), O.backproject(s1, go1)) <= TOL32
    with pytest.raises(ValueError):
        pn.backproject_sampled(torch.ones(g.sino_shape(), device="cuda"), g, "texture")
    for bad in (-1, 17):
        with pytest.raises(pn.PnError):
            pn.backproject_sampled(torch.ones(g.sino_shape(), device="cuda"), g, "direct", weight_bits=bad)
