"""PyTorch-facing operators (PYRO-NN update, Sec. 2.4 "PyTorch Integration").

Torch supplies device memory and the current stream; every operator is one
call into the native library, which runs the gfx950 kernels:

  forward(vol, geom)      A     -> pn_forward
  forward_sampled(...)    A     -> pn_forward_sampled (sampler interpolation)
  backproject_sampled(...)      -> pn_backproject_sampled (sampler interpolation)
  adjoint(sino, geom)     A^T   -> pn_adjoint
  backproject(sino, geom)       -> pn_backproject (voxel-driven, (W0/W)^2)
  splat(vol, geom)        B^T   -> pn_splat (transpose of the back-projection)

``Projection`` is the autograd pair: its backward is the exact adjoint
kernel, so gradients of any loss of A x are analytic (Sec. 2);
``BackProjection``'s backward is the splat projector, the exact transpose
of the voxel-driven back-projection.  The layer
classes mirror the paper's naming (Listing 1).
"""
from __future__ import annotations

import ctypes

import torch

from . import _native as N
from .geometry import Geometry

_DT = {torch.float32: N.PN_F32, torch.bfloat16: N.PN_BF16, torch.float16: N.PN_F16}


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _prep(t, name, tail):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU (the operators have no CPU implementation)")
    if t.dtype not in _DT:
        raise TypeError(f"{name}: unsupported dtype {t.dtype} (float32, bfloat16, float16)")
    batched = t.dim() == len(tail) + 1
    if not batched and t.dim() != len(tail):
        raise ValueError(f"{name}: expected shape [B,]{list(tail)}, got {list(t.shape)}")
    if tuple(t.shape[-len(tail):]) != tuple(tail):
        raise ValueError(f"{name}: expected trailing shape {list(tail)}, got {list(t.shape)}")
    t = t.contiguous()
    tb = t if batched else t.unsqueeze(0)
    return tb, batched


def _run(fn, where, geom: Geometry, src, src_tail, dst_tail, out_dtype):
    x, batched = _prep(src, where, src_tail)
    out_dtype = out_dtype or x.dtype
    if out_dtype not in _DT:
        raise TypeError(f"unsupported output dtype {out_dtype}")
    out = torch.empty((x.shape[0],) + tuple(dst_tail), dtype=out_dtype, device=x.device)
    with torch.cuda.device(x.device):
        rc = fn(geom.c_struct(), x.shape[0], ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                _DT[x.dtype], _DT[out_dtype], _stream(x.device))
    N.check(rc, where)
    return out if batched else out[0]


def forward(vol, geom: Geometry, out_dtype=None):
    """A vol: [B,]nz,ny,nx -> [B,]n_views,rows,cols (ray-driven Joseph)."""
    return _run(N.lib.pn_forward, "pn_forward", geom, vol, geom.vol_shape, geom.sino_shape(), out_dtype)


_SOURCES = {"bordered": 0, "direct": 1}


def forward_sampled(vol, geom: Geometry, source="bordered", weight_bits=0, out_dtype=None):
    """A vol with sampler interpolation (pn_forward_sampled): every bilinear
    tap is a separate load through the caches, from zero-bordered copies of
    the volume (``source="bordered"``, extra device memory, no bounds
    checks) or from ``vol`` itself (``"direct"``, no extra memory).
    ``weight_bits`` = B > 0 rounds the interpolation weights to multiples of
    2^-B, as fixed-function filtering hardware does; 0 keeps FP32 weights
    (then the result matches ``forward`` to FP32 rounding)."""
    if source not in _SOURCES:
        raise ValueError(f"source must be one of {sorted(_SOURCES)}")
    src, bits = _SOURCES[source], int(weight_bits)

    def fn(g, b, x, o, dti, dto, st):
        return N.lib.pn_forward_sampled(g, b, x, o, dti, dto, src, bits, st)

    return _run(fn, "pn_forward_sampled", geom, vol, geom.vol_shape, geom.sino_shape(), out_dtype)


def adjoint(sino, geom: Geometry, out_dtype=None):
    """A^T sino: [B,]n_views,rows,cols -> [B,]nz,ny,nx (exact adjoint of forward)."""
    return _run(N.lib.pn_adjoint, "pn_adjoint", geom, sino, geom.sino_shape(), geom.vol_shape, out_dtype)


def adjoint_noalloc(sino, geom: Geometry, out_dtype=None):
    """A^T sino through pn_adjoint_noalloc: the same result as ``adjoint``
    with no device allocation inside the library (its tables live in a
    fixed per-GPU scratch array; calls on one GPU must not overlap)."""
    return _run(N.lib.pn_adjoint_noalloc, "pn_adjoint_noalloc", geom, sino, geom.sino_shape(), geom.vol_shape,
                out_dtype)


def backproject(sino, geom: Geometry, out_dtype=None):
    """Voxel-driven (W0/W)^2-weighted back-projection: sino -> volume."""
    return _run(N.lib.pn_backproject, "pn_backproject", geom, sino, geom.sino_shape(), geom.vol_shape, out_dtype)


def backproject_sampled(sino, geom: Geometry, source="bordered", weight_bits=0, out_dtype=None):
    """Back-projection with sampler interpolation (pn_backproject_sampled):
    every bilinear detector tap a separate load through the caches, from a
    zero-bordered copy of the sinogram (``source="bordered"``, extra device
    memory) or from ``sino`` itself (``"direct"``: the caller's data, no
    extra memory).  ``weight_bits`` as ``forward_sampled``."""
    if source not in _SOURCES:
        raise ValueError(f"source must be one of {sorted(_SOURCES)}")
    src, bits = _SOURCES[source], int(weight_bits)

    def fn(g, b, x, o, dti, dto, st):
        return N.lib.pn_backproject_sampled(g, b, x, o, dti, dto, src, bits, st)

    return _run(fn, "pn_backproject_sampled", geom, sino, geom.sino_shape(), geom.vol_shape, out_dtype)


def splat(vol, geom: Geometry, out_dtype=None):
    """Transpose of ``backproject`` (pn_splat): every voxel's (W0/W)^2-weighted
    value spread over the bilinear taps of its projection; volume -> sino."""
    return _run(N.lib.pn_splat, "pn_splat", geom, vol, geom.vol_shape, geom.sino_shape(), out_dtype)


_FILTERS = {"ram-lak": 0, "shepp-logan": 1}


def fbp_filter(sino, geom: Geometry, kind="ram-lak", out_dtype=None):
    """Row filter of the filtered back-projection (pn_filter): cosine weights
    (fan, cone), the discrete Ram-Lak or Shepp-Logan kernel along detector
    rows, scaled by pi / n_views / (pixel pitch at the rotation axis)."""
    if kind not in _FILTERS:
        raise ValueError(f"filter kind must be one of {sorted(_FILTERS)}")
    k = _FILTERS[kind]

    def fn(g, b, x, o, dti, dto, st):
        return N.lib.pn_filter(g, b, x, o, dti, dto, k, st)

    return _run(fn, "pn_filter", geom, sino, geom.sino_shape(), geom.sino_shape(), out_dtype)


def fbp(sino, geom: Geometry, kind="ram-lak", out_dtype=None):
    """Filtered back-projection (FBP for parallel beams, FDK for fan and cone
    beams on a full orbit): the back-projection of fbp_filter(sino)."""
    return backproject(fbp_filter(sino, geom, kind, torch.float32), geom, out_dtype or sino.dtype)


def gaussian_noise_(x, mean=0.0, sigma=1.0, seed=0):
    """In place: x += mean + sigma * z, z standard normal from Philox4x64-10
    (pn_gaussian_noise); a pure function of (seed, flat index, x)."""
    if not x.is_cuda or not x.is_contiguous() or x.dtype not in _DT:
        raise ValueError("gaussian_noise_ needs a contiguous CUDA tensor of float32, bfloat16 or float16")
    with torch.cuda.device(x.device):
        rc = N.lib.pn_gaussian_noise(x.numel(), ctypes.c_void_p(x.data_ptr()), _DT[x.dtype], float(mean),
                                     float(sigma), int(seed) & (2 ** 64 - 1), _stream(x.device))
    N.check(rc, "pn_gaussian_noise")
    return x


def detector_jitter(sino, max_shift=1, seed=0):
    """A copy of sino with every detector row moved by its own random integer
    shift in -max_shift .. max_shift along the columns (pn_detector_jitter)."""
    if not sino.is_cuda or not sino.is_contiguous() or sino.dtype not in _DT or sino.dim() < 1:
        raise ValueError("detector_jitter needs a contiguous CUDA tensor of float32, bfloat16 or float16")
    out = torch.empty_like(sino)
    cols = sino.shape[-1]
    with torch.cuda.device(sino.device):
        rc = N.lib.pn_detector_jitter(sino.numel() // max(cols, 1), cols, ctypes.c_void_p(sino.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), _DT[sino.dtype], int(max_shift),
                                      int(seed) & (2 ** 64 - 1), _stream(sino.device))
    N.check(rc, "pn_detector_jitter")
    return out


def gantry_blur(sino, angle_start, angle_step, taps=3):
    """A copy of sino [B,]views,rows,cols with each projection blurred by a
    `taps`-sample line kernel turned to its acquisition angle
    angle_start + k angle_step (pn_gantry_blur)."""
    if not sino.is_cuda or not sino.is_contiguous() or sino.dtype not in _DT or sino.dim() not in (3, 4):
        raise ValueError("gantry_blur needs a contiguous CUDA [B,]views,rows,cols tensor")
    s4 = sino if sino.dim() == 4 else sino.unsqueeze(0)
    b, nv, rows, cols = s4.shape
    out = torch.empty_like(sino)
    with torch.cuda.device(sino.device):
        rc = N.lib.pn_gantry_blur(b, nv, rows, cols, ctypes.c_void_p(sino.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  _DT[sino.dtype], float(angle_start), float(angle_step), int(taps),
                                  _stream(sino.device))
    N.check(rc, "pn_gantry_blur")
    return out


def ring_artifacts_(sino, columns, gain=0.0, views=None):
    """In place: detector columns `columns` of sino [B,]views,rows,cols
    scaled by gain over the view range `views` (a (start, stop) pair, default
    all) (pn_ring_artifacts)."""
    if not sino.is_cuda or not sino.is_contiguous() or sino.dtype not in _DT or sino.dim() not in (3, 4):
        raise ValueError("ring_artifacts_ needs a contiguous CUDA [B,]views,rows,cols tensor")
    s4 = sino if sino.dim() == 4 else sino.unsqueeze(0)
    b, nv, rows, cols = s4.shape
    v0, v1 = (0, nv) if views is None else (int(views[0]), int(views[1]))
    col = (ctypes.c_int32 * max(len(columns), 1))(*[int(c) for c in columns])
    with torch.cuda.device(sino.device):
        rc = N.lib.pn_ring_artifacts(b, nv, rows, cols, ctypes.c_void_p(sino.data_ptr()), _DT[sino.dtype], col,
                                     len(columns), float(gain), v0, v1, _stream(sino.device))
    N.check(rc, "pn_ring_artifacts")
    return sino


def _batched(fn, where, pairs, src_tail_of, dst_tail_of, out_dtype):
    """pairs: list of (tensor, geometry), one problem each (no batch axis)."""
    if not pairs:
        return []
    dts = {t.dtype for t, _ in pairs}
    devs = {t.device for t, _ in pairs}
    if len(dts) != 1 or len(devs) != 1:
        raise ValueError(f"{where}: all problems must share dtype and device")
    dt = dts.pop()
    dev = devs.pop()
    out_dtype = out_dtype or dt
    probs = (N.PnProblem * len(pairs))()
    keep, outs = [], []
    for i, (t, g) in enumerate(pairs):
        x, batched = _prep(t, where, src_tail_of(g))
        if batched:
            raise ValueError(f"{where}: batched problems take one volume/sinogram each")
        o = torch.empty(dst_tail_of(g), dtype=out_dtype, device=dev)
        probs[i].geom = g.c_struct()
        probs[i].in_ = x.data_ptr()
        probs[i].out = o.data_ptr()
        keep.append(x)
        outs.append(o)
    with torch.cuda.device(dev):
        rc = fn(probs, len(pairs), _DT[dt], _DT[out_dtype], _stream(dev))
    N.check(rc, where)
    return outs


def forward_batched(pairs, out_dtype=None):
    return _batched(N.lib.pn_forward_batched, "pn_forward_batched", pairs, lambda g: g.vol_shape,
                    lambda g: g.sino_shape(), out_dtype)


def adjoint_batched(pairs, out_dtype=None):
    return _batched(N.lib.pn_adjoint_batched, "pn_adjoint_batched", pairs, lambda g: g.sino_shape(),
                    lambda g: g.vol_shape, out_dtype)


def backproject_batched(pairs, out_dtype=None):
    return _batched(N.lib.pn_backproject_batched, "pn_backproject_batched", pairs, lambda g: g.sino_shape(),
                    lambda g: g.vol_shape, out_dtype)


class BatchPlan:
    """A fixed problem set run many times (pn_batch_create / pn_batch_run):
    one launch per kernel group over all problems, replayed from a HIP graph
    the library captures.  ``op`` is "forward", "adjoint" or "backproject";
    ``pairs`` are (input tensor, geometry) with one problem each.  The
    outputs are allocated here; ``run()`` re-reads the inputs' current
    contents (change them in place, not by rebinding) and returns the
    outputs."""

    _OPS = {"forward": 0, "adjoint": 1, "backproject": 2}

    def __init__(self, op, pairs, out_dtype=None):
        if op not in self._OPS:
            raise ValueError(f"unknown operator {op!r}")
        if not pairs:
            raise ValueError("a batch plan needs at least one problem")
        fwd = op == "forward"
        src = (lambda g: g.vol_shape) if fwd else (lambda g: g.sino_shape())
        dst = (lambda g: g.sino_shape()) if fwd else (lambda g: g.vol_shape)
        dts = {t.dtype for t, _ in pairs}
        devs = {t.device for t, _ in pairs}
        if len(dts) != 1 or len(devs) != 1:
            raise ValueError("all problems must share dtype and device")
        dt, self.device = dts.pop(), devs.pop()
        out_dtype = out_dtype or dt
        probs = (N.PnProblem * len(pairs))()
        self.inputs, self.outputs, self.geometries = [], [], []
        for i, (t, g) in enumerate(pairs):
            x, batched = _prep(t, "BatchPlan", src(g))
            if batched:
                raise ValueError("batch plans take one volume/sinogram per problem")
            if x.data_ptr() != t.data_ptr():
                raise ValueError("batch plan inputs must be contiguous tensors (they are read in place)")
            o = torch.empty(dst(g), dtype=out_dtype, device=self.device)
            probs[i].geom = g.c_struct()
            probs[i].in_ = x.data_ptr()
            probs[i].out = o.data_ptr()
            self.inputs.append(x)
            self.outputs.append(o)
            self.geometries.append(g)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = N.lib.pn_batch_create(self._OPS[op], probs, len(pairs), _DT[dt], _DT[out_dtype], ctypes.byref(h))
        N.check(rc, "pn_batch_create")
        self._h = h

    def run(self):
        if self._h is None:
            raise RuntimeError("batch plan already closed")
        with torch.cuda.device(self.device):
            N.check(N.lib.pn_batch_run(self._h, _stream(self.device)), "pn_batch_run")
        return self.outputs

    def close(self):
        """Frees the graph and work lists (after waiting for the device)."""
        if getattr(self, "_h", None) is not None:
            torch.cuda.synchronize(self.device)
            N.lib.pn_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------- autograd --


_INTERP = {"staged": None, "sampler": "bordered", "sampler-direct": "direct"}


class Projection(torch.autograd.Function):
    """y = A x; dL/dx = A^T dL/dy (the adjoint kernel).

    ``interp`` picks how A interpolates: "staged" (the default, volume tiles
    staged through LDS), "sampler" or "sampler-direct" (``forward_sampled``
    from the bordered copies or from the volume itself, ``weight_bits`` as
    there).  The gradient is the exact adjoint of A with FP32 weights in
    every case; with weight_bits > 0 it is therefore the adjoint of the
    unquantised operator."""

    @staticmethod
    def forward(ctx, vol, geom, interp="staged", weight_bits=0):
        if interp not in _INTERP:
            raise ValueError(f"interp must be one of {sorted(_INTERP)}")
        ctx.geom = geom
        ctx.vol_dtype = vol.dtype
        if _INTERP[interp] is None:
            return forward(vol, geom)
        return forward_sampled(vol, geom, _INTERP[interp], weight_bits)

    @staticmethod
    def backward(ctx, grad):
        return adjoint(grad.contiguous(), ctx.geom, out_dtype=ctx.vol_dtype), None, None, None


class AdjointProjection(torch.autograd.Function):
    """x = A^T y; dL/dy = A dL/dx."""

    @staticmethod
    def forward(ctx, sino, geom):
        ctx.geom = geom
        ctx.sino_dtype = sino.dtype
        return adjoint(sino, geom)

    @staticmethod
    def backward(ctx, grad):
        return forward(grad.contiguous(), ctx.geom, out_dtype=ctx.sino_dtype), None


class BackProjection(torch.autograd.Function):
    """x = B q (voxel-driven back-projection); dL/dq = B^T dL/dx (the splat
    projector).  ``interp`` and ``weight_bits`` as ``Projection`` (the
    sampler variants are ``backproject_sampled``); the gradient is the
    transpose of B with FP32 weights in every case."""

    @staticmethod
    def forward(ctx, sino, geom, interp="staged", weight_bits=0):
        if interp not in _INTERP:
            raise ValueError(f"interp must be one of {sorted(_INTERP)}")
        ctx.geom = geom
        ctx.sino_dtype = sino.dtype
        if _INTERP[interp] is None:
            return backproject(sino, geom)
        return backproject_sampled(sino, geom, _INTERP[interp], weight_bits)

    @staticmethod
    def backward(ctx, grad):
        return splat(grad.contiguous(), ctx.geom, out_dtype=ctx.sino_dtype), None, None, None


class SplatProjection(torch.autograd.Function):
    """y = B^T x (splat projector); dL/dx = B dL/dy (the back-projection)."""

    @staticmethod
    def forward(ctx, vol, geom):
        ctx.geom = geom
        ctx.vol_dtype = vol.dtype
        return splat(vol, geom)

    @staticmethod
    def backward(ctx, grad):
        return backproject(grad.contiguous(), ctx.geom, out_dtype=ctx.vol_dtype), None


class _Layer(torch.nn.Module):
    def __init__(self, geom: Geometry):
        super().__init__()
        self.geom = geom


class _ProjLayer(_Layer):
    """A projection layer; ``interp`` and ``weight_bits`` as ``Projection``."""

    def __init__(self, geom: Geometry, interp="staged", weight_bits=0):
        super().__init__(geom)
        if interp not in _INTERP:
            raise ValueError(f"interp must be one of {sorted(_INTERP)}")
        self.interp, self.weight_bits = interp, int(weight_bits)

    def forward(self, x):
        return Projection.apply(x, self.geom, self.interp, self.weight_bits)


class ParallelProjection2D(_ProjLayer):
    pass


class FanProjection2D(_ProjLayer):
    pass


class ConeProjection3D(_ProjLayer):
    pass


class _BackProjLayer(_ProjLayer):
    """A back-projection layer; ``interp`` and ``weight_bits`` as ``Projection``."""

    def forward(self, y):
        return BackProjection.apply(y, self.geom, self.interp, self.weight_bits)


class ParallelBackProjection2D(_BackProjLayer):
    pass


class FanBackProjection2D(_BackProjLayer):
    pass


class ConeBackProjection3D(_BackProjLayer):
    pass


def unrolled_gd(x0, y, geom: Geometry, alpha: float, steps: int, checkpoint: bool = True):
    """``steps`` gradient steps x <- x - alpha A^T (A x - y) on 0.5||Ax - y||^2,
    differentiable end to end.  With ``checkpoint`` each step's activations
    are recomputed in the backward pass instead of stored."""
    import torch.utils.checkpoint as cp

    def step(x):
        return x - alpha * AdjointProjection.apply(Projection.apply(x, geom) - y, geom)

    x = x0
    for _ in range(steps):
        x = cp.checkpoint(step, x, use_reentrant=False) if checkpoint else step(x)
    return x
