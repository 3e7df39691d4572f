"""Autotuner (PN_AUTOTUNE=1, PN_TUNE_CACHE=<file>): the adjoint's block
shape, the forward's views per workgroup and the back-projection's block
depth.

The switches are read once per process, so the tuned runs happen in a child
process.  Each tuned operator must agree with the oracle as any other
variant does, each choice must be written to the cache file, and a second
process must take them from the file without timing again.
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import math, sys
sys.path.insert(0, {root!r})
import numpy as np, torch
import oracle as O, workloads as W
import paper_2511_08427_amd as pn
shp, sp, det, ds = (36, 44, 40), (0.5, 0.5, 0.5), (37, 45), (1.0, 1.0)
g = pn.cone_geometry(shp, sp, det, ds, 30, 750.0, 1200.0)
go = O.circular_cone(shp, sp, det, ds, 30, 2 * math.pi, 750.0, 1200.0)
q = O.forward(W.ellipsoid_phantom_3d(3, shp, sp)[0], go)
ref = O.adjoint(q, go)
x = torch.from_numpy(W.ellipsoid_phantom_3d(3, shp, sp)[0]).float().cuda()
y = pn.forward(x, g)                                      # tunes the forward
assert torch.equal(y, pn.forward(x, g))
e_f = np.linalg.norm(y.double().cpu().numpy() - q) / np.linalg.norm(q)
assert e_f <= 1e-5, e_f
qd = torch.from_numpy(q).float().cuda()
at = pn.adjoint(qd, g)                                    # tunes (first call of the plan)
at2 = pn.adjoint(qd, g)                                   # uses the choice
err = np.linalg.norm(at.double().cpu().numpy() - ref) / np.linalg.norm(ref)
assert err <= 1e-5, err
assert torch.equal(at, at2)
bp = pn.backproject(qd, g)                                # tunes the back-projection
assert torch.equal(bp, pn.backproject(qd, g))
e_b = np.linalg.norm(bp.double().cpu().numpy() - O.backproject(q, go)) / np.linalg.norm(O.backproject(q, go))
assert e_b <= 1e-5, e_b
print("OK", e_f, err, e_b, flush=True)
"""


def _child(tmp_path, cache):
    env = dict(os.environ, PN_AUTOTUNE="1", PN_TUNE_CACHE=str(cache))
    script = tmp_path / "child.py"
    script.write_text(CHILD.format(root=ROOT))
    r = subprocess.run([sys.executable, str(script)], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK" in r.stdout


def test_autotune_choice_and_cache(tmp_path):
    cache = tmp_path / "tune.txt"
    _child(tmp_path, cache)
    lines = sorted(cache.read_text().splitlines())
    assert len(lines) == 3, lines
    for op, line in zip(("adj", "bp", "fwd"), lines):
        assert line.startswith(op + " 36 44 40 37 45 30 1 "), line
    _child(tmp_path, cache)  # the second process reads the choices
    assert len(cache.read_text().splitlines()) == 3
