"""The oracle's pins catch plausible mistakes (CPU only).

Each case plants one mistake in a copy of the oracle -- the C ray loops
compiled from an edited copy of oracle.c into a temporary directory, or a
Python function of the oracle package replaced for the duration of the
check -- and requires at least one pin of tests/test_oracle_pins.py to
fail.  The shipped oracle is never modified.
"""
import concurrent.futures
import inspect
import os
import subprocess
import sys

import pytest

import test_oracle_pins as PINS

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, text in oracle.c, replacement): each text occurs exactly once
C_MUTANTS = [
    ("bilinear weights swapped", "w[cnt] = (tb ? wb : 1.0 - wb) * (tc", "w[cnt] = (tb ? 1.0 - wb : wb) * (tc"),
    ("ray length per plane dropped", "double ds = g->s[a] * dnorm / fabs(ray->d[a]);", "double ds = g->s[a];"),
    ("sign of v in the cone ray", "ray->d[i] = Mi[3 * i] * u + Mi[3 * i + 1] * v + Mi[3 * i + 2];",
     "ray->d[i] = Mi[3 * i] * u - Mi[3 * i + 1] * v + Mi[3 * i + 2];"),
    ("origin sign", "xi0[i] = (ray->x0[i] - g->o[i]) / g->s[i];", "xi0[i] = (ray->x0[i] + g->o[i]) / g->s[i];"),
    ("BP distance weight inverted", "double W0 = p[11];\n            double wt = (W0 / W) * (W0 / W);",
     "double W0 = p[11];\n            double wt = (W / W0) * (W / W0);"),
    ("u and v swapped in BP", "detector_sample(img, nv, nu, U / W, V / W, 3, wbits)",
     "detector_sample(img, nv, nu, V / W, U / W, 3, wbits)"),
    ("fan direction component", "ray->d[1] = i10 * u + i11;", "ray->d[1] = i10 * u - i11;"),
    ("adjoint reads a mirrored column", "double q = sino[(k * nv + r) * nu + c];",
     "double q = sino[(k * nv + r) * nu + (nu - 1 - c)];"),
    ("3-D parallel base point sign", "ray->x0[i] = ca * a[i] + cb * b[i];", "ray->x0[i] = ca * a[i] - cb * b[i];"),
    ("2-D parallel base point sign", "ray->x0[0] = a * t;", "ray->x0[0] = -a * t;"),
    ("splat distance weight dropped", "const double wt = (W0 / W) * (W0 / W) * val;", "const double wt = val;"),
    ("splat column taps swapped", "img[r * nu + c] += wt * fvw * (tu ? wu : 1.0 - wu);",
     "img[r * nu + c] += wt * fvw * (tu ? 1.0 - wu : wu);"),
    ("rounded weights truncated instead of rounded", "if (t - q >= 0.5) q += 1.0;", "if (t - q > 1.0) q += 1.0;"),
    ("rounded weights with one bit fewer", "double sc = ldexp(1.0, wbits);", "double sc = ldexp(1.0, wbits - 1);"),
    ("second in-plane weight not rounded", "double fc = floor(pc), wc = tap_weight(pc - fc, wbits);",
     "double fc = floor(pc), wc = pc - fc;"),
    ("ties rounded downward", "if (t - q >= 0.5) q += 1.0;", "if (t - q > 0.5) q += 1.0;"),
    ("back-projection row weight not rounded", "double fv = floor(v), wv = tap_weight(v - fv, wbits);",
     "double fv = floor(v), wv = v - fv;"),
]


def _build_mutant(tmpdir, i, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, old
    path = os.path.join(tmpdir, f"mut{i}.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    lib = os.path.join(tmpdir, f"libmut{i}.so")
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", path, "-o", lib, "-lm"], check=True)
    return lib


def _pins_fail(lib):
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(HERE, "test_oracle_pins.py")], cwd=ROOT, env=env, capture_output=True, text=True)
    return r.returncode == 1, r.stdout[-400:]


def test_every_c_mutant_fails_a_pin(tmp_path):
    libs = [_build_mutant(str(tmp_path), i, old, new) for i, (_, old, new) in enumerate(C_MUTANTS)]
    with concurrent.futures.ThreadPoolExecutor(4) as ex:
        results = list(ex.map(_pins_fail, libs))
    survivors = [C_MUTANTS[i][0] for i, (failed, _) in enumerate(results) if not failed]
    assert not survivors, f"mutants that pass every pin: {survivors}"


def _mutated(fn, old, new):
    """A copy of oracle function `fn` with `old` replaced by `new` in its
    source, defined in the oracle module's namespace."""
    src = inspect.getsource(fn)
    assert src.count(old) == 1, old
    ns = {}
    exec(compile(src.replace(old, new), f"<mutant {fn.__name__}>", "exec"), fn.__globals__, ns)
    return ns[fn.__name__]


def _fails(pin, O):
    name, kw = (pin, {}) if isinstance(pin, str) else pin
    try:
        getattr(PINS, name)(O, **kw)
    except AssertionError:
        return True
    return False


@pytest.mark.parametrize("name,fn,old,new,pins", [
    ("cosine weight dropped", "cosine_weights", "out[k] = (1.0 / (np.linalg.norm(Q[-1]) * np.linalg.norm(d, axis=0)))",
     "out[k] = np.ones(d.shape[1])",
     ["test_cosine_weights_are_cosines_to_the_detector_normal", "test_fan_fdk_short_source_distance_reconstructs_disk",
      "test_cone_fdk_short_source_distance_reconstructs_ball"]),
    ("cosine weight squared", "cosine_weights", "out[k] = (1.0 / (np.linalg.norm(Q[-1]) * np.linalg.norm(d, axis=0)))",
     "out[k] = ((1.0 / (np.linalg.norm(Q[-1]) * np.linalg.norm(d, axis=0))) ** 2)",
     ["test_cosine_weights_are_cosines_to_the_detector_normal", "test_fan_fdk_short_source_distance_reconstructs_disk",
      "test_cone_fdk_short_source_distance_reconstructs_ball"]),
    ("cosine weight inverted", "cosine_weights", "out[k] = (1.0 / (np.linalg.norm(Q[-1]) * np.linalg.norm(d, axis=0)))",
     "out[k] = (np.linalg.norm(Q[-1]) * np.linalg.norm(d, axis=0))",
     ["test_cosine_weights_are_cosines_to_the_detector_normal", "test_fan_fdk_short_source_distance_reconstructs_disk",
      "test_cone_fdk_short_source_distance_reconstructs_ball"]),
    ("Ram-Lak centre tap", "ramp_kernel", "g[0] = 0.25", "g[0] = 0.5",
     [("test_filter_kernel_frequency_response", {"kind": "ram-lak"}), "test_fbp_parallel_reconstructs_disk"]),
    ("FBP angular factor", "fbp_filter", "(math.pi / nviews)", "(2 * math.pi / nviews)",
     ["test_fbp_parallel_reconstructs_disk", "test_fan_fdk_short_source_distance_reconstructs_disk"]),
    ("helical feed inverted magnification", "trajectory_vectors", "h = pitch * det_shape[0] * det_spacing[0] * sid / sdd",
     "h = pitch * det_shape[0] * det_spacing[0] * sdd / sid", ["test_helical_trajectory_has_the_requested_pitch"]),
    ("sinusoid amplitude", "trajectory_vectors", "amp = vol_shape[0] * vol_spacing[0] / 4.0",
     "amp = vol_shape[0] * vol_spacing[0] / 2.0", ["test_sinusoidal_trajectory_amplitude_and_frequency"]),
    ("sinusoid frequency", "trajectory_vectors", "dz = amp * np.sin(2 * beta)", "dz = amp * np.sin(beta)",
     ["test_sinusoidal_trajectory_amplitude_and_frequency"]),
    ("perturbed panel sheared", "trajectory_vectors", "ev = dv * (-sp * uh + cp * vh)", "ev = dv * (sp * uh + cp * vh)",
     ["test_perturbed_trajectory_statistics"]),
])
def test_python_mutant_fails_a_pin(oracle_lib, monkeypatch, name, fn, old, new, pins):
    O = oracle_lib
    monkeypatch.setattr(O, fn, _mutated(getattr(O, fn), old, new))
    failed = [p for p in pins if _fails(p, O)]
    assert failed, f"mutant '{name}' passes {pins}"
