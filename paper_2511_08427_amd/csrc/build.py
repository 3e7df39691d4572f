"""Builds libpyronn_mi.so (HIP kernels for gfx950 + the C-ABI host library).

Run from anywhere:  python paper_2511_08427_amd/csrc/build.py
"""
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libpyronn_mi.so")
SOURCES = ["pn_kernels.hip", "pn_sampler.hip", "pn_signal.hip", "pn_host.cpp", "pn_geometry.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # keep FP32 arithmetic out of packed (v_pk_*_f32) instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-command-line-argument",
    "-I" + os.path.join(ROOT, "include"),
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)


def build(verbose=False):
    """Compiles every source to an object in parallel, then links."""
    tmp = LIB + ".tmp"
    objdir = tempfile.mkdtemp(prefix="pyronn_mi_build_")
    try:
        compile_flags = [f for f in FLAGS if f != "-shared"]
        procs = []
        objs = []
        for src in SOURCES:
            obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
            objs.append(obj)
            procs.append((src, _run([HIPCC] + compile_flags + ["-c", os.path.join(HERE, src), "-o", obj], verbose)))
        for src, pr in procs:
            out, err = pr.communicate()
            if pr.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n" + err)
            err = "\n".join(l for l in err.splitlines() if "packed-fp32-ops" not in l and l.strip())
            if err and verbose:
                print(err, file=sys.stderr)
        pr = _run([HIPCC] + FLAGS + objs + ["-o", tmp], verbose)
        out, err = pr.communicate()
        if pr.returncode != 0:
            raise RuntimeError("link failed:\n" + err)
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
