"""Compile the HIP library ``_lib/libpdg.so`` for gfx950 (in-tree).

Usage: ``python paper_1702_00169_amd/build.py`` (run by path: importing the
package itself loads the library, which may not exist yet) or ``build()``.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "libpdg.so")
SOURCES = ["pdg_host.cpp", "pdg_sweep.hip", "pdg_local.hip", "pdg_dense.hip", "pdg_fused.hip"]

# Packed-FP32 VALU forms are kept out of the generated code on purpose.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose=False, jobs=2, out=None, defines=()):
    """Compile every source and link the shared library; raises on failure.

    ``out`` and ``defines`` (e.g. ``["PDG_NONTEMPORAL=1"]``) build a variant
    library elsewhere for comparisons; the default builds ``_lib/libpdg.so``."""
    os.makedirs(LIBDIR, exist_ok=True)
    target = out or LIB
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(LIBDIR, os.path.splitext(src)[0] + ".o")
        cmd = [_hipcc()] + HIP_FLAGS + ["-D" + d for d in defines] + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    failed = False
    for cmd, proc in procs:
        out, _ = proc.communicate()
        if verbose and out:
            sys.stdout.write(out)
        if proc.returncode != 0:
            sys.stderr.write(out)
            failed = True
    if failed:
        raise RuntimeError("HIP compilation failed")
    tmp = target + ".tmp"
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout)
        raise RuntimeError("link failed")
    os.replace(tmp, target)
    for obj in objs:
        os.remove(obj)
    return target


if __name__ == "__main__":
    print(build(verbose=True))
