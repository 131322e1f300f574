"""Build the stfem shared library (HIP kernels for gfx950 + host C++) in-tree.

Usage: python -m paper_2504_07269_amd.build   (or build() from Python)
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libstfem.so")
SOURCES = ["kernels.hip", "fdm.cpp", "eig.cpp", "assembly.cpp"]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the stfem library needs ROCm's hipcc")


def build(verbose=False):
    """Compile every source for gfx950 into paper_2504_07269_amd/libstfem.so."""
    objs = []
    flags = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-pthread",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(HERE, "..", "include"), "-Wno-unused-command-line-argument"]
    builddir = os.path.join(HERE, "_build")
    os.makedirs(builddir, exist_ok=True)
    procs = []
    for src in SOURCES:
        obj = os.path.join(builddir, os.path.splitext(src)[0] + ".o")
        lang = (["-x", "hip"] if src.endswith(".hip")
                else ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"])
        cmd = [hipcc()] + flags + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    for src, cmd, p in procs:
        out, _ = p.communicate()
        if verbose or p.returncode != 0:
            sys.stderr.write(out)
        if p.returncode != 0:
            raise RuntimeError("compilation of %s failed:\n%s" % (src, " ".join(cmd)))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("link failed: " + " ".join(cmd))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
