"""Build the gfx950 HIP library libpse.so in-tree (hipcc, explicit flags).

Every HIP source is compiled for gfx950 only; packed-FP32 instruction
selection is disabled.  Objects go to _build/, the library next to this file.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpse.so")
BUILD = os.path.join(ROOT, "_build")
SOURCES = ["capi.hip", "k_particles.hip", "k_grid.hip", "k_precond.hip", "k_full.hip", "fg_host.cpp", "params_host.cpp",
           "precond_host.cpp", "lanczos_host.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wno-unused-result", "-I" + os.path.join(ROOT, "include")]


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    procs = []
    objs = []
    for s in SOURCES:
        src = os.path.join(SRC, s)
        obj = os.path.join(BUILD, os.path.splitext(s)[0] + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if s.endswith(".cpp") else []
        cmd = [HIPCC] + FLAGS + lang + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = False
    for s, p in procs:
        out, _ = p.communicate()
        txt = out.decode(errors="replace")
        if p.returncode != 0:
            failed = True
            sys.stderr.write(f"--- {s} failed ---\n{txt}\n")
        elif verbose and txt.strip():
            sys.stderr.write(f"--- {s} ---\n{txt}\n")
    if failed:
        raise RuntimeError("HIP build failed")
    tmp = OUT + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "-shared", "-fPIC", "-pthread", "--offload-arch=gfx950", "-o", tmp] + objs)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(OUT)
