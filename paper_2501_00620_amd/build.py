"""Build liblbm.so in-tree for gfx950 with hipcc.

The library is linked from separately compiled units, built in parallel: the C ABI and the
two-pass, projected and diagnostic kernels (lbm_api.hip), the serving runtime (lbm_server.hip),
the allocation-free entry point (lbm_noalloc.hip), and the fused sweeps once per storage type
(lbm_sweep.hip with -DLBM_SWEEP_S=0..3).  Objects go to paper_2501_00620_amd/_build/.

Every HIP translation unit is compiled with packed FP32 instructions disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``) and with ``-ffp-contract=on``: a multiply
and an add are fused only where one source expression holds both, so each kernel that inlines
the per-site arithmetic rounds it the same way (a served lattice steps bit for bit as it would
alone, whatever the surrounding kernel).
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblbm.so")
OBJDIR = os.path.join(HERE, "_build")
# (source, extra defines, object name)
UNITS = [("lbm_api.hip", [], "lbm_api.o"), ("lbm_server.hip", [], "lbm_server.o"),
         ("lbm_noalloc.hip", [], "lbm_noalloc.o")] + \
        [("lbm_sweep.hip", ["-DLBM_SWEEP_S=%d" % s], "lbm_sweep_s%d.o" % s) for s in range(4)]
SOURCES = sorted({u[0] for u in UNITS})
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=on",
            "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                    if "packed-fp32-ops" not in l or "error" in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + out)
    if verbose and out.strip():
        print(out, file=sys.stderr)


def build(verbose=False, jobs=None):
    """Compile all HIP units (in parallel) and link paper_2501_00620_amd/liblbm.so; returns its path."""
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(len(UNITS), max(1, os.cpu_count() or 1))

    def compile_unit(u):
        src, defs, obj = u
        out = os.path.join(OBJDIR, obj)
        _run([HIPCC] + flags() + defs + ["-c", os.path.join(CSRC, src), "-o", out], verbose)
        return out

    with ThreadPoolExecutor(max_workers=jobs) as pool:
        objs = list(pool.map(compile_unit, UNITS))
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
