"""Build libgsraster.so (the HIP library behind include/gsraster.h) for gfx950.

Each translation unit is compiled with hipcc to a position-independent object
and the objects are linked into one shared library in the package directory.
The projection and binning units are compiled without floating-point
contraction, which keeps radii, tile rectangles and depth keys bit-exact.

    python -m paper_2409_06765_amd.build
"""
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libgsraster.so")
ARCH = os.environ.get("GSR_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", os.path.join(ROOT, "include"),
          "-I", CSRC, "-Wall", "-Wno-unused-function",
          # packed FP32 instructions are disabled for every device compilation
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
UNITS = {
    "abi.hip": [],
    "project.hip": ["-ffp-contract=off"],
    "intersect.hip": ["-ffp-contract=off"],
    "raster_fwd.hip": [],
    "raster_bwd.hip": ["-munsafe-fp-atomics"],
    "train.hip": [],
}


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False, units=None):
    os.makedirs(OUT_DIR, exist_ok=True)
    hipcc = _hipcc()
    procs = []
    objs = []
    for src, extra in UNITS.items():
        obj = os.path.join(OUT_DIR, src.replace(".hip", ".o"))
        objs.append(obj)
        if units is not None and src not in units and os.path.exists(obj):
            continue
        cmd = [hipcc, "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + extra
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, pr in procs:
        out, _ = pr.communicate()
        text = out.decode(errors="replace")
        # the host pass does not know the device-only feature flag; that warning is expected
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if pr.returncode != 0:
            failed.append(src)
            print("\n".join(lines), file=sys.stderr)
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        print(r.stdout.decode(errors="replace"), file=sys.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    t0 = time.time()
    path = build(verbose="-v" in sys.argv)
    print(f"built {path} in {time.time() - t0:.1f}s")
