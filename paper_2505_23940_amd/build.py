"""Build libfvib.so (HIP, gfx950) in-tree with hipcc.

Each source is compiled to an object in its own hipcc process (in parallel),
then the objects are linked into one shared library.

Usage: python -m paper_2505_23940_amd.build   (or build() from Python).
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
OBJ_DIR = os.path.join(OUT_DIR, "obj")
LIB = os.path.join(OUT_DIR, "libfvib.so")

SOURCES = ["fvib_api.hip", "k_momentum.hip", "k_poisson.hip", "k_ib.hip", "k_adjoint.hip",
           "k_loss.hip", "k_fdm.hip", "k_fft.hip", "k_les.hip"]

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if verbose and (res.stdout or res.stderr):
        sys.stderr.write(res.stdout + res.stderr)
    return res


def _stale(src, obj, headers):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in [src] + headers)


def build(verbose: bool = False, jobs: int = 0, incremental: bool = False) -> str:
    """Compile every HIP source and link them into one shared library;
    returns its path.  incremental=True recompiles only sources newer than
    their objects (or any header)."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objs = [os.path.join(OBJ_DIR, os.path.splitext(s)[0] + ".o") for s in srcs]
    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    headers += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    cmds = [[hipcc] + FLAGS + inc + ["-c", os.path.join(CSRC, s), "-o", o]
            for s, o in zip(srcs, objs)
            if not incremental or _stale(os.path.join(CSRC, s), o, headers)]
    jobs = jobs or max(1, min(len(cmds), 8, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda c: _run(c, verbose), cmds))
    failed = [(c[-3], r) for c, r in zip(cmds, results) if r.returncode != 0]
    if failed:
        for s, r in failed:
            sys.stderr.write(f"---- {s}\n" + r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libfvib.so: " + ", ".join(s for s, _ in failed))
    tmp = LIB + ".tmp"
    res = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp], verbose)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libfvib.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))
