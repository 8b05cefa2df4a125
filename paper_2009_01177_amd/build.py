"""Build the HIP library in-tree: paper_2009_01177_amd/libtor_hip.so (gfx950).

Usage: python -m paper_2009_01177_amd.build [--force]
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtor_hip.so")
ARCH = os.environ.get("TOR_OFFLOAD_ARCH", "gfx950")

# -ffp-contract=off: the error-free transforms must not be fused; wanted
# fusions are written as explicit fma().  Packed FP32 ops are disabled.
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=" + ARCH,
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def deps():
    return sources() + sorted(glob.glob(os.path.join(CSRC, "*.h*"))) + [os.path.join(ROOT, "include", "tor.h")]


def up_to_date() -> bool:
    if not os.path.exists(LIB):
        return False
    t = os.path.getmtime(LIB)
    return all(os.path.getmtime(p) <= t for p in deps())


OBJ_DIR = os.path.join(HERE, "_build")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.run(cmd, capture_output=True, text=True)


PHASE_LIB = os.path.join(HERE, "libtor_hip_phase.so")


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every source to an object (in parallel, one hipcc per
    source: each object carries its own gfx950 code), then link the shared
    library.  The Schur kernels are compiled a second time with their
    per-phase clocks (TOR_PHASE_CLOCKS) and linked with the same other
    objects into libtor_hip_phase.so, which tor_debug_phase_clocks reads
    (load it with TOR_LIBRARY)."""
    if not force and up_to_date() and os.path.exists(PHASE_LIB):
        return LIB
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    cflags = [f for f in FLAGS if f != "-shared"]
    inc = ["-I", os.path.join(ROOT, "include")]
    jobs = []
    for src in sources():
        obj = os.path.join(OBJ_DIR, os.path.basename(src) + ".o")
        jobs.append((obj, [hipcc] + cflags + inc + ["-c", src, "-o", obj]))
    schur = os.path.join(CSRC, "tor_schur.hip")
    phase_obj = os.path.join(OBJ_DIR, "tor_schur_phase.o")
    jobs.append((phase_obj, [hipcc] + cflags + ["-DTOR_PHASE_CLOCKS"] + inc + ["-c", schur, "-o", phase_obj]))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda j: _run(j[1], verbose), jobs))
    for (obj, cmd), r in zip(jobs, results):
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed (%d) on %s" % (r.returncode, cmd[-3]))
    main_objs = [o for o, _ in jobs if o != phase_obj]
    phase_objs = [phase_obj] + [o for o in main_objs if not o.endswith("tor_schur.hip.o")]
    for out, objs in ((LIB, main_objs), (PHASE_LIB, phase_objs)):
        tmp = out + ".tmp%d" % os.getpid()
        r = _run([hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs, verbose)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc link failed (%d)" % r.returncode)
        os.replace(tmp, out)
    build_c_client(verbose)
    return LIB


C_CLIENT = os.path.join(ROOT, "tests", "c_client", "tor_client")


def build_c_client(verbose: bool = False) -> str:
    """The plain C client of the ABI that the tests run (gcc, no Python or
    PyTorch): linked against the in-tree libtor_hip.so, found at run time
    relative to the binary."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    src = C_CLIENT + ".c"
    tmp = C_CLIENT + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
           "-I", os.path.join(ROOT, "include"), src, "-L", HERE, "-ltor_hip", "-L", os.path.join(rocm, "lib"),
           "-lamdhip64", "-Wl,-rpath,$ORIGIN/../../paper_2009_01177_amd", "-Wl,-rpath," + os.path.join(rocm, "lib"),
           "-o", tmp]
    r = _run(cmd, verbose)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("gcc failed (%d) on %s" % (r.returncode, src))
    os.replace(tmp, C_CLIENT)
    return C_CLIENT


if __name__ == "__main__":
    build(force=True, verbose=True)
    print(LIB)
    print(PHASE_LIB)
