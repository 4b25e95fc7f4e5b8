"""Build librw.so for gfx950 in-tree with hipcc (translation units in parallel)."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
UNITS = ["rw_api.hip", "rw_doe_mixed.hip", "rw_doe_fp32.hip", "rw_doe_fp64.hip", "rw_dft.hip"]
OUT = os.path.join(HERE, "librw.so")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
BUILD_DIR = os.path.join(HERE, "_build")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    return r.returncode, r.stdout + r.stderr


def _stale(obj, unit):
    """An object is stale if it is missing or older than its unit or any header."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    srcs = [os.path.join(CSRC, unit)] + [os.path.join(CSRC, h) for h in os.listdir(CSRC)
                                         if h.endswith(".h")]
    srcs.append(os.path.join(os.path.dirname(HERE), "include", "rw.h"))
    return any(os.path.getmtime(x) > t for x in srcs)


def build(verbose=False, jobs=None, incremental=False):
    """Compile every unit (incremental=True: only units older than their sources)
    and link librw.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs, cmds = [], []
    for u in UNITS:
        o = os.path.join(BUILD_DIR, u.replace(".hip", ".o"))
        objs.append(o)
        if incremental and not _stale(o, u):
            continue
        cmds.append([hipcc] + FLAGS + ["-c", "-o", o, os.path.join(CSRC, u)])
    jobs = jobs or max(1, min(len(cmds), os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_run, cmds))
    for (rc, out), cmd in zip(results, cmds):
        if rc != 0:
            sys.stderr.write(out)
            raise RuntimeError("hipcc failed: " + " ".join(cmd[-1:]))
        if verbose:
            sys.stderr.write(out)
    tmp = OUT + ".tmp"
    rc, out = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    if rc != 0:
        sys.stderr.write(out)
        raise RuntimeError("hipcc failed to link librw.so")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))
