"""Build libbsm.so (HIP, gfx950) in-tree.

Each .hip source is compiled to an object in parallel with hipcc, then the
objects are linked into paper_1401_3733_amd/libbsm.so.  Packed-FP32
instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbsm.so")
DEV_STAMP = os.path.join(HERE, "libbsm.dev")   # present only for restricted development builds
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-Wno-unknown-warning-option"]


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))


def _stale(src: str, obj: str) -> bool:
    if not os.path.exists(obj):
        return True
    stamp = os.path.join(BUILD, "dev_dmask")
    prev = open(stamp).read() if os.path.exists(stamp) else ""
    if prev != os.environ.get("BSM_DEV_D", "").strip():
        return True
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    deps.append(os.path.join(HERE, "..", "include", "bsm.h"))
    return any(os.path.getmtime(d) > t for d in deps)


def _dmask():
    """BSM_DEV_D="3,6" (development only) compiles just those d_R."""
    v = os.environ.get("BSM_DEV_D", "").strip()
    if not v:
        return None
    return sum(1 << int(x) for x in v.split(","))


def _compile(src: str, force: bool = True) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    if not force and not _stale(src, obj):
        return obj
    mask = _dmask()
    extra = [f"-DBSM_DMASK={mask:#x}"] if mask is not None else []
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-8000:]}")
    return obj


def build(jobs: int | None = None, verbose: bool = True, force: bool = True) -> str:
    """Compile every source (force=False: only sources whose object is older
    than the source or any header) and link libbsm.so."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), srcs))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-8000:]}")
    os.replace(tmp, LIB)
    for stamp in (os.path.join(BUILD, "dev_dmask"), DEV_STAMP):
        if _dmask() is not None:
            open(stamp, "w").write(os.environ["BSM_DEV_D"])
        elif os.path.exists(stamp):
            os.remove(stamp)
    if _dmask() is not None:
        print(f"WARNING: development build, d_R restricted to {os.environ['BSM_DEV_D']}", file=sys.stderr)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(force="--incremental" not in sys.argv)
