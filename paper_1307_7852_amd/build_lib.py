"""Builds libknng.so (gfx950) from csrc/ with hipcc, in-tree."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libknng.so")
OBJ = os.path.join(os.path.dirname(HERE), "_build")
SOURCES = ["knng_api.cpp", "divide.hip", "leaf.hip", "graph.hip", "mlp.hip", "rows.hip"]
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
FLAGS = ["-I", INCLUDE, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-mcode-object-version=5", "-Wall", "-Wno-unused-result",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


HEADERS = [os.path.join(SRC, "knng_internal.h"), os.path.join(SRC, "knng_dev.h"),
           os.path.join(os.path.dirname(HERE), "include", "knng.h")]


def _stale(src, obj):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in [os.path.join(SRC, src)] + HEADERS)


def _compile(src, force=True):
    obj = os.path.join(OBJ, src + ".o")
    if not force and not _stale(src, obj):
        return src, 0, "", obj
    cmd = ["hipcc", "-x", "hip", "-c", os.path.join(SRC, src), "-o", obj] + FLAGS
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    return src, r.returncode, err, obj


def build(verbose=True, force=True):
    """Compiles every source (force) or only stale ones, then links."""
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=4) as ex:
        res = list(ex.map(lambda s: _compile(s, force), SOURCES))
    ok = True
    for src, rc, err, _ in res:
        if err.strip() and verbose:
            print(f"[{src}]\n{err}", file=sys.stderr)
        ok &= rc == 0
    if not ok:
        raise RuntimeError("HIP compilation failed")
    tmp = OUT + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + [r[3] for r in res]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(force="--incremental" not in sys.argv))
