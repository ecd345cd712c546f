"""Build libls.so (HIP, gfx950) in-tree.

Every source under csrc/ is compiled with hipcc into _build/ (in parallel)
and linked into paper_2212_11403_amd/libls.so. Packed FP32 instructions are
disabled for device code (-target-feature -packed-fp32-ops).
"""

from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libls.so")
ARCH = os.environ.get("LS_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found; libls needs ROCm's hipcc")
    return p


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _headers_mtime():
    hs = glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    return max((os.path.getmtime(h) for h in hs), default=0.0)


def _deps_mtime(dep_file: str):
    """Newest modification time of the repository files a previous compile
    read (from its make-style dependency file), or None if unknown."""
    try:
        text = open(dep_file).read().replace("\\\n", " ")
    except OSError:
        return None
    newest = 0.0
    for tok in text.split(":", 1)[-1].split():
        if tok.startswith(ROOT) or not os.path.isabs(tok):
            path = tok if os.path.isabs(tok) else os.path.join(BUILD, tok)
            if not os.path.exists(path):
                return None
            newest = max(newest, os.path.getmtime(path))
    return newest


def _compile(src: str, force: bool, keep_asm: bool):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    dep = obj + ".d"
    deps = _deps_mtime(dep)
    newest = max(os.path.getmtime(src), os.path.getmtime(__file__),
                 _headers_mtime() if deps is None else deps)
    if not force and os.path.exists(obj) and os.path.getmtime(obj) >= newest:
        return obj, 0.0, ""
    t0 = time.time()
    cmd = [hipcc()] + FLAGS + ["-MMD", "-MF", dep, "-c", src, "-o", obj + ".tmp"]
    if keep_asm and src.endswith(".hip"):
        cmd += ["-save-temps=obj"]
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=BUILD)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {os.path.basename(src)}:\n{r.stderr[-4000:]}")
    os.replace(obj + ".tmp", obj)
    # date the object by when the compile started, so that a source edited
    # while it compiled still counts as newer next time
    os.utime(obj, (t0, t0))
    noise = "\n".join(line for line in r.stderr.splitlines() if "packed-fp32-ops" not in line)
    return obj, time.time() - t0, noise


def build(force: bool = False, jobs: int | None = None, keep_asm: bool = False,
          verbose: bool = False) -> str:
    """Compile and link libls.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(_compile, s, force, keep_asm): s for s in srcs}
        for f in cf.as_completed(futs):
            obj, dt, noise = f.result()
            objs.append(obj)
            if verbose and dt:
                print(f"  compiled {os.path.basename(futs[f])} in {dt:.1f}s", flush=True)
            if verbose and noise.strip():
                print(noise, flush=True)
    tmp = LIB + f".{os.getpid()}.tmp"
    r = subprocess.run([hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp]
                       + sorted(objs), capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    t0 = time.time()
    path = build(force="--force" in sys.argv, keep_asm="--asm" in sys.argv, verbose=True)
    print(f"built {path} in {time.time() - t0:.1f}s")
