"""Build the HIP library ``libpdhcg.so`` (gfx950) in-tree with hipcc."""
from __future__ import annotations

import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpdhcg.so")
ARCH = os.environ.get("PDHCG_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")) + glob.glob(os.path.join(HERE, "csrc", "*.cpp")))


def build(verbose: bool = False) -> str:
    """Compile every HIP/C++ source of the library into libpdhcg.so (always
    recompiles): one object per source, compiled in parallel (each hipcc runs
    its host and device passes), then linked.  Returns the library path."""
    import shutil
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    inc = ["-I", os.path.join(ROOT, "include")]
    obj_dir = tempfile.mkdtemp(prefix="pdhcg_build_")
    try:
        objs = [os.path.join(obj_dir, os.path.basename(src) + ".o") for src in sources()]
        compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]

        def compile_one(pair):
            src, obj = pair
            cmd = ["hipcc", *compile_flags, *inc, "-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd))
            return subprocess.run(cmd, capture_output=True, text=True)

        workers = max(1, min(len(objs), os.cpu_count() or 1, 8))
        with ThreadPoolExecutor(max_workers=workers) as pool:
            results = list(pool.map(compile_one, zip(sources(), objs)))
        for src, res in zip(sources(), results):
            if res.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n" + res.stdout + res.stderr)
        tmp = LIB + f".tmp{os.getpid()}"
        cmd = ["hipcc", *HIPCC_FLAGS, "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd))
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("hipcc link failed:\n" + res.stdout + res.stderr)
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(obj_dir, ignore_errors=True)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    hdrs = glob.glob(os.path.join(HERE, "csrc", "*.hpp")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    return any(os.path.getmtime(f) > t for f in sources() + hdrs)


if __name__ == "__main__":
    print(build(verbose=True))
