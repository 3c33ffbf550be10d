"""Build libbpfa.so for gfx950 with hipcc (in-tree, next to this file)."""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_DIR = os.path.join(HERE, "_lib")
LIB_PATH = os.path.join(LIB_DIR, "libbpfa.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay disabled: the compiler must not form them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def _run(cmd):
    return subprocess.run(cmd, capture_output=True, text=True)


def build(verbose=False, extra=(), jobs=None):
    """Compile every source to an object in parallel, then link the shared library."""
    import concurrent.futures
    import tempfile
    os.makedirs(LIB_DIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    jobs = jobs or min(16, os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="bpfa_build_") as obj_dir:
        cmds, objs = [], []
        for src in sources():
            obj = os.path.join(obj_dir, os.path.basename(src) + ".o")
            objs.append(obj)
            cmds.append([hipcc, *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-c",
                         "-o", obj, src])
        with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(_run, cmds))
        for cmd, res in zip(cmds, results):
            if verbose:
                print(" ".join(cmd), flush=True)
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise RuntimeError("hipcc failed on %s" % cmd[-1])
            if verbose and res.stderr:
                sys.stderr.write(res.stderr)
        tmp = LIB_PATH + ".tmp"
        res = _run([hipcc, *HIPCC_FLAGS, *extra, "-o", tmp, *objs])
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libbpfa.so")
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
