"""Build libcm.so (HIP kernels for gfx950 + C++ host runtime) in-tree with hipcc."""
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libcm.so")

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             # packed FP32 (v_pk_*_f32) stays off: plain scalar FP32 only
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-ffp-contract=fast", "-munsafe-fp-atomics"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off"]


def sources():
    hip = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    cpp = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".cpp"))
    return hip, cpp


def _stale(src: str, obj: str) -> bool:
    """An object is stale when it is older than its source or any header."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    heads = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".h", ".cuh"))]
    heads.append(os.path.join(HERE, "..", "include", "cm.h"))
    return any(os.path.getmtime(x) > t for x in [src] + heads)


def build(verbose: bool = False, jobs: int = 8, incremental: bool = False) -> str:
    """Compile every source (incremental=True: only objects older than their
    source or any header) and link libcm.so."""
    hip, cpp = sources()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    t0 = time.time()
    for src in hip + cpp:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        if incremental and not _stale(src, obj):
            continue
        if src.endswith(".hip"):
            cmd = ["hipcc", "-c", "-x", "hip", src, "-o", obj, "-I", CSRC] + HIP_FLAGS
        else:
            cmd = ["hipcc", "-c", "-x", "c++", src, "-o", obj, "-I", CSRC, "-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"] + HOST_FLAGS
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = False
    for src, p in procs:
        out = p.communicate()[0].decode()
        lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if p.returncode != 0:
            failed = True
            sys.stderr.write(f"--- {src}\n" + "\n".join(lines) + "\n")
        elif verbose and lines:
            sys.stderr.write(f"--- {src}\n" + "\n".join(lines) + "\n")
    if failed:
        raise RuntimeError("libcm build failed")
    tmp = OUT + ".tmp"
    cmd = ["hipcc", "-shared", "-o", tmp] + objs + ["--offload-arch=gfx950", "-lpthread"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("libcm link failed:\n" + r.stdout.decode())
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT} in {time.time() - t0:.1f}s")
    return OUT


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
