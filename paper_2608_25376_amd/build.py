"""Build ``libuavq.so`` (host code + HIP kernels for gfx950) in-tree with hipcc."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libuavq.so")
SOURCES = ["uavq_host.cpp", "uavq_kernels.hip", "uavq_sweep_chunk.hip", "uavq_sweep_chunk_wide.hip", "uavq_sweep_chunk_big.hip",
           "uavq_sweep_big.hip", "uavq_refresh.hip",
           "uavq_warm.hip", "uavq_pt.hip"]
HEADERS = ["uavq_internal.h", "uavq_kargs.h", "uavq_device.h", "uavq_factored.h", "uavq_chunk.h", os.path.join("..", "..", "include", "uavq.h")]
ARCH = os.environ.get("UAVQ_OFFLOAD_ARCH", "gfx950")


def _hipcc():
    h = shutil.which("hipcc")
    if h:
        return h
    if os.path.exists("/opt/rocm/bin/hipcc"):
        return "/opt/rocm/bin/hipcc"
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES] + [os.path.normpath(os.path.join(CSRC, h)) for h in HEADERS]


def stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in sources())


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and not stale():
        return LIB
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]
    # Packed FP32 instructions stay off in all device code.
    dev = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    # The chunked walk's per-chunk loops must unroll fully for five and six
    # chunks (m <= 384), or the lane's arrays move to scratch memory; the other
    # kernels of the file compile to the same code with or without this.
    per_file = {"uavq_kernels.hip": ["-mllvm", "-pragma-unroll-threshold=200000"],
                "uavq_sweep_chunk.hip": ["-mllvm", "-pragma-unroll-threshold=200000"],
                "uavq_sweep_chunk_wide.hip": ["-mllvm", "-pragma-unroll-threshold=200000"],
                "uavq_sweep_chunk_big.hip": ["-mllvm", "-pragma-unroll-threshold=200000"],
                "uavq_sweep_big.hip": ["-mllvm", "-pragma-unroll-threshold=200000"]}
    objs, cmds = [], []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(objdir, os.path.splitext(s)[0] + ".o")
        if s.endswith(".hip"):
            cmd = [hipcc, "-x", "hip"] + dev + common + per_file.get(s, []) + ["-c", src, "-o", obj]
        else:
            cmd = [hipcc, "-x", "c++"] + common + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        cmds.append(cmd)
        objs.append(obj)
    # the sources compile independently: one compiler process each
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(len(cmds), 8)) as ex:
        for r in list(ex.map(lambda c: subprocess.run(c), cmds)):
            if r.returncode != 0:
                raise subprocess.CalledProcessError(r.returncode, r.args)
    tmp = LIB + ".tmp"
    subprocess.run([hipcc, "-shared", "--offload-arch=" + ARCH, "-o", tmp] + objs, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose="-v" in sys.argv))
