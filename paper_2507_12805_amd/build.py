"""Build libpmklc.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpmklc.so")
SOURCES = ["step_kernel.hip", "step_mfma.hip", "step_chip.hip", "seq_kernels.hip", "dm_op.hip", "tf_kernels.hip", "gru_train.hip",
           "api.cpp"]
# the matrix-core step kernel's instances, one object per GEMM precision,
# optimiser and workgroup width (compiled side by side)
VARIANTS = [(bf, adam, nt) for bf in (1, 0) for adam in (0, 1) for nt in (256, 512)]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    cmds, objs = [], []
    for bf, adam, nt in VARIANTS:
        name = f"launch_mfma_{'bf16' if bf else 'f32'}_{'adam' if adam else 'sgd'}_{nt}"
        obj = os.path.join(bdir, name + ".o")
        cmds.append(["hipcc", *FLAGS, f"-DPMKLC_VARIANT={name}", f"-DPMKLC_BF16={bf}", f"-DPMKLC_ADAM={adam}",
                     f"-DPMKLC_NT={nt}", "-c", os.path.join(CSRC, "step_mfma_inst.hip"), "-o", obj])
        objs.append(obj)
    for src in SOURCES:
        obj = os.path.join(bdir, src + ".o")
        lang = [] if src.endswith(".hip") else ["-x", "hip"]
        cmds.append(["hipcc", *FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # the sources compile independently: run them side by side
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
        list(ex.map(subprocess.check_call, cmds))
    tmp = LIB + f".tmp{os.getpid()}"
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
