"""Build libmriadmm.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2006_14080_amd.build                  # compile every source
    python -m paper_2006_14080_amd.build --asm DIR        # also write the gfx950 assembly to DIR

Every HIP source is compiled with packed-FP32 instruction selection disabled
(``-packed-fp32-ops``); the host pass warns that it does not know the
feature, which is harmless.
"""
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmriadmm.so")
SOURCES = ["api.hip", "plan.hip", "server.hip", "nudft.hip", "solver.hip", "nufft.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; a ROCm toolchain is required to build libmriadmm")


def flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-I", CSRC]


def build(verbose: bool = False, asm: str = "") -> str:
    """Compile every source into libmriadmm.so; with `asm` (a directory) also
    write each source's device assembly there."""
    cc = hipcc()
    tmp = tempfile.mkdtemp(prefix="mriadmm_build_")
    try:
        objs = []
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            cmd = [cc, *flags(), "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            res = subprocess.run(cmd, stderr=subprocess.PIPE, text=True)
            errs = "\n".join(l for l in res.stderr.splitlines()
                             if "packed-fp32-ops' is not a recognized feature" not in l)
            if res.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{errs}")
            if verbose and errs.strip():
                print(errs, file=sys.stderr)
            objs.append(obj)
            if asm:
                out = os.path.join(asm, src + ".s")
                os.makedirs(asm, exist_ok=True)
                subprocess.run([cc, *flags(), "--cuda-device-only", "-S",
                                os.path.join(CSRC, src), "-o", out], check=True,
                               stderr=subprocess.PIPE)
        tmp_lib = LIB + ".tmp"
        subprocess.run([cc, "-shared", f"--offload-arch={ARCH}", *objs, "-o", tmp_lib], check=True)
        os.replace(tmp_lib, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    asm_dir = sys.argv[sys.argv.index("--asm") + 1] if "--asm" in sys.argv else ""
    print(build(verbose="-v" in sys.argv, asm=asm_dir))
