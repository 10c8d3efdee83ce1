"""Build libfdlb.so in-tree for gfx950 with hipcc.

Every HIP source is compiled with packed-FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops); objects go to _build/.  The compiler's
resource report for every kernel (registers, scratch, waves per SIMD) is kept in
_build/kernel_resources.json, and the build fails if a step kernel (or the hybrid channel's
march kernel) uses scratch memory: a
spilled or stack-held value in the velocity loop is a performance bug that no test would see.
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfdlb.so")
ARCH = os.environ.get("FDLB_OFFLOAD_ARCH", "gfx950")

COMMON = ["-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", CSRC]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


REPORT = ["-Rpass-analysis=kernel-resource-usage"]
FIELDS = {"SGPRs": "sgpr", "VGPRs": "vgpr", "AGPRs": "agpr", "ScratchSize [bytes/lane]": "scratch",
          "Occupancy [waves/SIMD]": "waves_per_simd", "LDS Size [bytes/block]": "lds"}


def parse_resources(text: str) -> dict:
    """Kernel name -> resource figures, from the compiler's kernel-resource-usage remarks."""
    out, name = {}, None
    for line in text.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            out[name] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z][^:]*?):\s+(-?\d+)\b", line)
        if name and m and m.group(1) in FIELDS:
            out[name][FIELDS[m.group(1)]] = int(m.group(2))
    return out


def _compile(src: str):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = ["hipcc", "-c", *COMMON, "-o", obj, src]
    if src.endswith(".cpp"):
        cmd = ["hipcc", "-c", "-x", "hip", *COMMON, "-o", obj, src]
    if src.endswith(".hip"):
        cmd += REPORT
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    res = parse_resources(r.stderr)
    if r.stderr.strip():
        # the host pass warns that it does not know the GPU-only feature flag, and the resource
        # remarks (with their source excerpts) go to the report file; other warnings stay visible
        lines = [l for l in r.stderr.splitlines()
                 if ("warning:" in l or "error:" in l) and "packed-fp32-ops" not in l]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")
    return obj, res


def build(jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(srcs))) as ex:
        done = list(ex.map(_compile, srcs))
    objs = [o for o, _ in done]
    res = {}
    for _, r in done:
        res.update(r)
    with open(os.path.join(BUILD, "kernel_resources.json"), "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
    spilled = sorted(k for k, v in res.items()
                     if ("step_kernel" in k or "hybrid_march" in k) and v.get("scratch", 0) > 0)
    if spilled:
        raise RuntimeError("step kernels use scratch memory (spills or a stack copy): " + ", ".join(spilled))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    build_examples()
    return LIB


EXAMPLE = os.path.join(HERE, "examples", "cavity_c")


def build_examples() -> str:
    """The C consumer of the library (plain C against include/fdlb.h, linked to libfdlb.so and
    the HIP runtime of /opt/rocm; it finds libfdlb.so one directory up through its rpath)."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    src = os.path.join(HERE, "examples", "cavity_c.c")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(HERE, "..", "include"),
           "-I", os.path.join(rocm, "include"), "-o", EXAMPLE, src, "-L", HERE, "-lfdlb",
           "-L", os.path.join(rocm, "lib"), "-lamdhip64", f"-Wl,-rpath,$ORIGIN/..", f"-Wl,-rpath,{os.path.join(rocm, 'lib')}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"example build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return EXAMPLE


if __name__ == "__main__":
    print(build())
