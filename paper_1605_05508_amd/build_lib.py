"""Compile libktf.so (HIP for gfx950) in place, next to this file.

Every HIP translation unit under csrc/ (*.hip) is compiled with hipcc for
gfx950, the host-only ones (*.cpp, no HIP) with g++, and all are linked into
one shared library exporting the C-ABI of include/ktf.h.  Packed FP32
instructions are disabled for all device code.
"""
import concurrent.futures as cf
import glob
import json
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libktf.so")
ARCH = os.environ.get("KTF_OFFLOAD_ARCH", "gfx950")

# A kernel's by-value argument structure is copied to private memory and
# read from there unless the optimiser can prove the copy redundant, which
# it stops trying past a number of uses (300 by default): the building's
# score kernel reads its arguments in more places than that and would keep
# a 1.3 KB copy per lane in scratch.  The limit is raised for every file;
# below it the code is the same.
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-instcombine-max-copied-from-constant-users=4096",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-command-line-argument"]


HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall"]
# the compiler's per-kernel resource report (registers, scratch, occupancy),
# kept in _build/resources.json for the test that guards against kernels
# falling into scratch memory
REMARKS = ["-Rpass-analysis=kernel-resource-usage"]


def _resources(text):
    """Kernel name -> {vgpr, sgpr, scratch, occupancy} from the remarks."""
    out, cur = {}, None
    for line in text.splitlines():
        m = re.search(r"remark:\s+Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        for key, pat in (("vgpr", r"remark:\s+VGPRs: (\d+)"), ("sgpr", r"remark:\s+TotalSGPRs: (\d+)"),
                         ("scratch", r"ScratchSize \[bytes/lane\]: (\d+)"),
                         ("occupancy", r"Occupancy \[waves/SIMD\]: (\d+)")):
            m = re.search(pat, line)
            if m and cur is not None:
                cur[key] = int(m.group(1))
    return out


def _compile(src):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    if src.endswith(".cpp"):
        cmd = ["g++", *HOST_FLAGS, "-c", src, "-o", obj]
    else:
        cmd = ["hipcc", *FLAGS, *REMARKS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, (_resources(r.stderr) if src.endswith(".hip") else {})


def build(verbose=False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = min(len(srcs), max(1, (os.cpu_count() or 4) // 2), 8)
    with cf.ThreadPoolExecutor(jobs) as ex:
        done = list(ex.map(_compile, srcs))
    objs = [o for o, _ in done]
    res = {}
    for _, r in done:
        res.update(r)
    with open(os.path.join(OBJ, "resources.json"), "w") as f:
        json.dump({"arch": ARCH, "kernels": res}, f, indent=0, sort_keys=True)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
