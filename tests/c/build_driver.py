"""Compile the plain host program that drives the C-ABI (fit_from_c) next
to this file, linked against the package's libktf.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_1605_05508_amd")
EXE = os.path.join(HERE, "fit_from_c")


def build(verbose=False) -> str:
    cmd = ["hipcc", "-O2", "-std=c++17", "--offload-arch=gfx950", os.path.join(HERE, "fit_from_c.cpp"),
           "-o", EXE + ".tmp", "-L" + PKG, "-lktf", "-Wl,-rpath,$ORIGIN/../../paper_1605_05508_amd"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(EXE + ".tmp", EXE)
    if verbose:
        print("built", EXE)
    return EXE


if __name__ == "__main__":
    build(verbose=True)
