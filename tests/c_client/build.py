"""Compile the plain-C client of the C ABI (lj_nve.c) against libmd950.so.

Host code only: gcc with the HIP runtime's C headers (which need the AMD platform macro)
and libamdhip64 for device memory; the run path of the library is relative to the
executable, so the pair travels with the repository.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
EXE = os.path.join(HERE, "lj_nve")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROCM, "include"), "-I" + os.path.join(ROOT, "include"),
           os.path.join(HERE, "lj_nve.c"), "-o", EXE + ".tmp",
           "-L" + os.path.join(ROOT, "paper_2511_22951_amd"), "-lmd950",
           "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_2511_22951_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("C client build failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(EXE + ".tmp", EXE)
    return EXE


if __name__ == "__main__":
    print(build(verbose=True))
