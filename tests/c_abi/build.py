"""Builds the plain C consumer of the libclue ABI (test infrastructure).

gcc compiles it as host C against include/clue.h and the HIP runtime's C
API, and links it to the in-tree libclue.so by a relative rpath."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "clue_c_consumer.c")
OUT = os.path.join(HERE, "clue_c_consumer")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), SRC, "-o", OUT + ".tmp",
           "-L", os.path.join(ROOT, "paper_2001_09761_amd"), "-l:libclue.so",
           "-Wl,-rpath,$ORIGIN/../../paper_2001_09761_amd", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"gcc failed ({r.returncode}):\n{r.stderr}")
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
