"""Build the C client wc_solve_file with gcc against include/wc.h, the in-tree
libwc.so and the HIP runtime (no hipcc, no Python at run time)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.abspath(os.path.join(HERE, "..", ".."))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
BIN = os.path.join(HERE, "wc_solve_file")


def build() -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           "-D__HIP_PLATFORM_AMD__",  # the HIP runtime headers serve C callers on AMD this way
           os.path.join(HERE, "wc_solve_file.c"), "-o", BIN,
           "-L", os.path.join(ROOT, "paper_1709_08785_amd"), "-lwc",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_1709_08785_amd:" + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("gcc failed for the C client:\n%s\n%s" % (r.stdout, r.stderr))
    return BIN


if __name__ == "__main__":
    print("built", build())
