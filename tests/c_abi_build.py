"""Build tests/c_abi_step.c (a C99 caller of the step library) with the host C compiler,
against include/rbstep.h, the in-tree librbstep.so and the HIP runtime."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2601_22074_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build_c_caller(out_path: str) -> str:
    # the HIP runtime header selects its platform from this macro (the library is AMD-only)
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           os.path.join(ROOT, "tests", "c_abi_step.c"), "-L", PKG, "-lrbstep",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath," + PKG, "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", out_path]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out_path
